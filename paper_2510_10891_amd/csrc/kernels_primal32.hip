// Instantiations of the fused primal half of eq.(hpr) (A^T product, box projection, reflection, Halpern averaging)
// kernels, FP32 storage.
#include "csr.h"

namespace hpr {

template void launch_primal_step<float>(const DevCsr<float>&, const DevProb<float>&, const DevIter<float>&, const Ctrl*, int, bool,
                              hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace hpr
