// Instantiations of the fused primal half of eq.(hpr) (A^T product, box projection, reflection, Halpern averaging)
// kernels, FP64 storage.
#include "csr.h"

namespace hpr {

template void launch_primal_step<double>(const DevCsr<double>&, const DevProb<double>&, const DevIter<double>&, const Ctrl*, int, bool,
                              hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace hpr
