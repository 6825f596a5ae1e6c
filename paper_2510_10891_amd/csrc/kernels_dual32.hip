// Instantiations of the fused dual half of eq.(hpr) (A product, row projection, reflection, Halpern averaging)
// kernels, FP32 storage.
#include "csr.h"

namespace hpr {

template void launch_dual_step<float>(const DevCsr<float>&, const DevProb<float>&, const DevIter<float>&, const Ctrl*, int, bool,
                              hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace hpr
