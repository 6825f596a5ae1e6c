// Instantiations of the fused dual half of eq.(hpr) (A product, row projection, reflection, Halpern averaging)
// kernels, FP64 storage.
#include "csr.h"

namespace hpr {

template void launch_dual_step<double>(const DevCsr<double>&, const DevProb<double>&, const DevIter<double>&, const Ctrl*, int, bool,
                              hipStream_t, hipEvent_t, hipEvent_t);

}  // namespace hpr
