// Instantiation of the FP64 check reductions over the rows of A^T: FP32 storage.
#include "csr.h"

namespace hpr {

template void launch_check_cols<float, float, float>(const DevCsr<float>&, const DevProb<float>&, const DevIter<float>&,
                                              const Ctrl*, double*, hipStream_t);

}  // namespace hpr
