// Instantiation of the FP64 check reductions over the rows of A^T: the FP64 re-evaluation of an FP32 candidate point (FP64 matrix and data, FP32 iterates).
#include "csr.h"

namespace hpr {

template void launch_check_cols<double, double, float>(const DevCsr<double>&, const DevProb<double>&, const DevIter<float>&,
                                              const Ctrl*, double*, hipStream_t);

}  // namespace hpr
