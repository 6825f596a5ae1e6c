// Instantiations of the FP64 check reductions over the rows of A: FP64 storage, FP32
// storage, and the FP64 re-evaluation of an FP32 candidate point (FP64 matrix and data,
// FP32 iterates).
#include "csr.h"

namespace hpr {

template void launch_check_rows<double, double, double>(const DevCsr<double>&, const DevProb<double>&,
                                                     const DevIter<double>&, const Ctrl*, double*, hipStream_t);
template void launch_check_rows<float, float, float>(const DevCsr<float>&, const DevProb<float>&, const DevIter<float>&,
                                                  const Ctrl*, double*, hipStream_t);
template void launch_check_rows<double, double, float>(const DevCsr<double>&, const DevProb<double>&,
                                                    const DevIter<float>&, const Ctrl*, double*, hipStream_t);

}  // namespace hpr
