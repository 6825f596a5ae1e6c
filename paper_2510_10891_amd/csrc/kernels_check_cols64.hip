// Instantiation of the FP64 check reductions over the rows of A^T: FP64 storage.
#include "csr.h"

namespace hpr {

template void launch_check_cols<double, double, double>(const DevCsr<double>&, const DevProb<double>&, const DevIter<double>&,
                                              const Ctrl*, double*, hipStream_t);

}  // namespace hpr
