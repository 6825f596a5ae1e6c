// Instantiations of the plain matrix product (the power method's A~ and A~^T products).
#include "csr.h"

namespace hpr {

template void launch_spmv<double>(const DevCsr<double>&, const double*, double*, hipStream_t);
template void launch_spmv<float>(const DevCsr<float>&, const float*, float*, hipStream_t);

}  // namespace hpr
