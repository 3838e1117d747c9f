// Explicit instantiations of the Schwarz kernels.
#include "fdm_impl.h"

namespace sem {
template void launch_fdm_m<double, 39>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 40>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 41>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 42>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 43>(const FdmArgs<double> &, hipStream_t);
}  // namespace sem
