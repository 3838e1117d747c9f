// Explicit instantiations of the Schwarz kernels.
#include "fdm_impl.h"

namespace sem {
template void launch_fdm_m<double, 21>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 22>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 23>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 24>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 25>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 26>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 27>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 28>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 29>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 30>(const FdmArgs<double> &, hipStream_t);
}  // namespace sem
