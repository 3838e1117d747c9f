// Explicit instantiations of the Schwarz kernels.
#include "fdm_impl.h"

namespace sem {
template void launch_fdm_m<double, 2>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 3>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 4>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 5>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 6>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 7>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 8>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 9>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 10>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 11>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 12>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 13>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 14>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 15>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 16>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 17>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 18>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 19>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 20>(const FdmArgs<double> &, hipStream_t);
}  // namespace sem
