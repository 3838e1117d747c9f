// Explicit instantiations of the Schwarz kernels.
#include "fdm_impl.h"

namespace sem {
template void launch_fdm_m<double, 31>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 32>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 33>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 34>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 35>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 36>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 37>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 38>(const FdmArgs<double> &, hipStream_t);
}  // namespace sem
