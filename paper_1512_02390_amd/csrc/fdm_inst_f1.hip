// Explicit instantiations of the Schwarz kernels.
#include "fdm_impl.h"

namespace sem {
template void launch_fdm_m<float, 21>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 22>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 23>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 24>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 25>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 26>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 27>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 28>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 29>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 30>(const FdmArgs<float> &, hipStream_t);
}  // namespace sem
