// Explicit instantiations of the Schwarz kernels.
#include "fdm_impl.h"

namespace sem {
template void launch_fdm_m<float, 2>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 3>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 4>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 5>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 6>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 7>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 8>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 9>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 10>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 11>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 12>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 13>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 14>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 15>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 16>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 17>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 18>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 19>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 20>(const FdmArgs<float> &, hipStream_t);
}  // namespace sem
