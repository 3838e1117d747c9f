// Explicit instantiations of the Schwarz kernels.
#include "fdm_impl.h"

namespace sem {
template void launch_fdm_m<float, 31>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 32>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 33>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 34>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 35>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 36>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 37>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 38>(const FdmArgs<float> &, hipStream_t);
}  // namespace sem
