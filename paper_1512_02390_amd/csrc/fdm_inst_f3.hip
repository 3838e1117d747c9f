// Explicit instantiations of the Schwarz kernels.
#include "fdm_impl.h"

namespace sem {
template void launch_fdm_m<float, 39>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 40>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 41>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 42>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 43>(const FdmArgs<float> &, hipStream_t);
}  // namespace sem
