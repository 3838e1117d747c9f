// Explicit instantiations of the Schwarz kernels.
#include "fdm_impl.h"

namespace sem {
template void launch_fdm_m<float, 44>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 45>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 46>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 47>(const FdmArgs<float> &, hipStream_t);
template void launch_fdm_m<float, 48>(const FdmArgs<float> &, hipStream_t);
}  // namespace sem
