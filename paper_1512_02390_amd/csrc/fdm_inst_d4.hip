// Explicit instantiations of the Schwarz kernels.
#include "fdm_impl.h"

namespace sem {
template void launch_fdm_m<double, 44>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 45>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 46>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 47>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm_m<double, 48>(const FdmArgs<double> &, hipStream_t);
}  // namespace sem
