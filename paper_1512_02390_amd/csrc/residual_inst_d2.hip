// Explicit instantiations of the residual kernels.
#include "residual_impl.h"

namespace sem {
template void launch_residual_p<double, 21>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 22>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 23>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 24>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 25>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 26>(const ResidualArgs<double> &, hipStream_t);
}  // namespace sem
