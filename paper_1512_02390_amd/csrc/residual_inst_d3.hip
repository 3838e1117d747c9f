// Explicit instantiations of the residual kernels.
#include "residual_impl.h"

namespace sem {
template void launch_residual_p<double, 27>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 28>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 29>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 30>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 31>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 32>(const ResidualArgs<double> &, hipStream_t);
}  // namespace sem
