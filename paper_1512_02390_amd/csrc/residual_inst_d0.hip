// Explicit instantiations of the residual kernels.
#include "residual_impl.h"

namespace sem {
template void launch_residual_p<double, 1>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 2>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 3>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 4>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 5>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 6>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 7>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 8>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 9>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 10>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 11>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 12>(const ResidualArgs<double> &, hipStream_t);
}  // namespace sem
