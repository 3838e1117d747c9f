// Explicit instantiations of the residual kernels.
#include "residual_impl.h"

namespace sem {
template void launch_residual_p<double, 13>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 14>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 15>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 16>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 17>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 18>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 19>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual_p<double, 20>(const ResidualArgs<double> &, hipStream_t);
}  // namespace sem
