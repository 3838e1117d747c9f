// Explicit instantiations of the residual kernels.
#include "residual_impl.h"

namespace sem {
template void launch_residual_p<float, 27>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 28>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 29>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 30>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 31>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 32>(const ResidualArgs<float> &, hipStream_t);
}  // namespace sem
