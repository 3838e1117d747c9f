// Explicit instantiations of the residual kernels.
#include "residual_impl.h"

namespace sem {
template void launch_residual_p<float, 1>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 2>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 3>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 4>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 5>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 6>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 7>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 8>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 9>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 10>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 11>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 12>(const ResidualArgs<float> &, hipStream_t);
}  // namespace sem
