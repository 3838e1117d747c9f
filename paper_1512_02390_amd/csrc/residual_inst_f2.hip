// Explicit instantiations of the residual kernels.
#include "residual_impl.h"

namespace sem {
template void launch_residual_p<float, 21>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 22>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 23>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 24>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 25>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 26>(const ResidualArgs<float> &, hipStream_t);
}  // namespace sem
