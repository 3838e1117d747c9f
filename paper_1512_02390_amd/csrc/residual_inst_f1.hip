// Explicit instantiations of the residual kernels.
#include "residual_impl.h"

namespace sem {
template void launch_residual_p<float, 13>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 14>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 15>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 16>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 17>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 18>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 19>(const ResidualArgs<float> &, hipStream_t);
template void launch_residual_p<float, 20>(const ResidualArgs<float> &, hipStream_t);
}  // namespace sem
