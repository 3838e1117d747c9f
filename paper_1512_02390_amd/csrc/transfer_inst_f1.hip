// Explicit instantiations of the transfer kernels.
#include "transfer_impl.h"

namespace sem {
template void launch_restrict_p<float, 17>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 17>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 18>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 18>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 19>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 19>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 20>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 20>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 21>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 21>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 22>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 22>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 23>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 23>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 24>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 24>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 25>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 25>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 26>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 26>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 27>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 27>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 28>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 28>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 29>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 29>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 30>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 30>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 31>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 31>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 32>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 32>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
}  // namespace sem
