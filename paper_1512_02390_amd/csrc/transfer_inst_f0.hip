// Explicit instantiations of the transfer kernels.
#include "transfer_impl.h"

namespace sem {
template void launch_restrict_p<float, 2>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 2>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 3>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 3>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 4>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 4>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 5>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 5>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 6>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 6>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 7>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 7>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 8>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 8>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 9>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 9>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 10>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 10>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 11>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 11>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 12>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 12>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 13>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 13>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 14>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 14>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 15>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 15>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
template void launch_restrict_p<float, 16>(const Grid &, const Grid &, const float *, float *, float *, const float *, hipStream_t);
template void launch_prolong_p<float, 16>(const Grid &, const Grid &, const float *, float *, const float *, hipStream_t);
}  // namespace sem
