// Explicit instantiations of the transfer kernels.
#include "transfer_impl.h"

namespace sem {
template void launch_restrict_p<double, 2>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 2>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 3>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 3>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 4>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 4>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 5>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 5>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 6>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 6>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 7>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 7>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 8>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 8>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 9>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 9>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 10>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 10>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 11>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 11>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 12>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 12>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 13>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 13>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 14>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 14>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 15>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 15>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 16>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 16>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
}  // namespace sem
