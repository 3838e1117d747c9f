// Explicit instantiations of the transfer kernels.
#include "transfer_impl.h"

namespace sem {
template void launch_restrict_p<double, 17>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 17>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 18>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 18>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 19>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 19>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 20>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 20>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 21>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 21>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 22>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 22>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 23>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 23>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 24>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 24>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 25>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 25>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 26>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 26>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 27>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 27>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 28>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 28>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 29>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 29>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 30>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 30>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 31>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 31>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
template void launch_restrict_p<double, 32>(const Grid &, const Grid &, const double *, double *, double *, const double *, hipStream_t);
template void launch_prolong_p<double, 32>(const Grid &, const Grid &, const double *, double *, const double *, hipStream_t);
}  // namespace sem
