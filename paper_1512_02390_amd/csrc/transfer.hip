// Dispatch of the p-multigrid transfer kernels by fine order; the kernels
// themselves are in transfer_impl.h.
#include "kernels.h"

namespace sem {

template <typename T, int PF>
void launch_restrict_p(const Grid &gf, const Grid &gc, const T *rf, T *fc, T *uc_zero,
                       const T *ET, hipStream_t s);
template <typename T, int PF>
void launch_prolong_p(const Grid &gf, const Grid &gc, const T *uc, T *uf, const T *E,
                      hipStream_t s);

template <typename T>
void launch_restrict(const Grid &gf, const Grid &gc, const T *rf, T *fc, T *uc_zero, const T *ET,
                     hipStream_t s) {
  switch (gf.p) {
#define SEM_CASE(P) \
  case P:           \
    launch_restrict_p<T, P>(gf, gc, rf, fc, uc_zero, ET, s); \
    break;
    SEM_CASE(2) SEM_CASE(3) SEM_CASE(4) SEM_CASE(5) SEM_CASE(6) SEM_CASE(7) SEM_CASE(8) SEM_CASE(9) SEM_CASE(10) SEM_CASE(11) SEM_CASE(12) SEM_CASE(13) SEM_CASE(14) SEM_CASE(15) SEM_CASE(16) SEM_CASE(17) SEM_CASE(18) SEM_CASE(19) SEM_CASE(20) SEM_CASE(21) SEM_CASE(22) SEM_CASE(23) SEM_CASE(24) SEM_CASE(25) SEM_CASE(26) SEM_CASE(27) SEM_CASE(28) SEM_CASE(29) SEM_CASE(30) SEM_CASE(31) SEM_CASE(32)
#undef SEM_CASE
    default:
      break;
  }
}

template <typename T>
void launch_prolong(const Grid &gf, const Grid &gc, const T *uc, T *uf, const T *E,
                    hipStream_t s) {
  switch (gf.p) {
#define SEM_CASE(P) \
  case P:           \
    launch_prolong_p<T, P>(gf, gc, uc, uf, E, s); \
    break;
    SEM_CASE(2) SEM_CASE(3) SEM_CASE(4) SEM_CASE(5) SEM_CASE(6) SEM_CASE(7) SEM_CASE(8) SEM_CASE(9) SEM_CASE(10) SEM_CASE(11) SEM_CASE(12) SEM_CASE(13) SEM_CASE(14) SEM_CASE(15) SEM_CASE(16) SEM_CASE(17) SEM_CASE(18) SEM_CASE(19) SEM_CASE(20) SEM_CASE(21) SEM_CASE(22) SEM_CASE(23) SEM_CASE(24) SEM_CASE(25) SEM_CASE(26) SEM_CASE(27) SEM_CASE(28) SEM_CASE(29) SEM_CASE(30) SEM_CASE(31) SEM_CASE(32)
#undef SEM_CASE
    default:
      break;
  }
}

template void launch_restrict<double>(const Grid &, const Grid &, const double *, double *,
                                      double *, const double *, hipStream_t);
template void launch_restrict<float>(const Grid &, const Grid &, const float *, float *, float *,
                                     const float *, hipStream_t);
template void launch_prolong<double>(const Grid &, const Grid &, const double *, double *,
                                     const double *, hipStream_t);
template void launch_prolong<float>(const Grid &, const Grid &, const float *, float *,
                                    const float *, hipStream_t);

}  // namespace sem
