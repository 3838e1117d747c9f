// Dispatch of the sum-factorised residual kernels by polynomial order; the
// kernels themselves are in residual_impl.h.
#include "kernels.h"

namespace sem {

template <typename T, int P>
void launch_residual_p(const ResidualArgs<T> &a, hipStream_t s);

template <typename T>
void launch_residual(const ResidualArgs<T> &a, hipStream_t s) {
  switch (a.g.p) {
#define SEM_CASE(P) \
  case P:           \
    launch_residual_p<T, P>(a, s); \
    break;
    SEM_CASE(1) SEM_CASE(2) SEM_CASE(3) SEM_CASE(4) SEM_CASE(5) SEM_CASE(6) SEM_CASE(7)
    SEM_CASE(8) SEM_CASE(9) SEM_CASE(10) SEM_CASE(11) SEM_CASE(12) SEM_CASE(13) SEM_CASE(14)
    SEM_CASE(15) SEM_CASE(16) SEM_CASE(17) SEM_CASE(18) SEM_CASE(19) SEM_CASE(20) SEM_CASE(21)
    SEM_CASE(22) SEM_CASE(23) SEM_CASE(24) SEM_CASE(25) SEM_CASE(26) SEM_CASE(27) SEM_CASE(28)
    SEM_CASE(29) SEM_CASE(30) SEM_CASE(31) SEM_CASE(32)
#undef SEM_CASE
    default:
      break;
  }
}

template void launch_residual<double>(const ResidualArgs<double> &, hipStream_t);
template void launch_residual<float>(const ResidualArgs<float> &, hipStream_t);

}  // namespace sem
