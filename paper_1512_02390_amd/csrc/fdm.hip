// Dispatch of the fast-diagonalisation Schwarz kernels by tile width; the
// kernels themselves are in fdm_impl.h.
#include "kernels.h"

namespace sem {

template <typename T, int M>
void launch_fdm_m(const FdmArgs<T> &a, hipStream_t s);

template <typename T>
void launch_fdm(const FdmArgs<T> &a, hipStream_t s) {
  switch (a.m) {
#define SEM_CASE(M) \
  case M:           \
    launch_fdm_m<T, M>(a, s); \
    break;
    SEM_CASE(2) SEM_CASE(3) SEM_CASE(4) SEM_CASE(5) SEM_CASE(6) SEM_CASE(7) SEM_CASE(8)
    SEM_CASE(9) SEM_CASE(10) SEM_CASE(11) SEM_CASE(12) SEM_CASE(13) SEM_CASE(14) SEM_CASE(15)
    SEM_CASE(16) SEM_CASE(17) SEM_CASE(18) SEM_CASE(19) SEM_CASE(20) SEM_CASE(21) SEM_CASE(22)
    SEM_CASE(23) SEM_CASE(24) SEM_CASE(25) SEM_CASE(26) SEM_CASE(27) SEM_CASE(28) SEM_CASE(29)
    SEM_CASE(30) SEM_CASE(31) SEM_CASE(32) SEM_CASE(33) SEM_CASE(34) SEM_CASE(35) SEM_CASE(36)
    SEM_CASE(37) SEM_CASE(38) SEM_CASE(39) SEM_CASE(40) SEM_CASE(41) SEM_CASE(42) SEM_CASE(43)
    SEM_CASE(44) SEM_CASE(45) SEM_CASE(46) SEM_CASE(47) SEM_CASE(48)
#undef SEM_CASE
    default:
      break;
  }
}

template void launch_fdm<double>(const FdmArgs<double> &, hipStream_t);
template void launch_fdm<float>(const FdmArgs<float> &, hipStream_t);

}  // namespace sem
