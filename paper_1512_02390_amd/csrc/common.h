// Small device helpers shared by the kernel files.
#pragma once
#include <hip/hip_runtime.h>

namespace sem {

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Value of a nodal array at (row, col) with the boundary treatment of the
// problem: Dirichlet nodes on or outside the boundary read as zero, periodic
// indices wrap.  rows/cols are the stored array sizes.
template <typename T>
__device__ __forceinline__ T node_value(const T *__restrict__ a, int row, int col, int rows,
                                        int cols, int periodic) {
  if (periodic) {
    row = wrap(row, rows);
    col = wrap(col, cols);
    return a[(long)row * cols + col];
  }
  if (row < 1 || row > rows - 2 || col < 1 || col > cols - 2) return T(0);
  return a[(long)row * cols + col];
}

__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }

// Returns p unchanged, but hides its value from the optimiser, so that loads
// through it are not merged with loads through an earlier copy of the same
// pointer.  Used to keep wave-uniform operator tables from being held in
// scalar registers across independent uses.
template <typename T>
__device__ __forceinline__ const T *opaque(const T *p) {
  asm volatile("" : "+s"(p));
  return p;
}

// Read-only operator tables viewed through the constant address space: the
// compiler then fetches wave-uniform rows with scalar loads even in kernels
// that store to global memory (which it cannot otherwise prove disjoint).
template <typename T>
using cptr = const T __attribute__((address_space(4))) *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p) {
  return (cptr<T>)(p);
}

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace sem
