// Small device helpers shared by the kernel files.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace sem {

// Kernel timing.  When the calling host thread has armed an event pair, the
// next launches made through klaunch record the start of the first one and
// the end of every one (so a launcher with two kernels is timed from the
// first kernel's start to the second's end).  The events are written by the
// kernel dispatch itself (hipExtLaunchKernel), so the measured time is the
// kernels' own, without the dispatch gap a separate event record would add.
struct LaunchTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};
LaunchTiming &launch_timing();   // per host thread; defined in misc.hip

template <typename F, typename... Args>
inline void klaunch(F kernel, dim3 grid, dim3 block, unsigned shm, hipStream_t s,
                    Args... args) {
  LaunchTiming &t = launch_timing();
  if (t.stop) {
    hipExtLaunchKernelGGL(kernel, grid, block, shm, s, t.start, t.stop, 0, args...);
    t.start = nullptr;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
  }
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Value of a nodal array at (row, col) with the boundary treatment of the
// problem: Dirichlet nodes on or outside the boundary read as zero, periodic
// indices wrap.  rows/cols are the stored array sizes.
// Branch-free: the load always goes to an existing node (index 0 for nodes
// that read as zero) and the value is selected afterwards, so consecutive
// calls issue their loads back to back instead of one basic block each.
// The same with an early return for nodes that read as zero: fewer memory
// requests where whole wavefronts fall outside the domain (measured faster in
// the transfer kernels, whose strips start one element outside).
template <typename T>
__device__ __forceinline__ T node_value_guarded(const T *__restrict__ a, int row, int col,
                                                int rows, int cols, int periodic) {
  if (periodic) {
    row = wrap(row, rows);
    col = wrap(col, cols);
    return a[(long)row * cols + col];
  }
  if (row < 1 || row > rows - 2 || col < 1 || col > cols - 2) return T(0);
  return a[(long)row * cols + col];
}

// No branch on the boundary type either: the wrapped index, clamped into the
// array, is formed in both cases and always loaded (for Dirichlet it only
// matters where the node is a zero anyway), and bitwise, not short-circuit,
// operators form the test.  A branch here (on the uniform boundary type, or
// around the index arithmetic) ends the scheduling region at every call, and
// the loads of an unrolled loop of calls then wait one by one.
template <typename T>
__device__ __forceinline__ T node_value(const T *__restrict__ a, int row, int col, int rows,
                                        int cols, int periodic) {
  const int rw = min(max(wrap(row, rows), 0), rows - 1);
  const int cw = min(max(wrap(col, cols), 0), cols - 1);
  const bool ok = (periodic != 0) | ((row >= 1) & (row <= rows - 2) & (col >= 1) & (col <= cols - 2));
  const T v = a[(long)rw * cols + cw];
  return ok ? v : T(0);
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
