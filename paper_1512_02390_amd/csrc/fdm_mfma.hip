// Weighted additive Schwarz correction (Section 3.1, Algorithm 2) with the
// fast-diagonalisation solve on the matrix cores: BF16 or FP16 operands, FP32
// accumulation (the reduced-precision smoother of the mixed-precision
// V-cycle; the outer residual and CG stay FP64).  Same result as k_fdm up to
// the rounding of the operands:
//     du = W_y S_y [ D_s .* (S_y^T R S_x) ] S_x^T W_x,  u += du.
//
// One 64-lane wavefront per work item (elements of one subdomain type pair,
// processed one after another).  The m x m tile is padded to n = 16 NB and
// cut into 16 x 16 blocks; every block product is one or two
// v_mfma_f32_16x16x32_{f16,bf16} (K = 32 per instruction).  The
// accumulator of a block holds rows 4 (l / 16) + j, j < 4, of column l % 16
// in lane l; two vertically adjacent accumulator blocks therefore give, in
// lane l, eight values of one column at rows {4g + j} and {16 + 4g + j}
// (g = l / 16): exactly an A operand of the transposed tile for a K = 32
// chunk, once the contraction index k is taken in that order.  The B
// operands (the factor matrices) are laid out with the same k order at set-
// up (MfmaOps), so the chain
//     P1^T = R^T S_y,  P2 = P1 S_x (.* D_s / nu_bar),  Q^T = P2^T (W_y S_y)^T,
//     du = Q S_x^T
// passes every intermediate from accumulators to operands in registers.
// The factor operands arrive pre-converted and pre-scaled: one 16-byte load
// per lane and block, shared through the caches by all wavefronts of a type.
// FP16 intermediates are scaled tile by tile by powers of two (exact), and
// the correction is scaled back before the scatter (FP32 atomic adds, one
// tile row at a time from LDS).
#include "common.h"
#include "kernels.h"

#include <stdexcept>
#include <type_traits>

namespace sem {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

struct OpBF16 {
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  // BF16 keeps the FP32 exponent range: no scaling needed
  static constexpr bool kScaled = false;
  // FP32 -> BF16 bits, round to nearest even (inputs are finite)
  static __device__ __forceinline__ short cvt(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
  }
  static __device__ __forceinline__ f32x4 mma(v8 a, v8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

struct OpF16 {
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  // FP16 has a 5-bit exponent (normal range 2^-14 .. 65504): every
  // intermediate tile is scaled by a power of two that brings its largest
  // magnitude into [0.5, 1) before the conversion, so no entry overflows and
  // underflow only touches entries below 2^-14 of the tile's largest one
  static constexpr bool kScaled = true;
  static __device__ __forceinline__ short cvt(float x) {
    return __builtin_bit_cast(short, (_Float16)x);   // round to nearest even
  }
  static __device__ __forceinline__ f32x4 mma(v8 a, v8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// a[i] through a 32-bit byte offset from the array's base (arrays below 2^30
// words): the load then takes the base from scalar registers and the offset
// from one vector register, instead of a 64-bit address per load.
__device__ __forceinline__ float ld_off(const float *__restrict__ a, unsigned i) {
  return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(a) + (i << 2));
}

// Largest magnitude over the wavefront's NB x NB accumulator blocks.
template <int NB>
__device__ __forceinline__ float wave_amax(const f32x4 (&Y)[NB][NB]) {
  float v = 0.f;
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J < NB; ++J)
#pragma unroll
      for (int j = 0; j < 4; ++j) v = fmaxf(v, fabsf(Y[I][J][j]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

// e with amax = f 2^e, f in [0.5, 1) (0 for a zero tile): scaling by 2^-e
// is exact and puts the largest magnitude into [0.5, 1).
__device__ __forceinline__ int scale_exp(float amax) {
  return amax > 0.f ? __builtin_amdgcn_frexp_expf(amax) : 0;
}

// Accumulators -> A operands of the next product (the tile transposed):
// chunk c of column block I takes accumulator blocks (2c, I) and (2c+1, I)
// (zero when 2c+1 = NB).  With scaled operands the tile is first brought to
// [0.5, 1) and the exponent added to E.
template <class Op, int NB>
__device__ __forceinline__ void to_operands(const f32x4 (&Y)[NB][NB],
                                            typename Op::v8 (&Xa)[(NB + 1) / 2][NB], int &E) {
  constexpr int KC = (NB + 1) / 2;
  float sc = 1.f;
  if constexpr (Op::kScaled) {
    const int e = scale_exp(wave_amax<NB>(Y));
    E += e;
    sc = ldexpf(1.f, -e);
  }
#pragma unroll
  for (int c = 0; c < KC; ++c)
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      s16x8 v;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[j] = Op::cvt(Y[2 * c][I][j] * sc);
        v[4 + j] = (2 * c + 1 < NB) ? Op::cvt(Y[2 * c + 1][I][j] * sc) : (short)0;
      }
      Xa[c][I] = __builtin_bit_cast(typename Op::v8, v);
    }
}

typedef const uint4 __attribute__((address_space(1))) *gptr4;

// The lane's B operands of one factor matrix: KC x NB blocks, 16 bytes each
// (through a global-space pointer: the operand tables are device memory).
template <class Op, int NB>
__device__ __forceinline__ void load_operands(gptr4 B, int lane,
                                              typename Op::v8 (&b)[(NB + 1) / 2][NB]) {
#pragma unroll
  for (int c = 0; c < (NB + 1) / 2; ++c)
#pragma unroll
    for (int J = 0; J < NB; ++J) b[c][J] = __builtin_bit_cast(typename Op::v8, B[(c * NB + J) * 64 + lane]);
}

// Y = X^T B block by block: Y[I][J] = sum_c Xa[c][I] b[c][J].
template <class Op, int NB>
__device__ __forceinline__ void product(const typename Op::v8 (&Xa)[(NB + 1) / 2][NB],
                                        const typename Op::v8 (&b)[(NB + 1) / 2][NB],
                                        f32x4 (&Y)[NB][NB]) {
  constexpr int KC = (NB + 1) / 2;
#pragma unroll
  for (int J = 0; J < NB; ++J)
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < KC; ++c) acc = Op::mma(Xa[c][I], b[c][J], acc);
      Y[I][J] = acc;
    }
}

template <class Op, int NB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NB > 2 ? 3 : 4))) void k_fdm_mfma(FdmArgs<float> A) {
  typedef typename Op::v8 v8;
  constexpr int KC = (NB + 1) / 2;
  constexpr int MAT = KC * NB * 64;   // uint4 per operand matrix
  const FdmTask *__restrict__ task = A.tasks + blockIdx.x;
  const int ty = task->ty, tx = task->tx, cnt = task->count;
  const int lane0 = threadIdx.x;
  const Grid g = A.g;
  const int per = g.periodic;
  const uint4 *__restrict__ By = A.mo.by + (long)ty * 2 * MAT;   // S_y, (W_y S_y)^T
  const uint4 *__restrict__ Bx = A.mo.bx + (long)tx * 2 * MAT;   // S_x, S_x^T
  const int Ef = A.mo.ey[2 * ty] + A.mo.ey[2 * ty + 1] + A.mo.ex[2 * tx] + A.mo.ex[2 * tx + 1];
  // 1 / (lambda_y + lambda_x) of the type pair, read in accumulator layout
  // with every element's gather (cached: all elements of the work item use it)
  const float *__restrict__ dv = A.dinv + ((long)ty * A.ntx + tx) * A.m * A.m;

  constexpr int N = 16 * NB;   // padded tile width
  constexpr int LS = 65;        // LDS row stride: one word per lane, plus one
  __shared__ float tile[N * LS];
  // Memory round trips, not the matrix cores, set the time of a work item:
  // every load whose address is known is issued in one batch, and the
  // scheduling barriers keep the compiler from interleaving the batch with
  // its uses (which would wait on the loads one by one).  Narrow tiles hold
  // all four factor operands for the whole work item; wide ones load the
  // first two with the gather and the others after the first and second
  // products (the register budget of three wavefronts per SIMD).
  constexpr bool kHoldAll = NB <= 2;
  v8 b1[KC][NB], b2[KC][NB], b3[KC][NB], b4[KC][NB];
  if constexpr (kHoldAll) {
    load_operands<Op, NB>((gptr4)By, lane0, b1);          // S_y
    load_operands<Op, NB>((gptr4)Bx, lane0, b2);          // S_x
    load_operands<Op, NB>((gptr4)By + MAT, lane0, b3);    // (W_y S_y)^T
    load_operands<Op, NB>((gptr4)Bx + MAT, lane0, b4);    // S_x^T
  }
  for (int e = 0; e < cnt; ++e) {
    // The tile width, the lane index and the wide tiles' operand addresses
    // pass an optimisation barrier: otherwise the compiler hoists the
    // element-independent index arithmetic and loads out of the loop and
    // keeps them (or their spill slots) live across it.
    int m = A.m, lane = lane0;
    asm volatile("" : "+s"(m));
    asm volatile("" : "+v"(lane));
    const int c16 = lane & 15;        // column within a block
    const int r4 = (lane >> 4) * 4;   // first of the lane's 4 rows within a block
    const gptr4 Bye = (gptr4)(kHoldAll ? By : opaque(By));
    const gptr4 Bxe = (gptr4)(kHoldAll ? Bx : opaque(Bx));
    const int packed = task->elem[e];
    const int ey = packed >> 16, ex = packed & 0xffff;
    const int row0 = ey * g.p - A.n_o, col0 = ex * g.p - A.n_o;
    const float s = A.nuinv ? A.nuinv[(long)ey * g.nx + ex] : 1.0f;
    if constexpr (!kHoldAll) {
      load_operands<Op, NB>(Bye, lane, b1);
      load_operands<Op, NB>(Bxe, lane, b2);
    }
    // R in accumulator layout (block (K, I) holds rows 16K + r4 + j, columns
    // 16I + c16 of the tile).  Addresses are wrapped (periodic) or clamped
    // into the array (Dirichlet), so every load is valid; padding and
    // positions that are not unknowns are zeroed afterwards by 0/1 factors.
    int growv[NB][4], gcolv[NB];
#pragma unroll
    for (int K = 0; K < NB; ++K)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rr = row0 + 16 * K + r4 + j;
        const int rw = rr < 0 ? rr + g.rows : (rr >= g.rows ? rr - g.rows : rr);
        growv[K][j] = per ? rw : min(max(rr, 0), g.rows - 1);
      }
#pragma unroll
    for (int I = 0; I < NB; ++I) {
      const int cc = col0 + 16 * I + c16;
      const int cw = cc < 0 ? cc + g.cols : (cc >= g.cols ? cc - g.cols : cc);
      gcolv[I] = per ? cw : min(max(cc, 0), g.cols - 1);
    }
    f32x4 Y[NB][NB];
#pragma unroll
    for (int K = 0; K < NB; ++K)
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int j = 0; j < 4; ++j) Y[K][I][j] = ld_off(A.r, (unsigned)(growv[K][j] * g.cols + gcolv[I]));
    // D_s / nu_bar in accumulator layout (indices clamped into the m x m
    // tile, padding zeroed where it is applied): narrow tiles load it with
    // the gather, wide ones after the second product
    float dv4[NB][NB][4];
    auto load_dv = [&]() {
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J < NB; ++J)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            dv4[I][J][j] = ld_off(dv, (unsigned)(min(16 * I + r4 + j, m - 1) * m + min(16 * J + c16, m - 1)));
    };
    if constexpr (kHoldAll) load_dv();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int K = 0; K < NB; ++K)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int a = 16 * K + r4 + j, rr = row0 + a;
        const float rf = ((a < m) & (per | ((rr >= 1) & (rr <= g.rows - 2)))) ? 1.f : 0.f;
#pragma unroll
        for (int I = 0; I < NB; ++I) {
          const int n = 16 * I + c16, cc = col0 + n;
          const float cf = ((n < m) & (per | ((cc >= 1) & (cc <= g.cols - 2)))) ? 1.f : 0.f;
          Y[K][I][j] *= rf * cf;
        }
      }
    int E = Ef;   // du = 2^E times the last accumulator (scaled operands)
    v8 Xa[KC][NB];
    to_operands<Op, NB>(Y, Xa, E);
    product<Op, NB>(Xa, b1, Y);                   // P1^T = R^T S_y
    if constexpr (!kHoldAll) {
      load_operands<Op, NB>(Bye + MAT, lane, b3);
      __builtin_amdgcn_sched_barrier(0);
    }
    to_operands<Op, NB>(Y, Xa, E);
    product<Op, NB>(Xa, b2, Y);                   // P2 = P1 S_x
    if constexpr (!kHoldAll) {
      load_dv();
      load_operands<Op, NB>(Bxe + MAT, lane, b4);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J) {              // .* D_s / nu_bar
        const int n = 16 * J + c16;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int k = 16 * I + r4 + j;
          Y[I][J][j] *= ((k < m) & (n < m)) ? dv4[I][J][j] * s : 0.f;
        }
      }
    to_operands<Op, NB>(Y, Xa, E);
    product<Op, NB>(Xa, b3, Y);                   // Q^T = P2^T (W_y S_y)^T
    to_operands<Op, NB>(Y, Xa, E);
    product<Op, NB>(Xa, b4, Y);                   // du = Q S_x^T
    const float back = Op::kScaled ? ldexpf(1.f, E) : 1.f;
    const float *__restrict__ we = A.wel ? A.wel + ((long)ey * g.nx + ex) * 2 * m : nullptr;
    // weighted scatter-add through LDS: the accumulators go back to the tile,
    // then one tile row per iteration with lane = tile column
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int J = 0; J < NB; ++J)
#pragma unroll
        for (int j = 0; j < 4; ++j) tile[(16 * I + r4 + j) * LS + 16 * J + c16] = Y[I][J][j];
    {
      const int gc = per ? wrap(col0 + lane, g.cols) : col0 + lane;
      const bool okc = lane < m && (per || (gc >= 1 && gc <= g.cols - 2));
      const float wxn = okc ? (we ? we[m + lane] : A.wx[(long)ex * m + lane]) * back : 0.f;
      // The tile's rows in groups of four (their LDS reads issued together),
      // unrolled over the padded width so that per-row values stay in
      // registers.  With per-element weights the row weights and the nodes'
      // normalisation are loaded for all rows first, in one batch: a load
      // between two atomics would make the wavefront wait for the atomics.
      constexpr int RB = 4;
      auto scatter = [&](auto learned) {
        constexpr bool kW = decltype(learned)::value;
        float fw[kW ? N : 1];
        if constexpr (kW) {
          const int gcc = min(max(gc, 0), g.cols - 1);   // lanes >= m: any column
#pragma unroll
          for (int a = 0; a < N; ++a) {
            const int ac = min(a, m - 1);
            const int gr = per ? wrap(row0 + ac, g.rows) : min(max(row0 + ac, 0), g.rows - 1);
            fw[a] = we[ac] * ld_off(A.dnorm, (unsigned)(gr * g.cols + gcc));
          }
        }
#pragma unroll
        for (int a0 = 0; a0 < N; a0 += RB) {
          if (a0 >= m) break;
          float cv[RB];
#pragma unroll
          for (int t = 0; t < RB; ++t) cv[t] = tile[(a0 + t) * LS + lane] * wxn;
#pragma unroll
          for (int t = 0; t < RB; ++t) {
            const int a = a0 + t;
            const int gr = per ? wrap(row0 + a, g.rows) : row0 + a;
            if (okc && a < m && (per || (gr >= 1 && gr <= g.rows - 2))) {
              float c = cv[t];
              if constexpr (kW) c *= fw[a];
              atomic_add(&A.u[(long)gr * g.cols + gc], c);
            }
          }
        }
      };
      if (we)
        scatter(std::true_type{});
      else
        scatter(std::false_type{});
    }
  }
}

}  // namespace

template <class Op>
static void launch_op(const FdmArgs<float> &a, hipStream_t s) {
  if (a.m <= 32)
    klaunch((k_fdm_mfma<Op, 2>), dim3(a.ntasks), dim3(64), 0, s, a);
  else
    klaunch((k_fdm_mfma<Op, 3>), dim3(a.ntasks), dim3(64), 0, s, a);
}

void launch_fdm_mfma(const FdmArgs<float> &a, bool fp16, hipStream_t s) {
  if (a.ntasks <= 0) return;
  if (a.m > 48 || a.m < kMfmaMinTile)
    throw std::runtime_error("matrix-core Schwarz kernel: tile width outside [17, 48]");
  if (!a.mo.by || !a.mo.bx || !a.mo.ey || !a.mo.ex)
    throw std::runtime_error("matrix-core Schwarz kernel: operand tables missing");
  if ((long)a.g.rows * a.g.cols >= (1L << 30))
    throw std::runtime_error("matrix-core Schwarz kernel: node array of 2^30 words or more");
  if (fp16)
    launch_op<OpF16>(a, s);
  else
    launch_op<OpBF16>(a, s);
}

}  // namespace sem
