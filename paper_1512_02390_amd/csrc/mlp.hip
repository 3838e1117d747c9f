// Learned Schwarz parameters (project extension): element features and a
// d_in -> 64 -> 64 -> d_out multilayer perceptron (tanh hidden layers,
// logistic output) with forward, backward and Adam kernels, FP32.
//
// One 64-lane wavefront per workgroup; lane j owns hidden unit j of both
// layers.  W2 (64 x 64) is staged once per workgroup in LDS with a padded
// stride, so the forward pass reads row j (lane j) and the backward pass
// column k (lane k) without bank conflicts.  Samples are spread over the
// workgroups with a grid stride; each workgroup keeps its gradient in
// registers and writes one partial row, and a second kernel sums the rows in
// a fixed order (deterministic) and applies Adam.
#include "common.h"
#include "kernels.h"

namespace sem {
namespace {

constexpr int kW = 64;

struct Off {
  int w1, b1, w2, b2, w3, b3, n;
};

__host__ __device__ inline Off offsets(int d_in, int d_out) {
  Off o;
  o.w1 = 0;
  o.b1 = kW * d_in;
  o.w2 = o.b1 + kW;
  o.b2 = o.w2 + kW * kW;
  o.w3 = o.b2 + kW;
  o.b3 = o.w3 + d_out * kW;
  o.n = o.b3 + d_out;
  return o;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  return v;
}

template <bool GRAD>
__global__ __launch_bounds__(64) void k_mlp(const float *__restrict__ P, int d_in, int d_out,
                                            const float *__restrict__ X,
                                            const float *__restrict__ T, long n,
                                            float *__restrict__ Y, float *__restrict__ part,
                                            long stride, float inv_n) {
  __shared__ float w2[kW][kW + 1];
  __shared__ float hb[kW];
  __shared__ float db[kW];
  const int j = threadIdx.x;
  const Off o = offsets(d_in, d_out);
  for (int i = j; i < kW * kW; i += kW) w2[i / kW][i % kW] = P[o.w2 + i];
  float w1[kMlpMaxIn];
#pragma unroll
  for (int i = 0; i < kMlpMaxIn; ++i) w1[i] = i < d_in ? P[o.w1 + j * d_in + i] : 0.0f;
  const float b1 = P[o.b1 + j], b2 = P[o.b2 + j];
  float w3[kMlpMaxOut], b3[kMlpMaxOut];
#pragma unroll
  for (int q = 0; q < kMlpMaxOut; ++q) {
    w3[q] = q < d_out ? P[o.w3 + q * kW + j] : 0.0f;
    b3[q] = q < d_out ? P[o.b3 + q] : 0.0f;
  }
  float gw1[kMlpMaxIn] = {}, gw2[kW] = {}, gw3[kMlpMaxOut] = {}, gb3[kMlpMaxOut] = {};
  float gb1 = 0.0f, gb2 = 0.0f, lsum = 0.0f;
  __syncthreads();
  for (long s = blockIdx.x; s < n; s += gridDim.x) {
    const float *x = X + s * d_in;
    float xv[kMlpMaxIn];
#pragma unroll
    for (int i = 0; i < kMlpMaxIn; ++i) xv[i] = i < d_in ? x[i] : 0.0f;
    float a1 = b1;
#pragma unroll
    for (int i = 0; i < kMlpMaxIn; ++i) a1 = fmaf(w1[i], xv[i], a1);
    const float h1 = tanhf(a1);
    __syncthreads();              // previous sample's readers of hb / db are done
    hb[j] = h1;
    __syncthreads();
    float a2 = b2;
#pragma unroll 16
    for (int k = 0; k < kW; ++k) a2 = fmaf(w2[j][k], hb[k], a2);
    const float h2 = tanhf(a2);
    float y[kMlpMaxOut];
#pragma unroll
    for (int q = 0; q < kMlpMaxOut; ++q) {
      y[q] = 0.0f;
      if (q < d_out) {
        const float z = wave_sum(w3[q] * h2) + b3[q];
        y[q] = 1.0f / (1.0f + expf(-z));
        if (Y && j == 0) Y[s * d_out + q] = y[q];
      }
    }
    if constexpr (GRAD) {
      float dh2 = 0.0f;
#pragma unroll
      for (int q = 0; q < kMlpMaxOut; ++q) {
        if (q < d_out) {
          const float r = y[q] - T[s * d_out + q];
          lsum = fmaf(0.5f * r, r, lsum);
          const float dz = r * inv_n * y[q] * (1.0f - y[q]);
          gw3[q] = fmaf(dz, h2, gw3[q]);
          gb3[q] += dz;
          dh2 = fmaf(w3[q], dz, dh2);
        }
      }
      const float dz2 = dh2 * (1.0f - h2 * h2);
      gb2 += dz2;
#pragma unroll 16
      for (int k = 0; k < kW; ++k) gw2[k] = fmaf(dz2, hb[k], gw2[k]);
      db[j] = dz2;
      __syncthreads();
      float dh1 = 0.0f;
#pragma unroll 16
      for (int i = 0; i < kW; ++i) dh1 = fmaf(w2[i][j], db[i], dh1);
      const float dz1 = dh1 * (1.0f - h1 * h1);
      gb1 += dz1;
#pragma unroll
      for (int i = 0; i < kMlpMaxIn; ++i) gw1[i] = fmaf(dz1, xv[i], gw1[i]);
    }
  }
  if constexpr (GRAD) {
    float *out = part + blockIdx.x * stride;
    for (int i = 0; i < d_in; ++i) out[o.w1 + j * d_in + i] = gw1[i];
    out[o.b1 + j] = gb1;
    for (int k = 0; k < kW; ++k) out[o.w2 + j * kW + k] = gw2[k];
    out[o.b2 + j] = gb2;
    for (int q = 0; q < d_out; ++q) out[o.w3 + q * kW + j] = gw3[q];
    if (j == 0) {
      for (int q = 0; q < d_out; ++q) out[o.b3 + q] = gb3[q];
      out[o.n] = lsum * inv_n;
    }
  }
}

// Sum of the partial rows (fixed order) for every parameter and the loss;
// optional copy of the gradient, optional Adam update.
__global__ void k_mlp_reduce(const float *__restrict__ part, int nblk, long stride, long np,
                             float *__restrict__ grad, float *__restrict__ loss,
                             float *__restrict__ P, float *__restrict__ m, float *__restrict__ v,
                             float lr, float c1, float c2, int adam) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > np) return;
  float g = 0.0f;
  for (int b = 0; b < nblk; ++b) g += part[b * stride + i];
  if (i == np) {
    if (loss) *loss = g;
    return;
  }
  if (grad) grad[i] = g;
  if (adam) {
    const float mi = 0.9f * m[i] + 0.1f * g;
    const float vi = 0.999f * v[i] + 0.001f * g * g;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
  }
}

// Features of every element (e = ey * nx + ex), d_in = 8:
//   log2(h_x/h_y), ln nu_bar, ln nu_bar of the 4 neighbours minus ln nu_bar
//   (left, right, lower, upper; 0 at a Dirichlet side), ln(max nu / min nu)
//   over the element's nodes, p / 32.
__global__ void k_features(Grid g, const double *__restrict__ nu, const double *__restrict__ nuinv,
                           const double *__restrict__ hx, const double *__restrict__ hy,
                           float *__restrict__ F) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.nx * g.ny) return;
  const int ey = e / g.nx, ex = e - (e / g.nx) * g.nx;
  float *f = F + (long)e * kMlpFeatures;
  f[0] = (float)log2(hx[ex] / hy[ey]);
  const double lb = nuinv ? -log(nuinv[e]) : 0.0;
  f[1] = (float)lb;
  const int dy[4] = {0, 0, -1, 1}, dx[4] = {-1, 1, 0, 0};
  for (int k = 0; k < 4; ++k) {
    int jy = ey + dy[k], jx = ex + dx[k];
    double c = 0.0;
    if (g.periodic) {
      jy = wrap(jy, g.ny);
      jx = wrap(jx, g.nx);
      if (nuinv) c = -log(nuinv[jy * g.nx + jx]) - lb;
    } else if (jy >= 0 && jy < g.ny && jx >= 0 && jx < g.nx) {
      if (nuinv) c = -log(nuinv[jy * g.nx + jx]) - lb;
    }
    f[2 + k] = (float)c;
  }
  double lo = 1.0, hi = 1.0;
  if (nu) {
    lo = INFINITY;
    hi = 0.0;
    for (int b = 0; b <= g.p; ++b) {
      int row = ey * g.p + b;
      if (g.periodic && row == g.rows) row = 0;
      for (int a = 0; a <= g.p; ++a) {
        int col = ex * g.p + a;
        if (g.periodic && col == g.cols) col = 0;
        const double v = nu[(long)row * g.cols + col];
        lo = fmin(lo, v);
        hi = fmax(hi, v);
      }
    }
  }
  f[6] = (float)log(hi / lo);
  f[7] = (float)(g.p / 32.0);
}

}  // namespace

long mlp_num_params(int d_in, int d_out) { return offsets(d_in, d_out).n; }

void launch_mlp(const float *P, int d_in, int d_out, const float *X, const float *T, long n,
                float *Y, float *part, long stride, int nblk, hipStream_t s) {
  if (n <= 0) return;
  const float inv_n = 1.0f / (float)n;
  if (part)
    hipLaunchKernelGGL(k_mlp<true>, dim3(nblk), dim3(kW), 0, s, P, d_in, d_out, X, T, n, Y, part,
                       stride, inv_n);
  else
    hipLaunchKernelGGL(k_mlp<false>, dim3(nblk), dim3(kW), 0, s, P, d_in, d_out, X, T, n, Y,
                       part, stride, inv_n);
}

void launch_mlp_reduce(const float *part, int nblk, long stride, long np, float *grad, float *loss,
                       float *P, float *m, float *v, float lr, float c1, float c2, int adam,
                       hipStream_t s) {
  const int threads = 256;
  hipLaunchKernelGGL(k_mlp_reduce, dim3(ceil_div(np + 1, threads)), dim3(threads), 0, s, part,
                     nblk, stride, np, grad, loss, P, m, v, lr, c1, c2, adam);
}

void launch_features(const Grid &g, const double *nu, const double *nuinv, const double *hx,
                     const double *hy, float *F, hipStream_t s) {
  const int n = g.nx * g.ny;
  hipLaunchKernelGGL(k_features, dim3(ceil_div(n, 64)), dim3(64), 0, s, g, nu, nuinv, hx, hy, F);
}

}  // namespace sem
