// C-ABI of the learned Schwarz parameters (project extension): the MLP handle
// (forward, gradient, Adam training step on the device) and the reduction of
// per-element predictions to the per-level overlaps and per-grid-line width
// scales that sem_setup accepts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/sem.h"
#include "kernels.h"

using namespace sem;

namespace {
constexpr int kMlpWidth = 64;
constexpr int kMlpBlocks = 256;   // workgroups of the gradient kernel (partial rows)
}  // namespace

struct sem_mlp_ctx {
  hipStream_t stream = nullptr;
  int d_in = 0, d_out = 0;
  long np = 0, stride = 0;
  float *P = nullptr, *m = nullptr, *v = nullptr, *part = nullptr, *loss = nullptr;
  long t = 0;
  ~sem_mlp_ctx() {
    for (float *q : {P, m, v, part, loss})
      if (q) (void)hipFree(q);
  }
};

namespace {

int blocks_for(long n) { return (int)std::max(1L, std::min<long>(kMlpBlocks, n)); }

sem_status hip_status(hipError_t e) { return e == hipSuccess ? SEM_OK : SEM_EHIP; }

sem_status read_loss(sem_mlp h, float *loss) {
  if (!loss) return SEM_OK;
  float v = 0.0f;
  hipError_t e = hipMemcpyAsync(&v, h->loss, sizeof(float), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  *loss = v;
  return hip_status(e);
}

// Forward + backward on n samples into the partial rows.
void grad_pass(sem_mlp h, const float *x, const float *t, long n) {
  launch_mlp(h->P, h->d_in, h->d_out, x, t, n, nullptr, h->part, h->stride, blocks_for(n),
             h->stream);
}

}  // namespace

extern "C" {

sem_status sem_mlp_num_params(int32_t d_in, int32_t width, int32_t d_out, int64_t *n) {
  if (!n) return SEM_EINVAL;
  if (d_in < 1 || d_out < 1 || width < 1) return SEM_EINVAL;
  if (d_in > kMlpMaxIn || d_out > kMlpMaxOut || width != kMlpWidth) return SEM_EUNSUP;
  *n = mlp_num_params(d_in, d_out);
  return SEM_OK;
}

sem_status sem_mlp_create(int32_t d_in, int32_t width, int32_t d_out, const float *params,
                          void *stream, sem_mlp *out) {
  if (!out || !params) return SEM_EINVAL;
  *out = nullptr;
  int64_t np = 0;
  sem_status s = sem_mlp_num_params(d_in, width, d_out, &np);
  if (s != SEM_OK) return s;
  auto *h = new (std::nothrow) sem_mlp_ctx();
  if (!h) return SEM_ENOMEM;
  h->stream = static_cast<hipStream_t>(stream);
  h->d_in = d_in;
  h->d_out = d_out;
  h->np = np;
  h->stride = np + 1;
  const size_t bytes = np * sizeof(float);
  bool ok = hipMalloc(&h->P, bytes) == hipSuccess && hipMalloc(&h->m, bytes) == hipSuccess &&
            hipMalloc(&h->v, bytes) == hipSuccess &&
            hipMalloc(&h->part, (size_t)kMlpBlocks * h->stride * sizeof(float)) == hipSuccess &&
            hipMalloc(&h->loss, sizeof(float)) == hipSuccess;
  if (!ok) {
    delete h;
    return SEM_ENOMEM;
  }
  hipError_t e = hipMemcpy(h->P, params, bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(h->m, 0, bytes);
  if (e == hipSuccess) e = hipMemset(h->v, 0, bytes);
  if (e != hipSuccess) {
    delete h;
    return SEM_EHIP;
  }
  *out = h;
  return SEM_OK;
}

sem_status sem_mlp_destroy(sem_mlp h) {
  if (!h) return SEM_EINVAL;
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return SEM_OK;
}

sem_status sem_mlp_forward(sem_mlp h, const float *x, int64_t n, float *y) {
  if (!h || n < 0 || (n > 0 && (!x || !y))) return SEM_EINVAL;
  launch_mlp(h->P, h->d_in, h->d_out, x, nullptr, n, y, nullptr, 0, blocks_for(n), h->stream);
  return hip_status(hipGetLastError());
}

sem_status sem_mlp_gradient(sem_mlp h, const float *x, const float *t, int64_t n, float *grad,
                            float *loss) {
  if (!h || !grad || n < 1 || !x || !t) return SEM_EINVAL;
  grad_pass(h, x, t, n);
  launch_mlp_reduce(h->part, blocks_for(n), h->stride, h->np, grad, h->loss, nullptr, nullptr,
                    nullptr, 0.0f, 0.0f, 0.0f, 0, h->stream);
  sem_status s = hip_status(hipGetLastError());
  return s == SEM_OK ? read_loss(h, loss) : s;
}

sem_status sem_mlp_train_step(sem_mlp h, const float *x, const float *t, int64_t n, float lr,
                              float *loss) {
  if (!h || n < 1 || !x || !t || !(lr >= 0.0f)) return SEM_EINVAL;
  grad_pass(h, x, t, n);
  h->t += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)h->t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)h->t)));
  launch_mlp_reduce(h->part, blocks_for(n), h->stride, h->np, nullptr, h->loss, h->P, h->m, h->v,
                    lr, c1, c2, 1, h->stream);
  sem_status s = hip_status(hipGetLastError());
  return s == SEM_OK ? read_loss(h, loss) : s;
}

sem_status sem_mlp_get_params(sem_mlp h, float *params) {
  if (!h || !params) return SEM_EINVAL;
  hipError_t e = hipMemcpyAsync(params, h->P, h->np * sizeof(float), hipMemcpyDeviceToHost,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return hip_status(e);
}

sem_status sem_learned_params(const float *pred, int32_t nx, int32_t ny, int32_t p, int32_t bc,
                              int32_t *overlaps, double *alpha_x, double *alpha_y) {
  if (!pred || !overlaps || !alpha_x || !alpha_y || nx < 1 || ny < 1 || p < 1) return SEM_EINVAL;
  if (bc != SEM_BC_DIRICHLET && bc != SEM_BC_PERIODIC) return SEM_EINVAL;
  const bool per = bc == SEM_BC_PERIODIC;
  const long ne = (long)nx * ny;
  std::vector<double> a(ne);
  double qsum = 0.0;
  for (long e = 0; e < ne; ++e) {
    const double al = pred[2 * e], q = pred[2 * e + 1];
    if (!std::isfinite(al) || !std::isfinite(q)) return SEM_ENAN;
    a[e] = std::min(std::max(al, 0.1), 1.0);
    qsum += q;
  }
  const double rho = 0.5 * qsum / (double)ne;
  // width scale of a grid line: mean over the elements touching it
  for (int i = 0; i <= nx; ++i) {
    int c0 = i - 1, c1 = i;
    if (per && (i == 0 || i == nx)) c0 = nx - 1, c1 = 0;
    double s = 0.0;
    int cnt = 0;
    for (int c : {c0, c1}) {
      if (c < 0 || c >= nx) continue;
      for (int r = 0; r < ny; ++r) s += a[(long)r * nx + c];
      cnt += ny;
    }
    alpha_x[i] = s / cnt;
  }
  for (int j = 0; j <= ny; ++j) {
    int r0 = j - 1, r1 = j;
    if (per && (j == 0 || j == ny)) r0 = ny - 1, r1 = 0;
    double s = 0.0;
    int cnt = 0;
    for (int r : {r0, r1}) {
      if (r < 0 || r >= ny) continue;
      for (int c = 0; c < nx; ++c) s += a[(long)r * nx + c];
      cnt += nx;
    }
    alpha_y[j] = s / cnt;
  }
  // overlap per level: ceil(rho p_l), within [1, p_l - 1] and the tile limit
  std::vector<int> orders{p};
  while (orders.back() > 1) orders.push_back((orders.back() + 1) / 2);
  std::reverse(orders.begin(), orders.end());
  overlaps[0] = 0;
  for (size_t l = 1; l < orders.size(); ++l) {
    const int pl = orders[l];
    int n = (int)std::ceil(rho * pl);
    n = std::min(std::max(n, 1), std::min(pl - 1, (kMaxTile - 1 - pl) / 2));
    overlaps[l] = n;
  }
  return SEM_OK;
}

}  // extern "C"
