// C-ABI of the 3-D Poisson extension (sem3_*): set-up of all p-multigrid
// levels on a tensor-product mesh with Dirichlet boundaries, and the host-
// driven V-cycle (Algorithm 3) and MGCG (Algorithm 4) loops over the 3-D
// kernels.  Every arithmetic step on vectors runs in HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sem.h"
#include "host_math.h"
#include "internal.h"
#include "kernels.h"
#include "kernels3.h"

using namespace sem;

namespace {

struct Fail3 {
  sem_status s;
  std::string msg;
};

#define HIP3(x)                                                                     \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) throw Fail3{SEM_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// Device buffer owned by the handle.
struct Buf {
  void *p = nullptr;
  Buf() = default;
  Buf(const Buf &) = delete;
  Buf &operator=(const Buf &) = delete;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

// Band form of a dense matrix's rows (see Axis3Args): start, count, values.
struct Band {
  int B = 0;
  int32_t *start = nullptr, *cnt = nullptr;
  double *val = nullptr;
  int rows = 0, cols = 0;
};

// One direction of one level: subdomain types and weights.
struct Dir3 {
  int ntypes = 0;
  double *S = nullptr, *ST = nullptr, *lam = nullptr, *wts = nullptr;
  int32_t *type_of = nullptr;
};

struct Level3 {
  int p = 1, n_o = 0, m = 0;
  int N[3] = {0, 0, 0};   // nodes along x, y, z
  long n() const { return (long)N[0] * N[1] * N[2]; }
  double *Lhat = nullptr, *w = nullptr;
  double *s[3] = {nullptr, nullptr, nullptr}, *mh[3] = {nullptr, nullptr, nullptr};
  Dir3 dir[3];
  double *E = nullptr;    // interpolation from level l-1, (p+1) x (p_{l-1}+1)
  double *u = nullptr, *f = nullptr, *r = nullptr;
};

}  // namespace

struct sem3_ctx {
  hipStream_t stream = nullptr;
  int ne[3] = {0, 0, 0};
  std::vector<Level3> lev;
  std::vector<std::unique_ptr<Buf>> pool;
  // coarse fast diagonalisation: per direction S (nu x nu) as bands
  Band cfwd[3], cbwd[3];       // x -> compact (S^T), compact -> node array (S)
  double *clam[3] = {nullptr, nullptr, nullptr};
  double *cS[3] = {nullptr, nullptr, nullptr};   // dense S per direction (one-workgroup solve)
  int nu[3] = {0, 0, 0};
  double *ct1 = nullptr, *ct2 = nullptr;
  // MGCG
  double *r = nullptr, *ro = nullptr, *pv = nullptr, *q = nullptr, *z = nullptr;
  double *partial = nullptr, *scal = nullptr;
  double *part_rr = nullptr, *part_d2 = nullptr;   // MGCG partial sums (device)
  double *pin = nullptr;                           // r.r partials for the stopping test (pinned)
  std::string err;
  ~sem3_ctx() {
    if (pin) (void)hipHostFree(pin);
  }
};

namespace {

template <typename T>
T *dev_alloc(sem3_ctx *h, size_t n) {
  h->pool.emplace_back(new Buf());
  if (n == 0) return nullptr;
  if (hipMalloc(&h->pool.back()->p, n * sizeof(T)) != hipSuccess)
    throw Fail3{SEM_ENOMEM, "hipMalloc failed"};
  return static_cast<T *>(h->pool.back()->p);
}

template <typename T>
T *dev_upload(sem3_ctx *h, const std::vector<T> &v) {
  T *d = dev_alloc<T>(h, v.size());
  if (!v.empty()) HIP3(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

// Band form of the rows of a dense row-major matrix (rows x cols).
Band make_band(sem3_ctx *h, const std::vector<double> &A, int rows, int cols) {
  std::vector<int32_t> st(rows), cn(rows);
  int B = 1;
  for (int i = 0; i < rows; ++i) {
    int a = -1, b = -1;
    for (int j = 0; j < cols; ++j)
      if (A[(size_t)i * cols + j] != 0.0) {
        if (a < 0) a = j;
        b = j;
      }
    st[i] = a < 0 ? 0 : a;
    cn[i] = a < 0 ? 0 : b - a + 1;
    B = std::max(B, cn[i]);
  }
  std::vector<double> v((size_t)rows * B, 0.0);
  for (int i = 0; i < rows; ++i)
    for (int q = 0; q < cn[i]; ++q) v[(size_t)i * B + q] = A[(size_t)i * cols + st[i] + q];
  Band bd;
  bd.B = B;
  bd.rows = rows;
  bd.cols = cols;
  bd.start = dev_upload(h, st);
  bd.cnt = dev_upload(h, cn);
  bd.val = dev_upload(h, v);
  return bd;
}

// out = band product of in along axis (0 z, 1 y, 2 x); dims of out.
void axis(sem3_ctx *h, const Band &b, const double *in, double *out, int d0, int d1, int d2,
          int ax, bool acc, bool zero_bnd) {
  Axis3Args a{d0, d1, d2, ax, b.cols, in, out, b.start, b.cnt, b.val, b.B, acc ? 1 : 0,
              zero_bnd ? 1 : 0};
  launch3_axis(a, h->stream);
}

// 1-D global matrices of one direction on one level (Dirichlet, all nodes).
void line_matrices(const std::vector<double> &br, int p, Mat &L, Vec &M) {
  const int n = (int)br.size() - 1, N = n * p + 1;
  Vec xi, w;
  gll_rule(p, xi, w);
  Mat Lh = ref_stiffness(p);
  L = Mat(N, N);
  M.assign(N, 0.0);
  for (int e = 0; e < n; ++e) {
    const double hE = br[e + 1] - br[e];
    for (int a = 0; a <= p; ++a) {
      M[e * p + a] += 0.5 * hE * w[a];
      for (int b = 0; b <= p; ++b) L(e * p + a, e * p + b) += (2.0 / hE) * Lh(a, b);
    }
  }
}

void residual3(sem3_ctx *h, int l, const double *u, const double *f, double *r) {
  Level3 &L = h->lev[l];
  Res3Args a{h->ne[0], h->ne[1], h->ne[2], L.p, L.N[0], L.N[1], L.N[2], u, f, r,
             L.Lhat, L.w, L.s[0], L.s[1], L.s[2], L.mh[0], L.mh[1], L.mh[2]};
  launch3_residual(a, h->stream);
}

void fdm3(sem3_ctx *h, int l, const double *r, double *u) {
  Level3 &L = h->lev[l];
  Fdm3Args a{h->ne[0], h->ne[1], h->ne[2], L.p, L.n_o, L.m, L.N[0], L.N[1], L.N[2], r, u,
             L.dir[0].S, L.dir[0].ST, L.dir[0].lam, L.dir[1].S, L.dir[1].ST, L.dir[1].lam,
             L.dir[2].S, L.dir[2].ST, L.dir[2].lam, L.dir[0].type_of, L.dir[1].type_of,
             L.dir[2].type_of, L.dir[0].wts, L.dir[1].wts, L.dir[2].wts};
  launch3_fdm(a, h->stream);
}

void smooth3(sem3_ctx *h, int l, double *u, const double *f, int n_it, bool u_is_zero) {
  Level3 &L = h->lev[l];
  for (int it = 0; it < n_it; ++it) {
    const double *r = f;
    if (!(it == 0 && u_is_zero)) {
      residual3(h, l, u, f, L.r);
      r = L.r;
    }
    fdm3(h, l, r, u);
  }
}

// fc = I^T rf (fine level l to l-1), boundary of fc zero.
Transfer3Args transfer_args(sem3_ctx *h, int l, const double *in, double *out) {
  Level3 &F = h->lev[l], &C = h->lev[l - 1];
  return Transfer3Args{h->ne[0], h->ne[1], h->ne[2], F.p,   F.N[0], F.N[1], F.N[2],
                       C.N[0],   C.N[1],   C.N[2],   F.E, in,     out};
}

void restrict3(sem3_ctx *h, int l, const double *rf, double *fc) {
  HIP3(hipMemsetAsync(fc, 0, h->lev[l - 1].n() * sizeof(double), h->stream));
  launch3_restrict(transfer_args(h, l, rf, fc), h->stream);
}

// uf += I uc.
void prolong3(sem3_ctx *h, int l, const double *uc, double *uf) {
  launch3_prolong(transfer_args(h, l, uc, uf), h->stream);
}

// u0 = A_0^{-1} f0 by global fast diagonalisation on the p = 1 level.
void coarse3(sem3_ctx *h, const double *f0, double *u0) {
  Level3 &L = h->lev[0];
  const int *N = L.N, *n = h->nu;
  if (n[0] >= 1 && n[1] >= 1 && n[2] >= 1 && n[0] <= kCoarse3Max && n[1] <= kCoarse3Max &&
      n[2] <= kCoarse3Max) {
    Coarse3Args a{{n[0], n[1], n[2]}, {N[0], N[1], N[2]}, f0, u0,
                  {h->cS[0], h->cS[1], h->cS[2]}, {h->clam[0], h->clam[1], h->clam[2]}};
    launch3_coarse(a, h->stream);
    return;
  }
  axis(h, h->cfwd[0], f0, h->ct1, N[2], N[1], n[0], 2, false, false);
  axis(h, h->cfwd[1], h->ct1, h->ct2, N[2], n[1], n[0], 1, false, false);
  axis(h, h->cfwd[2], h->ct2, h->ct1, n[2], n[1], n[0], 0, false, false);
  launch3_eig_divide(h->ct1, n[2], n[1], n[0], h->clam[2], h->clam[1], h->clam[0], h->stream);
  axis(h, h->cbwd[0], h->ct1, h->ct2, n[2], n[1], N[0], 2, false, false);
  axis(h, h->cbwd[1], h->ct2, h->ct1, n[2], N[1], N[0], 1, false, false);
  axis(h, h->cbwd[2], h->ct1, u0, N[2], N[1], N[0], 0, false, false);
}

void vcycle3(sem3_ctx *h, double *u, const double *f, const int32_t *ns1, const int32_t *ns2) {
  const int L = (int)h->lev.size() - 1;
  auto s1 = [&](int l) { return ns1 ? ns1[l] : 1; };
  auto s2 = [&](int l) { return ns2 ? ns2[l] : 0; };
  std::vector<double *> uu(L + 1), ff(L + 1);
  uu[L] = u;
  ff[L] = const_cast<double *>(f);
  for (int l = 0; l < L; ++l) {
    uu[l] = h->lev[l].u;
    ff[l] = h->lev[l].f;
  }
  for (int l = L; l >= 1; --l) {
    smooth3(h, l, uu[l], ff[l], s1(l), l < L);
    residual3(h, l, uu[l], ff[l], h->lev[l].r);
    restrict3(h, l, h->lev[l].r, ff[l - 1]);
    if (l - 1 > 0)
      HIP3(hipMemsetAsync(uu[l - 1], 0, h->lev[l - 1].n() * sizeof(double), h->stream));
  }
  coarse3(h, ff[0], uu[0]);
  for (int l = 1; l <= L; ++l) {
    prolong3(h, l, uu[l - 1], uu[l]);
    smooth3(h, l, uu[l], ff[l], s2(l), false);
  }
}

double dot3(sem3_ctx *h, const double *x, const double *y, long n) {
  launch_dot(x, y, n, h->partial, h->scal, h->stream);
  double v = 0.0;
  HIP3(hipMemcpyAsync(&v, h->scal, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP3(hipStreamSynchronize(h->stream));
  return v;
}

void setup3(sem3_ctx *h, const sem_mesh3 *mesh, int p, const sem_overlap *ov, int wf) {
  if (!mesh || !ov || !mesh->xb || !mesh->yb || !mesh->zb) throw Fail3{SEM_EINVAL, "null argument"};
  if (p < 1 || p > 32) throw Fail3{SEM_EINVAL, "p must lie in [1, 32]"};
  const int ne[3] = {mesh->nx, mesh->ny, mesh->nz};
  for (int d = 0; d < 3; ++d)
    if (ne[d] < 1 || ne[d] > 4096) throw Fail3{SEM_EINVAL, "bad element counts"};
  if (!(wf == SEM_W_TOPHAT || (wf >= 1 && wf % 2 == 1)))
    throw Fail3{SEM_EINVAL, "3-D weight function must be odd kappa or top hat"};
  if (ov->rule == SEM_NO_FIXED && ov->n_o < 0) throw Fail3{SEM_EINVAL, "n_o < 0"};
  std::vector<double> br[3];
  const double *src[3] = {mesh->xb, mesh->yb, mesh->zb};
  for (int d = 0; d < 3; ++d) {
    br[d].assign(src[d], src[d] + ne[d] + 1);
    for (int e = 0; e < ne[d]; ++e)
      if (!(br[d][e + 1] > br[d][e])) throw Fail3{SEM_EDOM, "breaks not increasing"};
  }
  std::vector<int> orders{p};
  while (orders.back() > 1) orders.push_back((orders.back() + 1) / 2);
  std::reverse(orders.begin(), orders.end());
  const int L = (int)orders.size() - 1;
  for (int d = 0; d < 3; ++d) h->ne[d] = ne[d];
  h->lev.resize(L + 1);
  for (int l = 0; l <= L; ++l) {
    Level3 &lv = h->lev[l];
    lv.p = orders[l];
    if (l > 0) {
      int v;
      switch (ov->rule) {
        case SEM_NO_FIXED: v = ov->n_o; break;
        case SEM_NO_CEIL_P8: v = (lv.p + 7) / 8; break;
        case SEM_NO_FLOOR_P8: v = lv.p / 8; break;
        case SEM_NO_CEIL_P2: v = (lv.p + 1) / 2; break;
        default: throw Fail3{SEM_EINVAL, "unknown overlap rule"};
      }
      lv.n_o = std::max(0, std::min(v, lv.p - 1));
      lv.m = lv.p + 1 + 2 * lv.n_o;
      if (lv.m > kMaxTile3) throw Fail3{SEM_EUNSUP, "3-D subdomain width p+1+2n_o above 15"};
    }
    for (int d = 0; d < 3; ++d) lv.N[d] = ne[d] * lv.p + 1;
    Vec xi, w;
    gll_rule(lv.p, xi, w);
    lv.Lhat = dev_upload(h, ref_stiffness(lv.p).a);
    lv.w = dev_upload(h, w);
    for (int d = 0; d < 3; ++d) {
      std::vector<double> s(ne[d]), mh(ne[d]);
      for (int e = 0; e < ne[d]; ++e) {
        s[e] = 2.0 / (br[d][e + 1] - br[d][e]);
        mh[e] = 0.5 * (br[d][e + 1] - br[d][e]);
      }
      lv.s[d] = dev_upload(h, s);
      lv.mh[d] = dev_upload(h, mh);
      if (l > 0) {
        DirFdm fd = build_direction(br[d], lv.p, lv.n_o, 0, wf, nullptr);
        lv.dir[d].ntypes = fd.ntypes;
        lv.dir[d].S = dev_upload(h, fd.S);
        lv.dir[d].ST = dev_upload(h, fd.ST);
        lv.dir[d].lam = dev_upload(h, fd.lam);
        lv.dir[d].wts = dev_upload(h, fd.wts);
        std::vector<int32_t> to(fd.type_of.begin(), fd.type_of.end());
        lv.dir[d].type_of = dev_upload(h, to);
      }
    }
    if (l > 0) {
      // transfers from level l-1: the reference interpolation E(a, c) = l_c(xi_a)
      const int pc = orders[l - 1];
      Vec xic, wc;
      gll_rule(pc, xic, wc);
      lv.E = dev_upload(h, lagrange_eval(xic, xi).a);   // (p+1) x (pc+1), row-major
    }
    const long n = lv.n();
    if (l < L) {
      lv.u = dev_alloc<double>(h, n);
      lv.f = dev_alloc<double>(h, n);
    }
    lv.r = dev_alloc<double>(h, n);
    HIP3(hipMemset(lv.r, 0, n * sizeof(double)));
  }
  // coarse fast diagonalisation (level 0, p = 1)
  {
    Level3 &c = h->lev[0];
    for (int d = 0; d < 3; ++d) {
      Mat Lg;
      Vec Mg;
      line_matrices(br[d], 1, Lg, Mg);
      const int N = c.N[d], nu = N - 2;
      h->nu[d] = nu;
      Mat Li(nu, nu);
      Vec Mi(nu);
      for (int a = 0; a < nu; ++a) {
        Mi[a] = Mg[a + 1];
        for (int b = 0; b < nu; ++b) Li(a, b) = Lg(a + 1, b + 1);
      }
      Vec lam;
      Mat S;
      if (nu > 0) gen_eig_diag(Li, Mi, lam, S);
      // forward: compact o = sum_a S(a, o) x(a + 1); backward: node g = sum_o S(g - 1, o) y(o)
      std::vector<double> Fw((size_t)nu * N, 0.0), Bw((size_t)N * nu, 0.0);
      for (int o = 0; o < nu; ++o)
        for (int a = 0; a < nu; ++a) Fw[(size_t)o * N + a + 1] = S(a, o);
      for (int g = 1; g <= nu; ++g)
        for (int o = 0; o < nu; ++o) Bw[(size_t)g * nu + o] = S(g - 1, o);
      h->cfwd[d] = make_band(h, Fw, nu, N);
      h->cbwd[d] = make_band(h, Bw, N, nu);
      h->clam[d] = dev_upload(h, lam);
      std::vector<double> Sd((size_t)nu * nu);
      for (int a = 0; a < nu; ++a)
        for (int o = 0; o < nu; ++o) Sd[(size_t)a * nu + o] = S(a, o);
      h->cS[d] = dev_upload(h, Sd);
    }
    const long nc = c.n();
    h->ct1 = dev_alloc<double>(h, nc);
    h->ct2 = dev_alloc<double>(h, nc);
  }
  const long n = h->lev[L].n();
  h->r = dev_alloc<double>(h, n);
  h->ro = dev_alloc<double>(h, n);
  h->pv = dev_alloc<double>(h, n);
  h->q = dev_alloc<double>(h, n);
  h->z = dev_alloc<double>(h, n);
  h->partial = dev_alloc<double>(h, kRedBlocks);
  h->scal = dev_alloc<double>(h, 8);
  h->part_rr = dev_alloc<double>(h, kRedBlocks);
  h->part_d2 = dev_alloc<double>(h, 2 * kRedBlocks);
  HIP3(hipHostMalloc(reinterpret_cast<void **>(&h->pin), kRedBlocks * sizeof(double),
                     hipHostMallocDefault));
  HIP3(hipDeviceSynchronize());
}

sem_status guard3(sem3_ctx *h, const std::function<void()> &fn) {
  try {
    fn();
    if (h) {
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) throw Fail3{SEM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e)};
    }
    return SEM_OK;
  } catch (const Fail3 &f) {
    if (h) h->err = f.msg;
    return f.s;
  } catch (const std::bad_alloc &) {
    if (h) h->err = "host allocation failed";
    return SEM_ENOMEM;
  } catch (const std::exception &e) {
    if (h) h->err = e.what();
    return SEM_EUNSUP;
  }
}

bool level_ok(sem3_ctx *h, int l) { return h && l >= 0 && l < (int)h->lev.size(); }

}  // namespace

extern "C" {

sem_status sem3_setup(const sem_mesh3 *mesh, int32_t p, const sem_overlap *overlap, int32_t wf,
                      void *stream, sem3_handle *out) {
  if (!out) return SEM_EINVAL;
  *out = nullptr;
  std::unique_ptr<sem3_ctx> h(new sem3_ctx());
  h->stream = static_cast<hipStream_t>(stream);
  sem_status s = guard3(nullptr, [&] {
    // argument checks first: they need no device
    if (!mesh || !overlap) throw Fail3{SEM_EINVAL, "null argument"};
  });
  if (s != SEM_OK) return s;
  s = guard3(h.get(), [&] { setup3(h.get(), mesh, p, overlap, wf); });
  if (s != SEM_OK) return s;
  *out = h.release();
  return SEM_OK;
}

sem_status sem3_destroy(sem3_handle h) {
  delete h;
  return SEM_OK;
}

sem_status sem3_num_levels(sem3_handle h, int32_t *n) {
  if (!h || !n) return SEM_EINVAL;
  *n = (int32_t)h->lev.size();
  return SEM_OK;
}

sem_status sem3_level_info(sem3_handle h, int32_t level, int32_t *p, int32_t *n_o, int64_t *nodes) {
  if (!level_ok(h, level)) return SEM_EINVAL;
  const Level3 &L = h->lev[level];
  if (p) *p = L.p;
  if (n_o) *n_o = L.n_o;
  if (nodes)
    for (int d = 0; d < 3; ++d) nodes[d] = L.N[d];
  return SEM_OK;
}

sem_status sem3_residual(sem3_handle h, int32_t level, const double *u, const double *f,
                         double *r) {
  if (!level_ok(h, level) || !u || !r) return SEM_EINVAL;
  return guard3(h, [&] { residual3(h, level, u, f, r); });
}

sem_status sem3_schwarz_smooth(sem3_handle h, int32_t level, double *u, const double *f,
                               int32_t n_it) {
  if (!level_ok(h, level) || level < 1 || !u || !f || n_it < 0) return SEM_EINVAL;
  return guard3(h, [&] { smooth3(h, level, u, f, n_it, false); });
}

sem_status sem3_restrict(sem3_handle h, int32_t level, const double *rf, double *fc) {
  if (!level_ok(h, level) || level < 1 || !rf || !fc) return SEM_EINVAL;
  return guard3(h, [&] { restrict3(h, level, rf, fc); });
}

sem_status sem3_prolong_add(sem3_handle h, int32_t level, const double *uc, double *uf) {
  if (!level_ok(h, level) || level < 1 || !uc || !uf) return SEM_EINVAL;
  return guard3(h, [&] { prolong3(h, level, uc, uf); });
}

sem_status sem3_coarse_solve(sem3_handle h, const double *f0, double *u0) {
  if (!h || !f0 || !u0) return SEM_EINVAL;
  return guard3(h, [&] { coarse3(h, f0, u0); });
}

sem_status sem3_vcycle(sem3_handle h, double *u, const double *f, const int32_t *ns1,
                       const int32_t *ns2) {
  if (!h || !u || !f) return SEM_EINVAL;
  return guard3(h, [&] { vcycle3(h, u, f, ns1, ns2); });
}

sem_status sem3_pcg_solve(sem3_handle h, double *u, const double *f, int32_t imax, double rtol,
                          const int32_t *ns1, const int32_t *ns2, int32_t *iters, double *hist) {
  if (!h || !u || !f || imax < 0 || !(rtol > 0.0)) return SEM_EINVAL;
  bool converged = false;
  sem_status s = guard3(h, [&] {
    const int L = (int)h->lev.size() - 1;
    const long n = h->lev[L].n();
    const size_t bytes = n * sizeof(double);
    hipStream_t st = h->stream;
    // Algorithm 4 as in the 2-D solver: device scalars, the update fused with
    // the r.r partials and the zero initial guess of the next cycle, the
    // Polak-Ribiere products in one pass, one host round trip per iteration
    // (the stopping test); r and r_old swap buffers instead of copying.
    double *r = h->r, *ro = h->ro;
    double *delta = h->scal + 0, *delta_next = h->scal + 1;
    residual3(h, L, u, f, r);
    const double r0 = std::sqrt(dot3(h, r, r, n));
    if (hist) hist[0] = r0;
    if (!std::isfinite(r0)) throw Fail3{SEM_ENAN, "non-finite initial residual"};
    int it = 0;
    if (r0 == 0.0) {
      converged = true;
    } else {
      HIP3(hipMemsetAsync(h->pv, 0, bytes, st));
      vcycle3(h, h->pv, r, ns1, ns2);
      launch_dot(h->pv, r, n, h->partial, delta, st);
      for (it = 1; it <= imax; ++it) {
        residual3(h, L, h->pv, nullptr, h->q);   // q = A p
        const int npq = launch_dot_partials(h->pv, h->q, n, h->partial, st);
        // alpha = delta / p.q; u += alpha p; r_new = r - alpha q (into r_old's
        // buffer); r.r partials; z = 0 for the next cycle
        const int nrr = launch_cg_update2(delta, h->partial, npq, u, h->pv, r, ro, h->q, n,
                                          h->part_rr, st, nullptr, nullptr, h->z);
        std::swap(r, ro);
        if (it == 1) HIP3(hipMemsetAsync(ro, 0, bytes, st));   // r_old starts at zero
        HIP3(hipMemcpyAsync(h->pin, h->part_rr, nrr * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP3(hipStreamSynchronize(st));
        double rr = 0.0;
        for (int b = 0; b < nrr; ++b) rr += h->pin[b];
        const double rn = std::sqrt(rr);
        if (hist) hist[it] = rn;
        if (!std::isfinite(rn)) throw Fail3{SEM_ENAN, "non-finite residual"};
        if (rn <= rtol * r0) {
          converged = true;
          break;
        }
        vcycle3(h, h->z, r, ns1, ns2);
        // beta = z.(r - r_old) / delta; p = z + beta p; next delta = z.r
        launch_dot2_partials(h->z, r, ro, n, h->part_d2, st);
        launch_cg_direction2(h->part_d2, delta, delta_next, h->pv, h->z, n, st);
        std::swap(delta, delta_next);
      }
      if (it > imax) it = imax;
    }
    if (iters) *iters = it;
    HIP3(hipStreamSynchronize(h->stream));
  });
  if (s != SEM_OK) return s;
  return converged ? SEM_OK : SEM_ENOCONV;
}

const char *sem3_last_error(sem3_handle h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"
