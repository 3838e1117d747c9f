// C-ABI of the SEM Schwarz / p-multigrid solver: set-up of all levels and the
// host-driven V-cycle (Algorithm 3) and MGCG (Algorithm 4) loops.  Every
// arithmetic step on vectors runs in the HIP kernels of this library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <thread>
#include <vector>

#include "../../include/sem.h"
#include "common.h"
#include "host_math.h"
#include "internal.h"
#include "kernels.h"

using namespace sem;

namespace {

struct Fail {
  sem_status s;
  std::string msg;
};

#define HIP_OK(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess)                                                          \
      throw Fail{SEM_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)};        \
  } while (0)

// Device buffer owned by the handle.
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  void alloc(size_t n) {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = n;
    if (n == 0) return;
    if (hipMalloc(&p, n) != hipSuccess) throw Fail{SEM_ENOMEM, "hipMalloc failed"};
  }
  template <typename T>
  T *as() const { return static_cast<T *>(p); }
};

template <typename T>
T *upload(std::vector<std::unique_ptr<DBuf>> &pool, const std::vector<double> &h) {
  pool.emplace_back(new DBuf());
  DBuf &b = *pool.back();
  b.alloc(h.size() * sizeof(T));
  if (h.empty()) return nullptr;
  std::vector<T> tmp(h.begin(), h.end());
  HIP_OK(hipMemcpy(b.p, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
  return b.as<T>();
}

template <typename T>
T *dalloc(std::vector<std::unique_ptr<DBuf>> &pool, size_t n) {
  pool.emplace_back(new DBuf());
  pool.back()->alloc(n * sizeof(T));
  return pool.back()->as<T>();
}

// Copies a host array of any trivially copyable type to a new device buffer.
template <typename T>
T *upload_raw(std::vector<std::unique_ptr<DBuf>> &pool, const std::vector<T> &h) {
  pool.emplace_back(new DBuf());
  DBuf &b = *pool.back();
  b.alloc(h.size() * sizeof(T));
  if (h.empty()) return nullptr;
  HIP_OK(hipMemcpy(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return b.as<T>();
}

// FP32 -> BF16 bits, round to nearest even (finite inputs).
uint16_t bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
uint16_t f16_bits(float x) {
  const _Float16 h = (_Float16)x;   // round to nearest even
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

// Matrix-core B operands of one direction's subdomain types (MfmaOps):
// B(t, q, k, n) is entry (k, n) of matrix q in {0, 1} of type t.  Values
// are laid out [t][q][KC][NB][lane][8] with the permuted k order of the
// kernel, scaled by 2^-e per matrix (FP16; e = 0 for BF16).
template <typename F>
void mfma_operands(const F &B, int ntypes, int m, bool fp16, std::vector<uint16_t> &vals,
                   std::vector<int32_t> &exps) {
  const int NB = (m + 15) / 16, KC = (NB + 1) / 2;
  vals.assign((size_t)ntypes * 2 * KC * NB * 64 * 8, 0);
  exps.assign((size_t)ntypes * 2, 0);
  for (int t = 0; t < ntypes; ++t)
    for (int q = 0; q < 2; ++q) {
      int e = 0;
      if (fp16) {
        double amax = 0.0;
        for (int k = 0; k < m; ++k)
          for (int n = 0; n < m; ++n) amax = std::max(amax, std::fabs(B(t, q, k, n)));
        if (amax > 0.0) std::frexp(amax, &e);   // amax = f 2^e, f in [0.5, 1)
      }
      exps[(size_t)t * 2 + q] = e;
      const double sc = std::ldexp(1.0, -e);
      for (int c = 0; c < KC; ++c)
        for (int J = 0; J < NB; ++J)
          for (int l = 0; l < 64; ++l)
            for (int v = 0; v < 8; ++v) {
              const int g = l / 16;
              const int k = 32 * c + (v < 4 ? 4 * g + v : 16 + 4 * g + v - 4);
              const int n = 16 * J + l % 16;
              const float x = (k < m && n < m) ? (float)(B(t, q, k, n) * sc) : 0.f;
              vals[((((size_t)t * 2 + q) * KC + c) * NB + J) * 512 + (size_t)l * 8 + v] =
                  fp16 ? f16_bits(x) : bf16_bits(x);
            }
    }
}

// MfmaOps of a set of subdomain types: y types from S_y^T and diag(w_y) S_y
// (B = S_y and (W_y S_y)^T), x types from S_x (B = S_x and S_x^T).
MfmaOps build_mfma_ops(std::vector<std::unique_ptr<DBuf>> &pool, const std::vector<double> &SyT, const std::vector<double> &SyW,
                       int nty, const std::vector<double> &Sx, int ntx, int m, bool fp16) {
  const size_t mm = (size_t)m * m;
  std::vector<uint16_t> vy, vx;
  std::vector<int32_t> ey, ex;
  mfma_operands([&](int t, int q, int k, int n) {
    return (q == 0 ? SyT : SyW)[t * mm + (size_t)n * m + k];
  }, nty, m, fp16, vy, ey);
  mfma_operands([&](int t, int q, int k, int n) {
    return q == 0 ? Sx[t * mm + (size_t)k * m + n] : Sx[t * mm + (size_t)n * m + k];
  }, ntx, m, fp16, vx, ex);
  MfmaOps mo;
  mo.by = reinterpret_cast<const uint4 *>(upload_raw<uint16_t>(pool, vy));
  mo.bx = reinterpret_cast<const uint4 *>(upload_raw<uint16_t>(pool, vx));
  mo.ey = upload_raw<int32_t>(pool, ey);
  mo.ex = upload_raw<int32_t>(pool, ex);
  return mo;
}

// Tables of one level in one precision.
template <typename T>
struct Tables {
  T *Lhat = nullptr, *D = nullptr, *w = nullptr;
  T *sx = nullptr, *sy = nullptr, *mx = nullptr, *my = nullptr;
  T *Sx = nullptr, *SxT = nullptr, *SyW = nullptr, *SyT = nullptr, *dinv = nullptr;
  T *wx = nullptr, *nuinv = nullptr, *nu = nullptr, *nuT = nullptr, *DT = nullptr;
  T *gy = nullptr, *gx = nullptr;  // flux scratch of the variable-nu residual
  T *E = nullptr, *ET = nullptr;  // interpolation from level l-1 and its transpose
};


// Schwarz tables of the subdomains of one overlap value when every element
// carries its own parameters (sem_weights.elem_params).
template <typename T>
struct FdmTab {
  T *Sx = nullptr, *SxT = nullptr, *SyW = nullptr, *SyT = nullptr, *dinv = nullptr;
  T *wel = nullptr;   // per element: 1-D weights along y, then along x
};
struct Seg {
  int n_o = 0, m = 0, ntasks = 0, ntx = 0;
  FdmTask *tasks = nullptr;
  FdmTab<double> d;
  FdmTab<float> f;
  MfmaOps mo;   // matrix-core operands (BF16 / FP16 precision, m >= kMfmaMinTile)
};

struct Level {
  int p = 1, n_o = 0, m = 0;
  std::vector<Seg> segs;                     // per-element parameters: one per overlap value
  double *dnorm = nullptr;                   // 1 / (sum of subdomain weights) per node
  float *dnormf = nullptr;
  Grid g{};
  std::vector<double> xc, yc;     // node coordinates
  std::vector<double> nu_host;    // nodal nu (variable coefficient)
  Tables<double> td;
  Tables<float> tf;
  FdmTask *tasks = nullptr;
  int ntasks = 0, ntx = 0, nty = 0;
  MfmaOps mo;   // matrix-core operands (BF16 / FP16 precision, m >= kMfmaMinTile)
  int32_t *tx_of = nullptr, *ty_of = nullptr;   // subdomain type per element column / row
  // level vectors (FP64 and FP32)
  double *u = nullptr, *f = nullptr, *r = nullptr;
  float *uf = nullptr, *ff = nullptr, *rf = nullptr;
  long n() const { return (long)g.rows * g.cols; }
};

}  // namespace

struct sem_ctx {
  hipStream_t stream = nullptr;
  int precision = SEM_FP64;
  int bc = SEM_BC_DIRICHLET;
  bool mult = false;   // multiplicative Schwarz (SEM_W_MULT) on levels l > 0
  bool varnu = false;
  std::vector<Level> lev;
  std::vector<std::unique_ptr<DBuf>> pool;
  // coarse solver
  int cnx = 0, cny = 0;           // unknowns per direction on level 0
  long coff = 0;                  // offset of the unknown block in the node array
  double *cSx = nullptr, *cSy = nullptr, *cDinv = nullptr, *cT1 = nullptr, *cT2 = nullptr;
  double *cSxT = nullptr, *cSyT = nullptr;   // transposes (coalesced operands of k_sandwich)
  double *cMinv = nullptr;        // dense inverse (variable nu)
  double *cf = nullptr;           // projected copy of f0 (periodic)
  double *cu64 = nullptr, *cf64 = nullptr;  // FP64 coarse vectors for the FP32 cycle
  // PCG / reductions
  double *pr = nullptr, *pp = nullptr, *pq = nullptr, *pz = nullptr, *pro = nullptr;
  double *partial = nullptr, *scal = nullptr;  // scal: device scalars
  // element widths and 1/nu_bar per element (element features)
  double *hx = nullptr, *hy = nullptr, *enuinv = nullptr, *enu = nullptr;  // enu: finest nodal nu
  // optional kernel timing on one level: event pairs of timed launches, with
  // the kind of launch (sem_timing_kind) of each pair
  int time_level = -1;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
  std::string err;
  // pinned host slots and events for reading residual norms asynchronously
  double *pin = nullptr;                   // 2 slots of kRedBlocks r.r partials (pinned)
  double *part_rr = nullptr, *part_d2 = nullptr;   // MGCG partial sums (device)
  hipEvent_t nev[2] = {nullptr, nullptr};
  ~sem_ctx() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : nev)
      if (e) (void)hipEventDestroy(e);
    if (pin) (void)hipHostFree(pin);
  }
};

namespace {

int level_overlap(int rule, int n_o, int pl) {
  int v;
  switch (rule) {
    case SEM_NO_FIXED: v = n_o; break;
    case SEM_NO_CEIL_P8: v = (pl + 7) / 8; break;
    case SEM_NO_FLOOR_P8: v = pl / 8; break;
    case SEM_NO_CEIL_P2: v = (pl + 1) / 2; break;
    default: throw Fail{SEM_EINVAL, "unknown overlap rule"};
  }
  return std::max(0, std::min(v, pl - 1));
}

// Work items of a level's Schwarz kernel: EPW = 64/m elements of one
// subdomain type pair per wavefront, grouped by type pair anywhere in the
// mesh; `only` (optional) restricts the list to a subset of the elements.
std::vector<FdmTask> build_tasks(const DirFdm &fx, const DirFdm &fy, int nx, int ny, int m,
                                 const std::vector<char> *only = nullptr) {
  const int epw = std::min(64 / m, kTaskSlots);
  std::vector<FdmTask> tasks;
  for (int ty = 0; ty < fy.ntypes; ++ty)
    for (int tx = 0; tx < fx.ntypes; ++tx) {
      FdmTask cur{};
      cur.ty = ty;
      cur.tx = tx;
      for (int ey = 0; ey < ny; ++ey) {
        if (fy.type_of[ey] != ty) continue;
        for (int ex = 0; ex < nx; ++ex) {
          if (fx.type_of[ex] != tx) continue;
          if (only && !(*only)[(size_t)ey * nx + ex]) continue;
          cur.elem[cur.count++] = (ey << 16) | ex;
          if (cur.count == epw) {
            tasks.push_back(cur);
            cur.count = 0;
          }
        }
      }
      if (cur.count) tasks.push_back(cur);
    }
  return tasks;
}

template <typename T>
void upload_tables(sem_ctx *h, Level &L, Tables<T> &t, const std::vector<double> &Lhat,
                   const std::vector<double> &D, const std::vector<double> &DT,
                   const std::vector<double> &w,
                   const std::vector<double> &sx, const std::vector<double> &sy,
                   const std::vector<double> &mx, const std::vector<double> &my,
                   const DirFdm *fx, const DirFdm *fy, const std::vector<double> &dinv,
                   const std::vector<double> &nuinv, const std::vector<double> &E) {
  auto &P = h->pool;
  t.Lhat = upload<T>(P, Lhat);
  t.D = upload<T>(P, D);
  t.DT = upload<T>(P, DT);
  t.w = upload<T>(P, w);
  t.sx = upload<T>(P, sx);
  t.sy = upload<T>(P, sy);
  t.mx = upload<T>(P, mx);
  t.my = upload<T>(P, my);
  if (fx) {
    t.Sx = upload<T>(P, fx->S);
    t.SxT = upload<T>(P, fx->ST);
    t.SyW = upload<T>(P, fy->SW);
    t.SyT = upload<T>(P, fy->ST);
    t.dinv = upload<T>(P, dinv);
    t.wx = upload<T>(P, fx->wts);
  }
  if (!nuinv.empty()) t.nuinv = upload<T>(P, nuinv);
  if (!L.nu_host.empty()) {
    // nu times the GLL weight of the contraction direction (a node on an
    // element interface has local index 0 or p, whose weights are equal);
    // the row-direction table is transposed: that flux reads nu along rows
    // with one lane per row, which is coalesced in this layout
    const int R = L.g.rows, Cc = L.g.cols, pp = L.p;
    std::vector<double> ny_((size_t)R * Cc), nx_((size_t)R * Cc);
    for (int r = 0; r < R; ++r)
      for (int c = 0; c < Cc; ++c) {
        const double v = L.nu_host[(size_t)r * Cc + c];
        ny_[(size_t)r * Cc + c] = v * w[r % pp];
        nx_[(size_t)c * R + r] = v * w[c % pp];
      }
    t.nu = upload<T>(P, ny_);
    t.nuT = upload<T>(P, nx_);
    t.gy = dalloc<T>(P, (size_t)L.g.ny * (pp + 1) * Cc);
    t.gx = dalloc<T>(P, (size_t)L.g.nx * (pp + 1) * R);
  }
  if (!E.empty()) {
    t.E = upload<T>(P, E);
    const int nr = L.p + 1, nc = (int)(E.size() / nr);
    std::vector<double> ET(E.size());
    for (int a = 0; a < nr; ++a)
      for (int c = 0; c < nc; ++c) ET[(size_t)c * nr + a] = E[(size_t)a * nc + c];
    t.ET = upload<T>(P, ET);
  }
}

std::vector<double> flat(const Mat &M) { return M.a; }

// Dense matrix of B(nu) (or A) on the unknowns of a p = 1 level, assembled
// from 4x4 element matrices by GLL quadrature (Section 4).
Mat coarse_dense(const Level &L, const std::vector<double> &xb, const std::vector<double> &yb) {
  const Grid &g = L.g;
  const int per = g.periodic;
  const int nux = per ? g.cols : g.cols - 2, nuy = per ? g.rows : g.rows - 2;
  const int n = nux * nuy;
  Mat B(n, n);
  auto num = [&](int row, int col) -> int {
    if (per) return (row % g.rows) * nux + (col % g.cols);
    if (row < 1 || row > g.rows - 2 || col < 1 || col > g.cols - 2) return -1;
    return (row - 1) * nux + (col - 1);
  };
  // p = 1: GLL points -1, 1, weights 1, 1; D = [[-1/2, 1/2], [-1/2, 1/2]]
  const double Dm[2][2] = {{-0.5, 0.5}, {-0.5, 0.5}};
  for (int ey = 0; ey < g.ny; ++ey)
    for (int ex = 0; ex < g.nx; ++ex) {
      const double hx = xb[ex + 1] - xb[ex], hy = yb[ey + 1] - yb[ey];
      double nu[2][2];
      int id[2][2];
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const int row = (ey + b) % (per ? g.rows : 1 << 30), col = (ex + a) % (per ? g.cols : 1 << 30);
          nu[b][a] = L.nu_host.empty() ? 1.0 : L.nu_host[(size_t)row * g.cols + col];
          id[b][a] = num(ey + b, ex + a);
        }
      // element matrix K[(b,a),(d,c)]
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          if (id[b][a] < 0) continue;
          for (int d = 0; d < 2; ++d)
            for (int c = 0; c < 2; ++c) {
              if (id[d][c] < 0) continue;
              // x part: (hy/hx) sum_q w_q w_b nu D[q][a] D[q][c] delta_bd
              double v = 0.0;
              if (b == d)
                for (int q = 0; q < 2; ++q) v += (hy / hx) * nu[b][q] * Dm[q][a] * Dm[q][c];
              if (a == c)
                for (int q = 0; q < 2; ++q) v += (hx / hy) * nu[q][a] * Dm[q][b] * Dm[q][d];
              B(id[b][a], id[d][c]) += v;
            }
        }
    }
  return B;
}

// Overlap of an element with overlap ratio rho on a level of order p_l:
// ceil(rho p_l), clamped to [1, p_l - 1] and to a subdomain width of at most
// kMaxTile nodes.
int element_overlap(double rho, int pl) {
  int v = (int)std::ceil(rho * pl - 1e-12);
  v = std::min(std::max(v, 1), std::min(pl - 1, (kMaxTile - pl - 1) / 2));
  return std::max(v, 0);
}

// Per-element Schwarz parameters on one level: one segment of tables and
// work items per distinct overlap, per-element 1-D weights, and the node
// array 1/D of the Shepard normalisation (D = sum of the subdomain weights).
void build_segments(sem_ctx *h, Level &lv, const std::vector<double> &xb,
                    const std::vector<double> &yb, int per, int wf, const float *ep, bool mixed) {
  const int nx = lv.g.nx, ny = lv.g.ny, p = lv.p;
  const long ne = (long)nx * ny;
  const bool mfma = h->precision == SEM_MIXED_BF16 || h->precision == SEM_MIXED_FP16;
  std::vector<int> no(ne);
  for (long e = 0; e < ne; ++e) no[e] = element_overlap(ep[2 * e + 1], p);
  std::vector<int> vals(no.begin(), no.end());
  std::sort(vals.begin(), vals.end());
  vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
  Vec xi, wq;
  gll_rule(p, xi, wq);
  const int R = lv.g.rows, Cc = lv.g.cols;
  std::vector<double> Dsum((size_t)R * Cc, 0.0);
  // extended coordinate of window position k (Section 3.1) and whether the
  // node there is an unknown
  auto ext = [&](int k, int n_o) {
    const int t = k - n_o;
    return t < 0 ? xi[p + t] - 2.0 : (t > p ? xi[t - p] + 2.0 : xi[t]);
  };
  for (int v : vals) {
    Seg sg;
    sg.n_o = v;
    sg.m = p + 1 + 2 * v;
    const int m = sg.m;
    DirFdm fx = build_direction(xb, p, v, per, wf, nullptr, true);
    DirFdm fy = build_direction(yb, p, v, per, wf, nullptr, true);
    sg.ntx = fx.ntypes;
    std::vector<double> dinv((size_t)fy.ntypes * fx.ntypes * m * m);
    for (int ty = 0; ty < fy.ntypes; ++ty)
      for (int tx = 0; tx < fx.ntypes; ++tx)
        for (int a = 0; a < m; ++a)
          for (int c = 0; c < m; ++c)
            dinv[(((size_t)ty * fx.ntypes + tx) * m + a) * m + c] =
                1.0 / (fy.lam[(size_t)ty * m + a] + fx.lam[(size_t)tx * m + c]);
    std::vector<char> mine(ne, 0);
    std::vector<double> wel((size_t)ne * 2 * m, 0.0);
    const double delta = xi[v + 1] + 1.0;
    for (int ey = 0; ey < ny; ++ey)
      for (int ex = 0; ex < nx; ++ex) {
        const long e = (long)ey * nx + ex;
        if (no[e] != v) continue;
        mine[e] = 1;
        const double a = ep[2 * e];
        double *wy = &wel[(size_t)e * 2 * m], *wx = wy + m;
        std::vector<int> rows(m), cols(m);
        for (int k = 0; k < m; ++k) {
          int gr = ey * p - v + k, gc = ex * p - v + k;
          bool vr, vc;
          if (per) {
            gr = ((gr % R) + R) % R;
            gc = ((gc % Cc) + Cc) % Cc;
            vr = vc = true;
          } else {
            vr = gr >= 1 && gr <= R - 2;
            vc = gc >= 1 && gc <= Cc - 2;
          }
          rows[k] = vr ? gr : -1;
          cols[k] = vc ? gc : -1;
          const double x = ext(k, v);
          if (vr)
            wy[k] = wf == SEM_W_ARITH ? 1.0
                                      : weight_fn(wf, x, a * delta, a * delta, !per && ey == 0,
                                                  !per && ey == ny - 1);
          if (vc)
            wx[k] = wf == SEM_W_ARITH ? 1.0
                                      : weight_fn(wf, x, a * delta, a * delta, !per && ex == 0,
                                                  !per && ex == nx - 1);
        }
        for (int i = 0; i < m; ++i)
          for (int j = 0; j < m; ++j)
            if (rows[i] >= 0 && cols[j] >= 0) Dsum[(size_t)rows[i] * Cc + cols[j]] += wy[i] * wx[j];
      }
    std::vector<FdmTask> tasks = build_tasks(fx, fy, nx, ny, m, &mine);
    sg.ntasks = (int)tasks.size();
    if (sg.ntasks) {
      h->pool.emplace_back(new DBuf());
      h->pool.back()->alloc(tasks.size() * sizeof(FdmTask));
      sg.tasks = h->pool.back()->as<FdmTask>();
      HIP_OK(hipMemcpy(sg.tasks, tasks.data(), tasks.size() * sizeof(FdmTask),
                       hipMemcpyHostToDevice));
    }
    auto fill = [&](auto &t, auto tag) {
      using T = decltype(tag);
      t.Sx = upload<T>(h->pool, fx.S);
      t.SxT = upload<T>(h->pool, fx.ST);
      t.SyW = upload<T>(h->pool, fy.SW);   // unweighted: W = 1 in build_direction
      t.SyT = upload<T>(h->pool, fy.ST);
      t.dinv = upload<T>(h->pool, dinv);
      t.wel = upload<T>(h->pool, wel);
    };
    fill(sg.d, double());
    if (mixed) fill(sg.f, float());
    if (mfma && m >= kMfmaMinTile)
      sg.mo = build_mfma_ops(h->pool, fy.ST, fy.SW, fy.ntypes, fx.S, fx.ntypes, m,
                             h->precision == SEM_MIXED_FP16);
    lv.segs.push_back(sg);
  }
  std::vector<double> dn((size_t)R * Cc, 0.0);
  for (size_t i = 0; i < dn.size(); ++i) dn[i] = Dsum[i] > 0.0 ? 1.0 / Dsum[i] : 0.0;
  lv.dnorm = upload<double>(h->pool, dn);
  if (mixed) lv.dnormf = upload<float>(h->pool, dn);
}

// Window of subdomain e along one axis: for every position t of
// [e p - n_o, (e+1) p + n_o], the global node (-1 beyond a Dirichlet end)
// and whether it is an unknown; [first, last] is the range of positions
// that are nodes.
struct AxisWindow {
  std::vector<int> node;
  std::vector<char> valid;
  int first = -1, last = -1;
};

AxisWindow axis_window(int e, int p, int n_o, int N, int per) {
  AxisWindow w;
  const int m = p + 1 + 2 * n_o;
  for (int t = 0; t < m; ++t) {
    int g = e * p - n_o + t;
    bool exists, valid;
    if (per) {
      g = ((g % N) + N) % N;
      exists = valid = true;
    } else {
      exists = g >= 0 && g <= N - 1;
      valid = g >= 1 && g <= N - 2;
    }
    w.node.push_back(exists ? g : -1);
    w.valid.push_back(valid);
    if (exists) {
      if (w.first < 0) w.first = t;
      w.last = t;
    }
  }
  return w;
}

// 1-D stiffness and lumped mass on the window of subdomain e, weighted by a
// coefficient given per window position (coef[t], t in [first, last]):
// GLL quadrature over the elements e - 1, e, e + 1 that exist, with local
// node q of element e + d at position d p + q + n_o and its coefficient
// taken at that position clamped to [first, last].
void weighted_window_ops(const std::vector<double> &br, int e, int p, int n_o, int per,
                         const AxisWindow &win, const Vec &coef, const Vec &w, const Mat &D,
                         Mat &Ls, Vec &Ms) {
  const int n = (int)br.size() - 1;
  const int m = p + 1 + 2 * n_o;
  Ls = Mat(m, m);
  Ms.assign(m, 0.0);
  Vec c(p + 1);
  for (int d = -1; d <= 1; ++d) {
    int E = e + d;
    if (per)
      E = (E + n) % n;
    else if (E < 0 || E >= n)
      continue;
    const double h = br[E + 1] - br[E];
    for (int q = 0; q <= p; ++q)
      c[q] = coef[std::min(std::max(d * p + q + n_o, win.first), win.last)];
    for (int a = 0; a <= p; ++a) {
      const int ka = d * p + a + n_o;
      if (ka < 0 || ka >= m) continue;
      Ms[ka] += 0.5 * h * w[a] * c[a];
      for (int b = 0; b <= p; ++b) {
        const int kb = d * p + b + n_o;
        if (kb < 0 || kb >= m) continue;
        double sum = 0.0;
        for (int r = 0; r <= p; ++r) sum += w[r] * c[r] * D(r, a) * D(r, b);
        Ls(ka, kb) += (2.0 / h) * sum;
      }
    }
  }
}

// Fast-diagonalisation factors of (Ls, Ms) on the valid positions, padded
// with identity rows (lambda = 1) at the others: S (m x m), lambda (m).
void padded_factors(const Mat &Ls, const Vec &Ms, const std::vector<char> &valid, Vec &Sp,
                    Vec &lp) {
  const int m = (int)valid.size();
  std::vector<int> vi, ii;
  for (int k = 0; k < m; ++k) (valid[k] ? vi : ii).push_back(k);
  const int nv = (int)vi.size();
  Mat L(nv, nv);
  Vec M(nv);
  for (int a = 0; a < nv; ++a) {
    M[a] = Ms[vi[a]];
    for (int b = 0; b < nv; ++b) L(a, b) = Ls(vi[a], vi[b]);
  }
  Vec lam;
  Mat S;
  gen_eig_diag(L, M, lam, S);
  Sp.assign((size_t)m * m, 0.0);
  lp.assign(m, 1.0);
  for (int a = 0; a < nv; ++a) {
    lp[a] = lam[a];
    for (int c2 = 0; c2 < nv; ++c2) Sp[(size_t)vi[a] * m + c2] = S(a, c2);
  }
  for (size_t t = 0; t < ii.size(); ++t) Sp[(size_t)ii[t] * m + nv + t] = 1.0;
}

// Separable local coefficients (sem_weights.local_solve =
// SEM_LOCAL_SEPARABLE): for subdomain e = ey nx + ex, log nu on the window's
// nodes is fitted as alpha(x) + beta(y) by least squares (column means minus
// the grand mean, row means); the local operator M_b (x) L_a + L_b (x) M_a
// with a = exp(alpha), b = exp(beta) (weighted_window_ops) is diagonalised
// per direction.  fx / fy come in from build_direction (the paper's weights)
// and leave with one type per subdomain, type e in both directions; dinv
// holds one eigenvalue-sum tile per subdomain (indexed by the x type, the
// kernels' pair stride being 0), and every task holds one subdomain.
void build_separable(const Level &lv, const std::vector<double> &xb, const std::vector<double> &yb,
                     int per, DirFdm &fx, DirFdm &fy, std::vector<double> &dinv,
                     std::vector<FdmTask> &tasks) {
  const int nx = lv.g.nx, ny = lv.g.ny, p = lv.p, n_o = lv.n_o, m = lv.m;
  const int R = lv.g.rows, Cc = lv.g.cols;
  const long ne = (long)nx * ny;
  Vec xi, w;
  gll_rule(p, xi, w);
  const Mat D = lagrange_derivative(xi);
  std::vector<AxisWindow> wx(nx), wy(ny);
  for (int e = 0; e < nx; ++e) wx[e] = axis_window(e, p, n_o, Cc, per);
  for (int e = 0; e < ny; ++e) wy[e] = axis_window(e, p, n_o, R, per);
  const size_t mm = (size_t)m * m;
  std::vector<double> Sx(ne * mm), SxT(ne * mm), SyW(ne * mm), SyT(ne * mm), dv(ne * mm);
  auto work = [&](long e) {
    const int ey = (int)(e / nx), ex = (int)(e % nx);
    const AxisWindow &ax = wx[ex], &ay = wy[ey];
    const int nxw = ax.last - ax.first + 1, nyw = ay.last - ay.first + 1;
    // least-squares split of log nu over the window's node grid
    std::vector<double> lg((size_t)nyw * nxw);
    for (int j = 0; j < nyw; ++j)
      for (int i = 0; i < nxw; ++i)
        lg[(size_t)j * nxw + i] =
            std::log(lv.nu_host[(size_t)ay.node[ay.first + j] * Cc + ax.node[ax.first + i]]);
    double grand = 0.0;
    for (double v : lg) grand += v;
    grand /= (double)lg.size();
    Vec ca(m, 0.0), cb(m, 0.0);
    for (int i = 0; i < nxw; ++i) {
      double s = 0.0;
      for (int j = 0; j < nyw; ++j) s += lg[(size_t)j * nxw + i];
      ca[ax.first + i] = std::exp(s / nyw - grand);
    }
    for (int j = 0; j < nyw; ++j) {
      double s = 0.0;
      for (int i = 0; i < nxw; ++i) s += lg[(size_t)j * nxw + i];
      cb[ay.first + j] = std::exp(s / nxw);
    }
    Mat La, Lb;
    Vec Ma, Mb, Spx, lx, Spy, ly;
    weighted_window_ops(xb, ex, p, n_o, per, ax, ca, w, D, La, Ma);
    weighted_window_ops(yb, ey, p, n_o, per, ay, cb, w, D, Lb, Mb);
    padded_factors(La, Ma, ax.valid, Spx, lx);
    padded_factors(Lb, Mb, ay.valid, Spy, ly);
    const double *wyv = fy.wts.data() + (size_t)ey * m;
    for (int a = 0; a < m; ++a)
      for (int c = 0; c < m; ++c) {
        Sx[e * mm + (size_t)a * m + c] = Spx[(size_t)a * m + c];
        SxT[e * mm + (size_t)a * m + c] = Spx[(size_t)c * m + a];
        SyW[e * mm + (size_t)a * m + c] = wyv[a] * Spy[(size_t)a * m + c];
        SyT[e * mm + (size_t)a * m + c] = Spy[(size_t)c * m + a];
        dv[e * mm + (size_t)a * m + c] = 1.0 / (ly[a] + lx[c]);
      }
  };
  // the subdomains are independent: spread them over the host's cores
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::atomic<long> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < nth; ++t)
    pool.emplace_back([&] {
      for (long e = next++; e < ne; e = next++) work(e);
    });
  for (std::thread &t : pool) t.join();
  fx.ntypes = fy.ntypes = (int)ne;
  fx.S = std::move(Sx);
  fx.ST = std::move(SxT);
  fy.SW = std::move(SyW);
  fy.ST = std::move(SyT);
  dinv = std::move(dv);
  tasks.clear();
  for (long e = 0; e < ne; ++e) {
    FdmTask t{};
    t.ty = t.tx = (int)e;
    t.count = 1;
    t.elem[0] = (int)(((e / nx) << 16) | (e % nx));
    tasks.push_back(t);
  }
}

void setup_impl(sem_ctx *h, const sem_mesh *mesh, int p, const sem_overlap *ov,
                const sem_weights *wts, const double *nu) {
  if (!mesh || !ov || !wts || !mesh->xb || !mesh->yb) throw Fail{SEM_EINVAL, "null argument"};
  if (p < 1) throw Fail{SEM_EINVAL, "p must be >= 1"};
  if (p > kMaxOrder) throw Fail{SEM_EUNSUP, "p above 32"};
  const int nx = mesh->nx, ny = mesh->ny, per = mesh->bc == SEM_BC_PERIODIC;
  if (nx < 1 || ny < 1 || nx > 65535 || ny > 65535) throw Fail{SEM_EINVAL, "bad element counts"};
  if (mesh->bc != SEM_BC_DIRICHLET && !per) throw Fail{SEM_EINVAL, "bad boundary condition"};
  if (per && (nx < 3 || ny < 3)) throw Fail{SEM_EINVAL, "periodic needs at least 3 elements"};
  if (ov->rule == SEM_NO_FIXED && ov->n_o < 0) throw Fail{SEM_EINVAL, "n_o < 0"};
  if (!(wts->wf == SEM_W_TOPHAT || wts->wf == SEM_W_ARITH || wts->wf == SEM_W_MULT ||
        (wts->wf >= 1 && wts->wf % 2 == 1)))
    throw Fail{SEM_EINVAL, "weight function must be odd kappa, top hat, arithmetic or multiplicative"};
  if (wts->wf == SEM_W_MULT &&
      (nu || h->precision != SEM_FP64 || wts->alpha_x || wts->alpha_y || wts->elem_params ||
       wts->local_solve != SEM_LOCAL_MEAN))
    throw Fail{SEM_EUNSUP, "multiplicative Schwarz: Poisson, FP64, paper weights only"};
  std::vector<double> xb(mesh->xb, mesh->xb + nx + 1), yb(mesh->yb, mesh->yb + ny + 1);
  for (int i = 0; i < nx; ++i)
    if (!(xb[i + 1] > xb[i])) throw Fail{SEM_EDOM, "x breaks not increasing"};
  for (int i = 0; i < ny; ++i)
    if (!(yb[i + 1] > yb[i])) throw Fail{SEM_EDOM, "y breaks not increasing"};
  if (wts->local_solve != SEM_LOCAL_MEAN && wts->local_solve != SEM_LOCAL_SEPARABLE)
    throw Fail{SEM_EINVAL, "unknown local solve"};
  if (wts->local_solve == SEM_LOCAL_SEPARABLE && (!nu || wts->elem_params))
    throw Fail{SEM_EINVAL, "separable local solves need nu and exclude per-element parameters"};
  if (wts->elem_params) {
    if (wts->alpha_x || wts->alpha_y)
      throw Fail{SEM_EINVAL, "per-element parameters exclude per-line width scales"};
    for (long e = 0; e < (long)nx * ny; ++e) {
      const double a = wts->elem_params[2 * e], r = wts->elem_params[2 * e + 1];
      if (!(std::isfinite(a) && a > 0.0 && a <= 1.0) || !(std::isfinite(r) && r >= 0.0))
        throw Fail{SEM_EINVAL, "per-element parameters: alpha in (0, 1], rho >= 0"};
    }
  }
  for (const double *a : {wts->alpha_x, wts->alpha_y}) {
    if (!a) continue;
    const int n = (a == wts->alpha_x ? nx : ny) + 1;
    for (int i = 0; i < n; ++i)
      if (!(a[i] > 0.0 && a[i] <= 1.0)) throw Fail{SEM_EINVAL, "width scales must lie in (0, 1]"};
  }
  h->bc = mesh->bc;
  h->varnu = nu != nullptr;
  h->mult = wts->wf == SEM_W_MULT;
  {
    std::vector<double> wx(nx), wy(ny);
    for (int e = 0; e < nx; ++e) wx[e] = xb[e + 1] - xb[e];
    for (int e = 0; e < ny; ++e) wy[e] = yb[e + 1] - yb[e];
    h->hx = upload<double>(h->pool, wx);
    h->hy = upload<double>(h->pool, wy);
  }
  // level orders p_L = p, p_{l-1} = ceil(p_l / 2)
  std::vector<int> orders{p};
  while (orders.back() > 1) orders.push_back((orders.back() + 1) / 2);
  std::reverse(orders.begin(), orders.end());
  const int L = (int)orders.size() - 1;
  h->lev.resize(L + 1);
  for (int l = 0; l <= L; ++l) {
    Level &lv = h->lev[l];
    lv.p = orders[l];
    if (l == 0) {
      lv.n_o = 0;
    } else if (wts->elem_params) {
      lv.n_o = 0;
      for (long e = 0; e < (long)nx * ny; ++e)
        lv.n_o = std::max(lv.n_o, element_overlap(wts->elem_params[2 * e + 1], lv.p));
    } else if (ov->per_level) {
      lv.n_o = ov->per_level[l];
      if (lv.n_o < 0 || lv.n_o > lv.p - 1) throw Fail{SEM_EINVAL, "per-level overlap outside [0, p_l - 1]"};
    } else {
      lv.n_o = level_overlap(ov->rule, ov->n_o, lv.p);
    }
    lv.m = lv.p + 1 + 2 * lv.n_o;
    if (l > 0 && lv.m > kMaxTile) throw Fail{SEM_EUNSUP, "subdomain width p+1+2n_o above 48"};
    lv.g = Grid{nx, ny, lv.p, per ? ny * lv.p : ny * lv.p + 1, per ? nx * lv.p : nx * lv.p + 1, per};
    Vec xi, w;
    gll_rule(lv.p, xi, w);
    lv.xc.assign(lv.g.cols, 0.0);
    lv.yc.assign(lv.g.rows, 0.0);
    for (int e = 0; e < nx; ++e)
      for (int a = 0; a <= lv.p; ++a) {
        int c = e * lv.p + a;
        if (per && c == lv.g.cols) continue;
        lv.xc[c] = xb[e] + 0.5 * (xb[e + 1] - xb[e]) * (xi[a] + 1.0);
      }
    for (int e = 0; e < ny; ++e)
      for (int a = 0; a <= lv.p; ++a) {
        int r = e * lv.p + a;
        if (per && r == lv.g.rows) continue;
        lv.yc[r] = yb[e] + 0.5 * (yb[e + 1] - yb[e]) * (xi[a] + 1.0);
      }
  }
  // variable coefficient: nodal nu on every level, element means on the top
  std::vector<double> nubar;
  if (nu) {
    Level &top = h->lev[L];
    top.nu_host.assign(nu, nu + top.n());
    for (double v : top.nu_host)
      if (!(v > 0.0) || !std::isfinite(v)) throw Fail{SEM_EDOM, "nu must be positive and finite"};
    Vec xiL, wL;
    gll_rule(top.p, xiL, wL);
    nubar.assign((size_t)nx * ny, 0.0);
    for (int ey = 0; ey < ny; ++ey)
      for (int ex = 0; ex < nx; ++ex) {
        double s = 0.0;
        for (int b = 0; b <= top.p; ++b)
          for (int a = 0; a <= top.p; ++a) {
            int row = (ey * top.p + b) % top.g.rows, col = (ex * top.p + a) % top.g.cols;
            if (!per) { row = ey * top.p + b; col = ex * top.p + a; }
            s += wL[a] * wL[b] * top.nu_host[(size_t)row * top.g.cols + col];
          }
        nubar[(size_t)ey * nx + ex] = s / 4.0;
      }
    for (int l = 0; l < L; ++l) {
      Level &lv = h->lev[l];
      Vec xi, w;
      gll_rule(lv.p, xi, w);
      Mat E = lagrange_eval(xiL, xi);  // (p_l+1) x (p_L+1)
      lv.nu_host.assign(lv.n(), 0.0);
      // element by element, sum-factorised: along x first (T), then along y
      std::vector<double> T((size_t)(top.p + 1) * (lv.p + 1));
      for (int ey = 0; ey < ny; ++ey)
        for (int ex = 0; ex < nx; ++ex) {
          for (int d = 0; d <= top.p; ++d) {
            int row = ey * top.p + d;
            if (per) row %= top.g.rows;
            for (int a = 0; a <= lv.p; ++a) {
              double t = 0.0;
              for (int c = 0; c <= top.p; ++c) {
                int col = ex * top.p + c;
                if (per) col %= top.g.cols;
                t += E(a, c) * top.nu_host[(size_t)row * top.g.cols + col];
              }
              T[(size_t)d * (lv.p + 1) + a] = t;
            }
          }
          for (int b = 0; b <= lv.p; ++b)
            for (int a = 0; a <= lv.p; ++a) {
              double s = 0.0;
              for (int d = 0; d <= top.p; ++d) s += E(b, d) * T[(size_t)d * (lv.p + 1) + a];
              int row = ey * lv.p + b, col = ex * lv.p + a;
              if (per) { row %= lv.g.rows; col %= lv.g.cols; }
              lv.nu_host[(size_t)row * lv.g.cols + col] = s;
            }
        }
    }
  }
  std::vector<double> nuinv;
  for (double v : nubar) nuinv.push_back(1.0 / v);
  if (!nuinv.empty()) h->enuinv = upload<double>(h->pool, nuinv);
  if (nu) h->enu = upload<double>(h->pool, h->lev.back().nu_host);
  const bool mixed = h->precision != SEM_FP64;
  // per-level tables
  for (int l = 0; l <= L; ++l) {
    Level &lv = h->lev[l];
    Vec xi, w;
    gll_rule(lv.p, xi, w);
    Mat D = lagrange_derivative(xi);
    Mat Lh = ref_stiffness(lv.p);
    std::vector<double> sx(nx), sy(ny), mx(nx), my(ny);
    for (int e = 0; e < nx; ++e) { sx[e] = 2.0 / (xb[e + 1] - xb[e]); mx[e] = 0.5 * (xb[e + 1] - xb[e]); }
    for (int e = 0; e < ny; ++e) { sy[e] = 2.0 / (yb[e + 1] - yb[e]); my[e] = 0.5 * (yb[e + 1] - yb[e]); }
    std::vector<double> E;
    if (l > 0) {
      Vec xic, wc;
      gll_rule(h->lev[l - 1].p, xic, wc);
      E = flat(lagrange_eval(xic, xi));
    }
    DirFdm fx, fy;
    std::vector<double> dinv;
    const bool single = l > 0 && !wts->elem_params;
    const bool separable = single && wts->local_solve == SEM_LOCAL_SEPARABLE;
    if (l > 0 && wts->elem_params)
      build_segments(h, lv, xb, yb, per, wts->wf, wts->elem_params, mixed);
    if (single) {
      // (the multiplicative method uses no weights: unit weights)
      fx = build_direction(xb, lv.p, lv.n_o, per, wts->wf, wts->alpha_x, h->mult);
      fy = build_direction(yb, lv.p, lv.n_o, per, wts->wf, wts->alpha_y, h->mult);
      if (h->mult) {
        std::vector<int32_t> txo(fx.type_of.begin(), fx.type_of.end()),
            tyo(fy.type_of.begin(), fy.type_of.end());
        lv.tx_of = upload_raw<int32_t>(h->pool, txo);
        lv.ty_of = upload_raw<int32_t>(h->pool, tyo);
      }
      const int m = lv.m;
      lv.ntx = fx.ntypes;
      lv.nty = fy.ntypes;
      std::vector<FdmTask> tasks;
      if (separable) {
        build_separable(lv, xb, yb, per, fx, fy, dinv, tasks);
        lv.ntx = 0;   // pair index = x type = subdomain
        lv.nty = fy.ntypes;
      } else {
        dinv.resize((size_t)fy.ntypes * fx.ntypes * m * m);
        for (int ty = 0; ty < fy.ntypes; ++ty)
          for (int tx = 0; tx < fx.ntypes; ++tx)
            for (int a = 0; a < m; ++a)
              for (int c = 0; c < m; ++c)
                dinv[(((size_t)ty * fx.ntypes + tx) * m + a) * m + c] =
                    1.0 / (fy.lam[(size_t)ty * m + a] + fx.lam[(size_t)tx * m + c]);
        tasks = build_tasks(fx, fy, nx, ny, m);
      }
      lv.ntasks = (int)tasks.size();
      h->pool.emplace_back(new DBuf());
      h->pool.back()->alloc(tasks.size() * sizeof(FdmTask));
      lv.tasks = h->pool.back()->as<FdmTask>();
      HIP_OK(hipMemcpy(lv.tasks, tasks.data(), tasks.size() * sizeof(FdmTask), hipMemcpyHostToDevice));
    }
    // the separable local operators carry nu themselves: no 1/nu_bar scaling
    const std::vector<double> &ninv = (l > 0 && !separable) ? nuinv : std::vector<double>();
    std::vector<double> DTv((size_t)(lv.p + 1) * (lv.p + 1));
    for (int a = 0; a <= lv.p; ++a)
      for (int b = 0; b <= lv.p; ++b) DTv[(size_t)a * (lv.p + 1) + b] = D(b, a);
    upload_tables<double>(h, lv, lv.td, flat(Lh), flat(D), DTv, w, sx, sy, mx, my, single ? &fx : nullptr,
                          single ? &fy : nullptr, dinv, ninv, E);
    if (mixed)
      upload_tables<float>(h, lv, lv.tf, flat(Lh), flat(D), DTv, w, sx, sy, mx, my, single ? &fx : nullptr,
                           single ? &fy : nullptr, dinv, ninv, E);
    if (single && lv.m >= kMfmaMinTile &&
        (h->precision == SEM_MIXED_BF16 || h->precision == SEM_MIXED_FP16))
      lv.mo = build_mfma_ops(h->pool, fy.ST, fy.SW, fy.ntypes, fx.S, fx.ntypes, lv.m,
                             h->precision == SEM_MIXED_FP16);
    // vectors
    const long n = lv.n();
    if (l < L) {
      lv.u = dalloc<double>(h->pool, n);
      lv.f = dalloc<double>(h->pool, n);
    }
    lv.r = dalloc<double>(h->pool, n);
    if (mixed) {
      lv.uf = dalloc<float>(h->pool, n);
      lv.ff = dalloc<float>(h->pool, n);
      lv.rf = dalloc<float>(h->pool, n);
    }
  }
  // coarse solver (level 0, p = 1)
  {
    Level &c = h->lev[0];
    h->cnx = per ? c.g.cols : c.g.cols - 2;
    h->cny = per ? c.g.rows : c.g.rows - 2;
    h->coff = per ? 0 : (long)c.g.cols + 1;
    if (h->varnu) {
      const long n = (long)h->cnx * h->cny;
      if (n > 6000) throw Fail{SEM_EUNSUP, "coarse grid too large for the dense variable-nu solve"};
      Mat B = coarse_dense(c, xb, yb);
      if (per) {
        double tr = 0.0;
        for (long i = 0; i < n; ++i) tr += B(i, i);
        const double s = tr / ((double)n * n);
        for (long i = 0; i < n; ++i)
          for (long j = 0; j < n; ++j) B(i, j) += s;
      }
      if (!spd_inverse(B)) throw Fail{SEM_EINVAL, "coarse operator not positive definite"};
      h->cMinv = upload<double>(h->pool, B.a);
    } else {
      // global fast diagonalisation of A_0 = M_y (x) L_x + L_y (x) M_x
      auto dir = [&](const std::vector<double> &br, int n_un, std::vector<double> &S,
                     std::vector<double> &lam) {
        const int n = (int)br.size() - 1;
        const int N = per ? n : n + 1;
        Mat Lg(N, N);
        Vec Mg(N, 0.0);
        for (int e = 0; e < n; ++e) {
          const double hh = br[e + 1] - br[e];
          const int i0 = e, i1 = per ? (e + 1) % N : e + 1;
          Mg[i0] += 0.5 * hh;
          Mg[i1] += 0.5 * hh;
          Lg(i0, i0) += 1.0 / hh;
          Lg(i1, i1) += 1.0 / hh;
          Lg(i0, i1) -= 1.0 / hh;
          Lg(i1, i0) -= 1.0 / hh;
        }
        const int o = per ? 0 : 1;
        Mat Lu(n_un, n_un);
        Vec Mu(n_un);
        for (int i = 0; i < n_un; ++i) {
          Mu[i] = Mg[i + o];
          for (int j = 0; j < n_un; ++j) Lu(i, j) = Lg(i + o, j + o);
        }
        Mat Sm;
        gen_eig_diag(Lu, Mu, lam, Sm);
        S = Sm.a;
      };
      if (std::max(h->cnx, h->cny) > 2048)
        throw Fail{SEM_EUNSUP, "coarse grid above 2048 unknowns per direction"};
      std::vector<double> Sx, Sy, lx, ly;
      dir(xb, h->cnx, Sx, lx);
      dir(yb, h->cny, Sy, ly);
      std::vector<double> Dv((size_t)h->cny * h->cnx);
      const double lmax = lx.back() + ly.back();
      for (int j = 0; j < h->cny; ++j)
        for (int i = 0; i < h->cnx; ++i) {
          const double s = ly[j] + lx[i];
          Dv[(size_t)j * h->cnx + i] = (per && std::fabs(s) < 1e-12 * lmax) ? 0.0 : 1.0 / s;
        }
      h->cSx = upload<double>(h->pool, Sx);
      h->cSy = upload<double>(h->pool, Sy);
      auto transpose = [](const std::vector<double> &A, int n) {
        std::vector<double> T(A.size());
        for (int a = 0; a < n; ++a)
          for (int b = 0; b < n; ++b) T[(size_t)b * n + a] = A[(size_t)a * n + b];
        return T;
      };
      h->cSxT = upload<double>(h->pool, transpose(Sx, h->cnx));
      h->cSyT = upload<double>(h->pool, transpose(Sy, h->cny));
      h->cDinv = upload<double>(h->pool, Dv);
      h->cT1 = dalloc<double>(h->pool, (size_t)h->cnx * h->cny);
      h->cT2 = dalloc<double>(h->pool, (size_t)h->cnx * h->cny);
    }
    h->cf = dalloc<double>(h->pool, c.n());
    if (mixed) {
      h->cu64 = dalloc<double>(h->pool, c.n());
      h->cf64 = dalloc<double>(h->pool, c.n());
    }
  }
  // PCG vectors
  {
    const long n = h->lev[L].n();
    h->pr = dalloc<double>(h->pool, n);
    h->pp = dalloc<double>(h->pool, n);
    h->pq = dalloc<double>(h->pool, n);
    h->pz = dalloc<double>(h->pool, n);
    h->pro = dalloc<double>(h->pool, n);
    const Grid &gt = h->lev[L].g;
    const long nblk = std::max({residual_blocks(gt, false, 8), residual_blocks(gt, true, 8),
                                residual_blocks(gt, false, 4), residual_blocks(gt, true, 4)});
    h->partial = dalloc<double>(h->pool, std::max<long>(2 * kRedBlocks, nblk));
    h->scal = dalloc<double>(h->pool, 16);
    h->part_rr = dalloc<double>(h->pool, kRedBlocks);
    h->part_d2 = dalloc<double>(h->pool, 2 * kRedBlocks);
    HIP_OK(hipHostMalloc(reinterpret_cast<void **>(&h->pin), 2 * kRedBlocks * sizeof(double),
                         hipHostMallocDefault));
    for (hipEvent_t &e : h->nev) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  if (!noalloc_prepare()) throw Fail{SEM_EHIP, "device symbol lookup failed"};
  HIP_OK(hipDeviceSynchronize());
}

// ---------------------------------------------------------------------------
// Level operations (templated on the working precision)
// ---------------------------------------------------------------------------
template <typename T>
Tables<T> &tabs(Level &L);
template <>
Tables<double> &tabs<double>(Level &L) { return L.td; }
template <>
Tables<float> &tabs<float>(Level &L) { return L.tf; }

// Arms the kernel-timing events for the launches made while it lives, when
// timing is enabled for level l (see sem_timing_enable).
struct TimedLaunch {
  bool on = false;
  TimedLaunch(sem_ctx *h, int l, int kind) {
    if (l != h->time_level || h->ev_used + 2 > h->ev.size()) return;
    launch_timing() = LaunchTiming{h->ev[h->ev_used], h->ev[h->ev_used + 1]};
    h->ev_kind[h->ev_used / 2] = kind;
    h->ev_used += 2;
    on = true;
  }
  ~TimedLaunch() {
    if (on) launch_timing() = LaunchTiming{};
  }
};

template <typename T>
void residual(sem_ctx *h, int l, const T *u, const T *f, T *out, const T *dot_x = nullptr,
              double *dot_res = nullptr) {
  Level &L = h->lev[l];
  Tables<T> &t = tabs<T>(L);
  // the kernels load f and dot_x through one set of registers
  if (f && dot_x) throw Fail{SEM_EINVAL, "residual: right-hand side and dot operand both given"};
  ResidualArgs<T> a{L.g, u, f, out, t.Lhat, t.D, t.DT, t.w, t.sx, t.sy, t.mx, t.my, t.nu, t.nuT,
                    t.gy, t.gx, dot_x, dot_x ? h->partial : nullptr};
  {
    TimedLaunch tl(h, l, f ? SEM_TIME_RESIDUAL : SEM_TIME_APPLY);
    launch_residual<T>(a, h->stream);
  }
  // dot_res = sum of dot_x * out, from the kernel's per-block partial sums
  // (without dot_res they stay in h->partial for the consumer to add)
  if (dot_x && dot_res)
    launch_reduce(h->partial, (int)residual_blocks(L.g, t.nu != nullptr, sizeof(T)), dot_res,
                  h->stream);
}

template <typename T>
FdmTab<T> &seg_tabs(Seg &s);
template <>
FdmTab<double> &seg_tabs<double>(Seg &s) { return s.d; }
template <>
FdmTab<float> &seg_tabs<float>(Seg &s) { return s.f; }
template <typename T>
T *level_dnorm(Level &L);
template <>
double *level_dnorm<double>(Level &L) { return L.dnorm; }
template <>
float *level_dnorm<float>(Level &L) { return L.dnormf; }

template <typename T>
void launch_fdm_prec(sem_ctx *h, const FdmArgs<T> &a) {
  if constexpr (std::is_same<T, float>::value) {
    const bool mfma = h->precision == SEM_MIXED_BF16 || h->precision == SEM_MIXED_FP16;
    if (mfma && a.m >= kMfmaMinTile) {
      launch_fdm_mfma(a, h->precision == SEM_MIXED_FP16, h->stream);
      return;
    }
  }
  launch_fdm<T>(a, h->stream);
}

template <typename T>
void fdm(sem_ctx *h, int l, const T *r, T *u) {
  Level &L = h->lev[l];
  Tables<T> &t = tabs<T>(L);
  if (!L.segs.empty()) {
    // per-element parameters: one launch per overlap value, all adding into u
    TimedLaunch tl(h, l, SEM_TIME_SCHWARZ);
    for (Seg &sg : L.segs) {
      FdmTab<T> &st = seg_tabs<T>(sg);
      FdmArgs<T> a{L.g, sg.n_o, sg.m, sg.tasks, sg.ntasks, r, u, st.Sx, st.SxT, st.SyW, st.SyT,
                   st.dinv, sg.ntx, nullptr, t.nuinv};
      a.wel = st.wel;
      a.dnorm = level_dnorm<T>(L);
      a.mo = sg.mo;
      launch_fdm_prec<T>(h, a);
    }
    return;
  }
  FdmArgs<T> a{L.g, L.n_o, L.m, L.tasks, L.ntasks, r, u, t.Sx, t.SxT, t.SyW, t.SyT, t.dinv, L.ntx,
               t.wx, t.nuinv};
  a.mo = L.mo;
  TimedLaunch tl(h, l, SEM_TIME_SCHWARZ);
  launch_fdm_prec<T>(h, a);
}

// n_it sweeps of Algorithm 1 on level l > 0 (SEM_W_MULT, FP64 only).
void smooth_mult(sem_ctx *h, int l, double *u, const double *f, int n_it) {
  Level &L = h->lev[l];
  Tables<double> &t = L.td;
  MultArgs a{L.g,   L.n_o,  L.m,   n_it,  f,     u,      t.Lhat, t.w,  t.sx,  t.sy,     t.mx,
             t.my,  t.SyW,  t.SyT, t.Sx,  t.SxT, t.dinv, L.ntx,  L.tx_of, L.ty_of};
  TimedLaunch tl(h, l, SEM_TIME_SCHWARZ);
  launch_mult(a, h->stream);
}

// n_it sweeps of Algorithm 2; if u_is_zero the first residual is f itself.
template <typename T>
void smooth(sem_ctx *h, int l, T *u, const T *f, T *rbuf, int n_it, bool u_is_zero) {
  if constexpr (std::is_same<T, double>::value) {
    if (h->mult) {
      smooth_mult(h, l, u, f, n_it);
      return;
    }
  }
  for (int it = 0; it < n_it; ++it) {
    const T *r = f;
    if (!(it == 0 && u_is_zero)) {
      residual<T>(h, l, u, f, rbuf);
      r = rbuf;
    }
    fdm<T>(h, l, r, u);
  }
}

// f_c = I_l^T r_f; uc_zero (optional) is cleared in the same pass.
template <typename T>
void restrict_(sem_ctx *h, int l, const T *rf, T *fc, T *uc_zero) {
  Level &F = h->lev[l], &C = h->lev[l - 1];
  TimedLaunch tl(h, l, SEM_TIME_RESTRICT);
  launch_restrict<T>(F.g, C.g, rf, fc, uc_zero, tabs<T>(F).ET, h->stream);
}

// u_f += I_l u_c
template <typename T>
void prolong_add(sem_ctx *h, int l, const T *uc, T *uf) {
  Level &F = h->lev[l], &C = h->lev[l - 1];
  TimedLaunch tl(h, l, SEM_TIME_PROLONG);
  launch_prolong<T>(F.g, C.g, uc, uf, tabs<T>(F).E, h->stream);
}

// u0 = A_0^+ f0 in FP64.  u0_clear: u0 is already zero at every node (the
// restriction of the V-cycle clears it), so only the unknowns are written.
void coarse_solve64(sem_ctx *h, const double *f0, double *u0, bool u0_clear = false) {
  Level &c = h->lev[0];
  hipStream_t s = h->stream;
  const double *f = f0;
  if (c.g.periodic) {
    HIP_OK(hipMemcpyAsync(h->cf, f0, c.n() * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_sum(h->cf, c.n(), h->partial, h->scal + 8, s);
    launch_sub_mean(c.g, h->cf, h->scal + 8, s);
    f = h->cf;
  }
  const int nx = h->cnx, ny = h->cny;
  const long ld = c.g.cols;
  if (nx == 0 || ny == 0) {  // no coarse unknowns (one Dirichlet element)
    if (!u0_clear) launch_fill<double>(u0, c.n(), 0.0, s);
    return;
  }
  if (!u0_clear) launch_fill<double>(u0, c.n(), 0.0, s);
  if (h->cMinv) {
    launch_dense_matvec<double>(nx * ny, h->cMinv, f, h->coff, (int)ld, nx, u0, s);
  } else if (nx <= kSandwichMax && ny <= kSandwichMax) {
    // T2 = (S_y^T F S_x) .* Dinv ; U = S_y T2 S_x^T, one launch each
    // L(i, k) = S_y(k, i) read from S_y itself (lrs = 1); S_y and S_x^T read
    // through the stored transposes, so that every operand read is coalesced
    launch_sandwich<double, double>(ny, nx, h->cSy, 1, ny, f + h->coff, ld, h->cSx, nx, 1,
                                    h->cDinv, nx, h->cT2, nx, s);
    launch_sandwich<double, double>(ny, nx, h->cSyT, 1, ny, h->cT2, nx, h->cSxT, nx, 1, nullptr,
                                    0, u0 + h->coff, ld, s);
  } else {
    // T1 = S_y^T F ; T2 = (T1 S_x) .* Dinv ; T3 = S_y T2 ; U = T3 S_x^T
    launch_gemm(ny, nx, ny, h->cSy, 1, ny, f + h->coff, ld, 1, h->cT1, nx, nullptr, 0, s);
    launch_gemm(ny, nx, nx, h->cT1, nx, 1, h->cSx, nx, 1, h->cT2, nx, h->cDinv, nx, s);
    launch_gemm(ny, nx, ny, h->cSy, ny, 1, h->cT2, nx, 1, h->cT1, nx, nullptr, 0, s);
    launch_gemm(ny, nx, nx, h->cT1, nx, 1, h->cSx, 1, nx, u0 + h->coff, ld, nullptr, 0, s);
  }
  if (c.g.periodic) {
    launch_sum(u0, c.n(), h->partial, h->scal + 8, s);
    launch_sub_mean(c.g, u0, h->scal + 8, s);
  }
}

void coarse_solve(sem_ctx *h, const double *f0, double *u0, bool u0_clear) {
  coarse_solve64(h, f0, u0, u0_clear);
}
// The FP32 cycle's coarse solve: FP64 arithmetic read from and written to the
// FP32 arrays directly where the problem has no mean to project out; through
// FP64 copies otherwise.
void coarse_solve(sem_ctx *h, const float *f0, float *u0, bool u0_clear) {
  Level &c = h->lev[0];
  hipStream_t s = h->stream;
  const long n = c.n(), ld = c.g.cols;
  const int nx = h->cnx, ny = h->cny;
  const bool direct = !c.g.periodic && nx > 0 && ny > 0 &&
                      (h->cMinv || (nx <= kSandwichMax && ny <= kSandwichMax));
  if (direct) {
    if (!u0_clear) launch_fill<float>(u0, n, 0.0f, s);
    if (h->cMinv) {
      launch_dense_matvec<float>(nx * ny, h->cMinv, f0, h->coff, (int)ld, nx, u0, s);
    } else {
      launch_sandwich<float, double>(ny, nx, h->cSy, 1, ny, f0 + h->coff, ld, h->cSx, nx, 1,
                                     h->cDinv, nx, h->cT2, nx, s);
      launch_sandwich<double, float>(ny, nx, h->cSyT, 1, ny, h->cT2, nx, h->cSxT, nx, 1, nullptr,
                                     0, u0 + h->coff, ld, s);
    }
    return;
  }
  launch_convert<float, double>(f0, h->cf64, n, 1.0, s);
  coarse_solve64(h, h->cf64, h->cu64);
  launch_convert<double, float>(h->cu64, u0, n, 1.0, s);
}

template <typename T>
struct LevelVecs {
  static T *u(Level &L) { return L.u; }
  static T *f(Level &L) { return L.f; }
  static T *r(Level &L) { return L.r; }
};
template <>
struct LevelVecs<float> {
  static float *u(Level &L) { return L.uf; }
  static float *f(Level &L) { return L.ff; }
  static float *r(Level &L) { return L.rf; }
};

// Algorithm 3 on arrays of precision T.  uL/fL are the top-level arrays;
// u_zero tells that uL is zero on entry.
template <typename T>
void vcycle_impl(sem_ctx *h, T *uL, const T *fL, const int32_t *ns1, const int32_t *ns2,
                 bool u_zero) {
  using V = LevelVecs<T>;
  const int L = (int)h->lev.size() - 1;
  std::vector<T *> u(L + 1);
  std::vector<const T *> f(L + 1);
  u[L] = uL;
  f[L] = fL;
  for (int l = L; l >= 1; --l) {
    Level &lv = h->lev[l];
    const bool zero = (l < L) || u_zero;  // u_l was cleared by the restriction above it
    if (l < L) u[l] = V::u(lv);
    const int n1 = ns1 ? ns1[l] : 1;
    smooth<T>(h, l, u[l], f[l], V::r(lv), n1, zero);
    const T *rr = f[l];
    if (!(zero && n1 == 0)) {
      residual<T>(h, l, u[l], f[l], V::r(lv));
      rr = V::r(lv);
    }
    Level &cl = h->lev[l - 1];
    T *fc = V::f(cl);
    // the restriction also clears the next level's correction (level 0
    // included: the coarse solve then writes only the unknowns)
    restrict_<T>(h, l, rr, fc, V::u(cl));
    f[l - 1] = fc;
  }
  // with a single level (p = 1) the cycle is the coarse solve on the caller's array
  if (L > 0) u[0] = V::u(h->lev[0]);
  coarse_solve(h, f[0], u[0], L > 0);
  for (int l = 1; l <= L; ++l) {
    Level &lv = h->lev[l];
    if (l < L) u[l] = V::u(lv);
    prolong_add<T>(h, l, u[l - 1], u[l]);
    smooth<T>(h, l, u[l], f[l], V::r(lv), ns2 ? ns2[l] : 0, false);
  }
}

// Preconditioner z = MG(0, r) in the handle's precision (FP64 in, FP64 out).
// prepared: the cycle's inputs were already written by the CG update (r in
// FP32 and a zero initial guess).  d2_part (mixed precision only): when
// non-null, the partial sums of z.(r - ro) and z.r (launch_dot2_partials'
// layout) come out of the pass that converts z back to FP64.
void precondition(sem_ctx *h, const double *r, double *z, const int32_t *ns1, const int32_t *ns2,
                  bool prepared = false, const double *ro = nullptr, double *d2_part = nullptr) {
  Level &top = h->lev.back();
  const long n = top.n();
  if (h->precision != SEM_FP64) {
    if (!prepared) {
      launch_convert<double, float>(r, top.ff, n, 1.0, h->stream);
      launch_fill<float>(top.uf, n, 0.0f, h->stream);
    }
    vcycle_impl<float>(h, top.uf, top.ff, ns1, ns2, true);
    if (d2_part)
      launch_convert_dot2_partials(top.uf, z, r, ro, n, d2_part, h->stream);
    else
      launch_convert<float, double>(top.uf, z, n, 1.0, h->stream);
  } else {
    if (!prepared) launch_fill<double>(z, n, 0.0, h->stream);
    vcycle_impl<double>(h, z, r, ns1, ns2, true);
  }
}

double read_scalar(sem_ctx *h, const double *d) {
  double v;
  HIP_OK(hipMemcpyAsync(&v, d, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_OK(hipStreamSynchronize(h->stream));
  return v;
}

}  // namespace

// ---------------------------------------------------------------------------
// C entry points
// ---------------------------------------------------------------------------
namespace {
sem_status guard(sem_ctx *h, const std::function<void()> &fn) {
  try {
    fn();
    if (h) {
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) throw Fail{SEM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e)};
    }
    return SEM_OK;
  } catch (const Fail &f) {
    if (h) h->err = f.msg;
    return f.s;
  } catch (const std::bad_alloc &) {
    if (h) h->err = "host allocation failed";
    return SEM_ENOMEM;
  } catch (const std::exception &e) {
    if (h) h->err = e.what();
    return SEM_EINVAL;
  }
}
thread_local std::string g_setup_err;
}  // namespace

extern "C" {

sem_status sem_setup(const sem_mesh *mesh, int32_t p, const sem_overlap *overlap,
                     const sem_weights *weights, const double *nu, int32_t precision,
                     void *stream, sem_handle *out) {
  if (!out) return SEM_EINVAL;
  *out = nullptr;
  auto *h = new (std::nothrow) sem_ctx();
  if (!h) return SEM_ENOMEM;
  h->stream = static_cast<hipStream_t>(stream);
  if (precision != SEM_FP64 && precision != SEM_MIXED_FP32 && precision != SEM_MIXED_BF16 &&
      precision != SEM_MIXED_FP16) {
    g_setup_err = "unknown precision";
    delete h;
    return SEM_EINVAL;
  }
  h->precision = precision;
  sem_status s = guard(h, [&] { setup_impl(h, mesh, p, overlap, weights, nu); });
  if (s != SEM_OK) {
    g_setup_err = h->err;
    delete h;
    return s;
  }
  *out = h;
  return SEM_OK;
}

sem_status sem_destroy(sem_handle h) {
  if (!h) return SEM_EINVAL;
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return SEM_OK;
}

sem_status sem_num_levels(sem_handle h, int32_t *nlevels) {
  if (!h || !nlevels) return SEM_EINVAL;
  *nlevels = (int32_t)h->lev.size();
  return SEM_OK;
}

sem_status sem_level_info(sem_handle h, int32_t level, int32_t *p_l, int32_t *n_o, int64_t *rows,
                          int64_t *cols) {
  if (!h || level < 0 || level >= (int)h->lev.size()) return SEM_EINVAL;
  const Level &L = h->lev[level];
  if (p_l) *p_l = L.p;
  if (n_o) *n_o = L.n_o;
  if (rows) *rows = L.g.rows;
  if (cols) *cols = L.g.cols;
  return SEM_OK;
}

sem_status sem_node_coords(sem_handle h, int32_t level, double *x, double *y) {
  if (!h || level < 0 || level >= (int)h->lev.size() || !x || !y) return SEM_EINVAL;
  const Level &L = h->lev[level];
  std::copy(L.xc.begin(), L.xc.end(), x);
  std::copy(L.yc.begin(), L.yc.end(), y);
  return SEM_OK;
}

sem_status sem_mass(sem_handle h, const double *f_nodal, double *b) {
  if (!h || !f_nodal || !b) return SEM_EINVAL;
  return guard(h, [&] {
    Level &L = h->lev.back();
    launch_mass<double>(L.g, f_nodal, b, L.td.w, L.td.mx, L.td.my, h->stream);
  });
}

sem_status sem_residual(sem_handle h, int32_t level, const double *u, const double *f, double *r) {
  if (!h || !u || !r || level < 0 || level >= (int)h->lev.size()) return SEM_EINVAL;
  return guard(h, [&] { residual<double>(h, level, u, f, r); });
}

sem_status sem_schwarz_smooth(sem_handle h, int32_t level, double *u, const double *f, int32_t n_it) {
  if (!h || !u || !f || level < 1 || level >= (int)h->lev.size() || n_it < 0) return SEM_EINVAL;
  return guard(h, [&] {
    Level &L = h->lev[level];
    launch_zero_boundary<double>(L.g, u, h->stream);
    smooth<double>(h, level, u, f, L.r, n_it, false);
  });
}

sem_status sem_restrict(sem_handle h, int32_t level, const double *r_fine, double *f_coarse) {
  if (!h || !r_fine || !f_coarse || level < 1 || level >= (int)h->lev.size()) return SEM_EINVAL;
  return guard(h, [&] { restrict_<double>(h, level, r_fine, f_coarse, nullptr); });
}

sem_status sem_prolong_add(sem_handle h, int32_t level, const double *u_coarse, double *u_fine) {
  if (!h || !u_coarse || !u_fine || level < 1 || level >= (int)h->lev.size()) return SEM_EINVAL;
  return guard(h, [&] { prolong_add<double>(h, level, u_coarse, u_fine); });
}

sem_status sem_coarse_solve(sem_handle h, const double *f0, double *u0) {
  if (!h || !f0 || !u0) return SEM_EINVAL;
  return guard(h, [&] { coarse_solve64(h, f0, u0); });
}

sem_status sem_vcycle(sem_handle h, double *u, const double *f, const int32_t *ns1,
                      const int32_t *ns2) {
  if (!h || !u || !f) return SEM_EINVAL;
  return guard(h, [&] {
    Level &top = h->lev.back();
    launch_zero_boundary<double>(top.g, u, h->stream);
    if (h->precision != SEM_FP64) {
      // MG(u, f) = u + MG(0, f - A u): residual in FP64, cycle in FP32
      residual<double>(h, (int)h->lev.size() - 1, u, f, h->pr);
      precondition(h, h->pr, h->pz, ns1, ns2);
      launch_axpy(1.0, h->pz, u, top.n(), h->stream);
    } else {
      vcycle_impl<double>(h, u, f, ns1, ns2, false);
    }
  });
}

sem_status sem_pcg_solve(sem_handle h, double *u, const double *f, int32_t imax, double rtol,
                         const int32_t *ns1, const int32_t *ns2, int32_t *iters, double *res_hist) {
  if (!h || !u || !f || imax < 0) return SEM_EINVAL;
  sem_status conv = SEM_OK;
  sem_status s = guard(h, [&] {
    Level &top = h->lev.back();
    const int L = (int)h->lev.size() - 1;
    const long n = top.n();
    hipStream_t st = h->stream;
    double *r = h->pr, *p = h->pp, *q = h->pq, *z = h->pz, *ro = h->pro;
    // device scalars: [0], [7] delta (alternating), [2] r.r, [8] sums
    double *sc = h->scal;
    launch_zero_boundary<double>(top.g, u, st);
    const double *fp = f;
    if (top.g.periodic) {
      // project the right side onto the range of A (remove its mean); q is
      // free until the loop starts
      HIP_OK(hipMemcpyAsync(q, f, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      launch_sum(q, n, h->partial, sc + 8, st);
      launch_sub_mean(top.g, q, sc + 8, st);
      fp = q;
    }
    residual<double>(h, L, u, fp, r);
    launch_dot(r, r, n, h->partial, sc + 2, st);
    const double r0 = std::sqrt(read_scalar(h, sc + 2));
    if (!std::isfinite(r0)) throw Fail{SEM_ENAN, "non-finite initial residual"};
    if (res_hist) res_hist[0] = r0;
    if (r0 == 0.0) {   // u is already the solution: no iteration (and no 0/0 in alpha)
      if (iters) *iters = 0;
      return;
    }
    precondition(h, r, p, ns1, ns2);
    launch_dot(p, r, n, h->partial, sc + 0, st);
    // The stopping test of iteration k needs ||r_k|| on the host.  Its copy
    // into pinned memory is queued behind the update, and, unless the
    // residual history predicts that this test will pass, the next
    // iteration's preconditioner, direction and A p (which write only z, p,
    // r_old, q and scalars, never u or r) are queued before the host waits
    // for it, so the device does not idle during the round trip.  When the
    // test passes, queued work is discarded; u and r are final.
    // No reduction has a launch of its own: the kernels that consume a dot
    // product add its partial sums themselves (fixed order), and the host
    // adds the r.r partials it copies for the stopping test.
    const int npq = (int)residual_blocks(top.g, top.td.nu != nullptr, sizeof(double));
    auto q_and_pq = [&] {
      residual<double>(h, L, p, nullptr, q, p);   // q = A p; p.q partials in h->partial
    };
    const bool mixed = h->precision != SEM_FP64;
    double *delta = sc + 0, *delta_next = sc + 7;   // z.r, alternating between two slots
    auto next_direction = [&] {
      // the update below already wrote the cycle's inputs (prepared)
      precondition(h, r, z, ns1, ns2, true, ro, mixed ? h->part_d2 : nullptr);
      if (!mixed) launch_dot2_partials(z, r, ro, n, h->part_d2, st);   // z.(r - r_old), z.r
      // beta = z.(r - r_old) / delta; p = z + beta p; next delta = z.r
      launch_cg_direction2(h->part_d2, delta, delta_next, p, z, n, st);
      std::swap(delta, delta_next);
    };
    int it = 0;
    bool done = false;
    double prev1 = r0, prev2 = 0.0;   // the last two residual norms
    if (!done && imax > 0) q_and_pq();
    for (it = 1; it <= imax && !done; ++it) {
      // alpha = delta / p.q; also writes the next cycle's inputs
      // the new residual goes into the buffer of the one before the current
      // one, and the current one becomes r_old (Algorithm 4's first r_old is zero)
      const int nrr = launch_cg_update2(delta, h->partial, npq, u, p, r, ro, q, n, h->part_rr,
                                        st, mixed ? top.ff : nullptr, mixed ? top.uf : nullptr,
                                        mixed ? nullptr : z);
      std::swap(r, ro);
      if (it == 1) launch_fill<double>(ro, n, 0.0, st);
      double *slot = h->pin + (size_t)(it & 1) * kRedBlocks;
      HIP_OK(hipMemcpyAsync(slot, h->part_rr, nrr * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_OK(hipEventRecord(h->nev[it & 1], st));
      // predicted ||r_k|| from the last two reductions
      const double pred = prev2 > 0.0 ? prev1 * (prev1 / prev2) : prev1;
      const bool ahead = it < imax && !(pred <= 4.0 * rtol * r0);
      if (ahead) {
        next_direction();
        q_and_pq();
      }
      HIP_OK(hipEventSynchronize(h->nev[it & 1]));
      double rr = 0.0;   // the partials in a fixed order
      for (int b = 0; b < nrr; ++b) rr += slot[b];
      const double rn = std::sqrt(rr);
      if (res_hist) res_hist[it] = rn;
      if (!std::isfinite(rn)) throw Fail{SEM_ENAN, "non-finite residual"};
      if (rn <= rtol * r0) {
        done = true;
        break;
      }
      if (!ahead && it < imax) {
        next_direction();
        q_and_pq();
      }
      prev2 = prev1;
      prev1 = rn;
    }
    if (iters) *iters = done ? std::min(it, imax) : imax;
    if (!done) conv = SEM_ENOCONV;
  });
  if (s != SEM_OK) return s;
  if (conv != SEM_OK) h->err = "imax reached";
  return conv;
}

sem_status sem_timing_enable(sem_handle h, int32_t level, int32_t on) {
  if (!h || level < 1 || level >= (int)h->lev.size()) return SEM_EINVAL;
  return guard(h, [&] {
    if (on) {
      if (h->ev.empty()) {
        h->ev.resize(2 * 65536);
        h->ev_kind.assign(65536, 0);
        for (auto &e : h->ev) HIP_OK(hipEventCreate(&e));
      }
      h->time_level = level;
    } else {
      h->time_level = -1;
    }
    h->ev_used = 0;
  });
}

sem_status sem_timing_read_all(sem_handle h, int64_t *count, double *total_ms) {
  if (!h || !count || !total_ms) return SEM_EINVAL;
  return guard(h, [&] {
    HIP_OK(hipStreamSynchronize(h->stream));
    for (int k = 0; k < SEM_TIME_KINDS; ++k) {
      count[k] = 0;
      total_ms[k] = 0.0;
    }
    for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
      float ms = 0.0f;
      HIP_OK(hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]));
      const int k = h->ev_kind[i / 2];
      count[k] += 1;
      total_ms[k] += ms;
    }
    h->ev_used = 0;
  });
}

sem_status sem_timing_read(sem_handle h, int64_t *count, double *total_ms) {
  if (!h || !count || !total_ms) return SEM_EINVAL;
  int64_t c[SEM_TIME_KINDS];
  double t[SEM_TIME_KINDS];
  const sem_status st = sem_timing_read_all(h, c, t);
  if (st != SEM_OK) return st;
  *count = c[SEM_TIME_SCHWARZ];
  *total_ms = t[SEM_TIME_SCHWARZ];
  return SEM_OK;
}

sem_status sem_elem_features(sem_handle h, float *feat) {
  if (!h || !feat) return SEM_EINVAL;
  return guard(h, [&] {
    Level &top = h->lev.back();
    launch_features(top.g, h->enu, h->enuinv, h->hx, h->hy, feat,
                    h->stream);
  });
}

}  // extern "C"

namespace sem {
bool handle_top(sem_handle h, hipStream_t *stream, long *nodes) {
  if (!h || h->lev.empty()) return false;
  *stream = h->stream;
  *nodes = h->lev.back().n();
  return true;
}
void handle_error(sem_handle h, const char *msg) {
  if (h) h->err = msg;
}
}  // namespace sem

extern "C" {

sem_status sem_norm(sem_handle h, const double *x, double *out) {
  if (!h || !x || !out) return SEM_EINVAL;
  return guard(h, [&] {
    Level &top = h->lev.back();
    launch_dot(x, x, top.n(), h->partial, h->scal + 10, h->stream);
    *out = std::sqrt(read_scalar(h, h->scal + 10));
  });
}

const char *sem_strerror(sem_status s) {
  switch (s) {
    case SEM_OK: return "ok";
    case SEM_EINVAL: return "invalid argument";
    case SEM_EDOM: return "argument outside the domain (breaks or nu)";
    case SEM_ENOMEM: return "out of memory";
    case SEM_EHIP: return "HIP runtime error";
    case SEM_ENOCONV: return "no convergence within imax";
    case SEM_ENAN: return "non-finite value";
    case SEM_EUNSUP: return "unsupported by this library";
  }
  return "unknown status";
}

const char *sem_last_error(sem_handle h) { return h ? h->err.c_str() : g_setup_err.c_str(); }

}  // extern "C"
