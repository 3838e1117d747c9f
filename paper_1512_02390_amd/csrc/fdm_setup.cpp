// Subdomain types along one direction of a tensor-product mesh: restricted
// 1-D operators, their fast-diagonalisation factors and the 1-D weights
// (Section 3.1).  Shared by the 2-D and 3-D set-ups.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/sem.h"
#include "host_math.h"
#include "internal.h"

namespace sem {

// Subdomain types, factors and weights along one direction (Section 3.1).
DirFdm build_direction(const std::vector<double> &br, int p, int n_o, int periodic, int wf,
                       const double *alpha, bool unweighted) {
  const int n = (int)br.size() - 1;
  const int m = p + 1 + 2 * n_o;
  const int N = periodic ? n * p : n * p + 1;
  Vec xi, w;
  gll_rule(p, xi, w);
  Mat Lh = ref_stiffness(p);
  DirFdm out;
  out.type_of.assign(n, -1);
  out.wts.assign((size_t)n * m, 0.0);
  std::vector<std::vector<double>> sigL, sigM;  // signatures of known types
  std::vector<std::vector<char>> sigV;
  std::vector<std::vector<double>> sigW;
  // multiplicity of every node over the 1-D subdomains (arithmetic weights)
  std::vector<int> count(N, 0);
  auto glob = [&](int e, int k, bool &valid) {
    int g = e * p - n_o + k;
    if (periodic) {
      g = ((g % N) + N) % N;
      valid = true;
    } else {
      valid = g >= 1 && g <= N - 2;
    }
    return g;
  };
  for (int e = 0; e < n; ++e)
    for (int k = 0; k < m; ++k) {
      bool v;
      int g = glob(e, k, v);
      if (v) count[g]++;
    }
  const double delta = xi[n_o + 1] + 1.0;
  for (int e = 0; e < n; ++e) {
    // restricted 1-D stiffness and mass on the window [e p - n_o, (e+1) p + n_o]
    Mat Ls(m, m);
    Vec Ms(m, 0.0);
    std::vector<char> valid(m);
    for (int k = 0; k < m; ++k) {
      bool v;
      glob(e, k, v);
      valid[k] = v;
    }
    for (int d = -1; d <= 1; ++d) {
      int E = e + d;
      if (!periodic && (E < 0 || E >= n)) continue;
      int Ew = periodic ? (E + n) % n : E;
      const double h = br[Ew + 1] - br[Ew];
      for (int a = 0; a <= p; ++a) {
        const int ka = d * p + a + n_o;
        if (ka < 0 || ka >= m) continue;
        Ms[ka] += 0.5 * h * w[a];
        for (int b = 0; b <= p; ++b) {
          const int kb = d * p + b + n_o;
          if (kb < 0 || kb >= m) continue;
          Ls(ka, kb) += (2.0 / h) * Lh(a, b);
        }
      }
    }
    // weights of this subdomain (eq. weight function, or counting for w_a)
    std::vector<double> we(m, 0.0);
    {
      const double al = alpha ? alpha[e] : 1.0;
      const double ar = alpha ? alpha[periodic && e == n - 1 ? 0 : e + 1] : 1.0;
      for (int k = 0; k < m; ++k) {
        bool v;
        int g = glob(e, k, v);
        if (!v) continue;
        if (unweighted) {
          we[k] = 1.0;   // per-element weights are applied by the kernel
        } else if (wf == SEM_W_ARITH) {
          we[k] = 1.0 / count[g];
        } else {
          const int t = k - n_o;
          const double x = t < 0 ? xi[p + t] - 2.0 : (t > p ? xi[t - p] + 2.0 : xi[t]);
          const bool satl = !periodic && e == 0, satr = !periodic && e == n - 1;
          we[k] = weight_fn(wf, x, al * delta, ar * delta, satl, satr);
        }
      }
    }
    // signature and type lookup (equal matrices to 1e-12, equal weights)
    std::vector<double> sl, sm;
    for (int i = 0; i < m; ++i) {
      sm.push_back(valid[i] ? Ms[i] : 0.0);
      for (int j = 0; j < m; ++j) sl.push_back(valid[i] && valid[j] ? Ls(i, j) : 0.0);
    }
    int type = -1;
    for (int t = 0; t < out.ntypes && type < 0; ++t) {
      if (sigV[t] != valid) continue;
      double dmax = 0.0, smax = 0.0;
      for (size_t i = 0; i < sl.size(); ++i) {
        dmax = std::max(dmax, std::fabs(sl[i] - sigL[t][i]));
        smax = std::max(smax, std::fabs(sl[i]));
      }
      for (size_t i = 0; i < sm.size(); ++i) {
        dmax = std::max(dmax, std::fabs(sm[i] - sigM[t][i]) * smax / (std::fabs(sm[i]) + 1e-300));
      }
      double wmax = 0.0;
      for (int i = 0; i < m; ++i) wmax = std::max(wmax, std::fabs(we[i] - sigW[t][i]));
      if (dmax <= 1e-12 * smax && wmax <= 1e-15) type = t;
    }
    if (type < 0) {
      type = out.ntypes++;
      sigL.push_back(sl);
      sigM.push_back(sm);
      sigV.push_back(valid);
      sigW.push_back(we);
      // generalised eigenproblem on the valid positions, padded with identity
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
      std::vector<double> Sp((size_t)m * m, 0.0), lp(m, 1.0);
      for (int a = 0; a < nv; ++a) {
        lp[a] = lam[a];
        for (int c = 0; c < nv; ++c) Sp[(size_t)vi[a] * m + c] = S(a, c);
      }
      for (size_t t = 0; t < ii.size(); ++t) Sp[(size_t)ii[t] * m + nv + t] = 1.0;
      out.S.insert(out.S.end(), Sp.begin(), Sp.end());
      for (int a = 0; a < m; ++a)
        for (int c = 0; c < m; ++c) out.ST.push_back(Sp[(size_t)c * m + a]);
      for (int a = 0; a < m; ++a)
        for (int c = 0; c < m; ++c) out.SW.push_back(we[a] * Sp[(size_t)a * m + c]);
      out.lam.insert(out.lam.end(), lp.begin(), lp.end());
    }
    out.type_of[e] = type;
    std::copy(we.begin(), we.end(), out.wts.begin() + (size_t)e * m);
  }
  return out;
}

}  // namespace sem
