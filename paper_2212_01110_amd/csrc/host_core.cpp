// Host-only parts of the library (no HIP); see host_core.h.
#include "host_core.h"

#include <cmath>
#include <limits>

namespace spk {

namespace {

bool is_finite(double v) { return std::isfinite(v); }

// ---- small dense FP64 helpers (row-major)
// C[m][n] (+)= A[m][k] * B[k][n]
void gemm(int m, int n, int k, const double* A, const double* B, double* C, bool acc) {
  if (!acc) std::fill(C, C + (size_t)m * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int l = 0; l < k; ++l) {
      const double a = A[(size_t)i * k + l];
      if (a == 0.0) continue;
      const double* b = B + (size_t)l * n;
      double* c = C + (size_t)i * n;
      for (int j = 0; j < n; ++j) c[j] += a * b[j];
    }
}
// C[m][n] (+)= A[k][m]' * B[k][n]
void gemm_tn(int m, int n, int k, const double* A, const double* B, double* C, bool acc) {
  if (!acc) std::fill(C, C + (size_t)m * n, 0.0);
  for (int l = 0; l < k; ++l)
    for (int i = 0; i < m; ++i) {
      const double a = A[(size_t)l * m + i];
      if (a == 0.0) continue;
      const double* b = B + (size_t)l * n;
      double* c = C + (size_t)i * n;
      for (int j = 0; j < n; ++j) c[j] += a * b[j];
    }
}
// In-place Cholesky (lower) of an SPD n x n matrix; false if not SPD.
bool cholesky(int n, double* A) {
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(d > 0.0) || !is_finite(d)) return false;
    d = std::sqrt(d);
    A[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = s / d;
    }
  }
  return true;
}
// Inverse of an SPD matrix from its lower Cholesky factor Lc.
void chol_inverse(int n, const double* Lc, double* Inv) {
  std::vector<double> col(n);
  for (int e = 0; e < n; ++e) {
    std::fill(col.begin(), col.end(), 0.0);
    col[e] = 1.0;
    for (int i = 0; i < n; ++i) {  // L y = e
      double s = col[i];
      for (int k = 0; k < i; ++k) s -= Lc[(size_t)i * n + k] * col[k];
      col[i] = s / Lc[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {  // L' x = y
      double s = col[i];
      for (int k = i + 1; k < n; ++k) s -= Lc[(size_t)k * n + i] * col[k];
      col[i] = s / Lc[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) Inv[(size_t)i * n + e] = col[i];
  }
}

// ---- exact nested AV@R cost of a trajectory (eq. original-problem)
double avar_exact(const std::vector<double>& Z, const std::vector<double>& p, double a) {
  if (a == 0.0) return *std::max_element(Z.begin(), Z.end());
  double best = std::numeric_limits<double>::infinity();
  for (double t : Z) {
    double s = 0;
    for (size_t k = 0; k < Z.size(); ++k) s += p[k] * std::max(Z[k] - t, 0.0);
    best = std::min(best, t + s / a);
  }
  return best;
}

}  // namespace

double nested_cost(const Tree& T, int nx, int nu, const double* q, const double* r, const double* qN,
                   const double* a_risk, const std::vector<double>& x, const std::vector<double>& u) {
  std::vector<double> V(T.nn, 0.0);
  for (int j = T.nl; j < T.nn; ++j) {
    double s = 0;
    for (int k = 0; k < nx; ++k) s += qN[(size_t)j * nx + k] * x[(size_t)j * nx + k] * x[(size_t)j * nx + k];
    V[j] = s;
  }
  for (int i = T.nl - 1; i >= 0; --i) {
    std::vector<double> Z, p;
    for (int c = T.fc[i]; c < T.fc[i] + T.nch[i]; ++c) {
      double l = V[c];
      for (int k = 0; k < nx; ++k) l += q[(size_t)c * nx + k] * x[(size_t)i * nx + k] * x[(size_t)i * nx + k];
      for (int k = 0; k < nu; ++k) l += r[(size_t)c * nu + k] * u[(size_t)i * nu + k] * u[(size_t)i * nu + k];
      Z.push_back(l);
      p.push_back(T.pcond[c]);
    }
    V[i] = avar_exact(Z, p, a_risk[i]);
  }
  return V[0];
}

int build_tree(int32_t nn, const int32_t* anc, const double* prob, Tree& T) {
  if (!anc || !prob || nn < 2) return SPOCK_EINVAL;
  T = Tree{};
  T.nn = nn;
  T.anc.assign(anc, anc + nn);
  T.prob.assign(prob, prob + nn);
  if (T.anc[0] != -1) return SPOCK_ETREE;
  T.stage.assign(nn, 0);
  T.nch.assign(nn, 0);
  T.fc.assign(nn, -1);
  for (int i = 1; i < nn; ++i) {
    const int a = T.anc[i];
    if (a < 0 || a >= i) return SPOCK_ETREE;
    if (a < T.anc[i - 1]) return SPOCK_ETREE;  // breadth-first: ancestors nondecreasing
    T.stage[i] = T.stage[a] + 1;
    if (T.stage[i] < T.stage[i - 1]) return SPOCK_ETREE;
    if (T.nch[a] == 0) T.fc[a] = i;
    T.nch[a]++;
  }
  T.N = T.stage[nn - 1];
  T.nl = 0;
  for (int i = 0; i < nn; ++i) {
    if (T.nch[i] > 0) {
      if (i != T.nl) return SPOCK_ETREE;  // nonleaf nodes must precede leaves
      T.nl++;
    } else if (T.stage[i] != T.N) {
      return SPOCK_ETREE;  // leaves only at the last stage
    }
  }
  if (T.N < 1) return SPOCK_ETREE;
  T.stage_off.assign(T.N + 2, nn);
  for (int i = nn - 1; i >= 0; --i) T.stage_off[T.stage[i]] = i;
  T.stage_off[T.N + 1] = nn;
  // probabilities
  for (int i = 0; i < nn; ++i)
    if (!(T.prob[i] > 0.0) || !is_finite(T.prob[i])) return SPOCK_EPROB;
  if (std::fabs(T.prob[0] - 1.0) > 1e-10) return SPOCK_EPROB;
  T.pcond.assign(nn, 1.0);
  for (int i = 0; i < T.nl; ++i) {
    double s = 0;
    for (int c = T.fc[i]; c < T.fc[i] + T.nch[i]; ++c) s += T.prob[c];
    if (std::fabs(s - T.prob[i]) > 1e-10 * T.prob[i]) return SPOCK_EPROB;
    for (int c = T.fc[i]; c < T.fc[i] + T.nch[i]; ++c) T.pcond[c] = T.prob[c] / T.prob[i];
  }
  return SPOCK_OK;
}

int check_problem_data(const Tree& T, const spock_problem_data& dd) {
  const spock_problem_data* d = &dd;
  const int nn = T.nn, nl = T.nl, nx = d->nx, nu = d->nu;
  // data checks
  for (int c = 1; c < nn; ++c) {
    for (int e = 0; e < nx * nx; ++e) if (!is_finite(d->A[(size_t)c * nx * nx + e])) return SPOCK_EINVAL;
    for (int e = 0; e < nx * nu; ++e) if (!is_finite(d->B[(size_t)c * nx * nu + e])) return SPOCK_EINVAL;
    for (int k = 0; k < nx; ++k) if (!(d->q[(size_t)c * nx + k] > 0.0) || !is_finite(d->q[(size_t)c * nx + k])) return SPOCK_EINVAL;
    for (int k = 0; k < nu; ++k) if (!(d->r[(size_t)c * nu + k] > 0.0) || !is_finite(d->r[(size_t)c * nu + k])) return SPOCK_EINVAL;
  }
  for (int j = nl; j < nn; ++j)
    for (int k = 0; k < nx; ++k) if (!(d->qN[(size_t)j * nx + k] >= 0.0) || !is_finite(d->qN[(size_t)j * nx + k])) return SPOCK_EINVAL;
  for (int i = 0; i < nn; ++i)
    for (int k = 0; k < nx; ++k) {
      const double lo = d->xmin[(size_t)i * nx + k], hi = d->xmax[(size_t)i * nx + k];
      if (std::isnan(lo) || std::isnan(hi) || lo > hi) return SPOCK_EBOX;
    }
  for (int i = 0; i < nl; ++i) {
    for (int k = 0; k < nu; ++k) {
      const double lo = d->umin[(size_t)i * nu + k], hi = d->umax[(size_t)i * nu + k];
      if (std::isnan(lo) || std::isnan(hi) || lo > hi) return SPOCK_EBOX;
    }
    if (!(d->a_risk[i] >= 0.0 && d->a_risk[i] <= 1.0)) return SPOCK_EINVAL;
  }

  return SPOCK_OK;
}

int factor_alg1(const Tree& T, const spock_problem_data& dd, Factor& F) {
  const spock_problem_data* d = &dd;
  const int nn = T.nn, nl = T.nl, nx = d->nx, nu = d->nu;
  // ---- Alg. 1, FP64: stage N-1 down to 0; nodes of a stage in parallel
  F.P.assign((size_t)nn * nx * nx, 0.0);
  F.Abar.assign((size_t)nn * nx * nx, 0.0);
  F.K.assign((size_t)nl * nu * nx, 0.0);
  F.Rinv.assign((size_t)nl * nu * nu, 0.0);
  F.W.assign((size_t)nl * nx * nu, 0.0);
  std::vector<double>& Pm = F.P;
  std::vector<double>& Abar = F.Abar;
  std::vector<double>& K = F.K;
  std::vector<double>& Rinv = F.Rinv;
  std::vector<double>& W = F.W;
  for (int j = nl; j < nn; ++j)
    for (int k = 0; k < nx; ++k) Pm[(size_t)j * nx * nx + (size_t)k * nx + k] = 1.0;
  bool ok = true;
  for (int t = T.N - 1; t >= 0; --t) {
    const int first = T.stage_off[t], count = T.stage_off[t + 1] - first;
    std::vector<char> good(count, 1);
    parallel_for(count, [&](int f) {
      const int i = first + f;
      std::vector<double> Rt((size_t)nu * nu, 0.0), SA((size_t)nu * nx, 0.0), Pt((size_t)nu * nx),
          PB((size_t)nx * nu), tmp((size_t)nx * nx), Lc((size_t)nu * nu);
      for (int k = 0; k < nu; ++k) Rt[(size_t)k * nu + k] = 1.0;
      for (int c = T.fc[i]; c < T.fc[i] + T.nch[i]; ++c) {
        const double* Bc = d->B + (size_t)c * nx * nu;
        const double* Ac = d->A + (size_t)c * nx * nx;
        const double* Pc = Pm.data() + (size_t)c * nx * nx;
        gemm_tn(nu, nx, nx, Bc, Pc, Pt.data(), false);          // P~ = B'P
        gemm(nu, nu, nx, Pt.data(), Bc, Rt.data(), true);       // R~ += P~ B
        gemm(nu, nx, nx, Pt.data(), Ac, SA.data(), true);       // sum P~ A
      }
      Lc = Rt;
      if (!cholesky(nu, Lc.data())) {
        good[f] = 0;
        return;
      }
      double* Ri = Rinv.data() + (size_t)i * nu * nu;
      chol_inverse(nu, Lc.data(), Ri);
      double* Ki = K.data() + (size_t)i * nu * nx;
      gemm(nu, nx, nu, Ri, SA.data(), Ki, false);
      for (int e = 0; e < nu * nx; ++e) Ki[e] = -Ki[e];
      double* Pi = Pm.data() + (size_t)i * nx * nx;
      gemm_tn(nx, nx, nu, Ki, Ki, Pi, false);                    // K'K
      for (int k = 0; k < nx; ++k) Pi[(size_t)k * nx + k] += 1.0;
      double* Wi = W.data() + (size_t)i * nx * nu;
      std::fill(Wi, Wi + (size_t)nx * nu, 0.0);
      for (int c = T.fc[i]; c < T.fc[i] + T.nch[i]; ++c) {
        const double* Bc = d->B + (size_t)c * nx * nu;
        const double* Ac = d->A + (size_t)c * nx * nx;
        const double* Pc = Pm.data() + (size_t)c * nx * nx;
        double* Ab = Abar.data() + (size_t)c * nx * nx;
        std::copy(Ac, Ac + (size_t)nx * nx, Ab);
        gemm(nx, nx, nu, Bc, Ki, Ab, true);                       // Abar = A + B K
        gemm(nx, nx, nx, Pc, Ab, tmp.data(), false);              // P Abar
        gemm_tn(nx, nx, nx, Ab, tmp.data(), Pi, true);            // += Abar' P Abar
        gemm(nx, nu, nx, Pc, Bc, PB.data(), false);               // P B
        gemm_tn(nx, nu, nx, Ab, PB.data(), Wi, true);             // W += Abar' P B
      }
      for (int e = 0; e < nx * nx; ++e)
        if (!is_finite(Pi[e])) good[f] = 0;
    });
    for (char g : good) ok = ok && g;
    if (!ok) return SPOCK_EFACTOR;
  }

  return SPOCK_OK;
}

double norm_L_blocks(const Tree& T, const spock_problem_data& dd) {
  const spock_problem_data* d = &dd;
  const int nn = T.nn, nl = T.nl, nx = d->nx, nu = d->nu;
  // ---- ||L||: block-diagonal after a column permutation; closed forms per block
  double best2 = 0.5;  // tau^c and leaf s^j columns: rows (1/2, 1/2)
  for (int i = 0; i < nl; ++i) {
    for (int k = 0; k < nx; ++k) {
      double s = 1.0;
      for (int c = T.fc[i]; c < T.fc[i] + T.nch[i]; ++c) s += d->q[(size_t)c * nx + k];
      best2 = std::max(best2, s);
    }
    for (int k = 0; k < nu; ++k) {
      double s = 1.0;
      for (int c = T.fc[i]; c < T.fc[i] + T.nch[i]; ++c) s += d->r[(size_t)c * nu + k];
      best2 = std::max(best2, s);
    }
    // (y^i, s^i) block [[I, 0], [-b', 1]]: sigma^2 = 1 + beta^2/2 + beta sqrt(1 + beta^2/4)
    double b2 = 1.0;
    for (int c = T.fc[i]; c < T.fc[i] + T.nch[i]; ++c) b2 += T.pcond[c] * T.pcond[c];
    const double beta = std::sqrt(b2);
    best2 = std::max(best2, 1.0 + 0.5 * b2 + beta * std::sqrt(1.0 + 0.25 * b2));
  }
  for (int j = nl; j < nn; ++j)
    for (int k = 0; k < nx; ++k) best2 = std::max(best2, 1.0 + d->qN[(size_t)j * nx + k]);
  return std::sqrt(best2);
}

int build_flow_items(const Tree& T, int nc, int chunk_codes, std::vector<int>& items, std::vector<int>& pbase,
                     int& nslots, int& nbwd) {
  if (nc < 1) return SPOCK_EINVAL;
  items.clear();
  pbase.assign(T.nl, 0);
  nslots = 0;
  for (int i = T.nl - 1; i >= 0; --i) {
    const int J = (T.nch[i] + nc - 1) / nc;
    if (J >= chunk_codes) return SPOCK_EINVAL;
    for (int j = 0; j < J; ++j) items.push_back(i * chunk_codes + j);
    if (J > 1) {
      pbase[i] = nslots;
      nslots += J - 1;
    }
  }
  nbwd = (int)items.size();
  for (int i = 0; i < T.nl; ++i)
    for (int j = 0, J = (T.nch[i] + nc - 1) / nc; j < J; ++j) items.push_back(i * chunk_codes + j);
  return SPOCK_OK;
}

}  // namespace spk
