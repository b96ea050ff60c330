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
  const bool dense = d->Qm || d->Rm || d->QNm;
  for (int c = 1; c < nn; ++c) {
    for (int e = 0; e < nx * nx; ++e) if (!is_finite(d->A[(size_t)c * nx * nx + e])) return SPOCK_EINVAL;
    for (int e = 0; e < nx * nu; ++e) if (!is_finite(d->B[(size_t)c * nx * nu + e])) return SPOCK_EINVAL;
    if (dense) continue;
    for (int k = 0; k < nx; ++k) if (!(d->q[(size_t)c * nx + k] > 0.0) || !is_finite(d->q[(size_t)c * nx + k])) return SPOCK_EINVAL;
    for (int k = 0; k < nu; ++k) if (!(d->r[(size_t)c * nu + k] > 0.0) || !is_finite(d->r[(size_t)c * nu + k])) return SPOCK_EINVAL;
  }
  if (dense) {
    const int rc = check_dense_costs(T, *d);
    if (rc) return rc;
  } else {
    for (int j = nl; j < nn; ++j)
      for (int k = 0; k < nx; ++k) if (!(d->qN[(size_t)j * nx + k] >= 0.0) || !is_finite(d->qN[(size_t)j * nx + k])) return SPOCK_EINVAL;
  }
  // the boxes (unless general constraints replace them) and AV@R's a
  // (unless a general risk replaces it)
  if (!d->cons) {
    if (!d->xmin || !d->xmax || !d->umin || !d->umax) return SPOCK_EINVAL;
    for (int i = 0; i < nn; ++i)
      for (int k = 0; k < nx; ++k) {
        const double lo = d->xmin[(size_t)i * nx + k], hi = d->xmax[(size_t)i * nx + k];
        if (std::isnan(lo) || std::isnan(hi) || lo > hi) return SPOCK_EBOX;
      }
    for (int i = 0; i < nl; ++i)
      for (int k = 0; k < nu; ++k) {
        const double lo = d->umin[(size_t)i * nu + k], hi = d->umax[(size_t)i * nu + k];
        if (std::isnan(lo) || std::isnan(hi) || lo > hi) return SPOCK_EBOX;
      }
  }
  if (!d->risk) {
    if (!d->a_risk) return SPOCK_EINVAL;
    for (int i = 0; i < nl; ++i)
      if (!(d->a_risk[i] >= 0.0 && d->a_risk[i] <= 1.0)) return SPOCK_EINVAL;
  }
  return SPOCK_OK;
}

namespace {
// Symmetric eigendecomposition by cyclic Jacobi (row-major k x k; A is
// overwritten by its eigenvalues on the diagonal, V receives the vectors as
// columns).
void sym_jacobi(int k, std::vector<double>& A, std::vector<double>& V) {
  V.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int p = 0; p < k; ++p) {
      dia += A[(size_t)p * k + p] * A[(size_t)p * k + p];
      for (int q = p + 1; q < k; ++q) off += A[(size_t)p * k + q] * A[(size_t)p * k + q];
    }
    if (off <= 1e-32 * std::max(dia, 1e-300)) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = A[(size_t)p * k + q];
        if (apq == 0.0) continue;
        const double th = 0.5 * (A[(size_t)q * k + q] - A[(size_t)p * k + p]) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int r = 0; r < k; ++r) {
          const double arp = A[(size_t)r * k + p], arq = A[(size_t)r * k + q];
          A[(size_t)r * k + p] = c * arp - sn * arq;
          A[(size_t)r * k + q] = sn * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {
          const double apr = A[(size_t)p * k + r], aqr = A[(size_t)q * k + r];
          A[(size_t)p * k + r] = c * apr - sn * aqr;
          A[(size_t)q * k + r] = sn * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {
          const double vrp = V[(size_t)r * k + p], vrq = V[(size_t)r * k + q];
          V[(size_t)r * k + p] = c * vrp - sn * vrq;
          V[(size_t)r * k + q] = sn * vrp + c * vrq;
        }
      }
  }
}
}  // namespace

double sym_max_eig(int k, std::vector<double> A) {
  std::vector<double> V;
  sym_jacobi(k, A, V);
  double m = -std::numeric_limits<double>::infinity();
  for (int i = 0; i < k; ++i) m = std::max(m, A[(size_t)i * k + i]);
  return m;
}

int build_general(const Tree& T, const spock_problem_data& d, int max_block, GeneralLayout& G) {
  const int nn = T.nn, nl = T.nl, nx = d.nx, nu = d.nu;
  G = GeneralLayout{};
  G.ny.assign(nl, 0);
  G.nnu.assign(nl, 0);
  G.kpos.assign(nl, 0);
  const spock_risk_data* R = d.risk;
  const spock_constraint_data* C = d.cons;
  if (R && (!R->ny || !R->nnu || !R->kpos || !R->E || !R->b)) return SPOCK_EINVAL;
  long long ne = 0, nb = 0, nf = 0;
  for (int i = 0; i < nl; ++i) {
    const int n = T.nch[i];
    if (R) {
      G.ny[i] = R->ny[i];
      G.nnu[i] = R->nnu[i];
      G.kpos[i] = R->kpos[i];
      if (G.ny[i] < 1 || G.nnu[i] < 0 || G.kpos[i] < 0 || G.kpos[i] > G.ny[i]) return SPOCK_EINVAL;
    } else {
      G.ny[i] = 2 * n + 1;
      G.kpos[i] = 2 * n;
    }
    if (G.ny[i] + 2 * n > max_block) return SPOCK_EUNSUPPORTED;
    ne += (long long)G.ny[i] * n;
    nb += G.ny[i];
    nf += (long long)G.ny[i] * G.nnu[i];
  }
  if (R && nf > 0 && !R->F) return SPOCK_EINVAL;
  // E, b (AV@R: E = [a I; -I; 1'], b = (p, 0, 1))
  G.E.assign(ne, 0.0);
  G.b.assign(nb, 0.0);
  G.Eoff.assign(nl, 0);
  G.yoff.assign(nl, 0);
  std::vector<long long> Foff(nl, 0);
  {
    long long oe = 0, ob = 0, of = 0;
    for (int i = 0; i < nl; ++i) {
      const int n = T.nch[i], ny = G.ny[i];
      G.Eoff[i] = oe;
      G.yoff[i] = ob;
      Foff[i] = of;
      if (R) {
        for (long long e = 0; e < (long long)ny * n; ++e) G.E[oe + e] = R->E[oe + e];
        for (int k = 0; k < ny; ++k) G.b[ob + k] = R->b[ob + k];
      } else {
        const double a = d.a_risk[i];
        for (int k = 0; k < n; ++k) {
          G.E[oe + (size_t)k * n + k] = a;
          G.E[oe + (size_t)(n + k) * n + k] = -1.0;
          G.E[oe + (size_t)(2 * n) * n + k] = 1.0;
          G.b[ob + k] = T.pcond[T.fc[i] + k];
        }
        G.b[ob + 2 * n] = 1.0;
      }
      oe += (long long)ny * n;
      ob += ny;
      of += (long long)ny * G.nnu[i];
    }
  }
  for (double v : G.E) if (!is_finite(v)) return SPOCK_EINVAL;
  for (double v : G.b) if (!is_finite(v)) return SPOCK_EINVAL;
  if (R && nf > 0)
    for (long long e = 0; e < nf; ++e) if (!is_finite(R->F[e])) return SPOCK_EINVAL;
  // constraints
  if (C) {
    if (C->nc < 1 || C->ncN < 1 || !C->Gx || !C->Gu || !C->cmin || !C->cmax || !C->GN || !C->cNmin || !C->cNmax)
      return SPOCK_EINVAL;
    G.nc = C->nc;
    G.ncN = C->ncN;
    for (int i = 0; i < nl; ++i) {
      for (int e = 0; e < G.nc * nx; ++e) if (!is_finite(C->Gx[(size_t)i * G.nc * nx + e])) return SPOCK_EINVAL;
      for (int e = 0; e < G.nc * nu; ++e) if (!is_finite(C->Gu[(size_t)i * G.nc * nu + e])) return SPOCK_EINVAL;
      for (int r = 0; r < G.nc; ++r) {
        const double lo = C->cmin[(size_t)i * G.nc + r], hi = C->cmax[(size_t)i * G.nc + r];
        if (std::isnan(lo) || std::isnan(hi) || lo > hi) return SPOCK_EBOX;
      }
    }
    for (int j = nl; j < nn; ++j) {
      for (int e = 0; e < G.ncN * nx; ++e) if (!is_finite(C->GN[(size_t)j * G.ncN * nx + e])) return SPOCK_EINVAL;
      for (int r = 0; r < G.ncN; ++r) {
        const double lo = C->cNmin[(size_t)j * G.ncN + r], hi = C->cNmax[(size_t)j * G.ncN + r];
        if (std::isnan(lo) || std::isnan(hi) || lo > hi) return SPOCK_EBOX;
      }
    }
  } else {
    G.nc = nx + nu;
    G.ncN = nx;
  }
  // offsets and sizes
  G.z2off.assign(nl, 0);
  G.e1off.assign(nl, 0);
  long long oz = 1 + (long long)nn * nx + (long long)nl * nu, oe1 = 0;
  for (int i = 0; i < nl; ++i) {
    G.z2off[i] = oz;
    oz += G.ny[i] + 2LL * T.nch[i];
    G.e1off[i] = oe1;
    oe1 += G.ny[i] + 1 + G.nc;
  }
  G.nz = oz;
  G.eE2 = oe1;
  G.eE3 = G.eE2 + (long long)(nn - 1) * (nx + nu + 2);
  G.neta = G.eE3 + (long long)(nn - nl) * (G.ncN + nx + 2);
  // S2 projectors: I - G'(GG')^+ G with G = [E' -I -I; F' 0 0]
  G.Poff.assign(nl, 0);
  long long op = 0;
  for (int i = 0; i < nl; ++i) {
    G.Poff[i] = op;
    op += (long long)(G.ny[i] + 2 * T.nch[i]) * (G.ny[i] + 2 * T.nch[i]);
  }
  G.PS2.assign(op, 0.0);
  std::vector<char> good(nl, 1);
  parallel_for(nl, [&](int i) {
    const int n = T.nch[i], ny = G.ny[i], nnu = G.nnu[i], m = ny + 2 * n, rows = n + nnu;
    std::vector<double> Gm((size_t)rows * m, 0.0);
    const double* E = G.E.data() + G.Eoff[i];
    for (int c = 0; c < n; ++c) {
      for (int k = 0; k < ny; ++k) Gm[(size_t)c * m + k] = E[(size_t)k * n + c];
      Gm[(size_t)c * m + ny + c] = -1.0;
      Gm[(size_t)c * m + ny + n + c] = -1.0;
    }
    if (R)
      for (int f = 0; f < nnu; ++f)
        for (int k = 0; k < ny; ++k) Gm[(size_t)(n + f) * m + k] = R->F[Foff[i] + (size_t)k * nnu + f];
    std::vector<double> GG((size_t)rows * rows, 0.0), V;
    for (int a = 0; a < rows; ++a)
      for (int b = 0; b < rows; ++b) {
        double acc = 0;
        for (int k = 0; k < m; ++k) acc += Gm[(size_t)a * m + k] * Gm[(size_t)b * m + k];
        GG[(size_t)a * rows + b] = acc;
      }
    sym_jacobi(rows, GG, V);
    double lmax = 0;
    for (int a = 0; a < rows; ++a) lmax = std::max(lmax, GG[(size_t)a * rows + a]);
    // pseudo-inverse of GG' on its range
    std::vector<double> Pinv((size_t)rows * rows, 0.0);
    for (int e = 0; e < rows; ++e) {
      const double lam = GG[(size_t)e * rows + e];
      if (!(lam > 1e-12 * lmax)) continue;
      for (int a = 0; a < rows; ++a)
        for (int b = 0; b < rows; ++b) Pinv[(size_t)a * rows + b] += V[(size_t)a * rows + e] * V[(size_t)b * rows + e] / lam;
    }
    // P = I - G' Pinv G
    std::vector<double> PG((size_t)rows * m, 0.0);
    for (int a = 0; a < rows; ++a)
      for (int k = 0; k < m; ++k) {
        double acc = 0;
        for (int b = 0; b < rows; ++b) acc += Pinv[(size_t)a * rows + b] * Gm[(size_t)b * m + k];
        PG[(size_t)a * m + k] = acc;
      }
    double* Pm = G.PS2.data() + G.Poff[i];
    for (int r = 0; r < m; ++r)
      for (int k = 0; k < m; ++k) {
        double acc = (r == k) ? 1.0 : 0.0;
        for (int a = 0; a < rows; ++a) acc -= Gm[(size_t)a * m + r] * PG[(size_t)a * m + k];
        Pm[(size_t)r * m + k] = acc;
        if (!is_finite(acc)) good[i] = 0;
      }
  });
  for (char g : good)
    if (!g) return SPOCK_EINVAL;
  return SPOCK_OK;
}

double norm_L_general(const Tree& T, const spock_problem_data& d, const GeneralLayout& G) {
  const int nn = T.nn, nl = T.nl, nx = d.nx, nu = d.nu, k = nx + nu;
  const spock_constraint_data* C = d.cons;
  std::vector<double> best(std::max(nl, 1), 0.5);
  parallel_for(nl, [&](int i) {
    double b2 = 0;
    for (int e = 0; e < G.ny[i]; ++e) b2 += G.b[G.yoff[i] + e] * G.b[G.yoff[i] + e];
    double v = 1.0 + 0.5 * b2 + std::sqrt(b2) * std::sqrt(1.0 + 0.25 * b2);
    // (x^i, u^i) block: Gamma'Gamma + sum_c diag(q^c, r^c)
    std::vector<double> M((size_t)k * k, 0.0);
    if (C) {
      for (int r = 0; r < G.nc; ++r) {
        std::vector<double> row(k);
        for (int o = 0; o < nx; ++o) row[o] = C->Gx[((size_t)i * G.nc + r) * nx + o];
        for (int o = 0; o < nu; ++o) row[nx + o] = C->Gu[((size_t)i * G.nc + r) * nu + o];
        for (int a = 0; a < k; ++a)
          for (int b = 0; b < k; ++b) M[(size_t)a * k + b] += row[a] * row[b];
      }
    } else {
      for (int a = 0; a < k; ++a) M[(size_t)a * k + a] = 1.0;
    }
    for (int c = T.fc[i]; c < T.fc[i] + T.nch[i]; ++c) {
      if (d.Qm) {  // (Q^{1/2})'Q^{1/2} = Q
        for (int a = 0; a < nx; ++a)
          for (int b = 0; b < nx; ++b) M[(size_t)a * k + b] += d.Qm[((size_t)c * nx + a) * nx + b];
        for (int a = 0; a < nu; ++a)
          for (int b = 0; b < nu; ++b) M[(size_t)(nx + a) * k + nx + b] += d.Rm[((size_t)c * nu + a) * nu + b];
        continue;
      }
      for (int o = 0; o < nx; ++o) M[(size_t)o * k + o] += d.q[(size_t)c * nx + o];
      for (int o = 0; o < nu; ++o) M[(size_t)(nx + o) * k + nx + o] += d.r[(size_t)c * nu + o];
    }
    v = std::max(v, sym_max_eig(k, M));
    best[i] = std::max(best[i], v);
  });
  double b2max = 0.5;
  for (double v : best) b2max = std::max(b2max, v);
  for (int j = nl; j < nn; ++j) {
    std::vector<double> M((size_t)nx * nx, 0.0);
    if (C) {
      for (int r = 0; r < G.ncN; ++r)
        for (int a = 0; a < nx; ++a)
          for (int b = 0; b < nx; ++b)
            M[(size_t)a * nx + b] += C->GN[((size_t)j * G.ncN + r) * nx + a] * C->GN[((size_t)j * G.ncN + r) * nx + b];
    } else {
      for (int a = 0; a < nx; ++a) M[(size_t)a * nx + a] = 1.0;
    }
    if (d.QNm) {
      for (int a = 0; a < nx; ++a)
        for (int b = 0; b < nx; ++b) M[(size_t)a * nx + b] += d.QNm[((size_t)j * nx + a) * nx + b];
    } else {
      for (int o = 0; o < nx; ++o) M[(size_t)o * nx + o] += d.qN[(size_t)j * nx + o];
    }
    b2max = std::max(b2max, sym_max_eig(nx, M));
  }
  return std::sqrt(b2max);
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

int build_post_blocks(const Tree& T, int cap, std::vector<int>& bfam) {
  bfam.clear();
  int count = 0;
  for (int f = 0; f < T.nl; ++f) {
    if (f == 0 || (count > 0 && count + T.nch[f] > cap)) {
      bfam.push_back(f);
      count = 0;
    }
    count += T.nch[f];
  }
  const int nb = (int)bfam.size();
  bfam.push_back(T.nl);
  return nb;
}

namespace {
// eigenvalues (ascending order not needed) and vectors of a symmetric n x n block
void sym_eig(int n, const double* M, std::vector<double>& lam, std::vector<double>& V) {
  std::vector<double> A(M, M + (size_t)n * n);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < a; ++b) A[(size_t)a * n + b] = A[(size_t)b * n + a] = 0.5 * (A[(size_t)a * n + b] + A[(size_t)b * n + a]);
  sym_jacobi(n, A, V);
  lam.resize(n);
  for (int a = 0; a < n; ++a) lam[a] = A[(size_t)a * n + a];
}

int check_block(int n, const double* M, bool definite) {
  double mx = 0;
  for (int e = 0; e < n * n; ++e) {
    if (!is_finite(M[e])) return SPOCK_EINVAL;
    mx = std::max(mx, std::fabs(M[e]));
  }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < a; ++b)
      if (std::fabs(M[(size_t)a * n + b] - M[(size_t)b * n + a]) > 1e-12 * std::max(1.0, mx)) return SPOCK_EINVAL;
  std::vector<double> lam, V;
  sym_eig(n, M, lam, V);
  double lmin = lam[0], lmax = lam[0];
  for (double l : lam) {
    lmin = std::min(lmin, l);
    lmax = std::max(lmax, l);
  }
  if (definite ? !(lmin > 0.0) : (lmin < -1e-12 * std::max(1.0, lmax))) return SPOCK_EINVAL;
  return SPOCK_OK;
}

void root_block(int n, const double* M, double* out) {
  std::vector<double> lam, V;
  sym_eig(n, M, lam, V);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double s = 0;
      for (int k = 0; k < n; ++k) s += V[(size_t)a * n + k] * std::sqrt(std::max(lam[k], 0.0)) * V[(size_t)b * n + k];
      out[(size_t)a * n + b] = s;
    }
}
}  // namespace

int check_dense_costs(const Tree& T, const spock_problem_data& d) {
  if (!d.Qm || !d.Rm || !d.QNm) return SPOCK_EINVAL;
  const int nx = d.nx, nu = d.nu;
  for (int c = 1; c < T.nn; ++c) {
    if (check_block(nx, d.Qm + (size_t)c * nx * nx, false)) return SPOCK_EINVAL;
    if (check_block(nu, d.Rm + (size_t)c * nu * nu, true)) return SPOCK_EINVAL;
  }
  for (int j = T.nl; j < T.nn; ++j)
    if (check_block(nx, d.QNm + (size_t)j * nx * nx, false)) return SPOCK_EINVAL;
  return SPOCK_OK;
}

void dense_cost_roots(const Tree& T, const spock_problem_data& d, std::vector<double>& Qh, std::vector<double>& Rh,
                      std::vector<double>& QNh) {
  const int nn = T.nn, nx = d.nx, nu = d.nu;
  Qh.assign((size_t)nn * nx * nx, 0.0);
  Rh.assign((size_t)nn * nu * nu, 0.0);
  QNh.assign((size_t)nn * nx * nx, 0.0);
  parallel_for(nn, [&](int c) {
    if (c >= 1) {
      root_block(nx, d.Qm + (size_t)c * nx * nx, Qh.data() + (size_t)c * nx * nx);
      root_block(nu, d.Rm + (size_t)c * nu * nu, Rh.data() + (size_t)c * nu * nu);
    }
    if (c >= T.nl) root_block(nx, d.QNm + (size_t)c * nx * nx, QNh.data() + (size_t)c * nx * nx);
  });
}

}  // namespace spk

