// Kernels of general problems: a conic risk measure (E, F, b, K) at every
// nonleaf node (section 4.3) and polyhedral constraints Gamma_x x + Gamma_u u
// in C (section 4.1, eq. constraints) in place of AV@R and the boxes. Only
// the parts of T that touch y, the constraint rows and the leaves' rows
// change; the Alg. 2 sweeps are shared with every other problem.
//
// One thread per family (nonleaf node i with its children). Every row of L
// and every column of L* belongs to exactly one family:
//   rows:    group 1 of i (y^i, s^i - b'y^i, the nc constraint rows), group
//            2 of each child (the SOC block), group 3 of each leaf child
//            (ncN constraint rows, then its SOC block);
//   columns: y^i, s^i, x^i, u^i, tau of each child, and x^j, s^j of each
//            leaf child.
#include "device_common.h"

#include <math.h>

namespace spk {

namespace {

constexpr int kGenThreads = 256;

// Offsets in the general layout.
template <typename S>
struct GOff {
  const DevProb<S>& P;
  const GenDev<S>& G;
  __device__ GOff(const DevProb<S>& p, const GenDev<S>& g) : P(p), G(g) {}
  __device__ long long x(int i) const { return 1 + (long long)i * P.nx; }
  __device__ long long u(int i) const { return P.zU + (long long)i * P.nu; }
  __device__ long long y(int i) const { return G.z2off[i]; }
  __device__ long long tau(int c) const {
    const int a = P.anc[c];
    return G.z2off[a] + G.ny[a] + (c - P.fc[a]);
  }
  __device__ long long s(int c) const {
    if (c == 0) return 0;
    const int a = P.anc[c];
    return G.z2off[a] + G.ny[a] + P.nch[a] + (c - P.fc[a]);
  }
  __device__ long long e1(int i) const { return G.e1off[i]; }
  __device__ long long e1s(int i) const { return G.e1off[i] + G.ny[i]; }
  __device__ long long e1c(int i) const { return e1s(i) + 1; }
  __device__ long long e2(int c) const { return G.eE2 + (long long)(c - 1) * (P.nx + P.nu + 2); }
  __device__ long long e3(int j) const { return G.eE3 + (long long)(j - P.nl) * (G.ncN + P.nx + 2); }
  __device__ long long e3q(int j) const { return e3(j) + G.ncN; }
  __device__ const S* Gx(int i) const { return G.Gx + (size_t)i * G.nc * P.nx; }
  __device__ const S* Gu(int i) const { return G.Gu + (size_t)i * G.nc * P.nu; }
  __device__ const S* GN(int j) const { return G.GN + (size_t)(j - P.nl) * G.ncN * P.nx; }
  // Row o of a cost root applied to the vector f(base + k), k < n: kind 0
  // Q^c (on x), 1 R^c (on u), 2 Q_N^c (on x). Dense symmetric roots when the
  // problem has dense costs, else the roots of the diagonals. The roots are
  // symmetric, so the same rows give the L* columns.
  template <typename F>
  __device__ S croot(int kind, int c, int o, long long base, F&& f) const {
    const int n = kind == 1 ? P.nu : P.nx;
    const S* M = kind == 0 ? G.Qh : (kind == 1 ? G.Rh : G.QNh);
    if (M) {
      const S* row = M + ((size_t)c * n + o) * n;
      S acc = 0;
      for (int k = 0; k < n; ++k) acc += row[k] * f(base + k);
      return acc;
    }
    const S* dg = kind == 0 ? P.sq : (kind == 1 ? P.sr : P.sqN);
    return dg[(size_t)c * n + o] * f(base + o);
  }
};

// (L* eta) on column x^i of nonleaf i, component o: Gamma_x' eta_c plus the
// children's Q^{1/2} rows.
template <typename S>
__device__ S lt_x(const GOff<S>& O, const S* eta, int i, int o) {
  const DevProb<S>& P = O.P;
  const int nx = P.nx, nc = O.G.nc;
  const S* gx = O.Gx(i);
  const long long ec = O.e1c(i);
  S acc = 0;
  for (int r = 0; r < nc; ++r) acc += gx[(size_t)r * nx + o] * eta[ec + r];
  auto ev = [&](long long e) { return eta[e]; };
  for (int c = P.fc[i]; c < P.fc[i] + P.nch[i]; ++c) acc += O.croot(0, c, o, O.e2(c), ev);
  return acc;
}
template <typename S>
__device__ S lt_u(const GOff<S>& O, const S* eta, int i, int o) {
  const DevProb<S>& P = O.P;
  const int nx = P.nx, nu = P.nu, nc = O.G.nc;
  const S* gu = O.Gu(i);
  const long long ec = O.e1c(i);
  S acc = 0;
  for (int r = 0; r < nc; ++r) acc += gu[(size_t)r * nu + o] * eta[ec + r];
  auto ev = [&](long long e) { return eta[e]; };
  for (int c = P.fc[i]; c < P.fc[i] + P.nch[i]; ++c) acc += O.croot(1, c, o, O.e2(c) + nx, ev);
  return acc;
}
// column x^j of leaf j: Gamma_N' eta_cN + Q_N^{1/2} eta_q
template <typename S>
__device__ S lt_xleaf(const GOff<S>& O, const S* eta, int j, int o) {
  const DevProb<S>& P = O.P;
  const int nx = P.nx, ncN = O.G.ncN;
  const S* gn = O.GN(j);
  const long long e3 = O.e3(j);
  S acc = O.croot(2, j, o, O.e3q(j), [&](long long e) { return eta[e]; });
  for (int r = 0; r < ncN; ++r) acc += gn[(size_t)r * nx + o] * eta[e3 + r];
  return acc;
}
// column s^c: the s-row of c when c is nonleaf, else half the sum of its
// group-3 pair
template <typename S>
__device__ S lt_s(const GOff<S>& O, const S* eta, int c) {
  if (c < O.P.nl) return eta[O.e1s(c)];
  const long long e = O.e3q(c) + O.P.nx;
  return S(0.5) * (eta[e] + eta[e + 1]);
}
// row r of Gamma_x x^i + Gamma_u u^i for the vector z
template <typename S>
__device__ S l_c(const GOff<S>& O, const S* z, int i, int r) {
  const DevProb<S>& P = O.P;
  const S* gx = O.Gx(i) + (size_t)r * P.nx;
  const S* gu = O.Gu(i) + (size_t)r * P.nu;
  S acc = 0;
  for (int o = 0; o < P.nx; ++o) acc += gx[o] * z[O.x(i) + o];
  for (int o = 0; o < P.nu; ++o) acc += gu[o] * z[O.u(i) + o];
  return acc;
}
template <typename S>
__device__ S l_cN(const GOff<S>& O, const S* z, int j, int r) {
  const DevProb<S>& P = O.P;
  const S* gn = O.GN(j) + (size_t)r * P.nx;
  S acc = 0;
  for (int o = 0; o < P.nx; ++o) acc += gn[o] * z[O.x(j) + o];
  return acc;
}
// s^i - b'y^i
template <typename S>
__device__ S l_s(const GOff<S>& O, const S* z, int i) {
  const S* b = O.G.b + O.G.yoff[i];
  S acc = z[O.s(i)];
  for (int k = 0; k < O.G.ny[i]; ++k) acc -= b[k] * z[O.y(i) + k];
  return acc;
}

// prox of g* on the translated SOC block (eq. S3-def, shift (0,..,0,1/2,-1/2))
// of len entries at w (then the two trailing scalars): out = w - alpha
// (shift + proj_SOC(w / alpha - shift)); one thread.
template <typename S>
__device__ void soc_prox_one(const S* w, S* out, int len, S al) {
  const S ia = S(1) / al;
  double n2 = 0;
  for (int o = 0; o < len; ++o) {
    const double t = (double)(w[o] * ia);
    n2 += t * t;
  }
  const S va = w[len] * ia - S(0.5);
  const S t = w[len + 1] * ia + S(0.5);
  const S nrm = (S)sqrt(n2 + (double)va * (double)va);
  S scale, pt;
  if (nrm <= t) {
    scale = S(1);
    pt = t;
  } else if (nrm <= -t) {
    scale = S(0);
    pt = S(0);
  } else {
    const S cc = S(0.5) * (nrm + t);
    scale = cc / nrm;
    pt = cc;
  }
  for (int o = 0; o < len; ++o) out[o] = w[o] - al * (scale * (w[o] * ia));
  out[len] = w[len] - al * (S(0.5) + scale * va);
  out[len + 1] = w[len + 1] - al * (S(-0.5) + pt);
}

// prox of g* on the rows of family i for the dual argument at w (rows as in
// eta), written to out: group 1 (K* on y, R_+ on the s-row, C^i on the
// constraint rows), group 2 of every child, group 3 of leaf children.
// The SOC blocks go through out itself (the argument is read first).
template <typename S>
__device__ void fam_gen_prox(const GOff<S>& O, const S* w, S* out, int i) {
  const DevProb<S>& P = O.P;
  const GenDev<S>& G = O.G;
  const S al = P.alpha, ia = S(1) / al;
  const long long e1 = O.e1(i);
  const int ny = G.ny[i], kp = G.kpos[i];
  for (int k = 0; k < ny; ++k) {
    const S v = w[e1 + k];
    out[e1 + k] = k < kp ? (v < S(0) ? v : S(0)) : S(0);
  }
  {
    const S v = w[O.e1s(i)];
    out[O.e1s(i)] = v < S(0) ? v : S(0);
  }
  const long long ec = O.e1c(i);
  for (int r = 0; r < G.nc; ++r) {
    const S v = w[ec + r];
    out[ec + r] = v - al * clampv(v * ia, G.cmin[(size_t)i * G.nc + r], G.cmax[(size_t)i * G.nc + r]);
  }
  for (int c = P.fc[i]; c < P.fc[i] + P.nch[i]; ++c) {
    soc_prox_one<S>(w + O.e2(c), out + O.e2(c), P.nx + P.nu, al);
    if (c >= P.nl) {
      const long long e3 = O.e3(c);
      const size_t lj = (size_t)(c - P.nl) * G.ncN;
      for (int r = 0; r < G.ncN; ++r) {
        const S v = w[e3 + r];
        out[e3 + r] = v - al * clampv(v * ia, G.cNmin[lj + r], G.cNmax[lj + r]);
      }
      soc_prox_one<S>(w + O.e3q(c), out + O.e3q(c), P.nx, al);
    }
  }
}

// rows of L z owned by family i, written into eta (or, with scale and base,
// eta = base + scale L z)
template <typename S>
__device__ void fam_gen_L(const GOff<S>& O, const S* z, S* eta, int i, const S* base, S scale) {
  const DevProb<S>& P = O.P;
  const GenDev<S>& G = O.G;
  const int nx = P.nx, nu = P.nu;
  auto put = [&](long long e, S v) { eta[e] = base ? base[e] + scale * v : v; };
  const long long e1 = O.e1(i);
  for (int k = 0; k < G.ny[i]; ++k) put(e1 + k, z[O.y(i) + k]);
  put(O.e1s(i), l_s<S>(O, z, i));
  for (int r = 0; r < G.nc; ++r) put(O.e1c(i) + r, l_c<S>(O, z, i, r));
  for (int c = P.fc[i]; c < P.fc[i] + P.nch[i]; ++c) {
    const long long e2 = O.e2(c);
    auto zv = [&](long long e) { return z[e]; };
    for (int o = 0; o < nx; ++o) put(e2 + o, O.croot(0, c, o, O.x(i), zv));
    for (int o = 0; o < nu; ++o) put(e2 + nx + o, O.croot(1, c, o, O.u(i), zv));
    const S th = S(0.5) * z[O.tau(c)];
    put(e2 + nx + nu, th);
    put(e2 + nx + nu + 1, th);
    if (c >= P.nl) {
      const long long e3 = O.e3(c);
      for (int r = 0; r < G.ncN; ++r) put(e3 + r, l_cN<S>(O, z, c, r));
      const long long e3q = O.e3q(c);
      for (int o = 0; o < nx; ++o) put(e3q + o, O.croot(2, c, o, O.x(c), zv));
      const S sh = S(0.5) * z[O.s(c)];
      put(e3q + nx, sh);
      put(e3q + nx + 1, sh);
    }
  }
}

// columns of L* eta owned by family i, written into z (or z = base + scale L* eta)
template <typename S>
__device__ void fam_gen_Lt(const GOff<S>& O, const S* eta, S* z, int i, const S* base, S scale) {
  const DevProb<S>& P = O.P;
  const GenDev<S>& G = O.G;
  const int nx = P.nx, nu = P.nu;
  auto put = [&](long long e, S v) { z[e] = base ? base[e] + scale * v : v; };
  const S es = eta[O.e1s(i)];
  const S* b = G.b + G.yoff[i];
  for (int k = 0; k < G.ny[i]; ++k) put(O.y(i) + k, eta[O.e1(i) + k] - b[k] * es);
  put(O.s(i), es);
  for (int o = 0; o < nx; ++o) put(O.x(i) + o, lt_x<S>(O, eta, i, o));
  for (int o = 0; o < nu; ++o) put(O.u(i) + o, lt_u<S>(O, eta, i, o));
  for (int c = P.fc[i]; c < P.fc[i] + P.nch[i]; ++c) {
    const long long e2 = O.e2(c) + nx + nu;
    put(O.tau(c), S(0.5) * (eta[e2] + eta[e2 + 1]));
    if (c >= P.nl) {
      for (int o = 0; o < nx; ++o) put(O.x(c) + o, lt_xleaf<S>(O, eta, c, o));
      put(O.s(c), lt_s<S>(O, eta, c));
    }
  }
}

// ---------------------------------------------------------------- kernels
// pre-pass of T: xbar, ubar = (x, u) - alpha L* eta; leaf children seed the
// backward sweep with q = -xbar; the (y, tau, s) block of the step
// z - alpha L* eta is projected on S2 (kernel of [E' -I -I; F' 0 0], the
// projector formed offline); s^0 - alpha at the root.
template <typename S>
__global__ void __launch_bounds__(kGenThreads) k_gen_pre(DevProb<S> P, GenDev<S> G, const S* __restrict__ z,
                                                       const S* __restrict__ eta, S* __restrict__ zout,
                                                       S* __restrict__ xbar, S* __restrict__ ubar,
                                                       S* __restrict__ qbuf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.nl) return;
  const GOff<S> O(P, G);
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i], ny = G.ny[i];
  const S al = P.alpha;
  for (int o = 0; o < nx; ++o) xbar[(size_t)i * nx + o] = z[O.x(i) + o] - al * lt_x<S>(O, eta, i, o);
  for (int o = 0; o < nu; ++o) ubar[(size_t)i * nu + o] = z[O.u(i) + o] - al * lt_u<S>(O, eta, i, o);
  if (fc >= P.nl)  // children are leaves
    for (int c = fc; c < fc + n; ++c)
      for (int o = 0; o < nx; ++o)
        qbuf[(size_t)c * nx + o] = -(z[O.x(c) + o] - al * lt_xleaf<S>(O, eta, c, o));
  // the (y, tau, s) block after the step, then its projection on S2
  S w[kGenMaxBlock];
  const S es = eta[O.e1s(i)];
  const S* b = G.b + G.yoff[i];
  for (int k = 0; k < ny; ++k) w[k] = z[O.y(i) + k] - al * (eta[O.e1(i) + k] - b[k] * es);
  for (int k = 0; k < n; ++k) {
    const int c = fc + k;
    const long long e2 = O.e2(c) + nx + nu;
    w[ny + k] = z[O.tau(c)] - al * S(0.5) * (eta[e2] + eta[e2 + 1]);
    w[ny + n + k] = z[O.s(c)] - al * lt_s<S>(O, eta, c);
  }
  const int m = ny + 2 * n;
  const S* Pm = G.PS2 + G.Poff[i];
  const long long zb = O.y(i);
  for (int r = 0; r < m; ++r) {
    S acc = 0;
    for (int k = 0; k < m; ++k) acc += Pm[(size_t)r * m + k] * w[k];
    zout[zb + r] = acc;
  }
  if (i == 0) zout[0] = z[0] - al * es - al;
}

// post-pass of T: eta+ = prox_{alpha g*}(eta + alpha L (2 z+ - z)) on the
// family's rows, and the residual statistics of r = v - T(v) on its rows
// (||r_eta||^2, <r_eta, L r_z>, |r_eta / alpha - L r_z|) and columns
// (||r_z||^2, |r_z / alpha - L* r_eta|).
template <typename S>
__global__ void __launch_bounds__(kGenThreads) k_gen_post(DevProb<S> P, GenDev<S> G, const S* __restrict__ z,
                                                        const S* __restrict__ eta, const S* __restrict__ zout,
                                                        S* __restrict__ eout, double* __restrict__ partials) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  StatAcc st;
  if (i < P.nl) {
    const GOff<S> O(P, G);
    const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i], ny = G.ny[i];
    const S al = P.alpha;
    const double ia = 1.0 / (double)al;
    // z2 = 2 z+ - z on the entries the family's rows read, via a lambda
    auto zz = [&](long long e) { return S(2) * zout[e] - z[e]; };
    auto rz = [&](long long e) { return z[e] - zout[e]; };
    // ---- rows: the prox argument w = eta + alpha L(2 z+ - z) into eout,
    // then the prox in place (fam_gen_prox reads w first)
    const long long e1 = O.e1(i);
    for (int k = 0; k < ny; ++k) eout[e1 + k] = eta[e1 + k] + al * zz(O.y(i) + k);
    {
      const S* b = G.b + G.yoff[i];
      S ls = zz(O.s(i));
      for (int k = 0; k < ny; ++k) ls -= b[k] * zz(O.y(i) + k);
      eout[O.e1s(i)] = eta[O.e1s(i)] + al * ls;
    }
    for (int r = 0; r < G.nc; ++r) {
      const S* gx = O.Gx(i) + (size_t)r * nx;
      const S* gu = O.Gu(i) + (size_t)r * nu;
      S acc = 0;
      for (int o = 0; o < nx; ++o) acc += gx[o] * zz(O.x(i) + o);
      for (int o = 0; o < nu; ++o) acc += gu[o] * zz(O.u(i) + o);
      eout[O.e1c(i) + r] = eta[O.e1c(i) + r] + al * acc;
    }
    for (int c = fc; c < fc + n; ++c) {
      const long long e2 = O.e2(c);
      for (int o = 0; o < nx; ++o) eout[e2 + o] = eta[e2 + o] + al * O.croot(0, c, o, O.x(i), zz);
      for (int o = 0; o < nu; ++o) eout[e2 + nx + o] = eta[e2 + nx + o] + al * O.croot(1, c, o, O.u(i), zz);
      const S th = S(0.5) * zz(O.tau(c));
      eout[e2 + nx + nu] = eta[e2 + nx + nu] + al * th;
      eout[e2 + nx + nu + 1] = eta[e2 + nx + nu + 1] + al * th;
      if (c >= P.nl) {
        const long long e3 = O.e3(c), e3q = O.e3q(c);
        for (int r = 0; r < G.ncN; ++r) {
          const S* gn = O.GN(c) + (size_t)r * nx;
          S acc = 0;
          for (int o = 0; o < nx; ++o) acc += gn[o] * zz(O.x(c) + o);
          eout[e3 + r] = eta[e3 + r] + al * acc;
        }
        for (int o = 0; o < nx; ++o) eout[e3q + o] = eta[e3q + o] + al * O.croot(2, c, o, O.x(c), zz);
        const S sh = S(0.5) * zz(O.s(c));
        eout[e3q + nx] = eta[e3q + nx] + al * sh;
        eout[e3q + nx + 1] = eta[e3q + nx + 1] + al * sh;
      }
    }
    fam_gen_prox<S>(O, eout, eout, i);
    // ---- row statistics: r_eta = eta - eta+ against (L r_z) on the row
    auto row = [&](long long e, S Lrz) { st.row((double)(eta[e] - eout[e]), (double)Lrz, ia); };
    for (int k = 0; k < ny; ++k) row(e1 + k, rz(O.y(i) + k));
    {
      const S* b = G.b + G.yoff[i];
      S ls = rz(O.s(i));
      for (int k = 0; k < ny; ++k) ls -= b[k] * rz(O.y(i) + k);
      row(O.e1s(i), ls);
    }
    for (int r = 0; r < G.nc; ++r) {
      const S* gx = O.Gx(i) + (size_t)r * nx;
      const S* gu = O.Gu(i) + (size_t)r * nu;
      S acc = 0;
      for (int o = 0; o < nx; ++o) acc += gx[o] * rz(O.x(i) + o);
      for (int o = 0; o < nu; ++o) acc += gu[o] * rz(O.u(i) + o);
      row(O.e1c(i) + r, acc);
    }
    for (int c = fc; c < fc + n; ++c) {
      const long long e2 = O.e2(c);
      for (int o = 0; o < nx; ++o) row(e2 + o, O.croot(0, c, o, O.x(i), rz));
      for (int o = 0; o < nu; ++o) row(e2 + nx + o, O.croot(1, c, o, O.u(i), rz));
      row(e2 + nx + nu, S(0.5) * rz(O.tau(c)));
      row(e2 + nx + nu + 1, S(0.5) * rz(O.tau(c)));
      if (c >= P.nl) {
        const long long e3 = O.e3(c), e3q = O.e3q(c);
        for (int r = 0; r < G.ncN; ++r) {
          const S* gn = O.GN(c) + (size_t)r * nx;
          S acc = 0;
          for (int o = 0; o < nx; ++o) acc += gn[o] * rz(O.x(c) + o);
          row(e3 + r, acc);
        }
        for (int o = 0; o < nx; ++o) row(e3q + o, O.croot(2, c, o, O.x(c), rz));
        row(e3q + nx, S(0.5) * rz(O.s(c)));
        row(e3q + nx + 1, S(0.5) * rz(O.s(c)));
      }
    }
    // ---- column statistics: r_z against (L* r_eta) on the column, with
    // r_eta = eta - eta+ (rows the same thread has just written)
    auto col = [&](long long e, S Ltre) { st.col((double)rz(e), (double)Ltre, ia); };
    auto re = [&](long long e) { return eta[e] - eout[e]; };
    {
      const S* b = G.b + G.yoff[i];
      const S res = re(O.e1s(i));
      for (int k = 0; k < ny; ++k) col(O.y(i) + k, re(e1 + k) - b[k] * res);
      col(O.s(i), res);
    }
    for (int o = 0; o < nx; ++o) {
      const S* gx = O.Gx(i);
      S acc = 0;
      for (int r = 0; r < G.nc; ++r) acc += gx[(size_t)r * nx + o] * re(O.e1c(i) + r);
      for (int c = fc; c < fc + n; ++c) acc += O.croot(0, c, o, O.e2(c), re);
      col(O.x(i) + o, acc);
    }
    for (int o = 0; o < nu; ++o) {
      const S* gu = O.Gu(i);
      S acc = 0;
      for (int r = 0; r < G.nc; ++r) acc += gu[(size_t)r * nu + o] * re(O.e1c(i) + r);
      for (int c = fc; c < fc + n; ++c) acc += O.croot(1, c, o, O.e2(c) + nx, re);
      col(O.u(i) + o, acc);
    }
    for (int c = fc; c < fc + n; ++c) {
      const long long e2 = O.e2(c) + nx + nu;
      col(O.tau(c), S(0.5) * (re(e2) + re(e2 + 1)));
      if (c >= P.nl) {
        const long long e3 = O.e3(c), e3q = O.e3q(c);
        for (int o = 0; o < nx; ++o) {
          const S* gn = O.GN(c);
          S acc = O.croot(2, c, o, e3q, re);
          for (int r = 0; r < G.ncN; ++r) acc += gn[(size_t)r * nx + o] * re(e3 + r);
          col(O.x(c) + o, acc);
        }
        col(O.s(c), S(0.5) * (re(e3q + nx) + re(e3q + nx + 1)));
      }
    }
  }
  block_stats(st, partials);
}

template <typename S>
__global__ void k_gen_L(DevProb<S> P, GenDev<S> G, const S* __restrict__ z, S* __restrict__ eta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.nl) return;
  fam_gen_L<S>(GOff<S>(P, G), z, eta, i, nullptr, S(1));
}
template <typename S>
__global__ void k_gen_Lt(DevProb<S> P, GenDev<S> G, const S* __restrict__ eta, S* __restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.nl) return;
  fam_gen_Lt<S>(GOff<S>(P, G), eta, z, i, nullptr, S(1));
}
template <typename S>
__global__ void k_gen_prox_gstar(DevProb<S> P, GenDev<S> G, const S* __restrict__ w, S* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.nl) return;
  fam_gen_prox<S>(GOff<S>(P, G), w, out, i);
}
// M d = (d_z - alpha L* d_eta, d_eta - alpha L d_z)
template <typename S>
__global__ void k_gen_M(DevProb<S> P, GenDev<S> G, const S* __restrict__ d, S* __restrict__ Md) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.nl) return;
  const GOff<S> O(P, G);
  fam_gen_Lt<S>(O, d + P.nz, Md, i, d, -P.alpha);
  fam_gen_L<S>(O, d, Md + P.nz, i, d + P.nz, -P.alpha);
}

template <typename S>
const GenDev<S>& gen_of(const Problem& P);
template <>
const GenDev<double>& gen_of<double>(const Problem& P) { return P.gd64; }
template <>
const GenDev<float>& gen_of<float>(const Problem& P) { return P.gd32; }
template <typename S>
const DevProb<S>& dev_of_g(const Problem& P);
template <>
const DevProb<double>& dev_of_g<double>(const Problem& P) { return P.dp64; }
template <>
const DevProb<float>& dev_of_g<float>(const Problem& P) { return P.dp32; }

int gen_blocks(const Problem& P) { return (P.tree->nl + kGenThreads - 1) / kGenThreads; }

}  // namespace

int gen_post_blocks(const Problem& P) { return gen_blocks(P); }

template <typename S>
hipError_t launch_gen_pre(const Problem& P, const S* z, const S* eta, S* zout, S* xbar, S* ubar, S* qbuf,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_gen_pre<S>, dim3(gen_blocks(P)), dim3(kGenThreads), 0, st, dev_of_g<S>(P), gen_of<S>(P), z,
                     eta, zout, xbar, ubar, qbuf);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_gen_post(const Problem& P, const S* z, const S* eta, const S* zout, S* eout, double* partials,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_gen_post<S>, dim3(gen_blocks(P)), dim3(kGenThreads), 0, st, dev_of_g<S>(P), gen_of<S>(P),
                     z, eta, zout, eout, partials);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_gen_L(const Problem& P, const S* z, S* eta, hipStream_t st) {
  hipLaunchKernelGGL(k_gen_L<S>, dim3(gen_blocks(P)), dim3(kGenThreads), 0, st, dev_of_g<S>(P), gen_of<S>(P), z,
                     eta);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_gen_Lt(const Problem& P, const S* eta, S* z, hipStream_t st) {
  hipLaunchKernelGGL(k_gen_Lt<S>, dim3(gen_blocks(P)), dim3(kGenThreads), 0, st, dev_of_g<S>(P), gen_of<S>(P), eta,
                     z);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_gen_prox_gstar(const Problem& P, const S* w, S* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gen_prox_gstar<S>, dim3(gen_blocks(P)), dim3(kGenThreads), 0, st, dev_of_g<S>(P),
                     gen_of<S>(P), w, out);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_gen_M(const Problem& P, const S* d, S* Md, hipStream_t st) {
  hipLaunchKernelGGL(k_gen_M<S>, dim3(gen_blocks(P)), dim3(kGenThreads), 0, st, dev_of_g<S>(P), gen_of<S>(P), d,
                     Md);
  return hipGetLastError();
}

#define SPK_GEN_INST(S)                                                                                    \
  template hipError_t launch_gen_pre<S>(const Problem&, const S*, const S*, S*, S*, S*, S*, hipStream_t);     \
  template hipError_t launch_gen_post<S>(const Problem&, const S*, const S*, const S*, S*, double*,          \
                                         hipStream_t);                                                     \
  template hipError_t launch_gen_L<S>(const Problem&, const S*, S*, hipStream_t);                           \
  template hipError_t launch_gen_Lt<S>(const Problem&, const S*, S*, hipStream_t);                          \
  template hipError_t launch_gen_prox_gstar<S>(const Problem&, const S*, S*, hipStream_t);                  \
  template hipError_t launch_gen_M<S>(const Problem&, const S*, S*, hipStream_t);
SPK_GEN_INST(double)
SPK_GEN_INST(float)

}  // namespace spk
