// Device code shared by the per-stage kernels and the batched block engine:
// canonical offsets, team reductions, proximal maps and the per-family steps
// of the CP operator (section 5 splitting; Alg. 2 sweeps).
#pragma once
#include "spock_internal.h"

#include <math.h>

namespace spk {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ void wave_lds_sync() {
  // Teams live inside one wavefront and exchange values through LDS only:
  // the ordering is at wavefront scope and for LDS alone, so global loads
  // stay free to move across it.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <int T>
__device__ __forceinline__ double team_sum(double v) {
#pragma unroll
  for (int m = T / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, T);
  return v;
}

template <typename S>
__device__ __forceinline__ S clampv(S v, S lo, S hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Loads and stores of values that other workgroups produce or consume
// within one launch (C = true): agent-coherent accesses (they bypass the
// non-coherent caches), so a workgroup publishes them with a plain wait for
// its stores instead of writing back the whole L2. C = false: plain access.
template <bool C, typename S>
__device__ __forceinline__ S ld_c(const S* p) {
  if constexpr (C) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
template <bool C, typename S>
__device__ __forceinline__ void st_c(S* p, S v) {
  if constexpr (C) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}

// acc[c] += sum_k Mt[k*nout + o] * vin[k], o = lane + c*T (o < nout);
// D bounds the output dimension (compile-time chunk count C = ceil(D / T)).
template <typename S, int T, int D = kMaxDim>
__device__ __forceinline__ void mv_acc(S (&acc)[(D + T - 1) / T], const S* __restrict__ Mt,
                                       int nin, int nout, const S* vin, int lane) {
  constexpr int C = (D + T - 1) / T;
  int k = 0;
  for (; k + 4 <= nin; k += 4) {
    const S v0 = vin[k], v1 = vin[k + 1], v2 = vin[k + 2], v3 = vin[k + 3];
    const S* r0 = Mt + (size_t)k * nout;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int o = lane + c * T;
      if (o < nout) {
        const S m0 = r0[o], m1 = r0[nout + o], m2 = r0[2 * nout + o], m3 = r0[3 * nout + o];
        acc[c] += m0 * v0 + m1 * v1 + m2 * v2 + m3 * v3;
      }
    }
  }
  for (; k < nin; ++k) {
    const S vk = vin[k];
    const S* r0 = Mt + (size_t)k * nout;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int o = lane + c * T;
      if (o < nout) acc[c] += r0[o] * vk;
    }
  }
}

// Offsets in the canonical layout (closed forms of the breadth-first sizes).
template <typename S>
struct Off {
  const DevProb<S>& P;
  __device__ Off(const DevProb<S>& p) : P(p) {}
  __device__ long long x(int i) const { return 1 + (long long)i * P.nx; }
  __device__ long long u(int i) const { return P.zU + (long long)i * P.nu; }
  // z2 block of nonleaf i: y (2n+1), tau (n), s (n)
  __device__ long long z2(int i) const { return P.zZ2 + 4LL * (P.fc[i] - 1) + i; }
  // slot of s^c in its ancestor's block (s^0 at 0)
  __device__ long long s(int c) const {
    if (c == 0) return 0;
    const int a = P.anc[c];
    const int n = P.nch[a];
    return z2(a) + 3LL * n + 1 + (c - P.fc[a]);
  }
  __device__ long long tau(int c) const {
    const int a = P.anc[c];
    const int n = P.nch[a];
    return z2(a) + 2LL * n + 1 + (c - P.fc[a]);
  }
  // eta group 1 of nonleaf i: y (2n+1), s-row, x (nx), u (nu)
  __device__ long long e1(int i) const {
    return 2LL * (P.fc[i] - 1) + (long long)i * (2 + P.nx + P.nu);
  }
  __device__ long long e1s(int i) const { return e1(i) + 2LL * P.nch[i] + 1; }
  __device__ long long e1x(int i) const { return e1s(i) + 1; }
  __device__ long long e1u(int i) const { return e1x(i) + P.nx; }
  // eta group 2 of non-root c: x (nx), u (nu), a, b
  __device__ long long e2(int c) const { return P.eE2 + (long long)(c - 1) * (P.nx + P.nu + 2); }
  // eta group 3 of leaf j: x (nx), Q_N^{1/2} x (nx), a, b
  __device__ long long e3(int j) const { return P.eE3 + (long long)(j - P.nl) * (2 * P.nx + 2); }
};

// Running residual statistics of one lane (FP64).
struct StatAcc {
  double rz2 = 0, re2 = 0, cross = 0, xip = 0, xid = 0;
  __device__ void col(double rz, double Ltre, double ia) {
    rz2 += rz * rz;
    xip = fmax(xip, fabs(rz * ia - Ltre));
  }
  __device__ void row(double re, double Lrz, double ia) {
    re2 += re * re;
    cross += re * Lrz;
    xid = fmax(xid, fabs(re * ia - Lrz));
  }
};

// prox of g* on a translated SOC block (eq. S3-def, shift (0,..,0,1/2,-1/2)):
// out = w - alpha (shift + proj_SOC(w/alpha - shift)). The vector part is
// distributed over the team (wv[c] for components o = lane + c*T < len);
// the two trailing scalars (wa, wb) are held by every lane.
template <typename S, int T, int D = kMaxDim>
__device__ __forceinline__ void soc_prox(const S* wv, S* outv, int len, S wa, S wb, S& outa,
                                         S& outb, S al, int lane) {
  constexpr int C = (D * 2 + T - 1) / T;
  const S ia = S(1) / al;
  double part = 0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    if (o < len) {
      const double t = (double)(wv[c] * ia);
      part += t * t;
    }
  }
  const S va = wa * ia - S(0.5);
  const S t = wb * ia + S(0.5);
  const double n2 = team_sum<T>(part) + (double)va * (double)va;
  const S nrm = (S)sqrt(n2);
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
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    if (o < len) outv[c] = wv[c] - al * (scale * (wv[c] * ia));
  }
  outa = wa - al * (S(0.5) + scale * va);
  outb = wb - al * (S(-0.5) + pt);
}

// ---------------------------------------------------------------- family pieces
// The functions below run on one team of T lanes (T <= 64, inside one
// wavefront); lane o owns components o, o+T, ... of node vectors.

// xbar, ubar of nonleaf i: (x, u) - alpha (L* eta) on columns x^i, u^i.
template <typename S, int T, int D = kMaxDim>
__device__ __forceinline__ void fam_xbar_ubar(const DevProb<S>& P, const Off<S>& O,
                                              const S* __restrict__ z, const S* __restrict__ eta,
                                              int i, int lane, S (&xb)[(D + T - 1) / T],
                                              S (&ub)[(D + T - 1) / T]) {
  constexpr int C = (D + T - 1) / T;
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  const S al = P.alpha;
  const long long e1x = O.e1x(i), e1u = O.e1u(i);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    xb[c] = 0;
    ub[c] = 0;
    if (o < nx) {
      S acc = eta[e1x + o];
      for (int k = 0; k < n; ++k) acc += P.sq[(size_t)(fc + k) * nx + o] * eta[O.e2(fc + k) + o];
      xb[c] = z[O.x(i) + o] - al * acc;
    }
    if (o < nu) {
      S acc = eta[e1u + o];
      for (int k = 0; k < n; ++k) acc += P.sr[(size_t)(fc + k) * nu + o] * eta[O.e2(fc + k) + nx + o];
      ub[c] = z[O.u(i) + o] - al * acc;
    }
  }
}

// q of a child for the backward sweep: -xbar at a leaf (Alg. 2 start), the
// stored q otherwise. Component o < nx.
template <typename S>
__device__ __forceinline__ S fam_child_q(const DevProb<S>& P, const Off<S>& O, const S* __restrict__ z,
                                         const S* __restrict__ eta, const S* __restrict__ qbuf, int ch,
                                         int o) {
  const int nx = P.nx;
  if (ch >= P.nl) {
    const long long e3 = O.e3(ch);
    return -(z[O.x(ch) + o] - P.alpha * (eta[e3 + o] + P.sqN[(size_t)ch * nx + o] * eta[e3 + nx + o]));
  }
  return qbuf[(size_t)ch * nx + o];
}

// S2 projection of the z2 block of nonleaf i after the step z - alpha L* eta,
// and s^0 - alpha at the root. Closed form of the projection on the kernel of
// G = [aI, -I, 1, -I, -I]: (G G')^{-1} = (I - 11'/(c+n))/c, c = a^2 + 3.
template <typename S, int T, int D = kMaxDim, bool CZ = false>
__device__ __forceinline__ void fam_s2(const DevProb<S>& P, const Off<S>& O, const S* __restrict__ z,
                                       const S* __restrict__ eta, S* __restrict__ zout, int i,
                                       int lane) {
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  const S al = P.alpha;
  const long long zb = O.z2(i);
  const long long e1 = O.e1(i);
  const S es = eta[O.e1s(i)];
  const S a = P.a[i];
  const S y3h = z[zb + 2 * n] - al * (eta[e1 + 2 * n] - es);
  double gsum = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const S cc = a * a + S(3);
    const S Gs = pass ? (S)team_sum<T>(gsum) : S(0);
    double wsum = 0;
    for (int k = lane; k < n; k += T) {
      const int ch = fc + k;
      const S y1h = z[zb + k] - al * (eta[e1 + k] - P.p[ch] * es);
      const S y2h = z[zb + n + k] - al * eta[e1 + n + k];
      const long long e2c = O.e2(ch) + nx + nu;
      const S th = z[zb + 2 * n + 1 + k] - al * S(0.5) * (eta[e2c] + eta[e2c + 1]);
      S Lts;
      if (ch < P.nl) {
        Lts = eta[O.e1s(ch)];
      } else {
        const long long e3c = O.e3(ch) + 2 * nx;
        Lts = S(0.5) * (eta[e3c] + eta[e3c + 1]);
      }
      const S sh = z[zb + 3 * n + 1 + k] - al * Lts;
      const S g = a * y1h - y2h + y3h - th - sh;
      if (!pass) {
        gsum += (double)g;
      } else {
        const S w = (g - Gs / (cc + S(n))) / cc;
        wsum += (double)w;
        st_c<CZ>(zout + zb + k, y1h - a * w);
        st_c<CZ>(zout + zb + n + k, y2h + w);
        st_c<CZ>(zout + zb + 2 * n + 1 + k, th + w);
        st_c<CZ>(zout + zb + 3 * n + 1 + k, sh + w);
      }
    }
    if (pass) {
      const S Ws = (S)team_sum<T>(wsum);
      if (lane == 0) {
        st_c<CZ>(zout + zb + 2 * n, y3h - Ws);
        if (i == 0) st_c<CZ>(zout, z[0] - al * es - al);
      }
    }
  }
}

// Dual update and residual statistics of the rows of child ch (group 2, and
// group 3 if ch is a leaf) and of the columns tau^ch (and x^ch, s^ch at a
// leaf). xp/xo: x+^i and x^i (lane chunks); vu: u+^i in LDS; xc: x+^ch (lane
// chunks); vr: LDS scratch of 2*VM; gx, gu accumulate the group-2 part of
// L* r_eta on columns x^i, u^i.
template <typename S, int T, int D = kMaxDim, bool CZ = false>
__device__ __forceinline__ void fam_dual_child(const DevProb<S>& P, const Off<S>& O,
                                               const S* __restrict__ z, const S* __restrict__ eta,
                                               const S* __restrict__ zout, S* __restrict__ eout, int i,
                                               int ch, int lane, const S (&xp)[(D + T - 1) / T],
                                               const S (&xo)[(D + T - 1) / T], const S* vu,
                                               const S (&xc)[(D + T - 1) / T], S* vr,
                                               S (&gx)[(D + T - 1) / T],
                                               S (&gu)[(D + T - 1) / T], StatAcc& st) {
  constexpr int C = (D + T - 1) / T;
  constexpr int C2 = (2 * D + T - 1) / T;
  const int nx = P.nx, nu = P.nu;
  const S al = P.alpha;
  const S ia = S(1) / al;
  const long long ui = O.u(i);
  // ---- group 2: (Q^{1/2} x^i, R^{1/2} u^i, tau/2, tau/2) in SOC + shift
  const long long e2 = O.e2(ch);
  const long long tpos = O.tau(ch);
  const S tau = z[tpos], taup = ld_c<CZ>(zout + tpos);
  S wv[C2], ov[C2], lz[C2];
#pragma unroll
  for (int c = 0; c < C2; ++c) {
    const int o = lane + c * T;
    wv[c] = 0;
    ov[c] = 0;
    lz[c] = 0;
    if (o < nx) {
      const S xpo = xp[c < C ? c : C - 1], xoo = xo[c < C ? c : C - 1];
      const S sqv = P.sq[(size_t)ch * nx + o];
      wv[c] = eta[e2 + o] + al * sqv * (S(2) * xpo - xoo);
      lz[c] = sqv * (xoo - xpo);
    } else if (o < nx + nu) {
      const int ou = o - nx;
      const S upo = vu[ou], uoo = z[ui + ou];
      const S srv = P.sr[(size_t)ch * nu + ou];
      wv[c] = eta[e2 + o] + al * srv * (S(2) * upo - uoo);
      lz[c] = srv * (uoo - upo);
    }
  }
  const S wa = eta[e2 + nx + nu] + al * S(0.5) * (S(2) * taup - tau);
  const S wb = eta[e2 + nx + nu + 1] + al * S(0.5) * (S(2) * taup - tau);
  S oa, ob;
  soc_prox<S, T, D>(wv, ov, nx + nu, wa, wb, oa, ob, al, lane);
  const S rtau = tau - taup;
#pragma unroll
  for (int c = 0; c < C2; ++c) {
    const int o = lane + c * T;
    if (o < nx + nu) {
      eout[e2 + o] = ov[c];
      const S re = eta[e2 + o] - ov[c];
      vr[o] = re;
      st.row((double)re, (double)lz[c], (double)ia);
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    if (o < nx) gx[c] += P.sq[(size_t)ch * nx + o] * vr[o];
    if (o < nu) gu[c] += P.sr[(size_t)ch * nu + o] * vr[nx + o];
  }
  wave_lds_sync();
  if (lane == 0) {
    const S rea = eta[e2 + nx + nu] - oa, reb = eta[e2 + nx + nu + 1] - ob;
    eout[e2 + nx + nu] = oa;
    eout[e2 + nx + nu + 1] = ob;
    st.row((double)rea, 0.5 * (double)rtau, (double)ia);
    st.row((double)reb, 0.5 * (double)rtau, (double)ia);
    st.col((double)rtau, 0.5 * ((double)rea + (double)reb), (double)ia);
  }
  if (ch < P.nl) return;
  // ---- group 3 of a leaf: box on x, (Q_N^{1/2} x, s/2, s/2) in SOC + shift
  const long long e3 = O.e3(ch);
  const long long spos = O.s(ch);
  const S sv = z[spos], svp = ld_c<CZ>(zout + spos);
  S wq[C2], oq[C2];
  S rex[C], xin[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    rex[c] = 0;
    xin[c] = 0;
    if (o < nx) {
      const S xcin = z[O.x(ch) + o];
      xin[c] = xcin;
      const S wbx = eta[e3 + o] + al * (S(2) * xc[c] - xcin);
      const S pb = wbx - al * clampv(wbx * ia, P.xlo[(size_t)ch * nx + o], P.xhi[(size_t)ch * nx + o]);
      eout[e3 + o] = pb;
      rex[c] = eta[e3 + o] - pb;
      st.row((double)rex[c], (double)(xcin - xc[c]), (double)ia);
    }
  }
#pragma unroll
  for (int c = 0; c < C2; ++c) {
    const int o = lane + c * T;
    wq[c] = 0;
    oq[c] = 0;
    if (c < C && o < nx) {
      const int cc = c < C ? c : C - 1;
      wq[c] = eta[e3 + nx + o] + al * P.sqN[(size_t)ch * nx + o] * (S(2) * xc[cc] - xin[cc]);
    }
  }
  const S wsa = eta[e3 + 2 * nx] + al * S(0.5) * (S(2) * svp - sv);
  const S wsb = eta[e3 + 2 * nx + 1] + al * S(0.5) * (S(2) * svp - sv);
  S osa, osb;
  soc_prox<S, T, D>(wq, oq, nx, wsa, wsb, osa, osb, al, lane);
  const S rs = sv - svp;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    if (o < nx) {
      eout[e3 + nx + o] = oq[c];
      const S reqv = eta[e3 + nx + o] - oq[c];
      const S sqn = P.sqN[(size_t)ch * nx + o];
      st.row((double)reqv, (double)(sqn * (xin[c] - xc[c])), (double)ia);
      // column x^ch of a leaf: L* r_eta = r_eta(box) + Q_N^{1/2} r_eta(q)
      st.col((double)(xin[c] - xc[c]), (double)(rex[c] + sqn * reqv), (double)ia);
    }
  }
  if (lane == 0) {
    eout[e3 + 2 * nx] = osa;
    eout[e3 + 2 * nx + 1] = osb;
    const S rea3 = eta[e3 + 2 * nx] - osa, reb3 = eta[e3 + 2 * nx + 1] - osb;
    st.row((double)rea3, 0.5 * (double)rs, (double)ia);
    st.row((double)reb3, 0.5 * (double)rs, (double)ia);
    st.col((double)rs, 0.5 * ((double)rea3 + (double)reb3), (double)ia);
  }
}

// Dual update of group 1 of nonleaf i: y in K* = R^{2n}_+ x R, s - b'y in
// R_+, (x, u) in the box; columns y^i, s^i, x^i, u^i of L* r_eta.
template <typename S, int T, int D = kMaxDim, bool CZ = false>
__device__ __forceinline__ void fam_dual_node(const DevProb<S>& P, const Off<S>& O,
                                              const S* __restrict__ z, const S* __restrict__ eta,
                                              const S* __restrict__ zout, S* __restrict__ eout, int i,
                                              int lane, const S (&xp)[(D + T - 1) / T],
                                              const S (&xo)[(D + T - 1) / T],
                                              const S (&up)[(D + T - 1) / T],
                                              const S (&uo)[(D + T - 1) / T],
                                              const S (&gx)[(D + T - 1) / T],
                                              const S (&gu)[(D + T - 1) / T], StatAcc& st) {
  constexpr int C = (D + T - 1) / T;
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  const S al = P.alpha;
  const S ia = S(1) / al;
  const long long zb = O.z2(i);
  const long long e1 = O.e1(i);
  const long long spos = O.s(i);
  const S si = z[spos], sip = ld_c<CZ>(zout + spos);
  double bw = 0, bry = 0;
  for (int k = lane; k < n; k += T) {
    const S pk = P.p[fc + k];
    const S y1 = z[zb + k], y1p = ld_c<CZ>(zout + zb + k);
    bw += (double)(pk * (S(2) * y1p - y1));
    bry += (double)(pk * (y1 - y1p));
  }
  const S y3 = z[zb + 2 * n], y3p = ld_c<CZ>(zout + zb + 2 * n);
  const S bW = (S)team_sum<T>(bw) + (S(2) * y3p - y3);
  const S bR = (S)team_sum<T>(bry) + (y3 - y3p);
  const S ws = eta[e1 + 2 * n + 1] + al * ((S(2) * sip - si) - bW);
  const S es_new = ws < S(0) ? ws : S(0);
  const S res_ = eta[e1 + 2 * n + 1] - es_new;
  for (int k = lane; k < 2 * n + 1; k += T) {
    const S y = z[zb + k], yp = ld_c<CZ>(zout + zb + k);
    const S w = eta[e1 + k] + al * (S(2) * yp - y);
    const S ep = (k < 2 * n) ? (w < S(0) ? w : S(0)) : S(0);
    eout[e1 + k] = ep;
    const S re = eta[e1 + k] - ep;
    const S ry = y - yp;
    st.row((double)re, (double)ry, (double)ia);
    const S bk = (k < n) ? P.p[fc + k] : ((k == 2 * n) ? S(1) : S(0));
    st.col((double)ry, (double)(re - bk * res_), (double)ia);
  }
  if (lane == 0) {
    eout[e1 + 2 * n + 1] = es_new;
    const S rsi = si - sip;
    st.row((double)res_, (double)(rsi - bR), (double)ia);
    st.col((double)rsi, (double)res_, (double)ia);
  }
  const long long e1x = O.e1x(i), e1u = O.e1u(i);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    if (o < nx) {
      const S w = eta[e1x + o] + al * (S(2) * xp[c] - xo[c]);
      const S ep = w - al * clampv(w * ia, P.xlo[(size_t)i * nx + o], P.xhi[(size_t)i * nx + o]);
      eout[e1x + o] = ep;
      const S re = eta[e1x + o] - ep;
      const S rz = xo[c] - xp[c];
      st.row((double)re, (double)rz, (double)ia);
      st.col((double)rz, (double)(re + gx[c]), (double)ia);
    }
    if (o < nu) {
      const S w = eta[e1u + o] + al * (S(2) * up[c] - uo[c]);
      const S ep = w - al * clampv(w * ia, P.ulo[(size_t)i * nu + o], P.uhi[(size_t)i * nu + o]);
      eout[e1u + o] = ep;
      const S re = eta[e1u + o] - ep;
      const S rz = uo[c] - up[c];
      st.row((double)re, (double)rz, (double)ia);
      st.col((double)rz, (double)(re + gu[c]), (double)ia);
    }
  }
}

// Fixed-order block reduction of the statistics into one partial record.
__device__ __forceinline__ void block_stats(const StatAcc& st, double* __restrict__ partials) {
  __shared__ double red[kStats][256];
  red[0][threadIdx.x] = st.rz2;
  red[1][threadIdx.x] = st.re2;
  red[2][threadIdx.x] = st.cross;
  red[3][threadIdx.x] = st.xip;
  red[4][threadIdx.x] = st.xid;
  __syncthreads();
  for (int s = blockDim.x / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
      red[2][threadIdx.x] += red[2][threadIdx.x + s];
      red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + s]);
      red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x < kStats) partials[(size_t)blockIdx.x * kStats + threadIdx.x] = red[threadIdx.x][0];
}

// Backward step of nonleaf i by one team (Alg. 2 backward sweep with
// W = sum_c Abar^c' P^c B^c): d = R~^{-1}(ubar - sum_c B^c' q^c),
// q = K'(d - ubar) + W d - xbar + sum_c Abar^c' q^c. LDS: 3 VM per team.
template <typename S, int T, int D = kMaxDim>
__device__ __forceinline__ void fam_bwd_team(const DevProb<S>& P, const S* __restrict__ xbar,
                                             const S* __restrict__ ubar, S* __restrict__ qbuf,
                                             S* __restrict__ dbuf, int i, int lane, S* lds, int VM) {
  constexpr int C = (D + T - 1) / T;
  S* vq = lds;
  S* vg = vq + VM;
  S* vd = vg + VM;
  const int nx = P.nx, nu = P.nu;
  const int fc = P.fc[i], n = P.nch[i];
  S xb[C], ub[C], sA[C], h[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    xb[c] = (o < nx) ? xbar[(size_t)i * nx + o] : S(0);
    ub[c] = (o < nu) ? ubar[(size_t)i * nu + o] : S(0);
    sA[c] = h[c] = 0;
  }
  for (int k = 0; k < n; ++k) {
    const int ch = fc + k;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int o = lane + c * T;
      if (o < nx) vq[o] = qbuf[(size_t)ch * nx + o];
    }
    wave_lds_sync();
    mv_acc<S, T, D>(h, P.BR + (size_t)ch * nx * nu, nx, nu, vq, lane);
    mv_acc<S, T, D>(sA, P.AbR + (size_t)ch * nx * nx, nx, nx, vq, lane);
    wave_lds_sync();
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    if (o < nu) vg[o] = ub[c] - h[c];
  }
  wave_lds_sync();
  S dv[C];
#pragma unroll
  for (int c = 0; c < C; ++c) dv[c] = 0;
  mv_acc<S, T, D>(dv, P.Rinv + (size_t)i * nu * nu, nu, nu, vg, lane);
  wave_lds_sync();
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    if (o < nu) {
      vg[o] = dv[c] - ub[c];
      vd[o] = dv[c];
      dbuf[(size_t)i * nu + o] = dv[c];
    }
  }
  wave_lds_sync();
  S qi[C];
#pragma unroll
  for (int c = 0; c < C; ++c) qi[c] = sA[c] - xb[c];
  mv_acc<S, T, D>(qi, P.KR + (size_t)i * nu * nx, nu, nx, vg, lane);
  mv_acc<S, T, D>(qi, P.WC + (size_t)i * nu * nx, nu, nx, vd, lane);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    if (o < nx) qbuf[(size_t)i * nx + o] = qi[c];
  }
  wave_lds_sync();
}

// Forward step of nonleaf i by one team (Alg. 2 forward sweep):
// u = K x + d, x^c = Abar^c x + B^c d; x^0 = x0 at the root. LDS: 2 VM.
template <typename S, int T, int D = kMaxDim>
__device__ __forceinline__ void fam_fwd_team(const DevProb<S>& P, S* __restrict__ zout,
                                             const S* __restrict__ dbuf, const double* __restrict__ x0,
                                             int i, int lane, S* lds, int VM) {
  constexpr int C = (D + T - 1) / T;
  S* vx = lds;
  S* vd = vx + VM;
  const Off<S> O(P);
  const int nx = P.nx, nu = P.nu;
  const int fc = P.fc[i], n = P.nch[i];
  const long long ui = O.u(i);
  S up[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    up[c] = 0;
    if (o < nx) {
      S xv;
      if (i == 0) {
        xv = (S)x0[o];
        zout[1 + o] = xv;
      } else {
        xv = zout[O.x(i) + o];
      }
      vx[o] = xv;
    }
    if (o < nu) {
      const S dd = dbuf[(size_t)i * nu + o];
      vd[o] = dd;
      up[c] = dd;
    }
  }
  wave_lds_sync();
  mv_acc<S, T, D>(up, P.KC + (size_t)i * nx * nu, nx, nu, vx, lane);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    if (o < nu) zout[ui + o] = up[c];
  }
  for (int k = 0; k < n; ++k) {
    const int ch = fc + k;
    S xc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) xc[c] = 0;
    mv_acc<S, T, D>(xc, P.AbC + (size_t)ch * nx * nx, nx, nx, vx, lane);
    mv_acc<S, T, D>(xc, P.BC + (size_t)ch * nu * nx, nu, nx, vd, lane);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int o = lane + c * T;
      if (o < nx) zout[O.x(ch) + o] = xc[c];
    }
  }
  wave_lds_sync();
}

// pre-pass of family i by one team: xbar, ubar; leaf children's q = -xbar;
// S2 projection of the z2 block; s^0 - alpha at the root.
template <typename S, int T, int D = kMaxDim>
__device__ __forceinline__ void fam_pre_team(const DevProb<S>& P, const S* __restrict__ z,
                                             const S* __restrict__ eta, S* __restrict__ zout,
                                             S* __restrict__ xbar, S* __restrict__ ubar,
                                             S* __restrict__ qbuf, int i, int lane) {
  constexpr int C = (D + T - 1) / T;
  const Off<S> O(P);
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  S xb[C], ub[C];
  fam_xbar_ubar<S, T, D>(P, O, z, eta, i, lane, xb, ub);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    if (o < nx) xbar[(size_t)i * nx + o] = xb[c];
    if (o < nu) ubar[(size_t)i * nu + o] = ub[c];
  }
  if (fc >= P.nl) {  // children are leaves
    for (int k = 0; k < n; ++k)
      for (int o = lane; o < nx; o += T)
        qbuf[(size_t)(fc + k) * nx + o] = fam_child_q<S>(P, O, z, eta, qbuf, fc + k, o);
  }
  fam_s2<S, T, D>(P, O, z, eta, zout, i, lane);
}

// post-pass of family i by one team: dual update and residual statistics.
// LDS: 3 VM per team.
template <typename S, int T, int D = kMaxDim, bool CZ = false>
__device__ __forceinline__ void fam_post_team(const DevProb<S>& P, const S* __restrict__ z,
                                              const S* __restrict__ eta, const S* __restrict__ zout,
                                              S* __restrict__ eout, int i, int lane, S* lds, int VM,
                                              StatAcc& st) {
  constexpr int C = (D + T - 1) / T;
  S* vu = lds;
  S* vr = vu + VM;
  const Off<S> O(P);
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  const long long ui = O.u(i);
  S xp[C], xo[C], up[C], uo[C], gx[C], gu[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int o = lane + c * T;
    xp[c] = xo[c] = up[c] = uo[c] = gx[c] = gu[c] = 0;
    if (o < nx) {
      xp[c] = ld_c<CZ>(zout + O.x(i) + o);
      xo[c] = z[O.x(i) + o];
    }
    if (o < nu) {
      up[c] = ld_c<CZ>(zout + ui + o);
      uo[c] = z[ui + o];
      vu[o] = up[c];
    }
  }
  wave_lds_sync();
  for (int k = 0; k < n; ++k) {
    const int ch = fc + k;
    S xc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int o = lane + c * T;
      xc[c] = (o < nx) ? ld_c<CZ>(zout + O.x(ch) + o) : S(0);
    }
    fam_dual_child<S, T, D, CZ>(P, O, z, eta, zout, eout, i, ch, lane, xp, xo, vu, xc, vr, gx, gu, st);
  }
  fam_dual_node<S, T, D, CZ>(P, O, z, eta, zout, eout, i, lane, xp, xo, up, uo, gx, gu, st);
  wave_lds_sync();
}

// M d = (d_z - alpha L* d_eta, d_eta - alpha L d_z), the metric of the
// SuperMann line search (Alg. 3): one team of T lanes per family writes the
// family's columns of L* (y^i, s^i, x^i, u^i, tau^c, and x^c, s^c of leaf
// children) and its rows of L (groups 1, 2 of its children, 3 of its leaf
// children), so every entry of M d is written once.
template <typename S, int T>
__device__ __forceinline__ void fam_apply_M(const DevProb<S>& P, const S* __restrict__ d, S* __restrict__ Md, int i,
                                            int lane) {
  const Off<S> O(P);
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  const S al = P.alpha;
  const S* dz = d;
  const S* de = d + P.nz;
  S* mz = Md;
  S* me = Md + P.nz;
  const long long zb = O.z2(i), e1 = O.e1(i);
  const S es = de[O.e1s(i)];
  // columns y^i and s^i of L*; rows y and s - b'y of group 1
  double by = 0;
  for (int k = lane; k < 2 * n + 1; k += T) {
    const S bk = (k < n) ? P.p[fc + k] : ((k == 2 * n) ? S(1) : S(0));
    const S yk = dz[zb + k];
    mz[zb + k] = yk - al * (de[e1 + k] - bk * es);
    me[e1 + k] = de[e1 + k] - al * yk;
    by += (double)(bk * yk);
  }
  const S bys = (S)team_sum<T>(by);
  if (lane == 0) {
    mz[O.s(i)] = dz[O.s(i)] - al * es;
    me[O.e1s(i)] = es - al * (dz[O.s(i)] - bys);
  }
  // columns x^i, u^i; rows x, u of group 1 and of the children's group 2
  for (int o = lane; o < nx; o += T) {
    const S xo = dz[O.x(i) + o];
    S acc = de[O.e1x(i) + o];
    for (int k = 0; k < n; ++k) {
      const int c = fc + k;
      const S sq = P.sq[(size_t)c * nx + o];
      const long long e2 = O.e2(c) + o;
      acc += sq * de[e2];
      me[e2] = de[e2] - al * sq * xo;
    }
    mz[O.x(i) + o] = xo - al * acc;
    me[O.e1x(i) + o] = de[O.e1x(i) + o] - al * xo;
  }
  for (int o = lane; o < nu; o += T) {
    const S uo = dz[O.u(i) + o];
    S acc = de[O.e1u(i) + o];
    for (int k = 0; k < n; ++k) {
      const int c = fc + k;
      const S sr = P.sr[(size_t)c * nu + o];
      const long long e2 = O.e2(c) + nx + o;
      acc += sr * de[e2];
      me[e2] = de[e2] - al * sr * uo;
    }
    mz[O.u(i) + o] = uo - al * acc;
    me[O.e1u(i) + o] = de[O.e1u(i) + o] - al * uo;
  }
  // tau^c and the two scalars of group 2
  for (int k = lane; k < n; k += T) {
    const int c = fc + k;
    const long long e2 = O.e2(c) + nx + nu;
    const S tc = dz[O.tau(c)];
    mz[O.tau(c)] = tc - al * S(0.5) * (de[e2] + de[e2 + 1]);
    me[e2] = de[e2] - al * S(0.5) * tc;
    me[e2 + 1] = de[e2 + 1] - al * S(0.5) * tc;
  }
  if (fc < P.nl) return;
  // leaf children: columns x^c, s^c; rows of group 3
  for (int k = 0; k < n; ++k) {
    const int c = fc + k;
    const long long e3 = O.e3(c);
    for (int o = lane; o < nx; o += T) {
      const S xc = dz[O.x(c) + o];
      const S sqn = P.sqN[(size_t)c * nx + o];
      mz[O.x(c) + o] = xc - al * (de[e3 + o] + sqn * de[e3 + nx + o]);
      me[e3 + o] = de[e3 + o] - al * xc;
      me[e3 + nx + o] = de[e3 + nx + o] - al * sqn * xc;
    }
    if (lane == 0) {
      const S sc = dz[O.s(c)];
      mz[O.s(c)] = sc - al * S(0.5) * (de[e3 + 2 * nx] + de[e3 + 2 * nx + 1]);
      me[e3 + 2 * nx] = de[e3 + 2 * nx] - al * S(0.5) * sc;
      me[e3 + 2 * nx + 1] = de[e3 + 2 * nx + 1] - al * S(0.5) * sc;
    }
  }
}

// Tagged words: element e of a vector occupies kTW<S> 64-bit words, each
// holding (epoch << 32) | one 32-bit half of the value.
template <typename S>
constexpr int kTW = sizeof(S) / 4;

template <typename S>
__device__ __forceinline__ void put_tagged(unsigned long long* p, S v, unsigned tag) {
  unsigned h[kTW<S>];
  __builtin_memcpy(h, &v, sizeof(S));
  const unsigned long long hi = (unsigned long long)tag << 32;
#pragma unroll
  for (int k = 0; k < kTW<S>; ++k) __hip_atomic_store(p + k, hi | h[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename S>
__device__ __forceinline__ bool get_tagged(const unsigned long long* p, unsigned tag, S& v) {
  unsigned h[kTW<S>];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < kTW<S>; ++k) {
    const unsigned long long w = __hip_atomic_load(p + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ok = ok && (unsigned)(w >> 32) == tag;
    h[k] = (unsigned)w;
  }
  __builtin_memcpy(&v, h, sizeof(S));
  return ok;
}

}  // namespace spk
