// HIP kernels (gfx950) of the SPOCK hot path: one Chambolle-Pock operator T
// under the splitting of section 5, plus the vector kernels of the
// SuperMann / Anderson layer (section 6).
//
// Work decomposition. Every nonleaf node i owns a "family": itself and its
// children. A team of T lanes (T in {8,16,32,64}, inside one wavefront) runs
// one family; lane o owns component o (and o+T, o+2T, ...) of every state or
// input vector. A stage of the tree is one launch: all families of a stage
// are independent (the "in parallel" loops of Alg. 1 and Alg. 2).
//
//  backward launch (stage N-1 .. 0), family i:
//    xbar, ubar = (x, u) - alpha (L* eta)       [L* columns of family i]
//    q of leaf children = -xbar(leaf)            [Alg. 2 initialisation]
//    d = R~^{-1}(ubar - sum_c B^c' q^c)
//    q = K'(d - ubar) - xbar + W d + sum_c Abar^c' q^c,
//        with W = sum_c Abar^c' P^c B^c          [Alg. 2, regrouped]
//    S2 projection of the family's z2 block and s^0 - alpha at the root
//  forward launch (stage 0 .. N-1), family i:
//    u = K x + d, x^c = Abar^c x + B^c d          [Alg. 2 forward sweep]
//    eta+ = prox_{alpha g*}(eta + alpha L(2 z+ - z)) on the family's rows
//    residual statistics of r = v - T(v): ||r_z||^2, ||r_eta||^2,
//    <r_eta, L r_z>, ||xi_p||_inf, ||xi_d||_inf   [section 3, Alg. 3]
// Every row of L and every column of L* belongs to exactly one family, so
// L r_z and L* r_eta are formed locally without a second pass.
#include "device_common.h"

#include <math.h>
#include <algorithm>
#include <cstdint>
#include <initializer_list>

namespace spk {

// ---------------------------------------------------------------- pre / post passes
// Both passes are fully parallel over families (no recursion): team of T
// lanes per family, 256 / T families per block, one launch for the tree.

// pre-pass: xbar, ubar = (x, u) - alpha L* eta on columns x^i, u^i; leaf
// children seed the backward sweep with q = -xbar (Alg. 2 start); the z2
// block is projected on S2; s^0 - alpha at the root.
template <typename S, int T>
__global__ void __launch_bounds__(256) k_pre(DevProb<S> P, const S* __restrict__ z,
                                             const S* __restrict__ eta, S* __restrict__ zout,
                                             S* __restrict__ xbar, S* __restrict__ ubar,
                                             S* __restrict__ qbuf) {
  const int lane = threadIdx.x % T;
  const int f = blockIdx.x * (blockDim.x / T) + threadIdx.x / T;
  if (f >= P.nl) return;  // whole teams only; no block barrier below
  fam_pre_team<S, T>(P, z, eta, zout, xbar, ubar, qbuf, f, lane);
}

// post-pass: eta+ = prox_{alpha g*}(eta + alpha L(2 z+ - z)) on the family's
// rows and the residual statistics of r = v - T(v) on its rows and columns.
template <typename S, int T>
__global__ void __launch_bounds__(256) k_post(DevProb<S> P, const S* __restrict__ z,
                                              const S* __restrict__ eta, const S* __restrict__ zout,
                                              S* __restrict__ eout, int VM,
                                              double* __restrict__ partials) {
  extern __shared__ unsigned char smem_raw[];
  S* smem = reinterpret_cast<S*>(smem_raw);
  const int lane = threadIdx.x % T;
  const int team = threadIdx.x / T;
  const int f = blockIdx.x * (blockDim.x / T) + team;
  StatAcc st;
  if (f < P.nl) fam_post_team<S, T>(P, z, eta, zout, eout, f, lane, smem + (size_t)team * 3 * VM, VM, st);
  block_stats(st, partials);
}

// node-parallel post-pass: the same update and statistics as k_post, with
// the children of a family on separate teams. Block b owns the families
// [bfam[b], bfam[b + 1]) and their children (one contiguous run of at most
// cap nodes). Phase A: a team per child does the rows of group 2 (and group
// 3 at a leaf) and leaves that child's part of L* r_eta on the columns x^i,
// u^i of its parent in LDS. Phase B: a team per family adds those parts in
// child order (the order the family-serial kernel uses) and does group 1
// and the columns x^i, u^i. No family chain: every child is independent.
template <typename S, int T>
__global__ void __launch_bounds__(256) k_post_nodes(DevProb<S> P, const int* __restrict__ bfam,
                                                    const S* __restrict__ z, const S* __restrict__ eta,
                                                    const S* __restrict__ zout, S* __restrict__ eout, int VM,
                                                    double* __restrict__ partials) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int TPB = 256 / T;
  constexpr int C = (kMaxDim + T - 1) / T;
  S* smem = reinterpret_cast<S*>(smem_raw);
  const int lane = threadIdx.x % T;
  const int team = threadIdx.x / T;
  const int nx = P.nx, nu = P.nu, GW = nx + nu;
  S* mine = smem + (size_t)team * 3 * VM;  // u+ of the parent (VM), scratch (2 VM)
  S* G = smem + (size_t)TPB * 3 * VM;      // [children of the block][nx + nu]
  const Off<S> O(P);
  const int f0 = bfam[blockIdx.x], f1 = bfam[blockIdx.x + 1];
  const int c0 = P.fc[f0];
  const int c1 = P.fc[f1 - 1] + P.nch[f1 - 1];
  StatAcc st;
  for (int ch = c0 + team; ch < c1; ch += TPB) {
    const int i = P.anc[ch];
    const long long ui = O.u(i);
    S xp[C], xo[C], xc[C], gx[C], gu[C];
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int o = lane + c * T;
      xp[c] = xo[c] = xc[c] = gx[c] = gu[c] = 0;
      if (o < nx) {
        xp[c] = zout[O.x(i) + o];
        xo[c] = z[O.x(i) + o];
        if (ch >= P.nl) xc[c] = zout[O.x(ch) + o];
      }
      if (o < nu) mine[o] = zout[ui + o];
    }
    wave_lds_sync();
    fam_dual_child<S, T>(P, O, z, eta, zout, eout, i, ch, lane, xp, xo, mine, xc, mine + VM, gx, gu, st);
    S* g = G + (size_t)(ch - c0) * GW;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int o = lane + c * T;
      if (o < nx) g[o] = gx[c];
      if (o < nu) g[nx + o] = gu[c];
    }
  }
  __syncthreads();
  for (int f = f0 + team; f < f1; f += TPB) {
    const long long ui = O.u(f);
    const int fc = P.fc[f], n = P.nch[f];
    S xp[C], xo[C], up[C], uo[C], gx[C], gu[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int o = lane + c * T;
      xp[c] = xo[c] = up[c] = uo[c] = gx[c] = gu[c] = 0;
      if (o < nx) {
        xp[c] = zout[O.x(f) + o];
        xo[c] = z[O.x(f) + o];
      }
      if (o < nu) {
        up[c] = zout[ui + o];
        uo[c] = z[ui + o];
      }
    }
    for (int k = 0; k < n; ++k) {
      const S* g = G + (size_t)(fc + k - c0) * GW;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int o = lane + c * T;
        if (o < nx) gx[c] += g[o];
        if (o < nu) gu[c] += g[nx + o];
      }
    }
    fam_dual_node<S, T>(P, O, z, eta, zout, eout, f, lane, xp, xo, up, uo, gx, gu, st);
  }
  block_stats(st, partials);
}

// Flat post-pass: one wavefront per unit, a unit being a nonleaf family
// (group 1 of i and group 2 of each child c) or a leaf (group 3). The rows
// and columns a unit touches are exactly those of the family-serial form,
// so no unit waits on another. A family's columns x^i and u^i share one
// index k < nx + nu with the first rows of each child's group 2, so every
// lane holds the same two components of all of them. Offsets are
// arithmetic in i once fc[i] and nch[i] are read, and the slot of s^i in
// its ancestor's block comes from spos[i]: one level of scalar loads, then
// every data load of the unit at once. Statistics: wavefront shuffles,
// then the block's four wavefronts in order, one record per block.
template <typename S>
__device__ __forceinline__ void flat_family(const DevProb<S>& P, const Off<S>& O, const long long* __restrict__ spos,
                                            const S* __restrict__ z, const S* __restrict__ eta,
                                            const S* __restrict__ zout, S* __restrict__ eout, int i, int lane,
                                            StatAcc& st) {
  const int nx = P.nx, nu = P.nu, K = nx + nu;
  const int fc = P.fc[i], n = P.nch[i];
  const S al = P.alpha;
  const S ia = S(1) / al;
  const long long e1 = O.e1(i), e1x = e1 + 2LL * n + 2, zb = O.z2(i);
  const long long xi = O.x(i), ui = O.u(i);
  const long long sp = spos[i];
  // One batch of loads, with clamped indices and no branches, so that
  // every load of the unit is in flight at once: columns x^i, u^i (slot s:
  // k = lane + 64 s), the y block (one entry per lane when 2n + 1 <= 64)
  // and the scalars.
  // FP64 loads the box rows' and the y block's operands after the cone
  // blocks (fewer live registers across them)
  constexpr bool kLateBox = sizeof(S) == 8;
  bool on[2];
  S zp[2], zo[2], lo[2], hi[2], eb[2], gc[2];
  auto load_box = [&](int s) {
    const int k = lane + 64 * s;
    const int kk = on[s] ? k : 0;
    const bool isx = kk < nx;
    const size_t bi = isx ? (size_t)i * nx + kk : (size_t)i * nu + (kk - nx);
    lo[s] = (isx ? P.xlo : P.ulo)[bi];
    hi[s] = (isx ? P.xhi : P.uhi)[bi];
    eb[s] = eta[e1x + kk];
  };
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int k = lane + 64 * s;
    on[s] = k < K;
    const int kk = on[s] ? k : 0;
    const bool isx = kk < nx;
    const long long zi = isx ? xi + kk : ui + (kk - nx);
    zp[s] = zout[zi];
    zo[s] = z[zi];
    if (!kLateBox) load_box(s);
    gc[s] = 0;
  }
  const int ny = 2 * n + 1;
  const int ky = lane < ny ? lane : 0;
  S yv, ypv, eyv, pk, si, sip, y3, y3p, es;
  auto load_y = [&]() {
    yv = z[zb + ky];
    ypv = zout[zb + ky];
    eyv = eta[e1 + ky];
    pk = P.p[fc + (lane < n ? lane : 0)];
    si = z[sp];
    sip = zout[sp];
    y3 = z[zb + 2 * n];
    y3p = zout[zb + 2 * n];
    es = eta[e1 + 2 * n + 1];
  };
  if (!kLateBox) load_y();
  // group 2 of every child: (Q^{1/2} x^i, R^{1/2} u^i, tau/2, tau/2)
  for (int c = fc; c < fc + n; ++c) {
    const long long e2 = O.e2(c);
    const long long tp = zb + 2LL * n + 1 + (c - fc);
    S sc[2], ev[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int kk = on[s] ? lane + 64 * s : 0;
      sc[s] = kk < nx ? P.sq[(size_t)c * nx + kk] : P.sr[(size_t)c * nu + (kk - nx)];
      ev[s] = eta[e2 + kk];
    }
    const S tau = z[tp], taup = zout[tp];
    const S ea = eta[e2 + K], ebb = eta[e2 + K + 1];
    S wv[2], ov[2], lz[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      wv[s] = on[s] ? ev[s] + al * sc[s] * (S(2) * zp[s] - zo[s]) : S(0);
      lz[s] = sc[s] * (zo[s] - zp[s]);
      ov[s] = 0;
    }
    const S wa = ea + al * S(0.5) * (S(2) * taup - tau);
    const S wb = ebb + al * S(0.5) * (S(2) * taup - tau);
    S oa, ob;
    soc_prox<S, 64, 64>(wv, ov, K, wa, wb, oa, ob, al, lane);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (on[s]) {
        eout[e2 + lane + 64 * s] = ov[s];
        const S re = ev[s] - ov[s];
        st.row((double)re, (double)lz[s], (double)ia);
        gc[s] += sc[s] * re;
      }
    }
    if (lane == 0) {
      const S rtau = tau - taup;
      const S rea = ea - oa, reb = ebb - ob;
      eout[e2 + K] = oa;
      eout[e2 + K + 1] = ob;
      st.row((double)rea, 0.5 * (double)rtau, (double)ia);
      st.row((double)reb, 0.5 * (double)rtau, (double)ia);
      st.col((double)rtau, 0.5 * ((double)rea + (double)reb), (double)ia);
    }
  }
  // group 1: the boxes on (x^i, u^i) and the columns x^i, u^i
  if (kLateBox) {
#pragma unroll
    for (int s = 0; s < 2; ++s) load_box(s);
    load_y();
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (on[s]) {
      const S w = eb[s] + al * (S(2) * zp[s] - zo[s]);
      const S ep = w - al * clampv(w * ia, lo[s], hi[s]);
      eout[e1x + lane + 64 * s] = ep;
      const S re = eb[s] - ep;
      const S rz = zo[s] - zp[s];
      st.row((double)re, (double)rz, (double)ia);
      st.col((double)rz, (double)(re + gc[s]), (double)ia);
    }
  }
  // group 1: y in K* = R^{2n}_+ x R and the row s^i - b'y
  double bw = lane < n ? (double)(pk * (S(2) * ypv - yv)) : 0.0;
  double bry = lane < n ? (double)(pk * (yv - ypv)) : 0.0;
  for (int k = lane + 64; k < n; k += 64) {  // more than 64 children
    const S pq = P.p[fc + k];
    const S y1 = z[zb + k], y1p = zout[zb + k];
    bw += (double)(pq * (S(2) * y1p - y1));
    bry += (double)(pq * (y1 - y1p));
  }
  const S bW = (S)team_sum<64>(bw) + (S(2) * y3p - y3);
  const S bR = (S)team_sum<64>(bry) + (y3 - y3p);
  const S ws = es + al * ((S(2) * sip - si) - bW);
  const S es_new = ws < S(0) ? ws : S(0);
  const S res_ = es - es_new;
  auto yrow = [&](int k, S y, S yp, S e, S pq) {
    const S w = e + al * (S(2) * yp - y);
    const S ep = (k < 2 * n) ? (w < S(0) ? w : S(0)) : S(0);
    eout[e1 + k] = ep;
    const S re = e - ep;
    const S ry = y - yp;
    st.row((double)re, (double)ry, (double)ia);
    const S bk = (k < n) ? pq : ((k == 2 * n) ? S(1) : S(0));
    st.col((double)ry, (double)(re - bk * res_), (double)ia);
  };
  if (lane < ny) yrow(lane, yv, ypv, eyv, pk);
  for (int k = lane + 64; k < ny; k += 64) yrow(k, z[zb + k], zout[zb + k], eta[e1 + k], k < n ? P.p[fc + k] : S(0));
  if (lane == 0) {
    eout[e1 + 2 * n + 1] = es_new;
    const S rsi = si - sip;
    st.row((double)res_, (double)(rsi - bR), (double)ia);
    st.col((double)rsi, (double)res_, (double)ia);
  }
}

// Leaf j: group 3 (box on x^j, (Q_N^{1/2} x^j, s/2, s/2) in the SOC) and
// the columns x^j, s^j; one batch of loads as in flat_family.
template <typename S>
__device__ __forceinline__ void flat_leaf(const DevProb<S>& P, const Off<S>& O, const long long* __restrict__ spos,
                                          const S* __restrict__ z, const S* __restrict__ eta,
                                          const S* __restrict__ zout, S* __restrict__ eout, int j, int lane,
                                          StatAcc& st) {
  const int nx = P.nx;
  const S al = P.alpha;
  const S ia = S(1) / al;
  const long long e3 = O.e3(j), xj = O.x(j);
  const long long sp = spos[j];
  const bool on = lane < nx;
  const int kk = on ? lane : 0;
  const S xc = zout[xj + kk], xin = z[xj + kk];
  const S ebx = eta[e3 + kk], eq = eta[e3 + nx + kk];
  const S lo = P.xlo[(size_t)j * nx + kk], hi = P.xhi[(size_t)j * nx + kk];
  const S sqn = P.sqN[(size_t)j * nx + kk];
  const S sv = z[sp], svp = zout[sp];
  const S ea = eta[e3 + 2 * nx], ebb = eta[e3 + 2 * nx + 1];
  const S w = ebx + al * (S(2) * xc - xin);
  const S pb = w - al * clampv(w * ia, lo, hi);
  const S rex = ebx - pb;
  S wq[2] = {on ? eq + al * sqn * (S(2) * xc - xin) : S(0), S(0)}, oq[2] = {S(0), S(0)};
  const S wsa = ea + al * S(0.5) * (S(2) * svp - sv);
  const S wsb = ebb + al * S(0.5) * (S(2) * svp - sv);
  S osa, osb;
  soc_prox<S, 64, 64>(wq, oq, nx, wsa, wsb, osa, osb, al, lane);
  if (on) {
    eout[e3 + lane] = pb;
    st.row((double)rex, (double)(xin - xc), (double)ia);
    eout[e3 + nx + lane] = oq[0];
    const S req = eq - oq[0];
    st.row((double)req, (double)(sqn * (xin - xc)), (double)ia);
    st.col((double)(xin - xc), (double)(rex + sqn * req), (double)ia);
  }
  if (lane == 0) {
    const S rs = sv - svp;
    eout[e3 + 2 * nx] = osa;
    eout[e3 + 2 * nx + 1] = osb;
    const S rea = ea - osa, reb = ebb - osb;
    st.row((double)rea, 0.5 * (double)rs, (double)ia);
    st.row((double)reb, 0.5 * (double)rs, (double)ia);
    st.col((double)rs, 0.5 * ((double)rea + (double)reb), (double)ia);
  }
}

// Four wavefronts per SIMD: FP32 needs 122 VGPRs; FP64 (133 with the late
// loads) is held to 128 at 12 bytes of scratch, measured faster than three.
template <typename S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_post_flat(DevProb<S> P, const long long* __restrict__ spos,
                                                   const S* __restrict__ z, const S* __restrict__ eta,
                                                   const S* __restrict__ zout, S* __restrict__ eout,
                                                   double* __restrict__ partials) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Off<S> O(P);
  StatAcc st;
  const int stride = gridDim.x * 4;
  for (int u = blockIdx.x * 4 + wave; u < P.nn; u += stride) {
    if (u < P.nl) flat_family<S>(P, O, spos, z, eta, zout, eout, u, lane, st);
    else flat_leaf<S>(P, O, spos, z, eta, zout, eout, u, lane, st);
  }
  // wavefront, then the four wavefronts in order
  double v[kStats] = {st.rz2, st.re2, st.cross, st.xip, st.xid};
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    v[0] += __shfl_xor(v[0], m, 64);
    v[1] += __shfl_xor(v[1], m, 64);
    v[2] += __shfl_xor(v[2], m, 64);
    v[3] = fmax(v[3], __shfl_xor(v[3], m, 64));
    v[4] = fmax(v[4], __shfl_xor(v[4], m, 64));
  }
  __shared__ double red[4][kStats];
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kStats; ++k) red[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < kStats) {
    const int k = threadIdx.x;
    double a = red[0][k];
    for (int w = 1; w < 4; ++w) a = (k < 3) ? a + red[w][k] : fmax(a, red[w][k]);
    partials[(size_t)blockIdx.x * kStats + k] = a;
  }
}

// Blocks of the flat post-pass: the resident blocks per compute unit (one
// wavefront per SIMD each; as many as the registers allow) times the
// compute units, each wavefront looping over units; at most one statistics
// record per nonleaf node plus one (the partials' size).
int flat_post_blocks(const Problem& P) {
  const int units = (P.tree->nn + 3) / 4;
  return std::max(1, std::min({units, P.tree->nl + 1, P.flat_bpc * P.ncu}));
}
template <typename S>
int flat_post_occupancy() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_post_flat<S>, 256, 0) != hipSuccess || nb < 1) nb = 1;
  return nb;
}
template int flat_post_occupancy<double>();
template int flat_post_occupancy<float>();

// ---------------------------------------------------------------- team sweeps
// One team of T lanes per family; one launch per stage.
template <typename S, int T>
__global__ void __launch_bounds__(256) k_bwd(DevProb<S> P, const S* __restrict__ xbar,
                                             const S* __restrict__ ubar, S* __restrict__ qbuf,
                                             S* __restrict__ dbuf, int first, int count, int VM) {
  extern __shared__ unsigned char smem_raw[];
  S* smem = reinterpret_cast<S*>(smem_raw);
  const int lane = threadIdx.x % T;
  const int team = threadIdx.x / T;
  const int f = blockIdx.x * (blockDim.x / T) + team;
  if (f >= count) return;  // whole teams only; no block barrier below
  fam_bwd_team<S, T>(P, xbar, ubar, qbuf, dbuf, first + f, lane, smem + (size_t)team * 3 * VM, VM);
}

template <typename S, int T>
__global__ void __launch_bounds__(256) k_fwd(DevProb<S> P, S* __restrict__ zout,
                                             const S* __restrict__ dbuf,
                                             const double* __restrict__ x0, int first, int count,
                                             int VM) {
  extern __shared__ unsigned char smem_raw[];
  S* smem = reinterpret_cast<S*>(smem_raw);
  const int lane = threadIdx.x % T;
  const int team = threadIdx.x / T;
  const int f = blockIdx.x * (blockDim.x / T) + team;
  if (f >= count) return;
  fam_fwd_team<S, T>(P, zout, dbuf, x0, first + f, lane, smem + (size_t)team * 2 * VM, VM);
}

// ---------------------------------------------------------------- workgroup sweeps
// One 256-thread workgroup (4 wavefronts) per family. Every mat-vec is split
// over the input index across the 4 wavefronts; inside a wavefront the lanes
// form G = floor(64 / nout) groups (G = 1 when nout > 32), each group reading
// one input row, so one load instruction covers G consecutive rows of the
// input-major matrix. All matrix loads of a family are issued into registers
// before the first barrier; partial sums are combined in LDS in a fixed order.
constexpr int kWG = 256;
constexpr int kKJ = 16;         // max loads per lane per mat-vec: ceil(64 / 4)
constexpr int kMaxLevels = 64;  // stages a subtree-owning workgroup walks

template <typename S>
struct MvRegs {
  S m[kKJ];
};

struct MvGeom {
  int G, o, kg, stride;
  bool act;
  __device__ __forceinline__ MvGeom(int nout) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    G = nout > 32 ? 1 : 64 / nout;
    const int g = lane / nout;
    o = lane - g * nout;
    act = g < G;
    kg = w * G + g;
    stride = 4 * G;
  }
};

template <typename S>
__device__ __forceinline__ void mv_load(MvRegs<S>& r, const S* __restrict__ M, int nin, int nout) {
  const MvGeom g(nout);
#pragma unroll
  for (int j = 0; j < kKJ; ++j) {
    const int k = g.kg + g.stride * j;
    r.m[j] = (g.act && k < nin) ? M[(size_t)k * nout + g.o] : S(0);
  }
}

// partial sum of this thread, written to red[kg * nout + o]
template <typename S>
__device__ __forceinline__ void mv_partial(const MvRegs<S>& r, const S* v, int nin, int nout, S* red) {
  const MvGeom g(nout);
  if (!g.act) return;
  S acc = 0;
#pragma unroll
  for (int j = 0; j < kKJ; ++j) {
    const int k = g.kg + g.stride * j;
    if (k < nin) acc += r.m[j] * v[k];
  }
  red[g.kg * nout + g.o] = acc;
}

// y[o] = sum over the 4 G partials of output o (call with o = threadIdx.x < nout)
template <typename S>
__device__ __forceinline__ S mv_sum(const S* red, int nout, int o) {
  const int G = nout > 32 ? 1 : 64 / nout;
  S s = 0;
  for (int q = 0; q < 4 * G; ++q) s += red[q * nout + o];
  return s;
}

// Prefetch of up to 8 byte ranges into L2: thread t reads one 32-bit word of
// lines t, t + 256, ... of the concatenated ranges (128-byte lines), so a later
// family's loads hit L2. The words are folded into acc, which the caller
// keeps alive.
struct Ranges {
  const char* p[8] = {};
  int lines[8] = {};
  int n = 0;
  __device__ __forceinline__ void add(const void* ptr, size_t bytes) {
    p[n] = static_cast<const char*>(ptr);
    lines[n] = (int)((bytes + 127) / 128);
    ++n;
  }
};

__device__ __forceinline__ void touch(const Ranges& R, unsigned& acc) {
  int total = 0;
#pragma unroll
  for (int r = 0; r < 8; ++r)
    if (r < R.n) total += R.lines[r];
  for (int l = threadIdx.x; l < total; l += kWG) {
    int off = l;
#pragma unroll
    for (int r = 0; r < 8; ++r) {  // fixed trip count keeps R in registers
      if (r < R.n) {
        if (off >= 0 && off < R.lines[r]) acc ^= *reinterpret_cast<const unsigned*>(R.p[r] + (size_t)off * 128);
        off -= R.lines[r];
      }
    }
  }
}

// Backward data of family j (matrices, xbar, ubar) pulled into L2.
template <typename S>
__device__ __forceinline__ void prefetch_bwd(const DevProb<S>& P, const S* xbar, const S* ubar,
                                             const S* qbuf, int j, unsigned& acc) {
  const int nx = P.nx, nu = P.nu, fc = P.fc[j], n = P.nch[j];
  Ranges R;
  R.add(P.AbR + (size_t)fc * nx * nx, sizeof(S) * n * nx * nx);
  R.add(P.BR + (size_t)fc * nx * nu, sizeof(S) * n * nx * nu);
  R.add(P.Rinv + (size_t)j * nu * nu, sizeof(S) * nu * nu);
  R.add(P.KR + (size_t)j * nu * nx, sizeof(S) * nu * nx);
  R.add(P.WC + (size_t)j * nu * nx, sizeof(S) * nu * nx);
  R.add(xbar + (size_t)j * nx, sizeof(S) * nx);
  R.add(ubar + (size_t)j * nu, sizeof(S) * nu);
  touch(R, acc);
  (void)qbuf;
}

// Forward data of family j (matrices and d) pulled into L2.
template <typename S>
__device__ __forceinline__ void prefetch_fwd(const DevProb<S>& P, const S* dbuf, int j, unsigned& acc) {
  const int nx = P.nx, nu = P.nu, fc = P.fc[j], n = P.nch[j];
  Ranges R;
  R.add(P.AbC + (size_t)fc * nx * nx, sizeof(S) * n * nx * nx);
  R.add(P.BC + (size_t)fc * nu * nx, sizeof(S) * n * nu * nx);
  R.add(P.KC + (size_t)j * nx * nu, sizeof(S) * nx * nu);
  R.add(dbuf + (size_t)j * nu, sizeof(S) * nu);
  touch(R, acc);
}

// Backward step of family i by the whole workgroup (called uniformly).
// `next` (or -1) is the family this workgroup handles afterwards; its data is
// prefetched into L2 once this family's own loads are in flight.
template <typename S>
__device__ void bwd_family_wg(const DevProb<S>& P, const S* __restrict__ xbar,
                              const S* __restrict__ ubar, S* __restrict__ qbuf,
                              S* __restrict__ dbuf, int i, int next, unsigned& pf) {
  __shared__ S vq[kMaxDim], vg[kMaxDim], vd[kMaxDim], sA[kMaxDim], hh[kMaxDim], xbs[kMaxDim],
      ubs[kMaxDim];
  __shared__ S red1[kWG], red2[kWG];
  const int t = threadIdx.x;
  const int nx = P.nx, nu = P.nu;
  const int fc = P.fc[i], n = P.nch[i];
  MvRegs<S> mR, mK, mW, mA, mB;
  mv_load(mA, P.AbR + (size_t)fc * nx * nx, nx, nx);  // first child, prefetched
  mv_load(mB, P.BR + (size_t)fc * nx * nu, nx, nu);
  mv_load(mR, P.Rinv + (size_t)i * nu * nu, nu, nu);
  mv_load(mK, P.KR + (size_t)i * nu * nx, nu, nx);
  mv_load(mW, P.WC + (size_t)i * nu * nx, nu, nx);
  if (t < nx) xbs[t] = xbar[(size_t)i * nx + t];
  if (t < nu) ubs[t] = ubar[(size_t)i * nu + t];
  if (t < 64) {
    sA[t] = 0;
    hh[t] = 0;
  }
  S qnext = (t < nx) ? qbuf[(size_t)fc * nx + t] : S(0);
  for (int k = 0; k < n; ++k) {
    const int ch = fc + k;
    if (t < nx) vq[t] = qnext;
    __syncthreads();
    // this family's own loads have all been consumed: the next family's data
    // now streams into L2 while this one computes
    if (k == 0 && next >= 0) prefetch_bwd(P, xbar, ubar, qbuf, next, pf);
    mv_partial(mA, vq, nx, nx, red1);
    mv_partial(mB, vq, nx, nu, red2);
    if (k + 1 < n) {  // prefetch the next child's matrices and q
      mv_load(mA, P.AbR + (size_t)(ch + 1) * nx * nx, nx, nx);
      mv_load(mB, P.BR + (size_t)(ch + 1) * nx * nu, nx, nu);
      if (t < nx) qnext = qbuf[(size_t)(ch + 1) * nx + t];
    }
    __syncthreads();
    if (t < nx) sA[t] += mv_sum(red1, nx, t);
    if (t < nu) hh[t] += mv_sum(red2, nu, t);
    __syncthreads();
  }
  // d = R~^{-1}(ubar - h)
  if (t < nu) vg[t] = ubs[t] - hh[t];
  __syncthreads();
  mv_partial(mR, vg, nu, nu, red1);
  __syncthreads();
  if (t < nu) {
    const S dv = mv_sum(red1, nu, t);
    vd[t] = dv;
    dbuf[(size_t)i * nu + t] = dv;
    vg[t] = dv - ubs[t];
  }
  __syncthreads();
  // q = K'(d - ubar) + W d - xbar + sum Abar' q
  mv_partial(mK, vg, nu, nx, red1);
  mv_partial(mW, vd, nu, nx, red2);
  __syncthreads();
  if (t < nx) qbuf[(size_t)i * nx + t] = mv_sum(red1, nx, t) + mv_sum(red2, nx, t) - xbs[t] + sA[t];
  __syncthreads();  // LDS reuse by the next family of this workgroup
}

template <typename S>
__global__ void __launch_bounds__(kWG) k_bwd_wg(DevProb<S> P, const S* __restrict__ xbar,
                                                const S* __restrict__ ubar, S* __restrict__ qbuf,
                                                S* __restrict__ dbuf, int first) {
  unsigned pf = 0;
  bwd_family_wg<S>(P, xbar, ubar, qbuf, dbuf, first + blockIdx.x, -1, pf);
}

// Descendant ranges of subtree root r (stage tc) down to the last nonleaf
// stage: nodes of a subtree at one stage are contiguous (breadth-first order
// with contiguous children). lo[l], hi[l] (LDS) belong to stage tc + l;
// thread 0 fills them, the caller's barrier publishes them.
template <typename S>
__device__ __forceinline__ int subtree_levels(const DevProb<S>& P, int r, int tc, int* lo, int* hi) {
  const int levels = P.N - tc;  // nonleaf stages tc .. N-1
  if (threadIdx.x == 0) {
    lo[0] = r;
    hi[0] = r + 1;
    for (int l = 1; l < levels; ++l) {
      lo[l] = P.fc[lo[l - 1]];
      hi[l] = P.fc[hi[l - 1] - 1] + P.nch[hi[l - 1] - 1];
    }
  }
  __syncthreads();
  return levels;
}

// Backward sweep over whole subtrees rooted at stage tc: one workgroup per
// subtree walks its stages bottom-up, so the stages below tc need no launch
// of their own.
template <typename S>
__global__ void __launch_bounds__(kWG) k_bwd_tail_wg(DevProb<S> P, const S* __restrict__ xbar,
                                                     const S* __restrict__ ubar, S* __restrict__ qbuf,
                                                     S* __restrict__ dbuf, int tc, int root_first,
                                                     int nroots) {
  __shared__ int lo[kMaxLevels], hi[kMaxLevels];
  unsigned pf = 0;
  for (int r = blockIdx.x; r < nroots; r += gridDim.x) {
    const int levels = subtree_levels(P, root_first + r, tc, lo, hi);
    for (int l = levels - 1; l >= 0; --l) {
      const int a = lo[l], b = hi[l];
      for (int i = a; i < b; ++i) {
        const int next = (i + 1 < b) ? i + 1 : (l > 0 ? lo[l - 1] : -1);
        bwd_family_wg<S>(P, xbar, ubar, qbuf, dbuf, i, next, pf);
      }
    }
    __syncthreads();  // before the ranges are overwritten
  }
  if (P.nn < 0) qbuf[0] = S(pf);  // never true: keeps the prefetch loads alive
}

// Forward step of family i by the whole workgroup.
template <typename S>
__device__ void fwd_family_wg(const DevProb<S>& P, S* __restrict__ zout, const S* __restrict__ dbuf,
                              const double* __restrict__ x0, int i, int next, unsigned& pf) {
  __shared__ S vx[kMaxDim], vd[kMaxDim];
  __shared__ S red1[kWG], red2[kWG];
  const int t = threadIdx.x;
  const Off<S> O(P);
  const int nx = P.nx, nu = P.nu;
  const int fc = P.fc[i], n = P.nch[i];
  const long long ui = O.u(i);
  MvRegs<S> mK, mA, mB;
  mv_load(mA, P.AbC + (size_t)fc * nx * nx, nx, nx);  // first child, prefetched
  mv_load(mB, P.BC + (size_t)fc * nu * nx, nu, nx);
  mv_load(mK, P.KC + (size_t)i * nx * nu, nx, nu);
  if (t < nx) {
    S xv;
    if (i == 0) {
      xv = (S)x0[t];
      zout[1 + t] = xv;
    } else {
      xv = zout[O.x(i) + t];
    }
    vx[t] = xv;
  }
  if (t < nu) vd[t] = dbuf[(size_t)i * nu + t];
  __syncthreads();
  mv_partial(mK, vx, nx, nu, red1);
  if (next >= 0) prefetch_fwd(P, dbuf, next, pf);  // after this family's loads were consumed
  __syncthreads();
  if (t < nu) zout[ui + t] = mv_sum(red1, nu, t) + vd[t];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const int ch = fc + k;
    mv_partial(mA, vx, nx, nx, red1);
    mv_partial(mB, vd, nu, nx, red2);
    if (k + 1 < n) {  // prefetch the next child's matrices
      mv_load(mA, P.AbC + (size_t)(ch + 1) * nx * nx, nx, nx);
      mv_load(mB, P.BC + (size_t)(ch + 1) * nu * nx, nu, nx);
    }
    __syncthreads();
    if (t < nx) zout[O.x(ch) + t] = mv_sum(red1, nx, t) + mv_sum(red2, nx, t);
    __syncthreads();
  }
}

template <typename S>
__global__ void __launch_bounds__(kWG) k_fwd_wg(DevProb<S> P, S* __restrict__ zout,
                                                const S* __restrict__ dbuf,
                                                const double* __restrict__ x0, int first) {
  unsigned pf = 0;
  fwd_family_wg<S>(P, zout, dbuf, x0, first + blockIdx.x, -1, pf);
}

// Forward sweep over whole subtrees rooted at stage tc (top-down per subtree).
template <typename S>
__global__ void __launch_bounds__(kWG) k_fwd_tail_wg(DevProb<S> P, S* __restrict__ zout,
                                                     const S* __restrict__ dbuf,
                                                     const double* __restrict__ x0, int tc,
                                                     int root_first, int nroots) {
  __shared__ int lo[kMaxLevels], hi[kMaxLevels];
  unsigned pf = 0;
  for (int r = blockIdx.x; r < nroots; r += gridDim.x) {
    const int levels = subtree_levels(P, root_first + r, tc, lo, hi);
    for (int l = 0; l < levels; ++l) {
      const int a = lo[l], b = hi[l];
      for (int i = a; i < b; ++i) {
        const int next = (i + 1 < b) ? i + 1 : (l + 1 < levels ? lo[l + 1] : -1);
        fwd_family_wg<S>(P, zout, dbuf, x0, i, next, pf);
      }
    }
    __syncthreads();  // before the ranges are overwritten
  }
  if (P.nn < 0) zout[0] = S(pf);  // never true: keeps the prefetch loads alive
}

// Hands stats[0..8) to the host mailbox: the values, then the epoch with
// system-scope release (one thread).
__device__ void publish_stats(const double* vals, Publish pub) {
  for (int s = 0; s < 8; ++s) pub.mb->v[s] = vals[s];
  __hip_atomic_store(&pub.mb->flag, pub.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Sums the per-block statistics into {xi_p, xi_d, omega^2, rz2, re2, cross};
// NaN when the error word of the dataflow sweeps is set (a bounded wait gave
// up); then, when pub.mb is set, publishes out[0..8) to the host.
__global__ void __launch_bounds__(256) k_reduce_stats(const double* __restrict__ partials, int nblk, double alpha,
                               double* __restrict__ out, const unsigned* __restrict__ err, Publish pub) {
  // per thread over records t, t + 256, ...; then wavefront shuffles and
  // the four wavefronts in order (one barrier)
  double a[kStats] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    const double* p = partials + (size_t)b * kStats;
    a[0] += p[0];
    a[1] += p[1];
    a[2] += p[2];
    a[3] = fmax(a[3], p[3]);
    a[4] = fmax(a[4], p[4]);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    a[0] += __shfl_xor(a[0], m, 64);
    a[1] += __shfl_xor(a[1], m, 64);
    a[2] += __shfl_xor(a[2], m, 64);
    a[3] = fmax(a[3], __shfl_xor(a[3], m, 64));
    a[4] = fmax(a[4], __shfl_xor(a[4], m, 64));
  }
  __shared__ double red[4][kStats];
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < kStats; ++k) red[threadIdx.x >> 6][k] = a[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[kStats];
#pragma unroll
    for (int k = 0; k < kStats; ++k) t[k] = red[0][k];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      t[0] += red[w][0];
      t[1] += red[w][1];
      t[2] += red[w][2];
      t[3] = fmax(t[3], red[w][3]);
      t[4] = fmax(t[4], red[w][4]);
    }
    double r[8];
    r[0] = t[3];
    r[1] = t[4];
    r[2] = t[0] + t[1] - 2.0 * alpha * t[2];
    r[3] = t[0];
    r[4] = t[1];
    r[5] = t[2];
    if (err && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)
      for (int k = 0; k < 6; ++k) r[k] = __builtin_nan("");
    for (int k = 0; k < 6; ++k) out[k] = r[k];
    if (pub.mb) {
      r[6] = out[6];
      r[7] = out[7];
      publish_stats(r, pub);
    }
  }
}

// ---------------------------------------------------------------- launch T
template <typename S>
static const DevProb<S>& dev_of(const Problem& P);
template <>
const DevProb<double>& dev_of<double>(const Problem& P) { return P.dp64; }
template <>
const DevProb<float>& dev_of<float>(const Problem& P) { return P.dp32; }

template <typename S, int T>
static void launch_sweeps_team(const Problem& P, const DevProb<S>& D, S* zout, const double* x0,
                               const S* xbar, const S* ubar, S* q, S* d, hipStream_t st) {
  const Tree& tr = *P.tree;
  const int tpb = 256 / T;
  const int VM = (std::max(P.nx, P.nu) + 3) & ~3;
  for (int t = tr.N - 1; t >= 0; --t) {
    const int first = tr.stage_off[t];
    const int count = tr.stage_off[t + 1] - first;
    hipLaunchKernelGGL((k_bwd<S, T>), dim3((count + tpb - 1) / tpb), dim3(256),
                       (size_t)tpb * 3 * VM * sizeof(S), st, D, xbar, ubar, q, d, first, count, VM);
  }
  for (int t = 0; t < tr.N; ++t) {
    const int first = tr.stage_off[t];
    const int count = tr.stage_off[t + 1] - first;
    hipLaunchKernelGGL((k_fwd<S, T>), dim3((count + tpb - 1) / tpb), dim3(256),
                       (size_t)tpb * 2 * VM * sizeof(S), st, D, zout, d, x0, first, count, VM);
  }
}

template <typename S>
static void launch_sweeps_wg(const Problem& P, const DevProb<S>& D, S* zout, const double* x0,
                             const S* xbar, const S* ubar, S* q, S* d, hipStream_t st, int cut) {
  const Tree& tr = *P.tree;
  const int tc = cut;  // stages >= tc are walked by subtree-owning workgroups
  if (tc < tr.N) {
    const int roots = tr.stage_off[tc + 1] - tr.stage_off[tc];
    hipLaunchKernelGGL(k_bwd_tail_wg<S>, dim3(roots), dim3(kWG), 0, st, D, xbar, ubar, q, d, tc,
                       tr.stage_off[tc], roots);
  }
  for (int t = std::min(tc, tr.N) - 1; t >= 0; --t) {
    const int first = tr.stage_off[t];
    const int count = tr.stage_off[t + 1] - first;
    hipLaunchKernelGGL(k_bwd_wg<S>, dim3(count), dim3(kWG), 0, st, D, xbar, ubar, q, d, first);
  }
  for (int t = 0; t < std::min(tc, tr.N); ++t) {
    const int first = tr.stage_off[t];
    const int count = tr.stage_off[t + 1] - first;
    hipLaunchKernelGGL(k_fwd_wg<S>, dim3(count), dim3(kWG), 0, st, D, zout, d, x0, first);
  }
  if (tc < tr.N) {
    const int roots = tr.stage_off[tc + 1] - tr.stage_off[tc];
    hipLaunchKernelGGL(k_fwd_tail_wg<S>, dim3(roots), dim3(kWG), 0, st, D, zout, d, x0, tc,
                       tr.stage_off[tc], roots);
  }
}

template <typename S, int T>
static void launch_pre(const Problem& P, const DevProb<S>& D, const S* z, const S* eta, S* zout,
                       S* xbar, S* ubar, S* q, hipStream_t st) {
  const int tpb = 256 / T;
  hipLaunchKernelGGL((k_pre<S, T>), dim3((P.tree->nl + tpb - 1) / tpb), dim3(256), 0, st, D, z, eta,
                     zout, xbar, ubar, q);
}

static int pp_index(int T) { return T == 8 ? 0 : T == 16 ? 1 : T == 32 ? 2 : 3; }

template <typename S, int T>
static void launch_post(const Problem& P, const DevProb<S>& D, const S* z, const S* eta,
                        const S* zout, S* eout, double* partials, hipStream_t st) {
  if (P.post_flat) {
    hipLaunchKernelGGL(k_post_flat<S>, dim3(flat_post_blocks(P)), dim3(256), 0, st, D, P.d_spos, z, eta, zout,
                       eout, partials);
    return;
  }
  const int tpb = 256 / T;
  const int VM = (std::max(P.nx, P.nu) + 3) & ~3;
  const int k = pp_index(T);
  if (P.pblk_n[k] > 0) {
    const size_t lds = ((size_t)tpb * 3 * VM + (size_t)P.pblk_cap[k] * (P.nx + P.nu)) * sizeof(S);
    hipLaunchKernelGGL((k_post_nodes<S, T>), dim3(P.pblk_n[k]), dim3(256), lds, st, D, P.d_pblk[k], z, eta, zout,
                       eout, VM, partials);
    return;
  }
  hipLaunchKernelGGL((k_post<S, T>), dim3((P.tree->nl + tpb - 1) / tpb), dim3(256),
                     (size_t)tpb * 3 * VM * sizeof(S), st, D, z, eta, zout, eout, VM, partials);
}

// Number of statistic records written by the post-pass.
int post_blocks(const Problem& P) {
  if (P.general) return gen_post_blocks(P);
  if (P.post_flat) return flat_post_blocks(P);
  const int k = pp_index(P.team_pp);
  if (P.pblk_n[k] > 0) return P.pblk_n[k];
  const int tpb = 256 / P.team_pp;
  return (P.tree->nl + tpb - 1) / tpb;
}

template <typename S>
hipError_t launch_T(const Problem& P, const S* v, S* Tv, const double* x0, S* q, S* d, S* xbar,
                    S* ubar, double* partials, double* stats_dev, hipStream_t st,
                    const S* eta_zero, bool dual, Publish pub, SweepMap map) {
  const DevProb<S>& D = dev_of<S>(P);
  const int team = map.team > 0 ? map.team : P.team;
  const int cut = map.team > 0 ? map.cut : P.cut;
  const S* z = v;
  const S* eta = dual ? v + P.nz : eta_zero;
  S* zout = Tv;
  S* eout = dual ? Tv + P.nz : nullptr;
  auto mark = [&](int k) {
    if (P.prof) (void)hipEventRecord(P.prof[k], st);
  };
  mark(0);
  if (P.general) {
    const hipError_t e = launch_gen_pre<S>(P, z, eta, zout, xbar, ubar, q, st);
    if (e != hipSuccess) return e;
  } else {
    switch (P.team_pp) {
      case 8: launch_pre<S, 8>(P, D, z, eta, zout, xbar, ubar, q, st); break;
      case 16: launch_pre<S, 16>(P, D, z, eta, zout, xbar, ubar, q, st); break;
      case 32: launch_pre<S, 32>(P, D, z, eta, zout, xbar, ubar, q, st); break;
      default: launch_pre<S, 64>(P, D, z, eta, zout, xbar, ubar, q, st); break;
    }
  }
  mark(1);
  switch (team) {
    case kTeamFlow: {
      const hipError_t e = launch_sweeps_flow<S>(P, D, zout, x0, xbar, ubar, q, d, st);
      if (e != hipSuccess) return e;
      break;
    }
    case 8: launch_sweeps_team<S, 8>(P, D, zout, x0, xbar, ubar, q, d, st); break;
    case 16: launch_sweeps_team<S, 16>(P, D, zout, x0, xbar, ubar, q, d, st); break;
    case 32: launch_sweeps_team<S, 32>(P, D, zout, x0, xbar, ubar, q, d, st); break;
    case 64: launch_sweeps_team<S, 64>(P, D, zout, x0, xbar, ubar, q, d, st); break;
    default: launch_sweeps_wg<S>(P, D, zout, x0, xbar, ubar, q, d, st, cut); break;
  }
  mark(2);
  if (dual) {
    if (P.general) {
      const hipError_t e = launch_gen_post<S>(P, z, eta, zout, eout, partials, st);
      if (e != hipSuccess) return e;
    } else {
      switch (P.team_pp) {
        case 8: launch_post<S, 8>(P, D, z, eta, zout, eout, partials, st); break;
        case 16: launch_post<S, 16>(P, D, z, eta, zout, eout, partials, st); break;
        case 32: launch_post<S, 32>(P, D, z, eta, zout, eout, partials, st); break;
        default: launch_post<S, 64>(P, D, z, eta, zout, eout, partials, st); break;
      }
    }
    mark(3);
    hipLaunchKernelGGL(k_reduce_stats, dim3(1), dim3(256), 0, st, partials, post_blocks(P),
                       (double)D.alpha, stats_dev, team == kTeamFlow ? (const unsigned*)P.flow.err : nullptr,
                       pub);
  }
  mark(4);
  return hipGetLastError();
}
template hipError_t launch_T<double>(const Problem&, const double*, double*, const double*, double*,
                                     double*, double*, double*, double*, double*, hipStream_t,
                                     const double*, bool, Publish, SweepMap);
template hipError_t launch_T<float>(const Problem&, const float*, float*, const double*, float*,
                                    float*, float*, float*, double*, double*, hipStream_t, const float*,
                                    bool, Publish, SweepMap);

// ---------------------------------------------------------------- L and L*
// One wavefront per family (grid-stride over families, four per block):
// the family's rows of L (group 1 of i, group 2 of each child, group 3 of
// leaf children) and its columns of L* (y^i, s^i, x^i, u^i, tau^c, and x^c,
// s^c of leaf children), lanes over components. Every entry is written by
// exactly one family; sums over children run in child order.
template <typename S>
__global__ void __launch_bounds__(256) k_apply_L(DevProb<S> P, const S* __restrict__ z, S* __restrict__ eta,
                                                 long long is) {
  z += (size_t)blockIdx.y * is;  // instance blockIdx.y of a batch (stride is)
  eta += (size_t)blockIdx.y * is;
  const int lane = threadIdx.x & 63;
  const Off<S> O(P);
  const int nx = P.nx, nu = P.nu, K = nx + nu;
  for (int i = blockIdx.x * 4 + (int)(threadIdx.x >> 6); i < P.nl; i += gridDim.x * 4) {
    const int fc = P.fc[i], n = P.nch[i];
    const long long zb = O.z2(i), e1 = O.e1(i), e1x = e1 + 2LL * n + 2;
    double by = 0;
    for (int k = lane; k < 2 * n + 1; k += 64) {
      const S y = z[zb + k];
      eta[e1 + k] = y;
      if (k < n) by += (double)(P.p[fc + k] * y);
    }
    by = team_sum<64>(by) + (double)z[zb + 2 * n];
    if (lane == 0) eta[e1 + 2 * n + 1] = z[O.s(i)] - (S)by;
    for (int k = lane; k < K; k += 64) eta[e1x + k] = k < nx ? z[O.x(i) + k] : z[O.u(i) + (k - nx)];
    for (int c = fc; c < fc + n; ++c) {
      const long long e2 = O.e2(c);
      for (int k = lane; k < K; k += 64)
        eta[e2 + k] = k < nx ? P.sq[(size_t)c * nx + k] * z[O.x(i) + k]
                             : P.sr[(size_t)c * nu + (k - nx)] * z[O.u(i) + (k - nx)];
      if (lane == 0) {
        const S th = S(0.5) * z[zb + 2LL * n + 1 + (c - fc)];
        eta[e2 + K] = th;
        eta[e2 + K + 1] = th;
      }
      if (c >= P.nl) {
        const long long e3 = O.e3(c);
        for (int o = lane; o < nx; o += 64) {
          const S xc = z[O.x(c) + o];
          eta[e3 + o] = xc;
          eta[e3 + nx + o] = P.sqN[(size_t)c * nx + o] * xc;
        }
        if (lane == 0) {
          const S sh = S(0.5) * z[zb + 3LL * n + 1 + (c - fc)];
          eta[e3 + 2 * nx] = sh;
          eta[e3 + 2 * nx + 1] = sh;
        }
      }
    }
  }
}

template <typename S>
__global__ void __launch_bounds__(256) k_apply_Lt(DevProb<S> P, const S* __restrict__ eta, S* __restrict__ z,
                                                  long long is) {
  eta += (size_t)blockIdx.y * is;  // instance blockIdx.y of a batch (stride is)
  z += (size_t)blockIdx.y * is;
  const int lane = threadIdx.x & 63;
  const Off<S> O(P);
  const int nx = P.nx, nu = P.nu, K = nx + nu;
  for (int i = blockIdx.x * 4 + (int)(threadIdx.x >> 6); i < P.nl; i += gridDim.x * 4) {
    const int fc = P.fc[i], n = P.nch[i];
    const long long zb = O.z2(i), e1 = O.e1(i), e1x = e1 + 2LL * n + 2;
    const S es = eta[e1 + 2 * n + 1];
    for (int k = lane; k < 2 * n + 1; k += 64) {
      const S bk = (k < n) ? P.p[fc + k] : ((k == 2 * n) ? S(1) : S(0));
      z[zb + k] = eta[e1 + k] - bk * es;
    }
    if (lane == 0) z[O.s(i)] = es;
    for (int k = lane; k < K; k += 64) {
      S acc = eta[e1x + k];
      if (k < nx) {
        for (int c = fc; c < fc + n; ++c) acc += P.sq[(size_t)c * nx + k] * eta[O.e2(c) + k];
        z[O.x(i) + k] = acc;
      } else {
        const int o = k - nx;
        for (int c = fc; c < fc + n; ++c) acc += P.sr[(size_t)c * nu + o] * eta[O.e2(c) + k];
        z[O.u(i) + o] = acc;
      }
    }
    for (int c = fc; c < fc + n; ++c) {
      const long long e2 = O.e2(c);
      if (lane == 0) z[zb + 2LL * n + 1 + (c - fc)] = S(0.5) * (eta[e2 + K] + eta[e2 + K + 1]);
      if (c >= P.nl) {
        const long long e3 = O.e3(c);
        for (int o = lane; o < nx; o += 64)
          z[O.x(c) + o] = eta[e3 + o] + P.sqN[(size_t)c * nx + o] * eta[e3 + nx + o];
        if (lane == 0) z[zb + 3LL * n + 1 + (c - fc)] = S(0.5) * (eta[e3 + 2 * nx] + eta[e3 + 2 * nx + 1]);
      }
    }
  }
}

// Blocks of the wavefront-per-family kernels: every family its wavefront,
// up to 8192 blocks (then grid-stride).
int family_wave_blocks(int nl) { return std::max(1, std::min((nl + 3) / 4, 8192)); }

// M d of one problem: one team of T lanes per family.
template <typename S, int T>
__global__ void __launch_bounds__(256) k_apply_M(DevProb<S> P, const S* __restrict__ d, S* __restrict__ Md) {
  const int lane = threadIdx.x % T;
  const int i = blockIdx.x * (blockDim.x / T) + threadIdx.x / T;
  if (i >= P.nl) return;
  fam_apply_M<S, T>(P, d, Md, i, lane);
}

template <typename S>
hipError_t launch_M(const Problem& P, const S* d, S* Md, hipStream_t st) {
  if (P.general) return launch_gen_M<S>(P, d, Md, st);
  const DevProb<S>& D = dev_of<S>(P);
  const int T = P.team_pp, tpb = 256 / T;
  const dim3 grid((P.tree->nl + tpb - 1) / tpb);
  switch (T) {
    case 8: hipLaunchKernelGGL((k_apply_M<S, 8>), grid, dim3(256), 0, st, D, d, Md); break;
    case 16: hipLaunchKernelGGL((k_apply_M<S, 16>), grid, dim3(256), 0, st, D, d, Md); break;
    case 32: hipLaunchKernelGGL((k_apply_M<S, 32>), grid, dim3(256), 0, st, D, d, Md); break;
    default: hipLaunchKernelGGL((k_apply_M<S, 64>), grid, dim3(256), 0, st, D, d, Md); break;
  }
  return hipGetLastError();
}
template hipError_t launch_M<double>(const Problem&, const double*, double*, hipStream_t);
template hipError_t launch_M<float>(const Problem&, const float*, float*, hipStream_t);

// prox of g* (test entry point): one thread per family, serial SOC norms.
template <typename S>
__device__ void soc_prox_serial(const S* w, S* out, int len, S al) {
  // len counts the vector part; w[len], w[len+1] are the two scalars
  const S ia = S(1) / al;
  double n2 = 0;
  for (int o = 0; o < len; ++o) n2 += (double)(w[o] * ia) * (double)(w[o] * ia);
  const S va = w[len] * ia - S(0.5);
  const S t = w[len + 1] * ia + S(0.5);
  n2 += (double)va * (double)va;
  const S nrm = (S)sqrt(n2);
  S scale, pt;
  if (nrm <= t) { scale = 1; pt = t; }
  else if (nrm <= -t) { scale = 0; pt = 0; }
  else { const S cc = S(0.5) * (nrm + t); scale = cc / nrm; pt = cc; }
  for (int o = 0; o < len; ++o) out[o] = w[o] - al * scale * (w[o] * ia);
  out[len] = w[len] - al * (S(0.5) + scale * va);
  out[len + 1] = w[len + 1] - al * (S(-0.5) + pt);
}

template <typename S>
__global__ void k_prox_gstar(DevProb<S> P, const S* __restrict__ w, S* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.nl) return;
  const Off<S> O(P);
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  const S al = P.alpha, ia = S(1) / al;
  const long long e1 = O.e1(i);
  for (int k = 0; k < 2 * n; ++k) out[e1 + k] = w[e1 + k] < S(0) ? w[e1 + k] : S(0);
  out[e1 + 2 * n] = S(0);
  out[e1 + 2 * n + 1] = w[e1 + 2 * n + 1] < S(0) ? w[e1 + 2 * n + 1] : S(0);
  for (int o = 0; o < nx; ++o) {
    const S v = w[O.e1x(i) + o];
    out[O.e1x(i) + o] = v - al * clampv(v * ia, P.xlo[(size_t)i * nx + o], P.xhi[(size_t)i * nx + o]);
  }
  for (int o = 0; o < nu; ++o) {
    const S v = w[O.e1u(i) + o];
    out[O.e1u(i) + o] = v - al * clampv(v * ia, P.ulo[(size_t)i * nu + o], P.uhi[(size_t)i * nu + o]);
  }
  for (int k = 0; k < n; ++k) {
    const int c = fc + k;
    soc_prox_serial<S>(w + O.e2(c), out + O.e2(c), nx + nu, al);
    if (c >= P.nl) {
      const long long e3 = O.e3(c);
      for (int o = 0; o < nx; ++o) {
        const S v = w[e3 + o];
        out[e3 + o] = v - al * clampv(v * ia, P.xlo[(size_t)c * nx + o], P.xhi[(size_t)c * nx + o]);
      }
      soc_prox_serial<S>(w + e3 + nx, out + e3 + nx, nx, al);
    }
  }
}

template <typename S>
hipError_t launch_L(const Problem& P, const S* z, S* eta, hipStream_t st) {
  if (P.general) return launch_gen_L<S>(P, z, eta, st);
  hipLaunchKernelGGL(k_apply_L<S>, dim3(family_wave_blocks(P.tree->nl)), dim3(256), 0, st, dev_of<S>(P), z, eta,
                     0LL);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_L_batch(const Problem& P, const S* z, S* eta, long long is, int B, hipStream_t st) {
  if (P.general) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_apply_L<S>, dim3(family_wave_blocks(P.tree->nl), B), dim3(256), 0, st, dev_of<S>(P), z, eta,
                     is);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_Lt_batch(const Problem& P, const S* eta, S* z, long long is, int B, hipStream_t st) {
  if (P.general) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_apply_Lt<S>, dim3(family_wave_blocks(P.tree->nl), B), dim3(256), 0, st, dev_of<S>(P), eta, z,
                     is);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_Lt(const Problem& P, const S* eta, S* z, hipStream_t st) {
  if (P.general) return launch_gen_Lt<S>(P, eta, z, st);
  hipLaunchKernelGGL(k_apply_Lt<S>, dim3(family_wave_blocks(P.tree->nl)), dim3(256), 0, st, dev_of<S>(P), eta, z,
                     0LL);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_prox_gstar(const Problem& P, const S* w, S* out, hipStream_t st) {
  if (P.general) return launch_gen_prox_gstar<S>(P, w, out, st);
  const int nl = P.tree->nl;
  hipLaunchKernelGGL(k_prox_gstar<S>, dim3((nl + 127) / 128), dim3(128), 0, st, dev_of<S>(P), w, out);
  return hipGetLastError();
}
template hipError_t launch_L_batch<double>(const Problem&, const double*, double*, long long, int, hipStream_t);
template hipError_t launch_L_batch<float>(const Problem&, const float*, float*, long long, int, hipStream_t);
template hipError_t launch_Lt_batch<double>(const Problem&, const double*, double*, long long, int, hipStream_t);
template hipError_t launch_Lt_batch<float>(const Problem&, const float*, float*, long long, int, hipStream_t);
template hipError_t launch_L<double>(const Problem&, const double*, double*, hipStream_t);
template hipError_t launch_L<float>(const Problem&, const float*, float*, hipStream_t);
template hipError_t launch_Lt<double>(const Problem&, const double*, double*, hipStream_t);
template hipError_t launch_Lt<float>(const Problem&, const float*, float*, hipStream_t);
template hipError_t launch_prox_gstar<double>(const Problem&, const double*, double*, hipStream_t);
template hipError_t launch_prox_gstar<float>(const Problem&, const float*, float*, hipStream_t);

// ---------------------------------------------------------------- vector kernels
constexpr int kVecBlocks = 1024;
int dots_blocks(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < kVecBlocks ? (b < 1 ? 1 : b) : kVecBlocks);
}

// Streaming vector kernels read and write 16 bytes per lane (float4 /
// double2, kVW elements): enough bytes in flight per wavefront to cover the
// HBM latency. Elements past the last whole vector, and every element when a
// pointer is not 16-byte aligned, take the scalar path of the same kernel.
template <typename S>
constexpr int kVW = 16 / (int)sizeof(S);
template <typename S>
struct Vec16;
template <>
struct Vec16<float> {
  using T = float4;
};
template <>
struct Vec16<double> {
  using T = double2;
};
template <typename S>
__device__ __forceinline__ void ld16(const S* __restrict__ p, long long k, S (&a)[kVW<S>]) {
  const typename Vec16<S>::T x = reinterpret_cast<const typename Vec16<S>::T*>(p)[k];
  __builtin_memcpy(a, &x, 16);
}
template <typename S>
__device__ __forceinline__ void st16(S* __restrict__ p, long long k, const S (&a)[kVW<S>]) {
  typename Vec16<S>::T x;
  __builtin_memcpy(&x, a, 16);
  reinterpret_cast<typename Vec16<S>::T*>(p)[k] = x;
}
static bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
// whole vectors of the vector path (0 when some pointer is unaligned)
template <typename S>
static long long nvec16(long long n, std::initializer_list<const void*> ptrs) {
  for (const void* q : ptrs)
    if (q && !al16(q)) return 0;
  return n / kVW<S>;
}
#define SPK_GRID_LOOP(k, lo, hi)                                                             \
  for (long long k = (lo) + blockIdx.x * (long long)blockDim.x + threadIdx.x; k < (hi); \
       k += (long long)gridDim.x * blockDim.x)

// out = a x + b y (y may be null)
template <typename S>
__global__ void __launch_bounds__(256) k_lincomb(long long n, long long nv, S* __restrict__ out, double a,
                                                 const S* __restrict__ x, double b, const S* __restrict__ y) {
  constexpr int W = kVW<S>;
  SPK_GRID_LOOP(k, 0, nv) {
    S xv[W], yv[W], o[W];
    ld16(x, k, xv);
    if (y) ld16(y, k, yv);
#pragma unroll
    for (int c = 0; c < W; ++c) o[c] = (S)(a * (double)xv[c] + (y ? b * (double)yv[c] : 0.0));
    st16(out, k, o);
  }
  SPK_GRID_LOOP(e, nv * W, n) {
    double v = a * (double)x[e];
    if (y) v += b * (double)y[e];
    out[e] = (S)v;
  }
}
template <typename S>
hipError_t launch_lincomb(long long n, S* out, double a, const S* x, double b, const S* y,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb<S>, dim3(dots_blocks(n)), dim3(256), 0, st, n, nvec16<S>(n, {out, x, y}), out, a,
                     x, b, y);
  return hipGetLastError();
}
// out = a x + b y + c w
template <typename S>
__global__ void __launch_bounds__(256) k_lincomb3(long long n, long long nv, S* __restrict__ out, double a,
                                                  const S* __restrict__ x, double b, const S* __restrict__ y,
                                                  double c, const S* __restrict__ w) {
  constexpr int W = kVW<S>;
  SPK_GRID_LOOP(k, 0, nv) {
    S xv[W], yv[W], wv[W], o[W];
    ld16(x, k, xv);
    ld16(y, k, yv);
    ld16(w, k, wv);
#pragma unroll
    for (int q = 0; q < W; ++q) o[q] = (S)(a * (double)xv[q] + b * (double)yv[q] + c * (double)wv[q]);
    st16(out, k, o);
  }
  SPK_GRID_LOOP(e, nv * W, n) out[e] = (S)(a * (double)x[e] + b * (double)y[e] + c * (double)w[e]);
}
template <typename S>
hipError_t launch_lincomb3(long long n, S* out, double a, const S* x, double b, const S* y,
                           double c, const S* w, hipStream_t st) {
  hipLaunchKernelGGL(k_lincomb3<S>, dim3(dots_blocks(n)), dim3(256), 0, st, n, nvec16<S>(n, {out, x, y, w}), out,
                     a, x, b, y, c, w);
  return hipGetLastError();
}
template <typename S>
__global__ void k_fill(long long n, S* __restrict__ out, double val) {
  SPK_GRID_LOOP(e, 0, n) out[e] = (S)val;
}
template <typename S>
hipError_t launch_fill(long long n, S* out, double val, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<S>, dim3(dots_blocks(n)), dim3(256), 0, st, n, out, val);
  return hipGetLastError();
}

// Block-deterministic reduction of up to 8 per-thread sums.
template <int K>
__device__ void block_sums(double (&acc)[K], double* partials) {
  __shared__ double red[8][256];
  for (int j = 0; j < K; ++j) red[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int s = blockDim.x / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int j = 0; j < K; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + s];
    __syncthreads();
  }
  if ((int)threadIdx.x < K) partials[(size_t)blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// Sums K <= 8 columns of nblk partial records (stride 8) in a fixed order:
// thread t takes records t, t + 256, ..., then a tree over the threads (a
// 256-thread block; the sums end in red[j][0]).
__device__ void final_sums_in(const double* __restrict__ partials, int nblk, int K, double (*red)[256]) {
  const int t = threadIdx.x;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = t; b < nblk; b += 256) {
    const double* p = partials + (size_t)b * 8;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < K) s[j] += p[j];
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) red[j][t] = s[j];
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (t < h)
#pragma unroll
      for (int j = 0; j < 8; ++j) red[j][t] += red[j][t + h];
    __syncthreads();
  }
}
__global__ void __launch_bounds__(256) k_final_sums(const double* __restrict__ partials, int nblk, int K,
                                                    double* __restrict__ out) {
  __shared__ double red[8][256];
  final_sums_in(partials, nblk, K, red);
  if ((int)threadIdx.x < K) out[threadIdx.x] = red[threadIdx.x][0];
}

// Reduction finished inside the launch, in two levels of tagged records.
// Each block's sums (fixed-order tree) go to its record as tagged words
// (epoch << 32 | half; record r holds 8 doubles, rec[(r * 8 + j) * 2 + {0,1}]).
// Blocks arrive in groups of kGroup on device-scope counters; the last block
// of a group sums the group's records in block order into a group record
// (after the kMaxRecBlocks block records), and the last group to finish sums
// the group records in order. The records carry the launch's tag, so readers
// poll until they arrive and no fence orders them against the counts; each
// last arriver resets its counter for the next launch.
constexpr int kGroup = kRedGroup;
constexpr int kMaxRecBlocks = kRedMaxBlocks;
static_assert(kVecBlocks <= kMaxRecBlocks, "one record per block of a vector kernel");
constexpr unsigned kRecSpin = 1u << 20;  // polls of one record word before giving up (NaN)

__device__ double poll_tagged(const unsigned long long* w, unsigned tag) {
  double v = 0;
  unsigned it = 0;
  while (!get_tagged<double>(w, tag, v) && ++it < kRecSpin) __builtin_amdgcn_s_sleep(1);
  return it < kRecSpin ? v : __builtin_nan("");
}

// Sums the first n records at base in order (256 threads; thread r * 8 + j
// reads column j of record r, n <= 32); column sums end in red[j][0].
__device__ void sum_records(const unsigned long long* base, int n, int K, unsigned tag, double (*red)[256]) {
  const int t = threadIdx.x, r = t >> 3, j = t & 7;
  red[j][r] = (r < n && j < K) ? poll_tagged(base + ((size_t)r * 8 + j) * 2, tag) : 0.0;
  __syncthreads();
  if (t < 8) {
    double s = 0;
    for (int q = 0; q < n; ++q) s += red[t][q];
    red[t][0] = s;  // row 0 of column t: only this thread touches column t here
  }
  __syncthreads();
}

__device__ bool arrive(unsigned* c, unsigned expected) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    last = atomicAdd(c, 1u) == expected - 1;
    if (last) atomicExch(c, 0u);
  }
  __syncthreads();
  return last != 0;
}

// Block sums of acc, then the grid sums: true in the one block that holds
// them (red[j][0], j < K) at the end.
template <int K, typename F>
__device__ bool grid_sums_tagged(const double* acc, unsigned long long* rec, unsigned* counters, unsigned tag,
                                 double (*red)[256], F&& on_group_last) {
  for (int j = 0; j < K; ++j) red[j][threadIdx.x] = acc[j];
  __syncthreads();
  for (int s = blockDim.x / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int j = 0; j < K; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + s];
    __syncthreads();
  }
  const int b = blockIdx.x, nb = gridDim.x;
  if ((int)threadIdx.x < K) put_tagged<double>(rec + ((size_t)b * 8 + threadIdx.x) * 2, red[threadIdx.x][0], tag);
  const int g = b / kGroup, ng = (nb + kGroup - 1) / kGroup;
  const int gsize = min(kGroup, nb - g * kGroup);
  if (!arrive(counters + g, gsize)) return false;
  on_group_last();  // loads the final block may need, issued before its polls
  sum_records(rec + (size_t)g * kGroup * 16, gsize, K, tag, red);
  unsigned long long* grec = rec + (size_t)kMaxRecBlocks * 16;
  if ((int)threadIdx.x < K) put_tagged<double>(grec + ((size_t)g * 8 + threadIdx.x) * 2, red[threadIdx.x][0], tag);
  if (!arrive(counters + kMaxRecBlocks / kGroup, ng)) return false;
  sum_records(grec, ng, K, tag, red);
  return true;
}

// out[j] = <x_j, y_j>, j < k <= 8
template <typename S>
__global__ void k_dots(long long n, int k, VecPtrs<S> xs, VecPtrs<S> ys, double* __restrict__ partials) {
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    for (int j = 0; j < k; ++j) acc[j] += (double)xs.p[j][e] * (double)ys.p[j][e];
  block_sums<8>(acc, partials);
}
template <typename S>
hipError_t launch_dots(long long n, int k, VecPtrs<S> xs, VecPtrs<S> ys,
                       double* partials, double* out_dev, hipStream_t st) {
  const int nb = dots_blocks(n);
  hipLaunchKernelGGL(k_dots<S>, dim3(nb), dim3(256), 0, st, n, k, xs, ys, partials);
  hipLaunchKernelGGL(k_final_sums, dim3(1), dim3(256), 0, st, partials, nb, k, out_dev);
  return hipGetLastError();
}

// <v - Tv, w> into *out; the last block to finish sums the records and
// publishes stats[0..8) (with out among them) when pub.mb is set
template <typename S>
__global__ void __launch_bounds__(256) k_rdot(long long n, long long nv, const S* __restrict__ v,
                                              const S* __restrict__ Tv, const S* __restrict__ w,
                                              unsigned long long* __restrict__ rec,
                                              unsigned* __restrict__ counter, unsigned tag, double* out,
                                              const double* stats, Publish pub) {
  __shared__ double red[8][256];
  constexpr int W = kVW<S>;
  double acc[1] = {0};
  SPK_GRID_LOOP(k, 0, nv) {
    S a[W], b[W], c[W];
    ld16(v, k, a);
    ld16(Tv, k, b);
    ld16(w, k, c);
#pragma unroll
    for (int q = 0; q < W; ++q) acc[0] += ((double)a[q] - (double)b[q]) * (double)c[q];
  }
  SPK_GRID_LOOP(e, nv * W, n) acc[0] += ((double)v[e] - (double)Tv[e]) * (double)w[e];
  if (!grid_sums_tagged<1>(acc, rec, counter, tag, red, [] {})) return;
  if (threadIdx.x == 0) {
    *out = red[0][0];
    if (pub.mb) {
      double r[8];
      for (int k = 0; k < 8; ++k) r[k] = stats[k];
      publish_stats(r, pub);
    }
  }
}
template <typename S>
hipError_t launch_rdot(long long n, const S* v, const S* Tv, const S* w, unsigned long long* rec, unsigned* counter,
                       unsigned tag, double* out_dev, const double* stats, Publish pub, hipStream_t st) {
  const int nb = dots_blocks(n);
  hipLaunchKernelGGL(k_rdot<S>, dim3(nb), dim3(256), 0, st, n, nvec16<S>(n, {v, Tv, w}), v, Tv, w, rec, counter,
                     tag, out_dev, stats, pub);
  return hipGetLastError();
}

// d = -r - sum_j gamma_j (dV_j - dR_j), M columns; step = base + d when
// step is set
template <typename S, int M>
__device__ __forceinline__ void aa_dir_body(long long n, long long nv, const S* __restrict__ r, const VecPtrs<S>& dE,
                                            const double* __restrict__ gamma, S* __restrict__ d,
                                            const S* __restrict__ base, S* __restrict__ step) {
  constexpr int W = kVW<S>;
  double g[M];
#pragma unroll
  for (int j = 0; j < M; ++j) g[j] = gamma[j];
  SPK_GRID_LOOP(k, 0, nv) {
    S rv[W], ev[M][W], o[W];
    ld16(r, k, rv);
#pragma unroll
    for (int j = 0; j < M; ++j) ld16(dE.p[j], k, ev[j]);
    double acc[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
      acc[q] = -(double)rv[q];
#pragma unroll
      for (int j = 0; j < M; ++j) acc[q] -= g[j] * (double)ev[j][q];
      o[q] = (S)acc[q];
    }
    st16(d, k, o);
    if (step) {
      S bv[W];
      ld16(base, k, bv);
#pragma unroll
      for (int q = 0; q < W; ++q) o[q] = (S)((double)bv[q] + acc[q]);
      st16(step, k, o);
    }
  }
  SPK_GRID_LOOP(e, nv * W, n) {
    double acc = -(double)r[e];
#pragma unroll
    for (int j = 0; j < M; ++j) acc -= g[j] * (double)dE.p[j][e];
    d[e] = (S)acc;
    if (step) step[e] = (S)((double)base[e] + acc);
  }
}
// The direction of the columns the last push used (ring->dk of them, slots
// ring->dslot; E of slot s at eb + s * stride).
template <typename S>
__global__ void __launch_bounds__(256) k_aa_dir(long long n, long long nv, const S* __restrict__ r,
                                                const S* __restrict__ eb, long long stride,
                                                const AARingDev* __restrict__ ring,
                                                const double* __restrict__ gamma, S* __restrict__ d,
                                                const S* __restrict__ base, S* __restrict__ step) {
  const int m = ring->dk;
  VecPtrs<S> dE{};
#pragma unroll
  for (int j = 0; j < kAAMax; ++j) dE.p[j] = j < m ? eb + ring->dslot[j] * stride : eb;
  switch (m) {
    case 1: aa_dir_body<S, 1>(n, nv, r, dE, gamma, d, base, step); break;
    case 2: aa_dir_body<S, 2>(n, nv, r, dE, gamma, d, base, step); break;
    case 3: aa_dir_body<S, 3>(n, nv, r, dE, gamma, d, base, step); break;
    default: aa_dir_body<S, 4>(n, nv, r, dE, gamma, d, base, step); break;
  }
}
// Anderson step on the device (section 6.2, type-II; one thread, k <= 4):
// the Gram row of the newest difference and the right-hand side <dR_j, r>
// come from the push dot products; the oldest columns are dropped until the
// Gram matrix of the kept ones has lambda_min / lambda_max >= 1e-12 (the
// singular-value ratio 1e-6 of the residual differences; cyclic Jacobi until
// the test is decided) and a Cholesky factor; gamma solves G gamma = rhs. gamma
// is written for every column of the order (0 for dropped ones), and the
// device ring takes the new order (the kept columns) and the direction's
// columns.
// Fixed-size (N <= 4) helpers, fully unrolled so that the matrices stay in
// registers.
template <int N>
__device__ __forceinline__ bool dev_chol(double (&A)[16]) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double d = A[j * 4 + j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= A[j * 4 + k] * A[j * 4 + k];
    if (!(d > 0.0) || !isfinite(d)) return false;
    d = sqrt(d);
    A[j * 4 + j] = d;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      double s = A[i * 4 + j];
#pragma unroll
      for (int k = 0; k < j; ++k) s -= A[i * 4 + k] * A[j * 4 + k];
      A[i * 4 + j] = s / d;
    }
  }
  return true;
}

// Rank test of a symmetric N x N matrix: lambda_min / lambda_max >= 1e-12
// with lambda_max > 0. Cyclic Jacobi sweeps until the test is decided: with
// off the sum of squares of the upper off-diagonal entries, every eigenvalue
// lies within e = sqrt(2 off) of a diagonal entry (Weyl), so the extreme
// eigenvalues are within e of the smallest and largest diagonal entries.
template <int N>
__device__ __forceinline__ bool dev_rank_ok(double (&A)[16]) {
  constexpr double kTol = 1e-12;
  for (int sweep = 0;; ++sweep) {
    double off = 0, dmin = A[0], dmax = A[0];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      dmin = fmin(dmin, A[i * 4 + i]);
      dmax = fmax(dmax, A[i * 4 + i]);
#pragma unroll
      for (int j = i + 1; j < N; ++j) off += A[i * 4 + j] * A[i * 4 + j];
    }
    const double e = sqrt(2.0 * off);
    if (dmax - e > 0.0 && dmin - e >= kTol * (dmax + e)) return true;           // certainly passes
    if (dmax + e <= 0.0 || (dmax - e > 0.0 && dmin + e < kTol * (dmax - e))) return false;  // certainly fails
    if (sweep == 60 || off < 1e-300) return dmax > 0.0 && dmin >= kTol * dmax;  // the diagonal is the spectrum
#pragma unroll
    for (int p = 0; p < N; ++p)
#pragma unroll
      for (int q = p + 1; q < N; ++q) {
        const double apq = A[p * 4 + q];
        if (apq != 0.0) {
          const double th = 0.5 * (A[q * 4 + q] - A[p * 4 + p]) / apq;
          const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
          for (int k = 0; k < N; ++k) {
            const double akp = A[k * 4 + p], akq = A[k * 4 + q];
            A[k * 4 + p] = c * akp - s * akq;
            A[k * 4 + q] = s * akp + c * akq;
          }
#pragma unroll
          for (int k = 0; k < N; ++k) {
            const double apk = A[p * 4 + k], aqk = A[q * 4 + k];
            A[p * 4 + k] = c * apk - s * aqk;
            A[q * 4 + k] = s * apk + c * aqk;
          }
        }
      }
  }
}

// Rank test and solve for the last N of the k active columns (rows/cols
// `off..off+N` of Gk, right-hand side rk); true when kept.
template <int N, int off>
__device__ __forceinline__ bool dev_aa_try(const double (&Gk)[16], const double (&rk)[4], double (&g)[4]) {
  double E[16], L[16];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) E[i * 4 + j] = L[i * 4 + j] = Gk[(off + i) * 4 + off + j];
  if (!dev_rank_ok<N>(E) || !dev_chol<N>(L)) return false;
  double y[4];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = rk[off + i];
#pragma unroll
    for (int j = 0; j < i; ++j) s -= L[i * 4 + j] * y[j];
    y[i] = s / L[i * 4 + i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double s = y[i];
#pragma unroll
    for (int j = i + 1; j < N; ++j) s -= L[j * 4 + i] * g[off + j];
    g[off + i] = s / L[i * 4 + i];
  }
  return true;
}

// Tries the last K - DROP columns, then fewer; the number kept (0: none).
template <int K, int DROP>
__device__ __forceinline__ int aa_try_from(const double (&Gk)[16], const double (&rk)[4], double (&g)[4]) {
  if constexpr (DROP >= K) {
    return 0;
  } else {
    if (dev_aa_try<K - DROP, DROP>(Gk, rk, g)) return K - DROP;
    return aa_try_from<K, DROP + 1>(Gk, rk, g);
  }
}

// MO columns before the push (all indices fixed at compile time). Gold:
// the Gram entries of the old columns (oldest first), read before the sums
// were done; the new column's entries and the right-hand side <dR_j, r>
// come from the dots. The new row is stored in G (by slot) for later pushes.
template <int MO>
__device__ __forceinline__ void aa_solve_dev(double* __restrict__ G, const double (&dots)[8],
                                             const double (&Gold)[16], const AAPush& a,
                                             double* __restrict__ gamma, AARingDev* __restrict__ ring) {
  const int m = a.m, slot = a.slot;
#pragma unroll
  for (int j = 0; j < MO; ++j) {
    G[a.order_old[j] * m + slot] = dots[j];
    G[slot * m + a.order_old[j]] = dots[j];
  }
  G[slot * m + slot] = dots[MO];
  constexpr int k = MO + 1;  // order_new = order_old + [slot]
  // Gram matrix and right-hand side of the active columns, in registers
  double Gk[16], rk[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    rk[i] = i < MO ? dots[MO + 1 + i] : (i == MO ? dots[2 * MO + 1] : 0.0);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      Gk[i * 4 + j] = (i < MO && j < MO) ? Gold[i * 4 + j]
                    : (i == MO && j < MO) ? dots[j]
                    : (j == MO && i < MO) ? dots[i]
                    : (i == MO && j == MO) ? dots[MO] : 0.0;
  }
  double g[4] = {0, 0, 0, 0};
  // drop the oldest columns until the rest pass the rank test
  const int kept = aa_try_from<k, 0>(Gk, rk, g);
  if (kept == 0) g[0] = g[1] = g[2] = g[3] = 0.0;
#pragma unroll
  for (int j = 0; j < k; ++j) gamma[j] = g[j];
  // the ring: the direction uses the k columns (dropped ones with gamma 0);
  // the next push keeps the newest `kept`
  int ord[4] = {0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < MO; ++j) ord[j] = a.order_old[j];
  ord[MO] = slot;
  ring->dk = k;
#pragma unroll
  for (int j = 0; j < k; ++j) ring->dslot[j] = ord[j];
  ring->cnt = kept;
#pragma unroll
  for (int j = 0; j < k; ++j) {
    int sel = 0;
#pragma unroll
    for (int q = 0; q < k; ++q) sel = (q == k - kept + j) ? ord[q] : sel;
    if (j < kept) ring->order[j] = sel;
  }
}

// Anderson push: r = v - Tv, dV = v - vprev, dR = r - rprev, with the
// difference E = dV - dR stored in place of dV (the direction needs only E);
// dots[j] = <dR_old_j, dR_new> (j < m_old), dots[m_old] = <dR_new, dR_new>,
// dots[m_old+1+j] = <dR_old_j, r>, dots[2 m_old + 1] = <dR_new, r>, summed
// in a fixed order by the last block to finish, which then solves for gamma.
template <typename S, int MO>
__device__ __forceinline__ void aa_push_body(long long n, long long nv, const S* __restrict__ v,
                                             const S* __restrict__ vprev, const S* __restrict__ Tv,
                                             const S* __restrict__ rprev, S* __restrict__ r_out,
                                             S* __restrict__ dV_new, S* __restrict__ dR_new, const VecPtrs<S>& dR_old,
                                             unsigned long long* __restrict__ rec, unsigned* __restrict__ counter,
                                             unsigned tag, double* __restrict__ G, const AAPush& a,
                                             double* __restrict__ gamma, AARingDev* __restrict__ ring,
                                             double (*red)[256]) {
  constexpr int m_old = MO;
  constexpr int W = kVW<S>;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // one element: r, dR and E = dV - dR, and the dot-product terms
  auto elem = [&](S vv, S tv, S rp, S vp, const S (&o)[MO > 0 ? MO : 1], S& r, S& dr, S& ev) {
    r = vv - tv;
    dr = r - rp;
    ev = (S)(((double)vv - (double)vp) - (double)dr);
#pragma unroll
    for (int j = 0; j < m_old; ++j) {
      acc[j] += (double)o[j] * (double)dr;
      acc[m_old + 1 + j] += (double)o[j] * (double)r;
    }
    acc[m_old] += (double)dr * (double)dr;
    acc[2 * m_old + 1] += (double)dr * (double)r;
  };
  SPK_GRID_LOOP(k, 0, nv) {
    S vv[W], tv[W], rp[W], vp[W], ov[MO > 0 ? MO : 1][W], r[W], dr[W], ev[W];
    ld16(v, k, vv);
    ld16(Tv, k, tv);
    ld16(rprev, k, rp);
    ld16(vprev, k, vp);
#pragma unroll
    for (int j = 0; j < MO; ++j) ld16(dR_old.p[j], k, ov[j]);
#pragma unroll
    for (int q = 0; q < W; ++q) {
      S o[MO > 0 ? MO : 1];
#pragma unroll
      for (int j = 0; j < MO; ++j) o[j] = ov[j][q];
      elem(vv[q], tv[q], rp[q], vp[q], o, r[q], dr[q], ev[q]);
    }
    st16(r_out, k, r);
    st16(dR_new, k, dr);
    st16(dV_new, k, ev);
  }
  SPK_GRID_LOOP(e, nv * W, n) {
    S o[MO > 0 ? MO : 1];
#pragma unroll
    for (int j = 0; j < MO; ++j) o[j] = dR_old.p[j][e];
    S r, dr, ev;
    elem(v[e], Tv[e], rprev[e], vprev[e], o, r, dr, ev);
    r_out[e] = r;
    dR_new[e] = dr;
    dV_new[e] = ev;
  }
  double Gold[16];
  auto load_gram = [&] {
    if (threadIdx.x == 0)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) Gold[i * 4 + j] = (i < MO && j < MO) ? G[a.order_old[i] * a.m + a.order_old[j]] : 0.0;
  };
  if (!grid_sums_tagged<2 * m_old + 2>(acc, rec, counter, tag, red, load_gram)) return;
  if (threadIdx.x == 0) {
    double dots[8];
    for (int k = 0; k < 8; ++k) dots[k] = red[k][0];
    aa_solve_dev<MO>(G, dots, Gold, a, gamma, ring);
  }
}
// The push reads the ring as the last push's solve left it: the new column
// takes the oldest slot when the ring is full, else the lowest free one; the
// dots run against the other columns of the order.
template <typename S>
__global__ void __launch_bounds__(256) k_aa_push(long long n, long long nv, const S* __restrict__ v,
                                                 const S* __restrict__ vprev, const S* __restrict__ Tv,
                                                 const S* __restrict__ rprev, S* __restrict__ r_out,
                                                 S* __restrict__ eb, S* __restrict__ rb, long long stride,
                                                 unsigned long long* __restrict__ rec,
                                                 unsigned* __restrict__ counter, unsigned tag, double* __restrict__ G,
                                                 AARingDev* __restrict__ ring, double* __restrict__ gamma) {
  __shared__ double red[8][256];
  // (fixed indices and selects only, so that nothing lands in scratch)
  AAPush a{};
  a.m = ring->m;
  const int cnt = ring->cnt;
  int o[kAAMax];
#pragma unroll
  for (int j = 0; j < kAAMax; ++j) o[j] = ring->order[j];
  const bool full = cnt == a.m;
  a.mo = full ? cnt - 1 : cnt;
#pragma unroll
  for (int j = 0; j < kAAMax; ++j) a.order_old[j] = full ? (j + 1 < kAAMax ? o[j + 1] : 0) : o[j];
  int fr = kAAMax;  // lowest slot not in the order
#pragma unroll
  for (int s = kAAMax - 1; s >= 0; --s) {
    bool used = false;
#pragma unroll
    for (int j = 0; j < kAAMax; ++j) used = used || (j < cnt && o[j] == s);
    if (!used && s < a.m) fr = s;
  }
  a.slot = full ? o[0] : fr;
  VecPtrs<S> dR_old{};
#pragma unroll
  for (int j = 0; j < kAAMax - 1; ++j) dR_old.p[j] = j < a.mo ? rb + a.order_old[j] * stride : nullptr;
  S* dV_new = eb + a.slot * stride;
  S* dR_new = rb + a.slot * stride;
  switch (a.mo) {
    case 0: aa_push_body<S, 0>(n, nv, v, vprev, Tv, rprev, r_out, dV_new, dR_new, dR_old, rec, counter, tag, G, a, gamma, ring, red); break;
    case 1: aa_push_body<S, 1>(n, nv, v, vprev, Tv, rprev, r_out, dV_new, dR_new, dR_old, rec, counter, tag, G, a, gamma, ring, red); break;
    case 2: aa_push_body<S, 2>(n, nv, v, vprev, Tv, rprev, r_out, dV_new, dR_new, dR_old, rec, counter, tag, G, a, gamma, ring, red); break;
    default: aa_push_body<S, 3>(n, nv, v, vprev, Tv, rprev, r_out, dV_new, dR_new, dR_old, rec, counter, tag, G, a, gamma, ring, red); break;
  }
}
// 16-byte vector path when the bases and the stride keep every slot aligned
template <typename S>
static bool slots_aligned(const S* eb, const S* rb, long long stride) {
  return al16(eb) && (!rb || al16(rb)) && ((stride * (long long)sizeof(S)) & 15) == 0;
}
template <typename S>
hipError_t launch_aa_push(long long n, const S* v, const S* vprev, const S* Tv, const S* rprev, S* r_out, S* eb,
                          S* rb, long long stride, unsigned long long* rec, unsigned* counter, unsigned tag,
                          double* G, AARingDev* ring, double* gamma, hipStream_t st) {
  const long long nv = slots_aligned<S>(eb, rb, stride) ? nvec16<S>(n, {v, vprev, Tv, rprev, r_out}) : 0;
  hipLaunchKernelGGL(k_aa_push<S>, dim3(dots_blocks(n)), dim3(256), 0, st, n, nv, v, vprev, Tv, rprev, r_out, eb,
                     rb, stride, rec, counter, tag, G, ring, gamma);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_aa_dir(long long n, const S* r, const S* eb, long long stride, const AARingDev* ring,
                         const double* gamma_dev, S* d, const S* base, S* step, hipStream_t st) {
  const long long nv = slots_aligned<S>(eb, nullptr, stride) ? nvec16<S>(n, {r, d, base, step}) : 0;
  hipLaunchKernelGGL(k_aa_dir<S>, dim3(dots_blocks(n)), dim3(256), 0, st, n, nv, r, eb, stride, ring, gamma_dev, d,
                     base, step);
  return hipGetLastError();
}

// Krylov basis kernels of the adjoint GMRES. The basis vectors are
// V_j = basis + j * stride. k_basis_dots: block (c, j) sums chunk c of
// <V_j, x> (j < n; <x, x> for j = n when the grid has n + 1 rows) in FP64
// into part[j * gridDim.x + c]; k_basis_final adds the chunks in order.
template <typename S>
__global__ void __launch_bounds__(256) k_basis_dots(long long nv, int n, const S* __restrict__ basis,
                                                    long long stride, const S* __restrict__ x,
                                                    double* __restrict__ part) {
  const int j = blockIdx.y;
  const S* v = j < n ? basis + (size_t)j * (size_t)stride : x;
  const long long chunk = (nv + gridDim.x - 1) / gridDim.x;
  const long long e0 = (long long)blockIdx.x * chunk;
  const long long e1 = e0 + chunk < nv ? e0 + chunk : nv;
  double acc = 0;
  for (long long e = e0 + threadIdx.x; e < e1; e += 256) acc += (double)v[e] * (double)x[e];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)j * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}
__global__ void __launch_bounds__(256) k_basis_final(const double* __restrict__ part, int cb, int m,
                                                     double* __restrict__ out, double* __restrict__ host_out) {
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    double acc = 0;
    for (int c = 0; c < cb; ++c) acc += part[(size_t)j * cb + c];
    out[j] = acc;
    if (host_out) host_out[j] = acc;  // mapped pinned memory, visible once the kernel completes
  }
}
// chunks per basis vector: about 8192 elements each, at most kBasisChunks
static int basis_chunks(long long nv) {
  const long long c = (nv + 8191) / 8192;
  return (int)(c < 1 ? 1 : (c > kBasisChunks ? kBasisChunks : c));
}
template <typename S>
hipError_t launch_basis_dots(long long nv, int n, const S* basis, long long stride, const S* x, bool xx,
                             double* part, double* out_dev, hipStream_t st, double* host_out) {
  if (n < 0 || n + (xx ? 1 : 0) > kBasisMax + 1 || n + (xx ? 1 : 0) < 1) return hipErrorInvalidValue;
  const int cb = basis_chunks(nv), m = n + (xx ? 1 : 0);
  hipLaunchKernelGGL(k_basis_dots<S>, dim3(cb, m), dim3(256), 0, st, nv, n, basis, stride, x, part);
  hipLaunchKernelGGL(k_basis_final, dim3(1), dim3(256), 0, st, part, cb, m, out_dev, host_out);
  return hipGetLastError();
}
// out = a x + sum_{j < n} C.c[j] V_j (out may be x: each element is read
// before it is written, by the same thread)
template <typename S>
__global__ void __launch_bounds__(256) k_basis_mix(long long nv, int n, const S* __restrict__ basis,
                                                   long long stride, BasisCoef C, double a, const S* x, S* out) {
  SPK_GRID_LOOP(e, 0, nv) {
    double acc = a * (double)x[e];
    for (int j = 0; j < n; ++j) acc += C.c[j] * (double)basis[(size_t)j * (size_t)stride + e];
    out[e] = (S)acc;
  }
}
template <typename S>
hipError_t launch_basis_mix(long long nv, int n, const S* basis, long long stride, const BasisCoef& C, double a,
                            const S* x, S* out, hipStream_t st) {
  if (n < 0 || n > kBasisMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_basis_mix<S>, dim3(dots_blocks(nv)), dim3(256), 0, st, nv, n, basis, stride, C, a, x, out);
  return hipGetLastError();
}

// In-place Gram-Schmidt pass with device-resident coefficients: x -= sum_{j
// < n} c[j] V_j; when norm, the result is also scaled by 1 / sqrt(c[n] -
// sum_j c[j]^2) (c[n] = <x, x> before the pass; 0 when that is not
// positive), so no coefficient has to travel to the host first.
template <typename S>
__global__ void __launch_bounds__(256) k_basis_orth(long long nv, int n, const S* __restrict__ basis,
                                                    long long stride, const double* __restrict__ c, int norm,
                                                    S* x) {
  double scale = 1.0;
  if (norm) {
    double h2 = c[n];
    for (int j = 0; j < n; ++j) h2 -= c[j] * c[j];
    scale = h2 > 0.0 ? 1.0 / sqrt(h2) : 0.0;
  }
  SPK_GRID_LOOP(e, 0, nv) {
    double acc = (double)x[e];
    for (int j = 0; j < n; ++j) acc -= c[j] * (double)basis[(size_t)j * (size_t)stride + e];
    x[e] = (S)(acc * scale);
  }
}
template <typename S>
hipError_t launch_basis_orth(long long nv, int n, const S* basis, long long stride, const double* c_dev, bool norm,
                             S* x, hipStream_t st) {
  if (n < 0 || n > kBasisMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_basis_orth<S>, dim3(dots_blocks(nv)), dim3(256), 0, st, nv, n, basis, stride, c_dev,
                     norm ? 1 : 0, x);
  return hipGetLastError();
}

// Column mix for the QR-updated Anderson step: out_i = sum_j C[i][j] in_j
// over the elements (i < nout, j < nin, both <= kMixMax). Every thread reads
// all inputs of its elements before it writes, so outputs may alias inputs.
template <typename S>
__global__ void __launch_bounds__(256) k_colmix(long long n, ColMix<S> M) {
  SPK_GRID_LOOP(e, 0, n) {
    double x[kMixMax];
#pragma unroll
    for (int j = 0; j < kMixMax; ++j) x[j] = j < M.nin ? (double)M.in[j][e] : 0.0;
#pragma unroll
    for (int i = 0; i < kMixMax; ++i) {
      if (i >= M.nout) break;
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < kMixMax; ++j) acc += j < M.nin ? M.c[i][j] * x[j] : 0.0;
      M.out[i][e] = (S)acc;
    }
  }
}
template <typename S>
hipError_t launch_colmix(long long n, const ColMix<S>& M, hipStream_t st) {
  if (M.nin < 1 || M.nin > kMixMax || M.nout < 1 || M.nout > kMixMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_colmix<S>, dim3(dots_blocks(n)), dim3(256), 0, st, n, M);
  return hipGetLastError();
}

#define SPK_INST(S)                                                                                \
  template hipError_t launch_lincomb<S>(long long, S*, double, const S*, double, const S*,         \
                                        hipStream_t);                                              \
  template hipError_t launch_lincomb3<S>(long long, S*, double, const S*, double, const S*, double, \
                                         const S*, hipStream_t);                                   \
  template hipError_t launch_fill<S>(long long, S*, double, hipStream_t);                          \
  template hipError_t launch_dots<S>(long long, int, VecPtrs<S>, VecPtrs<S>, double*, double*,     \
                                     hipStream_t);                                                 \
  template hipError_t launch_rdot<S>(long long, const S*, const S*, const S*, unsigned long long*,  \
                                     unsigned*, unsigned, double*, const double*, Publish,          \
                                     hipStream_t);                                                  \
  template hipError_t launch_aa_push<S>(long long, const S*, const S*, const S*, const S*, S*, S*,  \
                                        S*, long long, unsigned long long*, unsigned*, unsigned,    \
                                        double*, AARingDev*, double*, hipStream_t);                 \
  template hipError_t launch_aa_dir<S>(long long, const S*, const S*, long long, const AARingDev*,  \
                                       const double*, S*, const S*, S*, hipStream_t);              \
  template hipError_t launch_colmix<S>(long long, const ColMix<S>&, hipStream_t);                  \
  template hipError_t launch_basis_dots<S>(long long, int, const S*, long long, const S*, bool, double*, \
                                           double*, hipStream_t, double*);                              \
  template hipError_t launch_basis_mix<S>(long long, int, const S*, long long, const BasisCoef&, double,   \
                                          const S*, S*, hipStream_t);                                     \
  template hipError_t launch_basis_orth<S>(long long, int, const S*, long long, const double*, bool, S*,  \
                                           hipStream_t);
SPK_INST(double)
SPK_INST(float)

}  // namespace spk
