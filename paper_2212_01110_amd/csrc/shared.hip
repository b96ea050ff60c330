// Shared-tree batched form: B instances of one problem (the same tree, dynamics,
// costs, boxes and risk parameters) that differ only in x0 and in their
// iterates. Every instance runs Alg. 3 (or CP) with its own decisions; the
// instances advance in lockstep rounds, one evaluation of the CP operator T
// (section 3) per round for all of them, so that the Riccati-type sweeps of
// the S1 projection (Alg. 2) see B right-hand sides per node at once: each
// per-node mat-vec of the single-instance form becomes a product of the
// node's factored matrix with a [dimension x 16 instances] tile on the
// matrix cores (MFMA 16x16x4, FP32 or FP64).
//
// Layout: vector buffers hold instance b at base + b * vs (the vector layout
// of a single problem, vs >= n_v); the sweep buffers q, xbar [Bp][nn][nx] and
// d, ubar [Bp][nn][nu] likewise, so the node-local passes (pre-pass, post-pass
// with the residual statistics, M) run the single-instance family steps on
// each instance. Bp rounds B up to 16; the extra columns run on zeros.
//
// The host keeps each instance's state machine (Alg. 3: K0, line search with
// K1/K2, KM) and its Anderson ring and solves the Gram systems in FP64 from
// device dot products; the device does every vector operation.
#include "device_common.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

namespace spk {

typedef float shf4 __attribute__((ext_vector_type(4)));
typedef double shd4 __attribute__((ext_vector_type(4)));

// One 16x16x4 step D = A B + C on a wavefront. Lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; register r of lane l holds D[row(l / 16, r)][l % 16]:
// row 4 (l / 16) + r for FP32, (l / 16) + 4 r for FP64 (both measured).
template <typename S>
struct Mfma;
template <>
struct Mfma<float> {
  using acc_t = shf4;
  __device__ static acc_t step(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int kk, int r) { return 4 * kk + r; }
};
template <>
struct Mfma<double> {
  using acc_t = shd4;
  __device__ static acc_t step(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int kk, int r) { return kk + 4 * r; }
};

constexpr int kShCols = 16;   // instances per MFMA tile
constexpr int kShWaves = 16;  // wavefronts per workgroup of the sweeps
constexpr int kShRed = 1024;  // threads of the per-instance reductions

// acc += A[m0 .. m0 + 16)[0 .. nin) X, A input-major (element (out o, in k)
// at k nout + o), X column j (instance) at x + j * xs, element k at +k;
// nin <= 64. The operands of 8 steps (32 inputs) are loaded before their
// MFMAs, so a chain waits for one round of loads per 32 inputs.
template <typename S>
__device__ __forceinline__ void tile_mma(typename Mfma<S>::acc_t& acc, const S* __restrict__ A, int nout, int nin,
                                         int m0, const S* __restrict__ x, long long xs, int lane) {
  const int r = lane & 15, kk = lane >> 4;
  const int m = m0 + r;
  const S* xj = x + (size_t)r * xs;
  for (int k0 = 0; k0 < nin; k0 += 32) {
    S a[8], b[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = k0 + 4 * t + kk;
      const bool in = k < nin;
      a[t] = (in && m < nout) ? A[(size_t)k * nout + m] : S(0);
      b[t] = in ? xj[k] : S(0);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (k0 + 4 * t < nin) acc = Mfma<S>::step(a[t], b[t], acc);
  }
}

template <typename S>
__device__ __forceinline__ typename Mfma<S>::acc_t zero_acc() {
  typename Mfma<S>::acc_t a;
  a[0] = a[1] = a[2] = a[3] = S(0);
  return a;
}

// ---------------------------------------------------------------- T on B instances
// pre-pass of every (family, instance)
template <typename S, int T>
__global__ void __launch_bounds__(256) k_sh_pre(DevProb<S> P, const S* __restrict__ v, S* __restrict__ Tv,
                                                S* __restrict__ xbar, S* __restrict__ ubar, S* __restrict__ q,
                                                long long vs) {
  const int lane = threadIdx.x % T;
  const int f = blockIdx.x * (blockDim.x / T) + threadIdx.x / T;
  if (f >= P.nl) return;
  const size_t b = blockIdx.y;
  const long long wx = (long long)P.nn * P.nx, wu = (long long)P.nn * P.nu;
  const S* z = v + b * vs;
  fam_pre_team<S, T>(P, z, z + P.nz, Tv + b * vs, xbar + b * wx, ubar + b * wu, q + b * wx, f, lane);
}

// The sweeps of Alg. 2 for 16 instances per workgroup, workgroup barriers
// between stages. The work of a stage is split into (node, 16-row tile)
// items spread over the wavefronts: backward, the tiles of d^i and of q^i
// (independent given the children's q); forward, the tiles of u^i and of
// every child's x^c (independent given x^i and d^i). Backward (one mat-vec
// phase): d^i = R~^{-1} ubar^i + sum_c Bt^c q^c, q^i = P1 ubar^i - xbar^i +
// sum_c At^c q^c. Forward: u^i = K x^i + d^i, x^c = Abar^c x^i + B^c d^i.
//
// Phases (one launch each): kShWhole walks every stage, one workgroup per
// 16-instance tile group. With a cut stage tc, the subtrees rooted at stage
// tc are independent: kShBwdSub runs one workgroup per (tile group,
// subtree) over the subtree's stages bottom-up, kShBwdTop the stages above
// tc, kShFwdTop the root state and the stages above tc, kShFwdSub the
// subtrees top-down; so more compute units share the wide stages.
constexpr int kShWhole = 0, kShBwdSub = 1, kShBwdTop = 2, kShFwdTop = 3, kShFwdSub = 4;
constexpr int kShMaxLevels = 128;  // subtree levels a workgroup keeps in LDS

struct ShSweepArgs {
  int maxch, phase, tc, nsub;  // nsub: subtrees (nodes of stage tc) per tile group
};

template <typename S>
__device__ __forceinline__ void sh_bwd_nodes(const DevProb<S>& P, int i0, int i1, S* q0, S* d0, const S* xb0,
                                             const S* ub0, long long wx, long long wu, int lane, int wave) {
  using acc_t = typename Mfma<S>::acc_t;
  const int col = lane & 15, kk = lane >> 4;
  const int nx = P.nx, nu = P.nu;
  const int tu = (nu + 15) / 16, tx = (nx + 15) / 16;
  const int items = (i1 - i0) * (tu + tx);
  for (int it = wave; it < items; it += kShWaves) {
    const int i = i0 + it / (tu + tx), sub = it % (tu + tx);
    const int fc = P.fc[i], n = P.nch[i];
    acc_t acc = zero_acc<S>();
    if (sub < tu) {  // d^i, rows 16 sub ..
      const int m0 = 16 * sub;
      tile_mma<S>(acc, P.Rinv + (size_t)i * nu * nu, nu, nu, m0, ub0 + (size_t)i * nu, wu, lane);
      for (int k = 0; k < n; ++k)
        tile_mma<S>(acc, P.BtR + (size_t)(fc + k) * nx * nu, nu, nx, m0, q0 + (size_t)(fc + k) * nx, wx, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + Mfma<S>::row(kk, r);
        if (m < nu) d0[(size_t)col * wu + (size_t)i * nu + m] = acc[r];
      }
    } else {  // q^i
      const int m0 = 16 * (sub - tu);
      tile_mma<S>(acc, P.P1C + (size_t)i * nu * nx, nx, nu, m0, ub0 + (size_t)i * nu, wu, lane);
      for (int k = 0; k < n; ++k)
        tile_mma<S>(acc, P.AtR + (size_t)(fc + k) * nx * nx, nx, nx, m0, q0 + (size_t)(fc + k) * nx, wx, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + Mfma<S>::row(kk, r);
        if (m < nx) {
          const size_t e = (size_t)col * wx + (size_t)i * nx + m;
          q0[e] = acc[r] - xb0[e];
        }
      }
    }
  }
}

template <typename S>
__device__ __forceinline__ void sh_fwd_nodes(const DevProb<S>& P, int i0, int i1, S* z0, const S* d0, long long vs,
                                             long long wu, int maxch, int lane, int wave) {
  using acc_t = typename Mfma<S>::acc_t;
  const int col = lane & 15, kk = lane >> 4;
  const int nx = P.nx, nu = P.nu;
  const int tu = (nu + 15) / 16, tx = (nx + 15) / 16;
  const Off<S> O(P);
  const int per = tu + maxch * tx;
  const int items = (i1 - i0) * per;
  for (int it = wave; it < items; it += kShWaves) {
    const int i = i0 + it / per, sub = it % per;
    const int fc = P.fc[i], n = P.nch[i];
    const S* xi = z0 + O.x(i);
    const S* di = d0 + (size_t)i * nu;
    acc_t acc = zero_acc<S>();
    if (sub < tu) {  // u^i
      const int m0 = 16 * sub;
      tile_mma<S>(acc, P.KC + (size_t)i * nx * nu, nu, nx, m0, xi, vs, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + Mfma<S>::row(kk, r);
        if (m < nu) z0[(size_t)col * vs + O.u(i) + m] = acc[r] + di[(size_t)col * wu + m];
      }
    } else {  // x^c of child k
      const int k = (sub - tu) / tx, m0 = 16 * ((sub - tu) % tx);
      if (k >= n) continue;
      const int c = fc + k;
      tile_mma<S>(acc, P.AbC + (size_t)c * nx * nx, nx, nx, m0, xi, vs, lane);
      tile_mma<S>(acc, P.BC + (size_t)c * nu * nx, nx, nu, m0, di, wu, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + Mfma<S>::row(kk, r);
        if (m < nx) z0[(size_t)col * vs + O.x(c) + m] = acc[r];
      }
    }
  }
}

template <typename S>
__global__ void __launch_bounds__(64 * kShWaves) k_sh_sweeps(DevProb<S> P, const int* __restrict__ stage_off,
                                                              S* __restrict__ Tv, const double* __restrict__ x0s,
                                                              S* __restrict__ xbar, S* __restrict__ ubar,
                                                              S* __restrict__ q, S* __restrict__ d, long long vs,
                                                              ShSweepArgs A) {
  __shared__ int lo[kShMaxLevels], hi[kShMaxLevels];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool sub = A.phase == kShBwdSub || A.phase == kShFwdSub;
  const int g = sub ? blockIdx.x / A.nsub : blockIdx.x;  // tile group
  const size_t b0 = (size_t)g * kShCols;
  const int nx = P.nx, nu = P.nu;
  const long long wx = (long long)P.nn * nx, wu = (long long)P.nn * nu;
  const Off<S> O(P);
  S* q0 = q + b0 * wx;
  S* d0 = d + b0 * wu;
  const S* xb0 = xbar + b0 * wx;
  const S* ub0 = ubar + b0 * wu;
  S* z0 = Tv + b0 * vs;
  if (sub) {
    // node ranges of the subtree rooted at node stage_off[tc] + r, one per
    // nonleaf stage tc .. N-1
    const int r = blockIdx.x % A.nsub;
    const int levels = P.N - A.tc;
    if (threadIdx.x == 0) {
      lo[0] = stage_off[A.tc] + r;
      hi[0] = lo[0] + 1;
      for (int l = 1; l < levels; ++l) {
        lo[l] = P.fc[lo[l - 1]];
        hi[l] = P.fc[hi[l - 1] - 1] + P.nch[hi[l - 1] - 1];
      }
    }
    __syncthreads();
    if (A.phase == kShBwdSub) {
      for (int l = levels - 1; l >= 0; --l) {
        sh_bwd_nodes<S>(P, lo[l], hi[l], q0, d0, xb0, ub0, wx, wu, lane, wave);
        __syncthreads();
      }
    } else {
      for (int l = 0; l < levels; ++l) {
        sh_fwd_nodes<S>(P, lo[l], hi[l], z0, d0, vs, wu, A.maxch, lane, wave);
        __syncthreads();
      }
    }
    return;
  }
  const int tb = A.phase == kShWhole ? P.N : A.tc;  // stages [0, tb) here
  if (A.phase == kShWhole || A.phase == kShBwdTop) {
    for (int t = tb - 1; t >= 0; --t) {
      sh_bwd_nodes<S>(P, stage_off[t], stage_off[t + 1], q0, d0, xb0, ub0, wx, wu, lane, wave);
      __syncthreads();
    }
  }
  if (A.phase == kShWhole || A.phase == kShFwdTop) {
    // root state of every instance
    for (int e = threadIdx.x; e < kShCols * nx; e += blockDim.x) {
      const int j = e / nx, o = e % nx;
      z0[(size_t)j * vs + O.x(0) + o] = (S)x0s[(b0 + j) * nx + o];
    }
    __syncthreads();
    for (int t = 0; t < tb; ++t) {
      sh_fwd_nodes<S>(P, stage_off[t], stage_off[t + 1], z0, d0, vs, wu, A.maxch, lane, wave);
      __syncthreads();
    }
  }
}

// post-pass of every (family, instance): dual update and the instance's
// residual statistics (block records at partials + b * gridDim.x * kStats)
template <typename S, int T>
__global__ void __launch_bounds__(256) k_sh_post(DevProb<S> P, const S* __restrict__ v, S* __restrict__ Tv,
                                                 long long vs, int VM, double* __restrict__ partials) {
  extern __shared__ unsigned char smem_raw[];
  S* smem = reinterpret_cast<S*>(smem_raw);
  const int lane = threadIdx.x % T;
  const int team = threadIdx.x / T;
  const int f = blockIdx.x * (blockDim.x / T) + team;
  const size_t b = blockIdx.y;
  const S* z = v + b * vs;
  S* zo = Tv + b * vs;
  StatAcc st;
  if (f < P.nl) fam_post_team<S, T>(P, z, z + P.nz, zo, zo + P.nz, f, lane, smem + (size_t)team * 3 * VM, VM, st);
  block_stats(st, partials + b * gridDim.x * kStats);
}

// Statistics of instance blockIdx.x from its nblk records (fixed order):
// out[b][0..5] = xi_p, xi_d, omega^2, |r_z|^2, |r_eta|^2, <r_eta, L r_z>.
__global__ void __launch_bounds__(256) k_sh_stats(const double* __restrict__ partials, int nblk, double alpha,
                                                  double* __restrict__ out) {
  __shared__ double red[kStats][256];
  const double* p0 = partials + (size_t)blockIdx.x * nblk * kStats;
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    const double* p = p0 + (size_t)k * kStats;
    a0 += p[0];
    a1 += p[1];
    a2 += p[2];
    a3 = fmax(a3, p[3]);
    a4 = fmax(a4, p[4]);
  }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  red[2][threadIdx.x] = a2;
  red[3][threadIdx.x] = a3;
  red[4][threadIdx.x] = a4;
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
  if (threadIdx.x == 0) {
    double* o = out + (size_t)blockIdx.x * 8;
    o[0] = red[3][0];
    o[1] = red[4][0];
    o[2] = red[0][0] + red[1][0] - 2.0 * alpha * red[2][0];
    o[3] = red[0][0];
    o[4] = red[1][0];
    o[5] = red[2][0];
  }
}

// Fixed-order sum of K per-thread values over the workgroup (wavefront
// butterflies, then the wavefront sums in order); the result in red[j][0].
template <int K>
__device__ __forceinline__ void sh_block_sums(double (&acc)[K], double (*red)[kShRed / 64]) {
#pragma unroll
  for (int j = 0; j < K; ++j)
    for (int o = 32; o >= 1; o >>= 1) acc[j] += __shfl_xor(acc[j], o, 64);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int j = 0; j < K; ++j) red[j][w] = acc[j];
  __syncthreads();
  if ((int)threadIdx.x < K) {
    double s = 0;
    for (int k = 0; k < nw; ++k) s += red[threadIdx.x][k];
    red[threadIdx.x][0] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- vector steps
// Buffers of the engine, each [Bp][vs]: the roles of the single-instance
// solver (one copy per instance, no role swaps: accepted points are copied).
template <typename S>
struct ShVec {
  S* v;     // iterate
  S* tv;    // T(v)
  S* vprev; // previous iterate
  S* rprev; // previous residual
  S* rcur;  // residual v - T(v)
  S* dir;   // direction
  S* md;    // M dir
  S* vt;    // point of the next evaluation
  S* tvt;   // T(vt)
  S* spare; // v + dir
  S* E;     // Anderson columns dV - dR, slot s at E + s * Bp * vs
  S* R;     // Anderson columns dR, slot s at R + s * Bp * vs
  long long vs, nv, slot;  // instance stride, vector length, slot stride
};

// vt = c0 v + c1 dir + c2 vt + c3 tvt + c4 rcur + c5 spare + c6 tv for the
// instances with mask[b] (coefficients c[b][0..6], zero terms skipped)
template <typename S>
__global__ void __launch_bounds__(256) k_sh_cand(ShVec<S> V, const double* __restrict__ coef,
                                                 const int* __restrict__ mask) {
  const size_t b = blockIdx.y;
  if (!mask[b]) return;
  const double* c = coef + b * 8;
  const size_t o = b * V.vs;
  const S* src[7] = {V.v + o, V.dir + o, V.vt + o, V.tvt + o, V.rcur + o, V.spare + o, V.tv + o};
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < V.nv; e += (long long)gridDim.x * blockDim.x) {
    double acc = 0;
#pragma unroll
    for (int j = 0; j < 7; ++j)
      if (c[j] != 0.0) acc += c[j] * (double)src[j][e];
    V.vt[o + e] = (S)acc;
  }
}

// Accepting the evaluated point: mode 1 v = vt, tv = tvt; mode 2 also
// vprev = v, rprev = rcur first (the ring of Alg. 3's accepted iterates).
template <typename S>
__global__ void __launch_bounds__(256) k_sh_commit(ShVec<S> V, const int* __restrict__ mode) {
  const size_t b = blockIdx.y;
  const int md = mode[b];
  if (md == 0) return;
  const size_t o = b * V.vs;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < V.nv; e += (long long)gridDim.x * blockDim.x) {
    const size_t k = o + e;
    if (md == 2) {
      V.vprev[k] = V.v[k];
      V.rprev[k] = V.rcur[k];
    }
    V.v[k] = V.vt[k];
    V.tv[k] = V.tvt[k];
  }
}

// Residual r = v - T(v) of the accepted point (mode >= 1); with mode 2 the
// Anderson push: dR = r - rprev into slot ns, E = (v - vprev) - dR, and the
// dot products dots[b][s] = <dR_s, dR>, dots[b][kAAMax + s] = <dR_s, r> for
// s < m (the new slot's own column included). One workgroup per instance.
template <typename S>
__global__ void __launch_bounds__(kShRed) k_sh_push(ShVec<S> V, const int* __restrict__ mode, const int* __restrict__ ns,
                                                    int m, double* __restrict__ dots) {
  __shared__ double red[2 * kAAMax][kShRed / 64];
  const size_t b = blockIdx.x;
  const int md = mode[b];
  if (md == 0) return;
  const size_t o = b * V.vs;
  const int slot = ns[b];
  double acc[2 * kAAMax];
#pragma unroll
  for (int j = 0; j < 2 * kAAMax; ++j) acc[j] = 0;
  for (long long e = threadIdx.x; e < V.nv; e += blockDim.x) {
    const size_t k = o + e;
    const S vv = V.v[k];
    const S r = vv - V.tv[k];
    V.rcur[k] = r;
    if (md == 2) {
      const S dr = r - V.rprev[k];
      V.R[(size_t)slot * V.slot + k] = dr;
      V.E[(size_t)slot * V.slot + k] = (S)(((double)vv - (double)V.vprev[k]) - (double)dr);
#pragma unroll
      for (int s = 0; s < kAAMax; ++s)
        if (s < m) {
          const double ds = (s == slot) ? (double)dr : (double)V.R[(size_t)s * V.slot + k];
          acc[s] += ds * (double)dr;
          acc[kAAMax + s] += ds * (double)r;
        }
    }
  }
  if (md != 2) return;  // uniform over the workgroup
  sh_block_sums<2 * kAAMax>(acc, red);
  if ((int)threadIdx.x < 2 * kAAMax) dots[b * 2 * kAAMax + threadIdx.x] = red[threadIdx.x][0];
}

// dir = -r - sum_s gamma[b][s] E_s, spare = v + dir (mask[b])
template <typename S>
__global__ void __launch_bounds__(256) k_sh_dir(ShVec<S> V, const double* __restrict__ gamma,
                                                const int* __restrict__ mask) {
  const size_t b = blockIdx.y;
  if (!mask[b]) return;
  const size_t o = b * V.vs;
  const double* g = gamma + b * kAAMax;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < V.nv; e += (long long)gridDim.x * blockDim.x) {
    const size_t k = o + e;
    double acc = -(double)V.rcur[k];
#pragma unroll
    for (int s = 0; s < kAAMax; ++s)
      if (g[s] != 0.0) acc -= g[s] * (double)V.E[(size_t)s * V.slot + k];
    V.dir[k] = (S)acc;
    V.spare[k] = (S)((double)V.v[k] + acc);
  }
}

// md = M dir (mask[b]), one team of T lanes per family
template <typename S, int T>
__global__ void __launch_bounds__(256) k_sh_M(DevProb<S> P, ShVec<S> V, const int* __restrict__ mask) {
  const size_t b = blockIdx.y;
  if (!mask[b]) return;
  const int lane = threadIdx.x % T;
  const int i = blockIdx.x * (blockDim.x / T) + threadIdx.x / T;
  if (i >= P.nl) return;
  fam_apply_M<S, T>(P, V.dir + b * V.vs, V.md + b * V.vs, i, lane);
}

// out[b] = <vt - tvt, md> (mask[b]), one workgroup per instance
template <typename S>
__global__ void __launch_bounds__(kShRed) k_sh_rdot(ShVec<S> V, const int* __restrict__ mask, double* __restrict__ out) {
  __shared__ double red[1][kShRed / 64];
  const size_t b = blockIdx.x;
  if (!mask[b]) return;
  const size_t o = b * V.vs;
  double acc[1] = {0};
  for (long long e = threadIdx.x; e < V.nv; e += blockDim.x)
    acc[0] += ((double)V.vt[o + e] - (double)V.tvt[o + e]) * (double)V.md[o + e];
  sh_block_sums<1>(acc, red);
  if (threadIdx.x == 0) out[b] = red[0][0];
}

// ---------------------------------------------------------------- host engine
namespace {

enum ShPhase { kShInit, kShK0, kShLS, kShK2, kShKM, kShCP, kShDone };

struct ShStats {
  double xip = 0, xid = 0, om2 = 0;
  double xi() const { return std::max(xip, xid); }
  double omega() const { return std::sqrt(std::max(om2, 0.0)); }
  bool ok() const { return std::isfinite(xip) && std::isfinite(xid) && std::isfinite(om2); }
};

// Anderson ring of one instance, the same rules as the single-instance
// device ring: the new column takes the oldest slot when m columns are kept,
// else the lowest free slot; the oldest columns are dropped until the Gram
// matrix of the rest passes the rank test (lambda_min / lambda_max >= 1e-12,
// cyclic Jacobi until decided) and has a Cholesky factor.
struct ShRing {
  int m = 1, cnt = 0, order[kAAMax] = {0, 0, 0, 0};
  double G[kAAMax][kAAMax] = {};
  int slot = 0, mo = 0, order_old[kAAMax] = {0, 0, 0, 0};

  void begin_push() {
    const bool full = cnt == m;
    mo = full ? cnt - 1 : cnt;
    for (int j = 0; j < kAAMax; ++j) order_old[j] = full ? (j + 1 < kAAMax ? order[j + 1] : 0) : order[j];
    int fr = kAAMax;
    for (int s = kAAMax - 1; s >= 0; --s) {
      bool used = false;
      for (int j = 0; j < cnt; ++j) used = used || order[j] == s;
      if (!used && s < m) fr = s;
    }
    slot = full ? order[0] : fr;
  }

  static bool rank_ok(int n, double A[kAAMax][kAAMax]) {
    const double kTol = 1e-12;
    for (int sweep = 0;; ++sweep) {
      double off = 0, dmin = A[0][0], dmax = A[0][0];
      for (int i = 0; i < n; ++i) {
        dmin = std::min(dmin, A[i][i]);
        dmax = std::max(dmax, A[i][i]);
        for (int j = i + 1; j < n; ++j) off += A[i][j] * A[i][j];
      }
      const double e = std::sqrt(2.0 * off);
      if (dmax - e > 0.0 && dmin - e >= kTol * (dmax + e)) return true;
      if (dmax + e <= 0.0 || (dmax - e > 0.0 && dmin + e < kTol * (dmax - e))) return false;
      if (sweep == 60 || off < 1e-300) return dmax > 0.0 && dmin >= kTol * dmax;
      for (int p = 0; p < n; ++p)
        for (int q = p + 1; q < n; ++q) {
          const double apq = A[p][q];
          if (apq == 0.0) continue;
          const double th = 0.5 * (A[q][q] - A[p][p]) / apq;
          const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
          const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
          for (int k = 0; k < n; ++k) {
            const double akp = A[k][p], akq = A[k][q];
            A[k][p] = c * akp - s * akq;
            A[k][q] = s * akp + c * akq;
          }
          for (int k = 0; k < n; ++k) {
            const double apk = A[p][k], aqk = A[q][k];
            A[p][k] = c * apk - s * aqk;
            A[q][k] = s * apk + c * aqk;
          }
        }
    }
  }

  static bool chol(int n, double L[kAAMax][kAAMax]) {
    for (int j = 0; j < n; ++j) {
      double d = L[j][j];
      for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
      if (!(d > 0.0) || !std::isfinite(d)) return false;
      d = std::sqrt(d);
      L[j][j] = d;
      for (int i = j + 1; i < n; ++i) {
        double s = L[i][j];
        for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
        L[i][j] = s / d;
      }
    }
    return true;
  }

  // dots as written by k_sh_push; gamma by slot (0 for unused or dropped)
  void solve(const double* dots, double* gamma_by_slot) {
    for (int j = 0; j < mo; ++j) {
      G[order_old[j]][slot] = dots[order_old[j]];
      G[slot][order_old[j]] = dots[order_old[j]];
    }
    G[slot][slot] = dots[slot];
    const int k = mo + 1;
    int ord[kAAMax];
    for (int j = 0; j < mo; ++j) ord[j] = order_old[j];
    ord[mo] = slot;
    double rk[kAAMax];
    for (int j = 0; j < k; ++j) rk[j] = dots[kAAMax + ord[j]];
    double g[kAAMax] = {0, 0, 0, 0};
    int kept = 0;
    for (int drop = 0; drop < k && kept == 0; ++drop) {
      const int n = k - drop;
      double E[kAAMax][kAAMax], L[kAAMax][kAAMax];
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) E[i][j] = L[i][j] = G[ord[drop + i]][ord[drop + j]];
      if (!rank_ok(n, E) || !chol(n, L)) continue;
      double y[kAAMax];
      for (int i = 0; i < n; ++i) {
        double s = rk[drop + i];
        for (int j = 0; j < i; ++j) s -= L[i][j] * y[j];
        y[i] = s / L[i][i];
      }
      for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int j = i + 1; j < n; ++j) s -= L[j][i] * g[drop + j];
        g[drop + i] = s / L[i][i];
      }
      kept = n;
    }
    for (int s = 0; s < kAAMax; ++s) gamma_by_slot[s] = 0.0;
    for (int j = 0; j < k; ++j) gamma_by_slot[ord[j]] = g[j];
    cnt = kept;
    for (int j = 0; j < kept; ++j) order[j] = ord[k - kept + j];
  }
};

struct ShInst {
  int phase = kShDone;
  bool active = false, have_prev = false;
  double tol = 0, zeta = 0, omega_safe = 0, omega = 0, tau = 1;
  int k = 0, ls = 0;
  ShStats Sc;
  ShRing ring;
  spock_info info{};
};

// Device workspace of the engine (kept between calls, not thread safe).
struct ShCache {
  void* mem = nullptr;
  size_t bytes = 0;
  void* host = nullptr;  // pinned staging (parameters up, results down)
  size_t host_bytes = 0;
};
ShCache& sh_cache() {
  static ShCache c;
  return c;
}

template <typename S>
const DevProb<S>& sh_dev(const Problem& P);
template <>
const DevProb<double>& sh_dev<double>(const Problem& P) { return P.dp64; }
template <>
const DevProb<float>& sh_dev<float>(const Problem& P) { return P.dp32; }

#define SH_TRY(x)                             \
  do {                                        \
    if ((x) != hipSuccess) return SPOCK_EHIP; \
  } while (0)

template <typename S, int T>
void sh_launch_post(const Problem& P, const DevProb<S>& D, const ShVec<S>& V, double* partials, int Bp,
                    hipStream_t st) {
  const int tpb = 256 / T;
  const int VM = (std::max(P.nx, P.nu) + 3) & ~3;
  const dim3 grid((P.tree->nl + tpb - 1) / tpb, Bp);
  hipLaunchKernelGGL((k_sh_post<S, T>), grid, dim3(256), (size_t)tpb * 3 * VM * sizeof(S), st, D, V.vt, V.tvt, V.vs,
                     VM, partials);
}

template <typename S, int T>
void sh_launch_pre(const Problem& P, const DevProb<S>& D, const ShVec<S>& V, S* xbar, S* ubar, S* q, int Bp,
                   hipStream_t st) {
  const int tpb = 256 / T;
  const dim3 grid((P.tree->nl + tpb - 1) / tpb, Bp);
  hipLaunchKernelGGL((k_sh_pre<S, T>), grid, dim3(256), 0, st, D, V.vt, V.tvt, xbar, ubar, q, V.vs);
}

template <typename S, int T>
void sh_launch_M(const Problem& P, const DevProb<S>& D, const ShVec<S>& V, const int* mask, int Bp, hipStream_t st) {
  const int tpb = 256 / T;
  const dim3 grid((P.tree->nl + tpb - 1) / tpb, Bp);
  hipLaunchKernelGGL((k_sh_M<S, T>), grid, dim3(256), 0, st, D, V, mask);
}

}  // namespace

template <typename S>
int shared_solve(Problem& P, int B, const double* const* x0, const spock_settings& s, void* const* vio,
                 spock_info* infos, hipStream_t st) {
  const Tree& Tr = *P.tree;
  const DevProb<S>& D = sh_dev<S>(P);
  const int nx = P.nx, nu = P.nu, T = P.team_pp;
  const long long nv = P.nz + P.neta;
  const long long vs = (nv + 63) & ~63LL;
  const int Bp = (B + kShCols - 1) / kShCols * kShCols;
  const int tpb = 256 / T;
  const int nblk = (Tr.nl + tpb - 1) / tpb;
  const size_t nvec = (size_t)Bp * vs;
  // device layout
  size_t off = 0;
  auto reserve = [&](size_t b) {
    const size_t o = off;
    off += (b + 255) & ~size_t(255);
    return o;
  };
  const size_t o_vec = reserve(sizeof(S) * nvec * (10 + 2 * kAAMax));
  const size_t o_qx = reserve(sizeof(S) * (size_t)Bp * Tr.nn * nx * 2);
  const size_t o_du = reserve(sizeof(S) * (size_t)Bp * Tr.nn * nu * 2);
  const size_t o_x0 = reserve(sizeof(double) * (size_t)Bp * nx);
  const size_t o_part = reserve(sizeof(double) * (size_t)Bp * nblk * kStats);
  const size_t o_res = reserve(sizeof(double) * (size_t)Bp * (8 + 1 + 2 * kAAMax));  // stats, rdot, dots
  // parameters of the steps of a round, one staging slot per step (the host
  // writes a slot only after the previous round's synchronisation, so no
  // queued copy reads a slot the host is changing): coefficients [Bp][8],
  // gamma [Bp][kAAMax], then int arrays mask, mode, slot [Bp]
  const size_t par_bytes = ((sizeof(double) * (size_t)Bp * (8 + kAAMax) + sizeof(int) * (size_t)Bp * 3) + 255) & ~size_t(255);
  enum { kParRdot, kParCommit, kParPush, kParDir, kParCand, kParSlots };
  const size_t o_par = reserve(par_bytes * kParSlots);
  ShCache& C = sh_cache();
  if (C.bytes < off) {
    if (C.mem) (void)hipFree(C.mem);
    C.mem = nullptr;
    C.bytes = 0;
    if (hipMalloc(&C.mem, off) != hipSuccess) return SPOCK_ENOMEM;
    C.bytes = off;
  }
  const size_t res_bytes = ((sizeof(double) * (size_t)Bp * (8 + 1 + 2 * kAAMax)) + 255) & ~size_t(255);
  const size_t hbytes = res_bytes + par_bytes * kParSlots;
  if (C.host_bytes < hbytes) {
    if (C.host) (void)hipHostFree(C.host);
    C.host = nullptr;
    C.host_bytes = 0;
    if (hipHostMalloc(&C.host, hbytes, 0) != hipSuccess) return SPOCK_ENOMEM;
    C.host_bytes = hbytes;
  }
  char* base = static_cast<char*>(C.mem);
  // every vector starts at zero (padding instances stay at zero)
  SH_TRY(hipMemsetAsync(base, 0, off, st));
  ShVec<S> V{};
  S* vb = reinterpret_cast<S*>(base + o_vec);
  S** roles[10] = {&V.v, &V.tv, &V.vprev, &V.rprev, &V.rcur, &V.dir, &V.md, &V.vt, &V.tvt, &V.spare};
  for (int r = 0; r < 10; ++r) *roles[r] = vb + (size_t)r * nvec;
  V.E = vb + (size_t)10 * nvec;
  V.R = V.E + (size_t)kAAMax * nvec;
  V.vs = vs;
  V.nv = nv;
  V.slot = (long long)nvec;
  S* qx = reinterpret_cast<S*>(base + o_qx);
  S* q = qx;
  S* xbar = qx + (size_t)Bp * Tr.nn * nx;
  S* du = reinterpret_cast<S*>(base + o_du);
  S* d = du;
  S* ubar = du + (size_t)Bp * Tr.nn * nu;
  double* x0s = reinterpret_cast<double*>(base + o_x0);
  double* partials = reinterpret_cast<double*>(base + o_part);
  double* res = reinterpret_cast<double*>(base + o_res);
  double* stats_d = res;                        // [Bp][8]
  double* rdot_d = res + (size_t)Bp * 8;        // [Bp]
  double* dots_d = rdot_d + Bp;                 // [Bp][2 kAAMax]
  char* par_d = base + o_par;
  // host staging: results, then the parameter slots
  double* hres = static_cast<double*>(C.host);
  double* hstats = hres;
  double* hrdot = hres + (size_t)Bp * 8;
  double* hdots = hrdot + Bp;
  char* par_h = static_cast<char*>(C.host) + res_bytes;
  struct Par {
    double* coef;
    double* gamma;
    int* mask;
    int* mode;
    int* slot;
  };
  auto par_at = [&](char* base_p, int k) {
    char* p = base_p + (size_t)k * par_bytes;
    Par r;
    r.coef = reinterpret_cast<double*>(p);
    r.gamma = r.coef + (size_t)Bp * 8;
    r.mask = reinterpret_cast<int*>(r.gamma + (size_t)Bp * kAAMax);
    r.mode = r.mask + Bp;
    r.slot = r.mode + Bp;
    return r;
  };
  auto clear = [&](int k) { std::memset(par_h + (size_t)k * par_bytes, 0, par_bytes); };
  auto upload = [&](int k) -> int {
    SH_TRY(hipMemcpyAsync(par_d + (size_t)k * par_bytes, par_h + (size_t)k * par_bytes, par_bytes,
                          hipMemcpyHostToDevice, st));
    return SPOCK_OK;
  };
  const dim3 vgrid((unsigned)std::min<long long>((nv + 255) / 256, 64), Bp);

  // instances: x0 in the root box, warm start into vt
  std::vector<ShInst> I(Bp);
  std::vector<double> hx(nx);
  for (int b = 0; b < B; ++b) {
    ShInst& in = I[b];
    in.info = spock_info{};
    in.info.mapping = kTeamShared;
    in.info.V_nested = std::nan("");
    SH_TRY(hipMemcpyAsync(hx.data(), x0[b], sizeof(double) * nx, hipMemcpyDeviceToHost, st));
    SH_TRY(hipStreamSynchronize(st));
    bool inside = true;
    for (int o = 0; o < nx; ++o) inside = inside && hx[o] >= P.xlo0[o] && hx[o] <= P.xhi0[o];
    if (!inside) {
      in.info.status = SPOCK_REJECTED;
      continue;
    }
    SH_TRY(hipMemcpyAsync(x0s + (size_t)b * nx, x0[b], sizeof(double) * nx, hipMemcpyDeviceToDevice, st));
    SH_TRY(hipMemcpyAsync(V.vt + (size_t)b * vs, vio[b], sizeof(S) * nv, hipMemcpyDeviceToDevice, st));
    in.active = true;
    in.phase = kShInit;
    in.ring.m = s.m;
  }
  const bool cp = s.method == SPOCK_METHOD_CP;
  auto finish = [&](int b, int status) -> int {
    ShInst& in = I[b];
    in.info.status = status;
    in.info.iters = in.k;
    in.info.xi = in.Sc.xi();
    in.active = false;
    in.phase = kShDone;
    SH_TRY(hipMemcpyAsync(vio[b], V.tv + (size_t)b * vs, sizeof(S) * nv, hipMemcpyDeviceToDevice, st));
    return SPOCK_OK;
  };
  auto any_active = [&]() {
    for (int b = 0; b < B; ++b)
      if (I[b].active) return true;
    return false;
  };
  enum { cV = 0, cDIR = 1, cVT = 2, cTVT = 3, cRCUR = 4, cSPARE = 5, cTV = 6 };
  auto set_cand = [&](int b, std::initializer_list<std::pair<int, double>> terms) {
    const Par c = par_at(par_h, kParCand);
    for (int j = 0; j < 8; ++j) c.coef[(size_t)b * 8 + j] = 0.0;
    for (auto& t : terms) c.coef[(size_t)b * 8 + t.first] += t.second;
    c.mask[b] = 1;
  };
  const Par hp_rdot = par_at(par_h, kParRdot), dp_rdot = par_at(par_d, kParRdot);
  const Par hp_com = par_at(par_h, kParCommit), dp_com = par_at(par_d, kParCommit);
  const Par hp_push = par_at(par_h, kParPush), dp_push = par_at(par_d, kParPush);
  const Par hp_dir = par_at(par_h, kParDir), dp_dir = par_at(par_d, kParDir);
  const Par dp_cand = par_at(par_d, kParCand);
  const int sweep_grid = Bp / kShCols;
  int maxch = 1;
  for (int i = 0; i < Tr.nl; ++i) maxch = std::max(maxch, Tr.nch[i]);
  // cut stage of the sweeps: the first stage with at least 8 nodes, if it
  // has nonleaf stages below it (at most kShMaxLevels) and is not the root
  // stage; SPOCK_SH_CUT overrides (0: one launch over the whole tree)
  int sh_cut = 0;
  for (int t = 1; t < Tr.N; ++t)
    if (Tr.stage_off[t + 1] - Tr.stage_off[t] >= 8) {
      sh_cut = t;
      break;
    }
  if (const char* env = std::getenv("SPOCK_SH_CUT")) sh_cut = std::atoi(env);
  if (sh_cut < 1 || sh_cut >= Tr.N || Tr.N - sh_cut > kShMaxLevels) sh_cut = 0;
  std::vector<char> prep(Bp), head(Bp);
  while (any_active()) {
    // ---- one evaluation of T at vt for every instance
    switch (T) {
      case 8: sh_launch_pre<S, 8>(P, D, V, xbar, ubar, q, Bp, st); break;
      case 16: sh_launch_pre<S, 16>(P, D, V, xbar, ubar, q, Bp, st); break;
      case 32: sh_launch_pre<S, 32>(P, D, V, xbar, ubar, q, Bp, st); break;
      default: sh_launch_pre<S, 64>(P, D, V, xbar, ubar, q, Bp, st); break;
    }
    if (sh_cut > 0) {
      const int nsub = Tr.stage_off[sh_cut + 1] - Tr.stage_off[sh_cut];
      for (int ph : {kShBwdSub, kShBwdTop, kShFwdTop, kShFwdSub}) {
        const ShSweepArgs A{maxch, ph, sh_cut, nsub};
        const bool subph = ph == kShBwdSub || ph == kShFwdSub;
        hipLaunchKernelGGL(k_sh_sweeps<S>, dim3(subph ? sweep_grid * nsub : sweep_grid), dim3(64 * kShWaves), 0, st,
                           D, P.d_stage_off, V.tvt, x0s, xbar, ubar, q, d, vs, A);
      }
    } else {
      const ShSweepArgs A{maxch, kShWhole, 0, 1};
      hipLaunchKernelGGL(k_sh_sweeps<S>, dim3(sweep_grid), dim3(64 * kShWaves), 0, st, D, P.d_stage_off, V.tvt, x0s,
                         xbar, ubar, q, d, vs, A);
    }
    switch (T) {
      case 8: sh_launch_post<S, 8>(P, D, V, partials, Bp, st); break;
      case 16: sh_launch_post<S, 16>(P, D, V, partials, Bp, st); break;
      case 32: sh_launch_post<S, 32>(P, D, V, partials, Bp, st); break;
      default: sh_launch_post<S, 64>(P, D, V, partials, Bp, st); break;
    }
    hipLaunchKernelGGL(k_sh_stats, dim3(Bp), dim3(256), 0, st, partials, nblk, P.alpha, stats_d);
    // <vt - T(vt), M d> of the instances in a line search
    clear(kParRdot);
    bool any_ls = false;
    for (int b = 0; b < B; ++b)
      if (I[b].active && I[b].phase == kShLS) any_ls = hp_rdot.mask[b] = 1;
    if (any_ls) {
      if (int rc = upload(kParRdot)) return rc;
      hipLaunchKernelGGL(k_sh_rdot<S>, dim3(Bp), dim3(kShRed), 0, st, V, dp_rdot.mask, rdot_d);
    }
    SH_TRY(hipGetLastError());
    SH_TRY(hipMemcpyAsync(hres, res, sizeof(double) * (size_t)Bp * 9, hipMemcpyDeviceToHost, st));
    SH_TRY(hipStreamSynchronize(st));
    // ---- per-instance decisions (Alg. 3)
    clear(kParCommit);
    clear(kParPush);
    clear(kParDir);
    clear(kParCand);
    std::fill(prep.begin(), prep.end(), 0);
    std::fill(head.begin(), head.end(), 0);
    for (int b = 0; b < B; ++b) {
      ShInst& in = I[b];
      if (!in.active) continue;
      ShStats St;
      St.xip = hstats[(size_t)b * 8 + 0];
      St.xid = hstats[(size_t)b * 8 + 1];
      St.om2 = hstats[(size_t)b * 8 + 2];
      in.info.t_evals++;
      switch (in.phase) {
        case kShInit:
          in.Sc = St;
          in.info.xi0 = St.xi();
          in.tol = std::max(s.eps_abs, s.eps_rel * in.info.xi0);
          in.zeta = in.omega_safe = St.omega();
          hp_com.mode[b] = 1;
          if (!St.ok()) {
            in.phase = kShDone;  // returned after the commit below
            in.info.status = SPOCK_NUMERICAL;
          } else if (cp) {
            head[b] = 1;
          } else {
            prep[b] = 1;
          }
          break;
        case kShCP:
          hp_com.mode[b] = 1;
          in.Sc = St;
          ++in.k;
          if (!St.ok()) {
            in.phase = kShDone;
            in.info.status = SPOCK_NUMERICAL;
          } else {
            head[b] = 1;
          }
          break;
        case kShK0:
        case kShK2:
        case kShKM:
          hp_com.mode[b] = 2;
          in.have_prev = true;
          in.Sc = St;
          ++in.k;
          if (!St.ok()) {
            in.phase = kShDone;
            in.info.status = SPOCK_NUMERICAL;
          } else {
            prep[b] = 1;
          }
          break;
        case kShLS: {
          bool backtrack = false;
          if (!St.ok()) {
            backtrack = true;
          } else {
            const double om_t = St.omega();
            if (om_t == 0.0 || (in.omega <= in.omega_safe && om_t <= s.c1 * in.omega)) {  // K1
              hp_com.mode[b] = 2;
              in.have_prev = true;
              in.Sc = St;
              in.omega_safe = om_t + std::pow(s.c2, in.k);
              in.info.n_k1++;
              ++in.k;
              prep[b] = 1;
            } else {
              const double rho = om_t * om_t - in.tau * hrdot[b];
              if (rho >= s.sigma * om_t * in.omega) {  // K2: v - c (vt - T vt)
                const double c = s.lambda * rho / (om_t * om_t);
                set_cand(b, {{cV, 1.0}, {cVT, -c}, {cTVT, c}});
                in.info.n_k2++;
                in.phase = kShK2;
              } else {
                backtrack = true;
              }
            }
          }
          if (backtrack) {
            in.tau *= s.beta;
            in.info.n_backtracks++;
            if (++in.ls < s.max_ls) {
              set_cand(b, {{cV, 1.0}, {cDIR, in.tau}});
            } else {  // plain KM step
              set_cand(b, {{cV, 1.0}, {cRCUR, -s.lambda}});
              in.info.n_km++;
              in.phase = kShKM;
            }
          }
          break;
        }
        default:
          break;
      }
    }
    // ---- the push parameters (host state only), then commit and push
    // parameters in one upload (adjacent slots)
    bool any_prep = false, any_push = false;
    for (int b = 0; b < B; ++b) {
      if (!prep[b]) continue;
      ShInst& in = I[b];
      any_prep = true;
      hp_push.mode[b] = in.have_prev ? 2 : 1;
      if (in.have_prev) {
        in.ring.begin_push();
        hp_push.slot[b] = in.ring.slot;
        any_push = true;
      }
      hp_dir.mask[b] = 1;
    }
    static_assert(kParPush == kParCommit + 1, "adjacent staging slots");
    SH_TRY(hipMemcpyAsync(par_d + (size_t)kParCommit * par_bytes, par_h + (size_t)kParCommit * par_bytes,
                          2 * par_bytes, hipMemcpyHostToDevice, st));
    // ---- accept the evaluated points (the K2 and KM candidates above read
    // only rows of instances that commit nothing this round)
    hipLaunchKernelGGL(k_sh_commit<S>, vgrid, dim3(256), 0, st, V, dp_com.mode);
    for (int b = 0; b < B; ++b)  // ended numerically: T of the point reached
      if (I[b].active && I[b].phase == kShDone)
        if (int rc = finish(b, I[b].info.status)) return rc;
    // ---- residual, Anderson push, Gram solve and direction
    if (any_prep) {
      hipLaunchKernelGGL(k_sh_push<S>, dim3(Bp), dim3(kShRed), 0, st, V, dp_push.mode, dp_push.slot, s.m, dots_d);
      if (any_push) {
        SH_TRY(hipMemcpyAsync(hdots, dots_d, sizeof(double) * (size_t)Bp * 2 * kAAMax, hipMemcpyDeviceToHost, st));
        SH_TRY(hipStreamSynchronize(st));
      }
      for (int b = 0; b < B; ++b) {
        if (!prep[b]) continue;
        if (I[b].have_prev) I[b].ring.solve(hdots + (size_t)b * 2 * kAAMax, hp_dir.gamma + (size_t)b * kAAMax);
        head[b] = 1;
      }
    }
    // ---- top of the next iteration of Alg. 3
    bool any_m = false;
    for (int b = 0; b < B; ++b) {
      ShInst& in = I[b];
      if (!head[b] || !in.active) continue;
      if (in.Sc.xi() <= in.tol) {
        if (int rc = finish(b, SPOCK_CONVERGED)) return rc;
        continue;
      }
      if (in.k >= s.max_iters) {
        if (int rc = finish(b, SPOCK_MAXITER)) return rc;
        continue;
      }
      if (cp) {
        set_cand(b, {{cTV, 1.0}});
        in.phase = kShCP;
        continue;
      }
      in.omega = in.Sc.omega();
      if (in.omega <= s.c0 * in.zeta) {  // K0: v + d
        in.zeta = in.omega;
        in.info.n_k0++;
        set_cand(b, {{cSPARE, 1.0}});
        in.phase = kShK0;
        continue;
      }
      any_m = true;  // M d (marked in the slot array), then the line search from tau = 1
      par_at(par_h, kParCand).slot[b] = 1;
      in.tau = 1.0;
      in.ls = 0;
      set_cand(b, {{cV, 1.0}, {cDIR, 1.0}});
      in.phase = kShLS;
    }
    // direction and candidate parameters in one upload (adjacent slots);
    // the direction kernel writes dir and spare, which the copies of the
    // instances that finished above do not read
    static_assert(kParCand == kParDir + 1, "adjacent staging slots");
    SH_TRY(hipMemcpyAsync(par_d + (size_t)kParDir * par_bytes, par_h + (size_t)kParDir * par_bytes, 2 * par_bytes,
                          hipMemcpyHostToDevice, st));
    if (any_prep) hipLaunchKernelGGL(k_sh_dir<S>, vgrid, dim3(256), 0, st, V, dp_dir.gamma, dp_dir.mask);
    if (any_m) {
      switch (T) {
        case 8: sh_launch_M<S, 8>(P, D, V, dp_cand.slot, Bp, st); break;
        case 16: sh_launch_M<S, 16>(P, D, V, dp_cand.slot, Bp, st); break;
        case 32: sh_launch_M<S, 32>(P, D, V, dp_cand.slot, Bp, st); break;
        default: sh_launch_M<S, 64>(P, D, V, dp_cand.slot, Bp, st); break;
      }
    }
    hipLaunchKernelGGL(k_sh_cand<S>, vgrid, dim3(256), 0, st, V, dp_cand.coef, dp_cand.mask);
    SH_TRY(hipGetLastError());
  }
  // s^0 of each returned point
  for (int b = 0; b < B; ++b) {
    ShInst& in = I[b];
    infos[b] = in.info;
    if (in.info.status == SPOCK_REJECTED) continue;
    S s0;
    SH_TRY(hipMemcpyAsync(&s0, vio[b], sizeof(S), hipMemcpyDeviceToHost, st));
    SH_TRY(hipStreamSynchronize(st));
    infos[b].V_s0 = (double)s0;
  }
  SH_TRY(hipStreamSynchronize(st));
  return SPOCK_OK;
}

// ================================================================ batched adjoint
// The adjoint fixed point of section 3 (see spock_backward) for B instances
// of one problem at once: every vector holds the instances `vs` elements
// apart, the S1 part of J_T' runs the shared-tree sweeps above (zero root
// state, zero dual), J_G, L and L* run with an instance grid dimension, and
// every instance runs its own restarted GMRES; the Arnoldi steps advance in
// lockstep, an instance leaving its cycle (small residual or breakdown) keeps
// computing but its columns are not used.
namespace {

// out[o_i] = a x[x_i] + c y[y_i] + e w[w_i] on entries [0, len) of every
// instance b (operand p at p.ptr + b * p.is + p.off); y, w may be null.
template <typename S>
struct BOp {
  S* p;
  long long is, off;
};
template <typename S>
__global__ void __launch_bounds__(256) k_blin3(long long len, BOp<S> out, double a, BOp<S> x, double c, BOp<S> y,
                                               double e, BOp<S> w) {
  const size_t b = blockIdx.y;
  S* o = out.p + b * out.is + out.off;
  const S* xp = x.p + b * x.is + x.off;
  const S* yp = y.p ? y.p + b * y.is + y.off : nullptr;
  const S* wp = w.p ? w.p + b * w.is + w.off : nullptr;
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < len; k += (long long)gridDim.x * blockDim.x) {
    double acc = a * (double)xp[k];
    if (yp) acc += c * (double)yp[k];
    if (wp) acc += e * (double)wp[k];
    o[k] = (S)acc;
  }
}

// Per instance b: out[2 b] = max_k |x_k - y_k|, out[2 b + 1] = max_k |x_k|
// over its first n entries (one block of 1024 threads per instance).
template <typename S>
__global__ void __launch_bounds__(1024) k_bmaxdiff(long long n, const S* __restrict__ x, const S* __restrict__ y,
                                                   long long is, double* __restrict__ out) {
  const size_t b = blockIdx.x;
  const S* xb = x + b * is;
  const S* yb = y + b * is;
  double m0 = 0, m1 = 0;
  for (long long k = threadIdx.x; k < n; k += blockDim.x) {
    m0 = fmax(m0, fabs((double)xb[k] - (double)yb[k]));
    m1 = fmax(m1, fabs((double)xb[k]));
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    m0 = fmax(m0, __shfl_xor(m0, m, 64));
    m1 = fmax(m1, __shfl_xor(m1, m, 64));
  }
  __shared__ double r0[16], r1[16];
  if ((threadIdx.x & 63) == 0) {
    r0[threadIdx.x >> 6] = m0;
    r1[threadIdx.x >> 6] = m1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0, a1 = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      a0 = fmax(a0, r0[w]);
      a1 = fmax(a1, r1[w]);
    }
    out[2 * b] = a0;
    out[2 * b + 1] = a1;
  }
}

// Krylov basis of instance b at basis + b * bs (vector j at + j * vs), its
// vector x at x + b * xs. k_bdots: block (c, j, b) sums chunk c of <V_j, x>
// (j < n; <x, x> for j = n) into part[(b * m + j) * cb + c], m = gridDim.y;
// k_bdots_final (block b) adds the chunks in order into out[b * ldo + j].
template <typename S>
__global__ void __launch_bounds__(256) k_bdots(long long nv, int n, const S* __restrict__ basis, long long bs,
                                               long long vs, const S* __restrict__ x, long long xs,
                                               double* __restrict__ part) {
  const int j = blockIdx.y, m = gridDim.y;
  const size_t b = blockIdx.z;
  const S* xb = x + b * xs;
  const S* v = j < n ? basis + b * bs + (size_t)j * vs : xb;
  const long long chunk = (nv + gridDim.x - 1) / gridDim.x;
  const long long e0 = (long long)blockIdx.x * chunk;
  const long long e1 = e0 + chunk < nv ? e0 + chunk : nv;
  double acc = 0;
  for (long long e = e0 + threadIdx.x; e < e1; e += 256) acc += (double)v[e] * (double)xb[e];
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) acc += __shfl_xor(acc, k, 64);
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    part[((size_t)b * m + j) * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}
__global__ void __launch_bounds__(256) k_bdots_final(const double* __restrict__ part, int cb, int m,
                                                     double* __restrict__ out, int ldo) {
  const size_t b = blockIdx.x;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    double acc = 0;
    for (int c = 0; c < cb; ++c) acc += part[((size_t)b * m + j) * cb + c];
    out[b * ldo + j] = acc;
  }
}
// x_b += sgn sum_{j < n} c_b[j] V_j (c_b = c + b * ldc, device); with norm,
// then scaled by 1 / sqrt(c_b[n] - sum_j c_b[j]^2) (0 if not positive)
template <typename S>
__global__ void __launch_bounds__(256) k_bcomb(long long nv, int n, const S* __restrict__ basis, long long bs,
                                               long long vs, const double* __restrict__ c, int ldc, double sgn,
                                               int norm, S* x, long long xs) {
  const size_t b = blockIdx.y;
  const double* cb = c + b * ldc;
  const S* Vb = basis + b * bs;
  S* xb = x + b * xs;
  double scale = 1.0;
  if (norm) {
    double h2 = cb[n];
    for (int j = 0; j < n; ++j) h2 -= cb[j] * cb[j];
    scale = h2 > 0.0 ? 1.0 / sqrt(h2) : 0.0;
  }
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nv; e += (long long)gridDim.x * blockDim.x) {
    double acc = (double)xb[e];
    for (int j = 0; j < n; ++j) acc += sgn * cb[j] * (double)Vb[(size_t)j * vs + e];
    xb[e] = (S)(acc * scale);
  }
}

}  // namespace

template <typename S>
int shared_backward(Problem& P, int B, const void* const* vstar, const double* const* x0, double gV,
                    const double* const* gu0, double* const* gx0, double* const* gq, double* const* gqN,
                    const spock_settings& s, spock_info* infos, hipStream_t st) {
  const Tree& Tr = *P.tree;
  const DevProb<S>& D = sh_dev<S>(P);
  const int nx = P.nx, nu = P.nu, T = P.team_pp;
  const long long nz = P.nz, ne = P.neta, nv = nz + ne;
  const long long vs = (nv + 63) & ~63LL;
  const int Bp = (B + kShCols - 1) / kShCols * kShCols;
  const double al = P.alpha;
  constexpr int kMax = 120;  // Krylov vectors per cycle at most
  int R = sizeof(S) * (size_t)(kMax + 1) * (size_t)vs * (size_t)Bp <= (size_t(2) << 30) ? kMax : 30;
  if (const char* env = std::getenv("SPOCK_ADJ_RESTART")) R = std::max(2, std::min(kMax, std::atoi(env)));
  const long long bs = (long long)(R + 1) * vs;  // basis stride between instances
  const int cb = std::max(1, std::min(64, (int)((nv + 8191) / 8192)));
  const int ldc = kMax + 2;
  // ---- device memory: 14 batch vectors, the bases, sweep buffers, x0s,
  // coefficients and partial sums
  enum { kV, kTv, kDz, kLdz, kB, kG, kW, kAw, kLb, kCz, kLa, kTz, kTe, kIn, kNVec };
  const size_t nvec = (size_t)Bp * vs;
  size_t off = 0;
  auto reserve = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t o_vec = reserve(sizeof(S) * nvec * kNVec);
  const size_t o_bas = reserve(sizeof(S) * (size_t)Bp * bs);
  const size_t o_qx = reserve(sizeof(S) * (size_t)Bp * Tr.nn * nx * 2);
  const size_t o_du = reserve(sizeof(S) * (size_t)Bp * Tr.nn * nu * 2);
  const size_t o_x0 = reserve(sizeof(double) * (size_t)Bp * nx * 2);
  const size_t o_c = reserve(sizeof(double) * (size_t)Bp * ldc * 3);
  const size_t o_part = reserve(sizeof(double) * (size_t)Bp * (kMax + 2) * cb);
  const size_t o_md = reserve(sizeof(double) * (size_t)Bp * 2);
  const size_t o_mu = reserve(sizeof(S) * (size_t)Tr.nn * nx);
  void* mem = nullptr;
  if (hipMalloc(&mem, off) != hipSuccess) return SPOCK_ENOMEM;
  struct Guard {
    void* m;
    ~Guard() { (void)hipFree(m); }
  } guard{mem};
  char* base = static_cast<char*>(mem);
  SH_TRY(hipMemsetAsync(base, 0, off, st));  // padding instances stay at zero
  S* vec[kNVec];
  for (int r = 0; r < kNVec; ++r) vec[r] = reinterpret_cast<S*>(base + o_vec) + (size_t)r * nvec;
  S* basis = reinterpret_cast<S*>(base + o_bas);
  S* q = reinterpret_cast<S*>(base + o_qx);
  S* xbar = q + (size_t)Bp * Tr.nn * nx;
  S* d = reinterpret_cast<S*>(base + o_du);
  S* ubar = d + (size_t)Bp * Tr.nn * nu;
  double* x0s = reinterpret_cast<double*>(base + o_x0);
  double* x0zero = x0s + (size_t)Bp * nx;
  double* cdev = reinterpret_cast<double*>(base + o_c);  // [Bp][ldc] x 3: pass 1, pass 2, mix
  double* c1 = cdev;
  double* c2 = cdev + (size_t)Bp * ldc;
  double* cm = cdev + 2 * (size_t)Bp * ldc;
  double* part = reinterpret_cast<double*>(base + o_part);
  double* md = reinterpret_cast<double*>(base + o_md);
  S* mu = reinterpret_cast<S*>(base + o_mu);
  const int vb = (int)std::min<long long>((nv + 255) / 256, 64);
  auto op = [&](int r, long long o = 0) { return BOp<S>{vec[r], vs, o}; };
  auto lin3 = [&](long long len, BOp<S> o, double a, BOp<S> x, double c = 0, BOp<S> y = BOp<S>{nullptr, 0, 0},
                  double e = 0, BOp<S> w = BOp<S>{nullptr, 0, 0}) -> int {
    hipLaunchKernelGGL(k_blin3<S>, dim3(vb, Bp), dim3(256), 0, st, len, o, a, x, c, y, e, w);
    SH_TRY(hipGetLastError());
    return SPOCK_OK;
  };
  // ---- inputs: v* and x0 of every instance, the cotangents
  for (int b = 0; b < B; ++b) {
    SH_TRY(hipMemcpyAsync(vec[kV] + (size_t)b * vs, vstar[b], sizeof(S) * nv, hipMemcpyDeviceToDevice, st));
    SH_TRY(hipMemcpyAsync(x0s + (size_t)b * nx, x0[b], sizeof(double) * nx, hipMemcpyDeviceToDevice, st));
  }
  {
    const size_t head = 1 + (size_t)Tr.nn * nx + nu;
    std::vector<S> hg((size_t)B * head, S(0));
    std::vector<double> hu(nu);
    for (int b = 0; b < B; ++b) {
      hg[(size_t)b * head] = (S)gV;
      if (gu0 && gu0[b]) {
        SH_TRY(hipMemcpy(hu.data(), gu0[b], sizeof(double) * nu, hipMemcpyDeviceToHost));
        for (int k = 0; k < nu; ++k) hg[(size_t)b * head + 1 + (size_t)Tr.nn * nx + k] = (S)hu[k];
      }
    }
    for (int b = 0; b < B; ++b)
      SH_TRY(hipMemcpyAsync(vec[kG] + (size_t)b * vs, hg.data() + (size_t)b * head, sizeof(S) * head,
                            hipMemcpyHostToDevice, st));
    SH_TRY(hipStreamSynchronize(st));  // hg is a local buffer
  }
  // T of the instances without (with) the dual part: pre-pass, then the
  // sweeps in the phases of the shared-tree form
  int maxch = 1;
  for (int i = 0; i < Tr.nl; ++i) maxch = std::max(maxch, Tr.nch[i]);
  int sh_cut = 0;
  for (int t = 1; t < Tr.N; ++t)
    if (Tr.stage_off[t + 1] - Tr.stage_off[t] >= 8) {
      sh_cut = t;
      break;
    }
  if (const char* env = std::getenv("SPOCK_SH_CUT")) sh_cut = std::atoi(env);
  if (sh_cut < 1 || sh_cut >= Tr.N || Tr.N - sh_cut > kShMaxLevels) sh_cut = 0;
  const int sweep_grid = Bp / kShCols;
  auto prox = [&](S* in, S* out, const double* xs0) -> int {
    const int tpb = 256 / T;
    const dim3 grid((Tr.nl + tpb - 1) / tpb, Bp);
    switch (T) {
      case 8: hipLaunchKernelGGL((k_sh_pre<S, 8>), grid, dim3(256), 0, st, D, in, out, xbar, ubar, q, vs); break;
      case 16: hipLaunchKernelGGL((k_sh_pre<S, 16>), grid, dim3(256), 0, st, D, in, out, xbar, ubar, q, vs); break;
      case 32: hipLaunchKernelGGL((k_sh_pre<S, 32>), grid, dim3(256), 0, st, D, in, out, xbar, ubar, q, vs); break;
      default: hipLaunchKernelGGL((k_sh_pre<S, 64>), grid, dim3(256), 0, st, D, in, out, xbar, ubar, q, vs); break;
    }
    if (sh_cut > 0) {
      const int nsub = Tr.stage_off[sh_cut + 1] - Tr.stage_off[sh_cut];
      for (int ph : {kShBwdSub, kShBwdTop, kShFwdTop, kShFwdSub}) {
        const ShSweepArgs A{maxch, ph, sh_cut, nsub};
        const bool subph = ph == kShBwdSub || ph == kShFwdSub;
        hipLaunchKernelGGL(k_sh_sweeps<S>, dim3(subph ? sweep_grid * nsub : sweep_grid), dim3(64 * kShWaves), 0, st,
                           D, P.d_stage_off, out, xs0, xbar, ubar, q, d, vs, A);
      }
    } else {
      const ShSweepArgs A{maxch, kShWhole, 0, 1};
      hipLaunchKernelGGL(k_sh_sweeps<S>, dim3(sweep_grid), dim3(64 * kShWaves), 0, st, D, P.d_stage_off, out, xs0,
                         xbar, ubar, q, d, vs, A);
    }
    SH_TRY(hipGetLastError());
    return SPOCK_OK;
  };
  // pre-prox point of the dual update at v*: b* = eta* + alpha L (2 z+ - z*)
  if (int r = prox(vec[kV], vec[kTv], x0s)) return r;
  if (int r = lin3(nz, op(kDz), 2.0, op(kTv), -1.0, op(kV))) return r;
  SH_TRY(launch_L_batch<S>(P, vec[kDz], vec[kLdz], vs, Bp, st));
  if (int r = lin3(ne, op(kB), 1.0, op(kV, nz), al, op(kLdz))) return r;
  // one application of the transposed operator to vec[kIn]: lb, tz, cz, la
  auto partial = [&](int in) -> int {
    SH_TRY(launch_jg_batch<S>(P, vec[kB], vec[in] + nz, vec[kLb], vs, Bp, st));  // lambda_b = J_G w_eta
    SH_TRY(launch_Lt_batch<S>(P, vec[kLb], vec[kTz], vs, Bp, st));              // L* lambda_b
    if (int r = lin3(nz, op(kCz), 1.0, op(in), 2.0 * al, op(kTz))) return r;    // w_z + 2 alpha L* lambda_b
    if (int r = prox(vec[kCz], vec[kLa], x0zero)) return r;                      // J_f c (zero dual part)
    if (int r = lin3(1, op(kLa), 1.0, op(kCz))) return r;                        // identity on s^0
    return SPOCK_OK;
  };
  // A(w) = J_T(v*)' w + g into vec[kAw]
  auto apply_A = [&](int in) -> int {
    if (int r = partial(in)) return r;
    SH_TRY(launch_L_batch<S>(P, vec[kLa], vec[kTe], vs, Bp, st));
    if (int r = lin3(nz, op(kAw), 1.0, op(kLa), -al, op(kTz), 1.0, op(kG))) return r;
    if (int r = lin3(ne, op(kAw, nz), 1.0, op(kLb), -al, op(kTe), 1.0, op(kG, nz))) return r;
    return SPOCK_OK;
  };
  auto bdots = [&](int n, const S* x, long long xs, bool xx, double* out) -> int {
    const int m = n + (xx ? 1 : 0);
    hipLaunchKernelGGL(k_bdots<S>, dim3(cb, m, Bp), dim3(256), 0, st, nv, n, basis, bs, vs, x, xs, part);
    hipLaunchKernelGGL(k_bdots_final, dim3(Bp), dim3(256), 0, st, part, cb, m, out, ldc);
    SH_TRY(hipGetLastError());
    return SPOCK_OK;
  };
  auto bcomb = [&](int n, const double* c, double sgn, bool norm, S* x, long long xs) -> int {
    hipLaunchKernelGGL(k_bcomb<S>, dim3(vb, Bp), dim3(256), 0, st, nv, n, basis, bs, vs, c, ldc, sgn, norm ? 1 : 0, x,
                       xs);
    SH_TRY(hipGetLastError());
    return SPOCK_OK;
  };
  auto V = [&](int j) { return basis + (size_t)j * vs; };  // vector j of instance 0 (instances bs apart)
  // ---- restarted GMRES per instance, Arnoldi steps in lockstep
  SH_TRY(hipMemcpyAsync(vec[kW], vec[kG], sizeof(S) * nvec, hipMemcpyDeviceToDevice, st));
  const double tol = std::max(s.eps_abs, 1e-15);
  std::vector<int> kk(B, 0), state(B, 0);  // state: 0 running, 1 converged, 2 numerical, 3 max_iters
  std::vector<double> diff(B, 0.0);
  std::vector<double> hmd((size_t)Bp * 2), hc1((size_t)Bp * ldc), hc2((size_t)Bp * ldc), hcm((size_t)Bp * ldc);
  std::vector<double> Hm((size_t)B * (kMax + 1) * kMax), cs((size_t)B * kMax), sn((size_t)B * kMax),
      gvv((size_t)B * (kMax + 1));
  std::vector<int> jn(B), incyc(B);
  auto running = [&]() {
    for (int b = 0; b < B; ++b)
      if (state[b] == 0) return true;
    return false;
  };
  while (running()) {
    // true residual of every instance at w
    SH_TRY(hipMemcpyAsync(vec[kIn], vec[kW], sizeof(S) * nvec, hipMemcpyDeviceToDevice, st));
    if (int r = apply_A(kIn)) return r;
    hipLaunchKernelGGL(k_bmaxdiff<S>, dim3(Bp), dim3(1024), 0, st, nv, vec[kW], vec[kAw], vs, md);
    SH_TRY(hipGetLastError());
    SH_TRY(hipMemcpyAsync(hmd.data(), md, sizeof(double) * 2 * Bp, hipMemcpyDeviceToHost, st));
    SH_TRY(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b) {
      if (state[b] != 0) continue;
      ++kk[b];
      diff[b] = hmd[2 * b];
      if (!std::isfinite(diff[b])) state[b] = 2;
      else if (diff[b] <= tol * std::max(1.0, hmd[2 * b + 1])) state[b] = 1;
      else if (kk[b] >= s.max_iters) state[b] = 3;
    }
    if (!running()) break;
    // V_0 = (A(w) - w) / |.| for every instance
    if (int r = lin3(nv, BOp<S>{basis, bs, 0}, 1.0, op(kAw), -1.0, op(kW))) return r;
    if (int r = bdots(0, V(0), bs, true, c1)) return r;
    SH_TRY(hipMemcpyAsync(hc1.data(), c1, sizeof(double) * Bp * ldc, hipMemcpyDeviceToHost, st));
    SH_TRY(hipStreamSynchronize(st));
    if (int r = bcomb(0, c1, 1.0, true, V(0), bs)) return r;
    std::fill(Hm.begin(), Hm.end(), 0.0);
    for (int b = 0; b < B; ++b) {
      const double beta = std::sqrt(std::max(hc1[(size_t)b * ldc], 0.0));
      gvv[(size_t)b * (kMax + 1)] = beta;
      jn[b] = 0;
      incyc[b] = state[b] == 0 && beta > 0.0 && std::isfinite(beta);
      if (state[b] == 0 && !(beta > 0.0)) state[b] = std::isfinite(beta) ? 1 : 2;
    }
    auto any_in = [&]() {
      for (int b = 0; b < B; ++b)
        if (incyc[b]) return true;
      return false;
    };
    for (int j = 0; j < R && any_in(); ++j) {
      SH_TRY(hipMemcpy2DAsync(vec[kIn], sizeof(S) * vs, V(j), sizeof(S) * bs, sizeof(S) * nv, Bp,
                              hipMemcpyDeviceToDevice, st));
      if (int r = apply_A(kIn)) return r;
      // V_{j+1} = V_j - A(V_j) + g, two Gram-Schmidt passes, normalisation
      if (int r = lin3(nv, BOp<S>{V(j + 1), bs, 0}, 1.0, op(kIn), -1.0, op(kAw), 1.0, op(kG))) return r;
      if (int r = bdots(j + 1, V(j + 1), bs, false, c1)) return r;
      if (int r = bcomb(j + 1, c1, -1.0, false, V(j + 1), bs)) return r;
      if (int r = bdots(j + 1, V(j + 1), bs, true, c2)) return r;
      if (int r = bcomb(j + 1, c2, -1.0, true, V(j + 1), bs)) return r;
      SH_TRY(hipMemcpyAsync(hc1.data(), c1, sizeof(double) * Bp * ldc, hipMemcpyDeviceToHost, st));
      SH_TRY(hipMemcpyAsync(hc2.data(), c2, sizeof(double) * Bp * ldc, hipMemcpyDeviceToHost, st));
      SH_TRY(hipStreamSynchronize(st));
      for (int b = 0; b < B; ++b) {
        if (!incyc[b]) continue;
        ++kk[b];
        double* Hb = Hm.data() + (size_t)b * (kMax + 1) * kMax;
        auto H = [&](int i, int jj) -> double& { return Hb[(size_t)i * kMax + jj]; };
        double* csb = cs.data() + (size_t)b * kMax;
        double* snb = sn.data() + (size_t)b * kMax;
        double* gv = gvv.data() + (size_t)b * (kMax + 1);
        const double* h1 = hc1.data() + (size_t)b * ldc;
        const double* h2 = hc2.data() + (size_t)b * ldc;
        double hn = h2[j + 1];
        for (int i = 0; i <= j; ++i) {
          H(i, j) = h1[i] + h2[i];
          hn -= h2[i] * h2[i];
        }
        hn = std::sqrt(std::max(hn, 0.0));
        H(j + 1, j) = hn;
        for (int i = 0; i < j; ++i) {
          const double xv = H(i, j), yv = H(i + 1, j);
          H(i, j) = csb[i] * xv + snb[i] * yv;
          H(i + 1, j) = -snb[i] * xv + csb[i] * yv;
        }
        const double rr = std::hypot(H(j, j), H(j + 1, j));
        csb[j] = rr > 0.0 ? H(j, j) / rr : 1.0;
        snb[j] = rr > 0.0 ? H(j + 1, j) / rr : 0.0;
        H(j, j) = rr;
        H(j + 1, j) = 0.0;
        gv[j + 1] = -snb[j] * gv[j];
        gv[j] = csb[j] * gv[j];
        jn[b] = j + 1;
        const double thr = tol * std::max(1.0, hmd[2 * b + 1]);
        if (!std::isfinite(gv[j + 1]) || std::fabs(gv[j + 1]) <= 0.5 * thr || !(hn > 0.0) || kk[b] >= s.max_iters)
          incyc[b] = 0;
      }
    }
    // w += V y per instance (H y = g, upper triangular; zero for the others)
    std::fill(hcm.begin(), hcm.end(), 0.0);
    int nmax = 0;
    for (int b = 0; b < B; ++b) {
      if (state[b] != 0 || jn[b] == 0) continue;
      const double* Hb = Hm.data() + (size_t)b * (kMax + 1) * kMax;
      const double* gv = gvv.data() + (size_t)b * (kMax + 1);
      double* y = hcm.data() + (size_t)b * ldc;
      for (int i = jn[b] - 1; i >= 0; --i) {
        double t = gv[i];
        for (int l = i + 1; l < jn[b]; ++l) t -= Hb[(size_t)i * kMax + l] * y[l];
        y[i] = Hb[(size_t)i * kMax + i] != 0.0 ? t / Hb[(size_t)i * kMax + i] : 0.0;
      }
      nmax = std::max(nmax, jn[b]);
    }
    SH_TRY(hipMemcpyAsync(cm, hcm.data(), sizeof(double) * Bp * ldc, hipMemcpyHostToDevice, st));
    if (int r = bcomb(nmax, cm, 1.0, false, vec[kW], vs)) return r;
    SH_TRY(hipStreamSynchronize(st));  // hcm is reused
  }
  // gradients from the converged adjoints
  SH_TRY(hipMemcpyAsync(vec[kIn], vec[kW], sizeof(S) * nvec, hipMemcpyDeviceToDevice, st));
  if (int r = partial(kIn)) return r;
  for (int b = 0; b < B; ++b) {
    SH_TRY(launch_phiT<S>(P, vec[kCz] + (size_t)b * vs, mu, st));
    std::vector<S> hm(nx);
    SH_TRY(hipMemcpyAsync(hm.data(), mu, nx * sizeof(S), hipMemcpyDeviceToHost, st));
    SH_TRY(hipStreamSynchronize(st));
    std::vector<double> outv(nx);
    for (int k = 0; k < nx; ++k) outv[k] = hm[k];
    SH_TRY(hipMemcpy(gx0[b], outv.data(), nx * sizeof(double), hipMemcpyHostToDevice));
    double* gqb = gq ? gq[b] : nullptr;
    double* gqNb = gqN ? gqN[b] : nullptr;
    if (gqb) SH_TRY(hipMemsetAsync(gqb, 0, sizeof(double) * (size_t)Tr.nn * nx, st));
    if (gqNb) SH_TRY(hipMemsetAsync(gqNb, 0, sizeof(double) * (size_t)Tr.nn * nx, st));
    if (gqb || gqNb)
      SH_TRY(launch_grad_q<S>(P, vec[kV] + (size_t)b * vs, vec[kLa] + (size_t)b * vs, vec[kLb] + (size_t)b * vs, gqb,
                              gqNb, st));
    spock_info loc{};
    loc.V_nested = std::numeric_limits<double>::quiet_NaN();
    loc.status = state[b] == 1 ? SPOCK_CONVERGED : (state[b] == 2 ? SPOCK_NUMERICAL : SPOCK_MAXITER);
    loc.iters = kk[b];
    loc.t_evals = kk[b];
    loc.xi = diff[b];
    loc.mapping = kTeamShared;
    infos[b] = loc;
  }
  SH_TRY(hipStreamSynchronize(st));
  return SPOCK_OK;
}

template int shared_backward<double>(Problem&, int, const void* const*, const double* const*, double,
                                     const double* const*, double* const*, double* const*, double* const*,
                                     const spock_settings&, spock_info*, hipStream_t);
template int shared_backward<float>(Problem&, int, const void* const*, const double* const*, double,
                                    const double* const*, double* const*, double* const*, double* const*,
                                    const spock_settings&, spock_info*, hipStream_t);

template int shared_solve<double>(Problem&, int, const double* const*, const spock_settings&, void* const*,
                                  spock_info*, hipStream_t);
template int shared_solve<float>(Problem&, int, const double* const*, const spock_settings&, void* const*,
                                 spock_info*, hipStream_t);

}  // namespace spk
