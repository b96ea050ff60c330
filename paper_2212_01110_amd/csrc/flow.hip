// Dataflow form of the CP operator T: the whole evaluation (pre-pass, both
// Alg. 2 sweeps, the dual update and the residual statistics) in ONE
// persistent launch, so the 2N + 3 dependent launches of the per-stage form
// and their dispatch latency disappear.
//
// Work items, in this order:
//   [0, nl)              backward step of family nl-1-t (reverse breadth-first:
//                        every child family comes first), with the pre-pass
//                        of the family fused in (xbar, ubar, leaf seeds, S2)
//   [nl, 2 nl)           forward step of family t-nl (breadth-first: the
//                        parent comes first), with the dual update of the
//                        family's rows and its statistics record fused in
//   [2 nl, 2 nl + nr)    fixed-order sum of 256 statistics records
//   2 nl + nr            final sum of the nr chunk records into the six
//                        statistics of T (only when the dual part is formed)
// Workgroup b runs items b, b + G, b + 2G, ... (G = grid size, every
// workgroup resident). An item waits only on items with a smaller index:
// the smallest unfinished item therefore never waits, and the launch drains.
// Completion is published per family in a 32-bit flag holding
// base + {1: q and d written, 2: x of the children written, 3: statistics
// record written}, base = 4 * (launch epoch), compared modulo 2^32, so no
// flag is ever cleared. Values crossing workgroups are stored and loaded
// agent-coherent (they bypass the per-XCD L2's non-coherent lines), so
// publishing is a wait for the wavefront's stores, not an L2 write-back,
// and observing is a wait for the flag load. Every wait is
// bounded; a wait that gives up raises an error word and the statistics of
// the launch come out as NaN (no wave ever spins without end).
//
// Matrices of an item are copied into LDS with direct global-to-LDS loads,
// all issued before the item's first wait, so an item costs one HBM round
// trip plus its dependency wait; the mat-vecs then run from LDS.
#include "device_common.h"

#include <math.h>
#include <algorithm>

namespace spk {

namespace {

constexpr int kFW = 256;                 // threads per workgroup (4 wavefronts)
constexpr unsigned kSpinLimit = 1u << 21;  // polls of one bounded wait
constexpr int kFoldMax = 16;             // partial sums per mat-vec output

typedef __attribute__((address_space(3))) void lds_void;

// Word offsets of the dynamic LDS regions (32-bit words; every region is a
// whole number of 64-word rows so that a wavefront copy may overrun it).
struct FlowLds {
  int esz;         // words per element
  int sA, sB;      // per-child strides of the Abar and B regions
  int oA, oB, oR, oK, oW, oQ, oRed;
  int nc;          // children per chunk
  __host__ __device__ static int pad(int w) { return (w + 63) & ~63; }
  __host__ __device__ FlowLds(int nx, int nu, int nc_, int esz_) {
    esz = esz_;
    nc = nc_;
    sA = pad(nx * nx * esz);
    sB = pad(nx * nu * esz);
    oA = 0;
    oB = oA + nc * sA;
    oR = oB + nc * sB;
    oK = oR + pad(nu * nu * esz);
    oW = oK + pad(nx * nu * esz);
    oQ = oW + pad(nx * nu * esz);
    oRed = oQ + pad(nc * kMaxDim * esz);
    words_ = oRed + pad((nc + 1) * kFW * esz);
  }
  int words_;
  __host__ __device__ int bytes() const { return words_ * 4; }
};

// Copies nwords 32-bit words from global memory into LDS (dst = word
// offset); wavefront w issues rows w, w + 4, ... of 64 words. Lanes past the
// end re-read the last word (in bounds) into the region's padding.
__device__ __forceinline__ void dma_words(const void* src, unsigned* lds, int dst, int nwords) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned* s = static_cast<const unsigned*>(src);
  for (int r = w; r * 64 < nwords; r += 4) {
    int e = r * 64 + lane;
    e = e < nwords ? e : nwords - 1;
    __builtin_amdgcn_global_load_lds(s + e, (lds_void*)(lds + dst + r * 64), 4, 0, 0);
  }
}

__device__ __forceinline__ void wait_vm() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

// Partial mat-vec from LDS: M input-major (element (out o, in k) at
// k * nout + o), v (nin) in LDS; thread t < G * nout adds the products of
// inputs k = g, g + G, ... (g = t / nout) of output o = t % nout to red[t].
template <typename S>
__device__ __forceinline__ void mv_part(const S* M, const S* v, int nin, int nout, S* red, bool acc) {
  const int G = min(kFW / nout, kFoldMax), span = G * nout, t = threadIdx.x;
  if (t < span) {
    const int g = t / nout;
    S a = acc ? red[t] : S(0);
    const int n = nin * nout;
    int k = g;
    for (int e = t; e < n; e += span, k += G) a += M[e] * v[k];
    red[t] = a;
  }
}

template <typename S>
__device__ __forceinline__ S mv_fold(const S* red, int nout, int o) {
  const int G = min(kFW / nout, kFoldMax);
  S s = 0;
  for (int g = 0; g < G; ++g) s += red[g * nout + o];
  return s;
}

__device__ __forceinline__ unsigned ld_flag(const unsigned* f) {
  return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publishes value v in flag f once this wavefront's earlier stores are
// complete. Every value another workgroup reads is stored agent-coherent
// (st_c), so waiting for the stores to be acknowledged orders them before
// the flag; no L2 write-back is needed.
__device__ __forceinline__ void release_flag(unsigned* f, unsigned v) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  wait_vm();
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(f, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits (bounded) until flag f reaches base + want within the current epoch;
// the caller acquires afterwards. Gives up at once when the error word is set.
__device__ __forceinline__ void wait_flag(const unsigned* f, unsigned base, unsigned want,
                                          unsigned* err) {
  for (unsigned it = 0; it < kSpinLimit; ++it) {
    const unsigned d = ld_flag(f) - base;
    if (d >= want && d <= 3u) return;
    if ((it & 255u) == 255u && ld_flag(err) != 0u) return;
    __builtin_amdgcn_s_sleep(2);
  }
  __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// After a wait: the flag loads are complete before any later load issues;
// the values behind the flag are then read agent-coherent (ld_c).
__device__ __forceinline__ void acquire() {
  wait_vm();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename S>
struct FlowArgs {
  DevProb<S> P;
  const S* z;
  const S* eta;
  S* zout;
  S* eout;
  const double* x0;
  S* q;
  S* d;
  double* partials;   // [nl][kStats]
  double* part2;      // [nr][kStats]
  double* stats;      // [6]
  unsigned* flag;     // [nl]
  unsigned* flag2;    // [nr]
  unsigned* err;      // [1]
  unsigned base;
  int nc, nr, items, dual;
};

// ---------------------------------------------------------------- backward item
template <typename S>
__device__ void flow_bwd(const FlowArgs<S>& A, const FlowLds& L, unsigned* lds, int i) {
  __shared__ S xb[kMaxDim], ub[kMaxDim], sAv[kMaxDim], vg[kMaxDim], vd[kMaxDim];
  const DevProb<S>& P = A.P;
  const Off<S> O(P);
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  const int es = L.esz;
  S* M = reinterpret_cast<S*>(lds);
  S* qv = reinterpret_cast<S*>(lds + L.oQ);
  S* redA = reinterpret_cast<S*>(lds + L.oRed);
  S* redB = redA + kFW;
  const bool leafkids = fc >= P.nl;
  for (int k0 = 0; k0 < n; k0 += L.nc) {
    const int kc = min(L.nc, n - k0);
    for (int k = 0; k < kc; ++k) {
      dma_words(P.AbR + (size_t)(fc + k0 + k) * nx * nx, lds, L.oA + k * L.sA, nx * nx * es);
      dma_words(P.BR + (size_t)(fc + k0 + k) * nx * nu, lds, L.oB + k * L.sB, nx * nu * es);
    }
    if (k0 == 0) {
      dma_words(P.Rinv + (size_t)i * nu * nu, lds, L.oR, nu * nu * es);
      dma_words(P.KR + (size_t)i * nu * nx, lds, L.oK, nu * nx * es);
      dma_words(P.WC + (size_t)i * nu * nx, lds, L.oW, nu * nx * es);
      if (w == 0) {  // xbar, ubar of the family (pre-pass)
        S xbv[1], ubv[1];
        fam_xbar_ubar<S, 64, 64>(P, O, A.z, A.eta, i, lane, xbv, ubv);
        xb[lane] = xbv[0];
        ub[lane] = ubv[0];
      } else if (w == 1) {  // S2 projection of the z2 block, s^0 at the root
        fam_s2<S, 64, 64, true>(P, O, A.z, A.eta, A.zout, i, lane);
      }
    }
    // q of the children of this chunk
    if (leafkids) {
      if (w == 2)
        for (int k = 0; k < kc; ++k)
          if (lane < nx) qv[k * kMaxDim + lane] = fam_child_q<S>(P, O, A.z, A.eta, A.q, fc + k0 + k, lane);
    } else if (w == 3) {
      if (lane < kc) wait_flag(A.flag + fc + k0 + lane, A.base, 1u, A.err);
      acquire();
      for (int k = 0; k < kc; ++k)
        if (lane < nx) qv[k * kMaxDim + lane] = ld_c<true>(A.q + (size_t)(fc + k0 + k) * nx + lane);
    }
    wait_vm();
    __syncthreads();
    for (int k = 0; k < kc; ++k) {
      mv_part<S>(M + L.oA / es + k * (L.sA / es), qv + k * kMaxDim, nx, nx, redA, k0 + k > 0);
      mv_part<S>(M + L.oB / es + k * (L.sB / es), qv + k * kMaxDim, nx, nu, redB, k0 + k > 0);
    }
    __syncthreads();  // matrices and q consumed before the next chunk's copies
  }
  // d = R~^{-1}(ubar - sum_c B^c' q^c)
  if (t < nx) sAv[t] = mv_fold<S>(redA, nx, t);
  if (t < nu) vg[t] = ub[t] - mv_fold<S>(redB, nu, t);
  __syncthreads();
  mv_part<S>(M + L.oR / es, vg, nu, nu, redA, false);
  __syncthreads();
  if (t < nu) {
    const S dv = mv_fold<S>(redA, nu, t);
    vd[t] = dv;
    st_c<true>(A.d + (size_t)i * nu + t, dv);
  }
  __syncthreads();
  if (t < nu) vg[t] = vd[t] - ub[t];
  __syncthreads();
  // q = K'(d - ubar) + W d - xbar + sum_c Abar^c' q^c
  mv_part<S>(M + L.oK / es, vg, nu, nx, redA, false);
  mv_part<S>(M + L.oW / es, vd, nu, nx, redB, false);
  __syncthreads();
  if (t < nx) st_c<true>(A.q + (size_t)i * nx + t, mv_fold<S>(redA, nx, t) + mv_fold<S>(redB, nx, t) - xb[t] + sAv[t]);
  // q and d were written by wavefront 0, the S2 block by wavefront 1 before
  // the last barriers (which waited for those stores)
  if (w == 0) release_flag(A.flag + i, A.base + 1u);
  __syncthreads();  // LDS reuse by the next item
}

// ---------------------------------------------------------------- forward item
template <typename S>
__device__ void flow_fwd(const FlowArgs<S>& A, const FlowLds& L, unsigned* lds, int i) {
  __shared__ S vx[kMaxDim], vd[kMaxDim];
  __shared__ S post_lds[3 * kMaxDim];
  const DevProb<S>& P = A.P;
  const Off<S> O(P);
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  const int es = L.esz;
  S* M = reinterpret_cast<S*>(lds);
  S* red = reinterpret_cast<S*>(lds + L.oRed);
  for (int k0 = 0; k0 < n; k0 += L.nc) {
    const int kc = min(L.nc, n - k0);
    for (int k = 0; k < kc; ++k) {
      dma_words(P.AbC + (size_t)(fc + k0 + k) * nx * nx, lds, L.oA + k * L.sA, nx * nx * es);
      dma_words(P.BC + (size_t)(fc + k0 + k) * nu * nx, lds, L.oB + k * L.sB, nx * nu * es);
    }
    if (k0 == 0) {
      dma_words(P.KC + (size_t)i * nx * nu, lds, L.oK, nx * nu * es);
      if (w == 0) {
        // x^i from the parent's step (x0 at the root), d^i from the backward sweep
        if (i == 0) wait_flag(A.flag, A.base, 1u, A.err);
        else wait_flag(A.flag + P.anc[i], A.base, 2u, A.err);
        acquire();
        if (lane < nx) {
          S xv;
          if (i == 0) {
            xv = (S)A.x0[lane];
            st_c<true>(A.zout + 1 + lane, xv);
          } else {
            xv = ld_c<true>(A.zout + O.x(i) + lane);
          }
          vx[lane] = xv;
        }
        if (lane < nu) vd[lane] = ld_c<true>(A.d + (size_t)i * nu + lane);
      }
    }
    wait_vm();
    __syncthreads();
    if (k0 == 0) mv_part<S>(M + L.oK / es, vx, nx, nu, red + L.nc * kFW, false);
    for (int k = 0; k < kc; ++k) {
      mv_part<S>(M + L.oA / es + k * (L.sA / es), vx, nx, nx, red + k * kFW, false);
      mv_part<S>(M + L.oB / es + k * (L.sB / es), vd, nu, nx, red + k * kFW, true);
    }
    __syncthreads();
    if (k0 == 0 && t < nu) st_c<true>(A.zout + O.u(i) + t, mv_fold<S>(red + L.nc * kFW, nu, t) + vd[t]);
    for (int k = 0; k < kc; ++k)
      if (t < nx) st_c<true>(A.zout + O.x(fc + k0 + k) + t, mv_fold<S>(red + k * kFW, nx, t));
    __syncthreads();  // red and the matrices are reused by the next chunk / item
  }
  if (w != 0) return;
  // u^i and the children's x were written by wavefront 0 (threads < 64)
  release_flag(A.flag + i, A.base + 2u);
  if (!A.dual) return;
  StatAcc st;
  fam_post_team<S, 64, 64, true>(P, A.z, A.eta, A.zout, A.eout, i, lane, post_lds, kMaxDim, st);
  double r0 = st.rz2, r1 = st.re2, r2 = st.cross, r3 = st.xip, r4 = st.xid;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    r0 += __shfl_xor(r0, m, 64);
    r1 += __shfl_xor(r1, m, 64);
    r2 += __shfl_xor(r2, m, 64);
    r3 = fmax(r3, __shfl_xor(r3, m, 64));
    r4 = fmax(r4, __shfl_xor(r4, m, 64));
  }
  if (lane == 0) {
    double* p = A.partials + (size_t)i * kStats;
    st_c<true>(p + 0, r0);
    st_c<true>(p + 1, r1);
    st_c<true>(p + 2, r2);
    st_c<true>(p + 3, r3);
    st_c<true>(p + 4, r4);
  }
  release_flag(A.flag + i, A.base + 3u);
}

// ---------------------------------------------------------------- statistics items
// Fixed-order reduction of the five statistics over the workgroup: a
// butterfly inside each wavefront, then the four wavefront sums in order.
// Ends with the total in thread 0's v.
__device__ __forceinline__ void block_reduce5(double (&v)[kStats], double* wsum) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    v[0] += __shfl_xor(v[0], m, 64);
    v[1] += __shfl_xor(v[1], m, 64);
    v[2] += __shfl_xor(v[2], m, 64);
    v[3] = fmax(v[3], __shfl_xor(v[3], m, 64));
    v[4] = fmax(v[4], __shfl_xor(v[4], m, 64));
  }
  if (lane == 0)
#pragma unroll
    for (int s = 0; s < kStats; ++s) wsum[w * kStats + s] = v[s];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kFW / 64; ++q) {
      v[0] += wsum[q * kStats + 0];
      v[1] += wsum[q * kStats + 1];
      v[2] += wsum[q * kStats + 2];
      v[3] = fmax(v[3], wsum[q * kStats + 3]);
      v[4] = fmax(v[4], wsum[q * kStats + 4]);
    }
  }
}

template <typename S>
__device__ void flow_chunk(const FlowArgs<S>& A, int j, double* wsum) {
  const int t = threadIdx.x;
  const int f = j * kFW + t;
  double v[kStats] = {0, 0, 0, 0, 0};
  if (f < A.P.nl) {
    wait_flag(A.flag + f, A.base, 3u, A.err);
    acquire();
    const double* p = A.partials + (size_t)f * kStats;
#pragma unroll
    for (int s = 0; s < kStats; ++s) v[s] = ld_c<true>(p + s);
  }
  block_reduce5(v, wsum);
  if (t == 0)
#pragma unroll
    for (int s = 0; s < kStats; ++s) st_c<true>(A.part2 + (size_t)j * kStats + s, v[s]);
  if (t < 64) release_flag(A.flag2 + j, A.base + 1u);
  __syncthreads();  // wsum reuse
}

template <typename S>
__device__ void flow_final(const FlowArgs<S>& A, double* wsum) {
  const int t = threadIdx.x;
  double v[kStats] = {0, 0, 0, 0, 0};
  for (int j = t; j < A.nr; j += kFW) {
    wait_flag(A.flag2 + j, A.base, 1u, A.err);
    acquire();
    const double* p = A.part2 + (size_t)j * kStats;
    v[0] += ld_c<true>(p + 0);
    v[1] += ld_c<true>(p + 1);
    v[2] += ld_c<true>(p + 2);
    v[3] = fmax(v[3], ld_c<true>(p + 3));
    v[4] = fmax(v[4], ld_c<true>(p + 4));
  }
  block_reduce5(v, wsum);
  if (t == 0) {
    // a bounded wait that gave up (now or earlier) poisons the statistics;
    // the host clears the error word before the next solve
    const bool bad = ld_flag(A.err) != 0u;
    const double nan = __builtin_nan("");
    const double al = (double)A.P.alpha;
    A.stats[0] = bad ? nan : v[3];
    A.stats[1] = bad ? nan : v[4];
    A.stats[2] = bad ? nan : v[0] + v[1] - 2.0 * al * v[2];
    A.stats[3] = bad ? nan : v[0];
    A.stats[4] = bad ? nan : v[1];
    A.stats[5] = bad ? nan : v[2];
  }
  __syncthreads();
}

// W: minimum wavefronts per SIMD the register allocation must allow (2:
// no spills; 4: twice the resident workgroups, some registers spilled).
template <typename S, int W>
__global__ void __launch_bounds__(kFW) __attribute__((amdgpu_waves_per_eu(W, 8))) k_T_flow(FlowArgs<S> A) {
  extern __shared__ __align__(16) unsigned flow_lds[];
  __shared__ double wsum[(kFW / 64) * kStats];
  const FlowLds L(A.P.nx, A.P.nu, A.nc, (int)(sizeof(S) / 4));
  const int nl = A.P.nl;
  // Items run in increasing order in every workgroup. After a forward item
  // wavefront 0 alone finishes the dual update; the other wavefronts go on
  // to the next item (its first barrier waits for wavefront 0), touching no
  // LDS the dual update uses.
  for (int it = blockIdx.x; it < A.items; it += gridDim.x) {
    if (it < nl) {
      flow_bwd<S>(A, L, flow_lds, nl - 1 - it);
    } else if (it < 2 * nl) {
      flow_fwd<S>(A, L, flow_lds, it - nl);
    } else if (it < 2 * nl + A.nr) {
      flow_chunk<S>(A, it - 2 * nl, wsum);
    } else {
      flow_final<S>(A, wsum);
    }
  }
}

}  // namespace

// LDS bytes of the dataflow launch with nc children per chunk.
int flow_lds_bytes(int nx, int nu, int nc, int elem) { return FlowLds(nx, nu, nc, elem / 4).bytes(); }

template <typename S>
const void* flow_kernel(int occ) {
  return occ >= 4 ? reinterpret_cast<const void*>(&k_T_flow<S, 4>) : reinterpret_cast<const void*>(&k_T_flow<S, 2>);
}
template const void* flow_kernel<double>(int);
template const void* flow_kernel<float>(int);

template <typename S>
hipError_t launch_T_flow(const Problem& P, const DevProb<S>& D, const S* z, const S* eta, S* zout, S* eout,
                         const double* x0, S* q, S* d, double* partials, double* stats, bool dual,
                         hipStream_t st) {
  const FlowState& F = P.flow;
  if (!F.flag || F.grid <= 0) return hipErrorInvalidValue;
  FlowArgs<S> A;
  A.P = D;
  A.z = z;
  A.eta = eta;
  A.zout = zout;
  A.eout = eout;
  A.x0 = x0;
  A.q = q;
  A.d = d;
  A.partials = partials;
  A.part2 = F.part2;
  A.stats = stats;
  A.flag = F.flag;
  A.flag2 = F.flag2;
  A.err = F.err;
  A.base = 4u * (unsigned)(P.flow_epoch++);
  A.nc = F.nc;
  A.nr = (P.tree->nl + kFW - 1) / kFW;
  A.dual = dual ? 1 : 0;
  A.items = 2 * P.tree->nl + (dual ? A.nr + 1 : 0);
  const int grid = std::min(F.grid, A.items);
  const size_t lds = (size_t)flow_lds_bytes(P.nx, P.nu, F.nc, (int)sizeof(S));
  void* args[] = {&A};
  return hipLaunchCooperativeKernel(flow_kernel<S>(F.occ), dim3(grid), dim3(kFW), args, (unsigned)lds, st);
}
template hipError_t launch_T_flow<double>(const Problem&, const DevProb<double>&, const double*, const double*,
                                          double*, double*, const double*, double*, double*, double*, double*,
                                          bool, hipStream_t);
template hipError_t launch_T_flow<float>(const Problem&, const DevProb<float>&, const float*, const float*,
                                         float*, float*, const double*, float*, float*, double*, double*, bool,
                                         hipStream_t);

}  // namespace spk
