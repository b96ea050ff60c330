// Dataflow form of the two Alg. 2 sweeps: both sweeps of one evaluation of
// T in ONE persistent launch, in place of 2N dependent per-stage launches
// and their dispatch latency. The fully parallel pre-pass (xbar, ubar, leaf
// seeds, S2) runs before it and the parallel post-pass (dual update and
// statistics) after it, as in the per-stage form.
//
// Work items: one per chunk of (at most nc) children of a family; the
// backward items come first, families in reverse breadth-first order (every
// child family comes first), then the forward items in breadth-first order
// (the parent comes first), the chunks of a family in increasing order.
// A family with several chunks has them on different workgroups at the same
// time: in the forward sweep each writes its own children's states; in the
// backward sweep each but the last publishes its partial sums
// sum_c At^c q^c and sum_c Bt^c q^c (the regrouped one-phase step below),
// which the last one adds, in chunk order, to its own before the family's
// step.
// Workgroup b runs items b, b + G, b + 2G, ... (G = grid size = the
// resident capacity: the occupancy query bounded by the build's register
// budget and by the LDS in 512-byte blocks; a cooperative launch guarantees
// residency, a plain one, the default, has it whenever the device runs
// nothing else). An item waits only on items with a smaller index, so the
// smallest unfinished item never waits and the launch drains.
//
// Values crossing workgroups (q and d of the backward step, x of the
// forward step) travel as tagged words: each 32-bit half of a value shares a
// 64-bit word with the launch epoch and is stored and loaded as one
// agent-coherent atomic (it bypasses the non-coherent per-XCD L2 lines). A
// consumer polls the data itself until every tag equals the epoch: no
// separate flag, no wait for store acknowledgements, no cache write-back or
// invalidation, and nothing is ever cleared (old epochs never match). Every
// poll loop is bounded: a loop that gives up raises an error word, later
// loops return at once, and the statistics of the evaluation come out as NaN
// (no wave ever spins without end).
//
// The matrices of an item, with its xbar/ubar rows (and the leaf seeds) from
// the pre-pass, are copied into LDS by direct global-to-LDS loads issued
// before the item's dependency wait: an item costs one HBM round trip, its
// wait, and one phase of LDS mat-vecs, cut into wavefront-uniform units
// (one output block and one input range per wavefront, lane = output).
#include "device_common.h"

#include <math.h>
#include <algorithm>

namespace spk {

namespace {

constexpr int kFW = 256;                   // threads per workgroup (4 wavefronts)

typedef __attribute__((address_space(3))) void lds_void;

// Word offsets of the dynamic LDS regions (32-bit words; every region is a
// whole number of 64-word rows so that a wavefront copy may overrun it).
// The mat-vec partial sums take 64 elements per unit of work, at most
// max(4, nc + 1) units per item.
struct FlowLds {
  int esz;     // words per element
  int sA, sB;  // per-child strides of the At / Abar and Bt / B regions
  int oA, oB, oR, oK, oQ, oX, oU, oRed;  // oK: P1 (backward) or K (forward)
  int nc;      // children per chunk
  int words;
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
    oQ = oK + pad(nx * nu * esz);  // children's q (chunk), row stride nx
    oX = oQ + pad(nc * nx * esz);  // xbar (backward) or x (forward)
    oU = oX + pad(nx * esz);       // ubar (backward) or d (forward)
    oRed = oU + pad(nu * esz);
    words = oRed + pad((nc + 1 > 4 ? nc + 1 : 4) * 64 * esz);
  }
  __host__ __device__ int bytes() const { return words * 4; }
};

// Copies nwords 32-bit words from global memory into LDS (dst = word
// offset, a multiple of 64). From a 16-byte aligned source, whole rows of
// 256 words go as 16 bytes per lane (lane l fills words 4l..4l+3 of the
// row); the rest (all of it from an unaligned source) goes in rows of 64
// words, 4 bytes per lane, lanes past the end re-reading the last word (in
// bounds) into the region's padding. Wavefront w issues rows w', w' + 4, ...
// (w' = w rotated by `rot`, so that small copies spread over the
// wavefronts).
__device__ __forceinline__ void dma_words(const void* src, unsigned* lds, int dst, int nwords, int rot) {
  const int lane = threadIdx.x & 63, w = ((threadIdx.x >> 6) + rot) & 3;
  // uniform base + 32-bit lane byte offset (scalar-base addressing)
  const char* s = static_cast<const char*>(src);
  int done = 0;
  if ((reinterpret_cast<uintptr_t>(src) & 15u) == 0) {
    const int rows = nwords >> 8;
    for (int r = w; r < rows; r += 4)
      __builtin_amdgcn_global_load_lds(s + (unsigned)((r * 256 + lane * 4) * 4), (lds_void*)(lds + dst + r * 256), 16, 0,
                                       0);
    done = rows << 8;
  }
  const int rest = nwords - done;
  for (int r = w; r * 64 < rest; r += 4) {
    int e = r * 64 + lane;
    e = e < rest ? e : rest - 1;
    __builtin_amdgcn_global_load_lds(s + (unsigned)((done + e) * 4), (lds_void*)(lds + dst + done + r * 64), 4, 0, 0);
  }
}

__device__ __forceinline__ void wait_vm() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

// Partial mat-vec from LDS: M input-major (element (out o, in k) at
// k * nout + o), v (nin) in LDS. Thread t < G * nout (g = t / nout,
// o = t % nout) sums the
// products of the inputs k in [g * kb, (g + 1) * kb), kb a multiple of 4:
// the vector is read four entries at a time, the matrix down one column
// with a single running address, into red[t] (added to it when acc).
// ---------------------------------------------------------------- mat-vec phase
// An item's products form output blocks (backward: q and d; forward: each
// child's x and, in chunk 0, u). Block b has n_b <= 64 outputs over an
// input of l_b entries, the concatenation of a head segment and equal
// segments (one matrix each, stored input-major: entry (k, o) at k n_b + o).
// A block is cut into contiguous input ranges, the units of work; a unit
// runs on one wavefront with lane o on output o, so that the lanes of a
// wavefront never diverge. Unit u writes its partial sums to red[64 u + o].

// a0 + a1 += sum over inputs k in [k0, k1) of M[k nout + o] v[k]
template <typename S>
__device__ __forceinline__ void dot_range(const S* M, const S* v, int nout, int o, int k0, int k1, S& a0, S& a1) {
  const S* mp = M + k0 * nout + o;
  int k = k0;
  for (; k + 4 <= k1; k += 4, mp += 4 * nout) {
    const S v0 = v[k], v1 = v[k + 1], v2 = v[k + 2], v3 = v[k + 3];
    const S m0 = mp[0], m1 = mp[nout], m2 = mp[2 * nout], m3 = mp[3 * nout];
    a0 += m0 * v0 + m2 * v2;
    a1 += m1 * v1 + m3 * v3;
  }
  for (; k < k1; ++k, mp += nout) a0 += mp[0] * v[k];
}

// Output o's sum over inputs [r0, r1) of the concatenation of a head
// segment (nh inputs: matrix Mh, vector vh) and cnt segments of ns inputs
// (segment k: matrix Ms + k ms, vector vs + k vk).
template <typename S>
__device__ __forceinline__ S dot_concat(const S* Mh, const S* vh, int nh, const S* Ms, int ms, const S* vs, int vk,
                                        int ns, int cnt, int nout, int o, int r0, int r1) {
  S a0 = 0, a1 = 0;
  if (r0 < nh) dot_range<S>(Mh, vh, nout, o, r0, min(r1, nh), a0, a1);
  r0 = max(r0 - nh, 0);
  r1 -= nh;
  for (int k = r0 / ns; k < cnt && k * ns < r1; ++k) {
    const int b = k * ns;
    dot_range<S>(Ms + k * ms, vs + k * vk, nout, o, max(r0 - b, 0), min(r1 - b, ns), a0, a1);
  }
  return a0 + a1;
}

// Input range of part p of a block of len inputs cut into P parts: [r0, r1)
// with ranges of a multiple of 4 inputs (the last one shorter, possibly empty).
__device__ __forceinline__ int part_len(int len, int P) { return (((len + P - 1) / P) + 3) & ~3; }

// Output o summed over the P units of a block, whose partial sums start at
// red, `stride` apart (unit order: even units, odd units, then the two added).
template <typename S>
__device__ __forceinline__ S fold_units(const S* red, int P, int o, int stride = 64) {
  S s0 = 0, s1 = 0;
  int p = 0;
  for (; p + 1 < P; p += 2) {
    s0 += red[p * stride + o];
    s1 += red[(p + 1) * stride + o];
  }
  if (p < P) s0 += red[p * stride + o];
  return s0 + s1;
}

// One child per chunk, narrow n_u: every range lies inside one segment, so
// the ranges of the n_u-output block share one wavefront as lane groups of
// n_u (same loop, per-lane base pointers). Half of n_x, rounded down to 4.
__device__ __forceinline__ int half4(int n) { return (n / 2) & ~3; }

__device__ __forceinline__ unsigned ld_flag(const unsigned* f) {
  return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}




// One wavefront polls the n tagged elements at src until all carry `tag`
// (bounded), copying the values to dst (LDS).
template <typename S>
__device__ __forceinline__ void wait_tagged(const unsigned long long* src, int n, unsigned tag, S* dst,
                                            unsigned* err, unsigned spin) {
  const int lane = threadIdx.x & 63;
  for (unsigned it = 0; it < spin; ++it) {
    bool ok = true;
    for (int e = lane; e < n; e += 64) {
      S v;
      ok = get_tagged<S>(src + (size_t)e * kTW<S>, tag, v) && ok;
      dst[e] = v;
    }
    if (__all(ok)) return;
    if ((it & 255u) == 255u && ld_flag(err) != 0u) return;
    __builtin_amdgcn_s_sleep(1);
  }
  __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Same for two sources at once (one memory round trip per poll).
template <typename S>
__device__ __forceinline__ void wait_tagged2(const unsigned long long* srcA, int nA, S* dstA,
                                             const unsigned long long* srcB, int nB, S* dstB, unsigned tag,
                                             unsigned* err, unsigned spin) {
  const int lane = threadIdx.x & 63;
  for (unsigned it = 0; it < spin; ++it) {
    bool ok = true;
    for (int e = lane; e < nA; e += 64) {
      S v;
      ok = get_tagged<S>(srcA + (size_t)e * kTW<S>, tag, v) && ok;
      dstA[e] = v;
    }
    for (int e = lane; e < nB; e += 64) {
      S v;
      ok = get_tagged<S>(srcB + (size_t)e * kTW<S>, tag, v) && ok;
      dstB[e] = v;
    }
    if (__all(ok)) return;
    if ((it & 255u) == 255u && ld_flag(err) != 0u) return;
    __builtin_amdgcn_s_sleep(1);
  }
  __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename S>
struct FlowArgs {
  DevProb<S> P;
  S* zout;
  const double* x0;
  const S* xbar;
  const S* ubar;
  const S* seeds;            // q of the leaf children (pre-pass), plain
  unsigned long long* qt;    // [nl][nx] tagged q
  unsigned long long* dt;    // [nl][nu] tagged d
  unsigned long long* xt;    // [nn][nx] tagged x (forward step of the parent)
  unsigned long long* pt;    // [slots][nx + nu] tagged partial sums of backward chunks
  const int* items;          // family * kChunkCodes + chunk: backward items, then forward
  const int* pbase;          // [nl] first partial slot of a family with several chunks
  unsigned* err;             // [1]
  unsigned tag;
  unsigned spin;             // polls of one bounded wait before it gives up
  int nc, nbwd, nitems;
};

// Sums, in slot order, entries ea and eb (-1: none) of the first n partial
// records at pp (stride rs elements), polled together by the calling thread
// until every word carries tag (bounded).
template <typename S>
__device__ __forceinline__ void sum_partials(const unsigned long long* pp, int n, int rs, int ea, int eb,
                                             unsigned tag, unsigned* err, unsigned spin, S& sa, S& sb) {
  for (unsigned it = 0; it < spin; ++it) {
    bool ok = true;
    S a = 0, b = 0;
    for (int q = 0; q < n; ++q) {
      S v;
      if (ea >= 0) {
        ok = get_tagged<S>(pp + ((size_t)q * rs + ea) * kTW<S>, tag, v) && ok;
        a += v;
      }
      if (eb >= 0) {
        ok = get_tagged<S>(pp + ((size_t)q * rs + eb) * kTW<S>, tag, v) && ok;
        b += v;
      }
    }
    if (ok) {
      sa = a;
      sb = b;
      return;
    }
    if ((it & 255u) == 255u && ld_flag(err) != 0u) return;
    __builtin_amdgcn_s_sleep(1);
  }
  __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- backward item
// Alg. 2 backward step in one mat-vec phase: substituting
// g = ubar - sum_c B^c' q^c into d = R~^{-1} g and q = M1 g - K' ubar - xbar
// + sum_c Abar^c' q^c (M1 = (K' + W) R~^{-1}) gives
//   d = R~^{-1} ubar + sum_c Bt^c q^c,   q = P1 ubar - xbar + sum_c At^c q^c
// with Bt^c = -R~^{-1} B^c', At^c = Abar^c' - M1 B^c', P1 = M1 - K' formed
// offline in FP64 (equal to Alg. 2's step in exact arithmetic).
// Chunk j of family i (children j nc, ...). Wavefront 3 polls the chunk's
// children's q while the copies are in flight. A chunk that is not the
// family's last publishes its two partial sums; the last chunk accumulates
// P1 ubar and R~^{-1} ubar with its children's products (same outputs, same
// partial-sum slots), adds the earlier chunks' partial sums (chunk order)
// and publishes d and q.
template <typename S>
__device__ void flow_bwd(const FlowArgs<S>& A, const FlowLds L, unsigned* lds, int i, int j) {
  const DevProb<S>& P = A.P;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  const int es = L.esz;
  S* M = reinterpret_cast<S*>(lds);
  const S* qv = reinterpret_cast<const S*>(lds + L.oQ);
  const S* xb = reinterpret_cast<const S*>(lds + L.oX);
  const S* ub = reinterpret_cast<const S*>(lds + L.oU);
  S* red = reinterpret_cast<S*>(lds + L.oRed);  // units q0, q1, d0, d1
  const bool leafkids = fc >= P.nl;
  const int k0 = j * L.nc, kc = min(L.nc, n - k0);
  const bool last = k0 + kc == n;
  int rot = 0;
  for (int k = 0; k < kc; ++k) {
    dma_words(P.AtR + (size_t)(fc + k0 + k) * nx * nx, lds, L.oA + k * L.sA, nx * nx * es, rot++);
    dma_words(P.BtR + (size_t)(fc + k0 + k) * nx * nu, lds, L.oB + k * L.sB, nx * nu * es, rot++);
  }
  if (last) {
    dma_words(P.Rinv + (size_t)i * nu * nu, lds, L.oR, nu * nu * es, rot++);
    dma_words(P.P1C + (size_t)i * nu * nx, lds, L.oK, nu * nx * es, rot++);
    dma_words(A.xbar + (size_t)i * nx, lds, L.oX, nx * es, rot++);
    dma_words(A.ubar + (size_t)i * nu, lds, L.oU, nu * es, rot++);
  }
  if (leafkids)  // seeds -xbar of the leaf children, written by the pre-pass
    dma_words(A.seeds + (size_t)(fc + k0) * nx, lds, L.oQ, kc * nx * es, rot++);
  else if (w == 3)  // children's q from their backward items
    wait_tagged<S>(A.qt + (size_t)(fc + k0) * nx * kTW<S>, kc * nx, A.tag, reinterpret_cast<S*>(lds + L.oQ), A.err, A.spin);
  wait_vm();
  __syncthreads();
  const bool narrow = kc == 1 && 3 * nu <= 64;
  if (narrow) {
    // three ranges per block: the last chunk's ubar and the two halves of
    // q^c, else the thirds of q^c; q block on wavefronts 0-2 (lane = output),
    // d block on wavefront 3 (lane group g of n_u lanes = range g)
    const int g = w < 3 ? w : lane / nu, o = w < 3 ? lane : lane - g * nu;
    const bool dblk = w == 3;
    const int h = half4(nx), k3 = part_len(nx, 3);
    const bool head = last && g == 0;
    const int ra = last ? (g == 2 ? h : 0) : g * k3;
    const int rb = last ? (g == 0 ? nu : g == 1 ? h : nx) : min(nx, ra + k3);
    const int nout = dblk ? nu : nx;
    const S* Mp = M + (head ? (dblk ? L.oR : L.oK) : (dblk ? L.oB : L.oA)) / es;
    if (o < nout && g < 3) {
      S a0 = 0, a1 = 0;
      dot_range<S>(Mp, head ? ub : qv, nout, o, ra, rb, a0, a1);
      red[(dblk ? 192 + g * nu : g * 64) + o] = a0 + a1;
    }
  } else {
    // q block [P1 | At^c ...] and d block [R~^{-1} | Bt^c ...] over
    // [ubar; q^c ...] (ubar only in the family's last chunk), two units each
    const int nh = last ? nu : 0, len = nh + kc * nx, kb = part_len(len, 2);
    const bool dblk = w >= 2;
    const int nout = dblk ? nu : nx, r0 = (w & 1) * kb;
    if (lane < nout)
      red[w * 64 + lane] = dot_concat<S>(M + (dblk ? L.oR : L.oK) / es, ub, nh, M + (dblk ? L.oB : L.oA) / es,
                                         (dblk ? L.sB : L.sA) / es, qv, nx, nx, kc, nout, lane, r0, min(len, r0 + kb));
  }
  __syncthreads();
  // q: units at red (stride 64); d: at red + 128 (stride 64) or red + 192 (stride n_u)
  const int nun = narrow ? 3 : 2;
  const S* redd = red + (narrow ? 192 : 128);
  const int dstr = narrow ? nu : 64;
  if (!last) {
    unsigned long long* pp = A.pt + (size_t)(A.pbase[i] + j) * (nx + nu) * kTW<S>;
    if (t < nx) put_tagged<S>(pp + (size_t)t * kTW<S>, fold_units<S>(red, nun, t), A.tag);
    if (t < nu) put_tagged<S>(pp + (size_t)(nx + t) * kTW<S>, fold_units<S>(redd, nun, t, dstr), A.tag);
    __syncthreads();  // LDS reuse by the next item
    return;
  }
  // this chunk's sums after the earlier chunks' (chunk order)
  const int nprev = k0 / L.nc;
  const unsigned long long* pp = nprev > 0 ? A.pt + (size_t)A.pbase[i] * (nx + nu) * kTW<S> : nullptr;
  S sa = 0, sb = 0;
  if (nprev > 0 && (t < nx || t < nu))
    sum_partials<S>(pp, nprev, nx + nu, t < nx ? t : -1, t < nu ? nx + t : -1, A.tag, A.err, A.spin, sa, sb);
  if (t < nx) put_tagged<S>(A.qt + ((size_t)i * nx + t) * kTW<S>, sa + fold_units<S>(red, nun, t) - xb[t], A.tag);
  if (t < nu) put_tagged<S>(A.dt + ((size_t)i * nu + t) * kTW<S>, sb + fold_units<S>(redd, nun, t, dstr), A.tag);
  __syncthreads();  // LDS reuse by the next item
}

// ---------------------------------------------------------------- forward item
// u = K x + d (chunk 0); x^c = Abar^c x + B^c d for the chunk's children;
// x^0 = x0 at the root. Wavefront 0 polls d (the family's backward step) and
// x (the parent's forward step) while the copies are in flight.
template <typename S>
__device__ void flow_fwd(const FlowArgs<S>& A, const FlowLds L, unsigned* lds, int i, int j) {
  const DevProb<S>& P = A.P;
  const Off<S> O(P);
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  const int es = L.esz;
  S* M = reinterpret_cast<S*>(lds);
  S* vx = reinterpret_cast<S*>(lds + L.oX);
  S* vd = reinterpret_cast<S*>(lds + L.oU);
  S* red = reinterpret_cast<S*>(lds + L.oRed);  // units: each child's, then u's
  const int k0 = j * L.nc, kc = min(L.nc, n - k0);
  int rot = 1;
  for (int k = 0; k < kc; ++k) {
    dma_words(P.AbC + (size_t)(fc + k0 + k) * nx * nx, lds, L.oA + k * L.sA, nx * nx * es, rot++);
    dma_words(P.BC + (size_t)(fc + k0 + k) * nu * nx, lds, L.oB + k * L.sB, nx * nu * es, rot++);
  }
  if (j == 0) dma_words(P.KC + (size_t)i * nx * nu, lds, L.oK, nx * nu * es, rot++);
  if (w == 0) {
    if (i != 0) {  // d and x polled together
      wait_tagged2<S>(A.dt + (size_t)i * nu * kTW<S>, nu, vd, A.xt + (size_t)i * nx * kTW<S>, nx, vx, A.tag, A.err, A.spin);
    } else {
      wait_tagged<S>(A.dt, nu, A.tag, vd, A.err, A.spin);
      if (lane < nx) {
        const S xv = (S)A.x0[lane];
        if (j == 0) A.zout[1 + lane] = xv;
        vx[lane] = xv;
      }
    }
  }
  wait_vm();
  __syncthreads();
  // child k: [Abar^c | B^c] [x; d] in Pc units; u (chunk 0): K x in Pu units.
  // Up to 4 blocks share the 4 wavefronts (the split with the shortest
  // longest range); more blocks take one unit each, the wavefronts in turn.
  const int lx = nx + nu;
  const bool narrow = kc == 1 && j == 0 && 2 * nu <= 64;
  int Pc = 1, Pu = j == 0 ? 1 : 0;
  if (narrow) {
    // x: ranges Abar x (two halves) and B d on wavefronts 0-2 (lane =
    // output); u: the two halves of K x on wavefront 3 (lane groups of n_u)
    Pc = 3;
    Pu = 0;
    const int h = half4(nx);
    const int g = w < 3 ? w : lane / nu, o = w < 3 ? lane : lane - g * nu;
    const int nout = w < 3 ? nx : nu;
    const bool bd = w < 3 && g == 2;  // the B d range
    const S* Mp = M + (w == 3 ? L.oK : bd ? L.oB : L.oA) / es;
    const int ra = bd ? 0 : (g == 1 ? h : 0);
    const int rb = bd ? nu : (g == 0 ? h : nx);
    if (o < nout && g < (w < 3 ? 3 : 2)) {
      S a0 = 0, a1 = 0;
      dot_range<S>(Mp, bd ? vd : vx, nout, o, ra, rb, a0, a1);
      red[(w < 3 ? g * 64 : 192 + g * nu) + o] = a0 + a1;
    }
  } else if (kc + Pu < 4) {
    if (j != 0) {
      Pc = 4 / kc;
    } else if (kc == 2) {
      Pu = 2;
    } else {
      int best = 1 << 30;
      for (int pc = 1; pc <= 3; ++pc) {
        const int m = max(part_len(lx, pc), part_len(nx, 4 - pc));
        if (m < best) {
          best = m;
          Pc = pc;
          Pu = 4 - pc;
        }
      }
    }
  }
  const int kbx = part_len(lx, Pc), kbu = Pu > 0 ? part_len(nx, Pu) : 0, nux = kc * Pc;
  for (int u = narrow ? 4 : w; u < nux + Pu; u += 4) {
    if (u < nux) {
      const int k = u / Pc, r0 = (u - k * Pc) * kbx;
      if (lane < nx)
        red[u * 64 + lane] = dot_concat<S>(M + L.oA / es + k * (L.sA / es), vx, nx, M + L.oB / es + k * (L.sB / es),
                                           0, vd, 0, nu, 1, nx, lane, r0, min(lx, r0 + kbx));
    } else {
      const int r0 = (u - nux) * kbu;
      if (lane < nu)
        red[u * 64 + lane] = dot_concat<S>(M + L.oK / es, vx, nx, M, 0, vx, 0, 1, 0, nu, lane, r0, min(nx, r0 + kbu));
    }
  }
  __syncthreads();
  if (j == 0 && t < nu)
    A.zout[O.u(i) + t] = (narrow ? fold_units<S>(red + 192, 2, t, nu) : fold_units<S>(red + nux * 64, Pu, t)) + vd[t];
  for (int k = 0; k < kc; ++k)
    if (t < nx) {
      const S xc = fold_units<S>(red + k * Pc * 64, Pc, t);
      A.zout[O.x(fc + k0 + k) + t] = xc;
      if (fc + k0 + k < P.nl) put_tagged<S>(A.xt + ((size_t)(fc + k0 + k) * nx + t) * kTW<S>, xc, A.tag);
    }
  __syncthreads();  // red and the matrices are reused by the next item
}

// W: wavefronts per SIMD the register allocation targets (4 to 7).
template <typename S, int W>
__global__ void __launch_bounds__(kFW) __attribute__((amdgpu_waves_per_eu(W, W))) k_T_flow(FlowArgs<S> A) {
  extern __shared__ __align__(16) unsigned flow_lds[];
  const FlowLds L(A.P.nx, A.P.nu, A.nc, (int)(sizeof(S) / 4));
  // items run in increasing order in every workgroup: its backward items,
  // then its forward items (two loops, so that the two kinds of item do not
  // hold registers at the same time)
  int it = blockIdx.x;
  for (; it < A.nbwd; it += gridDim.x) {
    const int code = A.items[it];
    flow_bwd<S>(A, L, flow_lds, code / kChunkCodes, code % kChunkCodes);
  }
  for (; it < A.nitems; it += gridDim.x) {
    const int code = A.items[it];
    flow_fwd<S>(A, L, flow_lds, code / kChunkCodes, code % kChunkCodes);
  }
}

}  // namespace

// LDS bytes of the dataflow launch with nc children per chunk.
int flow_lds_bytes(int nx, int nu, int nc, int elem) { return FlowLds(nx, nu, nc, elem / 4).bytes(); }

template <typename S>
const void* flow_kernel(int occ) {
  switch (occ) {
    case 7: return reinterpret_cast<const void*>(&k_T_flow<S, 7>);
    case 6: return reinterpret_cast<const void*>(&k_T_flow<S, 6>);
    case 5: return reinterpret_cast<const void*>(&k_T_flow<S, 5>);
    default: return reinterpret_cast<const void*>(&k_T_flow<S, 4>);
  }
}
template const void* flow_kernel<double>(int);
template const void* flow_kernel<float>(int);

template <typename S>
hipError_t launch_sweeps_flow(const Problem& P, const DevProb<S>& D, S* zout, const double* x0, const S* xbar,
                              const S* ubar, S* q, S* d, hipStream_t st) {
  const FlowState& F = P.flow;
  if (!F.qt || F.grid <= 0) return hipErrorInvalidValue;
  FlowArgs<S> A;
  A.P = D;
  A.zout = zout;
  A.x0 = x0;
  A.xbar = xbar;
  A.ubar = ubar;
  A.seeds = q;
  (void)d;
  A.qt = F.qt;
  A.dt = F.dt;
  A.xt = F.xt;
  A.pt = F.pt;
  A.items = F.items;
  A.pbase = F.pbase;
  A.err = F.err;
  A.spin = F.spin;
  if (++P.flow_epoch == 0u) P.flow_epoch = 1u;  // tag 0 is the cleared state
  A.tag = P.flow_epoch;
  A.nc = F.nc;
  A.nbwd = F.nbwd;
  A.nitems = 2 * F.nbwd;
  const int grid = std::min(F.grid, A.nitems);
  const size_t lds = (size_t)flow_lds_bytes(P.nx, P.nu, F.nc, (int)sizeof(S));
  void* args[] = {&A};
  if (F.coop) return hipLaunchCooperativeKernel(flow_kernel<S>(F.occ), dim3(grid), dim3(kFW), args, (unsigned)lds, st);
  // plain launch of a grid sized to the resident capacity (every wait is
  // bounded, so a grid that were not all resident ends with the error word
  // set, never hangs)
  return hipLaunchKernel(flow_kernel<S>(F.occ), dim3(grid), dim3(kFW), args, lds, st);
}
template hipError_t launch_sweeps_flow<double>(const Problem&, const DevProb<double>&, double*, const double*,
                                               const double*, const double*, double*, double*, hipStream_t);
template hipError_t launch_sweeps_flow<float>(const Problem&, const DevProb<float>&, float*, const double*,
                                              const float*, const float*, float*, float*, hipStream_t);

}  // namespace spk
