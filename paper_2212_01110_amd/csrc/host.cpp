// Host side of the SPOCK library: tree validation, the offline factorisation
// of Alg. 1 in FP64, ||L|| from the block-diagonal structure of L, the device
// layout, and the host-driven CP / SPOCK iteration (section 3, Alg. 3) built
// on the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <thread>
#include <vector>

#include "spock_internal.h"

using namespace spk;

struct spock_tree {
  Tree t;
};
struct spock_problem {
  Problem p;
};

namespace {

#define HIP_TRY(x)                          \
  do {                                      \
    if ((x) != hipSuccess) return SPOCK_EHIP; \
  } while (0)

int next_pow2_team(int v) {
  int t = 8;
  while (t < v && t < 64) t <<= 1;
  return t;
}

template <typename S>
S* align_ptr(char*& cur, size_t count) {
  uintptr_t a = reinterpret_cast<uintptr_t>(cur);
  a = (a + 255) & ~uintptr_t(255);
  S* out = reinterpret_cast<S*>(a);
  cur = reinterpret_cast<char*>(a + count * sizeof(S));
  return out;
}

// Builds the device layout of precision S from the FP64 factorisation.
template <typename S>
int upload(Problem& P, const spock_problem_data& d, const std::vector<double>& Abar,
           const std::vector<double>& K, const std::vector<double>& Rinv, const std::vector<double>& W) {
  const Tree& T = *P.tree;
  const int nn = T.nn, nl = T.nl, nx = P.nx, nu = P.nu;
  // sizes (elements)
  const size_t nvec = (size_t)nn * (4 * nx + 3 * nu) + 2 * (size_t)nn + 64;
  const size_t nmat = (size_t)nn * (3 * nx * nx + 3 * nx * nu) + (size_t)nl * (2 * nu * nx + nu * nu + 3 * nx * nu);
  const size_t bytes = (nvec + nmat) * sizeof(S) + (3 * (size_t)nn + T.N + 2 + 4 * ((size_t)nl + 2)) * sizeof(int) +
                       (size_t)nn * sizeof(long long) + 72 * 256;
  std::vector<char> host(bytes, 0);
  void* dmem = nullptr;
  if (hipMalloc(&dmem, bytes) != hipSuccess) return SPOCK_ENOMEM;
  // Offsets are aligned relative to the start of the block, so a host
  // pointer and its device twin sit at the same offset.
  size_t off = 0;
  auto take = [&](size_t count, auto tag) {
    using U = decltype(tag);
    off = (off + 255) & ~size_t(255);
    U* h = reinterpret_cast<U*>(host.data() + off);
    U* dv = reinterpret_cast<U*>(static_cast<char*>(dmem) + off);
    off += count * sizeof(U);
    return std::make_pair(h, dv);
  };
  DevProb<S> D{};
  D.nn = nn; D.nl = nl; D.nx = nx; D.nu = nu; D.N = T.N;
  D.nz = P.nz; D.neta = P.neta;
  D.zU = 1 + (long long)nn * nx;
  D.zZ2 = D.zU + (long long)nl * nu;
  D.eE2 = 2LL * (nn - 1) + (long long)nl * (2 + nx + nu);
  D.eE3 = D.eE2 + (long long)(nn - 1) * (nx + nu + 2);
  D.alpha = (S)P.alpha;
  auto fcp = take(nn, int{});
  auto nchp = take(nn, int{});
  auto ancp = take(nn, int{});
  auto sop = take(T.N + 2, int{});
  for (int t = 0; t < T.N + 2; ++t) sop.first[t] = T.stage_off[t];
  P.d_stage_off = sop.second;
  for (int i = 0; i < nn; ++i) {
    fcp.first[i] = T.fc[i];
    nchp.first[i] = T.nch[i];
    ancp.first[i] = T.anc[i];
  }
  D.fc = fcp.second; D.nch = nchp.second; D.anc = ancp.second;
  // slot of s^c in its ancestor's z2 block (y 2n+1, tau n, s n), for the
  // flat post-pass
  {
    auto sp = take(nn, 0LL);
    sp.first[0] = 0;
    for (int c = 1; c < nn; ++c) {
      const int a = T.anc[c];
      const long long z2a = D.zZ2 + 4LL * (T.fc[a] - 1) + a;
      sp.first[c] = z2a + 3LL * T.nch[a] + 1 + (c - T.fc[a]);
    }
    P.d_spos = sp.second;
  }
  {
    const char* pm = std::getenv("SPOCK_POST");
    P.post_flat = pm && std::string(pm) == "flat";
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
      P.ncu = ncu;
    P.flat_bpc = flat_post_occupancy<S>();
  }
  // block tables of the node-parallel post-pass (one per team size); a
  // table is dropped when its LDS (per team 3 VM, per child slot nx + nu)
  // would exceed 64 KiB, and all are dropped under SPOCK_POST=family
  {
    const char* pm = std::getenv("SPOCK_POST");
    const bool family_only = pm && std::string(pm) == "family";
    int maxnch = 1;
    for (int i = 0; i < nl; ++i) maxnch = std::max(maxnch, T.nch[i]);
    const int VM = (std::max(nx, nu) + 3) & ~3;
    std::vector<int> bf;
    for (int k = 0; k < 4; ++k) {
      const int tpb = 256 >> (3 + k);
      const int cap = std::max(tpb, maxnch);
      const size_t lds = ((size_t)tpb * 3 * VM + (size_t)cap * (nx + nu)) * sizeof(S);
      P.pblk_n[k] = 0;
      P.pblk_cap[k] = cap;
      P.d_pblk[k] = nullptr;
      if (family_only || lds > 65536) continue;
      const int nb = build_post_blocks(T, cap, bf);
      auto tb = take((size_t)nb + 1, int{});
      std::copy(bf.begin(), bf.end(), tb.first);
      P.d_pblk[k] = tb.second;
      P.pblk_n[k] = nb;
    }
  }
  auto pp = take(nn, S{});
  auto ap = take(nn, S{});
  for (int i = 0; i < nn; ++i) {
    pp.first[i] = (S)T.pcond[i];
    ap.first[i] = d.a_risk ? (S)d.a_risk[i] : S(0);
  }
  D.p = pp.second; D.a = ap.second;
  auto sqp = take((size_t)nn * nx, S{});
  auto sqNp = take((size_t)nn * nx, S{});
  auto xlop = take((size_t)nn * nx, S{});
  auto xhip = take((size_t)nn * nx, S{});
  auto srp = take((size_t)nn * nu, S{});
  auto ulop = take((size_t)nn * nu, S{});
  auto uhip = take((size_t)nn * nu, S{});
  // (general problems carry their constraints elsewhere; their boxes may be absent)
  const S inf = std::numeric_limits<S>::infinity();
  for (size_t e = 0; e < (size_t)nn * nx; ++e) {
    sqp.first[e] = (S)std::sqrt(d.q[e]);
    sqNp.first[e] = (S)std::sqrt(d.qN[e]);
    xlop.first[e] = d.xmin ? (S)d.xmin[e] : -inf;
    xhip.first[e] = d.xmax ? (S)d.xmax[e] : inf;
  }
  for (size_t e = 0; e < (size_t)nn * nu; ++e) {
    srp.first[e] = (S)std::sqrt(d.r[e]);
    ulop.first[e] = d.umin ? (S)d.umin[e] : -inf;
    uhip.first[e] = d.umax ? (S)d.umax[e] : inf;
  }
  D.sq = sqp.second; D.sqN = sqNp.second; D.xlo = xlop.second; D.xhi = xhip.second;
  D.sr = srp.second; D.ulo = ulop.second; D.uhi = uhip.second;
  auto AbRp = take((size_t)nn * nx * nx, S{});
  auto AbCp = take((size_t)nn * nx * nx, S{});
  auto BRp = take((size_t)nn * nx * nu, S{});
  auto BCp = take((size_t)nn * nx * nu, S{});
  for (int c = 1; c < nn; ++c) {
    const double* Ab = Abar.data() + (size_t)c * nx * nx;
    const double* Bm = d.B + (size_t)c * nx * nu;
    S* r1 = AbRp.first + (size_t)c * nx * nx;
    S* c1 = AbCp.first + (size_t)c * nx * nx;
    for (int r = 0; r < nx; ++r)
      for (int k = 0; k < nx; ++k) {
        r1[(size_t)r * nx + k] = (S)Ab[(size_t)r * nx + k];
        c1[(size_t)k * nx + r] = (S)Ab[(size_t)r * nx + k];
      }
    S* r2 = BRp.first + (size_t)c * nx * nu;
    S* c2 = BCp.first + (size_t)c * nx * nu;
    for (int r = 0; r < nx; ++r)
      for (int j = 0; j < nu; ++j) {
        r2[(size_t)r * nu + j] = (S)Bm[(size_t)r * nu + j];
        c2[(size_t)j * nx + r] = (S)Bm[(size_t)r * nu + j];
      }
  }
  D.AbR = AbRp.second; D.AbC = AbCp.second; D.BR = BRp.second; D.BC = BCp.second;
  auto KRp = take((size_t)nl * nu * nx, S{});
  auto KCp = take((size_t)nl * nu * nx, S{});
  auto Rip = take((size_t)nl * nu * nu, S{});
  auto WCp = take((size_t)nl * nu * nx, S{});
  for (int i = 0; i < nl; ++i) {
    const double* Km = K.data() + (size_t)i * nu * nx;     // [nu][nx]
    const double* Wm = W.data() + (size_t)i * nx * nu;     // [nx][nu]
    for (int j = 0; j < nu; ++j)
      for (int k = 0; k < nx; ++k) {
        KRp.first[(size_t)i * nu * nx + (size_t)j * nx + k] = (S)Km[(size_t)j * nx + k];
        KCp.first[(size_t)i * nu * nx + (size_t)k * nu + j] = (S)Km[(size_t)j * nx + k];
      }
    for (int e = 0; e < nu * nu; ++e) Rip.first[(size_t)i * nu * nu + e] = (S)Rinv[(size_t)i * nu * nu + e];
    for (int r = 0; r < nx; ++r)
      for (int j = 0; j < nu; ++j) WCp.first[(size_t)i * nu * nx + (size_t)j * nx + r] = (S)Wm[(size_t)r * nu + j];
  }
  D.KR = KRp.second; D.KC = KCp.second; D.Rinv = Rip.second; D.WC = WCp.second;
  // M1 = (K' + W) R~^{-1} (n_x x n_u, FP64): with g = ubar - sum_c B^c' q^c,
  // the backward step is d = R~^{-1} g, q = M1 g - K' ubar - xbar + sum_c Abar^c' q^c
  // (the same recursion regrouped); stored like W
  auto M1p = take((size_t)nl * nu * nx, S{});
  auto P1p = take((size_t)nl * nu * nx, S{});
  std::vector<double> M1d((size_t)nl * nx * nu);  // M1[r][j], FP64
  parallel_for(nl, [&](int i) {
    const double* Km = K.data() + (size_t)i * nu * nx;  // [nu][nx]
    const double* Wm = W.data() + (size_t)i * nx * nu;  // [nx][nu]
    const double* Ri = Rinv.data() + (size_t)i * nu * nu;
    for (int r = 0; r < nx; ++r)
      for (int j = 0; j < nu; ++j) {
        double acc = 0;
        for (int l = 0; l < nu; ++l) acc += (Km[(size_t)l * nx + r] + Wm[(size_t)r * nu + l]) * Ri[(size_t)l * nu + j];
        M1d[(size_t)i * nx * nu + (size_t)r * nu + j] = acc;
        M1p.first[(size_t)i * nu * nx + (size_t)j * nx + r] = (S)acc;
        P1p.first[(size_t)i * nu * nx + (size_t)j * nx + r] = (S)(acc - Km[(size_t)j * nx + r]);
      }
  });
  D.M1C = M1p.second;
  D.P1C = P1p.second;
  // per child c of family i: At^c = Abar^c' - M1 B^c' (element (out o, in k)
  // at k nx + o), Bt^c = -R~^{-1} B^c' (element (out o, in k) at k nu + o)
  auto AtRp = take((size_t)nn * nx * nx, S{});
  auto BtRp = take((size_t)nn * nx * nu, S{});
  parallel_for(nn - 1, [&](int c1) {
    const int c = c1 + 1, i = T.anc[c];
    const double* Ab = Abar.data() + (size_t)c * nx * nx;  // Abar[k][o]
    const double* Bm = d.B + (size_t)c * nx * nu;          // B[k][j]
    const double* M1 = M1d.data() + (size_t)i * nx * nu;   // M1[o][j]
    const double* Ri = Rinv.data() + (size_t)i * nu * nu;  // R~^{-1}[o][j]
    for (int k = 0; k < nx; ++k) {
      for (int o = 0; o < nx; ++o) {
        double acc = Ab[(size_t)k * nx + o];
        for (int j = 0; j < nu; ++j) acc -= M1[(size_t)o * nu + j] * Bm[(size_t)k * nu + j];
        AtRp.first[(size_t)c * nx * nx + (size_t)k * nx + o] = (S)acc;
      }
      for (int o = 0; o < nu; ++o) {
        double acc = 0;
        for (int j = 0; j < nu; ++j) acc += Ri[(size_t)o * nu + j] * Bm[(size_t)k * nu + j];
        BtRp.first[(size_t)c * nx * nu + (size_t)k * nu + o] = (S)(-acc);
      }
    }
  });
  D.AtR = AtRp.second;
  D.BtR = BtRp.second;
  const size_t used = off;
  if (used > bytes) {
    (void)hipFree(dmem);
    return SPOCK_ENOMEM;
  }
  if (hipMemcpy(dmem, host.data(), used, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(dmem);
    return SPOCK_EHIP;
  }
  // Read the tree index arrays back: every kernel indexes through them.
  {
    std::vector<int> chk(3 * (size_t)nn);
    if (hipMemcpy(chk.data(), D.fc, nn * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(chk.data() + nn, D.nch, nn * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(chk.data() + 2 * nn, D.anc, nn * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipFree(dmem);
      return SPOCK_EHIP;
    }
    for (int i = 0; i < nn; ++i)
      if (chk[i] != T.fc[i] || chk[nn + i] != T.nch[i] || chk[2 * nn + i] != T.anc[i]) {
        (void)hipFree(dmem);
        return SPOCK_EHIP;
      }
  }
  P.dmem = dmem;
  if constexpr (sizeof(S) == 8) P.dp64 = D; else P.dp32 = D;
  return SPOCK_OK;
}

// Device data of a general problem (layout G from build_general): offsets,
// E, b, the S2 projectors and the constraint rows (the identity rows and
// bounds of the boxes when d has no constraint data).
template <typename S>
int upload_general(Problem& P, const spock_problem_data& d, const GeneralLayout& GL) {
  const Tree& T = *P.tree;
  const int nn = T.nn, nl = T.nl, nx = P.nx, nu = P.nu, nc = GL.nc, ncN = GL.ncN, nleaf = nn - nl;
  // constraint rows as arrays (boxes: Gamma = identity)
  std::vector<double> Gx((size_t)nl * nc * nx, 0.0), Gu((size_t)nl * nc * nu, 0.0), cmin((size_t)nl * nc),
      cmax((size_t)nl * nc), GN((size_t)nleaf * ncN * nx, 0.0), cNmin((size_t)nleaf * ncN), cNmax((size_t)nleaf * ncN);
  const spock_constraint_data* C = d.cons;
  for (int i = 0; i < nl; ++i) {
    if (C) {
      std::copy(C->Gx + (size_t)i * nc * nx, C->Gx + (size_t)(i + 1) * nc * nx, Gx.begin() + (size_t)i * nc * nx);
      std::copy(C->Gu + (size_t)i * nc * nu, C->Gu + (size_t)(i + 1) * nc * nu, Gu.begin() + (size_t)i * nc * nu);
      std::copy(C->cmin + (size_t)i * nc, C->cmin + (size_t)(i + 1) * nc, cmin.begin() + (size_t)i * nc);
      std::copy(C->cmax + (size_t)i * nc, C->cmax + (size_t)(i + 1) * nc, cmax.begin() + (size_t)i * nc);
    } else {
      for (int o = 0; o < nx; ++o) {
        Gx[((size_t)i * nc + o) * nx + o] = 1.0;
        cmin[(size_t)i * nc + o] = d.xmin[(size_t)i * nx + o];
        cmax[(size_t)i * nc + o] = d.xmax[(size_t)i * nx + o];
      }
      for (int o = 0; o < nu; ++o) {
        Gu[((size_t)i * nc + nx + o) * nu + o] = 1.0;
        cmin[(size_t)i * nc + nx + o] = d.umin[(size_t)i * nu + o];
        cmax[(size_t)i * nc + nx + o] = d.umax[(size_t)i * nu + o];
      }
    }
  }
  for (int j = nl; j < nn; ++j) {
    const size_t l = (size_t)(j - nl);
    if (C) {
      std::copy(C->GN + (size_t)j * ncN * nx, C->GN + (size_t)(j + 1) * ncN * nx, GN.begin() + l * ncN * nx);
      std::copy(C->cNmin + (size_t)j * ncN, C->cNmin + (size_t)(j + 1) * ncN, cNmin.begin() + l * ncN);
      std::copy(C->cNmax + (size_t)j * ncN, C->cNmax + (size_t)(j + 1) * ncN, cNmax.begin() + l * ncN);
    } else {
      for (int o = 0; o < nx; ++o) {
        GN[(l * ncN + o) * nx + o] = 1.0;
        cNmin[l * ncN + o] = d.xmin[(size_t)j * nx + o];
        cNmax[l * ncN + o] = d.xmax[(size_t)j * nx + o];
      }
    }
  }
  // one block: 64-bit offsets, 32-bit counts, then the S arrays
  std::vector<char> host;
  size_t off = 0;
  std::vector<std::pair<size_t, size_t>> parts;  // (offset, bytes)
  auto place = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    parts.push_back({off, bytes});
    off += bytes;
    return parts.size() - 1;
  };
  std::vector<double> Qh, Rh, QNh;
  if (d.Qm) dense_cost_roots(T, d, Qh, Rh, QNh);
  const size_t i_Qh = place(sizeof(S) * Qh.size()), i_Rh = place(sizeof(S) * Rh.size()),
               i_QNh = place(sizeof(S) * QNh.size());
  const size_t i_z2 = place(8 * nl), i_e1 = place(8 * nl), i_Eo = place(8 * nl), i_yo = place(8 * nl),
               i_Po = place(8 * nl), i_ny = place(4 * nl), i_kp = place(4 * nl),
               i_E = place(sizeof(S) * GL.E.size()), i_b = place(sizeof(S) * GL.b.size()),
               i_P = place(sizeof(S) * GL.PS2.size()), i_Gx = place(sizeof(S) * Gx.size()),
               i_Gu = place(sizeof(S) * Gu.size()), i_cmin = place(sizeof(S) * cmin.size()),
               i_cmax = place(sizeof(S) * cmax.size()), i_GN = place(sizeof(S) * GN.size()),
               i_cNmin = place(sizeof(S) * cNmin.size()), i_cNmax = place(sizeof(S) * cNmax.size());
  host.assign(off + 256, 0);
  auto put64 = [&](size_t k, const std::vector<long long>& v) { std::memcpy(host.data() + parts[k].first, v.data(), 8 * v.size()); };
  auto put32 = [&](size_t k, const std::vector<int>& v) { std::memcpy(host.data() + parts[k].first, v.data(), 4 * v.size()); };
  auto putS = [&](size_t k, const std::vector<double>& v) {
    S* dst = reinterpret_cast<S*>(host.data() + parts[k].first);
    for (size_t e = 0; e < v.size(); ++e) dst[e] = (S)v[e];
  };
  put64(i_z2, GL.z2off);
  put64(i_e1, GL.e1off);
  put64(i_Eo, GL.Eoff);
  put64(i_yo, GL.yoff);
  put64(i_Po, GL.Poff);
  put32(i_ny, GL.ny);
  put32(i_kp, GL.kpos);
  putS(i_E, GL.E);
  putS(i_b, GL.b);
  putS(i_P, GL.PS2);
  putS(i_Gx, Gx);
  putS(i_Gu, Gu);
  putS(i_cmin, cmin);
  putS(i_cmax, cmax);
  putS(i_GN, GN);
  putS(i_cNmin, cNmin);
  putS(i_cNmax, cNmax);
  putS(i_Qh, Qh);
  putS(i_Rh, Rh);
  putS(i_QNh, QNh);
  void* mem = nullptr;
  if (hipMalloc(&mem, host.size()) != hipSuccess) return SPOCK_ENOMEM;
  if (hipMemcpy(mem, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(mem);
    return SPOCK_EHIP;
  }
  char* base = static_cast<char*>(mem);
  GenDev<S> G;
  G.nc = nc;
  G.ncN = ncN;
  G.eE2 = GL.eE2;
  G.eE3 = GL.eE3;
  G.z2off = reinterpret_cast<const long long*>(base + parts[i_z2].first);
  G.e1off = reinterpret_cast<const long long*>(base + parts[i_e1].first);
  G.Eoff = reinterpret_cast<const long long*>(base + parts[i_Eo].first);
  G.yoff = reinterpret_cast<const long long*>(base + parts[i_yo].first);
  G.Poff = reinterpret_cast<const long long*>(base + parts[i_Po].first);
  G.ny = reinterpret_cast<const int*>(base + parts[i_ny].first);
  G.kpos = reinterpret_cast<const int*>(base + parts[i_kp].first);
  G.E = reinterpret_cast<const S*>(base + parts[i_E].first);
  G.b = reinterpret_cast<const S*>(base + parts[i_b].first);
  G.PS2 = reinterpret_cast<const S*>(base + parts[i_P].first);
  G.Gx = reinterpret_cast<const S*>(base + parts[i_Gx].first);
  G.Gu = reinterpret_cast<const S*>(base + parts[i_Gu].first);
  G.cmin = reinterpret_cast<const S*>(base + parts[i_cmin].first);
  G.cmax = reinterpret_cast<const S*>(base + parts[i_cmax].first);
  G.GN = reinterpret_cast<const S*>(base + parts[i_GN].first);
  G.cNmin = reinterpret_cast<const S*>(base + parts[i_cNmin].first);
  G.cNmax = reinterpret_cast<const S*>(base + parts[i_cNmax].first);
  if (d.Qm) {
    G.Qh = reinterpret_cast<const S*>(base + parts[i_Qh].first);
    G.Rh = reinterpret_cast<const S*>(base + parts[i_Rh].first);
    G.QNh = reinterpret_cast<const S*>(base + parts[i_QNh].first);
  }
  P.gmem = mem;
  P.general = true;
  if constexpr (sizeof(S) == 8) P.gd64 = G; else P.gd32 = G;
  return SPOCK_OK;
}

// Family-to-lane mapping: team size (or kTeamWG), the first stage walked by
// subtree-owning workgroups (kTeamWG only; N = none), and the offsets of the
// forward-sweep statistic records of every launch.
void set_mapping(Problem& P, int team, int cut) {
  const Tree& T = *P.tree;
  P.team = team;
  P.teams_per_block = (team == kTeamWG || team == kTeamFlow) ? 1 : 256 / team;
  P.cut = (team == kTeamWG) ? std::max(cut, std::max(0, T.N - 64)) : T.N;
  if (P.cut > T.N) P.cut = T.N;
}

// Default cut: the first stage with at least 256 nodes (enough subtrees to
// fill the device), or none.
int default_cut(const Tree& T) {
  for (int t = 0; t < T.N; ++t)
    if (T.stage_off[t + 1] - T.stage_off[t] >= 256) return t;
  return T.N;
}

// LDS bytes per block of a mapping (team kernels size their LDS at launch).
size_t mapping_lds(const Problem& P, int team, size_t elem) {
  if (team == kTeamWG || team == kTeamFlow) return 0;
  const int VM = (std::max(P.nx, P.nu) + 3) & ~3;
  return (size_t)(256 / team) * 5 * VM * elem + kStats * 256 * sizeof(double);
}

}  // namespace

// ============================================================== tree
extern "C" int spock_tree_create(int32_t nn, const int32_t* anc, const double* prob, spock_tree** out) {
  if (!out) return SPOCK_EINVAL;
  Tree T;
  const int rc = build_tree(nn, anc, prob, T);
  if (rc) return rc;
  spock_tree* h = new (std::nothrow) spock_tree;
  if (!h) return SPOCK_ENOMEM;
  h->t = std::move(T);
  *out = h;
  return SPOCK_OK;
}

extern "C" int spock_tree_destroy(spock_tree* t) {
  if (!t) return SPOCK_EINVAL;
  delete t;
  return SPOCK_OK;
}

extern "C" int spock_tree_shape(const spock_tree* t, int32_t* N, int32_t* nl, int32_t* nleaf) {
  if (!t) return SPOCK_EINVAL;
  if (N) *N = t->t.N;
  if (nl) *nl = t->t.nl;
  if (nleaf) *nleaf = t->t.nn - t->t.nl;
  return SPOCK_OK;
}

// ============================================================== problem
extern "C" int spock_problem_factor(const spock_tree* th, const spock_problem_data* d, spock_problem** out) {
  if (!th || !d || !out) return SPOCK_EINVAL;
  const Tree& T = th->t;
  const int nn = T.nn, nl = T.nl, nx = d->nx, nu = d->nu;
  if (nx < 1 || nu < 1) return SPOCK_EINVAL;
  if (nx > kMaxDim || nu > kMaxDim) return SPOCK_EUNSUPPORTED;
  if (d->precision != SPOCK_FP64 && d->precision != SPOCK_FP32) return SPOCK_EINVAL;
  const bool dense = d->Qm || d->Rm || d->QNm;
  if (!d->A || !d->B || (!dense && (!d->q || !d->r || !d->qN))) return SPOCK_EINVAL;
  {
    const int rc = check_problem_data(T, *d);
    if (rc) return rc;
  }
  // dense costs: their diagonals stand in where a diagonal is stored (the
  // special-form arrays, which the general kernels do not read)
  spock_problem_data dd = *d;
  std::vector<double> qdiag, rdiag, qNdiag;
  if (dense) {
    qdiag.assign((size_t)nn * nx, 0.0);
    rdiag.assign((size_t)nn * nu, 0.0);
    qNdiag.assign((size_t)nn * nx, 0.0);
    for (int c = 0; c < nn; ++c) {
      for (int o = 0; o < nx; ++o) {
        qdiag[(size_t)c * nx + o] = std::max(0.0, d->Qm[((size_t)c * nx + o) * nx + o]);
        qNdiag[(size_t)c * nx + o] = std::max(0.0, d->QNm[((size_t)c * nx + o) * nx + o]);
      }
      for (int o = 0; o < nu; ++o) rdiag[(size_t)c * nu + o] = std::max(0.0, d->Rm[((size_t)c * nu + o) * nu + o]);
    }
    dd.q = qdiag.data();
    dd.r = rdiag.data();
    dd.qN = qNdiag.data();
  }
  d = &dd;
  // general conic risk, polyhedral constraints or dense costs: the general
  // layout, S2 projectors and kernels
  const bool general = d->risk || d->cons || dense;
  GeneralLayout GL;
  if (general) {
    const int rc = build_general(T, *d, kGenMaxBlock, GL);
    if (rc) return rc;
  }
  // ---- Alg. 1, FP64
  Factor fac;
  if (factor_alg1(T, *d, fac) != SPOCK_OK) return SPOCK_EFACTOR;
  const std::vector<double>& Abar = fac.Abar;
  const std::vector<double>& K = fac.K;
  const std::vector<double>& Rinv = fac.Rinv;
  const std::vector<double>& W = fac.W;
  // ---- ||L||: block-diagonal after a column permutation; closed forms per block
  const double normL = general ? norm_L_general(T, *d, GL) : norm_L_blocks(T, *d);
  double alpha = d->alpha;
  if (alpha <= 0.0) alpha = 0.99 / normL;
  else if (!(alpha * normL < 1.0)) return SPOCK_EINVAL;

  spock_problem* h = new (std::nothrow) spock_problem;
  if (!h) return SPOCK_ENOMEM;
  Problem& P = h->p;
  P.tree = &T;
  P.precision = d->precision;
  P.nx = nx;
  P.nu = nu;
  P.nz = 1 + (long long)nn * nx + (long long)nl * nu + 4LL * (nn - 1) + nl;
  P.neta = 2LL * (nn - 1) + 2LL * nl + (long long)nl * (nx + nu) + (long long)(nn - 1) * (nx + nu + 2) +
           (long long)(nn - nl) * (2 * nx + 2);
  if (general) {
    P.nz = GL.nz;
    P.neta = GL.neta;
  }
  P.alpha = alpha;
  P.normL = normL;
  if (!d->cons) {  // the root box that x0 must lie in
    P.xlo0.assign(d->xmin, d->xmin + nx);
    P.xhi0.assign(d->xmax, d->xmax + nx);
  }
  P.q.assign(d->q, d->q + (size_t)nn * nx);
  P.r.assign(d->r, d->r + (size_t)nn * nu);
  P.qN.assign(d->qN, d->qN + (size_t)nn * nx);
  if (d->a_risk) P.a_risk.assign(d->a_risk, d->a_risk + nn);
  int team = std::max(nx, nu) >= 24 ? kTeamWG : next_pow2_team(std::max(nx, nu));
  const size_t elem = d->precision == SPOCK_FP64 ? 8 : 4;
  if (mapping_lds(P, team, elem) > 64 * 1024) team = kTeamWG;
  if (const char* env = std::getenv("SPOCK_TEAM")) {
    const int v = std::atoi(env);
    if (v == 8 || v == 16 || v == 32 || v == 64 || v == kTeamWG || v == kTeamFlow) {
      team = mapping_lds(P, v, elem) > 64 * 1024 ? kTeamWG : v;
      P.tuned = true;  // fixed by the caller's environment
    }
  }
  int cut = default_cut(T);
  if (const char* env = std::getenv("SPOCK_CUT")) cut = std::atoi(env);
  set_mapping(P, team, cut);
  P.team_pp = next_pow2_team(std::max(nx, nu));
  if (const char* env = std::getenv("SPOCK_TEAM_PP")) {
    const int v = std::atoi(env);
    if ((v == 8 || v == 16 || v == 32 || v == 64) && v * 4 >= P.team_pp) P.team_pp = v;
  }
  int rc = (d->precision == SPOCK_FP64) ? upload<double>(P, *d, Abar, K, Rinv, W)
                                        : upload<float>(P, *d, Abar, K, Rinv, W);
  if (rc == SPOCK_OK && general)
    rc = (d->precision == SPOCK_FP64) ? upload_general<double>(P, *d, GL) : upload_general<float>(P, *d, GL);
  if (rc != SPOCK_OK) {
    if (P.dmem) (void)hipFree(P.dmem);
    if (P.gmem) (void)hipFree(P.gmem);
    delete h;
    return rc;
  }
  *out = h;
  return SPOCK_OK;
}

extern "C" int spock_problem_destroy(spock_problem* p) {
  if (!p) return SPOCK_EINVAL;
  if (p->p.dmem) (void)hipFree(p->p.dmem);
  if (p->p.gmem) (void)hipFree(p->p.gmem);
  if (p->p.work) (void)hipFree(p->p.work);
  if (p->p.flow.mem) (void)hipFree(p->p.flow.mem);
  if (p->p.mbox) (void)hipHostFree(p->p.mbox);
  delete p;
  return SPOCK_OK;
}

extern "C" int spock_problem_sizes(const spock_problem* p, int64_t* nz, int64_t* neta, double* alpha,
                                   double* normL) {
  if (!p) return SPOCK_EINVAL;
  if (nz) *nz = p->p.nz;
  if (neta) *neta = p->p.neta;
  if (alpha) *alpha = p->p.alpha;
  if (normL) *normL = p->p.normL;
  return SPOCK_OK;
}

extern "C" int spock_problem_mapping(const spock_problem* p, int32_t* mapping, int32_t* flow_grid,
                                     int32_t* flow_failed) {
  if (!p) return SPOCK_EINVAL;
  if (mapping) *mapping = p->p.team;
  if (flow_grid) *flow_grid = p->p.team == kTeamFlow ? p->p.flow.grid : 0;
  if (flow_failed) *flow_failed = p->p.flow_failed ? 1 : 0;
  return SPOCK_OK;
}

extern "C" void spock_settings_default(spock_settings* s) {
  if (!s) return;
  s->eps_abs = 1e-4;
  s->eps_rel = 1e-4;
  s->max_iters = 20000;
  s->method = SPOCK_METHOD_SPOCK;
  s->m = 3;
  s->max_ls = 20;
  s->c0 = 0.99;
  s->c1 = 0.99;
  s->c2 = 0.99;
  s->beta = 0.5;
  s->sigma = 0.1;
  s->lambda = 1.0;
  s->compute_nested = 0;
  s->anderson = SPOCK_AA_AUTO;
}

extern "C" const char* spock_version(void) { return "spock-mi355x 0.1 (gfx950)"; }

// ============================================================== workspace
namespace {

// Anderson memory: up to kAAMax with the device Gram solve, up to kMaxMem
// with the QR-updated least squares
constexpr int kMaxMem = 10;

template <typename S>
struct Work {
  S* q = nullptr;
  S* d = nullptr;
  S* xbar = nullptr;
  S* ubar = nullptr;
  double* partials = nullptr;
  double* stats = nullptr;    // [8]
  double* dots = nullptr;     // [16]
  double* gamma = nullptr;    // [8]
  double* aaG = nullptr;      // Anderson Gram matrix [16] (by slot)
  double* vpart = nullptr;    // vector-kernel partials [blocks][8]
  double* qrdots = nullptr;   // dot products of the QR-updated Anderson step [64]
  S* eta_zero = nullptr;      // n_eta zeros
  double* x0_zero = nullptr;  // kMaxDim zeros (autotuning input)
  S* pool[10 + 2 * kMaxMem];  // n_v buffers
  unsigned* counters = nullptr;       // arrival counts of the push and the rdot [2][kRedCounters]
  unsigned long long* rec = nullptr;  // tagged records of their grid sums [kRedRecWords]
  AARingDev* ring = nullptr;          // Anderson ring (device)
  unsigned tag = 0;                   // tag of their last launch (never 0 once launched)
  unsigned next_tag() { return ++tag == 0u ? ++tag : tag; }
};

// Sizes and allocates the state of the dataflow form of the sweeps for
// precision S: children per LDS chunk (largest count whose LDS stays within
// the budget, at least one), resident workgroups from the occupancy of the
// kernel at the register budget occ, and the flags (zeroed once; they are
// epoch-tagged). The error word is cleared on every call (each API call
// starts clean).
// Test knobs of the dataflow form, read on every sizing call:
// SPOCK_FLOW_GRID caps the grid (fewer workgroups, each running more items,
// so small trees also take the multi-item drain), SPOCK_FLOW_SPIN sets the
// polls of one bounded wait (0: every wait gives up at once, which forces the
// error path with every kernel still ending normally).
void flow_knobs(FlowState& F) {
  F.grid = F.resident;
  F.spin = 1u << 21;
  if (const char* env = std::getenv("SPOCK_FLOW_GRID")) {
    const int cap = std::atoi(env);
    if (cap > 0 && F.grid > 0) F.grid = std::min(F.grid, cap);
  }
  if (const char* env = std::getenv("SPOCK_FLOW_SPIN")) F.spin = (unsigned)std::strtoul(env, nullptr, 10);
}

template <typename S>
int ensure_flow(Problem& P, int occ = 0, int budget = 0) {
  FlowState& F = P.flow;
  const Tree& T = *P.tree;
  if (occ == 0) occ = F.mem ? F.occ : 5;
  if (budget == 0) budget = F.mem ? F.budget : 32 * 1024;
  if (const char* env = std::getenv("SPOCK_FLOW_OCC")) occ = std::max(4, std::min(7, std::atoi(env)));
  if (const char* env = std::getenv("SPOCK_FLOW_LDS")) budget = std::max(4096, std::atoi(env));
  if (F.mem && F.elem == (int)sizeof(S) && F.occ == occ && F.budget == budget) {
    if (hipMemset(F.err, 0, sizeof(unsigned)) != hipSuccess) return SPOCK_EHIP;
    flow_knobs(F);
    return SPOCK_OK;
  }
  if (F.mem) (void)hipFree(F.mem);
  F = FlowState{};
  int maxch = 1;
  for (int i = 0; i < T.nl; ++i) maxch = std::max(maxch, T.nch[i]);
  int nc = std::min(maxch, 8);
  while (nc > 1 && flow_lds_bytes(P.nx, P.nu, nc, (int)sizeof(S)) > budget) --nc;
  const int lds = flow_lds_bytes(P.nx, P.nu, nc, (int)sizeof(S));
  int dev = 0, ncu = 0, coop = 0, nb = 0, smax = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SPOCK_EHIP;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return SPOCK_EHIP;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess) return SPOCK_EHIP;
  if (hipDeviceGetAttribute(&smax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return SPOCK_EHIP;
  const bool fits = lds <= smax;
  if (fits && lds > 64 * 1024 &&
      hipFuncSetAttribute(flow_kernel<S>(occ), hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
    return SPOCK_EHIP;
  if (fits && hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, flow_kernel<S>(occ), 256, (size_t)lds) != hipSuccess)
    return SPOCK_EHIP;
  // Residency is what the waits rely on, so the count is also bounded by
  // what the build guarantees: occ wavefronts per SIMD (the register budget
  // the kernel is compiled for; one wavefront of each workgroup per SIMD)
  // and the LDS in blocks of 512 bytes out of 160 KiB per CU. The occupancy
  // query alone granted grids that were not all resident (it reported the
  // same register count for every budget and left the LDS rounding out).
  if (fits && nb > 0) {
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, flow_kernel<S>(occ)) != hipSuccess) return SPOCK_EHIP;
    const int by_lds = (160 * 1024) / std::max(512, ((lds + (int)fa.sharedSizeBytes + 511) / 512) * 512);
    const int bound = std::min(occ, by_lds);
    if (std::getenv("SPOCK_FLOW_DEBUG"))
      std::fprintf(stderr, "[flow] occ %d nc %d lds %d: query %d per CU -> %d per CU\n", occ, nc, lds, nb,
                   std::min(nb, bound));
    nb = std::min(nb, bound);
  }
  // items: one per chunk of nc children; backward (reverse breadth-first),
  // then forward (breadth-first); partial slots for families of several chunks
  std::vector<int> items, pbase;
  int nslots = 0, nbwd = 0;
  if (build_flow_items(T, nc, kChunkCodes, items, pbase, nslots, nbwd) != SPOCK_OK) return SPOCK_EINVAL;
  const size_t tw = sizeof(S) / 4;  // tagged words per element
  const size_t nq = (size_t)T.nl * P.nx * tw, nd = (size_t)T.nl * P.nu * tw, nxw = (size_t)T.nn * P.nx * tw;
  const size_t npw = (size_t)nslots * (P.nx + P.nu) * tw;
  const size_t tagged = sizeof(unsigned long long) * (nq + nd + nxw + npw);
  const size_t bytes = 256 + tagged + sizeof(int) * (items.size() + pbase.size());
  if (hipMalloc(&F.mem, bytes) != hipSuccess) return SPOCK_ENOMEM;
  if (hipMemset(F.mem, 0, bytes) != hipSuccess) return SPOCK_EHIP;
  F.err = static_cast<unsigned*>(F.mem);
  F.qt = reinterpret_cast<unsigned long long*>(static_cast<char*>(F.mem) + 256);
  F.dt = F.qt + nq;
  F.xt = F.dt + nd;
  F.pt = F.xt + nxw;
  F.items = reinterpret_cast<int*>(static_cast<char*>(F.mem) + 256 + tagged);
  F.pbase = F.items + items.size();
  F.nbwd = nbwd;
  if (hipMemcpy(F.items, items.data(), sizeof(int) * items.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(F.pbase, pbase.data(), sizeof(int) * pbase.size(), hipMemcpyHostToDevice) != hipSuccess)
    return SPOCK_EHIP;
  F.nc = nc;
  F.occ = occ;
  F.budget = budget;
  if (const char* env = std::getenv("SPOCK_FLOW_COOP")) F.coop = std::atoi(env) != 0;
  F.elem = (int)sizeof(S);
  F.grid = (coop && fits) ? nb * ncu : 0;
  F.resident = F.grid;
  flow_knobs(F);
  return SPOCK_OK;
}

template <typename S>
int ensure_work(Problem& P, Work<S>& W) {
  const Tree& T = *P.tree;
  const long long nv = P.nz + P.neta;
  const int nblk = dots_blocks(nv);
  size_t bytes = 0;
  auto add = [&](size_t b) { bytes += (b + 255) & ~size_t(255); };
  add(sizeof(S) * (size_t)T.nn * P.nx);
  add(sizeof(S) * (size_t)T.nn * P.nu);
  add(sizeof(S) * (size_t)T.nn * P.nx);
  add(sizeof(S) * (size_t)T.nn * P.nu);
  add(sizeof(double) * (size_t)(T.nl + 1) * kStats);  // enough for every mapping
  add(sizeof(double) * 8);
  add(sizeof(double) * 16);
  add(sizeof(double) * 8);
  add(sizeof(double) * 32);
  add(sizeof(double) * (size_t)nblk * 8);
  add(sizeof(double) * 64);
  add(sizeof(unsigned) * 2 * kRedCounters);
  add(sizeof(unsigned long long) * kRedRecWords);
  add(sizeof(AARingDev));
  add(sizeof(S) * (size_t)P.neta);
  add(sizeof(double) * kMaxDim);
  for (int k = 0; k < 10 + 2 * kMaxMem; ++k) add(sizeof(S) * (size_t)nv);
  if (P.work_bytes < bytes) {
    if (P.work) (void)hipFree(P.work);
    P.work = nullptr;
    P.work_bytes = 0;
    if (hipMalloc(&P.work, bytes) != hipSuccess) return SPOCK_ENOMEM;
    P.work_bytes = bytes;
    if (hipMemset(P.work, 0, bytes) != hipSuccess) return SPOCK_EHIP;
  }
  // base-relative offsets, in the same order as the size computation above
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = static_cast<char*>(P.work) + off;
    off += (b + 255) & ~size_t(255);
    return p;
  };
  W.q = reinterpret_cast<S*>(take(sizeof(S) * (size_t)T.nn * P.nx));
  W.d = reinterpret_cast<S*>(take(sizeof(S) * (size_t)T.nn * P.nu));
  W.xbar = reinterpret_cast<S*>(take(sizeof(S) * (size_t)T.nn * P.nx));
  W.ubar = reinterpret_cast<S*>(take(sizeof(S) * (size_t)T.nn * P.nu));
  W.partials = reinterpret_cast<double*>(take(sizeof(double) * (size_t)(T.nl + 1) * kStats));
  W.stats = reinterpret_cast<double*>(take(sizeof(double) * 8));
  W.dots = reinterpret_cast<double*>(take(sizeof(double) * 16));
  W.gamma = reinterpret_cast<double*>(take(sizeof(double) * 8));
  W.aaG = reinterpret_cast<double*>(take(sizeof(double) * 32));
  W.vpart = reinterpret_cast<double*>(take(sizeof(double) * (size_t)nblk * 8));
  W.qrdots = reinterpret_cast<double*>(take(sizeof(double) * 64));
  W.counters = reinterpret_cast<unsigned*>(take(sizeof(unsigned) * 2 * kRedCounters));
  W.rec = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long) * kRedRecWords));
  W.ring = reinterpret_cast<AARingDev*>(take(sizeof(AARingDev)));
  W.eta_zero = reinterpret_cast<S*>(take(sizeof(S) * (size_t)P.neta));
  W.x0_zero = reinterpret_cast<double*>(take(sizeof(double) * kMaxDim));
  for (int k = 0; k < 10 + 2 * kMaxMem; ++k) W.pool[k] = reinterpret_cast<S*>(take(sizeof(S) * (size_t)nv));
  if (off > P.work_bytes) return SPOCK_ENOMEM;
  // the layout depends on the precision: the counts and the tagged records
  // (tag 0: never written) start cleared here
  if (hipMemset(W.counters, 0, sizeof(unsigned) * 2 * kRedCounters) != hipSuccess) return SPOCK_EHIP;
  if (hipMemset(W.rec, 0, sizeof(unsigned long long) * kRedRecWords) != hipSuccess) return SPOCK_EHIP;
  W.tag = 0;
  if (!P.mbox) {
    void* hp = nullptr;
    if (hipHostMalloc(&hp, sizeof(Mailbox), hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
      return SPOCK_ENOMEM;
    std::memset(hp, 0, sizeof(Mailbox));
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess) {
      (void)hipHostFree(hp);
      return SPOCK_EHIP;
    }
    P.mbox = static_cast<Mailbox*>(hp);
    P.mbox_dev = static_cast<Mailbox*>(dp);
    P.mbox_epoch = 0;
  }
  if (P.team == kTeamFlow && P.flow_failed) set_mapping(P, kTeamWG, default_cut(*P.tree));
  if (P.team == kTeamFlow) {
    const int rc = ensure_flow<S>(P);
    if (rc) return rc;
    // the dataflow form does not fit (LDS) or cannot be launched resident:
    // per-stage workgroup launches instead
    if (P.flow.grid <= 0) set_mapping(P, kTeamWG, default_cut(*P.tree));
  }
  return SPOCK_OK;
}

// Picks the fastest family-to-lane mapping for this problem by timing T on
// a zero iterate (a few repetitions per candidate).
template <typename S>
int autotune(Problem& P, hipStream_t st) {
  if (P.tuned) return SPOCK_OK;
  Work<S> W;
  int rc = ensure_work<S>(P, W);
  if (rc) return rc;
  const long long nv = P.nz + P.neta;
  HIP_TRY(launch_fill<S>(nv, W.pool[0], 0.0, st));
  HIP_TRY(hipMemsetAsync(W.x0_zero, 0, sizeof(double) * kMaxDim, st));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const Tree& T = *P.tree;
  std::vector<std::pair<int, int>> cands = {{8, T.N}, {16, T.N}, {32, T.N}, {64, T.N}, {kTeamWG, T.N}};
  // dataflow form: register budget (4 to 7 wavefronts per SIMD) and LDS
  // budget (children per chunk against workgroups per CU); the cut field
  // carries occ * 1000 + LDS budget in KiB
  for (int code : {4024, 5024, 6024, 7024, 4032, 5032, 6032, 7032, 4040, 5040, 5046})
    if (!P.flow_failed && ensure_flow<S>(P, code / 1000, (code % 1000) * 1024) == SPOCK_OK && P.flow.grid > 0)
      cands.push_back({kTeamFlow, code});
  int ncut = 0;
  for (int t = std::max(0, T.N - 64); t < T.N && ncut < 3; ++t)
    if (T.stage_off[t + 1] - T.stage_off[t] >= 128) {
      cands.push_back({kTeamWG, t});
      ++ncut;
    }
  float best = 1e30f;
  std::pair<int, int> best_map = {P.team, P.cut};
  for (auto c : cands) {
    if (mapping_lds(P, c.first, sizeof(S)) > 64 * 1024) continue;
    if (c.first == kTeamFlow &&
        (ensure_flow<S>(P, c.second / 1000, (c.second % 1000) * 1024) != SPOCK_OK || P.flow.grid <= 0))
      continue;
    set_mapping(P, c.first, c.second);
    HIP_TRY(launch_T<S>(P, W.pool[0], W.pool[1], W.x0_zero, W.q, W.d, W.xbar, W.ubar, W.partials, W.stats, st,
                        W.eta_zero, true));
    HIP_TRY(hipEventRecord(e0, st));
    for (int r = 0; r < 3; ++r)
      HIP_TRY(launch_T<S>(P, W.pool[0], W.pool[1], W.x0_zero, W.q, W.d, W.xbar, W.ubar, W.partials, W.stats, st,
                          W.eta_zero, true));
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (c.first == kTeamFlow) {
      // a bounded wait that gave up (a grid that was not all resident):
      // the candidate is rejected, whatever its time
      unsigned err = 0;
      HIP_TRY(hipMemcpy(&err, P.flow.err, sizeof(unsigned), hipMemcpyDeviceToHost));
      if (err != 0u) {
        HIP_TRY(hipMemset(P.flow.err, 0, sizeof(unsigned)));
        continue;
      }
    }
    if (ms < best) {
      best = ms;
      best_map = c;
    }
  }
  if (best_map.first == kTeamFlow &&
      ensure_flow<S>(P, best_map.second / 1000, (best_map.second % 1000) * 1024) != SPOCK_OK)
    return SPOCK_EHIP;
  set_mapping(P, best_map.first, best_map.second);
  // lanes per family of the parallel pre/post passes (fewer lanes: more
  // families in flight per workgroup, longer per-lane loops)
  {
    const int tmin = next_pow2_team(std::max(P.nx, P.nu));
    float best_pp = 1e30f;
    int pick = P.team_pp;
    for (int tpp : {16, 32, 64}) {
      if (tpp * 4 < tmin) continue;  // at most 4 components per lane
      P.team_pp = tpp;
      HIP_TRY(launch_T<S>(P, W.pool[0], W.pool[1], W.x0_zero, W.q, W.d, W.xbar, W.ubar, W.partials, W.stats, st,
                          W.eta_zero, true));
      HIP_TRY(hipEventRecord(e0, st));
      for (int r = 0; r < 3; ++r)
        HIP_TRY(launch_T<S>(P, W.pool[0], W.pool[1], W.x0_zero, W.q, W.d, W.xbar, W.ubar, W.partials, W.stats,
                            st, W.eta_zero, true));
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_pp) {
        best_pp = ms;
        pick = tpp;
      }
    }
    P.team_pp = pick;
    // the flat post-pass against the team forms at that team size (the
    // pre-pass keeps its team size either way); SPOCK_POST fixes the form
    if (!std::getenv("SPOCK_POST")) {
      P.post_flat = true;
      HIP_TRY(launch_T<S>(P, W.pool[0], W.pool[1], W.x0_zero, W.q, W.d, W.xbar, W.ubar, W.partials, W.stats, st,
                          W.eta_zero, true));
      HIP_TRY(hipEventRecord(e0, st));
      for (int r = 0; r < 3; ++r)
        HIP_TRY(launch_T<S>(P, W.pool[0], W.pool[1], W.x0_zero, W.q, W.d, W.xbar, W.ubar, W.partials, W.stats,
                            st, W.eta_zero, true));
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      P.post_flat = ms < best_pp;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P.tuned = true;
  return SPOCK_OK;
}

// Internal status: a bounded wait of the dataflow sweeps gave up during the
// call (its workgroups were not all resident), so the results it produced
// are void. The entry points then switch the problem to the per-stage
// workgroup form (flow_fallback) and redo the call; it never reaches the
// caller.
constexpr int kFlowGaveUp = 1000;

// Reads the error word of the dataflow sweeps (synchronises the stream).
int flow_gave_up(const Problem& P, hipStream_t st, bool& gave_up) {
  gave_up = false;
  if (P.team != kTeamFlow || !P.flow.err) return SPOCK_OK;
  unsigned err = 0;
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemcpy(&err, P.flow.err, sizeof(unsigned), hipMemcpyDeviceToHost));
  gave_up = err != 0u;
  return SPOCK_OK;
}

// After a give-up: clear the word and run the per-stage workgroup form from
// now on (the problem never returns to the dataflow form).
int flow_fallback(Problem& P) {
  if (P.flow.err) HIP_TRY(hipMemset(P.flow.err, 0, sizeof(unsigned)));
  P.flow_failed = true;
  set_mapping(P, kTeamWG, default_cut(*P.tree));
  return SPOCK_OK;
}

struct Stats {
  double xip = 0, xid = 0, om2 = 0, rz2 = 0, re2 = 0, cross = 0;
  double xi() const { return std::max(xip, xid); }
  double omega() const { return std::sqrt(std::max(om2, 0.0)); }
  bool ok() const { return std::isfinite(xip) && std::isfinite(xid) && std::isfinite(om2); }
};

template <typename S>
struct Solver {
  Problem& P;
  Work<S> W;
  hipStream_t st;
  const double* x0;
  long long nv;
  int t_evals = 0;
  std::vector<double> hbuf = std::vector<double>(16);

  Solver(Problem& p, hipStream_t s, const double* x) : P(p), st(s), x0(x), nv(p.nz + p.neta) {}

  // T(v) and its statistics; with md, also <v - T(v), md> (line search),
  // fetched in the same transfer (statistics slot 6)
  int T(const S* v, S* Tv, Stats& out, const S* md = nullptr, double* rdot = nullptr) {
    unsigned long long ep = 0;
    const int rc = launch(v, Tv, ep, md);
    return rc ? rc : wait(ep, out, rdot);
  }
  // queues T(v) (and <v - T(v), md>) with its statistics published to the
  // mailbox under the returned epoch
  int launch(const S* v, S* Tv, unsigned long long& epoch, const S* md = nullptr) {
    const Publish pub{P.mbox_dev, ++P.mbox_epoch};
    HIP_TRY(launch_T<S>(P, v, Tv, x0, W.q, W.d, W.xbar, W.ubar, W.partials, W.stats, st, W.eta_zero, true,
                        md ? Publish{} : pub));
    if (md)
      HIP_TRY(launch_rdot<S>(nv, v, Tv, md, W.rec, W.counters + kRedCounters, W.next_tag(), W.stats + 6, W.stats, pub, st));
    epoch = pub.epoch;
    return SPOCK_OK;
  }
  int wait(unsigned long long epoch, Stats& out, double* rdot = nullptr) {
    const int rc = wait_mailbox(epoch);
    if (rc) return rc;
    for (int k = 0; k < 8; ++k) hbuf[k] = P.mbox->v[k];
    if (rdot) *rdot = hbuf[6];
    out.xip = hbuf[0];
    out.xid = hbuf[1];
    out.om2 = hbuf[2];
    out.rz2 = hbuf[3];
    out.re2 = hbuf[4];
    out.cross = hbuf[5];
    ++t_evals;
    if (!out.ok()) {  // NaN statistics: a dataflow wait that gave up, or the iterate itself
      bool gave_up = false;
      const int rc = flow_gave_up(P, st, gave_up);
      if (rc) return rc;
      if (gave_up) return kFlowGaveUp;
    }
    return SPOCK_OK;
  }
  // Polls the mailbox for the epoch; every 4096 polls the stream is asked
  // whether it drained (then the epoch must be there) or failed.
  int wait_mailbox(unsigned long long epoch) {
    for (unsigned n = 1;; ++n) {
      if (__atomic_load_n(&P.mbox->flag, __ATOMIC_ACQUIRE) == epoch) return SPOCK_OK;
      if ((n & 4095u) == 0u) {
        const hipError_t e = hipStreamQuery(st);
        if (e == hipSuccess)
          return __atomic_load_n(&P.mbox->flag, __ATOMIC_ACQUIRE) == epoch ? SPOCK_OK : SPOCK_EHIP;
        if (e != hipErrorNotReady) return SPOCK_EHIP;
      }
    }
  }
  int fetch(double* dst, const double* src, int k) {
    HIP_TRY(hipMemcpyAsync(dst, src, k * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SPOCK_OK;
  }
};

// Anderson ring: slots of the active columns, oldest first (the Gram matrix
// and the right-hand side, indexed by slot, live on the device).

// Solves the Gram system for the active columns after applying the rank rule
// (drop the oldest column while lambda_min/lambda_max(G) < 1e-12, i.e.
// sigma_min/sigma_max(dR) < 1e-6). Returns the number of columns kept.

// Singular values extremes of a k x k matrix (one-sided Jacobi on its
// columns, FP64): smin and smax.
void sv_extremes(int k, const double (*R)[kMaxMem], double& smin, double& smax) {
  double A[kMaxMem][kMaxMem];
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) A[i][j] = R[i][j];
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        double a = 0, b = 0, c = 0;
        for (int i = 0; i < k; ++i) {
          a += A[i][p] * A[i][p];
          b += A[i][q] * A[i][q];
          c += A[i][p] * A[i][q];
        }
        if (c == 0.0 || std::fabs(c) <= 1e-17 * std::sqrt(a * b)) continue;
        off = std::max(off, std::fabs(c) / std::sqrt(a * b));
        const double z = (b - a) / (2.0 * c);
        const double t = (z >= 0 ? 1.0 : -1.0) / (std::fabs(z) + std::sqrt(1.0 + z * z));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int i = 0; i < k; ++i) {
          const double x = A[i][p], y = A[i][q];
          A[i][p] = cs * x - sn * y;
          A[i][q] = sn * x + cs * y;
        }
      }
    if (off <= 1e-15) break;
  }
  smin = std::numeric_limits<double>::infinity();
  smax = 0.0;
  for (int j = 0; j < k; ++j) {
    double n2 = 0;
    for (int i = 0; i < k; ++i) n2 += A[i][j] * A[i][j];
    smin = std::min(smin, std::sqrt(n2));
    smax = std::max(smax, std::sqrt(n2));
  }
}

// Anderson step with the least squares min ||M^R gamma - r|| solved through
// a thin QR factorisation M^R = Q R that is updated at every push (section
// 6.2). A new column is orthogonalised against Q by classical Gram-Schmidt
// with one reorthogonalisation; the oldest column is removed by Givens
// rotations that bring R[:, 1:] back to triangular form, the same rotations
// mixing the columns of Q; gamma solves R gamma = Q'r. The rank rule drops the
// oldest column while sigma_min / sigma_max(R) < 1e-6 (those of M^R). The
// vectors (Q, and E = dV - dR) stay on the device; R, the rotations and gamma
// are FP64 on the host, which reads 2-3 small batches of dot products per push.
template <typename S>
struct QrAnderson {
  int m = 0, k = 0;            // memory and active columns
  long long nv = 0;
  S* E[kMaxMem] = {};          // slots of E = dV - dR
  S* Q[kMaxMem] = {};          // slots of the orthonormal columns
  int ord[kMaxMem] = {};       // slot of active column j, oldest first
  double R[kMaxMem][kMaxMem] = {};
  double qr[kMaxMem] = {};     // Q'r for the current r
  double gamma[kMaxMem] = {};
  double* dots_dev = nullptr;
  double* part = nullptr;
  hipStream_t st = nullptr;

  int free_slot() const {
    for (int sl = 0; sl < m; ++sl) {
      bool used = false;
      for (int j = 0; j < k; ++j) used = used || ord[j] == sl;
      if (!used) return sl;
    }
    return -1;
  }
  // pairs (xs[j], ys[j]) j < n into h[j] (n <= 24), one synchronisation
  int dots(int n, const S* const* xs, const S* const* ys, double* h) {
    for (int b = 0; b < n; b += 8) {
      VecPtrs<S> X{}, Y{};
      const int c = std::min(8, n - b);
      for (int j = 0; j < c; ++j) {
        X.p[j] = xs[b + j];
        Y.p[j] = ys[b + j];
      }
      HIP_TRY(launch_dots<S>(nv, c, X, Y, part, dots_dev + b, st));
    }
    HIP_TRY(hipMemcpyAsync(h, dots_dev, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SPOCK_OK;
  }
  // w <- w - sum_j h_j Q_j
  int subtract(S* w, const double* h) {
    if (k == 0) return SPOCK_OK;
    ColMix<S> M;
    M.nin = k + 1;
    M.nout = 1;
    M.in[0] = w;
    M.c[0][0] = 1.0;
    for (int j = 0; j < k; ++j) {
      M.in[1 + j] = Q[ord[j]];
      M.c[0][1 + j] = -h[j];
    }
    M.out[0] = w;
    HIP_TRY(launch_colmix<S>(nv, M, st));
    return SPOCK_OK;
  }
  // removes the oldest column: Givens rotations on R[:, 1:], the same
  // rotations on the columns of Q and on Q'r
  int drop_oldest() {
    if (k == 0) return SPOCK_OK;
    double H[kMaxMem][kMaxMem] = {}, Wm[kMaxMem][kMaxMem] = {};
    for (int i = 0; i < k; ++i) {
      Wm[i][i] = 1.0;
      for (int j = 0; j + 1 < k; ++j) H[i][j] = R[i][j + 1];
    }
    for (int j = 0; j + 1 < k; ++j) {
      const double a = H[j][j], b = H[j + 1][j], r = std::hypot(a, b);
      const double c = r > 0.0 ? a / r : 1.0, sn = r > 0.0 ? b / r : 0.0;
      for (int l = 0; l < k - 1; ++l) {
        const double x = H[j][l], y = H[j + 1][l];
        H[j][l] = c * x + sn * y;
        H[j + 1][l] = -sn * x + c * y;
      }
      for (int i = 0; i < k; ++i) {  // W <- W G_j', columns j, j + 1
        const double x = Wm[i][j], y = Wm[i][j + 1];
        Wm[i][j] = c * x + sn * y;
        Wm[i][j + 1] = -sn * x + c * y;
      }
      const double x = qr[j], y = qr[j + 1];
      qr[j] = c * x + sn * y;
      qr[j + 1] = -sn * x + c * y;
    }
    if (k > 1) {
      ColMix<S> M;
      M.nin = k;
      M.nout = k - 1;
      for (int i = 0; i < k; ++i) M.in[i] = Q[ord[i]];
      // the new columns go to the slots of columns 1..k-1 (inputs are read first)
      for (int j = 0; j + 1 < k; ++j) {
        M.out[j] = Q[ord[j + 1]];
        for (int i = 0; i < k; ++i) M.c[j][i] = Wm[i][j];
      }
      HIP_TRY(launch_colmix<S>(nv, M, st));
    }
    for (int j = 0; j + 1 < k; ++j) ord[j] = ord[j + 1];
    for (int i = 0; i < kMaxMem; ++i)
      for (int j = 0; j < kMaxMem; ++j) R[i][j] = (i < k - 1 && j < k - 1) ? H[i][j] : 0.0;
    for (int j = k - 1; j < kMaxMem; ++j) qr[j] = 0.0;
    --k;
    return SPOCK_OK;
  }
  // push of the newest difference pair and solve; r = v - Tv, then d and
  // step = v + d
  int push_and_direction(const S* v, const S* vprev, const S* Tv, const S* rprev, S* r, S* d, S* step) {
    if (k == m) {
      const int rc = drop_oldest();
      if (rc) return rc;
    }
    const int sl = free_slot();
    if (sl < 0) return SPOCK_EINVAL;
    S* w = Q[sl];
    {  // r = v - Tv, dR = r - rprev (into the new Q slot), E = dV - dR = Tv + rprev - vprev
      ColMix<S> M;
      M.nin = 4;
      M.nout = 3;
      M.in[0] = v;
      M.in[1] = Tv;
      M.in[2] = rprev;
      M.in[3] = vprev;
      M.out[0] = r;
      M.out[1] = w;
      M.out[2] = E[sl];
      const double cr[4] = {1, -1, 0, 0}, cw[4] = {1, -1, -1, 0}, ce[4] = {0, 1, 1, -1};
      for (int j = 0; j < 4; ++j) {
        M.c[0][j] = cr[j];
        M.c[1][j] = cw[j];
        M.c[2][j] = ce[j];
      }
      HIP_TRY(launch_colmix<S>(nv, M, st));
    }
    const S* xs[24];
    const S* ys[24];
    double h[24], h1[kMaxMem] = {}, h2[kMaxMem] = {};
    // Q'w and Q'r
    for (int j = 0; j < k; ++j) {
      xs[j] = Q[ord[j]];
      ys[j] = w;
      xs[k + j] = Q[ord[j]];
      ys[k + j] = r;
    }
    int rc = k ? dots(2 * k, xs, ys, h) : SPOCK_OK;
    if (rc) return rc;
    for (int j = 0; j < k; ++j) {
      h1[j] = h[j];
      qr[j] = h[k + j];
    }
    if ((rc = subtract(w, h1))) return rc;
    // reorthogonalisation
    if (k) {
      for (int j = 0; j < k; ++j) {
        xs[j] = Q[ord[j]];
        ys[j] = w;
      }
      if ((rc = dots(k, xs, ys, h2))) return rc;
      if ((rc = subtract(w, h2))) return rc;
    }
    xs[0] = w;
    ys[0] = w;
    xs[1] = w;
    ys[1] = r;
    if ((rc = dots(2, xs, ys, h))) return rc;
    const double rho = std::sqrt(std::max(h[0], 0.0));
    {
      ColMix<S> M;  // normalise
      M.nin = 1;
      M.nout = 1;
      M.in[0] = w;
      M.out[0] = w;
      M.c[0][0] = rho > 0.0 ? 1.0 / rho : 0.0;
      HIP_TRY(launch_colmix<S>(nv, M, st));
    }
    for (int j = 0; j < k; ++j) R[j][k] = h1[j] + h2[j];
    for (int j = 0; j <= k; ++j) R[k][j] = 0.0;
    R[k][k] = rho;
    qr[k] = rho > 0.0 ? h[1] / rho : 0.0;
    ord[k] = sl;
    ++k;
    // rank rule: drop the oldest column while sigma_min / sigma_max < 1e-6
    while (k > 0) {
      double smin = 0, smax = 0;
      sv_extremes(k, R, smin, smax);
      if (smax > 0.0 && smin / smax >= 1e-6) break;
      if ((rc = drop_oldest())) return rc;
    }
    // gamma = R^{-1} Q'r
    for (int i = k - 1; i >= 0; --i) {
      double acc = qr[i];
      for (int j = i + 1; j < k; ++j) acc -= R[i][j] * gamma[j];
      gamma[i] = acc / R[i][i];
    }
    ColMix<S> M;  // d = -r - sum_j gamma_j E_j, step = v + d
    M.nin = k + 2;
    M.nout = 2;
    M.in[0] = r;
    M.in[1] = v;
    M.c[0][0] = -1.0;
    M.c[1][0] = -1.0;
    M.c[1][1] = 1.0;
    for (int j = 0; j < k; ++j) {
      M.in[2 + j] = E[ord[j]];
      M.c[0][2 + j] = -gamma[j];
      M.c[1][2 + j] = -gamma[j];
    }
    M.out[0] = d;
    M.out[1] = step;
    HIP_TRY(launch_colmix<S>(nv, M, st));
    return SPOCK_OK;
  }
};

template <typename S>
int solve_impl(Problem& P, const double* x0, const spock_settings& s, S* vio, spock_info& info,
               hipStream_t st) {
  Solver<S> SV(P, st, x0);
  int rc = ensure_work<S>(P, SV.W);
  if (rc) return rc;
  Work<S>& W = SV.W;
  const long long nv = SV.nv;
  const double al = P.alpha;
  // roles over the buffer pool
  S* v = W.pool[0];
  S* Tv = W.pool[1];
  S* vprev = W.pool[2];
  S* rprev = W.pool[3];
  S* rcur = W.pool[4];
  S* dir = W.pool[5];
  S* Md = W.pool[6];
  S* vt = W.pool[7];
  S* Tvt = W.pool[8];
  S* spare = W.pool[9];
  S* dV[kMaxMem];
  S* dR[kMaxMem];
  for (int k = 0; k < kMaxMem; ++k) {
    dV[k] = W.pool[10 + k];
    dR[k] = W.pool[10 + kMaxMem + k];
  }
  HIP_TRY(hipMemcpyAsync(v, vio, sizeof(S) * nv, hipMemcpyDeviceToDevice, st));
  Stats S0, Sc, St;
  rc = SV.T(v, Tv, S0);
  if (rc) return rc;
  Sc = S0;
  info.xi0 = S0.xi();
  const double tol = std::max(s.eps_abs, s.eps_rel * info.xi0);
  int k = 0;
  auto finish = [&](int status) -> int {
    HIP_TRY(hipMemcpyAsync(vio, Tv, sizeof(S) * nv, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    info.status = status;
    info.iters = k;
    info.t_evals = SV.t_evals;
    info.xi = Sc.xi();
    return SPOCK_OK;
  };
  if (!S0.ok()) return finish(SPOCK_NUMERICAL);

  if (s.method == SPOCK_METHOD_CP) {
    for (;;) {
      if (Sc.xi() <= tol) return finish(SPOCK_CONVERGED);
      if (k >= s.max_iters) return finish(SPOCK_MAXITER);
      std::swap(v, Tv);
      rc = SV.T(v, Tv, Sc);
      if (rc) return rc;
      ++k;
      if (!Sc.ok()) return finish(SPOCK_NUMERICAL);
    }
  }

  // ---- SPOCK (Alg. 3 with the residual formed before the tests)
  double zeta = S0.omega(), omega_safe = S0.omega();
  bool have_prev = false;
  // The Anderson ring (column order, Gram matrix, rank rule) lives on the
  // device, so the residual, the push, the Gram solve, the direction d and
  // the K0 candidate v + d of an iterate are queued right behind its
  // evaluation of T, before the host reads the statistics that decide the
  // step: the host's decision overlaps that work.
  // the slots' vectors sit at one stride in the pool (E at dV[0] + s stride,
  // dR at dR[0] + s stride)
  const long long sstride = dV[1] - dV[0];
  for (int j = 0; j < kAAMax; ++j)
    if (dV[j] - dV[0] != j * sstride || dR[j] - dR[0] != j * sstride) return SPOCK_EINVAL;
  {
    AARingDev r0{};
    r0.m = s.m;
    HIP_TRY(hipMemcpyAsync(W.ring, &r0, sizeof(r0), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  // QR-updated least squares (memory up to kMaxMem), else the device Gram solve
  const bool use_qr = s.anderson == SPOCK_AA_QR || (s.anderson == SPOCK_AA_AUTO && s.m > kAAMax);
  QrAnderson<S> qa;
  if (use_qr) {
    qa.m = s.m;
    qa.nv = nv;
    qa.dots_dev = W.qrdots;
    qa.part = W.vpart;
    qa.st = st;
    for (int j = 0; j < s.m; ++j) {
      qa.E[j] = dV[j];
      qa.Q[j] = dR[j];
    }
  }
  // r = v - Tv, the Anderson push and Gram solve, d, and spare = v + d for
  // the current iterate (stream-ordered after its T)
  auto prepare = [&]() -> int {
    if (have_prev && use_qr) return qa.push_and_direction(v, vprev, Tv, rprev, rcur, dir, spare);
    if (have_prev) {
      HIP_TRY(launch_aa_push<S>(nv, v, vprev, Tv, rprev, rcur, dV[0], dR[0], sstride, W.rec, W.counters,
                                W.next_tag(), W.aaG, W.ring, W.gamma, st));
      HIP_TRY(launch_aa_dir<S>(nv, rcur, dV[0], sstride, W.ring, W.gamma, dir, v, spare, st));
    } else {
      HIP_TRY(launch_lincomb<S>(nv, rcur, 1.0, v, -1.0, Tv, st));
      HIP_TRY(launch_lincomb<S>(nv, dir, -1.0, rcur, 0.0, nullptr, st));
      HIP_TRY(launch_lincomb<S>(nv, spare, 1.0, v, 1.0, dir, st));
    }
    return SPOCK_OK;
  };
  // T of the new iterate, its preparation queued behind it, then its
  // statistics (the QR step reads dot products, so it follows the wait)
  auto eval_next = [&]() -> int {
    unsigned long long ep = 0;
    int r = SV.launch(v, Tv, ep);
    if (!r && !use_qr) r = prepare();
    if (!r) r = SV.wait(ep, Sc);
    if (!r && use_qr) r = prepare();
    return r;
  };
  auto accept_prev = [&]() {
    std::swap(vprev, v);      // vprev <- old v
    std::swap(rprev, rcur);   // rprev <- old r
    have_prev = true;
  };
  rc = prepare();
  if (rc) return rc;
  for (;;) {
    if (Sc.xi() <= tol) return finish(SPOCK_CONVERGED);
    if (k >= s.max_iters) return finish(SPOCK_MAXITER);
    const double omega = Sc.omega();
    if (omega <= s.c0 * zeta) {  // K0: spare = v + d, formed with the direction
      accept_prev();
      std::swap(v, spare);       // v <- v_old + d ; spare <- old vprev
      zeta = omega;
      info.n_k0++;
      rc = eval_next();
      if (rc) return rc;
      ++k;
      if (!Sc.ok()) return finish(SPOCK_NUMERICAL);
      continue;
    }
    // M d = (d_z - alpha L* d_eta, d_eta - alpha L d_z), formed once per iteration
    HIP_TRY(launch_M<S>(P, dir, Md, st));
    double tau = 1.0;
    bool accepted = false;
    for (int ls = 0; ls < s.max_ls; ++ls) {
      HIP_TRY(launch_lincomb<S>(nv, vt, 1.0, v, tau, dir, st));
      double rdot = 0;
      rc = SV.T(vt, Tvt, St, Md, &rdot);
      if (rc) return rc;
      if (!St.ok()) {
        tau *= s.beta;
        info.n_backtracks++;
        continue;
      }
      const double om_t = St.omega();
      if (om_t == 0.0 || (omega <= omega_safe && om_t <= s.c1 * omega)) {  // K1
        accept_prev();
        std::swap(v, vt);
        std::swap(Tv, Tvt);
        Sc = St;
        omega_safe = om_t + std::pow(s.c2, k);
        info.n_k1++;
        rc = prepare();
        if (rc) return rc;
        accepted = true;
        break;
      }
      const double rho = om_t * om_t - tau * rdot;
      if (rho >= s.sigma * om_t * omega) {  // K2: v - lambda rho / om_t^2 (vt - Tvt)
        const double c = s.lambda * rho / (om_t * om_t);
        HIP_TRY(launch_lincomb3<S>(nv, spare, 1.0, v, -c, vt, c, Tvt, st));
        accept_prev();
        std::swap(v, spare);
        info.n_k2++;
        rc = eval_next();
        if (rc) return rc;
        accepted = true;
        break;
      }
      tau *= s.beta;
      info.n_backtracks++;
    }
    if (!accepted) {  // plain KM step
      HIP_TRY(launch_lincomb<S>(nv, spare, 1.0, v, -s.lambda, rcur, st));
      accept_prev();
      std::swap(v, spare);
      info.n_km++;
      rc = eval_next();
      if (rc) return rc;
    }
    ++k;
    if (!Sc.ok()) return finish(SPOCK_NUMERICAL);
  }
}

}  // namespace

extern "C" int spock_solve(spock_problem* ph, const double* x0_dev, const spock_settings* s, void* v_io,
                           spock_info* info, void* stream) {
  if (!ph || !x0_dev || !s || !v_io || !info) return SPOCK_EINVAL;
  if (s->method != SPOCK_METHOD_CP && s->method != SPOCK_METHOD_SPOCK) return SPOCK_EINVAL;
  if (s->method == SPOCK_METHOD_SPOCK && (s->m < 1 || s->m > kMaxMem)) return SPOCK_EINVAL;
  if (s->anderson != SPOCK_AA_AUTO && s->anderson != SPOCK_AA_GRAM && s->anderson != SPOCK_AA_QR)
    return SPOCK_EINVAL;
  if (s->method == SPOCK_METHOD_SPOCK && s->anderson == SPOCK_AA_GRAM && s->m > kAAMax) return SPOCK_EINVAL;
  if (!(s->eps_abs >= 0 && s->eps_rel >= 0) || s->max_iters < 0 || s->max_ls < 1) return SPOCK_EINVAL;
  if (!(s->beta > 0 && s->beta < 1 && s->sigma > 0 && s->sigma < 1 && s->lambda > 0 && s->lambda < 2))
    return SPOCK_EINVAL;
  Problem& P = ph->p;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  // x0 must lie in the root's state box
  std::vector<double> hx(P.nx);
  HIP_TRY(hipMemcpyAsync(hx.data(), x0_dev, P.nx * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int k = 0; k < (int)P.xlo0.size(); ++k)
    if (!(hx[k] >= P.xlo0[k] && hx[k] <= P.xhi0[k])) return SPOCK_EBOX;
  spock_info loc{};
  loc.V_nested = std::numeric_limits<double>::quiet_NaN();
  {
    const int rt = (P.precision == SPOCK_FP64) ? autotune<double>(P, st) : autotune<float>(P, st);
    if (rt) return rt;
  }
  loc.mapping = P.team;
  int rc = (P.precision == SPOCK_FP64)
               ? solve_impl<double>(P, x0_dev, *s, static_cast<double*>(v_io), loc, st)
               : solve_impl<float>(P, x0_dev, *s, static_cast<float*>(v_io), loc, st);
  if (rc == kFlowGaveUp) {
    // v_io is written only at the end of a solve: redo it from the same
    // start with the per-stage form
    rc = flow_fallback(P);
    if (rc) return rc;
    loc = spock_info{};
    loc.V_nested = std::numeric_limits<double>::quiet_NaN();
    loc.mapping = P.team;
    loc.flow_fallback = 1;
    rc = (P.precision == SPOCK_FP64) ? solve_impl<double>(P, x0_dev, *s, static_cast<double*>(v_io), loc, st)
                                     : solve_impl<float>(P, x0_dev, *s, static_cast<float*>(v_io), loc, st);
  }
  if (rc) return rc;
  // s^0 and, on request, the nested cost of the returned trajectory
  const Tree& T = *P.tree;
  const size_t nxu = (size_t)T.nn * P.nx + (size_t)T.nl * P.nu;
  std::vector<double> hv(1 + nxu);
  if (P.precision == SPOCK_FP64) {
    HIP_TRY(hipMemcpy(hv.data(), v_io, (s->compute_nested ? 1 + nxu : 1) * sizeof(double),
                      hipMemcpyDeviceToHost));
  } else {
    std::vector<float> hf(1 + nxu);
    HIP_TRY(hipMemcpy(hf.data(), v_io, (s->compute_nested ? 1 + nxu : 1) * sizeof(float),
                      hipMemcpyDeviceToHost));
    for (size_t e = 0; e < hf.size(); ++e) hv[e] = hf[e];
  }
  loc.V_s0 = hv[0];
  if (s->compute_nested && !P.general) {
    std::vector<double> x(hv.begin() + 1, hv.begin() + 1 + (size_t)T.nn * P.nx);
    std::vector<double> u(hv.begin() + 1 + (size_t)T.nn * P.nx, hv.end());
    loc.V_nested = nested_cost(T, P.nx, P.nu, P.q.data(), P.r.data(), P.qN.data(), P.a_risk.data(), x, u);
  }
  loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *info = loc;
  return SPOCK_OK;
}

// ============================================================== operator entry points
extern "C" int spock_apply_L(spock_problem* ph, const void* z, void* eta, void* stream) {
  if (!ph || !z || !eta) return SPOCK_EINVAL;
  Problem& P = ph->p;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = (P.precision == SPOCK_FP64)
                     ? launch_L<double>(P, static_cast<const double*>(z), static_cast<double*>(eta), st)
                     : launch_L<float>(P, static_cast<const float*>(z), static_cast<float*>(eta), st);
  return e == hipSuccess ? SPOCK_OK : SPOCK_EHIP;
}

extern "C" int spock_apply_Lt(spock_problem* ph, const void* eta, void* z, void* stream) {
  if (!ph || !z || !eta) return SPOCK_EINVAL;
  Problem& P = ph->p;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = (P.precision == SPOCK_FP64)
                     ? launch_Lt<double>(P, static_cast<const double*>(eta), static_cast<double*>(z), st)
                     : launch_Lt<float>(P, static_cast<const float*>(eta), static_cast<float*>(z), st);
  return e == hipSuccess ? SPOCK_OK : SPOCK_EHIP;
}

extern "C" int spock_prox_gstar(spock_problem* ph, const void* w, void* out, void* stream) {
  if (!ph || !w || !out) return SPOCK_EINVAL;
  Problem& P = ph->p;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = (P.precision == SPOCK_FP64)
                     ? launch_prox_gstar<double>(P, static_cast<const double*>(w), static_cast<double*>(out), st)
                     : launch_prox_gstar<float>(P, static_cast<const float*>(w), static_cast<float*>(out), st);
  return e == hipSuccess ? SPOCK_OK : SPOCK_EHIP;
}

namespace {
// With the dataflow form, the operator entry points synchronise to read
// the sweeps' error word; after a give-up they switch the problem to the
// per-stage form and evaluate again.
template <typename S>
int prox_f_impl(Problem& P, const S* zin, const double* x0, S* zout, hipStream_t st) {
  for (int attempt = 0;; ++attempt) {
    Work<S> W;
    int rc = ensure_work<S>(P, W);
    if (rc) return rc;
    HIP_TRY(launch_fill<S>(P.neta, W.eta_zero, 0.0, st));
    HIP_TRY(launch_T<S>(P, zin, zout, x0, W.q, W.d, W.xbar, W.ubar, W.partials, W.stats, st, W.eta_zero, false));
    bool gave_up = false;
    rc = flow_gave_up(P, st, gave_up);
    if (rc) return rc;
    if (!gave_up) return SPOCK_OK;
    if (attempt > 0) return SPOCK_EHIP;
    rc = flow_fallback(P);
    if (rc) return rc;
  }
}
template <typename S>
int T_impl(Problem& P, const S* v, const double* x0, S* Tv, double* stats, hipStream_t st) {
  Work<S> W;
  int rc = ensure_work<S>(P, W);
  if (rc) return rc;
  HIP_TRY(launch_T<S>(P, v, Tv, x0, W.q, W.d, W.xbar, W.ubar, W.partials, W.stats, st, W.eta_zero, true));
  bool gave_up = false;
  rc = flow_gave_up(P, st, gave_up);
  if (rc) return rc;
  if (gave_up) {
    rc = flow_fallback(P);
    if (rc) return rc;
    return T_impl<S>(P, v, x0, Tv, stats, st);
  }
  if (stats) {
    HIP_TRY(hipMemcpyAsync(stats, W.stats, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  return SPOCK_OK;
}
}  // namespace

extern "C" int spock_prox_f(spock_problem* ph, const void* zin, const double* x0, void* zout, void* stream) {
  if (!ph || !zin || !zout || !x0) return SPOCK_EINVAL;
  Problem& P = ph->p;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return (P.precision == SPOCK_FP64)
             ? prox_f_impl<double>(P, static_cast<const double*>(zin), x0, static_cast<double*>(zout), st)
             : prox_f_impl<float>(P, static_cast<const float*>(zin), x0, static_cast<float*>(zout), st);
}

extern "C" int spock_T(spock_problem* ph, const void* v, const double* x0, void* Tv, double* stats,
                       void* stream) {
  if (!ph || !v || !Tv || !x0) return SPOCK_EINVAL;
  Problem& P = ph->p;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return (P.precision == SPOCK_FP64)
             ? T_impl<double>(P, static_cast<const double*>(v), x0, static_cast<double*>(Tv), stats, st)
             : T_impl<float>(P, static_cast<const float*>(v), x0, static_cast<float*>(Tv), stats, st);
}

// ============================================================== allocation-free T
// Fixed device scratch of the allocation-free entry point: the sweep
// buffers (q, d, xbar, ubar) and the statistic partials of one evaluation of
// T. Every GPU the library runs on holds its own copy until the process
// ends. Host code never uses the array's name as an address: the device
// address comes from hipGetSymbolAddress, once per device.
namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kScratchDevices = 64;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

int scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return SPOCK_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SPOCK_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SPOCK_OK;
}

template <typename S>
int T_noalloc_impl(const Problem& P, const S* v, const double* x0, S* Tv, double* stats, hipStream_t st) {
  const Tree& T = *P.tree;
  size_t off = 0;
  auto place = [&](size_t bytes) {
    const size_t at = off;
    off = (off + bytes + 255) & ~size_t(255);
    return at;
  };
  const size_t oq = place(sizeof(S) * (size_t)T.nn * P.nx), od = place(sizeof(S) * (size_t)T.nn * P.nu);
  const size_t oxb = place(sizeof(S) * (size_t)T.nn * P.nx), oub = place(sizeof(S) * (size_t)T.nn * P.nu);
  const size_t opart = place(sizeof(double) * (size_t)(T.nl + 1) * kStats), ostat = place(sizeof(double) * 8);
  if (off > kScratchBytes) return SPOCK_ETOOBIG;
  void* base = nullptr;
  int rc = scratch_address(&base);
  if (rc) return rc;
  char* b = static_cast<char*>(base);
  // the per-stage sweeps (the dataflow form keeps exchange buffers of its own)
  SweepMap map;
  if (P.team == kTeamFlow) {
    map.team = kTeamWG;
    map.cut = std::max(default_cut(T), std::max(0, T.N - 64));
  } else {
    map.team = P.team;
    map.cut = P.cut;
  }
  // every scratch word an evaluation reads it first writes: nothing needs clearing
  HIP_TRY(launch_T<S>(P, v, Tv, x0, reinterpret_cast<S*>(b + oq), reinterpret_cast<S*>(b + od),
                      reinterpret_cast<S*>(b + oxb), reinterpret_cast<S*>(b + oub),
                      reinterpret_cast<double*>(b + opart), reinterpret_cast<double*>(b + ostat), st, nullptr,
                      true, Publish{}, map));
  if (stats) {
    HIP_TRY(hipMemcpyAsync(stats, b + ostat, 6 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  return SPOCK_OK;
}
}  // namespace

extern "C" int spock_T_noalloc(spock_problem* ph, const void* v, const double* x0, void* Tv, double* stats,
                               void* stream) {
  if (!ph || !v || !Tv || !x0) return SPOCK_EINVAL;
  const Problem& P = ph->p;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return (P.precision == SPOCK_FP64)
             ? T_noalloc_impl<double>(P, static_cast<const double*>(v), x0, static_cast<double*>(Tv), stats, st)
             : T_noalloc_impl<float>(P, static_cast<const float*>(v), x0, static_cast<float*>(Tv), stats, st);
}

extern "C" int spock_profile_T(spock_problem* ph, const void* v, const double* x0, void* Tv, int32_t reps,
                               double* us, void* stream) {
  if (!ph || !v || !Tv || !x0 || !us || reps < 1) return SPOCK_EINVAL;
  Problem& P = ph->p;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // untimed evaluation first (autotuning-free: the current mapping is used)
  int rc = (P.precision == SPOCK_FP64)
               ? T_impl<double>(P, static_cast<const double*>(v), x0, static_cast<double*>(Tv), nullptr, st)
               : T_impl<float>(P, static_cast<const float*>(v), x0, static_cast<float*>(Tv), nullptr, st);
  if (rc) return rc;
  hipEvent_t ev[5];
  for (int k = 0; k < 5; ++k)
    if (hipEventCreate(&ev[k]) != hipSuccess) return SPOCK_EHIP;
  double acc[5] = {0, 0, 0, 0, 0};
  P.prof = ev;
  for (int r = 0; r < reps && rc == SPOCK_OK; ++r) {
    rc = (P.precision == SPOCK_FP64)
             ? T_impl<double>(P, static_cast<const double*>(v), x0, static_cast<double*>(Tv), nullptr, st)
             : T_impl<float>(P, static_cast<const float*>(v), x0, static_cast<float*>(Tv), nullptr, st);
    if (rc) break;
    if (hipEventSynchronize(ev[4]) != hipSuccess) rc = SPOCK_EHIP;
    for (int k = 0; k < 4 && rc == SPOCK_OK; ++k) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, ev[k], ev[k + 1]) != hipSuccess) rc = SPOCK_EHIP;
      acc[k] += ms;
      acc[4] += ms;
    }
  }
  P.prof = nullptr;
  for (int k = 0; k < 5; ++k) (void)hipEventDestroy(ev[k]);
  if (rc) return rc;
  for (int k = 0; k < 5; ++k) us[k] = acc[k] * 1e3 / reps;
  return SPOCK_OK;
}

// ============================================================== batched
namespace {

struct BatchCache {
  void* work = nullptr;
  size_t bytes = 0;
  void* desc = nullptr;
  size_t desc_bytes = 0;
  double* infos = nullptr;
  size_t infos_n = 0;
  std::vector<std::pair<std::vector<long long>, int>> tuned;  // key -> team
  // the instantiated graph of the last launch, reused while its arguments
  // (descriptor and info buffers, settings, team, grid) stay the same
  hipGraphExec_t exec = nullptr;
  std::vector<unsigned char> exec_key;
  hipStream_t cap = nullptr;  // capture stream (created once)
};
BatchCache& batch_cache() {
  static BatchCache c;
  return c;
}

template <typename S>
int batched_impl(int B, spock_problem* const* probs, const double* const* x0, const spock_settings& st,
                 void* const* vio, spock_info* infos, hipStream_t stream) {
  BatchCache& C = batch_cache();
  const Problem& P0 = probs[0]->p;
  const int nx = P0.nx, nu = P0.nu;
  const size_t pool = batched_pool_vectors();
  // workspace: pool vectors + sweep buffers per instance
  std::vector<size_t> off(B);
  size_t total = 0;
  for (int b = 0; b < B; ++b) {
    const Problem& P = probs[b]->p;
    off[b] = total;
    const size_t elems = pool * (size_t)(P.nz + P.neta) + (size_t)P.tree->nn * (2 * nx + 2 * nu);
    total += (elems * sizeof(S) + 255) & ~size_t(255);
  }
  if (C.bytes < total) {
    if (C.work) (void)hipFree(C.work);
    C.work = nullptr;
    C.bytes = 0;
    if (hipMalloc(&C.work, total) != hipSuccess) return SPOCK_ENOMEM;
    C.bytes = total;
  }
  std::vector<BatchInst<S>> h(B);
  for (int b = 0; b < B; ++b) {
    const Problem& P = probs[b]->p;
    h[b].P = (sizeof(S) == 8) ? *reinterpret_cast<const DevProb<S>*>(&P.dp64)
                              : *reinterpret_cast<const DevProb<S>*>(&P.dp32);
    h[b].stage_off = P.d_stage_off;
    h[b].x0 = x0[b];
    h[b].vio = static_cast<S*>(vio[b]);
    h[b].work = reinterpret_cast<S*>(static_cast<char*>(C.work) + off[b]);
    h[b].nv = P.nz + P.neta;
  }
  const size_t dbytes = sizeof(BatchInst<S>) * B;
  if (C.desc_bytes < dbytes) {
    if (C.desc) (void)hipFree(C.desc);
    C.desc = nullptr;
    C.desc_bytes = 0;
    if (hipMalloc(&C.desc, dbytes) != hipSuccess) return SPOCK_ENOMEM;
    C.desc_bytes = dbytes;
  }
  if (C.infos_n < (size_t)B * 16) {
    if (C.infos) (void)hipFree(C.infos);
    C.infos = nullptr;
    C.infos_n = 0;
    if (hipMalloc(&C.infos, sizeof(double) * 16 * B) != hipSuccess) return SPOCK_ENOMEM;
    C.infos_n = (size_t)B * 16;
  }
  HIP_TRY(hipMemcpyAsync(C.desc, h.data(), dbytes, hipMemcpyHostToDevice, stream));
  BatchSettings bs{st.eps_abs, st.eps_rel, st.max_iters, st.method, st.m, st.max_ls, st.c0, st.c1,
                   st.c2, st.beta, st.sigma, st.lambda, 1};
  const int VM = (std::max(nx, nu) + 3) & ~3;
  const int grid = B;
  const auto* dev_desc = static_cast<const BatchInst<S>*>(C.desc);
  // ---- team size: autotuned once per batch shape (short runs, no output)
  std::vector<long long> key = {nx, nu, (long long)sizeof(S), B};
  for (int b = 0; b < B; ++b) key.push_back(probs[b]->p.tree->nn);
  // the block engine needs T >= max(nx, nu) lanes per family
  const int tmin = next_pow2_team(std::max(nx, nu));
  int team = -1;
  if (const char* env = std::getenv("SPOCK_BATCH_TEAM")) {
    const int v = std::atoi(env);
    if (v == 8 || v == 16 || v == 32 || v == 64) team = std::max(v, tmin);
  }
  for (auto& kv : C.tuned)
    if (team < 0 && kv.first == key) team = kv.second;
  if (team < 0) {
    BatchSettings tb = bs;
    tb.write_out = 0;
    tb.max_iters = std::min(st.max_iters, 20);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    for (int cand : {8, 16, 32, 64}) {
      if (cand < tmin) continue;
      if ((size_t)(256 / cand) * 3 * VM * sizeof(S) > 48 * 1024) continue;
      HIP_TRY(hipEventRecord(e0, stream));
      HIP_TRY(launch_solve_batched<S>(dev_desc, B, tb, cand, VM, C.infos, grid, stream));
      HIP_TRY(hipEventRecord(e1, stream));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) {
        best = ms;
        team = cand;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (team < 0) team = 64;
    C.tuned.push_back({key, team});
  }
  // ---- the persistent launch, captured in a graph (instantiated once per
  // set of launch arguments and kept)
  {
    std::vector<unsigned char> key2(sizeof(BatchSettings) + 6 * sizeof(long long));
    const long long parts[6] = {(long long)(uintptr_t)dev_desc, (long long)(uintptr_t)C.infos, B, team, VM,
                                (long long)sizeof(S)};
    std::memcpy(key2.data(), &bs, sizeof(BatchSettings));
    std::memcpy(key2.data() + sizeof(BatchSettings), parts, sizeof(parts));
    if (!C.exec || C.exec_key != key2) {
      if (C.exec) (void)hipGraphExecDestroy(C.exec);
      C.exec = nullptr;
      C.exec_key.clear();
      if (!C.cap) HIP_TRY(hipStreamCreateWithFlags(&C.cap, hipStreamNonBlocking));
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(C.cap, hipStreamCaptureModeThreadLocal));
      const hipError_t le = launch_solve_batched<S>(dev_desc, B, bs, team, VM, C.infos, grid, C.cap);
      const hipError_t ee = hipStreamEndCapture(C.cap, &graph);
      if (le != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return SPOCK_EHIP;
      }
      hipGraphExec_t exec = nullptr;
      const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) return SPOCK_EHIP;
      C.exec = exec;
      C.exec_key = key2;
    }
  }
  HIP_TRY(hipGraphLaunch(C.exec, stream));
  std::vector<double> hi((size_t)16 * B);
  HIP_TRY(hipMemcpyAsync(hi.data(), C.infos, sizeof(double) * 16 * B, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  for (int b = 0; b < B; ++b) {
    const double* r = hi.data() + (size_t)16 * b;
    spock_info& I = infos[b];
    I = spock_info{};
    I.status = (int)r[0];
    I.iters = (int)r[1];
    I.t_evals = (int)r[2];
    I.n_k0 = (int)r[3];
    I.n_k1 = (int)r[4];
    I.n_k2 = (int)r[5];
    I.n_km = (int)r[6];
    I.n_backtracks = (int)r[7];
    I.V_s0 = r[8];
    I.xi0 = r[9];
    I.xi = r[10];
    I.V_nested = std::numeric_limits<double>::quiet_NaN();
    I.mapping = team;
  }
  return SPOCK_OK;
}

}  // namespace

extern "C" int spock_solve_batched(int32_t B, spock_problem* const* probs, const double* const* x0,
                                   const spock_settings* s, void* const* v_io, spock_info* infos,
                                   void* stream) {
  if (B < 1 || !probs || !x0 || !s || !v_io || !infos) return SPOCK_EINVAL;
  if (s->method != SPOCK_METHOD_CP && s->method != SPOCK_METHOD_SPOCK) return SPOCK_EINVAL;
  // the batched engine keeps the Gram solve in the workgroup: memory up to kAAMax
  if (s->method == SPOCK_METHOD_SPOCK && (s->m < 1 || s->m > kAAMax || s->anderson == SPOCK_AA_QR))
    return SPOCK_EINVAL;
  if (!(s->eps_abs >= 0 && s->eps_rel >= 0) || s->max_iters < 0 || s->max_ls < 1) return SPOCK_EINVAL;
  if (!(s->beta > 0 && s->beta < 1 && s->sigma > 0 && s->sigma < 1 && s->lambda > 0 && s->lambda < 2))
    return SPOCK_EINVAL;
  for (int b = 0; b < B; ++b) {
    if (!probs[b] || !x0[b] || !v_io[b]) return SPOCK_EINVAL;
    const Problem& P = probs[b]->p;
    if (P.precision != probs[0]->p.precision || P.nx != probs[0]->p.nx || P.nu != probs[0]->p.nu)
      return SPOCK_EINVAL;
    if (P.general) return SPOCK_EUNSUPPORTED;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  // instances of one problem (one tree and one set of data): the shared-tree
  // form with the sweeps on the matrix cores, unless SPOCK_SHARED=0
  bool shared = B >= 2;
  for (int b = 1; b < B && shared; ++b) shared = probs[b] == probs[0];
  if (const char* env = std::getenv("SPOCK_SHARED")) shared = shared && std::string(env) != "0";
  int rc;
  if (shared)
    rc = (probs[0]->p.precision == SPOCK_FP64) ? shared_solve<double>(probs[0]->p, B, x0, *s, v_io, infos, st)
                                               : shared_solve<float>(probs[0]->p, B, x0, *s, v_io, infos, st);
  else
    rc = (probs[0]->p.precision == SPOCK_FP64) ? batched_impl<double>(B, probs, x0, *s, v_io, infos, st)
                                               : batched_impl<float>(B, probs, x0, *s, v_io, infos, st);
  if (rc) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int b = 0; b < B; ++b) {
    infos[b].seconds = secs;
    if (s->compute_nested && infos[b].status != 3) {
      const Problem& P = probs[b]->p;
      const Tree& T = *P.tree;
      const size_t nxu = (size_t)T.nn * P.nx + (size_t)T.nl * P.nu;
      std::vector<double> hv(1 + nxu);
      if (P.precision == SPOCK_FP64) {
        HIP_TRY(hipMemcpy(hv.data(), v_io[b], (1 + nxu) * sizeof(double), hipMemcpyDeviceToHost));
      } else {
        std::vector<float> hf(1 + nxu);
        HIP_TRY(hipMemcpy(hf.data(), v_io[b], (1 + nxu) * sizeof(float), hipMemcpyDeviceToHost));
        for (size_t e = 0; e < hf.size(); ++e) hv[e] = hf[e];
      }
      std::vector<double> x(hv.begin() + 1, hv.begin() + 1 + (size_t)T.nn * P.nx);
      std::vector<double> u(hv.begin() + 1 + (size_t)T.nn * P.nx, hv.end());
      infos[b].V_nested = nested_cost(T, P.nx, P.nu, P.q.data(), P.r.data(), P.qN.data(), P.a_risk.data(), x, u);
    }
  }
  return SPOCK_OK;
}

// ============================================================== backward
namespace {

template <typename S>
int backward_once(Problem& P, const S* vstar, const double* x0, double gV, const double* gu0,
                  double* gx0, double* gq, double* gqN, const spock_settings& s, spock_info& info,
                  hipStream_t st) {
  Work<S> W;
  int rc = ensure_work<S>(P, W);
  if (rc) return rc;
  const Tree& T = *P.tree;
  const long long nz = P.nz, ne = P.neta, nv = nz + ne;
  const double al = P.alpha;
  S* Tv = W.pool[0];
  S* dz = W.pool[1];
  S* Ldz = W.pool[2];
  S* b = W.pool[3];
  S* g = W.pool[4];
  S* w = W.pool[5];
  S* wn = W.pool[6];
  S* lb = W.pool[7];
  S* cz = W.pool[8];
  S* la = W.pool[9];
  S* tz = W.pool[10];
  S* te = W.pool[11];
  // pre-prox point of the dual update at v*: b* = eta* + alpha L (2 z+ - z*)
  HIP_TRY(launch_T<S>(P, vstar, Tv, x0, W.q, W.d, W.xbar, W.ubar, W.partials, W.stats, st, W.eta_zero, true));
  HIP_TRY(launch_lincomb<S>(nz, dz, 2.0, Tv, -1.0, vstar, st));
  HIP_TRY(launch_L<S>(P, dz, Ldz, st));
  HIP_TRY(launch_lincomb<S>(ne, b, 1.0, vstar + nz, al, Ldz, st));
  // cotangent of v*: gV on s^0, gu0 on u^0
  HIP_TRY(launch_fill<S>(nv, g, 0.0, st));
  {
    std::vector<S> head(1 + (size_t)T.nn * P.nx + P.nu, S(0));
    HIP_TRY(hipMemcpyAsync(head.data(), g, head.size() * sizeof(S), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    head[0] = (S)gV;
    if (gu0) {
      std::vector<double> hu(P.nu);
      HIP_TRY(hipMemcpy(hu.data(), gu0, P.nu * sizeof(double), hipMemcpyDeviceToHost));
      const size_t u0 = 1 + (size_t)T.nn * P.nx;  // u^0 follows every x^i
      for (int k = 0; k < P.nu; ++k) head[u0 + k] = (S)hu[k];
    }
    HIP_TRY(hipMemcpyAsync(g, head.data(), head.size() * sizeof(S), hipMemcpyHostToDevice, st));
  }
  HIP_TRY(launch_lincomb<S>(nv, w, 1.0, g, 0.0, nullptr, st));
  S* zeros = W.pool[12];
  HIP_TRY(launch_fill<S>(nv, zeros, 0.0, st));
  HIP_TRY(hipMemsetAsync(W.x0_zero, 0, sizeof(double) * kMaxDim, st));
  HIP_TRY(launch_fill<S>(ne, W.eta_zero, 0.0, st));
  // one application of the transposed operator: writes lb, tz, cz, la
  auto partial = [&](const S* wv) -> int {
    HIP_TRY(launch_jg<S>(P, b, wv + nz, lb, st));                  // lambda_b = J_G w_eta
    HIP_TRY(launch_Lt<S>(P, lb, tz, st));                          // L* lambda_b
    HIP_TRY(launch_lincomb<S>(nz, cz, 1.0, wv, 2.0 * al, tz, st)); // c = w_z + 2 alpha L* lambda_b
    HIP_TRY(launch_T<S>(P, cz, la, W.x0_zero, W.q, W.d, W.xbar, W.ubar, W.partials, W.stats, st,
                        W.eta_zero, false));                         // J_f c (S1 with x0 = 0, S2)
    HIP_TRY(launch_copy_elem<S>(la, cz, st));                        // identity on s^0
    return SPOCK_OK;
  };
  const double tol = std::max(s.eps_abs, 1e-15);
  int k = 0;
  double diff = 0;
  info.status = SPOCK_MAXITER;
  std::vector<double> hd(2);
  // w -> A(w) = J_T(v*)' w + g (affine): the transposed operator, L of its
  // dual part, and the cotangent
  auto apply_A = [&](const S* wv, S* out) -> int {
    if (int r = partial(wv)) return r;
    HIP_TRY(launch_L<S>(P, la, te, st));
    HIP_TRY(launch_lincomb3<S>(nz, out, 1.0, la, -al, tz, 1.0, g, st));
    HIP_TRY(launch_lincomb3<S>(ne, out + nz, 1.0, lb, -al, te, 1.0, g + nz, st));
    return SPOCK_OK;
  };
  // The fixed point of the affine map solves (I - J_T') w = g: restarted
  // GMRES (kAdjRestart Krylov vectors, 120 or 30 as below unless
  // SPOCK_ADJ_RESTART gives 2 to 120; about 3x fewer evaluations of A than the plain iteration on the
  // 95-node tree at 1e-12; on eight instances of that tree 120 takes 35%
  // fewer evaluations than 30, and with the Gram-Schmidt passes as single
  // launches over the whole basis an evaluation costs the same at either
  // length; classical Gram-Schmidt with one
  // reorthogonalisation, FP64 dot products and Hessenberg least squares on
  // the host), M v = v - A(v) + g. Convergence is judged on the true
  // residual |w - A(w)|_inf <= eps max(1, |w|_inf) at every restart; k counts
  // the evaluations of A.
  constexpr int kAdjMax = 120;
  // Small problems are launch-bound, and the passes cost little at any
  // length; on large ones the passes stream the basis (about 4 reads of it
  // per step), so the length stays at 30 once the basis would pass 256 MiB.
  int kAdjRestart = sizeof(S) * (size_t)(kAdjMax + 1) * (size_t)nv <= (size_t(256) << 20) ? kAdjMax : 30;
  if (const char* env = std::getenv("SPOCK_ADJ_RESTART")) kAdjRestart = std::max(2, std::min(kAdjMax, std::atoi(env)));
  S* Aw = wn;
  static_assert(kAdjMax + 1 <= kBasisMax, "basis kernels hold every Krylov vector");
  // Krylov vectors, the dot products of one Gram-Schmidt pass and their
  // per-chunk partial sums
  const size_t basis_bytes = (sizeof(S) * (size_t)(kAdjRestart + 1) * (size_t)nv + 255) & ~size_t(255);
  const size_t dots_bytes = sizeof(double) * 2 * (kAdjMax + 2);  // the two passes' coefficients
  void* kmem = nullptr;
  if (hipMalloc(&kmem, basis_bytes + dots_bytes + sizeof(double) * (size_t)(kAdjMax + 2) * kBasisChunks) !=
      hipSuccess)
    return SPOCK_ENOMEM;
  struct KrylovGuard {
    void* p;
    ~KrylovGuard() { (void)hipFree(p); }
  } guard{kmem};
  S* basis = static_cast<S*>(kmem);
  auto V = [&](int j) { return basis + (size_t)j * (size_t)nv; };
  double* dots_dev = reinterpret_cast<double*>(static_cast<char*>(kmem) + basis_bytes);
  double* dots_part = reinterpret_cast<double*>(static_cast<char*>(kmem) + basis_bytes + dots_bytes);
  // h[i] = <V_i, x> for i < n, and h[n] = <x, x> when xx: one pair of
  // launches and one synchronisation
  auto dots_with = [&](int n, const S* x, double* h, bool xx) -> int {
    HIP_TRY(launch_basis_dots<S>(nv, n, basis, nv, x, xx, dots_part, dots_dev, st));
    HIP_TRY(hipMemcpyAsync(h, dots_dev, sizeof(double) * (n + (xx ? 1 : 0)), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SPOCK_OK;
  };
  // out = a x + sum_{i < n} c_i V_i (out may be x), one launch
  auto mix = [&](S* out, double a, const S* x, int n, const double* c) -> int {
    BasisCoef C{};
    for (int j = 0; j < n; ++j) C.c[j] = c[j];
    HIP_TRY(launch_basis_mix<S>(nv, n, basis, nv, C, a, x, out, st));
    return SPOCK_OK;
  };
  // Arnoldi steps are pipelined: the passes take their coefficients from
  // device memory, the reduction kernels also write them to mapped pinned
  // host memory, and the host reduces column j of the Hessenberg matrix
  // while step j + 1 runs (two slots, alternating).
  double* d1 = dots_dev;
  double* d2 = dots_dev + (kAdjMax + 2);
  double* hp = nullptr;
  if (hipHostMalloc(reinterpret_cast<void**>(&hp), sizeof(double) * 4 * (kAdjMax + 2),
                    hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
    return SPOCK_ENOMEM;
  hipEvent_t evs[2] = {nullptr, nullptr};
  struct PipeGuard {
    double* hp;
    hipEvent_t* ev;
    ~PipeGuard() {
      for (int e = 0; e < 2; ++e)
        if (ev[e]) (void)hipEventDestroy(ev[e]);
      (void)hipHostFree(hp);
    }
  } pguard{hp, evs};
  for (int e = 0; e < 2; ++e)
    if (hipEventCreateWithFlags(&evs[e], hipEventDisableTiming) != hipSuccess) return SPOCK_EHIP;
  double* hp_dev = nullptr;  // the kernels write the slots through this view
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&hp_dev), hp, 0) != hipSuccess) return SPOCK_EHIP;
  auto norm_inf_check = [&](const S* x, const S* Ax, double& res, double& xn) -> int {
    HIP_TRY(launch_maxdiff<S>(nv, x, Ax, W.vpart, W.dots, st));
    HIP_TRY(launch_maxdiff<S>(nv, x, zeros, W.vpart, W.dots + 1, st));
    HIP_TRY(hipMemcpyAsync(hd.data(), W.dots, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    res = hd[0];
    xn = hd[1];
    return SPOCK_OK;
  };
  for (;;) {
    if (int r = apply_A(w, Aw)) return r;
    ++k;
    double xn = 0;
    if (int r = norm_inf_check(w, Aw, diff, xn)) return r;
    bool gave_up = false;
    rc = flow_gave_up(P, st, gave_up);
    if (rc) return rc;
    if (gave_up) return kFlowGaveUp;
    if (!std::isfinite(diff)) {
      info.status = SPOCK_NUMERICAL;
      break;
    }
    const double thr = tol * std::max(1.0, xn);
    if (diff <= thr) {
      info.status = SPOCK_CONVERGED;
      break;
    }
    if (k >= s.max_iters) break;
    // r = A(w) - w = g - M w; V_0 = r / |r|
    HIP_TRY(launch_lincomb<S>(nv, V(0), 1.0, Aw, -1.0, w, st));
    double beta = 0;
    if (int r = dots_with(0, V(0), &beta, true)) return r;
    beta = std::sqrt(beta);
    if (!(beta > 0.0) || !std::isfinite(beta)) {
      info.status = std::isfinite(beta) ? SPOCK_CONVERGED : SPOCK_NUMERICAL;
      break;
    }
    HIP_TRY(launch_lincomb<S>(nv, V(0), 1.0 / beta, V(0), 0.0, nullptr, st));
    std::vector<double> Hm((size_t)(kAdjMax + 1) * kAdjMax, 0.0);
    auto H = [&](int i, int j) -> double& { return Hm[(size_t)i * kAdjMax + j]; };
    double cs[kAdjMax] = {}, sn[kAdjMax] = {}, gv[kAdjMax + 1] = {};
    gv[0] = beta;
    int jn = 0;
    // column j of H from slot j & 1 (the two passes' dots, <v, v> before
    // the second); true when the Krylov space is done (small residual or a
    // breakdown): the step launched after it is then discarded
    auto column = [&](int j) -> int {
      HIP_TRY(hipEventSynchronize(evs[j & 1]));
      const double* h1 = hp + (size_t)(j & 1) * 2 * (kAdjMax + 2);
      const double* h2 = h1 + (kAdjMax + 2);
      double hn = h2[j + 1];
      for (int i = 0; i <= j; ++i) {
        H(i, j) = h1[i] + h2[i];
        hn -= h2[i] * h2[i];
      }
      hn = std::sqrt(std::max(hn, 0.0));
      H(j + 1, j) = hn;
      for (int i = 0; i < j; ++i) {  // earlier rotations on column j
        const double x = H(i, j), y = H(i + 1, j);
        H(i, j) = cs[i] * x + sn[i] * y;
        H(i + 1, j) = -sn[i] * x + cs[i] * y;
      }
      const double rr = std::hypot(H(j, j), H(j + 1, j));
      cs[j] = rr > 0.0 ? H(j, j) / rr : 1.0;
      sn[j] = rr > 0.0 ? H(j + 1, j) / rr : 0.0;
      H(j, j) = rr;
      H(j + 1, j) = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      jn = j + 1;
      if (!std::isfinite(gv[j + 1])) return 1;
      if (std::fabs(gv[j + 1]) <= 0.5 * thr || !(hn > 0.0)) return 1;
      return 0;
    };
    int j = 0;
    bool done = false;
    for (; j < kAdjRestart && k < s.max_iters; ++j) {
      // V_{j+1} <- M V_j = V_j - A(V_j) + g, then two Gram-Schmidt passes
      // and the normalisation, all on the device
      if (int r = apply_A(V(j), Aw)) return r;
      ++k;
      HIP_TRY(launch_lincomb3<S>(nv, V(j + 1), 1.0, V(j), -1.0, Aw, 1.0, g, st));
      double* slot = hp_dev + (size_t)(j & 1) * 2 * (kAdjMax + 2);
      HIP_TRY(launch_basis_dots<S>(nv, j + 1, basis, nv, V(j + 1), false, dots_part, d1, st, slot));
      HIP_TRY(launch_basis_orth<S>(nv, j + 1, basis, nv, d1, false, V(j + 1), st));
      HIP_TRY(launch_basis_dots<S>(nv, j + 1, basis, nv, V(j + 1), true, dots_part, d2, st, slot + (kAdjMax + 2)));
      HIP_TRY(launch_basis_orth<S>(nv, j + 1, basis, nv, d2, true, V(j + 1), st));
      HIP_TRY(hipEventRecord(evs[j & 1], st));
      if (j > 0) {
        const int r = column(j - 1);
        if (r < 0) return r;
        if (r > 0) {
          done = true;
          break;
        }
      }
    }
    if (!done && j > 0) {
      const int r = column(j - 1);
      if (r < 0) return r;
    }
    // w += V y, H y = g (upper triangular)
    double y[kAdjMax] = {};
    for (int i = jn - 1; i >= 0; --i) {
      double t = gv[i];
      for (int l = i + 1; l < jn; ++l) t -= H(i, l) * y[l];
      y[i] = H(i, i) != 0.0 ? t / H(i, i) : 0.0;
    }
    if (int r = mix(w, 1.0, w, jn, y)) return r;
  }
  info.iters = k;
  info.xi = diff;
  // gradients from the converged adjoint
  rc = partial(w);
  if (rc) return rc;
  {
    bool gave_up = false;
    rc = flow_gave_up(P, st, gave_up);
    if (rc) return rc;
    if (gave_up) return kFlowGaveUp;
  }
  S* mu = W.q;
  HIP_TRY(launch_phiT<S>(P, cz, mu, st));
  {
    std::vector<S> hm(P.nx);
    HIP_TRY(hipMemcpyAsync(hm.data(), mu, P.nx * sizeof(S), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<double> out(P.nx);
    for (int j = 0; j < P.nx; ++j) out[j] = hm[j];
    HIP_TRY(hipMemcpy(gx0, out.data(), P.nx * sizeof(double), hipMemcpyHostToDevice));
  }
  if (gq) HIP_TRY(hipMemsetAsync(gq, 0, sizeof(double) * (size_t)T.nn * P.nx, st));
  if (gqN) HIP_TRY(hipMemsetAsync(gqN, 0, sizeof(double) * (size_t)T.nn * P.nx, st));
  if (gq || gqN) HIP_TRY(launch_grad_q<S>(P, vstar, la, lb, gq, gqN, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SPOCK_OK;
}

// The adjoint iteration; redone from its start with the per-stage form if a
// bounded wait of the dataflow sweeps gave up during it.
template <typename S>
int backward_impl(Problem& P, const S* vstar, const double* x0, double gV, const double* gu0,
                  double* gx0, double* gq, double* gqN, const spock_settings& s, spock_info& info,
                  hipStream_t st) {
  int rc = backward_once<S>(P, vstar, x0, gV, gu0, gx0, gq, gqN, s, info, st);
  if (rc != kFlowGaveUp) return rc;
  rc = flow_fallback(P);
  if (rc) return rc;
  info.flow_fallback = 1;
  info.mapping = P.team;
  rc = backward_once<S>(P, vstar, x0, gV, gu0, gx0, gq, gqN, s, info, st);
  return rc == kFlowGaveUp ? SPOCK_EHIP : rc;
}

}  // namespace

extern "C" int spock_backward_batched(spock_problem* ph, int32_t B, const void* const* v_star,
                                      const double* const* x0, double gV, const double* const* gu0,
                                      double* const* grad_x0, double* const* grad_q, double* const* grad_qN,
                                      const spock_settings* s, spock_info* infos, void* stream) {
  if (!ph || B < 1 || !v_star || !x0 || !grad_x0 || !s || !infos || s->max_iters < 1) return SPOCK_EINVAL;
  for (int b = 0; b < B; ++b)
    if (!v_star[b] || !x0[b] || !grad_x0[b]) return SPOCK_EINVAL;
  Problem& P = ph->p;
  if (P.general) return SPOCK_EUNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<spock_info> loc(B);
  const int rc = (P.precision == SPOCK_FP64)
                     ? shared_backward<double>(P, B, v_star, x0, gV, gu0, grad_x0, grad_q, grad_qN, *s, loc.data(), st)
                     : shared_backward<float>(P, B, v_star, x0, gV, gu0, grad_x0, grad_q, grad_qN, *s, loc.data(), st);
  if (rc) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int b = 0; b < B; ++b) {
    loc[b].seconds = secs;
    infos[b] = loc[b];
  }
  return SPOCK_OK;
}

extern "C" int spock_backward(spock_problem* ph, const void* v_star, const double* x0, double gV,
                              const double* gu0, double* grad_x0, double* grad_q, double* grad_qN,
                              const spock_settings* s, spock_info* info, void* stream) {
  if (!ph || !v_star || !x0 || !grad_x0 || !s || !info || s->max_iters < 1) return SPOCK_EINVAL;
  Problem& P = ph->p;
  if (P.general) return SPOCK_EUNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const auto t0 = std::chrono::steady_clock::now();
  spock_info loc{};
  loc.V_nested = std::numeric_limits<double>::quiet_NaN();
  {  // the sweep mapping and pass forms, as for a solve (once per problem)
    const int rt = (P.precision == SPOCK_FP64) ? autotune<double>(P, st) : autotune<float>(P, st);
    if (rt) return rt;
  }
  loc.mapping = P.team;
  const int rc = (P.precision == SPOCK_FP64)
                     ? backward_impl<double>(P, static_cast<const double*>(v_star), x0, gV, gu0, grad_x0,
                                             grad_q, grad_qN, *s, loc, st)
                     : backward_impl<float>(P, static_cast<const float*>(v_star), x0, gV, gu0, grad_x0,
                                            grad_q, grad_qN, *s, loc, st);
  if (rc) return rc;
  loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *info = loc;
  return SPOCK_OK;
}
