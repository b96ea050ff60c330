// Batched block engine: one 256-thread workgroup per instance runs the whole
// SPOCK iteration (Alg. 3 with Anderson directions, section 6) on its own
// tree without returning to the host. The CP operator T (section 3) is
// evaluated with the same per-family team steps as the per-stage kernels,
// separated by workgroup barriers instead of launches: pre-pass, backward
// sweep stage N-1..0, forward sweep stage 0..N-1, post-pass with residual
// statistics. Trees of different shapes and sizes share one launch.
#include "device_common.h"

#include <algorithm>

namespace spk {

constexpr int kBT = 256;     // threads per instance
constexpr int kBMem = 4;     // Anderson memory supported
constexpr int kBPool = 10 + 2 * kBMem;

// ---- block-wide reductions (fixed order) -----------------------------------
__device__ __forceinline__ void blk_sum(double (&v)[8], int k, double* red /*[8][kBT]*/) {
  for (int j = 0; j < k; ++j) red[j * kBT + threadIdx.x] = v[j];
  __syncthreads();
  for (int s = kBT / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int j = 0; j < k; ++j) red[j * kBT + threadIdx.x] += red[j * kBT + threadIdx.x + s];
    __syncthreads();
  }
  for (int j = 0; j < k; ++j) v[j] = red[j * kBT];
  __syncthreads();
}

__device__ __forceinline__ void blk_stats(const StatAcc& st, double* red, double (&out)[5]) {
  red[0 * kBT + threadIdx.x] = st.rz2;
  red[1 * kBT + threadIdx.x] = st.re2;
  red[2 * kBT + threadIdx.x] = st.cross;
  red[3 * kBT + threadIdx.x] = st.xip;
  red[4 * kBT + threadIdx.x] = st.xid;
  __syncthreads();
  for (int s = kBT / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0 * kBT + threadIdx.x] += red[0 * kBT + threadIdx.x + s];
      red[1 * kBT + threadIdx.x] += red[1 * kBT + threadIdx.x + s];
      red[2 * kBT + threadIdx.x] += red[2 * kBT + threadIdx.x + s];
      red[3 * kBT + threadIdx.x] = fmax(red[3 * kBT + threadIdx.x], red[3 * kBT + threadIdx.x + s]);
      red[4 * kBT + threadIdx.x] = fmax(red[4 * kBT + threadIdx.x], red[4 * kBT + threadIdx.x + s]);
    }
    __syncthreads();
  }
  for (int j = 0; j < 5; ++j) out[j] = red[j * kBT];
  __syncthreads();
}

struct BStats {
  double xip = 0, xid = 0, om2 = 0;
  __device__ double xi() const { return fmax(xip, xid); }
  __device__ double omega() const { return sqrt(fmax(om2, 0.0)); }
  __device__ bool ok() const { return isfinite(xip) && isfinite(xid) && isfinite(om2); }
};

// ---- small FP64 linear algebra on one lane ---------------------------------
__device__ bool dev_cholesky(int n, double* A) {
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0) || !isfinite(d)) return false;
    d = sqrt(d);
    A[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / d;
    }
  }
  return true;
}

// extreme eigenvalues of a symmetric n x n (n <= 4) matrix, cyclic Jacobi
__device__ void dev_eig_extremes(int n, const double* G, double& lmin, double& lmax) {
  double A[16];
  for (int e = 0; e < n * n; ++e) A[e] = G[e];
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double th = 0.5 * (A[q * n + q] - A[p * n + p]) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  lmin = lmax = A[0];
  for (int i = 1; i < n; ++i) {
    lmin = fmin(lmin, A[i * n + i]);
    lmax = fmax(lmax, A[i * n + i]);
  }
}

// ---- the per-instance solver -------------------------------------------------
// T lanes per family with T >= max(nx, nu): every lane owns one component,
// so the per-lane vectors of the family steps have a single entry (D = T).
template <typename S, int T>
struct BlockSolver {
  const BatchInst<S>& I;
  const DevProb<S>& P;
  const BatchSettings& s;
  S* lds_team;    // team regions, 3 VM each
  double* red;    // [8][kBT]
  int VM, lane, team, nteams;
  S* q;
  S* d;
  S* xbar;
  S* ubar;
  int t_evals = 0;

  __device__ BlockSolver(const BatchInst<S>& inst, const BatchSettings& st, S* lds, double* r, int vm)
      : I(inst), P(inst.P), s(st), lds_team(lds), red(r), VM(vm) {
    lane = threadIdx.x % T;
    team = threadIdx.x / T;
    nteams = kBT / T;
    const long long nv = I.nv;
    S* base = I.work + (size_t)kBPool * nv;
    q = base;
    d = q + (size_t)P.nn * P.nx;
    xbar = d + (size_t)P.nn * P.nu;
    ubar = xbar + (size_t)P.nn * P.nx;
  }
  __device__ S* pool(int k) const { return I.work + (size_t)k * I.nv; }

  // Tv = T(v) and the residual statistics of v - T(v) (one out-of-line copy:
  // Alg. 3 calls it from several places)
  __device__ __noinline__ BStats Teval(const S* v, S* Tv) {
    const S* z = v;
    const S* eta = v + P.nz;
    S* zout = Tv;
    S* eout = Tv + P.nz;
    S* mylds = lds_team + (size_t)team * 3 * VM;
    for (int f = team; f < P.nl; f += nteams) fam_pre_team<S, T, T>(P, z, eta, zout, xbar, ubar, q, f, lane);
    __syncthreads();
    for (int t = P.N - 1; t >= 0; --t) {
      const int a = I.stage_off[t], b = I.stage_off[t + 1];
      for (int i = a + team; i < b; i += nteams) fam_bwd_team<S, T, T>(P, xbar, ubar, q, d, i, lane, mylds, VM);
      __syncthreads();
    }
    for (int t = 0; t < P.N; ++t) {
      const int a = I.stage_off[t], b = I.stage_off[t + 1];
      for (int i = a + team; i < b; i += nteams) fam_fwd_team<S, T, T>(P, zout, d, I.x0, i, lane, mylds, VM);
      __syncthreads();
    }
    StatAcc st;
    for (int f = team; f < P.nl; f += nteams) fam_post_team<S, T, T>(P, z, eta, zout, eout, f, lane, mylds, VM, st);
    __syncthreads();
    double o[5];
    blk_stats(st, red, o);
    ++t_evals;
    BStats r;
    r.xip = o[3];
    r.xid = o[4];
    r.om2 = o[0] + o[1] - 2.0 * (double)P.alpha * o[2];
    return r;
  }

  __device__ __noinline__ void lincomb(S* out, double a, const S* x, double b, const S* y) {
    for (long long e = threadIdx.x; e < I.nv; e += kBT) {
      double v = a * (double)x[e];
      if (y) v += b * (double)y[e];
      out[e] = (S)v;
    }
    __syncthreads();
  }
  __device__ __noinline__ void lincomb3(S* out, double a, const S* x, double b, const S* y, double c,
                                        const S* w) {
    for (long long e = threadIdx.x; e < I.nv; e += kBT)
      out[e] = (S)(a * (double)x[e] + b * (double)y[e] + c * (double)w[e]);
    __syncthreads();
  }
  __device__ __noinline__ double rdot(const S* v, const S* Tv, const S* w) {
    double acc[8] = {0};
    for (long long e = threadIdx.x; e < I.nv; e += kBT)
      acc[0] += ((double)v[e] - (double)Tv[e]) * (double)w[e];
    blk_sum(acc, 1, red);
    return acc[0];
  }
  // M d = (d_z - alpha L* d_eta, d_eta - alpha L d_z), node-local per family
  __device__ __noinline__ void apply_M(const S* dv, S* Md) {
    const Off<S> O(P);
    const S al = P.alpha;
    const S* dz = dv;
    const S* de = dv + P.nz;
    S* mz = Md;
    S* me = Md + P.nz;
    const int nx = P.nx, nu = P.nu;
    for (int i = threadIdx.x; i < P.nl; i += kBT) {
      const int fc = P.fc[i], n = P.nch[i];
      const long long zb = O.z2(i), e1 = O.e1(i);
      // rows of group 1: eta-part minus alpha L(d_z)
      S by = dz[zb + 2 * n];
      for (int k = 0; k < n; ++k) by += P.p[fc + k] * dz[zb + k];
      for (int k = 0; k < 2 * n + 1; ++k) me[e1 + k] = de[e1 + k] - al * dz[zb + k];
      me[e1 + 2 * n + 1] = de[e1 + 2 * n + 1] - al * (dz[O.s(i)] - by);
      for (int o = 0; o < nx; ++o) me[O.e1x(i) + o] = de[O.e1x(i) + o] - al * dz[O.x(i) + o];
      for (int o = 0; o < nu; ++o) me[O.e1u(i) + o] = de[O.e1u(i) + o] - al * dz[O.u(i) + o];
      // columns of family i: z-part minus alpha L*(d_eta)
      const S es = de[O.e1s(i)];
      for (int k = 0; k < 2 * n + 1; ++k) {
        const S bk = (k < n) ? P.p[fc + k] : ((k == 2 * n) ? S(1) : S(0));
        mz[zb + k] = dz[zb + k] - al * (de[e1 + k] - bk * es);
      }
      mz[O.s(i)] = dz[O.s(i)] - al * es;
      for (int o = 0; o < nx; ++o) {
        S acc = de[O.e1x(i) + o];
        for (int k = 0; k < n; ++k) acc += P.sq[(size_t)(fc + k) * nx + o] * de[O.e2(fc + k) + o];
        mz[O.x(i) + o] = dz[O.x(i) + o] - al * acc;
      }
      for (int o = 0; o < nu; ++o) {
        S acc = de[O.e1u(i) + o];
        for (int k = 0; k < n; ++k) acc += P.sr[(size_t)(fc + k) * nu + o] * de[O.e2(fc + k) + nx + o];
        mz[O.u(i) + o] = dz[O.u(i) + o] - al * acc;
      }
      for (int k = 0; k < n; ++k) {
        const int c = fc + k;
        const long long e2 = O.e2(c);
        for (int o = 0; o < nx; ++o) me[e2 + o] = de[e2 + o] - al * P.sq[(size_t)c * nx + o] * dz[O.x(i) + o];
        for (int o = 0; o < nu; ++o)
          me[e2 + nx + o] = de[e2 + nx + o] - al * P.sr[(size_t)c * nu + o] * dz[O.u(i) + o];
        const S th = S(0.5) * dz[O.tau(c)];
        me[e2 + nx + nu] = de[e2 + nx + nu] - al * th;
        me[e2 + nx + nu + 1] = de[e2 + nx + nu + 1] - al * th;
        mz[O.tau(c)] = dz[O.tau(c)] - al * S(0.5) * (de[e2 + nx + nu] + de[e2 + nx + nu + 1]);
        if (c >= P.nl) {
          const long long e3 = O.e3(c);
          for (int o = 0; o < nx; ++o) {
            me[e3 + o] = de[e3 + o] - al * dz[O.x(c) + o];
            me[e3 + nx + o] = de[e3 + nx + o] - al * P.sqN[(size_t)c * nx + o] * dz[O.x(c) + o];
            mz[O.x(c) + o] = dz[O.x(c) + o] - al * (de[e3 + o] + P.sqN[(size_t)c * nx + o] * de[e3 + nx + o]);
          }
          const S sh = S(0.5) * dz[O.s(c)];
          me[e3 + 2 * nx] = de[e3 + 2 * nx] - al * sh;
          me[e3 + 2 * nx + 1] = de[e3 + 2 * nx + 1] - al * sh;
          mz[O.s(c)] = dz[O.s(c)] - al * S(0.5) * (de[e3 + 2 * nx] + de[e3 + 2 * nx + 1]);
        }
      }
    }
    __syncthreads();
  }

  __device__ void run(double* out) {
    __shared__ double Gs[kBMem * kBMem], rhs[kBMem], gam[kBMem];
    __shared__ int kept_sh;
    int order[kBMem] = {0, 0, 0, 0};  // active Anderson slots, oldest first (same in every thread)
    const long long nv = I.nv;
    const double al = (double)P.alpha;
    S* v = pool(0);
    S* Tv = pool(1);
    S* vprev = pool(2);
    S* rprev = pool(3);
    S* rcur = pool(4);
    S* dir = pool(5);
    S* Md = pool(6);
    S* vt = pool(7);
    S* Tvt = pool(8);
    S* spare = pool(9);
    // Anderson columns j: dV(j) = pool(10 + j), dR(j) = pool(10 + kBMem + j)
    // x0 must lie in the root's state box
    bool box_ok = true;
    for (int o = 0; o < P.nx; ++o) box_ok = box_ok && I.x0[o] >= (double)P.xlo[o] && I.x0[o] <= (double)P.xhi[o];
    int status = 0, k = 0, n_k0 = 0, n_k1 = 0, n_k2 = 0, n_km = 0, n_bt = 0;
    double xi0 = 0, xi = 0;
    if (!box_ok) {
      status = 3;
    } else {
      for (long long e = threadIdx.x; e < nv; e += kBT) v[e] = I.vio[e];
      __syncthreads();
      BStats S0 = Teval(v, Tv), Sc = S0, St;
      xi0 = S0.xi();
      const double tol = fmax(s.eps_abs, s.eps_rel * xi0);
      double zeta = S0.omega(), omega_safe = S0.omega();
      int nord = 0;  // active Anderson columns, oldest first in order[]
      bool have_prev = false;
      status = -1;
      if (!S0.ok()) status = 2;
      while (status < 0) {
        if (Sc.xi() <= tol) { status = 0; break; }
        if (k >= s.max_iters) { status = 1; break; }
        if (s.method == SPOCK_METHOD_CP) {
          S* tmp = v; v = Tv; Tv = tmp;
          Sc = Teval(v, Tv);
          ++k;
          if (!Sc.ok()) status = 2;
          continue;
        }
        // ---- residual r = v - T(v) and the Anderson buffers
        if (have_prev) {
          int slot = 0;
          if (nord == s.m) {
            slot = order[0];
            for (int j = 1; j < nord; ++j) order[j - 1] = order[j];
            --nord;
          } else {
            for (int c = s.m - 1; c >= 0; --c) {  // a slot not in use
              bool used = false;
              for (int j = 0; j < nord; ++j) used = used || order[j] == c;
              if (!used) slot = c;
            }
          }
          // <dR_j, dR_new> (j < nord), <dR_new, dR_new>, <dR_j, r>, <dR_new, r>;
          // fixed-trip loops keep the accumulators in registers
          double aG[kBMem] = {0, 0, 0, 0}, aR[kBMem] = {0, 0, 0, 0}, aNN = 0, aNR = 0;
          const S* oldc[kBMem];
#pragma unroll
          for (int j = 0; j < kBMem; ++j) oldc[j] = pool(10 + kBMem + order[j < nord ? j : 0]);
          for (long long e = threadIdx.x; e < nv; e += kBT) {
            const S vv = v[e];
            const S r = vv - Tv[e];
            rcur[e] = r;
            const S dr = r - rprev[e];
            pool(10 + slot)[e] = vv - vprev[e];
            pool(10 + kBMem + slot)[e] = dr;
#pragma unroll
            for (int j = 0; j < kBMem; ++j) {
              if (j < nord) {
                const double ob = (double)oldc[j][e];
                aG[j] += ob * (double)dr;
                aR[j] += ob * (double)r;
              }
            }
            aNN += (double)dr * (double)dr;
            aNR += (double)dr * (double)r;
          }
          double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
          for (int j = 0; j < nord; ++j) {
            acc[j] = aG[j];
            acc[nord + 1 + j] = aR[j];
          }
          acc[nord] = aNN;
          acc[2 * nord + 1] = aNR;
          blk_sum(acc, 2 * nord + 2, red);
          if (threadIdx.x == 0) {
            for (int j = 0; j < nord; ++j) {
              Gs[order[j] * kBMem + slot] = acc[j];
              Gs[slot * kBMem + order[j]] = acc[j];
              rhs[order[j]] = acc[nord + 1 + j];
            }
            Gs[slot * kBMem + slot] = acc[nord];
            rhs[slot] = acc[2 * nord + 1];
          }
          order[nord] = slot;
          ++nord;
          __syncthreads();
        } else {
          lincomb(rcur, 1.0, v, -1.0, Tv);
        }
        // ---- Gram solve with the rank rule (thread 0): drop the oldest column
        // while lambda_min/lambda_max(G) < 1e-12; gam[] follows order[drop..]
        if (threadIdx.x == 0) {
          int first = 0;
          while (first < nord) {
            const int kk = nord - first;
            double Gsub[kBMem * kBMem];
            for (int a = 0; a < kk; ++a)
              for (int b = 0; b < kk; ++b) Gsub[a * kk + b] = Gs[order[first + a] * kBMem + order[first + b]];
            double lmin, lmax;
            dev_eig_extremes(kk, Gsub, lmin, lmax);
            if (lmax > 0.0 && lmin / lmax >= 1e-12 && dev_cholesky(kk, Gsub)) {
              double y[kBMem];
              for (int i = 0; i < kk; ++i) {
                double sm = rhs[order[first + i]];
                for (int j = 0; j < i; ++j) sm -= Gsub[i * kk + j] * y[j];
                y[i] = sm / Gsub[i * kk + i];
              }
              for (int i = kk - 1; i >= 0; --i) {
                double sm = y[i];
                for (int j = i + 1; j < kk; ++j) sm -= Gsub[j * kk + i] * gam[j];
                gam[i] = sm / Gsub[i * kk + i];
              }
              break;
            }
            ++first;
          }
          kept_sh = nord - first;
        }
        __syncthreads();
        {
          const int drop = nord - kept_sh;
          for (int j = 0; j + drop < nord; ++j) order[j] = order[j + drop];
          nord = kept_sh;
        }
        for (long long e = threadIdx.x; e < nv; e += kBT) {
          double acc = -(double)rcur[e];
          for (int j = 0; j < nord; ++j)
            acc -= gam[j] * ((double)pool(10 + order[j])[e] - (double)pool(10 + kBMem + order[j])[e]);
          dir[e] = (S)acc;
        }
        __syncthreads();
        const double omega = Sc.omega();
        if (omega <= s.c0 * zeta) {  // K0
          lincomb(spare, 1.0, v, 1.0, dir);
          S* t1 = vprev; vprev = v; v = spare; spare = t1;
          S* t2 = rprev; rprev = rcur; rcur = t2;
          have_prev = true;
          zeta = omega;
          ++n_k0;
          Sc = Teval(v, Tv);
          ++k;
          if (!Sc.ok()) status = 2;
          continue;
        }
        apply_M(dir, Md);
        double tau = 1.0;
        bool accepted = false;
        for (int ls = 0; ls < s.max_ls; ++ls) {
          lincomb(vt, 1.0, v, tau, dir);
          St = Teval(vt, Tvt);
          if (!St.ok()) { tau *= s.beta; ++n_bt; continue; }
          const double om_t = St.omega();
          if (om_t == 0.0 || (omega <= omega_safe && om_t <= s.c1 * omega)) {  // K1
            S* t1 = vprev; vprev = v; v = vt; vt = t1;
            S* t2 = rprev; rprev = rcur; rcur = t2;
            S* t3 = Tv; Tv = Tvt; Tvt = t3;
            have_prev = true;
            Sc = St;
            omega_safe = om_t + pow(s.c2, (double)k);
            ++n_k1;
            accepted = true;
            break;
          }
          const double rho = om_t * om_t - tau * rdot(vt, Tvt, Md);
          if (rho >= s.sigma * om_t * omega) {  // K2
            const double c = s.lambda * rho / (om_t * om_t);
            lincomb3(spare, 1.0, v, -c, vt, c, Tvt);
            S* t1 = vprev; vprev = v; v = spare; spare = t1;
            S* t2 = rprev; rprev = rcur; rcur = t2;
            have_prev = true;
            ++n_k2;
            Sc = Teval(v, Tv);
            accepted = true;
            break;
          }
          tau *= s.beta;
          ++n_bt;
        }
        if (!accepted) {  // plain KM step
          lincomb(spare, 1.0, v, -s.lambda, rcur);
          S* t1 = vprev; vprev = v; v = spare; spare = t1;
          S* t2 = rprev; rprev = rcur; rcur = t2;
          have_prev = true;
          ++n_km;
          Sc = Teval(v, Tv);
        }
        ++k;
        if (!Sc.ok()) status = 2;
      }
      xi = Sc.xi();
      if (s.write_out)
        for (long long e = threadIdx.x; e < nv; e += kBT) I.vio[e] = Tv[e];
      __syncthreads();
      if (threadIdx.x == 0) out[8] = (double)Tv[0];
    }
    if (threadIdx.x == 0) {
      out[0] = status;
      out[1] = k;
      out[2] = t_evals;
      out[3] = n_k0;
      out[4] = n_k1;
      out[5] = n_k2;
      out[6] = n_km;
      out[7] = n_bt;
      out[9] = xi0;
      out[10] = xi;
    }
  }
};

template <typename S, int T>
__global__ void __launch_bounds__(kBT) k_solve_batched(const BatchInst<S>* __restrict__ insts, int B,
                                                       BatchSettings s, int VM, double* __restrict__ infos) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[8 * kBT];
  S* lds = reinterpret_cast<S*>(smem_raw);
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    BlockSolver<S, T> solver(insts[b], s, lds, red, VM);
    solver.run(infos + (size_t)b * 16);
    __syncthreads();
  }
}

template <typename S>
hipError_t launch_solve_batched(const BatchInst<S>* insts_dev, int B, const BatchSettings& s, int team,
                                int VM, double* infos_dev, int grid, hipStream_t st) {
  const size_t lds = (size_t)(kBT / team) * 3 * VM * sizeof(S);
  switch (team) {
    case 8: hipLaunchKernelGGL((k_solve_batched<S, 8>), dim3(grid), dim3(kBT), lds, st, insts_dev, B, s, VM, infos_dev); break;
    case 16: hipLaunchKernelGGL((k_solve_batched<S, 16>), dim3(grid), dim3(kBT), lds, st, insts_dev, B, s, VM, infos_dev); break;
    case 32: hipLaunchKernelGGL((k_solve_batched<S, 32>), dim3(grid), dim3(kBT), lds, st, insts_dev, B, s, VM, infos_dev); break;
    default: hipLaunchKernelGGL((k_solve_batched<S, 64>), dim3(grid), dim3(kBT), lds, st, insts_dev, B, s, VM, infos_dev); break;
  }
  return hipGetLastError();
}
template hipError_t launch_solve_batched<double>(const BatchInst<double>*, int, const BatchSettings&, int,
                                                 int, double*, int, hipStream_t);
template hipError_t launch_solve_batched<float>(const BatchInst<float>*, int, const BatchSettings&, int,
                                                int, double*, int, hipStream_t);

size_t batched_pool_vectors() { return kBPool; }

}  // namespace spk
