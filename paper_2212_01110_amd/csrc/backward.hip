// Kernels of the implicit differentiation at the fixed point v* = T(v*):
// the Jacobian of prox_{alpha g*} at the pre-prox point b* (section 5.4:
// G(b) = b - alpha proj_S3(b / alpha), so J_G = I - J_proj(b* / alpha)),
// the transpose of the root-state map of the S1 projection (Alg. 2 with zero
// data: u = K x, x^c = Abar^c x), and the cost-weight gradients.
#include "device_common.h"

namespace spk {

// J_G d on a translated SOC block by one wavefront: vector part of len <=
// 128 entries (lane o holds entries o and o + 64), then the two trailing
// scalars a (entry len) and b (entry len + 1); b_ is the block of b*.
template <typename S>
__device__ void soc_jg_wave(const S* __restrict__ b_, const S* __restrict__ din, S* __restrict__ dout, int len,
                            S al, int lane) {
  const S ia = S(1) / al;
  S bv[2], dv[2];
  double r2p = 0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int o = lane + 64 * s;
    const int oo = o < len ? o : 0;
    bv[s] = o < len ? b_[oo] : S(0);
    dv[s] = o < len ? din[oo] : S(0);
    r2p += (double)(bv[s] * ia) * (double)(bv[s] * ia);
  }
  const S va = b_[len] * ia - S(0.5);
  const S t = b_[len + 1] * ia + S(0.5);
  const double r2 = team_sum<64>(r2p) + (double)va * (double)va;
  const S r = (S)sqrt(r2);
  const S da = din[len], dt = din[len + 1];
  if (r <= t) {  // inside the cone: proj Jacobian = I, J_G = 0
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (lane + 64 * s < len) dout[lane + 64 * s] = S(0);
    if (lane == 0) {
      dout[len] = S(0);
      dout[len + 1] = S(0);
    }
    return;
  }
  if (r <= -t) {  // polar cone: proj Jacobian = 0, J_G = I
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (lane + 64 * s < len) dout[lane + 64 * s] = dv[s];
    if (lane == 0) {
      dout[len] = da;
      dout[len + 1] = dt;
    }
    return;
  }
  // J_proj (x, t) -> 1/2 [ (1 + t/r) dx - (t/r) xh (xh.dx) + xh dt ; xh.dx + dt ],
  // xh = x / r, x = (b_vec / alpha, b_a / alpha - 1/2)
  const S ir = S(1) / r;
  double xdp = 0;
#pragma unroll
  for (int s = 0; s < 2; ++s) xdp += (double)(bv[s] * ia * ir) * (double)dv[s];
  const double xd = team_sum<64>(xdp) + (double)(va * ir) * (double)da;
  const S tr = t * ir;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (lane + 64 * s < len) {
      const S xh = bv[s] * ia * ir;
      const S jp = S(0.5) * ((S(1) + tr) * dv[s] - tr * xh * (S)xd + xh * dt);
      dout[lane + 64 * s] = dv[s] - jp;
    }
  }
  if (lane == 0) {
    const S xh = va * ir;
    const S jp = S(0.5) * ((S(1) + tr) * da - tr * xh * (S)xd + xh * dt);
    dout[len] = da - jp;
    dout[len + 1] = dt - S(0.5) * ((S)xd + dt);
  }
}

// out = J_G(b*) w on every block of S3: one wavefront per family (group 1
// of i, group 2 of each child, group 3 of leaf children), grid-stride.
template <typename S>
__global__ void __launch_bounds__(256) k_jg(DevProb<S> P, const S* __restrict__ b, const S* __restrict__ w,
                                            S* __restrict__ out, long long is) {
  b += (size_t)blockIdx.y * is;  // instance blockIdx.y of a batch (stride is)
  w += (size_t)blockIdx.y * is;
  out += (size_t)blockIdx.y * is;
  const int lane = threadIdx.x & 63;
  const Off<S> O(P);
  const int nx = P.nx, nu = P.nu;
  const S al = P.alpha, ia = S(1) / al;
  for (int i = blockIdx.x * 4 + (int)(threadIdx.x >> 6); i < P.nl; i += gridDim.x * 4) {
    const int fc = P.fc[i], n = P.nch[i];
    const long long e1 = O.e1(i);
    for (int k = lane; k < 2 * n; k += 64) out[e1 + k] = (b[e1 + k] <= S(0)) ? w[e1 + k] : S(0);  // K*: max(.,0)
    if (lane == 0) {
      out[e1 + 2 * n] = S(0);                                                       // free entry
      out[e1 + 2 * n + 1] = (b[e1 + 2 * n + 1] <= S(0)) ? w[e1 + 2 * n + 1] : S(0);  // R_+
    }
    for (int o = lane; o < nx; o += 64) {
      const long long e = O.e1x(i) + o;
      const S v = b[e] * ia;
      const bool in = v > P.xlo[(size_t)i * nx + o] && v < P.xhi[(size_t)i * nx + o];
      out[e] = in ? S(0) : w[e];
    }
    for (int o = lane; o < nu; o += 64) {
      const long long e = O.e1u(i) + o;
      const S v = b[e] * ia;
      const bool in = v > P.ulo[(size_t)i * nu + o] && v < P.uhi[(size_t)i * nu + o];
      out[e] = in ? S(0) : w[e];
    }
    for (int c = fc; c < fc + n; ++c) {
      const long long e2 = O.e2(c);
      soc_jg_wave<S>(b + e2, w + e2, out + e2, nx + nu, al, lane);
      if (c >= P.nl) {
        const long long e3 = O.e3(c);
        for (int o = lane; o < nx; o += 64) {
          const S v = b[e3 + o] * ia;
          const bool in = v > P.xlo[(size_t)c * nx + o] && v < P.xhi[(size_t)c * nx + o];
          out[e3 + o] = in ? S(0) : w[e3 + o];
        }
        soc_jg_wave<S>(b + e3 + nx, w + e3 + nx, out + e3 + nx, nx, al, lane);
      }
    }
  }
}

// Transpose of the root-state map Phi of the S1 projection, one stage per
// launch (stage N-1 .. 0): mu^j = c_x^j at leaves, mu^i = c_x^i + K^i' c_u^i +
// sum_c Abar^c' mu^c; mu^0 is the gradient with respect to x0.
template <typename S>
__global__ void k_phiT(DevProb<S> P, const S* __restrict__ cz, S* __restrict__ mu, int first, int count) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= count) return;
  const int i = first + f;
  const Off<S> O(P);
  const int nx = P.nx, nu = P.nu, fc = P.fc[i], n = P.nch[i];
  for (int k = 0; k < nx; ++k) {
    double acc = (double)cz[O.x(i) + k];
    for (int j = 0; j < nu; ++j) acc += (double)P.KR[(size_t)i * nu * nx + (size_t)j * nx + k] * (double)cz[O.u(i) + j];
    for (int cc = 0; cc < n; ++cc) {
      const int c = fc + cc;
      const S* Ab = P.AbR + (size_t)c * nx * nx;  // row-major Abar: (Abar' mu)_k = sum_r Abar[r][k] mu_r
      const bool leaf = c >= P.nl;
      for (int r = 0; r < nx; ++r) {
        const double m = leaf ? (double)cz[O.x(c) + r] : (double)mu[(size_t)c * nx + r];
        acc += (double)Ab[(size_t)r * nx + k] * m;
      }
    }
    mu[(size_t)i * nx + k] = (S)acc;
  }
}

// Cost-weight gradients from the adjoint quantities: for a non-root c with
// ancestor i, d/dq^c_k = alpha (x*_{i,k} lb_{c,k} - la_{x^i,k} eta*_{c,k}) / (2 sqrt(q^c_k))
// on the group-2 x rows; for a leaf j, the same with group 3 and Q_N.
template <typename S>
__global__ void k_grad_q(DevProb<S> P, const S* __restrict__ vstar, const S* __restrict__ la,
                         const S* __restrict__ lb, double* __restrict__ gq, double* __restrict__ gqN) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.nn || c == 0) return;
  const Off<S> O(P);
  const int nx = P.nx;
  const int i = P.anc[c];
  const S* z = vstar;
  const S* eta = vstar + P.nz;
  const double al = (double)P.alpha;
  if (gq) {
    const long long e2 = O.e2(c);
    for (int k = 0; k < nx; ++k) {
      const double sq = (double)P.sq[(size_t)c * nx + k];
      const double d = al * ((double)z[O.x(i) + k] * (double)lb[e2 + k] - (double)la[O.x(i) + k] * (double)eta[e2 + k]);
      gq[(size_t)c * nx + k] = d / (2.0 * sq);
    }
  }
  if (gqN && c >= P.nl) {
    const long long e3q = O.e3(c) + nx;
    for (int k = 0; k < nx; ++k) {
      const double sq = (double)P.sqN[(size_t)c * nx + k];
      const double d = al * ((double)z[O.x(c) + k] * (double)lb[e3q + k] - (double)la[O.x(c) + k] * (double)eta[e3q + k]);
      gqN[(size_t)c * nx + k] = sq > 0.0 ? d / (2.0 * sq) : 0.0;
    }
  }
}

// max |a - b| over n entries, per block, then over blocks (one launch each)
template <typename S>
__global__ void k_maxdiff(long long n, const S* __restrict__ a, const S* __restrict__ b,
                          double* __restrict__ partials) {
  __shared__ double red[256];
  double m = 0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    m = fmax(m, fabs((double)a[e] - (double)b[e]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}
__global__ void k_max_final(const double* __restrict__ partials, int nblk, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double m = 0;
  for (int b = 0; b < nblk; ++b) m = fmax(m, partials[b]);
  out[0] = m;
}

__global__ void k_copy_elem_d(double* dst, const double* src) { dst[0] = src[0]; }
template <typename S>
__global__ void k_copy_elem(S* dst, const S* src) { dst[0] = src[0]; }

// ---- launchers
template <typename S>
hipError_t launch_copy_elem(S* dst, const S* src, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_elem<S>, dim3(1), dim3(1), 0, st, dst, src);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_jg(const Problem& P, const S* b, const S* w, S* out, hipStream_t st) {
  const DevProb<S>& D = (sizeof(S) == 8) ? *reinterpret_cast<const DevProb<S>*>(&P.dp64)
                                         : *reinterpret_cast<const DevProb<S>*>(&P.dp32);
  hipLaunchKernelGGL(k_jg<S>, dim3(family_wave_blocks(P.tree->nl)), dim3(256), 0, st, D, b, w, out, 0LL);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_jg_batch(const Problem& P, const S* b, const S* w, S* out, long long is, int B, hipStream_t st) {
  const DevProb<S>& D = (sizeof(S) == 8) ? *reinterpret_cast<const DevProb<S>*>(&P.dp64)
                                         : *reinterpret_cast<const DevProb<S>*>(&P.dp32);
  hipLaunchKernelGGL(k_jg<S>, dim3(family_wave_blocks(P.tree->nl), B), dim3(256), 0, st, D, b, w, out, is);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_phiT(const Problem& P, const S* cz, S* mu, hipStream_t st) {
  const DevProb<S>& D = (sizeof(S) == 8) ? *reinterpret_cast<const DevProb<S>*>(&P.dp64)
                                         : *reinterpret_cast<const DevProb<S>*>(&P.dp32);
  const Tree& T = *P.tree;
  for (int t = T.N - 1; t >= 0; --t) {
    const int first = T.stage_off[t], count = T.stage_off[t + 1] - first;
    hipLaunchKernelGGL(k_phiT<S>, dim3((count + 127) / 128), dim3(128), 0, st, D, cz, mu, first, count);
  }
  return hipGetLastError();
}
template <typename S>
hipError_t launch_grad_q(const Problem& P, const S* vstar, const S* la, const S* lb, double* gq, double* gqN,
                         hipStream_t st) {
  const DevProb<S>& D = (sizeof(S) == 8) ? *reinterpret_cast<const DevProb<S>*>(&P.dp64)
                                         : *reinterpret_cast<const DevProb<S>*>(&P.dp32);
  hipLaunchKernelGGL(k_grad_q<S>, dim3((P.tree->nn + 127) / 128), dim3(128), 0, st, D, vstar, la, lb, gq, gqN);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_maxdiff(long long n, const S* a, const S* b, double* partials, double* out, hipStream_t st) {
  const int nb = dots_blocks(n);
  hipLaunchKernelGGL(k_maxdiff<S>, dim3(nb), dim3(256), 0, st, n, a, b, partials);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(64), 0, st, partials, nb, out);
  return hipGetLastError();
}

#define SPK_BINST(S)                                                                                  \
  template hipError_t launch_copy_elem<S>(S*, const S*, hipStream_t);                                 \
  template hipError_t launch_jg<S>(const Problem&, const S*, const S*, S*, hipStream_t);              \
  template hipError_t launch_jg_batch<S>(const Problem&, const S*, const S*, S*, long long, int, hipStream_t); \
  template hipError_t launch_phiT<S>(const Problem&, const S*, S*, hipStream_t);                      \
  template hipError_t launch_grad_q<S>(const Problem&, const S*, const S*, const S*, double*, double*, \
                                       hipStream_t);                                                  \
  template hipError_t launch_maxdiff<S>(long long, const S*, const S*, double*, double*, hipStream_t);
SPK_BINST(double)
SPK_BINST(float)

}  // namespace spk
