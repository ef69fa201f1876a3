// Separate displacement and alignment weights (w != w', Eq. 4 with all its
// terms).  The alignment (centring and rotation) uses w', the distance and
// its derivative use w, so the rotation is no longer stationary for D and
// Eq. 4 keeps its centre-of-mass and rotation terms:
//   dD_i/dx_k = 2 w_k d_ik - 2 w'_k sum_j w_j d_ij + w'_k Gamma_i^T a_c,ik,
// d_ik = x_c,k - R_i a_c,ik, Gamma_i = d(G_i : R_i)/dM_i the rotation adjoint
// of G_i = dD_i/dR = -2 sum_j w_j d_ij a_c,ij^T (Section 3 machinery).
//
// Three passes:
//   1. one wave per landmark: M = sum_j w'_j a_c x_c^T and
//      N = sum_j w_j a_c x_c^T (FP64), the quaternion eigenproblem of M,
//      D = G_x^w + G_a^w - 2 tr(R N), G = -2 (N^T - R C_aa) with the
//      landmark's C_aa = sum_j w_j a_c a_c^T, Gamma = adjoint(G), and
//      R mu_a (mu_a = sum_j w_j a_c);
//   2. one workgroup: log-sum-exp weights c_i = -lambda p_i (q_i - s), p_i,
//      s, z and the per-landmark sums of R mu_a;
//   3. the landmark coordinates again, FP64: per atom
//      sum_i c_i R_i a_c, sum_i c_i Gamma_i^T a_c and the same with p_i.
#include <algorithm>

#include "pcv_internal.h"
#include "pcv_math.h"

namespace pcv {

namespace {

__device__ __forceinline__ double wsum64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per landmark: G_a^w, mu_a (3), C_aa (6: xx xy xz yy yz zz), with a_c
// centred by the alignment weights (ca).
template <typename T>
__global__ __launch_bounds__(256) void f2_stats_kernel(F2Args a) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= a.L) return;
  const T* A = (const T*)a.A + (size_t)i * 3 * a.n_pad;
  const double c0 = a.ca[3 * (size_t)i], c1 = a.ca[3 * (size_t)i + 1], c2 = a.ca[3 * (size_t)i + 2];
  double v[10] = {0.0};
  for (int j = lane; j < a.n; j += 64) {
    const double w = a.wd[j];
    const double x = (double)A[j] - c0, y = (double)A[a.n_pad + j] - c1, z = (double)A[2 * a.n_pad + j] - c2;
    v[0] += w * (x * x + y * y + z * z);
    v[1] += w * x;
    v[2] += w * y;
    v[3] += w * z;
    v[4] += w * x * x;
    v[5] += w * x * y;
    v[6] += w * x * z;
    v[7] += w * y * y;
    v[8] += w * y * z;
    v[9] += w * z * z;
  }
#pragma unroll
  for (int k = 0; k < 10; ++k) v[k] = wsum64(v[k]);
  if (lane == 0) {
    a.Gaw[i] = v[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) a.mua[3 * (size_t)i + d] = v[1 + d];
#pragma unroll
    for (int k = 0; k < 6; ++k) a.Caa[6 * (size_t)i + k] = v[4 + k];
  }
}

// The frame: x centred by w' (FP64 planes), G_x^{w'}, G_x^w, mu_x = sum w x_c.
template <typename T>
__global__ __launch_bounds__(256) void f2_frame_kernel(F2Args a, const T* __restrict__ x) {
  __shared__ double sh[4 * 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double v[3] = {0.0, 0.0, 0.0};
  for (int j = tid; j < a.n; j += 256) {
    const double wp = a.wa[j];
#pragma unroll
    for (int d = 0; d < 3; ++d) v[d] += wp * (double)x[3 * (size_t)j + d];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double s = wsum64(v[d]);
    if (lane == 0) sh[wave * 8 + d] = s;
  }
  __syncthreads();
  double c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) c[d] = ((sh[d] + sh[8 + d]) + sh[16 + d]) + sh[24 + d];
  __syncthreads();
  double u[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // Gx', Gxw, mu_x (3), finite flag
  for (int j = tid; j < a.n_pad; j += 256) {
    double xc[3] = {0.0, 0.0, 0.0};
    if (j < a.n) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double xv = (double)x[3 * (size_t)j + d];
        if (!isfinite(xv)) u[5] = 1.0;
        xc[d] = xv - c[d];
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) a.xc[(size_t)d * a.n_pad + j] = xc[d];
    const double r2 = xc[0] * xc[0] + xc[1] * xc[1] + xc[2] * xc[2];
    const double wp = j < a.n ? a.wa[j] : 0.0, w = j < a.n ? a.wd[j] : 0.0;
    u[0] += wp * r2;
    u[1] += w * r2;
#pragma unroll
    for (int d = 0; d < 3; ++d) u[2 + d] += w * xc[d];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double s = wsum64(u[k]);
    if (lane == 0) sh[wave * 8 + k] = s;
  }
  __syncthreads();
  if (tid < 6) {
    const double s = ((sh[tid] + sh[8 + tid]) + sh[16 + tid]) + sh[24 + tid];
    if (tid < 5) a.fs[tid] = s;
    else if (s != 0.0 && a.status) *a.status = 1;
  }
}

// Pass 1: one wave per landmark.
template <typename T>
__global__ __launch_bounds__(256) void f2_pass1_kernel(F2Args a, double* __restrict__ dout) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= a.L) return;
  const T* A = (const T*)a.A + (size_t)i * 3 * a.n_pad;
  const double c0 = a.ca[3 * (size_t)i], c1 = a.ca[3 * (size_t)i + 1], c2 = a.ca[3 * (size_t)i + 2];
  double v[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) v[k] = 0.0;
  for (int j = lane; j < a.n; j += 64) {
    const double ac[3] = {(double)A[j] - c0, (double)A[a.n_pad + j] - c1, (double)A[2 * a.n_pad + j] - c2};
    const double xc[3] = {a.xc[j], a.xc[a.n_pad + j], a.xc[2 * (size_t)a.n_pad + j]};
    const double wp = a.wa[j], w = a.wd[j];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const double p = ac[r] * xc[cc];
        v[r * 3 + cc] = fma(wp, p, v[r * 3 + cc]);
        v[9 + r * 3 + cc] = fma(w, p, v[9 + r * 3 + cc]);
      }
  }
#pragma unroll
  for (int k = 0; k < 18; ++k) v[k] = wsum64(v[k]);
  if (lane != 0) return;
  const double Gxp = a.fs[0], Gxw = a.fs[1];
  double M[9], N[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    M[k] = v[k];
    N[k] = v[9 + k];
  }
  double F[10], lam, q[4], R[9];
  const int fb = top_eigenpair(M, 0.5 * (Gxp + a.Ga[i]), F, lam, q);
  if (fb && a.fallbacks) atomicAdd((unsigned long long*)a.fallbacks, 1ull);
  quat_to_rot(q, R);
  // D = G_x^w + G_a^w - 2 sum_j w_j x_c . (R a_c) = ... - 2 sum_ab R_ab N_ba
  double tr = 0.0;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) tr = fma(R[r * 3 + cc], N[cc * 3 + r], tr);
  double D = Gxw + a.Gaw[i] - 2.0 * tr;
  D = D < 0.0 ? 0.0 : D;
  // G = -2 (N^T - R C_aa)
  const double* cp = a.Caa + 6 * (size_t)i;
  const double C[9] = {cp[0], cp[1], cp[2], cp[1], cp[3], cp[4], cp[2], cp[4], cp[5]};
  double G[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const double RC = R[r * 3 + 0] * C[0 * 3 + cc] + R[r * 3 + 1] * C[1 * 3 + cc] + R[r * 3 + 2] * C[2 * 3 + cc];
      G[r * 3 + cc] = -2.0 * (N[cc * 3 + r] - RC);
    }
  double Gam[9];
  rotation_adjoint(F, lam, q, G, Gam);
  dout[i] = D;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    a.Rl[9 * (size_t)i + k] = R[k];
    a.Gl[9 * (size_t)i + k] = Gam[k];
  }
  const double* mu = a.mua + 3 * (size_t)i;
#pragma unroll
  for (int r = 0; r < 3; ++r)
    a.Rmu[3 * (size_t)i + r] = R[r * 3 + 0] * mu[0] + R[r * 3 + 1] * mu[1] + R[r * 3 + 2] * mu[2];
}

// Pass 2: s, z, the weights c_i and p_i, and K_c = sum c_i R_i mu_a,i,
// K_p = sum p_i R_i mu_a,i (fs[5..10]).  One workgroup of 256.
__global__ __launch_bounds__(256) void f2_lse_kernel(F2Args a, const double* __restrict__ D, double* __restrict__ sz,
                                                     long long* __restrict__ counters) {
  __shared__ double sh[4 * 8];
  __shared__ double tot[8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double m = INFINITY;
  for (int i = tid; i < a.L; i += 256) m = fmin(m, D[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off, 64));
  if (lane == 0) sh[wave] = m;
  __syncthreads();
  m = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
  __syncthreads();
  double v[2] = {0.0, 0.0};
  for (int i = tid; i < a.L; i += 256) {
    const double e = exp(-a.lam * (D[i] - m));
    v[0] += e;
    v[1] += e * a.q[i];
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double s = wsum64(v[k]);
    if (lane == 0) sh[wave * 8 + k] = s;
  }
  __syncthreads();
  if (tid < 2) tot[tid] = ((sh[tid] + sh[8 + tid]) + sh[16 + tid]) + sh[24 + tid];
  __syncthreads();
  const double Z = tot[0], s = tot[1] / Z;
  double k6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = tid; i < a.L; i += 256) {
    const double p = exp(-a.lam * (D[i] - m)) / Z;
    const double c = -a.lam * p * (a.q[i] - s);
    a.cw[i] = c;
    a.pw[i] = p;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      k6[d] += c * a.Rmu[3 * (size_t)i + d];
      k6[3 + d] += p * a.Rmu[3 * (size_t)i + d];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double t = wsum64(k6[k]);
    if (lane == 0) sh[wave * 8 + k] = t;
  }
  __syncthreads();
  if (tid < 6) a.fs[5 + tid] = ((sh[tid] + sh[8 + tid]) + sh[16 + tid]) + sh[24 + tid];
  if (tid == 0) {
    sz[0] = s;
    sz[1] = m - log(Z) / a.lam;
    if (counters) {
      counters[CNT_EVALS] += 1;
      counters[CNT_EXPENSIVE] += a.L;
    }
  }
}

// Pass 3: per atom, 12 sums over a chunk of landmarks (64 atoms x 4 waves).
template <typename T>
__global__ __launch_bounds__(256) void f2_grad_kernel(F2Args a, double* __restrict__ part) {
  __shared__ double red[3][12][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const int chunk = blockIdx.y;
  const int per = (a.L + gridDim.y - 1) / gridDim.y;
  const int i0 = chunk * per, i1 = min(a.L, i0 + per);
  const bool in = j < a.n_pad;
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  for (int i = i0 + g; i < i1; i += 4) {
    const T* Ai = (const T*)a.A + (size_t)i * 3 * a.n_pad;
    const double* ci = a.ca + 3 * (size_t)i;
    const double b0 = (in ? (double)Ai[j] : ci[0]) - ci[0];
    const double b1 = (in ? (double)Ai[a.n_pad + j] : ci[1]) - ci[1];
    const double b2 = (in ? (double)Ai[2 * a.n_pad + j] : ci[2]) - ci[2];
    const double* R = a.Rl + 9 * (size_t)i;
    const double* Gm = a.Gl + 9 * (size_t)i;
    const double r[3] = {R[0] * b0 + R[1] * b1 + R[2] * b2, R[3] * b0 + R[4] * b1 + R[5] * b2,
                         R[6] * b0 + R[7] * b1 + R[8] * b2};
    const double t[3] = {Gm[0] * b0 + Gm[3] * b1 + Gm[6] * b2, Gm[1] * b0 + Gm[4] * b1 + Gm[7] * b2,
                         Gm[2] * b0 + Gm[5] * b1 + Gm[8] * b2};   // Gamma^T a_c
    const double c = a.cw[i], p = a.pw[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      acc[d] = fma(c, r[d], acc[d]);
      acc[3 + d] = fma(c, t[d], acc[3 + d]);
      acc[6 + d] = fma(p, r[d], acc[6 + d]);
      acc[9 + d] = fma(p, t[d], acc[9 + d]);
    }
  }
  if (g > 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) red[g - 1][k][lane] = acc[k];
  }
  __syncthreads();
  if (g == 0 && in) {
#pragma unroll
    for (int k = 0; k < 12; ++k)
      part[((size_t)chunk * 12 + k) * a.n_pad + j] = ((acc[k] + red[0][k][lane]) + red[1][k][lane]) + red[2][k][lane];
  }
}

// The chunk partials summed per atom (64 atoms x 4 waves; wave g takes
// chunks g, g + 4, ..., the four wave sums added in order through LDS), then
// ds_k = -2 w_k S_Rc + w'_k S_Gc + 2 w'_k K_c
// dz_k = 2 w_k (x_c,k - S_Rp) + w'_k S_Gp - 2 w'_k (mu_x - K_p)
template <typename T>
__global__ __launch_bounds__(256) void f2_out_kernel(F2Args a, int chunks, const double* __restrict__ part,
                                                     T* __restrict__ ds, T* __restrict__ dz) {
  __shared__ double red[3][12][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const bool in = j < a.n;
  double s[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) s[k] = 0.0;
  if (in) {
    for (int c = g; c < chunks; c += 4) {
      double v[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) v[k] = part[((size_t)c * 12 + k) * a.n_pad + j];
#pragma unroll
      for (int k = 0; k < 12; ++k) s[k] += v[k];
    }
  }
  if (g > 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) red[g - 1][k][lane] = s[k];
  }
  __syncthreads();
  if (g != 0 || !in) return;
#pragma unroll
  for (int k = 0; k < 12; ++k) s[k] = ((s[k] + red[0][k][lane]) + red[1][k][lane]) + red[2][k][lane];
  const double w = a.wd[j], wp = a.wa[j];
  // s[0..2] S_Rc, s[3..5] S_Gc, s[6..8] S_Rp, s[9..11] S_Gp
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (ds) ds[3 * (size_t)j + d] = (T)(-2.0 * w * s[d] + wp * s[3 + d] + 2.0 * wp * a.fs[5 + d]);
    if (dz)
      dz[3 * (size_t)j + d] = (T)(2.0 * w * (a.xc[(size_t)d * a.n_pad + j] - s[6 + d]) + wp * s[9 + d] -
                                  2.0 * wp * (a.fs[2 + d] - a.fs[8 + d]));
  }
}

}  // namespace

int f2_chunks(int n_pad, int L) {
  const int tiles = (n_pad + 63) / 64;
  int c = std::max(1, 1024 / tiles);
  c = std::min(c, std::max(1, L / 16));
  return std::min(c, 64);
}

template <typename T>
hipError_t launch_f2_stats(const F2Args& a, hipStream_t st) {
  hipLaunchKernelGGL((f2_stats_kernel<T>), dim3((a.L + 3) / 4), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_f2_eval(const F2Args& a, const void* x, double* sz, void* ds, void* dz, double* dout,
                          long long* counters, hipStream_t st) {
  hipLaunchKernelGGL((f2_frame_kernel<T>), dim3(1), dim3(256), 0, st, a, (const T*)x);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((f2_pass1_kernel<T>), dim3((a.L + 3) / 4), dim3(256), 0, st, a, dout);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(f2_lse_kernel, dim3(1), dim3(256), 0, st, a, (const double*)dout, sz, counters);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (!ds && !dz) return hipSuccess;
  const int chunks = f2_chunks(a.n_pad, a.L);
  hipLaunchKernelGGL((f2_grad_kernel<T>), dim3((a.n_pad + 63) / 64, chunks), dim3(256), 0, st, a, a.part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((f2_out_kernel<T>), dim3((a.n + 63) / 64), dim3(256), 0, st, a, chunks,
                     (const double*)a.part, (T*)ds, (T*)dz);
  return hipGetLastError();
}

template hipError_t launch_f2_stats<float>(const F2Args&, hipStream_t);
template hipError_t launch_f2_stats<double>(const F2Args&, hipStream_t);
template hipError_t launch_f2_eval<float>(const F2Args&, const void*, double*, void*, void*, double*, long long*,
                                          hipStream_t);
template hipError_t launch_f2_eval<double>(const F2Args&, const void*, double*, void*, void*, double*, long long*,
                                           hipStream_t);

}  // namespace pcv
