// Property maps with several properties per reference (Eq. 2 with a vector
// q_i): after the exact pass has written every D_i and R_i, one workgroup
// forms the shared weights and every component S_k, and a second pass over
// the landmark coordinates accumulates all P gradients at once,
//   dS_k/dx_j = w_j sum_i W_ik r_ij,   W_ik = 2 lambda p_i (q_ik - S_k),
// with r_ij = R_i (a_ij - c_i) (the x part drops out because
// sum_i p_i (q_ik - S_k) = 0).  The gradient pass is FP64 throughout: the
// weights sum to zero, so the sum cancels and FP32 would lose digits.
#include <algorithm>

#include "pcv_internal.h"

namespace pcv {

namespace {

constexpr int kLseThreads = 256;

// Fixed-order workgroup sums of NV values (result in every thread).
template <int NV>
__device__ void wg_sum(double v[NV], double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = v[k];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) sh[wave * NV + k] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = 0.0;
    for (int w = 0; w < kLseThreads / 64; ++w) t += sh[w * NV + k];
    v[k] = t;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kLseThreads) void props_lse_kernel(const double* __restrict__ D, int L, int P,
                                                                const double* __restrict__ q, double lam,
                                                                double* __restrict__ S, double* __restrict__ W) {
  __shared__ double sh[(kLseThreads / 64) * (kPropsMax + 1)];
  __shared__ double Sk[kPropsMax];
  double m = INFINITY;
  for (int i = threadIdx.x; i < L; i += kLseThreads) m = fmin(m, D[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  m = INFINITY;
  for (int w = 0; w < kLseThreads / 64; ++w) m = fmin(m, sh[w]);
  __syncthreads();
  double v[kPropsMax + 1];
#pragma unroll
  for (int k = 0; k <= kPropsMax; ++k) v[k] = 0.0;
  for (int i = threadIdx.x; i < L; i += kLseThreads) {
    const double e = exp(-lam * (D[i] - m));
    v[kPropsMax] += e;
#pragma unroll
    for (int k = 0; k < kPropsMax; ++k)
      if (k < P) v[k] += e * q[(size_t)i * P + k];
  }
  wg_sum<kPropsMax + 1>(v, sh);
  const double Z = v[kPropsMax];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kPropsMax; ++k)
      if (k < P) {
        Sk[k] = v[k] / Z;
        S[k] = v[k] / Z;
      }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < L; i += kLseThreads) {
    const double f = 2.0 * lam * exp(-lam * (D[i] - m)) / Z;
    for (int k = 0; k < P; ++k) W[(size_t)i * P + k] = f * (q[(size_t)i * P + k] - Sk[k]);
  }
}

// Workgroup = 64 atoms x 4 waves; wave g takes landmarks i0 + g, i0 + g + 4, ...
// of its chunk; the four wave sums are added in order through LDS.
template <typename T>
__global__ __launch_bounds__(256) void props_grad_kernel(PropsArgs a, const double* __restrict__ W,
                                                         double* __restrict__ part) {
  __shared__ double red[3][kPropsMax * 3][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const int chunk = blockIdx.y;
  const int per = (a.L + gridDim.y - 1) / gridDim.y;
  const int i0 = chunk * per, i1 = min(a.L, i0 + per);
  const bool in = j < a.n_pad;
  const T* A = (const T*)a.A;
  double acc[kPropsMax][3];
  for (int k = 0; k < kPropsMax; ++k) acc[k][0] = acc[k][1] = acc[k][2] = 0.0;
  for (int i = i0 + g; i < i1; i += 4) {
    const T* ai = A + (size_t)i * 3 * a.n_pad;
    const double c0 = a.ca[3 * (size_t)i], c1 = a.ca[3 * (size_t)i + 1], c2 = a.ca[3 * (size_t)i + 2];
    const double* R = a.R + (size_t)i * 9;
    const double b0 = (in ? (double)ai[j] : c0) - c0;
    const double b1 = (in ? (double)ai[a.n_pad + j] : c1) - c1;
    const double b2 = (in ? (double)ai[2 * a.n_pad + j] : c2) - c2;
    const double r0 = R[0] * b0 + R[1] * b1 + R[2] * b2;
    const double r1 = R[3] * b0 + R[4] * b1 + R[5] * b2;
    const double r2 = R[6] * b0 + R[7] * b1 + R[8] * b2;
    const double* Wi = W + (size_t)i * a.P;
#pragma unroll
    for (int k = 0; k < kPropsMax; ++k) {
      if (k < a.P) {
        const double wk = Wi[k];
        acc[k][0] = fma(wk, r0, acc[k][0]);
        acc[k][1] = fma(wk, r1, acc[k][1]);
        acc[k][2] = fma(wk, r2, acc[k][2]);
      }
    }
  }
  if (g > 0) {
#pragma unroll
    for (int k = 0; k < kPropsMax; ++k)
#pragma unroll
      for (int d = 0; d < 3; ++d) red[g - 1][k * 3 + d][lane] = acc[k][d];
  }
  __syncthreads();
  if (g == 0 && in) {
#pragma unroll
    for (int k = 0; k < kPropsMax; ++k) {
      if (k < a.P) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double s =
              ((acc[k][d] + red[0][k * 3 + d][lane]) + red[1][k * 3 + d][lane]) + red[2][k * 3 + d][lane];
          part[(((size_t)chunk * a.P + k) * 3 + d) * a.n_pad + j] = s;
        }
      }
    }
  }
}

// dS_k/dx_j = w_j * (chunk partials added in chunk order); grid (3 n / 256
// rounded up, P), one component per row.  The loads are issued eight at a
// time (independent of the running sum), so a thread waits for one round
// trip per eight chunks rather than per chunk.  With x_rounded every
// workgroup also leaves its share of dS_k/dx . (x - x') in corr (x - x' =
// (w x_c - fl32(w x_c)) / w, so the share is the chunk sum times that
// residual); props_correct_kernel adds them to S_k.
template <typename T>
__global__ __launch_bounds__(256) void props_reduce_kernel(PropsArgs a, int chunks, const double* __restrict__ part,
                                                           T* __restrict__ dS) {
  __shared__ double sh[4];
  const int k = blockIdx.y;
  const int n3 = 3 * a.n;
  const int r = blockIdx.x * 256 + threadIdx.x;
  double term = 0.0;
  if (r < n3) {
    const int j = r / 3, d = r - 3 * j;
    const size_t stride = (size_t)a.P * 3 * a.n_pad;
    const double* p = part + ((size_t)k * 3 + d) * a.n_pad + j;
    double s = 0.0;
    int c = 0;
    for (; c + 8 <= chunks; c += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = p[(size_t)(c + u) * stride];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < chunks; ++c) s += p[(size_t)c * stride];
    if (dS) dS[(size_t)k * n3 + r] = (T)(a.w[j] * s);
    if (a.x_rounded) {
      const double xw = a.xw[(size_t)d * a.n_pad + j];
      term = s * (xw - (double)(float)xw);
    }
  }
  if (!a.x_rounded) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) term += __shfl_xor(term, off, 64);
  if (lane == 0) sh[wave] = term;
  __syncthreads();
  if (threadIdx.x == 0) a.corr[(size_t)k * gridDim.x + blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// S_k += its nb rounding shares, in block order (wave k of the workgroup).
__global__ __launch_bounds__(64 * kPropsMax) void props_correct_kernel(const double* __restrict__ corr, int nb, int P,
                                                                       double* __restrict__ S) {
  const int k = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (k >= P) return;
  double v = 0.0;
  for (int b = lane; b < nb; b += 64) v += corr[(size_t)k * nb + b];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) S[k] += v;
}

}  // namespace

int props_corr_doubles(int n) { return (3 * n + 255) / 256; }

int props_chunks(int n_pad, int L) {
  const int tiles = (n_pad + 63) / 64;
  int c = std::max(1, 1024 / tiles);
  c = std::min(c, std::max(1, L / 16));
  return std::min(c, 64);
}

template <typename T>
hipError_t launch_props(const PropsArgs& a, const double* q, double lam, double* S, double* W, double* part,
                        void* dS, hipStream_t st) {
  if (a.P < 1 || a.P > kPropsMax || a.L < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(props_lse_kernel, dim3(1), dim3(kLseThreads), 0, st, a.D, a.L, a.P, q, lam, S, W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || (dS == nullptr && !a.x_rounded)) return e;
  const int chunks = props_chunks(a.n_pad, a.L);
  hipLaunchKernelGGL((props_grad_kernel<T>), dim3((a.n_pad + 63) / 64, chunks), dim3(256), 0, st, a, W, part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nb = props_corr_doubles(a.n);
  hipLaunchKernelGGL((props_reduce_kernel<T>), dim3(nb, a.P), dim3(256), 0, st, a, chunks, part, (T*)dS);
  e = hipGetLastError();
  if (e != hipSuccess || !a.x_rounded) return e;
  hipLaunchKernelGGL(props_correct_kernel, dim3(1), dim3(64 * kPropsMax), 0, st, a.corr, nb, a.P, S);
  return hipGetLastError();
}

template hipError_t launch_props<float>(const PropsArgs&, const double*, double, double*, double*, double*, void*,
                                        hipStream_t);
template hipError_t launch_props<double>(const PropsArgs&, const double*, double, double*, double*, double*, void*,
                                         hipStream_t);

}  // namespace pcv
