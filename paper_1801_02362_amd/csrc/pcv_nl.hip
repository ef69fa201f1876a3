// Neighbour list (Section 2; with the close structure, Section 3.2): choose
// the M references nearest to the current structure from a full pass's
// distances, and gather their stored data into a compact landmark set that
// the engines stream on the steps between list updates.
#include "pcv_internal.h"

namespace pcv {

namespace {

constexpr int kSelectMax = 8192;   // references one selection workgroup sorts in LDS

// Sort key of a distance: non-negative doubles order like their bit
// patterns; -0 counts as 0; NaN goes after every number.
__device__ __forceinline__ unsigned long long dist_key(double d) {
  if (!(d >= 0.0)) return 0x7FF8000000000000ull;
  if (d == 0.0) return 0ull;
  return (unsigned long long)__double_as_longlong(d);
}

// One workgroup: bitonic sort of (key, index) pairs in LDS, nearest first,
// ties to the lower index; the first M indices become the list.
__global__ __launch_bounds__(1024) void nl_select_kernel(const double* __restrict__ D, int N, int P, int M,
                                                         int* __restrict__ members) {
  __shared__ unsigned long long key[kSelectMax];
  __shared__ int idx[kSelectMax];
  for (int i = threadIdx.x; i < P; i += 1024) {
    key[i] = (i < N) ? dist_key(D[i]) : ~0ull;
    idx[i] = i;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += 1024) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const unsigned long long ki = key[i], kl = key[l];
          const int ii = idx[i], il = idx[l];
          const bool gt = ki > kl || (ki == kl && ii > il);
          if (gt == up) {
            key[i] = kl;
            key[l] = ki;
            idx[i] = il;
            idx[l] = ii;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < M; i += 1024) members[i] = idx[i];
}

// One workgroup per list member: its landmark coordinates, centroid, G_a,
// property and saved rotation.
template <typename T>
__global__ __launch_bounds__(256) void nl_gather_kernel(NlGather g, const int* __restrict__ flag, int run_if) {
  if (flag != nullptr && *flag != run_if) return;
  const int k = blockIdx.x;
  const int i = g.members[k];
  const size_t row = (size_t)3 * g.n_pad;
  const T* src = (const T*)g.A + (size_t)i * row;
  T* dst = (T*)g.A_nl + (size_t)k * row;
  for (size_t e = threadIdx.x; e < row; e += 256) dst[e] = src[e];
  const int t = threadIdx.x;
  if (t < 3) g.ca_nl[3 * k + t] = g.ca[3 * (size_t)i + t];
  if (t == 3) g.Ga_nl[k] = g.Ga[i];
  if (t == 4) g.q_nl[k] = g.q[i];
  if (t >= 16 && t < 25) g.Rsave_nl[9 * k + (t - 16)] = g.Rsave[9 * (size_t)i + (t - 16)];
}

}  // namespace

int nl_select_max() { return kSelectMax; }

hipError_t launch_nl_select(const double* D, int N, int M, int* members, hipStream_t st) {
  if (N < 1 || N > kSelectMax || M < 1 || M > N) return hipErrorInvalidValue;
  int P = 1;
  while (P < N) P <<= 1;
  hipLaunchKernelGGL(nl_select_kernel, dim3(1), dim3(1024), 0, st, D, N, P, M, members);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_nl_gather(const NlGather& g, const int* flag, int run_if, hipStream_t st) {
  if (g.M < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((nl_gather_kernel<T>), dim3(g.M), dim3(256), 0, st, g, flag, run_if);
  return hipGetLastError();
}

template hipError_t launch_nl_gather<float>(const NlGather&, const int*, int, hipStream_t);
template hipError_t launch_nl_gather<double>(const NlGather&, const int*, int, hipStream_t);

}  // namespace pcv
