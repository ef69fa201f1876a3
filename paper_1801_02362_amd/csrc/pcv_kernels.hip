// HIP kernels for path collective variables with a floating close structure
// (arXiv:1801.02362), written for gfx950 (CDNA4, wave64).
//
// Data flow of one evaluation:
//   prep        centre x with the weights (FP64), Gx, and for Algorithm 2 the
//               exact superposition of the close structure y onto x, the
//               reassignment decision D(x, y) > epsilon and the y <- x update.
//   engine      stream every landmark once: FP64 correlation (Eq. 3 via the
//               top quaternion eigenvalue), or the composed rotation of
//               Eq. 5; fold exp(-lambda D_i) weights into per-atom
//               accumulators of residuals with a running minimum (online
//               log-sum-exp), so that the derivatives (Eq. 4 / Eq. 6) need no
//               second read of the landmarks.
//   merge       combine the per-item partials into s, z (Eq. 2) and the atom
//               gradients; the close-structure merge also applies the
//               derivative of R_xy.
#include "pcv_internal.h"
#include "pcv_math.h"
#include "pcv_stream.h"

namespace pcv {

template <typename T> struct AccT { using type = float; };
template <> struct AccT<double> { using type = double; };

// ----------------------------------------------------------------- reductions
template <int NV>
__device__ __forceinline__ void wave_sum(double v[NV], int width) {
  for (int off = width >> 1; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], off, 64);
  }
}

// Sum NV doubles over the whole block; every thread receives the result.
// sh must hold (BS/64)*NV doubles.
template <int NV, int BS>
__device__ void block_sum(double v[NV], double* sh) {
  wave_sum<NV>(v, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[wave * NV + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < BS / 64; ++w) s += sh[w * NV + k];
    v[k] = s;
  }
}

// block_sum for the frame preparation's latency-bound reductions: each
// wave folds its values nine at a time with lane swaps (wave_sum9_store,
// a few VALU operations per value instead of six cross-lane shuffles),
// then every thread adds the waves' sums in wave order.  sh must hold
// (BS/64) * 9 * ceil(NV/9) doubles.
template <int NV, int BS>
__device__ void block_sum_swap(double v[NV], double* sh) {
  constexpr int NC = (NV + 8) / 9;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();   // the previous user of sh is done
#pragma unroll
  for (int ch = 0; ch < NC; ++ch) {
    double w9[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) w9[k] = (ch * 9 + k < NV) ? v[ch * 9 + k] : 0.0;
    wave_sum9_store(w9, sh + (wave * NC + ch) * 9, lane);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < BS / 64; ++w) s += sh[(w * NC + k / 9) * 9 + k % 9];
    v[k] = s;
  }
}

template <int BS>
__device__ double block_min(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double m = sh[0];
  for (int w = 1; w < BS / 64; ++w) m = fmin(m, sh[w]);
  return m;
}

// Sum NV doubles over a team of ts lanes (ts a power of two, 16..WG).  Teams
// of up to 64 lanes reduce inside the wave; wider teams finish through LDS
// (red holds (WG/64)*NV doubles).  Must be reached by the whole workgroup
// when ts > 64.
template <int NV>
__device__ __forceinline__ void team_sum(double v[NV], int ts, double* red) {
  wave_sum<NV>(v, ts < 64 ? ts : 64);
  if (ts > 64) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
    }
    __syncthreads();
    const int wpt = ts >> 6;
    const int w0 = (wave / wpt) * wpt;
    double s = 0.0;
    if (lane < NV)
      for (int w = 0; w < wpt; ++w) s += red[(w0 + w) * NV + lane];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = __shfl(s, k, 64);
  }
}

// max(v, 0) that keeps NaN (fmax would return 0 for a NaN distance).
__device__ __forceinline__ double clamp0(double v) { return v < 0.0 ? 0.0 : v; }

__device__ __forceinline__ double scale_to(double m_from, double m_to, double lam) {
  return (m_from == INFINITY) ? 0.0 : exp(-lam * (m_from - m_to));
}

// ------------------------------------------------------------ landmark load
// One workgroup per landmark: FP64 weighted centroid and Ga, and the AoS to
// SoA copy (values unchanged, atom axis zero padded to n_pad).
template <typename T>
__global__ __launch_bounds__(256) void load_kernel(const T* __restrict__ in, T* __restrict__ A,
                                                   double* __restrict__ ca, double* __restrict__ Ga,
                                                   const double* __restrict__ w, int n, int n_pad) {
  __shared__ double sh[4 * 3];
  const int i = blockIdx.x;
  const T* src = in + (size_t)i * n * 3;
  double c[3] = {0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < n; j += 256) {
    const double wj = w[j];
    c[0] = fma(wj, (double)src[3 * j + 0], c[0]);
    c[1] = fma(wj, (double)src[3 * j + 1], c[1]);
    c[2] = fma(wj, (double)src[3 * j + 2], c[2]);
  }
  block_sum<3, 256>(c, sh);
  double g[1] = {0.0};
  T* dst = A + (size_t)i * 3 * n_pad;
  for (int j = threadIdx.x; j < n_pad; j += 256) {
    if (j < n) {
      const double wj = w[j];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T v = src[3 * j + d];
        const double dv = (double)v - c[d];
        g[0] = fma(wj * dv, dv, g[0]);
        dst[(size_t)d * n_pad + j] = v;
      }
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) dst[(size_t)d * n_pad + j] = T(0);
    }
  }
  block_sum<1, 256>(g, sh);
  if (threadIdx.x == 0) {
    ca[3 * i + 0] = c[0];
    ca[3 * i + 1] = c[1];
    ca[3 * i + 2] = c[2];
    Ga[i] = g[0];
  }
}

// Exact distance between consecutive landmarks (for the sharpness lambda).
template <typename T>
__global__ __launch_bounds__(256) void pair_msd_kernel(const T* __restrict__ A, const double* __restrict__ ca,
                                                       const double* __restrict__ Ga,
                                                       const double* __restrict__ w, int n, int n_pad,
                                                       double* __restrict__ out) {
  __shared__ double sh[4 * 9];
  const int i = blockIdx.x;
  const T* a = A + (size_t)i * 3 * n_pad;
  const T* x = A + (size_t)(i + 1) * 3 * n_pad;
  double M[9] = {0.0};
  for (int j = threadIdx.x; j < n; j += 256) {
    const double wj = w[j];
    double av[3], xv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      av[d] = (double)a[(size_t)d * n_pad + j] - ca[3 * i + d];
      xv[d] = wj * ((double)x[(size_t)d * n_pad + j] - ca[3 * (i + 1) + d]);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) M[r * 3 + c] = fma(av[r], xv[c], M[r * 3 + c]);
  }
  block_sum<9, 256>(M, sh);
  if (threadIdx.x == 0) {
    double F[10], lam, q[4];
    const double G = Ga[i] + Ga[i + 1];
    top_eigenpair(M, 0.5 * G, F, lam, q);
    out[i] = clamp0(G - 2.0 * lam);
  }
}

// ------------------------------------------------------------ frame prep
// CACHE: atoms per thread whose x and w (and y) the first pass keeps in
// registers for the second (one global round trip fewer); atoms past
// CACHE * BS are loaded again.  The sums are taken in the same order either way.  With y
// (a centred structure [3][n_pad], FP64) the second pass also forms the
// correlation My = sum_j y_j (w_j x_c,j)^T (row-major, 9 values).  sh holds
// (BS / 64) * 18 doubles (block_sum_swap of up to 14 values).
template <typename T, int BS, int CACHE = 0>
__device__ void centre_frame(const PrepArgs& a, const T* x, double* sh, double& Gx, bool& finite,
                             double c[3], double g32[4], const double* y = nullptr, double* My = nullptr) {
  constexpr int KC = CACHE > 0 ? CACHE : 1;
  T xk[KC][3];
  double wk[KC], yk[KC][3];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  auto acc1 = [&](double wj, const T* xv) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double xd = (double)xv[d];
      if (!isfinite(xd)) v[3] += 1.0;
      v[d] = fma(wj, xd, v[d]);
    }
  };
#pragma unroll
  for (int k = 0; k < CACHE; ++k) {
    const int j = threadIdx.x + k * BS;
    if (j < a.n) {
      wk[k] = a.w[j];
#pragma unroll
      for (int d = 0; d < 3; ++d) xk[k][d] = x[3 * j + d];
      if (y) {
#pragma unroll
        for (int d = 0; d < 3; ++d) yk[k][d] = y[(size_t)d * a.n_pad + j];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < CACHE; ++k)
    if (threadIdx.x + k * BS < a.n) acc1(wk[k], xk[k]);
  for (int j = threadIdx.x + CACHE * BS; j < a.n; j += BS) acc1(a.w[j], x + 3 * j);
  // Lane-swap sums pay off at 256 threads (300 atoms: 4.4 -> 4.0 us for
  // the exact prep); at 512 threads the shuffle tree was faster (9.2 against
  // 10.2 us at 5,000 atoms, same box), so the wide launch keeps it.
  if constexpr (BS == 256) block_sum_swap<4, BS>(v, sh);
  else block_sum<4, BS>(v, sh);
  finite = (v[3] == 0.0);
  c[0] = v[0]; c[1] = v[1]; c[2] = v[2];
  // g[0]: Gx; g[1]: sum (w x rounded to T)^2 / w; g[2..4]: sum of w x
  // rounded to T; g[5..13]: the correlation with y.
  double g[14] = {0.0};
  auto acc2 = [&](int j, double wj, const T* xv, const double* yc) {
    const double iw = wj > 0.0 ? 1.0 / wj : 0.0;
    double xwv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double xd = (double)xv[d] - c[d];
      xwv[d] = wj * xd;
      a.xw[(size_t)d * a.n_pad + j] = xwv[d];
      if (a.xw32) a.xw32[(size_t)d * a.n_x + j] = (float)xwv[d];
      g[0] = fma(wj * xd, xd, g[0]);
      const double r = (double)(T)xwv[d];
      g[1] = fma(r * r, iw, g[1]);
      g[2 + d] += r;
    }
    if (y) {
      const double yv[3] = {yc ? yc[0] : y[j], yc ? yc[1] : y[(size_t)a.n_pad + j],
                            yc ? yc[2] : y[2 * (size_t)a.n_pad + j]};
#pragma unroll
      for (int r0 = 0; r0 < 3; ++r0)
#pragma unroll
        for (int c0 = 0; c0 < 3; ++c0) g[5 + r0 * 3 + c0] = fma(yv[r0], xwv[c0], g[5 + r0 * 3 + c0]);
    }
  };
  auto pad = [&](int j) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      a.xw[(size_t)d * a.n_pad + j] = 0.0;
      if (a.xw32) a.xw32[(size_t)d * a.n_x + j] = 0.f;
    }
  };
#pragma unroll
  for (int k = 0; k < CACHE; ++k) {
    const int j = threadIdx.x + k * BS;
    if (j < a.n) acc2(j, wk[k], xk[k], y ? yk[k] : nullptr);
    else if (j < a.n_pad) pad(j);
  }
  for (int j = threadIdx.x + CACHE * BS; j < a.n_pad; j += BS) {
    if (j < a.n) acc2(j, a.w[j], x + 3 * j, nullptr);
    else pad(j);
  }
  if (y) {
    block_sum_swap<14, BS>(g, sh);
#pragma unroll
    for (int k = 0; k < 9; ++k) My[k] = g[5 + k];
  } else {
    if constexpr (BS == 256) block_sum_swap<5, BS>(g, sh);
    else block_sum<5, BS>(g, sh);
  }
  Gx = g[0];
  g32[0] = g[1] - (g[2] * g[2] + g[3] * g[3] + g[4] * g[4]);
  g32[1] = g[2];
  g32[2] = g[3];
  g32[3] = g[4];
}

// One workgroup per problem (the batched path and Algorithm 1); BS threads
// (256 when every structure has at most 1,024 atoms, else 512), each
// keeping up to 8,192 / BS of its atoms in registers between the passes.
template <typename T, int BS>
__global__ __launch_bounds__(BS) void prep_kernel(const PrepArgs* __restrict__ args,
                                                  const void* __restrict__ x_base) {
  __shared__ double sh[(BS / 64) * 9];
  const PrepArgs a = args[blockIdx.x];
  const T* x = (const T*)x_base + 3 * a.x_off;
  double Gx, c[3], g32[4];
  bool finite;
  centre_frame<T, BS, (BS >= 512 ? 16 : 4)>(a, x, sh, Gx, finite, c, g32);
  if (threadIdx.x == 0) {
    *a.Gx = Gx;
    *a.Gx32 = g32[0];
    a.xres[0] = g32[1];
    a.xres[1] = g32[2];
    a.xres[2] = g32[3];
    if (!finite) *a.status = 1;
    if (a.counters) {
      a.counters[CNT_EVALS] += 1;
      a.counters[CNT_EXPENSIVE] += a.L;
    }
  }
}

// Algorithm 2, first part: centre x, superpose the close structure y onto x
// exactly (D_xy, R_xy and the eigen-system kept for the derivative of R_xy),
// decide the reassignment (strict D_xy > epsilon; always on the first frame or
// when forced), move y <- x when reassigning, update the counters.
template <typename T>
// 256 threads: the serial eigen-solve of thread 0 keeps its arrays in
// registers (at 1024 threads the per-thread register budget forces them to
// scratch memory, one cache round trip per access).
__global__ __launch_bounds__(256) void prep_close_kernel(PrepArgs a, const T* __restrict__ x,
                                                         CloseArgs cs, Outs nan_outs) {
  constexpr int BS = 256;
  __shared__ double sh[16 * 14];
  __shared__ int s_flag;
  double Gx, c[3], g32[4];
  bool finite;
  // With a close structure, its correlation with x is formed in the same
  // pass that writes the centred x.
  const int init = __builtin_amdgcn_readfirstlane(*cs.init);
  // Thread 0's scalars (G_y, the forced flag, the counters) are fetched now,
  // so their latency hides behind the frame pass; no other kernel touches
  // them while this one runs.
  double gy0 = 0.0;
  int force0 = 0;
  long long cnt[4] = {0, 0, 0, 0};   // frames, recomputes, expensive, approx
  if (threadIdx.x == 0) {
    gy0 = *cs.Gy;
    force0 = *cs.force;
    cnt[0] = cs.counters[CNT_FRAMES];
    cnt[1] = cs.counters[CNT_RECOMPUTES];
    cnt[2] = cs.counters[CNT_EXPENSIVE];
    cnt[3] = cs.counters[CNT_APPROX];
  }
  double M[9];
  centre_frame<T, BS, 4>(a, x, sh, Gx, finite, c, g32, init ? cs.y64 : nullptr, M);
  double Dxy = NAN;
  if (init) {
    if (threadIdx.x == 0) {
      double F[10], lam, q[4], R[9];
      const double G = Gx + gy0;
      top_eigenpair(M, 0.5 * G, F, lam, q);
      Dxy = clamp0(G - 2.0 * lam);
      quat_to_rot(q, R);
      for (int k = 0; k < 10; ++k) cs.Fxy[k] = F[k];
      for (int k = 0; k < 4; ++k) cs.qxy[k] = q[k];
      for (int k = 0; k < 9; ++k) cs.Rxy[k] = R[k];
      *cs.lamxy = lam;
    }
  }
  if (threadIdx.x == 0) {
    int flag;
    if (!finite) flag = -1;
    else if (!init || force0 || Dxy > cs.eps) flag = 1;
    else flag = 0;
    *cs.Dxy = Dxy;
    *cs.flag = flag;
    *cs.force = 0;
    *a.Gx = Gx;
    *a.Gx32 = g32[0];
    a.xres[0] = g32[1];
    a.xres[1] = g32[2];
    a.xres[2] = g32[3];
    if (!finite) *a.status = 1;
    if (nan_outs.rec) *nan_outs.rec = flag;
    s_flag = flag;
    if (flag >= 0) {
      cs.counters[CNT_FRAMES] = cnt[0] + 1;
      long long expensive = cnt[2] + (init ? 1 : 0);
      if (flag == 1) {
        cs.counters[CNT_RECOMPUTES] = cnt[1] + 1;
        expensive += cs.L;
        *cs.Gy = Gx;
        *cs.init = 1;
      } else {
        cs.counters[CNT_APPROX] = cnt[3] + 1;
      }
      cs.counters[CNT_EXPENSIVE] = expensive;
    }
  }
  __syncthreads();
  const int flag = s_flag;
  if (flag == 1) {
    for (int j = threadIdx.x; j < a.n_pad; j += BS) {
#pragma unroll
      for (int d = 0; d < 3; ++d) cs.y64[(size_t)d * a.n_pad + j] = (j < a.n) ? (double)x[3 * j + d] - c[d] : 0.0;
    }
  } else if (flag == -1) {
    T* ds = (T*)nan_outs.ds;
    T* dz = (T*)nan_outs.dz;
    for (int j = threadIdx.x; j < 3 * a.n; j += BS) {
      if (ds) ds[j] = T(NAN);
      if (dz) dz[j] = T(NAN);
    }
    if (threadIdx.x == 0) {
      nan_outs.sz[0] = NAN;
      nan_outs.sz[1] = NAN;
    }
  }
}

// ------------------------------------------------------------------ engine
// Landmark streaming engine.  A workgroup of WG threads splits into teams of
// ts lanes (per problem); a team owns one landmark at a time and each lane
// owns atoms lane + ts*k (k < APT), so every landmark is read exactly once,
// coalesced, straight from HBM into registers (with the next landmark
// prefetched).  Per landmark:
//   * FP64 correlation M = sum_j a_j (w_j x_j)^T from the stored coordinates;
//     x is centred in FP64, so the landmark translation drops out without
//     re-rounding the landmark;
//   * EXACT: top eigenvalue of the quaternion matrix -> D = Gx + Ga - 2 lambda
//     and R (Eq. 3); APPROX: D~ = Gx + Ga - 2 tr((R_xy R_{a_i y}) M) (Eq. 5)
//     with R = R_{a_i y};
//   * online log-sum-exp: e_i = exp(-lambda (D_i - m)) against the running
//     minimum m, accumulators rescaled when m drops;
//   * per-atom FP64 accumulators of the rotated, centred landmark
//     r_i = R (a_i - c_i):  U = sum e_i (q_i - q0) r_i,  V = sum e_i r_i.
//     The residuals x - r_i of Eq. 4 / Eq. 6 are formed in the merge, where
//     the x part cancels exactly (sum_i p_i (q_i - s) = 0), so no FP32
//     rounding of a large residual enters the gradient.
// Each work item (a landmark range of one problem) ends with a tree merge of
// the teams through LDS and writes one partial (m, Z, S, q0, U, V).
template <typename T, int WG, int APT>
__global__ __launch_bounds__(WG) void engine_kernel(const Problem* __restrict__ probs,
                                                    const Item* __restrict__ items,
                                                    const int* __restrict__ wg_off, int mode,
                                                    const int* __restrict__ flag, int run_if,
                                                    double* __restrict__ dout) {
  using part_t = typename AccT<T>::type;
  {
    const Problem* pr = probs;
    if (!gate_launch(flag, run_if, mode, pr)) return;
    probs = pr;
  }
  extern __shared__ double smem[];
  double* red = smem;                       // (WG/64)*9
  double* mh = smem + (WG / 64) * 9;        // (WG/32)*3
  double* mv = mh + (WG / 32) * 3;          // (WG/2)*6
  const int tid = threadIdx.x;
  const int it_end = wg_off[blockIdx.x + 1];
  for (int it = wg_off[blockIdx.x]; it < it_end; ++it) {
    const Item item = items[it];
    const Problem& P = probs[item.prob];
    const int ts = P.ts;
    const int teams = WG / ts;
    const int team = tid / ts;
    const int lane = tid - team * ts;
    const int n_pad = P.n_pad;
    const T* __restrict__ A = (const T*)P.A;
    const double lam = P.lam;
    const double Gx = *P.Gx;

    double xw[3][APT];
#pragma unroll
    for (int k = 0; k < APT; ++k) {
      const int j = lane + ts * k;
      const bool in = j < n_pad;
#pragma unroll
      for (int d = 0; d < 3; ++d) xw[d][k] = in ? P.xw[(size_t)d * n_pad + j] : 0.0;
    }
    double U[3][APT], V[3][APT];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int k = 0; k < APT; ++k) { U[d][k] = 0.0; V[d][k] = 0.0; }
    double tU[3] = {0.0, 0.0, 0.0}, tV[3] = {0.0, 0.0, 0.0};   // sum e (q - q0) R c, sum e R c
    double m = INFINITY, Z = 0.0, S = 0.0;
    const double q0 = P.q[item.i0];

    T ac[3][APT], an[3][APT];
    auto load = [&](T (&dst)[3][APT], int i) {
      const T* src = A + (size_t)i * 3 * n_pad;
#pragma unroll
      for (int k = 0; k < APT; ++k) {
        const int j = lane + ts * k;
        const bool in = j < n_pad;
#pragma unroll
        for (int d = 0; d < 3; ++d) dst[d][k] = in ? src[(size_t)d * n_pad + j] : T(0);
      }
    };
    const int len = item.i1 - item.i0;
    const int iters = (len + teams - 1) / teams;
    int i = item.i0 + team;
    if (i < item.i1) load(ac, i);
    else {
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int k = 0; k < APT; ++k) ac[d][k] = T(0);
    }
    for (int r = 0; r < iters; ++r, i += teams) {
      const bool active = i < item.i1;
      if (i + teams < item.i1) load(an, i + teams);
      // FP64 correlation partial over this lane's atoms.
      double M[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) M[k] = 0.0;
#pragma unroll
      for (int k = 0; k < APT; ++k) {
        const double a0 = (double)ac[0][k], a1 = (double)ac[1][k], a2 = (double)ac[2][k];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          M[0 * 3 + c] = fma(a0, xw[c][k], M[0 * 3 + c]);
          M[1 * 3 + c] = fma(a1, xw[c][k], M[1 * 3 + c]);
          M[2 * 3 + c] = fma(a2, xw[c][k], M[2 * 3 + c]);
        }
      }
      team_sum<9>(M, ts, red);
      if (active) {
        const double Ga = P.Ga[i];
        double D, R[9];
        if (mode == MODE_APPROX) {
          const double* Rs = P.Rsave + (size_t)i * 9;
          const double* Rx = P.Rxy;
          double tr = 0.0;
#pragma unroll
          for (int r0 = 0; r0 < 3; ++r0)
#pragma unroll
            for (int c0 = 0; c0 < 3; ++c0) {
              // (R_xy R_{a_i y})[c0][r0] contracted with M[r0][c0]
              const double rt = Rx[c0 * 3 + 0] * Rs[0 * 3 + r0] + Rx[c0 * 3 + 1] * Rs[1 * 3 + r0] +
                                Rx[c0 * 3 + 2] * Rs[2 * 3 + r0];
              tr = fma(rt, M[r0 * 3 + c0], tr);
            }
          D = clamp0(Gx + Ga - 2.0 * tr);
#pragma unroll
          for (int k = 0; k < 9; ++k) R[k] = Rs[k];
        } else {
          double F[10], lmax, qv[4];
          const int fb = top_eigenpair(M, 0.5 * (Gx + Ga), F, lmax, qv);
          if (fb && lane == 0 && P.fallbacks) atomicAdd((unsigned long long*)P.fallbacks, 1ull);
          D = clamp0(Gx + Ga - 2.0 * lmax);
          quat_to_rot(qv, R);
          if (mode == MODE_EXACT_SAVE && lane == 0) {
#pragma unroll
            for (int k = 0; k < 9; ++k) P.Rsave[(size_t)i * 9 + k] = R[k];
          }
        }
        if (dout != nullptr && lane == 0) dout[i] = D;
        if (D < m) {
          const double sc = scale_to(m, D, lam);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
#pragma unroll
            for (int k = 0; k < APT; ++k) { U[d][k] *= sc; V[d][k] *= sc; }
            tU[d] *= sc;
            tV[d] *= sc;
          }
          Z *= sc;
          S *= sc;
          m = D;
        }
        const double e = exp(-lam * (D - m));
        const double qi = P.q[i];
        Z += e;
        S = fma(e, qi, S);
        const double al = e * (qi - q0);
        const double* cap = P.ca + (size_t)i * 3;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double rc = R[d * 3 + 0] * cap[0] + R[d * 3 + 1] * cap[1] + R[d * 3 + 2] * cap[2];
          tU[d] = fma(al, rc, tU[d]);
          tV[d] = fma(e, rc, tV[d]);
        }
#pragma unroll
        for (int k = 0; k < APT; ++k) {
          const double a0 = (double)ac[0][k], a1 = (double)ac[1][k], a2 = (double)ac[2][k];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const double rr = fma(R[d * 3 + 0], a0, fma(R[d * 3 + 1], a1, R[d * 3 + 2] * a2));
            U[d][k] = fma(al, rr, U[d][k]);
            V[d][k] = fma(e, rr, V[d][k]);
          }
        }
      }
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int k = 0; k < APT; ++k) ac[d][k] = an[d][k];
    }
    // Centre the rotated landmarks: r = R a - R c.
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int k = 0; k < APT; ++k) { U[d][k] -= tU[d]; V[d][k] -= tV[d]; }

    // Tree merge of the teams of this workgroup, one atom slot k at a time.
    for (int stride = teams >> 1; stride >= 1; stride >>= 1) {
      __syncthreads();
      if (team >= stride && team < 2 * stride && lane == 0) {
        const int sl = team - stride;
        mh[sl * 3 + 0] = m;
        mh[sl * 3 + 1] = Z;
        mh[sl * 3 + 2] = S;
      }
      __syncthreads();
      double f1 = 0.0, f2 = 0.0, mn = m;
      if (team < stride) {
        const double m2 = mh[team * 3 + 0];
        mn = fmin(m, m2);
        f1 = scale_to(m, mn, lam);
        f2 = scale_to(m2, mn, lam);
        Z = Z * f1 + mh[team * 3 + 1] * f2;
        S = S * f1 + mh[team * 3 + 2] * f2;
      }
#pragma unroll
      for (int k = 0; k < APT; ++k) {
        __syncthreads();
        if (team >= stride && team < 2 * stride) {
          const int sl = team - stride;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            mv[(size_t)(sl * 6 + d) * ts + lane] = U[d][k];
            mv[(size_t)(sl * 6 + 3 + d) * ts + lane] = V[d][k];
          }
        }
        __syncthreads();
        if (team < stride) {
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            U[d][k] = U[d][k] * f1 + mv[(size_t)(team * 6 + d) * ts + lane] * f2;
            V[d][k] = V[d][k] * f1 + mv[(size_t)(team * 6 + 3 + d) * ts + lane] * f2;
          }
        }
      }
      if (team < stride) m = mn;
    }
    if (team == 0) {
      part_t* pu = partial_u<part_t>(P.vec, item.slot, n_pad);
      double* pv = partial_v<part_t>(P.vec, item.slot, n_pad);
#pragma unroll
      for (int k = 0; k < APT; ++k) {
        const int j = lane + ts * k;
        if (j < n_pad) {
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            pu[(size_t)d * n_pad + j] = (part_t)U[d][k];
            pv[(size_t)d * n_pad + j] = V[d][k];
          }
        }
      }
      if (lane == 0) {
        double* h = P.hdr + (size_t)item.slot * 4;
        h[0] = m;
        h[1] = Z;
        h[2] = S;
        h[3] = q0;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ merges
// Global (m, Z, S) of one problem from its item headers.
template <int BS>
__device__ void global_lse(const Problem& P, double* sh, double& m, double& Z, double& S) {
  double ml = INFINITY;
  for (int g = threadIdx.x; g < P.n_slots; g += BS) ml = fmin(ml, ldg(P.hdr + (size_t)g * 4));
  m = block_min<BS>(ml, sh);
  double v[2] = {0.0, 0.0};
  for (int g = threadIdx.x; g < P.n_slots; g += BS) {
    const double f = scale_to(ldg(P.hdr + (size_t)g * 4), m, P.lam);
    v[0] = fma(f, ldg(P.hdr + (size_t)g * 4 + 1), v[0]);
    v[1] = fma(f, ldg(P.hdr + (size_t)g * 4 + 2), v[1]);
  }
  block_sum<2, BS>(v, sh);
  Z = v[0];
  S = v[1];
}

// Header (m, Z, S, q0) of slot threadIdx.x, fetched before the merge's other
// loads so that its round trip overlaps theirs.
struct HdrSlot {
  double m, z, s, q;
};
// Loads are unconditional (clamped to the last slot) so that none of them
// waits for another; the values of threads past the slots are then replaced.
__device__ __forceinline__ HdrSlot hdr_first(const Problem& P) {
  const bool in = (int)threadIdx.x < P.n_slots;
  const double* h = P.hdr + (size_t)min((int)threadIdx.x, P.n_slots - 1) * 4;
  const double m = ldg(h + 0), z = ldg(h + 1), s = ldg(h + 2), q = ldg(h + 3);
  // Keep the scheduler from moving later loads ahead of these.
  __builtin_amdgcn_sched_barrier(0);
  return {in ? m : INFINITY, in ? z : 0.0, in ? s : 0.0, in ? q : 0.0};
}

// The log-sum-exp of global_lse from the first pass's headers in h (slots
// threadIdx.x + k BS for k >= 1 are read here), with every slot's weight
// f_g = exp(-lambda (m_g - m)) and q0_g - s staged in fw[g], fdq[g]
// (kMaxCloseSlots entries each).  Ends with a workgroup barrier.
template <int BS>
__device__ void lse_stage(const Problem& P, const HdrSlot& h, double* lsh, double* fw, double* fdq, double& m,
                          double& Z, double& S) {
  const int ns = P.n_slots;
  const double lam = P.lam;
  double ml = h.m;
  for (int g = threadIdx.x + BS; g < ns; g += BS) ml = fmin(ml, ldg(P.hdr + (size_t)g * 4));
  m = block_min<BS>(ml, lsh);
  const double f0 = scale_to(h.m, m, lam);
  double v[2] = {f0 * h.z, f0 * h.s};
  for (int g = threadIdx.x + BS; g < ns; g += BS) {
    const double f = scale_to(ldg(P.hdr + (size_t)g * 4), m, lam);
    v[0] = fma(f, ldg(P.hdr + (size_t)g * 4 + 1), v[0]);
    v[1] = fma(f, ldg(P.hdr + (size_t)g * 4 + 2), v[1]);
    fw[g] = f;
  }
  block_sum<2, BS>(v, lsh);
  Z = v[0];
  S = v[1];
  const double s = S / Z;
  if ((int)threadIdx.x < ns) {
    fw[threadIdx.x] = f0;
    fdq[threadIdx.x] = h.q - s;
  }
  for (int g = threadIdx.x + BS; g < ns; g += BS) fdq[g] = ldg(P.hdr + (size_t)g * 4 + 3) - s;
  __syncthreads();
}

// Rounding-correction share of one merge workgroup (see Problem::x_rounded),
// called by its whole first wave: lane a holds, for its atom j and the
// workgroup's coordinate c, ds_j,c d_j,c and dz_j,c d_j,c with
// d = x - x' = (w x_c - fl32(w x_c)) / w (zero for atoms past n).  blk is the
// workgroup's index among the 3 ceil(n / 64) that serve the problem;
// sz_correct_kernel adds the shares in index order.
__device__ void rounding_share(const Problem& P, double cs, double cz, int blk) {
  for (int off = 32; off >= 1; off >>= 1) {
    cs += __shfl_xor(cs, off, 64);
    cz += __shfl_xor(cz, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    stg(P.corr + 2 * (size_t)blk, cs);
    stg(P.corr + 2 * (size_t)blk + 1, cz);
  }
}

// This workgroup's terms of the correction for atom j, coordinate c, given
// the gradient sums gs, gz the merge formed for it.
__device__ __forceinline__ void rounding_terms(const Problem& P, int j, int c, double gs, double gz, double Z,
                                               double& cs, double& cz) {
  cs = 0.0;
  cz = 0.0;
  if (j >= P.n) return;
  const double wj = P.w[j];
  const double xw = P.xw[(size_t)c * P.n_pad + j];
  const double dw = xw - (double)(float)xw;   // w_j (x - x')_j,c
  if (wj <= 0.0 || dw == 0.0) return;
  cs = 2.0 * P.lam * gs / Z * dw;             // ds/dx_j,c (x - x')_j,c
  cz = 2.0 * (xw / wj - gz / Z) * dw;         // dz/dx_j,c (x - x')_j,c
}

// Algorithm 1 merge: s, z (Eq. 2) and, with r_ik the rotated centred
// landmarks, ds/dx_k = -2 lambda w_k sum_i p_i (q_i - s)(x_k - r_ik)
//                    = (2 lambda w_k / Z) sum_g f_g (U_g + (q0_g - s) V_g),
// dz/dx_k = 2 w_k sum_i p_i (x_k - r_ik) = 2 (w_k x_k - w_k / Z sum_g f_g V_g).
// Grid (atom blocks of 64, 3 coordinates, problems); the 256 threads of a
// workgroup are 64 atoms x 4 slot groups, so every slot's partial is read
// coalesced and the work spreads over 4x more workgroups than atom tiles of
// 256 would give.  The four group sums are added in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void merge_exact_kernel(const Problem* __restrict__ probs, Outs o,
                                                          const int* __restrict__ flag, int run_if) {
  using acc = typename AccT<T>::type;
  __shared__ double sh[8];
  __shared__ double fq[2][kMaxCloseSlots];
  __shared__ double red[2][4][64];
  const Problem& P = probs[blockIdx.z];
  // The gate flag and the problem's fields are read together: the empty
  // statement takes them all, so their loads are issued before the first
  // branch instead of one round trip after another.
  const int fl = flag != nullptr ? *flag : run_if;
  asm volatile("" ::"s"(fl), "s"(P.n), "s"(P.n_pad), "s"(P.n_slots), "s"(P.hdr), "s"(P.vec), "s"(P.w), "s"(P.xw),
               "s"(P.lam));
  if (fl != run_if) return;
  if ((int)blockIdx.x * 64 >= P.n) return;
  const int c = blockIdx.y;
  const int a = threadIdx.x & 63, sg = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + a;
  const int n_pad = P.n_pad, ns = P.n_slots;
  const bool jin = j < n_pad;
  // Loads that do not depend on the log-sum-exp: the first wave's per-atom
  // inputs, the slot headers and the first 16 partials of each wave (slots
  // sg, sg + 4, ..., sg + 60).
  // Every load is issued unconditionally at a clamped index (slot, atom)
  // and only used when in range, so none waits for another; the headers go
  // first, since loads complete in issue order and the log-sum-exp needs
  // them before the partials.
  const HdrSlot h = hdr_first(P);
  const int jc = min(j, P.n - 1);
  const double wj = ldg(P.w + jc), xwj = ldg(P.xw + (size_t)c * n_pad + jc);
  const int jp = min(j, n_pad - 1);
  acc u[16];
  double v[16];
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    const int g = min(sg + 4 * b, ns - 1);
    u[b] = ldg_nt(partial_u<acc>(P.vec, g, n_pad) + (size_t)c * n_pad + jp);
    v[b] = ldg_nt(partial_v<acc>(P.vec, g, n_pad) + (size_t)c * n_pad + jp);
  }
  double m, Z, S;
  lse_stage<256>(P, h, sh, fq[0], fq[1], m, Z, S);
  const double s = S / Z;
  double gs = 0.0, gz = 0.0;
  if (jin) {
    // Slots in order; 16 of them are loaded before any is added, so a wave
    // waits for one round trip per 16 slots.
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      const int g = sg + 4 * b;
      if (g < ns) {
        const double f = fq[0][g];
        gs = fma(f, fma(fq[1][g], v[b], (double)u[b]), gs);
        gz = fma(f, v[b], gz);
      }
    }
    int t = sg + 64;
    for (; t + 60 < ns; t += 64) {
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        u[b] = ldg_nt(partial_u<acc>(P.vec, t + 4 * b, n_pad) + (size_t)c * n_pad + j);
        v[b] = ldg_nt(partial_v<acc>(P.vec, t + 4 * b, n_pad) + (size_t)c * n_pad + j);
      }
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        const double f = fq[0][t + 4 * b];
        gs = fma(f, fma(fq[1][t + 4 * b], v[b], (double)u[b]), gs);
        gz = fma(f, v[b], gz);
      }
    }
#pragma unroll 4
    for (; t < ns; t += 4) {
      const double uu = (double)ldg_nt(partial_u<acc>(P.vec, t, n_pad) + (size_t)c * n_pad + j);
      const double vv = ldg_nt(partial_v<acc>(P.vec, t, n_pad) + (size_t)c * n_pad + j);
      const double f = fq[0][t];
      gs = fma(f, fma(fq[1][t], vv, uu), gs);
      gz = fma(f, vv, gz);
    }
  }
  red[0][sg][a] = gs;
  red[1][sg][a] = gz;
  __syncthreads();
  if (sg == 0) {
    gs = ((red[0][0][a] + red[0][1][a]) + red[0][2][a]) + red[0][3][a];
    gz = ((red[1][0][a] + red[1][1][a]) + red[1][2][a]) + red[1][3][a];
    if (j < P.n) {
      const size_t at = 3 * ((size_t)P.out_off + j) + c;
      if (o.ds) ((T*)o.ds)[at] = (T)(2.0 * P.lam * wj * gs / Z);
      if (o.dz) ((T*)o.dz)[at] = (T)(2.0 * (xwj - wj * gz / Z));
    }
    if (P.x_rounded) {
      double cs, cz;
      rounding_terms(P, j, c, gs, gz, Z, cs, cz);
      rounding_share(P, cs, cz, c * ((P.n + 63) / 64) + (int)blockIdx.x);
    }
  }
  if (blockIdx.x == 0 && c == 0 && threadIdx.x == 0) {
    o.sz[2 * P.out_idx + 0] = s;
    o.sz[2 * P.out_idx + 1] = m - log(Z) / P.lam;
  }
}

// (s, z) of each problem with x_rounded plus its merge workgroups' rounding
// shares, added in workgroup order (one wave per problem; launched after
// the merge, gated like it).
__global__ __launch_bounds__(64) void sz_correct_kernel(const Problem* __restrict__ probs, Outs o,
                                                        const int* __restrict__ flag, int run_if) {
  const Problem& P = probs[blockIdx.x];
  // Gate flag and fields read together (see merge_exact_kernel).
  const int fl = flag != nullptr ? *flag : run_if;
  asm volatile("" ::"s"(fl), "s"(P.x_rounded), "s"(P.n), "s"(P.corr), "s"(P.out_idx));
  if (fl != run_if || !P.x_rounded) return;
  const int nblk = 3 * ((P.n + 63) / 64);
  // Eight shares per lane are loaded before any is added (one round trip
  // up to 512 shares, i.e. 10,922 atoms); larger structures loop.
  typedef double pair_t __attribute__((ext_vector_type(2)));
  double as = 0.0, az = 0.0;
  for (int b0 = 0; b0 < nblk; b0 += 512) {
    pair_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + threadIdx.x + 64 * u;
      v[u] = b < nblk ? *reinterpret_cast<const pair_t*>(P.corr + 2 * (size_t)b) : pair_t{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      as += v[u][0];
      az += v[u][1];
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    as += __shfl_xor(as, off, 64);
    az += __shfl_xor(az, off, 64);
  }
  if (threadIdx.x == 0) {
    o.sz[2 * P.out_idx + 0] += as;
    o.sz[2 * P.out_idx + 1] += az;
  }
}

// Algorithm 2 merge for the approximate step.  The partials accumulate
// b_ik = R_{a_i y} (a_ik - c_i) (landmarks in y's frame):
//   beta_k  = sum_i c_i b_ik = -(lambda/Z) sum_g f_g (U_g + (q0_g - s) V_g),
//   betaz_k = sum_i p_i b_ik = (1/Z) sum_g f_g V_g,
// the explicit Eq. 6 terms ds/dx_k = -2 w_k R_xy beta_k and
// dz/dx_k = 2 (w_k x_k - w_k R_xy betaz_k), and the rotation term: with
// G = -2 sum_j w_j x_j beta_j^T (the symmetric part of Eq. 6's contraction
// has no tangent component), Gamma = d(G:R_xy)/dM_xy and the contribution
// w_k sum_a Gamma_ac y_k[a].
//
// Stage 1 (one workgroup per 64 atoms and coordinate c, 4 slot groups):
// beta_c and betaz_c of its atoms and its share of column c of the two 3x3
// contractions G (6 values).  Stage 2 (one workgroup): G summed over the
// tiles in a fixed order, the two rotation adjoints, and per atom the
// explicit terms (R_xy beta, R_xy betaz) plus the rotation terms.
// gtmp layout: [0, 3 n_pad) beta, [3 n_pad, 6 n_pad) betaz,
// [6 n_pad, 6 n_pad + 18 * tiles) G shares (entry r * 3 + c of G_s, then of
// G_z, per tile).
constexpr int kBetaThreads = 256;

// Last-arrival test of a workgroup's first wave, called by all its lanes
// after the wave's global writes: true in exactly one of the nblk
// workgroups of the launch, which then sees every other workgroup's writes
// and must return *ticket to 0.
__device__ bool last_arrival(unsigned* ticket, int nblk) {
  __threadfence();
  unsigned v = 0;
  if ((threadIdx.x & 63) == 0) v = atomicAdd(ticket, 1u);
  v = __shfl(v, 0, 64);
  const bool last = v == (unsigned)nblk - 1;
  if (last) __threadfence();
  return last;
}

// The exact merge (as merge_exact_kernel) of one tile of 64 atoms and
// coordinate c: the reassignment branch of a close-structure step served by
// the same launch.
template <typename T, int BS>
__device__ void merge_exact_tile(const Problem& P, const Outs& o, int tile, int c, unsigned* ticket) {
  using acc = typename AccT<T>::type;
  constexpr int NG = BS / 64;
  __shared__ double xsh[2 * NG];
  __shared__ double xfq[2][256];
  __shared__ double xred[2][NG][64];
  double m, Z, S;
  global_lse<BS>(P, xsh, m, Z, S);
  const double s = S / Z;
  const int a = threadIdx.x & 63, sg = threadIdx.x >> 6;
  const int j = tile * 64 + a;
  const int n_pad = P.n_pad;
  double gs = 0.0, gz = 0.0;
  for (int g0 = 0; g0 < P.n_slots; g0 += 256) {
    __syncthreads();
    const int g = g0 + threadIdx.x;
    if (threadIdx.x < 256 && g < P.n_slots) {
      xfq[0][threadIdx.x] = scale_to(ldg(P.hdr + (size_t)g * 4), m, P.lam);
      xfq[1][threadIdx.x] = ldg(P.hdr + (size_t)g * 4 + 3) - s;
    }
    __syncthreads();
    const int gn = min(256, P.n_slots - g0);
    if (j < n_pad) {
#pragma unroll 4
      for (int t = sg; t < gn; t += NG) {
        const double u = (double)ldg_nt(partial_u<acc>(P.vec, g0 + t, n_pad) + (size_t)c * n_pad + j);
        const double v = ldg_nt(partial_v<acc>(P.vec, g0 + t, n_pad) + (size_t)c * n_pad + j);
        const double f = xfq[0][t];
        gs = fma(f, fma(xfq[1][t], v, u), gs);
        gz = fma(f, v, gz);
      }
    }
  }
  xred[0][sg][a] = gs;
  xred[1][sg][a] = gz;
  __syncthreads();
  if (sg == 0) {
    double ts = 0.0, tz = 0.0;
    for (int q = 0; q < NG; ++q) {
      ts += xred[0][q][a];
      tz += xred[1][q][a];
    }
    if (j < P.n) {
      const double wj = P.w[j];
      const size_t at = 3 * ((size_t)P.out_off + j) + c;
      if (o.ds) ((T*)o.ds)[at] = (T)(2.0 * P.lam * wj * ts / Z);
      if (o.dz) ((T*)o.dz)[at] = (T)(2.0 * (P.xw[(size_t)c * n_pad + j] - wj * tz / Z));
    }
    if (P.x_rounded) {
      double cs, cz;
      rounding_terms(P, j, c, ts, tz, Z, cs, cz);
      rounding_share(P, cs, cz, c * (int)gridDim.x + tile);
      // With a ticket the last workgroup adds the shares (tiles x 3 of
      // them, in order) and writes (s, z); otherwise the second kernel does.
      if (ticket != nullptr && last_arrival(ticket, 3 * (int)gridDim.x)) {
        const int nblk = 3 * (int)gridDim.x;
        double as = 0.0, az = 0.0;
        for (int b = a; b < nblk; b += 64) {
          as += P.corr[2 * (size_t)b];
          az += P.corr[2 * (size_t)b + 1];
        }
        for (int off = 32; off >= 1; off >>= 1) {
          as += __shfl_xor(as, off, 64);
          az += __shfl_xor(az, off, 64);
        }
        if (a == 0) {
          o.sz[2 * P.out_idx + 0] = s + as;
          o.sz[2 * P.out_idx + 1] = m - log(Z) / P.lam + az;
          *ticket = 0u;
        }
      }
    }
  }
  if (tile == 0 && c == 0 && threadIdx.x == 0 && !(ticket != nullptr && P.x_rounded)) {
    o.sz[2 * P.out_idx + 0] = s;
    o.sz[2 * P.out_idx + 1] = m - log(Z) / P.lam;
  }
}

// Eq. 6 second stage of the approximate step, run by the first BS threads
// of a workgroup (BS = 64: one wave, the others may have exited): G of the
// s and z terms summed over the tiles' shares in gtmp (fixed order), the two
// rotation adjoints Gamma, then per atom the explicit terms -2 w R_xy beta
// and 2 (w x - w R_xy betaz) plus the rotation terms, and (s, z).
template <typename T, int BS>
__device__ void close_final_stage(const Problem& P, const Outs& o, const CloseArgs& cs,
                                  const double* __restrict__ gtmp, int tiles, double m, double Z, double S,
                                  double* sh, double* gam) {
  const int t = threadIdx.x;
  const int n = P.n, n_pad = P.n_pad;
  auto sync = [&]() {
    if (BS == 64) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
      __syncthreads();
    }
  };
  if (t < 18) {
    double g = 0.0;
    for (int k = 0; k < tiles; ++k) g += gtmp[6 * (size_t)n_pad + (size_t)k * 18 + t];
    sh[t] = g;
  }
  sync();
  // The two adjoints (for s and for z) are independent: two lanes of one
  // wave (BS = 64) or the first lanes of two waves.
  constexpr int tz = BS > 64 ? 64 : 1;
  if (t == 0 || t == tz) {
    const int h = t == 0 ? 0 : 9;
    double F[10], qv[4], G[9], Gm[9];
    for (int k = 0; k < 10; ++k) F[k] = cs.Fxy[k];
    for (int k = 0; k < 4; ++k) qv[k] = cs.qxy[k];
    for (int k = 0; k < 9; ++k) G[k] = sh[h + k];
    rotation_adjoint(F, *cs.lamxy, qv, G, Gm);
    for (int k = 0; k < 9; ++k) gam[h + k] = Gm[k];
  }
  sync();
  T* ds = (T*)o.ds;
  T* dz = (T*)o.dz;
  const double* Rx = cs.Rxy;
  for (int j = t; j < n; j += BS) {
    double y[3], be[3], bz[3], xw[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      y[d] = cs.y64[(size_t)d * n_pad + j];
      be[d] = gtmp[(size_t)d * n_pad + j];
      bz[d] = gtmp[3 * (size_t)n_pad + (size_t)d * n_pad + j];
      xw[d] = P.xw[(size_t)d * n_pad + j];
    }
    const double wj = P.w[j];
#pragma unroll
    for (int c0 = 0; c0 < 3; ++c0) {
      const double rb = Rx[c0 * 3 + 0] * be[0] + Rx[c0 * 3 + 1] * be[1] + Rx[c0 * 3 + 2] * be[2];
      const double rzb = Rx[c0 * 3 + 0] * bz[0] + Rx[c0 * 3 + 1] * bz[1] + Rx[c0 * 3 + 2] * bz[2];
      const double rs = wj * (gam[0 * 3 + c0] * y[0] + gam[1 * 3 + c0] * y[1] + gam[2 * 3 + c0] * y[2]);
      const double rz = wj * (gam[9 + 0 * 3 + c0] * y[0] + gam[9 + 1 * 3 + c0] * y[1] + gam[9 + 2 * 3 + c0] * y[2]);
      if (ds) ds[3 * j + c0] = (T)(-2.0 * wj * rb + rs);
      if (dz) dz[3 * j + c0] = (T)(2.0 * (xw[c0] - wj * rzb) + rz);
    }
  }
  if (t == 0) {
    o.sz[0] = S / Z;
    o.sz[1] = m - log(Z) / P.lam;
  }
}

// The approximate step's merge in one pass when the engine left per-item
// XU / XV sums (Problem::xuv): G_s = (2 lambda / Z) sum_g f_g (XU_g +
// (q0_g - s) XV_g) and G_z = -(2 / Z) sum_g f_g XV_g are formed by every
// workgroup from the item sums, so each can finish its own atoms (all three
// coordinates of 64 atoms; the workgroups of coordinates 1 and 2 of the
// grid have nothing to do).  Wave 0 forms the log-sum-exp, G and the two
// rotation adjoints while the other waves sum the item partials of the
// tile's atoms.
//
// The step is a chain of dependent round trips, so the problem's fields are
// read together with the step flag, and every load that does not depend on
// the log-sum-exp is issued before it: wave 0's item headers (slots a + 64 k,
// k < 4), the y -> x eigen-system and its first two item sums, and the
// first kOnePassPrefetch partials of each other wave; the adjoints'
// Cholesky factor (from the eigen-system only) is formed while they are in
// flight.  Returns false when the caller has to run the reassignment branch
// (flag 1 with an exact problem), true otherwise.
constexpr int kOnePassPrefetch = 12;
template <typename T, int BS>
__device__ bool close_merge_one(const Problem& P, const CloseArgs& cs, const Outs& o, int tile, int c,
                                bool has_exact) {
  using acc = typename AccT<T>::type;
  constexpr int NG = BS / 64;    // wave 0: log-sum-exp, G and the adjoints; waves 1..NG-1: the partials
  constexpr int NW = NG - 1;
  constexpr int PF = kOnePassPrefetch;
  constexpr int KH = 4;          // header slots per wave-0 lane read ahead
  static_assert(3 * PF == 36, "wave 0 keeps two item sums (2 x 18 doubles) in the partials' registers");
  __shared__ double fq1[2][kMaxCloseSlots];
  __shared__ double red1[6][NW][64];
  __shared__ double gsum[18], gam1[18];
  // The problem's fields, read with the flag (one round trip for all).
  const int n_pad = P.n_pad, ns = P.n_slots, n = P.n;
  const double lam = P.lam;
  const double* __restrict__ hdr = P.hdr;
  void* vec = P.vec;
  const double* __restrict__ xuv = P.xuv;
  const double* __restrict__ xwp = P.xw;
  const double* __restrict__ wp = P.w;
  const int flag = __builtin_amdgcn_readfirstlane(ldg(cs.flag));
  // An empty statement that takes the fields: their loads are issued before
  // the flag's branch instead of being moved behind it.
  asm volatile("" ::"s"(n_pad), "s"(ns), "s"(n), "s"(lam), "s"(hdr), "s"(vec), "s"(xuv), "s"(xwp), "s"(wp));
  if (flag == 1 && has_exact) return false;
  if (flag != 0 || c != 0) return true;
  const int a = threadIdx.x & 63, sg = threadIdx.x >> 6;
  const int j = tile * 64 + a;
  const bool jin = j < n_pad;
  // Wave 0: headers first (loads complete in issue order), then the
  // eigen-system.
  double hm[KH], hz[KH], hs[KH], hq[KH];
  double F[10], qv[4], lxy = 0.0;
  if (sg == 0) {
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const double* h = hdr + (size_t)min(a + 64 * k, ns - 1) * 4;
      hm[k] = ldg(h + 0);
      hz[k] = ldg(h + 1);
      hs[k] = ldg(h + 2);
      hq[k] = ldg(h + 3);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 10; ++k) F[k] = ldg(cs.Fxy + k);
#pragma unroll
    for (int k = 0; k < 4; ++k) qv[k] = ldg(cs.qxy + k);
    lxy = ldg(cs.lamxy);
  }
  // pv: a partial-summing wave's V partials of its first PF items, or wave
  // 0's item sums of items a and a + 64 (entries 0..17 and 18..35).  One
  // unconditional load per register at a clamped index, the address chosen
  // per wave (no branch, so no value has to be complete before the sums;
  // wave 0's pu loads are not used).
  double pv[PF][3];
  acc pu[PF][3];
  {
    const int jp = min(j, n_pad - 1);
#pragma unroll
    for (int b = 0; b < PF; ++b) {
      const int g = max(0, min(sg - 1 + NW * b, ns - 1));
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int k = 3 * b + d;
        const double* x0 = xuv + (size_t)min(a + 64 * (k / 18), ns - 1) * 18 + k % 18;
        const double* pvp = partial_v<acc>(vec, g, n_pad) + (size_t)d * n_pad + jp;
        pu[b][d] = ldg_nt(partial_u<acc>(vec, g, n_pad) + (size_t)d * n_pad + jp);
        pv[b][d] = ldg_nt(sg == 0 ? x0 : pvp);
      }
    }
  }
  double m = 0.0, Z = 0.0, S = 0.0;
  AdjointFactor af;
  if (sg == 0) {
    if (a < 2) adjoint_factor(F, lxy, qv, af);
    // Log-sum-exp over the item headers (lane-local in slot order, then a
    // fixed xor tree): (m, Z, S), and every slot's f_g and q0_g - s into LDS.
    double ml = INFINITY;
#pragma unroll
    for (int k = 0; k < KH; ++k) ml = (a + 64 * k < ns) ? fmin(ml, hm[k]) : ml;
    for (int g = a + 64 * KH; g < ns; g += 64) ml = fmin(ml, ldg(hdr + (size_t)g * 4));
    for (int off = 32; off > 0; off >>= 1) ml = fmin(ml, __shfl_xor(ml, off, 64));
    m = ml;
    double fk[KH], zl = 0.0, sl = 0.0;
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      fk[k] = (a + 64 * k < ns) ? scale_to(hm[k], m, lam) : 0.0;
      zl = fma(fk[k], hz[k], zl);
      sl = fma(fk[k], hs[k], sl);
    }
    for (int g = a + 64 * KH; g < ns; g += 64) {
      const double f = scale_to(ldg(hdr + (size_t)g * 4), m, lam);
      zl = fma(f, ldg(hdr + (size_t)g * 4 + 1), zl);
      sl = fma(f, ldg(hdr + (size_t)g * 4 + 2), sl);
      fq1[0][g] = f;
    }
    for (int off = 32; off > 0; off >>= 1) {
      zl += __shfl_xor(zl, off, 64);
      sl += __shfl_xor(sl, off, 64);
    }
    Z = zl;
    S = sl;
    const double s = S / Z;
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const int g = a + 64 * k;
      if (g < ns) {
        fq1[0][g] = fk[k];
        fq1[1][g] = hq[k] - s;
      }
    }
    for (int g = a + 64 * KH; g < ns; g += 64) fq1[1][g] = ldg(hdr + (size_t)g * 4 + 3) - s;
  }
  __syncthreads();
  double su[3] = {0.0, 0.0, 0.0}, sv[3] = {0.0, 0.0, 0.0};
  double y[3], xw[3], wj, Rx[9];
  if (sg == 0) {
    // The atom's inputs of the final stage, in flight during the sums
    // (clamped atom; only atoms below n are written).
    const int jc = min(j, n - 1);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      y[d] = ldg(cs.y64 + (size_t)d * n_pad + jc);
      xw[d] = ldg(xwp + (size_t)d * n_pad + jc);
    }
    wj = ldg(wp + jc);
#pragma unroll
    for (int k = 0; k < 9; ++k) Rx[k] = ldg(cs.Rxy + k);
    // Item sums, lane t taking items t, t + 64, ... (fixed order), then G
    // as fixed-order wave sums and the two adjoints in lanes 0 (s) and 1 (z).
    double g18[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) g18[k] = 0.0;
    auto add_item = [&](int g, const double (&xp)[18]) {
      const double f = fq1[0][g], dq = fq1[1][g];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        g18[k] = fma(f, fma(dq, xp[9 + k], xp[k]), g18[k]);
        g18[9 + k] = fma(f, xp[9 + k], g18[9 + k]);
      }
    };
    {
      double x0[18], x1[18];
#pragma unroll
      for (int k = 0; k < 18; ++k) {
        x0[k] = pv[k / 3][k % 3];
        x1[k] = pv[(18 + k) / 3][(18 + k) % 3];
      }
      if (a < ns) add_item(a, x0);
      if (a + 64 < ns) add_item(a + 64, x1);
    }
    for (int g = a + 128; g < ns; g += 64) {
      double xp[18];
#pragma unroll
      for (int k = 0; k < 18; ++k) xp[k] = ldg(xuv + (size_t)g * 18 + k);
      add_item(g, xp);
    }
    wave_sum9_store(g18, gsum, a);
    wave_sum9_store(g18 + 9, gsum + 9, a);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (a < 2) {
      const int h = a == 0 ? 0 : 9;
      const double sc = a == 0 ? 2.0 * lam / Z : -2.0 / Z;
      double G[9], Gm[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) G[k] = sc * gsum[h + k];
      adjoint_apply(af, qv, G, Gm);
#pragma unroll
      for (int k = 0; k < 9; ++k) gam1[h + k] = Gm[k];
    }
  } else if (jin) {
    // Items g = sg - 1 + NW b: the prefetched ones, then the rest with four
    // in flight before any is added.
#pragma unroll
    for (int b = 0; b < PF; ++b) {
      const int g = sg - 1 + NW * b;
      if (g < ns) {
        const double f = fq1[0][g], dq = fq1[1][g];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          su[d] = fma(f, fma(dq, pv[b][d], (double)pu[b][d]), su[d]);
          sv[d] = fma(f, pv[b][d], sv[d]);
        }
      }
    }
    int g = sg - 1 + NW * PF;
    for (; g + 3 * NW < ns; g += 4 * NW) {
      acc u[4][3];
      double v[4][3];
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          u[b][d] = ldg_nt(partial_u<acc>(vec, g + NW * b, n_pad) + (size_t)d * n_pad + j);
          v[b][d] = ldg_nt(partial_v<acc>(vec, g + NW * b, n_pad) + (size_t)d * n_pad + j);
        }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const double f = fq1[0][g + NW * b], dq = fq1[1][g + NW * b];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          su[d] = fma(f, fma(dq, v[b][d], (double)u[b][d]), su[d]);
          sv[d] = fma(f, v[b][d], sv[d]);
        }
      }
    }
    for (; g < ns; g += NW) {
      const double f = fq1[0][g], dq = fq1[1][g];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double u = (double)ldg_nt(partial_u<acc>(vec, g, n_pad) + (size_t)d * n_pad + j);
        const double v = ldg_nt(partial_v<acc>(vec, g, n_pad) + (size_t)d * n_pad + j);
        su[d] = fma(f, fma(dq, v, u), su[d]);
        sv[d] = fma(f, v, sv[d]);
      }
    }
  }
  if (sg != 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      red1[d][sg - 1][a] = su[d];
      red1[3 + d][sg - 1][a] = sv[d];
    }
  }
  __syncthreads();
  if (sg != 0 || j >= n) return true;
  const double iz = 1.0 / Z;
  double be[3], bz[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double t0 = 0.0, t1 = 0.0;
    for (int q = 0; q < NW; ++q) {
      t0 += red1[d][q][a];
      t1 += red1[3 + d][q][a];
    }
    be[d] = -lam * iz * t0;
    bz[d] = t1 * iz;
  }
  T* ds = (T*)o.ds;
  T* dz = (T*)o.dz;
#pragma unroll
  for (int c0 = 0; c0 < 3; ++c0) {
    const double rb = Rx[c0 * 3 + 0] * be[0] + Rx[c0 * 3 + 1] * be[1] + Rx[c0 * 3 + 2] * be[2];
    const double rzb = Rx[c0 * 3 + 0] * bz[0] + Rx[c0 * 3 + 1] * bz[1] + Rx[c0 * 3 + 2] * bz[2];
    const double rs = wj * (gam1[0 * 3 + c0] * y[0] + gam1[1 * 3 + c0] * y[1] + gam1[2 * 3 + c0] * y[2]);
    const double rz = wj * (gam1[9 + 0 * 3 + c0] * y[0] + gam1[9 + 1 * 3 + c0] * y[1] + gam1[9 + 2 * 3 + c0] * y[2]);
    if (ds) ds[3 * j + c0] = (T)(-2.0 * wj * rb + rs);
    if (dz) dz[3 * j + c0] = (T)(2.0 * (xw[c0] - wj * rzb) + rz);
  }
  if (tile == 0 && a == 0) {
    o.sz[0] = S * iz;
    o.sz[1] = m - log(Z) / lam;
  }
  return true;
}

// fuse 1: the close-merge ticket is used, so the last workgroup runs the
// second stage (and, on reassignment steps, the rounding correction);
// fuse 2 (launched with kOnePassThreads): as 1 on reassignment steps, and
// the approximate step in one pass (close_merge_one).
constexpr int kOnePassThreads = 512;
template <typename T, int BS>
__global__ __launch_bounds__(BS) void merge_close_beta_kernel(const Problem* __restrict__ prob, CloseArgs cs,
                                                              double* __restrict__ gtmp,
                                                              const Problem* __restrict__ prob_exact, Outs o,
                                                              int fuse) {
  using acc = typename AccT<T>::type;  // partial storage type
  constexpr int NG = kBetaThreads / 64;   // slot groups
  const int c = blockIdx.y;
  if constexpr (BS == kOnePassThreads) {
    if (!close_merge_one<T, BS>(*prob, cs, o, blockIdx.x, c, prob_exact != nullptr))
      merge_exact_tile<T, BS>(*prob_exact, o, blockIdx.x, c, fuse ? cs.ticket : nullptr);
    return;
  }
  const int flag = __builtin_amdgcn_readfirstlane(*cs.flag);
  if (flag == 1 && prob_exact != nullptr) {
    merge_exact_tile<T, BS>(*prob_exact, o, blockIdx.x, c, fuse ? cs.ticket : nullptr);
    return;
  }
  if (flag != 0) return;
  if constexpr (BS != kOnePassThreads) {
  if (fuse == 2) return;   // launched with kOnePassThreads only
  __shared__ double sh[2 * NG];
  __shared__ double fq[2][256];
  __shared__ double red[2][NG][64];
  const Problem& P = *prob;
  double m, Z, S;
  global_lse<kBetaThreads>(P, sh, m, Z, S);
  const double s = S / Z;
  const double lam = P.lam;
  const int n_pad = P.n_pad;
  const int a = threadIdx.x & 63, sg = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + a;
  double su = 0.0, sv = 0.0;
  for (int g0 = 0; g0 < P.n_slots; g0 += 256) {
    __syncthreads();
    const int g = g0 + threadIdx.x;
    if (g < P.n_slots) {
      fq[0][threadIdx.x] = scale_to(ldg(P.hdr + (size_t)g * 4), m, lam);
      fq[1][threadIdx.x] = ldg(P.hdr + (size_t)g * 4 + 3) - s;
    }
    __syncthreads();
    const int gn = min(256, P.n_slots - g0);
    if (j < n_pad) {
#pragma unroll 4
      for (int t = sg; t < gn; t += NG) {
        const double u = (double)ldg_nt(partial_u<acc>(P.vec, g0 + t, n_pad) + (size_t)c * n_pad + j);
        const double v = ldg_nt(partial_v<acc>(P.vec, g0 + t, n_pad) + (size_t)c * n_pad + j);
        const double f = fq[0][t];
        su = fma(f, fma(fq[1][t], v, u), su);
        sv = fma(f, v, sv);
      }
    }
  }
  red[0][sg][a] = su;
  red[1][sg][a] = sv;
  __syncthreads();
  if (sg != 0) return;
  // Wave 0: beta_c, betaz_c of the tile's atoms and column c of its G share.
  double G[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (j < n_pad) {
    double a0 = 0.0, b0 = 0.0;
    for (int q = 0; q < NG; ++q) {
      a0 += red[0][q][a];
      b0 += red[1][q][a];
    }
    const double be = -lam / Z * a0, bz = b0 / Z;
    gtmp[(size_t)c * n_pad + j] = be;
    gtmp[3 * (size_t)n_pad + (size_t)c * n_pad + j] = bz;
    if (j < P.n) {
#pragma unroll
      for (int r0 = 0; r0 < 3; ++r0) {
        const double xw = P.xw[(size_t)r0 * n_pad + j];
        G[r0] = -2.0 * xw * be;
        G[3 + r0] = -2.0 * xw * bz;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k)
    for (int off = 32; off > 0; off >>= 1) G[k] += __shfl_xor(G[k], off, 64);
  if (a == 0) {
    double* gs = gtmp + 6 * (size_t)n_pad + (size_t)blockIdx.x * 18;
#pragma unroll
    for (int r0 = 0; r0 < 3; ++r0) {
      gs[r0 * 3 + c] = G[r0];
      gs[9 + r0 * 3 + c] = G[3 + r0];
    }
  }
  if (fuse == 1 && last_arrival(cs.ticket, (int)(gridDim.x * gridDim.y))) {
    __shared__ double fsh[18], fgam[18];
    close_final_stage<T, 64>(P, o, cs, gtmp, (int)gridDim.x, m, Z, S, fsh, fgam);
    if (a == 0) *cs.ticket = 0u;
  }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void merge_close_final_kernel(const Problem* __restrict__ prob, Outs o,
                                                                CloseArgs cs, const double* __restrict__ gtmp,
                                                                int tiles, const Problem* __restrict__ prob_exact) {
  constexpr int BS = 256;
  const int flag = *cs.flag;   // tested once the independent loads below are in flight
  if (flag == 1 && prob_exact != nullptr) {
    // Reassignment branch: the exact merge of the first kernel wrote (s, z)
    // and, with x_rounded, its rounding shares (3 tiles workgroups).
    if (threadIdx.x < 64) {
      const Problem& E = *prob_exact;
      if (!E.x_rounded) return;
      double as = 0.0, az = 0.0;
      for (int b = threadIdx.x; b < 3 * tiles; b += 64) {
        as += E.corr[2 * (size_t)b];
        az += E.corr[2 * (size_t)b + 1];
      }
      for (int off = 32; off >= 1; off >>= 1) {
        as += __shfl_xor(as, off, 64);
        az += __shfl_xor(az, off, 64);
      }
      if (threadIdx.x == 0) {
        o.sz[2 * E.out_idx + 0] += as;
        o.sz[2 * E.out_idx + 1] += az;
      }
    }
    return;
  }
  if (flag != 0) return;
  __shared__ double lsh[2 * (BS / 64)];
  __shared__ double fsh[18], gam[18];
  const Problem& P = *prob;
  double m, Z, S;
  global_lse<BS>(P, lsh, m, Z, S);
  close_final_stage<T, BS>(P, o, cs, gtmp, tiles, m, Z, S, fsh, gam);
}

__global__ void set_int_kernel(int* p, int v) { *p = v; }
__global__ void count_kernel(long long* c, int which, long long add) { c[which] += add; }

// ------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_load_landmarks(const T* in, T* A, double* ca, double* Ga, const double* w,
                                 int n, int n_pad, int L, hipStream_t st) {
  if (L <= 0) return hipSuccess;
  hipLaunchKernelGGL((load_kernel<T>), dim3(L), dim3(256), 0, st, in, A, ca, Ga, w, n, n_pad);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pair_msd(const T* A, const double* ca, const double* Ga, const double* w,
                           int n, int n_pad, int L, double* out, hipStream_t st) {
  if (L < 2) return hipSuccess;
  hipLaunchKernelGGL((pair_msd_kernel<T>), dim3(L - 1), dim3(256), 0, st, A, ca, Ga, w, n, n_pad, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prep(const PrepArgs* d_args, const void* x_base, int n_prob, int max_n, hipStream_t st) {
  if (max_n <= 1024)
    hipLaunchKernelGGL((prep_kernel<T, 256>), dim3(n_prob), dim3(256), 0, st, d_args, x_base);
  else
    hipLaunchKernelGGL((prep_kernel<T, 512>), dim3(n_prob), dim3(512), 0, st, d_args, x_base);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prep_close(PrepArgs pa, const void* x, CloseArgs ca, Outs outs, hipStream_t st) {
  hipLaunchKernelGGL((prep_close_kernel<T>), dim3(1), dim3(256), 0, st, pa, (const T*)x, ca, outs);
  return hipGetLastError();
}

size_t engine_lds_bytes(EngineCfg cfg, int ts, bool fp64) {
  (void)fp64;
  size_t b = (size_t)(cfg.wg / 64) * 9 * 8 + (size_t)(cfg.wg / 32) * 3 * 8;
  if (cfg.wg / ts > 1) b += (size_t)(cfg.wg / 2) * 6 * 8;
  return b;
}

#define PCV_ENGINE_CASES_F32(X) X(256, 1) X(256, 2) X(256, 4) X(256, 8) X(512, 8) X(512, 10) X(512, 16)
#define PCV_ENGINE_CASES_F64(X) X(256, 1) X(256, 2) X(256, 4) X(256, 8)

bool engine_supported(EngineCfg cfg, bool fp64) {
#define PCV_CASE(W, P) if (cfg.wg == W && cfg.apt == P) return true;
  if (fp64) { PCV_ENGINE_CASES_F64(PCV_CASE) }
  else { PCV_ENGINE_CASES_F32(PCV_CASE) }
#undef PCV_CASE
  return false;
}

void engine_configs(bool fp64, EngineCfg* out, int* count) {
  int k = 0;
#define PCV_CASE(W, P) out[k++] = EngineCfg{W, P};
  if (fp64) { PCV_ENGINE_CASES_F64(PCV_CASE) }
  else { PCV_ENGINE_CASES_F32(PCV_CASE) }
#undef PCV_CASE
  *count = k;
}

hipError_t engine_init_attributes() {
  hipError_t e = hipSuccess;
#define PCV_CASE_T(T, W, P)                                                                   \
  {                                                                                           \
    hipError_t r = hipFuncSetAttribute((const void*)engine_kernel<T, W, P>,                  \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024); \
    if (r != hipSuccess) e = r;                                                               \
  }
#define PCV_CASE_F(W, P) PCV_CASE_T(float, W, P)
#define PCV_CASE_D(W, P) PCV_CASE_T(double, W, P)
  PCV_ENGINE_CASES_F32(PCV_CASE_F)
  PCV_ENGINE_CASES_F64(PCV_CASE_D)
#undef PCV_CASE_F
#undef PCV_CASE_D
#undef PCV_CASE_T
  return e;
}

template <typename T, int WG, int APT>
static hipError_t launch_engine_inst(int grid, size_t lds, const Problem* probs, const Item* items,
                                     const int* wg_off, int mode, const int* flag, int run_if,
                                     double* dout, hipStream_t st) {
  hipLaunchKernelGGL((engine_kernel<T, WG, APT>), dim3(grid), dim3(WG), lds, st, probs, items,
                     wg_off, mode, flag, run_if, dout);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_engine(EngineCfg cfg, int grid, size_t lds, const Problem* probs, const Item* items,
                         const int* wg_off, int mode, const int* flag, int run_if, double* dout,
                         hipStream_t st) {
#define PCV_CASE(W, P)                                                                        \
  if (cfg.wg == W && cfg.apt == P)                                                            \
    return launch_engine_inst<T, W, P>(grid, lds, probs, items, wg_off, mode, flag, run_if,  \
                                       dout, st);
  if constexpr (sizeof(T) == 8) { PCV_ENGINE_CASES_F64(PCV_CASE) }
  else { PCV_ENGINE_CASES_F32(PCV_CASE) }
#undef PCV_CASE
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_merge_exact(const Problem* probs, Outs outs, int n_prob, int max_n_pad,
                              const int* flag, int run_if, hipStream_t st, bool rounded) {
  dim3 grid((max_n_pad + 63) / 64, 3, n_prob);
  hipLaunchKernelGGL((merge_exact_kernel<T>), grid, dim3(256), 0, st, probs, outs, flag, run_if);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !rounded) return e;
  hipLaunchKernelGGL(sz_correct_kernel, dim3(n_prob), dim3(64), 0, st, probs, outs, flag, run_if);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_merge_close(const Problem* prob, int n_pad, Outs outs, CloseArgs ca, double* gtmp,
                              hipStream_t st, const Problem* prob_exact, bool one_pass) {
  const int tiles = (n_pad + 63) / 64;
  const int fuse = one_pass ? 2 : (n_pad <= kCloseFuseMaxPad ? 1 : 0);
  if (one_pass)
    hipLaunchKernelGGL((merge_close_beta_kernel<T, kOnePassThreads>), dim3(tiles, 3), dim3(kOnePassThreads), 0, st,
                       prob, ca, gtmp, prob_exact, outs, fuse);
  else
    hipLaunchKernelGGL((merge_close_beta_kernel<T, kBetaThreads>), dim3(tiles, 3), dim3(kBetaThreads), 0, st, prob,
                       ca, gtmp, prob_exact, outs, fuse);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || fuse) return e;
  hipLaunchKernelGGL((merge_close_final_kernel<T>), dim3(1), dim3(256), 0, st, prob, outs, ca, gtmp, tiles,
                     prob_exact);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t st) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_count(long long* c, int which, long long add, hipStream_t st) {
  hipLaunchKernelGGL(count_kernel, dim3(1), dim3(1), 0, st, c, which, add);
  return hipGetLastError();
}

#define PCV_INST(T)                                                                                  \
  template hipError_t launch_load_landmarks<T>(const T*, T*, double*, double*, const double*, int, \
                                               int, int, hipStream_t);                             \
  template hipError_t launch_pair_msd<T>(const T*, const double*, const double*, const double*,    \
                                         int, int, int, double*, hipStream_t);                     \
  template hipError_t launch_prep<T>(const PrepArgs*, const void*, int, int, hipStream_t);              \
  template hipError_t launch_prep_close<T>(PrepArgs, const void*, CloseArgs, Outs, hipStream_t);   \
  template hipError_t launch_engine<T>(EngineCfg, int, size_t, const Problem*, const Item*,        \
                                       const int*, int, const int*, int, double*, hipStream_t);    \
  template hipError_t launch_merge_exact<T>(const Problem*, Outs, int, int, const int*, int,       \
                                            hipStream_t, bool);                                    \
  template hipError_t launch_merge_close<T>(const Problem*, int, Outs, CloseArgs, double*, hipStream_t, \
                                            const Problem*, bool);
PCV_INST(float)
PCV_INST(double)

}  // namespace pcv
