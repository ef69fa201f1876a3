// Split-role landmark streaming engine for gfx950.
//
// One workgroup of 512 threads = 8 waves with three roles that form a
// three-stage pipeline over batches of B landmarks (one barrier per step):
//
//   wave 0      solver: per landmark of the batch one lane sums the
//               correlation partials, solves the quaternion eigenproblem in
//               FP64 (exact modes) or composes R_xy R_{a_i y} (approximate
//               mode), and folds the batch into the running log-sum-exp
//               (m, Z, S); it publishes R_i, e_i (q_i - q0), e_i and the
//               rescale factor of the batch through LDS.
//   correlation waves (3, or 2 for large structures): async copies (global_load_lds_dwordx4) bring the
//               next batch of landmarks from HBM into an LDS double buffer
//               while the current batch is contracted with the centred,
//               weighted structure held in registers, M = sum_j a_j (w_j x_j)^T
//               in FP64; groups of g lanes share one landmark and reduce
//               inside the wave.
//   gradient waves (the rest): every lane owns atoms j = lane + 64 NGW k and keeps
//               U = sum_i e_i (q_i - q0) r_i (FP32) and V = sum_i e_i r_i
//               (FP64) for the rotated centred landmarks r_i = R_i (a_i - c_i),
//               re-reading the landmark coordinates of two batches ago
//               (recently streamed, so served by the caches).
//
// Step t: correlation of batch t | solve of batch t-1 | gradient of batch t-2.
// The solver's FP64 eigen code lives in its own branch, so its registers do
// not add to the gradient waves' per-atom state.  Each work item (a landmark
// range of one problem) writes one partial (m, Z, S, q0, U, V) in the same
// format as engine_kernel, so the merge kernels are shared.
#include "pcv_internal.h"
#include "pcv_math.h"
#include "pcv_stream.h"

namespace pcv {

namespace {

template <typename T> struct Part2 { using type = float; };
template <> struct Part2<double> { using type = double; };
template <typename T> struct UAcc { using type = float; };
template <> struct UAcc<double> { using type = double; };

constexpr int kWG2 = 512;
constexpr int kRes = 13;    // doubles per landmark result: R[9], al, be, sc, dq

__device__ __forceinline__ double clamp0_2(double v) { return v < 0.0 ? 0.0 : v; }
__device__ __forceinline__ double scale2(double m_from, double m_to, double lam) {
  return (m_from == INFINITY) ? 0.0 : exp(-lam * (m_from - m_to));
}

template <int NV>
__device__ __forceinline__ void xor_sum(double v[NV], int width) {
  for (int off = width >> 1; off > 0; off >>= 1) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], off, 64);
  }
}

}  // namespace

// LDS layout (bytes from the dynamic shared base):
//   [0, 2*lbuf)                 landmark double buffer
//   part: 2 x bmax x 3 x 9      correlation partials (doubles)
//   res:  3 x bmax x kRes       solver results (doubles)
//   misc: 16                    item totals (m, Z, S, centroid-residual sums)
size_t engine2_lds_bytes(size_t lbuf, int bmax) {
  return 2 * lbuf + (size_t)(2 * bmax * 3 * 9 + 3 * bmax * kRes + 16) * sizeof(double);
}

// Per-item context shared by the three roles.
template <typename T>
struct E2Item {
  const Problem* P;
  int i0, i1, slot, n_pad, B, g, nb;
  double lam, q0;
  size_t lm_elems;     // elements of one landmark (3 n_pad)
  const T* A;
  char* lbase;
  double* part;
  double* res;
  double* misc;
  int lbuf_bytes, bmax, mode;
  double* dout;
};

// Async copy of batch b (contiguous landmarks) into its LDS buffer: 1 KiB per
// wave instruction (16 B per lane), then 256 B pieces for the tail (a
// landmark is 12 n_pad or 24 n_pad bytes with n_pad a multiple of 64).
template <typename T, int NCW>
__device__ __forceinline__ void e2_issue(const E2Item<T>& c, int b, int cw, int lane) {
  const int i0 = c.i0 + b * c.B;
  const int cnt = min(c.B, c.i1 - i0);
  const size_t bytes = (size_t)cnt * c.lm_elems * sizeof(T);
  const int chunks = (int)(bytes / 1024);
  const int tails = (int)((bytes - (size_t)chunks * 1024) / 256);
  const char* src = reinterpret_cast<const char*>(c.A + (size_t)i0 * c.lm_elems);
  char* dst = c.lbase + (size_t)(b & 1) * c.lbuf_bytes;
  for (int ch = cw; ch < chunks; ch += NCW)
    __builtin_amdgcn_global_load_lds((const void*)(src + (size_t)ch * 1024 + lane * 16),
                                     (__attribute__((address_space(3))) void*)(dst + (size_t)ch * 1024), 16, 0,
                                     kStreamPolicy);
  for (int tc = cw; tc < tails; tc += NCW) {
    const size_t off = (size_t)chunks * 1024 + (size_t)tc * 256;
    __builtin_amdgcn_global_load_lds((const void*)(src + off + lane * 4),
                                     (__attribute__((address_space(3))) void*)(dst + off), 4, 0, kStreamPolicy);
  }
}

// Correlation waves: nb + 3 pipeline steps (one barrier each) + 1 item-end barrier.
// Opaque copy of a lane index: keeps the compiler from hoisting a role's
// per-atom address arithmetic into the shared kernel prologue, where the
// address registers of all three roles would be live at the same time.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Same for a register-resident value: its conversions are redone where it is
// used instead of being hoisted (and kept live) as loop invariants.
template <typename T>
__device__ __forceinline__ T pin(T v) {
  asm volatile("" : "+v"(v));
  return v;
}

template <typename T, int NCW, int APTC>
__device__ __forceinline__ void e2_corr(const E2Item<T>& c, int cw, int lane_in) {
  const int lane = opaque(lane_in);
  const int g = c.g, n_pad = c.n_pad;
  const int cidx = cw * 64 + lane;
  const int grp = cidx / g, lg = cidx - grp * g;
  const int ngrp = (NCW * 64) / g;
  T xw[3][APTC];
  for (int t = -1; t < c.nb + 2; ++t) {
    if (t < 0) {
      const double* xwp = c.P->xw;
#pragma unroll
      for (int k = 0; k < APTC; ++k) {
        const int j = lg + g * k;
        const bool in = j < n_pad;
#pragma unroll
        for (int d = 0; d < 3; ++d) xw[d][k] = in ? (T)ldg(xwp + (size_t)d * n_pad + j) : T(0);
      }
      e2_issue<T, NCW>(c, 0, cw, lane);
    } else {
      if (t + 1 < c.nb) e2_issue<T, NCW>(c, t + 1, cw, lane);
      if (t < c.nb) {
        const int i0 = c.i0 + t * c.B;
        const int cnt = min(c.B, c.i1 - i0);
        const T* lb = reinterpret_cast<const T*>(c.lbase + (size_t)(t & 1) * c.lbuf_bytes);
        double* pt = c.part + (size_t)(t & 1) * c.bmax * 3 * 9;
        const int rounds = (c.B + ngrp - 1) / ngrp;
        for (int rr = 0; rr < rounds; ++rr) {
          const int b = rr * ngrp + grp;
          const bool act = b < cnt;
          double M[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) M[k] = 0.0;
          if (act) {
            const T* la = lb + (size_t)b * c.lm_elems;
            const int lgo = opaque(lg);   // per-landmark address arithmetic, not hoisted
            constexpr int kCC = 4;
#pragma unroll
            for (int k0 = 0; k0 < APTC; k0 += kCC) {
#pragma unroll
              for (int k = k0; k < (k0 + kCC < APTC ? k0 + kCC : APTC); ++k) {
                const int j = lgo + g * k;
                if (j < n_pad) {
                  const double a0 = (double)la[j], a1 = (double)la[n_pad + j], a2 = (double)la[2 * n_pad + j];
                  const double x0 = (double)pin(xw[0][k]), x1 = (double)pin(xw[1][k]), x2 = (double)pin(xw[2][k]);
                  M[0] = fma(a0, x0, M[0]); M[1] = fma(a0, x1, M[1]); M[2] = fma(a0, x2, M[2]);
                  M[3] = fma(a1, x0, M[3]); M[4] = fma(a1, x1, M[4]); M[5] = fma(a1, x2, M[5]);
                  M[6] = fma(a2, x0, M[6]); M[7] = fma(a2, x1, M[7]); M[8] = fma(a2, x2, M[8]);
                }
              }
              __builtin_amdgcn_sched_barrier(0);
            }
          }
          xor_sum<9>(M, g < 64 ? g : 64);
          if (act) {
            if (g <= 64) {
              if (lg == 0) {
#pragma unroll
                for (int k = 0; k < 9; ++k) pt[((size_t)b * 3 + 0) * 9 + k] = M[k];
              }
            } else if (lane == 0) {
#pragma unroll
              for (int k = 0; k < 9; ++k) pt[((size_t)b * 3 + cw) * 9 + k] = M[k];
            }
          }
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  __syncthreads();
}

// Solver wave: nb + 3 pipeline steps + 1 item-end barrier.
template <typename T, int NCW>
__device__ __forceinline__ void e2_solve(const E2Item<T>& c, int lane_in) {
  const int lane = opaque(lane_in);
  const Problem& P = *c.P;
  const double lam = c.lam;
  // Reference property of U = sum e (q - q0) r: the property of the running
  // minimum's landmark (keeps U small where the weights are large).
  double q0 = c.q0;
  double m = INFINITY, Z = 0.0, S = 0.0, tU[3] = {0.0, 0.0, 0.0}, tV[3] = {0.0, 0.0, 0.0};
  for (int t = -1; t < c.nb + 2; ++t) {
    const int tb = t - 1;
    if (tb >= 0 && tb < c.nb) {
      const int i0 = c.i0 + tb * c.B;
      const int cnt = min(c.B, c.i1 - i0);
      const double* pt = c.part + (size_t)(tb & 1) * c.bmax * 3 * 9;
      double* rs = c.res + (size_t)(tb % 3) * c.bmax * kRes;
      const double Gxx = ldg(P.Gx32);
      const int np = (c.g <= 64) ? 1 : NCW;
      for (int b0 = 0; b0 < cnt; b0 += 64) {
        const int b = b0 + lane;
        const bool act = b < cnt;
        // Lanes beyond the batch take part in the wave reductions with D = +inf.
        double D = INFINITY, R[9], qi = 0.0, c3[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 9; ++k) R[k] = 0.0;
        if (act) {
          const int i = i0 + b;
          double Mc[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) Mc[k] = pt[((size_t)b * 3 + 0) * 9 + k];
          double cap[3], xr[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            cap[d] = ldg(P.ca + (size_t)i * 3 + d);
            xr[d] = ldg(P.xres + d);
          }
          for (int p = 1; p < np; ++p)
#pragma unroll
            for (int k = 0; k < 9; ++k) Mc[k] += pt[((size_t)b * 3 + p) * 9 + k];
          // The correlation used w_j x_j rounded to T, whose sum (xres) is not
          // exactly zero; remove its coupling to the landmark centroid.
#pragma unroll
          for (int r0 = 0; r0 < 3; ++r0)
#pragma unroll
            for (int c0 = 0; c0 < 3; ++c0) Mc[r0 * 3 + c0] = fma(-cap[r0], xr[c0], Mc[r0 * 3 + c0]);
          const double Ga = ldg(P.Ga + i);
          if (c.mode == MODE_APPROX) {
            double Rs[9], Rx[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
              Rs[k] = ldg(P.Rsave + (size_t)i * 9 + k);
              Rx[k] = ldg(P.Rxy + k);
            }
            double tr = 0.0;
#pragma unroll
            for (int r0 = 0; r0 < 3; ++r0)
#pragma unroll
              for (int c0 = 0; c0 < 3; ++c0) {
                const double rt = Rx[c0 * 3 + 0] * Rs[0 * 3 + r0] + Rx[c0 * 3 + 1] * Rs[1 * 3 + r0] +
                                  Rx[c0 * 3 + 2] * Rs[2 * 3 + r0];
                tr = fma(rt, Mc[r0 * 3 + c0], tr);
              }
            D = clamp0_2(Gxx + Ga - 2.0 * tr);
#pragma unroll
            for (int k = 0; k < 9; ++k) R[k] = Rs[k];
          } else {
            double F[10], lmax, qv[4];
            const int fb = top_eigenpair(Mc, 0.5 * (Gxx + Ga), F, lmax, qv);
            if (fb && P.fallbacks) atomicAdd((unsigned long long*)P.fallbacks, 1ull);
            D = clamp0_2(Gxx + Ga - 2.0 * lmax);
            quat_to_rot(qv, R);
            if (c.mode == MODE_EXACT_SAVE) {
#pragma unroll
              for (int k = 0; k < 9; ++k) stg(P.Rsave + (size_t)i * 9 + k, R[k]);
            }
          }
          if (c.dout != nullptr) stg(c.dout + i, D);
          qi = ldg(P.q + i);
          // residual of the centroid split used by the gradient waves: c - (T)c
#pragma unroll
          for (int d = 0; d < 3; ++d) c3[d] = cap[d] - (double)(T)cap[d];
        }
        double mb = act ? D : INFINITY;
        for (int off = 32; off > 0; off >>= 1) mb = fmin(mb, __shfl_xor(mb, off, 64));
        const double mn = fmin(m, mb);
        const double sc = scale2(m, mn, lam);
        double dq = 0.0;
        if (mn < m) {
          const unsigned long long hit = __ballot(act && D == mb);
          const int src = hit ? __ffsll((long long)hit) - 1 : 0;   // lowest lane holding the minimum
          const double qn = __shfl(qi, src, 64);
          dq = q0 - qn;
          q0 = qn;
        }
        const double e = act ? exp(-lam * (D - mn)) : 0.0;
        const double al = e * (qi - q0);
        double sums[8];
        sums[0] = e;
        sums[1] = e * qi;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double rc = R[d * 3 + 0] * c3[0] + R[d * 3 + 1] * c3[1] + R[d * 3 + 2] * c3[2];
          sums[2 + d] = al * rc;
          sums[5 + d] = e * rc;
        }
        xor_sum<8>(sums, 64);
        Z = Z * sc + sums[0];
        S = S * sc + sums[1];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          tU[d] = fma(dq, tV[d], tU[d]) * sc + sums[2 + d];
          tV[d] = tV[d] * sc + sums[5 + d];
        }
        m = mn;
        if (act) {
          double* r = rs + (size_t)b * kRes;
#pragma unroll
          for (int k = 0; k < 9; ++k) r[k] = R[k];
          r[9] = al;
          r[10] = e;
          r[11] = (b == b0) ? sc : 1.0;   // rescale once, before the sub-batch's first landmark
          r[12] = (b == b0) ? dq : 0.0;
        }
      }
    }
    __syncthreads();
  }
  if (lane == 0) {
    c.misc[0] = m;
    c.misc[1] = Z;
    c.misc[2] = S;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      c.misc[3 + d] = tU[d];
      c.misc[6 + d] = tV[d];
    }
    double* h = P.hdr + (size_t)c.slot * 4;
    stg(h + 0, m);
    stg(h + 1, Z);
    stg(h + 2, S);
    stg(h + 3, q0);
  }
  __syncthreads();
}

// Gradient waves: nb + 3 pipeline steps + 1 item-end barrier, then the partial.
template <typename T, int NGW, int APTG>
__device__ __forceinline__ void e2_grad(const E2Item<T>& c, int gw, int lane_in) {
  const int lane = opaque(lane_in);
  using part_t = typename Part2<T>::type;
  using uacc = typename UAcc<T>::type;
  const int n_pad = c.n_pad;
  constexpr int kGL = 64 * NGW;   // gradient lanes
  const int gidx = gw * 64 + lane;
  uacc U[3][APTG];
  double V[3][APTG];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int k = 0; k < APTG; ++k) { U[d][k] = uacc(0); V[d][k] = 0.0; }
  for (int t = -1; t < c.nb + 2; ++t) {
    const int tb = t - 2;
    if (tb >= 0 && tb < c.nb) {
      const int i0 = c.i0 + tb * c.B;
      const int cnt = min(c.B, c.i1 - i0);
      const double* rs = c.res + (size_t)(tb % 3) * c.bmax * kRes;
      for (int b = 0; b < cnt; ++b) {
        const double* r = rs + (size_t)b * kRes;
        const double sc = r[11];
        if (sc != 1.0) {
          // The running minimum moved: rescale, and move U's reference
          // property with it, U' = U + (q0 - q0') V (V is FP64).
          const double dq = r[12];
#pragma unroll
          for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int k = 0; k < APTG; ++k) {
              const double v = V[d][k];
              U[d][k] = (uacc)(fma(dq, v, (double)U[d][k]) * sc);
              V[d][k] = v * sc;
            }
        }
        // r = R (a - c) in the coordinate type (its rounding is independent
        // per atom and landmark); V accumulates it in FP64.
        T Rt[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) Rt[k] = (T)r[k];
        const double be = r[10];
        const uacc alf = (uacc)r[9];
        const int i = i0 + b;
        const T* la = c.A + (size_t)i * c.lm_elems;
        const double* cap = c.P->ca + (size_t)i * 3;
        const T ch0 = (T)ldg(cap + 0), ch1 = (T)ldg(cap + 1), ch2 = (T)ldg(cap + 2);
        const int gio = opaque(gidx);   // per-landmark address arithmetic, not hoisted
        // All of this lane's atoms of the landmark are loaded before use so
        // their cache round trips overlap.
        T a[3][APTG];
#pragma unroll
        for (int k = 0; k < APTG; ++k) {
          const int j = gio + kGL * k;
          const bool in = j < n_pad;
          a[0][k] = in ? ldg(la + j) : ch0;
          a[1][k] = in ? ldg(la + n_pad + j) : ch1;
          a[2][k] = in ? ldg(la + 2 * n_pad + j) : ch2;
        }
#pragma unroll
        for (int k = 0; k < APTG; ++k) {
          const T a0 = a[0][k] - ch0, a1 = a[1][k] - ch1, a2 = a[2][k] - ch2;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const T rr = fma(Rt[d * 3 + 0], a0, fma(Rt[d * 3 + 1], a1, Rt[d * 3 + 2] * a2));
            U[d][k] = fma(alf, (uacc)rr, U[d][k]);
            V[d][k] = fma(be, (double)rr, V[d][k]);
          }
        }
      }
    }
    __syncthreads();
  }
  __syncthreads();   // item totals published by the solver
  part_t* pu = partial_u<part_t>(c.P->vec, c.slot, n_pad);
  double* pv = partial_v<part_t>(c.P->vec, c.slot, n_pad);
#pragma unroll
  for (int k = 0; k < APTG; ++k) {
    const int j = gidx + kGL * k;
    if (j < n_pad) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        stg(pu + (size_t)d * n_pad + j, (part_t)((double)U[d][k] - c.misc[3 + d]));
        stg(pv + (size_t)d * n_pad + j, V[d][k] - c.misc[6 + d]);
      }
    }
  }
}

template <typename T, int NCW, int APTC, int APTG>
__global__ __launch_bounds__(kWG2) void engine2_kernel(const Problem* __restrict__ probs,
                                                       const Item* __restrict__ items,
                                                       const int* __restrict__ wg_off, int mode,
                                                       const int* __restrict__ flag, int run_if,
                                                       double* __restrict__ dout, int lbuf_bytes, int bmax) {
  {
    const Problem* pr = probs;
    if (!gate_launch(flag, run_if, mode, pr)) return;
    probs = pr;
  }
  extern __shared__ double smem[];
  // The role is uniform per wave (scalar), so each wave runs exactly the
  // barriers of its own role loop; every role executes nb + 4 per item.
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  E2Item<T> c;
  c.lbase = reinterpret_cast<char*>(smem);
  c.part = reinterpret_cast<double*>(c.lbase + 2 * (size_t)lbuf_bytes);
  c.res = c.part + 2 * bmax * 3 * 9;
  c.misc = c.res + 3 * bmax * kRes;
  c.lbuf_bytes = lbuf_bytes;
  c.bmax = bmax;
  c.mode = mode;
  c.dout = dout;
  const int it_end = wg_off[blockIdx.x + 1];
  for (int it = wg_off[blockIdx.x]; it < it_end; ++it) {
    const Item item = items[it];
    c.P = probs + item.prob;
    c.i0 = item.i0;
    c.i1 = item.i1;
    c.slot = item.slot;
    c.n_pad = c.P->n_pad;
    c.B = c.P->bsz;
    c.g = c.P->cg;
    c.nb = (item.i1 - item.i0 + c.B - 1) / c.B;
    c.lam = c.P->lam;
    c.q0 = c.P->q[item.i0];
    c.lm_elems = (size_t)3 * c.n_pad;
    c.A = (const T*)c.P->A;
    if (wave == 0) e2_solve<T, NCW>(c, lane);
    else if (wave <= NCW) e2_corr<T, NCW, APTC>(c, wave - 1, lane);
    else e2_grad<T, 7 - NCW, APTG>(c, wave - 1 - NCW, lane);
    __syncthreads();   // LDS is reused by the next item
  }
}

#define PCV_ENGINE2_CASES_F32(X) X(3, 4, 2) X(3, 8, 4) X(3, 16, 8) X(2, 40, 16)
#define PCV_ENGINE2_CASES_F64(X) X(3, 4, 2) X(3, 8, 4) X(3, 16, 8)

void engine2_configs(bool fp64, int* ncw, int* aptc, int* aptg, int* count) {
  int k = 0;
#define PCV_CASE(W, C, G) { ncw[k] = W; aptc[k] = C; aptg[k] = G; ++k; }
  if (fp64) { PCV_ENGINE2_CASES_F64(PCV_CASE) }
  else { PCV_ENGINE2_CASES_F32(PCV_CASE) }
#undef PCV_CASE
  *count = k;
}

hipError_t engine2_init_attributes() {
  hipError_t e = hipSuccess;
#define PCV_CASE_T(T, W, C, G)                                                                \
  {                                                                                           \
    hipError_t r = hipFuncSetAttribute((const void*)engine2_kernel<T, W, C, G>,              \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024); \
    if (r != hipSuccess) e = r;                                                               \
  }
#define PCV_CASE_F(W, C, G) PCV_CASE_T(float, W, C, G)
#define PCV_CASE_D(W, C, G) PCV_CASE_T(double, W, C, G)
  PCV_ENGINE2_CASES_F32(PCV_CASE_F)
  PCV_ENGINE2_CASES_F64(PCV_CASE_D)
#undef PCV_CASE_F
#undef PCV_CASE_D
#undef PCV_CASE_T
  return e;
}

template <typename T>
hipError_t launch_engine2(int ncw, int aptc, int aptg, int grid, size_t lds, int lbuf_bytes, int bmax,
                          const Problem* probs, const Item* items, const int* wg_off, int mode,
                          const int* flag, int run_if, double* dout, hipStream_t st) {
#define PCV_CASE(W, C, G)                                                                     \
  if (ncw == W && aptc == C && aptg == G) {                                                   \
    hipLaunchKernelGGL((engine2_kernel<T, W, C, G>), dim3(grid), dim3(kWG2), lds, st, probs,  \
                       items, wg_off, mode, flag, run_if, dout, lbuf_bytes, bmax);            \
    return hipGetLastError();                                                                 \
  }
  if constexpr (sizeof(T) == 8) { PCV_ENGINE2_CASES_F64(PCV_CASE) }
  else { PCV_ENGINE2_CASES_F32(PCV_CASE) }
#undef PCV_CASE
  return hipErrorInvalidValue;
}

template hipError_t launch_engine2<float>(int, int, int, int, size_t, int, int, const Problem*, const Item*,
                                          const int*, int, const int*, int, double*, hipStream_t);
template hipError_t launch_engine2<double>(int, int, int, int, size_t, int, int, const Problem*, const Item*,
                                           const int*, int, const int*, int, double*, hipStream_t);

}  // namespace pcv
