// Multi-landmark streaming engine for mid-size FP32 structures on gfx950
// (up to 2048 padded atoms, 8 blocks of 256).
//
// A step covers K landmarks at once.  Its work is cut into units
// u = k * nblk + b (landmark lane k < K, atom block b < nblk); worker wave w
// of the seven owns the units w, w + 7, w + 14 (at most SPW), so with
// K = floor(7 SPW / nblk) nearly every worker slot carries a block in every
// step, whatever the structure size.  Per step:
//
//   * workers: each owned unit's block arrives through the wave's private
//     LDS copy ring (global_load_lds_dwordx4, partial vmcnt waits), is read
//     into registers once, and is contracted with the shared FP32 copy of
//     w_j x_c,j in LDS into the unit's correlation sums (FP64), reduced over
//     the wave with DPP moves;
//   * one LDS-only barrier;
//   * solver wave: lane k adds the nblk unit sums of landmark k, solves its
//     quaternion eigenproblem (Section 3; K independent solves side by
//     side), and the K distances join the running log-sum-exp (Eq. 2) with
//     one wave minimum; every lane keeps its own Z, S sums against the
//     common running minimum, so no other cross-lane reduction is needed
//     until the item ends;
//   * workers, after the barrier, add the gradient terms of the previous
//     step from the registers they kept, U += e (q - q0) R (a - c) (FP32)
//     and V += e R (a - c) (FP64), and go on to contract the next step.
//
// With K > 1 several workers accumulate the same atoms (for different
// landmark lanes); each worker then writes its own partial (sub-slot w of the
// item, zero where it owns none of a block), and the merge kernels add the
// sub-slots like any other partials.  With K = 1 every block has one owner
// and the item writes a single partial.  Results do not depend on timing:
// every sum is taken in a fixed order.
#include "pcv_internal.h"
#include "pcv_math.h"
#include "pcv_stream.h"

namespace pcv {

namespace {

constexpr int kWG4 = 512;
constexpr int kW4 = 7;                 // worker waves
constexpr int kBlk4 = 256;             // atoms per block: 64 lanes x 4
constexpr int kBF4 = 3 * kBlk4;        // floats of one block of one landmark
constexpr int kMaxBlk4 = 8;            // blocks of the shared structure copy
constexpr int kMaxUnits4 = kW4 * 3;    // units per step (SPW <= 3)
constexpr int kRing4 = 6;              // copy-ring slots per worker wave
constexpr int kRes4 = 16;              // doubles per landmark result: R[9], al, e, -, c[3], -

static_assert(kW4 * kRing4 * kBF4 * 4 + kMaxBlk4 * kBF4 * 4 +
                  (2 * kMaxUnits4 * 10 + 2 * kMaxUnits4 * kRes4 + 2 + 16) * 8 <= 160 * 1024,
              "engine 4 LDS budget");

__shared__ double e4_part[2][kMaxUnits4][10];      // unit correlation sums (row padded to 80 B)
__shared__ double e4_res[2][kMaxUnits4][kRes4];    // per landmark lane
__shared__ double e4_sc[2];                        // rescale factor of the step
__shared__ double e4_misc[16];                     // item totals

__device__ __forceinline__ double clamp0_4(double v) { return v < 0.0 ? 0.0 : v; }

__device__ __forceinline__ unsigned lds_addr(const float* p) {
  return (unsigned)(size_t)((const __attribute__((address_space(3))) float*)p);
}

struct E4Item {
  const Problem* P;
  int i0, nL, slot, n_pad, nblk, K, R;
  double lam, q0;
};

// ------------------------------------------------------------------ worker
// ring: this wave's copy ring; xs: the workgroup's FP32 copy of w_j x_c,j
// (nblk blocks, x/y/z planes of 256 atoms each).
template <int SPW>
__device__ __forceinline__ void e4_worker(const E4Item& c, int w, int lane, float* ring, float* xs) {
  constexpr int RS = kRing4;
  const int n_pad = c.n_pad, nblk = c.nblk, K = c.K, nL = c.nL;
  const int T = (nL + K - 1) / K;
  const int ufull = K * nblk;
  int uk[SPW], ub[SPW];   // landmark lane and block of slot s (wave-uniform)
#pragma unroll
  for (int s = 0; s < SPW; ++s) {
    const int u = w + kW4 * s;
    uk[s] = u / nblk;
    ub[s] = u - uk[s] * nblk;
  }
  // Owned slots active in step t: a prefix s < nact(t).
  auto nact = [&](int t) {
    const int lim = min(K, nL - t * K) * nblk;
    int a = 0;
#pragma unroll
    for (int s = 0; s < SPW; ++s) a += (w + kW4 * s < lim) ? 1 : 0;
    return a;
  };
  const int na_full = T > 0 ? nact(0) : 0;
  const int NB = T > 0 ? (T - 1) * na_full + nact(T - 1) : 0;   // blocks this wave streams
  const float* A = (const float*)c.P->A;

  // Shared structure copy: worker w stages blocks w and w + 7 (through
  // registers), then every wave meets at a barrier before any copy starts.
  {
    const int n_x = c.P->n_x;
    const float* xsrc = c.P->xw32;
    for (int b = w; b < nblk; b += kW4) {
      const int j0 = b * kBlk4 + lane * 4;
      f4v xv[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) xv[d] = ldg(reinterpret_cast<const f4v*>(xsrc + (size_t)d * n_x + j0));
#pragma unroll
      for (int d = 0; d < 3; ++d) *reinterpret_cast<f4v*>(xs + (b * 3 + d) * kBlk4 + lane * 4) = xv[d];
    }
  }
  bar_lds();

  // Copy stream: the owned active units in (step, slot) order.  Lanes past
  // the structure copy nothing (their ring bytes are zeroed after reading).
  int it_t = 0, it_s = 0, it_na = na_full, it_slot = 0, issued = 0;
  auto issue_next = [&]() {
    const int k = (it_s == 0) ? uk[0] : ((it_s == 1) ? uk[SPW > 1 ? 1 : 0] : uk[SPW - 1]);
    const int b = (it_s == 0) ? ub[0] : ((it_s == 1) ? ub[SPW > 1 ? 1 : 0] : ub[SPW - 1]);
    const int j0 = b * kBlk4 + lane * 4;
    const float* src = A + (size_t)(c.i0 + it_t * K + k) * 3 * n_pad + j0;
    float* dst = ring + it_slot * kBF4;
    if (j0 < n_pad) {
#pragma unroll
      for (int d = 0; d < 3; ++d)
        __builtin_amdgcn_global_load_lds((const void*)(src + (size_t)d * n_pad),
                                         (__attribute__((address_space(3))) void*)(dst + d * kBlk4), 16, 0, 0);
    }
    if (++it_s == it_na) {
      it_s = 0;
      ++it_t;
      it_na = (it_t < T) ? nact(it_t) : 0;
    }
    if (++it_slot == RS) it_slot = 0;
    ++issued;
  };
  // The previous item's partial stores count in vmcnt too: let them finish
  // so that the partial waits below count this item's copies only.
  wait_vm(0);
  for (int b = 0; b < RS && b < NB; ++b) issue_next();

  float U[SPW][3][4];
  double V[SPW][3][4];
#pragma unroll
  for (int s = 0; s < SPW; ++s)
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int e = 0; e < 4; ++e) { U[s][d][e] = 0.f; V[s][d][e] = 0.0; }

  float a0[SPW][3][4], a1[SPW][3][4];
  int rd_slot = 0, consumed = 0;
  const unsigned ring_addr = lds_addr(ring) + lane * 16;
  const unsigned xs_addr = lds_addr(xs) + lane * 16;

  // Step t: contract the owned units of step t into `cur` (phase A), then the
  // gradient of step t - 1 from `prev` (phase B).
  auto step = [&](int t, float (&cur)[SPW][3][4], float (&prev)[SPW][3][4]) {
    if (t < T) {
      const int lim = min(K, nL - t * K) * nblk;
#pragma unroll
      for (int s = 0; s < SPW; ++s) {
        if (w + kW4 * s < lim) {
          wait_vm(3 * (issued - consumed - 1));
          f4v p0, p1, p2;
          read_block<0>(ring_addr + (unsigned)(rd_slot * kBF4 * 4), p0, p1, p2);
          ++consumed;
          if (++rd_slot == RS) rd_slot = 0;
          if (issued < NB) issue_next();
          f4v x0, x1, x2;
          read_block<0>(xs_addr + (unsigned)(ub[s] * kBF4 * 4), x0, x1, x2);
          const bool in = ub[s] * kBlk4 + lane * 4 < n_pad;
          double M[9];
#pragma unroll
          for (int q = 0; q < 9; ++q) M[q] = 0.0;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float c0 = in ? p0[e] : 0.f, c1 = in ? p1[e] : 0.f, c2 = in ? p2[e] : 0.f;
            cur[s][0][e] = c0; cur[s][1][e] = c1; cur[s][2][e] = c2;
            const double y0 = x0[e], y1 = x1[e], y2 = x2[e];
            const double b0 = c0, b1 = c1, b2 = c2;
            M[0] = fma(b0, y0, M[0]); M[1] = fma(b0, y1, M[1]); M[2] = fma(b0, y2, M[2]);
            M[3] = fma(b1, y0, M[3]); M[4] = fma(b1, y1, M[4]); M[5] = fma(b1, y2, M[5]);
            M[6] = fma(b2, y0, M[6]); M[7] = fma(b2, y1, M[7]); M[8] = fma(b2, y2, M[8]);
          }
#pragma unroll
          for (int q = 0; q < 9; ++q) M[q] = wave_sum_to63(M[q]);
          if (lane == 63) {
            double* pp = e4_part[t & 1][w + kW4 * s];
#pragma unroll
            for (int q = 0; q < 9; ++q) pp[q] = M[q];
          }
        }
      }
    }
    bar_lds();
    if (t >= 1) {
      const int tp = t - 1;
      const int limp = min(K, nL - tp * K) * nblk;
      const double sc = e4_sc[tp & 1];
      if (sc != 1.0) {
        const float scf = (float)sc;
#pragma unroll
        for (int s = 0; s < SPW; ++s)
#pragma unroll
          for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int e = 0; e < 4; ++e) { U[s][d][e] *= scf; V[s][d][e] *= sc; }
      }
#pragma unroll
      for (int s = 0; s < SPW; ++s) {
        if (w + kW4 * s < limp) {
          const double* rs = e4_res[tp & 1][uk[s]];
          float Rt[9];
#pragma unroll
          for (int q = 0; q < 9; ++q) Rt[q] = (float)rs[q];
          const float alf = (float)rs[9];
          const double be = rs[10];
          const float ch0 = (float)rs[12], ch1 = (float)rs[13], ch2 = (float)rs[14];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float b0 = prev[s][0][e] - ch0, b1 = prev[s][1][e] - ch1, b2 = prev[s][2][e] - ch2;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const float r = fmaf(Rt[d * 3 + 0], b0, fmaf(Rt[d * 3 + 1], b1, Rt[d * 3 + 2] * b2));
              U[s][d][e] = fmaf(alf, r, U[s][d][e]);
              V[s][d][e] = fma(be, (double)r, V[s][d][e]);
            }
          }
        }
      }
    }
  };

  for (int t = 0; t <= T; t += 2) {
    step(t, a0, a1);
    if (t + 1 <= T) step(t + 1, a1, a0);
  }

  bar_lds();   // item totals published by the solver
  double mu[3], mv[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) { mu[d] = e4_misc[3 + d]; mv[d] = e4_misc[6 + d]; }
  // 16-byte stores of a lane's four consecutive atoms (n_pad is a multiple
  // of 64, so a group of four is either wholly inside or wholly past it).
  auto store = [&](int slot, int b, const float (&u)[3][4], const double (&v)[3][4], bool corr) {
    const int j0 = b * kBlk4 + lane * 4;
    if (j0 >= n_pad) return;
    float* pu = partial_u<float>(c.P->vec, slot, n_pad);
    double* pv = partial_v<float>(c.P->vec, slot, n_pad);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double cu = corr ? mu[d] : 0.0, cv = corr ? mv[d] : 0.0;
      f4v u4;
      d2v v01, v23;
#pragma unroll
      for (int e = 0; e < 4; ++e) u4[e] = (float)((double)u[d][e] - cu);
      v01[0] = v[d][0] - cv;
      v01[1] = v[d][1] - cv;
      v23[0] = v[d][2] - cv;
      v23[1] = v[d][3] - cv;
      stg(reinterpret_cast<f4v*>(pu + (size_t)d * n_pad + j0), u4);
      stg(reinterpret_cast<d2v*>(pv + (size_t)d * n_pad + j0), v01);
      stg(reinterpret_cast<d2v*>(pv + (size_t)d * n_pad + j0 + 2), v23);
    }
  };
  if (c.R == 1) {
    // One landmark lane: every block has exactly one owner.
#pragma unroll
    for (int s = 0; s < SPW; ++s)
      if (w + kW4 * s < ufull) store(c.slot, ub[s], U[s], V[s], true);
  } else {
    // Sub-slot w: this worker's sums per block (zero for blocks it does not
    // own); the centroid-residual totals go to sub-slot 0 only.
    for (int b = 0; b < nblk; ++b) {
      float su[3][4];
      double sv[3][4];
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int e = 0; e < 4; ++e) { su[d][e] = 0.f; sv[d][e] = 0.0; }
#pragma unroll
      for (int s = 0; s < SPW; ++s) {
        if (w + kW4 * s < ufull && ub[s] == b) {
#pragma unroll
          for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int e = 0; e < 4; ++e) { su[d][e] += U[s][d][e]; sv[d][e] += V[s][d][e]; }
        }
      }
      store(c.slot + w, b, su, sv, w == 0);
    }
  }
}

// ------------------------------------------------------------------ solver
__device__ __forceinline__ void e4_solver(const E4Item& c, int lane, int mode, double* dout) {
  const Problem& P = *c.P;
  const double lam = c.lam, q0 = c.q0;
  const int nL = c.nL, K = c.K, nblk = c.nblk;
  const int T = (nL + K - 1) / K;
  bar_lds();   // structure copy staged by the workers
  const double Gxx = ldg(P.Gx32);
  double xres[3], Rx[9];
#pragma unroll
  for (int d = 0; d < 3; ++d) xres[d] = ldg(P.xres + d);
#pragma unroll
  for (int k = 0; k < 9; ++k) Rx[k] = (mode == MODE_APPROX) ? ldg(P.Rxy + k) : 0.0;
  double m = INFINITY;
  // Per-lane sums (landmark lane = lane) against the common running minimum.
  double Z = 0.0, S = 0.0, tU[3] = {0.0, 0.0, 0.0}, tV[3] = {0.0, 0.0, 0.0};
  // Per-landmark inputs of lane k, fetched one step ahead of use (lanes past
  // the step read landmark i0, in bounds, and stay inactive).
  auto fetch = [&](int t, double cap[3], double& Ga, double& qi, double Rs[9]) {
    const int off = t * K + lane;
    const int i = c.i0 + ((lane < K && off < nL) ? off : 0);
#pragma unroll
    for (int d = 0; d < 3; ++d) cap[d] = ldg(P.ca + (size_t)i * 3 + d);
    Ga = ldg(P.Ga + i);
    qi = ldg(P.q + i);
#pragma unroll
    for (int k = 0; k < 9; ++k) Rs[k] = (mode == MODE_APPROX) ? ldg(P.Rsave + (size_t)i * 9 + k) : 0.0;
  };
  double cap[3], Ga = 0.0, qi = 0.0, Rs[9];
  if (T > 0) fetch(0, cap, Ga, qi, Rs);
  for (int t = 0; t <= T; ++t) {
    bar_lds();
    if (t < T) {
      const int Kt = min(K, nL - t * K);
      const bool act = lane < Kt;
      const int i = c.i0 + t * K + lane;
      const double cc[3] = {cap[0], cap[1], cap[2]};
      const double Gai = Ga, qv = qi;
      double Rsv[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) Rsv[k] = Rs[k];
      if (t + 1 < T) fetch(t + 1, cap, Ga, qi, Rs);
      double D = INFINITY, R[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) R[k] = 0.0;
      if (act) {
        // Correlation of landmark lane k: its nblk unit sums in block order.
        double Mc[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) Mc[q] = 0.0;
        for (int b = 0; b < nblk; ++b) {
          const double* pp = e4_part[t & 1][lane * nblk + b];
#pragma unroll
          for (int q = 0; q < 9; ++q) Mc[q] += pp[q];
        }
        // The workers used w_j x_j rounded to FP32, whose sum (xres) is not
        // exactly zero; remove its coupling to the landmark centroid.
#pragma unroll
        for (int r0 = 0; r0 < 3; ++r0)
#pragma unroll
          for (int c0 = 0; c0 < 3; ++c0) Mc[r0 * 3 + c0] = fma(-cc[r0], xres[c0], Mc[r0 * 3 + c0]);
        if (mode == MODE_APPROX) {
          double tr = 0.0;
#pragma unroll
          for (int r0 = 0; r0 < 3; ++r0)
#pragma unroll
            for (int c0 = 0; c0 < 3; ++c0) {
              const double rt = Rx[c0 * 3 + 0] * Rsv[0 * 3 + r0] + Rx[c0 * 3 + 1] * Rsv[1 * 3 + r0] +
                                Rx[c0 * 3 + 2] * Rsv[2 * 3 + r0];
              tr = fma(rt, Mc[r0 * 3 + c0], tr);
            }
          D = clamp0_4(Gxx + Gai - 2.0 * tr);
#pragma unroll
          for (int k = 0; k < 9; ++k) R[k] = Rsv[k];
        } else {
          double F[10], lmax, qq[4];
          const int fb = top_eigenpair(Mc, 0.5 * (Gxx + Gai), F, lmax, qq);
          if (fb && P.fallbacks) atomicAdd((unsigned long long*)P.fallbacks, 1ull);
          D = clamp0_4(Gxx + Gai - 2.0 * lmax);
          quat_to_rot(qq, R);
          if (mode == MODE_EXACT_SAVE) {
#pragma unroll
            for (int k = 0; k < 9; ++k) stg(P.Rsave + (size_t)i * 9 + k, R[k]);
          }
        }
        if (dout != nullptr) stg(dout + i, D);
      }
      // Step minimum over the landmark lanes (inactive lanes hold +inf).
      const double rm = row_min16(D);
      const double mb = fmin(fmin(__shfl(rm, 0, 64), __shfl(rm, 16, 64)), fmin(__shfl(rm, 32, 64), __shfl(rm, 48, 64)));
      const double mn = fmin(m, mb);
      const double sc = (m == INFINITY) ? 0.0 : ((mn == m) ? 1.0 : exp(-lam * (m - mn)));
      const double e = act ? exp(-lam * (D - mn)) : 0.0;
      const double al = e * (qv - q0);
      Z = Z * sc + e;
      S = S * sc + e * qv;
      // Residual of the centroid split the workers use (c - (float)c).
      const double c3[3] = {cc[0] - (double)(float)cc[0], cc[1] - (double)(float)cc[1],
                            cc[2] - (double)(float)cc[2]};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double rc = R[d * 3 + 0] * c3[0] + R[d * 3 + 1] * c3[1] + R[d * 3 + 2] * c3[2];
        tU[d] = tU[d] * sc + al * rc;
        tV[d] = tV[d] * sc + e * rc;
      }
      m = mn;
      if (act) {
        double* r = e4_res[t & 1][lane];
#pragma unroll
        for (int q = 0; q < 9; ++q) r[q] = R[q];
        r[9] = al;
        r[10] = e;
#pragma unroll
        for (int d = 0; d < 3; ++d) r[12 + d] = cc[d];
      }
      if (lane == 0) e4_sc[t & 1] = sc;
    }
  }
  // Item totals: the per-lane sums added over the wave in a fixed order.
  Z = wave_sum_to63(Z);
  S = wave_sum_to63(S);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    tU[d] = wave_sum_to63(tU[d]);
    tV[d] = wave_sum_to63(tV[d]);
  }
  if (lane == 63) {
    e4_misc[0] = m;
    e4_misc[1] = Z;
    e4_misc[2] = S;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      e4_misc[3 + d] = tU[d];
      e4_misc[6 + d] = tV[d];
    }
  }
  const double Zt = __shfl(Z, 63, 64), St = __shfl(S, 63, 64);   // all lanes active here
  if (lane < c.R) {
    double* h = P.hdr + (size_t)(c.slot + lane) * 4;
    stg(h + 0, m);
    stg(h + 1, lane == 0 ? Zt : 0.0);
    stg(h + 2, lane == 0 ? St : 0.0);
    stg(h + 3, q0);
  }
  bar_lds();
}

}  // namespace

template <int SPW>
__global__ __launch_bounds__(kWG4) void engine4_kernel(const Problem* __restrict__ probs,
                                                       const Item* __restrict__ items,
                                                       const int* __restrict__ wg_off, int mode,
                                                       const int* __restrict__ flag, int run_if,
                                                       double* __restrict__ dout) {
  __shared__ float ring[kW4 * kRing4 * kBF4];
  __shared__ float xs[kMaxBlk4 * kBF4];
  if (flag != nullptr && *flag != run_if) return;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int it_end = wg_off[blockIdx.x + 1];
  for (int it = wg_off[blockIdx.x]; it < it_end; ++it) {
    const Item item = items[it];
    E4Item c;
    c.P = probs + item.prob;
    c.i0 = item.i0;
    c.nL = item.i1 - item.i0;
    c.slot = item.slot;
    c.n_pad = c.P->n_pad;
    c.nblk = (c.n_pad + kBlk4 - 1) / kBlk4;
    c.K = c.P->bsz;
    c.R = e4_subslots(c.K);
    c.lam = c.P->lam;
    c.q0 = c.P->q[item.i0];
    // Shapes the host planner never produces are skipped by every wave alike.
    if (c.nL < 1 || c.nblk > kMaxBlk4 || c.K < 1 || c.K * c.nblk > kW4 * SPW) continue;
    if (wave < kW4) e4_worker<SPW>(c, wave, lane, ring + wave * kRing4 * kBF4, xs);
    else e4_solver(c, lane, mode, dout);
    bar_lds();   // LDS is reused by the next item
  }
}

int engine4_lanes(int n_pad, int spw) {
  const int nblk = (n_pad + kBlk4 - 1) / kBlk4;
  if (nblk < 1 || nblk > kMaxBlk4 || spw < 2 || spw > 3) return 0;
  return (kW4 * spw) / nblk;
}

template <>
hipError_t launch_engine4<float>(int spw, int grid, const Problem* probs, const Item* items, const int* wg_off,
                                 int mode, const int* flag, int run_if, double* dout, hipStream_t st) {
  switch (spw) {
    case 2: hipLaunchKernelGGL(engine4_kernel<2>, dim3(grid), dim3(kWG4), 0, st, probs, items, wg_off, mode, flag,
                               run_if, dout); break;
    case 3: hipLaunchKernelGGL(engine4_kernel<3>, dim3(grid), dim3(kWG4), 0, st, probs, items, wg_off, mode, flag,
                               run_if, dout); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t launch_engine4<double>(int, int, const Problem*, const Item*, const int*, int, const int*, int, double*,
                                  hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace pcv
