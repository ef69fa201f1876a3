// Multi-landmark streaming engine for mid-size FP32 structures on gfx950
// (up to 2048 padded atoms, 8 blocks of 256).
//
// A step covers K landmarks at once.  Its work is cut into units
// u = k * nblk + b (landmark lane k < K, atom block b < nblk); worker wave w
// of the seven owns the run of units w SPW ... w SPW + SPW - 1, so with
// K = floor(7 SPW / nblk) nearly every worker slot carries a block in every
// step, whatever the structure size, and a worker's units of one landmark
// are adjacent (their correlation sums are added before one wave
// reduction).  Per step:
//
//   * workers: each owned unit's block arrives through the wave's private
//     LDS copy ring (global_load_lds_dwordx4, partial vmcnt waits), is read
//     into registers once, and is contracted with the shared FP32 copy of
//     w_j x_c,j in LDS into correlation sums (FP64), reduced over the wave
//     with DPP moves once per landmark the worker touches;
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
// With K > 1 several units accumulate the same atoms (for different
// landmark lanes); at the end of a work item their U and V go through the
// idle copy rings in LDS and are added per block in landmark-lane order, so
// every item writes one partial.  Results do not depend on timing: every sum
// is taken in a fixed order.
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
__shared__ double e4_dq[2];                        // shift of the reference property q0 in the step
__shared__ double e4_misc[16];                     // item totals

static_assert(kMaxUnits4 * kBF4 * 8 <= kW4 * kRing4 * kBF4 * 4, "unit sums (FP64) fit in the copy rings");

__device__ __forceinline__ double clamp0_4(double v) { return v < 0.0 ? 0.0 : v; }

__device__ __forceinline__ unsigned lds_addr(const float* p) {
  return (unsigned)(size_t)((const __attribute__((address_space(3))) float*)p);
}

struct E4Item {
  const Problem* P;
  int i0, nL, slot, n_pad, nblk, K;
  double lam, q0;
};

// ------------------------------------------------------------------ worker
// ring: this wave's copy ring; rings: all seven (reused at the item end);
// xs: the workgroup's FP32 copy of w_j x_c,j (nblk blocks, x/y/z planes of
// 256 atoms each).
template <int SPW>
__device__ __forceinline__ void e4_worker(const E4Item& c, int w, int lane, float* ring, float* rings, float* xs) {
  constexpr int RS = kRing4;
  const int n_pad = c.n_pad, nblk = c.nblk, K = c.K, nL = c.nL;
  const int T = (nL + K - 1) / K;
  const int ufull = K * nblk;
  int uk[SPW], ub[SPW];   // landmark lane and block of slot s (wave-uniform)
#pragma unroll
  for (int s = 0; s < SPW; ++s) {
    const int u = w * SPW + s;
    uk[s] = u / nblk;
    ub[s] = u - uk[s] * nblk;
  }
  // Owned slots active in step t: a prefix s < nact(t).
  auto nact = [&](int t) {
    const int lim = min(K, nL - t * K) * nblk;
    int a = 0;
#pragma unroll
    for (int s = 0; s < SPW; ++s) a += (w * SPW + s < lim) ? 1 : 0;
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
                                         (__attribute__((address_space(3))) void*)(dst + d * kBlk4), 16, 0,
                                         kStreamPolicy);
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
      double M[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) M[q] = 0.0;
#pragma unroll
      for (int s = 0; s < SPW; ++s) {
        const int u = w * SPW + s;
        if (u < lim) {
          wait_vm(3 * (issued - consumed - 1));
          f4v p0, p1, p2;
          read_block<0>(ring_addr + (unsigned)(rd_slot * kBF4 * 4), p0, p1, p2);
          ++consumed;
          if (++rd_slot == RS) rd_slot = 0;
          if (issued < NB) issue_next();
          f4v x0, x1, x2;
          read_block<0>(xs_addr + (unsigned)(ub[s] * kBF4 * 4), x0, x1, x2);
          const bool in = ub[s] * kBlk4 + lane * 4 < n_pad;
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
          // A run of units of one landmark ends here: reduce it once and
          // store it at this unit; the run's earlier units store zeros.
          const bool last = (s == SPW - 1) || (u + 1 >= lim) || (uk[s < SPW - 1 ? s + 1 : s] != uk[s]);
          double* pp = e4_part[t & 1][u];
          if (last) {
            wave_sum9_store(M, pp, lane);
#pragma unroll
            for (int q = 0; q < 9; ++q) M[q] = 0.0;
          } else if (lane == 63) {
#pragma unroll
            for (int q = 0; q < 9; ++q) pp[q] = 0.0;
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
        // The running minimum moved: rescale, and move U's reference
        // property with it, U' = U + (q0 - q0') V (V is FP64).
        const double dq = e4_dq[tp & 1];
#pragma unroll
        for (int s = 0; s < SPW; ++s)
#pragma unroll
          for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const double v = V[s][d][e];
              U[s][d][e] = (float)(fma(dq, v, (double)U[s][d][e]) * sc);
              V[s][d][e] = v * sc;
            }
      }
#pragma unroll
      for (int s = 0; s < SPW; ++s) {
        if (w * SPW + s < limp) {
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
  float* pu = partial_u<float>(c.P->vec, c.slot, n_pad);
  double* pv = partial_v<float>(c.P->vec, c.slot, n_pad);
  if (K == 1) {
    // One landmark lane: every block has exactly one owner.
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      const int j0 = ub[s] * kBlk4 + lane * 4;
      if (w * SPW + s < ufull && j0 < n_pad) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          f4v u4;
          d2v v01, v23;
#pragma unroll
          for (int e = 0; e < 4; ++e) u4[e] = (float)((double)U[s][d][e] - mu[d]);
          v01[0] = V[s][d][0] - mv[d];
          v01[1] = V[s][d][1] - mv[d];
          v23[0] = V[s][d][2] - mv[d];
          v23[1] = V[s][d][3] - mv[d];
          stg(reinterpret_cast<f4v*>(pu + (size_t)d * n_pad + j0), u4);
          stg(reinterpret_cast<d2v*>(pv + (size_t)d * n_pad + j0), v01);
          stg(reinterpret_cast<d2v*>(pv + (size_t)d * n_pad + j0 + 2), v23);
        }
      }
    }
    return;
  }
  // K > 1: unit sums through the idle copy rings (unit u at u * kBF4 floats
  // for U, u * kBF4 doubles for V), then block b (owned by worker b mod 7)
  // adds its K units in landmark-lane order.  Three barriers, matched by the
  // solver.
#pragma unroll
  for (int s = 0; s < SPW; ++s) {
    const int u = w * SPW + s;
    if (u < ufull) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        f4v u4;
#pragma unroll
        for (int e = 0; e < 4; ++e) u4[e] = U[s][d][e];
        *reinterpret_cast<f4v*>(rings + (size_t)u * kBF4 + d * kBlk4 + lane * 4) = u4;
      }
    }
  }
  bar_lds();
  for (int b = w; b < nblk; b += kW4) {
    const int j0 = b * kBlk4 + lane * 4;
    f4v acc[3] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    for (int k = 0; k < K; ++k) {
      const float* src = rings + (size_t)(k * nblk + b) * kBF4 + lane * 4;
#pragma unroll
      for (int d = 0; d < 3; ++d) acc[d] += *reinterpret_cast<const f4v*>(src + d * kBlk4);
    }
    if (j0 < n_pad) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        f4v u4;
#pragma unroll
        for (int e = 0; e < 4; ++e) u4[e] = (float)((double)acc[d][e] - mu[d]);
        stg(reinterpret_cast<f4v*>(pu + (size_t)d * n_pad + j0), u4);
      }
    }
  }
  bar_lds();
  double* vr = reinterpret_cast<double*>(rings);
#pragma unroll
  for (int s = 0; s < SPW; ++s) {
    const int u = w * SPW + s;
    if (u < ufull) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        d2v v01, v23;
        v01[0] = V[s][d][0];
        v01[1] = V[s][d][1];
        v23[0] = V[s][d][2];
        v23[1] = V[s][d][3];
        double* dst = vr + (size_t)u * kBF4 + d * kBlk4 + lane * 4;
        *reinterpret_cast<d2v*>(dst) = v01;
        *reinterpret_cast<d2v*>(dst + 2) = v23;
      }
    }
  }
  bar_lds();
  for (int b = w; b < nblk; b += kW4) {
    const int j0 = b * kBlk4 + lane * 4;
    d2v acc[3][2] = {};
    for (int k = 0; k < K; ++k) {
      const double* src = vr + (size_t)(k * nblk + b) * kBF4 + lane * 4;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        acc[d][0] += *reinterpret_cast<const d2v*>(src + d * kBlk4);
        acc[d][1] += *reinterpret_cast<const d2v*>(src + d * kBlk4 + 2);
      }
    }
    if (j0 < n_pad) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        d2v v01 = acc[d][0], v23 = acc[d][1];
        v01[0] -= mv[d];
        v01[1] -= mv[d];
        v23[0] -= mv[d];
        v23[1] -= mv[d];
        stg(reinterpret_cast<d2v*>(pv + (size_t)d * n_pad + j0), v01);
        stg(reinterpret_cast<d2v*>(pv + (size_t)d * n_pad + j0 + 2), v23);
      }
    }
  }
}

// ------------------------------------------------------------------ solver
__device__ __forceinline__ void e4_solver(const E4Item& c, int lane, int mode, double* dout) {
  const Problem& P = *c.P;
  const double lam = c.lam;
  // Reference property of U = sum e (q - q0) r: the property of the running
  // minimum's landmark, so that U stays small where the weights are large
  // and the merge's U + (q0 - s) V does not cancel.
  double q0 = c.q0;
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
  // Approximate steps with Problem::xuv: XU = sum e (q - q0) T_i and
  // XV = sum e T_i with T_i[r][c] = sum_j (w x_c)_j,r (R_i (a_ij - c_i))_c =
  // (R_i M_i)[c][r], the item's share of Eq. 6's G, kept like tU / tV.
  const bool want_xuv = mode == MODE_APPROX && P.xuv != nullptr;
  double XU[9], XV[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) { XU[k] = 0.0; XV[k] = 0.0; }
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
      double D = INFINITY, R[9], Mc[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) R[k] = 0.0;
#pragma unroll
      for (int q = 0; q < 9; ++q) Mc[q] = 0.0;
      if (act) {
        // Correlation of landmark lane k: its nblk unit sums in block order.
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
      double dq = 0.0;
      if (mn < m) {
        const unsigned long long hit = __ballot(act && D == mb);
        const int src = hit ? __ffsll((long long)hit) - 1 : 0;   // lowest lane holding the minimum
        const double qn = __shfl(qv, src, 64);
        dq = q0 - qn;
        q0 = qn;
      }
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
        tU[d] = fma(dq, tV[d], tU[d]) * sc + al * rc;
        tV[d] = tV[d] * sc + e * rc;
      }
      if (want_xuv) {
#pragma unroll
        for (int r0 = 0; r0 < 3; ++r0)
#pragma unroll
          for (int c0 = 0; c0 < 3; ++c0) {
            const double tv = R[c0 * 3 + 0] * Mc[0 * 3 + r0] + R[c0 * 3 + 1] * Mc[1 * 3 + r0] +
                              R[c0 * 3 + 2] * Mc[2 * 3 + r0];
            const int k = r0 * 3 + c0;
            XU[k] = fma(dq, XV[k], XU[k]) * sc + al * tv;
            XV[k] = XV[k] * sc + e * tv;
          }
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
      if (lane == 0) {
        e4_sc[t & 1] = sc;
        e4_dq[t & 1] = dq;
      }
    }
  }
  // Item totals: the per-lane sums added over the wave in a fixed order; the
  // header carries the final reference property.
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
  if (lane == 63) {
    double* h = P.hdr + (size_t)c.slot * 4;
    stg(h + 0, m);
    stg(h + 1, Z);
    stg(h + 2, S);
    stg(h + 3, q0);
  }
  if (want_xuv) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      XU[k] = wave_sum_to63(XU[k]);
      XV[k] = wave_sum_to63(XV[k]);
    }
    if (lane == 63) {
      double* x = P.xuv + (size_t)c.slot * 18;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        stg(x + k, XU[k]);
        stg(x + 9 + k, XV[k]);
      }
    }
  }
  bar_lds();
  if (K > 1) {   // the workers' three barriers of the unit-sum reduction
    bar_lds();
    bar_lds();
    bar_lds();
  }
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
  {
    const Problem* pr = probs;
    if (!gate_launch(flag, run_if, mode, pr)) return;
    probs = pr;
  }
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
    c.lam = c.P->lam;
    c.q0 = c.P->q[item.i0];
    // Shapes the host planner never produces are skipped by every wave alike.
    if (c.nL < 1 || c.nblk > kMaxBlk4 || c.K < 1 || c.K * c.nblk > kW4 * SPW) continue;
    if (wave < kW4) e4_worker<SPW>(c, wave, lane, ring + wave * kRing4 * kBF4, ring, xs);
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
