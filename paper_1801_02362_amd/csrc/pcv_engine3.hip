// Streaming landmark engine for large structures on gfx950 (FP32 coordinates).
//
// One 512-thread workgroup per CU: seven worker waves and one solver wave.
// The atoms are cut into blocks of 256 (64 lanes x 4 atoms); worker wave w
// owns blocks w, w + 7, w + 14, w + 21 (at most BPW of them) for every
// landmark of its work item, so each worker keeps its atoms' share of the
// centred, weighted structure in registers and streams only its own
// coordinates:
//
//   * a private ring of block slots in LDS is filled by asynchronous
//     HBM -> LDS copies (global_load_lds_dwordx4, 16 B per lane); a wave
//     waits only for the oldest block it needs (partial vmcnt), so the
//     younger copies stay in flight across the pipeline barrier;
//   * the landmark is read from its slot into registers once; it feeds the
//     correlation M = sum_j a_j (w_j x_j)^T (FP64 accumulation) at once and
//     the gradient one step later, when the rotation is known;
//   * one barrier per landmark t: before it, the workers contract landmark t
//     and publish its correlation; after it, the solver wave solves the
//     quaternion eigenproblem of t (Section 3) and folds it into the running
//     log-sum-exp (Eq. 2) while the workers add the gradient terms of t - 1,
//     U += e (q - q0) R (a - c) in FP32 and V += e R (a - c) in FP64 (FP32
//     over the item at four blocks per wave), and go on to contract t + 1.
//     The solve is thus hidden behind a whole gradient-plus-correlation
//     step; correlation and result slots are double-buffered by landmark
//     parity.
//
// Workers reduce their 9 correlation sums over the wave by transposed
// halving (lane swaps, then DPP row sums); the solver adds the 7 worker sums
// in a fixed order, so results do not depend on timing.  Each work item writes one partial (m, Z, S, q0, U, V)
// in the format of the other engines, so the merge kernels are shared.
//
// Synchronisation: the copies are the only vector-memory operations the
// workers issue inside the landmark loop, so "wait until at most k copy
// instructions are outstanding" is an exact per-slot wait.  Barriers wait on
// LDS traffic only (the compiler's workgroup barrier would also drain the
// copies in flight), and slot reads are inline assembly that waits for its
// own results, so the compiler never adds a full vmcnt wait in front of them.
#include "pcv_internal.h"
#include "pcv_math.h"
#include "pcv_stream.h"

namespace pcv {

namespace {

constexpr int kWG3 = 512;
constexpr int kWorkers3 = 7;
constexpr int kBlk3 = 256;                      // atoms per block: 64 lanes x 4
constexpr int kBlkFloats3 = 3 * kBlk3;          // one block of one landmark (x, y, z planes)

// Copy-ring depth (block slots per worker wave) for BPW blocks per wave: the
// ring and the wave's FP32 structure share about 150 KB of LDS.
constexpr int ring_slots(int bpw) { return bpw >= 4 ? 3 : (bpw == 3 ? 4 : (bpw == 2 ? 5 : 6)); }

// Accumulator of V = sum e R (a - c): FP64, except at four blocks per wave,
// where the registers of a wave hold 16 atoms per lane and V is kept in FP32
// over the item (the merge adds the item partials in FP64).
template <int BPW>
struct E3VAcc { typedef double type; };
template <>
struct E3VAcc<4> { typedef float type; };

__shared__ double e3_part[2][kWorkers3][9];
__shared__ double e3_res[2][16];
__shared__ double e3_misc[16];

// Block k of a wave's structure area (k is a constant after unrolling).
__device__ __forceinline__ void read_xblock(int k, unsigned addr, f4v& p0, f4v& p1, f4v& p2) {
  switch (k) {
    case 0: read_block<0>(addr, p0, p1, p2); break;
    case 1: read_block<kBlkFloats3 * 4>(addr, p0, p1, p2); break;
    case 2: read_block<2 * kBlkFloats3 * 4>(addr, p0, p1, p2); break;
    default: read_block<3 * kBlkFloats3 * 4>(addr, p0, p1, p2); break;
  }
}

__device__ __forceinline__ double clamp0_3(double v) { return v < 0.0 ? 0.0 : v; }

struct E3Item {
  const Problem* P;
  int i0, nL, slot, n_pad;
  double lam, q0;
};

// ------------------------------------------------------------------ worker
// ring: this wave's RS block slots; xs: this wave's BPW blocks of w_j x_j (FP32).
template <int BPW>
__device__ __forceinline__ void e3_worker(const E3Item& c, int w, int lane, float* ring, float* xs) {
  constexpr int RS = ring_slots(BPW);
  const int n_pad = c.n_pad;
  const int nblk = (n_pad + kBlk3 - 1) / kBlk3;
  int nbw = 0;
#pragma unroll
  for (int k = 0; k < BPW; ++k) nbw += (w + kWorkers3 * k < nblk) ? 1 : 0;
  const int nL = c.nL;
  const int NB = nL * nbw;   // blocks streamed by this wave
  const float* A = (const float*)c.P->A;
  const unsigned ring_addr = (unsigned)(size_t)((__attribute__((address_space(3))) float*)ring) + lane * 16;

  // Copy stream: block b = t * nbw + k of this wave (landmark t, block w + 7k).
  int it_t = 0, it_k = 0, it_slot = 0, issued = 0;
  auto issue_next = [&]() {
    const int j0 = (w + kWorkers3 * it_k) * kBlk3 + lane * 4;
    const int jj = j0 < n_pad ? j0 : 0;   // lanes past the structure copy in-bounds data (x = 0 there)
    const float* src = A + (size_t)(c.i0 + it_t) * 3 * n_pad + jj;
    float* dst = ring + it_slot * kBlkFloats3;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      __builtin_amdgcn_global_load_lds((const void*)(src + (size_t)d * n_pad),
                                       (__attribute__((address_space(3))) void*)(dst + d * kBlk3), 16, 0,
                                       kStreamPolicy);
    if (++it_k == nbw) { it_k = 0; ++it_t; }
    if (++it_slot == RS) it_slot = 0;
    ++issued;
  };
  // This lane's atoms j = (w + 7k) * 256 + 4 lane + e of w_j x_c,j (FP32,
  // zero past the structure) go to the wave's LDS area through registers
  // before any copy is issued.
  {
    const int n_x = c.P->n_x;
    const float* xsrc = c.P->xw32;
    f4v xv[BPW][3];
#pragma unroll
    for (int k = 0; k < BPW; ++k) {
      if (k < nbw) {
        const int j0 = (w + kWorkers3 * k) * kBlk3 + lane * 4;
#pragma unroll
        for (int d = 0; d < 3; ++d) xv[k][d] = ldg(reinterpret_cast<const f4v*>(xsrc + (size_t)d * n_x + j0));
      }
    }
#pragma unroll
    for (int k = 0; k < BPW; ++k) {
      if (k < nbw) {
#pragma unroll
        for (int d = 0; d < 3; ++d) *reinterpret_cast<f4v*>(xs + (k * 3 + d) * kBlk3 + lane * 4) = xv[k][d];
      }
    }
  }
  const unsigned xs_addr = (unsigned)(size_t)((__attribute__((address_space(3))) float*)xs) + lane * 16;
  for (int b = 0; b < RS && b < NB; ++b) issue_next();

  using VT = typename E3VAcc<BPW>::type;
  float U[BPW][3][4];
  VT V[BPW][3][4];
#pragma unroll
  for (int k = 0; k < BPW; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int e = 0; e < 4; ++e) { U[k][d][e] = 0.f; V[k][d][e] = VT(0); }

  float a0[BPW][3][4], a1[BPW][3][4];
  int rd_slot = 0, consumed = 0;

  // One pipeline step: landmark t into `cur` + correlation (phase A), then
  // gradient of t - 1 from `prev` (phase B).
  auto step = [&](int t, float (&cur)[BPW][3][4], float (&prev)[BPW][3][4]) {
    if (t < nL) {
      double M[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) M[q] = 0.0;
#pragma unroll
      for (int k = 0; k < BPW; ++k) {
        if (k < nbw) {
          wait_vm(3 * (issued - consumed - 1));
          f4v p0, p1, p2;
          read_block<0>(ring_addr + (unsigned)(rd_slot * kBlkFloats3 * 4), p0, p1, p2);
          ++consumed;
          if (++rd_slot == RS) rd_slot = 0;
          if (issued < NB) issue_next();
          f4v x0, x1, x2;
          read_xblock(k, xs_addr, x0, x1, x2);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            cur[k][0][e] = p0[e]; cur[k][1][e] = p1[e]; cur[k][2][e] = p2[e];
            const double y0 = x0[e], y1 = x1[e], y2 = x2[e];
            const double b0 = p0[e], b1 = p1[e], b2 = p2[e];
            M[0] = fma(b0, y0, M[0]); M[1] = fma(b0, y1, M[1]); M[2] = fma(b0, y2, M[2]);
            M[3] = fma(b1, y0, M[3]); M[4] = fma(b1, y1, M[4]); M[5] = fma(b1, y2, M[5]);
            M[6] = fma(b2, y0, M[6]); M[7] = fma(b2, y1, M[7]); M[8] = fma(b2, y2, M[8]);
          }
        }
      }
      wave_sum9_store(M, e3_part[t & 1][w], lane);
    }
    bar_lds();
    if (t >= 1) {
      const double* rs = e3_res[(t - 1) & 1];
      const double sc = rs[11];
      if (sc != 1.0) {
        // The running minimum moved: rescale, and move U's reference
        // property with it, U' = U + (q0 - q0') V.
        const double dq = rs[15];
#pragma unroll
        for (int k = 0; k < BPW; ++k)
#pragma unroll
          for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const double v = (double)V[k][d][e];
              U[k][d][e] = (float)(fma(dq, v, (double)U[k][d][e]) * sc);
              V[k][d][e] = (VT)(v * sc);
            }
      }
      float Rt[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) Rt[q] = (float)rs[q];
      const float alf = (float)rs[9];
      const double be = rs[10];
      const float ch0 = (float)rs[12], ch1 = (float)rs[13], ch2 = (float)rs[14];
#pragma unroll
      for (int k = 0; k < BPW; ++k) {
        if (k < nbw) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float b0 = prev[k][0][e] - ch0, b1 = prev[k][1][e] - ch1, b2 = prev[k][2][e] - ch2;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const float r = fmaf(Rt[d * 3 + 0], b0, fmaf(Rt[d * 3 + 1], b1, Rt[d * 3 + 2] * b2));
              U[k][d][e] = fmaf(alf, r, U[k][d][e]);
              V[k][d][e] = (VT)fma((VT)be, (VT)r, V[k][d][e]);
            }
          }
        }
      }
    }
  };

  for (int t = 0; t <= nL; t += 2) {
    step(t, a0, a1);
    if (t + 1 <= nL) step(t + 1, a1, a0);
  }

  bar_lds();   // item totals published by the solver
  float* pu = partial_u<float>(c.P->vec, c.slot, n_pad);
  double* pv = partial_v<float>(c.P->vec, c.slot, n_pad);
  double mu[3], mv[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) { mu[d] = e3_misc[3 + d]; mv[d] = e3_misc[6 + d]; }
  // 16-byte stores: a lane's four consecutive atoms (n_pad is a multiple of
  // 64, so a group of four is either wholly inside or wholly past it).
#pragma unroll
  for (int k = 0; k < BPW; ++k) {
    if (k < nbw) {
      const int j0 = (w + kWorkers3 * k) * kBlk3 + lane * 4;
      if (j0 < n_pad) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          f4v u4;
          d2v v01, v23;
#pragma unroll
          for (int e = 0; e < 4; ++e) u4[e] = (float)((double)U[k][d][e] - mu[d]);
          v01[0] = (double)V[k][d][0] - mv[d];
          v01[1] = (double)V[k][d][1] - mv[d];
          v23[0] = (double)V[k][d][2] - mv[d];
          v23[1] = (double)V[k][d][3] - mv[d];
          stg(reinterpret_cast<f4v*>(pu + (size_t)d * n_pad + j0), u4);
          stg(reinterpret_cast<d2v*>(pv + (size_t)d * n_pad + j0), v01);
          stg(reinterpret_cast<d2v*>(pv + (size_t)d * n_pad + j0 + 2), v23);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ solver
__device__ __forceinline__ void e3_solver(const E3Item& c, int lane, int mode, double* dout) {
  const Problem& P = *c.P;
  // The per-landmark arrays' addresses, held in scalar registers for the
  // whole item: read through P inside the loop they would be fetched again
  // after every barrier (its memory clobber), and the prefetch of the next
  // landmark's scalars would wait for that round trip under the full
  // landmark stream.
  const double* const ca_p = uniform_ptr(P.ca);
  const double* const Ga_p = uniform_ptr(P.Ga);
  const double* const q_p = uniform_ptr(P.q);
  double* const Rsave_p = uniform_ptr(P.Rsave);
  long long* const fallbacks_p = uniform_ptr(P.fallbacks);
  double* const hdr_p = uniform_ptr(P.hdr);
  const double lam = c.lam;
  // Reference property of U = sum e (q - q0) r: the property of the running
  // minimum's landmark (keeps U small where the weights are large).
  double q0 = c.q0;
  const int nL = c.nL;
  const double Gxx = ldg(P.Gx32);
  double xres[3], Rx[9];
#pragma unroll
  for (int d = 0; d < 3; ++d) xres[d] = ldg(P.xres + d);
#pragma unroll
  for (int k = 0; k < 9; ++k) Rx[k] = (mode == MODE_APPROX) ? ldg(P.Rxy + k) : 0.0;
  double m = INFINITY, Z = 0.0, S = 0.0, tU[3] = {0.0, 0.0, 0.0}, tV[3] = {0.0, 0.0, 0.0};
  // Per-landmark inputs of 64 landmarks at a time, lane k holding landmark
  // blk + k; a landmark's values are taken with readlane (scalar registers).
  // The next block is fetched half a block ahead, so no step waits for a
  // memory round trip (under the full landmark stream a load issued one
  // step ahead is not back in time).
  double bca[3], bGa, bq, bRs[9];      // current block
  double nca[3], nGa, nq, nRs[9];      // next block, in flight
  auto fetch_block = [&](int blk, double (&ca3)[3], double& Ga1, double& q1, double (&Rs9)[9]) {
    const int t = blk + lane;
    const int i = c.i0 + (t < nL ? t : nL - 1);
#pragma unroll
    for (int d = 0; d < 3; ++d) ca3[d] = ldg(ca_p + (size_t)i * 3 + d);
    Ga1 = ldg(Ga_p + i);
    q1 = ldg(q_p + i);
#pragma unroll
    for (int k = 0; k < 9; ++k) Rs9[k] = (mode == MODE_APPROX) ? ldg(Rsave_p + (size_t)i * 9 + k) : 0.0;
  };
  fetch_block(0, bca, bGa, bq, bRs);
  if (nL > 64) fetch_block(64, nca, nGa, nq, nRs);
  for (int t = 0; t <= nL; ++t) {
    bar_lds();
    if (t < nL) {
      const int i = c.i0 + t;
      const int k64 = t & 63;
      if (k64 == 0 && t > 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) bca[d] = nca[d];
        bGa = nGa;
        bq = nq;
#pragma unroll
        for (int k = 0; k < 9; ++k) bRs[k] = nRs[k];
      }
      if (k64 == 32 && t + 32 < nL) fetch_block(t + 32, nca, nGa, nq, nRs);
      const double cc[3] = {readlane_f64(bca[0], k64), readlane_f64(bca[1], k64), readlane_f64(bca[2], k64)};
      const double Gai = readlane_f64(bGa, k64), qv = readlane_f64(bq, k64);
      double Rsv[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) Rsv[k] = (mode == MODE_APPROX) ? readlane_f64(bRs[k], k64) : 0.0;
      // Correlation of landmark t: the seven worker sums added in a fixed order.
      double ssum = 0.0;
      {
        const double(*pp)[9] = e3_part[t & 1];
        const int l9 = lane < 9 ? lane : 0;
        double pv[kWorkers3];
#pragma unroll
        for (int p = 0; p < kWorkers3; ++p) pv[p] = pp[p][l9];
#pragma unroll
        for (int p = 0; p < kWorkers3; ++p) ssum += pv[p];
      }
      double Mc[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) Mc[k] = readlane_f64(ssum, k);
      // The workers used w_j x_j rounded to FP32, whose sum (xres) is not
      // exactly zero; remove its coupling to the landmark centroid.
#pragma unroll
      for (int r0 = 0; r0 < 3; ++r0)
#pragma unroll
        for (int c0 = 0; c0 < 3; ++c0) Mc[r0 * 3 + c0] = fma(-cc[r0], xres[c0], Mc[r0 * 3 + c0]);
      double D, R[9];
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
        D = clamp0_3(Gxx + Gai - 2.0 * tr);
#pragma unroll
        for (int k = 0; k < 9; ++k) R[k] = Rsv[k];
      } else {
        double F[10], lmax, qq[4];
        const int fb = top_eigenpair(Mc, 0.5 * (Gxx + Gai), F, lmax, qq);
        if (fb && lane == 0 && fallbacks_p) atomicAdd((unsigned long long*)fallbacks_p, 1ull);
        D = clamp0_3(Gxx + Gai - 2.0 * lmax);
        quat_to_rot(qq, R);
        if (mode == MODE_EXACT_SAVE) {
          double rv = 0.0;
#pragma unroll
          for (int q = 0; q < 9; ++q) rv = (lane == q) ? R[q] : rv;
          if (lane < 9) stg(Rsave_p + (size_t)i * 9 + lane, rv);
        }
      }
      if (dout != nullptr && lane == 0) stg(dout + i, D);
      const double mn = fmin(m, D);
      const double sc = (m == INFINITY) ? 0.0 : ((mn == m) ? 1.0 : exp(-lam * (m - mn)));
      double dq = 0.0;
      if (mn < m) {
        dq = q0 - qv;
        q0 = qv;
      }
      const double e = exp(-lam * (D - mn));
      const double al = e * (qv - q0);
      Z = Z * sc + e;
      S = S * sc + e * qv;
      // Residual of the centroid split the workers use (c - (float)c).
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double c3[3] = {cc[0] - (double)(float)cc[0], cc[1] - (double)(float)cc[1],
                              cc[2] - (double)(float)cc[2]};
        const double rc = R[d * 3 + 0] * c3[0] + R[d * 3 + 1] * c3[1] + R[d * 3 + 2] * c3[2];
        tU[d] = fma(dq, tV[d], tU[d]) * sc + al * rc;
        tV[d] = tV[d] * sc + e * rc;
      }
      m = mn;
      // Lane k publishes entry k (selects, not a register-array index).
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < 9; ++q) v = (lane == q) ? R[q] : v;
      v = (lane == 9) ? al : v;
      v = (lane == 10) ? e : v;
      v = (lane == 11) ? sc : v;
#pragma unroll
      for (int d = 0; d < 3; ++d) v = (lane == 12 + d) ? cc[d] : v;
      v = (lane == 15) ? dq : v;
      if (lane < 16) e3_res[t & 1][lane] = v;
    }
  }
  if (lane == 0) {
    e3_misc[0] = m;
    e3_misc[1] = Z;
    e3_misc[2] = S;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      e3_misc[3 + d] = tU[d];
      e3_misc[6 + d] = tV[d];
    }
    double* h = hdr_p + (size_t)c.slot * 4;
    stg(h + 0, m);
    stg(h + 1, Z);
    stg(h + 2, S);
    stg(h + 3, q0);
  }
  bar_lds();
}

// ------------------------------------------------------ register-stream worker
// Engine 5: the same pipeline and solver, with the landmark blocks streamed
// HBM -> registers (global_load_dwordx4, non-temporal) instead of through an
// LDS copy ring.  A worker keeps two register sets of its BPW blocks and one
// LDS slot per block; at the step between barriers t and t + 1 it
//   * adds the gradient terms of landmark t - 1 from the slot (the solver
//     published its rotation before barrier t),
//   * moves landmark t (set X, correlated one step earlier) into the slot,
//   * issues the loads of landmark t + 2 into set X,
//   * contracts landmark t + 1 from set Y (loaded one step earlier) and
//     publishes its correlation before barrier t + 1.
// Each landmark is thus in flight for about one step and held for about
// one, and every wave touches only its own slot and structure blocks in LDS.
// The loads are unconditional (lanes past the structure, and blocks the
// wave does not own, read the structure copy instead, which the caches
// hold), so the number of outstanding loads is static and the wait before a
// set's use leaves the younger set's loads in flight.
template <int BPW>
__device__ __forceinline__ void e5_worker(const E3Item& c, int w, int lane, float* slot, float* xs) {
  const int n_pad = c.n_pad;
  const int nblk = (n_pad + kBlk3 - 1) / kBlk3;
  int nbw = 0;
#pragma unroll
  for (int k = 0; k < BPW; ++k) nbw += (w + kWorkers3 * k < nblk) ? 1 : 0;
  const int nL = c.nL;
  const float* xsrc = c.P->xw32;
  const int n_x = c.P->n_x;
  // The item's landmarks through one buffer descriptor (range-checked: an
  // offset past the item reads zeros and touches no memory).  Lanes holding
  // no atom of the structure, and blocks the wave does not own, start from
  // such an offset, so every load is issued unconditionally and the count of
  // outstanding loads is the same on every path.  The item must stay below
  // 2 GiB so that offsets do not wrap.
  const __amdgpu_buffer_rsrc_t rsrc = make_rsrc((const float*)c.P->A + (size_t)c.i0 * 3 * n_pad, nL * 3 * n_pad * 4);
  int voff[BPW];
#pragma unroll
  for (int k = 0; k < BPW; ++k) {
    const int j0 = (w + kWorkers3 * k) * kBlk3 + lane * 4;
    voff[k] = (k < nbw && j0 < n_pad) ? j0 * 4 : kOutOfRange;
  }
  // Structure blocks into the wave's LDS area (zero past the structure).
  {
    f4v xv[BPW][3];
#pragma unroll
    for (int k = 0; k < BPW; ++k) {
      if (k < nbw) {
        const int j0 = (w + kWorkers3 * k) * kBlk3 + lane * 4;
#pragma unroll
        for (int d = 0; d < 3; ++d) xv[k][d] = ldg(reinterpret_cast<const f4v*>(xsrc + (size_t)d * n_x + j0));
      }
    }
#pragma unroll
    for (int k = 0; k < BPW; ++k) {
      if (k < nbw) {
#pragma unroll
        for (int d = 0; d < 3; ++d) *reinterpret_cast<f4v*>(xs + (k * 3 + d) * kBlk3 + lane * 4) = xv[k][d];
      }
    }
  }
  // Landmark t of the item into S.  The whole offset is the lane's (the
  // range-checked part of a buffer address): past the item (t >= nL) it is
  // at least the descriptor's byte count, so the load is still issued and
  // returns zeros, with no condition for the compiler to branch on.
  auto load = [&](f4v (&S)[BPW][3], int t) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int base = (t * 3 + d) * n_pad * 4;
#pragma unroll
      for (int k = 0; k < BPW; ++k)
        S[k][d] = __builtin_bit_cast(
            f4v, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff[k] + base, 0, kStreamPolicy));
    }
  };
  auto corr = [&](const f4v (&S)[BPW][3], int t) {
    double M[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) M[q] = 0.0;
#pragma unroll
    for (int k = 0; k < BPW; ++k) {
      if (k < nbw) {
        const f4v* xp = reinterpret_cast<const f4v*>(xs + k * kBlkFloats3) + lane;
        const f4v x0 = xp[0], x1 = xp[kBlk3 / 4], x2 = xp[kBlk3 / 2];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double y0 = x0[e], y1 = x1[e], y2 = x2[e];
          const double b0 = S[k][0][e], b1 = S[k][1][e], b2 = S[k][2][e];
          M[0] = fma(b0, y0, M[0]); M[1] = fma(b0, y1, M[1]); M[2] = fma(b0, y2, M[2]);
          M[3] = fma(b1, y0, M[3]); M[4] = fma(b1, y1, M[4]); M[5] = fma(b1, y2, M[5]);
          M[6] = fma(b2, y0, M[6]); M[7] = fma(b2, y1, M[7]); M[8] = fma(b2, y2, M[8]);
        }
      }
    }
    wave_sum9_store(M, e3_part[t & 1][w], lane);
  };
  auto stash = [&](const f4v (&S)[BPW][3]) {
#pragma unroll
    for (int k = 0; k < BPW; ++k) {
      if (k < nbw) {
        f4v* sp = reinterpret_cast<f4v*>(slot + k * kBlkFloats3) + lane;
        sp[0] = S[k][0];
        sp[kBlk3 / 4] = S[k][1];
        sp[kBlk3 / 2] = S[k][2];
      }
    }
  };

  float U[BPW][3][4];
  double V[BPW][3][4];
#pragma unroll
  for (int k = 0; k < BPW; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int e = 0; e < 4; ++e) { U[k][d][e] = 0.f; V[k][d][e] = 0.0; }

  // Gradient terms of landmark t from the slot: U += e (q - q0) R (a - c),
  // V += e R (a - c), after the rescale the solver signalled.
  auto grad = [&](int t) {
    const double* rs = e3_res[t & 1];
    const double sc = rs[11];
    if (sc != 1.0) {
      const double dq = rs[15];
#pragma unroll
      for (int k = 0; k < BPW; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double v = V[k][d][e];
            U[k][d][e] = (float)(fma(dq, v, (double)U[k][d][e]) * sc);
            V[k][d][e] = v * sc;
          }
    }
    float Rt[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) Rt[q] = (float)rs[q];
    const float alf = (float)rs[9];
    const double be = rs[10];
    const float ch0 = (float)rs[12], ch1 = (float)rs[13], ch2 = (float)rs[14];
#pragma unroll
    for (int k = 0; k < BPW; ++k) {
      if (k < nbw) {
        const f4v* sp = reinterpret_cast<const f4v*>(slot + k * kBlkFloats3) + lane;
        const f4v p0 = sp[0], p1 = sp[kBlk3 / 4], p2 = sp[kBlk3 / 2];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float b0 = p0[e] - ch0, b1 = p1[e] - ch1, b2 = p2[e] - ch2;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const float r = fmaf(Rt[d * 3 + 0], b0, fmaf(Rt[d * 3 + 1], b1, Rt[d * 3 + 2] * b2));
            U[k][d][e] = fmaf(alf, r, U[k][d][e]);
            V[k][d][e] = fma(be, (double)r, V[k][d][e]);
          }
        }
      }
    }
  };

  f4v S0[BPW][3], S1[BPW][3];
  // One step between barriers t and t + 1: X holds landmark t, Y landmark
  // t + 1.  Loads are issued on every path (zeros past the item), so the
  // compiler's count of outstanding loads is exact and the wait before the
  // contraction of Y leaves X's new loads in flight.
  auto seg = [&](int t, f4v (&X)[BPW][3], f4v (&Y)[BPW][3]) {
    if (t >= 1) grad(t - 1);
    stash(X);
    load(X, t + 2);
    if (t + 1 < nL) corr(Y, t + 1);
    bar_lds();
  };
  load(S0, 0);
  load(S1, 1);
  corr(S0, 0);
  bar_lds();
  int t = 0;
  for (; t + 1 < nL; t += 2) {
    seg(t, S0, S1);
    seg(t + 1, S1, S0);
  }
  if (t < nL) seg(t, S0, S1);
  grad(nL - 1);

  bar_lds();   // item totals published by the solver
  float* pu = partial_u<float>(c.P->vec, c.slot, n_pad);
  double* pv = partial_v<float>(c.P->vec, c.slot, n_pad);
  double mu[3], mv[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) { mu[d] = e3_misc[3 + d]; mv[d] = e3_misc[6 + d]; }
#pragma unroll
  for (int k = 0; k < BPW; ++k) {
    if (k < nbw) {
      const int j0 = (w + kWorkers3 * k) * kBlk3 + lane * 4;
      if (j0 < n_pad) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          f4v u4;
          d2v v01, v23;
#pragma unroll
          for (int e = 0; e < 4; ++e) u4[e] = (float)((double)U[k][d][e] - mu[d]);
          v01[0] = V[k][d][0] - mv[d];
          v01[1] = V[k][d][1] - mv[d];
          v23[0] = V[k][d][2] - mv[d];
          v23[1] = V[k][d][3] - mv[d];
          stg(reinterpret_cast<f4v*>(pu + (size_t)d * n_pad + j0), u4);
          stg(reinterpret_cast<d2v*>(pv + (size_t)d * n_pad + j0), v01);
          stg(reinterpret_cast<d2v*>(pv + (size_t)d * n_pad + j0 + 2), v23);
        }
      }
    }
  }
}

}  // namespace

template <int BPW>
__global__ __launch_bounds__(kWG3) void engine3_kernel(const Problem* __restrict__ probs,
                                                       const Item* __restrict__ items,
                                                       const int* __restrict__ wg_off, int mode,
                                                       const int* __restrict__ flag, int run_if,
                                                       double* __restrict__ dout) {
  constexpr int RS = ring_slots(BPW);
  __shared__ float ring[kWorkers3 * RS * kBlkFloats3];
  __shared__ float xs[kWorkers3 * BPW * kBlkFloats3];
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
    E3Item c;
    c.P = probs + item.prob;
    c.i0 = item.i0;
    c.nL = item.i1 - item.i0;
    c.slot = item.slot;
    c.n_pad = c.P->n_pad;
    c.lam = c.P->lam;
    c.q0 = c.P->q[item.i0];
    if (wave < kWorkers3)
      e3_worker<BPW>(c, wave, lane, ring + wave * RS * kBlkFloats3, xs + wave * BPW * kBlkFloats3);
    else e3_solver(c, lane, mode, dout);
    bar_lds();   // LDS is reused by the next item
  }
}

int engine3_max_blocks(int bpw) { return kWorkers3 * bpw; }

template <>
hipError_t launch_engine3<float>(int bpw, int grid, const Problem* probs, const Item* items, const int* wg_off,
                                 int mode, const int* flag, int run_if, double* dout, hipStream_t st) {
  switch (bpw) {
    case 1: hipLaunchKernelGGL(engine3_kernel<1>, dim3(grid), dim3(kWG3), 0, st, probs, items, wg_off, mode, flag,
                               run_if, dout); break;
    case 2: hipLaunchKernelGGL(engine3_kernel<2>, dim3(grid), dim3(kWG3), 0, st, probs, items, wg_off, mode, flag,
                               run_if, dout); break;
    case 3: hipLaunchKernelGGL(engine3_kernel<3>, dim3(grid), dim3(kWG3), 0, st, probs, items, wg_off, mode, flag,
                               run_if, dout); break;
    case 4: hipLaunchKernelGGL(engine3_kernel<4>, dim3(grid), dim3(kWG3), 0, st, probs, items, wg_off, mode, flag,
                               run_if, dout); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t launch_engine3<double>(int, int, const Problem*, const Item*, const int*, int, const int*, int, double*,
                                  hipStream_t) {
  return hipErrorInvalidValue;
}

// Engine 5 (register-stream workers, same solver): up to 7 * BPW blocks.
template <int BPW>
__global__ __launch_bounds__(kWG3) void engine5_kernel(const Problem* __restrict__ probs,
                                                       const Item* __restrict__ items,
                                                       const int* __restrict__ wg_off, int mode,
                                                       const int* __restrict__ flag, int run_if,
                                                       double* __restrict__ dout) {
  __shared__ float slot[kWorkers3 * BPW * kBlkFloats3];
  __shared__ float xs[kWorkers3 * BPW * kBlkFloats3];
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
    E3Item c;
    c.P = probs + item.prob;
    c.i0 = item.i0;
    c.nL = item.i1 - item.i0;
    c.slot = item.slot;
    c.n_pad = c.P->n_pad;
    c.lam = c.P->lam;
    c.q0 = c.P->q[item.i0];
    if (wave < kWorkers3)
      e5_worker<BPW>(c, wave, lane, slot + wave * BPW * kBlkFloats3, xs + wave * BPW * kBlkFloats3);
    else e3_solver(c, lane, mode, dout);
    bar_lds();   // LDS is reused by the next item
  }
}

int engine5_max_blocks(int bpw) { return kWorkers3 * bpw; }

template <>
hipError_t launch_engine5<float>(int bpw, int grid, const Problem* probs, const Item* items, const int* wg_off,
                                 int mode, const int* flag, int run_if, double* dout, hipStream_t st) {
  switch (bpw) {
    case 1: hipLaunchKernelGGL(engine5_kernel<1>, dim3(grid), dim3(kWG3), 0, st, probs, items, wg_off, mode, flag,
                               run_if, dout); break;
    case 2: hipLaunchKernelGGL(engine5_kernel<2>, dim3(grid), dim3(kWG3), 0, st, probs, items, wg_off, mode, flag,
                               run_if, dout); break;
    case 3: hipLaunchKernelGGL(engine5_kernel<3>, dim3(grid), dim3(kWG3), 0, st, probs, items, wg_off, mode, flag,
                               run_if, dout); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <>
hipError_t launch_engine5<double>(int, int, const Problem*, const Item*, const int*, int, const int*, int, double*,
                                  hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace pcv
