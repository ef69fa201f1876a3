// Device helpers shared by the streaming landmark engines that copy landmark
// blocks HBM -> LDS asynchronously (global_load_lds) and synchronise with
// LDS-only barriers.
#pragma once

#include <hip/hip_runtime.h>

namespace pcv {

typedef float f4v __attribute__((ext_vector_type(4)));

// Cache policy of the landmark copies: non-temporal (the nt bit).  Every
// landmark byte is read once per launch; marked streaming, the copies run
// about 8 % faster at 5,000 atoms x 10,000 landmarks than with the default
// policy (measured on MI355X).
constexpr int kStreamPolicy = 2;
typedef double d2v __attribute__((ext_vector_type(2)));

// Word 3 of a raw buffer descriptor on gfx9-family chips: 32-bit data
// format, no swizzle (loads of whole dwords, range-checked against the
// descriptor's byte count).
constexpr int kRawBufferWord3 = 0x00020000;
// A buffer offset past any descriptor's range: such a load returns zeros.
constexpr int kOutOfRange = 0x7ffffff0;

// Lane k's value (k wave-uniform) in scalar registers.
__device__ __forceinline__ double readlane_f64(double v, int k) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, k);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), k);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// A pointer that is the same in every lane, as a wave-uniform (scalar) value.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const unsigned long long a = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  return (T*)(((unsigned long long)hi << 32) | lo);
}

// Raw buffer descriptor of `bytes` bytes at p.  The address must be the same
// in every lane; it is made wave-uniform explicitly (read from the first
// lane), so the descriptor lives in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(uniform_ptr((void*)p), (short)0, __builtin_amdgcn_readfirstlane(bytes),
                                           kRawBufferWord3);
}

// LDS-only workgroup barrier: the asynchronous copies in flight are not
// waited for (the compiler's workgroup barrier would drain them).
__device__ __forceinline__ void bar_lds() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0); vmcnt and expcnt not waited for
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Wait until at most n vector-memory instructions of this wave are
// outstanding (n a multiple of 3, at most 15).
__device__ __forceinline__ void wait_vm(int n) {
#define PCV_VM(N) __builtin_amdgcn_s_waitcnt(((N) & 15) | (((N) >> 4) << 14) | 0x0F70)
  switch (n) {
    case 0: PCV_VM(0); break;
    case 3: PCV_VM(3); break;
    case 6: PCV_VM(6); break;
    case 9: PCV_VM(9); break;
    case 12: PCV_VM(12); break;
    default: PCV_VM(15); break;
  }
#undef PCV_VM
}

// Three 16-byte LDS reads (the x, y, z planes of one 256-atom block, 1 KiB
// apart, OFF bytes past addr) that wait for their own data.
template <int OFF>
__device__ __forceinline__ void read_block(unsigned addr, f4v& p0, f4v& p1, f4v& p2) {
  static_assert(OFF >= 0 && OFF + 2048 < 65536, "ds offset field");
  asm volatile(
      "ds_read_b128 %0, %3 offset:%4\n\t"
      "ds_read_b128 %1, %3 offset:%5\n\t"
      "ds_read_b128 %2, %3 offset:%6\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(p0), "=&v"(p1), "=&v"(p2)   // early clobber: results must not reuse the address register
      : "v"(addr), "i"(OFF), "i"(OFF + 1024), "i"(OFF + 2048)
      : "memory");
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xF, true);
  return __builtin_bit_cast(double, (long long)(unsigned)lo | ((long long)hi << 32));
}

// Sum over each row of 16 lanes (every lane of the row receives it).
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);   // row_half_mirror
  v += dpp_f64<0x140>(v);   // row_mirror
  return v;
}

// Sum over the whole wave; lane 63 receives the total (rows 1 and 3 add the
// last lane of the row below, then rows 2 and 3 add lane 31).  Rows that a
// broadcast does not write receive 0 and keep their value.
__device__ __forceinline__ double wave_sum_to63(double v) {
  v = row_sum16(v);
  v += dpp_f64<0x142, 0xA>(v);   // row_bcast:15
  v += dpp_f64<0x143, 0xC>(v);   // row_bcast:31
  return v;
}

// 64-bit lane exchanges through gfx950's swap instructions.  swap32: lanes
// 32-63 of a trade places with lanes 0-31 of b, so afterwards a holds
// (a[0..31], b[0..31]) and b holds (a[32..63], b[32..63]).  swap16: the same
// between the odd rows of a and the even rows of b (rows of 16 lanes), so a
// holds rows (a0, b0, a2, b2) and b rows (a1, b1, a3, b3).
__device__ __forceinline__ double join_f64(unsigned lo, unsigned hi) {
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | (unsigned long long)lo);
}
__device__ __forceinline__ void swap32_f64(double& a, double& b) {
  const unsigned long long ia = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ib = __builtin_bit_cast(unsigned long long, b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ia, (unsigned)ib, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
  a = join_f64(lo[0], hi[0]);
  b = join_f64(lo[1], hi[1]);
}
__device__ __forceinline__ void swap16_f64(double& a, double& b) {
  const unsigned long long ia = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ib = __builtin_bit_cast(unsigned long long, b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ia, (unsigned)ib, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
  a = join_f64(lo[0], hi[0]);
  b = join_f64(lo[1], hi[1]);
}

// Wave sums of nine values, stored to out[0..8] by the lanes that end up
// holding them.  Transposed halving: a swap32 and one add fold a pair of
// values into one register (value 2k in lanes 0-31, 2k+1 in lanes 32-63),
// a swap16 and one add fold two of those into one register holding four
// values (rows: 4k, 4k+2, 4k+1, 4k+3), and a row sum finishes each row, so
// 9 values cost 5 + 3 folds and 3 row sums instead of 9 full-wave sums.
__device__ __forceinline__ void wave_sum9_store(const double v[9], double* out, int lane) {
  double w[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double a = v[2 * k], b = (2 * k + 1 < 9) ? v[2 * k + 1] : 0.0;
    swap32_f64(a, b);
    w[k] = a + b;
  }
  double u[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double a = w[2 * k], b = (2 * k + 1 < 5) ? w[2 * k + 1] : 0.0;
    swap16_f64(a, b);
    u[k] = a + b;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) u[k] = row_sum16(u[k]);
  if ((lane & 15) == 15) {
    const int r = lane >> 4;
    const int off = r == 1 ? 2 : (r == 2 ? 1 : r);   // rows hold values (0, 2, 1, 3) of each group of four
    out[off] = u[0];
    out[4 + off] = u[1];
    if (r == 0) out[8] = u[2];
  }
}

// Minimum over each row of 16 lanes (every lane of the row receives it).
// Lanes must hold finite values or +inf.
__device__ __forceinline__ double row_min16(double v) {
  v = fmin(v, dpp_f64<0xB1>(v));
  v = fmin(v, dpp_f64<0x4E>(v));
  v = fmin(v, dpp_f64<0x141>(v));
  v = fmin(v, dpp_f64<0x140>(v));
  return v;
}

}  // namespace pcv
