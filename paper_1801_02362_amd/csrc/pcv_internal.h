// Internal descriptors shared by the kernels and the C ABI implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcv {

// Engine modes (the per-landmark step of the landmark streaming kernel).
enum Mode : int {
  MODE_EXACT = 0,       // Algorithm 1: solve every landmark's rotation (Eq. 3)
  MODE_EXACT_SAVE = 1,  // Algorithm 2, reassignment: as EXACT and save R_{a_i y}
  MODE_APPROX = 2,      // Algorithm 2, usual step: R_xy R_{a_i y} (Eq. 5)
};

// One (structure, landmark set) problem as the engine sees it.  Landmark
// coordinates are SoA [L][3][n_pad] exactly as the caller gave them (not
// re-rounded); their weighted centroids and Ga = sum_j w_j |a_j - c|^2 are
// FP64.  xw = w_j * x_c,j in FP64 (SoA [3][n_pad]) feeds the correlation
// and, in the merges, the residuals x_c - R a.
struct Problem {
  const void* A;
  const double* ca;     // [L][3]
  const double* Ga;     // [L]
  const double* q;      // [L]
  const double* w;      // [n_pad], normalised, zero padded
  const double* xw;     // [3][n_pad]
  const double* Gx;     // [1]
  const double* Rxy;    // [9] (APPROX)
  double* Rsave;        // [L][9]: read in APPROX, written in EXACT_SAVE
  double* hdr;          // [n_slots][4]: m, Z, S, q0 per item
  void* vec;            // per slot: U [3][n_pad] (coordinate type), then V [3][n_pad] (FP64)
  long long* fallbacks; // counter of Jacobi fallbacks (may be null)
  const double* Gx32;   // [1] sum_j (w_j x_j rounded to T)^2 / w_j - |xres|^2 (split-role engine)
  const double* xres;   // [3] sum_j (w_j x_j rounded to T): centring residual of that rounding
  int n, n_pad, L, ts, n_slots;
  int bsz;              // split-role engine: landmarks per pipeline batch
  int cg;               // split-role engine: lanes per landmark in the correlation stage
  int out_off;          // atom offset of this problem in concatenated inputs/outputs
  int out_idx;          // index of this problem's (s, z) pair
  double lam;
  const float* xw32;    // [3][n_x] w_j x_c,j rounded to FP32, zero past n (large-structure engine)
  int n_x;              // plane stride of xw32: n_pad rounded up to 256
  // FP32 engines 2-5 contract with fl32(w_j x_c,j): their distances, s and z
  // are those of the structure x' = fl32(w x_c) / w.  With x_rounded set,
  // (s, z) gain the first-order difference dS/dx . (x - x'): each exact
  // merge workgroup leaves its share in corr ([3 ceil(n / 64)][2]) and the
  // kernel after the merge adds the shares in workgroup order.
  int x_rounded;
  double* corr;
  // Approximate steps of engine 4: per item the 3x3 sums XU and XV of
  // T_i = sum_j (w x_c)_j (R_i (a_ij - c_i))^T weighted like the partials U
  // and V ([n_slots][18]); null elsewhere.  With them the close merge is one
  // kernel (Eq. 6's G comes from the items, not from every atom).
  double* xuv;
};

struct Item {
  int prob, i0, i1, slot;
};

// Global-memory access through an explicit address space: descriptor
// pointers are generic, and without this the compiler emits flat loads, which
// also occupy the LDS counter and serialise LDS waits behind HBM loads.
template <typename T>
__device__ __forceinline__ T ldg(const T* p) {
  return *((const __attribute__((address_space(1))) T*)p);
}
template <typename T>
__device__ __forceinline__ void stg(T* p, T v) {
  *((__attribute__((address_space(1))) T*)p) = v;
}
// Streaming (non-temporal) global load: data read once.
template <typename T>
__device__ __forceinline__ T ldg_nt(const T* p) {
  return __builtin_nontemporal_load((const __attribute__((address_space(1))) T*)p);
}

// Partial accumulators of one work item: U = sum e (q - q0) r in the
// coordinate type, V = sum e r in FP64 (the merge multiplies V by q0 - s).
template <typename T>
__host__ __device__ inline size_t partial_bytes(int n_pad) {
  return (size_t)3 * n_pad * (sizeof(T) + sizeof(double));
}
template <typename T>
__host__ __device__ inline T* partial_u(void* vec, int slot, int n_pad) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(vec) + (size_t)slot * partial_bytes<T>(n_pad));
}
template <typename T>
__host__ __device__ inline double* partial_v(void* vec, int slot, int n_pad) {
  return reinterpret_cast<double*>(reinterpret_cast<char*>(partial_u<T>(vec, slot, n_pad)) +
                                   (size_t)3 * n_pad * sizeof(T));
}

// Launches gated by the close-structure flag (Algorithm 2).  run_if = 0 or
// 1: the launch works only when the flag equals it.  run_if = kRunDual: one
// launch serves both branches, the reassignment (probs + MODE_EXACT_SAVE)
// when the flag is 1 and the approximate step (probs + MODE_APPROX) when it
// is 0, with probs pointing at the handle's problem array; nothing for -1.
constexpr int kRunDual = -2;
__device__ __forceinline__ bool gate_launch(const int* flag, int run_if, int& mode, const Problem*& probs) {
  if (flag == nullptr) return true;
  const int f = __builtin_amdgcn_readfirstlane(*flag);   // one value for the whole wave
  if (run_if != kRunDual) return f == run_if;
  if (f == 1) {
    mode = MODE_EXACT_SAVE;
    probs += MODE_EXACT_SAVE;
    return true;
  }
  if (f == 0) {
    mode = MODE_APPROX;
    probs += MODE_APPROX;
    return true;
  }
  return false;
}

// Output base pointers of one call (problem p writes at atom offset
// out_off and (s, z) pair out_idx).
struct Outs {
  void* ds;     // [n][3] coordinate type, or null
  void* dz;     // [n][3] or null
  double* sz;   // [2] per problem
  int* rec;     // close step: 1 reassigned, 0 approximate, -1 bad input (or null)
};

struct PrepArgs {
  long long x_off;  // atom offset of this structure in the caller's AoS input
  const double* w;  // [n_pad]
  double* xw;       // [3][n_pad]
  double* Gx;       // [1]
  double* Gx32;     // [1] see Problem::Gx32
  double* xres;     // [3] see Problem::xres
  int* status;      // [1]: sticky, set to 1 on non-finite input
  long long* counters;  // optional: CNT_EVALS / CNT_EXPENSIVE for Algorithm 1
  int n, n_pad, L;
  float* xw32;          // optional: FP32 copy of xw, plane stride n_x (padding stays zero)
  int n_x;
};

// Device-resident close-structure state (Algorithm 2).
struct CloseArgs {
  double* y64;      // [3][n_pad] centred close structure
  double* Gy;       // [1]
  double* Fxy;      // [10] quaternion matrix of y onto x
  double* lamxy;    // [1]
  double* qxy;      // [4]
  double* Rxy;      // [9]
  double* Dxy;      // [1]
  int* flag;        // [1]: 1 reassign, 0 approximate, -1 skip (bad input)
  int* init;        // [1]
  int* force;       // [1]
  long long* counters;  // [8]: frames, recomputes, expensive_msd, approx_frames
  double eps;
  int L;
  unsigned* ticket;     // [1] arrival count of the close merge's workgroups (0 between launches)
};

enum Counter { CNT_FRAMES = 0, CNT_RECOMPUTES = 1, CNT_EXPENSIVE = 2, CNT_APPROX = 3,
               CNT_EVALS = 4, CNT_FALLBACK = 5, CNT_N = 8 };

struct EngineCfg {
  int wg;    // threads per workgroup
  int apt;   // atoms per thread
};

// Split-role engine instantiation: correlation waves (the other 7 - ncw
// non-solver waves do gradients), atoms per correlation lane / gradient lane.
struct Engine2Cfg {
  int ncw;
  int aptc;
  int aptg;
};

// ---- launchers (pcv_kernels.hip) -------------------------------------------
// All return hipSuccess or the launch error.
template <typename T>
hipError_t launch_load_landmarks(const T* in, T* A, double* ca, double* Ga, const double* w,
                                 int n, int n_pad, int L, hipStream_t st);
template <typename T>
hipError_t launch_pair_msd(const T* A, const double* ca, const double* Ga, const double* w,
                           int n, int n_pad, int L, double* out, hipStream_t st);
template <typename T>
hipError_t launch_prep(const PrepArgs* d_args, const void* x_base, int n_prob, int max_n, hipStream_t st);
template <typename T>
hipError_t launch_prep_close(PrepArgs pa, const void* x, CloseArgs ca, Outs outs, hipStream_t st);
template <typename T>
hipError_t launch_engine(EngineCfg cfg, int grid, size_t lds_bytes, const Problem* probs,
                         const Item* items, const int* wg_off, int mode, const int* flag,
                         int run_if, double* dout, hipStream_t st);
template <typename T>
hipError_t launch_merge_exact(const Problem* probs, Outs outs, int n_prob, int max_n_pad,
                              const int* flag, int run_if, hipStream_t st, bool rounded);
// prob_exact (may be null): the reassignment's problem; when given, the
// same launch also performs the exact merge on reassignment steps, so the
// separate flag-gated launch_merge_exact is not needed.  one_pass: the
// approximate problem carries per-item XU / XV sums (Problem::xuv) and the
// merge is a single pass.  Otherwise structures of up to kCloseFuseMaxPad
// padded atoms finish in the last workgroup of the first kernel (one launch
// per step) and larger ones use a second, single-workgroup kernel.
constexpr int kCloseFuseMaxPad = 1024;
// Most work items (slots) of one problem; the one-pass close merge keeps
// their log-sum-exp weights in LDS.
constexpr int kMaxCloseSlots = 2048;
template <typename T>
hipError_t launch_merge_close(const Problem* prob, int n_pad, Outs outs, CloseArgs ca, double* gtmp,
                              hipStream_t st, const Problem* prob_exact = nullptr, bool one_pass = false);
hipError_t launch_set_int(int* p, int v, hipStream_t st);
hipError_t launch_count(long long* counters, int which, long long add, hipStream_t st);

template <typename T>
hipError_t launch_engine2(int ncw, int aptc, int aptg, int grid, size_t lds, int lbuf_bytes, int bmax,
                          const Problem* probs, const Item* items, const int* wg_off, int mode,
                          const int* flag, int run_if, double* dout, hipStream_t st);
void engine2_configs(bool fp64, int* ncw, int* aptc, int* aptg, int* count);
hipError_t engine2_init_attributes();
size_t engine2_lds_bytes(size_t lbuf, int bmax);

// Large-structure engine (FP32 only): bpw = 256-atom blocks per worker wave
// (1 to 4; a structure may have up to 7 * bpw blocks).
template <typename T>
hipError_t launch_engine3(int bpw, int grid, const Problem* probs, const Item* items, const int* wg_off, int mode,
                          const int* flag, int run_if, double* dout, hipStream_t st);
int engine3_max_blocks(int bpw);
// Register-stream variant of engine 3 (FP32): the same blocks and solver,
// landmarks streamed HBM -> registers; bpw 1 to 3.
template <typename T>
hipError_t launch_engine5(int bpw, int grid, const Problem* probs, const Item* items, const int* wg_off, int mode,
                          const int* flag, int run_if, double* dout, hipStream_t st);
int engine5_max_blocks(int bpw);

// Multi-landmark engine (FP32, n_pad <= 2048): spw = units (landmark lane,
// 256-atom block) per worker wave (2 or 3).  A problem's Problem::bsz is its
// landmark lanes K per step, at most engine4_lanes(n_pad, spw) (0: the
// structure does not fit).
template <typename T>
hipError_t launch_engine4(int spw, int grid, const Problem* probs, const Item* items, const int* wg_off, int mode,
                          const int* flag, int run_if, double* dout, hipStream_t st);
int engine4_lanes(int n_pad, int spw);


// Neighbour list: the full landmark set's stored data and the compact list
// set the members are gathered into.
struct NlGather {
  const int* members;   // [M] indices into the full set
  int M, n_pad;
  const void* A;        // [L][3][n_pad] coordinate type
  const double* ca;     // [L][3]
  const double* Ga;     // [L]
  const double* q;      // [L]
  const double* Rsave;  // [L][9]
  void* A_nl;           // [M][3][n_pad]
  double* ca_nl;        // [M][3]
  double* Ga_nl;        // [M]
  double* q_nl;         // [M]
  double* Rsave_nl;     // [M][9]
};
// The M smallest of D[0..N) (nearest first, ties to the lower index) into
// members; N <= nl_select_max().
hipError_t launch_nl_select(const double* D, int N, int M, int* members, hipStream_t st);
int nl_select_max();
// Gather the members' rows; skipped unless flag is null or *flag == run_if.
template <typename T>
hipError_t launch_nl_gather(const NlGather& g, const int* flag, int run_if, hipStream_t st);

// Property maps (several properties per reference): the exact pass's
// distances D and rotations R, the landmark set and the properties.
constexpr int kPropsMax = 8;
struct PropsArgs {
  const void* A;        // [L][3][n_pad] coordinate type
  const double* ca;     // [L][3]
  const double* R;      // [L][9] rotations of the exact pass
  const double* D;      // [L] distances of the exact pass
  const double* w;      // [n_pad] normalised weights
  int L, n, n_pad, P;
  // With x_rounded (FP32 engines, see Problem::x_rounded) the gradient pass
  // always runs and S_k gains dS_k/dx . (x - x'): xw is w x_c in FP64
  // ([3][n_pad]), corr holds props_corr_doubles(n) shares per component.
  const double* xw;
  int x_rounded;
  double* corr;
};
// Landmark chunks of the gradient pass (its partials: chunks x P x 3 x n_pad doubles).
int props_chunks(int n_pad, int L);
// Reduce workgroups per component (the rounding-correction shares per component).
int props_corr_doubles(int n);
// S [P] (device), W [L][P] scratch, part scratch, dS [P][n][3] or null.
template <typename T>
hipError_t launch_props(const PropsArgs& a, const double* q, double lam, double* S, double* W, double* part,
                        void* dS, hipStream_t st);

// Separate displacement weights (w != w'): device buffers of the handle.
struct F2Args {
  const void* A;           // [L][3][n_pad] coordinate type
  const double* ca;        // [L][3] centroids by the alignment weights
  const double* Ga;        // [L] sum w' |a_c|^2
  double* Gaw;             // [L] sum w |a_c|^2
  double* mua;             // [L][3] sum w a_c
  double* Caa;             // [L][6] sum w a_c a_c^T (xx xy xz yy yz zz)
  const double* wa;        // [n_pad] alignment weights w' (normalised)
  const double* wd;        // [n_pad] displacement weights w (normalised)
  double* xc;              // [3][n_pad] centred frame (FP64)
  double* fs;              // [11]: G_x^{w'}, G_x^w, mu_x[3], K_c[3], K_p[3]
  double* Rl;              // [L][9] rotations
  double* Gl;              // [L][9] rotation adjoints Gamma
  double* Rmu;             // [L][3] R mu_a
  double* cw;              // [L] ds weights c_i
  double* pw;              // [L] dz weights p_i
  double* part;            // [chunks][12][n_pad]
  const double* q;         // [L] properties
  int* status;             // sticky non-finite flag
  long long* fallbacks;    // Jacobi fallbacks (may be null)
  double lam;
  int L, n, n_pad;
};
int f2_chunks(int n_pad, int L);
template <typename T>
hipError_t launch_f2_stats(const F2Args& a, hipStream_t st);
template <typename T>
hipError_t launch_f2_eval(const F2Args& a, const void* x, double* sz, void* ds, void* dz, double* dout,
                          long long* counters, hipStream_t st);

bool engine_supported(EngineCfg cfg, bool fp64);
void engine_configs(bool fp64, EngineCfg* out, int* count);   // the compiled menu
hipError_t engine_init_attributes();
size_t engine_lds_bytes(EngineCfg cfg, int ts, bool fp64);

}  // namespace pcv
