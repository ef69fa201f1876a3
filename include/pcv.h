/*
 * pcv.h -- C ABI of the MI355X (gfx950) path-collective-variable library.
 *
 * Path collective variables after Pazurikova, Olha, Krenek, Spiwok,
 * "Acceleration of Mean Square Distance Calculations with Floating Close
 * Structure in Metadynamics Simulations" (arXiv:1801.02362):
 *
 *   D(x, a_i)  Eq. 3: mean square distance after optimal superposition
 *              (weighted centring, then the rotation from the top eigenpair
 *              of the 4x4 quaternion matrix, Section 3);
 *   s(x)       Eq. 2 with the landmark index as property (Section 2):
 *              s = sum_i q_i exp(-lambda D_i) / sum_i exp(-lambda D_i),
 *              q_i = i (1-based) unless the caller passes properties;
 *   z(x)       -(1/lambda) ln sum_i exp(-lambda D_i) (distance from the path);
 *   ds/dx, dz/dx   by the chain rule over Eq. 4 (exact) or Eq. 6 (close
 *              structure), with respect to the raw (uncentred) coordinates;
 *   Algorithm 2   the floating close structure y: every call superposes y
 *              onto x exactly; if D(x, y) > epsilon (strict) y <- x and all
 *              landmark rotations are recomputed and saved, otherwise each
 *              landmark rotation is approximated by R_xy R_{a_i y} (Eq. 5).
 *
 * Units: nm and nm^2; lambda in nm^-2.  Weights are normalised to sum to
 * one; by default one set serves alignment and displacement (w = w'), and
 * pcv_set_displacement_weights() gives the distance its own set.
 *
 * Memory: every coordinate, gradient and result pointer named "device" is
 * HIP device memory owned by the caller (for example a torch tensor); the
 * library never frees it.  Coordinates are AoS [n][3] (or [L][n][3]) in the
 * handle's precision: float for PCV_FP32, double for PCV_FP64.  "host"
 * pointers are read during the call only.  The handle owns its own device
 * copies of the landmarks and all workspace; the evaluation calls allocate
 * nothing (the stated exceptions: pcv_path_lambda, the first
 * pcv_eval_properties call, and HIP events while kernel timing is on).
 *
 * Streams: all work is enqueued on the handle's stream and returns without
 * waiting (except where stated).  Results land in device memory; the caller
 * synchronises that stream before reading them on the host.
 *
 * Errors: every entry point returns a pcv_status; no exception crosses the
 * ABI.  pcv_last_error() gives a message for the last failing call on a
 * handle.  A non-finite input structure is detected on the device: outputs
 * are filled with NaN, the close-structure state and counters are left
 * unchanged, and pcv_check() reports PCV_ENONFINITE.
 *
 * Threads: a handle is not thread-safe; use one handle per host thread.
 */
#ifndef PCV_H
#define PCV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pcv_status {
  PCV_OK = 0,
  PCV_EINVAL = -1,        /* bad argument (null pointer, negative size, bad option) */
  PCV_ESTATE = -2,        /* call order (e.g. evaluate before landmarks are loaded) */
  PCV_ESHAPE = -3,        /* size outside what the kernels support */
  PCV_ENONFINITE = -4,    /* NaN or Inf in an input structure */
  PCV_EHIP = -5,          /* HIP runtime error */
  PCV_ENOMEM = -6,        /* device allocation failed */
  PCV_EUNSUPPORTED = -7   /* valid request the library does not implement */
} pcv_status;

enum { PCV_FP32 = 32, PCV_FP64 = 64 };

typedef struct pcv_options {
  int device;        /* HIP device ordinal */
  void* stream;      /* hipStream_t to enqueue on; NULL = the null stream */
  int precision;     /* PCV_FP32 or PCV_FP64: coordinate and gradient type */
  double eps;        /* close-structure threshold on D(x, y), nm^2 (Section 5: 0.01) */
  int use_graph;     /* nonzero: replay each call's kernel sequence from a cached
                        hipGraph (keyed by the call's pointers); 0 (the default):
                        launch the kernels directly, which on MI355X is faster for
                        these short sequences (300 x 500 exact step 27.6 us direct,
                        35.3 us through a graph) */
} pcv_options;

typedef struct pcv_stats {
  int64_t frames;          /* close-structure calls with finite input */
  int64_t recomputes;      /* reassignments of the close structure (incl. the first call) */
  int64_t expensive_msd;   /* exact superpositions: 1 per call with a close structure + L per reassignment */
  int64_t approx_frames;   /* calls served by Eq. 5 */
  int64_t exact_evals;     /* pcv_eval calls (each L exact superpositions) */
  int64_t eigen_fallbacks; /* landmark solves that used the Jacobi fallback (degenerate spectrum) */
} pcv_stats;

typedef struct pcv_handle pcv_handle;

/* Default options: device 0, null stream, FP32, eps = 0.01 nm^2, direct launches (use_graph = 0). */
void pcv_default_options(pcv_options* opt);

/* Create a handle on opt->device.  *out receives the handle (NULL on error). */
pcv_status pcv_create(pcv_handle** out, const pcv_options* opt);

/* Release the handle and its device memory (waits for its stream). NULL is a no-op. */
pcv_status pcv_destroy(pcv_handle* h);

/*
 * Load the landmark (reference) structures a_i of Eq. 2 (Section 2).
 *   n_atoms      atoms per structure, 1 .. pcv_max_atoms()
 *   n_landmarks  L >= 1
 *   coords       device, AoS [L][n][3] in the handle precision; copied (SoA,
 *                values unchanged), so the caller may free it afterwards
 *   q            host [L] properties q_i, or NULL for q_i = i (1-based)
 *   w            host [n] non-negative weights (alignment = displacement),
 *                or NULL for uniform; normalised to sum to one
 *   lambda       sharpness > 0 (nm^-2); see pcv_path_lambda()
 * Resets the close-structure state and counters.  Synchronises the stream.
 */
pcv_status pcv_load_landmarks(pcv_handle* h, int n_atoms, int n_landmarks, const void* coords,
                              const double* q, const double* w, double lambda);

/* Largest supported n_atoms for the handle's precision. */
int pcv_max_atoms(int precision);

/*
 * lambda = factor / mean_i D(a_i, a_{i+1}) over consecutive loaded landmarks
 * (exact Eq. 3 distances computed on the device), the usual path-CV choice.
 * Writes *lambda_out (host); does NOT change the handle's lambda.
 * Synchronises the stream.  Needs L >= 2.
 */
pcv_status pcv_path_lambda(pcv_handle* h, double factor, double* lambda_out);

/* Change lambda without reloading (resets the close-structure state). */
pcv_status pcv_set_lambda(pcv_handle* h, double lambda);

/*
 * Algorithm 1 (no neighbour list): exact D to every landmark, s, z and their
 * gradients for structure x.
 *   x      device [n][3]
 *   sz     device double[2]: s, z
 *   ds_dx  device [n][3] or NULL;  dz_dx  device [n][3] or NULL
 *   msd    device double[L] (the exact D_i) or NULL
 * FP32 handles on engines 2-5 contract the landmarks with w x_c rounded to
 * FP32; s and z include the first-order correction dS/dx . (x - x') for
 * that rounding (likewise the property maps), the D_i do not (they are
 * within the FP32 MSD bound either way).
 */
pcv_status pcv_eval(pcv_handle* h, const void* x, double* sz, void* ds_dx, void* dz_dx, double* msd);

/*
 * Algorithm 2: one step with the floating close structure.  Outputs as in
 * pcv_eval; msd receives D_i on reassignment steps and the Eq. 5
 * approximations otherwise.  recomputed (device int or NULL) receives 1 on a
 * reassignment step, 0 on an approximate step, -1 for non-finite input.
 * The decision is taken on the device; no host synchronisation per call.
 */
pcv_status pcv_eval_close(pcv_handle* h, const void* x, double* sz, void* ds_dx, void* dz_dx,
                          double* msd, int* recomputed);

/* Force the next pcv_eval_close to reassign (y <- x, all rotations recomputed). */
pcv_status pcv_force_reassign(pcv_handle* h);

/* Reassign now: y <- x and recompute every saved rotation R_{a_i y}. */
pcv_status pcv_update_close(pcv_handle* h, const void* x);

/*
 * Neighbour list (Section 2; with the close structure, Section 3.2).
 * With M > 0, pcv_eval and pcv_eval_close use the M references nearest to
 * the structure, refreshed every `stride` calls (calls counted from 0 after
 * this one; call t refreshes when t is a multiple of stride; pcv_update_close
 * is not counted).  A refreshing call evaluates all L references (its s, z
 * and gradients use all of them) and keeps the M nearest, ties to the lower
 * index: pcv_eval by the exact distances, pcv_eval_close by that call's
 * distances (exact when it reassigns the close structure, Eq. 5 otherwise).
 * Other calls evaluate the members only: pcv_eval exactly, pcv_eval_close by
 * Eq. 5 -- except on a reassignment, which evaluates all L exactly (its CV
 * uses all of them) and refreshes the members' saved rotations without
 * changing the members.  Counters follow Section 6.2: expensive_msd grows by
 * L on a refreshing pcv_eval call and by M on the others; pcv_eval_close
 * counts as without a list (1 per call + L per reassignment).
 *   M       0 switches the list off; otherwise 1 <= M <= L
 *   stride  >= 1
 * PCV_EINVAL for bad M / stride; PCV_EUNSUPPORTED when L > 8192.  While a
 * list is on, the msd output of pcv_eval / pcv_eval_close must be NULL.
 * Allocates M (3 n_pad coordinates + 14 doubles) + L doubles of device
 * memory and synchronises the stream; loading landmarks switches it off.
 */
pcv_status pcv_set_neighbour_list(pcv_handle* h, int M, int stride);
/* The current members (host copy, nearest first as chosen; the first M
 * references before the first refresh).  *count = M (0 when off); members
 * (NULL: only the count) must hold `capacity` >= M ints.  Synchronises the
 * stream. */
pcv_status pcv_get_neighbour_list(pcv_handle* h, int* members, int capacity, int* count);

/*
 * Property maps with several properties per reference (Eq. 2 with a vector
 * q_i; Section 2): S_k = sum_i q_ik e^{-lambda D_i} / sum_i e^{-lambda D_i}
 * and dS_k/dx for k < P, from the exact distances (Algorithm 1, every
 * reference, whether or not a neighbour list is set).
 *   q      device double [L][P], row i = properties of landmark i
 *   S      device double [P]
 *   dS_dx  device [P][n][3] in the coordinate type, or NULL
 *   P      1..8
 * Counts as one exact evaluation (expensive_msd += L).  The first call
 * allocates L P + (chunks P 3 n_pad) doubles of scratch (kept until the next
 * landmark load); later calls allocate nothing.  Two passes over the
 * landmarks: the exact pass (rotations kept) and the gradient pass.
 */
pcv_status pcv_eval_properties(pcv_handle* h, const void* x, int P, const double* q, double* S, void* dS_dx);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation and outputs as pcv_eval_properties, with its scratch (the
 * weights W, L P doubles rounded up to 256 bytes, and the gradient-pass
 * partials, chunks P 3 n_pad doubles) taken from a fixed 16 MiB device array
 * that the library holds on every GPU it runs on until the process ends.
 * Calls no allocating routine and records no graph; launches eagerly on the
 * handle's stream.  PCV_EINVAL when the scratch would exceed 16 MiB.  Every
 * call on one GPU shares that GPU's array (each call overwrites it before
 * reading it): calls that overlap in time on one GPU (other streams, other
 * threads, other handles) race and must be serialised by the caller.
 */
pcv_status pcv_eval_properties_noalloc(pcv_handle* h, const void* x, int P, const double* q, double* S,
                                       void* dS_dx);

/*
 * Separate displacement weights w (Section 3.1, Eq. 4 with w != w'): the
 * weights given to pcv_load_landmarks stay the alignment weights w' (centre
 * of mass and rotation); w_disp sets the per-atom weights of the distance,
 *   D_i = sum_j w_j |x_c,j - R_i a_c,ij|^2   (R_i, centres by w'),
 * and its gradient then keeps the centre-of-mass and rotation terms of Eq. 4.
 *   w_disp  host [n] finite, >= 0, positive sum (normalised to sum to one),
 *           copied; NULL switches the separate weights off (D by w' again)
 * While set, pcv_eval takes a three-pass FP64-accumulating path (outputs and
 * graph reuse as before; msd receives these D_i), and pcv_eval_close,
 * pcv_update_close, pcv_eval_properties, pcv_set_neighbour_list and the
 * surrogate's fallback step return PCV_EUNSUPPORTED (pcv_set_displacement_weights
 * itself refuses while a neighbour list is on).  Allocates about
 * L (31 doubles) + 3 n_pad + chunks 12 n_pad doubles (chunks <= 64) and
 * synchronises the stream; loading landmarks switches it off.
 */
pcv_status pcv_set_displacement_weights(pcv_handle* h, const double* w_disp);

/*
 * Checkpoint and resume of the state that carries between steps (Algorithm 2
 * and the neighbour list of Section 2): the close structure y, G_y, the saved
 * rotations R_{a_i y} (Section 3.2), the first-frame and forced-reassignment
 * flags, the counters, and the neighbour list (M, stride, call count,
 * members and their saved rotations).  Landmarks, lambda, eps, weights and
 * the plan are configuration and are not part of the state.
 *   pcv_save_state: buf = host buffer of *bytes bytes, or NULL to query the
 *     size (*bytes receives it); PCV_EINVAL (and the size in *bytes) when
 *     the buffer is too small.
 *   pcv_load_state: buf = host bytes written by pcv_save_state for a handle
 *     with the same precision, atom count and landmark set (checked against
 *     a fingerprint of the landmarks: PCV_ESHAPE / PCV_EINVAL otherwise).  A
 *     saved neighbour list replaces the handle's (allocating as
 *     pcv_set_neighbour_list does).  Evaluations after a load continue
 *     exactly as they would have on the saved handle.
 * Both synchronise the stream.
 */
pcv_status pcv_save_state(pcv_handle* h, void* buf, size_t* bytes);
pcv_status pcv_load_state(pcv_handle* h, const void* buf, size_t bytes);

/* Counters (synchronises the stream). */
pcv_status pcv_get_stats(pcv_handle* h, pcv_stats* out);
pcv_status pcv_reset_stats(pcv_handle* h);

/* Synchronise the stream and report a deferred device-side error (non-finite
 * input since the last check), clearing it. */
pcv_status pcv_check(pcv_handle* h);

/*
 * Tiling of the landmark streaming kernel.  Five engines exist:
 *   engine 1  teams of `team` lanes, one landmark per team at a time, `apt`
 *             atoms per lane, `wg` threads per workgroup; every lane of a team
 *             takes part in the per-landmark eigen-solve.  Any n up to
 *             pcv_max_atoms().
 *   engine 2  split roles in a 512-thread workgroup: one solver wave, three
 *             correlation waves reading batches of `batch` landmarks from LDS
 *             (async copies), four gradient waves owning the atoms; `apt` and
 *             `aptg` are the compiled atoms per correlation / gradient lane,
 *             `team` the lanes per landmark in the correlation stage
 *             (16, 32, 64 or 192).  Needs the landmark batch to fit in LDS.
 *   engine 3  large FP32 structures: seven worker waves each own up to `apt`/4
 *           blocks of 256 atoms (apt = 4, 8, 12 or 16, so at most 7 * apt * 64
 *           atoms) and stream them through a private LDS copy ring; one solver
 *           wave; one barrier per landmark.  `team`, `aptg`, `batch` unused.
 *           The default for 5,633 to 7,168 padded atoms.
 *   engine 4  FP32 structures of up to 2,048 padded atoms (the default there,
 *           and the batched walkers' engine): seven worker waves own units
 *           (landmark lane, 256-atom block), `apt`/4 = 2 or 3 units each, and
 *           `batch` landmarks (lanes) are processed per step, at most
 *           floor(7 * (apt / 4) / blocks); one solver wave solves the lanes side
 *           by side.  `team`, `aptg` unused.
 *   engine 5  FP32 structures of up to 7 * (apt / 4) * 256 atoms (apt = 4, 8
 *           or 12): engine 3's blocks and solver with the landmark blocks
 *           streamed HBM -> registers by range-checked buffer loads (two
 *           register sets and one LDS slot per worker).  The default for 2,049
 *           to 5,376 padded atoms.  `team`, `aptg`, `batch` unused.
 * `grid` is an output; `items` <= 0 selects the default number of work items.
 */
typedef struct pcv_plan {
  int engine;
  int wg;
  int apt;
  int team;
  int aptg;
  int batch;
  int grid;
  int items;
} pcv_plan;

pcv_status pcv_get_plan(pcv_handle* h, pcv_plan* out);
/* Validate and apply a plan (synchronises the stream; PCV_EUNSUPPORTED if the
 * tiling is not compiled in or cannot hold the loaded structure). */
pcv_status pcv_set_plan(pcv_handle* h, const pcv_plan* plan);

/*
 * Kernel timing for roofline measurements.  While enabled, calls run eagerly
 * (no graph replay) and HIP events are recorded on the handle's stream around
 * every launch of the landmark streaming kernel.  pcv_get_kernel_timing
 * synchronises and returns the summed duration (ms) and launch count since
 * timing was enabled.
 */
pcv_status pcv_set_kernel_timing(pcv_handle* h, int enable);
pcv_status pcv_get_kernel_timing(pcv_handle* h, double* engine_ms, int64_t* engine_launches);

/*
 * Streaming-read ceiling of the device (a measurement utility, not part of
 * the method): reads `bytes` of device memory at src once with the landmark
 * engines' load path (16-byte non-temporal loads, two sets per wave in
 * flight, eight waves per workgroup) and writes, per workgroup, the FP64 sum
 * of its contiguous chunk's floats to wg_sums[0 .. grid).  src must be
 * 16-byte aligned, bytes a multiple of 16, 1 <= grid <= 65536.  Asynchronous
 * on `stream` (a hipStream_t or NULL); allocates nothing.
 */
pcv_status pcv_stream_read(const void* src, size_t bytes, double* wg_sums, int grid, void* stream);

const char* pcv_status_string(pcv_status s);
const char* pcv_last_error(const pcv_handle* h);

/* ------------------------------------------------------------------------
 * Batched walkers: many independent (structure, landmark set) problems of
 * uneven size evaluated by one persistent launch of the landmark engine
 * (exact Algorithm 1 per walker), optionally replayed from a hipGraph.
 * ---------------------------------------------------------------------- */
typedef struct pcv_batch pcv_batch;

pcv_status pcv_batch_create(pcv_batch** out, const pcv_options* opt);
pcv_status pcv_batch_destroy(pcv_batch* b);

/*
 * Load W walkers.
 *   n_atoms[W], n_landmarks[W]   host; n_atoms[w] <= pcv_max_atoms()
 *   coords      device, concatenation over walkers of AoS [L_w][n_w][3]
 *   lambdas     host [W]
 * Properties are q_i = i and weights uniform per walker.  Synchronises.
 */
pcv_status pcv_batch_load(pcv_batch* b, int n_walkers, const int* n_atoms, const int* n_landmarks,
                          const void* coords, const double* lambdas);

/*
 * Choose tiles and schedule.  tune = 0: built-in heuristic; tune = 1: time
 * every candidate on the device (each must reproduce the heuristic plan's
 * results within tolerance to be eligible) and keep the fastest; the choice
 * is cached in the JSON file named by cache_path (may be NULL).
 * Synchronises.  Needs a prior pcv_batch_load.
 */
pcv_status pcv_batch_plan(pcv_batch* b, int tune, const char* cache_path);

/*
 * Evaluate all walkers:
 *   x_all   device, concatenation of [n_w][3]
 *   sz_all  device double[W][2]
 *   ds_all, dz_all  device, concatenation of [n_w][3], or NULL
 */
pcv_status pcv_batch_eval(pcv_batch* b, const void* x_all, double* sz_all, void* ds_all, void* dz_all);

/* Description of the chosen plan (static string owned by the batch). */
/* Kernel timing of the batch's landmark streaming launch (as
 * pcv_set_kernel_timing / pcv_get_kernel_timing for a single handle: while
 * enabled, calls run eagerly with HIP events around the engine launch; the
 * getter synchronises and returns the summed ms and launch count). */
pcv_status pcv_batch_set_kernel_timing(pcv_batch* b, int enable);
pcv_status pcv_batch_get_kernel_timing(pcv_batch* b, double* engine_ms, int64_t* engine_launches);
const char* pcv_batch_plan_string(const pcv_batch* b);
const char* pcv_batch_last_error(const pcv_batch* b);

/* ------------------------------------------------------------------------
 * Learned surrogate (a project addition beside the paper's method): an MLP
 * maps a structure, superposed onto a fixed reference with the Eq. 3 /
 * Section 3 rotation, to the standardised path variables (s, z) of Eq. 2;
 * ds/dx and dz/dx come from its backward pass chained through the alignment.
 * Layers: 3n -> H -> H -> H -> 2 with SiLU.  GEMMs run on the matrix cores
 * with BF16 operands and FP32 accumulation; master weights, Adam moments,
 * biases and activations before rounding are FP32.
 *
 * Parameters are one flat FP32 array: for l = 1..4, W_l [fan_in][fan_out]
 * (row-major) followed by b_l [fan_out].  Initial values are the caller's
 * (the library draws no random numbers).
 * ---------------------------------------------------------------------- */
typedef struct pcv_mlp pcv_mlp;

typedef struct pcv_mlp_stats {
  int64_t steps;            /* pcv_mlp_step calls */
  int64_t surrogate_steps;  /* answered by the surrogate (drift <= epsilon) */
  int64_t exact_steps;      /* answered exactly (drift > epsilon, first step, forced) */
  int64_t judged_steps;     /* exact steps that had an anchor: the surrogate's answer was judged */
  double max_abs_ds;        /* judge: max |s_surrogate - s_exact| over judged steps */
  double max_abs_dz;
  double mean_abs_ds;
  double mean_abs_dz;
} pcv_mlp_stats;

/*
 * Create a surrogate for structures of n_atoms atoms.
 *   opt         device and stream (FP32 only; graphs per opt->use_graph)
 *   hidden      hidden width H (>= 16)
 *   max_batch   largest batch of any later call
 *   ref         host [n][3] FP64 reference structure the inputs are aligned to
 *   w           host [n] alignment weights or NULL (uniform); normalised
 * Parameters start at zero: call pcv_mlp_set_params before use.
 */
pcv_status pcv_mlp_create(pcv_mlp** out, const pcv_options* opt, int n_atoms, int hidden, int max_batch,
                          const double* ref, const double* w);
pcv_status pcv_mlp_destroy(pcv_mlp* m);
long long pcv_mlp_param_count(const pcv_mlp* m);
/* Host FP32 parameters in (resets Adam's moments and step) / out.  Synchronise. */
pcv_status pcv_mlp_set_params(pcv_mlp* m, const float* params, long long count);
pcv_status pcv_mlp_get_params(pcv_mlp* m, float* params, long long count);
/* Host copy of the gradients of the last pcv_mlp_train_step (same layout). */
pcv_status pcv_mlp_get_grads(pcv_mlp* m, float* grads, long long count);
/* Output scaling: s = mean[0] + sd[0] y0, z = mean[1] + sd[1] y1. */
pcv_status pcv_mlp_set_scaling(pcv_mlp* m, const double mean[2], const double sd[2]);

/*
 * Align B structures (device [B][n][3] FP32) onto the reference: x' = R^T
 * (x - c), device outputs [B][3n] as BF16 bits (uint16) and/or FP32 (either
 * may be NULL).  Used to build training inputs.
 */
pcv_status pcv_mlp_align(pcv_mlp* m, const float* x, int B, uint16_t* xa_bf16, float* xa_f32);

/* Network outputs (standardised, device [B][2] FP32) for B aligned BF16 inputs [B][3n]. */
pcv_status pcv_mlp_forward(pcv_mlp* m, const uint16_t* inputs, int B, float* y);

/*
 * One Adam step (beta 0.9 / 0.999, eps 1e-8, learning rate lr) on the mean
 * over the batch of the squared error summed over both outputs.
 *   inputs   device [B][3n] BF16 aligned structures
 *   targets  device [B][2] FP32 standardised (s, z)
 *   loss     device float or NULL (the loss before the step)
 */
pcv_status pcv_mlp_train_step(pcv_mlp* m, const uint16_t* inputs, const float* targets, int B, float lr,
                              float* loss);

/*
 * Surrogate (s, z) and gradients for B raw structures.
 *   x      device [B][n][3] FP32;  sz  device double [B][2]
 *   ds_dx, dz_dx   device [B][n][3] FP32 or NULL (alignment derivative included)
 */
pcv_status pcv_mlp_eval(pcv_mlp* m, const float* x, int B, double* sz, float* ds_dx, float* dz_dx);

/*
 * One step with fallback (Algorithm 2's drift test with the surrogate in
 * place of Eq. 5): the exact handle h (FP32, same n) superposes its close
 * structure y onto x; if D(x, y) > epsilon (or on its first step / when
 * forced) the exact path answers, y <- x, and the surrogate's error on this
 * frame is recorded (the judge); otherwise the surrogate answers, anchored on
 * the last exact step: s = f_s(x) + (s_exact(y) - f_s(y)), likewise z
 * (before the first exact step, f(x) itself).  Gradients are the network's.
 *   x      device [n][3];  sz device double[2];  ds_dx, dz_dx device [n][3] or NULL
 *   used_surrogate   device int or NULL: 1 surrogate, 0 exact
 * The decision stays on the device (no host synchronisation).
 */
pcv_status pcv_mlp_step(pcv_mlp* m, pcv_handle* h, const float* x, double* sz, float* ds_dx, float* dz_dx,
                        int* used_surrogate);
pcv_status pcv_mlp_get_stats(pcv_mlp* m, pcv_mlp_stats* out);
pcv_status pcv_mlp_reset_stats(pcv_mlp* m);

/*
 * Checkpoint and resume of the surrogate's training state (a project
 * addition): the FP32 master parameters, Adam's two moment vectors and step
 * count, the output scaling and the fallback step's anchor.  The network
 * shape (atoms, width) and the reference structure are configuration.
 *   pcv_mlp_save_state: buf = host buffer of *bytes bytes, or NULL to query
 *     the size (*bytes receives it); PCV_EINVAL (and the size in *bytes)
 *     when the buffer is too small.
 *   pcv_mlp_load_state: buf = host bytes written by pcv_mlp_save_state for a
 *     surrogate of the same shape (PCV_ESHAPE otherwise, PCV_EINVAL for a
 *     damaged buffer).  Training steps after a load continue exactly as
 *     they would have on the saved handle.
 * Both synchronise the stream.
 */
pcv_status pcv_mlp_save_state(pcv_mlp* m, void* buf, size_t* bytes);
pcv_status pcv_mlp_load_state(pcv_mlp* m, const void* buf, size_t bytes);
const char* pcv_mlp_last_error(const pcv_mlp* m);

/* ------------------------------------------------------------------------
 * Metadynamics bias on the path variables (Eq. 1).
 *
 * Hills w exp(-(s - s_k)^2 / (2 sigma_s^2) - (z - z_k)^2 / (2 sigma_z^2))
 * deposited at earlier CV values are summed on a regular (s, z) grid, as in
 * the paper's runs (one height per hill, one width per CV; the paper's single
 * sigma is sigma_s = sigma_z).  Every node holds the exact hill sum and its
 * derivatives dV/ds, dV/dz, d2V/dsdz; between nodes the bias is their bicubic
 * Hermite interpolant; outside the grid it is zero.  The handle owns the
 * grid (4 ns nz doubles of device memory); all calls are asynchronous on the
 * options' stream unless stated.  A bias handle is not thread-safe.
 */
typedef struct pcv_bias pcv_bias;
typedef struct pcv_bias_options {
  int device;              /* HIP device ordinal */
  void* stream;            /* hipStream_t; NULL = the null stream */
  double s_min, s_max;     /* s range of the grid (nodes s_min + i (s_max - s_min)/(ns - 1)) */
  int ns;                  /* nodes along s, >= 2 */
  double z_min, z_max;     /* z range (nm^2) */
  int nz;                  /* nodes along z, >= 2 (ns nz <= 2^28) */
  double height;           /* hill height w (energy units) */
  double sigma_s, sigma_z; /* hill widths, > 0 */
} pcv_bias_options;

/* PCV_EINVAL for a bad range, size, height or width; PCV_ENOMEM / PCV_EHIP. */
pcv_status pcv_bias_create(pcv_bias** out, const pcv_bias_options* opt);
pcv_status pcv_bias_destroy(pcv_bias* b);

/* Eq. 1, one more hill at the CV values in device memory: sz_dev[0] = s,
 * sz_dev[1] = z (for example the sz output of pcv_eval_close).  Non-finite
 * values deposit nothing.  Deposits are applied in stream order. */
pcv_status pcv_bias_deposit(pcv_bias* b, const double* sz_dev);

/* Bias at the CV values sz_dev (device double[2]) and its gradient on the
 * atoms, dV/dx_k = dV/ds ds/dx_k + dV/dz dz/dx_k (the bias force is its
 * negative).
 *   n_atoms, precision   size and coordinate type (PCV_FP32 / PCV_FP64) of
 *                        ds_dx, dz_dx and grad_out, device [n][3]
 *   grad_out             device [n][3] or NULL (then ds_dx, dz_dx unused);
 *                        must not alias ds_dx or dz_dx
 *   v_dev                device double[3] or NULL: V, dV/ds, dV/dz
 *   in_range_dev         device int or NULL: 1 inside the grid, 0 outside
 *                        (V and its derivatives are 0 there) */
pcv_status pcv_bias_gradient(pcv_bias* b, const double* sz_dev, int n_atoms, int precision, const void* ds_dx,
                             const void* dz_dx, void* grad_out, double* v_dev, int* in_range_dev);
/* Hills deposited so far (host counter). */
pcv_status pcv_bias_hills(const pcv_bias* b, long long* count);
/* Copy the grid to host memory [4][ns][nz] (V, dV/ds, dV/dz, d2V/dsdz);
 * synchronises the stream. */
pcv_status pcv_bias_get_grid(pcv_bias* b, double* host_out);
const char* pcv_bias_last_error(const pcv_bias* b);

#ifdef __cplusplus
}
#endif

#endif /* PCV_H */
