/*
 * sd.h -- C ABI of the MI355X (gfx950) all-pairs Stokesian-dynamics library.
 *
 * Computes, for N spheres of radius a in a fluid of viscosity eta, the
 * mobility product of Eq. (7a) of Kopp & Hoefling (2012),
 *     v_i = mu0 F_i + sum_{j != i} T(r_i - r_j) F_j,   mu0 = 1/(6 pi eta a),
 * with the Rotne-Prager pair tensor T of Eq. (7b) or the Oseen tensor G of
 * Eq. (4), and advances positions with it (Sec. 3.1, steps 1 and 3).  The
 * mobility matrix is never stored (Sec. 3.1): every pair block is evaluated on
 * the fly on the GPU.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers into memory owned by the caller
 *    (e.g. PyTorch tensors), except where a parameter says "host".
 *  - `stream` is a hipStream_t (NULL = the null stream).  Every call only
 *    enqueues work on `stream` and returns; results are ready once the stream
 *    has reached that point.  Calls that enqueue work on the same device and
 *    share library workspace (see sd_release) must not run concurrently on
 *    different streams.
 *  - Errors are returned as sd_status; the library never aborts.  A failed
 *    argument check enqueues nothing.  sd_last_error() gives a message for the
 *    last failure of the calling thread.  NaN/Inf inputs are not checked; they
 *    propagate into the results (every row of a product sums a term of every
 *    particle, so one non-finite position or force makes every row
 *    non-finite), and leave no state behind.  In a periodic box positions enter
 *    as fixed-point records: a non-finite position becomes an unspecified
 *    point of the box there.
 *  - Output arrays may not alias input arrays unless a parameter says so.
 *  - Layouts:
 *      "f32x4[n]"  n records of 4 floats  (x, y, z, w), 16-byte aligned, w ignored
 *      "f64x4[n]"  n records of 4 doubles (x, y, z, w), 32-byte aligned, w ignored
 *      "f64[3n]"   n records of 3 doubles (x, y, z), 8-byte aligned
 *    Positions and forces use f32x4 for the FP32 precisions and f64x4 for
 *    SD_FP64; velocities, time-loop positions and gradients are always f64[3n].
 *  - Pair blocks at distance r < 2a (overlapping spheres), r = 0 for i != j
 *    (coincident spheres) and the self term are evaluated in FP64 in every
 *    precision.  Coincident spheres contribute mu0 F_j with the overlap form
 *    (its r -> 0 limit) and nothing otherwise.
 */
#ifndef SD_H
#define SD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sd_status {
    SD_OK = 0,
    SD_EINVAL = 1,        /* bad size, null pointer, bad parameter or enum value */
    SD_EALIGN = 2,        /* a pointer is not aligned as its layout requires */
    SD_ENOMEM = 3,        /* library workspace could not be allocated */
    SD_EDEVICE = 4,       /* a HIP runtime call or kernel launch failed */
    SD_EUNSUPPORTED = 5   /* valid arguments the library does not implement */
} sd_status;

typedef enum sd_tensor {
    SD_RPY = 0,           /* Rotne-Prager tensor, Eq. (7b) */
    SD_OSEEN = 1          /* Oseen tensor, Eq. (4) */
} sd_tensor;

typedef enum sd_overlap {
    SD_OVERLAP_NONE = 0,  /* the far form of the tensor at every r > 0 */
    SD_OVERLAP_RPY = 1    /* r < 2a: mu0[(1 - 9r/32a) I + (3r/32a) rhat rhat]
                             (Rotne-Prager-Yamakawa regularisation; not in the
                             paper, which defines T for r >= 2a only).
                             Ignored for SD_OSEEN. */
} sd_overlap;

typedef enum sd_precision {
    SD_FP32_KAHAN = 0,    /* FP32 pair evaluation, Kahan-compensated FP32
                             per-particle accumulation (the paper's "single
                             precision tensor, higher-precision accumulation",
                             Sec. 3.2): terms summed in FP32 in blocks of
                             sd_kernel_config.kahan_block, each block added
                             with compensation; split rows added in FP64.
                             The pair-symmetric kernel (variant 2) compensates
                             the i side so; the terms it hands to j are summed
                             in FP32 over at most 32 pairs, those sums in FP64
                             over the i-block, rounded to FP32 once per i-block
                             and j and added in FP64 */
    SD_FP64 = 1,          /* FP64 throughout */
    SD_FP32_PLAIN = 2     /* FP32 evaluation and plain FP32 accumulation */
} sd_precision;

typedef enum sd_integrator {
    SD_EULER = 0,         /* x += dt v (Sec. 3.1, step 1) */
    SD_AB2 = 1            /* x += dt (3/2 v_k - 1/2 v_{k-1}); the step with
                             global index 0 is an Euler step (not in the paper) */
} sd_integrator;

typedef struct sd_params {
    double a;             /* sphere radius, > 0 */
    double eta;           /* shear viscosity, > 0 */
    int32_t tensor;       /* sd_tensor */
    int32_t overlap;      /* sd_overlap */
    double box[3];        /* periodic box: {0, 0, 0} = free space, or a cubic box
                             {L, L, L} with L > 2a, in which each pair
                             interacts through its nearest image only
                             (footnote of Sec. 3.1: no sum over images).
                             Positions may lie outside [0, L); the time loop
                             keeps them unwrapped.  A pair exactly half a box
                             apart along an axis has two nearest images; which
                             one a path takes follows from its rounding (the
                             FP32 paths stage positions as 32-bit fixed-point
                             fractions of L and take -L/2 at an exact tie).
                             Other boxes: SD_EUNSUPPORTED (SD_EINVAL for
                             negative or non-finite sides, or L <= 2a).
                             Supported by the product, the time loop and the
                             lubrication correction; the adjoint and batched
                             entry points return SD_EUNSUPPORTED for a box. */
} sd_params;

/* ------------------------------------------------------------------ product */

/*
 * mobility_apply -- v = M(x) F, Eq. (7a); step 3 of the algorithm of Sec. 3.1.
 *   n      number of particles, >= 1
 *   pos    f32x4[n] (FP32 precisions) or f64x4[n] (SD_FP64): positions
 *   force  same layout as pos: forces F_j
 *   vel    f64[3n], written: velocities v_i
 * Returns SD_EINVAL for n < 1, null pointers, a <= 0, eta <= 0 or unknown
 * enum values; SD_EALIGN for misaligned pos/force/vel.
 */
sd_status mobility_apply(const sd_params* p, int64_t n, const void* pos, const void* force,
                         double* vel, int32_t precision, void* stream);

/*
 * mobility_apply_noalloc -- mobility_apply for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, layouts, checks and
 * results (to the accuracy of the precision; it always runs the one-sided
 * kernel, variant 0) as mobility_apply, but it calls no hipMalloc, hipFree or
 * allocating library routine: its j-split partials (and, in a periodic box,
 * the fixed-point position records) live in a static device array of
 * SD_NOALLOC_SCRATCH_BYTES (32 MiB) per device, held from the library's load
 * until the process ends.  n is limited to what the array holds: 24 n bytes
 * (40 n in a periodic box with an FP32 precision), i.e. n <= 1398101
 * (838860); larger n returns SD_EINVAL.  Every call on a device shares that
 * device's array: calls that overlap on one device (other streams, other
 * threads) race, and the caller must order them.
 */
#define SD_NOALLOC_SCRATCH_BYTES (32u << 20)
sd_status mobility_apply_noalloc(const sd_params* p, int64_t n, const void* pos,
                                 const void* force, double* vel, int32_t precision,
                                 void* stream);

/*
 * mobility_adjoint -- reverse-mode derivative of the product.  For a
 * cotangent lam (dL/dv):
 *   grad_pos   f64[3n], written: d/dx [lam . M(x) F]
 *              = sum_{j != i} grad_r [lam_i . T(r) F_j + lam_j . T(r) F_i] at r = x_i - x_j
 *   grad_force f64[3n], written unless NULL: M(x)^T lam = M(x) lam, by the block
 *              symmetry mu_ij = mu_ji (Secs. 3.2, 3.3)
 *   lam        same layout as force (f32x4[n] / f64x4[n])
 * The gradient at r = 2a is the one-sided one of the far form; at r = 0 the
 * pair contributes no gradient.  Errors as mobility_apply.
 */
sd_status mobility_adjoint(const sd_params* p, int64_t n, const void* pos, const void* force,
                           const void* lam, double* grad_pos, double* grad_force,
                           int32_t precision, void* stream);

/* ---------------------------------------------------------------- time loop */

/*
 * sd_step -- one step of dx/dt = M(x) F with constant forces (Sec. 3.1):
 * v_k = M(x_k) F is computed from the positions before they move, then
 *   SD_EULER: x_{k+1} = x_k + dt v_k
 *   SD_AB2:   x_{k+1} = x_k + dt (3/2 v_k - 1/2 v_{k-1}),  Euler if step_index == 0
 *   x          f64[3n], in/out: FP64 master positions (the pair kernel reads an
 *              FP32 copy; pairs closer than 2a use x directly, in FP64)
 *   force      f32x4[n] or f64x4[n] as in mobility_apply
 *   v_prev     f64[3n] or NULL (Euler).  AB2: in = v_{k-1} (ignored when
 *              step_index == 0), out = v_k.  Required for AB2.
 *   v_out      f64[3n] or NULL: receives v_k
 *   dt > 0, step_index >= 0 (global index of this step)
 */
sd_status sd_step(const sd_params* p, int64_t n, double* x, const void* force, double* v_prev,
                  double* v_out, double dt, int64_t step_index, int32_t integrator,
                  int32_t precision, void* stream);

/*
 * sd_run -- `steps` consecutive sd_step calls with step indices step0,
 * step0+1, ...; bitwise identical to calling sd_step that many times.
 *   x_checkpoints  f64[(steps / checkpoint_every + 1) * 3n] or NULL: frame q
 *                  receives x at step step0 + q * checkpoint_every (frame 0 =
 *                  the initial x).  checkpoint_every >= 1 when non-NULL.
 * Other arguments as sd_step.  steps == 0 is a no-op (frame 0 is still written).
 */
sd_status sd_run(const sd_params* p, int64_t n, double* x, const void* force, double* v_prev,
                 double dt, int64_t steps, int64_t step0, int32_t integrator, int32_t precision,
                 double* x_checkpoints, int64_t checkpoint_every, void* stream);

/*
 * sd_set_graph_mode -- how sd_run launches its steps when no checkpoints are
 * requested and profiling is off: 0 = every kernel launched on the stream;
 * 1 (default) = for n <= 16384, where a step is launch-bound, chunks of 16
 * steps are captured once into a HIP graph (on a private capture stream,
 * kernel nodes only) and replayed on the caller's stream; 2 = graphs at every
 * n.  The results are identical in every mode (the same kernels in the same
 * order).  The captured graph is cached per device and rebuilt when any
 * argument, size, parameter, kernel shape or workspace it captured changes;
 * sd_release frees it.
 */
sd_status sd_set_graph_mode(int32_t mode);

/*
 * sd_run_adjoint -- gradients of a loss L(x_steps) through `steps` Euler steps
 * started at x0 (discrete adjoint of sd_run with SD_EULER, step0 = 0):
 *   lam_steps = grad_xN;  lam_k = lam_{k+1} + dt d/dx[lam_{k+1} . M(x_k) F]
 *   grad_x0 = lam_0,  grad_force = sum_k dt M(x_k) lam_{k+1}
 *   x0            f64[3n], read only
 *   x_checkpoints as written by sd_run(x0, ..., checkpoint_every) or NULL
 *                 (then the library runs the forward pass itself and keeps
 *                 every checkpoint_every-th state); each segment of
 *                 checkpoint_every steps is recomputed from its checkpoint
 *   grad_xN       f64[3n] (dL/dx_steps), read only
 *   grad_x0, grad_force  f64[3n], written
 * SD_EUNSUPPORTED for other integrators.
 */
sd_status sd_run_adjoint(const sd_params* p, int64_t n, const double* x0, const void* force,
                         double dt, int64_t steps, int32_t precision, const double* x_checkpoints,
                         int64_t checkpoint_every, const double* grad_xN, double* grad_x0,
                         double* grad_force, void* stream);

/* -------------------------------------------------------------- lubrication */

/* Truncation of the lubrication correction (Sec. 2.3). */
typedef struct sd_lub {
    double s_cut;         /* pairs with s = r/a - 2 < s_cut get the correction (paper: 1) */
    double s_min;         /* s is clamped to >= s_min at contact or overlap (not in
                             the paper); 0 < s_min < s_cut */
} sd_lub;

/*
 * lubrication_forces -- step 2 of the algorithm of Sec. 3.1 with external
 * forces and the singular lubrication friction of Eq. (8):
 *   f_out_i = f_ext_i - sum_{j: s_ij < s_cut} zeta(r_i - r_j) (v_i - v_j),
 *   mu0 zeta(r) = [1/(4s) - 9/40 log s] rhat rhat - 1/6 log s (I - rhat rhat).
 *   x, v, f_out  f64[3n]; f_ext f64[3n] or NULL (zero).  FP64 throughout.
 * Close pairs are found with a cell list rebuilt on the device (no host
 * round trip); the result is deterministic.
 */
sd_status lubrication_forces(const sd_params* p, const sd_lub* lub, int64_t n, const double* x,
                             const double* v, const double* f_ext, double* f_out, void* stream);

/*
 * sd_run_lub -- `steps` steps of the three-step loop of Sec. 3.1 with
 * lubrication: F_k = lubrication_forces(x_k, v_{k-1}, f_ext); v_k = M(x_k) F_k;
 * x_{k+1} = x_k + dt v_k (Euler) or AB2 (step index 0 is Euler).
 *   f_ext   f64[3n] external forces (constant)
 *   v_prev  f64[3n], in: velocities before the first step (the paper uses the
 *           previous step's; zero switches the correction off for the first
 *           step), out: velocities of the last step
 *   other arguments as sd_run.
 */
sd_status sd_run_lub(const sd_params* p, const sd_lub* lub, int64_t n, double* x,
                     const double* f_ext, double* v_prev, double dt, int64_t steps, int64_t step0,
                     int32_t integrator, int32_t precision, void* stream);

/* ------------------------------------------------------------------ batched */

/* Many independent clusters: particles of different clusters do not interact
 * (each cluster is its own free-space suspension). */
typedef struct sd_batch sd_batch;

/*
 * sd_batch_create -- plan for n_clusters clusters; cluster c owns particles
 * [offsets[c], offsets[c+1]).  offsets: HOST int64[n_clusters + 1],
 * offsets[0] == 0, non-decreasing; sizes up to SD_BATCH_MAX_CLUSTER.  The plan
 * orders clusters longest first for the persistent kernel's work queue and
 * owns a small device buffer; it is bound to the current device.
 */
#define SD_BATCH_MAX_CLUSTER 1024
sd_status sd_batch_create(const sd_params* p, int64_t n_clusters, const int64_t* offsets,
                          sd_batch** out);
sd_status sd_batch_destroy(sd_batch* b);
int64_t sd_batch_particles(const sd_batch* b);

/*
 * mobility_apply_batched -- per-cluster products, layouts as mobility_apply
 * over all sum_c N_c particles.
 */
sd_status mobility_apply_batched(sd_batch* b, const void* pos, const void* force, double* vel,
                                 int32_t precision, void* stream);

/*
 * sd_run_batched -- `steps` steps of every cluster in ONE persistent kernel
 * launch (each workgroup pulls clusters from a queue and keeps a cluster in
 * LDS for all steps).  x f64[3 total] in/out, force f32x4[total] (FP32
 * precisions) or f64x4[total] (SD_FP64).  use_graph != 0 launches through a
 * captured HIP graph cached in the plan.  Step indices start at 0.
 */
sd_status sd_run_batched(sd_batch* b, double* x, const void* force, double dt, int64_t steps,
                         int32_t integrator, int32_t precision, int32_t use_graph, void* stream);

/*
 * Shape of the persistent kernel of a plan: `workgroup` lanes per work-group
 * (128, 256 or 512; 0 = the default 256) and `per_cu` resident work-groups
 * per CU (0 = automatic: 1024 lanes per CU; at most 16; always limited by
 * the 160 KiB of LDS per CU).  Changing it drops the plan's cached graph.
 */
sd_status sd_batch_set_config(sd_batch* b, int32_t workgroup, int32_t per_cu);
sd_status sd_batch_get_config(const sd_batch* b, int32_t* workgroup, int32_t* per_cu);

/*
 * sd_batch_autotune -- times sd_run_batched(x, force, dt, steps, integrator,
 * precision) for every work-group size (128, 256, 512) with three residency
 * choices (automatic, half, double), each on a copy of x in library workspace
 * (x is not modified; median of three launches after a warm-up), and keeps
 * the fastest shape in the plan.  report (may be NULL) receives a JSON
 * summary of every candidate.  Synchronous: returns after the timing.
 */
sd_status sd_batch_autotune(sd_batch* b, const double* x, const void* force, double dt,
                            int64_t steps, int32_t integrator, int32_t precision, char* report,
                            int64_t report_len, void* stream);

/* ---------------------------------------------------------- precision study */

/* Precision of the accumulation of the pair sum sum_{j != i} T(r_i - r_j) F_j
 * (the "HI" of Sec. 4).  The first three evaluate pair terms in FP32 (near
 * pairs, r^2 < (2a)^2 (1 + 1e-3), in FP64 as in mobility_apply). */
typedef enum sd_acc_mode {
    SD_ACC_FP32 = 0,      /* plain FP32 sum ("single") */
    SD_ACC_KAHAN = 1,     /* FP32 sum with Kahan compensation per term */
    SD_ACC_DS = 2,        /* double-single sum: error-free FP32 two-sum of the
                             running (hi, lo) pair and each term */
    SD_ACC_FP64 = 3       /* pair terms and sum in FP64 */
} sd_acc_mode;

/* Precision of the positions and of the Euler update x += dt v. */
typedef enum sd_pos_mode {
    SD_POS_FP32 = 0,      /* FP32 positions ("single") */
    SD_POS_DS = 1,        /* double-single positions (hi, lo) in FP32 */
    SD_POS_FP64 = 2
} sd_pos_mode;

/* One run of the study. */
typedef struct sd_cluster_spec {
    int32_t acc;          /* sd_acc_mode */
    int32_t pos;          /* sd_pos_mode */
    double dt;            /* Euler time step, > 0 */
    int64_t steps;        /* steps of this call, >= 0 */
    int64_t stride;       /* a frame every `stride` steps; 0 = none */
} sd_cluster_spec;

#define SD_CLUSTER_MAX_N 64
#define SD_CLUSTER_MAX_RUNS 4096

/*
 * sd_cluster_run -- the numerical-stability study of Sec. 4: `runs`
 * independent Euler integrations of one small free-space cluster of n spheres
 * (n <= SD_CLUSTER_MAX_N, e.g. the four sedimenting spheres of Fig. 4), each
 * with its own accumulation and position precision and time step, all in ONE
 * kernel launch (one wave per run, one lane per sphere; every step stays in
 * registers and LDS).
 *   specs  HOST sd_cluster_spec[runs]
 *   state  device f64[runs][2][3n], in/out: run r's position of sphere i is
 *          state[r][0][i] + state[r][1][i] (row-major xyz); a call loads it
 *          into the run's precision and stores it back exactly (FP32 and FP64
 *          runs store lo = 0, double-single runs their (hi, lo) pair), so
 *          consecutive calls continue one trajectory.  Initialise with
 *          hi = x0, lo = 0.
 *   force  device f64[3n], the constant force on each sphere (all runs)
 *   traj   device f64, or NULL when every stride is 0: the frames of run 0,
 *          then of run 1, ...; run r writes floor(steps_r / stride_r) frames
 *          of 3n values, frame k being the positions after (k + 1) stride_r
 *          steps of this call.
 * The box of p must be zero (SD_EUNSUPPORTED otherwise).  The run records
 * are uploaded into library workspace and the call waits for `stream` once
 * before launching (a long study calls it per chunk of millions of steps).
 */
sd_status sd_cluster_run(const sd_params* p, int64_t n, int32_t runs, const sd_cluster_spec* specs,
                         double* state, const double* force, double* traj, void* stream);

/* ----------------------------------------------- memory-access benchmarks */

/* The O(N^2) memory-access micro-benchmarks of App. A (not on the product's
 * path; they characterise the j-data paths the product kernel chooses from). */
typedef enum sd_mb_kernel {
    SD_MB_NAIVE = 0,        /* every thread reads its N elements from global memory */
    SD_MB_SMALLTILING = 1,  /* the first wave (64 threads) fills LDS tiles of 64
                               elements; the work-group of 128 threads reads them
                               (two buffers: the next tile is fetched while the
                               current one is summed) */
    SD_MB_TILING = 2        /* the whole work-group fills tiles of 128 elements */
} sd_mb_kernel;

typedef enum sd_mb_map {
    SD_MB_LINEAR = 0,       /* access k reads element k */
    SD_MB_STRIDED = 1,      /* element k p mod N, p = 131 */
    SD_MB_UNORDERED = 2     /* element (k p + j M) mod N, M = 64, j the global id of
                               the reading thread (naive) or of the thread that
                               loads the tile slot (tiled kernels) */
} sd_mb_map;

typedef enum sd_mb_elem { SD_MB_FLOAT = 0, SD_MB_FLOAT4 = 1 } sd_mb_elem;

#define SD_MB_MAX_N (1 << 22)

/*
 * sd_membench -- one launch of N threads in work-groups of 128:
 *   out[j] = in[j] + sum over the N accesses of in[map(k)]
 * (elementwise for float4).  The tiled kernels visit element m + k of the
 * array through the map of the thread that loads tile slot k, for tiles
 * m = 0, TILE, 2 TILE, ... (the last tile is cut at N).
 *   in, out  device float[n] or float4[n] (16-byte aligned), n <= SD_MB_MAX_N.
 */
sd_status sd_membench(int32_t kind, int32_t map, int32_t elem, int64_t n, const void* in,
                      void* out, void* stream);

/* ------------------------------------------------------------------- tuning */

/* Kernel shape of the all-pairs product. */
typedef struct sd_kernel_config {
    int32_t variant;      /* 0 = j-tiles staged in LDS, 1 = j data through the
                             scalar cache, 2 = pair symmetry (FP32 precisions
                             only): every pair of particles in different
                             blocks evaluated once, T(r_ij) F_i handed to j
                             (block symmetry of M, Sec. 3.3); block * ilp
                             <= 512, kahan_block 0, 4, 8, or 16 or 32
                             with block 256 and ilp 2 (those two run the
                             chunk loop in generated assembly); library
                             workspace of about 6 n^2 / (block * ilp)
                             bytes.  The automatic choice takes it from
                             n = 16384 on (block 256, ilp 2, kahan_block
                             32 for SD_FP32_KAHAN) while that workspace
                             stays within 1 GiB */
    int32_t block;        /* work-group size (64, 128 or 256; variant 2: 128,
                             256 or 512) */
    int32_t splits;       /* j-range splits (>= 1): extra work-groups per i-block */
    int32_t ilp;          /* particles i per lane (1 or 2) */
    int32_t kahan_block;  /* SD_FP32_KAHAN: pair terms summed in FP32 before each
                             compensated add (1 = per term, 2, 4, or 8 with
                             block >= 128; variant 2 also 16 or 32); 0 for
                             the other precisions.  Variant 2 sums the
                             j side in FP32 over at most 32 terms before
                             its FP64 sums, whatever the value */
} sd_kernel_config;

/* Force a configuration for a precision (NULL restores automatic choice). */
sd_status sd_set_kernel_config(int32_t precision, const sd_kernel_config* cfg);
/* The configuration mobility_apply would use for n particles. */
sd_status sd_get_kernel_config(int32_t precision, int64_t n, sd_kernel_config* out);

/*
 * sd_autotune -- time candidate configurations on n synthetic particles and
 * install the fastest for that precision and size class (the automatic
 * choice is among the candidates).  report (host buffer, may be NULL)
 * receives a JSON summary, truncated to report_len: the candidate count, the
 * automatic choice's time ("default_ms") and the fastest shapes in order.
 * Synchronises the stream; allocates temporary device memory.
 */
sd_status sd_autotune(const sd_params* p, int64_t n, int32_t precision, void* stream,
                      char* report, int64_t report_len);
/* sd_autotune_clear -- drop every entry sd_autotune installed for a
 * precision, so that the automatic choice (or a forced configuration) applies
 * again at every size.  Host-only; no device work. */
sd_status sd_autotune_clear(int32_t precision);

/* ---------------------------------------------------------------- profiling */

/* When enabled, the library brackets every launch of its pair kernel with HIP
 * events on the launch stream and accumulates the elapsed times. */
sd_status sd_profile_enable(int32_t on);
/* Pair-kernel launches and their total time since the last reset (waits for
 * the recorded events). */
sd_status sd_profile_read(int64_t* launches, double* total_ms);
sd_status sd_profile_reset(void);
/* Per-launch pair-kernel times (ms) since the last reset, in launch order: the
 * first min(cap, count) are written to ms (host buffer of cap floats, may be
 * NULL when cap is 0); *count (may be NULL) receives how many are held (at
 * most 65536 after a reset).  Waits for the recorded events. */
sd_status sd_profile_times(float* ms, int64_t cap, int64_t* count);

/* -------------------------------------------------------------- observables */

/*
 * sd_mean_vector -- out[0..2] = (1/n) sum_i v_i for v f64[3n] (e.g. the
 * centre-of-mass velocity of the sedimenting suspensions of Secs. 3.3 and 4).
 * Summed in a fixed order that depends on n only (contiguous ranges of
 * particles, then their partial sums): the result is deterministic.  Uses
 * library workspace (24 bytes per 1024 particles, at most 24 KiB).
 * out: device f64[3].
 */
sd_status sd_mean_vector(int64_t n, const double* v, double* out, void* stream);

/*
 * sd_premise_counts -- pairs that break the premise of the far-field tensor.
 * The Rotne-Prager tensor of Eq. 4 keeps the mobility matrix positive definite
 * only while every pair distance is r >= 2a (Sec. 2.2).  The product kernels
 * (mobility_apply, mobility_apply_noalloc, sd_step, sd_run, sd_run_lub; every
 * precision and kernel variant) count on their device the unordered pairs
 * i < j they meet with 0 < r < 2a (*sub2a) and with r = 0 (*coincident:
 * distinct particles at one point); r is the FP64 distance the pair's near-field
 * evaluation uses (FP64 master positions in the time loops, the staged FP32
 * positions in mobility_apply; nearest image in a periodic box).  Under
 * SD_OVERLAP_NONE these pairs were evaluated with the far form of Eq. 4
 * (coincident ones contribute nothing); under SD_OVERLAP_RPY with the overlap
 * form.  The counts accumulate over calls until a read with reset != 0 zeroes
 * them; calls on several streams of one device share them.  The batched,
 * cluster and adjoint entry points do not count.
 *   sub2a, coincident  host int64 (either may be NULL)
 * Reads the current device's counters in stream order and synchronises the
 * stream; SD_EDEVICE if that fails.
 */
sd_status sd_premise_counts(int64_t* sub2a, int64_t* coincident, int32_t reset, void* stream);

/* --------------------------------------------------------------------- misc */

/*
 * sd_pack -- stage vectors for the product entry points: f64[3n] -> f32x4[n]
 * (FP32 precisions, values rounded to nearest) or f64x4[n] (SD_FP64), w = 0.
 * This is the FP64 -> FP32 staging step the time loop applies to positions
 * before every product.
 */
sd_status sd_pack(int64_t n, const double* v, void* out, int32_t precision, void* stream);

/* Frees library-owned device workspace on every device (staging copies,
 * split partials).  Safe to call at any time when no library work is pending. */
sd_status sd_release(void);
const char* sd_status_string(int32_t status);
const char* sd_last_error(void);
/* 100 * major + minor; 110 added the periodic box (sd_params.box), the
 * lubrication entry points, the precision study, the micro-benchmarks and the
 * batched-kernel shape. */
#define SD_VERSION 110
int32_t sd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SD_H */
