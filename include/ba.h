/*
 * ba.h -- C ABI of the MI355X (gfx950) cluster bundle-adjustment library.
 *
 * The library minimises, for one cluster C_l of overlapping images at a time
 * (Sec. 3.2 of "Real-Time Bundle Adjustment for Ultra-High-Resolution UAV
 * Imagery Using Adaptive Patch-Based Feature Tracking"), the robust
 * reprojection cost of Eq. (7)
 *
 *     E = 1/2 sum_{k in C_l} sum_{j in J_k} rho( |p_kj - pi(K R_k^T (X_j - T_k))|^2 / sigma^2 )
 *       + 1/2 sum_{free k} ( |Log(R_prior,k^T R_k)|^2_{sigma_omega} + |T_k - T_prior,k|^2_{sigma_T} )
 *
 * with the pinhole projection of Eq. (5) extended by Brown radial terms
 * k1, k2 on the normalised coordinates, rho the Huber function on the squared
 * whitened residual norm, and pose priors at the GNSS/IMU-derived initial
 * poses T_k^(0), R_k^(0) (Sec. 3.2).  Images marked fixed keep their pose
 * (the first half of the inter-cluster overlap, Sec. 3.2).  The minimiser is
 * Levenberg-Marquardt: IRLS Gauss-Newton normal equations, Marquardt diagonal
 * scaling D = clamp(diag H, 1e-6, 1e32), Nielsen's damping update, the damped
 * system solved by eliminating the points (Schur complement), a Cholesky
 * factorisation of the reduced camera system in FP64 (or, for large systems
 * such as a whole-flight global adjustment, preconditioned conjugate
 * gradients with a block-Jacobi 6x6 preconditioner) and point
 * back-substitution.  All of it runs in HIP kernels on the GPU.
 *
 * Conventions
 *   R_k  camera->world rotation, row-major 3x3 (columns = camera axes in the
 *        world frame); T_k projection centre.  X_c = R_k^T (X_j - T_k), camera
 *        z forward, image y down (Eq. 3/5: pi(x, y, z) = (x/z, y/z)).
 *   obs_uv pixel coordinates, origin at the image corner; principal point
 *        (cx, cy); focal length f in pixels.
 *   Rotation update R <- R Exp(d_omega) (right perturbation).
 *   Any consistent metric world frame (ENU, ECEF); the library shifts all
 *   coordinates by the mean camera centre internally, in FP64.
 *
 * Memory and threads
 *   Every array passed in is a HOST pointer owned by the caller and is only
 *   read during the call (submit copies what it needs).  Every output buffer
 *   is caller-allocated host memory.  The library owns all device memory: one
 *   arena of hbm_budget_bytes allocated by ba_create, from which each admitted
 *   cluster takes one block, freed when the cluster is released.
 *   All functions are thread-safe.  With serve = 1 a runtime thread inside
 *   the context runs the continuous-batching loop (ba_solve/ba_wait).
 *   Functions return BA_OK (0) or a negative ba_error; nothing is thrown or
 *   aborted across the ABI.  ba_last_error gives a message for the last
 *   failure of the context.
 */
#ifndef BA_H
#define BA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ba_ctx ba_ctx;
typedef int64_t ba_ticket;

enum ba_error {
  BA_OK = 0,
  BA_E_ARG = -1,      /* invalid argument: bad index, non-finite value, size limit */
  BA_E_NOMEM = -2,    /* the cluster can never fit the arena, or device allocation failed */
  BA_E_AGAIN = -3,    /* queue full, or (ba_step) no slot/memory free right now: retry */
  BA_E_STATE = -4,    /* operation not valid in the ticket's current state */
  BA_E_DEVICE = -5,   /* HIP runtime error; the context is unusable afterwards */
  BA_E_TIMEOUT = -7   /* ba_wait timed out */
};

enum ba_precision {
  BA_FP64 = 0,   /* plain: residuals, Jacobians, Schur assembly and solve in FP64 */
  BA_MIXED = 1   /* residuals, Jacobians, Schur assembly in FP32 (FP32 accumulation);
                    reduced-system Cholesky, one refinement step of the camera
                    update, cost reductions and gain ratio in FP64 */
};

enum ba_solver {
  BA_SOLVER_AUTO = 0,   /* dense Cholesky up to BA_MAX_FREE_CAMS free cameras, PCG above */
  BA_SOLVER_DENSE = 1,  /* FP64 Cholesky of the reduced camera system in 16x16 blocks */
  BA_SOLVER_PCG = 2     /* conjugate gradients on the block-sparse reduced camera system,
                           block-Jacobi 6x6 preconditioner; FP32 matrix-vector products in
                           BA_MIXED, FP64 dot products and updates; no estimated intrinsics */
};

enum ba_solve_status {
  BA_ST_QUEUED = 0,     /* waiting for a slot / arena memory */
  BA_ST_RUNNING = 1,    /* admitted, iterations in progress */
  BA_ST_MAXITER = 2,    /* ran max_iters iterations */
  BA_ST_CONVERGED = 3,  /* an accepted step decreased E by less than ftol * E */
  BA_ST_STALLED = 4,    /* damping exceeded 1e32 after rejected steps */
  BA_ST_BAD_INIT = 5    /* the initial state has a point at non-positive depth */
};

/* Context options.  A count or tolerance of 0 selects its default; a negative
 * one makes ba_create return BA_E_ARG. */
typedef struct {
  int32_t device;            /* HIP device ordinal */
  void* stream;              /* hipStream_t to run on (e.g. torch.cuda.current_stream().cuda_stream);
                                NULL: the context creates its own stream */
  size_t hbm_budget_bytes;   /* arena size for cluster state; 0 -> 1 GiB */
  int32_t max_slots;         /* clusters resident on the device at once; 0 -> 256 */
  int32_t max_queue;         /* submitted clusters waiting for admission; 0 -> 4096 */
  int32_t precision;         /* enum ba_precision */
  int32_t serve;             /* 1: start the continuous-batching runtime thread */
  int32_t iters_per_tick;    /* LM iterations between control read-backs (batched solve,
                                serving tick); 0 -> 10.  A serving tick is cut short
                                when a cluster reaches its iteration cap */
  int32_t chunks_per_wg;     /* 64-observation chunks per workgroup of the point-major
                                kernels; 0 -> 16 */
  int32_t chunks_per_task;   /* 64-lane chunks per wavefront task of the block kernel;
                                0 -> 4 */
  int32_t solver;            /* enum ba_solver */
  int32_t pcg_max_iters;     /* conjugate-gradient iterations per LM step; 0 -> 500 */
  double pcg_tol;            /* stop when |r| <= pcg_tol |b| (the forcing term of an inexact
                                LM step); 0 -> 0.1 */
  int32_t resident_cams;     /* capacity of the device-resident camera state keyed by global
                                ID (see ba_cluster.use_resident); 0 -> 8192 */
  int32_t resident_points;   /* capacity of the resident point state; 0 -> 4194304.  The
                                store (96 B per camera, 24 B per point) is allocated at the
                                first cluster that uses it, outside the arena */
  int32_t batch_streams;     /* batched solves and the serving loop run S parts of the running
                                clusters (of about equal assembly work) on S streams when at
                                least 4 S clusters run, so that one part's latency-bound
                                kernels overlap the others' assembly; 1: one stream;
                                0 -> 2; at most 4, else BA_E_ARG */
  /* Device-memory provider, e.g. PyTorch's caching allocator.  With both
   * set, every device allocation of the context (the arena, the slot
   * tables, the launch lists, the resident store) is dev_alloc(bytes,
   * alloc_user), and each is returned by dev_free(ptr, alloc_user) before
   * ba_destroy returns (or before a failing ba_create returns).  A block
   * must be device memory of the context's device, aligned to 256 bytes,
   * valid until freed; NULL means out of memory (BA_E_NOMEM).  The hooks
   * are called from the thread of ba_create, ba_submit_cluster(s) or
   * ba_destroy, never from the serving thread.  Both NULL: hipMalloc /
   * hipFree.  Only one of them set: BA_E_ARG. */
  void* (*dev_alloc)(size_t bytes, void* user);
  void (*dev_free)(void* ptr, void* user);
  void* alloc_user;
  /* Layout threads.  0: ba_submit_cluster(s) validate and lay a cluster out
   * on the calling thread and report every invalid input at once.  n (1..64):
   * a pool of n host threads lays submitted clusters out in the background,
   * so that the caller and the serving loop are not held up by it;
   * ba_submit_cluster(s) then check only what needs no layout (sizes, arrays
   * present, resident IDs unique; BA_E_ARG), copy the cluster and return.  A
   * cluster the pool refuses (the remaining checks of ba_submit_cluster, or
   * a footprint larger than the arena) is dropped from the queue and
   * reported by ba_wait, ba_step, ba_solve_batch and ba_fetch on its ticket
   * (BA_E_ARG / BA_E_NOMEM with the message).  ba_step and ba_solve_batch
   * wait for their clusters' layout.  Negative or above 64: BA_E_ARG. */
  int32_t stage_threads;
} ba_options;

/* One cluster (ba_submit_cluster).  C = n_cams, P = n_points, O = n_obs. */
typedef struct {
  int32_t n_cams, n_points, n_obs;
  int32_t intr_mask;            /* intrinsics estimated with the poses (the intrinsic border of
                                   the reduced system): bit 0 k1, bit 1 k2, bit 2 f, bit 3 cx,
                                   bit 4 cy; any subset, each an extra column of the reduced
                                   system after the cameras' (other bits: BA_E_ARG); f, cx, cy
                                   (self-calibration, a variant Sec. 5 names) start at the
                                   values below */
  const double* R;              /* [9C] initial rotations, camera->world, row-major */
  const double* T;              /* [3C] initial projection centres */
  const double* X;              /* [3P] initial tie points */
  const double* k;              /* [2]  initial k1, k2 */
  const double* prior_R;        /* [9C] GNSS/IMU attitude prior */
  const double* prior_T;        /* [3C] GNSS/IMU position prior */
  const double* prior_sigma;    /* [6C] sigma_omega[3] (rad), sigma_T[3] (m); a component
                                   with sigma <= 0 or non-finite is switched off */
  const uint8_t* fixed;         /* [C] 1: pose held constant (no unknowns, no prior) */
  const int32_t* obs_cam;       /* [O] camera index of each observation */
  const int32_t* obs_pt;        /* [O] point index of each observation */
  const double* obs_uv;         /* [2O] observed pixel (u, v) */
  double f, cx, cy;             /* focal length and principal point, pixels */
  double sigma_px;              /* observation standard deviation, pixels (> 0) */
  double huber_delta;           /* Huber threshold on |e|, pixels (> 0) */
  int32_t max_iters;            /* LM iterations (1..4096) */
  int32_t stop_on_ftol;         /* 1: stop when an accepted step has (E - E') < ftol E */
  double lambda0;               /* initial damping (clamped to [1e-16, 1e32]); NaN: the damping
                                   the last cluster written back to the resident state ended
                                   with, or 1e-4 when there is none */
  double ftol;
  /* Resident state across overlapping clusters (Sec. 3.2: consecutive clusters
   * share images and tie points; the next cluster starts from the previous
   * one's solution).  cam_ids / point_ids give each camera and point a global
   * ID (unique within the cluster).  With use_resident = 1:
   *  - every ID written back by an earlier cluster takes its initial value
   *    (R, T or X) from the device-resident state, and the caller's value for it
   *    is ignored; priors always come from the caller;
   *  - the cluster is admitted only after every earlier-submitted cluster that
   *    shares an ID with it has finished and written back (or was released), so
   *    overlapping clusters run in submission order;
   *  - when it finishes (any status but BA_ST_BAD_INIT) its final poses and
   *    points are written back under their IDs, on the device.
   * With use_resident = 0 the IDs are ignored and nothing is read or written.
   *
   * fuse_resident = 1 (with use_resident) writes the poses back by the pose
   * fusion of Sec. 3.2, Eq. (8): a free camera whose ID already holds a pose
   * written back by an earlier cluster gets the weighted mean of that pose and
   * this cluster's, the weights being match counts: this cluster's
   * observations of the camera, and the accumulated weight stored with the
   * earlier pose.  Positions are averaged linearly; rotations along the
   * geodesic, R = R_old Exp(w_new / (w_old + w_new) Log(R_old^T R_new)).
   * The stored weight becomes w_old + w_new.  Fixed cameras (the retained
   * first half of the overlap) and cameras seen for the first time are
   * written back as solved, with weight w_new; points are always written back
   * as solved.  ba_fetch returns the cluster's own solution, not the fused
   * poses (see ba_resident_poses). */
  const int64_t* cam_ids;       /* [C] or NULL (required with use_resident) */
  const int64_t* point_ids;     /* [P] or NULL (required with use_resident) */
  int32_t use_resident;
  int32_t fuse_resident;
} ba_cluster;

/* Results (ba_fetch).  Every pointer may be NULL (not written); the
 * caller allocates each array.  The Levenberg-Marquardt quantities follow the
 * minimisation of Eq. (7) (Sec. 3.2); the reprojection statistics are the
 * ones Sec. 3.3 and Table 1 report (mean and standard deviation of the
 * reprojection error norm). */
typedef struct {
  double* R;                    /* [9C] */
  double* T;                    /* [3C] */
  double* X;                    /* [3P] */
  double* k;                    /* [2]  */
  double* cost_log;             /* [max_iters + 1]: E before the first iteration and after each;
                                   entries past the last iteration run are NaN */
  int32_t status;               /* enum ba_solve_status */
  int32_t iterations, accepted, rejected;
  double lambda;                /* damping after the last iteration */
  double initial_cost, final_cost;
  double t_submit, t_admit, t_done;   /* seconds on the library's steady clock: t_submit when
                                         ba_submit_cluster(s) was entered, t_admit when the
                                         cluster took its slot, t_done when the serving loop
                                         retired it (0 outside the serving loop) */
  int64_t cg_iters;             /* conjugate-gradient iterations over all LM iterations (PCG solver; else 0) */
  double* intr;                 /* [3] f, cx, cy (estimated, or as submitted) */
  double* lambda_log;           /* [max_iters]: the damping each iteration's step was solved with
                                   (NaN past the last iteration run) */
  int32_t* accepted_log;        /* [max_iters]: 1 if the iteration's trial was accepted, 0 if it was
                                   rejected (a cost that did not decrease enough, a failed
                                   factorisation, or a point at non-positive depth), -1 past the
                                   last iteration run */
  double nu;                    /* damping growth factor after the last iteration */
  /* Reprojection error |p_obs - p^| (pixels, FP64, on the device) at the fetched state, over
   * the observations at positive depth: count, RMS, mean, population standard deviation, and
   * the same restricted to inliers |p_obs - p^| <= 3 huber_delta. */
  int64_t n_reproj, n_inliers;
  double reproj_rms, reproj_mean, reproj_std;
  double inlier_mean, inlier_std;
} ba_result;

/* Limits enforced by ba_submit_cluster (BA_E_ARG beyond them). */
#define BA_MAX_FREE_CAMS 24     /* free cameras per cluster for the dense solver (m <= 149) */
#define BA_MAX_CAMS 512         /* cameras per cluster, fixed ones included (also the PCG limit) */
#define BA_MAX_OBS_PER_POINT 64 /* a point's observations share one 64-lane wavefront */

/* Create a context on options->device.  Allocates the arena.
 * Errors: BA_E_ARG (bad options), BA_E_NOMEM, BA_E_DEVICE. */
int ba_create(const ba_options* options, ba_ctx** out);

/* Stop the runtime thread, free all device memory and the context. */
int ba_destroy(ba_ctx* ctx);

/* Validate and copy one cluster (Eq. 7 problem data, Sec. 3.2), admit it to a
 * device slot if a slot and arena memory are free, else queue it.  Checks:
 * indices in range, finite inputs, 1..64 observations per observed point,
 * no camera twice on one point, <= BA_MAX_CAMS cameras, <= BA_MAX_FREE_CAMS free
 * cameras for the dense solver, no estimated intrinsics with the PCG solver,
 * unique global IDs when use_resident is set.
 * Errors: BA_E_ARG, BA_E_NOMEM (larger than the whole arena, or the resident
 * store is full), BA_E_AGAIN (queue full), BA_E_DEVICE. */
int ba_submit_cluster(ba_ctx* ctx, const ba_cluster* cluster, ba_ticket* ticket);

/* Submit n clusters that arrive together (clusters [n]): they are validated
 * and laid out on up to 8 host threads at once, then queued in array order,
 * exactly as n calls of ba_submit_cluster in that order would (resident IDs
 * order them the same way).  Writes tickets [n].  A cluster that fails
 * validation (with stage_threads > 0: the checks made at submission) fails
 * the call before any is queued (BA_E_ARG, the message names its index;
 * every ticket 0).  A later error (BA_E_NOMEM: resident
 * store full, BA_E_AGAIN: queue full, BA_E_DEVICE) leaves the clusters
 * before it queued with their tickets, and the rest with ticket 0. */
int ba_submit_clusters(ba_ctx* ctx, int32_t n, const ba_cluster* clusters, ba_ticket* tickets);

/* Run up to n_iters LM iterations of one cluster now, on the calling thread,
 * reading the LM status back after every iteration (the plain, host-driven
 * loop).  Admits the cluster first if it is still queued.  A resident cluster
 * that finishes writes its state back before this returns.
 * Errors: BA_E_ARG (unknown ticket), BA_E_AGAIN (no slot or memory free),
 * BA_E_STATE (the cluster is owned by the serving loop, or it uses resident
 * state that an unfinished earlier cluster has still to write), BA_E_DEVICE. */
int ba_step(ba_ctx* ctx, ba_ticket ticket, int32_t n_iters);

/* Solve the given clusters together to termination on the calling thread:
 * every LM iteration of every cluster is one batched launch series, with LM
 * control on the device (no host round trip per iteration).  All tickets must
 * be admitted or admissible at once.  Errors as ba_step. */
int ba_solve_batch(ba_ctx* ctx, const ba_ticket* tickets, int32_t n);

/* Hand the cluster to the continuous-batching loop (context created with
 * serve = 1): it is admitted when a slot and memory free up, iterated with
 * the other resident clusters, and retired on termination.  Returns at once.
 * Errors: BA_E_ARG, BA_E_STATE (no serving loop, or already solving). */
int ba_solve(ba_ctx* ctx, ba_ticket ticket);

/* Wait until a cluster handed to ba_solve has terminated.  timeout_s < 0
 * waits forever.  Errors: BA_E_ARG, BA_E_STATE (not handed to ba_solve, or
 * released while waiting), BA_E_TIMEOUT. */
int ba_wait(ba_ctx* ctx, ba_ticket ticket, double timeout_s);

/* Copy the cluster's current (or final) state and statistics into result
 * (origin shift undone in FP64 on the device).  Errors: BA_E_ARG,
 * BA_E_STATE (still queued or being solved by the serving loop), BA_E_DEVICE. */
int ba_fetch(ba_ctx* ctx, ba_ticket ticket, ba_result* result);

/* Forget a ticket and free its slot and arena block.  A cluster handed to
 * ba_solve and not yet finished is cancelled instead: the call returns at
 * once and the serving loop drops the cluster at its next tick boundary
 * (its resident state is not written back, and no later cluster waits for
 * it); ba_wait on it then returns BA_E_STATE.  Errors: BA_E_ARG (unknown
 * ticket), BA_E_DEVICE. */
int ba_release(ba_ctx* ctx, ba_ticket ticket);

/* The device-resident poses of n camera IDs (world frame, as last written
 * back; with fuse_resident, the fused poses of Eq. (8)), copied to host
 * arrays R [9n] (row-major, camera->world), T [3n] and w [n] (the stored
 * match-count weight); w may be NULL.  Waits for the library's streams.
 * Errors: BA_E_ARG (NULL arrays, n < 0, or an ID never written back),
 * BA_E_STATE (an ID has a pending writer: a submitted cluster holding it has
 * not finished), BA_E_DEVICE. */
int ba_resident_poses(ba_ctx* ctx, int32_t n, const int64_t* cam_ids, double* R, double* T, double* w);

/* Bytes of arena the cluster would take once admitted (its admission
 * footprint), or 0 if the cluster is invalid. */
size_t ba_footprint(ba_ctx* ctx, const ba_cluster* cluster);

/* Per-kernel timing with HIP events that the dispatches of an LM iteration
 * record themselves on the context's stream (off by default).  `kernels` is
 * a bitmask of (1 << enum ba_prof_kernel) selecting the kernels to time
 * (BA_PROF_ALL: every one; 0: off); each timed kernel costs two event records
 * per launch.  ba_profile_read adds up the elapsed time and the number of
 * timed launches per kernel since the last read, in the order of
 * enum ba_prof_kernel, into caller arrays of BA_PROF_N entries, and resets
 * the counters.  The Schur-block tasks are one launch in BA_MIXED (timed as
 * BA_PROF_BLOCKS; BA_PROF_PAIRBLK then marks an empty interval) and two in
 * BA_FP64 (camera tasks as BA_PROF_BLOCKS, pair tasks as BA_PROF_PAIRBLK).
 * When the batch holds self-calibrating clusters, the point, block and
 * back-substitution kernels run as two launches each (ordinary clusters,
 * then self-calibrating ones); the slot's time then runs from the start of
 * the first to the end of the second.  BA_PROF_PCG runs from before the first
 * conjugate-gradient launch of the iteration to after the last (one
 * cooperative launch per such cluster).
 * Errors: BA_E_ARG, BA_E_DEVICE. */
enum ba_prof_kernel { BA_PROF_POINT = 0, BA_PROF_BLOCKS = 1, BA_PROF_PAIRBLK = 2, BA_PROF_REDUCE = 3,
                      BA_PROF_SOLVE = 4, BA_PROF_BACKSUB = 5, BA_PROF_LM = 6, BA_PROF_PCG = 7,
                      BA_PROF_N = 8 };
#define BA_PROF_ALL ((1 << BA_PROF_N) - 1)
int ba_profile_enable(ba_ctx* ctx, int32_t kernels);
int ba_profile_read(ba_ctx* ctx, double* total_ms, int64_t* launches);

const char* ba_strerror(int code);
const char* ba_last_error(ba_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* BA_H */
