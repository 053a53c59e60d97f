// Internal device-side data layout of the cluster bundle-adjustment library.
// Shared by the runtime (ba_runtime.cpp) and the kernels (ba_kernels.hip);
// not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ba_consts.h"

namespace bagpu {


// Read-only description of one resident cluster; written once at admission.
struct SlotDesc {
  int C, P, L, n_chunks, n_wg, pad0;      // cameras, points, observation lanes, point chunks, workgroups
  int m, n_free, kcol0, kcol1;            // reduced system size, free cameras, intrinsic columns (-1: fixed)
  int psize, pstride;                     // dense system doubles (16x16 blocks), vector stride (psize + 3m)
  int max_iters, stop_on_ftol, mixed, nb;  // nb: 16x16 blocks per side of the dense reduced system
  int Lc, Lq, n_tasks, n_cam_tasks, n_cam_task_wg, n_pair_task_wg, n_targets, n_pt_part;
  int sparse, nnzb, pcg_max_iters, pad1;  // sparse: block-CSR reduced system solved by PCG
  // reduced-system column of each intrinsic (0 k1, 1 k2, 2 f, 3 cx, 4 cy; -1:
  // fixed; kcol0, kcol1 repeat those of k1, k2); sc = 1 when f, cx or cy is
  // estimated (self-calibration)
  int kcolt[kIntr], sc, pad2[2];
  double pcg_tol;
  double f, cx, cy, inv_sigma, huber_dt, ftol, lambda0;
  // point chunks: 64 consecutive internal points with the same observation
  // count n; observation t (camera order) of the chunk's lane l sits in
  // observation lane first + 64 t + l
  const int4* pchunk;                     // [n_chunks] {first observation lane, n, first point, valid points}
  const int* wg_chunk;                    // [n_wg + 1] first chunk of each point-pass workgroup
  const int* ob_cam;                      // [L] camera of each observation lane (0 for padding)
  double* ob_uv64;                        // [2L] u - cx, v - cy  (uploaded raw, shifted in place)
  float* ob_uv32;                         // [2L]
  // camera lanes: observations of free cameras sorted by (camera, point), each
  // camera's run padded to whole 64-lane chunks; pixels are read from the
  // observation lanes
  const int* cl_pt;                       // [Lc] point index, -1 for padding
  const int* cl_ob;                       // [Lc] observation lane, 0 for padding
  // pair lanes: observation pairs of one point with both cameras free, sorted
  // by camera-pair block, each block's run padded to whole chunks
  const int* ql_pt;                       // [Lq] point index, -1 for padding
  const int2* ql_ob;                      // [Lq] observation lanes of camera a and b
  const int4* tasks;                      // [n_tasks] camera tasks (by camera), then pair tasks (by block)
  const int4* targets;                    // [n_targets] reduction targets with their task ranges
  // cameras
  double* cam[2];                         // [C][12] state buffers
  double* prior;                          // [C][18]
  double* pterm[2];                       // [C][16] prior terms (e 6, J 9, pad) of each state buffer's cameras
  const int* cam_col;                     // [C] first reduced-system column, -1 if fixed
  double* raw_cam;                        // [C][30] R (9), T (3), R_prior (9), T_prior (3), sigma (6)
  // points
  double* X[2];                           // [P][3] state buffers (origin-shifted)
  float* X32[2];                          // [P][3] FP32 shadows of X
  void* ptv;                              // [P][16] Real: Q, g, Z (+1 pad) from the last point pass
  void* ptd;                              // [P][4] Real: D_V (+1 pad)
  void* ptz;                              // [P][12] Real, self-calibration only: Z rows of f, cx, cy
  const int* pt_orig;                     // [P] caller index of each internal point
  // reduced camera system
  void* task_part;                        // [n_tasks][72] Real: per-task block sums
  void* pt_part;                          // [n_pt_part][32] Real: per point-pass wavefront intrinsic sums
  double* Sg;                             // [pstride] reduced: S_acc in 16x16 blocks of the lower block
                                          //   triangle, rows padded to 17 (psize), then g, bS, diag U (m each)
  double* Sd;                             // [nb(nb+1)/2][272] damped S in 16x16 blocks, for the refinement step
  // sparse reduced system (PCG): block rows of the free cameras, diagonal block first
  const int* brow;                        // [F + 1]
  const int* bcol;                        // [nnzb] free-camera column of each block
  const int2* tslot;                      // [n_targets] block slots of a target: (a,b) and (b,a)
  double* Sblk;                           // [nnzb][6][kSbRow] FP64 blocks, row-major, rows padded
  float* Sblk32;                          // [nnzb][6][kSbRow] FP32 copy for the mixed-precision products
  double* pcgw;                           // [7m + 20 kMaxCgWG + 8] PCG work: gradient with priors, clamped
                                          //   diagonal, z_0, u and z (two buffers each), workgroup parts of the sums
                                          //   (set-up and final; CG steps, two buffers), barrier words
  const int* pcg_part;                    // [pcg_G + 1] first block row of each PCG workgroup
  int pcg_G, pcg_rows_max;                // PCG workgroups; most block rows of one of them
  int pcg_smem, pad3;                     // dynamic LDS bytes of the PCG launch
  // resident state keyed by global IDs (shared by the context's clusters)
  int n_rin_cam, n_rin_pt, n_rout_cam, n_rout_pt;
  double* res_cam;                        // [cap][12] world frame: R row-major (9), T (3)
  double* res_cam_w;                      // [cap] match-count weight of each resident pose
  double* res_pt;                         // [cap][3] world frame
  const int2* rin_cam;                    // [n_rin_cam] (camera, row) read at admission
  const int2* rin_pt;                     // [n_rin_pt] (internal point, row) read at admission
  const int4* rout_cam;                   // [n_rout_cam] (camera, row, observations of the camera,
                                          //   1: fuse with the resident pose by Eq. 8) written back
  const int2* rout_pt;                    // [n_rout_pt] (caller's point index, row) written back
  double* dc;                             // [m] camera / intrinsic update
  double* cost_part;                      // [n_wg][2] sum rho(s'), sum of point parts of the predicted reduction
  int* bad_part;                          // [n_wg] trial observations at non-positive depth
  double* cost_log;                       // [max_iters + 1]
  double* lambda_log;                     // [max_iters] damping each iteration's step was solved with
  int* acc_log;                           // [max_iters] 1: the iteration's trial was accepted
  double* stat_part;                      // [n_wg][kStatVals] reprojection statistics of the exported state
  double* out;                            // [12C + 3P + 5 + kStatVals] export staging: R, T, X, intrinsics,
                                          //   then the cluster's reprojection sums at the exported state
};

// Levenberg-Marquardt control of one cluster, updated on the device.
struct SlotCtl {
  double origin[3];
  double k[2][5];                         // intrinsics per state buffer: k1, k2, f, and the principal
                                          //   point's offset (x, y) from the caller's (cx, cy)
  double lambda, nu, E, E_prior_trial, pred_c, E0;
  int cur, status, iter, accepted, rejected, solve_ok, point_fail, bad_init;
  int cg_iters, pad;                      // conjugate-gradient iterations, summed over LM iterations
  double cg_b0;                           // |b| of the first conjugate-gradient solve (forcing-term scale)
};

// Launch helpers (ba_kernels.hip).  `act` lists the slots of the batch,
// `wg_off` the prefix sums of their chunk-kernel workgroup counts.
struct Batch {
  const SlotDesc* desc;
  SlotCtl* ctl;
  const int* act;
  const int* wg_off;                      // point-lane chunk workgroups
  const int* tkc_off;                     // camera-task workgroups (4 tasks each)
  const int* tkp_off;                     // pair-task workgroups (4 tasks each)
  const int* tg_off;                      // reduction targets
  int n_act;
  int total_wg, total_tkc_wg, total_tkp_wg, total_tg;
  int max_m, max_C, max_pstride, max_nb;
  int any_sparse, any_dense, any_sc, pad;   // any_sc: a self-calibrating cluster in the batch
};

// A cluster solved by conjugate gradients: its slot, workgroups and LDS bytes
// (one cooperative launch each).
struct SparseLaunch {
  int slot, G, smem;
};

// max_rin: largest resident gather list of the batch (0: none).
hipError_t launch_prep(const Batch& b, int max_P_L, int max_rin, hipStream_t st);
hipError_t launch_initial_cost(const Batch& b, hipStream_t st);
// ev (optional): 16 events, the start and end of each of the eight kernels
// of the iteration (point, camera blocks, pair blocks, reduce, dense solve,
// back-substitution, LM, PCG solve), recorded by the dispatches themselves
// for the kernels whose bit is set in `timed`.
hipError_t launch_iteration(const Batch& b, bool mixed, hipStream_t st, hipEvent_t* ev = nullptr, int timed = 0,
                            const SparseLaunch* sp = nullptr, int n_sp = 0);
// Dynamic LDS bytes of the conjugate-gradient launch of a cluster: its
// workgroups' largest block range (bytes: block values and block columns),
// m and F.
size_t pcg_lds_bytes(size_t block_bytes, int m, int F, int rows_max);
hipError_t launch_export(const Batch& b, int max_P, hipStream_t st);
// Writes the exported state of the batch's clusters back to the resident
// store (after launch_export); max_rout: largest write-back list.
hipError_t launch_writeback(const Batch& b, int max_rout, hipStream_t st);

size_t real_size(bool mixed);

}  // namespace bagpu
