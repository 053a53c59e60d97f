// Constants of the device-side layout shared by the host runtime, the host
// layout (ba_stage.cpp, which builds without HIP) and the kernels.  Not part
// of the public ABI.
#pragma once

namespace bagpu {

constexpr int kWave = 64;                 // CDNA wavefront
constexpr int kWG = 256;                  // threads per workgroup of the chunk kernels
constexpr int kWavesPerWG = kWG / kWave;
constexpr int kMaxFreeCams = 24;          // reduced system m <= 6*24 + 5 = 149
constexpr int kMaxCams = 512;             // camera table kept in LDS by the point-lane kernels
constexpr int kCamVals = 12;              // R row-major (9), T - origin (3)
constexpr int kPriorVals = 18;            // R_prior (9), T_prior - origin (3), 1/sigma (6)
constexpr int kPtermVals = 16;            // cached prior terms of a camera: residual (6), Jacobian block (9), pad
constexpr int kPtVals = 16;               // per point: Q (6 packed symmetric), g (3), Z (6), pad (1)
constexpr int kTaskVals = 72;             // per block task partial: camera task 51 values (69 when
                                          // self-calibrating), pair task 36
constexpr int kPtPartVals = 32;           // per point-pass wavefront: intrinsic-intrinsic terms (9, or 30
                                          // when self-calibrating)
constexpr int kPtzVals = 12;              // per point when self-calibrating: Z rows of f, cx, cy (9), pad (3)
constexpr int kStatVals = 6;              // reprojection sums of one point-lane workgroup: observations,
                                          // sum |e|, sum |e|^2, and the same over the inliers (|e| <= 3 delta)
constexpr int kIntr = 5;                  // intrinsic state: k1, k2, f, principal-point offset x, y
constexpr int kSolveTb = 16;              // block size of the dense reduced-system factorisation
constexpr int kSolveTbVals = kSolveTb * (kSolveTb + 1);   // doubles per block (rows padded to 17)
constexpr int kCgThreads = 512;           // threads per workgroup of the conjugate-gradient solve
constexpr int kCgWaves = kCgThreads / kWave;
constexpr int kMaxCgWG = 128;             // workgroups of one cluster's conjugate-gradient solve, at most
// block rows of one conjugate-gradient workgroup, at most: their owner
// threads fit in wavefront 0, and each scalar row of S p has a thread
constexpr int kCgMaxRows = kWave < kCgThreads / 6 ? kWave : kCgThreads / 6;
constexpr int kSbRow = 8;                 // sparse reduced-system block: 6 rows padded to 8 values
constexpr int kSbVals = 6 * kSbRow;       //   (16-byte aligned rows for vector loads)
// Work items of the block-assembly kernel (one wavefront each) and of its
// reduction: int4 {kind << 24 | cam_a << 12 | cam_b, begin, end/count, 0}.
enum TaskKind { TASK_CAM = 0, TASK_PAIR = 1, TARGET_INTR = 2 };

enum SlotStatus { ST_QUEUED = 0, ST_RUNNING = 1, ST_MAXITER = 2, ST_CONVERGED = 3, ST_STALLED = 4, ST_BAD_INIT = 5 };

}  // namespace bagpu
