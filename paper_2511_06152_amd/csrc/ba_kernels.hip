// HIP kernels (gfx950) of the cluster bundle-adjustment library.
//
// One Levenberg-Marquardt iteration over a batch of resident clusters is five
// launches, each covering every cluster of the batch:
//
//   k_assemble<Real>   per observation: residual of Eq. (5) with k1/k2 radial
//                      terms, Huber IRLS weight (robust rho of Eq. 6/7),
//                      analytic Jacobians; per point (wavefront-segmented sum):
//                      V_j, g_j, damped inverse; per camera pair: Schur
//                      complement blocks accumulated in LDS (ds_add), one
//                      partial reduced system per workgroup
//   k_reduce           fixed-order sum of the workgroup partials, in FP64
//   k_solve            one workgroup per cluster: pose priors, Marquardt
//                      damping, FP64 Cholesky of the reduced camera system,
//                      triangular solves (+ one FP64 refinement step in mixed
//                      mode), trial camera poses and prior cost, camera part of
//                      the predicted reduction
//   k_backsub<Real>    per point back-substitution, trial points, and the FP64
//                      trial cost of every observation
//   k_lm               gain ratio, accept/reject, Nielsen damping update,
//                      termination; flips the state buffers on acceptance
//
// Observations are laid out in 64-lane chunks sorted by (point, camera), so a
// point's observations are contiguous lanes of one wavefront.  Real is double
// (plain path) or float (mixed path: FP32 residuals, Jacobians and Schur
// accumulation; FP64 solve, cost reductions and gain ratio).
#include <math.h>

#include "ba_device.h"

namespace bagpu {
namespace {

constexpr double kLambdaMin = 1e-16, kLambdaMax = 1e32;
constexpr double kDiagMin = 1e-6, kDiagMax = 1e32;
constexpr double kAcceptRatio = 1e-3;

__device__ __forceinline__ int find_slot(const int* __restrict__ wg_off, int n_act, int b) {
  int lo = 0, hi = n_act - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wg_off[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Packed storage of a symmetric matrix: element (r, c), r <= c.
__device__ __forceinline__ int pidx(int r, int c) { return c * (c + 1) / 2 + r; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T> __device__ __forceinline__ T clampd(T d) {
  return d < T(kDiagMin) ? T(kDiagMin) : (d > T(kDiagMax) ? T(kDiagMax) : d);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
  return v;
}

// ---- SO(3) (FP64) -----------------------------------------------------------

__device__ void so3_exp(const double w[3], double R[9]) {
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double th = sqrt(th2);
  double a, b;
  if (th < 1e-8) { a = 1.0; b = 0.5; }
  else { a = sin(th) / th; b = (1.0 - cos(th)) / th2; }
  const double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double k2 = 0;
      for (int l = 0; l < 3; ++l) k2 += K[3 * i + l] * K[3 * l + j];
      R[3 * i + j] = (i == j ? 1.0 : 0.0) + a * K[3 * i + j] + b * k2;
    }
}

__device__ void so3_log(const double R[9], double w[3]) {
  double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
  c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
  const double th = acos(c);
  const double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
  if (th < 1e-6) {
    const double s = 0.5 * (1.0 + th * th / 6.0);
    for (int i = 0; i < 3; ++i) w[i] = s * v[i];
  } else if (th < M_PI - 1e-6) {
    const double s = th / (2.0 * sin(th));
    for (int i = 0; i < 3; ++i) w[i] = s * v[i];
  } else {
    int k = 0;
    if (R[4] > R[4 * k]) k = 1;
    if (R[8] > R[4 * k]) k = 2;
    const double d = sqrt(0.5 * (R[4 * k] + 1.0));
    double a[3];
    for (int i = 0; i < 3; ++i) a[i] = (i == k) ? d : 0.25 * (R[3 * i + k] + R[3 * k + i]) / d;
    const double n = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const double sg = (a[0] * v[0] + a[1] * v[1] + a[2] * v[2]) < 0 ? -1.0 : 1.0;
    for (int i = 0; i < 3; ++i) w[i] = sg * th * a[i] / n;
  }
}

// Whitened prior residual e[6] of camera state cam (R, T) and its Jacobian
// block d e_omega / d domega = diag(1/sigma_omega) Jr^-1(phi) (3x3).
__device__ void prior_terms(const double* __restrict__ cam, const double* __restrict__ pr, double e[6],
                            double J[9]) {
  double M[9];   // R_prior^T R
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      M[3 * i + j] = pr[i] * cam[j] + pr[3 + i] * cam[3 + j] + pr[6 + i] * cam[6 + j];
  double phi[3];
  so3_log(M, phi);
  const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  const double th = sqrt(th2);
  const double cc = th < 1e-4 ? 1.0 / 12.0 + th2 / 720.0 : 1.0 / th2 - (1.0 + cos(th)) / (2.0 * th * sin(th));
  const double K[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
  for (int i = 0; i < 3; ++i) {
    e[i] = phi[i] * pr[12 + i];
    e[3 + i] = (cam[9 + i] - pr[9 + i]) * pr[15 + i];
    for (int j = 0; j < 3; ++j) {
      double k2 = 0;
      for (int l = 0; l < 3; ++l) k2 += K[3 * i + l] * K[3 * l + j];
      J[3 * i + j] = ((i == j ? 1.0 : 0.0) + 0.5 * K[3 * i + j] + cc * k2) * pr[12 + i];
    }
  }
}

// ---- per-observation model ------------------------------------------------------

template <typename R>
struct ObsJ {
  R xc[3];
  R e[2];       // whitened residual
  R w;          // IRLS weight rho'(s)
  R Jp[2][3];   // whitened d(u,v)/dX
  R Jw[2][3];   // whitened d(u,v)/d omega
  R Jk[2][2];   // whitened d(u,v)/d(k1, k2)
};

// Residual, Huber weight and Jacobians of one observation.  cam = R (9,
// row-major, camera->world), T (3).  Invalid lanes get w = 0 and finite values.
template <typename R>
__device__ __forceinline__ void obs_model(const R* __restrict__ cam, const R X0, const R X1, const R X2, const R u,
                                          const R v, const R f, const R k1, const R k2, const R is, const R dt,
                                          bool valid, ObsJ<R>& o) {
  const R d0 = X0 - cam[9], d1 = X1 - cam[10], d2 = X2 - cam[11];
  R x = cam[0] * d0 + cam[3] * d1 + cam[6] * d2;
  R y = cam[1] * d0 + cam[4] * d1 + cam[7] * d2;
  R z = cam[2] * d0 + cam[5] * d1 + cam[8] * d2;
  if (!valid || !(z > R(0))) { x = R(0); y = R(0); z = R(1); valid = false; }
  o.xc[0] = x; o.xc[1] = y; o.xc[2] = z;
  const R iz = R(1) / z;
  const R a = x * iz, b = y * iz;
  const R r2 = a * a + b * b;
  const R D = R(1) + k1 * r2 + k2 * r2 * r2;
  const R fis = f * is;
  o.e[0] = (f * D * a - u) * is;
  o.e[1] = (f * D * b - v) * is;
  const R s = o.e[0] * o.e[0] + o.e[1] * o.e[1];
  o.w = valid ? (s <= dt * dt ? R(1) : dt / sqrt(s)) : R(0);
  const R q = k1 + R(2) * k2 * r2;
  const R A00 = fis * (D + R(2) * a * a * q), A01 = fis * (R(2) * a * b * q), A11 = fis * (D + R(2) * b * b * q);
  const R Jx[2][3] = {{A00 * iz, A01 * iz, -(A00 * a + A01 * b) * iz},
                      {A01 * iz, A11 * iz, -(A01 * a + A11 * b) * iz}};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) o.Jp[i][j] = Jx[i][0] * cam[3 * j] + Jx[i][1] * cam[3 * j + 1] + Jx[i][2] * cam[3 * j + 2];
    o.Jw[i][0] = Jx[i][1] * z - Jx[i][2] * y;
    o.Jw[i][1] = Jx[i][2] * x - Jx[i][0] * z;
    o.Jw[i][2] = Jx[i][0] * y - Jx[i][1] * x;
  }
  const R r4 = r2 * r2;
  o.Jk[0][0] = fis * r2 * a; o.Jk[0][1] = fis * r4 * a;
  o.Jk[1][0] = fis * r2 * b; o.Jk[1][1] = fis * r4 * b;
}

// Camera-side whitened Jacobian column r (0..5) of row i: [Jw | -Jp].
template <typename R>
__device__ __forceinline__ R jc(const ObsJ<R>& o, int i, int r) { return r < 3 ? o.Jw[i][r] : -o.Jp[i][r - 3]; }

// Huber rho of the squared whitened norm s, dt = delta / sigma.
__device__ __forceinline__ double huber_rho(double s, double dt) {
  return s <= dt * dt ? s : 2.0 * dt * sqrt(s) - dt * dt;
}

// FP64 residual rho(s) of one observation; returns false at non-positive depth.
__device__ __forceinline__ bool obs_rho(const double* __restrict__ cam, const double X[3], double u, double v, double f,
                                        double k1, double k2, double is, double dt, double* rho) {
  const double d0 = X[0] - cam[9], d1 = X[1] - cam[10], d2 = X[2] - cam[11];
  const double x = cam[0] * d0 + cam[3] * d1 + cam[6] * d2;
  const double y = cam[1] * d0 + cam[4] * d1 + cam[7] * d2;
  const double z = cam[2] * d0 + cam[5] * d1 + cam[8] * d2;
  if (!(z > 0.0)) { *rho = 0.0; return false; }
  const double a = x / z, b = y / z;
  const double r2 = a * a + b * b;
  const double D = 1.0 + k1 * r2 + k2 * r2 * r2;
  const double e0 = (f * D * a - u) * is, e1 = (f * D * b - v) * is;
  *rho = huber_rho(e0 * e0 + e1 * e1, dt);
  return true;
}

// Inverse of the 3x3 SPD matrix (a00 a01 a02 a11 a12 a22) via Cholesky.
template <typename R>
__device__ __forceinline__ bool spd3_inv(const R A[6], R Q[6]) {
  const R l00s = A[0];
  if (!(l00s > R(0))) return false;
  const R l00 = sqrt(l00s);
  const R l10 = A[1] / l00, l20 = A[2] / l00;
  const R l11s = A[3] - l10 * l10;
  if (!(l11s > R(0))) return false;
  const R l11 = sqrt(l11s);
  const R l21 = (A[4] - l20 * l10) / l11;
  const R l22s = A[5] - l20 * l20 - l21 * l21;
  if (!(l22s > R(0))) return false;
  const R l22 = sqrt(l22s);
  const R i00 = R(1) / l00, i11 = R(1) / l11, i22 = R(1) / l22;
  const R i10 = -l10 * i00 * i11;
  const R i21 = -l21 * i11 * i22;
  const R i20 = -(l20 * i00 + l21 * i10) * i22;
  Q[0] = i00 * i00 + i10 * i10 + i20 * i20;
  Q[1] = i10 * i11 + i20 * i21;
  Q[2] = i20 * i22;
  Q[3] = i11 * i11 + i21 * i21;
  Q[4] = i21 * i22;
  Q[5] = i22 * i22;
  return true;
}

template <typename R>
__device__ __forceinline__ R qel(const R Q[6], int i, int j) {
  const int a = i < j ? i : j, b = i < j ? j : i;
  return Q[a == 0 ? b : (a == 1 ? 2 + b : 5)];
}

// ---- admission: origin shift, state buffers, LM control ---------------------------

__global__ void k_prep_slot(Batch bt) {
  const int s = bt.act[blockIdx.x];
  const SlotDesc& d = bt.desc[s];
  SlotCtl& c = bt.ctl[s];
  __shared__ double org[3];
  if (threadIdx.x == 0) {
    double o[3] = {0, 0, 0};
    for (int k = 0; k < d.C; ++k)
      for (int i = 0; i < 3; ++i) o[i] += d.raw_cam[30 * k + 9 + i];
    for (int i = 0; i < 3; ++i) { org[i] = o[i] / d.C; c.origin[i] = org[i]; }
    double l0 = d.lambda0;
    if (!(l0 >= kLambdaMin)) l0 = kLambdaMin;
    if (l0 > kLambdaMax) l0 = kLambdaMax;
    c.lambda = l0;
    c.nu = 2.0;
    c.cur = 0;
    c.status = ST_RUNNING;
    c.iter = c.accepted = c.rejected = 0;
    c.solve_ok = 1;
    c.point_fail = 0;
    c.bad_init = 0;
    c.k[1][0] = c.k[0][0];
    c.k[1][1] = c.k[0][1];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < d.C; k += blockDim.x) {
    const double* r = d.raw_cam + 30 * k;
    for (int b = 0; b < 2; ++b) {
      double* cam = d.cam[b] + kCamVals * k;
      for (int i = 0; i < 9; ++i) cam[i] = r[i];
      for (int i = 0; i < 3; ++i) cam[9 + i] = r[9 + i] - org[i];
    }
    double* pr = d.prior + kPriorVals * k;
    for (int i = 0; i < 9; ++i) pr[i] = r[12 + i];
    for (int i = 0; i < 3; ++i) pr[9 + i] = r[21 + i] - org[i];
    for (int i = 0; i < 6; ++i) {
      const double sg = r[24 + i];
      pr[12 + i] = (sg > 0.0 && isfinite(sg)) ? 1.0 / sg : 0.0;
    }
  }
}

__global__ void k_prep_points(Batch bt) {
  const int s = bt.act[blockIdx.y];
  const SlotDesc& d = bt.desc[s];
  const SlotCtl& c = bt.ctl[s];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.P) {
    for (int t = 0; t < 3; ++t) {
      const double x = d.X[0][3 * i + t] - c.origin[t];
      d.X[0][3 * i + t] = x;
      d.X[1][3 * i + t] = x;
      d.X32[0][3 * i + t] = (float)x;
      d.X32[1][3 * i + t] = (float)x;
    }
  }
  if (i < d.L) {
    const double u = d.lane_uv64[2 * i] - d.cx, v = d.lane_uv64[2 * i + 1] - d.cy;
    d.lane_uv64[2 * i] = u;
    d.lane_uv64[2 * i + 1] = v;
    d.lane_uv32[2 * i] = (float)u;
    d.lane_uv32[2 * i + 1] = (float)v;
  }
}

// ---- FP64 cost of the current state (admission) -----------------------------------

__global__ __launch_bounds__(kWG) void k_cost0(Batch bt) {
  extern __shared__ double sh_cam[];
  const int si = find_slot(bt.wg_off, bt.n_act, blockIdx.x);
  const int s = bt.act[si];
  const int wgl = blockIdx.x - bt.wg_off[si];
  const SlotDesc& d = bt.desc[s];
  const SlotCtl& c = bt.ctl[s];
  const int cur = c.cur;
  for (int i = threadIdx.x; i < d.C * kCamVals; i += kWG) sh_cam[i] = d.cam[cur][i];
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const double k1 = c.k[cur][0], k2 = c.k[cur][1];
  double acc = 0.0;
  int bad = 0;
  const int c0 = wgl * d.cpw, c1 = min(c0 + d.cpw, d.n_chunks);
  for (int ch = c0 + wave; ch < c1; ch += kWavesPerWG) {
    const int idx = ch * kWave + lane;
    const int pt = d.lane_pt[idx];
    if (pt >= 0) {
      const int cam = d.lane_cam[idx];
      const double X[3] = {d.X[cur][3 * pt], d.X[cur][3 * pt + 1], d.X[cur][3 * pt + 2]};
      double rho;
      if (obs_rho(sh_cam + kCamVals * cam, X, d.lane_uv64[2 * idx], d.lane_uv64[2 * idx + 1], d.f, k1, k2,
                  d.inv_sigma, d.huber_dt, &rho)) acc += rho;
      else ++bad;
    }
  }
  __shared__ double red[kWavesPerWG];
  __shared__ int redb[kWavesPerWG];
  acc = wave_sum(acc);
  bad = wave_sum(bad);
  if (lane == 0) { red[wave] = acc; redb[wave] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    int b = 0;
    for (int w = 0; w < kWavesPerWG; ++w) { t += red[w]; b += redb[w]; }
    d.cost_part[2 * wgl] = t;
    d.cost_part[2 * wgl + 1] = 0.0;
    d.bad_part[wgl] = b;
  }
}

__global__ void k_init(Batch bt) {
  const int s = bt.act[blockIdx.x];
  const SlotDesc& d = bt.desc[s];
  SlotCtl& c = bt.ctl[s];
  if (threadIdx.x != 0) return;
  double rho = 0.0;
  int bad = 0;
  for (int w = 0; w < d.n_wg; ++w) { rho += d.cost_part[2 * w]; bad += d.bad_part[w]; }
  double pr = 0.0;
  for (int k = 0; k < d.C; ++k) {
    if (d.cam_col[k] < 0) continue;
    double e[6], J[9];
    prior_terms(d.cam[c.cur] + kCamVals * k, d.prior + kPriorVals * k, e, J);
    for (int i = 0; i < 6; ++i) pr += e[i] * e[i];
  }
  const double E = 0.5 * rho + 0.5 * pr;
  c.E = E;
  c.E0 = E;
  d.cost_log[0] = E;
  if (bad > 0 || !isfinite(E)) { c.status = ST_BAD_INIT; c.bad_init = bad > 0 ? bad : 1; }
  else if (d.max_iters <= 0) c.status = ST_MAXITER;
}

// ---- assembly: residuals, Jacobians, point blocks, Schur complement ----------------
//
// LDS: acc[pstride] (packed S, g, bS, diag U), cameras [C][12], camera columns
// [C], per-wave scratch [4][kScr][64].
template <typename R>
__global__ __launch_bounds__(kWG) void k_assemble(Batch bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int si = find_slot(bt.wg_off, bt.n_act, blockIdx.x);
  const int s = bt.act[si];
  const int wgl = blockIdx.x - bt.wg_off[si];
  const SlotDesc& d = bt.desc[s];
  SlotCtl& c = bt.ctl[s];
  if (c.status != ST_RUNNING) return;
  const int m = d.m, psize = d.psize, pstride = d.pstride;
  R* acc = reinterpret_cast<R*>(smem);
  R* scam = acc + bt.max_pstride;
  R* scr_all = scam + bt.max_C * kCamVals;
  int* scol = reinterpret_cast<int*>(scr_all + kWavesPerWG * kScr * kWave);
  const int cur = c.cur;
  for (int i = threadIdx.x; i < pstride; i += kWG) acc[i] = R(0);
  for (int i = threadIdx.x; i < d.C * kCamVals; i += kWG) scam[i] = (R)d.cam[cur][i];
  for (int i = threadIdx.x; i < d.C; i += kWG) scol[i] = d.cam_col[i];
  __syncthreads();

  R* g_acc = acc + psize;
  R* bs_acc = g_acc + m;
  R* du_acc = bs_acc + m;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  R* scr = scr_all + wave * kScr * kWave;
  const double lambda = c.lambda;
  const R lam = (R)lambda;
  const R f = (R)d.f, is = (R)d.inv_sigma, dt = (R)d.huber_dt;
  const R k1 = (R)c.k[cur][0], k2 = (R)c.k[cur][1];
  const int kc0 = d.kcol0, kc1 = d.kcol1;
  const bool intr = (kc0 >= 0) || (kc1 >= 0);
  const bool mixed = sizeof(R) == 4;
  R* __restrict__ ptv = reinterpret_cast<R*>(d.ptv);
  // per-lane running sums of the intrinsic-intrinsic terms
  R iU00 = 0, iU01 = 0, iU11 = 0, ig0 = 0, ig1 = 0, id0 = 0, id1 = 0, ib0 = 0, ib1 = 0;
  bool fail = false;

  const int c0 = wgl * d.cpw, c1 = min(c0 + d.cpw, d.n_chunks);
  for (int ch = c0 + wave; ch < c1; ch += kWavesPerWG) {
    const int idx = ch * kWave + lane;
    const int pt = d.lane_pt[idx];
    const bool valid = pt >= 0;
    const int cam = valid ? d.lane_cam[idx] : 0;
    const int seg = d.lane_seg[idx];
    const int sb = seg >> 8, sl = seg & 255;
    const int maxl = wave_max(sl);
    const bool head = valid && sb == lane;
    R X0 = 0, X1 = 0, X2 = 0, u = 0, v = 0;
    if (valid) {
      if (mixed) {
        X0 = (R)d.X32[cur][3 * pt]; X1 = (R)d.X32[cur][3 * pt + 1]; X2 = (R)d.X32[cur][3 * pt + 2];
        u = (R)d.lane_uv32[2 * idx]; v = (R)d.lane_uv32[2 * idx + 1];
      } else {
        X0 = (R)d.X[cur][3 * pt]; X1 = (R)d.X[cur][3 * pt + 1]; X2 = (R)d.X[cur][3 * pt + 2];
        u = (R)d.lane_uv64[2 * idx]; v = (R)d.lane_uv64[2 * idx + 1];
      }
    }
    ObsJ<R> o;
    obs_model<R>(scam + kCamVals * cam, X0, X1, X2, u, v, f, k1, k2, is, dt, valid, o);
    const R w = o.w;
    R wJp[2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int t = 0; t < 3; ++t) wJp[i][t] = w * o.Jp[i][t];

    // --- point blocks: segmented sums over the point's lanes -------------------
    R vals[15];
    vals[0] = o.Jp[0][0] * wJp[0][0] + o.Jp[1][0] * wJp[1][0];
    vals[1] = o.Jp[0][0] * wJp[0][1] + o.Jp[1][0] * wJp[1][1];
    vals[2] = o.Jp[0][0] * wJp[0][2] + o.Jp[1][0] * wJp[1][2];
    vals[3] = o.Jp[0][1] * wJp[0][1] + o.Jp[1][1] * wJp[1][1];
    vals[4] = o.Jp[0][1] * wJp[0][2] + o.Jp[1][1] * wJp[1][2];
    vals[5] = o.Jp[0][2] * wJp[0][2] + o.Jp[1][2] * wJp[1][2];
#pragma unroll
    for (int t = 0; t < 3; ++t) vals[6 + t] = wJp[0][t] * o.e[0] + wJp[1][t] * o.e[1];
    R Wi[2][3];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int t = 0; t < 3; ++t) Wi[b][t] = o.Jk[0][b] * wJp[0][t] + o.Jk[1][b] * wJp[1][t];
    const int nv = intr ? 15 : 9;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int t = 0; t < 3; ++t) vals[9 + 3 * b + t] = Wi[b][t];
    wave_sync();
    for (int i = 0; i < nv; ++i) scr[i * kWave + lane] = vals[i];
    wave_sync();
    R sum[15];
#pragma unroll
    for (int i = 0; i < 15; ++i) sum[i] = R(0);
    for (int t = 0; t < maxl; ++t) {
      if (t < sl) {
        const int src = sb + t;
        for (int i = 0; i < nv; ++i) sum[i] += scr[i * kWave + src];
      }
    }
    // damped point block and its inverse
    R Dp[3] = {clampd(sum[0]), clampd(sum[3]), clampd(sum[5])};
    R Vl[6] = {sum[0] + lam * Dp[0], sum[1], sum[2], sum[3] + lam * Dp[1], sum[4], sum[5] + lam * Dp[2]};
    R Q[6];
    if (!spd3_inv(Vl, Q)) {
      if (valid) fail = true;
      for (int i = 0; i < 6; ++i) Q[i] = R(0);
    }
    const R gp[3] = {sum[6], sum[7], sum[8]};
    if (head) {
      R* pv = ptv + kPtVals * (size_t)pt;
      for (int i = 0; i < 6; ++i) pv[i] = Q[i];
      for (int i = 0; i < 3; ++i) pv[6 + i] = gp[i];
      for (int i = 0; i < 3; ++i) pv[9 + i] = Dp[i];
    }

    // --- camera-side blocks of this observation -----------------------------
    const int fi = valid ? scol[cam] : -1;
    R Wc[6][3];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int t = 0; t < 3; ++t) Wc[r][t] = jc(o, 0, r) * wJp[0][t] + jc(o, 1, r) * wJp[1][t];
    R Y[6][3];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int t = 0; t < 3; ++t)
        Y[r][t] = Wc[r][0] * qel(Q, 0, t) + Wc[r][1] * qel(Q, 1, t) + Wc[r][2] * qel(Q, 2, t);
    const R Z[2][3] = {{sum[9], sum[10], sum[11]}, {sum[12], sum[13], sum[14]}};
    if (fi >= 0) {
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        const R jr0 = jc(o, 0, r), jr1 = jc(o, 1, r);
#pragma unroll
        for (int cc = r; cc < 6; ++cc) {
          const R uval = w * (jr0 * jc(o, 0, cc) + jr1 * jc(o, 1, cc));
          const R val = uval - (Y[r][0] * Wc[cc][0] + Y[r][1] * Wc[cc][1] + Y[r][2] * Wc[cc][2]);
          atomicAdd(&acc[pidx(fi + r, fi + cc)], val);
          if (cc == r) atomicAdd(&du_acc[fi + r], uval);
        }
        atomicAdd(&g_acc[fi + r], w * (jr0 * o.e[0] + jr1 * o.e[1]));
        atomicAdd(&bs_acc[fi + r], Y[r][0] * gp[0] + Y[r][1] * gp[1] + Y[r][2] * gp[2]);
        if (kc0 >= 0)
          atomicAdd(&acc[pidx(fi + r, kc0)], w * (jr0 * o.Jk[0][0] + jr1 * o.Jk[1][0]) -
                                                 (Y[r][0] * Z[0][0] + Y[r][1] * Z[0][1] + Y[r][2] * Z[0][2]));
        if (kc1 >= 0)
          atomicAdd(&acc[pidx(fi + r, kc1)], w * (jr0 * o.Jk[0][1] + jr1 * o.Jk[1][1]) -
                                                 (Y[r][0] * Z[1][0] + Y[r][1] * Z[1][1] + Y[r][2] * Z[1][2]));
      }
    }
    if (intr) {
      iU00 += w * (o.Jk[0][0] * o.Jk[0][0] + o.Jk[1][0] * o.Jk[1][0]);
      iU01 += w * (o.Jk[0][0] * o.Jk[0][1] + o.Jk[1][0] * o.Jk[1][1]);
      iU11 += w * (o.Jk[0][1] * o.Jk[0][1] + o.Jk[1][1] * o.Jk[1][1]);
      id0 += w * (o.Jk[0][0] * o.Jk[0][0] + o.Jk[1][0] * o.Jk[1][0]);
      id1 += w * (o.Jk[0][1] * o.Jk[0][1] + o.Jk[1][1] * o.Jk[1][1]);
      ig0 += w * (o.Jk[0][0] * o.e[0] + o.Jk[1][0] * o.e[1]);
      ig1 += w * (o.Jk[0][1] * o.e[0] + o.Jk[1][1] * o.e[1]);
      if (head) {
        R ZQ[2][3];
        for (int b = 0; b < 2; ++b)
          for (int t = 0; t < 3; ++t)
            ZQ[b][t] = Z[b][0] * qel(Q, 0, t) + Z[b][1] * qel(Q, 1, t) + Z[b][2] * qel(Q, 2, t);
        iU00 -= ZQ[0][0] * Z[0][0] + ZQ[0][1] * Z[0][1] + ZQ[0][2] * Z[0][2];
        iU01 -= ZQ[0][0] * Z[1][0] + ZQ[0][1] * Z[1][1] + ZQ[0][2] * Z[1][2];
        iU11 -= ZQ[1][0] * Z[1][0] + ZQ[1][1] * Z[1][1] + ZQ[1][2] * Z[1][2];
        ib0 += ZQ[0][0] * gp[0] + ZQ[0][1] * gp[1] + ZQ[0][2] * gp[2];
        ib1 += ZQ[1][0] * gp[0] + ZQ[1][1] * gp[1] + ZQ[1][2] * gp[2];
      }
    }

    // --- camera-camera blocks of observation pairs of this point -------------
    if (maxl > 1) {
      wave_sync();
#pragma unroll
      for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int t = 0; t < 3; ++t) scr[(3 * r + t) * kWave + lane] = Wc[r][t];
      wave_sync();
      for (int t = 0; t < maxl; ++t) {
        const int src = sb + (t < sl ? t : 0);
        const int fib = __shfl(fi, src, kWave);
        if (t < sl && fi >= 0 && fib > fi) {
          R Wb[6][3];
#pragma unroll
          for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q) Wb[r][q] = scr[(3 * r + q) * kWave + src];
#pragma unroll
          for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int cc = 0; cc < 6; ++cc)
              atomicAdd(&acc[pidx(fi + r, fib + cc)],
                        -(Y[r][0] * Wb[cc][0] + Y[r][1] * Wb[cc][1] + Y[r][2] * Wb[cc][2]));
        }
      }
    }
  }
  if (fail) atomicOr(&c.point_fail, 1);
  if (intr) {
    iU00 = wave_sum(iU00); iU01 = wave_sum(iU01); iU11 = wave_sum(iU11);
    id0 = wave_sum(id0); id1 = wave_sum(id1);
    ig0 = wave_sum(ig0); ig1 = wave_sum(ig1);
    ib0 = wave_sum(ib0); ib1 = wave_sum(ib1);
    if (lane == 0) {
      if (kc0 >= 0) {
        atomicAdd(&acc[pidx(kc0, kc0)], iU00);
        atomicAdd(&du_acc[kc0], id0);
        atomicAdd(&g_acc[kc0], ig0);
        atomicAdd(&bs_acc[kc0], ib0);
      }
      if (kc1 >= 0) {
        atomicAdd(&acc[pidx(kc1, kc1)], iU11);
        atomicAdd(&du_acc[kc1], id1);
        atomicAdd(&g_acc[kc1], ig1);
        atomicAdd(&bs_acc[kc1], ib1);
      }
      if (kc0 >= 0 && kc1 >= 0) atomicAdd(&acc[pidx(kc0, kc1)], iU01);
    }
  }
  __syncthreads();
  R* part = reinterpret_cast<R*>(d.partial) + (size_t)wgl * pstride;
  for (int i = threadIdx.x; i < pstride; i += kWG) part[i] = acc[i];
}

// ---- fixed-order reduction of the workgroup partials ---------------------------

template <typename R>
__global__ __launch_bounds__(256) void k_reduce(Batch bt) {
  const int s = bt.act[blockIdx.y];
  const SlotDesc& d = bt.desc[s];
  if (bt.ctl[s].status != ST_RUNNING) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.pstride) return;
  const R* part = reinterpret_cast<const R*>(d.partial);
  double t = 0.0;
  for (int w = 0; w < d.n_wg; ++w) t += (double)part[(size_t)w * d.pstride + i];
  d.Sg[i] = t;
}

// ---- damped reduced-camera-system solve (one workgroup per cluster) ------------

constexpr int kSolveThreads = 256;

__device__ void tri_solve(const double* __restrict__ L, double* x, int m, int tid) {
  // L L^T x = x (in place), packed lower storage L(i, j) = L[pidx(j, i)], j <= i.
  for (int k = 0; k < m; ++k) {
    if (tid == 0) x[k] = x[k] / L[pidx(k, k)];
    __syncthreads();
    const double xk = x[k];
    for (int i = k + 1 + tid; i < m; i += kSolveThreads) x[i] -= L[pidx(k, i)] * xk;
    __syncthreads();
  }
  for (int k = m - 1; k >= 0; --k) {
    if (tid == 0) x[k] = x[k] / L[pidx(k, k)];
    __syncthreads();
    const double xk = x[k];
    for (int i = tid; i < k; i += kSolveThreads) x[i] -= L[pidx(i, k)] * xk;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kSolveThreads) void k_solve(Batch bt) {
  extern __shared__ double sd[];
  const int s = bt.act[blockIdx.x];
  const SlotDesc& d = bt.desc[s];
  SlotCtl& c = bt.ctl[s];
  if (c.status != ST_RUNNING) return;
  const int tid = threadIdx.x;
  const int m = d.m, psize = d.psize;
  double* A = sd;              // packed, factorised in place
  double* gv = A + psize;      // gradient (camera side, with priors)
  double* Dv = gv + m;         // clamped diagonal of H
  double* xv = Dv + m;         // right-hand side / solution
  double* rv = xv + m;         // refinement residual
  double* red = rv + m;        // reduction scratch [kSolveThreads]
  __shared__ int ok;
  const double lambda = c.lambda;
  const int cur = c.cur;
  for (int i = tid; i < psize; i += kSolveThreads) A[i] = d.Sg[i];
  for (int i = tid; i < m; i += kSolveThreads) {
    gv[i] = d.Sg[psize + i];
    xv[i] = d.Sg[psize + m + i];        // bS for now
    Dv[i] = d.Sg[psize + 2 * m + i];    // diag U for now
  }
  if (tid == 0) ok = (c.point_fail == 0);
  __syncthreads();
  // pose priors of the free cameras (each thread owns whole camera blocks)
  for (int k = tid; k < d.C; k += kSolveThreads) {
    const int col = d.cam_col[k];
    if (col < 0) continue;
    double e[6], J[9];
    prior_terms(d.cam[cur] + kCamVals * k, d.prior + kPriorVals * k, e, J);
    const double* pr = d.prior + kPriorVals * k;
    for (int r = 0; r < 3; ++r) {
      for (int q = r; q < 3; ++q) {
        const double h = J[r] * J[q] + J[3 + r] * J[3 + q] + J[6 + r] * J[6 + q];
        A[pidx(col + r, col + q)] += h;
        if (q == r) Dv[col + r] += h;
      }
      gv[col + r] += J[r] * e[0] + J[3 + r] * e[1] + J[6 + r] * e[2];
      const double it = pr[15 + r];
      A[pidx(col + 3 + r, col + 3 + r)] += it * it;
      Dv[col + 3 + r] += it * it;
      gv[col + 3 + r] += it * e[3 + r];
    }
  }
  __syncthreads();
  for (int i = tid; i < m; i += kSolveThreads) {
    const double Di = clampd(Dv[i]);
    Dv[i] = Di;
    A[pidx(i, i)] += lambda * Di;
    xv[i] = -gv[i] + xv[i];
    rv[i] = xv[i];
  }
  __syncthreads();
  if (d.mixed)
    for (int i = tid; i < psize; i += kSolveThreads) d.Sd[i] = A[i];
  // right-looking Cholesky, packed lower: L(i, j) at pidx(j, i)
  for (int k = 0; k < m; ++k) {
    if (tid == 0) {
      const double a = A[pidx(k, k)];
      if (!(a > 0.0) || !isfinite(a)) ok = 0;
      else A[pidx(k, k)] = sqrt(a);
    }
    __syncthreads();
    if (!ok) break;
    const double dkk = A[pidx(k, k)];
    for (int i = k + 1 + tid; i < m; i += kSolveThreads) A[pidx(k, i)] /= dkk;
    __syncthreads();
    const int rows = m - k - 1;
    const int total = rows * (rows + 1) / 2;
    for (int e = tid; e < total; e += kSolveThreads) {
      int ii = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
      while (ii * (ii + 1) / 2 > e) --ii;
      while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
      const int jj = e - ii * (ii + 1) / 2;
      const int i = k + 1 + ii, j = k + 1 + jj;   // j <= i
      A[pidx(j, i)] -= A[pidx(k, i)] * A[pidx(k, j)];
    }
    __syncthreads();
  }
  if (!ok) {
    if (tid == 0) c.solve_ok = 0;
    return;
  }
  tri_solve(A, xv, m, tid);
  if (d.mixed) {
    // one FP64 refinement step: r = b - S_damped x, S_damped from the global copy
    for (int i = tid; i < m; i += kSolveThreads) {
      double t = rv[i];
      for (int j = 0; j < m; ++j) t -= d.Sd[i <= j ? pidx(i, j) : pidx(j, i)] * xv[j];
      rv[i] = t;
    }
    __syncthreads();
    tri_solve(A, rv, m, tid);
    for (int i = tid; i < m; i += kSolveThreads) xv[i] += rv[i];
    __syncthreads();
  }
  // camera part of the predicted reduction, fixed-order tree
  double p = 0.0;
  for (int i = tid; i < m; i += kSolveThreads) p += xv[i] * (lambda * Dv[i] * xv[i] - gv[i]);
  red[tid] = p;
  __syncthreads();
  for (int w = kSolveThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  for (int i = tid; i < m; i += kSolveThreads) d.dc[i] = xv[i];
  // trial cameras, intrinsics and prior cost
  const int nxt = 1 - cur;
  double pc = 0.0;
  for (int k = tid; k < d.C; k += kSolveThreads) {
    const double* cm = d.cam[cur] + kCamVals * k;
    double* cn = d.cam[nxt] + kCamVals * k;
    const int col = d.cam_col[k];
    if (col < 0) {
      for (int i = 0; i < kCamVals; ++i) cn[i] = cm[i];
      continue;
    }
    const double wv[3] = {xv[col], xv[col + 1], xv[col + 2]};
    double E[9];
    so3_exp(wv, E);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) cn[3 * i + j] = cm[3 * i] * E[j] + cm[3 * i + 1] * E[3 + j] + cm[3 * i + 2] * E[6 + j];
    for (int i = 0; i < 3; ++i) cn[9 + i] = cm[9 + i] + xv[col + 3 + i];
    double e[6], J[9];
    prior_terms(cn, d.prior + kPriorVals * k, e, J);
    for (int i = 0; i < 6; ++i) pc += e[i] * e[i];
  }
  __syncthreads();
  double* red2 = rv;   // reuse (m >= 0); use red for the prior sum
  (void)red2;
  const double predc = red[0];
  __syncthreads();
  red[tid] = pc;
  __syncthreads();
  for (int w = kSolveThreads / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    c.pred_c = predc;
    c.E_prior_trial = 0.5 * red[0];
    c.k[nxt][0] = c.k[cur][0] + (d.kcol0 >= 0 ? xv[d.kcol0] : 0.0);
    c.k[nxt][1] = c.k[cur][1] + (d.kcol1 >= 0 ? xv[d.kcol1] : 0.0);
  }
}

// ---- back-substitution, trial points and FP64 trial cost -------------------------

template <typename R>
__global__ __launch_bounds__(kWG) void k_backsub(Batch bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int si = find_slot(bt.wg_off, bt.n_act, blockIdx.x);
  const int s = bt.act[si];
  const int wgl = blockIdx.x - bt.wg_off[si];
  const SlotDesc& d = bt.desc[s];
  const SlotCtl& c = bt.ctl[s];
  if (c.status != ST_RUNNING || !c.solve_ok || c.point_fail) return;
  double* tcam = reinterpret_cast<double*>(smem);               // trial cameras FP64
  R* scam = reinterpret_cast<R*>(tcam + bt.max_C * kCamVals);  // current cameras
  R* sdc = scam + bt.max_C * kCamVals;                         // camera update
  R* scr_all = sdc + bt.max_m + 2;
  int* scol = reinterpret_cast<int*>(scr_all + kWavesPerWG * 3 * kWave);
  const int cur = c.cur, nxt = 1 - cur;
  for (int i = threadIdx.x; i < d.C * kCamVals; i += kWG) {
    tcam[i] = d.cam[nxt][i];
    scam[i] = (R)d.cam[cur][i];
  }
  for (int i = threadIdx.x; i < d.m; i += kWG) sdc[i] = (R)d.dc[i];
  for (int i = threadIdx.x; i < d.C; i += kWG) scol[i] = d.cam_col[i];
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  R* scr = scr_all + wave * 3 * kWave;
  const double lambda = c.lambda;
  const R f = (R)d.f, is = (R)d.inv_sigma, dt = (R)d.huber_dt;
  const R k1 = (R)c.k[cur][0], k2 = (R)c.k[cur][1];
  const double tk1 = c.k[nxt][0], tk2 = c.k[nxt][1];
  const int kc0 = d.kcol0, kc1 = d.kcol1;
  const R dk0 = kc0 >= 0 ? sdc[kc0] : R(0), dk1 = kc1 >= 0 ? sdc[kc1] : R(0);
  const bool mixed = sizeof(R) == 4;
  const R* __restrict__ ptv = reinterpret_cast<const R*>(d.ptv);
  double rho_sum = 0.0, pred_sum = 0.0;
  int bad = 0;
  const int c0 = wgl * d.cpw, c1 = min(c0 + d.cpw, d.n_chunks);
  for (int ch = c0 + wave; ch < c1; ch += kWavesPerWG) {
    const int idx = ch * kWave + lane;
    const int pt = d.lane_pt[idx];
    const bool valid = pt >= 0;
    const int cam = valid ? d.lane_cam[idx] : 0;
    const int seg = d.lane_seg[idx];
    const int sb = seg >> 8, sl = seg & 255;
    const int maxl = wave_max(sl);
    const bool head = valid && sb == lane;
    double Xd[3] = {0, 0, 0};
    R X0 = 0, X1 = 0, X2 = 0, u = 0, v = 0;
    if (valid) {
      Xd[0] = d.X[cur][3 * pt]; Xd[1] = d.X[cur][3 * pt + 1]; Xd[2] = d.X[cur][3 * pt + 2];
      if (mixed) {
        X0 = (R)d.X32[cur][3 * pt]; X1 = (R)d.X32[cur][3 * pt + 1]; X2 = (R)d.X32[cur][3 * pt + 2];
        u = (R)d.lane_uv32[2 * idx]; v = (R)d.lane_uv32[2 * idx + 1];
      } else {
        X0 = (R)Xd[0]; X1 = (R)Xd[1]; X2 = (R)Xd[2];
        u = (R)d.lane_uv64[2 * idx]; v = (R)d.lane_uv64[2 * idx + 1];
      }
    }
    ObsJ<R> o;
    obs_model<R>(scam + kCamVals * cam, X0, X1, X2, u, v, f, k1, k2, is, dt, valid, o);
    const int fi = valid ? scol[cam] : -1;
    // t = W_c^T dc + W_i^T dk, with W = w J_side^T J_p
    R tv[3] = {0, 0, 0};
    {
      R jd[2] = {0, 0};   // J_side * d (2-vector)
      if (fi >= 0) {
#pragma unroll
        for (int r = 0; r < 6; ++r) {
          jd[0] += jc(o, 0, r) * sdc[fi + r];
          jd[1] += jc(o, 1, r) * sdc[fi + r];
        }
      }
      jd[0] += o.Jk[0][0] * dk0 + o.Jk[0][1] * dk1;
      jd[1] += o.Jk[1][0] * dk0 + o.Jk[1][1] * dk1;
#pragma unroll
      for (int t = 0; t < 3; ++t) tv[t] = o.w * (o.Jp[0][t] * jd[0] + o.Jp[1][t] * jd[1]);
    }
    wave_sync();
    for (int t = 0; t < 3; ++t) scr[t * kWave + lane] = tv[t];
    wave_sync();
    R ts[3] = {0, 0, 0};
    for (int t = 0; t < maxl; ++t) {
      if (t < sl) {
        const int src = sb + t;
        for (int q = 0; q < 3; ++q) ts[q] += scr[q * kWave + src];
      }
    }
    double Xn[3] = {Xd[0], Xd[1], Xd[2]};
    if (valid) {
      const R* pv = ptv + kPtVals * (size_t)pt;
      R Q[6];
      for (int i = 0; i < 6; ++i) Q[i] = pv[i];
      const R rr[3] = {-pv[6] - ts[0], -pv[7] - ts[1], -pv[8] - ts[2]};
      R dp[3];
      for (int t = 0; t < 3; ++t) dp[t] = qel(Q, t, 0) * rr[0] + qel(Q, t, 1) * rr[1] + qel(Q, t, 2) * rr[2];
      for (int t = 0; t < 3; ++t) Xn[t] = Xd[t] + (double)dp[t];
      if (head) {
        for (int t = 0; t < 3; ++t) {
          const double dd = (double)dp[t];
          pred_sum += dd * (lambda * (double)pv[9 + t] * dd - (double)pv[6 + t]);
          d.X[nxt][3 * pt + t] = Xn[t];
          d.X32[nxt][3 * pt + t] = (float)Xn[t];
        }
      }
      double rho;
      if (obs_rho(tcam + kCamVals * cam, Xn, d.lane_uv64[2 * idx], d.lane_uv64[2 * idx + 1], d.f, tk1, tk2,
                  d.inv_sigma, d.huber_dt, &rho)) rho_sum += rho;
      else ++bad;
    }
  }
  __shared__ double red[2 * kWavesPerWG];
  __shared__ int redb[kWavesPerWG];
  rho_sum = wave_sum(rho_sum);
  pred_sum = wave_sum(pred_sum);
  bad = wave_sum(bad);
  if (lane == 0) { red[2 * wave] = rho_sum; red[2 * wave + 1] = pred_sum; redb[wave] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, p = 0.0;
    int b = 0;
    for (int w = 0; w < kWavesPerWG; ++w) { a += red[2 * w]; p += red[2 * w + 1]; b += redb[w]; }
    d.cost_part[2 * wgl] = a;
    d.cost_part[2 * wgl + 1] = p;
    d.bad_part[wgl] = b;
  }
}

// ---- Levenberg-Marquardt control ---------------------------------------------------

__global__ void k_lm(Batch bt) {
  const int s = bt.act[blockIdx.x];
  const SlotDesc& d = bt.desc[s];
  SlotCtl& c = bt.ctl[s];
  if (threadIdx.x != 0 || c.status != ST_RUNNING) return;
  bool ok = c.solve_ok && !c.point_fail;
  double E2 = INFINITY, pred = 0.0, rho = -INFINITY;
  if (ok) {
    double rs = 0.0, ps = 0.0;
    int bad = 0;
    for (int w = 0; w < d.n_wg; ++w) { rs += d.cost_part[2 * w]; ps += d.cost_part[2 * w + 1]; bad += d.bad_part[w]; }
    if (bad > 0) ok = false;
    E2 = 0.5 * rs + c.E_prior_trial;
    pred = 0.5 * (c.pred_c + ps);
    if (!isfinite(E2)) ok = false;
    if (ok && pred > 0.0) rho = (c.E - E2) / pred;
  }
  const bool accept = ok && rho > kAcceptRatio;
  bool conv = false, stall = false;
  if (accept) {
    const double E = c.E;
    const double rel = (E - E2) / (E > 0.0 ? E : 1e-300);
    c.cur = 1 - c.cur;
    c.E = E2;
    const double t = 2.0 * rho - 1.0;
    double fac = 1.0 - t * t * t;
    if (fac < 1.0 / 3.0) fac = 1.0 / 3.0;
    double lam = c.lambda * fac;
    if (lam < kLambdaMin) lam = kLambdaMin;
    c.lambda = lam;
    c.nu = 2.0;
    c.accepted += 1;
    conv = d.stop_on_ftol && rel < d.ftol;
  } else {
    c.rejected += 1;
    c.lambda *= c.nu;
    c.nu *= 2.0;
    stall = c.lambda > kLambdaMax;
  }
  c.iter += 1;
  d.cost_log[c.iter] = c.E;
  c.status = conv ? ST_CONVERGED : (stall ? ST_STALLED : (c.iter >= d.max_iters ? ST_MAXITER : ST_RUNNING));
  c.solve_ok = 1;
  c.point_fail = 0;
}

// ---- export: undo the origin shift --------------------------------------------------

__global__ void k_export(Batch bt) {
  const int s = bt.act[blockIdx.y];
  const SlotDesc& d = bt.desc[s];
  const SlotCtl& c = bt.ctl[s];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int cur = c.cur;
  if (i < d.P)
    for (int t = 0; t < 3; ++t) d.out[12 * d.C + 3 * i + t] = d.X[cur][3 * i + t] + c.origin[t];
  if (i < d.C) {
    const double* cm = d.cam[cur] + kCamVals * i;
    for (int t = 0; t < 9; ++t) d.out[9 * i + t] = cm[t];
    for (int t = 0; t < 3; ++t) d.out[9 * d.C + 3 * i + t] = cm[9 + t] + c.origin[t];
  }
  if (i == 0) {
    d.out[12 * d.C + 3 * d.P] = c.k[cur][0];
    d.out[12 * d.C + 3 * d.P + 1] = c.k[cur][1];
  }
}

template <typename R>
size_t assemble_smem(const Batch& b) {
  return sizeof(R) * ((size_t)b.max_pstride + (size_t)b.max_C * kCamVals + (size_t)kWavesPerWG * kScr * kWave) +
         sizeof(int) * (size_t)b.max_C;
}

template <typename R>
size_t backsub_smem(const Batch& b) {
  return sizeof(double) * (size_t)b.max_C * kCamVals +
         sizeof(R) * ((size_t)b.max_C * kCamVals + (size_t)b.max_m + 2 + (size_t)kWavesPerWG * 3 * kWave) +
         sizeof(int) * (size_t)b.max_C;
}

size_t solve_smem(const Batch& b) {
  const size_t psize = (size_t)b.max_m * (b.max_m + 1) / 2;
  return sizeof(double) * (psize + 4 * (size_t)b.max_m + kSolveThreads);
}

// Raises a kernel's dynamic-LDS limit to what a launch needs (once per size).
hipError_t ensure_smem(const void* fn, size_t bytes) {
  struct Entry { const void* fn; size_t bytes; };
  static Entry tab[16];
  static int n = 0;
  int i = 0;
  for (; i < n; ++i)
    if (tab[i].fn == fn) break;
  if (i < n && tab[i].bytes >= bytes) return hipSuccess;
  if (bytes <= 64 * 1024) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  if (i == n && n < 16) ++n;
  if (i < 16) tab[i] = Entry{fn, bytes};
  return hipSuccess;
}

}  // namespace

size_t real_size(bool mixed) { return mixed ? sizeof(float) : sizeof(double); }

hipError_t launch_prep(const Batch& b, int max_P_L, hipStream_t st) {
  if (b.n_act == 0) return hipSuccess;
  hipLaunchKernelGGL(k_prep_slot, dim3(b.n_act), dim3(64), 0, st, b);
  if (max_P_L > 0) hipLaunchKernelGGL(k_prep_points, dim3((max_P_L + 255) / 256, b.n_act), dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_initial_cost(const Batch& b, hipStream_t st) {
  if (b.n_act == 0) return hipSuccess;
  if (b.total_wg > 0)
    hipLaunchKernelGGL(k_cost0, dim3(b.total_wg), dim3(kWG), sizeof(double) * b.max_C * kCamVals, st, b);
  hipLaunchKernelGGL(k_init, dim3(b.n_act), dim3(64), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_iteration(const Batch& b, bool mixed, hipStream_t st, hipEvent_t* ev) {
  if (b.n_act == 0) return hipSuccess;
  const dim3 red_grid((b.max_pstride + 255) / 256, b.n_act);
  hipError_t e;
  const size_t s_solve = solve_smem(b);
  if ((e = ensure_smem((const void*)k_solve, s_solve))) return e;
  const size_t sa = mixed ? assemble_smem<float>(b) : assemble_smem<double>(b);
  const size_t sb = mixed ? backsub_smem<float>(b) : backsub_smem<double>(b);
  const void* fa = mixed ? (const void*)k_assemble<float> : (const void*)k_assemble<double>;
  const void* fb = mixed ? (const void*)k_backsub<float> : (const void*)k_backsub<double>;
  if ((e = ensure_smem(fa, sa))) return e;
  if ((e = ensure_smem(fb, sb))) return e;
  auto mark = [&](int i) { if (ev) (void)hipEventRecord(ev[i], st); };
  mark(0);
  if (b.total_wg > 0) {
    if (mixed) hipLaunchKernelGGL(k_assemble<float>, dim3(b.total_wg), dim3(kWG), sa, st, b);
    else hipLaunchKernelGGL(k_assemble<double>, dim3(b.total_wg), dim3(kWG), sa, st, b);
  }
  mark(1);
  if (b.max_pstride > 0) {
    if (mixed) hipLaunchKernelGGL(k_reduce<float>, red_grid, dim3(256), 0, st, b);
    else hipLaunchKernelGGL(k_reduce<double>, red_grid, dim3(256), 0, st, b);
  }
  mark(2);
  hipLaunchKernelGGL(k_solve, dim3(b.n_act), dim3(kSolveThreads), s_solve, st, b);
  mark(3);
  if (b.total_wg > 0) {
    if (mixed) hipLaunchKernelGGL(k_backsub<float>, dim3(b.total_wg), dim3(kWG), sb, st, b);
    else hipLaunchKernelGGL(k_backsub<double>, dim3(b.total_wg), dim3(kWG), sb, st, b);
  }
  mark(4);
  hipLaunchKernelGGL(k_lm, dim3(b.n_act), dim3(64), 0, st, b);
  mark(5);
  return hipGetLastError();
}

hipError_t launch_export(const Batch& b, int max_P, hipStream_t st) {
  if (b.n_act == 0) return hipSuccess;
  const int n = max_P > b.max_C ? max_P : (b.max_C > 0 ? b.max_C : 1);
  hipLaunchKernelGGL(k_export, dim3((n + 255) / 256, b.n_act), dim3(256), 0, st, b);
  return hipGetLastError();
}

}  // namespace bagpu
