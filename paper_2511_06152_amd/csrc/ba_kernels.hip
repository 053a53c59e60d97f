// HIP kernels (gfx950) of the cluster bundle-adjustment library.
//
// One Levenberg-Marquardt iteration over a batch of resident clusters is six
// launches in the mixed path (seven in the plain FP64 path), each covering
// every cluster of the batch:
//
//   k_point<Real>     one lane per point, over its observations: residual of
//                     Eq. (5) with k1/k2 radial terms, Huber IRLS weight
//                     (robust rho of Eq. 6/7), point Jacobian; V_j, g_j in
//                     registers and the damped inverse
//   k_blocks<float>   one wavefront per task: a free camera's diagonal Schur
//   (k_camblk<double>, block (U_kk - sum W Q W^T, gradient, intrinsic border)
//    k_pairblk<double>) over its observations, or one camera-pair block
//                     (- sum W_a Q W_b^T) over the observation pairs of that
//                     pair of cameras; register sums, fixed-order reductions
//   k_reduce<Real>    per target block: fixed-order sum of its task partials
//                     into the reduced camera system (16x16 blocks), in FP64
//   k_solve           one workgroup per cluster: pose priors, Marquardt
//                     damping, FP64 Cholesky of the reduced camera system in
//                     16x16 blocks (matrix-core panel and trailing updates),
//                     triangular solves (+ one FP64 refinement step in mixed
//                     mode), trial camera poses and prior cost
//   k_pcg             (large systems instead of k_solve) block-Jacobi
//                     preconditioned conjugate gradients on the block-sparse
//                     reduced system
//   k_backsub<Real>   per point back-substitution, trial points, and the FP64
//                     trial cost of every observation
//   k_lm              gain ratio, accept/reject, Nielsen damping update,
//                     termination; flips the state buffers on acceptance
//
// No accumulation uses atomics, so every sum runs in a fixed order and a
// cluster's result is the same alone or inside any batch.  Real is double
// (plain path) or float (mixed path: FP32 residuals, Jacobians and Schur
// accumulation; FP64 reduction, solve, cost and gain ratio).
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_ext.h>
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

// Logical workgroup index of this workgroup.  Workgroups are dispatched to the
// eight XCDs round-robin (physical block b runs on XCD b % 8); the mapping
// gives each XCD one contiguous eighth of the logical range, so the clusters
// of a batch (contiguous in logical order) stay within one XCD's L2.
__device__ __forceinline__ int xcd_block() {
  const int b = blockIdx.x, G = gridDim.x;
  const int q = G >> 3, r = G & 7, x = b & 7, slot = b >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + slot;
}

// Packed storage of a symmetric matrix: element (r, c), r <= c.
__device__ __forceinline__ int pidx(int r, int c) { return c * (c + 1) / 2 + r; }

// The dense reduced system in 16x16 FP64 blocks (the layout the reduction
// writes and the dense solve loads, row stride 17): block (I, J), I >= J, of
// the lower block triangle at tblk(I, J); diagonal blocks hold both triangles.
constexpr int kTbS = kSolveTb + 1;              // row stride of a block (doubles)
constexpr int kTbV = kSolveTb * kTbS;           // doubles per block
__device__ __forceinline__ int tblk(int I, int J) { return (I * (I + 1) / 2 + J) * kTbV; }   // I >= J

// Stores element (p, q) = (q, p) of the symmetric system into its blocked
// place(s).
__device__ __forceinline__ void sput(double* Sb, int p, int q, double t) {
  const int P = p / kSolveTb, Q = q / kSolveTb;
  if (P >= Q) Sb[tblk(P, Q) + (p % kSolveTb) * kTbS + q % kSolveTb] = t;
  if (Q >= P) Sb[tblk(Q, P) + (q % kSolveTb) * kTbS + p % kSolveTb] = t;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T> __device__ __forceinline__ T clampd(T d) {
  return d < T(kDiagMin) ? T(kDiagMin) : (d > T(kDiagMax) ? T(kDiagMax) : d);
}

// Explicit fused multiply-add (the build does not contract a * b + c by itself)
// and the depth reciprocal: the hardware reciprocal (1 ulp) in FP32, exact in FP64.
__device__ __forceinline__ float fm(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fm(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float rcp(float z) { return __builtin_amdgcn_rcpf(z); }
__device__ __forceinline__ double rcp(double z) { return 1.0 / z; }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

// Per-point record (kPtVals Real): vector loads/stores of its first n values.
__device__ __forceinline__ void pt_load(const float* __restrict__ p, float* v, int n) {
  for (int i = 0; i < n; i += 4) {
    const float4 t = *reinterpret_cast<const float4*>(p + i);
    v[i] = t.x; v[i + 1] = t.y; v[i + 2] = t.z; v[i + 3] = t.w;
  }
}
__device__ __forceinline__ void pt_load(const double* __restrict__ p, double* v, int n) {
  for (int i = 0; i < n; i += 2) {
    const double2 t = *reinterpret_cast<const double2*>(p + i);
    v[i] = t.x; v[i + 1] = t.y;
  }
}
template <int N>
__device__ __forceinline__ void pt_store(float* p, const float* v) {
#pragma unroll
  for (int i = 0; i < N; i += 4) *reinterpret_cast<float4*>(p + i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
}
template <int N>
__device__ __forceinline__ void pt_store(double* p, const double* v) {
#pragma unroll
  for (int i = 0; i < N; i += 2) *reinterpret_cast<double2*>(p + i) = make_double2(v[i], v[i + 1]);
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

// Global-memory view of a device pointer.  Loads and stores through it are
// global rather than generic (flat) operations: they count on the vector
// memory counter only, so the waits for LDS and scalar loads in the chunk
// loops do not also wait for them.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> gmem(T* p) { return (gptr<T>)p; }

// First N values of a per-point record, as vector loads.
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));
template <int N>
__device__ __forceinline__ void rec_load(gptr<const float> p, float* v) {
#pragma unroll
  for (int i = 0; i < N; i += 4) {
    const vf4 t = *reinterpret_cast<gptr<const vf4>>(p + i);
    v[i] = t.x; v[i + 1] = t.y; v[i + 2] = t.z; v[i + 3] = t.w;
  }
}
template <int N>
__device__ __forceinline__ void rec_load(gptr<const double> p, double* v) {
#pragma unroll
  for (int i = 0; i < N; i += 2) {
    const vd2 t = *reinterpret_cast<gptr<const vd2>>(p + i);
    v[i] = t.x; v[i + 1] = t.y;
  }
}

template <int N>
__device__ __forceinline__ void rec_store(gptr<float> p, const float* v) {
#pragma unroll
  for (int i = 0; i < N; i += 4) *reinterpret_cast<gptr<vf4>>(p + i) = vf4{v[i], v[i + 1], v[i + 2], v[i + 3]};
}
template <int N>
__device__ __forceinline__ void rec_store(gptr<double> p, const double* v) {
#pragma unroll
  for (int i = 0; i < N; i += 2) *reinterpret_cast<gptr<vd2>>(p + i) = vd2{v[i], v[i + 1]};
}

// FP32 or FP64 views of the point state and the observed pixels.
template <typename R> __device__ __forceinline__ gptr<const R> pts_of(const SlotDesc& d, int cur);
template <> __device__ __forceinline__ gptr<const float> pts_of<float>(const SlotDesc& d, int cur) { return gmem((const float*)d.X32[cur]); }
template <> __device__ __forceinline__ gptr<const double> pts_of<double>(const SlotDesc& d, int cur) { return gmem((const double*)d.X[cur]); }
template <typename R> __device__ __forceinline__ gptr<const R> uv_of(const double* p64, const float* p32);
template <> __device__ __forceinline__ gptr<const float> uv_of<float>(const double*, const float* p32) { return gmem(p32); }
template <> __device__ __forceinline__ gptr<const double> uv_of<double>(const double* p64, const float*) { return gmem(p64); }

// A wave-uniform value marked as such, so that it is kept in scalar registers.
__device__ __forceinline__ float uniform(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uniform(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ---- SO(3) (FP64) -----------------------------------------------------------

// Rotations below kSo3Series rad take the Taylor series of the SO(3) maps
// (truncation below 1e-24 relative there, far under FP64 rounding), which
// skips the transcendental functions on the common path: LM steps and prior
// residuals are small rotations.
constexpr double kSo3Series = 0.02;

__device__ __forceinline__ void so3_exp(const double w[3], double R[9]) {
  const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  double a, b;
  if (th2 < kSo3Series * kSo3Series) {
    // a = sin(t)/t, b = (1 - cos t)/t^2
    a = 1.0 + th2 * (-1.0 / 6.0 + th2 * (1.0 / 120.0 + th2 * (-1.0 / 5040.0 + th2 * (1.0 / 362880.0))));
    b = 0.5 + th2 * (-1.0 / 24.0 + th2 * (1.0 / 720.0 + th2 * (-1.0 / 40320.0 + th2 * (1.0 / 3628800.0))));
  } else {
    const double th = sqrt(th2);
    a = sin(th) / th;
    b = (1.0 - cos(th)) / th2;
  }
  const double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  #pragma unroll
  for (int i = 0; i < 3; ++i)
    #pragma unroll
    for (int j = 0; j < 3; ++j) {
      double k2 = 0;
      #pragma unroll
      for (int l = 0; l < 3; ++l) k2 += K[3 * i + l] * K[3 * l + j];
      R[3 * i + j] = (i == j ? 1.0 : 0.0) + a * K[3 * i + j] + b * k2;
    }
}

__device__ __forceinline__ void so3_log(const double R[9], double w[3]) {
  double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
  c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
  const double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
  // v = 2 sin(t) axis: for a small angle, w = (t / (2 sin t)) v with
  // t / sin t = asin(n) / n, n = sin t, in series
  const double n2 = 0.25 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  if (c > 0.0 && n2 < kSo3Series * kSo3Series) {
    const double r = 1.0 + n2 * (1.0 / 6.0 + n2 * (3.0 / 40.0 + n2 * (5.0 / 112.0 + n2 * (35.0 / 1152.0))));
    #pragma unroll
    for (int i = 0; i < 3; ++i) w[i] = 0.5 * r * v[i];
    return;
  }
  const double th = acos(c);
  if (th < 1e-6) {
    const double s = 0.5 * (1.0 + th * th / 6.0);
    #pragma unroll
    for (int i = 0; i < 3; ++i) w[i] = s * v[i];
  } else if (th < M_PI - 1e-6) {
    const double s = th / (2.0 * sin(th));
    #pragma unroll
    for (int i = 0; i < 3; ++i) w[i] = s * v[i];
  } else {
    // Near pi: the axis from the largest diagonal entry of (R + I) / 2 = a a^T.
    const int k = (R[4] > R[0]) ? ((R[8] > R[4]) ? 2 : 1) : ((R[8] > R[0]) ? 2 : 0);
    const double Rkk = k == 0 ? R[0] : (k == 1 ? R[4] : R[8]);
    const double dd = sqrt(0.5 * (Rkk + 1.0));
    double a[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double rik = k == 0 ? R[3 * i] : (k == 1 ? R[3 * i + 1] : R[3 * i + 2]);
      const double rki = k == 0 ? R[i] : (k == 1 ? R[3 + i] : R[6 + i]);
      a[i] = (i == k) ? dd : 0.25 * (rik + rki) / dd;
    }
    const double n = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const double sg = (a[0] * v[0] + a[1] * v[1] + a[2] * v[2]) < 0 ? -1.0 : 1.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) w[i] = sg * th * a[i] / n;
  }
}

// Whitened prior residual e[6] of camera state cam (R, T) and its Jacobian
// block d e_omega / d domega = diag(1/sigma_omega) Jr^-1(phi) (3x3).
__device__ __forceinline__ void prior_terms(const double* __restrict__ cam, const double* __restrict__ pr,
                                            double e[6], double J[9]) {
  double M[9];   // R_prior^T R
  #pragma unroll
  for (int i = 0; i < 3; ++i)
    #pragma unroll
    for (int j = 0; j < 3; ++j)
      M[3 * i + j] = pr[i] * cam[j] + pr[3 + i] * cam[3 + j] + pr[6 + i] * cam[6 + j];
  double phi[3];
  so3_log(M, phi);
  const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  // cc = 1/t^2 - (1 + cos t) / (2 t sin t) = 1/12 + t^2/720 + t^4/30240 + t^6/1209600 + ...
  double cc;
  if (th2 < kSo3Series * kSo3Series) {
    cc = 1.0 / 12.0 + th2 * (1.0 / 720.0 + th2 * (1.0 / 30240.0 + th2 * (1.0 / 1209600.0)));
  } else {
    const double th = sqrt(th2);
    cc = 1.0 / th2 - (1.0 + cos(th)) / (2.0 * th * sin(th));
  }
  const double K[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
  #pragma unroll
  for (int i = 0; i < 3; ++i) {
    e[i] = phi[i] * pr[12 + i];
    e[3 + i] = (cam[9 + i] - pr[9 + i]) * pr[15 + i];
    #pragma unroll
    for (int j = 0; j < 3; ++j) {
      double k2 = 0;
      #pragma unroll
      for (int l = 0; l < 3; ++l) k2 += K[3 * i + l] * K[3 * l + j];
      J[3 * i + j] = ((i == j ? 1.0 : 0.0) + 0.5 * K[3 * i + j] + cc * k2) * pr[12 + i];
    }
  }
}

// Cached prior terms of one camera (e, J of prior_terms), kept per state
// buffer: written when a state's cameras are formed (admission, trial
// cameras), read by the solve of the iteration that starts from that state.
__device__ __forceinline__ void pterm_store(double* __restrict__ p, const double e[6], const double J[9]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = e[i];
#pragma unroll
  for (int i = 0; i < 9; ++i) p[6 + i] = J[i];
}
__device__ __forceinline__ void pterm_load(const double* __restrict__ p, double e[6], double J[9]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) e[i] = p[i];
#pragma unroll
  for (int i = 0; i < 9; ++i) J[i] = p[6 + i];
}

// ---- per-observation model ------------------------------------------------------

template <typename R, int NK = 2>
struct ObsJ {
  R xc[3];
  R e[2];       // whitened residual
  R w;          // IRLS weight rho'(s)
  R Jp[2][3];   // whitened d(u,v)/dX
  R Jw[2][3];   // whitened d(u,v)/d omega
  R Jk[2][NK];  // whitened d(u,v)/d(k1, k2[, f, cx, cy])
};

// Intrinsic Jacobian columns an observation carries: k1, k2, and with
// self-calibration also f, cx, cy (column t is always intrinsic t).
template <bool SC>
constexpr int kNk = SC ? kIntr : 2;

// Residual, Huber weight and Jacobians of one observation.  cam = R (9,
// row-major, camera->world), T (3).  Invalid lanes get w = 0 and finite values.
// SC (self-calibration): the prediction adds the principal point's offset
// (cxo, cyo), and the Jacobian has the columns of all five intrinsics (k1,
// k2, f, cx, cy) instead of k1, k2 only.
template <typename R, bool SC = false>
__device__ __forceinline__ void obs_model(const R* __restrict__ cam, const R X0, const R X1, const R X2, const R u,
                                          const R v, const R f, const R k1, const R k2, const R is, const R dt,
                                          bool valid, ObsJ<R, kNk<SC>>& o, const R cxo = R(0), const R cyo = R(0)) {
  const R d0 = X0 - cam[9], d1 = X1 - cam[10], d2 = X2 - cam[11];
  R x = fm(cam[6], d2, fm(cam[3], d1, cam[0] * d0));
  R y = fm(cam[7], d2, fm(cam[4], d1, cam[1] * d0));
  R z = fm(cam[8], d2, fm(cam[5], d1, cam[2] * d0));
  if (!valid || !(z > R(0))) { x = R(0); y = R(0); z = R(1); valid = false; }
  o.xc[0] = x; o.xc[1] = y; o.xc[2] = z;
  const R iz = rcp(z);
  const R a = x * iz, b = y * iz;
  const R r2 = fm(a, a, b * b);
  const R D = fm(r2, fm(k2, r2, k1), R(1));     // 1 + k1 r^2 + k2 r^4
  const R fD = f * D;
  const R fis = f * is;
  if constexpr (SC) {
    o.e[0] = fm(fD, a, cxo - u) * is;
    o.e[1] = fm(fD, b, cyo - v) * is;
  } else {
    o.e[0] = fm(fD, a, -u) * is;
    o.e[1] = fm(fD, b, -v) * is;
  }
  const R s = fm(o.e[0], o.e[0], o.e[1] * o.e[1]);
  o.w = valid ? (s <= dt * dt ? R(1) : dt * rsq(s)) : R(0);
  const R q2 = R(2) * fm(R(2) * k2, r2, k1);     // 2 (k1 + 2 k2 r^2)
  const R A00 = fis * fm(q2 * a, a, D), A01 = fis * (q2 * a * b), A11 = fis * fm(q2 * b, b, D);
  const R Jx[2][3] = {{A00 * iz, A01 * iz, -fm(A00, a, A01 * b) * iz},
                      {A01 * iz, A11 * iz, -fm(A01, a, A11 * b) * iz}};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) o.Jp[i][j] = fm(Jx[i][2], cam[3 * j + 2], fm(Jx[i][1], cam[3 * j + 1], Jx[i][0] * cam[3 * j]));
    o.Jw[i][0] = fm(Jx[i][1], z, -(Jx[i][2] * y));
    o.Jw[i][1] = fm(Jx[i][2], x, -(Jx[i][0] * z));
    o.Jw[i][2] = fm(Jx[i][0], y, -(Jx[i][1] * x));
  }
  const R fr2 = fis * r2, fr4 = fr2 * r2;
  if constexpr (SC) {
    // whitened d(u, v)/d(k1, k2, f, cx, cy): f r^2 (a, b), f r^4 (a, b), D (a, b), (1, 0), (0, 1)
    const R Da = is * D * a, Db = is * D * b;
    o.Jk[0][0] = fr2 * a; o.Jk[0][1] = fr4 * a; o.Jk[0][2] = Da; o.Jk[0][3] = is;   o.Jk[0][4] = R(0);
    o.Jk[1][0] = fr2 * b; o.Jk[1][1] = fr4 * b; o.Jk[1][2] = Db; o.Jk[1][3] = R(0); o.Jk[1][4] = is;
  } else {
    o.Jk[0][0] = fr2 * a; o.Jk[0][1] = fr4 * a;
    o.Jk[1][0] = fr2 * b; o.Jk[1][1] = fr4 * b;
  }
}

// Camera-side whitened Jacobian column r (0..5) of row i: [Jw | -Jp].
template <typename R, int NK>
__device__ __forceinline__ R jc(const ObsJ<R, NK>& o, int i, int r) { return r < 3 ? o.Jw[i][r] : -o.Jp[i][r - 3]; }

// Huber rho of the squared whitened norm s, dt = delta / sigma.
__device__ __forceinline__ double huber_rho(double s, double dt) {
  return s <= dt * dt ? s : 2.0 * dt * sqrt(s) - dt * dt;
}

// FP64 residual rho(s) of one observation; returns false at non-positive depth.
// ki: the intrinsic state (k1, k2, f, principal-point offset x, y).
__device__ __forceinline__ bool obs_rho(const double* __restrict__ cam, const double X[3], double u, double v,
                                        const double* ki, double is, double dt, double* rho) {
  const double k1 = ki[0], k2 = ki[1], f = ki[2];
  const double d0 = X[0] - cam[9], d1 = X[1] - cam[10], d2 = X[2] - cam[11];
  const double x = cam[0] * d0 + cam[3] * d1 + cam[6] * d2;
  const double y = cam[1] * d0 + cam[4] * d1 + cam[7] * d2;
  const double z = cam[2] * d0 + cam[5] * d1 + cam[8] * d2;
  if (!(z > 0.0)) { *rho = 0.0; return false; }
  const double iz = 1.0 / z;
  const double a = x * iz, b = y * iz;
  const double r2 = a * a + b * b;
  const double D = 1.0 + k1 * r2 + k2 * r2 * r2;
  const double e0 = (f * D * a + ki[3] - u) * is, e1 = (f * D * b + ki[4] - v) * is;
  *rho = huber_rho(e0 * e0 + e1 * e1, dt);
  return true;
}

// Inverse of the 3x3 SPD matrix (a00 a01 a02 a11 a12 a22) via Cholesky.
template <typename R>
__device__ __forceinline__ bool spd3_inv(const R A[6], R Q[6]) {
  if (!(A[0] > R(0))) return false;
  const R i00 = rsq(A[0]);
  const R l10 = A[1] * i00, l20 = A[2] * i00;
  const R l11s = A[3] - l10 * l10;
  if (!(l11s > R(0))) return false;
  const R i11 = rsq(l11s);
  const R l21 = (A[4] - l20 * l10) * i11;
  const R l22s = A[5] - l20 * l20 - l21 * l21;
  if (!(l22s > R(0))) return false;
  const R i22 = rsq(l22s);
  const R i10 = -l10 * i00 * i11;
  const R i21 = -l21 * i11 * i22;
  const R i20 = -fm(l20, i00, l21 * i10) * i22;
  Q[0] = fm(i00, i00, fm(i10, i10, i20 * i20));
  Q[1] = fm(i10, i11, i20 * i21);
  Q[2] = i20 * i22;
  Q[3] = fm(i11, i11, i21 * i21);
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
    c.cg_iters = 0;
    c.cg_b0 = 0.0;
    for (int t = 0; t < 5; ++t) c.k[1][t] = c.k[0][t];
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

// Initial values of cameras and points known to the resident store, before
// the origin shift (world frame, over the caller's values).
__global__ void k_res_gather(Batch bt) {
  const int s = bt.act[blockIdx.y];
  const SlotDesc& d = bt.desc[s];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.n_rin_cam) {
    const int2 e = d.rin_cam[i];
    double* r = d.raw_cam + 30 * (size_t)e.x;
    const double* src = d.res_cam + 12 * (size_t)e.y;
    for (int t = 0; t < 12; ++t) r[t] = src[t];
  }
  if (i < d.n_rin_pt) {
    const int2 e = d.rin_pt[i];
    for (int t = 0; t < 3; ++t) d.X[0][3 * (size_t)e.x + t] = d.res_pt[3 * (size_t)e.y + t];
  }
}

// Final state (export staging, world frame) into the resident store.  A camera
// flagged for fusion whose row holds an earlier cluster's pose (weight > 0)
// gets the match-count weighted mean of Eq. (8): T linearly, R along the
// geodesic from the stored rotation; the row's weight accumulates.
__global__ void k_res_scatter(Batch bt) {
  const int s = bt.act[blockIdx.y];
  const SlotDesc& d = bt.desc[s];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.n_rout_cam) {
    const int4 e = d.rout_cam[i];
    double* dst = d.res_cam + 12 * (size_t)e.y;
    double Rn[9], Tn[3];
    for (int t = 0; t < 9; ++t) Rn[t] = d.out[9 * (size_t)e.x + t];
    for (int t = 0; t < 3; ++t) Tn[t] = d.out[9 * (size_t)d.C + 3 * (size_t)e.x + t];
    const double wn = (double)e.z, wo = d.res_cam_w[e.y];
    if (e.w && wo > 0.0) {
      const double a = wn / (wo + wn);
      double Ro[9], M[9];
      for (int t = 0; t < 9; ++t) Ro[t] = dst[t];
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) M[3 * r + q] = Ro[r] * Rn[q] + Ro[3 + r] * Rn[3 + q] + Ro[6 + r] * Rn[6 + q];
      double phi[3], E[9];
      so3_log(M, phi);
      for (int t = 0; t < 3; ++t) phi[t] *= a;
      so3_exp(phi, E);
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) dst[3 * r + q] = Ro[3 * r] * E[q] + Ro[3 * r + 1] * E[3 + q] + Ro[3 * r + 2] * E[6 + q];
      for (int t = 0; t < 3; ++t) dst[9 + t] = (wo * dst[9 + t] + wn * Tn[t]) / (wo + wn);
      d.res_cam_w[e.y] = wo + wn;
    } else {
      for (int t = 0; t < 9; ++t) dst[t] = Rn[t];
      for (int t = 0; t < 3; ++t) dst[9 + t] = Tn[t];
      d.res_cam_w[e.y] = wn;
    }
  }
  if (i < d.n_rout_pt) {
    const int2 e = d.rout_pt[i];
    for (int t = 0; t < 3; ++t) d.res_pt[3 * (size_t)e.y + t] = d.out[12 * (size_t)d.C + 3 * (size_t)e.x + t];
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
    const double u = d.ob_uv64[2 * i] - d.cx, v = d.ob_uv64[2 * i + 1] - d.cy;
    d.ob_uv64[2 * i] = u;
    d.ob_uv64[2 * i + 1] = v;
    d.ob_uv32[2 * i] = (float)u;
    d.ob_uv32[2 * i + 1] = (float)v;
  }
}

// ---- FP64 cost of the current state (admission) -----------------------------------

__global__ __launch_bounds__(kWG) void k_cost0(Batch bt) {
  const int bx = xcd_block();
  extern __shared__ double sh_cam[];
  if (bt.n_act == 0) return;   // empty dispatch that only carries timing events
  const int si = find_slot(bt.wg_off, bt.n_act, bx);
  const int s = bt.act[si];
  const int wgl = bx - bt.wg_off[si];
  const SlotDesc& d = bt.desc[s];
  const SlotCtl& c = bt.ctl[s];
  const int cur = c.cur;
  for (int i = threadIdx.x; i < d.C * kCamVals; i += kWG) sh_cam[i] = d.cam[cur][i];
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const double* ki = c.k[cur];
  double acc = 0.0;
  int bad = 0;
  // one lane per point of a chunk, over its observations
  for (int ch = d.wg_chunk[wgl] + wave; ch < d.wg_chunk[wgl + 1]; ch += kWavesPerWG) {
    const int4 pc = d.pchunk[ch];
    if (lane >= pc.w) continue;
    const int pt = pc.z + lane;
    const double X[3] = {d.X[cur][3 * pt], d.X[cur][3 * pt + 1], d.X[cur][3 * pt + 2]};
    for (int t = 0; t < pc.y; ++t) {
      const int idx = pc.x + t * kWave + lane;
      double rho;
      if (obs_rho(sh_cam + kCamVals * d.ob_cam[idx], X, d.ob_uv64[2 * idx], d.ob_uv64[2 * idx + 1], ki, d.inv_sigma,
                  d.huber_dt, &rho)) acc += rho;
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
  // one wavefront: strided lane sums in order, then a fixed xor tree
  double rho = 0.0, pr = 0.0;
  int bad = 0;
  for (int w = threadIdx.x; w < d.n_wg; w += kWave) {
    rho += d.cost_part[2 * w];
    bad += d.bad_part[w];
  }
  for (int k = threadIdx.x; k < d.C; k += kWave) {
    if (d.cam_col[k] < 0) continue;
    double e[6], J[9];
    prior_terms(d.cam[c.cur] + kCamVals * k, d.prior + kPriorVals * k, e, J);
    pterm_store(d.pterm[c.cur] + kPtermVals * k, e, J);
    #pragma unroll
    for (int i = 0; i < 6; ++i) pr += e[i] * e[i];
  }
  rho = wave_sum(rho);
  pr = wave_sum(pr);
  bad = wave_sum(bad);
  if (threadIdx.x != 0) return;
  const double E = 0.5 * rho + 0.5 * pr;
  c.E = E;
  c.E0 = E;
  d.cost_log[0] = E;
  if (bad > 0 || !isfinite(E)) { c.status = ST_BAD_INIT; c.bad_init = bad > 0 ? bad : 1; }
  else if (d.max_iters <= 0) c.status = ST_MAXITER;
}

// ---- point pass: damped point blocks --------------------------------------------
//
// One lane per point: the 64 points of a chunk have the same observation
// count n, and the lane walks its point's observations in camera order (one
// 64-lane row of the chunk's observation-major lanes each), so that the sums
// V_j, g_j, Z_j stay in registers.  Writes, per point, Q = (V + lambda
// D_V)^-1, g_p, D_V and Z = sum of the intrinsic rows of W; per wavefront,
// the intrinsic-intrinsic sums (U part of all observations, Schur part of all
// points).

template <typename R, bool INTR, bool SC>
__device__ __forceinline__ void point_pass(const SlotDesc& d, SlotCtl& c, const R* scam, int wgl, int wave,
                                           int lane) {
  constexpr int NK = kNk<SC>, NS = NK * (NK + 1) / 2, NI = NS + 3 * NK;
  constexpr int NV = INTR ? 9 + 3 * NK : 9;
  const int cur = c.cur;
  const R lam = (R)c.lambda;
  // f is the state's (it equals d.f unless self-calibrating); the principal
  // point's offset and the intrinsic types matter only when self-calibrating
  const R f = SC ? (R)c.k[cur][2] : (R)d.f, is = (R)d.inv_sigma, dt = (R)d.huber_dt;
  const R k1 = (R)c.k[cur][0], k2 = (R)c.k[cur][1];
  const R cxo = SC ? (R)c.k[cur][3] : R(0), cyo = SC ? (R)c.k[cur][4] : R(0);
  const gptr<R> ptv = gmem(reinterpret_cast<R*>(d.ptv)), ptd = gmem(reinterpret_cast<R*>(d.ptd));
  const gptr<const int> ocam = gmem(d.ob_cam);
  const gptr<const R> Xs = pts_of<R>(d, cur), uvs = uv_of<R>(d.ob_uv64, d.ob_uv32);
  // intrinsic sums: S (packed upper triangle, NS), g (NK), diag U (NK), Schur part of b (NK)
  R iv[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) iv[i] = R(0);
  bool fail = false;
  const int c0 = d.wg_chunk[wgl], c1 = d.wg_chunk[wgl + 1];
  for (int ch = c0 + wave; ch < c1; ch += kWavesPerWG) {
    const int4 pc = d.pchunk[ch];
    const int n = pc.y;
    // padding lanes read the chunk's first point and the padding lanes'
    // camera 0 and pixel 0, then zero what they read
    const bool valid = lane < pc.w;
    const int pt = pc.z + (valid ? lane : 0);
    const R X0r = Xs[3 * pt], X1r = Xs[3 * pt + 1], X2r = Xs[3 * pt + 2];
    const R X0 = valid ? X0r : R(0), X1 = valid ? X1r : R(0), X2 = valid ? X2r : R(0);
    // the next observation's camera and pixel are requested one ahead
    int idx = pc.x + lane;
    int cam_n = ocam[idx];
    R u_n = uvs[2 * idx], v_n = uvs[2 * idx + 1];
    R sum[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) sum[i] = R(0);
    for (int t = 0; t < n; ++t) {
      const int cam = cam_n;
      const R u = valid ? u_n : R(0), v = valid ? v_n : R(0);
      if (t + 1 < n) {
        idx += kWave;
        cam_n = ocam[idx];
        u_n = uvs[2 * idx];
        v_n = uvs[2 * idx + 1];
      }
      ObsJ<R, NK> o;
      obs_model<R, SC>(scam + kCamVals * cam, X0, X1, X2, u, v, f, k1, k2, is, dt, valid, o, cxo, cyo);
      const R w = o.w;
      R wJp[2][3];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 3; ++q) wJp[i][q] = w * o.Jp[i][q];
      R vals[NV];
      vals[0] = fm(o.Jp[0][0], wJp[0][0], o.Jp[1][0] * wJp[1][0]);
      vals[1] = fm(o.Jp[0][0], wJp[0][1], o.Jp[1][0] * wJp[1][1]);
      vals[2] = fm(o.Jp[0][0], wJp[0][2], o.Jp[1][0] * wJp[1][2]);
      vals[3] = fm(o.Jp[0][1], wJp[0][1], o.Jp[1][1] * wJp[1][1]);
      vals[4] = fm(o.Jp[0][1], wJp[0][2], o.Jp[1][1] * wJp[1][2]);
      vals[5] = fm(o.Jp[0][2], wJp[0][2], o.Jp[1][2] * wJp[1][2]);
#pragma unroll
      for (int q = 0; q < 3; ++q) vals[6 + q] = fm(wJp[0][q], o.e[0], wJp[1][q] * o.e[1]);
      if constexpr (INTR) {
#pragma unroll
        for (int b = 0; b < NK; ++b)
#pragma unroll
          for (int q = 0; q < 3; ++q) vals[9 + 3 * b + q] = fm(o.Jk[0][b], wJp[0][q], o.Jk[1][b] * wJp[1][q]);
      }
      // the point's sums, in camera order
#pragma unroll
      for (int i = 0; i < NV; ++i) sum[i] += vals[i];
      if constexpr (INTR) {
        int e = 0;
#pragma unroll
        for (int a = 0; a < NK; ++a) {
          const R uaa = w * fm(o.Jk[0][a], o.Jk[0][a], o.Jk[1][a] * o.Jk[1][a]);
          iv[e++] += uaa;
#pragma unroll
          for (int b = a + 1; b < NK; ++b) iv[e++] += w * fm(o.Jk[0][a], o.Jk[0][b], o.Jk[1][a] * o.Jk[1][b]);
          iv[NS + a] += w * fm(o.Jk[0][a], o.e[0], o.Jk[1][a] * o.e[1]);
          iv[NS + NK + a] += uaa;
        }
      }
    }
    const R Dp[3] = {clampd(sum[0]), clampd(sum[3]), clampd(sum[5])};
    const R Vl[6] = {fm(lam, Dp[0], sum[0]), sum[1], sum[2], fm(lam, Dp[1], sum[3]), sum[4], fm(lam, Dp[2], sum[5])};
    R Q[6];
    if (!spd3_inv(Vl, Q)) {
      if (valid) fail = true;
#pragma unroll
      for (int i = 0; i < 6; ++i) Q[i] = R(0);
    }
    if (valid) {
      R rec[kPtVals];
#pragma unroll
      for (int i = 0; i < 6; ++i) rec[i] = Q[i];
#pragma unroll
      for (int i = 0; i < 3; ++i) rec[6 + i] = sum[6 + i];
#pragma unroll
      for (int i = 0; i < 6; ++i) rec[9 + i] = INTR ? sum[(9 + i) % NV] : R(0);
      rec[15] = R(0);
      rec_store<kPtVals>(ptv + kPtVals * (size_t)pt, rec);
      if constexpr (SC) {
        R rz[kPtzVals];
#pragma unroll
        for (int i = 0; i < kPtzVals; ++i) rz[i] = i < 9 ? sum[(15 + i) % NV] : R(0);
        rec_store<kPtzVals>(gmem(reinterpret_cast<R*>(d.ptz)) + kPtzVals * (size_t)pt, rz);
      }
      const R dr[4] = {Dp[0], Dp[1], Dp[2], R(0)};
      rec_store<4>(ptd + 4 * (size_t)pt, dr);
      if constexpr (INTR) {
        R Z[NK][3], ZQ[NK][3];
#pragma unroll
        for (int b = 0; b < NK; ++b)
#pragma unroll
          for (int q = 0; q < 3; ++q) Z[b][q] = sum[(9 + 3 * b + q) % NV];
#pragma unroll
        for (int b = 0; b < NK; ++b)
#pragma unroll
          for (int q = 0; q < 3; ++q) ZQ[b][q] = fm(Z[b][0], qel(Q, 0, q), fm(Z[b][1], qel(Q, 1, q), Z[b][2] * qel(Q, 2, q)));
        int e = 0;
#pragma unroll
        for (int a = 0; a < NK; ++a)
#pragma unroll
          for (int b = a; b < NK; ++b, ++e) iv[e] -= fm(ZQ[a][0], Z[b][0], fm(ZQ[a][1], Z[b][1], ZQ[a][2] * Z[b][2]));
#pragma unroll
        for (int a = 0; a < NK; ++a) iv[NS + 2 * NK + a] += fm(ZQ[a][0], sum[6], fm(ZQ[a][1], sum[7], ZQ[a][2] * sum[8]));
      }
    }
  }
  if (fail) atomicOr(&c.point_fail, 1);
  if constexpr (INTR) {
    R* pp = reinterpret_cast<R*>(d.pt_part) + (size_t)(wgl * kWavesPerWG + wave) * kPtPartVals;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const R t = wave_sum(iv[i]);
      if (lane == 0) pp[i] = t;
    }
  }
}

// The point pass over every cluster of the batch.  SC: the launch for
// self-calibrating clusters (f, cx or cy estimated); each instantiation skips
// the other kind, so that the common one keeps its register allocation.
template <typename R, bool SC>
__global__ __launch_bounds__(kWG) void k_point(Batch bt) {
  const int bx = xcd_block();
  extern __shared__ __align__(16) unsigned char smem[];
  if (bt.n_act == 0) return;   // empty dispatch that only carries timing events
  const int si = __builtin_amdgcn_readfirstlane(find_slot(bt.wg_off, bt.n_act, bx));
  const int s = __builtin_amdgcn_readfirstlane(bt.act[si]);
  const int wgl = bx - bt.wg_off[si];
  const SlotDesc& d = bt.desc[s];
  SlotCtl& c = bt.ctl[s];
  if (c.status != ST_RUNNING || (d.sc != 0) != SC) return;
  R* scam = reinterpret_cast<R*>(smem);
  const int cur = c.cur;
  for (int i = threadIdx.x; i < d.C * kCamVals; i += kWG) scam[i] = (R)d.cam[cur][i];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  if constexpr (SC) point_pass<R, true, true>(d, c, scam, wgl, wave, lane);
  else if ((d.kcol0 >= 0) || (d.kcol1 >= 0)) point_pass<R, true, false>(d, c, scam, wgl, wave, lane);
  else point_pass<R, false, false>(d, c, scam, wgl, wave, lane);
}

// ---- block passes: camera-diagonal and camera-pair blocks of the Schur complement ----
//
// One wavefront per task (k_camblk: camera tasks, k_pairblk: pair tasks; two
// kernels so that each gets the register allocation it needs).  A camera
// task sums, over a run of observations of one free camera, its diagonal
// block U_kk - sum Y W^T, g_k, sum Y g_p, diag U_kk and its intrinsic border;
// a pair task sums -Y_a W_b^T over a run of observation pairs (same point,
// cameras a < b).  W = w J_c^T J_p and Y = W Q (Q = V^-1 of the point) are
// never formed: each term is a 2x2 or 2-vector quantity of the observation
// pushed through the 2x6 camera Jacobian (see the kernels).  Sums stay in
// registers and are reduced across the wavefront in a fixed order: no
// atomics, so a cluster's result does not depend on what else is in the batch.

template <typename R>
__device__ __forceinline__ void load_cam(const double* __restrict__ src, R* dst) {
#pragma unroll
  for (int i = 0; i < kCamVals; ++i) dst[i] = uniform((R)src[i]);
}

// T = J_p Q (2 x 3) for the packed symmetric 3x3 Q.
template <typename R, int NK>
__device__ __forceinline__ void jp_q(const ObsJ<R, NK>& o, const R* Q, R T[2][3]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int t = 0; t < 3; ++t)
      T[a][t] = fm(o.Jp[a][2], qel(Q, 2, t), fm(o.Jp[a][1], qel(Q, 1, t), o.Jp[a][0] * qel(Q, 0, t)));
}

// Wavefront sums of N per-lane values written to out[0..N): N full-wave
// reductions for FP64; for FP32 a reduce-scatter in six halving stages, each
// pairing a lane with one that differs in one lane-index bit (bits 5 and 4 by
// the CDNA4 cross-half swaps, bits 3..0 by DPP moves inside a row).  At each
// stage the lower lane keeps the sum of the first half of its values, the
// upper lane of the second half, so ~N exchanges replace 6 N, and lane l ends
// up holding the whole-wave sum of one value, stored with one instruction.
// The summation tree is fixed, so the result depends on the inputs only.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <int N, int STAGE>
__device__ __forceinline__ void rs_stage(float* v, int lane) {
  constexpr int H = (N + 1) / 2;
  if constexpr (STAGE < 2) {
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const unsigned a = __float_as_uint(v[i]), b = i + H < N ? __float_as_uint(v[i + H]) : 0u;
      // swap a's upper 32 (16) lanes with b's lower 32 (16): each lane then
      // holds its own value of one half and its partner's of the same half
      const auto r = STAGE == 0 ? __builtin_amdgcn_permlane32_swap(a, b, false, false)
                                : __builtin_amdgcn_permlane16_swap(a, b, false, false);
      v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
  } else {
    const bool hi = (lane >> (5 - STAGE)) & 1;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const float a = v[i], b = i + H < N ? v[i + H] : 0.0f;
      const float keep = hi ? b : a, send = hi ? a : b;
      float got;
      if constexpr (STAGE == 2) got = dpp_mov<0x128>(send);        // row_ror:8: partner lane ^ 8
      else if constexpr (STAGE == 3) got = dpp_mov<0x141>(send);   // row_half_mirror: lane ^ 7
      else if constexpr (STAGE == 4) got = dpp_mov<0x4E>(send);    // quad_perm 2,3,0,1: lane ^ 2
      else got = dpp_mov<0xB1>(send);                              // quad_perm 1,0,3,2: lane ^ 1
      v[i] = keep + got;
    }
  }
  if constexpr (STAGE < 5) rs_stage<H, STAGE + 1>(v, lane);
}

// Index of the value lane `lane` holds after rs_stage<N, 0>, or -1 (padding).
template <int N>
__device__ __forceinline__ int rs_index(int lane) {
  int n[7] = {N};
#pragma unroll
  for (int s = 0; s < 6; ++s) n[s + 1] = (n[s] + 1) / 2;
  int l = 0;
  bool ok = true;
#pragma unroll
  for (int s = 5; s >= 0; --s) {
    l += ((lane >> (5 - s)) & 1) * n[s + 1];
    ok = ok && l < n[s];
  }
  return ok ? l : -1;
}

template <int N>
__device__ __forceinline__ void wave_store(double (&acc)[N], double* out, int lane) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double t = wave_sum(acc[i]);
    if (lane == 0) out[i] = t;
  }
}
template <int N>
__device__ __forceinline__ void wave_store(float (&acc)[N], float* out, int lane) {
  rs_stage<N, 0>(acc, lane);
  const int j = rs_index<N>(lane);
  if (j >= 0) out[j] = acc[0];
}

// Camera task t of a cluster (one wavefront).  INTR: at least one of k1, k2
// is estimated; both borders are then summed (the reduction writes only the
// estimated ones).  SC: the borders of all five intrinsics are summed (69
// values: the 51 of the k1/k2 layout, then f, cx, cy).
template <typename R, bool INTR, bool SC>
__device__ __forceinline__ void camblk_task_k(const SlotDesc& d, const SlotCtl& c, int t, int lane) {
  constexpr int NK = kNk<SC>, NA = 39 + 6 * NK;
  const int4 tk = d.tasks[t];
  const int ka = (tk.x >> 12) & 0xfff, kb = tk.x & 0xfff;
  const int cur = c.cur;
  // f is the state's (it equals d.f unless self-calibrating); the principal
  // point's offset and the intrinsic types matter only when self-calibrating
  const R f = SC ? (R)c.k[cur][2] : (R)d.f, is = (R)d.inv_sigma, dt = (R)d.huber_dt;
  const R k1 = (R)c.k[cur][0], k2 = (R)c.k[cur][1];
  const R cxo = SC ? (R)c.k[cur][3] : R(0), cyo = SC ? (R)c.k[cur][4] : R(0);
  const bool mixed = sizeof(R) == 4;
  const R* __restrict__ ptv = reinterpret_cast<const R*>(d.ptv);
  R* part = reinterpret_cast<R*>(d.task_part) + (size_t)t * kTaskVals;
  R ca[kCamVals];
  load_cam(d.cam[cur] + kCamVals * ka, ca);
  (void)kb;
  const gptr<const R> recz = gmem(reinterpret_cast<const R*>(d.ptz));

    const gptr<const int> cl_pt = gmem(d.cl_pt), cl_ob = gmem(d.cl_ob);
    const gptr<const R> Xs = pts_of<R>(d, cur), uvs = uv_of<R>(d.ob_uv64, d.ob_uv32), recs = gmem(ptv);
    R acc[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] = R(0);
    // Loads are unconditional: padding lanes read point 0 and observation
    // lane 0 (finite state, record and pixel) and the observation model
    // gives them weight 0, which zeroes every term they add.  The next
    // chunk's point and observation lane are requested a chunk ahead.
    const int ch_end = tk.y + tk.z;
    int pt_next = cl_pt[tk.y * kWave + lane], ob_next = cl_ob[tk.y * kWave + lane];
    for (int ch = tk.y; ch < ch_end; ++ch) {
      const int idx = ch * kWave + lane;
      const int pt = pt_next, ob = ob_next;
      if (ch + 1 < ch_end) {
        pt_next = cl_pt[idx + kWave];
        ob_next = cl_ob[idx + kWave];
      }
      const bool valid = pt >= 0;
      const int ps = valid ? pt : 0;
      const R X0 = Xs[3 * ps], X1 = Xs[3 * ps + 1], X2 = Xs[3 * ps + 2], u = uvs[2 * ob], v = uvs[2 * ob + 1];
      R rec[kPtVals];
      rec_load<kPtVals>(recs + kPtVals * (size_t)ps, rec);
      R rz[SC ? kPtzVals : 1];
      if constexpr (SC) rec_load<kPtzVals>(recz + kPtzVals * (size_t)ps, rz);
      ObsJ<R, NK> o;
      obs_model<R, SC>(ca, X0, X1, X2, u, v, f, k1, k2, is, dt, valid, o, cxo, cyo);
      const R* Q = rec;
      const R* gp = rec + 6;
      const R w = o.w;
      // With W = w J_c^T J_p and Y = W Q, every term of the observation goes
      // through 2-vectors: U - Y W^T = J_c^T M J_c with the 2x2
      // M = w I - w^2 J_p Q J_p^T; Y g_p = J_c^T (w T g_p); the intrinsic
      // border w J_c^T J_k - Y Z^T = J_c^T w (J_k - T Z^T), where T = J_p Q.
      R T[2][3];
      jp_q(o, Q, T);
      const R w2 = w * w;
      const R P00 = fm(T[0][2], o.Jp[0][2], fm(T[0][1], o.Jp[0][1], T[0][0] * o.Jp[0][0]));
      const R P01 = fm(T[0][2], o.Jp[1][2], fm(T[0][1], o.Jp[1][1], T[0][0] * o.Jp[1][0]));
      const R P11 = fm(T[1][2], o.Jp[1][2], fm(T[1][1], o.Jp[1][1], T[1][0] * o.Jp[1][0]));
      const R M00 = fm(-w2, P00, w), M01 = -w2 * P01, M11 = fm(-w2, P11, w);
      const R ve0 = w * o.e[0], ve1 = w * o.e[1];
      const R vg0 = w * fm(T[0][2], gp[2], fm(T[0][1], gp[1], T[0][0] * gp[0]));
      const R vg1 = w * fm(T[1][2], gp[2], fm(T[1][1], gp[1], T[1][0] * gp[0]));
      R vk[NK][2];   // [intrinsic][row]
#pragma unroll
      for (int q = 0; q < NK; ++q) {
        vk[q][0] = vk[q][1] = R(0);
        if (!INTR) continue;
        const R* z = q < 2 ? rec + 9 + 3 * q : rz + 3 * (q - 2);
#pragma unroll
        for (int a = 0; a < 2; ++a) vk[q][a] = w * (o.Jk[a][q] - fm(T[a][2], z[2], fm(T[a][1], z[1], T[a][0] * z[0])));
      }
      R a0[6], a1[6], G0[6], G1[6];   // J_c rows and M J_c
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        a0[r] = jc(o, 0, r);
        a1[r] = jc(o, 1, r);
        G0[r] = fm(M00, a0[r], M01 * a1[r]);
        G1[r] = fm(M01, a0[r], M11 * a1[r]);
      }
      int e = 0;
#pragma unroll
      for (int r = 0; r < 6; ++r) {
#pragma unroll
        for (int cc = r; cc < 6; ++cc, ++e) acc[e] = fm(a0[r], G0[cc], fm(a1[r], G1[cc], acc[e]));
        acc[21 + r] = fm(a0[r], ve0, fm(a1[r], ve1, acc[21 + r]));
        acc[27 + r] = fm(a0[r], vg0, fm(a1[r], vg1, acc[27 + r]));
        acc[33 + r] = fm(w * a0[r], a0[r], fm(w * a1[r], a1[r], acc[33 + r]));
        if (INTR) {
#pragma unroll
          for (int q = 0; q < NK; ++q)
            acc[39 + 6 * q + r] = fm(a0[r], vk[q][0], fm(a1[r], vk[q][1], acc[39 + 6 * q + r]));
        }
      }
    }
    if constexpr (SC) {
      // a wavefront reduce-scatter takes at most 64 values: two of them
      R lo[51], hi[NA - 51];
#pragma unroll
      for (int i = 0; i < 51; ++i) lo[i] = acc[i];
#pragma unroll
      for (int i = 51; i < NA; ++i) hi[i - 51] = acc[i];
      wave_store(lo, part, lane);
      wave_store(hi, part + 51, lane);
    } else {
      wave_store(acc, part, lane);
    }
}

template <typename R, bool SC>
__device__ __forceinline__ void camblk_task(const SlotDesc& d, const SlotCtl& c, int t, int lane) {
  if constexpr (SC) camblk_task_k<R, true, true>(d, c, t, lane);
  else if (d.kcol0 >= 0 || d.kcol1 >= 0) camblk_task_k<R, true, false>(d, c, t, lane);
  else camblk_task_k<R, false, false>(d, c, t, lane);
}

// Pair task t of a cluster (one wavefront).
template <typename R, bool SC>
__device__ __forceinline__ void pairblk_task_k(const SlotDesc& d, const SlotCtl& c, int t, int lane) {
  const int4 tk = d.tasks[t];
  const int ka = (tk.x >> 12) & 0xfff, kb = tk.x & 0xfff;
  const int cur = c.cur;
  const R f = SC ? (R)c.k[cur][2] : (R)d.f, is = (R)d.inv_sigma, dt = (R)d.huber_dt;
  const R k1 = (R)c.k[cur][0], k2 = (R)c.k[cur][1];
  const R cxo = SC ? (R)c.k[cur][3] : R(0), cyo = SC ? (R)c.k[cur][4] : R(0);
  const bool mixed = sizeof(R) == 4;
  const R* __restrict__ ptv = reinterpret_cast<const R*>(d.ptv);
  R* part = reinterpret_cast<R*>(d.task_part) + (size_t)t * kTaskVals;
  R ca[kCamVals];
  load_cam(d.cam[cur] + kCamVals * ka, ca);

    R cb[kCamVals];
    load_cam(d.cam[cur] + kCamVals * kb, cb);
    const gptr<const int> ql_pt = gmem(d.ql_pt);
    const gptr<const int> ql_ob = gmem(reinterpret_cast<const int*>(d.ql_ob));
    const gptr<const R> Xs = pts_of<R>(d, cur), uvs = uv_of<R>(d.ob_uv64, d.ob_uv32), recs = gmem(ptv);
    R acc[36];
#pragma unroll
    for (int i = 0; i < 36; ++i) acc[i] = R(0);
    // Loads are unconditional: padding lanes read point 0 and observation
    // lane 0 (finite state, record and pixels) and the observation model
    // gives them weight 0, which zeroes every term they add.  The next
    // chunk's point and observation lanes are requested a chunk ahead.
    const int ch_end = tk.y + tk.z;
    int pt_next = ql_pt[tk.y * kWave + lane];
    int lo_next[2] = {ql_ob[2 * (tk.y * kWave + lane)], ql_ob[2 * (tk.y * kWave + lane) + 1]};
    for (int ch = tk.y; ch < ch_end; ++ch) {
      const int idx = ch * kWave + lane;
      const int pt = pt_next;
      const int lo[2] = {lo_next[0], lo_next[1]};   // observation lanes of the pair
      if (ch + 1 < ch_end) {
        pt_next = ql_pt[idx + kWave];
        lo_next[0] = ql_ob[2 * (idx + kWave)];
        lo_next[1] = ql_ob[2 * (idx + kWave) + 1];
      }
      const bool valid = pt >= 0;
      const int ps = valid ? pt : 0;
      const R X0 = Xs[3 * ps], X1 = Xs[3 * ps + 1], X2 = Xs[3 * ps + 2];
      const R ua = uvs[2 * lo[0]], va = uvs[2 * lo[0] + 1], ub = uvs[2 * lo[1]], vb = uvs[2 * lo[1] + 1];
      R Q[8];
      rec_load<sizeof(R) == 8 ? 6 : 8>(recs + kPtVals * (size_t)ps, Q);
      // -Y_a W_b^T = J_ca^T M J_cb with the 2x2 M = -w_a w_b J_pa Q J_pb^T.
      R a0[6], a1[6], T[2][3], wa;
      {
        ObsJ<R, kNk<SC>> oa;
        obs_model<R, SC>(ca, X0, X1, X2, ua, va, f, k1, k2, is, dt, valid, oa, cxo, cyo);
        jp_q(oa, Q, T);
#pragma unroll
        for (int r = 0; r < 6; ++r) {
          a0[r] = jc(oa, 0, r);
          a1[r] = jc(oa, 1, r);
        }
        wa = oa.w;
      }
      ObsJ<R, kNk<SC>> ob;
      obs_model<R, SC>(cb, X0, X1, X2, ub, vb, f, k1, k2, is, dt, valid, ob, cxo, cyo);
      const R ww = -wa * ob.w;
      R M[2][2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          M[i][j] = ww * fm(T[i][2], ob.Jp[j][2], fm(T[i][1], ob.Jp[j][1], T[i][0] * ob.Jp[j][0]));
      R G0[6], G1[6];
#pragma unroll
      for (int cc = 0; cc < 6; ++cc) {
        const R b0 = jc(ob, 0, cc), b1 = jc(ob, 1, cc);
        G0[cc] = fm(M[0][0], b0, M[0][1] * b1);
        G1[cc] = fm(M[1][0], b0, M[1][1] * b1);
      }
#pragma unroll
      for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) acc[6 * r + cc] = fm(a0[r], G0[cc], fm(a1[r], G1[cc], acc[6 * r + cc]));
    }
    wave_store(acc, part, lane);
}

template <typename R, bool SC>
__device__ __forceinline__ void pairblk_task(const SlotDesc& d, const SlotCtl& c, int t, int lane) {
  pairblk_task_k<R, SC>(d, c, t, lane);
}

// Slot of logical workgroup b when cluster i owns workgroups
// [off_a[i] + off_b[i], off_a[i + 1] + off_b[i + 1]).
__device__ __forceinline__ int find_slot2(const int* __restrict__ off_a, const int* __restrict__ off_b, int n_act,
                                          int b) {
  int lo = 0, hi = n_act - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off_a[mid] + off_b[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Camera and pair tasks of every cluster in one launch (the FP32 path): a
// cluster's workgroups are contiguous, its camera tasks first, so its two
// kinds of task run side by side on one XCD and read its points through one
// L2, and the launch has one tail instead of two.  The self-calibrating
// instantiation (69 camera-task sums) is allowed more registers than four
// waves per SIMD leave, so that it does not spill.
template <typename R, bool SC>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(SC ? 2 : 4))) void k_blocks(Batch bt) {
  const int bx = xcd_block();
  if (bt.n_act == 0) return;   // empty dispatch that only carries timing events
  const int si = __builtin_amdgcn_readfirstlane(find_slot2(bt.tkc_off, bt.tkp_off, bt.n_act, bx));
  const int s = __builtin_amdgcn_readfirstlane(bt.act[si]);
  const SlotDesc& d = bt.desc[s];
  const SlotCtl& c = bt.ctl[s];
  if (c.status != ST_RUNNING || (d.sc != 0) != SC) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int loc = bx - (bt.tkc_off[si] + bt.tkp_off[si]);
  const int ncw = bt.tkc_off[si + 1] - bt.tkc_off[si];
  if (loc < ncw) {
    const int t = loc * kWavesPerWG + wave;
    if (t < d.n_cam_tasks) camblk_task<R, SC>(d, c, t, lane);
  } else {
    const int t = d.n_cam_tasks + (loc - ncw) * kWavesPerWG + wave;
    if (t < d.n_tasks) pairblk_task<R, SC>(d, c, t, lane);
  }
}

// The two kinds of task as separate launches (the FP64 path, whose pair tasks
// need fewer registers than its camera tasks).
template <typename R, bool SC>
__global__ __launch_bounds__(kWG) void k_camblk(Batch bt) {
  const int bx = xcd_block();
  if (bt.n_act == 0) return;   // empty dispatch that only carries timing events
  const int si = __builtin_amdgcn_readfirstlane(find_slot(bt.tkc_off, bt.n_act, bx));
  const int s = __builtin_amdgcn_readfirstlane(bt.act[si]);
  const SlotDesc& d = bt.desc[s];
  const SlotCtl& c = bt.ctl[s];
  if (c.status != ST_RUNNING || (d.sc != 0) != SC) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int t = (bx - bt.tkc_off[si]) * kWavesPerWG + wave;
  if (t < d.n_cam_tasks) camblk_task<R, SC>(d, c, t, threadIdx.x % kWave);
}
template <typename R, bool SC>
__global__ __launch_bounds__(kWG) void k_pairblk(Batch bt) {
  const int bx = xcd_block();
  if (bt.n_act == 0) return;   // empty dispatch that only carries timing events
  const int si = __builtin_amdgcn_readfirstlane(find_slot(bt.tkp_off, bt.n_act, bx));
  const int s = __builtin_amdgcn_readfirstlane(bt.act[si]);
  const SlotDesc& d = bt.desc[s];
  const SlotCtl& c = bt.ctl[s];
  if (c.status != ST_RUNNING || (d.sc != 0) != SC) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int t = d.n_cam_tasks + (bx - bt.tkp_off[si]) * kWavesPerWG + wave;
  if (t < d.n_tasks) pairblk_task<R, SC>(d, c, t, threadIdx.x % kWave);
}

// ---- reduction of the task partials into the reduced system -----------------------
//
// One workgroup per target (a free camera's diagonal block and borders, a
// camera-pair block, or the intrinsic block); sums its task range in order.

__device__ __forceinline__ void tri6(int v, int* r, int* c) {
  int rr = 0, len = 6;
  while (v >= len) { v -= len; ++rr; --len; }
  *r = rr;
  *c = rr + v;
}

constexpr int kReduceThreads = 256;

// Sums vals[k * stride + v] for k in [lo, hi) in a fixed order: thread
// (v, q) adds every sub-th entry starting at lo + q, then the sub partial sums
// of each value are added in q order.
template <typename R>
__device__ double fixed_sum(const R* __restrict__ vals, int stride, int nvals, int lo, int hi, double* sh, int tid) {
  const int sub = kReduceThreads / nvals;
  const int v = tid / sub, q = tid % sub;
  double t = 0.0;
  if (v < nvals)
    for (int k = lo + q; k < hi; k += sub) t += (double)vals[(size_t)k * stride + v];
  sh[tid] = t;
  __syncthreads();
  double r = 0.0;
  if (tid < nvals)
    for (int i = 0; i < sub; ++i) r += sh[tid * sub + i];
  return r;
}

template <typename R>
__global__ __launch_bounds__(kReduceThreads) void k_reduce(Batch bt) {
  const int bx = xcd_block();
  __shared__ double sh[kReduceThreads];
  if (bt.n_act == 0) return;   // empty dispatch that only carries timing events
  const int si = find_slot(bt.tg_off, bt.n_act, bx);
  const int s = bt.act[si];
  const SlotDesc& d = bt.desc[s];
  if (bt.ctl[s].status != ST_RUNNING) return;
  const int4 tg = d.targets[bx - bt.tg_off[si]];
  const int kind = tg.x >> 24, ka = (tg.x >> 12) & 0xfff, kb = tg.x & 0xfff;
  const int v = threadIdx.x;
  const int m = d.m, psize = d.psize;
  // intrinsic columns the kernels sum: k1, k2, and f, cx, cy when self-calibrating
  const int nk = d.sc ? kIntr : 2;
  double* Sg = d.Sg;
  if (kind == TARGET_INTR) {
    // point-pass sums: S (packed upper triangle), g, diag U, Schur part of b
    const int ns = nk * (nk + 1) / 2;
    const double t = fixed_sum(reinterpret_cast<const R*>(d.pt_part), kPtPartVals, ns + 3 * nk, tg.y, tg.z, sh, v);
    if (v >= ns + 3 * nk) return;
    if (v < ns) {
      int a = 0, r = v;
      while (r >= nk - a) { r -= nk - a; ++a; }
      const int ca = d.kcolt[a], cb = d.kcolt[a + r];
      if (ca >= 0 && cb >= 0) sput(Sg, ca, cb, t);
      return;
    }
    const int q = (v - ns) / nk, col = d.kcolt[(v - ns) % nk];
    if (col < 0) return;
    Sg[psize + (q == 0 ? 0 : q == 1 ? 2 * m : m) + col] = t;
    return;
  }
  const int nvals = kind == TASK_CAM ? 39 + 6 * nk : 36;
  const double t = fixed_sum(reinterpret_cast<const R*>(d.task_part), kTaskVals, nvals, tg.y, tg.z, sh, v);
  if (v >= nvals) return;
  const int fa = d.cam_col[ka];
  if (d.sparse) {
    // block-CSR reduced system: both orientations of a pair block, full diagonal blocks
    const int2 sl = d.tslot[bx - bt.tg_off[si]];
    if (kind == TASK_PAIR) {
      const int r = v / 6, cc = v % 6;
      d.Sblk[kSbVals * (size_t)sl.x + kSbRow * r + cc] = t;
      d.Sblk[kSbVals * (size_t)sl.y + kSbRow * cc + r] = t;
      d.Sblk32[kSbVals * (size_t)sl.x + kSbRow * r + cc] = (float)t;
      d.Sblk32[kSbVals * (size_t)sl.y + kSbRow * cc + r] = (float)t;
      return;
    }
    if (v < 21) {
      int r, cc;
      tri6(v, &r, &cc);
      d.Sblk[kSbVals * (size_t)sl.x + kSbRow * r + cc] = t;
      d.Sblk[kSbVals * (size_t)sl.x + kSbRow * cc + r] = t;
      return;
    }
  }
  if (kind == TASK_PAIR) {
    const int fb = d.cam_col[kb];
    sput(Sg, fa + v / 6, fb + v % 6, t);
    return;
  }
  if (v < 21) {
    int r, cc;
    tri6(v, &r, &cc);
    sput(Sg, fa + r, fa + cc, t);
  } else if (v < 27) Sg[psize + fa + (v - 21)] = t;
  else if (v < 33) Sg[psize + m + fa + (v - 27)] = t;
  else if (v < 39) Sg[psize + 2 * m + fa + (v - 33)] = t;
  else {
    const int col = d.kcolt[(v - 39) / 6];
    if (col >= 0) sput(Sg, fa + (v - 39) % 6, col, t);
  }
}

// ---- damped reduced-camera-system solve (one workgroup per cluster) ------------
//
// The damped system is held in LDS as the lower triangle of 16x16 FP64 blocks
// (the padding rows and columns are identity; each block row is padded to 17
// doubles so that 16 lanes reading one column hit 16 distinct bank pairs).
// Right-looking block Cholesky: one wavefront factors the diagonal block and
// forms the inverse of its factor; the panel (A_IK L_KK^-T) and the trailing
// update (A_IJ -= L_IK L_JK^T) are 16x16x16 FP64 products on the matrix cores
// (v_mfma_f64_16x16x4), spread over the four wavefronts.  The block
// triangular solves use the inverted diagonal blocks; in mixed mode one FP64
// refinement step runs against a copy of the damped system (LDS when it fits,
// global memory otherwise).

constexpr int kSolveWG = 256;                   // four wavefronts
constexpr int kSolveWk = 2 * kSolveTb * kSolveTb + kSolveTb;   // factor scratch + solve vector
constexpr size_t kSolveLdsCap = 150 * 1024;
static_assert(kSolveTb * ((6 * kMaxFreeCams + kIntr + kSolveTb - 1) / kSolveTb) <= kSolveWG,
              "one thread per unknown of the padded system in the solve's load");

// LDS doubles of the solve kernel for a batch whose largest system has nbm
// blocks per side, without and with the refinement copy.  Every cluster of the
// batch uses at most this layout, so the copy decision is made per launch.
__host__ __device__ inline size_t solve_lds_base(int nbm) {
  const size_t nb = (size_t)nbm;
  return nb * (nb + 1) / 2 * kTbV + nb * kTbV + 5 * kSolveTb * nb + kSolveWk;
}
__host__ __device__ inline bool solve_lds_copy(int nbm) {
  const size_t nb = (size_t)nbm;
  return sizeof(double) * (solve_lds_base(nbm) + nb * (nb + 1) / 2 * kTbV) <= kSolveLdsCap;
}


__device__ __forceinline__ void decode_tri(int e, int* ii, int* jj) {   // e -> (ii >= jj)
  int i = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  while (i * (i + 1) / 2 > e) --i;
  while ((i + 1) * (i + 2) / 2 <= e) ++i;
  *ii = i;
  *jj = e - i * (i + 1) / 2;
}

// In-place Cholesky of the 6x6 SPD block a (row-major, lower triangle used)
// and the lower-triangular inverse of the factor into li; in registers.
__device__ __forceinline__ bool chol6_inv(double* __restrict__ a, double* __restrict__ li) {
  double L[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) L[i][j] = j <= i ? a[6 * i + j] : 0.0;
  double inv[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double dj = L[j][j];
#pragma unroll
    for (int t = 0; t < j; ++t) dj -= L[j][t] * L[j][t];
    if (!(dj > 0.0) || !isfinite(dj)) return false;
    dj = sqrt(dj);
    L[j][j] = dj;
    inv[j] = 1.0 / dj;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double v = L[i][j];
#pragma unroll
      for (int t = 0; t < j; ++t) v -= L[i][t] * L[j][t];
      L[i][j] = v * inv[j];
    }
  }
  double I[6][6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
#pragma unroll
    for (int r = 0; r < 6; ++r) I[r][c] = 0.0;
    I[c][c] = inv[c];
#pragma unroll
    for (int r = c + 1; r < 6; ++r) {
      double v = 0.0;
#pragma unroll
      for (int t = c; t < r; ++t) v += L[r][t] * I[t][c];
      I[r][c] = -v * inv[r];
    }
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (j <= i) a[6 * i + j] = L[i][j];
      li[6 * i + j] = I[i][j];
    }
  return true;
}

typedef double double4_t __attribute__((ext_vector_type(4)));

// Lane l's value of v from lane `src` (wave-uniform result).
__device__ __forceinline__ double readlane_d(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/sqrt(x) for x > 0: the hardware estimate (about 23 correct bits) and one
// Newton step y <- y + y (1 - x y^2) / 2, which doubles the correct bits.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 1; ++it) {
    const double e = __builtin_fma(-x, y * y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
  }
  return y;
}

// Cholesky factor of the 16x16 SPD block a (full symmetric storage, stride
// kTbS) and the inverse of the factor into li (lower, zeros above); one
// wavefront.  Lane c + 16 g holds rows g, g+4, g+8, g+12 of column c of the
// block and of the inverse (forward substitution of L X = I, column by column
// alongside the factorisation).  Column j: the lanes holding row j form
// L[c][j] and X[j][c] and post them to LDS; every lane then updates its four
// rows.  The next pivot is formed from two lane reads before that update, so
// the LDS round trip stays off the pivot chain; the column steps have no
// branches (every group posts to its own slot, updates are masked), so the
// unrolled steps can overlap.  wk: 2 x 256 doubles scratch.  Returns false
// (wave-uniform) when a pivot is not positive and finite.
__device__ bool chol16_inv(const double* __restrict__ a, double* __restrict__ li, double* __restrict__ wk, int lane) {
  constexpr int T = kSolveTb;
  const int c = lane & (T - 1), g = lane >> 4;
  double* colL = wk;           // [j % 4][group][c] = L[c][j]
  double* rowX = wk + T * T;   // [j % 4][group][c] = X[j][c]
  double v[4], x[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = a[(4 * k + g) * kTbS + c];
    x[k] = (4 * k + g == c) ? 1.0 : 0.0;
  }
  bool good = true;
  double piv = readlane_d(v[0], 0);
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const int jg = j & 3, jk = j >> 2, slot = (j & 3) * 4 * T;
    good = good && piv > 0.0 && piv < 1e300;
    const double rs = rsqrt_nr(piv);
    const double l = c >= j ? v[jk] * rs : 0.0;   // L[c][j], meaningful in group jg
    const double xj = x[jk] * rs;                  // X[j][c], meaningful in group jg
    double pn = 1.0;
    if (j + 1 < T) {
      const double lt = readlane_d(l, (j + 1) + 16 * jg);                            // L[j+1][j]
      const double dv = readlane_d(v[(j + 1) >> 2], (j + 1) + 16 * ((j + 1) & 3));   // A[j+1][j+1]
      pn = __builtin_fma(-lt, lt, dv);
    }
    colL[slot + g * T + c] = l;
    rowX[slot + g * T + c] = xj;
    x[jk] = g == jg ? xj : x[jk];
    wave_sync();
    const double lc = colL[slot + jg * T + c], xc = rowX[slot + jg * T + c];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double lij = 4 * k + g > j ? colL[slot + jg * T + 4 * k + g] : 0.0;   // L[i][j], rows below j
      v[k] = __builtin_fma(-lij, lc, v[k]);
      x[k] = __builtin_fma(-lij, xc, x[k]);
    }
    piv = pn;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) li[(4 * k + g) * kTbS + c] = x[k];
  wave_sync();
  return good;
}

// 16x16 block product on the matrix cores: out = cin + sgn * P Q^T, with P, Q,
// cin and out blocks of stride kTbS (out may alias cin or P); one wavefront.
// Operand layouts of v_mfma_f64_16x16x4: A lane l -> (row l%16, k l/16),
// B lane l -> (k l/16, column l%16), C/D lane l, register r -> (row l/16 + 4r,
// column l%16).
__device__ __forceinline__ void mfma_blk(const double* P, const double* Q,
                                         const double* cin, double* out, double sgn, int lane) {
  const int lo = lane & 15, hi = lane >> 4;
  double pa[4], qb[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    pa[s] = sgn * P[lo * kTbS + 4 * s + hi];
    qb[s] = Q[lo * kTbS + 4 * s + hi];
  }
  double4_t acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = cin ? cin[(hi + 4 * r) * kTbS + lo] : 0.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[s], qb[s], acc, 0, 0, 0);
  wave_sync();   // every lane's operands are read before any result lands (out may alias them)
#pragma unroll
  for (int r = 0; r < 4; ++r) out[(hi + 4 * r) * kTbS + lo] = acc[r];
}

__global__ __launch_bounds__(kSolveWG) void k_solve(Batch bt) {
  extern __shared__ double sd[];
  const int s = bt.act[blockIdx.x];
  const SlotDesc& d = bt.desc[s];
  SlotCtl& c = bt.ctl[s];
  if (c.status != ST_RUNNING || d.sparse) return;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave), lane = tid % kWave;
  const int m = d.m, psize = d.psize, nb = d.nb;
  const int np = nb * kSolveTb, ntri = nb * (nb + 1) / 2;
  double* A = sd;                    // [ntri] lower block triangle
  double* Li = A + ntri * kTbV;      // [nb] inverses of the diagonal factor blocks
  double* gv = Li + nb * kTbV;       // [np] gradient of the camera side (with priors)
  double* Dv = gv + np;              // [np] clamped diagonal of H
  double* xv = Dv + np;              // [np] solution
  double* bv = xv + np;              // [np] right-hand side
  double* rv = bv + np;              // [np] refinement residual
  double* wk = rv + np;              // [kSolveWk] factor scratch, solve vector
  double* Sl = wk + kSolveWk;        // [ntri] damped copy, when it fits
  __shared__ int ok;
  const double lambda = c.lambda;
  const int cur = c.cur;
  // Load: the reduced system's blocks (written in this layout by the
  // reduction) with coalesced row reads; padding rows and columns beyond m
  // are those of the identity.  Thread tid owns element (tid / 16, tid % 16)
  // of every block; kLd blocks are requested at once.  The cached pose-prior
  // terms of camera tid are requested first.
  constexpr int kLd = 16;
  // global (not generic) loads: they count on the vector-memory counter only,
  // so waits for scalar loads do not wait for them
  typedef const __attribute__((address_space(1))) double* gdp;
  const gdp __restrict__ Sg = (gdp)d.Sg;
  const int er = tid / kSolveTb, ec = tid % kSolveTb;
  double val[kLd];
  auto fetch = [&](int b0) {
    int bi = 0, bj = b0;
    while (bj > bi) bj -= ++bi;   // block b0 -> (bi, bj), bj <= bi (uniform)
#pragma unroll
    for (int u = 0; u < kLd; ++u) {
      const int p = kSolveTb * bi + er, q = kSolveTb * bj + ec;
      val[u] = (p == q) ? 1.0 : 0.0;
      if (b0 + u < ntri && p < m && q < m) val[u] = Sg[(b0 + u) * kTbV + er * kTbS + ec];
      if (++bj > bi) { ++bi; bj = 0; }
    }
  };
  auto put = [&](int b0) {
#pragma unroll
    for (int u = 0; u < kLd; ++u)
      if (b0 + u < ntri) A[(b0 + u) * kTbV + er * kTbS + ec] = val[u];
  };
  const int pk = min(tid, d.C - 1);
  // the prior terms of camera tid at the current state (cached when that
  // state's cameras were formed), requested first
  double pe[6], pJ[9], pis[3];   // pis: 1/sigma of the position prior, three axes
  {
    const gdp gt = (gdp)d.pterm[cur] + kPtermVals * pk;
#pragma unroll
    for (int i = 0; i < 6; ++i) pe[i] = gt[i];
#pragma unroll
    for (int i = 0; i < 9; ++i) pJ[i] = gt[6 + i];
    const gdp gs = (gdp)d.prior + kPriorVals * pk + 15;
#pragma unroll
    for (int i = 0; i < 3; ++i) pis[i] = gs[i];
  }
  const int pcol = tid < d.C ? d.cam_col[tid] : -1;
  // what the closing wavefront needs (camera tid's state and prior, the
  // intrinsics), requested now so that its loads are off the kernel's tail
  double fcam[kCamVals], fpr[kPriorVals], kcur[kIntr];
  if (tid < kWave) {
    const gdp gc = (gdp)d.cam[cur] + kCamVals * pk, gp = (gdp)d.prior + kPriorVals * pk;
#pragma unroll
    for (int i = 0; i < kCamVals; ++i) fcam[i] = gc[i];
#pragma unroll
    for (int i = 0; i < kPriorVals; ++i) fpr[i] = gp[i];
#pragma unroll
    for (int t = 0; t < kIntr; ++t) kcur[t] = c.k[cur][t];
  }
  __asm__ volatile("" ::: "memory");
  fetch(0);
  // gradient, bS and diag U of unknown tid (np <= 160 < kSolveWG), in the same batch
  const bool vreal = tid < m;
  const double g0 = vreal ? Sg[psize + tid] : 0.0, b0v = vreal ? Sg[psize + m + tid] : 0.0,
               d0 = vreal ? Sg[psize + 2 * m + tid] : 0.0;
  put(0);
  for (int b0 = kLd; b0 < ntri; b0 += kLd) {
    fetch(b0);
    put(b0);
  }
  if (tid < np) {
    gv[tid] = g0;
    xv[tid] = b0v;   // bS for now
    Dv[tid] = d0;    // diag U for now
  }
  if (tid == 0) ok = (c.point_fail == 0);
  __syncthreads();
  // Pose priors of the free cameras, one thread per camera (disjoint entries).
  // Element (p, q) is stored when p's block row is at or below q's; the
  // diagonal blocks hold both triangles.
  auto add_prior = [&](int col, const double* e, const double* J, const double* is) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double h = J[r] * J[q] + J[3 + r] * J[3 + q] + J[6 + r] * J[6 + q];
        const int p0 = col + r, q1 = col + q;
        if (p0 / kSolveTb >= q1 / kSolveTb)
          A[tblk(p0 / kSolveTb, q1 / kSolveTb) + (p0 % kSolveTb) * kTbS + q1 % kSolveTb] += h;
        if (q == r) Dv[col + r] += h;
      }
      gv[col + r] += J[r] * e[0] + J[3 + r] * e[1] + J[6 + r] * e[2];
      const double it = is[r];
      const int p3 = col + 3 + r;
      A[tblk(p3 / kSolveTb, p3 / kSolveTb) + (p3 % kSolveTb) * (kTbS + 1)] += it * it;
      Dv[col + 3 + r] += it * it;
      gv[col + 3 + r] += it * e[3 + r];
    }
  };
  if (pcol >= 0) add_prior(pcol, pe, pJ, pis);
  for (int k = tid + kSolveWG; k < d.C; k += kSolveWG) {   // clusters of more than 256 cameras
    const int col = d.cam_col[k];
    if (col < 0) continue;
    double e[6], J[9];
    pterm_load(d.pterm[cur] + kPtermVals * k, e, J);
    add_prior(col, e, J, d.prior + kPriorVals * k + 15);
  }
  __syncthreads();
  // Marquardt damping and the right-hand side.
  for (int p = tid; p < np; p += kSolveWG) {
    if (p < m) {
      const double Di = clampd(Dv[p]);
      Dv[p] = Di;
      A[tblk(p / kSolveTb, p / kSolveTb) + (p % kSolveTb) * (kTbS + 1)] += lambda * Di;
      bv[p] = -gv[p] + xv[p];
    } else {
      Dv[p] = 0.0;
      bv[p] = 0.0;
    }
    xv[p] = bv[p];
  }
  __syncthreads();
  const bool lds_copy = solve_lds_copy(bt.max_nb);
  if (d.mixed) {
    if (lds_copy) for (int e = tid; e < ntri * kTbV; e += kSolveWG) Sl[e] = A[e];
    else for (int e = tid; e < ntri * kTbV; e += kSolveWG) d.Sd[e] = A[e];
    __syncthreads();
  }
  // Right-looking block Cholesky.
  for (int K = 0; K < nb; ++K) {
    if (wave == 0) {
      const bool good = chol16_inv(A + tblk(K, K), Li + K * kTbV, wk, lane);
      if (!good && lane == 0) ok = 0;
    }
    __syncthreads();
    if (!ok) break;
    // panel: L_IK = A_IK L_KK^-T
    for (int I = K + 1 + wave; I < nb; I += kSolveWG / kWave)
      mfma_blk(A + tblk(I, K), Li + K * kTbV, nullptr, A + tblk(I, K), 1.0, lane);
    __syncthreads();
    // trailing update: A_IJ -= L_IK L_JK^T for K < J <= I
    const int R = nb - K - 1;
    for (int pr = wave; pr < R * (R + 1) / 2; pr += kSolveWG / kWave) {
      int ii, jj;
      decode_tri(pr, &ii, &jj);
      const int I = K + 1 + ii, J = K + 1 + jj;
      mfma_blk(A + tblk(I, K), A + tblk(J, K), A + tblk(I, J), A + tblk(I, J), -1.0, lane);
    }
    __syncthreads();
  }
  if (!ok) {
    if (tid == 0) c.solve_ok = 0;
    return;
  }
  // W = L^-1, block lower triangular, in place of L's off-diagonal blocks
  // (its diagonal blocks are the inverted factor blocks Li), block row by
  // block row: W_IJ = -Li_I sum_{K=J}^{I-1} L_IK W_KJ on the matrix cores,
  // wavefront w taking the columns J = w, w + 4, w + 8.  The running sum
  // stays in the product's accumulator, which is also the B operand layout
  // of the product by Li_I.  Then every solve is two matrix-vector products,
  // x = W^T (W b), all threads at once.
  {
    const int lo = lane & 15, hi = lane >> 4;
    for (int I = 1; I < nb; ++I) {
      double4_t res[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int J = wave + 4 * q;
        res[q] = double4_t{0.0, 0.0, 0.0, 0.0};
        if (J >= I) continue;
        double4_t t = {0.0, 0.0, 0.0, 0.0};
        for (int K = J; K < I; ++K) {
          const double* P = A + tblk(I, K);
          const double* Q = K == J ? Li + J * kTbV : A + tblk(K, J);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            t = __builtin_amdgcn_mfma_f64_16x16x4f64(P[lo * kTbS + 4 * u + hi], Q[(4 * u + hi) * kTbS + lo], t, 0, 0,
                                                      0);
        }
        const double* L = Li + I * kTbV;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          res[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-L[lo * kTbS + 4 * u + hi], t[u], res[q], 0, 0, 0);
      }
      __syncthreads();   // every wavefront has read block row I of L
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int J = wave + 4 * q;
        if (J >= I) continue;
        double* out = A + tblk(I, J);
#pragma unroll
        for (int r = 0; r < 4; ++r) out[(hi + 4 * r) * kTbS + lo] = res[q][r];
      }
      __syncthreads();
    }
  }
  double* yv = wk;   // [np]
  // out = W^T (W in); out may be in
  auto wsolve = [&](const double* in, double* out) {
    for (int p = tid; p < np; p += kSolveWG) {   // y = W in, one row each
      const int I = p / kSolveTb, r = p % kSolveTb;
      double s0 = 0.0, s1 = 0.0;
      for (int J = 0; J <= I; ++J) {
        const double* row = (J == I ? Li + I * kTbV : A + tblk(I, J)) + r * kTbS;
#pragma unroll
        for (int q = 0; q < kSolveTb; q += 2) {
          s0 = __builtin_fma(row[q], in[kSolveTb * J + q], s0);
          s1 = __builtin_fma(row[q + 1], in[kSolveTb * J + q + 1], s1);
        }
      }
      yv[p] = s0 + s1;
    }
    __syncthreads();
    for (int p = tid; p < np; p += kSolveWG) {   // out = W^T y, one column each
      const int J = p / kSolveTb, c = p % kSolveTb;
      double s0 = 0.0, s1 = 0.0;
      for (int I = J; I < nb; ++I) {
        const double* col = (I == J ? Li + J * kTbV : A + tblk(I, J)) + c;
#pragma unroll
        for (int r = 0; r < kSolveTb; r += 2) {
          s0 = __builtin_fma(col[r * kTbS], yv[kSolveTb * I + r], s0);
          s1 = __builtin_fma(col[(r + 1) * kTbS], yv[kSolveTb * I + r + 1], s1);
        }
      }
      out[p] = s0 + s1;
    }
    __syncthreads();
  };
  wsolve(bv, xv);
  if (d.mixed) {
    // one FP64 refinement step: r = b - S_damped x, then dx = S^-1 r, x += dx
    const double* Sd = lds_copy ? Sl : d.Sd;
    for (int p = tid; p < np; p += kSolveWG) {
      const int P = p / kSolveTb, pr_ = p % kSolveTb;
      double t0 = bv[p], t1 = 0.0;
      for (int Q = 0; Q < nb; ++Q) {
        const double* B = Sd + (P >= Q ? tblk(P, Q) + pr_ * kTbS : tblk(Q, P) + pr_);
        const int stride = P >= Q ? 1 : kTbS;
#pragma unroll
        for (int q = 0; q < kSolveTb; q += 2) {
          t0 = __builtin_fma(-B[stride * q], xv[kSolveTb * Q + q], t0);
          t1 = __builtin_fma(-B[stride * (q + 1)], xv[kSolveTb * Q + q + 1], t1);
        }
      }
      rv[p] = t0 + t1;
    }
    __syncthreads();
    wsolve(rv, rv);
    for (int p = tid; p < np; p += kSolveWG) xv[p] += rv[p];
    __syncthreads();
  }
  if (tid >= kWave) return;
  // From here on one wavefront: predicted decrease, trial cameras, prior cost.
  double pacc = 0.0;
  for (int p = tid; p < m; p += kWave) pacc += xv[p] * (lambda * Dv[p] * xv[p] - gv[p]);
  const double predc = wave_sum(pacc);
  for (int p = tid; p < m; p += kWave) d.dc[p] = xv[p];
  const int nxt = 1 - cur;
  double pc = 0.0;
  for (int k = tid; k < d.C; k += kWave) {
    // the first camera of each lane from the registers loaded at the start
    double cm[kCamVals], pr[kPriorVals];
    const bool pre = k == tid;
#pragma unroll
    for (int i = 0; i < kCamVals; ++i) cm[i] = pre ? fcam[i] : d.cam[cur][kCamVals * k + i];
    double* cn = d.cam[nxt] + kCamVals * k;
    const int col = pre ? pcol : d.cam_col[k];
    if (col < 0) {
      for (int i = 0; i < kCamVals; ++i) cn[i] = cm[i];
      continue;
    }
#pragma unroll
    for (int i = 0; i < kPriorVals; ++i) pr[i] = pre ? fpr[i] : d.prior[kPriorVals * k + i];
    const double wv[3] = {xv[col], xv[col + 1], xv[col + 2]};
    double E[9], cv[kCamVals];
    so3_exp(wv, E);
    #pragma unroll
    for (int i = 0; i < 3; ++i)
      #pragma unroll
      for (int j = 0; j < 3; ++j) cv[3 * i + j] = cm[3 * i] * E[j] + cm[3 * i + 1] * E[3 + j] + cm[3 * i + 2] * E[6 + j];
    #pragma unroll
    for (int i = 0; i < 3; ++i) cv[9 + i] = cm[9 + i] + xv[col + 3 + i];
    #pragma unroll
    for (int i = 0; i < kCamVals; ++i) cn[i] = cv[i];
    double e[6], J[9];
    prior_terms(cv, pr, e, J);
    pterm_store(d.pterm[nxt] + kPtermVals * k, e, J);
    #pragma unroll
    for (int i = 0; i < 6; ++i) pc += e[i] * e[i];
  }
  pc = wave_sum(pc);
  if (tid == 0) {
    c.pred_c = predc;
    c.E_prior_trial = 0.5 * pc;
    for (int t = 0; t < 5; ++t) c.k[nxt][t] = kcur[t] + (d.kcolt[t] >= 0 ? xv[d.kcolt[t]] : 0.0);
  }
}

// ---- damped reduced-camera-system solve by preconditioned conjugate gradients ------
//
// For large reduced systems (a whole-flight adjustment: hundreds of cameras),
// the Schur complement is kept as 6x6 blocks of the co-visible camera pairs
// (block CSR, both orientations) and solved by conjugate gradients with the
// inverse diagonal blocks as block-Jacobi preconditioner.  One cooperative
// launch per such cluster: G workgroups, each owning a contiguous range of
// block rows, whose blocks it copies into LDS once and keeps there for the
// whole solve (in mixed mode the FP32 copy: FP32 products and accumulation;
// dot products, the preconditioner and the updates are FP64).  Thread t of a
// workgroup owns block row r0 + t (x, r in registers, its preconditioner
// block in LDS; at most kCgMaxRows rows, so the owners are in wavefront 0
// and every scalar row of S p has a thread: up to four, each taking every
// fourth block).  Every
// workgroup keeps the entries of the direction p that its rows' blocks
// multiply (its halo: the block columns of its blocks) in LDS, updated the
// same way in every workgroup.
//
// One grid barrier per CG step.  With q = S p and u = M^-1 q, step i needs
// p.q and r.z, and the next step's scalars follow from sums over vectors
// that are known before the step's update x += alpha p, r -= alpha q,
// z -= alpha u:
//   r'.r' = r.r - 2 alpha r.q + alpha^2 q.q,
//   r'.z' = r.z - 2 alpha q.z + alpha^2 q.u     (r.u = q.z: M symmetric).
// So the owners post their parts of p.q, r.q, q.q, q.z, q.u, r.r, r.z
// (summed over wavefront 0) and their rows of z = M^-1 r (recomputed from r
// every step) and u, together; after the barrier every wavefront of every
// workgroup adds the G parts by the same butterfly (all take the same
// decisions), the owners update their rows of x and r, and every workgroup
// forms its halo of the next p from z and u.  r.r and r.z are taken fresh
// from the vectors each step and z is recomputed from r, so the expansions
// only carry one step's rounding (of order eps times the step's r.r and
// r.z), never an error accumulated from earlier steps.  The (z, u) pairs and
// the parts are double-buffered by step parity: a workgroup posts step i + 1
// only after the barrier of step i, which every workgroup reaches only after
// reading what step i - 1 posted.

namespace cg = cooperative_groups;

constexpr int kCgSums = 7;                // p.q, r.q, q.q, q.z, q.u, r.r, r.z
constexpr int kCgPartStride = 8;          // doubles per workgroup part (7 used)
constexpr long kCgSpinCap = 1L << 22;     // polls before a barrier wait gives up (seconds)
// halo entries of p per thread, at most (the halo is at most all m <= 6 kMaxCams entries)
constexpr int kCgHalo = (6 * kMaxCams + kCgThreads - 1) / kCgThreads;

// Sums over the workgroup in a fixed order (N values at once); every thread
// gets the sums.
template <int N>
__device__ __forceinline__ void wg_sum(double v[N], double* red, int tid) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
  __syncthreads();
  if ((tid % kWave) == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) red[i * kCgWaves + tid / kWave] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kCgWaves; ++w) t += red[i * kCgWaves + w];
    v[i] = t;
  }
}

__device__ __forceinline__ double2 wg_sum2(double a, double b, double* red, int tid) {
  double v[2] = {a, b};
  wg_sum<2>(v, red, tid);
  return make_double2(v[0], v[1]);
}

// Parts of the G workgroups, added in workgroup order (every thread the same sums).
__device__ __forceinline__ double2 grid_sum2(const double2* __restrict__ parts, int G) {
  double2 t = make_double2(0.0, 0.0);
  for (int w = 0; w < G; ++w) {
    const double2 v = parts[w];
    t.x += v.x;
    t.y += v.y;
  }
  return t;
}

// Grid barrier of the conjugate-gradient launch: a counter that only grows
// (across launches too, wrapping at 2^32).  A workgroup arrives by adding 1
// (release at agent scope: its earlier global writes become visible to any
// workgroup that then acquires) and waits, acquiring, until the counter has
// passed `target` (the launch's base plus G per barrier).  Every workgroup of
// a cooperative launch is resident and passes the same barriers, so every
// wait ends.  As a guard all the same, a wait that has not ended after
// kCgSpinCap polls raises the launch's abort word, and every wait returns
// false as soon as it sees that word set: the whole grid then leaves early
// (the solve is reported failed) instead of waiting on a missing workgroup.
__device__ __forceinline__ bool cg_barrier(unsigned* ctr, unsigned target, unsigned* abort_word, int* ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    long n = 0;
    while ((int)(__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        *ok = 0;
        break;
      }
      if (++n > kCgSpinCap) {
        __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *ok = 0;
        break;
      }
    }
  }
  __syncthreads();
  return *ok != 0;
}

// z = Li^T Li r for one 6x6 block (Li: packed lower triangle, row-major).
__device__ __forceinline__ void pcg_precond(const double* Li, const double r[6], double z[6]) {
  double y[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double t = 0.0;
#pragma unroll
    for (int c = 0; c <= i; ++c) t = fm(Li[i * (i + 1) / 2 + c], r[c], t);
    y[i] = t;
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    double t = 0.0;
#pragma unroll
    for (int i = 5; i >= c; --i) t = fm(Li[i * (i + 1) / 2 + c], y[i], t);
    z[c] = t;
  }
}

// This workgroup's rows of S p from LDS: its blocks Sl, its block-row
// starts brl and block columns bcl (both relative to its first block), and p
// (read in the product's precision: FP32 copy [F][8] in mixed mode, FP64 [m]
// otherwise).  spt adjacent lanes (1, 2 or 4; 6 nr spt <= kCgThreads) share
// a scalar row q (local: block row q / 6, row q % 6 of it), each taking every
// spt-th block, and add their parts by a fixed butterfly; the first of them
// writes Apl[q].
template <typename B, int PS>
__device__ __forceinline__ void cg_spmv(const B* __restrict__ Sl, const int* __restrict__ brl,
                                        const int* __restrict__ bcl, int nr, int spt, const B* pB, double* Apl,
                                        int tid) {
  const int q = tid / spt, j = tid % spt;
  B acc = B(0);
  if (q < 6 * nr) {
    const int bl = q / 6, r = q % 6;
    const int ka = brl[bl], kb = brl[bl + 1];
    for (int k = ka + j; k < kb; k += spt) {
      const B* row = Sl + kSbVals * (size_t)k + kSbRow * r;
      const B* pp = pB + PS * bcl[k];
#pragma unroll
      for (int cc = 0; cc < 6; ++cc) acc = fm(row[cc], pp[cc], acc);
    }
  }
  for (int off = 1; off < spt; off <<= 1) acc += __shfl_xor(acc, off, kWave);
  if (q < 6 * nr && j == 0) Apl[q] = (double)acc;
}

__global__ __launch_bounds__(kCgThreads) void k_pcg(Batch bt, int s) {
  extern __shared__ __attribute__((aligned(16))) double sv[];
  __shared__ double red[2 * kCgWaves];
  __shared__ int own_cam[kWave];
  __shared__ int brl[kWave + 1];
  __shared__ int hmark[kMaxCams];
  __shared__ int hcol[kMaxCams];
  __shared__ int n_halo;
  __shared__ unsigned bar_base;
  __shared__ int bar_ok;
  const SlotDesc& d = bt.desc[s];
  SlotCtl& c = bt.ctl[s];
  // read by every workgroup before anything is written: the same decision everywhere
  if (c.status != ST_RUNNING || !d.sparse) return;
  cg::grid_group grid = cg::this_grid();
  const int tid = threadIdx.x, wg = blockIdx.x, G = gridDim.x;
  const int lane = tid % kWave;
  const int F = d.n_free, m = d.m;
  const int r0 = d.pcg_part[wg], r1 = d.pcg_part[wg + 1], nr = r1 - r0;   // nr <= kCgMaxRows
  const int* const brow = d.brow;
  const int* const bcol = d.bcol;
  const int k0 = brow[r0], nblk = brow[r1] - k0;
  const bool mixed = d.mixed != 0;
  const int spt = 6 * nr * 4 <= kCgThreads ? 4 : 6 * nr * 2 <= kCgThreads ? 2 : 1;
  // global work: gradient with priors, clamped diagonal, z_0, (z, u) pairs
  // (two buffers), the set-up and final parts, the CG parts (two buffers),
  // the barrier words
  double* gv = d.pcgw;
  double* Dv = gv + m;
  double* zg = Dv + m;
  double2* zug = reinterpret_cast<double2*>(zg + m);               // [2][m]
  double2* part = zug + 2 * m;                                      // [2][kMaxCgWG]
  double* cgp = reinterpret_cast<double*>(part + 2 * kMaxCgWG);    // [2][kMaxCgWG][kCgPartStride]
  unsigned* ctr = reinterpret_cast<unsigned*>(cgp + 2 * kMaxCgWG * kCgPartStride);
  unsigned* abort_word = ctr + 1;
  // LDS: this workgroup's blocks and their block columns, p (FP64, and FP32
  // in mixed mode; only the halo entries are kept), its rows of S p, its
  // preconditioner blocks
  const size_t sbytes = (mixed ? sizeof(float) : sizeof(double)) * kSbVals * (size_t)nblk;
  int* bcl = reinterpret_cast<int*>(reinterpret_cast<unsigned char*>(sv) + sbytes);
  double* pl = sv + (sbytes + sizeof(int) * (size_t)nblk + 7) / 8;
  float* p32l = reinterpret_cast<float*>(pl + m);
  double* Apl = pl + m + 4 * F;
  double* Lf = Apl + 6 * d.pcg_rows_max;
  const float* S32l = reinterpret_cast<const float*>(sv);
  const double* S64l = sv;
  const double lambda = c.lambda;
  const int cur = c.cur;
  if (tid == 0) {
    // no workgroup arrives at a CG barrier or reads the abort word before the
    // set-up grid barrier below
    bar_base = __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bar_ok = 1;
    if (wg == 0) __hip_atomic_store(abort_word, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  for (int k = tid; k < nr; k += kCgThreads) own_cam[k] = -1;
  for (int k = tid; k <= nr; k += kCgThreads) brl[k] = brow[r0 + k] - k0;
  for (int k = tid; k < F; k += kCgThreads) hmark[k] = 0;
  __syncthreads();
  for (int k = tid; k < nblk; k += kCgThreads) {
    const int col = bcol[k0 + k];
    bcl[k] = col;
    hmark[col] = 1;
  }
  for (int k = tid; k < d.C; k += kCgThreads) {
    const int col = d.cam_col[k];
    if (col >= 0 && col / 6 >= r0 && col / 6 < r1) own_cam[col / 6 - r0] = k;
  }
  __syncthreads();
  // the halo, in increasing block column (wavefront 0 compacts the marks)
  if (tid < kWave) {
    int n = 0;
    for (int f0 = 0; f0 < F; f0 += kWave) {
      const int f = f0 + lane;
      const bool on = f < F && hmark[f] != 0;
      const unsigned long long bits = __ballot(on);
      if (on) hcol[n + __popcll(bits & ((1ull << lane) - 1ull))] = f;
      n += __popcll(bits);
    }
    if (lane == 0) n_halo = n;
  }
  // Owner set-up: priors and damping into the diagonal block, preconditioner,
  // right-hand side, z_0 = M^-1 r_0 (= p_0).
  const bool own = tid < nr;
  double xr[6], rr[6];
  double part_rr = 0.0, part_rz = 0.0, fails = 0.0;
  if (own) {
    const int f = r0 + tid, k = own_cam[tid], col = 6 * f;
    double g[6], Dg[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      g[a] = d.Sg[col + a];
      rr[a] = d.Sg[m + col + a];      // bS for now
      Dg[a] = d.Sg[2 * m + col + a];  // diag U for now
    }
    double* Ab = d.Sblk + kSbVals * (size_t)brow[f];
    double blkv[36];
#pragma unroll
    for (int i = 0; i < 36; ++i) blkv[i] = Ab[kSbRow * (i / 6) + i % 6];
    double e[6], J[9];
    pterm_load(d.pterm[cur] + kPtermVals * k, e, J);
    const double* pr = d.prior + kPriorVals * k;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double h = J[a] * J[q] + J[3 + a] * J[3 + q] + J[6 + a] * J[6 + q];
        blkv[6 * a + q] += h;
        if (q == a) Dg[a] += h;
      }
      g[a] += J[a] * e[0] + J[3 + a] * e[1] + J[6 + a] * e[2];
      const double it = pr[15 + a];
      blkv[6 * (3 + a) + 3 + a] += it * it;
      Dg[3 + a] += it * it;
      g[3 + a] += it * e[3 + a];
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      Dg[a] = clampd(Dg[a]);
      blkv[7 * a] += lambda * Dg[a];
      gv[col + a] = g[a];
      Dv[col + a] = Dg[a];
      rr[a] = -g[a] + rr[a];
      xr[a] = 0.0;
    }
    float* A32 = d.Sblk32 + kSbVals * (size_t)brow[f];
#pragma unroll
    for (int i = 0; i < 36; ++i) {
      Ab[kSbRow * (i / 6) + i % 6] = blkv[i];
      A32[kSbRow * (i / 6) + i % 6] = (float)blkv[i];
    }
    double li[36];
    if (!chol6_inv(blkv, li)) fails = 1.0;
    double* L = Lf + 21 * tid;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int cc = 0; cc <= i; ++cc) L[i * (i + 1) / 2 + cc] = li[6 * i + cc];
    double z[6];
    pcg_precond(L, rr, z);
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      zg[col + a] = z[a];
      part_rr = fm(rr[a], rr[a], part_rr);
      part_rz = fm(rr[a], z[a], part_rz);
    }
  }
  // this workgroup's blocks into LDS (their diagonal blocks as just damped)
  __syncthreads();
  if (mixed) {
    const float4* src = reinterpret_cast<const float4*>(d.Sblk32 + kSbVals * (size_t)k0);
    float4* dst = reinterpret_cast<float4*>(sv);
    for (int i = tid; i < nblk * kSbVals / 4; i += kCgThreads) dst[i] = src[i];
  } else {
    const double2* src = reinterpret_cast<const double2*>(d.Sblk + kSbVals * (size_t)k0);
    double2* dst = reinterpret_cast<double2*>(sv);
    for (int i = tid; i < nblk * kSbVals / 2; i += kCgThreads) dst[i] = src[i];
  }
  {
    const double2 t = wg_sum2(part_rr, part_rz, red, tid);
    const double fl = wg_sum2(fails, 0.0, red, tid).x;
    if (tid == 0) {
      part[wg] = t;
      part[kMaxCgWG + wg] = make_double2(fl, 0.0);
    }
  }
  grid.sync();
  const double2 s0 = grid_sum2(part, G);
  const double nfail = grid_sum2(part + kMaxCgWG, G).x;
  if (nfail > 0.0 || c.point_fail) {
    if (wg == 0 && tid == 0) c.solve_ok = 0;
    return;
  }
  // this thread's halo entries of p (index, or -1), and p_0 = z_0 there
  const int nh6 = 6 * n_halo;
  int qh[kCgHalo];
#pragma unroll
  for (int u = 0; u < kCgHalo; ++u) {
    const int e = tid + u * kCgThreads;
    qh[u] = e < nh6 ? 6 * hcol[e / 6] + e % 6 : -1;
    if (qh[u] >= 0) {
      const double v = zg[qh[u]];
      pl[qh[u]] = v;
      if (mixed) p32l[kSbRow * (qh[u] / 6) + qh[u] % 6] = (float)v;
    }
  }
  const double bnorm = sqrt(s0.x);
  const int max_it = d.pcg_max_iters;
  // Forcing term of the inexact step: |r| <= eta |b| with
  // eta = min(pcg_tol, sqrt(|b| / |b_0|)), |b_0| the first solve's right-hand
  // side: the inexact-Newton choice that keeps superlinear local convergence
  // while the early steps stay cheap.
  const double b0 = c.cg_b0 > 0.0 ? c.cg_b0 : bnorm;
  const double tol = b0 > 0.0 ? fmin(d.pcg_tol, sqrt(bnorm / b0)) : d.pcg_tol;
  const unsigned base = bar_base;
  bool good = true;
  int it = 0;
  for (; it < max_it && bnorm > 0.0;) {
    __syncthreads();
    // q = S p for this workgroup's rows
    if (mixed) cg_spmv<float, kSbRow>(S32l, brl, bcl, nr, spt, p32l, Apl, tid);
    else cg_spmv<double, 6>(S64l, brl, bcl, nr, spt, pl, Apl, tid);
    __syncthreads();
    // owners (wavefront 0): z = M^-1 r, u = M^-1 q, their rows of (z, u),
    // their parts of p.q, r.q, q.q, q.z, q.u, r.r, r.z summed over the wavefront
    double2* zub = zug + (size_t)(it & 1) * m;
    double* pb = cgp + (size_t)(it & 1) * kMaxCgWG * kCgPartStride;
    double pown[6], qown[6];
    if (tid < kWave) {
      double sums[kCgSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (own) {
        const int col = 6 * (r0 + tid);
        double u[6], z[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          qown[a] = Apl[6 * tid + a];
          pown[a] = pl[col + a];
        }
        pcg_precond(Lf + 21 * tid, qown, u);
        pcg_precond(Lf + 21 * tid, rr, z);
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          zub[col + a] = make_double2(z[a], u[a]);
          sums[0] = fm(pown[a], qown[a], sums[0]);
          sums[1] = fm(rr[a], qown[a], sums[1]);
          sums[2] = fm(qown[a], qown[a], sums[2]);
          sums[3] = fm(qown[a], z[a], sums[3]);
          sums[4] = fm(qown[a], u[a], sums[4]);
          sums[5] = fm(rr[a], rr[a], sums[5]);
          sums[6] = fm(rr[a], z[a], sums[6]);
        }
      }
#pragma unroll
      for (int i = 0; i < kCgSums; ++i) sums[i] = wave_sum(sums[i]);
      if (lane == 0) {
        double2* dst = reinterpret_cast<double2*>(pb + kCgPartStride * wg);
        dst[0] = make_double2(sums[0], sums[1]);
        dst[1] = make_double2(sums[2], sums[3]);
        dst[2] = make_double2(sums[4], sums[5]);
        dst[3] = make_double2(sums[6], 0.0);
      }
    }
    ++it;
    if (!cg_barrier(ctr, base + (unsigned)it * (unsigned)G, abort_word, &bar_ok)) {
      good = false;
      break;
    }
    // this thread's halo entries of (z, u), requested before the parts are added
    double2 zu[kCgHalo];
#pragma unroll
    for (int u = 0; u < kCgHalo; ++u) zu[u] = qh[u] >= 0 ? zub[qh[u]] : make_double2(0.0, 0.0);
    // every wavefront: the G parts, added by the same butterfly everywhere
    // (lane l takes parts l and l + 64)
    double t[kCgSums] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int h = 0; h < kMaxCgWG / kWave; ++h) {
      const int w = lane + h * kWave;
      if (w < G) {
        const double2* src = reinterpret_cast<const double2*>(pb + kCgPartStride * w);
        const double2 v0 = src[0], v1 = src[1], v2 = src[2], v3 = src[3];
        t[0] += v0.x;
        t[1] += v0.y;
        t[2] += v1.x;
        t[3] += v1.y;
        t[4] += v2.x;
        t[5] += v2.y;
        t[6] += v3.x;
      }
    }
#pragma unroll
    for (int i = 0; i < kCgSums; ++i) t[i] = wave_sum(t[i]);
    const double pAp = t[0], rz = t[6];
    if (!(pAp > 0.0) || !isfinite(pAp)) {
      good = false;
      break;
    }
    const double alpha = rz / pAp;
    const double rr_new = fmax(fm(alpha * alpha, t[2], fm(-2.0 * alpha, t[1], t[5])), 0.0);
    const double rz_new = fm(alpha * alpha, t[4], fm(-2.0 * alpha, t[3], rz));
    if (own) {
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        xr[a] = fm(alpha, pown[a], xr[a]);
        rr[a] = fm(-alpha, qown[a], rr[a]);
      }
    }
    if (sqrt(rr_new) <= tol * bnorm) break;
    const double beta = rz_new / rz;
    // the halo of the next p = (z - alpha u) + beta p, the same in every workgroup
#pragma unroll
    for (int u = 0; u < kCgHalo; ++u) {
      const int q = qh[u];
      if (q >= 0) {
        const double v = fm(beta, pl[q], fm(-alpha, zu[u].y, zu[u].x));
        pl[q] = v;
        if (mixed) p32l[kSbRow * (q / 6) + q % 6] = (float)v;
      }
    }
  }
  if (!good) {
    // the same decision in every workgroup (a failed pAp), or an abandoned wait
    if (tid == 0) c.solve_ok = 0;
    return;
  }
  // Solution, predicted camera-side reduction, trial cameras and their prior
  // cost: owners for their cameras, workgroup 0 copies the fixed ones.
  double part_pred = 0.0, pc = 0.0;
  const int nxt = 1 - cur;
  if (own) {
    const int col = 6 * (r0 + tid), k = own_cam[tid];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      d.dc[col + a] = xr[a];
      part_pred += xr[a] * (lambda * Dv[col + a] * xr[a] - gv[col + a]);
    }
    const double* cm = d.cam[cur] + kCamVals * k;
    double* cn = d.cam[nxt] + kCamVals * k;
    double E[9], cv[kCamVals];
    so3_exp(xr, E);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) cv[3 * i + j] = cm[3 * i] * E[j] + cm[3 * i + 1] * E[3 + j] + cm[3 * i + 2] * E[6 + j];
#pragma unroll
    for (int i = 0; i < 3; ++i) cv[9 + i] = cm[9 + i] + xr[3 + i];
#pragma unroll
    for (int i = 0; i < kCamVals; ++i) cn[i] = cv[i];
    double e[6], J[9];
    prior_terms(cv, d.prior + kPriorVals * k, e, J);
    pterm_store(d.pterm[nxt] + kPtermVals * k, e, J);
#pragma unroll
    for (int i = 0; i < 6; ++i) pc += e[i] * e[i];
  }
  if (wg == 0) {
    for (int k = tid; k < d.C; k += kCgThreads) {
      if (d.cam_col[k] >= 0) continue;
      const double* cm = d.cam[cur] + kCamVals * k;
      double* cn = d.cam[nxt] + kCamVals * k;
      for (int i = 0; i < kCamVals; ++i) cn[i] = cm[i];
    }
  }
  {
    const double2 t = wg_sum2(part_pred, pc, red, tid);
    if (tid == 0) part[wg] = t;
  }
  // every workgroup has passed the same `it` CG barriers
  if (!cg_barrier(ctr, base + (unsigned)(it + 1) * (unsigned)G, abort_word, &bar_ok)) {
    if (tid == 0) c.solve_ok = 0;
    return;
  }
  if (wg == 0 && tid == 0) {
    const double2 t = grid_sum2(part, G);
    c.pred_c = t.x;
    c.E_prior_trial = 0.5 * t.y;
    for (int q = 0; q < 5; ++q) c.k[nxt][q] = c.k[cur][q];
    c.cg_iters += it;
    if (!(c.cg_b0 > 0.0)) c.cg_b0 = bnorm;
  }
}

// ---- back-substitution, trial points and FP64 trial cost -------------------------

template <typename R, bool SC>
__global__ __launch_bounds__(kWG) void k_backsub(Batch bt) {
  const int bx = xcd_block();
  extern __shared__ __align__(16) unsigned char smem[];
  if (bt.n_act == 0) return;   // empty dispatch that only carries timing events
  const int si = __builtin_amdgcn_readfirstlane(find_slot(bt.wg_off, bt.n_act, bx));
  const int s = __builtin_amdgcn_readfirstlane(bt.act[si]);
  const int wgl = bx - bt.wg_off[si];
  const SlotDesc& d = bt.desc[s];
  const SlotCtl& c = bt.ctl[s];
  if (c.status != ST_RUNNING || !c.solve_ok || c.point_fail || (d.sc != 0) != SC) return;
  double* tcam = reinterpret_cast<double*>(smem);               // trial cameras FP64
  R* scam = reinterpret_cast<R*>(tcam + bt.max_C * kCamVals);  // current cameras
  R* sdc = scam + bt.max_C * kCamVals;                         // camera update
  int* scol = reinterpret_cast<int*>(sdc + bt.max_m + 2);
  const int cur = c.cur, nxt = 1 - cur;
  for (int i = threadIdx.x; i < d.C * kCamVals; i += kWG) {
    tcam[i] = d.cam[nxt][i];
    scam[i] = (R)d.cam[cur][i];
  }
  for (int i = threadIdx.x; i < d.m; i += kWG) sdc[i] = (R)d.dc[i];
  for (int i = threadIdx.x; i < d.C; i += kWG) scol[i] = d.cam_col[i];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave), lane = threadIdx.x % kWave;
  const double lambda = c.lambda;
  const R f = SC ? (R)c.k[cur][2] : (R)d.f, is = (R)d.inv_sigma, dt = (R)d.huber_dt;
  const R k1 = (R)c.k[cur][0], k2 = (R)c.k[cur][1];
  const R cxo = SC ? (R)c.k[cur][3] : R(0), cyo = SC ? (R)c.k[cur][4] : R(0);
  const double* tki = c.k[nxt];   // trial intrinsics
  constexpr int NK = kNk<SC>;
  R dk[NK];   // intrinsic update (0 for fixed intrinsics)
#pragma unroll
  for (int t = 0; t < NK; ++t) dk[t] = d.kcolt[t] >= 0 ? sdc[d.kcolt[t]] : R(0);
  const gptr<const R> ptv = gmem(reinterpret_cast<const R*>(d.ptv)), ptd = gmem(reinterpret_cast<const R*>(d.ptd));
  const gptr<const int> ocam = gmem(d.ob_cam);
  const gptr<const double> Xc = gmem((const double*)d.X[cur]), uv64 = gmem((const double*)d.ob_uv64);
  const gptr<double> Xn64 = gmem(d.X[nxt]);
  const gptr<float> Xn32 = gmem(d.X32[nxt]);
  double rho_sum = 0.0, pred_sum = 0.0;
  int bad = 0;
  const int c0 = d.wg_chunk[wgl], c1 = d.wg_chunk[wgl + 1];
  // one lane per point of a chunk: its observations twice, first for
  // t = sum_obs W^T dc (FP32), then for the FP64 trial residuals at the moved
  // point.  Padding lanes read the chunk's first point and the padding
  // lanes' camera 0 and pixel 0, and do not use them.
  for (int ch = c0 + wave; ch < c1; ch += kWavesPerWG) {
    const int4 pc = d.pchunk[ch];
    const int n = pc.y;
    const bool valid = lane < pc.w;
    const int pt = pc.z + (valid ? lane : 0);
    // The FP64 point and pixel serve both models: their FP32 shadows are these
    // values rounded, so they are not read again.
    const double Xr[3] = {Xc[3 * pt], Xc[3 * pt + 1], Xc[3 * pt + 2]};
    R pv[12], dv[4];
    rec_load<sizeof(R) == 8 ? 10 : 12>(ptv + kPtVals * (size_t)pt, pv);
    rec_load<4>(ptd + 4 * (size_t)pt, dv);
    const double Xd[3] = {valid ? Xr[0] : 0.0, valid ? Xr[1] : 0.0, valid ? Xr[2] : 0.0};
    const R X0 = (R)Xd[0], X1 = (R)Xd[1], X2 = (R)Xd[2];
    int idx = pc.x + lane;
    int cam_n = ocam[idx];
    double u_n = uv64[2 * idx], v_n = uv64[2 * idx + 1];
    R ts[3] = {0, 0, 0};
    for (int t = 0; t < n; ++t) {
      const int cam = cam_n;
      const double ud = valid ? u_n : 0.0, vd = valid ? v_n : 0.0;
      if (t + 1 < n) {
        idx += kWave;
        cam_n = ocam[idx];
        u_n = uv64[2 * idx];
        v_n = uv64[2 * idx + 1];
      }
      const R u = (R)ud, v = (R)vd;
      ObsJ<R, NK> o;
      obs_model<R, SC>(scam + kCamVals * cam, X0, X1, X2, u, v, f, k1, k2, is, dt, valid, o, cxo, cyo);
      const int fi = valid ? scol[cam] : -1;
      // t = W_c^T dc + W_i^T dk, with W = w J_side^T J_p
      R jd[2] = {0, 0};   // J_side * d (2-vector)
      if (fi >= 0) {
#pragma unroll
        for (int r = 0; r < 6; ++r) {
          jd[0] = fm(jc(o, 0, r), sdc[fi + r], jd[0]);
          jd[1] = fm(jc(o, 1, r), sdc[fi + r], jd[1]);
        }
      }
      if constexpr (SC) {
#pragma unroll
        for (int q = NK - 1; q >= 0; --q) {
          jd[0] = fm(o.Jk[0][q], dk[q], jd[0]);
          jd[1] = fm(o.Jk[1][q], dk[q], jd[1]);
        }
      } else {
        jd[0] = fm(o.Jk[0][0], dk[0], fm(o.Jk[0][1], dk[1], jd[0]));
        jd[1] = fm(o.Jk[1][0], dk[0], fm(o.Jk[1][1], dk[1], jd[1]));
      }
      // the point's sum, in camera order
#pragma unroll
      for (int q = 0; q < 3; ++q) ts[q] += o.w * fm(o.Jp[0][q], jd[0], o.Jp[1][q] * jd[1]);
    }
    if (!valid) continue;
    double Xn[3];
    {
      const R* Q = pv;
      const R rr[3] = {-pv[6] - ts[0], -pv[7] - ts[1], -pv[8] - ts[2]};
      R dp[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) dp[q] = fm(qel(Q, q, 2), rr[2], fm(qel(Q, q, 1), rr[1], qel(Q, q, 0) * rr[0]));
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double dd = (double)dp[q];
        Xn[q] = Xd[q] + dd;
        pred_sum += dd * (lambda * (double)dv[q] * dd - (double)pv[6 + q]);
        Xn64[3 * pt + q] = Xn[q];
        Xn32[3 * pt + q] = (float)Xn[q];
      }
    }
    // the observations again (cached), the next one requested one ahead
    idx = pc.x + lane;
    cam_n = ocam[idx];
    u_n = uv64[2 * idx];
    v_n = uv64[2 * idx + 1];
    for (int t = 0; t < n; ++t) {
      const int cam = cam_n;
      const double u = u_n, v = v_n;
      if (t + 1 < n) {
        idx += kWave;
        cam_n = ocam[idx];
        u_n = uv64[2 * idx];
        v_n = uv64[2 * idx + 1];
      }
      double rho;
      if (obs_rho(tcam + kCamVals * cam, Xn, u, v, tki, d.inv_sigma, d.huber_dt, &rho)) rho_sum += rho;
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
  if (c.status != ST_RUNNING) return;
  // Workgroup parts of the trial cost: lane l sums parts l, l + 64, ... in
  // order, then a fixed xor tree (one wavefront; the same order in any batch).
  double rs = 0.0, ps = 0.0;
  int bad = 0;
  for (int w = threadIdx.x; w < d.n_wg; w += kWave) {
    rs += d.cost_part[2 * w];
    ps += d.cost_part[2 * w + 1];
    bad += d.bad_part[w];
  }
  rs = wave_sum(rs);
  ps = wave_sum(ps);
  bad = wave_sum(bad);
  if (threadIdx.x != 0) return;
  bool ok = c.solve_ok && !c.point_fail;
  double E2 = INFINITY, pred = 0.0, rho = -INFINITY;
  if (ok) {
    if (bad > 0) ok = false;
    E2 = 0.5 * rs + c.E_prior_trial;
    pred = 0.5 * (c.pred_c + ps);
    if (!isfinite(E2)) ok = false;
    if (ok && pred > 0.0) rho = (c.E - E2) / pred;
  }
  const bool accept = ok && rho > kAcceptRatio;
  d.lambda_log[c.iter] = c.lambda;
  d.acc_log[c.iter] = accept ? 1 : 0;
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

// ---- reprojection statistics of the exported state --------------------------------
//
// Sec. 3.3 and Table 1 report the mean and standard deviation of the
// reprojection error norm |p_kj - p^_kj| (pixels) over the observations.  One
// lane per observation at the current state in FP64; per workgroup the sums
// (observations, sum |e|, sum |e|^2, and the same over the inliers |e| <= 3
// delta) in a fixed order.  Observations at non-positive depth are not counted.

__global__ __launch_bounds__(kWG) void k_stats(Batch bt) {
  const int bx = xcd_block();
  extern __shared__ double sh_cam[];
  const int si = find_slot(bt.wg_off, bt.n_act, bx);
  const int s = bt.act[si];
  const int wgl = bx - bt.wg_off[si];
  const SlotDesc& d = bt.desc[s];
  const SlotCtl& c = bt.ctl[s];
  const int cur = c.cur;
  for (int i = threadIdx.x; i < d.C * kCamVals; i += kWG) sh_cam[i] = d.cam[cur][i];
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const double* ki = c.k[cur];
  const double lim = 3.0 * d.huber_dt / d.inv_sigma;   // 3 delta, pixels
  double acc[kStatVals] = {0, 0, 0, 0, 0, 0};
  for (int ch = d.wg_chunk[wgl] + wave; ch < d.wg_chunk[wgl + 1]; ch += kWavesPerWG) {
    const int4 pc = d.pchunk[ch];
    if (lane >= pc.w) continue;
    const int pt = pc.z + lane;
    const double X[3] = {d.X[cur][3 * pt], d.X[cur][3 * pt + 1], d.X[cur][3 * pt + 2]};
    for (int t = 0; t < pc.y; ++t) {
      const int idx = pc.x + t * kWave + lane;
      const double* cam = sh_cam + kCamVals * d.ob_cam[idx];
      const double d0 = X[0] - cam[9], d1 = X[1] - cam[10], d2 = X[2] - cam[11];
      const double x = cam[0] * d0 + cam[3] * d1 + cam[6] * d2;
      const double y = cam[1] * d0 + cam[4] * d1 + cam[7] * d2;
      const double z = cam[2] * d0 + cam[5] * d1 + cam[8] * d2;
      if (!(z > 0.0)) continue;
      const double a = x / z, b = y / z, r2 = a * a + b * b;
      const double D = 1.0 + ki[0] * r2 + ki[1] * r2 * r2;
      const double ex = ki[2] * D * a + ki[3] - d.ob_uv64[2 * idx];
      const double ey = ki[2] * D * b + ki[4] - d.ob_uv64[2 * idx + 1];
      const double e2 = ex * ex + ey * ey, e = sqrt(e2);
      acc[0] += 1.0;
      acc[1] += e;
      acc[2] += e2;
      if (e <= lim) {
        acc[3] += 1.0;
        acc[4] += e;
        acc[5] += e2;
      }
    }
  }
  __shared__ double red[kWavesPerWG][kStatVals];
#pragma unroll
  for (int t = 0; t < kStatVals; ++t) {
    const double v = wave_sum(acc[t]);
    if (lane == 0) red[wave][t] = v;
  }
  __syncthreads();
  if (threadIdx.x < kStatVals) {
    double v = 0.0;
    for (int w = 0; w < kWavesPerWG; ++w) v += red[w][threadIdx.x];
    d.stat_part[kStatVals * (size_t)wgl + threadIdx.x] = v;
  }
}

// ---- export: undo the origin shift --------------------------------------------------

__global__ void k_export(Batch bt) {
  const int s = bt.act[blockIdx.y];
  const SlotDesc& d = bt.desc[s];
  const SlotCtl& c = bt.ctl[s];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int cur = c.cur;
  if (i < d.P) {
    const int o = d.pt_orig[i];
    for (int t = 0; t < 3; ++t) d.out[12 * d.C + 3 * o + t] = d.X[cur][3 * i + t] + c.origin[t];
  }
  if (i < d.C) {
    const double* cm = d.cam[cur] + kCamVals * i;
    for (int t = 0; t < 9; ++t) d.out[9 * i + t] = cm[t];
    for (int t = 0; t < 3; ++t) d.out[9 * d.C + 3 * i + t] = cm[9 + t] + c.origin[t];
  }
  if (i < kStatVals) {   // the workgroups' reprojection sums, in workgroup order
    double v = 0.0;
    for (int w = 0; w < d.n_wg; ++w) v += d.stat_part[kStatVals * (size_t)w + i];
    d.out[12 * d.C + 3 * d.P + 5 + i] = v;
  }
  if (i == 0) {
    d.out[12 * d.C + 3 * d.P] = c.k[cur][0];
    d.out[12 * d.C + 3 * d.P + 1] = c.k[cur][1];
    d.out[12 * d.C + 3 * d.P + 2] = c.k[cur][2];
    d.out[12 * d.C + 3 * d.P + 3] = d.cx + c.k[cur][3];
    d.out[12 * d.C + 3 * d.P + 4] = d.cy + c.k[cur][4];
  }
}

template <typename R, bool SC>
size_t point_smem(const Batch& b) {
  return sizeof(R) * (size_t)b.max_C * kCamVals;
}

template <typename R>
size_t backsub_smem(const Batch& b) {
  return sizeof(double) * (size_t)b.max_C * kCamVals + sizeof(R) * ((size_t)b.max_C * kCamVals + (size_t)b.max_m + 2) +
         sizeof(int) * (size_t)b.max_C;
}


size_t solve_smem(const Batch& b) {
  const size_t nb = (size_t)b.max_nb, blk = nb * (nb + 1) / 2 * kTbV;
  return sizeof(double) * (solve_lds_base(b.max_nb) + (solve_lds_copy(b.max_nb) ? blk : 0));
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

hipError_t launch_prep(const Batch& b, int max_P_L, int max_rin, hipStream_t st) {
  if (b.n_act == 0) return hipSuccess;
  if (max_rin > 0) hipLaunchKernelGGL(k_res_gather, dim3((max_rin + 255) / 256, b.n_act), dim3(256), 0, st, b);
  hipLaunchKernelGGL(k_prep_slot, dim3(b.n_act), dim3(64), 0, st, b);
  if (max_P_L > 0) hipLaunchKernelGGL(k_prep_points, dim3((max_P_L + 255) / 256, b.n_act), dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_initial_cost(const Batch& b, hipStream_t st) {
  if (b.n_act == 0) return hipSuccess;
  if (b.total_wg > 0) {
    const size_t sc = sizeof(double) * b.max_C * kCamVals;
    hipError_t e = ensure_smem((const void*)k_cost0, sc);
    if (e) return e;
    hipLaunchKernelGGL(k_cost0, dim3(b.total_wg), dim3(kWG), sc, st, b);
  }
  hipLaunchKernelGGL(k_init, dim3(b.n_act), dim3(64), 0, st, b);
  return hipGetLastError();
}

// Launches one kernel; with events, the dispatch itself records the kernel's
// start and end (hipExtLaunchKernelGGL), so the measured time is the kernel's.
template <typename K>
void launch(K kernel, dim3 grid, dim3 block, size_t smem, hipStream_t st, hipEvent_t* ev, int slot, const Batch& b) {
  if (ev) hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)smem, st, ev[2 * slot], ev[2 * slot + 1], 0, b);
  else hipLaunchKernelGGL(kernel, grid, block, smem, st, b);
}

// Launches the ordinary instantiation of a kernel and, when `sc`, the
// self-calibrating one right after it (each skips the other kind of cluster).
// With events, the slot spans both: the first dispatch records the start, the
// last the end.
template <typename K1, typename K2>
void launch_both(K1 k1, K2 k2, bool sc, dim3 grid, dim3 block, size_t smem1, size_t smem2, hipStream_t st,
                 hipEvent_t* ev, int slot, const Batch& b) {
  if (!sc) return launch(k1, grid, block, smem1, st, ev, slot, b);
  if (!ev) {
    hipLaunchKernelGGL(k1, grid, block, smem1, st, b);
    hipLaunchKernelGGL(k2, grid, block, smem2, st, b);
    return;
  }
  hipExtLaunchKernelGGL(k1, grid, block, (uint32_t)smem1, st, ev[2 * slot], nullptr, 0, b);
  hipExtLaunchKernelGGL(k2, grid, block, (uint32_t)smem2, st, nullptr, ev[2 * slot + 1], 0, b);
}

size_t pcg_lds_bytes(size_t block_bytes, int m, int F, int rows_max) {
  return (block_bytes + 7) / 8 * 8 + sizeof(double) * ((size_t)m + 4 * (size_t)F + 27 * (size_t)rows_max);
}

hipError_t launch_iteration(const Batch& b, bool mixed, hipStream_t st, hipEvent_t* ev_all, int timed,
                            const SparseLaunch* spl, int n_sp) {
  if (b.n_act == 0) return hipSuccess;
  hipError_t e;
  const size_t s_solve = solve_smem(b);
  if ((e = ensure_smem((const void*)k_solve, s_solve))) return e;
  const size_t sp = mixed ? point_smem<float, false>(b) : point_smem<double, false>(b);
  const size_t sps = mixed ? point_smem<float, true>(b) : point_smem<double, true>(b);
  const size_t sb = mixed ? backsub_smem<float>(b) : backsub_smem<double>(b);
  {
    const void* fn[4] = {mixed ? (const void*)k_backsub<float, false> : (const void*)k_backsub<double, false>,
                         mixed ? (const void*)k_backsub<float, true> : (const void*)k_backsub<double, true>,
                         mixed ? (const void*)k_point<float, false> : (const void*)k_point<double, false>,
                         mixed ? (const void*)k_point<float, true> : (const void*)k_point<double, true>};
    for (int i = 0; i < 4; ++i)
      if ((i & 1) == 0 || b.any_sc)
        if ((e = ensure_smem(fn[i], i < 2 ? sb : (i == 2 ? sp : sps)))) return e;
  }
  // Events of kernel slot k, or none when it is not timed.
  auto evk = [&](int k) { return (ev_all && ((timed >> k) & 1)) ? ev_all : nullptr; };
  // Every timed kernel needs a dispatch to carry its events, also when a
  // batch has no work for it: a one-block launch that returns at once.
  // Self-calibrating clusters run in a second launch of the same kernel
  // (launch_both); a slot's events then span the two launches.
  const dim3 g_pt(b.total_wg > 0 ? b.total_wg : 1), g_tg(b.total_tg > 0 ? b.total_tg : 1);
  Batch nob = b;
  nob.n_act = 0;
  const bool sc = b.any_sc != 0;
  if (b.total_wg > 0 || evk(0)) {
    const Batch& bb = b.total_wg > 0 ? b : nob;
    const bool s2 = sc && b.total_wg > 0;
    if (mixed) launch_both(k_point<float, false>, k_point<float, true>, s2, g_pt, dim3(kWG), sp, sps, st, evk(0), 0, bb);
    else launch_both(k_point<double, false>, k_point<double, true>, s2, g_pt, dim3(kWG), sp, sps, st, evk(0), 0, bb);
  }
  if (mixed) {
    // camera and pair tasks in one launch (slot 1); slot 2 marks an empty interval
    const int nwg = b.total_tkc_wg + b.total_tkp_wg;
    if (nwg > 0 || evk(1))
      launch_both(k_blocks<float, false>, k_blocks<float, true>, sc && nwg > 0, dim3(nwg > 0 ? nwg : 1), dim3(kWG), 0,
                  0, st, evk(1), 1, nwg > 0 ? b : nob);
    if (evk(2) && ((e = hipEventRecord(ev_all[4], st)) || (e = hipEventRecord(ev_all[5], st)))) return e;
  } else {
    if (b.total_tkc_wg > 0 || evk(1)) {
      const int n = b.total_tkc_wg;
      launch_both(k_camblk<double, false>, k_camblk<double, true>, sc && n > 0, dim3(n > 0 ? n : 1), dim3(kWG), 0, 0,
                  st, evk(1), 1, n > 0 ? b : nob);
    }
    if (b.total_tkp_wg > 0 || evk(2)) {
      const int n = b.total_tkp_wg;
      launch_both(k_pairblk<double, false>, k_pairblk<double, true>, sc && n > 0, dim3(n > 0 ? n : 1), dim3(kWG), 0,
                  0, st, evk(2), 2, n > 0 ? b : nob);
    }
  }
  if (b.total_tg > 0 || evk(3)) {
    const Batch& bb = b.total_tg > 0 ? b : nob;
    if (mixed) launch(k_reduce<float>, g_tg, dim3(kReduceThreads), 0, st, evk(3), 3, bb);
    else launch(k_reduce<double>, g_tg, dim3(kReduceThreads), 0, st, evk(3), 3, bb);
  }
  // A solver with no cluster in the batch is not launched; with timing on, its
  // events mark an empty interval.
  if (b.any_dense) launch(k_solve, dim3(b.n_act), dim3(kSolveWG), s_solve, st, evk(4), 4, b);
  else if (evk(4) && ((e = hipEventRecord(ev_all[8], st)) || (e = hipEventRecord(ev_all[9], st)))) return e;
  // conjugate gradients: one cooperative launch per such cluster (its
  // workgroups meet at grid barriers); timed from before the first to after
  // the last
  if (evk(7) && (e = hipEventRecord(ev_all[14], st))) return e;
  for (int i = 0; i < n_sp; ++i) {
    if ((e = ensure_smem((const void*)k_pcg, (size_t)spl[i].smem))) return e;
    int slot = spl[i].slot;
    Batch bb = b;
    void* args[] = {&bb, &slot};
    if ((e = hipLaunchCooperativeKernel((const void*)k_pcg, dim3(spl[i].G), dim3(kCgThreads), args,
                                        (unsigned)spl[i].smem, st)))
      return e;
  }
  if (evk(7) && (e = hipEventRecord(ev_all[15], st))) return e;
  if (b.total_wg > 0 || evk(5)) {
    const Batch& bb = b.total_wg > 0 ? b : nob;
    const bool s2 = sc && b.total_wg > 0;
    if (mixed) launch_both(k_backsub<float, false>, k_backsub<float, true>, s2, g_pt, dim3(kWG), sb, sb, st, evk(5), 5, bb);
    else launch_both(k_backsub<double, false>, k_backsub<double, true>, s2, g_pt, dim3(kWG), sb, sb, st, evk(5), 5, bb);
  }
  launch(k_lm, dim3(b.n_act), dim3(64), 0, st, evk(6), 6, b);
  return hipGetLastError();
}

hipError_t launch_writeback(const Batch& b, int max_rout, hipStream_t st) {
  if (b.n_act == 0 || max_rout <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_res_scatter, dim3((max_rout + 255) / 256, b.n_act), dim3(256), 0, st, b);
  return hipGetLastError();
}

hipError_t launch_export(const Batch& b, int max_P, hipStream_t st) {
  if (b.n_act == 0) return hipSuccess;
  if (b.total_wg > 0) {
    const size_t sc = sizeof(double) * b.max_C * kCamVals;
    hipError_t e = ensure_smem((const void*)k_stats, sc);
    if (e) return e;
    hipLaunchKernelGGL(k_stats, dim3(b.total_wg), dim3(kWG), sc, st, b);
  }
  int n = max_P > b.max_C ? max_P : (b.max_C > 0 ? b.max_C : 1);
  if (n < kStatVals) n = kStatVals;
  hipLaunchKernelGGL(k_export, dim3((n + 255) / 256, b.n_act), dim3(256), 0, st, b);
  return hipGetLastError();
}

}  // namespace bagpu
