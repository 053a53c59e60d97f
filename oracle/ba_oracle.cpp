// FP64 CPU oracle for cluster bundle adjustment.
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
// benchmark's CPU-baseline leg load this library.  It shares no code, header,
// constant or helper with the HIP library; the product path never calls it.
//
// What it computes (paper: "Real-Time Bundle Adjustment for Ultra-High-
// Resolution UAV Imagery Using Adaptive Patch-Based Feature Tracking",
// Sec. 3.2):
//   * the reprojection of tie point X_j in image I_k, Eq. (5):
//       p_kj = pi(K R_k^T (X_j - T_k)),  pi(x, y, z) = (x/z, y/z)  (Eq. 3 notes),
//     with R_k camera->world and T_k the projection centre (the conventions
//     Eq. (3) uses when it back-projects with R_0 K^-1 and adds T_0), extended
//     by the Brown radial terms k1, k2 on the normalised coordinates;
//   * the robust cluster cost of Eq. (7) (same form as Eq. (6)), with rho the
//     Huber function acting on the squared norm of the 2-vector residual, the
//     residual whitened by sigma_px, plus GNSS/IMU pose-prior terms on the
//     navigation-derived initial poses T_k^(0), R_k^(0) (Sec. 3.2), and a 1/2
//     factor that leaves the minimiser unchanged;
//   * its minimisation by Levenberg-Marquardt (IRLS Gauss-Newton normal
//     equations, Marquardt diagonal scaling, Nielsen damping update), with the
//     damped normal equations solved by eliminating the points (Schur
//     complement on the reduced camera system), a dense Cholesky of that
//     system and point back-substitution.  The paper names no optimiser; these
//     are readings of the method, held identical on both implementations.
//   * images whose poses are held fixed (the first half of the inter-cluster
//     overlap, Sec. 3.2) carry no unknowns.
//
// Unknown ordering: for each free camera in camera order (omega[3], T[3]),
// then the estimated intrinsics of the cluster in the order k1 (bit 0 of
// intr_mask), k2 (bit 1), f (bit 2), cx (bit 3), cy (bit 4) -- f, cx, cy being
// the focal length and principal point of K, the k1, k2 the radial terms --
// then the points (X, Y, Z) in point order.  The intrinsic state is the
// vector k[5] = (k1, k2, f, cx, cy).  Rotation update: R <- R Exp(domega).
//
// Everything is plain loops in double precision; no blocking, fusion or
// reordering beyond the textbook definitions.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace {

struct OrScene {                 // mirrored field by field in oracle/__init__.py
  int32_t n_cams, n_points, n_obs;
  int32_t intr_mask;
  const int32_t* obs_cam;        // [O]
  const int32_t* obs_pt;         // [O]
  const double* obs_uv;          // [2O] pixel, corner origin
  const double* prior_R;         // [9C] row-major
  const double* prior_T;         // [3C]
  const double* prior_sigma;     // [6C] sigma_omega[3] (rad), sigma_T[3] (m); <=0 or inf: off
  const uint8_t* fixed;          // [C]
  double f, cx, cy;
  double sigma_px, huber_delta;
};

struct OrOptions {
  int32_t max_iters;
  int32_t stop_on_ftol;          // 0: run exactly max_iters iterations
  double lambda0;
  double ftol;
};

struct OrStats {
  int32_t iterations, accepted, rejected, status;   // status 0 max-iters, 1 converged, 2 stalled
  double lambda, nu;
};

const double kInf = std::numeric_limits<double>::infinity();
const double kLambdaMin = 1e-16, kLambdaMax = 1e32;
const double kDiagMin = 1e-6, kDiagMax = 1e32;
const double kAcceptRatio = 1e-3;

// ---- SO(3) ---------------------------------------------------------------

void skew(const double w[3], double K[9]) {
  K[0] = 0;     K[1] = -w[2]; K[2] = w[1];
  K[3] = w[2];  K[4] = 0;     K[5] = -w[0];
  K[6] = -w[1]; K[7] = w[0];  K[8] = 0;
}

void matmul3(const double A[9], const double B[9], double C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}

// Exp of a rotation vector (Rodrigues; second-order series for tiny angles).
void so3_exp(const double w[3], double R[9]) {
  double th = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  double K[9], K2[9];
  skew(w, K);
  matmul3(K, K, K2);
  double a, b;
  if (th < 1e-8) { a = 1.0; b = 0.5; }
  else { a = std::sin(th) / th; b = (1.0 - std::cos(th)) / (th * th); }
  for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0 ? 1.0 : 0.0) + a * K[i] + b * K2[i];
}

// Log of a rotation matrix, returned as a rotation vector.
void so3_log(const double R[9], double w[3]) {
  double tr = R[0] + R[4] + R[8];
  double c = 0.5 * (tr - 1.0);
  if (c > 1.0) c = 1.0;
  if (c < -1.0) c = -1.0;
  double th = std::acos(c);
  double v[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};   // 2 sin(th) * axis
  if (th < 1e-6) {
    double s = 0.5 * (1.0 + th * th / 6.0);
    for (int i = 0; i < 3; ++i) w[i] = s * v[i];
  } else if (th < M_PI - 1e-6) {
    double s = th / (2.0 * std::sin(th));
    for (int i = 0; i < 3; ++i) w[i] = s * v[i];
  } else {
    // Near pi: axis from the largest diagonal entry of (R + I) / 2 = a a^T.
    int k = 0;
    if (R[4] > R[k * 4]) k = 1;
    if (R[8] > R[k * 4]) k = 2;
    double a[3];
    double d = std::sqrt(0.5 * (R[k * 4] + 1.0));
    for (int i = 0; i < 3; ++i) a[i] = (i == k) ? d : 0.5 * (R[3 * i + k] + R[3 * k + i]) / (2.0 * d);
    double n = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double sg = (a[0] * v[0] + a[1] * v[1] + a[2] * v[2]) < 0 ? -1.0 : 1.0;
    for (int i = 0; i < 3; ++i) w[i] = sg * th * a[i] / n;
  }
}

// Inverse right Jacobian of SO(3): d Log(Exp(phi) Exp(d)) / d d at d = 0.
void so3_jr_inv(const double phi[3], double J[9]) {
  double th = std::sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
  double K[9], K2[9];
  skew(phi, K);
  matmul3(K, K, K2);
  double c;
  if (th < 1e-4) c = 1.0 / 12.0 + th * th / 720.0;
  else c = 1.0 / (th * th) - (1.0 + std::cos(th)) / (2.0 * th * std::sin(th));
  for (int i = 0; i < 9; ++i) J[i] = (i % 4 == 0 ? 1.0 : 0.0) + 0.5 * K[i] + c * K2[i];
}

// ---- camera model (Eq. 5 with radial terms) ----------------------------

struct Proj {
  double xc[3];      // point in the camera frame
  double a, b, r2, D;
  double uv[2];      // predicted pixel
};

void project(const double R[9], const double T[3], const double X[3], double f, double cx,
             double cy, double k1, double k2, Proj& p) {
  double d[3] = {X[0] - T[0], X[1] - T[1], X[2] - T[2]};
  for (int i = 0; i < 3; ++i) p.xc[i] = R[0 + i] * d[0] + R[3 + i] * d[1] + R[6 + i] * d[2];  // R^T d
  p.a = p.xc[0] / p.xc[2];
  p.b = p.xc[1] / p.xc[2];
  p.r2 = p.a * p.a + p.b * p.b;
  p.D = 1.0 + k1 * p.r2 + k2 * p.r2 * p.r2;
  p.uv[0] = f * p.D * p.a + cx;
  p.uv[1] = f * p.D * p.b + cy;
}

// Huber on the squared whitened residual norm s; dt = delta / sigma.
double huber_rho(double s, double dt) { return s <= dt * dt ? s : 2.0 * dt * std::sqrt(s) - dt * dt; }
double huber_w(double s, double dt) { return s <= dt * dt ? 1.0 : dt / std::sqrt(s); }

// Jacobians of the predicted pixel (u, v) of one observation, row-major 2xN:
// Jk for (k1, k2), Ji for (f, cx, cy).
struct ObsJac {
  double Jw[6], JT[6], Jp[6], Jk[4], Ji[6];
};

void obs_jacobian(const double R[9], const Proj& p, double f, double k1, double k2, ObsJac& J) {
  const double a = p.a, b = p.b, z = p.xc[2];
  const double q = k1 + 2.0 * k2 * p.r2;
  // A = d(u,v)/d(a,b)
  const double A[4] = {f * (p.D + 2.0 * a * a * q), f * 2.0 * a * b * q,
                       f * 2.0 * a * b * q,         f * (p.D + 2.0 * b * b * q)};
  // B = d(a,b)/d xc = (1/z) [[1,0,-a],[0,1,-b]]
  const double B[6] = {1.0 / z, 0.0, -a / z, 0.0, 1.0 / z, -b / z};
  double Jx[6];   // d(u,v)/d xc = A B
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) Jx[3 * i + j] = A[2 * i + 0] * B[0 + j] + A[2 * i + 1] * B[3 + j];
  // d xc / d X = R^T  ->  Jp = Jx R^T ; d xc / d T = -R^T
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += Jx[3 * i + k] * R[3 * j + k];   // (R^T)[k][j] = R[j][k]
      J.Jp[3 * i + j] = s;
      J.JT[3 * i + j] = -s;
    }
  // Right perturbation R Exp(dw): xc -> Exp(-dw) xc, d xc / d dw = [xc]x
  double Kx[9];
  skew(p.xc, Kx);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += Jx[3 * i + k] * Kx[3 * k + j];
      J.Jw[3 * i + j] = s;
    }
  const double r4 = p.r2 * p.r2;
  J.Jk[0] = f * p.r2 * a; J.Jk[1] = f * r4 * a;
  J.Jk[2] = f * p.r2 * b; J.Jk[3] = f * r4 * b;
  // u = f D a + cx, v = f D b + cy
  J.Ji[0] = p.D * a; J.Ji[1] = 1.0; J.Ji[2] = 0.0;
  J.Ji[3] = p.D * b; J.Ji[4] = 0.0; J.Ji[5] = 1.0;
}

// project() with the intrinsic state k = (k1, k2, f, cx, cy)
void project_k(const double R[9], const double T[3], const double X[3], const double* k, Proj& p) {
  project(R, T, X, k[2], k[3], k[4], k[0], k[1], p);
}

double inv_sigma(double s) { return (s > 0.0 && std::isfinite(s)) ? 1.0 / s : 0.0; }

// Pose prior residual of camera k (whitened) and d e_omega / d domega.
void prior_residual(const OrScene& sc, int k, const double R[9], const double T[3], double e[6],
                    double Jw[9]) {
  const double* Rp = sc.prior_R + 9 * k;
  const double* Tp = sc.prior_T + 3 * k;
  const double* sg = sc.prior_sigma + 6 * k;
  double RtR[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int l = 0; l < 3; ++l) s += Rp[3 * l + i] * R[3 * l + j];
      RtR[3 * i + j] = s;
    }
  double phi[3];
  so3_log(RtR, phi);
  double Jr[9];
  so3_jr_inv(phi, Jr);
  for (int i = 0; i < 3; ++i) {
    double iw = inv_sigma(sg[i]), it = inv_sigma(sg[3 + i]);
    e[i] = phi[i] * iw;
    e[3 + i] = (T[i] - Tp[i]) * it;
    for (int j = 0; j < 3; ++j) Jw[3 * i + j] = Jr[3 * i + j] * iw;
  }
}

// ---- unknown layout ---------------------------------------------------------

struct Layout {
  std::vector<int> cam_col;   // first column of a free camera, -1 if fixed
  int n_free = 0, n_intr = 0, m = 0;
  int k_col[5] = {-1, -1, -1, -1, -1};
  long N = 0;
};

Layout make_layout(const OrScene& sc) {
  Layout L;
  L.cam_col.assign(sc.n_cams, -1);
  for (int k = 0; k < sc.n_cams; ++k)
    if (!sc.fixed[k]) L.cam_col[k] = 6 * L.n_free++;
  int c = 6 * L.n_free;
  for (int b = 0; b < 5; ++b)
    if (sc.intr_mask & (1 << b)) L.k_col[b] = c++;
  L.n_intr = c - 6 * L.n_free;
  L.m = c;
  L.N = (long)L.m + 3L * sc.n_points;
  return L;
}

// ---- cost ------------------------------------------------------------------

// E = 1/2 sum_obs rho(s) + 1/2 sum_free-cams |e_prior|^2 ; +inf if any depth <= 0.
double cost(const OrScene& sc, const double* R, const double* T, const double* X, const double* k) {
  const double dt = sc.huber_delta / sc.sigma_px;
  double E = 0.0;
  for (int o = 0; o < sc.n_obs; ++o) {
    const int c = sc.obs_cam[o], j = sc.obs_pt[o];
    Proj p;
    project_k(R + 9 * c, T + 3 * c, X + 3 * j, k, p);
    if (!(p.xc[2] > 0.0)) return kInf;
    double ex = (p.uv[0] - sc.obs_uv[2 * o]) / sc.sigma_px;
    double ey = (p.uv[1] - sc.obs_uv[2 * o + 1]) / sc.sigma_px;
    E += 0.5 * huber_rho(ex * ex + ey * ey, dt);
  }
  for (int c = 0; c < sc.n_cams; ++c) {
    if (sc.fixed[c]) continue;
    double e[6], Jw[9];
    prior_residual(sc, c, R + 9 * c, T + 3 * c, e, Jw);
    for (int i = 0; i < 6; ++i) E += 0.5 * e[i] * e[i];
  }
  return E;
}

// ---- dense Cholesky ----------------------------------------------------------

bool cholesky(std::vector<double>& A, int n) {       // in place, lower triangle
  for (int j = 0; j < n; ++j) {
    double d = A[(long)j * n + j];
    for (int k = 0; k < j; ++k) d -= A[(long)j * n + k] * A[(long)j * n + k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    d = std::sqrt(d);
    A[(long)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[(long)i * n + j];
      for (int k = 0; k < j; ++k) s -= A[(long)i * n + k] * A[(long)j * n + k];
      A[(long)i * n + j] = s / d;
    }
  }
  return true;
}

void cholesky_solve(const std::vector<double>& L, int n, std::vector<double>& x) {
  for (int i = 0; i < n; ++i) {
    double s = x[i];
    for (int k = 0; k < i; ++k) s -= L[(long)i * n + k] * x[k];
    x[i] = s / L[(long)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int k = i + 1; k < n; ++k) s -= L[(long)k * n + i] * x[k];
    x[i] = s / L[(long)i * n + i];
  }
}

// Inverse of a symmetric positive-definite 3x3 matrix via its Cholesky factor.
bool spd3_inverse(const double V[9], double Q[9]) {
  std::vector<double> L(V, V + 9);
  if (!cholesky(L, 3)) return false;
  for (int c = 0; c < 3; ++c) {
    std::vector<double> x(3, 0.0);
    x[c] = 1.0;
    cholesky_solve(L, 3, x);
    for (int r = 0; r < 3; ++r) Q[3 * r + c] = x[r];
  }
  return true;
}

double clamp_diag(double d) { return d < kDiagMin ? kDiagMin : (d > kDiagMax ? kDiagMax : d); }

// ---- one damped Gauss-Newton step by Schur complement -----------------------
//
// Builds, at the current state, the IRLS normal equations
//   H = sum w J~^T J~ + sum Jpr^T Jpr ,  g = sum w J~^T e~ + sum Jpr^T epr,
// with J~ = J / sigma_px, e~ = e / sigma_px, w = rho'(s), partitioned as
//   [ U   W ] [dc]   [-gc]
//   [ W^T V ] [dp] = [-gp]
// and solves (H + lambda D) delta = -g, D = clamp(diag H), by
//   S = U_l - W V_l^-1 W^T,  b = -gc + W V_l^-1 gp,  S dc = b,
//   dp_j = V_l,j^-1 (-gp_j - W_j^T dc).
// Returns 0 on success, 1 when a pivot of S or of a point block is not
// positive.  pred = 1/2 delta^T (lambda D delta - g).
int schur_step(const OrScene& sc, const Layout& L, const double* R, const double* T,
               const double* X, const double* k, double lambda, double* delta, double* pred) {
  const int O = sc.n_obs, P = sc.n_points, m = L.m;
  const double is = 1.0 / sc.sigma_px, dt = sc.huber_delta / sc.sigma_px;

  std::vector<double> U((long)m * m, 0.0), gc(m, 0.0);
  std::vector<double> V(9L * P, 0.0), gp(3L * P, 0.0);
  constexpr int NR = 11;                    // camera-side rows: omega, T, k1, k2, f, cx, cy
  std::vector<double> Wo(3L * NR * O, 0.0); // per observation: NR camera-side rows x 3
  std::vector<int> idx((long)NR * O, -1);   // global column of each camera-side row

  for (int o = 0; o < O; ++o) {
    const int c = sc.obs_cam[o], j = sc.obs_pt[o];
    Proj p;
    project_k(R + 9 * c, T + 3 * c, X + 3 * j, k, p);
    if (!(p.xc[2] > 0.0)) return 1;
    ObsJac J;
    obs_jacobian(R + 9 * c, p, k[2], k[0], k[1], J);
    double e[2] = {(p.uv[0] - sc.obs_uv[2 * o]) * is, (p.uv[1] - sc.obs_uv[2 * o + 1]) * is};
    const double w = huber_w(e[0] * e[0] + e[1] * e[1], dt);
    // Camera-side Jacobian A (2 x NR) (columns absent -> idx -1).
    double A[2][NR];
    for (int i = 0; i < 2; ++i) {
      for (int t = 0; t < 3; ++t) { A[i][t] = J.Jw[3 * i + t] * is; A[i][3 + t] = J.JT[3 * i + t] * is; }
      A[i][6] = J.Jk[2 * i + 0] * is;
      A[i][7] = J.Jk[2 * i + 1] * is;
      for (int t = 0; t < 3; ++t) A[i][8 + t] = J.Ji[3 * i + t] * is;
    }
    int* id = &idx[(long)NR * o];
    if (L.cam_col[c] >= 0)
      for (int t = 0; t < 6; ++t) id[t] = L.cam_col[c] + t;
    for (int b = 0; b < 5; ++b) id[6 + b] = L.k_col[b];
    double Jp[2][3];
    for (int i = 0; i < 2; ++i)
      for (int t = 0; t < 3; ++t) Jp[i][t] = J.Jp[3 * i + t] * is;

    for (int r = 0; r < NR; ++r) {
      if (id[r] < 0) continue;
      for (int s = 0; s < NR; ++s) {
        if (id[s] < 0) continue;
        U[(long)id[r] * m + id[s]] += w * (A[0][r] * A[0][s] + A[1][r] * A[1][s]);
      }
      gc[id[r]] += w * (A[0][r] * e[0] + A[1][r] * e[1]);
      for (int t = 0; t < 3; ++t) Wo[3L * NR * o + 3 * r + t] = w * (A[0][r] * Jp[0][t] + A[1][r] * Jp[1][t]);
    }
    for (int r = 0; r < 3; ++r) {
      for (int s = 0; s < 3; ++s) V[9L * j + 3 * r + s] += w * (Jp[0][r] * Jp[0][s] + Jp[1][r] * Jp[1][s]);
      gp[3L * j + r] += w * (Jp[0][r] * e[0] + Jp[1][r] * e[1]);
    }
  }
  // Pose priors of free cameras.
  for (int c = 0; c < sc.n_cams; ++c) {
    if (L.cam_col[c] < 0) continue;
    double e[6], Jw[9];
    prior_residual(sc, c, R + 9 * c, T + 3 * c, e, Jw);
    double Jpr[6][6] = {};
    for (int i = 0; i < 3; ++i) {
      for (int j = 0; j < 3; ++j) Jpr[i][j] = Jw[3 * i + j];
      Jpr[3 + i][3 + i] = inv_sigma(sc.prior_sigma[6 * c + 3 + i]);
    }
    const int c0 = L.cam_col[c];
    for (int r = 0; r < 6; ++r) {
      for (int s = 0; s < 6; ++s) {
        double h = 0;
        for (int i = 0; i < 6; ++i) h += Jpr[i][r] * Jpr[i][s];
        U[(long)(c0 + r) * m + c0 + s] += h;
      }
      double gg = 0;
      for (int i = 0; i < 6; ++i) gg += Jpr[i][r] * e[i];
      gc[c0 + r] += gg;
    }
  }

  // Observations of each point.
  std::vector<int> ptr(P + 1, 0), list(O);
  for (int o = 0; o < O; ++o) ptr[sc.obs_pt[o] + 1]++;
  for (int j = 0; j < P; ++j) ptr[j + 1] += ptr[j];
  {
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int o = 0; o < O; ++o) list[fill[sc.obs_pt[o]]++] = o;
  }

  // Damping and reduced camera system.
  std::vector<double> Dc(m), S((long)m * m), b(m);
  for (int r = 0; r < m; ++r) Dc[r] = clamp_diag(U[(long)r * m + r]);
  for (long i = 0; i < (long)m * m; ++i) S[i] = U[i];
  for (int r = 0; r < m; ++r) { S[(long)r * m + r] += lambda * Dc[r]; b[r] = -gc[r]; }

  std::vector<double> Q(9L * P), Dp(3L * P);
  for (int j = 0; j < P; ++j) {
    double Vl[9];
    for (int i = 0; i < 9; ++i) Vl[i] = V[9L * j + i];
    for (int t = 0; t < 3; ++t) {
      Dp[3L * j + t] = clamp_diag(V[9L * j + 4 * t]);
      Vl[4 * t] += lambda * Dp[3L * j + t];
    }
    if (!spd3_inverse(Vl, &Q[9L * j])) return 1;
    const double* Qj = &Q[9L * j];
    for (int ia = ptr[j]; ia < ptr[j + 1]; ++ia) {
      const int oa = list[ia];
      const double* Wa = &Wo[3L * NR * oa];
      const int* ida = &idx[(long)NR * oa];
      // Y = W_a Q
      double Y[NR][3];
      for (int r = 0; r < NR; ++r)
        for (int t = 0; t < 3; ++t) {
          double s = 0;
          for (int u = 0; u < 3; ++u) s += Wa[3 * r + u] * Qj[3 * u + t];
          Y[r][t] = s;
        }
      for (int r = 0; r < NR; ++r) {
        if (ida[r] < 0) continue;
        b[ida[r]] += Y[r][0] * gp[3L * j] + Y[r][1] * gp[3L * j + 1] + Y[r][2] * gp[3L * j + 2];
      }
      for (int ib = ptr[j]; ib < ptr[j + 1]; ++ib) {
        const int ob = list[ib];
        const double* Wb = &Wo[3L * NR * ob];
        const int* idb = &idx[(long)NR * ob];
        for (int r = 0; r < NR; ++r) {
          if (ida[r] < 0) continue;
          for (int s = 0; s < NR; ++s) {
            if (idb[s] < 0) continue;
            S[(long)ida[r] * m + idb[s]] -= Y[r][0] * Wb[3 * s] + Y[r][1] * Wb[3 * s + 1] + Y[r][2] * Wb[3 * s + 2];
          }
        }
      }
    }
  }

  std::vector<double> dc(b);
  if (m > 0) {
    std::vector<double> Lc(S);
    if (!cholesky(Lc, m)) return 1;
    cholesky_solve(Lc, m, dc);
  }

  double pr = 0.0;
  for (int r = 0; r < m; ++r) {
    delta[r] = dc[r];
    pr += dc[r] * (lambda * Dc[r] * dc[r] - gc[r]);
  }
  for (int j = 0; j < P; ++j) {
    double rhs[3] = {-gp[3L * j], -gp[3L * j + 1], -gp[3L * j + 2]};
    for (int ia = ptr[j]; ia < ptr[j + 1]; ++ia) {
      const int oa = list[ia];
      const double* Wa = &Wo[3L * NR * oa];
      const int* ida = &idx[(long)NR * oa];
      for (int r = 0; r < NR; ++r) {
        if (ida[r] < 0) continue;
        for (int t = 0; t < 3; ++t) rhs[t] -= Wa[3 * r + t] * dc[ida[r]];
      }
    }
    for (int t = 0; t < 3; ++t) {
      double d = Q[9L * j + 3 * t] * rhs[0] + Q[9L * j + 3 * t + 1] * rhs[1] + Q[9L * j + 3 * t + 2] * rhs[2];
      delta[m + 3L * j + t] = d;
      pr += d * (lambda * Dp[3L * j + t] * d - gp[3L * j + t]);
    }
  }
  *pred = 0.5 * pr;
  return 0;
}

// x' = x (+) delta
void apply_update(const OrScene& sc, const Layout& L, const double* R, const double* T,
                  const double* X, const double* k, const double* delta, double* R2, double* T2,
                  double* X2, double* k2) {
  for (int c = 0; c < sc.n_cams; ++c) {
    if (L.cam_col[c] < 0) {
      std::memcpy(R2 + 9 * c, R + 9 * c, 9 * sizeof(double));
      std::memcpy(T2 + 3 * c, T + 3 * c, 3 * sizeof(double));
      continue;
    }
    const double* d = delta + L.cam_col[c];
    double E[9];
    so3_exp(d, E);
    matmul3(R + 9 * c, E, R2 + 9 * c);
    for (int i = 0; i < 3; ++i) T2[3 * c + i] = T[3 * c + i] + d[3 + i];
  }
  for (int b = 0; b < 5; ++b) k2[b] = k[b] + (L.k_col[b] >= 0 ? delta[L.k_col[b]] : 0.0);
  for (long i = 0; i < 3L * sc.n_points; ++i) X2[i] = X[i] + delta[L.m + i];
}

}  // namespace

extern "C" {

// Predicted pixels uv[2O], depths z[O], whitened residuals e[2O], s[O], rho[O], w[O].
// Any output pointer may be NULL.  Returns the number of observations with z <= 0.
int or_residuals(const OrScene* sc, const double* R, const double* T, const double* X,
                 const double* k, double* uv, double* z, double* e, double* s, double* rho,
                 double* w) {
  const double dt = sc->huber_delta / sc->sigma_px;
  int bad = 0;
  for (int o = 0; o < sc->n_obs; ++o) {
    const int c = sc->obs_cam[o], j = sc->obs_pt[o];
    Proj p;
    project_k(R + 9 * c, T + 3 * c, X + 3 * j, k, p);
    if (!(p.xc[2] > 0.0)) ++bad;
    double ex = (p.uv[0] - sc->obs_uv[2 * o]) / sc->sigma_px;
    double ey = (p.uv[1] - sc->obs_uv[2 * o + 1]) / sc->sigma_px;
    double ss = ex * ex + ey * ey;
    if (uv) { uv[2 * o] = p.uv[0]; uv[2 * o + 1] = p.uv[1]; }
    if (z) z[o] = p.xc[2];
    if (e) { e[2 * o] = ex; e[2 * o + 1] = ey; }
    if (s) s[o] = ss;
    if (rho) rho[o] = huber_rho(ss, dt);
    if (w) w[o] = huber_w(ss, dt);
  }
  return bad;
}

// Unwhitened Jacobians of the predicted pixel per observation, row-major 2x3 /
// 2x3 / 2x3 / 2x2 / 2x3: Jw (right rotation perturbation), JT, JX, Jk (k1, k2),
// Ji (f, cx, cy).
void or_jacobians(const OrScene* sc, const double* R, const double* T, const double* X,
                  const double* k, double* Jw, double* JT, double* JX, double* Jk, double* Ji) {
  for (int o = 0; o < sc->n_obs; ++o) {
    const int c = sc->obs_cam[o], j = sc->obs_pt[o];
    Proj p;
    project_k(R + 9 * c, T + 3 * c, X + 3 * j, k, p);
    ObsJac J;
    obs_jacobian(R + 9 * c, p, k[2], k[0], k[1], J);
    std::memcpy(Jw + 6 * o, J.Jw, sizeof J.Jw);
    std::memcpy(JT + 6 * o, J.JT, sizeof J.JT);
    std::memcpy(JX + 6 * o, J.Jp, sizeof J.Jp);
    std::memcpy(Jk + 4 * o, J.Jk, sizeof J.Jk);
    std::memcpy(Ji + 6 * o, J.Ji, sizeof J.Ji);
  }
}

// Whitened prior residuals e[6C] (omega[3], T[3]) and d e_omega / d domega [9C].
void or_prior(const OrScene* sc, const double* R, const double* T, double* e, double* Jw) {
  for (int c = 0; c < sc->n_cams; ++c) prior_residual(*sc, c, R + 9 * c, T + 3 * c, e + 6 * c, Jw + 9 * c);
}

double or_cost(const OrScene* sc, const double* R, const double* T, const double* X, const double* k) {
  return cost(*sc, R, T, X, k);
}

// Number of unknowns N and reduced-system size m.
void or_dims(const OrScene* sc, int64_t* N, int32_t* m) {
  Layout L = make_layout(*sc);
  *N = L.N;
  *m = L.m;
}

// One damped step delta[N] at the state; returns 0 or 1 (non-positive pivot).
int or_step(const OrScene* sc, const double* R, const double* T, const double* X, const double* k,
            double lambda, double* delta, double* pred) {
  Layout L = make_layout(*sc);
  return schur_step(*sc, L, R, T, X, k, lambda, delta, pred);
}

void or_apply(const OrScene* sc, const double* R, const double* T, const double* X, const double* k,
              const double* delta, double* R2, double* T2, double* X2, double* k2) {
  Layout L = make_layout(*sc);
  apply_update(*sc, L, R, T, X, k, delta, R2, T2, X2, k2);
}

// Levenberg-Marquardt on the cluster, state (R, T, X, k) updated in place.
// cost_log[max_iters+1]: E before the first iteration and after each one.
// lambda_log / rho_log / accepted_log [max_iters]: damping used, gain ratio,
// and whether the trial was accepted, per iteration (any may be NULL).
int or_solve(const OrScene* sc, double* R, double* T, double* X, double* k, const OrOptions* opt,
             double* cost_log, double* lambda_log, double* rho_log, int32_t* accepted_log,
             OrStats* st) {
  Layout L = make_layout(*sc);
  const int C = sc->n_cams, P = sc->n_points;
  std::vector<double> delta(L.N), R2(9L * C), T2(3L * C), X2(3L * P), k2(5);
  double lambda = opt->lambda0;
  if (!(lambda >= kLambdaMin)) lambda = kLambdaMin;
  if (lambda > kLambdaMax) lambda = kLambdaMax;
  double nu = 2.0;
  double E = cost(*sc, R, T, X, k);
  cost_log[0] = E;
  st->iterations = st->accepted = st->rejected = 0;
  st->status = 0;
  for (int it = 0; it < opt->max_iters; ++it) {
    if (lambda_log) lambda_log[it] = lambda;
    double pred = 0.0;
    int bad = schur_step(*sc, L, R, T, X, k, lambda, delta.data(), &pred);
    double E2 = kInf, rho = -kInf;
    if (!bad) {
      apply_update(*sc, L, R, T, X, k, delta.data(), R2.data(), T2.data(), X2.data(), k2.data());
      E2 = cost(*sc, R2.data(), T2.data(), X2.data(), k2.data());
      if (std::isfinite(E2) && pred > 0.0) rho = (E - E2) / pred;
    }
    if (rho_log) rho_log[it] = rho;
    st->iterations = it + 1;
    const bool accept = !bad && std::isfinite(E2) && rho > kAcceptRatio;
    if (accepted_log) accepted_log[it] = accept ? 1 : 0;
    if (accept) {
      const double rel = (E - E2) / (E > 0.0 ? E : 1e-300);
      std::memcpy(R, R2.data(), R2.size() * sizeof(double));
      std::memcpy(T, T2.data(), T2.size() * sizeof(double));
      std::memcpy(X, X2.data(), X2.size() * sizeof(double));
      for (int b = 0; b < 5; ++b) k[b] = k2[b];
      E = E2;
      const double t = 2.0 * rho - 1.0;
      double fac = 1.0 - t * t * t;
      if (fac < 1.0 / 3.0) fac = 1.0 / 3.0;
      lambda *= fac;
      if (lambda < kLambdaMin) lambda = kLambdaMin;
      nu = 2.0;
      st->accepted++;
      cost_log[it + 1] = E;
      if (opt->stop_on_ftol && rel < opt->ftol) { st->status = 1; break; }
    } else {
      st->rejected++;
      lambda *= nu;
      nu *= 2.0;
      cost_log[it + 1] = E;
      if (lambda > kLambdaMax) { st->status = 2; break; }
    }
  }
  st->lambda = lambda;
  st->nu = nu;
  return 0;
}

}  // extern "C"
