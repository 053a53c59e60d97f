// Footprints, footprint overlaps and the GNSS/IMU patch transfer of Eq. (3)
// over a digital surface model (Sec. 3.1), for gfx950; the C ABI of
// include/ba_geo.h.
//
// Kernels
//   k_footprint_rays, k_patch_rays
//               one thread per pixel ray: the ray's first crossing with the
//               bilinear DSM (marched in half-cell steps of horizontal
//               travel, then refined by a safeguarded Illinois iteration).  Footprints: five rays per image
//               (corners and centre).  Patch transfer: one ray per patch of
//               each source image; the crossing is kept as (x, y, z, lam).
//   k_overlap   one workgroup per footprint i, its threads over j > i: area of
//               the intersection of the two corner quadrilaterals
//               (Sutherland-Hodgman clip of one convex polygon by the other).
//   k_project   one thread per (source image, patch), looping over the
//               source's destination images: Eq. (3)'s projection of the
//               patch's ground point (read once) into each destination and
//               the wrap-around re-initialisation; coalesced 16-byte uv
//               stores, the dominant traffic of the transfer.
// The DSM heights (float32) stay in device memory for the context's life; a
// flight's raster is tens of kilobytes and sits in L2 across the launches.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ba_geo.h"

namespace {

constexpr int kBlock = 256;
constexpr int kMaxSteps = 65536;     // march steps per ray, at most
constexpr int kRefine = 64;         // root-refinement iterations per ray, at most

struct Dsm {
  const float* h;                    // [ny][nx]
  int nx, ny;
  double x0, y0, cell, inv_cell, hmin, hmax;
};

struct Cam {
  double f, cx, cy;
  int w, hgt;
};

// Bilinear height at (x, y), the position clamped to the raster; the heights
// are read from `h` (the global raster, or its copy in LDS).
__device__ __forceinline__ double dsm_h(const Dsm& m, const float* h, double x, double y) {
  double gx = (x - m.x0) * m.inv_cell, gy = (y - m.y0) * m.inv_cell;
  gx = fmin(fmax(gx, 0.0), (double)(m.nx - 1));
  gy = fmin(fmax(gy, 0.0), (double)(m.ny - 1));
  const int i = min((int)floor(gx), m.nx - 2), j = min((int)floor(gy), m.ny - 2);
  const double fx = gx - i, fy = gy - j;
  const float* r0 = h + (size_t)j * m.nx + i;
  const float* r1 = r0 + m.nx;
  const double a = r0[0], b = r0[1], c = r1[0], d = r1[1];
  return (1.0 - fx) * (1.0 - fy) * a + fx * (1.0 - fy) * b + (1.0 - fx) * fy * c + fx * fy * d;
}

// Height of the ray above the surface at depth lam.
__device__ __forceinline__ double ray_gap(const Dsm& m, const float* h, const double T[3], const double d[3],
                                          double lam) {
  return T[2] + lam * d[2] - dsm_h(m, h, T[0] + lam * d[0], T[1] + lam * d[1]);
}

// First crossing of T + lam d with the DSM (heights read from h); false when
// the ray misses.
__device__ __forceinline__ bool ray_dsm(const Dsm& m, const float* h, const double T[3], const double d[3],
                                        double* lam_out) {
  if (!(d[2] < 0.0)) return false;
  const double lam_a = fmax(0.0, (T[2] - m.hmax) / -d[2]);
  const double lam_b = (T[2] - m.hmin) / -d[2];
  if (!(lam_b > 0.0)) return false;
  const double g_a = ray_gap(m, h, T, d, lam_a);
  if (g_a <= 0.0) {
    *lam_out = lam_a;
    return true;
  }
  const double dxy = hypot(d[0], d[1]);
  int n = 1;
  if (dxy != 0.0) {
    const double steps = ceil((lam_b - lam_a) * dxy / (0.5 * m.cell));
    n = steps >= (double)kMaxSteps ? kMaxSteps : max(1, (int)steps);
  }
  double lo = lam_a, hi = lam_b, glo = g_a, ghi = 1.0;
  for (int s = 1; s <= n; ++s) {
    const double lam = s == n ? lam_b : lam_a + (lam_b - lam_a) * s / n;
    const double gs = ray_gap(m, h, T, d, lam);
    if (gs <= 0.0) {
      hi = lam;
      ghi = gs;
      break;
    }
    lo = lam;
    glo = gs;
  }
  if (ghi > 0.0) {           // rounding kept the lowest sample above the surface: no crossing to refine
    *lam_out = lam_b;
    return true;
  }
  // Illinois (modified regula falsi) inside the bracket, the midpoint when
  // the secant point leaves it; until the bracket is within 1e-12 of the
  // depth or a sample lands on the surface.
  int side = 0;
  for (int it = 0; it < kRefine && hi - lo > 1e-12 * hi; ++it) {
    double mid = hi - ghi * (hi - lo) / (ghi - glo);
    if (!(mid > lo && mid < hi)) mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    const double gm = ray_gap(m, h, T, d, mid);
    if (gm > 0.0) {
      lo = mid;
      glo = gm;
      if (side < 0) ghi *= 0.5;
      side = -1;
    } else {
      hi = mid;
      ghi = gm;
      if (side > 0) glo *= 0.5;
      side = 1;
      if (gm == 0.0) break;
    }
  }
  *lam_out = hi;
  return true;
}

// World direction R K^-1 (u, v, 1) of a pixel.
__device__ void pixel_dir(const double* R, const Cam& k, double u, double v, double d[3]) {
  const double a = (u - k.cx) / k.f, b = (v - k.cy) / k.f;
  for (int r = 0; r < 3; ++r) d[r] = R[3 * r] * a + R[3 * r + 1] * b + R[3 * r + 2];
}

// Footprint rays: ray r = 5 image + corner; ground [n][5][3], status per ray.
__global__ __launch_bounds__(kBlock) void k_footprint_rays(Dsm m, Cam k, int n, const double* __restrict__ R,
                                                           const double* __restrict__ T, double* __restrict__ ground,
                                                           int* __restrict__ ray_ok) {
  const float* h = m.h;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 5 * n) return;
  const int img = r / 5, c = r % 5;
  const double u = (c == 1 || c == 2) ? (double)k.w : (c == 4 ? 0.5 * k.w : 0.0);
  const double v = (c == 2 || c == 3) ? (double)k.hgt : (c == 4 ? 0.5 * k.hgt : 0.0);
  double d[3], Tc[3];
  pixel_dir(R + 9 * (size_t)img, k, u, v, d);
  for (int t = 0; t < 3; ++t) Tc[t] = T[3 * (size_t)img + t];
  double lam;
  const bool ok = ray_dsm(m, h, Tc, d, &lam);
  for (int t = 0; t < 3; ++t) ground[3 * (size_t)r + t] = ok ? Tc[t] + lam * d[t] : NAN;
  ray_ok[r] = ok ? 1 : 0;
}

// Patch rays: ray r = n_patch slot + patch of source image src[slot]; out
// (x, y, z, lam) per ray.
__global__ __launch_bounds__(kBlock) void k_patch_rays(Dsm m, Cam k, int n_src, int n_patch, const int* __restrict__ src,
                                                       const double* __restrict__ R, const double* __restrict__ T,
                                                       const double* __restrict__ uv0, double4* __restrict__ gp) {
  const float* h = m.h;
  const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (size_t)n_src * n_patch) return;
  const int slot = (int)(r / n_patch), q = (int)(r % n_patch);
  const int img = src[slot];
  double d[3], Tc[3];
  pixel_dir(R + 9 * (size_t)img, k, uv0[2 * (size_t)q], uv0[2 * (size_t)q + 1], d);
  for (int t = 0; t < 3; ++t) Tc[t] = T[3 * (size_t)img + t];
  double lam;
  if (ray_dsm(m, h, Tc, d, &lam)) gp[r] = make_double4(Tc[0] + lam * d[0], Tc[1] + lam * d[1], Tc[2] + lam * d[2], lam);
  else gp[r] = make_double4(NAN, NAN, NAN, NAN);
}

// Signed area (counter-clockwise positive), shoelace.
__device__ double signed_area(const double* x, const double* y, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    const int j = i + 1 == n ? 0 : i + 1;
    s += x[i] * y[j] - x[j] * y[i];
  }
  return 0.5 * s;
}

// Loads the corner quadrilateral of footprint i in counter-clockwise order;
// false when it is missing or not convex.
__device__ bool load_quad(const double* __restrict__ ground, int i, double x[4], double y[4]) {
  for (int c = 0; c < 4; ++c) {
    x[c] = ground[15 * (size_t)i + 3 * c];
    y[c] = ground[15 * (size_t)i + 3 * c + 1];
  }
  for (int c = 0; c < 4; ++c)
    if (!(isfinite(x[c]) && isfinite(y[c]))) return false;
  if (signed_area(x, y, 4) < 0.0) {
    double t = x[1]; x[1] = x[3]; x[3] = t;
    t = y[1]; y[1] = y[3]; y[3] = t;
  }
  for (int c = 0; c < 4; ++c) {
    const int b = (c + 1) & 3, e = (c + 2) & 3;
    if ((x[b] - x[c]) * (y[e] - y[b]) - (y[b] - y[c]) * (x[e] - x[b]) < 0.0) return false;
  }
  return true;
}

constexpr int kClipMax = 9;   // 4 vertices + at most one more per clipping edge

// Area of the part of quadrilateral (ax, ay) inside convex CCW quadrilateral (bx, by).
__device__ double clip_area(const double ax[4], const double ay[4], const double bx[4], const double by[4]) {
  double px[kClipMax], py[kClipMax], qx[kClipMax], qy[kClipMax];
  int n = 4;
  for (int c = 0; c < 4; ++c) { px[c] = ax[c]; py[c] = ay[c]; }
  for (int e = 0; e < 4 && n > 0; ++e) {
    const double x0 = bx[e], y0 = by[e], ex = bx[(e + 1) & 3] - x0, ey = by[(e + 1) & 3] - y0;
    int m = 0;
    for (int i = 0; i < n; ++i) {
      const int j = i + 1 == n ? 0 : i + 1;
      const double sp = ex * (py[i] - y0) - ey * (px[i] - x0);
      const double sq = ex * (py[j] - y0) - ey * (px[j] - x0);
      if (sp >= 0.0 && m < kClipMax) { qx[m] = px[i]; qy[m] = py[i]; ++m; }
      if ((sp >= 0.0) != (sq >= 0.0) && m < kClipMax) {
        const double t = sp / (sp - sq);
        qx[m] = px[i] + (px[j] - px[i]) * t;
        qy[m] = py[i] + (py[j] - py[i]) * t;
        ++m;
      }
    }
    n = m;
    for (int i = 0; i < n; ++i) { px[i] = qx[i]; py[i] = qy[i]; }
  }
  return n >= 3 ? fabs(signed_area(px, py, n)) : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_overlap(int n, const double* __restrict__ ground, double* __restrict__ area) {
  const int i = blockIdx.x;
  double ax[4], ay[4];
  const bool ok_i = load_quad(ground, i, ax, ay);
  const size_t row = (size_t)i * n - (size_t)i * (i + 1) / 2;
  for (int j = i + 1 + threadIdx.x; j < n; j += blockDim.x) {
    double bx[4], by[4];
    const bool ok_j = load_quad(ground, j, bx, by);
    area[row + (j - i - 1)] = (ok_i && ok_j) ? clip_area(ax, ay, bx, by) : NAN;
  }
}

// Cluster membership from footprints (Sec. 3.1: overlapping images, within
// and across strips, are found by comparing footprints; Sec. 3.2: the
// cluster of the current image and its overlapping images).  One thread per
// triggering image i (flight order).  Images a, b overlap when both
// footprints exist (convex corner quadrilaterals, finite centre) and their
// intersection covers at least min_overlap of the smaller footprint.  The
// cluster: i; its in-strip predecessors i-1, i-2, ... (at most max_back,
// each overlapping the image after it); the earlier images of other strips
// overlapping i, nearest first by footprint-centre distance (ties: lower
// index); cut at max_cams; none below min_cams.  Members leave in ascending
// order with their fixed flag (other strips, and in-strip predecessors more
// than free_back steps back).  The candidate list of each thread is kept
// sorted in LDS.
constexpr int kMemberThreads = 64;
constexpr int kMaxMembers = 64;

struct MemberRule {
  int max_back, free_back, max_cams, min_cams;
  double min_overlap;
};

__device__ bool quad_area(const double* __restrict__ ground, int k, double x[4], double y[4], double* a) {
  if (!load_quad(ground, k, x, y)) return false;
  if (!(isfinite(ground[15 * (size_t)k + 12]) && isfinite(ground[15 * (size_t)k + 13]))) return false;
  *a = fabs(signed_area(x, y, 4));
  return true;
}

__global__ __launch_bounds__(kMemberThreads) void k_members(int n, const double* __restrict__ ground,
                                                            const int* __restrict__ strip, MemberRule rule,
                                                            int* __restrict__ members, unsigned char* __restrict__ fixed,
                                                            int* __restrict__ count) {
  __shared__ double s_d[kMemberThreads][kMaxMembers];
  __shared__ int s_j[kMemberThreads][kMaxMembers];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double* cd = s_d[threadIdx.x];
  int* cj = s_j[threadIdx.x];
  const int cap = rule.max_cams;
  int* out = members + (size_t)i * cap;
  unsigned char* fo = fixed + (size_t)i * cap;
  for (int t = 0; t < cap; ++t) { out[t] = -1; fo[t] = 0; }
  double xi[4], yi[4], ai = 0.0;
  const bool oki = quad_area(ground, i, xi, yi, &ai);
  // in-strip predecessors, each overlapping the image after it
  int n_own = 0;
  {
    double xb[4], yb[4], ab = ai;
    bool okb = oki;
    for (int t = 0; t < 4; ++t) { xb[t] = xi[t]; yb[t] = yi[t]; }
    for (int j = i - 1; j >= 0 && n_own < rule.max_back && strip[j] == strip[i]; --j) {
      double xa[4], ya[4], aa;
      const bool oka = quad_area(ground, j, xa, ya, &aa);
      if (!(oka && okb) || !(clip_area(xa, ya, xb, yb) >= rule.min_overlap * fmin(aa, ab))) break;
      cj[n_own++] = j;
      for (int t = 0; t < 4; ++t) { xb[t] = xa[t]; yb[t] = ya[t]; }
      ab = aa;
    }
  }
  // earlier images of other strips overlapping i: the nearest (d2, j) first,
  // kept in a sorted list of at most `room` entries after the in-strip ones
  const int room = max(0, cap - 1 - n_own);
  int n_x = 0;
  if (oki && room > 0) {
    const double cxi = ground[15 * (size_t)i + 12], cyi = ground[15 * (size_t)i + 13];
    for (int j = 0; j < i; ++j) {
      if (strip[j] == strip[i]) continue;
      double xa[4], ya[4], aa;
      if (!quad_area(ground, j, xa, ya, &aa)) continue;
      if (!(clip_area(xi, yi, xa, ya) >= rule.min_overlap * fmin(ai, aa))) continue;
      const double dx = ground[15 * (size_t)j + 12] - cxi, dy = ground[15 * (size_t)j + 13] - cyi;
      const double d2 = dx * dx + dy * dy;
      // insertion into the sorted list (ascending d2, then j; j rises, so an
      // equal d2 goes after the entries already there)
      int pos = n_x;
      while (pos > 0 && cd[n_own + pos - 1] > d2) --pos;
      if (pos >= room) continue;
      const int last = min(n_x, room - 1);
      for (int t = last; t > pos; --t) {
        cd[n_own + t] = cd[n_own + t - 1];
        cj[n_own + t] = cj[n_own + t - 1];
      }
      cd[n_own + pos] = d2;
      cj[n_own + pos] = j;
      if (n_x < room) ++n_x;
    }
  }
  const int total = 1 + n_own + n_x;
  if (total < rule.min_cams) {
    count[i] = 0;
    return;
  }
  // ascending order: i is larger than every other member
  int m = 0;
  for (int t = 0; t < n_own + n_x; ++t) {
    const int j = cj[t];
    int pos = m;
    while (pos > 0 && out[pos - 1] > j) {
      out[pos] = out[pos - 1];
      fo[pos] = fo[pos - 1];
      --pos;
    }
    out[pos] = j;
    fo[pos] = (strip[j] == strip[i] && i - j <= rule.free_back) ? 0 : 1;
    ++m;
  }
  out[m] = i;
  fo[m] = 0;
  count[i] = m + 1;
}

// Eq. (3): the ground point of source patch q projected into each image the
// source is paired with, then wrapped into the image (re-initialisation at
// the opposite edge).  One thread per (source, patch): the ground point is
// read once and each destination's camera is uniform across the workgroup
// (blockIdx.y = source slot).  Pair e of source slot s (e in
// [src_off[s], src_off[s+1])) writes row pidx[e] of uv and flags.
__global__ __launch_bounds__(kBlock) void k_project(Cam k, int n_patch, int slot0, const int* __restrict__ src_off,
                                                    const int* __restrict__ pidx, const int* __restrict__ pdst,
                                                    const double* __restrict__ R, const double* __restrict__ T,
                                                    const double4* __restrict__ gp, double2* __restrict__ uv,
                                                    int* __restrict__ flags) {
  const int slot = slot0 + blockIdx.y;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_patch) return;
  const double4 g = gp[(size_t)slot * n_patch + q];
  const bool hit = isfinite(g.w);
  const int e1 = src_off[slot + 1];
  for (int e = src_off[slot]; e < e1; ++e) {
    const int dst = pdst[e];
    const size_t row = (size_t)pidx[e] * n_patch + q;
    const double* Rd = R + 9 * (size_t)dst;
    const double dx = g.x - T[3 * (size_t)dst], dy = g.y - T[3 * (size_t)dst + 1], dz = g.z - T[3 * (size_t)dst + 2];
    const double xc = Rd[0] * dx + Rd[3] * dy + Rd[6] * dz;
    const double yc = Rd[1] * dx + Rd[4] * dy + Rd[7] * dz;
    const double zc = Rd[2] * dx + Rd[5] * dy + Rd[8] * dz;
    int fl = BA_GEO_OK;
    double u = NAN, v = NAN;
    if (!hit || !(zc > 0.0)) {
      fl = BA_GEO_MISS;
    } else {
      u = k.f * xc / zc + k.cx;
      v = k.f * yc / zc + k.cy;
      if (!(u >= 0.0 && u < k.w && v >= 0.0 && v < k.hgt)) {
        u -= k.w * floor(u / k.w);
        v -= k.hgt * floor(v / k.hgt);
        fl = BA_GEO_REINIT;
      }
    }
    uv[row] = make_double2(u, v);
    flags[row] = fl;
  }
}

// ---- scratch of the allocation-free patch transfer ---------------------------------
//
// ba_patch_transfer_noalloc keeps its work buffers (the source list, the
// pairs grouped by source, the ground point of every source patch) in this
// file-scope array instead of memory it allocates.  Each device the library
// runs on holds its own copy until the process ends; in host code the name is
// only a stand-in, so kernels get the device address that hipGetSymbolAddress
// returns for the current device (resolved once per device at
// ba_geo_create).  Every call on a device shares that device's copy: calls
// that overlap on one device race.
constexpr size_t kScratchBytes = size_t(16) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;   // per device ordinal; nullptr until resolved

// Device address of `scratch` on `device`, which must be the current device.
hipError_t scratch_addr(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_addr.size() <= device) g_scratch_addr.resize(device + 1, nullptr);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

}  // namespace

struct ba_geo {
  int device = 0;
  void* scratch = nullptr;           // this device's address of the allocation-free transfer's scratch
  hipStream_t stream = nullptr;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};   // start, before the last kernel, end
  Dsm dsm{};
  float* d_h = nullptr;
  std::vector<void*> bufs;           // work buffers, grown on demand
  std::vector<size_t> caps;
  double total_ms = 0.0, last_ms = 0.0;
  std::string err;
};

namespace {

int gfail(ba_geo* g, int code, const std::string& msg) {
  g->err = msg;
  return code;
}

#define GEOCHK(g, expr)                                                                    \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return gfail(g, BA_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Device buffer `slot` of at least `bytes` bytes (kept and grown across calls).
int buf(ba_geo* g, int slot, size_t bytes, void** out) {
  if ((int)g->bufs.size() <= slot) {
    g->bufs.resize(slot + 1, nullptr);
    g->caps.resize(slot + 1, 0);
  }
  if (g->caps[slot] < bytes) {
    if (g->bufs[slot]) (void)hipFree(g->bufs[slot]);
    g->bufs[slot] = nullptr;
    g->caps[slot] = 0;
    if (hipMalloc(&g->bufs[slot], std::max<size_t>(bytes, 256)) != hipSuccess)
      return gfail(g, BA_E_NOMEM, "cannot allocate a work buffer");
    g->caps[slot] = std::max<size_t>(bytes, 256);
  }
  *out = g->bufs[slot];
  return BA_OK;
}

bool cam_ok(const ba_pinhole* c) {
  return c && std::isfinite(c->f) && c->f > 0 && std::isfinite(c->cx) && std::isfinite(c->cy) && c->width > 0 &&
         c->height > 0;
}

Cam to_cam(const ba_pinhole* c) { return Cam{c->f, c->cx, c->cy, c->width, c->height}; }

// Ends a call's launches: `split` says whether ev[1] marks the start of its
// last kernel (else the last kernel is timed from the start).
int finish(ba_geo* g, bool split) {
  GEOCHK(g, hipEventRecord(g->ev[2], g->stream));
  GEOCHK(g, hipStreamSynchronize(g->stream));
  float tot = 0.0f, last = 0.0f;
  GEOCHK(g, hipEventElapsedTime(&tot, g->ev[0], g->ev[2]));
  if (split) GEOCHK(g, hipEventElapsedTime(&last, g->ev[1], g->ev[2]));
  g->total_ms = tot;
  g->last_ms = split ? last : tot;
  return BA_OK;
}

// Validates the pairs and groups them by source image (stable in pair order):
// src [n_src] the source images in order of first use, src_off [n_src + 1],
// and per grouped pair e its pair index pidx[e] and destination pdst[e].
int group_pairs(ba_geo* g, int32_t n_img, int32_t n_pairs, const int32_t* pairs, std::vector<int>& src,
                std::vector<int>& src_off, std::vector<int>& pidx, std::vector<int>& pdst) {
  std::vector<int> slot_of(n_img, -1);
  src.clear();
  for (int p = 0; p < n_pairs; ++p) {
    const int a = pairs[2 * p], b = pairs[2 * p + 1];
    if (a < 0 || a >= n_img || b < 0 || b >= n_img) return gfail(g, BA_E_ARG, "pair index out of range");
    if (slot_of[a] < 0) {
      slot_of[a] = (int)src.size();
      src.push_back(a);
    }
  }
  const int n_src = (int)src.size();
  src_off.assign(n_src + 1, 0);
  pidx.resize(n_pairs);
  pdst.resize(n_pairs);
  for (int p = 0; p < n_pairs; ++p) ++src_off[slot_of[pairs[2 * p]] + 1];
  for (int s = 0; s < n_src; ++s) src_off[s + 1] += src_off[s];
  std::vector<int> fill(src_off.begin(), src_off.end() - 1);
  for (int p = 0; p < n_pairs; ++p) {
    const int e = fill[slot_of[pairs[2 * p]]]++;
    pidx[e] = p;
    pdst[e] = pairs[2 * p + 1];
  }
  return BA_OK;
}

// The two kernels of a transfer on the context's stream, events around them:
// the patch rays of every source image, then the projections.
int launch_transfer(ba_geo* g, const Cam& k, int n_src, int n_patch, int n_pairs, const int* dSrc, const int* dOff,
                    const int* dPidx, const int* dPdst, const double* dR, const double* dT, const double* dUv0,
                    double4* dGp, double2* dUv, int* dFl) {
  GEOCHK(g, hipEventRecord(g->ev[0], g->stream));
  const size_t rays = (size_t)n_src * n_patch;
  hipLaunchKernelGGL(k_patch_rays, dim3((unsigned)((rays + kBlock - 1) / kBlock)), dim3(kBlock), 0, g->stream, g->dsm,
                     k, n_src, n_patch, dSrc, dR, dT, dUv0, dGp);
  GEOCHK(g, hipGetLastError());
  GEOCHK(g, hipEventRecord(g->ev[1], g->stream));
  if (n_pairs > 0) {
    const unsigned bx = (unsigned)((n_patch + kBlock - 1) / kBlock);
    for (int s0 = 0; s0 < n_src; s0 += 65535) {
      const unsigned by = (unsigned)std::min(65535, n_src - s0);
      hipLaunchKernelGGL(k_project, dim3(bx, by), dim3(kBlock), 0, g->stream, k, n_patch, s0, dOff, dPidx, dPdst, dR,
                         dT, (const double4*)dGp, dUv, dFl);
      GEOCHK(g, hipGetLastError());
    }
  }
  return finish(g, true);
}

}  // namespace

extern "C" {

int ba_geo_create(int32_t device, const ba_dsm* dsm, ba_geo** out) {
  if (!dsm || !out || !dsm->h || dsm->nx < 2 || dsm->ny < 2 || !(dsm->cell > 0) || !std::isfinite(dsm->cell) ||
      !std::isfinite(dsm->x0) || !std::isfinite(dsm->y0))
    return BA_E_ARG;
  const size_t nn = (size_t)dsm->nx * dsm->ny;
  double hmin = INFINITY, hmax = -INFINITY;
  for (size_t i = 0; i < nn; ++i) {
    if (!std::isfinite(dsm->h[i])) return BA_E_ARG;
    hmin = std::min(hmin, (double)dsm->h[i]);
    hmax = std::max(hmax, (double)dsm->h[i]);
  }
  ba_geo* g = new ba_geo();
  g->device = device;
  auto bail = [&](int code) {
    ba_geo_destroy(g);
    return code;
  };
  if (hipSetDevice(device) != hipSuccess) return bail(BA_E_DEVICE);
  if (scratch_addr(device, &g->scratch) != hipSuccess) return bail(BA_E_DEVICE);
  if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) return bail(BA_E_DEVICE);
  for (hipEvent_t& e : g->ev)
    if (hipEventCreate(&e) != hipSuccess) return bail(BA_E_DEVICE);
  if (hipMalloc(&g->d_h, nn * sizeof(float)) != hipSuccess) return bail(BA_E_NOMEM);
  if (hipMemcpy(g->d_h, dsm->h, nn * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return bail(BA_E_DEVICE);
  g->dsm = Dsm{g->d_h, dsm->nx, dsm->ny, dsm->x0, dsm->y0, dsm->cell, 1.0 / dsm->cell, hmin, hmax};
  *out = g;
  return BA_OK;
}

int ba_geo_destroy(ba_geo* g) {
  if (!g) return BA_E_ARG;
  (void)hipSetDevice(g->device);
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  for (void* p : g->bufs)
    if (p) (void)hipFree(p);
  if (g->d_h) (void)hipFree(g->d_h);
  for (hipEvent_t e : g->ev)
    if (e) (void)hipEventDestroy(e);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
  return BA_OK;
}

int ba_footprints(ba_geo* g, int32_t n, const double* R, const double* T, const ba_pinhole* cam, double* ground,
                  int32_t* status) {
  if (!g) return BA_E_ARG;
  if (n < 0 || !cam_ok(cam)) return gfail(g, BA_E_ARG, "bad image count or camera");
  if (n == 0) return BA_OK;
  if (!R || !T || !ground || !status) return gfail(g, BA_E_ARG, "missing array");
  if (n > (1 << 26)) return gfail(g, BA_E_ARG, "too many images");
  GEOCHK(g, hipSetDevice(g->device));
  void *dR, *dT, *dG, *dOk;
  int rc;
  if ((rc = buf(g, 0, 72 * (size_t)n, &dR)) || (rc = buf(g, 1, 24 * (size_t)n, &dT)) ||
      (rc = buf(g, 2, 120 * (size_t)n, &dG)) || (rc = buf(g, 3, 20 * (size_t)n, &dOk)))
    return rc;
  GEOCHK(g, hipMemcpyAsync(dR, R, 72 * (size_t)n, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipMemcpyAsync(dT, T, 24 * (size_t)n, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipEventRecord(g->ev[0], g->stream));
  const int rays = 5 * n;
  hipLaunchKernelGGL(k_footprint_rays, dim3((rays + kBlock - 1) / kBlock), dim3(kBlock), 0, g->stream, g->dsm,
                     to_cam(cam), n, (const double*)dR, (const double*)dT, (double*)dG, (int*)dOk);
  GEOCHK(g, hipGetLastError());
  if ((rc = finish(g, false))) return rc;
  std::vector<int> ok(rays);
  GEOCHK(g, hipMemcpy(ground, dG, 120 * (size_t)n, hipMemcpyDeviceToHost));
  GEOCHK(g, hipMemcpy(ok.data(), dOk, 4 * (size_t)rays, hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) {
    status[i] = BA_GEO_OK;
    for (int c = 0; c < 5; ++c)
      if (!ok[5 * i + c]) status[i] = BA_GEO_MISS;
  }
  return BA_OK;
}

int ba_footprint_overlaps(ba_geo* g, int32_t n, const double* ground, double* area) {
  if (!g) return BA_E_ARG;
  if (n < 0 || n > 65536) return gfail(g, BA_E_ARG, "footprint count out of range (0..65536)");
  if (n < 2) return BA_OK;
  if (!ground || !area) return gfail(g, BA_E_ARG, "missing array");
  GEOCHK(g, hipSetDevice(g->device));
  const size_t np = (size_t)n * (n - 1) / 2;
  void *dG, *dA;
  int rc;
  if ((rc = buf(g, 2, 120 * (size_t)n, &dG)) || (rc = buf(g, 4, 8 * np, &dA))) return rc;
  GEOCHK(g, hipMemcpyAsync(dG, ground, 120 * (size_t)n, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipEventRecord(g->ev[0], g->stream));
  hipLaunchKernelGGL(k_overlap, dim3(n - 1), dim3(kBlock), 0, g->stream, n, (const double*)dG, (double*)dA);
  GEOCHK(g, hipGetLastError());
  if ((rc = finish(g, false))) return rc;
  GEOCHK(g, hipMemcpy(area, dA, 8 * np, hipMemcpyDeviceToHost));
  return BA_OK;
}

int ba_patch_transfer(ba_geo* g, int32_t n_img, const double* R, const double* T, int32_t n_patch,
                      const double* uv0, int32_t n_pairs, const int32_t* pairs, const ba_pinhole* cam, double* uv,
                      int32_t* flags, double* lam) {
  if (!g) return BA_E_ARG;
  if (n_img < 0 || n_patch < 0 || n_pairs < 0 || !cam_ok(cam)) return gfail(g, BA_E_ARG, "bad counts or camera");
  if (n_img == 0 || n_patch == 0) {
    if (n_pairs > 0 && n_img == 0) return gfail(g, BA_E_ARG, "pairs without images");
    return BA_OK;
  }
  if (!R || !T || !uv0 || (n_pairs > 0 && (!pairs || !uv || !flags))) return gfail(g, BA_E_ARG, "missing array");
  for (int i = 0; i < 2 * n_patch; ++i)
    if (!std::isfinite(uv0[i])) return gfail(g, BA_E_ARG, "non-finite patch centre");
  std::vector<int> src, src_off, pidx, pdst;
  int rc = group_pairs(g, n_img, n_pairs, pairs, src, src_off, pidx, pdst);
  if (rc) return rc;
  const int n_src = (int)src.size();
  if (lam)
    for (size_t i = 0; i < (size_t)n_img * n_patch; ++i) lam[i] = NAN;
  if (n_src == 0) return BA_OK;
  const size_t rays = (size_t)n_src * n_patch, total = (size_t)n_pairs * n_patch;
  GEOCHK(g, hipSetDevice(g->device));
  void *dR, *dT, *dUv0, *dSrc, *dOff, *dPidx, *dPdst, *dGp, *dUv, *dFl;
  if ((rc = buf(g, 0, 72 * (size_t)n_img, &dR)) || (rc = buf(g, 1, 24 * (size_t)n_img, &dT)) ||
      (rc = buf(g, 5, 16 * (size_t)n_patch, &dUv0)) || (rc = buf(g, 6, 4 * (size_t)n_src, &dSrc)) ||
      (rc = buf(g, 7, 4 * (size_t)(n_src + 1), &dOff)) || (rc = buf(g, 8, 4 * (size_t)n_pairs, &dPidx)) ||
      (rc = buf(g, 12, 4 * (size_t)n_pairs, &dPdst)) || (rc = buf(g, 9, 32 * rays, &dGp)) ||
      (rc = buf(g, 10, 16 * total, &dUv)) || (rc = buf(g, 11, 4 * total, &dFl)))
    return rc;
  GEOCHK(g, hipMemcpyAsync(dR, R, 72 * (size_t)n_img, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipMemcpyAsync(dT, T, 24 * (size_t)n_img, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipMemcpyAsync(dUv0, uv0, 16 * (size_t)n_patch, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipMemcpyAsync(dSrc, src.data(), 4 * (size_t)n_src, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipMemcpyAsync(dOff, src_off.data(), 4 * (size_t)(n_src + 1), hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipMemcpyAsync(dPidx, pidx.data(), 4 * (size_t)n_pairs, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipMemcpyAsync(dPdst, pdst.data(), 4 * (size_t)n_pairs, hipMemcpyHostToDevice, g->stream));
  if ((rc = launch_transfer(g, to_cam(cam), n_src, n_patch, n_pairs, (const int*)dSrc, (const int*)dOff,
                            (const int*)dPidx, (const int*)dPdst, (const double*)dR, (const double*)dT,
                            (const double*)dUv0, (double4*)dGp, (double2*)dUv, (int*)dFl)))
    return rc;
  if (total > 0) {
    GEOCHK(g, hipMemcpy(uv, dUv, 16 * total, hipMemcpyDeviceToHost));
    GEOCHK(g, hipMemcpy(flags, dFl, 4 * total, hipMemcpyDeviceToHost));
  }
  if (lam) {
    std::vector<double> gp(4 * rays);
    GEOCHK(g, hipMemcpy(gp.data(), dGp, 32 * rays, hipMemcpyDeviceToHost));
    for (int s = 0; s < n_src; ++s)
      for (int q = 0; q < n_patch; ++q) lam[(size_t)src[s] * n_patch + q] = gp[4 * ((size_t)s * n_patch + q) + 3];
  }
  return BA_OK;
}

int ba_patch_transfer_noalloc(ba_geo* g, int32_t n_img, const double* R, const double* T, int32_t n_patch,
                              const double* uv0, int32_t n_pairs, const int32_t* pairs, const ba_pinhole* cam,
                              double* uv, int32_t* flags) {
  if (!g) return BA_E_ARG;
  if (n_img < 0 || n_patch < 0 || n_pairs < 0 || !cam_ok(cam)) return gfail(g, BA_E_ARG, "bad counts or camera");
  if (n_img == 0 || n_patch == 0 || n_pairs == 0) {
    if (n_pairs > 0 && n_img == 0) return gfail(g, BA_E_ARG, "pairs without images");
    return BA_OK;
  }
  if (!R || !T || !uv0 || !pairs || !uv || !flags) return gfail(g, BA_E_ARG, "missing array");
  if (!g->scratch) return gfail(g, BA_E_DEVICE, "scratch address not resolved");
  std::vector<int> src, src_off, pidx, pdst;
  int rc = group_pairs(g, n_img, n_pairs, pairs, src, src_off, pidx, pdst);
  if (rc) return rc;
  const int n_src = (int)src.size();
  // scratch layout, each part 256-byte aligned: src, src_off, pidx, pdst, ground points
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t o_off = al(4 * (size_t)n_src), o_pidx = o_off + al(4 * (size_t)(n_src + 1));
  const size_t o_pdst = o_pidx + al(4 * (size_t)n_pairs), o_gp = o_pdst + al(4 * (size_t)n_pairs);
  const size_t need = o_gp + 32 * (size_t)n_src * n_patch;
  if (need > kScratchBytes)
    return gfail(g, BA_E_ARG, "transfer needs " + std::to_string(need) + " bytes of scratch (source images x patches x 32 "
                 "bytes, plus the pair lists); the allocation-free entry point holds " + std::to_string(kScratchBytes));
  GEOCHK(g, hipSetDevice(g->device));
  char* sp = (char*)g->scratch;
  GEOCHK(g, hipMemcpyAsync(sp, src.data(), 4 * (size_t)n_src, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipMemcpyAsync(sp + o_off, src_off.data(), 4 * (size_t)(n_src + 1), hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipMemcpyAsync(sp + o_pidx, pidx.data(), 4 * (size_t)n_pairs, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipMemcpyAsync(sp + o_pdst, pdst.data(), 4 * (size_t)n_pairs, hipMemcpyHostToDevice, g->stream));
  return launch_transfer(g, to_cam(cam), n_src, n_patch, n_pairs, (const int*)sp, (const int*)(sp + o_off),
                         (const int*)(sp + o_pidx), (const int*)(sp + o_pdst), R, T, uv0, (double4*)(sp + o_gp),
                         (double2*)uv, (int*)flags);
}

int ba_cluster_membership(ba_geo* g, int32_t n, const double* ground, const int32_t* strip,
                          const ba_cluster_rule* rule, int32_t* members, uint8_t* fixed, int32_t* count) {
  if (!g) return BA_E_ARG;
  if (n < 0 || n > 65536) return gfail(g, BA_E_ARG, "image count out of range (0..65536)");
  if (!rule || rule->max_back < 0 || rule->free_back < 0 || rule->max_cams < 1 || rule->max_cams > kMaxMembers ||
      rule->min_cams < 1 || rule->min_cams > rule->max_cams || !(rule->min_overlap >= 0.0) ||
      !(rule->min_overlap <= 1.0))
    return gfail(g, BA_E_ARG, "bad cluster rule (1 <= min_cams <= max_cams <= 64, 0 <= min_overlap <= 1)");
  if (n == 0) return BA_OK;
  if (!ground || !strip || !members || !fixed || !count) return gfail(g, BA_E_ARG, "missing array");
  GEOCHK(g, hipSetDevice(g->device));
  const size_t cap = (size_t)rule->max_cams;
  void *dG, *dS, *dM, *dF, *dC;
  int rc;
  if ((rc = buf(g, 2, 120 * (size_t)n, &dG)) || (rc = buf(g, 13, 4 * (size_t)n, &dS)) ||
      (rc = buf(g, 14, 4 * cap * n, &dM)) || (rc = buf(g, 15, cap * n, &dF)) || (rc = buf(g, 3, 4 * (size_t)n, &dC)))
    return rc;
  GEOCHK(g, hipMemcpyAsync(dG, ground, 120 * (size_t)n, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipMemcpyAsync(dS, strip, 4 * (size_t)n, hipMemcpyHostToDevice, g->stream));
  GEOCHK(g, hipEventRecord(g->ev[0], g->stream));
  const MemberRule r{rule->max_back, rule->free_back, rule->max_cams, rule->min_cams, rule->min_overlap};
  hipLaunchKernelGGL(k_members, dim3((n + kMemberThreads - 1) / kMemberThreads), dim3(kMemberThreads), 0, g->stream, n,
                     (const double*)dG, (const int*)dS, r, (int*)dM, (unsigned char*)dF, (int*)dC);
  GEOCHK(g, hipGetLastError());
  if ((rc = finish(g, false))) return rc;
  GEOCHK(g, hipMemcpy(members, dM, 4 * cap * n, hipMemcpyDeviceToHost));
  GEOCHK(g, hipMemcpy(fixed, dF, cap * n, hipMemcpyDeviceToHost));
  GEOCHK(g, hipMemcpy(count, dC, 4 * (size_t)n, hipMemcpyDeviceToHost));
  return BA_OK;
}

int ba_geo_last_ms(ba_geo* g, double* total_ms, double* last_ms) {
  if (!g) return BA_E_ARG;
  if (total_ms) *total_ms = g->total_ms;
  if (last_ms) *last_ms = g->last_ms;
  return BA_OK;
}

const char* ba_geo_last_error(ba_geo* g) { return g ? g->err.c_str() : "no context"; }

}  // extern "C"
