// Host runtime of the cluster bundle-adjustment library: the C ABI of ba.h,
// validation and observation layout at submission, the HBM arena and its
// admission control, resident-cluster slots, batched launch series, and the
// continuous-batching serving thread.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <atomic>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/ba.h"
#include "ba_device.h"

using namespace bagpu;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---- arena: first-fit free list with coalescing -------------------------------------

class Arena {
 public:
  void init(size_t size) { free_.clear(); free_[0] = size; size_ = size; }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
    }
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0;
};

// ---- a submitted cluster, laid out for the device ------------------------------------

struct Staged {
  int C = 0, P = 0, O = 0, L = 0, n_chunks = 0, m = 0, n_free = 0, kcol0 = -1, kcol1 = -1;
  int kcolt[kIntr] = {-1, -1, -1, -1, -1}, sc = 0;   // column of each intrinsic; f, cx or cy estimated
  int max_iters = 0, stop_on_ftol = 0;
  double f = 0, cx = 0, cy = 0, sigma = 1, delta = 1, lambda0 = 1e-4, ftol = 0, k[2] = {0, 0};
  std::vector<double> raw_cam;   // [C][30]
  std::vector<double> X;         // [3P] internal point order
  std::vector<int> pt_orig;      // [P] caller index of each internal point
  std::vector<int> cam_col;      // [C]
  std::vector<int> lane_pt, lane_meta;
  std::vector<double> lane_uv;   // [2L]
  int Lc = 0, Lq = 0, nb = 0, n_wg = 0, n_pt_part = 0, n_cam_tasks = 0;
  std::vector<int> cl_pt, ql_pt;               // camera lanes [Lc], pair lanes [Lq]
  std::vector<double> cl_uv, ql_uv;            // [2Lc], [4Lq] raw pixels
  std::vector<int4> tasks, targets;
  // sparse (PCG) reduced system: block CSR over the free cameras, diagonal first
  int sparse = 0;
  std::vector<int> brow, bcol;   // [F + 1], [nnzb]
  std::vector<int2> tslot;       // [n_targets] block slots (a,b), (b,a) of each target
  // resident state: global IDs (caller order) when the cluster uses it;
  // observations per camera (the match-count weights of Eq. 8 fusion)
  bool resident = false, fuse = false;
  std::vector<int64_t> cam_ids, point_ids;
  std::vector<int> cam_nobs;
};

struct Layout {                  // byte offsets inside a slot block
  size_t lane_pt, lane_meta, uv64, uv32, cl_pt, cl_uv64, cl_uv32, ql_pt, ql_uv64, ql_uv32, tasks, targets,
      cam0, cam1, prior, cam_col, raw_cam, X0, X1, X320, X321, ptv, ptd, ptz, pt_orig, task_part, pt_part, Sg, Sd, dc,
      brow, bcol, tslot, Sblk, Sblk32, pcgw, rin_cam, rin_pt, rout_cam, rout_pt, cost_part,
      bad_part, cost_log, lambda_log, acc_log, stat_part, out, total;
  int n_wg, psize, pstride;
};

Layout make_layout(const Staged& s, bool mixed) {
  Layout l{};
  const size_t rs = real_size(mixed);
  l.n_wg = s.n_wg;
  // the sparse form keeps no packed triangle: Sg holds g, bS, diag U only
  l.psize = s.sparse ? 0 : s.m * (s.m + 1) / 2;
  l.pstride = (int)align_up((size_t)l.psize + 3 * (size_t)s.m, 4);
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes, 256); return at; };
  l.lane_pt = take(4 * (size_t)s.L);
  l.lane_meta = take(4 * (size_t)s.L);
  l.uv64 = take(16 * (size_t)s.L);
  l.uv32 = take(8 * (size_t)s.L);
  l.cl_pt = take(4 * (size_t)s.Lc);
  l.cl_uv64 = take(16 * (size_t)s.Lc);
  l.cl_uv32 = take(8 * (size_t)s.Lc);
  l.ql_pt = take(4 * (size_t)s.Lq);
  l.ql_uv64 = take(32 * (size_t)s.Lq);
  l.ql_uv32 = take(16 * (size_t)s.Lq);
  l.tasks = take(sizeof(int4) * s.tasks.size());
  l.targets = take(sizeof(int4) * s.targets.size());
  l.cam0 = take(8 * (size_t)kCamVals * s.C);
  l.cam1 = take(8 * (size_t)kCamVals * s.C);
  l.prior = take(8 * (size_t)kPriorVals * s.C);
  l.cam_col = take(4 * (size_t)s.C);
  l.raw_cam = take(8 * 30 * (size_t)s.C);
  l.X0 = take(24 * (size_t)s.P);
  l.X1 = take(24 * (size_t)s.P);
  l.X320 = take(12 * (size_t)s.P);
  l.X321 = take(12 * (size_t)s.P);
  l.ptv = take(rs * kPtVals * (size_t)s.P);
  l.ptd = take(rs * 4 * (size_t)s.P);
  l.ptz = take(s.sc ? rs * kPtzVals * (size_t)s.P : 0);
  l.pt_orig = take(4 * (size_t)s.P);
  l.task_part = take(rs * kTaskVals * s.tasks.size());
  l.pt_part = take(rs * kPtPartVals * (size_t)s.n_pt_part);
  l.Sg = take(8 * (size_t)l.pstride);
  l.Sd = take(s.sparse ? 0 : 8 * kSolveTbVals * (size_t)s.nb * (s.nb + 1) / 2);
  l.dc = take(8 * (size_t)s.m);
  const size_t nnzb = s.bcol.size();
  l.brow = take(4 * s.brow.size());
  l.bcol = take(4 * nnzb);
  l.tslot = take(sizeof(int2) * s.tslot.size());
  l.Sblk = take(8 * (size_t)kSbVals * nnzb);
  l.Sblk32 = take(4 * (size_t)kSbVals * nnzb);
  l.pcgw = take(8 * 2 * (size_t)(s.sparse ? s.m : 0));
  const size_t rc = s.resident ? (size_t)s.C : 0, rp = s.resident ? (size_t)s.P : 0;
  l.rin_cam = take(sizeof(int2) * rc);
  l.rin_pt = take(sizeof(int2) * rp);
  l.rout_cam = take(sizeof(int4) * rc);
  l.rout_pt = take(sizeof(int2) * rp);
  l.cost_part = take(16 * (size_t)l.n_wg);
  l.bad_part = take(4 * (size_t)l.n_wg);
  l.cost_log = take(8 * ((size_t)s.max_iters + 1));
  l.lambda_log = take(8 * (size_t)s.max_iters);
  l.acc_log = take(4 * (size_t)s.max_iters);
  l.stat_part = take(8 * (size_t)kStatVals * l.n_wg);
  l.out = take(8 * (12 * (size_t)s.C + 3 * (size_t)s.P + 5 + kStatVals));
  l.total = o;
  return l;
}

// splitmix64 finaliser: spreads IDs over a power-of-two table.
inline uint64_t mix_id(int64_t id) {
  uint64_t z = (uint64_t)id + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Global ID -> row, open addressing with linear probing (the resident store's
// index; looked up for every camera and point of every resident cluster).
class IdMap {
 public:
  const int* find(int64_t id) const {
    if (n_ == 0) return nullptr;
    for (size_t h = mix_id(id) & mask_;; h = (h + 1) & mask_) {
      if (!used_[h]) return nullptr;
      if (key_[h] == id) return &val_[h];
    }
  }
  void insert(int64_t id, int v) {     // id must not be present
    if (2 * (n_ + 1) > key_.size()) grow();
    size_t h = mix_id(id) & mask_;
    while (used_[h]) h = (h + 1) & mask_;
    used_[h] = 1;
    key_[h] = id;
    val_[h] = v;
    ++n_;
  }
  size_t size() const { return n_; }

 private:
  void grow() {
    const size_t cap = key_.empty() ? 1024 : 2 * key_.size();
    std::vector<int64_t> k(cap);
    std::vector<int> v(cap);
    std::vector<uint8_t> u(cap, 0);
    const size_t m = cap - 1;
    for (size_t i = 0; i < key_.size(); ++i)
      if (used_[i]) {
        size_t h = mix_id(key_[i]) & m;
        while (u[h]) h = (h + 1) & m;
        u[h] = 1;
        k[h] = key_[i];
        v[h] = val_[i];
      }
    key_.swap(k);
    val_.swap(v);
    used_.swap(u);
    mask_ = m;
  }
  std::vector<int64_t> key_;
  std::vector<int> val_;
  std::vector<uint8_t> used_;
  size_t mask_ = 0, n_ = 0;
};

// True when the n IDs are pairwise distinct.
bool ids_unique(const int64_t* id, int n) {
  size_t cap = 16;
  while (cap < 2 * (size_t)n) cap <<= 1;
  std::vector<int64_t> key(cap);
  std::vector<uint8_t> used(cap, 0);
  for (int i = 0; i < n; ++i) {
    size_t h = mix_id(id[i]) & (cap - 1);
    for (; used[h]; h = (h + 1) & (cap - 1))
      if (key[h] == id[i]) return false;
    used[h] = 1;
    key[h] = id[i];
  }
  return true;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

int4 mk4(int kind, int a, int b, int y, int z) { return make_int4((kind << 24) | (a << 12) | b, y, z, 0); }

// Validates the cluster and builds its work lists (integer bookkeeping only):
//  * point lanes: observations sorted by (point, camera), packed greedily into
//    64-lane chunks so that no point's observations straddle a chunk;
//  * camera lanes: observations of each free camera in point order, each
//    camera's run padded to whole chunks, cut into tasks of <= cpt chunks;
//  * pair lanes: the observation pairs of each point whose two cameras are
//    free, grouped by camera pair, padded and cut into tasks likewise;
//  * reduction targets: each free camera, each camera pair, the intrinsics.
int stage(const ba_cluster* c, Staged& s, std::string& err, int cpw, int cpt, int solver) {
  if (!c) { err = "cluster is NULL"; return BA_E_ARG; }
  const int C = c->n_cams, P = c->n_points, O = c->n_obs;
  if (C < 1 || C > kMaxCams || P < 0 || O < 0) { err = "sizes out of range (1 <= n_cams <= 512)"; return BA_E_ARG; }
  if (!c->R || !c->T || !c->k || !c->prior_R || !c->prior_T || !c->prior_sigma || !c->fixed ||
      (P > 0 && !c->X) || (O > 0 && (!c->obs_cam || !c->obs_pt || !c->obs_uv))) {
    err = "missing input array"; return BA_E_ARG;
  }
  if (c->max_iters < 1 || c->max_iters > 4096) { err = "max_iters must be in 1..4096"; return BA_E_ARG; }
  if (!(c->sigma_px > 0) || !(c->huber_delta > 0) || !std::isfinite(c->sigma_px) || !std::isfinite(c->huber_delta) ||
      !std::isfinite(c->f) || !std::isfinite(c->cx) || !std::isfinite(c->cy) || !(c->f > 0)) {
    err = "bad camera or noise parameters"; return BA_E_ARG;
  }
  if (!finite_all(c->R, 9 * (size_t)C) || !finite_all(c->T, 3 * (size_t)C) || !finite_all(c->k, 2) ||
      !finite_all(c->prior_R, 9 * (size_t)C) || !finite_all(c->prior_T, 3 * (size_t)C) ||
      (P > 0 && !finite_all(c->X, 3 * (size_t)P)) || (O > 0 && !finite_all(c->obs_uv, 2 * (size_t)O))) {
    err = "non-finite input"; return BA_E_ARG;
  }
  for (size_t i = 0; i < 6 * (size_t)C; ++i)
    if (std::isnan(c->prior_sigma[i])) { err = "NaN prior sigma"; return BA_E_ARG; }
  if (c->use_resident != 0 && c->use_resident != 1) { err = "use_resident must be 0 or 1"; return BA_E_ARG; }
  if (c->fuse_resident != 0 && c->fuse_resident != 1) { err = "fuse_resident must be 0 or 1"; return BA_E_ARG; }
  if (c->fuse_resident && !c->use_resident) { err = "fuse_resident needs use_resident"; return BA_E_ARG; }
  if (c->use_resident) {
    if (!c->cam_ids || (P > 0 && !c->point_ids)) { err = "use_resident needs cam_ids and point_ids"; return BA_E_ARG; }
    if (!ids_unique(c->cam_ids, C)) { err = "duplicate camera ID in the cluster"; return BA_E_ARG; }
    if (!ids_unique(c->point_ids, P)) { err = "duplicate point ID in the cluster"; return BA_E_ARG; }
  }
  s = Staged();
  s.C = C; s.P = P; s.O = O;
  if (c->use_resident) {
    s.resident = true;
    s.fuse = c->fuse_resident != 0;
    s.cam_ids.assign(c->cam_ids, c->cam_ids + C);
    s.point_ids.assign(c->point_ids, c->point_ids + P);
    s.cam_nobs.assign(C, 0);
    for (int o = 0; o < O; ++o)   // indices are range-checked below; count only valid ones here
      if (c->obs_cam[o] >= 0 && c->obs_cam[o] < C) ++s.cam_nobs[c->obs_cam[o]];
  }
  s.max_iters = c->max_iters; s.stop_on_ftol = c->stop_on_ftol;
  s.f = c->f; s.cx = c->cx; s.cy = c->cy; s.sigma = c->sigma_px; s.delta = c->huber_delta;
  s.lambda0 = c->lambda0; s.ftol = c->ftol; s.k[0] = c->k[0]; s.k[1] = c->k[1];
  s.cam_col.assign(C, -1);
  for (int k = 0; k < C; ++k)
    if (!c->fixed[k]) s.cam_col[k] = 6 * s.n_free++;
  if (solver == BA_SOLVER_PCG) s.sparse = 1;
  else if (solver == BA_SOLVER_AUTO) s.sparse = s.n_free > kMaxFreeCams;
  else if (solver != BA_SOLVER_DENSE) { err = "unknown solver"; return BA_E_ARG; }
  if (!s.sparse && s.n_free > kMaxFreeCams) { err = "more than BA_MAX_FREE_CAMS free cameras for the dense solver"; return BA_E_ARG; }
  if (c->intr_mask & ~31) { err = "intr_mask has bits beyond k1, k2, f, cx, cy"; return BA_E_ARG; }
  if (s.sparse && c->intr_mask) { err = "the PCG solver does not estimate intrinsics"; return BA_E_ARG; }
  // the estimated intrinsics' columns follow the cameras', in bit order
  int col = 6 * s.n_free;
  for (int b = 0; b < kIntr; ++b)
    if (c->intr_mask & (1 << b)) s.kcolt[b] = col++;
  s.kcol0 = s.kcolt[0];
  s.kcol1 = s.kcolt[1];
  s.sc = (c->intr_mask & ~3) != 0;
  s.m = col;
  s.raw_cam.resize(30 * (size_t)C);
  for (int k = 0; k < C; ++k) {
    double* r = &s.raw_cam[30 * (size_t)k];
    std::memcpy(r, c->R + 9 * k, 9 * sizeof(double));
    std::memcpy(r + 9, c->T + 3 * k, 3 * sizeof(double));
    std::memcpy(r + 12, c->prior_R + 9 * k, 9 * sizeof(double));
    std::memcpy(r + 21, c->prior_T + 3 * k, 3 * sizeof(double));
    std::memcpy(r + 24, c->prior_sigma + 6 * k, 6 * sizeof(double));
  }
  for (int o = 0; o < O; ++o) {
    const int cam = c->obs_cam[o], pt = c->obs_pt[o];
    if (cam < 0 || cam >= C || pt < 0 || pt >= P) { err = "observation index out of range"; return BA_E_ARG; }
  }
  // Internal point order: Morton (z-order) of the initial ground position, so
  // that a camera's observations touch nearby point records.  Ties keep the
  // caller's order (LSD radix sort of key << 32 | index on the key bits).
  {
    double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
    for (int j = 0; j < P; ++j)
      for (int t = 0; t < 2; ++t) {
        lo[t] = std::min(lo[t], c->X[3 * (size_t)j + t]);
        hi[t] = std::max(hi[t], c->X[3 * (size_t)j + t]);
      }
    std::vector<uint64_t> kj(P), tmp(P);
    for (int j = 0; j < P; ++j) {
      uint32_t q[2];
      for (int t = 0; t < 2; ++t) {
        const double span = hi[t] - lo[t];
        const double u = span > 0 ? (c->X[3 * (size_t)j + t] - lo[t]) / span : 0.0;
        q[t] = (uint32_t)std::min(65535.0, std::max(0.0, u * 65535.0));
      }
      uint32_t k = 0;
      for (int b = 0; b < 16; ++b) k |= ((q[0] >> b) & 1u) << (2 * b) | ((q[1] >> b) & 1u) << (2 * b + 1);
      kj[j] = (uint64_t)k << 32 | (uint32_t)j;
    }
    for (int shift = 32; shift < 64; shift += 11) {
      size_t cnt_d[2049] = {0};
      for (int j = 0; j < P; ++j) ++cnt_d[((kj[j] >> shift) & 2047u) + 1];
      for (int d = 0; d < 2048; ++d) cnt_d[d + 1] += cnt_d[d];
      for (int j = 0; j < P; ++j) tmp[cnt_d[(kj[j] >> shift) & 2047u]++] = kj[j];
      kj.swap(tmp);
    }
    s.pt_orig.resize(P);
    for (int n = 0; n < P; ++n) s.pt_orig[n] = (int)(uint32_t)kj[n];
  }
  std::vector<int> inv(P), opt(O);
  for (int n = 0; n < P; ++n) inv[s.pt_orig[n]] = n;
  for (int o = 0; o < O; ++o) opt[o] = inv[c->obs_pt[o]];
  s.X.resize(3 * (size_t)P);
  for (int n = 0; n < P; ++n)
    for (int t = 0; t < 3; ++t) s.X[3 * (size_t)n + t] = c->X[3 * (size_t)s.pt_orig[n] + t];
  // observations per point
  std::vector<int> cnt(P + 1, 0);
  for (int o = 0; o < O; ++o)
    if (++cnt[opt[o] + 1] > BA_MAX_OBS_PER_POINT) { err = "more than 64 observations of one point"; return BA_E_ARG; }
  for (int j = 0; j < P; ++j) cnt[j + 1] += cnt[j];
  // observations in (point, camera) order: a counting sort by camera, then a
  // stable one by point; then their camera, pixel and point in that order
  std::vector<int> order(O);
  {
    std::vector<int> by_cam(O), cc(C + 1, 0);
    for (int o = 0; o < O; ++o) ++cc[c->obs_cam[o] + 1];
    for (int k = 0; k < C; ++k) cc[k + 1] += cc[k];
    for (int o = 0; o < O; ++o) by_cam[cc[c->obs_cam[o]]++] = o;
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (int t = 0; t < O; ++t) order[fill[opt[by_cam[t]]]++] = by_cam[t];
  }
  std::vector<int> scam(O), spt(O);
  std::vector<double> suv(2 * (size_t)O);
  for (int j = 0; j < P; ++j)
    for (int t = cnt[j]; t < cnt[j + 1]; ++t) {
      const int o = order[t];
      scam[t] = c->obs_cam[o];
      spt[t] = j;
      suv[2 * (size_t)t] = c->obs_uv[2 * (size_t)o];
      suv[2 * (size_t)t + 1] = c->obs_uv[2 * (size_t)o + 1];
      if (t > cnt[j] && scam[t] == scam[t - 1]) { err = "a camera observes one point twice"; return BA_E_ARG; }
    }
  // greedy packing into 64-lane chunks
  std::vector<int> start(P, 0);
  int pos = 0;
  for (int j = 0; j < P; ++j) {
    const int n = cnt[j + 1] - cnt[j];
    if (n == 0) continue;
    if ((pos % kWave) + n > kWave) pos = (int)align_up(pos, kWave);
    start[j] = pos;
    pos += n;
  }
  s.L = (int)align_up(pos, kWave);
  s.n_chunks = s.L / kWave;
  s.lane_pt.assign(s.L, -1);
  // lane word: camera (9 bits) | segment start in the chunk << 9 (6 bits) |
  // segment length << 15 (7 bits) | the chunk's longest segment << 22 (7 bits)
  s.lane_meta.resize(s.L);
  s.lane_uv.assign(2 * (size_t)s.L, 0.0);
  for (int i = 0; i < s.L; ++i) s.lane_meta[i] = ((i % kWave) << 9) | (1 << 15);
  std::vector<int> chunk_max(s.n_chunks, 1);
  for (int j = 0; j < P; ++j) {
    const int n = cnt[j + 1] - cnt[j];
    for (int t = 0; t < n; ++t) {
      const int so = cnt[j] + t, lane = start[j] + t;
      s.lane_pt[lane] = j;
      s.lane_meta[lane] = scam[so] | ((start[j] % kWave) << 9) | (n << 15);
      chunk_max[lane / kWave] = std::max(chunk_max[lane / kWave], n);
      s.lane_uv[2 * (size_t)lane] = suv[2 * (size_t)so];
      s.lane_uv[2 * (size_t)lane + 1] = suv[2 * (size_t)so + 1];
    }
  }
  for (int i = 0; i < s.L; ++i) s.lane_meta[i] |= chunk_max[i / kWave] << 22;
  s.n_wg = (s.n_chunks + cpw - 1) / cpw;
  const bool intr = s.m > 6 * s.n_free;   // an intrinsic is estimated
  s.n_pt_part = intr ? s.n_wg * kWavesPerWG : 0;
  s.nb = (s.m + kSolveTb - 1) / kSolveTb;
  const int F = s.n_free;
  std::vector<int> free_cam(F);
  for (int k = 0; k < C; ++k)
    if (s.cam_col[k] >= 0) free_cam[s.cam_col[k] / 6] = k;
  // camera lanes and tasks: each free camera's observations in point order
  std::vector<int> coff(F + 1, 0);
  for (int t = 0; t < O; ++t) {
    const int col = s.cam_col[scam[t]];
    if (col >= 0) ++coff[col / 6 + 1];
  }
  for (int fi = 0; fi < F; ++fi) coff[fi + 1] += coff[fi];
  std::vector<int> cobs(coff[F]);
  {
    std::vector<int> fill(coff.begin(), coff.end() - 1);
    for (int t = 0; t < O; ++t) {
      const int col = s.cam_col[scam[t]];
      if (col >= 0) cobs[fill[col / 6]++] = t;
    }
  }
  for (int fi = 0; fi < F; ++fi) s.Lc += (int)align_up(coff[fi + 1] - coff[fi], kWave);
  s.cl_pt.assign(s.Lc, -1);
  s.cl_uv.assign(2 * (size_t)s.Lc, 0.0);
  std::vector<int2> cam_range(F);
  for (int fi = 0, base = 0; fi < F; ++fi) {
    const int n = coff[fi + 1] - coff[fi];
    for (int t = 0; t < n; ++t) {
      const int so = cobs[coff[fi] + t];
      const size_t lane = (size_t)base * kWave + t;
      s.cl_pt[lane] = spt[so];
      s.cl_uv[2 * lane] = suv[2 * (size_t)so];
      s.cl_uv[2 * lane + 1] = suv[2 * (size_t)so + 1];
    }
    const int nch = (int)(align_up(n, kWave) / kWave);
    cam_range[fi].x = (int)s.tasks.size();
    for (int ch = 0; ch < nch; ch += cpt) s.tasks.push_back(mk4(TASK_CAM, free_cam[fi], 0, base + ch, std::min(cpt, nch - ch)));
    cam_range[fi].y = (int)s.tasks.size();
    base += nch;
  }
  s.n_cam_tasks = (int)s.tasks.size();
  // pair lanes and tasks, blocks (fa < fb) in row-major upper-triangle order;
  // within a block the pairs (point, obs a, obs b) in point order
  const int nblk = F * (F - 1) / 2;
  auto blk = [F](int fa, int fb) { return fa * F - fa * (fa + 1) / 2 + (fb - fa - 1); };
  std::vector<int> poff(nblk + 1, 0);
  for (int j = 0; j < P; ++j)
    for (int ta = cnt[j]; ta < cnt[j + 1]; ++ta) {
      const int ca = s.cam_col[scam[ta]];
      if (ca < 0) continue;
      for (int tb = ta + 1; tb < cnt[j + 1]; ++tb) {
        const int cb = s.cam_col[scam[tb]];
        if (cb >= 0) ++poff[blk(ca / 6, cb / 6) + 1];
      }
    }
  for (int b = 0; b < nblk; ++b) poff[b + 1] += poff[b];
  std::vector<int3> pairs(poff[nblk]);
  {
    std::vector<int> fill(poff.begin(), poff.end() - 1);
    for (int j = 0; j < P; ++j)
      for (int ta = cnt[j]; ta < cnt[j + 1]; ++ta) {
        const int ca = s.cam_col[scam[ta]];
        if (ca < 0) continue;
        for (int tb = ta + 1; tb < cnt[j + 1]; ++tb) {
          const int cb = s.cam_col[scam[tb]];
          if (cb >= 0) pairs[fill[blk(ca / 6, cb / 6)]++] = make_int3(j, ta, tb);
        }
      }
  }
  auto blk_empty = [&](int b) { return poff[b + 1] == poff[b]; };
  for (int b = 0; b < nblk; ++b) s.Lq += (int)align_up(poff[b + 1] - poff[b], kWave);
  s.ql_pt.assign(s.Lq, -1);
  s.ql_uv.assign(4 * (size_t)s.Lq, 0.0);
  std::vector<int2> blk_range(nblk);
  for (int fa = 0, base = 0; fa < F; ++fa)
    for (int fb = fa + 1; fb < F; ++fb) {
      const int b = blk(fa, fb), n = poff[b + 1] - poff[b];
      for (int t = 0; t < n; ++t) {
        const int3 pr = pairs[poff[b] + t];
        const size_t lane = (size_t)base * kWave + t;
        s.ql_pt[lane] = pr.x;
        s.ql_uv[4 * lane] = suv[2 * (size_t)pr.y];
        s.ql_uv[4 * lane + 1] = suv[2 * (size_t)pr.y + 1];
        s.ql_uv[4 * lane + 2] = suv[2 * (size_t)pr.z];
        s.ql_uv[4 * lane + 3] = suv[2 * (size_t)pr.z + 1];
      }
      const int nch = (int)(align_up(n, kWave) / kWave);
      blk_range[b].x = (int)s.tasks.size();
      for (int ch = 0; ch < nch; ch += cpt)
        s.tasks.push_back(mk4(TASK_PAIR, free_cam[fa], free_cam[fb], base + ch, std::min(cpt, nch - ch)));
      blk_range[b].y = (int)s.tasks.size();
      base += nch;
    }
  for (int fi = 0; fi < F; ++fi) s.targets.push_back(mk4(TASK_CAM, free_cam[fi], 0, cam_range[fi].x, cam_range[fi].y));
  if (!s.sparse) {
    for (int fa = 0; fa < F; ++fa)
      for (int fb = fa + 1; fb < F; ++fb) {
        const int2 r = blk_range[blk(fa, fb)];
        s.targets.push_back(mk4(TASK_PAIR, free_cam[fa], free_cam[fb], r.x, r.y));
      }
    if (intr) s.targets.push_back(mk4(TARGET_INTR, 0, 0, 0, s.n_pt_part));
    return BA_OK;
  }
  // Block CSR of the co-visible free-camera pairs.  Row fa lists its diagonal
  // block, then the non-empty blocks (fa, fb) in increasing fb.  Each pair
  // target writes its block and the transpose.
  std::vector<std::vector<int>> nbr(F);
  for (int fa = 0; fa < F; ++fa)
    for (int fb = fa + 1; fb < F; ++fb)
      if (!blk_empty(blk(fa, fb))) {
        nbr[fa].push_back(fb);
        nbr[fb].push_back(fa);
      }
  s.brow.assign(F + 1, 0);
  std::vector<int> diag_slot(F);
  std::map<std::pair<int, int>, int> slot_of;
  for (int fa = 0; fa < F; ++fa) {
    s.brow[fa] = (int)s.bcol.size();
    diag_slot[fa] = (int)s.bcol.size();
    s.bcol.push_back(fa);
    std::sort(nbr[fa].begin(), nbr[fa].end());
    for (int fb : nbr[fa]) {
      slot_of[{fa, fb}] = (int)s.bcol.size();
      s.bcol.push_back(fb);
    }
  }
  s.brow[F] = (int)s.bcol.size();
  for (int fi = 0; fi < F; ++fi) s.tslot.push_back(make_int2(diag_slot[fi], diag_slot[fi]));
  for (int fa = 0; fa < F; ++fa)
    for (int fb = fa + 1; fb < F; ++fb) {
      if (blk_empty(blk(fa, fb))) continue;
      const int2 r = blk_range[blk(fa, fb)];
      s.targets.push_back(mk4(TASK_PAIR, free_cam[fa], free_cam[fb], r.x, r.y));
      s.tslot.push_back(make_int2(slot_of[{fa, fb}], slot_of[{fb, fa}]));
    }
  return BA_OK;
}

enum TicketState { TK_QUEUED, TK_RESIDENT, TK_DONE };

struct Ticket {
  ba_ticket id = 0;
  TicketState state = TK_QUEUED;
  bool serving = false;           // owned by the serving loop until done
  std::unique_ptr<Staged> staged; // until admission
  int C = 0, P = 0, max_iters = 0;
  size_t bytes = 0;
  int slot = -1;
  double t_submit = 0, t_admit = 0, t_done = 0;
  // results cached when the serving loop retires the cluster
  std::vector<double> out, cost_log, lambda_log;
  std::vector<int> acc_log;
  SlotCtl ctl{};
  // resident state: rows of the store per camera and per point (caller order),
  // clusters that must write back first, and whether this one has finished
  // with the store (written back, or nothing to write)
  bool resident = false, res_done = false;
  std::vector<int> cam_rows, pt_rows;
  std::vector<ba_ticket> deps;
};

struct Slot {
  bool used = false;
  ba_ticket ticket = 0;
  size_t off = 0, bytes = 0;
  Layout lay{};
  SlotDesc desc{};
  bool mixed = false;
};

// Per-launcher device batch arrays and pinned mirrors.
struct Launcher {
  int* d_act = nullptr;
  int* d_wgoff = nullptr;   // [4][max_slots + 1]: point-chunk, camera-task, pair-task, target workgroup prefixes
  int* h_act = nullptr;     // pinned: [max_slots] act, then [4][max_slots + 1] prefixes
  SlotCtl* h_ctl = nullptr; // pinned readback of all slots' control blocks
  hipEvent_t ev = nullptr;
  hipEvent_t copy_ev = nullptr;  // after the last upload from h_act
  bool copy_pending = false;
};

}  // namespace

struct ba_ctx {
  ba_options opt{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char* arena_base = nullptr;
  Arena arena;
  SlotDesc* d_desc = nullptr;
  SlotCtl* d_ctl = nullptr;
  std::vector<Slot> slots;
  std::map<ba_ticket, std::unique_ptr<Ticket>> tickets;
  std::deque<ba_ticket> queue;    // FIFO of queued tickets (admission order)
  ba_ticket next_id = 1;
  std::mutex mu;
  std::condition_variable cv;     // wakes the serving thread
  std::vector<ba_ticket> cancel;  // released while the serving loop owns them
  std::condition_variable done_cv;
  std::thread th;
  bool stop = false;
  bool dead = false;
  std::string last_error;
  Launcher api, srv;
  // Batched solves split a batch into parts on separate streams, so that one
  // part's latency-bound kernels (reduce, solve, LM) overlap the others'
  // assembly kernels.  Part 0 uses the launchers above and `stream`.
  static constexpr int kMaxParts = 4;
  Launcher api_p[kMaxParts], srv_p[kMaxParts];   // [0] unused
  hipStream_t stream_p[kMaxParts] = {};           // [0] unused
  hipEvent_t fork_ev = nullptr, join_ev[kMaxParts] = {};
  // kernel timing (ba_profile_enable)
  int prof = 0;                   // bitmask of timed kernels
  std::vector<int> prof_set_mask; // mask each used event set was recorded with
  std::vector<std::array<hipEvent_t, 2 * BA_PROF_N>> prof_ev;  // one set per iteration since the last harvest
  size_t prof_used = 0;
  double prof_ms[BA_PROF_N] = {};
  int64_t prof_n[BA_PROF_N] = {};
  // resident state keyed by global IDs (allocated at first use)
  struct ResRow { ba_ticket pending = 0; bool valid = false; };
  double* res_cam = nullptr;      // [cap][12]
  double* res_cam_w = nullptr;    // [cap] match-count weight of each pose (Eq. 8)
  double* res_pt = nullptr;       // [cap][3]
  IdMap res_cam_row, res_pt_row;
  std::vector<ResRow> res_cam_meta, res_pt_meta;
  double res_lambda = NAN;        // damping the last written-back cluster ended with
};

namespace {

int fail(ba_ctx* c, int code, const std::string& msg) {
  c->last_error = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                                    \
  do {                                                                                       \
    hipError_t e__ = (expr);                                                                 \
    if (e__ != hipSuccess) {                                                                 \
      (ctx)->dead = true;                                                                    \
      return fail((ctx), BA_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e__));  \
    }                                                                                        \
  } while (0)

// Device memory of the context: the caller's provider when it gave one, else
// hipMalloc / hipFree.
hipError_t dmalloc(ba_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (!c->opt.dev_alloc) return hipMalloc(p, bytes);
  void* q = c->opt.dev_alloc(bytes, c->opt.alloc_user);
  if (!q) return hipErrorOutOfMemory;
  if ((uintptr_t)q % 256) {
    c->opt.dev_free(q, c->opt.alloc_user);
    return hipErrorInvalidValue;
  }
  *p = q;
  return hipSuccess;
}

void dfree(ba_ctx* c, void* p) {
  if (!p) return;
  if (c->opt.dev_free) c->opt.dev_free(p, c->opt.alloc_user);
  else (void)hipFree(p);
}

int init_launcher(ba_ctx* c, Launcher& l) {
  const int S = c->opt.max_slots;
  HIPCHK(c, dmalloc(c, (void**)&l.d_act, sizeof(int) * S));
  HIPCHK(c, dmalloc(c, (void**)&l.d_wgoff, sizeof(int) * 4 * (S + 1)));
  HIPCHK(c, hipHostMalloc(&l.h_act, sizeof(int) * (S + 4 * (S + 1)), hipHostMallocDefault));
  HIPCHK(c, hipHostMalloc(&l.h_ctl, sizeof(SlotCtl) * S, hipHostMallocDefault));
  HIPCHK(c, hipEventCreateWithFlags(&l.ev, hipEventDisableTiming));
  HIPCHK(c, hipEventCreateWithFlags(&l.copy_ev, hipEventDisableTiming));
  return BA_OK;
}

void free_launcher(ba_ctx* c, Launcher& l) {
  dfree(c, l.d_act);
  dfree(c, l.d_wgoff);
  if (l.h_act) (void)hipHostFree(l.h_act);
  if (l.h_ctl) (void)hipHostFree(l.h_ctl);
  if (l.ev) (void)hipEventDestroy(l.ev);
  if (l.copy_ev) (void)hipEventDestroy(l.copy_ev);
  l = Launcher();
}

// Builds and uploads the batch arrays of the given slots on launcher l.
int make_batch(ba_ctx* c, Launcher& l, const std::vector<int>& slots, Batch& b) {
  const int S = c->opt.max_slots;
  int* act = l.h_act;
  int* off = l.h_act + S;
  // The pinned arrays are rewritten below: the previous upload from them must
  // have been executed by the stream first.
  if (l.copy_pending) {
    HIPCHK(c, hipEventSynchronize(l.copy_ev));
    l.copy_pending = false;
  }
  int* tkc = off + (S + 1);
  int* tkp = tkc + (S + 1);
  int* tgo = tkp + (S + 1);
  b = Batch{};
  b.desc = c->d_desc;
  b.ctl = c->d_ctl;
  b.act = l.d_act;
  b.wg_off = l.d_wgoff;
  b.tkc_off = l.d_wgoff + (S + 1);
  b.tkp_off = l.d_wgoff + 2 * (S + 1);
  b.tg_off = l.d_wgoff + 3 * (S + 1);
  b.n_act = (int)slots.size();
  int tot = 0, tc = 0, tp = 0, tg = 0;
  for (int i = 0; i < b.n_act; ++i) {
    const Slot& sl = c->slots[slots[i]];
    act[i] = slots[i];
    off[i] = tot;
    tkc[i] = tc;
    tkp[i] = tp;
    tgo[i] = tg;
    tot += sl.lay.n_wg;
    tc += sl.desc.n_cam_task_wg;
    tp += sl.desc.n_pair_task_wg;
    tg += sl.desc.n_targets;
    b.max_m = std::max(b.max_m, sl.desc.m);
    b.max_C = std::max(b.max_C, sl.desc.C);
    b.max_pstride = std::max(b.max_pstride, sl.lay.pstride);
    // the dense solve's LDS layout is sized by the dense clusters only
    if (sl.desc.sc) b.any_sc = 1;
    if (sl.desc.sparse) b.any_sparse = 1;
    else b.any_dense = 1, b.max_nb = std::max(b.max_nb, sl.desc.nb);
  }
  off[b.n_act] = tot;
  tkc[b.n_act] = tc;
  tkp[b.n_act] = tp;
  tgo[b.n_act] = tg;
  b.total_wg = tot;
  b.total_tkc_wg = tc;
  b.total_tkp_wg = tp;
  b.total_tg = tg;
  if (b.n_act == 0) return BA_OK;
  HIPCHK(c, hipMemcpyAsync(l.d_act, act, sizeof(int) * b.n_act, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(l.d_wgoff, off, sizeof(int) * 4 * (S + 1), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipEventRecord(l.copy_ev, c->stream));
  l.copy_pending = true;
  return BA_OK;
}

// Copies the control blocks of all slots to the launcher's pinned mirror and waits.
int harvest_prof(ba_ctx* c);

int read_ctl(ba_ctx* c, Launcher& l) {
  HIPCHK(c, hipMemcpyAsync(l.h_ctl, c->d_ctl, sizeof(SlotCtl) * c->opt.max_slots, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipEventRecord(l.ev, c->stream));
  HIPCHK(c, hipEventSynchronize(l.ev));
  if (c->prof_used) return harvest_prof(c);
  return BA_OK;
}

bool is_finished(int status) { return status != ST_RUNNING && status != ST_QUEUED; }

// ---- resident state ---------------------------------------------------------------

bool deps_done(ba_ctx* c, const Ticket& t) {
  for (ba_ticket dep : t.deps) {
    auto it = c->tickets.find(dep);
    if (it != c->tickets.end() && !it->second->res_done) return false;
  }
  return true;
}

// Assigns store rows to the cluster's IDs (new IDs get new rows) and records
// which earlier clusters must write back before it may read them.  Caller
// holds mu.
int res_register(ba_ctx* c, Ticket& t, const Staged& s) {
  const int capC = c->opt.resident_cams, capP = c->opt.resident_points;
  if (!c->res_cam) {
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, BA_E_DEVICE, "hipSetDevice failed");
    if (dmalloc(c, (void**)&c->res_cam, sizeof(double) * 12 * (size_t)capC) != hipSuccess ||
        dmalloc(c, (void**)&c->res_cam_w, sizeof(double) * (size_t)capC) != hipSuccess ||
        dmalloc(c, (void**)&c->res_pt, sizeof(double) * 3 * (size_t)capP) != hipSuccess) {
      return fail(c, BA_E_NOMEM, "cannot allocate the resident store");
    }
    if (hipMemset(c->res_cam_w, 0, sizeof(double) * (size_t)capC) != hipSuccess)
      return fail(c, BA_E_DEVICE, "cannot clear the resident weights");
  }
  size_t new_c = 0, new_p = 0;
  for (int64_t id : s.cam_ids) new_c += c->res_cam_row.find(id) ? 0 : 1;
  for (int64_t id : s.point_ids) new_p += c->res_pt_row.find(id) ? 0 : 1;
  if (c->res_cam_meta.size() + new_c > (size_t)capC || c->res_pt_meta.size() + new_p > (size_t)capP)
    return fail(c, BA_E_NOMEM, "resident store full");
  std::unordered_set<ba_ticket> deps;
  ba_ticket seen = 0;              // the last earlier writer looked at (runs of IDs share one)
  auto reg = [&](int64_t id, IdMap& rows, std::vector<ba_ctx::ResRow>& meta) {
    const int* r = rows.find(id);
    int row;
    if (!r) {
      row = (int)meta.size();
      rows.insert(id, row);
      meta.emplace_back();
    } else {
      row = *r;
    }
    const ba_ticket p = meta[row].pending;
    if (p && p != seen) {
      seen = p;
      auto pt = c->tickets.find(p);
      if (pt != c->tickets.end() && !pt->second->res_done) deps.insert(p);
    }
    meta[row].pending = t.id;
    return row;
  };
  t.cam_rows.resize(s.C);
  t.pt_rows.resize(s.P);
  for (int k = 0; k < s.C; ++k) t.cam_rows[k] = reg(s.cam_ids[k], c->res_cam_row, c->res_cam_meta);
  for (int j = 0; j < s.P; ++j) t.pt_rows[j] = reg(s.point_ids[j], c->res_pt_row, c->res_pt_meta);
  t.deps.assign(deps.begin(), deps.end());
  std::sort(t.deps.begin(), t.deps.end());
  t.resident = true;
  return BA_OK;
}

// Moves the ticket's staged data into a free slot and arena block.  Returns
// BA_E_AGAIN when no slot or memory is free.  Caller holds mu.
int admit_one(ba_ctx* c, Ticket& t) {
  int slot = -1;
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (!c->slots[i].used) { slot = i; break; }
  if (slot < 0) return BA_E_AGAIN;
  const Staged& s = *t.staged;
  const bool mixed = c->opt.precision == BA_MIXED;
  Layout lay = make_layout(s, mixed);
  size_t off = 0;
  if (!c->arena.alloc(lay.total, &off)) return BA_E_AGAIN;
  Slot& sl = c->slots[slot];
  sl.used = true;
  sl.ticket = t.id;
  sl.off = off;
  sl.bytes = lay.total;
  sl.lay = lay;
  sl.mixed = mixed;
  char* base = c->arena_base + off;
  SlotDesc& d = sl.desc;
  d = SlotDesc{};
  d.C = s.C; d.P = s.P; d.L = s.L; d.n_chunks = s.n_chunks; d.n_wg = lay.n_wg; d.cpw = c->opt.chunks_per_wg;
  d.m = s.m; d.n_free = s.n_free; d.kcol0 = s.kcol0; d.kcol1 = s.kcol1;
  for (int t = 0; t < kIntr; ++t) d.kcolt[t] = s.kcolt[t];
  d.sc = s.sc;
  d.psize = lay.psize; d.pstride = lay.pstride;
  d.max_iters = s.max_iters; d.stop_on_ftol = s.stop_on_ftol; d.mixed = mixed ? 1 : 0; d.nb = s.nb;
  d.Lc = s.Lc; d.Lq = s.Lq; d.n_tasks = (int)s.tasks.size(); d.n_cam_tasks = s.n_cam_tasks;
  d.n_cam_task_wg = (d.n_cam_tasks + kWavesPerWG - 1) / kWavesPerWG;
  d.n_pair_task_wg = (d.n_tasks - d.n_cam_tasks + kWavesPerWG - 1) / kWavesPerWG;
  d.n_targets = (int)s.targets.size(); d.n_pt_part = s.n_pt_part;
  d.f = s.f; d.cx = s.cx; d.cy = s.cy; d.inv_sigma = 1.0 / s.sigma; d.huber_dt = s.delta / s.sigma;
  d.ftol = s.ftol;
  d.lambda0 = std::isnan(s.lambda0) ? (std::isnan(c->res_lambda) ? 1e-4 : c->res_lambda) : s.lambda0;
  d.sparse = s.sparse; d.nnzb = (int)s.bcol.size();
  d.pcg_max_iters = c->opt.pcg_max_iters; d.pcg_tol = c->opt.pcg_tol;
  d.lane_pt = (const int*)(base + lay.lane_pt);
  d.lane_meta = (const int*)(base + lay.lane_meta);
  d.lane_uv64 = (double*)(base + lay.uv64);
  d.lane_uv32 = (float*)(base + lay.uv32);
  d.cl_pt = (const int*)(base + lay.cl_pt);
  d.cl_uv64 = (double*)(base + lay.cl_uv64);
  d.cl_uv32 = (float*)(base + lay.cl_uv32);
  d.ql_pt = (const int*)(base + lay.ql_pt);
  d.ql_uv64 = (double*)(base + lay.ql_uv64);
  d.ql_uv32 = (float*)(base + lay.ql_uv32);
  d.tasks = (const int4*)(base + lay.tasks);
  d.targets = (const int4*)(base + lay.targets);
  d.cam[0] = (double*)(base + lay.cam0);
  d.cam[1] = (double*)(base + lay.cam1);
  d.prior = (double*)(base + lay.prior);
  d.cam_col = (const int*)(base + lay.cam_col);
  d.raw_cam = (double*)(base + lay.raw_cam);
  d.X[0] = (double*)(base + lay.X0);
  d.X[1] = (double*)(base + lay.X1);
  d.X32[0] = (float*)(base + lay.X320);
  d.X32[1] = (float*)(base + lay.X321);
  d.ptv = base + lay.ptv;
  d.ptd = base + lay.ptd;
  d.ptz = base + lay.ptz;
  d.pt_orig = (const int*)(base + lay.pt_orig);
  d.task_part = base + lay.task_part;
  d.pt_part = base + lay.pt_part;
  d.Sg = (double*)(base + lay.Sg);
  d.Sd = (double*)(base + lay.Sd);
  d.dc = (double*)(base + lay.dc);
  d.brow = (const int*)(base + lay.brow);
  d.bcol = (const int*)(base + lay.bcol);
  d.tslot = (const int2*)(base + lay.tslot);
  d.Sblk = (double*)(base + lay.Sblk);
  d.Sblk32 = (float*)(base + lay.Sblk32);
  d.pcgw = (double*)(base + lay.pcgw);
  std::vector<int2> rin_c, rin_p, rout_p;
  std::vector<int4> rout_c;
  if (t.resident) {
    for (int k = 0; k < s.C; ++k) {
      const int row = t.cam_rows[k];
      rout_c.push_back(make_int4(k, row, s.cam_nobs[k], s.fuse && s.cam_col[k] >= 0 ? 1 : 0));
      if (c->res_cam_meta[row].valid) rin_c.push_back(make_int2(k, row));
    }
    for (int n = 0; n < s.P; ++n) {
      const int j = s.pt_orig[n], row = t.pt_rows[j];
      rout_p.push_back(make_int2(j, row));
      if (c->res_pt_meta[row].valid) rin_p.push_back(make_int2(n, row));
    }
  }
  d.n_rin_cam = (int)rin_c.size(); d.n_rin_pt = (int)rin_p.size();
  d.n_rout_cam = (int)rout_c.size(); d.n_rout_pt = (int)rout_p.size();
  d.res_cam = c->res_cam;
  d.res_cam_w = c->res_cam_w;
  d.res_pt = c->res_pt;
  d.rin_cam = (const int2*)(base + lay.rin_cam);
  d.rin_pt = (const int2*)(base + lay.rin_pt);
  d.rout_cam = (const int4*)(base + lay.rout_cam);
  d.rout_pt = (const int2*)(base + lay.rout_pt);
  d.cost_part = (double*)(base + lay.cost_part);
  d.bad_part = (int*)(base + lay.bad_part);
  d.cost_log = (double*)(base + lay.cost_log);
  d.lambda_log = (double*)(base + lay.lambda_log);
  d.acc_log = (int*)(base + lay.acc_log);
  d.stat_part = (double*)(base + lay.stat_part);
  d.out = (double*)(base + lay.out);
  hipStream_t st = c->stream;
  HIPCHK(c, hipMemcpyAsync(base + lay.lane_pt, s.lane_pt.data(), 4 * (size_t)s.L, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(base + lay.lane_meta, s.lane_meta.data(), 4 * (size_t)s.L, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(base + lay.uv64, s.lane_uv.data(), 16 * (size_t)s.L, hipMemcpyHostToDevice, st));
  if (s.Lc) {
    HIPCHK(c, hipMemcpyAsync(base + lay.cl_pt, s.cl_pt.data(), 4 * (size_t)s.Lc, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(base + lay.cl_uv64, s.cl_uv.data(), 16 * (size_t)s.Lc, hipMemcpyHostToDevice, st));
  }
  if (s.Lq) {
    HIPCHK(c, hipMemcpyAsync(base + lay.ql_pt, s.ql_pt.data(), 4 * (size_t)s.Lq, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(base + lay.ql_uv64, s.ql_uv.data(), 32 * (size_t)s.Lq, hipMemcpyHostToDevice, st));
  }
  if (!s.tasks.empty())
    HIPCHK(c, hipMemcpyAsync(base + lay.tasks, s.tasks.data(), sizeof(int4) * s.tasks.size(), hipMemcpyHostToDevice, st));
  if (!s.targets.empty())
    HIPCHK(c, hipMemcpyAsync(base + lay.targets, s.targets.data(), sizeof(int4) * s.targets.size(),
                             hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(base + lay.cam_col, s.cam_col.data(), 4 * (size_t)s.C, hipMemcpyHostToDevice, st));
  if (s.sparse) {
    HIPCHK(c, hipMemcpyAsync(base + lay.brow, s.brow.data(), 4 * s.brow.size(), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(base + lay.bcol, s.bcol.data(), 4 * s.bcol.size(), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(base + lay.tslot, s.tslot.data(), sizeof(int2) * s.tslot.size(), hipMemcpyHostToDevice, st));
  }
  HIPCHK(c, hipMemcpyAsync(base + lay.raw_cam, s.raw_cam.data(), 8 * 30 * (size_t)s.C, hipMemcpyHostToDevice, st));
  if (s.P > 0) {
    HIPCHK(c, hipMemcpyAsync(base + lay.X0, s.X.data(), 24 * (size_t)s.P, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(base + lay.pt_orig, s.pt_orig.data(), 4 * (size_t)s.P, hipMemcpyHostToDevice, st));
  }
  auto up2 = [&](size_t off, const std::vector<int2>& v) {
    return v.empty() ? hipSuccess : hipMemcpyAsync(base + off, v.data(), sizeof(int2) * v.size(), hipMemcpyHostToDevice, st);
  };
  HIPCHK(c, up2(lay.rin_cam, rin_c));
  HIPCHK(c, up2(lay.rin_pt, rin_p));
  if (!rout_c.empty())
    HIPCHK(c, hipMemcpyAsync(base + lay.rout_cam, rout_c.data(), sizeof(int4) * rout_c.size(), hipMemcpyHostToDevice, st));
  HIPCHK(c, up2(lay.rout_pt, rout_p));
  HIPCHK(c, hipMemcpyAsync(c->d_desc + slot, &d, sizeof(SlotDesc), hipMemcpyHostToDevice, st));
  SlotCtl ctl{};
  ctl.k[0][0] = s.k[0];
  ctl.k[0][1] = s.k[1];
  ctl.k[0][2] = s.f;      // principal-point offsets start at 0
  ctl.status = ST_RUNNING;
  HIPCHK(c, hipMemcpyAsync(c->d_ctl + slot, &ctl, sizeof(SlotCtl), hipMemcpyHostToDevice, st));
  // The staged host data must stay alive until the copies above have run.
  HIPCHK(c, hipStreamSynchronize(st));
  t.slot = slot;
  t.state = TK_RESIDENT;
  t.t_admit = now_s();
  t.staged.reset();
  return BA_OK;
}

// Runs prep and the initial FP64 cost for newly admitted slots.
int start_slots(ba_ctx* c, Launcher& l, const std::vector<int>& slots) {
  if (slots.empty()) return BA_OK;
  Batch b;
  int rc = make_batch(c, l, slots, b);
  if (rc) return rc;
  int maxPL = 0, maxRin = 0;
  for (int s : slots) {
    const SlotDesc& d = c->slots[s].desc;
    maxPL = std::max({maxPL, d.P, d.L, d.Lc, 2 * d.Lq});
    maxRin = std::max({maxRin, d.n_rin_cam, d.n_rin_pt});
  }
  HIPCHK(c, launch_prep(b, maxPL, maxRin, c->stream));
  HIPCHK(c, launch_initial_cost(b, c->stream));
  return BA_OK;
}

// Adds up the kernel times of the event sets recorded since the last call.
// The stream must have passed the last recorded event.
int harvest_prof(ba_ctx* c) {
  for (size_t i = 0; i < c->prof_used; ++i) {
    auto& ev = c->prof_ev[i];
    for (int k = 0; k < BA_PROF_N; ++k) {
      if (!((c->prof_set_mask[i] >> k) & 1)) continue;
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
      c->prof_ms[k] += ms;
      c->prof_n[k] += 1;
    }
  }
  c->prof_used = 0;
  return BA_OK;
}

int run_iterations(ba_ctx* c, Launcher& l, const std::vector<int>& slots, int n_iters) {
  Batch b;
  int rc = make_batch(c, l, slots, b);
  if (rc) return rc;
  const bool mixed = c->opt.precision == BA_MIXED;
  for (int i = 0; i < n_iters; ++i) {
    hipEvent_t* ev = nullptr;
    if (c->prof) {
      if (c->prof_used == c->prof_ev.size()) {
        std::array<hipEvent_t, 2 * BA_PROF_N> set;
        for (auto& e : set) HIPCHK(c, hipEventCreate(&e));
        c->prof_ev.push_back(set);
        c->prof_set_mask.push_back(0);
      }
      c->prof_set_mask[c->prof_used] = c->prof;
      ev = c->prof_ev[c->prof_used++].data();
    }
    HIPCHK(c, launch_iteration(b, mixed, c->stream, ev, c->prof));
  }
  return BA_OK;
}

// n LM iterations of disjoint groups of slots, part p on stream p (part 0 on
// the context's stream, with launcher l0); the context's stream then waits
// for every part.
int run_iterations_parts(ba_ctx* c, bool serving, const std::vector<std::vector<int>>& parts, int n_iters) {
  const int P = (int)parts.size();
  Batch b[ba_ctx::kMaxParts];
  int rc;
  for (int p = 0; p < P; ++p) {
    Launcher& l = p == 0 ? (serving ? c->srv : c->api) : (serving ? c->srv_p[p] : c->api_p[p]);
    if ((rc = make_batch(c, l, parts[p], b[p]))) return rc;   // uploads on the context's stream
  }
  HIPCHK(c, hipEventRecord(c->fork_ev, c->stream));
  for (int p = 1; p < P; ++p) HIPCHK(c, hipStreamWaitEvent(c->stream_p[p], c->fork_ev, 0));
  const bool mixed = c->opt.precision == BA_MIXED;
  for (int i = 0; i < n_iters; ++i) {
    for (int p = 0; p < P; ++p) {
      hipEvent_t* ev = nullptr;
      if (c->prof) {
        if (c->prof_used == c->prof_ev.size()) {
          std::array<hipEvent_t, 2 * BA_PROF_N> set;
          for (auto& e : set) HIPCHK(c, hipEventCreate(&e));
          c->prof_ev.push_back(set);
          c->prof_set_mask.push_back(0);
        }
        c->prof_set_mask[c->prof_used] = c->prof;
        ev = c->prof_ev[c->prof_used++].data();
      }
      HIPCHK(c, launch_iteration(b[p], mixed, p ? c->stream_p[p] : c->stream, ev, c->prof));
    }
  }
  for (int p = 1; p < P; ++p) {
    HIPCHK(c, hipEventRecord(c->join_ev[p], c->stream_p[p]));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->join_ev[p], 0));
  }
  return BA_OK;
}

// Splits running slots into `P` parts of about equal assembly work (point
// workgroups), in slot order.
void split_parts(ba_ctx* c, const std::vector<int>& act, int P, std::vector<std::vector<int>>& parts) {
  size_t total = 0;
  for (int s : act) total += (size_t)c->slots[s].desc.n_wg;
  parts.assign(P, {});
  size_t acc = 0;
  for (int s : act) {
    const int p = (int)std::min<size_t>(P - 1, acc * P / std::max<size_t>(total, 1));
    parts[p].push_back(s);
    acc += (size_t)c->slots[s].desc.n_wg;
  }
  parts.erase(std::remove_if(parts.begin(), parts.end(), [](const std::vector<int>& v) { return v.empty(); }),
              parts.end());
}

// Iterations of the running slots, split across streams when there are enough.
int run_tick(ba_ctx* c, bool serving, const std::vector<int>& act, int n_iters) {
  const int P = c->opt.batch_streams;
  if (P > 1 && (int)act.size() >= 4 * P) {
    std::vector<std::vector<int>> parts;
    split_parts(c, act, P, parts);
    return run_iterations_parts(c, serving, parts, n_iters);
  }
  return run_iterations(c, serving ? c->srv : c->api, act, n_iters);
}

// Exports the listed slots' state into their ticket caches (synchronous).
int export_slots(ba_ctx* c, Launcher& l, const std::vector<int>& slots) {
  if (slots.empty()) return BA_OK;
  Batch b;
  int rc = make_batch(c, l, slots, b);
  if (rc) return rc;
  int maxP = 0;
  for (int s : slots) maxP = std::max(maxP, c->slots[s].desc.P);
  HIPCHK(c, launch_export(b, maxP, c->stream));
  for (int s : slots) {
    Slot& sl = c->slots[s];
    Ticket& t = *c->tickets[sl.ticket];
    t.out.resize(12 * (size_t)sl.desc.C + 3 * (size_t)sl.desc.P + 5 + kStatVals);
    t.cost_log.resize((size_t)sl.desc.max_iters + 1);
    t.lambda_log.resize((size_t)sl.desc.max_iters);
    t.acc_log.resize((size_t)sl.desc.max_iters);
    HIPCHK(c, hipMemcpyAsync(t.out.data(), sl.desc.out, 8 * t.out.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(t.cost_log.data(), sl.desc.cost_log, 8 * t.cost_log.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(t.lambda_log.data(), sl.desc.lambda_log, 8 * t.lambda_log.size(), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(t.acc_log.data(), sl.desc.acc_log, 4 * t.acc_log.size(), hipMemcpyDeviceToHost, c->stream));
  }
  // Finished resident clusters write their state back (once).
  std::vector<int> wb, done;
  for (int s : slots) {
    Ticket& t = *c->tickets[c->slots[s].ticket];
    const int st = l.h_ctl[s].status;
    if (!t.resident || t.res_done || !is_finished(st)) continue;
    done.push_back(s);
    if (st != ST_BAD_INIT) wb.push_back(s);
  }
  if (!wb.empty()) {
    Batch bw;
    if ((rc = make_batch(c, l, wb, bw))) return rc;
    int maxR = 0;
    for (int s : wb) maxR = std::max({maxR, c->slots[s].desc.n_rout_cam, c->slots[s].desc.n_rout_pt});
    HIPCHK(c, launch_writeback(bw, maxR, c->stream));
  }
  rc = read_ctl(c, l);
  if (rc) return rc;
  for (int s : slots) c->tickets[c->slots[s].ticket]->ctl = l.h_ctl[s];
  for (int s : done) {
    Ticket& t = *c->tickets[c->slots[s].ticket];
    if (l.h_ctl[s].status != ST_BAD_INIT) {
      for (int row : t.cam_rows) c->res_cam_meta[row].valid = true;
      for (int row : t.pt_rows) c->res_pt_meta[row].valid = true;
      c->res_lambda = l.h_ctl[s].lambda;
    }
    for (int row : t.cam_rows)
      if (c->res_cam_meta[row].pending == t.id) c->res_cam_meta[row].pending = 0;
    for (int row : t.pt_rows)
      if (c->res_pt_meta[row].pending == t.id) c->res_pt_meta[row].pending = 0;
    t.res_done = true;
  }
  if (!done.empty()) c->cv.notify_all();
  return BA_OK;
}

void free_slot(ba_ctx* c, int s) {
  Slot& sl = c->slots[s];
  if (!sl.used) return;
  c->arena.release(sl.off, sl.bytes);
  sl = Slot();
}

// Admits queued tickets in FIFO order while slots and memory allow.  When
// `serving_only`, only tickets handed to the serving loop are admitted.  A
// ticket that waits for earlier clusters to write back resident state is
// passed over (later tickets that do not depend on it go ahead).
int admit_queue(ba_ctx* c, std::vector<int>& admitted, bool serving_only) {
  for (auto it = c->queue.begin(); it != c->queue.end();) {
    Ticket& t = *c->tickets[*it];
    if ((serving_only && !t.serving) || !deps_done(c, t)) { ++it; continue; }
    int rc = admit_one(c, t);
    if (rc == BA_E_AGAIN) break;
    if (rc) return rc;
    admitted.push_back(t.slot);
    it = c->queue.erase(it);
  }
  return BA_OK;
}

// A serving ticket is queued that could be admitted now (its resident
// dependencies have written back).
bool serving_queued(ba_ctx* c) {
  for (ba_ticket id : c->queue) {
    const Ticket& t = *c->tickets[id];
    if (t.serving && deps_done(c, t)) return true;
  }
  return false;
}

// One serving tick: retire finished clusters, admit queued ones, iterate.
Ticket* find_ticket(ba_ctx* c, ba_ticket id);

void serve_loop(ba_ctx* c) {
  (void)hipSetDevice(c->device);
  std::vector<int> active;
  std::unique_lock<std::mutex> lk(c->mu);
  while (!c->stop) {
    // cancel: clusters released while the loop owned them.  The previous
    // tick has completed on the device, so their slots can be freed; they
    // write nothing back, and a ticket that no longer exists holds back no
    // later cluster.
    if (!c->cancel.empty()) {
      for (ba_ticket id : c->cancel) {
        Ticket* t = find_ticket(c, id);
        if (!t) continue;
        if (t->state == TK_RESIDENT) {
          active.erase(std::remove(active.begin(), active.end(), t->slot), active.end());
          free_slot(c, t->slot);
        }
        c->queue.erase(std::remove(c->queue.begin(), c->queue.end(), id), c->queue.end());
        c->tickets.erase(id);
      }
      c->cancel.clear();
      c->done_cv.notify_all();
    }
    // retire
    std::vector<int> fin;
    for (int s : active)
      if (is_finished(c->srv.h_ctl[s].status)) fin.push_back(s);
    if (!fin.empty()) {
      if (export_slots(c, c->srv, fin)) break;
      const double t_done = now_s();
      for (int s : fin) {
        Ticket& t = *c->tickets[c->slots[s].ticket];
        t.state = TK_DONE;
        t.serving = false;
        t.slot = -1;
        t.t_done = t_done;
        free_slot(c, s);
      }
      active.erase(std::remove_if(active.begin(), active.end(),
                                  [&](int s) { return std::find(fin.begin(), fin.end(), s) != fin.end(); }),
                   active.end());
      c->done_cv.notify_all();
    }
    // admit
    std::vector<int> adm;
    if (admit_queue(c, adm, true)) break;
    if (!adm.empty()) {
      if (start_slots(c, c->srv, adm)) break;
      active.insert(active.end(), adm.begin(), adm.end());
    }
    if (active.empty()) {
      c->cv.wait(lk, [&] { return c->stop || serving_queued(c) || !c->cancel.empty(); });
      continue;
    }
    if (run_tick(c, true, active, c->opt.iters_per_tick)) break;
    if (hipMemcpyAsync(c->srv.h_ctl, c->d_ctl, sizeof(SlotCtl) * c->opt.max_slots, hipMemcpyDeviceToHost, c->stream) ||
        hipEventRecord(c->srv.ev, c->stream)) {
      c->dead = true;
      break;
    }
    lk.unlock();
    const hipError_t e = hipEventSynchronize(c->srv.ev);
    lk.lock();
    if (e != hipSuccess) { c->dead = true; c->last_error = hipGetErrorString(e); break; }
    if (c->prof_used && harvest_prof(c)) break;
  }
  if (c->dead) c->done_cv.notify_all();
}

Ticket* find_ticket(ba_ctx* c, ba_ticket id) {
  auto it = c->tickets.find(id);
  return it == c->tickets.end() ? nullptr : it->second.get();
}

// Ensures a ticket outside the serving loop is resident (admits it out of turn).
int ensure_resident(ba_ctx* c, Ticket& t, std::vector<int>& admitted) {
  if (t.serving) return fail(c, BA_E_STATE, "cluster is owned by the serving loop");
  if (t.state == TK_RESIDENT) return BA_OK;
  if (t.state == TK_DONE) return fail(c, BA_E_STATE, "cluster already retired");
  if (!deps_done(c, t))
    return fail(c, BA_E_STATE, "cluster reads resident state that an unfinished earlier cluster has still to write");
  int rc = admit_one(c, t);
  if (rc == BA_E_AGAIN) return fail(c, BA_E_AGAIN, "no free slot or arena memory");
  if (rc) return rc;
  c->queue.erase(std::remove(c->queue.begin(), c->queue.end(), t.id), c->queue.end());
  admitted.push_back(t.slot);
  return BA_OK;
}

}  // namespace

namespace {
int enqueue_staged(ba_ctx* c, std::unique_ptr<Staged> st, ba_ticket* ticket, double t_submit);
}  // namespace

extern "C" {

const char* ba_strerror(int code) {
  switch (code) {
    case BA_OK: return "ok";
    case BA_E_ARG: return "invalid argument";
    case BA_E_NOMEM: return "out of memory";
    case BA_E_AGAIN: return "try again";
    case BA_E_STATE: return "invalid state";
    case BA_E_DEVICE: return "device error";
    case BA_E_TIMEOUT: return "timeout";
    default: return "unknown error";
  }
}

const char* ba_last_error(ba_ctx* c) { return c ? c->last_error.c_str() : "no context"; }

int ba_create(const ba_options* opt, ba_ctx** out) {
  if (!opt || !out) return BA_E_ARG;
  *out = nullptr;
  if (opt->precision != BA_FP64 && opt->precision != BA_MIXED) return BA_E_ARG;
  if ((opt->dev_alloc == nullptr) != (opt->dev_free == nullptr)) return BA_E_ARG;
  // 0 selects a field's default; a negative count is an error
  if (opt->max_slots < 0 || opt->max_queue < 0 || opt->iters_per_tick < 0 || opt->chunks_per_wg < 0 ||
      opt->chunks_per_task < 0 || opt->pcg_max_iters < 0 || opt->pcg_tol < 0 || opt->resident_cams < 0 ||
      opt->resident_points < 0)
    return BA_E_ARG;
  auto c = std::make_unique<ba_ctx>();
  c->opt = *opt;
  if (c->opt.hbm_budget_bytes == 0) c->opt.hbm_budget_bytes = (size_t)1 << 30;
  if (c->opt.max_slots <= 0) c->opt.max_slots = 256;
  if (c->opt.max_queue <= 0) c->opt.max_queue = 4096;
  if (c->opt.iters_per_tick <= 0) c->opt.iters_per_tick = 2;
  if (c->opt.chunks_per_wg <= 0) c->opt.chunks_per_wg = 16;
  if (c->opt.chunks_per_task <= 0) c->opt.chunks_per_task = 4;
  if (c->opt.pcg_max_iters <= 0) c->opt.pcg_max_iters = 500;
  if (!(c->opt.pcg_tol > 0)) c->opt.pcg_tol = 0.1;
  if (c->opt.batch_streams == 0) c->opt.batch_streams = 2;
  if (c->opt.batch_streams < 1 || c->opt.batch_streams > ba_ctx::kMaxParts) return BA_E_ARG;
  if (c->opt.resident_cams <= 0) c->opt.resident_cams = 8192;
  if (c->opt.resident_points <= 0) c->opt.resident_points = 1 << 22;
  if (c->opt.solver < BA_SOLVER_AUTO || c->opt.solver > BA_SOLVER_PCG || c->opt.pcg_max_iters > 100000 ||
      !(c->opt.pcg_tol < 1)) return BA_E_ARG;
  if (c->opt.max_slots > 65536 || c->opt.chunks_per_wg > 4096 || c->opt.chunks_per_task > 4096) return BA_E_ARG;
  c->device = opt->device;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return BA_E_DEVICE;
  if (c->device < 0 || c->device >= ndev) return BA_E_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return BA_E_DEVICE;
  if (opt->stream) c->stream = (hipStream_t)opt->stream;
  else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return BA_E_DEVICE;
    c->own_stream = true;
  }
  // from here on a failure releases what was set up (ba_destroy copes with a
  // partly built context)
  auto bail = [&](int code) {
    ba_destroy(c.release());
    return code;
  };
  if (dmalloc(c.get(), (void**)&c->arena_base, c->opt.hbm_budget_bytes) != hipSuccess) return bail(BA_E_NOMEM);
  c->arena.init(c->opt.hbm_budget_bytes);
  if (dmalloc(c.get(), (void**)&c->d_desc, sizeof(SlotDesc) * c->opt.max_slots) != hipSuccess ||
      dmalloc(c.get(), (void**)&c->d_ctl, sizeof(SlotCtl) * c->opt.max_slots) != hipSuccess)
    return bail(BA_E_NOMEM);
  if (hipMemset(c->d_ctl, 0, sizeof(SlotCtl) * c->opt.max_slots) != hipSuccess) return bail(BA_E_DEVICE);
  c->slots.resize(c->opt.max_slots);
  if (init_launcher(c.get(), c->api) || init_launcher(c.get(), c->srv)) return bail(BA_E_DEVICE);
  if (hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess) return bail(BA_E_DEVICE);
  for (int p = 1; p < c->opt.batch_streams; ++p) {
    if (init_launcher(c.get(), c->api_p[p]) || init_launcher(c.get(), c->srv_p[p]) ||
        hipStreamCreateWithFlags(&c->stream_p[p], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->join_ev[p], hipEventDisableTiming) != hipSuccess)
      return bail(BA_E_DEVICE);
  }
  for (int i = 0; i < c->opt.max_slots; ++i) c->srv.h_ctl[i] = SlotCtl{};
  if (hipDeviceSynchronize() != hipSuccess) return bail(BA_E_DEVICE);
  ba_ctx* raw = c.release();
  if (opt->serve) raw->th = std::thread(serve_loop, raw);
  *out = raw;
  return BA_OK;
}

int ba_destroy(ba_ctx* c) {
  if (!c) return BA_E_ARG;
  {
    std::lock_guard<std::mutex> g(c->mu);
    c->stop = true;
  }
  c->cv.notify_all();
  if (c->th.joinable()) c->th.join();
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (int p = 1; p < ba_ctx::kMaxParts; ++p)
    if (c->stream_p[p]) (void)hipStreamSynchronize(c->stream_p[p]);
  free_launcher(c, c->api);
  for (int p = 1; p < ba_ctx::kMaxParts; ++p) {
    free_launcher(c, c->api_p[p]);
    free_launcher(c, c->srv_p[p]);
    if (c->stream_p[p]) (void)hipStreamDestroy(c->stream_p[p]);
    if (c->join_ev[p]) (void)hipEventDestroy(c->join_ev[p]);
  }
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  free_launcher(c, c->srv);
  for (auto& set : c->prof_ev)
    for (auto& e : set) (void)hipEventDestroy(e);
  dfree(c, c->d_desc);
  dfree(c, c->d_ctl);
  dfree(c, c->arena_base);
  dfree(c, c->res_cam);
  dfree(c, c->res_cam_w);
  dfree(c, c->res_pt);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return BA_OK;
}

size_t ba_footprint(ba_ctx* c, const ba_cluster* cl) {
  if (!c) return 0;
  Staged s;
  std::string err;
  if (stage(cl, s, err, c->opt.chunks_per_wg, c->opt.chunks_per_task, c->opt.solver)) return 0;
  return make_layout(s, c->opt.precision == BA_MIXED).total;
}

int ba_submit_cluster(ba_ctx* c, const ba_cluster* cl, ba_ticket* ticket) {
  const double t_submit = now_s();   // latency runs from here: validation and layout included
  if (!c || !ticket) return BA_E_ARG;
  auto st = std::make_unique<Staged>();
  std::string err;
  int rc = stage(cl, *st, err, c->opt.chunks_per_wg, c->opt.chunks_per_task, c->opt.solver);
  std::lock_guard<std::mutex> g(c->mu);
  if (rc) return fail(c, rc, err);
  return enqueue_staged(c, std::move(st), ticket, t_submit);
}

int ba_submit_clusters(ba_ctx* c, int32_t n, const ba_cluster* cl, ba_ticket* tickets) {
  const double t_submit = now_s();
  if (!c || n < 0 || (n > 0 && (!cl || !tickets))) return BA_E_ARG;
  for (int i = 0; i < n; ++i) tickets[i] = 0;
  std::vector<std::unique_ptr<Staged>> st(n);
  std::vector<int> rc(n, BA_OK);
  std::vector<std::string> err(n);
  {
    // lay the clusters out on up to 8 host threads; they share nothing
    std::atomic<int> next{0};
    auto work = [&]() {
      for (int i; (i = next.fetch_add(1)) < n;) {
        st[i] = std::make_unique<Staged>();
        rc[i] = stage(&cl[i], *st[i], err[i], c->opt.chunks_per_wg, c->opt.chunks_per_task, c->opt.solver);
      }
    };
    const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
    const int nt = std::min({n, hw, 8});
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
  }
  std::lock_guard<std::mutex> g(c->mu);
  for (int i = 0; i < n; ++i)
    if (rc[i]) return fail(c, rc[i], "cluster " + std::to_string(i) + ": " + err[i]);
  for (int i = 0; i < n; ++i) {
    const int r = enqueue_staged(c, std::move(st[i]), &tickets[i], t_submit);
    if (r) return r;
  }
  return BA_OK;
}

}  // extern "C"

namespace {

// Queues a laid-out cluster (registering its resident IDs) and returns its
// ticket.  Caller holds mu.
int enqueue_staged(ba_ctx* c, std::unique_ptr<Staged> st, ba_ticket* ticket, double t_submit) {
  int rc;
  if (c->dead) return fail(c, BA_E_DEVICE, "context is unusable after a device error");
  const size_t bytes = make_layout(*st, c->opt.precision == BA_MIXED).total;
  if (bytes > c->arena.size()) return fail(c, BA_E_NOMEM, "cluster footprint exceeds the arena");
  if ((int)c->queue.size() >= c->opt.max_queue) return fail(c, BA_E_AGAIN, "admission queue full");
  auto t = std::make_unique<Ticket>();
  t->id = c->next_id;
  if (st->resident && (rc = res_register(c, *t, *st))) return rc;
  c->next_id++;
  t->C = st->C;
  t->P = st->P;
  t->max_iters = st->max_iters;
  t->bytes = bytes;
  t->t_submit = t_submit;
  t->staged = std::move(st);
  const ba_ticket id = t->id;
  c->tickets[id] = std::move(t);
  c->queue.push_back(id);
  *ticket = id;
  return BA_OK;
}

}  // namespace

extern "C" {

int ba_step(ba_ctx* c, ba_ticket id, int32_t n_iters) {
  if (!c) return BA_E_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  if (c->dead) return fail(c, BA_E_DEVICE, "context is unusable after a device error");
  Ticket* t = find_ticket(c, id);
  if (!t) return fail(c, BA_E_ARG, "unknown ticket");
  if (n_iters < 0) return fail(c, BA_E_ARG, "negative iteration count");
  HIPCHK(c, hipSetDevice(c->device));
  std::vector<int> adm;
  int rc = ensure_resident(c, *t, adm);
  if (rc) return rc;
  if ((rc = start_slots(c, c->api, adm))) return rc;
  const std::vector<int> one{t->slot};
  if ((rc = read_ctl(c, c->api))) return rc;
  for (int i = 0; i < n_iters; ++i) {
    if (c->api.h_ctl[t->slot].status != ST_RUNNING) break;
    if ((rc = run_iterations(c, c->api, one, 1))) return rc;
    if ((rc = read_ctl(c, c->api))) return rc;
  }
  if (t->resident && !t->res_done && is_finished(c->api.h_ctl[t->slot].status)) return export_slots(c, c->api, one);
  return BA_OK;
}

int ba_solve_batch(ba_ctx* c, const ba_ticket* ids, int32_t n) {
  if (!c || (n > 0 && !ids) || n < 0) return BA_E_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  if (c->dead) return fail(c, BA_E_DEVICE, "context is unusable after a device error");
  HIPCHK(c, hipSetDevice(c->device));
  std::vector<int> adm, slots;
  for (int i = 0; i < n; ++i) {
    Ticket* t = find_ticket(c, ids[i]);
    if (!t) return fail(c, BA_E_ARG, "unknown ticket");
    int rc = ensure_resident(c, *t, adm);
    if (rc) return rc;
    slots.push_back(t->slot);
  }
  int rc = start_slots(c, c->api, adm);
  if (rc) return rc;
  if ((rc = read_ctl(c, c->api))) return rc;
  const int per = c->opt.iters_per_tick;
  for (;;) {
    std::vector<int> act;
    for (int s : slots)
      if (c->api.h_ctl[s].status == ST_RUNNING) act.push_back(s);
    if (act.empty()) break;
    if ((rc = run_tick(c, false, act, per))) return rc;
    if ((rc = read_ctl(c, c->api))) return rc;
  }
  std::vector<int> wb;
  for (int s : slots)
    if (c->tickets[c->slots[s].ticket]->resident && !c->tickets[c->slots[s].ticket]->res_done) wb.push_back(s);
  return wb.empty() ? BA_OK : export_slots(c, c->api, wb);
}

int ba_solve(ba_ctx* c, ba_ticket id) {
  if (!c) return BA_E_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  Ticket* t = find_ticket(c, id);
  if (!t) return fail(c, BA_E_ARG, "unknown ticket");
  if (!c->opt.serve) return fail(c, BA_E_STATE, "context has no serving loop");
  if (t->serving || t->state != TK_QUEUED) return fail(c, BA_E_STATE, "cluster is not queued");
  t->serving = true;
  c->cv.notify_all();
  return BA_OK;
}

int ba_wait(ba_ctx* c, ba_ticket id, double timeout_s) {
  if (!c) return BA_E_ARG;
  std::unique_lock<std::mutex> lk(c->mu);
  Ticket* t = find_ticket(c, id);
  if (!t) return fail(c, BA_E_ARG, "unknown ticket");
  if (!t->serving && t->state != TK_DONE) return fail(c, BA_E_STATE, "cluster was not handed to ba_solve");
  // the ticket may be released (and removed) while this thread waits
  auto pred = [&] {
    Ticket* x = find_ticket(c, id);
    return !x || x->state == TK_DONE || c->dead;
  };
  if (timeout_s < 0) c->done_cv.wait(lk, pred);
  else if (!c->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return BA_E_TIMEOUT;
  t = find_ticket(c, id);
  if (!t) return fail(c, BA_E_STATE, "cluster was released while waiting");
  if (c->dead && t->state != TK_DONE) return fail(c, BA_E_DEVICE, "serving loop stopped on a device error");
  return BA_OK;
}

int ba_fetch(ba_ctx* c, ba_ticket id, ba_result* r) {
  if (!c || !r) return BA_E_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  Ticket* t = find_ticket(c, id);
  if (!t) return fail(c, BA_E_ARG, "unknown ticket");
  if (t->serving) return fail(c, BA_E_STATE, "cluster is being solved by the serving loop");
  if (t->state == TK_QUEUED) return fail(c, BA_E_STATE, "cluster is still queued");
  if (t->state == TK_RESIDENT) {
    if (c->dead) return fail(c, BA_E_DEVICE, "context is unusable after a device error");
    HIPCHK(c, hipSetDevice(c->device));
    const std::vector<int> one{t->slot};
    int rc = export_slots(c, c->api, one);
    if (rc) return rc;
  }
  const int C = t->C, P = t->P;
  const double* o = t->out.data();
  if (r->R) std::memcpy(r->R, o, 9 * sizeof(double) * C);
  if (r->T) std::memcpy(r->T, o + 9 * C, 3 * sizeof(double) * C);
  if (r->X && P > 0) std::memcpy(r->X, o + 12 * C, 3 * sizeof(double) * P);
  if (r->k) std::memcpy(r->k, o + 12 * C + 3 * (size_t)P, 2 * sizeof(double));
  if (r->intr) std::memcpy(r->intr, o + 12 * C + 3 * (size_t)P + 2, 3 * sizeof(double));
  const SlotCtl& ctl = t->ctl;
  const int n_log = std::min(ctl.iter, t->max_iters) + 1;
  if (r->cost_log) {
    for (int i = 0; i <= t->max_iters; ++i) r->cost_log[i] = i < n_log ? t->cost_log[i] : NAN;
  }
  if (r->lambda_log)
    for (int i = 0; i < t->max_iters; ++i) r->lambda_log[i] = i < n_log - 1 ? t->lambda_log[i] : NAN;
  if (r->accepted_log)
    for (int i = 0; i < t->max_iters; ++i) r->accepted_log[i] = i < n_log - 1 ? t->acc_log[i] : -1;
  {
    // reprojection statistics from the sums of the exported state
    const double* st = o + 12 * C + 3 * (size_t)P + 5;
    const double n = st[0], ni = st[3];
    r->n_reproj = (int64_t)n;
    r->reproj_rms = n > 0 ? std::sqrt(st[2] / n) : NAN;
    r->reproj_mean = n > 0 ? st[1] / n : NAN;
    r->reproj_std = n > 0 ? std::sqrt(std::max(0.0, st[2] / n - r->reproj_mean * r->reproj_mean)) : NAN;
    r->n_inliers = (int64_t)ni;
    r->inlier_mean = ni > 0 ? st[4] / ni : NAN;
    r->inlier_std = ni > 0 ? std::sqrt(std::max(0.0, st[5] / ni - r->inlier_mean * r->inlier_mean)) : NAN;
  }
  r->nu = t->ctl.nu;
  r->status = ctl.status;
  r->iterations = ctl.iter;
  r->accepted = ctl.accepted;
  r->rejected = ctl.rejected;
  r->lambda = ctl.lambda;
  r->initial_cost = ctl.E0;
  r->final_cost = ctl.E;
  r->t_submit = t->t_submit;
  r->t_admit = t->t_admit;
  r->t_done = t->t_done;
  r->cg_iters = ctl.cg_iters;
  return BA_OK;
}

int ba_profile_enable(ba_ctx* c, int32_t kernels) {
  if (!c || (kernels & ~BA_PROF_ALL)) return BA_E_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  c->prof = kernels;
  return BA_OK;
}

int ba_profile_read(ba_ctx* c, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return BA_E_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  (void)hipSetDevice(c->device);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int rc = harvest_prof(c);
  if (rc) return rc;
  for (int k = 0; k < BA_PROF_N; ++k) {
    total_ms[k] = c->prof_ms[k];
    launches[k] = c->prof_n[k];
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  return BA_OK;
}

int ba_resident_poses(ba_ctx* c, int32_t n, const int64_t* ids, double* R, double* T, double* w) {
  if (!c) return BA_E_ARG;
  if (n < 0 || (n > 0 && (!ids || !R || !T))) return fail(c, BA_E_ARG, "bad resident pose query");
  std::lock_guard<std::mutex> g(c->mu);
  std::vector<int> rows(n);
  for (int i = 0; i < n; ++i) {
    const int* r = c->res_cam_row.find(ids[i]);
    if (!r) return fail(c, BA_E_ARG, "camera ID never submitted");
    const ba_ctx::ResRow& m = c->res_cam_meta[*r];
    if (m.pending) {
      auto pt = c->tickets.find(m.pending);
      if (pt != c->tickets.end() && !pt->second->res_done)
        return fail(c, BA_E_STATE, "camera ID has an unfinished writer");
    }
    if (!m.valid) return fail(c, BA_E_ARG, "camera ID never written back");
    rows[i] = *r;
  }
  if (n == 0) return BA_OK;
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double v[12], wr = 0.0;
  for (int i = 0; i < n; ++i) {
    const size_t r = (size_t)rows[i];
    HIPCHK(c, hipMemcpy(v, c->res_cam + 12 * r, sizeof(v), hipMemcpyDeviceToHost));
    std::copy(v, v + 9, R + 9 * (size_t)i);
    std::copy(v + 9, v + 12, T + 3 * (size_t)i);
    if (w) {
      HIPCHK(c, hipMemcpy(&wr, c->res_cam_w + r, sizeof(double), hipMemcpyDeviceToHost));
      w[i] = wr;
    }
  }
  return BA_OK;
}

int ba_release(ba_ctx* c, ba_ticket id) {
  if (!c) return BA_E_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  Ticket* t = find_ticket(c, id);
  if (!t) return fail(c, BA_E_ARG, "unknown ticket");
  if (t->serving) {   // cancelled: the serving loop drops it at its next tick boundary
    if (std::find(c->cancel.begin(), c->cancel.end(), id) == c->cancel.end()) c->cancel.push_back(id);
    c->cv.notify_all();
    return BA_OK;
  }
  if (t->state == TK_RESIDENT) {
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    free_slot(c, t->slot);
  }
  c->queue.erase(std::remove(c->queue.begin(), c->queue.end(), id), c->queue.end());
  c->tickets.erase(id);
  return BA_OK;
}

}  // extern "C"
