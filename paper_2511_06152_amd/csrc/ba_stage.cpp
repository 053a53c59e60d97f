// Host layout of a submitted cluster: validation and the work lists the
// kernels read (ba_stage.h).  Plain C++: no HIP.
#include "ba_stage.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>

namespace bagpu {

namespace {

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

I4 mk4(int kind, int a, int b, int y, int z) { return I4{(kind << 24) | (a << 12) | b, y, z, 0}; }

// Spreads the 16 low bits of x to the even bit positions.
uint32_t spread16(uint32_t x) {
  x &= 0xffffu;
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

// Scratch arrays of one layout, kept per thread so that a thread that lays
// out cluster after cluster reuses their storage.
struct Work {
  std::vector<int> nobs, inv, opt, cnt, order, by_cam, cc, fill, scam, spt, oblane, free_cam, coff, cbase, cend, pcount,
      pbase, brow0, sfree;
  std::vector<uint64_t> kj, tmp;
  std::vector<double> suv;
  std::vector<I2> cam_range, blk_range;
};

template <typename T, typename A>
void keep_storage(std::vector<T, A>& dst, std::vector<T, A>& src) {
  dst.swap(src);
  dst.clear();
}

}  // namespace

void reset_keep(Staged& s) {
  Staged f;
  keep_storage(f.raw_cam, s.raw_cam);
  keep_storage(f.X, s.X);
  keep_storage(f.pt_orig, s.pt_orig);
  keep_storage(f.cam_col, s.cam_col);
  keep_storage(f.pchunk, s.pchunk);
  keep_storage(f.wg_chunk, s.wg_chunk);
  keep_storage(f.ob_cam, s.ob_cam);
  keep_storage(f.ob_uv, s.ob_uv);
  keep_storage(f.cl_pt, s.cl_pt);
  keep_storage(f.cl_ob, s.cl_ob);
  keep_storage(f.ql_pt, s.ql_pt);
  keep_storage(f.ql_ob, s.ql_ob);
  keep_storage(f.tasks, s.tasks);
  keep_storage(f.targets, s.targets);
  keep_storage(f.brow, s.brow);
  keep_storage(f.bcol, s.bcol);
  keep_storage(f.tslot, s.tslot);
  keep_storage(f.cam_ids, s.cam_ids);
  keep_storage(f.point_ids, s.point_ids);
  keep_storage(f.cam_nobs, s.cam_nobs);
  s = std::move(f);
}

uint64_t mix_id(int64_t id) {
  uint64_t z = (uint64_t)id + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

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
  reset_keep(s);
  thread_local Work w;
  // the scratch of a very large cluster (a whole flight) is not kept
  struct Trim {
    Work& w;
    bool big;
    ~Trim() { if (big) w = Work(); }
  } trim{w, (size_t)O > kKeepObs};
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
  // Internal point order: by the number of observations, then Morton (z-)
  // order of the initial ground position, so that the 64 points of a
  // point chunk have the same observation count and a camera's observations
  // touch nearby point records.  Ties keep the caller's order (LSD radix sort
  // of key << 32 | index on the key bits, then a stable counting sort by count).
  std::vector<int>& nobs = w.nobs;
  nobs.assign(P, 0);
  for (int o = 0; o < O; ++o)
    if (++nobs[c->obs_pt[o]] > BA_MAX_OBS_PER_POINT) { err = "more than 64 observations of one point"; return BA_E_ARG; }
  {
    double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
    for (int j = 0; j < P; ++j)
      for (int t = 0; t < 2; ++t) {
        lo[t] = std::min(lo[t], c->X[3 * (size_t)j + t]);
        hi[t] = std::max(hi[t], c->X[3 * (size_t)j + t]);
      }
    std::vector<uint64_t>& kj = w.kj;
    std::vector<uint64_t>& tmp = w.tmp;
    kj.resize(P);
    tmp.resize(P);
    for (int j = 0; j < P; ++j) {
      uint32_t q[2];
      for (int t = 0; t < 2; ++t) {
        const double span = hi[t] - lo[t];
        const double u = span > 0 ? (c->X[3 * (size_t)j + t] - lo[t]) / span : 0.0;
        q[t] = (uint32_t)std::min(65535.0, std::max(0.0, u * 65535.0));
      }
      const uint32_t k = spread16(q[0]) | spread16(q[1]) << 1;   // x bits even, y bits odd
      kj[j] = (uint64_t)k << 32 | (uint32_t)j;
    }
    for (int shift = 32; shift < 64; shift += 11) {
      size_t cnt_d[2049] = {0};
      for (int j = 0; j < P; ++j) ++cnt_d[((kj[j] >> shift) & 2047u) + 1];
      for (int d = 0; d < 2048; ++d) cnt_d[d + 1] += cnt_d[d];
      for (int j = 0; j < P; ++j) tmp[cnt_d[(kj[j] >> shift) & 2047u]++] = kj[j];
      kj.swap(tmp);
    }
    int cls[BA_MAX_OBS_PER_POINT + 2] = {0};
    for (int j = 0; j < P; ++j) ++cls[nobs[j] + 1];
    for (int n = 0; n <= BA_MAX_OBS_PER_POINT; ++n) cls[n + 1] += cls[n];
    s.pt_orig.resize(P);
    for (int r = 0; r < P; ++r) {
      const int j = (int)(uint32_t)kj[r];
      s.pt_orig[cls[nobs[j]]++] = j;
    }
  }
  std::vector<int>& inv = w.inv;
  std::vector<int>& opt = w.opt;
  inv.resize(P);
  opt.resize(O);
  for (int n = 0; n < P; ++n) inv[s.pt_orig[n]] = n;
  for (int o = 0; o < O; ++o) opt[o] = inv[c->obs_pt[o]];
  s.X.resize(3 * (size_t)P);
  for (int n = 0; n < P; ++n)
    for (int t = 0; t < 3; ++t) s.X[3 * (size_t)n + t] = c->X[3 * (size_t)s.pt_orig[n] + t];
  // observations per point (internal order)
  std::vector<int>& cnt = w.cnt;
  cnt.assign(P + 1, 0);
  for (int n = 0; n < P; ++n) cnt[n + 1] = cnt[n] + nobs[s.pt_orig[n]];
  // observations in (point, camera) order: a counting sort by camera, then a
  // stable one by point; then their camera, pixel and point in that order
  std::vector<int>& order = w.order;
  order.resize(O);
  {
    std::vector<int>& by_cam = w.by_cam;
    std::vector<int>& cc = w.cc;
    by_cam.resize(O);
    cc.assign(C + 1, 0);
    for (int o = 0; o < O; ++o) ++cc[c->obs_cam[o] + 1];
    for (int k = 0; k < C; ++k) cc[k + 1] += cc[k];
    for (int o = 0; o < O; ++o) by_cam[cc[c->obs_cam[o]]++] = o;
    std::vector<int>& fill = w.fill;
    fill.assign(cnt.begin(), cnt.end() - 1);
    for (int t = 0; t < O; ++t) order[fill[opt[by_cam[t]]]++] = by_cam[t];
  }
  std::vector<int>& scam = w.scam;
  std::vector<int>& spt = w.spt;
  std::vector<double>& suv = w.suv;
  scam.resize(O);
  spt.resize(O);
  suv.resize(2 * (size_t)O);
  for (int j = 0; j < P; ++j)
    for (int t = cnt[j]; t < cnt[j + 1]; ++t) {
      const int o = order[t];
      scam[t] = c->obs_cam[o];
      spt[t] = j;
      suv[2 * (size_t)t] = c->obs_uv[2 * (size_t)o];
      suv[2 * (size_t)t + 1] = c->obs_uv[2 * (size_t)o + 1];
      if (t > cnt[j] && scam[t] == scam[t - 1]) { err = "a camera observes one point twice"; return BA_E_ARG; }
    }
  // point chunks: 64 consecutive points of one observation count n, their
  // observations stored observation-major (observation t of the chunk's lane l
  // at first + 64 t + l); the last chunk of a count is padded with lanes
  // that hold camera 0 and pixel 0
  for (int pb = 0; pb < P;) {
    const int n = cnt[pb + 1] - cnt[pb];
    int pe = pb + 1;
    while (pe < P && cnt[pe + 1] - cnt[pe] == n) ++pe;
    if (n > 0)
      for (int p0 = pb; p0 < pe; p0 += kWave) {
        s.pchunk.push_back(I4{s.L, n, p0, std::min(kWave, pe - p0)});
        s.L += kWave * n;
      }
    pb = pe;
  }
  s.n_chunks = (int)s.pchunk.size();
  s.ob_cam.resize(s.L);
  s.ob_uv.resize(2 * (size_t)s.L);
  std::vector<int>& oblane = w.oblane;   // observation lane of each observation in (point, camera) order
  oblane.resize(O);
  for (const I4& ch : s.pchunk) {
    for (int l = 0; l < ch.w; ++l)
      for (int t = 0; t < ch.y; ++t) {
        const int so = cnt[ch.z + l] + t;
        const int lane = ch.x + kWave * t + l;
        oblane[so] = lane;
        s.ob_cam[lane] = scam[so];
        s.ob_uv[2 * (size_t)lane] = suv[2 * (size_t)so];
        s.ob_uv[2 * (size_t)lane + 1] = suv[2 * (size_t)so + 1];
      }
    for (int l = ch.w; l < kWave; ++l)   // padding lanes
      for (int t = 0; t < ch.y; ++t) {
        const int lane = ch.x + kWave * t + l;
        s.ob_cam[lane] = 0;
        s.ob_uv[2 * (size_t)lane] = 0.0;
        s.ob_uv[2 * (size_t)lane + 1] = 0.0;
      }
  }
  // point-pass workgroups: runs of whole chunks holding at least cpw * 64
  // observation lanes each
  s.wg_chunk.assign(1, 0);
  for (int ch = 0, lanes = 0; ch < s.n_chunks; ++ch) {
    lanes += kWave * s.pchunk[ch].y;
    if (lanes >= cpw * kWave || ch + 1 == s.n_chunks) {
      s.wg_chunk.push_back(ch + 1);
      lanes = 0;
    }
  }
  s.n_wg = (int)s.wg_chunk.size() - 1;
  const bool intr = s.m > 6 * s.n_free;   // an intrinsic is estimated
  s.n_pt_part = intr ? s.n_wg * kWavesPerWG : 0;
  s.nb = (s.m + kSolveTb - 1) / kSolveTb;
  const int F = s.n_free;
  std::vector<int>& free_cam = w.free_cam;
  free_cam.resize(F);
  for (int k = 0; k < C; ++k)
    if (s.cam_col[k] >= 0) free_cam[s.cam_col[k] / 6] = k;
  // camera lanes and tasks: each free camera's observations in point order,
  // each lane naming its point and its observation lane
  std::vector<int>& sfree = w.sfree;   // free-camera index of each observation, -1 for a fixed camera
  sfree.resize(O);
  std::vector<int>& coff = w.coff;
  coff.assign(F + 1, 0);
  for (int t = 0; t < O; ++t) {
    const int col = s.cam_col[scam[t]];
    sfree[t] = col < 0 ? -1 : col / 6;
    if (col >= 0) ++coff[col / 6 + 1];
  }
  std::vector<int>& cbase = w.cbase;   // first lane of each camera's run
  cbase.assign(F + 1, 0);
  for (int fi = 0; fi < F; ++fi) cbase[fi + 1] = cbase[fi] + (int)align_up(coff[fi + 1], kWave);
  s.Lc = cbase[F];
  s.cl_pt.resize(s.Lc);
  s.cl_ob.resize(s.Lc);
  {
    std::vector<int>& fill = w.fill;
    fill.assign(cbase.begin(), cbase.end() - 1);
    for (int t = 0; t < O; ++t) {
      if (sfree[t] < 0) continue;
      const int lane = fill[sfree[t]]++;
      s.cl_pt[lane] = spt[t];
      s.cl_ob[lane] = oblane[t];
    }
    for (int fi = 0; fi < F; ++fi)   // padding lanes: point -1, observation lane 0
      for (int l = fill[fi]; l < cbase[fi + 1]; ++l) s.cl_pt[l] = -1, s.cl_ob[l] = 0;
  }
  std::vector<I2>& cam_range = w.cam_range;
  cam_range.resize(F);
  for (int fi = 0; fi < F; ++fi) {
    const int base = cbase[fi] / kWave, nch = (cbase[fi + 1] - cbase[fi]) / kWave;
    cam_range[fi].x = (int)s.tasks.size();
    for (int ch = 0; ch < nch; ch += cpt) s.tasks.push_back(mk4(TASK_CAM, free_cam[fi], 0, base + ch, std::min(cpt, nch - ch)));
    cam_range[fi].y = (int)s.tasks.size();
  }
  s.n_cam_tasks = (int)s.tasks.size();
  // pair lanes and tasks, blocks (fa < fb) in row-major upper-triangle order;
  // within a block the pairs in point order, each lane naming its point and
  // the observation lanes of its two observations
  const int nblk = F * (F - 1) / 2;
  auto blk = [F](int fa, int fb) { return fa * F - fa * (fa + 1) / 2 + (fb - fa - 1); };
  std::vector<int>& brow0 = w.brow0;   // block of (fa, fb) = brow0[fa] + fb
  brow0.resize(F);
  for (int fa = 0; fa < F; ++fa) brow0[fa] = blk(fa, fa + 1) - (fa + 1);
  std::vector<int>& pcount = w.pcount;
  pcount.assign(nblk, 0);
  for (int j = 0; j < P; ++j)
    for (int ta = cnt[j]; ta < cnt[j + 1]; ++ta) {
      const int fa = sfree[ta];
      if (fa < 0) continue;
      for (int tb = ta + 1; tb < cnt[j + 1]; ++tb)
        if (sfree[tb] >= 0) ++pcount[brow0[fa] + sfree[tb]];
    }
  std::vector<int>& pbase = w.pbase;   // first lane of each block's run
  pbase.assign(nblk + 1, 0);
  for (int b = 0; b < nblk; ++b) pbase[b + 1] = pbase[b] + (int)align_up(pcount[b], kWave);
  s.Lq = pbase[nblk];
  s.ql_pt.resize(s.Lq);
  s.ql_ob.resize(s.Lq);
  {
    std::vector<int>& fill = w.fill;
    fill.assign(pbase.begin(), pbase.end() - 1);
    for (int j = 0; j < P; ++j)
      for (int ta = cnt[j]; ta < cnt[j + 1]; ++ta) {
        const int fa = sfree[ta];
        if (fa < 0) continue;
        int* row = fill.data() + brow0[fa];
        for (int tb = ta + 1; tb < cnt[j + 1]; ++tb) {
          const int fb = sfree[tb];
          if (fb < 0) continue;
          const int lane = row[fb]++;
          s.ql_pt[lane] = j;
          s.ql_ob[lane] = I2{oblane[ta], oblane[tb]};
        }
      }
    for (int b = 0; b < nblk; ++b)   // padding lanes: point -1, observation lanes 0
      for (int l = fill[b]; l < pbase[b + 1]; ++l) s.ql_pt[l] = -1, s.ql_ob[l] = I2{0, 0};
  }
  auto blk_empty = [&](int b) { return pcount[b] == 0; };
  std::vector<I2>& blk_range = w.blk_range;
  blk_range.resize(nblk);
  for (int fa = 0; fa < F; ++fa)
    for (int fb = fa + 1; fb < F; ++fb) {
      const int b = blk(fa, fb);
      const int base = pbase[b] / kWave, nch = (pbase[b + 1] - pbase[b]) / kWave;
      blk_range[b].x = (int)s.tasks.size();
      for (int ch = 0; ch < nch; ch += cpt)
        s.tasks.push_back(mk4(TASK_PAIR, free_cam[fa], free_cam[fb], base + ch, std::min(cpt, nch - ch)));
      blk_range[b].y = (int)s.tasks.size();
    }
  for (int fi = 0; fi < F; ++fi) s.targets.push_back(mk4(TASK_CAM, free_cam[fi], 0, cam_range[fi].x, cam_range[fi].y));
  if (!s.sparse) {
    for (int fa = 0; fa < F; ++fa)
      for (int fb = fa + 1; fb < F; ++fb) {
        const I2 r = blk_range[blk(fa, fb)];
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
  for (int fi = 0; fi < F; ++fi) s.tslot.push_back(I2{diag_slot[fi], diag_slot[fi]});
  for (int fa = 0; fa < F; ++fa)
    for (int fb = fa + 1; fb < F; ++fb) {
      if (blk_empty(blk(fa, fb))) continue;
      const I2 r = blk_range[blk(fa, fb)];
      s.targets.push_back(mk4(TASK_PAIR, free_cam[fa], free_cam[fb], r.x, r.y));
      s.tslot.push_back(I2{slot_of[{fa, fb}], slot_of[{fb, fa}]});
    }
  return BA_OK;
}

}  // namespace bagpu
