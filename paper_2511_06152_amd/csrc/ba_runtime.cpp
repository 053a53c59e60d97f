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
#include "ba_stage.h"

using namespace bagpu;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

static_assert(sizeof(I4) == sizeof(int4) && sizeof(I2) == sizeof(int2), "layout tuples are uploaded as int4 / int2");

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

// Block rows of each conjugate-gradient workgroup: consecutive rows, at most
// min(ceil(F / 16), kCgMaxRows) per workgroup (about 16 workgroups: every
// conjugate-gradient step pays a grid barrier whose cost grows with the
// workgroup count, and on the 400-camera flight 16 beat 32, 64 and 128), and
// no more than keep the workgroup's blocks and block columns, the direction
// p and the row work of the most rows any workgroup may get in 150 KB of
// dynamic LDS (the kernel's static LDS, under 5 KB, fits in the rest of the
// 160 KB).  False when a single block row does not fit or more than
// kMaxCgWG workgroups would be needed.
bool pcg_partition(const Staged& s, bool mixed, std::vector<int>& part, int& rows_max, size_t& smem) {
  part.clear();
  rows_max = 0;
  smem = 0;
  if (!s.sparse) return true;
  const int F = s.n_free, m = s.m;
  // bytes per block in LDS: its values and its block column
  const size_t bb = (mixed ? 4 : 8) * (size_t)kSbVals + sizeof(int), budget = 150 * 1024;
  const int cap = std::max(1, std::min(kCgMaxRows, (F + 15) / 16));
  // p (FP64 and FP32 copy), and 27 values per row (S p rows, preconditioner)
  // for up to cap rows
  const size_t fixed = 8 * ((size_t)m + 4 * (size_t)F) + 216 * (size_t)cap;
  part.push_back(0);
  int rows = 0;
  size_t bytes = 0;
  for (int f = 0; f < F; ++f) {
    const size_t rb = bb * (size_t)(s.brow[f + 1] - s.brow[f]);
    if (rows > 0 && (rows == cap || fixed + bytes + rb > budget)) {
      part.push_back(f);
      rows = 0;
      bytes = 0;
    }
    if (fixed + rb > budget) return false;
    bytes += rb;
    ++rows;
    rows_max = std::max(rows_max, rows);
    smem = std::max(smem, pcg_lds_bytes(bytes, m, F, 0));
  }
  part.push_back(F);
  if ((int)part.size() - 1 > kMaxCgWG) return false;
  smem += 8 * 27 * (size_t)rows_max;
  return true;
}


// Byte offsets inside a slot block.  The arrays taken from the host come
// first, [0, upload_end), so that one copy of the cluster's upload image
// fills them; the arrays the device computes follow.
struct Layout {
  size_t pchunk, wg_chunk, ob_cam, uv64, uv32, cl_pt, cl_ob, ql_pt, ql_ob, tasks, targets,
      cam0, cam1, prior, pterm0, pterm1, cam_col, raw_cam, X0, X1, X320, X321, ptv, ptd, ptz, pt_orig, task_part, pt_part, Sg, Sd, dc,
      brow, bcol, tslot, Sblk, Sblk32, pcgw, pcg_part, rin_cam, rin_pt, rout_cam, rout_pt, cost_part,
      bad_part, cost_log, lambda_log, acc_log, stat_part, out, upload_end, total;
  int n_wg, psize, pstride;
  std::vector<int> part;         // conjugate-gradient workgroups' first block rows
  int pcg_rows_max;
  size_t pcg_smem;
  bool pcg_ok;
};

Layout make_layout(const Staged& s, bool mixed) {
  Layout l{};
  const size_t rs = real_size(mixed);
  l.n_wg = s.n_wg;
  // the sparse form keeps no packed triangle: Sg holds g, bS, diag U only
  // dense: the system in 16x16 blocks (lower block triangle, rows padded to 17)
  l.psize = s.sparse ? 0 : s.nb * (s.nb + 1) / 2 * kSolveTb * (kSolveTb + 1);
  l.pstride = (int)align_up((size_t)l.psize + 3 * (size_t)s.m, 4);
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes, 256); return at; };
  l.pcg_ok = pcg_partition(s, mixed, l.part, l.pcg_rows_max, l.pcg_smem);
  const size_t nnzb = s.bcol.size();
  // from the host (the camera and pair lanes name observation lanes; their
  // pixels are read from those)
  l.pchunk = take(sizeof(int4) * s.pchunk.size());
  l.wg_chunk = take(4 * s.wg_chunk.size());
  l.ob_cam = take(4 * (size_t)s.L);
  l.uv64 = take(16 * (size_t)s.L);
  l.cl_pt = take(4 * (size_t)s.Lc);
  l.cl_ob = take(4 * (size_t)s.Lc);
  l.ql_pt = take(4 * (size_t)s.Lq);
  l.ql_ob = take(8 * (size_t)s.Lq);
  l.tasks = take(sizeof(int4) * s.tasks.size());
  l.targets = take(sizeof(int4) * s.targets.size());
  l.cam_col = take(4 * (size_t)s.C);
  l.raw_cam = take(8 * 30 * (size_t)s.C);
  l.X0 = take(24 * (size_t)s.P);
  l.pt_orig = take(4 * (size_t)s.P);
  l.brow = take(4 * s.brow.size());
  l.bcol = take(4 * nnzb);
  l.tslot = take(sizeof(int2) * s.tslot.size());
  l.pcg_part = take(4 * l.part.size());
  l.upload_end = o;
  // computed on the device
  l.uv32 = take(8 * (size_t)s.L);
  l.cam0 = take(8 * (size_t)kCamVals * s.C);
  l.cam1 = take(8 * (size_t)kCamVals * s.C);
  l.prior = take(8 * (size_t)kPriorVals * s.C);
  l.pterm0 = take(8 * (size_t)kPtermVals * s.C);
  l.pterm1 = take(8 * (size_t)kPtermVals * s.C);
  l.X1 = take(24 * (size_t)s.P);
  l.X320 = take(12 * (size_t)s.P);
  l.X321 = take(12 * (size_t)s.P);
  l.ptv = take(rs * kPtVals * (size_t)s.P);
  l.ptd = take(rs * 4 * (size_t)s.P);
  l.ptz = take(s.sc ? rs * kPtzVals * (size_t)s.P : 0);
  l.task_part = take(rs * kTaskVals * s.tasks.size());
  l.pt_part = take(rs * kPtPartVals * (size_t)s.n_pt_part);
  l.Sg = take(8 * (size_t)l.pstride);
  l.Sd = take(s.sparse ? 0 : 8 * kSolveTbVals * (size_t)s.nb * (s.nb + 1) / 2);
  l.dc = take(8 * (size_t)s.m);
  l.Sblk = take(8 * (size_t)kSbVals * nnzb);
  l.Sblk32 = take(4 * (size_t)kSbVals * nnzb);
  l.pcgw = take(s.sparse ? 8 * (7 * (size_t)s.m + 20 * (size_t)kMaxCgWG + 8) : 0);
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

// Writes the cluster's upload image: every array the slot block takes from
// the host, at its offset below lay.upload_end (the alignment gaps are left
// as they are).
void pack_upload(const Staged& s, const Layout& lay, char* dst) {
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(dst + off, src, bytes);
  };
  put(lay.pchunk, s.pchunk.data(), sizeof(int4) * s.pchunk.size());
  put(lay.wg_chunk, s.wg_chunk.data(), 4 * s.wg_chunk.size());
  put(lay.ob_cam, s.ob_cam.data(), 4 * (size_t)s.L);
  put(lay.uv64, s.ob_uv.data(), 16 * (size_t)s.L);
  put(lay.cl_pt, s.cl_pt.data(), 4 * (size_t)s.Lc);
  put(lay.cl_ob, s.cl_ob.data(), 4 * (size_t)s.Lc);
  put(lay.ql_pt, s.ql_pt.data(), 4 * (size_t)s.Lq);
  put(lay.ql_ob, s.ql_ob.data(), 8 * (size_t)s.Lq);
  put(lay.tasks, s.tasks.data(), sizeof(I4) * s.tasks.size());
  put(lay.targets, s.targets.data(), sizeof(I4) * s.targets.size());
  put(lay.cam_col, s.cam_col.data(), 4 * (size_t)s.C);
  put(lay.raw_cam, s.raw_cam.data(), 8 * 30 * (size_t)s.C);
  put(lay.X0, s.X.data(), 24 * (size_t)s.P);
  put(lay.pt_orig, s.pt_orig.data(), 4 * (size_t)s.P);
  put(lay.brow, s.brow.data(), 4 * s.brow.size());
  put(lay.bcol, s.bcol.data(), 4 * s.bcol.size());
  put(lay.tslot, s.tslot.data(), sizeof(I2) * s.tslot.size());
  put(lay.pcg_part, lay.part.data(), 4 * lay.part.size());
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

enum TicketState { TK_QUEUED, TK_RESIDENT, TK_DONE, TK_INVALID };

// A submitted cluster's arrays, copied for background layout (stage_threads > 0).
struct ClusterCopy {
  ba_cluster c{};
  std::vector<double> R, T, X, k, prior_R, prior_T, prior_sigma, obs_uv;
  std::vector<uint8_t> fixed;
  std::vector<int32_t> obs_cam, obs_pt;
  std::vector<int64_t> cam_ids, point_ids;
  explicit ClusterCopy(const ba_cluster& in) : c(in) {
    const size_t C = (size_t)in.n_cams, P = (size_t)in.n_points, O = (size_t)in.n_obs;
    auto cp = [](auto& v, const auto* src, size_t n) {
      if (src) v.assign(src, src + n);
      return src ? v.data() : nullptr;
    };
    c.R = cp(R, in.R, 9 * C);
    c.T = cp(T, in.T, 3 * C);
    c.X = cp(X, in.X, 3 * P);
    c.k = cp(k, in.k, 2);
    c.prior_R = cp(prior_R, in.prior_R, 9 * C);
    c.prior_T = cp(prior_T, in.prior_T, 3 * C);
    c.prior_sigma = cp(prior_sigma, in.prior_sigma, 6 * C);
    c.fixed = cp(fixed, in.fixed, C);
    c.obs_cam = cp(obs_cam, in.obs_cam, O);
    c.obs_pt = cp(obs_pt, in.obs_pt, O);
    c.obs_uv = cp(obs_uv, in.obs_uv, 2 * O);
    c.cam_ids = cp(cam_ids, in.cam_ids, C);
    c.point_ids = cp(point_ids, in.point_ids, P);
  }
};

struct Ticket {
  ba_ticket id = 0;
  TicketState state = TK_QUEUED;
  bool serving = false;           // owned by the serving loop until done
  bool staging = false;           // laid out in the background; not admissible yet
  int err_code = 0;               // TK_INVALID: why the background layout refused it
  std::string err_msg;
  std::unique_ptr<Staged> staged; // until admission
  int staged_home = -1;           // the layout thread whose pool the Staged returns to
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
  bool early = false;        // admitted during a tick: uploaded and set up on up_stream, joins at the next boundary
  ba_ticket ticket = 0;
  size_t off = 0, bytes = 0;
  Layout lay{};
  SlotDesc desc{};
  bool mixed = false;
  // sources of the admission's small uploads, kept until the slot is freed
  SlotCtl ctl0{};
  std::vector<int2> rin_c, rin_p, rout_p;
  std::vector<int4> rout_c;
};

// Per-launcher device batch arrays and pinned mirrors.
struct Launcher {
  int* d_act = nullptr;
  int* d_wgoff = nullptr;   // [4][max_slots + 1]: point-chunk, camera-task, pair-task, target workgroup prefixes
  // pinned: kRing batch images, each [max_slots] act, then [4][max_slots + 1]
  // prefixes; consecutive batches use consecutive images, so that building
  // one seldom waits for the upload of the one before
  static constexpr int kRing = 4;
  int* h_act = nullptr;
  SlotCtl* h_ctl = nullptr; // pinned readback of all slots' control blocks
  hipEvent_t ev = nullptr;
  hipEvent_t copy_ev[kRing] = {};   // after the last upload from each image
  hipEvent_t exp_ev = nullptr;      // after the copies of the last export
  bool copy_pending[kRing] = {};
  int ring = 0;                     // the image the next batch is built in
  std::vector<SparseLaunch> sp;  // the batch's clusters solved by conjugate gradients
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
  // serving loop: clusters admitted while a tick runs are uploaded and set
  // up on their own stream (up_ev after the last of that work) and join at
  // the next boundary; exports of finished clusters run there too
  hipStream_t up_stream = nullptr;
  hipEvent_t up_ev = nullptr;
  // batch lists of the serving loop's work on up_stream: the set-up of
  // clusters admitted during a tick and the export of finished ones
  Launcher side;
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
  // background layout (ba_options.stage_threads > 0)
  std::vector<std::unique_ptr<Staged>> staged_pool;   // admitted layouts kept for reuse (mu)
  // the same, per layout thread: a thread lays its next cluster out in
  // storage it wrote last (measured: 1.66 -> 1.30 ms per paper-scale layout
  // in the serving loop, against one shared pool)
  std::vector<std::vector<std::unique_ptr<Staged>>> worker_pool;
  std::vector<std::thread> stagers;
  std::deque<std::pair<ba_ticket, std::unique_ptr<ClusterCopy>>> stage_jobs;
  std::condition_variable stage_cv;       // wakes the layout threads
  std::condition_variable staged_cv;      // a background layout finished
  bool stage_stop = false;
  // Pinned host buffers for the clusters' upload images (pin_mu): free ones
  // (buffer, capacity), the bytes allocated, and the buffers of uploads in
  // flight with the event that marks each upload's end.
  std::mutex pin_mu;
  std::vector<std::pair<char*, size_t>> pin_free;
  size_t pin_bytes = 0;
  struct PinFlight { std::shared_ptr<char> blob; hipEvent_t ev; };
  std::vector<PinFlight> pin_flight;
  std::vector<hipEvent_t> pin_events;     // idle events for pin_flight
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

// Pinned host memory for upload images: at most kPinnedPoolBytes in all, the
// buffers reused across clusters (capacities powers of two from 2 MiB).
constexpr size_t kPinnedPoolBytes = 256u << 20;

// Returns the buffers of finished uploads to the free list.
void pin_reap(ba_ctx* c) {
  std::vector<std::shared_ptr<char>> done;   // dropped on return, after pin_mu is released
  std::lock_guard<std::mutex> g(c->pin_mu);
  for (size_t i = 0; i < c->pin_flight.size();) {
    if (hipEventQuery(c->pin_flight[i].ev) == hipSuccess) {
      c->pin_events.push_back(c->pin_flight[i].ev);
      done.push_back(std::move(c->pin_flight[i].blob));
      c->pin_flight[i] = std::move(c->pin_flight.back());
      c->pin_flight.pop_back();
    } else {
      ++i;
    }
  }
}

// A pinned buffer of at least `bytes` (returned to the pool when the last
// pointer to it is dropped), or null when the pool is full.
std::shared_ptr<char> pin_get(ba_ctx* c, size_t bytes) {
  pin_reap(c);
  char* p = nullptr;
  size_t have = 0;
  {
    std::lock_guard<std::mutex> g(c->pin_mu);
    int best = -1;
    for (int i = 0; i < (int)c->pin_free.size(); ++i)
      if (c->pin_free[i].second >= bytes && (best < 0 || c->pin_free[i].second < c->pin_free[best].second)) best = i;
    if (best >= 0) {
      p = c->pin_free[best].first;
      have = c->pin_free[best].second;
      c->pin_free.erase(c->pin_free.begin() + best);
    } else {
      // sizes in powers of two from 2 MiB, so that a freed buffer serves the
      // next clusters of similar size (a new pinned allocation takes
      // milliseconds)
      have = size_t(2) << 20;
      while (have < bytes) have <<= 1;
      if (c->pin_bytes + have > kPinnedPoolBytes) return nullptr;
      c->pin_bytes += have;
    }
  }
  if (!p && hipHostMalloc((void**)&p, have, hipHostMallocDefault) != hipSuccess) {
    std::lock_guard<std::mutex> g(c->pin_mu);
    c->pin_bytes -= have;
    return nullptr;
  }
  return std::shared_ptr<char>(p, [c, have](char* q) {
    std::lock_guard<std::mutex> g(c->pin_mu);
    c->pin_free.emplace_back(q, have);
  });
}

// Behind a cluster's upload image, at admission: the slot's descriptor and
// initial control block, so that they too are copied from pinned memory
// (an asynchronous copy; one from ordinary memory can hold the admitting
// thread until the stream has drained).
constexpr size_t kTailDesc = (sizeof(SlotDesc) + 63) / 64 * 64;
constexpr size_t kTailBytes = 64 + kTailDesc + (sizeof(SlotCtl) + 63) / 64 * 64;
size_t tail_off(size_t image_bytes) { return (image_bytes + 63) / 64 * 64; }

// Packs the cluster's upload image: into pinned memory when the pool has
// room (its upload at admission is then asynchronous), else into ordinary
// memory.
void pack_staged(ba_ctx* c, Staged& s, const Layout& lay) {
  std::shared_ptr<char> b;
  if (lay.upload_end <= kPinnedPoolBytes / 4) b = pin_get(c, lay.upload_end + kTailBytes);
  s.blob_pinned = b != nullptr;
  if (!b) b = std::shared_ptr<char>(new char[lay.upload_end + kTailBytes], std::default_delete<char[]>());
  pack_upload(s, lay, b.get());
  s.blob = std::move(b);
  s.blob_bytes = lay.upload_end;
}

int init_launcher(ba_ctx* c, Launcher& l) {
  const int S = c->opt.max_slots;
  HIPCHK(c, dmalloc(c, (void**)&l.d_act, sizeof(int) * S));
  HIPCHK(c, dmalloc(c, (void**)&l.d_wgoff, sizeof(int) * 4 * (S + 1)));
  HIPCHK(c, hipHostMalloc(&l.h_act, sizeof(int) * (S + 4 * (S + 1)) * Launcher::kRing, hipHostMallocDefault));
  HIPCHK(c, hipHostMalloc(&l.h_ctl, sizeof(SlotCtl) * S, hipHostMallocDefault));
  HIPCHK(c, hipEventCreateWithFlags(&l.ev, hipEventDisableTiming));
  for (hipEvent_t& e : l.copy_ev) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  HIPCHK(c, hipEventCreateWithFlags(&l.exp_ev, hipEventDisableTiming));
  return BA_OK;
}

void free_launcher(ba_ctx* c, Launcher& l) {
  dfree(c, l.d_act);
  dfree(c, l.d_wgoff);
  if (l.h_act) (void)hipHostFree(l.h_act);
  if (l.h_ctl) (void)hipHostFree(l.h_ctl);
  if (l.ev) (void)hipEventDestroy(l.ev);
  for (hipEvent_t e : l.copy_ev)
    if (e) (void)hipEventDestroy(e);
  if (l.exp_ev) (void)hipEventDestroy(l.exp_ev);
  l = Launcher();
}

// Builds and uploads the batch arrays of the given slots on launcher l.
int make_batch(ba_ctx* c, Launcher& l, const std::vector<int>& slots, Batch& b, hipStream_t st = nullptr) {
  if (!st) st = c->stream;
  const int S = c->opt.max_slots;
  const int r = l.ring;
  l.ring = (l.ring + 1) % Launcher::kRing;
  int* act = l.h_act + (size_t)r * (S + 4 * (S + 1));
  int* off = act + S;
  // The image is rewritten below: the upload last made from it must have
  // been executed by the stream first.
  if (l.copy_pending[r]) {
    HIPCHK(c, hipEventSynchronize(l.copy_ev[r]));
    l.copy_pending[r] = false;
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
  l.sp.clear();
  int tot = 0, tc = 0, tp = 0, tg = 0;
  for (int i = 0; i < b.n_act; ++i) {
    const Slot& sl = c->slots[slots[i]];
    if (sl.desc.sparse) l.sp.push_back(SparseLaunch{slots[i], sl.desc.pcg_G, sl.desc.pcg_smem});
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
  HIPCHK(c, hipMemcpyAsync(l.d_act, act, sizeof(int) * b.n_act, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(l.d_wgoff, off, sizeof(int) * 4 * (S + 1), hipMemcpyHostToDevice, st));
  HIPCHK(c, hipEventRecord(l.copy_ev[r], st));
  l.copy_pending[r] = true;
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

// A Staged for the next layout: a recycled one (its vectors keep their
// storage) when the pool has one; `worker` >= 0: layout thread `worker`,
// which takes from its own pool.  Caller holds mu.
std::unique_ptr<Staged> take_staged(ba_ctx* c, int worker = -1) {
  auto& pool = worker >= 0 ? c->worker_pool[worker] : c->staged_pool;
  if (pool.empty()) return std::make_unique<Staged>();
  auto s = std::move(pool.back());
  pool.pop_back();
  return s;
}

// Returns an admitted cluster's Staged to the pool it came from (its upload
// image goes back to the pinned pool now), unless that pool is full or the
// cluster was very large.  Caller holds mu.
void recycle_staged(ba_ctx* c, std::unique_ptr<Staged> s, int home) {
  if (!s || (size_t)s->O > kKeepObs) return;
  auto& pool = home >= 0 ? c->worker_pool[home] : c->staged_pool;
  const size_t cap = home >= 0 ? 2 : (size_t)c->opt.stage_threads + 2;
  if (pool.size() >= cap) return;
  s->blob.reset();
  pool.push_back(std::move(s));
}

// Moves the ticket's staged data into a free slot and arena block.  Returns
// BA_E_AGAIN when no slot or memory is free.  Caller holds mu.
int admit_one(ba_ctx* c, Ticket& t, hipStream_t st) {
  int slot = -1;
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (!c->slots[i].used) { slot = i; break; }
  if (slot < 0) return BA_E_AGAIN;
  Staged& s = *t.staged;
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
  d.C = s.C; d.P = s.P; d.L = s.L; d.n_chunks = s.n_chunks; d.n_wg = lay.n_wg;
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
  d.pchunk = (const int4*)(base + lay.pchunk);
  d.wg_chunk = (const int*)(base + lay.wg_chunk);
  d.ob_cam = (const int*)(base + lay.ob_cam);
  d.ob_uv64 = (double*)(base + lay.uv64);
  d.ob_uv32 = (float*)(base + lay.uv32);
  d.cl_pt = (const int*)(base + lay.cl_pt);
  d.cl_ob = (const int*)(base + lay.cl_ob);
  d.ql_pt = (const int*)(base + lay.ql_pt);
  d.ql_ob = (const int2*)(base + lay.ql_ob);
  d.tasks = (const int4*)(base + lay.tasks);
  d.targets = (const int4*)(base + lay.targets);
  d.cam[0] = (double*)(base + lay.cam0);
  d.cam[1] = (double*)(base + lay.cam1);
  d.prior = (double*)(base + lay.prior);
  d.pterm[0] = (double*)(base + lay.pterm0);
  d.pterm[1] = (double*)(base + lay.pterm1);
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
  d.pcg_part = (const int*)(base + lay.pcg_part);
  d.pcg_G = lay.part.empty() ? 0 : (int)lay.part.size() - 1;
  d.pcg_rows_max = lay.pcg_rows_max;
  d.pcg_smem = (int)lay.pcg_smem;
  std::vector<int2>& rin_c = sl.rin_c;
  std::vector<int2>& rin_p = sl.rin_p;
  std::vector<int2>& rout_p = sl.rout_p;
  std::vector<int4>& rout_c = sl.rout_c;
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
  // the upload image in one copy: asynchronous from pinned memory (the buffer
  // goes back to the pool once the copies from it have run), else waited
  // for below
  if (!s.blob) pack_staged(c, s, lay);
  if (s.blob_bytes) HIPCHK(c, hipMemcpyAsync(base, s.blob.get(), s.blob_bytes, hipMemcpyHostToDevice, st));
  auto up2 = [&](size_t off, const std::vector<int2>& v) {
    return v.empty() ? hipSuccess : hipMemcpyAsync(base + off, v.data(), sizeof(int2) * v.size(), hipMemcpyHostToDevice, st);
  };
  HIPCHK(c, up2(lay.rin_cam, rin_c));
  HIPCHK(c, up2(lay.rin_pt, rin_p));
  if (!rout_c.empty())
    HIPCHK(c, hipMemcpyAsync(base + lay.rout_cam, rout_c.data(), sizeof(int4) * rout_c.size(), hipMemcpyHostToDevice, st));
  HIPCHK(c, up2(lay.rout_pt, rout_p));
  SlotCtl& ctl = sl.ctl0;
  ctl = SlotCtl{};
  ctl.k[0][0] = s.k[0];
  ctl.k[0][1] = s.k[1];
  ctl.k[0][2] = s.f;      // principal-point offsets start at 0
  ctl.status = ST_RUNNING;
  char* tail = s.blob.get() + tail_off(s.blob_bytes);
  std::memcpy(tail, &d, sizeof(SlotDesc));
  std::memcpy(tail + kTailDesc, &ctl, sizeof(SlotCtl));
  HIPCHK(c, hipMemcpyAsync(c->d_desc + slot, tail, sizeof(SlotDesc), hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->d_ctl + slot, tail + kTailDesc, sizeof(SlotCtl), hipMemcpyHostToDevice, st));
  if (s.blob_pinned) {
    hipEvent_t ev = nullptr;
    {
      std::lock_guard<std::mutex> g(c->pin_mu);
      if (!c->pin_events.empty()) {
        ev = c->pin_events.back();
        c->pin_events.pop_back();
      }
    }
    if (!ev) HIPCHK(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(c, hipEventRecord(ev, st));
    std::lock_guard<std::mutex> g(c->pin_mu);
    c->pin_flight.push_back({std::move(s.blob), ev});
  }
  // An image in ordinary memory must stay alive until its copy has run; the
  // small sources above live in the slot until it is freed.
  if (!s.blob_pinned) HIPCHK(c, hipStreamSynchronize(st));
  t.slot = slot;
  t.state = TK_RESIDENT;
  t.t_admit = now_s();
  recycle_staged(c, std::move(t.staged), t.staged_home);
  return BA_OK;
}

// Runs prep and the initial FP64 cost for newly admitted slots (on the
// context's stream unless st is given).
int start_slots(ba_ctx* c, Launcher& l, const std::vector<int>& slots, hipStream_t st = nullptr) {
  if (slots.empty()) return BA_OK;
  if (!st) st = c->stream;
  Batch b;
  int rc = make_batch(c, l, slots, b, st);
  if (rc) return rc;
  int maxPL = 0, maxRin = 0;
  for (int s : slots) {
    const SlotDesc& d = c->slots[s].desc;
    maxPL = std::max({maxPL, d.P, d.L});
    maxRin = std::max({maxRin, d.n_rin_cam, d.n_rin_pt});
  }
  HIPCHK(c, launch_prep(b, maxPL, maxRin, st));
  HIPCHK(c, launch_initial_cost(b, st));
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
    HIPCHK(c, launch_iteration(b, mixed, c->stream, ev, c->prof, l.sp.data(), (int)l.sp.size()));
  }
  return BA_OK;
}

// n LM iterations of disjoint groups of slots, part p on stream p (part 0 on
// the context's stream, with launcher l0); the context's stream then waits
// for every part.
int run_iterations_parts(ba_ctx* c, bool serving, const std::vector<std::vector<int>>& parts, int n_iters) {
  const int P = (int)parts.size();
  Batch b[ba_ctx::kMaxParts];
  Launcher* lp[ba_ctx::kMaxParts];
  int rc;
  for (int p = 0; p < P; ++p) {
    Launcher& l = p == 0 ? (serving ? c->srv : c->api) : (serving ? c->srv_p[p] : c->api_p[p]);
    lp[p] = &l;
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
      HIPCHK(c, launch_iteration(b[p], mixed, p ? c->stream_p[p] : c->stream, ev, c->prof, lp[p]->sp.data(),
                                 (int)lp[p]->sp.size()));
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

// An export in flight: each slot's result region (cost, damping and accept
// logs, reprojection sums, exported state: the block's tail from the cost
// log on) copied in stream order into pinned host memory, with what the
// finish needs once the slot itself may have been reused.
struct ExportJob {
  struct Item {
    ba_ticket ticket = 0;
    int C = 0, P = 0, max_iters = 0;
    size_t lam, acc, out;            // offsets in the region
    bool res_finish = false;         // a resident cluster done with the store
    SlotCtl ctl{};
    std::shared_ptr<char> buf;       // pinned, or ordinary memory when the pool is full
  };
  std::vector<Item> items;
};

// Enqueues the export of the listed slots: the export kernels, one copy per
// slot, the resident write-back of finished clusters, then l.exp_ev.
// l.h_ctl must hold the slots' current control blocks.  The work goes on
// the context's stream with l's batch lists, or on st with bl's.  Later work
// on that stream (uploads into a freed slot block) comes after the copies;
// work on another stream that reuses a freed block must wait for l.exp_ev.
int export_begin(ba_ctx* c, Launcher& l, const std::vector<int>& slots, ExportJob& job, Launcher* bl = nullptr,
                 hipStream_t st = nullptr) {
  job.items.clear();
  if (slots.empty()) return BA_OK;
  Launcher& bt = bl ? *bl : l;
  if (!st) st = c->stream;
  Batch b;
  int rc = make_batch(c, bt, slots, b, st);
  if (rc) return rc;
  int maxP = 0;
  for (int s : slots) maxP = std::max(maxP, c->slots[s].desc.P);
  HIPCHK(c, launch_export(b, maxP, st));
  std::vector<int> wb;
  for (int s : slots) {
    const Slot& sl = c->slots[s];
    const Ticket& t = *c->tickets[sl.ticket];
    ExportJob::Item it;
    it.ticket = t.id;
    it.C = sl.desc.C;
    it.P = sl.desc.P;
    it.max_iters = sl.desc.max_iters;
    it.lam = sl.lay.lambda_log - sl.lay.cost_log;
    it.acc = sl.lay.acc_log - sl.lay.cost_log;
    it.out = sl.lay.out - sl.lay.cost_log;
    it.ctl = l.h_ctl[s];
    const size_t bytes = sl.lay.total - sl.lay.cost_log;
    it.buf = pin_get(c, bytes);
    if (!it.buf) it.buf = std::shared_ptr<char>(new char[bytes], std::default_delete<char[]>());
    HIPCHK(c, hipMemcpyAsync(it.buf.get(), c->arena_base + sl.off + sl.lay.cost_log, bytes, hipMemcpyDeviceToHost,
                             st));
    // finished resident clusters write their state back (once)
    const int status = it.ctl.status;
    if (t.resident && !t.res_done && is_finished(status)) {
      it.res_finish = true;
      if (status != ST_BAD_INIT) wb.push_back(s);
    }
    job.items.push_back(std::move(it));
  }
  if (!wb.empty()) {
    Batch bw;
    if ((rc = make_batch(c, bt, wb, bw, st))) return rc;
    int maxR = 0;
    for (int s : wb) maxR = std::max({maxR, c->slots[s].desc.n_rout_cam, c->slots[s].desc.n_rout_pt});
    HIPCHK(c, launch_writeback(bw, maxR, st));
  }
  HIPCHK(c, hipEventRecord(l.exp_ev, st));
  return BA_OK;
}

// Waits for an export's copies and moves the results into the ticket caches;
// resident clusters that finished release their store rows.
int export_finish(ba_ctx* c, Launcher& l, ExportJob& job) {
  if (job.items.empty()) return BA_OK;
  HIPCHK(c, hipEventSynchronize(l.exp_ev));
  bool any_res = false;
  for (ExportJob::Item& it : job.items) {
    Ticket& t = *c->tickets[it.ticket];
    const char* r = it.buf.get();
    const double* lg = (const double*)r;
    t.cost_log.assign(lg, lg + it.max_iters + 1);
    const double* lm = (const double*)(r + it.lam);
    t.lambda_log.assign(lm, lm + it.max_iters);
    const int* ac = (const int*)(r + it.acc);
    t.acc_log.assign(ac, ac + it.max_iters);
    const double* o = (const double*)(r + it.out);
    t.out.assign(o, o + 12 * (size_t)it.C + 3 * (size_t)it.P + 5 + kStatVals);
    t.ctl = it.ctl;
    it.buf.reset();
    if (!it.res_finish) continue;
    any_res = true;
    if (it.ctl.status != ST_BAD_INIT) {
      for (int row : t.cam_rows) c->res_cam_meta[row].valid = true;
      for (int row : t.pt_rows) c->res_pt_meta[row].valid = true;
      c->res_lambda = it.ctl.lambda;
    }
    for (int row : t.cam_rows)
      if (c->res_cam_meta[row].pending == t.id) c->res_cam_meta[row].pending = 0;
    for (int row : t.pt_rows)
      if (c->res_pt_meta[row].pending == t.id) c->res_pt_meta[row].pending = 0;
    t.res_done = true;
  }
  job.items.clear();
  if (any_res) c->cv.notify_all();
  return BA_OK;
}

// Exports the listed slots' state into their ticket caches (synchronous).
int export_slots(ba_ctx* c, Launcher& l, const std::vector<int>& slots) {
  if (slots.empty()) return BA_OK;
  int rc = read_ctl(c, l);
  if (rc) return rc;
  ExportJob job;
  if ((rc = export_begin(c, l, slots, job))) return rc;
  return export_finish(c, l, job);
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
int admit_queue(ba_ctx* c, std::vector<int>& admitted, bool serving_only, bool early = false,
                hipEvent_t after = nullptr) {
  hipStream_t st = early ? c->up_stream : c->stream;
  bool any = false;
  for (auto it = c->queue.begin(); it != c->queue.end();) {
    Ticket& t = *c->tickets[*it];
    if (t.staging || (serving_only && !t.serving) || !deps_done(c, t)) { ++it; continue; }
    if (after) {   // the uploads may go into blocks whose export `after` ends
      HIPCHK(c, hipStreamWaitEvent(st, after, 0));
      after = nullptr;
    }
    int rc = admit_one(c, t, st);
    if (rc == BA_E_AGAIN) break;
    if (rc) return rc;
    c->slots[t.slot].early = early;
    any = true;
    admitted.push_back(t.slot);
    it = c->queue.erase(it);
  }
  if (early && any) HIPCHK(c, hipEventRecord(c->up_ev, c->up_stream));
  return BA_OK;
}

// A serving ticket is queued that could be admitted now (its resident
// dependencies have written back).
bool serving_queued(ba_ctx* c) {
  for (ba_ticket id : c->queue) {
    const Ticket& t = *c->tickets[id];
    if (t.serving && !t.staging && deps_done(c, t)) return true;
  }
  return false;
}

// LM iterations of the next serving tick: iters_per_tick, cut so that the
// tick ends when the first running cluster reaches its iteration cap (it is
// retired at once).  `adm`: slots admitted for this tick (their read-back
// control is not theirs yet).
int tick_iters(ba_ctx* c, const std::vector<int>& active, const std::vector<int>& adm) {
  int n = c->opt.iters_per_tick;
  for (int s : active) {
    const bool fresh = std::find(adm.begin(), adm.end(), s) != adm.end();
    const int rem = c->slots[s].desc.max_iters - (fresh ? 0 : c->srv.h_ctl[s].iter);
    n = std::min(n, std::max(rem, 1));
  }
  return n;
}

// One serving tick: retire finished clusters, admit queued ones, iterate.
Ticket* find_ticket(ba_ctx* c, ba_ticket id);

void serve_loop(ba_ctx* c) {
  (void)hipSetDevice(c->device);
  std::vector<int> active;
  bool early_pending = false;   // uploads on up_stream since the last boundary
  std::unique_lock<std::mutex> lk(c->mu);
  while (!c->stop) {
    // everything the compute stream does from here on comes after the
    // uploads of clusters admitted during the last tick (a block freed
    // below may have been theirs)
    if (early_pending) {
      if (hipStreamWaitEvent(c->stream, c->up_ev, 0) != hipSuccess) {
        c->dead = true;
        break;
      }
      early_pending = false;
    }
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
    // retire: the export is enqueued on up_stream, beside the next tick, and
    // the finished slots are freed at once (uploads into their blocks come
    // later on up_stream, or wait for the export); the next tick is launched
    // before the host waits for the export's copies
    std::vector<int> fin;
    for (int s : active)
      if (is_finished(c->srv.h_ctl[s].status)) fin.push_back(s);
    ExportJob job;
    std::vector<ba_ticket> fin_t;
    if (!fin.empty()) {
      if (export_begin(c, c->srv, fin, job, &c->side, c->up_stream)) break;
      for (int s : fin) {
        fin_t.push_back(c->slots[s].ticket);
        free_slot(c, s);
      }
      active.erase(std::remove_if(active.begin(), active.end(),
                                  [&](int s) { return std::find(fin.begin(), fin.end(), s) != fin.end(); }),
                   active.end());
    }
    // admit: the clusters uploaded and set up during the last tick, then the
    // queue (uploaded and set up on the context's stream, after the export
    // of a block they may reuse)
    std::vector<int> fresh, adm;
    for (int s = 0; s < (int)c->slots.size(); ++s)
      if (c->slots[s].used && c->slots[s].early) {
        c->slots[s].early = false;
        fresh.push_back(s);
      }
    if (admit_queue(c, adm, true, false, fin.empty() ? nullptr : c->srv.exp_ev)) break;
    if (!adm.empty() && start_slots(c, c->srv, adm)) break;
    fresh.insert(fresh.end(), adm.begin(), adm.end());
    active.insert(active.end(), fresh.begin(), fresh.end());
    if (!active.empty()) {
      if (run_tick(c, true, active, tick_iters(c, active, fresh))) break;
      if (hipMemcpyAsync(c->srv.h_ctl, c->d_ctl, sizeof(SlotCtl) * c->opt.max_slots, hipMemcpyDeviceToHost,
                         c->stream) ||
          hipEventRecord(c->srv.ev, c->stream)) {
        c->dead = true;
        break;
      }
    }
    if (!fin.empty()) {
      if (export_finish(c, c->srv, job)) break;
      const double t_done = now_s();
      for (ba_ticket id : fin_t) {
        Ticket& t = *c->tickets[id];
        t.state = TK_DONE;
        t.serving = false;
        t.slot = -1;
        t.t_done = t_done;
      }
      c->done_cv.notify_all();
    }
    if (active.empty()) {
      c->cv.wait(lk, [&] { return c->stop || serving_queued(c) || !c->cancel.empty(); });
      continue;
    }
    // Wait for the tick.  A cluster whose layout finishes meanwhile is
    // admitted now, its upload and set-up running on up_stream beside the
    // tick; it joins at the next boundary.  The event is polled with mu released
    // (submitters and layout threads take it meanwhile), so that the end of
    // the tick is seen within microseconds rather than after a timed sleep:
    // the device idles from there to the next tick's first launch.
    hipError_t e;
    bool failed = false;
    for (;;) {
      e = hipEventQuery(c->srv.ev);
      if (e != hipErrorNotReady) break;
      if (!c->stop && serving_queued(c)) {
        const size_t before = c->queue.size();
        std::vector<int> early;
        if (admit_queue(c, early, true, true)) { failed = true; break; }
        if (!early.empty() &&
            (start_slots(c, c->side, early, c->up_stream) || hipEventRecord(c->up_ev, c->up_stream) != hipSuccess)) {
          failed = true;
          break;
        }
        if (c->queue.size() != before) early_pending = true;
      }
      lk.unlock();
      const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(50);
      while ((e = hipEventQuery(c->srv.ev)) == hipErrorNotReady && std::chrono::steady_clock::now() < until)
        std::this_thread::yield();
      lk.lock();
    }
    if (failed) break;
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
  int rc = admit_one(c, t, c->stream);
  if (rc == BA_E_AGAIN) return fail(c, BA_E_AGAIN, "no free slot or arena memory");
  if (rc) return rc;
  c->queue.erase(std::remove(c->queue.begin(), c->queue.end(), t.id), c->queue.end());
  admitted.push_back(t.slot);
  return BA_OK;
}

}  // namespace

namespace {
int enqueue_staged(ba_ctx* c, std::unique_ptr<Staged> st, ba_ticket* ticket, double t_submit);
const char* copy_checks(const ba_cluster* cl);
int enqueue_copy(ba_ctx* c, std::unique_ptr<ClusterCopy> copy, ba_ticket* ticket, double t_submit);
int wait_staged(ba_ctx* c, std::unique_lock<std::mutex>& lk, ba_ticket id);
void stage_worker(ba_ctx* c, int worker);
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
      opt->resident_points < 0 || opt->stage_threads < 0 || opt->stage_threads > 64)
    return BA_E_ARG;
  auto c = std::make_unique<ba_ctx>();
  c->opt = *opt;
  if (c->opt.hbm_budget_bytes == 0) c->opt.hbm_budget_bytes = (size_t)1 << 30;
  if (c->opt.max_slots <= 0) c->opt.max_slots = 256;
  if (c->opt.max_queue <= 0) c->opt.max_queue = 4096;
  if (c->opt.iters_per_tick <= 0) c->opt.iters_per_tick = 10;
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
  if (c->opt.serve && (hipStreamCreateWithFlags(&c->up_stream, hipStreamNonBlocking) != hipSuccess ||
                       hipEventCreateWithFlags(&c->up_ev, hipEventDisableTiming) != hipSuccess ||
                       init_launcher(c.get(), c->side)))
    return bail(BA_E_DEVICE);
  for (int p = 1; p < c->opt.batch_streams; ++p) {
    if (init_launcher(c.get(), c->api_p[p]) || init_launcher(c.get(), c->srv_p[p]) ||
        hipStreamCreateWithFlags(&c->stream_p[p], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->join_ev[p], hipEventDisableTiming) != hipSuccess)
      return bail(BA_E_DEVICE);
  }
  for (int i = 0; i < c->opt.max_slots; ++i) c->srv.h_ctl[i] = SlotCtl{};
  if (hipDeviceSynchronize() != hipSuccess) return bail(BA_E_DEVICE);
  ba_ctx* raw = c.release();
  raw->worker_pool.resize(raw->opt.stage_threads);
  for (int i = 0; i < raw->opt.stage_threads; ++i) raw->stagers.emplace_back(stage_worker, raw, i);
  if (opt->serve) raw->th = std::thread(serve_loop, raw);
  *out = raw;
  return BA_OK;
}

int ba_destroy(ba_ctx* c) {
  if (!c) return BA_E_ARG;
  {
    std::lock_guard<std::mutex> g(c->mu);
    c->stop = true;
    c->stage_stop = true;
  }
  c->cv.notify_all();
  c->stage_cv.notify_all();
  for (auto& th : c->stagers)
    if (th.joinable()) th.join();
  if (c->th.joinable()) c->th.join();
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->up_stream) (void)hipStreamSynchronize(c->up_stream);
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
  if (c->up_ev) (void)hipEventDestroy(c->up_ev);
  if (c->up_stream) (void)hipStreamDestroy(c->up_stream);
  free_launcher(c, c->srv);
  free_launcher(c, c->side);
  // the tickets' upload images go back to the pool before it is freed
  c->tickets.clear();
  c->stage_jobs.clear();
  {
    std::vector<ba_ctx::PinFlight> fl;
    {
      std::lock_guard<std::mutex> g(c->pin_mu);
      fl.swap(c->pin_flight);
    }
    for (auto& f : fl) (void)hipEventDestroy(f.ev);
  }
  for (auto& f : c->pin_free) (void)hipHostFree(f.first);
  for (hipEvent_t e : c->pin_events) (void)hipEventDestroy(e);
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
  if (c->opt.stage_threads > 0) {   // background layout: the copy is made before mu is taken
    const char* why = copy_checks(cl);
    std::unique_ptr<ClusterCopy> copy;
    if (!why) copy = std::make_unique<ClusterCopy>(*cl);
    std::lock_guard<std::mutex> g(c->mu);
    if (why) return fail(c, BA_E_ARG, why);
    return enqueue_copy(c, std::move(copy), ticket, t_submit);
  }
  std::unique_ptr<Staged> st;
  {
    std::lock_guard<std::mutex> g(c->mu);
    st = take_staged(c);
  }
  std::string err;
  int rc = stage(cl, *st, err, c->opt.chunks_per_wg, c->opt.chunks_per_task, c->opt.solver);
  if (!rc) {
    const Layout lay = make_layout(*st, c->opt.precision == BA_MIXED);
    if (lay.pcg_ok && lay.total <= c->arena.size()) pack_staged(c, *st, lay);
  }
  std::lock_guard<std::mutex> g(c->mu);
  if (rc) return fail(c, rc, err);
  return enqueue_staged(c, std::move(st), ticket, t_submit);
}

int ba_submit_clusters(ba_ctx* c, int32_t n, const ba_cluster* cl, ba_ticket* tickets) {
  const double t_submit = now_s();
  if (!c || n < 0 || (n > 0 && (!cl || !tickets))) return BA_E_ARG;
  for (int i = 0; i < n; ++i) tickets[i] = 0;
  if (c->opt.stage_threads > 0) {   // background layout: queued in order, laid out by the pool
    // a cluster that fails the checks made at submission fails the call
    // before any is queued; the copies are made before mu is taken
    for (int i = 0; i < n; ++i)
      if (const char* why = copy_checks(&cl[i])) {
        std::lock_guard<std::mutex> g(c->mu);
        return fail(c, BA_E_ARG, "cluster " + std::to_string(i) + ": " + why);
      }
    std::vector<std::unique_ptr<ClusterCopy>> copy(n);
    for (int i = 0; i < n; ++i) copy[i] = std::make_unique<ClusterCopy>(cl[i]);
    std::lock_guard<std::mutex> g(c->mu);
    for (int i = 0; i < n; ++i) {
      const int r = enqueue_copy(c, std::move(copy[i]), &tickets[i], t_submit);
      if (r) {
        c->last_error = "cluster " + std::to_string(i) + ": " + c->last_error;
        return r;
      }
    }
    return BA_OK;
  }
  std::vector<std::unique_ptr<Staged>> st(n);
  {
    std::lock_guard<std::mutex> g(c->mu);
    for (auto& p : st) p = take_staged(c);
  }
  std::vector<int> rc(n, BA_OK);
  std::vector<std::string> err(n);
  {
    // lay the clusters out on up to 8 host threads; they share nothing
    std::atomic<int> next{0};
    auto work = [&]() {
      for (int i; (i = next.fetch_add(1)) < n;) {
        rc[i] = stage(&cl[i], *st[i], err[i], c->opt.chunks_per_wg, c->opt.chunks_per_task, c->opt.solver);
        if (!rc[i]) {
          const Layout lay = make_layout(*st[i], c->opt.precision == BA_MIXED);
          if (lay.pcg_ok && lay.total <= c->arena.size()) pack_staged(c, *st[i], lay);
        }
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

// Releases the resident-store rows a ticket registered (it will never write
// them back).  Caller holds mu.
void res_abandon(ba_ctx* c, Ticket& t) {
  for (int row : t.cam_rows)
    if (c->res_cam_meta[row].pending == t.id) c->res_cam_meta[row].pending = 0;
  for (int row : t.pt_rows)
    if (c->res_pt_meta[row].pending == t.id) c->res_pt_meta[row].pending = 0;
  t.res_done = true;
}

// A layout thread: lays out the queued copies in submission order of pickup;
// the result (or the reason it was refused) goes to the ticket.
void stage_worker(ba_ctx* c, int worker) {
  (void)hipSetDevice(c->device);   // for the pinned buffers of the upload images
  std::unique_lock<std::mutex> lk(c->mu);
  for (;;) {
    c->stage_cv.wait(lk, [&] { return c->stage_stop || !c->stage_jobs.empty(); });
    if (c->stage_stop) return;
    auto job = std::move(c->stage_jobs.front());
    c->stage_jobs.pop_front();
    auto st = take_staged(c, worker);
    lk.unlock();
    std::string err;
    const int rc = stage(&job.second->c, *st, err, c->opt.chunks_per_wg, c->opt.chunks_per_task, c->opt.solver);
    Layout lay;
    if (!rc) lay = make_layout(*st, c->opt.precision == BA_MIXED);
    if (!rc && lay.pcg_ok && lay.total <= c->arena.size()) pack_staged(c, *st, lay);
    lk.lock();
    Ticket* t = nullptr;
    auto it = c->tickets.find(job.first);
    if (it != c->tickets.end()) t = it->second.get();
    if (!t) {           // released meanwhile
      c->staged_cv.notify_all();
      continue;
    }
    int code = rc;
    if (!code && !lay.pcg_ok) {
      code = BA_E_ARG;
      err = "reduced system too dense for the conjugate-gradient solve";
    } else if (!code && lay.total > c->arena.size()) {
      code = BA_E_NOMEM;
      err = "cluster footprint exceeds the arena";
    }
    t->staging = false;
    if (code) {
      t->state = TK_INVALID;
      t->err_code = code;
      t->err_msg = err;
      t->serving = false;
      if (t->resident) res_abandon(c, *t);
      c->queue.erase(std::remove(c->queue.begin(), c->queue.end(), t->id), c->queue.end());
      c->done_cv.notify_all();
      c->cv.notify_all();
    } else {
      t->bytes = lay.total;
      t->staged = std::move(st);
      t->staged_home = worker;
      c->cv.notify_all();
    }
    c->staged_cv.notify_all();
  }
}

// Waits (releasing mu) until the ticket's background layout has finished;
// returns its refusal, if any.  Caller holds mu through lk.
int wait_staged(ba_ctx* c, std::unique_lock<std::mutex>& lk, ba_ticket id) {
  c->staged_cv.wait(lk, [&] {
    auto it = c->tickets.find(id);
    return it == c->tickets.end() || !it->second->staging;
  });
  auto it = c->tickets.find(id);
  if (it == c->tickets.end()) return fail(c, BA_E_ARG, "unknown ticket");
  if (it->second->state == TK_INVALID) return fail(c, it->second->err_code, it->second->err_msg);
  return BA_OK;
}

// The checks of a submitted cluster that need no layout (sizes, arrays
// present, resident IDs unique); nullptr when it passes them.  The rest run
// on a layout thread.
const char* copy_checks(const ba_cluster* cl) {
  if (!cl) return "cluster is NULL";
  const int C = cl->n_cams, P = cl->n_points, O = cl->n_obs;
  if (C < 1 || C > kMaxCams || P < 0 || O < 0) return "sizes out of range (1 <= n_cams <= 512)";
  if (!cl->R || !cl->T || !cl->k || !cl->prior_R || !cl->prior_T || !cl->prior_sigma || !cl->fixed ||
      (P > 0 && !cl->X) || (O > 0 && (!cl->obs_cam || !cl->obs_pt || !cl->obs_uv)))
    return "missing input array";
  if (cl->max_iters < 1 || cl->max_iters > 4096) return "max_iters must be in 1..4096";
  if (cl->use_resident != 0 && cl->use_resident != 1) return "use_resident must be 0 or 1";
  if (cl->use_resident) {
    if (!cl->cam_ids || (P > 0 && !cl->point_ids)) return "use_resident needs cam_ids and point_ids";
    if (!ids_unique(cl->cam_ids, C)) return "duplicate camera ID in the cluster";
    if (!ids_unique(cl->point_ids, P)) return "duplicate point ID in the cluster";
  }
  return nullptr;
}

// Queues a copy of a cluster that passed copy_checks for background layout.
// The caller makes the copy before it takes mu (a paper-scale cluster is a
// few MB: the serving thread and the layout threads do not wait for the
// copying).  Caller holds mu.
int enqueue_copy(ba_ctx* c, std::unique_ptr<ClusterCopy> copy, ba_ticket* ticket, double t_submit) {
  const ba_cluster* cl = &copy->c;
  const int C = cl->n_cams, P = cl->n_points;
  if (c->dead) return fail(c, BA_E_DEVICE, "context is unusable after a device error");
  if ((int)c->queue.size() >= c->opt.max_queue) return fail(c, BA_E_AGAIN, "admission queue full");
  auto t = std::make_unique<Ticket>();
  t->id = c->next_id;
  if (cl->use_resident) {
    Staged ids;   // the IDs alone: resident clusters are ordered at submission
    ids.C = C;
    ids.P = P;
    ids.cam_ids = copy->cam_ids;
    ids.point_ids = copy->point_ids;
    const int rc = res_register(c, *t, ids);
    if (rc) return rc;
  }
  c->next_id++;
  t->C = C;
  t->P = P;
  t->max_iters = cl->max_iters;
  t->t_submit = t_submit;
  t->staging = true;
  const ba_ticket id = t->id;
  c->tickets[id] = std::move(t);
  c->queue.push_back(id);
  c->stage_jobs.emplace_back(id, std::move(copy));
  c->stage_cv.notify_one();
  *ticket = id;
  return BA_OK;
}

// Queues a laid-out cluster (registering its resident IDs) and returns its
// ticket.  Caller holds mu.
int enqueue_staged(ba_ctx* c, std::unique_ptr<Staged> st, ba_ticket* ticket, double t_submit) {
  int rc;
  if (c->dead) return fail(c, BA_E_DEVICE, "context is unusable after a device error");
  const Layout lay = make_layout(*st, c->opt.precision == BA_MIXED);
  if (!lay.pcg_ok)
    return fail(c, BA_E_ARG, "reduced system too dense for the conjugate-gradient solve (a block row's blocks must "
                             "fit the LDS of one workgroup, at most 128 workgroups)");
  const size_t bytes = lay.total;
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
  std::unique_lock<std::mutex> g(c->mu);
  if (c->dead) return fail(c, BA_E_DEVICE, "context is unusable after a device error");
  Ticket* t = find_ticket(c, id);
  if (!t) return fail(c, BA_E_ARG, "unknown ticket");
  if (t->staging || t->state == TK_INVALID) {
    const int rc = wait_staged(c, g, id);
    if (rc) return rc;
    t = find_ticket(c, id);
    if (!t) return fail(c, BA_E_ARG, "unknown ticket");
  }
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
  std::unique_lock<std::mutex> g(c->mu);
  if (c->dead) return fail(c, BA_E_DEVICE, "context is unusable after a device error");
  HIPCHK(c, hipSetDevice(c->device));
  for (int i = 0; i < n; ++i) {
    Ticket* t = find_ticket(c, ids[i]);
    if (t && (t->staging || t->state == TK_INVALID)) {
      const int rc = wait_staged(c, g, ids[i]);
      if (rc) return rc;
    }
  }
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
  if (t->state == TK_INVALID) return fail(c, t->err_code, t->err_msg);
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
  if (t->state == TK_INVALID) return fail(c, t->err_code, t->err_msg);
  if (!t->serving && t->state != TK_DONE) return fail(c, BA_E_STATE, "cluster was not handed to ba_solve");
  // the ticket may be released (and removed) while this thread waits
  auto pred = [&] {
    Ticket* x = find_ticket(c, id);
    return !x || x->state == TK_DONE || x->state == TK_INVALID || c->dead;
  };
  if (timeout_s < 0) c->done_cv.wait(lk, pred);
  else if (!c->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) return BA_E_TIMEOUT;
  t = find_ticket(c, id);
  if (!t) return fail(c, BA_E_STATE, "cluster was released while waiting");
  if (t->state == TK_INVALID) return fail(c, t->err_code, t->err_msg);
  if (c->dead && t->state != TK_DONE) return fail(c, BA_E_DEVICE, "serving loop stopped on a device error");
  return BA_OK;
}

int ba_fetch(ba_ctx* c, ba_ticket id, ba_result* r) {
  if (!c || !r) return BA_E_ARG;
  std::lock_guard<std::mutex> g(c->mu);
  Ticket* t = find_ticket(c, id);
  if (!t) return fail(c, BA_E_ARG, "unknown ticket");
  if (t->state == TK_INVALID) return fail(c, t->err_code, t->err_msg);
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
  c->staged_cv.notify_all();   // a caller waiting for this cluster's layout
  return BA_OK;
}

}  // extern "C"
