// Host layout of a submitted cluster (no HIP: also built alone for the host
// tests under the sanitizers).  Validates a ba_cluster and builds the work
// lists the kernels read: point chunks, camera lanes, pair lanes, tasks and
// reduction targets, the point order (observation count, then Morton), and for the conjugate-gradient
// solve the block-CSR structure of the reduced camera system.  Not part of
// the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ba.h"
#include "ba_consts.h"

namespace bagpu {

// Plain integer tuples with the layout of HIP's int2 / int3 / int4 (they are
// uploaded as such).
struct I2 { int x, y; };
struct I3 { int x, y, z; };
struct I4 { int x, y, z, w; };

// Allocator that leaves trivially constructible values uninitialised on
// resize(): the layout writes every lane of its lane arrays (padding
// included), so zero-filling them first would only cost memory bandwidth.
template <typename T>
struct NoInit : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = NoInit<U>;
  };
  NoInit() = default;
  template <typename U>
  NoInit(const NoInit<U>&) {}
  template <typename U>
  void construct(U* p) noexcept {
    ::new ((void*)p) U;
  }
  template <typename U, typename... A>
  void construct(U* p, A&&... a) {
    ::new ((void*)p) U(std::forward<A>(a)...);
  }
};
template <typename T>
using lane_vec = std::vector<T, NoInit<T>>;

// A submitted cluster, laid out for the device.
struct Staged {
  int C = 0, P = 0, O = 0, L = 0, n_chunks = 0, m = 0, n_free = 0, kcol0 = -1, kcol1 = -1;
  int kcolt[kIntr] = {-1, -1, -1, -1, -1}, sc = 0;   // column of each intrinsic; f, cx or cy estimated
  int max_iters = 0, stop_on_ftol = 0;
  double f = 0, cx = 0, cy = 0, sigma = 1, delta = 1, lambda0 = 1e-4, ftol = 0, k[2] = {0, 0};
  std::vector<double> raw_cam;   // [C][30]
  std::vector<double> X;         // [3P] internal point order
  std::vector<int> pt_orig;      // [P] caller index of each internal point
  std::vector<int> cam_col;      // [C]
  // point chunks: {first observation lane, observations per point n, first
  // point, valid points}; observation t of lane l at first + 64 t + l
  std::vector<I4> pchunk;        // [n_chunks]
  std::vector<int> wg_chunk;     // [n_wg + 1] first chunk of each point-pass workgroup
  lane_vec<int> ob_cam;          // [L] camera of each observation lane (0 for padding)
  lane_vec<double> ob_uv;        // [2L] raw pixels (0 for padding)
  int Lc = 0, Lq = 0, nb = 0, n_wg = 0, n_pt_part = 0, n_cam_tasks = 0;
  // camera lanes [Lc]: point (-1 for padding) and observation lane (0 for
  // padding); pair lanes [Lq]: point and the observation lanes of its two
  // observations (camera a, camera b)
  lane_vec<int> cl_pt, cl_ob, ql_pt;
  lane_vec<I2> ql_ob;
  std::vector<I4> tasks, targets;
  // sparse (PCG) reduced system: block CSR over the free cameras, diagonal first
  int sparse = 0;
  std::vector<int> brow, bcol;   // [F + 1], [nnzb]
  std::vector<I2> tslot;         // [n_targets] block slots (a,b), (b,a) of each target
  // resident state: global IDs (caller order) when the cluster uses it;
  // observations per camera (the match-count weights of Eq. 8 fusion)
  bool resident = false, fuse = false;
  std::vector<int64_t> cam_ids, point_ids;
  std::vector<int> cam_nobs;
  // upload image: the arrays the slot block takes from the host, already at
  // their offsets in the block, in a buffer the runtime provides (pinned
  // host memory, returned to its pool when the pointer is dropped); empty
  // when none was available (the arrays above are then copied one by one)
  std::shared_ptr<char> blob;
  size_t blob_bytes = 0;
  bool blob_pinned = false;
};


inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// splitmix64 finaliser: spreads IDs over a power-of-two table.
uint64_t mix_id(int64_t id);

// True when the n IDs are pairwise distinct.
bool ids_unique(const int64_t* id, int n);

// Validates the cluster and builds its work lists (integer bookkeeping only):
//  * point chunks: points sorted by observation count, then Morton order,
//    cut into chunks of 64 points of one count n; the chunk's observations
//    stored observation-major (the t-th of each point, in camera order, in
//    one 64-lane row), and chunks grouped into point-pass workgroups;
//  * camera lanes: observations of each free camera in point order (point and
//    observation lane), each camera's run padded to whole chunks, cut into
//    tasks of <= cpt chunks;
//  * pair lanes: the observation pairs of each point whose two cameras are
//    free (point and both observation lanes), grouped by camera pair,
//    padded and cut into tasks likewise;
//  * reduction targets: each free camera, each camera pair, the intrinsics.
// Returns BA_OK, or BA_E_ARG with the reason in err.  `s` is reset first;
// the storage of its vectors is reused (a recycled Staged lays out the next
// cluster without new allocations or page faults).
int stage(const ba_cluster* c, Staged& s, std::string& err, int cpw, int cpt, int solver);

// Resets every field of s to its default, keeping the vectors' storage.
void reset_keep(Staged& s);

// Layouts of clusters up to this many observations keep their storage for the
// next one (per layout thread, and in the runtime's pool of Staged objects).
constexpr size_t kKeepObs = size_t(1) << 20;

}  // namespace bagpu
