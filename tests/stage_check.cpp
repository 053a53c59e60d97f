// Host harness of the cluster layout (paper_2511_06152_amd/csrc/ba_stage.cpp)
// for the CPU tests: built with the host compiler under AddressSanitizer and
// UndefinedBehaviorSanitizer (or ThreadSanitizer), it reads one cluster from
// a binary file, lays it out, and writes the layout to another file for the
// test to check.  With threads > 1 it lays the same cluster out on that many
// threads at once and exits non-zero unless every copy is identical.
//
// usage: stage_check <in> <out> <chunks_per_wg> <chunks_per_task> <solver> <threads>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../paper_2511_06152_amd/csrc/ba_stage.h"

using namespace bagpu;

namespace {

struct Reader {
  FILE* f;
  template <typename T>
  std::vector<T> vec(size_t n) {
    std::vector<T> v(n);
    if (n && fread(v.data(), sizeof(T), n, f) != n) {
      fprintf(stderr, "short input\n");
      exit(3);
    }
    return v;
  }
  template <typename T>
  T one() { return vec<T>(1)[0]; }
};

template <typename T, typename A>
void put(FILE* f, const std::vector<T, A>& v) {
  const int64_t n = (int64_t)v.size();
  fwrite(&n, sizeof n, 1, f);
  if (n) fwrite(v.data(), sizeof(T), v.size(), f);
}

bool same(const Staged& a, const Staged& b) {
  auto eq = [](const auto& x, const auto& y) {
    return x.size() == y.size() && (x.empty() || !memcmp(x.data(), y.data(), sizeof(x[0]) * x.size()));
  };
  return a.L == b.L && a.Lc == b.Lc && a.Lq == b.Lq && eq(a.pchunk, b.pchunk) && eq(a.wg_chunk, b.wg_chunk) &&
         eq(a.ob_cam, b.ob_cam) && eq(a.ob_uv, b.ob_uv) && eq(a.cl_pt, b.cl_pt) && eq(a.cl_ob, b.cl_ob) && eq(a.ql_pt, b.ql_pt) &&
         eq(a.ql_ob, b.ql_ob) && eq(a.tasks, b.tasks) && eq(a.targets, b.targets) && eq(a.pt_orig, b.pt_orig) &&
         eq(a.brow, b.brow) && eq(a.bcol, b.bcol) && eq(a.tslot, b.tslot) && eq(a.X, b.X) && eq(a.raw_cam, b.raw_cam);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 7) {
    fprintf(stderr, "usage: stage_check <in> <out> <chunks_per_wg> <chunks_per_task> <solver> <threads>\n");
    return 2;
  }
  FILE* fi = fopen(argv[1], "rb");
  if (!fi) return 2;
  Reader r{fi};
  ba_cluster c{};
  c.n_cams = r.one<int32_t>();
  c.n_points = r.one<int32_t>();
  c.n_obs = r.one<int32_t>();
  c.intr_mask = r.one<int32_t>();
  c.max_iters = r.one<int32_t>();
  c.use_resident = r.one<int32_t>();
  const size_t C = (size_t)std::max(c.n_cams, 0), P = (size_t)std::max(c.n_points, 0),
               O = (size_t)std::max(c.n_obs, 0);
  auto R = r.vec<double>(9 * C), T = r.vec<double>(3 * C), X = r.vec<double>(3 * P), k = r.vec<double>(2);
  auto pR = r.vec<double>(9 * C), pT = r.vec<double>(3 * C), ps = r.vec<double>(6 * C);
  auto fixed = r.vec<uint8_t>(C);
  auto oc = r.vec<int32_t>(O), op = r.vec<int32_t>(O);
  auto uv = r.vec<double>(2 * O);
  auto cam = r.vec<double>(5);
  auto cid = r.vec<int64_t>(c.use_resident ? C : 0), pid = r.vec<int64_t>(c.use_resident ? P : 0);
  fclose(fi);
  c.R = R.data(); c.T = T.data(); c.X = X.data(); c.k = k.data();
  c.prior_R = pR.data(); c.prior_T = pT.data(); c.prior_sigma = ps.data(); c.fixed = fixed.data();
  c.obs_cam = oc.data(); c.obs_pt = op.data(); c.obs_uv = uv.data();
  c.f = cam[0]; c.cx = cam[1]; c.cy = cam[2]; c.sigma_px = cam[3]; c.huber_delta = cam[4];
  c.lambda0 = 1e-4;
  c.ftol = 1e-10;
  if (c.use_resident) { c.cam_ids = cid.data(); c.point_ids = pid.data(); }
  const int cpw = atoi(argv[3]), cpt = atoi(argv[4]), solver = atoi(argv[5]), nth = atoi(argv[6]);

  std::vector<Staged> st(std::max(nth, 1));
  std::vector<std::string> err(st.size());
  std::vector<int> rc(st.size());
  if (nth > 1) {
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) th.emplace_back([&, t] { rc[t] = stage(&c, st[t], err[t], cpw, cpt, solver); });
    for (auto& x : th) x.join();
    for (int t = 1; t < nth; ++t)
      if (rc[t] != rc[0] || (rc[0] == 0 && !same(st[t], st[0]))) {
        fprintf(stderr, "layouts differ between threads\n");
        return 4;
      }
  } else {
    rc[0] = stage(&c, st[0], err[0], cpw, cpt, solver);
    if (rc[0] == 0) {
      // again into the same Staged on the same thread: its storage and the
      // thread's scratch are reused, and the layout must not change
      const Staged first = st[0];
      std::string e2;
      if (stage(&c, st[0], e2, cpw, cpt, solver) != 0 || !same(first, st[0])) {
        fprintf(stderr, "a reused layout differs\n");
        return 5;
      }
    }
  }
  FILE* fo = fopen(argv[2], "wb");
  if (!fo) return 2;
  const Staged& s = st[0];
  const int32_t hdr[12] = {rc[0], s.L, s.n_chunks, s.Lc, s.Lq, (int32_t)s.tasks.size(), (int32_t)s.targets.size(),
                           s.m, s.n_free, s.sparse, s.n_cam_tasks, s.n_wg};
  fwrite(hdr, sizeof hdr, 1, fo);
  put(fo, std::vector<char>(err[0].begin(), err[0].end()));
  if (rc[0] == 0) {
    put(fo, s.pt_orig);
    put(fo, s.pchunk);
    put(fo, s.wg_chunk);
    put(fo, s.ob_cam);
    put(fo, s.ob_uv);
    put(fo, s.cl_pt);
    put(fo, s.cl_ob);
    put(fo, s.ql_pt);
    put(fo, s.ql_ob);
    put(fo, s.tasks);
    put(fo, s.targets);
    put(fo, s.cam_col);
    put(fo, s.brow);
    put(fo, s.bcol);
  }
  fclose(fo);
  return 0;
}
