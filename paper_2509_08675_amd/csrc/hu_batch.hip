// Heterogeneous batches and the tile-variant autotuner.
//
// hu_pipeline_batch groups the jobs into classes of equal grid and bin layout, writes one FieldIO
// entry per job (seed, filter, outputs) into the workspace, and runs every class's pass sequence
// from one captured hipGraph: the classes hang off a fork-join over side streams, so small classes
// run beside large ones.  The instantiated graph is cached per batch structure and workspace and
// replayed on later calls; only the FieldIO table is uploaded each time.
//
// hu_autotune searches the plan of a shape class (the tile width of every kernel family, three
// schedule switches and the radix lists of the column passes) on a synthetic batch of the
// requested shape: starting from the default plan it flips one choice at a time and keeps it when
// the whole pass sequence gets faster; the plan is kept in memory and optionally in a JSON file
// (read back through $HUFIELD_TUNE_CACHE).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hu_host.hpp"

using namespace hu;

namespace {

constexpr int NSIDE = 4;

struct Class {
  hu_dims dims;
  hu_bins bins;
  bool has_bins;
  Geom g;
  std::vector<int> jobs;     // indices into the job array
  size_t io_off;             // first FieldIO entry of the class
  size_t work_off;           // workspace of the class
  Layout lay;
  bool want_cont, want_pm1;
  bool any_gen;
};

std::mutex g_bmu;
hipStream_t g_side[NSIDE] = {};
hipStream_t g_cap = nullptr;
hipEvent_t g_fork = nullptr, g_join[NSIDE] = {};
std::map<std::string, hipGraphExec_t> g_graphs;
// pinned staging for the FieldIO upload; reused once the previous upload has completed
FieldIO* g_stage = nullptr;
size_t g_stage_n = 0;
hipEvent_t g_stage_done = nullptr;

int ensure_streams() {
  if (g_cap) return HU_OK;
  HU_HIP(hipStreamCreateWithFlags(&g_cap, hipStreamNonBlocking));
  for (int i = 0; i < NSIDE; ++i) HU_HIP(hipStreamCreateWithFlags(&g_side[i], hipStreamNonBlocking));
  HU_HIP(hipEventCreateWithFlags(&g_fork, hipEventDisableTiming));
  for (int i = 0; i < NSIDE; ++i) HU_HIP(hipEventCreateWithFlags(&g_join[i], hipEventDisableTiming));
  return HU_OK;
}

TunePlan widest() { return TunePlan{{1, 1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0}}; }

int job_status(const hu_job& j, Geom* g) {
  int rc = make_geom(j.dims, g);
  if (rc) return rc;
  rc = check_filter(&j.filt, g->nd);
  if (rc) return rc;
  const bool want_spec = j.cont_sum || j.pm1_sum;
  if (want_spec) {
    rc = check_bins(&j.bins, g->nd);
    if (rc) return rc;
  }
  const void* ptrs[] = {j.field, j.pm1, j.stats, j.counts, j.cont_sum, j.cont_cnt, j.pm1_sum, j.pm1_cnt};
  bool any = false;
  for (const void* p : ptrs) {
    if (p && !aligned(p, 16)) return HU_ERR_ALIGN;
    any = any || p;
  }
  return any ? HU_OK : HU_ERR_ARG;
}

// classes in order of first appearance; the largest classes first so that they start earliest
int build_classes(const hu_job* jobs, int njobs, int32_t* status, std::vector<Class>& cls, size_t* total) {
  std::map<std::vector<long long>, int> idx;
  for (int i = 0; i < njobs; ++i) {
    Geom g;
    const int rc = job_status(jobs[i], &g);
    if (status) status[i] = rc;
    if (rc) continue;
    const bool hb = jobs[i].cont_sum || jobs[i].pm1_sum;
    std::vector<long long> key = {g.nd, g.n[0], g.n[1], g.n[2], hb ? jobs[i].bins.n_radial : 0,
                                  hb ? jobs[i].bins.n_angular : 0};
    auto it = idx.find(key);
    if (it == idx.end()) {
      Class c{};
      c.dims = jobs[i].dims;
      c.bins = jobs[i].bins;
      c.has_bins = hb;
      c.g = g;
      it = idx.emplace(key, (int)cls.size()).first;
      cls.push_back(c);
    }
    Class& c = cls[it->second];
    c.jobs.push_back(i);
    c.want_cont = c.want_cont || jobs[i].cont_sum;
    c.want_pm1 = c.want_pm1 || jobs[i].pm1_sum;
    c.any_gen = c.any_gen || filt_general(jobs[i].filt, g);
  }
  std::stable_sort(cls.begin(), cls.end(), [](const Class& a, const Class& b) {
    return (long long)a.jobs.size() * a.g.N > (long long)b.jobs.size() * b.g.N;
  });
  size_t off = up256((size_t)njobs * sizeof(FieldIO));
  size_t io = 0;
  for (Class& c : cls) {
    c.io_off = io;
    io += c.jobs.size();
    HU_TRY(layout(c.g, (int)c.jobs.size(), true, widest(), c.has_bins ? &c.bins : nullptr, &c.lay));
    c.work_off = off;
    off += c.lay.total;
  }
  *total = off;
  return HU_OK;
}

}  // namespace

extern "C" {

int hu_workspace_size_batch(const hu_job* jobs, int32_t njobs, size_t* bytes) {
  if (!jobs || njobs < 1 || !bytes) return HU_ERR_ARG;
  std::vector<Class> cls;
  HU_TRY(build_classes(jobs, njobs, nullptr, cls, bytes));
  return HU_OK;
}

int hu_pipeline_batch(const hu_job* jobs, int32_t njobs, float near_tol, int32_t* status, void* work,
                      size_t work_bytes, void* stream) {
  if (!jobs || njobs < 1) return HU_ERR_ARG;
  if (!std::isfinite(near_tol) || near_tol < 0.0f) return HU_ERR_ARG;
  if (!work || !aligned(work, 256)) return work ? HU_ERR_ALIGN : HU_ERR_ARG;
  std::vector<Class> cls;
  size_t total = 0;
  HU_TRY(build_classes(jobs, njobs, status, cls, &total));
  if (work_bytes < total) return HU_ERR_WORKSPACE;
  if (cls.empty()) return HU_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* w = reinterpret_cast<char*>(work);

  // per-field table, grouped by class
  std::vector<FieldIO> io;
  io.reserve(njobs);
  for (const Class& c : cls)
    for (int j : c.jobs) {
      const hu_job& jb = jobs[j];
      FieldIO f{};
      f.field = jb.field;
      f.pm1 = jb.pm1;
      f.stats = jb.stats;
      f.counts = jb.counts;
      f.cont_sum = jb.cont_sum;
      f.cont_cnt = jb.cont_cnt;
      f.pm1_sum = jb.pm1_sum;
      f.pm1_cnt = jb.pm1_cnt;
      f.seed = jb.seed;
      f.sigma_f = jb.filt.sigma_f;
      f.near_abs = (float)(near_tol * jb.filt.sigma_f);
      f.filt = filt_dev(jb.filt, c.g);
      io.push_back(f);
    }
  FieldIO* io_dev = reinterpret_cast<FieldIO*>(w);

  // graph key: the class structure, the tuned variants and the workspace
  std::string key;
  char buf[256];
  std::snprintf(buf, sizeof buf, "w%p|n%d|", work, njobs);
  key += buf;
  std::vector<TunePlan> plans;
  for (const Class& c : cls) {
    const TunePlan p = get_plan(c.g, c.has_bins ? &c.bins : nullptr, (int)c.jobs.size());
    plans.push_back(p);
    std::snprintf(buf, sizeof buf, "%d:%d,%d,%d:%d,%d:%zu:%d%d%d:", c.g.nd, c.g.n[0], c.g.n[1], c.g.n[2],
                  c.has_bins ? c.bins.n_radial : 0, c.has_bins ? c.bins.n_angular : 0, c.jobs.size(), c.want_cont,
                  c.want_pm1, c.any_gen);
    key += buf;
    for (int k = 0; k < NPASS; ++k) key += (char)('0' + p.v[k]);   // every plan entry: a changed
    key += '|';                                                     // plan captures a new graph
  }

  std::lock_guard<std::mutex> lk(g_bmu);
  HU_TRY(ensure_streams());
  for (const Class& c : cls) HU_TRY(prepare_tables(c.g, c.has_bins ? &c.bins : nullptr, st));
  if (!g_stage_done) HU_HIP(hipEventCreateWithFlags(&g_stage_done, hipEventDisableTiming));
  HU_HIP(hipEventSynchronize(g_stage_done));          // the previous upload has read the staging buffer
  if (g_stage_n < io.size()) {
    if (g_stage) (void)hipHostFree(g_stage);
    g_stage = nullptr;
    g_stage_n = 0;
    HU_HIP(hipHostMalloc((void**)&g_stage, io.size() * sizeof(FieldIO), hipHostMallocDefault));
    g_stage_n = io.size();
  }
  std::memcpy(g_stage, io.data(), io.size() * sizeof(FieldIO));
  HU_HIP(hipMemcpyAsync(io_dev, g_stage, io.size() * sizeof(FieldIO), hipMemcpyHostToDevice, st));
  HU_HIP(hipEventRecord(g_stage_done, st));

  auto it = g_graphs.find(key);
  if (it == g_graphs.end()) {
    const bool prof = g_prof;
    g_prof = false;                       // no timing events inside a captured graph
    hipGraph_t graph = nullptr;
    int rc = HU_OK;
    if (hipStreamBeginCapture(g_cap, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = HU_ERR_HIP;
    if (rc == HU_OK && hipEventRecord(g_fork, g_cap) != hipSuccess) rc = HU_ERR_HIP;
    for (int s = 0; rc == HU_OK && s < NSIDE; ++s)
      if (hipStreamWaitEvent(g_side[s], g_fork, 0) != hipSuccess) rc = HU_ERR_HIP;
    for (size_t i = 0; rc == HU_OK && i < cls.size(); ++i) {
      const Class& c = cls[i];
      ClassRun r{};
      r.g = c.g;
      r.B = (int)c.jobs.size();
      r.plan = plans[i];
      r.bins = c.has_bins ? &c.bins : nullptr;
      r.thresh = true;
      r.io = io_dev + c.io_off;
      r.want_cont = c.want_cont;
      r.want_pm1_spec = c.want_pm1;
      r.any_gen = c.any_gen;
      r.work = w + c.work_off;
      r.lay = c.lay;
      rc = enqueue_class(r, g_side[i % NSIDE]);
    }
    for (int s = 0; rc == HU_OK && s < NSIDE; ++s) {
      if (hipEventRecord(g_join[s], g_side[s]) != hipSuccess || hipStreamWaitEvent(g_cap, g_join[s], 0) != hipSuccess)
        rc = HU_ERR_HIP;
    }
    const hipError_t ec = hipStreamEndCapture(g_cap, &graph);
    g_prof = prof;
    if (rc != HU_OK || ec != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc != HU_OK ? rc : HU_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return HU_ERR_HIP;
    if (g_graphs.size() >= 16) {
      (void)hipGraphExecDestroy(g_graphs.begin()->second);
      g_graphs.erase(g_graphs.begin());
    }
    it = g_graphs.emplace(key, exec).first;
  }
  HU_HIP(hipGraphLaunch(it->second, st));
  return HU_OK;
}

int hu_plan_query(hu_dims dims, int32_t batch, const hu_bins* bins, int32_t* variants) {
  if (!variants || batch < 1) return HU_ERR_ARG;
  Geom g;
  HU_TRY(make_geom(dims, &g));
  if (bins) HU_TRY(check_bins(bins, g.nd));
  const TunePlan p = get_plan(g, bins, batch);
  for (int i = 0; i < NPASS; ++i) variants[i] = p.v[i];
  return HU_OK;
}

int hu_plan_set(hu_dims dims, int32_t batch, const hu_bins* bins, const int32_t* variants) {
  if (!variants || batch < 1) return HU_ERR_ARG;
  Geom g;
  HU_TRY(make_geom(dims, &g));
  if (bins) HU_TRY(check_bins(bins, g.nd));
  TunePlan p{};
  for (int i = 0; i < NPASS; ++i) {
    if (variants[i] != 0 && variants[i] != 1) return HU_ERR_ARG;
    p.v[i] = variants[i];
  }
  set_plan(plan_key(g, bins, batch), p);
  return HU_OK;
}

int hu_autotune(hu_dims dims, int32_t batch, const hu_bins* bins, const char* cache_path, double* ms_out) {
  Geom g;
  HU_TRY(make_geom(dims, &g));
  if (batch < 1 || !bins) return HU_ERR_ARG;
  HU_TRY(check_bins(bins, g.nd));
  const int B = batch;
  const int nb = bins->n_radial * bins->n_angular + 1;
  const int chunk = B < MAX_CHUNK ? B : MAX_CHUNK;
  Layout lay;
  HU_TRY(layout(g, chunk, true, widest(), bins, &lay));
  hipStream_t st = nullptr;
  HU_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  float* field = nullptr;
  int8_t* pm1 = nullptr;
  double *stats = nullptr, *cs = nullptr, *ps = nullptr;
  uint64_t *counts = nullptr, *cc = nullptr, *pc = nullptr;
  char* work = nullptr;
  int rc = HU_OK;
  auto mal = [&](void** p, size_t n) {
    if (rc == HU_OK && hipMalloc(p, n) != hipSuccess) rc = HU_ERR_HIP;
  };
  mal((void**)&field, sizeof(float) * g.N * B);
  mal((void**)&pm1, g.N * B);
  mal((void**)&stats, sizeof(double) * 4 * B);
  mal((void**)&counts, sizeof(uint64_t) * 2 * B);
  mal((void**)&cs, sizeof(double) * nb * B);
  mal((void**)&ps, sizeof(double) * nb * B);
  mal((void**)&cc, sizeof(uint64_t) * nb * B);
  mal((void**)&pc, sizeof(uint64_t) * nb * B);
  mal((void**)&work, lay.total);
  hu_filter f{};
  f.p = 2.0;
  f.semi[0] = f.semi[1] = f.semi[2] = 1.0;
  f.rot = 0.3;
  f.alpha = 2.0;
  f.k0 = 0.2;
  f.width = 0.05;
  f.sigma_f = 1.0;
  std::vector<uint64_t> seeds(B);
  for (int i = 0; i < B; ++i) seeds[i] = 1 + i;
  hu_outputs o{field, pm1, stats, counts, cs, cc, ps, pc};
  if (rc == HU_OK) rc = prepare_tables(g, bins, st);

  // the summed mean kernel time of the whole pass sequence under a plan (2 untimed runs, 5 timed)
  auto time_plan = [&](const TunePlan& plan) -> double {
    auto run = [&]() {
      const int step = plan.v[P_WHOLE] && whole_field_ok(g, nb) ? MAX_WHOLE_CHUNK : MAX_CHUNK;
      for (int f0 = 0; f0 < B && rc == HU_OK; f0 += step) {
        ClassRun r{};
        r.g = g;
        r.B = B - f0 < step ? B - f0 : step;
        r.plan = plan;
        r.bins = bins;
        r.thresh = true;
        r.filt = f;
        r.seeds = seeds.data() + f0;
        r.near_abs = 1e-5f;
        hu_outputs oc = o;
        oc.field += (long long)f0 * g.N;
        oc.pm1 += (long long)f0 * g.N;
        oc.stats += 4LL * f0;
        oc.counts += 2LL * f0;
        oc.cont_sum += (long long)f0 * nb;
        oc.cont_cnt += (long long)f0 * nb;
        oc.pm1_sum += (long long)f0 * nb;
        oc.pm1_cnt += (long long)f0 * nb;
        r.out = oc;
        r.work = work;
        r.lay = lay;
        rc = enqueue_class(r, st);
      }
    };
    run();
    run();
    if (rc == HU_OK && hipStreamSynchronize(st) != hipSuccess) rc = HU_ERR_HIP;
    if (rc != HU_OK) return 0.0;
    const bool prof = g_prof;
    rc = profile_reset(true);
    for (int k = 0; k < 5 && rc == HU_OK; ++k) run();
    std::vector<std::string> names;
    std::vector<long long> cnt;
    std::vector<double> ms;
    if (rc == HU_OK) rc = profile_collect(names, cnt, ms);
    (void)profile_reset(prof);
    double t = 0.0;
    for (double m : ms) t += m / 5.0;
    return t;
  };

  // paired comparison: the two plans timed alternately twice, the faster time of each kept, so
  // clock ramps and other drifts hit both alike
  auto paired = [&](const TunePlan& a, const TunePlan& b, double& ta, double& tb) {
    ta = tb = 1e30;
    for (int rep = 0; rep < 2 && rc == HU_OK; ++rep) {
      ta = std::min(ta, time_plan(a));
      tb = std::min(tb, time_plan(b));
    }
  };

  // coordinate search from the default plan: each choice flipped in turn, kept when the pass
  // sequence gets at least 1 % faster (the y-pass choices only exist in 3D, the radix choice where
  // a column length has an alternative list).  The GPU first runs the sequence for about 50 ms of
  // kernel time, so that its clocks have settled before the first comparison.
  double tried[NPASS] = {};
  TunePlan best{};
  double warm = 0.0;
  for (int i = 0; i < 64 && warm < 50.0 && rc == HU_OK; ++i) warm += 7.0 * time_plan(best);
  // a second sweep when the first changed something (choices interact: the split exchange only
  // adds resident workgroups together with the narrower filter tiles)
  for (int sweep = 0; sweep < 2 && rc == HU_OK; ++sweep) {
    bool changed = false;
    for (int k = 0; k < NPASS && rc == HU_OK; ++k) {
      if (g.nd == 2 && (k == P_COLY || k == P_YGROUP)) continue;
      if (k == P_RADIX && !plan_has_alt(g.n[0]) && !(g.nd == 3 && plan_has_alt(g.n[1]))) continue;
      if ((k == P_BSPLIT || k == P_FSPLIT) && !split_length(g.n[0])) continue;
      if (k == P_WHOLE && !whole_field_ok(g, nb)) continue;
      if (k == P_PLANE && !plane_ok(g)) continue;
      TunePlan cand = best;
      cand.v[k] ^= 1;
      double tb = 0.0, tc = 0.0;
      paired(best, cand, tb, tc);
      if (rc != HU_OK) break;
      tried[k] = tc;
      if (tc > 0.0 && tc < 0.99 * tb) {
        best = cand;
        changed = true;
      }
    }
    if (!changed) break;
  }
  // the default and the tuned plan measured side by side once the search is done; the default is
  // kept unless the tuned plan still wins there
  double t_default = 0.0, t_best = 0.0;
  if (rc == HU_OK) paired(TunePlan{}, best, t_default, t_best);
  bool same = true;
  for (int k = 0; k < NPASS; ++k) same = same && best.v[k] == 0;
  if (same || t_best >= t_default) {
    best = TunePlan{};
    t_default = t_best = std::min(t_default, t_best);
  }
  if (rc == HU_OK) {
    set_plan(plan_key(g, bins, B), best);
    if (ms_out) {
      ms_out[0] = t_default;
      ms_out[1] = t_best;
      for (int k = 0; k < NPASS; ++k) ms_out[2 + k] = tried[k];
    }
    if (cache_path) rc = save_plans(cache_path);
  }
  (void)hipStreamSynchronize(st);
  void* bufs[] = {field, pm1, stats, counts, cs, ps, cc, pc, work};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  (void)hipStreamDestroy(st);
  return rc;
}

}  // extern "C"
