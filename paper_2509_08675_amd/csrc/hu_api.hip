// C-ABI of the hyperuniform-field library: validation, per-size tables, workspace layout and the
// pass sequence of each entry point.  Declarations and contracts are in include/hufield.h.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <utility>
#include <vector>

#include "hufield.h"
#include "hu_internal.hpp"

using namespace hu;

namespace {

std::mutex g_mu;

// ---------------------------------------------------------------------------------------------
// per-device read-only tables, created on first use of a size and kept for the process
// ---------------------------------------------------------------------------------------------
std::map<std::pair<int, int>, float2*> g_tw, g_tw2;
std::map<std::pair<int, int>, double*> g_edges;

int current_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

// FP64 twiddles rounded once to FP32: tw[t] = exp(-2 pi i t / n) for t < count
int make_table(int n, int count, float2** out) {
  std::vector<float2> h(count);
  for (int t = 0; t < count; ++t) {
    const double a = 2.0 * M_PI * (double)t / (double)n;
    h[t] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
  float2* d = nullptr;
  if (hipMalloc(&d, sizeof(float2) * count) != hipSuccess) return HU_ERR_HIP;
  if (hipMemcpy(d, h.data(), sizeof(float2) * count, hipMemcpyHostToDevice) != hipSuccess) return HU_ERR_HIP;
  *out = d;
  return HU_OK;
}

int get_tw(int L, const float2** tw) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(current_device(), L);
  auto it = g_tw.find(key);
  if (it == g_tw.end()) {
    float2* d;
    int rc = make_table(L, L, &d);
    if (rc) return rc;
    it = g_tw.emplace(key, d).first;
  }
  *tw = it->second;
  return HU_OK;
}

int get_tw2(int L, const float2** tw2) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(current_device(), L);
  auto it = g_tw2.find(key);
  if (it == g_tw2.end()) {
    float2* d;
    int rc = make_table(2 * L, L, &d);
    if (rc) return rc;
    it = g_tw2.emplace(key, d).first;
  }
  *tw2 = it->second;
  return HU_OK;
}

// angular edge unit vectors e_j = (cos j pi / A, sin j pi / A), j = 1..A-1, with the 45, 90 and
// 135 degree edges set to exactly equal magnitudes so that the exact-tangent tests are exact
int get_edges(int na, const double** ex, const double** ey) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int m = na > 1 ? na - 1 : 1;
  auto key = std::make_pair(current_device(), na);
  auto it = g_edges.find(key);
  if (it == g_edges.end()) {
    std::vector<double> h(2 * m, 0.0);
    const double c = std::cos(M_PI / 4.0);
    for (int j = 1; j < na; ++j) {
      double x, y;
      if (4 * j == na) { x = c; y = c; }
      else if (2 * j == na) { x = 0.0; y = 1.0; }
      else if (4 * j == 3 * na) { x = -c; y = c; }
      else { x = std::cos(j * M_PI / na); y = std::sin(j * M_PI / na); }
      h[j - 1] = x;
      h[m + j - 1] = y;
    }
    double* d = nullptr;
    if (hipMalloc(&d, sizeof(double) * 2 * m) != hipSuccess) return HU_ERR_HIP;
    if (hipMemcpy(d, h.data(), sizeof(double) * 2 * m, hipMemcpyHostToDevice) != hipSuccess) return HU_ERR_HIP;
    it = g_edges.emplace(key, d).first;
  }
  *ex = it->second;
  *ey = it->second + m;
  return HU_OK;
}

// ---------------------------------------------------------------------------------------------
// bin geometry per (device, grid, bins): the bin of every half-spectrum mode as a u16 table
// (column-major for the axis-0 passes; kept when it is at most 64 MiB, else bins are computed in
// the kernels) and the per-bin mode counts, built once by a kernel on the caller's stream.
// ---------------------------------------------------------------------------------------------
struct BinGeo {
  uint16_t* table;
  unsigned long long* counts;
};
std::map<std::vector<long long>, BinGeo> g_bingeo;

// ---------------------------------------------------------------------------------------------
// profiling: events around every launch while enabled
// ---------------------------------------------------------------------------------------------
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
bool g_prof = false;
std::vector<ProfRec> g_recs;
std::vector<hipEvent_t> g_pool;
size_t g_pool_next = 0;

hipEvent_t pool_event() {
  if (g_pool_next == g_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_pool.push_back(e);
  }
  return g_pool[g_pool_next++];
}

template <class F>
hipError_t timed(const char* name, hipStream_t st, F&& f) {
  if (!g_prof) return f();
  hipEvent_t a = pool_event(), b = pool_event();
  if (!a || !b) return f();
  (void)hipEventRecord(a, st);
  hipError_t e = f();
  (void)hipEventRecord(b, st);
  g_recs.push_back({name, a, b});
  return e;
}

// ---------------------------------------------------------------------------------------------
// validation and geometry
// ---------------------------------------------------------------------------------------------
bool supported_len(long long n) {
  if (n < 4 || n > 2048) return false;
  long long m = n;
  if (m % 3 == 0) {
    m /= 3;
    if (n > 768) return false;
  }
  return (m & (m - 1)) == 0;
}

bool supported_row_len(long long L) {
  if (L < 2 || L > 1024) return false;
  long long m = L;
  if (m % 3 == 0) {
    m /= 3;
    if (L > 384) return false;
  }
  return (m & (m - 1)) == 0;
}

struct Geom {
  int nd;
  int n[3];
  int nx, nxh;
  long long N, Nh, nrows;
  long long D;
  int tiled;        // 2D: half spectrum in column groups of 4 (TW = 4); 3D: row-major
  long long Nhp;    // per-field half-spectrum storage (padded to whole column groups in 2D)
};

long long lcm_ll(long long a, long long b) { return a / std::gcd(a, b) * b; }

int make_geom(const hu_dims& d, Geom* g) {
  if (d.ndim != 2 && d.ndim != 3) return HU_ERR_ARG;
  g->nd = d.ndim;
  g->N = 1;
  g->D = 1;
  for (int i = 0; i < d.ndim; ++i) {
    if (!supported_len(d.n[i])) return HU_ERR_SIZE;
    g->n[i] = d.n[i];
    g->N *= d.n[i];
    g->D = lcm_ll(g->D, d.n[i]);
  }
  g->nx = d.n[d.ndim - 1];
  if (!supported_row_len(g->nx / 2)) return HU_ERR_SIZE;
  g->nxh = g->nx / 2 + 1;
  g->nrows = g->N / g->nx;
  g->Nh = g->nrows * g->nxh;
  g->tiled = d.ndim == 2 ? 1 : 0;
  g->Nhp = g->tiled ? g->nrows * ((g->nxh + 3) / 4 * 4) : g->Nh;
  if (g->N >= (1LL << 31)) return HU_ERR_SIZE;      // in-field offsets are 32-bit
  return HU_OK;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_filter(const hu_filter* f, int nd) {
  if (!f) return HU_ERR_ARG;
  if (!finite_pos(f->p) || !finite_pos(f->semi[0]) || !finite_pos(f->semi[1])) return HU_ERR_ARG;
  if (nd == 3 && !finite_pos(f->semi[2])) return HU_ERR_ARG;
  if (!finite_pos(f->alpha) || !finite_pos(f->width) || !finite_pos(f->sigma_f)) return HU_ERR_ARG;
  if (!std::isfinite(f->rot) || !std::isfinite(f->k0) || f->k0 < 0.0) return HU_ERR_ARG;
  return HU_OK;
}

int check_bins(const hu_bins* b, int nd) {
  if (!b) return HU_ERR_ARG;
  if (b->n_radial < 1 || b->n_angular < 1) return HU_ERR_ARG;
  if (b->n_angular > 1 && nd != 2) return HU_ERR_ARG;
  if ((long long)b->n_radial * b->n_angular + 1 > 8192) return HU_ERR_ARG;
  return HU_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t spec, partials, fstats, total;
  int tiles;
};

Layout layout(const Geom& g, int batch, bool need_stats) {
  Layout L{};
  size_t off = 0;
  L.spec = off;
  off += up256((size_t)batch * g.Nhp * sizeof(float2));
  L.tiles = col_tiles(g.n[0], g.Nh / g.n[0]);
  if (need_stats) {
    L.partials = off;
    off += up256((size_t)batch * L.tiles * 4 * sizeof(double));
    L.fstats = off;
    off += up256((size_t)batch * 8 * sizeof(double));
  }
  L.total = off;
  return L;
}

FiltDev filt_dev(const hu_filter& f) {
  FiltDev d{};
  d.cr = (float)std::cos(f.rot);
  d.sr = (float)std::sin(f.rot);
  d.ia = (float)(1.0 / f.semi[0]);
  d.ib = (float)(1.0 / f.semi[1]);
  d.ic = (float)(1.0 / f.semi[2]);
  d.p = (float)f.p;
  d.ip = (float)(1.0 / f.p);
  d.alpha = (float)f.alpha;
  d.k0 = (float)f.k0;
  d.inv2w2 = (float)(1.0 / (2.0 * f.width * f.width));
  const double ks = 0.5 * (f.k0 + std::sqrt(f.k0 * f.k0 + 4.0 * f.alpha * f.width * f.width));
  const double dd = ks - f.k0;
  d.lnchimax = (float)(f.alpha * std::log(ks) - dd * dd / (2.0 * f.width * f.width));
  d.rotated = (f.rot != 0.0) ? 1 : 0;
  return d;
}

Axis0Geom axis0(const Geom& g) {
  Axis0Geom a{};
  a.ndim = g.nd;
  a.n0 = g.n[0];
  a.ny = g.nd == 3 ? g.n[1] : 0;
  a.nx = g.nx;
  a.nxh = g.nxh;
  a.ncol = (int)(g.Nh / g.n[0]);
  a.inner0 = g.tiled ? 4 : a.ncol;
  a.kap0 = (float)(2.0 / g.n[0]);
  a.kapy = g.nd == 3 ? (float)(2.0 / g.n[1]) : 0.0f;
  a.kapx = (float)(2.0 / g.nx);
  a.dfac_0 = g.D / g.n[0];
  a.dfac_y = g.nd == 3 ? g.D / g.n[1] : 0;
  a.dfac_x = g.D / g.nx;
  return a;
}

int make_bindev(const Geom& g, const hu_bins& b, BinDev* bd) {
  bd->nr = b.n_radial;
  bd->na = b.n_angular;
  bd->D2 = g.D * g.D;
  bd->invD2 = (float)(1.0 / (double)(g.D * g.D));
  bd->fourR2 = 4LL * b.n_radial * b.n_radial;
  return get_edges(b.n_angular, &bd->ex, &bd->ey);
}

#define HU_TRY(expr)                         \
  do {                                       \
    int _rc = (expr);                        \
    if (_rc != HU_OK) return _rc;            \
  } while (0)
#define HU_HIP(expr)                         \
  do {                                       \
    if ((expr) != hipSuccess) return HU_ERR_HIP; \
  } while (0)

int get_bingeo(const Geom& g, const hu_bins& bins, const BinDev& bd, hipStream_t st, BinGeo* out) {
  std::vector<long long> key = {current_device(), g.nd, g.n[0], g.n[1], g.nd == 3 ? g.n[2] : 0,
                                bins.n_radial, bins.n_angular};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_bingeo.find(key);
    if (it != g_bingeo.end()) {
      *out = it->second;
      return HU_OK;
    }
  }
  const int nb = bins.n_radial * bins.n_angular + 1;
  BinGeo geo{nullptr, nullptr};
  HU_HIP(hipMalloc(&geo.counts, sizeof(unsigned long long) * nb));
  if ((size_t)g.Nh * sizeof(uint16_t) <= ((size_t)64 << 20)) HU_HIP(hipMalloc(&geo.table, sizeof(uint16_t) * g.Nh));
  HU_HIP(launch_zero_u64(reinterpret_cast<uint64_t*>(geo.counts), nb, st));
  BinGeomArgs ba{};
  ba.Nh = g.Nh;
  ba.gm = axis0(g);
  ba.bd = bd;
  ba.nb = nb;
  ba.table = geo.table;
  ba.counts = geo.counts;
  HU_HIP(launch_bin_geom(ba, st));
  HU_HIP(hipStreamSynchronize(st));          // complete before any stream can use it
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_bingeo.find(key);
  if (it != g_bingeo.end()) {                // another thread built it meanwhile
    (void)hipFree(geo.counts);
    if (geo.table) (void)hipFree(geo.table);
    *out = it->second;
    return HU_OK;
  }
  g_bingeo.emplace(key, geo);
  *out = geo;
  return HU_OK;
}

// The generator's pass sequence for one chunk of <= MAX_CHUNK fields whose outputs are already
// offset to the chunk.  Pass order (3D; 2D skips the y passes):
//   rows_r2c(noise) -> cols(y, fwd) -> cols_filter(z) -> cols(y, inv) -> rows_c2r
//   [-> cols(y, fwd) -> cols_bin(z)]   for the +-1 spectrum
int run_chunk(const Geom& g, int B, const hu_filter& f, const uint64_t* seeds, const hu_bins* bins,
              float near_abs, bool thresh, const hu_outputs& o, char* work, const Layout& lay, hipStream_t st) {
  const int Lrow = g.nx / 2;
  const float2 *tw_row, *tw2_row, *tw_0, *tw_1 = nullptr;
  HU_TRY(get_tw(Lrow, &tw_row));
  HU_TRY(get_tw2(Lrow, &tw2_row));
  HU_TRY(get_tw(g.n[0], &tw_0));
  if (g.nd == 3) HU_TRY(get_tw(g.n[1], &tw_1));
  const int nb = bins ? bins->n_radial * bins->n_angular + 1 : 0;
  BinDev bd{};
  BinGeo geo{nullptr, nullptr};
  if (bins) {
    HU_TRY(make_bindev(g, *bins, &bd));
    HU_TRY(get_bingeo(g, *bins, bd, st, &geo));
  }

  float2* spec = reinterpret_cast<float2*>(work + lay.spec);
  double* partials = reinterpret_cast<double*>(work + lay.partials);
  double* fstats = reinterpret_cast<double*>(work + lay.fstats);
  const uint32_t* cnt_src = reinterpret_cast<const uint32_t*>(geo.counts);

  // pass A: noise -> R2C rows; block 0 of each field sets up that field's accumulators
  RowsArgs ra{};
  ra.spec = spec;
  ra.Nh = g.Nhp;
  ra.tiled = g.tiled;
  ra.N = g.N;
  ra.nrows = g.nrows;
  for (int i = 0; i < B; ++i) ra.seeds[i] = seeds[i];
  ra.tw = tw_row;
  ra.tw2 = tw2_row;
  int fs = 0;
  if (o.cont_sum) ra.fill[fs++] = FillSpan{reinterpret_cast<uint32_t*>(o.cont_sum), nullptr, 2 * nb};
  if (o.cont_cnt) ra.fill[fs++] = FillSpan{reinterpret_cast<uint32_t*>(o.cont_cnt), cnt_src, 2 * nb};
  if (o.pm1_sum) ra.fill[fs++] = FillSpan{reinterpret_cast<uint32_t*>(o.pm1_sum), nullptr, 2 * nb};
  if (o.pm1_cnt) ra.fill[fs++] = FillSpan{reinterpret_cast<uint32_t*>(o.pm1_cnt), cnt_src, 2 * nb};
  if (o.counts) ra.fill[fs++] = FillSpan{reinterpret_cast<uint32_t*>(o.counts), nullptr, 4};
  ra.fill_spans = fs;
  HU_HIP(timed("rows_r2c_noise", st, [&] { return launch_rows_r2c(Lrow, SRC_NOISE, ra, B, st); }));

  ColsArgs cy{};
  if (g.nd == 3) {
    cy.spec = spec;
    cy.Nh = g.Nhp;
    cy.ncol = g.n[0] * g.nxh;
    cy.inner = g.nxh;
    cy.tw = tw_1;
    cy.sc = col_sched(g.n[1], cy.ncol, B);
    HU_HIP(timed("cols_y_fwd", st, [&] { return launch_cols(g.n[1], false, cy, B, st); }));
  }

  FilterArgs fa{};
  fa.spec = spec;
  fa.Nh = g.Nhp;
  fa.N = g.N;
  fa.gm = axis0(g);
  fa.sc = col_sched(g.n[0], fa.gm.ncol, B);
  fa.filt = filt_dev(f);
  fa.bd = bd;
  fa.nb = o.cont_sum ? nb : 0;
  fa.table = geo.table;
  fa.tw = tw_0;
  fa.partials = partials;
  fa.cont_sum = o.cont_sum;
  HU_HIP(timed("cols_filter", st, [&] { return launch_cols_filter(g.n[0], fa, B, st); }));
  FinalizeArgs fz{};
  fz.partials = partials;
  fz.ntiles = fa.sc.ntiles;
  fz.N = g.N;
  fz.sigma_f = f.sigma_f;
  fz.fstats = fstats;
  fz.stats = o.stats;
  fz.cont_sum = o.cont_sum;
  fz.nb = nb;
  HU_HIP(timed("finalize", st, [&] { return launch_finalize(fz, B, st); }));

  if (g.nd == 3) HU_HIP(timed("cols_y_inv", st, [&] { return launch_cols(g.n[1], true, cy, B, st); }));

  RowsZArgs za{};
  za.spec = spec;
  za.Nh = g.Nhp;
  za.tiled = g.tiled;
  za.N = g.N;
  za.nrows = g.nrows;
  za.tw = tw_row;
  za.tw2 = tw2_row;
  za.fstats = fstats;
  za.field = o.field;
  za.pm1 = o.pm1;
  za.counts = o.counts;
  za.near_tol = near_abs;
  HU_HIP(timed(thresh ? "rows_c2r_thresh" : "rows_c2r", st, [&] { return launch_rows_c2r(Lrow, thresh, za, B, st); }));

  if (thresh && o.pm1_sum) {
    if (g.nd == 3) HU_HIP(timed("cols_y_fwd", st, [&] { return launch_cols(g.n[1], false, cy, B, st); }));
    BinArgs ba{};
    ba.spec = spec;
    ba.Nh = g.Nhp;
    ba.N = g.N;
    ba.gm = axis0(g);
    ba.sc = col_sched(g.n[0], ba.gm.ncol, B);
    ba.bd = bd;
    ba.nb = nb;
    ba.table = geo.table;
    ba.tw = tw_0;
    ba.sum = o.pm1_sum;
    HU_HIP(timed("cols_bin", st, [&] { return launch_cols_bin(g.n[0], ba, B, st); }));
  }
  return HU_OK;
}

hu_outputs offset_outputs(const hu_outputs& o, long long f0, long long N, int nb) {
  hu_outputs r = o;
  if (r.field) r.field += f0 * N;
  if (r.pm1) r.pm1 += f0 * N;
  if (r.stats) r.stats += f0 * 4;
  if (r.counts) r.counts += f0 * 2;
  if (r.cont_sum) r.cont_sum += f0 * nb;
  if (r.cont_cnt) r.cont_cnt += f0 * nb;
  if (r.pm1_sum) r.pm1_sum += f0 * nb;
  if (r.pm1_cnt) r.pm1_cnt += f0 * nb;
  return r;
}

int run_generator(hu_dims dims, int32_t batch, const hu_filter* filt, const uint64_t* seeds, const hu_bins* bins,
                  float near_tol_rel, const hu_outputs& o, bool thresh, void* work, size_t work_bytes, void* stream) {
  Geom g;
  HU_TRY(make_geom(dims, &g));
  if (batch < 1 || !seeds) return HU_ERR_ARG;
  HU_TRY(check_filter(filt, g.nd));
  if (bins) HU_TRY(check_bins(bins, g.nd));
  if ((o.cont_sum || o.pm1_sum) && !bins) return HU_ERR_ARG;
  if (thresh && !o.pm1 && !o.pm1_sum && !o.counts && !o.field) return HU_ERR_ARG;
  if (!thresh && !o.field && !o.stats && !o.cont_sum) return HU_ERR_ARG;
  if (!std::isfinite(near_tol_rel) || near_tol_rel < 0.0f) return HU_ERR_ARG;
  const void* ptrs[] = {o.field, o.pm1, o.stats, o.counts, o.cont_sum, o.cont_cnt, o.pm1_sum, o.pm1_cnt};
  for (const void* p : ptrs)
    if (p && !aligned(p, 16)) return HU_ERR_ALIGN;
  if (!work || !aligned(work, 256)) return work ? HU_ERR_ALIGN : HU_ERR_ARG;
  const Layout lay = layout(g, batch < MAX_CHUNK ? batch : MAX_CHUNK, true);
  if (work_bytes < lay.total) return HU_ERR_WORKSPACE;
  const int nb = bins ? bins->n_radial * bins->n_angular + 1 : 0;
  const float near_abs = (float)(near_tol_rel * filt->sigma_f);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int f0 = 0; f0 < batch; f0 += MAX_CHUNK) {
    const int B = batch - f0 < MAX_CHUNK ? batch - f0 : MAX_CHUNK;
    hu_outputs oc = offset_outputs(o, f0, g.N, nb);
    HU_TRY(run_chunk(g, B, *filt, seeds + f0, bins, near_abs, thresh, oc, reinterpret_cast<char*>(work), lay, st));
  }
  return HU_OK;
}

}  // namespace

// =============================================================================================
// C-ABI
// =============================================================================================
extern "C" {

int hu_workspace_size(int op, hu_dims dims, int32_t batch, const hu_bins* bins, size_t* bytes) {
  if (!bytes || batch < 1) return HU_ERR_ARG;
  Geom g;
  HU_TRY(make_geom(dims, &g));
  if (bins) HU_TRY(check_bins(bins, g.nd));
  const int chunk = batch < MAX_CHUNK ? batch : MAX_CHUNK;
  switch (op) {
    case HU_OP_GEN_FIELD:
    case HU_OP_PIPELINE:
      *bytes = layout(g, chunk, true).total;
      return HU_OK;
    case HU_OP_POWER_SPECTRUM:
      *bytes = layout(g, chunk, false).total;
      return HU_OK;
    default:
      return HU_ERR_ARG;
  }
}

int hu_gen_field(hu_dims dims, int32_t batch, const hu_filter* filt, const uint64_t* seeds, float* field,
                 double* stats, const hu_bins* cont_bins, double* cont_sum, uint64_t* cont_cnt, void* work,
                 size_t work_bytes, void* stream) {
  hu_outputs o{};
  o.field = field;
  o.stats = stats;
  if (cont_bins) {
    if (!cont_sum) return HU_ERR_ARG;
    o.cont_sum = cont_sum;
    o.cont_cnt = cont_cnt;
  }
  if (!field) return HU_ERR_ARG;
  return run_generator(dims, batch, filt, seeds, cont_bins, 0.0f, o, false, work, work_bytes, stream);
}

int hu_pipeline(hu_dims dims, int32_t batch, const hu_filter* filt, const uint64_t* seeds, hu_bins bins,
                float near_tol, const hu_outputs* out, void* work, size_t work_bytes, void* stream) {
  if (!out) return HU_ERR_ARG;
  return run_generator(dims, batch, filt, seeds, &bins, near_tol, *out, true, work, work_bytes, stream);
}

int hu_threshold(hu_dims dims, int32_t batch, const float* field, int8_t* out, uint64_t* counts, float near_tol,
                 void* stream) {
  Geom g;
  HU_TRY(make_geom(dims, &g));
  if (batch < 1 || !field || !out) return HU_ERR_ARG;
  if (!std::isfinite(near_tol) || near_tol < 0.0f) return HU_ERR_ARG;
  if (!aligned(field, 16) || !aligned(out, 16) || (counts && !aligned(counts, 16))) return HU_ERR_ALIGN;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (counts) HU_HIP(timed("zero", st, [&] { return launch_zero_u64(counts, 2LL * batch, st); }));
  ThreshArgs a{field, out, counts, g.N, near_tol};
  HU_HIP(timed("threshold", st, [&] { return launch_threshold(a, batch, st); }));
  return HU_OK;
}

int hu_power_spectrum(hu_dims dims, int32_t batch, const void* x, int32_t dtype, hu_bins bins, double* sum,
                      uint64_t* cnt, void* work, size_t work_bytes, void* stream) {
  Geom g;
  HU_TRY(make_geom(dims, &g));
  HU_TRY(check_bins(&bins, g.nd));
  if (batch < 1 || !x || !sum) return HU_ERR_ARG;
  if (dtype != HU_F32 && dtype != HU_I8) return HU_ERR_ARG;
  if (!aligned(x, 16) || !aligned(sum, 16) || (cnt && !aligned(cnt, 16))) return HU_ERR_ALIGN;
  if (!work || !aligned(work, 256)) return work ? HU_ERR_ALIGN : HU_ERR_ARG;
  const Layout lay = layout(g, batch < MAX_CHUNK ? batch : MAX_CHUNK, false);
  if (work_bytes < lay.total) return HU_ERR_WORKSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int Lrow = g.nx / 2;
  const int nb = bins.n_radial * bins.n_angular + 1;
  const float2 *tw_row, *tw2_row, *tw_0, *tw_1 = nullptr;
  HU_TRY(get_tw(Lrow, &tw_row));
  HU_TRY(get_tw2(Lrow, &tw2_row));
  HU_TRY(get_tw(g.n[0], &tw_0));
  if (g.nd == 3) HU_TRY(get_tw(g.n[1], &tw_1));
  BinDev bd{};
  HU_TRY(make_bindev(g, bins, &bd));
  BinGeo geo{nullptr, nullptr};
  HU_TRY(get_bingeo(g, bins, bd, st, &geo));
  float2* spec = reinterpret_cast<float2*>(reinterpret_cast<char*>(work) + lay.spec);
  const size_t esz = dtype == HU_F32 ? 4 : 1;
  for (int f0 = 0; f0 < batch; f0 += MAX_CHUNK) {
    const int B = batch - f0 < MAX_CHUNK ? batch - f0 : MAX_CHUNK;
    RowsArgs ra{};
    ra.spec = spec;
    ra.Nh = g.Nhp;
  ra.tiled = g.tiled;
    ra.N = g.N;
    ra.nrows = g.nrows;
    ra.src = reinterpret_cast<const char*>(x) + (size_t)f0 * g.N * esz;
    ra.tw = tw_row;
    ra.tw2 = tw2_row;
    double* s = sum + (long long)f0 * nb;
    uint64_t* c = cnt ? cnt + (long long)f0 * nb : nullptr;
    int fs = 0;
    ra.fill[fs++] = FillSpan{reinterpret_cast<uint32_t*>(s), nullptr, 2 * nb};
    if (c) ra.fill[fs++] = FillSpan{reinterpret_cast<uint32_t*>(c), reinterpret_cast<const uint32_t*>(geo.counts), 2 * nb};
    ra.fill_spans = fs;
    const int src = dtype == HU_F32 ? SRC_F32 : SRC_I8;
    HU_HIP(timed("rows_r2c_load", st, [&] { return launch_rows_r2c(Lrow, src, ra, B, st); }));
    if (g.nd == 3) {
      ColsArgs cy{};
      cy.spec = spec;
      cy.Nh = g.Nhp;
      cy.ncol = g.n[0] * g.nxh;
      cy.inner = g.nxh;
      cy.tw = tw_1;
      cy.sc = col_sched(g.n[1], cy.ncol, B);
      HU_HIP(timed("cols_y_fwd", st, [&] { return launch_cols(g.n[1], false, cy, B, st); }));
    }
    BinArgs ba{};
    ba.spec = spec;
    ba.Nh = g.Nhp;
    ba.N = g.N;
    ba.gm = axis0(g);
    ba.sc = col_sched(g.n[0], ba.gm.ncol, B);
    ba.bd = bd;
    ba.nb = nb;
    ba.table = geo.table;
    ba.tw = tw_0;
    ba.sum = s;
    HU_HIP(timed("cols_bin", st, [&] { return launch_cols_bin(g.n[0], ba, B, st); }));
  }
  return HU_OK;
}

const char* hu_strerror(int code) {
  switch (code) {
    case HU_OK: return "ok";
    case HU_ERR_ARG: return "invalid argument";
    case HU_ERR_SIZE: return "grid size outside the supported set (2^k in 4..2048, 3*2^k in 6..768 per axis)";
    case HU_ERR_ALIGN: return "misaligned pointer (arrays need 16 bytes, workspace 256 bytes)";
    case HU_ERR_WORKSPACE: return "workspace smaller than hu_workspace_size";
    case HU_ERR_DEGENERATE: return "filter has no support on the lattice (max ln chi < -80)";
    case HU_ERR_HIP: return "HIP runtime error";
    case HU_ERR_UNSUPPORTED: return "unsupported request";
    default: return "unknown error";
  }
}

int hu_debug_philox(uint64_t seed, uint64_t first, uint64_t count, uint32_t* words, float* normals, void* stream) {
  if (count == 0) return HU_OK;
  if (!words && !normals) return HU_ERR_ARG;
  if (count > (1ull << 31)) return HU_ERR_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HU_HIP(launch_debug_philox(seed, first, count, words, normals, st));
  return HU_OK;
}

int hu_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof = on != 0;
  g_recs.clear();
  g_pool_next = 0;
  if (g_prof && g_pool.size() < 1024) {
    while (g_pool.size() < 1024) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return HU_ERR_HIP;
      g_pool.push_back(e);
    }
  }
  return HU_OK;
}

int hu_profile_read(char (*names)[48], int64_t* launches, double* total_ms, int cap) {
  std::lock_guard<std::mutex> lk(g_mu);
  std::vector<std::string> fam;
  std::vector<int64_t> cnt;
  std::vector<double> ms;
  for (const ProfRec& r : g_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return HU_ERR_HIP;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return HU_ERR_HIP;
    size_t i = 0;
    while (i < fam.size() && fam[i] != r.name) ++i;
    if (i == fam.size()) {
      fam.push_back(r.name);
      cnt.push_back(0);
      ms.push_back(0.0);
    }
    cnt[i] += 1;
    ms[i] += t;
  }
  const int n = (int)fam.size();
  for (int i = 0; i < n && i < cap; ++i) {
    if (names) {
      std::strncpy(names[i], fam[i].c_str(), 47);
      names[i][47] = 0;
    }
    if (launches) launches[i] = cnt[i];
    if (total_ms) total_ms[i] = ms[i];
  }
  return n;
}

}  // extern "C"
