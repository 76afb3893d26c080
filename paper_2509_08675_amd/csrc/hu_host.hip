// Host-side implementation shared by the C-ABI entry points (see hu_host.hpp).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <tuple>
#include <utility>

#include "hu_host.hpp"

namespace hu {

namespace {

std::mutex g_mu;
std::map<std::pair<int, int>, float2*> g_tw, g_tw2, g_tw_alt;   // g_tw_alt: tables of Plan<L, 1>
std::map<std::pair<int, int>, double*> g_edges;
std::map<std::vector<long long>, BinGeo> g_bingeo;

// Host bin tables of a grid and bin layout (built once, kept for the tile tables of other widths)
struct BinHost {
  std::vector<uint16_t> table;                 // [ncol][n0]: bin of each half-spectrum mode
  std::vector<unsigned long long> counts;      // [nb]: modes per bin with multiplicity
};
struct TileHost {
  std::vector<uint16_t> ltab;                  // [ncol][n0]: position in the tile's list of distinct bins
  std::vector<uint32_t> toff, coff, cpos, wpos;   // wpos: the inverse of cpos
  int nloc_max = 0;
};
std::map<std::vector<long long>, std::shared_ptr<BinHost>> g_binhost;    // {nd, n0, n1, n2, nr, na}
std::map<std::vector<long long>, std::shared_ptr<TileHost>> g_tilehost;  // ... + C
std::map<std::vector<long long>, TileBinDev> g_tiledev;                  // device + ... + C

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

// e_j = (cos j pi / A, sin j pi / A), j = 1..A-1, in FP64; the 45, 90 and 135 degree edges exact.
// h[0 .. m) holds the x components, h[m .. 2m) the y components, m = max(A - 1, 1).
std::vector<double> host_edges(int na) {
  const int m = na > 1 ? na - 1 : 1;
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
  return h;
}

int get_edges(int na, const double** ex, const double** ey) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int m = na > 1 ? na - 1 : 1;
  auto key = std::make_pair(current_device(), na);
  auto it = g_edges.find(key);
  if (it == g_edges.end()) {
    const std::vector<double> h = host_edges(na);
    double* d = nullptr;
    if (hipMalloc(&d, sizeof(double) * 2 * m) != hipSuccess) return HU_ERR_HIP;
    if (hipMemcpy(d, h.data(), sizeof(double) * 2 * m, hipMemcpyHostToDevice) != hipSuccess) return HU_ERR_HIP;
    it = g_edges.emplace(key, d).first;
  }
  *ex = it->second;
  *ey = it->second + m;
  return HU_OK;
}

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

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

long long lcm_ll(long long a, long long b) { return a / std::gcd(a, b) * b; }

// ---- tuned plans
std::map<std::string, TunePlan> g_plans;
bool g_plans_loaded = false;

void load_plans_locked() {
  if (g_plans_loaded) return;
  g_plans_loaded = true;
  const char* path = std::getenv("HUFIELD_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  std::fclose(f);
  // entries look like  "key": [v0, v1, ...]  (missing trailing entries are 0)
  size_t pos = 0;
  while ((pos = s.find("\": [", pos)) != std::string::npos) {
    const size_t q = s.rfind('"', pos - 1);
    if (q == std::string::npos) break;
    const std::string key = s.substr(q + 1, pos - q - 1);
    TunePlan p{};
    const char* c = s.c_str() + pos + 4;
    int n = 0;
    while (n < NPASS) {
      char* end = nullptr;
      const long x = std::strtol(c, &end, 10);
      if (end == c) break;
      p.v[n++] = x ? 1 : 0;
      c = end;
      while (*c == ' ' || *c == ',') ++c;
      if (*c == ']') break;
    }
    if (n >= 5) g_plans[key] = p;
    pos += 4;
  }
}

// ---- profiling
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
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

}  // namespace

bool g_prof = false;

hipError_t timed_impl(const char* name, hipStream_t st, hipError_t (*fn)(void*), void* ctx) {
  hipEvent_t a = pool_event(), b = pool_event();
  if (!a || !b) return fn(ctx);
  (void)hipEventRecord(a, st);
  hipError_t e = fn(ctx);
  (void)hipEventRecord(b, st);
  g_recs.push_back({name, a, b});
  return e;
}

int profile_reset(bool on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof = on;
  g_recs.clear();
  g_pool_next = 0;
  while (on && g_pool.size() < 2048) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return HU_ERR_HIP;
    g_pool.push_back(e);
  }
  return HU_OK;
}

int profile_collect(std::vector<std::string>& names, std::vector<long long>& launches, std::vector<double>& ms) {
  names.clear();
  launches.clear();
  ms.clear();
  for (const ProfRec& r : g_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return HU_ERR_HIP;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return HU_ERR_HIP;
    size_t i = 0;
    while (i < names.size() && names[i] != r.name) ++i;
    if (i == names.size()) {
      names.push_back(r.name);
      launches.push_back(0);
      ms.push_back(0.0);
    }
    launches[i] += 1;
    ms[i] += t;
  }
  return HU_OK;
}

// ---------------------------------------------------------------------------------------------
// Stage twiddle table of a length L (layout in hu_device.hpp, StageTab): for the forward radix
// list and then its reverse, the rows of every stage i >= 1, entry (k, r) = exp(-2 pi i t / L)
// with t = r k L / (NS_i R_i), FP64 rounded once to FP32.
template <int... Rs>
static std::vector<int> radix_vec(Radices<Rs...>) { return {Rs...}; }

static void append_stage_rows(int L, const std::vector<int>& rad, std::vector<float2>& h) {
  int ns = 1;
  for (size_t i = 0; i < rad.size(); ++i) {
    const int R = rad[i];
    if (ns > 1) {
      for (int k = 0; k < ns; ++k)
        for (int r = 0; r < rpad(R); ++r) {
          const long long t = (long long)r * k * (L / (ns * R));
          const double a = 2.0 * M_PI * (double)t / (double)L;
          h.push_back(make_float2((float)std::cos(a), (float)-std::sin(a)));
        }
    }
    ns *= R;
  }
}

template <int L, int RV>
static int make_stage_table_L(float2** out) {
  using F = typename Plan<L, RV>::fwd;
  std::vector<float2> h;
  append_stage_rows(L, radix_vec(F{}), h);
  if ((int)h.size() != StageTab<L, RV>::fwd) return HU_ERR_HIP;
  append_stage_rows(L, radix_vec(Reverse<F>{}), h);
  if ((int)h.size() != StageTab<L, RV>::total) return HU_ERR_HIP;
  h.push_back(make_float2(0.f, 0.f));           // never empty (lengths with one stage)
  float2* d = nullptr;
  if (hipMalloc(&d, sizeof(float2) * h.size()) != hipSuccess) return HU_ERR_HIP;
  if (hipMemcpy(d, h.data(), sizeof(float2) * h.size(), hipMemcpyHostToDevice) != hipSuccess) return HU_ERR_HIP;
  *out = d;
  return HU_OK;
}

#define HU_TW_LENGTHS(X) \
  X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) \
  X(1024) X(1536) X(2048)

static int make_stage_table(int L, int rv, float2** out) {
  switch (L) {
#define X(LL) case LL: return rv ? make_stage_table_L<LL, 1>(out) : make_stage_table_L<LL, 0>(out);
    HU_TW_LENGTHS(X)
#undef X
    default: return HU_ERR_SIZE;
  }
}

bool plane_ok(const Geom& g) {
  if (g.nd != 3) return false;
  const size_t lds = plane_lds_bytes(g.nx / 2, g.n[1]);
  return lds > 0 && lds + 1024 <= LDS_BYTES;
}

bool whole_field_ok(const Geom& g, int nb) {
  if (g.nd != 2) return false;
  const size_t lds = small_lds_bytes(g.nx / 2, g.n[0], nb);
  return lds > 0 && lds + 1024 <= LDS_BYTES;
}

bool plan_has_alt(int L) {
  switch (L) {
#define X(LL) case LL: return Plan<LL, 1>::alt;
    HU_TW_LENGTHS(X)
#undef X
    default: return false;
  }
}

int get_tw(int L, const float2** tw, int radix) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int rv = radix && plan_has_alt(L) ? 1 : 0;
  auto& tab = rv ? g_tw_alt : g_tw;
  auto key = std::make_pair(current_device(), L);
  auto it = tab.find(key);
  if (it == tab.end()) {
    float2* d;
    int rc = make_stage_table(L, rv, &d);
    if (rc) return rc;
    it = tab.emplace(key, d).first;
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

int make_geom(const hu_dims& d, Geom* g) {
  if (d.ndim != 2 && d.ndim != 3) return HU_ERR_ARG;
  g->nd = d.ndim;
  g->N = 1;
  g->D = 1;
  g->n[2] = 0;
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
  if (g->Nhp * 8 >= (1LL << 32)) return HU_ERR_SIZE; // byte offsets within one field's half spectrum
  return HU_OK;
}

int check_filter(const hu_filter* f, int nd) {
  if (!f) return HU_ERR_ARG;
  if (!finite_pos(f->p) || !finite_pos(f->semi[0]) || !finite_pos(f->semi[1])) return HU_ERR_ARG;
  if (nd == 3 && !finite_pos(f->semi[2])) return HU_ERR_ARG;
  if (f->prof_n != 0) {          // tabulated radial form: alpha, k0 and width unused
    if (f->prof_n < 2 || !f->prof || !finite_pos(f->prof_dk) || !finite_pos(f->sigma_f)) return HU_ERR_ARG;
    if (!aligned(f->prof, 4)) return HU_ERR_ALIGN;
    if (!std::isfinite(f->rot) || !std::isfinite(f->offset) || f->offset < 0.0) return HU_ERR_ARG;
    if (f->offset > 0.0) return HU_ERR_UNSUPPORTED;
    return HU_OK;
  }
  if (!std::isfinite(f->alpha) || !(f->alpha > -(double)nd) || !finite_pos(f->width) || !finite_pos(f->sigma_f))
    return HU_ERR_ARG;
  if (!std::isfinite(f->offset) || f->offset < 0.0) return HU_ERR_ARG;
  if (f->offset > 0.0 && f->alpha < 0.0) return HU_ERR_UNSUPPORTED;   // the offset is relative to a continuum peak
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

int tile_partials(const Geom& g, const hu_bins& bins, int C, int* M, int* nloc_max);

int layout(const Geom& g, int batch, bool need_stats, const TunePlan& plan, const hu_bins* bins, Layout* out) {
  Layout L{};
  size_t off = 0;
  L.spec = off;
  off += up256((size_t)batch * g.Nhp * sizeof(float2));
  (void)plan;
  L.tiles = 0;                                    // filter-pass tiles of either tile width
  for (int v = 0; v < NVARIANT; ++v) L.tiles = std::max(L.tiles, col_tiles(g.n[0], v, g.Nh / g.n[0]));
  if (need_stats) {
    L.partials = off;
    off += up256((size_t)batch * L.tiles * 4 * sizeof(double));
    L.fstats = off;
    off += up256((size_t)batch * 8 * sizeof(double));
    // per-tile counts of the last row pass, for either row-tile width
    // (or per plane, for the plane kernels of 3D grids)
    const int rt0 = row_tiles(g.nx / 2, 0, g.nrows), rt1 = row_tiles(g.nx / 2, 1, g.nrows);
    const int rtm = std::max(std::max(rt0, rt1), g.nd == 3 ? g.n[0] : 0);
    L.cpart = off;
    off += up256((size_t)batch * rtm * 2 * sizeof(uint32_t));
  }
  if (bins) {
    // room for the partials of either tile width (the plan of a later call may differ)
    int M = 0;
    for (int v = 0; v < NVARIANT; ++v) {
      int m = 0, nl = 0;
      HU_TRY(tile_partials(g, *bins, col_width(g.n[0], v), &m, &nl));
      M = m > M ? m : M;
    }
    if (need_stats) {
      L.Mc = M;
      L.parts_c = off;
      off += up256((size_t)batch * M * sizeof(double));
    }
    L.Mp = M;
    L.parts_p = off;
    off += up256((size_t)batch * M * sizeof(double));
  }
  L.queue = off;
  off += up256(NQUEUE * sizeof(unsigned));
  L.total = off;
  *out = L;
  return HU_OK;
}

// workgroups of a kernel that fit on the device at once (cached per device, kernel and LDS size)
hipError_t resident_blocks(const void* kern, int threads, size_t lds, int* slots) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, size_t>, int> cache;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const auto key = std::make_tuple(dev, kern, lds);
  std::lock_guard<std::mutex> lock(mu);
  const auto it = cache.find(key);
  if (it != cache.end()) {
    *slots = it->second;
    return hipSuccess;
  }
  int ncu = 0, per_cu = 0;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1 || ncu < 1) return hipErrorInvalidConfiguration;
  cache[key] = *slots = per_cu * ncu;
  return hipSuccess;
}

FiltDev filt_dev(const hu_filter& f, const Geom& g) {
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
  // the normalisation of Eq. (13), in FP64: ln chi at the continuum peak
  // K* = (k0 + sqrt(k0^2 + 4 alpha w^2)) / 2 for alpha >= 0 (the alpha ln K term is 0 for alpha = 0,
  // also at K* = k0 = 0); for alpha < 0 the continuum has no maximum as K -> 0, and the larger of
  // ln chi at k_low = min_i(2 / n_i) / (sqrt(d) max semi) -- a lower bound of every nonzero lattice
  // K -- and at the band's local maximum (when it exists) bounds chi on the lattice
  const double w2 = 2.0 * f.width * f.width;
  auto lnchi = [&](double K) { return (f.alpha != 0.0 ? f.alpha * std::log(K) : 0.0) - (K - f.k0) * (K - f.k0) / w2; };
  const double disc = f.k0 * f.k0 + 4.0 * f.alpha * f.width * f.width;
  const double ks = disc >= 0.0 ? 0.5 * (f.k0 + std::sqrt(disc)) : 0.0;
  double ref;
  if (f.alpha >= 0.0) {
    ref = f.alpha > 0.0 ? lnchi(ks) : 0.0;
  } else {
    int nmax = 0;
    double smax = 0.0;
    for (int i = 0; i < g.nd; ++i) {
      nmax = g.n[i] > nmax ? g.n[i] : nmax;
      smax = f.semi[i] > smax ? f.semi[i] : smax;
    }
    const double klow = (2.0 / nmax) / (std::sqrt((double)g.nd) * smax);
    ref = lnchi(klow);
    if (disc >= 0.0 && ks > 0.0) ref = std::fmax(ref, lnchi(ks));
  }
  d.lnchimax = (float)ref;
  d.offset = (float)f.offset;
  d.lnoffset = f.offset > 0.0 ? (float)std::log(f.offset) : -1.0e30f;
  d.rotated = (f.rot != 0.0) ? 1 : 0;
  // FP32 evaluation rounds each of alpha ln K, (K - k0)^2 / (2 w^2) and ln chi(K*) at 2^-24 of
  // its magnitude; near the band they are about their values at the reference K, and the field
  // error they cause grows with their sum (about 6e-8 of it, plus 5e-7; an emulation of the FP32
  // chain at 1024^2: 7e-7 at alpha = 0.5, 4e-6 at alpha = 20, 1.2e-5 at alpha = 100).  Above 32
  // (the paper's alpha = 20 .. 100) the filter is evaluated in FP64.
  const double kref = f.alpha > 0.0 ? ks : (f.alpha == 0.0 ? (f.k0 > 0.0 ? f.k0 : 0.0) : 0.0);
  const double tsum = (kref > 0.0 ? std::fabs(f.alpha * std::log(kref)) : 0.0) +
                      (kref - f.k0) * (kref - f.k0) / w2 + std::fabs(ref);
  d.prec64 = tsum > FP32_FILTER_TERMS ? 1 : 0;
  d.dcr = std::cos(f.rot);
  d.dsr = std::sin(f.rot);
  d.dia = 1.0 / f.semi[0];
  d.dib = 1.0 / f.semi[1];
  d.dic = 1.0 / f.semi[2];
  d.dp = f.p;
  d.dip = 1.0 / f.p;
  d.dalpha = f.alpha;
  d.dk0 = f.k0;
  d.dinv2w2 = 1.0 / w2;
  d.dlnchimax = ref;
  d.doffset = f.offset;
  if (f.prof_n > 0) {            // samples used as given: no continuum normalisation, no offset
    d.prof = f.prof;
    d.prof_n = f.prof_n;
    d.prof_idk = (float)(1.0 / f.prof_dk);
    d.lnchimax = 0.0f;
    d.offset = 0.0f;
    d.lnoffset = -1.0e30f;
    d.prec64 = 0;
  }
  return d;
}

bool filt_general(const hu_filter& f, const Geom& g) { return f.prof_n > 0 || filt_dev(f, g).prec64 != 0; }

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

// ---------------------------------------------------------------------------------------------
// Bin tables, built on the host.  The bin of a half-spectrum mode (exact integer radial rule and
// FP64 angular edge tests with separately rounded products; the library is compiled without
// multiply-add contraction): with D = lcm of the dims, q_i = m~_i D / n_i (q_x = m_x on the
// halved axis), r = the largest integer with r^2 D^2 <= 4 R^2 sum q_i^2; r >= R goes to the corner
// slot R A; in 2D the angular bin counts the edges e_j with e_jx q_y - e_jy q_x >= 0 after folding
// q to q_y >= 0 (q_y = 0 with q_x >= 0 on the half spectrum), the DC mode in bin 0.
// ---------------------------------------------------------------------------------------------
namespace {

int host_bin(long long s, long long qx, long long qy, long long D2, long long fourR2, int nr, int na,
             const std::vector<double>& ed) {
  const long long rhs = fourR2 * s;
  long long r = (long long)std::sqrt((double)rhs / (double)D2);
  while (r > 0 && r * r * D2 > rhs) --r;
  while ((r + 1) * (r + 1) * D2 <= rhs) ++r;
  if (r >= nr) return nr * na;
  int a = 0;
  if (na > 1 && s != 0) {
    if (qy < 0) { qy = -qy; qx = -qx; }
    const double dx = (double)qx, dy = (double)qy;
    const int m = na - 1;
    for (int j = 0; j < m; ++j) {
      const double t1 = ed[j] * dy;
      const double t2 = ed[m + j] * dx;
      if (t1 - t2 >= 0.0) ++a;
    }
  }
  return (int)r * na + a;
}

long long signed_index(long long m, long long n) { return m < n / 2 ? m : m - n; }

std::shared_ptr<BinHost> bin_host(const Geom& g, const hu_bins& bins) {
  const std::vector<long long> key = {g.nd, g.n[0], g.n[1], g.n[2], bins.n_radial, bins.n_angular};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_binhost.find(key);
    if (it != g_binhost.end()) return it->second;
  }
  const Axis0Geom a = axis0(g);
  const int nr = bins.n_radial, na = bins.n_angular, nb = nr * na + 1;
  const std::vector<double> ed = host_edges(na);
  const long long D2 = g.D * g.D, fourR2 = 4LL * nr * nr;
  auto h = std::make_shared<BinHost>();
  h->table.resize((size_t)a.ncol * a.n0);
  h->counts.assign(nb, 0ull);
  for (int gc = 0; gc < a.ncol; ++gc) {
    const int my = g.nd == 3 ? gc / a.nxh : 0;
    const int mx = gc - my * (g.nd == 3 ? a.nxh : 0);
    const long long qx = (long long)mx * a.dfac_x;
    const long long qy = g.nd == 3 ? signed_index(my, a.ny) * a.dfac_y : 0;
    const unsigned wm = (mx == 0 || 2 * mx == a.nx) ? 1u : 2u;
    uint16_t* row = h->table.data() + (size_t)gc * a.n0;
    for (int e = 0; e < a.n0; ++e) {
      const long long q0 = signed_index(e, a.n0) * a.dfac_0;
      const long long s = qx * qx + qy * qy + q0 * q0;
      const int bin = host_bin(s, qx, g.nd == 2 ? q0 : 0, D2, fourR2, nr, na, ed);
      row[e] = (uint16_t)bin;
      h->counts[bin] += wm;
    }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  return g_binhost.emplace(key, h).first->second;
}

// Tile tables for tiles of C columns: for tile t, its distinct bins in ascending order (their
// partials occupy [toff[t], toff[t + 1])), each mode's position in that list, and per bin the
// partial positions in tile order (CSR).
std::shared_ptr<TileHost> tile_host(const Geom& g, const hu_bins& bins, int C) {
  const std::vector<long long> key = {g.nd, g.n[0], g.n[1], g.n[2], bins.n_radial, bins.n_angular, C};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tilehost.find(key);
    if (it != g_tilehost.end()) return it->second;
  }
  const std::shared_ptr<BinHost> bh = bin_host(g, bins);
  const Axis0Geom a = axis0(g);
  const int nb = bins.n_radial * bins.n_angular + 1;
  const int ntiles = (a.ncol + C - 1) / C;
  auto th = std::make_shared<TileHost>();
  th->ltab.resize((size_t)a.ncol * a.n0);
  th->toff.assign(ntiles + 1, 0u);
  std::vector<int> mark(nb, -1), jpos(nb, 0);
  std::vector<int> lst, pbin;
  for (int t = 0; t < ntiles; ++t) {
    const int g0 = t * C, g1 = g0 + C < a.ncol ? g0 + C : a.ncol;
    lst.clear();
    for (size_t i = (size_t)g0 * a.n0; i < (size_t)g1 * a.n0; ++i) {
      const int b = bh->table[i];
      if (mark[b] != t) {
        mark[b] = t;
        lst.push_back(b);
      }
    }
    std::sort(lst.begin(), lst.end());
    for (size_t j = 0; j < lst.size(); ++j) {
      jpos[lst[j]] = (int)j;
      pbin.push_back(lst[j]);
    }
    for (size_t i = (size_t)g0 * a.n0; i < (size_t)g1 * a.n0; ++i) th->ltab[i] = (uint16_t)jpos[bh->table[i]];
    th->toff[t + 1] = th->toff[t] + (uint32_t)lst.size();
    th->nloc_max = std::max(th->nloc_max, (int)lst.size());
  }
  th->coff.assign(nb + 1, 0u);
  for (int b : pbin) th->coff[b + 1]++;
  for (int b = 0; b < nb; ++b) th->coff[b + 1] += th->coff[b];
  th->cpos.resize(pbin.size());
  std::vector<uint32_t> cur(th->coff.begin(), th->coff.end() - 1);
  for (size_t i = 0; i < pbin.size(); ++i) th->cpos[cur[pbin[i]]++] = (uint32_t)i;
  th->wpos.resize(pbin.size());
  for (size_t k = 0; k < pbin.size(); ++k) th->wpos[th->cpos[k]] = (uint32_t)k;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_tilehost.emplace(key, th).first->second;
}

template <class T>
int upload(const std::vector<T>& h, T** d) {
  const size_t n = h.empty() ? 1 : h.size();
  if (hipMalloc(d, sizeof(T) * n) != hipSuccess) return HU_ERR_HIP;
  if (!h.empty() && hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice) != hipSuccess)
    return HU_ERR_HIP;
  return HU_OK;
}

}  // namespace

int tile_partials(const Geom& g, const hu_bins& bins, int C, int* M, int* nloc_max) {
  if (C < 1) return HU_ERR_SIZE;
  const std::shared_ptr<TileHost> th = tile_host(g, bins, C);
  *M = (int)th->toff.back();
  *nloc_max = th->nloc_max;
  return HU_OK;
}

int get_bingeo(const Geom& g, const hu_bins& bins, BinGeo* out) {
  const std::vector<long long> key = {current_device(), g.nd, g.n[0], g.n[1], g.n[2], bins.n_radial, bins.n_angular};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_bingeo.find(key);
    if (it != g_bingeo.end()) {
      *out = it->second;
      return HU_OK;
    }
  }
  const std::shared_ptr<BinHost> bh = bin_host(g, bins);
  BinGeo geo{nullptr, nullptr};
  HU_TRY(upload(bh->table, &geo.table));
  HU_TRY(upload(bh->counts, &geo.counts));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_bingeo.find(key);
  if (it != g_bingeo.end()) {                // another thread built it meanwhile
    (void)hipFree(geo.counts);
    (void)hipFree(geo.table);
    *out = it->second;
    return HU_OK;
  }
  g_bingeo.emplace(key, geo);
  *out = geo;
  return HU_OK;
}

int get_tilebins(const Geom& g, const hu_bins& bins, int C, TileBinDev* out) {
  const std::vector<long long> key = {current_device(), g.nd, g.n[0], g.n[1], g.n[2], bins.n_radial, bins.n_angular, C};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tiledev.find(key);
    if (it != g_tiledev.end()) {
      *out = it->second;
      return HU_OK;
    }
  }
  if (C < 1) return HU_ERR_SIZE;
  const std::shared_ptr<TileHost> th = tile_host(g, bins, C);
  uint16_t* ltab = nullptr;
  uint32_t *toff = nullptr, *coff = nullptr, *wpos = nullptr;
  HU_TRY(upload(th->ltab, &ltab));
  HU_TRY(upload(th->toff, &toff));
  HU_TRY(upload(th->wpos, &wpos));
  HU_TRY(upload(th->coff, &coff));
  TileBinDev d{ltab, toff, wpos, coff, th->nloc_max, (int)th->toff.back(), bins.n_angular == 1 ? 1 : 0};
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tiledev.find(key);
  if (it != g_tiledev.end()) {
    (void)hipFree(ltab);
    (void)hipFree(toff);
    (void)hipFree(coff);
    (void)hipFree(wpos);
    *out = it->second;
    return HU_OK;
  }
  g_tiledev.emplace(key, d);
  *out = d;
  return HU_OK;
}

int tables_ready(const Geom& g, const hu_bins* bins) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int dev = current_device();
  if (!g_tw.count({dev, g.nx / 2}) || !g_tw2.count({dev, g.nx / 2}) || !g_tw.count({dev, g.n[0]}))
    return HU_ERR_TABLES;
  if (g.nd == 3 && !g_tw.count({dev, g.n[1]})) return HU_ERR_TABLES;
  if (plan_has_alt(g.n[0]) && !g_tw_alt.count({dev, g.n[0]})) return HU_ERR_TABLES;
  if (g.nd == 3 && plan_has_alt(g.n[1]) && !g_tw_alt.count({dev, g.n[1]})) return HU_ERR_TABLES;
  if (bins) {
    if (!g_edges.count({dev, bins->n_angular})) return HU_ERR_TABLES;
    const std::vector<long long> key = {dev, g.nd, g.n[0], g.n[1], g.n[2], bins->n_radial, bins->n_angular};
    if (!g_bingeo.count(key)) return HU_ERR_TABLES;
    for (int v = 0; v < NVARIANT; ++v) {
      std::vector<long long> kt = key;
      kt.push_back(col_width(g.n[0], v));
      if (!g_tiledev.count(kt)) return HU_ERR_TABLES;
    }
  }
  return HU_OK;
}

// every table a class needs, created before any launch (and before a graph capture); the tile
// tables for both tile widths, the stage tables for both radix choices
int prepare_tables(const Geom& g, const hu_bins* bins, hipStream_t st) {
  (void)st;
  const float2 *a, *b;
  HU_TRY(get_tw(g.nx / 2, &a));
  HU_TRY(get_tw2(g.nx / 2, &b));
  for (int rv = 0; rv < 2; ++rv) {
    HU_TRY(get_tw(g.n[0], &a, rv));
    if (g.nd == 3) HU_TRY(get_tw(g.n[1], &a, rv));
  }
  if (bins) {
    BinDev bd{};
    BinGeo geo;
    TileBinDev tb;
    HU_TRY(make_bindev(g, *bins, &bd));
    HU_TRY(get_bingeo(g, *bins, &geo));
    for (int v = 0; v < NVARIANT; ++v) HU_TRY(get_tilebins(g, *bins, col_width(g.n[0], v), &tb));
  }
  return HU_OK;
}

// ---------------------------------------------------------------------------------------------
std::string plan_key(const Geom& g, const hu_bins* bins, int batch) {
  const int bucket = batch < 2 ? 1 : batch < 8 ? 2 : batch < 32 ? 8 : 32;
  char buf[160];
  std::snprintf(buf, sizeof buf, "gfx950|%dx%dx%d|nb%d|b%d", g.n[0], g.n[1], g.nd == 3 ? g.n[2] : 1,
                bins ? bins->n_radial * bins->n_angular + 1 : 0, bucket);
  return buf;
}

TunePlan get_plan(const Geom& g, const hu_bins* bins, int batch) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_plans_locked();
  auto it = g_plans.find(plan_key(g, bins, batch));
  if (it != g_plans.end()) return it->second;
  return TunePlan{};
}

void set_plan(const std::string& key, const TunePlan& p) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_plans_locked();
  g_plans[key] = p;
}

int save_plans(const char* path) {
  std::lock_guard<std::mutex> lk(g_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return HU_ERR_ARG;
  std::fprintf(f, "{\n  \"format\": \"hufield plans: tile widths [rows_r2c, cols_y, cols_filter, rows_c2r, cols_bin], "
                  "schedules [bin_schedule, field_placement, y_group]\",\n  \"plans\": {\n");
  size_t i = 0;
  for (const auto& kv : g_plans) {
    const TunePlan& p = kv.second;
    std::fprintf(f, "    \"%s\": [", kv.first.c_str());
    for (int k = 0; k < NPASS; ++k) std::fprintf(f, "%d%s", p.v[k], k + 1 < NPASS ? ", " : "");
    std::fprintf(f, "]%s\n", ++i < g_plans.size() ? "," : "");
  }
  std::fprintf(f, "  }\n}\n");
  std::fclose(f);
  return HU_OK;
}

// ---------------------------------------------------------------------------------------------
int enqueue_class(const ClassRun& r, hipStream_t st) {
  const Geom& g = r.g;
  const int B = r.B;
  const bool batch_mode = r.io != nullptr;
  const hu_outputs& o = r.out;
  const int Lrow = g.nx / 2;
  const float2 *tw_row, *tw2_row, *tw_0, *tw_1 = nullptr;
  HU_TRY(get_tw(Lrow, &tw_row));
  HU_TRY(get_tw2(Lrow, &tw2_row));
  const int rad = r.plan.v[P_RADIX];        // the column passes' radix lists (tables to match)
  HU_TRY(get_tw(g.n[0], &tw_0, rad));
  if (g.nd == 3) HU_TRY(get_tw(g.n[1], &tw_1, rad));
  const int nb = r.bins ? r.bins->n_radial * r.bins->n_angular + 1 : 0;
  BinGeo geo{nullptr, nullptr};
  TileBinDev tb_c{}, tb_p{};
  if (r.bins) {
    HU_TRY(get_bingeo(g, *r.bins, &geo));
    HU_TRY(get_tilebins(g, *r.bins, col_width(g.n[0], r.plan.v[P_FILTER]), &tb_c));
    HU_TRY(get_tilebins(g, *r.bins, col_width(g.n[0], r.plan.v[P_BIN]), &tb_p));
    if (tb_c.M > r.lay.Mc || tb_p.M > r.lay.Mp) return HU_ERR_WORKSPACE;
  }
  const bool want_cont = batch_mode ? (r.want_cont && r.bins) : (o.cont_sum != nullptr);
  const bool want_pm1 = r.thresh && (batch_mode ? (r.want_pm1_spec && r.bins) : (o.pm1_sum != nullptr));

  // small 2D grids under plan entry whole_field: the whole path in one workgroup per field, the
  // half spectrum resident in LDS (the workspace is not touched)
  if (r.plan.v[P_WHOLE] && whole_field_ok(g, nb)) {
    if (!batch_mode && B > MAX_WHOLE_CHUNK) return HU_ERR_ARG;
    const float2* tw_c;
    HU_TRY(get_tw(g.n[0], &tw_c, 0));
    SmallArgs sa{};
    sa.io = r.io;
    if (!batch_mode) {
      for (int i = 0; i < B; ++i) sa.seeds[i] = r.seeds[i];
      sa.filt = filt_dev(r.filt, g);
      sa.sigma_f = r.filt.sigma_f;
      sa.near_abs = r.near_abs;
      sa.field = o.field;
      sa.pm1 = r.thresh ? o.pm1 : nullptr;
      sa.stats = o.stats;
      sa.counts = r.thresh ? o.counts : nullptr;
      sa.cont_sum = o.cont_sum;
      sa.cont_cnt = o.cont_cnt;
      sa.pm1_sum = o.pm1_sum;
      sa.pm1_cnt = o.pm1_cnt;
    }
    sa.thresh = r.thresh ? 1 : 0;
    sa.want_cont = want_cont ? 1 : 0;
    sa.want_pm1 = want_pm1 ? 1 : 0;
    sa.any_gen = (batch_mode ? r.any_gen : filt_general(r.filt, g)) ? 1 : 0;
    sa.nb = nb;
    sa.N = g.N;
    sa.gm = axis0(g);
    sa.table = geo.table;
    sa.counts_tab = geo.counts;
    sa.tw_row = tw_row;
    sa.tw2 = tw2_row;
    sa.tw_col = tw_c;
    HU_HIP(timed("field_lds", st, [&] { return launch_field_lds(Lrow, g.n[0], sa, B, st); }));
    return HU_OK;
  }

  if (!batch_mode && B > MAX_CHUNK) return HU_ERR_ARG;
  // 3D grids under plan entry plane: the x and y transforms of a plane in one kernel
  const bool planes = g.nd == 3 && r.plan.v[P_PLANE] && plane_ok(g);
  const float2* tw_y0 = nullptr;
  if (planes) HU_TRY(get_tw(g.n[1], &tw_y0, 0));
  float2* spec = reinterpret_cast<float2*>(r.work + r.lay.spec);
  double* partials = reinterpret_cast<double*>(r.work + r.lay.partials);
  double* fstats = reinterpret_cast<double*>(r.work + r.lay.fstats);
  double* parts_c = reinterpret_cast<double*>(r.work + r.lay.parts_c);
  double* parts_p = reinterpret_cast<double*>(r.work + r.lay.parts_p);
  unsigned* queue = reinterpret_cast<unsigned*>(r.work + r.lay.queue);
  const uint32_t* cnt_src = reinterpret_cast<const uint32_t*>(geo.counts);

  // pass A: noise -> R2C rows; block 0 of each field sets up that field's bin counts, block (0, 0)
  // clears the work counters of the persistent passes
  RowsArgs ra{};
  ra.spec = spec;
  ra.Nh = g.Nhp;
  ra.tiled = g.tiled;
  ra.N = g.N;
  ra.nrows = g.nrows;
  ra.tw = tw_row;
  ra.tw2 = tw2_row;
  ra.io = r.io;
  ra.nb = nb;
  ra.cnt_src = cnt_src;
  ra.zero = queue;
  ra.nzero = NQUEUE;
  if (!batch_mode) {
    for (int i = 0; i < B; ++i) ra.seeds[i] = r.seeds[i];
    int fs = 0;
    if (o.cont_cnt) ra.fill[fs++] = FillSpan{reinterpret_cast<uint32_t*>(o.cont_cnt), cnt_src, 2 * nb};
    if (o.pm1_cnt && r.thresh) ra.fill[fs++] = FillSpan{reinterpret_cast<uint32_t*>(o.pm1_cnt), cnt_src, 2 * nb};
    ra.fill_spans = fs;
  }
  if (planes) {
    ra.tw_y = tw_y0;
    HU_HIP(timed("plane_fwd", st, [&] { return launch_plane_fwd(Lrow, g.n[1], ra, g.n[0], B, st); }));
  } else {
    HU_HIP(timed("rows_r2c_noise", st, [&] { return launch_rows_r2c(Lrow, SRC_NOISE, r.plan.v[P_R2C], ra, B, st); }));
  }

  ColsArgs cy{};
  if (g.nd == 3) {
    cy.spec = spec;
    cy.Nh = g.Nhp;
    cy.ncol = g.n[0] * g.nxh;
    cy.inner = g.nxh;
    cy.tw = tw_1;
    cy.sc = col_sched(g.n[1], r.plan.v[P_COLY], cy.ncol, B, r.plan.v[P_YGROUP] ? 4 : Y_PASS_GROUP);
    if (!planes)
      HU_HIP(timed("cols_y_fwd", st, [&] { return launch_cols(g.n[1], false, r.plan.v[P_COLY], cy, st, rad); }));
  }
  // the fields of a tile on consecutive ids of one XCD (2D default) or field-major (3D default)
  const bool fields_xcd = (g.nd == 2) != (r.plan.v[P_FIELDS] != 0);

  FilterArgs fa{};
  fa.spec = spec;
  fa.Nh = g.Nhp;
  fa.N = g.N;
  fa.gm = axis0(g);
  // 2D: the fields of a tile share its slice of the bin table in one XCD's L2 (the 2D binning
  // pass 111 -> 103 us at 16 x 2048^2); 3D fields, 67 MB apart at 256^3, ran 3 % slower that way
  fa.sc = fields_xcd ? col_sched_fields(g.n[0], r.plan.v[P_FILTER], fa.gm.ncol, B)
                     : col_sched(g.n[0], r.plan.v[P_FILTER], fa.gm.ncol, B);
  if (!batch_mode) fa.filt = filt_dev(r.filt, g);
  fa.io = r.io;
  fa.tb = tb_c;
  fa.parts = want_cont ? parts_c : nullptr;
  fa.tw = tw_0;
  fa.partials = partials;
  fa.any_gen = (batch_mode ? r.any_gen : filt_general(r.filt, g)) ? 1 : 0;
  if (fa.sc.ntiles > r.lay.tiles) return HU_ERR_WORKSPACE;
  HU_HIP(timed("cols_filter", st, [&] { return launch_cols_filter(g.n[0], r.plan.v[P_FILTER], fa, st, rad, r.plan.v[P_FSPLIT]); }));
  FinalizeArgs fz{};
  fz.partials = partials;
  fz.ntiles = fa.sc.ntiles;
  fz.N = g.N;
  fz.sigma_f = batch_mode ? 1.0 : r.filt.sigma_f;
  fz.fstats = fstats;
  fz.stats = batch_mode ? nullptr : o.stats;
  fz.io = r.io;
  HU_HIP(timed("finalize", st, [&] { return launch_finalize(fz, B, st); }));

  if (g.nd == 3 && !planes)
    HU_HIP(timed("cols_y_inv", st, [&] { return launch_cols(g.n[1], true, r.plan.v[P_COLY], cy, st, rad); }));

  RowsZArgs za{};
  za.spec = spec;
  za.Nh = g.Nhp;
  za.tiled = g.tiled;
  za.N = g.N;
  za.nrows = g.nrows;
  za.tw = tw_row;
  za.tw2 = tw2_row;
  za.fstats = fstats;
  za.io = r.io;
  if (!batch_mode) {
    za.field = o.field;
    za.pm1 = o.pm1;
    za.near_tol = r.near_abs;
  }
  const bool want_counts = r.thresh && (batch_mode || o.counts != nullptr);
  uint32_t* cpart = reinterpret_cast<uint32_t*>(r.work + r.lay.cpart);
  za.cpart = want_counts ? cpart : nullptr;
  if (planes) {
    za.tw_y = tw_y0;
    za.pm1_spec = want_pm1 ? 1 : 0;
    HU_HIP(timed(r.thresh ? "plane_inv_thresh" : "plane_inv", st,
                 [&] { return launch_plane_inv(Lrow, g.n[1], za, r.thresh, g.n[0], B, st); }));
  } else {
    HU_HIP(timed(r.thresh ? "rows_c2r_thresh" : "rows_c2r", st,
                 [&] { return launch_rows_c2r(Lrow, r.thresh, r.plan.v[P_C2R], za, B, st); }));
  }

  if (want_pm1) {
    if (g.nd == 3 && !planes)
      HU_HIP(timed("cols_y_fwd", st, [&] { return launch_cols(g.n[1], false, r.plan.v[P_COLY], cy, st, rad); }));
    BinArgs ba{};
    ba.ntiles = col_tiles(g.n[0], r.plan.v[P_BIN], g.Nh / g.n[0]);
    ba.batch = B;
    ba.persistent = (g.nd == 3) != (r.plan.v[P_BINSCHED] != 0);
    ba.q = ItemQueue{queue + Q_BIN, ba.ntiles * B, 8};
    ba.sc = fields_xcd ? col_sched_fields(g.n[0], r.plan.v[P_BIN], g.Nh / g.n[0], B)
                       : col_sched(g.n[0], r.plan.v[P_BIN], g.Nh / g.n[0], B);
    ba.spec = spec;
    ba.Nh = g.Nhp;
    ba.gm = axis0(g);
    ba.tb = tb_p;
    ba.parts = parts_p;
    ba.tw = tw_0;
    HU_HIP(timed("cols_bin", st, [&] { return launch_cols_bin(g.n[0], r.plan.v[P_BIN], ba, st, rad, (g.nd == 2) != (r.plan.v[P_BSPLIT] != 0)); }));
  }
  if (want_cont || want_pm1 || want_counts) {
    SpecFinalArgs sf{};
    sf.nb = nb;
    if (want_cont) {
      sf.coff_c = tb_c.coff;
      sf.parts_c = parts_c;
      sf.M_c = tb_c.M;
      sf.fstats = fstats;
      sf.cont_sum = batch_mode ? nullptr : o.cont_sum;
    }
    if (want_pm1) {
      sf.coff_p = tb_p.coff;
      sf.parts_p = parts_p;
      sf.M_p = tb_p.M;
      sf.pscale = 1.0 / (double)g.N;
      sf.pm1_sum = batch_mode ? nullptr : o.pm1_sum;
    }
    if (want_counts) {
      sf.cpart = cpart;
      sf.ntc = planes ? g.n[0] : row_tiles(Lrow, r.plan.v[P_C2R], g.nrows);
      sf.counts = batch_mode ? nullptr : o.counts;
    }
    sf.io = r.io;
    HU_HIP(timed("spec_final", st, [&] { return launch_spec_final(sf, B, st); }));
  }
  return HU_OK;
}

}  // namespace hu

extern "C" int hu_debug_bin_tables(hu_dims dims, hu_bins bins, int32_t variant, int32_t* sizes, uint16_t* table,
                                   uint16_t* ltab, uint32_t* toff, uint32_t* coff, uint32_t* cpos) {
  using namespace hu;
  Geom g;
  HU_TRY(make_geom(dims, &g));
  HU_TRY(check_bins(&bins, g.nd));
  if (variant != 0 && variant != 1) return HU_ERR_ARG;
  const int C = col_width(g.n[0], variant);
  if (C < 1) return HU_ERR_SIZE;
  const std::shared_ptr<BinHost> bh = bin_host(g, bins);
  const std::shared_ptr<TileHost> th = tile_host(g, bins, C);
  const Axis0Geom a = axis0(g);
  if (sizes) {
    sizes[0] = a.ncol;
    sizes[1] = a.n0;
    sizes[2] = (int32_t)th->toff.size() - 1;
    sizes[3] = (int32_t)th->toff.back();
    sizes[4] = th->nloc_max;
    sizes[5] = C;
  }
  if (table) std::memcpy(table, bh->table.data(), bh->table.size() * sizeof(uint16_t));
  if (ltab) std::memcpy(ltab, th->ltab.data(), th->ltab.size() * sizeof(uint16_t));
  if (toff) std::memcpy(toff, th->toff.data(), th->toff.size() * sizeof(uint32_t));
  if (coff) std::memcpy(coff, th->coff.data(), th->coff.size() * sizeof(uint32_t));
  if (cpos) std::memcpy(cpos, th->cpos.data(), th->cpos.size() * sizeof(uint32_t));
  return HU_OK;
}
