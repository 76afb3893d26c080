// Host-side pieces shared by the C-ABI entry points: geometry and validation, per-size tables,
// workspace layouts, tuned plans, kernel timing, and the pass sequence of one class of
// same-shape fields.
#pragma once

#include <string>
#include <type_traits>
#include <vector>

#include "hufield.h"
#include "hu_internal.hpp"

#define HU_TRY(expr)                  \
  do {                                \
    int _rc = (expr);                 \
    if (_rc != HU_OK) return _rc;     \
  } while (0)
#define HU_HIP(expr)                               \
  do {                                             \
    if ((expr) != hipSuccess) return HU_ERR_HIP;   \
  } while (0)

namespace hu {

struct Geom {
  int nd;
  int n[3];
  int nx, nxh;
  long long N, Nh, nrows;
  long long D;      // lcm of the dims
  int tiled;        // 2D: half spectrum in column groups of 4; 3D: row-major
  long long Nhp;    // per-field half-spectrum storage (padded to whole column groups in 2D)
};

// Tunable choices of the pass sequence.  Entries 0-4: the tile width of each kernel family (0 the
// default, 1 half of it).  Entries 5-7: schedules (0 the default): P_BINSCHED the binning pass's
// (default one item per workgroup in 2D, persistent with a work counter in 3D; 1 the other one),
// P_FIELDS the axis-0 passes' placement of a tile's fields (default consecutive on one XCD in 2D,
// field-major in 3D; 1 the other one), P_YGROUP the 3D y passes' tiles per XCD group (16, or 4).
// Entry 8, P_RADIX: the radix lists of the column passes (y, filter, binning): 0 the default plan
// of each length, 1 its alternative order where the length has one (Plan<L, 1>).  Entries 9 and
// 10, P_BSPLIT and P_FSPLIT: the exchange of the binning and of the filter pass along axis 0,
// complex or split (real and imaginary parts in two rounds: half the LDS, more resident
// workgroups, two more barriers per exchange; axis-0 lengths >= 192).  Default: the binning pass
// split in 2D and complex in 3D, the filter pass complex; 1 the other one.  Entry 11, P_WHOLE:
// for 2D grids whose half spectrum fits in one workgroup's LDS (n_x and n0 up to 128), 1 runs the
// whole path as one kernel with one workgroup per field (whole_field_ok), 0 the pass sequence.
enum { P_R2C = 0, P_COLY = 1, P_FILTER = 2, P_C2R = 3, P_BIN = 4, P_BINSCHED = 5, P_FIELDS = 6, P_YGROUP = 7,
       P_RADIX = 8, P_BSPLIT = 9, P_FSPLIT = 10, P_WHOLE = 11, P_PLANE = 12, NPASS = 13 };
// Entry 12, P_PLANE: for 3D grids whose xy-plane fits in one workgroup's LDS, 1 runs the x and y
// transforms of a plane in one kernel (plane_ok): noise, R2C rows and the forward y pass in one,
// the inverse y pass, the last row pass and the y pass of the +-1 field in another.
constexpr size_t LDS_BYTES = 160 * 1024;     // per workgroup on gfx950
struct TunePlan {
  int v[NPASS];
};

// Workspace of one class: half spectra, the filter pass's per-tile statistics, per-field stats,
// the last row pass's per-tile sign counts, the tile partials of the continuous (parts_c) and the
// +-1 (parts_p) spectra, and the work counter of the persistent binning pass.
struct Layout {
  size_t spec, partials, fstats, cpart, parts_c, parts_p, queue, total;
  int tiles;
  int Mc, Mp;                    // tile partials per field of each spectrum (0: none)
};
enum { Q_BIN = 0, NQUEUE = 1 };

struct BinGeo {
  uint16_t* table;               // [ncol][n0] bin of each mode
  unsigned long long* counts;    // [nb] modes per bin with multiplicity
};

int make_geom(const hu_dims& d, Geom* g);
int check_filter(const hu_filter* f, int nd);
int check_bins(const hu_bins* b, int nd);
bool aligned(const void* p, size_t a);
size_t up256(size_t x);
// need_stats: the generator's layout (filter statistics, sign counts, both spectra); otherwise the
// binning of a stored input.  bins: null when no spectrum is binned.  Builds the host bin tables of
// the grid on first use (no device work).
int layout(const Geom& g, int batch, bool need_stats, const TunePlan& plan, const hu_bins* bins, Layout* out);
// the sum of the ln chi terms' magnitudes above which the filter is evaluated in FP64
constexpr double FP32_FILTER_TERMS = 32.0;
FiltDev filt_dev(const hu_filter& f, const Geom& g);
// the filter needs the general kernel instantiation (tabulated radial form or FP64 evaluation)
bool filt_general(const hu_filter& f, const Geom& g);
Axis0Geom axis0(const Geom& g);
int make_bindev(const Geom& g, const hu_bins& b, BinDev* bd);
// the stage table of length L under radix choice `radix` (the default list where L has no
// alternative)
int get_tw(int L, const float2** tw, int radix = 0);
bool plan_has_alt(int L);
// the grid (2D, n_x / 2 in 8 .. 64 and n0 in 16 .. 128, powers of two) and nb bins fit the
// whole-field kernel
bool whole_field_ok(const Geom& g, int nb);
// the 3D grid's plane fits the plane kernels
bool plane_ok(const Geom& g);
int get_tw2(int L, const float2** tw2);
int get_bingeo(const Geom& g, const hu_bins& bins, BinGeo* out);
// the tile-local bin tables of the axis-0 passes for tiles of C columns (device copy)
int get_tilebins(const Geom& g, const hu_bins& bins, int C, TileBinDev* out);
int prepare_tables(const Geom& g, const hu_bins* bins, hipStream_t st);
// HU_OK when every table prepare_tables would build already exists on the current device,
// else HU_ERR_TABLES (allocates nothing)
int tables_ready(const Geom& g, const hu_bins* bins);

// tuned plans: in-memory cache, loaded once from $HUFIELD_TUNE_CACHE when set
std::string plan_key(const Geom& g, const hu_bins* bins, int batch);
TunePlan get_plan(const Geom& g, const hu_bins* bins, int batch);
void set_plan(const std::string& key, const TunePlan& p);
int save_plans(const char* path);

// kernel timing (HIP events around each launch while enabled)
extern bool g_prof;
hipError_t timed_impl(const char* name, hipStream_t st, hipError_t (*fn)(void*), void* ctx);
template <class F>
hipError_t timed(const char* name, hipStream_t st, F&& f) {
  using FF = std::remove_reference_t<F>;
  if (!g_prof) return f();
  return timed_impl(name, st, [](void* c) { return (*static_cast<FF*>(c))(); }, const_cast<void*>(static_cast<const void*>(&f)));
}
int profile_reset(bool on);
int profile_collect(std::vector<std::string>& names, std::vector<long long>& launches, std::vector<double>& ms);

// One class of B same-shape fields through the whole pass sequence (3D; 2D skips the y passes):
//   rows_r2c(noise) -> cols(y, fwd) -> cols_filter(z) -> finalize -> cols(y, inv) -> rows_c2r
//   [-> cols(y, fwd) -> cols_bin(z)]   for the +-1 spectrum
// Uniform mode: one filter, seeds in `seeds`, outputs at out.* + field * stride (B <= MAX_CHUNK).
// Batch mode: `io` points at B device FieldIO entries with each field's parameters and outputs.
struct ClassRun {
  Geom g;
  int B;
  TunePlan plan;
  const hu_bins* bins;     // null: no spectra
  bool thresh;             // sign map, counts and the +-1 spectrum
  // uniform mode
  hu_filter filt;
  const uint64_t* seeds;
  float near_abs;
  hu_outputs out;
  // batch mode
  const FieldIO* io;
  bool want_cont, want_pm1_spec;
  bool any_gen;            // some job of the class uses a tabulated radial form or the FP64 filter
  // workspace of this class
  char* work;
  Layout lay;
};
int enqueue_class(const ClassRun& r, hipStream_t st);

// hu_gen_field / hu_pipeline for a uniform batch into the given workspace (thresh: sign map,
// counts and the +-1 spectrum); builds any missing per-size tables first
int run_generator(hu_dims dims, int32_t batch, const hu_filter* filt, const uint64_t* seeds, const hu_bins* bins,
                  float near_tol_rel, const hu_outputs& o, bool thresh, void* work, size_t work_bytes, void* stream);


}  // namespace hu
