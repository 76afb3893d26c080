// C-ABI entry points for uniform batches (one grid, one filter): hu_gen_field, hu_pipeline,
// hu_threshold, hu_power_spectrum, and the workspace query, error strings, the Philox dump and
// kernel timing.  Contracts are in include/hufield.h.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "hu_host.hpp"

using namespace hu;

namespace {

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

TunePlan widest_plan() { return TunePlan{{1, 1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0}}; }   // most tiles: largest partials

// workspace of hu_spectrum_grad: the noise spectrum, the per-bin weights, the per-tile partials
struct GradLayout {
  size_t spec, coef, partials, total;
  int tiles;
};
GradLayout grad_layout(const Geom& g, int nb) {
  GradLayout L{};
  L.spec = 0;
  L.coef = up256((size_t)g.Nhp * 8);
  L.partials = L.coef + up256((size_t)(nb + 1) * 8);
  L.tiles = col_tiles(g.n[0], 0, axis0(g).ncol);
  L.total = L.partials + up256((size_t)L.tiles * 8 * 8);
  return L;
}

// workspace of hu_window_variance: the half spectra of a chunk of fields, then the per-tile
// partial sums for every radius
struct WvarLayout {
  size_t spec, partials, total;
  int tiles;
};
WvarLayout wvar_layout(const Geom& g, int chunk) {
  WvarLayout L{};
  L.spec = 0;
  L.partials = up256((size_t)chunk * g.Nhp * 8);
  L.tiles = col_tiles(g.n[0], 0, axis0(g).ncol);
  L.total = L.partials + up256((size_t)chunk * L.tiles * HU_MAX_RADII * 8);
  return L;
}

// workspace of hu_filter_spectrum: the per-workgroup totals, then the per-workgroup bin rows
constexpr int FS_MAX_BLOCKS = 1024;
int fs_blocks(const Geom& g) {
  const long long chunk = 256LL * 16;
  const long long n = (g.Nh + chunk - 1) / chunk;
  return (int)(n < FS_MAX_BLOCKS ? n : FS_MAX_BLOCKS);
}
size_t fs_bytes(const Geom& g, int nb) { return up256((size_t)fs_blocks(g) * 8) + up256((size_t)fs_blocks(g) * nb * 8); }


}  // namespace

int hu::run_generator(hu_dims dims, int32_t batch, const hu_filter* filt, const uint64_t* seeds, const hu_bins* bins,
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
  const int chunk = batch < MAX_CHUNK ? batch : MAX_CHUNK;
  const TunePlan plan = get_plan(g, bins, batch);
  Layout lay;
  HU_TRY(layout(g, chunk, true, plan, bins, &lay));
  if (work_bytes < lay.total) return HU_ERR_WORKSPACE;
  const int nb = bins ? bins->n_radial * bins->n_angular + 1 : 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HU_TRY(prepare_tables(g, bins, st));
  // the whole-field kernel takes more fields per launch (it uses no workspace)
  const int step = plan.v[P_WHOLE] && whole_field_ok(g, nb) ? MAX_WHOLE_CHUNK : MAX_CHUNK;
  for (int f0 = 0; f0 < batch; f0 += step) {
    ClassRun r{};
    r.g = g;
    r.B = batch - f0 < step ? batch - f0 : step;
    r.plan = plan;
    r.bins = bins;
    r.thresh = thresh;
    r.filt = *filt;
    r.seeds = seeds + f0;
    r.near_abs = (float)(near_tol_rel * filt->sigma_f);
    r.out = offset_outputs(o, f0, g.N, nb);
    r.io = nullptr;
    r.work = reinterpret_cast<char*>(work);
    r.lay = lay;
    HU_TRY(enqueue_class(r, st));
  }
  return HU_OK;
}

extern "C" {

int hu_workspace_size(int op, hu_dims dims, int32_t batch, const hu_bins* bins, size_t* bytes) {
  if (!bytes || batch < 1) return HU_ERR_ARG;
  Geom g;
  HU_TRY(make_geom(dims, &g));
  if (bins) HU_TRY(check_bins(bins, g.nd));
  const int chunk = batch < MAX_CHUNK ? batch : MAX_CHUNK;
  Layout lay;
  switch (op) {
    case HU_OP_GEN_FIELD:
    case HU_OP_PIPELINE:
      HU_TRY(layout(g, chunk, true, widest_plan(), bins, &lay));
      *bytes = lay.total;
      return HU_OK;
    case HU_OP_POWER_SPECTRUM:
      if (!bins) return HU_ERR_ARG;
      HU_TRY(layout(g, chunk, false, widest_plan(), bins, &lay));
      *bytes = lay.total;
      return HU_OK;
    case HU_OP_LOSS:
      if (!bins) return HU_ERR_ARG;
      *bytes = grad_layout(g, bins->n_radial * bins->n_angular + 1).total;
      return HU_OK;
    case HU_OP_FILTER_SPECTRUM:
      if (!bins) return HU_ERR_ARG;
      *bytes = fs_bytes(g, bins->n_radial * bins->n_angular + 1);
      return HU_OK;
    case HU_OP_WINDOW_VARIANCE:
      *bytes = wvar_layout(g, chunk).total;
      return HU_OK;
    case HU_OP_TWO_POINT:
      HU_TRY(layout(g, chunk, true, TunePlan{}, nullptr, &lay));
      *bytes = lay.total;
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
  const TunePlan plan{{0, 0, 0, 0, 0}};
  Layout lay;
  HU_TRY(layout(g, batch < MAX_CHUNK ? batch : MAX_CHUNK, false, plan, &bins, &lay));
  if (work_bytes < lay.total) return HU_ERR_WORKSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HU_TRY(prepare_tables(g, &bins, st));
  const int Lrow = g.nx / 2;
  const int nb = bins.n_radial * bins.n_angular + 1;
  const float2 *tw_row, *tw2_row, *tw_0, *tw_1 = nullptr;
  HU_TRY(get_tw(Lrow, &tw_row));
  HU_TRY(get_tw2(Lrow, &tw2_row));
  HU_TRY(get_tw(g.n[0], &tw_0));
  if (g.nd == 3) HU_TRY(get_tw(g.n[1], &tw_1));
  BinGeo geo{nullptr, nullptr};
  HU_TRY(get_bingeo(g, bins, &geo));
  TileBinDev tb{};
  HU_TRY(get_tilebins(g, bins, col_width(g.n[0], 0), &tb));
  if (tb.M > lay.Mp) return HU_ERR_WORKSPACE;
  float2* spec = reinterpret_cast<float2*>(reinterpret_cast<char*>(work) + lay.spec);
  double* parts = reinterpret_cast<double*>(reinterpret_cast<char*>(work) + lay.parts_p);
  unsigned* queue = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(work) + lay.queue);
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
    ra.zero = queue;
    ra.nzero = NQUEUE;
    uint64_t* c = cnt ? cnt + (long long)f0 * nb : nullptr;
    int fs = 0;
    if (c) ra.fill[fs++] = FillSpan{reinterpret_cast<uint32_t*>(c), reinterpret_cast<const uint32_t*>(geo.counts), 2 * nb};
    ra.fill_spans = fs;
    const int src = dtype == HU_F32 ? SRC_F32 : SRC_I8;
    HU_HIP(timed("rows_r2c_load", st, [&] { return launch_rows_r2c(Lrow, src, 0, ra, B, st); }));
    if (g.nd == 3) {
      ColsArgs cy{};
      cy.spec = spec;
      cy.Nh = g.Nhp;
      cy.ncol = g.n[0] * g.nxh;
      cy.inner = g.nxh;
      cy.tw = tw_1;
      cy.sc = col_sched(g.n[1], 0, cy.ncol, B, Y_PASS_GROUP);
      HU_HIP(timed("cols_y_fwd", st, [&] { return launch_cols(g.n[1], false, 0, cy, st); }));
    }
    BinArgs ba{};
    ba.ntiles = col_tiles(g.n[0], 0, g.Nh / g.n[0]);
    ba.batch = B;
    ba.persistent = g.nd == 3 ? 1 : 0;
    ba.q = ItemQueue{queue + Q_BIN, ba.ntiles * B, 8};
    ba.sc = g.nd == 2 ? col_sched_fields(g.n[0], 0, g.Nh / g.n[0], B) : col_sched(g.n[0], 0, g.Nh / g.n[0], B);
    ba.spec = spec;
    ba.Nh = g.Nhp;
    ba.gm = axis0(g);
    ba.tb = tb;
    ba.parts = parts;
    ba.tw = tw_0;
    HU_HIP(timed("cols_bin", st, [&] { return launch_cols_bin(g.n[0], 0, ba, st); }));
    SpecFinalArgs sf{};
    sf.nb = nb;
    sf.coff_p = tb.coff;
    sf.parts_p = parts;
    sf.M_p = tb.M;
    sf.pscale = 1.0 / (double)g.N;
    sf.pm1_sum = sum + (long long)f0 * nb;
    HU_HIP(timed("spec_final", st, [&] { return launch_spec_final(sf, B, st); }));
  }
  return HU_OK;
}

int hu_filter_spectrum(hu_dims dims, const hu_filter* filt, hu_bins bins, double* sum, uint64_t* cnt, void* work,
                       size_t work_bytes, void* stream) {
  Geom g;
  HU_TRY(make_geom(dims, &g));
  HU_TRY(check_filter(filt, g.nd));
  HU_TRY(check_bins(&bins, g.nd));
  if (!sum) return HU_ERR_ARG;
  if (!aligned(sum, 16) || (cnt && !aligned(cnt, 16))) return HU_ERR_ALIGN;
  if (!work || !aligned(work, 256)) return work ? HU_ERR_ALIGN : HU_ERR_ARG;
  const int nb = bins.n_radial * bins.n_angular + 1;
  if (work_bytes < fs_bytes(g, nb)) return HU_ERR_WORKSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HU_TRY(prepare_tables(g, &bins, st));
  BinDev bd{};
  HU_TRY(make_bindev(g, bins, &bd));
  BinGeo geo{nullptr, nullptr};
  HU_TRY(get_bingeo(g, bins, &geo));
  FilterSpecArgs a{};
  a.gm = axis0(g);
  a.Nh = (long long)a.gm.ncol * a.gm.n0;
  a.filt = filt_dev(*filt, g);
  a.bd = bd;
  a.nb = nb;
  a.table = geo.table;
  a.sum = sum;
  a.partials = reinterpret_cast<double*>(work);
  a.nblocks = fs_blocks(g);
  a.rows = reinterpret_cast<double*>(reinterpret_cast<char*>(work) + up256((size_t)a.nblocks * 8));
  a.N = g.N;
  a.sigma_f = filt->sigma_f;
  a.counts = geo.counts;
  a.cnt = cnt;
  HU_HIP(timed("filter_spectrum", st, [&] { return launch_filter_spectrum(a, st); }));
  return HU_OK;
}

int hu_spectrum_loss(hu_bins bins, const double* sum, const uint64_t* cnt, const double* tsum, const uint64_t* tcnt,
                     double eps, double* loss, double* dL_dP, void* stream) {
  if (bins.n_radial < 1 || bins.n_angular < 1 || (long long)bins.n_radial * bins.n_angular + 1 > 8192)
    return HU_ERR_ARG;
  if (!sum || !cnt || !tsum || !tcnt || !loss || !dL_dP) return HU_ERR_ARG;
  if (!std::isfinite(eps) || eps < 0.0) return HU_ERR_ARG;
  const void* ptrs[] = {sum, cnt, tsum, tcnt, loss, dL_dP};
  for (const void* p : ptrs)
    if (!aligned(p, 8)) return HU_ERR_ALIGN;
  LossArgs a{sum, cnt, tsum, tcnt, bins.n_radial * bins.n_angular + 1, bins.n_angular, eps, loss, dL_dP};
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HU_HIP(timed("spectrum_loss", st, [&] { return launch_spectrum_loss(a, st); }));
  return HU_OK;
}

int hu_spectrum_grad(hu_dims dims, const hu_filter* filt, uint64_t seed, hu_bins bins, const double* dL_dP,
                     const double* cont_sum, const uint64_t* cont_cnt, const double* stats, double* grad, void* work,
                     size_t work_bytes, void* stream) {
  Geom g;
  HU_TRY(make_geom(dims, &g));
  HU_TRY(check_filter(filt, g.nd));
  if (filt->offset != 0.0) return HU_ERR_UNSUPPORTED;   // the adjoint differentiates sqrt(chi) only
  if (filt->prof_n != 0) return HU_ERR_UNSUPPORTED;     // ... of Eq. (13), not of a tabulated form
  HU_TRY(check_bins(&bins, g.nd));
  if (!dL_dP || !cont_sum || !cont_cnt || !stats || !grad) return HU_ERR_ARG;
  const void* ptrs[] = {dL_dP, cont_sum, cont_cnt, stats, grad};
  for (const void* p : ptrs)
    if (!aligned(p, 16)) return HU_ERR_ALIGN;
  if (!work || !aligned(work, 256)) return work ? HU_ERR_ALIGN : HU_ERR_ARG;
  const int nb = bins.n_radial * bins.n_angular + 1;
  const GradLayout lay = grad_layout(g, nb);
  if (work_bytes < lay.total) return HU_ERR_WORKSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HU_TRY(prepare_tables(g, &bins, st));
  const int Lrow = g.nx / 2;
  const float2 *tw_row, *tw2_row, *tw_0, *tw_1 = nullptr;
  HU_TRY(get_tw(Lrow, &tw_row));
  HU_TRY(get_tw2(Lrow, &tw2_row));
  HU_TRY(get_tw(g.n[0], &tw_0));
  if (g.nd == 3) HU_TRY(get_tw(g.n[1], &tw_1));
  BinDev bd{};
  HU_TRY(make_bindev(g, bins, &bd));
  BinGeo geo{nullptr, nullptr};
  HU_TRY(get_bingeo(g, bins, &geo));
  char* w = reinterpret_cast<char*>(work);
  float2* spec = reinterpret_cast<float2*>(w + lay.spec);
  double* coef = reinterpret_cast<double*>(w + lay.coef);
  double* partials = reinterpret_cast<double*>(w + lay.partials);

  // the noise spectrum W, transformed along every axis but axis 0 (as in the generator)
  RowsArgs ra{};
  ra.spec = spec;
  ra.Nh = g.Nhp;
  ra.tiled = g.tiled;
  ra.N = g.N;
  ra.nrows = g.nrows;
  ra.seeds[0] = seed;
  ra.tw = tw_row;
  ra.tw2 = tw2_row;
  ra.fill_spans = 0;
  HU_HIP(timed("rows_r2c_noise", st, [&] { return launch_rows_r2c(Lrow, SRC_NOISE, 0, ra, 1, st); }));
  if (g.nd == 3) {
    ColsArgs cy{};
    cy.spec = spec;
    cy.Nh = g.Nhp;
    cy.ncol = g.n[0] * g.nxh;
    cy.inner = g.nxh;
    cy.tw = tw_1;
    cy.sc = col_sched(g.n[1], 0, cy.ncol, 1, Y_PASS_GROUP);
    HU_HIP(timed("cols_y_fwd", st, [&] { return launch_cols(g.n[1], false, 0, cy, st); }));
  }
  GradCoefArgs ga{};
  ga.dL_dP = dL_dP;
  ga.cont_sum = cont_sum;
  ga.cont_cnt = cont_cnt;
  ga.stats = stats;
  ga.nb = nb;
  ga.N = g.N;
  ga.sigma_f = filt->sigma_f;
  ga.coef = coef;
  HU_HIP(timed("grad_coef", st, [&] { return launch_grad_coef(ga, st); }));
  AdjointArgs aa{};
  aa.gm = axis0(g);
  aa.ntiles = lay.tiles;
  aa.spec = spec;
  aa.Nh = g.Nhp;
  aa.filt = filt_dev(*filt, g);
  aa.width = (float)filt->width;
  aa.bd = bd;
  aa.nb = nb;
  aa.table = geo.table;
  aa.tw = tw_0;
  aa.coef = coef;
  aa.partials = partials;
  int rows = 0;
  HU_HIP(timed("cols_adjoint", st, [&] { return launch_cols_adjoint(g.n[0], aa, st, &rows); }));
  GradFinalArgs fa{partials, rows, grad};
  HU_HIP(timed("grad_final", st, [&] { return launch_grad_final(fa, st); }));
  return HU_OK;
}

int hu_window_variance(hu_dims dims, int32_t batch, const void* x, int32_t dtype, const double* radii,
                       int32_t n_radii, double* out, void* work, size_t work_bytes, void* stream) {
  Geom g;
  HU_TRY(make_geom(dims, &g));
  if (batch < 1 || !x || !out || !radii) return HU_ERR_ARG;
  if (dtype != HU_F32 && dtype != HU_I8) return HU_ERR_ARG;
  if (n_radii < 1 || n_radii > HU_MAX_RADII) return HU_ERR_ARG;
  for (int j = 0; j < n_radii; ++j)
    if (!std::isfinite(radii[j]) || radii[j] < 0.0 || radii[j] > 1e30) return HU_ERR_ARG;
  if (!aligned(x, 16) || !aligned(out, 16)) return HU_ERR_ALIGN;
  if (!work || !aligned(work, 256)) return work ? HU_ERR_ALIGN : HU_ERR_ARG;
  const int chunk = batch < MAX_CHUNK ? batch : MAX_CHUNK;
  const WvarLayout lay = wvar_layout(g, chunk);
  if (work_bytes < lay.total) return HU_ERR_WORKSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int Lrow = g.nx / 2;
  const float2 *tw_row, *tw2_row, *tw_0, *tw_1 = nullptr;
  HU_TRY(get_tw(Lrow, &tw_row));
  HU_TRY(get_tw2(Lrow, &tw2_row));
  HU_TRY(get_tw(g.n[0], &tw_0));
  if (g.nd == 3) HU_TRY(get_tw(g.n[1], &tw_1));
  char* w = reinterpret_cast<char*>(work);
  float2* spec = reinterpret_cast<float2*>(w + lay.spec);
  double* partials = reinterpret_cast<double*>(w + lay.partials);
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
    ra.fill_spans = 0;
    const int src = dtype == HU_F32 ? SRC_F32 : SRC_I8;
    HU_HIP(timed("rows_r2c_load", st, [&] { return launch_rows_r2c(Lrow, src, 0, ra, B, st); }));
    if (g.nd == 3) {
      ColsArgs cy{};
      cy.spec = spec;
      cy.Nh = g.Nhp;
      cy.ncol = g.n[0] * g.nxh;
      cy.inner = g.nxh;
      cy.tw = tw_1;
      cy.sc = col_sched(g.n[1], 0, cy.ncol, B, Y_PASS_GROUP);
      HU_HIP(timed("cols_y_fwd", st, [&] { return launch_cols(g.n[1], false, 0, cy, st); }));
    }
    WvarArgs wa{};
    wa.spec = spec;
    wa.Nh = g.Nhp;
    wa.gm = axis0(g);
    wa.sc = col_sched(g.n[0], 0, wa.gm.ncol, B);
    wa.tw = tw_0;
    wa.nr = n_radii;
    for (int j = 0; j < n_radii; ++j) wa.radii[j] = (float)radii[j];
    wa.partials = partials;
    HU_HIP(timed("cols_wvar", st, [&] { return launch_cols_wvar(g.n[0], wa, st); }));
    WvarFinalArgs fa{partials, wa.sc.ntiles, n_radii, 1.0 / ((double)g.N * (double)g.N), out + (size_t)f0 * n_radii};
    HU_HIP(timed("wvar_final", st, [&] { return launch_wvar_final(fa, B, st); }));
  }
  return HU_OK;
}

int hu_level_threshold(double phi, double sigma_f, double* t) {
  if (!t || !std::isfinite(phi) || !std::isfinite(sigma_f) || !(phi > 0.0) || !(phi < 1.0) || !(sigma_f > 0.0))
    return HU_ERR_ARG;
  // the upper tail p = min(phi, 1 - phi) (1 - phi is exact for phi >= 1/2), x >= 0 with
  // Q(x) = P(Z >= x) = erfc(x / sqrt 2) / 2 = p, and t = +-x.  Newton's method on ln Q(x) - ln p
  // (d ln Q / dx = -exp(-x^2/2) / (sqrt(2 pi) Q)) keeps relative precision deep in the tail;
  // a bisection bracket catches any step that leaves it.
  const bool upper = phi <= 0.5;
  const double p = upper ? phi : 1.0 - phi;
  double x = 0.0;
  if (p < 0.5) {
    const double rt2 = std::sqrt(2.0), rt2pi = std::sqrt(2.0 * 3.14159265358979323846);
    const double lp = std::log(p);
    double lo = 0.0, hi = 40.0;
    x = std::sqrt(-2.0 * lp);                              // above the root: Q(x) < exp(-x^2/2) / 2
    for (int it = 0; it < 100; ++it) {
      const double q = 0.5 * std::erfc(x / rt2);
      const double gx = std::log(q) - lp;
      if (gx > 0.0) lo = x; else hi = x;                  // ln Q decreases with x
      double xn = x + gx * q * rt2pi * std::exp(0.5 * x * x);
      if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
      const bool done = std::fabs(xn - x) <= 1e-15 * x;
      x = xn;
      if (done) break;
    }
  }
  *t = sigma_f * (upper ? x : -x);
  return HU_OK;
}

int hu_level_cut(hu_dims dims, int32_t batch, const float* field, double phi, double sigma_f, int8_t* out,
                 uint64_t* counts, float near_tol, void* stream) {
  Geom g;
  HU_TRY(make_geom(dims, &g));
  if (batch < 1 || !field || !out) return HU_ERR_ARG;
  if (!std::isfinite(near_tol) || near_tol < 0.0f) return HU_ERR_ARG;
  double t = 0.0;
  HU_TRY(hu_level_threshold(phi, sigma_f, &t));
  if (!aligned(field, 16) || !aligned(out, 16) || (counts && !aligned(counts, 16))) return HU_ERR_ALIGN;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (counts) HU_HIP(timed("zero", st, [&] { return launch_zero_u64(counts, 2LL * batch, st); }));
  ThreshArgs a{field, out, counts, g.N, near_tol, (float)t};
  HU_HIP(timed("threshold", st, [&] { return launch_threshold(a, batch, st); }));
  return HU_OK;
}

int hu_two_point(hu_dims dims, int32_t batch, const int8_t* pm1, float* s2, void* work, size_t work_bytes,
                 void* stream) {
  Geom g;
  HU_TRY(make_geom(dims, &g));
  if (batch < 1 || !pm1 || !s2) return HU_ERR_ARG;
  if (!aligned(pm1, 16) || !aligned(s2, 16)) return HU_ERR_ALIGN;
  if (!work || !aligned(work, 256)) return work ? HU_ERR_ALIGN : HU_ERR_ARG;
  const int chunk = batch < MAX_CHUNK ? batch : MAX_CHUNK;
  Layout lay;
  HU_TRY(layout(g, chunk, true, TunePlan{}, nullptr, &lay));
  if (work_bytes < lay.total) return HU_ERR_WORKSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int Lrow = g.nx / 2;
  const float2 *tw_row, *tw2_row, *tw_0, *tw_1 = nullptr;
  HU_TRY(get_tw(Lrow, &tw_row));
  HU_TRY(get_tw2(Lrow, &tw2_row));
  HU_TRY(get_tw(g.n[0], &tw_0));
  if (g.nd == 3) HU_TRY(get_tw(g.n[1], &tw_1));
  char* w = reinterpret_cast<char*>(work);
  float2* spec = reinterpret_cast<float2*>(w + lay.spec);
  double* fstats = reinterpret_cast<double*>(w + lay.fstats);
  for (int f0 = 0; f0 < batch; f0 += MAX_CHUNK) {
    const int B = batch - f0 < MAX_CHUNK ? batch - f0 : MAX_CHUNK;
    RowsArgs ra{};
    ra.spec = spec;
    ra.Nh = g.Nhp;
    ra.tiled = g.tiled;
    ra.N = g.N;
    ra.nrows = g.nrows;
    ra.src = pm1 + (size_t)f0 * g.N;
    ra.tw = tw_row;
    ra.tw2 = tw2_row;
    ra.fill_spans = 0;
    HU_HIP(timed("rows_r2c_load", st, [&] { return launch_rows_r2c(Lrow, SRC_I8, 0, ra, B, st); }));
    ColsArgs cy{};
    if (g.nd == 3) {
      cy.spec = spec;
      cy.Nh = g.Nhp;
      cy.ncol = g.n[0] * g.nxh;
      cy.inner = g.nxh;
      cy.tw = tw_1;
      cy.sc = col_sched(g.n[1], 0, cy.ncol, B, Y_PASS_GROUP);
      HU_HIP(timed("cols_y_fwd", st, [&] { return launch_cols(g.n[1], false, 0, cy, st); }));
    }
    SquareArgs sa{};
    sa.spec = spec;
    sa.Nh = g.Nhp;
    sa.N = g.N;
    sa.gm = axis0(g);
    sa.sc = col_sched(g.n[0], 0, sa.gm.ncol, B);
    sa.tw = tw_0;
    sa.fstats = fstats;
    HU_HIP(timed("cols_square", st, [&] { return launch_cols_square(g.n[0], sa, st); }));
    if (g.nd == 3) HU_HIP(timed("cols_y_inv", st, [&] { return launch_cols(g.n[1], true, 0, cy, st); }));
    RowsZArgs za{};
    za.spec = spec;
    za.Nh = g.Nhp;
    za.tiled = g.tiled;
    za.N = g.N;
    za.nrows = g.nrows;
    za.tw = tw_row;
    za.tw2 = tw2_row;
    za.fstats = fstats;
    za.field = s2 + (size_t)f0 * g.N;
    HU_HIP(timed("rows_c2r", st, [&] { return launch_rows_c2r(Lrow, false, 0, za, B, st); }));
  }
  return HU_OK;
}

int hu_small_k_exponent(const double* sum, const uint64_t* cnt, hu_bins bins, int32_t nfit, double* alpha) {
  if (!sum || !cnt || !alpha) return HU_ERR_ARG;
  const int R = bins.n_radial, A = bins.n_angular;
  if (R < 2 || A < 1 || nfit < 1 || nfit > R - 1) return HU_ERR_ARG;
  // least squares of y = ln P on x = ln k over the usable bins, in FP64
  double sx = 0.0, sy = 0.0, sxx = 0.0, sxy = 0.0;
  int n = 0;
  for (int r = 1; r <= nfit; ++r) {
    double s = 0.0, c = 0.0;
    for (int q = 0; q < A; ++q) {
      s += sum[(size_t)r * A + q];
      c += (double)cnt[(size_t)r * A + q];
    }
    if (!(c > 0.0) || !(s > 0.0)) continue;
    const double xv = std::log((r + 0.5) / R), yv = std::log(s / c);
    sx += xv;
    sy += yv;
    sxx += xv * xv;
    sxy += xv * yv;
    ++n;
  }
  if (n < 2) return HU_ERR_ARG;
  const double den = n * sxx - sx * sx;
  if (!(den > 0.0)) return HU_ERR_ARG;
  *alpha = (n * sxy - sx * sy) / den;
  return HU_OK;
}

int hu_hyperuniformity_class(double alpha, int32_t d, double tol) {
  if (std::fabs(alpha - 1.0) <= tol) return 1;
  if (alpha > 1.0) return 0;
  if (std::fabs(alpha) <= tol) return 3;
  if (alpha > 0.0) return 2;
  if (alpha > -(double)d) return 4;
  return 5;
}

const char* hu_strerror(int code) {
  switch (code) {
    case HU_OK: return "ok";
    case HU_ERR_ARG: return "invalid argument";
    case HU_ERR_SIZE: return "grid size outside the supported set (2^k in 4..2048, 3*2^k in 6..768 per axis, N < 2^31, half spectrum < 4 GiB)";
    case HU_ERR_ALIGN: return "misaligned pointer (arrays need 16 bytes, workspace 256 bytes)";
    case HU_ERR_WORKSPACE: return "workspace smaller than hu_workspace_size";
    case HU_ERR_DEGENERATE: return "filter has no support on the lattice (max ln chi < -80)";
    case HU_ERR_HIP: return "HIP runtime error";
    case HU_ERR_UNSUPPORTED: return "unsupported request";
    case HU_ERR_TABLES: return "the per-size tables of this grid and bin layout do not exist yet (hu_pipeline_noalloc allocates none: make any allocating call on the same grid and bins first)";
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

int hu_profile_enable(int on) { return profile_reset(on != 0); }

int hu_profile_read(char (*names)[48], int64_t* launches, double* total_ms, int cap) {
  std::vector<std::string> fam;
  std::vector<long long> cnt;
  std::vector<double> ms;
  HU_TRY(profile_collect(fam, cnt, ms));
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
