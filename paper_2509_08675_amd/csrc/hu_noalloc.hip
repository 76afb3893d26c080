// hu_pipeline_noalloc: hu_pipeline with its workspace in a fixed device array of the library, for
// callers that cannot allocate device memory (see include/hufield.h for the contract).
#include <map>
#include <mutex>

#include "hu_host.hpp"

using namespace hu;

namespace {

// The workspace of every hu_pipeline_noalloc call on a device.  In host code `scratch` names a
// host-side stand-in, not a device address: kernels get the per-device address that
// hipGetSymbolAddress returns for it.
static __device__ __align__(256) unsigned char scratch[HU_NOALLOC_WORK_BYTES];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> address of that device's copy of `scratch`

// the current device's address of `scratch`, looked up once per device
int scratch_ptr(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HU_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HU_ERR_HIP;
    it = g_scratch_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return HU_OK;
}

}  // namespace

extern "C" int hu_pipeline_noalloc(hu_dims dims, int32_t batch, const hu_filter* filt, const uint64_t* seeds,
                                   hu_bins bins, float near_tol, const hu_outputs* out, void* stream) {
  if (!out) return HU_ERR_ARG;
  Geom g;
  HU_TRY(make_geom(dims, &g));
  if (batch < 1 || !seeds) return HU_ERR_ARG;
  HU_TRY(check_bins(&bins, g.nd));
  // the half spectra alone beyond the fixed array: refused before anything else
  const int chunk = batch < MAX_CHUNK ? batch : MAX_CHUNK;
  if ((size_t)chunk * (size_t)g.Nhp * 8 > HU_NOALLOC_WORK_BYTES) return HU_ERR_WORKSPACE;
  // the tables must exist already: building them would allocate
  HU_TRY(tables_ready(g, &bins));
  // the whole workspace of this shape (the plan may be a tuned one): within the fixed array?
  Layout lay;
  HU_TRY(layout(g, chunk, true, get_plan(g, &bins, batch), &bins, &lay));
  if (lay.total > HU_NOALLOC_WORK_BYTES) return HU_ERR_WORKSPACE;
  void* work = nullptr;
  HU_TRY(scratch_ptr(&work));
  return run_generator(dims, batch, filt, seeds, &bins, near_tol, *out, true, work, HU_NOALLOC_WORK_BYTES, stream);
}
