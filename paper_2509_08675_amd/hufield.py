"""Python binding of libhufield.so (the C-ABI in include/hufield.h).

Argument marshalling only: every step of the hot path runs in the HIP kernels of the library.
PyTorch supplies device memory and the current stream.  There is no CPU fallback: if the
library is not built, importing this module raises ImportError.
"""

import ctypes
import os

import numpy as np
import torch

# HUFIELD_LIB selects another build of the same library (the host-sanitizer build of the tests)
_LIB_PATH = os.environ.get("HUFIELD_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhufield.so")

if not os.path.exists(_LIB_PATH):
    raise ImportError("libhufield.so is not built (run: python -m paper_2509_08675_amd.build); "
                      "the hyperuniform-field path has no CPU fallback")

_lib = ctypes.CDLL(_LIB_PATH)

HU_OK, HU_ERR_ARG, HU_ERR_SIZE, HU_ERR_ALIGN, HU_ERR_WORKSPACE, HU_ERR_DEGENERATE, HU_ERR_HIP, \
    HU_ERR_UNSUPPORTED, HU_ERR_TABLES = 0, -1, -2, -3, -4, -5, -6, -7, -8
HU_NOALLOC_WORK_BYTES = 128 << 20
HU_F32, HU_I8 = 0, 1
HU_OP_GEN_FIELD, HU_OP_PIPELINE, HU_OP_POWER_SPECTRUM, HU_OP_LOSS, HU_OP_FILTER_SPECTRUM = 0, 1, 2, 3, 4
HU_OP_WINDOW_VARIANCE = 5
HU_OP_TWO_POINT = 6
HU_MAX_RADII = 32
HU_CLASSES = ("hyperuniform class I", "hyperuniform class II", "hyperuniform class III",
              "nonhyperuniform (standard)", "antihyperuniform", "outside the classified range")


class hu_dims(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 3)]


class hu_filter(ctypes.Structure):
    _fields_ = [("p", ctypes.c_double), ("semi", ctypes.c_double * 3), ("rot", ctypes.c_double),
                ("alpha", ctypes.c_double), ("k0", ctypes.c_double), ("width", ctypes.c_double),
                ("sigma_f", ctypes.c_double), ("offset", ctypes.c_double),
                ("prof", ctypes.c_void_p), ("prof_n", ctypes.c_int32), ("prof_dk", ctypes.c_double)]


class hu_bins(ctypes.Structure):
    _fields_ = [("n_radial", ctypes.c_int32), ("n_angular", ctypes.c_int32)]


class hu_outputs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("field", "pm1", "stats", "counts", "cont_sum", "cont_cnt", "pm1_sum", "pm1_cnt")]


class hu_job(ctypes.Structure):
    _fields_ = [("dims", hu_dims), ("filt", hu_filter), ("seed", ctypes.c_uint64), ("bins", hu_bins)] + \
               [(n, ctypes.c_void_p) for n in
                ("field", "pm1", "stats", "counts", "cont_sum", "cont_cnt", "pm1_sum", "pm1_cnt")]


_vp, _sz, _i32, _u64, _f32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_uint64, ctypes.c_float
_P = ctypes.POINTER

_lib.hu_workspace_size.argtypes = [ctypes.c_int, hu_dims, _i32, _P(hu_bins), _P(_sz)]
_lib.hu_gen_field.argtypes = [hu_dims, _i32, _P(hu_filter), _P(_u64), _vp, _vp, _P(hu_bins), _vp, _vp, _vp, _sz,
                              _vp]
_lib.hu_threshold.argtypes = [hu_dims, _i32, _vp, _vp, _vp, _f32, _vp]
_lib.hu_power_spectrum.argtypes = [hu_dims, _i32, _vp, _i32, hu_bins, _vp, _vp, _vp, _sz, _vp]
_lib.hu_pipeline.argtypes = [hu_dims, _i32, _P(hu_filter), _P(_u64), hu_bins, _f32, _P(hu_outputs), _vp, _sz, _vp]
_lib.hu_pipeline_noalloc.argtypes = [hu_dims, _i32, _P(hu_filter), _P(_u64), hu_bins, _f32, _P(hu_outputs), _vp]
_lib.hu_strerror.argtypes = [ctypes.c_int]
_lib.hu_strerror.restype = ctypes.c_char_p
_lib.hu_debug_philox.argtypes = [_u64, _u64, _u64, _vp, _vp, _vp]
_lib.hu_profile_enable.argtypes = [ctypes.c_int]
_lib.hu_profile_read.argtypes = [_vp, _vp, _vp, ctypes.c_int]
_lib.hu_workspace_size_batch.argtypes = [_P(hu_job), _i32, _P(_sz)]
_lib.hu_pipeline_batch.argtypes = [_P(hu_job), _i32, _f32, _P(_i32), _vp, _sz, _vp]
_lib.hu_autotune.argtypes = [hu_dims, _i32, _P(hu_bins), ctypes.c_char_p, _P(ctypes.c_double)]
_lib.hu_plan_query.argtypes = [hu_dims, _i32, _P(hu_bins), _P(_i32)]
_lib.hu_plan_set.argtypes = [hu_dims, _i32, _P(hu_bins), _P(_i32)]
_lib.hu_filter_spectrum.argtypes = [hu_dims, _P(hu_filter), hu_bins, _vp, _vp, _vp, _sz, _vp]
_lib.hu_spectrum_grad.argtypes = [hu_dims, _P(hu_filter), _u64, hu_bins, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.hu_window_variance.argtypes = [hu_dims, _i32, _vp, _i32, _P(ctypes.c_double), _i32, _vp, _vp, _sz, _vp]
_lib.hu_small_k_exponent.argtypes = [_P(ctypes.c_double), _P(_u64), hu_bins, _i32, _P(ctypes.c_double)]
_lib.hu_hyperuniformity_class.argtypes = [ctypes.c_double, _i32, ctypes.c_double]
_lib.hu_level_threshold.argtypes = [ctypes.c_double, ctypes.c_double, _P(ctypes.c_double)]
_lib.hu_level_cut.argtypes = [hu_dims, _i32, _vp, ctypes.c_double, ctypes.c_double, _vp, _vp, _f32, _vp]
_lib.hu_two_point.argtypes = [hu_dims, _i32, _vp, _vp, _vp, _sz, _vp]
_lib.hu_debug_bin_tables.argtypes = [hu_dims, hu_bins, _i32, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.hu_spectrum_loss.argtypes = [hu_bins, _vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp]
for _f in ("hu_workspace_size", "hu_gen_field", "hu_threshold", "hu_power_spectrum", "hu_pipeline", "hu_pipeline_noalloc",
           "hu_debug_philox", "hu_profile_enable", "hu_profile_read", "hu_workspace_size_batch",
           "hu_pipeline_batch", "hu_autotune", "hu_plan_query", "hu_plan_set", "hu_filter_spectrum",
           "hu_spectrum_grad", "hu_window_variance", "hu_small_k_exponent", "hu_hyperuniformity_class",
           "hu_level_threshold", "hu_level_cut", "hu_two_point", "hu_debug_bin_tables", "hu_spectrum_loss"):
    getattr(_lib, _f).restype = ctypes.c_int


class HuError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed: %s (%d)" % (what, strerror(code), code))
        self.code = code


class DegenerateFilter(RuntimeError):
    """The filter has no support on the lattice (max ln chi < -80), reported by the kernels."""


def strerror(code):
    return _lib.hu_strerror(int(code)).decode()


def _check(rc, what):
    if rc != HU_OK:
        raise HuError(rc, what)


def lib_path():
    return _LIB_PATH


def lib_handle():
    return _lib


# ---------------------------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------------------------
def make_dims(dims):
    dims = tuple(int(n) for n in dims)
    d = hu_dims()
    d.ndim = len(dims)
    for i, n in enumerate(dims):
        d.n[i] = n
    return d


def make_filter(f):
    """hu_filter from a dict (keys p, semi, rot, alpha, k0, width, sigma_f, offset, and optionally
    prof, prof_dk) or an object with those attributes.  prof: a tabulated radial form, ln chi at
    K = i * prof_dk, as a contiguous 1-D float32 tensor on the device (kept alive by the caller
    for the duration of the call); alpha, k0 and width are then unused."""
    get = (lambda k, dflt=None: f.get(k, dflt)) if isinstance(f, dict) else (lambda k, dflt=None: getattr(f, k, dflt))
    h = hu_filter()
    prof = get("prof")
    h.p = float(get("p"))
    semi = tuple(get("semi", (1.0, 1.0, 1.0))) + (1.0,) * 3
    for i in range(3):
        h.semi[i] = float(semi[i])
    h.rot = float(get("rot", 0.0))
    h.alpha = float(get("alpha", 0.0 if prof is not None else None))
    h.k0 = float(get("k0", 0.0))
    h.width = float(get("width", 1.0 if prof is not None else None))
    h.sigma_f = float(get("sigma_f", 1.0))
    h.offset = float(get("offset", 0.0))
    if prof is not None:
        if not (isinstance(prof, torch.Tensor) and prof.is_cuda and prof.dtype == torch.float32
                and prof.dim() == 1 and prof.is_contiguous()):
            raise TypeError("prof must be a contiguous 1-D float32 tensor on the device")
        h.prof = prof.data_ptr()
        h.prof_n = prof.numel()
        h.prof_dk = float(get("prof_dk"))
    return h


def make_bins(bins):
    b = hu_bins()
    b.n_radial, b.n_angular = int(bins[0]), int(bins[1]) if len(bins) > 1 else 1
    return b


def _seeds(seeds):
    arr = (_u64 * len(seeds))()
    for i, s in enumerate(seeds):
        arr[i] = int(s) & 0xFFFFFFFFFFFFFFFF
    return arr


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def workspace_size(op, dims, batch, bins=None):
    out = _sz()
    b = make_bins(bins) if bins is not None else None
    _check(_lib.hu_workspace_size(int(op), make_dims(dims), int(batch), ctypes.byref(b) if b else None,
                                  ctypes.byref(out)), "hu_workspace_size")
    return int(out.value)


def alloc_workspace(op, dims, batch, bins=None, device="cuda"):
    n = workspace_size(op, dims, batch, bins)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


def _nb(bins):
    return int(bins[0]) * (int(bins[1]) if len(bins) > 1 else 1) + 1


def u64_view(t):
    """Host numpy uint64 view of a device int64 tensor written as uint64 by the library."""
    return t.detach().cpu().numpy().view(np.uint64)


# ---------------------------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------------------------
def gen_field(dims, filt, seeds, cont_bins=None, device="cuda", work=None, out=None):
    """Normalised fields [B, *dims] (FP32) plus stats [B, 4] and, if cont_bins, the continuous
    spectrum (sum [B, nb] FP64, cnt [B, nb] uint64-in-int64)."""
    dims = tuple(int(n) for n in dims)
    B = len(seeds)
    field = out if out is not None else torch.empty((B,) + dims, dtype=torch.float32, device=device)
    stats = torch.empty((B, 4), dtype=torch.float64, device=device)
    cs = cc = None
    b = None
    if cont_bins is not None:
        nb = _nb(cont_bins)
        cs = torch.empty((B, nb), dtype=torch.float64, device=device)
        cc = torch.empty((B, nb), dtype=torch.int64, device=device)
        b = make_bins(cont_bins)
    if work is None:
        work = alloc_workspace(HU_OP_GEN_FIELD, dims, B, cont_bins, device)
    h = make_filter(filt)
    _check(_lib.hu_gen_field(make_dims(dims), B, ctypes.byref(h), _seeds(seeds), _ptr(field), _ptr(stats),
                             ctypes.byref(b) if b else None, _ptr(cs), _ptr(cc), _ptr(work), work.numel(),
                             _stream(field.device)), "hu_gen_field")
    return dict(field=field, stats=stats, cont_sum=cs, cont_cnt=cc)


def threshold(field, near_tol=1e-5, out=None, counts=True):
    """Sign map of fields [B, *dims] (FP32, on device): +1 where field >= 0 else -1 (int8), and
    counts [B, 2] = (n_pos, #(|field| < near_tol))."""
    dims = tuple(field.shape[1:])
    B = field.shape[0]
    t = out if out is not None else torch.empty(field.shape, dtype=torch.int8, device=field.device)
    cnt = torch.empty((B, 2), dtype=torch.int64, device=field.device) if counts else None
    _check(_lib.hu_threshold(make_dims(dims), B, _ptr(field), _ptr(t), _ptr(cnt), float(near_tol),
                             _stream(field.device)), "hu_threshold")
    return t, cnt


def power_spectrum(x, bins, work=None):
    """Binned periodogram of real fields x [B, *dims] (float32 or int8 on device):
    sum [B, nb] FP64 and cnt [B, nb]."""
    dims = tuple(x.shape[1:])
    B = x.shape[0]
    if x.dtype == torch.float32:
        dt = HU_F32
    elif x.dtype == torch.int8:
        dt = HU_I8
    else:
        raise TypeError("power_spectrum takes float32 or int8 fields")
    nb = _nb(bins)
    s = torch.empty((B, nb), dtype=torch.float64, device=x.device)
    c = torch.empty((B, nb), dtype=torch.int64, device=x.device)
    if work is None:
        work = alloc_workspace(HU_OP_POWER_SPECTRUM, dims, B, bins, x.device)
    _check(_lib.hu_power_spectrum(make_dims(dims), B, _ptr(x), dt, make_bins(bins), _ptr(s), _ptr(c), _ptr(work),
                                  work.numel(), _stream(x.device)), "hu_power_spectrum")
    return s, c


def window_variance(x, radii, work=None):
    """Local variance over a spherical window of each radius (lattice units) of real fields
    x [B, *dims] (float32 or int8 on device): [B, len(radii)] FP64 (Eq. (1) in Fourier form)."""
    dims = tuple(x.shape[1:])
    B = x.shape[0]
    if x.dtype == torch.float32:
        dt = HU_F32
    elif x.dtype == torch.int8:
        dt = HU_I8
    else:
        raise TypeError("window_variance takes float32 or int8 fields")
    r = (ctypes.c_double * len(radii))(*[float(v) for v in radii])
    out = torch.empty((B, len(radii)), dtype=torch.float64, device=x.device)
    if work is None:
        work = alloc_workspace(HU_OP_WINDOW_VARIANCE, dims, B, None, x.device)
    _check(_lib.hu_window_variance(make_dims(dims), B, _ptr(x), dt, r, len(radii), _ptr(out), _ptr(work),
                                   work.numel(), _stream(x.device)), "hu_window_variance")
    return out


def small_k_exponent(bin_sum, bin_cnt, bins, nfit):
    """Small-k exponent of one binned spectrum (sum [nb] FP64 and cnt [nb], any device)."""
    def host(t):
        return t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)
    s = np.ascontiguousarray(host(bin_sum), dtype=np.float64)
    c = np.ascontiguousarray(host(bin_cnt).astype(np.uint64))   # counts are < 2^63
    if s.size < _nb(bins) or c.size < _nb(bins):
        raise ValueError("binned spectrum shorter than the bin layout")
    a = ctypes.c_double()
    _check(_lib.hu_small_k_exponent(s.ctypes.data_as(_P(ctypes.c_double)), c.ctypes.data_as(_P(_u64)),
                                    make_bins(bins), int(nfit), ctypes.byref(a)), "hu_small_k_exponent")
    return a.value


def hyperuniformity_class(alpha, d, tol=1e-6):
    """Name of the class of Eqs. (6)-(7) for a small-k exponent alpha in dimension d."""
    return HU_CLASSES[_lib.hu_hyperuniformity_class(float(alpha), int(d), float(tol))]


def level_threshold(phi, sigma_f=1.0):
    """t_phi = sigma_f Phi^-1(1 - phi) (host, FP64)."""
    t = ctypes.c_double()
    _check(_lib.hu_level_threshold(float(phi), float(sigma_f), ctypes.byref(t)), "hu_level_threshold")
    return t.value


def level_cut(field, phi, sigma_f=1.0, near_tol=0.0, out=None, counts=True):
    """+1 where field >= t_phi else -1 for fields [B, *dims] float32 on device; returns (map int8,
    counts [B, 2] int64 holding uint64 (n_pos, n_near) or None)."""
    dims = tuple(field.shape[1:])
    B = field.shape[0]
    if out is None:
        out = torch.empty(field.shape, dtype=torch.int8, device=field.device)
    c = torch.empty((B, 2), dtype=torch.int64, device=field.device) if counts else None
    _check(_lib.hu_level_cut(make_dims(dims), B, _ptr(field), float(phi), float(sigma_f), _ptr(out),
                             _ptr(c) if c is not None else None, float(near_tol), _stream(field.device)),
           "hu_level_cut")
    return out, c


def two_point(pm1, work=None, out=None):
    """S_2(r) of the +1 phase of +-1 maps pm1 [B, *dims] int8 on device: float32 [B, *dims], index
    r mod n per axis."""
    dims = tuple(pm1.shape[1:])
    B = pm1.shape[0]
    if pm1.dtype != torch.int8:
        raise TypeError("two_point takes int8 maps")
    if out is None:
        out = torch.empty(pm1.shape, dtype=torch.float32, device=pm1.device)
    if work is None:
        work = alloc_workspace(HU_OP_TWO_POINT, dims, B, None, pm1.device)
    _check(_lib.hu_two_point(make_dims(dims), B, _ptr(pm1), _ptr(out), _ptr(work), work.numel(),
                             _stream(pm1.device)), "hu_two_point")
    return out


class PipelineBuffers:
    """Preallocated outputs and workspace for repeated hu_pipeline calls on one configuration."""

    def __init__(self, dims, batch, bins, device="cuda", want=("field", "pm1", "stats", "counts", "cont", "pm1_spec")):
        dims = tuple(int(n) for n in dims)
        self.dims, self.batch, self.bins = dims, int(batch), tuple(bins)
        nb = _nb(bins)
        dev = device
        self.field = torch.empty((batch,) + dims, dtype=torch.float32, device=dev) if "field" in want else None
        self.pm1 = torch.empty((batch,) + dims, dtype=torch.int8, device=dev) if "pm1" in want else None
        self.stats = torch.empty((batch, 4), dtype=torch.float64, device=dev) if "stats" in want else None
        self.counts = torch.empty((batch, 2), dtype=torch.int64, device=dev) if "counts" in want else None
        if "cont" in want:
            self.cont_sum = torch.empty((batch, nb), dtype=torch.float64, device=dev)
            self.cont_cnt = torch.empty((batch, nb), dtype=torch.int64, device=dev)
        else:
            self.cont_sum = self.cont_cnt = None
        if "pm1_spec" in want:
            self.pm1_sum = torch.empty((batch, nb), dtype=torch.float64, device=dev)
            self.pm1_cnt = torch.empty((batch, nb), dtype=torch.int64, device=dev)
        else:
            self.pm1_sum = self.pm1_cnt = None
        self.work = alloc_workspace(HU_OP_PIPELINE, dims, batch, bins, dev)
        o = hu_outputs()
        for name in ("field", "pm1", "stats", "counts", "cont_sum", "cont_cnt", "pm1_sum", "pm1_cnt"):
            setattr(o, name, None if getattr(self, name) is None else getattr(self, name).data_ptr())
        self._out = o
        self._dims = make_dims(dims)
        self._bins = make_bins(bins)


def pipeline(bufs, filt, seeds, near_tol=1e-5):
    """The whole hot path into preallocated PipelineBuffers (asynchronous on the current stream)."""
    if len(seeds) != bufs.batch:
        raise ValueError("need one seed per field")
    h = make_filter(filt)
    dev = bufs.work.device
    _check(_lib.hu_pipeline(bufs._dims, bufs.batch, ctypes.byref(h), _seeds(seeds), bufs._bins, float(near_tol),
                            ctypes.byref(bufs._out), _ptr(bufs.work), bufs.work.numel(), _stream(dev)),
           "hu_pipeline")
    return bufs


def pipeline_noalloc(bufs, filt, seeds, near_tol=1e-5):
    """hu_pipeline_noalloc into the outputs of PipelineBuffers (its workspace is not used: the
    library's fixed device array is).  Raises HuError(HU_ERR_TABLES) if no allocating call has
    built this grid's tables yet, HuError(HU_ERR_WORKSPACE) beyond the array's size."""
    if len(seeds) != bufs.batch:
        raise ValueError("need one seed per field")
    h = make_filter(filt)
    _check(_lib.hu_pipeline_noalloc(bufs._dims, bufs.batch, ctypes.byref(h), _seeds(seeds), bufs._bins,
                                    float(near_tol), ctypes.byref(bufs._out), _stream(bufs.work.device)),
           "hu_pipeline_noalloc")
    return bufs


def check_degenerate(stats):
    """Raise DegenerateFilter if any field's stats flag says the filter has no lattice support."""
    st = stats.detach().cpu().numpy()
    bad = np.nonzero(st[:, 3] != 0)[0]
    if bad.size:
        raise DegenerateFilter("filter has no support on the lattice for fields %s (max ln chi %s)"
                               % (bad.tolist(), st[bad, 2].tolist()))


def debug_philox(seed, first, count, device="cuda"):
    """Raw Philox words [count, 4] (uint32 bits in int32) and the FP32 normals [count, 4]."""
    w = torch.empty((count, 4), dtype=torch.int32, device=device)
    z = torch.empty((count, 4), dtype=torch.float32, device=device)
    _check(_lib.hu_debug_philox(int(seed), int(first), int(count), _ptr(w), _ptr(z), _stream(w.device)),
           "hu_debug_philox")
    return w, z


def debug_bin_tables(dims, bins, variant=0):
    """The host-built bin tables of a grid (no device work): dict with ncol, n0, ntiles, M,
    nloc_max, width and the arrays table, ltab [ncol, n0] (uint16), toff, coff, cpos (uint32)."""
    import numpy as np
    d, b = make_dims(dims), make_bins(bins)
    sz = (ctypes.c_int32 * 6)()
    _check(_lib.hu_debug_bin_tables(d, b, int(variant), ctypes.addressof(sz), None, None, None, None, None),
           "hu_debug_bin_tables")
    ncol, n0, ntiles, M, nloc_max, width = list(sz)
    nb = b.n_radial * b.n_angular + 1
    table = np.empty((ncol, n0), np.uint16)
    ltab = np.empty((ncol, n0), np.uint16)
    toff = np.empty(ntiles + 1, np.uint32)
    coff = np.empty(nb + 1, np.uint32)
    cpos = np.empty(max(M, 1), np.uint32)
    _check(_lib.hu_debug_bin_tables(d, b, int(variant), None, table.ctypes.data, ltab.ctypes.data,
                                    toff.ctypes.data, coff.ctypes.data, cpos.ctypes.data), "hu_debug_bin_tables")
    return dict(ncol=ncol, n0=n0, ntiles=ntiles, M=M, nloc_max=nloc_max, width=width, table=table, ltab=ltab,
                toff=toff, coff=coff, cpos=cpos[:M])


def profile_enable(on=True):
    _check(_lib.hu_profile_enable(1 if on else 0), "hu_profile_enable")


def profile_read(cap=64):
    names = (ctypes.c_char * 48 * cap)()
    launches = (ctypes.c_int64 * cap)()
    ms = (ctypes.c_double * cap)()
    n = _lib.hu_profile_read(names, launches, ms, cap)
    if n < 0:
        raise HuError(n, "hu_profile_read")
    out = {}
    for i in range(min(n, cap)):
        out[bytes(names[i]).split(b"\0", 1)[0].decode()] = (int(launches[i]), float(ms[i]))
    return out


# ---------------------------------------------------------------------------------------------
# heterogeneous batches and the autotuner
# ---------------------------------------------------------------------------------------------
PASS_NAMES = ("rows_r2c", "cols_y", "cols_filter", "rows_c2r", "cols_bin", "bin_schedule", "field_placement",
              "y_group", "radix", "bin_exchange", "filter_exchange", "whole_field", "plane")


class BatchBuffers:
    """Outputs for a heterogeneous batch: job i gets field, pm1, stats, counts and, with bins,
    the continuous and +-1 spectra, each a device tensor; plus the batch workspace."""

    def __init__(self, jobs, device="cuda", want=("field", "pm1", "stats", "counts", "cont", "pm1_spec")):
        self.jobs = list(jobs)
        dev = device
        self.out = []
        arr = (hu_job * len(self.jobs))()
        for i, j in enumerate(self.jobs):
            dims = tuple(int(n) for n in j["dims"])
            o = {}
            if "field" in want:
                o["field"] = torch.empty(dims, dtype=torch.float32, device=dev)
            if "pm1" in want:
                o["pm1"] = torch.empty(dims, dtype=torch.int8, device=dev)
            if "stats" in want:
                o["stats"] = torch.empty(4, dtype=torch.float64, device=dev)
            if "counts" in want:
                o["counts"] = torch.empty(2, dtype=torch.int64, device=dev)
            bins = j.get("bins")
            if bins is not None:
                nb = _nb(bins)
                if "cont" in want:
                    o["cont_sum"] = torch.empty(nb, dtype=torch.float64, device=dev)
                    o["cont_cnt"] = torch.empty(nb, dtype=torch.int64, device=dev)
                if "pm1_spec" in want:
                    o["pm1_sum"] = torch.empty(nb, dtype=torch.float64, device=dev)
                    o["pm1_cnt"] = torch.empty(nb, dtype=torch.int64, device=dev)
            self.out.append(o)
            jb = arr[i]
            jb.dims = make_dims(dims)
            jb.filt = make_filter(j["filt"])
            jb.seed = int(j["seed"]) & 0xFFFFFFFFFFFFFFFF
            if bins is not None:
                jb.bins = make_bins(bins)
            for name in ("field", "pm1", "stats", "counts", "cont_sum", "cont_cnt", "pm1_sum", "pm1_cnt"):
                setattr(jb, name, o[name].data_ptr() if name in o else None)
        self._jobs = arr
        need = _sz()
        _check(_lib.hu_workspace_size_batch(arr, len(self.jobs), ctypes.byref(need)), "hu_workspace_size_batch")
        self.work = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=dev)
        self.status = (_i32 * len(self.jobs))()

    def set_seeds(self, seeds):
        for i, s in enumerate(seeds):
            self._jobs[i].seed = int(s) & 0xFFFFFFFFFFFFFFFF


def pipeline_batch(bufs, near_tol=1e-5):
    """The whole hot path for every job of a BatchBuffers in one submission (a replayed HIP graph).
    Returns the per-job status list (0 = ok)."""
    dev = bufs.work.device
    _check(_lib.hu_pipeline_batch(bufs._jobs, len(bufs.jobs), float(near_tol), bufs.status, _ptr(bufs.work),
                                  bufs.work.numel(), _stream(dev)), "hu_pipeline_batch")
    return list(bufs.status)


def autotune(dims, batch, bins, cache_path=None):
    """Search the plan of this shape class (hu_autotune); returns ({entry: 0 or 1}, dict of the
    default plan's and the tuned plan's summed kernel ms and, per entry, the ms with it flipped
    during the search (0 where not tried))."""
    ms = (ctypes.c_double * (2 + len(PASS_NAMES)))()
    b = make_bins(bins)
    _check(_lib.hu_autotune(make_dims(dims), int(batch), ctypes.byref(b),
                            cache_path.encode() if cache_path else None, ms), "hu_autotune")
    v = list(ms)
    return plan_query(dims, batch, bins), dict(default_ms=v[0], tuned_ms=v[1], flipped_ms=dict(zip(PASS_NAMES, v[2:])))


def plan_query(dims, batch, bins):
    v = (_i32 * len(PASS_NAMES))()
    b = make_bins(bins) if bins is not None else None
    _check(_lib.hu_plan_query(make_dims(dims), int(batch), ctypes.byref(b) if b else None, v), "hu_plan_query")
    return dict(zip(PASS_NAMES, list(v)))


def plan_set(dims, batch, bins, variants):
    variants = list(variants) + [0] * (len(PASS_NAMES) - len(variants))
    v = (_i32 * len(PASS_NAMES))(*[int(x) for x in variants])
    b = make_bins(bins) if bins is not None else None
    _check(_lib.hu_plan_set(make_dims(dims), int(batch), ctypes.byref(b) if b else None, v), "hu_plan_set")


# ---------------------------------------------------------------------------------------------
# differentiation with respect to the filter parameters
# ---------------------------------------------------------------------------------------------
THETA_NAMES = ("a", "b", "c", "p", "rot", "k0", "width")


def filter_with_theta(theta, alpha, sigma_f=1.0):
    """Filter dict from theta = (a, b, c, p, rot, k0, w) and the fixed alpha, sigma_f."""
    th = [float(x) for x in theta]
    return dict(semi=tuple(th[0:3]), p=th[3], rot=th[4], k0=th[5], width=th[6], alpha=float(alpha),
                sigma_f=float(sigma_f))


def filter_spectrum(dims, filt, bins, device="cuda", work=None):
    """Expected binned spectrum of the normalised field of a filter (no noise): sum [nb] FP64 and
    cnt [nb]; sum / cnt is the expected bin mean of the continuous spectrum."""
    dims = tuple(int(n) for n in dims)
    nb = _nb(bins)
    s = torch.empty(nb, dtype=torch.float64, device=device)
    c = torch.empty(nb, dtype=torch.int64, device=device)
    if work is None:
        work = alloc_workspace(HU_OP_FILTER_SPECTRUM, dims, 1, bins, device)
    h = make_filter(filt)
    _check(_lib.hu_filter_spectrum(make_dims(dims), ctypes.byref(h), make_bins(bins), _ptr(s), _ptr(c), _ptr(work),
                                   work.numel(), _stream(s.device)), "hu_filter_spectrum")
    return s, c


def spectrum_grad(dims, filt, seed, bins, dL_dP, cont_sum, cont_cnt, stats, work=None):
    """dL/dtheta [7] (device FP64) from dL/d(bin means) [nb] and one field's forward outputs
    (cont_sum [nb], cont_cnt [nb], stats [4] of gen_field with the same dims, filter, seed, bins)."""
    dims = tuple(int(n) for n in dims)
    dev = cont_sum.device
    grad = torch.empty(7, dtype=torch.float64, device=dev)
    if work is None:
        work = alloc_workspace(HU_OP_LOSS, dims, 1, bins, dev)
    h = make_filter(filt)
    dL = dL_dP.to(device=dev, dtype=torch.float64).contiguous()
    _check(_lib.hu_spectrum_grad(make_dims(dims), ctypes.byref(h), int(seed) & 0xFFFFFFFFFFFFFFFF, make_bins(bins),
                                 _ptr(dL), _ptr(cont_sum), _ptr(cont_cnt), _ptr(stats), _ptr(grad), _ptr(work),
                                 work.numel(), _stream(dev)), "hu_spectrum_grad")
    return grad


class FilterSpectrum(torch.autograd.Function):
    """theta [7] = (a, b, c, p, rot, k0, w) -> the binned continuous spectrum P [R*A] (bin means,
    0 for empty bins) of the field generated on `dims` from `seed` with those filter parameters
    (alpha and sigma_f fixed).  Forward: hu_gen_field; backward: hu_spectrum_grad (the noise is
    regenerated from the seed)."""

    @staticmethod
    def forward(ctx, theta, dims, seed, bins, alpha, sigma_f=1.0):
        dims = tuple(int(n) for n in dims)
        filt = filter_with_theta(theta.detach().cpu().tolist(), alpha, sigma_f)
        dev = theta.device if theta.is_cuda else torch.device("cuda")
        out = gen_field(dims, filt, [seed], cont_bins=bins, device=dev)
        check_degenerate(out["stats"])
        cs, cc, st = out["cont_sum"][0], out["cont_cnt"][0], out["stats"][0]
        cnt = cc[:-1].to(torch.float64)
        P = torch.where(cnt > 0, cs[:-1] / cnt.clamp(min=1.0), torch.zeros_like(cnt))
        ctx.save_for_backward(cs, cc, st)
        ctx.meta = (dims, int(seed), tuple(bins), filt, theta.device, theta.dtype)
        return P

    @staticmethod
    def backward(ctx, gP):
        cs, cc, st = ctx.saved_tensors
        dims, seed, bins, filt, tdev, tdt = ctx.meta
        dL = torch.zeros(cs.shape[0], dtype=torch.float64, device=cs.device)
        dL[:-1] = gP.to(device=cs.device, dtype=torch.float64)
        g = spectrum_grad(dims, filt, seed, bins, dL, cs, cc, st)
        return g.to(device=tdev, dtype=tdt), None, None, None, None, None


def spectrum_loss_value(bins, cont_sum, cont_cnt, tsum, tcnt, eps):
    """hu_spectrum_loss: the loss (device FP64 scalar) and dL/dP per bin (device FP64 [R*A+1]) of a
    field's binned spectrum against a target's."""
    dev = cont_sum.device
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    dL = torch.empty(cont_sum.shape[0], dtype=torch.float64, device=dev)
    _check(_lib.hu_spectrum_loss(make_bins(bins), _ptr(cont_sum), _ptr(cont_cnt), _ptr(tsum), _ptr(tcnt), float(eps),
                                 _ptr(loss), _ptr(dL), _stream(dev)), "hu_spectrum_loss")
    return loss[0], dL


class SpectrumLoss(torch.autograd.Function):
    """theta [7] -> the spectrum-matching loss of the field generated from `seed` with those filter
    parameters against the binned target spectrum (tsum, tcnt).  Forward: hu_gen_field and
    hu_spectrum_loss; backward: hu_spectrum_grad with the library's dL/dP (the noise is regenerated
    from the seed)."""

    @staticmethod
    def forward(ctx, theta, dims, seed, bins, alpha, sigma_f, tsum, tcnt, eps):
        dims = tuple(int(n) for n in dims)
        filt = filter_with_theta(theta.detach().cpu().tolist(), alpha, sigma_f)
        dev = theta.device if theta.is_cuda else torch.device("cuda")
        out = gen_field(dims, filt, [seed], cont_bins=bins, device=dev)
        check_degenerate(out["stats"])
        cs, cc, st = out["cont_sum"][0], out["cont_cnt"][0], out["stats"][0]
        loss, dL = spectrum_loss_value(bins, cs, cc, tsum, tcnt, eps)
        ctx.save_for_backward(cs, cc, st, dL)
        ctx.meta = (dims, int(seed), tuple(bins), filt, theta.device, theta.dtype)
        return loss.to(theta.dtype) if theta.dtype != torch.float64 else loss

    @staticmethod
    def backward(ctx, gL):
        cs, cc, st, dL = ctx.saved_tensors
        dims, seed, bins, filt, tdev, tdt = ctx.meta
        g = spectrum_grad(dims, filt, seed, bins, dL * gL.to(device=dL.device, dtype=torch.float64), cs, cc, st)
        return g.to(device=tdev, dtype=tdt), None, None, None, None, None, None, None, None


def spectrum_loss(theta, dims, seed, n_radial, target, alpha, sigma_f=1.0, eps_rel=1e-12):
    """Spectrum-matching loss L = mean over radial bins 1..R-1 with modes of
    (ln(P_b + eps) - ln(T_b + eps))^2, eps = eps_rel sigma_f^2, P the field's radial continuous
    spectrum and T the expected spectrum of the `target` filter, both binned by the library and
    the loss and its gradient computed by it (hu_spectrum_loss, hu_spectrum_grad); returns a scalar
    tensor differentiable in theta."""
    bins = (int(n_radial), 1)
    dev = theta.device if theta.is_cuda else torch.device("cuda")
    ts, tc = filter_spectrum(dims, target, bins, device=dev)
    return SpectrumLoss.apply(theta, dims, seed, bins, alpha, sigma_f, ts, tc, eps_rel * float(sigma_f) ** 2)