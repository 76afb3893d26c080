"""Host-side checks of the C-ABI library (no GPU needed).

* libhufield.so loads and exports every function that include/hufield.h declares;
* workspace sizes follow the documented layout;
* argument validation returns the documented error codes before anything touches a GPU.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hufield.h")
# HUFIELD_LIB: another build of the same library (the host-sanitizer run of these tests)
LIB = os.environ.get("HUFIELD_LIB") or os.path.join(ROOT, "paper_2509_08675_amd", "libhufield.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhufield.so not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\**\s+\**(hu_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("hu_gen_field", "hu_threshold", "hu_power_spectrum", "hu_pipeline", "hu_workspace_size",
              "hu_strerror", "hu_debug_philox"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.fixture(scope="module")
def hf():
    from paper_2509_08675_amd import hufield
    return hufield


def test_strerror(hf):
    assert hf.strerror(0) == "ok"
    assert "workspace" in hf.strerror(hf.HU_ERR_WORKSPACE)


def test_workspace_sizes(hf):
    # 2D 2048^2 x 16: half spectrum 16 * 2048 * 1025 complex64, stored in column groups of four
    # (1025 -> 1028 columns), statistics, and the FP64 tile partials of the two spectra (room for
    # either tile width)
    n = hf.workspace_size(hf.HU_OP_PIPELINE, (2048, 2048), 16, (128, 36))
    spec = 16 * 2048 * 1028 * 8
    M = max(hf.debug_bin_tables((2048, 2048), (128, 36), v)["M"] for v in (0, 1))
    parts = 2 * 16 * M * 8
    assert spec + parts <= n < spec + parts + (1 << 20)
    m = hf.workspace_size(hf.HU_OP_POWER_SPECTRUM, (256, 256, 256), 4, (128, 1))
    assert m >= 4 * 256 * 256 * 129 * 8
    # batches above 64 fields are processed in chunks of 64 that reuse the workspace
    assert hf.workspace_size(hf.HU_OP_PIPELINE, (64, 64), 200, (8, 1)) == \
        hf.workspace_size(hf.HU_OP_PIPELINE, (64, 64), 64, (8, 1))


# the largest accepted grids: each side at most 2048 (2^k) or 768 (3 * 2^k), and one field's FP32
# half spectrum below 4 GiB (the passes address it with unsigned 32-bit byte offsets): 768 x 1024^2
# (3.2 GB) passes, 1024^3 and 2048 x 1024 x 512 (4.3 GB) do not
@pytest.mark.parametrize("dims,code", [((100, 128), -2), ((4096, 64), -2), ((64, 2), -2), ((64,), -1),
                                       ((8, 8, 8, 8), -1), ((1536, 64), -2), ((64, 96), 0), ((768, 12), 0),
                                       ((2048, 2048), 0), ((768, 1024, 1024), 0), ((1024, 1024, 768), 0),
                                       ((1024, 1024, 1024), -2), ((2048, 1024, 512), -2), ((4, 4), 0)])
def test_size_validation(hf, dims, code):
    out = ctypes.c_size_t()
    d = hf.hu_dims()
    d.ndim = len(dims)
    for i, n in enumerate(dims[:3]):
        d.n[i] = n
    rc = hf.lib_handle().hu_workspace_size(hf.HU_OP_PIPELINE, d, 1, None, ctypes.byref(out))
    assert rc == code


def test_argument_errors_before_any_launch(hf):
    lib = hf.lib_handle()
    d = hf.make_dims((64, 64))
    seeds = (ctypes.c_uint64 * 1)(1)
    good = hf.make_filter(dict(p=2, semi=(1, 1, 1), rot=0, alpha=2, k0=0.2, width=0.05))
    fake = ctypes.c_void_p(1 << 20)           # never dereferenced: validation fails first
    for bad in (dict(p=0.0), dict(alpha=-2.0), dict(width=0.0), dict(k0=-0.1), dict(sigma_f=float("nan"))):
        f = hf.make_filter({**dict(p=2, semi=(1, 1, 1), rot=0, alpha=2, k0=0.2, width=0.05), **bad})
        rc = lib.hu_gen_field(d, 1, ctypes.byref(f), seeds, fake, None, None, None, None, fake, 1 << 30, None)
        assert rc == hf.HU_ERR_ARG
    # workspace too small
    rc = lib.hu_gen_field(d, 1, ctypes.byref(good), seeds, fake, None, None, None, None, fake, 16, None)
    assert rc == hf.HU_ERR_WORKSPACE
    # misaligned field pointer
    rc = lib.hu_gen_field(d, 1, ctypes.byref(good), seeds, ctypes.c_void_p((1 << 20) + 4), None, None, None, None,
                          fake, 1 << 30, None)
    assert rc == hf.HU_ERR_ALIGN
    # angular bins are 2D only
    b = hf.make_bins((16, 4))
    rc = lib.hu_power_spectrum(hf.make_dims((8, 8, 8)), 1, fake, hf.HU_F32, b, fake, None, fake, 1 << 30, None)
    assert rc == hf.HU_ERR_ARG
    rc = lib.hu_power_spectrum(d, 1, fake, 7, hf.make_bins((16, 1)), fake, None, fake, 1 << 30, None)
    assert rc == hf.HU_ERR_ARG
    # zero batch, null seeds
    rc = lib.hu_gen_field(d, 0, ctypes.byref(good), seeds, fake, None, None, None, None, fake, 1 << 30, None)
    assert rc == hf.HU_ERR_ARG
    rc = lib.hu_gen_field(d, 1, ctypes.byref(good), None, fake, None, None, None, None, fake, 1 << 30, None)
    assert rc == hf.HU_ERR_ARG


def test_tabulated_radial_form_argument_errors(hf):
    lib = hf._lib
    d = hf.make_dims((16, 16))
    seeds = (ctypes.c_uint64 * 1)(1)
    fake = ctypes.c_void_p(1 << 20)           # never dereferenced: validation fails first
    # the C struct: ten doubles, a pointer, an int32 (padded to 8) and a double
    assert ctypes.sizeof(hf.hu_filter) == 104

    def with_prof(**kw):
        f = hf.make_filter(dict(p=2, semi=(1, 1, 1), rot=0.3, alpha=2, k0=0.2, width=0.05))
        f.prof, f.prof_n, f.prof_dk = 1 << 20, 64, 0.05
        for k, v in kw.items():
            setattr(f, k, v)
        return f

    for f, code in ((with_prof(prof_n=1), hf.HU_ERR_ARG), (with_prof(prof=None), hf.HU_ERR_ARG),
                    (with_prof(prof_dk=0.0), hf.HU_ERR_ARG), (with_prof(prof_dk=float("inf")), hf.HU_ERR_ARG),
                    (with_prof(prof=(1 << 20) + 2), hf.HU_ERR_ALIGN), (with_prof(offset=1e-3), hf.HU_ERR_UNSUPPORTED)):
        rc = lib.hu_gen_field(d, 1, ctypes.byref(f), seeds, fake, None, None, None, None, fake, 1 << 30, None)
        assert rc == code, (rc, code)
    # the adjoint differentiates Eq. (13) only
    rc = lib.hu_spectrum_grad(d, ctypes.byref(with_prof()), 1, hf.make_bins((16, 1)), fake, fake, fake, fake, fake,
                              fake, 1 << 30, None)
    assert rc == hf.HU_ERR_UNSUPPORTED


def test_window_variance_argument_errors_and_workspace(hf):
    lib = hf.lib_handle()
    d = hf.make_dims((64, 64))
    fake = ctypes.c_void_p(1 << 20)
    radii = (ctypes.c_double * 3)(0.0, 2.0, 5.0)
    assert lib.hu_window_variance(d, 1, fake, hf.HU_F32, radii, 0, fake, fake, 1 << 30, None) == hf.HU_ERR_ARG
    assert lib.hu_window_variance(d, 1, fake, hf.HU_F32, radii, hf.HU_MAX_RADII + 1, fake, fake, 1 << 30,
                                  None) == hf.HU_ERR_ARG
    bad = (ctypes.c_double * 2)(1.0, -0.5)
    assert lib.hu_window_variance(d, 1, fake, hf.HU_F32, bad, 2, fake, fake, 1 << 30, None) == hf.HU_ERR_ARG
    nan = (ctypes.c_double * 1)(float("nan"))
    assert lib.hu_window_variance(d, 1, fake, hf.HU_F32, nan, 1, fake, fake, 1 << 30, None) == hf.HU_ERR_ARG
    assert lib.hu_window_variance(d, 1, fake, 9, radii, 3, fake, fake, 1 << 30, None) == hf.HU_ERR_ARG
    assert lib.hu_window_variance(d, 1, ctypes.c_void_p((1 << 20) + 4), hf.HU_F32, radii, 3, fake, fake, 1 << 30,
                                  None) == hf.HU_ERR_ALIGN
    assert lib.hu_window_variance(d, 1, fake, hf.HU_F32, radii, 3, fake, fake, 64, None) == hf.HU_ERR_WORKSPACE
    # workspace: the half spectrum of each field of a chunk, then tiles x HU_MAX_RADII partials per field
    n = hf.workspace_size(hf.HU_OP_WINDOW_VARIANCE, (256, 256, 256), 4)
    assert n >= 4 * 256 * 256 * 129 * 8 + 4 * (256 * 129 // 32) * hf.HU_MAX_RADII * 8


def test_small_k_exponent_matches_oracle(hf):
    import numpy as np
    from oracle import diagnostics as D
    rng = np.random.default_rng(3)
    for bins, nfit in (((64, 1), 10), ((32, 6), 7)):
        nb = bins[0] * bins[1] + 1
        cnt = rng.integers(1, 50, nb).astype(np.uint64)
        cnt[3] = 0                                   # an empty bin is skipped by both
        s = rng.uniform(0.5, 2.0, nb) * cnt
        got = hf.small_k_exponent(s, cnt, bins, nfit)
        ref = D.small_k_exponent(s, cnt.astype(float), bins[0], nfit, n_angular=bins[1])
        assert got == pytest.approx(ref, rel=1e-12, abs=1e-12)
    with pytest.raises(hf.HuError):
        hf.small_k_exponent(np.ones(65), np.zeros(65, np.uint64), (64, 1), 10)


def test_class_table_matches_oracle(hf):
    from oracle import diagnostics as D
    for alpha, d in ((3.0, 2), (1.0, 3), (1.0 + 1e-9, 2), (0.4, 3), (0.0, 2), (-1.5, 2), (-2.5, 2), (-2.5, 3)):
        assert hf.hyperuniformity_class(alpha, d) == D.CLASSES[D.hyperuniformity_class(alpha, d)]


def test_level_threshold_matches_oracle(hf):
    from oracle import twopoint as TP
    for phi in (0.5, 0.3, 0.05, 0.9, 1e-6, 1.0 - 1e-9, 0.999):
        for sf in (1.0, 2.5):
            t = hf.level_threshold(phi, sf)
            ref = TP.level_threshold(phi, sf)
            assert t == pytest.approx(ref, rel=1e-12, abs=1e-13)
    for bad in ((0.0, 1.0), (1.0, 1.0), (0.5, 0.0), (float("nan"), 1.0), (0.5, -1.0)):
        with pytest.raises(hf.HuError):
            hf.level_threshold(*bad)


def test_level_cut_and_two_point_argument_errors(hf):
    lib = hf.lib_handle()
    d = hf.make_dims((64, 64))
    fake = ctypes.c_void_p(1 << 20)
    assert lib.hu_level_cut(d, 1, fake, 0.0, 1.0, fake, None, 0.0, None) == hf.HU_ERR_ARG
    assert lib.hu_level_cut(d, 1, fake, 0.5, 0.0, fake, None, 0.0, None) == hf.HU_ERR_ARG
    assert lib.hu_level_cut(d, 1, fake, 0.5, 1.0, fake, None, -1.0, None) == hf.HU_ERR_ARG
    assert lib.hu_level_cut(d, 0, fake, 0.5, 1.0, fake, None, 0.0, None) == hf.HU_ERR_ARG
    assert lib.hu_level_cut(d, 1, ctypes.c_void_p((1 << 20) + 2), 0.5, 1.0, fake, None, 0.0,
                            None) == hf.HU_ERR_ALIGN
    assert lib.hu_two_point(d, 1, fake, fake, fake, 64, None) == hf.HU_ERR_WORKSPACE
    assert lib.hu_two_point(d, 1, None, fake, fake, 1 << 30, None) == hf.HU_ERR_ARG
    assert lib.hu_two_point(d, 1, ctypes.c_void_p((1 << 20) + 8), fake, fake, 1 << 30, None) == hf.HU_ERR_ALIGN
    n = hf.workspace_size(hf.HU_OP_TWO_POINT, (256, 256, 256), 4)
    assert n >= 4 * 256 * 256 * 129 * 8


def test_pipeline_noalloc_refusals_on_the_host(hf):
    """The allocation-free entry point refuses, before any launch, a shape whose workspace
    exceeds its fixed array and a shape whose per-size tables were never built."""
    lib = hf.lib_handle()
    fake = ctypes.c_void_p(1 << 20)
    o = hf.hu_outputs()
    o.field = fake
    filt = hf.make_filter(__import__("paper_2509_08675_amd.workloads", fromlist=["C2"]).C2["filt"])
    seeds = (ctypes.c_uint64 * 9)(*range(9))
    big = hf.make_dims((2048, 2048))
    assert hf.workspace_size(hf.HU_OP_PIPELINE, (2048, 2048), 9, (16, 1)) > hf.HU_NOALLOC_WORK_BYTES
    assert hf.workspace_size(hf.HU_OP_PIPELINE, (2048, 2048), 7, (16, 1)) <= hf.HU_NOALLOC_WORK_BYTES
    assert lib.hu_pipeline_noalloc(big, 9, ctypes.byref(filt), seeds, hf.make_bins((16, 1)), 1e-5,
                                   ctypes.byref(o), None) == hf.HU_ERR_WORKSPACE
    assert lib.hu_pipeline_noalloc(hf.make_dims((24, 48)), 1, ctypes.byref(filt), seeds, hf.make_bins((11, 3)),
                                   1e-5, ctypes.byref(o), None) == hf.HU_ERR_TABLES
    assert lib.hu_pipeline_noalloc(hf.make_dims((24, 48)), 1, ctypes.byref(filt), seeds, hf.make_bins((11, 3)),
                                   1e-5, None, None) == hf.HU_ERR_ARG
    assert lib.hu_pipeline_noalloc(hf.make_dims((24, 50)), 1, ctypes.byref(filt), seeds, hf.make_bins((11, 3)),
                                   1e-5, ctypes.byref(o), None) == hf.HU_ERR_SIZE
    assert "tables" in hf.strerror(hf.HU_ERR_TABLES)


def test_spectrum_loss_validation(hf):
    """The loss entry point checks its arguments on the host before any launch."""
    lib = hf.lib_handle()
    p = ctypes.c_void_p(1 << 20)
    odd = ctypes.c_void_p((1 << 20) + 4)
    b = hf.make_bins((16, 1))
    assert lib.hu_spectrum_loss(b, None, p, p, p, 1e-12, p, p, None) == hf.HU_ERR_ARG
    assert lib.hu_spectrum_loss(b, p, p, p, p, -1.0, p, p, None) == hf.HU_ERR_ARG
    assert lib.hu_spectrum_loss(b, p, p, p, p, float("nan"), p, p, None) == hf.HU_ERR_ARG
    assert lib.hu_spectrum_loss(hf.make_bins((0, 1)), p, p, p, p, 1e-12, p, p, None) == hf.HU_ERR_ARG
    assert lib.hu_spectrum_loss(b, odd, p, p, p, 1e-12, p, p, None) == hf.HU_ERR_ALIGN
