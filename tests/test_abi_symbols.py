"""The C-ABI library loads and exports every entry point include/mr.h declares;
argument validation that happens before any device work returns the
documented codes (no GPU needed: no call here reaches a kernel or a HIP
runtime call)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mr.h")
LIB = os.path.join(ROOT, "paper_2112_07537_amd", "libmr.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mr_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libmr.so not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_header_declares_the_hot_path():
    names = declared()
    for n in ("mr_grid_create", "mr_ghost", "mr_details", "mr_adapt", "mr_rk3_step"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    from paper_2112_07537_amd import mr
    src = open(mr.__file__).read()
    missing = [n for n in declared() if n not in src]
    assert not missing, missing


def test_validation_errors_without_device(lib):
    from paper_2112_07537_amd import mr
    lib.mr_grid_create.argtypes = [C.POINTER(mr.mr_config), C.c_void_p, C.c_void_p, C.c_size_t,
                                   C.POINTER(C.c_void_p)]
    lib.mr_grid_create.restype = C.c_int32
    lib.mr_last_error.restype = C.c_char_p
    h = C.c_void_p()
    bad = [dict(nb=12), dict(wavelet_N=3), dict(wavelet_Nt=1), dict(fd_order=1), dict(fd_order=7),
           dict(level_min=3, level_max=2), dict(prec=7), dict(n_fields=0), dict(exec_mode=5)]
    for over in bad:
        kw = dict(nb=16, wavelet_N=4, wavelet_Nt=2, fd_order=4, level_min=0, level_max=4, prec=0,
                  detail_ext=1, n_fields=1, exec_mode=0, eps_refine=1e-3, eps_coarsen=1e-5,
                  max_blocks=64)
        kw.update(over)
        c = mr.mr_config(**kw)
        assert lib.mr_grid_create(C.byref(c), None, None, 0, C.byref(h)) == mr.MR_EINVAL, over
        assert lib.mr_last_error()
        assert not h.value
    assert lib.mr_grid_create(None, None, None, 0, C.byref(h)) == mr.MR_EINVAL
    # a caller pool must be aligned and large enough (checked before any device call)
    ok = dict(nb=16, wavelet_N=4, wavelet_Nt=2, fd_order=4, level_min=0, level_max=4, prec=0,
              detail_ext=1, n_fields=1, exec_mode=0, eps_refine=1e-3, eps_coarsen=1e-5,
              max_blocks=64)
    c = mr.mr_config(**ok)
    lib.mr_pool_bytes.argtypes = [C.POINTER(mr.mr_config), C.POINTER(C.c_size_t)]
    lib.mr_pool_bytes.restype = C.c_int32
    need = C.c_size_t()
    assert lib.mr_pool_bytes(C.byref(c), C.byref(need)) == mr.MR_OK
    # fields, alternates and two work buffers of max_blocks blocks each
    assert need.value == 4 * 64 * 16 ** 3 * 8
    assert lib.mr_grid_create(C.byref(c), None, C.c_void_p(0x1000), need.value - 1,
                              C.byref(h)) == mr.MR_EINVAL
    assert lib.mr_grid_create(C.byref(c), None, C.c_void_p(0x1008), need.value,
                              C.byref(h)) == mr.MR_EINVAL
    assert not h.value
    # every entry point rejects a null grid handle
    for name, args in (("mr_ghost", (None, 0, 0)), ("mr_details", (None, 0, None, 1)),
                       ("mr_adapt", (None, 0, 0, None)), ("mr_sync", (None,)),
                       ("mr_tree_stats", (None, None)), ("mr_field_ptr", (None, 0, None))):
        f = getattr(lib, name)
        f.restype = C.c_int32
        assert f(*args) == mr.MR_EINVAL, name
    f = lib.mr_details_rk3_step
    f.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_void_p, C.c_int32]
    f.restype = C.c_int32
    assert f(None, 0, 0.1, None, None, 1) == mr.MR_EINVAL


def test_tuning_cache_format():
    """The autotuner's cache: keys (arch/nb/wavelet/fd/prec) map to knob sets
    of the mr_tuning fields within the accepted ranges."""
    from paper_2112_07537_amd import autotune as at
    from paper_2112_07537_amd import mr as m
    entries = at.load()
    for key, e in entries.items():
        arch, nb, w, fd, prec = key.split("/")
        assert arch.startswith("gfx") and nb.startswith("nb") and w.startswith("w")
        assert fd.startswith("fd") and prec in ("f32", "f64")
        assert set(e["knobs"]) == set(m.Grid.TUNING_KEYS)
        for k in ("lds_refine", "lds_restrict", "lds_subst"):
            assert 4096 <= e["knobs"][k] <= 65536
        assert e["knobs"]["subst_threads"] in (256, 512)
