"""The C ABI: libmhfd.so loads on a machine without a GPU and exports every
function include/mhfd.h declares; host-side argument checks return status
codes without touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mhfd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mhfd_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    from paper_2108_12050_amd import _lib
    assert declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2108_12050_amd import _lib
    L = _lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings():
    from paper_2108_12050_amd import _lib
    L = _lib.load()
    for code in range(6):
        assert L.mhfd_status_string(code)
    assert L.mhfd_status_string(99) == b"unknown status"


@pytest.mark.parametrize("bad", [dict(n_scales=0), dict(n_scales=33), dict(truncate=0.0),
                                 dict(overlap=-1.0), dict(polarity=5), dict(in_dtype=7),
                                 dict(max_h=0), dict(sigma_min=-1.0), dict(sigma_cap=-1.0),
                                 dict(sigma_cap=9.5), dict(sigma_cap=float("nan"))])
def test_create_plan_rejects_bad_config_on_host(bad):
    """Validation happens before any device call, so it runs without a GPU."""
    from paper_2108_12050_amd import _lib
    L = _lib.load()
    cfg = _lib.Config(n_scales=10, sigma_min=1.0, sigma_max=10.0, truncate=4.0, threshold=0.1,
                      overlap=0.5, polarity=0, in_dtype=0, max_h=64, max_w=64, max_candidates=0)
    for k, v in bad.items():
        setattr(cfg, k, v)
    h = C.c_void_p()
    assert L.mhfd_create_plan(C.byref(cfg), C.byref(h)) == 1
    assert L.mhfd_last_error()
    assert h.value is None


def test_sigma_cap_beyond_the_largest_radius_is_unsupported():
    from paper_2108_12050_amd import _lib
    L = _lib.load()
    cfg = _lib.Config(n_scales=10, sigma_min=1.0, sigma_max=10.0, truncate=4.0, threshold=0.1,
                      overlap=0.5, polarity=0, in_dtype=0, max_h=64, max_w=64, max_candidates=0,
                      sigma_cap=16.2)   # radius 65 > MHFD_MAX_RADIUS
    h = C.c_void_p()
    assert L.mhfd_create_plan(C.byref(cfg), C.byref(h)) == 2
    assert b"sigma_cap" in L.mhfd_last_error()


def test_null_arguments():
    from paper_2108_12050_amd import _lib
    L = _lib.load()
    assert L.mhfd_create_plan(None, None) == 1
    assert L.mhfd_destroy_plan(None) == 0
    assert L.mhfd_plan_scales(None, None, None) == -1
    assert L.mhfd_detect_workspace_size(None, 10, 10) == 0
    assert L.mhfd_detect(None, None, 1, 1, 1, None, 0, None, None, None, 0, None) == 1
    assert L.mhfd_log_stack(None, None, 1, 1, 1, None, None, 0, None) == 1
    assert L.mhfd_log_stack_workspace_size(None, 1, 1) == 0


@pytest.mark.parametrize("bad,status", [(dict(stretch=2), 1), (dict(criterion=2), 1),
                                        (dict(stretch=1), 2),                 # fp32 plan
                                        (dict(stretch=1, in_dtype=1, sigma_max=15.0), 2)])
def test_stretch_plan_checks_on_host(bad, status):
    """The histogram stretch takes 8-bit plans whose radii all use the
    matrix-core path (sigma 15 -> radius 60 > 56); checked before any device
    call."""
    from paper_2108_12050_amd import _lib
    L = _lib.load()
    cfg = _lib.Config(n_scales=10, sigma_min=1.0, sigma_max=10.0, truncate=4.0, threshold=0.1,
                      overlap=0.5, polarity=0, in_dtype=0, max_h=64, max_w=64, max_candidates=0)
    for k, v in bad.items():
        setattr(cfg, k, v)
    h = C.c_void_p()
    assert L.mhfd_create_plan(C.byref(cfg), C.byref(h)) == status
    assert L.mhfd_last_error()
    assert h.value is None


def test_stretch_levels_argument_checks():
    from paper_2108_12050_amd import _lib
    L = _lib.load()
    buf = (C.c_int32 * 258)()
    p = C.cast(buf, C.c_void_p)
    assert L.mhfd_stretch_levels(None, 4, 4, 4, p, p, None) == 1
    assert L.mhfd_stretch_levels(p, 0, 4, 4, p, p, None) == 1
    assert L.mhfd_stretch_levels(p, 4, 4, 3, p, p, None) == 1      # pitch < w
    assert L.mhfd_stretch_levels(p, 4, 4, 4, None, p, None) == 1
    assert L.mhfd_stretch_levels(p, 65536, 65536, 65536, p, p, None) == 2  # >= 2^31 pixels


@pytest.mark.parametrize("bad,status", [(dict(criterion=1), 2),                 # overlap 0.5
                                        (dict(criterion=1, overlap=1.0, n_scales=1), 1),
                                        (dict(criterion=1, overlap=1.0, sigma_max=15.0), 2)])
def test_dog_plan_checks_on_host(bad, status):
    """The paper's DoG criterion has no pruning (overlap >= 1), needs two
    scales and every radius on the matrix-core path."""
    from paper_2108_12050_amd import _lib
    L = _lib.load()
    cfg = _lib.Config(n_scales=10, sigma_min=1.0, sigma_max=10.0, truncate=4.0, threshold=0.1,
                      overlap=0.5, polarity=0, in_dtype=0, max_h=64, max_w=64, max_candidates=0)
    for k, v in bad.items():
        setattr(cfg, k, v)
    h = C.c_void_p()
    assert L.mhfd_create_plan(C.byref(cfg), C.byref(h)) == status
    assert h.value is None
