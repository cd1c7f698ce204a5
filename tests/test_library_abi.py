"""Host-side checks of libhslb.so that need no GPU: every entry point declared
in include/hslb.h is exported, the binding declares them all, and parameter
validation rejects bad input before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hslb.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hslb_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_0712_2247_amd import hslb
    if not os.path.exists(hslb.LIB_PATH):
        pytest.fail("libhslb.so is not built (run __graft_entry__.build())")
    return hslb


def test_header_declares_entry_points():
    names = _declared()
    assert "hslb_create" in names and "hslb_step" in names and "hslb_profiles" in names
    assert len(names) >= 19


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(lib.LIB_PATH)
    for name in _declared():
        assert hasattr(raw, name), name
    assert set(_declared()) <= set(lib.EXPORTS) | {"hslb_params"}


@pytest.mark.parametrize("bad", [
    dict(tau=0.5), dict(tau=0.4), dict(sigma=1), dict(sigma=9), dict(nx=5),
    dict(wall_lo=1, wall_hi=0), dict(wall_lo=10, wall_hi=10), dict(precision=7),
    dict(g2_model=3), dict(force_mode=5), dict(accel=(float("nan"), 0.0, 0.0)),
    dict(att_eps=1e-3, att_range=0.0), dict(att_eps=1e-3, att_range=10.5),
    dict(att_eps=float("inf"), att_range=2.0),
    # empty and degenerate grids, and grids beyond 32-bit node indices
    dict(nx=0), dict(ny=0), dict(nz=0), dict(nx=-4), dict(nz=3, wall_lo=2, wall_hi=2),
    dict(nx=1 << 20, ny=1 << 20), dict(tau=float("nan")), dict(tau=float("inf")),
])
def test_create_rejects_bad_parameters(lib, bad):
    kw = dict(nx=12, ny=12, nz=20, sigma=4, tau=1.0, wall_lo=2, wall_hi=2)
    kw.update(bad)
    p = lib.make_params(**kw)
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_create(p)
    assert ei.value.code == lib.HSLB_EINVAL
    assert lib.hslb_last_error(None)


@pytest.mark.parametrize("nx,ny,K,tol", [(48, 32, 50, 1e-3), (32, 30, 50, 1e-3), (32, 32, 0, 1e-3),
                                         (32, 32, 50, 0.0)])
def test_surrogate_geometry_and_judge_settings_are_validated(lib, nx, ny, K, tol):
    """The learned force needs nx % 32 == 0, ny % 4 == 0, K >= 1, tol > 0;
    rejected before any device work."""
    p = lib.make_params(nx, ny, 20, 4, 1.0, wall_lo=2, wall_hi=2, force_mode=lib.HSLB_FORCE_SURROGATE,
                        surr_check_every=K, surr_tol=tol)
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_create(p)
    assert ei.value.code == lib.HSLB_EINVAL


def test_attraction_is_rejected_with_the_learned_force_and_in_a_batch(lib):
    p = lib.make_params(32, 32, 20, 4, 1.0, wall_lo=2, wall_hi=2, force_mode=lib.HSLB_FORCE_SURROGATE,
                        att_eps=1e-3, att_range=2.0)
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_create(p)
    assert ei.value.code == lib.HSLB_EINVAL
    slits = [lib.make_params(16, 16, 24, 4, 1.0, wall_lo=2, wall_hi=2, precision=lib.HSLB_FP32,
                             att_eps=1e-3 * k, att_range=2.0) for k in range(2)]
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_batch_create(slits)
    assert ei.value.code == lib.HSLB_EINVAL


@pytest.mark.parametrize("bad", [
    dict(lattice=27),                                   # no such lattice
    dict(lattice=39, precision=1),                      # FP64 only
    dict(lattice=39, nz=6, wall_lo=2, wall_hi=2),       # 2 fluid layers: a link could cross both walls
    dict(lattice=39, nz=2, wall_lo=0, wall_hi=0, force_mode=2, nx=4, ny=4),
    dict(lattice=39, nx=32, ny=32, force_mode=1),       # no learned force
    dict(thermal=1),                                    # the thermal terms need 39 velocities
    dict(lattice=39, thermal=2),
])
def test_lattice_choice_is_validated(lib, bad):
    kw = dict(nx=12, ny=12, nz=20, sigma=4, tau=1.0, wall_lo=2, wall_hi=2)
    kw.update(bad)
    p = lib.make_params(**kw)
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_create(p)
    assert ei.value.code == lib.HSLB_EINVAL
    slits = [lib.make_params(16, 16, 24, 4, 1.0, wall_lo=2, wall_hi=2, lattice=39) for _ in range(2)]
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_batch_create(slits)
    assert ei.value.code == lib.HSLB_EINVAL


def test_trainer_and_network_op_arguments_are_validated(lib):
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_trainer_create(100, 1000)          # per-snapshot maximum above the capacity
    assert ei.value.code == lib.HSLB_EINVAL
    w = np.zeros(lib.HSLB_CNN_NWEIGHTS, dtype=np.float32)
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_cnn_op(lib.HSLB_CNN_FWD1, 30, 4, 4, True, w, np.zeros(480))   # nx % 32 != 0
    assert ei.value.code == lib.HSLB_EINVAL
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_cnn_op(lib.HSLB_CNN_DW2, 32, 4, 4, True, w, np.zeros(32 * 512))  # aux missing
    assert ei.value.code == lib.HSLB_EINVAL


def test_batch_arguments_are_validated(lib):
    """An empty batch, mixed storage precisions and an invalid slit among valid
    ones are rejected before any device work; the error names the slit."""
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_batch_create([])
    assert ei.value.code == lib.HSLB_EINVAL
    ok = lambda prec: lib.make_params(16, 16, 24, 4, 1.0, wall_lo=2, wall_hi=2, precision=prec)  # noqa: E731
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_batch_create([ok(lib.HSLB_FP32), ok(lib.HSLB_FP64)])
    assert ei.value.code == lib.HSLB_EINVAL and "mixed precisions" in str(ei.value)
    bad = lib.make_params(16, 16, 24, 4, 0.5, wall_lo=2, wall_hi=2, precision=lib.HSLB_FP32)
    with pytest.raises(lib.HslbError) as ei:
        lib.hslb_batch_create([ok(lib.HSLB_FP32), ok(lib.HSLB_FP32), bad])
    assert ei.value.code == lib.HSLB_EINVAL and "slit 2" in str(ei.value)
