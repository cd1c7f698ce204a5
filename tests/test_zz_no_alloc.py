"""The allocation-free force entry point (hslb_force_noalloc) through the C ABI
against hslb_force of an FP64 context initialised with the same fields: two
calls in a row on device arrays, the second on a smaller lattice, to the FP64
bar of the force readouts (1e-13 of the largest force).  The scratch array
keeps the first call's contents, so the second call also checks that nothing
stale is read."""
import numpy as np
import pytest
import torch

from paper_0712_2247_amd import hslb, workloads

pytestmark = pytest.mark.gpu


def _case(nx, ny, nz, sigma, walls, seed, with_u=True):
    nb = workloads.number_density(0.25, sigma)
    n, u = workloads.random_state((nz, ny, nx), nb, 0.05, 3e-3, seed=seed, solid_lo=walls, solid_hi=walls)
    p = hslb.make_params(nx, ny, nz, sigma, 0.9, accel=(1e-5, -2e-6, 0.0), wall_lo=walls, wall_hi=walls,
                         precision=hslb.HSLB_FP64)
    return p, n, (u if with_u else None)


def _noalloc(p, n, u):
    dev = torch.device("cuda:0")
    n_d = torch.from_numpy(np.ascontiguousarray(n).ravel()).to(dev)
    u_d = torch.from_numpy(np.ascontiguousarray(u).ravel()).to(dev) if u is not None else None
    F_d = torch.full((3 * n.size,), float("nan"), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    hslb.hslb_force_noalloc(p, n_d.data_ptr(), u_d.data_ptr() if u_d is not None else 0, F_d.data_ptr(),
                            stream.cuda_stream)
    stream.synchronize()
    return F_d.cpu().numpy().reshape((3,) + n.shape)


def _with_context(p, n, u):
    ctx = hslb.hslb_create(p)
    try:
        hslb.hslb_init(ctx, np.ascontiguousarray(n).ravel(),
                       None if u is None else np.ascontiguousarray(u).ravel())
        F = np.zeros(3 * n.size)
        hslb.hslb_force(ctx, F)
    finally:
        hslb.hslb_destroy(ctx)
    return F.reshape((3,) + n.shape)


def test_noalloc_force_matches_context_force_twice():
    for p, n, u in (_case(24, 20, 30, 8, 4, 11), _case(12, 13, 10, 3, 0, 12), _case(16, 12, 14, 5, 3, 13, False)):
        print(f"noalloc case {p.nx}x{p.ny}x{p.nz} sigma {p.sigma} walls {p.wall_lo}", flush=True)
        Fa = _noalloc(p, n, u)
        Fc = _with_context(p, n, u)
        scale = np.abs(Fc).max()
        assert scale > 0 and np.isfinite(Fa).all()
        err = np.abs(Fa - Fc).max() / scale
        print(f"noalloc: max error {err:.2e} of max |F| {scale:.3e}", flush=True)
        assert err <= 1e-13


def test_noalloc_rejects_what_does_not_fit():
    p, n, u = _case(24, 20, 30, 8, 4, 11)
    big = hslb.make_params(256, 256, 64, 8, 0.9, precision=hslb.HSLB_FP64)
    dev = torch.device("cuda:0")
    x = torch.zeros(3, dtype=torch.float64, device=dev)
    with pytest.raises(hslb.HslbError) as ei:
        hslb.hslb_force_noalloc(big, x.data_ptr(), 0, x.data_ptr(), 0)
    assert ei.value.code == hslb.HSLB_EINVAL and "scratch" in hslb.hslb_last_error(None)
    f32 = hslb.make_params(24, 20, 30, 8, 0.9, wall_lo=4, wall_hi=4, precision=hslb.HSLB_FP32)
    with pytest.raises(hslb.HslbError) as ei:
        hslb.hslb_force_noalloc(f32, x.data_ptr(), 0, x.data_ptr(), 0)
    assert ei.value.code == hslb.HSLB_EINVAL
