"""Python binding of libhslb.so: the C ABI of include/hslb.h under the same
names, plus a small ``Sim`` wrapper that owns one context.  Argument
marshalling only: every step of the method runs in the library's HIP kernels.

Importing works without a GPU; loading the library needs the built
``libhslb.so`` (``python -m paper_0712_2247_amd.build``) and fails loudly
without it -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhslb.so")

HSLB_OK = 0
HSLB_EINVAL = -1
HSLB_ENOMEM = -2
HSLB_EDEVICE = -3
HSLB_EUNSTABLE = -4
HSLB_ESTATE = -5
HSLB_ENOSURR = -6

HSLB_FP64 = 0
HSLB_FP32 = 1
HSLB_G2_PAPER = 0
HSLB_G2_CS = 1
HSLB_FORCE_EXACT = 0
HSLB_FORCE_SURROGATE = 1
HSLB_FORCE_OFF = 2
HSLB_D3Q19 = 0
HSLB_D3Q39 = 39
HSLB_SURR_CORRECTED = 0
HSLB_SURR_PLAIN = 1
HSLB_SURR_FROZEN = 2
HSLB_CNN_NWEIGHTS = 144067
(HSLB_CNN_FWD1, HSLB_CNN_FWD2, HSLB_CNN_FWD3, HSLB_CNN_DX3, HSLB_CNN_DX2, HSLB_CNN_DW1,
 HSLB_CNN_DW2, HSLB_CNN_DW3) = range(8)

# Every exported entry point of include/hslb.h.
EXPORTS = (
    "hslb_create", "hslb_destroy", "hslb_last_error", "hslb_set_stream", "hslb_init",
    "hslb_init_thermal", "hslb_thermal_fields",
    "hslb_step", "hslb_sync", "hslb_prepare", "hslb_step_count", "hslb_moments", "hslb_profiles",
    "hslb_force", "hslb_eta_bar", "hslb_attraction_potential", "hslb_set_solid", "hslb_get_populations",
    "hslb_set_populations",
    "hslb_set_watchdog", "hslb_set_shift_period", "hslb_set_graph",
    "hslb_checkpoint_size", "hslb_checkpoint_save", "hslb_checkpoint_load", "hslb_set_kernel_timing", "hslb_kernel_times",
    "hslb_get_timings", "hslb_copy_bandwidth", "hslb_set_collide_tiles",
    "hslb_batch_create", "hslb_batch_init", "hslb_batch_profiles", "hslb_batch_finite",
    "hslb_batch_set_config", "hslb_batch_set_launch", "hslb_batch_get_launch", "hslb_batch_autotune",
    "hslb_surrogate_set_weights", "hslb_surrogate_get_weights", "hslb_surrogate_set_mode",
    "hslb_surrogate_set_components",
    "hslb_surrogate_stats", "hslb_surrogate_force", "hslb_surrogate_save_snapshot", "hslb_surrogate_train",
    "hslb_trainer_create", "hslb_trainer_destroy", "hslb_trainer_last_error",
    "hslb_trainer_add_snapshot", "hslb_trainer_add_snapshot_host", "hslb_trainer_count",
    "hslb_trainer_set_weights", "hslb_trainer_get_weights", "hslb_trainer_eval",
    "hslb_trainer_grad", "hslb_trainer_step", "hslb_trainer_train", "hslb_cnn_op", "hslb_force_noalloc",
)


class hslb_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("wall_lo", ctypes.c_int32), ("wall_hi", ctypes.c_int32),
        ("sigma", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("accel", ctypes.c_double * 3),
        ("g2_model", ctypes.c_int32), ("wall_reg", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("force_mode", ctypes.c_int32),
        ("surr_check_every", ctypes.c_int32),
        ("surr_tol", ctypes.c_double),
        ("att_eps", ctypes.c_double), ("att_range", ctypes.c_double),
        ("lattice", ctypes.c_int32), ("thermal", ctypes.c_int32),
    ]


class HslbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hslb error {code}: {msg}")
        self.code = code


_lib = None
_P = ctypes.POINTER
_dp = _P(ctypes.c_double)
_fp = _P(ctypes.c_float)
_vp = ctypes.c_void_p


def load(path: Optional[str] = None):
    """Load libhslb.so once and declare every signature."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_0712_2247_amd.build` "
                          "(there is no non-GPU fallback)")
    lib = ctypes.CDLL(path)
    sig = {
        "hslb_create": (ctypes.c_int, [_P(hslb_params), _P(_vp)]),
        "hslb_destroy": (None, [_vp]),
        "hslb_last_error": (ctypes.c_char_p, [_vp]),
        "hslb_set_stream": (ctypes.c_int, [_vp, _vp]),
        "hslb_init": (ctypes.c_int, [_vp, _dp, _dp]),
        "hslb_init_thermal": (ctypes.c_int, [_vp, _dp, _dp, _dp]),
        "hslb_thermal_fields": (ctypes.c_int, [_vp, _dp, _dp]),
        "hslb_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
        "hslb_sync": (ctypes.c_int, [_vp]),
        "hslb_prepare": (ctypes.c_int, [_vp]),
        "hslb_step_count": (ctypes.c_int, [_vp, _P(ctypes.c_int64)]),
        "hslb_moments": (ctypes.c_int, [_vp, _dp, _dp]),
        "hslb_profiles": (ctypes.c_int, [_vp, _dp, _dp]),
        "hslb_force": (ctypes.c_int, [_vp, _dp]),
        "hslb_eta_bar": (ctypes.c_int, [_vp, _dp]),
        "hslb_attraction_potential": (ctypes.c_int, [_vp, _dp]),
        "hslb_set_solid": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_uint8)]),
        "hslb_get_populations": (ctypes.c_int, [_vp, _dp]),
        "hslb_set_populations": (ctypes.c_int, [_vp, _dp]),
        "hslb_set_watchdog": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_double]),
        "hslb_set_shift_period": (ctypes.c_int, [_vp, ctypes.c_int64]),
        "hslb_checkpoint_size": (ctypes.c_int, [_vp, _P(ctypes.c_int64)]),
        "hslb_checkpoint_save": (ctypes.c_int, [_vp, ctypes.c_void_p]),
        "hslb_checkpoint_load": (ctypes.c_int, [_vp, ctypes.c_void_p]),
        "hslb_set_graph": (ctypes.c_int, [_vp, ctypes.c_int32]),
        "hslb_set_collide_tiles": (ctypes.c_int, [_vp, ctypes.c_int32]),
        "hslb_set_kernel_timing": (ctypes.c_int, [_vp, ctypes.c_int32]),
        "hslb_kernel_times": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_void_p, _dp,
                                             _P(ctypes.c_int64), _P(ctypes.c_int32)]),
        "hslb_get_timings": (ctypes.c_int, [_vp, _dp, _dp]),
        "hslb_copy_bandwidth": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, _dp]),
        "hslb_force_noalloc": (ctypes.c_int, [_P(hslb_params), _vp, _vp, _vp, _vp]),
        "hslb_batch_create": (ctypes.c_int, [_P(hslb_params), ctypes.c_int32, _P(_vp)]),
        "hslb_batch_init": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp]),
        "hslb_batch_profiles": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp]),
        "hslb_batch_finite": (ctypes.c_int, [_vp, _P(ctypes.c_int32)]),
        "hslb_batch_set_config": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
        "hslb_batch_set_launch": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
        "hslb_batch_get_launch": (ctypes.c_int, [_vp, _P(ctypes.c_int32), _P(ctypes.c_int32), _P(ctypes.c_int32)]),
        "hslb_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_int32), _dp,
                                               ctypes.c_int32]),
        "hslb_surrogate_set_weights": (ctypes.c_int, [_vp, _fp, ctypes.c_int64]),
        "hslb_surrogate_get_weights": (ctypes.c_int, [_vp, _fp, ctypes.c_int64]),
        "hslb_surrogate_set_mode": (ctypes.c_int, [_vp, ctypes.c_int32]),
        "hslb_surrogate_set_components": (ctypes.c_int, [_vp, ctypes.c_int32]),
        "hslb_surrogate_stats": (ctypes.c_int, [_vp, _P(ctypes.c_int64), _P(ctypes.c_int64), _dp, _dp]),
        "hslb_surrogate_force": (ctypes.c_int, [_vp, _dp]),
        "hslb_surrogate_save_snapshot": (ctypes.c_int, [_vp, ctypes.c_char_p]),
        "hslb_surrogate_train": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_int32, ctypes.c_double, _dp]),
        "hslb_trainer_create": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64, _P(_vp)]),
        "hslb_trainer_destroy": (None, [_vp]),
        "hslb_trainer_last_error": (ctypes.c_char_p, [_vp]),
        "hslb_trainer_add_snapshot": (ctypes.c_int, [_vp, _vp, _P(ctypes.c_int32)]),
        "hslb_trainer_add_snapshot_host": (ctypes.c_int, [_vp] + [ctypes.c_int32] * 5 +
                                           [_dp, _dp, _P(ctypes.c_int32)]),
        "hslb_trainer_count": (ctypes.c_int, [_vp, _P(ctypes.c_int32)]),
        "hslb_trainer_set_weights": (ctypes.c_int, [_vp, _fp, ctypes.c_int64]),
        "hslb_trainer_get_weights": (ctypes.c_int, [_vp, _fp, ctypes.c_int64]),
        "hslb_trainer_eval": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _fp]),
        "hslb_trainer_grad": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _fp]),
        "hslb_trainer_step": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_double, _dp]),
        "hslb_trainer_train": (ctypes.c_int, [_vp, _P(ctypes.c_int32), ctypes.c_int32, ctypes.c_double, _dp]),
        "hslb_cnn_op": (ctypes.c_int, [ctypes.c_int32] * 5 + [_fp, _fp, _fp, _fp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _d(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_dp)


def _f(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_fp)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _chk(ctx, rc: int):
    if rc != HSLB_OK:
        raise HslbError(rc, load().hslb_last_error(ctx).decode())


# ----------------------------------------------------------- C-ABI mirror


def hslb_create(params: hslb_params):
    lib = load()
    ctx = _vp()
    rc = lib.hslb_create(ctypes.byref(params), ctypes.byref(ctx))
    if rc != HSLB_OK:
        raise HslbError(rc, lib.hslb_last_error(None).decode())
    return ctx


def hslb_destroy(ctx):
    load().hslb_destroy(ctx)


def hslb_last_error(ctx) -> str:
    return load().hslb_last_error(ctx).decode()


def hslb_set_stream(ctx, stream_handle: int):
    _chk(ctx, load().hslb_set_stream(ctx, _vp(stream_handle)))


def hslb_init(ctx, n: np.ndarray, u: Optional[np.ndarray]):
    _chk(ctx, load().hslb_init(ctx, _d(n), _d(u)))


def hslb_init_thermal(ctx, n: np.ndarray, u: Optional[np.ndarray], T: Optional[np.ndarray]):
    _chk(ctx, load().hslb_init_thermal(ctx, _d(n), _d(u), _d(T)))


def hslb_thermal_fields(ctx, T: Optional[np.ndarray], Q: Optional[np.ndarray]):
    _chk(ctx, load().hslb_thermal_fields(ctx, _d(T), _d(Q)))


def hslb_step(ctx, nsteps: int):
    _chk(ctx, load().hslb_step(ctx, int(nsteps)))


def hslb_sync(ctx):
    _chk(ctx, load().hslb_sync(ctx))


def hslb_prepare(ctx):
    _chk(ctx, load().hslb_prepare(ctx))


def hslb_step_count(ctx) -> int:
    v = ctypes.c_int64()
    _chk(ctx, load().hslb_step_count(ctx, ctypes.byref(v)))
    return v.value


def hslb_moments(ctx, n: Optional[np.ndarray], u: Optional[np.ndarray]):
    _chk(ctx, load().hslb_moments(ctx, _d(n), _d(u)))


def hslb_profiles(ctx, n_z: Optional[np.ndarray], u_z: Optional[np.ndarray]):
    _chk(ctx, load().hslb_profiles(ctx, _d(n_z), _d(u_z)))


def hslb_force(ctx, F: np.ndarray):
    _chk(ctx, load().hslb_force(ctx, _d(F)))


def hslb_eta_bar(ctx, eb: np.ndarray):
    _chk(ctx, load().hslb_eta_bar(ctx, _d(eb)))


def hslb_attraction_potential(ctx, phi: np.ndarray):
    _chk(ctx, load().hslb_attraction_potential(ctx, _d(phi)))


def hslb_set_solid(ctx, solid: np.ndarray):
    m = np.ascontiguousarray(np.asarray(solid) != 0, dtype=np.uint8)
    _chk(ctx, load().hslb_set_solid(ctx, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))


def hslb_get_populations(ctx, f: np.ndarray):
    _chk(ctx, load().hslb_get_populations(ctx, _d(f)))


def hslb_set_populations(ctx, f: np.ndarray):
    _chk(ctx, load().hslb_set_populations(ctx, _d(f)))


def hslb_set_watchdog(ctx, every: int, tol: float):
    _chk(ctx, load().hslb_set_watchdog(ctx, int(every), float(tol)))


def hslb_checkpoint_save(ctx) -> bytes:
    n = ctypes.c_int64()
    _chk(ctx, load().hslb_checkpoint_size(ctx, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _chk(ctx, load().hslb_checkpoint_save(ctx, buf))
    return buf.raw


def hslb_checkpoint_load(ctx, data: bytes):
    buf = ctypes.create_string_buffer(data, len(data))
    _chk(ctx, load().hslb_checkpoint_load(ctx, buf))


def hslb_set_shift_period(ctx, every: int):
    _chk(ctx, load().hslb_set_shift_period(ctx, int(every)))


def hslb_set_graph(ctx, enable: bool):
    _chk(ctx, load().hslb_set_graph(ctx, int(bool(enable))))


def hslb_set_collide_tiles(ctx, enable: bool):
    _chk(ctx, load().hslb_set_collide_tiles(ctx, int(bool(enable))))


def hslb_set_kernel_timing(ctx, enable: bool):
    _chk(ctx, load().hslb_set_kernel_timing(ctx, int(bool(enable))))


def hslb_kernel_times(ctx, cap: int = 32):
    names = (ctypes.c_char * 32 * cap)()
    ms = np.zeros(cap)
    cnt = np.zeros(cap, dtype=np.int64)
    count = ctypes.c_int32()
    _chk(ctx, load().hslb_kernel_times(ctx, cap, ctypes.cast(names, ctypes.c_void_p), _d(ms),
                                       cnt.ctypes.data_as(_P(ctypes.c_int64)),
                                       ctypes.byref(count)))
    out = {}
    for k in range(min(count.value, cap)):
        out[bytes(names[k]).split(b"\0", 1)[0].decode()] = (float(ms[k]), int(cnt[k]))
    return out


def hslb_get_timings(ctx):
    ms = ctypes.c_double()
    ml = ctypes.c_double()
    _chk(ctx, load().hslb_get_timings(ctx, ctypes.byref(ms), ctypes.byref(ml)))
    return ms.value, ml.value


def hslb_copy_bandwidth(nbytes: int, iters: int) -> float:
    v = ctypes.c_double()
    rc = load().hslb_copy_bandwidth(int(nbytes), int(iters), ctypes.byref(v))
    if rc != HSLB_OK:
        raise HslbError(rc, load().hslb_last_error(None).decode())
    return v.value


HSLB_FORCE_NOALLOC_BYTES = 64 << 20


def hslb_force_noalloc(params: hslb_params, n_dev: int, u_dev: Optional[int], F_dev: int, stream: int = 0):
    """The allocation-free force on device arrays given by address (FP64:
    n[N], u[3][N] or None, F[3][N]); queued on `stream` without a wait."""
    rc = load().hslb_force_noalloc(ctypes.byref(params), _vp(n_dev), _vp(u_dev) if u_dev else None, _vp(F_dev),
                                   _vp(stream) if stream else None)
    if rc != HSLB_OK:
        raise HslbError(rc, load().hslb_last_error(None).decode())


def hslb_batch_create(slits) -> ctypes.c_void_p:
    lib = load()
    arr = (hslb_params * len(slits))(*slits)
    ctx = _vp()
    rc = lib.hslb_batch_create(arr, len(slits), ctypes.byref(ctx))
    if rc != HSLB_OK:
        raise HslbError(rc, lib.hslb_last_error(None).decode())
    return ctx


def hslb_batch_init(ctx, slit: int, n: np.ndarray, u: Optional[np.ndarray]):
    _chk(ctx, load().hslb_batch_init(ctx, int(slit), _d(n), _d(u)))


def hslb_batch_profiles(ctx, slit: int, n_z: Optional[np.ndarray], u_z: Optional[np.ndarray]):
    _chk(ctx, load().hslb_batch_profiles(ctx, int(slit), _d(n_z), _d(u_z)))


def hslb_batch_finite(ctx, nslits: int) -> np.ndarray:
    flags = np.zeros(nslits, dtype=np.int32)
    _chk(ctx, load().hslb_batch_finite(ctx, flags.ctypes.data_as(_P(ctypes.c_int32))))
    return flags


def hslb_batch_set_config(ctx, grid_per_cu: int, order: int):
    _chk(ctx, load().hslb_batch_set_config(ctx, int(grid_per_cu), int(order)))


def hslb_batch_set_launch(ctx, phase_grid_per_cu: int, collide_grid_per_cu: int, order: int):
    _chk(ctx, load().hslb_batch_set_launch(ctx, int(phase_grid_per_cu), int(collide_grid_per_cu), int(order)))


def hslb_batch_get_launch(ctx):
    """(phase grid per CU, collide grid per CU, order) in effect."""
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _chk(ctx, load().hslb_batch_get_launch(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def hslb_batch_autotune(ctx, steps: int):
    """Returns (choice, us_per_step[12]) over the 12 launch configurations
    (see include/hslb.h); choice -1 when HSLB_TUNE_CACHE supplied the
    configuration (then us_per_step[0] is its stored time)."""
    choice = ctypes.c_int32()
    us = np.zeros(12)
    _chk(ctx, load().hslb_batch_autotune(ctx, int(steps), ctypes.byref(choice), _d(us), 12))
    return choice.value, us


def hslb_surrogate_set_weights(ctx, w: np.ndarray):
    w = _f32(w).ravel()
    _chk(ctx, load().hslb_surrogate_set_weights(ctx, _f(w), w.size))


def hslb_surrogate_get_weights(ctx) -> np.ndarray:
    w = np.zeros(HSLB_CNN_NWEIGHTS, dtype=np.float32)
    _chk(ctx, load().hslb_surrogate_get_weights(ctx, _f(w), w.size))
    return w


def hslb_surrogate_set_mode(ctx, mode: int):
    _chk(ctx, load().hslb_surrogate_set_mode(ctx, int(mode)))


def hslb_surrogate_set_components(ctx, mask: int):
    _chk(ctx, load().hslb_surrogate_set_components(ctx, int(mask)))


def hslb_surrogate_stats(ctx):
    """(checks, exact fallback steps, last residual, largest residual)."""
    c, f = ctypes.c_int64(), ctypes.c_int64()
    r, m = ctypes.c_double(), ctypes.c_double()
    _chk(ctx, load().hslb_surrogate_stats(ctx, ctypes.byref(c), ctypes.byref(f), ctypes.byref(r),
                                          ctypes.byref(m)))
    return c.value, f.value, r.value, m.value


def hslb_surrogate_force(ctx, F: np.ndarray):
    _chk(ctx, load().hslb_surrogate_force(ctx, _d(F)))


def hslb_surrogate_save_snapshot(ctx, path: str):
    _chk(ctx, load().hslb_surrogate_save_snapshot(ctx, os.fsencode(path)))


def hslb_surrogate_train(ctx, snapshot_dir: str, epochs: int, lr: float) -> float:
    L = ctypes.c_double()
    _chk(ctx, load().hslb_surrogate_train(ctx, os.fsencode(snapshot_dir), int(epochs), float(lr),
                                          ctypes.byref(L)))
    return L.value


def _tchk(tr, rc: int):
    if rc != HSLB_OK:
        raise HslbError(rc, load().hslb_trainer_last_error(tr).decode())


def hslb_trainer_create(capacity_nodes: int, max_snapshot_nodes: int):
    tr = _vp()
    _tchk(None, load().hslb_trainer_create(int(capacity_nodes), int(max_snapshot_nodes), ctypes.byref(tr)))
    return tr


def hslb_trainer_destroy(tr):
    load().hslb_trainer_destroy(tr)


def hslb_trainer_last_error(tr) -> str:
    return load().hslb_trainer_last_error(tr).decode()


def hslb_trainer_add_snapshot(tr, ctx) -> int:
    k = ctypes.c_int32()
    rc = load().hslb_trainer_add_snapshot(tr, ctx, ctypes.byref(k))
    _tchk(tr, rc)
    return k.value


def hslb_trainer_add_snapshot_host(tr, nx, ny, nz, wall_lo, wall_hi, eta, target) -> int:
    eta = np.ascontiguousarray(eta, dtype=np.float64).ravel()
    target = np.ascontiguousarray(target, dtype=np.float64).ravel()
    k = ctypes.c_int32()
    _tchk(tr, load().hslb_trainer_add_snapshot_host(tr, nx, ny, nz, wall_lo, wall_hi, _d(eta), _d(target),
                                                    ctypes.byref(k)))
    return k.value


def hslb_trainer_count(tr) -> int:
    k = ctypes.c_int32()
    _tchk(tr, load().hslb_trainer_count(tr, ctypes.byref(k)))
    return k.value


def hslb_trainer_set_weights(tr, w):
    w = _f32(w).ravel()
    _tchk(tr, load().hslb_trainer_set_weights(tr, _f(w), w.size))


def hslb_trainer_get_weights(tr) -> np.ndarray:
    w = np.zeros(HSLB_CNN_NWEIGHTS, dtype=np.float32)
    _tchk(tr, load().hslb_trainer_get_weights(tr, _f(w), w.size))
    return w


def hslb_trainer_eval(tr, k: int, out: Optional[np.ndarray] = None) -> float:
    L = ctypes.c_double()
    _tchk(tr, load().hslb_trainer_eval(tr, int(k), ctypes.byref(L), _f(out)))
    return L.value


def hslb_trainer_grad(tr, k: int, grad: Optional[np.ndarray] = None) -> float:
    L = ctypes.c_double()
    _tchk(tr, load().hslb_trainer_grad(tr, int(k), ctypes.byref(L), _f(grad)))
    return L.value


def hslb_trainer_step(tr, k: int, lr: float) -> float:
    L = ctypes.c_double()
    _tchk(tr, load().hslb_trainer_step(tr, int(k), float(lr), ctypes.byref(L)))
    return L.value


def hslb_trainer_train(tr, order, lr: float) -> float:
    order = np.ascontiguousarray(order, dtype=np.int32)
    L = ctypes.c_double()
    _tchk(tr, load().hslb_trainer_train(tr, order.ctypes.data_as(_P(ctypes.c_int32)), order.size, float(lr),
                                        ctypes.byref(L)))
    return L.value


_CNN_OUT = {HSLB_CNN_FWD1: 64, HSLB_CNN_FWD2: 64, HSLB_CNN_FWD3: 3, HSLB_CNN_DX3: 64, HSLB_CNN_DX2: 64}
_CNN_WOUT = {HSLB_CNN_DW1: 32 * 125 + 32, HSLB_CNN_DW2: 32 * 32 * 125 + 32, HSLB_CNN_DW3: 3 * 32 * 125 + 3}


def hslb_cnn_op(op: int, nx: int, ny: int, nz: int, zper: bool, w, inp, aux=None) -> np.ndarray:
    """One network operation on host data (see include/hslb.h)."""
    N = nx * ny * nz
    out = np.zeros(_CNN_OUT[op] * N if op in _CNN_OUT else _CNN_WOUT[op], dtype=np.float32)
    w = _f32(w).ravel()
    inp = _f32(inp).ravel()
    aux = None if aux is None else _f32(aux).ravel()
    _tchk(None, load().hslb_cnn_op(int(op), nx, ny, nz, int(bool(zper)), _f(w), _f(inp), _f(aux), _f(out)))
    return out


# ----------------------------------------------------------- convenience


def make_params(nx, ny, nz, sigma, tau, accel=(0.0, 0.0, 0.0), wall_lo=0, wall_hi=0,
                g2_model=HSLB_G2_PAPER, wall_reg=1, precision=HSLB_FP64,
                force_mode=HSLB_FORCE_EXACT, surr_check_every=50, surr_tol=1e-3, att_eps=0.0,
                att_range=0.0, lattice=HSLB_D3Q19, thermal=0) -> hslb_params:
    p = hslb_params()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.wall_lo, p.wall_hi = int(wall_lo), int(wall_hi)
    p.sigma = int(sigma)
    p.tau = float(tau)
    p.accel = (ctypes.c_double * 3)(*[float(a) for a in accel])
    p.g2_model, p.wall_reg = int(g2_model), int(wall_reg)
    p.precision, p.force_mode = int(precision), int(force_mode)
    p.surr_check_every, p.surr_tol = int(surr_check_every), float(surr_tol)
    p.att_eps, p.att_range = float(att_eps), float(att_range)
    p.lattice = int(lattice)
    p.thermal = int(thermal)
    return p


class Sim:
    """One lattice on the GPU.  Fields are float64 arrays shaped (nz, ny, nx),
    vectors (3, nz, ny, nx), populations (Q, nz, ny, nx) with Q = 19, or 39 for
    lattice=39 (the third-order lattice, FP64 only)."""

    def __init__(self, nx, ny, nz, sigma, tau, accel=(0.0, 0.0, 0.0), wall_lo=0, wall_hi=0,
                 precision="f64", g2_model=HSLB_G2_PAPER, wall_reg=1,
                 force_mode=HSLB_FORCE_EXACT, surr_check_every=50, surr_tol=1e-3, att_eps=0.0,
                 att_range=0.0, lattice=HSLB_D3Q19, thermal=0):
        prec = {"f64": HSLB_FP64, "f32": HSLB_FP32}[precision] if isinstance(precision, str) \
            else int(precision)
        self.params = make_params(nx, ny, nz, sigma, tau, accel, wall_lo, wall_hi, g2_model,
                                  wall_reg, prec, force_mode, surr_check_every, surr_tol, att_eps,
                                  att_range, lattice, thermal)
        self.q = 39 if int(lattice) == 39 else 19
        self.shape = (int(nz), int(ny), int(nx))
        self.N = int(nx) * int(ny) * int(nz)
        self.ctx = hslb_create(self.params)

    def close(self):
        if getattr(self, "ctx", None):
            hslb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def init(self, n, u=None, T=None):
        """Equilibrium of (n, u), and of the temperature T in a thermal context."""
        n = np.ascontiguousarray(n, dtype=np.float64).reshape(self.N)
        if u is not None:
            u = np.ascontiguousarray(u, dtype=np.float64).reshape(3 * self.N)
        if T is None:
            hslb_init(self.ctx, n, u)
        else:
            hslb_init_thermal(self.ctx, n, u, np.ascontiguousarray(T, dtype=np.float64).reshape(self.N))

    def thermal_fields(self):
        """Temperature and energy source C^(2), each (nz, ny, nx)."""
        T = np.zeros(self.N)
        Q = np.zeros(self.N)
        hslb_thermal_fields(self.ctx, T, Q)
        return T.reshape(self.shape), Q.reshape(self.shape)

    def step(self, nsteps=1):
        hslb_step(self.ctx, nsteps)

    def sync(self):
        hslb_sync(self.ctx)

    def prepare(self):
        """Capture every graph later steps replay (see hslb_prepare)."""
        hslb_prepare(self.ctx)

    def moments(self):
        n = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        hslb_moments(self.ctx, n, u)
        return n.reshape(self.shape), u.reshape((3,) + self.shape)

    def profiles(self):
        nz = self.shape[0]
        pn = np.zeros(nz)
        pu = np.zeros(3 * nz)
        hslb_profiles(self.ctx, pn, pu)
        return pn, pu.reshape(3, nz)

    def force(self):
        F = np.zeros(3 * self.N)
        hslb_force(self.ctx, F)
        return F.reshape((3,) + self.shape)

    def eta_bar(self):
        e = np.zeros(self.N)
        hslb_eta_bar(self.ctx, e)
        return e.reshape(self.shape)

    def set_solid(self, solid):
        """Solid mask shaped (nz, ny, nx), nonzero = solid; before init."""
        hslb_set_solid(self.ctx, np.asarray(solid).reshape(self.N))

    def attraction_potential(self):
        phi = np.zeros(self.N)
        hslb_attraction_potential(self.ctx, phi)
        return phi.reshape(self.shape)

    def get_populations(self):
        f = np.zeros(self.q * self.N)
        hslb_get_populations(self.ctx, f)
        return f.reshape((self.q,) + self.shape)

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.q * self.N)
        hslb_set_populations(self.ctx, f)

    def timings(self):
        return hslb_get_timings(self.ctx)

    def surrogate_force(self):
        F = np.zeros(3 * self.N)
        hslb_surrogate_force(self.ctx, F)
        return F.reshape((3,) + self.shape)

    @classmethod
    def from_workload(cls, wl, precision: Optional[str] = None, **kw):  # noqa: D102
        return cls(wl.nx, wl.ny, wl.nz, wl.sigma, wl.tau, accel=wl.accel, wall_lo=wl.wall_lo,
                   wall_hi=wl.wall_hi, precision=precision or wl.precision, **kw)


class Batch:
    """A ragged ensemble of slits advanced together on the GPU (one persistent
    launch per phase, K steps per HIP graph)."""

    def __init__(self, workloads_, precision="f32", **kw):
        prec = {"f64": HSLB_FP64, "f32": HSLB_FP32}[precision]
        self.wls = list(workloads_)
        self.params = [make_params(w.nx, w.ny, w.nz, w.sigma, w.tau, w.accel, w.wall_lo, w.wall_hi,
                                   precision=prec, **kw) for w in self.wls]
        self.ctx = hslb_batch_create(self.params)

    def close(self):
        if getattr(self, "ctx", None):
            hslb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def init(self, slit, n, u=None):
        w = self.wls[slit]
        N = w.nx * w.ny * w.nz
        n = np.ascontiguousarray(n, dtype=np.float64).reshape(N)
        if u is not None:
            u = np.ascontiguousarray(u, dtype=np.float64).reshape(3 * N)
        hslb_batch_init(self.ctx, slit, n, u)

    def init_all(self):
        for k, w in enumerate(self.wls):
            n, u = w.fields()
            self.init(k, n, u)

    def step(self, nsteps=1):
        hslb_step(self.ctx, nsteps)

    def sync(self):
        hslb_sync(self.ctx)

    def prepare(self):
        hslb_prepare(self.ctx)

    def profiles(self, slit):
        nz = self.wls[slit].nz
        pn = np.zeros(nz)
        pu = np.zeros(3 * nz)
        hslb_batch_profiles(self.ctx, slit, pn, pu)
        return pn, pu.reshape(3, nz)

    def finite(self):
        return hslb_batch_finite(self.ctx, len(self.wls)).astype(bool)

    def autotune(self, steps=20):
        return hslb_batch_autotune(self.ctx, steps)

    @property
    def fluid_nodes(self):
        return sum(w.fluid_nodes for w in self.wls)


class Trainer:
    """Snapshot store, weights and Adam state of the learned force on the GPU."""

    def __init__(self, capacity_nodes: int, max_snapshot_nodes: int):
        self.tr = hslb_trainer_create(capacity_nodes, max_snapshot_nodes)
        self.sizes = []

    def close(self):
        if getattr(self, "tr", None):
            hslb_trainer_destroy(self.tr)
            self.tr = None

    def __del__(self):
        self.close()

    def add(self, sim: Sim) -> int:
        k = hslb_trainer_add_snapshot(self.tr, sim.ctx)
        self.sizes.append(sim.shape)
        return k

    def add_host(self, eta, target, wall_lo=0, wall_hi=0) -> int:
        nz, ny, nx = np.shape(eta)
        k = hslb_trainer_add_snapshot_host(self.tr, nx, ny, nz, wall_lo, wall_hi, eta, target)
        self.sizes.append((nz, ny, nx))
        return k

    def __len__(self):
        return hslb_trainer_count(self.tr)

    def set_weights(self, w):
        hslb_trainer_set_weights(self.tr, w)

    def weights(self) -> np.ndarray:
        return hslb_trainer_get_weights(self.tr)

    def eval(self, k: int, want_out: bool = False):
        out = np.zeros((3,) + tuple(self.sizes[k]), dtype=np.float32) if want_out else None
        L = hslb_trainer_eval(self.tr, k, out)
        return (L, out) if want_out else L

    def grad(self, k: int):
        g = np.zeros(HSLB_CNN_NWEIGHTS, dtype=np.float32)
        L = hslb_trainer_grad(self.tr, k, g)
        return L, g

    def step(self, k: int, lr: float) -> float:
        return hslb_trainer_step(self.tr, k, lr)

    def train(self, order, lr: float) -> float:
        return hslb_trainer_train(self.tr, order, lr)
