"""Thin Python binding of libdgd (argument marshalling only).

Every function here has the name of the C entry point it calls and does
nothing but convert arguments: all arithmetic of the solve runs in the HIP
kernels behind the C-ABI (include/dgd.h).  PyTorch is used, when given, only
for device memory (workspaces, operator-apply buffers) and streams.

Importing this module loads paper_1907_06191_amd/libdgd.so and raises
ImportError if it is missing; there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libdgd.so not built at {LIB_PATH}: run python -m paper_1907_06191_amd.build")
try:
    # PyTorch first, so that the library binds to the HIP runtime PyTorch
    # loads (its workspaces and streams are then the library's own).
    import torch  # noqa: F401
except ImportError:
    pass
_lib = ctypes.CDLL(LIB_PATH)

DGD_OK = 0
DGD_EINVAL = -1
DGD_ENOMEM = -2
DGD_EDEVICE = -3
DGD_EUNSTABLE = -4
DGD_ENOTFREE = -5
DGD_FP64 = 0
DGD_FP32 = 1
DGD_BF16X3 = 2
DGD_OUTER_REFLECT = 0
DGD_OUTER_ABSORB = 1

_c_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class DGDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdgd error {code}: {msg}")
        self.code = code


def _sig(name, argtypes, restype=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = argtypes
    f.restype = restype
    return f


_sig("dgd_version", [])
_sig("dgd_last_error", [], ctypes.c_char_p)
_sig("dgd_set_option", [ctypes.c_char_p, ctypes.c_int64])
_sig("dgd_mesh_create", [ctypes.c_double, ctypes.c_int32, _c_dp, ctypes.c_int32, ctypes.POINTER(_vp)])
_sig("dgd_mesh_info", [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                       ctypes.POINTER(ctypes.c_int32), _c_dp])
_sig("dgd_mesh_elements", [_vp, _vp, _vp, _vp])
_sig("dgd_mesh_faces", [_vp, _vp])
_sig("dgd_mesh_destroy", [_vp], None)
_sig("dgd_operator_build", [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                            ctypes.c_double, ctypes.POINTER(_vp)])
_sig("dgd_operator_build_outer", [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                  ctypes.POINTER(_vp)])
_sig("dgd_operator_build_mixed", [_vp, _c_dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_int32, ctypes.c_double, ctypes.POINTER(_vp)])
_sig("dgd_operator_dt", [_vp, _c_dp, _c_dp])
_sig("dgd_operator_info", [_vp, ctypes.POINTER(ctypes.c_int32), _c_dp, ctypes.POINTER(ctypes.c_int32)])
_sig("dgd_workspace_size", [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)])
_sig("dgd_operator_apply", [_vp, _vp, _vp, ctypes.c_int32, _vp])
_sig("dgd_operator_destroy", [_vp], None)
_sig("dgd_run_create", [_vp, _c_dp, ctypes.c_int32, ctypes.c_double, _vp, ctypes.c_size_t, _vp,
                        ctypes.POINTER(_vp)])
_sig("dgd_run_advance", [_vp, ctypes.c_int64, ctypes.c_double])
_sig("dgd_run_moments", [_vp, _c_dp, ctypes.c_size_t])
_sig("dgd_run_shape", [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                       ctypes.POINTER(ctypes.c_int32)])
_sig("dgd_run_get_state", [_vp, _vp, ctypes.c_size_t])
_sig("dgd_run_set_state", [_vp, _vp, ctypes.c_size_t])
_sig("dgd_run_kernel", [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)])
_sig("dgd_run_step_count", [_vp, ctypes.POINTER(ctypes.c_int64)])
_sig("dgd_run_set_step_count", [_vp, ctypes.c_int64])
_sig("dgd_run_destroy", [_vp], None)
_sig("dgd_batch_workspace_size", [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)])
_sig("dgd_batch_create", [_vp, ctypes.c_int32, _c_dp, ctypes.c_int32, ctypes.c_double, _vp, ctypes.c_size_t,
                          _vp, ctypes.POINTER(_vp)])
_sig("dgd_batch_groups", [_vp, ctypes.POINTER(ctypes.c_int32), _vp, _vp, _vp, _vp])
_sig("dgd_batch_advance", [_vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_double])
_sig("dgd_batch_moments", [_vp, _c_dp, ctypes.c_size_t])
_sig("dgd_batch_shape", [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)])
_sig("dgd_batch_destroy", [_vp], None)
_sig("dgd_eap_solve_batch", [_vp, ctypes.c_int32, _c_dp, ctypes.c_int32, ctypes.c_double, _c_dp,
                             ctypes.c_int32, _c_dp, _c_dp, _vp, ctypes.c_size_t, _vp])
_sig("dgd_mesh_occupancy", [_vp, ctypes.c_int32, _vp])
_sig("dgd_surrogate_create", [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.POINTER(_vp)])
_sig("dgd_surrogate_n_params", [_vp, ctypes.POINTER(ctypes.c_int64)])
_sig("dgd_surrogate_get_params", [_vp, ctypes.c_int32, _vp])
_sig("dgd_surrogate_set_params", [_vp, ctypes.c_int32, _vp])
_sig("dgd_surrogate_loss_grad", [_vp, ctypes.c_int32, _vp, _c_dp, _c_dp, ctypes.c_int32, _c_dp, _vp])
_sig("dgd_surrogate_train", [_vp, _vp, _c_dp, _c_dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             ctypes.c_double, ctypes.c_uint64, _c_dp])
_sig("dgd_surrogate_predict", [_vp, _vp, _c_dp, ctypes.c_int32, ctypes.c_double, _c_dp, _c_dp, _vp])
_sig("dgd_surrogate_destroy", [_vp], None)
_sig("dgd_eap_solve_expm", [_vp, _c_dp, ctypes.c_int32, ctypes.c_double, _c_dp, ctypes.c_int32,
                            ctypes.c_double, _c_dp, _c_dp, ctypes.POINTER(ctypes.c_int64)])
_sig("dgd_eap_solve", [_vp, _c_dp, ctypes.c_int32, ctypes.c_double, _c_dp, ctypes.c_int32, _c_dp,
                       _c_dp, _vp, ctypes.c_size_t, _vp])
_sig("dgd_eap_solve_noalloc", [_vp, _c_dp, ctypes.c_int32, ctypes.c_double, _c_dp, ctypes.c_int32,
                               _c_dp, _c_dp, _vp])
_sig("dgd_autotune", [_vp, ctypes.c_int32, _vp, ctypes.POINTER(ctypes.c_int32), _c_dp])
_sig("dgd_run_signal", [_vp, _c_dp, ctypes.c_int32, _c_dp])
_sig("dgd_eap_solve_signal", [_vp, _c_dp, ctypes.c_int32, ctypes.c_double, _c_dp, ctypes.c_int32, _c_dp,
                              ctypes.c_int32, _c_dp, _c_dp, _vp, ctypes.c_size_t, _vp])
_sig("dgd_tune_export", [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)])
_sig("dgd_tune_import", [ctypes.c_char_p])
_sig("dgd_tune_clear", [], None)


def _check(rc):
    if rc != DGD_OK:
        raise DGDError(rc, _lib.dgd_last_error().decode())


def _f64(a, shape_tail=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape_tail is not None:
        a = a.reshape((-1,) + tuple(shape_tail))
    return a


def _ptr(a):
    return a.ctypes.data_as(_c_dp) if a is not None and a.size else None


def _dev_ptr(t):
    """Device pointer of a torch tensor (or an int address), else None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------ C names

def dgd_version() -> int:
    return _lib.dgd_version()


def dgd_set_option(name: str, value: int) -> None:
    _check(_lib.dgd_set_option(name.encode(), int(value)))


def dgd_autotune(op, n_points: int, stream=None):
    """Tune the stage launch shape of op at n_points right-hand sides.
    Returns (dict(epw, waves, xcd_remap, grid_per_cu), ms per stage launch)."""
    shape = (ctypes.c_int32 * 4)()
    ms = ctypes.c_double()
    _check(_lib.dgd_autotune(op, int(n_points), _stream_ptr(stream), shape, ctypes.byref(ms)))
    return dict(epw=shape[0], waves=shape[1], xcd_remap=shape[2], grid_per_cu=shape[3]), ms.value


def dgd_tune_export() -> str:
    n = ctypes.c_size_t()
    _check(_lib.dgd_tune_export(None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(_lib.dgd_tune_export(buf, n.value, ctypes.byref(n)))
    return buf.value.decode()


def dgd_tune_import(text: str) -> None:
    _check(_lib.dgd_tune_import(text.encode()))


def dgd_tune_clear() -> None:
    _lib.dgd_tune_clear()


def dgd_mesh_create(L_um: float, n_cells: int, disks) -> int:
    d = _f64(disks, (3,))
    out = _vp()
    _check(_lib.dgd_mesh_create(float(L_um), int(n_cells), _ptr(d), int(d.shape[0]), ctypes.byref(out)))
    return out.value


def dgd_mesh_info(mesh) -> dict:
    na, nf = ctypes.c_int64(), ctypes.c_int64()
    nc = ctypes.c_int32()
    rf = ctypes.c_double()
    _check(_lib.dgd_mesh_info(mesh, ctypes.byref(na), ctypes.byref(nf), ctypes.byref(nc), ctypes.byref(rf)))
    return dict(n_active=na.value, n_faces=nf.value, n_components=nc.value, removed_fraction=rf.value)


def dgd_mesh_elements(mesh):
    n = dgd_mesh_info(mesh)["n_active"]
    ci = np.zeros(n, dtype=np.int32)
    cj = np.zeros(n, dtype=np.int32)
    o = np.zeros(n, dtype=np.int8)
    _check(_lib.dgd_mesh_elements(mesh, ci.ctypes.data, cj.ctypes.data, o.ctypes.data))
    return ci, cj, o


def dgd_mesh_faces(mesh):
    n = dgd_mesh_info(mesh)["n_active"]
    nbr = np.zeros((n, 3), dtype=np.int32)
    _check(_lib.dgd_mesh_faces(mesh, nbr.ctypes.data))
    return nbr


def dgd_mesh_destroy(mesh) -> None:
    _lib.dgd_mesh_destroy(mesh)


def dgd_operator_build(mesh, p: int, D: float, eta: float, precision: int, dt_max_ms: float = 0.0) -> int:
    out = _vp()
    _check(_lib.dgd_operator_build(mesh, int(p), float(D), float(eta), int(precision), float(dt_max_ms),
                                   ctypes.byref(out)))
    return out.value


def dgd_operator_build_outer(mesh, p: int, D: float, eta: float, precision: int,
                             dt_max_ms: float = 0.0, outer: int = DGD_OUTER_REFLECT) -> int:
    out = _vp()
    _check(_lib.dgd_operator_build_outer(mesh, int(p), float(D), float(eta), int(precision),
                                         float(dt_max_ms), int(outer), ctypes.byref(out)))
    return out.value


def dgd_operator_build_mixed(mesh, disks, p: int, D: float, precision: int,
                             dt_max_ms: float = 0.0) -> int:
    d = _f64(disks).reshape(-1, 3) if disks is not None else np.zeros((0, 3))
    d = np.ascontiguousarray(d, dtype=np.float64)
    out = _vp()
    _check(_lib.dgd_operator_build_mixed(mesh, _ptr(d), int(d.shape[0]), int(p), float(D),
                                         int(precision), float(dt_max_ms), ctypes.byref(out)))
    return out.value


def dgd_operator_dt(op):
    dt, lam = ctypes.c_double(), ctypes.c_double()
    _check(_lib.dgd_operator_dt(op, ctypes.byref(dt), ctypes.byref(lam)))
    return dt.value, lam.value


def dgd_operator_info(op):
    np_ = ctypes.c_int32()
    prec = ctypes.c_int32()
    _check(_lib.dgd_operator_info(op, ctypes.byref(np_), None, ctypes.byref(prec)))
    nodes = np.zeros((2, np_.value, 2))
    _check(_lib.dgd_operator_info(op, ctypes.byref(np_), _ptr(nodes), ctypes.byref(prec)))
    return np_.value, nodes, prec.value


def dgd_workspace_size(op, n_points: int) -> int:
    b = ctypes.c_size_t()
    _check(_lib.dgd_workspace_size(op, int(n_points), ctypes.byref(b)))
    return b.value


def dgd_operator_apply(op, d_in, d_out, n_rhs: int, stream=None) -> None:
    _check(_lib.dgd_operator_apply(op, _dev_ptr(d_in), _dev_ptr(d_out), int(n_rhs), _stream_ptr(stream)))


def dgd_operator_destroy(op) -> None:
    _lib.dgd_operator_destroy(op)


def dgd_run_create(op, points, sigma0: float, workspace=None, ws_bytes: int = 0, stream=None) -> int:
    pts = _f64(points, (2,))
    out = _vp()
    if workspace is not None and not ws_bytes:
        ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib.dgd_run_create(op, _ptr(pts), int(pts.shape[0]), float(sigma0), _dev_ptr(workspace),
                               int(ws_bytes), _stream_ptr(stream), ctypes.byref(out)))
    return out.value


def dgd_run_advance(run, n_steps: int, dt_ms: float) -> None:
    _check(_lib.dgd_run_advance(run, int(n_steps), float(dt_ms)))


def dgd_run_shape(run):
    """(state values, start points, bytes per state value) of a run."""
    nv, npt, vb = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.dgd_run_shape(run, ctypes.byref(nv), ctypes.byref(npt), ctypes.byref(vb)))
    return nv.value, npt.value, vb.value


def dgd_run_moments(run, n_points: int = None, check: bool = True) -> np.ndarray:
    """Moments [n_points][6]; the buffer is sized from the run itself."""
    npt = dgd_run_shape(run)[1]
    if n_points is not None and n_points != npt:
        raise ValueError(f"run has {npt} start points, not {n_points}")
    out = np.zeros((npt, 6))
    rc = _lib.dgd_run_moments(run, _ptr(out), out.size)
    if check:
        _check(rc)
    return out


def _state_dtype(vb):
    return np.float64 if vb == 8 else np.float32


def dgd_run_get_state(run, n_values: int = None, dtype=None) -> np.ndarray:
    """The run's state as a flat array of its own type and length."""
    nv, _, vb = dgd_run_shape(run)
    dt = _state_dtype(vb)
    if n_values is not None and n_values != nv:
        raise ValueError(f"run holds {nv} state values, not {n_values}")
    if dtype is not None and np.dtype(dtype) != np.dtype(dt):
        raise ValueError(f"run state is {np.dtype(dt)}, not {np.dtype(dtype)}")
    out = np.zeros(nv, dtype=dt)
    _check(_lib.dgd_run_get_state(run, out.ctypes.data, out.nbytes))
    return out


def dgd_run_set_state(run, state: np.ndarray) -> None:
    nv, _, vb = dgd_run_shape(run)
    dt = _state_dtype(vb)
    s = np.ascontiguousarray(state)
    if s.dtype != np.dtype(dt) or s.size != nv:
        raise ValueError(f"run holds {nv} values of {np.dtype(dt)}; got {s.size} of {s.dtype}")
    _check(_lib.dgd_run_set_state(run, s.ctypes.data, s.nbytes))


def dgd_run_step_count(run) -> int:
    n = ctypes.c_int64()
    _check(_lib.dgd_run_step_count(run, ctypes.byref(n)))
    return n.value


def dgd_run_set_step_count(run, steps: int) -> None:
    _check(_lib.dgd_run_set_step_count(run, int(steps)))


KERNEL_NAMES = ("valu", "packed", "mfma", "mfma_bf16x3")


def dgd_run_kernel(run):
    """(kernel name, dict(epw, waves, xcd_remap, grid)) of the run's stage launches."""
    k = ctypes.c_int32()
    sh = (ctypes.c_int64 * 4)()
    _check(_lib.dgd_run_kernel(run, ctypes.byref(k), sh))
    return KERNEL_NAMES[k.value], dict(epw=sh[0], waves=sh[1], xcd_remap=sh[2], grid=sh[3])


def dgd_run_destroy(run) -> None:
    _lib.dgd_run_destroy(run)


def dgd_eap_solve(op, points, sigma0: float, deltas, workspace=None, ws_bytes: int = 0, stream=None):
    """Returns (sigma [n][nDelta][3], moments [n][nDelta][6])."""
    pts = _f64(points, (2,))
    d = _f64(deltas).ravel()
    n = pts.shape[0]
    sig = np.zeros((n, d.size, 3))
    mom = np.zeros((n, d.size, 6))
    if workspace is not None and not ws_bytes:
        ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib.dgd_eap_solve(op, _ptr(pts), n, float(sigma0), _ptr(d), int(d.size), _ptr(sig), _ptr(mom),
                              _dev_ptr(workspace), int(ws_bytes), _stream_ptr(stream)))
    return sig, mom


def dgd_eap_solve_noalloc(op, points, sigma0: float, deltas, stream=None):
    """dgd_eap_solve in the library's fixed device scratch (no allocation).
    Returns (sigma [n][nDelta][3], moments [n][nDelta][6])."""
    pts = _f64(points, (2,))
    d = _f64(deltas).ravel()
    n = pts.shape[0]
    sig = np.zeros((n, d.size, 3))
    mom = np.zeros((n, d.size, 6))
    _check(_lib.dgd_eap_solve_noalloc(op, _ptr(pts), n, float(sigma0), _ptr(d), int(d.size), _ptr(sig),
                                      _ptr(mom), _stream_ptr(stream)))
    return sig, mom


def dgd_run_signal(run, q, n_points: int) -> np.ndarray:
    """Complex signal [n_points][n_q] of the run's current state."""
    qq = _f64(q, (2,))
    out = np.zeros((n_points, qq.shape[0], 2))
    _check(_lib.dgd_run_signal(run, _ptr(qq), int(qq.shape[0]), _ptr(out)))
    return out[..., 0] + 1j * out[..., 1]


def dgd_eap_solve_signal(op, points, sigma0: float, deltas, q, workspace=None, ws_bytes: int = 0,
                         stream=None):
    """Returns (signal complex [n][nDelta][n_q], moments [n][nDelta][6])."""
    pts = _f64(points, (2,))
    d = _f64(deltas).ravel()
    qq = _f64(q, (2,))
    n = pts.shape[0]
    sig = np.zeros((n, d.size, qq.shape[0], 2))
    sg = np.zeros((n, d.size, 6))
    if workspace is not None and not ws_bytes:
        ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib.dgd_eap_solve_signal(op, _ptr(pts), n, float(sigma0), _ptr(d), int(d.size), _ptr(qq),
                                     int(qq.shape[0]), _ptr(sig), _ptr(sg), _dev_ptr(workspace),
                                     int(ws_bytes), _stream_ptr(stream)))
    return sig[..., 0] + 1j * sig[..., 1], sg


def dgd_mesh_occupancy(mesh, size: int = 64) -> np.ndarray:
    img = np.zeros((size, size), dtype=np.uint8)
    _check(_lib.dgd_mesh_occupancy(mesh, int(size), img.ctypes.data))
    return img


def _u8(images):
    return np.ascontiguousarray(np.asarray(images, dtype=np.uint8))


def dgd_surrogate_create(n_members: int, channels: int = 32, hidden: int = 256, seed: int = 0) -> int:
    out = _vp()
    _check(_lib.dgd_surrogate_create(int(n_members), int(channels), int(hidden), int(seed), ctypes.byref(out)))
    return out.value


def dgd_surrogate_n_params(s) -> int:
    n = ctypes.c_int64()
    _check(_lib.dgd_surrogate_n_params(s, ctypes.byref(n)))
    return n.value


def dgd_surrogate_get_params(s, member: int) -> np.ndarray:
    p = np.zeros(dgd_surrogate_n_params(s), dtype=np.float32)
    _check(_lib.dgd_surrogate_get_params(s, int(member), p.ctypes.data))
    return p


def dgd_surrogate_set_params(s, member: int, params) -> None:
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    _check(_lib.dgd_surrogate_set_params(s, int(member), p.ctypes.data))


def dgd_surrogate_loss_grad(s, member: int, images, log_deltas, targets):
    im = _u8(images)
    ld = _f64(log_deltas).ravel()
    tg = _f64(targets, (3,))
    g = np.zeros(dgd_surrogate_n_params(s), dtype=np.float32)
    loss = ctypes.c_double()
    _check(_lib.dgd_surrogate_loss_grad(s, int(member), im.ctypes.data, _ptr(ld), _ptr(tg), int(ld.size),
                                        ctypes.byref(loss), g.ctypes.data))
    return loss.value, g


def dgd_surrogate_train(s, images, log_deltas, targets, epochs: int, batch: int, lr: float,
                        shuffle_seed: int, n_members: int) -> np.ndarray:
    im = _u8(images)
    ld = _f64(log_deltas).ravel()
    tg = _f64(targets, (3,))
    losses = np.zeros((n_members, max(int(epochs), 1)))
    _check(_lib.dgd_surrogate_train(s, im.ctypes.data, _ptr(ld), _ptr(tg), int(ld.size), int(epochs), int(batch),
                                    float(lr), int(shuffle_seed), _ptr(losses)))
    return losses[:, :epochs]


def dgd_surrogate_predict(s, images, log_deltas, threshold: float):
    im = _u8(images)
    ld = _f64(log_deltas).ravel()
    n = ld.size
    mean = np.zeros((n, 3))
    spread = np.zeros(n)
    flag = np.zeros(n, dtype=np.uint8)
    _check(_lib.dgd_surrogate_predict(s, im.ctypes.data, _ptr(ld), n, float(threshold), _ptr(mean),
                                      _ptr(spread), flag.ctypes.data))
    return mean, spread, flag.astype(bool)


def dgd_surrogate_destroy(s) -> None:
    _lib.dgd_surrogate_destroy(s)


def _op_array(ops):
    handles = [o.handle if hasattr(o, "handle") else o for o in ops]
    return (_vp * len(handles))(*handles)


def dgd_eap_solve_expm(op, points, sigma0: float, deltas, lambda_bound: float = 0.0):
    """Returns (sigma [n][nDelta][3], moments [n][nDelta][6], operator applications)."""
    pts = _f64(points, (2,))
    d = _f64(deltas).ravel()
    n = pts.shape[0]
    sig = np.zeros((n, d.size, 3))
    mom = np.zeros((n, d.size, 6))
    na = ctypes.c_int64()
    _check(_lib.dgd_eap_solve_expm(op, _ptr(pts), n, float(sigma0), _ptr(d), int(d.size), float(lambda_bound),
                                   _ptr(sig), _ptr(mom), ctypes.byref(na)))
    return sig, mom, na.value


def dgd_batch_workspace_size(ops, n_points: int) -> int:
    b = ctypes.c_size_t()
    _check(_lib.dgd_batch_workspace_size(_op_array(ops), len(ops), int(n_points), ctypes.byref(b)))
    return b.value


def dgd_batch_create(ops, points, sigma0: float, workspace=None, ws_bytes: int = 0, stream=None) -> int:
    pts = _f64(points).reshape(len(ops), -1, 2)
    out = _vp()
    if workspace is not None and not ws_bytes:
        ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib.dgd_batch_create(_op_array(ops), len(ops), _ptr(pts), int(pts.shape[1]), float(sigma0),
                                 _dev_ptr(workspace), int(ws_bytes), _stream_ptr(stream), ctypes.byref(out)))
    return out.value


def dgd_batch_groups(batch):
    n = ctypes.c_int32()
    _check(_lib.dgd_batch_groups(batch, ctypes.byref(n), None, None, None, None))
    p = np.zeros(n.value, dtype=np.int32)
    size = np.zeros(n.value, dtype=np.int32)
    dt = np.zeros(n.value)
    dof = np.zeros(n.value, dtype=np.int64)
    _check(_lib.dgd_batch_groups(batch, ctypes.byref(n), p.ctypes.data, size.ctypes.data, dt.ctypes.data,
                                 dof.ctypes.data))
    return [dict(p=int(p[k]), size=int(size[k]), dt=float(dt[k]), dof=int(dof[k])) for k in range(n.value)]


def dgd_batch_advance(batch, group: int, n_steps: int, dt_ms: float) -> None:
    _check(_lib.dgd_batch_advance(batch, int(group), int(n_steps), float(dt_ms)))


def dgd_batch_shape(batch):
    """(geometries, start points per geometry) of a batch."""
    g, n = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.dgd_batch_shape(batch, ctypes.byref(g), ctypes.byref(n)))
    return g.value, n.value


def dgd_batch_moments(batch, n_geoms: int = None, n_points: int = None, check: bool = True) -> np.ndarray:
    """Moments [n_geoms][n_points][6]; the buffer is sized from the batch itself."""
    g, n = dgd_batch_shape(batch)
    if (n_geoms is not None and n_geoms != g) or (n_points is not None and n_points != n):
        raise ValueError(f"batch has {g} geometries x {n} start points")
    out = np.zeros((g, n, 6))
    rc = _lib.dgd_batch_moments(batch, _ptr(out), out.size)
    if check:
        _check(rc)
    return out


def dgd_batch_destroy(batch) -> None:
    _lib.dgd_batch_destroy(batch)


def dgd_eap_solve_batch(ops, points, sigma0: float, deltas, workspace=None, ws_bytes: int = 0, stream=None):
    """Returns (sigma [G][n][nDelta][3], moments [G][n][nDelta][6])."""
    pts = _f64(points).reshape(len(ops), -1, 2)
    d = _f64(deltas).ravel()
    G, n = pts.shape[0], pts.shape[1]
    sig = np.zeros((G, n, d.size, 3))
    mom = np.zeros((G, n, d.size, 6))
    if workspace is not None and not ws_bytes:
        ws_bytes = workspace.numel() * workspace.element_size()
    _check(_lib.dgd_eap_solve_batch(_op_array(ops), G, _ptr(pts), n, float(sigma0), _ptr(d), int(d.size),
                                    _ptr(sig), _ptr(mom), _dev_ptr(workspace), int(ws_bytes),
                                    _stream_ptr(stream)))
    return sig, mom


# ----------------------------------------------------------- RAII helpers

class Mesh:
    def __init__(self, L_um, n_cells, disks):
        self._destroy = _lib.dgd_mesh_destroy       # survives module teardown
        self.handle = dgd_mesh_create(L_um, n_cells, disks)

    def info(self):
        return dgd_mesh_info(self.handle)

    def elements(self):
        return dgd_mesh_elements(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


class Operator:
    def __init__(self, mesh: Mesh, p, D, eta, precision, dt_max_ms=0.0, outer=DGD_OUTER_REFLECT):
        self._destroy = _lib.dgd_operator_destroy
        self.mesh = mesh              # keeps the mesh alive
        self.outer = outer
        self.handle = dgd_operator_build_outer(mesh.handle, p, D, eta, precision, dt_max_ms, outer)

    @property
    def dt(self):
        return dgd_operator_dt(self.handle)[0]

    @property
    def lambda_max(self):
        return dgd_operator_dt(self.handle)[1]

    def info(self):
        return dgd_operator_info(self.handle)

    def workspace_size(self, n_points):
        return dgd_workspace_size(self.handle, n_points)

    def apply(self, x, y, n_rhs, stream=None):
        dgd_operator_apply(self.handle, x, y, n_rhs, stream)

    def solve(self, points, sigma0, deltas, workspace=None, stream=None):
        return dgd_eap_solve(self.handle, points, sigma0, deltas, workspace=workspace, stream=stream)

    def close(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


class MixedOperator(Operator):
    """The paper's mixed form on all pixels (k = 0 in the cells of `disks`);
    `mesh` normally holds every pixel (built with no disks)."""

    def __init__(self, mesh: Mesh, disks, p, D, precision, dt_max_ms=0.0):
        self._destroy = _lib.dgd_operator_destroy
        self.mesh = mesh
        self.outer = DGD_OUTER_REFLECT
        self.handle = dgd_operator_build_mixed(mesh.handle, disks, p, D, precision, dt_max_ms)


class Batch:
    def __init__(self, ops, points, sigma0, workspace=None, stream=None):
        self._destroy = _lib.dgd_batch_destroy
        self.ops = list(ops)
        pts = np.asarray(points, dtype=np.float64).reshape(len(self.ops), -1, 2)
        self.G, self.n = pts.shape[0], pts.shape[1]
        self.workspace = workspace
        self.handle = dgd_batch_create(self.ops, pts, sigma0, workspace=workspace, stream=stream)

    def groups(self):
        return dgd_batch_groups(self.handle)

    def advance(self, group, n_steps, dt_ms):
        dgd_batch_advance(self.handle, group, n_steps, dt_ms)

    def moments(self, check=True):
        return dgd_batch_moments(self.handle, self.G, self.n, check)

    def close(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


class Surrogate:
    def __init__(self, n_members=4, channels=32, hidden=256, seed=0):
        self._destroy = _lib.dgd_surrogate_destroy
        self.n_members = n_members
        self.handle = dgd_surrogate_create(n_members, channels, hidden, seed)

    def train(self, images, log_deltas, targets, epochs, batch=256, lr=1e-3, shuffle_seed=0):
        return dgd_surrogate_train(self.handle, images, log_deltas, targets, epochs, batch, lr, shuffle_seed,
                                   self.n_members)

    def predict(self, images, log_deltas, threshold=1e-3):
        return dgd_surrogate_predict(self.handle, images, log_deltas, threshold)

    def close(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


class Run:
    def __init__(self, op: Operator, points, sigma0, workspace=None, stream=None):
        self._destroy = _lib.dgd_run_destroy
        self.op = op
        self.n = int(np.asarray(points).reshape(-1, 2).shape[0])
        self.workspace = workspace
        self.handle = dgd_run_create(op.handle, points, sigma0, workspace=workspace, stream=stream)

    def advance(self, n_steps, dt_ms):
        dgd_run_advance(self.handle, n_steps, dt_ms)

    def moments(self, check=True):
        return dgd_run_moments(self.handle, self.n, check)

    def close(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()
