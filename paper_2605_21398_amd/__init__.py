"""Python binding of libregdock: the MI355X global search of probe-aware
contact registration by complementary-shape docking (arxiv 2605.21398).

The functions carry the names of the C ABI (include/regdock.h) and only
marshal arguments: every step runs in the HIP kernels of libregdock.so.
PyTorch provides device memory and the HIP stream.  There is no fallback:
if the library is not built, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libregdock.so")

REG_OK, REG_EINVAL, REG_ENOMEM, REG_EDEVICE, REG_EBUSY, REG_ENOTSUP, REG_EAGAIN, REG_ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7
_NAMES = {-1: "REG_EINVAL", -2: "REG_ENOMEM", -3: "REG_EDEVICE", -4: "REG_EBUSY", -5: "REG_ENOTSUP",
          -6: "REG_EAGAIN", -7: "REG_ECANCELED"}

# every entry point the header declares
EXPORTS = ["register_init", "score_rotations", "register_top_k", "register_free", "register_last_error",
           "register_info", "register_debug_object_grid", "register_debug_swept", "register_debug_swept_reach",
           "register_debug_correlation",
           "register_set_grids", "register_set_timing", "register_get_timing", "register_search_stats",
           "refine_se3", "register_debug_distance", "register_refine_stats", "register_server_create",
           "register_server_destroy", "register_submit", "register_poll", "register_wait", "register_server_stats",
           "register_server_last_error", "register_batch_create", "register_batch_run", "register_batch_outputs",
           "register_batch_free", "register_autotune", "register_tuned_batch", "register_tuned_schedule",
           "register_tune_save", "register_tune_load", "register_cached_bytes",
           "register_release_cached", "so3_super_fibonacci", "so3_geoball_sf", "so3_geoball_sf_noalloc",
           "register_set_rotations",
           "refine_se3_lbfgsb", "register_linear_edge"]


class RegError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class reg_mesh(ctypes.Structure):
    _fields_ = [("vertices", ctypes.c_void_p), ("n_vertices", ctypes.c_int32), ("faces", ctypes.c_void_p),
                ("n_faces", ctypes.c_int32), ("touchable", ctypes.c_void_p)]


class reg_probe(ctypes.Structure):
    _fields_ = [("radius_mm", ctypes.c_double), ("length_mm", ctypes.c_double)]


class reg_grid_spec(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("h_mm", ctypes.c_double), ("center_world", ctypes.c_double * 3)]


class reg_params(ctypes.Structure):
    _fields_ = [("tau_out1", ctypes.c_double), ("tau_in1", ctypes.c_double), ("rho", ctypes.c_double),
                ("tau_out2", ctypes.c_double), ("tau_in2", ctypes.c_double), ("k", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("b_t", ctypes.c_double), ("b_r", ctypes.c_double),
                ("eps", ctypes.c_double), ("max_iters", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("rescore", ctypes.c_int32), ("lanes", ctypes.c_int32), ("plane_variant", ctypes.c_int32),
                ("z_variant", ctypes.c_int32), ("rotate_object", ctypes.c_int32),
                ("split_plane", ctypes.c_int32)]


class reg_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("cache_bytes", ctypes.c_int64), ("fake", ctypes.c_int32), ("fake_us_per_rotation", ctypes.c_double)]


class reg_request(ctypes.Structure):
    _fields_ = [("mesh", reg_mesh), ("object_id", ctypes.c_int64), ("probe", reg_probe), ("poses", ctypes.c_void_p),
                ("n_poses", ctypes.c_int32), ("so3", ctypes.c_void_p), ("n_rot", ctypes.c_int32),
                ("grid", reg_grid_spec), ("params", reg_params), ("top_k", ctypes.c_int32), ("refine", ctypes.c_int32)]


class reg_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_top", ctypes.c_int32), ("best_score", ctypes.c_float),
                ("best_pose", ctypes.c_double * 7), ("best_J", ctypes.c_double), ("top_rot", ctypes.c_int32 * 16),
                ("top_score", ctypes.c_float * 16), ("top_pose", ctypes.c_double * 112),
                ("refined_pose", ctypes.c_double * 112), ("refined_J", ctypes.c_double * 16),
                ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_end_ns", ctypes.c_int64), ("footprint_bytes", ctypes.c_int64), ("error", ctypes.c_char * 128)]


class reg_server_stats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("running", ctypes.c_int64), ("done", ctypes.c_int64),
                ("in_use_bytes", ctypes.c_int64), ("budget_bytes", ctypes.c_int64), ("cache_hits", ctypes.c_int64),
                ("cache_misses", ctypes.c_int64), ("cache_bytes", ctypes.c_int64), ("cached_objects", ctypes.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libregdock.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2605_21398_amd.build`")
    # torch ships its own HIP runtime under the same SONAME; loading torch first
    # makes the dynamic loader bind libregdock to that one runtime instead of
    # bringing a second HSA runtime into the process.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    p, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.register_init.restype = ctypes.c_int
    L.register_init.argtypes = [ctypes.POINTER(reg_mesh), ctypes.POINTER(reg_probe), p, i32, p, i32,
                                ctypes.POINTER(reg_grid_spec), ctypes.POINTER(reg_params), p, ctypes.POINTER(p)]
    L.score_rotations.restype = ctypes.c_int
    L.score_rotations.argtypes = [p, i32, i32, p, p, p]
    L.register_top_k.restype = ctypes.c_int
    L.register_top_k.argtypes = [p, p, i32, i32, p]
    L.register_free.restype = None
    L.register_free.argtypes = [p]
    L.register_cached_bytes.restype = i64
    L.register_cached_bytes.argtypes = []
    L.so3_super_fibonacci.restype = ctypes.c_int
    L.so3_super_fibonacci.argtypes = [i32, p, p]
    L.so3_geoball_sf.restype = ctypes.c_int
    L.so3_geoball_sf.argtypes = [i32, p, ctypes.c_double, ctypes.c_double, p, p]
    L.so3_geoball_sf_noalloc.restype = ctypes.c_int
    L.so3_geoball_sf_noalloc.argtypes = [i32, p, ctypes.c_double, ctypes.c_double, p, p]
    L.register_linear_edge.restype = ctypes.c_int
    L.register_linear_edge.argtypes = [p, i32, ctypes.POINTER(reg_probe), p, i32, p, ctypes.c_double, ctypes.c_double,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    L.register_set_rotations.restype = ctypes.c_int
    L.register_set_rotations.argtypes = [p, p, i32]
    L.register_release_cached.restype = None
    L.register_release_cached.argtypes = []
    L.register_last_error.restype = ctypes.c_char_p
    L.register_last_error.argtypes = []
    L.register_info.restype = ctypes.c_int
    L.register_info.argtypes = [p, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64),
                                ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.register_debug_object_grid.restype = ctypes.c_int
    L.register_debug_object_grid.argtypes = [p, p, p]
    L.register_debug_swept.restype = ctypes.c_int
    L.register_debug_swept.argtypes = [p, p]
    L.register_debug_swept_reach.restype = ctypes.c_int
    L.register_debug_swept_reach.argtypes = [p, ctypes.POINTER(i64)]
    L.register_debug_correlation.restype = ctypes.c_int
    L.register_debug_correlation.argtypes = [p, i32, p]
    L.register_set_grids.restype = ctypes.c_int
    L.register_set_grids.argtypes = [p, p, p]
    L.register_search_stats.restype = ctypes.c_int
    L.register_search_stats.argtypes = [p] + [ctypes.POINTER(i64)] * 5
    L.register_set_timing.restype = ctypes.c_int
    L.register_set_timing.argtypes = [p, i32]
    L.register_get_timing.restype = ctypes.c_int
    L.register_get_timing.argtypes = [p, p, p, p]
    L.refine_se3.restype = ctypes.c_int
    L.refine_se3.argtypes = [p, p, i32, p, p, p]
    L.refine_se3_lbfgsb.restype = ctypes.c_int
    L.refine_se3_lbfgsb.argtypes = [p, p, i32, p, p, p]
    L.register_debug_distance.restype = ctypes.c_int
    L.register_debug_distance.argtypes = [p, p, p, p]
    L.register_refine_stats.restype = ctypes.c_int
    L.register_refine_stats.argtypes = [p, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.register_server_create.restype = ctypes.c_int
    L.register_server_create.argtypes = [ctypes.POINTER(reg_server_cfg), ctypes.POINTER(p)]
    L.register_server_destroy.restype = None
    L.register_server_destroy.argtypes = [p]
    L.register_submit.restype = ctypes.c_int
    L.register_submit.argtypes = [p, ctypes.POINTER(reg_request), ctypes.POINTER(ctypes.c_uint64)]
    L.register_poll.restype = ctypes.c_int
    L.register_poll.argtypes = [p, ctypes.c_uint64, ctypes.POINTER(reg_result)]
    L.register_wait.restype = ctypes.c_int
    L.register_wait.argtypes = [p, ctypes.c_uint64, i64, ctypes.POINTER(reg_result)]
    L.register_server_stats.restype = ctypes.c_int
    L.register_server_stats.argtypes = [p, ctypes.POINTER(reg_server_stats)]
    L.register_server_last_error.restype = ctypes.c_char_p
    L.register_server_last_error.argtypes = []
    L.register_batch_create.restype = ctypes.c_int
    L.register_batch_create.argtypes = [p, i32, i32, i32, i32, i32, ctypes.POINTER(p)]
    L.register_batch_run.restype = ctypes.c_int
    L.register_batch_run.argtypes = [p]
    L.register_batch_outputs.restype = ctypes.c_int
    L.register_batch_outputs.argtypes = [p, i32, p, p, p, p, p]
    L.register_batch_free.restype = None
    L.register_batch_free.argtypes = [p]
    L.register_autotune.restype = ctypes.c_int
    L.register_autotune.argtypes = [p, i32, ctypes.POINTER(i32)]
    L.register_tuned_batch.restype = ctypes.c_int
    L.register_tuned_batch.argtypes = [i32]
    L.register_tuned_schedule.restype = ctypes.c_int
    L.register_tuned_schedule.argtypes = [i32, p]
    L.register_tune_save.restype = ctypes.c_int
    L.register_tune_save.argtypes = [ctypes.c_char_p]
    L.register_tune_load.restype = ctypes.c_int
    L.register_tune_load.argtypes = [ctypes.c_char_p]
    _lib = L
    return L


def register_last_error() -> str:
    return load_library().register_last_error().decode()


def _check(rc: int):
    if rc != REG_OK:
        raise RegError(rc, register_last_error())


def _torch():
    import torch
    return torch


def _dev(x, dtype):
    """A contiguous device tensor of the given dtype (copies host data in)."""
    torch = _torch()
    if x is None:
        return None
    if not isinstance(x, torch.Tensor):
        x = torch.from_numpy(np.ascontiguousarray(x))
    return x.to(device="cuda", dtype=dtype).contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


@dataclass
class Handle:
    ptr: ctypes.c_void_p
    n: int
    m: int
    H: int
    batch: int
    n_rot: int
    stream: object

    def __del__(self):
        try:
            if self.ptr:
                load_library().register_free(self.ptr)
                self.ptr = None
        except Exception:
            pass


def register_init(vertices, faces, touchable, poses, so3, n: int, h_mm: float, center=(0.0, 0.0, 0.0),
                  radius_mm: float = 0.5, length_mm: float = 8.0, params: dict | None = None, stream=None) -> Handle:
    """Build a registration problem on the device (see register_init in the header)."""
    torch = _torch()
    L = load_library()
    V = _dev(vertices, torch.float32)
    F = _dev(faces, torch.int32)
    T = _dev(touchable, torch.uint8)
    P = _dev(poses, torch.float32)
    Q = _dev(so3, torch.float32)
    mesh = reg_mesh(_ptr(V).value, V.shape[0], _ptr(F).value, F.shape[0], _ptr(T).value if T is not None else None)
    probe = reg_probe(radius_mm, length_mm)
    grid = reg_grid_spec(n, h_mm, (ctypes.c_double * 3)(*[float(c) for c in center]))
    prm = reg_params()
    for k, v in (params or {}).items():
        setattr(prm, "lambda_" if k == "lambda" else k, v)
    st = stream if stream is not None else torch.cuda.current_stream()
    out = ctypes.c_void_p()
    _check(L.register_init(ctypes.byref(mesh), ctypes.byref(probe), _ptr(P), P.shape[0], _ptr(Q), Q.shape[0],
                           ctypes.byref(grid), ctypes.byref(prm), ctypes.c_void_p(st.cuda_stream), ctypes.byref(out)))
    n_, m_, b_, r_ = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    H_ = ctypes.c_int64()
    _check(L.register_info(out, ctypes.byref(n_), ctypes.byref(m_), ctypes.byref(H_), ctypes.byref(b_), ctypes.byref(r_)))
    return Handle(out, n_.value, m_.value, H_.value, b_.value, r_.value, st)


def score_rotations(h: Handle, first: int = 0, count: int | None = None, shift: bool = True, pose: bool = True,
                    out=None):
    """(scores f32 [count], shifts i32 [count,3] | None, poses f64 [count,7] | None) on the device."""
    torch = _torch()
    count = h.n_rot - first if count is None else count
    if out is None:
        sc = torch.empty(count, dtype=torch.float32, device="cuda")
        sh = torch.empty((count, 3), dtype=torch.int32, device="cuda") if shift else None
        po = torch.empty((count, 7), dtype=torch.float64, device="cuda") if pose else None
    else:
        sc, sh, po = out
    _check(load_library().score_rotations(h.ptr, first, count, _ptr(sc), _ptr(sh), _ptr(po)))
    return sc, sh, po


def register_top_k(h: Handle, scores, K: int):
    torch = _torch()
    s = _dev(scores, torch.float32)
    out = torch.empty(K, dtype=torch.int32, device="cuda")
    _check(load_library().register_top_k(h.ptr, _ptr(s), s.shape[0], K, _ptr(out)))
    return out


def register_free(h: Handle):
    if h.ptr:
        load_library().register_free(h.ptr)
        h.ptr = None


def register_info(h: Handle) -> dict:
    return dict(n=h.n, m=h.m, spectrum_elems=h.H, batch=h.batch, n_rot=h.n_rot)


def register_debug_object_grid(h: Handle):
    torch = _torch()
    O = torch.empty((h.n,) * 3, dtype=torch.float32, device="cuda")
    fo = torch.empty((h.n,) * 3, dtype=torch.float32, device="cuda")
    _check(load_library().register_debug_object_grid(h.ptr, _ptr(O), _ptr(fo)))
    return O, fo


def register_debug_swept(h: Handle):
    torch = _torch()
    S = torch.empty((h.m,) * 3, dtype=torch.uint8, device="cuda")
    _check(load_library().register_debug_swept(h.ptr, _ptr(S)))
    return S


def register_debug_swept_reach(h: Handle) -> int:
    """Max over occupied points of S_w of (2x-m)^2 + (2y-m)^2 + (2z-m)^2, as
    the search holds it (REG_ENOTSUP for the rotated-object search)."""
    v = ctypes.c_int64()
    _check(load_library().register_debug_swept_reach(h.ptr, ctypes.byref(v)))
    return v.value


def register_debug_correlation(h: Handle, rot: int):
    torch = _torch()
    C = torch.empty((h.n,) * 3, dtype=torch.float32, device="cuda")
    _check(load_library().register_debug_correlation(h.ptr, rot, _ptr(C)))
    return C


def register_set_grids(h: Handle, O=None, Sw=None):
    torch = _torch()
    Ot = _dev(O, torch.float32) if O is not None else None
    St = _dev(Sw, torch.uint8) if Sw is not None else None
    _check(load_library().register_set_grids(h.ptr, _ptr(Ot), _ptr(St)))
    torch.cuda.current_stream().synchronize()


def register_set_timing(h: Handle, enable: bool = True):
    _check(load_library().register_set_timing(h.ptr, 1 if enable else 0))


def register_get_timing(h: Handle) -> dict:
    """{kernel id: (total ms, launches, rotations)} for kernels 0, 1, 2."""
    ms = (ctypes.c_double * 3)()
    la = (ctypes.c_int64 * 3)()
    ro = (ctypes.c_int64 * 3)()
    _check(load_library().register_get_timing(h.ptr, ms, la, ro))
    return {k: (ms[k], la[k], ro[k]) for k in range(3)}


def register_search_stats(h: Handle) -> dict:
    v = [ctypes.c_int64() for _ in range(5)]
    _check(load_library().register_search_stats(h.ptr, *[ctypes.byref(x) for x in v]))
    return dict(rotations=v[0].value, candidates=v[1].value, overflows=v[2].value, uncertain=v[3].value,
                rescored=v[4].value)


def refine_se3(h: Handle, init_poses, solver: str = "gn"):
    """(poses f64 [K,7], J f64 [K], iters i32 [K]) on the device from K x 7 starts.
    solver: "gn" (damped Gauss-Newton) or "lbfgsb" (L-BFGS-B)."""
    torch = _torch()
    if solver not in ("gn", "lbfgsb"):
        raise ValueError(f"unknown solver {solver!r}")
    ip = _dev(init_poses, torch.float64)
    K = ip.shape[0]
    out = torch.empty((K, 7), dtype=torch.float64, device="cuda")
    J = torch.empty(K, dtype=torch.float64, device="cuda")
    it = torch.empty(K, dtype=torch.int32, device="cuda")
    L = load_library()
    fn = L.refine_se3 if solver == "gn" else L.refine_se3_lbfgsb
    _check(fn(h.ptr, _ptr(ip), K, _ptr(out), _ptr(J), _ptr(it)))
    return out, J, it


def register_debug_distance(h: Handle, R, p, n_poses: int):
    """Distance query at the object pose (R, p): float32 [n_poses, 8] on the device
    (d, witness xyz, normal xyz, face index bits)."""
    torch = _torch()
    Rh = np.ascontiguousarray(R, dtype=np.float64).reshape(9)
    ph = np.ascontiguousarray(p, dtype=np.float64).reshape(3)
    out = torch.empty((n_poses, 8), dtype=torch.float32, device="cuda")
    _check(load_library().register_debug_distance(h.ptr, Rh.ctypes.data_as(ctypes.c_void_p),
                                                  ph.ctypes.data_as(ctypes.c_void_p), _ptr(out)))
    return out


def register_refine_stats(h: Handle) -> dict:
    """Rounds and evaluations of the last refine_se3 call on the handle."""
    r, e = ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().register_refine_stats(h.ptr, ctypes.byref(r), ctypes.byref(e)))
    return dict(rounds=r.value, evaluations=e.value)


# ------------------------------------------------------------------ serving

def _server_check(rc: int):
    if rc != REG_OK:
        raise RegError(rc, load_library().register_server_last_error().decode())


def _result_dict(r: reg_result) -> dict:
    k = r.n_top
    return dict(status=r.status, n_top=k, best_score=r.best_score, best_pose=np.array(r.best_pose[:]),
                best_J=r.best_J, top_rot=np.array(r.top_rot[:k]), top_score=np.array(r.top_score[:k]),
                top_pose=np.array(r.top_pose[:7 * k]).reshape(k, 7),
                refined_pose=np.array(r.refined_pose[:7 * k]).reshape(k, 7), refined_J=np.array(r.refined_J[:k]),
                t_submit_ns=r.t_submit_ns, t_admit_ns=r.t_admit_ns, t_start_ns=r.t_start_ns, t_end_ns=r.t_end_ns,
                footprint_bytes=r.footprint_bytes, error=r.error.decode())


class Server:
    """A registration server (see the serving section of the header)."""

    def __init__(self, max_inflight: int = 4, mode: str = "continuous", hbm_budget_bytes: int = 0,
                 cache_bytes: int = 0, fake_us_per_rotation: float | None = None):
        L = load_library()
        cfg = reg_server_cfg(hbm_budget_bytes, max_inflight, 1 if mode == "serial" else 0, cache_bytes,
                             1 if fake_us_per_rotation is not None else 0, fake_us_per_rotation or 0.0)
        self.ptr = ctypes.c_void_p()
        _server_check(L.register_server_create(ctypes.byref(cfg), ctypes.byref(self.ptr)))

    def submit(self, vertices, faces, touchable, poses, so3, n: int, h_mm: float, center=(0.0, 0.0, 0.0),
               radius_mm: float = 0.5, length_mm: float = 8.0, object_id: int = -1, top_k: int = 16,
               refine=True, params: dict | None = None) -> int:
        """refine: False (none), True or "gn" (Gauss-Newton), "lbfgsb" (L-BFGS-B)."""
        mode = {False: 0, True: 1, "gn": 1, "lbfgsb": 2}.get(refine)
        if mode is None:
            raise ValueError(f"unknown refine mode {refine!r}")
        V = np.ascontiguousarray(vertices, dtype=np.float32)
        F = np.ascontiguousarray(faces, dtype=np.int32)
        T = None if touchable is None else np.ascontiguousarray(touchable, dtype=np.uint8)
        P = np.ascontiguousarray(poses, dtype=np.float32)
        Q = np.ascontiguousarray(so3, dtype=np.float32)
        hp = lambda a: a.ctypes.data_as(ctypes.c_void_p).value if a is not None else None
        prm = reg_params()
        for k, v in (params or {}).items():
            setattr(prm, "lambda_" if k == "lambda" else k, v)
        rq = reg_request(reg_mesh(hp(V), V.shape[0], hp(F), F.shape[0], hp(T)), object_id,
                         reg_probe(radius_mm, length_mm), hp(P), P.shape[0], hp(Q), Q.shape[0],
                         reg_grid_spec(n, h_mm, (ctypes.c_double * 3)(*[float(c) for c in center])), prm, top_k,
                         mode)
        t = ctypes.c_uint64()
        _server_check(load_library().register_submit(self.ptr, ctypes.byref(rq), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """The result dict, or None while the registration runs."""
        r = reg_result()
        rc = load_library().register_poll(self.ptr, ticket, ctypes.byref(r))
        if rc == REG_EAGAIN:
            return None
        _server_check(rc)
        return _result_dict(r)

    def wait(self, ticket: int, timeout_ms: int = -1):
        r = reg_result()
        rc = load_library().register_wait(self.ptr, ticket, timeout_ms, ctypes.byref(r))
        if rc == REG_EAGAIN:
            return None
        _server_check(rc)
        return _result_dict(r)

    def stats(self) -> dict:
        st = reg_server_stats()
        _server_check(load_library().register_server_stats(self.ptr, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in reg_server_stats._fields_}

    def close(self):
        if self.ptr:
            load_library().register_server_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- batching

class Batch:
    """Registrations of several handles captured as one hipGraph (see the
    batching section of the header)."""

    def __init__(self, handles, top_k: int = 16, refine=True, graph_rounds: int = 0, branches: int = 0):
        """refine: False (none), True or "gn" (Gauss-Newton), "lbfgsb" (L-BFGS-B)."""
        mode = {False: 0, True: 1, "gn": 1, "lbfgsb": 2}.get(refine)
        if mode is None:
            raise ValueError(f"unknown refine mode {refine!r}")
        L = load_library()
        self.handles = list(handles)
        arr = (ctypes.c_void_p * len(self.handles))(*[h.ptr.value for h in self.handles])
        self.ptr = ctypes.c_void_p()
        _check(L.register_batch_create(arr, len(self.handles), top_k, mode, graph_rounds, branches,
                                       ctypes.byref(self.ptr)))
        self.top_k = top_k

    def run(self):
        _check(load_library().register_batch_run(self.ptr))

    def outputs(self, i: int) -> dict:
        """Host copies of handle i's outputs of the last run."""
        torch = _torch()
        h = self.handles[i]
        K = min(self.top_k, h.n_rot)
        sc = torch.empty(h.n_rot, dtype=torch.float32, device="cuda")
        po = torch.empty((h.n_rot, 7), dtype=torch.float64, device="cuda")
        tp = torch.empty(K, dtype=torch.int32, device="cuda")
        rf = torch.empty((K, 7), dtype=torch.float64, device="cuda")
        J = torch.empty(K, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        _check(load_library().register_batch_outputs(self.ptr, i, _ptr(sc), _ptr(po), _ptr(tp), _ptr(rf), _ptr(J)))
        return dict(scores=sc.cpu().numpy(), poses=po.cpu().numpy(), top=tp.cpu().numpy(), refined=rf.cpu().numpy(),
                    J=J.cpu().numpy())

    def close(self):
        if self.ptr:
            load_library().register_batch_free(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def register_autotune(h: Handle, max_rotations: int = 512) -> int:
    b = ctypes.c_int32()
    _check(load_library().register_autotune(h.ptr, max_rotations, ctypes.byref(b)))
    return b.value


def register_tuned_batch(n: int) -> int:
    return load_library().register_tuned_batch(n)


PLANE_VARIANTS = ((256, 1), (256, 2), (512, 4), (1024, 4))  # (threads, waves per SIMD) of the plane passes
Z_THREADS = (128, 256, 512)


def register_tuned_schedule(n: int) -> dict:
    """The schedule recorded for canvas edge n (the defaults if none): batch,
    lanes, the plane variants of passes 1 and 3, the z variant, and the tuned
    timings."""
    out = (ctypes.c_double * 9)()
    rc = load_library().register_tuned_schedule(n, out)
    if rc < 0:
        _check(rc)
    v = list(out)
    return {"tuned": rc == 1, "batch": int(v[0]), "lanes": int(v[1]),
            "pass1_workgroup": PLANE_VARIANTS[int(v[2])], "pass3_workgroup": PLANE_VARIANTS[int(v[3])],
            "z_threads": Z_THREADS[int(v[4])], "us_per_rotation": {"pass1": v[5], "z": v[6], "pass3": v[7]},
            "search_ns_per_rotation": v[8]}


def register_tune_save(path: str):
    _check(load_library().register_tune_save(os.fsencode(path)))


def register_tune_load(path: str):
    _check(load_library().register_tune_load(os.fsencode(path)))


# -------------------------------------------------------- orientation samplers

def so3_super_fibonacci(n: int, stream=None):
    """n Super-Fibonacci unit quaternions (scalar first), float32 [n, 4] on the device."""
    torch = _torch()
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(load_library().so3_super_fibonacci(n, _ptr(out), ctypes.c_void_p(st.cuda_stream)))
    return out


def so3_geoball_sf(n: int, q0, theta: float, gamma: float = 0.0, stream=None):
    """n GeoBall-SF unit quaternions in the geodesic ball of radius theta (rad)
    around q0 (scalar first), float32 [n, 4] on the device; gamma 0 means n."""
    torch = _torch()
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    q = np.ascontiguousarray(q0, dtype=np.float64).reshape(4)
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(load_library().so3_geoball_sf(n, q.ctypes.data_as(ctypes.c_void_p), float(theta), float(gamma), _ptr(out),
                                          ctypes.c_void_p(st.cuda_stream)))
    return out


def so3_geoball_sf_noalloc(n: int, q0, theta: float, gamma: float = 0.0, out=None, stream=None):
    """so3_geoball_sf without device allocation in the library: the samples are
    written to `out` (float32 [>= n, 4] on the device; allocated here by torch
    if None) asynchronously on the stream."""
    torch = _torch()
    if out is None:
        out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() or out.numel() < 4 * n:
        raise ValueError("out must be a contiguous float32 device tensor of at least n x 4 values")
    q = np.ascontiguousarray(q0, dtype=np.float64).reshape(4)
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(load_library().so3_geoball_sf_noalloc(n, q.ctypes.data_as(ctypes.c_void_p), float(theta), float(gamma),
                                                 _ptr(out), ctypes.c_void_p(st.cuda_stream)))
    return out


def register_linear_edge(vertices, radius: float, length: float, poses, center, h: float,
                         tau_out1: float = 0.0):
    """(needed, edge): the canvas edge n_o + n_s - 1 at which the circular
    correlation equals the linear one, and the smallest supported edge at least
    that large (0 when none is).  Host arrays."""
    V = np.ascontiguousarray(vertices, dtype=np.float32).reshape(-1, 3)
    P = np.ascontiguousarray(poses, dtype=np.float32).reshape(-1, 7)
    c = np.ascontiguousarray(center, dtype=np.float64).reshape(3)
    probe = reg_probe(float(radius), float(length))
    need, edge = ctypes.c_int32(), ctypes.c_int32()
    rc = load_library().register_linear_edge(V.ctypes.data_as(ctypes.c_void_p), len(V), ctypes.byref(probe),
                                              P.ctypes.data_as(ctypes.c_void_p), len(P),
                                              c.ctypes.data_as(ctypes.c_void_p), float(h), float(tau_out1),
                                              ctypes.byref(need), ctypes.byref(edge))
    if rc != REG_ENOTSUP:
        _check(rc)
    return need.value, edge.value


def register_set_rotations(h: Handle, so3) -> None:
    """Replace the handle's SO(3) sample set (M x 4 unit quaternions)."""
    torch = _torch()
    Q = _dev(so3, torch.float32)
    h.n_rot = 0
    _check(load_library().register_set_rotations(h.ptr, _ptr(Q), Q.shape[0]))
    h.n_rot = int(Q.shape[0])


def register_cached_bytes() -> int:
    """Device bytes held by the library's memory cache (blocks of freed handles)."""
    return load_library().register_cached_bytes()


def register_release_cached() -> None:
    """Return every cached device block to HIP."""
    load_library().register_release_cached()
