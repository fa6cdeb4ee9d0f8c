"""Python binding of the mpois C ABI (include/mpois.h).

Argument marshalling only: every step of a solve runs in the HIP kernels of
libmpois.so.  PyTorch supplies device memory and streams.  There is no CPU
fallback: if the library is missing or no GPU is present, calls raise.

    plan = Plan((512, 512, 512), (h, h, h), ("N", "N", "N"), ("v", "v", "v"),
                approx="fd", prec="f32r", max_iter=2)
    plan.solve(rhs, phi)           # torch float64 tensors on the GPU
    plan.info()                    # {"iters", "rel_resid", "zero_mode_rhs"}
"""

import ctypes
import os

import numpy as np

__all__ = ["Plan", "BatchPlan", "MpoisError", "axis_eigenvalues", "axis_plan", "validate", "library_path",
           "load_library", "STATUS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBNAME = "libmpois.so"

BC = {"P": 0, "D": 1, "N": 2}
AXIS_CODE = {"P": 0, "D": 1, "N": 2, "DN": 3, "ND": 4}  # axis codes of the host helpers
GRID = {"v": 0, "s": 1}
APPROX = {"ps": 0, "fd": 1}
PREC = {"f64": 0, "f32": 1, "f32r": 2}
FLAG_GRAPH = 1
FLAG_TUNE = 2
FLAG_PROFILE = 4
FLAG_F64_ARITH = 8
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "out of device memory", 4: "device error",
          5: "refinement did not reach rtol", 6: "non-finite residual"}
KIND_NAMES = ["R2HC", "HC2R", "DCT-II", "DCT-III", "DST-II", "DST-III", "DCT-I", "DST-I", "DST-IV", "DCT-IV"]


class MpoisError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: mpois status {status} ({STATUS.get(status, '?')})")


class GridDesc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("h", ctypes.c_double * 3),
                ("bc", (ctypes.c_int * 2) * 3), ("grid", ctypes.c_int * 3), ("shift", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("rel_resid", ctypes.c_double), ("zero_mode_rhs", ctypes.c_double)]


_lib = None


def library_path():
    return os.path.join(_HERE, _LIBNAME)


def load_library():
    """Load libmpois.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1409_8116_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.mpois_plan_create.argtypes = [ctypes.POINTER(GridDesc), ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_uint, ctypes.POINTER(P)]
    lib.mpois_plan_create_batch.argtypes = [ctypes.POINTER(GridDesc), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_double, ctypes.c_int, ctypes.c_uint, ctypes.POINTER(P)]
    lib.mpois_execute.argtypes = [P, P, P, P]
    lib.mpois_execute_batch.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), P]
    lib.mpois_execute_noalloc.argtypes = [P, P, P, P]
    lib.mpois_execute_view.argtypes = [P, P, ctypes.POINTER(ctypes.c_int64), P, ctypes.POINTER(ctypes.c_int64), P]
    lib.mpois_project.argtypes = [P, ctypes.POINTER(P), P, ctypes.c_double, P, P]
    lib.mpois_get_info.argtypes = [P, P, ctypes.POINTER(Info)]
    lib.mpois_destroy.argtypes = [P]
    lib.mpois_workspace_bytes.argtypes = [P]
    lib.mpois_workspace_bytes.restype = ctypes.c_size_t
    lib.mpois_profile.argtypes = [P, P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.mpois_status_string.argtypes = [ctypes.c_int]
    lib.mpois_status_string.restype = ctypes.c_char_p
    lib.mpois_validate.argtypes = [ctypes.POINTER(GridDesc), ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.mpois_axis_eigenvalues.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                           ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    lib.mpois_axis_plan.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64] + [ctypes.POINTER(ctypes.c_int)] * 5 + \
        [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.mpois_kernel_shape.argtypes = [ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 4
    for name in ("mpois_kernel_shape", "mpois_plan_create", "mpois_plan_create_batch", "mpois_execute", "mpois_execute_batch",
                 "mpois_execute_noalloc", "mpois_execute_view", "mpois_project",
                 "mpois_get_info", "mpois_destroy", "mpois_validate", "mpois_axis_eigenvalues", "mpois_axis_plan",
                 "mpois_profile"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def make_desc(shape, h, bc, grid, shift=0.0):
    """Descriptor of one grid.  bc[i]: "P", "D", "N" (both faces), or a pair of
    face conditions such as ("D", "N") or the string "DN" (low face first)."""
    d = GridDesc()
    d.ndim = len(shape)
    if not 1 <= d.ndim <= 3:
        raise ValueError("ndim must be 1..3")
    for i, n in enumerate(shape):
        d.n[i] = int(n)
        d.h[i] = float(h[i])
        b = bc[i]
        if isinstance(b, str):
            lo, hi = (b, b) if len(b) == 1 else (b[0], b[1])
        else:
            lo, hi = b
        d.bc[i][0] = BC[lo]
        d.bc[i][1] = BC[hi]
        d.grid[i] = GRID[grid[i]]
    d.shift = float(shift)
    return d


def validate(shape, h, bc, grid, approx="fd", prec="f64", max_iter=1, shift=0.0):
    """Status code of mpois_validate (host only)."""
    return load_library().mpois_validate(ctypes.byref(make_desc(shape, h, bc, grid, shift)), APPROX[approx],
                                         PREC[prec], int(max_iter))


def axis_eigenvalues(bc, grid, approx, n, h):
    """Per-axis eigenvalues the library uses (Table 3 or 4), FP64, host only.
    bc: "P", "D", "N", or "DN" / "ND" for different faces."""
    out = np.zeros(int(n), dtype=np.float64)
    st = load_library().mpois_axis_eigenvalues(AXIS_CODE[bc], GRID[grid], APPROX[approx], int(n), float(h),
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if st:
        raise MpoisError(st, "axis_eigenvalues")
    return out


def axis_plan(bc, grid, n):
    """How the library transforms one axis (host only)."""
    vals = [ctypes.c_int() for _ in range(5)]
    rad = (ctypes.c_int * 32)()
    nr = ctypes.c_int()
    st = load_library().mpois_axis_plan(AXIS_CODE[bc], GRID[grid], int(n), ctypes.byref(vals[0]), ctypes.byref(vals[1]),
                                        ctypes.byref(vals[2]), ctypes.byref(vals[3]), rad, 32, ctypes.byref(nr))
    if st:
        raise MpoisError(st, "axis_plan")
    return {"forward": KIND_NAMES[vals[0].value], "backward": KIND_NAMES[vals[1].value], "M": vals[2].value,
            "P": vals[3].value, "radices": list(rad[:nr.value])}


def kernel_shape_name(cfg):
    """Readable name of a line-transform kernel configuration id."""
    v = [ctypes.c_int() for _ in range(4)]
    st = load_library().mpois_kernel_shape(int(cfg), *[ctypes.byref(x) for x in v])
    if st:
        return f"line_pass#{cfg}"
    t = "double" if v[0].value == 8 else "float"
    if cfg >= 300:
        return f"plane_pass#{cfg - 300}<{t}, {v[2].value}, n={v[3].value}>"
    if cfg >= 200:
        return f"line_pass_spec#{cfg - 200}<{t}, {v[1].value}, {v[2].value}, n={v[3].value}>"
    return f"line_pass<{t}, {v[1].value}, {v[2].value}, {v[3].value}>"


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _check_tensor(t, shape, dtype, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


class Plan:
    """One grid: mpois_plan_create / mpois_execute / mpois_destroy."""

    def __init__(self, shape, h, bc, grid, approx="fd", prec="f64", rtol=0.0, max_iter=2, graph=False, tune=False,
                 profile=False, f64_arith=False, shift=0.0):
        self.lib = load_library()
        self.shape = tuple(int(n) for n in shape)
        self.prec = prec
        self.bc = tuple(bc)
        flags = (FLAG_GRAPH if graph else 0) | (FLAG_TUNE if tune else 0) | (FLAG_PROFILE if profile else 0) | \
            (FLAG_F64_ARITH if f64_arith else 0)
        self._desc = make_desc(shape, h, bc, grid, shift)
        handle = ctypes.c_void_p()
        st = self.lib.mpois_plan_create(ctypes.byref(self._desc), APPROX[approx], PREC[prec], float(rtol),
                                        int(max_iter), flags, ctypes.byref(handle))
        if st:
            raise MpoisError(st, "mpois_plan_create")
        self._h = handle

    @classmethod
    def from_desc(cls, d, prec="f64", **kw):
        kw.setdefault("shift", d.get("shift", 0.0))
        return cls(d["shape"], d["h"], d["bc"], d["grid"], approx=d["approx"], prec=prec, **kw)

    @property
    def dtype(self):
        import torch
        return torch.float32 if self.prec == "f32" else torch.float64

    def solve(self, rhs, phi=None, stream=None):
        import torch
        _check_tensor(rhs, self.shape, self.dtype, "rhs")
        if phi is None:
            phi = torch.empty_like(rhs)
        _check_tensor(phi, self.shape, self.dtype, "phi")
        st = self.lib.mpois_execute(self._h, ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                                    _stream_ptr(stream))
        if st:
            raise MpoisError(st, "mpois_execute")
        return phi

    def solve_view(self, rhs, phi, stream=None):
        """mpois_execute_view: rhs and phi may be strided views (e.g. the interior
        of halo-padded tensors, t[1:-1, 1:-1]) of this plan's shape and dtype."""
        import torch
        for t, what in ((rhs, "rhs"), (phi, "phi")):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != self.dtype:
                raise TypeError(f"{what} must be a CUDA (HIP) tensor of {self.dtype}")
            if tuple(t.shape) != self.shape:
                raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {self.shape}")
        nd = len(self.shape)
        rs = (ctypes.c_int64 * nd)(*rhs.stride())
        ps = (ctypes.c_int64 * nd)(*phi.stride())
        st = self.lib.mpois_execute_view(self._h, ctypes.c_void_p(rhs.data_ptr()), rs, ctypes.c_void_p(phi.data_ptr()),
                                         ps, _stream_ptr(stream))
        if st:
            raise MpoisError(st, "mpois_execute_view")
        return phi

    def velocity_shapes(self):
        """Shapes of the staggered velocity components a projection step takes:
        n_d faces along axis d when it is periodic, n_d + 1 otherwise."""
        out = []
        for d, b in enumerate(self.bc):
            per = b == "P" or tuple(b) == ("P", "P")
            out.append(tuple(n + (0 if (e != d or per) else 1) for e, n in enumerate(self.shape)))
        return out

    def project(self, vel, p, adt, phi=None, stream=None):
        """mpois_project: one projection step.  vel (list of ndim tensors, the
        predicted velocity, corrected in place) and p (pressure, p += phi) as
        laid out by velocity_shapes(); returns phi."""
        import torch
        if len(vel) != len(self.shape):
            raise ValueError("one velocity component per axis")
        for u, shp in zip(vel, self.velocity_shapes()):
            _check_tensor(u, shp, self.dtype, "velocity component")
        _check_tensor(p, self.shape, self.dtype, "p")
        if phi is None:
            phi = torch.empty_like(p)
        _check_tensor(phi, self.shape, self.dtype, "phi")
        ptrs = (ctypes.c_void_p * len(vel))(*[u.data_ptr() for u in vel])
        st = self.lib.mpois_project(self._h, ptrs, ctypes.c_void_p(p.data_ptr()), float(adt),
                                    ctypes.c_void_p(phi.data_ptr()), _stream_ptr(stream))
        if st:
            raise MpoisError(st, "mpois_project")
        return phi

    def solve_noalloc(self, rhs, phi, stream=None):
        """mpois_execute_noalloc: the same solve with the library's static
        device scratch instead of the plan's workspace (allocates nothing)."""
        _check_tensor(rhs, self.shape, self.dtype, "rhs")
        _check_tensor(phi, self.shape, self.dtype, "phi")
        st = self.lib.mpois_execute_noalloc(self._h, ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                                            _stream_ptr(stream))
        if st:
            raise MpoisError(st, "mpois_execute_noalloc")
        return phi

    def info(self, stream=None, check=False):
        out = Info()
        st = self.lib.mpois_get_info(self._h, _stream_ptr(stream), ctypes.byref(out))
        if st and (check or st not in (5, 6)):
            raise MpoisError(st, "mpois_get_info")
        return {"iters": out.iters, "rel_resid": out.rel_resid, "zero_mode_rhs": out.zero_mode_rhs, "status": st}

    @property
    def workspace_bytes(self):
        return int(self.lib.mpois_workspace_bytes(self._h))

    def profile(self, stream=None):
        """Per-launch records of the last execute of a profiling plan:
        list of {"kernel", "ms", "bytes"}."""
        cap = 256
        ms = (ctypes.c_double * cap)()
        by = (ctypes.c_double * cap)()
        kid = (ctypes.c_int * cap)()
        cnt = ctypes.c_int()
        st = self.lib.mpois_profile(self._h, _stream_ptr(stream), cap, ms, by, kid, ctypes.byref(cnt))
        if st:
            raise MpoisError(st, "mpois_profile")
        return [{"kernel": kid[i], "ms": ms[i], "bytes": by[i]} for i in range(min(cap, cnt.value))]

    def close(self):
        if getattr(self, "_h", None):
            self.lib.mpois_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """Many independent grids of one ndim: mpois_plan_create_batch / mpois_execute_batch."""

    def __init__(self, descs, prec="f64", approx=None, rtol=0.0, max_iter=2, graph=False, tune=False,
                 f64_arith=False):
        self.lib = load_library()
        self.descs = list(descs)
        self.prec = prec
        approx = approx or self.descs[0]["approx"]
        arr = (GridDesc * len(self.descs))()
        for i, d in enumerate(self.descs):
            arr[i] = make_desc(d["shape"], d["h"], d["bc"], d["grid"], d.get("shift", 0.0))
        self._arr = arr
        flags = (FLAG_GRAPH if graph else 0) | (FLAG_TUNE if tune else 0) | (FLAG_F64_ARITH if f64_arith else 0)
        handle = ctypes.c_void_p()
        st = self.lib.mpois_plan_create_batch(arr, len(self.descs), APPROX[approx], PREC[prec], float(rtol),
                                              int(max_iter), flags, ctypes.byref(handle))
        if st:
            raise MpoisError(st, "mpois_plan_create_batch")
        self._h = handle

    def solve(self, rhs_list, phi_list, stream=None):
        import torch
        dtype = torch.float32 if self.prec == "f32" else torch.float64
        if len(rhs_list) != len(self.descs) or len(phi_list) != len(self.descs):
            raise ValueError("one rhs and one phi per grid")
        for d, r, p in zip(self.descs, rhs_list, phi_list):
            _check_tensor(r, d["shape"], dtype, "rhs")
            _check_tensor(p, d["shape"], dtype, "phi")
        n = len(self.descs)
        rp = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhs_list])
        pp = (ctypes.c_void_p * n)(*[p.data_ptr() for p in phi_list])
        st = self.lib.mpois_execute_batch(self._h, rp, pp, _stream_ptr(stream))
        if st:
            raise MpoisError(st, "mpois_execute_batch")
        return phi_list

    def info(self, stream=None):
        out = Info()
        st = self.lib.mpois_get_info(self._h, _stream_ptr(stream), ctypes.byref(out))
        if st not in (0, 5, 6):
            raise MpoisError(st, "mpois_get_info")
        return {"iters": out.iters, "rel_resid": out.rel_resid, "zero_mode_rhs": out.zero_mode_rhs, "status": st}

    def close(self):
        if getattr(self, "_h", None):
            self.lib.mpois_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
