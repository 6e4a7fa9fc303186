"""Thin ctypes binding of libibm (include/ibm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libibm.so.  Tensors are torch CUDA (HIP) tensors; shapes and
dtypes are checked here before their device pointers cross the C ABI, so
the kernels never see a buffer smaller than the layout they assume.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_void_p
from typing import Dict, Optional, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibm.so")

IBM_OK, IBM_ERR_ARG, IBM_ERR_OOM, IBM_ERR_DEVICE, IBM_ERR_STATE, IBM_ERR_UNSTABLE = 0, -1, -2, -3, -4, -5
IBM_FP64, IBM_FP32_STORAGE = 0, 1
IBM_CFR, IBM_CPG = 0, 1
IBM_B_EXP, IBM_B_EULER, IBM_B_TAYLOR2 = 0, 1, 2
ERR_NAMES = {IBM_ERR_ARG: "IBM_ERR_ARG", IBM_ERR_OOM: "IBM_ERR_OOM", IBM_ERR_DEVICE: "IBM_ERR_DEVICE",
             IBM_ERR_STATE: "IBM_ERR_STATE", IBM_ERR_UNSTABLE: "IBM_ERR_UNSTABLE"}

EXPORTED = [
    "ibm_create_grid", "ibm_set_geometry", "ibm_set_state", "ibm_get_state", "ibm_step",
    "ibm_solve_pressure", "ibm_stats", "ibm_set_diagnostics", "ibm_get_geometry", "ibm_get_ibm_list",
    "ibm_profile", "ibm_profile_read", "ibm_kernel_name", "ibm_num_kernels", "ibm_device_bytes",
    "ibm_destroy", "ibm_last_error", "ibm_tune_set", "ibm_tune_get", "ibm_autotune", "ibm_wall_shear",
    "ibm_set_wall_velocity", "ibm_set_y_faces", "ibm_stream_copy", "ibm_stream_mix", "ibm_solve_pressure_noalloc",
]
TUNE_PARAMS = {"momentum_planes": 0, "fftz_width": 1, "tri_rows": 2, "graph": 3, "graph_branches": 4,
               "tile_order": 5, "batch": 6, "momentum_cache": 7,
               "momentum_tile": 8}


class IbmGridDesc(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("forcing", c_int32),
                ("b_mode", c_int32), ("ibm", c_int32),
                ("lx", c_double), ("lz", c_double), ("y_lo", c_double), ("y_hi", c_double),
                ("nu", c_double), ("dt", c_double), ("q_target_or_pi", c_double), ("top", c_int32),
                ("projection", c_int32), ("pcg_max_iter", c_int32), ("pcg_tol", c_double)]


class IbmStats(ctypes.Structure):
    _fields_ = [("step", c_int64), ("time", c_double), ("q", c_double), ("pi_last", c_double),
                ("div_max_fullbox", c_double), ("div_max_internal_leak", c_double),
                ("poisson_rel_residual", c_double), ("rhs_mean_removed", c_double), ("ke", c_double),
                ("cfl_max", c_double), ("n_internal", c_int64 * 3), ("n_ibm", c_int64 * 3),
                ("n_p_internal", c_int64), ("nan_flag", c_int32), ("pcg_iters", c_int32)]


class IbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libibm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(hipcc, gfx950); there is no fallback path")
    lib = ctypes.CDLL(path)
    h = c_void_p
    sig = {
        "ibm_create_grid": (c_int32, [POINTER(IbmGridDesc), c_int32, c_int32, c_void_p, POINTER(h)]),
        "ibm_set_geometry": (c_int32, [h, c_int32, c_void_p, c_void_p, c_void_p]),
        "ibm_set_state": (c_int32, [h, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
        "ibm_get_state": (c_int32, [h, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
        "ibm_step": (c_int32, [h, c_int32]),
        "ibm_solve_pressure": (c_int32, [h, c_int32, c_void_p, c_void_p]),
        "ibm_stats": (c_int32, [h, c_int32, POINTER(IbmStats)]),
        "ibm_wall_shear": (c_int32, [h, c_int32, c_void_p, POINTER(c_double)]),
        "ibm_set_wall_velocity": (c_int32, [h, c_int32, c_double, c_double, c_double]),
        "ibm_set_y_faces": (c_int32, [h, c_int32, c_void_p]),
        "ibm_set_diagnostics": (c_int32, [h, c_int32]),
        "ibm_get_geometry": (c_int32, [h, c_int32, c_void_p, POINTER(c_int64)]),
        "ibm_get_ibm_list": (c_int32, [h, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
        "ibm_profile": (c_int32, [h, c_int32]),
        "ibm_profile_read": (c_int32, [h, POINTER(c_double), POINTER(c_int64), c_int32]),
        "ibm_kernel_name": (ctypes.c_char_p, [c_int32]),
        "ibm_num_kernels": (c_int32, []),
        "ibm_device_bytes": (c_int64, [h]),
        "ibm_tune_set": (c_int32, [h, c_int32, c_int32]),
        "ibm_tune_get": (c_int32, [h, c_int32, POINTER(c_int32)]),
        "ibm_autotune": (c_int32, [h, c_int32, POINTER(c_int32)]),
        "ibm_destroy": (c_int32, [h]),
        "ibm_last_error": (ctypes.c_char_p, [h]),
        "ibm_stream_copy": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p]),
        "ibm_stream_mix": (c_int32, [POINTER(c_void_p), c_int32, POINTER(c_void_p), c_int32, c_int64, c_void_p]),
        "ibm_solve_pressure_noalloc": (c_int32, [POINTER(IbmGridDesc), c_int32, c_void_p, c_void_p, c_void_p,
                                                 c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def stream_copy(dst: torch.Tensor, src: torch.Tensor, stream: Optional[torch.cuda.Stream] = None):
    """dst <- src with the library's streaming copy kernel (ibm_stream_copy): contiguous
    device tensors of the same size in bytes (a multiple of 16), on torch's current stream."""
    lib = load_library()
    if dst.device.type != "cuda" or src.device.type != "cuda" or not dst.is_contiguous() or not src.is_contiguous():
        raise TypeError("expected contiguous GPU tensors")
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("dst and src differ in size")
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    rc = lib.ibm_stream_copy(c_void_p(_ptr(dst)), c_void_p(_ptr(src)), nb, c_void_p(st.cuda_stream))
    if rc != IBM_OK:
        raise IbmError(rc, lib.ibm_last_error(None).decode())


def stream_mix(dsts, srcs, stream: Optional[torch.cuda.Stream] = None):
    """Every tensor of dsts <- the element-wise sum of the tensors of srcs (read as FP64)
    with the library's stream-mix kernel (ibm_stream_mix): 1..8 contiguous GPU tensors on
    each side, all of the same size in bytes (a multiple of 16), on torch's current stream."""
    lib = load_library()
    ts = list(dsts) + list(srcs)
    if any(t.device.type != "cuda" or not t.is_contiguous() for t in ts):
        raise TypeError("expected contiguous GPU tensors")
    nb = ts[0].numel() * ts[0].element_size()
    if any(t.numel() * t.element_size() != nb for t in ts):
        raise ValueError("the tensors differ in size")
    d = (c_void_p * max(1, len(dsts)))(*[_ptr(t) for t in dsts])
    s = (c_void_p * max(1, len(srcs)))(*[_ptr(t) for t in srcs])
    st = stream if stream is not None else torch.cuda.current_stream(ts[0].device)
    rc = lib.ibm_stream_mix(d, len(dsts), s, len(srcs), nb, c_void_p(st.cuda_stream))
    if rc != IBM_OK:
        raise IbmError(rc, lib.ibm_last_error(None).decode())


def solve_pressure_noalloc(c, rhs: torch.Tensor, phi: Optional[torch.Tensor] = None,
                           mean_removed: Optional[torch.Tensor] = None,
                           stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """ibm_solve_pressure_noalloc: the full-box pressure solve of the grid of case c
    (uniform wall-normal spacing) with the library's fixed work area.  rhs (and phi, if
    given) are contiguous GPU tensors of shape (ny-1, nz, nx) in float64 or float32 (the
    precision follows their dtype); mean_removed, if given, a GPU float64 tensor of one
    element.  Enqueued on torch's current stream; allocates no device memory in the library
    (phi is allocated here by torch when not given)."""
    lib = load_library()
    if getattr(c, "y_faces", None) is not None:
        raise ValueError("the allocation-free solve takes a uniform wall-normal grid (no y_faces)")
    shape = (c.ny - 1, c.nz, c.nx)
    if rhs.device.type != "cuda" or tuple(rhs.shape) != shape or not rhs.is_contiguous():
        raise ValueError(f"rhs must be a contiguous GPU tensor of shape {shape}")
    if rhs.dtype not in (torch.float64, torch.float32):
        raise TypeError("rhs must be float64 or float32")
    if phi is None:
        phi = torch.empty_like(rhs)
    if phi.device.type != "cuda" or tuple(phi.shape) != shape or phi.dtype != rhs.dtype or not phi.is_contiguous():
        raise ValueError("phi must match rhs")
    mp = None
    if mean_removed is not None:
        if mean_removed.device.type != "cuda" or mean_removed.dtype != torch.float64 or mean_removed.numel() < 1:
            raise ValueError("mean_removed must be a GPU float64 tensor")
        mp = c_void_p(_ptr(mean_removed))
    prec = IBM_FP64 if rhs.dtype == torch.float64 else IBM_FP32_STORAGE
    st = stream if stream is not None else torch.cuda.current_stream(rhs.device)
    d = _desc(c, True)
    rc = lib.ibm_solve_pressure_noalloc(ctypes.byref(d), prec, c_void_p(_ptr(rhs)), c_void_p(_ptr(phi)), mp,
                                        c_void_p(st.cuda_stream))
    if rc != IBM_OK:
        raise IbmError(rc, lib.ibm_last_error(None).decode())
    return phi


def _desc(c, ibm: bool) -> IbmGridDesc:
    return IbmGridDesc(c.nx, c.ny, c.nz, c.forcing, c.b_mode, 1 if ibm else 0, c.lx, c.lz, c.y_lo, c.y_hi, c.nu,
                       c.dt, c.q_target_or_pi, int(getattr(c, "top", 0)), int(getattr(c, "projection", 0)),
                       int(getattr(c, "pcg_max_iter", 0)), float(getattr(c, "pcg_tol", 0.0)))


class IbmGrid:
    """One channel instance, or an ensemble of independent instances (per-instance calls
    take `inst`), on the current HIP device and torch's current stream."""

    def __init__(self, nx: int, ny: int, nz: int, lx: float, lz: float, y_lo: float, y_hi: float,
                 nu: float, dt: float, forcing: int = IBM_CFR, q_target_or_pi: float = 0.0,
                 b_mode: int = IBM_B_EXP, ibm: bool = True, precision: str = "fp64",
                 stream: Optional[torch.cuda.Stream] = None, _descs=None):
        self.lib = load_library()
        if precision not in ("fp64", "fp32"):
            raise ValueError("precision must be 'fp64' or 'fp32'")
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if _descs is None:
            _descs = [IbmGridDesc(nx, ny, nz, forcing, b_mode, 1 if ibm else 0, lx, lz, y_lo, y_hi, nu, dt,
                                  q_target_or_pi)]
        n = len(_descs)
        self.descs = (IbmGridDesc * n)(*_descs)
        self.n_inst = n
        self.dims = [(d.nx, d.ny, d.nz) for d in _descs]
        self.nx, self.ny, self.nz = self.dims[0]
        self.shape = (self.ny - 1, self.nz, self.nx)
        self._h = c_void_p()
        rc = self.lib.ibm_create_grid(self.descs, n, IBM_FP64 if precision == "fp64" else IBM_FP32_STORAGE,
                                      c_void_p(self.stream.cuda_stream), ctypes.byref(self._h))
        self._check(rc, None)

    @classmethod
    def from_case(cls, c, precision: str = "fp64", ibm: bool = True, **kw) -> "IbmGrid":
        g = cls(0, 0, 0, 0, 0, 0, 0, 0, 0, precision=precision, _descs=[_desc(c, ibm)], **kw)
        if getattr(c, "y_faces", None) is not None:
            g.set_y_faces(c.y_faces)
        return g

    @classmethod
    def ensemble(cls, cases, precision: str = "fp32", ibm: bool = True, **kw) -> "IbmGrid":
        """Independent instances of ragged sizes advanced together by step()."""
        g = cls(0, 0, 0, 0, 0, 0, 0, 0, 0, precision=precision, _descs=[_desc(c, ibm) for c in cases], **kw)
        for i, c in enumerate(cases):
            if getattr(c, "y_faces", None) is not None:
                g.set_y_faces(c.y_faces, inst=i)
        return g

    def shape_of(self, inst: int = 0):
        nx, ny, nz = self.dims[inst]
        return (ny - 1, nz, nx)

    # -- helpers ---------------------------------------------------------------------------
    def _check(self, rc: int, h=-1):
        if rc != IBM_OK:
            hh = self._h if h == -1 else h
            msg = self.lib.ibm_last_error(hh).decode()
            raise IbmError(rc, msg)

    def _field(self, t: torch.Tensor, shape, dtype) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError("expected a torch tensor on the GPU")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        if t.dtype != dtype:
            raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
        return t.contiguous()

    def empty(self, inst: int = 0) -> torch.Tensor:
        return torch.empty(self.shape_of(inst), dtype=self.dtype, device=self.device)

    # -- API -------------------------------------------------------------------------------
    def set_geometry(self, sdf_u: torch.Tensor, sdf_v: torch.Tensor, sdf_w: torch.Tensor, inst: int = 0):
        nx, ny, nz = self.dims[inst]
        su = self._field(sdf_u, (ny + 1, nz, nx), torch.float64)
        sv = self._field(sdf_v, (ny, nz, nx), torch.float64)
        sw = self._field(sdf_w, (ny + 1, nz, nx), torch.float64)
        self._check(self.lib.ibm_set_geometry(self._h, inst, _ptr(su), _ptr(sv), _ptr(sw)))

    def set_state(self, u, v, w, p, inst: int = 0):
        ts = [self._field(t, self.shape_of(inst), self.dtype) for t in (u, v, w, p)]
        self._check(self.lib.ibm_set_state(self._h, inst, *[_ptr(t) for t in ts]))
        if not hasattr(self, "_keep"):
            self._keep = {}
        self._keep[inst] = ts   # keep the sources alive until the stream-ordered copies ran

    def get_state(self, inst: int = 0) -> Tuple[torch.Tensor, ...]:
        out = [self.empty(inst) for _ in range(4)]
        self._check(self.lib.ibm_get_state(self._h, inst, *[_ptr(t) for t in out]))
        return tuple(out)

    def step(self, nsteps: int = 1):
        self._check(self.lib.ibm_step(self._h, int(nsteps)))

    def solve_pressure(self, rhs: torch.Tensor, inst: int = 0) -> torch.Tensor:
        r = self._field(rhs, self.shape_of(inst), self.dtype)
        phi = self.empty(inst)
        self._check(self.lib.ibm_solve_pressure(self._h, inst, _ptr(r), _ptr(phi)))
        return phi

    def set_diagnostics(self, on: bool = True):
        self._check(self.lib.ibm_set_diagnostics(self._h, 1 if on else 0))

    def stats(self, raise_unstable: bool = False, inst: int = 0) -> Dict:
        s = IbmStats()
        rc = self.lib.ibm_stats(self._h, inst, ctypes.byref(s))
        if rc != IBM_OK and (rc != IBM_ERR_UNSTABLE or raise_unstable):
            self._check(rc)
        d = {f: getattr(s, f) for f, _ in IbmStats._fields_ if f not in ("n_internal", "n_ibm")}
        d["n_internal"] = list(s.n_internal)
        d["n_ibm"] = list(s.n_ibm)
        d["unstable"] = rc == IBM_ERR_UNSTABLE
        return d

    def set_y_faces(self, y_faces, inst: int = 0):
        """Stretched wall-normal grid: the ny face positions, increasing from y_lo to y_hi
        (ibm_set_y_faces; a geometry must be given afterwards)."""
        import numpy as np
        a = np.ascontiguousarray(np.asarray(y_faces, dtype=np.float64))
        if a.shape != (self.dims[inst][1],):
            raise ValueError(f"y_faces must hold {self.dims[inst][1]} values, got shape {a.shape}")
        self._check(self.lib.ibm_set_y_faces(self._h, inst, c_void_p(a.ctypes.data)))

    def set_wall_velocity(self, ub: float, vb: float = 0.0, wb: float = 0.0, inst: int = 0):
        """Velocity of the immersed walls (rigid translation; ibm_set_wall_velocity)."""
        self._check(self.lib.ibm_set_wall_velocity(self._h, inst, float(ub), float(vb), float(wb)))

    def wall_shear(self, inst: int = 0) -> Tuple[torch.Tensor, Tuple[float, float, float]]:
        """Spanwise-averaged south-wall shear stress tau(x_i) (device, float64) and
        (tau_0, tau_1c, tau_1s) of the current state (ibm_wall_shear)."""
        tau = torch.empty(self.shape_of(inst)[2], dtype=torch.float64, device=self.device)
        modes = (c_double * 3)()
        self._check(self.lib.ibm_wall_shear(self._h, inst, _ptr(tau), modes))
        return tau, (modes[0], modes[1], modes[2])

    def geometry(self, inst: int = 0) -> Tuple[torch.Tensor, list]:
        tags = torch.empty(self.shape_of(inst), dtype=torch.uint8, device=self.device)
        n = (c_int64 * 3)()
        self._check(self.lib.ibm_get_geometry(self._h, inst, _ptr(tags), n))
        return tags, list(n)

    def ibm_list(self, comp: int, inst: int = 0):
        _, n = self.geometry(inst)
        m = n[comp]
        idx = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        lam = torch.empty(max(m, 1), dtype=torch.float64, device=self.device)
        coef = torch.empty((3, max(m, 1), 2), dtype=torch.float64, device=self.device)
        self._check(self.lib.ibm_get_ibm_list(self._h, inst, comp, _ptr(idx), _ptr(lam), _ptr(coef)))
        return idx[:m], lam[:m], coef[:, :m]

    def kernel_names(self):
        return [self.lib.ibm_kernel_name(k).decode() for k in range(self.lib.ibm_num_kernels())]

    def profile(self, on=True):
        """on: True (all kernels), False (off), an int mask, or a list of kernel names."""
        if on is True:
            mask = -1
        elif on is False or on is None:
            mask = 0
        elif isinstance(on, int):
            mask = on
        else:
            names = self.kernel_names()
            mask = 0
            for n in on:
                mask |= 1 << names.index(n)
        self._check(self.lib.ibm_profile(self._h, int(mask)))

    def profile_read(self) -> Dict[str, Tuple[float, int]]:
        nk = self.lib.ibm_num_kernels()
        ms = (c_double * nk)()
        cnt = (c_int64 * nk)()
        self._check(self.lib.ibm_profile_read(self._h, ms, cnt, nk))
        return {self.lib.ibm_kernel_name(k).decode(): (ms[k], cnt[k]) for k in range(nk) if cnt[k] > 0}

    def tune(self, **knobs):
        """Set launch-shape knobs by name (momentum_planes, fftz_width, tri_rows, tile_order,
        graph, graph_branches, batch); 0 = automatic."""
        for k, v in knobs.items():
            self._check(self.lib.ibm_tune_set(self._h, TUNE_PARAMS[k], int(v)))

    def tuning(self) -> Dict[str, int]:
        out = {}
        for k, pid in TUNE_PARAMS.items():
            v = c_int32()
            self._check(self.lib.ibm_tune_get(self._h, pid, ctypes.byref(v)))
            out[k] = v.value
        return out

    def autotune(self, steps_per_trial: int = 2) -> Dict[str, int]:
        """Run the library's autotuner (state is saved and restored) and return the choice."""
        names = ["momentum_planes", "fftz_width", "tri_rows", "tile_order"]
        ch = (c_int32 * len(names))()
        self._check(self.lib.ibm_autotune(self._h, int(steps_per_trial), ch))
        return dict(zip(names, list(ch)))

    def device_bytes(self) -> int:
        return int(self.lib.ibm_device_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self.lib.ibm_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
