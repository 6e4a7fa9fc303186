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
    "ibm_destroy", "ibm_last_error",
]


class IbmGridDesc(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("forcing", c_int32),
                ("b_mode", c_int32), ("ibm", c_int32),
                ("lx", c_double), ("lz", c_double), ("y_lo", c_double), ("y_hi", c_double),
                ("nu", c_double), ("dt", c_double), ("q_target_or_pi", c_double)]


class IbmStats(ctypes.Structure):
    _fields_ = [("step", c_int64), ("time", c_double), ("q", c_double), ("pi_last", c_double),
                ("div_max_fullbox", c_double), ("div_max_internal_leak", c_double),
                ("poisson_rel_residual", c_double), ("rhs_mean_removed", c_double), ("ke", c_double),
                ("cfl_max", c_double), ("n_internal", c_int64 * 3), ("n_ibm", c_int64 * 3),
                ("n_p_internal", c_int64), ("nan_flag", c_int32), ("reserved", c_int32)]


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
        "ibm_set_diagnostics": (c_int32, [h, c_int32]),
        "ibm_get_geometry": (c_int32, [h, c_int32, c_void_p, POINTER(c_int64)]),
        "ibm_get_ibm_list": (c_int32, [h, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
        "ibm_profile": (c_int32, [h, c_int32]),
        "ibm_profile_read": (c_int32, [h, POINTER(c_double), POINTER(c_int64), c_int32]),
        "ibm_kernel_name": (ctypes.c_char_p, [c_int32]),
        "ibm_num_kernels": (c_int32, []),
        "ibm_device_bytes": (c_int64, [h]),
        "ibm_destroy": (c_int32, [h]),
        "ibm_last_error": (ctypes.c_char_p, [h]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


class IbmGrid:
    """One channel instance on the current HIP device and torch's current stream."""

    def __init__(self, nx: int, ny: int, nz: int, lx: float, lz: float, y_lo: float, y_hi: float,
                 nu: float, dt: float, forcing: int = IBM_CFR, q_target_or_pi: float = 0.0,
                 b_mode: int = IBM_B_EXP, ibm: bool = True, precision: str = "fp64",
                 stream: Optional[torch.cuda.Stream] = None):
        self.lib = load_library()
        if precision not in ("fp64", "fp32"):
            raise ValueError("precision must be 'fp64' or 'fp32'")
        self.precision = precision
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.desc = IbmGridDesc(nx, ny, nz, forcing, b_mode, 1 if ibm else 0, lx, lz, y_lo, y_hi, nu, dt,
                                q_target_or_pi)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.shape = (ny - 1, nz, nx)
        self._h = c_void_p()
        rc = self.lib.ibm_create_grid(ctypes.byref(self.desc), 1,
                                      IBM_FP64 if precision == "fp64" else IBM_FP32_STORAGE,
                                      c_void_p(self.stream.cuda_stream), ctypes.byref(self._h))
        self._check(rc, None)

    @classmethod
    def from_case(cls, c, precision: str = "fp64", ibm: bool = True, **kw) -> "IbmGrid":
        return cls(c.nx, c.ny, c.nz, c.lx, c.lz, c.y_lo, c.y_hi, c.nu, c.dt, c.forcing, c.q_target_or_pi,
                   c.b_mode, ibm=ibm, precision=precision, **kw)

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

    def empty(self) -> torch.Tensor:
        return torch.empty(self.shape, dtype=self.dtype, device=self.device)

    # -- API -------------------------------------------------------------------------------
    def set_geometry(self, sdf_u: torch.Tensor, sdf_v: torch.Tensor, sdf_w: torch.Tensor):
        ny, nz, nx = self.ny, self.nz, self.nx
        su = self._field(sdf_u, (ny + 1, nz, nx), torch.float64)
        sv = self._field(sdf_v, (ny, nz, nx), torch.float64)
        sw = self._field(sdf_w, (ny + 1, nz, nx), torch.float64)
        self._check(self.lib.ibm_set_geometry(self._h, 0, _ptr(su), _ptr(sv), _ptr(sw)))

    def set_state(self, u, v, w, p):
        ts = [self._field(t, self.shape, self.dtype) for t in (u, v, w, p)]
        self._check(self.lib.ibm_set_state(self._h, 0, *[_ptr(t) for t in ts]))
        self._keep = ts     # keep the sources alive until the stream-ordered copies ran

    def get_state(self) -> Tuple[torch.Tensor, ...]:
        out = [self.empty() for _ in range(4)]
        self._check(self.lib.ibm_get_state(self._h, 0, *[_ptr(t) for t in out]))
        return tuple(out)

    def step(self, nsteps: int = 1):
        self._check(self.lib.ibm_step(self._h, int(nsteps)))

    def solve_pressure(self, rhs: torch.Tensor) -> torch.Tensor:
        r = self._field(rhs, self.shape, self.dtype)
        phi = self.empty()
        self._check(self.lib.ibm_solve_pressure(self._h, 0, _ptr(r), _ptr(phi)))
        return phi

    def set_diagnostics(self, on: bool = True):
        self._check(self.lib.ibm_set_diagnostics(self._h, 1 if on else 0))

    def stats(self, raise_unstable: bool = False) -> Dict:
        s = IbmStats()
        rc = self.lib.ibm_stats(self._h, 0, ctypes.byref(s))
        if rc != IBM_OK and (rc != IBM_ERR_UNSTABLE or raise_unstable):
            self._check(rc)
        d = {f: getattr(s, f) for f, _ in IbmStats._fields_ if f not in ("n_internal", "n_ibm", "reserved")}
        d["n_internal"] = list(s.n_internal)
        d["n_ibm"] = list(s.n_ibm)
        d["unstable"] = rc == IBM_ERR_UNSTABLE
        return d

    def geometry(self) -> Tuple[torch.Tensor, list]:
        tags = torch.empty(self.shape, dtype=torch.uint8, device=self.device)
        n = (c_int64 * 3)()
        self._check(self.lib.ibm_get_geometry(self._h, 0, _ptr(tags), n))
        return tags, list(n)

    def ibm_list(self, comp: int):
        _, n = self.geometry()
        m = n[comp]
        idx = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        lam = torch.empty(max(m, 1), dtype=torch.float64, device=self.device)
        coef = torch.empty((3, max(m, 1), 2), dtype=torch.float64, device=self.device)
        self._check(self.lib.ibm_get_ibm_list(self._h, 0, comp, _ptr(idx), _ptr(lam), _ptr(coef)))
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
