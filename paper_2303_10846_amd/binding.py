"""Python binding of the cis C ABI (include/cis.h).

Argument marshalling only: every step of an iteration runs in the HIP
kernels of libcis.so.  torch provides the device memory (the
cis_device_buffers of a state) and the HIP stream.  There is no CPU fallback:
if the library is not built, or no GPU is present, creating a Solver raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

FP64 = 0
MIXED = 1
BC_WALL = 1
BC_FARFIELD = 2

_ERRORS = {-1: "CIS_E_INVALID_ARG", -2: "CIS_E_MESH", -3: "CIS_E_DVS", -4: "CIS_E_DEVICE",
           -5: "CIS_E_NONFINITE", -6: "CIS_E_UNSUPPORTED"}

EXPORTS = [
    "cis_last_error", "cis_mesh_create", "cis_mesh_info", "cis_mesh_destroy", "cis_dvs_create", "cis_dvs_destroy",
    "cis_state_required_bytes", "cis_state_create", "cis_state_set_numerics", "cis_state_destroy",
    "cis_state_init_equilibrium", "cis_state_set", "cis_state_get", "cis_iterate", "cis_residual", "cis_moments",
    "cis_wall_heat_flux", "cis_debug_stage", "cis_profile_enable", "cis_profile_read", "cis_state_set_bc",
    "cis_steady_residual", "cis_residual_vjp", "cis_adjoint_required_bytes", "cis_adjoint_solve", "cis_wall_loads",
    "cis_wall_coefficients_of_loads", "cis_wall_coefficients", "cis_iterate_noalloc", "cis_limiter_freeze",
    "cis_mesh_create_cells",
]
STAGE_NAMES = ["recon", "face", "macro", "residual", "micro", "update"]


class CisError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_ERRORS.get(status, status)}: {msg}")
        self.status = status


class Gas(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("R", "gamma", "Z", "delta", "omega0", "omega1", "mu_ref", "omega_vhs",
                                          "T_ref", "C_s")]


class Numerics(C.Structure):
    _fields_ = [("cfl", C.c_double), ("inv_dt", C.c_double), ("cfl_imp", C.c_double), ("lim_K", C.c_double),
                ("snap", C.c_double), ("limiter", C.c_int32), ("n_macro", C.c_int32), ("n_micro", C.c_int32),
                ("reserved", C.c_int32)]


class Bc(C.Structure):
    _fields_ = [("tag", C.c_int32), ("kind", C.c_int32), ("rho", C.c_double), ("U", C.c_double * 3),
                ("T", C.c_double)]


class MeshInfo(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("n_cells", "n_faces", "n_interior", "n_boundary", "n_colors", "max_faces")]


class BufferSizes(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("phi_bytes", "face_bytes", "cell6_bytes", "code_bytes", "total_bytes")]


class AdjointInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("rel_residual", C.c_double)]


class WallFace(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("area", C.c_double), ("n", C.c_double * 3), ("p", C.c_double),
                ("tau", C.c_double * 3), ("q", C.c_double)]


class WallRef(C.Structure):
    _fields_ = [("rho_inf", C.c_double), ("U_inf", C.c_double * 3), ("T_inf", C.c_double), ("A_ref", C.c_double),
                ("L_ref", C.c_double), ("x_ref", C.c_double * 3), ("lift_dir", C.c_double * 3)]


class WallCoef(C.Structure):
    _fields_ = [("Cp", C.c_double), ("Ctau", C.c_double), ("Ch", C.c_double)]


class WallTotals(C.Structure):
    _fields_ = [("force", C.c_double * 3), ("moment", C.c_double * 3), ("heat", C.c_double),
                ("e_drag", C.c_double * 3), ("e_lift", C.c_double * 3), ("CF", C.c_double * 3), ("Cd", C.c_double),
                ("Cl", C.c_double), ("CM", C.c_double * 3), ("Cm", C.c_double), ("CQ", C.c_double)]


class DeviceBuffers(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("G", "R", "dG", "dR", "resG", "resR", "faceG", "faceR", "W", "q", "upwind")]


_lib = None


def lib_path() -> str:
    """The library this process loads: $CIS_LIBRARY if set (alternative builds), else the in-tree build."""
    return os.environ.get("CIS_LIBRARY") or _build.LIB


def load(allow_build: bool = True):
    """Load libcis.so (building it first only if nothing is built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        if not allow_build or path != _build.LIB:
            raise RuntimeError(f"libcis.so is not built ({path}); run paper_2303_10846_amd/build.py")
        _build.build()
    lib = C.CDLL(path)
    P = C.c_void_p
    d = C.POINTER(C.c_double)
    i32 = C.POINTER(C.c_int32)
    i64 = C.POINTER(C.c_int64)
    st = C.c_int32
    lib.cis_last_error.restype = C.c_char_p
    lib.cis_last_error.argtypes = []
    lib.cis_mesh_create.restype = st
    lib.cis_mesh_create.argtypes = [d, C.c_int64, i32, C.c_int64, i32, i32, C.c_int64, i64, C.c_int64,
                                    C.POINTER(P)]
    lib.cis_mesh_create_cells.restype = st
    lib.cis_mesh_create_cells.argtypes = [d, C.c_int64, i32, i32, C.c_int64, i32, i32, C.c_int64, i64, C.c_int64,
                                          C.POINTER(P)]
    lib.cis_mesh_info.restype = st
    lib.cis_mesh_info.argtypes = [P, C.POINTER(MeshInfo)]
    lib.cis_mesh_destroy.restype = None
    lib.cis_mesh_destroy.argtypes = [P]
    lib.cis_dvs_create.restype = st
    lib.cis_dvs_create.argtypes = [d, d, C.c_int64, C.POINTER(P)]
    lib.cis_dvs_destroy.restype = None
    lib.cis_dvs_destroy.argtypes = [P]
    lib.cis_state_required_bytes.restype = st
    lib.cis_state_required_bytes.argtypes = [P, P, C.c_int32, C.POINTER(BufferSizes)]
    lib.cis_state_create.restype = st
    lib.cis_state_create.argtypes = [P, P, C.POINTER(Gas), C.POINTER(Numerics), C.POINTER(Bc), C.c_int32, C.c_int32,
                                     C.POINTER(DeviceBuffers), P, C.POINTER(P)]
    lib.cis_state_set_numerics.restype = st
    lib.cis_state_set_numerics.argtypes = [P, C.POINTER(Numerics)]
    lib.cis_state_destroy.restype = None
    lib.cis_state_destroy.argtypes = [P]
    lib.cis_state_init_equilibrium.restype = st
    lib.cis_state_init_equilibrium.argtypes = [P, d, C.c_int32]
    lib.cis_state_set.restype = st
    lib.cis_state_set.argtypes = [P, P, P, d, d]
    lib.cis_state_get.restype = st
    lib.cis_state_get.argtypes = [P, P, P, d, d]
    lib.cis_iterate.restype = st
    lib.cis_iterate.argtypes = [P, C.c_int32, d]
    lib.cis_limiter_freeze.restype = st
    lib.cis_limiter_freeze.argtypes = [P, P, C.c_int32]
    lib.cis_iterate_noalloc.restype = st
    lib.cis_iterate_noalloc.argtypes = [P, C.c_int32, d]
    lib.cis_residual.restype = st
    lib.cis_residual.argtypes = [P, P, P, d]
    lib.cis_moments.restype = st
    lib.cis_moments.argtypes = [P, d, d]
    lib.cis_wall_heat_flux.restype = st
    lib.cis_wall_heat_flux.argtypes = [P, C.c_int32, d]
    lib.cis_debug_stage.restype = st
    lib.cis_debug_stage.argtypes = [P, C.c_int32, d]
    lib.cis_profile_enable.restype = st
    lib.cis_profile_enable.argtypes = [P, C.c_int32]
    lib.cis_profile_read.restype = st
    lib.cis_profile_read.argtypes = [P, d, i64]
    lib.cis_wall_loads.restype = st
    lib.cis_wall_loads.argtypes = [P, C.c_int32, i64, P, d, d]
    lib.cis_wall_coefficients_of_loads.restype = st
    lib.cis_wall_coefficients_of_loads.argtypes = [P, C.c_int64, C.c_double, C.POINTER(WallRef), P,
                                                   C.POINTER(WallTotals)]
    lib.cis_wall_coefficients.restype = st
    lib.cis_wall_coefficients.argtypes = [P, C.c_int32, C.POINTER(WallRef), i64, P, C.POINTER(WallTotals)]
    lib.cis_state_set_bc.restype = st
    lib.cis_state_set_bc.argtypes = [P, C.POINTER(Bc), C.c_int32]
    lib.cis_steady_residual.restype = st
    lib.cis_steady_residual.argtypes = [P, C.c_int32, P, P, P, P, d]
    lib.cis_residual_vjp.restype = st
    lib.cis_residual_vjp.argtypes = [P, P, P, P, P, C.c_double, C.c_int32, C.c_int32, P, P, P, P, d]
    lib.cis_adjoint_required_bytes.restype = st
    lib.cis_adjoint_required_bytes.argtypes = [P, C.c_int32, i64]
    lib.cis_adjoint_solve.restype = st
    lib.cis_adjoint_solve.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                      C.c_int32, P,
                                      C.c_int64, P, d, d, C.POINTER(AdjointInfo)]
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise CisError(status, _lib.cis_last_error().decode())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _bc_array(bcs):
    return (Bc * len(bcs))(*[Bc(int(b["tag"]), int(b["kind"]), float(b["rho"]), (C.c_double * 3)(*map(float, b["U"])),
                               float(b["T"])) for b in bcs])


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def gas_struct(gas: dict) -> Gas:
    return Gas(*(float(gas[k]) for k in ("R", "gamma", "Z", "delta", "omega0", "omega1", "mu_ref", "omega_vhs",
                                         "T_ref")), float(gas.get("C_s", 0.0)))


def numerics_struct(num: dict) -> Numerics:
    return Numerics(float(num["cfl"]), float(num["inv_dt"]), float(num["cfl_imp"]), float(num["lim_K"]),
                    float(num["snap"]), int(num["limiter"]), int(num["n_macro"]), int(num["n_micro"]), 0)


class Mesh:
    def __init__(self, mesh: dict):
        lib = load()
        self.lib = lib
        xyz = np.ascontiguousarray(mesh["xyz"], dtype=np.float64)
        btag = np.ascontiguousarray(mesh["btag"], dtype=np.int32)
        off = np.ascontiguousarray(mesh["color_offsets"], dtype=np.int64)
        self.color_offsets = off
        h = C.c_void_p()
        ip = C.POINTER(C.c_int32)
        if "cells" in mesh:
            cells = np.ascontiguousarray(mesh["cells"], dtype=np.int32)
            kinds = np.ascontiguousarray(mesh["kinds"], dtype=np.int32)
            bface = np.ascontiguousarray(mesh["bface"], dtype=np.int32)
            _check(lib.cis_mesh_create_cells(_dp(xyz), len(xyz), cells.ctypes.data_as(ip), kinds.ctypes.data_as(ip),
                                             len(cells), bface.ctypes.data_as(ip), btag.ctypes.data_as(ip),
                                             len(bface), off.ctypes.data_as(C.POINTER(C.c_int64)), len(off) - 1,
                                             C.byref(h)))
        else:
            tets = np.ascontiguousarray(mesh["tets"], dtype=np.int32)
            btri = np.ascontiguousarray(mesh["btri"], dtype=np.int32)
            _check(lib.cis_mesh_create(_dp(xyz), len(xyz), tets.ctypes.data_as(ip), len(tets),
                                       btri.ctypes.data_as(ip), btag.ctypes.data_as(ip), len(btri),
                                       off.ctypes.data_as(C.POINTER(C.c_int64)), len(off) - 1, C.byref(h)))
        self.h = h
        info = MeshInfo()
        _check(lib.cis_mesh_info(h, C.byref(info)))
        self.info = info

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.cis_mesh_destroy(self.h)
            self.h = None


class Dvs:
    def __init__(self, u, w):
        lib = load()
        self.lib = lib
        u = np.ascontiguousarray(u, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        h = C.c_void_p()
        _check(lib.cis_dvs_create(_dp(u), _dp(w), len(w), C.byref(h)))
        self.h = h
        self.n = len(w)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.cis_dvs_destroy(self.h)
            self.h = None


class Solver:
    """One state of the scheme on the current GPU (device memory owned by torch tensors).
    row_offset > 0 starts every distribution and face array that many elements past the start of its allocation,
    so that the rows are element-aligned only (the library then runs its scalar kernels instead of the vector
    ones; used to test those paths)."""

    def __init__(self, case: dict, precision: str = "fp64", device: str = "cuda:0", num: dict = None,
                 gas: dict = None, bcs=None, stream=None, row_offset: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("paper_2303_10846_amd needs a ROCm GPU; none is visible")
        lib = load()
        self.lib = lib
        self.torch = torch
        self.device = torch.device(device)
        self.precision = FP64 if precision == "fp64" else MIXED
        self.dtype = torch.float64 if self.precision == FP64 else torch.float32
        self.np_dtype = np.float64 if self.precision == FP64 else np.float32
        self.mesh = Mesh(case["mesh"])
        self.dvs = Dvs(case["u"], case["w"])
        self.gas = dict(case["gas"] if gas is None else gas)
        self.num = dict(case["num"] if num is None else num)
        self.bcs = list(case["bcs"] if bcs is None else bcs)
        self.nc = int(self.mesh.info.n_cells)
        self.nf = int(self.mesh.info.n_faces)
        self.nv = int(self.dvs.n)
        sizes = BufferSizes()
        _check(lib.cis_state_required_bytes(self.mesh.h, self.dvs.h, self.precision, C.byref(sizes)))
        self.sizes = sizes
        with torch.cuda.device(self.device):
            def mk(n):
                if not row_offset:
                    return torch.empty(n, self.nv, dtype=self.dtype, device=self.device)
                flat = torch.empty(n * self.nv + int(row_offset), dtype=self.dtype, device=self.device)
                return flat[int(row_offset):].view(n, self.nv)

            self.G, self.R = mk(self.nc), mk(self.nc)
            self.dG, self.dR = mk(self.nc), mk(self.nc)
            self.resG, self.resR = mk(self.nc), mk(self.nc)
            self.faceG, self.faceR = mk(self.nf), mk(self.nf)
            self.W = torch.zeros(self.nc, 6, dtype=torch.float64, device=self.device)
            self.q = torch.zeros(self.nc, 6, dtype=torch.float64, device=self.device)
            # upwind codes: one byte per (cell, velocity) for 4 face slots, two (int16 storage of uint16) for 6
            self.upwind = torch.empty(self.nc, self.nv, dtype=torch.uint8 if self.mesh.info.max_faces == 4
                                      else torch.int16, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        bufs = DeviceBuffers(*(t.data_ptr() for t in (self.G, self.R, self.dG, self.dR, self.resG, self.resR,
                                                      self.faceG, self.faceR, self.W, self.q, self.upwind)))
        bc_arr = _bc_array(self.bcs)
        self._gas_s = gas_struct(self.gas)
        self._num_s = numerics_struct(self.num)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.cis_state_create(self.mesh.h, self.dvs.h, C.byref(self._gas_s), C.byref(self._num_s), bc_arr,
                                        len(self.bcs), self.precision, C.byref(bufs),
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.cis_state_destroy(self.h)
            self.h = None

    # -- state -------------------------------------------------------------
    def set_numerics(self, **changes):
        self.num.update(changes)
        self._num_s = numerics_struct(self.num)
        _check(self.lib.cis_state_set_numerics(self.h, C.byref(self._num_s)))

    def freeze_limiter(self, values=None, limiter: int = 3):
        """Store limiter values (cis_limiter_freeze) and switch to `limiter` (3: reconstruct with them; 4: also lower
        them where the computed limiter is smaller).  values: None takes those of the current state; otherwise a
        [2, nc, nv] array (G then R), e.g. of another state.  Returns the device tensor of stored values."""
        t = self.torch
        if values is None:
            self.L_frozen = t.empty(2, self.nc, self.nv, dtype=self.dtype, device=self.device)
        else:
            self.L_frozen = t.as_tensor(values).to(device=self.device, dtype=self.dtype).reshape(
                2, self.nc, self.nv).contiguous()
        _check(self.lib.cis_limiter_freeze(self.h, C.c_void_p(self.L_frozen.data_ptr()), 1 if values is None else 0))
        self.set_numerics(limiter=limiter)
        return self.L_frozen

    def unfreeze_limiter(self, limiter: int = 1):
        """Back to a computed limiter (1 by default) and detach the frozen values."""
        self.set_numerics(limiter=limiter)
        _check(self.lib.cis_limiter_freeze(self.h, None, 0))
        self.L_frozen = None

    def init_equilibrium(self, W0):
        W0 = np.ascontiguousarray(W0, dtype=np.float64)
        _check(self.lib.cis_state_init_equilibrium(self.h, _dp(W0), 1 if W0.ndim == 2 else 0))

    def set_state(self, G, R, W, q):
        G = np.ascontiguousarray(G, dtype=self.np_dtype)
        R = np.ascontiguousarray(R, dtype=self.np_dtype)
        W = np.ascontiguousarray(W, dtype=np.float64)
        q = np.ascontiguousarray(q, dtype=np.float64)
        _check(self.lib.cis_state_set(self.h, G.ctypes.data_as(C.c_void_p), R.ctypes.data_as(C.c_void_p), _dp(W),
                                      _dp(q)))

    def get_state(self):
        G = np.empty((self.nc, self.nv), dtype=self.np_dtype)
        R = np.empty((self.nc, self.nv), dtype=self.np_dtype)
        W = np.empty((self.nc, 6))
        q = np.empty((self.nc, 6))
        _check(self.lib.cis_state_get(self.h, G.ctypes.data_as(C.c_void_p), R.ctypes.data_as(C.c_void_p), _dp(W),
                                      _dp(q)))
        return G, R, W, q

    def moments(self):
        W = np.empty((self.nc, 6))
        q = np.empty((self.nc, 6))
        _check(self.lib.cis_moments(self.h, _dp(W), _dp(q)))
        return W, q

    # -- iteration ----------------------------------------------------------
    def iterate(self, n: int = 1) -> np.ndarray:
        hist = np.empty((n, 6))
        _check(self.lib.cis_iterate(self.h, int(n), _dp(hist)))
        return hist

    def iterate_noalloc(self, n: int = 1) -> np.ndarray:
        """iterate() through cis_iterate_noalloc: no device allocation, n <= 4096 per call."""
        hist = np.empty((n, 6))
        _check(self.lib.cis_iterate_noalloc(self.h, int(n), _dp(hist)))
        return hist

    def converge(self, tol: float = 1e-10, max_iter: int = 10000, cfl_schedule=None, chunk: int = 100,
                 callback=None):
        """Iterate until the global average residual (Step 7; the largest of its six components) falls below
        `tol`, the paper's steady-state criterion (1e-10, Sec. 4), or `max_iter` iterations have run.
        cfl_schedule: optional (iteration, cfl_imp) pairs, each applied from that iteration on (a small implicit
        step while a shock forms from rest, a larger one afterwards).  The residual is checked every `chunk`
        iterations; callback(iteration, history) runs after each chunk.  Returns (history, converged): the
        residual history and whether `tol` was reached (False when the run stopped at max_iter)."""
        switch = {int(i): float(c) for i, c in (cfl_schedule or ())}
        hist = []
        done = 0
        while done < max_iter:
            end = min(done + chunk, max_iter)
            while done < end:                   # one chunk, the step changed at its scheduled iterations
                if done in switch:
                    self.set_numerics(cfl_imp=switch[done])
                nxt = min([i for i in switch if done < i < end] + [end])
                hist.append(self.iterate(nxt - done))
                done = nxt
            h = np.concatenate(hist)
            if callback is not None:
                callback(done, h)
            if np.any(h.max(axis=1) < tol):
                return h, True
        return (np.concatenate(hist) if hist else np.empty((0, 6))), False

    def residual(self):
        """Explicit operator: micro flux F (torch, [nc][nv]) for G and R, macro flux F [nc][6] (numpy)."""
        FG = self.torch.empty_like(self.G)
        FR = self.torch.empty_like(self.R)
        Fm = np.empty((self.nc, 6))
        _check(self.lib.cis_residual(self.h, C.c_void_p(FG.data_ptr()), C.c_void_p(FR.data_ptr()), _dp(Fm)))
        return FG, FR, Fm

    def wall_heat_flux(self, tag: int) -> float:
        Q = C.c_double(0.0)
        _check(self.lib.cis_wall_heat_flux(self.h, int(tag), C.byref(Q)))
        return Q.value

    def wall_loads(self, tag: int) -> dict:
        """Per-face wall loads of `tag` (Eqs. 70-72 numerators) and the integrated force and heat load."""
        n = C.c_int64(0)
        _check(self.lib.cis_wall_loads(self.h, int(tag), C.byref(n), None, None, None))
        arr = (WallFace * max(n.value, 1))()
        F = np.zeros(3)
        Q = C.c_double(0.0)
        _check(self.lib.cis_wall_loads(self.h, int(tag), C.byref(n), C.cast(arr, C.c_void_p), _dp(F), C.byref(Q)))
        rec = np.ctypeslib.as_array(C.cast(arr, C.POINTER(C.c_double)), shape=(max(n.value, 1), 12))[: n.value].copy()
        return dict(x=rec[:, 0:3], area=rec[:, 3], n=rec[:, 4:7], p=rec[:, 7], tau=rec[:, 8:11], q=rec[:, 11],
                    force=F, heat=Q.value)

    def wall_coefficients(self, tag: int, rho_inf: float, U_inf, T_inf: float, A_ref: float = None,
                          L_ref: float = 1.0, x_ref=(0.0, 0.0, 0.0), lift_dir=None) -> dict:
        """Wall coefficients of `tag` (cis_wall_coefficients): C_p, C_tau, C_h per face (Eqs. 70-72) and, with
        A_ref, the force, moment and heat-load coefficients; see wall_coefficients() for the keys."""
        ref = _wall_ref(rho_inf, U_inf, T_inf, A_ref, L_ref, x_ref, lift_dir)
        n = C.c_int64(0)
        _check(self.lib.cis_wall_coefficients(self.h, int(tag), C.byref(ref), C.byref(n), None, None))
        coef = (WallCoef * max(n.value, 1))()
        tot = WallTotals()
        _check(self.lib.cis_wall_coefficients(self.h, int(tag), C.byref(ref), C.byref(n), C.cast(coef, C.c_void_p),
                                              C.byref(tot)))
        return _coef_dict(coef, n.value, tot, bool(A_ref))

    def profile(self, enable: bool = True):
        """Enable (and reset) per-stage hipEvent timing of iterate()."""
        _check(self.lib.cis_profile_enable(self.h, 1 if enable else 0))

    def profile_read(self):
        ms = np.zeros(6)
        n = np.zeros(6, dtype=np.int64)
        _check(self.lib.cis_profile_read(self.h, _dp(ms), n.ctypes.data_as(C.POINTER(C.c_int64))))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(STAGE_NAMES)}

    def debug_stage(self, name: str) -> np.ndarray:
        which = dict(dW=0, Wt=1, Fmac=2, tau_t=3)[name]
        out = np.empty(self.nc if name == "tau_t" else (self.nc, 6))
        _check(self.lib.cis_debug_stage(self.h, which, _dp(out)))
        return out

    # -- steady residual, VJP and adjoint (FP64) ------------------------------
    def set_bc(self, bcs):
        """Replace the boundary-condition values (same tags and kinds, same order)."""
        bcs = [dict(b) for b in bcs]
        _check(self.lib.cis_state_set_bc(self.h, _bc_array(bcs), len(bcs)))
        self.bcs = bcs

    def params(self, wall_tag: int, ff_tag: int) -> np.ndarray:
        """p = (T_w of wall_tag, rho_inf and |U_inf| of ff_tag); 0 where the tag is absent."""
        p = np.zeros(3)
        for b in self.bcs:
            if b["tag"] == wall_tag and b["kind"] == BC_WALL:
                p[0] = b["T"]
            if b["tag"] == ff_tag and b["kind"] == BC_FARFIELD:
                p[1] = b["rho"]
                p[2] = float(np.linalg.norm(b["U"]))
        return p

    def set_params(self, p, wall_tag: int, ff_tag: int):
        """Move p = (T_w, rho_inf, |U_inf|); U_inf keeps its direction."""
        bcs = [dict(b) for b in self.bcs]
        for b in bcs:
            if b["tag"] == wall_tag and b["kind"] == BC_WALL:
                b["T"] = float(p[0])
            if b["tag"] == ff_tag and b["kind"] == BC_FARFIELD:
                b["rho"] = float(p[1])
                m = float(np.linalg.norm(b["U"]))
                b["U"] = [u * float(p[2]) / m for u in b["U"]] if m > 0 else list(b["U"])
        self.set_bc(bcs)

    def _fp64_only(self):
        if self.precision != FP64:
            raise CisError(-6, "the steady residual, VJP and adjoint need an FP64 state")

    def steady_residual(self, wall_tag: int = -1):
        """R(x; p) at the current state: (rG, rR, rW, rq) device tensors and J (heat flux into wall_tag)."""
        t = self.torch
        rG, rR = t.empty_like(self.G), t.empty_like(self.R)
        rW, rq = t.empty_like(self.W), t.empty_like(self.q)
        J = C.c_double(0.0)
        _check(self.lib.cis_steady_residual(self.h, int(wall_tag), _ptr(rG), _ptr(rR), _ptr(rW), _ptr(rq),
                                            C.byref(J)))
        return rG, rR, rW, rq, J.value

    def residual_vjp(self, vG=None, vR=None, vW=None, vq=None, cJ: float = 0.0, wall_tag: int = -1,
                     ff_tag: int = -1):
        """(gG, gR, gW, gq) device tensors and gp (numpy [3]) = v^T dR/d(x, p) + cJ dJ/d(x, p)."""
        t = self.torch
        gG, gR = t.empty_like(self.G), t.empty_like(self.R)
        gW, gq = t.empty_like(self.W), t.empty_like(self.q)
        vs = [vG, vR, vW, vq]
        if any(v is not None for v in vs):
            ref = [self.G, self.R, self.W, self.q]
            vs = [(t.zeros_like(r) if v is None else v.to(device=r.device, dtype=t.float64).contiguous())
                  for v, r in zip(vs, ref)]
        gp = np.zeros(3)
        _check(self.lib.cis_residual_vjp(self.h, *[_ptr(v) for v in vs], float(cJ), int(wall_tag), int(ff_tag),
                                         _ptr(gG), _ptr(gR), _ptr(gW), _ptr(gq), _dp(gp)))
        return gG, gR, gW, gq, gp

    def adjoint(self, wall_tag: int, ff_tag: int = -1, restart: int = 60, max_iter: int = 3000,
                rtol: float = 1e-11, precond_pairs: int = 2, macro_pairs: int = 0) -> dict:
        """Discrete adjoint at the current state: dJ/dp for p = (T_w, rho_inf, |U_inf|), J and lambda.
        precond_pairs: Gauss-Seidel pairs of the transposed upwind transport operator as GMRES preconditioner
        (0: its diagonal).  macro_pairs > 0: block preconditioner over (phi, W, q), with that many transposed
        macro-system pairs after the transport sweeps."""
        t = self.torch
        nb = C.c_int64(0)
        _check(self.lib.cis_adjoint_required_bytes(self.h, int(restart), C.byref(nb)))
        work = t.empty(nb.value // 8, dtype=t.float64, device=self.device)
        lam = t.empty(2 * self.nc * self.nv + 12 * self.nc, dtype=t.float64, device=self.device)
        dJdp = np.zeros(3)
        J = C.c_double(0.0)
        info = AdjointInfo()
        _check(self.lib.cis_adjoint_solve(self.h, int(wall_tag), int(ff_tag), int(restart), int(max_iter),
                                          float(rtol), int(precond_pairs), int(macro_pairs), _ptr(work),
                                          nb.value, _ptr(lam),
                                          _dp(dJdp), C.byref(J), C.byref(info)))
        return dict(dJdp=dJdp, J=J.value, lam=lam, iterations=info.iterations, converged=bool(info.converged),
                    rel_residual=info.rel_residual)


def _steady_residual_function():
    import torch

    class SteadyResidual(torch.autograd.Function):
        """R(x; p) and J as a differentiable function of (p, G, R, W, q); backward is cis_residual_vjp.

        forward copies G, R, W, q into the solver's state buffers and moves its boundary conditions to p
        (CPU float64 [3]: T_w of wall_tag, rho_inf and |U_inf| of ff_tag).  backward restores the p and state of
        its own forward before taking the product, and leaves the solver there."""

        @staticmethod
        def forward(ctx, solver, wall_tag, ff_tag, p, G, R, W, q):
            solver._fp64_only()
            solver.set_params(p.detach().cpu().numpy(), wall_tag, ff_tag)
            with torch.no_grad():
                solver.G.copy_(G)
                solver.R.copy_(R)
                solver.W.copy_(W)
                solver.q.copy_(q)
            rG, rR, rW, rq, J = solver.steady_residual(wall_tag)
            ctx.solver, ctx.tags = solver, (wall_tag, ff_tag)
            ctx.p = p.detach().cpu().numpy().copy()
            ctx.save_for_backward(G, R, W, q)
            return rG, rR, rW, rq, torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, vG, vR, vW, vq, vJ):
            solver = ctx.solver
            G, R, W, q = ctx.saved_tensors
            # the product is taken at this graph's p and state, whatever the solver holds now
            solver.set_params(ctx.p, *ctx.tags)
            with torch.no_grad():
                solver.G.copy_(G)
                solver.R.copy_(R)
                solver.W.copy_(W)
                solver.q.copy_(q)
            cJ = float(vJ) if vJ is not None else 0.0
            vs = (vG, vR, vW, vq)
            gG, gR, gW, gq, gp = solver.residual_vjp(*vs, cJ=cJ, wall_tag=ctx.tags[0], ff_tag=ctx.tags[1])
            return None, None, None, torch.from_numpy(gp), gG, gR, gW, gq

    return SteadyResidual


_SR = None


def steady_residual_fn(solver, wall_tag, ff_tag, p, G, R, W, q):
    """Differentiable R(x; p), J (torch.autograd.Function around cis_steady_residual / cis_residual_vjp)."""
    global _SR
    if _SR is None:
        _SR = _steady_residual_function()
    return _SR.apply(solver, wall_tag, ff_tag, p, G, R, W, q)


def _wall_ref(rho_inf, U_inf, T_inf, A_ref, L_ref, x_ref, lift_dir) -> WallRef:
    return WallRef(float(rho_inf), (C.c_double * 3)(*[float(x) for x in U_inf]), float(T_inf), float(A_ref or 0.0),
                   float(L_ref), (C.c_double * 3)(*[float(x) for x in x_ref]),
                   (C.c_double * 3)(*([0.0, 0.0, 0.0] if lift_dir is None else [float(x) for x in lift_dir])))


def _coef_dict(coef, n: int, tot: WallTotals, with_ref: bool) -> dict:
    rec = np.ctypeslib.as_array(C.cast(coef, C.POINTER(C.c_double)), shape=(max(n, 1), 3))[:n].copy()
    out = dict(Cp=rec[:, 0], Ctau=rec[:, 1], Ch=rec[:, 2], force=np.array(tot.force), moment=np.array(tot.moment),
               heat=tot.heat, e_drag=np.array(tot.e_drag), e_lift=np.array(tot.e_lift))
    if with_ref:
        out.update(CF=np.array(tot.CF), Cd=tot.Cd, Cl=tot.Cl, CM=np.array(tot.CM), Cm=tot.Cm, CQ=tot.CQ)
    return out


def wall_coefficients(loads: dict, rho_inf: float, U_inf, T_inf: float, R: float = 0.5, A_ref: float = None,
                      L_ref: float = 1.0, x_ref=(0.0, 0.0, 0.0), lift_dir=None) -> dict:
    """Wall coefficients from per-face loads (the dict of Solver.wall_loads), computed by
    cis_wall_coefficients_of_loads: per face C_p = (p - p_inf)/q_inf, C_tau = |tau|/q_inf, C_h = q/(q_inf |U_inf|)
    (Eqs. 70-72) with q_inf = rho_inf |U_inf|^2/2 and p_inf = rho_inf R T_inf; with a reference area A_ref (and
    length L_ref, moment point x_ref, lift direction lift_dir) also CF, Cd, Cl, CM, Cm and CQ."""
    lib = load()
    n = len(loads["p"])
    arr = (WallFace * max(n, 1))()
    for f in range(n):
        arr[f] = WallFace((C.c_double * 3)(*loads["x"][f]), float(loads["area"][f]), (C.c_double * 3)(*loads["n"][f]),
                          float(loads["p"][f]), (C.c_double * 3)(*loads["tau"][f]), float(loads["q"][f]))
    ref = _wall_ref(rho_inf, U_inf, T_inf, A_ref, L_ref, x_ref, lift_dir)
    coef = (WallCoef * max(n, 1))()
    tot = WallTotals()
    _check(lib.cis_wall_coefficients_of_loads(C.cast(arr, C.c_void_p), n, float(R), C.byref(ref),
                                              C.cast(coef, C.c_void_p), C.byref(tot)))
    return _coef_dict(coef, n, tot, bool(A_ref))
