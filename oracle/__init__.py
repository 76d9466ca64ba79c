"""ORACLE -- test infrastructure only.

ctypes wrapper around ``cgks_oracle.c``, the plain FP64 CPU implementation of
the p-multigrid compact gas-kinetic scheme cycle.  Only the test suite,
``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may
import this package.  The HIP library never links or calls it and shares no
code with it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cgks_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

S2O4, S1O2 = 0, 1
LOW_KFVS, LOW_LF = 0, 1
FLUX_SMOOTH, FLUX_FULL = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                               "-std=gnu99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        d, i, l = C.c_double, C.c_int, C.c_long
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        lp = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.om_mesh_create.restype = P
        L.om_mesh_create.argtypes = [i, l, dp, l, l, lp, lp, lp, lp, ip, dp]
        L.om_mesh_destroy.argtypes = [P]
        L.om_mesh_n_colour.argtypes = [P]
        L.om_mesh_set_colour.argtypes = [P, ip]
        L.om_mesh_cells.argtypes = [P, dp, dp, dp, dp, ip]
        L.om_mesh_faces.argtypes = [P, ip, dp, dp, dp, dp, dp]
        L.om_recon_eval.argtypes = [P, P, dp, dp, l, lp, dp, dp, dp]
        L.om_recon_linear_cells.argtypes = [P, P, ip]
        L.om_gks_flux.argtypes = [i, d, d, d, dp, dp, dp, dp, dp]
        L.om_halfspace_state.argtypes = [i, d, dp, dp, dp]
        L.om_gks_flux_full.argtypes = [i, d, d, d, d, dp, dp, dp, dp, dp, dp, dp, dp]
        L.om_kfvs.argtypes = [i, d, dp, dp, dp]
        L.om_moment.restype = d
        L.om_moment.argtypes = [i, d, dp, i, i, i, i, i]
        L.om_micro_slope.argtypes = [i, d, dp, dp, dp]
        L.om_farfield_state.argtypes = [i, d, dp, dp, dp]
        L.om_ctx_create.restype = P
        L.om_ctx_create.argtypes = [P, P]
        L.om_ctx_destroy.argtypes = [P]
        L.om_ctx_dt.restype = d
        L.om_ctx_dt.argtypes = [P]
        L.om_ctx_force.argtypes = [P, dp]
        L.om_dt.restype = d
        L.om_dt.argtypes = [P, P, dp]
        L.om_stage.argtypes = [P, i, dp, dp]
        L.om_stage_combine.argtypes = [i, i, d, d, d, d, d, C.POINTER(d)]
        L.om_grad_combine.argtypes = [i, i, d, d, d, d, C.POINTER(d)]
        L.om_residual_high.argtypes = [P, dp, dp, dp]
        L.om_ho_sums.argtypes = [P, dp, dp, dp, dp, dp, dp]
        L.om_residual_low.argtypes = [P, P, dp, dp]
        L.om_lowlevel.argtypes = [P, P, dp, dp]
        L.om_res.restype = d
        L.om_res.argtypes = [l, dp, dp]
        L.om_cycle.argtypes = [P, dp, dp, C.POINTER(d)]
        _lib = L
    return _lib


class _CParams(C.Structure):
    _fields_ = [("gamma", C.c_double), ("mu", C.c_double), ("Pr", C.c_double), ("T_wall", C.c_double),
                ("W_inf", C.c_double * 5), ("cfl_high", C.c_double), ("cfl_low", C.c_double),
                ("n_implicit", C.c_int), ("n_sweeps", C.c_int), ("time_scheme", C.c_int),
                ("explicit_only", C.c_int), ("dt_fixed", C.c_double), ("low_flux", C.c_int),
                ("flux_kind", C.c_int), ("weno_eps", C.c_double)]


@dataclass
class Params:
    """Flow and solver parameters (see the oracle source for their use)."""
    W_inf: np.ndarray
    gamma: float = 1.4
    mu: float = 0.0
    Pr: float = 1.0
    T_wall: float = 1.0 / 1.4
    cfl_high: float = 0.4
    cfl_low: float = 1000.0
    n_implicit: int = 6
    n_sweeps: int = 2
    time_scheme: int = S2O4
    explicit_only: int = 0
    dt_fixed: float = 0.0
    low_flux: int = LOW_KFVS
    flux_kind: int = FLUX_SMOOTH
    weno_eps: float = 0.0

    def c(self):
        p = _CParams()
        p.gamma, p.mu, p.Pr, p.T_wall = self.gamma, self.mu, self.Pr, self.T_wall
        w = np.zeros(5)
        w[:len(self.W_inf)] = self.W_inf
        p.W_inf = (C.c_double * 5)(*w)
        p.cfl_high, p.cfl_low = self.cfl_high, self.cfl_low
        p.n_implicit, p.n_sweeps = self.n_implicit, self.n_sweeps
        p.time_scheme, p.explicit_only = self.time_scheme, self.explicit_only
        p.dt_fixed = self.dt_fixed
        p.low_flux = self.low_flux
        p.flux_kind = self.flux_kind
        p.weno_eps = self.weno_eps
        return p


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


class Mesh:
    """Oracle mesh: computes its own geometry, quadrature and colouring."""

    def __init__(self, m: dict, colour=None):
        """colour: optional caller colouring of the relaxation sweeps
        (replaces the oracle's own greedy colouring)."""
        L = lib()
        self.dim = int(m["dim"])
        self.nv = self.dim + 2
        self.n_cell = int(m["n_cell"])
        self.n_face = len(m["face_owner"])
        self._keep = dict(xyz=_c64(m["xyz"]), ptr=_i64(m["face_vert_ptr"]), fv=_i64(m["face_vert"]),
                          own=_i64(m["face_owner"]), nb=_i64(m["face_neigh"]),
                          bc=np.ascontiguousarray(m["face_bc"], dtype=np.int32), sh=_c64(m["face_shift"]))
        k = self._keep
        self.h = L.om_mesh_create(self.dim, len(k["xyz"]), k["xyz"], self.n_cell, self.n_face, k["ptr"], k["fv"],
                                  k["own"], k["nb"], k["bc"], k["sh"])
        if colour is not None:
            self._colour = np.ascontiguousarray(colour, np.int32)
            if L.om_mesh_set_colour(self.h, self._colour):
                raise ValueError("colouring: neighbours share a colour or an id is out of range")
        self.n_colour = L.om_mesh_n_colour(self.h)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.om_mesh_destroy(self.h)
            self.h = None

    def cells(self):
        n = self.n_cell
        vol, ctr, sec, h = np.zeros(n), np.zeros(n * self.dim), np.zeros(n * 6), np.zeros(n)
        col = np.zeros(n, np.int32)
        lib().om_mesh_cells(self.h, vol, ctr, sec, h, col)
        return dict(vol=vol, ctr=ctr.reshape(n, self.dim), sec=sec.reshape(n, 6), h=h, colour=col)

    def faces(self):
        f, d = self.n_face, self.dim
        ngp = np.zeros(f, np.int32)
        gx, gn, gw = np.zeros(f * 4 * d), np.zeros(f * 4 * d), np.zeros(f * 4)
        av, S = np.zeros(f * d), np.zeros(f)
        lib().om_mesh_faces(self.h, ngp, gx, gn, gw, av, S)
        return dict(ngp=ngp, gx=gx.reshape(f, 4, d), gn=gn.reshape(f, 4, d), gw=gw.reshape(f, 4),
                    avec=av.reshape(f, d), S=S)

    def _default_params(self, params):
        if params is None:
            W = np.zeros(self.nv)
            W[0], W[-1] = 1.0, 1.0 / (1.4 * 0.4)
            params = Params(W_inf=W)
        return params.c()

    def linear_cells(self, params=None, ghosts=True):
        """1 where the cell's stencil cannot fix a quadratic (linear fallback)."""
        out = np.zeros(self.n_cell, np.int32)
        p = self._default_params(params)
        lib().om_recon_linear_cells(self.h, C.byref(p) if ghosts else None, out)
        return out

    def recon_eval(self, W, dW, cells, x, params=None, ghosts=True):
        """Evaluate the reconstruction of cells[p] at x[p].  Boundary faces of
        those cells bring ghost rows built from params; ghosts=False leaves
        them out (pins of the least-squares machinery alone)."""
        cells = _i64(cells)
        n = len(cells)
        Wx, dWx = np.zeros(n * self.nv), np.zeros(n * self.dim * self.nv)
        p = self._default_params(params)
        st = lib().om_recon_eval(self.h, C.byref(p) if ghosts else None, _c64(W), _c64(dW), n, cells, _c64(x),
                                 Wx, dWx)
        if st:
            raise RuntimeError("oracle reconstruction failed")
        return Wx.reshape(n, self.nv), dWx.reshape(n, self.dim, self.nv)


class Solver:
    """Cycle context of the oracle (work arrays and stage data)."""

    def __init__(self, mesh: Mesh, params: Params):
        self.mesh = mesh
        self.params = params
        self._p = params.c()
        self.h = lib().om_ctx_create(mesh.h, C.byref(self._p))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.om_ctx_destroy(self.h)
            self.h = None

    @property
    def dt(self):
        return lib().om_ctx_dt(self.h)

    def force(self):
        f = np.zeros(3)
        lib().om_ctx_force(self.h, f)
        return f

    def stage(self, stage, W, dW):
        st = lib().om_stage(self.h, stage, W, dW)
        if st:
            raise RuntimeError(f"oracle stage failed ({st})")

    def residual_high(self, W, dW):
        R1 = np.zeros_like(W)
        st = lib().om_residual_high(self.h, _c64(W), _c64(dW), R1)
        if st:
            raise RuntimeError(f"oracle residual failed ({st})")
        return R1

    def ho_sums(self, W, dW):
        m = self.mesh
        F0, Ft = np.zeros((m.nv, m.n_cell)), np.zeros((m.nv, m.n_cell))
        G0, Gt = np.zeros((m.dim, m.nv, m.n_cell)), np.zeros((m.dim, m.nv, m.n_cell))
        st = lib().om_ho_sums(self.h, _c64(W), _c64(dW), F0, Ft, G0, Gt)
        if st:
            raise RuntimeError(f"oracle pass failed ({st})")
        return F0, Ft, G0, Gt

    def residual_low(self, U):
        R0 = np.zeros_like(U)
        st = lib().om_residual_low(self.mesh.h, C.byref(self._p), _c64(U), R0)
        if st:
            raise RuntimeError(f"oracle low residual failed ({st})")
        return R0

    def lowlevel(self, W, R1):
        st = lib().om_lowlevel(self.mesh.h, C.byref(self._p), W, _c64(R1))
        if st:
            raise RuntimeError(f"oracle low level failed ({st})")

    def dt_of(self, W):
        return lib().om_dt(self.mesh.h, C.byref(self._p), _c64(W))

    def cycle(self, W, dW):
        """One p-multigrid cycle in place on W [nv, n], dW [dim, nv, n]; returns Res."""
        r = C.c_double(0.0)
        st = lib().om_cycle(self.h, W, dW, C.byref(r))
        if st:
            raise RuntimeError(f"oracle cycle failed ({st})")
        return r.value


# ---- point functions (local face frame, axis 0 = normal) -------------
def gks_flux(W, dW, gamma=1.4, mu=0.0, Pr=1.0):
    W = _c64(W)
    dim = len(W) - 2
    F0, Ft, Wt = np.zeros(dim + 2), np.zeros(dim + 2), np.zeros(dim + 2)
    st = lib().om_gks_flux(dim, gamma, mu, Pr, W, _c64(dW).ravel(), F0, Ft, Wt)
    if st:
        raise RuntimeError("non-physical state")
    return F0, Ft, Wt


def gks_flux_full(WL, dWL, WR, dWR, dt, gamma=1.4, mu=0.0, Pr=1.0):
    """Full time-dependent solution in the face frame: (F0, Ft, W0, Wt)."""
    WL = _c64(WL)
    dim = len(WL) - 2
    out = [np.zeros(dim + 2) for _ in range(4)]
    st = lib().om_gks_flux_full(dim, gamma, mu, Pr, dt, WL, _c64(dWL).ravel(), _c64(WR), _c64(dWR).ravel(), *out)
    if st:
        raise RuntimeError("non-physical state")
    return tuple(out)


def halfspace_state(WL, WR, gamma=1.4):
    WL = _c64(WL)
    out = np.zeros_like(WL)
    if lib().om_halfspace_state(len(WL) - 2, gamma, WL, _c64(WR), out):
        raise RuntimeError("non-physical state")
    return out


def kfvs(UL, UR, gamma=1.4):
    UL = _c64(UL)
    out = np.zeros_like(UL)
    if lib().om_kfvs(len(UL) - 2, gamma, UL, _c64(UR), out):
        raise RuntimeError("non-physical state")
    return out


def farfield_state(W_in, W_inf, gamma=1.4):
    """Far-field boundary state from the interior state and the free stream,
    both in the face frame (axis 0 = outward normal)."""
    W_in = _c64(W_in)
    out = np.zeros_like(W_in)
    lib().om_farfield_state(len(W_in) - 2, gamma, W_in, _c64(W_inf), out)
    return out


def moment(W, a, b=0, c=0, e=0, half=0, gamma=1.4):
    W = _c64(W)
    return lib().om_moment(len(W) - 2, gamma, W, a, b, c, e, half)


def micro_slope(W, dWdx, gamma=1.4):
    W = _c64(W)
    out = np.zeros_like(W)
    lib().om_micro_slope(len(W) - 2, gamma, W, _c64(dWdx), out)
    return out


def stage_combine(scheme, stage, dt, Wn, L0, Lt0, Lt1=0.0):
    """The cell-average update of one stage (the code every cell takes)."""
    out = C.c_double(0.0)
    lib().om_stage_combine(scheme, stage, dt, Wn, L0, Lt0, Lt1, C.byref(out))
    return out.value


def grad_combine(scheme, stage, dt, G0, G, Gt):
    """The gradient update of one stage from Gauss-Green sums (the code every
    cell takes); G0 is the first stage's G, used at stage 1."""
    out = C.c_double(0.0)
    lib().om_grad_combine(scheme, stage, dt, G0, G, Gt, C.byref(out))
    return out.value


def res(Wold, Wnew):
    return lib().om_res(len(Wold), _c64(Wold), _c64(Wnew))
