"""MI355X p-multigrid compact gas-kinetic scheme (CGKS).

Thin ctypes binding of libcgks.so (see include/cgks.h).  Every step of the
cycle runs in the library's HIP kernels; this module only marshals arguments.
PyTorch supplies device memory (a uint8 tensor per batch) and the stream.
Importing works without a GPU; creating a bound batch needs one, and every
call fails loudly if the native library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CGKS_LIB_PATH selects another build of the same library (for A/B timing)
LIB_PATH = os.environ.get("CGKS_LIB_PATH") or os.path.join(_HERE, "libcgks.so")
_lib = None

OK, EINVAL, ENOMEM, EDEVICE, EMESH, ENONPHYS, EDIVERGED, ENOTCONV, EUNSUPPORTED = range(9)
S2O4, S1O2 = 0, 1
LOW_KFVS, LOW_LF = 0, 1
FLUX_SMOOTH, FLUX_FULL = 0, 1
FP64, MIXED32, MIXED32_R64 = 0, 1, 2
RESIDUAL_HIGH, RESIDUAL_LOW, RESIDUAL_NORM = 0, 1, 2

EXPORTS = ["cgks_status_string", "cgks_mesh_create", "cgks_mesh_create_faces", "cgks_mesh_query", "cgks_mesh_permutation",
           "cgks_mesh_geometry", "cgks_mesh_destroy", "cgks_batch_create", "cgks_batch_query", "cgks_batch_bind", "cgks_batch_destroy",
           "cgks_state_upload", "cgks_state_download", "cgks_state_device", "cgks_highorder_stage",
           "cgks_residual", "cgks_lowlevel_smooth", "cgks_cycle", "cgks_solve", "cgks_timing_enable",
           "cgks_timing_read", "cgks_graph_create", "cgks_graph_launch", "cgks_graph_destroy", "cgks_wall_force",
           "cgks_pool_create", "cgks_batch_admit", "cgks_batch_release", "cgks_batch_capacity", "cgks_batch_slot_info",
           "cgks_batch_autotune", "cgks_residual_high_noalloc"]
KERNEL_KINDS = ["dt", "recon", "flux", "cell", "low_face", "low_cell", "sweep", "prolong"]


class CgksError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        msg = lib().cgks_status_string(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})")


ORDER_TILE_DEFAULT = 4096   # CGKS_ORDER_TILE_DEFAULT of include/cgks.h


class _Desc(C.Structure):
    """cgks_mesh_desc: cell based."""
    _fields_ = [("dim", C.c_int), ("n_vert", C.c_int64), ("xyz", C.c_void_p), ("n_cell", C.c_int64),
                ("cell_type", C.c_void_p), ("cell_vert_ptr", C.c_void_p), ("cell_vert", C.c_void_p),
                ("n_bface", C.c_int64), ("bface_vert_ptr", C.c_void_p), ("bface_vert", C.c_void_p),
                ("bface_tag", C.c_void_p), ("bface_pair", C.c_void_p), ("colour", C.c_void_p),
                ("order_tile", C.c_int64)]


class _FaceDesc(C.Structure):
    """cgks_face_mesh_desc: face based."""
    _fields_ = [("dim", C.c_int), ("n_vert", C.c_int64), ("xyz", C.c_void_p), ("n_cell", C.c_int64),
                ("n_face", C.c_int64), ("face_vert_ptr", C.c_void_p), ("face_vert", C.c_void_p),
                ("face_owner", C.c_void_p), ("face_neigh", C.c_void_p), ("face_bc", C.c_void_p),
                ("face_shift", C.c_void_p), ("colour", C.c_void_p), ("order_tile", C.c_int64)]


class _Info(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_colour", C.c_int), ("n_cell", C.c_int64), ("n_face", C.c_int64),
                ("n_gp", C.c_int64), ("n_boundary_face", C.c_int64), ("n_planar_faces", C.c_int64)]


class _Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("mu", C.c_double), ("Pr", C.c_double), ("T_wall", C.c_double),
                ("W_inf", C.c_double * 5), ("cfl_high", C.c_double), ("cfl_low", C.c_double),
                ("n_implicit", C.c_int32), ("n_sweeps", C.c_int32), ("time_scheme", C.c_int32),
                ("explicit_only", C.c_int32), ("dt_fixed", C.c_double), ("low_flux", C.c_int32),
                ("flux_kind", C.c_int32), ("weno_eps", C.c_double), ("area_ref", C.c_double)]


class _SolveOpts(C.Structure):
    _fields_ = [("max_cycles", C.c_int32), ("tol", C.c_double), ("tol_abs", C.c_int32),
                ("check_every", C.c_int32), ("res_history", C.c_void_p)]


class _PoolDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32), ("max_cases", C.c_int32),
                ("max_cells", C.c_int64), ("max_faces", C.c_int64), ("max_gauss_points", C.c_int64),
                ("max_boundary_faces", C.c_int64), ("n_implicit", C.c_int32), ("n_sweeps", C.c_int32),
                ("time_scheme", C.c_int32), ("explicit_only", C.c_int32)]


class _SolveReport(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("converged", C.c_int32), ("res_first", C.c_double),
                ("res_last", C.c_double), ("status", C.c_int), ("force", C.c_double * 3), ("cd", C.c_double)]


def lib():
    """Load libcgks.so; raises if it has not been built.

    torch is imported first when present: libcgks.so then binds to the HIP
    runtime torch already loaded (same soname), so device pointers and
    streams from torch are valid in the library.  Without torch the library
    uses the system ROCm runtime."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libcgks.so not built ({LIB_PATH}); run paper_2109_09965_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, i32 = C.c_void_p, C.c_int32
        L.cgks_status_string.restype = C.c_char_p
        L.cgks_status_string.argtypes = [C.c_int]
        L.cgks_mesh_create.argtypes = [C.POINTER(_Desc), C.POINTER(P)]
        L.cgks_mesh_create_faces.argtypes = [C.POINTER(_FaceDesc), C.POINTER(P)]
        L.cgks_mesh_query.argtypes = [P, C.POINTER(_Info)]
        L.cgks_mesh_permutation.argtypes = [P, P, P]
        L.cgks_mesh_geometry.argtypes = [P, P, P, P]
        L.cgks_mesh_destroy.argtypes = [P]
        L.cgks_batch_create.argtypes = [P, P, i32, i32, C.POINTER(P)]
        L.cgks_batch_query.argtypes = [P, C.POINTER(C.c_size_t)]
        L.cgks_batch_bind.argtypes = [P, P, C.c_size_t, P]
        L.cgks_batch_destroy.argtypes = [P]
        L.cgks_state_upload.argtypes = [P, i32, P, P, P]
        L.cgks_state_download.argtypes = [P, i32, P, P, P]
        L.cgks_state_device.argtypes = [P, i32, C.POINTER(P), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.cgks_highorder_stage.argtypes = [P, i32, P]
        L.cgks_residual.argtypes = [P, i32, P, P]
        L.cgks_lowlevel_smooth.argtypes = [P, P, P]
        L.cgks_cycle.argtypes = [P, P, P]
        L.cgks_solve.argtypes = [P, C.POINTER(_SolveOpts), P, P]
        L.cgks_timing_enable.argtypes = [P, i32]
        L.cgks_graph_create.argtypes = [P, i32, P]
        L.cgks_graph_launch.argtypes = [P, P, P]
        L.cgks_graph_destroy.argtypes = [P]
        L.cgks_timing_read.argtypes = [P, P, P]
        L.cgks_wall_force.argtypes = [P, P, P, P]
        L.cgks_pool_create.argtypes = [C.POINTER(_PoolDesc), C.POINTER(P)]
        L.cgks_batch_admit.argtypes = [P, P, P, C.POINTER(C.c_int32), P]
        L.cgks_batch_release.argtypes = [P, i32, P]
        L.cgks_batch_capacity.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.cgks_batch_slot_info.argtypes = [P, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.cgks_batch_autotune.argtypes = [P, P, P]
        L.cgks_residual_high_noalloc.argtypes = [P, P, P]
        for name in EXPORTS:
            getattr(L, name).restype = C.c_int if name != "cgks_status_string" else C.c_char_p
        _lib = L
    return _lib


def _check(st, what):
    if st != OK:
        raise CgksError(st, what)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _check_tensor(t, min_numel, what):
    """A device buffer handed to the library must be a contiguous float64
    CUDA tensor with at least min_numel elements (the library writes or
    reads that many): anything else raises ValueError before the call."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != torch.float64:
        raise ValueError(f"{what}: expected float64, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{what}: expected a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous tensor")
    if t.numel() < min_numel:
        raise ValueError(f"{what}: {t.numel()} elements, the library needs {min_numel}")


def _host_array(a, shape, what):
    """Host state array as contiguous float64 of exactly `shape`."""
    a = np.ascontiguousarray(a, np.float64)
    if a.shape != tuple(shape):
        raise ValueError(f"{what}: shape {a.shape}, expected {tuple(shape)}")
    return a


@dataclass
class Params:
    """Per-case parameters (cgks_params); W_inf holds dim+2 conservative values."""
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
    area_ref: float = 0.0

    def c(self):
        p = _Params()
        p.gamma, p.mu, p.Pr, p.T_wall = self.gamma, self.mu, self.Pr, self.T_wall
        w = np.zeros(5)
        w[:len(self.W_inf)] = self.W_inf
        p.W_inf = (C.c_double * 5)(*w)
        p.cfl_high, p.cfl_low = self.cfl_high, self.cfl_low
        p.n_implicit, p.n_sweeps = self.n_implicit, self.n_sweeps
        p.time_scheme, p.explicit_only, p.dt_fixed = self.time_scheme, self.explicit_only, self.dt_fixed
        p.low_flux = self.low_flux
        p.flux_kind, p.weno_eps, p.area_ref = self.flux_kind, self.weno_eps, self.area_ref
        return p


class Mesh:
    """Host-side mesh handle.  A mesh dict with the cell-based keys
    (cell_type, cell_vert_ptr, cell_vert, bface_*) goes through
    cgks_mesh_create, which builds the faces in the library; faces=True, or
    a dict with only the face-based keys, through cgks_mesh_create_faces."""

    def __init__(self, m: dict, order_tile: int = 0, colour=None, faces: bool = False):
        """order_tile: cells per tile of the library cell order (tiles cut
        from a Morton curve of the cell centroids; 0 = library default).
        colour: optional caller colouring [n_cell] of the relaxation sweeps."""
        L = lib()
        self.dim = int(m["dim"])
        self.nv = self.dim + 2
        n_cell = int(m["n_cell"])
        col = None if colour is None else np.ascontiguousarray(colour, np.int32)
        if col is not None and col.shape != (n_cell,):
            raise ValueError(f"colour: shape {col.shape}, expected ({n_cell},)")
        xyz = np.ascontiguousarray(m["xyz"], np.float64)
        h = C.c_void_p()
        if "cell_type" in m and not faces:
            keep = dict(xyz=xyz, ct=np.ascontiguousarray(m["cell_type"], np.int32),
                        cp=np.ascontiguousarray(m["cell_vert_ptr"], np.int64),
                        cv=np.ascontiguousarray(m["cell_vert"], np.int64),
                        bp=np.ascontiguousarray(m["bface_vert_ptr"], np.int64),
                        bv=np.ascontiguousarray(m["bface_vert"], np.int64),
                        bt=np.ascontiguousarray(m["bface_tag"], np.int32),
                        bpair=np.ascontiguousarray(m["bface_pair"], np.int64), col=col)
            d = _Desc(self.dim, len(xyz), _ptr(xyz), n_cell, _ptr(keep["ct"]), _ptr(keep["cp"]), _ptr(keep["cv"]),
                      len(keep["bt"]), _ptr(keep["bp"]), _ptr(keep["bv"]), _ptr(keep["bt"]), _ptr(keep["bpair"]),
                      _ptr(col), int(order_tile))
            _check(L.cgks_mesh_create(C.byref(d), C.byref(h)), "cgks_mesh_create")
        else:
            keep = dict(xyz=xyz, ptr=np.ascontiguousarray(m["face_vert_ptr"], np.int64),
                        fv=np.ascontiguousarray(m["face_vert"], np.int64),
                        own=np.ascontiguousarray(m["face_owner"], np.int64),
                        nb=np.ascontiguousarray(m["face_neigh"], np.int64),
                        bc=np.ascontiguousarray(m["face_bc"], np.int32),
                        sh=np.ascontiguousarray(m["face_shift"], np.float64), col=col)
            d = _FaceDesc(self.dim, len(xyz), _ptr(xyz), n_cell, len(keep["own"]), _ptr(keep["ptr"]),
                          _ptr(keep["fv"]), _ptr(keep["own"]), _ptr(keep["nb"]), _ptr(keep["bc"]), _ptr(keep["sh"]),
                          _ptr(col), int(order_tile))
            _check(L.cgks_mesh_create_faces(C.byref(d), C.byref(h)), "cgks_mesh_create_faces")
        self.h = h
        info = _Info()
        _check(L.cgks_mesh_query(h, C.byref(info)), "cgks_mesh_query")
        self.info = info
        self.n_cell, self.n_face, self.n_gp = info.n_cell, info.n_face, info.n_gp
        self.n_colour = info.n_colour
        self.lib2caller = np.zeros(self.n_cell, np.int64)
        self.colour = np.zeros(self.n_cell, np.int32)
        _check(L.cgks_mesh_permutation(h, _ptr(self.lib2caller), _ptr(self.colour)), "cgks_mesh_permutation")

    def geometry(self):
        """Caller-order (vol, centroid, h) computed by the library."""
        n = self.n_cell
        vol, ctr, h = np.zeros(n), np.zeros((n, self.dim)), np.zeros(n)
        _check(lib().cgks_mesh_geometry(self.h, _ptr(vol), _ptr(ctr), _ptr(h)), "cgks_mesh_geometry")
        return vol, ctr, h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.cgks_mesh_destroy(self.h)
            self.h = None


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Batch:
    """A batch of cases bound to one device arena (a torch uint8 tensor)."""

    def __init__(self, meshes, params, precision=FP64, device="cuda", stream=None, _pool=None):
        L = lib()
        h = C.c_void_p()
        if _pool is None:
            self.meshes = list(meshes)
            self.params = list(params)
            n = len(self.meshes)
            arr_m = (C.c_void_p * n)(*[m.h.value for m in self.meshes])
            arr_p = (_Params * n)(*[p.c() for p in self.params])
            self._keep = (arr_m, arr_p)
            _check(L.cgks_batch_create(arr_m, arr_p, n, precision, C.byref(h)), "cgks_batch_create")
            self.dim = self.meshes[0].dim
        else:
            _check(L.cgks_pool_create(C.byref(_pool), C.byref(h)), "cgks_pool_create")
            self.meshes = [None] * _pool.max_cases
            self.params = [None] * _pool.max_cases
            self.dim = _pool.dim
        self.h = h
        self.precision = precision
        self._bind(device, stream)

    @classmethod
    def pool(cls, dim, max_cases, max_cells, max_faces, max_gauss_points, max_boundary_faces, precision=FP64,
             n_implicit=6, n_sweeps=2, time_scheme=S2O4, explicit_only=0, device="cuda", stream=None):
        """An empty pool of fixed capacity; cases enter with admit() and
        leave with release()."""
        q = _PoolDesc(dim, precision, max_cases, max_cells, max_faces, max_gauss_points, max_boundary_faces,
                      n_implicit, n_sweeps, time_scheme, explicit_only)
        return cls(None, None, precision=precision, device=device, stream=stream, _pool=q)

    def _bind(self, device, stream):
        import torch
        L = lib()
        nb = C.c_size_t()
        _check(L.cgks_batch_query(self.h, C.byref(nb)), "cgks_batch_query")
        self.nbytes = nb.value
        self.arena = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        base = self.arena.data_ptr()
        self._base = (base + 255) & ~255
        self.stream = stream
        _check(L.cgks_batch_bind(self.h, C.c_void_p(self._base), self.nbytes, _stream(stream)), "cgks_batch_bind")
        k, nc = C.c_int32(), C.c_int64()
        _check(L.cgks_batch_capacity(self.h, C.byref(k), C.byref(nc)), "cgks_batch_capacity")
        self.n_case = k.value
        self.NC = nc.value
        self.nv = self.dim + 2
        self._slots()

    def _slots(self):
        L = lib()
        self.cell_off = np.full(self.n_case, -1, np.int64)
        self.live = np.zeros(self.n_case, bool)
        for c in range(self.n_case):
            lv, off, n = C.c_int32(), C.c_int64(), C.c_int64()
            _check(L.cgks_batch_slot_info(self.h, c, C.byref(lv), C.byref(off), C.byref(n)), "cgks_batch_slot_info")
            self.live[c] = bool(lv.value)
            self.cell_off[c] = off.value

    def admit(self, mesh, params):
        """Admit a case into a free slot; returns the slot, or None when the
        pool has no room (CGKS_ENOMEM)."""
        slot = C.c_int32()
        st = lib().cgks_batch_admit(self.h, mesh.h, C.byref(params.c()), C.byref(slot), _stream(self.stream))
        if st == ENOMEM:
            return None
        _check(st, "cgks_batch_admit")
        c = slot.value
        self.graph_cycles = 0      # admission drops a captured graph
        self.meshes[c] = mesh
        self.params[c] = params
        self._slots()
        return c

    def release(self, slot):
        _check(lib().cgks_batch_release(self.h, slot, _stream(self.stream)), "cgks_batch_release")
        self.graph_cycles = 0      # release drops a captured graph
        self.meshes[slot] = None
        self.params[slot] = None
        self._slots()

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.cgks_batch_destroy(self.h)
            self.h = None

    def _case_mesh(self, c):
        if not (0 <= c < self.n_case) or self.meshes[c] is None:
            raise ValueError(f"case {c}: no case in this slot")
        return self.meshes[c]

    def upload(self, c, W, dW=None):
        n = self._case_mesh(c).n_cell
        W = _host_array(W, (self.nv, n), "W")
        dW = None if dW is None else _host_array(dW, (self.dim, self.nv, n), "dW")
        _check(lib().cgks_state_upload(self.h, c, _ptr(W), _ptr(dW), _stream(self.stream)), "cgks_state_upload")

    def download(self, c):
        m = self._case_mesh(c)
        W = np.zeros((self.nv, m.n_cell))
        dW = np.zeros((self.dim, self.nv, m.n_cell))
        _check(lib().cgks_state_download(self.h, c, _ptr(W), _ptr(dW), _stream(self.stream)), "cgks_state_download")
        return W, dW

    def highorder_stage(self, stage):
        _check(lib().cgks_highorder_stage(self.h, stage, _stream(self.stream)), "cgks_highorder_stage")

    def residual(self, kind):
        """Device tensor: [nv, NC] for HIGH/LOW (library order), [n_case] for NORM."""
        import torch
        n = self.n_case if kind == RESIDUAL_NORM else self.nv * self.NC
        out = torch.empty(n, dtype=torch.float64, device=self.arena.device)
        _check(lib().cgks_residual(self.h, kind, C.c_void_p(out.data_ptr()), _stream(self.stream)), "cgks_residual")
        return out if kind == RESIDUAL_NORM else out.view(self.nv, self.NC)

    def residual_high_noalloc(self, out=None):
        """R1 like residual(RESIDUAL_HIGH), computed with the library's fixed
        device scratch instead of the batch arena (the entry point for
        callers that cannot allocate).  out: float64 device tensor of
        nv * NC elements (allocated here when None)."""
        import torch
        if out is None:
            out = torch.empty(self.nv * self.NC, dtype=torch.float64, device=self.arena.device)
        _check_tensor(out, self.nv * self.NC, "out")
        _check(lib().cgks_residual_high_noalloc(self.h, C.c_void_p(out.data_ptr()), _stream(self.stream)),
               "cgks_residual_high_noalloc")
        return out.view(self.nv, self.NC)

    def to_caller(self, c, X):
        """[k, NC] library-order array (numpy) -> [k, n_c] in case c's caller order."""
        m = self.meshes[c]
        out = np.empty((X.shape[0], m.n_cell))
        out[:, m.lib2caller] = X[:, self.cell_off[c]:self.cell_off[c] + m.n_cell]
        return out

    def lowlevel_smooth(self, R1):
        _check_tensor(R1, self.nv * self.NC, "R1")
        _check(lib().cgks_lowlevel_smooth(self.h, C.c_void_p(R1.data_ptr()), _stream(self.stream)),
               "cgks_lowlevel_smooth")

    def cycle(self, res=None):
        if res is not None:
            _check_tensor(res, self.n_case, "res")
        ptr = C.c_void_p(res.data_ptr()) if res is not None else None
        _check(lib().cgks_cycle(self.h, ptr, _stream(self.stream)), "cgks_cycle")

    def graph_create(self, n_cycles):
        """Capture n_cycles cycles of every case as one replayable HIP graph."""
        _check(lib().cgks_graph_create(self.h, n_cycles, _stream(self.stream)), "cgks_graph_create")
        self.graph_cycles = n_cycles

    def graph_launch(self, res_history=None):
        """Replay the captured cycles; res_history: device float64 [n_cycles * n_case] or None."""
        if res_history is not None:
            if getattr(self, "graph_cycles", 0) <= 0:
                raise ValueError("graph_launch: no graph captured")
            _check_tensor(res_history, self.graph_cycles * self.n_case, "res_history")
        ptr = C.c_void_p(res_history.data_ptr()) if res_history is not None else None
        _check(lib().cgks_graph_launch(self.h, ptr, _stream(self.stream)), "cgks_graph_launch")

    def autotune(self):
        """Measure and keep the fastest launch shapes; returns them."""
        ch = np.zeros(5, np.int32)
        _check(lib().cgks_batch_autotune(self.h, _ptr(ch), _stream(self.stream)), "cgks_batch_autotune")
        self.graph_cycles = 0      # tuning drops a captured graph
        return dict(flux_block=int(ch[0]), cell_block=int(ch[1]), low_face_block=int(ch[2]),
                    low_cell_block=int(ch[3]), sweep_chunk=int(ch[4]))

    def wall_force(self):
        """[n_case, 3] force of the gas on the walls at the start of the latest cycle."""
        f = np.zeros((self.n_case, 3))
        _check(lib().cgks_wall_force(self.h, _ptr(f), None, _stream(self.stream)), "cgks_wall_force")
        return f

    def drag_coefficients(self):
        """[n_case] drag coefficients of the latest wall forces, computed by
        the library from each case's free stream and area_ref (NaN without)."""
        f = np.zeros((self.n_case, 3))
        cd = np.zeros(self.n_case)
        _check(lib().cgks_wall_force(self.h, _ptr(f), _ptr(cd), _stream(self.stream)), "cgks_wall_force")
        return cd

    def timing(self, enable=True):
        _check(lib().cgks_timing_enable(self.h, int(enable)), "cgks_timing_enable")

    def timing_read(self):
        """{kind: (total ms, launches)} since the previous read."""
        ms = np.zeros(len(KERNEL_KINDS))
        n = np.zeros(len(KERNEL_KINDS), np.int64)
        _check(lib().cgks_timing_read(self.h, _ptr(ms), _ptr(n)), "cgks_timing_read")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_KINDS)}

    def solve(self, max_cycles, tol, tol_abs=False, check_every=10, history=False):
        opts = _SolveOpts(max_cycles, tol, int(tol_abs), check_every, None)
        hist = None
        if history:
            hist = np.zeros((self.n_case, max_cycles))
            opts.res_history = hist.ctypes.data_as(C.c_void_p)
        rep = (_SolveReport * self.n_case)()
        _check(lib().cgks_solve(self.h, C.byref(opts), rep, _stream(self.stream)), "cgks_solve")
        # with 2 <= check_every <= 8 the library replaced any captured graph by
        # one of check_every cycles; otherwise the previous graph is kept
        if 2 <= check_every <= 8:
            self.graph_cycles = check_every
        out = [dict(cycles=r.cycles, converged=bool(r.converged), res_first=r.res_first, res_last=r.res_last,
                    status=r.status, force=np.array(r.force[:]), cd=r.cd) for r in rep]
        return out, hist
