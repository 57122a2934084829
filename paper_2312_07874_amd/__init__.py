"""Python binding of the esdsem C ABI (include/esdsem.h).

Argument marshalling only: every step of the residual, RK4 and VJP runs in the
HIP library libesdsem.so built in this directory (``python
paper_2312_07874_amd/build.py``).  Device buffers are torch CUDA (HIP) tensors;
streams are torch's current stream.  Importing this module fails loudly if the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np

import torch  # noqa: F401  (first: the library then shares the HIP runtime torch loads)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesdsem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2312_07874_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

ESD_OK = 0
STATUS = {0: "ESD_OK", -1: "ESD_EINVAL", -2: "ESD_EJACOBIAN", -3: "ESD_EADMISSIBLE", -4: "ESD_EUNSUPPORTED",
          -5: "ESD_ENONCONFORMING", -6: "ESD_EHIP", -7: "ESD_ENOMEM"}

FLUX_RANOCHA, FLUX_CHANDRASHEKAR = 0, 1
DISS_NONE, DISS_LLF_DAVIS, DISS_ENTROPY_JUMP, DISS_MATRIX = 0, 1, 2, 3

WARP_FN = ctypes.CFUNCTYPE(None, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)


class _MeshDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("degree", ctypes.c_int32), ("n_elements", ctypes.c_int64),
                ("elem_vertex_ids", ctypes.POINTER(ctypes.c_int64)),
                ("elem_vertex_coords", ctypes.POINTER(ctypes.c_double)),
                ("warp", WARP_FN), ("warp_ctx", ctypes.c_void_p)]


class _SchemeDesc(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("ecflux", ctypes.c_int32), ("dissipation", ctypes.c_int32)]


class _BatchDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_meshes", ctypes.c_int32), ("n_elements", ctypes.POINTER(ctypes.c_int64)),
                ("elem_vertex_ids", ctypes.POINTER(ctypes.POINTER(ctypes.c_int64))),
                ("elem_vertex_coords", ctypes.POINTER(ctypes.POINTER(ctypes.c_double))),
                ("elem_degree", ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))),
                ("warp", WARP_FN), ("warp_ctx", ctypes.c_void_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("degree", ctypes.c_int32), ("n_vars", ctypes.c_int32),
                ("n_modes", ctypes.c_int32), ("n_vol_nodes", ctypes.c_int32), ("n_facets", ctypes.c_int32),
                ("n_facet_nodes", ctypes.c_int32), ("n_elements", ctypes.c_int64), ("n_dof", ctypes.c_int64),
                ("flux_pairs_paper", ctypes.c_int64), ("flux_pairs_distinct", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_size_t), ("rk4_workspace_bytes", ctypes.c_size_t),
                ("vjp_workspace_bytes", ctypes.c_size_t), ("rk4_vjp_workspace_bytes", ctypes.c_size_t)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


_vp = ctypes.c_void_p
_c = ctypes.c_int
EXPORTS = {
    "esd_plan_create": (_c, [ctypes.POINTER(_MeshDesc), ctypes.POINTER(_SchemeDesc), ctypes.c_uint32,
                             ctypes.POINTER(_vp)]),
    "esd_plan_create_batched": (_c, [ctypes.POINTER(_BatchDesc), ctypes.POINTER(_SchemeDesc), ctypes.c_uint32,
                                     ctypes.POINTER(_vp)]),
    "esd_plan_buckets": (_c, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64)]),
    "esd_plan_element_map": (_c, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.c_int64]),
    "esd_plan_destroy": (None, [_vp]),
    "esd_plan_create_ex": (_c, [ctypes.POINTER(_MeshDesc), ctypes.POINTER(_SchemeDesc), ctypes.c_uint32,
                                ctypes.POINTER(_Allocator), ctypes.POINTER(_vp)]),
    "esd_plan_create_batched_ex": (_c, [ctypes.POINTER(_BatchDesc), ctypes.POINTER(_SchemeDesc), ctypes.c_uint32,
                                        ctypes.POINTER(_Allocator), ctypes.POINTER(_vp)]),
    "esd_plan_query": (_c, [_vp, ctypes.POINTER(PlanInfo)]),
    "esd_plan_host_array": (_c, [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64]),
    "esd_node_coords": (_c, [_vp, _vp, _vp]),
    "esd_project": (_c, [_vp, _vp, _vp, _vp]),
    "esd_residual": (_c, [_vp, _vp, _vp, _vp, _vp]),
    "esd_residual_noalloc": (_c, [_vp, _vp, _vp, _vp]),
    "esd_residual_dense": (_c, [_vp, _vp, _vp, _vp, _vp]),
    "esd_rk4": (_c, [_vp, _vp, ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp]),
    "esd_residual_vjp": (_c, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "esd_rk4_vjp": (_c, [_vp, _vp, ctypes.c_double, ctypes.c_int32, _vp, _vp, _vp]),
    "esd_diagnostics": (_c, [_vp, _vp, ctypes.POINTER(ctypes.c_double), _vp, _vp]),
    "esd_sync_status": (_c, [_vp, _vp]),
    "esd_plan_set_graphs": (_c, [_vp, ctypes.c_int32]),
    "esd_plan_set_fused": (_c, [_vp, ctypes.c_int32]),
    "esd_plan_set_deterministic": (_c, [_vp, ctypes.c_int32]),
    "esd_plan_autotune": (_c, [_vp, _vp, _vp, _vp]),
    "esd_plan_get_tuning": (_c, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
    "esd_plan_set_timing": (_c, [_vp, ctypes.c_int32]),
    "esd_plan_get_timing": (_c, [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int64)]),
    "esd_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in EXPORTS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class EsdError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.esd_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(rc: int, where: str):
    if rc != ESD_OK:
        raise EsdError(rc, where)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class TorchAllocator:
    """Device memory of a plan's own arrays (tables, geometry, connectivity,
    status flag) taken from torch's caching allocator (esd_allocator): the
    blocks are torch tensors held here until the library frees them."""

    def __init__(self):
        import torch
        self.blocks = {}

        def _alloc(nbytes, ctx):
            try:
                t = torch.empty(max(1, (int(nbytes) + 7) // 8), dtype=torch.float64, device="cuda")
            except RuntimeError:
                return None
            self.blocks[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, ctx):
            self.blocks.pop(ptr, None)

        self._fns = (ALLOC_FN(_alloc), FREE_FN(_free))
        self.struct = _Allocator(self._fns[0], self._fns[1], None)

    @property
    def bytes(self):
        return sum(t.numel() * 8 for t in self.blocks.values())


class Plan:
    """A mesh + scheme set up on the device (esd_plan_create; with
    allocator=TorchAllocator() its device arrays come from torch)."""

    def __init__(self, dim: int, degree: int, elem_vertex_ids, elem_vertex_coords,
                 warp: Optional[Callable[[np.ndarray], np.ndarray]] = None, gamma: float = 1.4,
                 ecflux: int = FLUX_RANOCHA, dissipation: int = DISS_LLF_DAVIS, host_only: bool = False,
                 allocator: Optional[TorchAllocator] = None):
        self._ids = np.ascontiguousarray(elem_vertex_ids, dtype=np.int64)
        self._xy = np.ascontiguousarray(elem_vertex_coords, dtype=np.float64)
        ne = self._ids.shape[0]
        if warp is not None:
            def _cb(n, xin, xout, ctx, _dim=dim, _warp=warp):
                a = np.ctypeslib.as_array(xin, shape=(n * _dim,)).reshape(n, _dim)
                b = np.ctypeslib.as_array(xout, shape=(n * _dim,)).reshape(n, _dim)
                b[...] = _warp(a.copy())
            self._cb = WARP_FN(_cb)
        else:
            self._cb = WARP_FN()
        desc = _MeshDesc(dim, degree, ne, self._ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         self._xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self._cb, None)
        sch = _SchemeDesc(gamma, ecflux, dissipation)
        h = _vp()
        self.allocator = allocator
        if allocator is None:
            _check(_lib.esd_plan_create(ctypes.byref(desc), ctypes.byref(sch), 1 if host_only else 0,
                                        ctypes.byref(h)), "esd_plan_create")
        else:
            _check(_lib.esd_plan_create_ex(ctypes.byref(desc), ctypes.byref(sch), 1 if host_only else 0,
                                           ctypes.byref(allocator.struct), ctypes.byref(h)), "esd_plan_create_ex")
        self._h = h
        self.info = PlanInfo()
        _check(_lib.esd_plan_query(self._h, ctypes.byref(self.info)), "esd_plan_query")
        self.dim, self.degree, self.gamma = dim, degree, gamma
        self._ws = None

    @classmethod
    def from_workload(cls, wl, degree=None, host_only=False, **kw):
        mesh = wl.mesh()
        return cls(mesh.dim, degree or wl.degree, mesh.elem_vertex_ids, mesh.elem_vertex_coords,
                   None if wl.warp.__name__ == "warp_none" else wl.warp, wl.gamma,
                   kw.get("ecflux", wl.ecflux), kw.get("dissipation", wl.dissipation), host_only)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:      # the module may already be torn down at exit
            _lib.esd_plan_destroy(h)
            self._h = None

    # ---- shapes
    @property
    def state_shape(self):
        return (self.info.n_elements, self.info.n_vars, self.info.n_modes)

    @property
    def nodal_shape(self):
        return (self.info.n_elements, self.info.n_vol_nodes, self.info.n_vars)

    def host_array(self, name: str) -> np.ndarray:
        i = self.info
        nf, nq, d = i.n_facets * i.n_facet_nodes, i.n_vol_nodes, i.dim
        shapes = {"x_vol": (i.n_elements, nq, d), "J": (i.n_elements, nq), "G": (i.n_elements, nq, d, d),
                  "nJ": (i.n_elements, nf, d), "Jf": (i.n_elements, nf), "x_fac": (i.n_elements, nf, d),
                  "nbr": (i.n_elements, nf)}
        out = np.empty(shapes[name], dtype=np.float64)
        _check(_lib.esd_plan_host_array(self._h, name.encode(), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        out.size), "esd_plan_host_array")
        return out

    # ---- device calls
    def workspace(self, kind: str = "residual"):
        """Device workspace (one buffer per plan, grown on demand) for
        kind = "residual", "rk4", "vjp" or "rk4_vjp"."""
        import torch
        nbytes = {"residual": self.info.workspace_bytes, "rk4": self.info.rk4_workspace_bytes,
                  "vjp": self.info.vjp_workspace_bytes, "rk4_vjp": self.info.rk4_vjp_workspace_bytes}[kind]
        if self._ws is None or self._ws.numel() * 8 < nbytes:
            self._ws = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device="cuda")
        return self._ws

    def node_coords(self):
        import torch
        x = torch.empty((self.info.n_elements, self.info.n_vol_nodes, self.dim), dtype=torch.float64, device="cuda")
        _check(_lib.esd_node_coords(self._h, _ptr(x), _stream()), "esd_node_coords")
        return x

    def project(self, u_nodal):
        import torch
        assert u_nodal.is_cuda and u_nodal.dtype == torch.float64 and u_nodal.is_contiguous()
        assert tuple(u_nodal.shape) == self.nodal_shape
        out = torch.empty(self.state_shape, dtype=torch.float64, device=u_nodal.device)
        _check(_lib.esd_project(self._h, _ptr(u_nodal), _ptr(out), _stream()), "esd_project")
        return out

    def residual(self, u, out=None):
        import torch
        assert u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()
        assert tuple(u.shape) == self.state_shape
        if out is None:
            out = torch.empty_like(u)
        _check(_lib.esd_residual(self._h, _ptr(u), _ptr(out), _ptr(self.workspace()), _stream()), "esd_residual")
        return out

    def residual_dense(self, u, out=None):
        """esd_residual_dense: the residual with all-pairs volume and facet loops."""
        import torch
        assert u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()
        assert tuple(u.shape) == self.state_shape
        if out is None:
            out = torch.empty_like(u)
        _check(_lib.esd_residual_dense(self._h, _ptr(u), _ptr(out), _ptr(self.workspace()), _stream()),
               "esd_residual_dense")
        return out

    def residual_noalloc(self, u, out):
        """esd_residual_noalloc: the residual into the caller's out, with the
        library's fixed device scratch as workspace (no allocation anywhere)."""
        import torch
        assert u.is_cuda and u.dtype == torch.float64 and u.is_contiguous()
        assert out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
        assert tuple(u.shape) == self.state_shape and tuple(out.shape) == self.state_shape
        _check(_lib.esd_residual_noalloc(self._h, _ptr(u), _ptr(out), _stream()), "esd_residual_noalloc")
        return out

    def rk4(self, u, dt: float, nsteps: int, ckpt=None):
        """In place on u; ckpt (optional) receives the stage inputs [4*nsteps, *state]."""
        assert u.is_contiguous() and tuple(u.shape) == self.state_shape
        _check(_lib.esd_rk4(self._h, _ptr(u), float(dt), int(nsteps), _ptr(self.workspace("rk4")),
                            _ptr(ckpt), _stream()), "esd_rk4")
        return u

    def vjp(self, u, vbar, out=None):
        """(d du~/dt / d u~)^T vbar (esd_residual_vjp)."""
        import torch
        assert u.is_contiguous() and vbar.is_contiguous()
        assert tuple(u.shape) == self.state_shape and tuple(vbar.shape) == self.state_shape
        if out is None:
            out = torch.empty_like(u)
        _check(_lib.esd_residual_vjp(self._h, _ptr(u), _ptr(vbar), _ptr(out), _ptr(self.workspace("vjp")),
                                     _stream()), "esd_residual_vjp")
        return out

    def rk4_vjp(self, ckpt, dt: float, nsteps: int, ubar):
        """Discrete adjoint of rk4: ubar (cotangent of the final state) is
        replaced in place by the cotangent of the initial state; ckpt holds the
        stage inputs written by rk4(..., ckpt=...)."""
        assert ckpt.is_contiguous() and ubar.is_contiguous() and tuple(ubar.shape) == self.state_shape
        assert ckpt.numel() == 4 * nsteps * ubar.numel()
        _check(_lib.esd_rk4_vjp(self._h, _ptr(ckpt), float(dt), int(nsteps), _ptr(ubar),
                                _ptr(self.workspace("rk4_vjp")), _stream()), "esd_rk4_vjp")
        return ubar

    def diagnostics(self, u):
        """Conserved integrals (per variable), entropy integral and entropy rate
        of the state u (esd_diagnostics; synchronises)."""
        assert u.is_contiguous() and tuple(u.shape) == self.state_shape
        out = np.zeros(self.dim + 4, dtype=np.float64)
        _check(_lib.esd_diagnostics(self._h, _ptr(u), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    _ptr(self.workspace("rk4")), _stream()), "esd_diagnostics")
        nc = self.dim + 2
        return {"conserved": out[:nc].copy(), "entropy": float(out[nc]), "entropy_rate": float(out[nc + 1])}

    def set_graphs(self, enable: bool):
        _check(_lib.esd_plan_set_graphs(self._h, 1 if enable else 0), "esd_plan_set_graphs")

    def set_fused(self, enable: bool):
        """RK4 stages as one launch that also projects the next stage input."""
        _check(_lib.esd_plan_set_fused(self._h, int(bool(enable))), "esd_plan_set_fused")

    def set_deterministic(self, enable: bool):
        """esd_plan_set_deterministic: fixed-order sums in the right-hand side
        (bitwise-repeatable residuals and RK4 steps)."""
        _check(_lib.esd_plan_set_deterministic(self._h, int(bool(enable))), "esd_plan_set_deterministic")

    def autotune(self, u):
        """Times the right-hand-side block-size candidates of every bucket on u
        and keeps the fastest; returns the chosen block sizes."""
        assert u.is_contiguous() and tuple(u.shape) == self.state_shape
        _check(_lib.esd_plan_autotune(self._h, _ptr(u), _ptr(self.workspace("rk4")), _stream()), "esd_plan_autotune")
        return self.tuning()

    def tuning(self):
        """Right-hand-side (K2) block size per bucket; tuning_k1() the K1 ones."""
        n = len(getattr(self, "buckets", [None]))
        out = (ctypes.c_int32 * (2 * n))()
        _check(_lib.esd_plan_get_tuning(self._h, out, 2 * n), "esd_plan_get_tuning")
        self._k1_blocks = [out[n + b] for b in range(n)]
        return [out[b] for b in range(n)]

    def tuning_k1(self):
        self.tuning()
        return self._k1_blocks

    def tuning_fused(self) -> bool:
        """Whether RK4 stages are fused (as set at creation, by autotune or set_fused)."""
        nb = len(getattr(self, "buckets", [None]))
        buf = (ctypes.c_int32 * (2 * nb + 1))()
        _check(_lib.esd_plan_get_tuning(self._h, buf, 2 * nb + 1), "esd_plan_get_tuning")
        return bool(buf[2 * nb])

    def set_timing(self, enable: bool):
        _check(_lib.esd_plan_set_timing(self._h, 1 if enable else 0), "esd_plan_set_timing")

    def get_timing(self):
        """(k1_ms, k2_ms, launches) summed since the last call (HIP events)."""
        a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(_lib.esd_plan_get_timing(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)),
               "esd_plan_get_timing")
        return a.value, b.value, n.value

    def sync_status(self):
        _check(_lib.esd_sync_status(self._h, _stream()), "esd_sync_status")


def _warp_callback(dim, warp):
    if warp is None:
        return WARP_FN()

    def _cb(n, xin, xout, ctx, _dim=dim, _warp=warp):
        a = np.ctypeslib.as_array(xin, shape=(n * _dim,)).reshape(n, _dim)
        b = np.ctypeslib.as_array(xout, shape=(n * _dim,)).reshape(n, _dim)
        b[...] = _warp(a.copy())
    return WARP_FN(_cb)


class BatchedPlan(Plan):
    """Several meshes with per-element degrees in one plan
    (esd_plan_create_batched).  The state is a flat tensor [n_dof] holding the
    buckets one after the other ([element][variable][mode] inside a bucket);
    nodal arrays are flat [n_nodes, ...] in the same bucket order."""

    def __init__(self, dim: int, meshes, warp=None, gamma: float = 1.4, ecflux: int = FLUX_RANOCHA,
                 dissipation: int = DISS_LLF_DAVIS, host_only: bool = False,
                 allocator: Optional[TorchAllocator] = None):
        """meshes: list of (elem_vertex_ids, elem_vertex_coords, elem_degree)."""
        self._ids = [np.ascontiguousarray(m[0], dtype=np.int64) for m in meshes]
        self._xy = [np.ascontiguousarray(m[1], dtype=np.float64) for m in meshes]
        self._deg = [np.ascontiguousarray(m[2], dtype=np.int32) for m in meshes]
        nm = len(meshes)
        self._ne = np.array([a.shape[0] for a in self._ids], dtype=np.int64)
        P64, PD, P32 = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)
        self._pid = (P64 * nm)(*[a.ctypes.data_as(P64) for a in self._ids])
        self._pxy = (PD * nm)(*[a.ctypes.data_as(PD) for a in self._xy])
        self._pdeg = (P32 * nm)(*[a.ctypes.data_as(P32) for a in self._deg])
        self._cb = _warp_callback(dim, warp)
        desc = _BatchDesc(dim, nm, self._ne.ctypes.data_as(P64), self._pid, self._pxy, self._pdeg, self._cb, None)
        sch = _SchemeDesc(gamma, ecflux, dissipation)
        h = _vp()
        self.allocator = allocator
        if allocator is None:
            _check(_lib.esd_plan_create_batched(ctypes.byref(desc), ctypes.byref(sch), 1 if host_only else 0,
                                                ctypes.byref(h)), "esd_plan_create_batched")
        else:
            _check(_lib.esd_plan_create_batched_ex(ctypes.byref(desc), ctypes.byref(sch), 1 if host_only else 0,
                                                   ctypes.byref(allocator.struct), ctypes.byref(h)),
                   "esd_plan_create_batched_ex")
        self._h = h
        self.info = PlanInfo()
        _check(_lib.esd_plan_query(self._h, ctypes.byref(self.info)), "esd_plan_query")
        self.dim, self.degree, self.gamma = dim, None, gamma
        self._ws = None
        nb = ctypes.c_int32()
        deg = (ctypes.c_int32 * 16)()
        nel = (ctypes.c_int64 * 16)()
        doff = (ctypes.c_int64 * 17)()
        noff = (ctypes.c_int64 * 17)()
        _check(_lib.esd_plan_buckets(self._h, ctypes.byref(nb), deg, nel, doff, noff), "esd_plan_buckets")
        self.buckets = [dict(degree=deg[b], n_elements=nel[b], dof=(doff[b], doff[b + 1]), nodes=(noff[b], noff[b + 1]))
                        for b in range(nb.value)]
        ne = int(self.info.n_elements)
        self.elem_bucket = np.empty(ne, dtype=np.int32)
        self.elem_slot = np.empty(ne, dtype=np.int64)
        _check(_lib.esd_plan_element_map(self._h, self.elem_bucket.ctypes.data_as(P32),
                                         self.elem_slot.ctypes.data_as(P64), ne), "esd_plan_element_map")

    @property
    def state_shape(self):
        return (int(self.info.n_dof),)

    @property
    def n_nodes(self):
        return int(self.buckets[-1]["nodes"][1])

    @property
    def nodal_shape(self):
        return (self.n_nodes, self.info.n_vars)

    def bucket_view(self, u, b):
        """[n_elements, n_vars, n_modes] view of bucket b of a flat state."""
        bk = self.buckets[b]
        a, e = bk["dof"]
        return u[a:e].view(bk["n_elements"], self.info.n_vars, -1)

    def node_coords(self):
        import torch
        x = torch.empty((self.n_nodes, self.dim), dtype=torch.float64, device="cuda")
        _check(_lib.esd_node_coords(self._h, _ptr(x), _stream()), "esd_node_coords")
        return x


def _autograd_residual():
    import torch

    class Residual(torch.autograd.Function):
        """du~/dt = R(u~) with the hand-written adjoint kernel as backward."""

        @staticmethod
        def forward(ctx, u, plan):
            ctx.plan = plan
            ctx.save_for_backward(u)
            return plan.residual(u.contiguous())

        @staticmethod
        def backward(ctx, g):
            (u,) = ctx.saved_tensors
            return ctx.plan.vjp(u.contiguous(), g.contiguous()), None

    return Residual


def residual(u, plan: Plan):
    """Differentiable residual (torch.autograd)."""
    return _autograd_residual().apply(u, plan)


def _autograd_rk4():
    import torch

    class RK4(torch.autograd.Function):
        """nsteps of classical RK4; backward is the discrete adjoint from the
        stored stage inputs."""

        @staticmethod
        def forward(ctx, u, plan, dt, nsteps):
            out = u.detach().clone().contiguous()
            ckpt = torch.empty((4 * nsteps,) + tuple(u.shape), dtype=u.dtype, device=u.device)
            plan.rk4(out, dt, nsteps, ckpt)
            ctx.plan, ctx.dt, ctx.nsteps = plan, dt, nsteps
            ctx.save_for_backward(ckpt)
            return out

        @staticmethod
        def backward(ctx, g):
            (ckpt,) = ctx.saved_tensors
            ub = g.detach().clone().contiguous()
            ctx.plan.rk4_vjp(ckpt, ctx.dt, ctx.nsteps, ub)
            return ub, None, None, None

    return RK4


def rk4(u, plan: Plan, dt: float, nsteps: int):
    """Differentiable RK4 solve (torch.autograd); keeps 4*nsteps stage states."""
    return _autograd_rk4().apply(u, plan, dt, nsteps)
