"""Thin ctypes binding of libswe.so (include/swe.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels (device) or its C++ mesh toolkit (host).  Host arrays are numpy
arrays; device buffers are torch CUDA tensors (``data_ptr()``), used as
plumbing for memory only.  Importing this module fails loudly when the
library has not been built.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SWE_LIBRARY selects another build of the same library (e.g. a variant
# compiled with different flags for a measurement)
LIB_PATH = os.environ.get("SWE_LIBRARY", os.path.join(HERE, "libswe.so"))

SWE_ABI_VERSION = 5
SWE_OK = 0
ERRORS = {-1: "SWE_ERR_ARG", -2: "SWE_ERR_MESH", -3: "SWE_ERR_STATE", -4: "SWE_ERR_NONFINITE",
          -5: "SWE_ERR_NEGATIVE_DEPTH", -6: "SWE_ERR_DEVICE", -7: "SWE_ERR_OOM",
          -8: "SWE_ERR_UNSUPPORTED"}
F32, F64 = 0, 1
HLLC1, MUSCL, WAF = 0, 1, 2
EULER, RK2 = 0, 1
MINMOD, SUPERBEE, VANALBADA, LEARNED, ZEROSLOPE = 0, 1, 2, 3, 4
WAF_SUPERBEE, WAF_GODUNOV, WAF_UNLIMITED = 0, 1, 2
HOST, DEVICE = 0, 1
BC_WALL, BC_TRANSMISSIVE, BC_INFLOW, BC_OUTFLOW, BC_HALO = -1, -2, -3, -4, -5
HEALTH_NONFINITE, HEALTH_NEGDEPTH, HEALTH_CLIPPED = 1, 2, 4
MLP_NPARAM = 1569
PAIR_RECORD = 40


class SweError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libswe.so not built ({LIB_PATH}); run python paper_2307_16758_amd/build.py")
# torch ships its own HIP runtime.  Loading it first makes libswe.so bind to
# that same runtime (same soname); loading libswe.so first would put two HIP
# runtimes in the process and torch would then see no GPU.
try:
    import torch  # noqa: F401
except ImportError:  # torch is optional: host toolkit and host buffers need no torch
    pass
_lib = C.CDLL(LIB_PATH)

i32p = C.POINTER(C.c_int32)
f64p = C.POINTER(C.c_double)


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class swe_config(C.Structure):
    _fields_ = [("abi_version", C.c_int), ("precision", C.c_int), ("scheme", C.c_int),
                ("integrator", C.c_int), ("limiter", C.c_int), ("waf_limiter", C.c_int),
                ("cfl_rule", C.c_int), ("device", C.c_int), ("g", C.c_double),
                ("cfl", C.c_double), ("eps", C.c_double), ("dt_max", C.c_double),
                ("block", C.c_int), ("cell_kernel", C.c_int), ("stream", C.c_void_p),
                ("waves", C.c_int), ("phi_every", C.c_int), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_user", C.c_void_p), ("waf_positivity", C.c_int),
                ("phi_in_stage", C.c_int)]


class swe_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("node_xy", f64p), ("n_owned", C.c_int32),
                ("n_total", C.c_int32), ("cell_nodes", i32p), ("cell_gid", C.POINTER(C.c_int64)),
                ("cell_nbr", i32p), ("cell_b", f64p), ("cell_manning", f64p),
                ("n_peers", C.c_int32), ("peer_part", i32p), ("recv_off", i32p),
                ("send_off", i32p), ("send_idx", i32p), ("inflow_q", C.c_double),
                ("inflow_length", C.c_double), ("outflow_stage", C.c_double)]


class swe_subdomain_view(C.Structure):
    _fields_ = [("n_owned", C.c_int32), ("n_total", C.c_int32), ("n_peers", C.c_int32),
                ("n_send", C.c_int32)] + [
        (n, i32p) for n in ("l2g", "layer", "owner", "nbr", "peers", "recv_off", "send_off",
                            "send_idx")]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("swe_config_default", None, [C.POINTER(swe_config)])
_sig("swe_create", C.c_int, [C.POINTER(swe_config), C.POINTER(C.c_void_p)])
_sig("swe_destroy", None, [C.c_void_p])
_sig("swe_last_error", C.c_char_p, [C.c_void_p])
_sig("swe_strerror", C.c_char_p, [C.c_int])
_sig("swe_mesh_upload", C.c_int, [C.c_void_p, C.POINTER(swe_mesh)])
_sig("swe_set_bc_series", C.c_int, [C.c_void_p, C.c_int, f64p, f64p])
_sig("swe_set_state", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                C.c_double])
_sig("swe_read_state", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int])
_sig("swe_step", C.c_int, [C.c_void_p, C.c_int, C.c_double])
_sig("swe_prepare", C.c_int, [C.c_void_p, C.c_double])
_sig("swe_step_overlap", C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p])
_sig("swe_step_kernel", C.c_int, [C.c_void_p, C.POINTER(C.c_char_p), C.POINTER(C.c_int)])
_sig("swe_snapshot", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p])
_sig("swe_mesh_upload_batch", C.c_int, [C.c_void_p, C.c_int, C.POINTER(swe_mesh)])
_sig("swe_set_bc_series_scenario", C.c_int, [C.c_void_p, C.c_int, C.c_int, f64p, f64p])
_sig("swe_batch_offsets", C.c_int, [C.c_void_p, i32p, i32p])
_sig("swe_scenario_times", C.c_int, [C.c_void_p, f64p])
_sig("swe_autotune", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)])
_sig("swe_sync", C.c_int, [C.c_void_p])
_sig("swe_time", C.c_int, [C.c_void_p, f64p])
_sig("swe_local_dt", C.c_int, [C.c_void_p, f64p])
_sig("swe_health", C.c_int, [C.c_void_p, C.POINTER(C.c_int)])
_sig("swe_pack_ghosts", C.c_int, [C.c_void_p, C.c_void_p])
_sig("swe_unpack_ghosts", C.c_int, [C.c_void_p, C.c_void_p])
_sig("swe_ghost_sizes", C.c_int, [C.c_void_p, i32p, i32p])
_sig("swe_last_step_ms", C.c_int, [C.c_void_p, C.POINTER(C.c_float)])
_sig("swe_limiter_set_weights", C.c_int, [C.c_void_p, C.POINTER(C.c_float)])
_sig("swe_limiter_phi", C.c_int, [C.c_void_p, C.c_void_p])
_sig("swe_limiter_pairs", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p])
_sig("swe_trainer_create", C.c_int, [C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_void_p)])
_sig("swe_trainer_destroy", None, [C.c_void_p])
_sig("swe_trainer_loss_grad", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                        C.POINTER(C.c_float), C.POINTER(C.c_float),
                                        C.POINTER(C.c_float)])
_sig("swe_trainer_step", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int32,
                                   C.POINTER(C.c_float), C.c_float, C.POINTER(C.c_float)])
_sig("swe_trainer_get_params", C.c_int, [C.c_void_p, C.POINTER(C.c_float)])
_sig("swe_trainer_loss_grad_static", C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                               C.c_int32, C.POINTER(C.c_float), C.c_void_p,
                                               C.c_void_p])
_sig("swe_dual_graph", C.c_int, [C.c_int32, C.c_int32, i32p, i32p])
_sig("swe_partition_bfs", C.c_int, [C.c_int32, i32p, C.c_int32, i32p])
_sig("swe_edge_length_sum", C.c_int, [C.c_int32, f64p, C.c_int32, i32p, C.POINTER(C.c_int8),
                                      C.c_int32, f64p])
_sig("swe_morton_keys", C.c_int, [C.c_int32, f64p, C.c_int32, i32p, C.POINTER(C.c_uint32)])
_sig("swe_subdomain_build", C.c_int, [C.c_int32, f64p, C.c_int32, i32p, i32p,
                                      C.POINTER(C.c_int8), i32p, C.c_int32, C.c_int32,
                                      C.c_int32, C.POINTER(C.c_void_p)])
_sig("swe_subdomain_build_all", C.c_int, [C.c_int32, f64p, C.c_int32, i32p, i32p,
                                          C.POINTER(C.c_int8), i32p, C.c_int32, C.c_int32,
                                          C.c_int32, C.POINTER(C.c_void_p)])
_sig("swe_subdomain_build_layers", C.c_int, [C.c_int32, f64p, C.c_int32, i32p,
                                             C.POINTER(C.c_int8), i32p, C.c_int32, C.c_int32,
                                             C.c_int32, C.POINTER(C.c_void_p), i32p])
_sig("swe_subdomain_view_get", C.c_int, [C.c_void_p, C.POINTER(swe_subdomain_view)])
_sig("swe_subdomain_free", None, [C.c_void_p])

EXPORTED = ["swe_config_default", "swe_create", "swe_destroy", "swe_last_error", "swe_strerror",
            "swe_mesh_upload", "swe_set_bc_series", "swe_set_state", "swe_read_state",
            "swe_snapshot", "swe_step", "swe_step_overlap", "swe_prepare", "swe_step_kernel", "swe_mesh_upload_batch", "swe_set_bc_series_scenario",
            "swe_batch_offsets", "swe_scenario_times", "swe_autotune", "swe_sync", "swe_time", "swe_local_dt", "swe_health",
            "swe_pack_ghosts", "swe_unpack_ghosts", "swe_ghost_sizes", "swe_last_step_ms",
            "swe_limiter_set_weights", "swe_limiter_phi", "swe_limiter_pairs",
            "swe_trainer_create", "swe_trainer_destroy", "swe_trainer_loss_grad",
            "swe_trainer_step", "swe_trainer_get_params", "swe_trainer_loss_grad_static",
            "swe_dual_graph", "swe_partition_bfs", "swe_edge_length_sum", "swe_morton_keys", "swe_subdomain_build",
            "swe_subdomain_build_all", "swe_subdomain_build_layers", "swe_subdomain_view_get",
            "swe_subdomain_free"]


def lib():
    return _lib


def _i32(a):
    return a.ctypes.data_as(i32p)


def _f64(a):
    return a.ctypes.data_as(f64p)


def _check(rc, ctx=None):
    if rc != SWE_OK:
        msg = _lib.swe_last_error(ctx).decode() if ctx else _lib.swe_strerror(rc).decode()
        raise SweError(rc, msg)


# ------------------------------------------------------------ host toolkit
def swe_dual_graph(n_nodes: int, cell_nodes: np.ndarray) -> np.ndarray:
    t = np.ascontiguousarray(cell_nodes, np.int32)
    nbr = np.empty(t.shape, np.int32)
    _check(_lib.swe_dual_graph(n_nodes, t.shape[0], _i32(t), _i32(nbr)))
    return nbr


def swe_partition_bfs(nbr: np.ndarray, P: int) -> np.ndarray:
    nb = np.ascontiguousarray(nbr, np.int32)
    part = np.empty(nb.shape[0], np.int32)
    _check(_lib.swe_partition_bfs(nb.shape[0], _i32(nb), P, _i32(part)))
    return part


def swe_edge_length_sum(node_xy, cell_nodes, bc, tag) -> float:
    x = np.ascontiguousarray(node_xy, np.float64)
    t = np.ascontiguousarray(cell_nodes, np.int32)
    b = np.ascontiguousarray(bc, np.int8)
    out = C.c_double()
    _check(_lib.swe_edge_length_sum(x.shape[0], _f64(x), t.shape[0], _i32(t),
                                    b.ctypes.data_as(C.POINTER(C.c_int8)), tag, C.byref(out)))
    return out.value


def swe_morton_keys(node_xy: np.ndarray, cell_nodes: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(node_xy, np.float64)
    t = np.ascontiguousarray(cell_nodes, np.int32)
    key = np.empty(t.shape[0], np.uint32)
    _check(_lib.swe_morton_keys(x.shape[0], _f64(x), t.shape[0], _i32(t),
                                key.ctypes.data_as(C.POINTER(C.c_uint32))))
    return key


@dataclass
class SubDomain:
    n_owned: int
    n_total: int
    l2g: np.ndarray
    layer: np.ndarray
    owner: np.ndarray
    nbr: np.ndarray
    peers: np.ndarray
    recv_off: np.ndarray
    send_off: np.ndarray
    send_idx: np.ndarray


def swe_subdomain_build(node_xy, cell_nodes, nbr, bc, part, P, p, k) -> SubDomain:
    x = np.ascontiguousarray(node_xy, np.float64)
    t = np.ascontiguousarray(cell_nodes, np.int32)
    nb = np.ascontiguousarray(nbr, np.int32)
    b = np.ascontiguousarray(bc, np.int8)
    pa = np.ascontiguousarray(part, np.int32)
    h = C.c_void_p()
    _check(_lib.swe_subdomain_build(x.shape[0], _f64(x), t.shape[0], _i32(t), _i32(nb),
                                    b.ctypes.data_as(C.POINTER(C.c_int8)), _i32(pa), P, p, k,
                                    C.byref(h)))
    return _take_subdomain(h)


def swe_subdomain_build_all(node_xy, cell_nodes, nbr, bc, part, P, k, threads=0) -> list:
    """Every part of the partition, built on ``threads`` host threads."""
    x = np.ascontiguousarray(node_xy, np.float64)
    t = np.ascontiguousarray(cell_nodes, np.int32)
    nb = np.ascontiguousarray(nbr, np.int32)
    b = np.ascontiguousarray(bc, np.int8)
    pa = np.ascontiguousarray(part, np.int32)
    hs = (C.c_void_p * P)()
    _check(_lib.swe_subdomain_build_all(x.shape[0], _f64(x), t.shape[0], _i32(t), _i32(nb),
                                        b.ctypes.data_as(C.POINTER(C.c_int8)), _i32(pa), P, k,
                                        int(threads), hs))
    return [_take_subdomain(C.c_void_p(h)) for h in hs]


def swe_subdomain_build_layers(node_xy, cell_nodes, bc, part, P, k, threads=0):
    """Every part built from its own cells and its potential neighbours'
    inner boundary layers (no global dual graph); returns (parts, number of
    potential neighbours of each part)."""
    x = np.ascontiguousarray(node_xy, np.float64)
    t = np.ascontiguousarray(cell_nodes, np.int32)
    b = np.ascontiguousarray(bc, np.int8)
    pa = np.ascontiguousarray(part, np.int32)
    hs = (C.c_void_p * P)()
    npot = np.zeros(P, np.int32)
    _check(_lib.swe_subdomain_build_layers(x.shape[0], _f64(x), t.shape[0], _i32(t),
                                           b.ctypes.data_as(C.POINTER(C.c_int8)), _i32(pa), P, k,
                                           int(threads), hs, _i32(npot)))
    return [_take_subdomain(C.c_void_p(h)) for h in hs], npot


def _take_subdomain(h) -> SubDomain:
    """Copy a built sub-domain's arrays and free the library's object."""
    v = swe_subdomain_view()
    _check(_lib.swe_subdomain_view_get(h, C.byref(v)))

    def arr(ptr, n):
        return np.ctypeslib.as_array(ptr, shape=(n,)).copy() if n > 0 else np.zeros(0, np.int32)

    sd = SubDomain(v.n_owned, v.n_total, arr(v.l2g, v.n_total), arr(v.layer, v.n_total),
                   arr(v.owner, v.n_total), arr(v.nbr, 3 * v.n_total).reshape(-1, 3),
                   arr(v.peers, v.n_peers), arr(v.recv_off, v.n_peers + 1),
                   arr(v.send_off, v.n_peers + 1), arr(v.send_idx, v.n_send))
    _lib.swe_subdomain_free(h)
    return sd


# --------------------------------------------------------------- the mesh
@dataclass
class MeshArrays:
    """Arrays of a swe_mesh (host side), kept alive while uploaded."""
    node_xy: np.ndarray
    n_owned: int
    cell_nodes: np.ndarray
    cell_gid: np.ndarray
    cell_nbr: np.ndarray
    cell_b: np.ndarray
    cell_manning: np.ndarray
    peers: np.ndarray
    recv_off: np.ndarray
    send_off: np.ndarray
    send_idx: np.ndarray
    inflow_q: float = 0.0
    inflow_length: float = 0.0
    outflow_stage: float = 0.0

    @property
    def n_total(self):
        return int(self.cell_nodes.shape[0])

    def c_struct(self) -> swe_mesh:
        for name in ("node_xy", "cell_b", "cell_manning"):
            setattr(self, name, np.ascontiguousarray(getattr(self, name), np.float64))
        for name in ("cell_nodes", "cell_nbr", "peers", "recv_off", "send_off", "send_idx"):
            setattr(self, name, np.ascontiguousarray(getattr(self, name), np.int32))
        self.cell_gid = np.ascontiguousarray(self.cell_gid, np.int64)
        m = swe_mesh()
        m.n_nodes = self.node_xy.shape[0]
        m.node_xy = _f64(self.node_xy)
        m.n_owned = self.n_owned
        m.n_total = self.n_total
        m.cell_nodes = _i32(self.cell_nodes)
        m.cell_gid = self.cell_gid.ctypes.data_as(C.POINTER(C.c_int64))
        m.cell_nbr = _i32(self.cell_nbr)
        m.cell_b = _f64(self.cell_b)
        m.cell_manning = _f64(self.cell_manning)
        m.n_peers = self.peers.shape[0]
        m.peer_part = _i32(self.peers)
        m.recv_off = _i32(self.recv_off)
        m.send_off = _i32(self.send_off)
        m.send_idx = _i32(self.send_idx)
        m.inflow_q = self.inflow_q
        m.inflow_length = self.inflow_length
        m.outflow_stage = self.outflow_stage
        return m


def mesh_from_subdomain(node_xy, cell_nodes, cell_b, cell_manning, sd: SubDomain,
                        inflow_q=0.0, inflow_length=0.0, outflow_stage=0.0) -> MeshArrays:
    l2g = sd.l2g
    return MeshArrays(node_xy=node_xy, n_owned=sd.n_owned, cell_nodes=cell_nodes[l2g],
                      cell_gid=l2g.astype(np.int64), cell_nbr=sd.nbr,
                      cell_b=np.asarray(cell_b)[l2g], cell_manning=np.asarray(cell_manning)[l2g],
                      peers=sd.peers, recv_off=sd.recv_off, send_off=sd.send_off,
                      send_idx=sd.send_idx, inflow_q=inflow_q, inflow_length=inflow_length,
                      outflow_stage=outflow_stage)


# ----------------------------------------------------------- the solver
def config(**kw) -> swe_config:
    cfg = swe_config()
    _lib.swe_config_default(C.byref(cfg))
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def _ptr(a, where):
    if where == DEVICE:
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(a.ctypes.data)


# contexts whose buffers come from PyTorch's allocator: destroyed at exit
# while torch is still there to take the buffers back
_torch_backed = weakref.WeakSet()


@atexit.register
def _close_torch_backed():
    for s in list(_torch_backed):
        s.close()


def torch_allocator(device=0, stream=None):
    """(alloc, free) callbacks of the context configuration that take the
    context's device buffers from PyTorch's caching allocator, associated
    with ``stream`` (a torch.cuda.Stream; None: torch's current stream)."""
    import torch

    def _alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
        except RuntimeError:
            return None                   # the library reports SWE_ERR_OOM

    def _free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    return ALLOC_FN(_alloc), FREE_FN(_free)


class Snapshot:
    """A state on its way to pinned host memory (Solver.snapshot)."""

    def __init__(self, host, done):
        self._host, self._done = host, done

    def ready(self):
        return self._done.query()

    def wait(self):
        """(h, hu, hv) as numpy arrays over the pinned buffer."""
        self._done.synchronize()
        a = self._host.numpy()
        return a[0], a[1], a[2]


class Solver:
    """One swe_ctx: a sub-domain (or a whole mesh) on one GPU."""

    def __init__(self, stream=None, allocator=None, **cfg_kw):
        """stream: a torch.cuda.Stream (or raw hipStream_t handle) to borrow, so
        that torch work on it and the library's work are ordered.
        allocator: None (hipMalloc) or "torch" (PyTorch's caching allocator
        owns the context's device buffers)."""
        if stream is not None:
            cfg_kw["stream"] = getattr(stream, "cuda_stream", stream)
        self._stream = stream             # keeps a borrowed torch stream alive
        self._alloc_cbs = None
        if allocator == "torch":
            torch_stream = stream if hasattr(stream, "cuda_stream") else None
            self._alloc_cbs = torch_allocator(cfg_kw.get("device", 0), torch_stream)
            cfg_kw["alloc"], cfg_kw["free"] = self._alloc_cbs
        elif allocator is not None:
            raise ValueError("allocator: None or 'torch'")
        self.cfg = config(**cfg_kw)
        self.dtype = np.float64 if self.cfg.precision == F64 else np.float32
        h = C.c_void_p()
        _check(_lib.swe_create(C.byref(self.cfg), C.byref(h)))
        self.ctx = h
        self.mesh = None
        if self._alloc_cbs is not None:
            _torch_backed.add(self)

    def close(self):
        if getattr(self, "ctx", None):
            _lib.swe_destroy(self.ctx)    # frees through the callbacks, still alive here
            self.ctx = None
        self._alloc_cbs = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, rc):
        _check(rc, self.ctx)

    def _n_total(self):
        return self.mesh.n_total if self.mesh is not None else 0

    def _devbuf(self, t, n, what, dtype=None):
        """Pointer of a device buffer the library will read or write ``n``
        elements of: a contiguous CUDA tensor of the context's precision (or
        ``dtype``) with at least ``n`` elements, else ValueError (a wrong
        buffer would otherwise be overrun on the device)."""
        import torch
        want = dtype if dtype is not None else (torch.float64 if self.dtype == np.float64
                                                else torch.float32)
        if not (hasattr(t, "data_ptr") and getattr(t, "is_cuda", False)):
            raise ValueError(f"{what}: a CUDA tensor is required")
        if not t.is_contiguous():
            raise ValueError(f"{what}: the tensor must be contiguous")
        if t.dtype != want:
            raise ValueError(f"{what}: dtype {t.dtype}, the context needs {want}")
        if t.numel() < n:
            raise ValueError(f"{what}: {t.numel()} elements, at least {n} needed")
        return C.c_void_p(t.data_ptr())

    def mesh_upload(self, mesh: MeshArrays):
        s = mesh.c_struct()
        self._chk(_lib.swe_mesh_upload(self.ctx, C.byref(s)))
        self.mesh = mesh

    def mesh_upload_batch(self, meshes):
        structs = (swe_mesh * len(meshes))(*[m.c_struct() for m in meshes])
        self._chk(_lib.swe_mesh_upload_batch(self.ctx, len(meshes), structs))
        self.meshes = list(meshes)
        n = C.c_int32()
        self._chk(_lib.swe_batch_offsets(self.ctx, C.byref(n), None))
        off = np.empty(n.value + 1, np.int32)
        self._chk(_lib.swe_batch_offsets(self.ctx, C.byref(n), _i32(off)))
        self.offsets = off
        self.mesh = MeshArrays(node_xy=np.zeros((1, 2)), n_owned=int(off[-1]),
                               cell_nodes=np.zeros((int(off[-1]), 3), np.int32),
                               cell_gid=np.zeros(0, np.int64), cell_nbr=np.zeros(0, np.int32),
                               cell_b=np.zeros(0), cell_manning=np.zeros(0),
                               peers=np.zeros(0, np.int32), recv_off=np.zeros(1, np.int32),
                               send_off=np.zeros(1, np.int32), send_idx=np.zeros(0, np.int32))

    def set_bc_series_scenario(self, scen, t, q):
        t = np.ascontiguousarray(t, np.float64)
        q = np.ascontiguousarray(q, np.float64)
        self._chk(_lib.swe_set_bc_series_scenario(self.ctx, int(scen), t.shape[0], _f64(t), _f64(q)))

    def scenario_times(self):
        out = np.empty(len(self.offsets) - 1, np.float64)
        self._chk(_lib.swe_scenario_times(self.ctx, _f64(out)))
        return out

    def autotune(self, n_steps=10):
        b, g = C.c_int(), C.c_int()
        self._chk(_lib.swe_autotune(self.ctx, int(n_steps), C.byref(b), C.byref(g)))
        return b.value, g.value

    def set_bc_series(self, t, q):
        t = np.ascontiguousarray(t, np.float64)
        q = np.ascontiguousarray(q, np.float64)
        self._chk(_lib.swe_set_bc_series(self.ctx, t.shape[0], _f64(t), _f64(q)))

    def set_state(self, h, hu, hv, t=0.0):
        if hasattr(h, "data_ptr"):
            where = DEVICE
            for a in (h, hu, hv):
                self._devbuf(a, self._n_total(), "set_state")
        else:
            where = HOST
            h, hu, hv = (np.ascontiguousarray(a, self.dtype) for a in (h, hu, hv))
        self._chk(_lib.swe_set_state(self.ctx, _ptr(h, where), _ptr(hu, where), _ptr(hv, where),
                                     where, float(t)))

    def read_state(self, out=None):
        if out is None:
            n = self.mesh.n_total
            out = tuple(np.empty(n, self.dtype) for _ in range(3))
            where = HOST
        else:
            where = DEVICE if hasattr(out[0], "data_ptr") else HOST
            for a in out:
                if where == DEVICE:
                    self._devbuf(a, self._n_total(), "read_state")
                elif not (a.flags.c_contiguous and a.dtype == self.dtype and a.size >= self._n_total()):
                    raise ValueError("read_state: contiguous host arrays of the context's dtype "
                                     "with n_total elements are required")
        self._chk(_lib.swe_read_state(self.ctx, *(_ptr(a, where) for a in out), where))
        return out

    def snapshot(self, side_stream=None):
        """The state as it stands after the steps queued so far, copied to
        pinned host memory on side_stream (a torch.cuda.Stream; one per
        context by default) while the following steps run: swe_snapshot
        into one of two device staging slots, then a copy on the side
        stream.  Returns a Snapshot; its wait() gives (h, hu, hv)."""
        import torch
        dev = torch.device("cuda", self.cfg.device)
        n = self.mesh.n_total
        if getattr(self, "_snap", None) is None:
            tdt = torch.float64 if self.dtype == np.float64 else torch.float32
            slots = [torch.empty((3, n), dtype=tdt, device=dev) for _ in range(2)]
            # the context's stream is not ordered after torch's: let any
            # earlier torch work on the recycled memory finish first
            torch.cuda.current_stream(dev).synchronize()
            self._snap = dict(slots=slots, done=[None, None], next=0,
                              side=torch.cuda.Stream(dev))
        st = self._snap
        side = side_stream if side_stream is not None else st["side"]
        i = st["next"]
        st["next"] = 1 - i
        if st["done"][i] is not None:
            st["done"][i].synchronize()       # the slot's previous copy has left
        buf = st["slots"][i]
        ready = torch.cuda.Event()
        ready.record(torch.cuda.current_stream(dev))   # creates the event; re-recorded below
        self._chk(_lib.swe_snapshot(self.ctx, *(C.c_void_p(buf[f].data_ptr()) for f in range(3)),
                                    C.c_void_p(ready.cuda_event)))
        host = torch.empty(buf.shape, dtype=buf.dtype, pin_memory=True)
        side.wait_event(ready)
        with torch.cuda.stream(side):
            host.copy_(buf, non_blocking=True)
        done = torch.cuda.Event()
        done.record(side)
        st["done"][i] = done
        return Snapshot(host, done)

    def step(self, n_steps, dt_fixed=0.0):
        self._chk(_lib.swe_step(self.ctx, int(n_steps), float(dt_fixed)))

    def prepare(self, dt_fixed=0.0):
        """Build the step graph for dt_fixed now (nothing runs)."""
        self._chk(_lib.swe_prepare(self.ctx, float(dt_fixed)))

    def step_kernel(self):
        """(kernel name, launches per step) of the configured step."""
        n, k = C.c_char_p(), C.c_int()
        self._chk(_lib.swe_step_kernel(self.ctx, C.byref(n), C.byref(k)))
        return n.value.decode(), k.value

    def sync(self):
        self._chk(_lib.swe_sync(self.ctx))

    def time(self):
        t = C.c_double()
        self._chk(_lib.swe_time(self.ctx, C.byref(t)))
        return t.value

    def local_dt(self):
        t = C.c_double()
        self._chk(_lib.swe_local_dt(self.ctx, C.byref(t)))
        return t.value

    def health(self):
        b = C.c_int()
        self._chk(_lib.swe_health(self.ctx, C.byref(b)))
        return b.value

    def ghost_sizes(self):
        a, b = C.c_int32(), C.c_int32()
        self._chk(_lib.swe_ghost_sizes(self.ctx, C.byref(a), C.byref(b)))
        return a.value, b.value

    def pack_ghosts(self, buf):
        """Send values of every peer into ``buf`` ([3][n_send] SoA)."""
        n_send, _ = self.ghost_sizes()
        self._chk(_lib.swe_pack_ghosts(self.ctx, self._devbuf(buf, 3 * n_send, "pack_ghosts")))

    def step_overlap(self, buf, dt_fixed=0.0, event=None):
        """One step with the high-overlap schedule: the last stage's threads
        write the send cells' new values into ``buf`` ([3][n_send] SoA) as
        they compute them (no pack launch); ``event`` (a torch.cuda.Event,
        optional) is recorded once the buffer is complete."""
        n_send, _ = self.ghost_sizes()
        ev = None
        if event is not None:
            if hasattr(event, "cuda_event"):
                if not event.cuda_event:   # torch creates its events lazily, at the first record
                    event.record()
                ev = C.c_void_p(event.cuda_event)
            else:
                ev = C.c_void_p(event)
        self._chk(_lib.swe_step_overlap(self.ctx, float(dt_fixed),
                                        self._devbuf(buf, 3 * n_send, "step_overlap"), ev))

    def unpack_ghosts(self, buf):
        """Ghost values of every peer from ``buf`` ([3][n_ghost] SoA)."""
        _, n_ghost = self.ghost_sizes()
        self._chk(_lib.swe_unpack_ghosts(self.ctx, self._devbuf(buf, 3 * n_ghost, "unpack_ghosts")))

    def last_step_ms(self):
        f = C.c_float()
        self._chk(_lib.swe_last_step_ms(self.ctx, C.byref(f)))
        return f.value

    # ---------------------------------------------------- learned limiter
    def limiter_set_weights(self, params):
        p = np.ascontiguousarray(params, np.float32)
        assert p.shape == (MLP_NPARAM,)
        self._chk(_lib.swe_limiter_set_weights(self.ctx, p.ctypes.data_as(C.POINTER(C.c_float))))

    def limiter_phi(self, out):
        """phi of every half-edge into a float32 CUDA tensor of 3*n_total."""
        import torch
        self._chk(_lib.swe_limiter_phi(self.ctx, self._devbuf(out, 3 * self._n_total(),
                                                              "limiter_phi", torch.float32)))

    def limiter_pairs(self, fine: "Solver", children, out):
        """children: int32 CUDA tensor [4*n_total]; out: float32 CUDA tensor
        [3*n_total*40]."""
        import torch
        n = self._n_total()
        self._chk(_lib.swe_limiter_pairs(
            self.ctx, fine.ctx, self._devbuf(children, 4 * n, "limiter_pairs children", torch.int32),
            self._devbuf(out, 3 * n * PAIR_RECORD, "limiter_pairs records", torch.float32)))


def trainer_loss_grad_static(params, rec, idx, wv, out, stream=None):
    """swe_trainer_loss_grad_static: loss and gradient for device parameters
    without any allocation.  params: float32 CUDA tensor [1569]; rec: float32
    CUDA tensor [n_rec*40]; idx: int32 CUDA tensor [n]; out: float32 CUDA
    tensor [1570] (gradient, then the loss); queued on `stream` (a torch
    stream; default: the current one), not synchronised."""
    import torch
    for t, n, dt, what in ((params, MLP_NPARAM, torch.float32, "params"),
                           (rec, PAIR_RECORD, torch.float32, "rec"),
                           (idx, 1, torch.int32, "idx"),
                           (out, MLP_NPARAM + 1, torch.float32, "out")):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == dt and t.numel() >= n):
            raise SweError(-1, f"trainer_loss_grad_static: {what} must be a contiguous "
                                        f"CUDA {dt} tensor of at least {n} elements")
    w = np.ascontiguousarray(wv, np.float32)
    assert w.shape == (4,)
    st = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    _check(_lib.swe_trainer_loss_grad_static(
        C.c_void_p(params.data_ptr()), C.c_void_p(rec.data_ptr()), rec.numel() // PAIR_RECORD,
        C.c_void_p(idx.data_ptr()), idx.numel(), w.ctypes.data_as(C.POINTER(C.c_float)),
        C.c_void_p(out.data_ptr()), C.c_void_p(st)))


class Trainer:
    """FP32 Adam trainer of the limiter network (device kernels)."""

    def __init__(self, init_params, device=0):
        p = np.ascontiguousarray(init_params, np.float32)
        assert p.shape == (MLP_NPARAM,)
        h = C.c_void_p()
        _check(_lib.swe_trainer_create(device, p.ctypes.data_as(C.POINTER(C.c_float)), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _lib.swe_trainer_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    @staticmethod
    def _wv(wv):
        w = np.ascontiguousarray(wv, np.float32)
        assert w.shape == (4,)
        return w

    def loss_grad(self, rec, idx, wv):
        w = self._wv(wv)
        loss = C.c_float()
        g = np.empty(MLP_NPARAM, np.float32)
        n_rec = rec.numel() // PAIR_RECORD
        _check(_lib.swe_trainer_loss_grad(self.h, C.c_void_p(rec.data_ptr()), n_rec,
                                          C.c_void_p(idx.data_ptr()), idx.numel(),
                                          w.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss),
                                          g.ctypes.data_as(C.POINTER(C.c_float))))
        return loss.value, g

    def step(self, rec, idx, wv, lr):
        w = self._wv(wv)
        loss = C.c_float()
        n_rec = rec.numel() // PAIR_RECORD
        _check(_lib.swe_trainer_step(self.h, C.c_void_p(rec.data_ptr()), n_rec,
                                     C.c_void_p(idx.data_ptr()), idx.numel(),
                                     w.ctypes.data_as(C.POINTER(C.c_float)), float(lr),
                                     C.byref(loss)))
        return loss.value

    def params(self):
        p = np.empty(MLP_NPARAM, np.float32)
        _check(_lib.swe_trainer_get_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float))))
        return p
