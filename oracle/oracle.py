"""TEST INFRASTRUCTURE ONLY -- Python access to the serial FP64 oracle.

Loads ``oracle/liboracle.so`` (built from ``swe_oracle.c`` and
``decomp_oracle.c`` with gcc, no fast-math, no FP contraction).  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark use
this module; the HIP library never imports it and it never imports the
library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "swe_oracle.c"), os.path.join(HERE, "decomp_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")

HLLC1, MUSCL, WAF = 0, 1, 2
EULER, RK2 = 0, 1
MINMOD, SUPERBEE, VANALBADA, LEARNED, ZEROSLOPE = 0, 1, 2, 3, 4
WAF_SUPERBEE, WAF_GODUNOV, WAF_UNLIMITED = 0, 1, 2
FL_NONFINITE, FL_NEGDEPTH, FL_CLIPPED = 1, 2, 4
MLP_IN, MLP_H = 14, 32
MLP_NPAR = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1


def build(force: bool = False) -> str:
    stale = not os.path.exists(LIB) or any(
        os.path.getmtime(s) > os.path.getmtime(LIB) for s in SRCS)
    if force or stale:
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-std=c99", "-fPIC", "-shared", "-o", tmp] + SRCS + ["-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [("g", C.c_double), ("cfl", C.c_double), ("eps", C.c_double),
                ("dt_max", C.c_double), ("scheme", C.c_int), ("integrator", C.c_int),
                ("limiter", C.c_int), ("waf_limiter", C.c_int), ("cfl_rule", C.c_int),
                ("mlp_bf16", C.c_int), ("inflow_q", C.c_double),
                ("inflow_len", C.c_double), ("outflow_stage", C.c_double),
                ("n_series", C.c_int), ("pad", C.c_int),
                ("series_t", C.POINTER(C.c_double)), ("series_q", C.POINTER(C.c_double)),
                ("mlp", C.POINTER(C.c_double)), ("waf_pos", C.c_int), ("phi_every", C.c_int)]


class _Sub(C.Structure):
    _fields_ = [("n_owned", C.c_int), ("n_total", C.c_int), ("n_peers", C.c_int),
                ("n_send", C.c_int)] + [
        (n, C.POINTER(C.c_int)) for n in
        ("l2g", "layer", "owner", "nbr", "peers", "recv_off", "send_off", "send_idx")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        _lib.or_mesh_new.restype = C.c_void_p
        _lib.or_mesh_new.argtypes = [C.c_int, dp, C.c_int, C.c_int, ip,
                                     C.POINTER(C.c_int64), ip, dp, dp]
        _lib.or_mesh_free.argtypes = [C.c_void_p]
        _lib.or_mesh_geometry.argtypes = [C.c_void_p] + [dp] * 7
        _lib.or_run.argtypes = [C.c_void_p, C.POINTER(_Params), dp, dp, dp, C.c_int,
                                C.c_double, dp, ip]
        _lib.or_dt.argtypes = [C.c_void_p, C.POINTER(_Params), dp, dp, dp, dp]
        _lib.or_interfaces.argtypes = [C.c_void_p, C.POINTER(_Params), dp, dp, dp,
                                       dp, dp, dp, dp, ip]
        _lib.or_riemann.argtypes = [C.POINTER(_Params), C.c_int, dp, dp, C.c_double, dp, dp]
        _lib.or_waf_positivity.argtypes = [C.POINTER(_Params), dp, dp, C.c_double, C.c_double,
                                           C.c_double, C.c_double, C.c_double, dp]
        _lib.or_limiter.restype = C.c_double
        _lib.or_limiter.argtypes = [C.c_int, C.c_double, C.c_double]
        _lib.or_superbee_A.restype = C.c_double
        _lib.or_superbee_A.argtypes = [C.c_double, C.c_double]
        _lib.or_bf16.restype = C.c_double
        _lib.or_bf16.argtypes = [C.c_double]
        _lib.or_mlp_forward.argtypes = [dp, C.c_int, dp, C.c_int, dp]
        _lib.or_mlp_loss_grad.restype = C.c_double
        _lib.or_mlp_loss_grad.argtypes = [dp, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        _lib.or_limiter_inputs.argtypes = [C.c_void_p, C.POINTER(_Params), dp, dp, dp, dp, dp]
        _lib.od_neighbors.argtypes = [C.c_int, C.c_int, ip, ip]
        _lib.od_partition.argtypes = [C.c_int, ip, C.c_int, ip]
        _lib.od_morton.argtypes = [C.c_int, dp, C.c_int, ip, C.POINTER(C.c_uint32)]
        _lib.od_subdomain.restype = C.POINTER(_Sub)
        _lib.od_subdomain.argtypes = [C.c_int, dp, C.c_int, ip, ip, C.POINTER(C.c_int8),
                                      ip, C.c_int, C.c_int, C.c_int]
        _lib.od_sub_free.argtypes = [C.POINTER(_Sub)]
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


@dataclass
class Params:
    g: float = 9.81
    cfl: float = 0.45
    eps: float = 1e-6
    dt_max: float = 0.0
    scheme: int = HLLC1
    integrator: int = EULER
    limiter: int = MINMOD
    waf_limiter: int = WAF_SUPERBEE
    waf_pos: int = 1
    phi_every: int = 1
    cfl_rule: int = 0
    mlp_bf16: int = 0
    inflow_q: float = 0.0
    inflow_len: float = 1.0
    outflow_stage: float = 0.0
    hydrograph: tuple | None = None
    mlp: np.ndarray | None = None
    _keep: list = field(default_factory=list, repr=False)

    def c(self) -> _Params:
        p = _Params(self.g, self.cfl, self.eps, self.dt_max, self.scheme, self.integrator,
                    self.limiter, self.waf_limiter, self.cfl_rule, self.mlp_bf16,
                    self.inflow_q, self.inflow_len, self.outflow_stage, 0, 0)
        p.waf_pos = self.waf_pos
        p.phi_every = self.phi_every
        self._keep = []
        if self.hydrograph is not None:
            t = np.ascontiguousarray(self.hydrograph[0], np.float64)
            q = np.ascontiguousarray(self.hydrograph[1], np.float64)
            self._keep += [t, q]
            p.n_series = t.shape[0]
            p.series_t, p.series_q = _d(t), _d(q)
        if self.mlp is not None:
            w = np.ascontiguousarray(self.mlp, np.float64)
            assert w.shape == (MLP_NPAR,)
            self._keep.append(w)
            p.mlp = _d(w)
        return p


def neighbors(n_nodes: int, tri: np.ndarray) -> np.ndarray:
    """Cell across each local edge (-1 if none), global numbering."""
    t = np.ascontiguousarray(tri, np.int32)
    nbr = np.empty(t.shape, np.int32)
    rc = lib().od_neighbors(n_nodes, t.shape[0], _i(t), _i(nbr))
    if rc != 0:
        raise ValueError(f"od_neighbors failed ({rc})")
    return nbr


def partition(nbr: np.ndarray, P: int) -> np.ndarray:
    nb = np.ascontiguousarray(nbr, np.int32)
    part = np.empty(nb.shape[0], np.int32)
    if lib().od_partition(nb.shape[0], _i(nb), P, _i(part)) != 0:
        raise ValueError("od_partition failed")
    return part


def morton(xy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(xy, np.float64)
    t = np.ascontiguousarray(tri, np.int32)
    k = np.empty(t.shape[0], np.uint32)
    lib().od_morton(x.shape[0], _d(x), t.shape[0], _i(t), k.ctypes.data_as(C.POINTER(C.c_uint32)))
    return k


@dataclass
class SubDomain:
    n_owned: int
    n_total: int
    l2g: np.ndarray
    layer: np.ndarray
    owner: np.ndarray
    nbr: np.ndarray        # [n_total, 3] local index or negative tag
    peers: np.ndarray
    recv_off: np.ndarray
    send_off: np.ndarray
    send_idx: np.ndarray


def subdomain(xy, tri, nbr_g, bc, part, P, p, k) -> SubDomain:
    x = np.ascontiguousarray(xy, np.float64)
    t = np.ascontiguousarray(tri, np.int32)
    nb = np.ascontiguousarray(nbr_g, np.int32)
    b = np.ascontiguousarray(bc, np.int8)
    pa = np.ascontiguousarray(part, np.int32)
    S = lib().od_subdomain(x.shape[0], _d(x), t.shape[0], _i(t), _i(nb),
                           b.ctypes.data_as(C.POINTER(C.c_int8)), _i(pa), P, p, k)
    s = S.contents

    def arr(ptr, n):
        return np.ctypeslib.as_array(ptr, shape=(max(n, 0),)).copy() if n > 0 else np.zeros(0, np.int32)

    out = SubDomain(s.n_owned, s.n_total, arr(s.l2g, s.n_total), arr(s.layer, s.n_total),
                    arr(s.owner, s.n_total), arr(s.nbr, 3 * s.n_total).reshape(-1, 3),
                    arr(s.peers, s.n_peers), arr(s.recv_off, s.n_peers + 1),
                    arr(s.send_off, s.n_peers + 1), arr(s.send_idx, s.n_send))
    lib().od_sub_free(S)
    return out


class Mesh:
    """Oracle mesh: cells numbered 0..n-1, ``nbr`` local index or negative tag."""

    def __init__(self, xy, tri, nbr, b, manning, gid=None, n_owned=None):
        self.xy = np.ascontiguousarray(xy, np.float64)
        self.tri = np.ascontiguousarray(tri, np.int32)
        self.nbr = np.ascontiguousarray(nbr, np.int32)
        n = self.tri.shape[0]
        self.n = n
        self.n_owned = n if n_owned is None else int(n_owned)
        self.gid = np.ascontiguousarray(np.arange(n) if gid is None else gid, np.int64)
        self.b = np.ascontiguousarray(b, np.float64)
        self.manning = np.ascontiguousarray(manning, np.float64)
        self.h = lib().or_mesh_new(self.xy.shape[0], _d(self.xy), n, self.n_owned,
                                   _i(self.tri), self.gid.ctypes.data_as(C.POINTER(C.c_int64)),
                                   _i(self.nbr), _d(self.b), _d(self.manning))
        if not self.h:
            raise ValueError("oracle rejected the mesh (orientation or neighbour table)")
        self._free = lib().or_mesh_free      # still reachable at interpreter exit

    def __del__(self):
        if getattr(self, "h", None) and getattr(self, "_free", None):
            self._free(self.h)
            self.h = None

    def geometry(self):
        n = self.n
        out = [np.empty(n) for _ in range(4)] + [np.empty(3 * n) for _ in range(3)]
        lib().or_mesh_geometry(self.h, *[_d(a) for a in out])
        area, cx, cy, inr, enx, eny, elen = out
        return dict(area=area, cx=cx, cy=cy, inr=inr, nx=enx.reshape(n, 3),
                    ny=eny.reshape(n, 3), len=elen.reshape(n, 3))

    def run(self, params: Params, h, hu, hv, nsteps, dt_fixed=0.0, t=0.0):
        h = np.array(h, np.float64, copy=True)
        hu = np.array(hu, np.float64, copy=True)
        hv = np.array(hv, np.float64, copy=True)
        tt = np.array([t], np.float64)
        fl = np.zeros(1, np.int32)
        p = params.c()
        rc = lib().or_run(self.h, C.byref(p), _d(h), _d(hu), _d(hv), int(nsteps),
                          float(dt_fixed), _d(tt), _i(fl))
        if rc != 0:
            raise RuntimeError("or_run failed (no wet cell and no dt_max)")
        return h, hu, hv, float(tt[0]), int(fl[0])

    def dt(self, params: Params, h, hu, hv) -> float:
        h, hu, hv = (np.ascontiguousarray(a, np.float64) for a in (h, hu, hv))
        out = np.zeros(1)
        p = params.c()
        if lib().or_dt(self.h, C.byref(p), _d(h), _d(hu), _d(hv), _d(out)) != 0:
            raise RuntimeError("or_dt failed")
        return float(out[0])

    def interfaces(self, params: Params, h, hu, hv):
        """h-, b-, u_n-, u_t- (own outward-normal frame) and second-order flag."""
        h, hu, hv = (np.ascontiguousarray(a, np.float64) for a in (h, hu, hv))
        n3 = 3 * self.n
        rh, rb, run, rut = (np.empty(n3) for _ in range(4))
        sec = np.empty(n3, np.int32)
        p = params.c()
        lib().or_interfaces(self.h, C.byref(p), _d(h), _d(hu), _d(hv), _d(rh), _d(rb),
                            _d(run), _d(rut), _i(sec))
        return rh.reshape(-1, 3), rb.reshape(-1, 3), run.reshape(-1, 3), \
            rut.reshape(-1, 3), sec.reshape(-1, 3)


def limiter_inputs(mesh: "Mesh", params: Params, h, hu, hv):
    """Per half-edge [n, 3, 32]: features[14], q[4], central slopes[4], d_mid,
    eligible, backward slopes[4], forward slopes[4]; and phi [n, 3] (0.5
    where not eligible)."""
    h, hu, hv = (np.ascontiguousarray(a, np.float64) for a in (h, hu, hv))
    out = np.empty((mesh.n, 3, 32))
    phi = np.empty((mesh.n, 3))
    p = params.c()
    lib().or_limiter_inputs(mesh.h, C.byref(p), _d(h), _d(hu), _d(hv), _d(out), _d(phi))
    return out, phi


def waf_positivity(params: Params, UL, UR, hL, RL, hR, RR, dt, F):
    """The positivity blend of WAF applied to the flux F of one edge."""
    UL, UR = (np.ascontiguousarray(a, np.float64) for a in (UL, UR))
    out = np.array(F, np.float64, copy=True)
    p = params.c()
    lib().or_waf_positivity(C.byref(p), _d(UL), _d(UR), float(hL), float(RL), float(hR),
                            float(RR), float(dt), _d(out))
    return out


def riemann(params: Params, scheme, UL, UR, dt_dx=0.0, ratio_in=None):
    ul = np.ascontiguousarray(UL, np.float64)
    ur = np.ascontiguousarray(UR, np.float64)
    F = np.zeros(3)
    p = params.c()
    ri = None if ratio_in is None else np.ascontiguousarray(ratio_in, np.float64)
    lib().or_riemann(C.byref(p), scheme, _d(ul), _d(ur), float(dt_dx),
                     _d(ri) if ri is not None else None, _d(F))
    return F


def limiter(kind, sb, sf) -> float:
    return lib().or_limiter(kind, float(sb), float(sf))


def superbee_A(r, c) -> float:
    return lib().or_superbee_A(float(r), float(c))


def bf16(x) -> float:
    return lib().or_bf16(float(x))


def mlp_forward(params, x, bf16_inputs=False):
    w = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, MLP_IN)
    phi = np.empty(x.shape[0])
    lib().or_mlp_forward(_d(w), x.shape[0], _d(x), int(bool(bf16_inputs)), _d(phi))
    return phi


def mlp_loss_grad(params, x, q, s, sb, sf, d, t, wv):
    """Loss of the limiter training and its gradient (see swe_oracle.c):
    misfit of q + d clip(phi s, sb, sf) against the targets t."""
    w = np.ascontiguousarray(params, np.float64)
    x = np.ascontiguousarray(x, np.float64).reshape(-1, MLP_IN)
    q, s, sb, sf, t = (np.ascontiguousarray(a, np.float64).reshape(-1, 4) for a in (q, s, sb, sf, t))
    d = np.ascontiguousarray(d, np.float64).ravel()
    wv = np.ascontiguousarray(wv, np.float64).ravel()
    g = np.zeros(MLP_NPAR)
    loss = lib().or_mlp_loss_grad(_d(w), x.shape[0], _d(x), _d(q), _d(s), _d(sb), _d(sf), _d(d),
                                  _d(t), _d(wv), _d(g))
    return loss, g


# ------------------------------------------------------------ scenario glue
def global_mesh(sc):
    """Oracle mesh of a whole scenario in its generator numbering."""
    nbr_g = neighbors(sc.mesh.n_nodes, sc.mesh.tri)
    nbr = np.where(nbr_g >= 0, nbr_g, sc.bc.astype(np.int32))
    nbr = np.where((nbr_g < 0) & (nbr == 0), -1, nbr)
    return Mesh(sc.mesh.xy, sc.mesh.tri, nbr, sc.b, sc.manning), nbr_g


def inflow_length(sc) -> float:
    """Total length of the inflow edges of a scenario."""
    p = sc.mesh.xy[sc.mesh.tri]
    q = np.roll(p, -1, axis=1)
    L = np.sqrt(((q - p) ** 2).sum(-1))
    return float(L[sc.bc == -3].sum())


def scenario_params(sc, **kw) -> Params:
    p = Params(**kw)
    p.inflow_q = sc.inflow_q
    p.inflow_len = max(inflow_length(sc), 1e-300)
    p.outflow_stage = sc.outflow_stage
    p.hydrograph = sc.hydrograph
    return p
