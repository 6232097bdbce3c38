"""Degenerate and boundary-size inputs through the C ABI.

* meshes smaller than one tile and meshes with a ragged last tile, for
  every block size, against the FP64 oracle;
* a single closed cell (the smallest mesh): only Manning friction acts;
* an all-dry domain, and a dam break onto a dry bed (moving wet/dry front);
* empty and oversized meshes, out-of-range batch sizes, calls out of order
  and zero-length ghost lists, each with its documented status.
"""
import ctypes as C
import math

import numpy as np
import pytest

from gpu_util import make_pair, state_errors, lib
from helpers import one_cell_basin
from oracle import oracle as O
from swe_inputs import river_channel, dam_break_channel, strip_riemann

pytestmark = pytest.mark.gpu


def _oracle_run(M, par, sc, l2g, nsteps, dt_fixed=0.0):
    return M.run(par, sc.h[l2g], sc.hu[l2g], sc.hv[l2g], nsteps, dt_fixed=dt_fixed)


def _vector_errors(g, r, n_owned):
    """max |gpu - oracle| over owned cells, relative to max |h| for the depth
    and to the largest momentum component for both momenta (on a 30-cell
    reach the lateral momentum is 1e-4 of the streamwise one, and round-off
    relative to that near-zero field alone says nothing)."""
    g = [np.asarray(x[:n_owned], np.float64) for x in g]
    r = [np.asarray(x[:n_owned], np.float64) for x in r[:3]]
    q = max(np.abs(r[1]).max(), np.abs(r[2]).max())
    return (np.abs(g[0] - r[0]).max() / np.abs(r[0]).max(),
            np.abs(g[1] - r[1]).max() / q, np.abs(g[2] - r[2]).max() / q)


@pytest.mark.parametrize("nx,ny", [(5, 3), (37, 9)])
@pytest.mark.parametrize("block", [64, 128, 256, 512])
def test_small_and_ragged_meshes(nx, ny, block):
    """30 cells (less than one tile of any size) and 666 cells (a ragged last
    tile for every block size) of a river reach with inflow, outlet, dry
    banks and bumps: MUSCL-superbee-RK2 in FP64 in CFL mode, every cell
    against the oracle."""
    sc = river_channel(Lx=40.0 * nx, Ly=40.0 * ny, nx=nx, ny=ny, seed=17, n_bumps=4,
                       inflow_q=50.0)
    assert sc.n_cells % block != 0
    s, M, par, pr = make_pair(sc, "muscl_superbee_rk2", precision=1, block=block)
    s.step(120)
    g = s.read_state()
    r = _oracle_run(M, par, sc, pr.sub.l2g, 120)
    errs = _vector_errors(g, r, pr.sub.n_owned)
    assert max(errs) <= 1e-10, errs
    assert s.time() == pytest.approx(r[3], rel=1e-12)


def test_ragged_tiles_bitwise_across_block_sizes():
    """The same FP32 state and clock for every block size when the last tile
    is ragged."""
    sc = river_channel(Lx=1480.0, Ly=360.0, nx=37, ny=9, seed=17, n_bumps=4, inflow_q=50.0)
    ref = None
    for block in (64, 128, 256, 512):
        s, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=0, block=block)
        s.step(60)
        out = s.read_state() + (s.time(),)
        if ref is None:
            ref = out
            continue
        for x, y in zip(ref[:3], out[:3]):
            assert np.array_equal(x, y), block
        assert ref[3] == out[3]


@pytest.mark.parametrize("name,prec", [("hllc1", 1), ("muscl_minmod_rk2", 1), ("waf", 1),
                                       ("muscl_minmod_rk2", 0)])
def test_single_closed_cell(name, prec):
    """One triangle with three walls: depth unchanged, the current decays by
    Manning friction alone (1/|u| = 1/|u0| + k t for the Euler schemes), and
    the GPU follows the oracle step for step."""
    h0, u0, v0, n = 1.3, 0.5, -0.25, 0.035
    sc = one_cell_basin(h=h0, u=u0, v=v0, n=n)
    s, M, par, pr = make_pair(sc, name, precision=prec)
    assert pr.mesh.n_owned == 1
    s.step(80)
    g = s.read_state()
    r = _oracle_run(M, par, sc, pr.sub.l2g, 80)
    # FP32: a few ulps per step, 80 steps of two stages
    tol = 1e-12 if prec == 1 else 1e-5
    assert max(state_errors(g, r[:3], 1)) <= tol
    assert s.time() == pytest.approx(r[3], rel=tol)
    assert abs(float(g[0][0]) - h0) <= (1e-14 if prec == 1 else 1e-7) * h0
    if name != "muscl_minmod_rk2":
        k = 9.81 * n * n * h0 ** (-4.0 / 3.0)
        speed = 1.0 / (1.0 / math.hypot(u0, v0) + k * s.time())
        assert math.isclose(math.hypot(g[1][0], g[2][0]) / g[0][0], speed, rel_tol=1e-12)


@pytest.mark.parametrize("prec", [1, 0])
def test_all_dry_domain(prec):
    """No wet cell: with dt_max the state stays exactly dry and every step
    takes dt_max; without it the step is zero and the clock stays put."""
    sc = dam_break_channel(Lx=20.0, Ly=4.0, nx=10, ny=2, h_left=0.0, h_right=0.0)
    for dt_max, t_end in ((0.25, 2.0), (0.0, 0.0)):
        s, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=prec, dt_max=dt_max)
        s.step(8)
        h, hu, hv = s.read_state()
        assert not h.any() and not hu.any() and not hv.any()
        assert s.time() == t_end
        assert s.health() == 0


@pytest.mark.parametrize("name", ["hllc1", "muscl_minmod_rk2", "waf"])
def test_dam_break_onto_dry_bed(name):
    """Ritter's problem on a strip (the dry side has h = 0 exactly): the
    wet/dry front moves into dry cells; FP64 GPU against the oracle in CFL
    mode, and mass exactly conserved between the walls."""
    sc = strip_riemann(L=20.0, W=1.0, nx=200, ny=4, x0=8.0, hL=1.0, hR=0.0, ends=-1)
    s, M, par, pr = make_pair(sc, name, precision=1)
    s.step(150)
    g = s.read_state()
    r = _oracle_run(M, par, sc, pr.sub.l2g, 150)
    errs = state_errors(g, r[:3], pr.sub.n_owned)
    # WAF switches discretely (the branches of its superbee ratio and
    # weights, and where its mass flux meets a cell's positivity bound): a
    # rounding-order difference can pick another branch at an isolated
    # edge, so it gets 1e-9
    assert max(errs) <= (1e-9 if name == "waf" else 1e-10), errs
    A = M.geometry()["area"]
    m0 = (A * sc.h[pr.sub.l2g]).sum()
    assert abs((A * g[0]).sum() - m0) <= 1e-12 * m0
    assert (g[0] > 0).sum() > (sc.h > 0).sum()          # the front has advanced


@pytest.mark.parametrize("prec", [1, 0])
def test_waf_on_a_river_stays_non_negative(prec):
    """WAF on a river with dry banks, bumps and inflow for 1500 CFL steps:
    with every edge's mass flux kept within its donor cells' shares (the
    positivity blend towards HLLC) no depth goes below zero at all (no
    negative depth, not even one clipped at round-off), and the state tracks
    the oracle's over the first steps.  Without the blend the oracle goes
    negative on this river (tests/test_oracle_physics.py)."""
    sc = river_channel(Lx=2000.0, Ly=400.0, nx=160, ny=32, seed=2)
    s, M, par, pr = make_pair(sc, "waf", precision=prec)
    s.step(20)
    g = s.read_state()
    r = _oracle_run(M, par, sc, pr.sub.l2g, 20)
    errs = _vector_errors(g, r, pr.sub.n_owned)
    assert max(errs) <= (1e-9 if prec == 1 else 1e-4), errs
    s.step(1480)
    h, _, _ = s.read_state()
    assert s.health() == 0 and h.min() >= 0.0


def _bare_mesh(n_total, n_nodes=3):
    """A mesh struct that declares sizes only (every array pointer NULL)."""
    swe, _ = lib()
    m = swe.swe_mesh()
    m.n_nodes = n_nodes
    m.n_owned = n_total
    m.n_total = n_total
    return m


ARG, MESH, STATE, UNSUPPORTED = -1, -2, -3, -8       # SWE_ERR_* of include/swe.h


def _status(fn, *args):
    swe, _ = lib()
    return getattr(swe._lib, fn)(*args)


def test_size_limits_and_call_order():
    swe, prepare_scenario = lib()
    for bad in (dict(waves=5), dict(block=96), dict(cell_kernel=2), dict(phi_every=4),
                dict(phi_every=-1)):
        with pytest.raises(swe.SweError) as e:
            swe.Solver(precision=0, **bad)
        assert e.value.code == ARG
    s32 = swe.Solver(precision=0)
    s64 = swe.Solver(precision=1)
    # no cells
    for s in (s32, s64):
        assert _status("swe_mesh_upload", s.ctx, C.byref(_bare_mesh(0))) == MESH
    # per-cell arrays beyond 4 GiB: checked before any array is read
    assert _status("swe_mesh_upload", s32.ctx, C.byref(_bare_mesh(90_000_000))) == UNSUPPORTED
    assert _status("swe_mesh_upload", s64.ctx, C.byref(_bare_mesh(45_000_000))) == UNSUPPORTED
    # just under the FP64 limit the sizes pass and the missing arrays are reported
    assert _status("swe_mesh_upload", s64.ctx, C.byref(_bare_mesh(44_000_000))) == MESH
    # batches: at least one mesh, at most 32768 (the count is checked first)
    one = (swe.swe_mesh * 1)(_bare_mesh(0))
    assert _status("swe_mesh_upload_batch", s32.ctx, 0, one) == ARG
    assert _status("swe_mesh_upload_batch", s32.ctx, 32769, one) == ARG
    # calls out of order
    assert _status("swe_step", s32.ctx, 1, C.c_double(0.0)) == STATE
    sc = dam_break_channel(Lx=20.0, Ly=4.0, nx=10, ny=2)
    pr = prepare_scenario(sc)
    s32.mesh_upload(pr.mesh)
    assert _status("swe_step", s32.ctx, 1, C.c_double(0.0)) == STATE
    h = np.empty(pr.mesh.n_total, np.float32)
    hp = C.c_void_p(h.ctypes.data)
    assert _status("swe_read_state", s32.ctx, hp, hp, hp, swe.HOST) == STATE
    s32.set_state(sc.h[pr.sub.l2g], sc.hu[pr.sub.l2g], sc.hv[pr.sub.l2g])
    assert _status("swe_step", s32.ctx, -1, C.c_double(0.0)) == ARG
    s32.step(0)                                   # zero steps: nothing happens
    assert s32.time() == 0.0
    # no ghost cells: pack and unpack have nothing to move and accept NULL
    assert s32.ghost_sizes() == (0, 0)
    assert _status("swe_pack_ghosts", s32.ctx, None) == swe.SWE_OK
    assert _status("swe_unpack_ghosts", s32.ctx, None) == swe.SWE_OK
    s32.step(3)
    assert s32.time() > 0.0 and s32.health() == 0
    s32.close()
    s64.close()
