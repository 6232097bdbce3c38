"""Sub-domains with k ghost layers on the GPU (Sec. 3.2 - 3.3, Sec. 6.3.1,
Sec. 6.4): the owned cells of a sub-domain equal the undecomposed GPU run
bitwise for floor(k/r) fixed-dt steps (r = stencil radius of one step), the
on-device pack gathers exactly the send lists, and P sub-domains that
exchange packed buffers through in-place receives reproduce the global run
bitwise."""
import numpy as np
import pytest

from gpu_util import make_pair, lib
from swe_inputs import grid_mesh
from swe_inputs.scenarios import _build
from swe_inputs.mesh import BC_WALL

pytestmark = pytest.mark.gpu

CASES = [("hllc1", 1), ("muscl_minmod_euler", 2), ("waf", 2), ("muscl_minmod_rk2", 4)]


def wavy_scenario(nx=40, ny=24, seed=13):
    mesh = grid_mesh(40.0, 24.0, nx, ny, seed=seed)
    sc = _build("wavy", mesh, lambda x, y: 0.01 * x + 0.05 * np.sin(y),
                lambda x, y, b: (np.ones_like(x), np.zeros_like(x), np.zeros_like(x)), 0.03,
                {s: BC_WALL for s in range(4)})
    c = mesh.centroids()
    sc.h = 1.0 + 0.3 * np.sin(0.9 * c[:, 0]) * np.cos(0.7 * c[:, 1]) - 0.002 * c[:, 0]
    sc.hu = 0.1 * sc.h * np.cos(c[:, 1])
    sc.hv = -0.05 * sc.h * np.sin(c[:, 0])
    return sc


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name,r", CASES)
def test_subdomain_equals_global(name, r, prec):
    swe, prepare_scenario = lib()
    sc = wavy_scenario()
    g, M, par, prg = make_pair(sc, name, precision=prec)
    dt = 0.5 * M.dt(par, sc.h[prg.sub.l2g], sc.hu[prg.sub.l2g], sc.hv[prg.sub.l2g])
    P = 4
    for k in (1, 2, 4):
        smax = k // r
        ref = {}
        for s in range(1, smax + 2):
            g.set_state(sc.h[prg.sub.l2g], sc.hu[prg.sub.l2g], sc.hv[prg.sub.l2g])
            g.step(s, dt)
            st = g.read_state()
            ref[s] = [np.empty_like(st[0]) for _ in range(3)]
            for f in range(3):
                ref[s][f][prg.sub.l2g] = st[f]
        for q in range(P):
            pr = prepare_scenario(sc, P=P, p=q, k=k, nbr_global=prg.nbr_global)
            sub, _, _, _ = make_pair(sc, name, precision=prec, prepared=pr)
            own = pr.sub.l2g[:pr.sub.n_owned]
            for s in range(1, smax + 2):
                sub.set_state(sc.h[pr.sub.l2g], sc.hu[pr.sub.l2g], sc.hv[pr.sub.l2g])
                sub.step(s, dt)
                st = sub.read_state()
                same = all(np.array_equal(st[f][:pr.sub.n_owned], ref[s][f][own]) for f in range(3))
                if s <= smax:
                    assert same, (name, prec, k, q, s)
                elif q == 0:
                    assert not same, (name, prec, k, q, s)


def test_pack_and_unpack():
    import torch
    swe, prepare_scenario = lib()
    sc = wavy_scenario()
    pr = prepare_scenario(sc, P=3, p=1, k=2)
    s, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=0, prepared=pr)
    s.step(3)
    n_send, n_ghost = s.ghost_sizes()
    assert n_send == pr.sub.send_idx.size and n_ghost == pr.sub.n_total - pr.sub.n_owned
    buf = torch.empty(3 * n_send, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    s.pack_ghosts(buf)
    s.sync()                          # the pack runs on the library's stream
    st = s.read_state()
    b = buf.cpu().numpy().reshape(3, n_send)
    for f in range(3):
        assert np.array_equal(b[f], st[f][pr.sub.send_idx])
    rec = torch.arange(3 * n_ghost, dtype=torch.float32, device="cuda") * 1e-3 + 0.5
    torch.cuda.synchronize()          # torch's writes before the library reads
    s.unpack_ghosts(rec)
    st2 = s.read_state()
    r = rec.cpu().numpy().reshape(3, n_ghost)
    for f in range(3):
        assert np.array_equal(st2[f][pr.sub.n_owned:], r[f])
        assert np.array_equal(st2[f][:pr.sub.n_owned], st[f][:pr.sub.n_owned])


@pytest.mark.parametrize("name,r", CASES)
def test_exchange_reproduces_global(name, r):
    """Fake communicator on one GPU: five sub-domain contexts, k = 4, packed
    send buffers copied device-to-device into the peers' receive blocks."""
    import torch
    swe, prepare_scenario = lib()
    sc = wavy_scenario()
    g, M, par, prg = make_pair(sc, name, precision=0)
    dt = 0.5 * M.dt(par, sc.h[prg.sub.l2g], sc.hu[prg.sub.l2g], sc.hv[prg.sub.l2g])
    k, P, rounds = 4, 5, 3
    per = k // r
    g.step(per * rounds, dt)
    gst = g.read_state()
    ref = [np.empty_like(gst[0]) for _ in range(3)]
    for f in range(3):
        ref[f][prg.sub.l2g] = gst[f]
    preps = [prepare_scenario(sc, P=P, p=q, k=k, nbr_global=prg.nbr_global) for q in range(P)]
    subs = [make_pair(sc, name, precision=0, prepared=pr)[0] for pr in preps]
    for _ in range(rounds):
        for s in subs:
            s.step(per, dt)
        packed = []
        for s, pr in zip(subs, preps):
            buf = torch.empty(3 * max(1, pr.sub.send_idx.size), dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            s.pack_ghosts(buf)
            s.sync()
            packed.append(buf[:3 * pr.sub.send_idx.size].view(3, -1))
        for q, (s, pr) in enumerate(zip(subs, preps)):
            n_ghost = pr.sub.n_total - pr.sub.n_owned
            rb = torch.empty(3, max(1, n_ghost), dtype=torch.float32, device="cuda")
            for j, src in enumerate(pr.sub.peers):
                ps = preps[src].sub
                js = list(ps.peers).index(q)
                rb[:, pr.sub.recv_off[j]:pr.sub.recv_off[j + 1]] = \
                    packed[src][:, ps.send_off[js]:ps.send_off[js + 1]]
            rv = rb[:, :n_ghost].contiguous().view(-1)
            torch.cuda.synchronize()
            s.unpack_ghosts(rv)
            s.sync()
    for s, pr in zip(subs, preps):
        st = s.read_state()
        own = pr.sub.l2g[:pr.sub.n_owned]
        for f in range(3):
            assert np.array_equal(st[f][:pr.sub.n_owned], ref[f][own]), (name, f)


def test_borrowed_stream_orders_with_torch():
    """With the caller's stream borrowed (swe_config.stream), torch work
    queued on that stream after a pack sees the packed buffer without any
    synchronisation, and an unpack sees torch's writes made before it."""
    import torch
    swe, prepare_scenario = lib()
    sc = wavy_scenario()
    pr = prepare_scenario(sc, P=3, p=1, k=2)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=0, prepared=pr, stream=st)
        s.step(4)
        n_send, n_ghost = s.ghost_sizes()
        buf = torch.zeros(3 * n_send, dtype=torch.float32, device="cuda")
        s.pack_ghosts(buf)
        packed = buf.clone()                       # queued on st, after the pack
        rec = torch.arange(3 * n_ghost, dtype=torch.float32, device="cuda") * 1e-3 + 0.25
        s.unpack_ghosts(rec)
    state = s.read_state()
    b = packed.cpu().numpy().reshape(3, n_send)
    r = rec.cpu().numpy().reshape(3, n_ghost)
    for f in range(3):
        assert np.array_equal(state[f][pr.sub.n_owned:], r[f])
    s2, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=0, prepared=pr)
    s2.step(4)
    ref = s2.read_state()
    for f in range(3):
        assert np.array_equal(b[f], ref[f][pr.sub.send_idx])


@pytest.mark.parametrize("name,k", [("hllc1", 2), ("waf", 2), ("muscl_minmod_euler", 4)])
def test_health_counts_owned_cells_only(name, k):
    """A ghost cell's new state is provisional (the next exchange replaces
    it), so a depth driven negative there raises no error; the same state in
    an owned cell does.  Lake at rest, except that the outermost ghost layer
    (or, as the control, as many owned cells) gets 20 m/s with a step far
    beyond its CFL limit: one Euler step cannot carry that layer's state to
    an owned cell, whose new states equal those of the unperturbed run
    bitwise."""
    swe, prepare_scenario = lib()
    sc = wavy_scenario()
    sc.h = np.maximum(1.2 - sc.b, 0.0)
    sc.hu = np.zeros_like(sc.h)
    sc.hv = np.zeros_like(sc.h)
    pr = prepare_scenario(sc, P=3, p=1, k=k)
    n_own = pr.sub.n_owned
    outer = np.where((pr.sub.nbr == swe.BC_HALO).any(axis=1))[0]
    assert outer.size > 0 and outer.min() >= n_own
    inner = np.arange(n_own // 2, n_own // 2 + outer.size)
    runs = {}
    for where, cells in (("none", outer[:0]), ("ghost", outer), ("owned", inner)):
        s, _, _, _ = make_pair(sc, name, precision=0, prepared=pr)
        h, hu, hv = (x[pr.sub.l2g].copy() for x in (sc.h, sc.hu, sc.hv))
        hu[cells] = 20.0 * h[cells]
        hv[cells] = -20.0 * h[cells]
        s.set_state(h, hu, hv)
        if where == "owned":
            with pytest.raises(swe.SweError):
                s.step(1, 5.0)
                s.sync()
            continue
        s.step(1, 5.0)
        s.sync()
        assert s.health() == 0, where
        runs[where] = s.read_state()
    for f in range(3):
        assert np.array_equal(runs["ghost"][f][:n_own], runs["none"][f][:n_own])
    g = runs["ghost"][0][outer]
    assert np.any((g == 0) | ~np.isfinite(g))   # the layer was driven dry (clipped)
