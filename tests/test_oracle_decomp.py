"""Pins of the oracle's ghost-layer machinery (Sec. 3.1 - 3.3) by brute force
on small meshes, and the sub-domain invariant of Sec. 6.3.1: with enough
ghost layers a sub-domain reproduces the undecomposed solution exactly."""
from collections import deque

import numpy as np
import pytest

from helpers import python_neighbors
from oracle import oracle as O
from swe_inputs import grid_mesh, dam_break_channel, river_channel
from swe_inputs.scenarios import _build, _flat_bed
from swe_inputs.mesh import BC_WALL


def small_mesh(nx=12, ny=8, seed=3):
    return grid_mesh(12.0, 8.0, nx, ny, seed)


def test_neighbors_match_dictionary():
    m = small_mesh()
    nb = O.neighbors(m.n_nodes, m.tri)
    np.testing.assert_array_equal(nb, python_neighbors(m.tri))
    # symmetric: c is the neighbour of its neighbour
    for c in range(m.n_cells):
        for k in nb[c]:
            if k >= 0:
                assert c in nb[k]


def test_neighbors_reject_bad_orientation():
    m = small_mesh(4, 3)
    tri = m.tri.copy()
    tri[5] = tri[5][[0, 2, 1]]
    with pytest.raises(ValueError):
        O.neighbors(m.n_nodes, tri)


def bfs_dist(nbr, sources):
    dist = np.full(nbr.shape[0], -1)
    q = deque()
    for s in sources:
        dist[s] = 0
        q.append(s)
    while q:
        c = q.popleft()
        for k in nbr[c]:
            if k >= 0 and dist[k] < 0:
                dist[k] = dist[c] + 1
                q.append(k)
    return dist


@pytest.mark.parametrize("P", [1, 3, 5, 8])
def test_partition_sizes_and_greedy_rule(P):
    m = small_mesh(16, 10)
    nb = O.neighbors(m.n_nodes, m.tri)
    part = O.partition(nb, P)
    n = m.n_cells
    sizes = np.bincount(part, minlength=P)
    np.testing.assert_array_equal(sizes, [n // P + (p < n % P) for p in range(P)])
    # each part starts at the lowest id not taken by earlier parts
    taken = np.zeros(n, bool)
    for p in range(P):
        first = np.where(~taken)[0][0]
        assert part[first] == p
        taken |= part == p


def morton_ref(xy, tri):
    c = xy[tri].sum(axis=1) / 3.0
    c = ((xy[tri[:, 0]] + xy[tri[:, 1]]) + xy[tri[:, 2]]) / 3.0
    lo = c.min(0)
    S = (c.max(0) - lo).max()
    q = np.clip(np.floor((c - lo) / S * 65536.0), 0, 65535).astype(np.uint64)
    key = np.zeros(c.shape[0], np.uint64)
    for b in range(16):
        key |= ((q[:, 0] >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        key |= ((q[:, 1] >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return key.astype(np.uint32)


def test_morton_keys():
    m = small_mesh(20, 9)
    np.testing.assert_array_equal(O.morton(m.xy, m.tri), morton_ref(m.xy, m.tri))


def brute_subdomain(m, nb, part, p, k):
    """All-pairs style brute force: distances from every part's cell set."""
    P = part.max() + 1
    d = {q: bfs_dist(nb, np.where(part == q)[0]) for q in range(P)}
    dp = d[p]
    ghosts = [c for c in range(m.n_cells) if 1 <= dp[c] <= k]
    peers = sorted({int(part[c]) for c in ghosts})
    send = {q: [c for c in range(m.n_cells) if part[c] == p and 1 <= d[q][c] <= k]
            for q in peers}
    return dp, ghosts, peers, send, d


@pytest.mark.parametrize("P,k", [(4, 1), (4, 2), (5, 3), (3, 4)])
def test_ghost_layers_brute_force(P, k):
    sc = dam_break_channel(Lx=16.0, Ly=10.0, nx=16, ny=10, x_dam=8.0)
    m = sc.mesh
    nb = O.neighbors(m.n_nodes, m.tri)
    part = O.partition(nb, P)
    key = morton_ref(m.xy, m.tri)
    for p in range(P):
        S = O.subdomain(m.xy, m.tri, nb, sc.bc, part, P, p, k)
        dp, ghosts, peers, send, d = brute_subdomain(m, nb, part, p, k)
        owned = np.where(part == p)[0]
        assert S.n_owned == owned.size
        assert sorted(S.l2g[:S.n_owned]) == sorted(owned)
        assert sorted(S.l2g[S.n_owned:]) == sorted(ghosts)
        np.testing.assert_array_equal(S.peers, peers)
        np.testing.assert_array_equal(S.layer, dp[S.l2g])
        np.testing.assert_array_equal(S.owner, part[S.l2g])
        # owned order: send cells by (destination tuple, morton, gid), then interior
        dest = {int(c): tuple(q for q in peers if c in set(send[q])) for c in owned}
        want = sorted([c for c in owned if dest[c]], key=lambda c: (dest[c], key[c], c)) + \
            sorted([c for c in owned if not dest[c]], key=lambda c: (key[c], c))
        np.testing.assert_array_equal(S.l2g[:S.n_owned], want)
        # ghosts: per owner ascending, (layer, morton, gid)
        gwant = sorted(ghosts, key=lambda c: (part[c], dp[c], key[c], c))
        np.testing.assert_array_equal(S.l2g[S.n_owned:], gwant)
        for j, q in enumerate(peers):
            blk = S.l2g[S.n_owned + S.recv_off[j]:S.n_owned + S.recv_off[j + 1]]
            assert np.all(part[blk] == q)
            sl = S.l2g[S.send_idx[S.send_off[j]:S.send_off[j + 1]]]
            np.testing.assert_array_equal(
                sl, sorted(send[q], key=lambda c: (d[q][c], key[c], c)))
        # local neighbour table: local ids, boundary tags, cut edges at layer k only
        g2l = {int(c): i for i, c in enumerate(S.l2g)}
        for i, c in enumerate(S.l2g):
            for mm in range(3):
                gk = nb[c, mm]
                v = S.nbr[i, mm]
                if gk >= 0 and int(gk) in g2l:
                    assert v == g2l[int(gk)]
                elif gk >= 0:
                    assert v == -5 and S.layer[i] == k
                else:
                    assert v == sc.bc[c, mm] and v < 0


def test_send_lists_land_in_place():
    """The send list p -> q is, cell for cell, q's receive block from p."""
    sc = river_channel(Lx=2000.0, Ly=400.0, nx=40, ny=10, seed=7)
    m = sc.mesh
    nb = O.neighbors(m.n_nodes, m.tri)
    P = 6
    part = O.partition(nb, P)
    for k in (1, 2, 4):
        subs = [O.subdomain(m.xy, m.tri, nb, sc.bc, part, P, p, k) for p in range(P)]
        owned_total = sum(S.n_owned for S in subs)
        assert owned_total == m.n_cells
        for p, S in enumerate(subs):
            for j, q in enumerate(S.peers):
                Sq = subs[q]
                jq = list(Sq.peers).index(p)
                sent = S.l2g[S.send_idx[S.send_off[j]:S.send_off[j + 1]]]
                recv = Sq.l2g[Sq.n_owned + Sq.recv_off[jq]:Sq.n_owned + Sq.recv_off[jq + 1]]
                np.testing.assert_array_equal(sent, recv)


def _sub_mesh(sc, S):
    l2g = S.l2g
    return O.Mesh(sc.mesh.xy, sc.mesh.tri[l2g], S.nbr, sc.b[l2g], sc.manning[l2g],
                  gid=l2g, n_owned=S.n_owned)


def _wavy(sc):
    c = sc.mesh.centroids()
    h = 1.0 + 0.3 * np.sin(0.9 * c[:, 0]) * np.cos(0.7 * c[:, 1]) - 0.002 * c[:, 0]
    return h, 0.1 * h * np.cos(c[:, 1]), -0.05 * h * np.sin(c[:, 0])


CASES = [("hllc1_euler", dict(scheme=O.HLLC1, integrator=O.EULER), 1),
         ("muscl_euler", dict(scheme=O.MUSCL, integrator=O.EULER, limiter=O.SUPERBEE), 2),
         ("waf_euler", dict(scheme=O.WAF, integrator=O.EULER), 2),
         ("muscl_rk2", dict(scheme=O.MUSCL, integrator=O.RK2, limiter=O.MINMOD), 4)]


@pytest.mark.parametrize("name,kw,r", CASES)
@pytest.mark.parametrize("k", [1, 2, 4])
def test_k_ghost_invariant(name, kw, r, k):
    """Fixed dt: owned cells of a sub-domain with k layers equal the global
    run bitwise for s <= floor(k/r) steps, and differ at floor(k/r)+1."""
    mesh = grid_mesh(20.0, 12.0, 20, 12, seed=13)
    sc = _build("wavy", mesh, lambda x, y: 0.01 * x + 0.05 * np.sin(y), lambda x, y, b:
                (np.ones_like(x), np.zeros_like(x), np.zeros_like(x)), 0.03,
                {s: BC_WALL for s in range(4)})
    sc.h, sc.hu, sc.hv = _wavy(sc)
    M, nb = O.global_mesh(sc)
    P = 4
    part = O.partition(nb, P)
    p = O.scenario_params(sc, **kw)
    dt = 0.5 * M.dt(p, sc.h, sc.hu, sc.hv)
    smax = k // r
    gl = [M.run(p, sc.h, sc.hu, sc.hv, s, dt_fixed=dt) for s in range(smax + 2)]
    for q in range(P):
        S = O.subdomain(sc.mesh.xy, sc.mesh.tri, nb, sc.bc, part, P, q, k)
        Ms = _sub_mesh(sc, S)
        own = S.l2g[:S.n_owned]
        for s in range(1, smax + 2):
            h, hu, hv, _, _ = Ms.run(p, sc.h[S.l2g], sc.hu[S.l2g], sc.hv[S.l2g], s, dt_fixed=dt)
            same = (np.array_equal(h[:S.n_owned], gl[s][0][own])
                    and np.array_equal(hu[:S.n_owned], gl[s][1][own])
                    and np.array_equal(hv[:S.n_owned], gl[s][2][own]))
            if s <= smax:
                assert same, (name, k, q, s)
            elif q == 0:
                assert not same, (name, k, q, s)   # negative control (too few layers)


@pytest.mark.parametrize("name,kw,r", CASES)
def test_exchange_reproduces_global_run(name, kw, r):
    """Fake communicator: P sub-domains step floor(k/r) steps, then every
    receive block is filled from the peer's packed send list; after several
    exchanges the owned cells equal the global run bitwise."""
    k = 4
    mesh = grid_mesh(20.0, 12.0, 20, 12, seed=17)
    sc = _build("wavy", mesh, _flat_bed, lambda x, y, b:
                (np.ones_like(x), np.zeros_like(x), np.zeros_like(x)), 0.0,
                {s: BC_WALL for s in range(4)})
    sc.h, sc.hu, sc.hv = _wavy(sc)
    M, nb = O.global_mesh(sc)
    P = 5
    part = O.partition(nb, P)
    p = O.scenario_params(sc, **kw)
    dt = 0.5 * M.dt(p, sc.h, sc.hu, sc.hv)
    per = k // r
    rounds = 3
    gh, ghu, ghv, _, _ = M.run(p, sc.h, sc.hu, sc.hv, per * rounds, dt_fixed=dt)
    subs = [O.subdomain(sc.mesh.xy, sc.mesh.tri, nb, sc.bc, part, P, q, k) for q in range(P)]
    meshes = [_sub_mesh(sc, S) for S in subs]
    st = [[sc.h[S.l2g].copy(), sc.hu[S.l2g].copy(), sc.hv[S.l2g].copy()] for S in subs]
    for _ in range(rounds):
        for q in range(P):
            st[q][0], st[q][1], st[q][2], _, _ = meshes[q].run(p, *st[q], per, dt_fixed=dt)
        packed = [[np.stack([v[S.send_idx] for v in st[q]])] for q, S in enumerate(subs)]
        for q, S in enumerate(subs):
            for j, src in enumerate(S.peers):
                Ss = subs[src]
                js = list(Ss.peers).index(q)
                buf = packed[src][0][:, Ss.send_off[js]:Ss.send_off[js + 1]]
                lo, hi = S.n_owned + S.recv_off[j], S.n_owned + S.recv_off[j + 1]
                for f in range(3):
                    st[q][f][lo:hi] = buf[f]
    for q, S in enumerate(subs):
        own = S.l2g[:S.n_owned]
        assert np.array_equal(st[q][0][:S.n_owned], gh[own])
        assert np.array_equal(st[q][1][:S.n_owned], ghu[own])
        assert np.array_equal(st[q][2][:S.n_owned], ghv[own])
