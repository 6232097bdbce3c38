"""High-overlap steps (Sec. 6.4: the send cells are computed first and
their exchange overlaps the interior): swe_step_overlap gives bitwise the
state, clock and send buffer of a plain step followed by a pack, for every
scheme, both precisions, several tile sizes and in CFL mode; a caller's
stream that waits on the pack event sees the finished buffer; sub-domain
contexts exchanging through overlapped steps reproduce the global run."""
import numpy as np
import pytest

from gpu_util import make_pair, lib
from test_gpu_ghosts import wavy_scenario, CASES

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("block", [64, 256])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("name,r", CASES)
def test_overlap_step_equals_step_and_pack(name, r, prec, block):
    import torch
    swe, prepare_scenario = lib()
    sc = wavy_scenario()
    tdt = torch.float32 if prec == 0 else torch.float64
    for cfl_mode in (False, True):
        pr = prepare_scenario(sc, P=3, p=1, k=2)
        a, _, _, _ = make_pair(sc, name, precision=prec, prepared=pr, block=block)
        b, _, _, _ = make_pair(sc, name, precision=prec, prepared=pr, block=block)
        n_send, _ = a.ghost_sizes()
        assert 0 < pr.sub.send_idx.max() + 1 < pr.sub.n_total
        dt = 0.0 if cfl_mode else 0.02
        ba = torch.empty(3 * n_send, dtype=tdt, device="cuda")
        bb = torch.empty(3 * n_send, dtype=tdt, device="cuda")
        side = torch.cuda.Stream()
        ev = torch.cuda.Event()
        for step in range(5):
            torch.cuda.synchronize()
            a.step(1, dt)
            a.pack_ghosts(ba)
            b.step_overlap(bb, dt, event=ev)
            with torch.cuda.stream(side):          # the caller's "exchange"
                side.wait_event(ev)
                xb = bb.clone()
            a.sync()
            b.sync()
            side.synchronize()
            sa, sb = a.read_state(), b.read_state()
            for f in range(3):
                assert np.array_equal(sa[f], sb[f]), (name, prec, block, cfl_mode, step, f)
            pa, pb, px = ba.cpu().numpy(), bb.cpu().numpy(), xb.cpu().numpy()
            assert np.array_equal(pa, pb) and np.array_equal(pa, px), (name, step)
            assert a.time() == b.time()
        a.close()
        b.close()


@pytest.mark.parametrize("name,r", [("hllc1", 1), ("muscl_minmod_rk2", 4)])
def test_exchange_through_overlapped_steps(name, r):
    """Five sub-domains, k = 4 layers, an exchange after every step (as the
    benchmark's sub-domain does), each step overlapped with its pack."""
    import torch
    swe, prepare_scenario = lib()
    sc = wavy_scenario()
    g, M, par, prg = make_pair(sc, name, precision=0)
    dt = 0.5 * M.dt(par, sc.h[prg.sub.l2g], sc.hu[prg.sub.l2g], sc.hv[prg.sub.l2g])
    k, P, steps = 4, 5, 6
    g.step(steps, dt)
    gst = g.read_state()
    ref = [np.empty_like(gst[0]) for _ in range(3)]
    for f in range(3):
        ref[f][prg.sub.l2g] = gst[f]
    preps = [prepare_scenario(sc, P=P, p=q, k=k, nbr_global=prg.nbr_global) for q in range(P)]
    subs = [make_pair(sc, name, precision=0, prepared=pr)[0] for pr in preps]
    bufs = [torch.empty(3 * max(1, pr.sub.send_idx.size), dtype=torch.float32, device="cuda")
            for pr in preps]
    for _ in range(steps):
        torch.cuda.synchronize()
        for s, bf in zip(subs, bufs):
            s.step_overlap(bf, dt)
        for s in subs:
            s.sync()
        packed = [bf[:3 * pr.sub.send_idx.size].view(3, -1) for bf, pr in zip(bufs, preps)]
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


def test_overlap_rejects_missing_buffer_and_works_without_ghosts():
    import torch
    swe, prepare_scenario = lib()
    sc = wavy_scenario()
    pr = prepare_scenario(sc, P=3, p=1, k=2)
    s, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=0, prepared=pr)
    with pytest.raises(ValueError):
        s.step_overlap(torch.empty(3, dtype=torch.float32, device="cuda"), 0.01)
    g, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=0)        # no send cells
    h, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=0)
    ev = torch.cuda.Event()
    for _ in range(3):
        g.step_overlap(torch.empty(1, dtype=torch.float32, device="cuda"), 0.01, event=ev)
        h.step(1, 0.01)
    ev.synchronize()
    for x, y in zip(g.read_state(), h.read_state()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("pis", [0, 1])
def test_overlap_steps_with_learned_phi_every(pis):
    """The learned limiter with the network every third step: overlapped
    steps evaluate phi on the same steps as plain ones (the step index since
    set_state), so seven overlapped steps give bitwise the state and send
    buffer of seven plain steps, each followed by a pack."""
    import torch
    from oracle import oracle as O
    swe, prepare_scenario = lib()
    sc = wavy_scenario()
    w = np.random.default_rng(5).normal(0.0, 0.3, O.MLP_NPAR).astype(np.float32)
    pr = prepare_scenario(sc, P=3, p=1, k=4)
    kw = dict(precision=0, prepared=pr, limiter=3, phi_every=3, phi_in_stage=pis)
    a, _, _, _ = make_pair(sc, "muscl_minmod_rk2", **kw)
    b, _, _, _ = make_pair(sc, "muscl_minmod_rk2", **kw)
    c, _, _, _ = make_pair(sc, "muscl_minmod_rk2", **dict(kw, phi_every=1))
    for s in (a, b, c):
        s.limiter_set_weights(w)
    n_send, _ = a.ghost_sizes()
    ba = torch.empty(3 * n_send, dtype=torch.float32, device="cuda")
    bb = torch.empty_like(ba)
    for _ in range(7):
        a.step(1, 0.02)
        a.pack_ghosts(ba)
        b.step_overlap(bb, 0.02)
        c.step(1, 0.02)
    a.sync()
    b.sync()
    sa, sb = a.read_state(), b.read_state()
    assert all(np.array_equal(x, y) for x, y in zip(sa, sb))
    assert np.array_equal(ba.cpu().numpy(), bb.cpu().numpy())
    # the schedule is in effect: every-step evaluation gives another state
    assert not np.array_equal(c.read_state()[1], sa[1])
    for s in (a, b, c):
        s.close()
