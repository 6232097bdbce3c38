"""Learned limiter on the GPU against the FP64 oracle: matrix-core (BF16)
inference of phi, MUSCL steps with the learned limiter, training records
built from a refined-mesh run, and the trainer's gradient.

Tolerances: BF16 operands carry 8 significant bits, so phi may differ from
the oracle's by a few BF16 ulps of the activations (the oracle rounds the
same layer inputs to BF16; the remaining difference is FP32 accumulation and
BF16 ties decided differently): max 2e-2, mean 2e-3.  The trainer runs in
FP32: per-tensor gradient error <= 1e-2 relative, cosine >= 0.999.
"""
import numpy as np
import pytest

from gpu_util import make_pair, lib
from oracle import oracle as O
from swe_inputs import river_channel, refine_scenario

pytestmark = pytest.mark.gpu


def swe_mod():
    return lib()[0]


def bf16_round(a):
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def params(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    w = rng.normal(0.0, scale, O.MLP_NPAR).astype(np.float32)
    return w


def flowing_state(sc, steps=150):
    M, _ = O.global_mesh(sc)
    p = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2)
    h, hu, hv, t, _ = M.run(p, sc.h, sc.hu, sc.hv, steps)
    return h, hu, hv


def small_river():
    return river_channel(Lx=2000.0, Ly=400.0, nx=80, ny=16, seed=6)


@pytest.mark.parametrize("prec", [0, 1])
def test_mfma_phi_matches_oracle(prec):
    import torch
    sc = small_river()
    h, hu, hv = flowing_state(sc)
    sc.h, sc.hu, sc.hv = h, hu, hv
    w = params()
    s, M, par, pr = make_pair(sc, "muscl_minmod_rk2", precision=prec, limiter=3)
    s.limiter_set_weights(w)
    phi = torch.empty(3 * pr.sub.n_total, dtype=torch.float32, device="cuda")
    s.limiter_phi(phi)
    g = phi.cpu().numpy().reshape(-1, 3)
    l2g = pr.sub.l2g
    dt = np.float32 if prec == 0 else np.float64
    par.mlp = bf16_round(w)
    par.mlp_bf16 = 1
    inp, ref = O.limiter_inputs(M, par, *(a[l2g].astype(dt).astype(np.float64) for a in (h, hu, hv)))
    elig = inp[..., 23] == 1.0
    assert elig.sum() > 1000
    d = np.abs(g - ref)
    print("phi max/mean diff", d[elig].max(), d[elig].mean())
    assert np.all(np.isnan(g[~elig]))
    assert d[elig].max() <= 2e-2 and d[elig].mean() <= 2e-3


@pytest.mark.parametrize("prec,tol", [(1, 1e-5), (0, 1e-3)])
def test_learned_limiter_steps(prec, tol):
    sc = small_river()
    h, hu, hv = flowing_state(sc)
    sc.h, sc.hu, sc.hv = h, hu, hv
    w = params(1)
    s, M, par, pr = make_pair(sc, "muscl_minmod_rk2", precision=prec, limiter=3)
    s.limiter_set_weights(w)
    l2g = pr.sub.l2g
    par.limiter = O.LEARNED
    par.mlp = bf16_round(w)
    par.mlp_bf16 = 1
    dt = M.dt(par, h[l2g], hu[l2g], hv[l2g])
    s.step(50, dt)
    gst = s.read_state()
    r = M.run(par, h[l2g], hu[l2g], hv[l2g], 50, dt_fixed=dt)
    errs = [np.abs(a - b).max() / np.abs(b).max() for a, b in zip(gst, r[:3])]
    print("learned limiter", prec, errs)
    assert max(errs) <= tol


@pytest.mark.parametrize("cell", [0, 1])
@pytest.mark.parametrize("prec,tol", [(1, 1e-5), (0, 1e-3)])
@pytest.mark.parametrize("pe", [2, 3, 6])
def test_phi_every_matches_oracle(prec, tol, pe, cell):
    """phi evaluated every pe steps (phi_every) against the oracle on the same
    schedule, 50 steps (graph chunks of six steps and two single steps), with
    the tiled and the one-thread-per-cell stage kernels; the every-step oracle
    run differs from both by more than the tolerance, so the schedule is what
    is being compared."""
    sc = small_river()
    h, hu, hv = flowing_state(sc)
    sc.h, sc.hu, sc.hv = h, hu, hv
    w = params(1)
    s, M, par, pr = make_pair(sc, "muscl_minmod_rk2", precision=prec, limiter=3, phi_every=pe,
                              cell_kernel=cell)
    s.limiter_set_weights(w)
    l2g = pr.sub.l2g
    par.limiter = O.LEARNED
    par.mlp = bf16_round(w)
    par.mlp_bf16 = 1
    dt = M.dt(par, h[l2g], hu[l2g], hv[l2g])
    s.step(50, dt)
    gst = s.read_state()
    par.phi_every = pe
    r = M.run(par, h[l2g], hu[l2g], hv[l2g], 50, dt_fixed=dt)
    par.phi_every = 1
    r1 = M.run(par, h[l2g], hu[l2g], hv[l2g], 50, dt_fixed=dt)
    errs = [np.abs(a - b).max() / np.abs(b).max() for a, b in zip(gst, r[:3])]
    sep = [np.abs(a - b).max() / np.abs(b).max() for a, b in zip(r1[:3], r[:3])]
    print("phi every", pe, prec, cell, errs, "every step vs schedule", sep)
    assert max(errs) <= tol
    assert max(sep) > 2 * tol


@pytest.mark.parametrize("pis", [0, 1])
def test_phi_every_launch_paths_agree(pis):
    """With phi_every = 3 the schedule follows the step index since
    set_state on every launch path: a graph-replayed run, single steps, and a
    run started off the graph's alignment give bitwise the same state; new
    weights make the next step evaluate phi (equal to a fresh run with those
    weights from the same state), and reading phi with swe_limiter_phi between
    evaluations leaves the run unchanged."""
    import torch
    sc = small_river()
    h, hu, hv = flowing_state(sc)
    sc.h, sc.hu, sc.hv = h, hu, hv
    w1, w2 = params(1), params(2)
    swe, prepare_scenario = lib()
    pr = prepare_scenario(sc)
    l2g = pr.sub.l2g
    M, _ = O.global_mesh(sc)
    dt = 0.5 * M.dt(O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2), h, hu, hv)

    def solver(w, state=None, t=0.0):
        s, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=0, prepared=pr, limiter=3,
                               phi_every=3, phi_in_stage=pis)
        s.limiter_set_weights(w)
        if state is not None:
            s.set_state(*state, t=t)
        return s

    a = solver(w1)
    a.step(24, dt)                       # four graph chunks
    b = solver(w1)
    for _ in range(24):
        b.step(1, dt)                    # single launches
    c = solver(w1)
    c.step(1, dt)
    c.step(2, dt)
    c.step(21, dt)                       # singles, then chunks from step 6 on
    d = solver(w1)
    d.step(4, dt)
    buf = torch.empty(3 * pr.sub.n_total, dtype=torch.float32, device="cuda")
    d.limiter_phi(buf)                   # between evaluations (steps 3 and 6)
    d.step(20, dt)
    ref = a.read_state()
    for s_ in (b, c, d):
        assert all(np.array_equal(x, y) for x, y in zip(s_.read_state(), ref))
    # new weights at step 4 (between evaluations): evaluated at once
    e = solver(w1)
    e.step(4, dt)
    mid, t_mid = e.read_state(), e.time()
    e.limiter_set_weights(w2)
    e.step(2, dt)
    f = solver(w2, state=mid, t=t_mid)
    f.step(2, dt)
    assert all(np.array_equal(x, y) for x, y in zip(e.read_state(), f.read_state()))
    g_ = solver(w1, state=mid, t=t_mid)
    g_.step(2, dt)
    assert not np.array_equal(g_.read_state()[1], f.read_state()[1])


@pytest.mark.parametrize("prec,integ,block,P", [(0, 1, 256, 1), (1, 1, 256, 1), (0, 0, 256, 1),
                                                 (0, 1, 64, 1), (0, 1, 512, 1), (0, 1, 256, 4)])
def test_network_in_stage_equals_separate_kernel(prec, integ, block, P):
    """phi evaluated by the stand-alone network kernel ahead of each step (the
    default) and inside the tiled kernel's first stage (the network on the
    stage's own stencil, the far side of a tile-crossing edge evaluated where
    it is needed) give bitwise the same states: RK2 and Euler, FP32 and
    FP64, every tile size, and a sub-domain with ghost layers."""
    sc = small_river()
    h, hu, hv = flowing_state(sc)
    sc.h, sc.hu, sc.hv = h, hu, hv
    w = params(1)
    swe, prepare_scenario = lib()
    pr = prepare_scenario(sc, P=P, p=1 if P > 1 else 0, k=4 if P > 1 else 0)
    dt = None
    states = []
    for pis in (0, 1):
        s, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=prec, prepared=pr, limiter=3,
                               integrator=integ, block=block, phi_in_stage=pis)
        s.limiter_set_weights(w)
        name, launches = s.step_kernel()
        assert launches == (2 if integ else 1) + 1 - pis, (name, launches)
        if dt is None:
            l2g = pr.sub.l2g
            M, _ = O.global_mesh(sc)
            par = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2 if integ else O.EULER)
            dt = 0.5 * M.dt(par, h, hu, hv)
        s.step(40, dt)
        states.append(s.read_state())
    for a, b in zip(*states):
        assert np.array_equal(a, b)
    assert np.all(np.isfinite(states[0][0]))


def fine_pair(sc, steps=100):
    """Coarse and red-refined scenario, the fine one run by the oracle and
    loaded into a solver; returns solvers, prepared meshes, the children map
    (coarse local -> fine local) and the fine state on the host."""
    import torch
    swe, prepare_scenario = lib()
    fs = refine_scenario(sc)
    fine, Mf, parf, prf = make_pair(fs, "muscl_minmod_rk2", precision=0)
    # the fine solution comes from the oracle (rounded to the solver's FP32),
    # so every input of the oracle calls below is the oracle's own
    lf = prf.sub.l2g
    rf = Mf.run(parf, fs.h[lf], fs.hu[lf], fs.hv[lf], steps)
    fine_host = tuple(x.astype(np.float32) for x in rf[:3])
    fine.set_state(*fine_host)
    coarse, Mc, parc, prc = make_pair(sc, "muscl_minmod_rk2", precision=0)
    g2l = np.empty(fs.n_cells, np.int64)
    g2l[prf.sub.l2g] = np.arange(prf.sub.n_total)
    gid = prc.sub.l2g
    ch = np.stack([g2l[4 * gid + k] for k in range(4)], 1).astype(np.int32)
    children = torch.from_numpy(ch.ravel().copy()).cuda()
    return coarse, fine, prc, prf, ch, children, fs, Mc, parc, fine_host


def test_pairs_records():
    import torch
    sc = small_river()
    coarse, fine, prc, prf, ch, children, fs, Mc, parc, fine_host = fine_pair(sc)
    n = prc.sub.n_total
    rec = torch.zeros(3 * n * swe_mod().PAIR_RECORD, dtype=torch.float32, device="cuda")
    coarse.limiter_pairs(fine, children, rec)
    R = rec.cpu().numpy().reshape(n, 3, swe_mod().PAIR_RECORD)
    fh, fhu, fhv = fine_host
    ch_h, ch_hu, ch_hv = fh[ch].astype(np.float64), fhu[ch].astype(np.float64), fhv[ch].astype(np.float64)
    # the restriction (mean of the four children) is the coarse state now
    h, hu, hv = coarse.read_state()
    np.testing.assert_allclose(h, ch_h.mean(1), rtol=1e-6, atol=1e-6)
    # the oracle's features of the same restriction, formed on the host from
    # the oracle's fine state
    inp, _ = O.limiter_inputs(Mc, parc, ch_h.mean(1), ch_hu.mean(1), ch_hv.mean(1))
    elig = inp[..., 23] == 1.0
    ok = R[..., 27] == 1.0
    assert ok.sum() > 1000 and np.all(elig[ok])
    np.testing.assert_allclose(R[..., 14:18][ok], inp[..., 14:18][ok], rtol=1e-4, atol=1e-5)
    np.testing.assert_allclose(R[..., 18:22][ok], inp[..., 18:22][ok], rtol=1e-3, atol=1e-5)
    np.testing.assert_allclose(R[..., 22], 0.5 * inp[..., 22], rtol=1e-6)   # target distance
    # backward and forward slopes (the training objective's TVD bound)
    np.testing.assert_allclose(R[..., 32:36][ok], inp[..., 24:28][ok], rtol=1e-3, atol=1e-5)
    np.testing.assert_allclose(R[..., 36:40][ok], inp[..., 28:32][ok], rtol=1e-3, atol=1e-5)
    assert np.abs(R[..., :14][ok] - inp[..., :14][ok]).max() < 1e-3
    # target depth: mean of the two children touching the edge
    for m in range(3):
        tgt = 0.5 * (ch_h[:, m] + ch_h[:, (m + 1) % 3])
        np.testing.assert_allclose(R[:, m, 23], tgt, rtol=1e-6, atol=1e-6)


def test_trainer_gradient_matches_oracle():
    import torch
    swe, _ = lib()
    sc = small_river()
    coarse, fine, prc, prf, ch, children, *_ = fine_pair(sc)
    n = prc.sub.n_total
    rec = torch.zeros(3 * n * swe.PAIR_RECORD, dtype=torch.float32, device="cuda")
    coarse.limiter_pairs(fine, children, rec)
    R = rec.cpu().numpy().reshape(-1, swe.PAIR_RECORD)
    valid = np.where(R[:, 27] == 1.0)[0].astype(np.int32)
    assert valid.size > 1000
    idx = torch.from_numpy(valid).cuda()
    w = params(3, scale=0.2)
    wv = np.array([1.0, 1.0, 0.5, 0.5], np.float32)
    tr = swe.Trainer(w)
    loss, g = tr.loss_grad(rec, idx, wv)
    V = R[valid].astype(np.float64)
    lo, go = O.mlp_loss_grad(w.astype(np.float64), V[:, :14], V[:, 14:18], V[:, 18:22],
                             V[:, 32:36], V[:, 36:40], V[:, 22], V[:, 23:27], wv.astype(np.float64))
    assert loss == pytest.approx(lo, rel=1e-3)
    sizes = [32 * 14, 32, 32 * 32, 32, 32, 1]
    off = 0
    for sz in sizes:
        a, b = g[off:off + sz].astype(np.float64), go[off:off + sz]
        off += sz
        nb = np.linalg.norm(b)
        if nb == 0:
            continue
        assert np.linalg.norm(a - b) <= 1e-2 * nb
        assert a @ b / (np.linalg.norm(a) * nb) >= 0.999


def test_training_reduces_loss():
    import torch
    swe, _ = lib()
    sc = small_river()
    coarse, fine, prc, prf, ch, children, *_ = fine_pair(sc, steps=200)
    n = prc.sub.n_total
    rec = torch.zeros(3 * n * swe.PAIR_RECORD, dtype=torch.float32, device="cuda")
    coarse.limiter_pairs(fine, children, rec)
    R = rec.view(-1, swe.PAIR_RECORD)
    valid = torch.nonzero(R[:, 27] == 1.0).flatten().to(torch.int32)
    tr = swe.Trainer(params(4, scale=0.1))
    wv = np.array([1.0, 1.0, 1.0, 1.0], np.float32)
    l0 = tr.loss_grad(rec, valid, wv)[0]
    for _ in range(300):
        tr.step(rec, valid, wv, 3e-3)
    l1 = tr.loss_grad(rec, valid, wv)[0]
    print("loss", l0, "->", l1)
    assert l1 < 0.9 * l0
