"""Pins of the oracle's learned-limiter network (FP64): analytic gradients
against central finite differences, output range, the sigmoid's fixed
points, and the limiter's reductions inside a MUSCL step (phi = 0 is the
zero-slope scheme bitwise; a NaN network falls back to minmod)."""
import numpy as np
import pytest

from oracle import oracle as O
from swe_inputs import river_channel


def random_params(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, O.MLP_NPAR)


def random_batch(n=40, seed=1):
    """Central slopes s with backward / forward slopes sb, sf around them:
    same signs with bounds both above and below |phi s| (the clip passes or
    binds), and a few of opposite signs (the clip gives zero)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.5, 1.5, (n, O.MLP_IN))
    q = rng.normal(size=(n, 4))
    s = rng.normal(size=(n, 4))
    sb = s * rng.uniform(0.1, 1.5, (n, 4))
    sf = s * rng.uniform(0.1, 1.5, (n, 4))
    sf[::7] *= -1.0
    d = rng.uniform(0.5, 2.0, n)
    t = q + rng.normal(scale=0.3, size=(n, 4))
    return x, q, s, sb, sf, d, t


def test_gradient_matches_finite_differences():
    w = random_params()
    x, q, s, sb, sf, d, t = random_batch()
    wv = np.array([1.0, 0.5, 2.0, 0.7])
    loss, g = O.mlp_loss_grad(w, x, q, s, sb, sf, d, t, wv)
    h = 1e-6
    fd = np.empty_like(w)
    for i in range(w.size):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd[i] = (O.mlp_loss_grad(wp, x, q, s, sb, sf, d, t, wv)[0]
                 - O.mlp_loss_grad(wm, x, q, s, sb, sf, d, t, wv)[0]) / (2 * h)
    scale = np.abs(fd).max()
    assert np.abs(g - fd).max() <= 1e-6 * scale
    assert loss > 0
    # the clip both passes and binds in this batch: the gradient differs from
    # the unclipped objective's (sb, sf far outside the bound)
    big = 1e6 * np.sign(s)
    _, g_free = O.mlp_loss_grad(w, x, q, s, big, big, d, t, wv)
    assert np.abs(g - g_free).max() > 1e-3 * scale


def test_training_loss_is_the_misfit_of_the_solver_reconstruction():
    """With d = d_mid and zero targets, the training loss of a network whose
    output is the constant phi0 equals the weighted mean square of the
    interface values that the oracle's learned MUSCL step reconstructs with
    phi0 (M.interfaces, an independent path through the solver): the
    objective measures the clipped values the solver evaluates."""
    sc = _river()
    M, h, hu, hv = _flowing(sc)
    w = np.zeros(O.MLP_NPAR)
    w[-1] = np.log(0.7 / 0.3)            # output bias: phi = 0.7 everywhere
    p = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2, limiter=O.LEARNED, mlp=w)
    inp, phi = O.limiter_inputs(M, p, h, hu, hv)
    rh, rb, run, rut, _ = M.interfaces(p, h, hu, hv)
    got = np.stack([rh, rh + rb, run, rut], -1)
    elig = (inp[..., 23] == 1.0) & (rh >= 0)
    E = inp[elig]
    assert E.shape[0] > 100 and np.allclose(phi[elig], 0.7)
    wv = np.array([1.0, 0.5, 2.0, 0.7])
    loss, _ = O.mlp_loss_grad(w, E[:, :14], E[:, 14:18], E[:, 18:22], E[:, 24:28], E[:, 28:32],
                              E[:, 22], np.zeros((E.shape[0], 4)), wv)
    direct = float(((got[elig] ** 2) * wv).sum(1).mean())
    assert loss == pytest.approx(direct, rel=1e-12)


def test_dumped_slopes_give_the_minmod_reconstruction():
    """The backward and forward slopes of the limiter-input dump: q + d_mid
    minmod(sb, sf) is the oracle's own minmod MUSCL reconstruction."""
    sc = _river()
    M, h, hu, hv = _flowing(sc)
    p = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2, limiter=O.MINMOD)
    inp, _ = O.limiter_inputs(M, p, h, hu, hv)
    mh, mb, mun, mut, _ = M.interfaces(p, h, hu, hv)
    elig = (inp[..., 23] == 1.0) & (mh >= 0)
    q, dm, sb, sf = inp[..., 14:18], inp[..., 22:23], inp[..., 24:28], inp[..., 28:32]
    mm = np.where(sb * sf > 0, np.sign(sf) * np.minimum(np.abs(sb), np.abs(sf)), 0.0)
    rec = q + dm * mm
    scale = np.abs(q).max(axis=(0, 1)) + 1.0
    assert (mm[elig] != 0).any()
    for i, got in enumerate((mh, mh + mb, mun, mut)):
        np.testing.assert_allclose(got[elig], rec[..., i][elig], rtol=0, atol=1e-12 * scale[i])


def test_output_range_and_fixed_points():
    w = random_params(2, scale=2.0)
    x, *_ = random_batch(200, 3)
    phi = O.mlp_forward(w, x)
    assert np.all((phi >= 0) & (phi <= 1))
    w0 = np.zeros(O.MLP_NPAR)
    assert np.all(O.mlp_forward(w0, x) == 0.5)
    w0[-1] = -1e3            # output bias: sigmoid saturates at 0
    assert np.all(O.mlp_forward(w0, x) == 0.0)
    # bf16 inputs move phi by at most a few bf16 ulps of the activations
    pb = O.mlp_forward(w, x, bf16_inputs=True)
    assert np.abs(pb - phi).max() < 3e-2


def _river():
    return river_channel(Lx=2000.0, Ly=400.0, nx=40, ny=8, seed=4)


def _flowing(sc):
    M, _ = O.global_mesh(sc)
    p = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2)
    h, hu, hv, t, _ = M.run(p, sc.h, sc.hu, sc.hv, 150)
    return M, h, hu, hv


def test_phi_zero_is_zero_slope_bitwise():
    sc = _river()
    M, h, hu, hv = _flowing(sc)
    w = np.zeros(O.MLP_NPAR)
    w[-1] = -1e3
    pl = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2, limiter=O.LEARNED, mlp=w)
    pz = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2, limiter=O.ZEROSLOPE)
    a = M.run(pl, h, hu, hv, 20)
    b = M.run(pz, h, hu, hv, 20)
    for i in range(3):
        assert np.array_equal(a[i], b[i])


def test_nan_network_falls_back_to_minmod():
    sc = _river()
    M, h, hu, hv = _flowing(sc)
    w = np.full(O.MLP_NPAR, np.nan)
    pl = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2, limiter=O.LEARNED, mlp=w)
    pm = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2, limiter=O.MINMOD)
    a = M.run(pl, h, hu, hv, 20)
    b = M.run(pm, h, hu, hv, 20)
    for i in range(3):
        assert np.array_equal(a[i], b[i])


def test_limiter_inputs_consistent_with_reconstruction():
    """phi = 1 is the monotonized central limiter on the central slope s of
    the limiter-input dump: q + d_mid * clip(s) with clip(s) = 0 where the
    backward and forward slopes disagree in sign, else sign(sf) *
    min(|s|, 2 min(|sb|, |sf|)).  The backward/forward information comes
    from the oracle's minmod reconstruction m = minmod(sb, sf) (|m| is the
    smaller slope, m = 0 at an extremum), so this checks the learned path
    against two independent pieces of the oracle and the textbook MC form."""
    sc = _river()
    M, h, hu, hv = _flowing(sc)
    w = np.zeros(O.MLP_NPAR)
    w[-1] = 1e3               # phi = 1
    p = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2, limiter=O.LEARNED, mlp=w)
    inp, phi = O.limiter_inputs(M, p, h, hu, hv)
    rh, rb, run, rut, sec = M.interfaces(p, h, hu, hv)
    pm = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2, limiter=O.MINMOD)
    mh, mb, mun, mut, _ = M.interfaces(pm, h, hu, hv)
    elig = inp[..., 23] == 1.0
    assert elig.sum() > 100
    assert np.all(phi[elig] == 1.0) and np.all(np.isnan(phi[~elig]))
    q, s, d = inp[..., 14:18], inp[..., 18:22], inp[..., 22:23]
    mm = (np.stack([mh, mh + mb, mun, mut], -1) - q) / d          # minmod slopes
    clip = np.where(mm == 0.0, 0.0, np.sign(mm) * np.minimum(np.abs(s), 2.0 * np.abs(mm)))
    rec = q + d * clip
    ok = elig & (rec[..., 0] >= 0) & (mh >= 0)
    assert (np.abs(clip) < np.abs(s))[ok].any()       # the bound is active somewhere
    scale = np.abs(q).max(axis=(0, 1)) + 1.0
    for i, got in enumerate((rh, rb + rh, run, rut)):
        np.testing.assert_allclose(got[ok], rec[..., i][ok], rtol=0, atol=1e-12 * scale[i])
    assert np.all(np.abs(inp[..., :12][elig][:, 0::3]) <= 1.0)


def test_training_target_lies_halfway_to_the_edge():
    """The target of a coarse half-edge is the mean of the two red-refinement
    children touching the edge; their mean centroid is exactly halfway from
    the coarse centroid to the edge midpoint, the distance the training
    records store (d_mid / 2)."""
    from swe_inputs.mesh import grid_mesh, refine_red
    m = grid_mesh(30.0, 20.0, 6, 4, seed=7)
    f = refine_red(m)
    cen = m.xy[m.tri].mean(1)
    fcen = f.xy[f.tri].mean(1)
    for e in range(3):
        mid = 0.5 * (m.xy[m.tri[:, e]] + m.xy[m.tri[:, (e + 1) % 3]])
        ch = 4 * np.arange(m.n_cells)
        tgt = 0.5 * (fcen[ch + e] + fcen[ch + (e + 1) % 3])
        np.testing.assert_allclose(tgt, cen + 0.5 * (mid - cen), rtol=0, atol=1e-12)
