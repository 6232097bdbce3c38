"""Pins of the oracle's Riemann solvers and limiters (Sec. 6.2) by special
cases that reduce to textbook formulas written out here independently."""
import math

import numpy as np
import pytest

from oracle import oracle as O

G = 9.81
P = O.Params()


def phys_flux(U):
    """G(U) of eq. eqswefinal in the normal frame, U = (h, q_n, q_t)."""
    h, qn, qt = U
    u, v = qn / h, qt / h
    return np.array([qn, qn * u + 0.5 * G * h * h, qn * v])


STATES = [(1.0, 0.3, -0.2), (0.5, -0.4, 0.1), (2.3, 1.7, 0.9), (0.05, 0.01, -0.02),
          (3.0, 30.0, 1.0), (1.2, -9.0, 0.4)]


@pytest.mark.parametrize("U", STATES)
@pytest.mark.parametrize("scheme", [O.HLLC1, O.WAF])
def test_consistency_equal_states(U, scheme):
    """U_L = U_R gives the physical flux (consistency of every scheme)."""
    F = O.riemann(P, scheme, U, U, 0.05, [1, 1, 1, 1, 0, 0, 0, 0])
    np.testing.assert_allclose(F, phys_flux(U), rtol=1e-13, atol=1e-13)


def test_supersonic_upwinding():
    UL, UR = (1.0, 5.0, 0.5), (0.8, 4.0, -0.3)     # u > sqrt(g h) on both sides
    np.testing.assert_allclose(O.riemann(P, O.HLLC1, UL, UR), phys_flux(UL), rtol=1e-14)
    UL, UR = (1.0, -5.0, 0.5), (0.8, -4.5, -0.3)
    np.testing.assert_allclose(O.riemann(P, O.HLLC1, UL, UR), phys_flux(UR), rtol=1e-14)


def _hll_star(UL, UR, SL, SR):
    GL, GR = phys_flux(UL), phys_flux(UR)
    return (SR * GL - SL * GR + SR * SL * (np.array(UR) - np.array(UL))) / (SR - SL)


def test_hllc_star_region_and_contact():
    """Subsonic case: components 1, 2 are the HLL star flux with the
    two-rarefaction estimate; component 3 is upwinded by the sign of S*."""
    hL, uL, vL, hR, uR, vR = 1.0, -0.3, 0.5, 0.9, 0.5, -0.3
    aL, aR = math.sqrt(G * hL), math.sqrt(G * hR)
    h0 = 0.5 * (hL + hR) - 0.25 * (uR - uL) * (hL + hR) / (aL + aR)
    assert h0 <= min(hL, hR)          # rarefaction branch
    hs = (0.5 * (aL + aR) + 0.25 * (uL - uR)) ** 2 / G
    pL = math.sqrt(0.5 * (hs + hL) * hs / hL ** 2) if hs > hL else 1.0
    pR = math.sqrt(0.5 * (hs + hR) * hs / hR ** 2) if hs > hR else 1.0
    SL, SR = uL - aL * pL, uR + aR * pR
    Ss = (SL * hR * (uR - SR) - SR * hL * (uL - SL)) / (hR * (uR - SR) - hL * (uL - SL))
    UL, UR = (hL, hL * uL, hL * vL), (hR, hR * uR, hR * vR)
    F = O.riemann(P, O.HLLC1, UL, UR)
    Fs = _hll_star(UL, UR, SL, SR)
    np.testing.assert_allclose(F[:2], Fs[:2], rtol=1e-13)
    assert abs(Ss) > 1e-3
    # S* > 0: left tangential velocity, S* < 0: right one
    assert F[2] == pytest.approx(F[0] * (vL if Ss > 0 else vR), rel=1e-13)
    # mirrored problem (x -> -x): the contact moves the other way, the other
    # side's v is taken
    F2 = O.riemann(P, O.HLLC1, (hR, -hR * uR, hR * vR), (hL, -hL * uL, hL * vL))
    assert F2[2] == pytest.approx(F2[0] * (vL if Ss > 0 else vR), rel=1e-13)
    assert F2[0] == pytest.approx(-F[0], rel=1e-13)


def test_shock_branch_estimate():
    hL, uL, hR, uR = 1.0, 2.0, 1.0, -2.0          # colliding streams: two shocks
    aL = aR = math.sqrt(G)
    h0 = 0.5 * (hL + hR) - 0.25 * (uR - uL) * (hL + hR) / (aL + aR)
    assert h0 > min(hL, hR)
    gL = math.sqrt(0.5 * G * (h0 + hL) / (h0 * hL))
    gR = math.sqrt(0.5 * G * (h0 + hR) / (h0 * hR))
    hs = (hL * gL + hR * gR + uL - uR) / (gL + gR)
    p = math.sqrt(0.5 * (hs + hL) * hs / hL ** 2)
    SL, SR = uL - aL * p, uR + aR * p
    UL, UR = (hL, hL * uL, 0.0), (hR, hR * uR, 0.0)
    F = O.riemann(P, O.HLLC1, UL, UR)
    np.testing.assert_allclose(F[:2], _hll_star(UL, UR, SL, SR)[:2], rtol=1e-13)
    assert abs(F[0]) < 1e-14                        # symmetric collision: no mass flux


def test_dry_bed_speeds():
    """Dry right state: S_L = u_L - a_L, S_R = u_L + 2 a_L (Toro)."""
    hL, uL = 1.3, 0.4
    aL = math.sqrt(G * hL)
    SL, SR = uL - aL, uL + 2 * aL
    UL, UR = (hL, hL * uL, 0.2 * hL), (0.0, 0.0, 0.0)
    F = O.riemann(P, O.HLLC1, UL, UR)
    Fs = _hll_star(UL, (1e-300, 0.0, 0.0), SL, SR)
    np.testing.assert_allclose(F[:2], Fs[:2], rtol=1e-12)
    # both dry: no flux
    assert np.all(O.riemann(P, O.HLLC1, (0.0, 0, 0), (1e-9, 0, 0)) == 0)
    # dry left, mirrored
    Fm = O.riemann(P, O.HLLC1, UR, (hL, -hL * uL, 0.2 * hL))
    assert Fm[0] == pytest.approx(-F[0], rel=1e-13)


def test_waf_godunov_limit_is_hllc():
    """A = 1 for every wave turns WAF into HLLC (bitwise: shared wave fan)."""
    p = O.Params(waf_limiter=O.WAF_GODUNOV)
    rng = np.random.default_rng(0)
    for _ in range(200):
        hL, hR = rng.uniform(0.05, 3, 2)
        uL, uR, vL, vR = rng.uniform(-3, 3, 4)
        UL, UR = (hL, hL * uL, hL * vL), (hR, hR * uR, hR * vR)
        Fw = O.riemann(p, O.WAF, UL, UR, rng.uniform(0.01, 0.2), rng.normal(size=8))
        Fh = O.riemann(p, O.HLLC1, UL, UR)
        assert np.array_equal(Fw[:2], Fh[:2])
        if not np.isclose(Fw[0], 0.0):
            # third component: same upwinding unless S* == 0 exactly
            assert Fw[2] == Fh[2]


def test_waf_unlimited_small_courant_is_central():
    """Unlimited weights (A = |c|) with dt/dx -> 0: w_L = w_R = 1/2, w_LR = 0."""
    p = O.Params(waf_limiter=O.WAF_UNLIMITED)
    UL, UR = (1.0, 0.3, 0.1), (0.7, -0.2, 0.4)
    F = O.riemann(p, O.WAF, UL, UR, 0.0)
    avg = 0.5 * (phys_flux(UL) + phys_flux(UR))
    np.testing.assert_allclose(F[:2], avg[:2], rtol=1e-14)
    assert F[2] == pytest.approx(0.5 * (UL[2] / UL[0] + UR[2] / UR[0]) * F[0], rel=1e-14)


def test_waf_superbee_reduces():
    """Superbee WAF: r <= 0 gives A = 1 (HLLC); 1/2 < r <= 1 gives A = |c|
    (the unlimited scheme)."""
    UL, UR = (1.0, 0.3, 0.1), (0.7, -0.2, 0.4)
    dtdx = 0.1
    # r = (qL - qLu)/(qR - qL) with q = given values; choose r = -1 for both sides
    neg = [1.0, 0.5, 0.5, 1.0, 0.1, 0.5, 0.9, 0.1]          # r_L=-1, r_R=-1, r*=-1... (h then v)
    F = O.riemann(O.Params(), O.WAF, UL, UR, dtdx, neg)
    Fh = O.riemann(O.Params(), O.HLLC1, UL, UR)
    np.testing.assert_allclose(F, Fh, rtol=1e-14)
    # r = 0.75 on every wave: upwind change 0.75 x local change on both sides
    qL, qR = 1.0, 0.5
    d = qR - qL
    mid = [qL, qR, qL - 0.75 * d, qR + 0.75 * d, 0.1, 0.5, 0.1 - 0.75 * 0.4, 0.5 + 0.75 * 0.4]
    F = O.riemann(O.Params(), O.WAF, UL, UR, dtdx, mid)
    Fu = O.riemann(O.Params(waf_limiter=O.WAF_UNLIMITED), O.WAF, UL, UR, dtdx, mid)
    np.testing.assert_allclose(F, Fu, rtol=1e-13)


def phi_superbee(r):
    return max(0.0, min(2 * r, 1.0), min(r, 2.0))


@pytest.mark.parametrize("c", [0.0, 0.3, -0.7, 1.0])
def test_superbee_A(c):
    for r in np.linspace(-1, 4, 101):
        assert O.superbee_A(r, c) == pytest.approx(1 - (1 - abs(c)) * phi_superbee(r), abs=1e-14)
    for r0 in (0.5, 1.0, 2.0):     # continuity at the breakpoints
        assert O.superbee_A(r0 - 1e-12, c) == pytest.approx(O.superbee_A(r0 + 1e-12, c), abs=1e-10)


def minmod(a, b):
    return 0.0 if a * b <= 0 else math.copysign(min(abs(a), abs(b)), a)


def superbee(a, b):
    if a * b <= 0:
        return 0.0
    return math.copysign(max(min(2 * abs(a), abs(b)), min(abs(a), 2 * abs(b))), a)


def test_beta_limiters_are_minbee_and_superbee():
    rng = np.random.default_rng(1)
    for a, b in rng.normal(size=(2000, 2)):
        assert O.limiter(O.MINMOD, a, b) == minmod(a, b)
        assert O.limiter(O.SUPERBEE, a, b) == pytest.approx(superbee(a, b), abs=0)
        va = O.limiter(O.VANALBADA, a, b)
        assert va == O.limiter(O.VANALBADA, b, a)
        if a * b > 0:
            assert min(a, b) - 1e-15 <= va <= max(a, b) + 1e-15
    assert O.limiter(O.MINMOD, 1.0, 0.0) == 0.0
    assert O.limiter(O.SUPERBEE, 0.0, 1.0) == 0.0


def test_bf16_rounding():
    assert O.bf16(1.0) == 1.0
    assert O.bf16(1.0 + 2 ** -8) == 1.0              # tie -> even
    assert O.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    assert O.bf16(-3.14159) == pytest.approx(-3.140625)


def van_albada_ratio_form(a, b):
    """Textbook van Albada slope limiter in ratio form: a * xi(r) with
    r = b / a and xi(r) = r (1 + r) / (1 + r^2) for r > 0, else 0."""
    if a == 0.0:
        return 0.0
    r = b / a
    return a * r * (1.0 + r) / (1.0 + r * r) if r > 0.0 else 0.0


def test_van_albada_values():
    """Values that tell van Albada apart from the other symmetric limiters
    bounded by the two slopes: at slopes (1, 3) van Albada gives 1.2, van
    Leer's 2ab/(a+b) 1.5, the monotonized central limiter 2, minmod 1; for one
    slope much larger than the other van Albada tends to the smaller one
    (van Leer to twice it)."""
    assert O.limiter(O.VANALBADA, 1.0, 3.0) == pytest.approx(1.2, rel=1e-15)
    assert O.limiter(O.VANALBADA, 3.0, 1.0) == pytest.approx(1.2, rel=1e-15)
    assert O.limiter(O.VANALBADA, -2.0, -6.0) == pytest.approx(-2.4, rel=1e-15)
    assert O.limiter(O.VANALBADA, 2.0, 2.0) == pytest.approx(2.0, rel=1e-15)
    assert O.limiter(O.VANALBADA, 1.0, 1e6) == pytest.approx(1.0, rel=2e-6)
    assert O.limiter(O.VANALBADA, 1.0, -3.0) == 0.0
    rng = np.random.default_rng(7)
    for a, b in rng.normal(size=(2000, 2)) * np.exp(rng.normal(size=(2000, 2))):
        assert O.limiter(O.VANALBADA, a, b) == pytest.approx(van_albada_ratio_form(a, b),
                                                             rel=1e-13, abs=1e-300)

