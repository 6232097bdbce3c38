"""The time-error study of the paper's three schemes on the wet-bed dam
break (Sec. 6.4, the time-error comparison): its exact depth against the
textbook Riemann solution (CPU), and on the GPU the ordering the paper
reports on the two smallest meshes of its ladder."""
import numpy as np
import pytest

import exact_riemann as E


def test_exact_depth_matches_textbook_riemann_solution():
    """The study's own exact depth of the wet-bed dam break (both sides at
    rest) against exact_riemann's general construction, at points in every
    region: the deep state, the rarefaction, the middle state, the shallow
    state."""
    from paper_2307_16758_amd.time_error import stoker_depth
    xi = np.linspace(-5.0, 5.0, 2001)
    ref, _ = E.sample(xi, 1.0, 0.0, 0.5, 0.0)
    got = stoker_depth(xi, 1.0, 0.5)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
    assert got.min() == 0.5 and got.max() == 1.0
    assert np.any((got > 0.5 + 1e-3) & (got < 1.0 - 1e-3))


@pytest.mark.gpu
def test_second_order_schemes_more_accurate():
    """On the 20k and 50k meshes: every scheme's error falls with the mesh,
    WAF and MUSCL (superbee) are more accurate than first-order HLLC on the
    same mesh, and MUSCL more than WAF, as the paper reports."""
    from paper_2307_16758_amd.time_error import LADDER, run
    res = {n: [run(nx, ny, n, t_end=2.0) for nx, ny in LADDER[:2]]
           for n in ("hllc1", "waf", "muscl_superbee")}
    for n, rows in res.items():
        print(n, [(r["cells"], r["l2"], r["gpu_s"]) for r in rows])
        assert rows[1]["l2"] < rows[0]["l2"], n
    for i in range(2):
        e1, ew, em = (res[n][i]["l2"] for n in ("hllc1", "waf", "muscl_superbee"))
        assert em < ew < e1, (i, e1, ew, em)
