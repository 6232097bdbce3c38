"""Time against error of the paper's three schemes on the wet-bed dam break
(Sec. 6.4, the time-error comparison; the dam break of Sec. 6.3).

First-order HLLC, WAF and MUSCL, with superbee limiting for both
second-order schemes as the paper uses them there (MUSCL with minmod as
well), on one GPU, on meshes of about 20,000 to 600,000 triangles.  The
error is the L2 norm of the depth at the cell centroids against the exact
solution at t_end, weighted by cell area; the time is the GPU time of the
steps (HIP events on the library stream).

    python -m paper_2307_16758_amd.time_error [--t-end 5] [--out results.json]
"""
from __future__ import annotations

import math

import numpy as np

from . import swe

G = 9.81

# (nx, ny) quads of the 100 x 20 m channel, two triangles each: 20,160 to
# 599,760 cells
LADDER = ((224, 45), (354, 71), (500, 100), (708, 141), (1000, 200), (1224, 245))

SCHEMES = {
    "hllc1": dict(scheme=swe.HLLC1, integrator=swe.EULER, limiter=swe.MINMOD),
    "waf": dict(scheme=swe.WAF, integrator=swe.EULER, waf_limiter=swe.WAF_SUPERBEE),
    "muscl_superbee": dict(scheme=swe.MUSCL, integrator=swe.RK2, limiter=swe.SUPERBEE),
    "muscl_minmod": dict(scheme=swe.MUSCL, integrator=swe.RK2, limiter=swe.MINMOD),
}


def stoker_depth(xi, h_left, h_right, g=G):
    """Exact depth of the dam break on a wet bed (both sides at rest,
    h_left > h_right > 0) at x - x_dam = xi * t: a rarefaction into the
    deep side and a shock into the shallow one around a middle state.
    The middle depth h_m makes the velocity behind the rarefaction,
    2 (sqrt(g h_left) - sqrt(g h_m)), equal to the velocity the shock's
    jump conditions give, (h_m - h_right) sqrt(g (h_m + h_right) / (2 h_m
    h_right)); the difference decreases in h_m on [h_right, h_left], so
    bisection finds it."""
    c_l = math.sqrt(g * h_left)

    def gap(h):
        return (2.0 * (c_l - math.sqrt(g * h))
                - (h - h_right) * math.sqrt(g * (h + h_right) / (2.0 * h * h_right)))

    lo, hi = h_right, h_left
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if gap(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    h_m = 0.5 * (lo + hi)
    c_m = math.sqrt(g * h_m)
    u_m = 2.0 * (c_l - c_m)
    s = h_m * u_m / (h_m - h_right)          # shock speed from mass conservation
    xi = np.asarray(xi, np.float64)
    fan = (2.0 * c_l - xi) / 3.0             # celerity inside the rarefaction
    return np.where(xi < -c_l, h_left,
                    np.where(xi < u_m - c_m, fan * fan / g,
                             np.where(xi < s, h_m, h_right)))


def run(nx, ny, name, t_end=5.0, precision=swe.F32, cfl=0.45):
    """One scheme on one mesh of the 100 x 20 m channel (dam at x = 50 m,
    1 m against 0.5 m, walls) to t_end: cells, L2 error of the depth, GPU
    seconds and steps."""
    from swe_inputs import dam_break_channel
    from .problem import prepare_scenario
    sc = dam_break_channel(Lx=100.0, Ly=20.0, nx=nx, ny=ny, x_dam=50.0)
    pr = prepare_scenario(sc)
    s = swe.Solver(precision=precision, cfl=cfl, **SCHEMES[name])
    try:
        s.mesh_upload(pr.mesh)
        l2g = pr.sub.l2g
        s.set_state(sc.h[l2g], sc.hu[l2g], sc.hv[l2g])
        gpu, steps = 0.0, 0
        while s.time() < t_end - 1e-12:
            dt = min(s.local_dt(), t_end - s.time())
            s.step(1, dt)
            gpu += s.last_step_ms() * 1e-3
            steps += 1
        h = s.read_state()[0].astype(np.float64)
    finally:
        s.close()
    c = sc.mesh.centroids()[l2g]
    p = sc.mesh.xy[sc.mesh.tri[l2g]]
    area = 0.5 * np.abs((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                        - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    exact = stoker_depth((c[:, 0] - 50.0) / t_end, 1.0, 0.5)
    l2 = math.sqrt(float(np.sum(area * (h - exact) ** 2) / np.sum(area)))
    return dict(cells=int(pr.sub.n_total), l2=l2, gpu_s=gpu, steps=steps)


def error_at_time(rows, t):
    """Error of a scheme's mesh ladder at GPU time t, interpolated log-log
    between the two runs around t (None outside the ladder's times)."""
    rows = sorted(rows, key=lambda r: r["gpu_s"])
    for a, b in zip(rows, rows[1:]):
        if a["gpu_s"] <= t <= b["gpu_s"]:
            w = math.log(t / a["gpu_s"]) / math.log(b["gpu_s"] / a["gpu_s"])
            return math.exp(math.log(a["l2"]) + w * (math.log(b["l2"]) - math.log(a["l2"])))
    return None


def study(ladder=LADDER, names=tuple(SCHEMES), t_end=5.0, log=print):
    out = {n: [] for n in names}
    # one-time costs (code loading at a kernel's first launch) stay out of
    # the timed runs
    for n in names:
        run(ladder[0][0], ladder[0][1], n, t_end=0.05)
    for nx, ny in ladder:
        for n in names:
            r = run(nx, ny, n, t_end)
            out[n].append(r)
            log(f"{n:15s} {r['cells']:8d} cells  L2(h) {r['l2']:.4e}  GPU {r['gpu_s'] * 1e3:8.2f} ms"
                f"  {r['steps']} steps")
    # first-order error at each second-order run's time: how much more
    # accurate the second-order scheme is for the same computation time
    for n in names:
        if n == "hllc1" or "hllc1" not in out:
            continue
        for r in out[n]:
            e = error_at_time(out["hllc1"], r["gpu_s"])
            r["hllc1_l2_at_same_time"] = e
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--t-end", type=float, default=5.0)
    ap.add_argument("--sizes", type=int, default=len(LADDER),
                    help="number of meshes of the ladder to run, smallest first")
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    res = study(LADDER[:a.sizes], t_end=a.t_end)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    main()
