"""Writes the stored oracle results of the full-length parity tests (calls
only the FP64 oracle and the input generators; nothing from the HIP path).

* config2_muscl_rk2_1000.npz: the 10 km x 2 km river (999,824 cells),
  minmod MUSCL-HLLC-RK2 with hydrostatic reconstruction and Manning
  friction, 1000 steps of the fixed step dt = the CFL step of the initial
  state (Sec. 6.1 with CFL 0.45; Sec. 6.2.3 for MUSCL).
* config3_full_muscl_rk2_100.npz: the 40 km x 8 km river (13,000,560 cells)
  from its dam-break start, the same scheme, 100 fixed steps.

Each file holds a uniform sample of cells (every 16th / 256th cell of the
generator numbering: ``ids``) with the oracle's h, hu, hv there (rounded to
float32: 6e-8 relative, far below the 1e-4 bar), the maximum |h|, |hu|,
|hv| over all cells (float64, the denominators of the relative error), the
total water volume sum(area h) and the step.

    python tests/golden/make_full_length.py [config2|config3]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from swe_inputs import config2, config3  # noqa: E402

CASES = {
    "config2": (config2, 1000, 16, "config2_muscl_rk2_1000.npz"),
    "config3": (config3, 100, 256, "config3_full_muscl_rk2_100.npz"),
}


def make(name):
    gen, steps, stride, fname = CASES[name]
    t0 = time.time()
    sc = gen()
    M, _ = O.global_mesh(sc)
    par = O.scenario_params(sc, scheme=O.MUSCL, integrator=O.RK2, limiter=O.MINMOD)
    dt = M.dt(par, sc.h, sc.hu, sc.hv)
    h, hu, hv, t, fl = M.run(par, sc.h, sc.hu, sc.hv, steps, dt_fixed=dt)
    area = M.geometry()["area"]
    ids = np.arange(0, sc.n_cells, stride, dtype=np.int32)
    np.savez_compressed(
        os.path.join(HERE, fname), ids=ids,
        h=h[ids].astype(np.float32), hu=hu[ids].astype(np.float32), hv=hv[ids].astype(np.float32),
        maxabs=np.array([np.abs(h).max(), np.abs(hu).max(), np.abs(hv).max()]),
        volume=np.array(float(np.sum(area * h))), dt=np.array(dt), steps=np.array(steps),
        n_cells=np.array(sc.n_cells), flags=np.array(fl))
    print(f"{name}: {sc.n_cells} cells, {steps} steps of {dt:.6g} s, flags {fl}, "
          f"{time.time() - t0:.0f} s -> {fname}", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(CASES)):
        make(n)
