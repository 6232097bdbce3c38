"""Solution output overlapping the steps (Sec. 5.2: solutions written while
the solver keeps computing).  swe_snapshot copies the state, as it stands
after the steps queued before it, into device staging buffers on the
context's stream; the binding moves it to pinned host memory on a side
stream while the following steps run.

* snapshots taken between queued steps equal synchronous reads of a twin
  context at the same step, bitwise (FP32, FP64, an ensemble context, a
  context on a torch stream with torch-allocated buffers), including the
  reuse of the two staging slots;
* buffers that are not device memory are refused and the context stays
  usable;
* on the million-cell river the snapshots cost less than the synchronous
  reads they replace (timings printed).
"""
import ctypes as C
import time

import numpy as np
import pytest

from gpu_util import make_pair, lib
from swe_inputs import river_channel, config2

pytestmark = pytest.mark.gpu

ARG = -1


def _river():
    return river_channel(Lx=2000.0, Ly=400.0, nx=160, ny=32, seed=2)


@pytest.mark.parametrize("prec", [0, 1])
def test_snapshots_equal_synchronous_reads(prec):
    sc = _river()
    a, _, _, pr = make_pair(sc, "muscl_minmod_rk2", precision=prec)
    b, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=prec, prepared=pr)
    plan = (10, 10, 7, 1, 25)                 # five snapshots: both slots reused
    snaps = []
    for n in plan:
        a.step(n)
        snaps.append(a.snapshot())
    a.step(5)                                 # queued behind the last snapshot
    for n, snap in zip(plan, snaps):
        b.step(n)
        ref = b.read_state()
        got = snap.wait()
        for f in range(3):
            assert got[f].dtype == ref[f].dtype
            assert np.array_equal(got[f], ref[f]), (n, f)
    b.step(5)
    for x, y in zip(a.read_state(), b.read_state()):
        assert np.array_equal(x, y)


def test_snapshot_on_a_borrowed_stream_with_torch_memory():
    """A context on a torch stream, its buffers from torch's allocator: the
    snapshot still equals a synchronous read at the same step, and torch work
    queued on that stream after the snapshot does not disturb it."""
    import torch
    sc = _river()
    st = torch.cuda.Stream()
    a, _, _, pr = make_pair(sc, "muscl_minmod_rk2", precision=0, stream=st, allocator="torch")
    b, _, _, _ = make_pair(sc, "muscl_minmod_rk2", precision=0, prepared=pr)
    with torch.cuda.stream(st):
        a.step(15)
        snap = a.snapshot()
        junk = torch.full((1 << 22,), 3.0, device="cuda")   # torch work behind it on st
        a.step(10)
    b.step(15)
    ref = b.read_state()
    got = snap.wait()
    for f in range(3):
        assert np.array_equal(got[f], ref[f])
    assert float(junk[0]) == 3.0
    b.step(10)
    for x, y in zip(a.read_state(), b.read_state()):
        assert np.array_equal(x, y)


def test_snapshot_of_an_ensemble_context():
    swe, prepare_scenario = lib()
    scs = [river_channel(Lx=800.0, Ly=200.0, nx=40 + 8 * i, ny=10, seed=30 + i) for i in range(3)]
    preps = [prepare_scenario(x) for x in scs]

    def ctx():
        s = swe.Solver(precision=0, scheme=1, integrator=1, limiter=0)
        s.mesh_upload_batch([p.mesh for p in preps])
        s.set_state(*(np.concatenate([getattr(x, f)[p.sub.l2g] for x, p in zip(scs, preps)])
                      for f in ("h", "hu", "hv")))
        return s
    a, b = ctx(), ctx()
    a.step(12)
    snap = a.snapshot()
    a.step(3)
    b.step(12)
    ref = b.read_state()
    got = snap.wait()
    assert got[0].size == a.offsets[-1]
    for f in range(3):
        assert np.array_equal(got[f], ref[f])


def test_snapshot_refuses_host_buffers():
    import torch
    swe, _ = lib()
    sc = _river()
    s, _, _, pr = make_pair(sc, "muscl_minmod_rk2", precision=0)
    n = pr.mesh.n_total
    host = [np.empty(n, np.float32) for _ in range(3)]
    ptrs = [C.c_void_p(x.ctypes.data) for x in host]
    assert swe._lib.swe_snapshot(s.ctx, *ptrs, None) == ARG
    dev = torch.empty((3, n), dtype=torch.float32, device="cuda")
    mixed = [C.c_void_p(dev[0].data_ptr()), ptrs[1], C.c_void_p(dev[2].data_ptr())]
    assert swe._lib.swe_snapshot(s.ctx, *mixed, None) == ARG
    assert swe._lib.swe_snapshot(s.ctx, None, *ptrs[1:], None) == ARG
    # the refused calls leave no error behind: steps, a device snapshot and a read work
    s.step(4)
    torch.cuda.synchronize()
    assert swe._lib.swe_snapshot(s.ctx, *(C.c_void_p(dev[f].data_ptr()) for f in range(3)),
                                 None) == swe.SWE_OK
    ref = s.read_state()
    got = dev.cpu().numpy()
    for f in range(3):
        assert np.array_equal(got[f], ref[f])
    assert s.health() == 0


def test_snapshots_overlap_the_steps():
    """Config 2 (999,824 cells, FP32 MUSCL-HLLC-RK2), 400 CFL steps with the
    state taken every 20 steps: asynchronous snapshots against synchronous
    reads into host memory."""
    import torch
    sc = config2()
    s, _, _, pr = make_pair(sc, "muscl_minmod_rk2", precision=0)
    s.step(40)
    s.sync()
    steps, every = 400, 20

    def timed(mode):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        snaps = []
        for _ in range(steps // every):
            s.step(every)
            if mode == "snapshot":
                snaps.append(s.snapshot())
            elif mode == "read":
                s.read_state()
        s.sync()
        for x in snaps:
            x.wait()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    timed("snapshot")                         # staging slots, pinned pool, side stream
    t_none, t_snap, t_read = timed("none"), timed("snapshot"), timed("read")
    per = 1e3 / (steps // every)
    print(f"400 steps: no output {1e3 * t_none:.1f} ms; a snapshot every 20 steps "
          f"+{per * (t_snap - t_none):.3f} ms each; a synchronous read every 20 steps "
          f"+{per * (t_read - t_none):.3f} ms each")
    assert t_snap < t_read
    assert s.health() == 0
