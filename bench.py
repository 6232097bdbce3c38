#!/usr/bin/env python3
"""Benchmark: cell-updates/s of the MUSCL-HLLC-RK2 step on one MI355X.

Workload (default ``config3_full``): the 40 km x 8 km meandering river,
5702 x 1140 quads = 13,000,560 triangles, bumpy bed with dry banks and
emerging islands, Manning n in [0.02, 0.05], a 2 m dam break at mid reach,
500 m^3/s inflow, fixed-stage outflow, FP32 state, minmod MUSCL +
hydrostatic reconstruction + HLLC + Manning + SSP-RK2, CFL 0.45.  One
"step" is one full time step: both RK2 stages (reconstruction, fluxes,
sources, friction, update) and the on-device CFL reduction for the next
step; the state stays in HBM for the whole timed region.

Timing: W untimed warm-up steps, then the step graph is built (no capture
inside a timed region), then five timed runs, each of K steps repeated
until the run lasts at least 200 ms; ``value`` = owned cells x steps /
seconds of the median run (host clock around the steps, stream synchronised
on both sides).

``roofline`` prices the step's dominant kernel against 8 TB/s with the
compact algorithmic byte model of the step (state in and out, bed,
Manning n, neighbour and node ids, node coordinates: 132 B per MUSCL-RK2
cell-update in FP32, 60 B per first-order Euler update in FP32, 88 B per
first-order FP64 update); its launch time comes from HIP events recorded on
the library's stream around each timed run.  ``frac_stored_model`` gives the
same time priced with the stored-geometry byte model (212 B per MUSCL-RK2
update).  ``traffic`` is the HBM bytes per launch read from the committed
rocprofv3 counter summary of the same kernel sources, or null.
``cpu_baseline`` times the serial FP64 oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def compact_bytes(precision, rk2):
    """Algorithmic HBM bytes per cell-update, compact model (what one step
    must move): per stage the state in (3 values) and out (3), bed and
    Manning n (1 each), three neighbour ids and three node ids (4 B each)
    and the node coordinates (about half a node per cell, 2 values); the
    second RK2 stage also reads U^n (3 values).  FP32: 60 B per stage,
    132 B per RK2 step.  The first-order FP64 figure leaves out Manning n
    (88 B), as that workload has none."""
    s = 8 if precision == 1 else 4
    stage = 3 * s + s + s + 12 + 12 + s + 3 * s
    if rk2:
        return 2 * stage + 3 * s
    return stage - (s if precision == 1 else 0)


def stored_bytes(precision, rk2):
    """The same with stored geometry instead of node coordinates (98 B +
    114 B per FP32 RK2 step; 102 B FP32 / 132 B FP64 per Euler step)."""
    if rk2:
        return 212 * (2 if precision == 1 else 1)
    return 132 if precision == 1 else 102


MUSCL_RK2 = dict(precision=0, scheme=1, integrator=1, limiter=0)


def workload(name):
    """(scenario or list of scenarios, solver options, parts P, ghost layers k)."""
    from swe_inputs import config1, config2, config3, ensemble_scenarios
    if name == "config1":
        return config1(), dict(precision=1, scheme=0, integrator=0, limiter=0), 1, 0
    if name == "config2":
        return config2(), MUSCL_RK2, 1, 0
    if name == "config3_full":
        return config3(), MUSCL_RK2, 1, 0
    if name == "config3_part":
        # one GPU's share: the largest of 32 greedy-BFS parts, 4 ghost layers
        # (one MUSCL-RK2 step per exchange), send buffers packed every step
        return config3(), MUSCL_RK2, 32, 4
    if name == "config5":
        return ensemble_scenarios(), MUSCL_RK2, 1, 0
    if name == "dambreak_1m":
        # WAF's own workload: config 1's wet dam break (h 1 m / 0.5 m, flat,
        # walls, dx = 0.5 m) widened to 1118 x 447 quads = 999,492 cells; the
        # rivers' dry banks break WAF's positivity
        from swe_inputs import dam_break_channel
        return (dam_break_channel(Lx=559.0, Ly=223.5, nx=1118, ny=447, x_dam=279.5),
                dict(precision=0, scheme=2, integrator=0, limiter=0), 1, 0)
    raise SystemExit(f"unknown workload {name}")


def exchange_interval(kw, k, requested=0):
    """Steps per exchange of a sub-domain with k ghost layers: a step reads
    r layers (4 for MUSCL-RK2, 2 for MUSCL-Euler and WAF, 1 for first-order
    HLLC), so k layers last k // r steps; ``requested`` (> 0) asks for a
    shorter interval."""
    radius = 4 if kw["integrator"] == 1 else (2 if kw["scheme"] != 0 else 1)
    most = max(1, k // radius)
    if requested > most:
        raise SystemExit(f"{k} ghost layers allow at most {most} steps per exchange")
    return requested if requested > 0 else most


def kernel_source_hash():
    """sha256 of the device sources (the .hip files and the headers they
    include; the host toolkit, .cpp built by g++, holds no device code): a
    traffic figure measured on other sources does not describe the present
    kernel."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2307_16758_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def measured_traffic(workload_name, kernel):
    """HBM bytes per stage launch from the committed PMC summary of this
    kernel and workload (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known
    size), or None when it is absent or was taken on different kernel
    sources."""
    f = os.path.join(ROOT, "profiles", f"{kernel}_{workload_name}_traffic.md")
    if not os.path.exists(f):
        return None
    vals = {}
    for line in open(f):
        if ":" in line and line.strip().startswith(("traffic_bytes_per_launch", "source_sha256")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_cpu():
    """Model name of the host CPU and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def _oracle_rate(sc, kw, seconds, mlp=None):
    """(cell-updates, steps, seconds) of the serial FP64 oracle on one
    scenario (its own neighbour search, in the generator's numbering): as
    many steps as fit in about ``seconds`` (at least one)."""
    from oracle import oracle as O
    M, _ = O.global_mesh(sc)
    p = O.scenario_params(sc, scheme=kw["scheme"], integrator=kw["integrator"],
                          limiter=kw["limiter"])
    if mlp is not None:
        p.mlp = mlp
    h, hu, hv, t = sc.h, sc.hu, sc.hv, 0.0
    steps, t0 = 0, time.perf_counter()
    while True:
        h, hu, hv, t, _ = M.run(p, h, hu, hv, 1, t=t)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return sc.n_cells * steps, steps, el


def _member_rate(args):
    """Worker of the aggregate baseline: ensemble member s on its own core."""
    s, kw, seconds, cpu = args
    if cpu is not None:
        os.sched_setaffinity(0, {cpu})
    from swe_inputs.scenarios import ensemble_member
    sc = ensemble_member(s)
    upd, steps, el = _oracle_rate(sc, kw, seconds)
    return sc.n_cells, steps, upd / el


def cpu_baseline(sc, kw, seconds, mlp=None):
    """Serial FP64 oracle on the same mesh, pinned to one core of this
    process's CPU set."""
    cpus = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    if cpus:
        os.sched_setaffinity(0, {cpus[0]})
    try:
        upd, steps, el = _oracle_rate(sc, kw, seconds, mlp)
    finally:
        if cpus:
            os.sched_setaffinity(0, set(cpus))
    model, ncpu, avail = host_cpu()
    return dict(value=upd / el, unit="cell-updates/s", cores=1, kind="oracle",
                sample=f"{sc.name}: {sc.n_cells} cells, first {steps} steps, serial FP64 "
                       f"({el:.1f} s, one core)",
                host_cpu=model, nproc=ncpu, cores_available=avail)


def cpu_baseline_aggregate(n_members, kw, seconds, max_workers=16):
    """The ensemble's fair CPU comparison: independent serial FP64 oracle
    processes, one per core (at most ``max_workers``), each stepping its own
    member for about ``seconds``; the aggregate is the sum of their rates."""
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    cpus = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else []
    w = max(1, min(max_workers, len(cpus) if cpus else (os.cpu_count() or 1), n_members))
    jobs = [(s, kw, seconds, cpus[s] if cpus else None) for s in range(w)]
    with ProcessPoolExecutor(max_workers=w, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_member_rate, jobs))
    model, ncpu, avail = host_cpu()
    cells = sum(r[0] for r in res)
    return dict(value=sum(r[2] for r in res), unit="cell-updates/s", cores=w, kind="oracle",
                sample=f"members 0-{w - 1} of the ensemble ({cells} cells), one serial FP64 "
                       f"oracle process per core, each about {seconds:.0f} s "
                       f"({min(r[1] for r in res)}-{max(r[1] for r in res)} steps)",
                host_cpu=model, nproc=ncpu, cores_available=avail)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=12)
    ap.add_argument("--runs", type=int, default=5, help="timed runs (the median is reported)")
    ap.add_argument("--min-run-ms", type=float, default=200.0,
                    help="each timed run repeats the K steps until it lasts this long")
    ap.add_argument("--workload", default="config3_full")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--cell-kernel", type=int, default=0)
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--scheme", choices=("muscl", "waf", "hllc1"), default="muscl",
                    help="waf / hllc1: first-order WAF or HLLC with explicit Euler (FP32) instead "
                         "of MUSCL-HLLC-RK2")
    ap.add_argument("--limiter", choices=("minmod", "learned"), default="minmod",
                    help="learned: the per-edge network (untrained weights: its cost, not its "
                         "accuracy) ahead of every stage")
    ap.add_argument("--phi-in-stage", type=int, default=0,
                    help="learned limiter: 1 evaluates the network inside the first stage "
                         "instead of in a kernel of its own ahead of each step")
    ap.add_argument("--phi-every", type=int, default=1, choices=(1, 2, 3, 6),
                    help="learned limiter: evaluate the network every PHI_EVERY steps (the "
                         "steps between reuse its last phi)")
    ap.add_argument("--snapshot-every", type=int, default=0, metavar="M",
                    help="take the state to pinned host memory every M steps (swe_snapshot, "
                         "copied on a side stream while the steps go on), inside the timed region")
    ap.add_argument("--overlap", action="store_true",
                    help="sub-domain workloads: each step with the high-overlap schedule "
                         "(swe_step_overlap: send cells' tiles, pack on a side stream while the "
                         "other tiles run) instead of a step followed by a pack")
    ap.add_argument("--exchange-every", type=int, default=0, metavar="M",
                    help="sub-domain workloads: steps per exchange (pack and unpack); 0: the "
                         "most the ghost layers allow, k // r for stencil radius r per step "
                         "(4 MUSCL-RK2, 2 WAF, 1 first-order HLLC)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times "
                         "(reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        # a gather-like read: 16 bytes out of every 128-byte line (one
        # reduction kernel), to check that the byte counters count whole
        # lines for scattered accesses too
        lines = src.view(-1, 32)[:, :4]
        part = lines.sum(dtype=torch.float32)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5,
                          "strided_read_lines": n // 32, "strided_read_line_bytes": 128 * (n // 32),
                          "strided_sum": float(part)}))
        return
    if args.gpus != 1:
        print("this benchmark runs on exactly one GPU: the path measured is one GPU's "
              "sub-domain (multi-GPU exchange is not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2307_16758_amd import swe
    from paper_2307_16758_amd.problem import prepare_scenario

    sc, kw, P, k = workload(args.workload)
    if args.scheme != "muscl":
        kw = dict(kw, scheme=2 if args.scheme == "waf" else 0, integrator=0)
    if args.limiter == "learned":
        kw = dict(kw, limiter=swe.LEARNED)
    s = swe.Solver(device=0, block=args.block, cell_kernel=args.cell_kernel,
                   phi_in_stage=args.phi_in_stage, phi_every=args.phi_every, **kw)
    mlp = None
    if args.limiter == "learned":
        from paper_2307_16758_amd.limiter_train import init_params
        mlp = init_params()
        s.limiter_set_weights(mlp)
    sendbuf = recvbuf = None
    if isinstance(sc, list):                      # batched ensemble
        preps = [prepare_scenario(x) for x in sc]
        s.mesh_upload_batch([p.mesh for p in preps])
        for i, x in enumerate(sc):
            if x.hydrograph is not None:
                s.set_bc_series_scenario(i, *x.hydrograph)
        s.set_state(np.concatenate([x.h[p.sub.l2g] for x, p in zip(sc, preps)]),
                    np.concatenate([x.hu[p.sub.l2g] for x, p in zip(sc, preps)]),
                    np.concatenate([x.hv[p.sub.l2g] for x, p in zip(sc, preps)]))
        n_owned = int(sum(p.sub.n_owned for p in preps))
        name = f"{len(sc)} scenarios"
    else:
        if P > 1:
            from paper_2307_16758_amd import swe as _s
            nbr = _s.swe_dual_graph(sc.mesh.n_nodes, sc.mesh.tri)
            part = _s.swe_partition_bfs(nbr, P)
            p = int(np.argmax(np.bincount(part, minlength=P)))
            pr = prepare_scenario(sc, P=P, p=p, k=k, nbr_global=nbr, part=part)
        else:
            pr = prepare_scenario(sc)
        s.mesh_upload(pr.mesh)
        if sc.hydrograph is not None:
            s.set_bc_series(*sc.hydrograph)
        l2g = pr.sub.l2g
        s.set_state(sc.h[l2g], sc.hu[l2g], sc.hv[l2g])
        n_owned = pr.sub.n_owned
        name = sc.name
        if P > 1:
            n_send, n_ghost = s.ghost_sizes()
            sendbuf = torch.empty(3 * max(1, n_send), dtype=torch.float32, device="cuda")
            # the peers' values of each exchange: the ghosts' initial state
            # stands in for them (no peer runs here), so the ghost layers
            # stay a fixed boundary instead of stepping beyond the CFL limit
            # of the owned cells
            g = l2g[n_owned:]
            recvbuf = torch.from_numpy(np.concatenate([sc.h[g], sc.hu[g], sc.hv[g]])
                                       .astype(np.float32)).cuda()
            torch.cuda.synchronize()

    exch = exchange_interval(kw, k, args.exchange_every) if sendbuf is not None else 1

    def whole(n):
        """n rounded up to whole exchange intervals."""
        return exch * -(-n // exch)

    tuned = s.autotune(10) if args.autotune else None
    s.step(args.warmup)
    if args.snapshot_every > 0:
        # staging slots, side stream and pinned pool are set up by the first
        # snapshots: part of the warm-up, like the kernels' first launches
        for _ in range(3):
            s.snapshot().wait()
    s.prepare()           # the step graph is captured here, outside every timed region
    s.sync()
    kname, launches_per_step = s.step_kernel()
    if "k_limiter_phi" in kname and args.phi_every > 1:
        # the network's launch runs on one step in phi_every
        launches_per_step -= 1.0 - 1.0 / args.phi_every
    plain = sendbuf is None and args.snapshot_every <= 0

    def one_run(nsteps):
        """Host seconds of nsteps steps of the timed job, and the HIP-event
        milliseconds of its kernels on the library stream (plain runs)."""
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if args.snapshot_every > 0:
            snaps, done = [], 0
            while done < nsteps:
                m = min(args.snapshot_every, nsteps - done)
                s.step(m)
                done += m
                snaps = snaps[-1:] + [s.snapshot()]   # older ones are complete (two slots)
            s.sync()
            for x in snaps:
                x.wait()
        elif sendbuf is None:
            s.step(nsteps)
            s.sync()
        elif args.overlap:
            for _ in range(nsteps // exch):   # per exchange interval, the last step's pack overlapped
                if exch > 1:
                    s.step(exch - 1)
                s.step_overlap(sendbuf)
                s.unpack_ghosts(recvbuf)
            s.sync()
        else:
            for _ in range(nsteps // exch):   # per exchange interval: steps, pack, unpack
                s.step(exch)
                s.pack_ghosts(sendbuf)
                s.unpack_ghosts(recvbuf)
            s.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, (s.last_step_ms() if plain else None)

    # one untimed run of K steps sizes the timed runs: K steps repeated
    # until a run lasts at least min_run_ms
    w0, _ = one_run(whole(args.steps))
    reps = max(1, int(np.ceil(args.min_run_ms * 1e-3 / max(w0, 1e-9))))
    per_run = whole(args.steps * reps)
    runs = [one_run(per_run) for _ in range(args.runs)]
    walls = sorted(r[0] for r in runs)
    wall = walls[len(walls) // 2]
    if plain:
        ev = sorted(r[1] for r in runs)
        gpu_ms = ev[len(ev) // 2]
    else:
        # the kernels alone (HIP events on the library stream) for the
        # roofline; the state moves on, which the timed job does not mind
        s.step(per_run)
        s.sync()
        gpu_ms = s.last_step_ms()
    health = s.health()

    rk2 = kw["integrator"] == 1
    prec = kw["precision"]
    launches = per_run * launches_per_step
    avg_launch_s = gpu_ms * 1e-3 / launches
    per_launch_bytes = compact_bytes(prec, rk2) * n_owned / launches_per_step
    achieved = per_launch_bytes / avg_launch_s / 1e9
    stored = stored_bytes(prec, rk2) * n_owned / launches_per_step / avg_launch_s / 1e9
    traffic = None
    if not args.cell_kernel and not tuned:
        traffic = measured_traffic(args.workload, kname)
    scheme_name = "MUSCL-HLLC" if rk2 else ("WAF" if kw["scheme"] == 2 else "HLLC")
    model, ncpu, avail = host_cpu()
    out = {
        "metric": "cell-updates/s ({}, {}, 1 GPU)".format(scheme_name, "FP32" if prec == 0 else "FP64"),
        "value": n_owned * per_run / wall,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / per_run,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == 0 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {name}, {n_owned} owned triangles, "
                               f"{'MUSCL-HLLC-RK2' if rk2 else scheme_name + '-Euler'}"
                               + (", learned limiter" if args.limiter == "learned" else "")
                               + (f" (network every {args.phi_every} steps)"
                                  if args.limiter == "learned" and args.phi_every > 1 else "")
                               + (f", part of {P} with {k} ghost layers + pack and unpack every "
                                  + (f"{exch} steps" if exch > 1 else "step")
                                  + (" (high-overlap steps)" if args.overlap else "") if P > 1 else "")
                               + (f", snapshot to host every {args.snapshot_every} steps"
                                  if args.snapshot_every > 0 else ""),
                   "cells": n_owned, "tuned_launch": tuned,
                   "parallelism": "single GPU" + (", one sub-domain" if P > 1 else ", single domain")},
        "timing": {"runs": args.runs, "steps_per_run": per_run, "stat": "median",
                   "run_ms": [1e3 * w for w in walls], "graph_prepared_before_timing": True},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kname, "launches_per_step": launches_per_step,
                     "avg_launch_us": avg_launch_s * 1e6,
                     "bytes_per_launch": per_launch_bytes,
                     "byte_model": f"compact, {compact_bytes(prec, rk2)} B per cell-update",
                     "frac_stored_model": stored / HBM_PEAK_GBS},
        "health_bits": health,
        "host": {"cpu": model, "nproc": ncpu, "cores_available": avail},
    }
    if not args.no_cpu_baseline:
        if isinstance(sc, list):    # the ensemble: one oracle process per core
            out["cpu_baseline"] = cpu_baseline_aggregate(len(sc), kw, args.cpu_seconds)
        else:
            out["cpu_baseline"] = cpu_baseline(sc, kw, args.cpu_seconds, mlp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
