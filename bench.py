"""Benchmark of the quasi-static plasma-response hot path on one MI355X.

A step is one quasi-static cycle of the headline workload (two-bunch blowout,
512 x 4096 r-xi grid, 16 ring particles per cell, u_th = 0.02, 1e6-particle
evolving beam, FP32 bulk with FP64 solves): beam current from the
macroparticles -> plasma loaded ahead of the beam -> plasma response over
all 4096 slices -> beam push over dt = 40 -> witness energy-gain diagnostic.
All inputs are synthetic, seeded and resident in HBM before timing starts.

Prints one JSON line.  value = plasma particle-slice updates per second
(n_plasma * (n_xi - 1) per step).  The roofline entry is for the dominant
kernel (the march), timed with HIP events on the stream it runs on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# Algorithmic bytes per plasma particle-slice update of the method's state in
# the mixed mode: (r, p_r) double read + write (32 B) and (l_z, D0, w) float
# read (12 B).
BYTES_PER_UPDATE = 44.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=float, default=1.0,
                    help="fraction of one plasma response timed with the CPU oracle")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--threads", type=int, default=None, help="march workgroup size override")
    return ap.parse_args()


def cpu_baseline(p, fraction: float):
    """The FP64 oracle on the host: one plasma response of the same workload
    (or its first `fraction` of slices)."""
    import numpy as np
    from oracle import oracle as O
    from paper_1411_3246_amd import inputs
    O.lib()
    n_xi = max(2, int(p.n_xi * fraction))
    q = p.replace(prec="fp64")
    st = O.load_plasma(q, inputs.plasma_draws(q))
    b = O.load_beam(q, inputs.beam_draws(q))
    jb, _ = O.beam_current_macro(q, b)
    sub = q.replace(n_xi=n_xi)
    t0 = time.perf_counter()
    O.march(sub, st, np.ascontiguousarray(jb[:n_xi]))
    dt = time.perf_counter() - t0
    upd = q.n_plasma * (n_xi - 1)
    return {"value": upd / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one FP64 plasma response, {n_xi} of {q.n_xi} slices, {q.n_plasma} particles "
                      f"per slice ({upd:.3g} updates, {dt:.1f} s, serial C)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "the multi-GPU layout is a design note, not an implementation", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1411_3246_amd import inputs, wake

    torch.cuda.set_device(0)
    p = inputs.blowout_response()
    sim = wake.Simulation(p, threads=args.threads)
    sim.load_beam()
    stream = torch.cuda.current_stream()
    upd_per_step = p.updates_per_response()

    def step(ev=None):
        sim.beam_current()
        sim.plan.init_plasma(sim.plasma, sim.plasma_draws)
        if ev is not None:
            ev[0].record(stream)
        sim.plan.plasma_response(sim.plasma, sim.jb, sim.fields, sim.workspace, sim.counters)
        if ev is not None:
            ev[1].record(stream)
        sim.push(1)
        sim.plan.mean_gain(sim.beam, 1, sim.out[0:1], sim.workspace)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    march_ms = sum(a.elapsed_time(b) for a, b in events) / args.steps

    value = upd_per_step * args.steps / elapsed
    counters = sim.counters_dict()
    gain = float(sim.out[0].item())
    achieved = BYTES_PER_UPDATE * upd_per_step / (march_ms * 1e-3) / 1e9
    line = {
        "metric": "plasma particle-slice updates/s at 1 GPU",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {"workload": p.name, "geometry": p.geom, "n_r": p.n_r, "n_xi": p.n_xi,
                   "ppc": p.ppc, "u_th": p.u_th, "n_beam": p.n_beam, "beam_steps_timed": args.steps,
                   "dt": p.dt, "precision": "FP32 bulk, FP64 solve/accumulation/xi integration",
                   "march_threads": sim.plan.threads},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_march_one", "ms_per_launch": march_ms,
                     "bytes_per_update": BYTES_PER_UPDATE},
        "diagnostics": {"witness_mean_gain_gamma": gain, "counters": counters},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
