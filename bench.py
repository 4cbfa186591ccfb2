"""Benchmark of the quasi-static plasma-response hot path on one MI355X.

Workload: the two-bunch blowout run (512 x 4096 r-xi grid over r <= 6,
xi in [0, 10), 16 ring particles per cell with u_th = 0.02, drive n_b = 8,
sigma_r = 0.3, sigma_z = 0.7, witness with 0.3 of its charge 4.5 behind,
1e6-particle beam at gamma = 4e4 with 0.1 % energy spread, dt = 40), FP32
bulk with FP64 field solves, deposit accumulation and xi integration.
Synthetic, seeded inputs resident in HBM before timing starts.

A step is one quasi-static cycle: beam current from the macroparticles ->
plasma (loaded ahead of the beam) marched through all 4096 slices -> beam
advanced by dt.  The timed region runs `--steps` cycles from the loaded beam
as one pipelined launch (responses of successive steps overlap across
workgroups) plus the witness energy-gain diagnostic.  `--mode sequential`
times the same cycles one response at a time instead.

Prints one JSON line.  value = plasma particle-slice updates per second
(n_plasma * (n_xi - 1) per step).  The roofline entry is for the dominant
kernel (the cycle kernel, or the march kernel in sequential mode), timed
with HIP events on the stream it runs on.
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
FP32_PEAK_TFLOPS = 157.3       # MI355X vector FP32
# Algorithmic bytes per plasma particle-slice update in the mixed mode: the
# method's particle state (r, p_r) in double read and written (32 B) and
# (l_z, D0, w) in float read (12 B) once per slice.
BYTES_PER_UPDATE = 44.0
# Algorithmic floating-point operations per update (both Heun stages of the
# per-particle work: radius and radial momentum, the S deposit, gamma and p_z
# from psi, seven moment deposits, the derivative and the state update, plus
# the per-slice grid solves spread over the particles; counted from the
# equations, an FMA as two).
FLOPS_PER_UPDATE = 190.0
# HBM bytes per update of the cycle kernel and of the batched march, from
# scaled FETCH_SIZE + WRITE_SIZE counter runs (rocprofv3 --pmc), recorded for
# a hash of the kernel sources; reported only while the sources match.
PROFILES = os.path.join(ROOT, "profiles")
# one record per launch size: 20 steps (groups of 8 workgroups) and 200
# steps (one workgroup per response)
CYCLE_COUNTERS = tuple(os.path.join(PROFILES, f"k_cycle_two-bunch-512x4096-ppc16-beam1e6{s}.counters.json")
                       for s in ("", "-200steps"))
SCAN_COUNTERS = os.path.join(PROFILES, "k_march_batch_scan-256.counters.json")
CONV_COUNTERS = {g: os.path.join(PROFILES, f"k_cycle_convergence-{g}-2048-ppc64.counters.json")
                 for g in ("cyl", "slab")}
KERNEL_SOURCES = ("wk_cycle_impl.h", "wk_march_impl.h", "wk_marcher.h", "wk_beam_dev.h", "wk_internal.h")


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1411_3246_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(paths, updates: float):
    """HBM bytes of a launch of `updates` particle-slice updates from the
    committed counter record of that launch size (one path or several), or
    None when the kernel sources changed since it was taken, or when no record
    is of this launch size (another step count changes the cycle's group size
    and so its exchange traffic)."""
    for path in ((paths,) if isinstance(paths, str) else paths):
        try:
            with open(path) as f:
                rec = json.load(f)
        except OSError:
            continue
        if source_hash() == rec.get("source_hash") and int(rec.get("updates", -1)) == int(updates):
            return rec["bytes_per_update"] * updates
    return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Host threads for the multi-core oracle run: the cores this process may
    use, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def roofline(updates: float, ms: float, traffic, kernel: str, launches: int) -> dict:
    """Roofline entry of a launch: algorithmic HBM bytes against the HBM peak.
    The method's algorithmic intensity (FLOPS_PER_UPDATE / BYTES_PER_UPDATE,
    about 4.3 flop/B) is below the FP32 ridge point (157.3 / 8 = 19.7 flop/B),
    so HBM is the roof; the FP32 fraction is given beside it."""
    achieved = BYTES_PER_UPDATE * updates / (ms * 1e-3) / 1e9
    flops = FLOPS_PER_UPDATE * updates / (ms * 1e-3) / 1e12
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel, "launches": launches,
            "ms_per_launch": ms / launches, "bytes_per_update": BYTES_PER_UPDATE,
            "traffic_unit": "bytes per launch",
            "intensity_flop_per_byte": FLOPS_PER_UPDATE / BYTES_PER_UPDATE,
            "fp32_tflops": flops, "fp32_frac": flops / FP32_PEAK_TFLOPS,
            "limiter": "latency: the per-slice chain of barriers and exchanges between the workgroups "
                       "of a response, not bandwidth or issue rate"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--mode", choices=["pipelined", "sequential"], default="pipelined")
    ap.add_argument("--cpu-sample", type=float, default=1.0,
                    help="fraction of one plasma response timed with the CPU oracle")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--threads", type=int, default=None, help="march workgroup size override")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--no-scan", action="store_true",
                    help="skip the batched 256-instance parameter scan")
    ap.add_argument("--scan-instances", type=int, default=256)
    ap.add_argument("--scan-reps", type=int, default=3, help="timed graph replays of the scan")
    ap.add_argument("--scan-cpu-slices", type=int, default=96,
                    help="slices of each scan instance in the multi-core oracle baseline")
    ap.add_argument("--workload", choices=["headline", "convergence", "te-scan", "table1-beam"],
                    default="headline",
                    help="convergence: the 2048-cell cylindrical (2048 x 16384) and slab (2048 x 8192) "
                         "runs, 64 particles per cell, 4e6 beam particles, against the 512-cell runs")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the gradient (adjoint / forward time) measurement")
    ap.add_argument("--grad-reps", type=int, default=3)
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
    return {"value": upd / dt, "unit": "updates/s", "cores": 1, "kind": "oracle", "cpu": cpu_model(),
            "sample": f"one FP64 plasma response of the same workload, {n_xi} of {q.n_xi} slices, "
                      f"{q.n_plasma} particles per slice ({upd:.3g} updates, {dt:.1f} s, serial C)"}


def scan_bench(args, log):
    """The batched parameter scan: every instance of the scan marched in one
    persistent launch (each instance by a group of workgroups sized to its
    cost, schedule picked by the autotuner, the whole pass replayed from a HIP
    graph), against the roofline and against the same instances run one
    standalone response at a time (each with its own group).

    The standalone time is measured on every instance with its xi window cut
    to 128 slices and scaled by (n_xi - 1) / 127 (a response costs the same
    per slice); the scaling is checked on a few instances run whole."""
    import torch
    from paper_1411_3246_amd import autotune, inputs, wake
    probs = inputs.scan_instances(args.scan_instances)
    scan = wake.Scan(probs)
    best, table = autotune.tune_scan(scan, log=log)
    groups = scan.groups
    scan.capture()
    stream = torch.cuda.current_stream()
    scan.replay()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    for _ in range(args.scan_reps):
        scan.replay()
    ev[1].record(stream)
    torch.cuda.synchronize()
    batched_ms = ev[0].elapsed_time(ev[1]) / args.scan_reps
    counters = wake.counters_dict(scan.counters)
    updates = scan.updates
    del scan
    torch.cuda.empty_cache()

    def standalone(qs, idx):
        sc = wake.Scan(qs)
        for i in idx:                    # warm-up of every kernel variant
            sc.run_one(i)
        torch.cuda.synchronize()
        out = []
        for i in idx:
            ev[0].record(stream)
            sc.run_one(i)
            ev[1].record(stream)
            ev[1].synchronize()
            out.append(ev[0].elapsed_time(ev[1]))
        del sc
        torch.cuda.empty_cache()
        return out

    cut = 128
    short = standalone([q.replace(n_xi=cut) for q in probs], range(len(probs)))
    est = [t * (q.n_xi - 1) / (cut - 1) for t, q in zip(short, probs)]
    check_idx = list(range(0, len(probs), max(1, len(probs) // 4)))[:4]
    whole = standalone([probs[i] for i in check_idx], range(len(check_idx)))
    seq_ms = sum(est)
    line = {
        "instances": len(probs),
        "updates": updates,
        "batched_ms": batched_ms,
        "batched_updates_per_s": updates / (batched_ms * 1e-3),
        "roofline": roofline(updates, batched_ms, measured_traffic(SCAN_COUNTERS, updates),
                             "k_march (batched)", 1),
        "standalone_ms_est": seq_ms,
        "batched_speedup": seq_ms / batched_ms,
        "standalone_scaling_check": [{"instance": probs[i].name, "whole_ms": w, "scaled_ms": est[i]}
                                     for i, w in zip(check_idx, whole)],
        "schedule": {"member_cap": best[0], "wg_per_cu": best[1], "workgroups": sum(groups),
                     "max_group": max(groups)},
        "tuner": table,
        "graph": True,
        "counters": counters,
        "recipe": "u_th~U[0,0.05], sep~U[3,6], n_r in {128,256,512,1024}, n_xi~U{1024..4096}, "
                  "ppc in {8..32 even}, fixed analytic two-bunch beam, mixed precision",
    }
    if not args.no_cpu:
        line["cpu_baseline"] = scan_cpu_baseline(probs, args.scan_cpu_slices)
    return line


def scan_cpu_baseline(probs, n_slices: int):
    """The FP64 oracle on every host thread this process may use: each
    thread marches whole instances of the scan (their first `n_slices`
    slices) one after another; the oracle is serial C, so the scan's
    instances are the unit of parallel work."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    from paper_1411_3246_amd import inputs
    O.lib()
    jobs = []
    for p in probs:
        q = p.replace(prec="fp64", n_xi=min(n_slices, p.n_xi))
        jobs.append(q)

    def setup(q):
        return q, O.load_plasma(q, inputs.plasma_draws(q)), np.ascontiguousarray(O.beam_current_analytic(q))

    def one(job):
        q, st, jb = job
        O.march(q, st, jb)
        return q.n_plasma * (q.n_xi - 1)

    threads = host_threads()
    with ThreadPoolExecutor(threads) as ex:
        ready = list(ex.map(setup, jobs))
        t0 = time.perf_counter()
        upd = sum(ex.map(one, ready))
        dt = time.perf_counter() - t0
    return {"value": upd / dt, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"every one of the {len(jobs)} scan instances in FP64, its first {n_slices} slices "
                      f"({upd:.3g} updates, {dt:.1f} s on {threads} threads, one instance per thread at a "
                      f"time; loading outside the timed marches)"}


def push_bench(sim, p):
    """The standalone beam push (wk_beam_push, Eqs. (8)-(11)): the beam
    advanced in one response's frozen fields, 1 and n_steps steps per launch,
    each the best of three runs timed with HIP events (the beam reloaded
    before each).  Bytes: the state (x, y, xi, px, py, pz, 48 B) is read and
    written once per launch and stays in registers between steps; each step
    gathers 3 fields at 4 nodes (12 loads of the field type), which the
    caches serve (the fields of one response are 34 MB in mixed precision)."""
    import torch
    sim.load_beam()
    sim.beam_current()
    sim.response()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    nb = p.n_beam
    field_bytes = 4 if p.prec == "mixed" else 8
    out = {"workload": p.name, "n_beam": nb, "field_type_bytes": field_bytes, "runs": []}
    for n in (1, p.n_steps):
        best = float("inf")
        for _ in range(3):
            sim.load_beam()
            torch.cuda.synchronize()
            ev[0].record(stream)
            sim.push(n)
            ev[1].record(stream)
            ev[1].synchronize()
            best = min(best, ev[0].elapsed_time(ev[1]))
        sec = best / 1e3
        out["runs"].append({
            "steps_per_launch": n, "ms": best,
            "particle_steps_per_s": nb * n / sec,
            "state_GB_per_s": 96.0 * nb / sec / 1e9,
            "gather_GB_per_s_from_cache": 12.0 * field_bytes * nb * n / sec / 1e9,
        })
    return out


def grad_bench(args, prec: str = "fp64"):
    """Gradient of the witness gain on the 256 x 2048, 16 ppc, 2e5-particle,
    20-step workload (blowout driver n_d = 8, u_th = 0.02, checkpoints every
    64 slices), in FP64 or mixed precision (float recorded march and float
    per-particle adjoint arithmetic): time of the plain forward (beam load +
    current + response + 20 pushes + gain), of the recording forward and of
    the reverse pass, each the best of a few runs timed with HIP events."""
    import torch
    from paper_1411_3246_amd import inputs, wake
    p = inputs.gradient_case().replace(prec=prec)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        best = float("inf")
        fn()
        torch.cuda.synchronize()
        for _ in range(args.grad_reps):
            ev[0].record(stream)
            fn()
            ev[1].record(stream)
            ev[1].synchronize()
            best = min(best, ev[0].elapsed_time(ev[1]))
        return best

    sim = wake.Simulation(p)

    def plain():
        sim.load_beam()
        sim.beam_current()
        sim.response()
        sim.push(p.n_steps)
        sim.plan.mean_gain(sim.beam, 1, sim.out[0:1], sim.workspace)

    fwd = timed(plain)
    g_plain = float(sim.out[0].item())
    del sim
    run = wake.GradientRun(p, every=64)
    rec = timed(run.forward)
    g = float(run.out[0].item())
    bwd = timed(run.backward)
    grad = run.grad.cpu().tolist()
    counters = wake.counters_dict(run.counters)
    del run
    torch.cuda.empty_cache()
    return {
        "workload": p.name, "n_d": p.bunches[0].n_peak, "u_th": p.u_th, "n_steps": p.n_steps,
        "checkpoint_every": 64, "precision": prec,
        "forward_ms": fwd, "recording_forward_ms": rec, "backward_ms": bwd,
        "adjoint_over_forward": bwd / fwd, "gradient_over_forward": (rec + bwd) / fwd,
        "objective": g, "objective_plain": g_plain,
        "gradient": dict(zip(inputs.THETA_NAMES, grad)),
        "counters": counters,
    }


def convergence_bench(args):
    """Convergence-scale runs, each against the same two-bunch workload at
    512 radial cells and a quarter of the slices (the headline grid).

    For the cylindrical (2048 x 16384) and slab (2048 x 8192, x <= 8) grids
    with 64 particles per cell and 4e6 beam particles: the first plasma
    response is compared with the 512-cell one on the coarse nodes (every
    4th node and slice): ||dE_z|| / ||E_z|| and the on-axis E_z spike behind
    the drive at both resolutions; then `--steps` pipelined cycles are timed
    (HIP events)."""
    import numpy as np
    import torch
    from paper_1411_3246_amd import inputs, wake
    out = {}
    for geom in ("cyl", "slab"):
        fine = inputs.convergence_cyl() if geom == "cyl" else inputs.convergence_slab()
        coarse = fine.replace(n_r=fine.n_r // 4, n_xi=fine.n_xi // 4, ppc=16, n_beam=1_000_000,
                              n_drive=int(round(1_000_000 / 1.3)), name=f"{fine.name}-coarse")
        ez = {}
        peak = {}
        for tag, p in (("coarse", coarse), ("fine", fine)):
            sim = wake.Simulation(p)
            sim.load_beam()
            sim.run_cycle(1)
            torch.cuda.synchronize()
            ez[tag] = sim.fields[1].double().cpu().numpy()
            peak[tag] = sim.ez_peak(3.0)
            print(f"# {geom} {tag} first response done", file=sys.stderr, flush=True)
            del sim
            torch.cuda.empty_cache()
        ef = ez["fine"][::4, ::4]
        ec = ez["coarse"]
        rel = float(np.linalg.norm(ef - ec) / np.linalg.norm(ec))
        sim = wake.Simulation(fine.replace(n_steps=args.steps))
        sim.load_beam()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(torch.cuda.current_stream())
        sim.run_cycle(args.steps)
        ev[1].record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        upd = fine.updates_per_response() * args.steps
        out[geom] = {
            "workload": fine.name, "n_r": fine.n_r, "n_xi": fine.n_xi, "ppc": fine.ppc, "r_max": fine.r_max,
            "n_beam": fine.n_beam, "steps": args.steps, "cycle_ms": ms, "updates": upd,
            "updates_per_s": upd / (ms * 1e-3),
            "ez_rel_l2_vs_512": rel, "ez_spike_fine": peak["fine"], "ez_spike_512": peak["coarse"],
            "witness_gain": sim.witness_gain(), "counters": sim.counters_dict(),
            "roofline": roofline(upd, ms, measured_traffic(CONV_COUNTERS[geom], upd),
                                 "k_cycle (large grid)", 1),
            "group": sim.plan.cycle_group(args.steps),
        }
        print(f"# {geom} cycle {ms:.0f} ms", file=sys.stderr, flush=True)
        del sim
        torch.cuda.empty_cache()
    return out


def te_scan_bench(args):
    """The Table I driver (fixed beam) in a plasma at T_e = 0, 1, 2, 5, 10,
    20, 30 eV on a 256 x 2800 grid over xi in [0, 14), and the slice-spacing
    ladder dxi = 0.02 ... 0.00125 for a cold and a 5 eV plasma: every instance
    in one batched launch; the on-axis E_z spike behind the drive and the
    on-axis E_z at the witness centre per instance."""
    import torch
    from paper_1411_3246_amd import inputs, wake
    probs = inputs.te_scan_instances(ladder=(700, 1400, 2800, 5600, 11200))
    scan = wake.Scan(probs)
    scan.threads = 1024
    scan.run()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(torch.cuda.current_stream())
    scan.run()
    ev[1].record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    rows = []
    xi_from = 3.5 * inputs.TABLE1["sigma_zd"] + 1.0
    for q, pl, f in zip(probs, scan.plans, scan.fields):
        pl.ez_peak(f, xi_from, out)
        k = int((q.bunches[1].xi_c - q.xi_min) / q.dxi)
        rows.append({"T_e_eV": round((q.u_th ** 2) * inputs.MC2_EV, 3), "dxi": q.dxi, "n_xi": q.n_xi,
                     "ez_spike": float(out.item()), "ez_witness_axis": float(f[1, k, 0].item())})
    return {"ms": ev[0].elapsed_time(ev[1]), "instances": len(probs), "updates": scan.updates,
            "counters": wake.counters_dict(scan.counters), "rows": rows}


def table1_trajectories(te: float) -> dict:
    """Plasma electron trajectories behind the Table I driver (fixed beam,
    256 x 2800, 16 ppc, FP64), every macroparticle recorded at every slice,
    the width in xi over which the expelled electrons come back to the axis
    (axis_crossings), and the E_r - B_theta field around the on-axis E_z
    spike.  W = E_r - B_theta is
    the radial force on a beam electron up to its sign (F_r = -W): W < 0 near
    the axis at the spike means a defocusing region."""
    import numpy as np
    import torch
    from paper_1411_3246_amd import diagnostics, inputs, wake
    p = inputs.facet_table1(te, n_r=256, n_xi=2800, ppc=16, prec="fp64")
    sim = wake.Simulation(p)
    sim.beam_current()
    stride = 1
    tr = sim.response_traj(stride).cpu().numpy()
    f = sim.fields.double().cpu().numpy()
    torch.cuda.synchronize()
    xi = p.xi_min + np.arange(p.n_xi) * p.dxi
    h = p.r_max / p.n_r
    xd = p.bunches[0].xi_c
    k_from = int(np.searchsorted(xi, xd + 1.0))
    ks = k_from + int(np.argmin(f[1, k_from:, 0]))
    crossing = diagnostics.axis_crossings(tr, xi, h, xd)
    w_axis = f[3, ks, 1:6]
    out = {
        "workload": p.name, "stride": stride, "recorded": int(tr.shape[1]),
        "spike_ez": float(f[1, ks, 0]), "spike_xi": float(xi[ks]),
        "axis_crossing": crossing,
        "W_at_spike_r_h_to_5h": [float(v) for v in w_axis],
        "W_map": {"xi": [float(xi[k]) for k in range(ks - 40, ks + 41, 10)],
                  "r": [float(j * h) for j in (1, 2, 4, 8, 16, 32)],
                  "W": [[float(f[3, k, j]) for j in (1, 2, 4, 8, 16, 32)] for k in range(ks - 40, ks + 41, 10)]},
        "spike_in_defocusing_region": bool(np.all(w_axis < 0.0)),
        "counters": sim.counters_dict(),
    }
    del sim
    torch.cuda.empty_cache()
    return out


def table1_beam_bench(args):
    """The Table I beam (1e6 macroparticles, zero emittance) evolved over
    1.14 m of plasma at 5e16 cm^-3 (1203 steps of 40 / omega_p) by the
    pipelined cycle, in a cold and in a 5 eV plasma (256 x 2800 grid):
    the witness energy spectrum (wk_gain_histogram, 0.5 GeV bins) with its
    mean and its peak, the spread, the drive's mean energy change and the
    on-axis spike; where the particles that leave the window are, by bunch;
    and the plasma trajectories and E_r - B_theta map of the fixed-beam
    response (table1_trajectories)."""
    import numpy as np
    import torch
    from paper_1411_3246_amd import inputs, wake
    out = {}
    gev = 0.51099895e-3
    n_bins, lo_gev, hi_gev = 80, -10.0, 30.0
    for te in (0.0, 5.0):
        p = inputs.facet_table1_beam(te)
        sim = wake.Simulation(p)
        sim.load_beam()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(torch.cuda.current_stream())
        sim.run_cycle(p.n_steps)
        ev[1].record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        hist = sim.gain_histogram(1, n_bins, lo_gev / gev, hi_gev / gev).cpu().numpy()
        b = {k: sim.beam[k].cpu().numpy() for k in ("x", "y", "xi", "px", "py", "pz", "gamma_init", "tag")}
        dg = np.sqrt(1 + b["px"] ** 2 + b["py"] ** 2 + b["pz"] ** 2) - b["gamma_init"]
        wit = b["tag"] == 1
        r = np.hypot(b["x"], b["y"])
        centres = lo_gev + (np.arange(n_bins) + 0.5) * (hi_gev - lo_gev) / n_bins
        peak = int(np.argmax(hist[1:-1]))
        outside = {}
        for name, sel in (("drive", ~wit), ("witness", wit)):
            outside[name] = {"particles": int(sel.sum()),
                             "beyond_r_max": int(np.sum(sel & (r > p.r_max))),
                             "behind_window": int(np.sum(sel & (b["xi"] >= p.xi_max))),
                             "ahead_of_window": int(np.sum(sel & (b["xi"] < p.xi_min)))}
        c = sim.counters_dict()
        out[f"{te:g}eV"] = {
            "workload": p.name, "steps": p.n_steps, "ms": ms,
            "updates_per_s": p.updates_per_response() * p.n_steps / (ms * 1e-3),
            "witness_mean_gain_GeV": sim.witness_gain() * gev,
            "witness_gain_std_GeV": float(dg[wit].std()) * gev,
            "witness_spectrum": {"bins_GeV": [lo_gev, hi_gev, n_bins], "underflow": int(hist[0]),
                                 "overflow": int(hist[-1]), "counts": [int(v) for v in hist[1:-1]],
                                 "peak_GeV": float(centres[peak])},
            "witness_p95_gain_GeV": float(np.quantile(dg[wit], 0.95)) * gev,
            "drive_mean_dgamma": float(dg[~wit].mean()), "ez_spike_last": sim.ez_peak(6.04),
            "outside_window_at_end": outside,
            "counters": c}
        print(f"# table1 beam {te:g} eV done", file=sys.stderr, flush=True)
        del sim
        torch.cuda.empty_cache()
        out[f"{te:g}eV"]["trajectories"] = table1_trajectories(te)
        print(f"# table1 trajectories {te:g} eV done", file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "the multi-GPU layout is a design note, not an implementation", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1411_3246_amd import inputs, wake

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # a plain 1 GiB device copy: the reference that HBM counter runs
        # scale FETCH_SIZE and WRITE_SIZE by
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        bcopy = torch.empty_like(a)
        bcopy.copy_(a)
        torch.cuda.synchronize()
        del a, bcopy
    if args.workload == "convergence":
        conv = convergence_bench(args)
        upd = sum(v["updates"] for v in conv.values())
        ms = sum(v["cycle_ms"] for v in conv.values())
        rec = {
            "metric": "plasma particle-slice updates/s at 1 GPU", "value": upd / (ms * 1e-3),
            "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": 0,
            "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
            "config": {"workload": "convergence-2048-cells (cylindrical 2048x16384 + slab 2048x8192)",
                       "ppc": 64, "n_beam": 4_000_000, "beam_steps_timed": args.steps},
            "convergence": conv}
        if not args.no_cpu:
            # the FP64 oracle on the first 192 slices of each grid's first
            # response, extrapolated linearly to a whole response and to the
            # timed steps (a response of these grids takes minutes on a core)
            cb = {}
            for geom, fine in (("cyl", inputs.convergence_cyl()), ("slab", inputs.convergence_slab())):
                r = cpu_baseline(fine, 192 / fine.n_xi)
                per_resp = fine.n_plasma * (fine.n_xi - 1) / r["value"]
                r["extrapolated"] = True
                r["extrapolated_s_per_response"] = per_resp
                r["extrapolated_s_for_timed_steps"] = per_resp * args.steps
                cb[geom] = r
            rec["cpu_baseline"] = cb
        print(json.dumps(rec), flush=True)
        return
    if args.workload == "table1-beam":
        tb = table1_beam_bench(args)
        upd = sum(v["updates_per_s"] * v["ms"] * 1e-3 for v in tb.values())
        ms = sum(v["ms"] for v in tb.values())
        print(json.dumps({
            "metric": "plasma particle-slice updates/s at 1 GPU", "value": upd / (ms * 1e-3),
            "unit": "updates/s", "n_gpus": 1, "steps": next(iter(tb.values()))["steps"], "warmup": 0,
            "ms_per_step": ms / sum(v["steps"] for v in tb.values()), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64", "data": "synthetic",
            "config": {"workload": "table1-beam-1.14m (256x2800, 16 ppc, 1e6 beam, cold and 5 eV)"},
            "table1_beam": tb}), flush=True)
        return
    if args.workload == "te-scan":
        ts = te_scan_bench(args)
        print(json.dumps({
            "metric": "plasma particle-slice updates/s at 1 GPU", "value": ts["updates"] / (ts["ms"] * 1e-3),
            "unit": "updates/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": ts["ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32/f64",
            "data": "synthetic", "config": {"workload": "table1-temperature-and-dxi-scan (256 cells, fixed beam)"},
            "te_scan": ts}), flush=True)
        return
    p = inputs.blowout_response().replace(n_steps=args.steps)
    sim = wake.Simulation(p, threads=args.threads)
    group = sim.plan.cycle_group(args.steps) if args.mode == "pipelined" else sim.plan.group
    stream = torch.cuda.current_stream()
    upd_per_step = p.updates_per_response()

    def run(n, ev=None):
        if args.mode == "pipelined":
            if ev is not None:
                ev[0].record(stream)
            sim.run_cycle(n)
            if ev is not None:
                ev[1].record(stream)
        else:
            t = 0.0
            for _ in range(n):
                sim.beam_current()
                sim.plan.init_plasma(sim.plasma, sim.plasma_draws)
                if ev is not None:
                    ev[0].record(stream)
                sim.plan.plasma_response(sim.plasma, sim.jb, sim.fields, sim.workspace, sim.counters)
                if ev is not None:
                    ev[1].record(stream)
                    torch.cuda.synchronize()
                    t += ev[0].elapsed_time(ev[1])
                sim.push(1)
            return t
        return None

    sim.load_beam()
    if args.warmup > 0:
        run(args.warmup)
    torch.cuda.synchronize()
    sim.load_beam()                       # the timed run starts from the loaded beam
    wake.zero_counters(sim.counters)
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kt = run(args.steps, ev)
    sim.plan.mean_gain(sim.beam, 1, sim.out[0:1], sim.workspace)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if args.mode == "pipelined":
        kernel_ms = ev[0].elapsed_time(ev[1])
        kernel, launches = "k_cycle", 1
    else:
        kernel_ms = kt
        kernel, launches = "k_march", args.steps
    updates = upd_per_step * args.steps
    value = updates / elapsed
    counters = sim.counters_dict()
    gain = float(sim.out[0].item())
    traffic = measured_traffic(CYCLE_COUNTERS, updates) if args.mode == "pipelined" else None
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
                   "dt": p.dt, "mode": args.mode,
                   "precision": "FP32 bulk; FP64 solves, deposit accumulation and xi integration",
                   "march_threads": sim.plan.threads, "group": group},
        "roofline": roofline(updates, kernel_ms, traffic, kernel, launches),
        "diagnostics": {"witness_mean_gain_gamma": gain, "counters": counters},
    }
    if args.mode == "pipelined":
        line["beam_push"] = push_bench(sim, p)
    if not args.no_scan:
        sc = scan_bench(args, lambda row: print(f"# tuner {row}", file=sys.stderr, flush=True))
        line["batched_scan"] = sc
        line["batched_speedup"] = sc["batched_speedup"]
        line["batched_updates_per_s"] = sc["batched_updates_per_s"]
    if not args.no_grad:
        gr = grad_bench(args, "fp64")
        gm = grad_bench(args, "mixed")
        line["gradient"] = gr
        line["gradient_mixed"] = gm
        line["adjoint_over_forward"] = gm["adjoint_over_forward"]
        line["adjoint_over_forward_fp64"] = gr["adjoint_over_forward"]
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
