"""Launch-shape autotuner.

Two choices are tuned by timing the real kernels with HIP events on the
launch stream, and cached:

* A standalone response (wk_plasma_response): the workgroup size (256, 512
  or 1024 threads) and the group of workgroups that marches it (1..16).  The
  choice depends on the grid (n_r), the particles per cell, the precision and
  the geometry and temperature class.  It is cached per such class, measured
  on the first slices of the problem's window: the per-slice work (push,
  deposit, solves, exchanges) does not depend on where the slice is.  The
  pipelined cycle keeps its own choice, which also weighs how many responses
  run at once.
* The batched scan: the schedule of its one persistent launch, i.e. the most
  particles a workgroup may hold (which sets how many workgroups march each
  instance and the launch shape that fits the largest share: 8192 the
  1024x8 shape, 4096 the 512x8, 2048 the 512x4) and the workgroups per
  compute unit; cached per batch (the multiset of its instance classes).

Results depend on the choice only through the summation order of the LDS
deposits.  The cache is a JSON file, by default
~/.cache/paper_1411_3246_amd/tune.json; each entry keeps the timings it was
chosen from and the device it was measured on.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

# (member cap, workgroups per CU; 0 = as many as fit)
CANDIDATES: Tuple[Tuple[int, int], ...] = ((8192, 0), (4096, 0), (4096, 1), (2048, 0), (2048, 1))
RESPONSE_THREADS: Tuple[int, ...] = (256, 512, 1024)
RESPONSE_GROUPS: Tuple[int, ...] = (1, 2, 4, 8, 16)


def default_cache_path() -> str:
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1411_3246_amd", "tune.json")


class TuneCache:
    """Tuned choices by key, kept in a JSON file (written on every store)."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or default_cache_path()
        self.entries: Dict[str, dict] = {}
        try:
            with open(self.path) as f:
                self.entries = json.load(f)
        except (OSError, ValueError):
            self.entries = {}

    def get(self, key: str) -> Optional[dict]:
        return self.entries.get(key)

    def put(self, key: str, entry: dict) -> None:
        self.entries[key] = entry
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def class_key(p) -> str:
    """The class a tuned response choice is cached for."""
    return f"{p.geom}-nr{p.n_r}-ppc{p.ppc}-{p.prec}-{'warm' if p.u_th > 0 else 'cold'}"


def _device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"


def time_response(p, threads: int, group: int, repeats: int = 2) -> float:
    """Milliseconds of one standalone response of problem p with a shape."""
    import torch
    from . import wake
    sim = wake.Simulation(p, threads=threads, group=group)
    sim.beam_current()
    stream = torch.cuda.current_stream()
    sim.response()                               # warm-up (kernel attributes, caches)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(repeats):
        sim.plan.init_plasma(sim.plasma, sim.plasma_draws)
        start.record(stream)
        sim.plan.plasma_response(sim.plasma, sim.jb, sim.fields, sim.workspace, sim.counters)
        end.record(stream)
        end.synchronize()
        best = min(best, start.elapsed_time(end))
    del sim
    return best


def tune_response(p, cache: Optional[TuneCache] = None, window: int = 128,
                  threads: Sequence[int] = RESPONSE_THREADS, groups: Sequence[int] = RESPONSE_GROUPS,
                  force: bool = False, log=None) -> Tuple[Tuple[int, int], List[dict], bool]:
    """(threads, group) of the fastest standalone response for p's class,
    timed on the first `window` slices of p (same slice spacing); from the
    cache when the class is there (unless force).  Returns the choice, the
    timing table and whether it came from the cache."""
    key = class_key(p)
    if cache is not None and not force:
        hit = cache.get(key)
        if hit is not None:
            return (hit["threads"], hit["group"]), hit.get("table", []), True
    n = min(window, p.n_xi)
    q = p.replace(n_xi=n, xi_max=p.xi_min + n * p.dxi, n_beam=0, n_drive=0, name=f"{p.name}-tune")
    table = []
    for t in threads:
        for g in groups:
            if g > p.n_r:
                continue
            ms = time_response(q, t, g)
            row = {"threads": t, "group": g, "ms_per_slice": ms / n}
            table.append(row)
            if log is not None:
                log(row)
    best = min(table, key=lambda r: r["ms_per_slice"])
    choice = (best["threads"], best["group"])
    if cache is not None:
        cache.put(key, {"threads": choice[0], "group": choice[1], "table": table, "window": n,
                        "device": _device_name()})
    return choice, table, False


def cached_response(p, cache: TuneCache) -> Optional[Tuple[int, int]]:
    """The cached (threads, group) of p's class, or None if the class has not
    been tuned: pass it to Simulation / Plan at construction (the workspace
    size depends on it)."""
    hit = cache.get(class_key(p))
    return None if hit is None else (hit["threads"], hit["group"])


def time_scan(scan, member_cap: int, wg_per_cu: int, repeats: int = 1) -> float:
    """Milliseconds of one batched pass (plasma loads + march) with a
    schedule."""
    import torch
    stream = torch.cuda.current_stream()
    scan.set_member_cap(member_cap)
    scan.threads, scan.wg_per_cu = 0, wg_per_cu
    scan.run()                                   # warm-up (kernel attributes, caches)
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(repeats):
        start.record(stream)
        scan.run()
        end.record(stream)
        end.synchronize()
        best = min(best, start.elapsed_time(end))
    return best


def scan_key(problems: Sequence) -> str:
    """The batch a tuned scan shape is cached for: the multiset of its
    instance classes and window lengths."""
    items = sorted(f"{class_key(q)}-nxi{q.n_xi}" for q in problems)
    return "scan-" + hashlib.sha256("\n".join(items).encode()).hexdigest()[:20]


def tune_scan(scan, candidates: Optional[Iterable[Tuple[int, int]]] = None,
              repeats: int = 1, log=None, cache: Optional[TuneCache] = None,
              force: bool = False) -> Tuple[Tuple[int, int], List[dict]]:
    """Time every candidate (member cap, workgroups per CU) on `scan`, set
    the fastest on it and return it with the table of timings; with a cache,
    a batch tuned before takes its cached schedule (table marked cached)."""
    key = scan_key(scan.problems)
    if cache is not None and not force:
        hit = cache.get(key)
        if hit is not None:
            scan.set_member_cap(hit["member_cap"])
            scan.threads, scan.wg_per_cu = 0, hit["wg_per_cu"]
            return (hit["member_cap"], hit["wg_per_cu"]), [dict(r, cached=True) for r in hit.get("table", [])]
    table = []
    for cap, per_cu in (candidates or CANDIDATES):
        ms = time_scan(scan, cap, per_cu, repeats)
        row = {"member_cap": cap, "wg_per_cu": per_cu, "ms": ms, "workgroups": sum(scan.groups)}
        table.append(row)
        if log is not None:
            log(row)
    best = min(table, key=lambda r: r["ms"])
    scan.set_member_cap(best["member_cap"])
    scan.threads, scan.wg_per_cu = 0, best["wg_per_cu"]
    if cache is not None:
        cache.put(key, {"member_cap": best["member_cap"], "wg_per_cu": best["wg_per_cu"], "table": table,
                        "device": _device_name()})
    return (best["member_cap"], best["wg_per_cu"]), table
