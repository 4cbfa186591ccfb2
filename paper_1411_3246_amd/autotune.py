"""Launch-shape autotuner for the batched plasma response.

The batched march runs one instance per workgroup; its speed depends on the
workgroup size (how many particles each thread carries, whether they stay in
registers) and on how many workgroups share a compute unit (latency hiding
against LDS and register pressure).  The tuner times each candidate shape on
the real batch with HIP events on the launch stream and keeps the fastest.
Results depend on the shape only through the summation order of the LDS
deposits.
"""
from __future__ import annotations

from typing import Iterable, List, Optional, Sequence, Tuple

CANDIDATES: Tuple[Tuple[int, int], ...] = ((256, 2), (256, 4), (512, 1), (512, 2), (1024, 1))


def time_scan(scan, threads: int, wg_per_cu: int, repeats: int = 1) -> float:
    """Milliseconds of one batched pass (plasma loads + march) with a shape."""
    import torch
    stream = torch.cuda.current_stream()
    scan.threads, scan.wg_per_cu = threads, wg_per_cu
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


def tune_scan(scan, candidates: Optional[Iterable[Tuple[int, int]]] = None,
              repeats: int = 1, log=None) -> Tuple[Tuple[int, int], List[dict]]:
    """Time every candidate (threads, workgroups per CU) on `scan`, set the
    fastest on it and return it with the table of timings."""
    table = []
    for threads, per_cu in (candidates or CANDIDATES):
        ms = time_scan(scan, threads, per_cu, repeats)
        row = {"threads": threads, "wg_per_cu": per_cu, "ms": ms}
        table.append(row)
        if log is not None:
            log(row)
    best = min(table, key=lambda r: r["ms"])
    scan.threads, scan.wg_per_cu = best["threads"], best["wg_per_cu"]
    return (best["threads"], best["wg_per_cu"]), table
