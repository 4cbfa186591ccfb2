"""Batched parameter scan on the GPU: one persistent launch of many uneven
fixed-beam instances, its launch shapes, the autotuner and HIP-graph replay,
each checked against the FP64 oracle (or, for shape and replay variants,
against the eager batched result) through the C ABI."""
import numpy as np
import pytest

from paper_1411_3246_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


@pytest.fixture(scope="module")
def W():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1411_3246_amd import wake
    wake.lib()
    return wake


def _np(t):
    return t.detach().cpu().double().numpy()


def _rel(a, b):
    den = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (den if den > 0 else 1.0)


def _l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def small_scan(n=10, prec="fp64", seed=3):
    """Scan instances with the scan's parameter ranges but grids the oracle
    finishes in seconds (ragged n_r, n_xi and ppc; warm and cold)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        u_th = 0.0 if i % 4 == 0 else float(rng.uniform(0.0, 0.05))
        out.append(inputs.facet_two_bunch(
            n_r=int(rng.choice([16, 24, 40, 64])), n_xi=int(rng.integers(64, 300)),
            ppc=int(rng.choice([2, 4, 6, 8])), u_th=u_th, sep=float(rng.uniform(3.0, 6.0)),
            n_beam=0, n_steps=0, prec=prec, n_d=1.0, seed=seed * 1000 + i, name=f"small-scan-{i}"))
    return out


def _oracle(O, q):
    return O.response(q, inputs.plasma_draws(q))


@pytest.fixture(scope="module")
def refs(O):
    return [_oracle(O, q) for q in small_scan()]


def test_scan_matches_oracle_every_shape(O, W, refs):
    """Every launch shape the tuner may pick gives the oracle's fields."""
    import torch
    from paper_1411_3246_amd import autotune
    scan = W.Scan(small_scan())
    shapes = [(0, threads, per_cu) for threads, per_cu in ((256, 2), (256, 4), (512, 1), (512, 2), (1024, 1))]
    shapes += [(cap, 0, per_cu) for cap, per_cu in autotune.CANDIDATES] + [(64, 0, 0)]
    for cap, threads, per_cu in shapes:
        print(f"schedule cap={cap} threads={threads} wg_per_cu={per_cu}", flush=True)
        scan.set_member_cap(cap)
        scan.threads, scan.wg_per_cu = threads, per_cu
        for f in scan.fields:
            f.zero_()
        scan.run()
        torch.cuda.synchronize()
        for q, f, ref in zip(scan.problems, scan.fields, refs):
            assert _rel(_np(f), ref["fields"]) <= 1e-10, (q.name, cap, threads, per_cu)
        if cap == 64:
            # members of at most 64 particles where 16 workgroups and n_r allow
            for q, g in zip(scan.problems, scan.groups):
                assert min(16, q.n_r, -(-q.n_plasma // 64)) <= g <= min(16, q.n_r), (q.name, g)
    c = W.counters_dict(scan.counters)
    assert c["nonfinite"] == 0


def test_scan_standalone_equals_batched(O, W, refs):
    import torch
    scan = W.Scan(small_scan())
    for i in range(len(scan.problems)):
        scan.run_one(i)
    torch.cuda.synchronize()
    for q, f, ref in zip(scan.problems, scan.fields, refs):
        assert _rel(_np(f), ref["fields"]) <= 1e-10, q.name


def test_autotuner_picks_a_valid_shape(O, W, refs):
    import torch
    from paper_1411_3246_amd import autotune
    scan = W.Scan(small_scan())
    best, table = autotune.tune_scan(scan)
    assert best in autotune.CANDIDATES and scan.member_cap == best[0]
    assert len(table) == len(autotune.CANDIDATES) and all(r["ms"] > 0 for r in table)
    # the schedules differ: smaller members mean more workgroups
    work = {r["member_cap"]: r["workgroups"] for r in table}
    assert work[2048] >= work[4096] >= work[8192]
    scan.run()
    torch.cuda.synchronize()
    for q, f, ref in zip(scan.problems, scan.fields, refs):
        assert _rel(_np(f), ref["fields"]) <= 1e-10, q.name


def test_graph_replays_match_eager(O, W, refs):
    """The whole pass (plasma loads, queue reset, batched march) captured in
    a HIP graph: several replays, with eager work and synchronizations in
    between, each equal to the oracle."""
    import torch
    scan = W.Scan(small_scan())
    scan.capture()
    other = W.Scan(small_scan(n=3, seed=11))
    for rep in range(3):
        print(f"graph replay {rep}", flush=True)
        for f in scan.fields:
            f.fill_(7.0)
        scan.replay()
        torch.cuda.synchronize()
        for q, f, ref in zip(scan.problems, scan.fields, refs):
            assert _rel(_np(f), ref["fields"]) <= 1e-10, (rep, q.name)
        other.run()                           # unrelated eager work between replays
        torch.cuda.synchronize()


def test_full_scan_sampled_against_oracle(O, W):
    """The 256-instance scan at its full sizes in mixed precision, launched as
    the benchmark launches it; the smallest instances are recomputed by the
    FP64 oracle one by one (E_z within 1e-3), all instances finite."""
    import torch
    probs = inputs.scan_instances(256)
    scan = W.Scan(probs)
    scan.run()
    torch.cuda.synchronize()
    c = W.counters_dict(scan.counters)
    assert c["nonfinite"] == 0
    order = sorted(range(len(probs)), key=lambda i: probs[i].updates_per_response())
    for i in order[:3]:
        q = probs[i]
        print(f"sampled instance {q.name} {q.n_r}x{q.n_xi} ppc={q.ppc} u_th={q.u_th:.4f}", flush=True)
        ref = _oracle(O, q.replace(prec="fp64"))
        f = _np(scan.fields[i])
        assert _l2(f[1], ref["fields"][1]) <= 1e-3, q.name
        assert _l2(f[0], ref["fields"][0]) <= 1e-3, q.name
    # the largest instance: properties that hold at any size
    big = order[-1]
    f = _np(scan.fields[big])
    assert np.all(np.isfinite(f))
    # first slice: the plasma is unperturbed, so psi, E_z and W vanish there
    for k in (0, 1, 3):
        assert np.max(np.abs(f[k, 0])) <= 1e-6 * max(np.max(np.abs(f[k])), 1e-30), k


def test_scan_tuning_is_cached(W, tmp_path):
    """A batch tuned once takes its cached shape the next time."""
    from paper_1411_3246_amd import autotune
    cache = autotune.TuneCache(str(tmp_path / "tune.json"))
    scan = W.Scan(small_scan())
    best, table = autotune.tune_scan(scan, candidates=autotune.CANDIDATES[:2], cache=cache)
    assert not any(r.get("cached") for r in table)
    other = W.Scan(small_scan())
    best2, table2 = autotune.tune_scan(other, cache=autotune.TuneCache(cache.path))
    assert best2 == best and (other.member_cap, other.wg_per_cu) == best
    assert all(r["cached"] for r in table2)


def test_response_tuning_per_class(O, W, tmp_path):
    """The standalone response tuned for (n_r, ppc, precision, geometry,
    temperature) on a short window: the choice is cached for the class, a
    second call takes it from the cache, and a response launched with it
    equals the oracle within 1e-10."""
    import torch
    from paper_1411_3246_amd import autotune
    cache = autotune.TuneCache(str(tmp_path / "tune.json"))
    p = inputs.facet_two_bunch(n_r=128, n_xi=200, ppc=8, u_th=0.02, n_d=1.0, n_beam=0, prec="fp64",
                               name="tune-128")
    choice, table, hit = autotune.tune_response(p, cache, window=48, threads=(256, 512), groups=(1, 2, 4))
    print("tuned", choice, table, flush=True)
    assert not hit and len(table) == 6 and all(r["ms_per_slice"] > 0 for r in table)
    again, _, hit = autotune.tune_response(p.replace(n_xi=400, xi_max=p.xi_min + 400 * p.dxi), cache)
    assert hit and again == choice
    assert autotune.cached_response(p, autotune.TuneCache(cache.path)) == choice
    ref = O.response(p, inputs.plasma_draws(p))
    sim = W.Simulation(p, threads=choice[0], group=choice[1])
    sim.jb.copy_(torch.from_numpy(np.ascontiguousarray(ref["jb"])))
    sim.response()
    torch.cuda.synchronize()
    assert (sim.plan.threads, sim.plan.group) == choice
    for i in range(4):
        assert _rel(_np(sim.fields[i]), ref["fields"][i]) <= 1e-10, i


def test_default_schedule_weights_cost_by_grid(W):
    """The library's batch schedule on the 256-instance scan's plans (mixed
    n_r): G_i = max(ceil(n_p / 8192), ceil(cost_i / (total / CUs))) with
    total = sum of n_p n_xi and cost_i = n_p n_xi n_r / (largest n_r),
    clipped to [1, min(16, n_r)]."""
    import ctypes as C
    import math
    import torch
    probs = inputs.scan_instances(256)
    plans = [W.Plan(q) for q in probs]
    handles = (C.c_void_p * len(plans))(*[p.handle for p in plans])
    got = [int(W.lib().wk_batch_group(len(plans), handles, i)) for i in range(len(plans))]
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    total = sum(float(q.n_plasma) * q.n_xi for q in probs)
    nr_max = max(q.n_r for q in probs)
    want = [max(1, min(16, q.n_r, max(math.ceil(q.n_plasma / 8192),
                                      math.ceil(float(q.n_plasma) * q.n_xi * q.n_r / nr_max / (total / cus)))))
            for q in probs]
    assert got == want
    # the weight matters here: a smaller grid gets fewer members than its
    # unweighted cost would give it
    unweighted = [max(1, min(16, q.n_r, max(math.ceil(q.n_plasma / 8192),
                                            math.ceil(float(q.n_plasma) * q.n_xi / (total / cus))))) for q in probs]
    assert sum(got) < sum(unweighted)
    assert all(g == u for g, u, q in zip(got, unweighted, probs) if q.n_r == nr_max)
