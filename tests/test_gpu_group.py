"""A response marched by a group of workgroups (deposits summed between
them in a fixed order), through the C ABI, against the FP64 oracle.

Bars: FP64 fields and particle state within 1e-10 of the oracle's scale per
field on non-chaotic cases; two runs of the same launch agree to 1e-13 (the
LDS deposits are the only order-dependent sums, so this bounds run-to-run
differences and would expose a missing barrier); the pipelined cycle with a
forced group against the oracle's sequential cycle.
"""
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
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def _response(W, p, jb, group=None, threads=None):
    import torch
    sim = W.Simulation(p, threads=threads, group=group)
    sim.jb.copy_(torch.from_numpy(np.ascontiguousarray(jb)))
    sim.response()
    torch.cuda.synchronize()
    return sim


def _moderate():
    return inputs.facet_two_bunch(n_r=96, n_xi=600, ppc=8, u_th=0.02, n_d=1.0, n_beam=0, prec="fp64",
                                  name="group-moderate")


@pytest.mark.parametrize("group", [1, 2, 3, 7, 16])
def test_group_fp64_matches_oracle(O, W, group):
    """Warm, moderate two-bunch driver, 96 cells x 8 per cell, FP64, the
    response marched by `group` workgroups: every field and the particle
    state within 1e-10 of the oracle."""
    p = _moderate()
    print(f"case {p.name} group={group}", flush=True)
    ref = O.response(p, inputs.plasma_draws(p))
    sim = _response(W, p, ref["jb"], group=group)
    assert sim.plan.group == group
    f = _np(sim.fields)
    errs = [_rel(f[i], ref["fields"][i]) for i in range(4)]
    print("group", group, "max rel error psi, E_z, B, W:", errs, flush=True)
    assert max(errs) <= 1e-10, errs
    for k in ("x", "y", "px", "py"):
        assert _rel(_np(sim.plasma[k]), ref["state"][k]) <= 1e-10, k
    c = sim.counters_dict()
    assert c["pipeline_abort"] == 0 and c["nonfinite"] == 0
    assert c["wall"] == int(ref["counters"][1]) and c["d_clamp"] == int(ref["counters"][0])


@pytest.mark.parametrize("group", [2, 5])
def test_group_cold_weak_bunch(O, W, group):
    """Cold plasma, weak single bunch (128 x 512, 4 per cell), FP64, split
    over `group` workgroups: within 1e-10."""
    p = inputs.weak_single_bunch()
    ref = O.response(p, None)
    sim = _response(W, p, ref["jb"], group=group)
    f = _np(sim.fields)
    for i in range(4):
        assert _rel(f[i], ref["fields"][i]) <= 1e-10, i


@pytest.mark.parametrize("threads,group", [(256, 1), (512, 1), (1024, 1), (256, 4), (512, 4)])
def test_repeatable(W, threads, group):
    """Two runs of the same launch agree to 1e-13 relative per field: the
    warm 32-cell case with one particle per thread at 256 threads and the
    moderate case."""
    import torch
    cases = [inputs.facet_two_bunch(n_r=32, n_xi=200, ppc=8, sep=3.5, u_th=0.02, n_beam=0, prec="fp64",
                                    name="warm-32"), _moderate()]
    for p in cases:
        if group > p.n_r:
            continue
        print(f"case {p.name} threads={threads} group={group}", flush=True)
        out = []
        for _ in range(2):
            sim = W.Simulation(p, threads=threads, group=group)
            sim.beam_current()
            sim.response()
            torch.cuda.synchronize()
            out.append(_np(sim.fields))
        for i in range(4):
            assert _rel(out[0][i], out[1][i]) <= 1e-13, (p.name, i)


def _beam_np(sim):
    return {k: _np(sim.beam[k]) for k in ("x", "y", "px", "py", "pz", "xi")}


@pytest.mark.parametrize("group", [1, 2, 3])
def test_cycle_group_matches_oracle(O, W, group):
    """The pipelined cycle with `group` workgroups per response (each with
    its own beam subset and bins), FP64, 5 steps: the beam, the last fields
    and the witness gain against the oracle's sequential cycle."""
    import torch
    p = inputs.facet_two_bunch(n_r=96, n_xi=400, ppc=8, u_th=0.02, n_d=1.0, n_beam=6000, n_steps=5,
                               prec="fp64", name="cycle-group")
    print(f"case {p.name} group={group}", flush=True)
    pipe = W.Simulation(p, group=group)
    assert pipe.plan.cycle_group(p.n_steps) == group
    pipe.load_beam()
    pipe.run_cycle(p.n_steps)
    torch.cuda.synchronize()
    c = W.read_counters(pipe.counters)
    assert c["pipeline_abort"] == 0 and c["beam_bin"] == 0 and c["beam_order"] == 0
    ref = O.cycle(p, inputs.plasma_draws(p), inputs.beam_draws(p), p.n_steps)
    a = _beam_np(pipe)
    for k in ("x", "y", "px", "py", "pz", "xi"):
        scale = max(1.0, np.max(np.abs(ref["beam"][k])))
        assert np.max(np.abs(a[k] - ref["beam"][k])) <= 1e-10 * scale, k
    assert _rel(_np(pipe.fields), ref["fields"]) <= 1e-10
    assert pipe.witness_gain() == pytest.approx(ref["witness_gain"], rel=1e-10)


@pytest.mark.parametrize("group", [1, 4])
def test_cycle_bunch_straddles_window_end(O, W, group):
    """A witness bunch that reaches past xi_max, so that the last xi bin and
    the outside bin hold beam particles in every step (the bins that the
    next response rewrites while the previous one finishes): pipelined cycle
    against the oracle's sequential cycle, FP64."""
    import torch
    p = inputs.facet_two_bunch(n_r=64, n_xi=300, ppc=4, u_th=0.02, n_d=1.0, sep=6.8, n_beam=8000,
                               n_steps=6, prec="fp64", name="straddle")
    print(f"case {p.name} group={group}", flush=True)
    pipe = W.Simulation(p, group=group)
    pipe.load_beam()
    xi = _np(pipe.beam["xi"])
    dxi = p.dxi
    assert np.sum(xi >= p.xi_max) > 0 and np.sum((xi >= p.xi_max - dxi) & (xi < p.xi_max)) > 0
    pipe.run_cycle(p.n_steps)
    torch.cuda.synchronize()
    c = W.read_counters(pipe.counters)
    assert c["pipeline_abort"] == 0 and c["beam_bin"] == 0 and c["beam_order"] == 0
    ref = O.cycle(p, inputs.plasma_draws(p), inputs.beam_draws(p), p.n_steps)
    a = _beam_np(pipe)
    for k in ("x", "pz", "xi"):
        scale = max(1.0, np.max(np.abs(ref["beam"][k])))
        assert np.max(np.abs(a[k] - ref["beam"][k])) <= 1e-10 * scale, k
    assert pipe.witness_gain() == pytest.approx(ref["witness_gain"], rel=1e-10)


@pytest.mark.parametrize("group,ppc", [(1, 4), (2, 4), (1, 80)], ids=["group1", "group2", "group1-16-per-thread"])
def test_cycle_movers_and_dense_bins(O, W, group, ppc):
    """A slow beam (gamma0 = 5, dt = 1: a twelfth of a slice per step) so
    that particles change xi bin in every step, and bins of about 1500
    particles per workgroup at 256 threads (beyond the chunks whose movers
    the bin pass keeps in registers): pipelined cycle against the oracle's
    sequential cycle, FP64, no bin escapes or order losses.  With 80 ppc (5120
    plasma particles) one workgroup marches 16 particles per thread, the
    shape that keeps one chunk of movers in registers."""
    import torch
    base = inputs.facet_two_bunch(n_r=32 if ppc == 4 else 64, n_xi=40, ppc=ppc, u_th=0.02, n_d=0.5,
                                  n_beam=60000, n_steps=4, prec="fp64", name="movers")
    p = base.replace(gamma0=5.0, dt=1.0)
    print(f"case {p.name} group={group}", flush=True)
    pipe = W.Simulation(p, threads=256, group=group)
    assert pipe.plan.cycle_group(p.n_steps) == group
    pipe.load_beam()
    xi0 = _np(pipe.beam["xi"])
    k0 = np.floor((xi0 - p.xi_min) / p.dxi)
    per_bin = np.bincount(k0[(k0 >= 0) & (k0 < p.n_xi)].astype(int), minlength=p.n_xi)
    assert per_bin.max() / group > 4 * 256
    pipe.run_cycle(p.n_steps)
    torch.cuda.synchronize()
    c = W.read_counters(pipe.counters)
    assert c["pipeline_abort"] == 0 and c["beam_bin"] == 0 and c["beam_order"] == 0
    moved = np.floor((_np(pipe.beam["xi"]) - p.xi_min) / p.dxi) != k0
    print("particles that changed bin:", int(moved.sum()), flush=True)
    assert moved.sum() > 0.1 * p.n_beam
    ref = O.cycle(p, inputs.plasma_draws(p), inputs.beam_draws(p), p.n_steps)
    a = _beam_np(pipe)
    for k in ("x", "y", "px", "pz", "xi"):
        scale = max(1.0, np.max(np.abs(ref["beam"][k])))
        assert np.max(np.abs(a[k] - ref["beam"][k])) <= 1e-10 * scale, k
    assert pipe.witness_gain() == pytest.approx(ref["witness_gain"], rel=1e-10)
