"""GPU (HIP, gfx950) vs FP64 oracle, through the C ABI.

Tolerances:
  * FP64 plans: max|gpu - oracle| / max|oracle| <= 1e-10 per field (and for
    the particle state), where the oracle's own sensitivity to 1-ulp
    perturbations stays below 1e-12; in the trajectory-crossing blowout the
    bound is ten times that sensitivity envelope.
  * Mixed plans: ||dE_z||_2 / ||E_z||_2 <= 1e-3; the other fields are
    reported with their own bounds.
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
    return np.max(np.abs(a - b)) / (den if den > 0 else 1.0)


def _l2(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def gpu_response(W, p, jb=None, threads=None):
    import torch
    sim = W.Simulation(p, threads=threads)
    if jb is None:
        sim.beam_current()
    else:
        sim.jb.copy_(torch.from_numpy(np.ascontiguousarray(jb)))
    sim.response()
    torch.cuda.synchronize()
    return sim


def oracle_response(O, p, jb=None):
    return O.response(p, inputs.plasma_draws(p), jb=jb)


def _state(sim):
    return {k: _np(sim.plasma[k]) for k in ("x", "y", "px", "py")}


def _check_fp64(O, W, p, tol=1e-10, threads=None):
    print(f"case {p.name} {p.geom} {p.n_r}x{p.n_xi} ppc={p.ppc} u_th={p.u_th} threads={threads}",
          flush=True)
    ref = oracle_response(O, p)
    sim = gpu_response(W, p, jb=ref["jb"], threads=threads)
    f = _np(sim.fields)
    errs = {name: float(_rel(f[i], ref["fields"][i])) for i, name in enumerate(("psi", "E_z", "B_theta", "W"))}
    print("max rel error per field:", errs, flush=True)
    for name, e in errs.items():
        assert e <= tol, (name, e)
    st = _state(sim)
    for k in ("x", "px", "y", "py"):
        if np.max(np.abs(ref["state"][k])) > 0:
            assert _rel(st[k], ref["state"][k]) <= tol, k
    c = sim.counters_dict()
    assert W.read_counters(sim.counters) == c        # the library's read-back agrees
    assert c["d_clamp"] == int(ref["counters"][0])
    assert c["wall"] == int(ref["counters"][1])
    assert c["nonfinite"] == 0
    return sim, ref


def test_library_loads_and_validates(W):
    with pytest.raises(W.WakeError):
        W.Plan(inputs.weak_single_bunch(ppc=0))


def test_weak_bunch_fp64_matches_oracle(O, W):
    """Cold plasma, fixed single bunch, 128 x 512, FP64: <= 1e-10."""
    _check_fp64(O, W, inputs.weak_single_bunch())


@pytest.mark.parametrize("threads", [256, 512, 1024])
def test_fp64_ragged_tiles(O, W, threads):
    """Particle counts that leave ragged tiles for every workgroup size."""
    p = inputs.weak_single_bunch(n_r=37, n_xi=96, ppc=3, n_b0=0.5)
    _check_fp64(O, W, p, threads=threads)


def test_fp64_minimal_grid(O, W):
    p = inputs.weak_single_bunch(n_r=2, n_xi=5, ppc=1, r_max=1.0, n_b0=0.3)
    _check_fp64(O, W, p)


def test_fp64_single_slice(O, W):
    p = inputs.weak_single_bunch(n_xi=1)
    _check_fp64(O, W, p)


def test_fp64_warm_moderate(O, W):
    """Warm plasma (Cartesian ring electrons), moderate two-bunch driver."""
    p = inputs.facet_two_bunch(n_r=96, n_xi=600, ppc=8, u_th=0.02, n_d=1.0, n_beam=0,
                               prec="fp64")
    _check_fp64(O, W, p)


@pytest.mark.parametrize("threads", [256, 512])
def test_fp64_warm_one_particle_per_thread(O, W, threads):
    """Warm two-bunch driver with one resident particle per thread at 256
    threads (32 cells x 8 per cell): the particle-slot addressing with the
    workgroup size as a compile-time constant."""
    p = inputs.facet_two_bunch(n_r=32, n_xi=200, ppc=8, sep=3.5, u_th=0.02, n_beam=0, prec="fp64")
    _check_fp64(O, W, p, threads=threads)


def test_fp64_slab(O, W):
    p = inputs.weak_single_bunch(geom="slab", r_max=8.0, n_r=128, n_xi=256, n_b0=0.3)
    _check_fp64(O, W, p)
    q = inputs.facet_two_bunch(n_r=64, n_xi=300, ppc=4, u_th=0.02, n_d=1.0, n_beam=0,
                               prec="fp64", geom="slab", r_max=8.0)
    _check_fp64(O, W, q)


def test_fp64_wall_reflections(O, W):
    """Warm plasma at a narrow wall: reflections counted as in the oracle."""
    p = inputs.facet_two_bunch(n_r=32, n_xi=400, ppc=4, u_th=0.05, n_d=0.5, r_max=1.5,
                               n_beam=0, prec="fp64")
    sim, ref = _check_fp64(O, W, p)
    assert int(ref["counters"][1]) > 0


def _envelope(O, p):
    """Oracle sensitivity: fields after a 1-ulp change of the initial radii."""
    st = O.load_plasma(p, inputs.plasma_draws(p))
    jb = O.beam_current_analytic(p)
    f0, _, _ = O.march(p, {k: v.copy() for k, v in st.items()}, jb)
    st["x"] = np.nextafter(st["x"], np.inf)
    f1, _, _ = O.march(p, st, jb)
    return f0, np.abs(f1 - f0)


def test_fp64_blowout_within_sensitivity_envelope(O, W):
    """Blowout with trajectory crossing: |gpu - oracle| <= 10 x the oracle's
    own 1-ulp sensitivity (plus 1e-10 of the field scale), slice by slice."""
    p = inputs.facet_two_bunch(n_r=128, n_xi=1024, ppc=8, u_th=0.02, n_beam=0, prec="fp64")
    f_ref, env = _envelope(O, p)
    sim = gpu_response(W, p)
    f = _np(sim.fields)
    for i in range(4):
        scale = np.max(np.abs(f_ref[i]))
        env_k = np.max(env[i], axis=1)            # per slice
        env_k = np.maximum.accumulate(env_k)
        err_k = np.max(np.abs(f[i] - f_ref[i]), axis=1)
        assert np.all(err_k <= 10 * env_k + 1e-10 * scale), i
    # ahead of trajectory crossing the strict bound holds
    k0 = int(2.0 / p.dxi)
    assert _rel(f[1, :k0], f_ref[1, :k0]) <= 1e-10


def test_mixed_blowout_ez_within_1e3(O, W):
    """FP32 bulk / FP64 solve: ||dE_z|| / ||E_z|| <= 1e-3 on the blowout case."""
    p = inputs.facet_two_bunch(n_r=256, n_xi=2048, ppc=16, u_th=0.02, n_beam=0, prec="mixed")
    ref = oracle_response(O, p.replace(prec="fp64"))
    sim = gpu_response(W, p)
    f = _np(sim.fields)
    e = [_l2(f[i], ref["fields"][i]) for i in range(4)]
    print("mixed L2 errors psi, E_z, B, W:", e, flush=True)
    assert e[1] <= 1e-3
    assert e[0] <= 1e-3 and e[3] <= 1e-2 and e[2] <= 1e-2


def test_beam_current_and_push_fp64(O, W):
    import torch
    p = inputs.facet_two_bunch(n_r=64, n_xi=256, ppc=4, u_th=0.0, n_beam=5000, n_steps=3,
                               prec="fp64")
    sim = W.Simulation(p)
    sim.load_beam()
    ob = O.load_beam(p, inputs.beam_draws(p))
    for k in ("x", "y", "xi", "pz", "w"):
        assert _rel(_np(sim.beam[k]), ob[k]) <= 1e-15, k
    sim.beam_current()
    torch.cuda.synchronize()
    jb_ref, nout = O.beam_current_macro(p, ob)
    assert _rel(_np(sim.jb), jb_ref) <= 1e-12
    sim.response()
    torch.cuda.synchronize()
    st = O.load_plasma(p, None)
    fields, _, _ = O.march(p, st, jb_ref)
    assert _rel(_np(sim.fields), fields) <= 1e-10
    sim.push(3, p.dt)
    torch.cuda.synchronize()
    O.beam_push(p, ob, fields, 3, p.dt)
    for k in ("x", "y", "px", "py", "pz", "xi"):
        assert np.max(np.abs(_np(sim.beam[k]) - ob[k])) <= 1e-10 * max(1.0, np.max(np.abs(ob[k]))), k
    g0 = O.beam_gamma(O.load_beam(p, inputs.beam_draws(p)))
    gain_ref = O.mean_gain(ob, g0, 1)
    assert sim.witness_gain() == pytest.approx(gain_ref, rel=1e-10, abs=1e-12)
    assert sim.ez_peak(3.0) == pytest.approx(O.ez_peak(p, fields, 3.0), rel=1e-10)


def test_cycle_mixed_witness_gain(O, W):
    """Three quasi-static cycles (current -> response -> push) in mixed
    precision vs the FP64 oracle: witness gain within 1e-3."""
    import torch
    p = inputs.facet_two_bunch(n_r=128, n_xi=1024, ppc=8, u_th=0.02, n_beam=20000, n_steps=3,
                               prec="mixed")
    sim = W.Simulation(p)
    sim.load_beam()
    for _ in range(p.n_steps):
        sim.step()
    torch.cuda.synchronize()
    ref = O.cycle(p.replace(prec="fp64"), inputs.plasma_draws(p), inputs.beam_draws(p), p.n_steps)
    g = sim.witness_gain()
    assert g == pytest.approx(ref["witness_gain"], rel=1e-3)
    assert sim.counters_dict()["nonfinite"] == 0


def test_batch_matches_standalone(O, W):
    """Uneven instances in one persistent launch == each run alone (FP64)."""
    import torch
    base = dict(n_beam=0, prec="fp64", u_th=0.02)
    probs = [inputs.facet_two_bunch(n_r=nr, n_xi=nx, ppc=ppc, sep=sep, **base)
             for (nr, nx, ppc, sep) in ((32, 200, 8, 3.5), (64, 333, 4, 4.0), (48, 129, 6, 5.0),
                                        (16, 400, 2, 3.0), (64, 64, 10, 6.0))]
    plans = [W.Plan(q) for q in probs]
    plasmas, jbs, fields = [], [], []
    counters = W.Plan.alloc_counters()
    W.zero_counters(counters)
    for q, pl in zip(probs, plans):
        t = pl.alloc_plasma()
        d = inputs.plasma_draws(q)
        pl.init_plasma(t, torch.from_numpy(d).cuda())
        jb = pl.alloc_jb()
        pl.beam_current_analytic(jb)
        plasmas.append(t)
        jbs.append(jb)
        fields.append(pl.alloc_fields())
    batch = W.Batch(plans)
    batch.describe(plasmas, jbs, fields, counters)
    batch.response()
    torch.cuda.synchronize()
    for q, f in zip(probs, fields):
        ref = oracle_response(O, q)
        assert _rel(_np(f), ref["fields"]) <= 1e-10, q.name


def test_full_size_blowout_first_response_mixed(O, W):
    """The headline workload's first plasma response (512 x 4096, 16 ppc,
    1e6-particle beam current) in mixed precision: E_z within 1e-3."""
    import torch
    p = inputs.blowout_response()
    sim = W.Simulation(p)
    sim.load_beam()
    sim.beam_current()
    sim.response()
    torch.cuda.synchronize()
    ob = O.load_beam(p, inputs.beam_draws(p))
    jb_ref, _ = O.beam_current_macro(p, ob)
    assert _rel(_np(sim.jb), jb_ref) <= 1e-12
    st = O.load_plasma(p, inputs.plasma_draws(p))
    fields, cnt, _ = O.march(p, st, jb_ref)
    f = _np(sim.fields)
    e = _l2(f[1], fields[1])
    print("full-size mixed L2 error E_z:", e, flush=True)
    assert e <= 1e-3
    assert sim.counters_dict()["nonfinite"] == 0


def _beam_np(sim):
    return {k: _np(sim.beam[k]) for k in ("x", "y", "px", "py", "pz", "xi")}


@pytest.mark.parametrize("prec", ["fp64"])
def test_pipelined_cycle_matches_sequential(O, W, prec):
    """The pipelined cycle (responses of successive beam steps on separate
    workgroups) gives the sequential cycle's beam, FP64, moderate driver."""
    import torch
    p = inputs.facet_two_bunch(n_r=96, n_xi=400, ppc=8, u_th=0.02, n_d=1.0, n_beam=6000,
                               n_steps=5, prec=prec)
    print("case", p.name, "steps", p.n_steps, flush=True)
    seq = W.Simulation(p)
    seq.load_beam()
    for _ in range(p.n_steps):
        seq.step()
    torch.cuda.synchronize()
    pipe = W.Simulation(p)
    pipe.load_beam()
    pipe.run_cycle(p.n_steps)
    torch.cuda.synchronize()
    c = pipe.counters_dict()
    assert c["pipeline_abort"] == 0 and c["beam_bin"] == 0
    assert W.read_counters(pipe.counters) == c
    a, b = _beam_np(pipe), _beam_np(seq)
    for k in a:
        scale = max(1.0, np.max(np.abs(b[k])))
        assert np.max(np.abs(a[k] - b[k])) <= 1e-10 * scale, k
    assert _rel(_np(pipe.fields), _np(seq.fields)) <= 1e-10
    # and the oracle's sequential cycle
    ref = O.cycle(p, inputs.plasma_draws(p), inputs.beam_draws(p), p.n_steps)
    for k in ("x", "pz", "xi"):
        scale = max(1.0, np.max(np.abs(ref["beam"][k])))
        assert np.max(np.abs(a[k] - ref["beam"][k])) <= 1e-10 * scale, k
    assert pipe.witness_gain() == pytest.approx(ref["witness_gain"], rel=1e-10)


def test_pipelined_cycle_mixed_blowout(O, W):
    """Blowout two-bunch driver, mixed precision, 8 pipelined steps vs the
    FP64 oracle: witness gain within 1e-3, no aborts, no bin escapes."""
    import torch
    p = inputs.facet_two_bunch(n_r=128, n_xi=1024, ppc=8, u_th=0.02, n_beam=20000, n_steps=8,
                               prec="mixed")
    pipe = W.Simulation(p)
    pipe.load_beam()
    pipe.run_cycle(p.n_steps)
    torch.cuda.synchronize()
    c = pipe.counters_dict()
    assert c["pipeline_abort"] == 0 and c["beam_bin"] == 0 and c["nonfinite"] == 0
    ref = O.cycle(p.replace(prec="fp64"), inputs.plasma_draws(p), inputs.beam_draws(p), p.n_steps)
    assert pipe.witness_gain() == pytest.approx(ref["witness_gain"], rel=1e-3)


@pytest.mark.parametrize("geom", ["cyl", "slab"])
def test_large_grid_rows_in_global_memory(O, W, geom):
    """Grids whose node rows exceed LDS (here 1200 cells) keep only the
    deposit rows in LDS and the field and solver rows in global memory:
    FP64 parity with the oracle on a short window."""
    p = inputs.facet_two_bunch(n_r=1200, n_xi=40, ppc=2, u_th=0.02, n_beam=0, prec="fp64", n_d=1.0,
                               geom=geom, r_max=6.0 if geom == "cyl" else 8.0, name=f"large-{geom}")
    _check_fp64(O, W, p)


def test_large_grid_mixed(O, W):
    p = inputs.facet_two_bunch(n_r=1400, n_xi=64, ppc=4, u_th=0.02, n_beam=0, prec="mixed", name="large-mixed")
    print(f"case {p.name}", flush=True)
    ref = oracle_response(O, p.replace(prec="fp64"))
    sim = gpu_response(W, p, jb=ref["jb"])
    f = _np(sim.fields)
    assert _l2(f[1], ref["fields"][1]) <= 1e-3
    assert _l2(f[0], ref["fields"][0]) <= 1e-3


@pytest.mark.parametrize("n_r", [1000, 1200])
def test_pipelined_cycle_large_grid(O, W, n_r):
    """Large grids in the pipelined cycle (node rows and beam-current rows in
    global memory; at 1000 cells only the cycle needs that, at 1200 the
    sequential march too): same beam and fields as the sequential cycle and
    the oracle, FP64."""
    import torch
    p = inputs.facet_two_bunch(n_r=n_r, n_xi=64, ppc=2, u_th=0.02, n_d=1.0, n_beam=4000, n_steps=3,
                               prec="fp64", name=f"cycle-large-{n_r}")
    print("case", p.name, flush=True)
    seq = W.Simulation(p)
    seq.load_beam()
    for _ in range(p.n_steps):
        seq.step()
    pipe = W.Simulation(p)
    pipe.load_beam()
    pipe.run_cycle(p.n_steps)
    torch.cuda.synchronize()
    c = pipe.counters_dict()
    assert c["pipeline_abort"] == 0 and c["beam_bin"] == 0 and c["nonfinite"] == 0
    a, b = _beam_np(pipe), _beam_np(seq)
    for k in a:
        scale = max(1.0, np.max(np.abs(b[k])))
        assert np.max(np.abs(a[k] - b[k])) <= 1e-10 * scale, k
    assert _rel(_np(pipe.fields), _np(seq.fields)) <= 1e-10
    ref = O.cycle(p, inputs.plasma_draws(p), inputs.beam_draws(p), p.n_steps)
    assert _rel(_np(pipe.fields), ref["fields"]) <= 1e-10
    assert pipe.witness_gain() == pytest.approx(ref["witness_gain"], rel=1e-10)


def test_headline_cycle_full_size(O, W):
    """The benchmark's workload and launch (512 x 4096, 16 ppc, 1e6 beam
    particles, pipelined cycle, mixed precision): three steps against the
    FP64 oracle's sequential cycle (last fields E_z within 1e-3, witness gain
    within 1e-3); then, after 199 steps, the 200th response against the
    oracle's response to the same (GPU-evolved) beam: E_z within 1e-3."""
    import torch
    p = inputs.blowout_response().replace(n_steps=3)
    print("case", p.name, "3 steps", flush=True)
    sim = W.Simulation(p)
    sim.load_beam()
    sim.run_cycle(3)
    torch.cuda.synchronize()
    ref = O.cycle(p.replace(prec="fp64"), inputs.plasma_draws(p), inputs.beam_draws(p), 3)
    f = _np(sim.fields)
    assert _l2(f[1], ref["fields"][1]) <= 1e-3
    assert sim.witness_gain() == pytest.approx(ref["witness_gain"], rel=1e-3)
    print("case", p.name, "199 + 1 steps", flush=True)
    sim = W.Simulation(p.replace(n_steps=200))
    sim.load_beam()
    sim.run_cycle(199)
    torch.cuda.synchronize()
    beam = {k: _np(v) for k, v in sim.beam.items() if k != "tag"}
    sim.run_cycle(1)
    torch.cuda.synchronize()
    c = sim.counters_dict()
    assert c["pipeline_abort"] == 0 and c["beam_bin"] == 0 and c["nonfinite"] == 0
    q = p.replace(prec="fp64")
    jb, _ = O.beam_current_macro(q, beam)
    ref = O.response(q, inputs.plasma_draws(q), jb=jb)
    f = _np(sim.fields)
    assert _l2(f[1], ref["fields"][1]) <= 1e-3
    assert _l2(f[0], ref["fields"][0]) <= 1e-3
