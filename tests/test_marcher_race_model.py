"""The marcher's barrier schedule, checked on the CPU.

The device marcher (dev::Marcher in csrc/wk_marcher.h, the code every march,
batch and cycle kernel runs), and the other kernels that coordinate the
threads of one workgroup (the Eq. (6)-direct march, the gradient's recording
and reverse marches, the beam current's cell sort and row sums), are
compiled for the host against a model of the device environment (tests/race_model/hip/hip_runtime.h): one OS thread
per GPU thread of one workgroup, every workgroup barrier a thread barrier,
every cross-lane operation (DPP row shifts and broadcasts, ds_bpermute) a
barrier of the 64 threads of its wavefront that exchanges their values, LDS
and global memory plain shared memory.  Built with ThreadSanitizer, a pair of
accesses to one address by two threads that no barrier orders, one of them a
write, is reported as a race; a barrier that not every thread reaches leaves the run
hanging, which the time limit reports.

The kernel headers are copied unchanged except for their three inline-asm
statements (the vmcnt and lgkmcnt waits and the compiler fence of the LDS
barrier), which become calls into the model; the copy is checked to contain
no other asm.  Each shape runs one response and its fields are compared with
the oracle's (FP64 within 1e-10 of each field's scale, mixed precision
||dE_z|| / ||E_z|| <= 1e-3), which shows that the model executes the march
faithfully, cross-lane operations included.

Some cases run on groups of 2 and 3 workgroups (the plain march, and both
marches of the gradient), each workgroup a process of its own over one
shared mapping of device memory: the exchanges between the members run as
on the device, and the results are held to the same bars; a copy with the
marcher's or the reverse march's exchange left out fails them.

What the model does not see: ordering of global memory by the LDS-only
barrier (on the GPU it orders LDS accesses only; the marcher keeps its
cross-thread data in LDS except for the large-grid rows, which use the
waiting barrier), and races between workgroups, whose exchanges rely on
tagged values rather than barriers (ThreadSanitizer checks the threads of
one process).
"""
import concurrent.futures
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

from paper_1411_3246_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1411_3246_amd", "csrc")
MODEL = os.path.join(HERE, "race_model")

MAINS = ("model_main.cpp", "model_direct_main.cpp", "model_adjoint_main.cpp", "model_beam_main.cpp")

ASM = {
    'asm volatile("s_waitcnt vmcnt(0)" ::: "memory");': "wk_model::wait_vm();",
    'asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");': "wk_model::wait_lgkm();",
    'asm volatile("" ::: "memory");': "wk_model::compiler_fence();",
}


def _build(d, mutate=None, mains=MAINS):
    """Copy the kernel headers into d (asm statements modelled, `mutate`
    applied to the marcher) and build the model there."""
    os.makedirs(d / "pkg" / "csrc")
    os.makedirs(d / "include")
    shutil.copy(os.path.join(ROOT, "include", "wake.h"), d / "include" / "wake.h")
    for name in ("wk_marcher.h", "wk_internal.h", "wk_direct.h", "wk_direct.hip", "wk_adjoint.hip",
                 "wk_adjoint_dev.h", "wk_beam.hip", "wk_beam_dev.h"):
        with open(os.path.join(CSRC, name)) as f:
            src = f.read()
        for old, new in ASM.items():
            src = src.replace(old, new)
        assert not re.search(r"\basm\b\s*(volatile)?\s*\(", src), f"unmodelled inline asm in {name}"
        # a kernel's dynamic LDS is the modelled workgroup's buffer
        src = re.sub(r"extern __shared__ double (\w+)\[\];", r"double* \1 = wk_model::dynamic_lds;", src)
        if mutate and name == "wk_marcher.h":
            src = mutate(src)
        with open(d / "pkg" / "csrc" / name, "w") as f:
            f.write(src)

    def compile_one(main):
        exe = str(d / main.replace(".cpp", ""))
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread", "-I", MODEL,
               "-I", str(d / "pkg" / "csrc"), os.path.join(MODEL, main), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
        assert r.returncode == 0, r.stderr[-4000:]
        return exe
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        return list(ex.map(compile_one, mains))


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("race_model")
    return _build(d), d


CASES = [
    # (shape, problem)
    ("f64-cyl-warm-256x4-res", dict(n_r=32, ppc=8, u_th=0.02)),
    ("f64-cyl-cold-256x4-res", dict(n_r=32, ppc=8, u_th=0.0)),
    ("f64-slab-warm-256x4-res", dict(n_r=32, ppc=8, u_th=0.02, geom="slab", r_max=8.0)),
    ("f64-cyl-warm-256x4-res", dict(n_r=64, ppc=16, u_th=0.02)),            # 4 per thread
    ("f64-cyl-warm-256x4-stream", dict(n_r=48, ppc=24, u_th=0.02)),         # two tiles
    ("f64-cyl-warm-512x4-res", dict(n_r=37, ppc=16, u_th=0.02)),            # ragged
    ("f64-cyl-warm-1024x8-res", dict(n_r=64, ppc=16, u_th=0.02)),
    ("f64-cyl-warm-512x8-big-stream", dict(n_r=40, ppc=16, u_th=0.02)),
    ("f32-cyl-warm-512x8-res", dict(n_r=64, ppc=32, u_th=0.02, prec="mixed")),
    ("f32-cyl-warm-512x8-big-res", dict(n_r=64, ppc=16, u_th=0.02, prec="mixed")),
    # groups of workgroups (a process per member): exchanges of S and of the
    # folded moments; a ragged split of 40 cells over 3 members with global
    # node rows per member
    ("f64-cyl-warm-256x4-res", dict(n_r=32, ppc=8, u_th=0.02, group=2)),
    ("f64-cyl-warm-512x8-big-stream", dict(n_r=40, ppc=16, u_th=0.02, group=3)),
]


def _write_input(path, p, st, jb):
    hdr = np.array([0 if p.geom == "cyl" else 1, 1 if p.u_th > 0 else 0, p.n_r, p.n_xi, p.ppc,
                    0 if p.prec == "fp64" else 1], dtype=np.int32)
    with open(path, "wb") as f:
        f.write(hdr.tobytes())
        f.write(np.array([len(st["x"])], dtype=np.int64).tobytes())
        f.write(np.array([p.r_max, p.r_max / p.n_r, p.dxi, p.d_min], dtype=np.float64).tobytes())
        for k in ("x", "y", "px", "py", "d0", "w", "nion"):
            f.write(np.ascontiguousarray(st[k], dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(jb, dtype=np.float64).tobytes())


@pytest.mark.parametrize("shape,kw", CASES,
                         ids=[f"{s}-{k['n_r']}x{k['ppc']}" + (f"-group{k['group']}" if "group" in k else "")
                              for s, k in CASES])
def test_barrier_schedule_race_free(model, oracle_lib, shape, kw):
    (exe, _, _, _), d = model
    r, p, fout, ref = _run(exe, d, oracle_lib, shape, kw)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stderr[-2000:]
    N1 = p.n_r + 1
    raw = np.fromfile(fout, dtype=np.float64, count=4 * p.n_xi * N1).reshape(4, p.n_xi, N1)
    cnt = np.fromfile(fout, dtype=np.uint64, offset=8 * 4 * p.n_xi * N1)
    assert cnt[-1] > 10 * p.n_xi                     # workgroup barriers passed
    f0 = ref["fields"]
    if p.prec == "fp64":
        for i in range(4):
            scale = np.max(np.abs(f0[i]))
            assert np.max(np.abs(raw[i] - f0[i])) <= 1e-10 * scale, (i, np.max(np.abs(raw[i] - f0[i])) / scale)
        assert int(cnt[0]) == int(ref["counters"][0]) and int(cnt[1]) == int(ref["counters"][1])
    else:
        assert np.linalg.norm(raw[1] - f0[1]) <= 1e-3 * np.linalg.norm(f0[1])


def test_model_reports_a_missing_barrier(tmp_path, oracle_lib):
    """The check has teeth: with the barrier between the stage-1 psi solve
    and the moment deposit (which gathers psi at the particles) taken out of
    a copy of the marcher, the model reports a race."""
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    cut = "            solve_psi(psi2);\n            sync();\n"

    def mutate(src):
        assert cut in src
        return src.replace(cut, "            solve_psi(psi2);\n", 1)
    (exe,) = _build(tmp_path, mutate, mains=("model_main.cpp",))
    r, _, _, _ = _run(exe, tmp_path, oracle_lib, "f64-cyl-warm-256x4-res", dict(n_r=32, ppc=8, u_th=0.02))
    assert "ThreadSanitizer: data race" in r.stderr, r.stderr[-2000:]
    assert "solve_psi" in r.stderr or "dep_moments" in r.stderr


def _run(exe, d, O, shape, kw):
    kw = dict(kw)
    group = kw.pop("group", 1)
    base = dict(n_xi=40, n_d=1.0, n_beam=0, prec="fp64")
    base.update(kw)
    full = inputs.facet_two_bunch(**base, name=f"model-{shape}")
    # the first 12 slices of the 40-slice window: into the drive bunch
    p = full.replace(n_xi=12, xi_max=full.xi_min + 12 * full.dxi)
    st = O.load_plasma(p, inputs.plasma_draws(p))
    jb = O.beam_current_analytic(p)
    ref = O.response(p.replace(prec="fp64"), inputs.plasma_draws(p))
    fin = str(d / f"{shape}-{p.n_r}-{group}.in")
    fout = str(d / f"{shape}-{p.n_r}-{group}.out")
    _write_input(fin, p, st, jb)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66 report_signal_unsafe=0 die_after_fork=0")
    r = subprocess.run([exe, fin, fout, shape, str(group)], capture_output=True, text=True, timeout=600, env=env)
    return r, p, fout, ref


@pytest.mark.parametrize("kw", [dict(u_th=0.02, n_d=0.3), dict(u_th=0.02, n_d=0.3, geom="slab", r_max=8.0)],
                         ids=["warm-cyl", "warm-slab"])
def test_direct_response_race_free(model, oracle_lib, kw):
    """The Eq. (6)-direct response (wk_direct.hip: the marcher's deposits and
    solves, block reductions by lane shuffles, GMRES with thread 0 applying
    the rotations) in the same model: race free, and its fields equal the
    oracle's direct march within 1e-10 + 10 tol of each field's scale (the
    Newton test stops anywhere within tol of the fixed point, so two
    evaluation orders may stop at iterates that far apart), Newton step
    counts within one of the oracle's."""
    (_, exe, _, _), d = model
    O = oracle_lib
    full = inputs.facet_two_bunch(n_r=24, n_xi=40, ppc=2, n_beam=0, prec="fp64", name="model-direct", **kw)
    # four slices of the 40-slice window, where the drive's head arrives
    p = full.replace(n_xi=4, xi_min=full.xi_min + 6 * full.dxi, xi_max=full.xi_min + 10 * full.dxi)
    st = O.load_plasma(p, inputs.plasma_draws(p))
    jb = O.beam_current_analytic(p)
    tol = 1e-10
    f0, c0, it0 = O.march_direct(p, {k: v.copy() for k, v in st.items()}, jb, tol=tol)
    fin, fout = str(d / "direct.in"), str(d / "direct.out")
    _write_input(fin, p, st, jb)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66 report_signal_unsafe=0")
    r = subprocess.run([exe, fin, fout, "8", repr(tol)], capture_output=True, text=True, timeout=900, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stderr[-2000:]
    N1 = p.n_r + 1
    n_f = 4 * p.n_xi * N1
    f = np.fromfile(fout, dtype=np.float64, count=n_f).reshape(4, p.n_xi, N1)
    n_cnt = 8                                        # WK_NCOUNTERS
    cnt = np.fromfile(fout, dtype=np.uint64, count=n_cnt, offset=8 * n_f)
    its = np.fromfile(fout, dtype=np.int32, offset=8 * n_f + 8 * n_cnt)
    top = np.max(np.abs(f0))
    for i in range(4):
        scale = np.max(np.abs(f0[i])) or top
        assert np.max(np.abs(f[i] - f0[i])) <= (1e-10 + 10 * tol) * scale, (i, np.max(np.abs(f[i] - f0[i])) / scale)
    assert np.max(np.abs(its - it0)) <= 1, (its, it0)
    assert int(cnt[0]) == int(c0[0]) and int(cnt[1]) == int(c0[1])


@pytest.mark.parametrize("geom,group", [("cyl", 2), ("slab", 3)])
def test_adjoint_march_race_free_and_consistent(model, oracle_lib, geom, group):
    """The plasma part of the gradient (wk_adjoint.hip): the recording
    forward march, then the reverse march (checkpointed segments of 8 slices)
    seeded by a random adjoint of the stored fields, in the same model: race
    free; the forward fields equal the oracle's within 1e-10; and the reverse
    march's adjoints of the initial state (x, y, p_x, p_y), of D0, of w and of
    the beam current satisfy <fbar, dF> = <ybar, dy> against central
    differences of the oracle's march in random directions (1e-6 relative
    plus 1e-7 absolute, at steps of 1e-6 or 1e-7).  With group > 1 both
    marches run on that many workgroups, each a process of its own over
    shared device memory: the exchanges between them run as on the device,
    ThreadSanitizer checks each workgroup's threads, and the results carry
    the same bars."""
    (_, _, exe, _), d = model
    O = oracle_lib
    kw = dict(geom="slab", r_max=8.0) if geom == "slab" else {}
    full = inputs.facet_two_bunch(n_r=16, n_xi=40, ppc=4, u_th=0.02, n_d=0.3, n_beam=0, prec="fp64",
                                  name=f"model-adjoint-{geom}", **kw)
    p = full.replace(n_xi=20, xi_max=full.xi_min + 20 * full.dxi)
    st = O.load_plasma(p, inputs.plasma_draws(p))
    jb = O.beam_current_analytic(p)
    N1, npart = p.n_r + 1, len(st["x"])
    rng = np.random.default_rng(5)
    fbar = rng.standard_normal((4, p.n_xi, N1))
    fin, ffb, fout = str(d / f"adj-{geom}-{group}.in"), str(d / f"adj-{geom}-{group}.fbar"), str(d / f"adj-{geom}-{group}.out")
    _write_input(fin, p, st, jb)
    fbar.tofile(ffb)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66 report_signal_unsafe=0 die_after_fork=0")
    r = subprocess.run([exe, fin, ffb, fout, "8", str(group)], capture_output=True, text=True, timeout=900, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stderr[-2000:]
    out = np.fromfile(fout)
    sizes = [4 * p.n_xi * N1, p.n_xi * N1, 4 * npart, npart, npart]
    F, jbbar, ybar, d0bar, wbar = np.split(out, np.cumsum(sizes)[:-1])
    F = F.reshape(4, p.n_xi, N1)

    def fwd(s, j):
        return O.march(p, {k: v.copy() for k, v in s.items()}, j)[0]
    F0 = fwd(st, jb)
    for i in range(4):
        assert np.max(np.abs(F[i] - F0[i])) <= 1e-10 * np.max(np.abs(F0[i])), i
    ybar = ybar.reshape(4, npart)
    bars = {"x": ybar[0], "px": ybar[2], "d0": d0bar, "w": wbar}
    if geom == "cyl":
        bars.update(y=ybar[1], py=ybar[3])
    else:
        bars.update(py=ybar[3])
    # a difference whose step straddles a node crossing is not a derivative:
    # each direction is differenced at two small steps, one must agree, to
    # 1e-6 relative plus 1e-7 absolute (the rounding of the quotients)
    def agree(diff, rhs):
        errs = [abs(diff(e) - rhs) for e in (1e-6, 1e-7)]
        return min(errs) <= 1e-6 * abs(rhs) + 1e-7, errs

    for key, bar in bars.items():
        dl = rng.standard_normal(npart)

        def diff(eps):
            sp = dict(st, **{key: st[key] + eps * dl})
            sm = dict(st, **{key: st[key] - eps * dl})
            return np.sum(fbar * (fwd(sp, jb) - fwd(sm, jb))) / (2 * eps)
        ok, errs = agree(diff, float(np.dot(bar, dl)))
        assert ok, (key, errs)
    dj = rng.standard_normal(jb.shape)

    def diff_jb(eps):
        return np.sum(fbar * (fwd(st, jb + eps * dj) - fwd(st, jb - eps * dj))) / (2 * eps)
    ok, errs = agree(diff_jb, float(np.sum(jbbar.reshape(jb.shape) * dj)))
    assert ok, ("jb", errs)


@pytest.mark.parametrize("n_beam,n_xi", [(20000, 16), (40000, 4)], ids=["short-cells", "long-cells"])
def test_beam_current_kernels_race_free(model, oracle_lib, n_beam, n_xi):
    """The beam current's cell sort (LDS bitonic runs; cells beyond one run
    take the merge path) and its ordered row sums in the same model: race
    free; every cell's indices come out ascending whatever order the scatter
    gave them; and the rows equal the oracle's within 1e-12."""
    (_, _, _, exe), d = model
    O = oracle_lib
    p = inputs.facet_two_bunch(n_r=32, n_xi=n_xi, ppc=2, n_beam=n_beam, n_steps=1, prec="fp64",
                               name=f"model-beam-{n_xi}")
    ob = O.load_beam(p, inputs.beam_draws(p))
    fin, fout = str(d / f"beam-{n_xi}.in"), str(d / f"beam-{n_xi}.out")
    with open(fin, "wb") as f:
        f.write(np.array([0 if p.geom == "cyl" else 1, p.n_r, p.n_xi], dtype=np.int32).tobytes())
        f.write(np.array([n_beam], dtype=np.int64).tobytes())
        f.write(np.array([p.r_max, p.r_max / p.n_r, p.xi_min, p.dxi], dtype=np.float64).tobytes())
        for k in ("x", "y", "xi", "w"):
            f.write(np.ascontiguousarray(ob[k], dtype=np.float64).tobytes())
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66 report_signal_unsafe=0")
    r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=900, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, r.stderr[-2000:]
    raw = np.fromfile(fout, dtype=np.uint8)
    start = np.frombuffer(raw[:4 * (n_xi + 1)].tobytes(), dtype=np.uint32)
    total = int(start[-1])
    order = np.frombuffer(raw[4 * (n_xi + 1):4 * (n_xi + 1 + total)].tobytes(), dtype=np.uint32)
    jb = np.frombuffer(raw[4 * (n_xi + 1 + total):].tobytes(), dtype=np.float64).reshape(n_xi, p.n_r + 1)
    if n_xi == 4:
        assert np.max(np.diff(start)) > 8192           # a cell beyond one LDS run
    for c in range(n_xi):
        seg = order[start[c]:start[c + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0), c
    jb_ref, _ = O.beam_current_macro(p, ob)
    assert np.max(np.abs(jb - jb_ref)) <= 1e-12 * np.max(np.abs(jb_ref))
