"""ctypes wrapper of the serial FP64 oracle (wake_oracle.c).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU-baseline
leg of the benchmark; never by the product path.  Takes problems and draws
from ``paper_1411_3246_amd.inputs`` and nothing else from the package.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_up = C.POINTER(C.c_uint64)


class OrProblem(C.Structure):
    _fields_ = [("geom", C.c_int32), ("n_r", C.c_int32), ("r_max", C.c_double),
                ("n_xi", C.c_int32), ("xi_min", C.c_double), ("xi_max", C.c_double),
                ("ppc", C.c_int32), ("u_th", C.c_double), ("n0", C.c_double),
                ("sigma_r", C.c_double), ("n_bunch", C.c_int32),
                ("n_peak", C.c_double * 2), ("sigma_z", C.c_double * 2),
                ("xi_c", C.c_double * 2), ("d_min", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(OrProblem)
        L.or_plasma_count.argtypes = [P]
        L.or_plasma_count.restype = C.c_int64
        L.or_load_plasma.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_beam_current_analytic.argtypes = [P, _dp]
        L.or_load_beam.argtypes = [P, C.c_int64, C.c_int64, C.c_double, C.c_double, _dp,
                                   _dp, _dp, _dp, _dp, _dp, _dp, _dp, _ip]
        L.or_beam_current_macro.argtypes = [P, C.c_int64, _dp, _dp, _dp, _dp, _dp, _lp]
        L.or_eval.argtypes = [P, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                              _dp, _dp, _dp, _dp, _lp]
        L.or_march.argtypes = [P, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                               _dp, _dp, _lp]
        L.or_beam_push.argtypes = [P, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                   C.c_int32, C.c_double, _lp]
        L.or_mean_gain.argtypes = [C.c_int64, _ip, C.c_int32, _dp, _dp, _dp, _dp, _dp]
        L.or_mean_gain.restype = C.c_double
        L.or_ez_peak.argtypes = [P, _dp, C.c_double]
        L.or_march_direct.argtypes = [P, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _lp,
                                      C.c_int32, C.c_double, _ip]
        L.or_march_traj.argtypes = [P, C.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _lp,
                                    C.c_int32, _dp]
        L.or_gain_histogram.argtypes = [C.c_int64, _ip, C.c_int32, _dp, _dp, _dp, _dp, C.c_int32,
                                        C.c_double, C.c_double, _up]
        L.or_ez_peak.restype = C.c_double
        L.or_thomas.argtypes = [C.c_int64, _dp, _dp, _dp, _dp, _dp]
        for name in ("or_load_plasma", "or_beam_current_analytic", "or_load_beam",
                     "or_beam_current_macro", "or_eval", "or_march", "or_beam_push",
                     "or_thomas"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.flags.c_contiguous
    if a.dtype == np.float64:
        return a.ctypes.data_as(_dp)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_ip)
    if a.dtype == np.int64:
        return a.ctypes.data_as(_lp)
    if a.dtype == np.uint64:
        return a.ctypes.data_as(_up)
    raise TypeError(a.dtype)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def problem(p) -> OrProblem:
    """Convert an inputs.Problem into the oracle's C struct."""
    q = OrProblem()
    q.geom = 0 if p.geom == "cyl" else 1
    q.n_r = p.n_r
    q.r_max = p.r_max
    q.n_xi = p.n_xi
    q.xi_min = p.xi_min
    q.xi_max = p.xi_max
    q.ppc = p.ppc
    q.u_th = p.u_th
    q.n0 = p.n0
    q.sigma_r = p.sigma_r
    q.n_bunch = len(p.bunches)
    for b, bb in enumerate(p.bunches):
        q.n_peak[b] = bb.n_peak
        q.sigma_z[b] = bb.sigma_z
        q.xi_c[b] = bb.xi_c
    q.d_min = p.d_min
    return q


def load_plasma(p, eps: Optional[np.ndarray]) -> Dict[str, np.ndarray]:
    q = problem(p)
    n = p.n_plasma
    st = {k: np.zeros(n) for k in ("x", "y", "px", "py", "d0", "w")}
    st["nion"] = np.zeros(p.n_r + 1)
    e = None if eps is None else np.ascontiguousarray(eps, dtype=np.float64)
    _check(lib().or_load_plasma(C.byref(q), _p(e), _p(st["x"]), _p(st["y"]), _p(st["px"]),
                                _p(st["py"]), _p(st["d0"]), _p(st["w"]), _p(st["nion"])),
           "load_plasma")
    return st


def beam_current_analytic(p) -> np.ndarray:
    q = problem(p)
    jb = np.zeros((p.n_xi, p.n_r + 1))
    _check(lib().or_beam_current_analytic(C.byref(q), _p(jb)), "beam_current_analytic")
    return jb


def load_beam(p, eps: np.ndarray) -> Dict[str, np.ndarray]:
    q = problem(p)
    n = p.n_beam
    b = {k: np.zeros(n) for k in ("x", "y", "px", "py", "pz", "xi", "w")}
    b["tag"] = np.zeros(n, dtype=np.int32)
    e = np.ascontiguousarray(eps, dtype=np.float64)
    _check(lib().or_load_beam(C.byref(q), n, p.n_drive, p.gamma0, p.rel_spread, _p(e),
                              _p(b["x"]), _p(b["y"]), _p(b["px"]), _p(b["py"]), _p(b["pz"]),
                              _p(b["xi"]), _p(b["w"]), _p(b["tag"])), "load_beam")
    return b


def beam_current_macro(p, b: Dict[str, np.ndarray]):
    q = problem(p)
    jb = np.zeros((p.n_xi, p.n_r + 1))
    nout = np.zeros(1, dtype=np.int64)
    _check(lib().or_beam_current_macro(C.byref(q), len(b["x"]), _p(b["x"]), _p(b["y"]),
                                       _p(b["xi"]), _p(b["w"]), _p(jb), _p(nout)),
           "beam_current_macro")
    return jb, int(nout[0])


def evaluate(p, st: Dict[str, np.ndarray], jb_row: np.ndarray):
    """One stage evaluation; returns dict with f (4, np), fields (4, N+1),
    mom (9, N+1) rows S, Jr, Jz, M1..M5, Q; part (3, np) D, gamma, p_z."""
    q = problem(p)
    n = len(st["x"])
    N1 = p.n_r + 1
    f = np.zeros((4, n))
    fields = np.zeros((4, N1))
    mom = np.zeros((9, N1))
    part = np.zeros((3, n))
    cnt = np.zeros(3, dtype=np.int64)
    jr = np.ascontiguousarray(jb_row, dtype=np.float64)
    _check(lib().or_eval(C.byref(q), n, _p(st["x"]), _p(st["y"]), _p(st["px"]), _p(st["py"]),
                         _p(st["d0"]), _p(st["w"]), _p(st["nion"]), _p(jr), _p(f), _p(fields),
                         _p(mom), _p(part), _p(cnt)), "eval")
    return {"f": f, "fields": fields, "mom": mom, "part": part, "counters": cnt}


def march(p, st: Dict[str, np.ndarray], jb: np.ndarray, diag: bool = False):
    """Plasma response; advances st in place.  Returns fields (4, n_xi, N+1),
    counters (clamps, wall reflections, nonfinite) and optional diag
    (3, n_xi, N+1) = S, J_r, J_z."""
    q = problem(p)
    N1 = p.n_r + 1
    fields = np.zeros((4, p.n_xi, N1))
    d = np.zeros((3, p.n_xi, N1)) if diag else None
    cnt = np.zeros(3, dtype=np.int64)
    jbc = np.ascontiguousarray(jb, dtype=np.float64)
    _check(lib().or_march(C.byref(q), len(st["x"]), _p(st["x"]), _p(st["y"]), _p(st["px"]),
                          _p(st["py"]), _p(st["d0"]), _p(st["w"]), _p(st["nion"]), _p(jbc),
                          _p(fields), _p(d), _p(cnt)), "march")
    return fields, cnt, d


def march_traj(p, st: Dict[str, np.ndarray], jb: np.ndarray, stride: int):
    """march() recording the radius of every stride-th particle at every
    slice; returns fields, counters and traj (n_xi, ceil(np / stride))."""
    q = problem(p)
    N1 = p.n_r + 1
    n = len(st["x"])
    fields = np.zeros((4, p.n_xi, N1))
    traj = np.zeros((p.n_xi, (n + stride - 1) // stride))
    cnt = np.zeros(3, dtype=np.int64)
    jbc = np.ascontiguousarray(jb, dtype=np.float64)
    _check(lib().or_march_traj(C.byref(q), n, _p(st["x"]), _p(st["y"]), _p(st["px"]), _p(st["py"]),
                               _p(st["d0"]), _p(st["w"]), _p(st["nion"]), _p(jbc), _p(fields), _p(cnt),
                               int(stride), _p(traj)), "march_traj")
    return fields, cnt, traj


def march_direct(p, st: Dict[str, np.ndarray], jb: np.ndarray, iters: int = 8, tol: float = 1e-10):
    """The response with B_theta from Eq. (6) directly (implicit d_xi E_z,
    Newton-GMRES per slice); returns fields, counters and the Newton steps
    used per slice."""
    q = problem(p)
    N1 = p.n_r + 1
    fields = np.zeros((4, p.n_xi, N1))
    cnt = np.zeros(3, dtype=np.int64)
    its = np.zeros(p.n_xi, dtype=np.int32)
    jbc = np.ascontiguousarray(jb, dtype=np.float64)
    _check(lib().or_march_direct(C.byref(q), len(st["x"]), _p(st["x"]), _p(st["y"]), _p(st["px"]),
                                 _p(st["py"]), _p(st["d0"]), _p(st["w"]), _p(st["nion"]), _p(jbc), _p(fields),
                                 _p(cnt), int(iters), float(tol), _p(its)), "march_direct")
    return fields, cnt, its


def gain_histogram(b: Dict[str, np.ndarray], gamma_before: np.ndarray, which: int, n_bins: int,
                   lo: float, hi: float) -> np.ndarray:
    hist = np.zeros(n_bins + 2, dtype=np.uint64)
    g0 = np.ascontiguousarray(gamma_before, dtype=np.float64)
    tag = np.ascontiguousarray(b["tag"], dtype=np.int32)
    px, py, pz = (np.ascontiguousarray(b[k], dtype=np.float64) for k in ("px", "py", "pz"))
    _check(lib().or_gain_histogram(len(px), _p(tag), which, _p(px), _p(py), _p(pz), _p(g0), n_bins,
                                   lo, hi, _p(hist)), "gain_histogram")
    return hist


def beam_push(p, b: Dict[str, np.ndarray], fields: np.ndarray, n_steps: int, dt: float) -> int:
    q = problem(p)
    nout = np.zeros(1, dtype=np.int64)
    fc = np.ascontiguousarray(fields, dtype=np.float64)
    _check(lib().or_beam_push(C.byref(q), len(b["x"]), _p(b["x"]), _p(b["y"]), _p(b["px"]),
                              _p(b["py"]), _p(b["pz"]), _p(b["xi"]), _p(fc), n_steps, dt,
                              _p(nout)), "beam_push")
    return int(nout[0])


def beam_gamma(b: Dict[str, np.ndarray]) -> np.ndarray:
    return np.sqrt(1.0 + b["px"] ** 2 + b["py"] ** 2 + b["pz"] ** 2)


def mean_gain(b: Dict[str, np.ndarray], gamma_before: np.ndarray, which: int = 1) -> float:
    g0 = np.ascontiguousarray(gamma_before, dtype=np.float64)
    return float(lib().or_mean_gain(len(b["x"]), _p(b["tag"]), which, _p(b["w"]), _p(g0),
                                    _p(b["px"]), _p(b["py"]), _p(b["pz"])))


def ez_peak(p, fields: np.ndarray, xi_from: float) -> float:
    q = problem(p)
    fc = np.ascontiguousarray(fields, dtype=np.float64)
    return float(lib().or_ez_peak(C.byref(q), _p(fc), xi_from))


def thomas(a, b, c, d) -> np.ndarray:
    a, b, c, d = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, d))
    x = np.zeros_like(d)
    _check(lib().or_thomas(len(d), _p(a), _p(b), _p(c), _p(d), _p(x)), "thomas")
    return x


# ---------------------------------------------------------------------------
# Whole runs
# ---------------------------------------------------------------------------

def response(p, plasma_eps=None, jb=None, diag: bool = False):
    """Load the plasma and run one plasma response for beam current jb
    (analytic Eq. (12) current when jb is None)."""
    st = load_plasma(p, plasma_eps)
    if jb is None:
        jb = beam_current_analytic(p)
    fields, cnt, d = march(p, st, jb, diag=diag)
    return {"state": st, "fields": fields, "counters": cnt, "diag": d, "jb": jb}


def cycle(p, plasma_eps, beam_eps, n_steps: int, frozen_after_first: bool = False):
    """Quasi-static cycle (Section II A: plasma response for the frozen beam,
    then the beam advanced in t), repeated n_steps times.  With
    frozen_after_first, one response is followed by n_steps pushes in its
    fields.  Returns the final beam, the last fields and diagnostics."""
    b = load_beam(p, beam_eps)
    g_init = beam_gamma(b)
    nout_dep = 0
    nout_push = 0
    counters = np.zeros(3, dtype=np.int64)
    fields = None
    if frozen_after_first:
        jb, nout_dep = beam_current_macro(p, b)
        st = load_plasma(p, plasma_eps)
        fields, cnt, _ = march(p, st, jb)
        counters += cnt
        nout_push = beam_push(p, b, fields, n_steps, p.dt)
    else:
        for _ in range(n_steps):
            jb, n1 = beam_current_macro(p, b)
            nout_dep += n1
            st = load_plasma(p, plasma_eps)
            fields, cnt, _ = march(p, st, jb)
            counters += cnt
            nout_push += beam_push(p, b, fields, 1, p.dt)
    return {"beam": b, "gamma_init": g_init, "fields": fields, "counters": counters,
            "n_out_deposit": nout_dep, "n_out_push": nout_push,
            "witness_gain": mean_gain(b, g_init, 1) if len(p.bunches) > 1 else None}


# ---------------------------------------------------------------------------
# Differentiable objective and its finite-difference gradient
# ---------------------------------------------------------------------------

def objective(p, n_steps: Optional[int] = None) -> float:
    """Witness mean gamma gain after one plasma response and n_steps beam
    steps in its frozen fields (Section II A cycle with the fields held), for
    the seeded draws of p."""
    from paper_1411_3246_amd import inputs
    n = p.n_steps if n_steps is None else n_steps
    r = cycle(p, inputs.plasma_draws(p), inputs.beam_draws(p), n, frozen_after_first=True)
    return r["witness_gain"]


def fd_gradient(p, rel_h: float = 1e-4, n_steps: Optional[int] = None,
                richardson: bool = True, which=None):
    """Central finite differences of objective() in each theta component
    (inputs.theta_of) with step rel_h |theta_i|; with richardson, the
    estimates at h and h/2 are combined, (4 D(h/2) - D(h)) / 3, and the
    difference between the two is returned as the truncation estimate."""
    from paper_1411_3246_amd import inputs
    th = inputs.theta_of(p)
    g = np.zeros(len(th))
    err = np.zeros(len(th))
    for i in (range(len(th)) if which is None else which):
        h = rel_h * abs(th[i])

        def central(hh):
            tp = th.copy(); tp[i] += hh
            tm = th.copy(); tm[i] -= hh
            return (objective(inputs.with_theta(p, tp), n_steps)
                    - objective(inputs.with_theta(p, tm), n_steps)) / (2.0 * hh)

        d1 = central(h)
        if richardson:
            d2 = central(0.5 * h)
            g[i] = (4.0 * d2 - d1) / 3.0
            err[i] = abs(d2 - d1)
        else:
            g[i] = d1
    return g, err
