"""Python binding of libwake (include/wake.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm); every step of the
computation runs in the HIP kernels of libwake.so.  The binding refuses to
run when the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwake.so")

WK_CYL, WK_SLAB = 0, 1
WK_FP64, WK_MIXED = 0, 1
COUNTER_NAMES = ["d_clamp", "wall", "nonfinite", "beam_out_deposit", "beam_out_push", "beam_bin",
                 "pipeline_abort", "beam_order"]
NCOUNTERS = 8


class WakeError(RuntimeError):
    pass


class WkBunch(C.Structure):
    _fields_ = [("n_peak", C.c_double), ("sigma_z", C.c_double), ("xi_c", C.c_double)]


class WkProblem(C.Structure):
    _fields_ = [("geom", C.c_int32), ("n_r", C.c_int32), ("r_max", C.c_double),
                ("n_xi", C.c_int32), ("xi_min", C.c_double), ("xi_max", C.c_double),
                ("ppc", C.c_int32), ("u_th", C.c_double), ("n0", C.c_double),
                ("sigma_r", C.c_double), ("n_bunch", C.c_int32), ("bunch", WkBunch * 2),
                ("n_beam", C.c_int64), ("n_drive", C.c_int64), ("gamma0", C.c_double),
                ("rel_spread", C.c_double), ("prec", C.c_int32), ("d_min", C.c_double)]


class WkSizes(C.Structure):
    _fields_ = [("n_plasma", C.c_int64), ("n_nodes", C.c_int64), ("plasma_state", C.c_size_t),
                ("plasma_const", C.c_size_t), ("plasma_draws", C.c_size_t), ("nion", C.c_size_t),
                ("beam_current", C.c_size_t), ("fields", C.c_size_t), ("beam_state", C.c_size_t),
                ("beam_tag", C.c_size_t), ("beam_draws", C.c_size_t), ("workspace", C.c_size_t),
                ("counters", C.c_size_t)]


class WkPlasmaBufs(C.Structure):
    _fields_ = [("d_x", C.c_void_p), ("d_y", C.c_void_p), ("d_px", C.c_void_p),
                ("d_py", C.c_void_p), ("d_d0", C.c_void_p), ("d_w", C.c_void_p),
                ("d_nion", C.c_void_p)]


class WkBeamBufs(C.Structure):
    _fields_ = [("d_x", C.c_void_p), ("d_y", C.c_void_p), ("d_px", C.c_void_p),
                ("d_py", C.c_void_p), ("d_pz", C.c_void_p), ("d_xi", C.c_void_p),
                ("d_w", C.c_void_p), ("d_gamma_init", C.c_void_p), ("d_tag", C.c_void_p)]


EXPORTS = [
    "wk_version", "wk_status_string", "wk_plan_create", "wk_plan_destroy", "wk_plan_sizes",
    "wk_last_error", "wk_counters_zero", "wk_counters_read", "wk_init_plasma", "wk_init_beam",
    "wk_beam_current_analytic", "wk_beam_current", "wk_plasma_response", "wk_plan_set_threads",
    "wk_plan_threads", "wk_batch_desc_bytes", "wk_batch_workspace_size", "wk_batch_group", "wk_batch_describe",
    "wk_batch_response", "wk_batch_response_shape", "wk_beam_push", "wk_mean_gain", "wk_ez_peak",
    "wk_cycle_workspace_size", "wk_cycle", "wk_plan_set_group", "wk_plan_group", "wk_cycle_group",
    "wk_plasma_response_noalloc", "wk_plasma_response_traj", "wk_gain_histogram",
    "wk_direct_workspace_size", "wk_plasma_response_direct",
    "wk_gradient_workspace_size", "wk_gradient_forward", "wk_gradient_backward",
]

_NON_STATUS = {"wk_version", "wk_status_string", "wk_last_error", "wk_plan_destroy",
               "wk_plan_threads", "wk_batch_desc_bytes", "wk_batch_workspace_size",
               "wk_cycle_workspace_size", "wk_gradient_workspace_size", "wk_plan_group", "wk_cycle_group",
               "wk_direct_workspace_size", "wk_batch_group"}

_lib = None


def lib():
    """Load libwake.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise WakeError(f"{LIB_PATH} is missing: build it with paper_1411_3246_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER(WkProblem)
    L.wk_version.restype = C.c_char_p
    L.wk_status_string.restype = C.c_char_p
    L.wk_status_string.argtypes = [C.c_int]
    L.wk_last_error.restype = C.c_char_p
    L.wk_plan_create.argtypes = [P, C.POINTER(vp)]
    L.wk_plan_destroy.argtypes = [vp]
    L.wk_plan_destroy.restype = None
    L.wk_plan_sizes.argtypes = [vp, C.POINTER(WkSizes)]
    L.wk_plan_set_threads.argtypes = [vp, i32]
    L.wk_plan_threads.argtypes = [vp]
    L.wk_plan_threads.restype = i32
    L.wk_plan_set_group.argtypes = [vp, i32]
    L.wk_plan_group.argtypes = [vp]
    L.wk_plan_group.restype = i32
    L.wk_cycle_group.argtypes = [vp, i32]
    L.wk_cycle_group.restype = i32
    L.wk_counters_zero.argtypes = [vp, vp]
    L.wk_counters_read.argtypes = [vp, vp, vp]
    L.wk_init_plasma.argtypes = [vp, C.POINTER(WkPlasmaBufs), vp, vp]
    L.wk_init_beam.argtypes = [vp, C.POINTER(WkBeamBufs), vp, vp]
    L.wk_beam_current_analytic.argtypes = [vp, vp, vp]
    L.wk_beam_current.argtypes = [vp, C.POINTER(WkBeamBufs), vp, vp, vp, vp]
    L.wk_plasma_response.argtypes = [vp, C.POINTER(WkPlasmaBufs), vp, vp, vp, vp, vp]
    L.wk_plasma_response_noalloc.argtypes = [vp, C.POINTER(WkPlasmaBufs), vp, vp, vp, vp]
    L.wk_plasma_response_traj.argtypes = [vp, C.POINTER(WkPlasmaBufs), vp, vp, vp, i32, vp, vp, vp]
    L.wk_gain_histogram.argtypes = [vp, C.POINTER(WkBeamBufs), i32, i32, d, d, vp, vp]
    L.wk_direct_workspace_size.argtypes = [vp]
    L.wk_direct_workspace_size.restype = C.c_size_t
    L.wk_plasma_response_direct.argtypes = [vp, C.POINTER(WkPlasmaBufs), vp, vp, vp, C.c_size_t, i32, d, vp, vp,
                                            vp]
    L.wk_batch_desc_bytes.argtypes = [i32]
    L.wk_batch_desc_bytes.restype = C.c_size_t
    L.wk_batch_workspace_size.argtypes = [i32, C.POINTER(vp)]
    L.wk_batch_workspace_size.restype = C.c_size_t
    L.wk_batch_group.argtypes = [i32, C.POINTER(vp), i32]
    L.wk_batch_group.restype = i32
    L.wk_batch_describe.argtypes = [i32, C.POINTER(vp), C.POINTER(WkPlasmaBufs), C.POINTER(vp),
                                    C.POINTER(vp), vp, C.c_size_t, vp, vp]
    L.wk_batch_response.argtypes = [i32, C.POINTER(vp), vp, vp, C.c_size_t, vp]
    L.wk_batch_response_shape.argtypes = [i32, C.POINTER(vp), vp, vp, C.c_size_t, i32, i32, vp]
    L.wk_gradient_workspace_size.argtypes = [vp, i32, i32]
    L.wk_gradient_workspace_size.restype = C.c_size_t
    L.wk_gradient_forward.argtypes = [vp, C.POINTER(WkPlasmaBufs), vp, C.POINTER(WkBeamBufs), vp, i32, d, i32,
                                      vp, vp, vp, C.c_size_t, vp, vp]
    L.wk_gradient_backward.argtypes = [vp, C.POINTER(WkPlasmaBufs), vp, C.POINTER(WkBeamBufs), vp, i32, d, i32,
                                       vp, vp, vp, vp, C.c_size_t, vp]
    L.wk_beam_push.argtypes = [vp, C.POINTER(WkBeamBufs), vp, i32, d, vp, vp]
    L.wk_mean_gain.argtypes = [vp, C.POINTER(WkBeamBufs), i32, vp, vp, vp]
    L.wk_ez_peak.argtypes = [vp, vp, d, vp, vp]
    L.wk_cycle_workspace_size.argtypes = [vp, i32]
    L.wk_cycle_workspace_size.restype = C.c_size_t
    L.wk_cycle.argtypes = [vp, C.POINTER(WkPlasmaBufs), C.POINTER(WkBeamBufs), i32, d, vp, vp,
                           C.c_size_t, vp, vp]
    for name in EXPORTS:
        if name not in _NON_STATUS:
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        L = lib()
        raise WakeError(f"{what}: {L.wk_status_string(rc).decode()} ({L.wk_last_error().decode()})")


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def problem_struct(p: inputs.Problem) -> WkProblem:
    s = WkProblem()
    s.geom = WK_CYL if p.geom == "cyl" else WK_SLAB
    s.n_r, s.r_max, s.n_xi = p.n_r, p.r_max, p.n_xi
    s.xi_min, s.xi_max = p.xi_min, p.xi_max
    s.ppc, s.u_th, s.n0 = p.ppc, p.u_th, p.n0
    s.sigma_r = p.sigma_r
    s.n_bunch = len(p.bunches)
    for b, bb in enumerate(p.bunches):
        s.bunch[b].n_peak, s.bunch[b].sigma_z, s.bunch[b].xi_c = bb.n_peak, bb.sigma_z, bb.xi_c
    s.n_beam, s.n_drive = p.n_beam, p.n_drive
    s.gamma0, s.rel_spread = p.gamma0, p.rel_spread
    s.prec = WK_FP64 if p.prec == "fp64" else WK_MIXED
    s.d_min = p.d_min
    return s


class Plan:
    """A validated problem and its launch shape (host-only)."""

    def __init__(self, problem: inputs.Problem, threads: Optional[int] = None, group: Optional[int] = None):
        self.problem = problem
        self._s = problem_struct(problem)
        h = C.c_void_p()
        _check(lib().wk_plan_create(C.byref(self._s), C.byref(h)), "wk_plan_create")
        self.handle = h
        if threads is not None:
            _check(lib().wk_plan_set_threads(self.handle, threads), "wk_plan_set_threads")
        if group is not None:
            _check(lib().wk_plan_set_group(self.handle, group), "wk_plan_set_group")
        sz = WkSizes()
        _check(lib().wk_plan_sizes(self.handle, C.byref(sz)), "wk_plan_sizes")
        self.sizes = sz

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.wk_plan_destroy(self.handle)
            self.handle = None

    @property
    def threads(self) -> int:
        return lib().wk_plan_threads(self.handle)

    @property
    def group(self) -> int:
        """Workgroups that march one response of wk_plasma_response."""
        return lib().wk_plan_group(self.handle)

    def set_group(self, group: int):
        """Workgroups per response (0: the library's choice); the workspace
        size is updated."""
        _check(lib().wk_plan_set_group(self.handle, group), "wk_plan_set_group")
        sz = WkSizes()
        _check(lib().wk_plan_sizes(self.handle, C.byref(sz)), "wk_plan_sizes")
        self.sizes = sz

    def cycle_group(self, n_steps: int) -> int:
        """Workgroups per response that wk_cycle uses for n_steps steps."""
        return lib().wk_cycle_group(self.handle, n_steps)

    @property
    def real_dtype(self):
        import torch
        return torch.float64 if self.problem.prec == "fp64" else torch.float32

    # -- buffers (torch tensors on the current device) -------------------------
    def alloc_plasma(self, device="cuda") -> Dict:
        import torch
        n = self.problem.n_plasma
        t = {k: torch.zeros(n, dtype=torch.float64, device=device) for k in ("x", "y", "px", "py")}
        t["d0"] = torch.zeros(n, dtype=self.real_dtype, device=device)
        t["w"] = torch.zeros(n, dtype=self.real_dtype, device=device)
        t["nion"] = torch.zeros(self.problem.n_r + 1, dtype=torch.float64, device=device)
        return t

    def alloc_beam(self, device="cuda") -> Dict:
        import torch
        n = self.problem.n_beam
        t = {k: torch.zeros(n, dtype=torch.float64, device=device)
             for k in ("x", "y", "px", "py", "pz", "xi", "w", "gamma_init")}
        t["tag"] = torch.zeros(n, dtype=torch.int32, device=device)
        return t

    def alloc_fields(self, device="cuda"):
        import torch
        p = self.problem
        return torch.zeros((4, p.n_xi, p.n_r + 1), dtype=self.real_dtype, device=device)

    def alloc_jb(self, device="cuda"):
        import torch
        p = self.problem
        return torch.zeros((p.n_xi, p.n_r + 1), dtype=torch.float64, device=device)

    def alloc_workspace(self, device="cuda"):
        import torch
        return torch.zeros(self.sizes.workspace, dtype=torch.uint8, device=device)

    @staticmethod
    def alloc_counters(device="cuda"):
        import torch
        return torch.zeros(NCOUNTERS, dtype=torch.int64, device=device)

    @staticmethod
    def plasma_bufs(t: Dict) -> WkPlasmaBufs:
        b = WkPlasmaBufs()
        b.d_x, b.d_y, b.d_px, b.d_py = _ptr(t["x"]), _ptr(t["y"]), _ptr(t["px"]), _ptr(t["py"])
        b.d_d0, b.d_w, b.d_nion = _ptr(t["d0"]), _ptr(t["w"]), _ptr(t["nion"])
        return b

    @staticmethod
    def beam_bufs(t: Dict) -> WkBeamBufs:
        b = WkBeamBufs()
        b.d_x, b.d_y, b.d_px, b.d_py = _ptr(t["x"]), _ptr(t["y"]), _ptr(t["px"]), _ptr(t["py"])
        b.d_pz, b.d_xi, b.d_w = _ptr(t["pz"]), _ptr(t["xi"]), _ptr(t["w"])
        b.d_gamma_init, b.d_tag = _ptr(t["gamma_init"]), _ptr(t["tag"])
        return b

    # -- calls -----------------------------------------------------------------
    def init_plasma(self, plasma: Dict, draws=None, stream=None):
        b = self.plasma_bufs(plasma)
        _check(lib().wk_init_plasma(self.handle, C.byref(b), _ptr(draws), _stream(stream)),
               "wk_init_plasma")

    def init_beam(self, beam: Dict, draws, stream=None):
        b = self.beam_bufs(beam)
        _check(lib().wk_init_beam(self.handle, C.byref(b), _ptr(draws), _stream(stream)),
               "wk_init_beam")

    def beam_current_analytic(self, jb, stream=None):
        _check(lib().wk_beam_current_analytic(self.handle, _ptr(jb), _stream(stream)),
               "wk_beam_current_analytic")

    def beam_current(self, beam: Dict, jb, workspace, counters, stream=None):
        b = self.beam_bufs(beam)
        _check(lib().wk_beam_current(self.handle, C.byref(b), _ptr(jb), _ptr(workspace),
                                     _ptr(counters), _stream(stream)), "wk_beam_current")

    def plasma_response(self, plasma: Dict, jb, fields, workspace, counters, stream=None):
        b = self.plasma_bufs(plasma)
        _check(lib().wk_plasma_response(self.handle, C.byref(b), _ptr(jb), _ptr(fields),
                                        _ptr(workspace), _ptr(counters), _stream(stream)),
               "wk_plasma_response")

    def plasma_response_traj(self, plasma: Dict, jb, fields, workspace, stride: int, traj, counters,
                             stream=None):
        """wk_plasma_response recording the radius of every stride-th particle per slice."""
        b = self.plasma_bufs(plasma)
        _check(lib().wk_plasma_response_traj(self.handle, C.byref(b), _ptr(jb), _ptr(fields), _ptr(workspace),
                                             int(stride), _ptr(traj), _ptr(counters), _stream(stream)),
               "wk_plasma_response_traj")

    def plasma_response_direct(self, plasma: Dict, jb, fields, workspace, counters, iters: int = 8,
                               tol: float = 1e-10, iterations=None, stream=None):
        """The response with B_theta from Eq. (6) as written (Newton-GMRES per
        slice on the implicit d_xi E_z); workspace of wk_direct_workspace_size
        bytes; iterations: optional int32[n_xi] of Newton steps per slice."""
        b = self.plasma_bufs(plasma)
        _check(lib().wk_plasma_response_direct(self.handle, C.byref(b), _ptr(jb), _ptr(fields), _ptr(workspace),
                                               workspace.numel() * workspace.element_size(), int(iters),
                                               float(tol), _ptr(iterations), _ptr(counters), _stream(stream)),
               "wk_plasma_response_direct")

    def gain_histogram(self, beam: Dict, which: int, n_bins: int, lo: float, hi: float, hist, stream=None):
        """Counts of gamma - gamma_init in n_bins bins of [lo, hi) (+ under/overflow)."""
        b = self.beam_bufs(beam)
        _check(lib().wk_gain_histogram(self.handle, C.byref(b), int(which), int(n_bins), float(lo), float(hi),
                                       _ptr(hist), _stream(stream)), "wk_gain_histogram")

    def plasma_response_noalloc(self, plasma: Dict, jb, fields, counters, stream=None):
        """wk_plasma_response with the library's static scratch in place of a workspace."""
        b = self.plasma_bufs(plasma)
        _check(lib().wk_plasma_response_noalloc(self.handle, C.byref(b), _ptr(jb), _ptr(fields),
                                                _ptr(counters), _stream(stream)),
               "wk_plasma_response_noalloc")

    def beam_push(self, beam: Dict, fields, n_steps: int, dt: float, counters, stream=None):
        b = self.beam_bufs(beam)
        _check(lib().wk_beam_push(self.handle, C.byref(b), _ptr(fields), n_steps, dt,
                                  _ptr(counters), _stream(stream)), "wk_beam_push")

    def mean_gain(self, beam: Dict, which: int, out, workspace, stream=None):
        b = self.beam_bufs(beam)
        _check(lib().wk_mean_gain(self.handle, C.byref(b), which, _ptr(out), _ptr(workspace),
                                  _stream(stream)), "wk_mean_gain")

    def cycle_workspace_bytes(self, n_steps: int) -> int:
        return lib().wk_cycle_workspace_size(self.handle, n_steps)

    def cycle(self, plasma: Dict, beam: Dict, n_steps: int, dt: float, ring, workspace, counters,
              stream=None):
        p = self.plasma_bufs(plasma)
        b = self.beam_bufs(beam)
        _check(lib().wk_cycle(self.handle, C.byref(p), C.byref(b), n_steps, dt, _ptr(ring),
                              _ptr(workspace), workspace.numel(), _ptr(counters), _stream(stream)),
               "wk_cycle")

    def ez_peak(self, fields, xi_from: float, out, stream=None):
        _check(lib().wk_ez_peak(self.handle, _ptr(fields), xi_from, _ptr(out), _stream(stream)),
               "wk_ez_peak")


def zero_counters(counters, stream=None):
    _check(lib().wk_counters_zero(_ptr(counters), _stream(stream)), "wk_counters_zero")


def counters_dict(counters) -> Dict[str, int]:
    v = counters.cpu().numpy()
    return {k: int(v[i]) for i, k in enumerate(COUNTER_NAMES)}


def read_counters(counters, stream=None) -> Dict[str, int]:
    """Counters through the library's own read-back; raises WakeError when
    non-finite fields were stored or a pipelined cycle gave up waiting."""
    out = (C.c_uint64 * NCOUNTERS)()
    _check(lib().wk_counters_read(_ptr(counters), C.addressof(out), _stream(stream)), "wk_counters_read")
    return {k: int(out[i]) for i, k in enumerate(COUNTER_NAMES)}


# ---------------------------------------------------------------------------
# Batched responses
# ---------------------------------------------------------------------------

class Batch:
    """Independent plasma responses of many plans in one persistent launch."""

    def __init__(self, plans: Sequence[Plan], device="cuda"):
        import torch
        self.plans = list(plans)
        n = len(self.plans)
        self._handles = (C.c_void_p * n)(*[p.handle for p in self.plans])
        self.ws_bytes = lib().wk_batch_workspace_size(n, self._handles)
        if self.ws_bytes == 0:
            raise WakeError("wk_batch_workspace_size failed")
        self.workspace = torch.zeros(self.ws_bytes, dtype=torch.uint8, device=device)
        self.desc_bytes = lib().wk_batch_desc_bytes(n)
        self.desc = torch.zeros(self.desc_bytes, dtype=torch.uint8, device=device)
        self._described = False

    def describe(self, plasmas: Sequence[Dict], jbs, fields, counters):
        import torch
        n = len(self.plans)
        pb = (WkPlasmaBufs * n)(*[Plan.plasma_bufs(t) for t in plasmas])
        jbp = (C.c_void_p * n)(*[_ptr(j) for j in jbs])
        fp = (C.c_void_p * n)(*[_ptr(f) for f in fields])
        host = (C.c_uint8 * self.desc_bytes)()
        _check(lib().wk_batch_describe(n, self._handles, pb, jbp, fp, _ptr(self.workspace),
                                       self.ws_bytes, _ptr(counters), C.cast(host, C.c_void_p)),
               "wk_batch_describe")
        blob = torch.frombuffer(bytearray(host), dtype=torch.uint8)
        self.desc.copy_(blob)
        self._described = True

    def response(self, stream=None, threads: int = 0, wg_per_cu: int = 0):
        """March every instance; threads / wg_per_cu = 0 keep the defaults."""
        if not self._described:
            raise WakeError("Batch.describe must be called first")
        _check(lib().wk_batch_response_shape(len(self.plans), self._handles, _ptr(self.desc),
                                             _ptr(self.workspace), self.ws_bytes, int(threads),
                                             int(wg_per_cu), _stream(stream)),
               "wk_batch_response_shape")


# ---------------------------------------------------------------------------
# Convenience: the quasi-static cycle on one plan
# ---------------------------------------------------------------------------

class Simulation:
    """Buffers and calls of one problem: plasma response for the frozen beam,
    then the beam advanced over dt (Section II A of the WAKE paper)."""

    def __init__(self, problem: inputs.Problem, threads: Optional[int] = None, device="cuda",
                 group: Optional[int] = None):
        import torch
        self.problem = problem
        self.plan = Plan(problem, threads, group)
        self.device = device
        self.plasma = self.plan.alloc_plasma(device)
        self.fields = self.plan.alloc_fields(device)
        self.jb = self.plan.alloc_jb(device)
        self.workspace = self.plan.alloc_workspace(device)
        self.counters = self.plan.alloc_counters(device)
        self.out = torch.zeros(4, dtype=torch.float64, device=device)
        pd = inputs.plasma_draws(problem)
        self.plasma_draws = None if pd is None else torch.from_numpy(pd).to(device)
        self.beam = None
        if problem.n_beam > 0:
            self.beam = self.plan.alloc_beam(device)
            self.beam_draws = torch.from_numpy(inputs.beam_draws(problem)).to(device)
        zero_counters(self.counters)

    def load_beam(self):
        if self.beam is not None:
            self.plan.init_beam(self.beam, self.beam_draws)

    def beam_current(self):
        if self.beam is None:
            self.plan.beam_current_analytic(self.jb)
        else:
            self.plan.beam_current(self.beam, self.jb, self.workspace, self.counters)

    def response(self):
        """Load the plasma ahead of the beam and march it through the window."""
        self.plan.init_plasma(self.plasma, self.plasma_draws)
        self.plan.plasma_response(self.plasma, self.jb, self.fields, self.workspace, self.counters)

    def response_traj(self, stride: int):
        """response() recording the radius of every stride-th plasma particle per
        slice; returns the (n_xi, ceil(n_plasma / stride)) tensor."""
        import torch
        n = (self.problem.n_plasma + stride - 1) // stride
        traj = torch.zeros((self.problem.n_xi, n), dtype=torch.float64, device=self.jb.device)
        self.plan.init_plasma(self.plasma, self.plasma_draws)
        self.plan.plasma_response_traj(self.plasma, self.jb, self.fields, self.workspace, stride, traj,
                                       self.counters)
        return traj

    def response_direct(self, iters: int = 8, tol: float = 1e-10):
        """response() with B_theta from Eq. (6) as written; returns the Newton
        steps used per slice (int32 tensor of n_xi)."""
        import torch
        dev = self.jb.device
        ws = torch.zeros(lib().wk_direct_workspace_size(self.plan.handle), dtype=torch.uint8, device=dev)
        its = torch.zeros(self.problem.n_xi, dtype=torch.int32, device=dev)
        self.plan.init_plasma(self.plasma, self.plasma_draws)
        self.plan.plasma_response_direct(self.plasma, self.jb, self.fields, ws, self.counters, iters, tol, its)
        return its

    def gain_histogram(self, which: int, n_bins: int, lo: float, hi: float):
        """Energy spectrum of the beam (tag == which; all if which < 0): counts
        in n_bins bins of [lo, hi) with under/overflow at both ends."""
        import torch
        hist = torch.zeros(n_bins + 2, dtype=torch.int64, device=self.jb.device)
        self.plan.gain_histogram(self.beam, which, n_bins, lo, hi, hist)
        return hist

    def response_noalloc(self):
        """response() through the allocation-free entry point."""
        self.plan.init_plasma(self.plasma, self.plasma_draws)
        self.plan.plasma_response_noalloc(self.plasma, self.jb, self.fields, self.counters)

    def push(self, n_steps: int = 1, dt: Optional[float] = None):
        self.plan.beam_push(self.beam, self.fields, n_steps, self.problem.dt if dt is None else dt,
                            self.counters)

    def step(self):
        """One beam step: beam current -> plasma response -> beam push."""
        self.beam_current()
        self.response()
        if self.beam is not None:
            self.push(1)

    def run_cycle(self, n_steps: int, dt: Optional[float] = None):
        """n_steps quasi-static cycles (current -> response -> push) with the
        responses of successive steps pipelined across workgroups.  Afterwards
        `fields` holds the last response."""
        import torch
        if self.beam is None:
            raise WakeError("run_cycle needs beam macroparticles")
        if getattr(self, "ring", None) is None:
            self.ring = torch.zeros((2,) + tuple(self.fields.shape), dtype=self.fields.dtype,
                                    device=self.device)
        need = self.plan.cycle_workspace_bytes(n_steps)
        if getattr(self, "cycle_ws", None) is None or self.cycle_ws.numel() < need:
            self.cycle_ws = torch.zeros(need, dtype=torch.uint8, device=self.device)
        self.plan.init_plasma(self.plasma, self.plasma_draws)
        self.plan.cycle(self.plasma, self.beam, n_steps, self.problem.dt if dt is None else dt,
                        self.ring, self.cycle_ws, self.counters)
        self.fields = self.ring[(n_steps - 1) % 2]

    def witness_gain(self) -> float:
        self.plan.mean_gain(self.beam, 1, self.out[0:1], self.workspace)
        return float(self.out[0].item())

    def ez_peak(self, xi_from: float) -> float:
        self.plan.ez_peak(self.fields, xi_from, self.out[1:2])
        return float(self.out[1].item())

    def counters_dict(self):
        return counters_dict(self.counters)


# ---------------------------------------------------------------------------
# Convenience: a parameter scan of fixed-beam instances in one launch
# ---------------------------------------------------------------------------

class Scan:
    """Independent fixed-beam plasma responses (any mix of grid sizes,
    temperatures and separations; one geometry and precision) with their
    buffers, run as one persistent batched launch.

    run() loads every plasma and marches all instances; run_one(i) marches
    instance i alone with the standalone entry point (the per-instance
    baseline of the batched launch); capture() records run() in a HIP graph."""

    def __init__(self, problems: Sequence[inputs.Problem], device="cuda"):
        import torch
        self.problems = list(problems)
        self.device = device
        self.plans = [Plan(q) for q in self.problems]
        self.plasma = [pl.alloc_plasma(device) for pl in self.plans]
        self.draws = []
        for q in self.problems:
            d = inputs.plasma_draws(q)
            self.draws.append(None if d is None else torch.from_numpy(d).to(device))
        self.jb = [pl.alloc_jb(device) for pl in self.plans]
        self.fields = [pl.alloc_fields(device) for pl in self.plans]
        self.counters = Plan.alloc_counters(device)
        ws = max(pl.sizes.workspace for pl in self.plans)
        self.workspace = torch.zeros(ws, dtype=torch.uint8, device=device)
        zero_counters(self.counters)
        for pl, jb in zip(self.plans, self.jb):
            pl.beam_current_analytic(jb)
        self.batch = Batch(self.plans, device)
        self.batch.describe(self.plasma, self.jb, self.fields, self.counters)
        self.threads = 0
        self.wg_per_cu = 0
        self.member_cap = 0
        self.graph = None

    def set_member_cap(self, cap: int):
        """Re-plan the batch so that no workgroup holds more than `cap`
        particles: instance i gets G_i = max(ceil(n_p / cap), ceil(cost_i /
        (total / compute units))) workgroups, at most 16 and n_r, with
        total = sum of n_p n_xi and cost_i = n_p n_xi n_r / (largest n_r):
        every member repeats the grid work of a slice, so instances with
        smaller grids are spread over fewer members.  cap = 0 restores the
        library's schedule (the same rule with cap 8192).  Drops a captured
        graph."""
        import math
        import torch
        if cap < 0:
            raise WakeError("member cap must be >= 0")
        cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
        total = sum(float(q.n_plasma) * q.n_xi for q in self.problems)
        per_cu = total / max(1, cus)
        nr_max = max(q.n_r for q in self.problems)
        for q, pl in zip(self.problems, self.plans):
            if cap == 0:
                pl.set_group(0)
                continue
            cost = float(q.n_plasma) * q.n_xi * q.n_r / nr_max
            g = max(math.ceil(q.n_plasma / cap), math.ceil(cost / per_cu))
            pl.set_group(max(1, min(g, 16, q.n_r)))
        ws = max(pl.sizes.workspace for pl in self.plans)
        if ws > self.workspace.numel():
            self.workspace = torch.zeros(ws, dtype=torch.uint8, device=self.device)
        self.batch = Batch(self.plans, self.device)
        self.batch.describe(self.plasma, self.jb, self.fields, self.counters)
        self.member_cap = cap
        self.graph = None

    @property
    def groups(self) -> List[int]:
        """Workgroups per instance of the current schedule (plan choice or
        the library's)."""
        return [int(lib().wk_batch_group(len(self.plans), self.batch._handles, i)) for i in range(len(self.plans))]

    @property
    def updates(self) -> int:
        """Plasma particle-slice updates of one pass over every instance."""
        return sum(q.updates_per_response() for q in self.problems)

    def load(self, stream=None):
        for pl, t, d in zip(self.plans, self.plasma, self.draws):
            pl.init_plasma(t, d, stream)

    def run(self, stream=None):
        self.load(stream)
        self.batch.response(stream, self.threads, self.wg_per_cu)

    def run_one(self, i: int, stream=None):
        pl = self.plans[i]
        pl.init_plasma(self.plasma[i], self.draws[i], stream)
        pl.plasma_response(self.plasma[i], self.jb[i], self.fields[i], self.workspace,
                           self.counters, stream)

    def capture(self):
        """Record run() (plasma loads, queue reset, batched march) in a HIP
        graph; replay() then submits the whole pass at once."""
        import torch
        self.run()                          # first use sets kernel attributes
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise WakeError("Scan.capture must be called first")
        self.graph.replay()


# ---------------------------------------------------------------------------
# Differentiable objective: witness gain after one response + frozen pushes
# ---------------------------------------------------------------------------

class GradientRun:
    """Buffers of one evaluation of the witness-gain objective and of its
    reverse-mode gradient (wk_gradient_forward / wk_gradient_backward).
    The problem must be FP64 with a two-bunch macroparticle beam."""

    def __init__(self, problem: inputs.Problem, n_steps: Optional[int] = None, every: int = 64,
                 device="cuda", threads: Optional[int] = None, group: Optional[int] = None):
        """group: workgroups of the reverse march (None: the library's
        choice, about two particles per thread and workgroup, at most 8)."""
        import torch
        self.problem = problem
        self.n_steps = problem.n_steps if n_steps is None else int(n_steps)
        self.every = int(every)
        self.plan = Plan(problem, threads)
        if group is not None:
            self.plan.set_group(int(group))
        self.device = device
        self.plasma = self.plan.alloc_plasma(device)
        self.beam = self.plan.alloc_beam(device)
        self.fields = self.plan.alloc_fields(device)
        self.counters = self.plan.alloc_counters(device)
        pd = inputs.plasma_draws(problem)
        self.plasma_draws = None if pd is None else torch.from_numpy(pd).to(device)
        self.beam_draws = torch.from_numpy(inputs.beam_draws(problem)).to(device)
        self.ws_bytes = lib().wk_gradient_workspace_size(self.plan.handle, self.n_steps, self.every)
        if self.ws_bytes == 0:
            raise WakeError("wk_gradient_workspace_size: " + lib().wk_last_error().decode())
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.out = torch.zeros(1, dtype=torch.float64, device=device)
        self.grad = torch.zeros(5, dtype=torch.float64, device=device)
        self.gbar = torch.ones(1, dtype=torch.float64, device=device)
        zero_counters(self.counters)

    def forward(self, stream=None):
        """Objective G on the device (self.out[0])."""
        pb = self.plan.plasma_bufs(self.plasma)
        bb = self.plan.beam_bufs(self.beam)
        _check(lib().wk_gradient_forward(self.plan.handle, C.byref(pb), _ptr(self.plasma_draws), C.byref(bb),
                                         _ptr(self.beam_draws), self.n_steps, float(self.problem.dt),
                                         self.every, _ptr(self.fields), _ptr(self.out), _ptr(self.workspace),
                                         self.ws_bytes, _ptr(self.counters), _stream(stream)),
               "wk_gradient_forward")
        return self.out

    def backward(self, gbar=None, stream=None):
        """d_gbar * dG/dtheta on the device (self.grad), theta in the order of
        inputs.THETA_NAMES."""
        if gbar is not None:
            self.gbar.copy_(gbar.reshape(1).to(self.gbar))
        pb = self.plan.plasma_bufs(self.plasma)
        bb = self.plan.beam_bufs(self.beam)
        _check(lib().wk_gradient_backward(self.plan.handle, C.byref(pb), _ptr(self.plasma_draws), C.byref(bb),
                                          _ptr(self.beam_draws), self.n_steps, float(self.problem.dt),
                                          self.every, _ptr(self.fields), _ptr(self.gbar), _ptr(self.grad),
                                          _ptr(self.workspace), self.ws_bytes, _stream(stream)),
               "wk_gradient_backward")
        return self.grad


def _witness_gain_function():
    import torch

    class WitnessGain(torch.autograd.Function):
        """G(theta): witness mean gamma gain after one plasma response and
        n_steps beam steps in its frozen fields, theta = (drive peak density,
        sigma_r, drive sigma_z, separation, u_th).  Forward and backward run
        the library's recording march and its hand-written adjoint."""

        @staticmethod
        def forward(ctx, theta, base, n_steps, every):
            p = inputs.with_theta(base, theta.detach().cpu().tolist())
            run = GradientRun(p, n_steps, every, device="cuda")
            g = run.forward().clone()
            ctx.run = run
            ctx.theta_device = theta.device
            return g.reshape(())

        @staticmethod
        def backward(ctx, gout):
            grad = ctx.run.backward(gout.detach().reshape(1).to("cuda", torch.float64)).clone()
            return grad.to(ctx.theta_device), None, None, None

    return WitnessGain


_WG = None


def witness_gain(theta, base: inputs.Problem, n_steps: Optional[int] = None, every: int = 64):
    """Differentiable witness gain (torch.autograd) of the two-bunch problem
    `base` with its parameters replaced by theta."""
    global _WG
    if _WG is None:
        _WG = _witness_gain_function()
    return _WG.apply(theta, base, base.n_steps if n_steps is None else n_steps, every)
