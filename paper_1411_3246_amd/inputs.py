"""Seeded synthetic inputs: problem descriptions and random draws.

This module is the only code shared by the HIP path and the CPU oracle.  It
holds none of the method's arithmetic: it describes problems (plasma,
bunches, grid, window) with the parameters named in the WAKE paper
(arXiv:1411.3246, Section II B Eq. (12) and Table I) and draws the seeded
random numbers that both sides take as inputs (standard normals; the
loaders turn them into particles).

Workload recipe (all inputs synthetic, no data files):
  * plasma: uniform density n0 = 1, thermal momenta u_th * N(0, 1) per
    component, drawn per mirrored particle pair;
  * beam: Eq. (12) two-bunch electron driver (drive + witness with a common
    sigma_r), macroparticles drawn from standard normals truncated to
    |eps| <= 3.5 (so every particle starts inside the window), energy
    gamma0 * (1 + rel_spread * eps), zero emittance.
"""
from __future__ import annotations

import dataclasses
import json
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

TRUNC = 3.5  # truncation of the standard normals used for beam positions


@dataclass
class Bunch:
    n_peak: float       # peak density in units of n_p
    sigma_z: float      # rms length in k_p^-1
    xi_c: float         # centre in xi (k_p^-1 behind the window head)


@dataclass
class Problem:
    """One plasma-response problem (normalized units: k_p^-1, n_p, m_e c)."""
    name: str = "problem"
    geom: str = "cyl"            # "cyl" (r-xi) or "slab" (x-xi, half domain)
    n_r: int = 128
    r_max: float = 6.0
    n_xi: int = 512
    xi_min: float = 0.0
    xi_max: float = 10.0
    ppc: int = 4
    u_th: float = 0.0
    n0: float = 1.0
    sigma_r: float = 0.5
    bunches: List[Bunch] = field(default_factory=list)
    d_min: float = 0.05
    # beam macroparticles (0 = fixed analytic beam current from Eq. (12))
    n_beam: int = 0
    n_drive: int = 0
    gamma0: float = 4.0e4
    rel_spread: float = 1.0e-3
    n_steps: int = 0             # beam steps (plasma response + push) per run
    dt: float = 40.0
    prec: str = "fp64"           # "fp64" or "mixed"
    seed: int = 0

    @property
    def n_plasma(self) -> int:
        return self.n_r * self.ppc

    @property
    def n_pairs(self) -> int:
        return self.n_plasma // 2 if self.u_th > 0 else 0

    @property
    def dxi(self) -> float:
        return (self.xi_max - self.xi_min) / self.n_xi

    def updates_per_response(self) -> int:
        """Plasma particle-slice updates in one response (n_p * (n_xi - 1))."""
        return self.n_plasma * (self.n_xi - 1)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)

    def to_json(self) -> str:
        return json.dumps(dataclasses.asdict(self))


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

# Witness length from the Table I ratio sigma_zw / sigma_zd = 0.81 / 1.44.
def _witness_for(q_ratio: float, n_d: float, sigma_zd: float, sep: float,
                 xi_d: float) -> Bunch:
    sigma_zw = sigma_zd * (0.81 / 1.44)
    # equal sigma_r: charge ratio = (n_w sigma_zw) / (n_d sigma_zd)
    n_w = q_ratio * n_d * sigma_zd / sigma_zw
    return Bunch(n_w, sigma_zw, xi_d + sep)


def weak_single_bunch(n_b0: float = 0.1, **kw) -> Problem:
    """Cold plasma, fixed single Gaussian bunch, 128 x 512 cylindrical grid,
    4 ring particles per cell, FP64 (the linear-regime closed-form case)."""
    p = Problem(name="weak-single-bunch-128x512", geom="cyl", n_r=128, r_max=6.0,
                n_xi=512, xi_min=0.0, xi_max=10.0, ppc=4, u_th=0.0, sigma_r=0.5,
                bunches=[Bunch(n_b0, 1.0, 4.0)], prec="fp64", seed=0)
    return p.replace(**kw)


def facet_two_bunch(n_r: int = 512, n_xi: int = 4096, ppc: int = 16, u_th: float = 0.02,
                    sep: float = 4.5, n_beam: int = 1_000_000, n_steps: int = 200,
                    prec: str = "mixed", geom: str = "cyl", r_max: float = 6.0,
                    n_d: float = 8.0, sigma_r: float = 0.3, sigma_zd: float = 0.7,
                    xi_d: float = 2.5, q_ratio: float = 0.3, seed: int = 0,
                    name: Optional[str] = None) -> Problem:
    """Blowout-regime two-bunch driver (drive n_d = 8, sigma_r = 0.3,
    sigma_zd = 0.7; witness with 0.3 of the drive charge, sep behind),
    warm plasma, evolving macroparticle beam at gamma = 4e4."""
    wit = _witness_for(q_ratio, n_d, sigma_zd, sep, xi_d)
    n_drive = int(round(n_beam / (1.0 + q_ratio))) if n_beam else 0
    return Problem(name=name or f"two-bunch-{geom}-{n_r}x{n_xi}-ppc{ppc}",
                   geom=geom, n_r=n_r, r_max=r_max, n_xi=n_xi, xi_min=0.0, xi_max=10.0,
                   ppc=ppc, u_th=u_th, sigma_r=sigma_r,
                   bunches=[Bunch(n_d, sigma_zd, xi_d), wit], n_beam=n_beam,
                   n_drive=n_drive, gamma0=4.0e4, rel_spread=1.0e-3,
                   n_steps=n_steps, dt=40.0, prec=prec, seed=seed)


def blowout_response() -> Problem:
    """512 x 4096 cylindrical, 16 ppc, u_th = 0.02, 1e6 beam particles,
    200 beam steps, FP32 bulk / FP64 solve (the headline workload)."""
    return facet_two_bunch(name="two-bunch-512x4096-ppc16-beam1e6")


def gradient_case(n_d: float = 8.0) -> Problem:
    """256 x 2048, 16 ppc, 2e5 beam particles, one response + 20 steps in
    its frozen fields, FP64 (the differentiable objective)."""
    return facet_two_bunch(n_r=256, n_xi=2048, ppc=16, n_beam=200_000, n_steps=20, n_d=n_d,
                           prec="fp64", name="two-bunch-256x2048-ppc16-beam2e5")


def convergence_cyl() -> Problem:
    return facet_two_bunch(n_r=2048, n_xi=16384, ppc=64, n_beam=4_000_000, n_steps=100,
                           name="two-bunch-2048x16384-ppc64-beam4e6")


def convergence_slab() -> Problem:
    return facet_two_bunch(n_r=2048, n_xi=8192, ppc=64, n_beam=4_000_000, n_steps=100,
                           geom="slab", r_max=8.0, name="two-bunch-slab-2048x8192-ppc64")


# Table I two-bunch driver in normalized units (n_p = 5e16 cm^-3, k_p^-1 = 23.7 um):
# drive n = 3.56, sigma_z = 1.44; witness n = 2.85, sigma_z = 0.81, 5.48 behind;
# common sigma_r = 0.42.
TABLE1 = dict(n_d=3.56, n_w=2.85, sigma_r=0.42, sigma_zd=1.44, sigma_zw=0.81, sep=5.48)
MC2_EV = 510998.95


def u_th_of(t_e_ev: float) -> float:
    """Thermal momentum spread per component (units of m_e c) of a plasma at
    temperature T_e: u_th = sqrt(k T_e / m_e c^2)."""
    return (t_e_ev / MC2_EV) ** 0.5 if t_e_ev > 0 else 0.0


def facet_table1(t_e_ev: float = 0.0, n_r: int = 256, n_xi: int = 1400, ppc: int = 16,
                 r_max: float = 6.0, xi_max: float = 14.0, prec: str = "mixed",
                 seed: int = 0) -> Problem:
    """The Table I FACET-like two-bunch driver as a fixed (analytic) beam on a
    window [0, xi_max) with the drive centred 3.5 sigma_zd behind its head,
    in a plasma at temperature t_e_ev (eV); ppc is made even when warm."""
    t = TABLE1
    xi_d = 3.5 * t["sigma_zd"]
    u = u_th_of(t_e_ev)
    if u > 0 and ppc % 2:
        ppc += 1
    return Problem(name=f"table1-T{t_e_ev:g}eV-{n_r}x{n_xi}", geom="cyl", n_r=n_r, r_max=r_max, n_xi=n_xi,
                   xi_min=0.0, xi_max=xi_max, ppc=ppc, u_th=u, sigma_r=t["sigma_r"],
                   bunches=[Bunch(t["n_d"], t["sigma_zd"], xi_d), Bunch(t["n_w"], t["sigma_zw"], xi_d + t["sep"])],
                   n_beam=0, n_steps=0, prec=prec, seed=seed)


def facet_table1_beam(t_e_ev: float = 0.0, n_r: int = 256, n_xi: int = 2800, ppc: int = 16,
                      n_beam: int = 1_000_000, length_m: float = 1.14, dt: float = 40.0,
                      prec: str = "mixed", seed: int = 0) -> Problem:
    """The Table I driver as beam macroparticles (energy 4e4 m_e c^2, 0.1 %
    spread, zero emittance) evolved over `length_m` metres of plasma at
    n_p = 5e16 cm^-3 (k_p^-1 = 23.7 um) in steps of dt."""
    p = facet_table1(t_e_ev, n_r=n_r, n_xi=n_xi, ppc=ppc, prec=prec, seed=seed)
    t = TABLE1
    q_ratio = (t["n_w"] * t["sigma_zw"]) / (t["n_d"] * t["sigma_zd"])
    steps = int(round(length_m / 23.7e-6 / dt))
    return p.replace(name=f"table1-beam-T{t_e_ev:g}eV-{n_r}x{n_xi}", n_beam=n_beam,
                     n_drive=int(round(n_beam / (1.0 + q_ratio))), gamma0=4.0e4, rel_spread=1.0e-3,
                     n_steps=steps, dt=dt)


def te_scan_instances(temps=(0.0, 1.0, 2.0, 5.0, 10.0, 20.0, 30.0), ladder=(700, 1400, 2800, 5600),
                      ladder_temps=(0.0, 5.0), n_r: int = 256, n_xi: int = 2800, ppc: int = 16,
                      prec: str = "mixed") -> List[Problem]:
    """The temperature scan of the Table I driver at one resolution, and the
    slice-spacing ladder for a cold and a 5 eV plasma (duplicates dropped)."""
    out, seen = [], set()
    for te in temps:
        key = (te, n_xi)
        seen.add(key)
        out.append(facet_table1(te, n_r=n_r, n_xi=n_xi, ppc=ppc, prec=prec))
    for te in ladder_temps:
        for nx in ladder:
            if (te, nx) in seen:
                continue
            seen.add((te, nx))
            out.append(facet_table1(te, n_r=n_r, n_xi=nx, ppc=ppc, prec=prec))
    return out


def scan_instances(n: int = 256, seed: int = 0, prec: str = "mixed") -> List[Problem]:
    """Parameter scan of independent fixed-beam instances with uneven sizes:
    u_th ~ U[0, 0.05], separation ~ U[3, 6], n_r in {128, 256, 512, 1024},
    n_xi ~ U{1024..4096}, ppc in {8, 10, ..., 32}."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        u_th = float(rng.uniform(0.0, 0.05))
        sep = float(rng.uniform(3.0, 6.0))
        n_r = int(rng.choice([128, 256, 512, 1024]))
        n_xi = int(rng.integers(1024, 4097))
        ppc = int(rng.choice(np.arange(8, 33, 2)))
        out.append(facet_two_bunch(n_r=n_r, n_xi=n_xi, ppc=ppc, u_th=u_th, sep=sep,
                                   n_beam=0, n_steps=0, prec=prec, seed=seed * 100003 + i,
                                   name=f"scan-{i}"))
    return out


# ---------------------------------------------------------------------------
# Parameters of the differentiable objective
# ---------------------------------------------------------------------------

THETA_NAMES = ("n_drive", "sigma_r", "sigma_z_drive", "separation", "u_th")


def theta_of(p: Problem) -> np.ndarray:
    """theta = (drive peak density, common sigma_r, drive sigma_z, witness
    separation behind the drive, thermal spread u_th) of a two-bunch problem.
    The drive peak density carries the drive charge at fixed widths; the
    witness keeps its own peak density and length."""
    d, w = p.bunches[0], p.bunches[1]
    return np.array([d.n_peak, p.sigma_r, d.sigma_z, w.xi_c - d.xi_c, p.u_th])


def with_theta(p: Problem, theta) -> Problem:
    """The problem p with the parameters theta (see theta_of); the random
    draws of both loaders depend only on the seed, so they stay fixed."""
    t = [float(v) for v in theta]
    d, w = p.bunches[0], p.bunches[1]
    return p.replace(sigma_r=t[1], u_th=t[4],
                     bunches=[Bunch(t[0], t[2], d.xi_c), Bunch(w.n_peak, w.sigma_z, d.xi_c + t[3])])


# ---------------------------------------------------------------------------
# Random draws (inputs to both loaders)
# ---------------------------------------------------------------------------

def _truncated_normals(rng: np.random.Generator, shape: Tuple[int, ...]) -> np.ndarray:
    out = rng.standard_normal(shape)
    bad = np.abs(out) > TRUNC
    while bad.any():
        out[bad] = rng.standard_normal(int(bad.sum()))
        bad = np.abs(out) > TRUNC
    return out


def plasma_draws(p: Problem, stream: int = 0) -> Optional[np.ndarray]:
    """Three standard normals per mirrored particle pair, shape (n_pairs, 3),
    or None for a cold plasma."""
    if p.u_th <= 0:
        return None
    rng = np.random.default_rng([p.seed, 1, stream])
    return np.ascontiguousarray(rng.standard_normal((p.n_pairs, 3)))


def beam_draws(p: Problem, stream: int = 0) -> Optional[np.ndarray]:
    """Four truncated standard normals per beam macroparticle (x, y, xi,
    energy), shape (n_beam, 4), or None for a fixed analytic beam."""
    if p.n_beam <= 0:
        return None
    rng = np.random.default_rng([p.seed, 2, stream])
    return np.ascontiguousarray(_truncated_normals(rng, (p.n_beam, 4)))


WORKLOADS = {
    "weak-single-bunch": weak_single_bunch,
    "blowout": blowout_response,
    "gradient": gradient_case,
    "convergence-cyl": convergence_cyl,
    "convergence-slab": convergence_slab,
}
