"""Linear-regime closed form of the wake of a weak Gaussian bunch.

Derived from the model of the WAKE paper (arXiv:1411.3246, Section II A,
Eqs. (1)-(7)) linearized in the beam density n_b for a cold plasma:
  (d_xi^2 + 1) dn = -n_b,   (lap_perp - 1) psi = dn,   E_z = d_xi psi,
  B_theta = n_b0 R'(r) G(xi),  E_r - B_theta = -d_r psi,
for n_b = n_b0 exp(-r^2/2 s_r^2) G(xi), G = exp(-(xi - xi0)^2 / 2 s_z^2),
with the beam switched on at xi = xi_min (the head of the window) and
psi(r_max) = 0:
  psi = n_b0 R(r) Zs(xi),  E_z = n_b0 R(r) Zc(xi),
  R(r) = int_0^{r_max} r' g(r, r') exp(-r'^2 / 2 s_r^2) dr',
  g = I0(r<) K0(r>) - K0(r_max)/I0(r_max) I0(r) I0(r'),
  Zs, Zc = int_{xi_min}^{xi} {sin, cos}(xi - xi') G(xi') dxi'.
Evaluated with SciPy quadrature and Bessel functions (independent of the
oracle).
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, special


def radial_profile(r: np.ndarray, sigma_r: float, r_max: float):
    """R(r) and R'(r) on the points r."""
    c = special.k0(r_max) / special.i0(r_max)

    def g(rr, rp):
        lo, hi = min(rr, rp), max(rr, rp)
        return special.i0(lo) * special.k0(hi) - c * special.i0(rr) * special.i0(rp)

    def dg(rr, rp):  # d/dr of g(r, r')
        if rr < rp:
            return special.i1(rr) * special.k0(rp) - c * special.i1(rr) * special.i0(rp)
        return -special.i0(rp) * special.k1(rr) - c * special.i1(rr) * special.i0(rp)

    R = np.zeros(len(r))
    dR = np.zeros(len(r))
    for i, rr in enumerate(r):
        pts = [rr] if 0.0 < rr < r_max else None
        src = lambda rp: rp * np.exp(-rp * rp / (2 * sigma_r ** 2))
        R[i] = integrate.quad(lambda rp: src(rp) * g(rr, rp), 0.0, r_max, points=pts,
                              limit=400, epsabs=1e-15, epsrel=1e-12)[0]
        dR[i] = integrate.quad(lambda rp: src(rp) * dg(rr, rp), 0.0, r_max, points=pts,
                               limit=400, epsabs=1e-15, epsrel=1e-12)[0]
    return R, dR


def longitudinal(xi: np.ndarray, xi0: float, sigma_z: float, xi_min: float = 0.0):
    """G(xi), Zs(xi), Zc(xi)."""
    G = lambda x: np.exp(-(x - xi0) ** 2 / (2 * sigma_z ** 2))
    Zs = np.array([integrate.quad(lambda t: np.sin(x - t) * G(t), xi_min, x, epsabs=1e-15,
                                  limit=200)[0] for x in xi])
    Zc = np.array([integrate.quad(lambda t: np.cos(x - t) * G(t), xi_min, x, epsabs=1e-15,
                                  limit=200)[0] for x in xi])
    return G(xi), Zs, Zc


def fields(p):
    """Closed-form psi, E_z, B_theta, W on the problem's (xi_k, r_j) nodes,
    each of shape (n_xi, n_r + 1), for a single-bunch problem."""
    b = p.bunches[0]
    r = np.arange(p.n_r + 1) * (p.r_max / p.n_r)
    xi = p.xi_min + np.arange(p.n_xi) * p.dxi
    R, dR = radial_profile(r, p.sigma_r, p.r_max)
    G, Zs, Zc = longitudinal(xi, b.xi_c, b.sigma_z, p.xi_min)
    n = b.n_peak
    psi = n * np.outer(Zs, R)
    ez = n * np.outer(Zc, R)
    bt = n * np.outer(G, dR)
    w = -n * np.outer(Zs, dR)
    return psi, ez, bt, w
