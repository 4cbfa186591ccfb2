"""Pins of the oracle gradient (central finite differences of the FP64
oracle's objective: witness mean gamma gain after one plasma response and 20
beam steps in its frozen fields) against what linear theory and the
structure of the objective fix.

In the linear regime the wake is proportional to the drive density and the
drive's wake at the witness depends on the separation only through the
witness position; with the frozen-field push the gain is minus the time
integral of E_z at the witness particles.  So
  dG/dn_d = -N_t dt <E_z^drive(r_b, xi_b)> / n_d,
  dG/dsep = -N_t dt <d_xi E_z^drive(r_b, xi_b)>,
with E_z^drive = n_d R(r) Zc(xi) from the closed form (Eqs. (1)-(7)
linearized, evaluated by quadrature independently of the oracle)."""
import numpy as np
import pytest

from paper_1411_3246_amd import inputs

from .linear_theory import longitudinal, radial_profile


def _weak(n_d=0.05, u_th=0.0, **kw):
    base = dict(n_r=128, n_xi=1024, ppc=4, u_th=u_th, n_beam=20000, n_steps=20, n_d=n_d,
                prec="fp64", name="weak-two-bunch")
    base.update(kw)
    return inputs.facet_two_bunch(**base)


def _witness_closed_form(p, O):
    """<E_z^drive> and <d_xi E_z^drive> over the witness macroparticles at
    their initial positions, from the closed form."""
    b = O.load_beam(p, inputs.beam_draws(p))
    wit = b["tag"] == 1
    r = np.hypot(b["x"][wit], b["y"][wit])
    xi = b["xi"][wit]
    d = p.bunches[0]
    rg = np.linspace(0.0, r.max() * 1.01 + 1e-9, 64)
    Rg, _ = radial_profile(rg, p.sigma_r, p.r_max)
    R = np.interp(r, rg, Rg)
    xs = np.linspace(xi.min() - 1e-6, xi.max() + 1e-6, 400)
    G, Zs, Zc = longitudinal(xs, d.xi_c, d.sigma_z, p.xi_min)
    zc = np.interp(xi, xs, Zc)
    dzc = np.interp(xi, xs, G - Zs)          # d/dxi Zc = G - Zs
    return d.n_peak * np.mean(R * zc), d.n_peak * np.mean(R * dzc)


def test_fd_gradient_is_converged(oracle_lib):
    """The central differences at h and h/2 agree (truncation well below the
    1e-4 gradient tolerance) for the components that do not move particles
    across grid nodes at first order."""
    O = oracle_lib
    p = _weak(u_th=0.005, n_r=32, n_xi=256, n_beam=2000)
    g, err = O.fd_gradient(p, which=(0, 2, 3))
    for i in (0, 2, 3):
        assert err[i] <= 1e-4 * abs(g[i]), (inputs.THETA_NAMES[i], g[i], err[i])


def test_drive_density_gradient_matches_linear_theory(oracle_lib):
    """Witness half a plasma period behind the drive (E_z extremum)."""
    O = oracle_lib
    p = _weak(sep=np.pi)
    g, _ = O.fd_gradient(p, which=(0,))
    ez, _ = _witness_closed_form(p, O)
    expect = -p.n_steps * p.dt * ez / p.bunches[0].n_peak
    assert g[0] == pytest.approx(expect, rel=2e-2)


def test_separation_gradient_matches_linear_theory(oracle_lib):
    """Witness at the zero crossing of the drive's E_z (largest slope)."""
    O = oracle_lib
    p = _weak(sep=1.5 * np.pi)
    g, _ = O.fd_gradient(p, which=(3,))
    _, dez = _witness_closed_form(p, O)
    expect = -p.n_steps * p.dt * dez
    assert g[3] == pytest.approx(expect, rel=5e-2)


def test_gain_is_linear_in_drive_density(oracle_lib):
    """(G(n_d) - G(0)) / n_d -> dG/dn_d with an error proportional to n_d."""
    O = oracle_lib
    dev = []
    for n_d in (0.1, 0.02):
        p = _weak(n_d=n_d, n_r=32, n_xi=256, n_beam=2000)
        g, _ = O.fd_gradient(p, which=(0,))
        th = inputs.theta_of(p)
        th0 = th.copy()
        th0[0] = 0.0
        secant = (O.objective(p) - O.objective(inputs.with_theta(p, th0))) / n_d
        dev.append(abs(secant - g[0]) / abs(g[0]))
    assert dev[1] < dev[0] / 3.0, dev
    assert dev[1] < 2e-2, dev
