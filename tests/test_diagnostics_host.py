"""Host checks of the trajectory post-processing on synthetic trajectories
whose axis crossings are known."""
import numpy as np

from paper_1411_3246_amd import diagnostics


def test_axis_crossings_of_synthetic_orbits():
    xi = np.linspace(0.0, 10.0, 2001)
    h = 0.02
    r0 = np.array([0.5, 0.8, 1.1, 1.5, 2.5, 0.3])
    cross_at = np.array([6.0, 6.1, 6.2, 6.3, 6.4, 0.0])
    tr = np.empty((xi.size, r0.size))
    for q in range(r0.size):
        r = np.full(xi.size, r0[q])
        if q < 4:
            # out to r0 + 1 after xi = 3, back through the axis at cross_at,
            # then out again to at most 0.5
            up = (xi >= 3.0) & (xi < 4.5)
            r[up] = r0[q] + (xi[up] - 3.0) / 1.5
            down = xi >= 4.5
            line = np.abs((r0[q] + 1.0) * (cross_at[q] - xi[down]) / (cross_at[q] - 4.5))
            r[down] = np.where(xi[down] < cross_at[q], line, np.minimum(line, 0.5))
        elif q == 4:
            r = r0[q] + np.where(xi > 3.0, 2.0, 0.0)       # loaded beyond r0 = 2: not counted
        tr[:, q] = r                                          # q = 5 never moves: not counted
    out = diagnostics.axis_crossings(tr, xi, h, xi_drive=2.5, thresholds=(2,))["below_2_cells"]
    assert out["electrons"] == 4
    # each first drop below 2 cells comes just before its crossing
    expect = cross_at[:4] - 2 * h * (cross_at[:4] - 4.5) / (r0[:4] + 1.0)
    assert abs(out["xi_mean"] - expect.mean()) < 2 * (xi[1] - xi[0])
    assert abs(out["xi_std"] - expect.std()) < 2 * (xi[1] - xi[0])
