"""Host-side checks of the C-ABI library (no GPU needed): the built library
loads, exports every function that include/wake.h declares, the binding
names the same set, and plan validation rejects bad problems before any
device work."""
import ctypes
import os
import re

import pytest

from paper_1411_3246_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wake.h")
LIB = os.path.join(ROOT, "paper_1411_3246_amd", "libwake.so")

DECL = re.compile(r"^(?:const char\s*\*|wk_status|size_t|int32_t|void)\s*\*?\s*(wk_\w+)\s*\(", re.M)


def declared():
    with open(HEADER) as f:
        return sorted(set(DECL.findall(f.read())))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libwake.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_api():
    names = declared()
    for must in ("wk_plan_create", "wk_init_plasma", "wk_init_beam", "wk_beam_current",
                 "wk_plasma_response", "wk_beam_push", "wk_batch_response", "wk_cycle",
                 "wk_mean_gain", "wk_ez_peak"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_1411_3246_amd import wake
    assert sorted(wake.EXPORTS) == declared()


def test_plan_validation_is_host_only():
    from paper_1411_3246_amd import wake
    good = wake.Plan(inputs.weak_single_bunch())
    assert good.sizes.n_plasma == 128 * 4 and good.sizes.n_nodes == 129
    for bad in (dict(n_r=1), dict(n_r=4096), dict(ppc=0), dict(n_xi=0), dict(r_max=-1.0),
                dict(u_th=0.01, ppc=3), dict(d_min=0.0), dict(xi_max=-1.0)):
        with pytest.raises(wake.WakeError):
            wake.Plan(inputs.weak_single_bunch(**bad))


def test_sizes_are_aligned_and_consistent():
    from paper_1411_3246_amd import wake
    p = inputs.blowout_response()
    s = wake.Plan(p).sizes
    assert s.n_plasma == p.n_plasma
    assert s.fields == 4 * p.n_xi * (p.n_r + 1) * 4          # float in mixed mode
    assert s.beam_current == p.n_xi * (p.n_r + 1) * 8
    for f in ("plasma_state", "plasma_const", "fields", "beam_current", "beam_state", "workspace"):
        assert getattr(s, f) % 256 == 0, f


def test_gradient_workspace_validation():
    """The gradient needs a two-bunch macroparticle beam; otherwise the size
    query returns 0 and says why.  FP64 and mixed plans are both accepted,
    the mixed one with two more plasma-sized double arrays."""
    import ctypes as C
    from paper_1411_3246_amd import wake
    L = wake.lib()
    good = wake.Plan(inputs.facet_two_bunch(n_r=32, n_xi=64, ppc=4, n_beam=1000, prec="fp64"))
    assert L.wk_gradient_workspace_size(good.handle, 20, 64) > 0
    mixed = wake.Plan(inputs.facet_two_bunch(n_r=32, n_xi=64, ppc=4, n_beam=1000, prec="mixed"))
    assert L.wk_gradient_workspace_size(mixed.handle, 20, 64) >= L.wk_gradient_workspace_size(good.handle, 20, 64)
    fixed = wake.Plan(inputs.facet_two_bunch(n_r=32, n_xi=64, ppc=4, n_beam=0, prec="fp64"))
    assert L.wk_gradient_workspace_size(fixed.handle, 20, 64) == 0
    assert b"two-bunch" in L.wk_last_error()
    assert L.wk_gradient_workspace_size(good.handle, 20, 0) == 0
    # larger checkpoint intervals need more segment scratch
    assert L.wk_gradient_workspace_size(good.handle, 20, 128) > L.wk_gradient_workspace_size(good.handle, 20, 8)


def test_batch_shape_validation():
    """Launch-shape arguments are checked before any device work."""
    import ctypes as C
    from paper_1411_3246_amd import wake
    L = wake.lib()
    plans = [wake.Plan(inputs.weak_single_bunch(n_r=16, n_xi=32))]
    h = (C.c_void_p * 1)(*[p.handle for p in plans])
    ws = L.wk_batch_workspace_size(1, h)
    fake = C.c_void_p(0x1000)
    assert L.wk_batch_response_shape(1, h, fake, fake, ws, 300, 0, None) == -1
    assert L.wk_batch_response_shape(1, h, fake, fake, ws, 256, 9, None) == -1
    assert L.wk_batch_response_shape(1, h, fake, fake, ws - 1 if ws > 0 else 0, 256, 1, None) != 0


def test_counter_read_rejects_null_pointers():
    """The read-back checks its pointers before touching the device."""
    import ctypes as C
    from paper_1411_3246_amd import wake
    L = wake.lib()
    buf = (C.c_uint64 * wake.NCOUNTERS)()
    assert L.wk_counters_read(None, C.addressof(buf), None) == -1
    assert L.wk_counters_read(C.c_void_p(0x1000), None, None) == -1


def test_large_grid_plans_are_accepted():
    """Up to 2048 radial cells: the plan workspace then carries the march's
    global node rows."""
    from paper_1411_3246_amd import wake
    small = wake.Plan(inputs.weak_single_bunch(n_r=512))
    big = wake.Plan(inputs.weak_single_bunch(n_r=2048))
    assert big.sizes.workspace >= small.sizes.workspace + 11 * 2050 * 8


def test_theta_roundtrip_and_table1_inputs():
    import numpy as np
    p = inputs.gradient_case()
    th = inputs.theta_of(p)
    q = inputs.with_theta(p, th * 1.1)
    assert np.allclose(inputs.theta_of(q), th * 1.1)
    assert q.bunches[1].n_peak == p.bunches[1].n_peak and q.bunches[1].sigma_z == p.bunches[1].sigma_z
    assert inputs.u_th_of(0.0) == 0.0
    assert abs(inputs.u_th_of(5.0) ** 2 * inputs.MC2_EV - 5.0) < 1e-9
    probs = inputs.te_scan_instances()
    keys = {(round(x.u_th, 12), x.n_xi) for x in probs}
    assert len(keys) == len(probs)                      # no duplicates
    b = inputs.facet_table1_beam(0.0)
    assert b.n_steps == 1203 and b.n_drive + (b.n_beam - b.n_drive) == b.n_beam
