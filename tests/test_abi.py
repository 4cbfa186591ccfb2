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
