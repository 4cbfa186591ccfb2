"""The autotuner's cache (host logic only): the classes a tuned choice is
kept for, the batch key of the scan and the JSON round trip."""
import json

from paper_1411_3246_amd import autotune, inputs


def test_class_key_separates_grid_ppc_precision_geometry_temperature():
    p = inputs.facet_two_bunch(n_r=256, n_xi=100, ppc=8, u_th=0.02, n_beam=0, prec="mixed")
    keys = {autotune.class_key(q) for q in (
        p, p.replace(n_r=512), p.replace(ppc=16), p.replace(prec="fp64"),
        p.replace(geom="slab"), p.replace(u_th=0.0))}
    assert len(keys) == 6
    # the window length and the drive do not change the class
    assert autotune.class_key(p.replace(n_xi=4000, xi_max=p.xi_min + 4000 * p.dxi)) == autotune.class_key(p)
    assert autotune.class_key(p.replace(n_beam=1000)) == autotune.class_key(p)


def test_scan_key_is_the_multiset_of_instances():
    probs = inputs.scan_instances(16, prec="mixed")
    k = autotune.scan_key(probs)
    assert autotune.scan_key(list(reversed(probs))) == k
    assert autotune.scan_key(probs[:-1]) != k
    assert autotune.scan_key([q.replace(prec="fp64") for q in probs]) != k


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = autotune.TuneCache(path)
    assert c.get("a") is None
    p = inputs.facet_two_bunch(n_r=128, n_xi=50, ppc=4, n_beam=0, prec="fp64")
    assert autotune.cached_response(p, c) is None
    c.put(autotune.class_key(p), {"threads": 512, "group": 4, "table": []})
    c2 = autotune.TuneCache(path)
    assert autotune.cached_response(p, c2) == (512, 4)
    assert autotune.cached_response(p.replace(ppc=8), c2) is None
    with open(path) as f:
        assert json.load(f)[autotune.class_key(p)]["group"] == 4


def test_unreadable_cache_starts_empty(tmp_path):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert autotune.TuneCache(str(path)).entries == {}
