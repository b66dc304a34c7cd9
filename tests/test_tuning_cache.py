"""Host logic of the autotune cache: keys follow what the tuning depends on, entries round-trip."""
import numpy as np

from paper_1504_00636_amd import tuning_cache as TC, vpm


def test_signature_and_key(tmp_path):
    off = np.concatenate([[0], np.cumsum([0, 1, 5, 600, 2000, 40000])])
    p = vpm.make_params(tol_x=0.1, tol_p=0.05, n_min_cell=2)
    sig = TC.population_signature(off, p)
    assert sig["n_cells"] == 6
    assert sum(sig["size_classes"]) == 6 and sig["size_classes"][0] == 1      # the empty cell
    k = TC.cache_key("gfx950", "7.0", vpm.VPM_F32, sig)
    assert k == TC.cache_key("gfx950", "7.0", vpm.VPM_F32, dict(sig))
    assert k != TC.cache_key("gfx942", "7.0", vpm.VPM_F32, sig)
    assert k != TC.cache_key("gfx950", "7.1", vpm.VPM_F32, sig)
    assert k != TC.cache_key("gfx950", "7.0", vpm.VPM_F64, sig)
    p2 = vpm.make_params(tol_x=0.1, tol_p=0.06, n_min_cell=2)
    assert k != TC.cache_key("gfx950", "7.0", vpm.VPM_F32, TC.population_signature(off, p2))


def test_store_lookup_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    assert TC.lookup(path, "k") is None
    t = vpm.make_tuning(ppl=8, bin_a_max=512, concurrent_bins=1)
    TC.store(path, "k", t, {"note": "test"})
    TC.store(path, "k2", vpm.make_tuning(), {})
    got = TC.lookup(path, "k")
    assert got.as_dict() == t.as_dict()
    assert TC.lookup(path, "k2").as_dict() == vpm.make_tuning().as_dict()
    open(path, "w").write("not json")
    assert TC.lookup(path, "k") is None
