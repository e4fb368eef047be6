"""CPU tests of the tuning cache file format (no device work)."""
import json

import pytest


@pytest.fixture(scope="module")
def A():
    import paper_2005_06191_amd as A
    A.binding.lib()
    return A


def test_cache_roundtrip(A, tmp_path):
    A.tune_clear()
    src = tmp_path / "in.json"
    src.write_text(json.dumps({
        "solve:k1:n3:f32:otf:L5,5,2,:nu5:nx19:s2": {"chunk": 1, "blocks_per_cu": 0, "xcd_order": 1,
                                                     "variant": 2, "ms": 5.5},
        "batch:f32:fam18,19,:n6:rows30:W14:T32": {"chunk": 4, "blocks_per_cu": 2, "xcd_order": 0,
                                                 "variant": 0, "ms": 12.25}}, indent=1))
    # the loader reads the spacing the writer produces
    txt = "{\n" + ",\n".join(
        f'  "{k}": {{"chunk": {v["chunk"]}, "blocks_per_cu": {v["blocks_per_cu"]}, '
        f'"xcd_order": {v["xcd_order"]}, "variant": {v["variant"]}, "ms": {v["ms"]:.6f}}}'
        for k, v in json.loads(src.read_text()).items()) + "\n}\n"
    src.write_text(txt)
    A.tune_load(str(src))
    assert A.tune_entries() == 2
    out = tmp_path / "out.json"
    A.tune_save(str(out))
    d = json.loads(out.read_text())
    assert d["batch:f32:fam18,19,:n6:rows30:W14:T32"]["chunk"] == 4
    assert d["solve:k1:n3:f32:otf:L5,5,2,:nu5:nx19:s2"]["variant"] == 2
    A.tune_clear()
    assert A.tune_entries() == 0


def test_cache_rejects_bad_entries(A, tmp_path):
    bad = tmp_path / "bad.json"
    bad.write_text('{\n  "k": {"chunk": 0, "blocks_per_cu": 0, "xcd_order": 1, "variant": 1, "ms": 1.0}\n}\n')
    with pytest.raises(A.AmyError):
        A.tune_load(str(bad))
    with pytest.raises(A.AmyError):
        A.tune_load(str(tmp_path / "missing.json"))


def test_batch_query_on_cpu(A):
    import workloads as W
    ps = W.batch_systems()
    assert A.batch_query(ps) > 0
    with pytest.raises(A.AmyError):
        A.batch_query([ps[0].with_(mode="stored")])
