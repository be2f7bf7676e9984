"""Autotuner bookkeeping on the CPU: size buckets and the JSON cache."""
from types import SimpleNamespace

from paper_2108_12742_amd import tune as T


def _p(eq, nx, ny=1, order=5):
    return SimpleNamespace(equation=eq, nx=nx, ny=ny, order=order)


def test_bucket_key_groups_by_equation_order_and_size():
    a = T.bucket_key([_p(2, 2048, 2048)])
    b = T.bucket_key([_p(2, 2000, 2100)])
    c = T.bucket_key([_p(2, 2048, 2048, order=7)])
    d = T.bucket_key([_p(1, 4096)] * 512)
    assert a == b and a != c and d.startswith("eq1-o5-") and "-m9-b" in d
    # the key names the library build, so a rebuilt library is tuned afresh
    assert a.endswith("-b" + T.build_id())


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("ENOAO_TUNE_CACHE", str(tmp_path / "sub" / "tune.json"))
    assert T.load_cache() == {}
    T.store("k1", {"workgroups_per_cu": 2, "y_strip_columns": 4, "ms_per_step": {"2/4": 1.0}})
    T.store("k2", {"workgroups_per_cu": 0, "y_strip_columns": 8, "ms_per_step": {}})
    c = T.load_cache()
    assert c["k1"]["y_strip_columns"] == 4 and c["k2"]["workgroups_per_cu"] == 0
