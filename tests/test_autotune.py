"""Autotuner host logic: shape-class keys and the JSON cache."""
from paper_1006_2183_amd import autotune as AT


def test_autotune_shape_key_and_cache(tmp_path):
    info = {"flops": 3000, "max_vec_flops": 70, "n_out_vec": 100}
    k1 = AT.shape_key("plus_times_f64", "csr", "numeric", [info])
    k2 = AT.shape_key("plus_times_f64", "csr", "numeric", [dict(info, flops=3500)])
    k3 = AT.shape_key("plus_times_f64", "csr", "numeric", [dict(info, flops=5000)])
    assert k1 == k2 != k3
    c = AT.TuneCache(str(tmp_path / "t.json"))
    c.put(k1, {"tuning": {"lds_bytes": 65536}, "ms": 1.0, "default_ms": 2.0, "tried": 3})
    assert AT.TuneCache(str(tmp_path / "t.json")).get(k1)["tuning"] == {"lds_bytes": 65536}
