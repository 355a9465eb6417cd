"""The benchmark's host-side plumbing: tile-shape keys and the lookup of a
committed counter record, which is refused when it was taken on other
kernel sources (the benchmark then reports traffic as unmeasured)."""
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
_spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
B = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(B)


def test_shape_key_names_shape_and_grid():
    t = {"tile_rows": 128, "lanes_per_row": 2, "cols_per_lane": 2, "loads_in_flight": 4,
         "waves_per_simd": 0, "workgroups": 1280}
    assert B.shape_key(4, t) == "4,128,1,2,4,0@1280"
    t2 = dict(t, lanes_per_row=4)       # two lane groups per row at V = 2, S = 4
    assert B.shape_key(4, t2) == "4,128,2,2,4,0@1280"


def test_traffic_lookup_refuses_other_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles", "spmm_diffusion3d_128_traffic.json")))
    key = next(iter(rec["per_shape"]))
    current = rec["kernel_hash"] == B.source_hash(B.SPMM_SOURCES)
    got = B.traffic_from_profiles("spmm_diffusion3d_128_traffic.json", key)
    assert got == (rec["per_shape"][key]["bytes_per_launch"] if current else None)
    assert B.traffic_from_profiles("spmm_diffusion3d_128_traffic.json", "no such shape") is None
    # the same lookup against another source set (a changed kernel) gives nothing
    assert B.traffic_from_profiles("spmm_diffusion3d_128_traffic.json", key,
                                   ("k_dense.hip",)) is None
    assert B.traffic_from_profiles("missing.json", key) is None


def test_traffic_lookup_by_kernel_name_on_any_grid():
    # the dense records are looked up by kernel name: the one entry of that
    # kernel, whatever grid it ran on
    rec = json.load(open(os.path.join(ROOT, "profiles", "dense_8192_traffic.json")))
    current = rec["kernel_hash"] == B.source_hash(B.DENSE_SOURCES)
    for key, ent in rec["per_shape"].items():
        name = key.split("@")[0]
        got = B.traffic_from_profiles("dense_8192_traffic.json", name, B.DENSE_SOURCES,
                                      any_grid=True)
        assert got == (ent["bytes_per_launch"] if current else None)
    assert B.traffic_from_profiles("dense_8192_traffic.json", "k_dense_f64<3>", B.DENSE_SOURCES,
                                   any_grid=True) is None
    # a name is not a key: without any_grid it matches nothing
    assert B.traffic_from_profiles("dense_8192_traffic.json", "k_dense_f64<1>",
                                   B.DENSE_SOURCES) is None
