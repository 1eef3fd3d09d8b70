"""The batch autotuner's JSON cache (host logic, no GPU): keys depend on the
device, the library build and the multiset of field shapes only; the file
round-trips, keeps other entries, and unreadable or foreign files read as
empty."""
import json

from paper_1805_07384_amd import fpsz


def _descs(spec):
    arr = (fpsz.FieldDesc * len(spec))()
    for i, (dt, dims, dom, psnr) in enumerate(spec):
        arr[i].ndim = len(dims)
        arr[i].dtype = dt
        for k, v in enumerate(list(dims) + [1] * (3 - len(dims))):
            arr[i].dims[k] = v
        arr[i].domain = dom
        arr[i].target_psnr = psnr
    return arr


def test_key_is_order_and_target_independent():
    a = _descs([(0, (64, 64), 0, 80.0), (1, (20000,), 1, 40.0)])
    b = _descs([(1, (20000,), 1, 120.0), (0, (64, 64), 0, 60.0)])
    assert fpsz.autotune_key(a, "dev") == fpsz.autotune_key(b, "dev")
    assert fpsz.autotune_key(a, "dev") != fpsz.autotune_key(a, "other")
    c = _descs([(0, (64, 65), 0, 80.0), (1, (20000,), 1, 40.0)])
    assert fpsz.autotune_key(a, "dev") != fpsz.autotune_key(c, "dev")
    d = _descs([(0, (64, 64), 1, 80.0), (1, (20000,), 1, 40.0)])
    assert fpsz.autotune_key(a, "dev") != fpsz.autotune_key(d, "dev")


def test_cache_round_trip_and_bad_files(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert fpsz.load_autotune_cache(path) == {}
    fpsz.store_autotune_cache(path, "k1", [[64, 512, 1024, 32]], 1.5)
    fpsz.store_autotune_cache(path, "k2", [[16, 32, 64, 8], [128, 256, 256, 128]], 2.5)
    e = fpsz.load_autotune_cache(path)
    assert e["k1"]["shapes"] == [[64, 512, 1024, 32]] and e["k2"]["best_ms"] == 2.5
    fpsz.store_autotune_cache(path, "k1", [[32, 64, 64, 8]], 1.0)
    e = fpsz.load_autotune_cache(path)
    assert e["k1"]["shapes"] == [[32, 64, 64, 8]] and "k2" in e
    with open(path, "w") as fh:
        fh.write("{not json")
    assert fpsz.load_autotune_cache(path) == {}
    with open(path, "w") as fh:
        json.dump({"version": 2, "entries": {}}, fh)
    assert fpsz.load_autotune_cache(path) == {}
    with open(path, "w") as fh:
        json.dump({"version": 1, "entries": {"a": {"shapes": [[1, 2, 3]], "best_ms": 1.0},
                                             "b": {"shapes": [[1, 2, 3, 0]], "best_ms": 1.0},
                                             "c": {"shapes": [[1, 2, 3, 4]], "best_ms": 1.0}}}, fh)
    assert list(fpsz.load_autotune_cache(path)) == ["c"]
