"""CPU-side checks of the C ABI: the library loads, exports every entry point
declared in include/fpsz.h, and its host-only calls (no device work) behave
as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fpsz.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fpsz_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1805_07384_amd import fpsz
    if not os.path.exists(fpsz.LIB_PATH):
        from paper_1805_07384_amd import build
        build.build()
    return fpsz.load_library()


def test_every_declared_symbol_is_exported_and_bound(lib):
    from paper_1805_07384_amd import fpsz
    names = _declared()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(lib, nm), nm
        assert nm in fpsz.SIGNATURES, nm


def test_binding_refuses_missing_library(tmp_path):
    from paper_1805_07384_amd import fpsz
    saved = fpsz._lib
    fpsz._lib = None
    try:
        with pytest.raises(fpsz.FpszError):
            fpsz.load_library(str(tmp_path / "nope.so"))
    finally:
        fpsz._lib = saved


def test_eb_rel_matches_oracle(lib, orc):
    from paper_1805_07384_amd import fpsz
    for p in np.linspace(0, 160, 81):
        assert fpsz.eb_rel(p) == orc.eb_rel(p)  # same closed form, same libm
    out = ctypes.c_double()
    assert lib.fpsz_eb_rel(float("inf"), ctypes.byref(out)) == fpsz.E_INVALID_ARG


def test_sizes_and_invalid_shapes(lib):
    from paper_1805_07384_amd import fpsz
    import torch
    for shape in [(1,), (8193,), (3, 5), (1800, 3600), (17, 17, 33), (512, 512, 512)]:
        for dt in (torch.float32, torch.float64):
            w = fpsz.compress_workspace_bytes(shape, dt)
            n = int(np.prod(shape))
            assert w >= 2 * n and w % 256 == 0
            assert fpsz.decompress_workspace_bytes(shape, dt) % 256 == 0
            b = fpsz.compress_bound(shape, dt)
            assert b >= n * (20 if dt == torch.float32 else 28)
    for bad in [(), (0,), (2, 0), (1, 2, 3, 4), (1 << 31,), (1 << 16, 1 << 15)]:
        with pytest.raises(fpsz.FpszError) as e:
            fpsz.compress_workspace_bytes(bad, torch.float32)
        assert e.value.status == fpsz.E_INVALID_ARG


def test_header_parser_on_oracle_blob(lib, orc):
    from paper_1805_07384_amd import fpsz, synth
    x = synth.field_2d_grf(100, 70, seed=9)
    blob, t = orc.compress(x, 60.0, trace=True)
    h = fpsz.parse_header(blob)
    assert h.shape == (100, 70) and h.ndim == 2
    assert h.info["eb"] == t["eb"] and h.info["vr"] == t["vr"]
    assert h.info["blob_bytes"] == len(blob)
    assert h.info["n_patches"] == t["n_patches"]
    bad = bytearray(blob)
    bad[0] ^= 1
    with pytest.raises(fpsz.FpszError):
        fpsz.parse_header(bytes(bad))
