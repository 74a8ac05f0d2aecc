"""The library's default tiling (host logic only: hb_default_tiling launches
nothing, and assumes the 256 CUs of the target part when no device is
visible).  Pins the region-shape rule and the z-march model on the grids
whose choices the design names: one round of 256 blocks of 32 x 16 tiles
with 128-plane marches on 256^3, 64 x 11 tiles with 256-plane marches on
512^3 (752 blocks, three rounds), 32 x 24 tiles on 384^3, and the
precision-dependent choice on the paper's 500^3 grid."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

LIB = os.path.join(ROOT, "paper_1803_01291_amd", "libhb.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhb.so not built")


@pytest.fixture(scope="module")
def hb():
    from paper_1803_01291_amd import hb as m
    m.load()
    return m


def tiling(hb, w, precision=0, flags=0):
    return hb.hb_default_tiling(hb.config_from_workload(w, precision, flags))


def test_benchmark_grid_one_round_of_32x16_tiles(hb):
    import synth_inputs as si
    w = si.config2()
    # 256 x 256 planes in 32 x 16 tiles: 8 x 16 = 128 columns, two 128-plane
    # z-chunks: 256 blocks, one per CU
    assert tiling(hb, w, 0) == (20, 128)
    assert tiling(hb, w, 1) == (20, 128)


@pytest.mark.parametrize("n,f64,f32c", [
    (512, (11, 256), (11, 256)),
    (384, (8, 96), (8, 96)),
    (500, (8, 167), (16, 250)),
    (160, (20, 32), (20, 32)),
    (128, (11, 13), (11, 13)),
])
def test_default_shapes(hb, n, f64, f32c):
    import synth_inputs as si
    w = si.config2(n=n)
    assert tiling(hb, w, 0) == f64
    assert tiling(hb, w, 1) == f32c


def test_slab_and_comparison_schemes(hb):
    import synth_inputs as si
    assert tiling(hb, si.slab_config()) == (11, 32)
    # the stage-pair and per-stage kernels: tiles of 64 columns x 16 rows,
    # 64-plane marches while one solve gives at least 256 tiles
    w = si.config2()
    assert tiling(hb, w, 0, hb.HB_PAIRWISE) == (16, 64)
    assert tiling(hb, w, 0, hb.HB_STAGEWISE) == (16, 64)


def test_invalid_config_is_rejected(hb):
    import synth_inputs as si
    cfg = hb.config_from_workload(si.config2(n=64))
    cfg.dt = 10.0
    with pytest.raises(hb.HBError) as e:
        hb.hb_default_tiling(cfg)
    assert e.value.code == hb.HB_E_CFL
    cfg = hb.config_from_workload(si.config2(n=64))
    cfg.n[0] = 0
    with pytest.raises(hb.HBError) as e:
        hb.hb_default_tiling(cfg)
    assert e.value.code == hb.HB_E_ARG
