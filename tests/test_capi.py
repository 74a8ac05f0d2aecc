"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/hb.h declares, and its pure-host entry points work."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hb_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1803_01291_amd import hb
    return hb.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header():
    from paper_1803_01291_amd import hb
    assert sorted(hb.exported_names()) == declared_functions()


def test_footprint_is_host_only(lib):
    from paper_1803_01291_amd import hb
    c = hb.make_config((256, 256, 256), (-16,) * 3, (16,) * 3, 2.0, 1.0, 0.005)
    fp = hb.hb_footprint(c)
    # whole-step scheme: the paired state (phi, psi) at two parities, 16 B per cell
    assert 2 * 256 ** 3 * 16 < fp < 2 * 280 ** 3 * 16
    c32 = hb.make_config((256, 256, 256), (-16,) * 3, (16,) * 3, 2.0, 1.0, 0.005, precision=hb.HB_F32C)
    # FP32c: (phi hi, psi hi, phi lo, psi lo) at two parities, 16 B per cell
    assert 2 * 256 ** 3 * 16 < hb.hb_footprint(c32) < 2 * 280 ** 3 * 16
    # the stage-pair and per-stage schemes keep 7 separate fields (G1..G3 too);
    # their rows round to 16 instead of 8 cells, hence the band
    for flags in (hb.HB_PAIRWISE, hb.HB_STAGEWISE):
        cp = hb.make_config((256, 256, 256), (-16,) * 3, (16,) * 3, 2.0, 1.0, 0.005, flags=flags)
        fields = hb.hb_footprint(cp) / (fp / 4)
        assert 6.9 < fields < 7.3
    bad = hb.make_config((0, 4, 4), (-1,) * 3, (1,) * 3, 1.0, 1.0, 0.01)
    assert hb.hb_footprint(bad) == 0


def test_plane_size_limit_is_rejected(lib):
    """The whole-step kernel addresses a plane with 32-bit byte offsets: an x-y
    plane of 2 GiB or more (16-byte cells, FP64 and FP32c) is rejected before
    anything is allocated (footprint 0, message)."""
    from paper_1803_01291_amd import hb
    for prec in (hb.HB_F64, hb.HB_F32C):
        ok = hb.make_config((11500, 11500, 1), (-1,) * 3, (1,) * 3, 1.0, 1.0, 1e-9,
                            flags=hb.HB_ALLOW_UNSTABLE, precision=prec)
        assert hb.hb_footprint(ok) > 0      # 11504 x 11504 x 16 B = 1.97 GiB per plane
    big = hb.make_config((11600, 11600, 1), (-1,) * 3, (1,) * 3, 1.0, 1.0, 1e-9,
                         flags=hb.HB_ALLOW_UNSTABLE)
    assert hb.hb_footprint(big) == 0        # 11608 x 11604 x 16 B = 2.007 GiB per plane
    assert "2 GiB" in hb.hb_last_error()


def test_batch_with_mixed_schemes_is_rejected(lib):
    """A batch shares its launches, so every solve must select the same scheme;
    the check runs before anything touches the device."""
    from paper_1803_01291_amd import hb
    a = hb.make_config((16, 16, 16), (-1,) * 3, (1,) * 3, 1.0, 1.0, 0.01)
    b = hb.make_config((16, 16, 16), (-1,) * 3, (1,) * 3, 1.0, 1.0, 0.01, flags=hb.HB_PAIRWISE)
    with pytest.raises(hb.HBError) as e:
        hb.hb_batch_create([a, b])
    assert e.value.code == hb.HB_E_ARG and "scheme" in str(e.value)


def test_pool_slot_count_is_bounded(lib):
    """A slot table sized by the caller is bounded (HB_E_ARG before anything is
    allocated or touches the device)."""
    from paper_1803_01291_amd import hb
    for slots in (0, (1 << 20) + 1):
        with pytest.raises(hb.HBError) as e:
            hb.hb_pool_create(1 << 30, slots)
        assert e.value.code == hb.HB_E_ARG


def test_binding_rejects_wrong_array_sizes(lib):
    """The C ABI takes no array sizes; the binding checks them against the grid
    before any call that would read or write the caller's memory."""
    from paper_1803_01291_amd import hb
    import numpy as np
    hb._GRIDS[("s", 12345)] = 4 * 5 * 6   # a grid the binding knows (no device call follows)
    try:
        with pytest.raises(ValueError, match="120"):
            hb.hb_set_initial(12345, np.zeros(119))
        with pytest.raises(ValueError, match="120"):
            hb.hb_read(12345, np.zeros(120), np.zeros(121))
        with pytest.raises(ValueError, match="share"):
            hb.hb_read(12345, np.zeros(120), np.zeros(120, np.float32))
    finally:
        del hb._GRIDS[("s", 12345)]
    with pytest.raises(ValueError, match="unknown"):
        hb.hb_set_initial(99999, np.zeros(8))
    cfg = hb.make_radial_config(100, 1e-3, 1.0, 1.0, 1e-5, 1)
    with pytest.raises(ValueError, match="nodes"):
        hb.hb_radial_solve([cfg, cfg], np.zeros(150), np.zeros(200))


def test_allocator_hook_arguments(lib):
    """hb_set_allocator takes both functions or neither (host-only check)."""
    import ctypes
    from paper_1803_01291_amd import hb
    cb = hb.HB_ALLOC_FN(lambda ctx, n, s: None)
    assert lib.hb_set_allocator(ctypes.cast(cb, ctypes.c_void_p), None, None) == hb.HB_E_ARG
    assert "both" in hb.hb_last_error()
    assert lib.hb_set_allocator(None, None, None) == hb.HB_OK
    with pytest.raises(ValueError):
        hb.hb_set_allocator(lambda n, s: 0, None)


def test_periodic_flag_needs_the_whole_step_scheme(lib):
    """HB_BC_PERIODIC is validated on the host: the whole-step scheme accepts
    it, the stage-pair and per-stage schemes do not (footprint 0 = invalid)."""
    from paper_1803_01291_amd import hb
    base = dict(n=(32, 16, 8), lo=(0.0,) * 3, hi=(8.0, 4.0, 2.0), mu2=2.0, lam=1.0, dt=0.01)
    assert hb.hb_footprint(hb.make_config(**base, flags=hb.HB_BC_PERIODIC)) > 0
    for f in (hb.HB_PAIRWISE, hb.HB_STAGEWISE):
        assert hb.hb_footprint(hb.make_config(**base, flags=hb.HB_BC_PERIODIC | f)) == 0
