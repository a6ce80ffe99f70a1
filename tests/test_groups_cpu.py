"""Host-side checks of the uneven-batch and tuning entry points (no device)."""

import pytest


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    return m


def test_workspace_groups_sizes(fp):
    ens = [(2, 30, L) for L in range(1, 9)] + [(0, 20, 4), (1, 50, 100)]
    groups = [(i, fp.C64, 0, 1000) for i in range(len(ens))]
    nb = fp.fp_workspace_bytes_groups(ens, groups)
    assert nb >= fp.fp_workspace_bytes((1, 50, 100), 1000, fp.C64)
    # HEA and LDS-sized brickwork groups need only descriptors and task lists
    small = fp.fp_workspace_bytes_groups(ens[:9], groups[:9])
    assert small < 10 << 20


def test_groups_validation(fp):
    with pytest.raises(fp.FPError):
        fp.fp_workspace_bytes_groups([(2, 30, 3)], [(1, fp.C64, 0, 10)])       # bad ensemble index
    with pytest.raises(fp.FPError):
        fp.fp_workspace_bytes_groups([(2, 30, 3)], [(0, 7, 0, 10)])            # unknown precision
    with pytest.raises(fp.FPError):
        fp.fp_workspace_bytes_groups([(2, 30, 3)], [(0, fp.C64, -1, 10)])      # pair range
    with pytest.raises(fp.FPError):
        fp.fp_workspace_bytes_groups([(2, 30, 9)], [(0, fp.C64, 0, 10)])       # 16-bit HEA boundary


def test_autotune_table_round_trip(fp):
    fp.fp_autotune_load("# comment\ngfx950 2 30 6 1 small 20000000 0.125000\ngfx950 0 20 8 1 large 5000000 2.500000\n")
    text = fp.fp_autotune_table()
    assert "gfx950 2 30 6 1 small 20000000" in text and "gfx950 0 20 8 1 large 5000000" in text
    with pytest.raises(fp.FPError):
        fp.fp_autotune_load("gfx950 2 30 6 1 medium 2e7 0.1\n")
    with pytest.raises(fp.FPError):
        fp.fp_autotune_load("gfx950 2 30 6 1 small 0 0.1\n")
    with pytest.raises(fp.FPError):
        fp.fp_autotune_load("garbage line\n")


def test_autotune_rejects_what_it_cannot_tune(fp):
    import ctypes
    choice = ctypes.c_int(-1)
    for ens in [fp.Ensemble(1, 50, 100), fp.Ensemble(0, 20, 10)]:  # per-pair plans; a boundary beyond LDS
        rc = fp.lib.fp_autotune(ctypes.byref(ens), fp.C64, ctypes.c_void_p(256), 1 << 30, ctypes.byref(choice), None)
        assert rc == fp.FP_ENOTIMPL
    assert fp.fp_autotune_workspace_bytes((1, 50, 100), fp.C64) == 0
    assert fp.fp_autotune_workspace_bytes((2, 30, 4), fp.C64) > 0
