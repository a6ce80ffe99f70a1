"""The reduction entry point that allocates nothing, against the one that
does: two calls in a row through the C-ABI (the second with fewer traces),
each equal bit for bit to fp_frame_potential on the same traces."""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fp():
    import paper_2205_09900_amd as m
    assert torch.cuda.is_available()
    return m


def test_noalloc_reduction_matches_allocating_one(fp):
    for n, kmax, seed in [(300001, 8, 11), (1000, 3, 12), (7, 2, 13)]:
        z = synth.heavy_tailed_traces(seed, n, scale=3.0)
        d = torch.from_numpy(np.stack([z.real, z.imag], 1).reshape(-1)).cuda()
        f0, se0 = fp.fp_frame_potential(d, n, kmax)
        f1, se1 = fp.fp_frame_potential_noalloc(d, n, kmax)
        assert f1 == f0 and se1 == se0, (n, f0, f1)


def test_noalloc_reduction_flags_nonfinite(fp):
    d = torch.zeros(40, dtype=torch.float64, device="cuda")
    d[5] = float("inf")
    with pytest.raises(fp.FPError) as e:
        fp.fp_frame_potential_noalloc(d, 20, 2)
    assert e.value.code == fp.FP_ENUMERIC
    d[5] = 1.0  # the next call on the same scratch is clean again
    f, _ = fp.fp_frame_potential_noalloc(d, 20, 1)
    assert f[0] == 1.0 / 20
