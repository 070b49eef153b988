"""GPU parity of the randomized volume sampling of initial states (Section 4,
the sampling paragraph; upsample_sample_volume) against
oracle/sampling_oracle.py: the samples, their order and their number are
bit-exact; no two samples overlap (brute force); edge cases."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import sampling_oracle as S
from workloads.generators import volume_candidates

from gpu_util import dev, host, log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sampler():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_01629_amd.upsampler import sample_volume
    return sample_volume


@pytest.mark.parametrize("geometry,n,r,top", [("heap", 200_000, 0.008, None), ("drain", 600_000, 0.0125, None),
                                              ("column", 300_000, 0.25 / 21.0 * 0.3, 0.4)])
def test_sampling_bitexact(sampler, geometry, n, r, top):
    cand, lo, hi = volume_candidates(geometry, n, [41, n], top=top)
    got = sampler(dev(cand, torch), r, lo, hi)
    torch.cuda.synchronize()
    ref, idx = S.sample_volume(cand, r, lo, hi)
    g = host(got)
    assert g.shape == ref.shape, (g.shape, ref.shape)
    np.testing.assert_array_equal(g, ref)
    assert not cKDTree(g.T.astype(np.float64)).query_pairs(2 * r * (1 - 1e-6))
    side, inv, lo32, dims = S.sampling_grid(r, lo, hi)
    log(f"sampling {geometry}: {n} candidates, r {r:.5f}, {np.prod(dims)} cells -> {g.shape[1]} samples, bit-exact")


def test_sampling_edges(sampler):
    from paper_2308_01629_amd import UpsampleError
    lo, hi, r = (0.0, 0.0, 0.0), (0.2, 0.2, 0.2), 0.01
    empty = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    assert sampler(empty, r, lo, hi).shape == (3, 0)
    one_cell = dev(np.array([[0.001, 0.002, 0.0015], [0.001, 0.0011, 0.002], [0.002, 0.001, 0.001]], np.float32),
                   torch)
    out = host(sampler(one_cell, r, lo, hi))
    np.testing.assert_array_equal(out, host(one_cell)[:, :1])
    cand, _, _ = volume_candidates("plain", 50_000, 3)
    cand = np.ascontiguousarray(np.clip(cand, 0.0, 0.2), dtype=np.float32)
    full = host(sampler(dev(cand, torch), r, lo, hi))
    with pytest.raises(UpsampleError, match="CAPACITY"):
        sampler(dev(cand, torch), r, lo, hi, max_out=full.shape[1] - 1)
    ref, _ = S.sample_volume(cand, r, lo, hi)
    np.testing.assert_array_equal(full, ref)
