"""Neighbour membership of the step kernel that upsample_advance and
upsample_run time, checked member by member against the oracle.

upsample_debug_step_members runs the same template instance as the timed
step (wave tiles, the box cull of the candidates, the weight form, the
matrix-core sums, the per-lane walk of spread-out waves) and exports, per HR
particle, the list entries meeting the exact float32 membership predicate.
Those ids must equal the oracle's neighbour set (brute-force-pinned KD-tree
route) bit for bit: a cull that dropped a member in the outer part of the
support, where its weight is too small for any float tolerance to notice,
fails here.  The entries that enter the sums (computed weight > 0) may differ
from the members only where the weight is below W_DISAGREE_MAX.  The debug
instance's stepped state must equal the timed kernel's bit for bit, so it is
the same arithmetic.
"""
import numpy as np
import pytest

from oracle import upsample_oracle as O
from workloads import configs
from workloads.generators import build_scene

from gpu_util import W_DISAGREE_MAX, dev, host, log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module")
def U():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_01629_amd.upsampler import Upsampler
    return Upsampler


def _sample(n, k, seed):
    if n <= k:
        return np.arange(n)
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False))


def _members_check(up, X, hx, hv, spec, n_sample, seed, label, rigid=None):
    """Timed kernel vs its debug instance (bit-identical state), then the
    exported members of a sample of particles vs the oracle's sets."""
    ox, ov = up.advance(hx, hv)
    # counts first, then the ids with room for the largest count
    _, _, count0, _, _, _ = up.debug_step_members(hx, hv, max_k=0)
    max_k = max(1, int(count0.max().item()))
    dx, dv, count, ids, count_w, wdis = up.debug_step_members(hx, hv, max_k=max_k)
    torch.cuda.synchronize()
    assert torch.equal(count, count0)
    assert torch.equal(ox, dx) and torch.equal(ov, dv), f"{label}: debug instance differs from the timed kernel"
    n = hx.shape[1]
    idx = _sample(n, n_sample, seed)
    ti = torch.from_numpy(idx).cuda()
    c = host(count[ti]).astype(np.int64)
    ids_s = host(ids[ti])
    hx_s = host(hx[:, ti])
    ip, jj = O.neighbours_kdtree(X, hx_s, spec.h, spec.h2_f)
    ref = np.diff(ip)
    miss = np.nonzero(c != ref)[0]
    assert miss.size == 0, (f"{label}: member count differs for {miss.size} of {idx.size} particles; first hr="
                            f"{idx[miss[0]]} gpu={c[miss[0]]} oracle={ref[miss[0]]}")
    for k in range(idx.size):
        got = np.sort(ids_s[k, :c[k]].astype(np.int64))
        np.testing.assert_array_equal(got, jj[ip[k]:ip[k + 1]], err_msg=f"{label}: hr {idx[k]}")
    # every lane: entries that enter the sums vs members
    cw = count_w.long()
    cm = count.long()
    differ = int((cw != cm).sum().item())
    wmax = float(wdis.max().item()) if n else 0.0
    assert wmax <= W_DISAGREE_MAX, f"{label}: an entry of weight {wmax:.3e} disagrees with membership"
    log(f"{label}: {idx.size} sampled member lists bit-exact (mean {ref.mean():.2f}, largest {max_k} members), "
        f"{differ} of {n} lanes with a weight/membership disagreement, largest such weight {wmax:.2e}")


CASES = [
    ("drain", 1, 0, None), ("drain", 1, 9, None), ("drain", 2, 9, None), ("drain", 4, 9, None),
    ("column", 1, 9, None), ("diff", 1, 9, None), ("drain_small", 1, 9, 0), ("drain_small", 1, 9, 16),
]


@pytest.mark.parametrize("name,groups,age,tile_max", CASES)
def test_timed_kernel_members_bitexact(U, name, groups, age, tile_max):
    """Full-size workloads (the drain at 1/16 for the per-lane walk of every
    wave, and at tile_max 16 for waves sent either way by their lanes'
    stencils): HR reordered as the timed run reorders, then ``age`` steps of
    upsample_run without a reorder (waves spread as particles drift), then the
    members of the next frame's step."""
    if name == "drain_small":
        sc = configs.drain(scale=1 / 16)
    else:
        sc = {"drain": configs.drain, "column": configs.column, "diff": configs.diff}[name]()
    log(f"members {name}: {sc.n_lr} LR, {sc.n_hr} HR, groups {groups}, {age} steps after a reorder, "
        f"tile_max {tile_max}")
    up = U.from_scene(sc)
    up.set_tuning(gather_groups=groups)
    spec = O.grid_spec(sc.r_lr, sc.domain_lo, sc.domain_hi)
    frames = [sc.lr_frame(t) for t in range(1, age + 2)]
    hx, hv = dev(sc.hr_x0, torch), dev(sc.hr_v0, torch)
    up.sort_hr(hx, hv, with_perm=False)
    if age:
        LX = dev(np.stack([f[0] for f in frames[:age]]), torch)
        LV = dev(np.stack([f[1] for f in frames[:age]]), torch)
        up.run(LX, LV, hx, hv, sort_every=0)
    if tile_max is not None:
        up.set_tuning(tile_max=tile_max)
    X, V = frames[age]
    up.build_grid(dev(X, torch), dev(V, torch))
    _members_check(up, X, hx, hv, spec, 4096, 100 + age, f"{name} G={groups} age={age}")
    up.close()


def test_timed_kernel_members_rigid_and_edges(U):
    """Rigid floor samples (the vector-form path with the rigid rule),
    particles outside the grid box and at the floor, a ragged count: every
    particle's members against the oracle."""
    sc = build_scene("heap", 3000, 40001, seed=[11, 1], rigid_floor=True)
    X, V = sc.lr_frame(2)
    rng = np.random.default_rng(3)
    hr_x = sc.hr_x0.copy()
    hr_x[:, :500] = rng.uniform(-0.3, 1.3, (3, 500)).astype(np.float32)
    hr_x[1, 500:1500] = (X[1, -1] + rng.uniform(-0.01, 0.03, 1000)).astype(np.float32)
    hr_v = rng.normal(0, 1.0, hr_x.shape).astype(np.float32)
    spec = O.grid_spec(sc.r_lr, sc.domain_lo, sc.domain_hi)
    for rigid in (True, False):
        up = U.from_scene(sc, max_lr=X.shape[1])
        hx, hv = dev(hr_x, torch), dev(hr_v, torch)
        up.sort_hr(hx, hv, with_perm=False)
        up.build_grid(dev(X, torch), dev(V, torch), dev(sc.lr_rigid, torch) if rigid else None)
        _members_check(up, X, hx, hv, spec, hr_x.shape[1], 1, f"heap rigid={rigid}")
        up.close()
