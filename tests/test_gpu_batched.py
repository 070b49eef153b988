"""GPU tests of the batched step (upsample_batch_*): per scene, bit-identical
to upsample_step on a handle with the same parameters -- through the HIP
graph (replayed several times, with eager work between replays) and eagerly --
plus rigid scenes, empty scenes, graph re-capture for new buffers, the
batched HR reorder against the per-scene one, and a sampled check of one
scene against the oracle."""
import numpy as np
import pytest

from workloads import configs
from workloads.generators import build_scene

from gpu_util import compare_step, dev, host, log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_01629_amd.batch import Batch
    from paper_2308_01629_amd.upsampler import Upsampler
    return Batch, Upsampler


def _scenes():
    sc = configs.batched(n_scenes=7, seed=11, hr_range=(3000, 60000))
    log("batched scenes: " + ", ".join(f"{s.name}:{s.n_lr}/{s.n_hr}" for s in sc))
    return sc


def _hr_state(scenes, seed):
    rng = np.random.default_rng(seed)
    return [s.hr_x0 for s in scenes], [rng.normal(0, 0.5, s.hr_x0.shape).astype(np.float32) for s in scenes]


@pytest.mark.parametrize("eager", [False, True])
def test_batched_equals_plain_bitexact(mods, eager):
    Batch, Upsampler = mods
    scenes = _scenes()
    b = Batch.from_scenes(scenes, eager=eager)
    plain = [Upsampler.from_scene(s) for s in scenes]
    hx0, hv0 = _hr_state(scenes, 1)
    # per-scene plain state and the packed batch state (stepped in place)
    px = [dev(a, torch) for a in hx0]
    pv = [dev(a, torch) for a in hv0]
    bx, bv = dev(b.pack_hr(hx0), torch), dev(b.pack_hr(hv0), torch)
    lx = torch.empty((3, b.total_lr), device="cuda")
    lv = torch.empty_like(lx)
    for t in range(1, 4):
        frames = [s.lr_frame(t) for s in scenes]
        lx.copy_(dev(b.pack_lr([f[0] for f in frames]), torch))
        lv.copy_(dev(b.pack_lr([f[1] for f in frames]), torch))
        b.step(lx, lv, bx, bv, out_x=bx, out_v=bv)
        # eager single-scene work between graph replays
        for s, up in enumerate(plain):
            X, V = dev(frames[s][0], torch), dev(frames[s][1], torch)
            px[s], pv[s] = up.step(X, V, None, px[s], pv[s])
        torch.cuda.synchronize()
        for s, (gx, gv) in enumerate(zip(b.split_hr(bx), b.split_hr(bv))):
            assert torch.equal(gx, px[s]) and torch.equal(gv, pv[s]), (t, s, scenes[s].name)
    info = b.info()
    log(f"batched eager={eager}: {info}")
    assert info["graphs_captured"] == (0 if eager else 1)
    assert info["tiles"] == sum((s.n_hr + 255) // 256 for s in scenes)


def test_batched_rigid_and_walls(mods):
    Batch, Upsampler = mods
    scenes = [build_scene("heap", 1500, 30001, seed=[21, 3], rigid_floor=True),
              build_scene("drain", 900, 20000, seed=[21, 4], rigid_floor=True),
              build_scene("column", 700, 9000, seed=[21, 5])]
    b = Batch.from_scenes(scenes)
    hx0, hv0 = _hr_state(scenes, 2)
    frames = [s.lr_frame(1) for s in scenes]
    rig = [s.lr_rigid if s.lr_rigid is not None else np.zeros(s.n_lr, np.uint8) for s in scenes]
    lrig = dev(np.concatenate(rig).astype(np.uint8), torch)
    ox, ov = b.step(dev(b.pack_lr([f[0] for f in frames]), torch), dev(b.pack_lr([f[1] for f in frames]), torch),
                    dev(b.pack_hr(hx0), torch), dev(b.pack_hr(hv0), torch), lr_rigid=lrig)
    for s, sc in enumerate(scenes):
        up = Upsampler.from_scene(sc)
        x1, v1 = up.step(dev(frames[s][0], torch), dev(frames[s][1], torch), dev(rig[s], torch),
                         dev(hx0[s], torch), dev(hv0[s], torch))
        torch.cuda.synchronize()
        assert torch.equal(b.split_hr(ox)[s], x1) and torch.equal(b.split_hr(ov)[s], v1), sc.name
    # one scene against the oracle on a sample
    s = 0
    idx = np.sort(np.random.default_rng(3).choice(scenes[s].n_hr, 4096, replace=False))
    r = compare_step(host(b.split_hr(ox)[s]), host(b.split_hr(ov)[s]), frames[s][0], frames[s][1], rig[s],
                     hx0[s], hv0[s], scenes[s].params(), scenes[s].box_length, idx=idx)
    log(f"batched rigid scene vs oracle: {r}")


def test_batched_empty_scenes_and_recapture(mods):
    Batch, Upsampler = mods
    base = configs.plain()
    kw = dict(r_lr=base.r_lr, r_hr=base.r_hr, dt=base.dt, g=tuple(base.g), domain_lo=tuple(base.domain_lo),
              domain_hi=tuple(base.domain_hi), walls=base.walls, c1=base.c1, c2=base.c2)
    n_lr = [base.n_lr, 0, base.n_lr, 37]
    n_hr = [base.n_hr, 5000, 0, 257]
    b = Batch([kw] * 4, n_lr, n_hr)
    rng = np.random.default_rng(5)
    X, V = base.lr_frame(1)
    lr_x = [X, np.zeros((3, 0), np.float32), X, X[:, :37]]
    lr_v = [V, np.zeros((3, 0), np.float32), V, V[:, :37]]
    hx0 = [base.hr_x0, rng.uniform(0.2, 0.8, (3, 5000)).astype(np.float32), np.zeros((3, 0), np.float32),
           base.hr_x0[:, :257]]
    hv0 = [rng.normal(0, 0.5, a.shape).astype(np.float32) for a in hx0]
    lx, lv = dev(b.pack_lr(lr_x), torch), dev(b.pack_lr(lr_v), torch)
    hx, hv = dev(b.pack_hr(hx0), torch), dev(b.pack_hr(hv0), torch)
    outs = [(torch.empty_like(hx), torch.empty_like(hv)) for _ in range(3)]
    res = []
    for k in range(6):   # three output buffer sets, each used twice: three captures
        ox, ov = outs[k % 3]
        b.step(lx, lv, hx, hv, out_x=ox, out_v=ov)
        res.append((ox.clone(), ov.clone()))
    torch.cuda.synchronize()
    assert b.info()["graphs_captured"] == 3
    for r in res[1:]:
        assert torch.equal(r[0], res[0][0]) and torch.equal(r[1], res[0][1])
    for s in (0, 1, 3):
        up = Upsampler(max_lr=max(n_lr[s], 1), max_hr=n_hr[s], **kw)
        x1, v1 = up.step(dev(lr_x[s], torch), dev(lr_v[s], torch), None, dev(hx0[s], torch), dev(hv0[s], torch))
        torch.cuda.synchronize()
        assert torch.equal(b.split_hr(res[0][0])[s], x1) and torch.equal(b.split_hr(res[0][1])[s], v1), s
    # no LR particles: free fall, v' = v + dt g, x' = x + dt v'
    v_ff = hv0[1] + np.float32(base.dt) * np.asarray(base.g, np.float32)[:, None]
    np.testing.assert_allclose(host(b.split_hr(res[0][1])[1]), v_ff, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("layout", ["in_order", "reversed"])
def test_batched_reorder_equals_plain_reorder(mods, layout):
    """upsample_batch_sort_hr sorts each scene's columns by the key
    upsample_sort_hr uses for that scene alone (scenes in column order: one
    counting sort over all scenes; reversed: one sort per scene).  The
    sequence of keys is the same and the permutation is one (particles of one
    fine cell may come in another order: the counting sort places them by
    arrival, a valid order of equal keys).  With the batch's permutation applied to the per-scene state,
    the batched steps that follow stay bit-identical to the per-scene steps."""
    from oracle import upsample_oracle as O
    from gpu_util import morton_sort_keys
    Batch, Upsampler = mods
    scenes = _scenes()
    offsets = None
    if layout == "reversed":   # scenes in reverse column order: the per-scene route
        offsets = np.concatenate([[0], np.cumsum([s.n_hr for s in scenes[::-1]])[:-1]])[::-1]
    b = Batch.from_scenes(scenes, hr_offsets=offsets)
    plain = [Upsampler.from_scene(s) for s in scenes]
    hx0, hv0 = _hr_state(scenes, 3)
    px = [dev(a, torch) for a in hx0]
    pv = [dev(a, torch) for a in hv0]
    bx, bv = dev(b.pack_hr(hx0), torch), dev(b.pack_hr(hv0), torch)
    lx = torch.empty((3, b.total_lr), device="cuda")
    lv = torch.empty_like(lx)
    for t in range(1, 7):
        frames = [s.lr_frame(t) for s in scenes]
        lx.copy_(dev(b.pack_lr([f[0] for f in frames]), torch))
        lv.copy_(dev(b.pack_lr([f[1] for f in frames]), torch))
        b.step(lx, lv, bx, bv, out_x=bx, out_v=bv)
        for s, up in enumerate(plain):
            px[s], pv[s] = up.step(dev(frames[s][0], torch), dev(frames[s][1], torch), None, px[s], pv[s])
        if t % 3 == 0:
            torch.cuda.synchronize()
            before = [host(x).copy() for x in px]
            perm = b.sort_hr(bx, bv)
            torch.cuda.synchronize()
            for s, (off, n) in enumerate(zip(b.hr_offsets, b.n_hr)):
                p = (perm[off:off + n] - off).long()
                assert torch.equal(torch.sort(p)[0], torch.arange(n, device="cuda")), (t, s, "not a permutation")
                # the single-scene reorder of the same columns: the same key sequence
                up = plain[s]
                cx, cv = px[s].clone(), pv[s].clone()
                q = up.sort_hr(cx, cv).long()
                spec = O.grid_spec(scenes[s].r_lr, scenes[s].domain_lo, scenes[s].domain_hi)
                tun = up.get_tuning()
                k_batch = morton_sort_keys(before[s][:, host(p)], spec, tun["sort_sub"], tun["sort_mode"])
                k_plain = morton_sort_keys(before[s][:, host(q)], spec, tun["sort_sub"], tun["sort_mode"])
                assert np.array_equal(k_batch, k_plain) and np.all(np.diff(k_batch) >= 0), (t, s, "keys")
                # follow the batch's order in the per-scene state
                px[s], pv[s] = px[s][:, p].contiguous(), pv[s][:, p].contiguous()
        torch.cuda.synchronize()
        for s, (gx, gv) in enumerate(zip(b.split_hr(bx), b.split_hr(bv))):
            assert torch.equal(gx, px[s]) and torch.equal(gv, pv[s]), (t, s, scenes[s].name)
    log(f"batched reorder ({layout}): {len(scenes)} scenes, two reorders: per-scene key order, steps bit-identical")
    b.close()
