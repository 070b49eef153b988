"""upsample_step_noalloc (no handle, no allocation: its LR-grid scratch is a
fixed device array inside the library) against upsample_step on a handle with
the default tuning, through the C ABI: bit-identical outputs on consecutive
calls, each later call smaller than the one before it (the array keeps the
last call's contents), at the array's maximum LR count, with rigid LR
particles, and the capacity errors."""
import numpy as np
import pytest

from workloads import configs
from workloads.generators import build_scene

from gpu_util import dev, log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_01629_amd import _lib, upsampler
    return upsampler, _lib


def _params(sc):
    return dict(r_lr=sc.r_lr, r_hr=sc.r_hr, dt=sc.dt, g=tuple(sc.g), domain_lo=tuple(sc.domain_lo),
                domain_hi=tuple(sc.domain_hi), walls=sc.walls, c1=sc.c1, c2=sc.c2)


def _pair(upsampler, sc, X, V, rigid, hx, hv):
    """(handle step, no-alloc step) outputs for the same inputs."""
    up = upsampler.Upsampler.from_scene(sc, max_lr=X.shape[1], max_hr=hx.shape[1])
    Xd, Vd = dev(X, torch), dev(V, torch)
    rd = None if rigid is None else dev(rigid, torch)
    hxd, hvd = dev(hx, torch), dev(hv, torch)
    a = up.step(Xd, Vd, rd, hxd, hvd)
    ox, ov = torch.full_like(hxd, float("nan")), torch.full_like(hvd, float("nan"))
    upsampler.step_noalloc(_params(sc), Xd, Vd, rd, hxd, hvd, ox, ov)
    torch.cuda.synchronize()
    up.close()
    return a, (ox, ov)


def test_noalloc_matches_step_on_consecutive_calls(mods):
    upsampler, _ = mods
    sc = configs.drain(scale=1 / 16)
    full = configs.drain()
    X, V = full.lr_frame(2)                       # 65,536 LR: the array's maximum
    assert X.shape[1] == 65536
    rng = np.random.default_rng(5)
    hv = rng.normal(0, 0.5, sc.hr_x0.shape).astype(np.float32)
    cases = [("max LR", X, V, sc.hr_x0, hv),
             ("smaller", X[:, :40001].copy(), V[:, :40001].copy(), sc.hr_x0[:, :70001].copy(), hv[:, :70001].copy()),
             ("smaller again", X[:, :777].copy(), V[:, :777].copy(), sc.hr_x0[:, :1025].copy(), hv[:, :1025].copy())]
    for name, Xc, Vc, hx, hvc in cases:
        (ax, av), (bx, bv) = _pair(upsampler, sc, Xc, Vc, None, hx, hvc)
        assert torch.equal(ax, bx) and torch.equal(av, bv), name
        log(f"no-alloc step, {name}: {Xc.shape[1]} LR, {hx.shape[1]} HR, bit-identical to upsample_step")


def test_noalloc_rigid_and_empty(mods):
    upsampler, _ = mods
    sc = build_scene("heap", 3000, 40001, seed=[11, 1], rigid_floor=True)
    X, V = sc.lr_frame(2)
    rng = np.random.default_rng(6)
    hv = rng.normal(0, 1.0, sc.hr_x0.shape).astype(np.float32)
    (ax, av), (bx, bv) = _pair(upsampler, sc, X, V, sc.lr_rigid, sc.hr_x0, hv)
    assert torch.equal(ax, bx) and torch.equal(av, bv)
    # then a smaller call without LR particles: free fall, as upsample_step
    e = np.zeros((3, 0), np.float32)
    (ax, av), (bx, bv) = _pair(upsampler, sc, e, e, None, sc.hr_x0[:, :999].copy(), hv[:, :999].copy())
    assert torch.equal(ax, bx) and torch.equal(av, bv)


def test_noalloc_capacity_errors(mods):
    upsampler, _lib = mods
    sc = configs.plain()
    X, V = sc.lr_frame(1)
    big = np.tile(X, (1, 33))[:, :_lib.NOALLOC_MAX_LR + 1].copy()
    hx = dev(sc.hr_x0[:, :64].copy(), torch)
    ox, ov = torch.empty_like(hx), torch.empty_like(hx)
    with pytest.raises(_lib.UpsampleError, match="CAPACITY"):
        upsampler.step_noalloc(_params(sc), dev(big, torch), dev(big, torch), None, hx, hx, ox, ov)
    p = _params(sc)
    p["domain_hi"] = (10.0, 10.0, 10.0)          # 56^3 cells at r = 0.02: above the maximum
    with pytest.raises(_lib.UpsampleError, match="CAPACITY"):
        upsampler.step_noalloc(p, dev(X, torch), dev(V, torch), None, hx, hx, ox, ov)
    q = _params(sc)
    q["validate"] = True
    with pytest.raises(_lib.UpsampleError, match="INVALID_ARG"):
        upsampler.step_noalloc(q, dev(X, torch), dev(V, torch), None, hx, hx, ox, ov)
    # the rejected calls enqueued nothing: a valid call still matches
    (ax, av), (bx, bv) = _pair(upsampler, sc, X, V, None, sc.hr_x0, sc.hr_v0)
    assert torch.equal(ax, bx) and torch.equal(av, bv)
