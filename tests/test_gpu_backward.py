"""GPU parity of the adjoint step and of the checkpointed rollout against the
oracle's reference gradient (tests/test_oracle_adjoint.py pins that to
float64 central differences).  Tolerance: norm-wise relative 1e-4 per step,
1e-3 over a rollout (float32 sums in a different order, float atomics)."""
import numpy as np
import pytest

from oracle import upsample_oracle as O
from workloads import configs
from workloads.generators import build_scene

from gpu_util import TOL_V, TOL_X, band_along, dev, host, log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def U():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_01629_amd.upsampler import Upsampler
    return Upsampler


def rel(got, ref):
    got = np.asarray(got, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30))


def _check_step(up, sc, X, V, rigid, hx, hv, gxo, gvo, tol=1e-4, idx=None):
    rig = None if rigid is None else dev(rigid, torch)
    gx, gv, glx, glv = up.step_backward(dev(X, torch), dev(V, torch), rig, dev(hx, torch), dev(hv, torch),
                                        dev(gxo, torch), dev(gvo, torch))
    torch.cuda.synchronize()
    sel = slice(None) if idx is None else idx
    b = O.step_backward(X, V, rigid, hx[:, sel], hv[:, sel], sc.params(), gxo[:, sel], gvo[:, sel])
    errs = {"g_lr_v": rel(host(glv), b["g_lr_v"]), "g_lr_x": rel(host(glx), b["g_lr_x"]),
            "gx": rel(host(gx)[:, sel], b["gx"]), "gv": rel(host(gv)[:, sel], b["gv"])}
    for k, e in errs.items():
        assert e < tol, (k, e, errs)
    return errs


@pytest.mark.parametrize("tiled", [1, 0])
def test_step_adjoint_plain(U, tiled):
    sc = configs.plain()
    up = U.from_scene(sc)
    up.set_tuning(adjoint_tiled=tiled)
    X, V = sc.lr_frame(2)
    rng = np.random.default_rng(1)
    hv = rng.normal(0, 0.5, sc.hr_x0.shape).astype(np.float32)
    gxo = rng.normal(size=sc.hr_x0.shape).astype(np.float32)
    gvo = rng.normal(size=sc.hr_x0.shape).astype(np.float32)
    errs = _check_step(up, sc, X, V, None, sc.hr_x0, hv, gxo, gvo)
    log(f"plain adjoint tiled={tiled}: {errs}")


def test_step_adjoint_rigid_walls_ragged(U):
    sc = build_scene("heap", 1500, 30001, seed=[21, 3], rigid_floor=True)
    X, V = sc.lr_frame(1)
    up = U.from_scene(sc, max_lr=X.shape[1])
    rng = np.random.default_rng(2)
    hx = sc.hr_x0.copy()
    hx[1, :2000] = rng.uniform(-0.01, 0.02, 2000).astype(np.float32)   # at the floor wall
    hv = rng.normal(0, 1.0, hx.shape).astype(np.float32)
    gxo = rng.normal(size=hx.shape).astype(np.float32)
    gvo = rng.normal(size=hx.shape).astype(np.float32)
    errs = _check_step(up, sc, X, V, sc.lr_rigid, hx, hv, gxo, gvo)
    log(f"rigid/walls adjoint: {errs}")


def test_step_adjoint_full_size_sampled(U):
    # the differentiation workload at full size; the upstream gradient is
    # non-zero on a sample of HR particles only, so the oracle needs just those
    sc = configs.diff()
    up = U.from_scene(sc)
    X, V = sc.lr_frame(3)
    rng = np.random.default_rng(3)
    idx = np.sort(rng.choice(sc.n_hr, 8192, replace=False))
    hv = rng.normal(0, 0.5, sc.hr_x0.shape).astype(np.float32)
    gxo = np.zeros(sc.hr_x0.shape, np.float32)
    gvo = np.zeros(sc.hr_x0.shape, np.float32)
    gxo[:, idx] = rng.normal(size=(3, idx.size))
    gvo[:, idx] = rng.normal(size=(3, idx.size))
    hx = dev(sc.hr_x0, torch)
    hvd = dev(hv, torch)
    perm = up.sort_hr(hx, hvd).long()          # the launch order the bench uses
    p = host(perm)
    errs = _check_step(up, sc, X, V, None, host(hx), host(hvd), gxo[:, p], gvo[:, p],
                       idx=np.nonzero(np.isin(p, idx))[0])
    log(f"diff full-size adjoint: {errs}")


def test_adjoint_tiled_matches_per_lane(U):
    sc = configs.drain(scale=1 / 16)
    up = U.from_scene(sc)
    X, V = (dev(a, torch) for a in sc.lr_frame(5))
    hx, hv = dev(sc.hr_x0, torch), dev(np.random.default_rng(4).normal(size=sc.hr_x0.shape).astype(np.float32), torch)
    up.sort_hr(hx, hv)
    g = torch.randn_like(hx), torch.randn_like(hv)
    out = {}
    for tiled in (0, 1):
        up.set_tuning(adjoint_tiled=tiled)
        out[tiled] = [host(t) for t in up.step_backward(X, V, None, hx, hv, *g)]
    # tiled, with the per-lane walk for every wave, for waves sent either way
    # by their lanes' stencils (limit 16), and for none
    for tmax in (0, 16, 1 << 30):
        up.set_tuning(adjoint_tiled=1, adjoint_tile_max=tmax)
        out[("limit", tmax)] = [host(t) for t in up.step_backward(X, V, None, hx, hv, *g)]
    torch.cuda.synchronize()
    for k, o in out.items():
        if k == 0:
            continue
        for a, b in zip(out[0], o):
            assert rel(b, a.astype(np.float64)) < 1e-5, k


def test_rollout_gradient(U):
    from paper_2308_01629_amd.autograd import rollout
    sc = build_scene("heap", 512, 8192, seed=[5, 11], with_target=True)
    T, every = 12, 4
    frames = [sc.lr_frame(t) for t in range(1, T + 1)]
    up = U.from_scene(sc)
    LX = torch.from_numpy(np.stack([f[0] for f in frames])).cuda().requires_grad_(True)
    LV = torch.from_numpy(np.stack([f[1] for f in frames])).cuda().requires_grad_(True)
    x0 = dev(sc.hr_x0, torch).requires_grad_(True)
    v0 = dev(sc.hr_v0, torch).requires_grad_(True)
    xT, vT = rollout(up, x0, v0, LX, LV, checkpoint_every=every)
    y = dev(sc.target, torch)
    loss = ((xT - y) ** 2).sum() / sc.n_hr
    loss.backward()
    torch.cuda.synchronize()
    L, g_X, g_V, gx0, _ = O.rollout_loss_grad(frames, sc.lr_rigid, sc.hr_x0, sc.hr_v0, sc.params(), sc.target)
    assert abs(float(loss.detach()) - L) <= 1e-5 * abs(L)
    e_v = rel(host(LV.grad).reshape(T, -1), np.stack(g_V).reshape(T, -1))
    e_x = rel(host(LX.grad).reshape(T, -1), np.stack(g_X).reshape(T, -1))
    e_0 = rel(host(x0.grad), gx0)
    log(f"rollout T={T}: loss {float(loss):.6e} vs {L:.6e}; rel err dV {e_v:.2e} dX {e_x:.2e} dx0 {e_0:.2e}")
    assert e_v < 1e-3 and e_x < 1e-3 and e_0 < 1e-3
    # the checkpoint interval does not change the gradient beyond float noise
    LV2 = LV.detach().clone().requires_grad_(True)
    xT2, _ = rollout(up, x0.detach(), v0.detach(), LX.detach(), LV2, checkpoint_every=T)
    (((xT2 - y) ** 2).sum() / sc.n_hr).backward()
    torch.cuda.synchronize()
    assert rel(host(LV2.grad), host(LV.grad).astype(np.float64)) < 1e-5


def test_rollout_reorder_is_transparent(U):
    # reordering the HR state at checkpoints changes trajectories and
    # gradients by rounding only, up to rare alpha-branch flips
    from paper_2308_01629_amd.autograd import rollout
    sc = configs.drain(scale=1 / 32)
    T, every = 9, 3
    frames = [sc.lr_frame(t) for t in range(1, T + 1)]
    up = U.from_scene(sc)
    LX = torch.from_numpy(np.stack([f[0] for f in frames])).cuda()
    LV = torch.from_numpy(np.stack([f[1] for f in frames])).cuda()
    shuffle = np.random.default_rng(7).permutation(sc.n_hr)
    x0 = dev(sc.hr_x0[:, shuffle].copy(), torch)
    v0 = dev(sc.hr_v0[:, shuffle].copy(), torch)
    w = torch.randn_like(x0)
    res = {}
    for reorder, re in ((False, 0), (True, 0), (True, 2)):
        LVg = LV.clone().requires_grad_(True)
        x0g = x0.clone().requires_grad_(True)
        xT, vT = rollout(up, x0g, v0, LX, LVg, checkpoint_every=every, reorder=reorder, reorder_every=re)
        (xT * w).sum().backward()
        torch.cuda.synchronize()
        res[(reorder, re)] = (xT.detach(), vT.detach(), host(LVg.grad), host(x0g.grad))
    # the trajectory in the original order, state by state, for the band check
    states = [(host(x0), host(v0))]
    xs, vs = x0, v0
    for t in range(T):
        xs, vs = up.step(LX[t], LV[t], None, xs, vs)
        states.append((host(xs), host(vs)))
    torch.cuda.synchronize()
    base = res[(False, 0)]
    assert torch.equal(base[0], xs) and torch.equal(base[1], vs)
    for key in ((True, 0), (True, 2)):
        r = res[key]
        ddx = (base[0] - r[0]).abs().amax(dim=0)
        ddv = ((base[1] - r[1]).abs() / torch.clamp(base[1].abs(), min=1.0)).amax(dim=0)
        off_idx = host(torch.nonzero((ddx > TOL_X * sc.box_length * T) | (ddv > TOL_V * T)).flatten())
        off = int(off_idx.size)
        e_v = rel(r[2], base[2].astype(np.float64))
        e_0 = rel(r[3], base[3].astype(np.float64))
        log(f"reorder rollout {key}: median |dx| {torch.median(ddx).item():.2e} rel |dv| "
            f"{torch.median(ddv).item():.2e}, {off} beyond; rel dV {e_v:.2e} dx0 {e_0:.2e}")
        # other waves round differently: a particle on an alpha or wall
        # threshold may take the other branch and follow another valid
        # trajectory; every particle that differs must have met a band
        banded = band_along(frames, states[:-1], off_idx, sc.params(),
                            drift=lambda t: TOL_X * sc.box_length * (t + 1))
        assert banded.all(), (key, int((~banded).sum()), off)
        assert off <= max(5, 1e-4 * sc.n_hr), (key, off)
        assert e_v < 1e-3 and e_0 < 1e-3


@pytest.mark.parametrize("case", ["plain", "rigid", "drain"])
def test_taped_step_and_adjoint(U, case):
    # the taped forward writes the same state as the plain step and records
    # the sums; the taped adjoint matches the recomputing one and the oracle
    if case == "rigid":
        sc = build_scene("heap", 1500, 30001, seed=[21, 3], rigid_floor=True)
        X, V = sc.lr_frame(1)
        up = U.from_scene(sc, max_lr=X.shape[1])
        rig = sc.lr_rigid
    else:
        sc = configs.plain() if case == "plain" else configs.drain(scale=1 / 16)
        X, V = sc.lr_frame(2)
        up = U.from_scene(sc)
        rig = None
    rng = np.random.default_rng(12)
    hx, hv = dev(sc.hr_x0, torch), dev(rng.normal(0, 0.5, sc.hr_x0.shape).astype(np.float32), torch)
    if case == "drain":
        up.sort_hr(hx, hv, with_perm=False)
    Xd, Vd = dev(X, torch), dev(V, torch)
    rd = None if rig is None else dev(rig, torch)
    tape = torch.empty((6, sc.n_hr), dtype=torch.float32, device="cuda")
    x0, v0 = up.step(Xd, Vd, rd, hx, hv)
    x1, v1 = up.step(Xd, Vd, rd, hx, hv, tape=tape)
    torch.cuda.synchronize()
    assert torch.equal(x0, x1) and torch.equal(v0, v1)
    # the record against the oracle's sums (membership of the float32 predicate)
    o = O.step(X, V, rig, host(hx), host(hv), sc.params())
    t = host(tape).astype(np.float64)
    np.testing.assert_allclose(t[0], o["S"], rtol=2e-5, atol=1e-6)
    np.testing.assert_allclose(t[4], o["M"], rtol=2e-5, atol=1e-6)
    gxo = torch.randn_like(hx)
    gvo = torch.randn_like(hv)
    a = up.step_backward(Xd, Vd, rd, hx, hv, gxo, gvo)
    b = up.step_backward(Xd, Vd, rd, hx, hv, gxo, gvo, tape=tape)
    torch.cuda.synchronize()
    for p_, q_ in zip(a, b):
        assert rel(host(q_), host(p_).astype(np.float64)) < 1e-5
    errs = _check_step(up, sc, X, V, rig, host(hx), host(hv), host(gxo), host(gvo))
    log(f"taped adjoint {case}: {errs}")


@pytest.mark.parametrize("case", ["plain", "rigid", "drain"])
def test_taped_adjoint_from_saved_grid(U, case):
    """The taped adjoint on a saved grid (upsample_grid_snapshot after the
    taped step, upsample_step_backward_taped_grid), with another frame's grid
    built on the handle in between, against the taped adjoint that rebuilds
    the grid: HR gradients bit for bit; LR gradients bit for bit with the
    deterministic LR sums and to float32 rounding with the atomic ones.  The
    saved-grid gradients are also checked against the oracle's."""
    if case == "rigid":
        sc = build_scene("heap", 1500, 30001, seed=[21, 3], rigid_floor=True)
        X, V = sc.lr_frame(1)
        X2, V2 = sc.lr_frame(2)
        rig = sc.lr_rigid
    else:
        sc = configs.plain() if case == "plain" else configs.drain(scale=1 / 16)
        X, V = sc.lr_frame(2)
        X2, V2 = sc.lr_frame(3)
        rig = None
    rng = np.random.default_rng(33)
    hx = dev(sc.hr_x0, torch)
    hv = dev(rng.normal(0, 0.5, sc.hr_x0.shape).astype(np.float32), torch)
    idx = None if sc.n_hr <= 65536 else np.sort(rng.choice(sc.n_hr, 4096, replace=False))
    sel = slice(None) if idx is None else idx
    gxo = np.zeros(sc.hr_x0.shape, np.float32)
    gvo = np.zeros(sc.hr_x0.shape, np.float32)
    gxo[:, sel] = rng.normal(size=gxo[:, sel].shape)
    gvo[:, sel] = rng.normal(size=gvo[:, sel].shape)
    Xd, Vd, X2d, V2d = dev(X, torch), dev(V, torch), dev(X2, torch), dev(V2, torch)
    rd = None if rig is None else dev(rig, torch)
    g = (dev(gxo, torch), dev(gvo, torch))
    for det in (False, True):
        up = U.from_scene(sc, deterministic_bwd=det, max_lr=X.shape[1])
        if case == "drain":
            up.sort_hr(hx, hv, with_perm=False)
        tape = torch.empty((6, sc.n_hr), dtype=torch.float32, device="cuda")
        up.step(Xd, Vd, rd, hx, hv, tape=tape)
        grid = up.grid_snapshot()
        assert grid.numel() == up.grid_snapshot_bytes() and up.grid_snapshot_bytes() % 256 == 0
        up.step(X2d, V2d, rd, hx, hv)  # the handle's grid is now another frame's
        a = up.step_backward(Xd, Vd, rd, hx, hv, *g, tape=tape)  # rebuilds frame (X, V)
        up.step(X2d, V2d, rd, hx, hv)
        b = up.step_backward(Xd, Vd, rd, hx, hv, *g, tape=tape, grid=grid)
        c = up.step_backward(Xd, Vd, rd, hx, hv, *g, tape=tape, grid=grid)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), (case, det)
        assert torch.equal(b[0], c[0]) and torch.equal(b[1], c[1]), (case, det)
        for p_, q_ in zip(a[2:], b[2:]):
            if det:
                assert torch.equal(p_, q_), (case, "deterministic LR gradients differ")
            else:
                assert rel(host(q_), host(p_).astype(np.float64)) < 1e-5, case
        o = O.step_backward(X, V, rig, host(hx)[:, sel], host(hv)[:, sel], sc.params(), gxo[:, sel],
                            gvo[:, sel])
        errs = {"g_lr_v": rel(host(b[3]), o["g_lr_v"]), "g_lr_x": rel(host(b[2]), o["g_lr_x"]),
                "gx": rel(host(b[0])[:, sel], o["gx"]), "gv": rel(host(b[1])[:, sel], o["gv"])}
        for k, e in errs.items():
            assert e < 1e-4, (case, det, k, e, errs)
        log(f"saved-grid taped adjoint {case} det={det}: {errs}")
        up.close()


def test_grid_snapshot_errors(U):
    # a snapshot before any grid is a call-order error; misaligned or short
    # snapshot buffers are rejected before any device work
    from paper_2308_01629_amd import _lib
    sc = configs.plain()
    up = U.from_scene(sc)
    nb = up.grid_snapshot_bytes()
    buf = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    assert buf.data_ptr() % 256 == 0
    L = _lib.lib()
    assert L.upsample_grid_snapshot(up._h, buf.data_ptr(), None) == _lib.ERR_CODES["UPSAMPLE_ERR_STATE"]
    X, V = sc.lr_frame(1)
    hx, hv = dev(sc.hr_x0, torch), dev(sc.hr_v0, torch)
    up.step(dev(X, torch), dev(V, torch), None, hx, hv)
    inv = _lib.ERR_CODES["UPSAMPLE_ERR_INVALID_ARG"]
    assert L.upsample_grid_snapshot(up._h, buf.data_ptr() + 16, None) == inv
    assert L.upsample_step_backward_taped_grid(up._h, buf.data_ptr() + 16, None, X.shape[1], None, None, 0,
                                               None, None, None, None, None, None, None, None) == inv
    with pytest.raises(ValueError):
        up.grid_snapshot(out=buf[:nb - 256])
    assert L.upsample_grid_snapshot(up._h, buf.data_ptr(), None) == 0
    torch.cuda.synchronize()
    up.close()


def test_adjoint_scratch_cleared_between_calls(U):
    # The tiled adjoint sums LR gradients by sorted index in handle scratch
    # that its last kernel empties again: repeated calls on one handle, and a
    # call with fewer LR particles in between, must give the same gradients.
    sc = configs.plain()
    up = U.from_scene(sc)
    X, V = sc.lr_frame(2)
    rng = np.random.default_rng(4)
    hx = dev(sc.hr_x0, torch)
    hv = dev(rng.normal(0, 0.5, sc.hr_x0.shape).astype(np.float32), torch)
    g = [dev(rng.normal(size=sc.hr_x0.shape).astype(np.float32), torch) for _ in range(2)]
    Xd, Vd = dev(X, torch), dev(V, torch)
    first = [host(t) for t in up.step_backward(Xd, Vd, None, hx, hv, *g)]
    half = X.shape[1] // 2
    up.step_backward(Xd[:, :half].contiguous(), Vd[:, :half].contiguous(), None, hx, hv, *g)
    again = [host(t) for t in up.step_backward(Xd, Vd, None, hx, hv, *g)]
    torch.cuda.synchronize()
    for a, b in zip(first, again):
        assert rel(b, a) < 1e-5, rel(b, a)
    assert np.abs(first[2]).sum() > 0 and np.abs(first[3]).sum() > 0


@pytest.mark.parametrize("case", ["plain", "rigid", "diff"])
def test_deterministic_backward(U, case):
    """UPSAMPLE_FLAG_DETERMINISTIC_BWD: repeated backward calls (recomputing
    and taped) give the same bits, the HR gradients equal the atomic
    adjoint's bit for bit (its tiled HR pass, and the per-lane one with
    adjoint_tiled 0), LR gradients are added to what the caller passes, and
    everything matches the oracle's reference gradient."""
    rig = None
    if case == "rigid":
        sc = build_scene("heap", 1500, 30001, seed=[21, 3], rigid_floor=True)
        X, V = sc.lr_frame(1)
        rig = sc.lr_rigid
    elif case == "plain":
        sc = configs.plain()
        X, V = sc.lr_frame(2)
    else:
        sc = configs.diff()
        X, V = sc.lr_frame(3)
    kw = dict(max_lr=X.shape[1])
    up = U.from_scene(sc, deterministic_bwd=True, **kw)
    ref = U.from_scene(sc, **kw)  # the atomic adjoint, the same HR pass
    rng = np.random.default_rng(21)
    hx = dev(sc.hr_x0, torch)
    hv = dev(rng.normal(0, 0.5, sc.hr_x0.shape).astype(np.float32), torch)
    if case == "diff":
        up.sort_hr(hx, hv, with_perm=False)
    idx = None if sc.n_hr <= 65536 else np.sort(rng.choice(sc.n_hr, 8192, replace=False))
    gxo = np.zeros(sc.hr_x0.shape, np.float32)
    gvo = np.zeros(sc.hr_x0.shape, np.float32)
    sel = slice(None) if idx is None else idx
    gxo[:, sel] = rng.normal(size=gxo[:, sel].shape)
    gvo[:, sel] = rng.normal(size=gvo[:, sel].shape)
    Xd, Vd = dev(X, torch), dev(V, torch)
    rd = None if rig is None else dev(rig, torch)
    g = (dev(gxo, torch), dev(gvo, torch))
    runs = [up.step_backward(Xd, Vd, rd, hx, hv, *g) for _ in range(3)]
    base = ref.step_backward(Xd, Vd, rd, hx, hv, *g)
    tape = torch.empty((6, sc.n_hr), dtype=torch.float32, device="cuda")
    up.step(Xd, Vd, rd, hx, hv, tape=tape)
    taped = [up.step_backward(Xd, Vd, rd, hx, hv, *g, tape=tape) for _ in range(2)]
    ones = (torch.ones_like(Xd), torch.ones_like(Vd))
    added = up.step_backward(Xd, Vd, rd, hx, hv, *g, g_lr_x=ones[0].clone(), g_lr_v=ones[1].clone())
    # the per-lane HR pass on both sides
    up.set_tuning(adjoint_tiled=0)
    ref.set_tuning(adjoint_tiled=0)
    lane = up.step_backward(Xd, Vd, rd, hx, hv, *g)
    lane_ref = ref.step_backward(Xd, Vd, rd, hx, hv, *g)
    torch.cuda.synchronize()
    assert torch.equal(lane[0], lane_ref[0]) and torch.equal(lane[1], lane_ref[1])
    for p_, q_ in zip(lane[2:], runs[0][2:]):
        assert rel(host(p_), host(q_).astype(np.float64)) < 1e-5
    for r in runs[1:]:
        for p_, q_ in zip(runs[0], r):
            assert torch.equal(p_, q_), "deterministic backward differs between calls"
    for p_, q_ in zip(taped[0], taped[1]):
        assert torch.equal(p_, q_), "deterministic taped backward differs between calls"
    assert torch.equal(runs[0][0], base[0]) and torch.equal(runs[0][1], base[1])
    assert torch.equal(added[2], 1.0 + runs[0][2]) and torch.equal(added[3], 1.0 + runs[0][3])
    for p_, q_ in zip(taped[0], runs[0]):
        assert rel(host(p_), host(q_).astype(np.float64)) < 1e-5
    for p_, q_ in zip(base[2:], runs[0][2:]):
        assert rel(host(q_), host(p_).astype(np.float64)) < 1e-5
    b = O.step_backward(X, V, rig, host(hx)[:, sel], host(hv)[:, sel], sc.params(), gxo[:, sel], gvo[:, sel])
    errs = {"g_lr_v": rel(host(runs[0][3]), b["g_lr_v"]), "g_lr_x": rel(host(runs[0][2]), b["g_lr_x"]),
            "gx": rel(host(runs[0][0])[:, sel], b["gx"]), "gv": rel(host(runs[0][1])[:, sel], b["gv"])}
    for k, e in errs.items():
        assert e < 1e-4, (k, e, errs)
    log(f"deterministic backward {case}: bitwise repeatable, {errs}")
