"""Pins of the oracle's adjoint (a reading: the paper does not differentiate the
step) against float64 central finite differences of the oracle's own forward,
and against the closed-form derivative of the one-neighbour case.  No GPU."""
import numpy as np
import pytest

from oracle import upsample_oracle as O
from workloads.generators import build_scene


def _prm(sc):
    return sc.params()


def _flags(o):
    return (o["A"].copy(), o["count"].copy(), o["wall"]["pushed"].copy(),
            o["wall"]["clipped"].copy(), _argmax(o))


def _argmax(o):
    ii, jj, w = o["ii"], o["jj"], o["w"]
    N = o["S"].size
    arg = np.full(N, -1)
    if ii.size:
        order = np.lexsort((jj, -w, ii))
        first = np.ones(order.size, bool)
        first[1:] = ii[order][1:] != ii[order][:-1]
        arg[ii[order][first]] = jj[order][first]
    return arg


def _same(f1, f2):
    return all(np.array_equal(a, b) for a, b in zip(f1, f2))


def test_single_neighbour_closed_form_derivative():
    r, dt = 0.02, 1.0 / 60.0
    prm = dict(r_lr=r, r_hr=0.005, dt=dt, g=np.array([0, -9.81, 0.0]), c1=O.C1, c2=O.C2,
               walls=np.zeros((0, 12), np.float32))
    hr_x = np.array([[0.3], [0.4], [0.5]], np.float32)
    lr_x = (hr_x + np.array([[0.02], [0.01], [-0.005]], np.float32)).astype(np.float32)
    V = np.array([[0.5], [-1.0], [2.0]], np.float32)
    v = np.array([[0.1], [0.2], [0.3]], np.float32)
    gx_out = np.array([[1.0], [2.0], [3.0]])
    gv_out = np.array([[-1.0], [0.5], [0.25]])
    b = O.step_backward(lr_x, V, None, hr_x, v, prm, gx_out, gv_out)
    d = lr_x.astype(np.float64) - hr_x.astype(np.float64)
    s = float(np.sum(d * d))
    h2 = 9 * np.float64(np.float32(r)) ** 2
    w = (1 - s / h2) ** 3
    # v' = w V + (1 - w)(v + dt g), x' = x + dt v'
    gvp = gv_out + dt * gx_out
    np.testing.assert_allclose(b["g_lr_v"], w * gvp, rtol=1e-13)
    np.testing.assert_allclose(b["gv"], (1 - w) * gvp, rtol=1e-13)
    # dv'/dw = V - (v + dt g); dw/dX = -6 (1 - s/h2)^2 (X - x) / h2
    dvdw = V.astype(np.float64) - (v.astype(np.float64) + dt * prm["g"][:, None])
    dwdX = -6.0 * (1 - s / h2) ** 2 * d / h2
    ref_X = float(np.sum(gvp * dvdw)) * dwdX
    np.testing.assert_allclose(b["g_lr_x"], ref_X, rtol=1e-12)
    np.testing.assert_allclose(b["gx"], gx_out - ref_X, rtol=1e-12)


@pytest.fixture(scope="module")
def small_heap():
    sc = build_scene("heap", 512, 8192, seed=[5, 99], with_target=True)
    X, V = sc.lr_frame(1)
    rng = np.random.default_rng(11)
    v = rng.normal(0, 0.5, sc.hr_x0.shape).astype(np.float32)
    rigid = (rng.uniform(size=sc.n_lr) < 0.1).astype(np.uint8)
    return sc, X, V, rigid, v


@pytest.mark.parametrize("space", ["lr_v", "lr_x", "hr_x", "hr_v"])
def test_step_adjoint_matches_central_fd(small_heap, space):
    sc, X, V, rigid, v = small_heap
    prm = _prm(sc)
    rng = np.random.default_rng({"lr_v": 1, "lr_x": 2, "hr_x": 3, "hr_v": 4}[space])
    inputs = {"lr_x": X.astype(np.float64), "lr_v": V.astype(np.float64),
              "hr_x": sc.hr_x0.astype(np.float64), "hr_v": v.astype(np.float64)}
    gx_out = rng.normal(size=sc.hr_x0.shape)
    gv_out = rng.normal(size=sc.hr_x0.shape)

    def run(inp):
        o = O.step(inp["lr_x"], inp["lr_v"], rigid, inp["hr_x"], inp["hr_v"], prm,
                   predicate="f64", keep=True)
        return float(np.sum(gx_out * o["x"]) + np.sum(gv_out * o["v"])), o

    b = O.step_backward(inputs["lr_x"], inputs["lr_v"], rigid, inputs["hr_x"], inputs["hr_v"], prm,
                        gx_out, gv_out, predicate="f64")
    grad = {"lr_x": b["g_lr_x"], "lr_v": b["g_lr_v"], "hr_x": b["gx"], "hr_v": b["gv"]}[space]
    eps = 1e-6 if space in ("lr_v", "hr_v") else 1e-8
    checked = 0
    for _ in range(40):
        direc = rng.normal(size=inputs[space].shape)
        if space in ("lr_x", "hr_x"):   # move a sparse subset so flips are rare
            direc *= rng.uniform(size=direc.shape[1]) < 0.05
        plus = dict(inputs)
        minus = dict(inputs)
        plus[space] = inputs[space] + eps * direc
        minus[space] = inputs[space] - eps * direc
        Lp, op = run(plus)
        Lm, om = run(minus)
        if not _same(_flags(op), _flags(om)):
            continue                    # a branch, argmax or wall flip: redraw
        fd = (Lp - Lm) / (2 * eps)
        an = float(np.sum(grad * direc))
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3 * np.abs(grad).sum() * eps + 1.0), (space, fd, an)
        checked += 1
        if checked == 16:
            break
    assert checked >= 12


def test_rollout_gradient_matches_fd():
    sc = build_scene("heap", 128, 1024, seed=[5, 7], with_target=True)
    prm = sc.params()
    T = 4
    frames = [tuple(a.astype(np.float64) for a in sc.lr_frame(t)) for t in range(1, T + 1)]
    x0, v0 = sc.hr_x0, sc.hr_v0

    def loss_and_flags(fr):
        x, v = x0.astype(np.float64), v0.astype(np.float64)
        flags = []
        for (X, V) in fr:
            o = O.step(X, V, sc.lr_rigid, x, v, prm, predicate="f64", keep=True)
            flags.append(_flags(o))
            x, v = o["x"], o["v"]
        d = x - sc.target.astype(np.float64)
        return float(np.sum(d * d) / x.shape[1]), flags

    L, g_X, g_V, _, _ = O.rollout_loss_grad(frames, sc.lr_rigid, x0, v0, prm, sc.target, predicate="f64")
    L2, _ = loss_and_flags(frames)
    assert abs(L - L2) < 1e-14
    rng = np.random.default_rng(3)
    eps = 1e-6
    checked = 0
    for _ in range(30):
        t = int(rng.integers(0, T))
        direc = rng.normal(size=frames[t][1].shape)
        fp = list(frames)
        fm = list(frames)
        fp[t] = (frames[t][0], frames[t][1] + eps * direc)
        fm[t] = (frames[t][0], frames[t][1] - eps * direc)
        Lp, flp = loss_and_flags(fp)
        Lm, flm = loss_and_flags(fm)
        if not all(_same(a, b) for a, b in zip(flp, flm)):
            continue
        fd = (Lp - Lm) / (2 * eps)
        an = float(np.sum(g_V[t] * direc))
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-6), (t, fd, an)
        checked += 1
        if checked == 12:
            break
    assert checked >= 8
