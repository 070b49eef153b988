"""GPU tests of the autotuner (upsample_autotune): it returns one of its
candidates, leaves the inputs untouched, caches its result in a JSON-lines
file, and a handle built from the result still matches the oracle."""
import json

import numpy as np
import pytest

from oracle import upsample_oracle as O
from workloads import configs

from gpu_util import compare_step, dev, host, log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KAPPAS = (0.51, 0.6, 0.75, 1.0001, 1.25)


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_01629_amd.upsampler import Upsampler, autotune
    return Upsampler, autotune


def test_autotune_cache_and_parity(mods, tmp_path):
    Upsampler, autotune = mods
    sc = configs.drain(scale=1 / 16)
    X, V = sc.lr_frame(2)
    hv0 = np.random.default_rng(8).normal(0, 0.5, sc.hr_x0.shape).astype(np.float32)
    lx, lv, hx, hv = dev(X, torch), dev(V, torch), dev(sc.hr_x0, torch), dev(hv0, torch)
    params = dict(r_lr=sc.r_lr, r_hr=sc.r_hr, dt=sc.dt, g=tuple(sc.g), domain_lo=tuple(sc.domain_lo),
                  domain_hi=tuple(sc.domain_hi), walls=sc.walls, c1=sc.c1, c2=sc.c2)
    cache = tmp_path / "tune.jsonl"
    r1 = autotune(params, lx, lv, hx, hv, cache_path=str(cache))
    torch.cuda.synchronize()
    log(f"autotune: {r1}")
    assert not r1["from_cache"] and r1["advance_ms"] > 0
    assert any(abs(r1["cell_factor"] - k) < 1e-6 for k in KAPPAS)
    assert r1["tuning"]["sort_sub"] in (1, 2) and r1["tuning"]["gather_groups"] in (1, 2)
    assert r1["tuning"]["tile_max"] in (384, 512, 768)
    assert np.array_equal(host(hx), sc.hr_x0) and np.array_equal(host(hv), hv0)   # inputs untouched
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and abs(json.loads(lines[0])["cell_factor"] - r1["cell_factor"]) < 1e-6
    r2 = autotune(params, lx, lv, hx, hv, cache_path=str(cache))
    assert r2["from_cache"] and r2["tuning"] == r1["tuning"] and abs(r2["cell_factor"] - r1["cell_factor"]) < 1e-6
    # a replay over three frames is a different problem with its own entry
    fr = [sc.lr_frame(t) for t in (2, 3, 4)]
    LX = dev(np.stack([f[0] for f in fr]), torch)
    LV = dev(np.stack([f[1] for f in fr]), torch)
    r3 = autotune(params, LX, LV, hx, hv, cache_path=str(cache))
    assert not r3["from_cache"] and len(cache.read_text().splitlines()) == 2
    assert np.array_equal(host(hx), sc.hr_x0) and np.array_equal(host(hv), hv0)
    # the tuned handle computes the same step (oracle parity on a sample)
    up = Upsampler.tuned(sc, lx, lv, hx, hv, cache_path=str(cache))
    assert up.autotune["from_cache"]
    sx, sv = hx.clone(), hv.clone()
    up.sort_hr(sx, sv, with_perm=False)
    x1, v1 = up.step(lx, lv, None, sx, sv)
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(9).choice(sc.n_hr, 16384, replace=False))
    s = compare_step(host(x1), host(v1), X, V, None, host(sx), host(sv), sc.params(), sc.box_length, idx=idx)
    log(f"tuned step vs oracle: {s}")
    gi = up.grid_info()
    spec = O.grid_spec(sc.r_lr, sc.domain_lo, sc.domain_hi, cell_factor=r1["cell_factor"])
    assert tuple(gi["dims"]) == tuple(spec.dims) and gi["reach"] == spec.reach
