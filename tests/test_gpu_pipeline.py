"""The upsampling driven by the GPU's own LR simulation (Section 3 feeding
Section 4): HR initial state by volume sampling, LR frames from the LR step at
dt_LR, HR steps of dt_HR against the interpolated LR state, with the static
boundary samples and the moving rigid bodies flagged rigid (the rigid rule of
Section 4 on bodies coupled to the sand by shape matching).  Each HR step is
compared with the oracle's step of the GPU's own state before it, every
particle, with the LR state the oracle interpolates from the GPU's frames."""
import numpy as np
import pytest

from oracle import multirate_oracle as MR
from workloads import lr_scenes as S
from workloads.generators import box_candidates, box_walls

from gpu_util import compare_step, dev, host, log

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DT_LR = 0.005
DT_HR = 1.0 / 60.0


@pytest.fixture(scope="module")
def libs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_01629_amd.lr_sim import LRSim
    from paper_2308_01629_amd.upsampler import Upsampler, sample_volume
    return LRSim, Upsampler, sample_volume


def test_impact_scene_upsampled_from_gpu_frames(libs):
    LRSim, Upsampler, sample_volume = libs
    sc = S.impact(True)
    L = float(sc.x[0, sc.body == S.STATIC].max()) - sc.r
    depth = float(sc.x[1, sc.body == S.GRANULAR].max())
    r_hr = sc.r / 3
    cand = box_candidates((0.0, 0.0, 0.0), (L, depth, L), 400_000, [61, 1])
    hx = sample_volume(dev(cand, torch), r_hr, (0.0, 0.0, 0.0), (L, depth, L))
    hv = torch.zeros_like(hx)
    n_hr = hx.shape[1]
    T = 4
    n_lr = int(np.ceil(T * DT_HR / DT_LR)) + 1
    sim = LRSim(sc.body, sc.inv_m, sc.rest, sc.r, sc.domain_lo, sc.domain_hi, dt=DT_LR, g=sc.g)
    x, v = dev(sc.x, torch), dev(sc.v, torch)
    fx, fv = sim.step(x, v, n_lr, frames=True)
    LX = torch.cat([dev(sc.x, torch)[None], fx]).contiguous()
    LV = torch.cat([dev(sc.v, torch)[None], fv]).contiguous()
    frames = [(host(LX[k]), host(LV[k])) for k in range(n_lr + 1)]
    walls = np.stack(box_walls(np.zeros(3), np.array([L, 1.0, L]))).astype(np.float32)
    up = Upsampler(sc.r, r_hr, DT_HR, sc.g, sc.domain_lo, sc.domain_hi, walls=walls, max_lr=sc.n, max_hr=n_hr)
    rigid_d = dev(sc.lr_rigid, torch)
    prm = dict(r_lr=float(np.float32(sc.r)), r_hr=float(np.float32(r_hr)), dt=float(np.float32(DT_HR)),
               g=np.asarray(sc.g, np.float32), c1=512.0 / 729.0, c2=0.6, domain_lo=sc.domain_lo,
               domain_hi=sc.domain_hi, walls=walls)
    rigid = sc.lr_rigid.astype(bool)
    box = float(np.max(sc.domain_hi - sc.domain_lo))
    moving = 0
    for n in range(T):
        x0, v0 = host(hx).copy(), host(hv).copy()
        up.run_multirate(LX, LV, hx, hv, n_steps=1, dt_lr=DT_LR, t_hr0=n * DT_HR, lr_rigid=rigid_d)
        torch.cuda.synchronize()
        (k, th), = MR.hr_schedule(n * DT_HR, DT_HR, 1, 0.0, DT_LR, len(frames))
        X, V = MR.lerp_frame_f32(*frames[k], *frames[k + 1], th)
        s = compare_step(host(hx), host(hv), X, V, rigid, x0, v0, prm, box)
        moving = max(moving, int((np.abs(V[:, sc.body >= 0]).max(axis=0) > 0.05).sum()))
        log(f"pipeline impact step {n}: frames {k}, {k + 1}, theta {th:.4f}, {n_hr} HR: {s}")
    assert moving > 0, "the rigid bodies should be moving"
    assert not sim.overflow()
    sim.close()
    up.close()


def test_column_collapse_full_size_sampled(libs):
    """The configuration the bench's pipeline leg times: the column collapse
    (23,609 LR) by the LR step, about 370k HR volume-sampled in the column
    (r_HR = 0.3 r_LR), HR steps of 1/60 s with a reorder; each step against
    the oracle on 4,096 sampled HR particles from the GPU's own state."""
    from workloads.generators import volume_candidates
    LRSim, Upsampler, sample_volume = libs
    sc = S.column_collapse()
    r_hr = 0.3 * sc.r
    top = float(sc.x[1, sc.body == S.GRANULAR].max()) + sc.r
    cand, lo, hi = volume_candidates("column", 8_000_000, [47, 2], top=top)
    hx = sample_volume(dev(cand, torch), r_hr, lo, hi)
    del cand
    hv = torch.zeros_like(hx)
    n_hr = hx.shape[1]
    T = 4
    n_lr = int(np.ceil(T * DT_HR / DT_LR)) + 1
    sim = LRSim(sc.body, sc.inv_m, sc.rest, sc.r, sc.domain_lo, sc.domain_hi, dt=DT_LR, g=sc.g)
    x, v = dev(sc.x, torch), dev(sc.v, torch)
    fx, fv = sim.step(x, v, n_lr, frames=True)
    LX = torch.cat([dev(sc.x, torch)[None], fx]).contiguous()
    LV = torch.cat([dev(sc.v, torch)[None], fv]).contiguous()
    frames = [(host(LX[k]), host(LV[k])) for k in range(n_lr + 1)]
    walls = np.stack(box_walls(np.zeros(3), np.array([2.0, 1.5, 2.0]))).astype(np.float32)
    up = Upsampler(sc.r, r_hr, DT_HR, sc.g, sc.domain_lo, sc.domain_hi, walls=walls, max_lr=sc.n, max_hr=n_hr)
    up.sort_hr(hx, hv, with_perm=False)
    rigid_d = dev(sc.lr_rigid, torch)
    prm = dict(r_lr=float(np.float32(sc.r)), r_hr=float(np.float32(r_hr)), dt=float(np.float32(DT_HR)),
               g=np.asarray(sc.g, np.float32), c1=512.0 / 729.0, c2=0.6, domain_lo=sc.domain_lo,
               domain_hi=sc.domain_hi, walls=walls)
    rigid = sc.lr_rigid.astype(bool)
    box = float(np.max(sc.domain_hi - sc.domain_lo))
    idx = np.sort(np.random.default_rng(9).choice(n_hr, 4096, replace=False))
    for n in range(T):
        x0, v0 = host(hx).copy(), host(hv).copy()
        up.run_multirate(LX, LV, hx, hv, n_steps=1, dt_lr=DT_LR, t_hr0=n * DT_HR, lr_rigid=rigid_d)
        torch.cuda.synchronize()
        (k, th), = MR.hr_schedule(n * DT_HR, DT_HR, 1, 0.0, DT_LR, len(frames))
        X, V = MR.lerp_frame_f32(*frames[k], *frames[k + 1], th)
        s = compare_step(host(hx), host(hv), X, V, rigid, x0, v0, prm, box, idx=idx)
        log(f"pipeline column step {n}: frames {k}, {k + 1}, theta {th:.4f}, {n_hr} HR (4,096 sampled): {s}")
    assert not sim.overflow()
    sim.close()
    up.close()


def test_drain_running_out_full_size_sampled(libs):
    """The drain by the LR step (65,536 granular LR on the static samples of
    its silo, hopper and plate, dt_LR = 0.0025 s by the CFL condition, up to
    64 pairs per particle), about 2M HR volume-sampled in the silo
    (r_HR = r_LR / 4) behind the drain's 11 analytic walls: 30 HR steps run
    while the sand starts through the orifice, then three HR steps, each
    against the oracle on 4,096 sampled HR particles from the GPU's own
    state."""
    from workloads.generators import make_geometry, volume_candidates
    LRSim, Upsampler, sample_volume = libs
    sc = S.drain_flow()
    r_hr = 0.25 * sc.r
    top = float(sc.x[1, sc.body == S.GRANULAR].max()) + sc.r
    cand, lo, hi = volume_candidates("drain", 16_000_000, [43, 1], top=top)
    hx = sample_volume(dev(cand, torch), r_hr, lo, hi)
    del cand
    hv = torch.zeros_like(hx)
    n_hr = hx.shape[1]
    T0, T = 30, 3
    dt_lr = sc.dt   # the CFL-limited step of the drain
    n_lr = int(np.ceil((T0 + T) * DT_HR / dt_lr)) + 1
    sim = LRSim(sc.body, sc.inv_m, sc.rest, sc.r, sc.domain_lo, sc.domain_hi, dt=dt_lr, g=sc.g, max_neighbors=64)
    x, v = dev(sc.x, torch), dev(sc.v, torch)
    fx, fv = sim.step(x, v, n_lr, frames=True)
    LX = torch.cat([dev(sc.x, torch)[None], fx]).contiguous()
    LV = torch.cat([dev(sc.v, torch)[None], fv]).contiguous()
    del fx, fv
    walls = np.stack(make_geometry("drain").walls).astype(np.float32)
    up = Upsampler(sc.r, r_hr, DT_HR, sc.g, sc.domain_lo, sc.domain_hi, walls=walls, max_lr=sc.n, max_hr=n_hr)
    up.sort_hr(hx, hv, with_perm=False)
    rigid_d = dev(sc.lr_rigid, torch)
    up.run_multirate(LX, LV, hx, hv, n_steps=T0, dt_lr=dt_lr, sort_every=10, lr_rigid=rigid_d)
    prm = dict(r_lr=float(np.float32(sc.r)), r_hr=float(np.float32(r_hr)), dt=float(np.float32(DT_HR)),
               g=np.asarray(sc.g, np.float32), c1=512.0 / 729.0, c2=0.6, domain_lo=sc.domain_lo,
               domain_hi=sc.domain_hi, walls=walls)
    rigid = sc.lr_rigid.astype(bool)
    box = float(np.max(sc.domain_hi - sc.domain_lo))
    idx = np.sort(np.random.default_rng(10).choice(n_hr, 4096, replace=False))
    below = int((host(LX[-1])[1, sc.body == S.GRANULAR] < 0.6).sum())
    for n in range(T0, T0 + T):
        x0, v0 = host(hx).copy(), host(hv).copy()
        up.run_multirate(LX, LV, hx, hv, n_steps=1, dt_lr=dt_lr, t_hr0=n * DT_HR, lr_rigid=rigid_d)
        torch.cuda.synchronize()
        k_th = MR.hr_schedule(n * DT_HR, DT_HR, 1, 0.0, dt_lr, n_lr + 1)
        (k, th), = k_th
        X, V = MR.lerp_frame_f32(host(LX[k]), host(LV[k]), host(LX[k + 1]), host(LV[k + 1]), th)
        s = compare_step(host(hx), host(hv), X, V, rigid, x0, v0, prm, box, idx=idx)
        log(f"pipeline drain step {n}: frames {k}, {k + 1}, theta {th:.4f}, {n_hr} HR (4,096 sampled), "
            f"{below} LR below the plate at the last frame: {s}")
    assert below > 0, "the sand should be running out"
    assert not sim.overflow()
    sim.close()
    up.close()
