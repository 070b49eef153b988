"""Throughput of the HR upsampling step on one MI355X.

One step = the whole hot path for one LR frame: LR grid rebuild (cell keys,
counting sort, cell ranges, sorted LR copy) and the fused gather / blend /
integrate / wall kernel over every HR particle, plus (every --sort-every steps)
the HR reorder by cell that keeps waves spatially coherent.

Default workload: the drain (65,536 LR, 4,194,304 HR, 60 degree hopper and
orifice walls).  Inputs are seeded synthetic data generated on the host and
uploaded before timing: the timed region starts with all LR frames and the HR
state resident in HBM.

Prints ONE JSON line.  Besides the headline value it carries the roofline of the
dominant kernel (the fused gather, timed with HIP events on its own stream),
the oracle timed on the host cores on a bounded sample, the backward/forward
time ratio on the differentiation workload and the batched-vs-plain speedup.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s
METRIC = "high-res particle updates/s + % HBM peak; backward/forward time ratio"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sort-every", type=int, default=10)
    ap.add_argument("--sort-sub", type=int, default=0, help="HR reorder sub-cells per axis (0: library default)")
    ap.add_argument("--groups", type=int, default=0, help="gather lane groups per wave (0: library default)")
    ap.add_argument("--cell-factor", type=float, default=0.0)
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the backward and batched legs")
    ap.add_argument("--only", choices=["drain", "diff", "batched"], default=None,
                    help="run one leg only (profiling)")
    return ap.parse_args()


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2308_01629_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_src: str, n_launch_units: dict):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, only when
    it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "advance_drain_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash(kernel_src):
        return None
    return rec.get("hbm_bytes_per_launch")


def drain_leg(args, torch, Upsampler):
    from workloads import configs
    t0 = time.time()
    sc = configs.drain()
    n_frames = args.warmup + args.steps
    log(f"drain: {sc.n_lr} LR, {sc.n_hr} HR, generating {n_frames} LR frames")
    frames = [sc.lr_frame(t) for t in range(1, n_frames + 1)]
    LX = torch.from_numpy(np.stack([f[0] for f in frames])).cuda()
    LV = torch.from_numpy(np.stack([f[1] for f in frames])).cuda()
    hx = torch.from_numpy(sc.hr_x0).cuda()
    hv = torch.from_numpy(sc.hr_v0).cuda()
    up = Upsampler.from_scene(sc, cell_factor=args.cell_factor)
    if args.sort_sub:
        up.set_tuning(sort_sub=args.sort_sub)
    if args.groups:
        up.set_tuning(gather_groups=args.groups)
    gi = up.grid_info()
    log(f"drain: setup {time.time() - t0:.1f}s, grid {gi['dims']} reach {gi['reach']} tuning {up.get_tuning()}")
    up.sort_hr(hx, hv, with_perm=False)
    # HR state ping-pongs between two buffer pairs: the reorder writes the other pair
    state = [hx, hv, torch.empty_like(hx), torch.empty_like(hv)]

    def run(first, count, timed_kernel=False):
        up.timing_enable(timed_kernel)
        for k in range(count):
            t = first + k
            if args.sort_every and t % args.sort_every == 0:
                up.sort_hr(state[0], state[1], with_perm=False, out_x=state[2], out_v=state[3])
                state[0], state[1], state[2], state[3] = state[2], state[3], state[0], state[1]
            up.step(LX[t], LV[t], None, state[0], state[1], out_x=state[0], out_v=state[1])

    run(0, args.warmup)
    torch.cuda.synchronize()
    # every repeat replays the same K steps from the same post-warm-up state
    x_snap, v_snap = state[0].clone(), state[1].clone()
    times = []
    for rep in range(args.repeats + 1):
        state[0].copy_(x_snap)
        state[1].copy_(v_snap)
        timed_kernel = rep == args.repeats   # last pass: per-launch events on the gather kernel
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s0.record()
        run(args.warmup, args.steps, timed_kernel=timed_kernel)
        s1.record()
        torch.cuda.synchronize()
        if timed_kernel:
            adv_ms, launches = up.timing_read()
            up.timing_enable(False)
            log(f"drain: gather kernel {adv_ms * 1e3 / max(launches, 1):.1f} us/launch over {launches}")
        else:
            times.append(s0.elapsed_time(s1) / 1e3)
            log(f"drain: repeat {rep}: {times[-1] * 1e3 / args.steps:.4f} ms/step")
    elapsed = float(np.median(times))
    ms_step = elapsed * 1e3 / args.steps
    n_cells = gi["n_cells"]
    adv_bytes = 48 * sc.n_hr + 32 * sc.n_lr + 4 * (n_cells + 1)
    step_bytes = 48 * sc.n_hr + 89 * sc.n_lr + 8 * n_cells
    adv_s = adv_ms / 1e3 / max(launches, 1)
    traffic = traffic_from_profiles("advance.hip", {})
    rf = {"bound": "hbm", "kernel": "k_advance (fused gather/blend/integrate/walls)",
          "achieved": adv_bytes / adv_s / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
          "frac": adv_bytes / adv_s / HBM_PEAK, "traffic": traffic,
          "algorithmic_bytes_per_launch": adv_bytes, "avg_launch_us": adv_s * 1e6}
    res = {"value": sc.n_hr * args.steps / elapsed, "ms_per_step": ms_step,
           "step_hbm_frac": step_bytes / (ms_step / 1e3) / HBM_PEAK,
           "config": {"workload": "drain", "n_lr": sc.n_lr, "n_hr": sc.n_hr, "r_lr": sc.r_lr,
                      "r_hr": sc.r_hr, "dt": sc.dt, "walls": int(sc.walls.shape[0]),
                      "grid": list(gi["dims"]), "reach": gi["reach"], "sort_every": args.sort_every,
                      "tuning": up.get_tuning()},
           "roofline": rf, "scene": sc, "frames": frames}
    up.close()
    return res


def cpu_baseline(sc, frames, budget_s=12.0):
    """The oracle as it stands on a bounded sample of the drain workload: the
    full LR frame, a seeded sample of HR particles, one step."""
    from oracle import upsample_oracle as O
    rng = np.random.default_rng(0)
    X, V = frames[0]
    prm = sc.params()
    done, t_used, n = 0, 0.0, 65536
    while t_used < budget_s and done < sc.n_hr:
        idx = rng.choice(sc.n_hr, size=n, replace=False)
        t0 = time.perf_counter()
        O.step(X, V, None, sc.hr_x0[:, idx], sc.hr_v0[:, idx], prm)
        t_used += time.perf_counter() - t0
        done += n
    return {"value": done / t_used, "unit": "HR particle-updates/s", "cores": O.WORKERS,
            "kind": "oracle",
            "sample": f"{done} HR particles of the drain workload (random {n}-particle batches, "
                      f"full 65,536-particle LR frame), one step each, {t_used:.1f} s; numpy "
                      f"float64, KD-tree queries on {O.WORKERS} threads"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the upsampling path has no multi-GPU leg in this "
              f"build); got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_2308_01629_amd.upsampler import Upsampler
    torch.cuda.set_device(0)

    out = {"metric": METRIC, "unit": "HR particle-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic"}
    d = drain_leg(args, torch, Upsampler)
    out.update({k: d[k] for k in ("value", "ms_per_step", "config", "roofline", "step_hbm_frac")})
    if not args.no_cpu_baseline:
        log("cpu baseline: timing the oracle")
        out["cpu_baseline"] = cpu_baseline(d["scene"], d["frames"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
