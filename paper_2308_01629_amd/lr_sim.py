"""PyTorch-facing wrapper of the LR simulation step (Section 3, Algorithm 1)
in libupsample.so: ``upsample_pbd_*``.

Positions and velocities are contiguous float32 device tensors [3, n]; the
particle types, inverse masses and rest offsets are host arrays copied at
construction.  Argument marshalling only: the step runs in the HIP library.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from ._lib import PBD_GRANULAR, PBD_STATIC, PbdParams, check, lib

__all__ = ["LRSim", "PBD_GRANULAR", "PBD_STATIC"]


def _soa(t: torch.Tensor, n: int, name: str) -> None:
    if not (t.is_cuda and t.dtype == torch.float32 and t.dim() == 2 and t.shape == (3, n) and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 device tensor of shape [3, {n}]")


class LRSim:
    """One LR particle system: body [n] (PBD_GRANULAR, PBD_STATIC or rigid
    body ids 0 .. B-1), inv_mass [n], rest [3, n] (rest offsets of rigid
    particles from their body's centre)."""

    def __init__(self, body, inv_mass, rest, r: float, domain_lo: Sequence[float], domain_hi: Sequence[float],
                 dt: float = 0.005, g=(0.0, -9.81, 0.0), mu_s: float = 0.35, mu_k: float = 0.3,
                 ground_y: float = 0.0, stab_iters: int = 2, solve_iters: int = 5, mass_scaling: bool = True,
                 max_neighbors: int = 32):
        self._L = lib()
        p = PbdParams()
        check(self._L.upsample_pbd_default_params(ctypes.byref(p)))
        p.r, p.dt = float(r), float(dt)
        for a in range(3):
            p.g[a] = float(g[a])
            p.domain_lo[a] = float(domain_lo[a])
            p.domain_hi[a] = float(domain_hi[a])
        p.mu_s, p.mu_k, p.ground_y = float(mu_s), float(mu_k), float(ground_y)
        p.stab_iters, p.solve_iters, p.mass_scaling = int(stab_iters), int(solve_iters), int(bool(mass_scaling))
        p.max_neighbors = int(max_neighbors)
        self.params = p
        body = np.ascontiguousarray(body, dtype=np.int32)
        n = body.shape[0]
        inv_mass = np.ascontiguousarray(inv_mass, dtype=np.float32)
        rest = np.ascontiguousarray(rest, dtype=np.float32)
        if inv_mass.shape != (n,) or rest.shape != (3, n):
            raise ValueError("inv_mass must be [n] and rest [3, n]")
        self.n = n
        h = ctypes.c_void_p()
        check(self._L.upsample_pbd_init(ctypes.byref(p), n, body.ctypes.data, inv_mass.ctypes.data,
                                        rest.ctypes.data, ctypes.byref(h)))
        self._h = h
        info = (ctypes.c_int64 * 5)()
        check(self._L.upsample_pbd_info(h, info))
        self.n_bodies, self.max_neighbors, self.n_cells, self.trace_len = (int(info[i]) for i in range(1, 5))

    def _check(self, rc: int) -> None:
        check(rc, self._h, self._L.upsample_pbd_last_error)

    def step(self, x: torch.Tensor, v: torch.Tensor, n_steps: int = 1, frames: bool = False, out=None):
        """Advances x, v in place by n_steps; with frames=True also returns the
        states after each step ([n_steps, 3, n] twice), written into
        out = (fx, fv) if given."""
        _soa(x, self.n, "x")
        _soa(v, self.n, "v")
        fx = fv = None
        if frames:
            if out is not None:
                fx, fv = out
                for t in (fx, fv):
                    if not (t.is_cuda and t.dtype == torch.float32 and t.shape == (n_steps, 3, self.n)
                            and t.is_contiguous()):
                        raise ValueError(f"frame buffers must be contiguous float32 [{n_steps}, 3, {self.n}]")
            else:
                fx = torch.empty((n_steps, 3, self.n), dtype=torch.float32, device=x.device)
                fv = torch.empty_like(fx)
        self._check(self._L.upsample_pbd_step(self._h, x.data_ptr(), v.data_ptr(), int(n_steps),
                                              None if fx is None else fx.data_ptr(),
                                              None if fv is None else fv.data_ptr(),
                                              torch.cuda.current_stream().cuda_stream))
        return (fx, fv) if frames else None

    def overflow(self) -> bool:
        f = ctypes.c_int64()
        self._check(self._L.upsample_pbd_status(self._h, ctypes.byref(f), torch.cuda.current_stream().cuda_stream))
        return bool(f.value)

    def debug_step(self, x: torch.Tensor, v: torch.Tensor) -> dict:
        """One step that records every stage (upsample_pbd_debug_step); x, v
        advance in place.  Returns host arrays: w, v_pred, xt_pred, stab
        [(x, xt)], solve [(frames [B, 12], xt)], x, v, and the pair lists
        pairs[phase] = (cnt [n], ids [n, K])."""
        _soa(x, self.n, "x")
        _soa(v, self.n, "v")
        n, K, B = self.n, self.max_neighbors, self.n_bodies
        tr = torch.empty(self.trace_len, dtype=torch.float32, device=x.device)
        cnt = torch.empty((2, n), dtype=torch.int32, device=x.device)
        ids = torch.empty((2, n, K), dtype=torch.int32, device=x.device)
        self._check(self._L.upsample_pbd_debug_step(self._h, x.data_ptr(), v.data_ptr(), tr.data_ptr(),
                                                    self.trace_len, cnt.data_ptr(), ids.data_ptr(),
                                                    torch.cuda.current_stream().cuda_stream))
        t = tr.cpu().numpy()
        off = 0

        def take(m, shape):
            nonlocal off
            a = t[off:off + m].reshape(shape)
            off += m
            return a

        out = {"w": take(n, (n,)), "v_pred": take(3 * n, (3, n)), "xt_pred": take(3 * n, (3, n))}
        out["stab"] = [(take(3 * n, (3, n)), take(3 * n, (3, n))) for _ in range(self.params.stab_iters)]
        out["solve"] = [(take(12 * B, (B, 12)), take(3 * n, (3, n))) for _ in range(self.params.solve_iters)]
        out["x"] = take(3 * n, (3, n))
        out["v"] = take(3 * n, (3, n))
        assert off == self.trace_len
        c = cnt.cpu().numpy().view(np.uint32)
        i = ids.cpu().numpy().view(np.uint32)
        out["pairs"] = [(c[0], i[0]), (c[1], i[1])]
        return out

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.upsample_pbd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
