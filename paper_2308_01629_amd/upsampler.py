"""PyTorch-facing wrapper of the C ABI: device tensors in, device tensors out.

Every array is a contiguous float32 CUDA (HIP) tensor of shape [3, n]
(structure of arrays).  Calls are enqueued on torch's current stream.  This
module only marshals arguments; all arithmetic runs in libupsample.so.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import GridInfo, Params, check, lib


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _soa(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float32 and t.dim() == 2 and t.shape[0] == 3
            and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 device tensor of shape [3, n]")
    return t


def _u8(t: Optional[torch.Tensor], n: int, name: str) -> Optional[torch.Tensor]:
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.uint8 and t.dim() == 1 and t.shape[0] == n and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous uint8 device tensor of shape [{n}]")
    return t


def _tape(t: torch.Tensor, n: int) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float32 and t.shape == (6, n) and t.is_contiguous()):
        raise ValueError(f"tape must be a contiguous float32 device tensor of shape [6, {n}]")
    return t


def _snapshot(t: torch.Tensor, nbytes: int) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.uint8 and t.dim() == 1 and t.numel() >= nbytes and t.is_contiguous()
            and t.data_ptr() % 256 == 0):
        raise ValueError(f"grid snapshot must be a contiguous 256-byte aligned uint8 device tensor of at least "
                         f"{nbytes} bytes")
    return t


def make_params(r_lr: float, r_hr: float, dt: float, g: Sequence[float], domain_lo, domain_hi,
                walls=None, max_lr: int = 0, max_hr: int = 0, c1: float = 512.0 / 729.0,
                c2: float = 0.6, cell_factor: float = 0.0, validate: bool = False,
                deterministic_bwd: bool = False):
    """Params struct plus the host wall buffer that must outlive the call using it."""
    p = Params()
    lib().upsample_default_params(ctypes.byref(p))
    p.r_lr, p.r_hr, p.dt = float(r_lr), float(r_hr), float(dt)
    for a in range(3):
        p.g[a] = float(g[a])
        p.domain_lo[a] = float(domain_lo[a])
        p.domain_hi[a] = float(domain_hi[a])
    p.c1, p.c2 = float(c1), float(c2)
    p.cell_factor = float(cell_factor)
    wbuf = None
    if walls is not None and len(walls):
        wbuf = np.ascontiguousarray(np.asarray(walls, dtype=np.float32).reshape(-1, _lib.WALL_FLOATS))
        p.n_walls = wbuf.shape[0]
        p.walls = wbuf.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    p.max_lr, p.max_hr = int(max_lr), int(max_hr)
    p.flags = (_lib.FLAG_VALIDATE if validate else 0) | (_lib.FLAG_DETERMINISTIC_BWD if deterministic_bwd else 0)
    return p, wbuf


def grid_info_for(**kw) -> dict:
    """Host-only grid of a parameter set (no device needed)."""
    p, _w = make_params(**kw)
    gi = GridInfo()
    check(lib().upsample_grid_info_for(ctypes.byref(p), ctypes.byref(gi)))
    return gi.as_dict()


def autotune(params: dict, lr_x, lr_v, hr_x, hr_v, lr_rigid=None, cache_path: Optional[str] = None) -> dict:
    """Fastest cell factor and launch knobs (upsample_autotune).  ``params``:
    the keyword arguments of :func:`make_params`; ``lr_x``, ``lr_v``: one
    frame [3, N_L] or consecutive frames [T, 3, N_L] of the run to replay."""
    p, _wbuf = make_params(**params)
    if lr_x.dim() == 2:
        lr_x, lr_v = lr_x.unsqueeze(0), lr_v.unsqueeze(0)
    if not (lr_x.is_cuda and lr_x.dtype == torch.float32 and lr_x.dim() == 3 and lr_x.shape[1] == 3
            and lr_x.is_contiguous() and lr_v.shape == lr_x.shape and lr_v.is_contiguous()
            and lr_v.dtype == torch.float32):
        raise ValueError("lr_x, lr_v must be contiguous float32 device tensors [T, 3, N_L]")
    n_frames, n_lr = lr_x.shape[0], lr_x.shape[2]
    n_hr = _soa(hr_x, "hr_x").shape[1]
    _soa(hr_v, "hr_v")
    _u8(lr_rigid, n_lr, "lr_rigid")
    r = _lib.AutotuneResult()
    check(lib().upsample_autotune(ctypes.byref(p), _ptr(lr_x), _ptr(lr_v), _ptr(lr_rigid), n_lr, n_frames,
                                  _ptr(hr_x), _ptr(hr_v), n_hr, cache_path.encode() if cache_path else None,
                                  _stream(), ctypes.byref(r)))
    t = r.tuning
    return {"cell_factor": float(r.cell_factor), "advance_ms": float(r.advance_ms),
            "from_cache": bool(r.from_cache),
            "tuning": {k: int(getattr(t, k)) for k in Upsampler.TUNING_KEYS}}


def step_noalloc(params: dict, lr_x, lr_v, lr_rigid, hr_x, hr_v, out_x, out_v) -> None:
    """upsample_step_noalloc: one step without a handle and without device
    allocation in the library (the caller passes the output tensors).
    ``params``: the keyword arguments of :func:`make_params`."""
    p, _wbuf = make_params(**params)
    nl = _soa(lr_x, "lr_x").shape[1]
    _soa(lr_v, "lr_v")
    _u8(lr_rigid, nl, "lr_rigid")
    n = _soa(hr_x, "hr_x").shape[1]
    for t, nm in ((hr_v, "hr_v"), (out_x, "out_x"), (out_v, "out_v")):
        _soa(t, nm)
    check(lib().upsample_step_noalloc(ctypes.byref(p), _ptr(lr_x), _ptr(lr_v), _ptr(lr_rigid), nl, _ptr(hr_x),
                                      _ptr(hr_v), _ptr(out_x), _ptr(out_v), n, _stream()))


def sample_volume(cand: torch.Tensor, r: float, lo, hi, max_out: Optional[int] = None) -> torch.Tensor:
    """upsample_sample_volume: one non-overlapping sample of radius r per cell
    of side 2r/sqrt(3), chosen among the candidates [3, M] (device float32);
    returns the samples [3, K] in cell-key order."""
    _soa(cand, "cand")
    m = cand.shape[1]
    cap = m if max_out is None else int(max_out)
    out = torch.empty((3, max(cap, 0)), dtype=torch.float32, device=cand.device)
    lo_c = (ctypes.c_float * 3)(*[float(v) for v in lo])
    hi_c = (ctypes.c_float * 3)(*[float(v) for v in hi])
    n = ctypes.c_int64()
    check(lib().upsample_sample_volume(_ptr(cand), m, float(r), lo_c, hi_c, _ptr(out), cap, ctypes.byref(n),
                                       _stream()))
    return out[:, :n.value].contiguous()


class Upsampler:
    """One handle of the library: a scene's parameters plus scratch for up to
    ``max_lr`` LR and ``max_hr`` HR particles."""

    def __init__(self, r_lr: float, r_hr: float, dt: float, g, domain_lo, domain_hi, walls=None,
                 max_lr: int = 0, max_hr: int = 0, c1: float = 512.0 / 729.0, c2: float = 0.6,
                 cell_factor: float = 0.0, validate: bool = False, deterministic_bwd: bool = False):
        self._L = lib()
        self.kw = dict(r_lr=r_lr, r_hr=r_hr, dt=dt, g=tuple(g), domain_lo=tuple(domain_lo),
                       domain_hi=tuple(domain_hi), walls=walls, max_lr=max_lr, max_hr=max_hr, c1=c1,
                       c2=c2, cell_factor=cell_factor, validate=validate, deterministic_bwd=deterministic_bwd)
        p, _wbuf = make_params(**self.kw)
        h = ctypes.c_void_p()
        check(self._L.upsample_init(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        self.max_lr, self.max_hr = int(max_lr), int(max_hr)

    @classmethod
    def from_scene(cls, scene, max_lr: Optional[int] = None, max_hr: Optional[int] = None, **kw):
        return cls(scene.r_lr, scene.r_hr, scene.dt, scene.g, scene.domain_lo, scene.domain_hi,
                   walls=scene.walls, max_lr=max_lr if max_lr is not None else scene.n_lr,
                   max_hr=max_hr if max_hr is not None else scene.n_hr, c1=scene.c1, c2=scene.c2, **kw)

    @classmethod
    def tuned(cls, scene, lr_x, lr_v, hr_x, hr_v, lr_rigid=None, cache_path: Optional[str] = None, **kw):
        """A handle for ``scene`` with the autotuned cell factor and knobs
        (measured on the given particles); the result dict is kept in .autotune."""
        params = dict(r_lr=scene.r_lr, r_hr=scene.r_hr, dt=scene.dt, g=tuple(scene.g),
                      domain_lo=tuple(scene.domain_lo), domain_hi=tuple(scene.domain_hi), walls=scene.walls,
                      c1=scene.c1, c2=scene.c2)
        res = autotune(params, lr_x, lr_v, hr_x, hr_v, lr_rigid=lr_rigid, cache_path=cache_path)
        up = cls.from_scene(scene, cell_factor=res["cell_factor"], **kw)
        up.set_tuning(**res["tuning"])
        up.autotune = res
        return up

    # -- plumbing
    def _check(self, rc: int) -> None:
        check(rc, self._h, self._L.upsample_last_error)

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.upsample_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def grid_info(self) -> dict:
        gi = GridInfo()
        self._check(self._L.upsample_get_grid_info(self._h, ctypes.byref(gi)))
        return gi.as_dict()

    # -- the path
    def build_grid(self, lr_x: torch.Tensor, lr_v: torch.Tensor, lr_rigid: Optional[torch.Tensor] = None):
        n = _soa(lr_x, "lr_x").shape[1]
        _soa(lr_v, "lr_v")
        _u8(lr_rigid, n, "lr_rigid")
        self._check(self._L.upsample_build_grid(self._h, _ptr(lr_x), _ptr(lr_v), _ptr(lr_rigid), n,
                                                _stream()))

    def advance(self, hr_x, hr_v, out_x=None, out_v=None):
        n = _soa(hr_x, "hr_x").shape[1]
        _soa(hr_v, "hr_v")
        out_x = torch.empty_like(hr_x) if out_x is None else _soa(out_x, "out_x")
        out_v = torch.empty_like(hr_v) if out_v is None else _soa(out_v, "out_v")
        self._check(self._L.upsample_advance(self._h, _ptr(hr_x), _ptr(hr_v), _ptr(out_x), _ptr(out_v),
                                             n, _stream()))
        return out_x, out_v

    def step(self, lr_x, lr_v, lr_rigid, hr_x, hr_v, out_x=None, out_v=None, tape=None):
        """One step; with ``tape`` ([6, N] float32, see upsample_step_taped)
        the forward sums are recorded for step_backward."""
        nl = _soa(lr_x, "lr_x").shape[1]
        _soa(lr_v, "lr_v")
        _u8(lr_rigid, nl, "lr_rigid")
        n = _soa(hr_x, "hr_x").shape[1]
        _soa(hr_v, "hr_v")
        out_x = torch.empty_like(hr_x) if out_x is None else _soa(out_x, "out_x")
        out_v = torch.empty_like(hr_v) if out_v is None else _soa(out_v, "out_v")
        if tape is None:
            self._check(self._L.upsample_step(self._h, _ptr(lr_x), _ptr(lr_v), _ptr(lr_rigid), nl,
                                              _ptr(hr_x), _ptr(hr_v), _ptr(out_x), _ptr(out_v), n,
                                              _stream()))
        else:
            _tape(tape, n)
            self._check(self._L.upsample_step_taped(self._h, _ptr(lr_x), _ptr(lr_v), _ptr(lr_rigid), nl,
                                                    _ptr(hr_x), _ptr(hr_v), _ptr(out_x), _ptr(out_v), n,
                                                    _ptr(tape), _stream()))
        return out_x, out_v

    def grid_snapshot_bytes(self) -> int:
        """Bytes of one saved grid (upsample_grid_snapshot_bytes)."""
        b = ctypes.c_int64()
        self._check(self._L.upsample_grid_snapshot_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def grid_snapshot(self, out=None):
        """Copy the handle's current LR grid into ``out`` (a uint8 device
        tensor of grid_snapshot_bytes() bytes, 256-byte aligned; allocated when
        None) and return it: upsample_grid_snapshot."""
        nb = self.grid_snapshot_bytes()
        if out is None:
            out = torch.empty(nb, dtype=torch.uint8, device="cuda")
        _snapshot(out, nb)
        self._check(self._L.upsample_grid_snapshot(self._h, _ptr(out), _stream()))
        return out

    def step_backward(self, lr_x, lr_v, lr_rigid, hr_x, hr_v, gx_out, gv_out,
                      g_lr_x=None, g_lr_v=None, gx_in=None, gv_in=None, tape=None, grid=None):
        """Returns (gx_in, gv_in, g_lr_x, g_lr_v); LR gradients are ADDED into
        g_lr_x / g_lr_v when given (zeros otherwise).  ``tape``: the record of
        the taped forward step on the same inputs (skips the recomputation).
        ``grid`` (with ``tape``): a grid_snapshot() taken after that taped
        step (skips the grid rebuild)."""
        if grid is not None and tape is None:
            raise ValueError("grid needs tape: only the taped adjoint reads a saved grid")
        nl = _soa(lr_x, "lr_x").shape[1]
        _soa(lr_v, "lr_v")
        _u8(lr_rigid, nl, "lr_rigid")
        n = _soa(hr_x, "hr_x").shape[1]
        for t, nm in ((hr_v, "hr_v"), (gx_out, "gx_out"), (gv_out, "gv_out")):
            _soa(t, nm)
        g_lr_x = torch.zeros_like(lr_x) if g_lr_x is None else _soa(g_lr_x, "g_lr_x")
        g_lr_v = torch.zeros_like(lr_v) if g_lr_v is None else _soa(g_lr_v, "g_lr_v")
        gx_in = torch.empty_like(hr_x) if gx_in is None else _soa(gx_in, "gx_in")
        gv_in = torch.empty_like(hr_v) if gv_in is None else _soa(gv_in, "gv_in")
        if tape is None:
            self._check(self._L.upsample_step_backward(
                self._h, _ptr(lr_x), _ptr(lr_v), _ptr(lr_rigid), nl, _ptr(hr_x), _ptr(hr_v), n,
                _ptr(gx_out), _ptr(gv_out), _ptr(gx_in), _ptr(gv_in), _ptr(g_lr_x), _ptr(g_lr_v), _stream()))
        elif grid is not None:
            _tape(tape, n)
            _snapshot(grid, self.grid_snapshot_bytes())
            self._check(self._L.upsample_step_backward_taped_grid(
                self._h, _ptr(grid), _ptr(lr_rigid), nl, _ptr(hr_x), _ptr(hr_v), n, _ptr(tape),
                _ptr(gx_out), _ptr(gv_out), _ptr(gx_in), _ptr(gv_in), _ptr(g_lr_x), _ptr(g_lr_v), _stream()))
        else:
            _tape(tape, n)
            self._check(self._L.upsample_step_backward_taped(
                self._h, _ptr(lr_x), _ptr(lr_v), _ptr(lr_rigid), nl, _ptr(hr_x), _ptr(hr_v), n, _ptr(tape),
                _ptr(gx_out), _ptr(gv_out), _ptr(gx_in), _ptr(gv_in), _ptr(g_lr_x), _ptr(g_lr_v), _stream()))
        return gx_in, gv_in, g_lr_x, g_lr_v

    def run(self, lr_x, lr_v, hr_x, hr_v, sort_every: int = 0, lr_rigid=None, perm=None):
        """Advance hr_x / hr_v in place through frames lr_x, lr_v [T, 3, N_L]
        (upsample_run); ``perm`` (int32 [N], optional) is updated through the
        reorders made every ``sort_every`` steps."""
        if not (lr_x.is_cuda and lr_x.dtype == torch.float32 and lr_x.dim() == 3 and lr_x.shape[1] == 3
                and lr_x.is_contiguous() and lr_v.shape == lr_x.shape and lr_v.is_contiguous()
                and lr_v.dtype == torch.float32):
            raise ValueError("lr_x, lr_v must be contiguous float32 device tensors [T, 3, N_L]")
        T, nl = lr_x.shape[0], lr_x.shape[2]
        _u8(lr_rigid, nl, "lr_rigid")
        n = _soa(hr_x, "hr_x").shape[1]
        _soa(hr_v, "hr_v")
        if perm is not None and not (perm.dtype == torch.int32 and perm.shape == (n,) and perm.is_contiguous()):
            raise ValueError("perm must be a contiguous int32 tensor of length N")
        self._check(self._L.upsample_run(self._h, _ptr(lr_x), _ptr(lr_v), _ptr(lr_rigid), nl, T, _ptr(hr_x),
                                         _ptr(hr_v), n, int(sort_every), _ptr(perm), _stream()))
        return hr_x, hr_v

    def run_multirate(self, lr_x, lr_v, hr_x, hr_v, n_steps: int, dt_lr: float, t_lr0: float = 0.0,
                      t_hr0: float = 0.0, sort_every: int = 0, lr_rigid=None, perm=None):
        """Advance hr_x / hr_v in place by ``n_steps`` HR steps against LR
        frames lr_x, lr_v [T, 3, N_L] at times t_lr0 + k dt_lr
        (upsample_run_multirate)."""
        if not (lr_x.is_cuda and lr_x.dtype == torch.float32 and lr_x.dim() == 3 and lr_x.shape[1] == 3
                and lr_x.is_contiguous() and lr_v.shape == lr_x.shape and lr_v.is_contiguous()
                and lr_v.dtype == torch.float32):
            raise ValueError("lr_x, lr_v must be contiguous float32 device tensors [T, 3, N_L]")
        T, nl = lr_x.shape[0], lr_x.shape[2]
        _u8(lr_rigid, nl, "lr_rigid")
        n = _soa(hr_x, "hr_x").shape[1]
        _soa(hr_v, "hr_v")
        if perm is not None and not (perm.dtype == torch.int32 and perm.shape == (n,) and perm.is_contiguous()):
            raise ValueError("perm must be a contiguous int32 tensor of length N")
        self._check(self._L.upsample_run_multirate(self._h, _ptr(lr_x), _ptr(lr_v), _ptr(lr_rigid), nl, T,
                                                   float(t_lr0), float(dt_lr), float(t_hr0), int(n_steps),
                                                   _ptr(hr_x), _ptr(hr_v), n, int(sort_every), _ptr(perm),
                                                   _stream()))
        return hr_x, hr_v

    def sort_hr(self, hr_x, hr_v, with_perm: bool = True, out_x=None, out_v=None):
        """Reorders the HR state by the sub-cell key of the handle's tuning
        (Hilbert by default; upsample_sort_hr): in place by
        default, or into out_x / out_v.  Returns the old index of each new
        position (int32) or None."""
        n = _soa(hr_x, "hr_x").shape[1]
        _soa(hr_v, "hr_v")
        ox = hr_x if out_x is None else _soa(out_x, "out_x")
        ov = hr_v if out_v is None else _soa(out_v, "out_v")
        perm = torch.empty(n, dtype=torch.int32, device=hr_x.device) if with_perm else None
        self._check(self._L.upsample_sort_hr(self._h, _ptr(hr_x), _ptr(hr_v), _ptr(ox), _ptr(ov), n,
                                             _ptr(perm), _stream()))
        return perm

    def permute(self, a, perm, b=None, scatter: bool = False, out_a=None, out_b=None):
        """Gather (a[:, perm]) or scatter (out[:, perm] = a) the columns of
        [3, N] arrays a and, if given, b; returns (out_a, out_b)."""
        n = _soa(a, "a").shape[1]
        if b is not None:
            _soa(b, "b")
        if perm.dtype != torch.int32 or perm.shape != (n,) or not perm.is_contiguous():
            raise ValueError("perm must be a contiguous int32 tensor of length N")
        oa = torch.empty_like(a) if out_a is None else _soa(out_a, "out_a")
        ob = None if b is None else (torch.empty_like(b) if out_b is None else _soa(out_b, "out_b"))
        self._check(self._L.upsample_permute(self._h, _ptr(a), _ptr(b), _ptr(oa), _ptr(ob), n, _ptr(perm),
                                             1 if scatter else 0, _stream()))
        return oa, ob

    # -- debug exports
    def debug_grid(self, n_lr: int, device="cuda"):
        info = self.grid_info()
        keys = torch.empty(n_lr, dtype=torch.int32, device=device)
        perm = torch.empty(n_lr, dtype=torch.int32, device=device)
        cs = torch.empty(info["n_cells"] + 1, dtype=torch.int32, device=device)
        self._check(self._L.upsample_debug_grid(self._h, _ptr(keys), _ptr(perm), _ptr(cs), _stream()))
        return keys, perm, cs

    def debug_lr_sorted(self, n_lr: int, device="cuda"):
        """The last build's LR positions and velocities in sorted order [3, N_L]."""
        x = torch.empty((3, n_lr), dtype=torch.float32, device=device)
        v = torch.empty((3, n_lr), dtype=torch.float32, device=device)
        self._check(self._L.upsample_debug_lr_sorted(self._h, _ptr(x), _ptr(v), _stream()))
        return x, v

    def debug_neighbors(self, hr_x, hr_v, max_k: int = 64):
        n = _soa(hr_x, "hr_x").shape[1]
        _soa(hr_v, "hr_v")
        count = torch.empty(n, dtype=torch.int32, device=hr_x.device)
        ids = torch.full((n, max_k), -1, dtype=torch.int32, device=hr_x.device)
        branch = torch.empty(n, dtype=torch.uint8, device=hr_x.device)
        self._check(self._L.upsample_debug_neighbors(self._h, _ptr(hr_x), _ptr(hr_v), n, _ptr(count),
                                                     _ptr(ids), max_k, _ptr(branch), _stream()))
        return count, ids, branch

    def debug_step_members(self, hr_x, hr_v, max_k: int = 64, out_x=None, out_v=None):
        """The step kernel's own instance with member exports
        (upsample_debug_step_members): returns (out_x, out_v, count, ids,
        count_w, w_disagree)."""
        n = _soa(hr_x, "hr_x").shape[1]
        _soa(hr_v, "hr_v")
        out_x = torch.empty_like(hr_x) if out_x is None else _soa(out_x, "out_x")
        out_v = torch.empty_like(hr_v) if out_v is None else _soa(out_v, "out_v")
        dev = hr_x.device
        count = torch.empty(n, dtype=torch.int32, device=dev)
        ids = torch.full((n, max_k), -1, dtype=torch.int32, device=dev) if max_k > 0 else None
        count_w = torch.empty(n, dtype=torch.int32, device=dev)
        wdis = torch.empty(n, dtype=torch.float32, device=dev)
        self._check(self._L.upsample_debug_step_members(self._h, _ptr(hr_x), _ptr(hr_v), _ptr(out_x), _ptr(out_v),
                                                        n, _ptr(count), _ptr(ids), max(max_k, 0), _ptr(count_w),
                                                        _ptr(wdis), _stream()))
        return out_x, out_v, count, ids, count_w, wdis

    # -- launch-shape knobs
    TUNING_KEYS = ("gather_groups", "sort_sub", "adjoint_tiled", "sort_mode", "tile_max", "adjoint_tile_max",
                   "wall_cull")

    def set_tuning(self, **kw) -> None:
        """Set launch-shape knobs (upsample_tuning); unnamed knobs keep their value."""
        t = _lib.Tuning()
        self._check(self._L.upsample_get_tuning(self._h, ctypes.byref(t)))
        for k, v in kw.items():
            if k not in self.TUNING_KEYS:
                raise KeyError(k)
            if v is not None:
                setattr(t, k, int(v))
        self._check(self._L.upsample_set_tuning(self._h, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = _lib.Tuning()
        self._check(self._L.upsample_get_tuning(self._h, ctypes.byref(t)))
        return {k: int(getattr(t, k)) for k in self.TUNING_KEYS}

    # -- kernel timing probe
    def timing_enable(self, enable: bool = True) -> None:
        self._check(self._L.upsample_timing_enable(self._h, 1 if enable else 0))

    def timing_read(self):
        ms = ctypes.c_double()
        k = ctypes.c_int64()
        self._check(self._L.upsample_timing_read(self._h, ctypes.byref(ms), ctypes.byref(k)))
        return float(ms.value), int(k.value)
