"""PyTorch-facing wrapper of the batched entry points (upsample_batch_*).

Scenes are laid out one after another: scene s occupies LR columns
``lr_offsets[s] .. lr_offsets[s] + n_lr[s] - 1`` of [3, total_lr] tensors and
HR columns ``hr_offsets[s] ..`` of [3, total_hr] tensors.  Argument
marshalling only; every step runs in libupsample.so.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import SceneDesc, check, lib
from .upsampler import _ptr, _soa, _stream, _u8, make_params


class Batch:
    """A fixed set of scenes stepped together in one graph-captured launch
    sequence (``eager=True``: direct launches)."""

    def __init__(self, params: Sequence[dict], n_lr: Sequence[int], n_hr: Sequence[int], eager: bool = False,
                 hr_offsets: Optional[Sequence[int]] = None):
        """``hr_offsets``: first HR column of each scene (default: the scenes
        one after another, in order)."""
        if not (len(params) == len(n_lr) == len(n_hr)) or not params:
            raise ValueError("params, n_lr and n_hr must have the same non-zero length")
        self._L = lib()
        self.n_lr = [int(v) for v in n_lr]
        self.n_hr = [int(v) for v in n_hr]
        self.lr_offsets = [int(v) for v in np.concatenate([[0], np.cumsum(self.n_lr)[:-1]])]
        if hr_offsets is None:
            hr_offsets = np.concatenate([[0], np.cumsum(self.n_hr)[:-1]])
        self.hr_offsets = [int(v) for v in hr_offsets]
        self.total_lr = int(sum(self.n_lr))
        self.total_hr = int(max(o + n for o, n in zip(self.hr_offsets, self.n_hr)))
        descs = (SceneDesc * len(params))()
        keep = []
        for s, kw in enumerate(params):
            p, wbuf = make_params(**kw)
            keep.append(wbuf)
            descs[s].params = p
            descs[s].lr_offset, descs[s].n_lr = self.lr_offsets[s], self.n_lr[s]
            descs[s].hr_offset, descs[s].n_hr = self.hr_offsets[s], self.n_hr[s]
        b = ctypes.c_void_p()
        check(self._L.upsample_batch_init(descs, len(params), _lib.BATCH_EAGER if eager else 0, ctypes.byref(b)))
        self._b = b
        del keep

    @classmethod
    def from_scenes(cls, scenes, cell_factor=0.0, eager: bool = False, hr_offsets=None) -> "Batch":
        """``cell_factor``: one kappa for every scene or one per scene."""
        kap = list(cell_factor) if np.ndim(cell_factor) else [float(cell_factor)] * len(scenes)
        params = [dict(r_lr=sc.r_lr, r_hr=sc.r_hr, dt=sc.dt, g=tuple(sc.g), domain_lo=tuple(sc.domain_lo),
                       domain_hi=tuple(sc.domain_hi), walls=sc.walls, c1=sc.c1, c2=sc.c2,
                       cell_factor=k) for sc, k in zip(scenes, kap)]
        return cls(params, [sc.n_lr for sc in scenes], [sc.n_hr for sc in scenes], eager=eager,
                   hr_offsets=hr_offsets)

    def _check(self, rc: int) -> None:
        check(rc, self._b, self._L.upsample_batch_last_error)

    def close(self) -> None:
        if getattr(self, "_b", None) is not None and self._b.value:
            self._L.upsample_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- layout helpers (host side)
    def pack_lr(self, arrays: Sequence[np.ndarray]) -> np.ndarray:
        """Concatenate per-scene [3, n_lr[s]] arrays into the batch layout."""
        return np.ascontiguousarray(np.concatenate([np.asarray(a, np.float32) for a in arrays], axis=1))

    def pack_hr(self, arrays: Sequence[np.ndarray]) -> np.ndarray:
        """Per-scene [3, n_hr[s]] arrays placed at their columns (gaps zero)."""
        out = np.zeros((3, self.total_hr), np.float32)
        for a, o, n in zip(arrays, self.hr_offsets, self.n_hr):
            out[:, o:o + n] = np.asarray(a, np.float32)
        return out

    def split_hr(self, t) -> List:
        """Per-scene column views of a [3, total_hr] array or tensor."""
        return [t[:, o:o + n] for o, n in zip(self.hr_offsets, self.n_hr)]

    # -- the step
    def step(self, lr_x, lr_v, hr_x, hr_v, lr_rigid: Optional[torch.Tensor] = None, out_x=None, out_v=None):
        """Advance every scene one step; returns (x', v') ([3, total_hr]).
        out_x / out_v may be hr_x / hr_v (in place)."""
        if _soa(lr_x, "lr_x").shape[1] != self.total_lr or _soa(lr_v, "lr_v").shape[1] != self.total_lr:
            raise ValueError(f"LR arrays must be [3, {self.total_lr}]")
        if _soa(hr_x, "hr_x").shape[1] != self.total_hr or _soa(hr_v, "hr_v").shape[1] != self.total_hr:
            raise ValueError(f"HR arrays must be [3, {self.total_hr}]")
        _u8(lr_rigid, self.total_lr, "lr_rigid")
        ox = torch.empty_like(hr_x) if out_x is None else _soa(out_x, "out_x")
        ov = torch.empty_like(hr_v) if out_v is None else _soa(out_v, "out_v")
        self._check(self._L.upsample_batch_step(self._b, _ptr(lr_x), _ptr(lr_v), _ptr(lr_rigid), _ptr(hr_x),
                                                _ptr(hr_v), _ptr(ox), _ptr(ov), _stream()))
        return ox, ov

    def sort_hr(self, hr_x, hr_v, with_perm: bool = True):
        """Reorders every scene's HR columns in place (upsample_batch_sort_hr);
        returns the old column of each new column (int32 [total_hr]) or None."""
        if _soa(hr_x, "hr_x").shape[1] != self.total_hr or _soa(hr_v, "hr_v").shape[1] != self.total_hr:
            raise ValueError(f"HR arrays must be [3, {self.total_hr}]")
        perm = torch.empty(self.total_hr, dtype=torch.int32, device=hr_x.device) if with_perm else None
        self._check(self._L.upsample_batch_sort_hr(self._b, _ptr(hr_x), _ptr(hr_v), _ptr(perm), _stream()))
        return perm

    def info(self) -> dict:
        out = (ctypes.c_int64 * 5)()
        self._check(self._L.upsample_batch_info(self._b, out))
        return {"total_lr": out[0], "total_hr": out[1], "tiles": out[2], "grid_blocks": out[3],
                "graphs_captured": out[4]}
