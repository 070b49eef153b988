"""The C ABI on the host (no GPU): the library loads, exports every symbol the
header declares, validates arguments before touching a device, and computes
the grid exactly as the oracle defines it."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import upsample_oracle as O
from paper_2308_01629_amd import _lib
from paper_2308_01629_amd.upsampler import grid_info_for, make_params
from workloads import configs

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "upsample.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(upsample_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = _declared()
    assert "upsample_step" in names and "upsample_step_backward" in names and "upsample_init" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding describes every declared function
    assert set(names) <= set(_lib.SIGNATURES), set(names) - set(_lib.SIGNATURES)


def _params(**over):
    kw = dict(r_lr=0.02, r_hr=0.005, dt=1 / 60, g=(0, -9.81, 0), domain_lo=(0, 0, 0),
              domain_hi=(1, 1, 1), max_lr=16, max_hr=16)
    kw.update(over)
    return make_params(**kw)


def _init(p):
    h = ctypes.c_void_p()
    rc = _lib.lib().upsample_init(ctypes.byref(p), ctypes.byref(h))
    return rc, h


def _no_gpu():
    try:
        import torch
        return not torch.cuda.is_available()
    except Exception:
        return True


@pytest.mark.parametrize("field,value,code", [
    ("r_lr", 0.0, "INVALID_ARG"), ("r_lr", float("nan"), "INVALID_ARG"), ("r_hr", -1.0, "INVALID_ARG"),
    ("dt", float("inf"), "INVALID_ARG"), ("cell_factor", -1.0, "INVALID_ARG"),
    ("cell_factor", 1e-4, "GRID_TOO_LARGE"), ("max_lr", -1, "INVALID_ARG"),
])
def test_invalid_params_rejected_before_device(field, value, code):
    p, _w = _params()
    setattr(p, field, value)
    rc, _ = _init(p)
    assert rc == _lib.ERR_CODES["UPSAMPLE_ERR_" + code]
    gi = _lib.GridInfo()
    assert _lib.lib().upsample_grid_info_for(ctypes.byref(p), ctypes.byref(gi)) == rc


def test_bad_domain_walls_and_grid_size():
    L = _lib.lib()
    p, _w = _params(domain_lo=(0, 1, 0), domain_hi=(1, 1, 1))
    assert _init(p)[0] == _lib.ERR_CODES["UPSAMPLE_ERR_INVALID_ARG"]
    p, _w = _params(r_lr=1e-4, domain_hi=(100, 100, 100))
    assert _init(p)[0] == _lib.ERR_CODES["UPSAMPLE_ERR_GRID_TOO_LARGE"]
    bad = np.zeros((1, 12), np.float32)
    bad[0, :3] = (0, 2, 0)     # not a unit normal
    p, _w = _params(walls=bad)
    assert _init(p)[0] == _lib.ERR_CODES["UPSAMPLE_ERR_INVALID_ARG"]
    p, _w = _params(walls=np.zeros((33, 12), np.float32))
    assert _init(p)[0] == _lib.ERR_CODES["UPSAMPLE_ERR_INVALID_ARG"]
    p, _w = _params(cell_factor=0.01, domain_hi=(0.1, 0.1, 0.1))   # stencil reach 100 > 64
    assert _init(p)[0] == _lib.ERR_CODES["UPSAMPLE_ERR_INVALID_ARG"]
    p, _w = _params()
    p.flags = 0x80
    assert _init(p)[0] == _lib.ERR_CODES["UPSAMPLE_ERR_INVALID_ARG"]
    assert L.upsample_init(None, None) == _lib.ERR_CODES["UPSAMPLE_ERR_INVALID_ARG"]


def test_null_handle_calls_rejected():
    L = _lib.lib()
    inv = _lib.ERR_CODES["UPSAMPLE_ERR_INVALID_ARG"]
    assert L.upsample_step(None, None, None, None, 0, None, None, None, None, 0, None) == inv
    assert L.upsample_build_grid(None, None, None, None, 0, None) == inv
    assert L.upsample_advance(None, None, None, None, None, 0, None) == inv
    assert L.upsample_step_backward(None, None, None, None, 0, None, None, 0, None, None, None, None,
                                    None, None, None) == inv
    assert L.upsample_sort_hr(None, None, None, None, None, 0, None, None) == inv
    assert L.upsample_step_taped(None, None, None, None, 0, None, None, None, None, 0, None, None) == inv
    assert L.upsample_step_backward_taped(None, None, None, None, 0, None, None, 0, None, None, None, None,
                                          None, None, None, None) == inv
    assert L.upsample_grid_snapshot_bytes(None, None) == inv
    assert L.upsample_grid_snapshot(None, None, None) == inv
    assert L.upsample_step_backward_taped_grid(None, None, None, 0, None, None, 0, None, None, None, None, None,
                                               None, None, None) == inv
    assert L.upsample_permute(None, None, None, None, None, 0, None, 0, None) == inv
    assert L.upsample_run(None, None, None, None, 0, 1, None, None, 0, 0, None, None) == inv
    assert L.upsample_autotune(None, None, None, None, 0, 1, None, None, 0, None, None, None) == inv
    assert L.upsample_destroy(None) == 0
    assert L.upsample_strerror(2).decode().startswith("particle count")


def _scene(p, lr_off, n_lr, hr_off, n_hr):
    d = _lib.SceneDesc()
    d.params = p
    d.lr_offset, d.n_lr, d.hr_offset, d.n_hr = lr_off, n_lr, hr_off, n_hr
    return d


def test_batch_table_validated_before_device():
    L = _lib.lib()
    inv = _lib.ERR_CODES["UPSAMPLE_ERR_INVALID_ARG"]
    b = ctypes.c_void_p()
    p, _w = _params()
    bad, _w2 = _params(r_lr=0.0)

    def init(scenes, flags=0):
        arr = (_lib.SceneDesc * len(scenes))(*scenes)
        return L.upsample_batch_init(arr, len(scenes), flags, ctypes.byref(b))

    assert L.upsample_batch_init(None, 1, 0, ctypes.byref(b)) == inv
    assert init([_scene(p, 0, 10, 0, 10)], flags=0x10) == inv
    assert init([_scene(p, 0, 10, 0, 10), _scene(p, 5, 10, 10, 10)]) == inv      # LR ranges overlap
    assert init([_scene(p, 0, 10, 0, 10), _scene(p, 10, 10, 9, 10)]) == inv      # HR ranges overlap
    assert init([_scene(p, -1, 10, 0, 10)]) == inv
    assert init([_scene(p, 0, 10, 0, 10), _scene(bad, 10, 10, 10, 10)]) == inv   # bad scene params
    small, _w3 = _params(r_lr=1e-4, domain_hi=(100, 100, 100))
    assert init([_scene(small, 0, 10, 0, 10)]) == _lib.ERR_CODES["UPSAMPLE_ERR_GRID_TOO_LARGE"]
    arr = (_lib.SceneDesc * 1)(_scene(p, 0, 10, 0, 10))
    assert L.upsample_batch_init(arr, 0, 0, ctypes.byref(b)) == inv
    assert L.upsample_batch_init(arr, 1, 0, None) == inv
    if _no_gpu():
        # unordered but disjoint ranges and empty scenes are a valid table
        ok = [_scene(p, 20, 10, 30, 10), _scene(p, 0, 20, 0, 30), _scene(p, 0, 0, 0, 0)]
        assert init(ok) == _lib.ERR_CODES["UPSAMPLE_ERR_NO_DEVICE"]
    assert L.upsample_batch_step(None, None, None, None, None, None, None, None, None) == inv
    assert L.upsample_batch_info(None, None) == inv
    assert L.upsample_batch_sort_hr(None, None, None, None, None) == inv
    assert L.upsample_batch_destroy(None) == 0
    assert L.upsample_batch_last_error(None).decode() == "null batch"


@pytest.mark.skipif(not _no_gpu(), reason="host without a GPU only")
def test_valid_init_without_device_reports_no_device():
    p, _w = _params()
    assert _init(p)[0] == _lib.ERR_CODES["UPSAMPLE_ERR_NO_DEVICE"]


@pytest.mark.parametrize("name", ["plain", "column", "drain", "diff"])
@pytest.mark.parametrize("cell_factor", [0.0, 1.0, 0.5, 1.7])
def test_host_grid_matches_oracle_definition(name, cell_factor):
    g, nl, nh, r, _ = configs.WORKLOADS[name]
    lo, hi = {"plain": ((0, 0, 0), (1, 1, 1)), "column": ((0, 0, 0), (2, 1.5, 2)),
              "drain": ((0, 0, 0), (1, 2.4, 1)), "diff": ((0, 0, 0), (1, 1, 1))}[name]
    gi = grid_info_for(r_lr=r, r_hr=r / 4, dt=1 / 60, g=(0, -9.81, 0), domain_lo=lo, domain_hi=hi,
                       cell_factor=cell_factor)
    spec = O.grid_spec(r, lo, hi, cell_factor)
    assert gi["dims"] == spec.dims
    assert gi["reach"] == spec.reach
    assert gi["cell_size"] == spec.cs
    assert np.float32(gi["inv_cell_size"]) == spec.inv_cs
    assert np.float32(gi["h2"]) == spec.h2_f


@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_hilbert_reference_is_a_face_neighbour_walk(bits):
    """The reorder test's Hilbert key: a bijection of the 2^bits cube onto
    [0, 8^bits) that steps to a face neighbour at every increment, starting at
    the origin."""
    from gpu_util import hilbert_index
    n = 1 << bits
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")).reshape(3, -1)
    k = hilbert_index(g, bits)
    assert np.array_equal(np.sort(k), np.arange(n ** 3))
    walk = g[:, np.argsort(k)]
    assert np.all(np.abs(np.diff(walk, axis=1)).sum(axis=0) == 1)
    assert np.all(walk[:, 0] == 0)

