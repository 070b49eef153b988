"""Host-side argument checks of upsample_sample_volume (no GPU needed)."""
import ctypes

from paper_2308_01629_amd import _lib


def _call(r, lo, hi, n_cand=10, max_out=10):
    n = ctypes.c_int64(-1)
    lo_c = (ctypes.c_float * 3)(*lo)
    hi_c = (ctypes.c_float * 3)(*hi)
    dummy = ctypes.c_void_p(16)  # never dereferenced: the call is rejected first
    rc = _lib.lib().upsample_sample_volume(dummy, n_cand, r, lo_c, hi_c, dummy, max_out, ctypes.byref(n), None)
    return rc, n.value


def test_sampling_rejects_before_device():
    E = _lib.ERR_CODES
    assert _call(0.0, (0, 0, 0), (1, 1, 1))[0] == E["UPSAMPLE_ERR_INVALID_ARG"]
    assert _call(float("nan"), (0, 0, 0), (1, 1, 1))[0] == E["UPSAMPLE_ERR_INVALID_ARG"]
    assert _call(0.01, (0, 1, 0), (1, 1, 1))[0] == E["UPSAMPLE_ERR_INVALID_ARG"]
    assert _call(1e-6, (0, 0, 0), (10, 10, 10))[0] == E["UPSAMPLE_ERR_GRID_TOO_LARGE"]
    assert _call(0.01, (0, 0, 0), (1, 1, 1), n_cand=-1)[0] == E["UPSAMPLE_ERR_INVALID_ARG"]
    rc, n = _call(0.01, (0, 0, 0), (1, 1, 1))
    assert n == 0 or rc != 0
