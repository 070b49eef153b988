"""Host-side argument checks of upsample_step_noalloc (no GPU needed): bad
parameters, the capacity limits of its fixed scratch and the VALIDATE flag
are rejected before any device call."""
import ctypes

from paper_2308_01629_amd import _lib
from paper_2308_01629_amd.upsampler import make_params


def _call(p, n_lr, n_hr):
    dummy = ctypes.c_void_p(16)  # never dereferenced: the call is rejected first
    return _lib.lib().upsample_step_noalloc(ctypes.byref(p), dummy, dummy, None, n_lr, dummy, dummy, dummy,
                                            dummy, n_hr, None)


def _p(**over):
    kw = dict(r_lr=0.02, r_hr=0.005, dt=1 / 60, g=(0, -9.81, 0), domain_lo=(0, 0, 0), domain_hi=(1, 1, 1))
    kw.update(over)
    return make_params(**kw)


def test_noalloc_rejects_before_device():
    E = _lib.ERR_CODES
    p, _w = _p(r_lr=0.0)
    assert _call(p, 10, 10) == E["UPSAMPLE_ERR_INVALID_ARG"]
    p, _w = _p()
    assert _call(p, _lib.NOALLOC_MAX_LR + 1, 10) == E["UPSAMPLE_ERR_CAPACITY"]
    assert _call(p, -1, 10) == E["UPSAMPLE_ERR_INVALID_ARG"]
    p, _w = _p(domain_hi=(10, 10, 10))  # 56^3 cells at r = 0.02
    assert _call(p, 10, 10) == E["UPSAMPLE_ERR_CAPACITY"]
    p, _w = _p(validate=True)
    assert _call(p, 10, 10) == E["UPSAMPLE_ERR_INVALID_ARG"]
    assert _lib.lib().upsample_step_noalloc(None, None, None, None, 0, None, None, None, None, 0, None) == \
        E["UPSAMPLE_ERR_INVALID_ARG"]
