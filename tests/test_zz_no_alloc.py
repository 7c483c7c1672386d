"""cl_step_noalloc (the allocation-free variant of cl_step, whose scratch
lives in a fixed device array of the library) against cl_step on identical
lattices, through the C ABI: two calls in a row, the second on a smaller
lattice, so that what the first call left in the shared array cannot leak
into the second.  Bars: FP64 within 1e-11 relative per step and norm-wise on
the fields; FP32 fields within 1e-4 relative on volume averages."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import make_lattice, oracle_seed

pytestmark = pytest.mark.gpu

KEYS = ["eta", "a", "H", "EK", "EG", "EV", "mean", "var", "r"]


def _pair(w, amp):
    s0 = oracle_seed(w, amp=amp)
    lats = []
    for _ in range(2):
        lat = make_lattice(w)
        lat.set_fields(s0.f, s0.p)
        lats.append(lat)
    return lats


def _compare(ra, rb, fa, fb, tol, fields_tol):
    for k in KEYS:
        a = np.asarray(ra[k], float)
        b = np.asarray(rb[k], float)
        scale = np.maximum(np.abs(a), 1e-300)
        if k in ("EK", "EV", "mean", "r"):
            # quantities that pass through zero: relative to their own range
            scale = np.maximum(np.max(np.abs(a)), 1e-300)
        err = np.max(np.abs(a - b) / scale)
        assert err <= tol, (k, err)
    for x, y in zip(fa, fb):
        assert np.max(np.abs(x - y)) <= fields_tol * np.max(np.abs(x))


def test_noalloc_matches_cl_step_two_calls_second_smaller():
    # first call: 64^3 two fields, FP64, self-consistent expansion, VV4, 30 steps
    w1 = W.C1.with_(N=64, k_ir=1.0, precision="fp64")
    ref, na = _pair(w1, amp=20.0)
    r_ref = ref.step("vv4", w1.dt, 30)
    print("case: 64^3 2-field fp64 vv4 30 steps", flush=True)
    r_na = na.step_noalloc("vv4", w1.dt, 30)
    _compare(r_ref, r_na, ref.get_fields(), na.get_fields(), 1e-11, 1e-11)
    # second call: a 16^3 single-field FP32 lattice (fewer workgroups, fewer steps)
    w2 = W.C0.with_(N=16, precision="fp32")
    ref2, na2 = _pair(w2, amp=10.0)
    r_ref2 = ref2.step("leapfrog", w2.dt, 7)
    print("case: 16^3 1-field fp32 leapfrog 7 steps", flush=True)
    r_na2 = na2.step_noalloc("leapfrog", w2.dt, 7)
    _compare(r_ref2, r_na2, ref2.get_fields(), na2.get_fields(), 1e-4, 1e-4)
    # and the first lattice continues from where it was, through either entry point
    r_ref = ref.step("leapfrog", w1.dt, 5)
    r_na = na.step_noalloc("leapfrog", w1.dt, 5)
    _compare(r_ref, r_na, ref.get_fields(), na.get_fields(), 1e-11, 1e-11)
    for x in (ref, na, ref2, na2):
        x.close()


def test_noalloc_limits():
    from paper_2607_24978_amd import _lib as lib
    w = W.C0.with_(N=16)
    lat = make_lattice(w)
    s0 = oracle_seed(w)
    lat.set_fields(s0.f, s0.p)
    with pytest.raises(lib.CLError) as e:
        lat.step_noalloc("leapfrog", w.dt, 4097)
    assert e.value.status == lib.CL_EINVAL
    with pytest.raises(lib.CLError) as e:
        lat.step_noalloc("rk4", w.dt, 2)
    assert e.value.status == lib.CL_EUNSUPPORTED
    assert lat.step_noalloc("leapfrog", w.dt, 0).size == 0
    lat.close()
