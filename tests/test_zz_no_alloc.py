"""The allocation-free contraction (sttsv_contract_noalloc) against the
allocating one (sttsv_contract) through the C ABI: same value and same
B x^(r-1) bit for bit, on two calls in a row, the second on a smaller
hypergraph (the static scratch keeps the first call's contents), and the
value against the oracle at 1e-12."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import sshopm_ref
from paper_2311_08595_amd import _lib
from paper_2311_08595_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _mixed(seed, n, m, r, kmin, kmax):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(kmin, kmax + 1, size=m)
    eptr, eidx = wl.uniform_members(rng, n, sizes)
    return eptr, eidx, wl.uniform_x(rng, n)


def _call(lib, fn, h, x, y):
    out = ctypes.c_double()
    rc = getattr(lib, fn)(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), ctypes.byref(out))
    assert rc == _lib.STTSV_OK, (fn, rc)
    return out.value


def test_noalloc_contraction_matches_allocating_one():
    import torch
    assert torch.cuda.is_available()
    lib = _lib.load()
    for seed, n, m, r in [(71, 3000, 12001, 12), (72, 700, 2003, 7)]:     # second call: smaller input
        print(f"[noalloc] n={n} m={m} r={r}", flush=True)
        eptr, eidx, x = _mixed(seed, n, m, r, 1, r)
        eptr = np.ascontiguousarray(eptr, dtype=np.int64)
        eidx = np.ascontiguousarray(eidx, dtype=np.int32)
        h = ctypes.c_void_p()
        assert lib.sttsv_plan(eptr.ctypes.data, eidx.ctypes.data, m, n, r, None, ctypes.byref(h)) == 0
        try:
            xd = torch.tensor(x, dtype=torch.float64, device="cuda")
            ya = torch.empty_like(xd)
            yb = torch.empty_like(xd)
            a = _call(lib, "sttsv_contract", h, xd, ya)
            b = _call(lib, "sttsv_contract_noalloc", h, xd, yb)
            c = _call(lib, "sttsv_contract_noalloc", h, xd, yb)      # again: the scratch holds the last call's values
            torch.cuda.synchronize()
            assert a == b == c
            assert ya.cpu().numpy().tobytes() == yb.cpu().numpy().tobytes()
            ref = sshopm_ref.contract(eptr, eidx, n, r, x)
            assert abs(b - ref) <= 1e-12 * abs(ref)
        finally:
            lib.sttsv_plan_destroy(h)


def test_noalloc_contraction_rejects_bad_arguments():
    lib = _lib.load()
    out = ctypes.c_double()
    assert lib.sttsv_contract_noalloc(None, None, None, ctypes.byref(out)) == _lib.STTSV_EINVAL
