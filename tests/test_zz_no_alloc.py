"""lbm_reduce_noalloc (the reduction with its scratch in a static device
array) against lbm_reduce, through the C ABI: two calls in a row, the second
on a smaller lattice; the static array keeps the last call's contents, so the
second call must not see the first one's."""
import ctypes as C

import numpy as np
import pytest

from paper_2203_01316_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available()
    from paper_2203_01316_amd import lbm
    return lbm


def _raw(L, g, fn, group, cols, nout=None):
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    out = np.full(nout or 3 + len(cols), np.nan)
    st = getattr(L._lib, fn)(g.ctx, int(group), cols.ctypes.data if len(cols) else None, len(cols),
                             out.ctypes.data, len(out))
    return st, out


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_reduce_noalloc_matches_reduce(L, storage):
    cases = [(192, 96, 9.5, [5, 40, 150, 190]), (40, 24, 4.5, [3, 30])]
    for nx, ny, r, cols in cases:
        flags, q, groups, u, rho0, H0 = W.heated_cylinder(nx, ny, r, u_in=0.04, amp=1e-3, seed=0)
        g = L.LBM(9, nx, ny, with_ns=True, storage=storage, nu=0.04, k=0.06, flags=flags, q=q, groups=groups)
        g.set_velocity(np.asarray(u, np.float32).astype(np.float64))
        g.init(H0, u=u, rho=rho0)
        g.step(37)
        st_a, ref = _raw(L, g, "lbm_reduce", 1, cols)
        st_b, got = _raw(L, g, "lbm_reduce_noalloc", 1, cols)
        assert st_a == L.OK and st_b == L.OK
        print(nx, ny, storage, ref, got)
        np.testing.assert_array_equal(got, ref)
        assert np.all(np.isfinite(got)) and got[0] > 0
        del g


def test_reduce_noalloc_rejects_too_many_columns(L):
    g = L.LBM(9, 80, 8, k=0.01)
    g.init(np.ones(640))
    st, _ = _raw(L, g, "lbm_reduce_noalloc", 0, list(range(65)))
    assert st == L.EINVAL
    assert b"64" in L._lib.lbm_last_error(g.ctx)
    st, out = _raw(L, g, "lbm_reduce_noalloc", 0, list(range(64)))
    assert st == L.OK
    st2, ref = _raw(L, g, "lbm_reduce", 0, list(range(64)))
    np.testing.assert_array_equal(out, ref)
