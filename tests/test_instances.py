"""Host-side instance helpers: renumbering the products gives the same LP, so
the oracle's best response moves with the products and nothing else changes."""
import numpy as np
import pytest

import oracle
from paper_2602_22421_amd.instances import make_instance, shuffle_products


@pytest.mark.parametrize("m", [None, 7])
def test_shuffle_products_same_problem(m):
    inst = make_instance(300, 40, m=m, size_lo=1, size_hi=12, zipf=1.1, seed=5)
    sh, pi = shuffle_products(inst, seed=9)
    assert sorted(pi.tolist()) == list(range(inst.n))
    assert np.array_equal(sh.seg_ptr, inst.seg_ptr) and sh.nnz == inst.nnz
    for l in range(inst.L):
        a, b = inst.seg_ptr[l], inst.seg_ptr[l + 1]
        row = sh.idx[a:b]
        assert np.all(np.diff(row) > 0)                       # rows stay sorted
        assert sorted(row.tolist()) == sorted(pi[inst.idx[a:b]].tolist())
    rng = np.random.default_rng(2)
    eta = rng.uniform(0, 1, inst.m) * 0.4 * (inst.r.mean() if m else inst.r)
    eta_sh = eta.copy()
    if m is None:
        eta_sh[pi] = eta
    x = oracle.best_response(inst, eta)
    y = oracle.best_response(sh, eta_sh)
    np.testing.assert_allclose(y["rho"][pi], x["rho"], rtol=1e-15, atol=0)
    np.testing.assert_allclose(y["S"][pi], x["S"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(y["seg_R"], x["seg_R"], rtol=1e-12, atol=1e-15)
    u_x = x["u"]
    u_y = y["u"][pi] if m is None else y["u"]
    np.testing.assert_allclose(u_y, u_x, rtol=1e-12, atol=1e-15)
    assert y["D"] == pytest.approx(x["D"], rel=1e-13)
