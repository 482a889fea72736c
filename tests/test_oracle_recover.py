"""Pins of the oracle's SBLP -> CBLP recovery (Section 4.4, the recovery
lemma, in its GAM form) (CPU only).

* the recovered nested assortments reproduce the given sales through the
  GAM choice probabilities (the plain definition of the sales a CBLP
  solution makes), and their probabilities are a distribution;
* a single best response is recovered as that one assortment offered all
  the time;
* the HiGHS optimum of the SBLP, recovered, is feasible for the enumerated
  CBLP and attains its optimum (CBLP = SBLP);
* the sets are nested (prefix-closed, the paper's three-product example).
"""
import numpy as np
import pytest

import oracle
import oracle.lp as lp
from paper_2602_22421_amd.instances import make_instance


def _sales_of(inst, rank, alpha):
    """Sales y_lj = lambda_l sum_q alpha(S_q) pi_lj(S_q) over the nested sets,
    with the GAM probabilities written out from their definition."""
    y = np.zeros(inst.nnz)
    for l in range(inst.L):
        b, e = inst.seg_ptr[l], inst.seg_ptr[l + 1]
        order = np.argsort(rank[b:e])
        v, w = inst.v[b:e].astype(float), inst.w[b:e].astype(float)
        for q in range(e - b):
            S = order[: q + 1]
            out = order[q + 1:]
            den = inst.v0[l] + v[S].sum() + w[out].sum()
            a = alpha[b + order[q]]
            y[b + S] += inst.lam[l] * a * v[S] / den
    return y


def _mixed_sales(inst, k, seed):
    """A convex combination of k best responses (each satisfies the SBLP
    rows of every segment, so their mixture does too)."""
    rng = np.random.default_rng(seed)
    wts = rng.dirichlet(np.ones(k))
    y = np.zeros(inst.nnz)
    for q in range(k):
        eta = rng.uniform(0, 1, inst.m) * inst.r
        y += wts[q] * oracle.best_response(inst, eta)["sales"]
    return y


@pytest.mark.parametrize("seed", range(4))
def test_recovery_reproduces_sales(seed):
    inst = make_instance(60, 12, size_lo=1, size_hi=8, seed=seed, cap_lo=0.3)
    y = _mixed_sales(inst, 5, seed)
    rank, alpha, alpha0 = oracle.recover(inst, y)
    assert np.all(alpha >= -1e-12) and np.all(alpha0 >= -1e-12)
    total = alpha0.copy()
    np.add.at(total, np.repeat(np.arange(inst.L), np.diff(inst.seg_ptr)), alpha)
    np.testing.assert_allclose(total, 1.0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(_sales_of(inst, rank, alpha), y, rtol=1e-10, atol=1e-13)


def test_single_best_response_is_one_assortment():
    inst = make_instance(40, 10, size_lo=2, size_hi=6, seed=3, cap_lo=0.3)
    eta = np.random.default_rng(1).uniform(0, 1, inst.m) * inst.r * 0.5
    y = oracle.best_response(inst, eta)["sales"]
    rank, alpha, alpha0 = oracle.recover(inst, y)
    for l in range(inst.L):
        b, e = inst.seg_ptr[l], inst.seg_ptr[l + 1]
        k = int(np.count_nonzero(y[b:e] > 0))
        if k == 0:
            assert alpha0[l] == pytest.approx(1.0) and not alpha[b:e].any()
            continue
        # the offered products come first; only the set of all of them is used
        assert set(np.nonzero(y[b:e] > 0)[0]) == set(np.nonzero(rank[b:e] < k)[0])
        used = alpha[b:e] > 1e-12
        assert used.sum() == 1 and rank[b:e][used][0] == k - 1
        assert alpha[b:e][used][0] == pytest.approx(1.0, rel=1e-12)
        assert abs(alpha0[l]) <= 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_recovered_lp_optimum_is_cblp_optimal(seed):
    inst = make_instance(4, 6, size_lo=2, size_hi=4, seed=seed, cap_lo=0.3)
    opt, _, y = lp.sblp(inst, return_sales=True)
    y = np.maximum(y, 0.0)
    rank, alpha, alpha0 = oracle.recover(inst, y)
    assert np.all(alpha >= -1e-9) and np.all(alpha0 >= -1e-9)
    ys = _sales_of(inst, rank, alpha)
    np.testing.assert_allclose(ys, y, rtol=1e-7, atol=1e-9)
    S = np.bincount(inst.idx, weights=ys, minlength=inst.n)
    assert np.all(S <= inst.c * (1 + 1e-7) + 1e-9)                 # capacity rows of eq. 2
    assert float(np.dot(inst.r, S)) == pytest.approx(opt, rel=1e-7)
    assert lp.cblp(inst)[0] == pytest.approx(opt, rel=1e-7)


def test_sets_are_nested():
    """Three products ordered by y/v: the only sets with time are the
    prefixes {1}, {1, 2}, {1, 2, 3} and the empty set."""
    inst = make_instance(1, 3, size_lo=3, size_hi=3, seed=0)
    inst.idx[:] = [0, 1, 2]
    inst.v[:] = [1.0, 2.0, 1.5]
    inst.w[:] = [0.1, 0.2, 0.3]
    inst.v0[:] = 1.0
    inst.lam[:] = 1.0
    # offer {0,1,2} 30% of the time, {0,1} 20%, {0} 10% (GAM sales)
    vt = inst.v - inst.w
    vt0 = 1.0 + inst.w.sum()
    y = np.zeros(3)
    for sets, x in (([0, 1, 2], 0.3), ([0, 1], 0.2), ([0], 0.1)):
        y[sets] += x * inst.v[sets] / (vt0 + vt[sets].sum())
    rank, alpha, alpha0 = oracle.recover(inst, y)
    assert list(rank) == [0, 1, 2]
    np.testing.assert_allclose(alpha, [0.1, 0.2, 0.3], rtol=1e-12)
    assert alpha0[0] == pytest.approx(0.4, rel=1e-12)
