"""Pins of the oracle's bid-price policy simulation (Section 5.1, the GO
policy on the market of Figure 4) (CPU only).

* the offer rule on hand-worked cases: the in-stock fallback when at most K
  products remain, the bid-price test r_j - eta_j >= 0 (zero margin
  included), the cut to the K largest margins and its tie rule;
* choices: a customer's purchase frequencies over many uniforms are the
  basic attraction model's probabilities v_j / (1 + sum_S v), and the
  decision thresholds sit exactly at the running preference sums;
* a batch conserves inventory (sales = min(demand, stock), stock never
  negative, revenue = r . sales);
* the capacity reading: the LP over T' identical batches sharing capacity c
  has T' times the optimum of one batch with capacity c / T' (HiGHS);
* the bid-price rule never withholds a product that the batch's LP optimum
  sells (HiGHS duals and sales);
* a sold-out product's dual raised to its revenue gives the LP without the
  product (the same dual value and sales);
* closed-loop special cases: abundant stock keeps every dual at zero, so
  the K highest prices are offered in every batch; with at most K products
  no LP is solved.
"""
import numpy as np
import pytest

import oracle
import oracle.lp as lp
from oracle import gosim
from paper_2602_22421_amd.instances import gosim_market, market_instance


def test_lp_inputs_hand_worked():
    c, tau = gosim.lp_inputs(np.array([0, 4, 8]), 4, np.array([10.0, 2.0, 3.0]), 0.1)
    np.testing.assert_array_equal(c, [0.0, 1.0, 2.0])
    # zero capacity takes the step of the smallest positive one (1.0)
    np.testing.assert_allclose(tau, [1.0, 1.0, 0.5], rtol=1e-15)
    c, tau = gosim.lp_inputs(np.array([0, 0]), 3, np.array([4.0, 2.0]), 0.5)
    np.testing.assert_array_equal(c, [0.0, 0.0])
    np.testing.assert_allclose(tau, [2.0, 2.0], rtol=1e-15)
    c32, tau32 = gosim.lp_inputs(np.array([1, 7]), 3, np.array([1.0, 2.0]), 0.1, np.float32)
    assert c32.dtype == np.float32 and tau32.dtype == np.float32
    assert c32[0] == np.float32(1.0 / 3.0)
    assert tau32[1] == np.float32(0.1 * 2.0 / float(np.float32(7.0 / 3.0)))


def test_sold_out_dual_removes_the_product():
    """Raising a sold-out product's dual to its revenue is the LP without it:
    the same dual value and sales as the instance whose consideration sets
    omit the product (no shadow attraction, so an absent product and an
    unoffered one weigh the same)."""
    mk = gosim_market(1, n=6, periods=1, customers=25, seed=4)
    inv = mk.inv0[0].copy()
    inv[[1, 4]] = 0
    c, _ = gosim.lp_inputs(inv // 30, 1, mk.r[0], 0.1)
    eta = np.random.default_rng(0).uniform(0, 0.5, 6) * mk.r[0]
    eta2 = gosim.sold_out_duals(inv, eta, mk.r[0])
    assert np.all(eta2[[1, 4]] >= mk.r[0][[1, 4]])
    np.testing.assert_array_equal(np.delete(eta2, [1, 4]), np.delete(eta, [1, 4]))
    full = market_instance(mk.prefs[0, 0], mk.r[0], c)
    keep = [0, 2, 3, 5]
    part = market_instance(mk.prefs[0, 0][:, keep], mk.r[0][keep], c[keep])
    a = oracle.best_response(full, eta2)
    b = oracle.best_response(part, eta2[keep])
    assert a["S"][1] == 0.0 and a["S"][4] == 0.0
    np.testing.assert_allclose(a["S"][keep], b["S"], rtol=1e-12)
    assert a["D"] == pytest.approx(b["D"], rel=1e-12)


def test_offer_hand_worked():
    # at most K in stock: all of them, whatever the duals say
    assert gosim.offer([0, 5, 3, 0], [99, 99, 99, 99], [1, 1, 1, 1], 2) == [1, 2]
    assert gosim.offer([0, 0, 0], [0, 0, 0], [1, 2, 3], 2) == []
    # margins [10, -1, 5, 4, 2]: the two largest
    assert gosim.offer([1] * 5, [0, 9, 1, 0, 0], [10, 8, 6, 4, 2], 2) == [0, 2]
    # ties go to the lower index
    assert gosim.offer([1, 1, 1], [0, 0, 0], [5, 5, 5], 2) == [0, 1]
    # every margin negative: nothing is offered
    assert gosim.offer([1, 1, 1], [2, 2, 2], [1, 1, 1], 2) == []
    # a zero margin passes the rule
    assert gosim.offer([1, 1, 1], [3, 2, 2], [3, 1, 1], 2) == [0]
    # out-of-stock products never pass, even with the largest margin
    assert gosim.offer([0, 1, 1, 1], [0, 0, 0, 0], [9, 3, 2, 1], 2) == [1, 2]
    # K = 3 keeps three, returned in product order
    assert gosim.offer([1] * 5, [0, 0, 0, 0, 0], [1, 5, 2, 4, 3], 3) == [1, 3, 4]


def test_choice_frequencies_are_bam():
    rng = np.random.default_rng(5)
    row = np.array([0.9, 0.6, 0.2, 0.3])
    S = [1, 3]
    W = 1.0 + 0.6 + 0.3
    N = 200_000
    u = rng.random(N)
    picks = np.array([gosim.choose(row, x, S) for x in u])
    for j, p in ((1, 0.6 / W), (3, 0.3 / W), (-1, 1.0 / W)):
        f = np.mean(picks == j)
        assert abs(f - p) < 5 * np.sqrt(p * (1 - p) / N), (j, f, p)
    # thresholds: product 1 for u W < 0.6, product 3 below 0.9, else none
    assert gosim.choose(row, np.nextafter(0.6 / W, 0), S) == 1
    assert gosim.choose(row, 0.0, S) == 1
    assert gosim.choose(row, 0.7 / W, S) == 3
    assert gosim.choose(row, 0.95 / W, S) == -1
    assert gosim.choose(row, 0.5, []) == -1


@pytest.mark.parametrize("seed", range(3))
def test_period_conserves_inventory(seed):
    mk = gosim_market(1, n=8, periods=1, customers=400, inv_hi=60, seed=seed)
    rng = np.random.default_rng(seed)
    eta = rng.uniform(0, 1, 8) * mk.r[0]
    inv = mk.inv0[0].copy()
    inv[rng.integers(0, 8)] = 0
    S, sales, inv2, rev = gosim.period(inv, eta, mk.r[0], mk.prefs[0, 0], mk.u[0, 0], 2)
    assert len(S) <= 2 and all(inv[j] > 0 for j in S)
    assert np.all(sales >= 0) and np.all(sales <= inv) and np.all(inv2 >= 0)
    np.testing.assert_array_equal(inv - inv2, sales)
    outside = np.setdiff1d(np.arange(8), S)
    assert np.all(sales[outside] == 0)
    # demand counted independently of the oracle's loop
    W = 1.0 + mk.prefs[0, 0][:, S].sum(axis=1)
    cum = np.cumsum(mk.prefs[0, 0][:, S], axis=1)
    x = mk.u[0, 0] * W
    first = np.argmax(x[:, None] < cum, axis=1)
    buys = (x[:, None] < cum).any(axis=1)
    demand = np.bincount(np.asarray(S)[first[buys]], minlength=8) if S else np.zeros(8, int)
    np.testing.assert_array_equal(sales, np.minimum(demand, inv))
    assert rev == pytest.approx(float(np.dot(mk.r[0], sales)), rel=1e-14)


def _replicate(inst, copies):
    """The LP of `copies` batches drawn alike: the segments repeated."""
    N, n = inst.L, inst.n
    prefs = np.tile(inst.v.reshape(N, n), (copies, 1))
    return market_instance(prefs, inst.r, inst.c)


@pytest.mark.parametrize("seed", range(3))
def test_prorated_capacity_reading(seed):
    mk = gosim_market(1, n=5, periods=1, customers=6, seed=seed)
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.2, 2.0, 5)
    for copies in (2, 3):
        multi = _replicate(market_instance(mk.prefs[0, 0], mk.r[0], c), copies)
        one = market_instance(mk.prefs[0, 0], mk.r[0], c / copies)
        opt_multi, eta_multi = lp.sblp(multi)
        opt_one, eta_one = lp.sblp(one)
        assert opt_multi == pytest.approx(copies * opt_one, rel=1e-7)
        # the prorated batch's duals are optimal for the whole horizon too
        assert oracle.dual_value(multi, eta_one) == pytest.approx(opt_multi, rel=1e-6)


@pytest.mark.parametrize("seed", range(3))
def test_bid_price_rule_keeps_what_the_lp_sells(seed):
    mk = gosim_market(1, n=6, periods=1, customers=30, seed=seed)
    c, _ = gosim.lp_inputs(mk.inv0[0] // 40, 1, mk.r[0], 0.1)
    inst = market_instance(mk.prefs[0, 0], mk.r[0], c)
    _, eta, y = lp.sblp(inst, return_sales=True)
    S = np.bincount(inst.idx, weights=y, minlength=inst.n)
    margin = mk.r[0] - eta
    sold = S > 1e-8
    assert np.all(margin[sold] >= -1e-7)
    assert np.all(S[margin < -1e-7] <= 1e-8)


def test_simulate_abundant_stock_offers_top_prices():
    mk = gosim_market(1, n=7, periods=4, customers=50, inv_lo=10**7, inv_hi=10**7 + 5, seed=1)
    out = gosim.simulate(mk.r[0], mk.inv0[0], mk.prefs[:, 0], mk.u[:, 0], 2, tau0=0.1,
                         tol=1e-3, max_iters=40, check_every=10)
    top = sorted(np.argsort(-mk.r[0], kind="stable")[:2].tolist())
    assert all(S == top for S in out["offers"])
    assert np.all(out["eta"] == 0.0)
    assert np.all(out["iters"] > 0)
    sold = out["sales"].sum(axis=0)
    np.testing.assert_array_equal(mk.inv0[0] - out["inv"][-1], sold)


def test_simulate_without_lp_when_few_products():
    mk = gosim_market(1, n=2, periods=3, customers=40, inv_hi=30, seed=2)
    out = gosim.simulate(mk.r[0], mk.inv0[0], mk.prefs[:, 0], mk.u[:, 0], 2, tau0=0.1,
                         tol=1e-3, max_iters=50)
    assert np.all(out["iters"] == 0)
    inv = mk.inv0[0]
    for t in range(3):
        assert out["offers"][t] == [j for j in range(2) if inv[j] > 0]
        inv = out["inv"][t]


@pytest.mark.parametrize("seed", range(2))
def test_simulate_tight_stock(seed):
    mk = gosim_market(1, n=10, periods=6, customers=120, inv_hi=40, seed=seed)
    out = gosim.simulate(mk.r[0], mk.inv0[0], mk.prefs[:, 0], mk.u[:, 0], 2, tau0=0.05,
                         tol=1e-2, max_iters=300, check_every=10)
    inv = out["inv"]
    assert np.all(inv >= 0)
    assert np.all(np.diff(np.vstack([mk.inv0[0][None], inv]), axis=0) <= 0)
    np.testing.assert_array_equal(mk.inv0[0] - inv[-1], out["sales"].sum(axis=0))
    for t in range(6):
        assert out["revenue"][t] == pytest.approx(float(np.dot(mk.r[0], out["sales"][t])),
                                                  rel=1e-14, abs=0)
    # scarce stock: the LP prices some products above zero
    assert np.any(out["eta"][out["iters"] > 0] > 0)
