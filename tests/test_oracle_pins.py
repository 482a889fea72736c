"""Pins of the FP64 oracle to facts outside itself (CPU only).

* brute force over every assortment of small segments;
* the root condition that defines R* (phi(R*) = 0);
* the textbook MNL result that revenue-ordered assortments are optimal;
* the paper's own inner solve (FAST-INNER, Algorithm 1, wrapped in a
  golden-section search over the no-purchase quantity, Section 4.1);
* the LP optimum of the enumerated CBLP (eqs. 1-4, GAM probabilities) and of
  the sales-based LP, solved by HiGHS: weak duality, tightness at the LP
  duals, CBLP = SBLP, and convergence of the iteration to the optimum;
* invariants: identical segments scale, an uncapacitated instance needs no
  dual price, and a hand-worked two-step example for the dual step (eq. 16).
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import oracle.lp as lp
from paper_2602_22421_amd.instances import (config_instance, make_instance, step_scale,
                                            tiny_instance)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_segment(rng, k, neg_frac=0.3):
    v = rng.uniform(0.5, 2.0, k)
    w = rng.uniform(0.0, 0.5, k) * v
    rho = rng.uniform(1.0, 100.0, k)
    rho[rng.random(k) < neg_frac] *= -0.3
    return rho, v, w, float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.5, 1.5))


def _brute(rho, v, w, v0, lam):
    """Max over all subsets of the GAM revenue rate, smallest maximiser."""
    k = len(rho)
    best, best_set = 0.0, ()
    for size in range(1, k + 1):
        for S in itertools.combinations(range(k), size):
            S = list(S)
            out = [q for q in range(k) if q not in S]
            den = v0 + v[S].sum() + w[out].sum()  # GAM denominator
            R = float(np.dot(rho[S], v[S]) / den)
            if R > best * (1 + 1e-13) + 1e-300:
                best, best_set = R, tuple(S)
    return best, best_set


@pytest.mark.parametrize("seed", range(40))
def test_segment_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 11))
    rho, v, w, v0, lam = _random_segment(rng, k)
    R, D, s = oracle.segment_response(rho, v, w, v0, lam)
    Rb, Sb = _brute(rho, v, w, v0, lam)
    assert R == pytest.approx(Rb, rel=1e-12, abs=1e-14)
    assert tuple(np.nonzero(s > 0)[0]) == Sb
    if Sb:
        den = v0 + v[list(Sb)].sum() + np.delete(w, list(Sb)).sum()
        np.testing.assert_allclose(s[list(Sb)], lam * v[list(Sb)] / den, rtol=1e-13)
        # z = lambda R* equals the reduced revenue of the sales
        assert lam * R == pytest.approx(float(np.dot(rho, s)), rel=1e-12)


@pytest.mark.parametrize("seed", range(20))
def test_threshold_root(seed):
    """R* > 0 is the root of phi(R) = sum_j (rho_j v_j - R vt_j)^+ - R vt_0."""
    rng = np.random.default_rng(100 + seed)
    k = int(rng.integers(1, 60))
    rho, v, w, v0, lam = _random_segment(rng, k)
    rho[0] = abs(rho[0]) + 1.0  # at least one product worth offering
    R, D, s = oracle.segment_response(rho, v, w, v0, lam)
    vt0 = v0 + w.sum()
    phi = np.maximum(rho * v - R * (v - w), 0.0).sum() - R * vt0
    assert R > 0
    assert abs(phi) <= 1e-11 * (np.abs(rho * v).sum())
    # offered set is exactly the entries whose key beats R*
    key = rho * v / (v - w)
    assert np.array_equal(s > 0, key > R)


def test_all_nonpositive_prices_offer_nothing():
    rho = np.array([-1.0, 0.0, -5.0])
    v = np.array([1.0, 2.0, 1.5])
    w = 0.2 * v
    R, D, s = oracle.segment_response(rho, v, w, 1.0, 1.0)
    assert R == 0.0 and not s.any() and D == pytest.approx(1.0 + w.sum())


@pytest.mark.parametrize("seed", range(20))
def test_mnl_revenue_ordered_closed_form(seed):
    """MNL (w = 0), eta = 0: the optimal assortment is revenue-ordered
    (Talluri and van Ryzin 2004): R* = max_q sum_{top q by r} r v / (v0 + sum v)."""
    rng = np.random.default_rng(200 + seed)
    k = int(rng.integers(1, 40))
    r = rng.uniform(1.0, 100.0, k)
    v = rng.uniform(0.5, 2.0, k)
    v0 = float(rng.uniform(0.2, 3.0))
    R, D, s = oracle.segment_response(r, v, np.zeros(k), v0, 1.0)
    order = np.argsort(-r, kind="stable")
    num = np.cumsum((r * v)[order])
    den = v0 + np.cumsum(v[order])
    q = int(np.argmax(num / den))
    assert R == pytest.approx(float(num[q] / den[q]), rel=1e-13)
    assert set(np.nonzero(s)[0]) == set(order[: q + 1].tolist())


def _fast_inner_value(t, rho, v, w, v0, lam):
    """Algorithm 1 of the paper at a fixed no-purchase level, GAM form.

    With t = s_0 / v_0 the scale rows cap s_j <= v_j t and the balance leaves
    a budget lambda - vt_0 t, spent at vt_j / v_j per unit of s_j.  Fill in
    decreasing value per unit of budget (rho_j v_j / vt_j; for MNL this is
    the paper's r_j - eta_j order) until the budget is gone.  The budget
    starts at lambda - vt_0 t, not lambda (the paper's initialisation leaves
    out the no-purchase share)."""
    vt = v - w
    vt0 = v0 + w.sum()
    budget = lam - vt0 * t
    val = 0.0
    for j in np.argsort(-(rho * v / vt), kind="stable"):
        if budget <= 0:
            break
        sj = min(v[j] * t, budget * v[j] / vt[j])
        val += rho[j] * sj
        budget -= sj * vt[j] / v[j]
    return val


def _golden_max(f, a, b, tol):
    g = (math.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c), f(d)
    while b - a > tol:
        if fc > fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = f(d)
    return max(fc, fd, f(a), f(b))


@pytest.mark.parametrize("seed", range(15))
def test_paper_fast_inner_with_golden_section(seed):
    rng = np.random.default_rng(300 + seed)
    k = int(rng.integers(1, 30))
    rho, v, w, v0, lam = _random_segment(rng, k)
    R, D, s = oracle.segment_response(rho, v, w, v0, lam)
    vt0 = v0 + w.sum()
    lo, hi = lam / (vt0 + (v - w).sum()), lam / vt0
    best = _golden_max(lambda t: _fast_inner_value(t, rho, v, w, v0, lam), lo, hi,
                       1e-13 * hi)
    assert best == pytest.approx(lam * R, rel=1e-9, abs=1e-12)


def _tiny(seed, resources):
    kw = {"a_lo": 0.5, "a_hi": 2.5} if resources == "weighted" else {}
    return tiny_instance(3, 5, m=3 if resources else None, seed=seed, size_lo=1,
                         size_hi=5, cap_lo=0.3, **kw)


@pytest.mark.parametrize("resources", [False, True, "weighted"])
@pytest.mark.parametrize("seed", range(6))
def test_cblp_equals_sblp_and_dual_is_tight(seed, resources):
    inst = _tiny(seed, resources)
    opt_c, eta_c = lp.cblp(inst)
    opt_s, eta_s = lp.sblp(inst)
    assert opt_s == pytest.approx(opt_c, rel=1e-9)
    # strong duality at the LP's capacity duals
    assert oracle.dual_value(inst, eta_c) == pytest.approx(opt_c, rel=1e-9)
    # weak duality everywhere else
    rng = np.random.default_rng(seed)
    for _ in range(10):
        eta = np.maximum(0.0, eta_c * rng.uniform(0.0, 2.0, inst.m) + rng.normal(0, 5, inst.m))
        assert oracle.dual_value(inst, eta) >= opt_c * (1 - 1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_best_response_sales_satisfy_gam_rows(seed):
    inst = config_instance(0, seed=seed)
    rng = np.random.default_rng(seed)
    br = oracle.best_response(inst, rng.uniform(0, 60, inst.m))
    assert lp.sblp_feasible(inst, br["sales"]) <= 1e-12


def test_identical_segments_scale():
    """L copies of one segment with capacity c behave like one segment with c/L."""
    one = make_instance(1, 6, size_lo=6, size_hi=6, seed=7, cap_lo=0.3)
    L = 5
    many = make_instance(1, 6, size_lo=6, size_hi=6, seed=7, cap_lo=0.3)
    many.L = L
    many.seg_ptr = np.arange(L + 1, dtype=np.int64) * 6
    for f in ("idx", "v", "w"):
        setattr(many, f, np.tile(getattr(one, f), L))
    many.v0 = np.repeat(one.v0, L)
    many.lam = np.repeat(one.lam, L)
    many.c = one.c * L
    opt1, eta1 = lp.sblp(one)
    optL, etaL = lp.sblp(many)
    assert optL == pytest.approx(L * opt1, rel=1e-9)
    tau1 = step_scale(one, 0.01)
    s1 = oracle.Solver(one, tau=tau1)
    sL = oracle.Solver(many, tau=tau1 / L)
    e1, t1 = s1.iterate(np.zeros(one.m), 25)
    eL, tL = sL.iterate(np.zeros(many.m), 25)
    np.testing.assert_allclose(eL, e1, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(tL[:, 0], L * t1[:, 0], rtol=1e-9)


def test_uncapacitated_needs_no_price():
    inst = config_instance(0)
    inst = inst.with_capacity(inst.c * 100.0)
    s = oracle.Solver(inst, tau=step_scale(inst, 0.01), check_every=1)
    eta, tr = s.iterate(np.zeros(inst.m), 2)
    assert not eta.any()
    # D = sum lambda R* = P at eta = 0 and the window average is feasible
    assert tr[1, 7] <= 1e-14
    opt, _ = lp.sblp(inst)
    assert tr[1, 5] == pytest.approx(opt, rel=1e-9)


def test_dual_step_hand_worked():
    """One segment, one product (v=2, w=0.5, v0=1, lambda=1, r=10, c=0.2).
    vt0 = 1.5, vt = 1.5.  At eta = 0: key = 10*2/1.5 = 13.33 > R* = 20/3,
    sales = 2/3, D = 20/3.  Step tau=0.5, mu=0.1:
        eta1 = max(0, 0.95*0 - 0.5*(0.2 - 2/3)) = 7/30.
    At eta1: rho = 10 - 7/30 = 293/30, R* = rho*2/3 = 293/45, sales 2/3,
        D2 = 0.2*7/30 + 293/45 = 0.046666... + 6.511111... = 6.557777...
        eta2 = 0.95*7/30 + 0.5*(2/3 - 0.2) = 0.221666... + 0.233333... = 0.455"""
    inst = make_instance(1, 1, size_lo=1, size_hi=1, seed=0)
    inst.v[:] = 2.0
    inst.w[:] = 0.5
    inst.v0[:] = 1.0
    inst.lam[:] = 1.0
    inst.r[:] = 10.0
    inst.c[:] = 0.2
    s = oracle.Solver(inst, tau=np.array([0.5]), mu=0.1, check_every=1)
    eta, tr = s.iterate(np.zeros(1), 2)
    assert tr[0, 0] == pytest.approx(20.0 / 3.0, rel=1e-14)
    assert tr[1, 0] == pytest.approx(0.2 * 7 / 30 + 293 / 45, rel=1e-14)
    assert eta[0] == pytest.approx(0.455, rel=1e-14)
    # the other trace columns, worked by hand:
    #   P: revenue r * sales = 10 * 2/3 at both steps (the product stays offered)
    #   Z: lambda R* = 20/3, then 293/45
    #   eta2: ||eta^{t-1}||^2 = 0, then (7/30)^2 (the duals each pass was taken at)
    #   infeas: (u - c)^+ / c = (2/3 - 0.2) / 0.2 = 7/3 at both steps
    #   dbest: min(20/3, 6.5577...) = the second bound
    #   theta: c / ubar = 0.2 / (2/3) = 0.3 at both checks (K = 1), so the
    #     bound LB = 0.3 * 20/3 = 2 (each window holds one step: it restarts
    #     after t = 1 and t = 2)
    #   step: 1 for the constant rule; gap = (dbest - 2) / dbest
    np.testing.assert_allclose(tr[:, 1], [20 / 3, 20 / 3], rtol=1e-14)
    np.testing.assert_allclose(tr[:, 2], [20 / 3, 293 / 45], rtol=1e-14)
    np.testing.assert_allclose(tr[:, 3], [0.0, (7 / 30) ** 2], rtol=1e-14, atol=0)
    np.testing.assert_allclose(tr[:, 4], [7 / 3, 7 / 3], rtol=1e-13)
    d2 = 0.2 * 7 / 30 + 293 / 45
    np.testing.assert_allclose(tr[:, 5], [20 / 3, d2], rtol=1e-14)
    np.testing.assert_allclose(tr[:, 9], [0.3, 0.3], rtol=1e-14)
    np.testing.assert_allclose(tr[:, 6], [2.0, 2.0], rtol=1e-14)
    np.testing.assert_allclose(tr[:, 8], [1.0, 1.0], rtol=0)
    np.testing.assert_allclose(tr[:, 7], [(20 / 3 - 2) / (20 / 3), (d2 - 2) / d2], rtol=1e-13)


def test_per_segment_bound_hand_worked():
    """Two segments with one product each (MNL, w = 0): segment 0 considers
    product 0 (v=1, v0=1, lambda=1, r=10, c=0.25), segment 1 product 1 (v=1,
    v0=1, lambda=1, r=4, c=1).  At eta = 0 each offers its product: sales
    1/2 each, revenues p = 5 and 2, P = 7.  Product 0 is over its capacity
    (ubar = 1/2 > 0.25: theta_0 = 1/2), product 1 is not (theta_1 = 1).
    With one step and K = 1: global bound theta P = 1/2 * 7 = 3.5; the
    per-segment bound scales only segment 0: 1/2 * 5 + 1 * 2 = 4.5."""
    inst = make_instance(2, 2, size_lo=1, size_hi=1, seed=0)
    inst.seg_ptr[:] = [0, 1, 2]
    inst.idx[:] = [0, 1]
    inst.v[:] = 1.0
    inst.w[:] = 0.0
    inst.v0[:] = 1.0
    inst.lam[:] = 1.0
    inst.r[:] = [10.0, 4.0]
    inst.c[:] = [0.25, 1.0]
    for perseg, lb in ((False, 3.5), (True, 4.5)):
        s = oracle.Solver(inst, tau=np.array([1e-9, 1e-9]), check_every=1, perseg=perseg)
        _, tr = s.iterate(np.zeros(2), 1)
        assert tr[0, 1] == pytest.approx(7.0, rel=1e-15)
        assert tr[0, 9] == pytest.approx(0.5, rel=1e-15)
        assert tr[0, 6] == pytest.approx(lb, rel=1e-15), perseg
        # the optimum lies inside [LB, D]: sell 0.25 of product 0 (its cap)
        # by offering it 1/2 of the time, and product 1 always: 2.5 + 2 = 4.5
        opt, _ = lp.sblp(inst)
        assert opt == pytest.approx(4.5, rel=1e-9)
        assert tr[0, 6] <= opt * (1 + 1e-12) <= tr[0, 0] * (1 + 1e-12)


def _golden_opt(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("opt"):
                return float(line.split()[1])
    raise KeyError(name)


def test_config0_lp_optimum_fixture():
    """The stored config-0 optimum (HiGHS on the SBLP) still holds."""
    inst = config_instance(0)
    opt, eta = lp.sblp(inst)
    assert opt == pytest.approx(_golden_opt("config0_lp.txt"), rel=1e-9)
    assert oracle.dual_value(inst, eta) == pytest.approx(opt, rel=1e-9)


def test_iteration_reaches_lp_optimum_config0():
    """Certified gap <= 1e-4 on the L=1000, n=50 workload; the bracket
    [LB, Dbest] contains the HiGHS optimum."""
    inst = config_instance(0)
    opt = _golden_opt("config0_lp.txt")
    s = oracle.Solver(inst, tau=step_scale(inst, 1.0), rule=oracle.RULE_POLYAK, gamma=1.0,
                      check_every=10)
    eta, last, ok = s.solve(np.zeros(inst.m), 1e-4, 5000)
    assert ok, last
    dbest, lb = last[5], last[6]
    assert lb <= opt * (1 + 1e-12) and dbest >= opt * (1 - 1e-12)
    assert abs(dbest - opt) / opt <= 1e-4 and abs(opt - lb) / opt <= 1e-4


@pytest.mark.parametrize("weights", [None, "int"])
@pytest.mark.parametrize("seed", range(3))
def test_iteration_brackets_lp_optimum_with_resources(seed, weights):
    kw = {"a_lo": 1, "a_hi": 3, "a_int": True} if weights else {}
    inst = make_instance(60, 12, m=5, size_lo=2, size_hi=6, seed=seed, cap_lo=0.3, **kw)
    if weights:
        assert np.any(inst.a_val > 1)
    opt, _ = lp.sblp(inst)
    s = oracle.Solver(inst, tau=step_scale(inst, 1.0), rule=oracle.RULE_POLYAK, gamma=1.0,
                      check_every=5, perseg=True)
    eta, tr = s.iterate(np.zeros(inst.m), 3000)
    assert np.all(tr[:, 0] >= opt * (1 - 1e-12))
    assert np.all(tr[:, 6] <= opt * (1 + 1e-12))
    assert tr[-1, 7] < 0.5  # bracket tightens; convergence speed is not pinned here
