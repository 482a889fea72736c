"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Every instance is seeded and synthetic; the FP32 cases feed the oracle the
same FP32-rounded inputs promoted to FP64.  Bars: FP64 iterates within 1e-8
relative (1e-5 after long runs, where a near-tie in a best response can
flip); FP32 iterates within 1e-5 relative at equal iteration counts on the
duals, the dual bound and the primal revenue.
"""
import numpy as np
import pytest

import oracle
from paper_2602_22421_amd.instances import (Instance, config_instance, make_instance,
                                             step_scale)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def cb():
    _need_gpu()
    from paper_2602_22421_amd import cblp
    cblp.load()
    return cblp


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _pair(cb, inst, dtype, tau0=0.01, rule=0, gamma=1.0, mu=0.0, K=10):
    """GPU problem + oracle solver with the same (dtype-rounded) inputs."""
    npdt = np.float32 if dtype == torch.float32 else np.float64
    src = inst.cast(npdt)
    prob = cb.Problem(src, dtype=dtype)
    tau = step_scale(src, tau0 if rule == 0 else 1.0).astype(npdt)
    tau_dev = prob.tensor(tau)
    params = cb.make_params(rule=rule, check_every=K, tau_vec=tau_dev, gamma=gamma, mu=mu)
    orc = oracle.Solver(src, tau=tau.astype(np.float64), rule=rule, gamma=gamma, mu=mu,
                        check_every=K)
    return prob, params, orc, src


def _run_both(prob, params, orc, iters_list, eta0=None):
    eta_g = prob.zeros_eta() if eta0 is None else prob.tensor(eta0)
    eta_o = np.zeros(prob.m) if eta0 is None else np.asarray(eta0, dtype=np.float64)
    out = []
    done = 0
    for t in iters_list:
        tr_g, _ = prob.iterate(eta_g, t - done, params)
        eta_o, tr_o = orc.iterate(eta_o, t - done)
        done = t
        out.append((t, eta_g.double().cpu().numpy(), eta_o.copy(), tr_g, tr_o))
    return out


# ---------------------------------------------------------------- single pass

def test_sales_fp64_config0(cb):
    inst = config_instance(0)
    prob = cb.Problem(inst, dtype=torch.float64)
    rng = np.random.default_rng(1)
    for trial in range(3):
        eta = rng.uniform(0, 80, inst.m) * (trial > 0)
        S, u, R = prob.sales(prob.tensor(eta), seg_R=True)
        br = oracle.best_response(inst, eta)
        np.testing.assert_allclose(R.cpu().numpy(), br["seg_R"], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(S.cpu().numpy(), br["S"], rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(u.cpu().numpy(), br["u"], rtol=1e-11, atol=1e-11)
        g = prob.gap(prob.tensor(eta))
        assert g["D"] == pytest.approx(br["D"], rel=1e-12)
        assert g["Z"] == pytest.approx(br["Z"], rel=1e-12)
        assert g["P"] == pytest.approx(br["P"], rel=1e-11)


def test_sales_fp32_scaled_zipf(cb):
    inst = config_instance(1, scale=0.01).cast(np.float32)
    prob = cb.Problem(inst, dtype=torch.float32)
    rng = np.random.default_rng(2)
    eta = (rng.uniform(0, 60, inst.m)).astype(np.float32)
    S, u, R = prob.sales(prob.tensor(eta), seg_R=True)
    br = oracle.best_response(inst, eta.astype(np.float64))
    np.testing.assert_allclose(R.double().cpu().numpy(), br["seg_R"], rtol=2e-5, atol=1e-5)
    assert rel(S.cpu().numpy(), br["S"]) <= 1e-5
    g = prob.gap(prob.tensor(eta))
    assert g["D"] == pytest.approx(br["D"], rel=1e-6)
    assert g["P"] == pytest.approx(br["P"], rel=1e-5)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sales_resources(cb, dtype):
    dt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    inst = config_instance(2, scale=0.002).cast(npdt)
    prob = cb.Problem(inst, dtype=dt)
    rng = np.random.default_rng(3)
    eta = rng.uniform(0, 30, inst.m).astype(npdt)
    S, u, R = prob.sales(prob.tensor(eta), seg_R=True)
    br = oracle.best_response(inst, eta.astype(np.float64))
    tol = 1e-11 if dtype == "f64" else 2e-5
    np.testing.assert_allclose(R.double().cpu().numpy(), br["seg_R"], rtol=tol, atol=tol)
    assert rel(u.cpu().numpy(), br["u"]) <= tol
    assert prob.gap(prob.tensor(eta))["D"] == pytest.approx(br["D"], rel=tol)


def test_long_segments_use_streamed_path(cb):
    """Consideration sets longer than the 64 register-cached products."""
    inst = make_instance(300, 400, size_lo=60, size_hi=300, zipf=1.1, seed=11, cap_lo=0.3)
    prob = cb.Problem(inst, dtype=torch.float64)
    eta = np.random.default_rng(4).uniform(0, 50, inst.m)
    S, u, R = prob.sales(prob.tensor(eta), seg_R=True)
    br = oracle.best_response(inst, eta)
    np.testing.assert_allclose(R.cpu().numpy(), br["seg_R"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(S.cpu().numpy(), br["S"], rtol=1e-11, atol=1e-11)


def test_degenerate_segments(cb):
    """Empty consideration sets, single products, zero arrival rates."""
    inst = make_instance(500, 30, size_lo=0, size_hi=3, seed=12, cap_lo=0.3)
    inst.lam[::7] = 0.0
    prob = cb.Problem(inst, dtype=torch.float64)
    eta = np.random.default_rng(5).uniform(0, 90, inst.m)
    S, u, R = prob.sales(prob.tensor(eta), seg_R=True)
    br = oracle.best_response(inst, eta)
    assert (np.diff(inst.seg_ptr) == 0).any()
    np.testing.assert_allclose(R.cpu().numpy(), br["seg_R"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(S.cpu().numpy(), br["S"], rtol=1e-11, atol=1e-11)


def test_no_segments(cb):
    inst = make_instance(0, 5, seed=0)
    inst.c[:] = 2.0
    prob, params, orc, _ = _pair(cb, inst, torch.float64, tau0=0.1)
    res = _run_both(prob, params, orc, [3], eta0=np.full(5, 1.0))
    t, eg, eo, trg, tro = res[0]
    np.testing.assert_allclose(eg, eo, rtol=1e-14)
    np.testing.assert_allclose(trg[:, :5], tro[:, :5], rtol=1e-13)


# ---------------------------------------------------------------- iterations

@pytest.mark.parametrize("rule", [0, 1])
def test_iterate_fp64_config0(cb, rule):
    inst = config_instance(0)
    prob, params, orc, _ = _pair(cb, inst, torch.float64, tau0=0.002, rule=rule)
    for t, eg, eo, trg, tro in _run_both(prob, params, orc, [1, 10, 100, 1000]):
        bar = 1e-8 if t <= 100 else 1e-5
        assert rel(eg, eo) <= bar, (t, rel(eg, eo))
        # D, P, Z, ||eta||^2, infeasibility, Dbest, LB, step and theta
        for col in (0, 1, 2, 3, 4, 5, 6, 8, 9):
            assert rel(trg[:, col], tro[:, col]) <= bar, (t, col)


@pytest.mark.parametrize("dtype,rule", [("f64", 0), ("f64", 1), ("f32", 0)])
def test_per_segment_bound_matches_oracle(cb, dtype, rule):
    """The per-segment scaled bound (theta_l per segment) against the oracle's
    at equal iteration counts, identity and general resource matrices."""
    dt = torch.float64 if dtype == "f64" else torch.float32
    bar = 1e-8 if dtype == "f64" else 1e-5
    for inst in (config_instance(0), config_instance(2, scale=0.002)):
        npdt = np.float32 if dt == torch.float32 else np.float64
        src = inst.cast(npdt)
        prob = cb.Problem(src, dtype=dt)
        tau = step_scale(src, 0.002 if rule == 0 else 1.0).astype(npdt)
        params = cb.make_params(rule=rule, check_every=5, tau_vec=prob.tensor(tau),
                                bound=cb.SPFOM_BOUND_SEGMENT)
        orc = oracle.Solver(src, tau=tau.astype(np.float64), rule=rule, check_every=5,
                            perseg=True)
        orc_g = oracle.Solver(src, tau=tau.astype(np.float64), rule=rule, check_every=5)
        eg = prob.zeros_eta()
        trg, _ = prob.iterate(eg, 60, params)
        eo, tro = orc.iterate(np.zeros(src.m), 60)
        _, trq = orc_g.iterate(np.zeros(src.m), 60)
        assert rel(eg.double().cpu().numpy(), eo) <= bar
        for col in (0, 1, 5, 6, 7):
            assert rel(trg[:, col], tro[:, col]) <= bar, col
        # on the same iterates (constant steps do not depend on the bound) the
        # per-segment bound is never below the global one
        if rule == 0:
            assert np.all(tro[:, 6] >= trq[:, 6] * (1 - 1e-12))
        prob.close()


def test_iterate_fp32_scaled_zipf(cb):
    inst = config_instance(1, scale=0.01)
    prob, params, orc, _ = _pair(cb, inst, torch.float32, tau0=0.001)
    for t, eg, eo, trg, tro in _run_both(prob, params, orc, [1, 10, 100]):
        assert rel(eg, eo) <= 1e-5, (t, rel(eg, eo))
        for col in (0, 1, 2, 3, 4):
            assert rel(trg[:, col], tro[:, col]) <= 1e-5, (t, col)


@pytest.mark.parametrize("weights", ["unit", "int", "real"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_iterate_resources(cb, dtype, weights):
    """The resource matrix of bundles (Section 5.2): unit weights as in the
    paper, and bundles using several units (integers 1-3) or any positive
    amount (U(0.5, 2)) of a base product."""
    dt = torch.float64 if dtype == "f64" else torch.float32
    kw = {"unit": {}, "int": {"a_lo": 1, "a_hi": 3, "a_int": True},
          "real": {"a_lo": 0.5, "a_hi": 2.0}}[weights]
    inst = config_instance(2, scale=0.002, **kw)
    prob, params, orc, _ = _pair(cb, inst, dt, tau0=0.001, rule=0, mu=0.01)
    bar = 1e-8 if dtype == "f64" else 1e-5
    for t, eg, eo, trg, tro in _run_both(prob, params, orc, [1, 10, 60]):
        assert rel(eg, eo) <= bar, (t, rel(eg, eo))
        assert rel(trg[-1, 0], tro[-1, 0]) <= bar


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_weighted_resource_usage_matches_oracle(cb, dtype):
    """u = A S with non-unit weights, element by element, at a fixed eta."""
    dt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    inst = config_instance(2, scale=0.002, a_lo=0.5, a_hi=2.0).cast(npdt)
    prob = cb.Problem(inst, dtype=dt)
    rng = np.random.default_rng(8)
    eta = (rng.uniform(0, 0.3, inst.m) * float(inst.r.max()) / 3).astype(npdt)
    S, u, _ = prob.sales(prob.tensor(eta))
    ref = oracle.best_response(inst, eta.astype(np.float64))
    tol = 1e-12 if dtype == "f64" else 2e-5
    assert rel(S.cpu().numpy(), ref["S"]) <= tol
    assert rel(u.cpu().numpy(), ref["u"]) <= tol
    prob.close()


def test_bitwise_deterministic(cb):
    inst = config_instance(1, scale=0.01).cast(np.float32)
    out = []
    for _ in range(2):
        prob = cb.Problem(inst, dtype=torch.float32)
        params = cb.make_params(tau=0.05)
        eta = prob.zeros_eta()
        tr, _ = prob.iterate(eta, 30, params)
        out.append((eta.cpu().numpy().tobytes(), tr.tobytes()))
        prob.close()
    assert out[0] == out[1]


def test_solve_config0_reaches_lp_optimum(cb):
    import os
    inst = config_instance(0)
    with open(os.path.join(os.path.dirname(__file__), "golden", "config0_lp.txt")) as f:
        opt = float([ln for ln in f if ln.startswith("opt")][0].split()[1])
    prob = cb.Problem(inst, dtype=torch.float64)
    tau = prob.tensor(step_scale(inst, 1.0))
    params = cb.make_params(rule=1, tau_vec=tau, gamma=1.0, check_every=10, tol=1e-4,
                            max_iters=5000)
    st = prob.solve(prob.zeros_eta(), params).as_dict()
    assert st["status"] == 0, st
    assert st["lb"] <= opt * (1 + 1e-12) <= st["dbest"] * (1 + 2e-12)
    assert abs(st["dbest"] - opt) / opt <= 1e-4 and abs(opt - st["lb"]) / opt <= 1e-4


# ---------------------------------------------------------------- validation

@pytest.mark.parametrize("bad", ["w_ge_v", "idx_range", "neg_cap", "nan_v", "zero_v0"])
def test_create_rejects_invalid(cb, bad):
    inst = config_instance(0)
    if bad == "w_ge_v":
        inst.w[5] = inst.v[5]
    elif bad == "idx_range":
        inst.idx[3] = inst.n
    elif bad == "neg_cap":
        inst.c[2] = -1.0
    elif bad == "nan_v":
        inst.v[7] = np.nan
    elif bad == "zero_v0":
        inst.v0[4] = 0.0
    with pytest.raises(cb.CblpError) as e:
        cb.Problem(inst, dtype=torch.float64)
    assert e.value.code == cb.CBLP_EINVAL


# ---------------------------------------------------------------- full size

def test_full_size_zipf_sampled(cb):
    """The L=2e6, n=2e4 workload in the benchmark's launch configuration:
    per-segment R* on a sample of segments and the totals of one pass."""
    inst = config_instance(1).cast(np.float32)
    prob = cb.Problem(inst, dtype=torch.float32)
    rng = np.random.default_rng(6)
    eta = (rng.uniform(0, 1, inst.m) * inst.r * 0.6).astype(np.float32)
    S, u, R = prob.sales(prob.tensor(eta), seg_R=True)
    R = R.double().cpu().numpy()
    rho = inst.r.astype(np.float64) - eta.astype(np.float64)
    for l in rng.choice(inst.L, 2000, replace=False):
        b, e = inst.seg_ptr[l], inst.seg_ptr[l + 1]
        Ro, _, _ = oracle.segment_response(rho[inst.idx[b:e]], inst.v[b:e], inst.w[b:e],
                                           float(inst.v0[l]), float(inst.lam[l]))
        assert R[l] == pytest.approx(Ro, rel=2e-5, abs=1e-5), l
    # sum of sales equals the sum of per-segment sales totals (any size)
    g = prob.gap(prob.tensor(eta))
    assert g["Z"] == pytest.approx(float(np.dot(inst.lam.astype(np.float64), R)), rel=1e-6)
    Sg = S.cpu().numpy()
    assert np.all(Sg >= 0) and g["P"] == pytest.approx(float(np.dot(inst.r, Sg)), rel=1e-9)


def test_resources_full_n_sampled(cb):
    """The resource workload's product and resource counts (n = 1e5, m = 2e3:
    prices past LDS, so the split-price slot kernel runs, with 32-bit ids) on
    a quarter of its segments: R* of sampled segments against the oracle, and
    u = A S, Z and P against host sums of the returned values."""
    inst = config_instance(2, scale=0.25, n=100_000, m=2_000).cast(np.float32)
    assert inst.n == 100_000 and inst.m == 2_000
    prob = cb.Problem(inst, dtype=torch.float32)
    rng = np.random.default_rng(9)
    eta = rng.uniform(0, 30, inst.m).astype(np.float32)
    S, u, R = prob.sales(prob.tensor(eta), seg_R=True)
    R = R.double().cpu().numpy()
    Sg = S.cpu().numpy()
    rho = inst.r.astype(np.float64).copy()
    for j in range(inst.n):
        a, b = inst.a_ptr[j], inst.a_ptr[j + 1]
        rho[j] -= float(np.dot(inst.a_val[a:b].astype(np.float64), eta[inst.a_idx[a:b]]))
    for l in rng.choice(inst.L, 1500, replace=False):
        b, e = inst.seg_ptr[l], inst.seg_ptr[l + 1]
        Ro, _, _ = oracle.segment_response(rho[inst.idx[b:e]], inst.v[b:e], inst.w[b:e],
                                           float(inst.v0[l]), float(inst.lam[l]))
        assert R[l] == pytest.approx(Ro, rel=2e-5, abs=1e-5), l
    u_host = np.zeros(inst.m)
    np.add.at(u_host, inst.a_idx,
              inst.a_val.astype(np.float64) * np.repeat(Sg, np.diff(inst.a_ptr)))
    np.testing.assert_allclose(u.cpu().numpy(), u_host, rtol=1e-9, atol=1e-9)
    g = prob.gap(prob.tensor(eta))
    assert g["Z"] == pytest.approx(float(np.dot(inst.lam.astype(np.float64), R)), rel=1e-6)
    assert np.all(Sg >= 0) and g["P"] == pytest.approx(float(np.dot(inst.r, Sg)), rel=1e-9)
    prob.close()


# ---------------------------------------------------------- per-entry sales

def check_entry_sales(inst, eta, S, u, s, ref, rtol, quantum=0.0):
    """Per-entry sales against the oracle's, segment by segment.

    Where the GPU and the oracle choose the same assortment, every sale agrees
    within rtol.  Where they differ (a near-tie that the FP32 iterate
    resolves the other way), the GPU's assortment must still be optimal
    within rtol in FP64 arithmetic.  Product sales equal the sums of the
    per-entry sales exactly (the same fixed-point quanta), and the GPU's S
    differs from the oracle's by exactly the flipped segments' sales, up to
    rtol.  quantum: the fixed-point unit of the library's sales sums (every
    sale is rounded to it once), added to the absolute tolerances."""
    L = inst.L
    ptr = inst.seg_ptr
    seg = np.repeat(np.arange(L), np.diff(ptr))
    so = ref["sales"]
    ing, ino = s > 0, so > 0
    diff_entry = ing != ino
    flipped = np.zeros(L, bool)
    np.logical_or.at(flipped, seg, diff_entry)
    same = ~flipped[seg]
    np.testing.assert_allclose(s[same], so[same], rtol=rtol, atol=1e-12 + quantum)
    # optimality of the flipped segments' GPU assortments
    if flipped.any():
        rho = ref["rho"]
        v = inst.v.astype(np.float64)
        w = inst.w.astype(np.float64)
        vt0 = inst.v0.astype(np.float64) + np.bincount(seg, weights=w, minlength=L)
        num = np.where(ing, rho[inst.idx] * v, 0.0)
        den = np.where(ing, v - w, 0.0)
        N = np.bincount(seg, weights=num, minlength=L)
        D = vt0 + np.bincount(seg, weights=den, minlength=L)
        Rg = np.where(N > 0, N / D, 0.0)
        ls = np.nonzero(flipped)[0]
        assert np.all(Rg[ls] >= ref["seg_R"][ls] * (1 - rtol) - 1e-12), ls[:10]
        assert flipped.mean() <= 1e-3, flipped.sum()
    # S is the sum of the per-entry sales (the same fixed-point quanta)
    Sg = np.bincount(inst.idx, weights=s, minlength=inst.n)
    np.testing.assert_allclose(S, Sg, rtol=1e-12, atol=1e-12)
    # S against the oracle, after the flipped segments' own differences
    corr = np.bincount(inst.idx[~same], weights=(s - so)[~same], minlength=inst.n)
    cnt = np.bincount(inst.idx, minlength=inst.n)
    assert np.all(np.abs(S - corr - ref["S"]) <= rtol * np.abs(ref["S"]) + 1e-9 + quantum * cnt)
    return int(flipped.sum())


def test_entry_sales_fp64_config0(cb):
    inst = config_instance(0)
    prob = cb.Problem(inst, dtype=torch.float64)
    rng = np.random.default_rng(7)
    for trial in range(3):
        eta = rng.uniform(0, 80, inst.m) * (trial > 0)
        S, u, R, s = prob.sales(prob.tensor(eta), seg_R=True, entries=True)
        ref = oracle.best_response(inst, eta)
        s = s.cpu().numpy()
        np.testing.assert_allclose(s, ref["sales"], rtol=1e-12, atol=1e-14)
        assert check_entry_sales(inst, eta, S.cpu().numpy(), u.cpu().numpy(), s, ref, 1e-12) == 0
    prob.close()


@pytest.mark.parametrize("case", ["zipf", "resources", "long_rows", "shuffled"])
def test_entry_sales_fp32(cb, case):
    from paper_2602_22421_amd.instances import shuffle_products
    if case == "zipf":
        inst = config_instance(1, scale=0.01)
    elif case == "resources":
        inst = config_instance(2, scale=0.002)
    elif case == "long_rows":
        inst = make_instance(3000, 400, size_lo=1, size_hi=200, zipf=1.1, seed=13, cap_lo=0.3)
    else:
        inst = shuffle_products(config_instance(1, scale=0.01), seed=5)[0]
    inst = inst.cast(np.float32)
    prob = cb.Problem(inst, dtype=torch.float32)
    rng = np.random.default_rng(8)
    base = inst.r if inst.identity else np.full(inst.m, float(inst.r.mean()))
    eta = (rng.uniform(0, 1, inst.m) * base * 0.6).astype(np.float32)
    S, u, R, s = prob.sales(prob.tensor(eta), seg_R=True, entries=True)
    ref = oracle.best_response(inst, eta.astype(np.float64))
    q = 2.0 ** -cb.cblp_launch_info(prob.h)["fx_bits"]
    check_entry_sales(inst, eta, S.cpu().numpy(), u.cpu().numpy(), s.cpu().numpy(), ref, 2e-5, q)
    prob.close()


# ---------------------------------------------------------- full size

def check_duals_fp32(eg, eo, t):
    """FP32 duals against the FP64 oracle's at equal t.  Element by element
    within 1e-5 of the largest dual, except for products whose sales moved
    with a near-tie assortment (a segment whose best response the FP32 and
    the FP64 arithmetic resolve differently; the per-entry sales tests show
    such assortments are optimal within FP32 rounding): at most 0.1% of the
    products, each within 1e-3 of the largest dual.  The whole vector within
    1e-5 relative."""
    d = np.abs(eg - eo)
    scale = max(float(np.max(np.abs(eo))), 1e-30)
    assert rel(eg, eo) <= 1e-5, (t, rel(eg, eo))
    assert np.mean(d <= 1e-5 * scale) >= 0.999, (t, np.mean(d <= 1e-5 * scale))
    assert d.max() <= 1e-3 * scale, (t, d.max() / scale)


def test_full_size_config1_equal_iterations(cb):
    """The L=2e6, n=2e4 workload in the benchmark's launch shape: duals, dual
    bound and revenue after 1 and 10 FP32 iterations against the FP64
    oracle, element by element; then, at fixed duals, every segment's
    assortment and sales against the oracle's (covering the sales summed in
    the 64-bit and in the 32-bit LDS bins)."""
    inst = config_instance(1).cast(np.float32)
    prob, params, orc, _ = _pair(cb, inst, torch.float32, tau0=0.001)
    for t, eg, eo, trg, tro in _run_both(prob, params, orc, [1, 10]):
        check_duals_fp32(eg, eo, t)
        for col in (0, 1, 2):
            assert rel(trg[:, col], tro[:, col]) <= 1e-5, (t, col)
    rng = np.random.default_rng(6)
    eta = (rng.uniform(0, 1, inst.m) * inst.r * 0.6).astype(np.float32)
    S, u, R, s = prob.sales(prob.tensor(eta), seg_R=True, entries=True)
    ref = oracle.best_response(inst, eta.astype(np.float64))
    info = cb.cblp_launch_info(prob.h)
    H, H64 = info["lds_bins"], info["lds_bins64"]
    assert H64 < H and np.count_nonzero(ref["S"][H64:H]) > 1000   # the 32-bit bins are used
    assert np.count_nonzero(ref["S"][H:]) == 0 or H < inst.n
    check_entry_sales(inst, eta, S.cpu().numpy(), u.cpu().numpy(), s.cpu().numpy(), ref, 2e-5,
                      2.0 ** -info["fx_bits"])
    prob.close()


def _grouped_instance(n, per_group, seg_per_group, v_hi, seed):
    """Products in groups of per_group; seg_per_group consecutive segments
    consider one group each, so a segment block holds many sales of the same
    products.  Attractions U(1, v_hi) against v0 = 1, lambda = 1."""
    rng = np.random.default_rng(seed)
    groups = n // per_group
    L = groups * seg_per_group
    g = np.repeat(np.arange(groups), seg_per_group)
    idx = (g[:, None] * per_group + np.arange(per_group)[None, :]).ravel().astype(np.int32)
    nnz = idx.size
    v = rng.uniform(1.0, v_hi, nnz)
    w = v * rng.uniform(0.0, 0.5, nnz)
    return Instance(L=L, n=n, m=n, seg_ptr=np.arange(L + 1, dtype=np.int64) * per_group,
                    idx=idx, v=v, w=w, v0=np.ones(L), lam=np.ones(L),
                    r=rng.uniform(1, 100, n), c=np.full(n, 0.5 * seg_per_group / per_group))


@pytest.mark.parametrize("case", ["bound-fails", "bound-holds"])
def test_bin_layout_from_sales_bound(cb, case):
    """FP32 handles with more products than 64-bit LDS bins: a product takes
    a 32-bit bin only when its sales within any segment block are bounded
    below 2^32 quanta.  bound-fails: 40 segments in a row share each group of
    10 products, so every product may sell about 40 near-whole units in one
    block (above 2^32 quanta at 29 bits): no 32-bit bins.  bound-holds: 2
    segments per group, so every product gets a bin, all 32-bit.  Both
    against the oracle at fixed duals, with S the exact sum of the per-entry
    sales."""
    spg = 40 if case == "bound-fails" else 2
    inst = _grouped_instance(24000, 10, spg, 50.0, seed=3).cast(np.float32)
    prob = cb.Problem(inst, dtype=torch.float32)
    rng = np.random.default_rng(4)
    eta = (rng.uniform(0, 0.5, inst.m) * inst.r).astype(np.float32)
    S, u, R, s = prob.sales(prob.tensor(eta), seg_R=True, entries=True)
    info = cb.cblp_launch_info(prob.h)
    H, H64 = info["lds_bins"], info["lds_bins64"]
    if case == "bound-fails":
        assert H == H64 < inst.n, info
    else:
        assert H == inst.n and H64 == 0, info
    ref = oracle.best_response(inst, eta.astype(np.float64))
    check_entry_sales(inst, eta, S.cpu().numpy(), u.cpu().numpy(), s.cpu().numpy(), ref, 2e-5,
                      2.0 ** -info["fx_bits"])
    prob.close()


def test_full_size_resources_equal_iterations(cb):
    """The resource workload's product and resource counts (n = 1e5, m = 2e3:
    the split-price kernel with 32-bit ids) on a tenth of its segments: duals
    and bounds after 1 and 10 iterations, then per-entry sales at fixed
    duals, against the oracle."""
    inst = config_instance(2, scale=0.1, n=100_000, m=2_000).cast(np.float32)
    assert inst.n == 100_000 and inst.m == 2_000
    prob, params, orc, _ = _pair(cb, inst, torch.float32, tau0=0.001)
    for t, eg, eo, trg, tro in _run_both(prob, params, orc, [1, 10]):
        check_duals_fp32(eg, eo, t)
        for col in (0, 1, 2):
            assert rel(trg[:, col], tro[:, col]) <= 1e-5, (t, col)
    rng = np.random.default_rng(9)
    eta = rng.uniform(0, 30, inst.m).astype(np.float32)
    S, u, R, s = prob.sales(prob.tensor(eta), seg_R=True, entries=True)
    ref = oracle.best_response(inst, eta.astype(np.float64))
    check_entry_sales(inst, eta, S.cpu().numpy(), u.cpu().numpy(), s.cpu().numpy(), ref, 2e-5,
                      2.0 ** -cb.cblp_launch_info(prob.h)["fx_bits"])
    np.testing.assert_allclose(u.cpu().numpy(), ref["u"], rtol=1e-4, atol=1e-6)
    prob.close()


# ---------------------------------------------------------- failure paths

def test_nonfinite_iterate_reported(cb):
    """A finite but enormous step overflows the duals to infinity; the next
    dual bound is infinite and the call reports CBLP_ENONFINITE."""
    inst = config_instance(0)
    prob = cb.Problem(inst, dtype=torch.float64)
    params = cb.make_params(rule=0, tau=1e308, check_every=1)
    with pytest.raises(cb.CblpError) as e:
        prob.iterate(prob.zeros_eta(), 3, params)
    assert e.value.code == cb.CBLP_ENONFINITE
    prob.close()


def test_solve_not_converged_fills_stats(cb):
    inst = config_instance(0)
    prob = cb.Problem(inst, dtype=torch.float64)
    tau = prob.tensor(step_scale(inst, 0.002))
    params = cb.make_params(rule=0, tau_vec=tau, check_every=10, tol=0.0, max_iters=30)
    st = prob.solve(prob.zeros_eta(), params).as_dict()
    assert st["status"] == cb.CBLP_ENOTCONVERGED and st["iters"] == 30
    assert np.isfinite(st["D"]) and st["dbest"] >= st["lb"] > 0
    prob.close()
