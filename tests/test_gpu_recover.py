"""SBLP -> CBLP recovery on the GPU (cblp_recover, through the C ABI)
against the oracle's (Section 4.4): ranks bit for bit, probabilities to FP64
rounding, on averaged best responses of the GPU's own iterations (identity
and general A, FP32 and FP64 instances, long rows, zero arrival rates), and
at full size on sampled segments."""
import numpy as np
import pytest

import oracle
from paper_2602_22421_amd.instances import config_instance, make_instance, step_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_22421_amd import cblp
    cblp.load()
    return cblp


def _averaged_sales(cb, prob, inst, k, seed):
    """The mean of the GPU's per-entry best responses at k random duals (a
    point that satisfies every segment's SBLP rows)."""
    rng = np.random.default_rng(seed)
    base = inst.r if inst.identity else np.full(inst.m, float(inst.r.mean()))
    y = torch.zeros(prob.nnz, dtype=torch.float64, device=prob.device)
    for _ in range(k):
        eta = prob.tensor(rng.uniform(0, 1, inst.m) * base * 0.7)
        _, _, _, s = prob.sales(eta, entries=True)
        y += s
    return y / k


@pytest.mark.parametrize("dtype,case", [("f64", "cfg0"), ("f32", "zipf"), ("f32", "resources"),
                                        ("f64", "long_rows")])
def test_recover_matches_oracle(cb, dtype, case):
    dt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    if case == "cfg0":
        inst = config_instance(0)
        inst.lam[::9] = 0.0                       # segments that never arrive
    elif case == "zipf":
        inst = config_instance(1, scale=0.005)
    elif case == "resources":
        inst = config_instance(2, scale=0.001)
    else:
        inst = make_instance(500, 300, size_lo=60, size_hi=150, zipf=1.1, seed=17, cap_lo=0.3)
    inst = inst.cast(npdt)
    prob = cb.Problem(inst, dtype=dt)
    y = _averaged_sales(cb, prob, inst, 4, seed=len(case))
    rank, alpha, alpha0 = prob.recover(y)
    ro, ao, a0o = oracle.recover(inst, y.cpu().numpy())
    assert np.array_equal(rank.cpu().numpy(), ro)
    np.testing.assert_allclose(alpha.cpu().numpy(), ao, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(alpha0.cpu().numpy(), a0o, rtol=0, atol=1e-12)
    # a distribution over the nested sets, up to the rounding of the sales:
    # each sale is a multiple of the fixed-point quantum, so a segment's
    # balance row holds within (entries + 1) quanta, relative to lambda_l
    q = 2.0 ** -cb.cblp_launch_info(prob.h)["fx_bits"]
    k = np.diff(inst.seg_ptr)
    lam = np.maximum(inst.lam.astype(np.float64), 1e-300)
    slack = (1e-6 if dtype == "f32" else 1e-12) + 4 * (k + 1) * q / lam
    assert np.all(alpha.cpu().numpy() >= -slack[np.repeat(np.arange(inst.L), k)])
    assert np.all(alpha0.cpu().numpy() >= -slack)
    prob.close()


def test_recover_full_size_sampled(cb):
    """The L=2e6 workload: the recovery of one best response is that
    assortment offered all the time; sampled segments against the oracle."""
    inst = config_instance(1).cast(np.float32)
    prob = cb.Problem(inst, dtype=torch.float32)
    rng = np.random.default_rng(5)
    eta = prob.tensor((rng.uniform(0, 1, inst.m) * inst.r * 0.6).astype(np.float32))
    _, _, _, s = prob.sales(eta, entries=True)
    rank, alpha, alpha0 = prob.recover(s)
    s, rank, alpha, alpha0 = (x.cpu().numpy() for x in (s, rank, alpha, alpha0))
    ptr = inst.seg_ptr
    seg = np.repeat(np.arange(inst.L), np.diff(ptr))
    offered = np.bincount(seg, weights=(s > 0).astype(float), minlength=inst.L)
    # every segment that buys anything is offered the set of all it buys, all
    # the time: the sales are rounded to fixed-point quanta, so the offered
    # products' y / v differ in their last digits and the nested sets inside
    # that one get probabilities of that order (below 1e-6 in all)
    main = (rank == offered[seg] - 1) & (s > 0)
    buys = offered > 0
    a_main = np.bincount(seg, weights=np.where(main, alpha, 0.0), minlength=inst.L)
    a_rest = np.bincount(seg, weights=np.where(main, 0.0, alpha), minlength=inst.L)
    assert np.all(np.abs(a_main[buys] - 1.0) <= 1e-6)
    assert np.all(np.abs(a_rest) <= 1e-6)
    assert np.all(np.abs(alpha0[~buys] - 1.0) <= 1e-12)
    for l in rng.choice(inst.L, 500, replace=False):
        b, e = ptr[l], ptr[l + 1]
        sub = inst.__class__(L=1, n=inst.n, m=inst.m, seg_ptr=np.array([0, e - b]),
                             idx=inst.idx[b:e], v=inst.v[b:e], w=inst.w[b:e],
                             v0=inst.v0[l:l + 1], lam=inst.lam[l:l + 1], r=inst.r, c=inst.c)
        ro, ao, a0o = oracle.recover(sub, s[b:e])
        assert np.array_equal(rank[b:e], ro), l
        np.testing.assert_allclose(alpha[b:e], ao, rtol=1e-12, atol=1e-15)
    prob.close()
