"""Products renumbered by falling degree inside the library (so that the LDS
bins and LDS prices serve the most entries) change nothing the caller sees.
Instances whose product ids are in random order are checked against the FP64
oracle for every kernel the shape selects (all prices in LDS, the popular
head of them with 16- or 32-bit ids, sales past the LDS bins, general A),
and the batch and the warm-start features of shuffled instances against the
single solver and the oracle's features."""
import numpy as np
import pytest

import oracle
import oracle.mlp as omlp
from paper_2602_22421_amd.instances import (batch_instance, make_instance, shuffle_products,
                                            step_scale)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_22421_amd import cblp
    cblp.load()
    return cblp


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, float) - np.asarray(b, float)) /
                 max(np.linalg.norm(np.asarray(b, float)), 1e-300))


CASES = [
    # (dtype, n, m): n = 3000 puts every price and bin in LDS; 30,000 takes the
    # split-price kernel with 16-bit ids and sales past the bins; 70,000 the one
    # with 32-bit ids; m = 40 a general resource matrix
    ("f64", 3000, None),
    ("f32", 3000, None),
    ("f32", 30000, None),
    ("f32", 70000, None),
    ("f32", 3000, 40),
    ("f64", 3000, 40),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_shuffled_matches_oracle(cb, case):
    dtype, n, m = CASES[case]
    dt = torch.float32 if dtype == "f32" else torch.float64
    npdt = np.float32 if dtype == "f32" else np.float64
    inst0 = make_instance(20000, n, m=m, size_lo=1, size_hi=40, zipf=1.1, cap_lo=0.2,
                          cap_hi=0.5, seed=31)
    inst = shuffle_products(inst0, seed=7)[0].cast(npdt)
    prob = cb.Problem(inst, dtype=dt)
    rng = np.random.default_rng(4)
    base = inst.r if inst.identity else np.full(inst.m, float(inst.r.mean()))
    eta = (rng.uniform(0, 1, inst.m) * base * 0.5).astype(npdt)
    S, u, R = prob.sales(prob.tensor(eta), seg_R=True)
    ref = oracle.best_response(inst, eta.astype(np.float64))
    if dtype == "f64":
        np.testing.assert_allclose(R.cpu().numpy(), ref["seg_R"], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(S.cpu().numpy(), ref["S"], rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(u.cpu().numpy(), ref["u"], rtol=1e-9, atol=1e-9)
    else:
        np.testing.assert_allclose(R.double().cpu().numpy(), ref["seg_R"], rtol=2e-5, atol=1e-5)
        assert rel(S.cpu().numpy(), ref["S"]) <= 1e-5
        assert rel(u.cpu().numpy(), ref["u"]) <= 1e-5
    # equal-iteration duals
    tau = step_scale(inst, 1e-3).astype(npdt)
    e2 = prob.zeros_eta()
    tr, _ = prob.iterate(e2, 12, cb.make_params(rule=0, tau_vec=prob.tensor(tau), check_every=4))
    orc = oracle.Solver(inst, tau=tau.astype(np.float64), check_every=4)
    eo, tro = orc.iterate(np.zeros(inst.m), 12)
    bar = 1e-9 if dtype == "f64" else 1e-5
    assert rel(e2.cpu().numpy(), eo) <= bar
    assert rel(tr[:, 0], tro[:, 0]) <= bar and rel(tr[:, 1], tro[:, 1]) <= bar
    prob.close()


def test_shuffled_batch_and_features(cb):
    insts = [shuffle_products(batch_instance(b, scale=0.004), seed=b)[0].cast(np.float32)
             for b in range(4)]
    probs = [cb.Problem(i, dtype=torch.float32) for i in insts]
    # features against the oracle's, product by product in the caller's numbering
    for p, i in zip(probs, insts):
        X = cb.features(p).cpu().numpy()
        np.testing.assert_allclose(X, omlp.features(i), rtol=2e-6, atol=2e-6)
    taus = [p.tensor(step_scale(i, 2e-3).astype(np.float32)) for p, i in zip(probs, insts)]
    params = cb.make_params(rule=0, tau=1.0, check_every=5)
    single = []
    for p, t in zip(probs, taus):
        e = p.zeros_eta()
        p.iterate(e, 15, cb.make_params(rule=0, tau_vec=t, check_every=5), trace=False)
        single.append(e.cpu().numpy())
        p.reset()
    batch = cb.Batch(probs)
    etas = [p.zeros_eta() for p in probs]
    batch.iterate(etas, 15, params, tau_vecs=taus)
    for q, (a, b) in enumerate(zip(single, etas)):
        assert np.array_equal(a, b.cpu().numpy()), q
    batch.close()
    for p in probs:
        p.close()
