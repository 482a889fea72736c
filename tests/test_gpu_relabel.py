"""Products renumbered by falling degree inside the library (so that the LDS
bins and LDS prices serve the most entries) change nothing the caller sees:
on instances whose product ids are in random order, every output agrees bit
for bit with the run that keeps the caller's numbering, for the single
solver (identity and general A, small bin counts, split prices), the batch
and the warm-start features."""
import numpy as np
import pytest

import oracle
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


def _set(monkeypatch, relabel, env):
    if relabel:
        monkeypatch.delenv("CBLP_RELABEL", raising=False)
    else:
        monkeypatch.setenv("CBLP_RELABEL", "0")
    for k, v in env.items():
        monkeypatch.setenv(k, v)


def _single(cb, inst, dt, monkeypatch, relabel, env):
    _set(monkeypatch, relabel, env)
    prob = cb.Problem(inst, dtype=dt)
    rng = np.random.default_rng(4)
    base = inst.r if inst.identity else np.full(inst.m, float(inst.r.mean()))
    eta = prob.tensor(rng.uniform(0, 1, inst.m) * base * 0.5)
    S, u, R = prob.sales(eta, seg_R=True)
    out = [S.cpu().numpy(), u.cpu().numpy(), R.cpu().numpy()]
    npdt = np.float32 if dt == torch.float32 else np.float64
    tau = prob.tensor(step_scale(inst, 1e-3).astype(npdt))
    e2 = prob.zeros_eta()
    tr, _ = prob.iterate(e2, 12, cb.make_params(rule=0, tau_vec=tau, check_every=4))
    out += [e2.cpu().numpy(), np.asarray(tr)]
    prob.close()
    return out


CASES = [
    # (dtype, n, m, env)
    ("f64", 3000, None, {}),
    ("f32", 3000, None, {}),
    ("f32", 3000, None, {"CBLP_SEG_BINS": "300"}),       # most products past the bins
    ("f32", 3000, None, {"CBLP_FLUSH": "rows", "CBLP_SEG_BINS": "300"}),
    ("f32", 3000, None, {"CBLP_SEG_VARIANT": "13"}),
    ("f32", 20000, None, {"CBLP_SEG_VARIANT": "19"}),    # split prices: head of 8192 in LDS
    ("f32", 20000, None, {"CBLP_SEG_VARIANT": "26"}),    # the same over the slot-major copy
    ("f32", 20000, None, {"CBLP_SEG_VARIANT": "27"}),
    ("f32", 70000, None, {"CBLP_SEG_VARIANT": "39"}),    # three parts, split prices, 32-bit ids
    ("f32", 3000, 40, {}),                               # general A
    ("f64", 3000, 40, {"CBLP_SEG_BINS": "300"}),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_relabel_bitwise(cb, case, monkeypatch):
    dtype, n, m, env = CASES[case]
    dt = torch.float32 if dtype == "f32" else torch.float64
    npdt = np.float32 if dtype == "f32" else np.float64
    inst0 = make_instance(20000, n, m=m, size_lo=1, size_hi=40, zipf=1.1, cap_lo=0.2,
                          cap_hi=0.5, seed=31)
    inst, _ = shuffle_products(inst0, seed=7)
    inst = inst.cast(npdt)
    ref = _single(cb, inst, dt, monkeypatch, False, env)
    got = _single(cb, inst, dt, monkeypatch, True, env)
    for k, (a, b) in enumerate(zip(ref, got)):
        assert np.array_equal(a, b), (case, k)


def test_relabel_matches_oracle(cb, monkeypatch):
    """FP64 sales of a shuffled instance against the oracle (the renumbering is
    undone inside the library)."""
    inst0 = make_instance(5000, 2500, size_lo=1, size_hi=30, zipf=1.1, seed=8)
    inst, _ = shuffle_products(inst0, seed=3)
    _set(monkeypatch, True, {"CBLP_SEG_BINS": "200"})
    prob = cb.Problem(inst, dtype=torch.float64)
    eta = np.random.default_rng(1).uniform(0, 1, inst.m) * inst.r * 0.5
    S, u, R = prob.sales(prob.tensor(eta), seg_R=True)
    ref = oracle.best_response(inst, eta)
    np.testing.assert_allclose(S.cpu().numpy(), ref["S"], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(R.cpu().numpy(), ref["seg_R"], rtol=1e-12, atol=1e-12)
    prob.close()


def test_relabel_batch_and_features(cb, monkeypatch):
    base = [shuffle_products(batch_instance(b, scale=0.004), seed=b)[0].cast(np.float32)
            for b in range(4)]

    def run(relabel):
        _set(monkeypatch, relabel, {})
        probs = [cb.Problem(i, dtype=torch.float32) for i in base]
        feats = [cb.features(p).cpu().numpy() for p in probs]
        taus = [p.tensor(step_scale(i, 2e-3).astype(np.float32)) for p, i in zip(probs, base)]
        batch = cb.Batch(probs)
        etas = [p.zeros_eta() for p in probs]
        rows = batch.iterate(etas, 15, cb.make_params(rule=0, tau=1.0, check_every=5),
                             tau_vecs=taus)
        out = feats + [e.cpu().numpy() for e in etas] + [np.asarray(rows)]
        batch.close()
        for p in probs:
            p.close()
        return out

    ref = run(False)
    got = run(True)
    for k, (a, b) in enumerate(zip(ref, got)):
        assert np.array_equal(a, b), k
