"""Learned warm start on the GPU: features, the MFMA forward pass, gradients
and Adam against the FP64 reference with the same BF16 rounding points,
training, and the gain over the cold start with its fallback."""
import numpy as np
import pytest

import oracle
import oracle.mlp as om
from paper_2602_22421_amd.instances import config_instance, make_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_22421_amd import cblp
    cblp.load()
    return cblp


def _rows(seed, rows):
    g = np.random.default_rng(seed)
    X = np.column_stack([g.uniform(0.1, 4.0, rows), g.uniform(0, 1, rows),
                         g.uniform(0, 4, rows), g.uniform(0, 4, rows)]).astype(np.float32)
    Y = g.uniform(0, 1, rows).astype(np.float32)
    return X, Y


def _params(seed):
    p = om.init_params(seed)
    g = np.random.default_rng(seed + 1)
    q = om.unpack(p)
    q["b1"][:] = g.normal(size=256) * 0.1
    q["b2"][:] = g.normal(size=256) * 0.1
    q["b3"][:] = 0.3
    return p.astype(np.float32)


# Forward tolerance.  Both sides round h1 = GELU(z1) to BF16, the GPU from
# its FP32 value, the reference from FP64; where h1 lies within FP32 error of
# a BF16 rounding boundary the two round to neighbouring BF16 values.  Such a
# row differs by at most one BF16 step of one h1_i carried to the output,
# ulp(h1_i) * sum_u |W2[i,u] w3_u| * max GELU' (GELU' <= 1.13); every other
# row differs only by FP32 accumulation (256 terms, about 256 * 2^-24 of the
# sum of |terms|), far below 1e-5 of the output scale here.
FWD_RTOL = 1e-5


def _flip_bound(p, X):
    q = om.unpack(p.astype(np.float64))
    h1 = om.gelu(X.astype(np.float64) @ om.bf16(q["W1"]) + q["b1"])
    ulp = 2.0 ** (np.floor(np.log2(np.abs(h1).max())) - 7)
    return ulp * np.max(np.abs(om.bf16(q["W2"])) @ np.abs(om.bf16(q["w3"]))) * 1.13


@pytest.mark.parametrize("rows", [1, 16, 1000, 4099])
def test_forward_matches_reference(cb, rows):
    net = cb.WarmStartNet(seed=1)
    p = _params(3)
    net.params = p
    X, _ = _rows(rows, rows)
    y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    ref, _ = om.forward(p.astype(np.float64), X.astype(np.float64), bf=True)
    err = np.abs(y - ref)
    tight = err <= FWD_RTOL * (np.abs(ref).max() + 1.0)
    assert tight.mean() >= 0.99, (tight.mean(), err.max())
    assert err.max() <= _flip_bound(p, X) + FWD_RTOL * (np.abs(ref).max() + 1.0)
    net.close()


def test_forward_single_path_exact(cb):
    """One live path (input 0 -> unit 5 -> unit 37 -> output): every product has one
    nonzero term, so the MFMA tile layout must put it in the right place."""
    p = np.zeros(om.NPARAM, np.float32)
    q = om.unpack(p)
    q["W1"][0, 5] = 0.75
    q["W2"][5, 37] = 1.5
    q["w3"][37] = -2.0
    q["b3"][0] = 0.25
    net = cb.WarmStartNet(seed=0)
    net.params = p
    X, _ = _rows(7, 50)
    y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    ref, _ = om.forward(p.astype(np.float64), X.astype(np.float64), bf=True)
    np.testing.assert_allclose(y, ref, rtol=1e-5, atol=1e-6)
    # and a different (i, u) gives a different answer: the test sees the layout
    q["W2"][5, 37], q["W2"][37, 5] = 0.0, 1.5
    q["w3"][37], q["w3"][5] = 0.0, -2.0
    net.params = p
    y2 = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    np.testing.assert_allclose(y2, 0.25, atol=1e-6)
    net.close()


def _blocks():
    off = np.cumsum([0] + [int(np.prod(s)) for _, s in om.SHAPES])
    return {name: slice(off[i], off[i + 1]) for i, (name, _) in enumerate(om.SHAPES)}


@pytest.mark.parametrize("rows", [37, 700])
def test_gradients_match_reference(cb, rows):
    net = cb.WarmStartNet(seed=2)
    p = _params(5)
    net.params = p
    X, Y = _rows(11 + rows, rows)
    loss, g = net.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda())
    g = g.cpu().numpy().astype(np.float64)
    lref, gref = om.gradients(p.astype(np.float64), X.astype(np.float64), Y.astype(np.float64))
    assert loss == pytest.approx(lref, rel=1e-4)
    for name, sl in _blocks().items():
        d = np.linalg.norm(g[sl] - gref[sl])
        # FP32 sums over rows and hidden units, plus rare BF16 boundary flips
        assert d <= 2e-4 * np.linalg.norm(gref[sl]) + 1e-9, (name, d, np.linalg.norm(gref[sl]))
    net.close()


# ------------------------------------------------ against the exact network
#
# The GPU network works with BF16 operands (8 significant bits, so each
# rounding to nearest is a relative error of at most U = 2^-8) and FP32
# sums.  Its answer is compared with the exact FP64 network (oracle.mlp with
# bf=False) within the spread that BF16 rounding produces: the exact network
# is evaluated SAMPLES times with every weight and every intermediate array
# (z1, h1, z2, h2, y and, backward, dZ2, dH1, dZ1) multiplied by independent
# factors 1 + U xi, xi uniform in [-1, 1] - wherever an implementation might
# round, not only where this one does - and the tolerance of each output
# entry is K standard deviations of those samples plus 2^-20 of the sum of
# |terms| for the FP32 sums.  Weight perturbations are shared by all rows of
# a sample, so errors that add up coherently over rows are covered.

U = 2.0 ** -8
F32 = 2.0 ** -20
K = 8.0
SAMPLES = 48


def _perturbed(p, X, Y, rng):
    """Exact network output and gradient with every array perturbed (rng:
    None for the unperturbed network)."""
    def f(a):
        a = np.asarray(a, dtype=np.float64)
        return a if rng is None else a * (1.0 + U * rng.uniform(-1.0, 1.0, a.shape))
    q = om.unpack(p.astype(np.float64))
    X = X.astype(np.float64)
    W1, W2, w3 = f(q["W1"]), f(q["W2"]), f(q["w3"])
    z1 = f(X @ W1 + q["b1"])
    h1 = f(om.gelu(z1))
    z2 = f(h1 @ W2 + q["b2"])
    h2 = f(om.gelu(z2))
    y = f(h2 @ w3 + q["b3"][0])
    if Y is None:
        return y, None
    e = 2.0 * (y - Y.astype(np.float64)) / X.shape[0]
    D2 = f(np.outer(e, w3) * om.gelu_prime(z2))
    dH1 = f(D2 @ W2.T)
    D1 = f(dH1 * om.gelu_prime(z1))
    g = dict(b3=np.array([e.sum()]), w3=h2.T @ e, b2=D2.sum(0), W2=h1.T @ D2,
             b1=D1.sum(0), W1=X.T @ D1)
    return y, om.pack(g)


def _exact_bounds(p, X, Y, seed=0):
    """(y, y_tol) and, with targets Y, (g, g_tol) of the exact network."""
    y, g = _perturbed(p, X, Y, None)
    rng = np.random.default_rng(seed)
    ys, gs = [], []
    for _ in range(SAMPLES):
        yp, gp = _perturbed(p, X, Y, rng)
        ys.append(yp)
        gs.append(gp)
    q = om.unpack(p.astype(np.float64))
    h1 = np.abs(om.gelu(X.astype(np.float64) @ q["W1"] + q["b1"]))
    mag_y = (h1 @ np.abs(q["W2"]) + np.abs(q["b2"])) @ np.abs(q["w3"]) + abs(q["b3"][0])
    ytol = K * np.std(ys, axis=0) + F32 * mag_y
    if Y is None:
        return (y, ytol), None
    gmag = np.abs(np.asarray(gs)).max(axis=0)
    gtol = K * np.std(gs, axis=0) + F32 * X.shape[0] * gmag
    return (y, ytol), (g, gtol)


@pytest.mark.parametrize("rows", [37, 1000])
def test_forward_matches_exact_network(cb, rows):
    net = cb.WarmStartNet(seed=1)
    p = _params(3)
    net.params = p
    X, _ = _rows(rows + 5, rows)
    y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    (ye, tol), _ = _exact_bounds(p, X, None)
    ye2, _ = om.forward(p.astype(np.float64), X.astype(np.float64), bf=False)
    np.testing.assert_allclose(ye, ye2, rtol=1e-12)
    err = np.abs(y - ye)
    assert np.all(err <= tol), (np.max(err / tol), int(np.argmax(err / tol)))
    # the bound is not vacuous: it is a small fraction of the output scale
    assert np.median(tol) <= 0.1 * np.median(np.abs(ye))
    net.close()


@pytest.mark.parametrize("rows", [37, 700])
def test_gradients_match_exact_network(cb, rows):
    """Every gradient entry against the exact FP64 network's, within the
    bound carried from the BF16 roundings (row counts that leave partial
    MFMA tiles)."""
    net = cb.WarmStartNet(seed=2)
    p = _params(5)
    net.params = p
    X, Y = _rows(11 + rows, rows)
    loss, g = net.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda())
    g = g.cpu().numpy().astype(np.float64)
    _, (ge, tol) = _exact_bounds(p, X, Y)
    _, gref = om.gradients(p.astype(np.float64), X.astype(np.float64), Y.astype(np.float64),
                           bf=False)
    np.testing.assert_allclose(ge, gref, rtol=1e-9, atol=1e-14)
    err = np.abs(g - ge)
    for name, sl in _blocks().items():
        bad = np.nonzero(err[sl] > tol[sl])[0]
        assert bad.size == 0, (name, bad[:5], err[sl][bad[:5]], tol[sl][bad[:5]])
    # a sign error or a transposed index in any block would exceed the bound
    # on its larger entries: the bound is well below them
    for name, sl in _blocks().items():
        big = np.abs(ge[sl]) >= 0.5 * np.abs(ge[sl]).max()
        assert np.all(tol[sl][big] < 0.5 * np.abs(ge[sl][big])), name
    net.close()


def test_adam_step_matches_reference(cb):
    net = cb.WarmStartNet(seed=3)
    p = _params(9)
    net.params = p
    X, Y = _rows(21, 300)
    lr = 1e-3
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    p64 = p.astype(np.float64)
    m = np.zeros_like(p64)
    v = np.zeros_like(p64)
    gs = []
    for step in (1, 2):
        net.train_step(Xd, Yd, lr)
        _, g = om.gradients(p64, X.astype(np.float64), Y.astype(np.float64))
        gs.append(g)
        p64, m, v = om.adam_step(p64, g, m, v, step, lr)
    got = net.params.astype(np.float64)
    # Adam's step m_hat / sqrt(v_hat) depends on the gradient's direction, so
    # it matches where the gradient is well resolved in FP32 (both steps'
    # |g| above 1e-4 of its block's largest); each step is at most lr long
    # (Cauchy-Schwarz on the moment sums), so no entry can differ by over 4 lr
    ok = np.ones(om.NPARAM, bool)
    for sl in _blocks().values():
        for g in gs:
            ok[sl] &= np.abs(g[sl]) > 1e-4 * np.abs(g[sl]).max()
    assert ok.mean() > 0.7
    np.testing.assert_allclose(got[ok], p64[ok], atol=0.02 * lr)
    assert np.max(np.abs(got - p64)) <= 4.0 * lr
    net.close()


def _feature_instance(kind):
    if kind == "cfg":       # the L=2e6 Zipf workload shrunk (n = 2000 < LDS-binned products)
        return config_instance(1, seed=5, scale=0.01)
    # more products than the LDS bins hold, and products no segment considers
    return make_instance(3000, 5000, size_lo=5, size_hi=50, zipf=1.1, cap_lo=0.2, cap_hi=0.5,
                         seed=5)


@pytest.mark.parametrize("kind", ["cfg", "wide"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_features_match_reference(cb, dtype, kind):
    dt = torch.float32 if dtype == "f32" else torch.float64
    inst = _feature_instance(kind).cast(np.float32 if dtype == "f32" else np.float64)
    prob = cb.Problem(inst, dtype=dt)
    X = cb.features(prob).cpu().numpy().astype(np.float64)
    ref = om.features(inst)
    if kind == "wide":
        assert (np.bincount(inst.idx, minlength=inst.n) == 0).any()
    np.testing.assert_allclose(X, ref, rtol=2e-6, atol=1e-7)
    # deterministic: a second call is bitwise equal
    X2 = cb.features(prob).cpu().numpy().astype(np.float64)
    assert np.array_equal(X, X2)
    prob.close()


def _resource_instance(weights):
    kw = {"unit": {}, "int": {"a_lo": 1, "a_hi": 3, "a_int": True},
          "real": {"a_lo": 0.5, "a_hi": 2.0}}[weights]
    return make_instance(4000, 600, m=90, res_lo=1, res_hi=3, size_lo=3, size_hi=20, zipf=1.1,
                         cap_lo=0.2, cap_hi=0.5, seed=6, **kw)


@pytest.mark.parametrize("weights", ["unit", "int", "real"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_resource_features_and_targets_match_reference(cb, dtype, weights):
    """Bundles over base products (Section 5.2): one feature row and one
    target per resource, from the product sums weighted by a_ij."""
    dt = torch.float32 if dtype == "f32" else torch.float64
    npdt = np.float32 if dtype == "f32" else np.float64
    inst = _resource_instance(weights).cast(npdt)
    prob = cb.Problem(inst, dtype=dt)
    X = cb.features(prob).cpu().numpy().astype(np.float64)
    assert X.shape == (inst.m, 4)
    np.testing.assert_allclose(X, om.features(inst), rtol=2e-6, atol=1e-7)
    assert np.array_equal(X, cb.features(prob).cpu().numpy().astype(np.float64))
    eta = (np.random.default_rng(3).uniform(0, 1, inst.m) * om.resource_scale(inst)).astype(npdt)
    Y = cb.targets(prob, prob.tensor(eta)).cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(Y, om.targets(inst, eta.astype(np.float64)), rtol=1e-6, atol=1e-7)
    prob.close()


def test_resource_prediction_and_fallback(cb):
    """wsnet_predict on a resource matrix gives max(y, 0) times each
    resource's scale, y the network on the resource features; wsnet_start
    keeps it only when its dual bound beats the cold start's."""
    inst = _resource_instance("int")
    prob = cb.Problem(inst, dtype=torch.float64)
    net = cb.WarmStartNet(seed=5)
    y = net.forward(cb.features(prob)).cpu().numpy().astype(np.float64)
    eta = net.predict(prob).cpu().numpy()
    np.testing.assert_allclose(eta, np.maximum(y, 0.0) * om.resource_scale(inst), rtol=2e-7)
    e2, info = net.start(prob)
    d0 = oracle.dual_value(inst, np.zeros(inst.m))
    dp = oracle.dual_value(inst, eta)
    assert info["D0"] == pytest.approx(d0, rel=1e-10)
    assert info["D_pred"] == pytest.approx(dp, rel=1e-10)
    assert info["used"] == (dp < d0)
    if not info["used"]:
        assert torch.all(e2 == 0)
    net.close()
    prob.close()


def test_training_reduces_loss(cb):
    from paper_2602_22421_amd import warmstart
    X, _ = _rows(31, 20000)
    # a smooth target of the kind the duals follow: scarce, valuable products
    Y = (np.maximum(0.0, 1.0 - X[:, 0]) * X[:, 1] + 0.05 * X[:, 2]).astype(np.float32)
    net = cb.WarmStartNet(seed=4)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    losses = warmstart.train(net, Xd, Yd, epochs=8, batch=1024, lr=2e-3)
    assert losses[-1] < 0.05 * losses[0], losses
    net.close()


def test_warm_start_gains_and_falls_back(cb):
    """Train on the duals of 12 solved instances (capacities 0.5-3x the
    full-offer demand, so the duals vary between 0 and the revenue), then
    solve a held-out instance from the prediction and from zero."""
    from paper_2602_22421_amd import warmstart
    gen = lambda s: make_instance(20000, 400, size_lo=5, size_hi=50, zipf=1.1, cap_lo=0.5,
                                  cap_hi=3.0, seed=s)
    spec = warmstart.SolveSpec(rule=cb.SPFOM_STEP_CONST, tau0=3e-3, tol=3e-2, max_iters=3000)
    stages = [(3e-3, 1500), (1e-3, 1000), (3e-4, 1000)]
    X, Y = warmstart.collect([gen(100 + s) for s in range(12)], spec, dtype=torch.float64,
                             stages=stages)
    net = cb.WarmStartNet(seed=5)
    losses = warmstart.train(net, X, Y, epochs=40, batch=2048, lr=3e-4)
    assert losses[-1] < 0.2 * float(Y.var())
    inst = gen(999)
    prob = cb.Problem(inst, dtype=torch.float64)
    cold, _ = warmstart.cold_solve(prob, inst, spec)
    warm, _ = warmstart.warm_solve(net, prob, inst, spec)
    assert warm["warm"] and warm["D_pred"] < warm["D0"]
    assert warm["status"] == 0
    # the cold start needs about twice the iterations to certify 3e-2
    assert cold["status"] != 0 or warm["iters"] < 0.75 * cold["iters"], (warm, cold)
    # a network that predicts huge duals is refused: the run equals the cold one
    bad = np.zeros(om.NPARAM, np.float32)
    bad[-1] = 1e3                       # y = b3 = 1000 for every product
    net.params = bad
    fb, _ = warmstart.warm_solve(net, prob, inst, spec)
    assert not fb["warm"] and fb["D_pred"] > fb["D0"]
    assert fb["iters"] == cold["iters"] and fb["dbest"] == cold["dbest"]
    prob.close()
    net.close()
