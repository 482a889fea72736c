"""Pins of the warm-start reference (oracle/mlp.py) to facts outside itself:
torch's BF16 conversion and GELU, finite differences and automatic
differentiation of the FP64 network, a network whose output has a closed form,
Adam's first step, and features that the instance generator fixes."""
import numpy as np
import pytest

import oracle.mlp as om
from paper_2602_22421_amd.instances import make_instance, tiny_instance

torch = pytest.importorskip("torch")


def test_bf16_matches_torch_rounding():
    g = np.random.default_rng(0)
    x = np.concatenate([g.normal(size=20000) * 10.0 ** g.integers(-8, 8, size=20000),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-40]])
    # exact ties: the low 16 bits are 0x8000, rounding goes to the even neighbour
    ties = (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).astype(np.uint32)
    x = np.concatenate([x, ties.view(np.float32).astype(np.float64)])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(om.bf16(x), ref)


def test_gelu_matches_torch_and_its_derivative():
    z = np.linspace(-8.0, 8.0, 4001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="none").numpy()
    np.testing.assert_allclose(om.gelu(z), ref, rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (om.gelu(z + h) - om.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(om.gelu_prime(z), fd, rtol=1e-7, atol=1e-8)


def _batch(seed, rows=24):
    g = np.random.default_rng(seed)
    X = np.column_stack([g.uniform(0.1, 1.0, rows), g.uniform(0, 1, rows),
                         g.uniform(0, 3, rows), g.uniform(0, 3, rows)])
    Y = g.uniform(0, 1, rows)
    return X, Y


def test_gradient_matches_finite_differences():
    X, Y = _batch(1)
    p = om.init_params(3)
    p[om.NPARAM - 1] = 0.2
    _, g = om.gradients(p, X, Y, bf=False)
    rng = np.random.default_rng(5)
    # a sample from every parameter block
    off = np.cumsum([0] + [int(np.prod(s)) for _, s in om.SHAPES])
    picks = np.concatenate([rng.integers(off[i], off[i + 1], size=6) for i in range(len(om.SHAPES))])
    for k in picks:
        h = 1e-6
        e = np.zeros_like(p)
        e[k] = h
        fd = (om.loss(p + e, X, Y, bf=False) - om.loss(p - e, X, Y, bf=False)) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-9), k


def test_gradient_matches_autograd():
    X, Y = _batch(2, rows=40)
    p = om.init_params(4)
    _, g = om.gradients(p, X, Y, bf=False)
    q = {k: torch.tensor(v.copy(), dtype=torch.float64, requires_grad=True)
         for k, v in om.unpack(p.copy()).items()}
    Xt, Yt = torch.from_numpy(X), torch.from_numpy(Y)
    gelu = lambda z: torch.nn.functional.gelu(z, approximate="none")
    y = gelu(gelu(Xt @ q["W1"] + q["b1"]) @ q["W2"] + q["b2"]) @ q["w3"] + q["b3"]
    torch.mean((y - Yt) ** 2).backward()
    ref = om.pack({k: q[k].grad.numpy() for k in q})
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("bf", [False, True])
def test_single_path_network_closed_form(bf):
    # one live path x0 -> unit 0 -> unit 0 -> output, weights exact in BF16
    a, b, c, b3 = 0.75, 1.5, -2.0, 0.25
    q = {"W1": np.zeros((4, 256)), "b1": np.zeros(256), "W2": np.zeros((256, 256)),
         "b2": np.zeros(256), "w3": np.zeros(256), "b3": np.array([b3])}
    q["W1"][0, 0], q["W2"][0, 0], q["w3"][0] = a, b, c
    x0 = np.array([-1.3, 0.0, 0.4, 2.2])
    X = np.column_stack([x0, np.ones(4), np.ones(4), np.ones(4)])
    Phi = lambda z: 0.5 * (1 + np.vectorize(__import__("math").erf)(z / np.sqrt(2)))
    h1 = a * x0 * Phi(a * x0)
    if bf:
        h1 = torch.from_numpy(h1.astype(np.float32)).to(torch.bfloat16).double().numpy()
    z2 = b * h1
    y_ref = c * z2 * Phi(z2) + b3
    y, _ = om.forward(om.pack(q), X, bf=bf)
    np.testing.assert_allclose(y, y_ref, rtol=1e-13, atol=1e-15)


class _RoundGrad(torch.autograd.Function):
    """Identity forward; the incoming gradient is rounded to BF16."""

    @staticmethod
    def forward(ctx, x):
        return x.view_as(x)

    @staticmethod
    def backward(ctx, g):
        return g.float().to(torch.bfloat16).double()


def _ste_bf16(x):
    """BF16-rounded value forward, identity gradient."""
    return x + (x.detach().float().to(torch.bfloat16).double() - x.detach())


def test_bf16_gradient_matches_autograd_with_rounding_hooks():
    X, Y = _batch(6, rows=32)
    p = om.init_params(7)
    _, g = om.gradients(p, X, Y, bf=True)
    q = {k: torch.tensor(v.copy(), dtype=torch.float64, requires_grad=True)
         for k, v in om.unpack(p.copy()).items()}
    Xt, Yt = torch.from_numpy(X), torch.from_numpy(Y)
    gelu = lambda z: torch.nn.functional.gelu(z, approximate="none")
    h1 = _ste_bf16(gelu(Xt @ _ste_bf16(q["W1"]) + q["b1"]))
    z2 = _RoundGrad.apply(h1 @ _ste_bf16(q["W2"])) + q["b2"]
    y = gelu(z2) @ _ste_bf16(q["w3"]) + q["b3"]
    torch.mean((y - Yt) ** 2).backward()
    ref = om.pack({k: q[k].grad.numpy() for k in q})
    # the two round the same FP64 values; a rare tie-breaking difference after
    # the FP32 conversion would show as one element off by a BF16 step
    np.testing.assert_allclose(g, ref, rtol=1e-9, atol=1e-13)
    _, ge = om.gradients(p, X, Y, bf=False)
    assert np.linalg.norm(g - ge) > 0


def test_adam_first_step_moves_by_lr_times_sign():
    g = np.array([3.0, -0.5, 0.0, 1e-3])
    p = np.array([1.0, 2.0, 3.0, 4.0])
    p1, m, v = om.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # m_hat = g and v_hat = g^2 at the first step
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_features_capacity_ratio_is_generator_factor():
    inst = make_instance(3000, 200, size_lo=3, size_hi=12, zipf=1.1, cap_lo=0.35, seed=9)
    X = om.features(inst)
    deg = np.bincount(inst.idx, minlength=inst.n)
    hit = deg > 0
    np.testing.assert_allclose(X[hit, 0], 0.35, rtol=1e-12)
    assert np.all(X[~hit, 0] == 4.0)
    np.testing.assert_allclose(X[:, 1], inst.r / inst.r.max(), rtol=1e-15)
    np.testing.assert_allclose(X[:, 3], np.log1p(deg * inst.n / inst.L), rtol=1e-15)


def test_features_brute_force_loops():
    inst = tiny_instance(7, 5, size_lo=1, size_hi=4, seed=2, cap_lo=0.3, cap_hi=0.6)
    d = [0.0] * inst.n
    a = [0.0] * inst.n
    for l in range(inst.L):
        lo, hi = inst.seg_ptr[l], inst.seg_ptr[l + 1]
        tot = inst.v0[l] + sum(inst.v[lo:hi])
        for q in range(lo, hi):
            d[inst.idx[q]] += inst.lam[l] * inst.v[q] / tot
            a[inst.idx[q]] += inst.v[q]
    X = om.features(inst)
    for j in range(inst.n):
        x0 = min(inst.c[j] / d[j], 4.0) if d[j] > 0 else 4.0
        assert X[j, 0] == pytest.approx(x0, rel=1e-13)
        assert X[j, 2] == pytest.approx(np.log1p(a[j] * inst.n / inst.L), rel=1e-13)


def test_resource_features_capacity_ratio_is_generator_factor():
    """Resources: c_i = f (A d)_i with the weights, so feature 0 is f."""
    inst = make_instance(3000, 200, m=40, size_lo=3, size_hi=12, zipf=1.1, cap_lo=0.35,
                         a_lo=1, a_hi=3, a_int=True, seed=9)
    X = om.features(inst)
    assert X.shape == (40, 4)
    prod = np.repeat(np.arange(inst.n), np.diff(inst.a_ptr))
    deg = np.bincount(inst.idx, minlength=inst.n).astype(float)
    hit = np.bincount(inst.a_idx, weights=deg[prod], minlength=inst.m) > 0
    np.testing.assert_allclose(X[hit, 0], 0.35, rtol=1e-12)
    assert np.all(X[~hit, 0] == 4.0)


def test_resource_features_brute_force_loops():
    inst = tiny_instance(9, 6, m=4, size_lo=1, size_hi=4, seed=3, cap_lo=0.3, cap_hi=0.6,
                         a_lo=0.5, a_hi=2.0)
    d = [0.0] * inst.n
    a = [0.0] * inst.n
    g = [0.0] * inst.n
    for l in range(inst.L):
        lo, hi = inst.seg_ptr[l], inst.seg_ptr[l + 1]
        tot = inst.v0[l] + sum(inst.v[lo:hi])
        for q in range(lo, hi):
            d[inst.idx[q]] += inst.lam[l] * inst.v[q] / tot
            a[inst.idx[q]] += inst.v[q]
            g[inst.idx[q]] += 1.0
    D, M, G = [0.0] * inst.m, [0.0] * inst.m, [0.0] * inst.m
    rb = [None] * inst.m
    for j in range(inst.n):
        for q in range(inst.a_ptr[j], inst.a_ptr[j + 1]):
            i, w = inst.a_idx[q], inst.a_val[q]
            D[i] += w * d[j]
            M[i] += w * a[j]
            G[i] += g[j]
            if w > 0:
                rb[i] = inst.r[j] / w if rb[i] is None else max(rb[i], inst.r[j] / w)
    rb = [0.0 if x is None else x for x in rb]
    X = om.features(inst)
    for i in range(inst.m):
        x0 = min(inst.c[i] / D[i], 4.0) if D[i] > 0 else 4.0
        assert X[i, 0] == pytest.approx(x0, rel=1e-13)
        assert X[i, 1] == pytest.approx(rb[i] / max(rb), rel=1e-13)
        assert X[i, 2] == pytest.approx(np.log1p(M[i] * inst.m / inst.L), rel=1e-13)
        assert X[i, 3] == pytest.approx(np.log1p(G[i] * inst.m / inst.L), rel=1e-13)
    np.testing.assert_allclose(om.resource_scale(inst), rb, rtol=1e-15)


def test_identity_as_a_matrix_gives_product_features():
    """A = I written out as a matrix gives the per-product features."""
    import dataclasses
    inst = make_instance(500, 30, size_lo=2, size_hi=8, seed=4, cap_lo=0.2, cap_hi=0.5)
    eye = dataclasses.replace(inst, a_ptr=np.arange(inst.n + 1, dtype=np.int64),
                              a_idx=np.arange(inst.n, dtype=np.int32), a_val=np.ones(inst.n))
    np.testing.assert_allclose(om.features(eye), om.features(inst), rtol=1e-14)
    eta = np.random.default_rng(0).uniform(0, 1, inst.n) * inst.r
    np.testing.assert_allclose(om.targets(eye, eta), om.targets(inst, eta), rtol=1e-15)
