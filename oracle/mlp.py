"""FP64 CPU reference of the learned warm start (test infrastructure only).

Only the tests, the package smoke check and the benchmark may use this module;
the solver library never imports or runs it.  It restates, in plain numpy:

* the features the warm start reads for each dual's row (definitions in the
  library header: capacity over full-offer demand, normalised revenue,
  attraction mass and degree; per product for A = I, per resource through the
  weights a_ij otherwise), computed straight from the instance's CSR rows;
* the network y = w3 . GELU(W2^T GELU(W1^T x + b1) + b2) + b3 and its
  mean-squared-error gradient by backpropagation, in FP64, with BF16 rounding
  (round to nearest even) applied at the points the GPU kernels round: every
  weight where it is used, the first hidden activation entering the 256 x 256
  product, and that layer's output gradient entering the two backward
  products.  ``bf16=False`` drops every rounding and gives the exact gradient
  of the FP64 network, which the tests pin to finite differences and to
  automatic differentiation;
* one Adam step (Kingma and Ba, Algorithm 1).

The learned warm start is not part of the paper's method (Section 7 lists
learning components as future work); it changes only the starting duals
eta^0 that SPFOM (Algorithm 2, Algorithm 3) takes as an input.
"""
from __future__ import annotations

import numpy as np

IN, HID = 4, 256
SHAPES = (("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("w3", (HID,)), ("b3", (1,)))
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p: np.ndarray) -> dict:
    """Views of the flat parameter vector in the library's layout."""
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x) -> np.ndarray:
    """Round to the nearest BF16 value, ties to even (values first rounded to
    FP32, as the GPU holds them)."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def _erf(x: np.ndarray) -> np.ndarray:
    from scipy.special import erf
    return erf(x)


def gelu(z: np.ndarray) -> np.ndarray:
    """GELU(z) = z Phi(z), Phi the standard normal CDF."""
    return 0.5 * z * (1.0 + _erf(z / np.sqrt(2.0)))


def gelu_prime(z: np.ndarray) -> np.ndarray:
    """d/dz z Phi(z) = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + _erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(p: np.ndarray, X: np.ndarray, bf: bool = True):
    """Network output y [rows] and the activations the backward pass needs."""
    rnd = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    q = unpack(np.asarray(p, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ rnd(q["W1"]) + q["b1"]
    h1 = rnd(gelu(z1))
    z2 = h1 @ rnd(q["W2"]) + q["b2"]
    h2 = gelu(z2)
    y = h2 @ rnd(q["w3"]) + q["b3"][0]
    return y, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2)


def loss(p: np.ndarray, X: np.ndarray, Y: np.ndarray, bf: bool = True) -> float:
    y, _ = forward(p, X, bf)
    return float(np.mean((y - np.asarray(Y, dtype=np.float64)) ** 2))


def gradients(p: np.ndarray, X: np.ndarray, Y: np.ndarray, bf: bool = True):
    """(loss, gradient [NPARAM]) of the mean squared error, by backpropagation."""
    rnd = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    q = unpack(np.asarray(p, dtype=np.float64))
    y, a = forward(p, X, bf)
    rows = y.shape[0]
    dy = 2.0 * (y - np.asarray(Y, dtype=np.float64)) / rows
    g = {}
    g["b3"] = np.array([dy.sum()])
    g["w3"] = a["h2"].T @ dy
    dz2 = np.outer(dy, rnd(q["w3"])) * gelu_prime(a["z2"])
    g["b2"] = dz2.sum(axis=0)
    g["W2"] = a["h1"].T @ rnd(dz2)
    dh1 = rnd(dz2) @ rnd(q["W2"]).T
    dz1 = dh1 * gelu_prime(a["z1"])
    g["b1"] = dz1.sum(axis=0)
    g["W1"] = a["X"].T @ dz1
    return float(np.mean((y - Y) ** 2)), pack(g)


def adam_step(p, g, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at 1-based step `step`; returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def _product_sums(inst):
    """Per product: sales with every set offered whole (d), attraction mass
    and the number of segments holding it."""
    L, n = int(inst.L), int(inst.n)
    ptr = np.asarray(inst.seg_ptr, dtype=np.int64)
    idx = np.asarray(inst.idx, dtype=np.int64)
    v = np.asarray(inst.v, dtype=np.float64)
    seg = np.repeat(np.arange(L), np.diff(ptr))
    tot = np.asarray(inst.v0, dtype=np.float64) + np.bincount(seg, weights=v, minlength=L)
    share = np.asarray(inst.lam, dtype=np.float64)[seg] * v / tot[seg]
    d = np.bincount(idx, weights=share, minlength=n)
    att = np.bincount(idx, weights=v, minlength=n)
    deg = np.bincount(idx, minlength=n).astype(np.float64)
    return d, att, deg


def resource_scale(inst) -> np.ndarray:
    """The scale of each dual: r_j for A = I; for a resource matrix, the
    largest revenue per unit of resource i over the products that use it,
    max r_j / a_ij over a_ij > 0 (0 if no product uses it)."""
    r = np.asarray(inst.r, dtype=np.float64)
    if inst.a_ptr is None:
        return r.copy()
    out = np.full(int(inst.m), -np.inf)
    prod = np.repeat(np.arange(int(inst.n)), np.diff(np.asarray(inst.a_ptr)))
    ai = np.asarray(inst.a_idx, dtype=np.int64)
    av = np.asarray(inst.a_val, dtype=np.float64)
    use = av > 0
    np.maximum.at(out, ai[use], r[prod[use]] / av[use])
    return np.where(np.isfinite(out), out, 0.0)


def features(inst) -> np.ndarray:
    """Features [m, 4] of every dual's row, straight from the CSR rows: per
    product for A = I (m = n); per resource i otherwise, from the product sums
    weighted by a_ij: D_i = sum_j a_ij d_j, mass sum_j a_ij att_j, and the
    entries touching i sum_j deg_j (over the stored entries of row i)."""
    L, m = int(inst.L), int(inst.m)
    d, att, deg = _product_sums(inst)
    if inst.a_ptr is not None:
        prod = np.repeat(np.arange(int(inst.n)), np.diff(np.asarray(inst.a_ptr)))
        ai = np.asarray(inst.a_idx, dtype=np.int64)
        av = np.asarray(inst.a_val, dtype=np.float64)
        d = np.bincount(ai, weights=av * d[prod], minlength=m)
        att = np.bincount(ai, weights=av * att[prod], minlength=m)
        deg = np.bincount(ai, weights=deg[prod], minlength=m)
    c = np.asarray(inst.c, dtype=np.float64)
    r = resource_scale(inst)
    X = np.empty((m, IN))
    with np.errstate(divide="ignore", invalid="ignore"):
        X[:, 0] = np.where(d > 0, np.minimum(c / np.where(d > 0, d, 1.0), 4.0), 4.0)
    rmax = max(float(r.max()) if m else 0.0, 0.0)
    X[:, 1] = r / rmax if rmax > 0 else 0.0
    s = m / L if L > 0 else 0.0
    X[:, 2] = np.log1p(att * s)
    X[:, 3] = np.log1p(deg * s)
    return X


def targets(inst, eta) -> np.ndarray:
    """What the network predicts: eta_i / scale_i (0 where the scale is <= 0)."""
    sc = resource_scale(inst)
    eta = np.asarray(eta, dtype=np.float64)
    return np.where(sc > 0, eta / np.where(sc > 0, sc, 1.0), 0.0)


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases (numpy's generator; the library draws
    its own initial weights, so tests set parameters explicitly)."""
    g = np.random.default_rng(seed)
    q = {"W1": g.normal(size=(IN, HID)) * np.sqrt(2.0 / IN), "b1": np.zeros(HID),
         "W2": g.normal(size=(HID, HID)) * np.sqrt(2.0 / HID), "b2": np.zeros(HID),
         "w3": g.normal(size=HID) * np.sqrt(1.0 / HID), "b3": np.zeros(1)}
    return pack(q)
