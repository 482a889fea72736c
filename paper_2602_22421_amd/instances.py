"""Seeded synthetic choice-based LP instances.

This module only draws inputs.  It holds none of the solver's arithmetic and is
the one piece of code shared by the HIP path's tests and benchmarks and by the
CPU oracle's tests.

An instance follows the problem statement of the paper (Section 3, model
setup): customer segments l in [L] with arrival rates lambda_l, products j in
[n] with revenues r_j, per-segment consideration sets N_l (stored as CSR rows),
nominal attractions v_lj and shadow attractions w_lj of the generalized
attraction model (Section 3, GAM choice probability), a no-purchase attraction
v_l0, and capacitated resources i in [m] with capacities c_i.  Products consume
resources through a matrix A (Section 5.2, NRM with bundling: a bundle uses
a_ij units of base product i; 0/1 in the paper, any nonnegative weight
here); A = identity (m == n) is the plain single-resource-per-product case of
Sections 3-4.

Notation: the paper names customers i in [n], products j in [m] and writes w for
the nominal and v for the shadow attraction.  Here segments are l in [L],
products j in [n], resources i in [m], v is the nominal and w the shadow
attraction.

Value recipe (all seeded through numpy's PCG64):
  * set sizes  |N_l| ~ U{size_lo..size_hi}
  * members    drawn without replacement, uniformly or with popularity
               p_j proportional to (j+1)^(-s) (Zipf, product index = rank)
  * v ~ U(0.5, 2), w = u*v with u ~ U(0, 0.5), v_l0 = 1
  * r ~ U(1, 100), lambda ~ U(0.5, 1.5) or LogNormal(0, 1)
  * capacities: c = f * d, where d_j is the expected demand for product j
    when every segment is offered its whole consideration set under the
    nominal attractions, and f is fixed or drawn U(cap_lo, cap_hi) per row.
    With a resource matrix, c_i = f_i * (A d)_i.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = ["Instance", "make_instance", "config_instance", "tiny_instance",
           "batch_instance", "step_scale", "minibatch_schedule", "Market",
           "gosim_market", "market_instance"]


@dataclasses.dataclass
class Instance:
    L: int
    n: int
    m: int
    seg_ptr: np.ndarray          # int64 [L+1]
    idx: np.ndarray              # int32 [nnz], product ids, sorted within a row
    v: np.ndarray                # float [nnz] nominal attraction
    w: np.ndarray                # float [nnz] shadow attraction, 0 <= w < v
    v0: np.ndarray               # float [L] no-purchase attraction
    lam: np.ndarray              # float [L] arrival rate
    r: np.ndarray                # float [n] revenue
    c: np.ndarray                # float [m] capacity
    a_ptr: Optional[np.ndarray] = None   # int64 [n+1] CSC of A by product
    a_idx: Optional[np.ndarray] = None   # int32 [nnzA] resource ids
    a_val: Optional[np.ndarray] = None   # float [nnzA] consumption
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.seg_ptr[-1])

    @property
    def identity(self) -> bool:
        return self.a_ptr is None

    @property
    def dtype(self):
        return self.v.dtype

    def cast(self, dtype) -> "Instance":
        """Copy with every real-valued array rounded to ``dtype``."""
        dt = np.dtype(dtype)
        f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=dt)
        return dataclasses.replace(
            self, v=f(self.v), w=f(self.w), v0=f(self.v0), lam=f(self.lam),
            r=f(self.r), c=f(self.c), a_val=f(self.a_val))

    def with_capacity(self, c) -> "Instance":
        return dataclasses.replace(self, c=np.ascontiguousarray(c, dtype=self.c.dtype))


def _popularity_cdf(n: int, s: float):
    """Cumulative popularity law p_j proportional to (j+1)^(-s), with a guide
    table that maps a uniform draw to a first candidate index."""
    p = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    cdf[-1] = 1.0
    G = 1 << 16
    guide = np.searchsorted(cdf, np.arange(G) / G, side="right").astype(np.int64)
    return cdf, guide


def _draw(rng, shape, n, law):
    if law is None:
        return rng.integers(0, n, size=shape, dtype=np.int64).astype(np.int32)
    cdf, guide = law
    u = rng.random(shape).ravel()
    out = guide[(u * guide.shape[0]).astype(np.int64)]
    # advance to the first index whose cumulative probability exceeds u
    todo = np.nonzero(cdf[out] <= u)[0]
    while todo.size:
        out[todo] += 1
        todo = todo[cdf[out[todo]] <= u[todo]]
    np.minimum(out, n - 1, out=out)
    return out.astype(np.int32).reshape(shape)


def _draw_sets(rng, sizes: np.ndarray, n: int, cdf) -> np.ndarray:
    """Rows of distinct members; returns a padded [rows, kmax] array whose
    entries past sizes[l] hold distinct sentinels >= n.  Duplicates are redrawn
    from the same popularity law until none remain, which samples without
    replacement."""
    rows = sizes.shape[0]
    kmax = int(sizes.max()) if rows else 0
    if kmax > n:
        raise ValueError("set size exceeds product count")
    sent = (n + np.arange(kmax, dtype=np.int64)).astype(np.int32)
    valid = np.arange(kmax)[None, :] < sizes[:, None]
    d = _draw(rng, (rows, kmax), n, cdf)
    d = np.where(valid, d, sent[None, :])
    todo = np.arange(rows)
    while todo.size:
        sub = np.sort(d[todo], axis=1)
        dup = np.zeros(sub.shape, dtype=bool)
        dup[:, 1:] = sub[:, 1:] == sub[:, :-1]
        has = dup.any(axis=1)
        d[todo] = sub
        todo = todo[has]
        if not todo.size:
            break
        sub = sub[has]
        dup = dup[has]
        fresh = _draw(rng, (int(dup.sum()),), n, cdf)
        sub[dup] = fresh
        d[todo] = sub
    return d


def _row_ids(ptr: np.ndarray) -> np.ndarray:
    """Row id of every CSR entry (int32)."""
    rows = ptr.shape[0] - 1
    mark = np.zeros(int(ptr[-1]) + 1, dtype=np.int32)
    np.add.at(mark, ptr[1:-1], 1) if rows < 4096 else _bump(mark, ptr)
    return np.cumsum(mark[:-1], dtype=np.int32)


def _bump(mark, ptr):
    # ptr[1:-1] may repeat for empty rows, so count with bincount
    mark += np.bincount(ptr[1:-1], minlength=mark.shape[0]).astype(np.int32)


def make_instance(L: int, n: int, *, m: Optional[int] = None, size_lo: int = 5,
                  size_hi: int = 10, zipf: Optional[float] = None,
                  lam_dist: str = "uniform", cap_lo: float = 0.3,
                  cap_hi: Optional[float] = None, cap_scale: float = 1.0,
                  res_lo: int = 1, res_hi: int = 3, shadow_hi: float = 0.5,
                  a_lo: float = 1.0, a_hi: Optional[float] = None, a_int: bool = False,
                  seed: int = 0, chunk: int = 1 << 20, name: str = "") -> Instance:
    """Draw one instance.  ``m`` None means A = identity (m = n); otherwise
    every product (a bundle, Section 5.2) consumes res_lo..res_hi distinct
    random resources (base products), at unit weight when ``a_hi`` is None,
    else at weights U(a_lo, a_hi) (``a_int``: integers U{a_lo..a_hi}, units
    of the base product per bundle).  ``cap_hi`` None means the capacity
    factor is exactly ``cap_lo``."""
    if L < 0 or n <= 0:
        raise ValueError("need L >= 0 and n > 0")
    size_hi = min(size_hi, n)
    size_lo = min(size_lo, size_hi)
    ss = np.random.SeedSequence(seed)
    g_size, g_mem, g_v, g_u, g_r, g_lam, g_cap, g_res = [
        np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(8)]

    sizes = g_size.integers(size_lo, size_hi + 1, size=L, dtype=np.int64)
    seg_ptr = np.zeros(L + 1, dtype=np.int64)
    np.cumsum(sizes, out=seg_ptr[1:])
    nnz = int(seg_ptr[-1])
    cdf = _popularity_cdf(n, zipf) if zipf is not None else None

    idx = np.empty(nnz, dtype=np.int32)
    for a in range(0, L, chunk):
        b = min(L, a + chunk)
        d = _draw_sets(g_mem, sizes[a:b], n, cdf)
        keep = d < n
        idx[seg_ptr[a]:seg_ptr[b]] = d[keep]

    v = g_v.uniform(0.5, 2.0, size=nnz)
    w = g_u.uniform(0.0, shadow_hi, size=nnz) * v
    r = g_r.uniform(1.0, 100.0, size=n)
    if lam_dist == "uniform":
        lam = g_lam.uniform(0.5, 1.5, size=L)
    elif lam_dist == "lognormal":
        lam = g_lam.lognormal(0.0, 1.0, size=L)
    else:
        raise ValueError(lam_dist)
    v0 = np.ones(L)

    # expected demand with every segment offered its whole consideration set
    seg_of = _row_ids(seg_ptr)
    tot = v0 + np.bincount(seg_of, weights=v, minlength=L)
    demand = np.bincount(idx, weights=lam[seg_of] * v / tot[seg_of], minlength=n)
    del seg_of

    a_ptr = a_idx = a_val = None
    if m is None:
        m = n
        row_demand = demand
    else:
        cnt = g_res.integers(res_lo, res_hi + 1, size=n, dtype=np.int64)
        a_ptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(cnt, out=a_ptr[1:])
        dd = _draw_sets(g_res, cnt, m, None)
        a_idx = dd[dd < m].astype(np.int32)
        if a_hi is None:
            a_val = np.ones(a_idx.shape[0])
        elif a_int:
            a_val = g_res.integers(int(a_lo), int(a_hi) + 1, size=a_idx.shape[0]).astype(np.float64)
        else:
            a_val = g_res.uniform(a_lo, a_hi, size=a_idx.shape[0])
        prod_of = _row_ids(a_ptr)
        row_demand = np.bincount(a_idx, weights=demand[prod_of] * a_val, minlength=m)

    if cap_hi is None:
        f = np.full(m, cap_lo)
    else:
        f = g_cap.uniform(cap_lo, cap_hi, size=m)
    c = f * row_demand * cap_scale

    return Instance(L=L, n=n, m=m, seg_ptr=seg_ptr, idx=idx, v=v, w=w, v0=v0,
                    lam=lam, r=r, c=c, a_ptr=a_ptr, a_idx=a_idx, a_val=a_val,
                    name=name)


# Workload shapes.  Config ids 0-2 name the three plain solver workloads:
#   0: L=1e3 segments, n=50 products, A=I, sets U{5..10} uniform, c=0.3 d
#   1: L=2e6, n=2e4, A=I, sets U{5..50} Zipf(1.1), c=U(0.2,0.5) d
#   2: L=1e7, n=1e5, m=2e3 resources (1-3 per product), sets U{3..30}
#      Zipf(1.1), lambda LogNormal(0,1), c=U(0.2,0.5) A d
_CONFIGS = {
    0: dict(L=1000, n=50, size_lo=5, size_hi=10, zipf=None, cap_lo=0.3,
            cap_hi=None, seed=0),
    1: dict(L=2_000_000, n=20_000, size_lo=5, size_hi=50, zipf=1.1,
            cap_lo=0.2, cap_hi=0.5, seed=1),
    2: dict(L=10_000_000, n=100_000, m=2000, size_lo=3, size_hi=30, zipf=1.1,
            lam_dist="lognormal", cap_lo=0.2, cap_hi=0.5, seed=2),
}

CONFIG_NAMES = {
    0: "plain-L1e3-n50-identity",
    1: "plain-L2e6-n2e4-zipf-identity",
    2: "plain-L1e7-n1e5-m2e3-zipf-resources",
}


def config_instance(cfg: int, *, seed: Optional[int] = None, scale: float = 1.0,
                    **over) -> Instance:
    """Instance of a named workload.  ``scale`` < 1 shrinks L (and n, m for the
    large workloads) keeping the distributions, for tests that need the
    workload's structure at a size the oracle finishes quickly."""
    kw = dict(_CONFIGS[cfg])
    if seed is not None:
        kw["seed"] = seed
    if scale != 1.0:
        kw["L"] = max(1, int(round(kw["L"] * scale)))
        if cfg in (1, 2):
            kw["n"] = max(kw["size_hi"], int(round(kw["n"] * scale ** 0.5)))
            if "m" in kw:
                kw["m"] = max(4, int(round(kw["m"] * scale ** 0.5)))
    kw.update(over)
    kw.setdefault("name", CONFIG_NAMES[cfg] + ("" if scale == 1.0 else f"-x{scale:g}"))
    return make_instance(**kw)


def batch_instance(b: int, *, periods: int = 16, base_seed: int = 3_000_000,
                   L_range=(1e3, 1e6), n_range=(100, 10_000),
                   scale: float = 1.0) -> Instance:
    """Instance b of a multi-period re-solve batch: L and n log-uniform,
    the plain Zipf generator, capacities scaled by the period fraction
    t_b / T with t_b = 1 + (b mod T)."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(base_seed + b)))
    lo, hi = np.log(L_range[0] * scale), np.log(L_range[1] * scale)
    L = max(1, int(round(np.exp(g.uniform(lo, hi)))))
    n = int(round(np.exp(g.uniform(np.log(n_range[0]), np.log(n_range[1])))))
    t = 1 + (b % periods)
    return make_instance(L, n, size_lo=5, size_hi=50, zipf=1.1, cap_lo=0.2,
                         cap_hi=0.5, cap_scale=t / periods,
                         seed=base_seed + b, name=f"batch{b}-t{t}of{periods}")


def tiny_instance(L: int, n: int, *, m: Optional[int] = None, size_lo=1,
                  size_hi=None, seed=0, **kw) -> Instance:
    """Small instance for brute-force and LP checks."""
    return make_instance(L, n, m=m, size_lo=size_lo,
                         size_hi=n if size_hi is None else size_hi, seed=seed,
                         **kw)


def shuffle_products(inst: Instance, seed: int = 0):
    """The same instance with its products renumbered by a random permutation
    pi (product j becomes pi[j]; rows re-sorted by the new ids; r, the
    consumption columns of A, and for A = I the capacities move with their
    product).  Returns (instance, pi).  Generated instances number products
    by popularity; this one does not."""
    rng = np.random.default_rng(seed)
    pi = rng.permutation(inst.n).astype(np.int32)
    new = pi[inst.idx]
    order = np.lexsort((new, _row_ids(inst.seg_ptr)))
    r = np.empty_like(inst.r)
    r[pi] = inst.r
    kw = {}
    if inst.identity:
        c = np.empty_like(inst.c)
        c[pi] = inst.c
        kw["c"] = c
    else:
        old = np.argsort(pi)                      # old id of each new id
        cnt = np.diff(inst.a_ptr)[old]
        a_ptr = np.zeros(inst.n + 1, dtype=np.int64)
        np.cumsum(cnt, out=a_ptr[1:])
        take = np.concatenate([np.arange(inst.a_ptr[j], inst.a_ptr[j + 1]) for j in old]) \
            if inst.n else np.zeros(0, dtype=np.int64)
        kw.update(a_ptr=a_ptr, a_idx=inst.a_idx[take].copy(), a_val=inst.a_val[take].copy())
    out = dataclasses.replace(inst, idx=np.ascontiguousarray(new[order]),
                              v=np.ascontiguousarray(inst.v[order]),
                              w=np.ascontiguousarray(inst.w[order]), r=r,
                              name=(inst.name + "-shuffled") if inst.name else "shuffled", **kw)
    return out, pi


def minibatch_schedule(L: int, B: int, iters: int, seed: int = 0,
                       mode: str = "independent") -> np.ndarray:
    """Segments sampled by the stochastic minibatch iterations: [iters, B]
    int32, distinct within a row.  independent: each row a uniform B-subset
    of [L] drawn afresh; epoch: consecutive rows walk through random
    permutations of [L] (every segment once per L / B rows)."""
    if not 0 < B <= L:
        raise ValueError("need 0 < B <= L")
    rng = np.random.default_rng(seed)
    out = np.empty((iters, B), dtype=np.int32)
    if mode == "independent":
        for t in range(iters):
            out[t] = rng.choice(L, B, replace=False)
    elif mode == "epoch":
        perm, pos = rng.permutation(L), 0
        for t in range(iters):
            if pos + B > L:
                perm, pos = rng.permutation(L), 0
            out[t] = perm[pos:pos + B]
            pos += B
    else:
        raise ValueError(mode)
    return out


def step_scale(inst: Instance, tau0: float) -> np.ndarray:
    """Per-row dual step tau_i = tau0 * max_j r_j / c_i: revenue units per unit
    of capacity, so tau0 is dimensionless.  Rows with c_i = 0 get the step of
    the smallest positive capacity."""
    c = np.asarray(inst.c, dtype=np.float64)
    pos = c > 0
    cmin = c[pos].min() if pos.any() else 1.0
    return tau0 * float(np.max(inst.r)) / np.where(pos, c, cmin)


@dataclasses.dataclass
class Market:
    """Inputs of the bid-price policy simulation (Section 5.1, the synthetic
    market of Figure 4) for ``runs`` independent runs: prices r [runs, n],
    initial inventories inv0 [runs, n] (int64), each batch's customer
    preferences prefs [periods, runs, N, n] and the uniforms u [periods,
    runs, N] that decide the customers' choices."""
    r: np.ndarray
    inv0: np.ndarray
    prefs: np.ndarray
    u: np.ndarray

    @property
    def periods(self) -> int:
        return int(self.prefs.shape[0])

    @property
    def runs(self) -> int:
        return int(self.r.shape[0])

    @property
    def customers(self) -> int:
        return int(self.prefs.shape[2])

    @property
    def n(self) -> int:
        return int(self.r.shape[1])

    def cast(self, dtype) -> "Market":
        dt = np.dtype(dtype)
        return dataclasses.replace(self, r=np.ascontiguousarray(self.r, dtype=dt),
                                   prefs=np.ascontiguousarray(self.prefs, dtype=dt))


def gosim_market(runs: int = 30, *, n: int = 40, periods: int = 100, customers: int = 1000,
                 price_lo: float = 1.0, price_hi: float = 20.0, inv_lo: int = 1,
                 inv_hi: int = 2000, seed: int = 0, dtype=np.float64) -> Market:
    """The market of Figure 4: prices U[price_lo, price_hi], integer initial
    inventories U{inv_lo..inv_hi}, every customer's preference for every
    product U(0, 1] (strictly positive: it is an attraction), fresh customers
    in every batch, and one U[0, 1) choice draw per customer."""
    ss = np.random.SeedSequence(seed)
    g_r, g_inv, g_pref, g_u = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(4)]
    r = g_r.uniform(price_lo, price_hi, size=(runs, n))
    inv0 = g_inv.integers(inv_lo, inv_hi + 1, size=(runs, n), dtype=np.int64)
    prefs = np.empty((periods, runs, customers, n), dtype=np.dtype(dtype))
    for t in range(periods):
        prefs[t] = 1.0 - g_pref.random((runs, customers, n))
    u = g_u.random((periods, runs, customers))
    return Market(r=np.ascontiguousarray(r, dtype=np.dtype(dtype)), inv0=inv0, prefs=prefs, u=u)


def market_instance(prefs: np.ndarray, r: np.ndarray, c: np.ndarray, name: str = "") -> Instance:
    """One batch's choice-based LP: every customer a segment of arrival rate 1
    whose consideration set is every product (rows in product order),
    nominal attraction = the customer's preference, no shadow attraction
    (the basic attraction model), no-purchase attraction 1, capacities c."""
    N, n = prefs.shape
    dt = prefs.dtype
    return Instance(L=N, n=n, m=n, seg_ptr=np.arange(N + 1, dtype=np.int64) * n,
                    idx=np.tile(np.arange(n, dtype=np.int32), N),
                    v=np.ascontiguousarray(prefs.ravel()), w=np.zeros(N * n, dtype=dt),
                    v0=np.ones(N, dtype=dt), lam=np.ones(N, dtype=dt),
                    r=np.ascontiguousarray(r, dtype=dt), c=np.ascontiguousarray(c, dtype=dt),
                    name=name)
