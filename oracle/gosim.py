"""FP64 CPU reference of the bid-price policy simulation (test infrastructure only).

Only the tests and the benchmark's CPU leg use this module; the solver library
never imports or runs it.  It restates, in plain Python and numpy, the global
optimisation (GO) policy of Section 5.1 on the synthetic market of Figure 4:
in every batch, products with no inventory leave the offer; if at most K
remain they are all offered, otherwise the batch's sales-based LP is solved
by SPFOM (``oracle.Solver``) and the bid-price rule offers the products whose
revenue is at least their capacity dual; the batch's customers then choose
under the basic attraction model and the inventory falls by what they buy.

Readings where the paper is silent (each is listed with the build's other
readings):

* the LP of batch t (of T) has the batch's own customers as segments and
  capacities inv / (T - t + 1): the multi-period LP of Section 5.1 with the
  remaining batches drawn like the current one splits into that many equal
  copies of it (pinned with an LP solver in the tests);
* the recommendation limit K holds per batch: when more than K products pass
  the bid-price rule, the K of largest margin r_j - eta_j are offered (ties
  to the lower product index);
* a customer's choice is decided by one uniform u: with W = 1 + the sum of
  the offered preferences (no-purchase attraction 1), the customer buys the
  first offered product (ascending index) whose running preference sum
  exceeds u W, or nothing;
* customers of a batch choose independently of one another; a product sells
  min(demand, inventory) units (the later customers of a sold-out product go
  without);
* the LP of each batch starts from the previous batch's duals (zero in the
  first), with the solver state reset; a product out of stock leaves that LP
  by a dual raised to its revenue (no assortment then holds it, which is the
  LP with the product removed).
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_2602_22421_amd.instances import market_instance


def lp_inputs(inv, periods_left: int, r, tau0: float, dtype=np.float64):
    """Capacities c_j = inv_j / periods_left of the current batch's LP and the
    per-row dual step tau_j = tau0 max_k r_k / c_j (a product without
    capacity takes the step of the smallest positive capacity, or of
    capacity 1 if there is none), each rounded once to ``dtype`` (the step
    from the rounded capacities)."""
    dt = np.dtype(dtype)
    c = (np.asarray(inv, dtype=np.float64) / float(periods_left)).astype(dt)
    cd = c.astype(np.float64)
    pos = cd > 0
    cmin = cd[pos].min() if pos.any() else 1.0
    rmax = float(np.max(np.asarray(r, dtype=np.float64)))
    tau = (tau0 * rmax / np.where(pos, cd, cmin)).astype(dt)
    return c, tau


def sold_out_duals(inv, eta, r):
    """The LP without the products out of stock: each such product's dual is
    raised to at least its revenue, so its margin r_j - eta_j <= 0 keeps it
    out of every segment's best response (zero sales at zero capacity) and
    c_j eta_j = 0 adds nothing to the dual value."""
    eta = np.array(eta, dtype=np.float64, copy=True)
    r = np.asarray(r, dtype=np.float64)
    out = np.asarray(inv) == 0
    eta[out] = np.maximum(eta[out], r[out])
    return eta


def offer(inv, eta, r, K: int):
    """Offered products of a batch, ascending: every product in stock if at
    most K are; else the bid-price rule (margin r_j - eta_j >= 0) cut to the
    K largest margins."""
    n = len(inv)
    avail = [j for j in range(n) if inv[j] > 0]
    if len(avail) <= K:
        return avail
    margin = {j: float(r[j]) - float(eta[j]) for j in avail}
    cand = [j for j in avail if margin[j] >= 0.0]
    cand.sort(key=lambda j: (-margin[j], j))
    return sorted(cand[:K])


def choose(pref_row, u: float, S):
    """The product one customer buys from the offered set S (ascending), or
    -1: the basic attraction model with no-purchase attraction 1, decided by
    the uniform u."""
    W = 1.0
    for j in S:
        W += float(pref_row[j])
    x = float(u) * W
    cum = 0.0
    for j in S:
        cum += float(pref_row[j])
        if x < cum:
            return j
    return -1


def period(inv, eta, r, prefs, u, K: int):
    """One batch: offer, choices, sales and the inventory left.  Returns
    (offered set, sales [n] int64, inventory [n] int64, revenue)."""
    inv = np.asarray(inv, dtype=np.int64)
    S = offer(inv, eta, r, K)
    counts = np.zeros(inv.shape[0], dtype=np.int64)
    for i in range(prefs.shape[0]):
        j = choose(prefs[i], u[i], S)
        if j >= 0:
            counts[j] += 1
    sales = np.minimum(counts, inv)
    rev = 0.0
    for j in S:
        rev += float(r[j]) * float(sales[j])
    return S, sales, inv - sales, rev


def simulate(r, inv0, prefs, u, K: int, *, tau0: float, tol: float, max_iters: int,
             check_every: int = 10, tau_decay: float = 1.0, decay_every: int = 1,
             rule: int = oracle.RULE_CONST, gamma: float = 1.0, eta0=None, batches=None):
    """The GO policy over the batches of one run.  prefs [T, N, n], u [T, N];
    ``batches`` stops after that many of the T batches (the horizon stays T).
    Returns a dict of per-batch offers, sales, revenue, inventory after the
    batch, LP iterations and last certified gap (0 where the LP was not
    solved) and the duals used."""
    T, N, n = prefs.shape
    inv = np.asarray(inv0, dtype=np.int64).copy()
    eta = np.zeros(n) if eta0 is None else np.array(eta0, dtype=np.float64)
    out = dict(offers=[], sales=np.zeros((T, n), dtype=np.int64), revenue=np.zeros(T),
               inv=np.zeros((T, n), dtype=np.int64), iters=np.zeros(T, dtype=np.int64),
               gap=np.zeros(T), eta=np.zeros((T, n)))
    for t in range(T if batches is None else min(T, int(batches))):
        if int(np.count_nonzero(inv > 0)) > K:
            c, tau = lp_inputs(inv, T - t, r, tau0, prefs.dtype)
            eta = sold_out_duals(inv, eta, r)
            inst = market_instance(np.asarray(prefs[t]), np.asarray(r), c)
            s = oracle.Solver(inst, tau=tau, rule=rule, gamma=gamma, check_every=check_every,
                              tau_decay=tau_decay, decay_every=decay_every)
            eta, last, _ = s.solve(eta, tol, max_iters)
            out["iters"][t] = s.t
            out["gap"][t] = last[7] if last is not None else 0.0
        S, sales, inv, rev = period(inv, eta, r, prefs[t], u[t], K)
        out["offers"].append(S)
        out["sales"][t] = sales
        out["revenue"][t] = rev
        out["inv"][t] = inv
        out["eta"][t] = eta
    return out
