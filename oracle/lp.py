"""The two LPs of Section 3 written out for an independent LP solver (HiGHS).

Test infrastructure: these pin the oracle's dual bound and limit, they are
not part of any solver path.

* ``cblp``: the choice-based LP (eqs. 1-4) with every assortment of every
  consideration set enumerated as a column, GAM choice probabilities
  (Section 3), a resource matrix A in the capacity rows (eq. 26 of
  Section 5.2; A = I gives eq. 2).  Exponential; tiny instances only.
* ``sblp``: the sales-based LP in its GAM form.  The paper writes eqs. 5-9
  for MNL only.  With vt_l0 = v_l0 + sum_{N_l} w and vt_lj = v_lj - w_lj, the
  GAM sales s_lj = sum_S x_l(S) pi_lj(S) satisfy the balance
  (vt_l0/v_l0) s_l0 + sum_j (vt_lj/v_lj) s_lj = lambda_l and the scale
  constraints s_lj / v_lj <= s_l0 / v_l0; with w = 0 this is eqs. 6-8.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog


def _resource_rows(inst):
    """Dense-free view of A as (resource, product, value) triplets."""
    if inst.a_ptr is None:
        j = np.arange(inst.n)
        return j, j, np.ones(inst.n)
    cnt = np.diff(inst.a_ptr)
    prod = np.repeat(np.arange(inst.n), cnt)
    return np.asarray(inst.a_idx), prod, np.asarray(inst.a_val, dtype=np.float64)


def _amat(inst):
    ri, pj, av = _resource_rows(inst)
    return sp.csr_matrix((av, (ri, pj)), shape=(inst.m, inst.n))


def cblp(inst):
    """Solve the enumerated CBLP.  Returns (OPT, capacity duals eta*[m])."""
    A = _amat(inst).toarray()
    cols_obj, cap_rows, bal_rows = [], [], []
    col = 0
    for l in range(inst.L):
        b, e = int(inst.seg_ptr[l]), int(inst.seg_ptr[l + 1])
        prods = np.asarray(inst.idx[b:e])
        v = np.asarray(inst.v[b:e], dtype=np.float64)
        w = np.asarray(inst.w[b:e], dtype=np.float64)
        v0 = float(inst.v0[l])
        k = e - b
        for mask in itertools.product((0, 1), repeat=k):
            inS = np.array(mask, dtype=bool)
            # GAM: products outside S still pull through their shadow attraction
            den = v0 + v[inS].sum() + w[~inS].sum()
            pi = np.where(inS, v / den, 0.0)
            cols_obj.append(float(np.dot(np.asarray(inst.r)[prods], pi)))
            use = np.zeros(inst.n)
            np.add.at(use, prods, pi)
            cap_rows.append(A @ use)
            bal_rows.append(l)
            col += 1
    c_obj = -np.array(cols_obj)
    A_ub = np.array(cap_rows).T if col else np.zeros((inst.m, 0))
    A_eq = sp.csr_matrix((np.ones(col), (bal_rows, np.arange(col))), shape=(inst.L, col))
    res = linprog(c_obj, A_ub=A_ub, b_ub=np.asarray(inst.c, dtype=np.float64), A_eq=A_eq,
                  b_eq=np.asarray(inst.lam, dtype=np.float64), bounds=(0, None),
                  method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    return -res.fun, -np.asarray(res.ineqlin.marginals)


def sblp(inst, return_sales: bool = False):
    """Solve the GAM sales-based LP.  Returns (OPT, capacity duals eta*[m]),
    and with return_sales also the optimal per-entry sales s_lj [nnz]."""
    L, nnz = int(inst.L), int(inst.seg_ptr[-1])
    sizes = np.diff(inst.seg_ptr)
    seg = np.repeat(np.arange(L), sizes)
    v = np.asarray(inst.v, dtype=np.float64)
    w = np.asarray(inst.w, dtype=np.float64)
    v0 = np.asarray(inst.v0, dtype=np.float64)
    vt0 = v0 + np.bincount(seg, weights=w, minlength=L)
    nv = nnz + L  # s_lj for every CSR entry, then s_l0 per segment
    cost = np.concatenate([-np.asarray(inst.r, dtype=np.float64)[inst.idx], np.zeros(L)])
    # capacity rows: u = A S with S_j = sum_l s_lj
    ri, pj, av = _resource_rows(inst)
    Aprod = sp.csr_matrix((np.ones(nnz), (np.asarray(inst.idx), np.arange(nnz))),
                          shape=(inst.n, nv))
    Acap = (_amat(inst) @ Aprod).tocsr()
    Abal = sp.csr_matrix((np.concatenate([(v - w) / v, vt0 / v0]),
                          (np.concatenate([seg, np.arange(L)]), np.arange(nv))),
                         shape=(L, nv))
    Asc = sp.csr_matrix((np.concatenate([1.0 / v, -1.0 / v0[seg]]),
                         (np.concatenate([np.arange(nnz), np.arange(nnz)]),
                          np.concatenate([np.arange(nnz), nnz + seg]))), shape=(nnz, nv))
    A_ub = sp.vstack([Acap, Asc]).tocsr()
    b_ub = np.concatenate([np.asarray(inst.c, dtype=np.float64), np.zeros(nnz)])
    res = linprog(cost, A_ub=A_ub, b_ub=b_ub, A_eq=Abal,
                  b_eq=np.asarray(inst.lam, dtype=np.float64), bounds=(0, None),
                  method="highs")
    if res.status != 0:
        raise RuntimeError(res.message)
    if return_sales:
        return -res.fun, -np.asarray(res.ineqlin.marginals[: inst.m]), np.asarray(res.x[:nnz])
    return -res.fun, -np.asarray(res.ineqlin.marginals[: inst.m])


def sblp_feasible(inst, sales, tol=1e-9):
    """Check best-response sales against the GAM balance and scale rows
    (capacity excluded).  Returns the max violation."""
    L = int(inst.L)
    sizes = np.diff(inst.seg_ptr)
    seg = np.repeat(np.arange(L), sizes)
    v = np.asarray(inst.v, dtype=np.float64)
    w = np.asarray(inst.w, dtype=np.float64)
    v0 = np.asarray(inst.v0, dtype=np.float64)
    lam = np.asarray(inst.lam, dtype=np.float64)
    vt0 = v0 + np.bincount(seg, weights=w, minlength=L)
    # s_l0 from the scale row at equality for the offered set: s_l0 = lambda v0 / D
    bal_prod = np.bincount(seg, weights=(v - w) / v * sales, minlength=L)
    # choose s_l0 making the balance exact, then check scale and sign
    s0 = (lam - bal_prod) * v0 / vt0
    viol_scale = np.max(sales / v - s0[seg] / v0[seg], initial=0.0)
    viol_sign = max(-np.min(s0, initial=0.0), -np.min(sales, initial=0.0))
    return max(viol_scale, viol_sign)
