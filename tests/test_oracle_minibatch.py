"""Pins of the oracle's stochastic minibatch SPFOM (Algorithm 2; Algorithm 3
with k B < L) and of the decaying constant step (CPU only).

* B = L re-solves every segment in every iteration: the full-batch
  iteration, bit for bit;
* a hand-worked two-segment example with B = 1, where the dual step uses a
  segment's stale sales;
* every segment's kept sales are its best response at the duals of the last
  iteration that sampled it, and the product sales are their sums;
* the step multiplier of the decaying schedule, worked by hand.
"""
import numpy as np
import pytest

import oracle
from paper_2602_22421_amd.instances import (config_instance, make_instance, minibatch_schedule,
                                            step_scale)


def test_full_minibatch_is_the_full_batch():
    inst = config_instance(0)
    tau = step_scale(inst, 0.002)
    full = oracle.Solver(inst, tau=tau, mu=0.01, check_every=10)
    eta_f, tr_f = full.iterate(np.zeros(inst.m), 30)
    mb = oracle.Minibatch(inst, tau=tau, mu=0.01)
    # every segment in every iteration, in a different order each time
    batch = minibatch_schedule(inst.L, inst.L, 30, seed=3)
    eta_m, tr_m = mb.iterate(np.zeros(inst.m), batch)
    assert np.array_equal(eta_m, eta_f)
    # revenue: the same sum, taken by product here and by segment there
    np.testing.assert_allclose(tr_m[:, 1], tr_f[:, 1], rtol=1e-13)
    assert np.array_equal(tr_m[:, 3], tr_f[:, 3])          # ||eta||^2
    assert np.array_equal(tr_m[:, 4], tr_f[:, 4])          # infeasibility


def _two_segments():
    inst = make_instance(2, 2, size_lo=1, size_hi=1, seed=0)
    inst.seg_ptr[:] = [0, 1, 2]
    inst.idx[:] = [0, 1]
    inst.v[:] = 1.0
    inst.w[:] = 0.0
    inst.v0[:] = 1.0
    inst.lam[:] = 1.0
    inst.r[:] = [10.0, 4.0]
    inst.c[:] = [0.25, 1.0]
    return inst


def test_minibatch_hand_worked():
    """Segment 0 considers product 0 (r=10, c=0.25), segment 1 product 1
    (r=4, c=1); v=1, w=0, v0=1, lambda=1; tau=0.5; B=1, sampling 0, 1, 0.
    Whenever a segment is solved it offers its product (its reduced revenue
    stays positive) and sells 1/(1+1) = 1/2.
      t=1: y0 = 1/2, y1 = 0 (not solved yet): S = (1/2, 0);
           eta = (0 + 0.5 (1/2 - 1/4), max(0, 0.5 (0 - 1))) = (1/8, 0);
           P = 10/2 = 5; infeas = (1/4) / (5/4) = 1/5
      t=2: y1 = 1/2 (y0 kept): S = (1/2, 1/2); eta = (1/4, 0); P = 7
      t=3: y0 = 1/2 again: eta = (3/8, 0); P = 7"""
    inst = _two_segments()
    mb = oracle.Minibatch(inst, tau=np.array([0.5, 0.5]))
    batch = np.array([[0], [1], [0]])
    eta = np.zeros(2)
    etas = []
    for t in range(3):
        eta, tr = mb.iterate(eta, batch[t:t + 1])
        etas.append(eta.copy())
        assert tr[0, 8] == 1.0 and tr[0, 0] == 0.0
        assert tr[0, 1] == pytest.approx([5.0, 7.0, 7.0][t], rel=1e-15)
        assert tr[0, 4] == pytest.approx(0.2, rel=1e-14)
    np.testing.assert_allclose(etas, [[1 / 8, 0], [1 / 4, 0], [3 / 8, 0]], rtol=1e-15)
    np.testing.assert_allclose(mb.y, [0.5, 0.5], rtol=1e-15)


def test_kept_sales_are_last_best_responses():
    inst = make_instance(300, 40, size_lo=2, size_hi=9, zipf=1.1, seed=5, cap_lo=0.3)
    tau = step_scale(inst, 0.01)
    B, T = 37, 25
    batch = minibatch_schedule(inst.L, B, T, seed=9)
    mb = oracle.Minibatch(inst, tau=tau)
    eta = np.zeros(inst.m)
    last_eta = {}
    for t in range(T):
        for l in batch[t]:
            last_eta[int(l)] = eta.copy()          # the duals it is solved at
        eta, tr = mb.iterate(eta, batch[t:t + 1])
    S = np.zeros(inst.n)
    for l in range(inst.L):
        b, e = inst.seg_ptr[l], inst.seg_ptr[l + 1]
        if l in last_eta:
            rho = inst.r - last_eta[l]
            _, _, s = oracle.segment_response(rho[inst.idx[b:e]], inst.v[b:e], inst.w[b:e],
                                              inst.v0[l], inst.lam[l])
            np.testing.assert_allclose(mb.y[b:e], s, rtol=0, atol=0)
        else:
            assert not mb.y[b:e].any()              # never sampled: y^0 = 0
        np.add.at(S, inst.idx[b:e], mb.y[b:e])
    # the last iteration's revenue is that of the kept sales
    assert tr[-1, 1] == pytest.approx(float(np.dot(inst.r, S)), rel=1e-12)


def test_decaying_step_hand_worked():
    """One product (v=2, w=0.5, v0=1, lambda=1, r=10, c=0.2: sales 2/3 at any
    duals below r), tau=0.3, tau_decay=0.5 every 2 iterations: multipliers
    1, 1, 1/2, 1/2, 1/4; each step adds tau * mult * (2/3 - 0.2)."""
    inst = make_instance(1, 1, size_lo=1, size_hi=1, seed=0)
    inst.v[:] = 2.0
    inst.w[:] = 0.5
    inst.v0[:] = 1.0
    inst.lam[:] = 1.0
    inst.r[:] = 10.0
    inst.c[:] = 0.2
    s = oracle.Solver(inst, tau=np.array([0.3]), tau_decay=0.5, decay_every=2)
    eta, tr = s.iterate(np.zeros(1), 5)
    mult = np.array([1, 1, 0.5, 0.5, 0.25])
    np.testing.assert_array_equal(tr[:, 8], mult)
    g = 2.0 / 3.0 - 0.2
    assert eta[0] == pytest.approx(0.3 * g * mult.sum(), rel=1e-14)
