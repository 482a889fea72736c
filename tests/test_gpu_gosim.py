"""The GO bid-price policy simulation (Section 5.1, Figure 4 market) and the
entry points it rests on, through the C ABI:

* cblp_refresh (new attractions and capacities on the structure of creation)
  gives the handle a fresh cblp_create of the new values would give, bit
  for bit, on every kernel layout (three-part FP32, 8-lane FP64);
* cblp_batch_mask: instances outside the mask keep their duals, the rest
  move exactly as without the mask;
* gosim_lp_inputs and gosim_period against the oracle's functions on the
  same inputs: exact (capacities, steps, offers, sales, stock, revenue);
* gosim_run in FP64 against the oracle's closed-loop simulation: the same
  offers, sales, revenue and LP iteration counts in every batch and run;
  in FP32 against the composition of its own steps and the invariants.
"""
import numpy as np
import pytest

import oracle
from oracle import gosim as ogs
from paper_2602_22421_amd.instances import (config_instance, gosim_market, make_instance,
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


def _revalued(inst, seed):
    """The same structure with new attractions and capacities."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.5, 2.0, inst.nnz)
    w = rng.uniform(0.0, 0.5, inst.nnz) * v
    c = inst.c * rng.uniform(0.5, 1.5, inst.m)
    import dataclasses
    return dataclasses.replace(inst, v=v, w=w, c=c)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_refresh_equals_fresh_handle(cb, dtype):
    dt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    a = config_instance(1, scale=0.01).cast(npdt)        # rows of 5..50: all three parts
    b = _revalued(a, 7).cast(npdt)
    pa = cb.Problem(a, dtype=dt)
    pb = cb.Problem(b, dtype=dt)
    eta0 = pa.tensor(np.random.default_rng(1).uniform(0, 0.5, a.m) * a.r)
    pa.refresh(v=b.v, w=b.w, c=b.c)
    Sa, ua, Ra = pa.sales(eta0, seg_R=True)
    Sb, ub, Rb = pb.sales(eta0, seg_R=True)
    assert torch.equal(Sa, Sb) and torch.equal(ua, ub) and torch.equal(Ra, Rb)
    tau = pa.tensor(step_scale(b, 0.002).astype(npdt))
    prm = cb.make_params(rule=0, tau_vec=tau, check_every=5)
    ea, eb = pa.zeros_eta(), pb.zeros_eta()
    ta, _ = pa.iterate(ea, 12, prm)
    tb, _ = pb.iterate(eb, 12, prm)
    assert torch.equal(ea, eb)
    assert np.array_equal(ta, tb)
    pa.close()
    pb.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_minibatch_after_refresh_equals_fresh_handle(cb, dtype):
    """A refresh restarts the minibatch state and rebuilds the minibatch
    kernel's per-segment records (v_t0 follows the new w): minibatch
    iterations after it equal those of a handle made from the new values."""
    from paper_2602_22421_amd.instances import minibatch_schedule
    dt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    a = config_instance(1, scale=0.01).cast(npdt)
    b = _revalued(a, 9).cast(npdt)
    pa = cb.Problem(a, dtype=dt)
    pb = cb.Problem(b, dtype=dt)
    tau = pa.tensor(step_scale(b, 0.002).astype(npdt))
    prm = cb.make_params(rule=0, tau_vec=tau)
    batch = minibatch_schedule(a.L, a.L // 10, 12, seed=3, mode="epoch")
    pa.minibatch(pa.zeros_eta(), batch[:4], prm)   # records of the old values
    pa.refresh(v=b.v, w=b.w, c=b.c)
    ea, eb = pa.zeros_eta(), pb.zeros_eta()
    ta = pa.minibatch(ea, batch, prm)
    tb = pb.minibatch(eb, batch, prm)
    assert torch.equal(ea, eb)
    assert np.array_equal(ta, tb)
    pa.close()
    pb.close()


def test_refresh_rejects_invalid_values(cb):
    a = make_instance(50, 8, seed=3)
    p = cb.Problem(a, dtype=torch.float64)
    w = a.w.copy()
    w[5] = a.v[5]                    # w must stay below v
    with pytest.raises(cb.CblpError) as e:
        p.refresh(w=w)
    assert e.value.code == cb.CBLP_EINVAL and "shadow" in str(e.value)
    c = a.c.copy()
    c[2] = -1.0
    with pytest.raises(cb.CblpError):
        p.refresh(w=a.w, c=c)
    p.refresh(c=a.c)                 # valid again
    p.close()


def test_batch_mask_keeps_masked_duals(cb):
    insts = [make_instance(300 + 50 * q, 20, size_hi=12, seed=q, cap_lo=0.3) for q in range(3)]
    probs = [cb.Problem(i, dtype=torch.float64) for i in insts]
    taus = [p.tensor(step_scale(i, 0.002)) for p, i in zip(probs, insts)]
    ref = []
    for p, t in zip(probs, taus):
        e = p.zeros_eta()
        p.iterate(e, 8, cb.make_params(rule=0, tau_vec=t, check_every=4))
        ref.append(e.cpu().numpy())
    probs2 = [cb.Problem(i, dtype=torch.float64) for i in insts]
    batch = cb.Batch(probs2)
    batch.mask([1, 0, 1])
    start = probs2[1].tensor(np.full(insts[1].m, 0.25))
    etas = [probs2[0].zeros_eta(), start.clone(), probs2[2].zeros_eta()]
    params = cb.make_params(rule=0, tau=1.0, check_every=4)
    batch.iterate(etas, 8, params, tau_vecs=taus)
    assert np.array_equal(etas[0].cpu().numpy(), ref[0])
    assert torch.equal(etas[1], start)
    assert np.array_equal(etas[2].cpu().numpy(), ref[2])
    out = batch.solve(etas, cb.make_params(rule=0, tau=1.0, check_every=4, tol=1e-9,
                                           max_iters=8), tau_vecs=taus)
    assert out[1]["iters"] == 0 and out[1]["status"] == cb.CBLP_OK
    assert out[0]["iters"] == 8 and out[2]["iters"] == 8
    assert torch.equal(etas[1], start)
    batch.mask(None)
    batch.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_lp_inputs_match_oracle(cb, dtype):
    dt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    rng = np.random.default_rng(4)
    runs, n = 5, 37
    inv = rng.integers(0, 2000, size=(runs, n)).astype(np.int64)
    inv[0, :5] = 0
    inv[3] = 0                                   # no capacity at all
    r = rng.uniform(1, 20, (runs, n)).astype(npdt)
    dev = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", t)
    c = torch.empty(runs, n, dtype=dt, device="cuda")
    tau = torch.empty_like(c)
    eta0 = (rng.uniform(0, 1.5, (runs, n)) * r).astype(npdt)   # some above r already
    for left in (1, 7, 100):
        eta = dev(eta0, dt)
        cb.gosim_lp_inputs(dev(inv, torch.int64), left, 0.003, dev(r, dt), c, tau, eta)
        torch.cuda.synchronize()
        for q in range(runs):
            c_ref, tau_ref = ogs.lp_inputs(inv[q], left, r[q], 0.003, npdt)
            assert np.array_equal(c[q].cpu().numpy(), c_ref), (left, q)
            assert np.array_equal(tau[q].cpu().numpy(), tau_ref), (left, q)
            eta_ref = ogs.sold_out_duals(inv[q], eta0[q], r[q]).astype(npdt)
            assert np.array_equal(eta[q].cpu().numpy(), eta_ref), (left, q)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("K", [1, 2, 3])
def test_period_matches_oracle(cb, dtype, K):
    dt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    mk = gosim_market(6, n=12, periods=1, customers=300, inv_hi=25, seed=K).cast(npdt)
    rng = np.random.default_rng(10 + K)
    inv = mk.inv0.copy()
    inv[1, 3:] = 0                               # run 1: three products left
    inv[2, :] = 0
    inv[2, 4] = 2                                # run 2: one product left
    eta = (rng.uniform(0, 1.3, (6, 12)) * mk.r).astype(npdt)   # some margins negative
    eta[4] = mk.r[4]                             # run 4: every margin exactly zero
    eta[5] = mk.r[5] + 1                         # run 5: every margin negative
    dev = lambda a, t: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", t)
    inv_d = dev(inv, torch.int64)
    offer = torch.empty(6, K, dtype=torch.int32, device="cuda")
    sales = torch.empty(6, 12, dtype=torch.int64, device="cuda")
    rev = torch.empty(6, dtype=torch.float64, device="cuda")
    stock = torch.empty(6, dtype=torch.int32, device="cuda")
    cb.gosim_period(K, dev(eta, dt), dev(mk.r, dt), dev(mk.prefs[0], dt), dev(mk.u[0], torch.float64),
                    inv_d, offer, sales, rev, stock)
    torch.cuda.synchronize()
    for q in range(6):
        S, s_ref, inv_ref, rev_ref = ogs.period(inv[q], eta[q], mk.r[q], mk.prefs[0, q], mk.u[0, q], K)
        got = [j for j in offer[q].cpu().numpy().tolist() if j >= 0]
        assert got == S, (q, got, S)
        assert np.array_equal(sales[q].cpu().numpy(), s_ref), q
        assert np.array_equal(inv_d[q].cpu().numpy(), inv_ref), q
        assert rev[q].item() == rev_ref, q
        assert stock[q].item() == int(np.count_nonzero(inv_ref > 0))
    assert np.all(sales.cpu().numpy()[5] == 0) and rev[5].item() == 0.0


def _params(cb, tol, max_iters, check):
    return cb.make_params(rule=0, tau=1.0, check_every=check, tol=tol, max_iters=max_iters)


def test_run_matches_oracle_f64(cb):
    mk = gosim_market(3, n=10, periods=5, customers=150, inv_hi=60, seed=11)
    sim = cb.GoSim(mk, dtype=torch.float64)
    K, tau0, tol, mx, ce = 2, 0.05, 1e-2, 200, 10
    out = sim.run(K, _params(cb, tol, mx, ce), tau0)
    for q in range(3):
        ref = ogs.simulate(mk.r[q], mk.inv0[q], mk.prefs[:, q], mk.u[:, q], K, tau0=tau0, tol=tol,
                           max_iters=mx, check_every=ce)
        assert np.array_equal(out["lp_iters"][:, q], ref["iters"]), q
        np.testing.assert_allclose(out["lp_gap"][:, q], ref["gap"], rtol=1e-9, atol=1e-12)
        for t in range(5):
            got = [j for j in out["offers"][t, q].tolist() if j >= 0]
            assert got == ref["offers"][t], (q, t)
        assert np.array_equal(out["sales"][:, q], ref["sales"]), q
        assert np.array_equal(out["revenue"][:, q], ref["revenue"]), q
        assert np.array_equal(out["inv"][q].cpu().numpy(), ref["inv"][-1]), q
        # the duals carried to the end agree with the oracle's to FP64 rounding
        np.testing.assert_allclose(out["eta"][q].cpu().numpy(), ref["eta"][-1], rtol=1e-9,
                                   atol=1e-9 * float(np.max(mk.r[q])))
    assert np.any(out["lp_iters"] > 0)
    sim.close()


def test_run_f32_is_its_steps(cb):
    """gosim_run in FP32 equals the composition of its steps driven from
    Python (lp inputs, refresh, one handle's solve, period), and keeps the
    simulation's invariants."""
    mk = gosim_market(2, n=9, periods=4, customers=120, inv_hi=50, seed=12).cast(np.float32)
    K, tau0, tol, mx, ce = 2, 0.05, 1e-2, 150, 10
    sim = cb.GoSim(mk, dtype=torch.float32)
    out = sim.run(K, _params(cb, tol, mx, ce), tau0)
    sim.close()
    for q in range(2):
        inst_v = mk.prefs[0, q]
        from paper_2602_22421_amd.instances import market_instance
        prob = cb.Problem(market_instance(inst_v, mk.r[q], np.zeros(9, np.float32)),
                          dtype=torch.float32)
        inv = torch.from_numpy(mk.inv0[q:q + 1].copy()).cuda()
        eta = prob.zeros_eta()
        tau = torch.empty(1, 9, dtype=torch.float32, device="cuda")
        c = torch.empty(1, 9, dtype=torch.float32, device="cuda")
        r = prob.r.view(1, 9)
        for t in range(4):
            stock = int((inv > 0).sum().item())
            cb.gosim_lp_inputs(inv, 4 - t, tau0, r, c, tau, eta.view(1, 9))
            iters = 0
            if stock > K:
                prob.refresh(v=mk.prefs[t, q].ravel(), c=c[0])
                prm = cb.make_params(rule=0, tau_vec=tau[0], check_every=ce, tol=tol, max_iters=mx)
                iters = prob.solve(eta, prm).iters
            assert iters == out["lp_iters"][t, q], (q, t)
            offer = torch.empty(1, K, dtype=torch.int32, device="cuda")
            sales = torch.empty(1, 9, dtype=torch.int64, device="cuda")
            rev = torch.empty(1, dtype=torch.float64, device="cuda")
            cb.gosim_period(K, eta.view(1, 9), r, torch.from_numpy(mk.prefs[t, q:q + 1]).cuda(),
                            torch.from_numpy(mk.u[t, q:q + 1]).cuda(), inv, offer, sales, rev)
            assert np.array_equal(offer[0].cpu().numpy(), out["offers"][t, q]), (q, t)
            assert np.array_equal(sales[0].cpu().numpy(), out["sales"][t, q]), (q, t)
            assert rev.item() == out["revenue"][t, q]
        prob.close()
    sold = out["sales"].sum(axis=0)
    assert np.all(sold <= mk.inv0) and np.all(out["sales"] >= 0)


def test_run_rejects_a_sparse_handle(cb):
    insts = [make_instance(40, 6, size_lo=2, size_hi=4, seed=q) for q in range(2)]
    probs = [cb.Problem(i, dtype=torch.float64) for i in insts]
    batch = cb.Batch(probs)
    T, R, N, n = 1, 2, 40, 6
    prefs = torch.ones(T, R, N, n, dtype=torch.float64, device="cuda")
    u = torch.zeros(T, R, N, dtype=torch.float64, device="cuda")
    r = torch.ones(R, n, dtype=torch.float64, device="cuda")
    inv = torch.ones(R, n, dtype=torch.int64, device="cuda")
    eta = torch.zeros(R, n, dtype=torch.float64, device="cuda")
    tau = torch.ones(R, n, dtype=torch.float64, device="cuda")
    with pytest.raises(cb.CblpError) as e:
        cb.gosim_run(batch.b, T, 2, prefs, u, r, inv, eta, tau, _params(cb, 1e-2, 10, 10), 0.1,
                     torch.empty(T, R, 2, dtype=torch.int32, device="cuda"),
                     torch.empty(T, R, n, dtype=torch.int64, device="cuda"),
                     torch.empty(T, R, dtype=torch.float64, device="cuda"))
    assert e.value.code == cb.CBLP_EINVAL
    batch.close()
