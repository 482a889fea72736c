"""Batched re-solves (several instances advanced by one persistent launch per
iteration) against the same instances solved one at a time, and against the
FP64 oracle."""
import numpy as np
import pytest

import oracle
import oracle.lp as lp
from paper_2602_22421_amd.instances import batch_instance, make_instance, step_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_22421_amd import cblp
    cblp.load()
    return cblp


def _setup(cb, insts, dtype, tau0=0.002, rule=0):
    npdt = np.float32 if dtype == torch.float32 else np.float64
    insts = [i.cast(npdt) for i in insts]
    probs = [cb.Problem(i, dtype=dtype) for i in insts]
    taus = [p.tensor(step_scale(i, tau0 if rule == 0 else 1.0).astype(npdt))
            for p, i in zip(probs, insts)]
    return insts, probs, taus


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_iterate_matches_single(cb, dtype):
    dt = torch.float64 if dtype == "f64" else torch.float32
    base = [batch_instance(b, scale=0.004) for b in range(6)]
    assert len({i.L for i in base}) > 1 and len({i.n for i in base}) > 1
    insts, singles, taus = _setup(cb, base, dt)
    iters = 25
    eta_single = []
    rows_single = []
    for p, t in zip(singles, taus):
        params = cb.make_params(rule=0, tau_vec=t, check_every=5)
        eta = p.zeros_eta()
        tr, _ = p.iterate(eta, iters, params)
        eta_single.append(eta.cpu().numpy())
        rows_single.append(tr[-1])
    _, probs, taus2 = _setup(cb, base, dt)
    batch = cb.Batch(probs)
    etas = [p.zeros_eta() for p in probs]
    params = cb.make_params(rule=0, tau=1.0, check_every=5)
    rows = batch.iterate(etas, iters, params, tau_vecs=taus2)
    for q in range(len(base)):
        # constant steps: the duals depend only on exact integer sales sums;
        # Z is a fixed-point sum and the FP64 partials are folded in the
        # single path's grouping, so every trace column agrees bit for bit
        assert np.array_equal(etas[q].cpu().numpy(), eta_single[q]), q
        assert np.array_equal(rows[q], rows_single[q]), (q, rows[q], rows_single[q])
    batch.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_solve_certifies_as_single(cb, dtype):
    """spfom_batch_solve and spfom_solve stop every instance at the same
    check with the same last trace row, bit for bit."""
    dt = torch.float64 if dtype == "f64" else torch.float32
    base = [batch_instance(b, scale=0.004) for b in range(6)] + \
        [make_instance(800, 40, size_lo=3, size_hi=9, cap_lo=0.5, cap_hi=3.0, seed=s) for s in (1, 2)]
    _, singles, taus = _setup(cb, base, dt, tau0=0.01)
    single = []
    for p, t in zip(singles, taus):
        prm = cb.make_params(rule=0, tau_vec=t, check_every=10, tol=0.05, max_iters=400,
                             tau_decay=0.7, decay_every=100)
        single.append(p.solve(p.zeros_eta(), prm).as_dict())
    _, probs, taus2 = _setup(cb, base, dt, tau0=0.01)
    batch = cb.Batch(probs)
    params = cb.make_params(rule=0, tau=1.0, check_every=10, tol=0.05, max_iters=400,
                            tau_decay=0.7, decay_every=100)
    outs = batch.solve([p.zeros_eta() for p in probs], params, tau_vecs=taus2)
    for q, (o, r) in enumerate(zip(outs, single)):
        assert o["iters"] == r["iters"] and o["status"] == r["status"], (q, o, r)
        for k in cb.TRACE_COLS:
            assert o[k] == r[k], (q, k, o[k], r[k])
    batch.close()


def test_batch_vs_oracle_fp32(cb):
    base = [batch_instance(b, scale=0.004) for b in (1, 2, 3)]
    insts, probs, taus = _setup(cb, base, torch.float32, tau0=0.001)
    batch = cb.Batch(probs)
    etas = [p.zeros_eta() for p in probs]
    params = cb.make_params(rule=0, tau=1.0, check_every=10)
    rows = batch.iterate(etas, 20, params, tau_vecs=taus)
    for q, inst in enumerate(insts):
        s = oracle.Solver(inst, tau=taus[q].double().cpu().numpy(), check_every=10)
        eo, tr = s.iterate(np.zeros(inst.m), 20)
        eg = etas[q].double().cpu().numpy()
        assert np.linalg.norm(eg - eo) <= 1e-5 * max(np.linalg.norm(eo), 1e-12), q
        assert rows[q, 0] == pytest.approx(tr[-1, 0], rel=1e-5)
    batch.close()


def test_batch_solve_reaches_lp_optimum(cb):
    # seeds on which the oracle's Polyak run certifies 1e-4 within 2100 iterations
    base = [make_instance(1000, 50, size_lo=5, size_hi=10, cap_lo=0.3, seed=s) for s in (0, 2, 4, 5)]
    insts, probs, taus = _setup(cb, base, torch.float64, rule=1)
    batch = cb.Batch(probs)
    etas = [p.zeros_eta() for p in probs]
    params = cb.make_params(rule=1, tau=1.0, gamma=1.0, check_every=10, tol=1e-4,
                            max_iters=4000)
    outs = batch.solve(etas, params, tau_vecs=taus)
    for q, (inst, o) in enumerate(zip(insts, outs)):
        opt, _ = lp.sblp(inst)
        assert o["status"] == 0, (q, o)
        assert o["lb"] <= opt * (1 + 1e-12) and o["dbest"] >= opt * (1 - 1e-12), (q, o, opt)
        assert o["gap"] <= 1e-4
    # each instance stopped at its own check
    assert all(o["iters"] % 10 == 0 and o["iters"] <= 4000 for o in outs)
    batch.close()


def test_batch_graph_replays_match_eager(cb):
    """spfom_batch_solve replays a captured graph; the same iterations issued
    eagerly give the same duals."""
    base = [batch_instance(b, scale=0.004) for b in range(4)]
    insts, p1, t1 = _setup(cb, base, torch.float32, tau0=0.001)
    b1 = cb.Batch(p1)
    e1 = [p.zeros_eta() for p in p1]
    params = cb.make_params(rule=0, tau=1.0, check_every=10, tol=0.0, max_iters=40)
    b1.solve(e1, params, tau_vecs=t1)          # 4 graph replays of 10 iterations
    _, p2, t2 = _setup(cb, base, torch.float32, tau0=0.001)
    b2 = cb.Batch(p2)
    e2 = [p.zeros_eta() for p in p2]
    for _ in range(4):
        b2.iterate(e2, 10, params, tau_vecs=t2)
        torch.cuda.synchronize()
    for q in range(len(base)):
        assert np.array_equal(e1[q].cpu().numpy(), e2[q].cpu().numpy()), q
    b1.close()
    b2.close()


def test_batch_decaying_step_matches_single(cb):
    """The decaying constant step in a batch: each instance's duals equal its
    own spfom_iterate bit for bit (the same multiplier tau_decay^k, formed by
    repeated products, on exact integer sales sums)."""
    base = [batch_instance(b, scale=0.004) for b in range(4)]
    dt = torch.float32
    _, singles, taus = _setup(cb, base, dt, tau0=0.004)
    iters = 23
    ref, steps = [], []
    for p, t in zip(singles, taus):
        params = cb.make_params(rule=0, tau_vec=t, check_every=5, tau_decay=0.5, decay_every=7)
        eta = p.zeros_eta()
        tr, _ = p.iterate(eta, iters, params)
        ref.append(eta.cpu().numpy())
        steps.append(tr[:, 8])
    np.testing.assert_array_equal(steps[0][[0, 6, 7, 13, 14, 22]], [1, 1, 0.5, 0.5, 0.25, 0.125])
    _, probs, taus2 = _setup(cb, base, dt, tau0=0.004)
    batch = cb.Batch(probs)
    etas = [p.zeros_eta() for p in probs]
    params = cb.make_params(rule=0, tau=1.0, check_every=5, tau_decay=0.5, decay_every=7)
    rows = batch.iterate(etas, iters, params, tau_vecs=taus2)
    for q in range(len(base)):
        assert np.array_equal(etas[q].cpu().numpy(), ref[q]), q
        assert rows[q, 8] == 0.125
    batch.close()


def test_batch_graph_follows_step_parameters(cb):
    """A solve whose step parameters differ from the previous solve's (same
    check_every) captures a new graph: its duals equal eager iterations with
    the new parameters."""
    base = [batch_instance(b, scale=0.004) for b in range(3)]
    _, p1, t1 = _setup(cb, base, torch.float32, tau0=0.004)
    b1 = cb.Batch(p1)
    plain = cb.make_params(rule=0, tau=1.0, check_every=10, tol=0.0, max_iters=20)
    b1.solve([p.zeros_eta() for p in p1], plain, tau_vecs=t1)
    decay = cb.make_params(rule=0, tau=1.0, check_every=10, tol=0.0, max_iters=30,
                           tau_decay=0.5, decay_every=4)
    e1 = [p.zeros_eta() for p in p1]
    b1.solve(e1, decay, tau_vecs=t1)
    _, p2, t2 = _setup(cb, base, torch.float32, tau0=0.004)
    b2 = cb.Batch(p2)
    e2 = [p.zeros_eta() for p in p2]
    b2.iterate(e2, 30, decay, tau_vecs=t2)
    for q in range(len(base)):
        assert np.array_equal(e1[q].cpu().numpy(), e2[q].cpu().numpy()), q
    b1.close()
    b2.close()


def test_batch_tune_cache_and_items_per_block(cb, tmp_path):
    """The tuning cache: a miss tunes and appends one line, a hit applies the
    stored variant and items per block without tuning; with 16 items per
    block the batch still gives each instance's own duals and trace rows bit
    for bit (integer sales, fixed-point Z, the single path's fold grouping)."""
    base = [batch_instance(b, scale=0.004) for b in range(5)]
    _, singles, taus = _setup(cb, base, torch.float32, tau0=0.004)
    ref = []
    for p, t in zip(singles, taus):
        prm = cb.make_params(rule=0, tau_vec=t, check_every=5)
        e = p.zeros_eta()
        tr, _ = p.iterate(e, 15, prm)
        ref.append((e.cpu().numpy(), tr[-1]))
    cache = str(tmp_path / "tune.txt")
    _, probs, taus2 = _setup(cb, base, torch.float32, tau0=0.004)
    batch = cb.Batch(probs)
    params = cb.make_params(rule=0, tau=1.0, check_every=5)
    v, ipb = batch.tune_cached([p.zeros_eta() for p in probs], params, cache, iters=2,
                               tau_vecs=taus2)
    lines = [ln for ln in open(cache).read().split("\n") if ln]
    assert len(lines) == 1 and lines[0].split()[1:] == [str(v), str(ipb)]
    assert ipb in (2, 4, 8, 16)
    key = lines[0].split()[0]
    with open(cache, "a") as f:
        f.write(f"{key} {v} 16\n")
    assert batch.tune_cached([p.zeros_eta() for p in probs], params, cache, iters=2,
                             tau_vecs=taus2) == (v, 16)
    assert len([ln for ln in open(cache).read().split("\n") if ln]) == 2
    etas = [p.zeros_eta() for p in probs]
    rows = batch.iterate(etas, 15, params, tau_vecs=taus2)
    for q in range(len(base)):
        assert np.array_equal(etas[q].cpu().numpy(), ref[q][0]), q
        assert np.array_equal(rows[q], ref[q][1]), q
    batch.close()


def test_batch_tune_picks_a_variant(cb):
    base = [batch_instance(b, scale=0.004) for b in range(3)]
    insts, probs, taus = _setup(cb, base, torch.float32, tau0=0.001)
    batch = cb.Batch(probs)
    etas = [p.zeros_eta() for p in probs]
    params = cb.make_params(rule=0, tau=1.0, check_every=5)
    v = batch.tune(etas, params, iters=3, tau_vecs=taus)
    assert v in (0, 1, 2, 3)
    assert batch.info()["variant"] == v
    rows = batch.iterate([p.zeros_eta() for p in probs], 5, params, tau_vecs=taus)
    assert np.all(np.isfinite(rows))
    batch.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batch_variants_agree(cb, dtype):
    """Every batched segment-kernel variant the batch can run gives the same
    duals bit for bit: the handles' own slot-major copies part by part (2-, 4-
    and 8-lane groups for FP32 handles, 8-lane for FP64), the row-major copy
    with the prices in LDS or from global memory."""
    dt = torch.float64 if dtype == "f64" else torch.float32
    base = [batch_instance(b, scale=0.004) for b in range(4)]
    ref = None
    seen = []
    for v in range(4):
        _, probs, taus = _setup(cb, base, dt)
        batch = cb.Batch(probs)
        try:
            batch.select(v)
        except cb.CblpError:
            batch.close()
            for p in probs:
                p.close()
            continue                            # not usable on these handles
        assert batch.info()["variant"] == v
        etas = [p.zeros_eta() for p in probs]
        batch.iterate(etas, 12, cb.make_params(rule=0, tau=1.0, check_every=4), tau_vecs=taus)
        out = [e.cpu().numpy() for e in etas]
        batch.close()
        for p in probs:
            p.close()
        seen.append(v)
        if ref is None:
            ref = out
        for q, (a, b) in enumerate(zip(ref, out)):
            assert np.array_equal(a, b), (v, q)
    # the handles' copies have 16-bit ids here (n <= 65,536): 3 needs 32-bit ones
    assert seen == [0, 1, 2], seen


def test_batch_solve_iteration_cap(cb):
    """spfom_batch_solve treats max_iters as spfom_solve does: a cap below
    check_every or not a multiple of it runs exactly max_iters iterations (the
    last block cut short), and the gap is tested only after whole blocks."""
    base = [batch_instance(b, scale=0.004) for b in range(3)]
    for cap in (0, 7, 23):
        _, probs, taus = _setup(cb, base, torch.float32, tau0=0.001)
        batch = cb.Batch(probs)
        etas = [p.zeros_eta() for p in probs]
        params = cb.make_params(rule=0, tau=1.0, check_every=10, tol=0.0, max_iters=cap)
        outs = batch.solve(etas, params, tau_vecs=taus)
        batch.close()
        singles = []
        for p, t in zip(probs, taus):
            e = p.zeros_eta()
            st = p.solve(e, cb.make_params(rule=0, tau_vec=t, check_every=10, tol=0.0,
                                           max_iters=cap)).as_dict()
            singles.append((st, e.cpu().numpy()))
        for q, o in enumerate(outs):
            assert o["iters"] == cap and singles[q][0]["iters"] == cap, (cap, q, o)
            assert o["status"] == 5 and singles[q][0]["status"] == 5
            assert np.array_equal(etas[q].cpu().numpy(), singles[q][1]), (cap, q)
        for p in probs:
            p.close()


@pytest.mark.parametrize("dtype,rule", [("f32", 0), ("f64", 0), ("f32", 1)])
def test_batch_solve_one_launch_matches_launches(cb, dtype, rule):
    """The one-launch solve (a persistent block per instance running its own
    iterations, folds and gap tests) and the per-iteration launches stop each
    instance at the same iteration with the same duals and last trace row,
    bit for bit; masked instances are left alone by both."""
    dt = torch.float64 if dtype == "f64" else torch.float32
    shapes = [(3000, 300), (800, 40), (5000, 1500), (1200, 700), (2500, 2000)]
    base = [make_instance(L, n, size_lo=3, size_hi=40, zipf=1.1, cap_lo=0.2, cap_hi=0.6, seed=10 + k)
            for k, (L, n) in enumerate(shapes)] + \
        [make_instance(800, 40, size_lo=3, size_hi=9, cap_lo=0.5, cap_hi=3.0, seed=s) for s in (1, 2)]
    mask = [1, 1, 0, 1, 1, 1, 1]
    res = {}
    for mode in (0, 1):
        _, probs, taus = _setup(cb, base, dt, tau0=0.01, rule=rule)
        batch = cb.Batch(probs)
        batch.persistent(mode)
        cb.cblp_batch_mask(batch.b, mask)
        etas = [p.zeros_eta() for p in probs]
        kw = dict(rule=rule, tau=1.0, check_every=10, tol=0.05, max_iters=403)
        if rule == 0:
            kw.update(tau_decay=0.7, decay_every=100)
        outs = batch.solve(etas, cb.make_params(**kw), tau_vecs=taus)
        res[mode] = (outs, [e.cpu().numpy() for e in etas])
        batch.close()
        for p in probs:
            p.close()
    (o0, e0), (o1, e1) = res[0], res[1]
    if rule == 0:   # some stop early, the others run to the cap (the last block cut short)
        assert any(o["status"] == 0 and o["iters"] < 403 for o, m in zip(o0, mask) if m)
        assert any(o["iters"] == 403 for o, m in zip(o0, mask) if m)
    for q in range(len(base)):
        assert o0[q]["iters"] == o1[q]["iters"] and o0[q]["status"] == o1[q]["status"], (q, o0[q], o1[q])
        for k in cb.TRACE_COLS:
            assert o0[q][k] == o1[q][k] or (np.isnan(o0[q][k]) and np.isnan(o1[q][k])), (q, k)
        assert np.array_equal(e0[q], e1[q]), q
    assert o1[2]["iters"] == 0 and not np.any(e1[2])


def test_batch_one_launch_needs_binned_products(cb):
    """The one-launch form is refused where a product has no LDS bin."""
    big = make_instance(200, 30000, size_lo=2, size_hi=4, seed=3)   # bins for 16,256 of 30,000
    _, probs, _ = _setup(cb, [big], torch.float32)
    batch = cb.Batch(probs)
    with pytest.raises(cb.CblpError) as e:
        batch.persistent(1)
    assert e.value.code == cb.CBLP_EINVAL
    batch.persistent(0)
    batch.persistent(-1)
    batch.close()
    probs[0].close()
