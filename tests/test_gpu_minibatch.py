"""Stochastic minibatch SPFOM on the GPU (spfom_minibatch, through the C
ABI) against the oracle's (Algorithm 2; Algorithm 3 with k B < L) at equal
iteration counts, the full minibatch against the full-batch kernels bit for
bit, invalid batches rejected, and the decaying constant step against the
oracle."""
import numpy as np
import pytest

import oracle
from paper_2602_22421_amd.instances import config_instance, minibatch_schedule, step_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_22421_amd import cblp
    cblp.load()
    return cblp


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dtype,cfg,frac,mode", [
    ("f64", 0, 0.1, "independent"),
    ("f64", 0, 0.5, "epoch"),
    ("f32", 1, 0.1, "epoch"),
    ("f64", 2, 0.05, "independent"),
])
def test_minibatch_matches_oracle(cb, dtype, cfg, frac, mode):
    dt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    inst = (config_instance(cfg) if cfg == 0 else config_instance(cfg, scale=0.01 if cfg == 1
                                                                  else 0.002)).cast(npdt)
    B = max(1, int(frac * inst.L))
    T = 40
    batch = minibatch_schedule(inst.L, B, T, seed=cfg + 11, mode=mode)
    tau = step_scale(inst, 0.002).astype(npdt)
    prob = cb.Problem(inst, dtype=dt)
    params = cb.make_params(rule=0, tau_vec=prob.tensor(tau))
    mb = oracle.Minibatch(inst, tau=tau.astype(np.float64), mu=0.0)
    eg, eo = prob.zeros_eta(), np.zeros(inst.m)
    bar = 1e-9 if dtype == "f64" else 1e-5
    done = 0
    for t in (1, 10, T):
        trg = prob.minibatch(eg, batch[done:t], params)
        eo, tro = mb.iterate(eo, batch[done:t])
        done = t
        assert rel(eg.double().cpu().numpy(), eo) <= bar, (t, rel(eg.double().cpu().numpy(), eo))
        for col in (1, 3, 4):
            assert rel(trg[:, col], tro[:, col]) <= bar, (t, col)
        assert np.all(trg[:, 0] == 0.0) and np.all(trg[:, 8] == 1.0)
    prob.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_minibatch_equals_full_batch(cb, dtype):
    """B = L: every segment is re-solved in every iteration, in the same
    rounding as the full-batch kernels, so the duals agree bit for bit."""
    dt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    inst = config_instance(1, scale=0.005).cast(npdt)
    tau = step_scale(inst, 0.002).astype(npdt)
    prob = cb.Problem(inst, dtype=dt)
    params = cb.make_params(rule=0, tau_vec=prob.tensor(tau), check_every=5)
    e_full = prob.zeros_eta()
    tr_full, _ = prob.iterate(e_full, 15, params)
    prob2 = cb.Problem(inst, dtype=dt)
    e_mb = prob2.zeros_eta()
    tr_mb = prob2.minibatch(e_mb, minibatch_schedule(inst.L, inst.L, 15, seed=2), params)
    assert np.array_equal(e_full.cpu().numpy(), e_mb.cpu().numpy())
    np.testing.assert_array_equal(tr_full[:, 1], tr_mb[:, 1])
    prob.close()
    prob2.close()


def test_minibatch_state_persists_and_resets(cb):
    """Two calls of 10 iterations equal one call of 20; spfom_reset starts
    the kept sales again from 0."""
    inst = config_instance(0)
    tau = step_scale(inst, 0.002)
    batch = minibatch_schedule(inst.L, 100, 20, seed=4)
    prob = cb.Problem(inst, dtype=torch.float64)
    params = cb.make_params(rule=0, tau_vec=prob.tensor(tau))
    e1 = prob.zeros_eta()
    prob.minibatch(e1, batch[:10], params)
    prob.minibatch(e1, batch[10:], params)
    prob.reset()
    e2 = prob.zeros_eta()
    prob.minibatch(e2, batch, params)
    assert np.array_equal(e1.cpu().numpy(), e2.cpu().numpy())
    prob.close()


@pytest.mark.parametrize("bad", ["out_of_range", "negative", "duplicate"])
def test_minibatch_rejects_bad_batches(cb, bad):
    inst = config_instance(0)
    prob = cb.Problem(inst, dtype=torch.float64)
    params = cb.make_params(rule=0, tau=0.01)
    batch = minibatch_schedule(inst.L, 8, 2, seed=1)
    if bad == "out_of_range":
        batch[1, 3] = inst.L
    elif bad == "negative":
        batch[0, 0] = -1
    else:
        batch[1, 5] = batch[1, 2]
    with pytest.raises(cb.CblpError) as e:
        prob.minibatch(prob.zeros_eta(), batch, params)
    assert e.value.code == cb.CBLP_EINVAL
    # a decaying or Polyak step is refused
    with pytest.raises(cb.CblpError):
        prob.minibatch(prob.zeros_eta(), batch[:1] * 0 + np.arange(8),
                       cb.make_params(rule=0, tau=0.01, tau_decay=0.5, decay_every=2))
    prob.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_decaying_step_matches_oracle(cb, dtype):
    dt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    inst = (config_instance(0) if dtype == "f64" else config_instance(1, scale=0.01)).cast(npdt)
    tau = step_scale(inst, 0.003).astype(npdt)
    prob = cb.Problem(inst, dtype=dt)
    params = cb.make_params(rule=0, tau_vec=prob.tensor(tau), check_every=10, tau_decay=0.7,
                            decay_every=7)
    eg = prob.zeros_eta()
    trg, _ = prob.iterate(eg, 50, params)
    orc = oracle.Solver(inst, tau=tau.astype(np.float64), check_every=10, tau_decay=0.7,
                        decay_every=7)
    eo, tro = orc.iterate(np.zeros(inst.m), 50)
    bar = 1e-8 if dtype == "f64" else 1e-5
    assert rel(eg.double().cpu().numpy(), eo) <= bar
    np.testing.assert_array_equal(trg[:, 8], tro[:, 8])      # the multipliers, bit for bit
    for col in (0, 1, 5, 6):
        assert rel(trg[:, col], tro[:, col]) <= bar, col
    prob.close()
