"""The segment kernels the library chooses from the shape agree bit for bit.

FP32 instances take the three-part kernel (2-, 4- and 8-lane groups) with all
prices in LDS when they fit, else with the popular head of them in LDS and
16-bit product ids (n <= 65,536) or 32-bit ids; FP64 instances take the
8-lane kernel with 16- or 32-bit ids.  Padding an instance with products
that no segment considers changes which kernel runs (and how many sales bins
sit in LDS, and how many of them are 32 bits wide) but not the answer for
the real products, so each padded run must give the unpadded run's sales,
usage, R* and duals bit for bit."""
import dataclasses

import numpy as np
import pytest

from paper_2602_22421_amd.instances import make_instance, step_scale

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_22421_amd import cblp
    cblp.load()
    return cblp


def _pad(inst, n):
    """The instance with products [inst.n, n) added; no segment considers them."""
    extra = n - inst.n
    rng = np.random.default_rng(n)
    r = np.concatenate([inst.r, rng.uniform(1, 100, extra).astype(inst.r.dtype)])
    c = np.concatenate([inst.c, np.ones(extra, dtype=inst.c.dtype)])
    return dataclasses.replace(inst, n=n, m=n, r=r, c=c)


def _run(cb, inst, dt, n0, tau0):
    prob = cb.Problem(inst, dtype=dt)
    rng = np.random.default_rng(11)
    eta0 = np.zeros(inst.m)
    eta0[:n0] = rng.uniform(0, 1, n0) * inst.r[:n0] * 0.5
    S, u, R = prob.sales(prob.tensor(eta0), seg_R=True)
    out = [S.cpu().numpy()[:n0], u.cpu().numpy()[:n0], R.cpu().numpy()]
    npdt = np.float32 if dt == torch.float32 else np.float64
    tau = np.concatenate([tau0, np.ones(inst.m - n0)]).astype(npdt)
    e2 = prob.zeros_eta()
    tr, _ = prob.iterate(e2, 5, cb.make_params(rule=0, tau_vec=prob.tensor(tau), check_every=5))
    out.append(e2.cpu().numpy()[:n0])
    info = cb.cblp_launch_info(prob.h)
    prob.close()
    return out, tr, info


@pytest.mark.parametrize("dtype,sizes", [("f32", (600, 30000, 70000)), ("f64", (600, 70000))])
def test_shape_chosen_kernels_agree(cb, dtype, sizes):
    dt = torch.float32 if dtype == "f32" else torch.float64
    npdt = np.float32 if dtype == "f32" else np.float64
    # rows of 1..80 entries: every group width, and rows past the register slots
    base = make_instance(30000, 600, size_lo=1, size_hi=80, zipf=1.1, cap_lo=0.2, cap_hi=0.5,
                         seed=21).cast(npdt)
    tau0 = step_scale(base, 1e-3)
    ref, tr_ref, info_ref = _run(cb, base, dt, base.n, tau0)
    bins = [(info_ref["lds_bins"], info_ref["lds_bins64"])]
    for n in sizes[1:]:
        got, tr, info = _run(cb, _pad(base, n), dt, base.n, tau0)
        bins.append((info["lds_bins"], info["lds_bins64"]))
        for k, (a, b) in enumerate(zip(ref, got)):
            assert np.array_equal(a, b), (n, k, info)
        # the FP64 sums over products only gain exact zeros
        np.testing.assert_allclose(tr[:, :3], tr_ref[:, :3], rtol=1e-14)
    if dtype == "f32":
        # all 600 prices and 64-bit bins in LDS; at n = 30,000 and 70,000 the
        # head of the prices in LDS and bins for fewer products than n (the rest
        # take global atomics): 64-bit ones only for the popular products whose
        # sales within a block may reach 2^32 quanta, 32-bit ones for the other
        # real products and the padding's head
        assert bins[0] == (600, 600), bins
        assert 600 < bins[1][0] < 30000 and 0 < bins[1][1] < 600, bins
        assert bins[2] == bins[1], bins
    else:
        assert all(b == b64 for b, b64 in bins), bins
