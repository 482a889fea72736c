"""The allocation-free entry point (cblp_gap_static, static device scratch)
against the existing one it varies (cblp_gap, and cblp_sales for the product
sales), through the C ABI: two calls in a row, the second on a smaller
instance, for FP64 and FP32 and a general resource matrix; sizes past its
static scratch are refused."""
import numpy as np
import pytest

from paper_2602_22421_amd.instances import config_instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_22421_amd import cblp
    cblp.load()
    return cblp


def _eta(inst, seed):
    rng = np.random.default_rng(seed)
    base = inst.r if inst.identity else np.full(inst.m, float(inst.r.mean()))
    return rng.uniform(0, 1, inst.m) * base * 0.6


def _compare(cb, inst, dt, seed):
    prob = cb.Problem(inst, dtype=dt)
    eta = prob.tensor(_eta(inst, seed))
    S_ref, _, _ = prob.sales(eta)
    g = prob.gap(eta)
    S = torch.full((inst.n,), -1.0, dtype=torch.float64, device=prob.device)
    bounds = torch.zeros(2, dtype=torch.float64, device=prob.device)
    cb.cblp_gap_static(prob, eta, S, bounds)
    torch.cuda.synchronize()
    # the same per-segment arithmetic and fixed-point scale: the same sales bits
    assert torch.equal(S, S_ref)
    D, P = bounds.cpu().numpy()
    assert D == pytest.approx(g["D"], rel=1e-12)
    assert P == pytest.approx(g["P"], rel=1e-12)
    prob.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_static_matches_gap_twice_second_smaller(cb, dtype):
    dt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    big = config_instance(1, scale=0.02).cast(npdt)       # 40,000 segments, 20,000 products
    small = config_instance(0).cast(npdt)                  # 1,000 segments, 50 products
    _compare(cb, big, dt, 1)
    _compare(cb, small, dt, 2)


def test_static_general_resources(cb):
    inst = config_instance(2, scale=0.002)
    _compare(cb, inst, torch.float64, 3)
    _compare(cb, config_instance(0), torch.float64, 4)


def test_static_refuses_sizes_past_its_scratch(cb):
    n = cb.cblp_gap_static_max_products() + 1
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    ptr = torch.zeros(1, dtype=torch.int64, device="cuda")
    from paper_2602_22421_amd.cblp import load, _ptr, _stream
    rc = load().cblp_gap_static(0, n, n, _ptr(ptr), None, None, None, None, None, _ptr(one),
                                None, None, None, _ptr(one), cb.CBLP_F64, _ptr(one), None,
                                _ptr(one), _stream())
    assert rc == cb.CBLP_EINVAL
    assert "static scratch" in cb.last_error()
