"""Learned warm start for spfom_solve: collect (features, dual) pairs from
solved instances, train the network on the GPU, start new solves from its
prediction, and fall back to the cold start when the prediction is worse.

The learned start is an addition to the paper's method (Section 7 leaves
learned components to future work).  It changes only the initial duals eta^0
that SPFOM (Algorithm 2) takes as input; the dual bound D(eta), the value of
the Lagrangian minimax of Section 4.1, and the averaged-primal lower bound
still certify the result, so a poor prediction can cost iterations but
never correctness.  The fallback compares D at the prediction with D at the
cold start eta = 0: D is an upper bound on the LP optimum for every eta >= 0,
and the smaller bound is the better start.

Every step runs in libcblp (features, targets, the training loop with its
forward, backward and Adam kernels, prediction, solves); torch only holds
device memory.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional, Sequence

import numpy as np
import torch

from . import cblp
from .instances import step_scale

__all__ = ["SolveSpec", "collect", "train", "warm_solve", "cold_solve"]


@dataclasses.dataclass
class SolveSpec:
    """Solver settings shared by the target solves and the evaluation."""
    rule: int = cblp.SPFOM_STEP_CONST
    tau0: float = 1e-3           # step scale: tau_i = tau0 max r / c_i (step_scale)
    gamma: float = 1.0
    check_every: int = 10
    tol: float = 1e-2
    max_iters: int = 3000

    def params(self, prob: "cblp.Problem", inst, tol: Optional[float] = None,
               max_iters: Optional[int] = None):
        npdt = np.float32 if prob.dtype == torch.float32 else np.float64
        tau = prob.tensor(step_scale(inst, self.tau0).astype(npdt))
        return cblp.make_params(rule=self.rule, tau_vec=tau, gamma=self.gamma,
                                check_every=self.check_every,
                                tol=self.tol if tol is None else tol,
                                max_iters=self.max_iters if max_iters is None else max_iters)


def collect(instances: Sequence, spec: SolveSpec, dtype=torch.float32,
            log: Optional[Callable[[str], None]] = None,
            stages: Optional[Sequence] = None):
    """Solve each instance cold and return (X [rows, 4], Y [rows]) on the
    device: the features of every product and its dual scaled by revenue,
    y_j = eta_j / r_j, the quantity the network predicts.

    ``stages`` None runs spfom_solve with ``spec``; otherwise it is a list of
    (tau0, iterations) pairs run one after the other by spfom_iterate (a
    coarse step to approach the duals, then finer ones), the targets being the
    duals after the last stage."""
    xs, ys = [], []
    for k, inst in enumerate(instances):
        prob = cblp.Problem(inst, dtype=dtype)
        eta = prob.zeros_eta()
        if stages is None:
            st = prob.solve(eta, spec.params(prob, inst)).as_dict()
        else:
            prob.reset()
            for tau0, iters in stages:
                p = dataclasses.replace(spec, tau0=tau0).params(prob, inst)
                _, s = prob.iterate(eta, int(iters), p, trace=False)
            st = s.as_dict()
        xs.append(cblp.features(prob))
        ys.append(cblp.targets(prob, eta))
        if log:
            log(f"collect {k}: {getattr(inst, 'name', '')} iters={st['iters']} "
                f"gap={st['gap']:.3e}")
        prob.close()
    return torch.cat(xs).contiguous(), torch.cat(ys).contiguous()


def train(net: "cblp.WarmStartNet", X: torch.Tensor, Y: torch.Tensor, *, epochs: int = 20,
          batch: int = 4096, lr: float = 1e-3, seed: int = 0,
          log: Optional[Callable[[str], None]] = None) -> List[float]:
    """Adam on shuffled minibatches (the library's training loop); returns
    the mean loss of each epoch."""
    losses = [float(x) for x in net.train(X, Y, epochs=epochs, batch=batch, lr=lr, seed=seed)]
    if log:
        for e, l in enumerate(losses):
            log(f"epoch {e}: loss {l:.5e}")
    return losses


def cold_solve(prob: "cblp.Problem", inst, spec: SolveSpec, **kw):
    """spfom_solve from eta = 0; returns (stats dict, eta)."""
    eta = prob.zeros_eta()
    st = prob.solve(eta, spec.params(prob, inst, **kw)).as_dict()
    return st, eta


def warm_solve(net: "cblp.WarmStartNet", prob: "cblp.Problem", inst, spec: SolveSpec, **kw):
    """spfom_solve from the network's prediction, or from eta = 0 when the
    prediction's dual bound is not below the cold start's.  Returns (stats
    dict with 'warm' (bool), 'D0', 'D_pred', 'predict_seconds'; eta)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eta, info = net.start(prob)   # prediction and cold fallback, in the library
    warm, d_pred, d_cold = info["used"], info["D_pred"], info["D0"]
    t_pred = time.perf_counter() - t0
    st = prob.solve(eta, spec.params(prob, inst, **kw)).as_dict()
    st.update(warm=warm, D0=d_cold, D_pred=d_pred, predict_seconds=t_pred)
    return st, eta
