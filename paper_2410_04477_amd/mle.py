"""Maximum-likelihood estimation of (sigma2, range, nugget) with L-BFGS on
log-parameters, driven by the adjoint gradient (VecchiaLogLik)."""
from __future__ import annotations

import dataclasses
import math
import time

import torch

from .model import BlockVecchia, vecchia_loglik

NUGGET_FLOOR = 1e-8  # log-parametrisation floor: eta_3 = log(nugget + floor)


@dataclasses.dataclass
class MLEResult:
    theta: tuple          # (sigma2, range, nugget)
    loglik: float
    evals: int
    iters: int
    seconds: float
    converged: bool


def fit(model: BlockVecchia, theta0, precision: str = "fp64", max_evals: int = 200, tol_rel: float = 1e-10,
        history: int = 10, polish_evals: int = 30) -> MLEResult:
    """L-BFGS (strong Wolfe line search) on eta = log(sigma2, range, nugget + floor),
    minimising -l / n.  Stops on relative change < tol_rel, small gradient, or
    max_evals evaluations.  With an FP32-bulk precision, a short FP64 L-BFGS
    pass (at most polish_evals evaluations) starts from the FP32 optimum: the
    FP32 gradient's rounding error can stop the line search early near the
    optimum, where the exact gradient is small."""
    if precision != "fp64" and polish_evals > 0:
        first = fit(model, theta0, precision, max_evals, tol_rel, history, 0)
        second = fit(model, first.theta, "fp64", polish_evals, tol_rel, history, 0)
        return MLEResult(second.theta, second.loglik, first.evals + second.evals, first.iters + second.iters,
                         first.seconds + second.seconds, second.converged)
    s2, rg, nug = (float(v) for v in theta0)
    eta = torch.tensor([math.log(s2), math.log(rg), math.log(nug + NUGGET_FLOOR)], dtype=torch.float64,
                       requires_grad=True)
    opt = torch.optim.LBFGS([eta], lr=1.0, max_iter=max_evals, max_eval=max_evals, history_size=history,
                            tolerance_grad=1e-9, tolerance_change=tol_rel, line_search_fn="strong_wolfe")
    n = model.n
    state = {"evals": 0, "best": -math.inf}

    def closure():
        opt.zero_grad()
        e = torch.exp(eta)
        params = torch.stack([e[0], e[1], e[2] - NUGGET_FLOOR])
        ll = vecchia_loglik(params, model, precision)
        if not torch.isfinite(ll):
            ll = torch.tensor(-1e300, dtype=torch.float64)  # pushes the line search back
        loss = -ll / n
        loss.backward()
        state["evals"] += 1
        state["best"] = max(state["best"], float(ll))
        return loss

    t0 = time.perf_counter()
    opt.step(closure)
    dt = time.perf_counter() - t0
    e = torch.exp(eta.detach())
    th = (float(e[0]), float(e[1]), float(e[2] - NUGGET_FLOOR))
    ll = float(model.loglik([model.theta(*th)], precision)[0][0])
    st = opt.state[opt._params[0]]
    return MLEResult(th, ll, state["evals"], int(st.get("n_iter", 0)), dt, state["evals"] < max_evals)
