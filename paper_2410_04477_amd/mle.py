"""Maximum-likelihood estimation of (sigma2, range, nugget), and optionally
the smoothness nu, with L-BFGS on transformed parameters, driven by the
adjoint gradient (VecchiaLogLik) and the library's d l / d nu."""
from __future__ import annotations

import dataclasses
import math
import time

import torch

from ._lib import VecchiaError
from .model import BlockVecchia, vecchia_loglik, vecchia_loglik_nu

NUGGET_FLOOR = 1e-8  # a zero starting nugget starts at eta_3 = log(NUGGET_FLOOR)
NU_LO, NU_HI = 0.06, 9.5   # nu = NU_LO + (NU_HI - NU_LO) sigmoid(eta_4), inside the Bessel form's [0.05, 10]


@dataclasses.dataclass
class MLEResult:
    theta: tuple          # (sigma2, range, nugget), plus nu when it is estimated
    loglik: float
    evals: int
    iters: int
    seconds: float
    converged: bool
    grad_eta: float = math.nan   # max |d l / d eta_k| / n at theta, FP64 adjoint
    restarts: int = 0


def _nu_to_eta(nu: float) -> float:
    u = (nu - NU_LO) / (NU_HI - NU_LO)
    return math.log(u / (1.0 - u))


def to_natural(eta: torch.Tensor, estimate_nu: bool = False) -> torch.Tensor:
    """(sigma2, range, nugget[, nu]) from the unconstrained eta: exp for the
    first three, so every eta maps inside the domain (sigma2, range, nugget > 0)
    however far the line search moves; nu = NU_LO + (NU_HI - NU_LO) sigmoid(eta_4)."""
    e = torch.exp(eta[:3])
    if estimate_nu:
        return torch.cat([e, (NU_LO + (NU_HI - NU_LO) * torch.sigmoid(eta[3])).reshape(1)])
    return e


def to_eta(theta, estimate_nu: bool = False) -> list:
    """Inverse of to_natural; a zero nugget starts at log(NUGGET_FLOOR)."""
    s2, rg, nug = (float(v) for v in theta[:3])
    e = [math.log(s2), math.log(rg), math.log(max(nug, NUGGET_FLOOR))]
    if estimate_nu:
        e.append(_nu_to_eta(float(theta[3])))
    return e


def stationarity(model: BlockVecchia, theta, estimate_nu: bool = False) -> float:
    """max_k |d l / d eta_k| / n at theta from the FP64 adjoint, eta the
    unconstrained parameters of fit (so a nugget driven to zero, where
    d l / d eta_3 = nugget d l / d nugget vanishes, counts as stationary)."""
    th = tuple(float(v) for v in theta)
    if estimate_nu:
        _, g, _, _, _ = model.loglik_grad_nu([model.theta(*th)], "fp64")
    else:
        _, g, _, _, _ = model.loglik_grad([model.theta(*th)], "fp64")
    g = g[0].cpu().numpy()
    ge = [g[k] * th[k] for k in range(3)]
    if estimate_nu:
        u = (th[3] - NU_LO) / (NU_HI - NU_LO)
        ge.append(g[3] * (NU_HI - NU_LO) * u * (1.0 - u))
    return float(max(abs(v) for v in ge)) / model.n


def fit(model: BlockVecchia, theta0, precision: str = "fp64", max_evals: int = 200, tol_rel: float = 1e-10,
        history: int = 10, polish_evals: int = 30, estimate_nu: bool = False, restarts: int = 3,
        stat_tol: float = 1e-7) -> MLEResult:
    """L-BFGS MLE (see _fit_once), then a stationarity check with the FP64
    adjoint: while max_k |d l / d eta_k| / n exceeds stat_tol, L-BFGS starts
    again in FP64 from the point reached (fresh curvature history), at most
    `restarts` times.  The line search of a long run can stop on a tiny
    relative change of the objective while the gradient is still clearly
    non-zero; a fresh start from there continues the ascent."""
    res = _fit_once(model, theta0, precision, max_evals, tol_rel, history, polish_evals, estimate_nu)
    res.grad_eta = stationarity(model, res.theta, estimate_nu)
    for k in range(restarts):
        if not res.grad_eta > stat_tol:
            break
        # torch's L-BFGS stops on an absolute change of the objective below
        # tolerance_change, which near a flat optimum can come before the
        # gradient is small: the restart asks for a far smaller change
        more = _fit_once(model, res.theta, "fp64", max(polish_evals, max_evals // 2), tol_rel * 1e-4, history, 0,
                         estimate_nu)
        better = more.loglik >= res.loglik
        res = MLEResult(more.theta if better else res.theta, max(more.loglik, res.loglik), res.evals + more.evals,
                        res.iters + more.iters, res.seconds + more.seconds, more.converged if better else res.converged,
                        restarts=k + 1)
        res.grad_eta = stationarity(model, res.theta, estimate_nu)
    return res


def _fit_once(model: BlockVecchia, theta0, precision: str = "fp64", max_evals: int = 200, tol_rel: float = 1e-10,
              history: int = 10, polish_evals: int = 30, estimate_nu: bool = False) -> MLEResult:
    """L-BFGS (strong Wolfe line search) on eta = log(sigma2, range, nugget),
    minimising -l / n.  Stops on relative change < tol_rel, small gradient, or
    max_evals evaluations.  With an FP32-bulk precision, a short FP64 L-BFGS
    pass (at most polish_evals evaluations) starts from the FP32 optimum: the
    FP32 gradient's rounding error can stop the line search early near the
    optimum, where the exact gradient is small.
    estimate_nu: nu joins the parameters (the paper estimates it with the
    others), through eta_4 = logit((nu - NU_LO) / (NU_HI - NU_LO)); theta0 may
    then carry a fourth entry, the starting nu (else the model's)."""
    if precision != "fp64" and polish_evals > 0:
        first = _fit_once(model, theta0, precision, max_evals, tol_rel, history, 0, estimate_nu)
        second = _fit_once(model, first.theta, "fp64", polish_evals, tol_rel, history, 0, estimate_nu)
        return MLEResult(second.theta, second.loglik, first.evals + second.evals, first.iters + second.iters,
                         first.seconds + second.seconds, second.converged)
    if estimate_nu:
        nu0 = float(theta0[3]) if len(theta0) > 3 else model.nu
        if not NU_LO < nu0 < NU_HI:
            raise ValueError(f"starting nu {nu0} outside ({NU_LO}, {NU_HI})")
        theta0 = tuple(theta0[:3]) + (nu0,)
    eta = torch.tensor(to_eta(theta0, estimate_nu), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.LBFGS([eta], lr=1.0, max_iter=max_evals, max_eval=max_evals, history_size=history,
                            tolerance_grad=1e-9, tolerance_change=tol_rel, line_search_fn="strong_wolfe")
    n = model.n
    state = {"evals": 0, "best": -math.inf}

    def closure():
        opt.zero_grad()
        params = to_natural(eta, estimate_nu)
        try:
            ll = vecchia_loglik_nu(params, model, precision) if estimate_nu else vecchia_loglik(params, model, precision)
        except VecchiaError:
            ll = None   # a theta the library rejects counts as a failed evaluation
        if ll is None or not torch.isfinite(ll):
            ll = 0.0 * params.sum() - 1e300   # pushes the line search back (keeps the graph for backward)
        loss = -ll / n
        loss.backward()
        state["evals"] += 1
        state["best"] = max(state["best"], float(ll))
        return loss

    t0 = time.perf_counter()
    opt.step(closure)
    dt = time.perf_counter() - t0
    th = tuple(float(v) for v in to_natural(eta.detach(), estimate_nu))
    ll = float(model.loglik([model.theta(*th)], precision)[0][0])
    st = opt.state[opt._params[0]]
    return MLEResult(th, ll, state["evals"], int(st.get("n_iter", 0)), dt, state["evals"] < max_evals)
