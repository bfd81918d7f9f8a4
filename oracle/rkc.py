"""Runge-Kutta-Chebyshev method, FP64 reference (test infrastructure only).

The paper (Sec. II) replaces explicit Euler by the s-stage, second-order RKC
scheme of its ref. [9] (Sommeijer, Shampine, Verwer, J. Comp. Appl. Math. 88,
1998), whose real stability interval grows with s^2, and applies it to the
non-diagonal M of eq. (2) by evaluating F(t, Y) = M^{-1}(b(t) - K(Y)Y) at
every stage. Everything below restates ref. [9]'s construction:

  damping eps = 2/13, w0 = 1 + eps/s^2, Chebyshev polynomials of the first
  kind T_j and their first two derivatives evaluated at w0,
  w1 = T_s'(w0) / T_s''(w0),
  b_j = T_j''(w0) / T_j'(w0)^2 (j >= 2), b_0 = b_1 = b_2, a_j = 1 - b_j T_j(w0),
  mu~_1 = b_1 w1, and for j >= 2
      mu_j = 2 b_j w0 / b_{j-1},  nu_j = -b_j / b_{j-2},
      mu~_j = 2 b_j w1 / b_{j-1}, gamma~_j = -a_{j-1} mu~_j,
  stage times c_0 = 0, c_1 = mu~_1, c_j = w1 T_j''(w0) / T_j'(w0) (c_s = 1).

One step from y_n:
  Y_0 = y_n,  Y_1 = Y_0 + mu~_1 tau F_0,
  Y_j = (1 - mu_j - nu_j) Y_0 + mu_j Y_{j-1} + nu_j Y_{j-2}
        + mu~_j tau F_{j-1} + gamma~_j tau F_0,     j = 2..s,
  y_{n+1} = Y_s,   with F_j = F(t_n + c_j tau, Y_j).
The stage stability polynomials are P_j(z) = a_j + b_j T_j(w0 + w1 z); the
scheme is stable for tau * rho <= beta(s) = (1 + w0) / w1.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np

DAMPING = 2.0 / 13.0


@dataclass
class RkcCoefficients:
    s: int
    w0: float
    w1: float
    T: np.ndarray  # T_j(w0), j = 0..s
    dT: np.ndarray  # T_j'(w0)
    ddT: np.ndarray  # T_j''(w0)
    a: np.ndarray
    b: np.ndarray
    mu: np.ndarray  # index j = 0..s (entries 0, 1 unused)
    nu: np.ndarray
    mu_t: np.ndarray
    gamma_t: np.ndarray
    c: np.ndarray
    beta: float  # stability boundary (1 + w0) / w1


def coefficients(s: int, damping: float = DAMPING) -> RkcCoefficients:
    """RKC(s) coefficients from ref. [9] (see module docstring)."""
    if s < 2:
        raise ValueError("RKC needs s >= 2 stages")
    w0 = 1.0 + damping / (s * s)
    T = np.zeros(s + 1)
    dT = np.zeros(s + 1)
    ddT = np.zeros(s + 1)
    T[0], T[1] = 1.0, w0
    dT[0], dT[1] = 0.0, 1.0
    ddT[0], ddT[1] = 0.0, 0.0
    for j in range(2, s + 1):
        T[j] = 2.0 * w0 * T[j - 1] - T[j - 2]
        dT[j] = 2.0 * T[j - 1] + 2.0 * w0 * dT[j - 1] - dT[j - 2]
        ddT[j] = 4.0 * dT[j - 1] + 2.0 * w0 * ddT[j - 1] - ddT[j - 2]
    w1 = dT[s] / ddT[s]

    b = np.zeros(s + 1)
    for j in range(2, s + 1):
        b[j] = ddT[j] / dT[j] ** 2
    b[0] = b[1] = b[2]
    a = 1.0 - b * T

    mu = np.zeros(s + 1)
    nu = np.zeros(s + 1)
    mu_t = np.zeros(s + 1)
    gamma_t = np.zeros(s + 1)
    mu_t[1] = b[1] * w1
    for j in range(2, s + 1):
        mu[j] = 2.0 * b[j] * w0 / b[j - 1]
        nu[j] = -b[j] / b[j - 2]
        mu_t[j] = 2.0 * b[j] * w1 / b[j - 1]
        gamma_t[j] = -a[j - 1] * mu_t[j]

    c = np.zeros(s + 1)
    c[1] = mu_t[1]
    for j in range(2, s + 1):
        c[j] = w1 * ddT[j] / dT[j]

    return RkcCoefficients(s, w0, w1, T, dT, ddT, a, b, mu, nu, mu_t, gamma_t, c, (1.0 + w0) / w1)


def step(
    F: Callable[[float, np.ndarray], np.ndarray],
    t: float,
    y: np.ndarray,
    tau: float,
    coef: RkcCoefficients,
    stages: Optional[List] = None,
    F0: Optional[np.ndarray] = None,
) -> np.ndarray:
    """One RKC(s) step of size tau from (t, y); returns y_{n+1} = Y_s.

    F is evaluated s times, at (t + c_j tau, Y_j) for j = 0..s-1 (s - 1 times
    when F0 = F(t, y) is given). If ``stages`` is a list, (t + c_j tau, Y_j,
    F_j) is appended for each evaluation, and (t + tau, Y_s, None) at the end.
    """
    s = coef.s
    Y0 = np.array(y, dtype=np.float64, copy=True)
    F0 = F(t, Y0) if F0 is None else np.asarray(F0, dtype=np.float64)
    if stages is not None:
        stages.append((t, Y0.copy(), F0.copy()))
    Yjm2 = Y0
    Yjm1 = Y0 + coef.mu_t[1] * tau * F0
    for j in range(2, s + 1):
        tj = t + coef.c[j - 1] * tau
        Fjm1 = F(tj, Yjm1)
        if stages is not None:
            stages.append((tj, Yjm1.copy(), Fjm1.copy()))
        Yj = (
            (1.0 - coef.mu[j] - coef.nu[j]) * Y0
            + coef.mu[j] * Yjm1
            + coef.nu[j] * Yjm2
            + coef.mu_t[j] * tau * Fjm1
            + coef.gamma_t[j] * tau * F0
        )
        Yjm2, Yjm1 = Yjm1, Yj
    if stages is not None:
        stages.append((t + tau, Yjm1.copy(), None))
    return Yjm1



# ----------------------------------------------------------------- adaptive
# Ref. [9] also controls the step: after a step from (t_n, y_n) to y_{n+1}
# with size tau it estimates the local error from the two end points and their
# slopes (a cubic Hermite comparison),
#     est = (12 (y_n - y_{n+1}) + 6 tau (F(t_n, y_n) + F(t_n + tau, y_{n+1}))) / 15,
# measures it in the weighted RMS norm
#     err = sqrt(mean_i (est_i / (atol + rtol max(|y_n,i|, |y_{n+1},i|)))^2),
# accepts the step when err <= 1 (F(t_{n+1}, y_{n+1}) is then the next step's
# first stage), and picks the next step size as
#     rejected:             tau <- 0.8 tau / err^(1/3)
#     accepted, first one:  tau <- tau max(0.1, min(10, 0.8 / err^(1/3)))
#     accepted, later:      tau <- tau max(0.1, min(10, 0.8 (tau / tau_prev) err_prev^(1/3) / err^(2/3)))
# (tau_prev, err_prev: size and error of the previous accepted step), clipped
# to [tau_min, tau_max] and to the end of the interval. The number of stages
# is the smallest s >= 2 whose stability boundary covers the step:
# beta(s) >= tau rho, with rho an upper bound of the spectral radius of the
# Jacobian at the step's start; beyond s_max the step is shortened instead.
# For eq. (2), rho = max over elements of sigma_e / eps_e (sigma the
# differential conductivity; pin P5's Rayleigh bound).


@dataclass
class AdaptiveRecord:
    t: float  # start of the attempted step
    tau: float
    s: int
    err: float
    accepted: bool


_BETA = {}


def beta(s: int) -> float:
    """Stability boundary (1 + w0) / w1 of RKC(s)."""
    if s not in _BETA:
        _BETA[s] = coefficients(s).beta
    return _BETA[s]


def stages_for(tau: float, rho: float, s_max: int):
    """(s, tau): the smallest s >= 2 with beta(s) >= tau rho, or s_max with tau
    shortened to beta(s_max) / rho when even s_max does not cover it."""
    if not rho > 0.0:
        return 2, tau
    for s in range(2, s_max + 1):
        if beta(s) >= tau * rho:
            return s, tau
    return s_max, beta(s_max) / rho


def error_estimate(y0, y1, f0, f1, tau):
    """Ref. [9]'s local error estimate of one step."""
    return (12.0 * (y0 - y1) + 6.0 * tau * (f0 + f1)) / 15.0


def error_norm(est, y0, y1, atol: float, rtol: float) -> float:
    """Weighted RMS norm of the estimate."""
    w = atol + rtol * np.maximum(np.abs(y0), np.abs(y1))
    return float(np.sqrt(np.mean((est / w) ** 2)))


def next_tau(tau, err, accepted, tau_prev=None, err_prev=None):
    """Step size after an attempt (ref. [9]'s controller, see above)."""
    if not accepted:
        return 0.8 * tau / err ** (1.0 / 3.0)
    if err == 0.0:
        return 10.0 * tau
    if tau_prev is None:
        fac = 0.8 / err ** (1.0 / 3.0)
    else:
        fac = 0.8 * (tau / tau_prev) * err_prev ** (1.0 / 3.0) / err ** (2.0 / 3.0)
    return tau * max(0.1, min(10.0, fac))


def adaptive(F, rho, t0: float, y0, t_end: float, tau0: float, atol: float, rtol: float, s_max: int = 250,
             tau_min: float = 0.0, tau_max: Optional[float] = None, max_attempts: int = 100000):
    """Integrate y' = F(t, y) from t0 to t_end with error-controlled RKC steps.

    rho(t, y): an upper bound of the Jacobian's spectral radius. Returns the
    accepted step-end states [(t_n, y_n)] (t0 first) and the record of every
    attempted step."""
    tau_max = (t_end - t0) if tau_max is None else tau_max
    t = t0
    y = np.array(y0, dtype=np.float64, copy=True)
    f = F(t, y)
    out = [(t, y.copy())]
    rec: List[AdaptiveRecord] = []
    tau = min(tau0, tau_max)
    tau_prev = err_prev = None
    while t < t_end:
        if len(rec) >= max_attempts:
            raise RuntimeError("adaptive RKC: too many attempts")
        last = tau >= t_end - t
        if last:
            tau = t_end - t
        s, tau_s = stages_for(tau, rho(t, y), s_max)
        if tau_s < tau:
            tau, last = tau_s, False
        y1 = step(F, t, y, tau, coefficients(s), F0=f)
        t1 = t_end if last else t + tau
        f1 = F(t1, y1)
        err = error_norm(error_estimate(y, y1, f, f1, tau), y, y1, atol, rtol)
        ok = err <= 1.0
        rec.append(AdaptiveRecord(t, tau, s, err, ok))
        if ok:
            t, y, f = t1, y1, f1
            out.append((t, y.copy()))
            new = next_tau(tau, err, True, tau_prev, err_prev)
            tau_prev, err_prev = tau, err
        else:
            new = next_tau(tau, err, False)
        if new < tau_min:
            raise RuntimeError("adaptive RKC: step size below tau_min")
        tau = min(new, tau_max)
    return out, rec
