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
) -> np.ndarray:
    """One RKC(s) step of size tau from (t, y); returns y_{n+1} = Y_s.

    F is evaluated s times, at (t + c_j tau, Y_j) for j = 0..s-1. If ``stages``
    is a list, (t + c_j tau, Y_j, F_j) is appended for each evaluation, and
    (t + tau, Y_s, None) at the end.
    """
    s = coef.s
    Y0 = np.array(y, dtype=np.float64, copy=True)
    F0 = F(t, Y0)
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

