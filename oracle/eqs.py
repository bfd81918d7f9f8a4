"""The semi-discrete EQS system and its time integration (test infrastructure only).

Eq. (2): M dx/dt + K(x)x = b, with M the permittivity-weighted P1 Laplacian,
K(x) the field-dependent conductivity matrix and b the contribution of the
inhomogeneous Dirichlet data. Reading of the Dirichlet treatment (the paper
only says b carries "inhomogeneous boundary conditions", Sec. II): the
Dirichlet nodes D are eliminated, the unknowns are the free nodes I, and with
x_bar = (Y on I, g(t) on D),
    M_II dY/dt = b(t) - [K(x_bar) x_bar]_I,   b(t) = -M_ID g'(t),
so the conductive coupling to the boundary is evaluated inside K(x_bar)x_bar
at each stage time and the capacitive coupling enters through b(t).

F(t, Y) = M_II^{-1}(b(t) - [K(x_bar)x_bar]_I) is what every RKC stage and the
explicit Euler step of eq. (3) evaluate. M_II is constant (Sec. II, the MRHS
observation); here it is factorised once (dense Cholesky when small) or
solved by SGS-PCG to a relative residual far below any GPU tolerance.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import fem, rkc

DENSE_LIMIT = 5000


def drive_values(amp, freq, phase, t):
    """g_k(t) = amp_k sin(2 pi freq_k t + phase_k) per drive k."""
    return amp * np.sin(2.0 * np.pi * freq * t + phase)


def drive_rates(amp, freq, phase, t):
    """g_k'(t) = 2 pi freq_k amp_k cos(2 pi freq_k t + phase_k)."""
    return 2.0 * np.pi * freq * amp * np.cos(2.0 * np.pi * freq * t + phase)


class EqsOracle:
    """FP64 reference for one EQS instance (a ``eqsgen.Case``)."""

    def __init__(self, case, solve_rtol: float = 1e-13, dense_limit: int = DENSE_LIMIT, solver: str = "sgs",
                 warm: bool = False, threads=None):
        """solver: "sgs" (serial symmetric Gauss-Seidel PCG) or "jacobi"
        (Jacobi PCG on OpenMP threads) for systems above dense_limit.
        warm: start every stage solve from the previous one's solution (the
        plain start vector of Sec. IV's multiple right-hand-side setting); the
        result still meets solve_rtol, so only the iteration count changes."""
        if solver not in ("sgs", "jacobi"):
            raise ValueError("solver must be 'sgs' or 'jacobi'")
        self.solver = solver
        self.warm = warm
        self.threads = threads
        self._prev = None
        self.case = case
        n = case.n_nodes
        is_dir = np.zeros(n, dtype=bool)
        is_dir[case.dir_nodes] = True
        self.dir_nodes = np.asarray(case.dir_nodes, dtype=np.int64)
        self.dir_drive = np.asarray(case.dir_drive, dtype=np.int64)
        self.free = np.flatnonzero(~is_dir)
        self.n_free = self.free.size
        M = fem.assemble_M(case)
        Mr = M[self.free]
        self.M = M
        self.M_II = Mr[:, self.free].tocsr()
        self.M_ID = Mr[:, self.dir_nodes].tocsr()
        self.solve_rtol = solve_rtol
        self.dense = self.n_free <= dense_limit
        if self.dense:
            self._chol = sla.cho_factor(self.M_II.toarray(), lower=True)
        self.last_iters = 0
        self.max_rate = 0.0  # max over evaluated stages of max_e sigma_e / eps_e

    # -- boundary data -----------------------------------------------------
    def g(self, t):
        c = self.case
        return drive_values(c.amp, c.freq, c.phase, t)[self.dir_drive]

    def gdot(self, t):
        c = self.case
        return drive_rates(c.amp, c.freq, c.phase, t)[self.dir_drive]

    def embed(self, Y, t):
        """x_bar: Y on the free nodes, g(t) on the Dirichlet nodes."""
        x = np.zeros(self.case.n_nodes)
        x[self.free] = Y
        x[self.dir_nodes] = self.g(t)
        return x

    def restrict(self, x):
        return np.asarray(x)[self.free]

    # -- operators ---------------------------------------------------------
    def b(self, t):
        """b(t) = -M_ID g'(t)."""
        return -(self.M_ID @ self.gdot(t))

    def Kx(self, t, Y):
        """[K(x_bar)x_bar]_I and max_e sigma_e/eps_e at the state (t, Y)."""
        y, rate = fem.apply_K(self.case, self.embed(Y, t), with_rate=True)
        return y[self.free], rate

    def stage_rhs(self, t, Y):
        """r = b(t) - [K(x_bar)x_bar]_I (the vector each stage hands to the solver)."""
        kx, rate = self.Kx(t, Y)
        self.max_rate = max(self.max_rate, rate)
        return self.b(t) - kx

    def solve(self, r, x0=None):
        """y = M_II^{-1} r (dense Cholesky, or PCG to solve_rtol from x0)."""
        if self.dense:
            self.last_iters = 0
            return sla.cho_solve(self._chol, r)
        if self.solver == "jacobi":
            res = fem.pcg_jacobi(self.M_II, r, x0=x0, rtol=self.solve_rtol, threads=self.threads)
        else:
            res = fem.pcg_sgs(self.M_II, r, x0=x0, rtol=self.solve_rtol)
        if res.status != 0:
            raise RuntimeError("oracle PCG failed: status %d relres %g" % (res.status, res.relres))
        self.last_iters = res.iters
        return res.x

    def F(self, t, Y):
        """F(t, Y) = M_II^{-1}(b(t) - [K(x_bar)x_bar]_I); with ``warm`` the
        solve starts from the previous evaluation's result."""
        y = self.solve(self.stage_rhs(t, Y), x0=self._prev if self.warm else None)
        if self.warm:
            self._prev = y
        return y

    # -- integrators -------------------------------------------------------
    def euler_step(self, t, Y, tau):
        """Eq. (3) as written: x^{n+1} = x^n + tau M^{-1}(b(t^{n+1}) - K(x^n)x^n)."""
        kx, _ = self.Kx(t, Y)
        return Y + tau * self.solve(self.b(t + tau) - kx)

    def check_stability(self, tau, coef):
        """Stability bound of RKC: tau * max sigma/eps <= beta(s).

        The generalised eigenvalues of the Jacobian of K(x)x against M lie in
        [min, max] of sigma_e/eps_e (element-wise Rayleigh quotients), so
        this is a sufficient condition for the step to be stable."""
        if tau * self.max_rate > coef.beta:
            raise RuntimeError(
                "RKC stability bound violated: tau*rho = %g > beta(%d) = %g"
                % (tau * self.max_rate, coef.s, coef.beta)
            )

    def spectral_bound(self, t, Y):
        """max_e sigma_e / eps_e at the state (t, Y): an upper bound of the
        spectral radius of M^{-1} times the Jacobian of K(x)x (element-wise
        Rayleigh quotients, pin P5), the rho of the adaptive stage choice."""
        _, rate = self.Kx(t, Y)
        return rate

    def rkc_adaptive(self, Y0, t0, t_end, tau0, atol, rtol, s_max=250, tau_max=None):
        """Error-controlled RKC from t0 to t_end (ref. [9]'s estimate and step
        control, stages from spectral_bound); returns the accepted step-end
        states [(t_n, Y_n)] and the record of every attempted step."""
        return rkc.adaptive(self.F, self.spectral_bound, t0, Y0, t_end, tau0, atol, rtol, s_max=s_max,
                            tau_max=tau_max)

    def rkc_trajectory(self, Y0, t0, tau, s, steps, stages=None, callback=None):
        """Integrate `steps` RKC(s) steps; returns the list of step-end states Y_n.

        If ``stages`` is a list, every step's stage record is appended to it."""
        coef = rkc.coefficients(s)
        Y = np.array(Y0, dtype=np.float64, copy=True)
        out = [Y.copy()]
        t = t0
        for n in range(steps):
            rec = [] if stages is not None else None
            Y = rkc.step(self.F, t, Y, tau, coef, rec)
            self.check_stability(tau, coef)
            t = t0 + (n + 1) * tau
            out.append(Y.copy())
            if stages is not None:
                stages.append(rec)
            if callback is not None:
                callback(n, t, Y)
        return out
