"""Newton's method on the discrete weak form (Sec. 2.2), the oracle way:
assembled sparse tangent and a direct sparse solve per Newton step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A load step moves the prescribed (Dirichlet) values from g_old to g_new.
Evaluating the residual with g_new imposed directly puts a jump into the
boundary layer of cells; instead the first Newton correction of the step is
the linearised response to the increment dg = g_new - g_old:

    K_ff du_f = -R_f(u) - K_fc dg,   du_c = dg

(the standard treatment of inhomogeneous Dirichlet data in Newton's method);
later corrections have du_c = 0 and are damped by backtracking: the step
length is halved until det F > 0 at every quadrature point and ||R||
decreases (at most 12 halvings).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fem import Problem


def newton(problem: Problem, u0, dirichlet_dofs, dirichlet_values, atol=1e-8, max_iter=30):
    """Solve R(u) = 0 for the free dofs with u = dirichlet_values on the
    constrained dofs (which must be the problem's constrained dofs), starting
    from u0 (whose constrained entries hold the previous Dirichlet values).
    Returns (u, list of ||R|| before each correction and at the end)."""
    u = np.array(u0, dtype=np.float64, copy=True)
    free_problem = Problem(problem.mesh, problem.mu, problem.lam, elem_mu_lam=problem.elem_mu_lam,
                           model=problem.model)
    dg = np.zeros_like(u)
    dg[dirichlet_dofs] = np.asarray(dirichlet_values) - u[dirichlet_dofs]
    hist = []
    for it in range(max_iter + 1):
        R = problem.residual(u)
        if it > 0:
            rn = float(np.linalg.norm(R))
            hist.append(rn)
            if rn <= atol:
                return u, hist
        K = problem.assemble_tangent(u)
        rhs = -R
        if it == 0:
            rhs = rhs - free_problem.assemble_tangent(u) @ dg
            rhs[dirichlet_dofs] = dg[dirichlet_dofs]
        du = spla.spsolve(K.tocsc(), rhs)
        if it == 0:
            u += du
            continue
        rn = hist[-1]
        a = 1.0
        for _ in range(13):
            trial = u + a * du
            if problem.min_jacobian(trial) > 0.0 and np.linalg.norm(problem.residual(trial)) < rn:
                break
            a *= 0.5
        else:
            raise RuntimeError(f"oracle Newton line search failed: {hist}")
        u = trial
    raise RuntimeError(f"oracle Newton did not converge: {hist}")
