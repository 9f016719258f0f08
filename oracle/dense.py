"""Dense FP64 tools for tiny meshes -- TEST INFRASTRUCTURE ONLY.

* ``dense_hessian``: the true energy Hessian over free DOFs, assembled
  column by column from the oracle's Neo-Hookean Hessian-vector product (or
  from central differences of the analytic gradient for the corotated model);
* ``newton``: full Newton with a backtracking line search on the total
  energy, used as an independent check that the Gauss-Seidel iteration
  reaches the equilibrium of Eq. (fem_qs);
* ``adjoint_dense``: the adjoint vector by a direct dense solve;
* ``linear_fem_stiffness``: textbook small-strain stiffness from the linear
  elasticity density of Eq. (le), psi = mu tr(eps^2) + lambda/2 tr(eps)^2,
  assembled with numpy from per-tet B matrices (no oracle code involved).
"""
from __future__ import annotations

import numpy as np

from . import COROTATED, energy_gradient, hvp, residual


def free_dofs(op):
    free = np.nonzero(op.is_dir == 0)[0]
    return free, (3 * free[:, None] + np.arange(3)[None, :]).reshape(-1)


def dense_hessian(op, x):
    """Full 3nv x 3nv energy Hessian at x."""
    n = 3 * op.nv
    H = np.zeros((n, n))
    if op.model == COROTATED:
        h = 1e-6
        for k in range(n):
            xp = np.array(x, dtype=np.float64).reshape(-1)
            xm = xp.copy()
            xp[k] += h
            xm[k] -= h
            H[:, k] = (energy_gradient(op, xp.reshape(-1, 3)).reshape(-1)
                       - energy_gradient(op, xm.reshape(-1, 3)).reshape(-1)) / (2 * h)
        return 0.5 * (H + H.T)
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        H[:, k] = hvp(op, x, e.reshape(-1, 3)).reshape(-1)
    return H


def newton(op, x0, tol=1e-12, max_iter=100):
    """Newton on the free DOFs with an Armijo backtracking line search.
    Returns (x, iterations, final relative residual)."""
    x = np.array(x0, dtype=np.float64).reshape(-1, 3)
    x[op.dirichlet_idx] = op.dirichlet_x
    _, fd = free_dofs(op)
    r0, E, _ = residual(op, x)
    if r0 == 0.0:
        return x, 0, 0.0
    for it in range(max_iter):
        g = energy_gradient(op, x).reshape(-1)[fd]
        rn = np.linalg.norm(g)
        if rn <= tol * r0:
            return x, it, rn / r0
        H = dense_hessian(op, x)[np.ix_(fd, fd)]
        try:
            w, Q = np.linalg.eigh(H)
            w = np.maximum(w, 1e-8 * max(1.0, np.abs(w).max()))
            d = -(Q @ ((Q.T @ g) / w))
        except np.linalg.LinAlgError:
            d = -g
        _, E0, _ = residual(op, x)
        t = 1.0
        while True:
            xt = x.copy().reshape(-1)
            xt[fd] += t * d
            xt = xt.reshape(-1, 3)
            _, Et, _ = residual(op, xt)
            if Et <= E0 + 1e-4 * t * float(g @ d) or t < 1e-12:
                break
            # near the minimum energy differences drop below round-off: accept
            # a step that is flat in energy to round-off and reduces |g|
            if Et <= E0 + 1e-13 * abs(E0) and \
                    np.linalg.norm(energy_gradient(op, xt).reshape(-1)[fd]) < rn:
                break
            t *= 0.5
        x = xt
    g = energy_gradient(op, x).reshape(-1)[fd]
    return x, max_iter, np.linalg.norm(g) / r0


def adjoint_dense(op, x, dL_dx):
    """Solve H_FF lam_F = dL/dx_F; returns lam [nv, 3] with zero Dirichlet rows."""
    _, fd = free_dofs(op)
    H = dense_hessian(op, x)[np.ix_(fd, fd)]
    lam = np.zeros(3 * op.nv)
    lam[fd] = np.linalg.solve(H, np.asarray(dL_dx, np.float64).reshape(-1)[fd])
    return lam.reshape(-1, 3)


def linear_fem_stiffness(X, tets, mu, lam):
    """Global stiffness of linear elasticity (Eq. le) on linear tets."""
    X = np.asarray(X, np.float64)
    nv = X.shape[0]
    K = np.zeros((3 * nv, 3 * nv))
    mu = np.broadcast_to(mu, (tets.shape[0],))
    lam = np.broadcast_to(lam, (tets.shape[0],))
    # elasticity tensor in Voigt form (xx, yy, zz, yz, xz, xy), engineering shear
    for e, t in enumerate(tets):
        P = np.hstack([np.ones((4, 1)), X[t]])
        Cinv = np.linalg.inv(P)          # rows 1..3 hold the shape-function gradients
        vol = abs(np.linalg.det(P)) / 6.0
        grads = Cinv[1:, :].T            # [4, 3]
        B = np.zeros((6, 12))
        for a in range(4):
            gx, gy, gz = grads[a]
            B[:, 3 * a:3 * a + 3] = [[gx, 0, 0], [0, gy, 0], [0, 0, gz],
                                     [0, gz, gy], [gz, 0, gx], [gy, gx, 0]]
        D = np.zeros((6, 6))
        D[:3, :3] = lam[e]
        D[:3, :3] += 2 * mu[e] * np.eye(3)
        D[3:, 3:] = mu[e] * np.eye(3)
        Ke = vol * B.T @ D @ B
        idx = (3 * np.asarray(t)[:, None] + np.arange(3)[None, :]).reshape(-1)
        K[np.ix_(idx, idx)] += Ke
    return K
