"""Oracle (test infrastructure only): the implicit chemistry solve of
multirate SDC mode 2 (eq. mrupdate2).

U* - h R(U*) = rhs for the chemistry source R (the REACT part of the
right-hand side).  R changes only the species densities (Section 2.1: the
total energy includes the formation enthalpies, so the chemistry has no
energy source), so the other components of U* are those of rhs; the species
densities come from Newton's method, cell by cell, with the Jacobian
dR/d(rho Y) assembled column by column from the oracle's forward-mode
(dual-number) tangent products.  Stopping rule: one iteration after the
first whose largest update is at most 1e-13 rho in every cell (at most 40).
"""
import numpy as np

import oracle


def implicit_reaction(om, rhs, h, dx, nthreads=0):
    rhs = np.asarray(rhs, dtype=np.float64)
    nU = rhs.shape[0]
    ns = nU - 5
    U = rhs.copy()
    rho = rhs[0]
    converged = False
    for _ in range(40):
        R = oracle.rhs(om, U, dx, parts=oracle.REACT, nthreads=nthreads)
        G = U[5:] - h * R[5:] - rhs[5:]
        J = np.empty((ns, ns) + rhs.shape[1:])
        for m in range(ns):
            w = np.zeros_like(U)
            w[5 + m] = 1.0
            _, jw = oracle.rhs_jvp(om, U, dx, w, parts=oracle.REACT, nthreads=nthreads)
            J[:, m] = -h * jw[5:]
            J[m, m] += 1.0
        # one small dense system per cell: J delta = G
        Jc = np.moveaxis(J.reshape(ns, ns, -1), 2, 0)
        Gc = np.moveaxis(G.reshape(ns, -1), 1, 0)[..., None]
        delta = np.moveaxis(np.linalg.solve(Jc, Gc)[..., 0], 0, 1).reshape(G.shape)
        U[5:] -= delta
        if converged:
            return U
        converged = bool(np.all(np.abs(delta).max(axis=0) <= 1e-13 * rho))
    raise RuntimeError("implicit chemistry solve did not converge")
