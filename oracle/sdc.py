"""Oracle (test infrastructure only): spectral deferred corrections.

Plain NumPy transcription of Section 3 of the paper:
  * collocation nodes and the integration matrices Q (integrals from the
    step start to each node) and S (node-to-node integrals) from exact
    integrals of the Lagrange interpolating polynomials (eqs. gaussapp,
    compact);
  * single-rate SDC: spread the initial value, then K sweeps of the
    forward-Euler correction (eq. expsdc), f(U_0) recycled across steps;
  * multirate SDC, mode 1 (eq. mrupdate): coarse component f1 on the coarse
    nodes, fine component f2 on the fine nodes, coarse term frozen at the
    coarse node to the left, p = floor(q / (M2/M1)); fine nodes of type (b)
    (one rule per coarse interval) or (c) (a rule repeated R times per coarse
    interval), with piecewise-polynomial S_{2,2} (figure on MRSDC nodes).
Function evaluations are counted (evaluation counts of the runtime table).
"""
import numpy as np
from numpy.polynomial import legendre


def gauss_lobatto(n):
    """n Gauss-Lobatto nodes on [0, 1]: the end points and the roots of P'_{n-1}."""
    if n < 2:
        raise ValueError("need at least two nodes")
    inner = legendre.Legendre.basis(n - 1).deriv().roots() if n > 2 else np.array([])
    x = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    return 0.5 * (x + 1.0)


def lagrange_integral(nodes, j, a, b):
    """int_a^b l_j(t) dt for the Lagrange basis polynomial l_j of `nodes`,
    by Gauss-Legendre quadrature (exact for this degree) with l_j evaluated in
    product form."""
    x, w = legendre.leggauss(len(nodes))
    t = 0.5 * (a + b) + 0.5 * (b - a) * x
    others = np.delete(nodes, j)
    lj = np.prod((t[:, None] - others[None, :]) / (nodes[j] - others[None, :]), axis=1)
    return 0.5 * (b - a) * np.dot(w, lj)


def q_matrix(nodes):
    """Q[m-1][j] = int_{tau_0}^{tau_m} l_j, m = 1..M (normalised step)."""
    M = len(nodes) - 1
    return np.array([[lagrange_integral(nodes, j, nodes[0], nodes[m])
                      for j in range(M + 1)] for m in range(1, M + 1)])


def s_matrix(nodes):
    """S[m][j] = int_{tau_m}^{tau_{m+1}} l_j, m = 0..M-1 (normalised step)."""
    M = len(nodes) - 1
    return np.array([[lagrange_integral(nodes, j, nodes[m], nodes[m + 1])
                      for j in range(M + 1)] for m in range(M)])


def mr_nodes(n_coarse, n_fine, repeat=1):
    """Coarse nodes (Gauss-Lobatto, n_coarse) and fine nodes: n_fine Gauss-Lobatto
    nodes on each of `repeat` equal sub-intervals of every coarse interval
    (type (b) for repeat = 1, type (c) otherwise).  Returns (t1, t2, pieces)
    where pieces lists the fine-node index ranges of each polynomial piece."""
    t1 = gauss_lobatto(n_coarse)
    g = gauss_lobatto(n_fine)
    t2 = [0.0]
    pieces = []
    for p in range(n_coarse - 1):
        a, b = t1[p], t1[p + 1]
        for r in range(repeat):
            lo = a + (b - a) * r / repeat
            hi = a + (b - a) * (r + 1) / repeat
            start = len(t2) - 1
            t2.extend(lo + (hi - lo) * g[1:])
            pieces.append((start, len(t2) - 1))
    t2 = np.array(t2)
    t2[-1] = 1.0
    return t1, t2, pieces


def mr_matrices(t1, t2, pieces):
    """S_{2,1} (M2 x (M1+1)): integrals over fine intervals of the coarse
    interpolant; S_{2,2} (M2 x (M2+1)): of the piecewise fine interpolant."""
    M1, M2 = len(t1) - 1, len(t2) - 1
    S21 = np.array([[lagrange_integral(t1, j, t2[q], t2[q + 1]) for j in range(M1 + 1)]
                    for q in range(M2)])
    S22 = np.zeros((M2, M2 + 1))
    for lo, hi in pieces:
        loc = t2[lo:hi + 1]
        for q in range(lo, hi):
            for jj in range(hi - lo + 1):
                S22[q, lo + jj] = lagrange_integral(loc, jj, t2[q], t2[q + 1])
    return S21, S22


class Counter:
    def __init__(self, f):
        self.f = f
        self.n = 0

    def __call__(self, U, t):
        self.n += 1
        return self.f(U, t)


def sdc_residual(U0, F, UM, q, dt):
    """Size of the SDC residual R = U_0 + dt q.F - U_M (eq. residual), q the
    last row of the integration matrix: the largest over state components of
    max|R_c| / max|U_0,c| (the paper leaves the norm open; this reading makes
    it independent of each component's units)."""
    R = U0 + dt * sum(qj * Fj for qj, Fj in zip(q, F)) - UM
    nc = R.shape[0]
    r = np.abs(R).reshape(nc, -1).max(axis=1)
    u = np.abs(U0).reshape(nc, -1).max(axis=1)
    return float(max(r[c] / u[c] for c in range(nc) if u[c] > 0))


def sdc_run(f, U0, t0, dt, nodes, K, nsteps, perturb=None, residual_ratio=0.0, history=None):
    """Single-rate SDC: nsteps steps of K sweeps each (eq. expsdc).
    f(U, t) -> dU/dt.  Returns the final state.  perturb (optional) is
    applied to every new node state (used to measure rounding sensitivity).

    residual_ratio > 1: after every sweep but a step's last the residual of
    eq. (residual) is measured, and the step's remaining sweeps are skipped
    once |R^{k-1}| / |R^k| < residual_ratio (the sweeps have stopped
    improving the collocation residual).  history (a list, optional)
    receives (step, sweep, |R|) of every measurement and ("sweeps", n) per
    step."""
    perturb = perturb or (lambda U: U)
    M = len(nodes) - 1
    S = s_matrix(nodes)
    q = S.sum(axis=0)
    dtau = np.diff(nodes) * dt
    U0 = np.array(U0, copy=True)
    F0 = f(U0, t0)
    for n in range(nsteps):
        tn = t0 + n * dt
        times = tn + nodes * dt
        Uk = [U0] * (M + 1)
        Fk = [F0] * (M + 1)
        rprev = None
        for k in range(K):
            Un = [U0]
            Fn = [F0]
            for m in range(M):
                if m > 0:
                    Fn.append(f(Un[m], times[m]))
                SF = sum(S[m, j] * Fk[j] for j in range(M + 1))
                Un.append(perturb(Un[m] + dtau[m] * (Fn[m] - Fk[m]) + dt * SF))
            Fn.append(f(Un[M], times[M]))
            Uk, Fk = Un, Fn
            if residual_ratio > 0 and k < K - 1:
                r = sdc_residual(U0, Fk, Uk[M], q, dt)
                if history is not None:
                    history.append((n, k, r))
                if r == 0.0 or (rprev is not None and rprev < residual_ratio * r):
                    break
                rprev = r
        if history is not None:
            history.append(("sweeps", k + 1))
        U0, F0 = Uk[M], Fk[M]
    return U0


def mrsdc_run(f1, f2, U0, t0, dt, t1, t2, pieces, K, nsteps, perturb=None):
    """Multirate SDC, mode 1 (eq. mrupdate): explicit forward-Euler corrections
    of both components on the fine nodes, f1 frozen at the coarse node to the
    left.  Returns the final state.  perturb as in sdc_run."""
    perturb = perturb or (lambda U: U)
    M1, M2 = len(t1) - 1, len(t2) - 1
    r = M2 // M1
    assert r * M1 == M2
    S21, S22 = mr_matrices(t1, t2, pieces)
    dtq = np.diff(t2) * dt
    U0 = np.array(U0, copy=True)
    F1_0 = f1(U0, t0)
    F2_0 = f2(U0, t0)
    for n in range(nsteps):
        tn = t0 + n * dt
        F1k = [F1_0] * (M1 + 1)
        F2k = [F2_0] * (M2 + 1)
        for k in range(K):
            F1n = [F1_0] + [None] * M1
            F2n = [F2_0] + [None] * M2
            U = U0
            for q in range(M2):
                p = q // r
                if q > 0:
                    F2n[q] = f2(U, tn + t2[q] * dt)
                    if q % r == 0:
                        F1n[p] = f1(U, tn + t1[p] * dt)
                S = sum(S22[q, j] * F2k[j] for j in range(M2 + 1)) + \
                    sum(S21[q, j] * F1k[j] for j in range(M1 + 1))
                U = perturb(U + dtq[q] * (F1n[p] - F1k[p]) + dtq[q] * (F2n[q] - F2k[q]) + dt * S)
            F2n[M2] = f2(U, tn + dt)
            F1n[M1] = f1(U, tn + dt)
            F1k, F2k = F1n, F2n
        U0, F1_0, F2_0 = U, F1k[M1], F2k[M2]
    return U0


def mrsdc2_run(f1, solve1, f2, U0, t0, dt, t1, t2, pieces, K, nsteps, perturb=None):
    """Multirate SDC, mode 2 (eq. mrupdate2): the stiff component f1 (the
    chemistry) on the coarse nodes t1, treated implicitly; f2 (advection-
    diffusion) on the fine nodes t2 with forward-Euler corrections.

    In coarse interval p the fine updates of eq. (mrupdate2) hold
    f1(U^{k+1}_{p+1}) fixed.  It is obtained first, by an implicit solve over
    the interval: U* = U^{k+1}_p + dt_p (f1(U*) - F1^k_{p+1})
    + dt sum_{q in p} (S21 F1^k + S22 F2^k)_q, i.e. one backward-Euler step of
    f1 (first-order BDF) with the interval's explicit update as forcing and
    the fine correction terms of f2 lagged; solve1(rhs, h) returns U* with
    U* - h f1(U*) = rhs.  X = f1(U*) is the new F1 at node p+1, and the fine
    sub-steps of the interval use it.  At the SDC fixed point U* is the
    interval's end state, so the sweeps converge to the multirate collocation
    solution, as in mode 1.  f1 of the end state starts the next step, f2 of
    it is the last sweep's.  perturb as in sdc_run."""
    perturb = perturb or (lambda U: U)
    M1, M2 = len(t1) - 1, len(t2) - 1
    r = M2 // M1
    assert r * M1 == M2
    S21, S22 = mr_matrices(t1, t2, pieces)
    dtq = np.diff(t2) * dt
    dtp = np.diff(t1) * dt
    U0 = np.array(U0, copy=True)
    F1_0 = f1(U0, t0)
    F2_0 = f2(U0, t0)
    for n in range(nsteps):
        tn = t0 + n * dt
        F1k = [F1_0] * (M1 + 1)
        F2k = [F2_0] * (M2 + 1)
        for k in range(K):
            F1n = [F1_0] + [None] * M1
            F2n = [F2_0] + [None] * M2
            U = U0
            for p in range(M1):
                qs = range(p * r, (p + 1) * r)
                Sq = {q: dt * (sum(S22[q, j] * F2k[j] for j in range(M2 + 1)) +
                               sum(S21[q, j] * F1k[j] for j in range(M1 + 1))) for q in qs}
                rhs = U - dtp[p] * F1k[p + 1] + sum(Sq[q] for q in qs)
                X = f1(solve1(rhs, dtp[p]), tn + t1[p + 1] * dt)
                F1n[p + 1] = X
                for q in qs:
                    if q > 0:
                        F2n[q] = f2(U, tn + t2[q] * dt)
                    U = perturb(U + dtq[q] * (X - F1k[p + 1]) + dtq[q] * (F2n[q] - F2k[q]) + Sq[q])
            F2n[M2] = f2(U, tn + dt)
            F1k, F2k = F1n, F2n
        U0, F1_0, F2_0 = U, f1(U, tn + dt), F2k[M2]
    return U0
