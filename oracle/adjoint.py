"""Oracle (test infrastructure only): reference gradients of the right-hand
side and of the SDC step, from their plain definitions.

  * Vector-Jacobian product of the right-hand side (eq. cns with the
    discretisation of Section 2.2):
        (J^T v)[q, c] = sum_i sum_p v[p, i] d f_p(i) / d U_q(c),
    each column J e_(q,c) taken from the forward-mode dual-number product of
    the oracle right-hand side.  f at an output cell depends on U only inside
    the 9x9x9 cube centred on it (nine-point lines, and mixed terms that
    differentiate the velocity gradient along a second direction), so the
    column of input cell c is evaluated only on the cube around c, and input
    cells whose cubes do not overlap share one dual seed.
  * Gradient with respect to ln A_j of every reaction: only the chemistry
    source depends on A, so each entry is one product with wA = e_j on the
    chemistry part.
  * Tangent of the single-rate SDC step (eq. expsdc): the step only forms
    linear combinations of states and right-hand-side values, so running the
    oracle SDC on the pair (U, dU) with the pair function
    (f(U), J(U) dU + J_A dlnA) gives the step and its directional derivative.
"""
import numpy as np

from . import ALL, REACT, rhs_jvp, rhs_jvp_cells
from . import sdc as osdc

HALF = 4   # half-width of the dependence cube of one output cell


def support(c, shape):
    """Distinct interior cells (x, y, z) of the periodic box `shape` = (nz, ny,
    nx) whose right-hand side can depend on input cell c = (x, y, z)."""
    nz, ny, nx = shape
    r = np.arange(-HALF, HALF + 1)
    xs = np.unique((c[0] + r) % nx)
    ys = np.unique((c[1] + r) % ny)
    zs = np.unique((c[2] + r) % nz)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def group_cells(cells, shape):
    """Greedy partition of input cells into groups whose supports are
    pairwise disjoint."""
    groups = []   # (cells, set of covered output cells)
    for c in cells:
        sup = {tuple(s) for s in support(c, shape)}
        for g in groups:
            if not (g[1] & sup):
                g[0].append(tuple(c))
                g[1].update(sup)
                break
        else:
            groups.append(([tuple(c)], set(sup)))
    return [g[0] for g in groups]


def rhs_vjp(om, U, dx, vbar, parts=ALL, cells=None, nthreads=0):
    """(J^T vbar)[q, c] for the listed input cells (array [n][3] of x, y, z;
    None = every cell, result [nU][nz][ny][nx]); otherwise [n][nU]."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    vbar = np.ascontiguousarray(vbar, dtype=np.float64)
    nU, nz, ny, nx = U.shape
    shape = (nz, ny, nx)
    full = cells is None
    if full:
        Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        cells = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    cells = [tuple(int(v) for v in c) for c in np.asarray(cells)]
    index = {c: n for n, c in enumerate(cells)}
    out = np.zeros((len(cells), nU))
    for group in group_cells(cells, shape):
        sups = [support(c, shape) for c in group]
        allsup = np.concatenate(sups)
        for q in range(nU):
            w = np.zeros_like(U)
            for c in group:
                w[q, c[2], c[1], c[0]] = 1.0
            jw = rhs_jvp_cells(om, U, dx, w, allsup, parts=parts, nthreads=nthreads)
            at = 0
            for c, sup in zip(group, sups):
                vs = vbar[:, sup[:, 2], sup[:, 1], sup[:, 0]].T      # [len(sup)][nU]
                out[index[c], q] = np.sum(vs * jw[at:at + len(sup)])
                at += len(sup)
    if full:
        return out.T.reshape(nU, nz, ny, nx)
    return out


def rhs_vjp_lnA(om, U, dx, vbar, nr, nthreads=0):
    """d <vbar, rhs> / d ln A_j for every reaction j."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    zero = np.zeros_like(U)
    g = np.zeros(nr)
    for j in range(nr):
        wA = np.zeros(nr)
        wA[j] = 1.0
        _, jv = rhs_jvp(om, U, dx, zero, wA, parts=REACT, nthreads=nthreads)
        g[j] = np.sum(vbar * jv)
    return g


def sdc_tangent(om, U0, dx, dt, n_coarse, sweeps, nsteps, wU, wA=None, nthreads=0):
    """Single-rate SDC step(s) and their directional derivative:
    returns (U_N, dU_N) for the direction (wU, wA)."""
    U0 = np.asarray(U0, dtype=np.float64)
    nU = U0.shape[0]

    def fpair(X, t):
        out, jv = rhs_jvp(om, X[:nU], dx, X[nU:], wA, parts=ALL, nthreads=nthreads)
        return np.concatenate([out, jv])

    X0 = np.concatenate([U0, np.asarray(wU, dtype=np.float64)])
    XN = osdc.sdc_run(fpair, X0, 0.0, dt, osdc.gauss_lobatto(n_coarse), sweeps, nsteps)
    return XN[:nU], XN[nU:]
