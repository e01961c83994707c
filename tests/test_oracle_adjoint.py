"""Pins of the oracle's reference gradients (CPU).

The oracle's vector-Jacobian product is assembled from forward-mode
dual-number columns; these tests tie it to things other than itself:
central differences of the plain right-hand side, the adjoint identity
<v, J w> = <J^T v, w> against whole-box products, the grouping of input
cells with disjoint dependence cubes, and central differences of the SDC
step (eq. expsdc) for the tangent SDC.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint as OA
from synth import fields, mechanism

DX = 1e-4


def _state(kind, shape, seed):
    mech = mechanism.load(kind)
    om = oracle.Mechanism(mech)
    U = oracle.prim_to_cons(om, fields.sines(shape, DX, mech["ns"], seed))
    return mech, om, U


def test_vjp_adjoint_identity_on_a_small_box():
    mech, om, U = _state("mech9", (4, 5, 6), 11)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(U.shape)
    scale = np.abs(U).max(axis=(1, 2, 3), keepdims=True)
    for parts in (oracle.HYP, oracle.DIFF, oracle.REACT):
        g = OA.rhs_vjp(om, U, DX, v, parts=parts)
        for _ in range(2):
            w = rng.standard_normal(U.shape) * scale
            _, jw = oracle.rhs_jvp(om, U, DX, w, parts=parts)
            a, b = np.sum(v * jw), np.sum(g * w)
            assert abs(a - b) <= 1e-12 * abs(a), (parts, a, b)


def test_vjp_entries_match_central_differences():
    """(J^T v)[q, c] against central differences of <v, rhs> over the cells
    whose right-hand side can depend on cell c."""
    mech, om, U = _state("mech9", (10, 10, 10), 12)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(U.shape)
    cells = np.array([[3, 4, 5], [0, 9, 2]])
    g = OA.rhs_vjp(om, U, DX, v, cells=cells)
    for n, c in enumerate(cells):
        sup = OA.support(c, U.shape[1:])
        for q in (0, 2, 4, 5, 9):
            h = 1e-6 * np.abs(U[q]).max()
            vals = []
            for sgn in (1.0, -1.0):
                Up = U.copy()
                Up[q, c[2], c[1], c[0]] += sgn * h
                f = oracle.rhs_cells(om, Up, DX, sup)
                vals.append(np.sum(v[:, sup[:, 2], sup[:, 1], sup[:, 0]].T * f))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - g[n, q]) <= 1e-5 * max(abs(g[n, q]), abs(fd)) + 1e-9, (c, q, fd, g[n, q])


def test_grouped_cells_equal_cells_taken_alone():
    mech, om, U = _state("mech9", (5, 6, 18), 13)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(U.shape)
    cells = np.array([[0, 2, 1], [9, 2, 1], [4, 0, 3]])
    assert len(OA.group_cells(cells, U.shape[1:])) == 2
    together = OA.rhs_vjp(om, U, DX, v, cells=cells)
    for n, c in enumerate(cells):
        alone = OA.rhs_vjp(om, U, DX, v, cells=c[None])
        np.testing.assert_allclose(together[n], alone[0], rtol=1e-14, atol=0)


def test_lnA_gradient_matches_central_differences_of_A():
    mech, om, U = _state("mech9", (4, 4, 4), 14)
    rng = np.random.default_rng(4)
    v = rng.standard_normal(U.shape)
    g = OA.rhs_vjp_lnA(om, U, DX, v, mech["nr"])
    for j in (0, 5, 17):
        vals = []
        for sgn in (1.0, -1.0):
            m2 = dict(mech)
            A = np.array(mech["A"], dtype=np.float64)
            A[j] *= np.exp(sgn * 1e-6)
            m2["A"] = A
            # only the chemistry source depends on A
            f = oracle.rhs(oracle.Mechanism(m2), U, DX, parts=oracle.REACT)
            vals.append(np.sum(v * f))
        fd = (vals[0] - vals[1]) / 2e-6
        assert abs(fd - g[j]) <= 1e-6 * abs(g[j]) + 1e-9 * abs(g).max(), (j, fd, g[j])


def test_sdc_tangent_matches_central_differences():
    mech, om, U = _state("mech9", (4, 4, 5), 15)
    dt = 2e-9
    rng = np.random.default_rng(5)
    w = rng.standard_normal(U.shape) * np.abs(U).max(axis=(1, 2, 3), keepdims=True)
    UN, dUN = OA.sdc_tangent(om, U, DX, dt, 4, 2, 2, w)
    h = 1e-7

    def step(X):
        from oracle import sdc
        return sdc.sdc_run(lambda V, t: oracle.rhs(om, V, DX), X, 0.0, dt, sdc.gauss_lobatto(4), 2, 2)

    fd = (step(U + h * w) - step(U - h * w)) / (2 * h)
    np.testing.assert_array_equal(UN, step(U))
    for q in range(U.shape[0]):
        assert np.abs(fd[q] - dUN[q]).max() <= 1e-6 * np.abs(dUN[q]).max(), q


@pytest.mark.parametrize("nsteps", [1, 2])
def test_sdc_tangent_is_linear_in_the_direction(nsteps):
    """Two directions and their sum: the tangent is linear (checks that the
    pair function keeps U and dU apart)."""
    mech, om, U = _state("mech9", (4, 4, 4), 16)
    dt = 2e-9
    rng = np.random.default_rng(6)
    scale = np.abs(U).max(axis=(1, 2, 3), keepdims=True)
    w1, w2 = rng.standard_normal(U.shape) * scale, rng.standard_normal(U.shape) * scale
    _, d1 = OA.sdc_tangent(om, U, DX, dt, 3, 2, nsteps, w1)
    _, d2 = OA.sdc_tangent(om, U, DX, dt, 3, 2, nsteps, w2)
    _, d12 = OA.sdc_tangent(om, U, DX, dt, 3, 2, nsteps, w1 + w2)
    for q in range(U.shape[0]):
        assert np.abs(d12[q] - d1[q] - d2[q]).max() <= 1e-12 * np.abs(d12[q]).max()
