"""Pins of the oracle's spectral deferred corrections (Section 3)."""
import math

import numpy as np
import pytest

from conftest import read_table
from oracle import sdc


def test_gauss_lobatto_nodes_and_weights():
    np.testing.assert_allclose(sdc.gauss_lobatto(3), [0.0, 0.5, 1.0], atol=1e-15)
    r5 = 1 / math.sqrt(5)
    np.testing.assert_allclose(sdc.gauss_lobatto(4), [0.0, (1 - r5) / 2, (1 + r5) / 2, 1.0], atol=1e-15)
    r21 = math.sqrt(21) / 14
    np.testing.assert_allclose(sdc.gauss_lobatto(5), [0.0, 0.5 - r21, 0.5, 0.5 + r21, 1.0], atol=1e-15)
    # last row of Q is the quadrature rule: Simpson, 4-point and 5-point Lobatto
    np.testing.assert_allclose(sdc.q_matrix(sdc.gauss_lobatto(3))[-1], [1 / 6, 2 / 3, 1 / 6], atol=1e-15)
    np.testing.assert_allclose(sdc.q_matrix(sdc.gauss_lobatto(4))[-1], [1 / 12, 5 / 12, 5 / 12, 1 / 12], atol=1e-15)
    np.testing.assert_allclose(sdc.q_matrix(sdc.gauss_lobatto(5))[-1],
                               [1 / 20, 49 / 180, 16 / 45, 49 / 180, 1 / 20], atol=1e-15)


def test_gl3_node_to_node_matrix():
    S = sdc.s_matrix(sdc.gauss_lobatto(3))
    np.testing.assert_allclose(S, [[5 / 24, 1 / 3, -1 / 24], [-1 / 24, 1 / 3, 5 / 24]], atol=1e-15)
    # rows of S are differences of rows of Q
    Q = sdc.q_matrix(sdc.gauss_lobatto(5))
    S5 = sdc.s_matrix(sdc.gauss_lobatto(5))
    np.testing.assert_allclose(np.cumsum(S5, axis=0), Q, atol=1e-14)


def _dahlquist(z, nodes, K):
    f = lambda u, t: z * u
    return sdc.sdc_run(f, np.array([1.0 + 0j]), 0.0, 1.0, nodes, K, 1)[0]


def test_sdc_order_grows_by_one_per_sweep():
    # on u' = lam u each sweep raises the local order by one, up to the
    # order of the 4-node Lobatto rule (6)
    nodes = sdc.gauss_lobatto(4)
    lam = -1.3 + 0.4j
    for K in range(1, 7):
        errs = [abs(_dahlquist(lam * h, nodes, K) - np.exp(lam * h)) for h in (0.1, 0.05)]
        order = math.log2(errs[0] / errs[1])
        assert order == pytest.approx(K + 1, abs=0.15), (K, order)


def test_sdc_converges_to_collocation_pade_33():
    # Lobatto IIIA collocation with 4 nodes has the (3,3) Pade stability function
    nodes = sdc.gauss_lobatto(4)
    for z in (-0.5, -0.2 + 0.3j, 0.25j):
        num = 1 + z / 2 + z * z / 10 + z ** 3 / 120
        den = 1 - z / 2 + z * z / 10 - z ** 3 / 120
        assert abs(_dahlquist(z, nodes, 40) - num / den) < 1e-13


def test_mrsdc_with_coincident_nodes_is_single_rate_sdc():
    A = np.array([[-2.0, 1.0], [0.5, -1.0]])
    B = np.array([[-5.0, 0.0], [1.0, -8.0]])
    f1 = lambda u, t: A @ u
    f2 = lambda u, t: B @ u + np.array([math.sin(t), 0.0])
    u0 = np.array([1.0, 0.5])
    # fine nodes equal to the coarse nodes, one interpolating polynomial over
    # all of them (a type-(a) hierarchy of a single level)
    t1 = sdc.gauss_lobatto(4)
    t2, pieces = t1.copy(), [(0, 3)]
    mr = sdc.mrsdc_run(f1, f2, u0, 0.0, 0.1, t1, t2, pieces, 6, 3)
    sr = sdc.sdc_run(lambda u, t: f1(u, t) + f2(u, t), u0, 0.0, 0.1, t1, 6, 3)
    np.testing.assert_allclose(mr, sr, rtol=1e-14)


def test_mr_matrices_rows_integrate_constants_and_linears():
    for n_fine, rep in ((5, 1), (3, 2), (9, 1)):
        t1, t2, pieces = sdc.mr_nodes(4, n_fine, rep)
        S21, S22 = sdc.mr_matrices(t1, t2, pieces)
        dtau = np.diff(t2)
        np.testing.assert_allclose(S21.sum(1), dtau, atol=1e-15)
        np.testing.assert_allclose(S22.sum(1), dtau, atol=1e-15)
        np.testing.assert_allclose(S21 @ t1, np.diff(t2 ** 2) / 2, atol=1e-15)
        np.testing.assert_allclose(S22 @ t2, np.diff(t2 ** 2) / 2, atol=1e-15)


@pytest.mark.parametrize("row", read_table("table6_counts.txt"))
def test_evaluation_counts_reproduce_runtime_table(row):
    name, n_fine, rep, dt, n_ad, n_r = row[0], int(row[1]), int(row[2]), float(row[3]) * 1e-9, int(row[4]), int(row[5])
    nsteps = round(4.2e-7 / dt)
    assert abs(nsteps * dt - 4.2e-7) < 1e-15
    f = lambda u, t: -1e6 * u
    c1, c2 = sdc.Counter(f), sdc.Counter(f)
    if n_fine == 0:
        sdc.sdc_run(c1, np.ones(1), 0.0, dt, sdc.gauss_lobatto(3), 4, nsteps)
        assert (c1.n, c1.n) == (n_ad, n_r)
    else:
        t1, t2, pieces = sdc.mr_nodes(3, n_fine, rep)
        sdc.mrsdc_run(c1, c2, np.ones(1), 0.0, dt, t1, t2, pieces, 4, nsteps)
        assert (c1.n, c2.n) == (n_ad, n_r)


def test_mrsdc_fourth_order_with_three_coarse_nodes():
    # the multirate scheme's order is set by the coarse rule (GL3 -> 4),
    # whatever the fine nodes (multirate convergence table)
    A = np.array([[-1.0, 0.3], [0.2, -0.5]])
    B = np.array([[-20.0, 5.0], [3.0, -15.0]])
    f1 = lambda u, t: A @ u
    f2 = lambda u, t: B @ u
    u0 = np.array([1.0, -0.3])
    from scipy.linalg import expm
    exact = expm((A + B) * 0.4) @ u0
    for n_fine, rep in ((5, 1), (3, 2), (9, 1)):
        t1, t2, pieces = sdc.mr_nodes(3, n_fine, rep)
        errs = []
        for n in (8, 16, 32):
            u = sdc.mrsdc_run(f1, f2, u0, 0.0, 0.4 / n, t1, t2, pieces, 4, n)
            errs.append(np.abs(u - exact).max())
        rate = math.log2(errs[1] / errs[2])
        assert rate == pytest.approx(4.0, abs=0.3), (n_fine, rep, errs)


def test_residual_is_the_collocation_defect():
    """sdc_residual against the same defect formed independently: the
    polynomial through the node values of F integrated exactly over the step
    (numpy's polynomial fit and integral), eq. (residual)."""
    rng = np.random.default_rng(4)
    nodes = sdc.gauss_lobatto(4)
    q = sdc.s_matrix(nodes).sum(axis=0)
    dt = 0.7
    U0 = rng.standard_normal((3, 5)) + 2.0
    F = [rng.standard_normal((3, 5)) for _ in nodes]
    UM = rng.standard_normal((3, 5))
    Fa = np.stack(F)                                     # [node][comp][cell]
    coef = np.polynomial.polynomial.polyfit(nodes, Fa.reshape(len(nodes), -1), len(nodes) - 1)
    integ = np.polynomial.polynomial.polyval(1.0, np.polynomial.polynomial.polyint(coef)) - \
        np.polynomial.polynomial.polyval(0.0, np.polynomial.polynomial.polyint(coef))
    R = U0 + dt * integ.reshape(3, 5) - UM
    expect = max(np.abs(R[c]).max() / np.abs(U0[c]).max() for c in range(3))
    assert abs(sdc.sdc_residual(U0, F, UM, q, dt) - expect) <= 1e-13 * expect


def test_residual_exit_stops_at_the_collocation_solution():
    """With the early exit the sweeps stop once the residual stagnates, and
    the result is the collocation solution ((3,3) Pade value for GL4)."""
    nodes = sdc.gauss_lobatto(4)
    z = -0.5
    f = lambda u, t: z * u
    hist = []
    u = sdc.sdc_run(f, np.array([1.0]), 0.0, 1.0, nodes, 40, 1, residual_ratio=1.5, history=hist)
    pade = (1 + z / 2 + z * z / 10 + z ** 3 / 120) / (1 - z / 2 + z * z / 10 - z ** 3 / 120)
    assert abs(u[0] - pade) < 1e-14
    sweeps = [h[1] for h in hist if h[0] == "sweeps"][0]
    assert 5 < sweeps < 40
    rs = [h[2] for h in hist if h[0] != "sweeps"]
    assert rs[-1] < 1e-15 and rs[0] > 1e-4
    # residual_ratio = 0 keeps the fixed sweep count
    u40 = sdc.sdc_run(f, np.array([1.0]), 0.0, 1.0, nodes, 40, 1)
    np.testing.assert_array_equal(u40, sdc.sdc_run(f, np.array([1.0]), 0.0, 1.0, nodes, 40, 1, residual_ratio=0.0))
