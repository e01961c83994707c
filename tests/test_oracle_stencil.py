"""Pins of the oracle's spatial operators against facts the paper and the
mathematics fix (Section 2.2 and the stencil appendix)."""
import math
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

from conftest import read_table

PARAMS = {r[0]: (float(Fraction(r[1])), float(Fraction(r[2]))) for r in read_table("stencil_params.txt")}
SMC = PARAMS["SMC"]


def test_first_derivative_exact_on_polynomials_degree_8(orc):
    rng = np.random.default_rng(0)
    x0, dx = 0.3, 0.1
    xs = x0 + dx * np.arange(-4, 5)
    for deg in range(9):
        c = rng.standard_normal(deg + 1)
        P = np.polynomial.Polynomial(c)
        got = orc.d1_point(P(xs), dx)
        assert got == pytest.approx(P.deriv()(x0), rel=1e-11, abs=1e-11)


def test_first_derivative_leading_error_term(orc):
    # u = x^9/9! at 0 with dx = 1: the eighth-order centred difference has
    # error -u^(9) dx^8 / 630 and this u has no higher derivatives.
    s = np.arange(-4, 5, dtype=np.float64)
    got = orc.d1_point(s ** 9 / math.factorial(9), 1.0)
    assert got == pytest.approx(-1.0 / 630.0, rel=1e-12)


@pytest.mark.parametrize("name", ["SMC", "ZERO", "OPTIMAL", "random"])
def test_narrow_exact_when_deg_a_plus_deg_u_at_most_9(orc, name):
    rng = np.random.default_rng(1)
    m47, m48 = PARAMS[name] if name != "random" else tuple(rng.uniform(-0.1, 0.1, 2))
    x0, dx = 0.2, 0.1
    xs = x0 + dx * np.arange(-4, 5)
    for da in range(10):
        for du in range(0, 10 - da):
            A = np.polynomial.Polynomial(rng.standard_normal(da + 1))
            Uu = np.polynomial.Polynomial(rng.standard_normal(du + 1))
            exact = (A * Uu.deriv()).deriv()(x0)
            got = orc.narrow_point(A(xs), Uu(xs), dx, m47, m48)
            scale = 1.0 + abs(exact)
            assert abs(got - exact) <= 1e-8 * scale, (da, du, got, exact)


@pytest.mark.parametrize("name", ["SMC", "ZERO", "OPTIMAL"])
def test_narrow_truncation_error_matches_printed_coefficients(orc, name):
    # a = x^n/n!, u = x^(10-n)/(10-n)! at x = 0, dx = 1: the exact value is 0
    # and every error term of eq. (truncerror) vanishes except the n-th,
    # whose coefficient multiplies dx^8 = 1.
    m47, m48 = (Fraction(v) for v in read_table("stencil_params.txt")[["SMC", "ZERO", "OPTIMAL"].index(name)][1:])
    s = np.arange(-4, 5, dtype=np.float64)
    for row in read_table("truncerror.txt"):
        n = int(row[0])
        coef = Fraction(row[1]) + Fraction(row[2]) * m47 + Fraction(row[3]) * m48
        a = s ** n / math.factorial(n)
        u = s ** (10 - n) / math.factorial(10 - n)
        got = orc.narrow_point(a, u, 1.0, float(m47), float(m48))
        assert got == pytest.approx(float(coef), rel=1e-9, abs=1e-13), (n, got, float(coef))


def test_smc_parameters_null_the_mixed_fifth_and_sixth_terms():
    # the SMC choice is the vertex where the a^(5)u^(5) and a^(6)u^(4) terms vanish
    rows = {int(r[0]): r for r in read_table("truncerror.txt")}
    m47, m48 = (Fraction(v) for v in read_table("stencil_params.txt")[0][1:])
    for n in (5, 6):
        r = rows[n]
        assert Fraction(r[1]) + Fraction(r[2]) * m47 + Fraction(r[3]) * m48 == 0


def test_narrow_constant_coefficient_is_textbook_second_difference(orc):
    expect = [-1 / 560, 8 / 315, -1 / 5, 8 / 5, -205 / 72, 8 / 5, -1 / 5, 8 / 315, -1 / 560]
    a = np.ones(9)
    for name in PARAMS:
        got = [orc.narrow_point(a, np.eye(9)[s], 1.0, *PARAMS[name]) for s in range(9)]
        np.testing.assert_allclose(got, expect, rtol=1e-13, atol=1e-15)


def _matrix(orc, a, m47, m48, dx=1.0):
    n = len(a)
    return np.stack([orc.narrow_periodic(a, np.eye(n)[j], dx, m47, m48) for j in range(n)], axis=1)


def test_narrow_flux_form_conserves_and_kills_constants(orc):
    rng = np.random.default_rng(2)
    n = 40
    a = np.exp(rng.standard_normal(n))
    A = _matrix(orc, a, *SMC)
    scale = np.abs(A).max()
    assert np.abs(A.sum(axis=0)).max() <= 1e-13 * scale   # column sums: sum_i L u = 0
    assert np.abs(A.sum(axis=1)).max() <= 1e-13 * scale   # row sums: L(a, const) = 0


def test_narrow_constant_a_symmetric_negative_semidefinite(orc):
    n = 32
    for name in PARAMS:
        A = _matrix(orc, np.full(n, 1.7), *PARAMS[name])
        assert np.abs(A - A.T).max() <= 1e-13
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).max() <= 1e-12


def test_narrow_variable_a_symmetric_part_negative_semidefinite(orc):
    # well-posedness for any a > 0, independent of (m47, m48)
    rng = np.random.default_rng(3)
    n = 32
    x = 2 * np.pi * np.arange(n) / n
    for name in PARAMS:
        for trial in range(5):
            a = np.exp(2.0 * np.sin(x + trial) + 0.5 * rng.standard_normal(n))
            A = _matrix(orc, a, *PARAMS[name])
            ev = np.linalg.eigvalsh(0.5 * (A + A.T))
            assert ev.max() <= 1e-12 * np.abs(ev).max()


def test_narrow_damps_nyquist_mode(orc):
    n = 16
    u = (-1.0) ** np.arange(n)
    for name in PARAMS:
        got = orc.narrow_periodic(np.ones(n), u, 1.0, *PARAMS[name])
        np.testing.assert_allclose(got, -2048.0 / 315.0 * u, rtol=1e-13)
    # the wide stencil D(D u) does not: the first derivative annihilates it
    assert np.abs(orc.d1_periodic(u, 1.0)).max() == 0.0


def test_eighth_order_convergence_on_sinusoids(orc):
    x = sp.symbols("x")
    a_e = 1 + sp.sin(x) / 2
    u_e = sp.sin(2 * x) * sp.cos(x) + sp.cos(3 * x)
    La = sp.lambdify(x, a_e, "numpy")
    Lu = sp.lambdify(x, u_e, "numpy")
    Ld = sp.lambdify(x, sp.diff(u_e, x), "numpy")
    Ln = sp.lambdify(x, sp.diff(a_e * sp.diff(u_e, x), x), "numpy")
    eD, eL = [], []
    for n in (32, 64, 128):
        xs = 2 * np.pi * np.arange(n) / n
        dx = 2 * np.pi / n
        eD.append(np.abs(orc.d1_periodic(Lu(xs), dx) - Ld(xs)).max())
        eL.append(np.abs(orc.narrow_periodic(La(xs), Lu(xs), dx, *SMC) - Ln(xs)).max())
    for e in (eD, eL):
        rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
        assert min(rates) > 7.5, rates


def test_sixth_order_family_exact_to_degree_7(orc):
    rng = np.random.default_rng(4)
    for m36 in (281 / 3600, 0.220063, 0.0):
        M = orc.narrow6_matrix(m36)
        x0, dx = 0.1, 0.1
        xs = x0 + dx * np.arange(-3, 4)   # offsets -3..3
        for da in range(8):
            for du in range(8 - da):
                A = np.polynomial.Polynomial(rng.standard_normal(da + 1))
                Uu = np.polynomial.Polynomial(rng.standard_normal(du + 1))
                av, uv = A(xs), Uu(xs)
                # H_{i+1/2} = sum_{m,n=-2..3} a_{i+m} M_mn u_{i+n}; centre index 3
                hp = sum(av[3 + m] * M[m + 2, k + 2] * uv[3 + k] for m in range(-2, 4) for k in range(-2, 4))
                hm = sum(av[2 + m] * M[m + 2, k + 2] * uv[2 + k] for m in range(-2, 4) for k in range(-2, 4))
                got = (hp - hm) / dx ** 2
                exact = (A * Uu.deriv()).deriv()(x0)
                assert abs(got - exact) <= 1e-8 * (1 + abs(exact)), (m36, da, du)


@pytest.mark.parametrize("name", ["SMC", "ZERO", "OPTIMAL"])
def test_heat_problem_t1_reproduces_table(orc, name):
    from oracle import heat
    rows = [r for r in read_table("table7_t1.txt") if r[0] == name]
    m47, m48 = PARAMS[name]
    sizes = (20, 40, 80) if name == "SMC" else (20, 40)
    for r in rows:
        n = int(r[1])
        if n not in sizes:
            continue
        u, X, Y = heat.run("T1", n, m47, m48)
        err = u - math.exp(-1.0) * np.sin(X) * np.sin(Y)
        linf, l2 = np.abs(err).max(), np.sqrt(np.mean(err ** 2))
        assert linf == pytest.approx(float(r[2]), rel=3e-3), (n, linf)
        assert l2 == pytest.approx(float(r[3]), rel=3e-3), (n, l2)
