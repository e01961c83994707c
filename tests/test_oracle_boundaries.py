"""Oracle pins of the physical-boundary stencils (Section 2.5) and of the
right-hand side on boxes with non-periodic directions.

Per the paper: at the fourth and third cells from a boundary the centred
stencils drop to sixth and fourth order (advection and diffusion), next to
the boundary to second-order centred diffusion and biased third-order
advection, and at the boundary cell to one-sided second-order diffusion and
third-order advection.  Pinned here by polynomial exactness (each stencil is
exact up to its degree and not one beyond), measured convergence orders,
the fourth-order narrow matrix's textbook reduction, and, for the full
right-hand side: a uniform state reduces to the chemistry, a state constant
along the non-periodic direction gives the periodic right-hand side, and
self-convergence along the non-periodic direction (order >= 7 mid-domain,
about 2 at the boundary)."""
import numpy as np
import pytest

import oracle
from synth import fields, mechanism

N = 24
H = 0.37
X = np.arange(N) * H - 3.1


def dist(i, n=N):
    return min(i, n - 1 - i)


# exact degree of each first-derivative closure by distance from the boundary
ADV_DEG = {0: 3, 1: 3, 2: 4, 3: 6}
DIF_DEG = {0: 2, 1: 2, 2: 4, 3: 6}


@pytest.mark.parametrize("kind,degs", [(0, ADV_DEG), (1, DIF_DEG)])
def test_first_derivative_closures_exact_to_their_degree(kind, degs):
    for p in range(0, 10):
        f = X ** p
        d = oracle.d1_line(f, H, kind)
        exact = p * X ** (p - 1) if p > 0 else np.zeros_like(X)
        for i in range(N):
            deg = degs.get(dist(i), 8)
            err = abs(d[i] - exact[i]) / max(1.0, np.abs(exact).max())
            if p <= deg:
                assert err < 1e-11, (kind, p, i, err)
            elif p == deg + 1:
                assert err > 1e-9, (kind, p, i, err)


@pytest.mark.parametrize("kind,orders", [(0, {0: 3, 1: 3, 2: 4, 3: 6}), (1, {0: 2, 1: 2, 2: 4, 3: 6})])
def test_first_derivative_closure_orders(kind, orders):
    errs = {}
    for n in (41, 81):
        h = 1.0 / (n - 1)
        x = np.arange(n) * h
        d = oracle.d1_line(np.sin(2 * x + 0.4), h, kind)
        e = np.abs(d - 2 * np.cos(2 * x + 0.4))
        errs[n] = {b: e[b] for b in range(4)}
        errs[n]["mid"] = e[n // 2]
    for b, o in orders.items():
        rate = np.log2(errs[41][b] / errs[81][b])
        assert abs(rate - o) < 0.35, (kind, b, rate)
    assert errs[81]["mid"] < 1e-12


def test_fourth_order_narrow_matrix():
    M = oracle.narrow4_matrix()
    # antisymmetric under the reflection about the face, zero corners
    np.testing.assert_allclose(M, -M[::-1, ::-1], atol=0)
    assert M[0, 3] == 0.0 and M[3, 0] == 0.0
    # a = 1: the textbook fourth-order second difference
    col = M.sum(axis=0)
    flux = np.array([0.0, *col]) - np.array([*col, 0.0])     # H_{i+1/2} - H_{i-1/2} weights on u_{i-2..i+2}
    np.testing.assert_allclose(flux, np.array([-1, 16, -30, 16, -1]) / 12.0, atol=1e-15)


def narrow_exact_case(p, q):
    a, u = X ** p, X ** q
    exact = np.zeros_like(X)
    if q >= 1:
        # (a u')' = (q x^(p+q-1))' = q (p+q-1) x^(p+q-2)
        k = p + q - 2
        exact = q * (p + q - 1) * (X ** k if k >= 0 else 0.0 * X)
    return a, u, exact


# exact total degree deg a + deg u of each narrow closure by distance
NARROW_DEG = {0: 2, 1: 3, 2: 5, 3: 7}


def test_narrow_closures_exact_to_their_degree():
    m47, m48 = 1059283 / 13608000, -856481 / 40824000
    for tot in range(0, 11):
        for p in range(0, tot + 1):
            q = tot - p
            a, u, exact = narrow_exact_case(p, q)
            a = a + 2.0   # keep the coefficient away from zero
            exact = exact + 2.0 * (q * (q - 1) * X ** (q - 2) if q >= 2 else 0.0 * X)
            L = oracle.narrow_line(a, u, H, m47, m48)
            # rounding: the size of the terms the stencil sums
            scale = max(1.0, np.abs(exact).max(), np.abs(a).max() * np.abs(u).max() / H ** 2)
            for i in range(N):
                deg = NARROW_DEG.get(dist(i), 9)
                err = abs(L[i] - exact[i]) / scale
                if tot <= deg:
                    assert err < 1e-12, (p, q, i, err)


def test_narrow_closure_orders_and_nonexactness():
    m47, m48 = 1059283 / 13608000, -856481 / 40824000
    errs = {}
    for n in (41, 81, 161):
        h = 1.0 / (n - 1)
        x = np.arange(n) * h
        a = 1.5 + np.cos(x)
        u = np.sin(3 * x + 0.2)
        exact = -np.sin(x) * 3 * np.cos(3 * x + 0.2) - 9 * a * np.sin(3 * x + 0.2)
        e = np.abs(oracle.narrow_line(a, u, h, m47, m48) - exact)
        errs[n] = [e[b] for b in range(4)] + [e[n // 2]]
    # grid pairs above the rounding floor (about 1e-11 at 161 points)
    for b, o, (n1, n2) in ((0, 2, (81, 161)), (1, 2, (81, 161)), (2, 4, (81, 161)), (3, 6, (41, 81))):
        rate = np.log2(errs[n1][b] / errs[n2][b])
        assert abs(rate - o) < 0.5, (b, rate)
    assert errs[81][4] < 1e-11
    # one degree beyond: the boundary cell is not exact for a = x^3, u = x
    a, u, exact = narrow_exact_case(3, 1)
    L = oracle.narrow_line(a + 2.0, u, H, m47, m48)
    assert abs(L[0] - exact[0]) > 1e-6


def _mech(kind="mech9"):
    return mechanism.load(kind)


@pytest.mark.parametrize("mask", [1, 2, 5, 7])
def test_uniform_state_is_the_chemistry(mask):
    m = _mech()
    shape = (9, 10, 11)
    prim = fields.sines(shape, 1e-4, m["ns"], 3)
    for k in ("T", "p"):
        prim[k] = np.full(shape, prim[k].flat[7])
    prim["Y"] = np.broadcast_to(prim["Y"][:, :1, :1, :1], prim["Y"].shape).copy()
    prim["u"] = np.zeros_like(prim["u"])
    om = oracle.Mechanism(m, nonperiodic=mask)
    U = oracle.prim_to_cons(om, prim)
    # differences of equal samples: the convective terms vanish exactly with
    # the boundary stencils too; the narrow rows sum to zero up to rounding
    assert np.abs(oracle.rhs(om, U, 1e-4, parts=oracle.HYP)).max() == 0.0
    ad = oracle.rhs(om, U, 1e-4, parts=oracle.AD)
    scale = np.abs(U).reshape(U.shape[0], -1).max(axis=1) / 1e-8
    assert np.all(np.abs(ad).reshape(U.shape[0], -1).max(axis=1) <= 1e-12 * scale)
    full = oracle.rhs(om, U, 1e-4)
    np.testing.assert_array_equal(full[5:], oracle.production(om, U))


def test_constant_along_the_boundary_normal_is_the_periodic_rhs():
    """Fields that vary only along y and z: every x-derivative vanishes with
    any stencil, so physical boundaries along x change nothing."""
    m = _mech("mech9le")
    shape = (10, 12, 9)
    prim = fields.sines(shape, 1e-4, m["ns"], 5)
    for k in ("T", "p"):
        prim[k] = np.broadcast_to(prim[k][:, :, :1], shape).copy()
    prim["Y"] = np.broadcast_to(prim["Y"][:, :, :, :1], prim["Y"].shape).copy()
    prim["u"] = np.broadcast_to(prim["u"][:, :, :, :1], prim["u"].shape).copy()
    U = oracle.prim_to_cons(oracle.Mechanism(m), prim)
    f_per = oracle.rhs(oracle.Mechanism(m), U, 1e-4)
    f_np = oracle.rhs(oracle.Mechanism(m, nonperiodic=1), U, 1e-4)
    # the x-derivatives of x-constant fields: exactly zero for the first
    # derivatives (differences), rounding of the narrow rows' sums otherwise
    scale = np.abs(f_per).reshape(f_per.shape[0], -1).max(axis=1)
    err = np.abs(f_np - f_per).reshape(f_per.shape[0], -1).max(axis=1)
    assert np.all(err <= 1e-13 * scale), err / scale
    f_per = oracle.rhs(oracle.Mechanism(m), U, 1e-4, parts=oracle.HYP)
    f_np = oracle.rhs(oracle.Mechanism(m, nonperiodic=1), U, 1e-4, parts=oracle.HYP)
    np.testing.assert_array_equal(f_np, f_per)


def _line_state(m, om, n, L):
    """Smooth non-periodic fields along x on n points spanning [0, L]."""
    h = L / (n - 1)
    x = np.arange(n) * h / L
    shape = (1, 1, n)
    ns = m["ns"]
    T = 1000.0 + 250.0 * np.sin(np.pi * x + 0.3)
    p = 101325.0 * (1.0 + 0.02 * np.cos(2.0 * x))
    u = np.stack([8.0 * np.sin(2.0 * x + 0.1), 5.0 * np.cos(1.5 * x), 3.0 * np.sin(x + 1.0)])
    w = 0.5 * (1.0 + np.sin(1.7 * x))
    ya = np.linspace(1.0, 2.0, ns)
    yb = np.linspace(2.0, 1.0, ns)
    Y = np.outer(ya / ya.sum(), w) + np.outer(yb / yb.sum(), 1.0 - w)
    prim = dict(T=T.reshape(shape), p=p.reshape(shape), u=u.reshape((3,) + shape), Y=Y.reshape((ns,) + shape))
    return oracle.prim_to_cons(om, prim), h


def test_self_convergence_along_the_boundary_normal():
    m = _mech("mech9le")
    om = oracle.Mechanism(m, nonperiodic=1)
    L = 1.6e-3
    R = {}
    for n in (17, 33, 65):
        U, h = _line_state(m, om, n, L)
        R[n] = oracle.rhs(om, U, (h, 1e-4, 1e-4), parts=oracle.AD)[:, 0, 0, :]
    # shared points: x = 0 (the boundary cell) and x = L/2
    for pos, lo in (("mid", 7.0), ("wall", 1.6)):
        idx = {n: (n // 2 if pos == "mid" else 0) for n in R}
        e1 = np.abs(R[17][:, idx[17]] - R[33][:, idx[33]])
        e2 = np.abs(R[33][:, idx[33]] - R[65][:, idx[65]])
        q = np.argmax(e1)                      # the component with the largest change
        rate = np.log2(e1[q] / e2[q])
        assert rate > lo, (pos, q, rate)


def test_rejects_small_boxes_and_the_wide_stencil():
    m = _mech()
    prim = fields.sines((9, 10, 7), 1e-4, m["ns"], 3)
    U = oracle.prim_to_cons(oracle.Mechanism(m), prim)
    with pytest.raises(RuntimeError):
        oracle.rhs(oracle.Mechanism(m, nonperiodic=1), U, 1e-4)      # nx = 7 < 8
    with pytest.raises(RuntimeError):
        oracle.rhs(oracle.Mechanism(m, wide=True, nonperiodic=2), U, 1e-4)
