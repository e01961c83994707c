"""Oracle pins of multirate SDC mode 2 (eq. mrupdate2): the stiff component
(chemistry) implicit on the coarse nodes, advection-diffusion explicit on the
fine nodes, and its implicit chemistry solve.

What fixes it, independently of the implementation:
  * on u' = a u + b u (a implicit, coarse; b explicit, fine) the sweeps
    converge to the multirate collocation solution, computed here directly
    as one linear system;
  * each sweep raises the order by one (local error O(dt^(K+1)));
  * a stiff implicit component (a dt = -1000) stays bounded and accurate,
    where the explicit treatment of the same component (mode 1) blows up;
  * with coincident coarse and fine nodes, modes 1 and 2 and single-rate SDC
    converge to one collocation solution of the full right-hand side (3D box);
  * on a uniform state (no transport) mode 2 converges to the collocation
    solution of the chemistry alone (single-rate SDC of the source);
  * the implicit solve satisfies its equation to rounding level, also for a
    step far beyond the explicit stability limit."""
import numpy as np
import pytest

import oracle
from oracle import implicit as OI
from oracle import sdc as osdc
from synth import fields, mechanism
from synth.workloads import time_step


def collocation_multirate(a, b, u0, dt, t1, t2, pieces):
    """u_q = u0 + dt sum_{q' < q} (S21 a u_coarse + S22 b u_fine)_{q'}: the
    collocation solution of the multirate quadrature, one linear solve."""
    S21, S22 = osdc.mr_matrices(t1, t2, pieces)
    M1, M2 = len(t1) - 1, len(t2) - 1
    r = M2 // M1
    Q21 = np.cumsum(S21, axis=0)
    Q22 = np.cumsum(S22, axis=0)
    A = np.eye(M2 + 1)
    rhs = np.zeros(M2 + 1)
    rhs[0] = u0
    for q in range(1, M2 + 1):
        for j in range(M1 + 1):
            A[q, j * r] -= dt * a * Q21[q - 1, j]
        for j in range(M2 + 1):
            A[q, j] -= dt * b * Q22[q - 1, j]
        rhs[q] = u0
    return np.linalg.solve(A, rhs)[-1]


def scalar_mode2(a, b, u0, dt, t1, t2, pieces, K, nsteps=1):
    f1 = lambda u, t: a * u
    f2 = lambda u, t: b * u
    solve1 = lambda rhs, h: rhs / (1.0 - h * a)
    return osdc.mrsdc2_run(f1, solve1, f2, np.array([u0]), 0.0, dt, t1, t2, pieces, K, nsteps)[0]


@pytest.mark.parametrize("nc,nf,rep", [(4, 5, 1), (3, 3, 2), (5, 3, 2)])
def test_scalar_converges_to_multirate_collocation(nc, nf, rep):
    t1, t2, pieces = osdc.mr_nodes(nc, nf, rep)
    a, b, dt = -3.0, 1.7, 0.2
    ref = collocation_multirate(a, b, 1.0, dt, t1, t2, pieces)
    got = scalar_mode2(a, b, 1.0, dt, t1, t2, pieces, 40)
    assert abs(got - ref) <= 1e-14
    # and the collocation solution is a high-order approximation of exp
    assert abs(ref - np.exp((a + b) * dt)) < 1e-5


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_each_sweep_raises_the_order(K):
    t1, t2, pieces = osdc.mr_nodes(4, 5, 1)
    a, b = -2.0, 1.0
    errs = []
    for dt in (0.05, 0.025):
        errs.append(abs(scalar_mode2(a, b, 1.0, dt, t1, t2, pieces, K) - np.exp((a + b) * dt)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > K + 1 - 0.35, (K, rate, errs)


def test_stiff_implicit_component_is_stable():
    t1, t2, pieces = osdc.mr_nodes(3, 3, 2)
    a, b, dt = -1.0e4, -1.0, 0.1
    u = scalar_mode2(a, b, 1.0, dt, t1, t2, pieces, 4, nsteps=10)
    assert abs(u) < 1e-3
    # the same component treated explicitly (mode 1 puts it on the fine
    # nodes with forward-Euler corrections) is unstable at this step
    f1 = lambda v, t: b * v
    f2 = lambda v, t: a * v
    with np.errstate(over="ignore", invalid="ignore"):
        v = osdc.mrsdc_run(f1, f2, np.array([1.0]), 0.0, dt, t1, t2, pieces, 4, 3)[0]
    assert not np.isfinite(v) or abs(v) > 1e6


def _box(kind="mech9", shape=(4, 5, 6), seed=9):
    m = mechanism.load(kind)
    om = oracle.Mechanism(m)
    U0 = oracle.prim_to_cons(om, fields.sines(shape, 1e-4, m["ns"], seed))
    return m, om, U0


def _mode2(om, dx, U0, dt, t1, t2, pieces, K, nsteps=1):
    f1 = lambda U, t: oracle.rhs(om, U, dx, parts=oracle.REACT)
    f2 = lambda U, t: oracle.rhs(om, U, dx, parts=oracle.AD)
    solve1 = lambda rhs, h: OI.implicit_reaction(om, rhs, h, dx)
    return osdc.mrsdc2_run(f1, solve1, f2, U0, 0.0, dt, t1, t2, pieces, K, nsteps)


def test_coincident_nodes_modes_agree_with_single_rate_collocation():
    """Fine nodes = coarse nodes (3 Gauss-Lobatto nodes) with one fine
    polynomial over the step (type (a)): modes 1 and 2 and single-rate SDC
    all converge to the collocation solution of the full right-hand side."""
    m, om, U0 = _box()
    dx, dt, K = 1e-4, time_step("box16_sdc"), 20
    t1 = osdc.gauss_lobatto(3)
    t2, pieces = t1.copy(), [(0, 2)]
    u2 = _mode2(om, dx, U0, dt, t1, t2, pieces, K)
    f1 = lambda U, t: oracle.rhs(om, U, dx, parts=oracle.AD)
    f2 = lambda U, t: oracle.rhs(om, U, dx, parts=oracle.REACT)
    u1 = osdc.mrsdc_run(f1, f2, U0, 0.0, dt, t1, t2, pieces, K, 1)
    f = lambda U, t: oracle.rhs(om, U, dx)
    us = osdc.sdc_run(f, U0, 0.0, dt, t1, K, 1)
    d = us - U0
    nq = d.shape[0]
    scale = np.abs(d).reshape(nq, -1).max(axis=1)
    for u in (u1, u2):
        err = np.abs(u - us).reshape(nq, -1).max(axis=1)
        assert np.all(err <= 1e-11 * scale), err / scale


def test_uniform_state_is_the_chemistry_collocation():
    """No transport on a uniform state at rest: mode 2 (4 coarse nodes with
    the chemistry, 5 fine nodes each) converges to the 4-node collocation
    solution of the chemistry source alone."""
    m = mechanism.load("mech9")
    om = oracle.Mechanism(m)
    shape = (4, 4, 4)
    prim = fields.sines(shape, 1e-4, m["ns"], 3)
    for k in ("T", "p"):
        prim[k] = np.full(shape, prim[k].flat[5])
    prim["Y"] = np.broadcast_to(prim["Y"][:, :1, :1, :1], prim["Y"].shape).copy()
    prim["u"] = np.zeros_like(prim["u"])
    U0 = oracle.prim_to_cons(om, prim)
    dx, dt = 1e-4, 4 * time_step("box16_sdc")
    t1, t2, pieces = osdc.mr_nodes(4, 5, 1)
    u2 = _mode2(om, dx, U0, dt, t1, t2, pieces, 20)
    f = lambda U, t: oracle.rhs(om, U, dx, parts=oracle.REACT)
    uc = osdc.sdc_run(f, U0, 0.0, dt, osdc.gauss_lobatto(4), 30, 1)
    d = uc[5:] - U0[5:]
    assert np.abs(d).max() > 1e-8 * np.abs(U0[5:]).max()     # the chemistry moves
    assert np.abs(u2[5:] - uc[5:]).max() <= 1e-10 * np.abs(d).max()
    assert np.abs(u2[:5] - U0[:5]).max() <= 1e-13 * np.abs(U0[:5]).max()


@pytest.mark.parametrize("hmul", [1.0, 300.0])
def test_implicit_solve_satisfies_its_equation(hmul):
    m, om, U0 = _box(shape=(3, 4, 5))
    dx = 1e-4
    h = hmul * time_step("box16_sdc")
    rhs = U0.copy()
    Us = OI.implicit_reaction(om, rhs, h, dx)
    np.testing.assert_array_equal(Us[:5], rhs[:5])
    R = oracle.rhs(om, Us, dx, parts=oracle.REACT)
    res = Us[5:] - h * R[5:] - rhs[5:]
    assert np.abs(res).max() <= 1e-14 * np.abs(rhs[5:]).max()
    if hmul > 1.0:
        # far beyond the explicit limit the step still lands between the
        # start and the equilibrium: mass fractions stay in [0, 1]
        Y = Us[5:] / Us[0]
        assert Y.min() > -1e-12 and Y.max() < 1.0 + 1e-12
