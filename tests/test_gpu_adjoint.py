"""Parity of the adjoint forms with the oracle: the vector-Jacobian product
of the right-hand side (rhs_vjp), the adjoint of the SDC step (sdc_step_vjp)
and their torch.autograd wrappers.  The library is called through its C-ABI.

Criterion: per state component q, max|g_q - g_ref,q| <= 1e-10 max|g_ref,q|
(g the product with respect to the state), the same for the ln A gradient
as a whole, and 1e-10 relative agreement of adjoint dot products
<vbar, J w> = <J^T vbar, w> where only the oracle's forward product is
affordable (full sizes, multi-step SDC).  The oracle's inputs are its own
conserved states, uploaded to the device, so both sides differentiate at
the same point."""
import numpy as np
import pytest

import oracle
from oracle import adjoint as OA
from synth import fields, mechanism
from synth.workloads import WORKLOADS, make_primitives, time_step

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1309_7327_amd import autograd as AG  # noqa: E402
from paper_1309_7327_amd import narrowsdc as N  # noqa: E402
import gpu_util as G  # noqa: E402

TOL = 1e-10
MECHS = {}


def mech(kind):
    if kind not in MECHS:
        m = mechanism.load(kind)
        ctx = N.Context(0)
        ctx.set_mechanism(m)
        MECHS[kind] = (m, oracle.Mechanism(m), ctx)
    return MECHS[kind]


def upload(U):
    """Oracle interior state -> ghosted device array (ghosts filled by the
    library on use)."""
    nU, nz, ny, nx = U.shape
    Ug = torch.zeros(N.ghosted_shape(nU, nz, ny, nx), dtype=torch.float64, device="cuda")
    N.interior(Ug).copy_(G.dev(U))
    return N.box(nx, ny, nz, 1e-4), Ug


def field_errors(g, ref):
    return [float(np.abs(g[q] - ref[q]).max() / max(np.abs(ref[q]).max(), 1e-300)) for q in range(ref.shape[0])]


def gpu_vjp(ctx, m, bx, Ug, v, parts=N.RHS_ALL):
    Ub = torch.zeros(v.shape, dtype=torch.float64, device="cuda")
    lA = torch.zeros(m["nr"], dtype=torch.float64, device="cuda")
    ctx.rhs_vjp(bx, Ug, G.dev(v), Ub, lA, parts)
    ctx.check_status()
    return G.host(Ub), G.host(lA)


@pytest.mark.parametrize("kind,shape,parts", [
    ("mech9", (5, 6, 7), N.RHS_HYP), ("mech9", (5, 6, 7), N.RHS_DIFF), ("mech9", (5, 6, 7), N.RHS_REACT),
    ("mech9", (5, 6, 7), N.RHS_ALL), ("mech9le", (6, 5, 4), N.RHS_ALL), ("mech21", (4, 5, 6), N.RHS_ALL),
    ("mech12", (5, 4, 6), N.RHS_ALL)])
def test_rhs_vjp_matches_oracle_on_small_boxes(kind, shape, parts):
    """Every entry of (d rhs/dU)^T v against the oracle's column-by-column
    definition; boxes smaller than the stencil, so lines wrap onto
    themselves."""
    m, om, ctx = mech(kind)
    U = oracle.prim_to_cons(om, fields.sines(shape, 1e-4, m["ns"], 3))
    v = np.random.default_rng(7).standard_normal(U.shape)
    bx, Ug = upload(U)
    print(f"rhs_vjp {kind} {shape} parts={parts}", flush=True)
    g, gA = gpu_vjp(ctx, m, bx, Ug, v, parts)
    ref = OA.rhs_vjp(om, U, 1e-4, v, parts=parts)
    errs = field_errors(g, ref)
    print("  per-field rel err", " ".join(f"{e:.1e}" for e in errs))
    assert max(errs) <= TOL
    if parts & N.RHS_REACT:
        refA = OA.rhs_vjp_lnA(om, U, 1e-4, v, m["nr"])
        eA = np.abs(gA - refA).max() / np.abs(refA).max()
        print(f"  lnA rel err {eA:.1e}")
        assert eA <= TOL
    else:
        assert np.all(gA == 0.0)


def test_rhs_vjp_full_size_box64():
    """The 64^3 adjoint workload: sampled entries against the oracle's
    definition, the ln A gradient, and one whole-box adjoint dot product."""
    wl = WORKLOADS["box64_adjoint"]
    m, om, ctx = mech(wl["mech"])
    U = oracle.prim_to_cons(om, make_primitives("box64_adjoint", m))
    rng = np.random.default_rng(5001)
    v = rng.standard_normal(U.shape)
    bx, Ug = upload(U)
    print("rhs_vjp box64_adjoint", flush=True)
    g, gA = gpu_vjp(ctx, m, bx, Ug, v)
    # 27 input cells on a lattice (spacing 21 > 8: disjoint dependence cubes)
    ax = np.array([3, 24, 45])
    cells = np.array([[x, y, z] for z in ax + 2 for y in ax + 1 for x in ax])
    ref = OA.rhs_vjp(om, U, 1e-4, v, cells=cells, nthreads=0)
    gs = g[:, cells[:, 2], cells[:, 1], cells[:, 0]].T
    errs = [float(np.abs(gs[:, q] - ref[:, q]).max() / np.abs(ref[:, q]).max()) for q in range(ref.shape[1])]
    print("  sampled per-field rel err", " ".join(f"{e:.1e}" for e in errs), flush=True)
    assert max(errs) <= TOL
    refA = OA.rhs_vjp_lnA(om, U, 1e-4, v, m["nr"])
    eA = np.abs(gA - refA).max() / np.abs(refA).max()
    print(f"  lnA rel err {eA:.1e}", flush=True)
    assert eA <= TOL
    w = rng.standard_normal(U.shape) * np.abs(U).max(axis=(1, 2, 3), keepdims=True)
    _, jw = oracle.rhs_jvp(om, U, 1e-4, w)
    a, b = float(np.sum(v * jw)), float(np.sum(g * w))
    print(f"  <v, J w> {a:.16e}  <J^T v, w> {b:.16e}", flush=True)
    assert abs(a - b) <= TOL * abs(a)


def test_rhs_vjp_deterministic_accumulating_and_tile_independent():
    m, om, ctx = mech("mech9")
    U = oracle.prim_to_cons(om, fields.sines((20, 18, 40), 1e-4, m["ns"], 5))
    v = np.random.default_rng(9).standard_normal(U.shape)
    bx, Ug = upload(U)
    vd = G.dev(v)
    outs = []
    for tiles in [((0, 0, 0), (0, 0, 0)), ((16, 4, 4), (16, 4, 4)), ((64, 2, 2), (8, 8, 4)),
                  ((8, 8, 2), (32, 8, 1))]:
        ctx.set_tiles(*tiles, grid_cap=37)
        Ub = torch.zeros(v.shape, dtype=torch.float64, device="cuda")
        lA = torch.zeros(m["nr"], dtype=torch.float64, device="cuda")
        ctx.rhs_vjp(bx, Ug, vd, Ub, lA)
        first = G.host(Ub).copy()
        ctx.rhs_vjp(bx, Ug, vd, Ub, lA)   # accumulates
        ctx.check_status()
        np.testing.assert_array_equal(G.host(Ub), 2.0 * first)
        outs.append((first, G.host(lA) / 2.0))
    ctx.set_tiles()
    for g, gA in outs[1:]:
        np.testing.assert_array_equal(g, outs[0][0])
        np.testing.assert_allclose(gA, outs[0][1], rtol=1e-13, atol=1e-13 * np.abs(outs[0][1]).max())


def _sdc_vjp(ctx, m, bx, Ug, dt, nsteps, sch, ub):
    nb = ctx.vjp_workspace_size(bx, sch, nsteps)
    ws = torch.empty(nb // 8 + 1, dtype=torch.float64, device="cuda")
    U0b = torch.empty(ub.shape, dtype=torch.float64, device="cuda")
    lA = torch.zeros(m["nr"], dtype=torch.float64, device="cuda")
    ctx.sdc_step_vjp(bx, Ug, dt, nsteps, sch, G.dev(ub), U0b, lA, ws, nb)
    ctx.check_status()
    return G.host(U0b), G.host(lA)


@pytest.mark.parametrize("nsteps,sweeps", [(1, 6), (5, 6), (2, 3)])
def test_sdc_step_vjp_adjoint_identity(nsteps, sweeps):
    """<ubar, dU_N> from the oracle's tangent SDC (eq. expsdc on the pair
    (U, dU)) against <U0_bar, w> + <lnA_bar, w_A> from the library, on the
    16^3 workload (4 Gauss-Lobatto nodes)."""
    m, om, ctx = mech("mech9")
    U = oracle.prim_to_cons(om, make_primitives("box16_sdc", m))
    dt = time_step("box16_sdc")
    bx, Ug = upload(U)
    rng = np.random.default_rng(100 + nsteps)
    ub = rng.standard_normal(U.shape)
    sch = N.scheme(4, sweeps, 0, 1)
    print(f"sdc_step_vjp 16^3 nsteps={nsteps} K={sweeps}", flush=True)
    g, gA = _sdc_vjp(ctx, m, bx, Ug, dt, nsteps, sch, ub)
    w = rng.standard_normal(U.shape) * np.abs(U).max(axis=(1, 2, 3), keepdims=True)
    wA = rng.standard_normal(m["nr"])
    _, dU = OA.sdc_tangent(om, U, 1e-4, dt, 4, sweeps, nsteps, w, wA)
    a = float(np.sum(ub * dU))
    b = float(np.sum(g * w) + np.sum(gA * wA))
    print(f"  <ub, J w> {a:.16e}  <J^T ub, w> {b:.16e}  rel {abs(a - b) / abs(a):.1e}", flush=True)
    assert abs(a - b) <= TOL * abs(a)


def test_sdc_step_vjp_full_size_central_differences():
    """The 64^3 workload through 5 steps: <ubar, (U_N(U0 + h w) - U_N(U0 - h w)) / 2h>
    from two forward runs of the library against <U0_bar, w> (agreement at
    the central-difference error, about 1e-7 relative)."""
    wl = WORKLOADS["box64_adjoint"]
    m, om, ctx = mech(wl["mech"])
    U = oracle.prim_to_cons(om, make_primitives("box64_adjoint", m))
    dt = time_step("box64_adjoint")
    nsteps = wl["steps"]
    sch = N.scheme(4, 6, 0, 1)
    bx, Ug = upload(U)
    rng = np.random.default_rng(6001)
    ub = rng.standard_normal(U.shape)
    print("sdc_step_vjp box64_adjoint 5 steps", flush=True)
    g, _ = _sdc_vjp(ctx, m, bx, Ug, dt, nsteps, sch, ub)
    w = rng.standard_normal(U.shape) * np.abs(U).max(axis=(1, 2, 3), keepdims=True)
    ws, nb = N.workspace(ctx, [bx], sch)
    h = 1e-7
    ends = []
    for sgn in (1.0, -1.0):
        _, Up = upload(U + sgn * h * w)
        ctx.sdc_step(bx, Up, dt, nsteps, sch, ws, nb)
        ctx.check_status()
        ends.append(G.host(N.interior(Up)))
    fd = float(np.sum(ub * (ends[0] - ends[1]))) / (2 * h)
    b = float(np.sum(g * w))
    print(f"  central difference {fd:.10e}  adjoint {b:.10e}  rel {abs(fd - b) / abs(b):.1e}", flush=True)
    assert abs(fd - b) <= 1e-6 * abs(b)


def test_autograd_wrappers():
    """torch.autograd through RhsFunction / SdcStepFunction gives the C-ABI
    products; ghost layers get zero gradient."""
    m, om, ctx = mech("mech9")
    U = oracle.prim_to_cons(om, fields.sines((8, 9, 10), 1e-4, m["ns"], 21))
    bx, Ug = upload(U)
    rng = np.random.default_rng(21)
    v = rng.standard_normal(U.shape)
    lnA = torch.log(torch.as_tensor(np.asarray(m["A"], dtype=np.float64))).requires_grad_(True)
    Ur = Ug.clone().requires_grad_(True)
    out = AG.rhs(ctx, bx, Ur, lnA)
    (gU, gA) = torch.autograd.grad((out * G.dev(v)).sum(), (Ur, lnA))
    ref, refA = gpu_vjp(ctx, m, bx, Ug.clone(), v)
    np.testing.assert_array_equal(G.host(N.interior(gU)), ref)
    np.testing.assert_array_equal(G.host(gA), refA)
    gh = G.host(gU).copy()
    gh[:, 4:-4, 4:-4, 4:-4] = 0.0
    assert np.all(gh == 0.0)
    # SDC step
    sch = N.scheme(4, 2, 0, 1)
    dt = time_step("box16_sdc")
    Ur = Ug.clone().requires_grad_(True)
    UN = AG.sdc_step(ctx, bx, Ur, lnA, dt, 2, sch)
    (gU, gA) = torch.autograd.grad((UN * G.dev(v)).sum(), (Ur, lnA))
    ref, refA = _sdc_vjp(ctx, m, bx, Ug.clone(), dt, 2, sch, v)
    np.testing.assert_array_equal(G.host(N.interior(gU)), ref)
    np.testing.assert_array_equal(G.host(gA), refA)
