"""Physical (non-periodic) boundaries on the GPU against the oracle: the
reduced-order boundary stencils of Section 2.5 along every direction whose
bit is set in box_desc.nonperiodic, through the C-ABI.  Both sides start from
the oracle's conserved state; the parity criterion is the suite's
(tests/gpu_util.py)."""
import numpy as np
import pytest

import oracle
from oracle import sdc as osdc
from synth import fields, mechanism
from synth.workloads import WORKLOADS, make_primitives, time_step

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1309_7327_amd import narrowsdc as N  # noqa: E402
import gpu_util as G  # noqa: E402

CTX = {}


def ctx_for(kind, ref=-1):
    if (kind, ref) not in CTX:
        m = mechanism.load(kind)
        ctx = N.Context(0)
        ctx.set_mechanism(m)
        ctx.set_reference_species(ref)
        CTX[kind, ref] = (m, ctx)
    return CTX[kind, ref]


def upload_box(om, prim, dx, mask):
    Uo = oracle.prim_to_cons(om, prim)
    nU, nz, ny, nx = Uo.shape
    h = np.broadcast_to(np.asarray(dx, dtype=np.float64), (3,))
    bx = N.box(nx, ny, nz, h[0], h[1], h[2], nonperiodic=mask)
    Ug = torch.zeros(N.ghosted_shape(nU, nz, ny, nx), dtype=torch.float64, device="cuda")
    N.interior(Ug).copy_(G.dev(Uo))
    return bx, Ug, Uo


@pytest.mark.parametrize("parts", [N.RHS_HYP, N.RHS_DIFF, N.RHS_ALL])
@pytest.mark.parametrize("kind,shape,dx,mask,ref", [
    ("mech9", (12, 10, 16), 1e-4, 1, -1),                       # x walls
    ("mech9le", (9, 11, 8), (1e-4, 1.2e-4, 0.9e-4), 7, -1),     # every direction, anisotropic, V_c active
    ("mech21", (10, 9, 12), 1e-4, 2, -1),                       # y walls, 21 species
    ("mech9", (24, 20, 36), 1e-4, 5, -1),                       # x and z walls, several tiles, ragged tails
    ("mech9le", (10, 12, 9), 1e-4, 4, 8),                       # z walls with a reference species
])
def test_rhs_eval_parity(kind, shape, dx, mask, ref, parts):
    m, ctx = ctx_for(kind, ref)
    om = oracle.Mechanism(m, ref_species=ref, nonperiodic=mask)
    prim = fields.sines(shape, dx, m["ns"], 61)
    bx, U, Uo = upload_box(om, prim, dx, mask)
    F = torch.zeros((5 + m["ns"],) + shape, dtype=torch.float64, device="cuda")
    ctx.rhs_eval(bx, U, F, parts)
    ctx.check_status()
    fref, floor = G.ulp_floor(lambda V: oracle.rhs(om, V, dx, parts=parts), Uo)
    ok, rep = G.compare(G.host(F), fref, floor)
    print(kind, shape, "mask", mask, "ref", ref, parts, G.fmt(rep))
    assert ok, G.fmt(rep)


@pytest.mark.parametrize("sch,nsteps,mask", [(dict(n_coarse=4, sweeps=4, n_fine=0), 2, 3),
                                             (dict(n_coarse=4, sweeps=3, n_fine=5, fine_repeat=1), 1, 1),
                                             (dict(n_coarse=3, sweeps=3, n_fine=3, fine_repeat=1, mode=2), 1, 6)])
def test_sdc_step_parity(sch, nsteps, mask):
    m, ctx = ctx_for("mech9")
    om = oracle.Mechanism(m, nonperiodic=mask)
    shape = (9, 8, 10)
    prim = fields.sines(shape, 1e-4, m["ns"], 63)
    bx, U, U0 = upload_box(om, prim, 1e-4, mask)
    dt = time_step("box16_sdc")
    s = N.scheme(sch["n_coarse"], sch["sweeps"], sch["n_fine"], sch.get("fine_repeat", 1), mode=sch.get("mode", 1))
    ws, nb = N.workspace(ctx, [bx], s)
    ctx.sdc_step(bx, U, dt, nsteps, s, ws, nb)
    ctx.check_status()
    Ug = G.interior(G.host(U))

    def step(V, pt):
        if sch["n_fine"] == 0:
            f = lambda W, t: oracle.rhs(om, W, 1e-4)
            return osdc.sdc_run(f, V, 0.0, dt, osdc.gauss_lobatto(sch["n_coarse"]), sch["sweeps"], nsteps, pt)
        t1, t2, pieces = osdc.mr_nodes(sch["n_coarse"], sch["n_fine"], sch["fine_repeat"])
        fa = lambda W, t: oracle.rhs(om, W, 1e-4, parts=oracle.AD)
        fr = lambda W, t: oracle.rhs(om, W, 1e-4, parts=oracle.REACT)
        if sch.get("mode", 1) == 2:
            from oracle import implicit as OI
            solve = lambda r, h: OI.implicit_reaction(om, r, h, 1e-4)
            return osdc.mrsdc2_run(fr, solve, fa, V, 0.0, dt, t1, t2, pieces, sch["sweeps"], nsteps, pt)
        return osdc.mrsdc_run(fa, fr, V, 0.0, dt, t1, t2, pieces, sch["sweeps"], nsteps, pt)

    ref, floor, dfloor = G.ulp_floor_step(step, U0)
    ok, rep = G.compare(Ug, ref, floor)
    okd, repd = G.compare(Ug - U0, ref - U0, dfloor, state=ref)
    print(sch, "mask", mask)
    print("U ", G.fmt(rep))
    print("dU", G.fmt(repd))
    assert ok and okd, G.fmt(repd)


def test_sampled_cells_of_full_size_rhs_with_x_walls():
    """The 128^3 turbulent flame with physical boundaries along x, at sampled
    cells including every boundary layer, in the bench's launch shapes."""
    name = "box128_mrsdc"
    wl = WORKLOADS[name]
    m, ctx = ctx_for(wl["mech"])
    om = oracle.Mechanism(m, nonperiodic=1)
    prim = make_primitives(name, m)
    bx, U, Ui = upload_box(om, prim, wl["dx"], 1)
    shape = wl["shape"]
    F = torch.zeros((5 + m["ns"],) + shape, dtype=torch.float64, device="cuda")
    ctx.rhs_eval(bx, U, F, N.RHS_ALL)
    ctx.check_status()
    Fh = G.host(F)
    rng = np.random.default_rng(11)
    cells = rng.integers(0, shape[0], size=(64, 3))
    for j, xb in enumerate([0, 1, 2, 3, 4, 123, 124, 125, 126, 127]):
        cells[j, 0] = xb
    ref = oracle.rhs_cells(om, Ui, wl["dx"], cells)
    rng2 = np.random.default_rng(12345)
    ref_p = oracle.rhs_cells(om, Ui * (1 + 2.0 ** -52 * rng2.standard_normal(Ui.shape)), wl["dx"], cells)
    got = np.stack([Fh[:, z, y, x] for x, y, z in cells])
    floor = np.abs(ref_p - ref).max(axis=0)
    ok, rep = G.compare(got.T, ref.T, floor)
    print(G.fmt(rep))
    assert ok, G.fmt(rep)


def test_static_batched_and_error_paths():
    m, ctx = ctx_for("mech9")
    om = oracle.Mechanism(m, nonperiodic=3)
    shape = (10, 9, 12)
    prim = fields.sines(shape, 1e-4, m["ns"], 65)
    bx, U, _ = upload_box(om, prim, 1e-4, 3)
    F1 = torch.zeros((5 + m["ns"],) + shape, dtype=torch.float64, device="cuda")
    F2 = torch.full_like(F1, np.nan)
    ctx.rhs_eval(bx, U, F1, N.RHS_ALL)
    ctx.rhs_eval_static(bx, U, F2, N.RHS_ALL)
    ctx.check_status()
    assert torch.equal(F1, F2)
    # a batch mixing boxes with and without walls equals the per-box loop
    boxes, Ub, Ul = [], [], []
    for j, (sh, mask) in enumerate([((9, 8, 10), 1), ((8, 12, 9), 0), ((11, 9, 8), 6)]):
        omj = oracle.Mechanism(m, nonperiodic=mask)
        b, Uj, _ = upload_box(omj, fields.sines(sh, 1e-4, m["ns"], 70 + j), 1e-4, mask)
        boxes.append(b)
        Ub.append(Uj)
        Ul.append(Uj.clone())
    s = N.scheme(4, 3, 0, 1)
    dt = time_step("box16_sdc")
    ws, nb = N.workspace(ctx, boxes, s)
    ctx.sdc_step_batched(boxes, Ub, dt, 1, s, ws, nb)
    for b, Uj in zip(boxes, Ul):
        w1, n1 = N.workspace(ctx, [b], s)
        ctx.sdc_step(b, Uj, dt, 1, s, w1, n1)
    ctx.check_status()
    for a, b in zip(Ub, Ul):
        assert torch.equal(G.interior(a), G.interior(b))
    # errors: fewer than 8 cells along a wall direction, bits beyond z, the
    # wide stencil, the adjoint
    small = N.box(7, 9, 9, 1e-4, nonperiodic=1)
    Us = torch.zeros(N.ghosted_shape(5 + m["ns"], 9, 9, 7), dtype=torch.float64, device="cuda")
    Fs = torch.zeros((5 + m["ns"], 9, 9, 7), dtype=torch.float64, device="cuda")
    with pytest.raises(N.NarrowSDCError):
        ctx.rhs_eval(small, Us, Fs, N.RHS_ALL)
    with pytest.raises(N.NarrowSDCError):
        ctx.rhs_eval(N.box(12, 10, 9, 1e-4, nonperiodic=8), U, F1, N.RHS_ALL)
    ctx.set_wide_stencil(True)
    try:
        with pytest.raises(N.NarrowSDCError):
            ctx.rhs_eval(bx, U, F1, N.RHS_ALL)
    finally:
        ctx.set_wide_stencil(False)
    with pytest.raises(N.NarrowSDCError):
        ctx.rhs_vjp(bx, U, torch.zeros_like(F1), torch.zeros_like(F1))
