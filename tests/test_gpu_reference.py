"""Reference-species form of the species diffusion (Section 2.1, with the
h_k - h_ref energy flux of Section 2.4): parity of the HIP path with the
oracle's reference form, through the C-ABI."""
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


def _ctx(kind, ref):
    m = mechanism.load(kind)
    ctx = N.Context(0)
    ctx.set_mechanism(m)
    ctx.set_reference_species(ref)
    return m, oracle.Mechanism(m, ref_species=ref), ctx


@pytest.mark.parametrize("parts", [N.RHS_DIFF, N.RHS_ALL])
@pytest.mark.parametrize("kind,shape,dx,ref", [
    ("mech9le", (5, 6, 7), (1e-4, 1.2e-4, 0.9e-4), 8),   # ragged, anisotropic; N2 as reference
    ("mech9le", (24, 20, 36), 1e-4, 0),                  # several tiles with ragged tails
    ("mech21", (9, 12, 20), 1e-4, 20),                   # 21 species (LDS accumulators)
])
def test_reference_species_rhs_parity(kind, shape, dx, ref, parts):
    m, om, ctx = _ctx(kind, ref)
    prim = fields.sines(shape, dx, m["ns"], 21)
    bx, U, Uo = G.oracle_state(om, prim, dx)
    F = torch.zeros((5 + m["ns"],) + shape, dtype=torch.float64, device="cuda")
    ctx.rhs_eval(bx, U, F, parts)
    ctx.check_status()
    fref, floor = G.ulp_floor(lambda V: oracle.rhs(om, V, dx, parts=parts), Uo)
    ok, rep = G.compare(G.host(F), fref, floor)
    print(kind, shape, ref, parts, G.fmt(rep))
    assert ok, G.fmt(rep)
    ctx.close()


@pytest.mark.parametrize("sch,nsteps", [(dict(n_coarse=3, sweeps=4, n_fine=0), 2),
                                        (dict(n_coarse=4, sweeps=6, n_fine=5, fine_repeat=1), 1)])
def test_reference_species_sdc_step_parity(sch, nsteps):
    m, om, ctx = _ctx("mech9le", 8)
    shape = (6, 5, 7)
    prim = fields.sines(shape, 1e-4, m["ns"], 23)
    bx, U, U0 = G.oracle_state(om, prim, 1e-4)
    U0g = U0
    dt = time_step("box16_sdc")
    s = N.scheme(sch["n_coarse"], sch["sweeps"], sch["n_fine"], sch.get("fine_repeat", 1))
    ws, nb = N.workspace(ctx, [bx], s)
    ctx.sdc_step(bx, U, dt, nsteps, s, ws, nb)
    ctx.check_status()
    Ug = G.interior(G.host(U))

    def step(V, pt):
        if sch["n_fine"] == 0:
            f = lambda W, t: oracle.rhs(om, W, 1e-4)
            return osdc.sdc_run(f, V, 0.0, dt, osdc.gauss_lobatto(sch["n_coarse"]), sch["sweeps"], nsteps, pt)
        f1 = lambda W, t: oracle.rhs(om, W, 1e-4, parts=oracle.AD)
        f2 = lambda W, t: oracle.rhs(om, W, 1e-4, parts=oracle.REACT)
        t1, t2, pieces = osdc.mr_nodes(sch["n_coarse"], sch["n_fine"], sch["fine_repeat"])
        return osdc.mrsdc_run(f1, f2, V, 0.0, dt, t1, t2, pieces, sch["sweeps"], nsteps, pt)
    ref, floor, dfloor = G.ulp_floor_step(step, U0)
    ok, rep = G.compare(Ug, ref, floor)
    okd, repd = G.compare(Ug - U0g, ref - U0, dfloor, state=ref)
    print("U ", G.fmt(rep))
    print("dU", G.fmt(repd))
    assert ok and okd, G.fmt(repd)
    ctx.close()


def test_sampled_cells_of_full_size_reference_species_rhs():
    """The 128^3 flame of the reference-species workload: right-hand side at
    sampled cells, in the launch configuration the bench times."""
    name = "box128_mrsdc_n2ref"
    wl = WORKLOADS[name]
    m, om, ctx = _ctx(wl["mech"], wl["ref_species"])
    prim = make_primitives(name, m)
    bx, U, Ui = G.oracle_state(om, prim, wl["dx"])
    shape = wl["shape"]
    F = torch.zeros((5 + m["ns"],) + shape, dtype=torch.float64, device="cuda")
    ctx.rhs_eval(bx, U, F, N.RHS_ALL)
    ctx.check_status()
    Fh = G.host(F)
    rng = np.random.default_rng(5)
    cells = rng.integers(0, shape[0], size=(48, 3))
    cells[:4] = [[0, 0, 0], [127, 127, 127], [0, 127, 3], [64, 0, 127]]
    ref = oracle.rhs_cells(om, Ui, wl["dx"], cells)
    rng2 = np.random.default_rng(12345)
    ref_p = oracle.rhs_cells(om, Ui * (1 + 2.0 ** -52 * rng2.standard_normal(Ui.shape)), wl["dx"], cells)
    got = np.stack([Fh[:, z, y, x] for x, y, z in cells])
    floor = np.abs(ref_p - ref).max(axis=0)
    ok, rep = G.compare(got.T, ref.T, floor)
    print(G.fmt(rep))
    assert ok, G.fmt(rep)
    ctx.close()


def test_reference_species_switching_and_errors():
    m, _, ctx = _ctx("mech9le", 8)
    shape, dx = (8, 9, 10), 1e-4
    prim = fields.sines(shape, dx, m["ns"], 25)
    bx, U = G.device_state(ctx, prim, dx)

    def rhs():
        F = torch.zeros((5 + m["ns"],) + shape, dtype=torch.float64, device="cuda")
        ctx.rhs_eval(bx, U, F, N.RHS_ALL)
        ctx.check_status()
        return G.host(F)

    f_ref = rhs()
    ctx.set_reference_species(-1)
    f_vc = rhs()
    assert not np.array_equal(f_ref, f_vc)
    # a fresh context in the default (correction-velocity) form agrees bitwise
    ctx2 = N.Context(0)
    ctx2.set_mechanism(m)
    _, U2 = G.device_state(ctx2, prim, dx)
    F2 = torch.zeros((5 + m["ns"],) + shape, dtype=torch.float64, device="cuda")
    ctx2.rhs_eval(bx, U2, F2, N.RHS_ALL)
    ctx2.check_status()
    np.testing.assert_array_equal(f_vc, G.host(F2))
    ctx2.close()
    ctx.set_reference_species(8)
    np.testing.assert_array_equal(rhs(), f_ref)
    for bad in (-2, m["ns"]):
        with pytest.raises(N.NarrowSDCError):
            ctx.set_reference_species(bad)
    # the adjoint covers the correction-velocity form only
    v = torch.zeros((5 + m["ns"],) + shape, dtype=torch.float64, device="cuda")
    with pytest.raises(N.NarrowSDCError):
        ctx.rhs_vjp(bx, U, v, torch.zeros_like(v))
    # a new mechanism starts in the correction-velocity form
    ctx.set_mechanism(m)
    np.testing.assert_array_equal(rhs(), f_vc)
    ctx.close()
