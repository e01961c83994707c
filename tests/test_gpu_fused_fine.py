"""Fine sub-steps of the multirate sweep (eq. mrupdate): the one-kernel forms
(quadrature increments kept in registers; above nine species on paired
lanes) against the two-kernel form
(streaming quadrature pass, then the sub-step kernel), through the C-ABI.
Both evaluate the same expressions in the same order, so the states after
whole multirate steps must agree bit for bit; the kernel profile shows
which form ran.  Parity of either form with the oracle is covered by the
multirate step tests of the parity suite, which run the default form."""
import pytest

from synth import fields, mechanism
from synth.workloads import make_primitives, time_step

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1309_7327_amd import narrowsdc as N  # noqa: E402
import gpu_util as G  # noqa: E402


def _run(kind, prim, dx, sch, nsteps, dt, fused):
    m = mechanism.load(kind)
    ctx = N.Context(0)
    ctx.set_mechanism(m)
    ctx.set_fused_fine(fused)
    bx, U = G.device_state(ctx, prim, dx)
    ws, nb = N.workspace(ctx, [bx], sch)
    ctx.profile(True)
    ctx.sdc_step(bx, U, dt, nsteps, sch, ws, nb)
    ctx.check_status()
    prof = ctx.profile_read()
    ctx.close()
    return U, prof


@pytest.mark.parametrize("kind,shape,sch,nsteps", [
    ("mech9", (7, 9, 70), (4, 3, 5, 1), 2),     # GL4 / GL5 type (b); x tile plus a ragged tail
    ("mech9le", (12, 10, 6), (4, 2, 3, 2), 1),  # GL3 repeated twice per coarse interval (type c)
    ("mech21", (5, 6, 9), (4, 2, 5, 1), 1),     # 21 species: the paired-lane one-kernel form
    ("mech21", (6, 5, 7), (4, 2, 3, 2), 1),     # 21 species, GL3 twice per interval (type c)
    ("mech9", (6, 5, 7), (3, 2, 5, 1), 1),      # three coarse nodes: the two-kernel form either way
    ("mech12", (6, 7, 5), (4, 2, 5, 1), 1),     # 12 species: six per lane of a pair
])
def test_fused_fine_equals_two_kernel_form(kind, shape, sch, nsteps):
    m = mechanism.load(kind)
    prim = fields.sines(shape, 1e-4, m["ns"], 31)
    s = N.scheme(*sch)
    dt = time_step("box16_sdc")
    Uf, pf = _run(kind, prim, 1e-4, s, nsteps, dt, True)
    Us, ps = _run(kind, prim, 1e-4, s, nsteps, dt, False)
    applies = sch[0] == 4 and (sch[2] - 1) * sch[3] == 4
    print(kind, shape, sch, "one-kernel form applies:", applies, {k: v[1] for k, v in pf.items()})
    assert ("mr_src" not in pf) == applies
    assert "mr_src" in ps and "mr_fine" in pf and "mr_fine" in ps
    assert torch.equal(Uf, Us), float((Uf - Us).abs().max())


def test_fused_fine_equals_two_kernel_form_at_full_size():
    """The 128^3, 9-species headline box, one multirate step."""
    m = mechanism.load("mech9")
    prim = make_primitives("box128_mrsdc", m)
    s = N.scheme(4, 6, 5, 1)
    dt = time_step("box128_mrsdc")
    Uf, pf = _run("mech9", prim, 1e-4, s, 1, dt, True)
    Us, ps = _run("mech9", prim, 1e-4, s, 1, dt, False)
    assert "mr_src" not in pf and "mr_src" in ps
    same = torch.equal(Uf, Us)
    diff = float((Uf - Us).abs().max())
    del Uf, Us
    torch.cuda.empty_cache()
    assert same, diff


def test_two_lanes_per_cell_with_an_odd_reaction_count():
    """Above nine species the fine sub-steps split a cell's reactions between
    two lanes (every other reaction each); with an odd count one lane takes one
    more.  83 of the 21-species mechanism's 84 reactions, one multirate step on
    a ragged box, against the oracle."""
    import numpy as np
    import oracle
    from oracle import sdc as osdc

    m = dict(mechanism.load("mech21"))
    keep = 83
    for k in ("A", "b", "Ea", "nu_f", "nu_r"):
        m[k] = np.ascontiguousarray(m[k][:keep])
    m["nr"] = keep
    om = oracle.Mechanism(m)
    ctx = N.Context(0)
    ctx.set_mechanism(m)
    shape = (5, 6, 7)
    prim = fields.sines(shape, 1e-4, m["ns"], 17)
    bx, U, U0 = G.oracle_state(om, prim, 1e-4)
    U0g = U0
    dt = time_step("box16_sdc")
    s = N.scheme(4, 2, 5, 1)
    ws, nb = N.workspace(ctx, [bx], s)
    ctx.profile(True)
    ctx.sdc_step(bx, U, dt, 1, s, ws, nb)
    ctx.check_status()
    assert "mr_fine" in ctx.profile_read()
    Ug = G.interior(G.host(U))
    ctx.close()

    def step(V, pt):
        f1 = lambda W, t: oracle.rhs(om, W, 1e-4, parts=oracle.AD)
        f2 = lambda W, t: oracle.rhs(om, W, 1e-4, parts=oracle.REACT)
        t1, t2, pieces = osdc.mr_nodes(4, 5, 1)
        return osdc.mrsdc_run(f1, f2, V, 0.0, dt, t1, t2, pieces, 2, 1, pt)

    ref, floor, dfloor = G.ulp_floor_step(step, U0)
    ok, rep = G.compare(Ug, ref, floor)
    okd, repd = G.compare(Ug - U0g, ref - U0, dfloor, state=ref)
    print("U ", G.fmt(rep))
    print("dU", G.fmt(repd))
    assert ok and okd, G.fmt(repd)


def test_two_lanes_per_cell_is_deterministic():
    """The paired-lane sub-step kernel sums a cell's production from its two
    lanes (in two waves, each lane into its own array, the two added in a
    fixed order): repeated 21-species multirate steps (several workgroups,
    ragged tail, whose cell slots past the box compute on the tile's first
    cell and store nothing) and other tile shapes, among them tiles of 64 and
    192 cells, give the same bits."""
    m = mechanism.load("mech21")
    shape = (20, 18, 40)
    prim = fields.sines(shape, 1e-4, m["ns"], 37)
    s = N.scheme(4, 2, 5, 1)
    dt = time_step("box16_sdc")
    ctx = N.Context(0)
    ctx.set_mechanism(m)
    outs = []
    for tiles in [None, None, ((16, 4, 4), (16, 4, 4)), ((8, 8, 1), (16, 4, 4)), ((16, 4, 3), (16, 4, 4))]:
        if tiles is not None:
            ctx.set_tiles(*tiles, grid_cap=37)
        bx, U = G.device_state(ctx, prim, 1e-4)
        ws, nb = N.workspace(ctx, [bx], s)
        ctx.profile(True)
        ctx.sdc_step(bx, U, dt, 1, s, ws, nb)
        ctx.check_status()
        assert "mr_fine" in ctx.profile_read()
        outs.append(U)
    ctx.set_tiles()
    ctx.close()
    for U in outs[1:]:
        assert torch.equal(U, outs[0]), float((U - outs[0]).abs().max())
