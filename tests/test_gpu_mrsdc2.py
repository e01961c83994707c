"""Multirate SDC mode 2 (eq. mrupdate2) on the GPU against the oracle: the
chemistry implicit on the coarse nodes (per-cell Newton solves of the
backward-Euler equation of each coarse interval), advection-diffusion
explicit on the fine nodes.  Both sides start from the oracle's conserved
state; the parity criterion is the suite's (tests/gpu_util.py)."""
import numpy as np
import pytest

import oracle
from oracle import implicit as OI
from oracle import sdc as osdc
from synth import fields, mechanism
from synth.workloads import time_step

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1309_7327_amd import narrowsdc as N  # noqa: E402
import gpu_util as G  # noqa: E402

MECHS = {}


def mech(kind):
    if kind not in MECHS:
        m = mechanism.load(kind)
        ctx = N.Context(0)
        ctx.set_mechanism(m)
        MECHS[kind] = (m, oracle.Mechanism(m), ctx)
    return MECHS[kind]


def oracle_mode2(om, dx, V, dt, nc, nf, rep, K, nsteps, pt=None):
    f1 = lambda U, t: oracle.rhs(om, U, dx, parts=oracle.REACT)
    f2 = lambda U, t: oracle.rhs(om, U, dx, parts=oracle.AD)
    solve1 = lambda rhs, h: OI.implicit_reaction(om, rhs, h, dx)
    t1, t2, pieces = osdc.mr_nodes(nc, nf, rep)
    return osdc.mrsdc2_run(f1, solve1, f2, V, 0.0, dt, t1, t2, pieces, K, nsteps, pt)


@pytest.mark.parametrize("kind,shape,sch,nsteps,dtmul", [
    ("mech9", (8, 8, 8), (3, 4, 3, 2), 2, 1.0),       # GL3 coarse, GL3 fine twice per interval
    ("mech9", (6, 7, 5), (4, 3, 5, 1), 1, 1.0),       # GL4 coarse, GL5 fine (type b)
    ("mech9le", (6, 5, 7), (3, 3, 3, 2), 1, 8.0),     # a step 8x the explicit workload's
    ("mech21", (5, 6, 7), (3, 2, 3, 1), 1, 1.0),      # 21 species
    ("mech12", (6, 5, 5), (3, 2, 3, 1), 1, 1.0),      # 12 species
])
def test_mode2_step_parity(kind, shape, sch, nsteps, dtmul):
    m, om, ctx = mech(kind)
    prim = fields.sines(shape, 1e-4, m["ns"], 41)
    bx, U, U0 = G.oracle_state(om, prim, 1e-4)
    dt = dtmul * time_step("box16_sdc")
    nc, K, nf, rep = sch
    s = N.scheme(nc, K, nf, rep, mode=2)
    ws, nb = N.workspace(ctx, [bx], s)
    print(f"mode 2 {kind} {shape} scheme {sch} steps {nsteps} dt x{dtmul}", flush=True)
    ctx.profile(True)
    ctx.sdc_step(bx, U, dt, nsteps, s, ws, nb)
    ctx.check_status()
    prof = ctx.profile_read()
    ctx.profile(False)
    assert "mr2_imp" in prof and "mr_fine" not in prof
    Ug = G.interior(G.host(U))
    ref, floor, dfloor = G.ulp_floor_step(lambda V, pt: oracle_mode2(om, 1e-4, V, dt, nc, nf, rep, K, nsteps, pt),
                                          U0)
    ok, rep_ = G.compare(Ug, ref, floor)
    okd, repd = G.compare(Ug - U0, ref - U0, dfloor, state=ref)
    print("U ", G.fmt(rep_))
    print("dU", G.fmt(repd))
    assert ok and okd, G.fmt(repd)


def test_mode2_batched_equals_per_box_loop_and_graph_replays():
    m, om, ctx = mech("mech9")
    shapes = [(6, 7, 8), (9, 5, 6), (4, 4, 12)]
    s = N.scheme(3, 3, 3, 2, mode=2)
    dt = time_step("box16_sdc")
    boxes, Ub, Ul = [], [], []
    for j, sh in enumerate(shapes):
        prim = fields.sines(sh, 1e-4, m["ns"], 50 + j)
        bx, U, _ = G.oracle_state(om, prim, 1e-4)
        boxes.append(bx)
        Ub.append(U)
        Ul.append(U.clone())
    ws, nb = N.workspace(ctx, boxes, s)
    ctx.sdc_step_batched(boxes, Ub, dt, 2, s, ws, nb)
    for bx, U in zip(boxes, Ul):
        w1, n1 = N.workspace(ctx, [bx], s)
        ctx.sdc_step(bx, U, dt, 2, s, w1, n1)
    ctx.check_status()
    for a, b in zip(Ub, Ul):
        assert torch.equal(G.interior(a), G.interior(b))
    # a captured step call replays to the eager result (same state and
    # workspace addresses on every call, eager work between the replays)
    bx = boxes[0]
    prim = fields.sines(shapes[0], 1e-4, m["ns"], 50)
    _, Ue, _ = G.oracle_state(om, prim, 1e-4)
    Uinit = Ue.clone()
    w1, n1 = N.workspace(ctx, [bx], s)
    ctx.sdc_step(bx, Ue, dt, 1, s, w1, n1)
    ctx.check_status()
    st = torch.cuda.Stream()
    Ur = torch.empty_like(Ue)
    ctx.set_graph(True)
    try:
        for _ in range(3):
            with torch.cuda.stream(st):
                Ur.copy_(Uinit)
            st.synchronize()
            ctx.sdc_step(bx, Ur, dt, 1, s, w1, n1, stream=st.cuda_stream)
            ctx.check_status(st.cuda_stream)
            assert torch.equal(G.interior(Ur), G.interior(Ue))
            torch.cuda.synchronize()
    finally:
        ctx.set_graph(False)


def test_mode2_argument_errors():
    m, om, ctx = mech("mech9")
    prim = fields.sines((4, 5, 6), 1e-4, m["ns"], 3)
    bx, U, _ = G.oracle_state(om, prim, 1e-4)
    for bad in (N.scheme(3, 2, 0, 1, mode=2), N.scheme(3, 2, 3, 1, mode=3), N.scheme(3, 2, 3, 1, mode=-1)):
        with pytest.raises(N.NarrowSDCError):
            ctx.workspace_size([bx], bad)
    # the adjoint covers single-rate SDC only
    s = N.scheme(3, 2, 3, 1, mode=2)
    with pytest.raises(N.NarrowSDCError):
        ctx.vjp_workspace_size(bx, s, 1)


def test_mode2_full_size_step_on_periodic_tiling():
    """The 128^3 implicit-chemistry workload's step in the benchmark's launch
    configuration, on a state that repeats a 16^3 box of the same recipe: the
    exact result is the 16^3 box's step repeated, which the oracle computes."""
    from synth.workloads import WORKLOADS, make_primitives
    name = "box128_mrsdc2"
    wl = WORKLOADS[name]
    m, om, ctx = mech(wl["mech"])
    sd = wl["scheme"]
    n = wl["shape"][0]
    small = make_primitives(name, m, shape_override=(16, 16, 16))
    U0s = oracle.prim_to_cons(om, small)
    reps_q = (1,) + (n // 16,) * 3
    bx, U = G.upload(np.tile(U0s, reps_q), wl["dx"])
    dt = time_step(name)
    s = N.scheme(sd["n_coarse"], sd["sweeps"], sd["n_fine"], sd["fine_repeat"], mode=2)
    ws, nb = N.workspace(ctx, [bx], s)
    print(f"mode 2 {name} 1 step", flush=True)
    ctx.sdc_step(bx, U, dt, 1, s, ws, nb)
    ctx.check_status()
    Ug = G.interior(G.host(U))
    del U, ws
    torch.cuda.empty_cache()
    ref, floor, dfloor = G.ulp_floor_step(
        lambda V, pt: oracle_mode2(om, wl["dx"], V, dt, sd["n_coarse"], sd["n_fine"], sd["fine_repeat"],
                                   sd["sweeps"], 1, pt), U0s)
    ok, rep_ = G.compare(Ug, np.tile(ref, reps_q), floor)
    okd, repd = G.compare(Ug - np.tile(U0s, reps_q), np.tile(ref - U0s, reps_q), dfloor, state=ref)
    print("U ", G.fmt(rep_))
    print("dU", G.fmt(repd))
    assert ok and okd, G.fmt(repd)
