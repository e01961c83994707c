"""Captured step graphs follow every change of what they depend on: the
stencil variant, the species-diffusion form, the fine-sweep form, the
mechanism and the multirate scheme, and steps with the residual early exit.
Each graph replay is compared bit for
bit with an eager (uncaptured) run of the same configuration, with eager
work and synchronisations between the replays."""
import numpy as np
import pytest

from synth import fields, mechanism
from synth.workloads import time_step

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1309_7327_amd import narrowsdc as N  # noqa: E402
import gpu_util as G  # noqa: E402

SHAPE = (10, 12, 16)     # (nz, ny, nx)
DX = 1e-4


def _configure(ctx, mechs, cfg):
    mech, wide, ref, fused = cfg
    ctx.set_mechanism(mechs[mech])
    ctx.set_wide_stencil(wide)
    ctx.set_reference_species(ref)
    ctx.set_fused_fine(fused)


def _run(ctx, bx, U0, sch, dt, nsteps, stream):
    U = U0.clone()
    ws, nb = N.workspace(ctx, [bx], sch)
    torch.cuda.synchronize()
    ctx.sdc_step(bx, U, dt, nsteps, sch, ws, nb, stream=stream.cuda_stream)
    ctx.check_status(stream.cuda_stream)
    return G.host(G.interior(U))


def test_graphs_follow_setters_and_schemes():
    mechs = {k: mechanism.load(k) for k in ("mech9", "mech9le")}
    ctx = N.Context(0)
    ctx.set_mechanism(mechs["mech9le"])
    prim = fields.sines(SHAPE, DX, 9, 77)
    bx, U0 = G.device_state(ctx, prim, DX)
    dt = time_step("box16_sdc")
    stream = torch.cuda.Stream()
    cfgs = [("mech9le", False, -1, True), ("mech9le", True, -1, True), ("mech9le", False, 8, True),
            ("mech9", False, -1, True), ("mech9le", False, -1, False)]
    schemes = [N.scheme(4, 3, 0, 1), N.scheme(4, 3, 5, 1), N.scheme(4, 3, 3, 2)]
    # eager references
    ctx.set_graph(False)
    ref = {}
    for ci, cfg in enumerate(cfgs):
        _configure(ctx, mechs, cfg)
        for si, sch in enumerate(schemes):
            ref[ci, si] = _run(ctx, bx, U0, sch, dt, 2, stream)
    # the variants really differ (otherwise the test could not see a stale graph)
    assert not np.array_equal(ref[0, 0], ref[1, 0])
    assert not np.array_equal(ref[0, 0], ref[2, 0])
    assert not np.array_equal(ref[0, 1], ref[0, 2])
    ctx.set_graph(True)
    try:
        # captured and replayed, switching configuration and alternating the
        # two multirate schemes between replays; every call uses the same
        # state and workspace addresses
        U = U0.clone()
        order = [(0, 1), (0, 2), (0, 1), (1, 0), (1, 1), (0, 0), (2, 1), (2, 2), (0, 1), (3, 1),
                 (0, 2), (4, 1), (4, 2), (0, 1), (1, 2), (0, 2)]
        wss = {}
        for ci, si in order:
            _configure(ctx, mechs, cfgs[ci])
            sch = schemes[si]
            if si not in wss:
                wss[si] = N.workspace(ctx, [bx], sch)
            ws, nb = wss[si]
            for rep in range(2):
                with torch.cuda.stream(stream):       # eager work between replays
                    U.copy_(U0)
                stream.synchronize()
                ctx.sdc_step(bx, U, dt, 2, sch, ws, nb, stream=stream.cuda_stream)
                ctx.check_status(stream.cuda_stream)
                got = G.host(G.interior(U))
                assert np.array_equal(got, ref[ci, si]), (cfgs[ci], si, rep)
                torch.cuda.synchronize()
    finally:
        ctx.set_graph(False)
        ctx.close()


def test_residual_exit_steps_replay_from_graphs():
    """The residual early exit decides on the device, so its steps are
    captured too: replays of a two-step call give the eager call's state,
    residuals and sweep count bit for bit, with eager work between them,
    and the exit really skipped sweeps."""
    mech = mechanism.load("mech9")
    ctx = N.Context(0)
    ctx.set_mechanism(mech)
    ctx.set_residual_exit(30.0)
    prim = fields.sines((8, 8, 8), DX, 9, 13)
    bx, U0 = G.device_state(ctx, prim, DX)
    dt = time_step("box16_sdc")
    stream = torch.cuda.Stream()
    sch = N.scheme(4, 14, 0, 1)
    ctx.set_graph(False)
    ref = _run(ctx, bx, U0, sch, dt, 2, stream)
    ref_norms, ref_sweeps = ctx.residual_history()
    assert 0 < ref_sweeps < 2 * 14 and len(ref_norms) > 0
    ctx.set_graph(True)
    try:
        U = U0.clone()
        ws, nb = N.workspace(ctx, [bx], sch)
        for rep in range(3):
            with torch.cuda.stream(stream):
                U.copy_(U0)
            stream.synchronize()
            ctx.sdc_step(bx, U, dt, 2, sch, ws, nb, stream=stream.cuda_stream)
            ctx.check_status(stream.cuda_stream)
            assert np.array_equal(G.host(G.interior(U)), ref), rep
            norms, sweeps = ctx.residual_history()
            assert sweeps == ref_sweeps and np.array_equal(norms, ref_norms), rep
            torch.cuda.synchronize()
    finally:
        ctx.set_graph(False)
        ctx.close()


def test_batched_residual_exit_steps_replay_from_graphs():
    """The same for a batch of boxes sharing the exit decision: replays of a
    two-step sdc_step_batched call give the eager call's states, residuals
    and sweep count bit for bit."""
    mech = mechanism.load("mech9")
    ctx = N.Context(0)
    ctx.set_mechanism(mech)
    ctx.set_residual_exit(30.0)
    boxes, init = [], []
    for shape, seed in (((8, 8, 8), 13), ((6, 5, 7), 21)):
        bx, U = G.device_state(ctx, fields.sines(shape, DX, 9, seed), DX)
        boxes.append(bx)
        init.append(U)
    dt = time_step("box16_sdc")
    stream = torch.cuda.Stream()
    sch = N.scheme(4, 14, 0, 1)
    ws, nb = N.workspace(ctx, boxes, sch)
    work = [u.clone() for u in init]
    ctx.sdc_step_batched(boxes, work, dt, 2, sch, ws, nb, stream=stream.cuda_stream)
    ctx.check_status(stream.cuda_stream)
    ref = [G.host(G.interior(u)) for u in work]
    ref_norms, ref_sweeps = ctx.residual_history()
    assert 0 < ref_sweeps < 2 * 14 and len(ref_norms) > 0
    ctx.set_graph(True)
    try:
        for rep in range(3):
            with torch.cuda.stream(stream):
                for w, u in zip(work, init):
                    w.copy_(u)
            stream.synchronize()
            ctx.sdc_step_batched(boxes, work, dt, 2, sch, ws, nb, stream=stream.cuda_stream)
            ctx.check_status(stream.cuda_stream)
            for w, r in zip(work, ref):
                assert np.array_equal(G.host(G.interior(w)), r), rep
            norms, sweeps = ctx.residual_history()
            assert sweeps == ref_sweeps and np.array_equal(norms, ref_norms), rep
            torch.cuda.synchronize()
    finally:
        ctx.set_graph(False)
        ctx.close()


def test_21_species_multirate_steps_replay_from_graphs():
    """The 21-species multirate step (its fine sweep on lane pairs that
    synchronise their workgroup) captured and replayed: every replay gives
    the eager call's bits."""
    mech = mechanism.load("mech21")
    ctx = N.Context(0)
    ctx.set_mechanism(mech)
    bx, U0 = G.device_state(ctx, fields.sines((6, 7, 20), DX, mech["ns"], 29), DX)
    dt = time_step("box16_sdc")
    stream = torch.cuda.Stream()
    sch = N.scheme(4, 2, 5, 1)
    ctx.set_graph(False)
    ref = _run(ctx, bx, U0, sch, dt, 2, stream)
    ctx.set_graph(True)
    try:
        U = U0.clone()
        ws, nb = N.workspace(ctx, [bx], sch)
        for rep in range(3):
            with torch.cuda.stream(stream):
                U.copy_(U0)
            stream.synchronize()
            ctx.sdc_step(bx, U, dt, 2, sch, ws, nb, stream=stream.cuda_stream)
            ctx.check_status(stream.cuda_stream)
            assert np.array_equal(G.host(G.interior(U)), ref), rep
            torch.cuda.synchronize()
    finally:
        ctx.set_graph(False)
        ctx.close()
