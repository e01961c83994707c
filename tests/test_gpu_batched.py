"""Batched boxes: one launch per stage over all boxes of uneven sizes,
HIP-graph replay of the step and the tile autotuner (all via the C-ABI)."""
import numpy as np
import pytest

import oracle
from oracle import sdc as osdc
from synth import fields, mechanism
from synth.workloads import WORKLOADS, batch_shapes, time_step

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1309_7327_amd import narrowsdc as N  # noqa: E402
import gpu_util as G  # noqa: E402

WL = WORKLOADS["batch240_sdc"]
SHAPES = batch_shapes(WL["seed"], WL["nbox"])


@pytest.fixture(scope="module")
def setup():
    m = mechanism.load(WL["mech"])
    ctx = N.Context(0)
    ctx.set_mechanism(m)
    return m, oracle.Mechanism(m), ctx


def _states(ctx, m, idx, om=None):
    """Device states of the boxes idx: the library's own conversion, or with
    om the oracle's conserved state uploaded (for oracle comparisons)."""
    boxes, Us = [], []
    for b in idx:
        prim = fields.sines(SHAPES[b], WL["dx"], m["ns"], WL["seed"] + b)
        if om is None:
            bx, U = G.device_state(ctx, prim, WL["dx"])
        else:
            bx, U, _ = G.oracle_state(om, prim, WL["dx"])
        boxes.append(bx)
        Us.append(U)
    return boxes, Us


def _run_batched(ctx, boxes, Us, sch, nsteps, dt, stream=None):
    ws, nb = N.workspace(ctx, boxes, sch)
    ctx.sdc_step_batched(boxes, Us, dt, nsteps, sch, ws, nb, stream=stream)
    ctx.check_status(stream)


def _run_loop(ctx, boxes, Us, sch, nsteps, dt):
    big = max(boxes, key=lambda b: (b.nx + 8) * (b.ny + 8) * (b.nz + 8))
    nb = max(ctx.workspace_size([b], sch) for b in boxes)
    ws = torch.empty(nb // 8 + 1, dtype=torch.float64, device="cuda")
    for bx, U in zip(boxes, Us):
        ctx.sdc_step(bx, U, dt, nsteps, sch, ws, nb)
    ctx.check_status()
    del big


@pytest.mark.parametrize("sch", [N.scheme(4, 6, 0, 1), N.scheme(4, 3, 5, 1)])
def test_batched_equals_per_box_loop(setup, sch):
    m, om, ctx = setup
    idx = [0, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144]
    dt = time_step("batch240_sdc")
    boxes, Ub = _states(ctx, m, idx)
    _, Ul = _states(ctx, m, idx)
    _run_batched(ctx, boxes, Ub, sch, 2, dt)
    _run_loop(ctx, boxes, Ul, sch, 2, dt)
    for a, b in zip(Ub, Ul):
        assert torch.equal(G.interior(a), G.interior(b))


def test_batched_boxes_match_oracle(setup):
    m, om, ctx = setup
    dt = time_step("batch240_sdc")
    # the two smallest boxes of the batch, advanced together with a large one
    order = np.argsort([np.prod(s) for s in SHAPES])
    idx = [int(order[0]), int(order[1]), int(order[-1])]
    boxes, Us = _states(ctx, m, idx, om)
    sch = N.scheme(4, 6, 0, 1)
    _run_batched(ctx, boxes, Us, sch, 1, dt)
    for j in range(2):
        b = idx[j]
        prim = fields.sines(SHAPES[b], WL["dx"], m["ns"], WL["seed"] + b)
        U0 = oracle.prim_to_cons(om, prim)
        f = lambda V, t: oracle.rhs(om, V, WL["dx"])
        ref, fl, dfl = G.ulp_floor_step(
            lambda V, pt: osdc.sdc_run(f, V, 0.0, dt, osdc.gauss_lobatto(4), 6, 1, pt), U0)
        ok, rep = G.compare(G.interior(G.host(Us[j])), ref, fl)
        print(SHAPES[b], G.fmt(rep))
        assert ok, G.fmt(rep)


def test_full_batch_equals_per_box_loop(setup):
    m, om, ctx = setup
    idx = list(range(len(SHAPES)))
    dt = time_step("batch240_sdc")
    sch = N.scheme(4, 6, 0, 1)
    boxes, Ub = _states(ctx, m, idx)
    _run_batched(ctx, boxes, Ub, sch, 1, dt)
    Ub = [G.host(G.interior(u)) for u in Ub]
    torch.cuda.empty_cache()
    _, Ul = _states(ctx, m, idx)
    _run_loop(ctx, boxes, Ul, sch, 1, dt)
    for a, b in zip(Ub, Ul):
        np.testing.assert_array_equal(a, G.host(G.interior(b)))


def test_graph_replays_match_eager(setup):
    m, om, ctx = setup
    idx = [0, 7, 19, 40, 77]
    dt = time_step("batch240_sdc")
    sch = N.scheme(4, 6, 5, 1)
    boxes, U0 = _states(ctx, m, idx)
    init = [u.clone() for u in U0]
    ref = [u.clone() for u in init]
    _run_batched(ctx, boxes, ref, sch, 2, dt)
    ref = [G.host(G.interior(u)) for u in ref]
    stream = torch.cuda.Stream()
    ctx.set_graph(True)
    ws, nb = N.workspace(ctx, boxes, sch)
    work = [u.clone() for u in init]        # the same state buffers every replay
    try:
        for replay in range(4):
            with torch.cuda.stream(stream):     # eager work between replays
                for w, i0 in zip(work, init):
                    w.copy_(i0)
            stream.synchronize()
            ctx.sdc_step_batched(boxes, work, dt, 2, sch, ws, nb, stream=stream.cuda_stream)
            ctx.check_status(stream.cuda_stream)
            for a, b in zip(work, ref):
                np.testing.assert_array_equal(G.host(G.interior(a)), b)
            torch.cuda.synchronize()
    finally:
        ctx.set_graph(False)


def test_autotuned_shapes_give_identical_results(setup):
    m, om, ctx = setup
    idx = list(range(0, len(SHAPES), 3))
    dt = time_step("batch240_sdc")
    sch = N.scheme(4, 2, 0, 1)
    boxes, Ua = _states(ctx, m, idx)
    _, Ub = _states(ctx, m, idx)
    _run_batched(ctx, boxes, Ua, sch, 1, dt)
    ws, nb = N.workspace(ctx, boxes, sch)
    choice = ctx.autotune(boxes, Ub, ws, nb)
    print("autotune choice", choice)
    assert choice[0] * choice[1] * choice[2] <= 256
    _run_batched(ctx, boxes, Ub, sch, 1, dt)
    for a, b in zip(Ua, Ub):
        assert torch.equal(G.interior(a), G.interior(b))


@pytest.mark.parametrize("variant", ["reference_species", "wide_stencil"])
def test_batched_variants_equal_per_box_loop(variant):
    """The reference-species and wide-stencil instances of the stencil
    passes walk the same (box, tile) work lists: batched = per-box loop."""
    m = mechanism.load("mech9le")
    ctx = N.Context(0)
    ctx.set_mechanism(m)
    if variant == "reference_species":
        ctx.set_reference_species(8)
    else:
        ctx.set_wide_stencil(True)
    idx = [0, 3, 8, 21]
    dt = time_step("batch240_sdc")
    sch = N.scheme(4, 4, 0, 1)
    boxes, Ub = _states(ctx, m, idx)
    _, Ul = _states(ctx, m, idx)
    _run_batched(ctx, boxes, Ub, sch, 1, dt)
    _run_loop(ctx, boxes, Ul, sch, 1, dt)
    for a, b in zip(Ub, Ul):
        assert torch.equal(G.interior(a), G.interior(b))
    ctx.close()


def test_batched_21_species_multirate_equals_per_box_loop():
    """Above nine species the fine sweep runs on lane pairs in two waves,
    launched with 128 threads whatever the tile: a batch of ragged boxes (one
    tile shape for all, so tiles cross the boxes' edges) gives the bits of the
    per-box loop (each box with its own default tile)."""
    m = mechanism.load("mech21")
    ctx = N.Context(0)
    ctx.set_mechanism(m)
    shapes = [(13, 9, 7), (24, 16, 16), (40, 11, 6)]
    dt = time_step("box16_sdc")
    sch = N.scheme(4, 2, 5, 1)

    def states():
        boxes, Us = [], []
        for j, sh in enumerate(shapes):
            bx, U = G.device_state(ctx, fields.sines(sh, 1e-4, m["ns"], 50 + j), 1e-4)
            boxes.append(bx)
            Us.append(U)
        return boxes, Us

    boxes, Ub = states()
    _, Ul = states()
    ctx.profile(True)
    _run_batched(ctx, boxes, Ub, sch, 1, dt)
    prof = ctx.profile_read()
    assert "mr_fine" in prof and "mr_src" not in prof
    ctx.profile(False)
    _run_loop(ctx, boxes, Ul, sch, 1, dt)
    for a, b in zip(Ub, Ul):
        assert torch.equal(G.interior(a), G.interior(b)), float((G.interior(a) - G.interior(b)).abs().max())
    ctx.close()
