"""SDC residual early exit (eq. residual): the HIP driver's residuals,
sweep counts and end states against the oracle's, through the C-ABI."""
import numpy as np
import pytest

import oracle
from oracle import sdc as osdc
from synth import fields, mechanism
from synth.workloads import time_step

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1309_7327_amd import narrowsdc as N  # noqa: E402
import gpu_util as G  # noqa: E402


def _ctx(kind):
    m = mechanism.load(kind)
    ctx = N.Context(0)
    ctx.set_mechanism(m)
    return m, oracle.Mechanism(m), ctx


@pytest.mark.parametrize("kind,shape,K,ratio,nsteps", [
    ("mech9", (8, 8, 8), 14, 30.0, 3),       # each step stops after 3 sweeps (ratios 142/9.4, 91/15, 65/22)
    ("mech9le", (6, 5, 7), 10, 20.0, 1),     # stops after 3 sweeps, the residual still shrinking (ratios 122, 11)
])
def test_residual_exit_parity(kind, shape, K, ratio, nsteps):
    m, om, ctx = _ctx(kind)
    ctx.set_residual_exit(ratio)
    prim = fields.sines(shape, 1e-4, m["ns"], 13)
    bx, U, U0 = G.oracle_state(om, prim, 1e-4)
    U0g = U0
    dt = time_step("box16_sdc")
    s = N.scheme(4, K, 0, 1)
    ws, nb = N.workspace(ctx, [bx], s)
    ctx.sdc_step(bx, U, dt, nsteps, s, ws, nb)
    ctx.check_status()
    norms, sweeps = ctx.residual_history()
    Ug = G.interior(G.host(U))
    hist = []
    f = lambda V, t: oracle.rhs(om, V, 1e-4)
    ref = osdc.sdc_run(f, U0, 0.0, dt, osdc.gauss_lobatto(4), K, nsteps, residual_ratio=ratio, history=hist)
    rs = np.array([h[2] for h in hist if h[0] != "sweeps"])
    osw = [h[1] for h in hist if h[0] == "sweeps"]
    print("sweeps", sweeps, osw, "residuals", norms, rs)
    assert sweeps < nsteps * K
    # every exit decision of these cases is far from the threshold (at least
    # 5% in the ratio) and taken on residuals far above rounding level
    # (>= 1e-10 of max|U_0|), where the two sides' residuals agree to ~1e-12
    # relative: the sweep counts must agree exactly
    prev = None
    for h in hist:
        if h[0] == "sweeps":
            prev = None
            continue
        assert h[2] > 1e-10
        if prev is not None:
            assert abs(np.log(prev / h[2]) - np.log(ratio)) > np.log(1.05), (prev, h[2])
        prev = h[2]
    assert sweeps == sum(osw)
    # the residual is a difference of states of order one (relative to
    # max|U_0|) formed in another rounding order: it agrees to rounding level
    # in absolute terms, 1e-14 (about 50 ulp), and to 1e-6 where it is large
    assert len(norms) == len(rs)
    np.testing.assert_allclose(norms, rs, rtol=1e-6, atol=1e-14)
    _, floor, dfloor = G.ulp_floor_step(
        lambda V, pt: osdc.sdc_run(f, V, 0.0, dt, osdc.gauss_lobatto(4), K, nsteps, pt, residual_ratio=ratio), U0)
    ok, rep = G.compare(Ug, ref, floor)
    okd, repd = G.compare(Ug - U0g, ref - U0, dfloor, state=ref)
    print("U ", G.fmt(rep))
    print("dU", G.fmt(repd))
    assert ok and okd, G.fmt(repd)
    ctx.close()


def _flat_sdc(om, U0s, dx, dt, K, nsteps, ratio, hist=None):
    """The oracle's step of several boxes advanced together: their interiors
    side by side along one cell axis, the right-hand side evaluated box by
    box, so the residual (and the exit decision) is the batch's.  Returns
    step(V, perturb) on the joined state and the split back into boxes."""
    nc = U0s[0].shape[0]
    sizes = [u[0].size for u in U0s]

    def split(V):
        out, o = [], 0
        for u, n in zip(U0s, sizes):
            out.append(V[:, o:o + n].reshape(u.shape))
            o += n
        return out

    def f(V, t):
        return np.concatenate([oracle.rhs(om, p, dx).reshape(nc, -1) for p in split(V)], axis=1)

    def step(V, pt):
        return osdc.sdc_run(f, V, 0.0, dt, osdc.gauss_lobatto(4), K, nsteps, pt, residual_ratio=ratio,
                            history=hist if pt is None else None)

    return step, split, np.concatenate([u.reshape(nc, -1) for u in U0s], axis=1)


def test_residual_exit_batched_parity():
    """Boxes advanced by one sdc_step_batched call share the exit decision:
    |R| is taken over all their interiors (the largest over components of
    max|R_c| / max|U_0,c|, both maxima over the batch).  Against the oracle
    run on the boxes joined along one cell axis."""
    m, om, ctx = _ctx("mech9")
    ratio, K, nsteps = 30.0, 14, 2
    ctx.set_residual_exit(ratio)
    dt = time_step("box16_sdc")
    boxes, Us, U0s = [], [], []
    for shape, seed in (((8, 8, 8), 13), ((6, 5, 7), 21)):
        bx, U, U0 = G.oracle_state(om, fields.sines(shape, 1e-4, m["ns"], seed), 1e-4)
        boxes.append(bx)
        Us.append(U)
        U0s.append(U0)
    s = N.scheme(4, K, 0, 1)
    ws, nb = N.workspace(ctx, boxes, s)
    ctx.sdc_step_batched(boxes, Us, dt, nsteps, s, ws, nb)
    ctx.check_status()
    norms, sweeps = ctx.residual_history()
    hist = []
    step, split, V0 = _flat_sdc(om, U0s, 1e-4, dt, K, nsteps, ratio, hist)
    Vend, floor, dfloor = G.ulp_floor_step(step, V0)
    ref = split(Vend)
    rs = np.array([h[2] for h in hist if h[0] != "sweeps"])
    osw = [h[1] for h in hist if h[0] == "sweeps"]
    print("sweeps", sweeps, osw, "residuals", norms, rs)
    # decisions far from the threshold (ratios 110 and 6.8, then 60 and 13)
    prev = None
    for h in hist:
        if h[0] == "sweeps":
            prev = None
            continue
        assert h[2] > 1e-10
        if prev is not None:
            assert abs(np.log(prev / h[2]) - np.log(ratio)) > np.log(1.05), (prev, h[2])
        prev = h[2]
    assert sweeps == sum(osw) < nsteps * K
    assert len(norms) == len(rs)
    np.testing.assert_allclose(norms, rs, rtol=1e-6, atol=1e-14)
    for U, r, U0 in zip(Us, ref, U0s):
        Ug = G.interior(G.host(U))
        ok, rep = G.compare(Ug, r, floor)
        okd, repd = G.compare(Ug - U0, r - U0, dfloor, state=r)
        print("U ", G.fmt(rep))
        print("dU", G.fmt(repd))
        assert ok and okd, G.fmt(repd)
    ctx.close()


def test_residual_exit_off_is_the_fixed_sweep_step_and_errors():
    m, om, ctx = _ctx("mech9")
    shape = (8, 9, 10)
    prim = fields.sines(shape, 1e-4, m["ns"], 15)
    dt = time_step("box16_sdc")
    s = N.scheme(4, 6, 0, 1)
    outs = []
    for ratio in (1.5, 0.0):
        ctx.set_residual_exit(ratio)
        bx, U = G.device_state(ctx, prim, 1e-4)
        ws, nb = N.workspace(ctx, [bx], s)
        ctx.sdc_step(bx, U, dt, 1, s, ws, nb)
        ctx.check_status()
        outs.append((G.host(U), ctx.residual_history()))
    assert outs[1][1][1] == 6 and len(outs[1][1][0]) == 0
    # a fresh context (exit off by default) gives the same bits
    m2, _, ctx2 = _ctx("mech9")
    bx, U = G.device_state(ctx2, prim, 1e-4)
    ws, nb = N.workspace(ctx2, [bx], s)
    ctx2.sdc_step(bx, U, dt, 1, s, ws, nb)
    np.testing.assert_array_equal(G.host(U), outs[1][0])
    ctx2.close()
    for bad in (0.5, 1.0, -2.0):
        with pytest.raises(N.NarrowSDCError):
            ctx.set_residual_exit(bad)
    ctx.set_residual_exit(1.5)
    bx, U = G.device_state(ctx, prim, 1e-4)
    with pytest.raises(N.NarrowSDCError):          # multirate scheme
        smr = N.scheme(4, 6, 5, 1)
        ws, nb = N.workspace(ctx, [bx], smr)
        ctx.sdc_step(bx, U, dt, 1, smr, ws, nb)
    with pytest.raises(N.NarrowSDCError):          # the adjoint
        v = torch.zeros((5 + m["ns"],) + shape, dtype=torch.float64, device="cuda")
        ctx.rhs_vjp(bx, U, v, torch.zeros_like(v))
    ctx.close()
