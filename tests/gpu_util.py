"""Helpers shared by the GPU tests: device states, oracle comparisons and the
parity criterion.

Parity criterion (per output field q): the HIP result f and the oracle's
f_ref agree if  max|f - f_ref| <= max(tol * max|f_ref|, 4 * floor_q),
(for a step increment dU the floor is at least one ulp of max|U_end|),
where floor_q = max|f_ref(U (1 + 2^-52 r)) - f_ref(U)| is the oracle's own
response to a random one-ulp relative perturbation of its input (r ~ N(0,1),
fixed seed).  tol is 1e-12 for right-hand sides and states.  The floor only
matters where the FP64 problem itself is worse conditioned than 1e-12 (the
momentum equations, where the pressure ~1e5 Pa is differenced over
dx = 1e-4 m); it is reported next to every comparison.
"""
import numpy as np
import torch

import oracle
from paper_1309_7327_amd import narrowsdc as N

NG = N.NG


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    return t.detach().to("cpu").numpy()


def interior(U):
    return U[:, NG:-NG, NG:-NG, NG:-NG]


def device_state(ctx, prim, dx):
    """Conserved ghosted state on the device from primitive fields (the HIP
    library's own conversion)."""
    nz, ny, nx = prim["T"].shape
    bx = N.box(nx, ny, nz, *np.broadcast_to(np.asarray(dx, dtype=np.float64), (3,)))
    ns = prim["Y"].shape[0]
    U = torch.zeros(N.ghosted_shape(5 + ns, nz, ny, nx), dtype=torch.float64, device="cuda")
    ctx.prim_to_cons(bx, dev(prim["p"]), dev(prim["T"]), dev(prim["Y"]), dev(prim["u"]), U)
    return bx, U


def ulp_floor(fn, U, seed=12345):
    """Per-field oracle response to a one-ulp random relative input change."""
    rng = np.random.default_rng(seed)
    f0 = fn(U)
    f1 = fn(U * (1.0 + 2.0 ** -52 * rng.standard_normal(U.shape)))
    return f0, np.abs(f1 - f0).reshape(f0.shape[0], -1).max(axis=1)


def ulp_floor_step(step, U0, seed=12345):
    """For a time-step map step(U, perturb): (step(U0), floor of the state,
    floor of the increment step(U) - U).  The floors are the change of the
    oracle's result when its input and every state it computes along the way
    are multiplied by (1 + 2^-52 r), r ~ N(0, 1): the FP64 rounding noise of
    the integration itself."""
    rng = np.random.default_rng(seed)
    U0p = U0 * (1.0 + 2.0 ** -52 * rng.standard_normal(U0.shape))
    pert = lambda U: U * (1.0 + 2.0 ** -52 * rng.standard_normal(U.shape))
    r0, r1 = step(U0, None), step(U0p, pert)
    nq = U0.shape[0]
    fU = np.abs(r1 - r0).reshape(nq, -1).max(axis=1)
    fd = np.abs((r1 - U0p) - (r0 - U0)).reshape(nq, -1).max(axis=1)
    return r0, fU, fd


def compare(f, fref, floor=None, tol=1e-12, state=None):
    """Returns (ok, report) under the parity criterion.  For increments
    dU = U_end - U_0 pass the end state as `state`: the increment cannot be
    more precise than the FP64 rounding of the state it is taken from, so
    the floor is at least one ulp of max|U_end| (the bound four)."""
    nq = fref.shape[0]
    rep = []
    ok = True
    for q in range(nq):
        err = float(np.abs(f[q] - fref[q]).max())
        scale = float(np.abs(fref[q]).max())
        fl = float(floor[q]) if floor is not None else 0.0
        if state is not None:
            fl = max(fl, 2.0 ** -52 * float(np.abs(state[q]).max()))
        bound = max(tol * scale, 4.0 * fl)
        ok &= err <= bound
        rep.append((q, err / scale if scale > 0 else err, fl / scale if scale > 0 else fl, err <= bound))
    return ok, rep


def fmt(rep):
    return " ".join(f"[{q}:{e:.1e}/{fl:.1e}{'' if ok else ' FAIL'}]" for q, e, fl, ok in rep)
