"""Helpers shared by the GPU tests: device states, oracle comparisons and the
parity criterion.

Parity criterion (per output field q): the HIP result f and the oracle's
f_ref agree if  max|f - f_ref| <= max(tol * max|f_ref|, 4 * floor_q),
(for a step increment dU the floor is at least one ulp of max|U_end|),
where floor_q = max|f_ref(U (1 + 2^-52 r)) - f_ref(U)| is the oracle's own
response to a random one-ulp relative perturbation of its input (r ~ N(0,1),
fixed seed).  tol is 1e-12 for right-hand sides and states.

Where the FP64 problem is conditioned better than 1e-12 (4 floor_q <=
1e-12 max|f_ref|: every right-hand-side field but momentum, every state
field after a step) the bound is 1e-12 relative.  The momentum equations difference the pressure
(~1e5 Pa) over dx = 1e-4 m, so a one-ulp change of the inputs moves their
right-hand side by 5e-12 to 1.6e-11 of its maximum: 1e-12 is below the
conditioning of the problem there, and the bound is 4 floor_q.  A step
increment dU is about 1e-4 of U, so one ulp of U is ~2e-12 of dU: the
increments are held to the floor as well.  Why 4: the
two sides round independently, each as if its input carried about one ulp
of noise, so their difference behaves like the response to sqrt(2) ulp;
and floor_q is one sample of a random maximum, whose spread over seeds is
at most 2.8x (pinned on the CPU: tests/test_parity_criterion.py).
sqrt(2) * 2.8 = 3.96 <= 4.  Fields held to the floor are marked '*' in the
report; the report gives every field's max-norm relative error.

Both sides of a comparison start from the same bits: the oracle's
conserved state, uploaded to the device (oracle_state, upload).
"""
import numpy as np
import torch

import oracle
from paper_1309_7327_amd import narrowsdc as N

NG = N.NG
# multiple of the oracle's one-ulp noise floor accepted where the problem's
# conditioning is worse than the relative tolerance (derivation above)
FLOOR_FACTOR = 4.0


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


def upload(U, dx):
    """An interior conserved state [nU][nz][ny][nx] (host) -> (box, ghosted
    device array); the library fills the ghost layers on use."""
    nU, nz, ny, nx = U.shape
    bx = N.box(nx, ny, nz, *np.broadcast_to(np.asarray(dx, dtype=np.float64), (3,)))
    Ug = torch.zeros(N.ghosted_shape(nU, nz, ny, nx), dtype=torch.float64, device="cuda")
    N.interior(Ug).copy_(dev(U))
    return bx, Ug


def oracle_state(om, prim, dx):
    """The oracle's conserved state from primitive fields, and the same bits
    on the device: both sides of a parity comparison start from one input,
    so input rounding is not counted twice.  Returns (box, device U, host U)."""
    Uo = oracle.prim_to_cons(om, prim)
    bx, Ug = upload(Uo, dx)
    return bx, Ug, Uo


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
        bound = max(tol * scale, FLOOR_FACTOR * fl)
        ok &= err <= bound
        rep.append((q, err / scale if scale > 0 else err, fl / scale if scale > 0 else fl, err <= bound,
                    FLOOR_FACTOR * fl > tol * scale))
    return ok, rep


def fmt(rep):
    """[field: max-norm relative error / relative floor], '*' where the field
    is held to the conditioning floor instead of 1e-12."""
    return " ".join(f"[{q}:{e:.1e}/{fl:.1e}{'*' if c else ''}{'' if ok else ' FAIL'}]"
                    for q, e, fl, ok, c in rep)
