"""The GPU parity criterion's noise-floor factor (tests/gpu_util.py), pinned
on the CPU with the oracle alone.

The criterion accepts 4 floor_q where the FP64 problem is worse conditioned
than 1e-12, floor_q being the oracle's response to one random one-ulp input
perturbation (one seed).  The factor rests on two facts checked here:
  * floor_q is a sample of a random maximum; over seeds it varies by at most
    2.8x in the fields where it sets the bound, so sqrt(2) * 2.8 <= 4 covers the difference of two independent
    roundings (the HIP path's and the oracle's);
  * only the momentum right-hand sides are conditioned worse than 1e-12
    (4 floor_q > 1e-12 max|f|); every other field is held to 1e-12."""
import numpy as np
import pytest

import oracle
from synth import fields, mechanism

SEEDS = list(range(12)) + [12345]


@pytest.mark.parametrize("kind,shape,dx", [("mech9", (8, 10, 12), 1e-4), ("mech9", (16, 16, 16), 1e-4),
                                           ("mech9le", (5, 6, 7), (1e-4, 1.2e-4, 0.9e-4))])
def test_noise_floor_spread_and_conditioned_fields(kind, shape, dx):
    m = mechanism.load(kind)
    om = oracle.Mechanism(m)
    prim = fields.sines(shape, dx, m["ns"], 21)
    U = oracle.prim_to_cons(om, prim)
    f0 = oracle.rhs(om, U, dx)
    nq = f0.shape[0]
    scale = np.abs(f0).reshape(nq, -1).max(axis=1)
    fl = []
    for seed in SEEDS:
        rng = np.random.default_rng(seed)
        f1 = oracle.rhs(om, U * (1.0 + 2.0 ** -52 * rng.standard_normal(U.shape)), dx)
        fl.append(np.abs(f1 - f0).reshape(nq, -1).max(axis=1))
    fl = np.array(fl)
    spread = fl.max(axis=0) / fl.min(axis=0)
    print("floor spread per field", np.array2string(spread, precision=2))
    print("relative floor (seed 12345)", np.array2string(fl[-1] / scale, precision=1))
    limited = 4.0 * fl.max(axis=0) > 1e-12 * scale
    assert list(np.nonzero(limited)[0]) == [1, 2, 3]
    # the spread matters only where the floor sets the bound
    assert np.all(spread[limited] <= 2.8)
    assert np.sqrt(2.0) * 2.8 <= 4.0
