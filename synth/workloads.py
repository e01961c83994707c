"""The named synthetic workloads (shapes, recipes, seeds, schemes).

  box16_sdc       16^3 periodic box, 9 species / 21 reactions, one full
                  right-hand side and one single-rate SDC step (4 Gauss-Lobatto
                  nodes, 6 sweeps).
  box128_mrsdc    128^3, 9/21, 10 multirate SDC steps: advection-diffusion on
                  4 Gauss-Lobatto nodes, chemistry on 5 Gauss-Lobatto nodes in
                  each coarse interval (4 sub-steps per fluid node), 6 sweeps.
  box256_mrsdc    256^3, 21 species / 84 reactions, 5 multirate steps.
  box128_mrsdc_wide   box128_mrsdc with the wide stencil D(a D u) for the
                  second-derivative terms.
  box128_mrsdc_n2ref  box128_mrsdc's flame and scheme with the non-unity
                  Lewis number variant of the 9-species mechanism and N2 as
                  the reference species of the species diffusion.
  batch240_sdc    240 independent boxes with edges drawn from {16..48},
                  9/21, single-rate SDC as box16_sdc.
  box64_adjoint   64^3, 9/21, vector-Jacobian product of the right-hand side.
  box64_sdc_resid 64^3, 9/21, single-rate SDC of up to 12 sweeps per step
                  with the residual early exit (ratio 1.5), 5 steps.
  box128_mrsdc_xwall  box128_mrsdc with physical boundaries at both ends of x
                  (the boundary stencils of Section 2.5) instead of periodic
                  wrap-around.
  box128_mrsdc2   box128_mrsdc's flame with multirate mode 2: the chemistry
                  implicit on 5 Gauss-Lobatto coarse nodes, advection-
                  diffusion on 3 Gauss-Lobatto nodes repeated twice in each
                  coarse interval, 4 sweeps, at a convective CFL number of 2
                  over the step (the node layout and CFL number of the
                  paper's stiff-chemistry jet), 5 steps.
All with dx = 1e-4 m.  The time step of each workload is frozen in the
manifest (tests/golden/manifest/dt.json): cfl min(dx) / max(|u_i| + c) with
cfl = 0.1 unless the workload names another.
"""
import json
import os

import numpy as np

from . import fields

MANIFEST = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "tests", "golden", "manifest")
SIZES = (16, 24, 32, 40, 48)

WORKLOADS = {
    "box16_sdc": dict(shape=(16, 16, 16), dx=1e-4, mech="mech9", recipe="sines", seed=1,
                      scheme=dict(kind="sdc", n_coarse=4, sweeps=6, n_fine=0), steps=1),
    "box128_mrsdc": dict(shape=(128, 128, 128), dx=1e-4, mech="mech9", recipe="turb", seed=2, kmax=16,
                         scheme=dict(kind="mrsdc", n_coarse=4, n_fine=5, fine_repeat=1, sweeps=6), steps=10),
    "box128_mrsdc_wide": dict(shape=(128, 128, 128), dx=1e-4, mech="mech9", recipe="turb", seed=2, kmax=16,
                              scheme=dict(kind="mrsdc", n_coarse=4, n_fine=5, fine_repeat=1, sweeps=6), steps=10,
                              wide=True),
    "box128_mrsdc_n2ref": dict(shape=(128, 128, 128), dx=1e-4, mech="mech9le", recipe="turb", seed=2, kmax=16,
                               scheme=dict(kind="mrsdc", n_coarse=4, n_fine=5, fine_repeat=1, sweeps=6), steps=10,
                               ref_species=8),
    "box256_mrsdc": dict(shape=(256, 256, 256), dx=1e-4, mech="mech21", recipe="turb", seed=3, kmax=32,
                         scheme=dict(kind="mrsdc", n_coarse=4, n_fine=5, fine_repeat=1, sweeps=6), steps=5),
    "batch240_sdc": dict(nbox=240, dx=1e-4, mech="mech9", recipe="sines", seed=1000,
                         scheme=dict(kind="sdc", n_coarse=4, sweeps=6, n_fine=0), steps=1),
    "box64_adjoint": dict(shape=(64, 64, 64), dx=1e-4, mech="mech9", recipe="sines", seed=5,
                          scheme=dict(kind="sdc", n_coarse=4, sweeps=6, n_fine=0), steps=5),
    "box64_sdc_resid": dict(shape=(64, 64, 64), dx=1e-4, mech="mech9", recipe="sines", seed=5,
                            scheme=dict(kind="sdc", n_coarse=4, sweeps=12, n_fine=0), steps=5,
                            residual_ratio=1.5),
    "box128_mrsdc_xwall": dict(shape=(128, 128, 128), dx=1e-4, mech="mech9", recipe="turb", seed=2, kmax=16,
                               scheme=dict(kind="mrsdc", n_coarse=4, n_fine=5, fine_repeat=1, sweeps=6), steps=10,
                               nonperiodic=1),
    "box128_mrsdc2": dict(shape=(128, 128, 128), dx=1e-4, mech="mech9", recipe="turb", seed=2, kmax=16,
                          scheme=dict(kind="mrsdc", n_coarse=5, n_fine=3, fine_repeat=2, sweeps=4, mode=2),
                          steps=5, cfl=2.0),
}


def batch_shapes(seed=1000, nbox=240):
    rng = np.random.default_rng(np.random.SeedSequence([seed, 303]))
    dims = rng.choice(SIZES, size=(nbox, 3))
    return [(int(d[2]), int(d[1]), int(d[0])) for d in dims]   # (nz, ny, nx)


def make_primitives(name, mech, box=None, shape_override=None):
    """Primitive fields of workload `name` (for the batch, of box index `box`;
    with box None, a list over all boxes)."""
    wl = WORKLOADS[name]
    ns = mech["ns"]
    if name == "batch240_sdc":
        shapes = batch_shapes(wl["seed"], wl["nbox"])
        if box is None:
            return [fields.sines(shapes[i], wl["dx"], ns, wl["seed"] + i) for i in range(len(shapes))]
        return fields.sines(shapes[box], wl["dx"], ns, wl["seed"] + box)
    shape = shape_override or wl["shape"]
    if wl["recipe"] == "sines":
        return fields.sines(shape, wl["dx"], ns, wl["seed"])
    return fields.turb(shape, wl["dx"], ns, wl["seed"], kmax=wl["kmax"])


def time_step(name):
    with open(os.path.join(MANIFEST, "dt.json")) as f:
        return float(json.load(f)[name])
