"""Writes the frozen workload manifest under tests/golden/manifest/.

For each synthetic mechanism it selects reactions from the seeded candidate
draws of ``synth.mechanism``: candidates are taken in their seeded order and
each gets up to 60 independent Arrhenius draws; the first draw whose forward
and reverse pseudo-first-order rates k c_tot^(n-1) (c_tot = p/(R T) at 1 atm)
stay below RATE_MAX for every T in [250, 2200] K is kept, so that explicit
forward-Euler sub-steps of the largest time step used with the mechanism are
stable (rate * 2 * DT_MAX <= 0.5).  The rate constants come from the oracle.

It then fixes each workload's time step from the oracle's thermodynamics:
dt = cfl min(dx) / max over cells of (|u|_max + c), c the sound speed of the
initial state, cfl = 0.1 (capped at DT_MAX) unless the workload names its
own (the implicit-chemistry workload: not capped, its chemistry is not
sub-stepped explicitly).

Run:  python tests/golden/make_manifest.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import fields, mechanism  # noqa: E402
from synth.workloads import WORKLOADS, make_primitives  # noqa: E402

RU = 8.31446261815324
DT_MAX = 2.0e-8
RATE_MAX = 0.25 / DT_MAX
T_SCREEN = np.linspace(250.0, 2200.0, 40)
SEEDS = {"mech9": 1309, "mech21": 7327, "mech9le": 1309}
OUT = os.path.join(ROOT, "tests", "golden", "manifest")


def screen(kind, seed):
    nr = mechanism.KIND[kind]["nr"]
    cands, perm = mechanism.candidate_order(kind, seed)
    chosen = []
    for ci in perm:
        ci = int(ci)
        for att in range(60):
            m = mechanism.assemble(kind, seed, [(ci, att)])
            om = oracle.Mechanism(m)
            nf = int(m["nu_f"][0].sum())
            nrv = int(m["nu_r"][0].sum())
            worst = 0.0
            for T in T_SCREEN:
                kf, kr = oracle.rate_constants(om, T)
                c = 101325.0 / (RU * T)
                worst = max(worst, kf[0] * c ** (nf - 1), kr[0] * c ** (nrv - 1))
            if worst <= RATE_MAX:
                chosen.append((ci, att))
                break
        if len(chosen) == nr:
            return chosen
    raise RuntimeError(f"{kind}: only {len(chosen)} of {nr} reactions pass the screen")


def sound_speed_dt(om, prims, dx, cfl=0.1):
    """cfl min(dx) / max(|u_i| + c) over every cell of every box."""
    speed = 0.0
    for prim in prims:
        U = oracle.prim_to_cons(om, prim)
        c = oracle.sound_speed(om, U)
        speed = max(speed, float(np.max(np.abs(prim["u"]).max(axis=0) + c)))
    return cfl * float(np.min(dx)) / speed


def main():
    os.makedirs(OUT, exist_ok=True)
    oracle.build()
    for kind, seed in SEEDS.items():
        chosen = screen(kind, seed)
        with open(os.path.join(OUT, f"{kind}.json"), "w") as f:
            json.dump({"kind": kind, "seed": seed, "rate_max": RATE_MAX, "chosen": chosen}, f, indent=1)
        print(kind, "reactions:", len(chosen))
    dts = {}
    for name, wl in WORKLOADS.items():
        m = mechanism.load(wl["mech"])
        om = oracle.Mechanism(m)
        prims = make_primitives(name, m)
        prims = prims if isinstance(prims, list) else [prims]
        if "cfl" in wl:
            dt = sound_speed_dt(om, prims, wl["dx"], wl["cfl"])
        else:
            dt = min(sound_speed_dt(om, prims, wl["dx"]), DT_MAX)
        dts[name] = dt
        print(name, "dt", dt)
    with open(os.path.join(OUT, "dt.json"), "w") as f:
        json.dump(dts, f, indent=1)


if __name__ == "__main__":
    main()
