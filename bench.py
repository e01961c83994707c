"""Benchmark: multirate SDC steps of the reacting Navier-Stokes right-hand side
on one MI355X (FP64), with the oracle timed on the host cores as a baseline.

Default workload: the largest single-box case, a 256^3 periodic box with 21
species / 84 reactions, turbulent velocity (k^-5/3 on shells 1..32, u_rms
5 m/s) and a planar two-front flame slab, MRSDC mode 1 with
advection-diffusion on 4 Gauss-Lobatto nodes and chemistry on 5
Gauss-Lobatto nodes per coarse interval, 6 sweeps.  One "step" is one MRSDC
time step of the whole box.  The line also carries the 128^3, 9-species
case's figures (same scheme) under "box128_mrsdc".

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                  [--no-cpu-baseline]

Prints one JSON line.  value = SDC steps/s (inputs resident in HBM) over the
timed region of exactly K steps; the line also carries Mcell
advection-diffusion and reaction evaluations per second, the roofline of the
dominant kernel and of the three stencil direction passes together (average
durations from HIP events recorded on the launch stream around every launch
of the timed region), the same K steps timed five more times with no
events attached (their per-step median: unprofiled_ms_per_step), and the
oracle baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz

# Algorithmic work per cell of each kernel kind (flops, HBM bytes), from the
# operation counts of the method (not of the implementation); an exponential
# or logarithm counts 25 flops.
def work_model(ns, nr, n_coarse, n_fine_per_interval, fused=False):
    nu = 5 + ns
    # primitive fields per cell: u, T, p, mu, lambda, rho D, the mean molecular
    # weight and Y (the mole fractions follow from Y and the mean molecular
    # weight, the species enthalpies from T)
    np_ = 9 + ns
    # one direction of the stencil pass: convective divergence, narrow row sums
    # shared per field and face pairs, first derivatives of the mixed and
    # correction-velocity terms
    narrow = (7 + ns) * 96 + (7 + 3 * ns) * 16
    first = 11 * (36 + 12 * ns) / 3.0
    dir_flops = narrow + first
    dir_bytes = 8 * (nu + np_ + 4 + 2 * nu)            # read U, P, 4 gradients; read+write dU/dt
    chem_flops = 32 * ns + 75 * nr
    # temperature from e: the mixture's six NASA coefficients (12 ns flops),
    # then three Newton iterations of a quintic, its derivative and the update
    newton = 12 * ns + 3 * 21
    r = n_fine_per_interval
    n1 = n_coarse
    # fine sub-sweep of one coarse interval: r chemistry sub-steps per cell
    # (Newton, rates, update with the precomputed increments) ...
    step_flops = r * (chem_flops + newton + 2 * nu)
    step_bytes = 8 * (2 * nu + r * nu + r * ns)
    # ... and the quadrature increments S21 F1 + S22 F2 of those sub-steps
    src_flops = r * (nu * (2 * n1 + 3) + ns * 2 * 6)
    src_bytes = 8 * (nu * (n1 + 1) + ns * (r + 1) + r * nu)
    if fused:
        # both in one kernel: the increments never reach HBM; read U, the
        # interval's f1 and f2 node values, write U and the new f2 values
        step_flops += src_flops
        step_bytes = 8 * (2 * nu + nu * (n1 + 1) + ns * (r + 1) + r * ns)
    # in evaluations without the chemistry (the multirate coarse component)
    # the x pass stores dU/dt without reading it first
    dir_x_bytes = dir_bytes - (8 * nu if r else 0)
    # multirate mode 2, implicit chemistry of one coarse interval per cell:
    # the interval's forcing (read U, f1 at the n1 coarse nodes, f2 at the
    # r + 1 fine nodes of the interval; write the new f1), then Newton's
    # method: per iteration the rates and their Jacobian (the chemistry, 16
    # sparse updates per reaction, the dense temperature column) and an LU
    # solve; counted as 3 iterations and the final rate evaluation
    nr_ = nr
    jac = chem_flops + newton + 32 * nr_ + 3 * ns * ns + (2 * ns ** 3) // 3 + 2 * ns * ns
    imp_flops = (n_coarse + r + 1) * nu * 2 + 4 * jac
    imp_bytes = 8 * (nu + n_coarse * ns + (r + 1) * nu + ns)
    return {
        "dir_x": (dir_flops, dir_x_bytes), "dir_y": (dir_flops, dir_bytes), "dir_z": (dir_flops, dir_bytes),
        "mr_fine": (step_flops, step_bytes), "mr_src": (src_flops, src_bytes),
        "prims": (newton + 40 * ns, 8 * (nu + np_)),
        "mr2_imp": (imp_flops, imp_bytes),
    }


def stored_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from committed rocprofv3 counter runs,
    if they were taken on the current kernel sources."""
    from paper_1309_7327_amd.rocpd_summary import source_hash
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(workload, mech, n_cells_full):
    """The oracle (plain C++ right-hand side + NumPy SDC driver) on a bounded
    sample: one step of the same scheme on a 64^3 box of the same recipe,
    scaled by cell count to the full box."""
    import oracle
    from oracle import sdc as osdc
    from synth.workloads import WORKLOADS, make_primitives, time_step
    wl = WORKLOADS[workload]
    om = oracle.Mechanism(mech, ref_species=wl.get("ref_species", -1), wide=wl.get("wide", False),
                          nonperiodic=wl.get("nonperiodic", 0))
    # about 10-30 s of host work: a 64^3 box with 9 species, 48^3 with 21,
    # 24^3 for the implicit-chemistry scheme (its Newton solves take the
    # oracle's tangent products)
    sch = wl["scheme"]
    edge = 24 if sch.get("mode", 1) == 2 else (64 if mech["ns"] <= 9 else 48)
    prim = make_primitives(workload, mech, shape_override=(edge,) * 3)
    U0 = oracle.prim_to_cons(om, prim)
    dt = time_step(workload)
    sch = wl["scheme"]
    dx = wl["dx"]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    if sch["kind"] == "sdc":
        f = lambda U, t: oracle.rhs(om, U, dx, nthreads=threads)
        osdc.sdc_run(f, U0, 0.0, dt, osdc.gauss_lobatto(sch["n_coarse"]), sch["sweeps"], 1,
                     residual_ratio=wl.get("residual_ratio", 0.0))
    elif sch.get("mode", 1) == 2:
        from oracle import implicit as OI
        f1 = lambda U, t: oracle.rhs(om, U, dx, parts=oracle.REACT, nthreads=threads)
        f2 = lambda U, t: oracle.rhs(om, U, dx, parts=oracle.AD, nthreads=threads)
        solve1 = lambda rhs, h: OI.implicit_reaction(om, rhs, h, dx, nthreads=threads)
        t1, t2, pieces = osdc.mr_nodes(sch["n_coarse"], sch["n_fine"], sch["fine_repeat"])
        osdc.mrsdc2_run(f1, solve1, f2, U0, 0.0, dt, t1, t2, pieces, sch["sweeps"], 1)
    else:
        f1 = lambda U, t: oracle.rhs(om, U, dx, parts=oracle.AD, nthreads=threads)
        f2 = lambda U, t: oracle.rhs(om, U, dx, parts=oracle.REACT, nthreads=threads)
        t1, t2, pieces = osdc.mr_nodes(sch["n_coarse"], sch["n_fine"], sch["fine_repeat"])
        osdc.mrsdc_run(f1, f2, U0, 0.0, dt, t1, t2, pieces, sch["sweeps"], 1)
    el = time.perf_counter() - t0
    return {"value": (edge ** 3 / n_cells_full) / el, "unit": "SDC steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"one step of the same scheme on a {edge}^3 box of the same recipe "
                      f"({el:.1f} s), scaled by cell count to {round(n_cells_full ** (1 / 3))}^3"}


def bench_adjoint(args):
    """The adjoint workload: vector-Jacobian product of the right-hand side
    and the adjoint of 5 single-rate SDC steps on a 64^3 box, each timed
    against its forward counterpart."""
    import numpy as np
    import torch
    from paper_1309_7327_amd import narrowsdc as N
    from synth import mechanism
    from synth.workloads import WORKLOADS, make_primitives, time_step

    wl = WORKLOADS[args.workload]
    mech = mechanism.load(wl["mech"])
    ns, nr = mech["ns"], mech["nr"]
    nU = 5 + ns
    nz, ny, nx = wl["shape"]
    ncell = nx * ny * nz
    dt = time_step(args.workload)
    sd = wl["scheme"]
    nsteps = wl["steps"]
    sch = N.scheme(sd["n_coarse"], sd["sweeps"], 0, 1)
    torch.cuda.set_device(0)
    ctx = N.Context(0)
    ctx.set_mechanism(mech)
    prim = make_primitives(args.workload, mech)
    bx = N.box(nx, ny, nz, wl["dx"])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    U = torch.zeros(N.ghosted_shape(nU, nz, ny, nx), dtype=torch.float64, device="cuda")
    ctx.prim_to_cons(bx, dev(prim["p"]), dev(prim["T"]), dev(prim["Y"]), dev(prim["u"]), U)
    g = torch.Generator(device="cuda").manual_seed(5001)
    vbar = torch.randn((nU, nz, ny, nx), dtype=torch.float64, device="cuda", generator=g)
    F = torch.empty_like(vbar)
    Ub = torch.zeros_like(vbar)
    lA = torch.zeros(nr, dtype=torch.float64, device="cuda")
    h = torch.cuda.current_stream().cuda_stream
    reps = max(args.steps, 1)

    def timed(fn, n):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    t_rhs = timed(lambda: ctx.rhs_eval(bx, U, F, N.RHS_ALL), reps)
    t_vjp = timed(lambda: ctx.rhs_vjp(bx, U, vbar, Ub, lA, N.RHS_ALL), reps)
    ws, nb = N.workspace(ctx, [bx], sch)
    U0 = U.clone()
    t_fwd = timed(lambda: (U.copy_(U0), ctx.sdc_step(bx, U, dt, nsteps, sch, ws, nb)), 2)
    nbv = ctx.vjp_workspace_size(bx, sch, nsteps)
    wsv = torch.empty(nbv // 8 + 1, dtype=torch.float64, device="cuda")
    U0b = torch.empty_like(vbar)
    t_adj = timed(lambda: ctx.sdc_step_vjp(bx, U0, dt, nsteps, sch, vbar, U0b, lA, wsv, nbv), 2)
    ctx.check_status()
    # per-kernel durations of one product (HIP events on the launch stream)
    ctx.profile(True)
    ctx.rhs_vjp(bx, U, vbar, Ub, lA, N.RHS_ALL)
    kern = ctx.profile_read(h)
    ctx.profile(False)
    ctx.check_status()
    np_ = 8 + 3 * ns
    # one direction adjoint call (coefficient, gather passes) covers every
    # cell; per cell it reads the state, the primitive and gradient lines
    # and the cotangent, and updates the three adjoint accumulators
    by_cell = 8 * (2 * nU + np_ + 4) + 16 * (nU + np_ + 4)
    dirk = [k for k in kern if k.startswith("dir_adj")]
    dominant = max(dirk, key=lambda k: kern[k][0])
    dur_ms = kern[dominant][0] / kern[dominant][1]
    ach = by_cell * ncell / (dur_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": stored_traffic(dominant, args.workload), "kernel": dominant, "avg_launch_ms": dur_ms}
    out = {
        "metric": "SDC adjoint steps/s (5 steps, checkpointed) and VJP time / RHS time (FP64, 1 MI355X)",
        "value": nsteps / t_adj, "unit": "SDC adjoint steps/s", "n_gpus": 1, "steps": reps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_adj / nsteps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "cells": ncell, "species": ns, "reactions": nr, "scheme": sd,
                   "steps": nsteps, "dt": dt},
        "rhs_ms": 1e3 * t_rhs, "vjp_ms": 1e3 * t_vjp, "vjp_over_rhs": t_vjp / t_rhs,
        "forward_steps_ms": 1e3 * t_fwd, "adjoint_steps_ms": 1e3 * t_adj, "adjoint_over_forward": t_adj / t_fwd,
        "kernels_ms": {k: round(v[0], 4) for k, v in kern.items()}, "roofline": roof,
        "hbm_copy_gbs": args.copy_gbs,
    }
    if not args.no_cpu_baseline:
        import oracle
        from oracle import adjoint as OA
        om = oracle.Mechanism(mech)
        Uo = oracle.prim_to_cons(om, prim)
        v = vbar.cpu().numpy()
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cells = np.array([[5, 6, 7], [30, 31, 32]])
        t0 = time.perf_counter()
        OA.rhs_vjp(om, Uo, wl["dx"], v, cells=cells, nthreads=threads)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": len(cells) / el / ncell, "unit": "rhs VJP/s", "cores": threads, "kind": "oracle",
            "sample": f"the oracle's definition of (d rhs/dU)^T v at {len(cells)} input cells of the "
                      f"{nx}^3 box ({el:.1f} s), scaled by cell count to one whole-box product; "
                      f"the library: {1.0 / t_vjp:.1f} VJP/s"}
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """Batched boxes: the whole batch advanced by one launch per stage (HIP
    graph replay, autotuned tile shapes) versus a loop of per-box calls."""
    import numpy as np
    import torch
    from paper_1309_7327_amd import narrowsdc as N
    from synth import fields, mechanism
    from synth.workloads import WORKLOADS, batch_shapes, time_step

    wl = WORKLOADS[args.workload]
    mech = mechanism.load(wl["mech"])
    ns = mech["ns"]
    shapes = batch_shapes(wl["seed"], wl["nbox"])
    dt = time_step(args.workload)
    sd = wl["scheme"]
    sch = N.scheme(sd["n_coarse"], sd["sweeps"], sd["n_fine"], sd.get("fine_repeat", 1))
    torch.cuda.set_device(0)
    ctx = N.Context(0)
    ctx.set_mechanism(mech)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    boxes, Us = [], []
    for i, shp in enumerate(shapes):
        prim = fields.sines(shp, wl["dx"], ns, wl["seed"] + i)
        bx = N.box(shp[2], shp[1], shp[0], wl["dx"])
        U = torch.zeros(N.ghosted_shape(5 + ns, *shp), dtype=torch.float64, device="cuda")
        ctx.prim_to_cons(bx, dev(prim["p"]), dev(prim["T"]), dev(prim["Y"]), dev(prim["u"]), U)
        boxes.append(bx)
        Us.append(U)
    ncell = sum(int(np.prod(s)) for s in shapes)
    ws, nb = N.workspace(ctx, boxes, sch)
    stream = torch.cuda.Stream()
    h = stream.cuda_stream
    choice = ctx.autotune(boxes, Us, ws, nb, stream=h)
    ctx.set_graph(True)
    if args.warmup > 0:
        ctx.sdc_step_batched(boxes, Us, dt, 1, sch, ws, nb, stream=h)   # captures the graph
    ctx.check_status(h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.sdc_step_batched(boxes, Us, dt, 1, sch, ws, nb, stream=h)
    stream.synchronize()
    t1 = time.perf_counter()
    ctx.check_status(h)
    ctx.set_graph(False)
    batched = args.steps / (t1 - t0)
    # per-box launch loop on the same stream
    nb1 = max(ctx.workspace_size([b], sch) for b in boxes)
    ws1 = torch.empty(nb1 // 8 + 1, dtype=torch.float64, device="cuda")
    for bx, U in zip(boxes, Us):
        ctx.sdc_step(bx, U, dt, 1, sch, ws1, nb1, stream=h)
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for bx, U in zip(boxes, Us):
            ctx.sdc_step(bx, U, dt, 1, sch, ws1, nb1, stream=h)
    stream.synchronize()
    t1 = time.perf_counter()
    loop = args.steps / (t1 - t0)
    # per-kernel durations of one batched step (HIP events on the launch stream)
    ctx.profile(True)
    ctx.sdc_step_batched(boxes, Us, dt, 1, sch, ws, nb, stream=h)
    kern = ctx.profile_read(h)
    ctx.profile(False)
    ctx.check_status(h)
    model = work_model(ns, mech["nr"], sd["n_coarse"], 0)
    dominant = max(kern, key=lambda k: kern[k][0])
    dur_ms = kern[dominant][0] / kern[dominant][1]
    roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None}
    if dominant in model:
        fl, by = model[dominant]
        roof = {"bound": "hbm", "achieved": by * ncell / (dur_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["fp64_tflops"] = fl * ncell / (dur_ms * 1e-3) / 1e12
    roof.update(kernel=dominant, avg_launch_ms=dur_ms, traffic=stored_traffic(dominant, args.workload))
    out = {
        "metric": "Mcell-RHS evals/s + SDC steps/s (FP64, 1 MI355X); achieved HBM GB/s vs peak",
        "value": batched, "unit": "SDC steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 / batched, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "boxes": len(boxes), "cells": ncell, "species": ns,
                   "scheme": sd, "dt": dt, "tile": list(choice)},
        "per_box_loop_steps_per_s": loop, "batched_over_loop": batched / loop,
        "mcell_rhs_evals_per_s": ncell * sd["sweeps"] * (sd["n_coarse"] - 1) * batched / 1e6,
        "kernels_ms": {k: round(v[0], 4) for k, v in kern.items()}, "roofline": roof,
        "hbm_copy_gbs": args.copy_gbs,
    }
    print(json.dumps(out), flush=True)


def copy_ceiling(torch, reps=5):
    """The practical HBM ceiling beside the 8 TB/s specification: bytes read
    plus written per second by a 1 GiB device-to-device tensor copy (best of
    `reps`, HIP events)."""
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * (1 << 30) / (best * 1e-3) / 1e9


def roofline_of(model, name, dur_ms, units):
    """Roofline entry of kernel kind `name` from its per-unit work model and
    average launch duration: "hbm" below the ridge, else "alu"."""
    fl, by = model[name]
    flops, bytes_ = fl * units, by * units
    if flops / bytes_ * HBM_PEAK_GBS * 1e9 < FP64_PEAK_TFLOPS * 1e12:
        roof = {"bound": "hbm", "achieved": bytes_ / (dur_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": flops / (dur_ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["fp64_tflops"] = flops / (dur_ms * 1e-3) / 1e12
    roof["hbm_gbs"] = bytes_ / (dur_ms * 1e-3) / 1e9
    return roof


def run_box(args, workload, steps, warmup, with_baseline):
    """Warm-up, then exactly `steps` SDC steps of one box timed with HIP
    events around every launch, then the same number of steps again with no
    events attached.  Returns the result fields of the JSON line."""
    import ctypes

    import numpy as np
    import torch
    from paper_1309_7327_amd import narrowsdc as N
    from synth import mechanism
    from synth.workloads import WORKLOADS, make_primitives, time_step

    wl = WORKLOADS[workload]
    mech = mechanism.load(wl["mech"])
    ns = mech["ns"]
    nz, ny, nx = wl["shape"]
    ncell = nx * ny * nz
    dx = wl["dx"]
    dt = time_step(workload)
    sch_d = wl["scheme"]
    if sch_d["kind"] == "sdc":
        sch = N.scheme(sch_d["n_coarse"], sch_d["sweeps"], 0, 1)
        r = 0
    else:
        sch = N.scheme(sch_d["n_coarse"], sch_d["sweeps"], sch_d["n_fine"], sch_d["fine_repeat"],
                       mode=sch_d.get("mode", 1))
        r = (sch_d["n_fine"] - 1) * sch_d["fine_repeat"]
    mode2 = sch_d.get("mode", 1) == 2

    ctx = N.Context(0)
    ctx.set_mechanism(mech)
    ctx.set_reference_species(wl.get("ref_species", -1))
    ctx.set_residual_exit(wl.get("residual_ratio", 0.0))
    ctx.set_wide_stencil(wl.get("wide", False))
    prim = make_primitives(workload, mech)
    bx = N.box(nx, ny, nz, dx, nonperiodic=wl.get("nonperiodic", 0))
    U = torch.zeros(N.ghosted_shape(5 + ns, nz, ny, nx), dtype=torch.float64, device="cuda")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    ctx.prim_to_cons(bx, dev(prim["p"]), dev(prim["T"]), dev(prim["Y"]), dev(prim["u"]), U)
    del prim
    ws, nb = N.workspace(ctx, [bx], sch)
    stream = torch.cuda.current_stream()

    if warmup > 0:
        ctx.sdc_step(bx, U, dt, warmup, sch, ws, nb)
    ctx.check_status()
    torch.cuda.synchronize()

    # timed region: exactly `steps` steps, per-launch HIP events on the
    # launch stream (their durations give the roofline entries)
    lib = N._lib
    lib.sdc_profile_enable(ctx.h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.sdc_step(bx, U, dt, steps, sch, ws, nb)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check_status()
    _, sweeps_done = ctx.residual_history()
    tot = (ctypes.c_double * 32)()
    cnt = (ctypes.c_int * 32)()
    nk = lib.sdc_profile_read(ctx.h, ctypes.c_void_p(stream.cuda_stream), tot, cnt)
    kern = {lib.sdc_kernel_name(i).decode(): (tot[i], cnt[i]) for i in range(nk) if cnt[i] > 0}
    lib.sdc_profile_enable(ctx.h, 0)
    # the same number of steps with no events attached, three times (their
    # median per step beside the timed region's figure)
    reps = []
    for _ in range(5):
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        ctx.sdc_step(bx, U, dt, steps, sch, ws, nb)
        torch.cuda.synchronize()
        reps.append(1e3 * (time.perf_counter() - t2) / steps)
    ctx.check_status()

    el = t1 - t0
    steps_per_s = steps / el
    M1 = sch_d["n_coarse"] - 1
    # with the residual early exit the sweeps taken replace K per step
    n_ad = (sweeps_done if wl.get("residual_ratio") else steps * sch_d["sweeps"]) * M1
    n_r = n_ad * r if r else n_ad
    if mode2:
        # mode 2: advection-diffusion on the fine nodes, one implicit
        # chemistry solve per coarse interval
        n_ad, n_r = n_ad * r, n_ad
    # the one-kernel fine sub-steps run for four coarse nodes, four fine
    # sub-steps per interval (above nine species on paired lanes)
    fused = sch_d["n_coarse"] == 4 and r == 4 and not mode2
    model = work_model(ns, mech["nr"], sch_d["n_coarse"], r, fused)
    dominant = max(kern, key=lambda k: kern[k][0])
    dur_ms = kern[dominant][0] / kern[dominant][1]
    if dominant in model:
        roof = roofline_of(model, dominant, dur_ms, ncell)
    else:
        roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None}
    roof["kernel"] = dominant
    roof["avg_launch_ms"] = dur_ms
    roof["traffic"] = stored_traffic(dominant, workload)
    # the stencil pass: the three direction kernels of one advection-diffusion
    # evaluation together
    stencil = None
    if all(k in kern for k in ("dir_x", "dir_y", "dir_z")):
        dms = sum(kern[k][0] / kern[k][1] for k in ("dir_x", "dir_y", "dir_z"))
        sfl = sum(model[k][0] for k in ("dir_x", "dir_y", "dir_z"))
        sby = sum(model[k][1] for k in ("dir_x", "dir_y", "dir_z"))
        stencil = {"kernels": "dir_x+dir_y+dir_z", "ms_per_evaluation": dms,
                   "fp64_tflops": sfl * ncell / (dms * 1e-3) / 1e12,
                   "hbm_gbs": sby * ncell / (dms * 1e-3) / 1e9}
        stencil["bound"] = "alu" if sfl / sby * HBM_PEAK_GBS * 1e9 >= FP64_PEAK_TFLOPS * 1e12 else "hbm"
        stencil["frac"] = (stencil["fp64_tflops"] / FP64_PEAK_TFLOPS if stencil["bound"] == "alu"
                           else stencil["hbm_gbs"] / HBM_PEAK_GBS)
    out = {
        "value": steps_per_s,
        "ms_per_step": 1e3 * el / steps,
        "unprofiled_ms_per_step": float(np.median(reps)),
        "unprofiled_ms_per_step_repeats": [round(v, 4) for v in reps],
        "config": {"workload": workload, "cells": ncell, "species": ns, "reactions": int(mech["nr"]),
                   "scheme": sch_d, "dt": dt,
                   "second_derivatives": "wide stencil D(a D u)" if wl.get("wide") else "narrow stencil",
                   "species_diffusion":
                   ("reference species %d" % wl["ref_species"]) if wl.get("ref_species", -1) >= 0
                   else "correction velocity",
                   "boundaries": "physical along " + "".join(a for d, a in enumerate("xyz")
                                                             if (wl.get("nonperiodic", 0) >> d) & 1)
                   if wl.get("nonperiodic", 0) else "periodic"},
        "mcell_ad_evals_per_s": ncell * n_ad / el / 1e6,
        ("mcell_implicit_chem_solves_per_s" if mode2 else "mcell_r_evals_per_s"): ncell * n_r / el / 1e6,
        "kernels_ms": {k: round(v[0], 4) for k, v in kern.items()},
        "roofline": roof,
        "stencil_roofline": stencil,
    }
    if wl.get("residual_ratio"):
        out["sweeps_per_step"] = sweeps_done / steps
    ctx.close()
    del U, ws
    torch.cuda.empty_cache()
    if with_baseline:
        out["cpu_baseline"] = cpu_baseline(workload, mech, ncell)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="box256_mrsdc")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 128^3 figures carried beside the default workload's")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X and has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1309_7327_amd import narrowsdc as N  # noqa: F401  (fails loudly if unbuilt)
    from synth.workloads import WORKLOADS

    wl = WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    args.copy_gbs = copy_ceiling(torch)
    if args.calibrate_copy:
        # 1 GiB device-to-device copy: the reference for the HBM byte counters
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if "nbox" in wl:
        return bench_batch(args)
    if args.workload == "box64_adjoint":
        return bench_adjoint(args)
    res = run_box(args, args.workload, args.steps, args.warmup, not args.no_cpu_baseline)
    out = {
        "metric": "Mcell-RHS evals/s + SDC steps/s (FP64, 1 MI355X); achieved HBM GB/s vs peak",
        "value": res.pop("value"),
        "unit": "SDC steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": res.pop("config"),
    }
    out.update(res)
    out["hbm_copy_gbs"] = args.copy_gbs
    if args.workload == "box256_mrsdc" and not args.no_extra:
        # the 128^3, 9-species case of the same scheme, as extra keys
        ex = run_box(args, "box128_mrsdc", 10, 1, False)
        out["box128_mrsdc"] = {k: ex[k] for k in ("value", "ms_per_step", "unprofiled_ms_per_step",
                                                  "mcell_ad_evals_per_s", "mcell_r_evals_per_s",
                                                  "kernels_ms", "roofline", "stencil_roofline")}
        out["box128_mrsdc"]["unit"] = "SDC steps/s"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
