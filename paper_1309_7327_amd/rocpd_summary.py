"""Summaries of rocprofv3 result databases (rocpd SQLite files) as the short
text records kept under profiles/.

  python -m paper_1309_7327_amd.rocpd_summary kernels DB --title TEXT --command CMD
      per-kernel calls / total / average duration (markdown, stdout)
  python -m paper_1309_7327_amd.rocpd_summary fp64 DB --title TEXT --command CMD
      per-kernel FP64 VALU instruction counts (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64,
      one run) and the FP64 rate they give over the dispatch durations of
      the same run, against the 78.6 TFLOP/s vector peak (markdown, stdout)
  python -m paper_1309_7327_amd.rocpd_summary traffic --fetch DB --write DB --workload NAME
        --out-dir DIR --command-fetch CMD --command-write CMD
      HBM bytes per launch of every library kernel from a FETCH_SIZE run and
      a WRITE_SIZE run (KiB per dispatch), each scaled by what the same
      counter reads for the 1 GiB device-to-device copy that
      `bench.py --calibrate-copy` issues first; writes
      traffic_<kernel>_<workload>.json per kernel kind and
      traffic_<workload>.md, stamped with the hash of the kernel sources.
  python -m paper_1309_7327_amd.rocpd_summary sq PASS1_DB PASS2_DB TRACE_DB --title TEXT --command CMD ...
      per-kernel SQ counters from two counter runs (the SQ_SET_1 and
      SQ_SET_2 lists below) and a kernel trace of the same command:
      instructions per wave, VALU busy share, share of wave time waiting,
      waves per SIMD, vector-memory and LDS instructions per wave, LDS bank
      conflicts per LDS active cycle (markdown, stdout)
"""
import argparse
import collections
import hashlib
import json
import os
import re
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ("kernels.hip", "adjoint.hip", "physics.h", "api.cpp", "nsdc_internal.h", "launch.h")
CALIB_BYTES = 1 << 30

_KINDS = [
    (r"k_prim_to_cons<", "prim_to_cons"), (r"k_ghost<", "ghost"), (r"k_prims<", "prims"),
    (r"k_vgrad<", "vgrad"), (r"k_dir<\d+, 0", "dir_x"), (r"k_dir<\d+, 1", "dir_y"), (r"k_dir<\d+, 2", "dir_z"),
    (r"k_chem<", "chem"), (r"k_sdc_node<", "sdc_node"), (r"k_mr_step<", "mr_fine"), (r"k_mr_fused<", "mr_fine"), (r"k_mr_pair<", "mr_fine"), (r"k_mr_pair_fused<", "mr_fine"),
    (r"k_mr_src<", "mr_src"), (r"k_mr2_imp<", "mr2_imp"), (r"k_mr2_node<", "sdc_node"),
    (r"k_adj_(coef|g1|g2|g3)<\d+, 0", "dir_adj_x"), (r"k_adj_(coef|g1|g2|g3)<\d+, 1", "dir_adj_y"),
    (r"k_adj_(coef|g1|g2|g3)<\d+, 2", "dir_adj_z"),
    (r"k_chem_adj<", "chem_adj"), (r"k_vgrad_adj<", "vgrad_adj"), (r"k_prims_adj<", "prims_adj"),
    (r"k_fold<", "fold"), (r"k_(fill0|axpy_multi|lincomb|lnA_reduce)\b", "adj_linalg"),
]


def source_hash():
    """Hash of the kernel and driver sources (a traffic record is valid only
    for the sources it was measured on)."""
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name):
    """Kernel name with its template arguments, without the parameter list."""
    m = re.search(r"nsdc::(k_\w+(?:<[^>]*>)?)", name)
    return m.group(1) if m else name[:60]


def kind_of(name):
    short = short_name(name)
    for pat, kind in _KINDS:
        if re.match(pat, short):
            return kind
    return None


def kernel_table(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration from kernels").fetchall()
    agg = collections.OrderedDict()
    for name, dur in rows:
        a = agg.setdefault(short_name(name), [0, 0.0])
        a[0] += 1
        a[1] += dur
    tot = sum(v[1] for v in agg.values()) or 1.0
    return sorted(((k, n, t, t / n, 100.0 * t / tot) for k, (n, t) in agg.items()), key=lambda r: -r[2])


def counters(db, counter):
    """{kernel kind or short name: [values per dispatch]} for one counter."""
    con = sqlite3.connect(db)
    out = collections.defaultdict(list)
    for name, cname, val in con.execute("select kernel_name, counter_name, value from counters_collection"):
        if cname == counter:
            out[name].append(val)
    return out


FP64_COUNTERS = ("SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                 "SQ_INSTS_VALU_TRANS_F64")
FP64_PEAK = 78.6e12


def fp64_table(db):
    """Per kernel: dispatches, mean duration (ns), mean wave instruction count
    per FP64 counter, and FLOP/s = 64 lanes x (ADD + MUL + 2 FMA + TRANS)
    per dispatch / duration (every lane of a wave counted active)."""
    con = sqlite3.connect(db)
    acc = collections.OrderedDict()
    for name, cname, val, t0, t1, did in con.execute(
            "select kernel_name, counter_name, value, start, end, dispatch_id from counters_collection"):
        if cname not in FP64_COUNTERS:
            continue
        a = acc.setdefault(short_name(name), {"disp": {}, "cnt": collections.defaultdict(float)})
        a["disp"][did] = t1 - t0
        a["cnt"][cname] += val
    rows = []
    for k, a in acc.items():
        n = len(a["disp"])
        dur = sum(a["disp"].values()) / n
        c = {cn: a["cnt"][cn] / n for cn in FP64_COUNTERS}
        fl = 64.0 * (c[FP64_COUNTERS[0]] + c[FP64_COUNTERS[1]] + 2.0 * c[FP64_COUNTERS[2]] + c[FP64_COUNTERS[3]])
        rows.append((k, n, dur, c, fl, fl / (dur * 1e-9) if dur > 0 else 0.0))
    return sorted(rows, key=lambda r: -r[2] * r[1])


SQ_SET_1 = ("SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
            "SQ_WAIT_ANY", "SQ_INSTS_VALU", "SQ_INSTS_LDS")
SQ_SET_2 = ("SQ_INSTS_SALU", "SQ_INSTS_SMEM", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_WAVES",
            "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_ANY", "SQ_INST_CYCLES_VMEM_RD")
CLOCK_HZ = 2.4e9
SIMDS = 1024


def counter_means(db):
    """{short kernel name: {counter: mean over dispatches of the per-dispatch total}}."""
    con = sqlite3.connect(db)
    acc = collections.defaultdict(lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    for name, cname, val, did in con.execute(
            "select kernel_name, counter_name, value, dispatch_id from counters_collection"):
        acc[short_name(name)][cname][did] += val
    return {k: {c: sum(d.values()) / len(d) for c, d in cs.items()} for k, cs in acc.items()}


def sq_table(db1, db2, trace_db):
    """Rows (kernel, avg ms, waves, VALU instr / wave, VALU busy, waiting,
    waves per SIMD, VMEM rd instr / wave, LDS instr / wave, bank conflicts /
    LDS active cycles), ordered by total trace time.  VALU busy counts every
    VALU instruction at the 4-cycle FP64 rate (a lower bound); waiting is
    SQ_WAIT_ANY / SQ_WAVE_CYCLES; waves per SIMD is SQ_WAVE_CYCLES x 4 over
    the dispatch's SIMD-cycles."""
    c1, c2 = counter_means(db1), counter_means(db2)
    rows = []
    for name, n, tot, avg, pct in kernel_table(trace_db):
        a, b = c1.get(name), c2.get(name)
        if not a or not b or not b.get("SQ_WAVES"):
            continue
        dur = avg * 1e-9
        waves = b["SQ_WAVES"]
        simd_cycles = dur * CLOCK_HZ * SIMDS
        lds_act = a.get("SQ_ACTIVE_INST_LDS", 0.0)
        rows.append((name, avg * 1e-6, waves, a["SQ_INSTS_VALU"] / waves,
                     a["SQ_INSTS_VALU"] * 4.0 / simd_cycles, a["SQ_WAIT_ANY"] / a["SQ_WAVE_CYCLES"],
                     a["SQ_WAVE_CYCLES"] * 4.0 / simd_cycles, b["SQ_INSTS_VMEM_RD"] / waves,
                     a["SQ_INSTS_LDS"] / waves, b["SQ_LDS_BANK_CONFLICT"] / lds_act if lds_act else 0.0))
    return rows


def traffic(fetch_db, write_db, workload, out_dir, cmd_fetch, cmd_write):
    f = counters(fetch_db, "FETCH_SIZE")
    w = counters(write_db, "WRITE_SIZE")
    copy_f = max(v for k, vs in f.items() if "copyBuffer" in k for v in vs)
    copy_w = max(v for k, vs in w.items() if "copyBuffer" in k for v in vs)
    ff = CALIB_BYTES / (copy_f * 1024.0)
    fw = CALIB_BYTES / (copy_w * 1024.0)
    # a kind may span several kernels (the direction adjoint launches four
    # per call): its bytes per call are the sum of their per-launch means
    by_kind = collections.defaultdict(lambda: collections.defaultdict(lambda: [[], []]))
    for k, vs in f.items():
        if kind_of(k):
            by_kind[kind_of(k)][short_name(k)][0].extend(vs)
    for k, vs in w.items():
        if kind_of(k):
            by_kind[kind_of(k)][short_name(k)][1].extend(vs)
    h = source_hash()
    lines = [f"# HBM traffic per launch: {workload}", "",
             "Commands (from the repository root; `cd /tmp && export TMPDIR=/tmp` before rocprofv3):", "",
             "```", cmd_fetch, cmd_write,
             f"python -m paper_1309_7327_amd.rocpd_summary traffic --fetch <fetch db> --write <write db> "
             f"--workload {workload} --out-dir profiles", "```", "",
             f"Calibration: the 1 GiB device-to-device copy reads {copy_f:.0f} KiB (FETCH_SIZE) and writes "
             f"{copy_w:.0f} KiB (WRITE_SIZE), so FETCH_SIZE is scaled by {ff:.3f} and WRITE_SIZE by {fw:.3f}.",
             f"Kernel sources hash {h}.", "",
             "| kernel | launches | FETCH_SIZE KiB (raw) | WRITE_SIZE KiB (raw) | HBM bytes per launch |",
             "|---|---:|---:|---:|---:|"]
    for kind in sorted(by_kind):
        ks = by_kind[kind]
        if any(not fv or not wv for fv, wv in ks.values()):
            continue
        mf = sum(sum(fv) / len(fv) for fv, _ in ks.values())
        mw = sum(sum(wv) / len(wv) for _, wv in ks.values())
        n = max(len(fv) for fv, _ in ks.values())
        b = mf * 1024.0 * ff + mw * 1024.0 * fw
        rec = {"kernel": kind, "workload": workload, "kernels": sorted(ks), "launches": n, "fetch_kib_raw": mf,
               "write_kib_raw": mw, "fetch_factor": ff, "write_factor": fw, "bytes_per_launch": b,
               "source_hash": h, "commands": [cmd_fetch, cmd_write]}
        with open(os.path.join(out_dir, f"traffic_{kind}_{workload}.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
        lines.append(f"| {kind} | {n} | {mf:.4g} | {mw:.4g} | {b:.4g} |")
    with open(os.path.join(out_dir, f"traffic_{workload}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("--title", default="kernel trace")
    k.add_argument("--command", default="")
    f = sub.add_parser("fp64")
    f.add_argument("db")
    f.add_argument("--title", default="FP64 instruction counts")
    f.add_argument("--command", default="")
    q = sub.add_parser("sq")
    q.add_argument("db1")
    q.add_argument("db2")
    q.add_argument("trace")
    q.add_argument("--title", default="SQ counters")
    q.add_argument("--command", action="append", default=[])
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--out-dir", default="profiles")
    t.add_argument("--command-fetch", default="")
    t.add_argument("--command-write", default="")
    a = ap.parse_args()
    if a.cmd == "kernels":
        print(f"# {a.title}\n")
        if a.command:
            print("Command (from the repository root):\n\n```\n" + a.command + "\n```\n")
        print(f"Kernel sources hash {source_hash()}.\n")
        print("| kernel | calls | total ns | average ns | % |\n|---|---:|---:|---:|---:|")
        for name, n, tot, avg, pct in kernel_table(a.db):
            print(f"| {name} | {n} | {tot:.0f} | {avg:.0f} | {pct:.2f} |")
    elif a.cmd == "fp64":
        print(f"# {a.title}\n")
        if a.command:
            print("Command (from the repository root):\n\n```\n" + a.command + "\n```\n")
        print(f"Kernel sources hash {source_hash()}. Wave-level instruction counts per dispatch (means); "
              "FLOP per dispatch = 64 x (ADD + MUL + 2 FMA + TRANS); rate over the dispatch durations of "
              "the same counter run; peak 78.6 TFLOP/s (FP64 vector).\n")
        print("| kernel | dispatches | avg ms | ADD_F64 | MUL_F64 | FMA_F64 | TRANS_F64 | GFLOP / dispatch "
              "| TFLOP/s | of peak |\n|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|")
        for k, n, dur, c, fl, rate in fp64_table(a.db):
            if fl == 0.0:
                continue
            print(f"| {k} | {n} | {dur * 1e-6:.3f} | {c[FP64_COUNTERS[0]]:.4g} | {c[FP64_COUNTERS[1]]:.4g} | "
                  f"{c[FP64_COUNTERS[2]]:.4g} | {c[FP64_COUNTERS[3]]:.4g} | {fl * 1e-9:.3f} | {rate * 1e-12:.2f} | "
                  f"{100.0 * rate / FP64_PEAK:.1f}% |")
    elif a.cmd == "sq":
        print(f"# {a.title}\n")
        if a.command:
            print("Commands (from the repository root; each pass its own run):\n\n```\n" + "\n".join(a.command)
                  + "\n```\n")
        print(f"Kernel sources hash {source_hash()}. Counters are chip-wide totals per dispatch, averaged over "
              "the dispatches of each kernel; durations from the kernel trace. VALU busy = SQ_INSTS_VALU x 4 "
              "cycles / (duration x 2.4 GHz x 1024 SIMDs), a lower bound; waiting = SQ_WAIT_ANY / "
              "SQ_WAVE_CYCLES (share of resident wave time in s_waitcnt); waves per SIMD = SQ_WAVE_CYCLES x 4 / "
              "(duration x 2.4 GHz x 1024).\n")
        print("| kernel | avg ms | waves | VALU instr / wave | VALU busy | waiting | waves per SIMD "
              "| VMEM rd instr / wave | LDS instr / wave | LDS bank-conflict / LDS active cycles |\n"
              "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|")
        for r in sq_table(a.db1, a.db2, a.trace):
            print(f"| {r[0]} | {r[1]:.3f} | {r[2]:.0f} | {r[3]:.0f} | {100 * r[4]:.0f}% | {100 * r[5]:.0f}% | "
                  f"{r[6]:.2f} | {r[7]:.0f} | {r[8]:.0f} | {100 * r[9]:.0f}% |")
    else:
        traffic(a.fetch, a.write, a.workload, a.out_dir, a.command_fetch, a.command_write)


if __name__ == "__main__":
    main()
