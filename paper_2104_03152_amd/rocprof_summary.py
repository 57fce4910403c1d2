"""Summarise rocprofv3 result databases into the short text files kept under
profiles/ (kernel-trace statistics, HBM traffic from PMC counters).

    python -m paper_2104_03152_amd.rocprof_summary trace <results.db> <out.md> "<command>" [bench.out]
    python -m paper_2104_03152_amd.rocprof_summary traffic <fetch.db> <write.db> \\
        <copy_fetch.db> <copy_write.db> <out.json> <out.md> "<command>"
    python -m paper_2104_03152_amd.rocprof_summary counters <pmc.db> <out.md> "<command>" "<title>"

A launch family of the library (the unit its HIP-event profile reports) is
one kernel, or, for small batches of NTTs, a block-phase and a column-phase
kernel issued back to back.  Per family launch: the summed duration (trace)
or the summed HBM bytes (traffic) of its kernels, divided by the number of
family launches (the dispatches of its first kernel).

Only the dispatches between the bench's two window markers (one-element
torch fill kernels around its timed steps) count, when the run has them.

Traffic: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of each kernel,
scaled by the ratio between the known bytes of a plain 2 GiB device copy
and what the same counters read for it.
"""
import collections
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 2 << 30  # the calibration copy moves 2 GiB each way
COPY_KERNEL = "copyBuffer"
MARKER = "FillFunctor"

# family -> (kernels that start a launch, kernels that complete it), as
# name fragments of the N=8192 instantiations.  Small batches run the fused
# forms (two-phase NTTs; the key switch's ModUp and ModDown in three kernels
# each, two each for rotations of coefficient-form ciphertexts; a ModDown
# fused with its rescale in three; rescale in three, or two into
# coefficient form), large batches one workgroup per limb.
FAMILIES = [
    ("ntt_inv", ["k_ntt_inv_1<13, false, 0>", "k_ntt_inv_1<13, true, 0>", "k_ntt_inv<13"], ["k_ntt_inv_2<13>"]),
    ("ntt_fwd", ["k_ntt_fwd_a<13, 0>", "k_ntt_fwd<13, 0, 0>"], ["k_ntt_fwd_b<13, 0, 0>"]),
    ("modup", ["k_ntt_inv_1<13, true, 1>", "k_ntt_inv_1<13, false, 1>", "k_cks_modup_cols<13>",
               "k_ntt_fwd_a<13, 1>", "k_ntt_fwd<13, 1, 0>"],
     ["k_ks_modup_cols<13>", "k_ntt_fwd_b<13, 1, 0>"]),
    ("moddown", ["k_ks_special_blocks<13>", "k_cks_inner_blocks<13>"],
     ["k_ks_moddown_cols<13, 0>", "k_ks_moddown_blocks<13, false>", "k_ks_moddown_resc_cols<13>",
      "k_ks_moddown_blocks<13, true>", "k_cks_moddown_cols<13, 0>"]),
    ("rescale", ["k_ntt_inv_1<13, false, 2>"],
     ["k_ks_moddown_cols<13, 1>", "k_ntt_fwd_b<13, 3, 1>", "k_cks_moddown_cols<13, 1>"]),
    ("moddown+rescale (one workgroup per limb)", ["k_ntt_fwd_a<13, 2>", "k_ntt_fwd<13, 2, 1>"],
     ["k_ntt_fwd_b<13, 2, 1>"]),
    ("hoisted_cols", ["k_hoist_special<13>"], ["k_hoist_cols<13>"]),
    ("hoisted_moddown", ["k_hoist_mac<13, true>", "k_hoist_mac_b<13, true>"], []),
    ("hoisted_replication", ["k_hoist_mac<13, false>", "k_hoist_mac_b<13, false>"], []),
    ("hoisted_inner", ["k_inner_hoisted"], []),
    ("keyswitch_inner", ["k_inner("], []),
]


def source_sha():
    h = hashlib.sha256()
    for name in ("ntt.hip", "kernels.hip", "modarith.h", "butterfly.h", "device.h"):
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short(name):
    return name.replace("(anonymous namespace)::", "").replace("void ", "")


def _match(name, frags):
    return any(f in name for f in frags)


def _families(per_kernel):
    """per_kernel: short name -> list of values (one per dispatch).  Returns
    family -> (launches, total value, kernel names)."""
    out = collections.OrderedDict()
    for fam, first, rest in FAMILIES:
        starts = [k for k in per_kernel if _match(k, first)]
        others = [k for k in per_kernel if _match(k, rest)]
        launches = sum(len(per_kernel[k]) for k in starts)
        if not launches:
            continue
        total = sum(sum(per_kernel[k]) for k in starts + others)
        out[fam] = (launches, total, starts + others)
    return out


def _window(rows):
    """rows: (dispatch_id, name, value).  Keeps those strictly between the
    first two marker dispatches (all of them without markers)."""
    marks = sorted(d for d, name, _ in rows if MARKER in name)
    if len(marks) < 2:
        return [(name, v) for _, name, v in rows if MARKER not in name]
    lo, hi = marks[0], marks[1]
    return [(name, v) for d, name, v in rows if lo < d < hi]


def _bench_profile(path):
    """kernel_profile of the bench JSON line printed by the traced run."""
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        for line in f:
            if line.startswith("{"):
                return json.loads(line).get("kernel_profile") or {}
    return {}


def trace(db_path, out_md, command, bench_out=None):
    ev = _bench_profile(bench_out)
    db = sqlite3.connect(db_path)
    rows = db.execute("select dispatch_id, name, duration from kernels").fetchall()
    per = collections.defaultdict(list)
    for name, dur in _window(rows):
        per[short(name)].append(float(dur))
    tot = sum(sum(v) for v in per.values())
    lines = ["# Kernel-trace statistics", "", "Command (run from the repository root):", "",
             "    " + command, "",
             "## Launch families (N = 8192)", "",
             "Kernel time per family launch over the timed steps (sum of its kernels); beside it "
             "the HIP-event time per launch that the bench measured without the profiler "
             "(launch to completion on the library stream, so it also holds the gap between the "
             "two phase kernels).", "",
             "| family | launches | kernel us per launch | HIP-event us per launch | kernels |",
             "|---|---|---|---|---|"]
    for fam, (n, total, names) in _families(per).items():
        e = ev.get(fam)
        lines.append("| %s | %d | %.2f | %s | %s |" % (
            fam, n, total / n / 1e3, "%.2f" % e["avg_launch_us"] if e else "-",
            ", ".join("`%s`" % k.split("(")[0] for k in names)))
    lines += ["", "## Kernels", "", "| kernel | calls | total ms | avg us | share |", "|---|---|---|---|---|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:24]:
        lines.append("| `%s` | %d | %.3f | %.2f | %.1f%% |" % (k.split("(")[0][:70], len(v), sum(v) / 1e6,
                                                            sum(v) / len(v) / 1e3, 100 * sum(v) / tot))
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter(db_path, counter):
    db = sqlite3.connect(db_path)
    rows = db.execute("select dispatch_id, kernel_name, value from counters_collection where counter_name=?",
                      (counter,)).fetchall()
    per = collections.defaultdict(list)
    for name, v in _window(rows):
        per[short(name)].append(float(v))
    return per


def traffic(fetch_db, write_db, cfetch_db, cwrite_db, out_json, out_md, command):
    cf = [v for k, vs in _counter(cfetch_db, "FETCH_SIZE").items() if COPY_KERNEL in k for v in vs]
    cw = [v for k, vs in _counter(cwrite_db, "WRITE_SIZE").items() if COPY_KERNEL in k for v in vs]
    # the largest dispatches are the 2 GiB copies
    cf, cw = max(cf), max(cw)
    fetch_scale = COPY_BYTES / (cf * 1024)
    write_scale = COPY_BYTES / (cw * 1024)
    fe, wr = _counter(fetch_db, "FETCH_SIZE"), _counter(write_db, "WRITE_SIZE")
    ffam, wfam = _families(fe), _families(wr)
    fams = {}
    lines = ["# HBM traffic from PMC counters (MNIST-shaped CNN at N = 8192)", "",
             "Commands (run from the repository root):", "", "    " + command, "",
             "Calibration: a plain 2 GiB device copy reads FETCH_SIZE = %.0f KiB and "
             "WRITE_SIZE = %.0f KiB per dispatch; scale factors %.4f (fetch) and %.4f (write)."
             % (cf, cw, fetch_scale, write_scale), "",
             "| family | launches | fetch KiB/launch | write KiB/launch | HBM bytes/launch | kernels |",
             "|---|---|---|---|---|---|"]
    for fam in ffam:
        if fam not in wfam:
            continue
        n, ftot, names = ffam[fam]
        nw, wtot, _ = wfam[fam]
        fb = ftot / n * 1024 * fetch_scale
        wb = wtot / nw * 1024 * write_scale
        fams[fam] = fb + wb
        lines.append("| %s | %d | %.1f | %.1f | %.0f | %s |" % (
            fam, n, fb / 1024, wb / 1024, fb + wb, ", ".join("`%s`" % k.split("(")[0] for k in names)))
    rec = {"source_sha256": source_sha(), "fetch_scale": fetch_scale, "write_scale": write_scale,
           "families": fams, "command": command}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def counters(db_path, out_md, command, title, top=14):
    db = sqlite3.connect(db_path)
    rows = db.execute("select dispatch_id, kernel_name, counter_name, value, duration, vgpr_count, "
                      "lds_block_size, workgroup_size from counters_collection").fetchall()
    disp = collections.defaultdict(dict)
    meta = {}
    for did, name, cn, v, dur, vg, lds, wg in rows:
        disp[did][cn] = float(v)
        meta[did] = (name, float(dur), vg, lds, wg)
    marks = sorted(d for d in disp if MARKER in meta[d][0])
    lo, hi = (marks[0], marks[1]) if len(marks) >= 2 else (-1, 1 << 62)
    per = collections.defaultdict(list)
    for d in disp:
        if lo < d < hi and MARKER not in meta[d][0]:
            per[short(meta[d][0])].append(d)
    lines = ["# %s" % title, "", "Command (run from the repository root):", "", "    " + command, "",
             "Per kernel over the profiled dispatches: VALUBusy (% of the time the vector ALUs issue), "
             "VALUUtilization (% of active lanes when they do), OccupancyPercent (% of the wave slots "
             "held), LDSBankConflict (% of the time LDS is stalled by bank conflicts), and VALU, LDS "
             "instructions and LDS wait cycles per wave (SQ_INSTS_VALU, SQ_INSTS_LDS, SQ_WAIT_INST_LDS "
             "over SQ_WAVES); duration-weighted means.", "",
             "| kernel | calls | avg us | VGPRs | LDS KiB | VALUBusy % | VALUUtil % | Occupancy % | "
             "LDS conflict % | VALU/wave | LDS/wave | LDS wait/wave |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    order = sorted(per.items(), key=lambda kv: -sum(meta[d][1] for d in kv[1]))[:top]
    kernels = {}
    for k, ds in order:
        tw = sum(meta[d][1] for d in ds) or 1.0

        def wavg(c):
            return sum(disp[d].get(c, 0.0) * meta[d][1] for d in ds) / tw

        waves = sum(disp[d].get("SQ_WAVES", 0.0) for d in ds) or 1.0

        def pw(c):
            return sum(disp[d].get(c, 0.0) for d in ds) / waves

        _, _, vg, lds, _ = meta[ds[0]]
        kernels[k.split("(")[0]] = {"calls": len(ds), "avg_us": tw / len(ds) / 1e3, "valu_busy_pct": wavg("VALUBusy"),
                                    "valu_util_pct": wavg("VALUUtilization"),
                                    "occupancy_pct": wavg("OccupancyPercent"),
                                    "valu_insts_per_wave": pw("SQ_INSTS_VALU")}
        lines.append("| `%s` | %d | %.2f | %d | %.1f | %.1f | %.1f | %.1f | %.2f | %.0f | %.0f | %.0f |" % (
            k.split("(")[0][:60], len(ds), tw / len(ds) / 1e3, vg, lds / 1024.0, wavg("VALUBusy"),
            wavg("VALUUtilization"), wavg("OccupancyPercent"), wavg("LDSBankConflict"), pw("SQ_INSTS_VALU"),
            pw("SQ_INSTS_LDS"), pw("SQ_WAIT_INST_LDS")))
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    rec = {"source_sha256": source_sha(), "command": command, "kernels": kernels}
    with open(os.path.splitext(out_md)[0] + ".json", "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5] if len(sys.argv) > 5 else None)
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    else:
        traffic(*sys.argv[2:9])
