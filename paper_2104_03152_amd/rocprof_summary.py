"""Summarise rocprofv3 result databases into the short text files kept under
profiles/ (kernel-trace statistics, HBM traffic from PMC counters).

    python -m paper_2104_03152_amd.rocprof_summary trace <results.db> <out.md> "<command>"
    python -m paper_2104_03152_amd.rocprof_summary traffic <fetch.db> <write.db> \
        <copy_fetch.db> <copy_write.db> <out.json> <out.md> "<command>"

Traffic: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of each kernel,
scaled by the ratio between the known bytes of a plain 2 GiB copy kernel
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

# kernel-name fragment -> profile family (launch-site grouping of the library)
FAMILIES = [
    ("k_ntt_inv<13>", "ntt_inv"),
    ("k_ntt_fwd<13, 0, 0>", "ntt_fwd"),
    ("k_ntt_fwd<13, 1, 0>", "modup"),
    ("k_ntt_fwd<13, 2, 1>", "moddown+rescale"),
    ("k_hoist_mac<13>", "hoisted_moddown"),
    ("k_inner_hoisted", "hoisted_inner"),
    ("k_inner(", "keyswitch_inner"),
]


def source_sha():
    h = hashlib.sha256()
    for name in ("ntt.hip", "kernels.hip", "modarith.h", "device.h"):
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short(name):
    return name.replace("(anonymous namespace)::", "").replace("void ", "")


def trace(db_path, out_md, command):
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, duration, grid_x, workgroup_x from kernels").fetchall()
    agg = collections.OrderedDict()
    for name, dur, gx, wx in rows:
        a = agg.setdefault(short(name).split("(")[0] if "<" not in name else short(name)[:60], [0, 0.0])
        a[0] += 1
        a[1] += dur
    tot = sum(v[1] for v in agg.values())
    lines = ["# Kernel-trace statistics", "", "Command (repo root on the GPU box):", "",
             "    " + command, "",
             "| kernel | calls | total ms | avg us | share |", "|---|---|---|---|---|"]
    for k, (n, d) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:20]:
        lines.append("| `%s` | %d | %.3f | %.2f | %.1f%% |" % (k, n, d / 1e6, d / n / 1e3, 100 * d / tot))
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def _counter(db_path, counter):
    db = sqlite3.connect(db_path)
    rows = db.execute("select kernel_name, value from counters_collection where counter_name=?",
                      (counter,)).fetchall()
    per = collections.defaultdict(list)
    for name, v in rows:
        per[short(name)].append(float(v))
    return per


def traffic(fetch_db, write_db, cfetch_db, cwrite_db, out_json, out_md, command):
    cf = [v for k, vs in _counter(cfetch_db, "FETCH_SIZE").items() if "kcopy" in k for v in vs]
    cw = [v for k, vs in _counter(cwrite_db, "WRITE_SIZE").items() if "kcopy" in k for v in vs]
    fetch_scale = COPY_BYTES / (sum(cf) / len(cf) * 1024)
    write_scale = COPY_BYTES / (sum(cw) / len(cw) * 1024)
    fe, wr = _counter(fetch_db, "FETCH_SIZE"), _counter(write_db, "WRITE_SIZE")
    fams = {}
    lines = ["# HBM traffic from PMC counters (MNIST-shaped CNN at N = 8192)", "",
             "Commands (repo root on the GPU box):", "", "    " + command, "",
             "Calibration: a plain 2 GiB copy kernel reads FETCH_SIZE = %.0f KiB and "
             "WRITE_SIZE = %.0f KiB per dispatch; scale factors %.4f (fetch) and %.4f (write)."
             % (sum(cf) / len(cf), sum(cw) / len(cw), fetch_scale, write_scale), "",
             "| family | kernel | dispatches | fetch KiB/launch | write KiB/launch | HBM bytes/launch |",
             "|---|---|---|---|---|---|"]
    for frag, fam in FAMILIES:
        fk = [k for k in fe if frag in k]
        wk = [k for k in wr if frag in k]
        if not fk or not wk:
            continue
        fv = [v for k in fk for v in fe[k]]
        wv = [v for k in wk for v in wr[k]]
        fb = sum(fv) / len(fv) * 1024 * fetch_scale
        wb = sum(wv) / len(wv) * 1024 * write_scale
        fams[fam] = fb + wb
        lines.append("| %s | `%s` | %d | %.1f | %.1f | %.0f |" % (fam, fk[0][:40], len(fv), fb / 1024,
                                                                   wb / 1024, fb + wb))
    if "moddown+rescale" in fams:
        fams["moddown"] = fams["rescale"] = fams["moddown+rescale"]
    rec = {"source_sha256": source_sha(), "fetch_scale": fetch_scale, "write_scale": write_scale,
           "families": fams, "command": command}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[3], sys.argv[4])
    else:
        traffic(*sys.argv[2:9])
