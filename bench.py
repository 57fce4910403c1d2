"""Encrypted-CNN inference benchmark on one MI355X.

One step = one encrypted inference of the MNIST-shaped network of the paper's
section 5 (conv 4 kernels 7x7 stride 3 -> pack -> square -> FC 256->64 ->
square -> FC 64->10) at N = 8192 with an 8-prime chain (60, 40 x 6, 60 bits)
and scale 2^40, on an input ciphertext already resident in HBM, with the
weights pre-encoded on the device (plans).  Every step runs the whole GPU
path: NTT/INTT, pointwise products, key switching (ModUp, inner product,
ModDown) for 357 rotations/relinearisations, automorphisms and rescales.

Prints one JSON line (see the field list at the bottom).  --gpus N with N > 1
exits: the library runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_network(H, g, x, d):
    """Plans for every layer, made from the intermediate ciphertexts of one
    untimed pass (they fix each layer's input level and scale)."""
    s_ = __import__("paper_2104_03152_amd.inputs", fromlist=["CNN_SHAPE"]).CNN_SHAPE
    conv = [H.he_conv_plan(g, x, d["conv_k"][c], s_["windows"], d["conv_b"][c])
            for c in range(s_["channels"])]
    parts = H.he_plan_apply_many(g, conv, x)
    s1 = H.he_square(g, H.he_pack(g, parts, s_["windows"]))
    fc1 = H.he_matmul_plan(g, s1, d["w1"], d["b1"])
    s2 = H.he_square(g, H.he_plan_apply(g, fc1, s1))
    fc2 = H.he_matmul_plan(g, s2, d["w2"], d["b2"])
    return conv, fc1, fc2


def step(H, g, net, x, width, stamp=None):
    conv, fc1, fc2 = net
    parts = H.he_plan_apply_many(g, conv, x)
    if stamp:
        stamp("conv")
    p = H.he_pack(g, parts, width)
    if stamp:
        stamp("pack")
    s1 = H.he_square(g, p)
    if stamp:
        stamp("square1")
    h = H.he_plan_apply(g, fc1, s1)
    if stamp:
        stamp("fc1")
    s2 = H.he_square(g, h)
    if stamp:
        stamp("square2")
    y = H.he_plan_apply(g, fc2, s2)
    if stamp:
        stamp("fc2")
    return y


def cnn_fp64(d):
    """Plain FP64 forward of the same network; the convolution slides each
    7x7 kernel over the image directly (no im2col), channel-major output."""
    img, k, s = d["img"], 7, 3
    o = (img.shape[0] - k) // s + 1
    conv = np.empty((d["conv_k"].shape[0], o, o))
    for c in range(conv.shape[0]):
        kern = d["conv_k"][c].reshape(k, k)
        for oy in range(o):
            for ox in range(o):
                conv[c, oy, ox] = (img[oy * s:oy * s + k, ox * s:ox * s + k] * kern).sum() + d["conv_b"][c]
    x = conv.reshape(-1) ** 2
    h = (x @ d["w1"] + d["b1"]) ** 2
    return h @ d["w2"] + d["b2"]


def cpu_baseline(params, d, budget_s):
    """The plain C oracle (single thread) on the host: one full encrypted
    inference of the same network (keys generated outside the timing)."""
    from oracle import oracle as O
    o = O.Oracle(params["log_n"], params["bits"], params["scale"], params["seed"])
    o.keygen()
    from paper_2104_03152_amd import inputs as I
    for st, lv in sorted(I.cnn_rotation_steps().items()):
        o.galois_keygen(st, lv)
    ct = o.encrypt(o.encode(O.im2col(d["img"], 7, 3), o.scale, o.L - 1), 0)
    t0 = time.perf_counter()
    n = 0
    out = None
    while True:
        out = o.cnn(ct, d["conv_k"], d["conv_b"], d["w1"], d["b1"], d["w2"], d["b2"])
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 3:
            break
    dt = time.perf_counter() - t0
    return n / dt, n, dt, out


def small_ops_table(H, I, torch, runs=1000, oracle_runs=5):
    """The N=4096 operation set (three primes 40, 20 | 40 bits, scale 2^20,
    secret-key encryption, x, y, p uniform in [-1, 1]^2048): per operation
    the GPU latency p50/p99 over `runs` synchronised calls, the oracle's time
    on this host (one thread, median), the largest error of the decrypted
    GPU result against plaintext arithmetic beside its tolerance, and whether
    the GPU ciphertext equals the oracle's bit for bit."""
    from oracle import oracle as O
    p = I.SMALL
    steps = [1 << t for t in range(11)]
    g = H.he_ctx_create(p["log_n"], p["bits"], p["scale"], p["seed"], auto_rescale=True)
    H.he_keygen(g, steps)
    o = O.Oracle(p["log_n"], p["bits"], p["scale"], p["seed"])
    o.keygen()
    for st in steps:
        o.galois_keygen(st)
    x, y, pv = I.small_vectors()
    gx = H.he_encrypt(g, H.he_encode(g, x, p["scale"], 1), 0, True)
    gy = H.he_encrypt(g, H.he_encode(g, y, p["scale"], 1), 1, True)
    gp = H.he_encode(g, pv, p["scale"], 1)
    ox = o.encrypt(o.encode(x, p["scale"], 1), 0, True)
    oy = o.encrypt(o.encode(y, p["scale"], 1), 1, True)
    op = o.encode(pv, p["scale"], 1)
    ops = {
        "add": (lambda: H.he_add(g, gx, gy), lambda: o.add(ox, oy), x + y, 1e-2),
        "mul_plain+rescale": (lambda: H.he_mul_plain(g, gx, gp), lambda: o.rescale(o.mul_plain(ox, op)),
                              x * pv, 1e-2),
        "mul_relin+rescale": (lambda: H.he_mul_relin(g, gx, gy), lambda: o.rescale(o.mul_relin(ox, oy)),
                              x * y, 1e-2),
        "rotate_1": (lambda: H.he_rotate(g, gx, 1), lambda: o.rotate(ox, 1), np.roll(x, -1), 2e-2),
        "sum_slots_2048": (lambda: H.he_sum_slots(g, gx, 2048), lambda: o.sum_slots(ox, 2048),
                           np.array([x.sum()]), 1.0),
    }
    table = {}
    for name, (gpu, orc, want, tol) in ops.items():
        r = gpu()
        H.he_sync(g)
        lat = []
        for _ in range(runs):
            t = time.perf_counter()
            r = gpu()
            H.he_sync(g)
            lat.append((time.perf_counter() - t) * 1e3)
        ot = []
        for _ in range(oracle_runs):
            t = time.perf_counter()
            ro = orc()
            ot.append((time.perf_counter() - t) * 1e3)
        dec = H.he_decode(g, H.he_decrypt(g, r), len(want))
        table[name] = {"gpu_p50_ms": float(np.percentile(lat, 50)), "gpu_p99_ms": float(np.percentile(lat, 99)),
                       "gpu_runs": runs, "oracle_ms": float(np.median(ot)), "oracle_runs": oracle_runs,
                       "max_abs_err": float(np.abs(dec - want).max()), "tolerance": tol,
                       "bit_exact_vs_oracle": bool(np.array_equal(H.he_ct_export(g, r), ro.data()))}
        del r
    del gx, gy, gp
    g.close()
    return {"params": "N=4096, primes (40, 20 | 40) bits, scale 2^20, secret-key encryption, 2048 slots",
            "ops": table}


def uneven_oracle_check(sample, seed=4):
    """The work queue's results for a sample of the N=4096 operations of the
    uneven mix against the oracle (same primes, seed and keys)."""
    from oracle import oracle as O
    o = O.Oracle(12, [50] * 9, 2.0 ** 40, seed)
    o.keygen()
    o.galois_keygen(1)
    ok = []
    for s in sample:
        a = o.ct_from_data(s["a"], s["lp"] - 1, 2.0 ** 40)
        if s["kind"] == 0:
            ref = o.rescale(o.mul_relin(a, o.ct_from_data(s["b"], s["lp"] - 1, 2.0 ** 40)))
        else:
            ref = o.rotate(a, 1)
        ok.append(bool(np.array_equal(ref.data(), s["out"])))
    return {"operations": len(ok), "bit_exact": all(ok) if ok else None}


def host_info():
    """The host the oracle runs on: CPU model, logical CPUs, and the CPUs this
    process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}


def cpu_parallel_worker(n_workers, budget_s):
    """(A child process without torch.)  The oracle's keys generated once,
    then n_workers forked processes each run full encrypted inferences of
    the same network for budget_s seconds: host throughput with every
    worker busy.  Prints one JSON line."""
    import multiprocessing as mp
    from oracle import oracle as O
    from paper_2104_03152_amd import inputs as I
    params, d = I.CNN, I.cnn_inputs()
    o = O.Oracle(params["log_n"], params["bits"], params["scale"], params["seed"])
    o.keygen()
    for st, lv in sorted(I.cnn_rotation_steps().items()):
        o.galois_keygen(st, lv)
    ct = o.encrypt(o.encode(O.im2col(d["img"], 7, 3), o.scale, o.L - 1), 0)
    ref = o.cnn(ct, d["conv_k"], d["conv_b"], d["w1"], d["b1"], d["w2"], d["b2"]).data()
    q = mp.get_context("fork").Queue()

    def work():
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            y = o.cnn(ct, d["conv_k"], d["conv_b"], d["w1"], d["b1"], d["w2"], d["b2"])
            n += 1
        q.put((n, bool(np.array_equal(y.data(), ref))))

    procs = [mp.get_context("fork").Process(target=work) for _ in range(n_workers)]
    t0 = time.perf_counter()
    for pr in procs:
        pr.start()
    res = [q.get() for _ in procs]
    for pr in procs:
        pr.join()
    dt = time.perf_counter() - t0
    n = sum(r[0] for r in res)
    print(json.dumps({"inferences": n, "seconds": dt, "workers": n_workers,
                      "all_equal": all(r[1] for r in res)}), flush=True)


def cpu_baseline_parallel(budget_s):
    """The oracle on every usable host CPU (at most 16, the GPU's share of
    the host): independent inferences in parallel processes."""
    import subprocess
    info = host_info()
    workers = max(1, min(16, info["usable_cpus"]))
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-workers", str(workers),
                        "--cpu-budget", str(budget_s)], capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-500:]}
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    rec["value"] = rec["inferences"] / rec["seconds"]
    rec["unit"] = "inferences/s"
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--latency-runs", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=8.0)
    ap.add_argument("--no-extra-bench", action="store_true",
                    help="skip the N=16384 NTT and key-switch benches (profiling runs)")
    ap.add_argument("--probe", action="store_true",
                    help="only measure the issue rates and copy bandwidth the roofline peaks use")
    ap.add_argument("--serving-requests", type=int, default=0,
                    help="requests per serving rate (default: enough for about 2 s per rate, at least 128)")
    ap.add_argument("--cpu-workers", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--ntt-only", action="store_true",
                    help="only run the batched N=16384 NTT bench (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 2 GiB buffer three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.cpu_workers:
        cpu_parallel_worker(args.cpu_workers, args.cpu_budget)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(requests/ciphertexts would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    log("importing torch")
    import torch
    import paper_2104_03152_amd as H
    from paper_2104_03152_amd import inputs as I

    assert torch.cuda.is_available(), "needs a GPU"
    if args.probe:
        print(json.dumps(probe(torch)), flush=True)
        return
    if args.ntt_only:
        print(json.dumps({"kernel_bench_n16384": kernel_bench(H, torch, I)}), flush=True)
        return
    if args.copy_calibration:
        # a plain device-to-device copy of known size: 2 GiB read, 2 GiB written
        src = torch.empty(1 << 28, dtype=torch.int64, device="cuda").random_()
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 3 x 2 GiB")
        return
    params = I.CNN
    shape = I.CNN_SHAPE
    d = I.cnn_inputs()
    log("context + keys")
    t0 = time.perf_counter()
    # the library's own stream (capturable into a graph)
    g = H.he_ctx_create(params["log_n"], params["bits"], params["scale"], params["seed"],
                        auto_rescale=True, stream=None)
    H.he_keygen(g, [])
    for st, lv in sorted(I.cnn_rotation_steps().items()):
        H.he_keygen_galois(g, st, lv)
    H.he_sync(g)
    keygen_s = time.perf_counter() - t0
    v = H.he_im2col(d["img"], shape["k"], shape["stride"])
    x = H.he_encrypt(g, H.he_encode(g, v, params["scale"], g.L - 1), 0, False)
    log("plans")
    net = build_network(H, g, x, d)
    ref = H.he_ct_export(g, step(H, g, net, x, shape["windows"]))

    log("warmup")
    for _ in range(args.warmup):
        y = step(H, g, net, x, shape["windows"])
    torch.cuda.synchronize()

    log("timed %d steps" % args.steps)
    torch.cuda.synchronize()
    window_marker(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        y = step(H, g, net, x, shape["windows"])
    H.he_sync(g)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    window_marker(torch)
    ms_per_step = dt * 1e3 / args.steps
    out = H.he_ct_export(g, y)
    bit_exact_repeat = bool(np.array_equal(out, ref))
    logits = H.he_decode(g, H.he_decrypt(g, y), shape["out"])
    logits_err = float(np.abs(logits - cnn_fp64(d)).max())

    # host time to enqueue one step (no synchronisation inside the step)
    H.he_sync(g)
    enq = []
    for _ in range(10):
        t1 = time.perf_counter()
        step(H, g, net, x, shape["windows"])
        enq.append((time.perf_counter() - t1) * 1e3)
        H.he_sync(g)
    enqueue_ms = float(np.median(enq))

    log("latency distribution")
    lat = []
    for _ in range(args.latency_runs):
        t1 = time.perf_counter()
        y = step(H, g, net, x, shape["windows"])
        H.he_sync(g)
        lat.append((time.perf_counter() - t1) * 1e3)
    lat = np.array(lat)

    log("per-stage times")
    stages = {}
    for _ in range(10):
        last = [time.perf_counter()]

        def stamp(name):
            H.he_sync(g)
            now = time.perf_counter()
            stages.setdefault(name, []).append((now - last[0]) * 1e3)
            last[0] = now
        H.he_sync(g)
        last[0] = time.perf_counter()
        step(H, g, net, x, shape["windows"], stamp)
    stage_ms = {k: float(np.median(v_)) for k, v_ in stages.items()}

    log("kernel profile (HIP events on the library stream)")
    fams = ["ntt_fwd", "ntt_inv", "modup", "moddown", "rescale", "keyswitch_inner", "hoisted_inner",
            "hoisted_cols", "hoisted_moddown", "hoisted_replication", "pointwise", "sample"]
    H.he_profile_enable(g, True)
    prof_steps = 5
    for _ in range(prof_steps):
        step(H, g, net, x, shape["windows"])
    H.he_sync(g)
    prof = {}
    for f in fams:
        n, ms, units, by = H.he_profile_read(g, f)
        if n:
            prof[f] = {"launches_per_step": n / prof_steps, "ms_per_step": ms / prof_steps,
                       "avg_launch_us": 1e3 * ms / n, "units_per_launch": units / n,
                       "bytes_per_launch": by / n}
    H.he_profile_enable(g, False)
    # the dominant kernel: the one-kernel family with the most time per step
    # (the two-phase families spread their time over three kernels each)
    single = [k for k in prof if k in SINGLE_KERNEL_FAMILIES]
    dom = max(single, key=lambda k: prof[k]["ms_per_step"]) if single else None
    roof = roofline_entry(dom, prof[dom], g.n) if dom else None

    log("graph: one captured step, replayed")
    graph_res = graph_replay(H, g, net, x, shape["windows"], ref, args.steps)

    kbench = ksbench = sweep = uneven = serving = None
    if not args.no_extra_bench:
        log("op sweep: the appendix unary/binary operation tables at N=8192")
        sweep = op_sweep(H, I)
        log("kernel bench: batched NTT at N=16384")
        kbench = kernel_bench(H, torch, I)
        log("key-switch bench: batched multiply/rotate at N=16384")
        ksbench = keyswitch_bench(H, I)
        log("uneven batching: 1024 ops over three ring degrees and seven levels")
        uneven = uneven_bench(H, I)
        log("serving: Poisson arrivals, CNN and logistic-regression requests")
        serving = serving_bench(H, I, d, n_requests=args.serving_requests)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        rate, n_inf, cdt, oy = cpu_baseline(params, d, args.cpu_budget)
        cpu = {"value": rate, "unit": "inferences/s", "cores": 1, "kind": "oracle",
               "sample": "%d full encrypted inference(s) of the same network, %.1f s, single "
                         "thread, keys generated outside the timing" % (n_inf, cdt),
               "bit_exact_vs_gpu": bool(np.array_equal(oy.data(), ref)),
               "host": host_info()}
        log("cpu baseline, every usable host CPU")
        cpu["parallel"] = cpu_baseline_parallel(args.cpu_budget)
        log("cpu baseline: N=4096 operation set, GPU beside the oracle")
        cpu["small_ops"] = small_ops_table(H, I, torch)
        if uneven is not None:
            cpu["uneven_oracle_sample"] = uneven_oracle_check(uneven.pop("oracle_sample"))

    if uneven is not None:
        uneven.pop("oracle_sample", None)  # checked by the CPU baseline leg, not reported
    res = {
        "metric": "encrypted-CNN inferences/s (N=8192, batch 1)",
        "value": 1e3 / ms_per_step,
        "unit": "inferences/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (28x28 uniform image, N(0,0.1^2) weights; MNIST and trained weights "
                "not available)",
        "config": {"workload": "encrypted MNIST-shaped CNN, batch 1: conv 4x7x7/3, square, FC "
                               "256->64, square, FC 64->10",
                   "ring_degree": 8192, "prime_bits": params["bits"], "scale": "2^40",
                   "galois_keys": len(I.cnn_rotation_steps()), "key_switches_per_step": 357},
        "latency_ms": ({"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                        "runs": int(len(lat))} if len(lat) else None),
        "stage_ms": stage_ms,
        "host_enqueue_ms": enqueue_ms,
        "kernel_profile": prof,
        "roofline": roof,
        "step_hbm": step_traffic(prof, g.n),
        "graph_replay": graph_res,
        "kernel_bench": kbench,
        "keyswitch_bench": ksbench,
        "op_sweep": sweep,
        "uneven_batching": uneven,
        "serving": serving,
        "cpu_baseline": cpu,
        "bit_exact_repeat": bit_exact_repeat,
        "logits_max_abs_err": logits_err,
        "keygen_s": keygen_s,
        "paper_context": "TenSEAL on AWS c4.4xlarge (16 vCPU Xeon E5-2666 v3): 887.06 ms full "
                         "forward at N=8192, 206-bit modulus, scale 2^21 (table 2); context only",
    }
    print(json.dumps(res), flush=True)


# Roofline of a kernel family.  NTT-type kernels (every family that runs the
# LDS NTT) are bound by VALU issue: the work unit is the butterfly, (N/2)
# log2 N per limb-NTT; the peak is the VALU issue rate (256 CUs x 4 SIMD16 x
# 16 lanes x 2.4 GHz = 39.3 T lane-instructions/s, FP64 FMA at full rate)
# over the VALU operation count of the cheaper of the two butterflies: the
# exact FP64 one (11 operations; the 64-bit integer Shoup butterfly takes
# about 27).  The inner products are bound by HBM (their key reads).
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
BUTTERFLY_INSTR = 11
SINGLE_KERNEL_FAMILIES = ("hoisted_moddown", "hoisted_replication", "hoisted_inner", "keyswitch_inner")
NTT_FAMILIES = ("ntt_fwd", "ntt_inv", "modup", "moddown", "rescale")
# key-switch inner products fused with transforms (the two-phase hoisted
# product): their algorithmic bytes are the key words they read
FUSED_FAMILIES = ("hoisted_cols", "hoisted_moddown", "hoisted_replication")


def cnn_step_algorithmic_bytes(n):
    """HBM bytes one inference must move at least: every key switch reads its
    key once at the level of use (2 Lp (Lp + 1) limbs; a key shared by the
    four conv channels once), every plaintext operand once, the input and
    output ciphertexts once; 8N bytes per limb."""
    key = lambda lp: 2 * lp * (lp + 1)
    uses = [(6, 6),              # conv: six rotation steps, one key each for the 4 channels
            (3, 5), (1, 5),      # packing rotations, first relinearisation
            (15 + 255, 4),       # FC1: replication and the 255 diagonal rotations
            (1, 3),              # second relinearisation
            (63 + 63, 2)]        # FC2: replication and the 63 diagonal rotations
    limbs = sum(c * key(lp) for c, lp in uses)
    limbs += 4 * 7 + 4 * 6 + 4 * 6   # conv kernels, channel masks, conv biases
    limbs += 256 * 4 + 3 + 64 * 2 + 1  # FC1, FC2 diagonals and biases
    limbs += 2 * 7 + 2 * 1           # input and output ciphertexts
    return 8 * n * limbs


def step_traffic(prof, n):
    """Measured HBM bytes per step (PMC counters of every profiled family
    times its launches per step) beside the algorithmic bytes."""
    alg = cnn_step_algorithmic_bytes(n)
    fams = {f: pmc_traffic(f) for f in prof}
    have = {f: v for f, v in fams.items() if v is not None}
    meas = sum(v * prof[f]["launches_per_step"] for f, v in have.items()) if have else None
    return {"algorithmic_bytes": alg, "counter_bytes_profiled_families": meas,
            "families_with_counters": sorted(have),
            "ratio": (meas / alg) if meas else None}


def roofline_entry(fam, p, n):
    t = p["avg_launch_us"] * 1e-6
    hbm = p["bytes_per_launch"] / t / 1e9
    traffic = pmc_traffic(fam)
    ratio = traffic / p["bytes_per_launch"] if traffic else None
    if fam in NTT_FAMILIES:
        bfly = p["units_per_launch"] * (n // 2) * (n.bit_length() - 1)
        ach = bfly / t / 1e9
        peak = VALU_LANE_OPS / BUTTERFLY_INSTR / 1e9
        return {"bound": "alu", "family": fam, "achieved": ach, "peak": peak,
                "unit": "G butterfly/s", "frac": ach / peak, "traffic": traffic,
                "hbm_gbs": hbm, "hbm_frac": hbm / HBM_PEAK_GBS,
                "avg_launch_us": p["avg_launch_us"], "units_per_launch": p["units_per_launch"],
                "algorithmic_bytes_per_launch": p["bytes_per_launch"]}
    if fam in FUSED_FAMILIES:
        # both roofs: the key reads against HBM, the measured VALU issue
        # (counters of the committed profile, when it matches the source)
        valu = pmc_valu(fam)
        bfly = p["units_per_launch"] * (n // 2) * (n.bit_length() - 1)
        return {"bound": "hbm", "family": fam, "achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hbm / HBM_PEAK_GBS, "traffic": traffic, "traffic_over_algorithmic": ratio,
                "valu_busy_pct": valu,
                "binding": None if valu is None else ("valu" if valu / 100 > hbm / HBM_PEAK_GBS else "hbm"),
                "butterfly_frac": bfly / (p["avg_launch_us"] * 1e-6) / (VALU_LANE_OPS / BUTTERFLY_INSTR),
                "avg_launch_us": p["avg_launch_us"], "algorithmic_bytes_per_launch": p["bytes_per_launch"],
                "algorithmic": "the key words of the launch's rotations and the diagonals, read once (the "
                               "column-phase output and the partial sums are intermediates of this design)"}
    return {"bound": "hbm", "family": fam, "achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": hbm / HBM_PEAK_GBS, "traffic": traffic, "traffic_over_algorithmic": ratio,
            "avg_launch_us": p["avg_launch_us"], "algorithmic_bytes_per_launch": p["bytes_per_launch"],
            "algorithmic": "the keys of the launch's rotations and their shared ModUp digits, read once"}


def source_hash():
    import hashlib
    src = os.path.join(ROOT, "paper_2104_03152_amd", "csrc")
    h = hashlib.sha256()
    for name in ("ntt.hip", "kernels.hip", "modarith.h", "butterfly.h", "device.h"):
        with open(os.path.join(src, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_valu(fam):
    """Duration-weighted VALUBusy (%) of a family's kernels from the committed
    counter profile of the CNN step, or None when the kernel source changed
    since it was taken."""
    from paper_2104_03152_amd.rocprof_summary import FAMILIES
    path = os.path.join(ROOT, "profiles", "cnn_n8192_valu_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != source_hash():
        return None
    frags = [fr for name, first, rest in FAMILIES if name == fam for fr in first + rest]
    ks = [v for k, v in rec.get("kernels", {}).items() if any(fr.split("(")[0] in k for fr in frags)]
    w = sum(v["calls"] * v["avg_us"] for v in ks)
    return sum(v["valu_busy_pct"] * v["calls"] * v["avg_us"] for v in ks) / w if w else None


def pmc_traffic(fam):
    """HBM bytes per launch measured by rocprofv3 PMC counters (FETCH_SIZE,
    WRITE_SIZE, calibrated by a copy kernel), valid only while the kernel
    source is unchanged since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != source_hash():
        return None
    return rec.get("families", {}).get(fam)


def graph_replay(H, g, net, x, width, ref, steps):
    """The same step captured once into a HIP graph (input: a copy of x) and
    replayed `steps` times; checked bit for bit against the eager output."""
    import numpy as np
    xin = H.he_drop_to(g, x, x.info()[0])
    H.he_sync(g)
    H.he_graph_begin(g)
    y = step(H, g, net, xin, width)
    graph = H.he_graph_end(g)
    H.he_graph_launch(g, graph)
    H.he_sync(g)
    exact = bool(np.array_equal(H.he_ct_export(g, y), ref))
    t0 = time.perf_counter()
    enq = 0.0
    for _ in range(steps):
        t1 = time.perf_counter()
        H.he_graph_launch(g, graph)
        enq += time.perf_counter() - t1
    H.he_sync(g)
    dt = time.perf_counter() - t0
    exact = exact and bool(np.array_equal(H.he_ct_export(g, y), ref))
    graph.free()
    return {"ms_per_step": dt * 1e3 / steps, "inferences_per_s": steps / dt,
            "host_launch_ms": enq * 1e3 / steps, "bit_exact_vs_eager": exact}


def probe(torch, blocks=2048, iters=4096, reps=3):
    """Issue rates of the instructions the NTT butterflies are built from,
    and the bandwidth of a plain device copy, on this GPU (the measured
    counterparts of the published peaks)."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2104_03152_amd", "libckks_probe.so"))
    lib.probe_rate.restype = C.c_double
    lib.probe_rate.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p]
    lib.probe_copy.restype = C.c_double
    lib.probe_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_longlong, C.c_int]
    out = torch.empty(blocks * 256, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    kinds = {0: "v_mad_u64_u32", 1: "v_mul_lo_u32", 2: "v_mul_hi_u32", 3: "v_fma_f64", 4: "v_add_u32"}
    rates = {}
    for k, name in kinds.items():
        best = min(lib.probe_rate(k, blocks, iters, out.data_ptr()) for _ in range(reps))
        assert best > 0, name
        r = blocks * 256 * iters * 8 / (best * 1e-3)
        rates[name] = {"t_per_s": r / 1e12, "frac_of_lane_peak": r / VALU_LANE_OPS}
    nbytes = 1 << 30
    src = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda").random_()
    dst = torch.empty_like(src)
    copies = {}
    for cb in (1024, 4096, 16384):
        best = min(lib.probe_copy(src.data_ptr(), dst.data_ptr(), nbytes, cb) for _ in range(reps))
        copies[str(cb)] = 2 * nbytes / (best * 1e-3) / 1e9
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    t = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        t.append(a.elapsed_time(b))
    return {"probe": "issue rates (one instruction kind, 8 independent chains per lane, %d x 256 lanes)"
                     % blocks,
            "lane_peak_t_per_s": VALU_LANE_OPS / 1e12, "rates": rates,
            "copy_gbs_by_blocks": copies, "torch_copy_gbs": 2 * nbytes / (min(t) * 1e-3) / 1e9,
            "hbm_peak_gbs": HBM_PEAK_GBS, "copy_bytes": nbytes}


def window_marker(torch):
    """A one-element fill kernel, the only torch kernel of the CNN run: the
    profile summaries keep the dispatches between the first two."""
    torch.full((1,), 1.0, device="cuda")
    torch.cuda.synchronize()


def kernel_bench(H, torch, I, n_ct=256, reps=5):
    """Batched forward + inverse NTT over 256 ciphertexts x 2 polys x 8
    limbs at N = 16384 (4096 limb-NTTs, 512 MiB per pass)."""
    p = I.RAW
    g = H.he_ctx_create(p["log_n"], p["bits"], p["scale"], p["seed"], stream=None)
    n, limbs = g.n, g.L
    # the autotuner picks the form and thread layout per launch size
    chosen, tune_rows = H.he_tune_ntt(g, n_ct * 2 * limbs)
    layouts = H.he_ntt_layouts(g)
    buf = torch.empty((n_ct * 2, limbs, n), dtype=torch.int64, device="cuda")
    for i in range(limbs):
        buf[:, i, :] = torch.randint(0, g.primes[i], (n_ct * 2, n), dtype=torch.int64, device="cuda")
    ref = buf.clone()
    torch.cuda.synchronize()
    H.he_ntt_forward(g, buf.data_ptr(), n_ct * 2, limbs)
    H.he_ntt_inverse(g, buf.data_ptr(), n_ct * 2, limbs)
    H.he_sync(g)
    H.he_profile_enable(g, True)
    for _ in range(reps):
        H.he_ntt_forward(g, buf.data_ptr(), n_ct * 2, limbs)
        H.he_ntt_inverse(g, buf.data_ptr(), n_ct * 2, limbs)
    H.he_sync(g)
    out = {}
    for fam in ("ntt_fwd", "ntt_inv"):
        cnt, ms, units, by = H.he_profile_read(g, fam)
        t = ms / cnt * 1e-3
        bfly = units / cnt * (n // 2) * (n.bit_length() - 1)
        out[fam] = {"limb_ntts_per_launch": units / cnt, "avg_launch_us": t * 1e6,
                    "limb_ntts_per_s": units / cnt / t, "hbm_gbs": by / cnt / t / 1e9,
                    "hbm_frac": by / cnt / t / 1e9 / HBM_PEAK_GBS,
                    "g_butterfly_s": bfly / t / 1e9,
                    "alu_frac": bfly / t / (VALU_LANE_OPS / BUTTERFLY_INSTR)}
    H.he_profile_enable(g, False)
    torch.cuda.synchronize()
    out["roundtrip_exact"] = bool(torch.equal(buf, ref))
    out["workload"] = "%d ciphertexts x 2 polys x %d limbs, N=%d, 50-bit primes" % (n_ct, limbs, n)
    out["tuning"] = {"layouts_log2_words_radix": layouts, "split_jobs": chosen,
                     "rows_us_fwd_plus_inv": [[round(v, 1) for v in r] for r in tune_rows],
                     "columns": "J, two-phase, layout 0, layout 1, ..."}
    del buf, ref
    g.close()
    return out


# the appendix tables of unary and binary operations (ms, 8 vCPU c4.2xlarge,
# N = 8192, 200-bit modulus): context for op_sweep
PAPER_OPS_MS = {
    "negate": [0.07, 0.07, 0.07, 0.13, 0.26], "square": [4.29, 4.29, 4.29, 8.49, 17.16],
    "polyval": [10.55, 10.46, 10.51, 21.32, 42.68], "add": [0.08, 0.08, 0.08, 0.16, 0.31],
    "multiply": [4.45, 4.34, 4.43, 8.84, 17.75], "sub": [0.08, 0.08, 0.08, 0.15, 0.3],
    "dot": [20.15, 23.96, 28.11, 55.94, 112.36], "add_plain": [0.8, 0.86, 1.07, 2.13, 4.19],
    "multiply_plain": [1.75, 1.81, 2.03, 4.02, 7.97], "sub_plain": [0.8, 0.86, 1.08, 2.14, 4.21],
    "dot_plain": [17.37, 21.36, 25.63, 51.14, 101.82]}


def op_sweep(H, I, shapes=(256, 1024, 4096, 8192, 16384), reps=10):
    """Each operation of the appendix tables on encrypted vectors of the
    given lengths at N = 8192 with a 200-bit chain (60, 40, 40, 60) and
    automatic rescaling.  A vector is a rank-1 tensor (he_tensor_*): lengths
    above N/2 span several ciphertexts (products as one batch).  `_plain`
    operands are encoded inside the timed call, as a plain tensor operand
    is; polyval evaluates 2X^2 + X; dot is the product followed by the sum
    over the vector.  Milliseconds per call, wall clock between
    synchronisations (host work included)."""
    import numpy as np
    g = H.he_ctx_create(13, [60, 40, 40, 60], 2.0 ** 40, 4, auto_rescale=True, stream=None)
    H.he_keygen(g, [1 << t for t in range(12)])
    rng = np.random.default_rng(4)
    out = {op: [] for op in PAPER_OPS_MS}
    top = g.L - 1
    for shape in shapes:
        xv, yv = rng.uniform(-1, 1, shape), rng.uniform(-1, 1, shape)
        X = H.he_tensor_encrypt(g, xv, 2.0 ** 40, top, 0)
        Y = H.he_tensor_encrypt(g, yv, 2.0 ** 40, top, 100)
        H.he_sync(g)
        ops = {
            "negate": lambda: H.he_tensor_negate(g, X),
            "square": lambda: H.he_tensor_square(g, X),
            "polyval": lambda: H.he_tensor_polyval(g, X, [0.0, 1.0, 2.0]),
            "add": lambda: H.he_tensor_add(g, X, Y),
            "multiply": lambda: H.he_tensor_mul(g, X, Y),
            "sub": lambda: H.he_tensor_sub(g, X, Y),
            "dot": lambda: H.he_tensor_dot(g, X, Y),
            "add_plain": lambda: H.he_tensor_add_plain(g, X, yv),
            "multiply_plain": lambda: H.he_tensor_mul_plain(g, X, yv),
            "sub_plain": lambda: H.he_tensor_sub_plain(g, X, yv),
            "dot_plain": lambda: H.he_tensor_dot_plain(g, X, yv),
        }
        for name, fn in ops.items():
            r = fn()
            H.he_sync(g)
            del r
            t = time.perf_counter()
            for _ in range(reps):
                r = fn()
            H.he_sync(g)
            out[name].append((time.perf_counter() - t) * 1e3 / reps)
            del r
        del X, Y
    g.close()
    return {"shapes": list(shapes), "ms": out, "paper_ms_8vcpu": PAPER_OPS_MS,
            "params": "N=8192, primes (60, 40, 40, 60), scale 2^40, auto rescale; rank-1 tensors"}


def serving_bench(H, I, d, qps_list=(10, 20, 50, 100, 200, 500, 1000, 2000), n_clients=8,
                  budget=8 << 30, seed=5, n_requests=0):
    """Poisson arrivals at each rate, half CNN and half logistic-regression
    requests (N=8192, the CNN's chain; LR feature dimension uniform in
    64..1024, weights and bias N(0, 1), inputs uniform in [-1, 1]); 16
    requests per client key set, eight key sets resident on the device;
    admission by an 8 GiB working-set budget.  Continuous batching against
    one-request-at-a-time service of the same requests; latency from
    arrival to the decrypt-ready result."""
    from paper_2104_03152_amd import serve as S
    t0 = time.perf_counter()
    clients = [S.Client(H, c, d) for c in range(n_clients)]
    setup_s = time.perf_counter() - t0
    out = {"clients": n_clients, "key_bytes_per_client": clients[0].key_bytes,
           "client_setup_s": setup_s, "budget_bytes": budget, "points": []}
    # warm-up: every client's pool holds the buffers of both request kinds
    # before either service mode is timed
    warm = S.make_requests(H, clients, 4 * n_clients * 2, 0, seed, per_client=8)
    S.serve(H, warm, budget, batched=True)
    S.reset(warm)
    S.serve(H, warm, budget, batched=False)
    del warm
    for qps in qps_list:
        n = n_requests or int(max(128, min(1000, 2 * qps)))
        reqs = S.make_requests(H, clients, n, qps, seed + qps)
        log("serving: %d QPS, %d requests, continuous batching" % (qps, n))
        lat_b = S.serve(H, reqs, budget, batched=True)
        sb = S.summary(lat_b, reqs)
        S.reset(reqs)
        log("serving: %d QPS, %d requests, one at a time" % (qps, n))
        lat_1 = S.serve(H, reqs, budget, batched=False)
        s1 = S.summary(lat_1, reqs)
        out["points"].append({"qps": qps, "requests": n,
                              "cnn": sum(r.kind == "cnn" for r in reqs),
                              "continuous_batching": sb, "one_at_a_time": s1})
        del reqs
    for c in clients:
        c.close()
    return out


def uneven_bench(H, I, n_ops=1024, seed=4):
    """1024 operations, each a multiply + relinearise + rescale or a
    rotation by one slot, on ring degree N in {4096, 8192, 16384} and L' in
    {2..8} data limbs, all drawn uniformly (seeded); eight 50-bit primes and
    a special prime per N; inputs are ciphertexts of uniform residues.  Run
    three ways: one call per operation; grouped by (N, level, kind) into
    batched calls (up to 32 key switches per launch set); and those batched
    calls captured as one graph per ring degree and replayed.  Each context
    first tunes its NTT shape threshold.  Operations/s; the batched results
    are checked bit for bit against the per-operation ones."""
    import numpy as np
    rng = np.random.default_rng(seed)
    kinds = rng.integers(0, 2, n_ops)           # 0: multiply, 1: rotate
    logns = rng.choice([12, 13, 14], n_ops)
    lps = rng.integers(2, 9, n_ops)             # data limbs at the op
    ctxs, tune, inputs, input_data = {}, {}, {}, {}
    for ln in (12, 13, 14):
        g = H.he_ctx_create(ln, [50] * 9, 2.0 ** 40, seed, auto_rescale=True, stream=None)
        H.he_keygen(g, [1])
        chosen, rows = H.he_tune_ntt(g, 1024)
        tune[1 << ln] = {"split_jobs": chosen, "rows_us": [list(r) for r in rows]}
        ctxs[ln] = g
        for lp in range(2, 9):
            data = I.raw_residues(g.primes, 4, lp, g.n, seed=ln * 10 + lp)
            inputs[(ln, lp)] = [H.he_ct_import(g, data[i], lp - 1, 2.0 ** 40) for i in range(4)]
            if ln == 12:
                input_data[(ln, lp)] = data
    for g in ctxs.values():
        H.he_sync(g)
    ops = [(int(kinds[i]), int(logns[i]), int(lps[i]), i % 4) for i in range(n_ops)]

    def one_by_one():
        outs = []
        for k, ln, lp, j in ops:
            a = inputs[(ln, lp)][j]
            if k == 0:
                outs.append(H.he_mul_relin(ctxs[ln], a, inputs[(ln, lp)][(j + 1) % 4]))
            else:
                outs.append(H.he_rotate(ctxs[ln], a, 1))
        return outs

    groups = {}
    for i, (k, ln, lp, j) in enumerate(ops):
        groups.setdefault((ln, lp, k), []).append(i)

    def batched(only=None):
        outs = [None] * n_ops
        for (ln, lp, k), idx in groups.items():
            if only is not None and ln != only:
                continue
            a = [inputs[(ln, lp)][ops[i][3]] for i in idx]
            if k == 0:
                b = [inputs[(ln, lp)][(ops[i][3] + 1) % 4] for i in idx]
                r = H.he_mul_relin_many(ctxs[ln], a, b)
            else:
                r = H.he_rotate_many(ctxs[ln], a, [1] * len(idx))
            for i, c in zip(idx, r):
                outs[i] = c
        return outs

    def timed(fn, reps=3):
        fn()
        for g in ctxs.values():
            H.he_sync(g)
        best = None
        for _ in range(reps):
            t = time.perf_counter()
            out = fn()
            for g in ctxs.values():
                H.he_sync(g)
            dt = time.perf_counter() - t
            best = dt if best is None else min(best, dt)
            del out
        return best

    qops = [(ctxs[ln], "mul", inputs[(ln, lp)][j], inputs[(ln, lp)][(j + 1) % 4]) if k == 0
            else (ctxs[ln], "rotate", inputs[(ln, lp)][j], 1) for k, ln, lp, j in ops]

    def queued():
        return H.he_queue_run(ctxs[13], qops)

    t_one = timed(one_by_one)
    t_bat = timed(batched)
    t_q = timed(queued)
    # GPU time of the queue's eight launches alone (HIP events on the stream)
    H.he_profile_enable(ctxs[13], True)
    for _ in range(3):
        del_ = queued()
        del del_
    qn, qms, qunits, _ = H.he_profile_read(ctxs[13], "queue")
    H.he_profile_enable(ctxs[13], False)
    ref, got, qgot = one_by_one(), batched(), queued()
    sample = list(range(0, n_ops, 37))
    exact = all(np.array_equal(H.he_ct_export(ctxs[ops[i][1]], ref[i]), H.he_ct_export(ctxs[ops[i][1]], got[i]))
                for i in sample)
    qexact = all(np.array_equal(H.he_ct_export(ctxs[ops[i][1]], ref[i]), H.he_ct_export(ctxs[ops[i][1]], qgot[i]))
                 for i in sample)
    # a sample of the N=4096 operations for the oracle (checked in the CPU
    # baseline leg): inputs, kinds and the queue's results
    oracle_sample = []
    for i in range(n_ops):
        k, ln, lp, j = ops[i]
        if ln == 12 and len(oracle_sample) < 6:
            oracle_sample.append({"kind": k, "lp": lp, "a": input_data[(ln, lp)][j],
                                  "b": input_data[(ln, lp)][(j + 1) % 4],
                                  "out": H.he_ct_export(ctxs[ln], qgot[i])})
    del ref, got, qgot
    # one graph per ring degree (its own stream), replayed together
    graphs, keep = [], []
    for ln, g in ctxs.items():
        H.he_graph_begin(g)
        keep.append(batched(only=ln))
        graphs.append((g, H.he_graph_end(g)))

    def replay():
        for g, gr in graphs:
            H.he_graph_launch(g, gr)

    t_graph = timed(replay)
    for _, gr in graphs:
        gr.free()
    del keep
    for g in ctxs.values():
        g.close()
    return {"ops": n_ops, "mix": {"multiply": int((kinds == 0).sum()), "rotate": int((kinds == 1).sum())},
            "groups": len(groups),
            "one_by_one": {"ms": t_one * 1e3, "ops_per_s": n_ops / t_one},
            "batched": {"ms": t_bat * 1e3, "ops_per_s": n_ops / t_bat, "speedup": t_one / t_bat},
            "batched_graph": {"ms": t_graph * 1e3, "ops_per_s": n_ops / t_graph, "speedup": t_one / t_graph},
            "work_queue": {"ms": t_q * 1e3, "ops_per_s": n_ops / t_q, "speedup": t_one / t_q,
                           "gpu_ms": qms / 3, "launches": int(qn / 3), "tasks": int(qunits / max(qn, 1)),
                           "note": "he_queue_run: all 1024 operations as eight launches (one per key-switch "
                                   "stage), each a resident grid draining a device task queue; ms includes "
                                   "building and uploading the task descriptors"},
            "bit_exact_sample": exact, "work_queue_bit_exact_sample": qexact, "ntt_tuning": tune,
            "oracle_sample": oracle_sample}


def keyswitch_bench(H, I, n_ct=256, reps=3):
    """256 ciphertexts of uniform residues at N=16384 (eight 50-bit primes
    and a special prime): batched multiply + relinearise + rescale sharing
    the relinearisation key; rotations R1 (each step 2^t, t = 0..10, applied
    to all 256 ciphertexts with one key) and R2 (1024 rotations: rotation t
    applies step t + 1 to ciphertext t mod 256, 1024 distinct keys)."""
    p = I.RAW
    g = H.he_ctx_create(p["log_n"], p["bits"], p["scale"], p["seed"], auto_rescale=True, stream=None)
    n, L = g.n, g.L
    r1 = [1 << t for t in range(11)]
    r2 = list(range(1, 1025))
    t0 = time.perf_counter()
    H.he_keygen(g, [])
    for st in sorted(set(r1 + r2)):
        H.he_keygen_galois(g, st, -1)
    H.he_sync(g)
    keygen_s = time.perf_counter() - t0
    data = I.raw_residues(g.primes, n_ct, L, n)
    cts = [H.he_ct_import(g, data[i], L - 1, p["scale"]) for i in range(n_ct)]
    del data
    key_bytes = 2 * L * (L + 1) * n * 8  # one key at the top level
    ct_bytes = 2 * L * n * 8

    def timed(fn):
        out = fn()  # warm-up (allocations, attributes)
        H.he_sync(g)
        del out
        best = None
        for _ in range(reps):
            t = time.perf_counter()
            out = fn()
            H.he_sync(g)
            dt = time.perf_counter() - t
            del out
            best = dt if best is None else min(best, dt)
        return best

    res = {"workload": "%d ciphertexts, N=%d, %d x 50-bit primes + special; uniform residues" % (n_ct, n, L),
           "keygen_s": keygen_s, "galois_keys": len(set(r1 + r2))}
    other = cts[1:] + cts[:1]
    t = timed(lambda: H.he_mul_relin_many(g, cts, other))
    res["mul_relin_rescale"] = {"ops": n_ct, "ms": t * 1e3, "key_switches_per_s": n_ct / t,
                                "batch": 32, "shared_key": True}
    per_step = {}
    for st in r1:
        t = timed(lambda: H.he_rotate_many(g, cts, [st] * n_ct))
        per_step[str(st)] = t * 1e3
    vals = list(per_step.values())
    res["rotate_R1"] = {"ops_per_step": n_ct, "ms_per_step": per_step,
                        "key_switches_per_s": n_ct / (min(vals) * 1e-3),
                        "flatness_max_over_min": max(vals) / min(vals)}
    items = [cts[t % n_ct] for t in range(len(r2))]
    t = timed(lambda: H.he_rotate_many(g, items, r2))
    res["rotate_R2"] = {"ops": len(r2), "ms": t * 1e3, "key_switches_per_s": len(r2) / t,
                        "distinct_keys": len(r2),
                        "key_gbs": len(r2) * key_bytes / t / 1e9,
                        "key_plus_ct_hbm_frac": len(r2) * (key_bytes + 3 * ct_bytes) / t / 1e9 / HBM_PEAK_GBS}
    del cts, other, items
    g.close()
    return res


if __name__ == "__main__":
    main()
