"""Encrypted-CNN inference benchmark on one MI355X.

One step = one encrypted inference of the MNIST-shaped network of the paper's
section 5 (conv 4 kernels 7x7 stride 3 -> pack -> square -> FC 256->64 ->
square -> FC 64->10) at N = 8192 with an 8-prime chain (60, 40 x 6, 60 bits)
and scale 2^40, on an input ciphertext already resident in HBM, with the
weights pre-encoded on the device (plans).  Every step runs the whole GPU
path: NTT/INTT, pointwise products, key switching (ModUp, inner product,
ModDown) for 357 rotations/relinearisations, automorphisms and rescales.

Prints one JSON line (see the field list at the bottom).  --gpus N with N > 1
exits: this build measures one GPU.
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


def cnn_fp64(d, im2col):
    v = im2col(d["img"], 7, 3).reshape(49, 64)
    conv = d["conv_k"] @ v + d["conv_b"][:, None]
    x = conv.reshape(256) ** 2
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--latency-runs", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=8.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(requests/ciphertexts would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    log("importing torch")
    import torch
    import paper_2104_03152_amd as H
    from paper_2104_03152_amd import inputs as I

    assert torch.cuda.is_available(), "needs a GPU"
    params = I.CNN
    shape = I.CNN_SHAPE
    d = I.cnn_inputs()
    log("context + keys")
    t0 = time.perf_counter()
    g = H.he_ctx_create(params["log_n"], params["bits"], params["scale"], params["seed"],
                        auto_rescale=True)
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
    t0 = time.perf_counter()
    for _ in range(args.steps):
        y = step(H, g, net, x, shape["windows"])
    H.he_sync(g)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    out = H.he_ct_export(g, y)
    bit_exact_repeat = bool(np.array_equal(out, ref))
    logits = H.he_decode(g, H.he_decrypt(g, y), shape["out"])
    logits_err = float(np.abs(logits - cnn_fp64(d, H.he_im2col)).max())

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
    fams = ["ntt_fwd", "ntt_inv", "modup", "moddown", "keyswitch_inner", "hoisted_inner",
            "hoisted_moddown", "pointwise", "rescale", "sample"]
    H.he_profile_enable(g, True)
    prof_steps = 5
    for _ in range(prof_steps):
        step(H, g, net, x, shape["windows"])
    H.he_sync(g)
    prof = {}
    for f in fams:
        n, ms = H.he_profile_read(g, f)
        if n:
            prof[f] = {"launches_per_step": n / prof_steps, "ms_per_step": ms / prof_steps,
                       "avg_launch_us": 1e3 * ms / n}
    H.he_profile_enable(g, False)

    # roofline of the dominant kernel family (largest summed time per step)
    dom = max(prof, key=lambda k: prof[k]["ms_per_step"]) if prof else None
    roof = None
    if dom:
        roof = roofline_entry(dom, prof[dom], g.n)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        rate, n_inf, cdt, oy = cpu_baseline(params, d, args.cpu_budget)
        cpu = {"value": rate, "unit": "inferences/s", "cores": 1, "kind": "oracle",
               "sample": "%d full encrypted inference(s) of the same network, %.1f s, single "
                         "thread, keys generated outside the timing" % (n_inf, cdt),
               "bit_exact_vs_gpu": bool(np.array_equal(oy.data(), ref))}

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
        "kernel_profile": prof,
        "roofline": roof,
        "cpu_baseline": cpu,
        "bit_exact_repeat": bit_exact_repeat,
        "logits_max_abs_err": logits_err,
        "keygen_s": keygen_s,
        "paper_context": "TenSEAL on AWS c4.4xlarge (16 vCPU Xeon E5-2666 v3): 887.06 ms full "
                         "forward at N=8192, 206-bit modulus, scale 2^21 (table 2); context only",
    }
    print(json.dumps(res), flush=True)


# Algorithmic HBM bytes per launch of each kernel family at ring degree n,
# from the per-unit figures (one limb = 8n bytes) and the units per launch
# recorded by the profile.  Filled in by roofline_entry.
def roofline_entry(fam, p, n):
    limb = 8.0 * n
    # per launch: a batched NTT reads and writes each limb once
    units = p.get("limbs_per_launch")
    if units is None:
        return {"bound": "alu", "family": fam, "avg_launch_us": p["avg_launch_us"],
                "achieved": None, "peak": None, "unit": None, "frac": None, "traffic": None}
    bytes_ = 2 * limb * units
    ach = bytes_ / (p["avg_launch_us"] * 1e-6) / 1e9
    return {"bound": "hbm", "family": fam, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None}


if __name__ == "__main__":
    main()
