"""Continuous-batching request loop over the C ABI: encrypted inference
requests of two kinds share one GPU.

- Clients.  Each client owns a context (its own key set, resident in device
  memory, and its own stream, so different clients' work overlaps on the
  GPU) and serves up to 16 requests.
- Requests.  `cnn`: the MNIST-shaped network of section 5 (conv, pack,
  square, FC1, square, FC2) on an encrypted im2col image.  `lr`: encrypted
  logistic-regression scoring, the dot product of section 3.1 (multiply by
  the plain weights, slot sum by rotations, add the bias).
- Admission.  A request enters service only while the ciphertext working
  sets of the requests in service fit in a device-memory budget (key sets
  are admitted with their client); the others wait in arrival order.
- Continuous batching.  Each scheduling round advances every request in
  service by one stage; requests at the same stage run as one batched call
  where the library has one, across clients (squares: he_mul_relin_across;
  the rotations of the slot sums: he_rotate_across), so their key switches
  share launches, each item with its own client's keys.  Requests that
  arrive while others are on the GPU join the next round.
- One-at-a-time.  The baseline serves requests strictly in arrival order,
  each to completion, on the same contexts.

Every result is the same ciphertext whether a request is served alone or in
a mix (the batched calls are bit-identical to the single ones).
"""
import collections
import time

import numpy as np

from . import inputs as I

CNN_BITS = [60, 40, 40, 40, 40, 40, 40, 60]
SCALE = 2.0 ** 40
REQS_PER_CLIENT = 16
# device working set per request in service (its ciphertexts and key-switch
# intermediates), the admission unit besides the key sets
WORKSET = {"cnn": 96 << 20, "lr": 16 << 20}


def lr_steps(d):
    return [1 << t for t in range(max(1, int(np.ceil(np.log2(d)))))]


class Client:
    """One key set: context, keys for the CNN and for slot sums of up to
    1024 values, and the CNN's plans."""

    def __init__(self, H, cid, net_weights):
        self.H, self.cid = H, cid
        g = H.he_ctx_create(13, CNN_BITS, SCALE, 1000 + cid, auto_rescale=True, stream=None)
        self.g = g
        H.he_keygen(g, [])
        levels = dict(I.cnn_rotation_steps())
        for st in lr_steps(1024):
            levels[st] = max(levels.get(st, -1), g.L - 2)
        for st, lv in sorted(levels.items()):
            H.he_keygen_galois(g, st, lv)
        self.key_bytes = H.he_key_bytes(g)
        d = net_weights
        s = I.CNN_SHAPE
        v = H.he_im2col(d["img"], s["k"], s["stride"])
        x = H.he_encrypt(g, H.he_encode(g, v, SCALE, g.L - 1), 0, False)
        conv = [H.he_conv_plan(g, x, d["conv_k"][c], s["windows"], d["conv_b"][c])
                for c in range(s["channels"])]
        parts = H.he_plan_apply_many(g, conv, x)
        s1 = H.he_square(g, H.he_pack(g, parts, s["windows"]))
        fc1 = H.he_matmul_plan(g, s1, d["w1"], d["b1"])
        s2 = H.he_square(g, H.he_plan_apply(g, fc1, s1))
        fc2 = H.he_matmul_plan(g, s2, d["w2"], d["b2"])
        H.he_plan_apply(g, fc2, s2)  # every plan applied once (device tables built)
        H.he_sync(g)
        self.plans = (conv, fc1, fc2)

    def close(self):
        self.plans = None
        self.g.close()


class Request:
    def __init__(self, rid, kind, client, arrival, ct, extra):
        self.rid, self.kind, self.client, self.arrival = rid, kind, client, arrival
        self.ct = ct          # the encrypted input (device resident)
        self.extra = extra    # lr: (d, weights plaintext, bias plaintext)
        self.stage = 0
        self.x = ct
        self.done = None
        self.out = None


# stages per kind: the last one produces the result
CNN_STAGES = ("conv", "pack", "square1", "fc1", "square2", "fc2")
LR_STAGES = ("mul", "sum", "bias")


def make_requests(H, clients, n, qps, seed, cnn_frac=0.5, per_client=REQS_PER_CLIENT):
    """n requests with Poisson arrivals at the given rate (all at once for
    qps = 0); request i belongs to client i // per_client; inputs are
    encrypted ahead (the client's upload) and LR weights encoded ahead."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, n) if qps > 0 else np.zeros(n)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    s = I.CNN_SHAPE
    for i in range(n):
        c = clients[(i // per_client) % len(clients)]
        g = c.g
        if rng.uniform() < cnn_frac:
            img = rng.uniform(0, 1, (28, 28))
            v = H.he_im2col(img, s["k"], s["stride"])
            ct = H.he_encrypt(g, H.he_encode(g, v, SCALE, g.L - 1), 10_000 + i, False)
            reqs.append(Request(i, "cnn", c, float(arrivals[i]), ct, {"img": img}))
        else:
            d = int(rng.integers(64, 1025))
            w, b = rng.normal(0, 1, d), float(rng.normal(0, 1))
            xv = rng.uniform(-1, 1, d)
            ct = H.he_encrypt(g, H.he_encode(g, xv, SCALE, g.L - 1), 10_000 + i, False)
            wp = H.he_encode(g, w, SCALE, g.L - 1)
            # the product rescales by the top data prime: the bias goes at that scale
            out_scale = SCALE * SCALE / g.primes[g.L - 1]
            bvec = np.zeros(g.n // 2)
            bvec[0] = b
            bp = H.he_encode(g, bvec, out_scale, g.L - 2)
            reqs.append(Request(i, "lr", c, float(arrivals[i]), ct,
                                {"d": d, "w": w, "b": b, "x": xv, "wp": wp, "bp": bp}))
    for c in clients:
        H.he_sync(c.g)
    return reqs


def _advance(H, kind, stage, reqs):
    """Run one stage for requests at the same stage (of one or several
    clients): the key switches of squares and slot-sum rotations run as one
    batch across the requests, each on its own client's keys."""
    s = I.CNN_SHAPE
    run = reqs[0].client.g
    if kind == "cnn":
        name = CNN_STAGES[stage]
        if name in ("square1", "square2"):
            outs = H.he_mul_relin_across(run, [r.x for r in reqs], [r.x for r in reqs])
            for r, o in zip(reqs, outs):
                r.x = o
        else:
            for r in reqs:
                g = r.client.g
                conv, fc1, fc2 = r.client.plans
                if name == "conv":
                    r.x = H.he_plan_apply_many(g, conv, r.x)
                elif name == "pack":
                    r.x = H.he_pack(g, r.x, s["windows"])
                elif name == "fc1":
                    r.x = H.he_plan_apply(g, fc1, r.x)
                else:
                    r.x = H.he_plan_apply(g, fc2, r.x)
        return stage + 1 == len(CNN_STAGES)
    name = LR_STAGES[stage]
    if name == "mul":
        for r in reqs:
            r.x = H.he_mul_plain(r.client.g, r.x, r.extra["wp"])
    elif name == "sum":
        # slot sums of different lengths: step j rotates every request that
        # still needs it, in one batched call
        steps = {r.rid: lr_steps(r.extra["d"]) for r in reqs}
        for j in range(max(len(v) for v in steps.values())):
            act = [r for r in reqs if j < len(steps[r.rid])]
            rots = H.he_rotate_across(run, [r.x for r in act], [steps[r.rid][j] for r in act])
            for r, o in zip(act, rots):
                r.x = H.he_add(r.client.g, r.x, o)
    else:
        for r in reqs:
            r.x = H.he_add_plain(r.client.g, r.x, r.extra["bp"])
    return stage + 1 == len(LR_STAGES)


def serve(H, reqs, budget_bytes, batched=True):
    """Serve the requests (arrival times relative to the start) and return
    per-request latency in ms.  batched=False serves them one at a time."""
    pending = collections.deque(sorted(reqs, key=lambda r: r.arrival))
    active = []
    used = 0
    t0 = time.perf_counter()
    lat = {}
    while pending or active:
        now = time.perf_counter() - t0
        if batched:
            while pending and pending[0].arrival <= now and used + WORKSET[pending[0].kind] <= budget_bytes:
                r = pending.popleft()
                used += WORKSET[r.kind]
                active.append(r)
        elif not active and pending and pending[0].arrival <= now:
            r = pending.popleft()
            active.append(r)
        if not active:
            wait = pending[0].arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.002))
            continue
        groups = collections.OrderedDict()
        for r in active:
            groups.setdefault((r.kind, r.stage), []).append(r)
        finished = []
        for (kind, stage), rs in groups.items():
            last = _advance(H, kind, stage, rs)
            for r in rs:
                r.stage += 1
                if last:
                    finished.append(r)
        if finished:
            for cid in sorted({r.client.cid for r in finished}):
                H.he_sync(next(r.client for r in finished if r.client.cid == cid).g)
            t = time.perf_counter() - t0
            for r in finished:
                r.done = t
                r.out = r.x
                lat[r.rid] = (t - r.arrival) * 1e3
                active.remove(r)
                if batched:
                    used -= WORKSET[r.kind]
    return lat


def reset(reqs):
    for r in reqs:
        r.stage, r.x, r.done, r.out = 0, r.ct, None, None


def summary(lat, reqs):
    v = np.array([lat[r.rid] for r in reqs])
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return {"p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99)),
            "inferences_per_s": len(reqs) / span if span > 0 else None, "requests": len(reqs)}
