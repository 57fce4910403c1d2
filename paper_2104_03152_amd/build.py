"""Build libckks_hip.so in-tree with hipcc for gfx950.

    python -m paper_2104_03152_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libckks_hip.so")
# issue-rate and bandwidth probes (bench.py --probe), outside the library ABI
PROBE_LIB = os.path.join(HERE, "libckks_probe.so")
PROBE_SRC = "probe.hip"
SOURCES = ["ntt.hip", "kernels.hip", "ckks.cpp", "encode.cpp"]
HEADERS = ["modarith.h", "butterfly.h", "device.h", "inner.h", "encode.h"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # packed FP32 instructions are disabled on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    tmpdir = os.path.join(HERE, "_build")
    os.makedirs(tmpdir, exist_ok=True)
    procs = []
    for s in SOURCES:
        o = os.path.join(tmpdir, s + ".o")
        cmd = [hipcc] + [f for f in FLAGS if f != "-shared"] + ["-c", os.path.join(CSRC, s), "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(o)
    failed = []
    for s, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed.append((s, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        for s, t in failed:
            sys.stderr.write("---- %s ----\n%s\n" % (s, t))
        raise RuntimeError("hipcc failed for " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    tmp = PROBE_LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([hipcc] + FLAGS + [os.path.join(CSRC, PROBE_SRC), "-o", tmp],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    os.replace(tmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
