"""Build the HIP library (libgamma.so) for gfx950 in-tree with hipcc.

Every source under csrc/ is compiled with --offload-arch=gfx950 and linked
into paper_2401_17018_amd/libgamma.so.  Packed-FP32 instructions are
disabled for all device code.

`python build.py --profile` builds libgamma_prof.so beside it instead: the
same library with GM_DFS_PROFILE=1, whose search kernel also splits its
wave-cycles into idle, level set-up, inner levels, last level and
hand-over (the cyc_* batch statistics).  Nothing loads it unless asked
(bench.py --library).
"""
from __future__ import annotations

import concurrent.futures
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libgamma.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(HERE, "..", "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


# kernels whose register use is recorded at build time (resources.json):
# the search kernel must keep three waves per SIMD without spilling
WATCH = {"k_dfs.hip"}


def _resources(stderr: str) -> dict:
    """Per-kernel figures from hipcc's kernel-resource-usage remarks."""
    out, cur = {}, None
    keys = {"VGPRs": "vgprs", "AGPRs": "agprs", "ScratchSize [bytes/lane]": "scratch_bytes",
            "Occupancy [waves/SIMD]": "occupancy", "VGPRs Spill": "vgpr_spill", "SGPRs Spill": "sgpr_spill",
            "LDS Size [bytes/block]": "lds_bytes"}
    for line in stderr.splitlines():
        if "remark:" not in line:
            continue
        body = line.split("remark:", 1)[1].split("[-Rpass")[0].strip()
        if body.startswith("Function Name:"):
            cur = body.split(":", 1)[1].strip()
            out[cur] = {}
        elif cur and ":" in body:
            name, val = body.rsplit(":", 1)
            if name.strip() in keys:
                try:
                    out[cur][keys[name.strip()]] = int(val.strip())
                except ValueError:
                    pass
    return out


def _compile(src: str, bdir: str = BUILD_DIR, extra=()) -> str:
    obj = os.path.join(bdir, os.path.basename(src) + ".o")
    cmd = ["hipcc"] + COMMON + DEVICE + list(extra)
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    watch = os.path.basename(src) in WATCH
    if watch:
        cmd += ["-Rpass-analysis=kernel-resource-usage"]
    cmd += ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-6000:]))
    if watch:
        with open(os.path.join(bdir, os.path.basename(src) + ".resources.json"), "w") as f:
            json.dump(_resources(r.stderr), f, indent=1)
    return obj


def build(verbose: bool = False, profile: bool = False) -> str:
    out = os.path.join(HERE, "libgamma_prof.so") if profile else OUT
    bdir = BUILD_DIR + ("_prof" if profile else "")
    extra = ["-DGM_DFS_PROFILE=1"] if profile else []
    os.makedirs(bdir, exist_ok=True)
    srcs = sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, bdir, extra), srcs))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-6000:])
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True, profile="--profile" in sys.argv[1:])
    sys.exit(0)
