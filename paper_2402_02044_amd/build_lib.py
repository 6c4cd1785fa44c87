"""Build liblvq.so (the gfx950 HIP library) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "liblvq.so")

SOURCES = ["lvq_host.hip", "k_encode.hip", "k_misc.hip", "k_cand4.hip", "k_cand8.hip",
           "k_scan4.hip", "k_scan8.hip", "k_mfma.hip", "k_mfma_full.hip", "k_mfma_wide.hip", "k_mfma_wide32.hip",
           "k_mfma_wide32r.hip", "k_mfma_wide16r.hip",
           "lvq_serve.hip", "k_probe.hip", "k_graph.hip",
           "lvq_noalloc.hip"]
# binary32 encoding must round every operation on its own
EXTRA = {"k_encode.hip": ["-ffp-contract=off"], "k_probe.hip": ["-ffp-contract=off"]}

ARCH = os.environ.get("LVQ_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-Wall", "-Wno-unused-function",
         # packed FP32 instructions are kept out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def _newest_header() -> float:
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hdrs.append(os.path.join(os.path.dirname(HERE), "include", "lvq.h"))
    return max(os.path.getmtime(h) for h in hdrs)


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    if incremental and os.path.exists(obj) and \
            os.path.getmtime(obj) > max(os.path.getmtime(os.path.join(CSRC, src)), _newest_header()):
        return obj
    cmd = [_hipcc()] + FLAGS + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    if out.strip():
        sys.stderr.write(out + "\n")
    return obj


def build(jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every source (incremental: only those older than their object
    file and the headers are reused) and link liblvq.so."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(8, len(srcs))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "-shared", "-fPIC", "-pthread", "--offload-arch=" + ARCH] + objs + ["-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(incremental="--incremental" in sys.argv))
