"""Build libsvconv.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1209_5823_amd.build        # or build() from Python

Every csrc/*.hip is compiled to an object under _build/ (in parallel), then
linked into paper_1209_5823_amd/libsvconv.so.  Importing the package loads
that library; nothing is compiled at import time.

The compiler's resource-usage report of every kernel is checked: a kernel
that spills registers to scratch memory fails the build, and the report is
kept in _build/resource_usage.json.
"""

import concurrent.futures
import json
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsvconv.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC,
    # no packed-FP32 VALU instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
# Per-file additions.  separable*.hip: the kernels fold up to four column
# factors of one parity on the same pair sums, in variants chosen at run time;
# machine CSE merges the pair sums of the variants ahead of the branch, and
# machine LICM and common-code hoisting lift them further, which keeps every
# pair sum of the window live at once and spills registers.
_SEP_FLAGS = ["-mllvm", "-disable-machine-cse", "-mllvm", "-disable-machine-licm",
              "-mllvm", "-simplifycfg-hoist-common=false"]
FILE_FLAGS = {"separable.hip": _SEP_FLAGS, "separable_adjoint.hip": _SEP_FLAGS}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _resource_usage(stderr):
    """{kernel: {"vgprs", "agprs", "scratch", "lds"}} from the resource-usage remarks."""
    usage, name = {}, None
    for line in stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            usage[name] = {}
            continue
        for key, pat in (("vgprs", r" VGPRs: (\d+)"), ("agprs", r" AGPRs: (\d+)"),
                         ("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"),
                         ("lds", r"LDS Size \[bytes/block\]: (\d+)")):
            m = re.search(pat, line)
            if m and name:
                usage[name][key] = int(m.group(1))
    return usage


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ([HIPCC] + FLAGS + FILE_FLAGS.get(os.path.basename(src), [])
           + ["-Rpass-analysis=kernel-resource-usage", "-c", src, "-o", obj])
    r = subprocess.run(cmd, capture_output=True, text=True)
    usage = _resource_usage(r.stderr)
    # the host pass does not know the packed-fp32 feature; that warning is
    # expected, and the resource-usage remarks are parsed, not shown
    err = "\n".join(l for l in r.stderr.splitlines()
                    if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l
                    and not re.match(r"\s*\d+ \|", l) and not re.match(r"\s*\|\s*\^", l))
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, err))
    return obj, err, usage


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    # a failed build leaves no library behind, so nothing loads a stale one
    if os.path.exists(LIB):
        os.remove(LIB)
    srcs = sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    usage = {}
    for obj, err, u in results:
        if err.strip() and verbose:
            print(err, file=sys.stderr)
        usage.update(u)
    with open(os.path.join(BUILD, "resource_usage.json"), "w") as f:
        json.dump(usage, f, indent=1, sort_keys=True)
    spills = {k: v["scratch"] for k, v in usage.items() if v.get("scratch", 0) > 0}
    if spills:
        raise RuntimeError("kernels spill registers to scratch memory (bytes per lane): %s" % spills)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for o, _, _ in results]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
