"""Compile the HIP library (gfx950) in-tree: paper_2006_09808_amd/libpd_hip.so.

    python -m paper_2006_09808_amd.build [--jobs N]

Every translation unit under csrc/ is compiled with hipcc in parallel, then
linked into one shared library exporting the C ABI of include/pd.h.
"""

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build", "hip")
LIB = os.path.join(PKG, "libpd_hip.so")
EXAMPLE = os.path.join(PKG, "examples", "pd_solve_file")

ARCH = "gfx950"
CXXFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # packed FP32 instructions are kept out of all generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # a*b+c fuses into an FMA only within one source expression, so the
    # rounding of every update is fixed by the source and not by how the
    # compiler unrolls or schedules a particular tile or team shape
    "-ffp-contract=on",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    "-Wall", "-Wno-unused-function",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def sources():
    out = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".hip") or f.endswith(".cpp"):
            out.append(os.path.join(CSRC, f))
    return out


def _compile(cc, src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [cc] + CXXFLAGS + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    msgs = [l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l]
    return src, obj, p.returncode, "\n".join(msgs)


def build(jobs=None, verbose=False):
    cc = hipcc()
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(16, os.cpu_count() or 4, len(srcs))
    t0 = time.time()
    objs = []
    failed = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for src, obj, rc, msg in ex.map(lambda s: _compile(cc, s), srcs):
            if rc != 0:
                failed.append((src, msg))
            elif verbose and msg.strip():
                print(msg, file=sys.stderr)
            objs.append(obj)
    if failed:
        for src, msg in failed:
            print("hipcc failed for %s:\n%s" % (src, msg), file=sys.stderr)
        raise RuntimeError("HIP build failed (%d translation units)" % len(failed))
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-Wl,--no-undefined"]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout)
    os.replace(tmp, LIB)
    # the C-ABI example program, linked against the library just built
    ex_src = os.path.join(PKG, "examples", "pd_solve_file.cpp")
    if os.path.exists(ex_src):
        cmd = [cc] + CXXFLAGS + [ex_src, "-o", EXAMPLE, "-L" + PKG, "-l:libpd_hip.so", "-Wl,-rpath,$ORIGIN/.."]
        p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if p.returncode != 0:
            raise RuntimeError("example build failed:\n" + p.stdout)
    if verbose:
        print("built %s from %d units in %.1f s" % (LIB, len(srcs), time.time() - t0), file=sys.stderr)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args()
    build(a.jobs, verbose=True)
