"""Build libtstream.so for gfx950 with hipcc (works without a GPU).

    python paper_2206_06302_amd/build.py            # rebuild everything
    python paper_2206_06302_amd/build.py --if-stale # only when sources changed

(Run by path: importing the package itself loads the library.)

Every translation unit is compiled with -ffp-contract=off (no contraction
beyond the explicit fma of the triad), without fast-math, and with the
packed-FP32 instructions disabled; exported symbols are the ts_* functions of
include/tstream.h only (-fvisibility=hidden elsewhere).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtstream.so")
ARCH = os.environ.get("TS_OFFLOAD_ARCH", "gfx950")

SOURCES = ["kern_f64.hip", "kern_f32.hip", "kern_bf16.hip", "kern_f16.hip", "kern_aux.hip", "kern_probe.hip",
           "capi.cpp", "capi_probe.cpp", "capi_tune.cpp", "capi_batch.cpp", "capi_async.cpp", "tune.cpp", "host_target.cpp",
           "transform.cpp", "host_transform.cpp"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
    "-fvisibility=hidden", "-Wall", "-Wextra", "-Wno-unused-parameter",
    "-I" + INCLUDE, "-I" + CSRC,
]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libtstream)")


def _inputs():
    return [os.path.join(CSRC, s) for s in SOURCES] + glob.glob(os.path.join(CSRC, "*.hpp")) + \
        [os.path.join(INCLUDE, "tstream.h"), os.path.join(CSRC, "libtstream.map")]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in _inputs())


def _compile(cc: str, src: str, obj: str) -> None:
    cmd = [cc, *COMMON, *DEVICE]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", src, "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
    if out.strip():
        print(out, file=sys.stderr)


def build(jobs: int | None = None, verbose: bool = False) -> str:
    cc = hipcc()
    jobs = jobs or min(8, os.cpu_count() or 4)
    with tempfile.TemporaryDirectory(prefix="tstream_build_") as tmp:
        objs = [os.path.join(tmp, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            futs = [ex.submit(_compile, cc, os.path.join(CSRC, s), o) for s, o in zip(SOURCES, objs)]
            for f in futs:
                f.result()
        tmp_lib = LIB + ".tmp%d" % os.getpid()
        cmd = [cc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp_lib, *objs,
               "-Wl,-rpath,/opt/rocm/lib", "-Wl,--no-undefined",
               "-Wl,--version-script=" + os.path.join(CSRC, "libtstream.map"), "-ldl"]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}")
        os.replace(tmp_lib, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--if-stale", action="store_true")
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args()
    if a.if_stale and not stale():
        print("up to date:", LIB)
        return
    build(a.j, verbose=True)


if __name__ == "__main__":
    main()
