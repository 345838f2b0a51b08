"""Build libsq.so (HIP, gfx950) in-tree with hipcc.

Every HIP source under csrc/ is compiled to an object in _build/ (in
parallel) and linked into paper_2011_13517_amd/libsq.so.  Packed-FP32
instructions are disabled for all device code.

A variant build for A/B measurements (``python -m paper_2011_13517_amd.build
--define A64_MFMA_DOTS=1 --name mfma``) compiles with extra macro definitions
into _build_<name>/ and links libsq_<name>.so beside the default library;
the Python binding loads it when SQ_LIB names it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsq.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-Wall"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src, build_dir=BUILD, extra=()):
    obj = os.path.join(build_dir, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC] + FLAGS + list(extra) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose: bool = True, defines=(), name: str = "") -> str:
    if name and not name.replace("_", "").isalnum():
        raise ValueError(f"variant name {name!r}: letters, digits and '_' only")
    for d in defines:
        if not d.split("=", 1)[0].replace("_", "").isalnum():
            raise ValueError(f"macro definition {d!r}: NAME or NAME=VALUE")
    build_dir = BUILD + (f"_{name}" if name else "")
    lib = LIB[:-3] + f"_{name}.so" if name else LIB
    extra = ["-D" + d for d in defines]
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, extra), srcs))
    tmp = lib + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}", file=sys.stderr)
    return lib


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--define", action="append", default=[], metavar="NAME=VALUE",
                    help="extra macro definition (variant builds)")
    ap.add_argument("--name", default="", help="variant name: libsq_<name>.so")
    args = ap.parse_args()
    if args.define and not args.name:
        ap.error("a build with --define needs --name (the default library stays as built)")
    build(defines=args.define, name=args.name)
