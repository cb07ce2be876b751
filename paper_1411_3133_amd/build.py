"""Build libmlbm.so for gfx950 in-tree with hipcc.

Each translation unit is compiled in parallel, then linked into one shared
library next to this file.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmlbm.so")
SOURCES = ["step.hip", "step_eq.hip", "aux.hip", "api.hip", "mlp.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions (some of their forms are unreliable here)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(HERE, "..", "include"),
]


def _up_to_date(obj: str, src: str) -> bool:
    """The object is newer than its source, every header and the flags."""
    if not os.path.exists(obj):
        return False
    deps = [src, __file__] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    deps.append(os.path.join(HERE, "..", "include", "mlbm.h"))
    return all(os.path.getmtime(obj) >= os.path.getmtime(d) for d in deps)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (or, with incremental, only those whose object is
    out of date) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        if incremental and _up_to_date(obj, os.path.join(CSRC, src)):
            continue
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = "\n".join(l for l in out.decode(errors="replace").splitlines()
                         if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed.append(src)
            print(text, file=sys.stderr, flush=True)
        elif verbose and text.strip():
            print(text, flush=True)
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs + \
          ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


# The runtime sanitizer driver (tests/native/api_sanitize.cpp): the host
# code of the runtime sources with AddressSanitizer and UndefinedBehavior-
# Sanitizer (host compilation only; the GPU code is built as usual), linked
# with the ordinary kernel objects of build().
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
SANITIZED = ["api.hip", "mlp.hip"]
DRIVER_SRC = os.path.join(HERE, "..", "tests", "native", "api_sanitize.cpp")
DRIVER = os.path.join(HERE, "api_sanitize")   # next to the library: it ships to the GPU with it


def build_sanitized(verbose: bool = False) -> str:
    objs = [os.path.join(BUILD, s.replace(".hip", ".o")) for s in SOURCES if s not in SANITIZED]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise RuntimeError("build() first: missing " + ", ".join(missing))
    cmds = []
    for src in SANITIZED:
        obj = os.path.join(BUILD, "asan_" + src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([HIPCC] + FLAGS + SANITIZE + ["-c", os.path.join(CSRC, src), "-o", obj])
    drv = os.path.join(BUILD, "asan_driver.o")
    objs.append(drv)
    cmds.append([HIPCC, "-x", "c++", "-std=c++17", "-O1"] + SANITIZE + ["-c", DRIVER_SRC, "-o", drv])
    procs = [(c, subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)) for c in cmds]
    for c, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            print(out.decode(errors="replace"), file=sys.stderr, flush=True)
            raise RuntimeError("hipcc failed: " + " ".join(c))
        if verbose:
            print(" ".join(c), flush=True)
    cmd = [HIPCC, "--offload-arch=gfx950", "-o", DRIVER] + objs + SANITIZE[:4] + \
          ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return DRIVER


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv)
    if "--sanitized" in sys.argv:
        build_sanitized(verbose="-v" in sys.argv)
