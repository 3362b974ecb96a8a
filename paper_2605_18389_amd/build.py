"""Build libshot.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2605_18389_amd.build   (or build() from Python).
The shared library lands next to this file and is what the Python binding loads.
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OUT = os.path.join(HERE, "libshot.so")
BUILD_DIR = os.path.join(HERE, "_build")

ARCH = os.environ.get("SHOT_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]
# Device code: gfx950 only.  Packed-FP32 VALU forms are disabled (they are
# emitted automatically from scalar float code otherwise).
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

SOURCES = [
    ("host_math.cpp", False),
    ("api.cpp", True),
    ("kernels.hip", True),
]


HASHED = ["api.cpp", "host_math.cpp", "host_math.h", "shot_internal.h", "kernels.hip"]


def source_hash():
    """Hash of everything libshot.so is built from: the C/HIP sources, the
    public header and the compile flags.  Stored in the library at build time
    (shot_build_id) and compared by the loader, which refuses a stale build."""
    import hashlib
    hs = hashlib.sha256()
    for name in HASHED:
        with open(os.path.join(CSRC, name), "rb") as f:
            hs.update(name.encode() + b"\0" + f.read() + b"\0")
    with open(os.path.join(INCLUDE, "shot.h"), "rb") as f:
        hs.update(b"shot.h\0" + f.read() + b"\0")
    hs.update(" ".join(COMMON[:5] + DEVICE + [ARCH]).encode())
    return hs.hexdigest()[:24]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=None):
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    procs = []
    build_id = source_hash()
    for src, is_hip in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc] + COMMON + [f'-DSHOT_SOURCE_HASH="{build_id}"']
        if is_hip:
            cmd += ["-x", "hip"] + DEVICE
        cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((src, out.decode(errors="replace")))
        elif verbose and out:
            print(out.decode(errors="replace"))
    if failed:
        msg = "\n".join(f"--- {s} ---\n{o}" for s, o in failed)
        raise RuntimeError("libshot build failed:\n" + msg)
    tmp = OUT + ".tmp"
    cmd = [hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("libshot link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
