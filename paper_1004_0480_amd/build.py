"""Build librdmi.so: the HIP kernels and the C ABI, for gfx950, in-tree.

Each translation unit compiles to an object under ``_build/`` (in parallel),
then hipcc links them into ``paper_1004_0480_amd/librdmi.so``.
"""
import hashlib
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librdmi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# -ffp-contract=off: every kernel variant rounds each operation the same way,
# so all plans give bitwise-identical fields.  Packed FP32 instructions are
# disabled.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


_INCLUDE_RE = re.compile(r'^\s*#\s*include\s+"([^"]+)"', re.M)


def _includes(path, seen):
    """Transitive project headers of a source file (quoted includes found in
    csrc/ or include/)."""
    with open(path, "rb") as fh:
        text = fh.read().decode("utf-8", "replace")
    for name in _INCLUDE_RE.findall(text):
        for d in (CSRC, INCLUDE):
            cand = os.path.join(d, name)
            if os.path.exists(cand) and cand not in seen:
                seen.add(cand)
                _includes(cand, seen)
                break
    return seen


def source_digest() -> str:
    """Hash of every kernel and engine source under csrc/: what the library
    is built from.  Baked into the library (rd_source_digest) so that a
    loaded binary can be matched with the sources beside it."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hpp", ".hip")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def _flags(src):
    f = list(FLAGS)
    if os.path.basename(src) == "rd_engine.hip":
        f += ["-DRD_SOURCE_DIGEST=\"%s\"" % source_digest()]
    return f


def _digest(src):
    """Object key: the flags, the source and the project headers it includes."""
    h = hashlib.sha256()
    h.update(" ".join(_flags(src)).encode())
    for path in [src] + sorted(_includes(src, set())):
        with open(path, "rb") as fh:
            h.update(path.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src, force, verbose):
    os.makedirs(BUILD, exist_ok=True)
    obj = os.path.join(BUILD, os.path.basename(src) + "." + _digest(src) + ".o")
    if os.path.exists(obj) and not force:
        return obj
    cmd = [HIPCC] + _flags(src) + ["-c", src, "-o", obj + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, err))
    os.replace(obj + ".tmp", obj)
    return obj


def build(force: bool = True, verbose: bool = False, jobs: int = 0) -> str:
    """Compile every translation unit (all of them when ``force``) and link."""
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force, verbose), sources()))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv, verbose="-v" in sys.argv))
