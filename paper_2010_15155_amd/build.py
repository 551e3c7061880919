"""Build ``libstkfmm.so`` in-tree: HIP sources with hipcc for gfx950, host
sources with g++, linked by hipcc.  Always recompiles when called."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libstkfmm.so")
ARCH = os.environ.get("STKFMM_ARCH", "gfx950")

HIP_SOURCES = ["kernels.hip", "api.hip", "mlp.hip", "wall.hip", "tree_gpu.hip", "periodic.hip"]
CPP_SOURCES = ["tree.cpp", "operators.cpp", "learn.cpp", "opcache.cpp"]
# the sources that compute the cached operators: their hash names the cache
# files, so a library built from changed operator code ignores older files
OPERATOR_SOURCES = ["operators.cpp", "internal.hpp", "pool.hpp", "opcache.cpp"]
HIP_FLAGS = ["-O3", "--offload-arch=" + ARCH, "-std=c++17", "-fPIC", "-Wall",
             # no packed FP32 instructions (v_pk_*_f32) anywhere
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
CPP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-pthread", "-I/opt/rocm/include"]


def _run(cmds, verbose):
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for cmd, p in procs:
        out, _ = p.communicate()
        text = "\n".join(l for l in out.decode(errors="replace").splitlines()
                         if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
        if p.returncode != 0:
            failed.append((cmd, text))
        elif verbose and text.strip():
            print(text, file=sys.stderr)
    if failed:
        msg = "\n\n".join(" ".join(c) + "\n" + t for c, t in failed)
        raise RuntimeError("build failed:\n" + msg)


def operator_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in OPERATOR_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs, cmds = [], []
    cpp_flags = CPP_FLAGS + ['-DKAFMM_OPS_SOURCE_HASH="%s"' % operator_source_hash()]
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        cmds.append(["hipcc"] + HIP_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    for s in CPP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        cmds.append(["g++"] + cpp_flags + ["-c", os.path.join(CSRC, s), "-o", o])
    _run(cmds, verbose)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-pthread", "-o", tmp] + objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
