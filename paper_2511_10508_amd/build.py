"""Build libpfmi.so in-tree: hipcc for gfx950, one object per source, in parallel.

    python -m paper_2511_10508_amd.build          # or build() from Python
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpfmi.so")
OBJ = os.path.join(os.path.dirname(HERE), "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

# -ffp-contract=off: only the explicit fma() calls fuse, so every kernel
# family evaluates a site bit for bit the same way.  Packed FP32 ops stay off.
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


def _stale(src, obj):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "pfmi.h"))
    return any(os.path.getmtime(d) > t for d in deps)


def _compile(src, force=True):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    if not force and not _stale(src, obj):
        return obj, ""
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if res.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (src, msgs))
    return obj, msgs


def build(jobs=None, verbose=False, force=True):
    """Compile every source and link paper_2511_10508_amd/libpfmi.so.

    force=True (the default) recompiles everything; force=False only sources
    older than their object or than any header."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(os.cpu_count() or 1, 16)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, force), srcs))
    if verbose:
        for _, msgs in results:
            if msgs:
                print(msgs)
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + \
          [o for o, _ in results] + ["-L" + os.path.join(ROCM, "lib"), "-lhipfft",
                                     "-lrocprofiler-sdk-roctx",
                                     "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="--incremental" not in sys.argv))
