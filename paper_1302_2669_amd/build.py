"""Builds libmcmcdec.so (the HIP kernels and the C-ABI) for gfx950, in-tree.

Every translation unit is compiled with hipcc in parallel and linked into
paper_1302_2669_amd/libmcmcdec.so.  `python -m paper_1302_2669_amd.build`
rebuilds unconditionally.
"""

import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmcmcdec.so")
ARCH = os.environ.get("MCMC_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return path


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src, obj):
    cmd = [hipcc()] + COMMON + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def _includes(path, seen):
    """The project files `path` includes (quoted includes, transitively)."""
    if path in seen or not os.path.exists(path):
        return
    seen.add(path)
    with open(path, "r") as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("#include \""):
                name = line.split('"')[1]
                _includes(os.path.normpath(os.path.join(os.path.dirname(path), name)), seen)


def _key(src):
    """Hash of a source, every project header it includes and the flags."""
    h = hashlib.sha256()
    h.update(" ".join(COMMON).encode())
    files = set()
    _includes(os.path.normpath(src), files)
    for f in sorted(files):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:24]


def _cost(src):
    """Rough compile cost of a source, for ordering the builds."""
    name = os.path.basename(src)
    if name.startswith("spacetime_win_"):
        L = int(name[len("spacetime_win_"):-len(".hip")])
        return 1000 + L * L
    if name.startswith(("chain_", "spacetime", "mwpm", "cnn")):
        return 500 + os.path.getsize(src) / 1000
    return os.path.getsize(src) / 1000


def build(jobs=None, verbose=True, cache=False):
    """Compile every source and link the library.  With cache=True (for
    development) an object whose source, headers and flags are unchanged is
    reused from _build/."""
    jobs = jobs or min(8, os.cpu_count() or 4)
    srcs = sources()
    cache_dir = os.path.join(HERE, "..", "_build")
    with tempfile.TemporaryDirectory(prefix="mcmcdec_build_") as tmp:
        objs, todo = [], []
        for s in srcs:
            if cache:
                os.makedirs(cache_dir, exist_ok=True)
                o = os.path.join(cache_dir, os.path.basename(s) + "." + _key(s) + ".o")
                if not os.path.exists(o):
                    todo.append((s, o))
            else:
                o = os.path.join(tmp, os.path.basename(s) + ".o")
                todo.append((s, o))
            objs.append(o)
        # longest compiles first (the unrolled space-time kernels, largest
        # code first, then the chain kernels), so that the pool ends together
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            futs = [ex.submit(_compile, s, o + ".part")
                    for s, o in sorted(todo, key=lambda t: _cost(t[0]), reverse=True)]
            for f in futs:
                f.result()
        for s, o in todo:
            os.replace(o + ".part", o)
        tmp_lib = LIB + ".tmp"
        cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp_lib] + objs
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
        os.replace(tmp_lib, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(cache="--cache" in sys.argv)
