"""Compile the HIP sources under csrc/ into libsbh.so (gfx950) with hipcc.

Every call recompiles.  Run as a script or call build()."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsbh.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["api.hip", "build.hip", "eval.hip", "brute.hip", "mlp.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         # keep the compiler from emitting packed fp32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    return obj, err


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                print(err)
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, check=True)
    os.replace(tmp, LIB)
    _record_revision()
    return LIB


def _record_revision():
    """Write the git revision the library was built from (with +dirty when its sources differ from
    it) beside the objects, for runs on a copy of the tree without .git."""
    root = os.path.dirname(HERE)
    try:
        sha = subprocess.run(["git", "rev-parse", "HEAD"], cwd=root, capture_output=True, text=True,
                             timeout=10).stdout.strip()
        dirty = subprocess.run(["git", "diff", "--quiet", "HEAD", "--", "paper_2506_02219_amd/csrc", "include"],
                               cwd=root, timeout=10).returncode != 0
    except Exception:
        return
    if sha:
        with open(os.path.join(OBJ, "source_revision.txt"), "w") as f:
            f.write(sha + ("+dirty" if dirty else "") + "\n")


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
