"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU).  libsbh's sources are compiled with the sanitizers on their host side
only (device code is built as usual), and the ABI tests that run without a GPU
(defaults, status strings, argument checks of every entry point, the
allocator's failure path) call that build in a subprocess that preloads the
ASan runtime; any sanitizer report is fatal."""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_02219_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["api.hip", "build.hip", "eval.hip", "brute.hip", "mlp.hip"]
# sanitizers on the host pass only (each -fsanitize= right after -Xarch_host)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

DRIVER = r'''
import sys, tempfile, pathlib
sys.path.insert(0, ROOT)
sys.path.insert(0, ROOT + "/tests")
import paper_2506_02219_amd as P
P.LIB_PATH = LIB
import test_abi as A
A.test_library_exports_every_declared_symbol()
A.test_status_strings_and_defaults()
A.test_struct_layouts_match_header(pathlib.Path(tempfile.mkdtemp()))
A.test_argument_errors_before_any_device_work()
A.test_allocator_failure_is_reported_and_leaks_nothing()
print("sanitized host code ok")
'''


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_library_host_code_under_sanitizers(tmp_path):
    rt = _asan_runtime()
    if not os.path.exists(HIPCC) or rt is None:
        pytest.skip("hipcc or the clang ASan runtime is not available")

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops"] + SAN + ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    lib = str(tmp_path / "libsbh_sanitized.so")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", lib] + objs, check=True)
    script = tmp_path / "drive.py"
    script.write_text(f"ROOT = {ROOT!r}\nLIB = {lib!r}\n" + DRIVER)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "sanitized host code ok" in r.stdout, (r.returncode, r.stdout[-2000:],
                                                                       r.stderr[-4000:])
