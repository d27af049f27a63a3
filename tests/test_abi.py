"""The C-ABI library loads on the CPU and exports every entry point that
include/sbh.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbh.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\*?\s*(sbh_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sbh_build", "sbh_eval", "sbh_brute", "sbh_free", "sbh_tree_info", "sbh_tree_export",
              "sbh_status_string", "sbh_last_error", "sbh_build_opts_default", "sbh_eval_opts_default",
              "sbh_mlp_forward", "sbh_mlp_pairs", "sbh_mlp_loss_grad", "sbh_mlp_train",
              "sbh_batch_create", "sbh_batch_launch", "sbh_batch_get_config", "sbh_batch_free",
              "sbh_tree_export_compressed", "sbh_tree_export_quadrupole"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2506_02219_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.fail("libsbh.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(P.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_defaults():
    import paper_2506_02219_amd as P
    L = P.lib()
    assert L.sbh_status_string(0) == b"SBH_OK"
    for code in (-1, -2, -3, -4, -5):
        assert L.sbh_status_string(code).startswith(b"SBH_E")
    o = P.EvalOpts()
    L.sbh_eval_opts_default(ctypes.byref(o))
    assert (round(o.eps, 6), o.alpha, o.group, o.rr_mode, o.proposal, o.batch, o.paths, o.mlp, o.subdomains,
            o.compressed, o.lod) == (0.001, 100.0, 1, 0, 0, 0, None, None, 0, 0, 0)
    b = P.BuildOpts()
    L.sbh_build_opts_default(ctypes.byref(b))
    assert (b.branching, b.leaf_size, b.max_level, b.compress, b.quadrupole) == (2, 8, 0, 0, 0)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes structures against sizeof / offsetof of the C header (compiled with gcc)."""
    import paper_2506_02219_amd as P
    src = tmp_path / "layout.c"
    fields = [("sbh_build_opts", None), ("sbh_eval_opts", None), ("sbh_eval_opts", "paths"),
              ("sbh_eval_opts", "mlp"), ("sbh_eval_opts", "batch"), ("sbh_eval_opts", "subdomains"),
              ("sbh_eval_opts", "compressed"), ("sbh_build_opts", "compress"),
              ("sbh_eval_opts", "lod"), ("sbh_build_opts", "quadrupole"), ("sbh_tree_desc", None),
              ("sbh_tree_desc", "lo"), ("sbh_tree_desc", "inv_side"), ("sbh_batch_item", None),
              ("sbh_batch_item", "nq"), ("sbh_batch_item", "kernel"), ("sbh_batch_config", None),
              ("sbh_batch_config", "ms")]
    exprs = ", ".join(f"(long)sizeof({s})" if f is None else f"(long)offsetof({s}, {f})" for s, f in fields)
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"sbh.h\"\n"
                   f"int main(void) {{ long v[] = {{{exprs}}}; for (int i = 0; i < {len(fields)}; ++i) "
                   "printf(\"%ld \", v[i]); return 0; }\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
                    "-I/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(P.BuildOpts), ctypes.sizeof(P.EvalOpts), P.EvalOpts.paths.offset, P.EvalOpts.mlp.offset,
            P.EvalOpts.batch.offset, P.EvalOpts.subdomains.offset, P.EvalOpts.compressed.offset,
            P.BuildOpts.compress.offset, P.EvalOpts.lod.offset, P.BuildOpts.quadrupole.offset,
            ctypes.sizeof(P.TreeDesc), P.TreeDesc.lo.offset, P.TreeDesc.inv_side.offset,
            ctypes.sizeof(P.BatchItem), P.BatchItem.nq.offset, P.BatchItem.kernel.offset, ctypes.sizeof(P.BatchConfig),
            P.BatchConfig.ms.offset]
    assert got == want


def test_argument_errors_before_any_device_work():
    """Argument checks run on the host before any HIP call, so they work here."""
    import paper_2506_02219_amd as P
    L = P.lib()
    h = ctypes.c_void_p()
    assert L.sbh_build(None, None, None, 10, None, None, ctypes.byref(h)) == -1
    assert b"NULL" in L.sbh_last_error()
    assert L.sbh_eval(None, None, 0, 0, 2.0, 1, 0, None, None, None) == -1
    assert L.sbh_brute(None, None, None, 0, None, 0, 0, None, 0, None, None) == -1
    assert L.sbh_free(None) == 0
    assert L.sbh_mlp_forward(None, None, 4, None, None) == -1
    assert L.sbh_mlp_pairs(None, None, 4, 0, 0, 3, None, None, None, None, None, None) == -1
    assert L.sbh_mlp_loss_grad(None, None, None, None, 0, None, None) == -1
    assert L.sbh_mlp_train(None, None, None, None, None, 0, 1, 64, 1e-3, 0, None, None) == -1
    o = P.EvalOpts()
    L.sbh_eval_opts_default(ctypes.byref(o))
    o.proposal = 1   # learned proposal without parameters
    one = ctypes.c_void_p(1)
    assert L.sbh_eval(one, one, 1, 0, 2.0, 1, 0, ctypes.byref(o), None, one) == -1
    assert b"mlp" in L.sbh_last_error()
    h = ctypes.c_void_p()
    assert L.sbh_batch_create(None, 1, 1, None, None, None, ctypes.byref(h)) == -1
    items = (P.BatchItem * 1)()
    assert L.sbh_batch_create(items, 0, 1, None, None, None, ctypes.byref(h)) == -1
    assert L.sbh_batch_create(items, 1, 1, None, None, None, ctypes.byref(h)) == -1   # no tree
    assert b"no tree" in L.sbh_last_error()
    assert L.sbh_batch_launch(None, 0, 0, None) == -1
    assert L.sbh_batch_free(None) == 0


def test_allocator_failure_is_reported_and_leaks_nothing():
    """An allocator that refuses: the build and the training workspace report SBH_ENOMEM before
    any kernel runs, and every allocation the library obtained has been returned."""
    import paper_2506_02219_amd as P
    L = P.lib()
    calls = {"alloc": 0, "live": 0}

    def alloc(nbytes, stream, ctx):
        calls["alloc"] += 1
        return None

    def free(ptr, nbytes, stream, ctx):
        calls["live"] -= 1

    fa, ff = P.ALLOC_FN(alloc), P.FREE_FN(free)
    assert L.sbh_set_allocator(ctypes.cast(fa, ctypes.c_void_p), None, None) == -1   # one of the two
    assert L.sbh_set_allocator(ctypes.cast(fa, ctypes.c_void_p), ctypes.cast(ff, ctypes.c_void_p), None) == 0
    try:
        fake = ctypes.c_void_p(4096)   # never dereferenced: the first allocation fails first
        h = ctypes.c_void_p()
        assert L.sbh_build(fake, fake, None, 100, None, None, ctypes.byref(h)) == -2
        assert h.value is None
        assert b"alloc" in L.sbh_last_error()
        assert L.sbh_mlp_loss_grad(fake, fake, fake, fake, 64, None, fake) == -2
        assert calls["alloc"] == 2 and calls["live"] == 0
    finally:
        assert L.sbh_set_allocator(None, None, None) == 0
