"""CPU checks of the native library: it is built, loads, and exports every
entry point include/gf.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(gf_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("gf_region_run", "gf_reduce", "gf_rpc_poll", "gf_ctx_create", "gf_ctx_destroy",
                     "gf_last_error", "gf_sync"):
        assert required in names


def test_library_loads_and_exports_every_declared_symbol():
    import paper_2306_11686_amd as gf
    lib = gf.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(gf.exported_symbols()) == set(declared_functions())


def test_binding_struct_layouts_match_header(tmp_path):
    import subprocess
    import paper_2306_11686_amd as gf
    from paper_2306_11686_amd import binding
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gf.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(gf_step),'
                   ' sizeof(gf_instance), sizeof(gf_launch), sizeof(gf_ctx_opts), sizeof(gf_run_stats),'
                   ' sizeof(gf_program), offsetof(gf_step, chunk), sizeof(gf_call_arg), sizeof(gf_call_stats),'
                   ' offsetof(gf_ctx_opts, rpc_payload)); return 0;}\n')
    src.write_text(src.read_text().replace('#include "gf.h"', '#include "gf.h"\n#include "gf_heap.h"')
                   .replace('offsetof(gf_ctx_opts, rpc_payload));', 'offsetof(gf_ctx_opts, rpc_payload));'
                            ' printf("%zu\\n", sizeof(gf_heap_opts));'))
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert got == [ctypes.sizeof(gf.Step), ctypes.sizeof(gf.Instance), ctypes.sizeof(gf.Launch),
                   ctypes.sizeof(binding.CtxOpts), ctypes.sizeof(binding.RunStats), ctypes.sizeof(gf.Program),
                   gf.Step.chunk.offset, ctypes.sizeof(gf.CallArg), ctypes.sizeof(gf.CallStats),
                   binding.CtxOpts.rpc_payload.offset, ctypes.sizeof(binding.HeapOpts)]


def test_binding_constants_match_header():
    """Enumerators and limits of the host-call interface agree with the
    header (compiled with gcc from include/gf.h)."""
    import subprocess
    import tempfile
    import paper_2306_11686_amd as gf
    names = ["GF_S_CALL", "GF_STEP_TIMED", "GF_CALLEE_FPRINTF", "GF_CALLEE_SNPRINTF", "GF_CALLEE_SSCANF",
             "GF_CALLEE_FWRITE", "GF_CALLEE_FREAD", "GF_ARG_CONST", "GF_ARG_SCALAR", "GF_ARG_ITER", "GF_ARG_REF", "GF_ARG_HEAPREF",
             "GF_REF_READ", "GF_REF_WRITE", "GF_REF_READWRITE", "GF_CALL_MAX_ARGS", "GF_CALL_MAX_REFS",
             "GF_CALL_MAX_SITES", "GF_S_PRINTF", "GF_STEP_BLOCKING", "GF_STEP_NOWAIT", "GF_R_OWNER", "GF_R_PHASES",
             "GF_HEAP_OP_MALLOC", "GF_HEAP_OP_FREE", "GF_HEAP_OP_FIND", "GF_HEAP_BENCH_ROUNDTRIP",
             "GF_HEAP_BENCH_HOLD", "GF_HEAP_BENCH_RELEASE"]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "c.c")
        body = " ".join(f'printf("%ld\\n", (long)({n}));' for n in names)
        open(src, "w").write(f'#include <stdio.h>\n#include "gf.h"\n#include "gf_heap.h"\n'
                             f'int main(void){{{body} return 0;}}\n')
        exe = os.path.join(d, "c")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    assert got == [getattr(gf, n) for n in names]


def test_programs_are_well_formed():
    from paper_2306_11686_amd import programs
    p = programs.cg(500)
    assert p.n_prologue == 2 and p.n_body == 12 and p.iters == 500
    # the two update axpbys (x += alpha p, r -= alpha q) are nowait; no other step is
    flags = [p.body[i].flags for i in range(p.n_body)]
    assert [p.body[i].kind for i in (4, 5)] == [5, 5] and flags[4] == flags[5] == 4
    assert all(f == 0 for i, f in enumerate(flags) if i not in (4, 5))
    assert all(programs.cg(3, nowait=False).body[i].flags == 0 for i in range(12))
    p3 = programs.jacobi3d(200)
    kinds = [p3.body[i].kind for i in range(p3.n_body)]
    assert kinds == [32, 2, 37, 36]
