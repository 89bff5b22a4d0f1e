"""CPU checks of the C ABI boundary: the library loads, exports every entry
point the header declares, the ctypes mirrors of the structs match the C
layout, and the defaults are the paper's GPSS parameters.  No kernel runs."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_0902_4424_amd import gpl1

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gp_l1.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char\*)\s+(gp_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 8
    lib = gpl1.load()
    for nm in names:
        assert hasattr(lib, nm), f"{nm} declared in gp_l1.h but not exported"
    assert set(names) == set(gpl1.SYMBOLS)
    out = subprocess.run(["nm", "-D", "--defined-only", gpl1.LIB_PATH],
                         capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (gp_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "gp_l1.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(gp_opts), sizeof(gp_result), sizeof(gp_instance));
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", offsetof(gp_opts, theta), offsetof(gp_opts, M_alpha),
         offsetof(gp_opts, f_target), offsetof(gp_opts, chunk), offsetof(gp_opts, fused_grid),
         offsetof(gp_opts, f_targets), offsetof(gp_opts, x0_fallback), offsetof(gp_result, x0_rejected));
  printf("%zu %zu %zu\n", offsetof(gp_opts, graph), offsetof(gp_result, reopened), offsetof(gp_opts, lookahead));
  printf("%zu %zu %zu\n", offsetof(gp_result, f), offsetof(gp_result, lambda_est),
         offsetof(gp_result, l1norm));
  printf("%zu %zu\n", offsetof(gp_instance, n), offsetof(gp_instance, rho));
  printf("%zu %zu\n", offsetof(gp_opts, trace), offsetof(gp_opts, trace_cap));
  return 0;
}''')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", f"-I{os.path.join(ROOT, 'include')}", str(prog), "-o", str(exe)],
                   check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    O, R, I = gpl1.GPOpts, gpl1.GPResult, gpl1.GPInstance
    want = [C.sizeof(O), C.sizeof(R), C.sizeof(I),
            O.theta.offset, O.M_alpha.offset, O.f_target.offset, O.chunk.offset,
            O.fused_grid.offset, O.f_targets.offset, O.x0_fallback.offset, R.x0_rejected.offset, O.graph.offset,
            R.reopened.offset, O.lookahead.offset, R.f.offset, R.lambda_est.offset, R.l1norm.offset,
            I.n.offset, I.rho.offset, O.trace.offset, O.trace_cap.offset]
    assert vals == want


def test_defaults_are_the_papers_gpss_parameters():
    o = gpl1.default_opts()
    # M = 1 (monotone), theta = 0.5, beta = 1e-4, alpha_min = 1e-10,
    # alpha_max = 1e10, tau_1 = 0.5, M_alpha = 2 (end of Section 3)
    assert (o.M, o.theta, o.beta, o.alpha_min, o.alpha_max, o.tau1, o.M_alpha) == \
        (1, 0.5, 1e-4, 1e-10, 1e10, 0.5, 2)
    assert o.backtrack_cap == 60 and o.f_target < 0 and o.refresh_every == 0
    assert not o.f_targets and o.fused_interleave == 0 and o.x0_fallback == 0 and o.graph == 0
    assert o.chunk == 64 and o.lookahead == 2
    with pytest.raises(TypeError):
        gpl1.default_opts(no_such_option=1)


def test_null_handle_is_rejected_without_gpu_work():
    lib = gpl1.load()
    assert lib.gp_last_error(None) == b"null handle"
    res = gpl1.GPResult()
    assert lib.gp_l1_solve(None, 1, None, 1, 1, 1, None, 1.0, None, 0.0, None, None,
                           C.byref(res), None) == -1
    assert lib.gp_l1_solve_noalloc(None, 1, None, 1, 1, 1, None, 1.0, None, 0.0, None, None,
                                   C.byref(res), None) == -1
    assert lib.gp_destroy(None) == 0
    assert lib.gp_l1_project(None, 0, None, 0, 1.0, None, None, None) == -1


def test_missing_library_fails_loudly(monkeypatch):
    # no fallback path: without the built library every entry point raises
    monkeypatch.setattr(gpl1, "_lib", None)
    monkeypatch.setattr(gpl1, "LIB_PATH", "/nonexistent/libgpl1.so")
    with pytest.raises(RuntimeError, match="missing"):
        gpl1.load()
    with pytest.raises(RuntimeError):
        gpl1.default_opts()


def test_option_helpers_without_gpu():
    # per-problem targets are carried as a host array kept alive by the struct
    o = gpl1.default_opts(f_targets=[1.0, 2.5, 3.0], x0_fallback=1, profile=8)
    assert o.x0_fallback == 1 and o.profile == 8
    assert [o.f_targets[i] for i in range(3)] == [1.0, 2.5, 3.0]
    gpl1._check_targets(o, 3)
    with pytest.raises(ValueError):
        gpl1._check_targets(o, 4)
    assert not gpl1.default_opts(f_targets=None).f_targets
    # the tuned-shape lookup adds the table's kernel shape unless one is given
    kw = gpl1._tuned(gpl1.GP_F32, 4096, 16384, {})
    assert {"fused_cfg", "fused_grid", "fused_interleave"} <= set(kw)
    assert gpl1._tuned(gpl1.GP_F32, 4096, 16384, {"fused_cfg": 2}) == {"fused_cfg": 2}
    assert gpl1._tuned(gpl1.GP_F32, 3, 5, {}) == {}


def test_header_constants_match_binding():
    src = open(HEADER).read()
    m = re.search(r"#define\s+GP_FUSED_PANELS\s+(\d+)", src)
    assert m and int(m.group(1)) == gpl1.GP_FUSED_PANELS
    m = re.search(r"#define\s+GP_TRACE_FIELDS\s+(\d+)", src)
    assert m and int(m.group(1)) == gpl1.TRACE_FIELDS == len(gpl1.TRACE_COLUMNS)
    m = re.search(r"#define\s+GP_NOALLOC_SCRATCH_BYTES\s+\((\d+)u\s*<<\s*(\d+)\)", src)
    assert m and (int(m.group(1)) << int(m.group(2))) == 32 << 20
