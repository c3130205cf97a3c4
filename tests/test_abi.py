"""The C-ABI library loads, exports every entry point include/mm.h declares,
and rejects invalid arguments before any device work (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mm.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1406_7459_amd import mm
    return mm.lib()


def test_header_declares_the_three_paper_calls():
    syms = declared_symbols()
    for s in ("mm_demag_setup", "mm_demag_apply", "mm_llg_step"):
        assert s in syms


def test_every_declared_symbol_is_exported(L):
    for s in declared_symbols():
        assert hasattr(L, s), s


def test_binding_covers_header():
    from paper_1406_7459_amd import mm
    assert sorted(mm.SYMBOLS) == declared_symbols()


def test_status_strings(L):
    from paper_1406_7459_amd import mm
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.mm_status_string(code)
    assert L.mm_status_string(mm.MM_EINVAL) == b"invalid argument"


@pytest.mark.parametrize("args", [
    (0, 4, 4, 1e-9, 1e-9, 1e-9), (4, -1, 4, 1e-9, 1e-9, 1e-9), (4, 4, 4, 0.0, 1e-9, 1e-9),
    (513, 4, 4, 1e-9, 1e-9, 1e-9), (4, 4, 1024, 1e-9, 1e-9, 1e-9), (4, 4, 4, float("nan"), 1e-9, 1e-9),
    (7, 600, 1, 1e-9, 1e-9, 1e-9), (4, 4, 4, 1e-9, -1e-9, 1e-9)])
def test_setup_rejects_bad_grid_before_device_work(L, args):
    h = C.c_void_p(123)
    rc = L.mm_demag_setup(*args, C.byref(h))
    assert rc == -1
    assert h.value is None
    buf = C.create_string_buffer(256)
    assert L.mm_last_error(buf, 256) > 0 and buf.value


# (1, 2^24, 1): 2^24 cells, but a padded x-y plane of (2^24 + 1) * 8 positions,
# beyond the first layer's 32-bit neighbour offsets
@pytest.mark.parametrize("grid", [(0, 4, 4), (4, 0, 4), (4, 4, -1), (512, 256, 257), (1, 1 << 24, 1)])
def test_surrogate_rejects_bad_grid_before_device_work(L, grid):
    from paper_1406_7459_amd import mm
    h = C.c_void_p(123)
    assert L.mm_sur_create(*grid, C.byref(h)) == mm.MM_EINVAL
    assert h.value is None


def test_null_arguments_are_rejected(L):
    from paper_1406_7459_amd import mm
    assert L.mm_demag_setup(4, 4, 4, 1e-9, 1e-9, 1e-9, None) == mm.MM_EINVAL
    assert L.mm_demag_apply(None, None, None, None) == mm.MM_EINVAL
    p = mm.LLGParams.make(Ms=8e5, A=1.3e-11)
    assert L.mm_llg_step(None, C.byref(p), None, 1, None, None) == mm.MM_EINVAL
    n = C.c_size_t(7)
    assert L.mm_plan_workspace_bytes(None, C.byref(n)) == mm.MM_EINVAL
    assert L.mm_plan_bind_workspace(None, None, 0) == mm.MM_EINVAL
    assert L.mm_batch_workspace_bytes(None, C.byref(n)) == mm.MM_EINVAL
    assert L.mm_batch_bind_workspace(None, None, 0) == mm.MM_EINVAL
    assert L.mm_sur_workspace_bytes(None, C.byref(n)) == mm.MM_EINVAL
    assert L.mm_sur_bind_workspace(None, None, 0) == mm.MM_EINVAL
    assert L.mm_sur_attach(None, None) == mm.MM_EINVAL
    assert L.mm_reduce(None, C.byref(p), None, None, None) == mm.MM_EINVAL
    assert L.mm_newell_tensor(4, 4, 4, 1e-9, 1e-9, 1e-9, None, None) == mm.MM_EINVAL
    L.mm_destroy(None)


def test_no_device_reports_enodev(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1406_7459_amd import mm
    h = C.c_void_p()
    assert L.mm_demag_setup(4, 4, 4, 1e-9, 1e-9, 1e-9, C.byref(h)) == mm.MM_ENODEV


def test_last_error_truncates(L):
    h = C.c_void_p()
    L.mm_demag_setup(0, 1, 1, 1.0, 1.0, 1.0, C.byref(h))
    buf = C.create_string_buffer(4)
    n = L.mm_last_error(buf, 4)
    assert n > 3 and len(buf.value) == 3


def test_params_and_stats_layout_match_header(tmp_path):
    """The ctypes mirrors of the header's structs have the header's field
    offsets and sizes, as a C compiler lays them out."""
    import subprocess
    from paper_1406_7459_amd import mm
    structs = {"mm_llg_params": mm.LLGParams, "mm_stats": mm.Stats, "mm_plan_info": mm.PlanInfo,
               "mm_sur_stats": mm.SurStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for ln in subprocess.check_output([str(exe)]).decode().split("\n"):
        if ln:
            a, b, c = ln.split()
            got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def test_stats_count_rule():
    from paper_1406_7459_amd import mm
    assert mm.Plan.stats_count(10, 0) == 1
    assert mm.Plan.stats_count(10, 3) == 4
    assert mm.Plan.stats_count(10, 5) == 2
    assert mm.Plan.stats_count(10, 10) == 1
    assert mm.Plan.stats_count(0, 0) == 1
