"""The C-ABI library loads and exports every entry point that include/flow.h declares (no GPU).

Also checks host-side argument validation that needs no device (errors are returned before any
launch) and that the Python binding mirrors the C structures.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flow.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:flow_status|const char\*)\s+(flow_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def flowlib():
    import paper_2011_10979_amd as fm
    if not os.path.exists(fm.LIB_PATH):
        from paper_2011_10979_amd import build
        build.build()
    return fm.lib()


def test_header_declares_the_documented_calls():
    names = declared_functions()
    for must in ("flow_create", "flow_solve", "flow_destroy", "flow_solve_batched", "flow_op_admm_iter",
                 "flow_op_pdr_iter", "flow_op_energy", "flow_op_linearize"):
        assert must in names


def test_library_exports_every_declared_symbol(flowlib):
    import paper_2011_10979_amd as fm
    out = subprocess.run(["nm", "-D", "--defined-only", fm.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(flow_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        getattr(flowlib, n)
    assert set(fm.EXPORTS) == set(declared_functions())


def test_params_struct_layout_matches(flowlib):
    import paper_2011_10979_amd as fm
    p = fm._Params()
    assert flowlib.flow_params_default(ctypes.byref(p)) == 0
    assert p.struct_size == ctypes.sizeof(fm._Params)
    assert (p.lam, p.c, p.relax, p.sigma, p.tau, p.intensity_scale) == (0.05, 0.05, 1.0, 2.0, 0.4, 255.0)
    assert (p.levels, p.warps, p.iters, p.gs_sweeps) == (5, 5, 50, 1)


def test_invalid_arguments_are_rejected_before_any_launch(flowlib):
    import paper_2011_10979_amd as fm
    p = fm.Params(relax=1.7).c_struct()          # outside (0, 1.618...) for rpADMMI
    st = flowlib.flow_op_admm_iter(None, None, None, None, None, None, 4, 4, 4, ctypes.byref(p), None)
    assert st == fm.FLOW_E_INVAL
    assert b"relaxation" in flowlib.flow_last_error()
    p = fm.Params(lam=-1.0).c_struct()
    assert flowlib.flow_solve(None, None, None, 8, 8, 8, ctypes.byref(p), None, None, 8, None, None) == fm.FLOW_E_INVAL
    assert flowlib.flow_op_downsample(None, 4, 4, 4, None, 2, None) == fm.FLOW_E_INVAL
    assert flowlib.flow_params_default(None) == fm.FLOW_E_INVAL
    assert flowlib.flow_destroy(None) == 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_2011_10979_amd as fm
    monkeypatch.setattr(fm, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(fm, "_lib", None)
    with pytest.raises(ImportError):
        fm.lib()


def test_binding_allocates_outputs_with_the_input_pitch():
    """Op outputs must share the input planes' row pitch: the kernels address every plane of a
    call with one pitch, and a dense output behind a padded input would be overrun."""
    import torch
    import paper_2011_10979_amd as fm
    base = torch.zeros(17, 64)
    t = base[:, :61]
    o = fm._like(t)
    assert o.shape == t.shape and o.stride() == t.stride()
    assert o.untyped_storage().nbytes() >= ((17 - 1) * 64 + 61) * 4
    dense = torch.empty_like(t)            # the layout that must be refused
    assert dense.stride() != t.stride()
    monkey = fm._plane
    try:
        fm._plane = lambda x, name="t": x
        with pytest.raises(ValueError):
            fm._same_layout(t, [("out", dense)], "op")
        fm._same_layout(t, [("out", o)], "op")
    finally:
        fm._plane = monkey


@pytest.mark.parametrize("cname,pyname", [("flow_params", "_Params"), ("flow_result", "_Result"),
                                          ("flow_stats", "_Stats"), ("flow_pair", "_Pair"),
                                          ("flow_admm_state", "_AdmmState"), ("flow_pdr_state", "_PdrState"),
                                          ("flow_server_stats", "_ServerStats")])
def test_struct_layouts_match_the_header(tmp_path, cname, pyname):
    """Size and every field offset of the ctypes mirror equal what a C compiler makes of flow.h."""
    import paper_2011_10979_amd as fm
    py = getattr(fm, pyname)
    fields = [f[0] for f in py._fields_]
    cfields = {"lam": "lambda"}
    src = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {",
           f'  printf("%zu\\n", sizeof({cname}));']
    for f in fields:
        src.append(f'  printf("%zu\\n", offsetof({cname}, {cfields.get(f, f)}));')
    src.append("  return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(c)], check=True, capture_output=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got[0] == ctypes.sizeof(py)
    assert got[1:] == [getattr(py, f).offset for f in fields]


def test_working_set_bytes_is_host_only_and_checked(flowlib):
    import paper_2011_10979_amd as fm
    vga = fm.working_set_bytes(480, 640)
    assert vga % 256 == 0
    # 9 pyramid / linearisation planes + 14 state planes per level (pitch 640), over 5 levels
    assert 23 * 4 * 480 * 640 < vga < 23 * 4 * 480 * 640 * 1.45
    assert fm.working_set_bytes(480, 640, levels=3) < vga
    assert fm.working_set_bytes(480, 640, storage="f16") < vga
    assert fm.working_set_bytes(480, 640, beta=0.05) > vga
    assert fm.working_set_bytes(131072, 64, levels=1) > 0                   # FLOW_MAX_SIDE rows
    for bad in ((1, 64, {}), (480, 640, {"levels": 17}), (40, 40, {"levels": 7}), (131073, 64, {"levels": 1}),
                (64, 131073, {"levels": 1})):
        with pytest.raises(fm.FlowError):
            fm.working_set_bytes(bad[0], bad[1], **bad[2])
