"""C-ABI library: it loads, exports every declared entry point, and its host-only calls
behave (no compute call is made here: this runs without a GPU)."""

import os
import re

import pytest

import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "plsqr.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(plsqr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_four_calls_and_helpers():
    names = _declared()
    for n in ("plsqr_create", "plsqr_set_operator", "plsqr_solve", "plsqr_poll", "plsqr_destroy",
              "plsqr_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1308_6634_amd import plsqr as P
    lib = P._lib
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(P.EXPORTED)


def test_auto_levels_matches_rule():
    from paper_1308_6634_amd import plsqr as P
    for dims in [(32, 32, 32), (48, 48, 48), (64, 64, 64), (96, 96, 96), (128, 128, 128),
                 (64, 64, 1), (6, 6, 6), (5, 8, 8), (12, 20, 1), (40, 24, 16)]:
        assert P.plsqr_auto_levels(*dims) == gen.auto_levels(dims), dims
    assert P.plsqr_auto_levels(0, 4, 4) == 0


def test_workspace_bytes():
    from paper_1308_6634_amd import plsqr as P
    pb = P.make_problem((64, 64, 64), outer=8, inner=40, levels=5)
    blur = P.plsqr_workspace_bytes(pb, P.PLSQR_OP_BLUR, 64 ** 3)
    dense = P.plsqr_workspace_bytes(pb, P.PLSQR_OP_DENSE, 4096)
    assert blur > 10 * 4 * 64 ** 3 and dense > 0
    assert P.plsqr_workspace_bytes(pb, 7, 4096) == 0
    big = P.plsqr_workspace_bytes(P.make_problem((128, 128, 128), outer=10, levels=6),
                                  P.PLSQR_OP_BLUR, 128 ** 3)
    assert 50e6 < big < 200e6


def test_create_errors_without_arguments():
    from paper_1308_6634_amd import plsqr as P
    with pytest.raises(P.PlsqrError):
        P.plsqr_create(device=-1)
    assert P.plsqr_destroy(None) == 0
    assert isinstance(P.plsqr_last_error(), str)


def _c_layout(struct, fields, tmp_path):
    """sizeof and offsetof of a struct of include/plsqr.h, compiled by the host C compiler."""
    import subprocess
    src = tmp_path / "layout.c"
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("name", ["plsqr_problem", "plsqr_operator", "plsqr_result"])
def test_ctypes_structs_match_the_header(name, tmp_path):
    from paper_1308_6634_amd import plsqr as P
    cls = getattr(P, name)
    fields = [f[0] for f in cls._fields_]
    size, offs = _c_layout(name, fields, tmp_path)
    assert size == __import__("ctypes").sizeof(cls)
    assert offs == [getattr(cls, f).offset for f in fields]


def test_workspace_bytes_hold_the_s4_vectors():
    from paper_1308_6634_amd import plsqr as P
    pb = P.make_problem((64, 64, 64), outer=8, inner=40, levels=5)
    base = P.plsqr_workspace_bytes(pb, P.PLSQR_OP_DENSE, 4096)
    pb.flags = P.PLSQR_FLAG_STOP_S4
    pb.eta, pb.delta = 1.1, 1.0
    s4 = P.plsqr_workspace_bytes(pb, P.PLSQR_OP_DENSE, 4096)
    assert s4 - base >= 2 * 4 * 4096
    pb.flags = P.PLSQR_FLAG_STOP_OUTER
    assert P.plsqr_workspace_bytes(pb, P.PLSQR_OP_DENSE, 4096) == base
