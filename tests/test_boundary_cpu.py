"""CPU checks of the C-ABI library: it loads, exports every symbol declared
in include/hf.h, and its host-side argument handling works without a GPU
(no compute calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hf.h")


def _declared():
    txt = open(HEADER).read()
    decl = r"^\s*(?:hf_status|void|const char)\s*\*?\s*(hf_[a-z_0-9]+)\s*\("
    return sorted(set(re.findall(decl, txt, flags=re.MULTILINE)))


def test_header_and_binding_agree():
    import paper_1911_10275_amd as hf
    assert sorted(hf.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    import paper_1911_10275_amd as hf
    lib = hf.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_options_and_null_handling():
    import paper_1911_10275_amd as hf
    lib = hf.load()
    o = hf.default_options()
    assert o.gmres_m == 60 and o.rtol == 1e-10 and o.precision == hf.HF_FP64
    assert o.rtol_inner == 1e-4 and o.ir_inner_cycles == 1 and o.b_stab == 10.0 and o.newton_maxit == 25
    assert lib.hf_create(C.byref(o), None) == hf.HF_EINVAL
    assert lib.hf_assemble(None, None) == hf.HF_EINVAL
    assert lib.hf_finalize(None) == hf.HF_EINVAL
    assert lib.hf_last_error(None) == b"null context"
    lib.hf_destroy(None)


def test_create_without_gpu_fails_cleanly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import paper_1911_10275_amd as hf
    with pytest.raises(hf.HFError) as ei:
        hf.Context()
    assert ei.value.status in (hf.HF_EDEVICE, hf.HF_EINVAL)


_STRUCTS = {"hf_options": "Options", "hf_material": "Material", "hf_sizes": "Sizes",
            "hf_solve_stats": "SolveStats", "hf_newton_stats": "NewtonStats",
            "hf_tuning": "Tuning", "hf_profile": "Profile"}


def test_struct_layouts_match_header(tmp_path):
    """Every struct of include/hf.h, compiled by the host C compiler, has the
    size and the field offsets of its ctypes mirror in the binding."""
    import shutil
    import subprocess
    import paper_1911_10275_amd as hf
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "hf.h"', "int main(void) {"]
    for cname, pname in _STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in getattr(hf, pname)._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            cname, what, val = line.split()
            got[(cname, what)] = int(val)
    for cname, pname in _STRUCTS.items():
        py = getattr(hf, pname)
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_documented_option_defaults_match_the_library():
    """Every '(default X)' that include/hf.h states for an hf_options field is
    the value hf_default_options sets."""
    import paper_1911_10275_amd as hf
    txt = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} hf_options;", txt, re.S).group(1)
    fields = re.findall(r"(?:int|double|void\s*\*)\s*(\w+);\s*/\*(.*?)\*/", body, re.S)
    o = hf.default_options()
    checked = 0
    for name, comment in fields:
        m = re.search(r"\(default\s*:?\s*([-+0-9.eE]+)", " ".join(comment.split()))
        if m is None:
            continue
        assert getattr(o, name) == pytest.approx(float(m.group(1))), name
        checked += 1
    assert checked >= 12
