"""The C-ABI library loads on the host and exports every symbol its header declares
(no compute call: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "g4hip.h")
LIB = os.path.join(ROOT, "paper_2010_03567_amd", "libg4hip.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(g4_\w+)\s*\(", src)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libg4hip.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libg4hip.so not built")
def test_invalid_args_rejected_on_host():
    """Host-side argument checks reject bad sizes and parameters before any device work."""
    import paper_2010_03567_amd.g4hip as g
    tp = g.tree_params(True, 1.0, leaf_max=8)
    with pytest.raises(g.G4Error):
        g.g4_workspace_bytes(tp, 0)
    bad = g.tree_params(True, 1.0, leaf_max=0)
    with pytest.raises(g.G4Error):
        g.g4_workspace_bytes(bad, 100)


def test_binding_refuses_to_run_without_library(tmp_path, monkeypatch):
    """Without the built library the binding raises instead of falling back."""
    import importlib.util
    src = os.path.join(ROOT, "paper_2010_03567_amd", "g4hip.py")
    d = tmp_path / "pkg"
    d.mkdir()
    (d / "g4hip.py").write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("g4hip_copy", d / "g4hip.py")
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)


def test_binding_structs_match_header(tmp_path):
    """The ctypes mirrors of the parameter and counter structs have the C header's
    size and field offsets (a silent mismatch would corrupt every call)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    import importlib.util
    src = os.path.join(ROOT, "paper_2010_03567_amd", "g4hip.py")
    spec = importlib.util.spec_from_file_location("g4hip_structs", src)
    mod = importlib.util.module_from_spec(spec)
    try:
        spec.loader.exec_module(mod)
    except ImportError:
        pytest.skip("libg4hip.so not built")
    structs = ("g4_tree_params", "g4_particles", "g4_walk_params", "g4_fmm_params", "g4_stats", "g4_pm_params",
               "g4_kdk_params", "g4_kdk_stats")
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void) {']
    for s in structs:
        lines.append(f'printf("{s} size %zu\\n", sizeof({s}));')
        for name, _ in getattr(mod, s)._fields_:
            lines.append(f'printf("{s} {name} %zu\\n", offsetof({s}, {name}));')
    lines.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(c)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        s, field, value = line.split()
        cls = getattr(mod, s)
        got = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(value), (s, field, got, value)
