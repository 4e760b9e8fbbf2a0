"""The C-ABI library loads on the CPU and exports every symbol include/drsf.h
declares (no compute calls: there is no GPU here)."""
from __future__ import annotations

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "drsf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(drsf_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("drsf_create", "drsf_apply", "drsf_destroy", "drsf_copy_out",
                     "drsf_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2607_20211_amd import drsf
    if not os.path.exists(drsf.LIB_PATH):
        pytest.skip("libdrsf.so not built")
    lib = drsf.load()
    missing = [s for s in declared_functions() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(drsf.EXPORTS) == set(declared_functions())
    assert "gfx950" in drsf.drsf_version()


def test_binding_has_no_cpu_fallback():
    """The binding routes every call to libdrsf.so and never imports the oracle."""
    src = open(os.path.join(ROOT, "paper_2607_20211_amd", "drsf.py")).read()
    assert "import oracle" not in src and "from oracle" not in src


def test_default_opts_layout_matches_the_header():
    """drsf_default_opts (host code, no device call) fills the C struct; the
    binding's ctypes mirror must read every field where the library wrote
    it: the documented defaults, up to the last field."""
    from paper_2607_20211_amd import drsf
    if not os.path.exists(drsf.LIB_PATH):
        pytest.skip("libdrsf.so not built")
    o = drsf.drsf_default_opts()
    assert o.validate_forest == 1 and o.profile == 0 and o.inputs_on_device == 0
    assert o.max_batch == 1 << 20 and o.delta_capacity == 0 and o.sweep_mode == 0
    assert o.rounds_queued == 0 and o.levels_queued == 0
    assert o.reverse_mode == 0 and o.replacement_mode == 0
    assert not o.dev_alloc and not o.dev_free and not o.alloc_user
    assert o.small_graph_vertices == 0 and o.small_threads == 0
    assert o.validate_batches == 1 and o.launch_mode == 0 and o.walk_limit == 0
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = text[text.index("typedef struct {", text.index("typedef struct drsf_ctx")):]
    body = body[:body.index("} drsf_opts;")]
    fields = re.findall(r"\b(\w+)\s*;", body) + re.findall(r"\(\*(\w+)\)", body)
    assert set(fields) == {f for f, _ in drsf.drsf_opts._fields_}


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes mirrors of drsf_opts and drsf_view have the C
    compiler's size and every field at the C offset (a mirror shorter than
    the C struct would let the library write past the Python buffer)."""
    import shutil
    import subprocess
    from paper_2607_20211_amd import drsf
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "drsf.h"', "int main(void) {"]
    for st in (drsf.drsf_opts, drsf.drsf_view):
        name = st.__name__
        lines.append(f'printf("{name} sizeof %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    want = {}
    for line in out:
        if line:
            name, field, val = line.split()
            want[(name, field)] = int(val)
    import ctypes
    for st in (drsf.drsf_opts, drsf.drsf_view):
        name = st.__name__
        assert ctypes.sizeof(st) == want[(name, "sizeof")], name
        for f, _ in st._fields_:
            assert getattr(st, f).offset == want[(name, f)], (name, f)
