"""The C-ABI library loads and exports every entry point include/vrc.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vrc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:vrc_status|const char \*)\s*(vrc_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    import paper_1706_07476_amd as vrc
    if not os.path.exists(vrc.LIB_PATH):
        from paper_1706_07476_amd import build
        build.build(force=False)
    return vrc.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("vrc_create", "vrc_set_mesh", "vrc_set_xs_tables", "vrc_create_tally", "vrc_cast_rays",
                     "vrc_read_tally", "vrc_load_tally", "vrc_reset_tally", "vrc_trace_rays"):
        assert required in names
    assert len(names) >= 17


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    import paper_1706_07476_amd as vrc
    assert sorted(vrc.exported_symbols()) == declared_functions()


def test_version_string(lib):
    import paper_1706_07476_amd as vrc
    assert "gfx950" in vrc.vrc_version()


def test_missing_library_fails_loudly(tmp_path):
    import paper_1706_07476_amd as vrc
    saved = vrc._lib
    try:
        vrc._lib = None
        with pytest.raises(vrc.VrcError):
            vrc.load_library(str(tmp_path / "nope.so"))
    finally:
        vrc._lib = saved


def test_batch_marshalling_checks_dtypes_and_lengths():
    import numpy as np
    import paper_1706_07476_amd as vrc
    a = [np.zeros(5, np.float32) for _ in range(8)]
    b = vrc.make_batch(a)
    assert b.n == 5 and b.fp64 == 0 and b.on_device == 0
    with pytest.raises(ValueError):
        vrc.make_batch(a[:7])
    bad = list(a)
    bad[3] = np.zeros(5, np.float64)
    with pytest.raises(ValueError):
        vrc.make_batch(bad)
    bad[3] = np.zeros(4, np.float32)
    with pytest.raises(ValueError):
        vrc.make_batch(bad)


def test_create_without_device_is_an_error_not_a_crash(lib):
    import torch
    import paper_1706_07476_amd as vrc
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(vrc.VrcError):
        vrc.vrc_create(0)


def test_binding_structs_match_the_header_layout(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets of the C struct (compiled with gcc)."""
    import shutil
    import subprocess
    import paper_1706_07476_amd as vrc
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [getattr(vrc, n) for n in dir(vrc) if n.startswith("vrc_") and isinstance(getattr(vrc, n), type)
               and issubclass(getattr(vrc, n), ctypes.Structure)]
    assert len(structs) >= 8
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for st in structs:
        name = st.__name__
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for st in structs:
        name = st.__name__
        assert got[(name, "size")] == ctypes.sizeof(st), name
        for f, _ in st._fields_:
            assert got[(name, f)] == getattr(st, f).offset, (name, f)
