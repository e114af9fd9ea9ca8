"""The C-ABI library loads and exports every entry point its header declares;
argument validation works without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "leafi.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(leafi_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2502_01836_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2502_01836_amd import build
        build.build()
    return _lib.load()


def test_every_declared_symbol_is_exported_and_bound(lib):
    from paper_2502_01836_amd import _lib
    names = _declared()
    assert len(names) >= 20
    bound = {n for n, _, _ in _lib.SIGNATURES}
    for n in names:
        assert hasattr(lib, n), f"{n} not exported"
        assert n in bound, f"{n} has no ctypes signature"


def test_version_and_defaults(lib):
    from paper_2502_01836_amd import _lib
    assert lib.leafi_version().decode().startswith("leafi")
    o = _lib.TrainOpts()
    lib.leafi_default_train_opts(ctypes.byref(o))
    assert (o.n_global, o.n_local, o.max_epochs, o.batch, o.patience) == (1500, 500, 1000, 64, 10)
    assert abs(o.lr0 - 0.01) < 1e-9 and abs(o.a - 2.0) < 1e-9 and o.th_override < 0
    s = _lib.SearchOpts()
    lib.leafi_default_search_opts(ctypes.byref(s))
    assert s.k_max == 1 and s.scan == 0 and s.n_schedule == 2 and list(s.schedule[:2]) == [1, 0]


def test_struct_sizes_match_header_layout(tmp_path):
    """The binding's structs have the sizes and field offsets a C compiler
    gives the header's (a program built against include/leafi.h prints them)."""
    import shutil
    import subprocess
    from paper_2502_01836_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = [("leafi_build_opts", _lib.BuildOpts), ("leafi_search_opts", _lib.SearchOpts),
             ("leafi_search_stats", _lib.SearchStats), ("leafi_info", _lib.Info),
             ("leafi_train_opts", _lib.TrainOpts), ("leafi_train_report", _lib.TrainReport)]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "leafi.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "sizes.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "sizes"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = []
    for _, py in pairs:
        want.append(ctypes.sizeof(py))
        want += [getattr(py, fname).offset for fname, _ in py._fields_]
    assert got == want


def test_null_handles_are_rejected_without_touching_the_gpu(lib):
    from paper_2502_01836_amd import _lib
    info = _lib.Info()
    assert lib.leafi_get_info(None, ctypes.byref(info)) == -1
    assert lib.leafi_export_boxes(None, None) == -1
    assert "NULL" in lib.leafi_last_error().decode()
    o = _lib.SearchOpts()
    lib.leafi_default_search_opts(ctypes.byref(o))
    assert lib.leafi_search_knn(None, None, 0, None, None, ctypes.byref(o), None, None, None, None) == -1
    F, A = _lib.FREE_FN, _lib.ALLOC_FN
    assert lib.leafi_create(A(), F(), None, None) == -1                     # out is NULL
    h = ctypes.c_void_p()
    only_alloc = A(lambda ctx, n, out: 1)
    assert lib.leafi_create(only_alloc, F(), None, ctypes.byref(h)) == -1   # alloc without free
    assert "both" in lib.leafi_last_error().decode() and not h.value
    assert lib.leafi_get_examples(None, None, None, None, None, None, None, None) == -1
    # sizes are validated before any device work
    assert lib.leafi_znorm(None, -1, 8, None, None) == -1
    assert lib.leafi_mlp_infer(None, 1, 8, 3, None, 1, None, None) == -1   # hidden not a multiple of 4
    assert lib.leafi_mlp_infer(None, 1, 6, 8, None, 1, None, None) == -1   # m not a multiple of 4
    assert lib.leafi_mlp_infer(None, 1, 2048, 8, None, 1, None, None) == -1  # m above 1024
    assert lib.leafi_mlp_sgd_step(None, 1, 8, 4, None, None, 65, 0.1, None, None) == -1  # batch > 64
    lib.leafi_destroy(None)


def test_python_binding_fails_loudly_without_library(tmp_path):
    from paper_2502_01836_amd import _lib
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            _lib.load(str(tmp_path / "missing.so"))
    finally:
        _lib._lib = saved
