"""The C ABI library loads and exports every function include/mrc.h declares
(no GPU calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mrc_[a-z0-9_]+)\s*\(", src)))


def test_header_compiles_as_c():
    r = subprocess.run(["gcc", "-x", "c", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", HEADER],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_library_exports_every_declared_function():
    from paper_1810_03099_amd import mrc
    if not os.path.exists(mrc.LIB_PATH):
        pytest.skip("libmrc.so not built")
    lib = ctypes.CDLL(mrc.LIB_PATH)
    decl = declared_functions()
    assert len(decl) >= 30
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(mrc.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", mrc.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (mrc_[a-z0-9_]+)", out))
    assert set(decl) <= exported


def test_binding_struct_sizes_match_header():
    from paper_1810_03099_amd import mrc
    prog = r'''
#include <stdio.h>
#include "mrc.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(mrc_docs), sizeof(mrc_ref_spec), sizeof(mrc_compare_opts),
         sizeof(mrc_pair), sizeof(mrc_hit), sizeof(mrc_compare_stats), sizeof(mrc_serve_opts), sizeof(mrc_result));
  return 0; }
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(src, "w").write(prog)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        sizes = [int(x) for x in subprocess.check_output([exe]).split()]
    want = [ctypes.sizeof(t) for t in (mrc.MrcDocs, mrc.MrcRefSpec, mrc.MrcCompareOpts, None, mrc.MrcHit,
                                       mrc.MrcCompareStats, mrc.MrcServeOpts, mrc.MrcResult) if t is not None]
    assert sizes[:3] == want[:3]
    assert sizes[3] == mrc.PAIR_DTYPE.itemsize == 16
    assert sizes[4:] == want[3:]


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1810_03099_amd import mrc
    monkeypatch.setattr(mrc, "_lib", None)
    monkeypatch.setattr(mrc, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(mrc.MrcUnavailable):
        mrc.lib()
