"""C ABI checks that need no GPU: the library loads, exports every function
include/chs.h declares, and rejects invalid arguments on the host before
touching a device."""
import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "chs.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chs_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2502_11602_amd import lib
    return lib()


def test_header_symbols_exported(L):
    names = _declared()
    assert "chs_build" in names and "chs_knn" in names and "chs_radius_search" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in chs.h but not exported"


def test_signatures_cover_header():
    from paper_2502_11602_amd import _lib
    assert set(_declared()) <= set(_lib.SIGNATURES), "binding misses a declared function"


def test_version_and_error_strings(L):
    assert L.chs_version().startswith(b"chs ")
    L.chs_free(None)  # NULL is ignored


def _params(**kw):
    from paper_2502_11602_amd._lib import BuildParams
    d = dict(flavor=0, dims=3, cell=(1.0, 1.0, 1.0), mixed_dense_pct=80, reserved=0,
             max_dense_cells=0)
    d.update(kw)
    return BuildParams(d["flavor"], d["dims"], (ctypes.c_double * 3)(*d["cell"]),
                       d["mixed_dense_pct"], d["reserved"], d["max_dense_cells"])


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("kw,n,msg", [
    (dict(), 0, b"n = 0"),
    (dict(), -5, b"outside"),
    (dict(dims=4), 10, b"dims"),
    (dict(dims=1), 10, b"dims"),
    (dict(flavor=7), 10, b"flavor"),
    (dict(cell=(0.0, 1.0, 1.0)), 10, b"cell[0]"),
    (dict(cell=(1.0, float("nan"), 1.0)), 10, b"cell[1]"),
    (dict(cell=(1.0, 1.0, -2.0)), 10, b"cell[2]"),
    (dict(mixed_dense_pct=101), 10, b"mixed_dense_pct"),
    (dict(reserved=1), 10, b"reserved"),
    (dict(max_dense_cells=-1), 10, b"max_dense_cells"),
])
def test_build_rejects_invalid(L, kw, n, msg):
    h = ctypes.c_void_p()
    p = _params(**kw)
    st = L.chs_build(FAKE, n, ctypes.byref(p), None, None, ctypes.byref(h))
    assert st == 1
    assert msg in L.chs_last_error()
    assert not h.value


def test_build_rejects_null(L):
    h = ctypes.c_void_p()
    p = _params()
    assert L.chs_build(None, 10, ctypes.byref(p), None, None, ctypes.byref(h)) == 1
    assert L.chs_build(FAKE, 10, None, None, None, ctypes.byref(h)) == 1
    assert L.chs_build(FAKE, 10, ctypes.byref(p), None, None, None) == 1


def test_queries_reject_null_index(L):
    from paper_2502_11602_amd._lib import Queries
    q = Queries(None, None, 0)
    tot = ctypes.c_int64()
    assert L.chs_radius_count(None, ctypes.byref(q), 1.0, FAKE, ctypes.byref(tot), None) == 1
    assert L.chs_knn(None, ctypes.byref(q), 8, float("inf"), FAKE, FAKE, None) == 1
    assert L.chs_radius_fill(None, ctypes.byref(q), 1.0, FAKE, FAKE, 0, None) == 1


def test_2d_cell_z_ignored(L):
    # with dims == 2 the z edge is not validated (it is not used)
    h = ctypes.c_void_p()
    p = _params(dims=2, cell=(1.0, 1.0, 0.0))
    st = L.chs_build(None, 10, ctypes.byref(p), None, None, ctypes.byref(h))
    assert st == 1 and b"NULL" in L.chs_last_error()


def test_agg_rejects_pair_slots_beyond_int32(L):
    # the backward regroups Q*K pair slots (plus Q centre slots) with int32
    # positions: Q*(K+1) must stay below 2^31
    Q, K = 40_000_000, 53  # Q*(K+1) = 2.16e9 > 2^31 - 1
    st = L.chs_gauss_agg_fwd(FAKE, FAKE, FAKE, 1000, Q, K, FAKE, 8, 0.25, 0, 0, FAKE, None)
    assert st == 1 and b"sizes" in L.chs_last_error()
    st = L.chs_gauss_agg_bwd(FAKE, FAKE, FAKE, 1000, Q, K, FAKE, 8, 0.25, 0, 0, FAKE, FAKE, FAKE,
                             None, None)
    assert st == 1 and b"sizes" in L.chs_last_error()


def test_coords_reject_null(L):
    assert L.chs_index_coords(None, FAKE, None) == 1
    assert b"NULL" in L.chs_last_error()


def test_set_option_rejects_bad_values(L):
    assert L.chs_index_set_option(None, 5, 16) == 1


def test_fill_chunks_reject_invalid(L):
    # checked on the host before any device access
    m = ctypes.c_int64(-1)
    assert L.chs_fill_chunks(None, 4, 10, None, None, 0, ctypes.byref(m), None) == 1
    assert L.chs_fill_chunks(FAKE, 4, 0, None, None, 0, ctypes.byref(m), None) == 1
    assert L.chs_fill_chunks(FAKE, -1, 10, None, None, 0, ctypes.byref(m), None) == 1
    assert L.chs_fill_chunks(FAKE, 4, 10, None, None, 3, ctypes.byref(m), None) == 1
    assert L.chs_fill_chunks(FAKE, 4, 10, None, None, 0, None, None) == 1


def test_knn_visited_rejects_null(L):
    from paper_2502_11602_amd._lib import Queries
    q = Queries(None, None, 5)
    assert L.chs_knn_visited(None, ctypes.byref(q), 8, float("inf"), FAKE, FAKE, FAKE, None) == 1
    assert b"NULL" in L.chs_last_error()


def test_header_compiles_and_links_as_c(tmp_path):
    """The boundary is a C ABI: chs.h compiles as C99 and a C program links
    against libchs.so and calls it (argument checks need no GPU)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "abi.c"
    src.write_text(
        '#include "chs.h"\n'
        "int main(void) {\n"
        "  chs_build_params p = {0};\n"
        "  chs_index ix = 0;\n"
        "  p.flavor = CHS_DENSE; p.dims = 3; p.cell[0] = p.cell[1] = p.cell[2] = 1.0;\n"
        "  if (chs_build(0, 10, &p, 0, 0, &ix) != CHS_E_INVALID) return 1;\n"
        "  if (chs_last_error()[0] == 0) return 2;\n"
        "  return chs_version() ? 0 : 3;\n"
        "}\n")
    lib_dir = os.path.join(root, "paper_2502_11602_amd")
    exe = tmp_path / "abi"
    cmd = [gcc, "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(root, "include"),
           "-I/opt/rocm/include", str(src), "-L" + lib_dir, "-l:libchs.so",
           "-Wl,-rpath," + lib_dir, "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=120)
    assert subprocess.run([str(exe)], timeout=60).returncode == 0
