"""The C ABI library loads and exports every symbol include/rewl.h declares
(CPU only: no compute call)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rewl.h")).read()
    return sorted(set(re.findall(r"^\s*(?:rewl_status|void|const char \*|int32_t|size_t)\s*\*?(rewl_\w+)\s*\(",
                                 txt, re.M)))


def test_library_exports_all_declared_symbols():
    from paper_1411_4212_amd.build import LIB
    assert os.path.exists(LIB), "librewl.so not built"
    lib = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_every_symbol():
    from paper_1411_4212_amd import rewl
    assert sorted(rewl.EXPORTED) == _declared()
    for n in _declared():
        assert callable(getattr(rewl, n))


def test_errors_without_device():
    """Argument checks and error reporting work before any GPU use."""
    from paper_1411_4212_amd import rewl
    import pytest
    with pytest.raises(rewl.RewlError) as e:
        rewl.rewl_create(0, 0, 99)
    assert e.value.code == -1
    assert "mode" in rewl.rewl_last_error()
    assert rewl.rewl_poll.__name__ == "rewl_poll"


def test_grid_cap_calls_check_arguments_without_device():
    """The grid-cap calls reject a null context; the autotuner's trial
    record has the layout the header declares (4 x int32, double, 2 x int32)."""
    import ctypes
    from paper_1411_4212_amd import rewl
    import pytest
    with pytest.raises(rewl.RewlError) as e:
        rewl.rewl_set_grid_cap(None, 4)
    assert e.value.code == -1
    with pytest.raises(rewl.RewlError) as e:
        rewl.rewl_get_grid_cap(None)
    assert e.value.code == -1
    assert ctypes.sizeof(rewl.rewl_tune_entry) == 32
    assert rewl.rewl_tune_entry.ms_per_segment.offset == 16
    assert rewl.rewl_tune_entry.max_blocks.offset == 24


def test_trace_record_layout():
    from paper_1411_4212_amd import rewl
    import oracle
    assert rewl.TRACE_DTYPE.itemsize == 24
    assert rewl.TRACE_DTYPE == oracle.TRACE_DTYPE


def test_binding_fails_loudly_without_library(tmp_path):
    """No CPU fallback: importing the binding without librewl.so raises."""
    import os
    import shutil
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = tmp_path / "paper_1411_4212_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(root, "paper_1411_4212_amd", "rewl.py"), pkg / "rewl.py")
    (pkg / "__init__.py").write_text("")
    r = subprocess.run([sys.executable, "-c", "import paper_1411_4212_amd.rewl"], cwd=str(tmp_path),
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "librewl.so is not built" in r.stderr


def test_bench_measured_figures_are_documented():
    """The traffic and instruction-mix figures bench.py reports are keyed by
    the digest of the kernel sources they were measured on (a changed kernel
    reports null until measured again); every such entry must come with the
    profile summary under profiles/ that documents it (its digest and its
    scaled byte count)."""
    import glob
    import bench
    assert set(bench.MEASURED_TRAFFIC) == set(bench.MEASURED_ISSUE)
    docs = [open(p).read() for p in glob.glob(os.path.join(ROOT, "profiles", "*.md"))]
    for (digest, workload, res), nbytes in bench.MEASURED_TRAFFIC.items():
        assert res in ("lds", "hbm")
        m, e = ("%.3e" % nbytes).split("e")
        mark = "%se%d" % (m, int(e))                         # e.g. 5.596e6, 5.015e10
        assert any(digest in d and mark in d for d in docs), (digest, workload, mark)
