"""CPU-side checks of the C ABI: the library loads, exports every function that
include/lpa.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lpa.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lpa_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2411_11468_amd import lpa
    return lpa.load_library()


def test_header_declares_the_core_calls():
    names = _declared_functions()
    for f in ("lpa_create", "lpa_run", "lpa_modularity", "lpa_destroy",
              "lpa_status_string", "lpa_last_error", "lpa_get_flags"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2411_11468_amd import lpa
    assert sorted(lpa.EXPORTED) == _declared_functions()


def test_struct_layouts_match_header():
    from paper_2411_11468_amd import lpa
    # sizes implied by the header's field lists on LP64
    assert ctypes.sizeof(lpa.lpa_csr) == 8 + 8 + 4 + 4 + 8 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(lpa.lpa_tuning) == 19 * 4
    assert ctypes.sizeof(lpa.lpa_options) == 4 + 4 + 8 + 4 + 4 + 8 + 4 + 4 + 4 + 4 + 4 + 4
    assert ctypes.sizeof(lpa.lpa_kernel_profile) == 24 + 8 + 8 + 8 + 8 + 8
    assert ctypes.sizeof(lpa.lpa_iter_stats) == 4 + 4 + 8 + 8 + 8 + 4 + 4
    assert ctypes.sizeof(lpa.lpa_train_options) == 4 + 4 + 4 + 4 + 8


def test_defaults(lib):
    from paper_2411_11468_amd import lpa
    o = lpa.default_options()
    assert (o.mode, o.max_iterations, o.tolerance, o.pl_period, o.prune) == \
        (lpa.MODE_ASYNC, 20, 0.05, 4, 1)
    t = lpa.default_tuning()
    assert (t.small4, t.small16, t.wave, t.block, t.hub_chunk, t.max_retries, t.xcd_local,
            t.hub_table_cap, t.relabel, t.probe, t.table_values) == \
        (4, 16, 512, 8192, 8192, 32, 3, 0, -1, 0, 0)


def test_status_strings(lib):
    assert lib.lpa_status_string(0) == b"ok"
    assert lib.lpa_status_string(1) == b"invalid argument"
    assert lib.lpa_status_string(99) == b"unknown status"


def test_null_arguments_rejected_without_gpu(lib):
    from paper_2411_11468_amd import lpa
    h = ctypes.c_void_p(123)
    assert lib.lpa_create(None, None, None, ctypes.byref(h)) == 1
    assert h.value is None
    assert b"NULL" in lib.lpa_last_error()
    assert lib.lpa_run(None, None, None, None, 0, None) == 1
    assert lib.lpa_modularity(None, None, None) == 1
    assert lib.lpa_get_flags(None, None) == 1
    lib.lpa_destroy(None)
    g = lpa.lpa_csr()
    g.num_vertices = -1
    assert lib.lpa_create(ctypes.byref(g), None, None, ctypes.byref(h)) == 1
    g.num_vertices = 10
    g.num_edges = 1 << 31
    g.offset_type = lpa.INDEX_I32
    g.offsets = ctypes.c_void_p(1)
    g.targets = ctypes.c_void_p(1)
    assert lib.lpa_create(ctypes.byref(g), None, None, ctypes.byref(h)) == 1
    assert b"int32 offsets" in lib.lpa_last_error()


def test_product_path_has_no_oracle_dependency():
    # the library package must not import, load or call the oracle
    pkg = os.path.join(ROOT, "paper_2411_11468_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.lower(), f


def test_one_hip_runtime_per_process():
    """liblpa.so must bind to the HIP runtime torch uses (same soname, two
    copies on disk): loading it through the binding maps only one."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2411_11468_amd import lpa\n"
            "lpa.load_library()\n"
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'amdhip64' in l}))"
            % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"
