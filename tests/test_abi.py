"""The C-ABI library: it loads on a machine without a GPU, exports every
function that include/heff.h declares, the Python binding names the same
set, and host-side argument checks reject null handles without touching the
device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "heff.h")
LIB = os.path.join(ROOT, "paper_2501_18263_amd", "libheff.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(heff_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2501_18263_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_path():
    names = declared()
    for must in ("heff_create", "heff_build_blocks", "heff_apply", "heff_diag", "heff_dav_create",
                 "heff_davidson_step", "heff_truncate", "heff_batch_create", "heff_batch_apply"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header(lib):
    src = open(os.path.join(ROOT, "paper_2501_18263_amd", "heff.py")).read()
    used = set(re.findall(r"_lib\.(heff_\w+)", src))
    assert set(declared()) <= used | {"heff_debug_op"}, sorted(set(declared()) - used)


def test_null_handles_are_rejected(lib):
    # HEFF_EINVAL (-1) from pure host-side checks; no device call is made
    d = ctypes.c_double()
    n = ctypes.c_int64()
    assert lib.heff_task_stats_variant(None, 0, ctypes.byref(d), ctypes.byref(n)) != 0
    assert lib.heff_task_stats_issued(None, 0, ctypes.byref(d), ctypes.byref(n)) != 0
    assert lib.heff_apply(None, None, 0, None, None) != 0
    assert lib.heff_diag(None, None, None) != 0


def test_binding_loads_one_hip_runtime():
    # importing the binding first (before anything imports PyTorch) must
    # leave a single HIP runtime in the process: the library's
    # libamdhip64.so.7 dependency is served by PyTorch's bundled runtime.
    # (Loaded the other way round, the system runtime and PyTorch's copy
    # both load, and context creation then fails on the GPU.)
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2501_18263_amd import heff\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read()\n"
            "print(len({l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}))\n") % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == "1"
