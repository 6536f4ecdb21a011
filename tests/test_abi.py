"""The C-ABI library loads and exports every function include/riann.h
declares (no GPU needed: nothing is called that touches a device)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "riann.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(riann_[a-z_]+)\s*\(", src)))


def test_header_declares_expected_calls():
    names = declared_functions()
    for n in ("riann_build", "riann_match_frame", "riann_full_search", "riann_match_batch",
              "riann_footprint", "riann_get_stats", "riann_save", "riann_load",
              "riann_destroy", "riann_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1508_07953_amd as r
    lib = ctypes.CDLL(r.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), f"{n} not exported"
    assert sorted(r.EXPORTS) == declared_functions()
    assert r.lib().riann_version() >> 16 == 1


def test_host_only_calls():
    """Calls that touch no device: footprint and argument checks."""
    import paper_1508_07953_amd as r
    b = r.footprint(16384, 16, 8, 1, 1, 720, 1280)
    assert b > 16384 * 64 and b < 200 * 2**20
    p = r.make_params(10, 2, 20, 1, 1)           # D = 400 > 256
    out = ctypes.c_int64()
    assert r.lib().riann_footprint(ctypes.byref(p), 0, 0, ctypes.byref(out)) == \
        r.RIANN_E_UNSUPPORTED
    assert b"256" in r.lib().riann_last_error()
    p = r.make_params(10, 11, 8, 1, 1)           # more keys than references
    assert r.lib().riann_footprint(ctypes.byref(p), 0, 0, ctypes.byref(out)) == \
        r.RIANN_E_INVALID


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the package before torch must not load a second HIP
    runtime beside torch's (the library binds to the one torch loads)."""
    import subprocess
    import sys
    code = ("import paper_1508_07953_amd, torch\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"
