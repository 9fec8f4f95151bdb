"""The library's host code (CSR ingest, sliced-ELL build, row order, two-hop
tile tables, Fermi-Dirac coefficients) built with AddressSanitizer and UBSan
by the host compiler, and the row order's threads also with ThreadSanitizer,
and run on seeded inputs (CPU only; the device code is not involved).  Any
sanitizer report fails the test."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from tests import test_host_tables as tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "paper_2209_00806_amd", "csrc", "host.cpp")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _build(tmp, main, sanitizers="address,undefined"):
    cxx = shutil.which("g++")
    if not cxx or not os.path.exists("/opt/rocm/lib/libamdhip64.so"):
        pytest.skip("g++ or the HIP runtime library is not available")
    out = os.path.join(tmp, os.path.splitext(os.path.basename(main))[0] + "_" + sanitizers.replace(",", "_"))
    cmd = [cxx, "-O1", "-g", "-std=c++17", f"-fsanitize={sanitizers}", "-fno-omit-frame-pointer",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", os.path.join(ROOT, "tests", main), HOST,
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return out


def _clean(r):
    text = r.stdout + r.stderr
    assert "runtime error" not in text and "AddressSanitizer" not in text and "LeakSanitizer" not in text, text


def test_csr_ingest_ell_and_order_under_sanitizers(tmp_path):
    exe = _build(str(tmp_path), "host_csr_check.cpp")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    _clean(r)
    assert r.returncode == 0, r.stdout + r.stderr
    ok, rejected, orders = int(r.stdout.split()[1]), int(r.stdout.split()[3]), int(r.stdout.split()[5])
    assert ok > 300 and rejected > 0 and orders == 3


def test_threaded_host_code_under_thread_sanitizer(tmp_path):
    """The same sweep built with ThreadSanitizer (the row order's worker
    threads share the row arrays of disjoint parts; the ingest's chunks share
    the input), then the two-hop tile tables of a lattice large enough to be
    built on threads; any reported race fails the test."""
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    exe = _build(str(tmp_path), "host_csr_check.cpp", "thread")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert "ThreadSanitizer" not in r.stdout + r.stderr, r.stdout + r.stderr
    assert r.returncode == 0, r.stdout + r.stderr
    assert int(r.stdout.split()[5]) == 3
    # the two-hop tile tables of a lattice large enough to be built on threads
    exe = _build(str(tmp_path), "host_tables_check.cpp", "thread")
    paths = tables._write(tempfile.mkdtemp(dir=str(tmp_path)), [tables.inputs.graphene(420, 420)])
    r = subprocess.run([exe, *paths, "1", "2", "32", "2"], capture_output=True, text=True, timeout=600, env=env)
    assert "ThreadSanitizer" not in r.stdout + r.stderr, r.stdout + r.stderr
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr


def test_tile_tables_under_sanitizers(tmp_path):
    exe = _build(str(tmp_path), "host_tables_check.cpp")
    for name in ("tbg_12x12", "batch_5"):
        paths = tables._write(tempfile.mkdtemp(dir=str(tmp_path)), tables.CASES[name]())
        for order in (0, 1):
            for log2u, ub in tables.WIDTHS[:3]:
                r = subprocess.run([exe, *paths, str(order), str(log2u), str(ub), "2"], capture_output=True,
                                   text=True, timeout=300, env=ENV)
                _clean(r)
                assert r.returncode in (0, 3), (name, order, log2u, ub, r.stdout, r.stderr)


def test_fermi_coefficients_under_sanitizers(tmp_path):
    exe = _build(str(tmp_path), "host_fermi_check.cpp")
    for beta, mu, f, tol in ((38.68, 0.0, 9.0, 1e-12), (5.0, -1.2, 9.0, 1e-13), (1e7, 0.0, 10.0, 1e-13)):
        out = os.path.join(str(tmp_path), "a.bin")
        r = subprocess.run([exe, repr(beta), repr(mu), repr(f), repr(tol), out], capture_output=True, text=True,
                           timeout=300, env=ENV)
        _clean(r)
        assert r.returncode in (0, 3), r.stdout + r.stderr
        if r.returncode == 0:
            assert np.all(np.isfinite(np.fromfile(out, dtype=np.float64)))
