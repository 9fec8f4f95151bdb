"""CPU test of the library's host-side Fermi-Dirac expansion (its own FFT)
against the oracle's (numpy's FFT) and against the Fermi function itself:
tests/host_fermi_check.cpp is compiled against host.cpp and run for a few
temperatures and chemical potentials."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("host_fermi") / "host_fermi_check")
    cmd = [hipcc, "-O2", "-std=c++17", "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "host_fermi_check.cpp"),
           os.path.join(ROOT, "paper_2209_00806_amd", "csrc", "host.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return out


def _run(checker, tmp_path, beta, mu, f, tol):
    out = os.path.join(str(tmp_path), "a.bin")
    r = subprocess.run([checker, repr(beta), repr(mu), repr(f), repr(tol), out], capture_output=True, timeout=120)
    return r.returncode, (np.fromfile(out, dtype=np.float64) if r.returncode == 0 else None)


@pytest.mark.parametrize("beta,mu,f", [(38.68, 0.0, 9.1), (10.0, -0.5, 8.3), (2.0, 1.7, 12.0), (400.0, 0.25, 9.0)])
def test_fermi_coefficients_match_oracle_and_function(checker, tmp_path, beta, mu, f):
    tol = 1e-13
    rc, a = _run(checker, tmp_path, beta, mu, f, tol)
    assert rc == 0
    ref = oracle.fermi_coeffs(beta, mu, f, tol, n_max=1 << 20)
    # same truncation reading; a coefficient within rounding of tol may land on
    # either side, so compare the common part and bound the rest by tol
    k = min(a.size, ref.size)
    assert abs(a.size - ref.size) <= 2
    assert np.max(np.abs(a[:k] - ref[:k])) < 1e-13
    assert np.all(np.abs(a[k:]) < 2 * tol) and np.all(np.abs(ref[k:]) < 2 * tol)
    # the series itself reproduces the Fermi function away from the
    # truncation scale (Chebyshev sum by the three-term recurrence)
    x = np.linspace(-0.999, 0.999, 801)
    t_prev, t_cur = np.ones_like(x), x.copy()
    s = a[0] * t_prev + (a[1] * t_cur if a.size > 1 else 0.0)
    for kk in range(2, a.size):
        t_prev, t_cur = t_cur, 2 * x * t_cur - t_prev
        s = s + a[kk] * t_cur
    assert np.max(np.abs(s - oracle.fermi(f * x, beta, mu))) < 1e-9


def test_fermi_expansion_declined_when_too_long(checker, tmp_path):
    # beta * rescale so large that more than 2^19 terms would be needed
    rc, _ = _run(checker, tmp_path, 1e7, 0.0, 10.0, 1e-13)
    assert rc == 3
