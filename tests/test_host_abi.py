"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
and its host-side logic (Bessel coefficients, truncation rule, input
validation) is right.  No compute call is made (there is no GPU here);
invalid inputs are rejected on the host before any device call."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2209_00806_amd import inputs, tbpm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "tbpm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tbpm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = tbpm.lib()
    names = _declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert "gfx950" in tbpm.version()


def test_launch_config_struct_matches_header():
    text = open(os.path.join(ROOT, "include", "tbpm.h")).read()
    body = re.search(r"typedef struct \{([^}]*)\} tbpm_launch_config;", text).group(1)
    fields = re.findall(r"int32_t\s+(\w+);", body)
    assert fields == [f[0] for f in tbpm.LaunchConfig._fields_]
    assert ctypes.sizeof(tbpm.LaunchConfig) == 4 * len(fields)


@pytest.mark.parametrize("z", [math.pi / 2, math.pi, 2 * math.pi, 10.3, 37.0, -2.5, 1e-9])
def test_library_bessel_vs_oracle(z):
    M = 60
    got = tbpm.bessel_j(z, M)
    ref = np.array([oracle.bessel_j(m, abs(z)) * ((-1) ** m if z < 0 else 1) for m in range(M)])
    assert np.max(np.abs(got - ref)) < 2e-16 * max(1.0, abs(z)) ** 0.5 * 4


@pytest.mark.parametrize("z,tol", [(math.pi, 1e-12), (2 * math.pi, 1e-12), (math.pi, 1e-16), (0.01, 1e-12),
                                   (1e-14, 1e-12), (25.0, 1e-10), (9.5 * math.pi / 9.0, 1e-12)])
def test_library_num_terms_matches_oracle(z, tol):
    assert tbpm.num_terms(z, tol) == oracle.n_terms(z, tol)


def _create(n, rp, col, val, ons):
    return tbpm.Hamiltonian(n, rp, col, val, ons)


def _expect(status_name, *args):
    with pytest.raises(tbpm.TBPMError) as ei:
        _create(*args)
    assert ei.value.name == status_name, str(ei.value)


def test_create_rejects_non_hermitian():
    lat = inputs.graphene(3, 3)
    val = lat.val.copy()
    val[5] *= 1.5
    _expect("TBPM_E_NOT_HERMITIAN", lat.n_orb, lat.row_ptr, lat.col, val, lat.onsite)
    # complex element whose partner is not its conjugate
    val = lat.val.copy()
    val[0] = val[0] + 0.3j
    _expect("TBPM_E_NOT_HERMITIAN", lat.n_orb, lat.row_ptr, lat.col, val, lat.onsite)


def test_create_rejects_missing_partner():
    rp = np.array([0, 1, 1], dtype=np.int64)
    _expect("TBPM_E_NOT_HERMITIAN", 2, rp, np.array([1], np.int32), np.array([1.0 + 0j]), np.zeros(2))


def test_create_rejects_bad_csr():
    lat = inputs.graphene(2, 2)
    rp = lat.row_ptr.copy()
    rp[3], rp[4] = rp[4], rp[3]
    _expect("TBPM_E_CSR", lat.n_orb, rp, lat.col, lat.val, lat.onsite)
    col = lat.col.copy()
    col[0] = lat.n_orb
    _expect("TBPM_E_CSR", lat.n_orb, lat.row_ptr, col, lat.val, lat.onsite)
    col = lat.col.copy()
    col[0] = 0  # row 0 diagonal
    _expect("TBPM_E_CSR", lat.n_orb, lat.row_ptr, col, lat.val, lat.onsite)
    rp = lat.row_ptr.copy()
    rp[0] = 1
    _expect("TBPM_E_CSR", lat.n_orb, rp, lat.col, lat.val, lat.onsite)


def test_create_rejects_non_finite_and_bad_sizes():
    lat = inputs.graphene(2, 2)
    val = lat.val.copy()
    val[2] = np.nan
    _expect("TBPM_E_ARG", lat.n_orb, lat.row_ptr, lat.col, val, lat.onsite)
    ons = lat.onsite.copy()
    ons[1] = np.inf
    _expect("TBPM_E_ARG", lat.n_orb, lat.row_ptr, lat.col, lat.val, ons)
    L = tbpm.lib()
    h = ctypes.c_void_p()
    assert L.tbpm_hamiltonian_create(0, None, None, None, None, 0, ctypes.byref(h)) == 1
    assert L.tbpm_hamiltonian_create(-5, None, None, None, None, 0, ctypes.byref(h)) == 1
    assert L.tbpm_hamiltonian_create(4, None, None, None, None, 0, None) == 1
    # unknown flags, and device pointers that are not device memory (host
    # arrays, NULL): refused on the host before any copy
    rp = np.array([0, 1, 2], dtype=np.int64)
    ci = np.array([1, 0], dtype=np.int32)
    va = np.array([1.0, 0.0, 1.0, 0.0])
    on = np.zeros(2)
    assert L.tbpm_hamiltonian_create(2, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, on.ctypes.data, 0x80,
                                     ctypes.byref(h)) == 1
    assert L.tbpm_hamiltonian_create(2, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, on.ctypes.data, 1,
                                     ctypes.byref(h)) == 1
    assert "device memory" in L.tbpm_last_error().decode()
    assert L.tbpm_hamiltonian_create(2, None, None, None, None, 1, ctypes.byref(h)) == 1
    assert not h.value


def test_entry_points_reject_null_and_bad_arguments():
    L = tbpm.lib()
    m = ctypes.c_int32()
    assert L.tbpm_num_terms(1.0, 0.0, ctypes.byref(m)) == 1
    assert L.tbpm_num_terms(float("nan"), 1e-12, ctypes.byref(m)) == 1
    assert L.tbpm_propagate(None, None, 1, 1, 0.1, 9.0, 1e-12, 0, None, None, 0, None, 0, None) == 1
    assert L.tbpm_dos(None, 4, 1, 0.1, 0, None, None, None) == 1
    assert L.tbpm_backward(None, None, 1, 1, 0.1, 9.0, 1e-12, None, 1, None, None, None, None) == 1
    assert L.tbpm_batch_create(None, 0, ctypes.byref(ctypes.c_void_p())) == 1
    assert L.tbpm_stream_copy(None, None, 16, None) == 1
    assert b"NULL" in L.tbpm_last_error() or len(L.tbpm_last_error()) > 0


def test_new_entry_points_reject_bad_arguments_on_the_host():
    """The entry points beyond the DOS validate their arguments before any
    device call (dummy non-NULL pointers are never dereferenced here)."""
    L = tbpm.lib()
    d = ctypes.c_void_p(64)
    assert L.tbpm_ac_cond(None, 8, 1, 0.1, 10.0, 1.0, 0, None, None, None) == 1
    assert L.tbpm_ac_cond(d, 8, 1, 0.1, 10.0, 0.0, 0, d, d, None) == 1          # area 0
    assert L.tbpm_ac_cond(d, 8, 1, 0.1, -1.0, 1.0, 0, d, d, None) == 1         # beta < 0
    assert L.tbpm_ac_corr(None, None, None, None, 1, 8, 0.1, 9.0, 1e-12, 10.0, 0.0, 1e-12, 0, None, 0, None) == 1
    assert L.tbpm_haydock(None, None, 1, 8, None, None, 0, None) == 1
    assert L.tbpm_haydock_ldos(d, d, 0, 1, d, 4, 0.1, d, None) == 1              # n_iter 0
    assert L.tbpm_haydock_ldos(d, d, 4, 1, d, 4, 0.0, d, None) == 1              # eps 0
    assert L.tbpm_kpm_moments(None, None, None, None, 1, 8, 4.0, None, None, None) == 1
    assert L.tbpm_kubo_bastin(d, 1, 4.0, -3.0, 3.0, 64, 10.0, d, 1, 1.0, d, d, d, None) == 1   # M < 2
    assert L.tbpm_kubo_bastin(d, 4097, 4.0, -3.0, 3.0, 64, 10.0, d, 1, 1.0, d, d, d, None) == 1  # M > LDS cap
    assert L.tbpm_kubo_bastin(d, 16, 4.0, -5.0, 3.0, 64, 10.0, d, 1, 1.0, d, d, d, None) == 1  # window
    assert L.tbpm_kubo_bastin(d, 16, 4.0, 3.0, -3.0, 64, 10.0, d, 1, 1.0, d, d, d, None) == 1  # e_lo > e_hi
    K = ctypes.c_int32()
    assert L.tbpm_fermi_cheb(-1.0, 0.0, 9.0, 1e-12, None, 0, ctypes.byref(K)) == 1
    assert L.tbpm_fermi_cheb(10.0, 0.0, 9.0, 0.5, None, 0, ctypes.byref(K)) == 1


@pytest.mark.parametrize("beta,mu", [(38.68, 0.0), (5.0, -1.2)])
def test_library_fermi_coefficients_vs_oracle(beta, mu):
    """tbpm_fermi_cheb (host; the library's own FFT) against the oracle's
    coefficients (NumPy's FFT) under the same truncation reading."""
    a = tbpm.fermi_coeffs(beta, mu, 9.0, 1e-13)
    ref = oracle.fermi_coeffs(beta, mu, 9.0, 1e-13, n_max=1 << 20)
    k = min(a.size, ref.size)
    assert abs(a.size - ref.size) <= 2
    assert np.max(np.abs(a[:k] - ref[:k])) < 1e-13


def test_header_is_plain_c_and_links(tmp_path):
    """include/tbpm.h is a C header: a C99 program (-pedantic, no C++)
    compiles against it, links libtbpm.so, and calls host-only entry points
    (version, Bessel coefficients, argument rejection) without a GPU."""
    import shutil
    import subprocess

    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    tbpm.lib()  # built
    src = tmp_path / "abi.c"
    src.write_text(
        '#include "tbpm.h"\n#include <math.h>\n#include <stdio.h>\n'
        "int main(void) {\n"
        "    double J[4];\n"
        "    int32_t M = 0;\n"
        "    if (!tbpm_version()) return 1;\n"
        "    if (tbpm_bessel_j(3.14159265358979, 4, J) != TBPM_OK) return 2;\n"
        "    if (tbpm_num_terms(3.14159265358979, 1e-12, &M) != TBPM_OK || M != 18) return 3;\n"
        "    if (tbpm_dos(0, 4, 1, 0.1, TBPM_WIN_HANN, 0, 0, 0) != TBPM_E_ARG) return 4;\n"
        '    printf("%.15f %d\\n", J[0], (int)M);\n'
        "    return 0;\n"
        "}\n")
    lib_dir = os.path.join(ROOT, "paper_2209_00806_amd")
    exe = str(tmp_path / "abi")
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", f"-I{os.path.join(ROOT, 'include')}",
                    str(src), f"-L{lib_dir}", "-ltbpm", f"-Wl,-rpath,{lib_dir}", "-lm", "-o", exe],
                   check=True, capture_output=True, timeout=120)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    j0, m = r.stdout.split()
    assert abs(float(j0) - oracle.bessel_j(0, math.pi)) < 1e-14 and int(m) == 18
