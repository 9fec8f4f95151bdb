"""GPU tests of tbpm_propagate_noalloc, the entry point that allocates no
device memory: its correlation and norms against tbpm_propagate's (the same
kernels in the plain launch shape) and against the oracle, on two calls in a
row with the second on a smaller input, in FP64 and FP32-mixed; its size
limit; and replays of a captured HIP graph of one call.

Bars: FP64 within 1e-12 of tbpm_propagate (identical kernels and launch
shape) and 1e-10 of the oracle, normwise over C; FP32-mixed within 1e-12 of
tbpm_propagate's FP32-mixed run and 1e-5 of the FP64 oracle.
"""
import ctypes
import math

import numpy as np
import pytest

import oracle
from paper_2209_00806_amd import inputs, tbpm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PLAIN = dict(wg_chunks=2, xcd_remap=1, nontemporal=1, unroll=1, staged=0, fused=0)


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _case(lat, S, nt, seed):
    psi0 = inputs.random_phase_states(np.random.default_rng(seed), lat.n_orb, S)
    f = max(oracle.gershgorin(lat.row_ptr, lat.val, lat.onsite), 1e-3) * 1.05
    return psi0, f, math.pi / f


def _noalloc_raw(H, psi0_d, nt, dt, f, prec, corr, norm2):
    """One call straight through the C ABI (ctypes), on torch's current stream."""
    S = psi0_d.shape[1]
    st = tbpm.lib().tbpm_propagate_noalloc(H.handle, psi0_d.data_ptr(), S, nt, dt, f, 1e-12, prec,
                                           corr.data_ptr(), 0 if norm2 is None else norm2.data_ptr(),
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, tbpm.lib().tbpm_last_error().decode()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_calls_against_propagate_and_oracle(precision):
    prec = tbpm.FP64 if precision == "fp64" else tbpm.FP32_MIXED
    cases = [  # second call smaller: fewer orbitals, states and steps
        ("graphene 40x36 disordered, S=3", inputs.graphene(40, 36, onsite=inputs.anderson(np.random.default_rng(11),
                                                                                         2 * 40 * 36, 1.0)), 3, 48),
        ("square 9x7 open, S=1", inputs.square(9, 7, pbc=False,
                                               onsite=inputs.anderson(np.random.default_rng(12), 63, 2.0)), 1, 20),
    ]
    for label, lat, S, nt in cases:
        print(f"case noalloc {precision} {label} nt={nt}", flush=True)
        psi0, f, dt = _case(lat, S, nt, seed=5)
        H = tbpm.Hamiltonian.from_lattice(lat)
        H.set_launch_config(**PLAIN)
        psi0_d = torch.from_numpy(psi0).cuda()
        corr = torch.full((nt, S), complex("nan+nanj"), dtype=torch.complex128, device="cuda")
        norm2 = torch.full((nt, S), float("nan"), dtype=torch.float64, device="cuda")
        _noalloc_raw(H, psi0_d, nt, dt, f, prec, corr, norm2)
        torch.cuda.synchronize()
        got, got_n = corr.cpu().numpy(), norm2.cpu().numpy()
        ref_c, ref_n = tbpm.propagate(H, psi0_d, nt, dt, f, precision=precision, return_norm=True)
        ref_c, ref_n = ref_c.cpu().numpy(), ref_n.cpu().numpy()
        ora, ora_n, _ = oracle.propagate(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f)
        assert np.all(np.isfinite(got)) and np.all(np.isfinite(got_n))
        assert _rel(got, ref_c) < 1e-12
        assert np.max(np.abs(got_n - ref_n)) < 1e-12
        bar = 1e-10 if prec == tbpm.FP64 else 1e-5
        assert _rel(got, ora) < bar
        assert np.max(np.abs(got_n - ora_n)) < bar
        H.close()


def test_without_norm_and_row_order():
    """norm2 = NULL, and a Hamiltonian renumbered on the device (bisection
    row order): the correlation matches tbpm_propagate on the same handle."""
    lat = inputs.graphene(96, 96, onsite=inputs.anderson(np.random.default_rng(13), 2 * 96 * 96, 1.0))
    S, nt = 2, 16
    psi0, f, dt = _case(lat, S, nt, seed=9)
    H = tbpm.Hamiltonian.from_lattice(lat)
    H.set_row_order(1)
    assert H.row_order() == 1
    H.set_launch_config(**PLAIN)
    psi0_d = torch.from_numpy(psi0).cuda()
    print("case noalloc bisection order, norm2 NULL", flush=True)
    got = tbpm.propagate_noalloc(H, psi0_d, nt, dt, f)
    torch.cuda.synchronize()
    ref = tbpm.propagate(H, psi0_d, nt, dt, f).cpu().numpy()
    assert _rel(got.cpu().numpy(), ref) < 1e-12
    H.close()


def test_size_limit_is_an_argument_error():
    """Work memory beyond the fixed scratch is refused before any work."""
    lat = inputs.graphene(256, 256)  # 131072 orbitals x 8 states x 64 B > 64 MiB
    H = tbpm.Hamiltonian.from_lattice(lat)
    psi0 = torch.zeros((lat.n_orb, 8), dtype=torch.complex128, device="cuda")
    psi0[:, :] = 1.0 / math.sqrt(lat.n_orb)
    with pytest.raises(tbpm.TBPMError) as e:
        tbpm.propagate_noalloc(H, psi0, 4, math.pi / 9.0, 9.0)
    assert e.value.name == "TBPM_E_ARG" and "no-allocation" in str(e.value)
    # the same size with one state fits
    got = tbpm.propagate_noalloc(H, psi0[:, :1].contiguous(), 4, math.pi / 9.0, 9.0)
    torch.cuda.synchronize()
    assert abs(got[0, 0].item() - 1.0) < 1e-12
    H.close()


def test_captured_graph_replays():
    """One call captured in a HIP graph (torch.cuda.graph): every replay,
    with eager work and synchronisations between replays, gives the eager
    result bit for bit."""
    lat = inputs.graphene(24, 20, onsite=inputs.anderson(np.random.default_rng(14), 960, 1.0))
    S, nt = 2, 24
    psi0, f, dt = _case(lat, S, nt, seed=4)
    H = tbpm.Hamiltonian.from_lattice(lat)
    H.set_launch_config(**PLAIN)
    psi0_d = torch.from_numpy(psi0).cuda()
    corr = torch.zeros((nt, S), dtype=torch.complex128, device="cuda")
    norm2 = torch.zeros((nt, S), dtype=torch.float64, device="cuda")
    print("case noalloc eager", flush=True)
    tbpm.propagate_noalloc(H, psi0_d, nt, dt, f, corr=corr, norm2=norm2)
    torch.cuda.synchronize()
    eager_c, eager_n = corr.cpu().numpy().copy(), norm2.cpu().numpy().copy()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    print("case noalloc capture", flush=True)
    with torch.cuda.graph(g, stream=s):
        tbpm.propagate_noalloc(H, psi0_d, nt, dt, f, corr=corr, norm2=norm2)
    torch.cuda.synchronize()
    for rep in range(3):
        corr.zero_()
        norm2.zero_()
        torch.cuda.synchronize()
        print(f"case noalloc replay {rep}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(corr.cpu().numpy(), eager_c)
        assert np.array_equal(norm2.cpu().numpy(), eager_n)
        # unrelated eager work on the same handle between replays
        tbpm.propagate(H, psi0_d, 8, dt, f)
    del g
    H.close()
