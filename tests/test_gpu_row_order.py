"""GPU checks of the internal row order (recursive-bisection renumbering):
everything that crosses the C ABI stays in the caller's orbital order, so a
handle propagated with the renumbered rows must agree with one that keeps
the caller's order (same arithmetic up to summation order within a row) and
with the oracle, for correlations, norms, checkpoints, gradients, device-side
value updates and batches."""
import math

import numpy as np
import pytest

import oracle
from paper_2209_00806_amd import inputs, tbpm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _complex_graphene(nx, ny, seed):
    rng = np.random.default_rng(seed)
    bi, bj, _, _ = inputs.graphene_bonds(nx, ny, pbc=True)
    bt = -2.7 * np.exp(1j * rng.uniform(0, 2 * np.pi, bi.shape[0]))
    ons = inputs.anderson(rng, 2 * nx * ny, 1.5)
    return inputs.from_bonds(2 * nx * ny, bi, bj, bt, ons)


CASES = {
    "graphene_s4": (lambda rng: inputs.graphene(40, 37, onsite=inputs.anderson(rng, 2960, 1.0)), 4),
    "complex_s3": (lambda rng: _complex_graphene(23, 19, 9), 3),
    "square_open_s1": (lambda rng: inputs.square(45, 31, pbc=False, onsite=inputs.anderson(rng, 1395, 2.0)), 1),
    "tbg_s2": (lambda rng: inputs.twisted_bilayer(16, 16, angle_deg=3.0), 2),
    "dimer_s2": (lambda rng: inputs.from_bonds(2, np.array([0]), np.array([1]), np.array([1.7]),
                                               np.array([0.2, -0.1])), 2),
}


@pytest.mark.parametrize("fused", [0, 1])
@pytest.mark.parametrize("case", sorted(CASES))
def test_renumbered_rows_match_caller_order(case, fused):
    print(f"case row order {case} fused={fused}", flush=True)
    rng = np.random.default_rng(61)
    make, S = CASES[case]
    lat = make(rng)
    psi0 = inputs.random_phase_states(rng, lat.n_orb, S)
    f = max(oracle.gershgorin(lat.row_ptr, lat.val, lat.onsite), 1e-3) * 1.02
    dt = math.pi / f
    nt = 40
    ref, ref_n2, _ = oracle.propagate(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f)
    H = tbpm.Hamiltonian.from_lattice(lat)
    res = {}
    for order in (0, 1):
        H.set_row_order(order)
        assert H.row_order() == (order if lat.n_orb >= 2 else 0)
        H.set_launch_config(2, 1, 1, 1, vec=min(2, 1 << (S.bit_length() - 1)), fused=fused)
        corr, n2, ck = tbpm.propagate(H, _dev(psi0), nt, dt, f, return_norm=True, ckpt_every=5)
        res[order] = (corr.cpu().numpy(), n2.cpu().numpy(), ck.cpu().numpy())
    for order in (0, 1):
        assert _rel(res[order][0], ref) < 1e-10, order
        assert np.max(np.abs(res[order][1] - ref_n2)) < 1e-10
    assert _rel(res[1][0], res[0][0]) < 1e-13
    # checkpoints are psi(m K dt) in the caller's order either way
    assert _rel(res[1][2], res[0][2]) < 1e-13


def test_renumbered_rows_backward_and_device_values():
    """Gradients (values in CSR order, on-site energies in orbital order) and a
    device-side value update agree between the two orders."""
    print("case row order backward", flush=True)
    rng = np.random.default_rng(62)
    lat = _complex_graphene(21, 17, 4)
    S, nt, K = 2, 24, 4
    psi0 = inputs.random_phase_states(rng, lat.n_orb, S)
    f = oracle.gershgorin(lat.row_ptr, lat.val, lat.onsite) * 1.05
    dt = math.pi / f
    g = _dev(rng.standard_normal((nt, S)) + 1j * rng.standard_normal((nt, S)))
    # a Hermitian perturbation with a different value on every element
    import scipy.sparse as sp

    n = lat.n_orb
    rows = np.repeat(np.arange(n), np.diff(lat.row_ptr))
    noise = sp.csr_matrix((rng.standard_normal(lat.nnz) + 1j * rng.standard_normal(lat.nnz), lat.col, lat.row_ptr),
                          shape=(n, n))
    herm = (noise + noise.conj().T) * 0.5
    new_val_h = lat.val + 0.02 * np.asarray(herm[rows, lat.col]).ravel()
    new_ons_h = lat.onsite + 0.05 * rng.standard_normal(n)
    new_val = _dev(new_val_h)
    new_ons = _dev(new_ons_h)
    out = {}
    for order in (0, 1):
        H = tbpm.Hamiltonian.from_lattice(lat)
        H.set_row_order(order)
        assert H.row_order() == order
        corr, ck = tbpm.propagate(H, _dev(psi0), nt, dt, f, ckpt_every=K)
        gval, gons = tbpm.backward(H, _dev(psi0), nt, dt, f, g, K, ck)
        H.set_values(new_val, new_ons)
        corr2 = tbpm.propagate(H, _dev(psi0), nt, dt, f)
        out[order] = [x.cpu().numpy() for x in (corr, gval, gons, corr2)]
        H.close()
    for a, b in zip(out[1], out[0]):
        assert _rel(a, b) < 1e-12
    rp, col = lat.row_ptr, lat.col
    ref2, _, _ = oracle.propagate(rp, col, new_val_h, new_ons_h, psi0, nt, dt, f)
    assert _rel(out[1][3], ref2) < 1e-10


def test_batch_members_keep_their_order():
    print("case row order batch", flush=True)
    rng = np.random.default_rng(63)
    lats = [inputs.graphene(19, 13, onsite=inputs.anderson(rng, 494, 1.0)), inputs.square(23, 11),
            inputs.twisted_bilayer(10, 10, angle_deg=5.0)]
    psis = [inputs.random_phase_states(rng, l.n_orb, 4) for l in lats]
    fs = [oracle.gershgorin(l.row_ptr, l.val, l.onsite) * 1.02 for l in lats]
    dts = [math.pi / f for f in fs]
    hams = [tbpm.Hamiltonian.from_lattice(l) for l in lats]
    hams[0].set_row_order(1)
    hams[2].set_row_order(1)
    B = tbpm.Batch(hams)
    for fused in (0, 1):
        B.set_launch_config(2, 1, 1, 1, fused=fused)
        corrs = B.propagate([_dev(p) for p in psis], 32, dts, fs)
        for l, p, f, dt, c in zip(lats, psis, fs, dts, corrs):
            ref, _, _ = oracle.propagate(l.row_ptr, l.col, l.val, l.onsite, p, 32, dt, f)
            assert _rel(c.cpu().numpy(), ref) < 1e-10


def test_automatic_order_renumbers_strip_ordered_graphene():
    """Graphene numbered cell by cell (strips) is renumbered automatically
    above the size threshold; a small Hamiltonian keeps the caller's order."""
    print("case row order automatic", flush=True)
    big = tbpm.Hamiltonian.from_lattice(inputs.graphene(128, 96))
    assert big.row_order() == 1
    small = tbpm.Hamiltonian.from_lattice(inputs.graphene(20, 20))
    assert small.row_order() == 0
