"""GPU parity for quasi-eigenstates (Sec. "Quasieigenstates", Eq. (quasi))
through the C ABI against the oracle: the windowed Fourier transform of
psi(t) over positive and negative times at chosen energies, normalised.

Bars: FP64 max |d Psi| <= 1e-9 per (energy, state) on unit-norm states and
||Psi||^2 to 1e-10 relative; FP32 <= 1e-5."""
import math

import numpy as np
import pytest

import oracle
from paper_2209_00806_amd import inputs, tbpm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _complex_graphene(nx, ny, seed):
    rng = np.random.default_rng(seed)
    bi, bj, _, _ = inputs.graphene_bonds(nx, ny, pbc=True)
    bt = -2.7 * np.exp(1j * rng.uniform(0, 2 * np.pi, bi.shape[0]))
    ons = inputs.anderson(rng, 2 * nx * ny, 1.5)
    return inputs.from_bonds(2 * nx * ny, bi, bj, bt, ons)


CASES = {
    "graphene_s2": (lambda rng: inputs.graphene(21, 19, onsite=inputs.anderson(rng, 798, 1.0)), 2),
    "complex_s1": (lambda rng: _complex_graphene(15, 13, 6), 1),
    "tbg_s3": (lambda rng: inputs.twisted_bilayer(12, 12, angle_deg=4.0), 3),
}
ENERGIES = [-2.7, -0.31, 0.0, 1.234, 5.5]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("order,fused", [(0, 0), (1, 2)])
@pytest.mark.parametrize("case", sorted(CASES))
def test_quasi_eigenstates_vs_oracle(case, order, fused, precision):
    print(f"case quasi {case} order={order} fused={fused} {precision}", flush=True)
    rng = np.random.default_rng(93)
    make, S = CASES[case]
    lat = make(rng)
    psi0 = inputs.random_phase_states(rng, lat.n_orb, S)
    f = oracle.gershgorin(lat.row_ptr, lat.val, lat.onsite) * 1.02
    dt = math.pi / f
    nt = 48
    ref, ref_n2 = oracle.quasi_eigenstates(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f, ENERGIES)
    H = tbpm.Hamiltonian.from_lattice(lat)
    H.set_row_order(order)
    H.set_launch_config(2, 1, 1, 1, fused=fused)
    got, n2 = tbpm.quasi_eigenstates(H, _dev(psi0), ENERGIES, nt, dt, f, precision=precision, return_norm=True)
    got = got.cpu().numpy()
    n2 = n2.cpu().numpy()
    bar = 1e-9 if precision == "fp64" else 1e-5
    for j in range(len(ENERGIES)):
        for s in range(S):
            assert np.max(np.abs(got[j][:, s] - ref[j][:, s])) < bar, (j, s)
    assert np.max(np.abs(n2 - ref_n2) / ref_n2) < (1e-10 if precision == "fp64" else 1e-5)
    assert np.allclose(np.linalg.norm(got, axis=1), 1.0)


def test_quasi_eigenstates_no_window_and_repeat():
    """Rectangular window, and a second call with other energies and steps on
    the same handle."""
    print("case quasi no window", flush=True)
    rng = np.random.default_rng(94)
    lat = inputs.graphene(17, 16, onsite=inputs.anderson(rng, 544, 0.5))
    psi0 = inputs.random_phase_states(rng, lat.n_orb, 1)
    f = oracle.gershgorin(lat.row_ptr, lat.val, lat.onsite) * 1.02
    dt = math.pi / f
    H = tbpm.Hamiltonian.from_lattice(lat)
    for nt, en, win in ((32, [0.7, -1.1], "none"), (64, [2.2], "hann")):
        ref, _ = oracle.quasi_eigenstates(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f, en, kind=win)
        got = tbpm.quasi_eigenstates(H, _dev(psi0), en, nt, dt, f, window=win).cpu().numpy()
        assert np.max(np.abs(got - ref)) < 1e-9


def test_quasi_eigenstate_argument_errors():
    lat = inputs.graphene(4, 4)
    H = tbpm.Hamiltonian.from_lattice(lat)
    psi0 = _dev(inputs.random_phase_states(np.random.default_rng(1), lat.n_orb, 1))
    with pytest.raises(tbpm.TBPMError):
        tbpm.quasi_eigenstates(H, psi0, [], 16, 0.3, 9.0)
    with pytest.raises(tbpm.TBPMError):
        tbpm.quasi_eigenstates(H, psi0, [float("nan")], 16, 0.3, 9.0)
    with pytest.raises(tbpm.TBPMError):
        tbpm.quasi_eigenstates(H, psi0, np.zeros(257), 16, 0.3, 9.0)
