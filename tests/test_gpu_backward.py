"""GPU parity of the adjoint path (tbpm_dos_backward + tbpm_backward) against
the oracle's discrete adjoint, finite differences and exact identities."""
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
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(np.asarray(b))), 1e-300))


def _complex_graphene(nx, ny, seed):
    rng = np.random.default_rng(seed)
    bi, bj, _, _ = inputs.graphene_bonds(nx, ny, pbc=True)
    bt = -2.7 * np.exp(1j * rng.uniform(0, 2 * np.pi, bi.shape[0]))
    return inputs.from_bonds(2 * nx * ny, bi, bj, bt, inputs.anderson(rng, 2 * nx * ny, 1.5))


LATTICES = {
    "graphene5x4_disorder": lambda: inputs.graphene(5, 4, onsite=inputs.anderson(np.random.default_rng(1), 40, 1.0)),
    "graphene4x3_complex": lambda: _complex_graphene(4, 3, 3),
    "square6x5_open": lambda: inputs.square(6, 5, pbc=False, onsite=inputs.anderson(np.random.default_rng(2), 30, 1.0)),
    "tbg5x5": lambda: inputs.twisted_bilayer(5, 5, angle_deg=6.0),
}


@pytest.mark.parametrize("K", [5, 64])
@pytest.mark.parametrize("S", [1, 3])
@pytest.mark.parametrize("name", sorted(LATTICES))
def test_backward_vs_oracle(name, S, K):
    print(f"case backward {name} S={S} K={K}", flush=True)
    lat = LATTICES[name]()
    rng = np.random.default_rng(17)
    psi0 = inputs.random_phase_states(rng, lat.n_orb, S)
    nt = 23
    f = oracle.gershgorin(lat.row_ptr, lat.val, lat.onsite) * 1.05
    dt = math.pi / f
    g = rng.standard_normal((nt, S)) + 1j * rng.standard_normal((nt, S))
    gval_r, gons_r = oracle.backward(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f, g)
    H = tbpm.Hamiltonian.from_lattice(lat)
    p0 = _dev(psi0)
    corr, ckpt = tbpm.propagate(H, p0, nt, dt, f, ckpt_every=K)
    gval, gons = tbpm.backward(H, p0, nt, dt, f, _dev(g), K, ckpt)
    gval = gval.cpu().numpy()
    gons = gons.cpu().numpy()
    if H.info()["is_complex"]:
        assert _rel(gval, gval_r) < 1e-10
    else:
        assert _rel(gval.real, gval_r.real) < 1e-10
    assert _rel(gons, gons_r) < 1e-10


def test_backward_single_step_and_short_runs():
    print("case backward short", flush=True)
    lat = LATTICES["graphene5x4_disorder"]()
    rng = np.random.default_rng(3)
    psi0 = inputs.random_phase_states(rng, lat.n_orb, 2)
    f = 9.0
    dt = math.pi / f
    H = tbpm.Hamiltonian.from_lattice(lat)
    for nt in (1, 2, 3):
        g = rng.standard_normal((nt, 2)) + 1j * rng.standard_normal((nt, 2))
        gval_r, gons_r = oracle.backward(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f, g)
        corr, ckpt = tbpm.propagate(H, _dev(psi0), nt, dt, f, ckpt_every=1)
        gval, gons = tbpm.backward(H, _dev(psi0), nt, dt, f, _dev(g), 1, ckpt)
        if nt == 1:
            assert np.all(gval.cpu().numpy() == 0) and np.all(gons.cpu().numpy() == 0)
        else:
            assert _rel(gval.cpu().numpy().real, gval_r.real) < 1e-10
            assert _rel(gons.cpu().numpy(), gons_r) < 1e-10


def test_dos_loss_gradient_vs_oracle_chain_and_fd():
    """L = sum_j (D_j - target_j)^2 through the autograd function: against the
    oracle chain (dos_adjoint -> backward) and central finite differences of the
    GPU forward on bond parameters."""
    print("case dos loss gradient", flush=True)
    from paper_2209_00806_amd import autograd as ag

    rng = np.random.default_rng(5)
    nx = ny = 6
    n_b = 3 * nx * ny
    bt = -2.7 * (1 + 0.05 * rng.standard_normal(n_b))
    lat = inputs.graphene(nx, ny, bond_t=bt, keep_bonds=True)
    tgt = inputs.graphene(nx, ny, keep_bonds=True)
    psi0 = inputs.random_phase_states(rng, lat.n_orb, 2)
    nt, f = 96, 9.0
    dt = math.pi / f
    H = tbpm.Hamiltonian.from_lattice(lat)
    p0 = _dev(psi0)
    ref_corr, _, _ = oracle.propagate(tgt.row_ptr, tgt.col, tgt.val, tgt.onsite, psi0, nt, dt, f)
    _, target = oracle.dos(ref_corr, dt)
    target_t = _dev(target)
    slot_ij = _dev(lat.slot_ij)
    slot_ji = _dev(lat.slot_ji)

    def loss_of(t_bonds, eps):
        val = ag.bond_values(lat.nnz, slot_ij, slot_ji, t_bonds)
        E, D = ag.tbpm_dos(H, val, eps, p0, nt, dt, f, ckpt_every=16)
        return torch.sum((D - target_t) ** 2)

    t_param = _dev(bt).requires_grad_(True)
    e_param = _dev(lat.onsite.copy()).requires_grad_(True)
    L = loss_of(t_param, e_param)
    L.backward()
    gt = t_param.grad.cpu().numpy()
    ge = e_param.grad.cpu().numpy()

    # oracle chain
    corr_o, _, _ = oracle.propagate(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f)
    _, D_o = oracle.dos(corr_o, dt)
    gD = 2 * (D_o - target)
    gc = oracle.dos_adjoint(gD, nt, 2, dt)
    gval_o, gons_o = oracle.backward(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f, gc)
    gt_o = (gval_o[lat.slot_ij] + gval_o[lat.slot_ji]).real
    assert _rel(gt, gt_o) < 1e-9
    assert _rel(ge, gons_o) < 1e-9

    # central finite differences on sampled bonds (GPU forward)
    with torch.no_grad():
        for b in rng.choice(n_b, 8, replace=False):
            vals = []
            for sgn in (1, -1):
                tt = t_param.detach().clone()
                tt[b] += sgn * 1e-4
                vals.append(loss_of(tt, e_param.detach()).item())
            fd = (vals[0] - vals[1]) / 2e-4
            assert abs(fd - gt[b]) < 1e-6 * max(abs(gt).max(), 1e-12), (b, fd, gt[b])


def test_shift_identity_medium():
    """sum_i dL/deps_i = Re sum_k conj(g_k) (-i k dt) C_k (H + d I multiplies C_k by e^{-i d k dt})."""
    print("case shift identity", flush=True)
    rng = np.random.default_rng(6)
    lat = inputs.graphene(48, 40, onsite=inputs.anderson(rng, 2 * 48 * 40, 1.0))
    S, nt = 4, 200
    psi0 = inputs.random_phase_states(rng, lat.n_orb, S)
    f = 9.5
    dt = math.pi / f
    H = tbpm.Hamiltonian.from_lattice(lat)
    p0 = _dev(psi0)
    corr, ckpt = tbpm.propagate(H, p0, nt, dt, f, tol=1e-15, ckpt_every=32)
    g = rng.standard_normal((nt, S)) + 1j * rng.standard_normal((nt, S))
    gval, gons = tbpm.backward(H, p0, nt, dt, f, _dev(g), 32, ckpt, tol=1e-15)
    c = corr.cpu().numpy()
    k = np.arange(nt)[:, None]
    rhs = float(np.real(np.sum(np.conj(g) * (-1j * k * dt) * c)))
    lhs = float(gons.sum().item())
    assert abs(lhs - rhs) < 1e-9 * max(1.0, abs(rhs))


@pytest.mark.parametrize("M_dt", [1.0, 0.25, 0.12])
@pytest.mark.parametrize("tier,vec", [(1, 1), (2, 2), (4, 4), (3, 2)])
@pytest.mark.parametrize("name", ["graphene9x8_disorder", "graphene6x5_complex", "square9x7_open"])
def test_backward_fused_shape_vs_oracle(name, tier, vec, M_dt):
    """The backward with the fused shape in the launch configuration: the
    segment replay two Clenshaw orders per launch and the adjoint two orders
    per launch (first pair, middle pairs, leftover single orders and the last
    order) with 1, 2 or 4 states per thread, against the oracle's adjoint and
    the plain shape.  Time steps of
    pi/f, pi/(4f) and 0.12 pi/f give series of 18, 11 and 9 terms: 17, 10 and
    8 adjoint orders, with and without single orders left after the pairs."""
    print(f"case backward fused {name} tier={tier} vec={vec} dt={M_dt}", flush=True)
    rng = np.random.default_rng(23)
    lats = {
        "graphene9x8_disorder": lambda: inputs.graphene(9, 8, onsite=inputs.anderson(rng, 144, 1.0)),
        "graphene6x5_complex": lambda: _complex_graphene(6, 5, 4),
        "square9x7_open": lambda: inputs.square(9, 7, pbc=False, onsite=inputs.anderson(rng, 63, 1.0)),
    }
    lat = lats[name]()
    S = 5  # padded to 8: with 4 states per thread, two units per row
    psi0 = inputs.random_phase_states(rng, lat.n_orb, S)
    nt = 19
    f = oracle.gershgorin(lat.row_ptr, lat.val, lat.onsite) * 1.05
    dt = M_dt * math.pi / f
    g = rng.standard_normal((nt, S)) + 1j * rng.standard_normal((nt, S))
    gval_r, gons_r = oracle.backward(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f, g)
    H = tbpm.Hamiltonian.from_lattice(lat)
    p0 = _dev(psi0)
    out = {}
    for fused in (0, tier):
        H.set_launch_config(2, 1, 1, 1, vec=vec if fused else 1, precision="fp64", fused=fused)
        corr, ckpt = tbpm.propagate(H, p0, nt, dt, f, ckpt_every=5)
        gval, gons = tbpm.backward(H, p0, nt, dt, f, _dev(g), 5, ckpt)
        out[fused] = (gval.cpu().numpy(), gons.cpu().numpy())
    gval, gons = out[tier]
    cmp = gval if H.info()["is_complex"] else gval.real
    ref = gval_r if H.info()["is_complex"] else gval_r.real
    assert _rel(cmp, ref) < 1e-10
    assert _rel(gons, gons_r) < 1e-10
    assert _rel(gval, out[0][0]) < 1e-12 and _rel(gons, out[0][1]) < 1e-12


@pytest.mark.parametrize("fused", [0, 2])
@pytest.mark.parametrize("name", ["graphene24x20_disorder", "graphene10x9_complex"])
def test_backward_bench_segmentation_k64(name, fused):
    """Checkpoints every K = 64 steps, as the differentiable bench leg takes
    them: 130 samples (checkpoints at steps 64 and 128: three segments, the
    last of one step) and 1024 samples (15 checkpoints: the 16 segments of
    the bench leg), 4 states, in the default shape and in the bench's tuned
    fused shape (LDS tier 2, 2 states per thread), against the oracle's
    discrete adjoint (which stores every step and takes no checkpoints)."""
    print(f"case backward K=64 {name} fused={fused}", flush=True)
    rng = np.random.default_rng(29)
    lat = {"graphene24x20_disorder": lambda: inputs.graphene(24, 20, onsite=inputs.anderson(rng, 960, 1.0)),
           "graphene10x9_complex": lambda: _complex_graphene(10, 9, 8)}[name]()
    S, K = 4, 64
    psi0 = inputs.random_phase_states(rng, lat.n_orb, S)
    f = oracle.gershgorin(lat.row_ptr, lat.val, lat.onsite) * 1.05
    dt = math.pi / f
    H = tbpm.Hamiltonian.from_lattice(lat)
    if fused:
        H.set_launch_config(2, 1, 1, 1, vec=2, precision="fp64", fused=fused)
    p0 = _dev(psi0)
    cplx = H.info()["is_complex"]
    for nt in (130, 1024):
        g = rng.standard_normal((nt, S)) + 1j * rng.standard_normal((nt, S))
        gval_r, gons_r = oracle.backward(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f, g)
        corr, ckpt = tbpm.propagate(H, p0, nt, dt, f, ckpt_every=K)
        assert ckpt.shape[0] == (nt - 2) // K
        gval, gons = tbpm.backward(H, p0, nt, dt, f, _dev(g), K, ckpt)
        gval = gval.cpu().numpy()
        gons = gons.cpu().numpy()
        assert _rel(gval if cplx else gval.real, gval_r if cplx else gval_r.real) < 1e-10, nt
        assert _rel(gons, gons_r) < 1e-10, nt


@pytest.mark.parametrize("fused", [0, 2])
def test_dos_loss_bench_segmentation_vs_oracle_chain(fused):
    """The differentiable bench leg's chain at a small size: per-bond
    hoppings -2.7 (1 + 0.05 N(0,1)), 4 states, 1024 samples, checkpoints
    every 64 steps, the loss on every 8th energy (256 energies) against a
    uniform-hopping target, through the torch.autograd.Function; the bond
    and on-site gradients against the oracle chain (DOS adjoint, then the
    discrete adjoint of the propagation)."""
    print(f"case dos loss K=64 1024 samples fused={fused}", flush=True)
    from paper_2209_00806_amd import autograd as ag

    rng = np.random.default_rng(41)
    nx, ny, S, nt, K, f = 12, 10, 4, 1024, 64, 9.0
    n_b = 3 * nx * ny
    bt = -2.7 * (1 + 0.05 * rng.standard_normal(n_b))
    lat = inputs.graphene(nx, ny, bond_t=bt, keep_bonds=True)
    tgt = inputs.graphene(nx, ny, keep_bonds=True)
    psi0 = inputs.random_phase_states(rng, lat.n_orb, S)
    dt = math.pi / f
    ref_corr, _, _ = oracle.propagate(tgt.row_ptr, tgt.col, tgt.val, tgt.onsite, psi0, nt, dt, f)
    _, target = oracle.dos(ref_corr, dt)
    sel = np.arange(0, 2 * nt, 8)
    H = tbpm.Hamiltonian.from_lattice(lat)
    if fused:
        H.set_launch_config(2, 1, 1, 1, vec=2, precision="fp64", fused=fused)
    p0 = _dev(psi0)
    t_param = _dev(bt).requires_grad_(True)
    e_param = _dev(lat.onsite.copy()).requires_grad_(True)
    val = ag.bond_values(lat.nnz, _dev(lat.slot_ij), _dev(lat.slot_ji), t_param)
    _, D = ag.tbpm_dos(H, val, e_param, p0, nt, dt, f, ckpt_every=K)
    sel_t = _dev(sel)
    L = torch.sum((D[sel_t] - _dev(target)[sel_t]) ** 2)
    L.backward()
    gt = t_param.grad.cpu().numpy()
    ge = e_param.grad.cpu().numpy()
    corr_o, _, _ = oracle.propagate(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f)
    _, D_o = oracle.dos(corr_o, dt)
    gD = np.zeros_like(D_o)
    gD[sel] = 2 * (D_o[sel] - target[sel])
    gc = oracle.dos_adjoint(gD, nt, S, dt)
    gval_o, gons_o = oracle.backward(lat.row_ptr, lat.col, lat.val, lat.onsite, psi0, nt, dt, f, gc)
    gt_o = (gval_o[lat.slot_ij] + gval_o[lat.slot_ji]).real
    assert abs(L.item() - float(np.sum((D_o[sel] - target[sel]) ** 2))) < 1e-10 * max(L.item(), 1e-300)
    assert _rel(gt, gt_o) < 1e-9
    assert _rel(ge, gons_o) < 1e-9
