"""CPU checks that the seeded generators build the workloads their recipes
state: the twisted bilayer of the magic-angle example (two rotated graphene
flakes, intralayer -2.7 eV, interlayer 0.48 eV exp(-(r - 3.35)/0.184) within
5 A), the uneven batch, the disordered graphene lattice and the random-phase
states of Eq. (ini_state).  Each check rebuilds the expected structure by
brute force from the atom positions or from the recipe's parameters, not from
the generator's own code path."""
import math

import numpy as np
import pytest

from paper_2209_00806_amd import inputs


def _pairs(lat):
    rows = np.repeat(np.arange(lat.n_orb), np.diff(lat.row_ptr))
    return rows, lat.col.astype(np.int64), lat.val


@pytest.mark.parametrize("nx,ny,angle", [(6, 5, 7.0), (9, 9, 3.0)])
@pytest.mark.parametrize("order", ["morton", "layer"])
def test_twisted_bilayer_matches_brute_force(nx, ny, angle, order):
    lat = inputs.twisted_bilayer(nx, ny, angle_deg=angle, order=order)
    n = lat.n_orb
    assert n == 4 * nx * ny
    assert np.all(lat.onsite == 0.0)
    pos = lat.pos
    top = pos[:, 2] > 1.0
    assert top.sum() == n // 2
    assert np.allclose(pos[top, 2], 3.35) and np.allclose(pos[~top, 2], 0.0)

    # the top layer is the bottom layer rotated by `angle` about the z axis
    th = math.radians(angle)
    rot = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    p_rot = pos[~top, :2] @ rot.T
    d2 = ((p_rot[:, None, :] - pos[top, None, :2].transpose(1, 0, 2)) ** 2).sum(-1)
    assert np.max(np.min(d2, axis=1)) < 1e-18
    # the bottom flake is centred at the origin
    assert np.allclose(pos[~top, :2].mean(axis=0), 0.0, atol=1e-9)

    # expected matrix from all pairs of atoms
    diff = pos[:, None, :] - pos[None, :, :]
    r = np.sqrt((diff ** 2).sum(-1))
    same = top[:, None] == top[None, :]
    want = np.zeros((n, n))
    intra = same & (np.abs(r - 1.42) < 1e-6)
    want[intra] = -2.7
    inter = (~same) & (r <= 5.0 + 1e-9)
    want[inter] = 0.48 * np.exp(-(r[inter] - 3.35) / 0.184)
    # every intralayer pair is either a nearest neighbour or farther than 2 A
    assert not np.any(same & (r > 1e-9) & (r < 2.0) & ~intra)

    got = np.zeros((n, n))
    i, j, v = _pairs(lat)
    assert np.all(np.imag(v) == 0.0)
    np.add.at(got, (i, j), np.real(v))
    assert np.array_equal(got != 0.0, want != 0.0)
    assert np.max(np.abs(got - want)) < 1e-12
    # each honeycomb atom has at most three intralayer neighbours
    assert np.max(intra.sum(axis=1)) == 3


def test_twisted_bilayer_rows_per_element_at_small_angle():
    """On a 40 x 40 flake at 1.05 degrees an interior row holds its 3
    intralayer neighbours plus every interlayer atom within 5 A, 16 to 21
    elements (18.9 on average), which is what makes the bilayer's rows wide."""
    lat = inputs.twisted_bilayer(40, 40, angle_deg=1.05)
    per_row = np.diff(lat.row_ptr)
    pos = lat.pos[:, :2]
    interior = np.linalg.norm(pos, axis=1) < 0.5 * np.max(np.abs(pos))
    m = per_row[interior].mean()
    assert 17.0 <= m <= 21.0, m


def test_batch_recipe():
    lats, states = inputs.workload_batch(64)
    assert len(lats) == 64 and len(states) == 64
    sizes = np.array([l.n_orb for l in lats], dtype=float)
    # log-uniform sizes in [1e4, 1e6], up to the rounding of the side length
    assert sizes.min() >= 1e4 * 0.97 and sizes.max() <= 1e6 * 1.03
    lo = np.log(sizes)
    assert np.ptp(lo) > 0.6 * math.log(100.0)
    for l, s in zip(lats, states):
        per_row = np.diff(l.row_ptr)
        # periodic graphene rows hold 3 elements, periodic square rows 4
        assert per_row.min() == per_row.max() and per_row[0] in (3, 4)
        w = l.meta["w"]
        assert 0.0 <= w <= 2.0
        assert np.max(np.abs(l.onsite)) <= w / 2.0
        assert s.shape == (l.n_orb, 4)
        assert np.allclose(np.abs(s), 1.0 / math.sqrt(l.n_orb), rtol=0, atol=1e-15)
    n_graphene = sum(1 for l in lats if np.diff(l.row_ptr)[0] == 3)
    assert 16 <= n_graphene <= 48, n_graphene
    # the same seed gives the same batch (its first eight members)
    lats2, states2 = inputs.workload_batch(8)
    assert all(np.array_equal(a.onsite, b.onsite) for a, b in zip(lats, lats2))
    assert all(np.array_equal(a, b) for a, b in zip(states, states2))


def test_disordered_graphene_recipe():
    lat, psi0 = inputs.workload_disordered_graphene(64, n_states=8)
    n = 2 * 64 * 64
    assert lat.n_orb == n and psi0.shape == (n, 8)
    # Anderson disorder U[-W/2, W/2] with W = 1
    assert np.max(np.abs(lat.onsite)) <= 0.5
    assert abs(lat.onsite.mean()) < 0.02 and abs(lat.onsite.var() - 1.0 / 12.0) < 0.01
    per_row = np.diff(lat.row_ptr)
    assert np.all(per_row == 3)
    assert np.allclose(np.real(lat.val), -2.7) and np.all(np.imag(lat.val) == 0.0)
    # random phases: |a_i| = 1/sqrt(N), phases uniform on [0, 2 pi)
    assert np.allclose(np.abs(psi0), 1.0 / math.sqrt(n), rtol=0, atol=1e-15)
    th = np.sort(np.mod(np.angle(psi0[:, 0]), 2 * math.pi)) / (2 * math.pi)
    ks = np.max(np.abs(th - (np.arange(n) + 0.5) / n))
    assert ks < 1.63 / math.sqrt(n) + 1.0 / n  # Kolmogorov-Smirnov at 1%
    # the states are drawn after the disorder, with the workload's own seed
    rng = np.random.default_rng(inputs.BASE_SEED + 1)
    ons = inputs.anderson(rng, n, 1.0)
    assert np.array_equal(ons, lat.onsite)
