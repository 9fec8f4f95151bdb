"""Seeded synthetic inputs for TBPM: tight-binding lattices and random-phase states.

This module only *generates inputs*; it holds none of the propagation
arithmetic, so both the HIP path and the CPU oracle can be fed from it.

Conventions (paper, Sec. "Tight-binding models", Eq. (hal) and the graphene
primitive-cell example of the usage section):

* A Hamiltonian is returned as a full Hermitian CSR of its *off-diagonal*
  matrix elements ``H_ij`` plus a real on-site vector ``eps_i``.  The value
  stored is the matrix element itself, so "t = -2.7 eV" means ``H_ij = -2.7``.
* The paper stores only half of the hoppings and recovers the rest from
  ``t_ij(R) = t_ji(-R)^*``; here both directions are written out explicitly.
  Duplicate (i, j) pairs (tiny periodic lattices) are summed.
* Random initial states follow Eq. (ini_state): ``a_i = exp(i theta_i)/sqrt(N)``
  with ``theta_i`` uniform in [0, 2 pi), drawn with NumPy's PCG64 in the
  order ``[state][orbital]`` and stored as ``psi0[orbital][state]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

#: base seed of the synthetic workloads; workload ``c`` uses ``BASE_SEED + c``
BASE_SEED = 20220902

# graphene primitive cell (usage section, graphene example): a = 2.46 A,
# lattice vectors a1 = (a, 0), a2 = (a/2, a*sqrt(3)/2); p_z orbitals at
# fractional (0, 0) and (1/3, 1/3)
GRAPHENE_A = 2.46
GRAPHENE_A1 = np.array([GRAPHENE_A, 0.0])
GRAPHENE_A2 = np.array([GRAPHENE_A / 2.0, GRAPHENE_A * math.sqrt(3.0) / 2.0])
GRAPHENE_ORB_FRAC = np.array([[0.0, 0.0], [1.0 / 3.0, 1.0 / 3.0]])
#: reduced hopping list of the primitive cell: (R1, R2, orb_i, orb_j)
GRAPHENE_REDUCED_HOPPINGS = ((0, 0, 0, 1), (1, 0, 1, 0), (0, 1, 1, 0))


@dataclass
class Lattice:
    """A tight-binding model in full Hermitian CSR form (off-diagonal part)."""

    n_orb: int
    row_ptr: np.ndarray  # int64 [n_orb + 1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # complex128 [nnz]
    onsite: np.ndarray  # float64 [n_orb]
    name: str = ""
    # optional bond parameterisation (real symmetric hoppings): bond b sets
    # H[bond_i[b], bond_j[b]] = H[bond_j[b], bond_i[b]] = bond_t[b]
    bond_i: np.ndarray | None = None
    bond_j: np.ndarray | None = None
    bond_t: np.ndarray | None = None
    # CSR slots of (i, j) and (j, i) for every bond
    slot_ij: np.ndarray | None = None
    slot_ji: np.ndarray | None = None
    pos: np.ndarray | None = None  # optional [n_orb, 3] Cartesian positions (A)
    # optional [nnz, 2] in-plane displacement r_j - r_i (A) of the hopping
    # stored at each CSR entry (i, j), for the current operator
    disp: np.ndarray | None = None
    area: float = 0.0  # area of the sample (A^2), when known
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def dense(self) -> np.ndarray:
        """Dense H including the diagonal (small lattices only)."""
        n = self.n_orb
        h = np.zeros((n, n), dtype=np.complex128)
        rows = np.repeat(np.arange(n), np.diff(self.row_ptr))
        np.add.at(h, (rows, self.col), self.val)
        h[np.arange(n), np.arange(n)] += self.onsite
        return h


def _coo_to_csr(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    """Sort by (row, col) and sum duplicates; returns row_ptr, col, val."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.complex128)
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    if key.size:
        starts = np.flatnonzero(np.concatenate(([True], key[1:] != key[:-1])))
        vals = np.add.reduceat(vals, starts)
        key = key[starts]
    r = key // n
    c = key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, c.astype(np.int32), vals


def _csr_slots(row_ptr: np.ndarray, col: np.ndarray, i: np.ndarray, j: np.ndarray) -> np.ndarray:
    """CSR position of entry (i, j) for each pair (the entry must exist)."""
    n = row_ptr.shape[0] - 1
    key = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr)) * n + col.astype(np.int64)
    q = i.astype(np.int64) * n + j.astype(np.int64)
    pos = np.searchsorted(key, q)
    assert np.all(key[pos] == q), "bond entry missing from CSR"
    return pos.astype(np.int64)


def from_bonds(n: int, bi: np.ndarray, bj: np.ndarray, bt: np.ndarray, onsite: np.ndarray,
               name: str = "", keep_bonds: bool = False, pos=None, disp=None) -> Lattice:
    """Full Hermitian CSR from a half list of bonds H[i, j] = t, H[j, i] = conj(t).
    ``disp`` [n_bonds, 2]: displacement r_j - r_i of each bond (stored per
    CSR entry, negated on (j, i)); the bonds must then not repeat an entry."""
    bi = np.asarray(bi, dtype=np.int64)
    bj = np.asarray(bj, dtype=np.int64)
    bt = np.asarray(bt)
    rows = np.concatenate([bi, bj])
    cols = np.concatenate([bj, bi])
    vals = np.concatenate([bt.astype(np.complex128), np.conj(bt.astype(np.complex128))])
    row_ptr, col, val = _coo_to_csr(n, rows, cols, vals)
    lat = Lattice(n, row_ptr, col, val, np.asarray(onsite, dtype=np.float64).copy(), name=name, pos=pos)
    if disp is not None:
        disp = np.asarray(disp, dtype=np.float64)
        sij = _csr_slots(row_ptr, col, bi, bj)
        sji = _csr_slots(row_ptr, col, bj, bi)
        if np.unique(np.concatenate([sij, sji])).size != 2 * bi.shape[0]:
            raise ValueError("bond displacements need bonds that do not repeat a matrix entry")
        lat.disp = np.zeros((col.shape[0], 2))
        lat.disp[sij] = disp
        lat.disp[sji] = -disp
    if keep_bonds:
        lat.bond_i, lat.bond_j = bi, bj
        lat.bond_t = np.asarray(bt, dtype=np.float64).copy()
        lat.slot_ij = _csr_slots(row_ptr, col, bi, bj)
        lat.slot_ji = _csr_slots(row_ptr, col, bj, bi)
    return lat


def graphene_bonds(nx: int, ny: int, pbc: bool = True):
    """Half bond list of an nx x ny graphene super-cell.

    Orbital index ``2*(i1*ny + i2) + o`` for cell (i1, i2) and orbital o in
    {0 (A), 1 (B)}.  Bonds are listed hopping-kind major: all k=0 bonds
    (one per cell, in cell order), then k=1, then k=2, following the reduced
    hopping list of the primitive cell: k=0 A(c)->B(c), k=1 B(c)->A(c+a1),
    k=2 B(c)->A(c+a2).
    With open boundaries the bonds that leave the sample are dropped.
    Returns (bi, bj, cell_index, k) arrays.
    """
    i1, i2 = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    i1 = i1.ravel()
    i2 = i2.ravel()
    cell = i1 * ny + i2
    out_i, out_j, out_c, out_k = [], [], [], []
    for k, (r1, r2, oi, oj) in enumerate(GRAPHENE_REDUCED_HOPPINGS):
        t1 = i1 + r1
        t2 = i2 + r2
        if pbc:
            t1 %= nx
            t2 %= ny
            keep = np.ones_like(t1, dtype=bool)
        else:
            keep = (t1 >= 0) & (t1 < nx) & (t2 >= 0) & (t2 < ny)
        tc = t1 * ny + t2
        out_i.append(2 * cell[keep] + oi)
        out_j.append(2 * tc[keep] + oj)
        out_c.append(cell[keep])
        out_k.append(np.full(int(keep.sum()), k))
    return (np.concatenate(out_i), np.concatenate(out_j), np.concatenate(out_c), np.concatenate(out_k))


def graphene_positions(nx: int, ny: int) -> np.ndarray:
    """Cartesian orbital positions (A, z = 0) of the super-cell, same order as the orbitals."""
    i1, i2 = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    cells = np.stack([i1.ravel(), i2.ravel()], axis=1).astype(np.float64)
    pos = np.empty((2 * cells.shape[0], 3))
    for o in range(2):
        frac = cells + GRAPHENE_ORB_FRAC[o]
        xy = frac[:, :1] * GRAPHENE_A1 + frac[:, 1:2] * GRAPHENE_A2
        pos[o::2, :2] = xy
        pos[o::2, 2] = 0.0
    return pos


def graphene(nx: int, ny: int, t: float = -2.7, pbc: bool = True, onsite=None,
             bond_t=None, keep_bonds: bool = False, with_pos: bool = False) -> Lattice:
    """Monolayer graphene nx x ny cells, nearest-neighbour hopping ``t`` (matrix element)."""
    bi, bj, _, kind = graphene_bonds(nx, ny, pbc)
    n = 2 * nx * ny
    bt = np.full(bi.shape[0], float(t)) if bond_t is None else np.asarray(bond_t, dtype=np.float64)
    ons = np.zeros(n) if onsite is None else np.asarray(onsite, dtype=np.float64)
    pos = graphene_positions(nx, ny) if with_pos else None
    disp = None
    if nx > 2 and ny > 2:  # smaller periodic cells repeat matrix entries
        lat_vec = np.stack([GRAPHENE_A1, GRAPHENE_A2])
        d_kind = np.array([(np.array([r1, r2]) + GRAPHENE_ORB_FRAC[oj] - GRAPHENE_ORB_FRAC[oi]) @ lat_vec
                           for (r1, r2, oi, oj) in GRAPHENE_REDUCED_HOPPINGS])
        disp = d_kind[kind]
    lat = from_bonds(n, bi, bj, bt, ons, name=f"graphene{nx}x{ny}", keep_bonds=keep_bonds, pos=pos, disp=disp)
    lat.area = nx * ny * abs(float(GRAPHENE_A1[0] * GRAPHENE_A2[1] - GRAPHENE_A1[1] * GRAPHENE_A2[0]))
    lat.meta.update(kind="graphene", nx=nx, ny=ny, pbc=pbc)
    return lat


def square(nx: int, ny: int, t: float = -2.7, pbc: bool = True, onsite=None) -> Lattice:
    """Square lattice, one orbital per site, index ``i1*ny + i2``, spacing 1 A."""
    i1, i2 = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    i1 = i1.ravel()
    i2 = i2.ravel()
    site = i1 * ny + i2
    bi, bj, bd = [], [], []
    for r1, r2 in ((1, 0), (0, 1)):
        t1, t2 = i1 + r1, i2 + r2
        if pbc:
            t1 %= nx
            t2 %= ny
            keep = np.ones_like(t1, dtype=bool)
        else:
            keep = (t1 < nx) & (t2 < ny)
        bi.append(site[keep])
        bj.append((t1 * ny + t2)[keep])
        bd.append(np.tile([float(r1), float(r2)], (int(keep.sum()), 1)))
    bi = np.concatenate(bi)
    bj = np.concatenate(bj)
    n = nx * ny
    ons = np.zeros(n) if onsite is None else np.asarray(onsite, dtype=np.float64)
    disp = np.concatenate(bd) if (not pbc or (nx > 2 and ny > 2)) else None
    lat = from_bonds(n, bi, bj, np.full(bi.shape[0], float(t)), ons, name=f"square{nx}x{ny}", disp=disp)
    lat.area = float(nx * ny)
    lat.meta.update(kind="square", nx=nx, ny=ny, pbc=pbc)
    return lat


def hofstadter(nx: int, ny: int, p: int, q: int, t: float = -1.0, onsite=None) -> Lattice:
    """Periodic square lattice (spacing 1 A) in a uniform magnetic field of
    p/q flux quanta per plaquette: Peierls phases in the Landau gauge
    A = (0, B x), i.e. the bond from (i1, i2) to (i1, i2 + 1) carries
    t exp(i 2 pi (p/q) i1).  Periodic in both directions when q divides nx.
    Bond displacements are kept for the current operator."""
    if nx % q != 0:
        raise ValueError("q must divide nx for a periodic gauge")
    lat = square(nx, ny, t=t, pbc=True, onsite=onsite)
    if lat.disp is None:
        raise ValueError("nx and ny must exceed 2")
    rows = np.repeat(np.arange(lat.n_orb), np.diff(lat.row_ptr))
    x = rows // ny
    # the y bond out of row i (disp (0, +1)) gets e^{+i 2 pi phi x_i}; its
    # reverse entry (disp (0, -1)) the conjugate
    phase = np.exp(2j * np.pi * (p / q) * x * lat.disp[:, 1])
    lat.val = lat.val * phase
    lat.name = f"hofstadter{nx}x{ny}_{p}/{q}"
    lat.meta.update(kind="hofstadter", flux=(p, q))
    return lat


def current_values(lat: Lattice, axis: int) -> np.ndarray:
    """Matrix elements of the current operator J_axis = -i sum_ij H_ij (r_j - r_i)_axis
    c_i^dagger c_j (Sec. "Optical conductivity"; e = hbar = 1) on the CSR
    pattern of ``lat``, aligned with lat.col.  Requires lat.disp."""
    if lat.disp is None:
        raise ValueError("the lattice carries no bond displacements")
    return -1j * lat.val * lat.disp[:, axis]


def anderson(rng: np.random.Generator, n: int, w: float) -> np.ndarray:
    """Anderson on-site disorder, uniform in [-w/2, w/2]."""
    return rng.uniform(-0.5 * w, 0.5 * w, size=n)


def random_phase_states(rng: np.random.Generator, n: int, n_states: int) -> np.ndarray:
    """Random-phase states ``exp(i theta)/sqrt(n)``, layout [n][n_states] complex128."""
    theta = rng.uniform(0.0, 2.0 * np.pi, size=(n_states, n))
    return np.ascontiguousarray((np.exp(1j * theta) / np.sqrt(n)).T)


def unit_states(n: int, orbitals) -> np.ndarray:
    """One state per listed orbital, with amplitude 1 on that orbital only
    (the initial state of the LDOS by propagation, Sec. "Local density of
    states"); layout [n][len(orbitals)] complex128."""
    orbitals = np.asarray(orbitals, dtype=np.int64)
    out = np.zeros((n, orbitals.shape[0]), dtype=np.complex128)
    out[orbitals, np.arange(orbitals.shape[0])] = 1.0
    return out


def local_random_states(rng: np.random.Generator, n: int, orbitals, n_states: int) -> np.ndarray:
    """Random phases on a set of orbitals only, normalised (the LDOS averaged
    over that set); layout [n][n_states] complex128."""
    orbitals = np.asarray(orbitals, dtype=np.int64)
    theta = rng.uniform(0.0, 2.0 * np.pi, size=(n_states, orbitals.shape[0]))
    out = np.zeros((n, n_states), dtype=np.complex128)
    out[orbitals, :] = (np.exp(1j * theta) / np.sqrt(orbitals.shape[0])).T
    return out


def gaussian_packet(pos: np.ndarray, center, sigma: float = 0.5, extent=(1.0, 1.0)) -> np.ndarray:
    """Real Gaussian wave packet exp(-r^2 / (2 sigma^2)) around ``center`` in
    the plane, with the x and y offsets scaled by ``extent`` (0 drops that
    direction: a one-dimensional packet), normalised; the initial state of the
    wave-function propagation example of the usage section.  Returns [n]
    complex128."""
    dx = (pos[:, 0] - center[0]) * extent[0]
    dy = (pos[:, 1] - center[1]) * extent[1]
    w = np.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma)).astype(np.complex128)
    return w / np.linalg.norm(w)


def morton_order(xy: np.ndarray, cell: float) -> np.ndarray:
    """Permutation that sorts points along a Z-order (Morton) curve of their 2D
    positions quantised to ``cell``; points in the same quantum keep their order."""
    q = np.floor((xy - xy.min(axis=0)) / cell).astype(np.uint64)

    def spread(v):  # interleave zeros between the low 32 bits
        v = v & np.uint64(0xFFFFFFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x0000FFFF0000FFFF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x3333333333333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x5555555555555555)
        return v

    code = spread(q[:, 0]) | (spread(q[:, 1]) << np.uint64(1))
    return np.argsort(code, kind="stable")


def twisted_bilayer(nx: int, ny: int, angle_deg: float = 1.05, d: float = 3.35,
                    a_cc: float = 1.42, t_intra: float = -2.7, t0: float = 0.48,
                    decay: float = 0.184, cutoff: float = 5.0, max_neighbors: int = 48,
                    order: str = "morton") -> Lattice:
    """Twisted bilayer honeycomb flake with open boundaries.

    Layer 1 is an nx x ny graphene flake (nearest-neighbour distance a_cc)
    centred at the origin; layer 2 is the same flake rotated by ``angle_deg``
    about the z axis and lifted to z = d.  Intralayer nearest neighbours carry
    ``t_intra``; every interlayer pair at 3D distance <= cutoff carries
    ``t0 * exp(-(r - d)/decay)``.

    ``order="layer"`` numbers layer 1 then layer 2 (each in graphene order);
    ``order="morton"`` numbers the atoms of both layers along a Z-order curve
    of their in-plane positions (quantum a_cc), so that orbitals close in
    space -- in either layer -- are close in index.
    """
    from scipy.spatial import cKDTree  # input generation only

    a = a_cc * math.sqrt(3.0)
    scale = a / GRAPHENE_A
    base = graphene(nx, ny, t=t_intra, pbc=False, with_pos=True)
    p1 = base.pos[:, :2] * scale
    p1 = p1 - p1.mean(axis=0)
    th = math.radians(angle_deg)
    rot = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    p2 = p1 @ rot.T
    n1 = p1.shape[0]
    rin = math.sqrt(max(cutoff * cutoff - d * d, 0.0))
    tree = cKDTree(p2)
    dist, idx = tree.query(p1, k=max_neighbors, distance_upper_bound=rin * (1 + 1e-12), workers=-1)
    ok = np.isfinite(dist)
    if ok[:, -1].any():
        raise RuntimeError("max_neighbors too small for the interlayer cutoff")
    li = np.repeat(np.arange(n1), max_neighbors).reshape(n1, max_neighbors)[ok]
    lj = idx[ok] + n1
    r3 = np.sqrt(dist[ok] ** 2 + d * d)
    tinter = t0 * np.exp(-(r3 - d) / decay)
    bi0, bj0, _, _ = graphene_bonds(nx, ny, pbc=False)
    bi = np.concatenate([bi0, bi0 + n1, li])
    bj = np.concatenate([bj0, bj0 + n1, lj])
    bt = np.concatenate([np.full(2 * bi0.shape[0], t_intra), tinter])
    pos = np.zeros((2 * n1, 3))
    pos[:n1, :2] = p1
    pos[n1:, :2] = p2
    pos[n1:, 2] = d
    if order == "morton":
        perm = morton_order(pos[:, :2], a_cc)  # new index -> old index
        inv = np.empty_like(perm)
        inv[perm] = np.arange(perm.shape[0])
        bi, bj, pos = inv[bi], inv[bj], pos[perm]
    elif order != "layer":
        raise ValueError(order)
    lat = from_bonds(2 * n1, bi, bj, bt, np.zeros(2 * n1), name=f"tbg{nx}x{ny}", pos=pos)
    lat.meta.update(kind="tbg", nx=nx, ny=ny, angle=angle_deg, order=order)
    return lat


# ----------------------------------------------------------------------------
# the paper-shaped workloads
# ----------------------------------------------------------------------------

def workload_graphene_dos(cells: int = 64, n_states: int = 1, seed_offset: int = 0):
    """Clean periodic graphene (usage-section example shape); returns (lattice, psi0)."""
    rng = np.random.default_rng(BASE_SEED + seed_offset)
    lat = graphene(cells, cells)
    psi0 = random_phase_states(rng, lat.n_orb, n_states)
    return lat, psi0


def workload_disordered_graphene(cells: int = 1024, n_states: int = 8, w: float = 1.0,
                                 seed_offset: int = 1):
    """Periodic graphene with Anderson disorder; disorder drawn first, then states."""
    rng = np.random.default_rng(BASE_SEED + seed_offset)
    n = 2 * cells * cells
    ons = anderson(rng, n, w)
    lat = graphene(cells, cells, onsite=ons)
    psi0 = random_phase_states(rng, n, n_states)
    return lat, psi0


def workload_twisted_bilayer(cells: int = 1024, n_states: int = 16, seed_offset: int = 2):
    rng = np.random.default_rng(BASE_SEED + seed_offset)
    lat = twisted_bilayer(cells, cells)
    psi0 = random_phase_states(rng, lat.n_orb, n_states)
    return lat, psi0


def workload_batch(n_ham: int = 64, n_min: float = 1e4, n_max: float = 1e6, n_states: int = 4,
                   seed_offset: int = 3):
    """Uneven batch: square or graphene by seed, log-uniform sizes, Anderson W ~ U[0, 2]."""
    rng = np.random.default_rng(BASE_SEED + seed_offset)
    lats, states = [], []
    for _ in range(n_ham):
        kind = "graphene" if rng.uniform() < 0.5 else "square"
        size = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        w = rng.uniform(0.0, 2.0)
        if kind == "graphene":
            L = max(3, int(round(math.sqrt(size / 2.0))))
            n = 2 * L * L
            lat = graphene(L, L, onsite=anderson(rng, n, w))
        else:
            L = max(3, int(round(math.sqrt(size))))
            n = L * L
            lat = square(L, L, onsite=anderson(rng, n, w))
        lat.meta["w"] = w
        lats.append(lat)
        states.append(random_phase_states(rng, lat.n_orb, n_states))
    return lats, states


def workload_bond_graphene(cells: int = 512, n_states: int = 4, rel_sigma: float = 0.05,
                           seed_offset: int = 4):
    """Graphene with per-bond hoppings -2.7*(1 + sigma*N(0,1)) and zero on-site.

    Returns (lattice with bond parameterisation, target lattice with uniform
    hopping and the same pattern, psi0).
    """
    rng = np.random.default_rng(BASE_SEED + seed_offset)
    n_bonds = 3 * cells * cells
    bt = -2.7 * (1.0 + rel_sigma * rng.standard_normal(n_bonds))
    lat = graphene(cells, cells, bond_t=bt, keep_bonds=True)
    target = graphene(cells, cells, keep_bonds=True)
    psi0 = random_phase_states(rng, lat.n_orb, n_states)
    return lat, target, psi0
