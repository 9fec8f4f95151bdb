"""CPU tests of the host logic behind the fused launch shape and the internal
row order: tests/host_tables_check.cpp is compiled against the library's
host.cpp and run on seeded lattices (plain and renumbered orders, several
state widths and LDS tiers).  It checks that the bisection order is a
permutation within each member, that every index the fused kernel takes
from the tile tables stays in bounds and names the right row, that every
row is owned by exactly one tile, and that a pair of Clenshaw orders
evaluated through the tables equals two orders computed from the CSR."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2209_00806_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("host_tables") / "host_tables_check")
    cmd = [hipcc, "-O2", "-std=c++17", "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "host_tables_check.cpp"),
           os.path.join(ROOT, "paper_2209_00806_amd", "csrc", "host.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return out


def _write(tmp, lats):
    rp, cols, vals, inst = [0], [], [], [0]
    for lat in lats:
        off = inst[-1]
        cols.append(lat.col.astype(np.int32) + off)
        vals.append(np.real(lat.val).astype(np.float64))
        rp.extend((lat.row_ptr[1:] + rp[-1]).tolist())
        inst.append(off + lat.n_orb)
    paths = [os.path.join(tmp, n) for n in ("rp", "col", "val", "inst")]
    np.asarray(rp, np.int64).tofile(paths[0])
    np.concatenate(cols).tofile(paths[1])
    np.concatenate(vals).tofile(paths[2])
    np.asarray(inst, np.int64).tofile(paths[3])
    return paths


CASES = {
    "graphene_37x29": lambda: [inputs.graphene(37, 29)],
    "square_open_45x31": lambda: [inputs.square(45, 31, pbc=False)],
    "tbg_12x12": lambda: [inputs.twisted_bilayer(12, 12, angle_deg=4.0)],
    "batch_5": lambda: [inputs.graphene(9, 7), inputs.square(13, 5), inputs.graphene(3, 2), inputs.square(1, 3),
                        inputs.graphene(20, 11)],
}

# (log2 units per row, bytes per unit): S = 8 FP64 with 1 and 2 states per
# thread, S = 1 FP64, S = 64 FP64, S = 16 FP32 with 4 states per thread
WIDTHS = [(3, 16), (2, 32), (0, 16), (6, 16), (2, 32)]


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("case", sorted(CASES))
def test_two_hop_tables_and_row_order(checker, tmp_path, case, order):
    paths = _write(str(tmp_path), CASES[case]())
    fits = 0
    for log2u, ub in WIDTHS:
        for tier in (1, 2, 4, 6):
            r = subprocess.run([checker, *paths, str(order), str(log2u), str(ub), str(tier)], capture_output=True,
                               text=True, timeout=120)
            if r.returncode == 3:
                assert "NOFIT" in r.stdout  # no tile fits: the library falls back to the plain shape
                continue
            assert r.returncode == 0, (case, order, log2u, ub, tier, r.stdout, r.stderr)
            assert r.stdout.startswith("OK")
            fits += 1
    assert fits > 0


def test_two_hop_tables_threaded_build(checker, tmp_path):
    """A lattice above the threading threshold (420 x 420 graphene, 1.06M
    stored elements): the tables are built in chunks on host threads and
    joined in tile order, and must pass the same checks (tables against the
    CSR, a pair of orders through them against the direct evaluation), in
    both row orders."""
    paths = _write(str(tmp_path), [inputs.graphene(420, 420)])
    for order in (0, 1):
        for log2u, ub in ((2, 32), (0, 16)):
            r = subprocess.run([checker, *paths, str(order), str(log2u), str(ub), "2"], capture_output=True,
                               text=True, timeout=300)
            assert r.returncode == 0 and r.stdout.startswith("OK"), (order, log2u, ub, r.stdout, r.stderr)
