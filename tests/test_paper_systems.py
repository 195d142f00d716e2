"""Pins against the benchmark systems the paper prints (Table "realistic",
fixture tests/golden/table_realistic.txt): atom counts from the cell counts,
the slab generator's size, and the oracle's list lengths on perfect lattices
where the printed interaction count is a closed shell of the crystal.

Shells (distance in units of the lattice constant a: atoms in the shell):
  BCC: sqrt(3)/2: 8, 1: 6, sqrt(2): 12, sqrt(11)/2: 24, sqrt(3): 8
  FCC: 1/sqrt(2): 12, 1: 6, sqrt(3/2): 24, sqrt(2): 12
so 14 interactions (Ta) are the first two BCC shells and 42 (Cu) the first
three FCC shells.  The W row's 59 is no closed shell of the perfect lattice
(58 = five shells); its count at 290 K includes thermal neighbours, so it is
only checked to lie between the shell counts around it.
"""
import os

import numpy as np
import pytest

from workloads import configs

HERE = os.path.dirname(os.path.abspath(__file__))
BASIS = {"BCC": 2, "FCC": 4}
# cumulative shell counts of the perfect lattices, with the shell radii / a
SHELLS = {
    "BCC": [(np.sqrt(3) / 2, 8), (1.0, 14), (np.sqrt(2), 26), (np.sqrt(11) / 2, 50),
            (np.sqrt(3), 58), (2.0, 64)],
    "FCC": [(1 / np.sqrt(2), 12), (1.0, 18), (np.sqrt(1.5), 42), (np.sqrt(2), 54)],
}


def _rows():
    rows = []
    with open(os.path.join(HERE, "golden", "table_realistic.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                el, lat, nx, ny, nz, atoms, inter = line.split()
                rows.append((el, lat, int(nx), int(ny), int(nz), int(atoms), int(inter)))
    return rows


ROWS = _rows()


def _fcc(n, a):
    ix, iy, iz = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([ix, iy, iz], axis=-1).reshape(-1, 1, 3).astype(np.float64)
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    return ((base + basis[None]) * a).reshape(-1, 3)


def test_fixture_rows():
    assert [r[0] for r in ROWS] == ["Cu", "W", "Ta"]


@pytest.mark.parametrize("row", ROWS, ids=[r[0] for r in ROWS])
def test_atom_count_is_cells_times_basis(row):
    _, lat, nx, ny, nz, atoms, _ = row
    assert nx * ny * nz * BASIS[lat] == atoms


def test_slab_generator_builds_the_bcc_slab():
    el, lat, nx, ny, nz, atoms, _ = ROWS[2]
    b = configs.slab(nx, ny, nz, seed=1)
    assert b.n == atoms == 801792
    # open x and y, periodic z
    assert b.box[0] < 0 and b.box[1] < 0 and b.box[2] > 0


@pytest.mark.parametrize("row", ROWS, ids=[r[0] for r in ROWS])
def test_interactions_per_atom_on_the_perfect_lattice(oracle_lib, row):
    el, lat, *_, inter = row
    shells = SHELLS[lat]
    counts = [c for _, c in shells]
    if inter not in counts:
        # not a closed shell: lies between two consecutive shell counts
        assert any(lo < inter < hi for lo, hi in zip(counts, counts[1:])), inter
        return
    k = counts.index(inter)
    a = 3.3
    # a list radius halfway between the last included shell and the next one
    r = 0.5 * (shells[k][0] + shells[k + 1][0]) * a
    n = max(3, int(np.ceil(3 * r / a)))
    x = configs.bcc_block(n, n, n, a) if lat == "BCC" else _fcc(n, a)
    cnt, _, _ = oracle_lib.neighbor_list(x, np.full(3, n * a), r)
    assert np.all(cnt == inter), (el, np.unique(cnt))
