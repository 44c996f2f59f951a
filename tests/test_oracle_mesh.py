"""Pins of the oracle's mesh tables: counts, uniqueness, neighbour symmetry."""
import numpy as np
import pytest

from oracle.mesh import BoxMesh


@pytest.mark.parametrize("dim,n", [(2, (8, 8)), (3, (4, 3, 2)), (3, (16, 16, 16))])
def test_face_tables(dim, n):
    lo, hi = (0.0,) * dim, (1.0,) * dim
    msh = BoxMesh(dim, n, lo, hi, 2)
    E = int(np.prod(n))
    n_int = sum((n[a] - 1) * E // n[a] for a in range(dim))
    assert len(msh.face_minus) == n_int
    pairs = set(zip(msh.face_minus.tolist(), msh.face_plus.tolist()))
    assert len(pairs) == n_int
    # neighbour tables are symmetric and agree with the face list
    for e in range(E):
        for a in range(dim):
            up = msh.nbr[e, 2 * a + 1]
            if up >= 0:
                assert msh.nbr[up, 2 * a] == e
                assert (e, up) in pairs
    n_bdry = sum(len(v) for v in msh.bfaces.values())
    assert n_bdry == sum(2 * E // n[a] for a in range(dim))
    # every element face is exactly one of: interior (counted from both sides) or boundary
    assert 2 * n_int + n_bdry == 2 * dim * E


def test_face_node_indices():
    msh = BoxMesh(3, (2, 2, 2), (0, 0, 0), (1, 1, 1), 2)
    # x- face of an element: local nodes with a = 0, ordered (b, c) with b fastest
    assert msh.fnodes[(0, -1)].tolist() == [0, 3, 6, 9, 12, 15, 18, 21, 24]
    assert msh.fnodes[(2, 1)].tolist() == list(range(18, 27))
    # face tabulations reduce to the face-node identity at the GLL points
    xp = BoxMesh(3, (1, 1, 1), (0, 0, 0), (1, 1, 1), 2, nq=3)
    assert xp.fnodes[(1, 1)].tolist() == [6, 7, 8, 15, 16, 17, 24, 25, 26]


def test_geometry_partition():
    msh = BoxMesh(3, (4, 2, 2), (0, 0, 0), (8, 2, 1), 3)
    # volume weights integrate the box volume; face weights the face areas
    assert abs(msh.wvol.sum() * msh.E - 16.0) < 1e-12
    assert abs(msh.fw[0].sum() - 1.0 * 0.5) < 1e-14
    assert abs(msh.diameter - np.sqrt(4 + 1 + 0.25)) < 1e-14
