"""Mesh generator invariants (T8): 6 n^3 positive tetrahedra filling the unit
cube, one-to-one periodic face pairing with odd vertex permutation, symmetric
orientation codes; seeded reproducibility."""
import numpy as np
import pytest

from workload import cube_mesh, random_dofs, random_materials, seed_for, dt_from_mesh
from workload.mesh import FACE_VERTS


@pytest.mark.parametrize("n,relabel", [(3, False), (5, True), (8, False)])
def test_mesh_invariants(n, relabel):
    m = cube_mesh(n, seed_for(0), relabel=relabel)
    E = m.E
    assert E == 6 * n ** 3
    X = m.X
    det = np.einsum("ei,ei->e", X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]))
    assert det.min() > 0
    assert det.sum() / 6 == pytest.approx(1.0, rel=1e-13)
    idx = np.arange(E)[:, None]
    nf = m.nface.astype(int)
    assert np.all(m.neigh[m.neigh, nf] == idx)
    assert np.all(m.nface[m.neigh, nf] == np.arange(4)[None, :])
    assert np.all(m.orient[m.neigh, nf] == m.orient)
    # the neighbour's face triple is an odd permutation of ours
    fv = np.array(FACE_VERTS)
    for e in range(0, E, 7):
        for s in range(4):
            mine = list(m.V[e, fv[s]])
            theirs = list(m.V[m.neigh[e, s], fv[nf[e, s]]])
            perm = [mine.index(v) for v in theirs]
            inv = sum(1 for i in range(3) for j in range(i + 1, 3) if perm[i] > perm[j])
            assert inv % 2 == 1
    assert set(np.unique(m.face_rot & 3)) <= {0, 1, 2, 3}


def test_seeded_reproducible():
    a = cube_mesh(4, 123)
    b = cube_mesh(4, 123)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.neigh, b.neigh)
    m1 = random_materials(10, 5)
    assert np.all((m1[:, 0] >= 2000) & (m1[:, 0] <= 3000))
    r = m1[:, 1] / m1[:, 2]
    assert np.all((r >= 1.6) & (r <= 2.0))
    q = random_dofs(1000, 9, 20, 3)
    assert abs(q.mean()) < 0.01 and abs(q.std() - 1) < 0.01
    dt = dt_from_mesh(cube_mesh(8, seed_for(0)), random_materials(3072, seed_for(0)))
    assert 5e-7 < dt < 9e-7
