"""The library's canonical numbering of general hexahedral meshes (a host
call, no device) against the oracle's own implementation of the same
definition: identical node ids, bit for bit, under random vertex
relabelling, cell rotations and cell order, for degrees 1 to 6; and the same
mesh errors rejected."""

import numpy as np
import pytest

import paper_2505_15535_amd as mfe
import synthetic
from oracle.mesh import HexMesh


def _mesh(m, seed):
    v, c = synthetic.cube_in_cube(m, jitter=0.1, rng=np.random.default_rng(seed))
    v, c, _, _ = synthetic.relabel(v, c, np.random.default_rng(seed + 1), shuffle_cells=True)
    return v, c


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_numbering_matches_oracle(p):
    v, c = _mesh(1 if p > 3 else 2, 100 + p)
    nodes, n_nodes = mfe.mfe_hex_numbering(c, p, v.shape[0])
    H = HexMesh(v, c, p)
    assert n_nodes == H.n_nodes
    assert np.array_equal(nodes, H.elem_nodes)


def test_box_as_hex_numbering():
    nx, ny, nz = 4, 3, 2
    c = synthetic.box_cells(nx, ny, nz)
    v = synthetic.box_vertices(nx, ny, nz)
    nodes, n_nodes = mfe.mfe_hex_numbering(c, 2, v.shape[0])
    assert n_nodes == (2 * nx + 1) * (2 * ny + 1) * (2 * nz + 1)
    assert np.array_equal(nodes, HexMesh(v, c, 2).elem_nodes)


def test_numbering_rejects_bad_meshes():
    v = synthetic.box_vertices(2, 1, 1)
    c = synthetic.box_cells(2, 1, 1)
    bad = c.copy()
    bad[0, 0] = v.shape[0]
    with pytest.raises(mfe.MfeError):
        mfe.mfe_hex_numbering(bad, 2, v.shape[0])
    bad = c.copy()
    bad[1, 3] = bad[1, 2]
    with pytest.raises(mfe.MfeError):
        mfe.mfe_hex_numbering(bad, 2, v.shape[0])
    bad = c.copy()
    bad[1, [0, 2]] = c[1, [2, 0]]          # crossed edges on the shared face
    with pytest.raises(mfe.MfeError):
        mfe.mfe_hex_numbering(bad, 2, v.shape[0])
    three = np.concatenate([c, c[:1]])      # the shared face in three cells
    with pytest.raises(mfe.MfeError):
        mfe.mfe_hex_numbering(three, 2, v.shape[0])
    with pytest.raises(mfe.MfeError):
        mfe.mfe_hex_numbering(c, 7, v.shape[0])
