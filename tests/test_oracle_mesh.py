"""Pins of the oracle's adjacency and geometry and of the input generators
(no GPU)."""
import numpy as np
import pytest

import synth
from oracle import mesh as om


def test_box_volumes_and_faces():
    m = synth.layered_box(4, 3, [100.0, 200.0, 300.0], 1200.0, 900.0, jitter=0.15, seed=1)
    g = om.geometry(m["tet_xyz"])
    assert g["vol"].sum() == pytest.approx(1200.0 * 900.0 * 600.0, rel=1e-12)
    nbr, nf = om.adjacency(m["tet_verts"], m["face_bc"])
    K = len(nbr)
    assert K == 4 * 3 * 3 * 6
    inner = nbr >= 0
    k, i = np.nonzero(inner)
    # symmetric matching with opposite normals
    assert np.all(nbr[nbr[k, i], nf[k, i]] == k)
    np.testing.assert_allclose(g["normals"][k, i], -g["normals"][nbr[k, i], nf[k, i]], atol=1e-12)
    np.testing.assert_allclose(g["areas"][k, i], g["areas"][nbr[k, i], nf[k, i]], rtol=1e-12)
    # boundary area = box surface
    bnd = ~inner
    assert g["areas"][bnd].sum() == pytest.approx(2 * (1200 * 900 + 1200 * 600 + 900 * 600), rel=1e-12)
    # free surface only on top
    top = m["face_bc"] == synth.BC_FREE
    assert g["areas"][top].sum() == pytest.approx(1200 * 900, rel=1e-12)
    np.testing.assert_allclose(g["normals"][top], np.broadcast_to([0, 0, 1.0], g["normals"][top].shape), atol=1e-12)


def test_reference_tet_and_kuhn_inradius():
    g = om.geometry(om.REF_VERTS[None])
    np.testing.assert_allclose(g["J"][0], np.eye(3))
    np.testing.assert_allclose(g["G"][0], np.eye(3))
    m = synth.kuhn_cube_periodic(6, 1000.0)
    g = om.geometry(m["tet_xyz"])
    h = 1000.0 / 6
    np.testing.assert_allclose(g["inradius"], h / (2 * (1 + np.sqrt(2))), rtol=1e-12)
    nbr, _ = om.adjacency(m["tet_verts"], m["face_bc"])
    assert np.all(nbr >= 0)            # periodic: every face matched
    assert g["vol"].sum() == pytest.approx(1e9, rel=1e-12)


def test_unmatched_untagged_face_is_an_error():
    m = synth.layered_box(2, 2, [100.0], 200.0, 200.0)
    bc = m["face_bc"].copy()
    bc[bc != 0] = 0
    with pytest.raises(om.MeshError):
        om.adjacency(m["tet_verts"], bc)


def test_locate_points_tie_break_lowest_index():
    m = synth.layered_box(2, 2, [100.0], 200.0, 200.0)
    # the box centre column edge: several tets touch (100, 100, -50)
    e, xi = om.locate_points(m["tet_xyz"], np.array([[100.0, 100.0, -50.0]]))
    X = m["tet_xyz"]
    cands = []
    for k in range(len(X)):
        J = np.stack([X[k, 1] - X[k, 0], X[k, 2] - X[k, 0], X[k, 3] - X[k, 0]], axis=1)
        r = np.linalg.solve(J, np.array([100.0, 100.0, -50.0]) - X[k, 0])
        if np.all(np.r_[1 - r.sum(), r] >= -1e-10):
            cands.append(k)
    assert len(cands) > 1 and e[0] == min(cands)


def test_full_size_box_count():
    # the anelastic LTS workload box: 67 x 67 columns, 37 layers -> 996,558 tets
    assert 67 * 67 * (4 + 3 + 30) * 6 == 996558
