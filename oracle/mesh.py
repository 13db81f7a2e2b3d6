"""Face adjacency and affine tetrahedron geometry (test infrastructure: CPU
oracle).

Sec. III-A (Discrete Formulation): conforming tetrahedral meshes; element k has four face neighbours
k_1..k_4 (the surface kernel needs them).  Face i of a tet is the face opposite
its local vertex i.  Two faces match when they carry the same three vertex ids
(periodic meshes reuse ids across the period while the coordinates stay
unwrapped).

Geometry of tet k with vertices X0..X3 in its given local order: the affine map
x(xi) = X0 + J xi with J = [X1-X0, X2-X0, X3-X0]; G = J^{-1} holds
d xi_c / d x_d.  Face normals point away from the opposite vertex.

Pins (tests/test_oracle_mesh.py): volumes sum to the box volume; every interior
face is matched exactly once from each side with opposite normals; the
reference tet maps to itself with J = I; inradius of the Kuhn tet.
"""
from __future__ import annotations

import numpy as np

REF_VERTS = np.array([[0.0, 0, 0], [1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
FACE_LOCAL = [[m for m in range(4) if m != i] for i in range(4)]


class MeshError(ValueError):
    pass


def adjacency(tet_verts, face_bc):
    """nbr [K,4] (neighbour element or -1), nbr_face [K,4] (its local face)."""
    K = tet_verts.shape[0]
    nbr = -np.ones((K, 4), dtype=np.int64)
    nbr_face = -np.ones((K, 4), dtype=np.int64)
    seen = {}
    for k in range(K):
        for i in range(4):
            key = tuple(sorted(int(tet_verts[k, m]) for m in FACE_LOCAL[i]))
            if key in seen:
                k2, i2 = seen.pop(key)
                nbr[k, i], nbr_face[k, i] = k2, i2
                nbr[k2, i2], nbr_face[k2, i2] = k, i
            else:
                seen[key] = (k, i)
    for (k, i) in seen.values():
        if face_bc[k, i] == 0:
            raise MeshError(f"face {i} of tet {k} has no neighbour and no boundary tag")
    inner = nbr >= 0
    if np.any(face_bc[inner] != 0):
        raise MeshError("a matched face carries a boundary tag")
    return nbr, nbr_face


def geometry(tet_xyz):
    X = np.asarray(tet_xyz, dtype=np.float64)
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)  # columns
    det = np.linalg.det(J)
    if np.any(np.abs(det) <= 0):
        raise MeshError("degenerate tetrahedron")
    G = np.linalg.inv(J)  # G[k, c, d] = d xi_c / d x_d
    normals = np.empty((X.shape[0], 4, 3))
    areas = np.empty((X.shape[0], 4))
    for i in range(4):
        a, b, c = FACE_LOCAL[i]
        cr = np.cross(X[:, b] - X[:, a], X[:, c] - X[:, a])
        nrm = np.linalg.norm(cr, axis=1)
        n = cr / nrm[:, None]
        s = np.einsum("kd,kd->k", n, X[:, i] - X[:, a])
        n[s > 0] *= -1.0
        normals[:, i] = n
        areas[:, i] = 0.5 * nrm
    vol = np.abs(det) / 6.0
    inradius = 3.0 * vol / areas.sum(axis=1)
    return dict(J=J, det=det, absdet=np.abs(det), G=G, normals=normals, areas=areas,
                vol=vol, inradius=inradius)


def locate_points(tet_xyz, pts, tol=1e-10):
    """Element containing each point (lowest element index among all tets whose
    barycentric coordinates are all >= -tol) and its reference coordinates."""
    X = np.asarray(tet_xyz, dtype=np.float64)
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    G = np.linalg.inv(J)
    elem = np.empty(len(pts), dtype=np.int64)
    xi = np.empty((len(pts), 3))
    for s, p in enumerate(np.asarray(pts, dtype=np.float64)):
        r = np.einsum("kcd,kd->kc", G, p[None, :] - X[:, 0])
        bary = np.concatenate([1.0 - r.sum(axis=1, keepdims=True), r], axis=1)
        ok = np.nonzero(np.all(bary >= -tol, axis=1))[0]
        if len(ok) == 0:
            raise MeshError(f"point {p} is outside the mesh")
        elem[s] = ok[0]
        xi[s] = r[ok[0]]
    return elem, xi
