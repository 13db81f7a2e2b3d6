"""Shared test helpers: build the same seeded workload for the oracle and the
GPU library, and the parity metric."""
import math

import numpy as np

import synth

GROUPS_ELASTIC = [(0, 6), (6, 9)]


def groups(nq):
    g = list(GROUPS_ELASTIC)
    for l in range((nq - 9) // 6):
        g.append((9 + 6 * l, 15 + 6 * l))
    return g


def parity(a, b):
    """Max over quantities of ||a_q - b_q|| / ||b_group(q)|| (relative L2 over
    all elements and modes; a quantity is measured against the norm of its
    group -- stresses, velocities, one mechanism's memory variables -- so that
    quantities that vanish do not divide by zero), and per element: the max
    over elements k and groups g of ||a_kg - b_kg|| / max(||b_kg||, rms_g),
    rms_g = ||b_g|| / sqrt(K), so that one wrong element of a large mesh is
    not diluted by the others."""
    worst = 0.0
    K = a.shape[0]
    for (g0, g1) in groups(a.shape[1]):
        den = np.linalg.norm(b[:, g0:g1])
        if den == 0:
            den = 1.0
        for q in range(g0, g1):
            worst = max(worst, np.linalg.norm(a[:, q] - b[:, q]) / den)
        ek = np.sqrt(np.sum((a[:, g0:g1] - b[:, g0:g1]) ** 2, axis=tuple(range(1, a.ndim))))
        bk = np.sqrt(np.sum(b[:, g0:g1] ** 2, axis=tuple(range(1, b.ndim))))
        worst = max(worst, float(np.max(ek / np.maximum(bk, den / math.sqrt(K)))))
    return worst


def seis_parity(a, b):
    """Relative L2 per receiver component group (stresses / velocities)."""
    worst = 0.0
    for (g0, g1) in GROUPS_ELASTIC:
        den = np.linalg.norm(b[..., g0:g1]) or 1.0
        worst = max(worst, np.linalg.norm(a[..., g0:g1] - b[..., g0:g1]) / den)
    return worst


def anelastic_setup(scale, order, n_clusters, seed=20, with_source=True, n_rec=6, lam=None):
    """Layered box workload (free surface on top, absorbing elsewhere, 3
    mechanisms, layered materials with perturbations, one Ricker source and
    surface receivers) at a given scale."""
    mesh = synth.loh_like_box(scale, seed=seed)
    mat = synth.layered_materials(mesh, seed + 1)
    attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
    box = mesh["box"]
    src = None
    if with_source:
        src = synth.ricker_sources(seed + 2, 1, ((box[0, 0] + 0.3 * (box[0, 1] - box[0, 0]), box[0, 0] + 0.7 * (box[0, 1] - box[0, 0])),
                                              (box[1, 0] + 0.3 * (box[1, 1] - box[1, 0]), box[1, 0] + 0.7 * (box[1, 1] - box[1, 0]))),
                                   (0.2 * -box[2, 0], 0.6 * -box[2, 0]), fc_range=(8.0, 8.0))
    rec = synth.surface_receivers(seed + 3, n_rec, ((box[0, 0] + 50, box[0, 1] - 50), (box[1, 0] + 50, box[1, 1] - 50)))
    return dict(mesh=mesh, mat=mat, attn=attn, src=src, rec=rec)


def gpu_context(w, order, n_clusters, fp64, lam=None, clusters=None, mechanisms=3, n_runs=1):
    from paper_2202_10313_amd import Context
    ctx = Context(order, mechanisms=mechanisms, n_clusters=n_clusters, fp64=fp64, cfl=0.5, lam=lam, n_runs=n_runs)
    m = w["mesh"]
    ctx.upload_mesh(m["tet_verts"], m["tet_xyz"], m["face_bc"])
    a = w.get("attn")
    if mechanisms:
        ctx.upload_materials(w["mat"]["rho"], w["mat"]["vp"], w["mat"]["vs"], a["omega"], a["yp"], a["ys"])
    else:
        ctx.upload_materials(w["mat"]["rho"], w["mat"]["vp"], w["mat"]["vs"])
    ctx.upload_clusters(clusters)
    return ctx


def random_direction_wavevector(seed, L=1000.0):
    """Plane-wave direction drawn uniformly on the sphere; the wave vector is
    rounded to the periodic lattice: m = round(2 n) (never zero)."""
    rng = np.random.default_rng(seed)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    m = np.round(2 * n)
    if not np.any(m):
        m[np.argmax(np.abs(n))] = 1.0
    return m / np.linalg.norm(m), 2 * math.pi * np.linalg.norm(m) / L


def face_adjacency(tet_verts):
    """[K,4] face neighbours (-1 = none) by sorting face vertex triples
    (vectorised, for million-element meshes)."""
    K = tet_verts.shape[0]
    rows = []
    for i in range(4):
        f = np.sort(tet_verts[:, [m for m in range(4) if m != i]], axis=1)
        rows.append(np.concatenate([f, np.arange(K)[:, None], np.full((K, 1), i)], axis=1))
    F = np.concatenate(rows)
    F = F[np.lexsort((F[:, 2], F[:, 1], F[:, 0]))]
    same = np.nonzero(np.all(F[1:, :3] == F[:-1, :3], axis=1))[0]
    nbr = -np.ones((K, 4), dtype=np.int64)
    a, b = F[same], F[same + 1]
    nbr[a[:, 3], a[:, 4]] = b[:, 3]
    nbr[b[:, 3], b[:, 4]] = a[:, 3]
    return nbr


def graph_ball(nbr, seeds, radius):
    """Element ids within `radius` face hops of the seeds."""
    seen = np.zeros(nbr.shape[0], dtype=bool)
    seen[seeds] = True
    front = np.asarray(seeds)
    for _ in range(radius):
        cand = nbr[front].ravel()
        cand = np.unique(cand[cand >= 0])
        cand = cand[~seen[cand]]
        seen[cand] = True
        front = cand
    return np.nonzero(seen)[0]


def submesh(mesh, ids, nbr):
    """Sub-mesh of the elements `ids`: faces whose neighbour is outside become
    absorbing."""
    idx = np.asarray(ids)
    inside = np.zeros(mesh["tet_verts"].shape[0], dtype=bool)
    inside[idx] = True
    bc = mesh["face_bc"][idx].copy()
    cut = (nbr[idx] >= 0) & ~inside[np.maximum(nbr[idx], 0)]
    bc[cut] = 2
    return dict(tet_verts=mesh["tet_verts"][idx], tet_xyz=mesh["tet_xyz"][idx], face_bc=bc)
