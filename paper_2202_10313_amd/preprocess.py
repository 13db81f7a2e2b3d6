"""Preprocessing pipeline (Sec. VI, Production Pipeline): velocity-aware
mesh sizing, LTS clusters with the lambda search, element and face weights,
partitioning, and the reorder by partition, time cluster and communication
role, written per partition as a mesh file and an annotation file.

The steps, as the paper describes them and as built here:

1. Target edge lengths from the velocity model: a fixed number of elements
   per wavelength, h = v_min / (f_max n_epw), with v_min the slowest wave
   speed (vs).  They are sampled on a regular background grid (the role the
   paper gives to its background meshes) and interpolated trilinearly.
2. A mesh that honours them.  The paper hands the size field to an external
   volume mesher; here a coarse Kuhn-split box is refined by conforming edge
   bisection: every edge longer than the target at its midpoint is split,
   and a split divides every tetrahedron that holds the edge, so the mesh
   stays conforming after every pass.  Each tetrahedron is split only along
   its own longest edge (ties broken by a fixed edge order): a tetrahedron
   that must be split first has its longest edge split, which may mark the
   other holders of that edge in turn (longest-edge propagation); this keeps
   the element shapes close to those of the Kuhn tetrahedra.
3. CFL steps, LTS clusters and the lambda search of Sec. V-A (Clustering),
   computed by the library's host routine (edg_cluster_host).
4. Weights (Sec. V-C, Distributed Memory): element weight 2^(N_c - l), the
   updates of an element of cluster l per LTS cycle; face weight
   2^(N_c - l_a) + 2^(N_c - l_b), the buffer transfers across the face per
   cycle.
5. A partition balanced in the element weights (weighted recursive
   coordinate bisection of the element centroids; a graph partitioner that
   also minimises the weighted face cut is not part of this build).
6. The reorder: by partition, then time cluster, then role (0: every face
   neighbour in the same partition, 1: some face neighbour in another
   partition), then original index; and per partition a mesh file and an
   annotation file (clusters, materials, roles, weights, the neighbour
   partition of every face) that hold what a solver process needs without
   further communication.

CLI: python -m paper_2202_10313_amd.preprocess --help
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from . import binding

# local vertex pairs of the six tetrahedron edges
EDGES = np.array([[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]], dtype=np.int64)
KUHN = np.array([[0, 1, 3, 7], [0, 1, 5, 7], [0, 2, 3, 7], [0, 2, 6, 7], [0, 4, 5, 7], [0, 4, 6, 7]],
                dtype=np.int64)


# --------------------------------------------------------------------------- size field

def target_edge_length(vs, f_max, elements_per_wavelength):
    """h = vs / (f_max n_epw): n_epw elements per shortest (S) wavelength."""
    return np.asarray(vs, dtype=np.float64) / (float(f_max) * float(elements_per_wavelength))


class BackgroundGrid:
    """Target edge lengths sampled on a regular grid over the domain,
    interpolated trilinearly (clamped at the grid's faces)."""

    def __init__(self, axes, h):
        self.axes = [np.asarray(a, dtype=np.float64) for a in axes]
        self.h = np.asarray(h, dtype=np.float64)
        if self.h.shape != tuple(len(a) for a in self.axes):
            raise ValueError("h must have one value per grid node")

    @classmethod
    def from_velocity(cls, vs_fn, box, spacing, f_max, elements_per_wavelength):
        """Sample vs_fn (points [n,3] -> vs [n]) at the nodes of a grid of
        about `spacing` over box [[x0,x1],[y0,y1],[z0,z1]]."""
        box = np.asarray(box, dtype=np.float64)
        axes = [np.linspace(lo, hi, max(2, int(np.ceil((hi - lo) / spacing)) + 1)) for lo, hi in box]
        X, Y, Z = np.meshgrid(*axes, indexing="ij")
        pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        h = target_edge_length(vs_fn(pts), f_max, elements_per_wavelength).reshape(X.shape)
        return cls(axes, h)

    def __call__(self, p):
        p = np.atleast_2d(np.asarray(p, dtype=np.float64))
        idx, frac = [], []
        for d, a in enumerate(self.axes):
            x = np.clip(p[:, d], a[0], a[-1])
            i = np.clip(np.searchsorted(a, x, side="right") - 1, 0, len(a) - 2)
            idx.append(i)
            frac.append((x - a[i]) / (a[i + 1] - a[i]))
        out = np.zeros(len(p))
        for cx in (0, 1):
            for cy in (0, 1):
                for cz in (0, 1):
                    w = ((frac[0] if cx else 1 - frac[0]) * (frac[1] if cy else 1 - frac[1]) *
                         (frac[2] if cz else 1 - frac[2]))
                    out += w * self.h[idx[0] + cx, idx[1] + cy, idx[2] + cz]
        return out


# --------------------------------------------------------------------------- meshing

def kuhn_box(box, n, top_bc=1, side_bc=2):
    """Coarse box mesh: n = (nx, ny, nz) cubes, each split into the six Kuhn
    tetrahedra; face tags: top (z = z1) `top_bc`, the other five `side_bc`."""
    box = np.asarray(box, dtype=np.float64)
    nx, ny, nz = (int(v) for v in n)
    gi, gj, gk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    lat = np.stack([gi.ravel(), gj.ravel(), gk.ravel()], axis=1)
    V = box[:, 0] + lat * ((box[:, 1] - box[:, 0]) / np.array([nx, ny, nz]))
    vid = lambda i, j, k: (i * (ny + 1) + j) * (nz + 1) + k  # noqa: E731
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    corners = np.stack([vid(ci + (c & 1), cj + ((c >> 1) & 1), ck + ((c >> 2) & 1)) for c in range(8)], axis=1)
    T = corners[:, KUHN].reshape(-1, 4)
    BC = np.zeros(T.shape, dtype=np.int8)
    top = box[2, 1]
    for i in range(4):
        f = V[T[:, [m for m in range(4) if m != i]]]          # [K,3,3]
        for d in range(3):
            for side in (0, 1):
                on = np.all(np.abs(f[:, :, d] - box[d, side]) <= 1e-9 * (1 + abs(box[d, side])), axis=1)
                BC[on, i] = top_bc if (d == 2 and side == 1 and np.isclose(box[d, side], top)) else side_bc
    return dict(vertices=V, tets=T, face_bc=BC)


def _edge_table(T, nv):
    """Unique edges of T: (edges [E,2], per-tet edge index [K,6])."""
    a = T[:, EDGES[:, 0]]
    b = T[:, EDGES[:, 1]]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = lo * np.int64(nv) + hi
    uk, inv = np.unique(key.ravel(), return_inverse=True)
    edges = np.stack([uk // nv, uk % nv], axis=1)
    return edges, inv.reshape(T.shape[0], 6)


def refine_to_size(mesh, size_fn, max_passes=40, slack=1.0):
    """Conforming edge bisection until every edge is at most slack x the
    target length at its midpoint.  mesh: dict(vertices [n,3], tets [K,4],
    face_bc [K,4] with the tag of the face opposite each local vertex).
    Returns the refined mesh and the number of passes."""
    V = np.asarray(mesh["vertices"], dtype=np.float64).copy()
    T = np.asarray(mesh["tets"], dtype=np.int64).copy()
    BC = np.asarray(mesh["face_bc"], dtype=np.int8).copy()
    for it in range(max_passes):
        edges, te = _edge_table(T, len(V))
        P0, P1 = V[edges[:, 0]], V[edges[:, 1]]
        length = np.linalg.norm(P1 - P0, axis=1)
        viol = length > slack * size_fn(0.5 * (P0 + P1))
        if not np.any(viol):
            return dict(vertices=V, tets=T, face_bc=BC), it
        # total order: longer first, then lower edge index; every
        # tetrahedron is split only along its own longest edge
        order = np.lexsort((np.arange(len(edges)), -length))
        rank = np.empty(len(edges), dtype=np.int64)
        rank[order] = np.arange(len(edges))
        choice = np.argmin(rank[te], axis=1)
        chosen_all = te[np.arange(len(T)), choice]
        # a tetrahedron with a violating edge needs its longest edge split;
        # so does every holder of an edge that is to be split (longest-edge
        # propagation), until the set is closed
        marked = np.any(viol[te], axis=1)
        while True:
            wanted = np.zeros(len(edges), dtype=bool)
            wanted[chosen_all[marked]] = True
            grow = np.any(wanted[te], axis=1) & ~marked
            if not np.any(grow):
                break
            marked |= grow
        # split the wanted edges that are the longest edge of every holder
        holders = np.bincount(te.ravel(), minlength=len(edges))
        votes = np.bincount(chosen_all, minlength=len(edges))
        split = wanted & (votes == holders)
        if not np.any(split):
            raise RuntimeError("edge bisection made no progress")
        has = split[chosen_all]
        chosen_edge = np.where(has, chosen_all, -1)
        new_id = np.full(len(edges), -1, dtype=np.int64)
        sid = np.nonzero(split)[0]
        new_id[sid] = len(V) + np.arange(len(sid))
        V = np.concatenate([V, 0.5 * (P0[sid] + P1[sid])])
        cut = has & split[np.maximum(chosen_edge, 0)]
        keep = ~cut
        k = np.nonzero(cut)[0]
        li, lj = EDGES[choice[k], 0], EDGES[choice[k], 1]
        m = new_id[chosen_edge[k]]
        c1, c2 = T[k].copy(), T[k].copy()
        c1[np.arange(len(k)), lj] = m                # keeps vertex at li
        c2[np.arange(len(k)), li] = m                # keeps vertex at lj
        b1, b2 = BC[k].copy(), BC[k].copy()
        b1[np.arange(len(k)), li] = 0                # the new inner face
        b2[np.arange(len(k)), lj] = 0
        T = np.concatenate([T[keep], c1, c2])
        BC = np.concatenate([BC[keep], b1, b2])
    raise RuntimeError(f"the size field is not met after {max_passes} passes")


def as_solver_mesh(mesh):
    """The solver's mesh form: tet_verts [K,4], tet_xyz [K,4,3], face_bc [K,4]."""
    T = mesh["tets"]
    return dict(tet_verts=T, tet_xyz=mesh["vertices"][T], face_bc=mesh["face_bc"])


# --------------------------------------------------------------------------- clusters, weights, partitions

def face_neighbours(T):
    """[K,4] element across the face opposite each local vertex (-1 = none)."""
    K = T.shape[0]
    rows = []
    for i in range(4):
        f = np.sort(T[:, [m for m in range(4) if m != i]], axis=1)
        rows.append(np.concatenate([f, np.arange(K)[:, None], np.full((K, 1), i)], axis=1))
    F = np.concatenate(rows)
    F = F[np.lexsort((F[:, 2], F[:, 1], F[:, 0]))]
    same = np.nonzero(np.all(F[1:, :3] == F[:-1, :3], axis=1))[0]
    nbr = -np.ones((K, 4), dtype=np.int64)
    a, b = F[same], F[same + 1]
    nbr[a[:, 3], a[:, 4]] = b[:, 3]
    nbr[b[:, 3], b[:, 4]] = a[:, 3]
    return nbr


def insphere_radius(X):
    """Insphere radii of tetrahedra X [K,4,3]: 3 |V| / (sum of face areas)."""
    e1, e2, e3 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]
    vol = np.abs(np.einsum("kd,kd->k", np.cross(e1, e2), e3)) / 6.0
    area = np.zeros(len(X))
    for i in range(4):
        f = X[:, [m for m in range(4) if m != i]]
        area += 0.5 * np.linalg.norm(np.cross(f[:, 1] - f[:, 0], f[:, 2] - f[:, 0]), axis=1)
    return 3.0 * vol / area


def cfl_steps(X, vp, order, cfl=0.5):
    """dt_k = C 2 r_k / ((2(O-1)+1) vp_k), the library's CFL rule."""
    return cfl * 2.0 * insphere_radius(X) / ((2.0 * (order - 1) + 1.0) * np.asarray(vp, dtype=np.float64))


def clusters(X, nbr, vp, order, n_clusters, cfl=0.5, lam=None):
    """Sec. V-A: interval assignment, normalisation, lambda search (or the
    given lambda), by the library's host routine.  Returns (cluster ids
    1..N_c, lambda, theoretical speedup, dt_min)."""
    dt = cfl_steps(X, vp, order, cfl)
    cl, lam_out, speedup = binding.cluster_host(dt, nbr, n_clusters, lam)
    return cl, lam_out, speedup, float(dt.min())


def weights(cl, nbr, n_clusters):
    """Element weights 2^(N_c - l) (updates per LTS cycle) and face weights
    [K,4] 2^(N_c - l_a) + 2^(N_c - l_b) (buffer transfers per cycle across
    the face; 0 on boundary faces)."""
    w = np.left_shift(1, n_clusters - np.asarray(cl, dtype=np.int64))
    wn = np.where(nbr >= 0, w[np.maximum(nbr, 0)], 0)
    return w, np.where(nbr >= 0, w[:, None] + wn, 0)


def partition_rcb(centroids, w, parts):
    """Weighted recursive coordinate bisection: split the longest extent at
    the weighted median in proportion to the parts on each side."""
    part = np.zeros(len(centroids), dtype=np.int64)

    def rec(idx, p0, n):
        if n == 1 or len(idx) == 0:
            part[idx] = p0
            return
        nl = n // 2
        c = centroids[idx]
        d = int(np.argmax(c.max(axis=0) - c.min(axis=0)))
        o = idx[np.argsort(c[:, d], kind="stable")]
        cw = np.cumsum(w[o])
        cutw = cw[-1] * nl / n
        s = int(np.searchsorted(cw, cutw)) + 1
        s = min(max(s, 1), len(o) - 1) if len(o) > 1 else len(o)
        rec(o[:s], p0, nl)
        rec(o[s:], p0 + nl, n - nl)

    rec(np.arange(len(centroids)), 0, int(parts))
    return part


def roles(part, nbr):
    """1 for elements with a face neighbour in another partition, else 0."""
    pn = np.where(nbr >= 0, part[np.maximum(nbr, 0)], part[:, None])
    return np.any(pn != part[:, None], axis=1).astype(np.int8)


def reorder(part, cl, role):
    """Permutation (new position -> old index): partition, then cluster,
    then role, then original index."""
    return np.lexsort((np.arange(len(cl)), role, cl, part))


# --------------------------------------------------------------------------- pipeline

def run(vs_fn, vp_fn, rho_fn, box, coarse, f_max, epw, order, n_clusters, parts=1, cfl=0.5, lam=None,
        background_spacing=None, top_bc=1, side_bc=2):
    """The whole pipeline on a box: returns dict(mesh (solver form, reordered),
    material arrays, cluster, lambda, speedup, dt_min, weights, partition,
    role, perm (new -> old index of the refined mesh), background grid)."""
    box = np.asarray(box, dtype=np.float64)
    ext = box[:, 1] - box[:, 0]
    n = np.maximum(1, np.ceil(ext / coarse).astype(int))
    bg = BackgroundGrid.from_velocity(vs_fn, box, background_spacing or float(ext.min()) / 32.0, f_max, epw)
    coarse_mesh = kuhn_box(box, n, top_bc=top_bc, side_bc=side_bc)
    fine, passes = refine_to_size(coarse_mesh, bg)
    m = as_solver_mesh(fine)
    X = m["tet_xyz"]
    cen = X.mean(axis=1)
    vs, vp, rho = vs_fn(cen), vp_fn(cen), rho_fn(cen)
    nbr = face_neighbours(m["tet_verts"])
    cl, lam_out, speedup, dt_min = clusters(X, nbr, vp, order, n_clusters, cfl, lam)
    w_el, w_face = weights(cl, nbr, n_clusters)
    part = partition_rcb(cen, w_el, parts)
    role = roles(part, nbr)
    perm = reorder(part, cl, role)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    nb_new = np.where(nbr[perm] >= 0, inv[np.maximum(nbr[perm], 0)], -1)
    return dict(mesh={k: v[perm] for k, v in m.items()}, rho=rho[perm], vp=vp[perm], vs=vs[perm],
                cluster=cl[perm], lam=lam_out, speedup=speedup, dt_min=dt_min, element_weight=w_el[perm],
                face_weight=w_face[perm], partition=part[perm], role=role[perm], nbr=nb_new, perm=perm,
                background=bg, passes=passes, n_clusters=n_clusters, order=order)


def write_partitions(res, prefix):
    """Per partition p: <prefix>_p<p>_mesh.npz (tet_verts, tet_xyz, face_bc,
    global ids in the reordered numbering) and <prefix>_p<p>_annot.npz
    (cluster, rho, vp, vs, role, element and face weights, the neighbour's
    global id and partition of every face, and the clustering figures), plus
    <prefix>_summary.json.  Plain arrays only (no pickles)."""
    part = res["partition"]
    files = []
    for p in range(int(part.max()) + 1):
        ids = np.nonzero(part == p)[0]
        nb = res["nbr"][ids]
        np.savez(f"{prefix}_p{p}_mesh.npz", global_id=ids, **{k: v[ids] for k, v in res["mesh"].items()})
        np.savez(f"{prefix}_p{p}_annot.npz", global_id=ids, cluster=res["cluster"][ids], rho=res["rho"][ids],
                 vp=res["vp"][ids], vs=res["vs"][ids], role=res["role"][ids],
                 element_weight=res["element_weight"][ids], face_weight=res["face_weight"][ids],
                 neighbour=nb, neighbour_partition=np.where(nb >= 0, part[np.maximum(nb, 0)], -1),
                 lam=res["lam"], speedup=res["speedup"], dt_min=res["dt_min"], n_clusters=res["n_clusters"],
                 order=res["order"])
        files.append((f"{prefix}_p{p}_mesh.npz", f"{prefix}_p{p}_annot.npz"))
    cl = res["cluster"]
    summary = {"tets": int(len(cl)), "passes": int(res["passes"]), "lambda": float(res["lam"]),
               "theoretical_lts_speedup": float(res["speedup"]), "dt_min": float(res["dt_min"]),
               "cluster_sizes": np.bincount(cl, minlength=res["n_clusters"] + 1)[1:].tolist(),
               "partition_weights": np.bincount(part, weights=res["element_weight"]).tolist(),
               "cut_face_weight": float(np.sum(np.where(
                   (res["nbr"] >= 0) & (part[np.maximum(res["nbr"], 0)] != part[:, None]), res["face_weight"], 0)) / 2),
               "files": files}
    with open(f"{prefix}_summary.json", "w") as f:
        json.dump(summary, f, indent=1)
    return summary


def layered_model(spec):
    """vs(depth) from 'd0:vs0,d1:vs1,...' (vs below depth d_i, depth = -z),
    vp = ratio vs, Gardner density 310 vp^0.25."""
    pairs = sorted((float(a), float(b)) for a, b in (item.split(":") for item in spec.split(",")))
    d = np.array([p[0] for p in pairs])
    v = np.array([p[1] for p in pairs])

    def vs(p):
        depth = -np.asarray(p)[:, 2]
        return v[np.clip(np.searchsorted(d, depth, side="right") - 1, 0, len(v) - 1)]
    return vs


def main(argv=None):
    ap = argparse.ArgumentParser(description="velocity-aware meshing, LTS clustering, partition and reorder")
    ap.add_argument("--box", type=float, nargs=6, required=True, metavar=("X0", "X1", "Y0", "Y1", "Z0", "Z1"))
    ap.add_argument("--layers", required=True, help="depth:vs pairs, e.g. '0:800,300:1000,600:1400,1000:2000'")
    ap.add_argument("--vpvs", type=float, default=1.8)
    ap.add_argument("--coarse", type=float, required=True, help="edge of the coarse cubes [m]")
    ap.add_argument("--fmax", type=float, required=True, help="highest frequency to resolve [Hz]")
    ap.add_argument("--epw", type=float, default=2.0, help="elements per shortest wavelength")
    ap.add_argument("--order", type=int, default=5)
    ap.add_argument("--clusters", type=int, default=3)
    ap.add_argument("--lam", type=float, default=None, help="fixed lambda (default: search)")
    ap.add_argument("--parts", type=int, default=1)
    ap.add_argument("--out", required=True, help="output prefix")
    a = ap.parse_args(argv)
    vs = layered_model(a.layers)
    box = np.array(a.box).reshape(3, 2)
    res = run(vs, lambda p: a.vpvs * vs(p), lambda p: 310.0 * (a.vpvs * vs(p)) ** 0.25, box, a.coarse, a.fmax,
              a.epw, a.order, a.clusters, a.parts, lam=a.lam)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    print(json.dumps(write_partitions(res, a.out), indent=1))


if __name__ == "__main__":
    main()
