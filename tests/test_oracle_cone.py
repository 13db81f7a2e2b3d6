"""The locality argument behind the full-size sampled parity test, checked on
the oracle alone: after one LTS cycle with N_c = 3 (4 finest steps), an
element's state equals the state computed on the sub-mesh of its 4-hop ball
(faces leaving the ball absorbing), with the whole mesh's clusters, lambda and
dt_min (Sec. V-B (Buffers and Algorithm): every update ending at time t reads
neighbour predictions that start at an earlier multiple of the finest step).
When every element is in the finest cluster a 3-hop ball is not enough, which
shows that the radius is tight and that the comparison sees a wrong
boundary."""
import numpy as np

import synth
from helpers import face_adjacency, graph_ball, parity, submesh
from oracle.solver import Oracle

ORDER, NC = 2, 3


def _workload():
    # 4 x 4 columns of the layered box's spacing and layering, 13 layers:
    # 1,248 tets in all three clusters
    h = 20000.0 / 67
    mesh = synth.layered_box(4, 4, [100.0] * 4 + [200.0] * 3 + [300.0] * 6, 4 * h, 4 * h, jitter=0.15, seed=20)
    mat = synth.layered_materials(mesh, 21)
    attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
    return mesh, mat, attn


def _run(mesh, mat, attn, ids, q0, lam, clusters, dt_min, nbr):
    """Oracle on the sub-mesh `ids` (None = whole mesh) for one cycle."""
    m = mesh if ids is None else submesh(mesh, ids, nbr)
    sel = slice(None) if ids is None else ids
    orc = Oracle(m, {k: mat[k][sel] for k in ("rho", "vp", "vs")}, ORDER,
                 attn=dict(omega=attn["omega"], yp=attn["yp"][sel], ys=attn["ys"][sel]), n_clusters=NC,
                 cfl=0.5, lam=lam, clusters=None if clusters is None else clusters[sel], dt_min=dt_min)
    orc.set_initial(q0[sel])
    orc.run(orc.sync_dt)
    return orc


def test_four_hop_cone_is_exact():
    mesh, mat, attn = _workload()
    nbr = face_adjacency(mesh["tet_verts"])
    K = mesh["tet_verts"].shape[0]
    q0 = synth.random_state(3, K, 27, 4)
    full = _run(mesh, mat, attn, None, q0, None, None, None, nbr)
    assert set(np.unique(full.cl)) == {1, 2, 3}
    ncl = np.where(nbr >= 0, full.cl[np.maximum(nbr, 0)], full.cl[:, None])
    interface = np.nonzero(np.any(ncl != full.cl[:, None], axis=1))[0]
    rng = np.random.default_rng(0)
    seeds = np.unique(np.concatenate([rng.choice(np.nonzero(full.cl == l)[0], 3, replace=False)
                                      for l in (1, 2, 3)] + [rng.choice(interface, 3, replace=False)]))
    U = graph_ball(nbr, seeds, 4)
    sub = _run(mesh, mat, attn, U, q0, full.lam_lts, full.cl, full.dt_min, nbr)
    assert parity(sub.Q[np.searchsorted(U, seeds)], full.Q[seeds]) <= 1e-12


def test_three_hops_are_not_enough_when_all_elements_are_finest():
    mesh, mat, attn = _workload()
    nbr = face_adjacency(mesh["tet_verts"])
    K = mesh["tet_verts"].shape[0]
    q0 = synth.random_state(4, K, 27, 4)
    ones = np.ones(K, dtype=np.int64)
    full = _run(mesh, mat, attn, None, q0, 1.0, ones, None, nbr)
    assert full.updates == 4 * K
    # interior elements of the 100 m layers (no boundary face within 4 hops)
    seeds = np.array([k for k in range(0, K, 7) if not np.any(mesh["face_bc"][graph_ball(nbr, [k], 4)])])[:4]
    assert len(seeds) > 0
    for hops, expect_exact in ((4, True), (3, False)):
        U = graph_ball(nbr, seeds, hops)
        sub = _run(mesh, mat, attn, U, q0, 1.0, ones, full.dt_min, nbr)
        err = parity(sub.Q[np.searchsorted(U, seeds)], full.Q[seeds])
        assert (err <= 1e-12) if expect_exact else (err > 1e-6), (hops, err)
