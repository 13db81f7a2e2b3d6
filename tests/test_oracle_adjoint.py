"""Pins of the oracle's discrete adjoint and material gradient (CPU).

* The closed-form flux maps (used only to differentiate the flux in the
  materials) equal the eigenvector-built Godunov flux of the forward oracle.
* Dot-product identity <G x, y> = <x, G^T y> for the state map G: initial DOFs
  -> (final DOFs, seismogram samples), elastic and anelastic, one to three
  clusters, free-surface and absorbing boundaries.
* The material gradient against central finite differences of a misfit along
  20 random directions (FP64, frozen clusters and time steps).
"""
import numpy as np
import pytest

import synth
from oracle import physics as ph
from oracle.adjoint import adjoint
from oracle.solver import Oracle

REC = dict(xyz=np.array([[150.0, 170.0, -20.0], [260.0, 300.0, -150.0]]), dt_sample=2e-3, n_samples=40)
SRC = dict(xyz=np.array([[200.0, 210.0, -90.0]]), moment=np.array([[1e9, -2e9, 0.5e9, 3e9, 1e9, -1e9]]),
           stf_kind=0, stf_params=np.array([[200.0, 0.004]]))


def _mesh(seed=3):
    mesh = synth.layered_box(2, 2, [100.0, 200.0], 400.0, 400.0, jitter=0.15, seed=seed)
    K = mesh["tet_verts"].shape[0]
    mat = synth.random_materials(K, 4)
    return mesh, mat


def _distance_clusters(orc, n_clusters):
    """Clusters 1 + graph distance from element 0, capped at N_c (neighbours
    differ by at most one, so the clustering is normalised)."""
    dist = np.full(orc.K, -1)
    dist[0] = 0
    front = [0]
    while front:
        nxt = []
        for k in front:
            for j in orc.nbr[k]:
                if j >= 0 and dist[j] < 0:
                    dist[j] = dist[k] + 1
                    nxt.append(j)
        front = nxt
    return np.minimum(1 + dist, n_clusters)


def test_closed_form_flux_equals_eigenvector_godunov():
    mesh, mat = _mesh()
    attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
    orc = Oracle(mesh, mat, 2, attn=attn)
    kinds = set()
    for i in range(4):
        nb = orc.nbr[:, i]
        other = np.where(nb >= 0, nb, np.arange(orc.K))
        kind = np.where(nb >= 0, 0, orc.face_bc[:, i])
        kinds |= set(kind.tolist())
        Fm, Fp = ph.flux_matrices_closed(orc.geo["normals"][:, i], orc.rho, orc.vp, orc.vs, orc.rho[other],
                                         orc.vp[other], orc.vs[other], kind, orc.omega)
        assert np.abs(Fm - orc.Fm[:, i]).max() <= 1e-13 * np.abs(orc.Fm[:, i]).max()
        assert np.abs(Fp - orc.Fp[:, i]).max() <= 1e-13 * np.abs(orc.Fm[:, i]).max()
    assert kinds == {0, 1, 2}


@pytest.mark.parametrize("order,mech,n_clusters", [(2, 0, 1), (3, 3, 2), (2, 3, 3), (4, 0, 2)])
def test_dot_product_identity(order, mech, n_clusters):
    mesh, mat = _mesh()
    attn = synth.attenuation_inputs(mat, mech, 0.1, 10.0) if mech else None
    base = Oracle(mesh, mat, order, attn=attn)
    cl = _distance_clusters(base, n_clusters)
    dt_min = float(base.dt_cfl.min()) / 2 ** (n_clusters - 1)

    def make():
        return Oracle(mesh, mat, order, attn=attn, n_clusters=n_clusters, lam=1.0, clusters=cl, dt_min=dt_min,
                      receivers=REC)

    orc = make()
    assert len(np.unique(orc.cl)) == n_clusters
    rng = np.random.default_rng(order + 10 * mech + 100 * n_clusters)
    x = synth.random_state(2, orc.K, orc.nq, orc.B)
    y = rng.standard_normal(orc.Q.shape) * np.where(np.arange(orc.nq) < 6, 1e-6, 1.0)[None, :, None]
    sb = rng.standard_normal((2, REC["n_samples"], 9))
    t = 2 * orc.sync_dt
    orc.set_initial(x)
    orc.run(t)
    assert np.any(orc.seis != 0)
    lhs = np.sum(orc.Q * y) + np.sum(orc.seis * sb)
    orc2 = make()
    res = adjoint(orc2, t, seis_b=sb, q_b=y, attn=attn)
    rhs = np.sum(x * res["q0_b"])
    scale = np.sum(np.abs(orc.Q * y)) + np.sum(np.abs(orc.seis * sb))
    assert abs(lhs - rhs) <= 1e-13 * scale, (lhs, rhs)


@pytest.mark.parametrize("mech", [3, 0])
def test_gradient_matches_central_differences(mech):
    mesh, mat = _mesh()
    K = mesh["tet_verts"].shape[0]
    attn = synth.attenuation_inputs(mat, mech, 0.1, 10.0) if mech else None
    base = Oracle(mesh, mat, 3, attn=attn, n_clusters=2, lam=None)
    assert len(np.unique(base.cl)) == 2
    frozen = dict(n_clusters=2, lam=base.lam_lts, clusters=base.cl, dt_min=base.dt_min)
    rng = np.random.default_rng(7 + mech)
    x = synth.random_state(2, K, base.nq, base.B)
    y = rng.standard_normal(base.Q.shape) * 1e-6
    sb = rng.standard_normal((2, REC["n_samples"], 9))
    t = 3 * base.sync_dt

    def J(m):
        o = Oracle(mesh, m, 3, attn=attn, receivers=REC, sources=SRC, **frozen)
        o.set_initial(x)
        o.run(t)
        return np.sum(o.Q * y) + np.sum(o.seis * sb)

    o = Oracle(mesh, mat, 3, attn=attn, receivers=REC, sources=SRC, **frozen)
    o.set_initial(x)
    res = adjoint(o, t, seis_b=sb, q_b=y, attn=attn)
    eps = 1e-5
    worst = 0.0
    for _ in range(20):
        d = {k: rng.standard_normal(K) * mat[k] for k in ("rho", "vp", "vs")}
        pred = sum(np.sum(res["g_" + k] * d[k]) for k in ("rho", "vp", "vs"))
        mp = {k: mat[k] + eps * d[k] for k in ("rho", "vp", "vs")}
        mm = {k: mat[k] - eps * d[k] for k in ("rho", "vp", "vs")}
        fd = (J(mp) - J(mm)) / (2 * eps)
        worst = max(worst, abs(pred - fd) / abs(fd))
    print(f"oracle gradient vs central differences (m={mech}): worst relative error {worst:.2e}")
    assert worst <= 1e-6
