"""Pins of the oracle's Jacobians and Riemann solver against closed forms and
library routines (no GPU)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import physics as ph


def _rand_unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _mats(rng, n):
    vs = rng.uniform(500, 3500, n)
    vp = vs * rng.uniform(1.6, 2.2, n)
    rho = rng.uniform(1800, 3000, n)
    lam, mu = ph.lame(rho, vp, vs)
    return rho, vp, vs, lam, mu


def _An(rho, lam, mu, n, m=0):
    A = ph.jacobians(rho, lam, mu, np.linspace(1, 2, m))
    return ph.normal_jacobian(A, n)


def test_elastic_eigenvalues():
    rng = np.random.default_rng(1)
    rho, vp, vs, lam, mu = _mats(rng, 20)
    n = _rand_unit(rng, 20)
    An = _An(rho, lam, mu, n)[:, :9, :9]
    for f in range(20):
        ev = np.sort(np.linalg.eigvals(An[f]).real)
        want = np.sort([vp[f], -vp[f], vs[f], vs[f], -vs[f], -vs[f], 0, 0, 0])
        np.testing.assert_allclose(ev, want, atol=1e-8 * vp[f])


def test_p_eigenvector_closed_form():
    rng = np.random.default_rng(2)
    rho, vp, vs, lam, mu = _mats(rng, 5)
    n = _rand_unit(rng, 5)
    An = _An(rho, lam, mu, n)[:, :9, :9]
    for f in range(5):
        sig = -(lam[f] * np.eye(3) + 2 * mu[f] * np.outer(n[f], n[f])) / vp[f]
        r = np.array([sig[0, 0], sig[1, 1], sig[2, 2], sig[0, 1], sig[1, 2], sig[0, 2], *n[f]])
        np.testing.assert_allclose(An[f] @ r, vp[f] * r, rtol=1e-12, atol=1e-6)


def test_anelastic_rows_scale_with_omega():
    rng = np.random.default_rng(3)
    rho, vp, vs, lam, mu = _mats(rng, 3)
    om = np.array([0.7, 3.0, 11.0])
    A = ph.jacobians(rho, lam, mu, om)
    for l in range(3):
        blk = A[:, :, 9 + 6 * l:15 + 6 * l, :]
        np.testing.assert_allclose(blk / om[l], A[:, :, 9:15, :] / om[0], rtol=1e-14)
    # memory rows only see velocities; memory columns are empty
    assert np.all(A[:, :, 9:, :6] == 0) and np.all(A[:, :, :, 9:] == 0)


def test_homogeneous_godunov_is_upwind():
    rng = np.random.default_rng(4)
    F = 12
    rho, vp, vs, lam, mu = _mats(rng, F)
    n = _rand_unit(rng, F)
    An = _An(rho, lam, mu, n)[:, :9, :9]
    Gm, Gp = ph.godunov_matrices(An, An, n, np.zeros(F, dtype=int))
    for f in range(F):
        absA = scipy.linalg.sqrtm(An[f] @ An[f]).real
        flux_m = An[f] @ Gm[f]
        flux_p = An[f] @ Gp[f]
        np.testing.assert_allclose(flux_m, 0.5 * (An[f] + absA), atol=1e-6 * np.abs(An[f]).max())
        np.testing.assert_allclose(flux_p, 0.5 * (An[f] - absA), atol=1e-6 * np.abs(An[f]).max())


def test_normal_incidence_reflection():
    rng = np.random.default_rng(5)
    rho, vp, vs, lam, mu = _mats(rng, 2)
    n = np.array([[0.0, 0.0, 1.0]])
    Am = _An(rho[:1], lam[:1], mu[:1], n)[:, :9, :9]
    Ap = _An(rho[1:], lam[1:], mu[1:], n)[:, :9, :9]
    Gm, Gp = ph.godunov_matrices(Am, Ap, n, np.zeros(1, dtype=int))
    Z1, Z2 = rho[0] * vp[0], rho[1] * vp[1]
    # right-going P wave in (-) with unit velocity along n: sigma_zz = -Z1
    sig = -(lam[0] * np.eye(3) + 2 * mu[0] * np.outer(n[0], n[0])) / vp[0]
    qin = np.array([sig[0, 0], sig[1, 1], sig[2, 2], sig[0, 1], sig[1, 2], sig[0, 2], 0, 0, 1.0])
    qs = Gm[0] @ qin
    refl = qs - qin
    # reflected velocity / incident velocity = (Z1-Z2)/(Z1+Z2); traction: (Z2-Z1)/(Z1+Z2)
    assert abs(refl[8] - (Z1 - Z2) / (Z1 + Z2)) < 1e-10
    assert abs(refl[2] / qin[2] - (Z2 - Z1) / (Z1 + Z2)) < 1e-10


def test_free_surface_zero_traction():
    rng = np.random.default_rng(6)
    F = 8
    rho, vp, vs, lam, mu = _mats(rng, F)
    n = _rand_unit(rng, F)
    An = _An(rho, lam, mu, n)[:, :9, :9]
    Gm, Gp = ph.godunov_matrices(An, An, n, np.ones(F, dtype=int))
    q = rng.normal(size=(F, 9))
    qs = np.einsum("fij,fj->fi", Gm, q)
    tr = np.einsum("fij,fj->fi", ph.traction_op(n), qs)
    np.testing.assert_allclose(tr, 0.0, atol=1e-9 * np.abs(q).max())
    assert np.all(Gp == 0)
    # normal-incidence reflection at the free surface: traction coefficient -1
    # (the interface velocity doubles)
    lam0, mu0 = lam[0], mu[0]
    nz = np.array([[0, 0, 1.0]])
    A0 = _An(rho[:1], lam[:1], mu[:1], nz)[:, :9, :9]
    G0, _ = ph.godunov_matrices(A0, A0, nz, np.ones(1, dtype=int))
    sig = -(lam0 * np.eye(3) + 2 * mu0 * np.eye(3)[2:3].T @ np.eye(3)[2:3]) / vp[0]
    qin = np.array([sig[0, 0], sig[1, 1], sig[2, 2], 0, 0, 0, 0, 0, 1.0])
    assert abs((G0[0] @ qin)[8] - 2.0) < 1e-10


def test_absorbing_equals_zero_ghost():
    rng = np.random.default_rng(7)
    F = 8
    rho, vp, vs, lam, mu = _mats(rng, F)
    n = _rand_unit(rng, F)
    An = _An(rho, lam, mu, n)[:, :9, :9]
    Ga, _ = ph.godunov_matrices(An, An, n, np.full(F, 2))
    Gi, _ = ph.godunov_matrices(An, An, n, np.zeros(F, dtype=int))
    # flux of the absorbing state == Godunov flux against a zero outside state
    np.testing.assert_allclose(An @ Ga, An @ Gi, atol=1e-7 * np.abs(An).max())


def test_coupling_structure():
    rng = np.random.default_rng(8)
    rho, vp, vs, lam, mu = _mats(rng, 4)
    om = np.array([1.0, 5.0, 20.0])
    yp = rng.uniform(0, 0.1, (4, 3))
    ys = rng.uniform(0, 0.1, (4, 3))
    E = ph.coupling(lam, mu, yp, ys, om)
    # pure dilatational memory (theta = I): stress change -(3 a + b) I = -(3K-ish)
    for l in range(3):
        th = np.zeros(27)
        th[9 + 6 * l:9 + 6 * l + 3] = 1.0
        ds = E @ th
        a = (lam + 2 * mu) * yp[:, l] - 2 * mu * ys[:, l]
        b = 2 * mu * ys[:, l]
        np.testing.assert_allclose(ds[:, :3], -(3 * a + b)[:, None] * np.ones((1, 3)), rtol=1e-13)
        # lambda*Y_lambda with Y_lambda = (1 + 2mu/lambda) Yp - (2mu/lambda) Ys
        ylam = (1 + 2 * mu / lam) * yp[:, l] - (2 * mu / lam) * ys[:, l]
        np.testing.assert_allclose(a, lam * ylam, rtol=1e-12)
        np.testing.assert_allclose(np.diagonal(E, axis1=1, axis2=2)[:, 9 + 6 * l:15 + 6 * l], -om[l])
