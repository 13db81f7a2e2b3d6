"""CPU checks of the library's face flux and of its reverse mode (the
transpose the adjoint kernels apply), through the host entry point
edg_godunov_host.  No device work.

* The flux equals -s (Fm q- + Fp q+) of the oracle's Godunov flux maps
  (elastic rows; the memory-variable rows per unit omega) for interior,
  free-surface and absorbing faces of heterogeneous media.
* Its reverse mode satisfies <u, out> = <qm_b, qm> + <qp_b, qp> (the flux is
  linear in the traces) and its parameter derivatives match central
  differences.
"""
import numpy as np
import pytest

from oracle import physics as ph
from paper_2202_10313_amd.binding import godunov_host


def _face(rng):
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    rho, rho_n = rng.uniform(1800, 3000, 2)
    vs, vs_n = rng.uniform(800, 3500, 2)
    vp, vp_n = vs * rng.uniform(1.6, 2.2), vs_n * rng.uniform(1.6, 2.2)
    return n, (rho, vp, vs), (rho_n, vp_n, vs_n)


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_flux_matches_oracle_godunov(bc):
    rng = np.random.default_rng(10 + bc)
    omega = np.array([0.7, 6.0, 60.0])
    for _ in range(5):
        n, (rho, vp, vs), (rho_n, vp_n, vs_n) = _face(rng)
        s = rng.uniform(0.1, 3.0)
        lam, mu = rho * vp * vp - 2 * rho * vs * vs, rho * vs * vs
        zpp, zsp = (rho_n * vp_n, rho_n * vs_n) if bc == 0 else (rho * vp, rho * vs)
        prm = np.array([*n, rho * vp, rho * vs, zpp, zsp, lam, mu, 1.0 / rho, s])
        qm = rng.standard_normal(9) * np.r_[np.full(6, 1e6), np.ones(3)]
        qp = rng.standard_normal(9) * np.r_[np.full(6, 1e6), np.ones(3)]
        out = godunov_host(bc, qm, qp, prm, np.zeros(15))[0]
        Fm, Fp = ph.flux_matrices_closed(n[None], np.array([rho]), np.array([vp]), np.array([vs]),
                                         np.array([rho_n]), np.array([vp_n]), np.array([vs_n]),
                                         np.array([bc]), omega)
        flux = Fm[0] @ qm + (Fp[0] @ qp if bc == 0 else 0.0)
        want = -s * flux
        np.testing.assert_allclose(out[:9], want[:9], rtol=1e-12, atol=1e-12 * np.abs(want[:9]).max())
        for l in range(3):
            w = want[9 + 6 * l: 15 + 6 * l] / omega[l]
            np.testing.assert_allclose(out[9:], w, rtol=1e-12, atol=1e-12 * np.abs(w).max())


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_reverse_mode_is_the_transpose(bc):
    rng = np.random.default_rng(20 + bc)
    for _ in range(5):
        n, (rho, vp, vs), (rho_n, vp_n, vs_n) = _face(rng)
        prm = np.array([*n, rho * vp, rho * vs, rho_n * vp_n, rho_n * vs_n, rho * vp * vp - 2 * rho * vs * vs,
                        rho * vs * vs, 1.0 / rho, 0.8])
        qm, qp, u = rng.standard_normal(9), rng.standard_normal(9), rng.standard_normal(15)
        out, qmb, qpb, _ = godunov_host(bc, qm, qp, prm, u)
        lhs = u @ out
        rhs = qmb @ qm + qpb @ qp
        assert abs(lhs - rhs) <= 1e-14 * (np.abs(u) @ np.abs(out))
        if bc != 0:
            assert not np.any(qpb)


@pytest.mark.parametrize("bc", [0, 1, 2])
def test_reverse_mode_parameter_derivatives(bc):
    # unit-scale parameters so that central differences resolve every term
    rng = np.random.default_rng(30 + bc)
    for _ in range(3):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        prm = np.array([*n, *rng.uniform(0.5, 1.5, 4), *rng.uniform(0.5, 1.5, 3), 0.37])
        qm, qp, u = rng.standard_normal(9), rng.standard_normal(9), rng.standard_normal(15)
        _, _, _, pb = godunov_host(bc, qm, qp, prm, u)
        for k, pi in enumerate([9, 7, 8, 3, 4, 5, 6]):    # 1/rho, lam, mu, Zp-, Zs-, Zp+, Zs+
            h = 1e-6
            pp, pm = prm.copy(), prm.copy()
            pp[pi] += h
            pm[pi] -= h
            fd = (u @ godunov_host(bc, qm, qp, pp, u)[0] - u @ godunov_host(bc, qm, qp, pm, u)[0]) / (2 * h)
            assert abs(pb[k] - fd) <= 1e-7 * max(1.0, abs(fd)), (k, pb[k], fd)
