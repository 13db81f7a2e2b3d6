"""Anelastic wave equations: Jacobians, coupling and the Riemann solver (test
infrastructure: CPU oracle).

Sec. III (ADER-DG Finite Element Method, eq. hyp_sys): q_t + A q_x + B q_y + C q_z = E q with
q = (sigma_xx, sigma_yy, sigma_zz, sigma_xy, sigma_yz, sigma_xz, u, v, w,
     theta^1_xx .. theta^1_xz, ..., theta^m_xx .. theta^m_xz).
The paper names u, v and "v" for the velocities; the third is read as w.
The Jacobians carry an elastic 9x9 block and an anelastic 6x9 block that only
touches the velocities; E couples the memory variables into the stresses and
relaxes them (its diagonal part E').  The paper delegates the entries to its
references; this oracle writes out the standard velocity-stress system:

  d/dt sigma      = lambda tr(eps') I + 2 mu eps'
                    - sum_l [a_l tr(theta^l) I + b_l theta^l]
  rho d/dt v      = div sigma
  d/dt theta^l    = omega_l (eps' - theta^l)        eps' = sym grad v

with a_l = (lambda + 2 mu) Y^P_l - 2 mu Y^S_l (= lambda Y^lambda_l) and
b_l = 2 mu Y^S_l.  lambda, mu are the unrelaxed moduli from (rho, vp, vs).
The relaxation sign is the decaying one (-omega_l); the time-kernel equation of
Sec. III-A (Discrete Formulation) prints +omega_l, the volume kernel -omega_l, and only the latter is
stable.

Riemann solver (the paper gives none): Godunov.  For a face with unit normal n
pointing from the element (-) to its neighbour (+), the interface state keeps
each side's outgoing characteristics and makes traction sigma n and velocity
continuous.  It is built here from eigenvectors: q*- = q- + R- alpha with R-
the eigenvectors of A_n^- with negative speeds, q*+ = q+ + R+ beta with R+ those
of A_n^+ with positive speeds, and the 6x6 continuity system solved for
(alpha, beta).  The flux seen by the element is A_n^- q*-.
Free surface: traction of q* is zero.  Absorbing: the incoming characteristic
amplitudes of q- are removed (projector built from left eigenvectors).

Pins (tests/test_oracle_physics.py): eigenvalues {+-vp, +-vs x2, 0 x3}; the
homogeneous flux equals 1/2 A_n (q- + q+) + 1/2 |A_n| (q- - q+) with
|A_n| = R |Lambda| R^-1; normal-incidence reflection (Z2-Z1)/(Z2+Z1); zero
traction at the free surface; absorbing flux equals the Godunov flux against a
zero ghost state.  The anelastic rows of the Jacobians and the coupling E are
pinned by the viscoelastic dispersion relation: the complex wavenumbers of
plane waves of q_t + A_n q_x = E q give, on the P and both S branches, the
fitted constant-Q law of a generalised Maxwell body (1/Q = Im k^2 / Re k^2
within the fit's +-5% of Qp, Qs over the band), the unrelaxed speeds at high
frequency and the relaxed ones, M_u (1 - sum_l Y_l), at low frequency; a
halved shear weight or unsymmetrised memory rows fail it.
"""
from __future__ import annotations

import numpy as np

SYM = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]
SYM_INDEX = {}
for _q, (_i, _j) in enumerate(SYM):
    SYM_INDEX[(_i, _j)] = _q
    SYM_INDEX[(_j, _i)] = _q
VEL = 6


def n_quantities(m: int) -> int:
    return 9 + 6 * m


def lame(rho, vp, vs):
    rho, vp, vs = (np.asarray(a, dtype=np.float64) for a in (rho, vp, vs))
    mu = rho * vs * vs
    lam = rho * vp * vp - 2.0 * mu
    return lam, mu


def jacobians(rho, lam, mu, omega):
    """A[K, 3, Nq, Nq]: Jacobians in x, y, z per element."""
    K = len(rho)
    m = len(omega)
    nq = n_quantities(m)
    A = np.zeros((K, 3, nq, nq))
    for d in range(3):
        for q, (i, j) in enumerate(SYM):
            for k in range(3):
                c = lam * (i == j) * (d == k) + mu * ((i == d) * (j == k) + (j == d) * (i == k))
                A[:, d, q, VEL + k] = -c
                for l in range(m):
                    A[:, d, 9 + 6 * l + q, VEL + k] = -omega[l] * 0.5 * ((i == d) * (j == k) + (j == d) * (i == k))
        for i in range(3):
            A[:, d, VEL + i, SYM_INDEX[(i, d)]] = -1.0 / rho
    return A


def coupling(lam, mu, yp, ys, omega):
    """E[K, Nq, Nq]: anelastic source matrix (zero for m = 0)."""
    K = len(lam)
    m = len(omega)
    nq = n_quantities(m)
    E = np.zeros((K, nq, nq))
    for l in range(m):
        a = (lam + 2.0 * mu) * yp[:, l] - 2.0 * mu * ys[:, l]
        b = 2.0 * mu * ys[:, l]
        base = 9 + 6 * l
        for q in range(6):
            E[:, q, base + q] -= b
            if q < 3:
                for r in range(3):
                    E[:, q, base + r] -= a
            E[:, base + q, base + q] = -omega[l]
    return E


def normal_jacobian(A, n):
    """A_n = sum_d n_d A_d for A[F,3,nq,nq], n[F,3]."""
    return np.einsum("fd,fdij->fij", n, A)


def traction_op(n):
    """Tr[F,3,9]: traction sigma n as a linear map of the elastic state."""
    F = n.shape[0]
    T = np.zeros((F, 3, 9))
    for i in range(3):
        for j in range(3):
            T[:, i, SYM_INDEX[(i, j)]] += n[:, j]
    return T


def velocity_op(F):
    V = np.zeros((F, 3, 9))
    for i in range(3):
        V[:, i, VEL + i] = 1.0
    return V


def _sorted_eig(M):
    """Real eigen-decomposition of matrices with real spectra, sorted by speed.
    LAPACK may return a complex-conjugate pair of eigenvectors for a repeated
    real eigenvalue (round-off imaginary parts); such a pair is replaced by the
    real and imaginary parts of its first member, which span the same real
    eigenspace."""
    w, R = np.linalg.eig(M)
    Rr = R.real.copy()
    for j in range(M.shape[1] - 1):
        pair = w.imag[:, j] > 0
        if np.any(pair):
            Rr[pair, :, j] = R[pair, :, j].real
            Rr[pair, :, j + 1] = R[pair, :, j].imag
    w = w.real
    order = np.argsort(w, axis=1, kind="stable")
    w = np.take_along_axis(w, order, axis=1)
    Rr = np.take_along_axis(Rr, order[:, None, :], axis=2)
    return w, Rr


def godunov_matrices(An_m, An_p, n, kind):
    """Interface-state maps: q*- = Gm q- + Gp q+ (elastic 9 components).

    An_m, An_p: [F,9,9] elastic normal Jacobians of the element and of its
    neighbour; kind [F]: 0 interior, 1 free surface, 2 absorbing."""
    F = An_m.shape[0]
    I9 = np.broadcast_to(np.eye(9), (F, 9, 9))
    wm, Rm = _sorted_eig(An_m)
    wp, Rp = _sorted_eig(An_p)
    Rin = Rm[:, :, :3]     # three most negative speeds: waves leaving the face into (-)
    Rout = Rp[:, :, 6:]    # three most positive speeds: waves leaving into (+)
    Tr = traction_op(n)
    Vl = velocity_op(F)
    Gm = np.zeros((F, 9, 9))
    Gp = np.zeros((F, 9, 9))

    inner = kind == 0
    if np.any(inner):
        M = np.zeros((F, 6, 6))
        M[:, :3, :3] = Tr @ Rin
        M[:, :3, 3:] = -(Tr @ Rout)
        M[:, 3:, :3] = Vl @ Rin
        M[:, 3:, 3:] = -(Vl @ Rout)
        rhs = np.concatenate([Tr, Vl], axis=1)          # applied to (q+ - q-)
        sol = np.linalg.solve(M[inner], rhs[inner])     # [f,6,9]
        S_alpha = sol[:, :3, :]
        Gp[inner] = Rin[inner] @ S_alpha
        Gm[inner] = I9[inner] - Gp[inner]
    free = kind == 1
    if np.any(free):
        TR = Tr[free] @ Rin[free]
        Gm[free] = I9[free] - Rin[free] @ np.linalg.solve(TR, Tr[free])
    absorb = kind == 2
    if np.any(absorb):
        # characteristic amplitudes alpha = R^-1 q- over the full eigenvector
        # basis R of A_n^-: the rows of R^-1 are the left eigenvectors dual
        # to exactly these right ones (a separate eigendecomposition of A_n^T
        # may pair the degenerate S-wave spaces differently); the incoming
        # amplitudes (the three most negative speeds) are removed
        Ra = Rm[absorb]
        amp = np.linalg.solve(Ra, np.broadcast_to(np.eye(9), Ra.shape))   # R^-1
        proj = Ra[:, :, :3] @ amp[:, :3, :]
        Gm[absorb] = I9[absorb] - proj
    return Gm, Gp


def flux_matrices_closed(n, rho, vp, vs, rho_n, vp_n, vs_n, kind, omega):
    """The element's face flux A_n q*- as Fm q- + Fp q+ (Fm, Fp [F, nq, 9]),
    written from the impedance form of the same Godunov state instead of
    eigenvectors, so that it is analytic in the materials and can be
    differentiated by complex steps (used for the adjoint's material
    derivatives; pinned against godunov_matrices in tests/test_oracle_adjoint.py).

    Normal and tangential parts of the interface velocity v* and traction t*
    for impedances Z = rho vp (normal) and rho vs (tangential) on each side:
      v* = (Z- v- + Z+ v+ + t+ - t-) / (Z- + Z+)
      t* = (Z+ t- + Z- t+ + Z- Z+ (v+ - v-)) / (Z- + Z+).
    Free surface: outside state (-t-, v-); absorbing: outside state 0; both
    with the element's own impedances.  A_n applied to a state depends only on
    its traction and velocity:
      stress (i,j):   -(lambda delta_ij n.v* + mu (n_i v*_j + n_j v*_i))
      velocity i:     -t*_i / rho
      memory (l,i,j): -omega_l (n_i v*_j + n_j v*_i) / 2."""
    n = np.asarray(n, dtype=np.float64)
    F = n.shape[0]
    m = len(omega)
    nq = n_quantities(m)
    kind = np.asarray(kind)
    rho, vp, vs, rho_n, vp_n, vs_n = (np.asarray(a) for a in (rho, vp, vs, rho_n, vp_n, vs_n))
    inner = kind == 0
    # outside material: own for boundaries
    rho_o = np.where(inner, rho_n, rho)
    vp_o = np.where(inner, vp_n, vp)
    vs_o = np.where(inner, vs_n, vs)
    zpm, zsm = rho * vp, rho * vs
    zpp, zsp = rho_o * vp_o, rho_o * vs_o
    lam = rho * vp * vp - 2.0 * rho * vs * vs
    mu = rho * vs * vs
    Tr = traction_op(n)                                  # [F,3,9]
    Vl = velocity_op(F)
    Pn = n[:, :, None] * n[:, None, :]                   # [F,3,3]
    Pt = np.eye(3)[None] - Pn

    def mix(a, b):   # P_n a_n + P_t a_t for per-face scalars a (normal), b (tangential)
        return Pn * a[:, None, None] + Pt * b[:, None, None]

    ip, is_ = 1.0 / (zpm + zpp), 1.0 / (zsm + zsp)
    # v* = Cvv- v- + Cvt- t- + Cvv+ v+ + Cvt+ t+ ; t* likewise
    Cvvm, Cvtm = mix(zpm * ip, zsm * is_), mix(-ip, -is_)
    Cvvp, Cvtp = mix(zpp * ip, zsp * is_), mix(ip, is_)
    Cttm, Ctvm = mix(zpp * ip, zsp * is_), mix(-zpm * zpp * ip, -zsm * zsp * is_)
    Cttp, Ctvp = mix(zpm * ip, zsm * is_), mix(zpm * zpp * ip, zsm * zsp * is_)
    # outside state as a map of the inside one for the boundaries
    free = (kind == 1)[:, None, None]
    absorb = (kind == 2)[:, None, None]
    # free: t+ = -t-, v+ = v-  -> fold into the minus-side maps
    Cvvm = Cvvm + np.where(free, Cvvp, 0.0)
    Cvtm = Cvtm - np.where(free, Cvtp, 0.0)
    Cttm = Cttm - np.where(free, Cttp, 0.0)
    Ctvm = Ctvm + np.where(free, Ctvp, 0.0)
    bnd = free | absorb
    Cvvp, Cvtp = np.where(bnd, 0.0, Cvvp), np.where(bnd, 0.0, Cvtp)
    Cttp, Ctvp = np.where(bnd, 0.0, Cttp), np.where(bnd, 0.0, Ctvp)
    Vm = Cvvm @ Vl + Cvtm @ Tr                           # v* from q- [F,3,9]
    Vp = Cvvp @ Vl + Cvtp @ Tr
    Tm = Cttm @ Tr + Ctvm @ Vl                           # t* from q-
    Tp = Cttp @ Tr + Ctvp @ Vl
    # flux rows as maps of (v*, t*)
    Fv = np.zeros((F, nq, 3), dtype=np.result_type(lam, n))
    Ft = np.zeros((F, nq, 3), dtype=np.result_type(rho, n))
    SYMP = [(0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2)]
    for q, (i, j) in enumerate(SYMP):
        for k in range(3):
            c = -(lam * (i == j) * n[:, k] + mu * ((i == k) * n[:, j] + (j == k) * n[:, i]))
            Fv[:, q, k] = c
            for l in range(m):
                Fv[:, 9 + 6 * l + q, k] = -omega[l] * 0.5 * ((i == k) * n[:, j] + (j == k) * n[:, i])
    for i in range(3):
        Ft[:, VEL + i, i] = -1.0 / rho
    Fm = Fv @ Vm + Ft @ Tm
    Fp = Fv @ Vp + Ft @ Tp
    return Fm, Fp
