"""Discrete adjoint of the oracle's forward map and the gradient of a
receiver misfit with respect to per-element rho, vp and vs (test
infrastructure: CPU oracle, FP64).

The paper names inversion for seismic velocities as a use of such solvers
(Sec. II (Related Work)) but gives no adjoint; this module is a reading written for the
adjoint kernels.  It is the exact transpose of the discrete scheme that
solver.Oracle computes -- time kernel, volume and surface kernels, the LTS
buffers B1/B2/B3 and their consumption rules (Sec. III-A (Discrete
Formulation), Sec. V-B (Buffers and Algorithm)) -- taken in the reverse order
of the forward schedule:

  forward (one advance between synchronisation points):
      predict(all); for each finest level: update(active); predict(active)
      (no prediction after the last level)
  adjoint: the same operations in reverse order, each replaced by its
      transpose, with the forward state before each operation restored from a
      tape (every intermediate is recomputed by the forward's own functions).

Transposes (bars are adjoints; each forward overwrite consumes and clears the
adjoint of what it overwrote):
  update   Q += V(T) + S(T, neighbour data) + source
           -> Tbar += V^T(Qbar) + S_own^T(Qbar); the neighbour-data part is
              scattered to the neighbours' buffer adjoints by the consumption
              rule (same cluster: B1bar; finer neighbour: B3bar; coarser
              neighbour: B2bar in the first half of its step, B1bar and -B2bar
              in the second);
  predict  T = sum_d c_d D_d, B1 = T^e, B2 = sum_d c'_d D_d^e, B3 (= or +=),
           D_{d+1} = L(D_d), receiver samples from D
           -> Dbar_d = c_d (Tbar + B1bar + B3bar) + c'_d B2bar + receiver
              terms; Dbar_{d-1} += L^T(Dbar_d) for d = O-1..1; Qbar += Dbar_0.
Sources do not depend on the state or the materials and drop out.

Material gradient.  The operators depend on the materials through the
Jacobians A_d (linear in lambda, mu, 1/rho), the anelastic coupling E (linear
in lambda, mu for fixed Y^P, Y^S) and the face flux maps Fm, Fp (the element's
Godunov flux A_n q*, a rational function of the materials of both sides).  The
sweep accumulates, per element and per face, the derivative of the adjoint
pairing with respect to every entry of these operators (time-summed
products of adjoints and forward intermediates); the gradient is their
contraction with the operator derivatives: exact for A and E (linear), by
complex steps for the flux maps (physics.flux_matrices_closed, analytic in
the materials).  Time steps, clusters, Y^P, Y^S and omega are held fixed.

Pins (tests/test_oracle_adjoint.py): the dot-product identity
<G x, y> = <x, G^T y> of the state map (initial DOFs -> final DOFs and
seismograms) on random vectors, and central finite differences of a misfit
along random material directions.
"""
from __future__ import annotations

import math

import numpy as np

from . import physics as _phys


class _Acc:
    def __init__(self, orc):
        K, nq = orc.K, orc.nq
        ne = orc.E.shape[1]
        self.gA = np.zeros((K, 3, nq, 9))
        self.gE = np.zeros((K, ne, ne))
        self.gFm = np.zeros((K, 4, nq, 9))
        self.gFp = np.zeros((K, 4, nq, 9))


class _Adj:
    def __init__(self, orc):
        self.Q = np.zeros_like(orc.Q)
        self.T = np.zeros_like(orc.T)
        self.B1 = np.zeros_like(orc.B1)
        self.B2 = np.zeros_like(orc.B2)
        self.B3 = np.zeros_like(orc.B3)


def _snapshot(orc):
    return (orc.Q.copy(), orc.T.copy(), orc.B1.copy(), orc.B2.copy(), orc.B3.copy(), orc.nstep.copy())


def _restore(orc, s):
    orc.Q[...], orc.T[...], orc.B1[...], orc.B2[...], orc.B3[...], orc.nstep[...] = s


def time_derivative_T(orc, idx, Yb, D, acc):
    """Transpose of Oracle.time_derivative at D (Yb: adjoint of its output);
    returns the adjoint of D and accumulates d<Yb, L(D)>/dA, d/dE."""
    e, P = len(idx), orc.Phi.shape[0]
    Dv = D @ orc.Phi.T
    Dref = (D[:, :9] @ orc.dPhi_cat.T).reshape(e, 9, 3, P)
    G = orc.geo["G"][idx]
    Dphys = (np.transpose(G, (0, 2, 1)) @ np.transpose(Dref, (0, 2, 1, 3)).reshape(e, 3, 9 * P)).reshape(e, 27, P)
    fb = Yb @ orc.wPhi.T                                             # [e,nq,P]
    gAf = -(fb @ np.transpose(Dphys, (0, 2, 1)))                     # [e,nq,(d,q)]
    acc.gA[idx] += np.transpose(gAf.reshape(e, orc.nq, 3, 9), (0, 2, 1, 3))
    Dphys_b = -(np.transpose(orc.A_flat[idx], (0, 2, 1)) @ fb)       # [e,27,P]
    Db = np.zeros_like(D)
    if orc.m > 0:
        acc.gE[idx] += fb @ np.transpose(Dv, (0, 2, 1))
        Db += (np.transpose(orc.E[idx], (0, 2, 1)) @ fb) @ orc.Phi
    else:
        acc.gE[idx] += fb @ np.transpose(Dv[:, :9], (0, 2, 1))
        Db[:, :9] += (np.transpose(orc.E[idx], (0, 2, 1)) @ fb) @ orc.Phi
    Dref_b = (G @ Dphys_b.reshape(e, 3, 9 * P)).reshape(e, 3, 9, P)
    Dref_b = np.transpose(Dref_b, (0, 2, 1, 3)).reshape(e, 9, 3 * P)
    Db[:, :9] += Dref_b @ orc.dPhi_cat
    return Db


def volume_T(orc, idx, Vb, acc):
    """Transpose of Oracle.volume (state T of the forward at this point)."""
    e, P, nq = len(idx), orc.Phi.shape[0], orc.nq
    Tv = orc.T[idx] @ orc.Phi.T                                      # [e,nq,P]
    G = orc.geo["G"][idx]
    X_b = Vb @ orc.dPhi_cat.T                                        # [e,nq,3P]
    ATref_b = np.transpose(X_b.reshape(e, nq, 3, P), (0, 2, 1, 3)) * orc.vw
    AT_b = (np.transpose(G, (0, 2, 1)) @ ATref_b.reshape(e, 3, nq * P)).reshape(e, 3, nq, P)
    acc.gA[idx] += AT_b @ np.transpose(Tv[:, None, :9, :], (0, 1, 3, 2))
    Tv_b = np.zeros_like(Tv)
    Tv_b[:, :9] += np.einsum("edrq,edrp->eqp", orc.A[idx], AT_b)
    w_b = Vb @ orc.wPhi.T
    if orc.m > 0:
        acc.gE[idx] += w_b @ np.transpose(Tv, (0, 2, 1))
        Tv_b += np.transpose(orc.E[idx], (0, 2, 1)) @ w_b
    else:
        acc.gE[idx] += w_b @ np.transpose(Tv[:, :9], (0, 2, 1))
        Tv_b[:, :9] += np.transpose(orc.E[idx], (0, 2, 1)) @ w_b
    return Tv_b @ orc.Phi


def surface_T(orc, idx, Qb, adj, acc):
    """Transpose of Oracle.surface: returns the adjoint of the element's own
    elastic time integral and scatters the neighbour-data adjoints into the
    neighbours' buffer adjoints."""
    Te = orc.T[idx, :9]
    Te_b = np.zeros_like(Te)
    for i in range(4):
        own = Te @ orc.Phi_face[i].T
        nbdata, inner = orc.neighbour_data(idx, i)
        phi_n = orc.combo_phi[np.maximum(orc.combo[idx, i], 0)]
        nbv = nbdata @ np.transpose(phi_n, (0, 2, 1))
        nbv[~inner] = 0.0
        flux_b = -orc.face_scale[idx, i][:, None, None] * (Qb @ (orc.fw[:, None] * orc.Phi_face[i]).T)
        acc.gFm[idx, i] += flux_b @ np.transpose(own, (0, 2, 1))
        acc.gFp[idx, i] += flux_b @ np.transpose(nbv, (0, 2, 1))
        Te_b += (np.transpose(orc.Fm[idx, i], (0, 2, 1)) @ flux_b) @ orc.Phi_face[i]
        nbv_b = np.transpose(orc.Fp[idx, i], (0, 2, 1)) @ flux_b
        nbv_b[~inner] = 0.0
        nb_b = nbv_b @ phi_n                                          # [e,9,B]
        e = np.nonzero(inner)[0]
        if len(e) == 0:
            continue
        k2 = orc.nbr[idx[e], i]
        rel = orc.cl[k2] - orc.cl[idx[e]]
        first = (orc.nstep[idx[e]] % 2) == 0
        same, finer = rel == 0, rel < 0
        c1, c2 = (rel > 0) & first, (rel > 0) & ~first
        np.add.at(adj.B1, k2[same], nb_b[e[same]])
        np.add.at(adj.B3, k2[finer], nb_b[e[finer]])
        np.add.at(adj.B2, k2[c1], nb_b[e[c1]])
        np.add.at(adj.B1, k2[c2], nb_b[e[c2]])
        np.add.at(adj.B2, k2[c2], -nb_b[e[c2]])
    return Te_b


def update_T(orc, idx, adj, acc):
    Qb = adj.Q[idx]
    adj.T[idx] += volume_T(orc, idx, Qb, acc)
    adj.T[idx, :9] += surface_T(orc, idx, Qb, adj, acc)


def predict_T(orc, idx, adj, acc, seis_b):
    D = orc.derivatives(idx)
    dt = orc.dt_elem[idx]
    Tb = adj.T[idx].copy()
    Tb[:, :9] += adj.B1[idx] + adj.B3[idx]
    T2b = adj.B2[idx].copy()
    even = (orc.nstep[idx] % 2) == 0
    adj.B3[idx[even]] = 0.0
    adj.T[idx] = 0.0
    adj.B1[idx] = 0.0
    adj.B2[idx] = 0.0
    Db = []
    for d in range(orc.O):
        c = dt ** (d + 1) / math.factorial(d + 1)
        c2 = (0.5 * dt) ** (d + 1) / math.factorial(d + 1)
        x = c[:, None, None] * Tb
        x[:, :9] += c2[:, None, None] * T2b
        Db.append(x)
    if seis_b is not None and orc.rec is not None:
        _receivers_T(orc, idx, Db, seis_b)
    for d in range(orc.O - 1, 0, -1):
        Db[d - 1] += time_derivative_T(orc, idx, Db[d], D[d - 1], acc)
    adj.Q[idx] += Db[0]


def _receivers_T(orc, idx, Db, seis_b):
    """Transpose of the receiver sampling of Oracle._sample_receivers."""
    r_of = {}
    for r, k in enumerate(orc.rec["elem"]):
        r_of.setdefault(int(k), []).append(r)
    dts = orc.rec["dt"]
    for pos, k in enumerate(idx):
        rs = r_of.get(int(k))
        if not rs:
            continue
        dt = orc.dt_elem[k]
        t0 = float(orc.nstep[k]) * dt
        t1 = float(orc.nstep[k] + 1) * dt
        eps = 1e-9 * dt
        s = max(0, int(math.floor((t0 - eps) / dts)) - 1)
        while s < orc.rec["ns"] and float(s) * dts < t1 - eps:
            ts = float(s) * dts
            if ts >= t0 - eps:
                for r in rs:
                    for d in range(orc.O):
                        w = (ts - t0) ** d / math.factorial(d)
                        Db[d][pos, :9] += w * np.outer(seis_b[r, s], orc.rec["phi"][r])
            s += 1


def _material_gradient(orc, acc, attn):
    """Contract the accumulated operator adjoints with the operator
    derivatives; returns d/d rho, d/d vp, d/d vs per element."""
    K, m = orc.K, orc.m
    inf = np.full(1, np.inf)
    # A is linear in (lambda, mu, 1/rho): derivative patterns by differences
    A0 = _phys.jacobians(inf, np.zeros(1), np.zeros(1), orc.omega)[0, :, :, :9]
    A_lam = _phys.jacobians(inf, np.ones(1), np.zeros(1), orc.omega)[0, :, :, :9] - A0
    A_mu = _phys.jacobians(inf, np.zeros(1), np.ones(1), orc.omega)[0, :, :, :9] - A0
    A_ri = _phys.jacobians(np.ones(1), np.zeros(1), np.zeros(1), orc.omega)[0, :, :, :9] - A0
    g_lam = np.einsum("kdrq,drq->k", acc.gA, A_lam)
    g_mu = np.einsum("kdrq,drq->k", acc.gA, A_mu)
    g_ri = np.einsum("kdrq,drq->k", acc.gA, A_ri)
    if m > 0:
        yp, ys = np.asarray(attn["yp"], dtype=np.float64), np.asarray(attn["ys"], dtype=np.float64)
        z, o = np.zeros(K), np.ones(K)
        E0 = _phys.coupling(z, z, yp, ys, orc.omega)
        E_lam = _phys.coupling(o, z, yp, ys, orc.omega) - E0
        E_mu = _phys.coupling(z, o, yp, ys, orc.omega) - E0
        g_lam += np.einsum("krq,krq->k", acc.gE, E_lam)
        g_mu += np.einsum("krq,krq->k", acc.gE, E_mu)
    rho, vp, vs = orc.rho, orc.vp, orc.vs
    g_rho = g_lam * (vp * vp - 2.0 * vs * vs) + g_mu * vs * vs - g_ri / (rho * rho)
    g_vp = g_lam * 2.0 * rho * vp
    g_vs = -g_lam * 4.0 * rho * vs + g_mu * 2.0 * rho * vs
    grads = [g_rho, g_vp, g_vs]
    # face flux maps: complex-step derivatives in the six materials of a face
    h = 1e-20
    for i in range(4):
        nb = orc.nbr[:, i]
        inner = nb >= 0
        other = np.where(inner, nb, np.arange(K))
        kind = np.where(inner, 0, orc.face_bc[:, i])
        if np.any(kind == 3):
            raise ValueError("the adjoint does not support the analytic-ghost test boundary")
        n = orc.geo["normals"][:, i]
        base = [rho, vp, vs, rho[other], vp[other], vs[other]]
        for p in range(6):
            args = [a.astype(np.complex128) for a in base]
            step = h * np.abs(base[p])
            args[p] = args[p] + 1j * step
            Fm, Fp = _phys.flux_matrices_closed(n, *args, kind, orc.omega)
            dFm = Fm.imag / step[:, None, None]
            dFp = Fp.imag / step[:, None, None]
            c = np.einsum("krq,krq->k", acc.gFm[:, i], dFm) + np.einsum("krq,krq->k", acc.gFp[:, i], dFp)
            if p < 3:
                grads[p] += c
            else:
                np.add.at(grads[p - 3], nb[inner], c[inner])
    return grads


def adjoint(orc, t_end, seis_b=None, q_b=None, attn=None):
    """Advance the oracle from its current synchronisation point to t_end
    (as Oracle.run) recording a tape, then sweep backwards.

    seis_b [n_rec, n_samples, 9]: adjoint of the seismogram samples recorded
    in the window; q_b [K, nq, B]: adjoint of the final DOFs (None = 0);
    attn: the anelastic inputs (omega, yp, ys) the oracle was built with
    (needed for the coupling derivatives when m > 0).
    Returns dict(q0_b, g_rho, g_vp, g_vs): the adjoint of the initial DOFs
    and the material gradient."""
    levels_per_cycle = 2 ** (orc.n_clusters - 1)
    t_now = orc.level * orc.dt_cluster[0]
    cycles = (t_end - t_now) / orc.sync_dt
    nc = int(round(cycles))
    if nc < 0 or abs(cycles - nc) > 1e-9 * max(1.0, abs(cycles)):
        raise ValueError("t_end is not a sync point")
    if orc.m > 0 and attn is None:
        raise ValueError("attn is required for anelastic materials")
    J = nc * levels_per_cycle
    tape = []
    allidx = np.arange(orc.K)
    period = 2 ** (orc.cl - 1)
    if J > 0:
        tape.append(("P", allidx, _snapshot(orc)))
        orc.predict(allidx)
        for j in range(1, J + 1):
            g = orc.level + j
            act = np.nonzero(g % period == 0)[0]
            tape.append(("U", act, _snapshot(orc)))
            orc.update(act)
            if j < J:
                tape.append(("P", act, _snapshot(orc)))
                orc.predict(act)
        orc.level += J
    final = _snapshot(orc)

    adj = _Adj(orc)
    acc = _Acc(orc)
    if q_b is not None:
        adj.Q[...] = q_b
    for op, idx, snap in reversed(tape):
        _restore(orc, snap)
        if op == "U":
            update_T(orc, idx, adj, acc)
        else:
            predict_T(orc, idx, adj, acc, seis_b)
    _restore(orc, final)
    g_rho, g_vp, g_vs = _material_gradient(orc, acc, attn)
    return dict(q0_b=adj.Q.copy(), g_rho=g_rho, g_vp=g_vp, g_vs=g_vs)
