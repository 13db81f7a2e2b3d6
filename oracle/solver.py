"""ADER-DG element update with clustered rate-2 LTS (test infrastructure: CPU
oracle, FP64, quadrature form).

What is computed, in the paper's order and notation (Sec. III-A Discrete Formulation, Sec. V-B Buffers and Algorithm):

  time kernel      d^{d+1}Q = L(d^dQ): the Cauchy-Kowalevski step, written
                   here as the L2 projection of -sum_d A_d dq/dx_d + E q onto
                   the element's polynomials (exact: the field is a polynomial
                   of degree <= O-1);
                   T_k(t0, dt) = sum_{d=0}^{O-1} dt^{d+1}/(d+1)! d^dQ_k(t0)
                   (eq. ader_taylor);
  volume kernel    V_k = M^-1 [ int grad(phi) . (A T) + int phi E T ];
  surface kernel   S_k = -M^-1 sum_i int_face phi (A_n^- q*), q* the
                   Godunov state of the element's own elastic time integral
                   (local part) and the neighbour data (neighbouring part);
  update           Q^{n+1} = Q^n + V + S^L + S^N  (eq. update);
  LTS buffers      B1 = T^e(t^n, dt), B2 = T^e(t^n, dt/2),
                   B3 = B1 if n even, B3 + B1 if n odd (eq. lts_buffers);
  neighbour data   same cluster: B1 of the neighbour; finer neighbour: its B3;
                   coarser neighbour: its B2 in the first half of its step,
                   B1 - B2 in the second (Sec. V-B (Buffers and Algorithm) walk-through);
  schedule         per finest level: first all updates of the clusters whose
                   step ends there, then all predictions of the clusters whose
                   step starts there.

Not in the paper ([reading]): point sources add -M phi(x_s)/|det J| times the
exact integral of the moment rate over the step to the stress modes, at the
end of the step of the source's element; receivers sample the element's
Taylor expansion sum_d (t-t^n)^d/d! d^dQ(x_r) at the sample times inside the
element's step, during its prediction (the 9 elastic quantities); the step
[t^n, t^n+dt) takes the samples in [t^n - eps, t^n + dt - eps), eps = 1e-9 dt,
so a sample on a step boundary belongs to the step that starts there even
where two implementations round the boundary differently.

Pins: tests/test_oracle_solver.py (plane waves, convergence order, ODE case
against expm, energy decay, momentum conservation, polynomial exactness,
GTS == single-cluster LTS) and tests/test_oracle_lts.py (the buffer walk-
through of Sec. V-B (Buffers and Algorithm) traced element by element).
"""
from __future__ import annotations

import math
import numpy as np

from . import lts as _lts
from . import mesh as _mesh
from . import physics as _phys
from .poly import Basis, FaceBasis, n_basis, n_face_basis
from .quad import tet_rule, tri_rule

STF_RICKER = 0
STF_HANN = 1


def stf_integral(kind, params, t):
    """Antiderivative of the unit moment rate (exact, no quadrature)."""
    if kind == STF_RICKER:
        fc, t0 = params[0], params[1]
        a = (math.pi * fc) ** 2
        tau = t - t0
        return tau * math.exp(-a * tau * tau)
    if kind == STF_HANN:
        t0, T = params[0], params[1]
        tau = t - t0
        if tau <= 0.0:
            return 0.0
        if tau >= T:
            return 1.0
        return (tau - T / (2 * math.pi) * math.sin(2 * math.pi * tau / T)) / T
    raise ValueError(kind)


class Oracle:
    def __init__(self, mesh, mat, order, attn=None, n_clusters=1, cfl=0.5, lam=1.0,
                 clusters=None, sources=None, receivers=None, ghost=None, dt_min=None):
        self.O = order
        self.B = n_basis(order)
        self.F = n_face_basis(order)
        self.m = 0 if attn is None else len(attn["omega"])
        self.nq = _phys.n_quantities(self.m)
        # ghost(x [N,3], t0, t1) -> [N,9]: time integral of a known exact
        # solution over [t0, t1]; faces tagged 3 use it as the outside state
        # (test-only boundary for polynomial-exactness checks)
        self.ghost = ghost
        self.tet_verts = np.asarray(mesh["tet_verts"], dtype=np.int64)
        self.tet_xyz = np.asarray(mesh["tet_xyz"], dtype=np.float64)
        self.face_bc = np.asarray(mesh["face_bc"], dtype=np.int64)
        self.K = self.tet_verts.shape[0]
        self.geo = _mesh.geometry(self.tet_xyz)
        self.nbr, self.nbr_face = _mesh.adjacency(self.tet_verts, self.face_bc)

        # materials
        self.rho = np.asarray(mat["rho"], dtype=np.float64)
        self.vp = np.asarray(mat["vp"], dtype=np.float64)
        self.vs = np.asarray(mat["vs"], dtype=np.float64)
        self.lam, self.mu = _phys.lame(self.rho, self.vp, self.vs)
        self.omega = np.zeros(0) if attn is None else np.asarray(attn["omega"], dtype=np.float64)
        yp = np.zeros((self.K, 0)) if attn is None else np.asarray(attn["yp"], dtype=np.float64)
        ys = np.zeros((self.K, 0)) if attn is None else np.asarray(attn["ys"], dtype=np.float64)
        A = _phys.jacobians(self.rho, self.lam, self.mu, self.omega)
        self.A = A[:, :, :, :9].copy()           # only elastic columns are non-zero
        self.E = _phys.coupling(self.lam, self.mu, yp, ys, self.omega)
        if self.m == 0:
            self.E = self.E[:, :9, :9]

        # face flux maps: F = Fm q- + Fp q+ (elastic traces in, all rows out)
        self.Fm = np.zeros((self.K, 4, self.nq, 9))
        self.Fp = np.zeros((self.K, 4, self.nq, 9))
        for i in range(4):
            n = self.geo["normals"][:, i]
            nb = self.nbr[:, i]
            other = np.where(nb >= 0, nb, np.arange(self.K))
            An_full = _phys.normal_jacobian(A, n)                     # [K,nq,nq] own material
            An_m = An_full[:, :9, :9]
            An_p = _phys.normal_jacobian(A[other][:, :, :9, :9], n)
            kind = np.where(nb >= 0, 0, self.face_bc[:, i])
            kind = np.where(kind == 3, 0, kind)        # analytic ghost: interior solve, same material
            Gm, Gp = _phys.godunov_matrices(An_m, An_p, n, kind)
            self.Fm[:, i] = An_full[:, :, :9] @ Gm
            self.Fp[:, i] = An_full[:, :, :9] @ Gp
        self.face_scale = 2.0 * self.geo["areas"] / self.geo["absdet"][:, None]

        # quadrature tables
        self.basis = Basis(order)
        self.vpts, self.vw = tet_rule(order + 1)
        self.Phi = self.basis.eval(self.vpts)            # [P,B]
        self.dPhi = self.basis.grad(self.vpts)           # [3,P,B]
        self.dPhi_cat = self.dPhi.reshape(-1, self.B)    # [(c,p),B]
        self.wPhi = self.vw[:, None] * self.Phi          # [P,B]
        # A_flat[k, r, (d, q)] = A_d[r, q] for the fused contraction over (d, q)
        self.A_flat = np.transpose(self.A, (0, 2, 1, 3)).reshape(self.K, self.nq, 27)
        fpts, self.fw = tri_rule(order + 1)
        bary = np.stack([1.0 - fpts[:, 0] - fpts[:, 1], fpts[:, 0], fpts[:, 1]], axis=1)  # [Pf,3]
        self.face_bary = bary
        self.Phi_face = []
        for i in range(4):
            xi = bary @ _mesh.REF_VERTS[_mesh.FACE_LOCAL[i]]
            self.Phi_face.append(self.basis.eval(xi))    # [Pf,B]
        self._build_neighbour_tables()

        # time clusters
        self.dt_cfl = _lts.cfl_steps(self.geo["inradius"], self.vp, order, cfl)
        self.n_clusters = n_clusters
        if clusters is not None:
            self.cl = np.asarray(clusters, dtype=np.int64)
            self.lam_lts = float(lam)
            self.speedup = _lts.speedup(self.cl, self.lam_lts, n_clusters)
        else:
            self.cl, self.lam_lts, self.speedup = _lts.cluster(self.dt_cfl, self.nbr, n_clusters, lam)
        # dt_min may be imposed (a sub-mesh advanced with the steps of a larger mesh)
        self.dt_min = float(self.dt_cfl.min()) if dt_min is None else float(dt_min)
        self.dt_cluster = _lts.cluster_dt(self.dt_min, self.lam_lts, n_clusters)
        self.dt_elem = self.dt_cluster[self.cl - 1]
        self.sync_dt = self.dt_cluster[-1]

        # state
        self.Q = np.zeros((self.K, self.nq, self.B))
        self.T = np.zeros((self.K, self.nq, self.B))
        self.B1 = np.zeros((self.K, 9, self.B))
        self.B2 = np.zeros((self.K, 9, self.B))
        self.B3 = np.zeros((self.K, 9, self.B))
        self.nstep = np.zeros(self.K, dtype=np.int64)
        self.level = 0
        self.updates = 0

        self._setup_sources(sources)
        self._setup_receivers(receivers)

    # ------------------------------------------------------------------ setup helpers
    def _build_neighbour_tables(self):
        """Basis values of the neighbour at the element's face points, via the
        shared vertex ids (cached per distinct (face, neighbour face, vertex
        correspondence) combination)."""
        self.combo = -np.ones((self.K, 4), dtype=np.int64)
        tables = {}
        for k in range(self.K):
            for i in range(4):
                k2 = self.nbr[k, i]
                if k2 < 0:
                    continue
                own = [int(self.tet_verts[k, a]) for a in _mesh.FACE_LOCAL[i]]
                loc2 = [int(np.nonzero(self.tet_verts[k2] == v)[0][0]) for v in own]
                key = (i, tuple(loc2))
                if key not in tables:
                    xi = self.face_bary @ _mesh.REF_VERTS[loc2]
                    tables[key] = (len(tables), self.basis.eval(xi))
                self.combo[k, i] = tables[key][0]
        self.combo_phi = np.stack([v[1] for v in sorted(tables.values(), key=lambda t: t[0])]) \
            if tables else np.zeros((1, len(self.fw), self.B))

    def _setup_sources(self, src):
        self.sources = []
        if src is None:
            return
        xyz = np.asarray(src["xyz"], dtype=np.float64).reshape(-1, 3)
        elem, xi = _mesh.locate_points(self.tet_xyz, xyz)
        phi = self.basis.eval(xi)
        params = np.asarray(src["stf_params"], dtype=np.float64).reshape(len(xyz), -1)
        for s in range(len(xyz)):
            self.sources.append(dict(elem=int(elem[s]), phi=phi[s], M=np.asarray(src["moment"][s], dtype=np.float64),
                                     kind=int(src["stf_kind"]), params=params[s]))

    def _setup_receivers(self, rec):
        self.rec = None
        if rec is None:
            return
        xyz = np.asarray(rec["xyz"], dtype=np.float64).reshape(-1, 3)
        elem, xi = _mesh.locate_points(self.tet_xyz, xyz)
        self.rec = dict(elem=elem, phi=self.basis.eval(xi), dt=float(rec["dt_sample"]),
                        ns=int(rec["n_samples"]))
        self.seis = np.zeros((len(xyz), self.rec["ns"], 9))

    # ------------------------------------------------------------------ kernels
    def time_derivative(self, idx, D):
        """One Cauchy-Kowalevski step d^{d+1}Q from d^dQ for elements idx:
        the L2 projection of -sum_d A_d dq/dx_d + E q."""
        e, P = len(idx), self.Phi.shape[0]
        Dv = D @ self.Phi.T                                         # [e,nq,P]
        Dref = (D[:, :9] @ self.dPhi_cat.T).reshape(e, 9, 3, P)     # d/dxi_c at points
        GT = np.transpose(self.geo["G"][idx], (0, 2, 1))           # [e,d,c]
        Dphys = GT @ np.transpose(Dref, (0, 2, 1, 3)).reshape(e, 3, 9 * P)   # d/dx_d: [e,d,(q,p)]
        f = -(self.A_flat[idx] @ Dphys.reshape(e, 27, P))
        if self.m > 0:
            f += self.E[idx] @ Dv
        else:
            f += self.E[idx] @ Dv[:, :9]
        return f @ self.wPhi                                        # [e,nq,B]

    def derivatives(self, idx):
        D = [self.Q[idx]]
        for _ in range(self.O - 1):
            D.append(self.time_derivative(idx, D[-1]))
        return D

    def predict(self, idx):
        if len(idx) == 0:
            return
        D = self.derivatives(idx)
        dt = self.dt_elem[idx]
        T = np.zeros_like(D[0])
        T2 = np.zeros((len(idx), 9, self.B))
        for d in range(self.O):
            c = dt ** (d + 1) / math.factorial(d + 1)
            c2 = (0.5 * dt) ** (d + 1) / math.factorial(d + 1)
            T += c[:, None, None] * D[d]
            T2 += c2[:, None, None] * D[d][:, :9]
        self.T[idx] = T
        self.B1[idx] = T[:, :9]
        self.B2[idx] = T2
        even = (self.nstep[idx] % 2) == 0
        self.B3[idx[even]] = T[even, :9]
        self.B3[idx[~even]] += T[~even, :9]
        if self.rec is not None:
            self._sample_receivers(idx, D)

    def volume(self, idx):
        """int grad(phi) . (A_d T) + int phi E T, divided by the mass |det J|."""
        e, P = len(idx), self.Phi.shape[0]
        T = self.T[idx]
        Tv = T @ self.Phi.T                                          # [e,nq,P]
        AT = self.A[idx] @ Tv[:, None, :9, :]                        # [e,3(d),nq,P]
        ATref = (self.geo["G"][idx] @ AT.reshape(e, 3, self.nq * P)).reshape(e, 3, self.nq, P)  # along xi_c
        ATref = np.transpose(ATref * self.vw, (0, 2, 1, 3)).reshape(e, self.nq, 3 * P)
        vol = ATref @ self.dPhi_cat
        vol += (self.E[idx] @ Tv) @ self.wPhi
        return vol

    def neighbour_data(self, idx, i):
        """Elastic time integral the neighbour across face i provides (9 x B)."""
        nb = self.nbr[idx, i]
        inner = nb >= 0
        out = np.zeros((len(idx), 9, self.B))
        if not np.any(inner):
            return out, inner
        e = np.nonzero(inner)[0]
        k2 = nb[e]
        rel = self.cl[k2] - self.cl[idx[e]]
        same, finer, coarser = rel == 0, rel < 0, rel > 0
        out[e[same]] = self.B1[k2[same]]
        out[e[finer]] = self.B3[k2[finer]]
        first = (self.nstep[idx[e]] % 2) == 0
        c1 = coarser & first
        c2 = coarser & ~first
        out[e[c1]] = self.B2[k2[c1]]
        out[e[c2]] = self.B1[k2[c2]] - self.B2[k2[c2]]
        if np.any(np.abs(rel) > 1):
            raise RuntimeError("cluster normalisation violated")
        return out, inner

    def surface(self, idx):
        dq = np.zeros((len(idx), self.nq, self.B))
        Te = self.T[idx, :9]
        for i in range(4):
            own = Te @ self.Phi_face[i].T                              # [e,9,Pf]
            nbdata, inner = self.neighbour_data(idx, i)
            phi_n = self.combo_phi[np.maximum(self.combo[idx, i], 0)]  # [e,Pf,B]
            nbv = nbdata @ np.transpose(phi_n, (0, 2, 1))
            nbv[~inner] = 0.0
            if self.ghost is not None:
                g = np.nonzero(self.face_bc[idx, i] == 3)[0]
                if len(g):
                    k = idx[g]
                    verts = self.tet_xyz[k][:, _mesh.FACE_LOCAL[i]]                 # [g,3,3]
                    x = np.einsum("pm,gmd->gpd", self.face_bary, verts)
                    dt = self.dt_elem[k]
                    for a in range(len(g)):
                        t0 = float(self.nstep[k[a]]) * dt[a]
                        nbv[g[a]] = self.ghost(x[a], t0, t0 + dt[a]).T
            flux = self.Fm[idx, i] @ own + self.Fp[idx, i] @ nbv
            dq -= self.face_scale[idx, i][:, None, None] * (flux @ (self.fw[:, None] * self.Phi_face[i]))
        return dq

    def update(self, idx):
        if len(idx) == 0:
            return
        self.Q[idx] += self.volume(idx) + self.surface(idx)
        for s in self.sources:
            k = s["elem"]
            pos = np.nonzero(idx == k)[0]
            if len(pos) == 0:
                continue
            n = self.nstep[k]
            dt = self.dt_elem[k]
            t0, t1 = float(n) * dt, float(n + 1) * dt
            w = stf_integral(s["kind"], s["params"], t1) - stf_integral(s["kind"], s["params"], t0)
            self.Q[k, :6, :] -= (w / self.geo["absdet"][k]) * s["M"][:, None] * s["phi"][None, :]
        self.nstep[idx] += 1
        self.updates += len(idx)

    def _sample_receivers(self, idx, D):
        r_of = {}
        for r, k in enumerate(self.rec["elem"]):
            r_of.setdefault(int(k), []).append(r)
        dts = self.rec["dt"]
        for pos, k in enumerate(idx):
            rs = r_of.get(int(k))
            if not rs:
                continue
            dt = self.dt_elem[k]
            t0 = float(self.nstep[k]) * dt
            t1 = float(self.nstep[k] + 1) * dt
            # the step takes the samples in [t0 - eps, t1 - eps), eps = 1e-9 dt:
            # a sample on a step boundary belongs to the step starting there
            eps = 1e-9 * dt
            s = max(0, int(math.floor((t0 - eps) / dts)) - 1)
            while s < self.rec["ns"] and float(s) * dts < t1 - eps:
                ts = float(s) * dts
                if ts >= t0 - eps:
                    for r in rs:
                        val = np.zeros(9)
                        for d in range(self.O):
                            val += (ts - t0) ** d / math.factorial(d) * (D[d][pos, :9] @ self.rec["phi"][r])
                        self.seis[r, s] = val
                s += 1

    # ------------------------------------------------------------------ driver
    def set_initial(self, Q):
        self.Q[...] = Q

    def run(self, t_end):
        """Advance every element from the current sync point to t_end (a
        multiple of the coarsest cluster step), clusters interleaved per finest
        level as in Sec. V-B (Buffers and Algorithm)."""
        levels_per_cycle = 2 ** (self.n_clusters - 1)
        t_now = self.level * self.dt_cluster[0]
        cycles = (t_end - t_now) / self.sync_dt
        nc = int(round(cycles))
        if nc < 0 or abs(cycles - nc) > 1e-9 * max(1.0, abs(cycles)):
            raise ValueError("t_end is not a sync point")
        J = nc * levels_per_cycle
        if J == 0:
            return
        allidx = np.arange(self.K)
        self.predict(allidx)
        period = 2 ** (self.cl - 1)
        for j in range(1, J + 1):
            g = self.level + j
            act = np.nonzero(g % period == 0)[0]
            self.update(act)
            if j < J:
                self.predict(act)
        self.level += J

    def time(self):
        return self.level * self.dt_cluster[0]


def project(tet_xyz, order, fn, nq_rule=None):
    """L2 projection of fn(x [N,3]) -> [N, nq] onto every element's basis
    (orthonormal reference basis, so the coefficients are plain quadrature
    sums); used to build initial states and exact references."""
    basis = Basis(order)
    pts, w = tet_rule(nq_rule or order + 6)
    Phi = basis.eval(pts)
    X = np.asarray(tet_xyz, dtype=np.float64)
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    x = X[:, 0][:, None, :] + np.einsum("kdc,pc->kpd", J, pts)        # [K,P,3]
    vals = fn(x.reshape(-1, 3)).reshape(x.shape[0], x.shape[1], -1)   # [K,P,nq]
    return np.einsum("kpq,p,pb->kqb", vals, w, Phi)


def plane_wave_p(direction, wavenumber, rho, vp, vs):
    """Exact elastic P plane wave q(x,t) = r sin(k.x - vp |k| t), unit
    velocity amplitude along the propagation direction."""
    n = np.asarray(direction, dtype=np.float64)
    n = n / np.linalg.norm(n)
    lam = rho * (vp * vp - 2 * vs * vs)
    mu = rho * vs * vs
    sig = -(lam * np.eye(3) + 2 * mu * np.outer(n, n)) / vp
    r = np.array([sig[0, 0], sig[1, 1], sig[2, 2], sig[0, 1], sig[1, 2], sig[0, 2], n[0], n[1], n[2]])
    kvec = wavenumber * n

    def q(x, t):
        ph = x @ kvec - vp * wavenumber * t
        return np.sin(ph)[:, None] * r[None, :]
    return q
