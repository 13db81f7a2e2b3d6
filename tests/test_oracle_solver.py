"""Pins of the oracle's ADER-DG update against closed-form solutions, exact
identities and invariants (no GPU)."""
import math

import numpy as np
import pytest
import scipy.linalg
from scipy.integrate import quad as sciquad

import synth
from oracle import physics as ph
from oracle.solver import Oracle, plane_wave_p, project, stf_integral


def rel_err(a, b):
    """Relative L2 error per quantity (quantities that vanish in b are
    measured against the largest quantity of the same kind)."""
    num = ((a - b) ** 2).sum(axis=(0, 2))
    den = (b ** 2).sum(axis=(0, 2))
    for g0, g1 in ((0, 6), (6, 9), (9, len(den))):
        if g1 > g0:
            top = den[g0:g1].max()
            # a kind that vanishes altogether is measured in absolute terms
            den[g0:g1] = np.maximum(den[g0:g1], 1e-20 * top) if top > 0 else 1.0
    return np.sqrt(num / den)


def test_c1_plane_wave_accuracy():
    """Periodic 6^3 Kuhn cube, O=3, 50 GTS steps at CFL 0.5 against the exact P wave."""
    mesh = synth.kuhn_cube_periodic(6, 1000.0)
    K = mesh["tet_verts"].shape[0]
    orc = Oracle(mesh, synth.homogeneous_materials(K), 3, cfl=0.5)
    assert K == 1296
    assert orc.sync_dt == pytest.approx(0.5 * 2 * 34.5178 / (5 * 6000.0), rel=1e-4)
    q = plane_wave_p([1, 0, 0], 2 * math.pi / 500.0, 2700.0, 6000.0, 3464.0)
    orc.set_initial(project(mesh["tet_xyz"], 3, lambda x: q(x, 0.0)))
    t = 50 * orc.sync_dt
    orc.run(t)
    err = rel_err(orc.Q, project(mesh["tet_xyz"], 3, lambda x: q(x, t)))
    assert err[6] < 0.03 and err[0] < 0.03


@pytest.mark.parametrize("order,n0", [(2, 3), (3, 2)])
def test_convergence_order(order, n0):
    direction = np.array([1.0, 2.0, 0.0])
    errs = []
    for n in (n0, 2 * n0):
        mesh = synth.kuhn_cube_periodic(n, 1000.0)
        K = mesh["tet_verts"].shape[0]
        orc = Oracle(mesh, synth.homogeneous_materials(K), order, cfl=0.5)
        q = plane_wave_p(direction, 2 * math.pi * math.sqrt(5) / 1000.0, 2700.0, 6000.0, 3464.0)
        orc.set_initial(project(mesh["tet_xyz"], order, lambda x: q(x, 0.0)))
        t = 0.02
        # end time on a sync point for both meshes: t is a multiple of both steps
        nsteps = int(math.ceil(t / orc.sync_dt))
        orc.sync_dt = orc.dt_cluster[-1] = orc.dt_cluster[0] = orc.dt_elem[:] = t / nsteps
        orc.run(t)
        ex = project(mesh["tet_xyz"], order, lambda x: q(x, t))
        errs.append(np.linalg.norm(orc.Q[:, 6:9] - ex[:, 6:9]) / np.linalg.norm(ex[:, 6:9]))
    rate = math.log2(errs[0] / errs[1])
    assert rate > order - 0.3, (errs, rate)


def _const_state(K, nq, B, vec):
    Q = np.zeros((K, nq, B))
    Q[:, :, 0] = vec[None, :] * math.sqrt(6.0)   # constant field = coefficient / sqrt(6)
    return Q


@pytest.mark.parametrize("order", [2, 4])
def test_ode_case_against_expm(order):
    """Spatially constant anelastic fields: one step equals the order-O Taylor
    polynomial of expm(E dt); its error to expm(E dt) falls like dt^(O+1)."""
    mesh = synth.kuhn_cube_periodic(2, 1000.0)
    K = mesh["tet_verts"].shape[0]
    mat = synth.homogeneous_materials(K, qp=20.0, qs=10.0)
    attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
    rng = np.random.default_rng(9)
    vec = rng.normal(size=27) * np.r_[np.full(6, 1e6), np.ones(3), np.full(18, 1e-2)]
    errs = []
    for scale in (1.0, 0.5):
        orc = Oracle(mesh, mat, order, attn=attn, cfl=0.5 * scale)
        orc.set_initial(_const_state(K, 27, orc.B, vec))
        dt = orc.sync_dt
        orc.run(dt)
        got = orc.Q[:, :, 0] / math.sqrt(6.0)
        assert np.abs(orc.Q[:, :, 1:]).max() < 1e-9 * np.abs(orc.Q[:, :, 0]).max()
        E = orc.E[0]
        want = scipy.linalg.expm(E * dt) @ vec
        scale = np.r_[np.full(6, np.abs(vec[:6]).max()), np.full(3, np.abs(vec[6:9]).max()),
                      np.full(18, np.abs(vec[9:]).max())]
        err = np.abs(got - want[None, :]).max(axis=0) / scale
        # rate measured on the stresses and the fastest mechanism (well above rounding)
        errs.append(max(err[:6].max(), err[21:27].max()))
        # memory rows: truncated exponential of -omega dt
        wdt = attn["omega"].max() * dt
        bound = wdt ** (order + 1) / math.factorial(order + 1) * math.exp(wdt)
        assert err[9:].max() <= bound
    assert math.log2(errs[0] / errs[1]) > order + 0.5


def test_memory_variables_decay():
    mesh = synth.kuhn_cube_periodic(2, 1000.0)
    K = mesh["tet_verts"].shape[0]
    mat = synth.homogeneous_materials(K, qp=20.0, qs=10.0)
    attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
    vec = np.zeros(27)
    vec[9:] = 1.0
    orc = Oracle(mesh, mat, 3, attn=attn)
    orc.set_initial(_const_state(K, 27, orc.B, vec))
    orc.run(5 * orc.sync_dt)
    th = orc.Q[0, 9:, 0] / math.sqrt(6.0)
    want = np.repeat(np.exp(-attn["omega"] * orc.time()), 6)
    np.testing.assert_allclose(th, want, rtol=1e-3)


def test_viscoelastic_plane_wave_closed_form():
    """Homogeneous anelastic medium, periodic cube: the exact solution is
    Im[expm((E - i |k| A_n) t) r] e^{i k.x}."""
    n = 4
    order = 4
    mesh = synth.kuhn_cube_periodic(n, 1000.0)
    K = mesh["tet_verts"].shape[0]
    mat = synth.homogeneous_materials(K, rho=2500.0, vp=4000.0, vs=2300.0, qp=12.0, qs=6.0)
    attn = synth.attenuation_inputs(mat, 3, 0.5, 50.0)
    orc = Oracle(mesh, mat, order, attn=attn)
    kdir = np.array([1.0, 0.0, 0.0])
    kn = 2 * math.pi / 1000.0
    lam, mu = ph.lame(mat["rho"][:1], mat["vp"][:1], mat["vs"][:1])
    A = ph.jacobians(mat["rho"][:1], lam, mu, attn["omega"])[0]
    An = np.einsum("d,dij->ij", kdir, A)
    E = orc.E[0]
    r = plane_wave_p(kdir, kn, 2500.0, 4000.0, 2300.0)(np.zeros((1, 3)) + [[250.0, 0, 0]], 0.0)[0]
    r = np.concatenate([r, np.zeros(18)])
    orc.set_initial(project(mesh["tet_xyz"], order, lambda x: np.sin(x @ (kn * kdir))[:, None] * r[None, :]))
    t = 30 * orc.sync_dt
    orc.run(t)
    at = scipy.linalg.expm((E - 1j * kn * An) * t) @ r.astype(complex)
    exact = project(mesh["tet_xyz"], order, lambda x: np.imag(np.exp(1j * (x @ (kn * kdir)))[:, None] * at[None, :]))
    elastic = project(mesh["tet_xyz"], order, lambda x: np.concatenate(
        [plane_wave_p(kdir, kn, 2500.0, 4000.0, 2300.0)(x, t), np.zeros((len(x), 18))], axis=1))
    e_exact = rel_err(orc.Q, exact)[6]
    e_elastic = rel_err(orc.Q, elastic)[6]
    assert e_exact < 0.01, e_exact
    assert e_elastic > 5 * e_exact      # the attenuation is really there


def _energy(orc):
    lam, mu = orc.lam[:, None], orc.mu[:, None]
    s = orc.Q[:, :6]
    v = orc.Q[:, 6:9]
    ss = (s[:, 0] ** 2 + s[:, 1] ** 2 + s[:, 2] ** 2 + 2 * (s[:, 3] ** 2 + s[:, 4] ** 2 + s[:, 5] ** 2))
    tr = s[:, 0] + s[:, 1] + s[:, 2]
    comp = ss / (2 * mu) - lam / (2 * mu * (3 * lam + 2 * mu)) * tr ** 2
    kin = orc.rho[:, None] * (v ** 2).sum(axis=1)
    return 0.5 * float(np.sum(orc.geo["absdet"][:, None] * (kin + comp)))


@pytest.mark.parametrize("order", [2, 4])
def test_energy_non_increasing_heterogeneous(order):
    mesh = synth.kuhn_cube_periodic(3, 1000.0, jitter=0.12, seed=2)
    K = mesh["tet_verts"].shape[0]
    mat = synth.random_materials(K, 5)
    orc = Oracle(mesh, mat, order, cfl=0.5)
    orc.set_initial(synth.random_state(6, K, 9, orc.B, scale_stress=1e7))
    e = [_energy(orc)]
    for s in range(8):
        orc.run(orc.time() + orc.sync_dt)
        e.append(_energy(orc))
    e = np.array(e)
    assert np.all(np.diff(e) <= 1e-13 * e[0]), np.diff(e) / e[0]
    assert e[-1] < e[0]


def test_momentum_conserved_heterogeneous_lts():
    mesh = synth.kuhn_cube_periodic(3, 1000.0, jitter=0.15, seed=3)
    K = mesh["tet_verts"].shape[0]
    mat = synth.random_materials(K, 7)
    orc = Oracle(mesh, mat, 3, n_clusters=3, lam=None)
    assert len(np.unique(orc.cl)) >= 2
    orc.set_initial(synth.random_state(8, K, 9, orc.B))
    p0 = np.sum(orc.geo["absdet"][:, None] * orc.rho[:, None] * orc.Q[:, 6:9, 0], axis=0)
    orc.run(2 * orc.sync_dt)
    p1 = np.sum(orc.geo["absdet"][:, None] * orc.rho[:, None] * orc.Q[:, 6:9, 0], axis=0)
    scale = np.sum(orc.geo["absdet"][:, None] * orc.rho[:, None] * np.abs(orc.Q[:, 6:9, 0]), axis=0)
    np.testing.assert_allclose(p1, p0, atol=1e-12 * scale.max())


def _simple_wave(order, c, r, n):
    """q(x, t) = r f(n.x - c t) with f(s) = s^(O-1) + s (a polynomial simple
    wave: exact for any f).  Returns value and exact time integral."""
    deg = max(order - 1, 1)

    def F(s):  # antiderivative of f
        return s ** (deg + 1) / (deg + 1) + s * s / 2

    def val(x, t):
        s = x @ n - c * t
        return (s ** deg + s)[:, None] * r[None, :]

    def integ(x, t0, t1):
        s0, s1 = x @ n - c * t0, x @ n - c * t1
        return ((F(s0) - F(s1)) / c)[:, None] * r[None, :]
    return val, integ


@pytest.mark.parametrize("order,nc", [(2, 1), (3, 3), (4, 3)])
def test_polynomial_exactness_lts(order, nc):
    """Polynomial simple waves are reproduced to rounding under GTS and LTS
    (buffers B1, B2, B1-B2, B3 all carry exact time integrals); receivers
    sample the exact solution."""
    mesh = synth.layered_box(3, 3, [100.0, 100.0, 300.0, 300.0], 900.0, 900.0, jitter=0.15, seed=4,
                             top_bc=3, side_bc=3)
    K = mesh["tet_verts"].shape[0]
    mat = synth.homogeneous_materials(K)
    n = np.array([0.48, 0.6, 0.64])
    n /= np.linalg.norm(n)
    sig = -(ph.lame(2700.0, 6000.0, 3464.0)[0] * np.eye(3) + 2 * ph.lame(2700.0, 6000.0, 3464.0)[1] * np.outer(n, n)) / 6000.0
    r = np.array([sig[0, 0], sig[1, 1], sig[2, 2], sig[0, 1], sig[1, 2], sig[0, 2], *n])
    L = 1000.0
    val, integ = _simple_wave(order, 6000.0 / L, r, n / L)   # s = (n.x - c t) / L
    rec = dict(xyz=np.array([[450.0, 450.0, -250.0], [100.0, 800.0, -50.0]]), dt_sample=2e-4, n_samples=40)
    orc = Oracle(mesh, mat, order, n_clusters=nc, lam=None if nc > 1 else 1.0, ghost=integ, receivers=rec)
    if nc > 1:
        assert len(np.unique(orc.cl)) >= 2
    orc.set_initial(project(mesh["tet_xyz"], order, lambda x: val(x, 0.0)))
    t = 2 * orc.sync_dt
    orc.run(t)
    exact = project(mesh["tet_xyz"], order, lambda x: val(x, t))
    scale = np.abs(exact).max(axis=(0, 2))
    err = np.abs(orc.Q - exact).max(axis=(0, 2)) / scale
    assert err.max() < 1e-11, err
    ns = int(t / rec["dt_sample"])
    for s in range(ns):
        want = val(rec["xyz"], s * rec["dt_sample"])
        np.testing.assert_allclose(orc.seis[:, s], want, rtol=1e-10, atol=1e-10 * scale.max())


def test_gts_lts_agree_within_discretisation_error():
    mesh = synth.kuhn_cube_periodic(4, 1000.0, jitter=0.15, seed=5)
    K = mesh["tet_verts"].shape[0]
    mat = synth.homogeneous_materials(K)
    order = 3
    q = plane_wave_p([1, 1, 0], 2 * math.pi * math.sqrt(2) / 1000.0, 2700.0, 6000.0, 3464.0)
    out = {}
    out[3] = Oracle(mesh, mat, order, n_clusters=3, lam=None)
    lts = out[3]
    out[1] = Oracle(mesh, mat, order, n_clusters=1, lam=lts.lam_lts)   # GTS at lam dt_min
    for orc in out.values():
        orc.set_initial(project(mesh["tet_xyz"], order, lambda x: q(x, 0.0)))
    assert len(np.unique(lts.cl)) >= 2
    t = 4 * lts.sync_dt
    steps = t / out[1].sync_dt
    assert abs(steps - round(steps)) < 1e-9
    for orc in out.values():
        orc.run(t)
    exact = project(mesh["tet_xyz"], order, lambda x: q(x, t))
    e_g = rel_err(out[1].Q, exact)[6]
    e_l = rel_err(lts.Q, exact)[6]
    d = rel_err(lts.Q, out[1].Q)[6]
    assert e_l < 2 * e_g + 1e-3 and d < 2 * max(e_g, e_l)


def test_stf_integrals_exact():
    for kind, params in ((0, (2.0, 0.75)), (1, (0.3, 0.8))):
        if kind == 0:
            a = (math.pi * params[0]) ** 2
            rate = lambda t: (1 - 2 * a * (t - params[1]) ** 2) * math.exp(-a * (t - params[1]) ** 2)
        else:
            rate = lambda t: (1 - math.cos(2 * math.pi * (t - params[0]) / params[1])) / params[1] \
                if params[0] <= t <= params[0] + params[1] else 0.0
        for (t0, t1) in ((0.0, 0.5), (0.4, 1.1), (0.9, 3.0)):
            want = sciquad(rate, t0, t1, points=[params[0], params[1]], limit=200)[0]
            assert abs(stf_integral(kind, params, t1) - stf_integral(kind, params, t0) - want) < 1e-10


def test_source_injects_exact_moment():
    """Homogeneous periodic medium: the domain integral of the stress changes only
    through the source, by -M (S(t) - S(0))."""
    mesh = synth.kuhn_cube_periodic(3, 1000.0, jitter=0.1, seed=9)
    K = mesh["tet_verts"].shape[0]
    mat = synth.homogeneous_materials(K)
    # depth range (-800, -200) puts z in [200, 800], inside the cube [0,1000]^3
    src = synth.ricker_sources(12, 2, ((200.0, 800.0), (200.0, 800.0)), (-800.0, -200.0), fc_range=(30.0, 40.0))
    orc = Oracle(mesh, mat, 3, sources=src)
    orc.set_initial(synth.random_state(3, K, 9, orc.B))
    tot = lambda: np.sum(orc.geo["absdet"][:, None] * orc.Q[:, :6, 0], axis=0) / math.sqrt(6.0)
    s0 = tot()
    t = 6 * orc.sync_dt
    orc.run(t)
    want = s0.copy()
    for s in range(2):
        p = src["stf_params"][s]
        want -= src["moment"][s] * (stf_integral(0, p, t) - stf_integral(0, p, 0.0))
    scale = np.sum(orc.geo["absdet"][:, None] * np.abs(orc.Q[:, :6, 0]), axis=0).max() / math.sqrt(6)
    np.testing.assert_allclose(tot(), want, atol=1e-12 * scale + 1e-6 * np.abs(src["moment"]).max())
