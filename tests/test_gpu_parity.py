"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle on the
same seeded inputs.  FP64 runs must agree to relative L2 <= 1e-11, FP32 runs
to <= 2e-5 (each FP32 result's error is printed)."""
import math

import numpy as np
import pytest

import synth
from oracle.solver import Oracle, plane_wave_p, project
from tests.helpers import anelastic_setup, gpu_context, parity, random_direction_wavevector, seis_parity

pytestmark = pytest.mark.gpu

TOL64 = 1e-11
TOL32 = 2e-5


def _c1(direction, kn, steps=50):
    mesh = synth.kuhn_cube_periodic(6, 1000.0)
    K = mesh["tet_verts"].shape[0]
    mat = synth.homogeneous_materials(K)
    w = dict(mesh=mesh, mat=mat)
    orc = Oracle(mesh, mat, 3, cfl=0.5)
    q = plane_wave_p(direction, kn, 2700.0, 6000.0, 3464.0)
    q0 = project(mesh["tet_xyz"], 3, lambda x: q(x, 0.0))
    orc.set_initial(q0)
    ctx = gpu_context(w, 3, 1, True, lam=1.0, mechanisms=0)
    ctx.set_initial(q0)
    t = steps * orc.sync_dt
    info = ctx.get_clusters()
    assert info["sync_dt"] == pytest.approx(orc.sync_dt, rel=1e-14)
    orc.run(t)
    ctx.advance_to(t)
    return ctx.read_dofs(), orc.Q, project(mesh["tet_xyz"], 3, lambda x: q(x, t))


def test_c1_plane_wave_axis_fp64():
    gpu, ref, exact = _c1([1.0, 0.0, 0.0], 2 * math.pi / 500.0)
    e = parity(gpu, ref)
    print(f"C1 axis FP64 parity {e:.3e}")
    assert e <= TOL64
    assert parity(gpu, exact) < 0.03


def test_c1_plane_wave_seeded_direction_fp64():
    n, kn = random_direction_wavevector(1)
    gpu, ref, exact = _c1(n, kn)
    e = parity(gpu, ref)
    print(f"C1 seeded-direction FP64 parity {e:.3e}, wavelength {2 * math.pi / kn:.1f} m")
    assert e <= TOL64


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_anelastic_lts_fp64(order):
    w = anelastic_setup("tiny", order, 3)
    orc = Oracle(w["mesh"], w["mat"], order, attn=w["attn"], n_clusters=3, lam=None, sources=w["src"],
                 receivers=dict(xyz=w["rec"], dt_sample=1e-3, n_samples=200))
    ctx = gpu_context(w, order, 3, True)
    info = ctx.get_clusters()
    assert np.array_equal(info["clusters"], orc.cl)
    assert info["lam"] == orc.lam_lts and info["sync_dt"] == pytest.approx(orc.sync_dt, rel=1e-15)
    assert len(np.unique(orc.cl)) >= 2
    q0 = synth.random_state(5, orc.K, 27, orc.B)
    orc.set_initial(q0)
    ctx.set_initial(q0)
    ctx.set_sources(w["src"]["xyz"], w["src"]["moment"], w["src"]["stf_kind"], w["src"]["stf_params"])
    ctx.set_receivers(w["rec"], 1e-3, 200)
    t = 2 * orc.sync_dt
    orc.run(t)
    ctx.advance_to(t)
    e = parity(ctx.read_dofs(), orc.Q)
    es = seis_parity(ctx.read_receivers(), orc.seis)
    print(f"anelastic LTS FP64 O={order}: dofs {e:.3e} receivers {es:.3e}")
    assert e <= TOL64 and es <= TOL64


@pytest.mark.parametrize("order", [3, 4, 5])
def test_anelastic_lts_fp32(order):
    w = anelastic_setup("tiny", order, 3)
    orc = Oracle(w["mesh"], w["mat"], order, attn=w["attn"], n_clusters=3, lam=None, sources=w["src"],
                 receivers=dict(xyz=w["rec"], dt_sample=1e-3, n_samples=200))
    ctx = gpu_context(w, order, 3, False)
    q0 = synth.random_state(6, orc.K, 27, orc.B)
    orc.set_initial(q0)
    ctx.set_initial(q0)
    ctx.set_sources(w["src"]["xyz"], w["src"]["moment"], w["src"]["stf_kind"], w["src"]["stf_params"])
    ctx.set_receivers(w["rec"], 1e-3, 200)
    t = 2 * orc.sync_dt
    orc.run(t)
    ctx.advance_to(t)
    e = parity(ctx.read_dofs(), orc.Q)
    es = seis_parity(ctx.read_receivers(), orc.seis)
    print(f"anelastic LTS FP32 O={order}: dofs {e:.3e} receivers {es:.3e}")
    assert e <= TOL32 and es <= TOL32


@pytest.mark.parametrize("order,fp64", [(4, True), (5, False)])
def test_elastic_lts_heterogeneous(order, fp64):
    """Elastic heterogeneous periodic mesh with 3 clusters (interior faces only,
    heterogeneous Godunov fluxes), several ragged groups."""
    mesh = synth.kuhn_cube_periodic(3, 1000.0, jitter=0.15, seed=3)
    K = mesh["tet_verts"].shape[0]
    mat = synth.random_materials(K, 7)
    w = dict(mesh=mesh, mat=mat)
    orc = Oracle(mesh, mat, order, n_clusters=3, lam=None)
    ctx = gpu_context(w, order, 3, fp64, mechanisms=0)
    assert np.array_equal(ctx.get_clusters()["clusters"], orc.cl)
    q0 = synth.random_state(8, K, 9, orc.B)
    orc.set_initial(q0)
    ctx.set_initial(q0)
    t = 3 * orc.sync_dt
    orc.run(t)
    ctx.advance_to(t)
    e = parity(ctx.read_dofs(), orc.Q)
    print(f"elastic heterogeneous LTS O={order} {'FP64' if fp64 else 'FP32'}: {e:.3e}")
    assert e <= (TOL64 if fp64 else TOL32)


@pytest.mark.parametrize("ncube", [1, 2])
def test_tiny_meshes_edge_cases(ncube):
    """K = 6 (a single Kuhn cube, one partly filled group) and K = 48, all
    boundary faces absorbing or free."""
    mesh = synth.layered_box(ncube, ncube, [100.0] * ncube, 100.0 * ncube, 100.0 * ncube)
    K = mesh["tet_verts"].shape[0]
    mat = synth.random_materials(K, 2)
    w = dict(mesh=mesh, mat=mat, attn=synth.attenuation_inputs(mat, 3, 0.1, 10.0))
    orc = Oracle(mesh, mat, 3, attn=w["attn"], n_clusters=2, lam=None)
    ctx = gpu_context(w, 3, 2, True)
    q0 = synth.random_state(4, K, 27, orc.B)
    orc.set_initial(q0)
    ctx.set_initial(q0)
    t = 2 * orc.sync_dt
    orc.run(t)
    ctx.advance_to(t)
    assert parity(ctx.read_dofs(), orc.Q) <= TOL64


def test_split_advance_is_bitwise_identical():
    w = anelastic_setup("tiny", 3, 3)
    q0 = synth.random_state(9, w["mesh"]["tet_verts"].shape[0], 27, 10)
    out = []
    for split in (False, True):
        ctx = gpu_context(w, 3, 3, False)
        ctx.set_initial(q0)
        ctx.set_sources(w["src"]["xyz"], w["src"]["moment"], w["src"]["stf_kind"], w["src"]["stf_params"])
        s = ctx.get_clusters()["sync_dt"]
        if split:
            ctx.advance_to(s)
            ctx.advance_to(2 * s)
            ctx.advance_to(3 * s)
        else:
            ctx.advance_to(3 * s)
        out.append(ctx.read_dofs())
    assert np.array_equal(out[0], out[1])


def test_error_codes():
    from paper_2202_10313_amd import Context, EdgError
    w = anelastic_setup("tiny", 3, 3)
    ctx = Context(3, mechanisms=3, n_clusters=3)
    with pytest.raises(EdgError) as ei:
        ctx.advance_to(1.0)
    assert ei.value.code == -2
    m = w["mesh"]
    bad = m["face_bc"].copy()
    bad[bad != 0] = 0
    with pytest.raises(EdgError) as ei:
        ctx.upload_mesh(m["tet_verts"], m["tet_xyz"], bad)
    assert ei.value.code == -6
    ctx = gpu_context(w, 3, 3, False)
    s = ctx.get_clusters()["sync_dt"]
    with pytest.raises(EdgError) as ei:
        ctx.advance_to(0.5 * s)
    assert ei.value.code == -5
    ctx.advance_to(s)
    with pytest.raises(EdgError):
        ctx.set_sources(np.array([[1e9, 0, 0]]), np.ones((1, 6)), 0, np.array([[2.0, 0.75]]))


@pytest.mark.parametrize("order,fp64", [(3, True), (5, False)])
def test_five_clusters(order, fp64):
    """The maximum N_c = 5: a column of layers 20, 40, ..., 640 m thick fills
    all five clusters (54 / 59 / 81 / 86 / 44 elements); one cycle is 16
    finest levels.  Anelastic, with a source and receivers."""
    mesh = synth.layered_box(3, 3, [20.0, 40.0, 80.0, 160.0, 320.0, 640.0], 1920.0, 1920.0, jitter=0.1, seed=5)
    K = mesh["tet_verts"].shape[0]
    mat = synth.homogeneous_materials(K, rho=2500.0, vp=3000.0, vs=1730.0, qp=173.0, qs=86.5)
    attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
    w = dict(mesh=mesh, mat=mat, attn=attn)
    src = synth.ricker_sources(31, 1, ((600.0, 1300.0), (600.0, 1300.0)), (30.0, 600.0), fc_range=(10.0, 10.0))
    src["stf_params"][:, 1] = 0.01
    rec = synth.surface_receivers(32, 4, ((200.0, 1700.0), (200.0, 1700.0)))
    orc = Oracle(mesh, mat, order, attn=attn, n_clusters=5, lam=None, sources=src,
                 receivers=dict(xyz=rec, dt_sample=2e-4, n_samples=400))
    assert set(np.unique(orc.cl)) == {1, 2, 3, 4, 5}
    ctx = gpu_context(w, order, 5, fp64)
    assert np.array_equal(ctx.get_clusters()["clusters"], orc.cl)
    q0 = synth.random_state(33, K, 27, orc.B)
    orc.set_initial(q0)
    ctx.set_initial(q0)
    ctx.set_sources(src["xyz"], src["moment"], src["stf_kind"], src["stf_params"])
    ctx.set_receivers(rec, 2e-4, 400)
    t = orc.sync_dt
    orc.run(t)
    ctx.advance_to(t)
    e = parity(ctx.read_dofs(), orc.Q)
    es = seis_parity(ctx.read_receivers(), orc.seis)
    print(f"five clusters O={order} {'FP64' if fp64 else 'FP32'}: dofs {e:.3e} receivers {es:.3e}")
    assert e <= (TOL64 if fp64 else TOL32) and es <= (TOL64 if fp64 else TOL32)


@pytest.mark.parametrize("mechanisms", [0, 3])
def test_order4_two_clusters_5k(mechanisms):
    """The oracle-sized mesh of the differentiation workload: the 2 x 2 x 1 km
    layered box (5,082 tets), O = 4, N_c = 2, FP32, elastic and anelastic."""
    w = anelastic_setup("small", 4, 2, with_source=False)
    K = w["mesh"]["tet_verts"].shape[0]
    attn = w["attn"] if mechanisms else None
    orc = Oracle(w["mesh"], w["mat"], 4, attn=attn, n_clusters=2, lam=None)
    assert set(np.unique(orc.cl)) == {1, 2}
    ctx = gpu_context(w, 4, 2, False, mechanisms=mechanisms)
    nq = 9 + 6 * mechanisms
    q0 = synth.random_state(34, K, nq, orc.B)
    orc.set_initial(q0)
    ctx.set_initial(q0)
    t = 2 * orc.sync_dt
    orc.run(t)
    ctx.advance_to(t)
    e = parity(ctx.read_dofs(), orc.Q)
    print(f"O=4 N_c=2 m={mechanisms} on {K} tets FP32: {e:.3e}")
    assert e <= TOL32


def test_receivers_on_shared_vertices_and_faces():
    """Receivers exactly on vertices and face centroids shared by several
    tets go to the lowest element index (DG fields differ between the
    elements, so a different choice would show in the seismograms)."""
    w = anelastic_setup("tiny", 3, 3, with_source=False)
    mesh = w["mesh"]
    K = mesh["tet_verts"].shape[0]
    # interior vertices (not on the box boundary) and interior face centroids
    verts = mesh["tet_xyz"].reshape(-1, 3)
    box = mesh["box"]
    inner = np.all((verts > box[:, 0] + 1.0) & (verts < box[:, 1] - 1.0), axis=1)
    pts = [verts[np.nonzero(inner)[0][i * 37]] for i in range(4)]
    nbr = __import__("helpers").face_adjacency(mesh["tet_verts"])
    for k in (30, 150, 301):   # faces whose other element has the lower index
        i = int(np.nonzero((nbr[k] >= 0) & (nbr[k] < k))[0][0])
        pts.append(mesh["tet_xyz"][k][[m for m in range(4) if m != i]].mean(axis=0))
    rec = np.array(pts)
    orc = Oracle(mesh, w["mat"], 3, attn=w["attn"], n_clusters=3, lam=None,
                 receivers=dict(xyz=rec, dt_sample=3.7e-4, n_samples=80))
    ctx = gpu_context(w, 3, 3, True)
    q0 = synth.random_state(40, K, 27, orc.B)
    orc.set_initial(q0)
    ctx.set_initial(q0)
    ctx.set_receivers(rec, 3.7e-4, 80)
    t = 2 * orc.sync_dt
    orc.run(t)
    ctx.advance_to(t)
    es = seis_parity(ctx.read_receivers(), orc.seis)
    print(f"receivers on shared vertices / faces: {es:.3e}")
    assert es <= TOL64


@pytest.mark.parametrize("order,fp64,div", [(3, True, 1), (3, True, 2), (5, False, 1)])
def test_receivers_on_step_boundaries(order, fp64, div):
    """Samples every finest step (div = 1) or half step (div = 2): every
    sample time sits on a step boundary of the finest cluster, every 2^l-th
    on one of cluster l as well.  Both sides give a boundary sample to the
    step that starts there (each step takes [t^n - eps, t^n + dt - eps),
    eps = 1e-9 dt, which absorbs the last-bit differences between their
    independently computed steps), so the seismograms agree; the sample at
    the end of the window belongs to the next, not yet predicted step and is
    zero on both."""
    w = anelastic_setup("tiny", order, 3)
    ctx = gpu_context(w, order, 3, fp64)
    info = ctx.get_clusters()
    dts = info["lam"] * info["dt_min"] / div
    t = 2 * info["sync_dt"]
    ns = int(round(t / dts)) + 1
    orc = Oracle(w["mesh"], w["mat"], order, attn=w["attn"], n_clusters=3, lam=None, sources=w["src"],
                 receivers=dict(xyz=w["rec"], dt_sample=dts, n_samples=ns))
    q0 = synth.random_state(9, orc.K, 27, orc.B)
    orc.set_initial(q0)
    ctx.set_initial(q0)
    ctx.set_sources(w["src"]["xyz"], w["src"]["moment"], w["src"]["stf_kind"], w["src"]["stf_params"])
    ctx.set_receivers(w["rec"], dts, ns)
    orc.run(t)
    ctx.advance_to(t)
    seis = ctx.read_receivers()
    es = seis_parity(seis, orc.seis)
    print(f"receivers on step boundaries O={order} {'FP64' if fp64 else 'FP32'} dt/{div}: {es:.3e}")
    assert es <= (TOL64 if fp64 else TOL32)
    assert np.all(seis[:, -1] == 0) and np.all(orc.seis[:, -1] == 0)
    assert np.all(np.any(seis[:, :-1] != 0, axis=2))
