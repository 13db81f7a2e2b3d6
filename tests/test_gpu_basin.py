"""The graded basin workload (one GPU's share of a high-frequency run): radially
graded jittered hexes, basin velocity model, five LTS clusters, a kinematic
finite source of Hann subfaults and surface receivers.

* Small construction (8,232 tets): full parity against the oracle over one
  LTS cycle (16 finest levels), FP64 O=3 and FP32 O=5.
* Full size (7,884,216 tets, O=5, FP32): the clustering of the whole mesh
  equals the oracle's bit for bit; random data in the union of 16-hop balls
  around one element of clusters 1, 3 and 5, one cycle; the oracle on that union
  alone must reproduce the sampled elements (one cycle of 16 finest steps
  reaches 16 face hops, see tests/test_oracle_cone.py), and elements beyond
  16 hops of the data stay exactly zero.
"""
import numpy as np
import pytest

import synth
from helpers import face_adjacency, graph_ball, groups, parity, seis_parity, submesh
from oracle.solver import Oracle

pytestmark = pytest.mark.gpu

TOL = {True: 1e-11, False: 2e-5}


def element_parity(a, b):
    worst = 0.0
    for (g0, g1) in groups(a.shape[0]):
        den = np.linalg.norm(b[g0:g1]) or 1.0
        worst = max(worst, np.linalg.norm(a[g0:g1] - b[g0:g1]) / den)
    return worst


def context(mesh, mat, attn, order, fp64):
    from paper_2202_10313_amd import Context
    ctx = Context(order, mechanisms=3, n_clusters=5, fp64=fp64, cfl=0.5, lam=None)
    ctx.upload_mesh(mesh["tet_verts"], mesh["tet_xyz"], mesh["face_bc"])
    ctx.upload_materials(mat["rho"], mat["vp"], mat["vs"], attn["omega"], attn["yp"], attn["ys"])
    ctx.upload_clusters(None)
    return ctx


@pytest.mark.parametrize("order,fp64", [(3, True), (5, False)])
def test_basin_small_parity(order, fp64):
    mesh = synth.basin_box("small", seed=30)
    K = mesh["tet_verts"].shape[0]
    mat = synth.basin_materials(mesh, 31)
    attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
    ctx = context(mesh, mat, attn, order, fp64)
    info = ctx.get_clusters()
    sync = info["sync_dt"]
    # 8 x 8 subfaults on a 1 km fault; rupture times compressed into the cycle,
    # moments scaled so the injection is comparable to the random state
    src = synth.kinematic_fault(32, (150.0, -100.0, -900.0), length=1000.0, width=1000.0, n_along=8, n_down=8)
    t0 = src["stf_params"][:, 0]
    src["stf_params"] = np.stack([0.5 * sync * t0 / t0.max(), np.full(len(t0), 0.5 * sync)], axis=1)
    src["moment"] = src["moment"] * 1e-3
    rec = synth.surface_receivers(33, 16, ((-2000.0, 2000.0), (-2000.0, 2000.0)))
    # sample spacing incommensurate with the steps: no sample time sits on a
    # step boundary, where the two sides may round to different steps
    ns, dts = 60, sync / 50.37
    orc = Oracle(mesh, mat, order, attn=attn, n_clusters=5, lam=None, sources=src,
                 receivers=dict(xyz=rec, dt_sample=dts, n_samples=ns))
    assert set(np.unique(orc.cl)) == {1, 2, 3, 4, 5}
    assert np.array_equal(info["clusters"], orc.cl)
    q0 = synth.random_state(34, K, 27, orc.B)
    orc.set_initial(q0)
    ctx.set_initial(q0)
    ctx.set_sources(src["xyz"], src["moment"], src["stf_kind"], src["stf_params"])
    ctx.set_receivers(rec, dts, ns)
    orc.run(sync)
    ctx.advance_to(sync)
    e = parity(ctx.read_dofs(), orc.Q)
    seis = ctx.read_receivers()
    es = seis_parity(seis, orc.seis)
    print(f"basin small O={order} {'FP64' if fp64 else 'FP32'}: clusters {np.bincount(orc.cl)[1:].tolist()}, "
          f"dofs {e:.3e} receivers {es:.3e}")
    worst = np.unravel_index(np.argmax(np.abs(seis - orc.seis)), seis.shape)
    assert e <= TOL[fp64] and es <= TOL[fp64], f"largest receiver difference at (receiver, sample, quantity) {worst}"


@pytest.mark.timeout(1000)
def test_basin_full_size_sampled_parity():
    import torch
    from oracle import lts as olts
    from oracle import mesh as omesh
    from paper_2202_10313_amd import Context

    def say(msg):
        print(f"[basin] {msg}", flush=True)

    mesh = synth.basin_box("full", seed=30)
    K = mesh["tet_verts"].shape[0]
    assert K == 7884216
    mat = synth.basin_materials(mesh, 31)
    attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
    nbr = face_adjacency(mesh["tet_verts"])
    geo = omesh.geometry(mesh["tet_xyz"])
    dt_cfl = olts.cfl_steps(geo["inradius"], mat["vp"], 5, 0.5)
    del geo
    say("oracle clustering of the whole mesh")
    cl, lam, speedup = olts.cluster(dt_cfl, nbr, 5, None)
    dt_min = float(dt_cfl.min())
    say(f"clusters {np.bincount(cl)[1:].tolist()}, lambda {lam}")

    torch.cuda.init()
    ctx = Context(5, mechanisms=3, n_clusters=5, fp64=False, cfl=0.5, lam=None,
                  stream=torch.cuda.current_stream().cuda_stream)
    ctx.upload_mesh(mesh["tet_verts"], mesh["tet_xyz"], mesh["face_bc"])
    ctx.upload_materials(mat["rho"], mat["vp"], mat["vs"], attn["omega"], attn["yp"], attn["ys"])
    ctx.upload_clusters(None)
    info = ctx.get_clusters()
    assert np.array_equal(info["clusters"], cl)
    assert info["lam"] == lam and abs(info["dt_min"] - dt_min) <= 1e-14 * dt_min
    assert abs(info["speedup"] - speedup) <= 1e-12 * speedup
    sync = info["sync_dt"]
    say("library clustering identical")

    rng = np.random.default_rng(35)
    samples = np.array([int(rng.choice(np.nonzero(cl == l)[0])) for l in (1, 3, 5)])
    U = graph_ball(nbr, samples, 16)
    say(f"samples {samples.tolist()} (clusters 1, 3, 5), patch union {len(U)} elements")
    q0 = synth.random_state(36, len(U), 27, 35)
    ctx.set_dofs_subset(U, q0)
    rec_xyz = mesh["tet_xyz"][samples[1]].mean(axis=0)[None]
    ns, dts = 20, sync / 20.37
    ctx.set_receivers(rec_xyz, dts, ns)
    u0 = ctx.element_updates()
    ctx.advance_to(sync)
    torch.cuda.synchronize()
    counts = np.bincount(cl, minlength=6)[1:]
    assert ctx.element_updates() - u0 == sum(int(counts[l]) << (4 - l) for l in range(5))
    q1 = ctx.read_dofs_subset(samples)
    seis = ctx.read_receivers()
    # exactly zero beyond 16 hops of the data (a random sample of such elements)
    reach = np.zeros(K, dtype=bool)
    reach[graph_ball(nbr, U, 16)] = True
    far = np.nonzero(~reach)[0]
    probe = rng.choice(far, 4000, replace=False)
    assert not np.any(ctx.read_dofs_subset(probe)), "non-zero DOFs beyond the 16-hop cone of the data"
    ctx.close()
    say("GPU cycle done; running the oracle on the patch union")

    sub = submesh(mesh, U, nbr)
    orc = Oracle(sub, {k: mat[k][U] for k in ("rho", "vp", "vs")}, 5,
                 attn=dict(omega=attn["omega"], yp=attn["yp"][U], ys=attn["ys"][U]), n_clusters=5, cfl=0.5,
                 lam=lam, clusters=cl[U], dt_min=dt_min,
                 receivers=dict(xyz=rec_xyz, dt_sample=dts, n_samples=ns))
    assert abs(orc.sync_dt - sync) <= 1e-14 * sync
    orc.set_initial(q0)
    orc.run(sync)
    errs = {int(k): element_parity(q1[i], orc.Q[np.searchsorted(U, k)]) for i, k in enumerate(samples)}
    e_rec = seis_parity(seis, orc.seis)
    say(f"sampled elements {errs}, receiver {e_rec:.2e}")
    assert max(errs.values()) <= TOL[False] and e_rec <= TOL[False]
