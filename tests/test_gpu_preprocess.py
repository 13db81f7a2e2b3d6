"""A mesh from the preprocessing pipeline through the solver: the library's
clustering of the velocity-aware mesh equals the tool's, and one LTS cycle
on it matches the oracle (FP64, O=3, two clusters)."""
import numpy as np
import pytest

import synth
from helpers import parity
from oracle.solver import Oracle
from paper_2202_10313_amd import preprocess as pp

pytestmark = pytest.mark.gpu


def test_preprocessed_mesh_runs_and_matches_the_oracle():
    from paper_2202_10313_amd import Context
    vs = pp.layered_model("0:400,100:900,300:1600")
    res = pp.run(vs, lambda p: 1.8 * vs(p), lambda p: 310.0 * (1.8 * vs(p)) ** 0.25,
                 np.array([[0.0, 1000.0], [0.0, 1000.0], [-500.0, 0.0]]), 250.0, 2.0, 2.0, 3, 3)
    mesh = res["mesh"]
    K = len(res["cluster"])
    mat = dict(rho=res["rho"], vp=res["vp"], vs=res["vs"])
    ctx = Context(3, mechanisms=0, n_clusters=3, fp64=True, cfl=0.5, lam=None)
    ctx.upload_mesh(mesh["tet_verts"], mesh["tet_xyz"], mesh["face_bc"])
    ctx.upload_materials(mat["rho"], mat["vp"], mat["vs"])
    ctx.upload_clusters(None)
    info = ctx.get_clusters()
    assert np.array_equal(info["clusters"], res["cluster"])
    assert info["lam"] == res["lam"] and info["speedup"] == pytest.approx(res["speedup"], rel=1e-13)
    print(f"preprocessed mesh: {K} tets, clusters {np.bincount(res['cluster'])[1:].tolist()}, "
          f"lambda {res['lam']}", flush=True)
    orc = Oracle(mesh, mat, 3, n_clusters=3, lam=None)
    q0 = synth.random_state(90, K, 9, orc.B)
    orc.set_initial(q0)
    ctx.set_initial(q0)
    t = orc.sync_dt
    orc.run(t)
    ctx.advance_to(t)
    e = parity(ctx.read_dofs(), orc.Q)
    print(f"preprocessed mesh, one LTS cycle FP64 O=3: {e:.3e}", flush=True)
    assert e <= 1e-11
