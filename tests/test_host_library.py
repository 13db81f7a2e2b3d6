"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-side precompute (reference matrices, clustering) agrees with the
oracle.  No device work."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import lts as olts
from oracle import mesh as omesh
from oracle.poly import Basis, FaceBasis
from oracle.quad import tet_rule, tri_rule
from paper_2202_10313_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "edge_lts.h")).read()
    declared = set(re.findall(r"\b(edg_[a-z_]+)\s*\(", hdr))
    assert declared == set(binding.EXPORTS)
    L = binding.lib()
    for name in declared:
        assert hasattr(L, name)


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_reference_matrices_match_oracle(order):
    K, Ft = binding.reference_matrices(order)
    b = Basis(order)
    pts, w = tet_rule(order + 1)
    Phi, dPhi = b.eval(pts), b.grad(pts)
    for c in range(3):
        want = (w[:, None] * Phi).T @ dPhi[c]          # int phi_b d_c phi_bb
        np.testing.assert_allclose(K[c], want, atol=1e-12)
    fb = FaceBasis(order)
    fp, fw = tri_rule(order + 1)
    psi = fb.eval(fp)
    bary = np.stack([1 - fp.sum(1), fp[:, 0], fp[:, 1]], axis=1)
    for i in range(4):
        verts = omesh.REF_VERTS[[m for m in range(4) if m != i]]   # ascending local order
        ph = b.eval(bary @ verts)
        np.testing.assert_allclose(Ft[i], (fw[:, None] * ph).T @ psi, atol=1e-12)


def test_clustering_matches_oracle():
    m = synth.loh_like_box("small", seed=20)
    K = m["tet_verts"].shape[0]
    mat = synth.layered_materials(m, 21)
    g = omesh.geometry(m["tet_xyz"])
    nbr, _ = omesh.adjacency(m["tet_verts"], m["face_bc"])
    dt = olts.cfl_steps(g["inradius"], mat["vp"], 5, 0.5)
    for nc, lam in ((3, None), (3, 0.8), (5, None)):
        cl_o, lam_o, sp_o = olts.cluster(dt, nbr, nc, lam)
        cl_l, lam_l, sp_l = binding.cluster_host(dt, nbr, nc, lam)
        assert lam_l == lam_o
        assert np.array_equal(cl_l, cl_o)
        assert sp_l == pytest.approx(sp_o, rel=1e-14)


def test_create_rejects_bad_config():
    with pytest.raises(binding.EdgError):
        binding.Context(order=7)
    with pytest.raises(binding.EdgError):
        binding.Context(order=3, mechanisms=2)
    # flag bits the header does not define
    with pytest.raises(binding.EdgError, match="EDG_EINVAL"):
        binding.Context(order=3, flags=32)
    with pytest.raises(binding.EdgError, match="EDG_EINVAL"):
        binding.Context(order=3, flags=binding.FLAG_POISON | 1 << 31)


def test_header_flags_and_codes_match_the_binding():
    """The debug flags and error codes the binding names are the header's."""
    import re
    text = open(os.path.join(ROOT, "include", "edge_lts.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define (EDG_\w+) (-?\d+)u?\b", text)}
    for name in ("GRAPH", "POISON", "SHUFFLE", "CHECK_FINITE", "POISON_EARLY"):
        assert defs["EDG_FLAG_" + name] == getattr(binding, "FLAG_" + name)
    for code, name in binding.ERRORS.items():
        assert defs[name] == code
