"""The preprocessing pipeline (paper_2202_10313_amd.preprocess; Sec. VI,
Production Pipeline) on the CPU: target edge lengths from a velocity model
and a wavelength resolution, a conforming mesh that meets them, the LTS
clustering against the oracle's, and the partition / reorder / file output."""
import numpy as np
import pytest

from oracle import lts as olts
from oracle import mesh as omesh
from paper_2202_10313_amd import preprocess as pp

LAYERS = "0:400,150:900,500:2000"
BOX = np.array([[0.0, 3000.0], [0.0, 3000.0], [-1500.0, 0.0]])


def _vs():
    return pp.layered_model(LAYERS)


@pytest.fixture(scope="module")
def result():
    vs = _vs()
    return pp.run(vs, lambda p: 1.8 * vs(p), lambda p: 310.0 * (1.8 * vs(p)) ** 0.25, BOX, 500.0, 2.0, 2.0, 4, 3,
                  parts=4)


def test_target_edge_lengths():
    """h = vs / (f_max n_epw): at 2 Hz and 2 elements per wavelength a
    400 m/s layer needs 100 m and a 2000 m/s layer 500 m; the background grid
    reproduces node values and interpolates linearly between nodes."""
    vs = _vs()
    assert np.allclose(pp.target_edge_length([400.0, 900.0, 2000.0], 2.0, 2.0), [100.0, 225.0, 500.0])
    bg = pp.BackgroundGrid.from_velocity(vs, BOX, 100.0, 2.0, 2.0)
    X, Y, Z = np.meshgrid(*bg.axes, indexing="ij")
    nodes = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    np.testing.assert_allclose(bg(nodes), vs(nodes) / 4.0, rtol=1e-14)
    a = nodes[0]
    b = a + np.array([bg.axes[0][1] - bg.axes[0][0], 0.0, 0.0])
    lin = pp.BackgroundGrid([bg.axes[0], bg.axes[1], bg.axes[2]], X + 2.0 * Y - Z)
    p = np.stack([np.linspace(0, 3000, 7), np.linspace(100, 2900, 7), np.linspace(-1400, -10, 7)], axis=1)
    np.testing.assert_allclose(lin(p), p[:, 0] + 2 * p[:, 1] - p[:, 2], rtol=1e-12)
    assert bg(0.5 * (a + b)[None]) == pytest.approx(0.5 * (bg(a[None]) + bg(b[None]))[0])


def test_mesh_meets_the_size_field_and_conforms(result):
    m = result["mesh"]
    X = m["tet_xyz"]
    L = np.stack([np.linalg.norm(X[:, i] - X[:, j], axis=1) for i, j in pp.EDGES], axis=1)
    mid = np.stack([0.5 * (X[:, i] + X[:, j]) for i, j in pp.EDGES], axis=1).reshape(-1, 3)
    h = result["background"](mid).reshape(-1, 6)
    assert np.all(L <= h * (1 + 1e-12))                     # every edge meets its target
    ratio = (L / h).max(axis=1)
    assert np.median(ratio) > 0.5                           # and the mesh is not over-refined
    # the exact model's targets hold away from the layer interfaces (the
    # background grid smooths the jumps over one grid spacing)
    depth = -mid[:, 2]
    far = np.all(np.abs(depth[:, None] - np.array([150.0, 500.0])[None]) > 100.0, axis=1).reshape(-1, 6)
    hx = (_vs()(mid) / 4.0).reshape(-1, 6)
    assert np.all((L <= hx * (1 + 1e-9))[far])
    # refined where the medium is slow: the elements within 50 m of the top
    # (one background spacing above the first interface) meet 100 m
    top = X[:, :, 2].min(axis=1) >= -50.0
    assert L[top].max() <= 100.0 + 1e-9 and L[~top].max() > 300.0
    # conforming: every face is matched once or tagged (the oracle's check)
    nbr, _ = omesh.adjacency(m["tet_verts"], m["face_bc"])
    vol = omesh.geometry(X)["absdet"].sum() / 6.0
    assert vol == pytest.approx(np.prod(BOX[:, 1] - BOX[:, 0]), rel=1e-12)
    assert np.array_equal(np.sort(nbr, axis=1), np.sort(result["nbr"], axis=1))
    # shapes stay within the similarity classes of the Kuhn tetrahedra
    r = pp.insphere_radius(X)
    assert (r / L.max(axis=1)).min() > 0.1
    # free surface on top, absorbing elsewhere
    assert np.any(m["face_bc"] == 1) and np.any(m["face_bc"] == 2)


def test_clusters_equal_the_oracle(result):
    """The tool's CFL steps, clusters, lambda and speedup (library host
    routine) against the oracle's Sec. V-A clustering of the same mesh."""
    m = result["mesh"]
    geo = omesh.geometry(m["tet_xyz"])
    dt = olts.cfl_steps(geo["inradius"], result["vp"], 4, 0.5)
    np.testing.assert_allclose(pp.cfl_steps(m["tet_xyz"], result["vp"], 4), dt, rtol=1e-13)
    nbr, _ = omesh.adjacency(m["tet_verts"], m["face_bc"])
    cl, lam, sp = olts.cluster(dt, nbr, 3, None)
    assert np.array_equal(cl, result["cluster"])
    assert lam == result["lam"] and sp == pytest.approx(result["speedup"], rel=1e-13)
    assert len(np.unique(cl)) >= 2


def test_partition_reorder_and_files(result, tmp_path):
    part, cl, role, nb = result["partition"], result["cluster"], result["role"], result["nbr"]
    K = len(cl)
    # the reordered numbering is sorted by partition, cluster, role
    key = (part * 10 + cl) * 2 + role
    assert np.all(np.diff(key) >= 0)
    # roles: a face neighbour in another partition
    other = np.any((nb >= 0) & (part[np.maximum(nb, 0)] != part[:, None]), axis=1)
    assert np.array_equal(role.astype(bool), other)
    # neighbours are mutual
    k, i = np.nonzero(nb >= 0)
    assert np.all(np.any(nb[nb[k, i]] == k[:, None], axis=1))
    # weights: 2^(Nc - l) per element; balanced partitions
    assert np.array_equal(result["element_weight"], 2 ** (3 - cl))
    pw = np.bincount(part, weights=result["element_weight"])
    assert len(pw) == 4 and pw.max() / pw.min() < 1.05
    # files: plain arrays that reassemble the mesh
    summary = pp.write_partitions(result, str(tmp_path / "prep"))
    ids = []
    for mf, af in summary["files"]:
        with np.load(mf, allow_pickle=False) as a, np.load(af, allow_pickle=False) as b:
            assert np.array_equal(a["global_id"], b["global_id"])
            np.testing.assert_array_equal(a["tet_xyz"], result["mesh"]["tet_xyz"][a["global_id"]])
            np.testing.assert_array_equal(b["cluster"], cl[b["global_id"]])
            ids.append(a["global_id"])
    assert np.array_equal(np.sort(np.concatenate(ids)), np.arange(K))
    assert summary["cluster_sizes"] == np.bincount(cl, minlength=4)[1:].tolist()
