"""Stress tests of the LTS buffer schedule (Sec. V-B (Buffers and
Algorithm)): with NaN poisoning every B1 / B2 / B3 face-trace slot is
overwritten with NaN right after the level of its last legal read (and every
slot at the start of an advance), and the element groups of each launch run
in a shuffled order.  A schedule that reads a slot after that point, or
depends on which groups run first, then changes the results: the poisoned,
shuffled runs must reproduce the plain runs bit for bit and stay finite.  A
self-test that poisons live slots shows that a stale read does reach the DOFs
and that the finite check reports it.

Covered: the two-wave FP32 kernel (O = 5) and the one-wave FP64 kernel
(O = 3), N_c = 3 with three runs and graph-replayed cycles, N_c = 5 with all
five clusters populated, the allocation-free advance, and the replays of the
checkpointed forward inside the adjoint's reverse sweep."""
import numpy as np
import pytest

import synth
from helpers import anelastic_setup

pytestmark = pytest.mark.gpu

ADVANCES = (3, 2, 4)     # cycles per edg_advance_to call


def _context(w, order, n_clusters, fp64, n_runs, flags):
    from paper_2202_10313_amd import Context
    m = w["mesh"]
    ctx = Context(order, mechanisms=3, n_clusters=n_clusters, fp64=fp64, cfl=0.5, lam=None, n_runs=n_runs,
                  flags=flags)
    ctx.upload_mesh(m["tet_verts"], m["tet_xyz"], m["face_bc"])
    a = w["attn"]
    ctx.upload_materials(w["mat"]["rho"], w["mat"]["vp"], w["mat"]["vs"], a["omega"], a["yp"], a["ys"])
    ctx.upload_clusters(None)
    K = m["tet_verts"].shape[0]
    box = m["box"]
    for r in range(n_runs):
        ctx.set_initial(synth.random_state(80 + r, K, 27, ctx.B), run=r)
        s = synth.ricker_sources(90 + r, 1, ((box[0, 0] + 0.3 * (box[0, 1] - box[0, 0]),
                                              box[0, 0] + 0.7 * (box[0, 1] - box[0, 0])),
                                             (box[1, 0] + 0.3 * (box[1, 1] - box[1, 0]),
                                              box[1, 0] + 0.7 * (box[1, 1] - box[1, 0]))),
                                 (0.2 * -box[2, 0], 0.6 * -box[2, 0]), fc_range=(8.0, 12.0))
        s["stf_params"][:, 1] = 0.02
        ctx.set_sources(s["xyz"], s["moment"], s["stf_kind"], s["stf_params"], run=r)
    ctx.set_receivers(w["rec"], 7.3e-4, 300)
    return ctx


def _states(ctx, n_runs, static=False):
    sync = ctx.get_clusters()["sync_dt"]
    adv = ctx.advance_to_static if static else ctx.advance_to
    out, done = [], 0
    for n in ADVANCES:
        done += n
        adv(done * sync)
        out.append([(ctx.read_dofs(run=r), ctx.read_receivers(run=r)) for r in range(n_runs)])
    return out


def _assert_same(a, b, label):
    for i, (sa, sb) in enumerate(zip(a, b)):
        for r, ((qa, ra), (qb, rb)) in enumerate(zip(sa, sb)):
            assert np.all(np.isfinite(qb)) and np.all(np.isfinite(rb)), f"{label}: NaN after advance {i}, run {r}"
            assert np.array_equal(qa, qb), f"{label}: dofs differ after advance {i}, run {r}"
            assert np.array_equal(ra, rb), f"{label}: seismograms differ after advance {i}, run {r}"


def _five_cluster_workload():
    mesh = synth.layered_box(3, 3, [20.0, 40.0, 80.0, 160.0, 320.0, 640.0], 1920.0, 1920.0, jitter=0.1, seed=5)
    K = mesh["tet_verts"].shape[0]
    mat = synth.homogeneous_materials(K, rho=2500.0, vp=3000.0, vs=1730.0, qp=173.0, qs=86.5)
    rec = synth.surface_receivers(32, 4, ((200.0, 1700.0), (200.0, 1700.0)))
    return dict(mesh=mesh, mat=mat, attn=synth.attenuation_inputs(mat, 3, 0.1, 10.0), rec=rec)


@pytest.mark.parametrize("order,fp64,n_clusters,graph", [(5, False, 3, True), (3, True, 3, False),
                                                         (5, False, 5, False), (3, True, 5, True)])
def test_poisoned_shuffled_runs_are_bit_identical(order, fp64, n_clusters, graph):
    from paper_2202_10313_amd import FLAG_CHECK_FINITE, FLAG_GRAPH, FLAG_POISON, FLAG_SHUFFLE
    print(f"[debug] poison+shuffle O={order} {'FP64' if fp64 else 'FP32'} N_c={n_clusters} graph={graph}",
          flush=True)
    w = anelastic_setup("tiny", order, 3, with_source=False) if n_clusters == 3 else _five_cluster_workload()
    runs = 3 if n_clusters == 3 else 1
    g = FLAG_GRAPH if graph else 0
    ref = _states(_context(w, order, n_clusters, fp64, runs, g), runs)
    dbg = _context(w, order, n_clusters, fp64, runs, g | FLAG_POISON | FLAG_SHUFFLE | FLAG_CHECK_FINITE)
    if n_clusters == 5:
        assert len(np.unique(dbg.get_clusters()["clusters"])) == 5
    _assert_same(ref, _states(dbg, runs), f"poison+shuffle O={order} N_c={n_clusters}")


def test_poisoned_allocation_free_advance_is_bit_identical():
    from paper_2202_10313_amd import FLAG_POISON, FLAG_SHUFFLE
    print("[debug] poison+shuffle, allocation-free advance, O=5 FP32", flush=True)
    w = anelastic_setup("tiny", 5, 3, with_source=False)
    ref = _states(_context(w, 5, 3, False, 2, 0), 2)
    _assert_same(ref, _states(_context(w, 5, 3, False, 2, FLAG_POISON | FLAG_SHUFFLE), 2, static=True),
                 "poisoned static advance")


@pytest.mark.parametrize("order,fp64", [(5, False), (3, True)])
def test_poisoner_self_test_reaches_the_dofs(order, fp64):
    """Poisoning the B1 slots that the next level still reads must turn DOFs
    into NaN, and the finite check must report it as EDG_ENONFINITE."""
    from paper_2202_10313_amd import FLAG_CHECK_FINITE, FLAG_POISON_EARLY, EdgError
    print(f"[debug] poisoner self-test O={order} {'FP64' if fp64 else 'FP32'}", flush=True)
    w = anelastic_setup("tiny", order, 3, with_source=False)
    ctx = _context(w, order, 3, fp64, 1, FLAG_POISON_EARLY)
    ctx.advance_to(2 * ctx.get_clusters()["sync_dt"])
    q = ctx.read_dofs()
    bad = ~np.isfinite(q)
    print(f"[debug] self-test: {bad.any(axis=(1, 2)).sum()} of {q.shape[0]} elements hold NaN", flush=True)
    assert bad.any()
    ctx = _context(w, order, 3, fp64, 1, FLAG_POISON_EARLY | FLAG_CHECK_FINITE)
    with pytest.raises(EdgError, match="EDG_ENONFINITE: [0-9]+ non-finite DOF words.*run 0, element [0-9]+"):
        ctx.advance_to(2 * ctx.get_clusters()["sync_dt"])


def test_finite_check_passes_a_clean_run_and_reports_planted_nans():
    """The finite check on a clean advance, then after a NaN planted by the
    caller in one DOF of run 1: the error names run 1 and an element whose
    DOFs are NaN, and run 0 stays finite."""
    import re
    from paper_2202_10313_amd import FLAG_CHECK_FINITE, EdgError
    w = anelastic_setup("tiny", 3, 3, with_source=False)
    ctx = _context(w, 3, 3, False, 2, FLAG_CHECK_FINITE)
    sync = ctx.get_clusters()["sync_dt"]
    ctx.advance_to(sync)
    q = ctx.read_dofs(run=1)
    q[q.shape[0] // 2, 7, 0] = np.nan
    ctx.set_initial(q, run=1)
    with pytest.raises(EdgError, match="EDG_ENONFINITE: [0-9]+ non-finite DOF words.*run 1, element") as ei:
        ctx.advance_to(2 * sync)
    k = int(re.search(r"element ([0-9]+)", str(ei.value)).group(1))
    assert not np.all(np.isfinite(ctx.read_dofs(run=1)[k]))
    assert np.all(np.isfinite(ctx.read_dofs(run=0)))


def test_poisoned_adjoint_agrees():
    """Checkpointed forward (replayed segments and the recorded final one)
    and reverse sweep with poisoning and shuffling on: the forward bit for
    bit, the adjoint to rounding."""
    from paper_2202_10313_amd import FLAG_POISON, FLAG_SHUFFLE
    print("[debug] poison+shuffle, checkpointed forward + adjoint, O=5 FP32", flush=True)
    w = anelastic_setup("tiny", 5, 3, with_source=True)
    rng = np.random.default_rng(5)
    out = []
    for flags in (0, FLAG_POISON | FLAG_SHUFFLE):
        ctx = _context(w, 5, 3, False, 1, flags)
        ctx.set_checkpointing(2)
        ctx.advance_to(5 * ctx.get_clusters()["sync_dt"])
        if not out:
            y = rng.standard_normal((ctx.K, ctx.nq, ctx.B)) * 1e-3
            sb = rng.standard_normal(ctx.read_receivers().shape)
        res = ctx.adjoint(dj_dseis=sb, dj_dq=y)
        out.append((ctx.read_dofs(), res))
        ctx.close()
    (qa, ra), (qb, rb) = out
    assert np.all(np.isfinite(qb)) and np.array_equal(qa, qb)
    # the reverse sweep sums some adjoint words with atomics, so repeated
    # sweeps agree to rounding, not bit for bit
    for key in ("q0_b", "g_rho", "g_vp", "g_vs"):
        assert np.all(np.isfinite(rb[key])), key
        e = np.linalg.norm(ra[key] - rb[key]) / np.linalg.norm(ra[key])
        print(f"[debug] poisoned adjoint {key}: {e:.2e}", flush=True)
        assert e <= 1e-6, key
