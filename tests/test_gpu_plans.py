"""Launch plans, the autotuner and graph-captured LTS cycles change only how
the element kernel is launched: every variant must reproduce the default
eager solve bit for bit (checked after each of several advances, so that
graph replays alternate with eager launches, host synchronisation and
reads)."""
import numpy as np
import pytest

import synth
from helpers import anelastic_setup, gpu_context

pytestmark = pytest.mark.gpu

ORDER = 5
RUNS = 3
ADVANCES = (3, 2, 4)     # cycles per edg_advance_to call


def configured(w, plan=None, flags=0, order=ORDER):
    from paper_2202_10313_amd import Context
    m = w["mesh"]
    ctx = Context(order, mechanisms=3, n_clusters=3, fp64=False, cfl=0.5, lam=None, n_runs=RUNS, flags=flags)
    ctx.upload_mesh(m["tet_verts"], m["tet_xyz"], m["face_bc"])
    a = w["attn"]
    ctx.upload_materials(w["mat"]["rho"], w["mat"]["vp"], w["mat"]["vs"], a["omega"], a["yp"], a["ys"])
    ctx.upload_clusters(None)
    K = m["tet_verts"].shape[0]
    for r in range(RUNS):
        ctx.set_initial(synth.random_state(60 + r, K, 27, ctx.B), run=r)
        s = synth.ricker_sources(70 + r, 1, ((300.0, 900.0), (300.0, 900.0)), (50.0, 250.0), fc_range=(8.0, 12.0))
        s["stf_params"][:, 1] = 0.02
        ctx.set_sources(s["xyz"], s["moment"], s["stf_kind"], s["stf_params"], run=r)
    ctx.set_receivers(w["rec"], 1e-3, 300)
    if plan is not None:
        ctx.set_plan(**plan)
    return ctx


def states(ctx):
    sync = ctx.get_clusters()["sync_dt"]
    out = []
    done = 0
    for n in ADVANCES:
        done += n
        ctx.advance_to(done * sync)
        out.append([(ctx.read_dofs(run=r), ctx.read_receivers(run=r)) for r in range(RUNS)])
    return out


def assert_same(a, b, label):
    for i, (sa, sb) in enumerate(zip(a, b)):
        for r, ((qa, ra), (qb, rb)) in enumerate(zip(sa, sb)):
            assert np.array_equal(qa, qb), f"{label}: dofs differ after advance {i}, run {r}"
            assert np.array_equal(ra, rb), f"{label}: seismograms differ after advance {i}, run {r}"


def test_plans_and_graph_replays_are_bit_identical():
    from paper_2202_10313_amd import FLAG_GRAPH
    w = anelastic_setup("tiny", ORDER, 3, with_source=False)
    ref = states(configured(w))
    for plan in (dict(xcd_remap=1, run_chunk=0), dict(xcd_remap=0, run_chunk=2), dict(xcd_remap=1, run_chunk=1)):
        assert_same(ref, states(configured(w, plan)), f"plan {plan}")
        print(f"plan {plan}: identical")
    assert_same(ref, states(configured(w, flags=FLAG_GRAPH)), "graph replay")
    assert_same(ref, states(configured(w, dict(xcd_remap=1, run_chunk=2), flags=FLAG_GRAPH)),
                "graph replay with run chunks and XCD remap")
    print("graph replays: identical")


@pytest.mark.parametrize("order", [4, 5])
def test_matrix_core_traces_agree_with_the_vector_traces(order):
    """The trace_mfma plan forms the traces of faces 0 and 1 on the matrix
    cores (one dense product, other summation order): equal to the default
    path to FP32 rounding after every advance, with its graph replays."""
    from paper_2202_10313_amd import FLAG_GRAPH
    w = anelastic_setup("tiny", order, 3, with_source=False)
    ref = states(configured(w, order=order))
    for flags in (0, FLAG_GRAPH):
        got = states(configured(w, dict(xcd_remap=1, run_chunk=0, trace_mfma=1), flags=flags, order=order))
        for i, (sa, sb) in enumerate(zip(ref, got)):
            for r, ((qa, ra), (qb, rb)) in enumerate(zip(sa, sb)):
                dq = np.max(np.abs(qa - qb)) / np.max(np.abs(qa))
                dr = np.max(np.abs(ra - rb)) / max(np.max(np.abs(ra)), 1e-30)
                assert dq < 2e-5 and dr < 2e-5, f"flags {flags}, advance {i}, run {r}: rel. diff {dq:.2e} / {dr:.2e}"
        print(f"trace_mfma (flags {flags}): max rel. diff within 2e-5")


def test_autotune_keeps_the_solution():
    w = anelastic_setup("tiny", ORDER, 3, with_source=False)
    ref = configured(w)
    tuned = configured(w)
    plan, ms = tuned.autotune(cycles=1)
    print(f"autotuned plan {plan}, {ms:.3f} ms per cycle")
    assert plan["xcd_remap"] in (0, 1) and plan["run_chunk"] in (0, 16, 8, 4) and ms > 0
    assert tuned.get_plan() == plan
    t = tuned.time()
    sync = ref.get_clusters()["sync_dt"]
    ref.advance_to(t)
    tuned.advance_to(t + 2 * sync)
    ref.advance_to(t + 2 * sync)
    for r in range(RUNS):
        assert np.array_equal(ref.read_dofs(run=r), tuned.read_dofs(run=r))
        assert np.array_equal(ref.read_receivers(run=r), tuned.read_receivers(run=r))


def test_bad_plan_rejected():
    from paper_2202_10313_amd import EdgError
    w = anelastic_setup("tiny", 3, 2, with_source=False)
    ctx = gpu_context(w, 3, 2, True)
    with pytest.raises(EdgError):
        ctx.set_plan(xcd_remap=2)
    with pytest.raises(EdgError):
        ctx.set_plan(run_chunk=-1)
    with pytest.raises(EdgError):
        ctx.set_plan(trace_mfma=2)
