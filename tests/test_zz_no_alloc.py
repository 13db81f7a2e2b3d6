"""The allocation-free advance, edg_advance_to_static, against edg_advance_to:
the same kernels on the same inputs with the face traces in the library's
static device array instead of the context's own buffers, so DOFs,
seismograms and update counts must agree bit for bit.  Two calls in a row on
one GPU, the second on a smaller mesh (the array keeps the first call's
contents), each made of two advances; then the errors of the entry point."""
import numpy as np
import pytest

import synth
from helpers import anelastic_setup, gpu_context
from paper_2202_10313_amd.binding import STATIC_SCRATCH_BYTES, EdgError

pytestmark = pytest.mark.gpu


def _inputs(w, order, n_runs, seed):
    box = w["mesh"]["box"]
    K = w["mesh"]["tet_verts"].shape[0]
    B = order * (order + 1) * (order + 2) // 6
    xy = ((box[0, 0] + 0.2 * (box[0, 1] - box[0, 0]), box[0, 0] + 0.8 * (box[0, 1] - box[0, 0])),
          (box[1, 0] + 0.2 * (box[1, 1] - box[1, 0]), box[1, 0] + 0.8 * (box[1, 1] - box[1, 0])))
    out = []
    for r in range(n_runs):
        src = synth.ricker_sources(seed + 10 * r, 1, xy, (0.2 * -box[2, 0], 0.6 * -box[2, 0]), fc_range=(6.0, 12.0))
        src["stf_params"][:, 1] = 0.02
        out.append(dict(q0=synth.random_state(seed + 10 * r + 1, K, 27, B), src=src))
    return out


def _compare(w, order, n_clusters, fp64, n_runs, seed):
    """Run the same inputs through edg_advance_to and edg_advance_to_static
    (two advances each: one cycle, then two more) and return both results."""
    inputs = _inputs(w, order, n_runs, seed)
    res = []
    for static in (False, True):
        ctx = gpu_context(w, order, n_clusters, fp64, n_runs=n_runs)
        for r, inp in enumerate(inputs):
            ctx.set_initial(inp["q0"], run=r)
            s = inp["src"]
            ctx.set_sources(s["xyz"], s["moment"], s["stf_kind"], s["stf_params"], run=r)
        ctx.set_receivers(w["rec"], 7.3e-4, 200)
        sync = ctx.get_clusters()["sync_dt"]
        adv = ctx.advance_to_static if static else ctx.advance_to
        adv(sync)
        adv(3 * sync)
        res.append(dict(q=[ctx.read_dofs(run=r) for r in range(n_runs)],
                        s=[ctx.read_receivers(run=r) for r in range(n_runs)],
                        u=ctx.element_updates(), t=ctx.time()))
        ctx.close()
    return res


def _assert_identical(res, what):
    a, b = res
    assert a["u"] == b["u"] and a["t"] == b["t"], what
    for r, (qa, qb) in enumerate(zip(a["q"], b["q"])):
        assert np.all(np.isfinite(qa)), what
        print(f"{what} run {r}: max |dq| {np.max(np.abs(qa - qb)):.3e}", flush=True)
        assert np.array_equal(qa, qb), (what, r)
    for r, (sa, sb) in enumerate(zip(a["s"], b["s"])):
        assert np.array_equal(sa, sb), (what, r)


def test_static_advance_equals_advance_twice_second_smaller():
    # first call: the 384-tet layered box, O=5, FP32, 3 clusters, 2 runs
    print("static advance: 384 tets, O=5, FP32, N_c=3, 2 runs", flush=True)
    big = anelastic_setup("tiny", 5, 3, with_source=False)
    _assert_identical(_compare(big, 5, 3, False, 2, 60), "K=384 O=5 FP32")
    # second call: a smaller mesh (48 tets, two layers), O=3, FP64, 2 clusters
    print("static advance: 48 tets, O=3, FP64, N_c=2, 1 run", flush=True)
    mesh = synth.layered_box(2, 2, [100.0, 200.0], 400.0, 400.0, jitter=0.1, seed=61)
    mat = synth.layered_materials(mesh, 62)
    small = dict(mesh=mesh, mat=mat, attn=synth.attenuation_inputs(mat, 3, 0.1, 10.0),
                 rec=synth.surface_receivers(63, 3, ((50.0, 350.0), (50.0, 350.0))))
    assert mesh["tet_verts"].shape[0] < 384
    _assert_identical(_compare(small, 3, 2, True, 1, 64), "K=48 O=3 FP64")


def test_static_advance_errors():
    w = anelastic_setup("tiny", 3, 2, with_source=False)
    ctx = gpu_context(w, 3, 2, True)
    sync = ctx.get_clusters()["sync_dt"]
    with pytest.raises(EdgError) as e:
        ctx.advance_to_static(0.5 * sync)          # not a synchronisation point
    assert e.value.code == -5
    ctx.set_checkpointing(1)
    with pytest.raises(EdgError) as e:
        ctx.advance_to_static(sync)                # checkpoints would allocate
    assert e.value.code == -2
    ctx.set_checkpointing(0)
    ctx.advance_to_static(sync)
    assert ctx.time() == pytest.approx(sync)
    ctx.close()
    # traces beyond the static array: the 5,082-tet box with 16 elastic runs
    # at O=5 in FP32 needs more than 256 MiB of face traces
    print("static advance: oversized context is refused", flush=True)
    w = anelastic_setup("small", 5, 2, with_source=False)
    ctx = gpu_context(w, 5, 2, False, mechanisms=0, n_runs=16)
    with pytest.raises(EdgError) as e:
        ctx.advance_to_static(ctx.get_clusters()["sync_dt"])
    assert e.value.code == -1 and str(STATIC_SCRATCH_BYTES) in str(e.value)
    assert ctx.time() == 0.0
    ctx.close()
