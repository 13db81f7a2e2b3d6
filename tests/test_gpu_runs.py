"""Batched runs: n independent runs (own initial state, own moment-tensor
source) share one mesh and advance in one launch per LTS level.  Every run
must equal, bit for bit, the single-run solve of the same inputs (the kernels
compute each (element, run) pair the same way), and one of them is checked
against the oracle as well."""
import numpy as np
import pytest

import synth
from helpers import anelastic_setup, gpu_context, parity, seis_parity
from oracle.solver import Oracle

pytestmark = pytest.mark.gpu

TOL = {True: 1e-11, False: 2e-5}


def run_inputs(w, order, n_runs, seed):
    """Per-run initial state and Ricker source (own location, moment tensor
    and centre frequency)."""
    box = w["mesh"]["box"]
    xy = ((box[0, 0] + 0.2 * (box[0, 1] - box[0, 0]), box[0, 0] + 0.8 * (box[0, 1] - box[0, 0])),
          (box[1, 0] + 0.2 * (box[1, 1] - box[1, 0]), box[1, 0] + 0.8 * (box[1, 1] - box[1, 0])))
    K = w["mesh"]["tet_verts"].shape[0]
    B = order * (order + 1) * (order + 2) // 6
    out = []
    for r in range(n_runs):
        src = synth.ricker_sources(seed + 10 * r, 1, xy, (0.2 * -box[2, 0], 0.6 * -box[2, 0]), fc_range=(6.0, 12.0))
        src["stf_params"][:, 1] = 0.02          # pulse centred early in the window
        out.append(dict(q0=synth.random_state(seed + 10 * r + 1, K, 27, B), src=src))
    return out


@pytest.mark.parametrize("order,fp64", [(3, True), (4, False), (5, False)])
def test_batched_runs_equal_single_runs(order, fp64):
    w = anelastic_setup("tiny", order, 3, with_source=False)
    n_runs = 3
    inputs = run_inputs(w, order, n_runs, 40)
    rec_dt, ns = 1e-3, 120
    batch = gpu_context(w, order, 3, fp64, n_runs=n_runs)
    for r, inp in enumerate(inputs):
        batch.set_initial(inp["q0"], run=r)
        s = inp["src"]
        batch.set_sources(s["xyz"], s["moment"], s["stf_kind"], s["stf_params"], run=r)
    batch.set_receivers(w["rec"], rec_dt, ns)
    t = 2 * batch.get_clusters()["sync_dt"]
    batch.advance_to(t)
    K = w["mesh"]["tet_verts"].shape[0]
    u_batch = batch.element_updates()
    for r, inp in enumerate(inputs):
        single = gpu_context(w, order, 3, fp64)
        single.set_initial(inp["q0"])
        s = inp["src"]
        single.set_sources(s["xyz"], s["moment"], s["stf_kind"], s["stf_params"])
        single.set_receivers(w["rec"], rec_dt, ns)
        single.advance_to(t)
        qb, qs = batch.read_dofs(run=r), single.read_dofs()
        sb, ss = batch.read_receivers(run=r), single.read_receivers()
        print(f"O={order} fp64={fp64} run {r}: max |dq| {np.max(np.abs(qb - qs)):.3e}, max |dseis| {np.max(np.abs(sb - ss)):.3e}")
        assert np.array_equal(qb, qs)
        assert np.array_equal(sb, ss)
        assert u_batch == n_runs * single.element_updates()
        single.close()
    # the last run against the oracle
    inp = inputs[-1]
    orc = Oracle(w["mesh"], w["mat"], order, attn=w["attn"], n_clusters=3, lam=None, sources=inp["src"],
                 receivers=dict(xyz=w["rec"], dt_sample=rec_dt, n_samples=ns))
    orc.set_initial(inp["q0"])
    orc.run(t)
    e = parity(batch.read_dofs(run=n_runs - 1), orc.Q)
    es = seis_parity(batch.read_receivers(run=n_runs - 1), orc.seis)
    print(f"O={order} fp64={fp64} batched run vs oracle: dofs {e:.3e} receivers {es:.3e}")
    assert e <= TOL[fp64] and es <= TOL[fp64]
    assert K > 0


def test_run_index_checked():
    from paper_2202_10313_amd import EdgError
    w = anelastic_setup("tiny", 3, 2, with_source=False)
    ctx = gpu_context(w, 3, 2, True, n_runs=2)
    B = 10
    K = w["mesh"]["tet_verts"].shape[0]
    with pytest.raises(EdgError):
        ctx.set_initial(np.zeros((K, 27, B)), run=2)
    with pytest.raises(EdgError):
        ctx.read_dofs(run=-1)
    with pytest.raises(EdgError):
        ctx.read_receivers(run=2)


@pytest.mark.parametrize("n_runs,chunk", [(16, 0), (32, 0), (32, 8)])
def test_many_runs_equal_single_runs(n_runs, chunk):
    """The fused batch at the widths of the batched workload (16 and 32 runs;
    32 also as 4 launches of 8 runs): every run equals its single-run solve
    bit for bit (O=4, FP32, 3 clusters, own initial state and source each)."""
    order = 4
    w = anelastic_setup("tiny", order, 3, with_source=False)
    inputs = run_inputs(w, order, n_runs, 70)
    rec_dt, ns = 1e-3, 60
    batch = gpu_context(w, order, 3, False, n_runs=n_runs)
    batch.set_plan(xcd_remap=1, run_chunk=chunk)
    for r, inp in enumerate(inputs):
        batch.set_initial(inp["q0"], run=r)
        s = inp["src"]
        batch.set_sources(s["xyz"], s["moment"], s["stf_kind"], s["stf_params"], run=r)
    batch.set_receivers(w["rec"], rec_dt, ns)
    t = 2 * batch.get_clusters()["sync_dt"]
    batch.advance_to(t)
    single = gpu_context(w, order, 3, False)
    single.set_receivers(w["rec"], rec_dt, ns)
    for r, inp in enumerate(inputs):
        single.rewind()
        single.set_initial(inp["q0"])
        s = inp["src"]
        single.set_sources(s["xyz"], s["moment"], s["stf_kind"], s["stf_params"])
        single.advance_to(t)
        assert np.array_equal(batch.read_dofs(run=r), single.read_dofs()), r
        assert np.array_equal(batch.read_receivers(run=r), single.read_receivers()), r
    print(f"{n_runs} runs (chunk {chunk}): every run bit-identical to its single-run solve", flush=True)
    batch.close()
    single.close()
