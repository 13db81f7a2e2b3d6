"""GPU discrete adjoint (edg_adjoint) against the oracle's discrete adjoint on
the same seeded inputs, plus properties that need no oracle: the dot-product
identity of the GPU's own forward and adjoint, independence of the checkpoint
interval, and central differences of a misfit along random material
directions.

Misfit of the tests: J = <seis, seisbar> + <Q(T), Qbar> for random seisbar,
Qbar (any differentiable misfit enters only through these two adjoints).
FP64: the adjoint of the initial DOFs to relative L2 <= 1e-11 per quantity
group, the material gradients to <= 1e-10 (norm-relative); FP32 runs state
their errors.
"""
import numpy as np
import pytest

import synth
from oracle.adjoint import adjoint as oracle_adjoint
from oracle.solver import Oracle
from tests.helpers import parity

pytestmark = pytest.mark.gpu

REC = dict(xyz=np.array([[150.0, 170.0, -20.0], [260.0, 300.0, -150.0]]), dt_sample=2e-3, n_samples=40)
SRC = dict(xyz=np.array([[200.0, 210.0, -90.0]]), moment=np.array([[1e9, -2e9, 0.5e9, 3e9, 1e9, -1e9]]),
           stf_kind=0, stf_params=np.array([[200.0, 0.004]]))
TOL64_Q, TOL64_G = 1e-11, 1e-10


def _mesh():
    mesh = synth.layered_box(2, 2, [100.0, 200.0], 400.0, 400.0, jitter=0.15, seed=3)
    K = mesh["tet_verts"].shape[0]
    return mesh, synth.random_materials(K, 4)


def _distance_clusters(nbr, n_clusters):
    dist = np.full(nbr.shape[0], -1)
    dist[0] = 0
    front = [0]
    while front:
        nxt = []
        for k in front:
            for j in nbr[k]:
                if j >= 0 and dist[j] < 0:
                    dist[j] = dist[k] + 1
                    nxt.append(j)
        front = nxt
    return np.minimum(1 + dist, n_clusters)


def _setup(order, mech, n_clusters, fp64, explicit=False):
    from paper_2202_10313_amd import Context
    mesh, mat = _mesh()
    attn = synth.attenuation_inputs(mat, mech, 0.1, 10.0) if mech else None
    cfl = 0.5 / 2 ** (n_clusters - 1) if explicit else 0.5
    ctx = Context(order, mechanisms=mech, n_clusters=n_clusters, fp64=fp64, cfl=cfl,
                  lam=1.0 if explicit else None)
    ctx.upload_mesh(mesh["tet_verts"], mesh["tet_xyz"], mesh["face_bc"])
    if mech:
        ctx.upload_materials(mat["rho"], mat["vp"], mat["vs"], attn["omega"], attn["yp"], attn["ys"])
    else:
        ctx.upload_materials(mat["rho"], mat["vp"], mat["vs"])
    cl = None
    if explicit:
        probe = Oracle(mesh, mat, 2)
        cl = _distance_clusters(probe.nbr, n_clusters)
    ctx.upload_clusters(cl)
    info = ctx.get_clusters()
    assert len(np.unique(info["clusters"])) == n_clusters
    frozen = dict(n_clusters=n_clusters, lam=info["lam"], clusters=info["clusters"], dt_min=info["dt_min"])
    return ctx, dict(mesh=mesh, mat=mat, attn=attn, order=order, frozen=frozen, sync=info["sync_dt"])


def _oracle(w, mat=None, sources=True):
    return Oracle(w["mesh"], mat or w["mat"], w["order"], attn=w["attn"], receivers=REC,
                  sources=SRC if sources else None, **w["frozen"])


def _inputs(ctx, seed):
    rng = np.random.default_rng(seed)
    x = synth.random_state(seed, ctx.K, ctx.nq, ctx.B)
    y = rng.standard_normal((ctx.K, ctx.nq, ctx.B)) * np.where(np.arange(ctx.nq) < 6, 1e-6, 1.0)[None, :, None]
    sb = rng.standard_normal((len(REC["xyz"]), REC["n_samples"], 9))
    return x, y, sb


def _run_gpu(ctx, x, y, sb, t, every, sources=True):
    if sources:
        ctx.set_sources(SRC["xyz"], SRC["moment"], SRC["stf_kind"], SRC["stf_params"])
    ctx.set_receivers(REC["xyz"], REC["dt_sample"], REC["n_samples"])
    ctx.set_checkpointing(every)
    ctx.set_initial(x)
    ctx.advance_to(t)
    qT, seis = ctx.read_dofs(), ctx.read_receivers()
    res = ctx.adjoint(dj_dseis=sb, dj_dq=y)
    return qT, seis, res


def _grad_err(res, ores):
    return max(np.linalg.norm(res[k] - ores[k]) / np.linalg.norm(ores[k]) for k in ("g_rho", "g_vp", "g_vs"))


@pytest.mark.parametrize("order,mech,n_clusters,explicit,every", [
    (3, 3, 2, False, 1), (2, 0, 3, True, 2), (4, 3, 2, False, 3), (5, 3, 2, False, 1), (4, 0, 2, False, 1)])
def test_adjoint_matches_oracle_fp64(order, mech, n_clusters, explicit, every):
    ctx, w = _setup(order, mech, n_clusters, True, explicit)
    x, y, sb = _inputs(ctx, order + mech)
    t = 3 * w["sync"]
    print(f"[adjoint] O={order} m={mech} Nc={n_clusters} every={every}", flush=True)
    qT, seis, res = _run_gpu(ctx, x, y, sb, t, every)
    orc = _oracle(w)
    orc.set_initial(x)
    ores = oracle_adjoint(orc, t, seis_b=sb, q_b=y, attn=w["attn"])
    e_fwd = parity(qT, orc.Q)
    e_q = parity(res["q0_b"], ores["q0_b"])
    e_g = _grad_err(res, ores)
    print(f"[adjoint] FP64 forward {e_fwd:.2e}  adjoint DOFs {e_q:.2e}  gradients {e_g:.2e}", flush=True)
    assert e_fwd <= 1e-11
    assert e_q <= TOL64_Q
    assert e_g <= TOL64_G
    # the context is back at the final state and time
    assert ctx.time() == pytest.approx(t, rel=1e-14)
    assert np.array_equal(ctx.read_dofs(), qT)


@pytest.mark.parametrize("order,mech", [(2, 3), (3, 3), (4, 3), (5, 3), (2, 0), (3, 0), (4, 0), (5, 0)])
def test_adjoint_matches_oracle_fp32(order, mech):
    """FP32 adjoint kernels, anelastic and elastic (the elastic variants of the
    two-wave transposed prediction at O = 4, 5 and the one-wave kernel at
    O = 2, 3)."""
    ctx, w = _setup(order, mech, 2, False)
    x, y, sb = _inputs(ctx, 40 + order + mech)
    t = 3 * w["sync"]
    qT, seis, res = _run_gpu(ctx, x, y, sb, t, 1)
    orc = _oracle(w)
    orc.set_initial(x)
    ores = oracle_adjoint(orc, t, seis_b=sb, q_b=y, attn=w["attn"])
    e_q = parity(res["q0_b"], ores["q0_b"])
    e_g = _grad_err(res, ores)
    print(f"[adjoint] FP32 O={order} m={mech}: adjoint DOFs {e_q:.2e}  gradients {e_g:.2e}", flush=True)
    assert e_q <= 2e-5
    assert e_g <= 1e-4


def test_dot_product_identity_on_the_gpu():
    ctx, w = _setup(3, 3, 2, True)
    x, y, sb = _inputs(ctx, 9)
    t = 2 * w["sync"]
    qT, seis, res = _run_gpu(ctx, x, y, sb, t, 1, sources=False)
    lhs = np.sum(qT * y) + np.sum(seis * sb)
    rhs = np.sum(x * res["q0_b"])
    scale = np.sum(np.abs(qT * y)) + np.sum(np.abs(seis * sb))
    print(f"[adjoint] GPU dot identity {abs(lhs - rhs) / scale:.2e}", flush=True)
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_checkpoint_interval_does_not_change_the_result():
    out = []
    for every in (1, 4):
        ctx, w = _setup(3, 3, 2, True)
        x, y, sb = _inputs(ctx, 11)
        out.append(_run_gpu(ctx, x, y, sb, 4 * w["sync"], every)[2])
        ctx.close()
    assert parity(out[0]["q0_b"], out[1]["q0_b"]) <= 1e-13
    assert _grad_err(out[0], out[1]) <= 1e-13


def test_recorded_segment_reuse_and_repeated_sweeps():
    """The final segment of a checkpointed advance records its level states
    and the sweep skips its replay: a forward split over two advance calls
    (the first call's record is stale), repeated sweeps after one forward
    (the first sweep's replays overwrite the record), and one segment over
    the whole window agree."""
    ctx, w = _setup(3, 3, 2, True)
    x, y, sb = _inputs(ctx, 17)
    s = w["sync"]
    ctx.set_sources(SRC["xyz"], SRC["moment"], SRC["stf_kind"], SRC["stf_params"])
    ctx.set_receivers(REC["xyz"], REC["dt_sample"], REC["n_samples"])
    ctx.set_checkpointing(1)
    ctx.set_initial(x)
    ctx.advance_to(2 * s)
    ctx.advance_to(3 * s)
    first = ctx.adjoint(dj_dseis=sb, dj_dq=y)
    again = ctx.adjoint(dj_dseis=sb, dj_dq=y)
    ctx.rewind()
    ctx.set_checkpointing(3)
    ctx.set_initial(x)
    ctx.advance_to(3 * s)
    whole = ctx.adjoint(dj_dseis=sb, dj_dq=y)
    for other in (again, whole):
        assert parity(first["q0_b"], other["q0_b"]) <= 1e-13
        assert _grad_err(first, other) <= 1e-13


@pytest.mark.parametrize("order,fp64", [(3, True), (3, False), (5, False)])
def test_recording_leaves_the_forward_unchanged(order, fp64):
    """A checkpointed advance (its final segment writes the reverse sweep's
    record from the forward kernels) gives the same DOFs and seismograms,
    bit for bit, as the plain advance."""
    out = []
    for every in (0, 3):
        ctx, w = _setup(order, 3, 2, fp64)
        x, y, sb = _inputs(ctx, 23)
        ctx.set_sources(SRC["xyz"], SRC["moment"], SRC["stf_kind"], SRC["stf_params"])
        ctx.set_receivers(REC["xyz"], REC["dt_sample"], REC["n_samples"])
        ctx.set_checkpointing(every)
        ctx.set_initial(x)
        ctx.advance_to(3 * w["sync"])
        out.append((ctx.read_dofs(), ctx.read_receivers()))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_material_upload_between_sweeps():
    """A sweep, a material upload, then another sweep: the second gradient is
    that of the new model (the chain-rule table kept on the device between
    sweeps is rebuilt after the upload), against the oracle's discrete
    adjoint on the new model."""
    ctx, w = _setup(3, 3, 2, True)
    x, y, sb = _inputs(ctx, 19)
    t = 2 * w["sync"]
    mat, attn = w["mat"], w["attn"]
    rng = np.random.default_rng(5)
    pert = {k: mat[k] * (1.0 + 0.03 * rng.uniform(-1.0, 1.0, ctx.K)) for k in ("rho", "vp", "vs")}
    _run_gpu(ctx, x, y, sb, t, 1)
    ctx.upload_materials(pert["rho"], pert["vp"], pert["vs"], attn["omega"], attn["yp"], attn["ys"])
    ctx.rewind()
    res = _run_gpu(ctx, x, y, sb, t, 1)[2]
    orc = _oracle(w, mat=pert)
    orc.set_initial(x)
    ores = oracle_adjoint(orc, t, seis_b=sb, q_b=y, attn=attn)
    e_q, e_g = parity(res["q0_b"], ores["q0_b"]), _grad_err(res, ores)
    print(f"[adjoint] after a material upload: adjoint DOFs {e_q:.2e}  gradients {e_g:.2e}", flush=True)
    assert e_q <= TOL64_Q
    assert e_g <= TOL64_G


def test_gradient_matches_central_differences_fp64():
    ctx, w = _setup(3, 3, 2, True)
    x, y, sb = _inputs(ctx, 13)
    t = 3 * w["sync"]
    _, _, res = _run_gpu(ctx, x, y, sb, t, 1)
    ctx.set_checkpointing(0)
    mat, attn = w["mat"], w["attn"]

    def J(m):
        ctx.upload_materials(m["rho"], m["vp"], m["vs"], attn["omega"], attn["yp"], attn["ys"])
        ctx.rewind()
        ctx.set_initial(x)
        ctx.advance_to(t)
        return np.sum(ctx.read_dofs() * y) + np.sum(ctx.read_receivers() * sb)

    rng = np.random.default_rng(3)
    eps, worst = 1e-5, 0.0
    for _ in range(20):
        d = {k: rng.standard_normal(ctx.K) * mat[k] for k in ("rho", "vp", "vs")}
        pred = sum(np.sum(res["g_" + k] * d[k]) for k in ("rho", "vp", "vs"))
        fd = (J({k: mat[k] + eps * d[k] for k in d}) - J({k: mat[k] - eps * d[k] for k in d})) / (2 * eps)
        worst = max(worst, abs(pred - fd) / abs(fd))
    print(f"[adjoint] GPU gradient vs central differences: {worst:.2e}", flush=True)
    assert worst <= 1e-6


def test_autograd_misfit_gradient():
    """torch.autograd through the library: the L2 misfit between the
    seismograms and data from a model perturbed by +-3% per element; the
    gradient equals the oracle's discrete adjoint for the same seismogram
    adjoint and central differences of the misfit."""
    import torch
    from paper_2202_10313_amd.autograd import Simulation
    ctx, w = _setup(3, 3, 2, True)
    ctx.set_sources(SRC["xyz"], SRC["moment"], SRC["stf_kind"], SRC["stf_params"])
    ctx.set_receivers(REC["xyz"], REC["dt_sample"], REC["n_samples"])
    t = 3 * w["sync"]
    mat, attn = w["mat"], w["attn"]
    x = synth.random_state(21, ctx.K, ctx.nq, ctx.B)
    sim = Simulation(ctx, t, attn["omega"], attn["yp"], attn["ys"], q0=x)
    dev = "cuda"
    rng = np.random.default_rng(17)
    pert = {k: mat[k] * (1 + rng.uniform(-0.03, 0.03, ctx.K)) for k in ("rho", "vp", "vs")}
    with torch.no_grad():
        d = sim.seismograms(*(torch.tensor(pert[k], device=dev) for k in ("rho", "vp", "vs")))
    dt = REC["dt_sample"]

    def misfit(m, grad=False):
        ps = [torch.tensor(m[k], device=dev, requires_grad=grad) for k in ("rho", "vp", "vs")]
        s = sim.seismograms(*ps)
        return 0.5 * ((s - d) ** 2).sum() * dt, s, ps

    J, s, ps = misfit(mat, grad=True)
    J.backward()
    g = {k: p.grad.cpu().numpy() for k, p in zip(("rho", "vp", "vs"), ps)}
    orc = _oracle(w)
    orc.set_initial(x)
    ores = oracle_adjoint(orc, t, seis_b=((s - d) * dt).detach().cpu().numpy(), attn=attn)
    e = max(np.linalg.norm(g[k] - ores["g_" + k]) / np.linalg.norm(ores["g_" + k]) for k in g)
    worst = 0.0
    eps = 1e-5
    for _ in range(3):
        dd = {k: rng.standard_normal(ctx.K) * mat[k] for k in g}
        pred = sum(np.sum(g[k] * dd[k]) for k in g)
        with torch.no_grad():
            fd = (misfit({k: mat[k] + eps * dd[k] for k in g})[0] - misfit({k: mat[k] - eps * dd[k] for k in g})[0])
        fd = float(fd) / (2 * eps)
        worst = max(worst, abs(pred - fd) / abs(fd))
    print(f"[adjoint] autograd: vs oracle {e:.2e}, vs central differences {worst:.2e}", flush=True)
    assert e <= TOL64_G
    assert worst <= 1e-6


@pytest.mark.parametrize("mech", [0, 3])
def test_adjoint_5k_tets_order4(mech):
    """The oracle-sized mesh of the differentiation workload (2 x 2 x 1 km
    layered box, 5,082 tets, O = 4, N_c = 2, 32 surface receivers): misfit
    against data from a +-3% perturbed model, GPU adjoint (FP64) against the
    oracle's discrete adjoint over two LTS cycles."""
    from tests.helpers import anelastic_setup, gpu_context
    w = anelastic_setup("small", 4, 2, with_source=True, n_rec=32)
    attn = w["attn"] if mech else None
    mat = w["mat"]
    ctx = gpu_context(w, 4, 2, True, mechanisms=mech)
    info = ctx.get_clusters()
    assert len(np.unique(info["clusters"])) == 2
    K, nq = ctx.K, ctx.nq
    x = synth.random_state(35, K, nq, ctx.B)
    dts, ns = 2.5e-4, 20
    ctx.set_sources(w["src"]["xyz"], w["src"]["moment"], w["src"]["stf_kind"], w["src"]["stf_params"])
    ctx.set_receivers(w["rec"], dts, ns)
    t = 2 * info["sync_dt"]
    # data from the perturbed model (same clusters and steps)
    rng = np.random.default_rng(55)
    pert = {k: mat[k] * (1 + rng.uniform(-0.03, 0.03, K)) for k in ("rho", "vp", "vs")}
    extra = (attn["omega"], attn["yp"], attn["ys"]) if mech else ()
    ctx.upload_materials(pert["rho"], pert["vp"], pert["vs"], *extra)
    ctx.set_initial(x)
    ctx.advance_to(t)
    d = ctx.read_receivers()
    ctx.upload_materials(mat["rho"], mat["vp"], mat["vs"], *extra)
    ctx.rewind()
    ctx.set_checkpointing(1)
    ctx.set_initial(x)
    ctx.advance_to(t)
    s = ctx.read_receivers()
    sb = (s - d) * dts
    res = ctx.adjoint(dj_dseis=sb)
    print(f"[adjoint] 5k tets O=4 m={mech}: running the oracle adjoint", flush=True)
    orc = Oracle(w["mesh"], mat, 4, attn=attn, n_clusters=2, lam=info["lam"], clusters=info["clusters"],
                 dt_min=info["dt_min"], sources=w["src"], receivers=dict(xyz=w["rec"], dt_sample=dts, n_samples=ns))
    orc.set_initial(x)
    ores = oracle_adjoint(orc, t, seis_b=sb, attn=attn)
    e_s = np.linalg.norm(orc.seis - s) / np.linalg.norm(orc.seis)
    e_q = parity(res["q0_b"], ores["q0_b"])
    e_g = _grad_err(res, ores)
    print(f"[adjoint] 5k tets O=4 m={mech} FP64: seismograms {e_s:.2e} adjoint DOFs {e_q:.2e} gradients {e_g:.2e}",
          flush=True)
    assert e_s <= 1e-11
    assert e_q <= TOL64_Q
    assert e_g <= TOL64_G


def test_adjoint_call_errors():
    """No checkpoints, dropped checkpoints and a negative interval are
    refused with EDG_ESTATE / EDG_EINVAL instead of computing anything."""
    from paper_2202_10313_amd import EdgError
    ctx, w = _setup(2, 0, 2, True)
    with pytest.raises(EdgError, match="EDG_ESTATE"):
        ctx.adjoint()
    ctx.set_checkpointing(1)
    ctx.set_initial(synth.random_state(1, ctx.K, ctx.nq, ctx.B))
    ctx.advance_to(w["sync"])
    ctx.upload_materials(w["mat"]["rho"], w["mat"]["vp"], w["mat"]["vs"])    # drops the checkpoints
    with pytest.raises(EdgError, match="EDG_ESTATE"):
        ctx.adjoint()
    with pytest.raises(EdgError, match="EDG_EINVAL"):
        ctx.set_checkpointing(-1)


def test_oversized_checkpoint_interval_is_refused():
    """A checkpoint interval whose level-state record cannot be allocated
    fails the advance with EDG_ENOMEM naming the bytes (the allocation is
    refused by the runtime before any kernel runs), and a usable interval
    works afterwards."""
    from paper_2202_10313_amd import EdgError
    ctx, w = _setup(2, 0, 2, True)
    ctx.set_checkpointing(1 << 30)
    ctx.set_initial(synth.random_state(1, ctx.K, ctx.nq, ctx.B))
    with pytest.raises(EdgError, match="EDG_ENOMEM.*bytes"):
        ctx.advance_to(w["sync"])
    ctx.rewind()
    ctx.set_checkpointing(1)
    ctx.set_initial(synth.random_state(1, ctx.K, ctx.nq, ctx.B))
    ctx.advance_to(w["sync"])
    g = ctx.adjoint(dj_dq=np.ones((ctx.K, ctx.nq, ctx.B)), want_q0=True)
    assert np.all(np.isfinite(g["q0_b"]))


def test_device_pointer_boundary_matches_host():
    """The device-pointer forms of edg_upload_materials, edg_read_receivers
    and edg_adjoint (on_device = 1) give what the host forms give: the
    material tables built on the device equal the host's, the seismograms
    and the initial-state adjoint (staged through the host) are the same
    words, and the gradients agree to rounding (the transposed prediction
    sums an element's gradient words with LDS atomics from both of its
    waves, in a timing-dependent order).  A material out of range in device
    memory is refused and changes nothing."""
    import torch
    from paper_2202_10313_amd import EdgError
    out = []
    for dev in (False, True):
        ctx, w = _setup(4, 3, 2, False)
        mat, attn = w["mat"], w["attn"]
        rng = np.random.default_rng(5)
        pert = {k: mat[k] * (1 + rng.uniform(-0.03, 0.03, ctx.K)) for k in ("rho", "vp", "vs")}
        if dev:
            ctx.upload_materials(*(torch.tensor(pert[k], device="cuda") for k in ("rho", "vp", "vs")),
                                 torch.tensor(attn["omega"], device="cuda"), torch.tensor(attn["yp"], device="cuda"),
                                 torch.tensor(attn["ys"], device="cuda"))
        else:
            ctx.upload_materials(pert["rho"], pert["vp"], pert["vs"], attn["omega"], attn["yp"], attn["ys"])
        x, y, sb = _inputs(ctx, 77)
        ctx.set_sources(SRC["xyz"], SRC["moment"], SRC["stf_kind"], SRC["stf_params"])
        ctx.set_receivers(REC["xyz"], REC["dt_sample"], REC["n_samples"])
        ctx.set_checkpointing(2)
        ctx.set_initial(x)
        ctx.advance_to(3 * w["sync"])
        if dev:
            seis = ctx.read_receivers_device("cuda").cpu().numpy()
            res = ctx.adjoint_device(torch.tensor(sb, device="cuda"), torch.tensor(y, device="cuda"), want_q0=True)
            res = {k: v.cpu().numpy() for k, v in res.items()}
            # out of range on the device: refused, the context is unchanged
            bad = torch.tensor(pert["vs"] * 10.0, device="cuda")
            with pytest.raises(EdgError) as e:
                ctx.upload_materials(torch.tensor(pert["rho"], device="cuda"), torch.tensor(pert["vp"], device="cuda"),
                                     bad, torch.tensor(attn["omega"], device="cuda"),
                                     torch.tensor(attn["yp"], device="cuda"), torch.tensor(attn["ys"], device="cuda"))
            assert e.value.code == -1
            res2 = ctx.adjoint(dj_dseis=sb, dj_dq=y)          # checkpoints and tables kept
            _assert_same_adjoint(res2, res)
        else:
            seis = ctx.read_receivers()
            res = ctx.adjoint(dj_dseis=sb, dj_dq=y)
        out.append((seis, res))
        ctx.close()
    (s0, r0), (s1, r1) = out
    assert np.array_equal(s0, s1)
    _assert_same_adjoint(r0, r1)


def _assert_same_adjoint(a, b):
    assert np.array_equal(a["q0_b"], b["q0_b"])
    for k in ("g_rho", "g_vp", "g_vs"):
        e = np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k])
        print(f"[adjoint] repeated sweep {k}: {e:.2e}", flush=True)
        assert e <= 1e-12, k


def test_autograd_stale_backward_raises():
    """A backward through a graph whose forward has been superseded by a
    later forward on the same Simulation raises instead of returning the
    later model's gradient; the latest graph's backward still works."""
    import torch
    from paper_2202_10313_amd.autograd import Simulation
    ctx, w = _setup(3, 0, 2, True)
    ctx.set_sources(SRC["xyz"], SRC["moment"], SRC["stf_kind"], SRC["stf_params"])
    ctx.set_receivers(REC["xyz"], REC["dt_sample"], REC["n_samples"])
    sim = Simulation(ctx, 2 * w["sync"], q0=synth.random_state(23, ctx.K, ctx.nq, ctx.B))
    mat = w["mat"]
    ps1 = [torch.tensor(mat[k], device="cuda", requires_grad=True) for k in ("rho", "vp", "vs")]
    J1 = (sim.seismograms(*ps1) ** 2).sum()
    ps2 = [torch.tensor(mat[k] * 1.01, device="cuda", requires_grad=True) for k in ("rho", "vp", "vs")]
    J2 = (sim.seismograms(*ps2) ** 2).sum()
    with pytest.raises(RuntimeError, match="later forward"):
        J1.backward()
    J2.backward()
    assert all(torch.isfinite(p.grad).all() and p.grad.abs().sum() > 0 for p in ps2)


def _runs_setup(order, fp64, n_runs, srcs):
    """A context of n_runs runs on the adjoint tests' mesh, each run with its
    own sources (srcs[r]: list of (xyz, moment) or empty)."""
    from paper_2202_10313_amd import Context
    mesh, mat = _mesh()
    attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
    ctx = Context(order, mechanisms=3, n_clusters=2, fp64=fp64, cfl=0.5, lam=None, n_runs=n_runs)
    ctx.upload_mesh(mesh["tet_verts"], mesh["tet_xyz"], mesh["face_bc"])
    ctx.upload_materials(mat["rho"], mat["vp"], mat["vs"], attn["omega"], attn["yp"], attn["ys"])
    ctx.upload_clusters(None)
    for r, s in enumerate(srcs):
        if s:
            xyz = np.array([p[0] for p in s])
            mom = np.array([p[1] for p in s])
            ctx.set_sources(xyz, mom, 0, np.tile(SRC["stf_params"], (len(s), 1)), run=r)
    ctx.set_receivers(REC["xyz"], REC["dt_sample"], REC["n_samples"])
    return ctx


@pytest.mark.parametrize("order,fp64,every", [(3, True, 1), (5, False, 2)])
def test_multi_run_adjoint_equals_single_runs(order, fp64, every):
    """n_runs = 3 (one source, none, two sources): the adjoint DOFs of each
    run equal the single-run sweep of that run, and the material gradients
    equal the sum of the single-run gradients."""
    srcs = [[(SRC["xyz"][0], SRC["moment"][0])], [],
            [(np.array([120.0, 280.0, -60.0]), SRC["moment"][0] * 0.5),
             (np.array([300.0, 120.0, -250.0]), SRC["moment"][0][::-1].copy())]]
    print(f"[adjoint] 3 runs O={order} {'FP64' if fp64 else 'FP32'} every={every}", flush=True)
    rng = np.random.default_rng(order)
    ctx = _runs_setup(order, fp64, 3, srcs)
    sync = ctx.get_clusters()["sync_dt"]
    xs = [synth.random_state(70 + r, ctx.K, ctx.nq, ctx.B) for r in range(3)]
    y = rng.standard_normal((3, ctx.K, ctx.nq, ctx.B)) * np.where(np.arange(ctx.nq) < 6, 1e-6, 1.0)[None, None, :, None]
    sb = rng.standard_normal((3, len(REC["xyz"]), REC["n_samples"], 9))
    ctx.set_checkpointing(every)
    for r in range(3):
        ctx.set_initial(xs[r], run=r)
    ctx.advance_to(4 * sync)
    qT = [ctx.read_dofs(run=r) for r in range(3)]
    res = ctx.adjoint(dj_dseis=sb, dj_dq=y)
    assert res["q0_b"].shape == (3, ctx.K, ctx.nq, ctx.B)
    assert all(np.array_equal(qT[r], ctx.read_dofs(run=r)) for r in range(3))
    g_sum = {k: 0.0 for k in ("g_rho", "g_vp", "g_vs")}
    tol_q, tol_g = (1e-12, 1e-12) if fp64 else (2e-6, 2e-5)
    for r in range(3):
        one = _runs_setup(order, fp64, 1, [srcs[r]])
        one.set_checkpointing(every)
        one.set_initial(xs[r])
        one.advance_to(4 * sync)
        assert np.array_equal(one.read_dofs(), qT[r])
        ref = one.adjoint(dj_dseis=sb[r], dj_dq=y[r])
        e = parity(res["q0_b"][r], ref["q0_b"])
        print(f"[adjoint] run {r}: adjoint DOFs vs single run {e:.2e}", flush=True)
        assert e <= tol_q
        for k in g_sum:
            g_sum[k] = g_sum[k] + ref[k]
        one.close()
    eg = max(np.linalg.norm(res[k] - g_sum[k]) / np.linalg.norm(g_sum[k]) for k in g_sum)
    print(f"[adjoint] gradient vs sum of single runs {eg:.2e}", flush=True)
    assert eg <= tol_g


@pytest.mark.parametrize("order,fp64", [(3, True), (5, False)])
def test_graph_captured_reverse_sweep(order, fp64):
    """EDG_FLAG_GRAPH: the backward levels of each segment are captured once
    per segment length and replayed (segments of 4, 4 and 2 levels, two
    runs, two sweeps in a row); the results equal the eager sweep."""
    from paper_2202_10313_amd import FLAG_GRAPH
    print(f"[adjoint] graph-captured sweep O={order} {'FP64' if fp64 else 'FP32'}", flush=True)
    srcs = [[(SRC["xyz"][0], SRC["moment"][0])], [(np.array([120.0, 280.0, -60.0]), SRC["moment"][0] * 0.5)]]
    rng = np.random.default_rng(3)
    out = []
    for flags in (0, FLAG_GRAPH):
        from paper_2202_10313_amd import Context
        mesh, mat = _mesh()
        attn = synth.attenuation_inputs(mat, 3, 0.1, 10.0)
        ctx = Context(order, mechanisms=3, n_clusters=2, fp64=fp64, cfl=0.5, lam=None, n_runs=2, flags=flags)
        ctx.upload_mesh(mesh["tet_verts"], mesh["tet_xyz"], mesh["face_bc"])
        ctx.upload_materials(mat["rho"], mat["vp"], mat["vs"], attn["omega"], attn["yp"], attn["ys"])
        ctx.upload_clusters(None)
        for r, s in enumerate(srcs):
            ctx.set_sources(np.array([s[0][0]]), np.array([s[0][1]]), 0, SRC["stf_params"], run=r)
            ctx.set_initial(synth.random_state(90 + r, ctx.K, ctx.nq, ctx.B), run=r)
        ctx.set_receivers(REC["xyz"], REC["dt_sample"], REC["n_samples"])
        ctx.set_checkpointing(2)
        ctx.advance_to(5 * ctx.get_clusters()["sync_dt"])
        if not out:
            y = rng.standard_normal((2, ctx.K, ctx.nq, ctx.B)) * 1e-3
            sb = rng.standard_normal((2, len(REC["xyz"]), REC["n_samples"], 9))
        out.append([ctx.adjoint(dj_dseis=sb, dj_dq=y) for _ in range(2)])
        ctx.close()
    tol = 1e-13 if fp64 else 1e-6
    for eager, graph in zip(out[0], out[1]):
        for key in ("q0_b", "g_rho", "g_vp", "g_vs"):
            e = np.linalg.norm(eager[key] - graph[key]) / np.linalg.norm(eager[key])
            print(f"[adjoint] graph vs eager {key}: {e:.2e}", flush=True)
            assert e <= tol, key


def test_multi_run_adjoint_device_pointers():
    """edg_adjoint on device pointers for a 2-run context (leading run axis on
    dJ/dseis, dJ/dQ and the initial-state adjoint) gives the host form's
    results."""
    import torch
    print("[adjoint] 2 runs, device pointers, O=4 FP32", flush=True)
    srcs = [[(SRC["xyz"][0], SRC["moment"][0])], [(np.array([120.0, 280.0, -60.0]), SRC["moment"][0] * 0.5)]]
    rng = np.random.default_rng(8)
    ctx = _runs_setup(4, False, 2, srcs)
    sync = ctx.get_clusters()["sync_dt"]
    for r in range(2):
        ctx.set_initial(synth.random_state(50 + r, ctx.K, ctx.nq, ctx.B), run=r)
    ctx.set_checkpointing(1)
    ctx.advance_to(3 * sync)
    y = rng.standard_normal((2, ctx.K, ctx.nq, ctx.B)) * 1e-3
    sb = rng.standard_normal((2, len(REC["xyz"]), REC["n_samples"], 9))
    host = ctx.adjoint(dj_dseis=sb, dj_dq=y)
    dev = ctx.adjoint_device(torch.tensor(sb, device="cuda"), torch.tensor(y, device="cuda"), want_q0=True)
    dev = {k: v.cpu().numpy() for k, v in dev.items()}
    assert dev["q0_b"].shape == (2, ctx.K, ctx.nq, ctx.B)
    _assert_same_adjoint(dev, host)
