"""Pins of the oracle's clustering and LTS buffer algebra against the paper's
worked examples, brute force and an independent time integration (no GPU)."""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import lts
from oracle.solver import Oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def test_cluster_example_three_lambda():
    g = GOLD["cluster_example_3"]
    for lam in (0.6, 0.8, 1.0):
        dt = np.array([1.0, g["dt_over_lambda_dtmin"] * lam, 10.0])
        dt_min = 1.0
        cl = lts.assign(dt, dt_min, lam, 5)
        assert cl[1] == g["cluster"]


def test_lambda_075_intervals():
    g = GOLD["lambda_075_intervals"]
    lam = g["lambda"]
    dt = np.array([1.0, 1.49, 1.5, 2.99, 3.0, 3.5])
    cl = lts.assign(dt, 1.0, lam, 3)
    assert list(cl) == [1, 1, 2, 2, 3, 3]
    steps = lts.cluster_dt(1.0, lam, 3)
    assert steps[2] == pytest.approx(g["bulk_dt_lambda"])
    assert lts.cluster_dt(1.0, 1.0, 3)[1] == pytest.approx(g["bulk_dt_one"])


def test_normalisation_example():
    g = GOLD["normalisation_example"]
    cl = np.array([g["initial"], g["neighbour"]])
    nbr = np.array([[1, -1, -1, -1], [0, -1, -1, -1]])
    assert lts.normalize(cl, nbr)[0] == g["final"]


def test_normalisation_is_graph_distance_fixpoint():
    rng = np.random.default_rng(3)
    for trial in range(5):
        K = 40
        nbr = -np.ones((K, 4), dtype=np.int64)
        # random graph with degree <= 4
        edges = set()
        for _ in range(70):
            a, b = rng.integers(0, K, 2)
            if a == b or (min(a, b), max(a, b)) in edges:
                continue
            fa, fb = np.nonzero(nbr[a] < 0)[0], np.nonzero(nbr[b] < 0)[0]
            if len(fa) and len(fb):
                nbr[a, fa[0]], nbr[b, fb[0]] = b, a
                edges.add((min(a, b), max(a, b)))
        cl0 = rng.integers(1, 6, K)
        # brute force: BFS distances
        INF = 10 ** 9
        dist = np.full((K, K), INF)
        for s in range(K):
            dist[s, s] = 0
            frontier = [s]
            while frontier:
                nxt = []
                for u in frontier:
                    for v in nbr[u]:
                        if v >= 0 and dist[s, v] == INF:
                            dist[s, v] = dist[s, u] + 1
                            nxt.append(v)
                frontier = nxt
        want = np.min(np.where(dist < INF, cl0[None, :] + dist, INF), axis=1)
        assert np.array_equal(lts.normalize(cl0, nbr), want)


def test_lambda_search_is_exhaustive_max():
    rng = np.random.default_rng(4)
    K = 300
    dt = np.exp(rng.uniform(0, 2.5, K))
    nbr = -np.ones((K, 4), dtype=np.int64)
    for k in range(K - 1):
        nbr[k, 0], nbr[k + 1, 1] = k + 1, k
    cl, lam, s = lts.cluster(dt, nbr, 4, None)
    best = max(((lts.speedup(lts.normalize(lts.assign(dt, dt.min(), i / 100, 4), nbr), i / 100, 4), i / 100)
                for i in range(51, 101)))
    assert s == pytest.approx(best[0], rel=1e-15)
    assert lam == max(i / 100 for i in range(51, 101)
                      if lts.speedup(lts.normalize(lts.assign(dt, dt.min(), i / 100, 4), nbr), i / 100, 4) == best[0])


def test_speedup_formula_matches_paper_loh3():
    # with the printed cluster sizes and speedups, the load share of the
    # dominant cluster follows from S = K / sum_l n_l / (2^(l-1) lam)
    g = GOLD["loh3_clustering"]
    for key in ("lambda_1", "lambda_08"):
        c = g[key]
        load = (c["count"] / (2 ** (c["cluster"] - 1) * c["lambda"])) / (g["K"] / c["speedup"])
        assert abs(load - c["load"]) < 0.003


# -------------------------------------------------------------- buffer walk-through

def star_mesh():
    """A centre tet k with one tet glued on each of its faces (k_1..k_4).
    Outer faces are absorbing."""
    V = np.array([[0.0, 0, 0], [100.0, 0, 0], [0, 100.0, 0], [0, 0, 100.0]])
    tets = [[0, 1, 2, 3]]
    xyz = [V.copy()]
    nid = 4
    for i in range(4):
        face = [m for m in range(4) if m != i]
        c = V[face].mean(axis=0)
        apex = 2 * c - V[i]            # reflect the opposite vertex through the face
        tets.append(face + [nid])
        xyz.append(np.vstack([V[face], apex]))
        nid += 1
    face_bc = np.full((5, 4), 2, dtype=np.int8)
    face_bc[0, :] = 0
    for t in range(1, 5):
        face_bc[t, 3] = 0              # face opposite the apex is the shared one
    return dict(tet_verts=np.array(tets, dtype=np.int64), tet_xyz=np.array(xyz), face_bc=face_bc)


class TracingOracle(Oracle):
    """Records every prediction's derivatives and every neighbour read."""

    def __init__(self, *a, **kw):
        self.preds = {}
        self.reads = []
        super().__init__(*a, **kw)

    def derivatives(self, idx):
        D = super().derivatives(idx)
        for pos, k in enumerate(idx):
            t0 = float(self.nstep[k]) * self.dt_elem[k]
            self.preds.setdefault(int(k), []).append((t0, [d[pos, :9].copy() for d in D]))
        return D

    def neighbour_data(self, idx, i):
        out, inner = super().neighbour_data(idx, i)
        for pos, k in enumerate(idx):
            if inner[pos]:
                self.reads.append((self._level, int(k), int(self.nbr[k, i]), out[pos].copy()))
        return out, inner

    def update(self, idx):
        super().update(idx)

    def run_traced(self, levels):
        allidx = np.arange(self.K)
        self._level = 0
        self.predict(allidx)
        period = 2 ** (self.cl - 1)
        for j in range(1, levels + 1):
            self._level = j
            act = np.nonzero(j % period == 0)[0]
            self.update(act)
            self.predict(act)


def _integral(pred_list, k, a, b, order):
    """Time integral over [a, b] of element k's Taylor expansion that was
    active at time a, by Gauss-Legendre quadrature (exact for its degree)."""
    t0, D = max((p for p in pred_list[k] if p[0] <= a + 1e-15), key=lambda p: p[0])
    x, w = np.polynomial.legendre.leggauss(order + 2)
    ts = (x + 1) / 2 * (b - a) + a
    ws = w / 2 * (b - a)
    out = 0.0
    for t, wt in zip(ts, ws):
        out = out + wt * sum((t - t0) ** d / math.factorial(d) * D[d] for d in range(order))
    return out


def test_lts_walkthrough_trace():
    mesh = star_mesh()
    K = 5
    mat = synth.homogeneous_materials(K)
    # k = 0 and k_2, k_3 step with 2 dt, k_1 with dt, k_4 with 4 dt (Fig. lts_scheme)
    clusters = np.array([2, 1, 2, 2, 3])
    order = 3
    orc = TracingOracle(mesh, mat, order, n_clusters=3, lam=1.0, clusters=clusters)
    orc.set_initial(synth.random_state(11, K, 9, orc.B))
    orc.run_traced(4)
    dt = orc.dt_cluster[0]
    reads = {(lv, c, n): d for (lv, c, n, d) in orc.reads}
    P = orc.preds
    # (b) level 1: only k_1 completes, using B2_k = T_k(t0, dt)
    assert {(lv, c) for (lv, c, n) in reads if lv == 1} == {(1, 1)}
    np.testing.assert_allclose(reads[(1, 1, 0)], _integral(P, 0, 0, dt, order), rtol=1e-12, atol=1e-9)
    # (c) level 2: k_1 uses B1_k - B2_k = T_k(t1, dt); k_2, k_3 use B1_k
    np.testing.assert_allclose(reads[(2, 1, 0)], _integral(P, 0, dt, 2 * dt, order), rtol=1e-11, atol=1e-9)
    for kk in (2, 3):
        np.testing.assert_allclose(reads[(2, kk, 0)], _integral(P, 0, 0, 2 * dt, order), rtol=1e-12, atol=1e-9)
    # k completes with k_1's accumulated B3 = T_k1(t0, dt) + T_k1(t1, dt)
    np.testing.assert_allclose(reads[(2, 0, 1)], _integral(P, 1, 0, dt, order) + _integral(P, 1, dt, 2 * dt, order),
                               rtol=1e-11, atol=1e-9)
    # ... and with k_4's B2 (first half of k_4's 4 dt step)
    np.testing.assert_allclose(reads[(2, 0, 4)], _integral(P, 4, 0, 2 * dt, order), rtol=1e-12, atol=1e-9)
    # (d) level 3: only k_1 again, B2_k of k's second prediction = T_k(t2, dt)
    assert {(lv, c) for (lv, c, n) in reads if lv == 3} == {(3, 1)}
    np.testing.assert_allclose(reads[(3, 1, 0)], _integral(P, 0, 2 * dt, 3 * dt, order), rtol=1e-11, atol=1e-9)
    # (e) level 4: k_4 uses B3_k = T_k(t0, 2dt) + T_k(t2, 2dt) = T_k(t0, 4dt)
    np.testing.assert_allclose(reads[(4, 4, 0)], _integral(P, 0, 0, 2 * dt, order) + _integral(P, 0, 2 * dt, 4 * dt, order),
                               rtol=1e-11, atol=1e-9)
    # k uses B1 - B2 of k_4 in its second half step
    np.testing.assert_allclose(reads[(4, 0, 4)], _integral(P, 4, 2 * dt, 4 * dt, order), rtol=1e-11, atol=1e-9)
    # every read happened at a level where the reader's own step ends
    for (lv, c, n) in reads:
        assert lv % 2 ** (clusters[c] - 1) == 0


# ------------------------------------------------------- schedule checker

def _piecewise_integral(preds, k, a, b, dt_k, order):
    """Exact time integral over [a, b] of element k's predictions, split at
    k's own step boundaries (each piece from the expansion of its step)."""
    out, t = 0.0, a
    while t < b - 1e-12 * dt_k:
        t1 = min(b, (math.floor(t / dt_k + 1e-9) + 1) * dt_k)
        out = out + _integral(preds, k, t, t1, order)
        t = t1
    return out


def _schedule_errors(orc, levels):
    """Every neighbour read of the traced run against the exact integral the
    buffers of Sec. V-B stand for: the reader finishing its step [a, b) needs
    the time integral of the neighbour's solution over exactly [a, b),
    whichever buffer (B1, B2, B1 - B2 or B3) provides it.  Returns the
    number of reads and the largest relative error."""
    worst, n = 0.0, 0
    for lv, c, nb, data in orc.reads:
        lc = orc.cl[c] - 1
        step = lv // 2 ** lc - 1
        dt_c = orc.dt_cluster[lc]
        a, b = step * dt_c, (step + 1) * dt_c
        ref = _piecewise_integral(orc.preds, nb, a, b, orc.dt_cluster[orc.cl[nb] - 1], orc.O)
        worst = max(worst, float(np.linalg.norm(data - ref) / max(np.linalg.norm(ref), 1e-300)))
        n += 1
    return n, worst


def _random_schedule_oracle(n_clusters, seed, cls=None):
    mesh = synth.layered_box(2, 2, [100.0, 200.0], 400.0, 400.0, jitter=0.15, seed=seed)
    K = mesh["tet_verts"].shape[0]
    mat = synth.random_materials(K, seed + 1)
    probe = Oracle(mesh, mat, 2)
    rng = np.random.default_rng(seed)
    cl = lts.normalize(rng.integers(1, n_clusters + 1, K), probe.nbr)
    orc = (cls or TracingOracle)(mesh, mat, 2, n_clusters=n_clusters, lam=1.0, clusters=cl)
    orc.set_initial(synth.random_state(seed + 2, K, 9, orc.B))
    return orc


@pytest.mark.parametrize("n_clusters,seed", [(2, 1), (3, 2), (4, 3), (5, 4)])
def test_schedule_checker_random_clusterings(n_clusters, seed):
    """Schedule checker of the oracle: random normalised clusterings with up
    to five clusters, two full cycles; every neighbour read is the exact
    integral over the reader's step."""
    orc = _random_schedule_oracle(n_clusters, seed)
    levels = 2 * 2 ** (n_clusters - 1)
    orc.run_traced(levels)
    present = len(np.unique(orc.cl))
    n, worst = _schedule_errors(orc, levels)
    print(f"schedule N_c={n_clusters} ({present} clusters present): {n} reads, worst {worst:.2e}")
    assert present >= min(n_clusters, 3) and n > 0
    assert worst <= 1e-10


class EarlyPredictOracle(TracingOracle):
    """A planted schedule mistake: each level predicts the next step before
    the steps that end there read the buffers."""

    def run_traced(self, levels):
        allidx = np.arange(self.K)
        self._level = 0
        self.predict(allidx)
        period = 2 ** (self.cl - 1)
        for j in range(1, levels + 1):
            self._level = j
            act = np.nonzero(j % period == 0)[0]
            self.nstep[act] += 1
            self.predict(act)
            self.nstep[act] -= 1
            self.update(act)


def test_schedule_checker_flags_a_planted_mistake():
    orc = _random_schedule_oracle(3, 2, cls=EarlyPredictOracle)
    orc.run_traced(8)
    n, worst = _schedule_errors(orc, 8)
    print(f"planted early prediction: {n} reads, worst {worst:.2e}")
    assert worst > 1e-3
