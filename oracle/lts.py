"""Clustered rate-2 local time stepping: CFL steps, clustering, normalisation,
lambda search (test infrastructure: CPU oracle).

Sec. V-A (Clustering):
  * dt_min = min_k dt_k^CFL;
  * N_c clusters C_l = [2^(l-1) lam dt_min, 2^l lam dt_min) for l < N_c and
    C_{N_c} = [2^(N_c-1) lam dt_min, inf), lam in (0.5, 1];
    an element joins the cluster whose interval holds its CFL step and then
    advances with the cluster's lower bound 2^(l-1) lam dt_min;
  * normalisation: neighbours may differ by at most one cluster; an element
    with a neighbour two or more clusters finer moves down (repeat to the
    fixpoint, which equals min_j (l_j + graph distance(k, j)));
  * lam is searched in steps of 0.01 and the theoretical speedup over GTS is
    maximised.

Readings (the paper is silent): the CFL step is
  dt_k = C * 2 r_k / ((2(O-1)+1) vp_k)   (r_k the insphere radius, C = cfl);
the speedup is evaluated after normalisation as
  S(lam) = K / sum_l n_l / (2^(l-1) lam),
summed in cluster order; candidates lam = i/100 for i = 51..100; ties go to the
larger lam.  Interval membership uses the products (lam*dt_min)*2^(l-1)
compared with dt_k in FP64 (the lower bound belongs to the interval).

Pins (tests/test_oracle_lts.py): the worked examples of Sec. V-A (Clustering)
(3 lam dt_min -> C_2; a C_3 element next to a C_1 element moves to C_2;
lam = 0.75 intervals); the normalisation fixpoint against brute-force graph
distances; the lambda search against exhaustive evaluation.
"""
from __future__ import annotations

import math
import numpy as np


def cfl_steps(inradius, vp, order, cfl):
    return cfl * 2.0 * np.asarray(inradius) / ((2 * (order - 1) + 1) * np.asarray(vp))


def assign(dt, dt_min, lam, n_clusters):
    """Cluster index 1..N_c (1 = finest) of every element, before normalisation."""
    base = lam * dt_min
    cl = np.ones(len(dt), dtype=np.int64)
    for l in range(2, n_clusters + 1):
        cl[dt >= math.ldexp(base, l - 1)] = l
    return cl


def normalize(cl, nbr):
    cl = cl.copy()
    while True:
        nb = np.where(nbr >= 0, cl[np.maximum(nbr, 0)], 1 << 40)
        new = np.minimum(cl, nb.min(axis=1) + 1)
        if np.array_equal(new, cl):
            return cl
        cl = new


def speedup(cl, lam, n_clusters):
    K = len(cl)
    denom = 0.0
    for l in range(1, n_clusters + 1):
        denom += np.count_nonzero(cl == l) / (math.ldexp(1.0, l - 1) * lam)
    return K / denom


def cluster(dt, nbr, n_clusters, lam=None):
    """(cluster ids, lam, theoretical speedup).  lam=None searches 0.51..1.00."""
    dt = np.asarray(dt, dtype=np.float64)
    dt_min = float(dt.min())
    if lam is not None:
        cl = normalize(assign(dt, dt_min, lam, n_clusters), nbr)
        return cl, float(lam), speedup(cl, lam, n_clusters)
    best = None
    for i in range(51, 101):
        lm = i / 100.0
        cl = normalize(assign(dt, dt_min, lm, n_clusters), nbr)
        s = speedup(cl, lm, n_clusters)
        if best is None or s >= best[2]:
            best = (cl, lm, s)
    return best


def cluster_dt(dt_min, lam, n_clusters):
    """Time step of every cluster l = 1..N_c (index 0 -> cluster 1)."""
    return np.array([math.ldexp(lam * dt_min, l - 1) for l in range(1, n_clusters + 1)])
