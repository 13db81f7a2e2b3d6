"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only *generates inputs*: tetrahedral meshes (vertex ids for the
topology, per-tet vertex coordinates for the geometry, boundary tags),
material fields, the constant-Q relaxation fit, moment-tensor point sources,
receiver positions and random initial states.  It holds none of the solver's
arithmetic (no basis functions, no fluxes, no time stepping), so importing it
from both the CPU oracle and the GPU path couples nothing.

Mesh convention (the C-ABI and the oracle both take this form):
  tet_verts [K,4] int64  vertex ids, used only to find shared faces
                         (periodic meshes reuse ids across the period);
  tet_xyz   [K,4,3] f64  vertex coordinates of each tet, in the same local
                         order as tet_verts;
  face_bc   [K,4] int8   per local face i (the face opposite local vertex i):
                         0 interior, 1 free surface, 2 absorbing.
"""
from __future__ import annotations

import math
import numpy as np

BC_INTERIOR = 0
BC_FREE = 1
BC_ABSORB = 2

# the six tets of a Kuhn (Freudenthal) split of a cube; cube corner c has
# offset (c & 1, (c >> 1) & 1, (c >> 2) & 1); every tet runs along the 0->7
# diagonal, so neighbouring cubes split conformingly.
KUHN_TETS = np.array([[0, 1, 3, 7], [0, 1, 5, 7], [0, 2, 3, 7],
                      [0, 2, 6, 7], [0, 4, 5, 7], [0, 4, 6, 7]], dtype=np.int64)


def _corner_offsets():
    return np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.int64)


def _hex_grid_tets(nx, ny, nz):
    """Tets of an nx*ny*nz hex grid as (cube index triple, corner index) pairs."""
    off = _corner_offsets()
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cubes = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1)  # [C,3]
    # corner lattice coordinates of every tet vertex: [C,6,4,3]
    lat = cubes[:, None, None, :] + off[KUHN_TETS][None, :, :, :]
    return lat.reshape(-1, 4, 3)


def _tag_box_faces(lat, n, bc_of_side):
    """face_bc for tets on a lattice box; bc_of_side[(axis, 0|1)] -> tag."""
    K = lat.shape[0]
    face_bc = np.zeros((K, 4), dtype=np.int8)
    for i in range(4):
        others = [m for m in range(4) if m != i]
        fl = lat[:, others, :]  # [K,3,3]
        for ax in range(3):
            for side, val in ((0, 0), (1, n[ax])):
                on = np.all(fl[:, :, ax] == val, axis=1)
                tag = bc_of_side.get((ax, side), BC_INTERIOR)
                face_bc[on, i] = tag
    return face_bc


def kuhn_cube_periodic(n: int, L: float, jitter: float = 0.0, seed: int = 0) -> dict:
    """Periodic cube [0,L]^3 of n^3 cubes, each Kuhn-split into 6 tets.

    Vertex ids wrap modulo n so faces on opposite sides of the box match;
    coordinates stay unwrapped so every tet keeps its true geometry.  jitter
    moves every (periodically identified) vertex by +-jitter*h per axis.
    """
    lat = _hex_grid_tets(n, n, n)
    h = L / n
    wrap = lat % n
    ids = (wrap[..., 0] * n + wrap[..., 1]) * n + wrap[..., 2]
    xyz = lat.astype(np.float64) * h
    if jitter > 0:
        d = np.random.default_rng(seed).uniform(-jitter * h, jitter * h, size=(n ** 3, 3))
        xyz = xyz + d[ids]
    return dict(tet_verts=ids.astype(np.int64), tet_xyz=xyz,
                face_bc=np.zeros((lat.shape[0], 4), dtype=np.int8),
                box=np.array([[0, L], [0, L], [0, L]], dtype=np.float64), periodic=True)


def layered_box(nx: int, ny: int, dz: list, Lx: float, Ly: float, jitter: float = 0.0,
                seed: int = 0, top_bc: int = BC_FREE, side_bc: int = BC_ABSORB,
                zjitter_boundaries: bool = False) -> dict:
    """Box [0,Lx]x[0,Ly]x[-sum(dz),0]: nx*ny hex columns, z-layers of thickness dz
    (listed from the top down), Kuhn-split.  The top face z=0 gets top_bc, the
    other five faces side_bc.  Interior vertices are jittered uniformly by
    +-jitter of the local spacing per axis; boundary vertices move only along
    their boundary plane(s)."""
    rng = np.random.default_rng(seed)
    dz = np.asarray(dz, dtype=np.float64)
    nz = len(dz)
    xs = np.linspace(0.0, Lx, nx + 1)
    ys = np.linspace(0.0, Ly, ny + 1)
    zs = np.concatenate([[0.0], -np.cumsum(dz)])[::-1]  # ascending: bottom .. 0
    hz_lo = np.concatenate([[np.inf], np.diff(zs)])       # spacing below each level
    hz_hi = np.concatenate([np.diff(zs), [np.inf]])
    hz = np.minimum(hz_lo, hz_hi)
    hx, hy = Lx / nx, Ly / ny
    I, J, Kz = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    P = np.stack([xs[I], ys[J], zs[Kz]], axis=-1)
    if jitter > 0:
        d = rng.uniform(-jitter, jitter, size=P.shape)
        d[..., 0] *= hx
        d[..., 1] *= hy
        d[..., 2] *= hz[Kz]
        d[..., 0][(I == 0) | (I == nx)] = 0.0
        d[..., 1][(J == 0) | (J == ny)] = 0.0
        d[..., 2][(Kz == 0) | (Kz == nz)] = 0.0
        P = P + d
    lat = _hex_grid_tets(nx, ny, nz)
    ids = (lat[..., 0] * (ny + 1) + lat[..., 1]) * (nz + 1) + lat[..., 2]
    xyz = P[lat[..., 0], lat[..., 1], lat[..., 2]]
    bc = {(0, 0): side_bc, (0, 1): side_bc, (1, 0): side_bc, (1, 1): side_bc,
          (2, 0): side_bc, (2, 1): top_bc}
    face_bc = _tag_box_faces(lat, (nx, ny, nz), bc)
    vol = np.einsum("ki,ki->k", np.cross(xyz[:, 1] - xyz[:, 0], xyz[:, 2] - xyz[:, 0]),
                    xyz[:, 3] - xyz[:, 0])
    ref = np.einsum("ki,ki->k", np.cross(lat[:, 1] - lat[:, 0], lat[:, 2] - lat[:, 0]).astype(float),
                    (lat[:, 3] - lat[:, 0]).astype(float))
    if np.any(np.sign(vol) != np.sign(ref)) or np.any(np.abs(vol) < 1e-9 * hx * hy * dz.min()):
        raise ValueError("jitter inverted or flattened a tetrahedron; lower it")
    return dict(tet_verts=ids.astype(np.int64), tet_xyz=xyz, face_bc=face_bc,
                box=np.array([[0, Lx], [0, Ly], [zs[0], 0.0]]), periodic=False)


def centroids(mesh: dict) -> np.ndarray:
    return mesh["tet_xyz"].mean(axis=1)


# --------------------------------------------------------------------------- materials

def gardner_rho(vp):
    """Gardner-type density [kg/m^3] from vp [m/s]."""
    return 310.0 * np.asarray(vp) ** 0.25


def layered_materials(mesh: dict, seed: int, sigma: float = 0.025, clip: float = 0.05,
                      vpvs: float = 1.8) -> dict:
    """vs by centroid depth (800 m/s near the top to 3500 m/s below 6 km),
    vp = vpvs*vs, Gardner density, a per-element Gaussian perturbation applied to
    vp and vs jointly, Qs = 50 vs[km/s] and Qp = 2 Qs."""
    rng = np.random.default_rng(seed)
    depth = -centroids(mesh)[:, 2]
    edges = [0, 300, 600, 1000, 2000, 4000, 6000]
    vals = [800.0, 1000.0, 1400.0, 2000.0, 2600.0, 3200.0, 3500.0]
    vs = np.full(depth.shape, vals[-1])
    for lo, hi, v in zip(edges[:-1], edges[1:], vals[:-1]):
        vs[(depth >= lo) & (depth < hi)] = v
    delta = np.clip(rng.normal(0.0, sigma, size=vs.shape), -clip, clip)
    vs = vs * (1.0 + delta)
    vp = vpvs * vs
    rho = gardner_rho(vp)
    qs = 50.0 * vs / 1000.0
    qp = 2.0 * qs
    return dict(rho=rho, vp=vp, vs=vs, qp=qp, qs=qs)


def homogeneous_materials(K: int, rho=2700.0, vp=6000.0, vs=3464.0, qp=None, qs=None) -> dict:
    out = dict(rho=np.full(K, float(rho)), vp=np.full(K, float(vp)), vs=np.full(K, float(vs)))
    if qp is not None:
        out["qp"] = np.full(K, float(qp))
        out["qs"] = np.full(K, float(qs))
    return out


def random_materials(K: int, seed: int) -> dict:
    """Strongly heterogeneous element-wise materials (for flux and energy tests)."""
    rng = np.random.default_rng(seed)
    vs = rng.uniform(1000.0, 3500.0, K)
    vp = vs * rng.uniform(1.6, 2.2, K)
    rho = rng.uniform(1800.0, 3000.0, K)
    qs = rng.uniform(20.0, 150.0, K)
    qp = qs * rng.uniform(1.5, 2.5, K)
    return dict(rho=rho, vp=vp, vs=vs, qp=qp, qs=qs)


def relaxation_frequencies(m: int, f_min: float, f_max: float) -> np.ndarray:
    """m angular relaxation frequencies, log-spaced over [f_min, f_max] Hz."""
    if m == 1:
        return np.array([2 * math.pi * math.sqrt(f_min * f_max)])
    return 2 * math.pi * np.exp(np.linspace(math.log(f_min), math.log(f_max), m))


def qfit(Q: np.ndarray, omega: np.ndarray, f_min: float, f_max: float) -> np.ndarray:
    """Least-squares weights Y_l [K,m] so that a generalised Maxwell body with
    relaxation frequencies omega approximates the frequency-independent quality
    factor Q over [f_min, f_max]:
        1/Q ~= sum_l Y_l (omega_l w + omega_l^2 / Q) / (omega_l^2 + w^2)
    sampled at 2m-1 log-spaced angular frequencies w (normal equations, one
    small system per element, solved in a batch)."""
    Q = np.asarray(Q, dtype=np.float64)
    w = 2 * math.pi * np.exp(np.linspace(math.log(f_min), math.log(f_max), 2 * len(omega) - 1))
    om = omega[None, None, :]
    A = (om * w[None, :, None] + om ** 2 / Q[:, None, None]) / (om ** 2 + w[None, :, None] ** 2)  # [K,n,m]
    b = np.broadcast_to((1.0 / Q)[:, None], (Q.shape[0], w.shape[0]))
    AtA = np.einsum("knl,knj->klj", A, A)
    Atb = np.einsum("knl,kn->kl", A, b)
    return np.linalg.solve(AtA, Atb[..., None])[..., 0]


def attenuation_inputs(mat: dict, m: int, f_min: float, f_max: float) -> dict:
    """omega [m] and the P/S weights Yp, Ys [K,m] for the anelastic solver."""
    omega = relaxation_frequencies(m, f_min, f_max)
    return dict(omega=omega, yp=qfit(mat["qp"], omega, f_min, f_max),
                ys=qfit(mat["qs"], omega, f_min, f_max))


# --------------------------------------------------------------------------- sources/receivers

STF_RICKER = 0   # moment rate (1 - 2a(t-t0)^2) exp(-a(t-t0)^2), a = (pi fc)^2
STF_HANN = 1     # moment rate (1 - cos(2 pi (t-t0)/T)) / T on [t0, t0+T]


def random_moment_tensor(rng, M0: float) -> np.ndarray:
    """Moment tensor (xx,yy,zz,xy,yz,xz) with i.i.d. normal entries scaled to
    scalar moment M0 = sqrt(sum_ij M_ij^2 / 2)."""
    m = rng.normal(size=6)
    full = np.sum(m[:3] ** 2) + 2 * np.sum(m[3:] ** 2)
    return m * (M0 / math.sqrt(full / 2.0))


def ricker_sources(seed: int, n: int, box_xy, depth_range, fc_range=(2.0, 2.0), M0=1e15) -> dict:
    """n moment-tensor point sources with Ricker moment rates.  stf_params
    rows are [fc, t0] with t0 = 1.5/fc."""
    rng = np.random.default_rng(seed)
    (x0, x1), (y0, y1) = box_xy
    xyz = np.stack([rng.uniform(x0, x1, n), rng.uniform(y0, y1, n),
                    -rng.uniform(depth_range[0], depth_range[1], n)], axis=1)
    fc = rng.uniform(fc_range[0], fc_range[1], n)
    moment = np.stack([random_moment_tensor(rng, M0) for _ in range(n)])
    return dict(xyz=xyz, moment=moment, stf_kind=STF_RICKER,
                stf_params=np.stack([fc, 1.5 / fc], axis=1))


def surface_receivers(seed: int, n: int, box_xy, z: float = 0.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    (x0, x1), (y0, y1) = box_xy
    return np.stack([rng.uniform(x0, x1, n), rng.uniform(y0, y1, n), np.full(n, z)], axis=1)


def random_state(seed: int, K: int, nq: int, nb: int, scale_stress=1e6, scale_vel=1.0,
                 scale_mem=1e-3) -> np.ndarray:
    """Random modal DOFs [K, nq, nb] (stresses ~ MPa, velocities ~ m/s)."""
    rng = np.random.default_rng(seed)
    q = rng.normal(size=(K, nq, nb))
    q[:, :6] *= scale_stress
    q[:, 6:9] *= scale_vel
    q[:, 9:] *= scale_mem
    return q


# --------------------------------------------------------------------------- named workloads

def loh_like_box(scale: str = "full", seed: int = 20) -> dict:
    """The layered 20x20x10 km box of the anelastic LTS workload (free surface on
    top, absorbing elsewhere, 67x67 columns, 4x100 m + 3x200 m + 30x300 m layers,
    jitter 15%, K = 996,558).  scale='small' gives a 2x2x1 km box with 100 m
    columns and the same top layering (K = 5,082, for the oracle-sized
    parity tests); scale='tiny' a 1.2 km box with K = 384)."""
    if scale == "full":
        return layered_box(67, 67, [100.0] * 4 + [200.0] * 3 + [300.0] * 30, 20000.0, 20000.0,
                           jitter=0.15, seed=seed)
    if scale == "small":
        return layered_box(11, 11, [100.0] * 4 + [200.0] * 3, 2000.0, 2000.0, jitter=0.15, seed=seed)
    if scale == "tiny":
        return layered_box(4, 4, [100.0] * 2 + [200.0] * 2, 1200.0, 1200.0, jitter=0.15, seed=seed)
    raise ValueError(scale)


def differentiation_box(scale: str = "full", seed: int = 50) -> dict:
    """The 10 x 10 x 5 km layered box of the gradient workload (free surface on
    top, absorbing elsewhere): 41 x 41 columns, layers 4 x 100 m, 3 x 200 m,
    13 x 307.7 m, jitter 10%, K = 201,720.  'small' is the 2 x 2 x 1 km box
    of loh_like_box('small') (K = 5,082) used for the oracle comparison."""
    if scale == "full":
        return layered_box(41, 41, [100.0] * 4 + [200.0] * 3 + [307.7] * 13, 10000.0, 10000.0,
                           jitter=0.10, seed=seed)
    return loh_like_box(scale, seed=seed)


# --------------------------------------------------------------------------- graded basin workload

def graded_box(xs, ys, zs, jitter: float = 0.0, seed: int = 0, top_bc: int = BC_FREE,
               side_bc: int = BC_ABSORB) -> dict:
    """Hex grid with the given (ascending) node coordinates per axis, Kuhn-split;
    zs ascends from the bottom to 0.  Interior vertices are jittered by
    +-jitter of the smaller adjacent spacing per axis; boundary vertices move
    only along their boundary plane(s).  Top face z = max gets top_bc, the
    other five side_bc."""
    rng = np.random.default_rng(seed)
    xs, ys, zs = (np.asarray(a, dtype=np.float64) for a in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1

    def spacing(a):
        d = np.diff(a)
        return np.minimum(np.concatenate([[np.inf], d]), np.concatenate([d, [np.inf]]))

    I, J, Kz = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    P = np.stack([xs[I], ys[J], zs[Kz]], axis=-1)
    if jitter > 0:
        d = rng.uniform(-jitter, jitter, size=P.shape)
        d[..., 0] *= spacing(xs)[I]
        d[..., 1] *= spacing(ys)[J]
        d[..., 2] *= spacing(zs)[Kz]
        d[..., 0][(I == 0) | (I == nx)] = 0.0
        d[..., 1][(J == 0) | (J == ny)] = 0.0
        d[..., 2][(Kz == 0) | (Kz == nz)] = 0.0
        P = P + d
    lat = _hex_grid_tets(nx, ny, nz)
    ids = (lat[..., 0] * (ny + 1) + lat[..., 1]) * (nz + 1) + lat[..., 2]
    xyz = P[lat[..., 0], lat[..., 1], lat[..., 2]]
    bc = {(0, 0): side_bc, (0, 1): side_bc, (1, 0): side_bc, (1, 1): side_bc,
          (2, 0): side_bc, (2, 1): top_bc}
    face_bc = _tag_box_faces(lat, (nx, ny, nz), bc)
    vol = np.einsum("ki,ki->k", np.cross(xyz[:, 1] - xyz[:, 0], xyz[:, 2] - xyz[:, 0]), xyz[:, 3] - xyz[:, 0])
    ref = np.einsum("ki,ki->k", np.cross(lat[:, 1] - lat[:, 0], lat[:, 2] - lat[:, 0]).astype(float),
                    (lat[:, 3] - lat[:, 0]).astype(float))
    if np.any(np.sign(vol) != np.sign(ref)):
        raise ValueError("jitter inverted a tetrahedron; lower it")
    return dict(tet_verts=ids.astype(np.int64), tet_xyz=xyz, face_bc=face_bc,
                box=np.array([[xs[0], xs[-1]], [ys[0], ys[-1]], [zs[0], zs[-1]]]), periodic=False)


def radial_axis(n: int, h: float, s0: float, gmax: float, centred: bool) -> np.ndarray:
    """Node coordinates of a uniform reference axis of n cells of size h mapped
    by x = u min(1 + |u|/s0, gmax): cells grow away from u = 0 (the basin
    centre, or the surface for the depth axis) up to a factor of about gmax."""
    u = (np.arange(n + 1) - (n / 2 if centred else 0)) * h
    return u * np.minimum(1.0 + np.abs(u) / s0, gmax)


BASIN = {
    # grid, reference spacing, grading, basin semi-axes [m]
    "full": dict(n=(138, 138, 69), h=50.0, s0=250.0, gmax=10.0, axes=(8000.0, 6000.0, 2500.0)),
    "small": dict(n=(14, 14, 7), h=50.0, s0=40.0, gmax=10.0, axes=(400.0, 300.0, 120.0)),
}


def basin_box(scale: str = "full", seed: int = 30) -> dict:
    """One GPU's share of a high-frequency basin run: a uniform grid of 50 m
    hexes graded radially about the basin centre at the surface (x = u min(1 +
    |u|/s0, gmax) per axis, depth from the surface likewise), jitter 15%,
    Kuhn-split.  'full': 138 x 138 x 69 cells (69 km x 69 km x 34.5 km),
    K = 7,884,216; 'small': 14 x 14 x 7 cells with steeper grading and a
    smaller basin, K = 8,232 (oracle-sized; both fill all five clusters)."""
    p = BASIN[scale]
    nx, ny, nz = p["n"]
    xs = radial_axis(nx, p["h"], p["s0"], p["gmax"], True)
    ys = radial_axis(ny, p["h"], p["s0"], p["gmax"], True)
    zs = -radial_axis(nz, p["h"], p["s0"], p["gmax"], False)[::-1]
    mesh = graded_box(xs, ys, zs, jitter=0.15, seed=seed)
    mesh["basin_axes"] = np.array(p["axes"])
    return mesh


def basin_materials(mesh: dict, seed: int, sigma: float = 0.025, clip: float = 0.05) -> dict:
    """Background vs(z) = 1500 + 3000 min(depth/12 km, 1)^0.6; inside the
    ellipsoidal basin (semi-axes in mesh['basin_axes'], centred at the surface
    origin) vs = 500 + 1000 e^2 with e the ellipsoidal radius; vp/vs = 2.0 at
    vs = 500 falling linearly to 1.7 at vs = 4500; Gardner density; the
    per-element Gaussian perturbation of the layered model; Qs = 50 vs[km/s],
    Qp = 2 Qs."""
    rng = np.random.default_rng(seed)
    c = centroids(mesh)
    depth = -c[:, 2]
    vs = 1500.0 + 3000.0 * np.minimum(depth / 12000.0, 1.0) ** 0.6
    a = mesh["basin_axes"]
    e = np.sqrt((c[:, 0] / a[0]) ** 2 + (c[:, 1] / a[1]) ** 2 + (depth / a[2]) ** 2)
    inside = e < 1.0
    vs = np.where(inside, 500.0 + 1000.0 * e ** 2, vs)
    ratio = np.clip(2.0 - 0.3 * (vs - 500.0) / 4000.0, 1.7, 2.0)
    d = np.clip(rng.normal(0.0, sigma, len(vs)), -clip, clip)
    vs = vs * (1.0 + d)
    vp = ratio * vs
    qs = 50.0 * vs / 1000.0
    return dict(rho=gardner_rho(vp), vp=vp, vs=vs, qs=qs, qp=2.0 * qs)


def double_couple(strike: float, dip: float, rake: float, M0: float) -> np.ndarray:
    """Moment tensor (xx,yy,zz,xy,yz,xz) of a double couple, x east, y north,
    z up, angles in radians (strike from north, clockwise)."""
    # slip vector and fault normal in (east, north, up)
    n = np.array([-math.sin(dip) * math.cos(strike), math.sin(dip) * math.sin(strike), math.cos(dip)])
    s = np.array([math.cos(rake) * math.sin(strike) - math.sin(rake) * math.cos(dip) * math.cos(strike),
                  math.cos(rake) * math.cos(strike) + math.sin(rake) * math.cos(dip) * math.sin(strike),
                  math.sin(rake) * math.sin(dip)])
    M = M0 * (np.outer(s, n) + np.outer(n, s))
    return np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[1, 2], M[0, 2]])


def kinematic_fault(seed: int, centre, length: float = 10000.0, width: float = 10000.0, n_along: int = 20,
                    n_down: int = 20, mu: float = 3.0e10, vr: float = 2800.0) -> dict:
    """Planar finite source of n_along x n_down double-couple subfaults with
    Hann moment rates: seeded strike, dip and rake; rupture time = distance
    from a seeded hypocentre / vr; rise time U[0.5, 1.5] s; peak slip rate
    U[0.5, 1.5] m/s (slip = peak rate x rise / 2, moment = mu x area x slip).
    stf_params rows are [t0, T] (Hann)."""
    rng = np.random.default_rng(seed)
    strike = rng.uniform(0.0, 2.0 * math.pi)
    dip = rng.uniform(math.radians(45.0), math.radians(85.0))
    rake = rng.uniform(-math.pi, math.pi)
    along = np.array([math.sin(strike), math.cos(strike), 0.0])
    down = np.cross(along, np.array([-math.sin(dip) * math.cos(strike), math.sin(dip) * math.sin(strike),
                                     math.cos(dip)]))
    if down[2] > 0:
        down = -down
    a = (np.arange(n_along) + 0.5) / n_along - 0.5
    b = (np.arange(n_down) + 0.5) / n_down - 0.5
    A, Bd = np.meshgrid(a * length, b * width, indexing="ij")
    xyz = np.asarray(centre)[None, :] + A.reshape(-1, 1) * along[None, :] + Bd.reshape(-1, 1) * down[None, :]
    hypo = xyz[rng.integers(len(xyz))]
    t0 = np.linalg.norm(xyz - hypo, axis=1) / vr
    rise = rng.uniform(0.5, 1.5, len(xyz))
    slip = rng.uniform(0.5, 1.5, len(xyz)) * rise / 2.0
    area = (length / n_along) * (width / n_down)
    moment = np.stack([double_couple(strike, dip, rake, mu * area * s) for s in slip])
    return dict(xyz=xyz, moment=moment, stf_kind=STF_HANN, stf_params=np.stack([t0, rise], axis=1))
