"""ctypes binding of the C-ABI in include/edge_lts.h.

Argument marshalling only: every step of the solver runs in libedge_lts.so
(host C++ and HIP kernels for gfx950).  Loading fails loudly when the library
has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("EDG_LIBRARY") or os.path.join(HERE, "lib", "libedge_lts.so")

EDG_OK = 0
STATIC_SCRATCH_BYTES = 256 << 20   # EDG_STATIC_SCRATCH_BYTES
ERRORS = {-1: "EDG_EINVAL", -2: "EDG_ESTATE", -3: "EDG_ENOMEM", -4: "EDG_EHIP",
          -5: "EDG_ENOTSYNC", -6: "EDG_EMESH", -7: "EDG_ECAP", -8: "EDG_ENONFINITE"}
BC_INTERIOR, BC_FREE, BC_ABSORB = 0, 1, 2
STF_RICKER, STF_HANN = 0, 1
FLAG_GRAPH = 1
# debug aids (edge_lts.h): NaN poisoning of dead trace slots, shuffled
# workgroup order, finite check after each advance, poisoner self-test
FLAG_POISON, FLAG_SHUFFLE, FLAG_CHECK_FINITE, FLAG_POISON_EARLY = 2, 4, 8, 16

# every symbol the header declares (checked by the CPU test-suite)
EXPORTS = ["edg_create", "edg_upload_mesh", "edg_upload_materials", "edg_upload_clusters",
           "edg_get_clusters", "edg_set_initial", "edg_set_dofs_subset", "edg_read_dofs_subset", "edg_set_sources", "edg_set_receivers",
           "edg_advance_to", "edg_advance_to_static", "edg_read_receivers", "edg_read_dofs", "edg_time", "edg_last_error",
           "edg_enable_timing", "edg_kernel_stats", "edg_element_updates", "edg_set_plan", "edg_get_plan",
           "edg_autotune", "edg_set_checkpointing", "edg_rewind", "edg_adjoint", "edg_destroy",
           "edg_reference_matrices", "edg_cluster_host", "edg_godunov_host"]


class EdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Plan(ctypes.Structure):
    _fields_ = [("xcd_remap", ctypes.c_int32), ("run_chunk", ctypes.c_int32), ("trace_mfma", ctypes.c_int32)]

    def as_dict(self):
        return dict(xcd_remap=self.xcd_remap, run_chunk=self.run_chunk, trace_mfma=self.trace_mfma)


class Config(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("mechanisms", ctypes.c_int32), ("n_runs", ctypes.c_int32),
                ("n_clusters", ctypes.c_int32), ("fp64", ctypes.c_int32), ("cfl", ctypes.c_double),
                ("lam", ctypes.c_double), ("hip_stream", ctypes.c_void_p), ("device", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


def lib():
    """The loaded libedge_lts.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "edg_create": (ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(_P)]),
            "edg_upload_mesh": (ctypes.c_int, [_P, _I64, _P, _P, _P]),
            "edg_upload_materials": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _I32]),
            "edg_upload_clusters": (ctypes.c_int, [_P, _P]),
            "edg_get_clusters": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
            "edg_set_initial": (ctypes.c_int, [_P, _I32, _P]),
            "edg_set_dofs_subset": (ctypes.c_int, [_P, _I32, _I64, _P, _P]),
            "edg_read_dofs_subset": (ctypes.c_int, [_P, _I32, _I64, _P, _P, _I64]),
            "edg_set_sources": (ctypes.c_int, [_P, _I32, _I64, _P, _P, _I32, _P]),
            "edg_set_receivers": (ctypes.c_int, [_P, _I64, _P, ctypes.c_double, _I64]),
            "edg_advance_to": (ctypes.c_int, [_P, ctypes.c_double]),
            "edg_advance_to_static": (ctypes.c_int, [_P, ctypes.c_double]),
            "edg_read_receivers": (ctypes.c_int, [_P, _I32, _P, _I64, _I32]),
            "edg_read_dofs": (ctypes.c_int, [_P, _I32, _P, _I64]),
            "edg_time": (ctypes.c_double, [_P]),
            "edg_last_error": (ctypes.c_char_p, [_P]),
            "edg_enable_timing": (ctypes.c_int, [_P, _I32]),
            "edg_kernel_stats": (ctypes.c_int, [_P, _P, _P, _P]),
            "edg_element_updates": (ctypes.c_int64, [_P]),
            "edg_set_plan": (ctypes.c_int, [_P, _P]),
            "edg_get_plan": (ctypes.c_int, [_P, _P]),
            "edg_autotune": (ctypes.c_int, [_P, _I32, _P, _P]),
            "edg_set_checkpointing": (ctypes.c_int, [_P, _I32]),
            "edg_rewind": (ctypes.c_int, [_P]),
            "edg_adjoint": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _I32]),
            "edg_destroy": (None, [_P]),
            "edg_reference_matrices": (ctypes.c_int, [_I32, _P, _P]),
            "edg_cluster_host": (ctypes.c_int, [_I64, _P, _P, _I32, ctypes.c_double, _P, _P, _P]),
            "edg_godunov_host": (ctypes.c_int, [_I32, _P, _P, _P, _P, _P, _P, _P, _P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _is_device(a):
    return getattr(a, "is_cuda", False)


def _dev_ptr(t):
    """Device pointer of a contiguous float64 CUDA tensor (no copy)."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("device arrays must be contiguous float64 CUDA tensors")
    return ctypes.c_void_p(t.data_ptr())


def n_basis(order):
    return order * (order + 1) * (order + 2) // 6


def n_face_basis(order):
    return order * (order + 1) // 2


class Context:
    """One solver context (edg_ctx): mesh, materials, clusters, state, sources
    and receivers of one device stream."""

    def __init__(self, order, mechanisms=0, n_clusters=1, fp64=False, cfl=0.5, lam=1.0,
                 stream=None, device=0, n_runs=1, flags=0):
        self._L = lib()
        cfg = Config(order, mechanisms, n_runs, n_clusters, int(bool(fp64)), float(cfl),
                     -1.0 if lam is None else float(lam), stream, device, int(flags))
        h = _P()
        rc = self._L.edg_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != EDG_OK:
            raise EdgError(rc, "edg_create failed")
        self.h = h
        self.order, self.m, self.n_runs = order, mechanisms, int(n_runs)
        self.B, self.nq = n_basis(order), 9 + 6 * mechanisms
        self.K = 0
        self.n_rec = 0
        self.n_samples = 0

    def _chk(self, rc):
        if rc != EDG_OK:
            raise EdgError(rc, self._L.edg_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self._L.edg_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # --- setup
    def upload_mesh(self, tet_verts, tet_xyz, face_bc=None):
        tv = np.ascontiguousarray(tet_verts, dtype=np.int64)
        xyz = _f64(tet_xyz)
        bc = None if face_bc is None else np.ascontiguousarray(face_bc, dtype=np.int8)
        self.K = tv.shape[0]
        self._chk(self._L.edg_upload_mesh(self.h, self.K, _ptr(tv), _ptr(xyz), _ptr(bc)))

    def upload_materials(self, rho, vp, vs, omega=None, yp=None, ys=None):
        """Host arrays, or CUDA tensors (then every array is read from device
        memory: on_device = 1; omega, yp, ys given on the host are moved to
        rho's device first)."""
        if _is_device(rho):
            import torch
            dev = rho.device
            arrs = [a if a is None or _is_device(a) else torch.as_tensor(np.asarray(a, dtype=np.float64), device=dev)
                    for a in (rho, vp, vs, omega, yp, ys)]
            arrs = [None if a is None else a.to(torch.float64).contiguous() for a in arrs]
            self._keep = arrs                # alive until the call returns
            self._chk(self._L.edg_upload_materials(self.h, *[None if a is None else _dev_ptr(a) for a in arrs], 1))
            return
        arrs = [_f64(a) for a in (rho, vp, vs, omega, yp, ys)]
        self._chk(self._L.edg_upload_materials(self.h, *[_ptr(a) for a in arrs], 0))

    def upload_clusters(self, clusters=None):
        cl = None if clusters is None else np.ascontiguousarray(clusters, dtype=np.int32)
        self._chk(self._L.edg_upload_clusters(self.h, _ptr(cl)))

    def get_clusters(self):
        cl = np.empty(self.K, dtype=np.int32)
        vals = [ctypes.c_double() for _ in range(4)]
        self._chk(self._L.edg_get_clusters(self.h, _ptr(cl), *[ctypes.byref(v) for v in vals]))
        dt_min, lam, sync_dt, speedup = (v.value for v in vals)
        return dict(clusters=cl, dt_min=dt_min, lam=lam, sync_dt=sync_dt, speedup=speedup)

    def set_initial(self, dofs, run=0):
        d = _f64(dofs, (self.K, self.nq, self.B))
        self._chk(self._L.edg_set_initial(self.h, run, _ptr(d)))

    def set_dofs_subset(self, ids, dofs, run=0):
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        d = _f64(dofs, (len(ids), self.nq, self.B))
        self._chk(self._L.edg_set_dofs_subset(self.h, run, len(ids), _ptr(ids), _ptr(d)))

    def read_dofs_subset(self, ids, run=0):
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        out = np.empty((len(ids), self.nq, self.B))
        self._chk(self._L.edg_read_dofs_subset(self.h, run, len(ids), _ptr(ids), _ptr(out), out.size))
        return out

    def set_sources(self, xyz, moment, stf_kind, stf_params, run=0):
        xyz = _f64(xyz).reshape(-1, 3)
        n = xyz.shape[0]
        mom = _f64(moment, (n, 6))
        par = _f64(stf_params, (n, 2))
        self._chk(self._L.edg_set_sources(self.h, run, n, _ptr(xyz), _ptr(mom), int(stf_kind), _ptr(par)))

    def set_receivers(self, xyz, dt_sample, n_samples):
        xyz = _f64(xyz).reshape(-1, 3)
        self.n_rec, self.n_samples = xyz.shape[0], int(n_samples)
        self._chk(self._L.edg_set_receivers(self.h, self.n_rec, _ptr(xyz), float(dt_sample), int(n_samples)))

    # --- stepping and output
    def advance_to(self, t):
        self._chk(self._L.edg_advance_to(self.h, float(t)))

    def advance_to_static(self, t):
        """edg_advance_to with the face traces in the library's static device
        array: the call allocates nothing."""
        self._chk(self._L.edg_advance_to_static(self.h, float(t)))

    def read_dofs(self, run=0):
        out = np.empty((self.K, self.nq, self.B))
        self._chk(self._L.edg_read_dofs(self.h, run, _ptr(out), out.size))
        return out

    def read_receivers(self, run=0):
        out = np.zeros((self.n_rec, self.n_samples, 9))
        self._chk(self._L.edg_read_receivers(self.h, run, _ptr(out), out.size, 0))
        return out

    def read_receivers_device(self, device, run=0):
        """Seismograms as a float64 tensor on `device` (device-to-device copy)."""
        import torch
        out = torch.zeros((self.n_rec, self.n_samples, 9), dtype=torch.float64, device=device)
        self._chk(self._L.edg_read_receivers(self.h, run, _dev_ptr(out), out.numel(), 1))
        return out

    def time(self):
        return self._L.edg_time(self.h)

    def enable_timing(self, on=True):
        self._chk(self._L.edg_enable_timing(self.h, int(bool(on))))

    def kernel_stats(self):
        n, u = ctypes.c_int64(), ctypes.c_int64()
        ms = ctypes.c_double()
        self._chk(self._L.edg_kernel_stats(self.h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(u)))
        return dict(launches=n.value, total_ms=ms.value, element_updates=u.value)

    def element_updates(self):
        return self._L.edg_element_updates(self.h)

    def set_plan(self, xcd_remap=0, run_chunk=0, trace_mfma=0):
        pl = Plan(int(xcd_remap), int(run_chunk), int(trace_mfma))
        self._chk(self._L.edg_set_plan(self.h, ctypes.byref(pl)))

    def get_plan(self):
        pl = Plan()
        self._chk(self._L.edg_get_plan(self.h, ctypes.byref(pl)))
        return pl.as_dict()

    # --- discrete adjoint
    def set_checkpointing(self, every_cycles):
        self._chk(self._L.edg_set_checkpointing(self.h, int(every_cycles)))

    def rewind(self):
        self._chk(self._L.edg_rewind(self.h))

    def adjoint(self, dj_dseis=None, dj_dq=None, want_q0=True):
        """Reverse sweep since the first checkpoint: returns dict(q0_b, g_rho,
        g_vp, g_vs) for the given misfit derivatives (None = 0).  With n_runs
        > 1 the misfit is the sum over the runs: dj_dseis [runs, n_rec,
        n_samples, 9], dj_dq and q0_b [runs, K, Nq, B]; the material
        gradients are the sums over the runs."""
        R = (self.n_runs,) if self.n_runs > 1 else ()
        sb = None if dj_dseis is None else _f64(dj_dseis, R + (self.n_rec, self.n_samples, 9))
        qb = None if dj_dq is None else _f64(dj_dq, R + (self.K, self.nq, self.B))
        q0 = np.empty(R + (self.K, self.nq, self.B)) if want_q0 else None
        g = [np.empty(self.K) for _ in range(3)]
        self._chk(self._L.edg_adjoint(self.h, _ptr(sb), _ptr(qb), _ptr(q0), *[_ptr(a) for a in g], 0))
        return dict(q0_b=q0, g_rho=g[0], g_vp=g[1], g_vs=g[2])

    def adjoint_device(self, dj_dseis, dj_dq=None, want_q0=False):
        """edg_adjoint on device tensors (on_device = 1): dj_dseis [n_rec,
        n_samples, 9] and dj_dq [K, Nq, B] CUDA float64 tensors (or None;
        with a leading run axis when n_runs > 1); returns dict(q0_b, g_rho,
        g_vp, g_vs) as tensors on the same device."""
        import torch
        dev = dj_dseis.device
        R = (self.n_runs,) if self.n_runs > 1 else ()
        sb = dj_dseis.to(torch.float64).contiguous().reshape(R + (self.n_rec, self.n_samples, 9))
        qb = None if dj_dq is None else dj_dq.to(torch.float64).contiguous().reshape(R + (self.K, self.nq, self.B))
        q0 = torch.empty(R + (self.K, self.nq, self.B), dtype=torch.float64, device=dev) if want_q0 else None
        g = [torch.empty(self.K, dtype=torch.float64, device=dev) for _ in range(3)]
        self._chk(self._L.edg_adjoint(self.h, _dev_ptr(sb), None if qb is None else _dev_ptr(qb),
                                      None if q0 is None else _dev_ptr(q0), *[_dev_ptr(a) for a in g], 1))
        return dict(q0_b=q0, g_rho=g[0], g_vp=g[1], g_vs=g[2])

    def autotune(self, cycles=1):
        """Advance `cycles` LTS cycles per candidate plan and keep the fastest;
        returns (plan, kernel ms per cycle of that plan)."""
        pl = Plan()
        ms = ctypes.c_double()
        self._chk(self._L.edg_autotune(self.h, int(cycles), ctypes.byref(pl), ctypes.byref(ms)))
        return pl.as_dict(), ms.value


def godunov_host(bc, qm, qp, prm, u):
    """Face flux of one mode and its reverse mode (host FP64): returns
    (out [15], qm_b [9], qp_b [9], pb [7])."""
    qm, qp, prm, u = _f64(qm), _f64(qp), _f64(prm), _f64(u)
    out, qmb, qpb, pb = np.empty(15), np.empty(9), np.empty(9), np.empty(7)
    rc = lib().edg_godunov_host(int(bc), _ptr(qm), _ptr(qp), _ptr(prm), _ptr(u), _ptr(out), _ptr(qmb), _ptr(qpb),
                                _ptr(pb))
    if rc != EDG_OK:
        raise EdgError(rc, "edg_godunov_host")
    return out, qmb, qpb, pb


def reference_matrices(order):
    B, F = n_basis(order), n_face_basis(order)
    K = np.empty((3, B, B))
    Ft = np.empty((4, B, F))
    rc = lib().edg_reference_matrices(order, _ptr(K), _ptr(Ft))
    if rc != EDG_OK:
        raise EdgError(rc, "edg_reference_matrices")
    return K, Ft


def cluster_host(dt, nbr, n_clusters, lam=None):
    dt = _f64(dt)
    nbr = np.ascontiguousarray(nbr, dtype=np.int64)
    cl = np.empty(len(dt), dtype=np.int32)
    lo, sp = ctypes.c_double(), ctypes.c_double()
    rc = lib().edg_cluster_host(len(dt), _ptr(dt), _ptr(nbr), n_clusters, -1.0 if lam is None else float(lam),
                                _ptr(cl), ctypes.byref(lo), ctypes.byref(sp))
    if rc != EDG_OK:
        raise EdgError(rc, "edg_cluster_host")
    return cl, lo.value, sp.value
