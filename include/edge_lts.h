/*
 * edge_lts.h -- C-ABI of the MI355X (gfx950) ADER-DG solver for the elastic
 * and anelastic wave equations on unstructured tetrahedral meshes, with
 * clustered rate-2 local time stepping.
 *
 * The operations follow Breuer & Heinecke, "Next-Generation Local Time
 * Stepping for the ADER-DG Finite Element Method" (arXiv 2202.10313):
 *   - the PDE and state vector: Sec. III (ADER-DG Finite Element Method), eq. hyp_sys (q = 6 stresses,
 *     3 velocities, 6m memory variables);
 *   - the element update: Sec. III-A (Discrete Formulation) (time kernel eq. ader_taylor with the
 *     Cauchy-Kowalevski recursion, volume and surface kernels, eq. update);
 *   - clusters and lambda: Sec. V-A (Clustering) (interval definition of C_1..C_Nc,
 *     normalisation, lambda search in steps of 0.01);
 *   - buffers and schedule: Sec. V-B (Buffers and Algorithm; eq. lts_buffers and the walk-through
 *     of Fig. lts_scheme).
 * Point sources, receivers, boundary conditions and the Riemann solver are not
 * specified by the paper; the choices made are documented per function.
 *
 * Conventions shared by every call:
 *   - return value 0 on success, a negative EDG_E* code on failure; the
 *     message of the last failure is available from edg_last_error(ctx);
 *     no call aborts the process or throws across the ABI;
 *   - every array argument is a host pointer owned by the caller and is only
 *     read (or written, for outputs) during the call; the library copies
 *     what it keeps.  The calls with an on_device argument take device
 *     pointers instead when it is 1 (FP64 arrays in device memory of the
 *     context's device, in the same layouts): they are read or written on
 *     the context's stream during the call (the caller orders the work that
 *     produces or consumes them with that stream) and the call returns after
 *     that work has completed;
 *   - element data is in the caller's element order and the caller's local
 *     vertex order; internally elements are reordered by cluster and each
 *     tet's vertices are sorted by vertex id, which the library undoes on
 *     every read;
 *   - floating-point inputs and outputs are FP64; the internal arithmetic is
 *     FP32 or FP64 as configured;
 *   - modal coefficients use the orthonormal Dubiner basis on the unit
 *     tetrahedron (0,0,0),(1,0,0),(0,1,0),(0,0,1) of the tet's own vertex
 *     order, ordered by total degree, then i, then j descending; quantity
 *     order sxx,syy,szz,sxy,syz,sxz,u,v,w, then the memory variables of each
 *     mechanism in the same stress-component order.
 */
#ifndef EDGE_LTS_H
#define EDGE_LTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EDG_OK 0
#define EDG_EINVAL -1    /* bad argument (size, range, null where required) */
#define EDG_ESTATE -2    /* call out of order (e.g. advance before clusters) */
#define EDG_ENOMEM -3    /* device or host allocation failed */
#define EDG_EHIP -4      /* a HIP runtime call failed */
#define EDG_ENOTSYNC -5  /* time is not a synchronisation point */
#define EDG_EMESH -6     /* non-conforming mesh, degenerate tet, unmatched face */
#define EDG_ECAP -7      /* output capacity too small */
#define EDG_ENONFINITE -8 /* EDG_FLAG_CHECK_FINITE: a DOF became NaN or infinite during the advance */

#define EDG_BC_INTERIOR 0
#define EDG_BC_FREE 1     /* free surface: zero traction (mirror state) */
#define EDG_BC_ABSORB 2   /* absorbing: no incoming characteristics (zero state) */

#define EDG_STF_RICKER 0  /* moment rate (1-2a(t-t0)^2) exp(-a(t-t0)^2), a=(pi fc)^2; params [fc, t0] */
#define EDG_STF_HANN 1    /* moment rate (1-cos(2 pi (t-t0)/T))/T on [t0,t0+T]; params [t0, T] */

typedef struct edg_ctx edg_ctx;

typedef struct {
  int32_t order;       /* O in 2..5 (B(O) = O(O+1)(O+2)/6 basis functions) */
  int32_t mechanisms;  /* relaxation mechanisms m: 0 (elastic) or 3 */
  int32_t n_runs;      /* independent runs sharing mesh, materials and clusters: 1..32 */
  int32_t n_clusters;  /* N_c in 1..5 */
  int32_t fp64;        /* 1: FP64 state and arithmetic, 0: FP32 */
  double cfl;          /* C in dt_k = C 2 r_k / ((2(O-1)+1) vp_k), r_k the insphere radius */
  double lambda;       /* lambda in (0.5, 1]; <= 0 searches 0.51..1.00 (max speedup, ties -> larger) */
  void* hip_stream;    /* hipStream_t the library launches on (NULL: its own stream) */
  int32_t device;      /* HIP device ordinal */
  uint32_t flags;      /* EDG_FLAG_* (EDG_EINVAL for other bits) */
} edg_config;

#define EDG_FLAG_GRAPH 1u  /* replay every full LTS cycle but the last of an edg_advance_to call as one
                              captured HIP graph (kernel nodes only; recaptured after a change of
                              sources, receivers, clusters or launch plan); edg_adjoint replays the
                              backward levels of its segments as graphs captured once per segment
                              length in that call */
/* Debug aids for the buffer schedule of Sec. V-B (Buffers and Algorithm); none changes a result that
 * is computed from legally read data, so with them on, a correct run gives bit-identical DOFs and
 * seismograms (they cost extra launches, so they are for tests, not production). */
#define EDG_FLAG_POISON 2u        /* after every level that finishes steps, overwrite with NaN each
                                     B1 / B2 / B3 face-trace slot whose last legal read was at that
                                     level, and every slot at the start of each advance: a read of a
                                     stale slot turns the DOFs it reaches into NaN */
#define EDG_FLAG_SHUFFLE 4u       /* run the element groups of every launch in a pseudo-random
                                     order (a fresh affine bijection of the workgroup ids per launch)
                                     instead of the plan's */
#define EDG_FLAG_CHECK_FINITE 8u  /* after every advance, count the NaN / infinite DOF words of all
                                     runs: EDG_ENONFINITE (the message names the count and the first
                                     run and caller element) instead of EDG_OK; the state stays as
                                     advanced */
#define EDG_FLAG_POISON_EARLY 16u /* self-test of EDG_FLAG_POISON: poison, after every finishing
                                     level, the B1 slot its predictions have just written (still to
                                     be read), so that the DOFs do turn into NaN */

/* Launch plan of the element-update kernel.  Every plan but trace_mfma gives
 * bit-identical results; only the speed differs. */
typedef struct {
  int32_t xcd_remap;  /* 1: the workgroups dealt to one XCD take a contiguous range of element
                         groups (neighbour traces then stay in that XCD's L2) */
  int32_t run_chunk;  /* runs per launch (0 = all runs in one launch) */
  int32_t trace_mfma; /* 1: the traces of faces 0 and 1 as one dense product on the matrix cores
                         (two-wave FP32 kernel, orders 4 and 5; elsewhere ignored).  Results
                         agree with the vector-ALU traces to FP32 rounding, not bit for bit. */
} edg_plan;

/* Create a context on cfg->device.  *out receives the handle (NULL on
 * failure; creation errors are returned only as codes). */
int edg_create(const edg_config* cfg, edg_ctx** out);

/* Mesh (Sec. III-A (Discrete Formulation): conforming unstructured tetrahedra).  tet_verts [K][4]:
 * vertex ids, used only to match faces (three shared ids = a shared face;
 * periodic meshes reuse ids across the period); tet_xyz [K][4][3]: the tet's
 * vertex coordinates in the same local order; face_bc [K][4]: EDG_BC_* per
 * local face i (the face opposite local vertex i), NULL = all interior.
 * EDG_EMESH if a face is shared by more than two tets, an unmatched face is
 * tagged interior, a matched face carries a boundary tag, a tet repeats a
 * vertex id or is degenerate. */
int edg_upload_mesh(edg_ctx* ctx, int64_t n_tets, const int64_t* tet_verts, const double* tet_xyz,
                    const int8_t* face_bc);

/* Materials per element (Sec. III (ADER-DG Finite Element Method), eq.
 * hyp_sys, whose Jacobians and anelastic source the paper takes from its
 * references): density rho [kg/m^3], unrelaxed P and S speeds vp, vs [m/s]
 * (rho > 0, vs > 0, vp > sqrt(4/3) vs, else EDG_EINVAL and nothing changes);
 * for m > 0, the relaxation frequencies omega [m] (rad/s, shared by all
 * elements) and the P/S weights yp, ys [K][m] of the generalised Maxwell body
 * (stress relaxes by -sum_l (a_l tr(theta^l) I + b_l theta^l),
 * a_l = (lambda+2mu) Yp_l - 2mu Ys_l, b_l = 2mu Ys_l; the memory variables
 * obey d/dt theta^l = omega_l (sym grad v - theta^l)).  The weights are
 * inputs, not quality factors: a constant-Q fit (Qp, Qs over a band) is the
 * caller's, so that both sides of a comparison use the same weights.
 * on_device = 1: all six arrays are device pointers; the range check and the
 * per-element tables are then computed on the device (no host copy of the
 * arrays unless a later edg_upload_clusters needs one).  After
 * edg_upload_clusters a re-upload re-derives the operators but keeps the
 * clusters, time steps and state (what a gradient check needs). */
int edg_upload_materials(edg_ctx* ctx, const double* rho, const double* vp, const double* vs,
                         const double* omega, const double* yp, const double* ys, int32_t on_device);

/* Time clusters (Sec. V-A (Clustering)).  cluster: [K] values 1..N_c in the caller's
 * element order (used as given; EDG_EINVAL if two face neighbours differ by
 * more than one), or NULL to derive them from the CFL steps, the interval
 * rule, normalisation and the lambda of the configuration.  Allocates the
 * device state of all n_runs runs (per run: the DOFs, B1 of every element,
 * B2 / B3 of the elements with a finer / coarser neighbour, each twice for
 * the step parity); the DOFs start at zero, the time at 0, and earlier
 * sources and receivers are dropped. */
int edg_upload_clusters(edg_ctx* ctx, const int32_t* cluster);

/* Derived clustering: cluster_out [K] (may be NULL), dt_min (smallest CFL
 * step), lambda, sync_dt (step of the coarsest cluster: the times
 * edg_advance_to accepts are its multiples) and the theoretical speedup over
 * global time stepping K / sum_l n_l / (2^(l-1) lambda).  Any pointer may be NULL. */
int edg_get_clusters(const edg_ctx* ctx, int32_t* cluster_out, double* dt_min, double* lambda,
                     double* sync_dt, double* speedup);

/* Modal DOFs [K][Nq][B] of run `run` (0..n_runs-1) at the current time.  Only
 * at a synchronisation point (always true between calls). */
int edg_set_initial(edg_ctx* ctx, int32_t run, const double* dofs);

/* DOFs of selected elements of run `run`: ids [n] caller element indices
 * (0..K-1; EDG_EINVAL otherwise), dofs / out [n][Nq][B] in the caller's vertex
 * order; cap = doubles available in out.  Only the 7-element groups holding
 * the elements are transferred, so a few elements of a large mesh are cheap to
 * set or probe; other elements keep their values.  Repeated ids: the last one
 * wins when setting. */
int edg_set_dofs_subset(edg_ctx* ctx, int32_t run, int64_t n, const int64_t* ids, const double* dofs);
int edg_read_dofs_subset(edg_ctx* ctx, int32_t run, int64_t n, const int64_t* ids, double* out, int64_t cap);

/* Moment-tensor point sources of run `run` (0..n_runs-1): xyz [n][3], moment
 * [n][6] (xx,yy,zz,xy,yz,xz, N m), stf_params [n][2] (see EDG_STF_*).  Each
 * source adds -M phi(x_s)/|det J| times the exact integral of its moment rate
 * over each step of the element that contains it (lowest element index on
 * ties); EDG_EINVAL if a point is outside the mesh.  Replaces the earlier
 * sources of that run only. */
int edg_set_sources(edg_ctx* ctx, int32_t run, int64_t n, const double* xyz, const double* moment,
                    int32_t stf_kind, const double* stf_params);

/* Receivers at xyz [n][3], the same for every run, sampling the 9 elastic
 * quantities every dt_sample from t = 0 (n_samples samples); each sample comes
 * from the Taylor expansion of the covering element's prediction for the step
 * that contains the sample time.  Clears the recorded samples of all runs. */
int edg_set_receivers(edg_ctx* ctx, int64_t n, const double* xyz, double dt_sample, int64_t n_samples);

/* Advance every element of every run to time t (a multiple of sync_dt, not
 * earlier than the current time; EDG_ENOTSYNC otherwise).  Each LTS level is
 * one launch for all runs (grid = element groups x runs).  Runs on the
 * context's stream and returns after the work has completed. */
int edg_advance_to(edg_ctx* ctx, double t);

/* ---- allocation-free advance ----------------------------------------------
 * For callers that cannot allocate device memory while they advance: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same as edg_advance_to, except that the B1 / B2 / B3 face
 * traces, which one advance from a synchronisation point writes before it
 * reads them, live in a static device array of EDG_STATIC_SCRATCH_BYTES per
 * GPU (held from the first call on that GPU until the process ends) instead
 * of the context's own buffers.  The call allocates nothing: no hipMalloc or
 * hipFree, no graph instantiation, no event creation; every level launches
 * eagerly (EDG_FLAG_GRAPH and timing do not apply).  The array is zeroed by a
 * fill kernel at the start of each call.  DOFs, seismograms and the element
 * update count are bit-identical to edg_advance_to.
 * Errors: EDG_EINVAL if the context's traces, n_runs x (T1 + T2 + T3 words)
 * x word bytes, exceed EDG_STATIC_SCRATCH_BYTES (the message gives both
 * sizes; about 44,000 elements at O = 5, FP32, one run); EDG_ESTATE before
 * edg_upload_clusters or with checkpointing on; EDG_ENOTSYNC as
 * edg_advance_to.  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (two threads, two contexts) race. */
#define EDG_STATIC_SCRATCH_BYTES (256ull << 20)
int edg_advance_to_static(edg_ctx* ctx, double t);

/* Recorded seismograms of run `run` (0..n_runs-1): out [n_rec][n_samples][9];
 * cap = number of doubles available (EDG_ECAP if smaller); on_device = 1:
 * out is a device pointer. */
int edg_read_receivers(edg_ctx* ctx, int32_t run, double* out, int64_t cap, int32_t on_device);

/* DOFs [K][Nq][B] of run `run` (0..n_runs-1) at the current time; cap = doubles
 * available. */
int edg_read_dofs(edg_ctx* ctx, int32_t run, double* out, int64_t cap);

/* Current simulation time (0 for a NULL context). */
double edg_time(const edg_ctx* ctx);

/* Message of the last failed call on ctx ("" if none; a static string for NULL). */
const char* edg_last_error(const edg_ctx* ctx);

/* Per-launch timing of the element-update kernel (HIP events on the
 * context's stream): enable != 0 starts recording; edg_kernel_stats returns
 * the number of timed launches, their total time [ms] and the number of
 * element updates they performed.  Timing adds a synchronisation per launch. */
int edg_enable_timing(edg_ctx* ctx, int32_t enable);
int edg_kernel_stats(const edg_ctx* ctx, int64_t* launches, double* total_ms, int64_t* element_updates);

/* Element updates (element x own step x run) performed so far. */
int64_t edg_element_updates(const edg_ctx* ctx);

/* Set / get the launch plan (default {0, 0}).  EDG_EINVAL for values out of
 * range. */
int edg_set_plan(edg_ctx* ctx, const edg_plan* plan);
int edg_get_plan(const edg_ctx* ctx, edg_plan* plan);

/* Autotuner: advances the simulation by `cycles` LTS cycles per candidate plan
 * (XCD remap on/off x runs per launch: all, 16, 8, 4), timing the element
 * kernel of each, and keeps the fastest.  The simulated time moves on by
 * (number of candidates) x cycles x sync_dt; the results are the same as with
 * any other plan.  best / ms_per_cycle (kernel time of the best candidate)
 * may be NULL.  The tuning cycles are left out of edg_kernel_stats. */
int edg_autotune(edg_ctx* ctx, int32_t cycles, edg_plan* best, double* ms_per_cycle);

/* ---- discrete adjoint -------------------------------------------------------
 * The paper names inversion for seismic velocities as a use of such solvers
 * (Sec. II (Related Work)) without an adjoint; these calls give the exact transpose of
 * the discrete LTS scheme of Sec. III-A (Discrete Formulation) and Sec. V-B
 * (Buffers and Algorithm) as this library computes it, for gradients of
 * receiver misfits with respect to per-element rho, vp and vs.  Time steps,
 * clusters, omega and the anelastic weights Yp, Ys are held fixed.  With
 * n_runs > 1 the misfit is the sum of the runs' misfits (the runs share the
 * materials, as the shots of one inversion do). */

/* every_cycles > 0: from now on edg_advance_to splits its cycles into
 * segments of at most every_cycles cycles and stores the state (device
 * memory, n_runs x K x Nq x B words each) at the start of every segment; 0
 * turns it off.  The buffers of dropped checkpoints stay allocated for the
 * next ones until edg_upload_clusters or edg_destroy.  With one run the final segment of each edg_advance_to call
 * also records, at every level, the state of the elements that start a step
 * there (device memory, reused by edg_adjoint; the forward kernels write
 * it; with several runs the reverse sweep replays that segment too): per LTS cycle
 * (element updates of the cycle) x Nq x B words, 1.9 x K x Nq x B at the
 * benchmark's three cluster sizes; an interval whose record does not fit fails
 * with EDG_ENOMEM naming the bytes it needs.  The segment runs without graph
 * replay; its launches are not counted by the timing queries.  Drops stored checkpoints.  EDG_EINVAL for a
 * negative interval.  The checkpoints are dropped again by edg_set_initial,
 * edg_set_dofs_subset, edg_upload_materials, edg_upload_clusters,
 * edg_set_sources and edg_rewind. */
int edg_set_checkpointing(edg_ctx* ctx, int32_t every_cycles);

/* Back to t = 0: DOFs, buffers and recorded seismograms are zeroed;
 * materials, clusters, time steps, sources and receivers stay.  With
 * edg_upload_materials (which keeps clusters and time steps) this re-runs a
 * simulation for perturbed materials. */
int edg_rewind(edg_ctx* ctx);

/* Reverse sweep over the advance since the first checkpoint: with the
 * derivative of a scalar misfit J with respect to the recorded seismogram
 * samples, dj_dseis [n_runs][n_rec][n_samples][9] (the layout of
 * edg_read_receivers per run; NULL = 0), and with respect to the current
 * DOFs, dj_dq [n_runs][K][Nq][B] (caller order; NULL = 0), writes dJ/d(DOFs
 * at the first checkpoint) to g_q0 [n_runs][K][Nq][B] and dJ/d rho, dJ/d vp,
 * dJ/d vs [K] (sums over the runs) to g_rho, g_vp, g_vs (any may be NULL).
 * The runs are swept one after the other.  Segments run backwards; each needs the states at the start of
 * every level ((levels per segment) x K x Nq x B words of device memory):
 * with one run, the segment the last edg_advance_to call recorded uses them
 * as they are, every other one is first replayed forward from its
 * checkpoint.  Then its levels run backwards through the adjoint kernels.
 * With one run, a checkpoint interval that covers the whole advance
 * therefore needs no replay at all.  All host arrays are caller-owned and only read or written
 * during the call; the DOFs and the time are those of before the call when it
 * returns.  EDG_ESTATE without checkpoints.  on_device = 1:
 * all six arrays are device pointers; dj_dseis is copied and the gradients
 * are scattered to caller order on the device, while dj_dq and g_q0 (DOF
 * layout conversions done by the host) are staged through host memory. */
int edg_adjoint(edg_ctx* ctx, const double* dj_dseis, const double* dj_dq, double* g_q0, double* g_rho,
                double* g_vp, double* g_vs, int32_t on_device);

/* Destroy the context and free its device memory (NULL is ignored). */
void edg_destroy(edg_ctx* ctx);

/* ---- host-only helpers (no device work; for tests and tools) ---------------- */

/* Reference matrices of the library's basis (Sec. III-A (Discrete Formulation)): K [3][B][B] with
 * K[c][b][bb] = int phi_b d(phi_bb)/d xi_c and Ft [4][B][F] with
 * Ft[i][b][f] = int_{face i} phi_b psi_f over the unit triangle, face i
 * opposite local vertex i parameterised by its vertices in ascending order. */
int edg_reference_matrices(int32_t order, double* K, double* Ft);

/* Clustering of Sec. V-A (Clustering) on host data: dt [K] CFL steps, nbr [K][4] face
 * neighbours (-1 = none); writes cluster [K] (1..N_c), lambda and speedup.
 * lambda_in <= 0 searches. */
int edg_cluster_host(int64_t K, const double* dt, const int64_t* nbr, int32_t n_clusters,
                     double lambda_in, int32_t* cluster, double* lambda_out, double* speedup_out);

/* The Godunov face flux of one face mode and its reverse mode (FP64 on the
 * host), as the kernels evaluate them: bc 0 interior, 1 free surface, 2
 * absorbing; qm, qp [9] inside / outside traces; prm = (nx, ny, nz, Zp-, Zs-,
 * Zp+, Zs+, lam, mu, 1/rho, s) with s = 2|S_i| / |det J|; writes out [15]
 * (9 elastic rows, 6 strain-rate rows of the memory variables, unscaled by
 * omega), and for the output adjoint u [15]: qm_b, qp_b [9] (transposed
 * flux maps) and pb [7] (derivatives of u . out in 1/rho, lam, mu, Zp-,
 * Zs-, Zp+, Zs+).  Returns -1 for bad arguments. */
int edg_godunov_host(int32_t bc, const double* qm, const double* qp, const double* prm, const double* u,
                     double* out, double* qm_b, double* qp_b, double* pb);

#ifdef __cplusplus
}
#endif
#endif
