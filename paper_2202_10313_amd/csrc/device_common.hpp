// Device helpers shared by the forward and adjoint kernels (internal):
// the lane mapping constants, the level clock, the workgroup -> (element
// group, run) map and the Godunov flux of one face mode.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace edg {

namespace {

constexpr int EPW = 7;   // elements per wave
constexpr int LPE = 9;   // lanes per element
constexpr int NSLOT = EPW * LPE;  // 63 elastic slots per mode in the tiled layout

__device__ __forceinline__ int sym_index(int i, int j) {
  // (0,0)->0 (1,1)->1 (2,2)->2 (0,1)->3 (1,2)->4 (0,2)->5
  if (i == j) return i;
  const int a = i < j ? i : j, b = i < j ? j : i;
  return a == 0 ? (b == 1 ? 3 : 5) : 4;
}

// A 9 x 3 table of small ints (< 32) packed 5 bits per row into one 64-bit
// word per column: looking up a lane-dependent row is then a shift, not a
// load from constant memory (which would cost a memory round trip).
constexpr unsigned long long pack_rows5(const int (&T)[9][3], int col) {
  unsigned long long w = 0;
  for (int r = 0; r < 9; ++r) w |= (unsigned long long)T[r][col] << (5 * r);
  return w;
}

__device__ __forceinline__ int cluster_of(const LevelArgs& a, int elem) {
  int c = 0;
#pragma unroll
  for (int l = 0; l < MAX_CLUSTERS - 1; ++l)
    if (l < a.n_clusters - 1 && elem >= a.cl_end[l]) c = l + 1;
  return c;
}

// Godunov flux of one face mode: qm / qp are the 9 elastic trace coefficients
// of this element and of the outside state; writes s * (A_n q*) for the 9
// elastic rows and s * (strain-rate flux) for the 6 memory-variable rows
// (unscaled by omega), where s = 2|S_i| / |det J| (the surface kernel's
// -(1/|det J|) int_face phi ... with the sign folded in).
template <class R>
__host__ __device__ __forceinline__ void godunov(const R* qm, const R* qp, R nx, R ny, R nz, R zpm, R zsm, R zpp, R zsp,
                                        R lam, R mu, R rho_inv, R s, int bc, R* out) {
  // tractions sigma n and velocities
  const R tmx = qm[0] * nx + qm[3] * ny + qm[5] * nz;
  const R tmy = qm[3] * nx + qm[1] * ny + qm[4] * nz;
  const R tmz = qm[5] * nx + qm[4] * ny + qm[2] * nz;
  const R vmx = qm[6], vmy = qm[7], vmz = qm[8];
  R tpx, tpy, tpz, vpx, vpy, vpz;
  if (bc == 0) {
    tpx = qp[0] * nx + qp[3] * ny + qp[5] * nz;
    tpy = qp[3] * nx + qp[1] * ny + qp[4] * nz;
    tpz = qp[5] * nx + qp[4] * ny + qp[2] * nz;
    vpx = qp[6]; vpy = qp[7]; vpz = qp[8];
  } else if (bc == 1) {  // free surface: mirror state (traction flips, velocity kept)
    tpx = -tmx; tpy = -tmy; tpz = -tmz;
    vpx = vmx; vpy = vmy; vpz = vmz;
  } else {               // absorbing: zero outside state
    tpx = tpy = tpz = R(0);
    vpx = vpy = vpz = R(0);
  }
  const R tnm = tmx * nx + tmy * ny + tmz * nz, vnm = vmx * nx + vmy * ny + vmz * nz;
  const R tnp = tpx * nx + tpy * ny + tpz * nz, vnp = vpx * nx + vpy * ny + vpz * nz;
  const R ip = R(1) / (zpm + zpp), is = R(1) / (zsm + zsp);
  const R vn = (zpm * vnm + zpp * vnp + tnp - tnm) * ip;
  const R tn = (zpp * tnm + zpm * tnp + zpm * zpp * (vnp - vnm)) * ip;
  // tangential parts
  const R tTmx = tmx - tnm * nx, tTmy = tmy - tnm * ny, tTmz = tmz - tnm * nz;
  const R vTmx = vmx - vnm * nx, vTmy = vmy - vnm * ny, vTmz = vmz - vnm * nz;
  const R tTpx = tpx - tnp * nx, tTpy = tpy - tnp * ny, tTpz = tpz - tnp * nz;
  const R vTpx = vpx - vnp * nx, vTpy = vpy - vnp * ny, vTpz = vpz - vnp * nz;
  const R zz = zsm * zsp;
  const R vx = vn * nx + (zsm * vTmx + zsp * vTpx + tTpx - tTmx) * is;
  const R vy = vn * ny + (zsm * vTmy + zsp * vTpy + tTpy - tTmy) * is;
  const R vz = vn * nz + (zsm * vTmz + zsp * vTpz + tTpz - tTmz) * is;
  const R tx = tn * nx + (zsp * tTmx + zsm * tTpx + zz * (vTpx - vTmx)) * is;
  const R ty = tn * ny + (zsp * tTmy + zsm * tTpy + zz * (vTpy - vTmy)) * is;
  const R tz = tn * nz + (zsp * tTmz + zsm * tTpz + zz * (vTpz - vTmz)) * is;
  // flux A_n q*: stresses -(lam (v.n) I + mu (n v^T + v n^T)), velocities -t/rho;
  // multiplied by -s for the surface term: +s (...)
  const R lvn = lam * vn;
  const R ms = mu * s;
  out[0] = s * lvn + R(2) * ms * nx * vx;
  out[1] = s * lvn + R(2) * ms * ny * vy;
  out[2] = s * lvn + R(2) * ms * nz * vz;
  out[3] = ms * (nx * vy + ny * vx);
  out[4] = ms * (ny * vz + nz * vy);
  out[5] = ms * (nx * vz + nz * vx);
  const R sr = s * rho_inv;
  out[6] = sr * tx;
  out[7] = sr * ty;
  out[8] = sr * tz;
  // memory-variable rows: -(1/2)(n v^T + v n^T), times -s
  const R hs = R(0.5) * s;
  out[9] = s * nx * vx;
  out[10] = s * ny * vy;
  out[11] = s * nz * vz;
  out[12] = hs * (nx * vy + ny * vx);
  out[13] = hs * (ny * vz + nz * vy);
  out[14] = hs * (nx * vz + nz * vx);
}

// Orders the LDS accesses of one wave: every lane's LDS stores before it are
// seen by every lane's LDS loads after it.  A wave's LDS instructions are
// performed in issue order, so no hardware barrier is needed; the fences keep
// the compiler from moving LDS accesses across.  For data written and read
// by the same wave only (a workgroup barrier where other waves are involved).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Steps of cluster cl at the processed level (see LevelArgs::clock).
__device__ __forceinline__ int step_new_of(const LevelArgs& a, int cl) {
  return (int)((*a.clock + a.jrel) >> cl);
}
__device__ __forceinline__ int step_fin_of(const LevelArgs& a, int cl) { return step_new_of(a, cl) - 1; }

// Linear workgroup id -> (element group, run).  Workgroups are dealt to the
// 8 XCDs round robin; with xcd_remap the ids of one XCD cover a contiguous
// range of the (run-major) group space, so neighbouring elements share that
// XCD's L2.  A bijection for any grid size; so is the optional affine shuffle
// after it (a debug aid: it changes which groups run together and first).
__device__ __forceinline__ void group_and_run(const LevelArgs& a, int& g, int& run) {
  const int nx = gridDim.x;
  int lin = blockIdx.x + blockIdx.y * nx;
  if (a.xcd_remap) {
    const int total = nx * gridDim.y;
    const int q = total / 8, r = total % 8;
    const int x = lin % 8, k = lin / 8;
    lin = x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
  }
  if (a.shuf_mul)   // the host keeps lin * shuf_mul + shuf_add below 2^32
    lin = (int)(((unsigned)lin * (unsigned)a.shuf_mul + (unsigned)a.shuf_add) % (unsigned)(nx * gridDim.y));
  g = lin % nx;
  run = a.run0 + lin / nx;
}

// State arrays are stacked run after run: the pointers of one run.
template <class R>
__device__ __forceinline__ void select_run(KPtrs& p, int run) {
  p.Qe = reinterpret_cast<R*>(p.Qe) + (size_t)run * p.run_qe;
  p.Qa = reinterpret_cast<R*>(p.Qa) + (size_t)run * p.run_qa;
  p.T1 = reinterpret_cast<R*>(p.T1) + (size_t)run * p.run_t1;
  p.T2 = reinterpret_cast<R*>(p.T2) + (size_t)run * p.run_t2;
  p.T3 = reinterpret_cast<R*>(p.T3) + (size_t)run * p.run_t3;
  p.recD = reinterpret_cast<R*>(p.recD) + (size_t)run * p.run_recd;
}

}  // namespace

}  // namespace edg
