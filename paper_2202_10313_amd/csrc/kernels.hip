// HIP kernels (gfx950) of the ADER-DG element update with clustered rate-2
// LTS: time kernel (Cauchy-Kowalevski), volume kernel, surface kernel with the
// Godunov flux, anelastic relaxation, B1/B2/B3 buffer output, point sources,
// receivers.  Sec. III-A (Discrete Formulation; eqs. ader_taylor, ader_derivative_elastic,
// ader_derivative_anelastic, volume, local/neigh surface kernels, update) and
// Sec. V-B (Buffers and Algorithm; eq. lts_buffers and the buffer consumption rules).
//
// Work mapping.  One wave (64 lanes) owns 7 elements; lane = 9*e + q holds the
// modal row q (0..5 stresses xx,yy,zz,xy,yz,xz; 6..8 velocities u,v,w) of
// element e, and all 6m memory variables of the modes b = q + 9 jb (the
// anelastic terms act mode by mode, so this spreads them evenly over the 9
// lanes and keeps each mechanism's trace inside one lane).  Reference-matrix
// products (K_c, F~_i, F^_i) act inside a row, so every lane applies the same
// sparse matrix: they are straight-line FMAs with compile-time constants
// (generated/refmats.h).  Products that mix rows (Jacobians, star matrices,
// flux solvers, anelastic coupling) go through a per-wave LDS exchange.
// Lane 63 repeats lane 54's work and never writes global memory.
//
// Differences from the paper's own kernel layout (prior art for Xeon):
//  * the star matrices are applied as "inverse Jacobian, then physical
//    Jacobian" (same product, re-associated) from ~20 compact per-element
//    parameters instead of stored 9x9 / 6x9 matrices;
//  * the flux solvers are evaluated on the fly (Godunov state in the face
//    normal frame) instead of stored 9x9 / 6x9 matrices;
//  * every element's local vertices are sorted by global vertex id, so both
//    sides of a face parameterise it identically and the 12 neighbour flux
//    matrices F-_{j,h} collapse to the 4 F~_j: buffers are stored as face
//    traces (B F~_j, 9 x F per face), produced once by their owner;
//  * the local and neighbouring surface contributions of a step are applied
//    together at the end of the step (one Godunov solve and one lift per face)
//    from the element's own B1 trace and the neighbour data;
//  * ping-pong trace slots (by step parity) let one launch per finest level
//    finish the step of every active element and start its next one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "generated/refmats.h"
#include "kernels.hpp"
#include "device_common.hpp"

namespace edg {

namespace {

template <class R, int O, int M>
struct LdsLayout {
  using RF = edg_gen::Ref<O>;
  static constexpr int B = RF::B, FP = RF::FP;
  static constexpr int FACE = 4 * 2 * LPE * FP;          // [face][side][row][f]
  static constexpr int GRAD = LPE * 3 * B;                // [row][dir][b]
  static constexpr int COUP = M > 0 ? 6 * B : 0;          // [stress comp][b]
  static constexpr int REGION = FACE > GRAD + COUP ? FACE : GRAD + COUP;
  static constexpr int TOTAL = EPW * REGION;              // lane 63 shares element 6's region
};

template <class R, int O, int M>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2)))
void k_level(KPtrs p, LevelArgs a) {
  using RF = edg_gen::Ref<O>;
  using L = LdsLayout<R, O, M>;
  constexpr int B = RF::B, F = RF::F, FP = RF::FP;
  constexpr int MM = M > 0 ? M : 1;
  constexpr int JB = (B + LPE - 1) / LPE;   // modes owned per lane for the memory variables
  __shared__ R lds[L::TOTAL];

  const int lane = threadIdx.x;
  const int e = lane / LPE, r = lane % LPE;
  const int ec = e < EPW ? e : EPW - 1;     // lane 63 duplicates lane 54 (same element, same row)
  const int q = e < EPW ? r : 0;
  int g, run;
  group_and_run(a, g, run);
  select_run<R>(p, run);
  const int elem = g * EPW + ec;
  const int cl = cluster_of(a, g * EPW);        // one cluster per workgroup (uniform)
  const bool valid = (e < EPW) && (elem < a.cl_vend[cl]);
  const int slot = ec * LPE + q;
  R* const reg = lds + ec * L::REGION;

  R* Qe = reinterpret_cast<R*>(p.Qe);
  R* Qa = reinterpret_cast<R*>(p.Qa);
  const R* P = reinterpret_cast<const R*>(p.P) + (size_t)elem * NPARAM;
  const int* FI = p.FI + (size_t)elem * FI_WORDS;
  const size_t Kp = (size_t)p.Kp;
  const size_t tstride = (size_t)4 * LPE * FP;   // per element in a trace slot

  const bool is_stress = q < 6;
  int qi = 0, qj = 0;                        // stress component (i, j) of this row
  if (q < 3) { qi = q; qj = q; }
  else if (q == 3) { qi = 0; qj = 1; }
  else if (q == 4) { qi = 1; qj = 2; }
  else if (q == 5) { qi = 0; qj = 2; }
  const R delta = q < 3 ? R(1) : R(0);

  // element parameters
  R G[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) G[c] = P[c];
  const R rho_inv = P[9], lam = P[10], mu = P[11], zp = P[12], zs = P[13];
  R al[MM], bl[MM], om[MM];
#pragma unroll
  for (int l = 0; l < MM; ++l) {
    al[l] = M > 0 ? P[14 + 2 * l] : R(0);
    bl[l] = M > 0 ? P[15 + 2 * l] : R(0);
    om[l] = M > 0 ? R(a.omega[l]) : R(0);
  }

  // elastic DOFs: this lane's row, all modes.  Memory variables: all
  // 6m components of the modes b = q + 9 jb owned by this lane.
  R qe[B];
  const size_t gbase = (size_t)g * B;
#pragma unroll
  for (int b = 0; b < B; ++b) qe[b] = Qe[(gbase + b) * NSLOT + slot];

  // rows of the gradient exchange this lane reads
  int rA = 0, rB = 0, rC = 0;   // velocity lane: sigma_{i,d} along d
  if (!is_stress) {
    const int i = q - 6;
    rA = sym_index(i, 0) * 3 * B + 0 * B;
    rB = sym_index(i, 1) * 3 * B + 1 * B;
    rC = sym_index(i, 2) * 3 * B + 2 * B;
  }
  const int eA = (6 + qi) * 3 * B + qj * B;   // d v_i / d x_j
  const int eB = (6 + qj) * 3 * B + qi * B;   // d v_j / d x_i
  const int d0 = 6 * 3 * B + 0 * B, d1 = 7 * 3 * B + 1 * B, d2 = 8 * 3 * B + 2 * B;
  R* const grad = reg;
  R* const coup = reg + L::GRAD;

  // ------------------------------------------------ surface: finish step n
  // (the memory variables are loaded afterwards; their surface term goes
  // through the LDS area `coup`)
  bool coup_pending = false;
  if (a.kind != KIND_PREDICT) {
    const int n = step_fin_of(a, cl);
    const R* T1 = reinterpret_cast<const R*>(p.T1);
    const R* T2 = reinterpret_cast<const R*>(p.T2);
    const R* T3 = reinterpret_cast<const R*>(p.T3);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int nb = FI[3 * i];
      const int code = FI[3 * i + 1];
      const size_t aux = (size_t)FI[3 * i + 2];
      const int j = code & 15, rel = ((code >> 8) & 15) - 1;
      const R* own = T1 + ((size_t)(n & 1) * Kp + elem) * tstride + (size_t)(i * LPE + q) * FP;
      R* dmn = reg + ((i * 2 + 0) * LPE + q) * FP;
      R* dpl = reg + ((i * 2 + 1) * LPE + q) * FP;
#pragma unroll
      for (int f = 0; f < FP; ++f) dmn[f] = own[f];
      if (nb >= 0) {
        const size_t nbo = (size_t)nb * tstride + (size_t)(j * LPE + q) * FP;
        if (rel == 0) {
          const R* s = T1 + (size_t)(n & 1) * Kp * tstride + nbo;
#pragma unroll
          for (int f = 0; f < FP; ++f) dpl[f] = s[f];
        } else if (rel < 0) {       // finer neighbour: its accumulated B3
          const R* s = T3 + ((size_t)(n & 1) * p.N3 + aux) * tstride + (size_t)(j * LPE + q) * FP;
#pragma unroll
          for (int f = 0; f < FP; ++f) dpl[f] = s[f];
        } else {                    // coarser neighbour: B2, then B1 - B2
          const int c = (n >> 1) & 1;
          const R* s2 = T2 + ((size_t)c * p.N2 + aux) * tstride + (size_t)(j * LPE + q) * FP;
          if ((n & 1) == 0) {
#pragma unroll
            for (int f = 0; f < FP; ++f) dpl[f] = s2[f];
          } else {
            const R* s1 = T1 + (size_t)c * Kp * tstride + nbo;
#pragma unroll
            for (int f = 0; f < FP; ++f) dpl[f] = s1[f] - s2[f];
          }
        }
      } else {
#pragma unroll
        for (int f = 0; f < FP; ++f) dpl[f] = R(0);
      }
    }
    __syncthreads();
    // Godunov solves: 4F (face, mode) items spread over the element's 9 lanes
#pragma unroll 1
    for (int rr = 0; rr < (4 * F + LPE - 1) / LPE; ++rr) {
      const int t = q + LPE * rr;
      if (t < 4 * F) {
        const int i = t / F, f = t % F;
        const int code = FI[3 * i + 1];
        const int bc = (code >> 4) & 15;
        const R* fp = P + 20 + 6 * i;
        R qm[9], qp[9], out[15];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          qm[k] = reg[((i * 2 + 0) * LPE + k) * FP + f];
          qp[k] = reg[((i * 2 + 1) * LPE + k) * FP + f];
        }
        const R zpp = bc == 0 ? fp[4] : zp, zsp = bc == 0 ? fp[5] : zs;
        godunov<R>(qm, qp, fp[0], fp[1], fp[2], zp, zs, zpp, zsp, lam, mu, rho_inv, fp[3], bc, out);
#pragma unroll
        for (int k = 0; k < 15; ++k) reg[((i * 2 + k / 9) * LPE + k % 9) * FP + f] = out[k];
      }
    }
    __syncthreads();
    R da[B];
    {
      R pf[4 * FP];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int f = 0; f < FP; ++f) pf[i * FP + f] = reg[((i * 2 + 0) * LPE + q) * FP + f];
      RF::lift(pf, qe);
      if (M > 0) {
#pragma unroll
        for (int b = 0; b < B; ++b) da[b] = R(0);
        if (is_stress) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int f = 0; f < FP; ++f) pf[i * FP + f] = reg[((i * 2 + 1) * LPE + q) * FP + f];
          RF::lift(pf, da);
        }
      }
    }
    if (M > 0) {
      // the strain-rate flux of stress component q, lifted, reaches the
      // memory variables of that component through the mode owners
      __syncthreads();
      if (is_stress && e < EPW)
#pragma unroll
        for (int b = 0; b < B; ++b) coup[q * B + b] = da[b];
      coup_pending = true;
    }
    __syncthreads();
  }

  R qa[JB][MM][6];
#pragma unroll
  for (int jb = 0; jb < JB; ++jb) {
    const int b = q + LPE * jb;
#pragma unroll
    for (int l = 0; l < MM; ++l)
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        qa[jb][l][c] = M > 0 ? Qa[((((size_t)g * JB + jb) * MM + l) * 6 + c) * NSLOT + slot] : R(0);
        if (M > 0 && coup_pending && b < B) qa[jb][l][c] += om[l] * coup[c * B + b];
      }
  }
  if (M > 0 && coup_pending) __syncthreads();

  if (a.kind == KIND_NEIGHBOR) {
    if (valid) {
#pragma unroll
      for (int b = 0; b < B; ++b) Qe[(gbase + b) * NSLOT + slot] = qe[b];
      if (M > 0)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb)
#pragma unroll
          for (int l = 0; l < MM; ++l)
#pragma unroll
            for (int c = 0; c < 6; ++c) Qa[((((size_t)g * JB + jb) * MM + l) * 6 + c) * NSLOT + slot] = qa[jb][l][c];
    }
    return;
  }

  // the start-of-step state, recorded for the reverse sweep when asked
  // (every element slot of the group; padding slots get the zeros their state holds)
  if (a.rec_e != nullptr && e < EPW) {
    R* const Re = reinterpret_cast<R*>(a.rec_e);
#pragma unroll
    for (int b = 0; b < B; ++b) Re[(gbase + b) * NSLOT + slot] = valid ? qe[b] : R(0);
    if (M > 0) {
      R* const Ra = reinterpret_cast<R*>(a.rec_a);
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int l = 0; l < MM; ++l)
#pragma unroll
          for (int c = 0; c < 6; ++c)
            Ra[((((size_t)g * JB + jb) * MM + l) * 6 + c) * NSLOT + slot] = valid ? qa[jb][l][c] : R(0);
    }
  }

  // ------------------------------------------------ time kernel: predict step nn
  const int nn = step_new_of(a, cl);
  const int eflags = FI[12];
  const bool need_b2 = __any((eflags & EF_HAS_FINER) != 0);
  const int rec_slot = FI[15];
  R de[B], te[B], t2[B];
  R dm[JB][MM][6];
#pragma unroll
  for (int b = 0; b < B; ++b) { de[b] = qe[b]; te[b] = R(0); t2[b] = R(0); }
#pragma unroll
  for (int jb = 0; jb < JB; ++jb)
#pragma unroll
    for (int l = 0; l < MM; ++l)
#pragma unroll
      for (int c = 0; c < 6; ++c) dm[jb][l][c] = qa[jb][l][c];

#pragma unroll 1
  for (int d = 0; d < O; ++d) {
    const R c_d = R(a.tc[cl][d]), h_d = R(a.th[cl][d]);
    const bool more = d + 1 < O;
#pragma unroll
    for (int b = 0; b < B; ++b) te[b] += c_d * de[b];
    if (need_b2)
#pragma unroll
      for (int b = 0; b < B; ++b) t2[b] += h_d * de[b];
    if (rec_slot >= 0 && valid) {
      R* rd = reinterpret_cast<R*>(p.recD) + (((size_t)rec_slot * O + d) * LPE + q) * B;
#pragma unroll
      for (int b = 0; b < B; ++b) rd[b] = de[b];
    }
    if (more) RF::ck_grad(de, G, grad + q * 3 * B);
    __syncthreads();
    if (M > 0) {
      // memory variables of the owned modes: coupling into the stresses
      // (-sum_l a_l tr(theta^l) I + b_l theta^l), the volume term
      // -omega_l T^{a,l}, and the next derivative omega_l (eps - theta^l)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const int b = q + LPE * jb;
        if (b < B) {
          R eps[6];
          if (more) {
            eps[0] = grad[6 * 3 * B + 0 * B + b];
            eps[1] = grad[7 * 3 * B + 1 * B + b];
            eps[2] = grad[8 * 3 * B + 2 * B + b];
            eps[3] = R(0.5) * (grad[6 * 3 * B + 1 * B + b] + grad[7 * 3 * B + 0 * B + b]);
            eps[4] = R(0.5) * (grad[7 * 3 * B + 2 * B + b] + grad[8 * 3 * B + 1 * B + b]);
            eps[5] = R(0.5) * (grad[6 * 3 * B + 2 * B + b] + grad[8 * 3 * B + 0 * B + b]);
          }
          R cp[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
          for (int l = 0; l < MM; ++l) {
            const R tr = dm[jb][l][0] + dm[jb][l][1] + dm[jb][l][2];
#pragma unroll
            for (int c = 0; c < 6; ++c) cp[c] -= bl[l] * dm[jb][l][c] + (c < 3 ? al[l] * tr : R(0));
#pragma unroll
            for (int c = 0; c < 6; ++c) {
              qa[jb][l][c] -= om[l] * c_d * dm[jb][l][c];
              if (more) dm[jb][l][c] = om[l] * (eps[c] - dm[jb][l][c]);
            }
          }
          if (e < EPW)
#pragma unroll
            for (int c = 0; c < 6; ++c) coup[c * B + b] = cp[c];
        }
      }
      __syncthreads();
    }
    if (is_stress) {
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const R cq = M > 0 ? coup[q * B + b] : R(0);
        if (M > 0) qe[b] += c_d * cq;                 // volume: E^l T^{a,l}
        if (more) {
          const R eps = R(0.5) * (grad[eA + b] + grad[eB + b]);
          const R div = grad[d0 + b] + grad[d1 + b] + grad[d2 + b];
          de[b] = lam * delta * div + R(2) * mu * eps + cq;
        }
      }
    } else if (more) {
#pragma unroll
      for (int b = 0; b < B; ++b) de[b] = rho_inv * (grad[rA + b] + grad[rB + b] + grad[rC + b]);
    }
    __syncthreads();
  }

  // ------------------------------------------------ buffers as face traces
  {
    R pt[4 * FP];
    RF::trace(te, pt);
    const size_t own = ((size_t)(nn & 1) * Kp + elem) * tstride + (size_t)q * FP;
    if (valid) {
      R* T1 = reinterpret_cast<R*>(p.T1);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int f = 0; f < FP; ++f) T1[own + (size_t)i * LPE * FP + f] = pt[i * FP + f];
    }
    if (eflags & EF_HAS_COARSER) {     // B3: restart on even steps, accumulate on odd
      R* T3 = reinterpret_cast<R*>(p.T3);
      const size_t o3 = ((size_t)((nn >> 1) & 1) * p.N3 + (size_t)FI[14]) * tstride + (size_t)q * FP;
      if (valid) {
        if ((nn & 1) == 0) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int f = 0; f < FP; ++f) T3[o3 + (size_t)i * LPE * FP + f] = pt[i * FP + f];
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int f = 0; f < FP; ++f) T3[o3 + (size_t)i * LPE * FP + f] += pt[i * FP + f];
        }
      }
    }
    if (need_b2) {                      // B2: half-step integral
      RF::trace(t2, pt);
      if (valid && (eflags & EF_HAS_FINER)) {
        R* T2 = reinterpret_cast<R*>(p.T2);
        const size_t o2 = ((size_t)(nn & 1) * p.N2 + (size_t)FI[13]) * tstride + (size_t)q * FP;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int f = 0; f < FP; ++f) T2[o2 + (size_t)i * LPE * FP + f] = pt[i * FP + f];
      }
    }
  }

  // ------------------------------------------------ volume kernel
  RF::vol_grad(te, G, grad + q * 3 * B);
  __syncthreads();
  if (M > 0) {
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) {
      const int b = q + LPE * jb;
      if (b < B) {
        R eps[6];
        eps[0] = grad[6 * 3 * B + 0 * B + b];
        eps[1] = grad[7 * 3 * B + 1 * B + b];
        eps[2] = grad[8 * 3 * B + 2 * B + b];
        eps[3] = R(0.5) * (grad[6 * 3 * B + 1 * B + b] + grad[7 * 3 * B + 0 * B + b]);
        eps[4] = R(0.5) * (grad[7 * 3 * B + 2 * B + b] + grad[8 * 3 * B + 1 * B + b]);
        eps[5] = R(0.5) * (grad[6 * 3 * B + 2 * B + b] + grad[8 * 3 * B + 0 * B + b]);
#pragma unroll
        for (int l = 0; l < MM; ++l)
#pragma unroll
          for (int c = 0; c < 6; ++c) qa[jb][l][c] -= om[l] * eps[c];
      }
    }
  }
  if (is_stress) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const R eps = R(0.5) * (grad[eA + b] + grad[eB + b]);
      const R div = grad[d0 + b] + grad[d1 + b] + grad[d2 + b];
      qe[b] -= lam * delta * div + R(2) * mu * eps;
    }
  } else {
#pragma unroll
    for (int b = 0; b < B; ++b) qe[b] -= rho_inv * (grad[rA + b] + grad[rB + b] + grad[rC + b]);
  }

  if (valid) {
#pragma unroll
    for (int b = 0; b < B; ++b) Qe[(gbase + b) * NSLOT + slot] = qe[b];
    if (M > 0)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int l = 0; l < MM; ++l)
#pragma unroll
          for (int c = 0; c < 6; ++c) Qa[((((size_t)g * JB + jb) * MM + l) * 6 + c) * NSLOT + slot] = qa[jb][l][c];
  }
}

// ---------------------------------------------------------------------------
// Two-wave variant (O = 4, 5, FP32): a workgroup of two waves owns 7
// elements.  Lane (e, q) of wave w keeps row q of element e for the modes
// [MB_w, MB_w+1) only (elementwise state halves, no register spill, two
// workgroups per SIMD); the reference-matrix products that need a whole row
// read it from the LDS row exchange RX, and their outputs are split between
// the waves (stiffness outputs balanced by non-zero count, two faces each for
// the traces, the wave's own modes for the lift).  The gradient exchange
// holds only the 18 (row, direction) pairs that are read: all three
// directions of the velocities, d_i sigma_ij of each stress row.
template <class R, int O, int M>
struct Lds2 {
  // Bank-conflict-free strides: with a row stride RS and an element stride
  // ES = 9 RS (mod 32), lane 9e+q addresses bank RS (9e + q) (mod 32), a
  // bijection for odd RS over the 63 working lanes.
  using RF = edg_gen::Ref<O>;
  static constexpr int B = RF::B, FP = RF::FP;
  static constexpr int up(int v, int m, int r) { return v + ((r - v % m) % m + m) % m; }
  static constexpr int BS = B % 2 ? B : B + 1;                 // row stride of mode rows (odd)
  static constexpr int FS = FP + 1;                            // row stride of face rows (odd)
  static constexpr int GRAD = 19 * BS;          // 18 used (row, dir) pairs + 1 dummy row
  static constexpr int COUP = 6 * BS;
  static constexpr int RX = LPE * BS;
  static constexpr int REST = GRAD + COUP + RX;
  static constexpr int REGION = up(REST, 32, (9 * BS) % 32);   // element stride of the mode areas
  static constexpr int FACE = up(4 * 2 * LPE * FS, 32, (9 * FS) % 32);  // element stride of the face area
  // At O = 5 the gradient, coupling and exchange areas are three arrays with
  // element strides of their own: the exchange keeps ES = 9 RS (mod 32) for
  // its row-wise accesses, while the gradient and coupling strides (7 and 24
  // mod 32) were chosen, with the slot table, for the fewest modelled
  // conflicts of their mode-owner and slot accesses (1,112 -> 813 cycles per
  // wave in the model).  At O = 4 that choice modelled worse: one region.
  static constexpr bool SPLIT = O == 5;
  static constexpr int GSTR = SPLIT ? up(GRAD, 32, 7) : REGION;
  static constexpr int CSTR = SPLIT ? up(COUP, 32, 24) : REGION;
  static constexpr int RSTR = SPLIT ? up(RX, 32, (9 * BS) % 32) : REGION;
  static constexpr int GOFF = 0;
  static constexpr int COFF = SPLIT ? EPW * GSTR : GRAD;
  static constexpr int ROFF = SPLIT ? COFF + EPW * CSTR : GRAD + COUP;
  static constexpr int MODES = SPLIT ? ROFF + EPW * RSTR : EPW * REGION;
  static constexpr int TOTAL = MODES > EPW * FACE ? MODES : EPW * FACE;
};

// An opaque copy of a lane index: addresses built from it are recomputed at
// the point of use instead of being kept live (as 64-bit register pairs)
// across the whole kernel.
__device__ __forceinline__ int fresh(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// slot of (row, direction) in the gradient exchange; 18 = not read (dummy).
// The assignment is the one with the fewest LDS bank conflicts (over the
// stiffness output writes, the strain reads of the memory variables and the
// star-product reads of a time-kernel step) found by a search over slot
// permutations for the strides above (one table per layout of Lds2).
template <int O>
__device__ __forceinline__ int gslot(int row, int dir) {
  constexpr int T4[9][3] = {{1, 18, 18}, {18, 6, 18}, {18, 18, 13}, {17, 12, 18}, {18, 14, 7},
                            {16, 18, 15}, {0, 2, 5}, {11, 10, 3}, {4, 8, 9}};
  constexpr int T5[9][3] = {{16, 18, 18}, {18, 0, 18}, {18, 18, 10}, {15, 1, 18}, {18, 12, 9},
                            {17, 18, 11}, {7, 4, 2}, {8, 3, 14}, {6, 5, 13}};
  constexpr unsigned long long W0 = pack_rows5(O == 5 ? T5 : T4, 0), W1 = pack_rows5(O == 5 ? T5 : T4, 1),
                               W2 = pack_rows5(O == 5 ? T5 : T4, 2);
  const unsigned long long w = dir == 0 ? W0 : (dir == 1 ? W1 : W2);   // selects, no table in memory
  return (int)((w >> (5 * row)) & 31);
}

// KIND is the launch kind (KIND_PREDICT, KIND_FUSED, KIND_NEIGHBOR) as a
// template parameter: one code path per kernel keeps the register allocation
// of the fused path free of the neighbour-only exit.  TM: the traces of faces
// 0 and 1 (the two densest) as one dense product on the matrix cores.
typedef float floatx16 __attribute__((ext_vector_type(16)));
template <class R, int O, int M, int KIND, bool TM = false>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2, 4)))
void k_level2(KPtrs p, LevelArgs a) {
  using RF = edg_gen::Ref<O>;
  using L = Lds2<R, O, M>;
  constexpr int B = RF::B, F = RF::F, FP = RF::FP;
  constexpr int MM = M > 0 ? M : 1;
  constexpr int NB0 = RF::MB1, NB1 = B - RF::MB1;
  constexpr int NBX = NB0 > NB1 ? NB0 : NB1;
  constexpr int JW = (NBX + LPE - 1) / LPE;      // owned memory modes per lane
  constexpr int JB = (B + LPE - 1) / LPE;        // memory-variable layout
  __shared__ R lds[L::TOTAL];
  // per element and face: normal, area ratio, neighbour impedances (the face
  // words of the parameter table) and the boundary kind, staged for the
  // Godunov items of the surface phase
  __shared__ R fdat[KIND != KIND_PREDICT ? EPW * 4 * 8 : 1];
  __shared__ int fbc[KIND != KIND_PREDICT ? EPW * 4 : 1];
  // per element: flags and own B3 slot, for the matrix-core trace's exports
  __shared__ int tme[TM ? EPW * 2 : 1];

  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave (uniform)
  const int lane = threadIdx.x & 63;
  const int e = lane / LPE, r = lane % LPE;
  const int ec = e < EPW ? e : EPW - 1;
  const int q = e < EPW ? r : 0;
  int g, run;
  group_and_run(a, g, run);
  select_run<R>(p, run);
  const int elem = g * EPW + ec;
  const int cl = cluster_of(a, g * EPW);        // one cluster per workgroup (uniform)
  const bool valid = (e < EPW) && (elem < a.cl_vend[cl]);
  const int slot = ec * LPE + q;
  const int base = w ? RF::MB1 : 0;
  const int nb = w ? NB1 : NB0;
  constexpr int BS = L::BS, FS = L::FS;
  R* const fac = lds + ec * L::FACE;          // face area (surface phase only)
  R* const grad = lds + L::GOFF + ec * L::GSTR;
  R* const coup = lds + L::COFF + ec * L::CSTR;
  R* const rx = lds + L::ROFF + ec * L::RSTR;

  // Global addresses are a per-workgroup (uniform, scalar) base plus a 32-bit
  // lane offset, so no 64-bit per-lane address has to stay live.
  constexpr int TS = 4 * LPE * FP;                // trace floats per element
  const size_t Kp = (size_t)p.Kp;
  const size_t tstride = (size_t)TS;
  R* const Qg = reinterpret_cast<R*>(p.Qe) + (size_t)g * B * NSLOT;
  R* const Qag = reinterpret_cast<R*>(p.Qa) + (size_t)g * JB * MM * 6 * NSLOT;
  const R* P = reinterpret_cast<const R*>(p.P) + (size_t)g * EPW * NPARAM + ec * NPARAM;
  const int* FI = p.FI + (size_t)g * EPW * FI_WORDS + ec * FI_WORDS;
  const size_t tg = (size_t)g * EPW * TS;        // this workgroup's first trace

  // The face records of the wave's two faces (and the face word codes to be
  // staged) are the first loads of the kernel: the neighbour gathers depend
  // on them, and loads complete in issue order.
  int fnb[2] = {-1, -1}, fcd[2] = {0, 0}, fax[2] = {0, 0};
  int fcode = 0;
  const bool stage = KIND != KIND_PREDICT && w == 0 && q < 4 && e < EPW;
  if constexpr (KIND != KIND_PREDICT) {
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) {
      fnb[ii] = FI[3 * (2 * w + ii)];
      fcd[ii] = FI[3 * (2 * w + ii) + 1];
      fax[ii] = FI[3 * (2 * w + ii) + 2];
    }
    if (stage) fcode = FI[3 * q + 1];
  }

  const bool is_stress = q < 6;
  int qi = 0, qj = 0;
  if (q < 3) { qi = q; qj = q; }
  else if (q == 3) { qi = 0; qj = 1; }
  else if (q == 4) { qi = 1; qj = 2; }
  else if (q == 5) { qi = 0; qj = 2; }
  const R delta = q < 3 ? R(1) : R(0);

  R G[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) G[c] = P[c];
  const R rho_inv = P[9], lam = P[10], mu = P[11], zp = P[12], zs = P[13];
  R al[MM], bl[MM], om[MM];
#pragma unroll
  for (int l = 0; l < MM; ++l) {
    al[l] = M > 0 ? P[14 + 2 * l] : R(0);
    bl[l] = M > 0 ? P[15 + 2 * l] : R(0);
    om[l] = M > 0 ? R(a.omega[l]) : R(0);
  }

  // LDS offsets (elements of `grad`) this lane writes and reads
  R* const gw0 = grad + gslot<O>(q, 0) * BS;
  R* const gw1 = grad + gslot<O>(q, 1) * BS;
  R* const gw2 = grad + gslot<O>(q, 2) * BS;
  // Star products without divergence: every lane forms
  //   wabc (g[sa] + g[sb] + g[sc]) + wde (g[sd] + g[se]) + wc coupling
  // stress row ij: lambda delta_ij div v + mu (d_j v_i + d_i v_j) + coupling,
  // velocity row i: (1/rho) sum_d d_d sigma_id (the last two reads unused).
  int sa, sb, sc, sd, se;
  R wabc, wde, wc;
  if (is_stress) {
    sa = gslot<O>(6, 0) * BS; sb = gslot<O>(7, 1) * BS; sc = gslot<O>(8, 2) * BS;
    sd = gslot<O>(6 + qi, qj) * BS; se = gslot<O>(6 + qj, qi) * BS;
    wabc = lam * delta; wde = mu; wc = R(1);
  } else {
    const int i = q - 6;
    sa = gslot<O>(sym_index(i, 0), 0) * BS; sb = gslot<O>(sym_index(i, 1), 1) * BS; sc = gslot<O>(sym_index(i, 2), 2) * BS;
    sd = sa; se = sb;
    wabc = rho_inv; wde = R(0); wc = R(0);
  }
  const int cs = (is_stress ? q : 0) * BS;     // coupling row read by this lane

  // The element state (elastic rows and the memory variables of the owned
  // modes) is loaded so that its latency overlaps the surface phase: after
  // the face-trace gathers are issued when there is one (they head the
  // critical path: face words, then the traces they point to), else here.
  R qe[NBX];
  R qa[JW][MM][6];
  auto load_state = [&]() {
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb)
      qe[lb] = lb < nb ? Qg[(base + lb) * NSLOT + slot] : R(0);
#pragma unroll
    for (int jw = 0; jw < JW; ++jw) {
      const int lb = q + LPE * jw, b = base + lb;
      const int jb = b / LPE;
#pragma unroll
      for (int l = 0; l < MM; ++l)
#pragma unroll
        for (int c = 0; c < 6; ++c)
          qa[jw][l][c] = (M > 0 && lb < nb) ? Qag[((jb * MM + l) * 6 + c) * NSLOT + slot] : R(0);
    }
  };
  if constexpr (KIND == KIND_PREDICT) load_state();

  // ------------------------------------------------ surface: finish step n
  bool coup_pending = false;
  if constexpr (KIND != KIND_PREDICT) {
    const int n = step_fin_of(a, cl);
    const R* T1 = reinterpret_cast<const R*>(p.T1);
    const R* T2 = reinterpret_cast<const R*>(p.T2);
    const R* T3 = reinterpret_cast<const R*>(p.T3);
    // the face words go to LDS after the gathers are issued (a store of a
    // loaded value waits for it)
    R fw[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    if (stage)
#pragma unroll
      for (int k = 0; k < 6; ++k) fw[k] = P[20 + 6 * q + k];
    // Neighbour data of the wave's two faces.  Each lane selects its sources
    // by arithmetic (same cluster: the neighbour's B1; finer: its B3;
    // coarser: its B2 in the first half step, B1 - B2 in the second; none:
    // zeros) and every load of both faces is issued before any is used, so
    // the memory latency is paid once rather than once per source kind.
    R vown[2][FP], v1[2][FP], v2[2][FP];
    bool none[2];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) {
      const int i = 2 * w + ii;
      const int nbr = fnb[ii];
      const int code = fcd[ii];
      const size_t aux = (size_t)fax[ii];
      const int j = code & 15, rel = ((code >> 8) & 15) - 1;
      const R* own = T1 + (size_t)(n & 1) * Kp * tstride + tg + (ec * TS + (i * LPE + q) * FP);
      const size_t fo = (size_t)(j * LPE + q) * FP;
      const int c = (n >> 1) & 1;
      const R* b1 = T1 + (size_t)(rel == 0 ? (n & 1) : c) * Kp * tstride + (size_t)nbr * tstride + fo;
      const R* b2 = T2 + ((size_t)c * p.N2 + aux) * tstride + fo;
      const R* b3 = T3 + ((size_t)(n & 1) * p.N3 + aux) * tstride + fo;
      const bool odd = (n & 1) != 0;
      const R* s1 = nbr < 0 ? own : (rel == 0 ? b1 : (rel < 0 ? b3 : (odd ? b1 : b2)));
      const bool sub = nbr >= 0 && rel > 0 && odd;
      none[ii] = nbr < 0;
      // (v2 is zeroed before its masked load: no write to a register with a
      // load in flight)
#pragma unroll
      for (int f = 0; f < FP; ++f) v2[ii][f] = R(0);
#pragma unroll
      for (int f = 0; f < FP; ++f) vown[ii][f] = own[f];
#pragma unroll
      for (int f = 0; f < FP; ++f) v1[ii][f] = s1[f];
      if (sub)
#pragma unroll
        for (int f = 0; f < FP; ++f) v2[ii][f] = b2[f];
    }
    if (stage) {
      R* d = fdat + (ec * 4 + q) * 8;
#pragma unroll
      for (int k = 0; k < 6; ++k) d[k] = fw[k];
      fbc[ec * 4 + q] = fcode;
    }
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) {
      const int i = 2 * w + ii;
      R* dmn = fac + ((i * 2 + 0) * LPE + q) * FS;
      R* dpl = fac + ((i * 2 + 1) * LPE + q) * FS;
#pragma unroll
      for (int f = 0; f < FP; ++f) {
        dmn[f] = vown[ii][f];
        dpl[f] = none[ii] ? R(0) : v1[ii][f] - v2[ii][f];
      }
    }
    // keep the state loads below behind these stores (the scheduler would
    // otherwise interleave them and wait for all loads before the barrier)
    __builtin_amdgcn_sched_barrier(0);
    load_state();
    __syncthreads();
#pragma unroll 2
    for (int rr = 0; rr < (4 * F + 2 * LPE - 1) / (2 * LPE); ++rr) {
      const int t = q + LPE * (w + 2 * rr);
      if (t < 4 * F) {
        const int i = t / F, f = t % F;
        const int bc = (fbc[ec * 4 + i] >> 4) & 15;
        const R* fp = fdat + (ec * 4 + i) * 8;
        R qm[9], qp[9], out[15];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          qm[k] = fac[((i * 2 + 0) * LPE + k) * FS + f];
          qp[k] = fac[((i * 2 + 1) * LPE + k) * FS + f];
        }
        const R zpp = bc == 0 ? fp[4] : zp, zsp = bc == 0 ? fp[5] : zs;
        godunov<R>(qm, qp, fp[0], fp[1], fp[2], zp, zs, zpp, zsp, lam, mu, rho_inv, fp[3], bc, out);
#pragma unroll
        for (int k = 0; k < 15; ++k) fac[((i * 2 + k / 9) * LPE + k % 9) * FS + f] = out[k];
      }
    }
    __syncthreads();
    R da[NBX];
    {
      R pf[4 * FP];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int f = 0; f < FP; ++f) pf[i * FP + f] = fac[((i * 2 + 0) * LPE + q) * FS + f];
      if (w == 0) RF::lift_p0(pf, qe); else RF::lift_p1(pf, qe);
      if (M > 0) {
#pragma unroll
        for (int lb = 0; lb < NBX; ++lb) da[lb] = R(0);
        if (is_stress) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int f = 0; f < FP; ++f) pf[i * FP + f] = fac[((i * 2 + 1) * LPE + q) * FS + f];
          if (w == 0) RF::lift_p0(pf, da); else RF::lift_p1(pf, da);
        }
      }
    }
    if (M > 0) {
      __syncthreads();
      if (is_stress && e < EPW)
#pragma unroll
        for (int lb = 0; lb < NBX; ++lb)
          if (lb < nb) coup[q * BS + base + lb] = da[lb];
      coup_pending = true;
      // the mode owners below read the coupling rows of their own wave's modes
      wave_lds_sync();
    } else {
      __syncthreads();
    }
  }

  if (M > 0 && coup_pending) {
#pragma unroll
    for (int jw = 0; jw < JW; ++jw) {
      const int lb = q + LPE * jw, b = base + lb;
      if (lb < nb)
#pragma unroll
        for (int l = 0; l < MM; ++l)
#pragma unroll
          for (int c = 0; c < 6; ++c) qa[jw][l][c] += om[l] * coup[c * BS + b];
    }
  }
  // (the next LDS stores follow the workgroup barrier that forms need_b2)

  if constexpr (KIND == KIND_NEIGHBOR) {
    if (valid) {
#pragma unroll
      for (int lb = 0; lb < NBX; ++lb)
        if (lb < nb) Qg[(base + lb) * NSLOT + slot] = qe[lb];
      if (M > 0)
#pragma unroll
        for (int jw = 0; jw < JW; ++jw) {
          const int lb = q + LPE * jw, b = base + lb, jb = b / LPE;
          if (lb < nb)
#pragma unroll
            for (int l = 0; l < MM; ++l)
#pragma unroll
              for (int c = 0; c < 6; ++c) Qag[((jb * MM + l) * 6 + c) * NSLOT + slot] = qa[jw][l][c];
        }
    }
    return;
  }

  // the start-of-step state, recorded for the reverse sweep when asked
  // (every element slot of the group; padding slots get the zeros their state holds)
  if (a.rec_e != nullptr && e < EPW) {
    R* const Re = reinterpret_cast<R*>(a.rec_e) + (size_t)g * B * NSLOT;
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb)
      if (lb < nb) Re[(base + lb) * NSLOT + slot] = valid ? qe[lb] : R(0);
    if (M > 0) {
      R* const Ra = reinterpret_cast<R*>(a.rec_a) + (size_t)g * JB * MM * 6 * NSLOT;
#pragma unroll
      for (int jw = 0; jw < JW; ++jw) {
        const int lb = q + LPE * jw, b = base + lb, jb = b / LPE;
        if (lb < nb)
#pragma unroll
          for (int l = 0; l < MM; ++l)
#pragma unroll
            for (int c = 0; c < 6; ++c) Ra[((jb * MM + l) * 6 + c) * NSLOT + slot] = valid ? qa[jw][l][c] : R(0);
      }
    }
  }

  // ------------------------------------------------ time kernel: predict step nn
  // The current derivative d^d Q lives only in the row exchange RX: each lane
  // writes its own modes of the next derivative there and reads them back for
  // the time integrals, so no register copy of it is kept across the loop.
  const int nn = step_new_of(a, cl);
  const int eflags = FI[12];
  if constexpr (TM) {
    if (w == 0 && q == 0 && e < EPW) {
      tme[ec * 2] = eflags;
      tme[ec * 2 + 1] = FI[14];
    }
  }
  const bool need_b2 = __syncthreads_or((eflags & EF_HAS_FINER) != 0);
  const int rec_slot = FI[15];
  R te[NBX], t2[NBX];
  R dm[JW][MM][6];
#pragma unroll
  for (int lb = 0; lb < NBX; ++lb) {
    te[lb] = R(0);
    t2[lb] = R(0);
    if (lb < nb) rx[q * BS + base + lb] = qe[lb];
  }
#pragma unroll
  for (int jw = 0; jw < JW; ++jw)
#pragma unroll
    for (int l = 0; l < MM; ++l)
#pragma unroll
      for (int c = 0; c < 6; ++c) dm[jw][l][c] = qa[jw][l][c];

#pragma unroll 1
  for (int d = 0; d < O; ++d) {
    const R c_d = R(a.tc[cl][d]), h_d = R(a.th[cl][d]);
    const bool more = d + 1 < O;
    __syncthreads();
    {
      R dv[NBX];
#pragma unroll
      for (int lb = 0; lb < NBX; ++lb) dv[lb] = lb < nb ? rx[q * BS + base + lb] : R(0);
#pragma unroll
      for (int lb = 0; lb < NBX; ++lb) te[lb] += c_d * dv[lb];
      if (need_b2)
#pragma unroll
        for (int lb = 0; lb < NBX; ++lb) t2[lb] += h_d * dv[lb];
      if (rec_slot >= 0 && valid) {
        R* rd = reinterpret_cast<R*>(p.recD) + (((size_t)rec_slot * O + d) * LPE + q) * B + base;
#pragma unroll
        for (int lb = 0; lb < NBX; ++lb)
          if (lb < nb) rd[lb] = dv[lb];
      }
    }
    if (more) {
      R full[B];
#pragma unroll
      for (int b = 0; b < B; ++b) full[b] = rx[q * BS + b];
      if (w == 0) RF::ck_grad_p0(full, G, gw0, gw1, gw2);
      else RF::ck_grad_p1(full, G, gw0, gw1, gw2);
    }
    __syncthreads();
    if (M > 0) {
#pragma unroll
      for (int jw = 0; jw < JW; ++jw) {
        const int lb = q + LPE * jw, b = base + lb;
        if (lb < nb) {
          R eps[6];
          if (more) {
            eps[0] = grad[gslot<O>(6, 0) * BS + b];
            eps[1] = grad[gslot<O>(7, 1) * BS + b];
            eps[2] = grad[gslot<O>(8, 2) * BS + b];
            eps[3] = R(0.5) * (grad[gslot<O>(6, 1) * BS + b] + grad[gslot<O>(7, 0) * BS + b]);
            eps[4] = R(0.5) * (grad[gslot<O>(7, 2) * BS + b] + grad[gslot<O>(8, 1) * BS + b]);
            eps[5] = R(0.5) * (grad[gslot<O>(6, 2) * BS + b] + grad[gslot<O>(8, 0) * BS + b]);
          }
          R cp[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
          for (int l = 0; l < MM; ++l) {
            const R tr = dm[jw][l][0] + dm[jw][l][1] + dm[jw][l][2];
#pragma unroll
            for (int c = 0; c < 6; ++c) cp[c] -= bl[l] * dm[jw][l][c] + (c < 3 ? al[l] * tr : R(0));
#pragma unroll
            for (int c = 0; c < 6; ++c) {
              qa[jw][l][c] -= om[l] * c_d * dm[jw][l][c];
              if (more) dm[jw][l][c] = om[l] * (eps[c] - dm[jw][l][c]);
            }
          }
          if (e < EPW)
#pragma unroll
            for (int c = 0; c < 6; ++c) coup[c * BS + b] = cp[c];
        }
      }
      // the coupling rows of a mode are read by the stress rows of the same
      // wave (the wave that owns the mode)
      wave_lds_sync();
    }
    // reads of three modes, then their stores of the next derivative (a store
    // into the row exchange between reads would, for the compiler, possibly
    // alias the next mode's reads and put an LDS wait behind every mode)
    constexpr int CH = 3;
#pragma unroll
    for (int l0 = 0; l0 < NBX; l0 += CH) {
      R nx[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) {
        const int lb = l0 + k, b = base + lb;
        nx[k] = R(0);
        if (lb < NBX && lb < nb) {
          const R cq = M > 0 ? wc * coup[cs + b] : R(0);
          if (M > 0) qe[lb] += c_d * cq;
          nx[k] = wabc * (grad[sa + b] + grad[sb + b] + grad[sc + b]) + wde * (grad[sd + b] + grad[se + b]) + cq;
        }
      }
      if (more)
#pragma unroll
        for (int k = 0; k < CH; ++k)
          if (l0 + k < NBX && l0 + k < nb) rx[q * BS + base + l0 + k] = nx[k];
    }
  }
  // (the barrier after the last loop's products orders every read of RX
  // before the time integral is written there)

  // ------------------------------------------------ traces and volume
  // (the matrix-core trace's coefficients are requested before the barrier,
  // so their latency overlaps it)
  float ftb[TM ? RF::MK : 1];
  if constexpr (TM)
#pragma unroll
    for (int st = 0; st < RF::MK; ++st) ftb[st] = RF::FT01[st * 64 + lane];
#pragma unroll
  for (int lb = 0; lb < NBX; ++lb)
    if (lb < nb) rx[q * BS + base + lb] = te[lb];
  __syncthreads();
  {
    R full[B];
#pragma unroll
    for (int b = 0; b < B; ++b) full[b] = rx[q * BS + b];
    if constexpr (!TM) {
    R pt[2 * FP];
    if (w == 0) RF::trace_p0(full, pt); else RF::trace_p1(full, pt);
    const int own = fresh(ec * TS + q * FP);
    if (valid) {
      R* T1 = reinterpret_cast<R*>(p.T1) + (size_t)(nn & 1) * Kp * tstride + tg;
#pragma unroll
      for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int f = 0; f < FP; ++f) T1[own + RF::tface(w, ii) * LPE * FP + f] = pt[ii * FP + f];
    }
    if ((eflags & EF_HAS_COARSER) && valid) {
      R* T3 = reinterpret_cast<R*>(p.T3) + ((size_t)((nn >> 1) & 1) * p.N3 + (size_t)FI[14]) * tstride;
      if ((nn & 1) == 0) {
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
          for (int f = 0; f < FP; ++f) T3[q * FP + RF::tface(w, ii) * LPE * FP + f] = pt[ii * FP + f];
      } else {
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
          for (int f = 0; f < FP; ++f) T3[q * FP + RF::tface(w, ii) * LPE * FP + f] += pt[ii * FP + f];
      }
    }
    } else {
      // faces 0 and 1 on the matrix cores: wave w multiplies the group's rows
      // [32 w, 32 w + 32) (row 9 e + q of the exchange; row 63 is padding) by
      // the two faces' trace coefficients, 32 columns (face, face mode), two
      // modes per step; its sparse face (3, or 2) stays on the vector ALUs
      static_assert(sizeof(R) == 4 && FP <= 16, "matrix-core trace: FP32, at most 16 face modes");
      floatx16 acc;
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] = 0.f;
      const int kh = lane >> 5;
      const int ar = 32 * w + (lane & 31), ae = ar / LPE, aq = ar - LPE * ae;
      const R* const arow = lds + L::ROFF + (ae < EPW ? ae : EPW - 1) * L::RSTR + aq * BS;
#pragma unroll
      for (int st = 0; st < RF::MK; ++st) {
        const int k = 2 * st + kh;
        const float av = (ar < EPW * LPE && k < B) ? arow[k] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, ftb[st], acc, 0, 0, 0);
      }
      R pt[FP];
      if (w == 0) RF::trace_f3(full, pt); else RF::trace_f2(full, pt);
      const int fs = w == 0 ? 3 : 2;
      R* const T1 = reinterpret_cast<R*>(p.T1) + (size_t)(nn & 1) * Kp * tstride + tg;
      const int own = fresh(ec * TS + q * FP);
      if (valid)
#pragma unroll
        for (int f = 0; f < FP; ++f) T1[own + fs * LPE * FP + f] = pt[f];
      if ((eflags & EF_HAS_COARSER) && valid) {
        R* T3 = reinterpret_cast<R*>(p.T3) + ((size_t)((nn >> 1) & 1) * p.N3 + (size_t)FI[14]) * tstride;
        if ((nn & 1) == 0) {
#pragma unroll
          for (int f = 0; f < FP; ++f) T3[q * FP + fs * LPE * FP + f] = pt[f];
        } else {
#pragma unroll
          for (int f = 0; f < FP; ++f) T3[q * FP + fs * LPE * FP + f] += pt[f];
        }
      }
      // accumulator register j holds row 32 w + 8 (j / 4) + 4 (lane / 32) +
      // j % 4, column lane % 32 = 16 face + face mode
      const int col = lane & 31, fc = col >> 4, ff = col & 15;
      if (ff < FP)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int m = 32 * w + 8 * (j >> 2) + 4 * kh + (j & 3);
          const int e2 = m / LPE, q2 = m - LPE * e2;
          if (m < EPW * LPE && g * EPW + e2 < a.cl_vend[cl]) {
            T1[e2 * TS + (fc * LPE + q2) * FP + ff] = acc[j];
            if (tme[e2 * 2] & EF_HAS_COARSER) {
              R* T3 = reinterpret_cast<R*>(p.T3) + ((size_t)((nn >> 1) & 1) * p.N3 + (size_t)tme[e2 * 2 + 1]) * tstride;
              if ((nn & 1) == 0) T3[(fc * LPE + q2) * FP + ff] = acc[j];
              else T3[(fc * LPE + q2) * FP + ff] += acc[j];
            }
          }
        }
    }
    if (w == 0) RF::vol_grad_p0(full, G, gw0, gw1, gw2);
    else RF::vol_grad_p1(full, G, gw0, gw1, gw2);
  }
  __syncthreads();
  if (M > 0) {
#pragma unroll
    for (int jw = 0; jw < JW; ++jw) {
      const int lb = q + LPE * jw, b = base + lb;
      if (lb < nb) {
        R eps[6];
        eps[0] = grad[gslot<O>(6, 0) * BS + b];
        eps[1] = grad[gslot<O>(7, 1) * BS + b];
        eps[2] = grad[gslot<O>(8, 2) * BS + b];
        eps[3] = R(0.5) * (grad[gslot<O>(6, 1) * BS + b] + grad[gslot<O>(7, 0) * BS + b]);
        eps[4] = R(0.5) * (grad[gslot<O>(7, 2) * BS + b] + grad[gslot<O>(8, 1) * BS + b]);
        eps[5] = R(0.5) * (grad[gslot<O>(6, 2) * BS + b] + grad[gslot<O>(8, 0) * BS + b]);
#pragma unroll
        for (int l = 0; l < MM; ++l)
#pragma unroll
          for (int c = 0; c < 6; ++c) qa[jw][l][c] -= om[l] * eps[c];
      }
    }
  }
#pragma unroll
  for (int lb = 0; lb < NBX; ++lb) {
    const int b = base + lb;
    if (lb < nb)
      qe[lb] -= wabc * (grad[sa + b] + grad[sb + b] + grad[sc + b]) + wde * (grad[sd + b] + grad[se + b]);
  }
  if (need_b2) {   // B2 traces from the half-step integral (RX is free again)
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb)
      if (lb < nb) rx[q * BS + base + lb] = t2[lb];
    __syncthreads();
    R full[B];
#pragma unroll
    for (int b = 0; b < B; ++b) full[b] = rx[q * BS + b];
    R pt[2 * FP];
    if (w == 0) RF::trace_p0(full, pt); else RF::trace_p1(full, pt);
    if (valid && (eflags & EF_HAS_FINER)) {
      R* T2 = reinterpret_cast<R*>(p.T2) + ((size_t)(nn & 1) * p.N2 + (size_t)FI[13]) * tstride;
      const int own = fresh(q * FP);
#pragma unroll
      for (int ii = 0; ii < 2; ++ii)
#pragma unroll
        for (int f = 0; f < FP; ++f) T2[own + RF::tface(w, ii) * LPE * FP + f] = pt[ii * FP + f];
    }
  }

  if (valid) {
    const int sl = fresh(slot);
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb)
      if (lb < nb) Qg[(base + lb) * NSLOT + sl] = qe[lb];
    if (M > 0)
#pragma unroll
      for (int jw = 0; jw < JW; ++jw) {
        const int lb = q + LPE * jw, b = base + lb, jb = b / LPE;
        if (lb < nb)
#pragma unroll
          for (int l = 0; l < MM; ++l)
#pragma unroll
            for (int c = 0; c < 6; ++c) Qag[((jb * MM + l) * 6 + c) * NSLOT + sl] = qa[jw][l][c];
      }
  }
}

// point sources: Q[stress] += -M phi(x_s) / |det J| * (S(t1) - S(t0)) for the
// step of the source's element that ends at this level
__device__ double stf_antiderivative(int kind, double p0, double p1, double t) {
  if (kind == 0) {  // Ricker moment rate: S = (t - t0) exp(-a (t - t0)^2), a = (pi fc)^2
    const double a = (M_PI * p0) * (M_PI * p0);
    const double tau = t - p1;
    return tau * exp(-a * tau * tau);
  }
  // Hann moment rate on [t0, t0 + T]
  const double tau = t - p0;
  if (tau <= 0.0) return 0.0;
  if (tau >= p1) return 1.0;
  return (tau - p1 / (2.0 * M_PI) * sin(2.0 * M_PI * tau / p1)) / p1;
}

template <class R, int O, int M>
__global__ void k_sources(KPtrs p, LevelArgs a, SrcArgs s) {
  constexpr int B = edg_gen::Ref<O>::B;
  constexpr int MM = M > 0 ? M : 1;
  (void)MM;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int src = t / (6 * B);
  if (src >= s.n) return;
  const int qb = t % (6 * B), qq = qb / B, b = qb % B;
  const int elem = s.elem[src];
  if (elem >= a.end) return;
  const int cl = cluster_of(a, elem);
  const double dt = a.dt[cl];
  const int n = step_fin_of(a, cl);
  const double t0 = (double)n * dt, t1 = (double)(n + 1) * dt;
  const double w = stf_antiderivative(s.kind[src], s.par[2 * src], s.par[2 * src + 1], t1) -
                   stf_antiderivative(s.kind[src], s.par[2 * src], s.par[2 * src + 1], t0);
  const double inc = -s.moment[6 * src + qq] * s.phi[(size_t)src * B + b] * s.inv_det[src] * w;
  const int g = elem / EPW, e = elem % EPW;
  R* Qe = reinterpret_cast<R*>(p.Qe) + (size_t)s.run[src] * p.run_qe;
  atomicAdd(&Qe[((size_t)g * B + b) * NSLOT + e * LPE + qq], R(inc));
}

// receivers: evaluate the predicted Taylor expansion at the sample times in
// [t^n, t^{n+1}) of every receiver whose element was predicted at this level
template <class R, int O, int M>
__global__ void k_receivers(KPtrs p, LevelArgs a, RecArgs r) {
  constexpr int B = edg_gen::Ref<O>::B;
  const int run = r.run0 + (int)blockIdx.y;
  select_run<R>(p, run);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int rec = t / LPE, q = t % LPE;
  if (rec >= r.n) return;
  double* const out = r.out + (size_t)run * r.n * r.ns * LPE;
  const int elem = r.elem[rec];
  if (elem >= a.end) return;
  const int cl = cluster_of(a, elem);
  const double dt = a.dt[cl];
  const int n = step_new_of(a, cl);
  const double t0 = (double)n * dt, t1 = (double)(n + 1) * dt;
  const R* D = reinterpret_cast<const R*>(p.recD) + (size_t)r.slot[rec] * O * LPE * B;
  double val[O];
  for (int d = 0; d < O; ++d) {
    double v = 0.0;
    for (int b = 0; b < B; ++b) v += (double)D[((size_t)d * LPE + q) * B + b] * r.phi[(size_t)rec * B + b];
    val[d] = v;
  }
  // step n takes the samples in [t0 - eps, t1 - eps), eps = 1e-9 dt: a sample
  // on (or within rounding of) a step boundary belongs to the step that
  // starts there, whichever way the two sides round the boundary
  const double eps = 1e-9 * dt, lo = t0 - eps, hi = t1 - eps;
  long long s = (long long)floor(lo / r.dt_sample) - 1;
  if (s < 0) s = 0;
  for (; s < r.ns && (double)s * r.dt_sample < hi; ++s) {
    const double ts = (double)s * r.dt_sample;
    if (ts < lo) continue;
    const double x = ts - t0;
    double acc = 0.0, pw = 1.0, fact = 1.0;
    for (int d = 0; d < O; ++d) {
      acc += pw / fact * val[d];
      pw *= x;
      fact *= (double)(d + 1);
    }
    out[((size_t)rec * r.ns + s) * LPE + q] = acc;
  }
}

}  // namespace

// advance the device level clock by d finest steps (end of a cycle)
__global__ void k_tick(long long* clock, long long d) {
  if (blockIdx.x == 0 && threadIdx.x == 0) clock[0] += d;
}

int launch_tick(long long* clock, long long d, hipStream_t st) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, st, clock, d);
  return (int)hipGetLastError();
}

__global__ void k_zero_words(uint32_t* p, size_t words) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0u;
}

int launch_zero_words(void* p, size_t words, hipStream_t st) {
  if (words == 0) return 0;
  const size_t blocks = std::min<size_t>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t*)p, words);
  return (int)hipGetLastError();
}

template <class R, int O, int M>
int launch_level(const KPtrs& p, const LevelArgs& a, int runs, hipStream_t st) {
  const int groups = (a.end + EPW - 1) / EPW;
  if (groups <= 0 || runs <= 0) return 0;
  const dim3 grid(groups, runs);
  if constexpr (std::is_same<R, float>::value && O >= 4) {
    if (a.kind == KIND_FUSED && a.trace_mfma)
      hipLaunchKernelGGL((k_level2<R, O, M, KIND_FUSED, true>), grid, dim3(128), 0, st, p, a);
    else if (a.kind == KIND_PREDICT && a.trace_mfma)
      hipLaunchKernelGGL((k_level2<R, O, M, KIND_PREDICT, true>), grid, dim3(128), 0, st, p, a);
    else if (a.kind == KIND_FUSED)
      hipLaunchKernelGGL((k_level2<R, O, M, KIND_FUSED>), grid, dim3(128), 0, st, p, a);
    else if (a.kind == KIND_PREDICT)
      hipLaunchKernelGGL((k_level2<R, O, M, KIND_PREDICT>), grid, dim3(128), 0, st, p, a);
    else
      hipLaunchKernelGGL((k_level2<R, O, M, KIND_NEIGHBOR>), grid, dim3(128), 0, st, p, a);
  } else
    hipLaunchKernelGGL((k_level<R, O, M>), grid, dim3(64), 0, st, p, a);
  return (int)hipGetLastError();
}

template <class R, int O, int M>
int launch_sources(const KPtrs& p, const LevelArgs& a, const SrcArgs& s, hipStream_t st) {
  if (s.n <= 0) return 0;
  constexpr int B = edg_gen::Ref<O>::B;
  const int total = s.n * 6 * B;
  hipLaunchKernelGGL((k_sources<R, O, M>), dim3((total + 255) / 256), dim3(256), 0, st, p, a, s);
  return (int)hipGetLastError();
}

template <class R, int O, int M>
int launch_receivers(const KPtrs& p, const LevelArgs& a, const RecArgs& r, int runs, hipStream_t st) {
  if (r.n <= 0 || runs <= 0) return 0;
  const int total = r.n * LPE;
  hipLaunchKernelGGL((k_receivers<R, O, M>), dim3((total + 127) / 128, runs), dim3(128), 0, st, p, a, r);
  return (int)hipGetLastError();
}

#define EDG_INST(R, O, M)                                                                        \
  template int launch_level<R, O, M>(const KPtrs&, const LevelArgs&, int, hipStream_t);         \
  template int launch_sources<R, O, M>(const KPtrs&, const LevelArgs&, const SrcArgs&, hipStream_t); \
  template int launch_receivers<R, O, M>(const KPtrs&, const LevelArgs&, const RecArgs&, int, hipStream_t);

EDG_KERNEL_INSTANCES

}  // namespace edg
