// HIP kernels (gfx950) of the discrete adjoint of the clustered rate-2 LTS
// ADER-DG update: the exact transpose of the forward kernels' arithmetic, for
// gradients of receiver misfits with respect to the materials.  The paper
// names inversion as a use (Sec. II (Related Work)) but gives no adjoint; the
// forward scheme it transposes is that of Sec. III-A (Discrete Formulation)
// and Sec. V-B (Buffers and Algorithm).
//
// The forward advance is a sequence of per-level launches: at finest level j
// the clusters whose step ends there finish it (surface update from the own
// B1 face trace and the neighbour data), then the clusters whose step starts
// there predict (time kernel, B1/B2/B3 traces, volume update).  The adjoint
// runs the levels backwards and, per level, first the transposed predictions
// (KIND_ADJ_PREDICT), then the transposed neighbour-data updates
// (KIND_ADJ_UPDATE), in two launches.
//
//  * ADJ_UPDATE (element k, step n ending at this level): the adjoint Qbar of
//    k does not change (the update is Q += ...); what flows out are the face
//    adjoints u = trace(Qbar) (9 elastic rows and the 6 omega-weighted sums of
//    the memory-variable rows, 15 x F per face), added to the slot the
//    neighbour across the face keeps for the buffer k read: same cluster ->
//    its B1 slot; coarser neighbour -> its B2 slot in the first half of its
//    step, B1 slot and minus B2 slot in the second; finer neighbour -> its B3
//    slot.  Each slot has one writer (the element across the face).
//  * ADJ_PREDICT (element j, step n starting here): recomputes the time
//    derivatives from the stored start-of-step state, then forms the adjoint
//    of the time integrals: the transposed volume kernel and own surface part
//    (from Qbar), plus the slots its neighbours filled, each pulled through
//    the transpose of the neighbour's flux (Godunov with the neighbour's
//    parameters); then runs the Cauchy-Kowalevski recursion backwards and adds
//    the adjoint of the start-of-step state to Qbar.  It clears the slots it
//    consumed (B3 after its even step, the first of the pair the coarser
//    neighbour read as one sum).  The transposed update also leaves u in S0,
//    where the two-wave transposed prediction reads its own flux's part.
//
// Material derivatives: every product that involves a material parameter
// (lam, mu, 1/rho, a_l, b_l, the impedances of the flux solver) adds its
// adjoint-weighted partial derivative to per-element FP64 words (NG);
// k_material_gradient applies the chain rule to rho, vp, vs.
//
// Work mapping: k_adjoint as the forward k_level (one wave of 64 lanes owns 7
// elements, lane 9e + q holds row q of element e for all modes and the memory
// variables of the modes q + 9 jb); k_adjoint2 (FP32, O = 4, 5, transposed
// prediction) as the forward k_level2 (two waves per 7 elements, modes split
// between them).  Reference-matrix products are the generated straight-line
// code and its transposes; row-mixing products go through LDS.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "generated/refmats.h"
#include "adjoint.hpp"
#include "device_common.hpp"

namespace edg {

namespace {

// Reverse mode of godunov(): for the adjoint u of its 15 outputs, adds
// (d out / d qm)^T u to qm_b, (d out / d qp)^T u to qp_b (interior faces) and
// the derivatives of <u, out> in (rho_inv, lam, mu, zpm, zsm, zpp, zsp) to
// pb[0..6].  out is linear in (qm, qp), so the parameter derivatives are
// bilinear: they use the states passed in (zeros for a side that another
// element accounts for).
template <class R>
__host__ __device__ __forceinline__ void godunov_adj(const R* u, const R* qm, const R* qp, R nx, R ny, R nz, R zpm,
                                                     R zsm, R zpp, R zsp, R lam, R mu, R rho_inv, R s, int bc,
                                                     R* qm_b, R* qp_b, R* pb) {
  const R n[3] = {nx, ny, nz};
  // forward intermediates
  R tm[3], vm[3], tp[3], vp[3];
  tm[0] = qm[0] * nx + qm[3] * ny + qm[5] * nz;
  tm[1] = qm[3] * nx + qm[1] * ny + qm[4] * nz;
  tm[2] = qm[5] * nx + qm[4] * ny + qm[2] * nz;
  vm[0] = qm[6]; vm[1] = qm[7]; vm[2] = qm[8];
  if (bc == 0) {
    tp[0] = qp[0] * nx + qp[3] * ny + qp[5] * nz;
    tp[1] = qp[3] * nx + qp[1] * ny + qp[4] * nz;
    tp[2] = qp[5] * nx + qp[4] * ny + qp[2] * nz;
    vp[0] = qp[6]; vp[1] = qp[7]; vp[2] = qp[8];
  } else if (bc == 1) {
    for (int c = 0; c < 3; ++c) { tp[c] = -tm[c]; vp[c] = vm[c]; }
  } else {
    for (int c = 0; c < 3; ++c) { tp[c] = R(0); vp[c] = R(0); }
  }
  const R tnm = tm[0] * nx + tm[1] * ny + tm[2] * nz, vnm = vm[0] * nx + vm[1] * ny + vm[2] * nz;
  const R tnp = tp[0] * nx + tp[1] * ny + tp[2] * nz, vnp = vp[0] * nx + vp[1] * ny + vp[2] * nz;
  const R ip = R(1) / (zpm + zpp), is = R(1) / (zsm + zsp);
  const R Y = zpm * vnm + zpp * vnp + tnp - tnm;
  const R Z = zpp * tnm + zpm * tnp + zpm * zpp * (vnp - vnm);
  const R vn = Y * ip, tn = Z * ip;
  const R zz = zsm * zsp;
  R tTm[3], vTm[3], tTp[3], vTp[3], W[3], X[3], v[3], t[3];
  for (int c = 0; c < 3; ++c) {
    tTm[c] = tm[c] - tnm * n[c];
    vTm[c] = vm[c] - vnm * n[c];
    tTp[c] = tp[c] - tnp * n[c];
    vTp[c] = vp[c] - vnp * n[c];
    W[c] = zsm * vTm[c] + zsp * vTp[c] + tTp[c] - tTm[c];
    X[c] = zsp * tTm[c] + zsm * tTp[c] + zz * (vTp[c] - vTm[c]);
    v[c] = vn * n[c] + W[c] * is;
    t[c] = tn * n[c] + X[c] * is;
  }
  // outputs -> v, t, material parameters
  R vb[3] = {R(0), R(0), R(0)}, tb[3] = {R(0), R(0), R(0)};
  R vnb = R(0), lamb = R(0), mub = R(0), rib = R(0);
  const R hs = R(0.5) * s;
  for (int c = 0; c < 3; ++c) {
    vnb += s * lam * u[c];
    lamb += s * vn * u[c];
    vb[c] += R(2) * mu * s * n[c] * u[c];
    mub += R(2) * s * n[c] * v[c] * u[c];
    tb[c] += s * rho_inv * u[6 + c];
    rib += s * t[c] * u[6 + c];
    vb[c] += s * n[c] * u[9 + c];
  }
  const int pa[3] = {0, 1, 0}, pc[3] = {1, 2, 2};   // (x,y), (y,z), (x,z)
  for (int k = 0; k < 3; ++k) {
    const int a = pa[k], b = pc[k];
    const R ue = u[3 + k], ua = u[12 + k];
    vb[b] += mu * s * n[a] * ue + hs * n[a] * ua;
    vb[a] += mu * s * n[b] * ue + hs * n[b] * ua;
    mub += s * (n[a] * v[b] + n[b] * v[a]) * ue;
  }
  // v = vn n + W is, t = tn n + X is
  R Wb[3], Xb[3];
  R isb = R(0), tnb = R(0);
  for (int c = 0; c < 3; ++c) {
    vnb += vb[c] * n[c];
    tnb += tb[c] * n[c];
    Wb[c] = vb[c] * is;
    Xb[c] = tb[c] * is;
    isb += vb[c] * W[c] + tb[c] * X[c];
  }
  R vTmb[3], vTpb[3], tTmb[3], tTpb[3];
  R zsmb = R(0), zspb = R(0), zzb = R(0);
  for (int c = 0; c < 3; ++c) {
    vTmb[c] = zsm * Wb[c] - zz * Xb[c];
    vTpb[c] = zsp * Wb[c] + zz * Xb[c];
    tTpb[c] = Wb[c] + zsm * Xb[c];
    tTmb[c] = -Wb[c] + zsp * Xb[c];
    zsmb += Wb[c] * vTm[c] + Xb[c] * tTp[c];
    zspb += Wb[c] * vTp[c] + Xb[c] * tTm[c];
    zzb += Xb[c] * (vTp[c] - vTm[c]);
  }
  zsmb += zsp * zzb;
  zspb += zsm * zzb;
  // tangential parts
  R tmb[3], vmb[3], tpb[3], vpb[3];
  R tnmb = R(0), vnmb = R(0), tnpb = R(0), vnpb = R(0);
  for (int c = 0; c < 3; ++c) {
    tmb[c] = tTmb[c];
    vmb[c] = vTmb[c];
    tpb[c] = tTpb[c];
    vpb[c] = vTpb[c];
    tnmb -= tTmb[c] * n[c];
    vnmb -= vTmb[c] * n[c];
    tnpb -= tTpb[c] * n[c];
    vnpb -= vTpb[c] * n[c];
  }
  // normal parts
  const R Yb = vnb * ip, Zb = tnb * ip;
  const R ipb = vnb * Y + tnb * Z;
  vnmb += zpm * Yb - zpm * zpp * Zb;
  vnpb += zpp * Yb + zpm * zpp * Zb;
  tnpb += Yb + zpm * Zb;
  tnmb += -Yb + zpp * Zb;
  R zpmb = Yb * vnm + Zb * (tnp + zpp * (vnp - vnm));
  R zppb = Yb * vnp + Zb * (tnm + zpm * (vnp - vnm));
  zpmb -= ipb * ip * ip;
  zppb -= ipb * ip * ip;
  zsmb -= isb * is * is;
  zspb -= isb * is * is;
  for (int c = 0; c < 3; ++c) {
    tmb[c] += tnmb * n[c];
    vmb[c] += vnmb * n[c];
    tpb[c] += tnpb * n[c];
    vpb[c] += vnpb * n[c];
  }
  // outside state
  if (bc == 0) {
    qp_b[0] += tpb[0] * nx;
    qp_b[1] += tpb[1] * ny;
    qp_b[2] += tpb[2] * nz;
    qp_b[3] += tpb[0] * ny + tpb[1] * nx;
    qp_b[4] += tpb[1] * nz + tpb[2] * ny;
    qp_b[5] += tpb[0] * nz + tpb[2] * nx;
    qp_b[6] += vpb[0];
    qp_b[7] += vpb[1];
    qp_b[8] += vpb[2];
  } else if (bc == 1) {
    for (int c = 0; c < 3; ++c) {
      tmb[c] -= tpb[c];
      vmb[c] += vpb[c];
    }
  }
  qm_b[0] += tmb[0] * nx;
  qm_b[1] += tmb[1] * ny;
  qm_b[2] += tmb[2] * nz;
  qm_b[3] += tmb[0] * ny + tmb[1] * nx;
  qm_b[4] += tmb[1] * nz + tmb[2] * ny;
  qm_b[5] += tmb[0] * nz + tmb[2] * nx;
  qm_b[6] += vmb[0];
  qm_b[7] += vmb[1];
  qm_b[8] += vmb[2];
  pb[0] += rib;
  pb[1] += lamb;
  pb[2] += mub;
  pb[3] += zpmb;
  pb[4] += zsmb;
  pb[5] += zppb;
  pb[6] += zspb;
}

template <class R, int O, int M>
struct AdjLds {
  using RF = edg_gen::Ref<O>;
  static constexpr int B = RF::B, FP = RF::FP;
  static constexpr int U = 0;                               // face adjoints [face][15][FP]
  static constexpr int PM = 4 * ADJ_ROWS * FP;              // traces / their adjoints [face][9][FP]
  static constexpr int FACE = PM + 4 * LPE * FP;
  static constexpr int GRD = 0;                             // gradients [row][dir][b]
  static constexpr int X = LPE * 3 * B;                     // rows [row][b]
  static constexpr int C = X + LPE * B;                     // stress components [c][b]
  static constexpr int MODE = C + 6 * B;
  static constexpr int REGION = FACE > MODE ? FACE : MODE;
  static constexpr int TOTAL = EPW * REGION;
};

// the element at 32-bit element offset i from a per-workgroup (uniform) base:
// the address is a scalar base plus a zero-extended 32-bit lane byte offset,
// so no 64-bit per-lane address stays live (or spills) across the long loops
template <class T>
__device__ __forceinline__ T& at(T* base, uint32_t i) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (size_t)(i * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ const T& at(const T* base, uint32_t i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (size_t)(i * (uint32_t)sizeof(T)));
}

// adds v to the element's gradient word w (LDS, FP64).  The elements' word
// arrays are NGS = NG + 1 doubles apart: with a stride of NG = 48 doubles the
// same word of every other element fell into one bank, so an atomic of a
// wave serialised over four elements' lanes
constexpr int NGS = NG + 1;
__device__ __forceinline__ void gadd(double* gs, int w, double v) { atomicAdd(gs + w, v); }

// DPP row shift right by N within 16-lane rows; lanes shifted in from
// outside the row read 0
template <int N>
__device__ __forceinline__ float dpp_row_shr(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x110 + N, 0xf, 0xf, true));
}
// the sum of v over the lanes of its 16-lane row (an inclusive scan by
// shifts 1, 2, 4, 8): complete in the row's last lane
__device__ __forceinline__ float row_sum16(float v) {
  v += dpp_row_shr<1>(v);
  v += dpp_row_shr<2>(v);
  v += dpp_row_shr<4>(v);
  v += dpp_row_shr<8>(v);
  return v;
}

// UPD: the transposed update (KIND_ADJ_UPDATE) only needs the weighted
// memory-variable rows in LDS, so it is its own instantiation with a small
// LDS footprint (more workgroups per CU).
template <class R, int O, int M, bool UPD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(UPD && sizeof(R) == 4 ? 4 : 1)))
void k_adjoint(KPtrs p, APtrs ad, LevelArgs a) {
  using RF = edg_gen::Ref<O>;
  using L = AdjLds<R, O, M>;
  constexpr int B = RF::B, F = RF::F, FP = RF::FP;
  constexpr int MM = M > 0 ? M : 1;
  constexpr int JB = (B + LPE - 1) / LPE;
  // FP32 keeps the memory-variable derivative adjoints in registers; FP64
  // (twice the registers) keeps them in lane-private LDS
  constexpr bool NM_LDS = sizeof(R) == 8 && M > 0 && !UPD;
  constexpr int RSTRIDE = UPD ? 6 * B : L::REGION;   // LDS words per element
  __shared__ R lds[EPW * RSTRIDE];
  __shared__ double gsh[UPD ? 1 : EPW * NGS];
  __shared__ R nmsh[(NM_LDS ? JB * MM * 6 : 1) * 64];

  const int lane = threadIdx.x;
  const int e = lane / LPE, r = lane % LPE;
  const bool act = e < EPW;                 // lane 63 computes a copy of lane 54 and never writes
  const int ec = act ? e : EPW - 1;
  const int q = act ? r : 0;
  const int g = blockIdx.x;
  const int elem = g * EPW + ec;
  const int cl = cluster_of(a, g * EPW);
  const bool valid = act && (elem < a.cl_vend[cl]);
  const int slot = ec * LPE + q;
  R* const reg = lds + ec * RSTRIDE;
  double* const gs = gsh + ec * NGS;
  const R* P = reinterpret_cast<const R*>(p.P) + (size_t)elem * NPARAM;
  const int* FI = p.FI + (size_t)elem * FI_WORDS;
  R* const Le = reinterpret_cast<R*>(ad.Le);
  R* const La = reinterpret_cast<R*>(ad.La);
  const size_t sstride = (size_t)4 * ADJ_ROWS * FP;         // per element in a slot array

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

  // adjoint state: this lane's elastic row (registers); the memory variables
  // of its modes are read from memory where they are used (fewer live
  // registers in the long kernel)
  R le[B];
  const size_t gbase = (size_t)g * B;
#pragma unroll
  for (int b = 0; b < B; ++b) le[b] = Le[(gbase + b) * NSLOT + slot];
  auto la_at = [&](int jb, int l, int c) -> R& { return La[((((size_t)g * JB + jb) * MM + l) * 6 + c) * NSLOT + slot]; };

  // omega-weighted memory-variable adjoints per stress component, rows [c][b]
  R* const Cx = reg + (UPD ? 0 : L::C);
  auto put_weighted = [&]() {
    if (M > 0) {
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const int b = q + LPE * jb;
        if (b < B && act)
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            R w = R(0);
#pragma unroll
            for (int l = 0; l < MM; ++l) w += om[l] * la_at(jb, l, c);
            Cx[c * B + b] = w;
          }
      }
    }
  };
  // face adjoints of this lane's rows: elastic row q, memory-variable row 9+q
  // (the weighted sums must be in Cx)
  R ue[4 * FP], ua[4 * FP];
  auto face_adjoints = [&]() {
    RF::trace(le, ue);
    R wrow[B];
#pragma unroll
    for (int b = 0; b < B; ++b) wrow[b] = (M > 0 && is_stress) ? Cx[q * B + b] : R(0);
    RF::trace(wrow, ua);
  };

  // ================================================================ ADJ_UPDATE
  if constexpr (UPD) {
    put_weighted();
    __syncthreads();
    if (!valid) return;
    const int n = step_fin_of(a, cl);
    // The own-flux face adjoints of this step go to S0, for the two-wave
    // transposed prediction (the Qbar it reads is unchanged until then); the
    // neighbour-data ones are added to the slot of the buffer read across each
    // face.  One face and one row kind at a time: pass 0 the elastic row q
    // from le, pass 1 the omega-weighted memory-variable row 9 + q of the
    // stress lanes from LDS (few live registers, several waves per SIMD).
    R* const S0 = reinterpret_cast<R*>(ad.S0) + (size_t)elem * sstride;
    R* const S1 = reinterpret_cast<R*>(ad.S1);
    R* const S2 = reinterpret_cast<R*>(ad.S2);
    R* const S3 = reinterpret_cast<R*>(ad.S3);
    // one face row's adjoints u to S0 and, added (or subtracted for -B2), to
    // the slot the neighbour across face i keeps for the buffer it read; the
    // face words (neighbour, code, its slot) come with the call
    auto scatter = [&](const R* u, int i, int row, int nb, int code, int fax) {
      R* const s0 = S0 + (size_t)(i * ADJ_ROWS + row) * FP;
      if (nb < 0) {
#pragma unroll
        for (int f = 0; f < FP; ++f) s0[f] = u[f];
        return;
      }
      const size_t aux = (size_t)fax;
      const int j = code & 15, rel = ((code >> 8) & 15) - 1;
      const size_t fo = (size_t)(j * ADJ_ROWS + row) * FP;
      R* d1;
      R* d2 = nullptr;
      if (rel == 0) {
        d1 = S1 + (size_t)nb * sstride + fo;
      } else if (rel < 0) {          // finer neighbour: its B3
        d1 = S3 + aux * sstride + fo;
      } else if ((n & 1) == 0) {     // coarser neighbour, first half: its B2
        d1 = S2 + aux * sstride + fo;
      } else {                       // coarser neighbour, second half: B1 - B2
        d1 = S1 + (size_t)nb * sstride + fo;
        d2 = S2 + aux * sstride + fo;
      }
      // the slot loads first, then the S0 stores (a wait for loads issued
      // after stores would also wait for the stores), then the updates
      R x1[FP], x2[FP];
#pragma unroll
      for (int f = 0; f < FP; ++f) { x1[f] = d1[f]; x2[f] = R(0); }
      if (d2)
#pragma unroll
        for (int f = 0; f < FP; ++f) x2[f] = d2[f];
#pragma unroll
      for (int f = 0; f < FP; ++f) s0[f] = u[f];
#pragma unroll
      for (int f = 0; f < FP; ++f) d1[f] = x1[f] + u[f];
      if (d2)
#pragma unroll
        for (int f = 0; f < FP; ++f) d2[f] = x2[f] - u[f];
    };
    // the face words of face i + 1 are requested before face i's trace, so
    // their latency overlaps it
    auto faces = [&](const R* t, int row) {
      R u[FP];
      int nb = FI[0], cd = FI[1], ax = FI[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int nb_i = nb, cd_i = cd, ax_i = ax;
        if (i < 3) {
          nb = FI[3 * (i + 1)];
          cd = FI[3 * (i + 1) + 1];
          ax = FI[3 * (i + 1) + 2];
        }
        if (i == 0) RF::trace_f0(t, u);
        else if (i == 1) RF::trace_f1(t, u);
        else if (i == 2) RF::trace_f2(t, u);
        else RF::trace_f3(t, u);
        scatter(u, i, row, nb_i, cd_i, ax_i);
      }
    };
    faces(le, q);
    if (M > 0 && is_stress) {
      R wrow[B];
#pragma unroll
      for (int b = 0; b < B; ++b) wrow[b] = Cx[q * B + b];
      faces(wrow, 9 + q);
    }
    return;
  }

  // ================================================================ ADJ_PREDICT
  for (int w = lane; w < EPW * NGS; w += 64) gsh[w] = 0.0;
  const int nn = step_new_of(a, cl);
  const int eflags = FI[12];
  const bool has_b2 = (eflags & EF_HAS_FINER) != 0;
  const bool has_b3 = (eflags & EF_HAS_COARSER) != 0;
  const bool any_b2 = __any(has_b2);
  const int rec_slot = FI[15];
  R* const grad = reg + L::GRD;
  R* const Xr = reg + L::X;
  R* const Ur = reg + L::U;
  R* const Pm = reg + L::PM;
  R* const De = reinterpret_cast<R*>(ad.De);
  R* const Da = reinterpret_cast<R*>(ad.Da);
  const int eA = (6 + qi) * 3 * B + qj * B;   // d v_i / d x_j
  const int eB = (6 + qj) * 3 * B + qi * B;   // d v_j / d x_i
  const int d0 = 6 * 3 * B + 0 * B, d1 = 7 * 3 * B + 1 * B, d2 = 8 * 3 * B + 2 * B;
  int rA = 0, rB = 0, rC = 0;
  if (!is_stress) {
    const int i = q - 6;
    rA = sym_index(i, 0) * 3 * B + 0 * B;
    rB = sym_index(i, 1) * 3 * B + 1 * B;
    rC = sym_index(i, 2) * 3 * B + 2 * B;
  }

  // ---------------------------------------------- forward recompute: D_d, T, T2
  R te[B], t2[B];
  {
    const R* Se = reinterpret_cast<const R*>(ad.Se);
    const R* Sa = reinterpret_cast<const R*>(ad.Sa);
    R de[B];
    R dm[JB][MM][6];
#pragma unroll
    for (int b = 0; b < B; ++b) { de[b] = Se[(gbase + b) * NSLOT + slot]; te[b] = R(0); t2[b] = R(0); }
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
      for (int l = 0; l < MM; ++l)
#pragma unroll
        for (int c = 0; c < 6; ++c)
          dm[jb][l][c] = M > 0 ? Sa[((((size_t)g * JB + jb) * MM + l) * 6 + c) * NSLOT + slot] : R(0);
#pragma unroll 1
    for (int d = 0; d < O; ++d) {
      const R c_d = R(a.tc[cl][d]), h_d = R(a.th[cl][d]);
      const bool more = d + 1 < O;
#pragma unroll
      for (int b = 0; b < B; ++b) { te[b] += c_d * de[b]; t2[b] += h_d * de[b]; }
      if (valid) {
#pragma unroll
        for (int b = 0; b < B; ++b) De[(((size_t)g * O + d) * B + b) * NSLOT + slot] = de[b];
        if (M > 0)
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
#pragma unroll
            for (int l = 0; l < MM; ++l)
#pragma unroll
              for (int c = 0; c < 6; ++c)
                Da[(((((size_t)g * O + d) * JB + jb) * MM + l) * 6 + c) * NSLOT + slot] = dm[jb][l][c];
      }
      if (!more) break;
      RF::ck_grad(de, G, grad + q * 3 * B);
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
            R cp[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
            for (int l = 0; l < MM; ++l) {
              const R tr = dm[jb][l][0] + dm[jb][l][1] + dm[jb][l][2];
#pragma unroll
              for (int c = 0; c < 6; ++c) cp[c] -= bl[l] * dm[jb][l][c] + (c < 3 ? al[l] * tr : R(0));
#pragma unroll
              for (int c = 0; c < 6; ++c) dm[jb][l][c] = om[l] * (eps[c] - dm[jb][l][c]);
            }
            if (act)
#pragma unroll
              for (int c = 0; c < 6; ++c) Cx[c * B + b] = cp[c];
          }
        }
        __syncthreads();
      }
      if (is_stress) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const R cq = M > 0 ? Cx[q * B + b] : R(0);
          const R eps = R(0.5) * (grad[eA + b] + grad[eB + b]);
          const R div = grad[d0 + b] + grad[d1 + b] + grad[d2 + b];
          de[b] = lam * delta * div + R(2) * mu * eps + cq;
        }
      } else {
#pragma unroll
        for (int b = 0; b < B; ++b) de[b] = rho_inv * (grad[rA + b] + grad[rB + b] + grad[rC + b]);
      }
      __syncthreads();
    }
  }

  // ---------------------------------------------- A. volume kernel
  R lte[B], lt2[B];     // adjoints of the element's time integrals (elastic rows)
#pragma unroll
  for (int b = 0; b < B; ++b) { lte[b] = R(0); lt2[b] = R(0); }
  // material terms: V = -(lam delta div + 2 mu eps) (stress), -rho_inv div(sigma) (velocity)
  RF::vol_grad(te, G, grad + q * 3 * B);
  __syncthreads();
  {
    double s = 0.0;
    if (is_stress) {
      double sl = 0.0;
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const R eps = R(0.5) * (grad[eA + b] + grad[eB + b]);
        const R div = grad[d0 + b] + grad[d1 + b] + grad[d2 + b];
        sl += (double)(le[b] * div);
        s += (double)(le[b] * R(2) * eps);
      }
      if (valid) {
        if (q < 3) gadd(gs, 1, -sl);
        gadd(gs, 2, -s);
      }
    } else {
#pragma unroll
      for (int b = 0; b < B; ++b) s += (double)(le[b] * (grad[rA + b] + grad[rB + b] + grad[rC + b]));
      if (valid) gadd(gs, 0, -s);
    }
  }
  __syncthreads();
  // exchange the adjoints the transposed volume kernel mixes: elastic rows,
  // and the omega-weighted memory-variable sums (the time kernel above reused
  // that area)
  if (act)
#pragma unroll
    for (int b = 0; b < B; ++b) Xr[q * B + b] = le[b];
  put_weighted();
  __syncthreads();
  {
    // adjoint of the gradient entries of this row (the volume kernel reads
    // the velocity gradients in the stress rows and memory variables, the
    // stress gradients in the velocity rows)
    R* const gb = grad + q * 3 * B;   // own row of the (now free) gradient area
    if (!is_stress) {
      const int i = q - 6;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int sk = sym_index(i, k);
        const R fm = i == k ? R(2) : R(1), fa = i == k ? R(1) : R(0.5);
#pragma unroll
        for (int b = 0; b < B; ++b) {
          R v = -fm * mu * Xr[sk * B + b] - (M > 0 ? fa * Cx[sk * B + b] : R(0));
          if (i == k) v -= lam * (Xr[0 * B + b] + Xr[1 * B + b] + Xr[2 * B + b]);
          if (act) gb[k * B + b] = v;
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        // entry (q, k) is read by velocity row i' with sym(i', k) == q
        int iv = -1;
        if (k == qj) iv = qi;
        else if (k == qi) iv = qj;
#pragma unroll
        for (int b = 0; b < B; ++b)
          if (act) gb[k * B + b] = iv >= 0 ? -rho_inv * Xr[(6 + iv) * B + b] : R(0);
      }
    }
    RF::vol_grad_T(gb, G, lte);
  }
  face_adjoints();
  __syncthreads();

  // ---------------------------------------------- B. own surface part
  R pt[4 * FP];
  RF::trace(te, pt);
  if (act) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int f = 0; f < FP; ++f) {
        Ur[(i * ADJ_ROWS + q) * FP + f] = ue[i * FP + f];
        if (is_stress) Ur[(i * ADJ_ROWS + 9 + q) * FP + f] = ua[i * FP + f];
        Pm[(i * LPE + q) * FP + f] = pt[i * FP + f];
      }
  }
  __syncthreads();
#pragma unroll 1
  for (int rr = 0; rr < (4 * F + LPE - 1) / LPE; ++rr) {
    const int t = q + LPE * rr;
    if (t < 4 * F && act) {
      const int i = t / F, f = t % F;
      const int bc = (FI[3 * i + 1] >> 4) & 15;
      const R* fp = P + 20 + 6 * i;
      R u[15], qm[9], zero9[9], qmb[9], qpb[9], pb[7];
#pragma unroll
      for (int k = 0; k < 15; ++k) u[k] = (M > 0 || k < 9) ? Ur[(i * ADJ_ROWS + k) * FP + f] : R(0);
#pragma unroll
      for (int k = 0; k < 9; ++k) { qm[k] = Pm[(i * LPE + k) * FP + f]; zero9[k] = R(0); qmb[k] = R(0); qpb[k] = R(0); }
#pragma unroll
      for (int k = 0; k < 7; ++k) pb[k] = R(0);
      const R zpp = bc == 0 ? fp[4] : zp, zsp = bc == 0 ? fp[5] : zs;
      godunov_adj<R>(u, qm, zero9, fp[0], fp[1], fp[2], zp, zs, zpp, zsp, lam, mu, rho_inv, fp[3], bc, qmb, qpb, pb);
#pragma unroll
      for (int k = 0; k < 9; ++k) Pm[(i * LPE + k) * FP + f] = qmb[k];
      if (valid) {
        gadd(gs, 0, pb[0]);
        gadd(gs, 1, pb[1]);
        gadd(gs, 2, pb[2]);
        gadd(gs, 3, pb[3]);
        gadd(gs, 4, pb[4]);
        gadd(gs, bc == 0 ? 11 + 2 * i : 3, pb[5]);
        gadd(gs, bc == 0 ? 12 + 2 * i : 4, pb[6]);
      }
    }
  }
  __syncthreads();
  {
    R pf[4 * FP];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int f = 0; f < FP; ++f) pf[i * FP + f] = Pm[(i * LPE + q) * FP + f];
    RF::lift(pf, lte);
  }
  __syncthreads();

  // ---------------------------------------------- C, D. neighbour data read from this element's buffers
  R* const S1 = reinterpret_cast<R*>(ad.S1);
  R* const S2 = reinterpret_cast<R*>(ad.S2);
  R* const S3 = reinterpret_cast<R*>(ad.S3);
#pragma unroll 1
  for (int phase = 0; phase < 2; ++phase) {
    // phase 0: B1 (and B3, the same trace); phase 1: B2
    if (phase == 1 && !any_b2) break;
    if (phase == 1) RF::trace(t2, pt);
    if (act) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool nbr = FI[3 * i] >= 0;
        R* s1 = phase == 0 ? S1 + (size_t)elem * sstride + (size_t)i * ADJ_ROWS * FP
                           : (has_b2 ? S2 + (size_t)FI[13] * sstride + (size_t)i * ADJ_ROWS * FP : nullptr);
        R* s3 = (phase == 0 && has_b3) ? S3 + (size_t)FI[14] * sstride + (size_t)i * ADJ_ROWS * FP : nullptr;
        const bool clear3 = (nn & 1) == 0;
#pragma unroll
        for (int f = 0; f < FP; ++f) {
          R ve = R(0), va = R(0);
          if (valid && nbr && s1) {
            ve = s1[q * FP + f];
            if (is_stress) va = s1[(9 + q) * FP + f];
            s1[q * FP + f] = R(0);
            if (is_stress) s1[(9 + q) * FP + f] = R(0);
          }
          if (valid && nbr && s3) {
            ve += s3[q * FP + f];
            if (is_stress) va += s3[(9 + q) * FP + f];
            if (clear3) {
              s3[q * FP + f] = R(0);
              if (is_stress) s3[(9 + q) * FP + f] = R(0);
            }
          }
          Ur[(i * ADJ_ROWS + q) * FP + f] = ve;
          if (is_stress) Ur[(i * ADJ_ROWS + 9 + q) * FP + f] = va;
          Pm[(i * LPE + q) * FP + f] = pt[i * FP + f];
        }
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int rr = 0; rr < (4 * F + LPE - 1) / LPE; ++rr) {
      const int t = q + LPE * rr;
      if (t < 4 * F && act) {
        const int i = t / F, f = t % F;
        const int nb = FI[3 * i];
        R qpb[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) qpb[k] = R(0);
        if (nb >= 0) {
          // the flux of the neighbour across face i, seen from its face j
          const int j = FI[3 * i + 1] & 15;
          const R* Pn = reinterpret_cast<const R*>(p.P) + (size_t)nb * NPARAM;
          const R* fn = Pn + 20 + 6 * j;
          R u[15], qpv[9], zero9[9], qmb[9], pb[7];
#pragma unroll
          for (int k = 0; k < 15; ++k) u[k] = (M > 0 || k < 9) ? Ur[(i * ADJ_ROWS + k) * FP + f] : R(0);
#pragma unroll
          for (int k = 0; k < 9; ++k) { qpv[k] = Pm[(i * LPE + k) * FP + f]; zero9[k] = R(0); qmb[k] = R(0); }
#pragma unroll
          for (int k = 0; k < 7; ++k) pb[k] = R(0);
          godunov_adj<R>(u, zero9, qpv, fn[0], fn[1], fn[2], Pn[12], Pn[13], fn[4], fn[5], Pn[10], Pn[11], Pn[9],
                         fn[3], 0, qmb, qpb, pb);
          if (valid)
#pragma unroll
            for (int k = 0; k < 7; ++k) gadd(gs, 19 + 7 * i + k, pb[k]);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) Pm[(i * LPE + k) * FP + f] = qpb[k];
      }
    }
    __syncthreads();
    {
      R pf[4 * FP];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int f = 0; f < FP; ++f) pf[i * FP + f] = Pm[(i * LPE + q) * FP + f];
      if (phase == 0) RF::lift(pf, lte);
      else if (has_b2) RF::lift(pf, lt2);
    }
    __syncthreads();
  }

  // ---------------------------------------------- E. time kernel backwards
  R nbe[B];                 // adjoint of D_{d+1} (elastic row)
  // adjoint of D_{d+1} (memory variables of the owned modes), lane-private LDS
  R nbm_r[NM_LDS ? 1 : JB][MM][6];
  auto nbm = [&](int jb, int l, int c) -> R& {
    if constexpr (NM_LDS) return nmsh[((jb * MM + l) * 6 + c) * 64 + lane];
    else return nbm_r[jb][l][c];
  };
#pragma unroll
  for (int b = 0; b < B; ++b) nbe[b] = R(0);
  if (M > 0)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
#pragma unroll
      for (int l = 0; l < MM; ++l)
#pragma unroll
        for (int c = 0; c < 6; ++c) nbm(jb, l, c) = R(0);
  R* const recDb = reinterpret_cast<R*>(ad.recDb);
#pragma unroll 1
  for (int d = O - 1; d >= 0; --d) {
    const R c_d = R(a.tc[cl][d]), h_d = R(a.th[cl][d]);
    const bool more = d + 1 < O;
    R de[B];
#pragma unroll
    for (int b = 0; b < B; ++b) de[b] = De[(((size_t)g * O + d) * B + b) * NSLOT + slot];
    R cur[B];
#pragma unroll
    for (int b = 0; b < B; ++b) cur[b] = c_d * lte[b] + h_d * lt2[b];
    if (rec_slot >= 0 && valid) {
      R* rd = recDb + (((size_t)rec_slot * O + d) * LPE + q) * B;
#pragma unroll
      for (int b = 0; b < B; ++b) { cur[b] += rd[b]; rd[b] = R(0); }
    }
    if (more) {
      // D_{d+1} = L(D_d): material terms with the forward gradients of D_d
      RF::ck_grad(de, G, grad + q * 3 * B);
      __syncthreads();
      {
        double s = 0.0;
        if (is_stress) {
          double sl = 0.0;
#pragma unroll
          for (int b = 0; b < B; ++b) {
            const R eps = R(0.5) * (grad[eA + b] + grad[eB + b]);
            const R div = grad[d0 + b] + grad[d1 + b] + grad[d2 + b];
            sl += (double)(nbe[b] * div);
            s += (double)(nbe[b] * R(2) * eps);
          }
          if (valid) {
            if (q < 3) gadd(gs, 1, sl);
            gadd(gs, 2, s);
          }
        } else {
#pragma unroll
          for (int b = 0; b < B; ++b) s += (double)(nbe[b] * (grad[rA + b] + grad[rB + b] + grad[rC + b]));
          if (valid) gadd(gs, 0, s);
        }
      }
      __syncthreads();
      // adjoint of the gradient entries read by D_{d+1}
      if (act)
#pragma unroll
        for (int b = 0; b < B; ++b) Xr[q * B + b] = nbe[b];
      if (M > 0) {
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) {
          const int b = q + LPE * jb;
          if (b < B && act)
#pragma unroll
            for (int c = 0; c < 6; ++c) {
              R w = R(0);
#pragma unroll
              for (int l = 0; l < MM; ++l) w += om[l] * nbm(jb, l, c);
              Cx[c * B + b] = w;
            }
        }
      }
      __syncthreads();
      R* const gb = grad + q * 3 * B;   // own row of the (now free) gradient area
      if (!is_stress) {
        const int i = q - 6;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int sk = sym_index(i, k);
          const R fm = i == k ? R(2) : R(1), fa = i == k ? R(1) : R(0.5);
#pragma unroll
          for (int b = 0; b < B; ++b) {
            R v = fm * mu * Xr[sk * B + b] + (M > 0 ? fa * Cx[sk * B + b] : R(0));
            if (i == k) v += lam * (Xr[0 * B + b] + Xr[1 * B + b] + Xr[2 * B + b]);
            if (act) gb[k * B + b] = v;
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          int iv = -1;
          if (k == qj) iv = qi;
          else if (k == qi) iv = qj;
#pragma unroll
          for (int b = 0; b < B; ++b)
            if (act) gb[k * B + b] = iv >= 0 ? rho_inv * Xr[(6 + iv) * B + b] : R(0);
        }
      }
      RF::ck_grad_T(gb, G, cur);
      __syncthreads();
    }
    if (M > 0) {
      // coupling E (memory variables -> stresses): cq_d enters the volume
      // term c_d cq_d and the next derivative
      if (is_stress && act)
#pragma unroll
        for (int b = 0; b < B; ++b) Xr[q * B + b] = c_d * le[b] + (more ? nbe[b] : R(0));
      __syncthreads();
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const int b = q + LPE * jb;
        if (b < B) {
          R cqb[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) cqb[c] = Xr[c * B + b];
          const R cqt = cqb[0] + cqb[1] + cqb[2];
#pragma unroll
          for (int l = 0; l < MM; ++l) {
            R dmd[6];
#pragma unroll
            for (int c = 0; c < 6; ++c)
              dmd[c] = Da[(((((size_t)g * O + d) * JB + jb) * MM + l) * 6 + c) * NSLOT + slot];
            const R tr = dmd[0] + dmd[1] + dmd[2];
            double ga = 0.0, gbb = 0.0;
            ga -= (double)(cqt * tr);
#pragma unroll
            for (int c = 0; c < 6; ++c) gbb -= (double)(cqb[c] * dmd[c]);
            if (valid) {
              gadd(gs, 5 + 2 * l, ga);
              gadd(gs, 6 + 2 * l, gbb);
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) {
              // -omega_l c_d T^a volume term, -omega_l theta in the next
              // derivative, coupling into the stresses
              R v = -om[l] * c_d * la_at(jb, l, c) - bl[l] * cqb[c] - (c < 3 ? al[l] * cqt : R(0));
              if (more) v -= om[l] * nbm(jb, l, c);
              nbm(jb, l, c) = v;
            }
          }
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < B; ++b) nbe[b] = cur[b];
  }
#pragma unroll
  for (int b = 0; b < B; ++b) le[b] += nbe[b];
  if (valid) {
#pragma unroll
    for (int b = 0; b < B; ++b) Le[(gbase + b) * NSLOT + slot] = le[b];
    if (M > 0)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int l = 0; l < MM; ++l)
#pragma unroll
          for (int c = 0; c < 6; ++c) la_at(jb, l, c) += nbm(jb, l, c);
  }
  __syncthreads();
  if (valid)
    for (int w = q; w < NG; w += LPE) ad.gacc[(size_t)elem * NG + w] += gsh[ec * NGS + w];
}

// ---------------------------------------------------------------------------
// Two-wave transposed prediction (FP32, O = 4, 5): a workgroup of two waves
// owns 7 elements, wave w keeps the modes [MB_w, MB_{w+1}) of every row (as
// the forward k_level2), so the per-lane state halves and two waves fit per
// SIMD.  Whole rows for the reference-matrix products come from the LDS row
// exchange; products write or read physical-gradient slots (the 18 (row,
// direction) pairs the star products use); the face data of the element's
// own flux come from S0 (written by the transposed update of the same step),
// so no face adjoint is formed here.
//
// The kernel is bound by memory latency at two waves per SIMD, so its state
// is arranged for few dependent round trips: addresses are a scalar base plus
// a 32-bit lane offset recomputed in the loops (no hoisted per-lane 64-bit
// addresses to spill); the per-wave scratch (forward memory-variable
// derivatives and then their adjoints, the star-product sums of each
// derivative's gradients, the time-integral adjoints, a copy of Qbar) is kept
// in lane-contiguous float4 chunks, one coalesced 1 KB access per instruction;
// the transposed surface runs one 16-lane DPP row per (element, face) pair
// with its face parameters staged in LDS and its gradient words summed over
// the row; the coupling block leaves the omega-weighted sums the next step
// needs in the LDS coupling rows; LDS reads that feed LDS stores are all
// issued before them; workgroup barriers stand only where another wave's LDS
// data is read.
template <class R, int O, int M>
struct AdjLds2 {
  using RF = edg_gen::Ref<O>;
  static constexpr int B = RF::B, FP = RF::FP;
  static constexpr int up(int v, int m, int r) { return v + ((r - v % m) % m + m) % m; }
  static constexpr int BS = B % 2 ? B : B + 1;       // odd row stride
  static constexpr int FS = FP + 1;
  static constexpr int NSL = 20;                     // 18 read pairs, unread dummy 18, zero row 19
  static constexpr int GRAD = NSL * BS;
  static constexpr int COUP = 6 * BS;
  static constexpr int RX = LPE * BS;
  static constexpr int PMW = 4 * LPE * FS;           // face traces / their adjoints [face][row][f]
  static constexpr int REST = GRAD + COUP + RX;
  static constexpr int REGION = up(REST > PMW + RX ? REST : PMW + RX, 32, (9 * BS) % 32);
  static constexpr int TOTAL = EPW * REGION;
};

// Per-wave scratch of the two-wave kernel, in float4 chunks that hold four
// consecutive values of one lane, 64 lanes side by side: an access is one
// coalesced 1 KB transfer per instruction instead of four dword ones.  An
// elastic block (a wave's modes of one row, NBX values) takes CE chunks, a
// memory-variable block (one owned mode's l * 6 + c, 6 MM values) CA.
template <int O, int M>
struct AdjScratch2 {
  using RF = edg_gen::Ref<O>;
  static constexpr int NB0 = RF::MB1, NB1 = RF::B - RF::MB1;
  static constexpr int NBX = NB0 > NB1 ? NB0 : NB1;
  static constexpr int JW = (NBX + LPE - 1) / LPE;
  static constexpr int MM = M > 0 ? M : 1;
  static constexpr int CE = (NBX + 3) / 4, CA = (6 * MM + 3) / 4;
  static constexpr int C6 = M > 0 ? 2 : 0;          // chunks of six words (one strain-like tensor)
  // memory variables: the adjoint of D_d^a is a closed-form sum over the
  // coupling adjoints of the steps >= d, so the scratch keeps those (six
  // words per mode and step) rather than D_d^a and its adjoint per mechanism
  static constexpr int EP = 0;                       // [O - 1][JW] strain rates of D_d (forward)
  static constexpr int HS = EP + (O - 1) * JW * C6;  // [O][JW] coupling adjoints cq_d
  static constexpr int LM = HS + O * JW * C6;        // [O][JW] the steps' Qbar^a terms (Lambda_d)
  static constexpr int DG = LM + O * JW * C6;        // [O - 1][2] star-product sums of grad D_d
  static constexpr int DT = DG + (O - 1) * 2 * CE;   // [2] time-integral adjoints (Δt, Δt/2)
  static constexpr int LE = DT + 2 * CE;             // Qbar's elastic rows (own modes)
  static constexpr int LA = LE + CE;                 // [JW] Qbar's memory variables (M > 0)
  static constexpr int CHUNKS = LA + (M > 0 ? JW * CA : 0);
  static constexpr int WAVE_FLOATS = CHUNKS * 64 * 4;
};
template <int N>
__device__ __forceinline__ void st_chunks(float* base, int l4, const float* v) {
#pragma unroll
  for (int k = 0; k < (N + 3) / 4; ++k) {
    const float4 x = make_float4(v[4 * k], 4 * k + 1 < N ? v[4 * k + 1] : 0.f, 4 * k + 2 < N ? v[4 * k + 2] : 0.f,
                                 4 * k + 3 < N ? v[4 * k + 3] : 0.f);
    *reinterpret_cast<float4*>(base + k * 256 + l4) = x;
  }
}
template <int N>
__device__ __forceinline__ void ld_chunks(const float* base, int l4, float* v) {
#pragma unroll
  for (int k = 0; k < (N + 3) / 4; ++k) {
    const float4 x = *reinterpret_cast<const float4*>(base + k * 256 + l4);
    v[4 * k] = x.x;
    if (4 * k + 1 < N) v[4 * k + 1] = x.y;
    if (4 * k + 2 < N) v[4 * k + 2] = x.z;
    if (4 * k + 3 < N) v[4 * k + 3] = x.w;
  }
}

// (row, direction) -> gradient slot: velocity rows all directions, stress row
// (i, j) directions i and j; 18 = not read, 19 = zeros
__device__ __forceinline__ int aslot(int row, int dir) {
  constexpr int T[9][3] = {{9, 18, 18}, {18, 10, 18}, {18, 18, 11}, {12, 13, 18}, {18, 14, 15},
                           {16, 18, 17}, {0, 1, 2}, {3, 4, 5}, {6, 7, 8}};
  constexpr unsigned long long W0 = pack_rows5(T, 0), W1 = pack_rows5(T, 1), W2 = pack_rows5(T, 2);
  const unsigned long long w = dir == 0 ? W0 : (dir == 1 ? W1 : W2);   // selects, no table in memory
  return (int)((w >> (5 * row)) & 31);
}

template <class R, int O, int M>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_adjoint2(KPtrs p, APtrs ad, LevelArgs a) {
  using RF = edg_gen::Ref<O>;
  using L = AdjLds2<R, O, M>;
  constexpr int B = RF::B, F = RF::F, FP = RF::FP;
  constexpr int MM = M > 0 ? M : 1;
  constexpr int NB0 = RF::MB1, NB1 = B - RF::MB1;
  constexpr int NBX = NB0 > NB1 ? NB0 : NB1;
  constexpr int JW = (NBX + LPE - 1) / LPE;      // owned memory modes per lane
  constexpr int JB = (B + LPE - 1) / LPE;        // memory-variable layout
  constexpr int BS = L::BS, FS = L::FS;
  __shared__ R lds[L::TOTAL];
  __shared__ double gsh[EPW * NGS];
  constexpr int FSTW = 17;
  __shared__ R fst[EPW * 4 * FSTW];
  __shared__ int fbc[EPW * 4];
  __shared__ R emat[EPW * 5];
  __shared__ int eint[EPW * 4];

  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int e = lane / LPE, r = lane % LPE;
  const bool act = e < EPW;
  const int ec = act ? e : EPW - 1;
  const int q = act ? r : 0;
  const int g = blockIdx.x;
  const int elem = g * EPW + ec;
  const int cl = cluster_of(a, g * EPW);
  const bool valid = act && (elem < a.cl_vend[cl]);
  // lane slot of the element-group layouts; re-declared opaque at the top of
  // the long loops, so the compiler recomputes addresses there instead of
  // hoisting (and spilling) one per access
  int slot = ec * LPE + q;
  int base = w ? RF::MB1 : 0;                      // opaque at the loop tops (see slot)
  int jb0 = (base + q) / LPE;                      // memory-variable block of the lane's first owned mode
  const int nb = w ? NB1 : NB0;
  R* const reg = lds + ec * L::REGION;
  R* const grad = reg;
  R* const coup = reg + L::GRAD;
  R* const rx = reg + L::GRAD + L::COUP;
  R* const pm = reg;                               // face area (overlaps grad / coup)
  double* const gs = gsh + ec * NGS;
  const R* P = reinterpret_cast<const R*>(p.P) + (size_t)elem * NPARAM;
  const int* FI = p.FI + (size_t)elem * FI_WORDS;
  R* const Le = reinterpret_cast<R*>(ad.Le) + (size_t)g * B * NSLOT;
  R* const La = reinterpret_cast<R*>(ad.La) + (size_t)g * JB * MM * 6 * NSLOT;
  // the wave's scratch block (AdjScratch2) and this lane's offset in a chunk
  using SC = AdjScratch2<O, M>;
  static_assert(sizeof(R) == 4, "float4 scratch chunks");
  float* const SW = reinterpret_cast<float*>(ad.De) + ((size_t)g * 2 + w) * SC::WAVE_FLOATS;
  int l4 = lane * 4;                               // re-declared opaque at the loop tops (see slot)
  auto stE = [&](int chunk, const R* v) { st_chunks<NBX>(SW + chunk * 256, l4, v); };
  auto ldE = [&](int chunk, R* v) { ld_chunks<NBX>(SW + chunk * 256, l4, v); };
  auto stA = [&](int chunk, const R* v) { st_chunks<6 * MM>(SW + chunk * 256, l4, v); };
  auto ldA = [&](int chunk, R* v) { ld_chunks<6 * MM>(SW + chunk * 256, l4, v); };
  auto st6 = [&](int chunk, const R* v) { st_chunks<6>(SW + chunk * 256, l4, v); };
  auto ld6 = [&](int chunk, R* v) { ld_chunks<6>(SW + chunk * 256, l4, v); };
  const size_t sstride = (size_t)4 * ADJ_ROWS * FP;

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
  // gradient slots this lane writes (forward products) and the star-product
  // reads: stress row ij: lam delta div v + mu (d_j v_i + d_i v_j);
  // velocity row i: rho_inv sum_d d_d sigma_id
  R* const gw0 = grad + aslot(q, 0) * BS;
  R* const gw1 = grad + aslot(q, 1) * BS;
  R* const gw2 = grad + aslot(q, 2) * BS;
  int sa, sb, sc, sd, se;
  if (is_stress) {
    sa = aslot(6, 0) * BS; sb = aslot(7, 1) * BS; sc = aslot(8, 2) * BS;
    sd = aslot(6 + qi, qj) * BS; se = aslot(6 + qj, qi) * BS;
  } else {
    const int i = q - 6;
    sa = aslot(sym_index(i, 0), 0) * BS; sb = aslot(sym_index(i, 1), 1) * BS; sc = aslot(sym_index(i, 2), 2) * BS;
    sd = sa; se = sb;
  }
  // transposed products read this row's gradient adjoints: the used slots, else zeros
  const R* const gt0 = grad + (aslot(q, 0) == 18 ? 19 : aslot(q, 0)) * BS;
  const R* const gt1 = grad + (aslot(q, 1) == 18 ? 19 : aslot(q, 1)) * BS;
  const R* const gt2 = grad + (aslot(q, 2) == 18 ? 19 : aslot(q, 2)) * BS;

  for (int i = threadIdx.x; i < EPW * NGS; i += 128) gsh[i] = 0.0;

  const int nn = step_new_of(a, cl);
  const int eflags = FI[12];
  const bool has_b2 = (eflags & EF_HAS_FINER) != 0;
  const bool has_b3 = (eflags & EF_HAS_COARSER) != 0;
  const bool any_b2 = __syncthreads_or(has_b2);
  const int rec_slot = FI[15];
  // the parameters of each (element, face) pair the transposed surface reads,
  // staged in LDS once (the face items then read no global parameter): the
  // own face words (normal, area weight, outer impedances), the neighbour's
  // 1/rho, lam, mu, Zp, Zs and its words of the shared face; fbc holds the
  // boundary kind and a has-neighbour bit (16)
  {
    const int u = w * LPE + q;
#pragma unroll
    for (int k = 0; k < (4 * FSTW + 2 * LPE - 1) / (2 * LPE); ++k) {
      const int idx = u + 2 * LPE * k;
      if (act && idx < 4 * FSTW) {
        const int i = idx / FSTW, wd = idx % FSTW;
        const int nbr = FI[3 * i], code = FI[3 * i + 1];
        R v = R(0);
        if (wd < 6) {
          v = P[20 + 6 * i + wd];
        } else if (nbr >= 0) {
          const R* Pn = reinterpret_cast<const R*>(p.P) + (size_t)nbr * NPARAM;
          v = wd < 11 ? Pn[9 + (wd - 6)] : Pn[20 + 6 * (code & 15) + (wd - 11)];
        }
        fst[(ec * 4 + i) * FSTW + wd] = v;
        if (wd == 0) fbc[ec * 4 + i] = ((code >> 4) & 15) | (nbr >= 0 ? 16 : 0);
      }
    }
  }
  // the element words the face items of other lanes read: (1/rho, lam, mu,
  // Zp, Zs) and (valid, own B2 slot, own B3 slot, flags)
  if (w == 0 && act && q == 0) {
    emat[ec * 5 + 0] = rho_inv;
    emat[ec * 5 + 1] = lam;
    emat[ec * 5 + 2] = mu;
    emat[ec * 5 + 3] = zp;
    emat[ec * 5 + 4] = zs;
    eint[ec * 4 + 0] = valid ? 1 : 0;
    eint[ec * 4 + 1] = FI[13];
    eint[ec * 4 + 2] = FI[14];
    eint[ec * 4 + 3] = eflags;
  }

  // ---------------------------------------------- forward recompute: D_d, T, T2
  R te[NBX], t2[NBX];
  {
    const R* Se = reinterpret_cast<const R*>(ad.Se) + (size_t)g * B * NSLOT;
    const R* Sa = reinterpret_cast<const R*>(ad.Sa) + (size_t)g * JB * MM * 6 * NSLOT;
    R dm[JW][MM][6];
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb) {
      te[lb] = R(0);
      t2[lb] = R(0);
      if (lb < nb && act) rx[q * BS + base + lb] = at(Se, (base + lb) * NSLOT + slot);
    }
#pragma unroll
    for (int jw = 0; jw < JW; ++jw) {
      const int lb = q + LPE * jw, b = base + lb, jb = jb0 + jw;
#pragma unroll
      for (int l = 0; l < MM; ++l)
#pragma unroll
        for (int c = 0; c < 6; ++c) dm[jw][l][c] = (M > 0 && lb < nb) ? at(Sa, ((jb * MM + l) * 6 + c) * NSLOT + slot) : R(0);
    }
#pragma unroll 1
    for (int d = 0; d < O; ++d) {
      asm volatile("" : "+v"(slot), "+v"(jb0), "+s"(base), "+v"(l4));
      const R c_d = R(a.tc[cl][d]), h_d = R(a.th[cl][d]);
      const bool more = d + 1 < O;
      __syncthreads();
      {
        R dv[NBX];
#pragma unroll
        for (int lb = 0; lb < NBX; ++lb) dv[lb] = lb < nb ? rx[q * BS + base + lb] : R(0);
#pragma unroll
        for (int lb = 0; lb < NBX; ++lb) { te[lb] += c_d * dv[lb]; t2[lb] += h_d * dv[lb]; }
      }
      if (!more) break;
      {
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
            eps[0] = grad[aslot(6, 0) * BS + b];
            eps[1] = grad[aslot(7, 1) * BS + b];
            eps[2] = grad[aslot(8, 2) * BS + b];
            eps[3] = R(0.5) * (grad[aslot(6, 1) * BS + b] + grad[aslot(7, 0) * BS + b]);
            eps[4] = R(0.5) * (grad[aslot(7, 2) * BS + b] + grad[aslot(8, 1) * BS + b]);
            eps[5] = R(0.5) * (grad[aslot(6, 2) * BS + b] + grad[aslot(8, 0) * BS + b]);
            // (the gradient words' pass at the end rebuilds D_d^a from these)
            st6(SC::EP + (d * JW + jw) * SC::C6, eps);
            R cp[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
            for (int l = 0; l < MM; ++l) {
              const R tr = dm[jw][l][0] + dm[jw][l][1] + dm[jw][l][2];
#pragma unroll
              for (int c = 0; c < 6; ++c) cp[c] -= bl[l] * dm[jw][l][c] + (c < 3 ? al[l] * tr : R(0));
#pragma unroll
              for (int c = 0; c < 6; ++c) dm[jw][l][c] = om[l] * (eps[c] - dm[jw][l][c]);
            }
            if (act)
#pragma unroll
              for (int c = 0; c < 6; ++c) coup[c * BS + b] = cp[c];
          }
        }
        // the coupling rows of a mode are read by the stress rows of the
        // wave that owns the mode
        wave_lds_sync();
      }
      // next derivative, own modes, into the row exchange (every lane's
      // full-row reads ended before the barrier after the products)
      {
        R nx[NBX], sab[NBX], sde[NBX];
#pragma unroll
        for (int lb = 0; lb < NBX; ++lb) {
          const int b = base + lb;
          sab[lb] = R(0);
          sde[lb] = R(0);
          if (lb < nb) {
            sab[lb] = grad[sa + b] + grad[sb + b] + grad[sc + b];
            if (is_stress) {
              const R cq = M > 0 ? coup[q * BS + b] : R(0);
              sde[lb] = grad[sd + b] + grad[se + b];
              nx[lb] = lam * delta * sab[lb] + mu * sde[lb] + cq;
            } else {
              nx[lb] = rho_inv * sab[lb];
            }
          }
        }
        // the sums the reverse loop pairs with the adjoint of D_{d+1}
        stE(SC::DG + (d * 2 + 0) * SC::CE, sab);
        stE(SC::DG + (d * 2 + 1) * SC::CE, sde);
        if (act)
#pragma unroll
          for (int lb = 0; lb < NBX; ++lb)
            if (lb < nb) rx[q * BS + base + lb] = nx[lb];
      }
    }
  }
  __syncthreads();

  // ---------------------------------------------- face phases
  // The element's traces (full rows through the row exchange, each wave the
  // traces of faces 2w, 2w+1), then per (face, face mode) the Godunov reverse
  // mode, then the lift of the trace adjoints to the wave's modes.
  R lte[NBX], lt2[NBX];
#pragma unroll
  for (int lb = 0; lb < NBX; ++lb) { lte[lb] = R(0); lt2[lb] = R(0); }
  R* const S0 = reinterpret_cast<R*>(ad.S0);
  R* const S1 = reinterpret_cast<R*>(ad.S1);
  R* const S2 = reinterpret_cast<R*>(ad.S2);
  R* const S3 = reinterpret_cast<R*>(ad.S3);
  const int slot2 = FI[13], slot3 = FI[14];
  auto face_phase = [&](const bool b2phase, const R (&tint)[NBX], R (&acc)[NBX]) {
    if (act)
#pragma unroll
      for (int lb = 0; lb < NBX; ++lb)
        if (lb < nb) rx[q * BS + base + lb] = tint[lb];
    __syncthreads();
    {
      R full[B], pt[2 * FP];
#pragma unroll
      for (int b = 0; b < B; ++b) full[b] = rx[q * BS + b];
      if (w == 0) RF::trace_p0(full, pt); else RF::trace_p1(full, pt);
      if (act)
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
          for (int f = 0; f < FP; ++f) pm[(RF::tface(w, ii) * LPE + q) * FS + f] = pt[ii * FP + f];
    }
    __syncthreads();
    // items (face i, mode f) of the whole group, one 16-lane DPP row per
    // (element, face) pair: row r = 8 rr + 4 w + lane / 16 takes element
    // r % 7 and face r / 7 (r < 28), lane f = lane % 16 its mode f (f < F).
    // A row's 15 modes are contiguous in the slot buffers and in the trace
    // area, and its gradient words are summed over the row with DPP and added
    // once by the row's last lane (which holds no item): the LDS atomics are
    // one lane per row instead of nine lanes per element.
    const int f = lane & 15;
#pragma unroll 1
    for (int rr = 0; rr < (4 * EPW + 7) / 8; ++rr) {
      const int r8 = 8 * rr + 4 * w + (lane >> 4);
      const bool pair = r8 < 4 * EPW;
      const int pe = pair ? r8 % EPW : 0, i = pair ? r8 / EPW : 0;
      const int* const ei = eint + pe * 4;
      const bool pvalid = pair && ei[0] != 0;
      const int fb = fbc[pe * 4 + i];
      const int bc = fb & 15;
      const bool nflux = (fb & 16) && pvalid;             // a neighbour across face i
      R pbo[7], pbn[7];
#pragma unroll
      for (int k = 0; k < 7; ++k) { pbo[k] = R(0); pbn[k] = R(0); }
      if (pair && f < F) {
        const size_t pel = (size_t)g * EPW + pe;
        const int eflg = ei[3];
        // every global operand of the item first, into registers zeroed
        // beforehand, and no use inside the branches that load them: one
        // memory latency per item
        R u0[15], ua[15], ub[15];
#pragma unroll
        for (int k = 0; k < 15; ++k) { u0[k] = R(0); ua[k] = R(0); ub[k] = R(0); }
        if (!b2phase) {
          const R* x = S0 + pel * sstride + (size_t)i * ADJ_ROWS * FP + f;
#pragma unroll
          for (int k = 0; k < 15; ++k)
            if (M > 0 || k < 9) u0[k] = x[k * FP];
        }
        R* const s1 = !nflux ? nullptr
                      : b2phase ? ((eflg & EF_HAS_FINER) ? S2 + (size_t)ei[1] * sstride : nullptr)
                                : S1 + pel * sstride;
        R* const s3 = (nflux && !b2phase && (eflg & EF_HAS_COARSER)) ? S3 + (size_t)ei[2] * sstride : nullptr;
        if (s1) {
          const R* x = s1 + (size_t)i * ADJ_ROWS * FP + f;
#pragma unroll
          for (int k = 0; k < 15; ++k)
            if (M > 0 || k < 9) ua[k] = x[k * FP];
        }
        if (s3) {
          const R* x = s3 + (size_t)i * ADJ_ROWS * FP + f;
#pragma unroll
          for (int k = 0; k < 15; ++k)
            if (M > 0 || k < 9) ub[k] = x[k * FP];
        }
        const R* const fs = fst + (pe * 4 + i) * FSTW;
        const R* const em = emat + pe * 5;
        R fpv[6], pnv[5], fnv[6], ev[5];
#pragma unroll
        for (int k = 0; k < 6; ++k) fpv[k] = fs[k];
#pragma unroll
        for (int k = 0; k < 5; ++k) pnv[k] = fs[6 + k];
#pragma unroll
        for (int k = 0; k < 6; ++k) fnv[k] = fs[11 + k];
#pragma unroll
        for (int k = 0; k < 5; ++k) ev[k] = em[k];
        // the slots read are cleared (B3 only after its even step)
        if (s1) {
          R* x = s1 + (size_t)i * ADJ_ROWS * FP + f;
#pragma unroll
          for (int k = 0; k < 15; ++k) x[k * FP] = R(0);
        }
        if (s3 && (nn & 1) == 0) {
          R* x = s3 + (size_t)i * ADJ_ROWS * FP + f;
#pragma unroll
          for (int k = 0; k < 15; ++k) x[k * FP] = R(0);
        }
        R u1[15];
#pragma unroll
        for (int k = 0; k < 15; ++k) u1[k] = ua[k] + ub[k];
        R* const pmp = lds + pe * L::REGION;             // the trace area of element pe
        R tr[9], zero9[9], tb[9], ob[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) { tr[k] = pmp[(i * LPE + k) * FS + f]; zero9[k] = R(0); tb[k] = R(0); ob[k] = R(0); }
        if (!b2phase) {
          // own flux: the element's trace is the inside state; its
          // (rho_inv, lam, mu, Zp, Zs) are ev
          const R zpp = bc == 0 ? fpv[4] : ev[3], zsp = bc == 0 ? fpv[5] : ev[4];
          godunov_adj<R>(u0, tr, zero9, fpv[0], fpv[1], fpv[2], ev[3], ev[4], zpp, zsp, ev[1], ev[2], ev[0], fpv[3], bc,
                         tb, ob, pbo);
        }
        if (nflux) {
          // the neighbour's flux reads this element's buffer: B1 (+ B3) or B2
          if (M == 0)
#pragma unroll
            for (int k = 9; k < 15; ++k) u1[k] = R(0);
          // (rho_inv, lam, mu, Zp, Zs) of the neighbour are its words 9..13
          godunov_adj<R>(u1, zero9, tr, fnv[0], fnv[1], fnv[2], pnv[3], pnv[4], fnv[4], fnv[5], pnv[1], pnv[2], pnv[0],
                         fnv[3], 0, ob, tb, pbn);
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) pmp[(i * LPE + k) * FS + f] = tb[k];
      }
      // the row sums, every lane taking part (uniform control flow)
      R so[7], sn[7];
#pragma unroll
      for (int k = 0; k < 7; ++k) { so[k] = row_sum16(pbo[k]); sn[k] = row_sum16(pbn[k]); }
      if (f == 15 && pvalid) {
        double* const gp = gsh + pe * NGS;
        if (!b2phase) {
#pragma unroll
          for (int k = 0; k < 5; ++k) gadd(gp, k, so[k]);
          gadd(gp, bc == 0 ? 11 + 2 * i : 3, so[5]);
          gadd(gp, bc == 0 ? 12 + 2 * i : 4, so[6]);
        }
        if (nflux)
#pragma unroll
          for (int k = 0; k < 7; ++k) gadd(gp, 19 + 7 * i + k, sn[k]);
      }
    }
    __syncthreads();
    {
      R pf[4 * FP];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int f = 0; f < FP; ++f) pf[i * FP + f] = pm[(i * LPE + q) * FS + f];
      // lifted into a fresh array, then added: accumulating into acc inside
      // the two branches lets the compiler merge their first accesses through
      // a pointer select, which keeps two entries of acc in scratch memory
      R lr[NBX];
#pragma unroll
      for (int lb = 0; lb < NBX; ++lb) lr[lb] = R(0);
      if (w == 0) RF::lift_p0(pf, lr); else RF::lift_p1(pf, lr);
#pragma unroll
      for (int lb = 0; lb < NBX; ++lb) acc[lb] += lr[lb];
    }
    __syncthreads();
  };
  if (any_b2) face_phase(true, t2, lt2);
  face_phase(false, te, lte);

  // ---------------------------------------------- volume kernel
  // V = -(lam delta div v + mu (d_j v_i + d_i v_j)) (stress), -rho_inv div sigma (velocity), -omega_l eps (memory)
  R le[NBX];
#pragma unroll
  for (int lb = 0; lb < NBX; ++lb) le[lb] = lb < nb ? at(Le, (base + lb) * NSLOT + slot) : R(0);
  stE(SC::LE, le);                                 // for the reverse loop's coupling blocks
  auto la_at = [&](int jb, int l, int c) -> R& { return at(La, ((jb * MM + l) * 6 + c) * NSLOT + slot); };
  if (act)
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb)
      if (lb < nb) rx[q * BS + base + lb] = te[lb];
  __syncthreads();
  {
    R full[B];
#pragma unroll
    for (int b = 0; b < B; ++b) full[b] = rx[q * BS + b];
    if (w == 0) RF::vol_grad_p0(full, G, gw0, gw1, gw2);
    else RF::vol_grad_p1(full, G, gw0, gw1, gw2);
  }
  if (threadIdx.x < 64 && act)      // zero row for the transposed products (written once, never overwritten)
    for (int b = q; b < BS; b += LPE) grad[19 * BS + b] = R(0);
  __syncthreads();
  // star-product adjoint pairings with the forward gradients: dV/dlam, dV/dmu, dV/drho_inv
  auto star_sums = [&](const R* ad_own, const R* ab, const R* de, const double sign) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb)
      if (lb < nb) {
        s0 += (double)(ad_own[lb] * ab[lb]);
        if (is_stress) s1 += (double)(ad_own[lb] * de[lb]);
      }
    if (valid) {
      if (is_stress) {
        if (q < 3) gadd(gs, 1, sign * s0);
        gadd(gs, 2, sign * s1);
      } else {
        gadd(gs, 0, sign * s0);
      }
    }
  };
  // the same pairing with the sums read from the gradient slots
  auto star_grams = [&](const R* ad_own, const double sign) {
    R ab[NBX], de[NBX];
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb) {
      const int b = base + lb;
      ab[lb] = R(0);
      de[lb] = R(0);
      if (lb < nb) {
        ab[lb] = grad[sa + b] + grad[sb + b] + grad[sc + b];
        if (is_stress) de[lb] = grad[sd + b] + grad[se + b];
      }
    }
    star_sums(ad_own, ab, de, sign);
  };
  star_grams(le, -1.0);
  // exchange: elastic adjoint rows, omega-weighted memory-variable adjoints
  // (own modes: the rows and coupling rows write_gb reads are written by
  // its own wave; the barrier below also ends every star-product read of
  // the gradient slots before write_gb overwrites them)
  if (act)
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb)
      if (lb < nb) rx[q * BS + base + lb] = le[lb];
  if (M > 0) {
#pragma unroll
    for (int jw = 0; jw < JW; ++jw) {
      const int lb = q + LPE * jw, b = base + lb, jb = jb0 + jw;
      R lv[6 * MM];
#pragma unroll
      for (int l = 0; l < MM; ++l)
#pragma unroll
        for (int c = 0; c < 6; ++c) lv[l * 6 + c] = lb < nb ? la_at(jb, l, c) : R(0);
      stA(SC::LA + jw * SC::CA, lv);               // for the final Qbar^a update
      // Lambda_d = sum_l omega_l^2 C_l(d) Qbar^a_l, C_l(d) = sum_{k >= d}
      // (-omega_l)^(k - d) c_k: the Qbar^a part of the omega-weighted
      // memory-variable adjoints of step d (see the reverse loop)
      {
        R Cl[MM];
#pragma unroll
        for (int l = 0; l < MM; ++l) Cl[l] = R(0);
#pragma unroll
        for (int d = O - 1; d >= 0; --d) {
          const R c_d = R(a.tc[cl][d]);
          R lm[6];
#pragma unroll
          for (int l = 0; l < MM; ++l) Cl[l] = c_d - om[l] * Cl[l];
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            lm[c] = R(0);
#pragma unroll
            for (int l = 0; l < MM; ++l) lm[c] += om[l] * om[l] * Cl[l] * lv[l * 6 + c];
          }
          if (lb < nb) st6(SC::LM + (d * JW + jw) * SC::C6, lm);
        }
      }
      if (lb < nb && act)
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          R v = R(0);
#pragma unroll
          for (int l = 0; l < MM; ++l) v += om[l] * lv[l * 6 + c];
          coup[c * BS + b] = v;
        }
    }
  }
  __syncthreads();
  // gradient-entry adjoints of this row, own modes, into its slots (sign s:
  // -1 for the volume kernel, +1 for the time kernel's next derivative)
  // Branch-free: every lane forms its three (row, direction) entries as
  //   A rx[r] + C coup[c] + L (rx[0] + rx[1] + rx[2]):
  // velocity row i, direction k: A = (1 + delta_ik) mu on exchange row
  //   sym(i, k), C = 1 (i = k) or 1/2 on coupling row sym(i, k) (anelastic
  //   only), L = delta_ik lam on the normal-stress rows;
  // stress row (qi, qj), direction k in {qi, qj}: A = rho_inv on the velocity
  //   row of the other index; directions a stress row does not use write nothing
  auto write_gb = [&](const R sgn) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      int rrow, crow;
      R A, C, Lw;
      bool wr;
      if (!is_stress) {
        const int i = q - 6, sk = sym_index(i, k);
        rrow = sk;
        crow = sk;
        A = (i == k ? R(2) : R(1)) * mu;
        C = i == k ? R(1) : R(0.5);
        Lw = i == k ? lam : R(0);
        wr = act;
      } else {
        const int iv = k == qj ? qi : (k == qi ? qj : -1);
        rrow = 6 + (iv < 0 ? 0 : iv);
        crow = 0;
        A = rho_inv;
        C = R(0);
        Lw = R(0);
        wr = act && iv >= 0;
      }
      // all reads of a direction, then its stores (the stores may alias the
      // exchange rows for the compiler, so interleaving them would serialise
      // every read behind the previous store)
      R v[NBX];
#pragma unroll
      for (int lb = 0; lb < NBX; ++lb) {
        const int b = base + lb;
        v[lb] = R(0);
        if (lb < nb) {
          v[lb] = A * rx[rrow * BS + b] + Lw * (rx[b] + rx[BS + b] + rx[2 * BS + b]);
          if (M > 0) v[lb] += C * coup[crow * BS + b];
        }
      }
      R* const dst = grad + aslot(q, k) * BS;
      if (wr)
#pragma unroll
        for (int lb = 0; lb < NBX; ++lb)
          if (lb < nb) dst[base + lb] = sgn * v[lb];
    }
  };
  write_gb(R(-1));
  __syncthreads();
  if (w == 0) RF::vol_grad_T_p0(gt0, gt1, gt2, G, lte);
  else RF::vol_grad_T_p1(gt0, gt1, gt2, G, lte);
  // the time-integral adjoints wait in memory (re-read with each
  // derivative's data), so they hold no registers across the loop below
  stE(SC::DT, lte);
  stE(SC::DT + SC::CE, lt2);
  // (no barrier: the reverse loop's first LDS writes are the wave's own
  // modes of the exchange rows, which the transposed product does not read)

  // ---------------------------------------------- time kernel backwards
  // nbe: adjoint of the next elastic derivative (registers); the
  // memory-variable adjoints are not carried: each step forms their
  // omega-weighted sum from the coupling adjoints of the steps before it
  R nbe[NBX];
#pragma unroll
  for (int lb = 0; lb < NBX; ++lb) nbe[lb] = R(0);
  R* const recDb = reinterpret_cast<R*>(ad.recDb);
#pragma unroll 1
  for (int d = O - 1; d >= 0; --d) {
    asm volatile("" : "+v"(slot), "+v"(jb0), "+s"(base), "+v"(l4));
    const R c_d = R(a.tc[cl][d]), h_d = R(a.th[cl][d]);
    const bool more = d + 1 < O;
    R cur[NBX];
    // the step's scratch operands in one batch: the time-integral adjoints
    // and the star-product sums of grad D_d (kept by the recompute) for the
    // material pairings
    R ab[NBX], de[NBX];
    {
      R x1[NBX], x2[NBX];
#pragma unroll
      for (int lb = 0; lb < NBX; ++lb) { x1[lb] = R(0); x2[lb] = R(0); ab[lb] = R(0); de[lb] = R(0); }
      ldE(SC::DT, x1);
      ldE(SC::DT + SC::CE, x2);
      if (more) {
        ldE(SC::DG + (2 * d) * SC::CE, ab);
        ldE(SC::DG + (2 * d + 1) * SC::CE, de);
      }
#pragma unroll
      for (int lb = 0; lb < NBX; ++lb) cur[lb] = c_d * x1[lb] + h_d * x2[lb];
    }
    if (rec_slot >= 0 && valid) {
      R* rd = recDb + (((size_t)rec_slot * O + d) * LPE + q) * B + base;
#pragma unroll
      for (int lb = 0; lb < NBX; ++lb)
        if (lb < nb) { cur[lb] += rd[lb]; rd[lb] = R(0); }
    }
    if (more) {
      star_sums(nbe, ab, de, 1.0);
      if (act)
#pragma unroll
        for (int lb = 0; lb < NBX; ++lb)
          if (lb < nb) rx[q * BS + base + lb] = nbe[lb];
      // (coup holds the omega-weighted sums of the next memory-variable
      // adjoint, written by the coupling block of the step before)
      __syncthreads();
      write_gb(R(1));
      __syncthreads();
      if (w == 0) RF::ck_grad_T_p0(gt0, gt1, gt2, G, cur);
      else RF::ck_grad_T_p1(gt0, gt1, gt2, G, cur);
      // (no barrier: the coupling block below writes the wave's own modes of
      // the exchange and coupling rows, which the transposed product does
      // not read; the next iteration's products follow its first barrier)
    }
    if (M > 0) {
      // the coupling E: cq_d enters the volume term c_d cq_d and the next
      // derivative.  The scratch operands of a mode block (Lambda_d and the
      // coupling adjoints of the later steps) are loaded in one batch.
      if (is_stress && act) {
        R lev[NBX];
        ldE(SC::LE, lev);
#pragma unroll
        for (int lb = 0; lb < NBX; ++lb)
          if (lb < nb) rx[q * BS + base + lb] = c_d * lev[lb] + (more ? nbe[lb] : R(0));
      }
      // the stress rows of a mode are read by its owner, in the same wave
      wave_lds_sync();
      // The adjoint of D_d^a in closed form: with s_l(k) = b_l cq_k + a_l
      // tr(cq_k) I (cq_k: the coupling adjoint of step k),
      //   abar_{l,d} = -omega_l C_l(d) Qbar^a_l - sum_{k >= d} (-omega_l)^(k-d) s_l(k),
      // so its omega-weighted sum over l, which the next (lower) derivative
      // needs, is -Lambda_d - sum_{k >= d} (beta_{k-d} cq_k + alpha_{k-d}
      // tr(cq_k) I) with beta_j = sum_l omega_l (-omega_l)^j b_l (alpha_j with
      // a_l).  The scratch keeps cq_k (six words) instead of the carried
      // adjoints of every mechanism.
      R bet[O], alp[O];
#pragma unroll
      for (int j = 0; j < O; ++j) { bet[j] = R(0); alp[j] = R(0); }
#pragma unroll
      for (int l = 0; l < MM; ++l) {
        R pw = om[l];
#pragma unroll
        for (int j = 0; j < O; ++j) {
          bet[j] += pw * bl[l];
          alp[j] += pw * al[l];
          pw *= -om[l];
        }
      }
#pragma unroll
      for (int jw = 0; jw < JW; ++jw) {
        const int lb = q + LPE * jw, b = base + lb;
        if (lb < nb) {
          R cqb[6], lm[6], hk[O - 1][6];
#pragma unroll
          for (int c = 0; c < 6; ++c) cqb[c] = rx[c * BS + b];
          ld6(SC::LM + (d * JW + jw) * SC::C6, lm);
#pragma unroll
          for (int kk = 0; kk < O - 1; ++kk) {
#pragma unroll
            for (int c = 0; c < 6; ++c) hk[kk][c] = R(0);
            if (d + 1 + kk < O) ld6(SC::HS + ((d + 1 + kk) * JW + jw) * SC::C6, hk[kk]);
          }
          st6(SC::HS + (d * JW + jw) * SC::C6, cqb);
          R ws[6];
          const R cqt = cqb[0] + cqb[1] + cqb[2];
#pragma unroll
          for (int c = 0; c < 6; ++c) ws[c] = -lm[c] - bet[0] * cqb[c] - (c < 3 ? alp[0] * cqt : R(0));
#pragma unroll
          for (int kk = 0; kk < O - 1; ++kk) {
            const R ht = hk[kk][0] + hk[kk][1] + hk[kk][2];
#pragma unroll
            for (int c = 0; c < 6; ++c) ws[c] -= bet[kk + 1] * hk[kk][c] + (c < 3 ? alp[kk + 1] * ht : R(0));
          }
          // the coupling term of the next (lower) derivative's adjoint: coup
          // is not touched again before the next step reads it
          if (act)
#pragma unroll
            for (int c = 0; c < 6; ++c) coup[c * BS + b] = ws[c];
        }
      }
      wave_lds_sync();
    }
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb) nbe[lb] = cur[lb];
  }
  // Qbar += the adjoint of D_0: every load first, then every store (a
  // read-modify-write per word would wait one memory latency per word: the
  // compiler must assume each store may alias the next load)
  if (valid) {
    R xe[NBX];
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb) xe[lb] = R(0);
    ldE(SC::LE, xe);                               // Qbar as staged (unchanged until here)
#pragma unroll
    for (int lb = 0; lb < NBX; ++lb)
      if (lb < nb) at(Le, (base + lb) * NSLOT + slot) = xe[lb] + nbe[lb];
  }
  double gab[2 * MM];
#pragma unroll
  for (int k = 0; k < 2 * MM; ++k) gab[k] = 0.0;
  if (M > 0 && valid) {
    // per owned mode block: Qbar^a_l += abar_{l,0} = -omega_l C_l(0) Qbar^a_l
    // - sum_k (-omega_l)^k s_l(k); and the anelastic-weight words
    // -sum_d cq_d . D_d^a_l (tensor and trace parts), with D_d^a rebuilt
    // from the state's memory variables and the stored strain rates by the
    // forward recursion of the time kernel
    const R* Sa = reinterpret_cast<const R*>(ad.Sa) + (size_t)g * JB * MM * 6 * NSLOT;
    R Cl0[MM];
#pragma unroll
    for (int l = 0; l < MM; ++l) {
      Cl0[l] = R(0);
#pragma unroll
      for (int d = O - 1; d >= 0; --d) Cl0[l] = R(a.tc[cl][d]) - om[l] * Cl0[l];
    }
#pragma unroll
    for (int jw = 0; jw < JW; ++jw) {
      const int lb = q + LPE * jw, jb = jb0 + jw;
      if (lb < nb) {
        R xl[6 * MM], h[O][6], ep[O - 1][6], dm[MM][6];
        ldA(SC::LA + jw * SC::CA, xl);
#pragma unroll
        for (int k = 0; k < O; ++k) ld6(SC::HS + (k * JW + jw) * SC::C6, h[k]);
#pragma unroll
        for (int k = 0; k < O - 1; ++k) ld6(SC::EP + (k * JW + jw) * SC::C6, ep[k]);
#pragma unroll
        for (int l = 0; l < MM; ++l)
#pragma unroll
          for (int c = 0; c < 6; ++c) dm[l][c] = at(Sa, ((jb * MM + l) * 6 + c) * NSLOT + slot);
#pragma unroll
        for (int l = 0; l < MM; ++l)
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            R v = -om[l] * Cl0[l] * xl[l * 6 + c];
            R pw = R(1);
#pragma unroll
            for (int k = 0; k < O; ++k) {
              const R ht = h[k][0] + h[k][1] + h[k][2];
              v -= pw * (bl[l] * h[k][c] + (c < 3 ? al[l] * ht : R(0)));
              pw *= -om[l];
            }
            la_at(jb, l, c) = xl[l * 6 + c] + v;
          }
#pragma unroll
        for (int d = 0; d < O; ++d) {
          const R cqt = h[d][0] + h[d][1] + h[d][2];
#pragma unroll
          for (int l = 0; l < MM; ++l) {
            const R tr = dm[l][0] + dm[l][1] + dm[l][2];
            gab[2 * l] -= (double)(cqt * tr);
#pragma unroll
            for (int c = 0; c < 6; ++c) gab[2 * l + 1] -= (double)(h[d][c] * dm[l][c]);
          }
          if (d + 1 < O)
#pragma unroll
            for (int l = 0; l < MM; ++l)
#pragma unroll
              for (int c = 0; c < 6; ++c) dm[l][c] = om[l] * (ep[d][c] - dm[l][c]);
        }
      }
    }
  }
  if (M > 0) {
    // the two waves add their words one after the other (LDS atomics of both
    // at once would sum in a timing-dependent order: results would not
    // repeat bit for bit)
    if (w == 0 && valid)
#pragma unroll
      for (int k = 0; k < 2 * MM; ++k) gadd(gs, 5 + k, gab[k]);
    __syncthreads();
    if (w == 1 && valid)
#pragma unroll
      for (int k = 0; k < 2 * MM; ++k) gadd(gs, 5 + k, gab[k]);
  }
  __syncthreads();
  // the element's gradient words, split between the two waves, loads first
  if (valid) {
    constexpr int NI = (NG + 2 * LPE - 1) / (2 * LPE);
    double* const gg = ad.gacc + (size_t)elem * NG;
    double x[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int i = q + LPE * (w + 2 * k);
      x[k] = i < NG ? gg[i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const int i = q + LPE * (w + 2 * k);
      if (i < NG) gg[i] = x[k] + gsh[ec * NGS + i];
    }
  }
}

// Chain rule from the per-element gradient words to d/d(rho, vp, vs), one
// thread per element (internal order), gathering what the face neighbours
// accumulated about this element.  mat [Kp][3 + 2m]: rho, vp, vs, Yp_l, Ys_l
// (rho = 0 marks padding).  out [Kp][3].
__device__ __forceinline__ void add_param(double* g, int which, double v, double rho, double vp, double vs) {
  switch (which) {
    case 0: g[0] -= v / (rho * rho); break;                                              // 1/rho
    case 1: g[0] += v * (vp * vp - 2 * vs * vs); g[1] += v * 2 * rho * vp; g[2] -= v * 4 * rho * vs; break;  // lam
    case 2: g[0] += v * vs * vs; g[2] += v * 2 * rho * vs; break;                        // mu
    case 3: g[0] += v * vp; g[1] += v * rho; break;                                       // Zp
    default: g[0] += v * vs; g[2] += v * rho; break;                                      // Zs
  }
}

__global__ void k_material_gradient(const double* gacc, const int* FI, const double* mat, int M, long long Kp,
                                    double* out) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= Kp) return;
  const int mw = 3 + 2 * M;
  const double rho = mat[k * mw], vp = mat[k * mw + 1], vs = mat[k * mw + 2];
  double g[3] = {0.0, 0.0, 0.0};
  if (rho > 0.0) {
    const double* x = gacc + k * NG;
    for (int t = 0; t < 5; ++t) add_param(g, t, x[t], rho, vp, vs);
    for (int l = 0; l < M; ++l) {   // a_l = rho vp^2 Yp - 2 rho vs^2 Ys, b_l = 2 rho vs^2 Ys
      const double yp = mat[k * mw + 3 + 2 * l], ys = mat[k * mw + 4 + 2 * l];
      const double ga = x[5 + 2 * l], gb = x[6 + 2 * l];
      g[0] += ga * (vp * vp * yp - 2 * vs * vs * ys) + gb * 2 * vs * vs * ys;
      g[1] += ga * 2 * rho * vp * yp;
      g[2] += -ga * 4 * rho * vs * ys + gb * 4 * rho * vs * ys;
    }
    const int* fi = FI + k * FI_WORDS;
    for (int i = 0; i < 4; ++i) {
      const int n = fi[3 * i];
      if (n < 0) continue;
      const int j = fi[3 * i + 1] & 15;          // the neighbour's face towards this element
      const double* y = x + 19 + 7 * i;          // this element's Zp, Zs in the neighbour's flux
      add_param(g, 3, y[5], rho, vp, vs);
      add_param(g, 4, y[6], rho, vp, vs);
      const double* xn = gacc + (long long)n * NG;
      add_param(g, 3, xn[11 + 2 * j], rho, vp, vs);   // this element's impedances in the neighbour's own flux
      add_param(g, 4, xn[12 + 2 * j], rho, vp, vs);
      const double* yn = xn + 19 + 7 * j;             // this element's own flux, accumulated by the neighbour
      for (int t = 0; t < 5; ++t) add_param(g, t, yn[t], rho, vp, vs);
    }
  }
  out[k * 3] = g[0];
  out[k * 3 + 1] = g[1];
  out[k * 3 + 2] = g[2];
}

// adjoint of the receiver samples: the derivatives of the receiver slots get
// sum_s (t_s - t^n)^d / d! * seisbar_s phi(x_r) for the samples in the step
// that starts at this level
template <class R, int O, int M>
__global__ void k_receivers_adj(KPtrs p, APtrs ad, LevelArgs a, RecArgs r, const double* seis_b) {
  constexpr int B = edg_gen::Ref<O>::B;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int rec = t / LPE, q = t % LPE;
  if (rec >= r.n) return;
  const int elem = r.elem[rec];
  if (elem >= a.end) return;
  const int cl = cluster_of(a, elem);
  const double dt = a.dt[cl];
  const int n = step_new_of(a, cl);
  const double t0 = (double)n * dt, t1 = (double)(n + 1) * dt;
  double vb[O];
  for (int d = 0; d < O; ++d) vb[d] = 0.0;
  // the samples of step n: [t0 - eps, t1 - eps), eps = 1e-9 dt (as sampled)
  const double eps = 1e-9 * dt, lo = t0 - eps, hi = t1 - eps;
  long long s = (long long)floor(lo / r.dt_sample) - 1;
  if (s < 0) s = 0;
  bool any = false;
  for (; s < r.ns && (double)s * r.dt_sample < hi; ++s) {
    const double ts = (double)s * r.dt_sample;
    if (ts < lo) continue;
    const double x = ts - t0, sb = seis_b[((size_t)rec * r.ns + s) * LPE + q];
    double pw = 1.0, fact = 1.0;
    for (int d = 0; d < O; ++d) {
      vb[d] += pw / fact * sb;
      pw *= x;
      fact *= (double)(d + 1);
    }
    any = true;
  }
  if (!any) return;
  R* D = reinterpret_cast<R*>(ad.recDb) + (size_t)r.slot[rec] * O * LPE * B;
  for (int d = 0; d < O; ++d)
    for (int b = 0; b < B; ++b) atomicAdd(&D[((size_t)d * LPE + q) * B + b], R(vb[d] * r.phi[(size_t)rec * B + b]));
}

}  // namespace

template <class R, int O, int M>
int launch_adjoint(const KPtrs& p, const APtrs& ad, const LevelArgs& a, hipStream_t st) {
  const int groups = (a.end + EPW - 1) / EPW;
  if (groups <= 0) return 0;
  if (a.kind == KIND_ADJ_UPDATE)
    hipLaunchKernelGGL((k_adjoint<R, O, M, true>), dim3(groups), dim3(64), 0, st, p, ad, a);
  else if constexpr (std::is_same<R, float>::value && O >= 4)
    hipLaunchKernelGGL((k_adjoint2<R, O, M>), dim3(groups), dim3(128), 0, st, p, ad, a);
  else
    hipLaunchKernelGGL((k_adjoint<R, O, M, false>), dim3(groups), dim3(64), 0, st, p, ad, a);
  return (int)hipGetLastError();
}

template <class R, int O, int M>
size_t adjoint_scratch_floats() {
  if constexpr (std::is_same<R, float>::value && O >= 4) return (size_t)2 * AdjScratch2<O, M>::WAVE_FLOATS;
  else return (size_t)O * edg_gen::Ref<O>::B * NSLOT;   // the one-wave kernel's time derivatives
}

template <class R, int O, int M>
int launch_receivers_adj(const KPtrs& p, const APtrs& ad, const LevelArgs& a, const RecArgs& r, const double* seis_b,
                         hipStream_t st) {
  if (r.n <= 0) return 0;
  const int total = r.n * LPE;
  hipLaunchKernelGGL((k_receivers_adj<R, O, M>), dim3((total + 127) / 128), dim3(128), 0, st, p, ad, a, r, seis_b);
  return (int)hipGetLastError();
}

int launch_material_gradient(const double* gacc, const int* FI, const double* mat, int M, long long Kp, double* out,
                             hipStream_t st) {
  if (Kp <= 0) return 0;
  hipLaunchKernelGGL(k_material_gradient, dim3((unsigned)((Kp + 255) / 256)), dim3(256), 0, st, gacc, FI, mat, M, Kp,
                     out);
  return (int)hipGetLastError();
}

#define EDG_ADJ_INST(R, O, M)                                                                    \
  template int launch_adjoint<R, O, M>(const KPtrs&, const APtrs&, const LevelArgs&, hipStream_t); \
  template size_t adjoint_scratch_floats<R, O, M>();                                              \
  template int launch_receivers_adj<R, O, M>(const KPtrs&, const APtrs&, const LevelArgs&, const RecArgs&, \
                                             const double*, hipStream_t);

EDG_FOR_EACH_VARIANT(EDG_ADJ_INST)

}  // namespace edg

// Host evaluation of the face flux and its reverse mode (FP64), for CPU
// checks of the adjoint's flux transpose.  prm = (nx, ny, nz, zpm, zsm, zpp,
// zsp, lam, mu, rho_inv, s); out [15]; qm_b, qp_b [9] and pb [7] are
// overwritten with the adjoint of the outputs u [15].
extern "C" int edg_godunov_host(int32_t bc, const double* qm, const double* qp, const double* prm, const double* u,
                                double* out, double* qm_b, double* qp_b, double* pb) {
  if (!qm || !qp || !prm || !u || !out || !qm_b || !qp_b || !pb || bc < 0 || bc > 2) return -1;
  edg::godunov<double>(qm, qp, prm[0], prm[1], prm[2], prm[3], prm[4], prm[5], prm[6], prm[7], prm[8], prm[9],
                       prm[10], bc, out);
  for (int k = 0; k < 9; ++k) qm_b[k] = qp_b[k] = 0.0;
  for (int k = 0; k < 7; ++k) pb[k] = 0.0;
  edg::godunov_adj<double>(u, qm, qp, prm[0], prm[1], prm[2], prm[3], prm[4], prm[5], prm[6], prm[7], prm[8], prm[9],
                           prm[10], bc, qm_b, qp_b, pb);
  return 0;
}
