// Interface between the host library and the adjoint kernels (internal).
#pragma once
#include "kernels.hpp"

namespace edg {

// ---- discrete adjoint (one run)
constexpr int KIND_ADJ_PREDICT = 3;  // transpose of a step's prediction (+ volume, own surface part)
constexpr int KIND_ADJ_UPDATE = 4;   // transpose of the neighbour-data part of a step's surface update
constexpr int ADJ_ROWS = 15;         // adjoint face rows: 9 elastic + 6 omega-weighted memory-variable sums
// Per-element gradient words (internal order, FP64): derivatives of the
// adjoint pairing in the parameters the kernels read.
//   [0] 1/rho  [1] lam  [2] mu  [3] Zp  [4] Zs  [5+2l] a_l  [6+2l] b_l
//   [11+2i], [12+2i]  the neighbour impedances Zp, Zs of face i (own flux)
//   [19+7f+0..6]      (1/rho, lam, mu, Zp, Zs, Zp+, Zs+) of the flux of the
//                     element across face f (its neighbour-data part)
constexpr int NG = 48;

struct APtrs {
  void* Le;          // adjoint of the elastic rows (Qe layout)
  void* La;          // adjoint of the memory variables (Qa layout)
  const void* Se;    // forward state at the start of the step (Qe layout)
  const void* Sa;    // (Qa layout)
  void* S0;          // [Kp][4][15][FP] face adjoints of the element's own flux (its last finished step)
  void* S1;          // [Kp][4][15][FP] adjoint face data for the element's B1 (per own face)
  void* S2;          // [N2][4][15][FP] for B2
  void* S3;          // [N3][4][15][FP] for B3
  void* De;          // scratch: adjoint_scratch_floats() words per element group
  void* Da;          // scratch: [G][O][JB][m][6][63]
  double* gacc;      // [Kp][NG]
  void* recDb;       // [slots][O][9][B] adjoint of the receiver derivatives
};

// d/d(rho, vp, vs) [Kp][3] from the gradient words (mat [Kp][3 + 2m]: rho,
// vp, vs, Yp_l, Ys_l in internal order; rho = 0 for padding)
int launch_material_gradient(const double* gacc, const int* FI, const double* mat, int M, long long Kp, double* out,
                             hipStream_t st);

template <class R, int O, int M>
int launch_adjoint(const KPtrs& p, const APtrs& ad, const LevelArgs& a, hipStream_t st);
// words of De per element group for the transposed prediction of this variant
template <class R, int O, int M>
size_t adjoint_scratch_floats();
template <class R, int O, int M>
int launch_receivers_adj(const KPtrs& p, const APtrs& ad, const LevelArgs& a, const RecArgs& r, const double* seis_b,
                         hipStream_t st);

}  // namespace edg
