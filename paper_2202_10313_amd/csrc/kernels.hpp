// Interface between the host library and the HIP kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace edg {

constexpr int MAX_CLUSTERS = 5;
constexpr int MAX_ORDER = 5;
constexpr int MAX_MECH = 3;
constexpr int NPARAM = 48;  // per-element parameter words (see host.cpp: pack_params)

constexpr int KIND_PREDICT = 0;   // time kernel + volume + buffers (start of an advance)
constexpr int KIND_FUSED = 1;     // finish step n (surface) + predict step n+1
constexpr int KIND_NEIGHBOR = 2;  // finish step n only (end of an advance)

constexpr int MAX_RUNS = 32;       // independent runs sharing one mesh

constexpr int EF_HAS_FINER = 1;    // some face neighbour is one cluster finer: export B2
constexpr int EF_HAS_COARSER = 2;  // some face neighbour is one cluster coarser: export B3

// Per-element integer record FI[Kp][FI_WORDS]:
//   [3i+0] neighbour across face i (internal index, -1 = none)
//   [3i+1] code = j | bc<<4 | (rel+1)<<8 (j: the neighbour's face, rel: its
//          cluster minus ours)
//   [3i+2] the neighbour's B2 slot (rel > 0) or B3 slot (rel < 0), else 0
//   [12] EF_* flags, [13] own B2 slot, [14] own B3 slot (-1 = none),
//   [15] receiver slot (-1 = none)
constexpr int FI_WORDS = 16;

struct KPtrs {
  void* Qe;          // [run][G][B][63] elastic rows, slot 9e+q
  void* Qa;          // [run][G][JB][m][6][63] memory variables of mode 9jb+q
  const void* P;     // [Kp][NPARAM] (shared by all runs)
  const int* FI;     // [Kp][FI_WORDS] (shared by all runs)
  void* T1;          // [run][2][Kp][4][9][FP] B1 face traces (parity of the step)
  void* T2;          // [run][2][N2][4][9][FP] B2 face traces of elements with a finer neighbour
  void* T3;          // [run][2][N3][4][9][FP] B3 face traces of elements with a coarser neighbour
  void* recD;        // [run][slots][O][9][B] time derivatives of receiver elements
  long long Kp;      // padded element count (multiple of 7)
  long long N2, N3;  // B2 / B3 slots per parity
  long long run_qe, run_qa, run_t1, run_t2, run_t3, run_recd;   // per-run strides (words)
};

struct LevelArgs {
  int run0;          // runs run0 + blockIdx.y take part
  int end;           // internal slots [0, end) take part (clusters are contiguous, finest first)
  int kind;
  int n_clusters;
  int cl_end[MAX_CLUSTERS];     // padded end of cluster l (multiple of EPW)
  int cl_vend[MAX_CLUSTERS];    // end of cluster l's real elements (the rest is padding)
  // The level being processed is *clock + jrel (finest steps from t = 0; the
  // clock is device memory so that a captured cycle can be replayed): at
  // level G cluster l (active iff G is a multiple of 2^l) ends its step
  // G/2^l - 1 and starts step G/2^l.  A start-of-advance prediction uses
  // jrel = 0 at a synchronisation point.
  const long long* clock;
  int jrel;
  int xcd_remap;     // 1: the workgroups of one XCD take a contiguous range of element groups
  int trace_mfma;    // 1: the traces of faces 0 and 1 on the matrix cores (two-wave FP32 kernel)
  // workgroup order shuffle (debug; 0 = off): workgroup id w runs the work of
  // id (w * shuf_mul + shuf_add) mod (workgroups of the launch), shuf_mul
  // coprime with that count and (count - 1) * shuf_mul + shuf_add < 2^32
  int shuf_mul, shuf_add;
  double dt[MAX_CLUSTERS];
  double tc[MAX_CLUSTERS][MAX_ORDER];  // dt^{d+1}/(d+1)!
  double th[MAX_CLUSTERS][MAX_ORDER];  // (dt/2)^{d+1}/(d+1)!
  double omega[MAX_MECH];
  // record for the reverse sweep (null on the plain path): the state at the
  // start of this level's predictions of the predicting element groups, in
  // the Qe / Qa layout of run 0 (single-run contexts only)
  void* rec_e;
  void* rec_a;
};

struct SrcArgs {
  int n;
  const int* run;         // [n] run of each source
  const int* elem;
  const int* kind;
  const double* par;      // [n][2]
  const double* moment;   // [n][6]
  const double* phi;      // [n][B]
  const double* inv_det;  // [n]
};

struct RecArgs {
  int n;
  const int* elem;
  const int* slot;
  const double* phi;      // [n][B]
  double dt_sample;
  long long ns;
  int run0;               // runs run0 + blockIdx.y take part
  double* out;            // [run][n][ns][9]
};

// materials in device memory, caller's element order: rho, vp, vs [K];
// yp, ys [K][M] (null for M = 0)
struct MatIn {
  const double* rho;
  const double* vp;
  const double* vs;
  const double* yp;
  const double* ys;
};
// adds the number of elements with rho <= 0, vs <= 0 or vp <= sqrt(4/3) vs to *bad
int launch_check_materials(const MatIn& m, long long K, unsigned* bad, hipStream_t st);
// the material words of the parameter table P [Kp][NPARAM] (1/rho, lambda,
// mu, Zp, Zs, a_l, b_l, the face neighbours' Zp, Zs) and the adjoint's
// material rows amat [Kp][3 + 2M] (rho, vp, vs, Yp_l, Ys_l; zeros for
// padding); i2u [Kp]: caller index of each internal slot (-1: padding);
// nbr [K][4]: caller index of the neighbour across each sorted-frame face
template <class R>
int launch_pack_materials(const MatIn& m, int M, long long Kp, const long long* i2u, const long long* nbr, R* P,
                          double* amat, hipStream_t st);
// g [Kp][3] (internal order) -> g_rho, g_vp, g_vs [K] (caller order; any may be null)
int launch_scatter_gradient(const double* g, const long long* i2u, long long Kp, double* g_rho, double* g_vp,
                            double* g_vs, hipStream_t st);

template <class R, int O, int M>
int launch_level(const KPtrs& p, const LevelArgs& a, int runs, hipStream_t st);
int launch_tick(long long* clock, long long d, hipStream_t st);
// zero `words` 32-bit words at p (a fill kernel: no memset node in a capture)
int launch_zero_words(void* p, size_t words, hipStream_t st);
template <class R, int O, int M>
int launch_sources(const KPtrs& p, const LevelArgs& a, const SrcArgs& s, hipStream_t st);
template <class R, int O, int M>
int launch_receivers(const KPtrs& p, const LevelArgs& a, const RecArgs& r, int runs, hipStream_t st);

// instantiated (precision, order, mechanisms) combinations
#define EDG_FOR_EACH_VARIANT(X) \
  X(float, 2, 0) X(float, 3, 0) X(float, 4, 0) X(float, 5, 0) \
  X(float, 2, 3) X(float, 3, 3) X(float, 4, 3) X(float, 5, 3) \
  X(double, 2, 0) X(double, 3, 0) X(double, 4, 0) X(double, 5, 0) \
  X(double, 2, 3) X(double, 3, 3) X(double, 4, 3) X(double, 5, 3)
#define EDG_KERNEL_INSTANCES EDG_FOR_EACH_VARIANT(EDG_INST)

}  // namespace edg
