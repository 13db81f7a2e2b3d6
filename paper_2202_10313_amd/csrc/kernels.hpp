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

constexpr int EF_HAS_FINER = 1;    // some face neighbour is one cluster finer: export B2
constexpr int EF_HAS_COARSER = 2;  // some face neighbour is one cluster coarser: export B3

struct KPtrs {
  void* Qe;          // [G][B][63] elastic rows, slot 9e+q
  void* Qa;          // [G][B][m][42] memory rows, slot 6e+q
  const void* P;     // [Kp][NPARAM]
  const int* FI;     // [Kp][4][2]: neighbour, code = j | bc<<4 | (rel+1)<<8
  const int* EF;     // [Kp] EF_* flags
  void* T1;          // [2][Kp][4][9][FP] B1 face traces
  void* T2;          // [2][Kp][4][9][FP] B2 face traces
  void* T3;          // [2][Kp][4][9][FP] B3 face traces
  const int* rec_slot;  // [Kp] receiver-element slot or -1 (may be null)
  void* recD;        // [slots][O][9][B] time derivatives of receiver elements
  long long Kp;      // padded element count (multiple of 7)
};

struct LevelArgs {
  int end;           // internal slots [0, end) take part (clusters are contiguous, finest first)
  int kind;
  int n_clusters;
  int cl_end[MAX_CLUSTERS];     // padded end of cluster l (multiple of EPW)
  int cl_vend[MAX_CLUSTERS];    // end of cluster l's real elements (the rest is padding)
  int step_fin[MAX_CLUSTERS];   // index of the step that ends at this level
  int step_new[MAX_CLUSTERS];   // index of the step that starts at this level
  double dt[MAX_CLUSTERS];
  double tc[MAX_CLUSTERS][MAX_ORDER];  // dt^{d+1}/(d+1)!
  double th[MAX_CLUSTERS][MAX_ORDER];  // (dt/2)^{d+1}/(d+1)!
  double omega[MAX_MECH];
};

struct SrcArgs {
  int n;
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
  double* out;            // [n][ns][9]
};

template <class R, int O, int M>
int launch_level(const KPtrs& p, const LevelArgs& a, hipStream_t st);
template <class R, int O, int M>
int launch_sources(const KPtrs& p, const LevelArgs& a, const SrcArgs& s, hipStream_t st);
template <class R, int O, int M>
int launch_receivers(const KPtrs& p, const LevelArgs& a, const RecArgs& r, hipStream_t st);

// instantiated (precision, order, mechanisms) combinations
#define EDG_FOR_EACH_VARIANT(X) \
  X(float, 2, 0) X(float, 3, 0) X(float, 4, 0) X(float, 5, 0) \
  X(float, 2, 3) X(float, 3, 3) X(float, 4, 3) X(float, 5, 3) \
  X(double, 2, 0) X(double, 3, 0) X(double, 4, 0) X(double, 5, 0) \
  X(double, 2, 3) X(double, 3, 3) X(double, 4, 3) X(double, 5, 3)
#define EDG_KERNEL_INSTANCES EDG_FOR_EACH_VARIANT(EDG_INST)

}  // namespace edg
