// Host side of the C-ABI (include/edge_lts.h): mesh processing, geometry,
// clusters, reordering, per-element tables, DOF conversion, the LTS level
// loop and device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "basis.hpp"
#include "edge_lts.h"
#include "kernels.hpp"
#include "adjoint.hpp"
#include "debug.hpp"

using namespace edg;

namespace {
constexpr int EPW = 7;
constexpr int LPE = 9;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};
}  // namespace

struct edg_ctx {
  edg_config cfg{};
  int O = 0, B = 0, F = 0, FP = 0, M = 0, NQ = 0;
  edg::Directions dirs{};   // stiffness directions of the generated kernels
  std::string err;
  hipStream_t stream = nullptr;
  bool own_stream = false;

  // mesh, caller's element order; faces indexed in the sorted-vertex frame
  int64_t K = 0;
  std::vector<std::array<int, 4>> perm;  // sorted local vertex m = caller's local vertex perm[m]
  std::vector<int64_t> nbr, nbr_face;    // [K][4]
  std::vector<int8_t> bc;                // [K][4]
  std::vector<double> Gm, absdet, inradius, normals, areas, X;  // X: sorted coords [K][4][3]
  bool have_mesh = false, have_mat = false, have_clusters = false;

  std::vector<double> rho, vp, vs, yp, ys, omega;

  struct Locator {              // bucket grid for point location
    bool ready = false;
    double lo[3], hi[3], h[3];
    int n[3];
    std::vector<size_t> start;  // [cells + 1]
    std::vector<int64_t> elem;
  } loc;

  std::vector<int> cl;  // 0-based cluster per caller element
  double dt_min = 0, lam = 1, speedup = 1;
  // internal order: clusters finest first, each cluster's range starting on a
  // group boundary (multiple of EPW); internal slots past a cluster's last
  // element up to the next boundary are padding (internal_to_user = -1)
  std::vector<int64_t> internal_to_user, user_to_internal;
  int cl_end[MAX_CLUSTERS] = {0};    // padded end (group aligned) of cluster l
  int cl_vend[MAX_CLUSTERS] = {0};   // end of cluster l's real elements
  int64_t cl_count[MAX_CLUSTERS] = {0};
  double dt_cl[MAX_CLUSTERS] = {0};
  int64_t level = 0;
  int64_t nstep[MAX_CLUSTERS] = {0};
  int64_t updates = 0;

  int64_t G = 0, Kp = 0;
  int runs = 1;                     // independent runs sharing the mesh
  int64_t N2 = 1, N3 = 1;           // B2 / B3 slots (elements with a finer / coarser neighbour)
  size_t run_qe = 0, run_qa = 0, run_t1 = 0, run_t2 = 0, run_t3 = 0, run_recd = 0;   // words per run
  std::vector<int> FI_host;         // [Kp][FI_WORDS]
  DevBuf Qe, Qa, P, FI, T1, T2, T3, RecD;
  // sources, per run
  struct Source {
    int elem, kind;
    double par[2], moment[6], idet;
    std::vector<double> phi;
  };
  std::vector<std::vector<Source>> src_of_run;
  int n_src = 0;
  DevBuf s_run, s_elem, s_kind, s_par, s_mom, s_phi, s_idet;
  // receivers
  int n_rec = 0;
  int64_t rec_ns = 0;
  double rec_dt = 0;
  DevBuf r_elem, r_slot, r_phi, r_out;

  std::vector<std::vector<double>> perm_mats;  // 24 B x B conversion matrices

  // launch plan (all but trace_mfma give bit-identical results) and cycle graph
  edg_plan plan{0, 0, 0};
  uint64_t shuf_seq = 0;             // launches shuffled so far (EDG_FLAG_SHUFFLE)
  DevBuf dbg;                        // non-finite count and first index (EDG_FLAG_CHECK_FINITE)
  DevBuf dclock;                     // level at the start of the current cycle (device)
  hipGraphExec_t cycle_exec = nullptr;
  hipGraph_t cycle_graph = nullptr;

  // checkpoints of the forward state (adjoint): every ckpt_every cycles an
  // advance starts a segment and stores the state at its start
  int ckpt_every = 0;
  std::vector<std::pair<int64_t, DevBuf>> ckpts;    // (level, Qe then Qa of every run)
  std::vector<DevBuf> ckpt_pool;     // buffers of dropped checkpoints, reused by the next ones
  // ahist holds, for the segment that starts at level hist_L0 and spans
  // hist_J levels, the state at the start of every level's predictions (the
  // final segment of a checkpointed advance records it; a replay rewrites it)
  bool hist_valid = false;
  // the adjoint face slots and receiver derivatives hold zeros (left so by a
  // completed reverse sweep: each is cleared by its reader)
  bool adj_clean = false;
  bool amat_valid = false;           // amat holds the materials of the current upload, internal order
  // materials uploaded from device memory: a device copy in caller order
  // (rho, vp, vs [K], yp, ys [K][m]); the host vectors are refreshed from it
  // when host code needs them
  bool mat_host_valid = true;
  DevBuf dmat, dflag;
  DevBuf d_i2u, d_nbr;               // internal_to_user [Kp], nbr [K][4] (int64, for device-side tables)
  int64_t hist_L0 = 0, hist_J = 0;
  int hist_run = 0;                  // the run whose level states ahist holds
  // adjoint buffers
  DevBuf aLe, aLa, aS0, aS1, aS2, aS3, aDe, aDa, agacc, arecDb, aseis, ahist, afinal, amat, agrad;

  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  size_t ev_used = 0;
  std::vector<int64_t> ev_updates;
  std::vector<int> ev_launches;
  int64_t t_launches = 0, t_updates = 0;
  double t_ms = 0;

  ~edg_ctx();
};

namespace {

int fail(edg_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return fail(ctx, EDG_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

void dev_free(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

void drop_checkpoints(edg_ctx* c) {
  // the buffers stay allocated for the next checkpoints (a hipMalloc of a
  // whole state per segment would otherwise sit inside every forward)
  for (auto& ck : c->ckpts) c->ckpt_pool.push_back(ck.second);
  c->ckpts.clear();
  c->hist_valid = false;
}

int dev_alloc(edg_ctx* c, DevBuf& b, size_t bytes) {
  dev_free(b);
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();   // the failed allocation's error must not be reported by a later launch check
    return fail(c, EDG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  return 0;
}

// keeps b if it already holds at least `bytes` (buffers reused across calls)
int dev_reserve(edg_ctx* c, DevBuf& b, size_t bytes) {
  if (b.p && b.bytes >= bytes) return 0;
  return dev_alloc(c, b, bytes);
}

int dev_upload(edg_ctx* c, DevBuf& b, const void* src, size_t bytes) {
  int rc = dev_alloc(c, b, bytes);
  if (rc) return rc;
  HIPCHK(c, hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
  return 0;
}

int perm_code(const std::array<int, 4>& p) {
  // lexicographic rank of the permutation (0..23)
  int code = 0;
  const int fact[4] = {6, 2, 1, 1};
  bool used[4] = {false, false, false, false};
  for (int m = 0; m < 4; ++m) {
    int r = 0;
    for (int v = 0; v < p[m]; ++v)
      if (!used[v]) ++r;
    code += r * fact[m];
    used[p[m]] = true;
  }
  return code;
}

const std::vector<double>& perm_matrix(edg_ctx* c, const std::array<int, 4>& p) {
  if (c->perm_mats.empty()) c->perm_mats.resize(24);
  auto& m = c->perm_mats[perm_code(p)];
  if (m.empty()) m = vertex_permutation_matrix(c->O, p.data());
  return m;
}

void inverse3(const double J[9], double G[9], double& det) {
  det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) + J[2] * (J[3] * J[7] - J[4] * J[6]);
  const double id = 1.0 / det;
  G[0] = (J[4] * J[8] - J[5] * J[7]) * id;
  G[1] = (J[2] * J[7] - J[1] * J[8]) * id;
  G[2] = (J[1] * J[5] - J[2] * J[4]) * id;
  G[3] = (J[5] * J[6] - J[3] * J[8]) * id;
  G[4] = (J[0] * J[8] - J[2] * J[6]) * id;
  G[5] = (J[2] * J[3] - J[0] * J[5]) * id;
  G[6] = (J[3] * J[7] - J[4] * J[6]) * id;
  G[7] = (J[1] * J[6] - J[0] * J[7]) * id;
  G[8] = (J[0] * J[4] - J[1] * J[3]) * id;
}

// Sec. V-A (Clustering): assign by interval, normalise to the neighbour rule,
// optional lambda search maximising K / sum_l n_l / (2^(l-1) lambda).
void cluster_assign(int64_t K, const double* dt, double dt_min, double lam, int Nc, std::vector<int>& cl) {
  cl.assign(K, 0);
  const double base = lam * dt_min;
  for (int64_t k = 0; k < K; ++k)
    for (int l = 1; l < Nc; ++l)
      if (dt[k] >= std::ldexp(base, l)) cl[k] = l;
}

void cluster_normalise(int64_t K, const int64_t* nbr, std::vector<int>& cl) {
  bool changed = true;
  while (changed) {
    changed = false;
    std::vector<int> nw(cl);
    for (int64_t k = 0; k < K; ++k) {
      int mn = 1 << 30;
      for (int i = 0; i < 4; ++i) {
        const int64_t n = nbr[k * 4 + i];
        if (n >= 0) mn = std::min(mn, cl[n]);
      }
      if (mn + 1 < nw[k]) {
        nw[k] = mn + 1;
        changed = true;
      }
    }
    cl.swap(nw);
  }
}

double cluster_speedup(const std::vector<int>& cl, double lam, int Nc) {
  std::vector<int64_t> cnt(Nc, 0);
  for (int v : cl) cnt[v]++;
  double denom = 0.0;
  for (int l = 0; l < Nc; ++l) denom += (double)cnt[l] / (std::ldexp(1.0, l) * lam);
  return (double)cl.size() / denom;
}

void cluster_all(int64_t K, const double* dt, const int64_t* nbr, int Nc, double lam_in, std::vector<int>& cl,
                 double& lam_out, double& speed) {
  double dt_min = dt[0];
  for (int64_t k = 1; k < K; ++k) dt_min = std::min(dt_min, dt[k]);
  if (lam_in > 0) {
    cluster_assign(K, dt, dt_min, lam_in, Nc, cl);
    cluster_normalise(K, nbr, cl);
    lam_out = lam_in;
    speed = cluster_speedup(cl, lam_in, Nc);
    return;
  }
  bool first = true;
  for (int i = 51; i <= 100; ++i) {
    const double lm = i / 100.0;
    std::vector<int> c;
    cluster_assign(K, dt, dt_min, lm, Nc, c);
    cluster_normalise(K, nbr, c);
    const double s = cluster_speedup(c, lm, Nc);
    if (first || s >= speed) {
      cl.swap(c);
      lam_out = lm;
      speed = s;
      first = false;
    }
  }
}

// the host copies of the materials (after an upload from device memory they
// are fetched from the library's device copy when host code first needs them)
int ensure_host_materials(edg_ctx* c) {
  if (c->mat_host_valid) return 0;
  const int64_t K = c->K;
  const int M = c->M;
  const double* d = (const double*)c->dmat.p;
  c->rho.resize(K);
  c->vp.resize(K);
  c->vs.resize(K);
  c->yp.resize((size_t)K * M);
  c->ys.resize((size_t)K * M);
  HIPCHK(c, hipMemcpyAsync(c->rho.data(), d, K * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->vp.data(), d + K, K * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->vs.data(), d + 2 * K, K * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (M > 0) {
    HIPCHK(c, hipMemcpyAsync(c->yp.data(), d + 3 * K, K * M * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ys.data(), d + 3 * K + K * M, K * M * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->mat_host_valid = true;
  return 0;
}

template <class R>
void pack_tables(edg_ctx* c, std::vector<R>& P, std::vector<int>& FI) {
  const int64_t Kp = c->Kp;
  P.assign((size_t)Kp * NPARAM, R(0));
  FI.assign((size_t)Kp * FI_WORDS, 0);
  // flags and compact B2 / B3 slots of every element (internal order)
  std::vector<int> flags(Kp, 0), s2(Kp, -1), s3(Kp, -1);
  int64_t n2 = 0, n3 = 0;
  for (int64_t ki = 0; ki < Kp; ++ki) {
    const int64_t k = c->internal_to_user[ki];
    if (k < 0) continue;
    for (int i = 0; i < 4; ++i) {
      const int64_t n = c->nbr[k * 4 + i];
      if (n < 0) continue;
      if (c->cl[n] < c->cl[k]) flags[ki] |= EF_HAS_FINER;
      if (c->cl[n] > c->cl[k]) flags[ki] |= EF_HAS_COARSER;
    }
    if (flags[ki] & EF_HAS_FINER) s2[ki] = (int)n2++;
    if (flags[ki] & EF_HAS_COARSER) s3[ki] = (int)n3++;
  }
  c->N2 = std::max<int64_t>(n2, 1);
  c->N3 = std::max<int64_t>(n3, 1);
  for (int64_t ki = 0; ki < Kp; ++ki) {
    int* fi = &FI[(size_t)ki * FI_WORDS];
    const int64_t k = c->internal_to_user[ki];
    fi[12] = flags[ki];
    fi[13] = s2[ki];
    fi[14] = s3[ki];
    fi[15] = -1;
    if (k < 0) {   // padding slot: no neighbours, zero parameters, never stored
      for (int i = 0; i < 4; ++i) fi[3 * i] = -1;
      continue;
    }
    R* p = &P[(size_t)ki * NPARAM];
    const double rho = c->rho[k], vp = c->vp[k], vs = c->vs[k];
    const double mu = rho * vs * vs, lam = rho * vp * vp - 2.0 * mu;
    // G' = V^-T G for the library's stiffness directions
    const double* G = &c->Gm[(size_t)k * 9];
    for (int kk = 0; kk < 3; ++kk)
      for (int d = 0; d < 3; ++d) {
        double sum = 0.0;
        for (int cc = 0; cc < 3; ++cc) sum += c->dirs.Vinv[cc * 3 + kk] * G[cc * 3 + d];
        p[kk * 3 + d] = R(sum);
      }
    p[9] = R(1.0 / rho);
    p[10] = R(lam);
    p[11] = R(mu);
    p[12] = R(rho * vp);
    p[13] = R(rho * vs);
    for (int l = 0; l < c->M; ++l) {
      const double ypl = c->yp[k * c->M + l], ysl = c->ys[k * c->M + l];
      p[14 + 2 * l] = R((lam + 2.0 * mu) * ypl - 2.0 * mu * ysl);
      p[15 + 2 * l] = R(2.0 * mu * ysl);
    }
    for (int i = 0; i < 4; ++i) {
      R* f = p + 20 + 6 * i;
      for (int d = 0; d < 3; ++d) f[d] = R(c->normals[(k * 4 + i) * 3 + d]);
      f[3] = R(2.0 * c->areas[k * 4 + i] / c->absdet[k]);
      const int64_t n = c->nbr[k * 4 + i];
      int nb_int = -1, j = 0, rel = 0, bc = c->bc[k * 4 + i], aux = 0;
      if (n >= 0) {
        f[4] = R(c->rho[n] * c->vp[n]);
        f[5] = R(c->rho[n] * c->vs[n]);
        nb_int = (int)c->user_to_internal[n];
        j = (int)c->nbr_face[k * 4 + i];
        rel = c->cl[n] - c->cl[k];
        bc = 0;
        if (rel > 0) aux = s2[nb_int];   // the coarser neighbour's B2
        if (rel < 0) aux = s3[nb_int];   // the finer neighbour's B3
      } else {
        f[4] = R(rho * vp);
        f[5] = R(rho * vs);
      }
      fi[3 * i] = nb_int;
      fi[3 * i + 1] = j | (bc << 4) | ((rel + 1) << 8);
      fi[3 * i + 2] = aux;
    }
  }
}

// DOF layout: elastic rows [G][B][63] at slot 9e+q (the lane of row q of
// element e); memory variables [G][JB][m][6][63] with mode b = r + 9 jb at
// slot 9e+r (the lane that owns mode b), JB = ceil(B/9)
inline int jb_count(const edg_ctx* c) { return (c->B + LPE - 1) / LPE; }
inline size_t qe_index(const edg_ctx* c, int64_t ki, int q, int b) {
  return ((size_t)(ki / EPW) * c->B + b) * (EPW * LPE) + (ki % EPW) * LPE + q;
}
inline size_t qa_index(const edg_ctx* c, int64_t ki, int l, int comp, int b) {
  const int jb = b / LPE, r = b % LPE;
  return ((((size_t)(ki / EPW) * jb_count(c) + jb) * c->M + l) * 6 + comp) * (EPW * LPE) + (ki % EPW) * LPE + r;
}
inline size_t qa_size(const edg_ctx* c) {
  return c->M > 0 ? (size_t)c->G * jb_count(c) * c->M * 6 * EPW * LPE : 1;
}

// caller-order DOFs [K][NQ][B] -> the tiled layout at dqe / dqa (device);
// the vertex-sorting basis changes are orthogonal, so adjoints convert the
// same way
template <class R>
int set_dofs_to(edg_ctx* c, void* dqe, void* dqa, const double* dofs) {
  const int B = c->B, NQ = c->NQ;
  std::vector<R> he((size_t)c->G * B * EPW * LPE, R(0));
  std::vector<R> ha(qa_size(c), R(0));
  std::vector<double> row(B);
  for (int64_t k = 0; k < c->K; ++k) {
    const int64_t ki = c->user_to_internal[k];
    const auto& C = perm_matrix(c, c->perm[k]);
    for (int q = 0; q < NQ; ++q) {
      const double* src = dofs + ((size_t)k * NQ + q) * B;
      bool zero = true;
      for (int bb = 0; bb < B && zero; ++bb) zero = src[bb] == 0.0;
      if (zero) continue;   // the staging buffer is already zero
      for (int b = 0; b < B; ++b) {
        double s = 0.0;
        for (int bb = 0; bb < B; ++bb) s += C[b * B + bb] * src[bb];
        row[b] = s;
      }
      for (int b = 0; b < B; ++b) {
        if (q < 9) he[qe_index(c, ki, q, b)] = R(row[b]);
        else ha[qa_index(c, ki, (q - 9) / 6, (q - 9) % 6, b)] = R(row[b]);
      }
    }
  }
  HIPCHK(c, hipMemcpy(dqe, he.data(), he.size() * sizeof(R), hipMemcpyHostToDevice));
  if (c->M > 0) HIPCHK(c, hipMemcpy(dqa, ha.data(), ha.size() * sizeof(R), hipMemcpyHostToDevice));
  return 0;
}

template <class R>
int set_dofs_t(edg_ctx* c, int run, const double* dofs) {
  return set_dofs_to<R>(c, (R*)c->Qe.p + run * c->run_qe, (R*)c->Qa.p + run * c->run_qa, dofs);
}

template <class R>
int get_dofs_from(edg_ctx* c, const void* dqe, const void* dqa, double* out) {
  const int B = c->B, NQ = c->NQ;
  std::vector<R> he((size_t)c->G * B * EPW * LPE);
  std::vector<R> ha(qa_size(c));
  HIPCHK(c, hipMemcpy(he.data(), dqe, he.size() * sizeof(R), hipMemcpyDeviceToHost));
  if (c->M > 0) HIPCHK(c, hipMemcpy(ha.data(), dqa, ha.size() * sizeof(R), hipMemcpyDeviceToHost));
  std::vector<double> row(B);
  for (int64_t k = 0; k < c->K; ++k) {
    const int64_t ki = c->user_to_internal[k];
    const auto& C = perm_matrix(c, c->perm[k]);
    for (int q = 0; q < NQ; ++q) {
      bool zero = true;
      for (int b = 0; b < B; ++b) {
        row[b] = q < 9 ? (double)he[qe_index(c, ki, q, b)] : (double)ha[qa_index(c, ki, (q - 9) / 6, (q - 9) % 6, b)];
        zero = zero && row[b] == 0.0;
      }
      double* dst = out + ((size_t)k * NQ + q) * B;
      if (zero) {
        for (int bb = 0; bb < B; ++bb) dst[bb] = 0.0;
        continue;
      }
      for (int bb = 0; bb < B; ++bb) {
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += C[b * B + bb] * row[b];
        dst[bb] = s;
      }
    }
  }
  return 0;
}

template <class R>
int get_dofs_t(edg_ctx* c, int run, double* out) {
  return get_dofs_from<R>(c, (R*)c->Qe.p + run * c->run_qe, (R*)c->Qa.p + run * c->run_qa, out);
}

// DOFs of selected elements: only the 7-element groups that hold them are
// copied (device -> host, and back when writing)
template <class R>
int subset_dofs_t(edg_ctx* c, int run, int64_t n, const int64_t* ids, const double* in, double* out) {
  const int B = c->B, NQ = c->NQ, JB = jb_count(c);
  const size_t qe_blk = (size_t)B * EPW * LPE;
  const size_t qa_blk = c->M > 0 ? (size_t)JB * c->M * 6 * EPW * LPE : 0;
  std::vector<int64_t> groups(n);
  for (int64_t i = 0; i < n; ++i) groups[i] = c->user_to_internal[ids[i]] / EPW;
  std::sort(groups.begin(), groups.end());
  groups.erase(std::unique(groups.begin(), groups.end()), groups.end());
  std::vector<R> he(groups.size() * qe_blk), ha(std::max<size_t>(groups.size() * qa_blk, 1));
  R* const dqe = (R*)c->Qe.p + run * c->run_qe;
  R* const dqa = (R*)c->Qa.p + run * c->run_qa;
  for (size_t j = 0; j < groups.size(); ++j) {
    HIPCHK(c, hipMemcpy(he.data() + j * qe_blk, dqe + groups[j] * qe_blk, qe_blk * sizeof(R), hipMemcpyDeviceToHost));
    if (qa_blk)
      HIPCHK(c, hipMemcpy(ha.data() + j * qa_blk, dqa + groups[j] * qa_blk, qa_blk * sizeof(R), hipMemcpyDeviceToHost));
  }
  std::vector<double> row(B);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t k = ids[i], ki = c->user_to_internal[k];
    const size_t j = std::lower_bound(groups.begin(), groups.end(), ki / EPW) - groups.begin();
    const int e = (int)(ki % EPW);
    const auto& C = perm_matrix(c, c->perm[k]);
    for (int q = 0; q < NQ; ++q) {
      auto at = [&](int b) -> R& {
        if (q < 9) return he[j * qe_blk + (size_t)b * (EPW * LPE) + e * LPE + q];
        const int l = (q - 9) / 6, comp = (q - 9) % 6, jb = b / LPE, r = b % LPE;
        return ha[j * qa_blk + ((size_t)(jb * c->M + l) * 6 + comp) * (EPW * LPE) + e * LPE + r];
      };
      if (in) {
        const double* src = in + ((size_t)i * NQ + q) * B;
        for (int b = 0; b < B; ++b) {
          double sum = 0.0;
          for (int bb = 0; bb < B; ++bb) sum += C[b * B + bb] * src[bb];
          at(b) = R(sum);
        }
      } else {
        for (int b = 0; b < B; ++b) row[b] = (double)at(b);
        double* dst = out + ((size_t)i * NQ + q) * B;
        for (int bb = 0; bb < B; ++bb) {
          double sum = 0.0;
          for (int b = 0; b < B; ++b) sum += C[b * B + bb] * row[b];
          dst[bb] = sum;
        }
      }
    }
  }
  if (in)
    for (size_t j = 0; j < groups.size(); ++j) {
      HIPCHK(c, hipMemcpy(dqe + groups[j] * qe_blk, he.data() + j * qe_blk, qe_blk * sizeof(R), hipMemcpyHostToDevice));
      if (qa_blk)
        HIPCHK(c, hipMemcpy(dqa + groups[j] * qa_blk, ha.data() + j * qa_blk, qa_blk * sizeof(R), hipMemcpyHostToDevice));
    }
  return 0;
}

// locate a point: lowest caller element index whose barycentrics are >= -tol
// bucket grid over the element bounding boxes (built on the first query):
// every element is listed, in ascending index, in each cell its padded box
// touches
void build_locator(edg_ctx* c) {
  auto& L = c->loc;
  const int64_t K = c->K;
  for (int d = 0; d < 3; ++d) {
    L.lo[d] = 1e300;
    L.hi[d] = -1e300;
  }
  std::vector<double> box((size_t)K * 6);
  for (int64_t k = 0; k < K; ++k) {
    const double* X = &c->X[(size_t)k * 12];
    for (int d = 0; d < 3; ++d) {
      double lo = std::min(std::min(X[d], X[3 + d]), std::min(X[6 + d], X[9 + d]));
      double hi = std::max(std::max(X[d], X[3 + d]), std::max(X[6 + d], X[9 + d]));
      const double pad = 1e-9 * (hi - lo + 1.0);
      lo -= pad;
      hi += pad;
      box[(size_t)k * 6 + d] = lo;
      box[(size_t)k * 6 + 3 + d] = hi;
      L.lo[d] = std::min(L.lo[d], lo);
      L.hi[d] = std::max(L.hi[d], hi);
    }
  }
  const int n = std::max(1, (int)std::cbrt((double)K / 4.0));
  for (int d = 0; d < 3; ++d) {
    L.n[d] = n;
    L.h[d] = (L.hi[d] - L.lo[d]) / n;
    if (!(L.h[d] > 0)) L.h[d] = 1.0;
  }
  auto cell = [&](int d, double v) { return std::min(L.n[d] - 1, std::max(0, (int)((v - L.lo[d]) / L.h[d]))); };
  const size_t ncell = (size_t)n * n * n;
  L.start.assign(ncell + 1, 0);
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int64_t> fill;
    if (pass == 1) {
      for (size_t i = 0; i < ncell; ++i) L.start[i + 1] += L.start[i];
      L.elem.resize(L.start[ncell]);
      fill.assign(L.start.begin(), L.start.end() - 1);
    }
    for (int64_t k = 0; k < K; ++k) {
      const double* b = &box[(size_t)k * 6];
      for (int i = cell(0, b[0]); i <= cell(0, b[3]); ++i)
        for (int j = cell(1, b[1]); j <= cell(1, b[4]); ++j)
          for (int l = cell(2, b[2]); l <= cell(2, b[5]); ++l) {
            const size_t ci = ((size_t)i * n + j) * n + l;
            if (pass == 0) L.start[ci + 1]++;
            else L.elem[fill[ci]++] = k;
          }
    }
  }
  L.ready = true;
}

// locate a point: lowest caller element index whose barycentrics are >= -tol
int64_t locate(edg_ctx* c, const double* x, double xi_sorted[3]) {
  const double tol = 1e-10;
  if (!c->loc.ready) build_locator(c);
  const auto& L = c->loc;
  int idx[3];
  for (int d = 0; d < 3; ++d) {
    if (!(x[d] >= L.lo[d] && x[d] <= L.hi[d])) return -1;
    idx[d] = std::min(L.n[d] - 1, std::max(0, (int)((x[d] - L.lo[d]) / L.h[d])));
  }
  const size_t ci = ((size_t)idx[0] * L.n[1] + idx[1]) * L.n[2] + idx[2];
  for (size_t e = L.start[ci]; e < L.start[ci + 1]; ++e) {
    const int64_t k = L.elem[e];
    const double* X = &c->X[(size_t)k * 12];
    const double* G = &c->Gm[(size_t)k * 9];
    double r[3];
    for (int cc = 0; cc < 3; ++cc) {
      r[cc] = 0.0;
      for (int d = 0; d < 3; ++d) r[cc] += G[cc * 3 + d] * (x[d] - X[d]);
    }
    if (r[0] >= -tol && r[1] >= -tol && r[2] >= -tol && 1.0 - r[0] - r[1] - r[2] >= -tol) {
      for (int d = 0; d < 3; ++d) xi_sorted[d] = r[d];
      return k;
    }
  }
  return -1;
}

template <class R, int O, int M>
struct Launch {
  static int level(const KPtrs& p, const LevelArgs& a, int runs, hipStream_t s) {
    return launch_level<R, O, M>(p, a, runs, s);
  }
  static int src(const KPtrs& p, const LevelArgs& a, const SrcArgs& sa, hipStream_t s) {
    return launch_sources<R, O, M>(p, a, sa, s);
  }
  static int rec(const KPtrs& p, const LevelArgs& a, const RecArgs& ra, int runs, hipStream_t s) {
    return launch_receivers<R, O, M>(p, a, ra, runs, s);
  }
};

typedef int (*LevelFn)(const KPtrs&, const LevelArgs&, int, hipStream_t);
typedef int (*SrcFn)(const KPtrs&, const LevelArgs&, const SrcArgs&, hipStream_t);
typedef int (*RecFn)(const KPtrs&, const LevelArgs&, const RecArgs&, int, hipStream_t);

struct Fns {
  LevelFn level = nullptr;
  SrcFn src = nullptr;
  RecFn rec = nullptr;
};

Fns pick(int fp64, int O, int M) {
  Fns f;
#define EDG_PICK(R, OO, MM)                                                         \
  if ((std::is_same<R, double>::value == (fp64 != 0)) && O == OO && M == MM) {      \
    f.level = &Launch<R, OO, MM>::level;                                            \
    f.src = &Launch<R, OO, MM>::src;                                                \
    f.rec = &Launch<R, OO, MM>::rec;                                                \
  }
  EDG_FOR_EACH_VARIANT(EDG_PICK)
#undef EDG_PICK
  return f;
}

KPtrs kptrs(const edg_ctx* c) {
  KPtrs p;
  p.Qe = c->Qe.p;
  p.Qa = c->Qa.p;
  p.P = c->P.p;
  p.FI = (const int*)c->FI.p;
  p.T1 = c->T1.p;
  p.T2 = c->T2.p;
  p.T3 = c->T3.p;
  p.recD = c->RecD.p;
  p.Kp = c->Kp;
  p.N2 = c->N2;
  p.N3 = c->N3;
  p.run_qe = (long long)c->run_qe;
  p.run_qa = (long long)c->run_qa;
  p.run_t1 = (long long)c->run_t1;
  p.run_t2 = (long long)c->run_t2;
  p.run_t3 = (long long)c->run_t3;
  p.run_recd = (long long)c->run_recd;
  return p;
}

LevelArgs base_args(const edg_ctx* c) {
  LevelArgs a;
  std::memset(&a, 0, sizeof a);
  a.n_clusters = c->cfg.n_clusters;
  for (int l = 0; l < MAX_CLUSTERS; ++l) {
    a.cl_end[l] = c->cl_end[l];
    a.cl_vend[l] = c->cl_vend[l];
    a.dt[l] = c->dt_cl[l];
    for (int d = 0; d < c->O; ++d) {
      double f = 1.0;
      for (int j = 2; j <= d + 1; ++j) f *= j;
      a.tc[l][d] = std::pow(c->dt_cl[l], d + 1) / f;
      a.th[l][d] = std::pow(0.5 * c->dt_cl[l], d + 1) / f;
    }
  }
  for (int l = 0; l < c->M; ++l) a.omega[l] = c->omega[l];
  a.clock = (const long long*)c->dclock.p;
  a.xcd_remap = c->plan.xcd_remap;
  a.trace_mfma = c->plan.trace_mfma;
  return a;
}

// EDG_FLAG_SHUFFLE: a fresh affine bijection of the workgroup order of one
// launch of `runs` runs (SplitMix64 over a per-context launch counter)
void shuffle_args(edg_ctx* c, LevelArgs& a, int runs) {
  a.shuf_mul = a.shuf_add = 0;
  if (!(c->cfg.flags & EDG_FLAG_SHUFFLE)) return;
  const long long total = (long long)((a.end + EPW - 1) / EPW) * runs;
  if (total < 2) return;
  auto next = [&]() {
    uint64_t z = (c->shuf_seq += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  // 32-bit device arithmetic: (total - 1) * m + add < 2^32
  const long long mmax = std::min<long long>(total - 1, (0xFFFFFFFFll - (total - 1)) / (total - 1));
  long long m = 1 + (long long)(next() % (uint64_t)mmax);
  while (std::gcd(m, total) != 1) m = m % mmax + 1;
  a.shuf_mul = (int)m;
  a.shuf_add = (int)(next() % (uint64_t)total);
}

// EDG_FLAG_POISON: after a level that finishes steps, NaN into the trace
// slots whose last legal read was at that level (all runs)
int poison_after(edg_ctx* c, const KPtrs& p, const LevelArgs& a0) {
  const uint32_t f = c->cfg.flags;
  if (!(f & (EDG_FLAG_POISON | EDG_FLAG_POISON_EARLY)) || a0.kind == KIND_PREDICT) return 0;
  LevelArgs a = a0;
  a.run0 = 0;
  const int early = (f & EDG_FLAG_POISON_EARLY) ? 1 : 0;
  const int rc = c->cfg.fp64 ? launch_poison_traces<double>(p, a, c->runs, c->FP, early, c->stream)
                             : launch_poison_traces<float>(p, a, c->runs, c->FP, early, c->stream);
  return rc ? fail(c, EDG_EHIP, std::string("poison kernel: ") + hipGetErrorString((hipError_t)rc)) : 0;
}

// EDG_FLAG_POISON: NaN into every trace slot at the start of an advance (all
// are written before they are read from a synchronisation point on)
int poison_all(edg_ctx* c, const KPtrs& p) {
  if (!(c->cfg.flags & EDG_FLAG_POISON)) return 0;
  const size_t rs = c->cfg.fp64 ? sizeof(double) : sizeof(float);
  const void* base[3] = {p.T1, p.T2, p.T3};
  const size_t words[3] = {c->runs * c->run_t1, c->runs * c->run_t2, c->runs * c->run_t3};
  for (int i = 0; i < 3; ++i) {
    const int rc = launch_poison_words(const_cast<void*>(base[i]), words[i] * rs / 4, c->stream);
    if (rc) return fail(c, EDG_EHIP, std::string("fill kernel: ") + hipGetErrorString((hipError_t)rc));
  }
  return 0;
}

// EDG_FLAG_CHECK_FINITE: EDG_ENONFINITE if a DOF word of any run is NaN or
// infinite (after an advance, with the stream synchronised)
int check_finite(edg_ctx* c) {
  if (!(c->cfg.flags & EDG_FLAG_CHECK_FINITE)) return 0;
  if (!c->dbg.p) return fail(c, EDG_ESTATE, "finite check: no device counter (upload clusters first)");
  const unsigned long long init[2] = {0ull, ~0ull};
  HIPCHK(c, hipMemcpyAsync(c->dbg.p, init, sizeof init, hipMemcpyHostToDevice, c->stream));
  const long long ne = (long long)(c->runs * c->run_qe), na = (long long)(c->runs * c->run_qa);
  auto* cnt = (unsigned long long*)c->dbg.p;
  int rc = c->cfg.fp64 ? launch_count_nonfinite<double>(c->Qe.p, ne, cnt, c->stream)
                       : launch_count_nonfinite<float>(c->Qe.p, ne, cnt, c->stream);
  unsigned long long ha[2] = {0, 0}, hb[2] = {0, 0};
  if (!rc) {
    HIPCHK(c, hipMemcpyAsync(ha, c->dbg.p, sizeof ha, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->dbg.p, init, sizeof init, hipMemcpyHostToDevice, c->stream));
    rc = c->cfg.fp64 ? launch_count_nonfinite<double>(c->Qa.p, na, cnt, c->stream)
                     : launch_count_nonfinite<float>(c->Qa.p, na, cnt, c->stream);
  }
  if (rc) return fail(c, EDG_EHIP, std::string("finite check kernel: ") + hipGetErrorString((hipError_t)rc));
  HIPCHK(c, hipMemcpyAsync(hb, c->dbg.p, sizeof hb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (ha[0] + hb[0] == 0) return 0;
  // the first bad word -> run and caller element (Qe [run][G][B][63],
  // Qa [run][G][JB][m][6][63]; slot 9e + q of group g is element 7g + e)
  const bool in_e = ha[0] > 0;
  const unsigned long long w = in_e ? ha[1] : hb[1];
  const size_t per_run = in_e ? c->run_qe : c->run_qa;
  const size_t run = w / per_run, rem = w % per_run, per_group = per_run / (size_t)c->G;
  const int64_t ki = (int64_t)(rem / per_group) * EPW + (int64_t)((rem % (EPW * LPE)) / LPE);
  const int64_t user = ki < (int64_t)c->internal_to_user.size() ? c->internal_to_user[ki] : -1;
  return fail(c, EDG_ENONFINITE, std::to_string(ha[0] + hb[0]) + " non-finite DOF words after the advance (first: run " +
                                     std::to_string(run) + ", element " + std::to_string(user) +
                                     (in_e ? ", elastic rows)" : ", memory variables)"));
}

// one LTS level for all runs, in chunks of plan.run_chunk runs per launch
int launch_runs(edg_ctx* c, const Fns& fn, const KPtrs& p, LevelArgs a) {
  const int chunk = c->plan.run_chunk > 0 ? std::min(c->plan.run_chunk, c->runs) : c->runs;
  for (int r0 = 0; r0 < c->runs; r0 += chunk) {
    a.run0 = r0;
    shuffle_args(c, a, std::min(chunk, c->runs - r0));
    const int rc = fn.level(p, a, std::min(chunk, c->runs - r0), c->stream);
    if (rc) return fail(c, EDG_EHIP, std::string("level kernel launch: ") + hipGetErrorString((hipError_t)rc));
  }
  return 0;
}

int timed_begin(edg_ctx* c, int64_t upd, int launches) {
  if (!c->timing) return 0;
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    c->ev_pool.push_back({e0, e1});
  }
  c->ev_updates.push_back(upd);
  c->ev_launches.push_back(launches);
  HIPCHK(c, hipEventRecord(c->ev_pool[c->ev_used].first, c->stream));
  return 0;
}

int timed_end(edg_ctx* c) {
  if (!c->timing) return 0;
  HIPCHK(c, hipEventRecord(c->ev_pool[c->ev_used++].second, c->stream));
  return 0;
}

// the captured cycle refers to argument values of the moment: drop it when they change
void drop_graph(edg_ctx* c) {
  if (c->cycle_exec) (void)hipGraphExecDestroy(c->cycle_exec);
  if (c->cycle_graph) (void)hipGraphDestroy(c->cycle_graph);
  c->cycle_exec = nullptr;
  c->cycle_graph = nullptr;
}

int launch_timed(edg_ctx* c, const Fns& fn, const KPtrs& p, const LevelArgs& a, int64_t upd) {
  int rc;
  if ((rc = timed_begin(c, upd, 1))) return rc;
  if ((rc = launch_runs(c, fn, p, a))) return rc;
  return timed_end(c);
}

}  // namespace

edg_ctx::~edg_ctx() {
  for (DevBuf* b : {&Qe, &Qa, &P, &FI, &T1, &T2, &T3, &RecD, &s_run, &s_elem, &s_kind, &s_par, &s_mom, &s_phi,
                    &s_idet, &r_elem, &r_slot, &r_phi, &r_out, &dclock, &aLe, &aLa, &aS0, &aS1, &aS2, &aS3, &aDe, &aDa,
                    &agacc, &arecDb, &aseis, &ahist, &afinal, &amat, &agrad, &dmat, &dflag, &d_i2u, &d_nbr, &dbg})
    dev_free(*b);
  for (auto& ck : ckpts) dev_free(ck.second);
  for (auto& b : ckpt_pool) dev_free(b);
  for (auto& e : ev_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  if (cycle_exec) (void)hipGraphExecDestroy(cycle_exec);
  if (cycle_graph) (void)hipGraphDestroy(cycle_graph);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

extern "C" {

int edg_create(const edg_config* cfg, edg_ctx** out) {
  if (!out) return EDG_EINVAL;
  *out = nullptr;
  if (!cfg) return EDG_EINVAL;
  if (cfg->order < 2 || cfg->order > MAX_ORDER) return EDG_EINVAL;
  if (!(cfg->mechanisms == 0 || cfg->mechanisms == 3)) return EDG_EINVAL;
  if (cfg->n_runs < 1 || cfg->n_runs > MAX_RUNS) return EDG_EINVAL;
  if (cfg->n_clusters < 1 || cfg->n_clusters > MAX_CLUSTERS) return EDG_EINVAL;
  if (!(cfg->cfl > 0) || cfg->lambda > 1.0 || (cfg->lambda > 0 && cfg->lambda <= 0.5)) return EDG_EINVAL;
  if (!pick(cfg->fp64, cfg->order, cfg->mechanisms).level) return EDG_EINVAL;
  if (cfg->flags & ~(EDG_FLAG_GRAPH | EDG_FLAG_POISON | EDG_FLAG_SHUFFLE | EDG_FLAG_CHECK_FINITE |
                     EDG_FLAG_POISON_EARLY))
    return EDG_EINVAL;
  if (hipSetDevice(cfg->device) != hipSuccess) return EDG_EHIP;
  edg_ctx* c = new (std::nothrow) edg_ctx;
  if (!c) return EDG_ENOMEM;
  c->cfg = *cfg;
  c->O = cfg->order;
  c->B = n_basis(c->O);
  c->F = n_face_basis(c->O);
  c->FP = (c->F + 3) / 4 * 4;
  c->M = cfg->mechanisms;
  c->NQ = 9 + 6 * c->M;
  c->dirs = edg::sparse_directions(c->O);
  c->runs = cfg->n_runs;
  c->src_of_run.assign(c->runs, {});
  if (cfg->hip_stream) {
    c->stream = (hipStream_t)cfg->hip_stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return EDG_EHIP;
    }
    c->own_stream = true;
  }
  *out = c;
  return EDG_OK;
}

int edg_upload_mesh(edg_ctx* c, int64_t K, const int64_t* tv, const double* xyz, const int8_t* face_bc) {
  if (!c) return EDG_EINVAL;
  if (K <= 0 || !tv || !xyz) return fail(c, EDG_EINVAL, "empty mesh or null arrays");
  if (K > (int64_t)0x7fffffff / 8) return fail(c, EDG_EINVAL, "too many tets");
  c->K = K;
  c->loc = edg_ctx::Locator{};
  c->perm.assign(K, {0, 1, 2, 3});
  c->nbr.assign(K * 4, -1);
  c->nbr_face.assign(K * 4, -1);
  c->bc.assign(K * 4, 0);
  c->Gm.assign(K * 9, 0.0);
  c->absdet.assign(K, 0.0);
  c->inradius.assign(K, 0.0);
  c->normals.assign(K * 12, 0.0);
  c->areas.assign(K * 4, 0.0);
  c->X.assign(K * 12, 0.0);
  c->have_mesh = c->have_mat = c->have_clusters = false;
  struct FaceKey {
    int64_t a, b, cc, id;
  };
  std::vector<FaceKey> faces((size_t)K * 4);
  for (int64_t k = 0; k < K; ++k) {
    std::array<int, 4>& p = c->perm[k];
    std::sort(p.begin(), p.end(), [&](int x, int y) { return tv[k * 4 + x] < tv[k * 4 + y]; });
    for (int m = 0; m + 1 < 4; ++m)
      if (tv[k * 4 + p[m]] == tv[k * 4 + p[m + 1]])
        return fail(c, EDG_EMESH, "tet " + std::to_string(k) + " repeats a vertex id");
    for (int m = 0; m < 4; ++m)
      for (int d = 0; d < 3; ++d) c->X[k * 12 + m * 3 + d] = xyz[(k * 4 + p[m]) * 3 + d];
    for (int i = 0; i < 4; ++i) {
      int64_t v[3], n = 0;
      for (int m = 0; m < 4; ++m)
        if (m != i) v[n++] = tv[k * 4 + p[m]];
      faces[k * 4 + i] = {v[0], v[1], v[2], k * 4 + i};
      c->bc[k * 4 + i] = face_bc ? face_bc[k * 4 + p[i]] : 0;
    }
    // geometry in the sorted frame
    const double* X = &c->X[k * 12];
    double J[9], Gi[9], det;
    for (int d = 0; d < 3; ++d)
      for (int m = 0; m < 3; ++m) J[d * 3 + m] = X[(m + 1) * 3 + d] - X[d];
    inverse3(J, Gi, det);
    if (!(std::fabs(det) > 0) || !std::isfinite(det)) return fail(c, EDG_EMESH, "degenerate tet " + std::to_string(k));
    for (int j = 0; j < 9; ++j) c->Gm[k * 9 + j] = Gi[j];
    c->absdet[k] = std::fabs(det);
    double asum = 0.0;
    for (int i = 0; i < 4; ++i) {
      int a[3], n = 0;
      for (int m = 0; m < 4; ++m)
        if (m != i) a[n++] = m;
      double e1[3], e2[3], cr[3];
      for (int d = 0; d < 3; ++d) {
        e1[d] = X[a[1] * 3 + d] - X[a[0] * 3 + d];
        e2[d] = X[a[2] * 3 + d] - X[a[0] * 3 + d];
      }
      cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
      cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
      cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
      const double nrm = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      double s = 0.0;
      for (int d = 0; d < 3; ++d) s += cr[d] * (X[i * 3 + d] - X[a[0] * 3 + d]);
      const double sg = s > 0 ? -1.0 : 1.0;
      for (int d = 0; d < 3; ++d) c->normals[(k * 4 + i) * 3 + d] = sg * cr[d] / nrm;
      c->areas[k * 4 + i] = 0.5 * nrm;
      asum += 0.5 * nrm;
    }
    c->inradius[k] = 3.0 * (c->absdet[k] / 6.0) / asum;
  }
  std::sort(faces.begin(), faces.end(), [](const FaceKey& x, const FaceKey& y) {
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    if (x.cc != y.cc) return x.cc < y.cc;
    return x.id < y.id;
  });
  for (size_t s = 0; s < faces.size();) {
    size_t e = s + 1;
    while (e < faces.size() && faces[e].a == faces[s].a && faces[e].b == faces[s].b && faces[e].cc == faces[s].cc) ++e;
    if (e - s > 2) return fail(c, EDG_EMESH, "a face is shared by more than two tets");
    if (e - s == 2) {
      const int64_t f0 = faces[s].id, f1 = faces[s + 1].id;
      if (c->bc[f0] != 0 || c->bc[f1] != 0) return fail(c, EDG_EMESH, "a matched face carries a boundary tag");
      c->nbr[f0] = f1 / 4;
      c->nbr_face[f0] = f1 % 4;
      c->nbr[f1] = f0 / 4;
      c->nbr_face[f1] = f0 % 4;
    } else {
      const int64_t f0 = faces[s].id;
      if (c->bc[f0] != EDG_BC_FREE && c->bc[f0] != EDG_BC_ABSORB)
        return fail(c, EDG_EMESH, "face " + std::to_string(f0 % 4) + " of tet " + std::to_string(f0 / 4) +
                                      " has no neighbour and no boundary tag");
    }
    s = e;
  }
  c->have_mesh = true;
  return EDG_OK;
}

}  // extern "C"

namespace {

// edg_upload_materials with device pointers: range check on the device
// (nothing changes if it fails), a device copy of the caller's arrays, and
// the material words of the tables rebuilt on the device
template <class R>
int upload_materials_device(edg_ctx* c, const double* rho, const double* vp, const double* vs, const double* omega,
                            const double* yp, const double* ys) {
  HIPCHK(c, hipSetDevice(c->cfg.device));
  const int64_t K = c->K;
  const int M = c->M;
  int rc;
  if ((rc = dev_reserve(c, c->dflag, sizeof(unsigned)))) return rc;
  HIPCHK(c, hipMemsetAsync(c->dflag.p, 0, sizeof(unsigned), c->stream));
  const MatIn in{rho, vp, vs, M > 0 ? yp : nullptr, M > 0 ? ys : nullptr};
  if ((rc = launch_check_materials(in, K, (unsigned*)c->dflag.p, c->stream)))
    return fail(c, EDG_EHIP, std::string("material check kernel: ") + hipGetErrorString((hipError_t)rc));
  unsigned bad = 0;
  std::vector<double> om(M);
  HIPCHK(c, hipMemcpyAsync(&bad, c->dflag.p, sizeof bad, hipMemcpyDeviceToHost, c->stream));
  if (M > 0) HIPCHK(c, hipMemcpyAsync(om.data(), omega, M * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (bad) return fail(c, EDG_EINVAL, std::to_string(bad) + " elements have materials out of range");
  const size_t mw = 3 + 2 * (size_t)M;
  if ((rc = dev_reserve(c, c->dmat, (size_t)K * mw * sizeof(double)))) return rc;
  double* d = (double*)c->dmat.p;
  HIPCHK(c, hipMemcpyAsync(d, rho, K * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(d + K, vp, K * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(d + 2 * K, vs, K * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (M > 0) {
    HIPCHK(c, hipMemcpyAsync(d + 3 * K, yp, K * M * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(d + 3 * K + K * M, ys, K * M * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  }
  c->omega = om;
  c->mat_host_valid = false;
  c->have_mat = true;
  drop_checkpoints(c);
  c->amat_valid = false;
  if (c->have_clusters) {   // re-derive the material words of the tables, keep clusters and state
    const MatIn own{d, d + K, d + 2 * K, M > 0 ? d + 3 * K : nullptr, M > 0 ? d + 3 * K + K * M : nullptr};
    if ((rc = dev_reserve(c, c->amat, (size_t)c->Kp * mw * sizeof(double)))) return rc;
    if ((rc = launch_pack_materials<R>(own, M, c->Kp, (const long long*)c->d_i2u.p, (const long long*)c->d_nbr.p,
                                       (R*)c->P.p, (double*)c->amat.p, c->stream)))
      return fail(c, EDG_EHIP, std::string("material table kernel: ") + hipGetErrorString((hipError_t)rc));
    c->amat_valid = true;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return EDG_OK;
}

}  // namespace

extern "C" {

int edg_upload_materials(edg_ctx* c, const double* rho, const double* vp, const double* vs, const double* omega,
                         const double* yp, const double* ys, int32_t on_device) {
  if (!c) return EDG_EINVAL;
  if (!c->have_mesh) return fail(c, EDG_ESTATE, "upload the mesh first");
  if (!rho || !vp || !vs) return fail(c, EDG_EINVAL, "null material array");
  if (c->M > 0 && (!omega || !yp || !ys)) return fail(c, EDG_EINVAL, "anelastic run needs omega, yp, ys");
  if (on_device != 0 && on_device != 1) return fail(c, EDG_EINVAL, "on_device must be 0 or 1");
  if (on_device)
    return c->cfg.fp64 ? upload_materials_device<double>(c, rho, vp, vs, omega, yp, ys)
                       : upload_materials_device<float>(c, rho, vp, vs, omega, yp, ys);
  const int64_t K = c->K;
  for (int64_t k = 0; k < K; ++k)
    if (!(rho[k] > 0) || !(vs[k] > 0) || !(vp[k] > std::sqrt(4.0 / 3.0) * vs[k]))
      return fail(c, EDG_EINVAL, "material of element " + std::to_string(k) + " out of range");
  c->rho.assign(rho, rho + K);
  c->vp.assign(vp, vp + K);
  c->vs.assign(vs, vs + K);
  if (c->M > 0) {
    c->omega.assign(omega, omega + c->M);
    c->yp.assign(yp, yp + K * c->M);
    c->ys.assign(ys, ys + K * c->M);
  } else {
    c->omega.clear();
  }
  c->have_mat = true;
  c->mat_host_valid = true;
  drop_checkpoints(c);
  c->amat_valid = false;
  if (c->have_clusters) {  // re-derive operators, keep clusters and state
    if (c->cfg.fp64) {
      std::vector<double> P;
      std::vector<int> FI;   // unchanged by materials (the device copy keeps the receiver slots)
      pack_tables<double>(c, P, FI);
      HIPCHK(c, hipMemcpy(c->P.p, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
      std::vector<float> P;
      std::vector<int> FI;
      pack_tables<float>(c, P, FI);
      HIPCHK(c, hipMemcpy(c->P.p, P.data(), P.size() * sizeof(float), hipMemcpyHostToDevice));
    }
  }
  return EDG_OK;
}

int edg_upload_clusters(edg_ctx* c, const int32_t* cluster) {
  if (!c) return EDG_EINVAL;
  if (!c->have_mesh || !c->have_mat) return fail(c, EDG_ESTATE, "upload mesh and materials first");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  int rc = ensure_host_materials(c);
  if (rc) return rc;
  drop_checkpoints(c);
  c->amat_valid = false;
  const int64_t K = c->K;
  const int Nc = c->cfg.n_clusters, O = c->O;
  std::vector<double> dt(K);
  for (int64_t k = 0; k < K; ++k) dt[k] = c->cfg.cfl * 2.0 * c->inradius[k] / ((2.0 * (O - 1) + 1.0) * c->vp[k]);
  c->dt_min = *std::min_element(dt.begin(), dt.end());
  if (cluster) {
    c->cl.assign(K, 0);
    for (int64_t k = 0; k < K; ++k) {
      if (cluster[k] < 1 || cluster[k] > Nc) return fail(c, EDG_EINVAL, "cluster id out of range");
      c->cl[k] = cluster[k] - 1;
    }
    for (int64_t k = 0; k < K; ++k)
      for (int i = 0; i < 4; ++i) {
        const int64_t n = c->nbr[k * 4 + i];
        if (n >= 0 && std::abs(c->cl[n] - c->cl[k]) > 1)
          return fail(c, EDG_EINVAL, "face neighbours differ by more than one cluster");
      }
    c->lam = c->cfg.lambda > 0 ? c->cfg.lambda : 1.0;
    c->speedup = cluster_speedup(c->cl, c->lam, Nc);
  } else {
    cluster_all(K, dt.data(), c->nbr.data(), Nc, c->cfg.lambda, c->cl, c->lam, c->speedup);
  }
  for (int l = 0; l < MAX_CLUSTERS; ++l) c->dt_cl[l] = std::ldexp(c->lam * c->dt_min, l);
  // reorder: by cluster, then caller order; every cluster range starts on a
  // group boundary so that a workgroup never mixes clusters
  for (int l = 0; l < MAX_CLUSTERS; ++l) c->cl_count[l] = 0;
  for (int64_t k = 0; k < K; ++k) c->cl_count[c->cl[k]]++;
  int64_t start[MAX_CLUSTERS + 1];
  start[0] = 0;
  for (int l = 0; l < MAX_CLUSTERS; ++l) {
    const int64_t vend = start[l] + (l < Nc ? c->cl_count[l] : 0);
    start[l + 1] = (vend + EPW - 1) / EPW * EPW;
    c->cl_vend[l] = (int)vend;
    c->cl_end[l] = (int)start[l + 1];
  }
  c->Kp = std::max<int64_t>(start[MAX_CLUSTERS], EPW);
  c->G = c->Kp / EPW;
  c->internal_to_user.assign(c->Kp, -1);
  c->user_to_internal.resize(K);
  {
    int64_t pos[MAX_CLUSTERS];
    for (int l = 0; l < MAX_CLUSTERS; ++l) pos[l] = start[l];
    for (int64_t k = 0; k < K; ++k) {
      const int64_t ki = pos[c->cl[k]]++;
      c->internal_to_user[ki] = k;
      c->user_to_internal[k] = ki;
    }
  }
  // device state: tables shared by the runs, then every run's state
  const size_t rs = c->cfg.fp64 ? sizeof(double) : sizeof(float);
  if ((rc = dev_upload(c, c->d_i2u, c->internal_to_user.data(), c->Kp * sizeof(int64_t))) ||
      (rc = dev_upload(c, c->d_nbr, c->nbr.data(), c->nbr.size() * sizeof(int64_t))))
    return rc;
  if (c->cfg.fp64) {
    std::vector<double> P;
    pack_tables<double>(c, P, c->FI_host);
    if ((rc = dev_upload(c, c->P, P.data(), P.size() * sizeof(double)))) return rc;
  } else {
    std::vector<float> P;
    pack_tables<float>(c, P, c->FI_host);
    if ((rc = dev_upload(c, c->P, P.data(), P.size() * sizeof(float)))) return rc;
  }
  if ((rc = dev_upload(c, c->FI, c->FI_host.data(), c->FI_host.size() * sizeof(int)))) return rc;
  const size_t ts = (size_t)4 * LPE * c->FP;   // trace words per element
  c->run_qe = (size_t)c->G * c->B * EPW * LPE;
  c->run_qa = c->M > 0 ? qa_size(c) : 0;
  c->run_t1 = 2 * (size_t)c->Kp * ts;
  c->run_t2 = 2 * (size_t)c->N2 * ts;
  c->run_t3 = 2 * (size_t)c->N3 * ts;
  const size_t R_ = (size_t)c->runs;
  drop_checkpoints(c);
  for (auto& b : c->ckpt_pool) dev_free(b);   // sized for the previous layout
  c->ckpt_pool.clear();
  if ((rc = dev_alloc(c, c->Qe, R_ * c->run_qe * rs))) return rc;
  if ((rc = dev_alloc(c, c->Qa, std::max<size_t>(R_ * c->run_qa, 1) * rs))) return rc;
  if ((rc = dev_alloc(c, c->T1, R_ * c->run_t1 * rs))) return rc;
  if ((rc = dev_alloc(c, c->T2, R_ * c->run_t2 * rs))) return rc;
  if ((rc = dev_alloc(c, c->T3, R_ * c->run_t3 * rs))) return rc;
  HIPCHK(c, hipMemset(c->Qe.p, 0, c->Qe.bytes));
  HIPCHK(c, hipMemset(c->Qa.p, 0, c->Qa.bytes));
  HIPCHK(c, hipMemset(c->T1.p, 0, c->T1.bytes));
  HIPCHK(c, hipMemset(c->T2.p, 0, c->T2.bytes));
  HIPCHK(c, hipMemset(c->T3.p, 0, c->T3.bytes));
  c->n_rec = 0;
  c->n_src = 0;
  for (auto& v : c->src_of_run) v.clear();
  drop_graph(c);
  if ((rc = dev_alloc(c, c->dclock, sizeof(long long)))) return rc;
  HIPCHK(c, hipMemset(c->dclock.p, 0, sizeof(long long)));
  if ((c->cfg.flags & EDG_FLAG_CHECK_FINITE) && !c->dbg.p &&
      (rc = dev_alloc(c, c->dbg, 2 * sizeof(unsigned long long))))
    return rc;
  c->level = 0;
  for (int l = 0; l < MAX_CLUSTERS; ++l) c->nstep[l] = 0;
  c->updates = 0;
  c->have_clusters = true;
  return EDG_OK;
}

int edg_get_clusters(const edg_ctx* c, int32_t* cl_out, double* dt_min, double* lam, double* sync_dt, double* sp) {
  if (!c) return EDG_EINVAL;
  if (!c->have_clusters) return EDG_ESTATE;
  if (cl_out)
    for (int64_t k = 0; k < c->K; ++k) cl_out[k] = c->cl[k] + 1;
  if (dt_min) *dt_min = c->dt_min;
  if (lam) *lam = c->lam;
  if (sync_dt) *sync_dt = c->dt_cl[c->cfg.n_clusters - 1];
  if (sp) *sp = c->speedup;
  return EDG_OK;
}

int edg_set_initial(edg_ctx* c, int32_t run, const double* dofs) {
  if (!c) return EDG_EINVAL;
  if (!c->have_clusters) return fail(c, EDG_ESTATE, "upload clusters first");
  if (run < 0 || run >= c->runs || !dofs) return fail(c, EDG_EINVAL, "bad run or null dofs");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  drop_checkpoints(c);
  return c->cfg.fp64 ? set_dofs_t<double>(c, run, dofs) : set_dofs_t<float>(c, run, dofs);
}

int edg_read_dofs(edg_ctx* c, int32_t run, double* out, int64_t cap) {
  if (!c) return EDG_EINVAL;
  if (!c->have_clusters) return fail(c, EDG_ESTATE, "upload clusters first");
  if (run < 0 || run >= c->runs || !out) return fail(c, EDG_EINVAL, "bad run or null output");
  if (cap < c->K * c->NQ * c->B) return fail(c, EDG_ECAP, "output capacity too small");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  return c->cfg.fp64 ? get_dofs_t<double>(c, run, out) : get_dofs_t<float>(c, run, out);
}

int edg_set_dofs_subset(edg_ctx* c, int32_t run, int64_t n, const int64_t* ids, const double* dofs) {
  if (!c) return EDG_EINVAL;
  if (!c->have_clusters) return fail(c, EDG_ESTATE, "upload clusters first");
  if (run < 0 || run >= c->runs || n < 0 || (n > 0 && (!ids || !dofs))) return fail(c, EDG_EINVAL, "bad arguments");
  for (int64_t i = 0; i < n; ++i)
    if (ids[i] < 0 || ids[i] >= c->K) return fail(c, EDG_EINVAL, "element index out of range");
  if (n == 0) return EDG_OK;
  HIPCHK(c, hipSetDevice(c->cfg.device));
  drop_checkpoints(c);
  return c->cfg.fp64 ? subset_dofs_t<double>(c, run, n, ids, dofs, nullptr)
                     : subset_dofs_t<float>(c, run, n, ids, dofs, nullptr);
}

int edg_read_dofs_subset(edg_ctx* c, int32_t run, int64_t n, const int64_t* ids, double* out, int64_t cap) {
  if (!c) return EDG_EINVAL;
  if (!c->have_clusters) return fail(c, EDG_ESTATE, "upload clusters first");
  if (run < 0 || run >= c->runs || n < 0 || (n > 0 && (!ids || !out))) return fail(c, EDG_EINVAL, "bad arguments");
  if (cap < n * c->NQ * c->B) return fail(c, EDG_ECAP, "output capacity too small");
  for (int64_t i = 0; i < n; ++i)
    if (ids[i] < 0 || ids[i] >= c->K) return fail(c, EDG_EINVAL, "element index out of range");
  if (n == 0) return EDG_OK;
  HIPCHK(c, hipSetDevice(c->cfg.device));
  return c->cfg.fp64 ? subset_dofs_t<double>(c, run, n, ids, nullptr, out)
                     : subset_dofs_t<float>(c, run, n, ids, nullptr, out);
}

int edg_set_sources(edg_ctx* c, int32_t run, int64_t n, const double* xyz, const double* moment, int32_t kind,
                    const double* par) {
  if (!c) return EDG_EINVAL;
  if (!c->have_clusters) return fail(c, EDG_ESTATE, "upload clusters first");
  if (run < 0 || run >= c->runs || n < 0 || (n > 0 && (!xyz || !moment || !par)))
    return fail(c, EDG_EINVAL, "bad source arguments");
  if (kind != EDG_STF_RICKER && kind != EDG_STF_HANN) return fail(c, EDG_EINVAL, "unknown source time function");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  drop_checkpoints(c);
  std::vector<edg_ctx::Source> list;
  for (int64_t s = 0; s < n; ++s) {
    double xi[3];
    const int64_t k = locate(c, xyz + 3 * s, xi);
    if (k < 0) return fail(c, EDG_EINVAL, "source " + std::to_string(s) + " is outside the mesh");
    edg_ctx::Source src;
    src.elem = (int)c->user_to_internal[k];
    src.kind = kind;
    src.par[0] = par[2 * s];
    src.par[1] = par[2 * s + 1];
    for (int m = 0; m < 6; ++m) src.moment[m] = moment[6 * s + m];
    src.idet = 1.0 / c->absdet[k];
    src.phi = eval_basis(c->O, xi);
    list.push_back(std::move(src));
  }
  c->src_of_run[run] = std::move(list);
  drop_graph(c);
  // the device list holds the sources of every run
  std::vector<int> rn, el, kd;
  std::vector<double> pr, mo, phi, idet;
  for (int r = 0; r < c->runs; ++r)
    for (const auto& src : c->src_of_run[r]) {
      rn.push_back(r);
      el.push_back(src.elem);
      kd.push_back(src.kind);
      pr.insert(pr.end(), src.par, src.par + 2);
      mo.insert(mo.end(), src.moment, src.moment + 6);
      phi.insert(phi.end(), src.phi.begin(), src.phi.end());
      idet.push_back(src.idet);
    }
  const size_t ns = rn.size();
  int rc;
  if ((rc = dev_upload(c, c->s_run, rn.data(), ns * sizeof(int)))) return rc;
  if ((rc = dev_upload(c, c->s_elem, el.data(), ns * sizeof(int)))) return rc;
  if ((rc = dev_upload(c, c->s_kind, kd.data(), ns * sizeof(int)))) return rc;
  if ((rc = dev_upload(c, c->s_par, pr.data(), pr.size() * sizeof(double)))) return rc;
  if ((rc = dev_upload(c, c->s_mom, mo.data(), mo.size() * sizeof(double)))) return rc;
  if ((rc = dev_upload(c, c->s_phi, phi.data(), phi.size() * sizeof(double)))) return rc;
  if ((rc = dev_upload(c, c->s_idet, idet.data(), ns * sizeof(double)))) return rc;
  c->n_src = (int)ns;
  return EDG_OK;
}

int edg_set_receivers(edg_ctx* c, int64_t n, const double* xyz, double dt_sample, int64_t ns) {
  if (!c) return EDG_EINVAL;
  if (!c->have_clusters) return fail(c, EDG_ESTATE, "upload clusters first");
  if (n < 0 || (n > 0 && (!xyz || !(dt_sample > 0) || ns <= 0))) return fail(c, EDG_EINVAL, "bad receiver arguments");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  std::vector<int> el(n), slot(n), rs_slot((size_t)c->Kp, -1);   // receiver slot per element
  std::vector<double> phi((size_t)n * c->B);
  int nslots = 0;
  for (int64_t r = 0; r < n; ++r) {
    double xi[3];
    const int64_t k = locate(c, xyz + 3 * r, xi);
    if (k < 0) return fail(c, EDG_EINVAL, "receiver " + std::to_string(r) + " is outside the mesh");
    const int64_t ki = c->user_to_internal[k];
    el[r] = (int)ki;
    if (rs_slot[ki] < 0) rs_slot[ki] = nslots++;
    slot[r] = rs_slot[ki];
    auto v = eval_basis(c->O, xi);
    std::copy(v.begin(), v.end(), phi.begin() + r * c->B);
  }
  int rc;
  for (int64_t ki = 0; ki < c->Kp; ++ki) c->FI_host[(size_t)ki * FI_WORDS + 15] = rs_slot[ki];
  if ((rc = dev_upload(c, c->FI, c->FI_host.data(), c->FI_host.size() * sizeof(int)))) return rc;
  const size_t rsz = c->cfg.fp64 ? sizeof(double) : sizeof(float);
  c->run_recd = (size_t)std::max(nslots, 1) * c->O * LPE * c->B;
  if ((rc = dev_alloc(c, c->RecD, (size_t)c->runs * c->run_recd * rsz))) return rc;
  if ((rc = dev_upload(c, c->r_elem, el.data(), n * sizeof(int)))) return rc;
  if ((rc = dev_upload(c, c->r_slot, slot.data(), n * sizeof(int)))) return rc;
  if ((rc = dev_upload(c, c->r_phi, phi.data(), phi.size() * sizeof(double)))) return rc;
  if ((rc = dev_alloc(c, c->r_out, (size_t)c->runs * std::max<int64_t>(n, 1) * ns * LPE * sizeof(double))))
    return rc;
  HIPCHK(c, hipMemset(c->r_out.p, 0, c->r_out.bytes));
  drop_graph(c);
  c->n_rec = (int)n;
  c->rec_ns = ns;
  c->rec_dt = dt_sample;
  return EDG_OK;
}

}  // extern "C" (the C++ helpers below have C++ linkage)

namespace {

struct AdvanceArgs {
  Fns fn;
  KPtrs p;
  SrcArgs sa;
  RecArgs ra;
};

AdvanceArgs advance_args(edg_ctx* c) {
  AdvanceArgs A;
  A.fn = pick(c->cfg.fp64, c->O, c->M);
  A.p = kptrs(c);
  A.sa.n = c->n_src;
  A.sa.run = (const int*)c->s_run.p;
  A.sa.elem = (const int*)c->s_elem.p;
  A.sa.kind = (const int*)c->s_kind.p;
  A.sa.par = (const double*)c->s_par.p;
  A.sa.moment = (const double*)c->s_mom.p;
  A.sa.phi = (const double*)c->s_phi.p;
  A.sa.inv_det = (const double*)c->s_idet.p;
  A.ra.n = c->n_rec;
  A.ra.elem = (const int*)c->r_elem.p;
  A.ra.slot = (const int*)c->r_slot.p;
  A.ra.phi = (const double*)c->r_phi.p;
  A.ra.dt_sample = c->rec_dt;
  A.ra.ns = c->rec_ns;
  A.ra.run0 = 0;
  A.ra.out = (double*)c->r_out.p;
  return A;
}

// finest level j (1..2^(Nc-1)) of a cycle: the coarsest cluster that ends a step there
int level_lmax(const edg_ctx* c, int64_t j) {
  int lmax = 0;
  for (int l = 1; l < c->cfg.n_clusters; ++l)
    if (j % ((int64_t)1 << l) == 0) lmax = l;
  return lmax;
}

int64_t level_updates(const edg_ctx* c, int lmax) {
  int64_t u = 0;
  for (int l = 0; l <= lmax; ++l) u += c->cl_count[l] * c->runs;
  return u;
}

// The launches of one LTS cycle (Sec. V-B: per finest level, the sources of
// the steps that end there, the fused finish-and-predict launch, the
// receivers of the new predictions), then the device clock tick.  `last`:
// the final level only finishes (no prediction is needed after the advance).
// `timed`: per-level events (not inside a graph capture).
int emit_cycle(edg_ctx* c, const AdvanceArgs& A, bool last, bool timed) {
  const int64_t per = (int64_t)1 << (c->cfg.n_clusters - 1);
  int rc;
  for (int64_t j = 1; j <= per; ++j) {
    const int lmax = level_lmax(c, j);
    LevelArgs a = base_args(c);
    a.jrel = (int)j;
    a.end = c->cl_end[lmax];
    if (c->n_src > 0 && (rc = A.fn.src(A.p, a, A.sa, c->stream)))
      return fail(c, EDG_EHIP, std::string("source kernel: ") + hipGetErrorString((hipError_t)rc));
    const bool fin = last && j == per;
    a.kind = fin ? KIND_NEIGHBOR : KIND_FUSED;
    if (timed) {
      if ((rc = launch_timed(c, A.fn, A.p, a, level_updates(c, lmax)))) return rc;
    } else if ((rc = launch_runs(c, A.fn, A.p, a))) {
      return rc;
    }
    if ((rc = poison_after(c, A.p, a))) return rc;
    if (!fin && c->n_rec > 0 && (rc = A.fn.rec(A.p, a, A.ra, c->runs, c->stream)))
      return fail(c, EDG_EHIP, std::string("receiver kernel: ") + hipGetErrorString((hipError_t)rc));
  }
  if ((rc = launch_tick((long long*)c->dclock.p, per, c->stream)))
    return fail(c, EDG_EHIP, std::string("clock kernel: ") + hipGetErrorString((hipError_t)rc));
  return 0;
}

int64_t cycle_updates(const edg_ctx* c) {
  const int64_t per = (int64_t)1 << (c->cfg.n_clusters - 1);
  int64_t u = 0;
  for (int64_t j = 1; j <= per; ++j) u += level_updates(c, level_lmax(c, j));
  return u;
}

// capture one full (non-final) cycle as a graph: only kernel launches, no
// memory set or copy nodes
int capture_cycle(edg_ctx* c, const AdvanceArgs& A) {
  drop_graph(c);
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  const int rc = emit_cycle(c, A, false, false);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(c, EDG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  c->cycle_graph = g;
  HIPCHK(c, hipGraphInstantiate(&c->cycle_exec, g, nullptr, nullptr, 0));
  return 0;
}

}  // namespace

namespace {

// words of the B1 / B2 / B3 face traces of every run (T1, T2, T3 in turn)
size_t trace_words(const edg_ctx* c) { return (size_t)c->runs * (c->run_t1 + c->run_t2 + c->run_t3); }

// nc >= 1 LTS cycles from the current synchronisation point: predict every
// element, then the cycles (the last one only finishes its steps).  traces:
// null for the context's own trace buffers, else the base of trace_words(c)
// words that hold them for this advance only (every level then launches
// eagerly and untimed: no graph, no event).  Within one advance from a
// synchronisation point every trace slot is written before it is read, so
// the traces carry nothing between calls.
int advance_cycles(edg_ctx* c, int64_t nc, char* traces = nullptr) {
  const int Nc = c->cfg.n_clusters;
  const int64_t per = (int64_t)1 << (Nc - 1);
  AdvanceArgs A = advance_args(c);
  if (traces) {
    const size_t rs = c->cfg.fp64 ? sizeof(double) : sizeof(float);
    A.p.T1 = traces;
    A.p.T2 = traces + (size_t)c->runs * c->run_t1 * rs;
    A.p.T3 = traces + (size_t)c->runs * (c->run_t1 + c->run_t2) * rs;
  }
  const bool timed = traces == nullptr;
  const bool graph = timed && (c->cfg.flags & EDG_FLAG_GRAPH) != 0;
  c->ev_used = 0;
  c->ev_updates.clear();
  c->ev_launches.clear();

  // predict every element at the start (level offset 0)
  LevelArgs a = base_args(c);
  a.kind = KIND_PREDICT;
  a.jrel = 0;
  a.end = c->cl_end[Nc - 1];
  int rc = poison_all(c, A.p);
  if (rc) return rc;
  rc = timed ? launch_timed(c, A.fn, A.p, a, 0) : launch_runs(c, A.fn, A.p, a);
  if (rc) return rc;
  if (c->n_rec > 0 && (rc = A.fn.rec(A.p, a, A.ra, c->runs, c->stream)))
    return fail(c, EDG_EHIP, std::string("receiver kernel: ") + hipGetErrorString((hipError_t)rc));
  for (int64_t k = 0; k < nc; ++k) {
    const bool last = k + 1 == nc;
    if (graph && !last) {
      if (!c->cycle_exec && (rc = capture_cycle(c, A))) return rc;
      if ((rc = timed_begin(c, cycle_updates(c), (int)per))) return rc;
      HIPCHK(c, hipGraphLaunch(c->cycle_exec, c->stream));
      if ((rc = timed_end(c))) return rc;
    } else if ((rc = emit_cycle(c, A, last, timed))) {
      return rc;
    }
    c->updates += cycle_updates(c);
  }
  c->level += nc * per;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if ((rc = check_finite(c))) return rc;
  if (c->timing) {
    for (size_t i = 0; i < c->ev_used; ++i) {
      float ms = 0.f;
      HIPCHK(c, hipEventElapsedTime(&ms, c->ev_pool[i].first, c->ev_pool[i].second));
      c->t_ms += ms;
      c->t_launches += c->ev_launches[i];
      c->t_updates += c->ev_updates[i];
    }
  }
  return EDG_OK;
}

// stores the current state of every run as a checkpoint at the current
// level: the elastic rows of all runs, then their memory variables
int store_checkpoint(edg_ctx* c) {
  const size_t rs = c->cfg.fp64 ? sizeof(double) : sizeof(float);
  const size_t we = c->runs * c->run_qe, wa = c->runs * c->run_qa;
  const size_t need = (we + wa) * rs;
  c->ckpts.emplace_back(c->level, DevBuf{});
  int rc = 0;
  auto it = std::find_if(c->ckpt_pool.begin(), c->ckpt_pool.end(), [&](const DevBuf& b) { return b.bytes >= need; });
  if (it != c->ckpt_pool.end()) {
    c->ckpts.back().second = *it;
    c->ckpt_pool.erase(it);
  } else {
    rc = dev_alloc(c, c->ckpts.back().second, need);
    if (rc && !c->ckpt_pool.empty()) {   // the pool's buffers are too small: give them back and retry
      for (auto& b : c->ckpt_pool) dev_free(b);
      c->ckpt_pool.clear();
      rc = dev_alloc(c, c->ckpts.back().second, need);
    }
  }
  if (rc) {
    c->ckpts.pop_back();
    return rc;
  }
  char* dst = (char*)c->ckpts.back().second.p;
  HIPCHK(c, hipMemcpyAsync(dst, c->Qe.p, we * rs, hipMemcpyDeviceToDevice, c->stream));
  if (wa) HIPCHK(c, hipMemcpyAsync(dst + we * rs, c->Qa.p, wa * rs, hipMemcpyDeviceToDevice, c->stream));
  return 0;
}

// ahist: per level of the longest segment (levels 0 .. J-1) the run-0 state
// of the element groups that predict there (groups [0, cl_end[lmax(j)] / 7),
// elastic words then memory-variable words), packed level after level
size_t hist_group_words(const edg_ctx* c) { return (c->run_qe + c->run_qa) / (size_t)c->G; }
size_t hist_level_groups(const edg_ctx* c, int64_t j) { return (size_t)c->cl_end[level_lmax(c, j)] / EPW; }
// words of the records of levels 0 .. j-1 (the pattern repeats every cycle)
size_t hist_words_before(const edg_ctx* c, int64_t j) {
  const int64_t per = (int64_t)1 << (c->cfg.n_clusters - 1);
  size_t cyc = 0, part = 0;
  for (int64_t i = 0; i < per; ++i) {
    const size_t g = hist_level_groups(c, i);
    cyc += g;
    if (i < j % per) part += g;
  }
  return ((size_t)(j / per) * cyc + part) * hist_group_words(c);
}
char* hist_rec_e(edg_ctx* c, int64_t j) {
  const size_t rs = c->cfg.fp64 ? sizeof(double) : sizeof(float);
  return (char*)c->ahist.p + hist_words_before(c, j) * rs;
}
char* hist_rec_a(edg_ctx* c, int64_t j) {
  const size_t rs = c->cfg.fp64 ? sizeof(double) : sizeof(float);
  return hist_rec_e(c, j) + hist_level_groups(c, j) * (c->run_qe / (size_t)c->G) * rs;
}
int hist_reserve(edg_ctx* c, int64_t levels) {
  const size_t rs = c->cfg.fp64 ? sizeof(double) : sizeof(float);
  const size_t bytes = hist_words_before(c, levels) * rs;
  if (c->ahist.p && c->ahist.bytes >= bytes) return 0;
  c->hist_valid = false;
  if (dev_reserve(c, c->ahist, bytes))
    return fail(c, EDG_ENOMEM, "the level-state record of a checkpoint segment (" + std::to_string(levels) +
                                   " levels) needs " + std::to_string(bytes) +
                                   " bytes of device memory: use a shorter checkpoint interval");
  return 0;
}

// The J levels of a segment from a synchronisation point, on the state p:
// a predict-only launch, fused finish + predict launches, a finish-only
// launch, each predicting launch also writing the state at the start of its
// predictions into level j's record of ahist.  The context's own advance
// (own = true) also samples the receivers and finishes the last steps; a
// replay stops after the last prediction (the finish is not needed).
int run_recorded_levels(edg_ctx* c, const AdvanceArgs& A, const KPtrs& p, int64_t J, bool own) {
  const int Nc = c->cfg.n_clusters;
  const size_t wa = c->run_qa;
  auto chk = [&](int e, const char* what) {
    return e ? fail(c, EDG_EHIP, std::string(what) + ": " + hipGetErrorString((hipError_t)e)) : 0;
  };
  int rc;
  LevelArgs a = base_args(c);
  a.run0 = 0;
  if ((rc = poison_all(c, p))) return rc;
  for (int64_t j = 0; j <= (own ? J : J - 1); ++j) {
    const int lmax = (j == 0 || j == J) ? Nc - 1 : level_lmax(c, j);
    a.jrel = (int)j;
    a.end = c->cl_end[lmax];
    if (j > 0 && c->n_src > 0 && (rc = chk(A.fn.src(p, a, A.sa, c->stream), "source kernel"))) return rc;
    a.kind = j == 0 ? KIND_PREDICT : (j == J ? KIND_NEIGHBOR : KIND_FUSED);
    a.rec_e = j < J ? (void*)hist_rec_e(c, j) : nullptr;
    a.rec_a = (j < J && wa) ? (void*)hist_rec_a(c, j) : nullptr;
    shuffle_args(c, a, 1);
    if ((rc = chk(A.fn.level(p, a, 1, c->stream), "level kernel"))) return rc;
    if ((rc = poison_after(c, p, a))) return rc;
    if (own && j < J && c->n_rec > 0 && (rc = chk(A.fn.rec(p, a, A.ra, c->runs, c->stream), "receiver kernel")))
      return rc;
  }
  return 0;
}

// nc >= 1 cycles as one segment whose level states the reverse sweep can use
// without a replay: every level runs as the neighbour-data update, the copy
// of the predicting groups' state into ahist, then the prediction (the
// forward split where the plain advance fuses it), with the level clock held
// at the segment start and the level offset counted over the segment
int advance_recorded(edg_ctx* c, int64_t nc) {
  const int Nc = c->cfg.n_clusters;
  const int64_t per = (int64_t)1 << (Nc - 1), J = nc * per;
  int rc = hist_reserve(c, std::max<int64_t>(J, (int64_t)c->ckpt_every * per));
  if (rc) return rc;
  c->hist_valid = false;
  c->ev_used = 0;
  c->ev_updates.clear();
  c->ev_launches.clear();
  const AdvanceArgs A = advance_args(c);
  auto chk = [&](int e, const char* what) {
    return e ? fail(c, EDG_EHIP, std::string(what) + ": " + hipGetErrorString((hipError_t)e)) : 0;
  };
  if ((rc = run_recorded_levels(c, A, A.p, J, true))) return rc;
  if ((rc = chk(launch_tick((long long*)c->dclock.p, J, c->stream), "clock kernel"))) return rc;
  c->updates += nc * cycle_updates(c);
  c->hist_L0 = c->level;
  c->hist_J = J;
  c->hist_run = 0;
  c->level += J;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->hist_valid = true;
  return check_finite(c);
}

// whole LTS cycles from the current time to t (EDG_ENOTSYNC unless t is a
// synchronisation point not before the current time)
int cycles_until(edg_ctx* c, double t, int64_t* nc) {
  const int Nc = c->cfg.n_clusters;
  const double sync = c->dt_cl[Nc - 1];
  const double t_now = (double)c->level * c->dt_cl[0];
  const double cycles = (t - t_now) / sync;
  const double ncd = std::nearbyint(cycles);
  if (!(ncd >= 0) || std::fabs(cycles - ncd) > 1e-9 * std::max(1.0, std::fabs(cycles)))
    return fail(c, EDG_ENOTSYNC, "time is not a synchronisation point after the current time");
  *nc = (int64_t)ncd;
  return 0;
}

}  // namespace

namespace edg {

// The allocation-free advance (edg_advance_to_static): the face traces of
// this advance live in the caller-provided device memory [base, base + cap).
int advance_to_traces(edg_ctx* c, double t, void* base, size_t cap) {
  if (!c->have_clusters) return fail(c, EDG_ESTATE, "upload clusters first");
  if (c->ckpt_every > 0)
    return fail(c, EDG_ESTATE, "the allocation-free advance stores no checkpoints: turn checkpointing off");
  const size_t rs = c->cfg.fp64 ? sizeof(double) : sizeof(float);
  const size_t need = trace_words(c) * rs;
  if (need > cap)
    return fail(c, EDG_EINVAL, "the face traces of this context need " + std::to_string(need) +
                                   " bytes; the static scratch holds " + std::to_string(cap));
  int64_t nc = 0;
  int rc = cycles_until(c, t, &nc);
  if (rc || nc == 0) return rc;
  // nothing is read before it is written, but the traces start from zeros
  // as the context's own buffers do after an upload
  if ((rc = launch_zero_words(base, need / 4, c->stream)))
    return fail(c, EDG_EHIP, std::string("fill kernel: ") + hipGetErrorString((hipError_t)rc));
  return advance_cycles(c, nc, (char*)base);
}

int ctx_device(const edg_ctx* c) { return c->cfg.device; }

int ctx_fail(edg_ctx* c, int code, const char* msg) { return fail(c, code, msg); }

}  // namespace edg

extern "C" {

int edg_advance_to(edg_ctx* c, double t) {
  if (!c) return EDG_EINVAL;
  if (!c->have_clusters) return fail(c, EDG_ESTATE, "upload clusters first");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  int64_t nc = 0;
  int rc0 = cycles_until(c, t, &nc);
  if (rc0 || nc == 0) return rc0;
  if (c->ckpt_every <= 0) return advance_cycles(c, nc);
  // checkpointed: segments of at most ckpt_every cycles, each one an advance
  // of its own that starts from a stored state; with one run the final one
  // records its level states, so the reverse sweep starts without a replay
  // (the record holds one run: with several, every segment is replayed)
  for (int64_t done = 0; done < nc;) {
    const int64_t seg = std::min<int64_t>(c->ckpt_every, nc - done);
    int rc = store_checkpoint(c);
    if (rc) return rc;
    if ((rc = done + seg == nc && c->runs == 1 ? advance_recorded(c, seg) : advance_cycles(c, seg))) return rc;
    done += seg;
  }
  return EDG_OK;
}

int edg_set_plan(edg_ctx* c, const edg_plan* plan) {
  if (!c) return EDG_EINVAL;
  if (!plan || (plan->xcd_remap != 0 && plan->xcd_remap != 1) || plan->run_chunk < 0 || plan->run_chunk > MAX_RUNS ||
      (plan->trace_mfma != 0 && plan->trace_mfma != 1))
    return fail(c, EDG_EINVAL, "bad launch plan");
  c->plan = *plan;
  drop_graph(c);
  return EDG_OK;
}

int edg_get_plan(const edg_ctx* c, edg_plan* plan) {
  if (!c || !plan) return EDG_EINVAL;
  *plan = c->plan;
  return EDG_OK;
}

int edg_autotune(edg_ctx* c, int32_t cycles, edg_plan* best_out, double* best_ms) {
  if (!c) return EDG_EINVAL;
  if (!c->have_clusters) return fail(c, EDG_ESTATE, "upload clusters first");
  if (cycles < 1) return fail(c, EDG_EINVAL, "cycles must be positive");
  std::vector<edg_plan> cand;
  for (int xcd = 0; xcd <= 1; ++xcd)
    for (int chunk : {0, 16, 8, 4})
      if (chunk == 0 || chunk < c->runs) cand.push_back(edg_plan{xcd, chunk, 0});
  const bool timing = c->timing;
  const int64_t l0 = c->t_launches, u0 = c->t_updates;
  const double m0 = c->t_ms;
  const double sync = c->dt_cl[c->cfg.n_clusters - 1];
  edg_plan best = c->plan;
  double best_t = 1e300;
  int rc;
  for (const edg_plan& pl : cand) {
    if ((rc = edg_set_plan(c, &pl))) return rc;
    c->timing = true;
    const double before = c->t_ms;
    rc = edg_advance_to(c, edg_time(c) + cycles * sync);
    const double spent = c->t_ms - before;
    c->timing = timing;
    if (rc) return rc;
    if (spent < best_t) {
      best_t = spent;
      best = pl;
    }
  }
  // the tuning cycles do not count in the kernel statistics
  c->t_launches = l0;
  c->t_updates = u0;
  c->t_ms = m0;
  if ((rc = edg_set_plan(c, &best))) return rc;
  if (best_out) *best_out = best;
  if (best_ms) *best_ms = best_t / cycles;
  return EDG_OK;
}

int edg_read_receivers(edg_ctx* c, int32_t run, double* out, int64_t cap, int32_t on_device) {
  if (!c) return EDG_EINVAL;
  if (run < 0 || run >= c->runs || !out) return fail(c, EDG_EINVAL, "bad run or null output");
  if (on_device != 0 && on_device != 1) return fail(c, EDG_EINVAL, "on_device must be 0 or 1");
  const int64_t need = (int64_t)c->n_rec * c->rec_ns * LPE;
  if (cap < need) return fail(c, EDG_ECAP, "output capacity too small");
  if (need == 0) return EDG_OK;
  HIPCHK(c, hipSetDevice(c->cfg.device));
  const double* src = (const double*)c->r_out.p + (size_t)run * need;
  if (on_device) {
    HIPCHK(c, hipMemcpyAsync(out, src, need * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    HIPCHK(c, hipMemcpy(out, src, need * sizeof(double), hipMemcpyDeviceToHost));
  }
  return EDG_OK;
}

int edg_set_checkpointing(edg_ctx* c, int32_t every_cycles) {
  if (!c) return EDG_EINVAL;
  if (every_cycles < 0) return fail(c, EDG_EINVAL, "negative checkpoint interval");
  (void)hipSetDevice(c->cfg.device);
  drop_checkpoints(c);
  c->ckpt_every = every_cycles;
  return EDG_OK;
}

int edg_rewind(edg_ctx* c) {
  if (!c) return EDG_EINVAL;
  if (!c->have_clusters) return fail(c, EDG_ESTATE, "upload clusters first");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  drop_checkpoints(c);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (DevBuf* b : {&c->Qe, &c->Qa, &c->T1, &c->T2, &c->T3, &c->RecD, &c->r_out})
    if (b->p) HIPCHK(c, hipMemset(b->p, 0, b->bytes));
  HIPCHK(c, hipMemset(c->dclock.p, 0, sizeof(long long)));
  c->level = 0;
  for (int l = 0; l < MAX_CLUSTERS; ++l) c->nstep[l] = 0;
  return EDG_OK;
}

}  // extern "C"

namespace {

// reverse sweep over the checkpointed segments (see edg_adjoint)
template <class R, int O, int M>
int adjoint_sweep(edg_ctx* c, const double* dj_seis, const double* dj_q, double* g_q0, double* g_rho, double* g_vp,
                  double* g_vs, bool dev) {
  const int Nc = c->cfg.n_clusters, FP = c->FP, JB = jb_count(c);
  const size_t rs = sizeof(R), we = c->run_qe, wa = c->run_qa;
  const size_t slot_words = (size_t)4 * ADJ_ROWS * FP;
  // Da is the one-wave kernel's (the two-wave kernel keeps its scratch in De)
  const bool two_wave = std::is_same<R, float>::value && O >= 4;
  const int64_t L_end = c->level;
  const size_t nck = c->ckpts.size();
  int64_t jmax = 1;
  for (size_t i = 0; i < nck; ++i) {
    const int64_t hi = i + 1 < nck ? c->ckpts[i + 1].first : L_end;
    jmax = std::max(jmax, hi - c->ckpts[i].first);
  }
  int rc;
  const size_t n_hist = (size_t)jmax;   // levels 0 .. J-1 of the longest segment
  const void* const slots_before[5] = {c->aS0.p, c->aS1.p, c->aS2.p, c->aS3.p, c->arecDb.p};
  if ((rc = dev_reserve(c, c->aLe, we * rs)) || (rc = dev_reserve(c, c->aLa, std::max<size_t>(wa, 1) * rs)) ||
      (rc = dev_reserve(c, c->aS0, (size_t)c->Kp * slot_words * rs)) ||
      (rc = dev_reserve(c, c->aS1, (size_t)c->Kp * slot_words * rs)) ||
      (rc = dev_reserve(c, c->aS2, (size_t)c->N2 * slot_words * rs)) ||
      (rc = dev_reserve(c, c->aS3, (size_t)c->N3 * slot_words * rs)) ||
      (rc = dev_reserve(c, c->aDe, (size_t)c->G * adjoint_scratch_floats<R, O, M>() * rs)) ||
      (rc = dev_reserve(c, c->aDa, std::max<size_t>(two_wave ? 0 : (size_t)c->G * O * JB * M * 6 * EPW * LPE, 1) * rs)) ||
      (rc = dev_reserve(c, c->agacc, (size_t)c->Kp * NG * sizeof(double))) ||
      (rc = dev_reserve(c, c->arecDb, std::max<size_t>(c->run_recd, 1) * rs)) ||
      (rc = dev_reserve(c, c->aseis, std::max<size_t>((size_t)c->n_rec * c->rec_ns * LPE, 1) * sizeof(double))) ||
      (rc = hist_reserve(c, (int64_t)n_hist)) || (rc = dev_reserve(c, c->afinal, (we + wa) * rs)))
    return rc;
  // the slots and receiver derivatives return to zero at the end of every
  // sweep (each is cleared by its reader; S0 is written before it is read);
  // they are cleared here after a (re)allocation and after a failed sweep
  const void* const slots_now[5] = {c->aS0.p, c->aS1.p, c->aS2.p, c->aS3.p, c->arecDb.p};
  bool clean = c->adj_clean;
  for (int i = 0; i < 5; ++i) clean = clean && slots_before[i] == slots_now[i];
  c->adj_clean = false;
  // the gradient words sum over the runs: J is the sum of the runs' misfits
  HIPCHK(c, hipMemsetAsync(c->agacc.p, 0, c->agacc.bytes, c->stream));
  if (!clean)
    for (DevBuf* b : {&c->aS0, &c->aS1, &c->aS2, &c->aS3, &c->arecDb})
      HIPCHK(c, hipMemsetAsync(b->p, 0, b->bytes, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // the replays run on a state of their own, so the context's DOFs stay
  // those of the final time; one run at a time, so the run stride of the
  // state is zero (the sources of run r land in the same state)
  char* rep_state = (char*)c->afinal.p;

  const AdvanceArgs A0 = advance_args(c);
  KPtrs p = kptrs(c);
  p.Qe = rep_state;
  p.Qa = rep_state + we * rs;
  p.run_qe = p.run_qa = 0;
  APtrs ad;
  ad.Le = c->aLe.p;
  ad.La = c->aLa.p;
  ad.S0 = c->aS0.p;
  ad.S1 = c->aS1.p;
  ad.S2 = c->aS2.p;
  ad.S3 = c->aS3.p;
  ad.De = c->aDe.p;
  ad.Da = c->aDa.p;
  ad.gacc = (double*)c->agacc.p;
  ad.recDb = c->arecDb.p;
  const double* seis_b = (const double*)c->aseis.p;
  auto hist_e = [&](int64_t j) { return (void*)hist_rec_e(c, j); };
  auto hist_a = [&](int64_t j) { return (void*)hist_rec_a(c, j); };
  auto chk = [&](int e, const char* what) {
    return e ? fail(c, EDG_EHIP, std::string(what) + ": " + hipGetErrorString((hipError_t)e)) : 0;
  };
  // the levels of a segment backwards: transposed predictions, then
  // transposed updates (kernel launches only)
  auto backward = [&](LevelArgs a, int64_t J) {
    int e;
    for (int64_t j = J; j >= 0; --j) {
      const int lmax = (j == 0 || j == J) ? Nc - 1 : level_lmax(c, j);
      a.jrel = (int)j;
      a.end = c->cl_end[lmax];
      if (j < J) {
        if (c->n_rec > 0 && dj_seis &&
            (e = chk(launch_receivers_adj<R, O, M>(p, ad, a, A0.ra, seis_b, c->stream), "receiver adjoint kernel")))
          return e;
        ad.Se = hist_e(j);
        ad.Sa = hist_a(j);
        a.kind = KIND_ADJ_PREDICT;
        if ((e = chk(launch_adjoint<R, O, M>(p, ad, a, c->stream), "adjoint kernel"))) return e;
      }
      if (j > 0) {
        a.kind = KIND_ADJ_UPDATE;
        if ((e = chk(launch_adjoint<R, O, M>(p, ad, a, c->stream), "adjoint kernel"))) return e;
      }
    }
    return 0;
  };
  const bool graph = (c->cfg.flags & EDG_FLAG_GRAPH) != 0;
  struct SegGraph {
    int64_t J;
    hipGraph_t g;
    hipGraphExec_t x;
  };
  std::vector<SegGraph> graphs;
  struct GraphsGuard {   // the graphs live for this sweep only
    std::vector<SegGraph>& v;
    ~GraphsGuard() {
      for (auto& q : v) {
        if (q.x) (void)hipGraphExecDestroy(q.x);
        if (q.g) (void)hipGraphDestroy(q.g);
      }
    }
  } graphs_guard{graphs};
  const size_t nqb = (size_t)c->K * c->NQ * c->B, nsb = (size_t)c->n_rec * c->rec_ns * LPE;
  size_t src_off = 0;
  for (int run = 0; run < c->runs; ++run) {
    // this run's sources (the device list holds the runs in order)
    AdvanceArgs A = A0;
    const size_t ns_run = c->src_of_run[run].size();
    if (ns_run > 0) {
      A.sa.n = (int)ns_run;
      A.sa.run += src_off;
      A.sa.elem += src_off;
      A.sa.kind += src_off;
      A.sa.par += 2 * src_off;
      A.sa.moment += 6 * src_off;
      A.sa.phi += (size_t)c->B * src_off;
      A.sa.inv_det += src_off;
    } else {
      A.sa.n = 0;
    }
    src_off += ns_run;
    for (DevBuf* b : {&c->aLe, &c->aLa, &c->aseis}) HIPCHK(c, hipMemsetAsync(b->p, 0, b->bytes, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (dj_q) {
      const double* q = dj_q + run * nqb;
      if (dev) {   // the DOF layout conversion runs on the host: stage through host memory
        std::vector<double> h(nqb);
        HIPCHK(c, hipMemcpy(h.data(), q, nqb * sizeof(double), hipMemcpyDeviceToHost));
        if ((rc = set_dofs_to<R>(c, c->aLe.p, c->aLa.p, h.data()))) return rc;
      } else if ((rc = set_dofs_to<R>(c, c->aLe.p, c->aLa.p, q))) {
        return rc;
      }
    }
    if (dj_seis && c->n_rec > 0) {
      const double* sb = dj_seis + run * nsb;
      if (dev) {
        HIPCHK(c, hipMemcpyAsync(c->aseis.p, sb, nsb * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
      } else {
        HIPCHK(c, hipMemcpy(c->aseis.p, sb, nsb * sizeof(double), hipMemcpyHostToDevice));
      }
    }
    for (size_t si = nck; si-- > 0;) {
      const int64_t L0 = c->ckpts[si].first;
      const int64_t J = (si + 1 < nck ? c->ckpts[si + 1].first : L_end) - L0;
      if (J <= 0) continue;
      const long long clock0 = (long long)L0;
      HIPCHK(c, hipMemcpyAsync(c->dclock.p, &clock0, sizeof clock0, hipMemcpyHostToDevice, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      LevelArgs a = base_args(c);
      a.run0 = 0;
      if (!(c->hist_valid && c->hist_L0 == L0 && c->hist_J == J && c->hist_run == run)) {
        // restore this run's state at the segment's start (checkpoints hold
        // the elastic rows of all runs, then their memory variables) and
        // replay the segment forward, keeping the state at the start of
        // every level's predictions
        c->hist_valid = false;
        const char* ck = (const char*)c->ckpts[si].second.p;
        HIPCHK(c, hipMemcpyAsync(rep_state, ck + run * we * rs, we * rs, hipMemcpyDeviceToDevice, c->stream));
        if (wa)
          HIPCHK(c, hipMemcpyAsync(rep_state + we * rs, ck + (c->runs * we + run * wa) * rs, wa * rs,
                                   hipMemcpyDeviceToDevice, c->stream));
        if ((rc = run_recorded_levels(c, A, p, J, false))) return rc;
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->hist_L0 = L0;
        c->hist_J = J;
        c->hist_run = run;
        c->hist_valid = true;
      }
      if (graph) {
        // the backward levels of a segment depend on its length only (the
        // record is addressed from the segment start, the clock is device
        // memory): captured once per length, replayed for every segment and run
        size_t gi = 0;
        while (gi < graphs.size() && graphs[gi].J != J) ++gi;
        if (gi == graphs.size()) {
          graphs.push_back({J, nullptr, nullptr});
          HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
          rc = backward(a, J);
          const hipError_t e = hipStreamEndCapture(c->stream, &graphs[gi].g);
          if (rc) return rc;
          if (e != hipSuccess) return fail(c, EDG_EHIP, std::string("adjoint graph capture: ") + hipGetErrorString(e));
          HIPCHK(c, hipGraphInstantiate(&graphs[gi].x, graphs[gi].g, nullptr, nullptr, 0));
        }
        HIPCHK(c, hipGraphLaunch(graphs[gi].x, c->stream));
      } else if ((rc = backward(a, J))) {
        return rc;
      }
      HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    if (g_q0) {
      double* out = g_q0 + run * nqb;
      if (dev) {
        std::vector<double> h(nqb);
        if ((rc = get_dofs_from<R>(c, c->aLe.p, c->aLa.p, h.data()))) return rc;
        HIPCHK(c, hipMemcpy(out, h.data(), nqb * sizeof(double), hipMemcpyHostToDevice));
      } else if ((rc = get_dofs_from<R>(c, c->aLe.p, c->aLa.p, out))) {
        return rc;
      }
    }
  }
  if (g_rho || g_vp || g_vs) {
    // chain rule on the device (gathers over face neighbours), then reorder
    // (the material table is uploaded once per material / cluster upload)
    if (!c->amat_valid) {
      if ((rc = ensure_host_materials(c))) return rc;
      const int mw = 3 + 2 * c->M;
      std::vector<double> mat((size_t)c->Kp * mw, 0.0);
      for (int64_t k = 0; k < c->K; ++k) {
        double* m = &mat[(size_t)c->user_to_internal[k] * mw];
        m[0] = c->rho[k];
        m[1] = c->vp[k];
        m[2] = c->vs[k];
        for (int l = 0; l < c->M; ++l) {
          m[3 + 2 * l] = c->yp[k * c->M + l];
          m[4 + 2 * l] = c->ys[k * c->M + l];
        }
      }
      if ((rc = dev_reserve(c, c->amat, mat.size() * sizeof(double)))) return rc;
      HIPCHK(c, hipMemcpy(c->amat.p, mat.data(), mat.size() * sizeof(double), hipMemcpyHostToDevice));
      c->amat_valid = true;
    }
    if ((rc = dev_reserve(c, c->agrad, (size_t)c->Kp * 3 * sizeof(double)))) return rc;
    if ((rc = chk(launch_material_gradient((const double*)c->agacc.p, (const int*)c->FI.p, (const double*)c->amat.p,
                                           c->M, c->Kp, (double*)c->agrad.p, c->stream),
                  "material gradient kernel")))
      return rc;
    if (dev) {
      if ((rc = chk(launch_scatter_gradient((const double*)c->agrad.p, (const long long*)c->d_i2u.p, c->Kp, g_rho,
                                            g_vp, g_vs, c->stream),
                    "gradient scatter kernel")))
        return rc;
      HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
      std::vector<double> gi((size_t)c->Kp * 3);
      HIPCHK(c, hipMemcpyAsync(gi.data(), c->agrad.p, gi.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipStreamSynchronize(c->stream));
      for (int64_t k = 0; k < c->K; ++k) {
        const double* x = &gi[(size_t)c->user_to_internal[k] * 3];
        if (g_rho) g_rho[k] = x[0];
        if (g_vp) g_vp[k] = x[1];
        if (g_vs) g_vs[k] = x[2];
      }
    }
  }
  const long long clock_end = (long long)L_end;
  HIPCHK(c, hipMemcpy(c->dclock.p, &clock_end, sizeof clock_end, hipMemcpyHostToDevice));
  c->adj_clean = true;
  return EDG_OK;
}

typedef int (*AdjFn)(edg_ctx*, const double*, const double*, double*, double*, double*, double*, bool);

AdjFn pick_adjoint(int fp64, int O, int M) {
  AdjFn f = nullptr;
#define EDG_PICK_ADJ(R, OO, MM) \
  if ((std::is_same<R, double>::value == (fp64 != 0)) && O == OO && M == MM) f = &adjoint_sweep<R, OO, MM>;
  EDG_FOR_EACH_VARIANT(EDG_PICK_ADJ)
#undef EDG_PICK_ADJ
  return f;
}

}  // namespace

extern "C" {

int edg_adjoint(edg_ctx* c, const double* dj_dseis, const double* dj_dq, double* g_q0, double* g_rho, double* g_vp,
                double* g_vs, int32_t on_device) {
  if (!c) return EDG_EINVAL;
  if (on_device != 0 && on_device != 1) return fail(c, EDG_EINVAL, "on_device must be 0 or 1");
  if (!c->have_clusters) return fail(c, EDG_ESTATE, "upload clusters first");
  if (c->ckpt_every <= 0 || c->ckpts.empty())
    return fail(c, EDG_ESTATE, "no checkpoints: enable checkpointing before the forward advance");
  if (c->ckpts.back().first > c->level) return fail(c, EDG_ESTATE, "checkpoints are ahead of the current time");
  HIPCHK(c, hipSetDevice(c->cfg.device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  AdjFn f = pick_adjoint(c->cfg.fp64, c->O, c->M);
  if (!f) return fail(c, EDG_EINVAL, "no adjoint kernel for this order / mechanism count");
  return f(c, dj_dseis, dj_dq, g_q0, g_rho, g_vp, g_vs, on_device != 0);
}

double edg_time(const edg_ctx* c) { return c ? (double)c->level * c->dt_cl[0] : 0.0; }

const char* edg_last_error(const edg_ctx* c) { return c ? c->err.c_str() : "null context"; }

int edg_enable_timing(edg_ctx* c, int32_t enable) {
  if (!c) return EDG_EINVAL;
  c->timing = enable != 0;
  if (c->timing) {
    c->t_launches = 0;
    c->t_updates = 0;
    c->t_ms = 0;
  }
  return EDG_OK;
}

int edg_kernel_stats(const edg_ctx* c, int64_t* launches, double* total_ms, int64_t* upd) {
  if (!c) return EDG_EINVAL;
  if (launches) *launches = c->t_launches;
  if (total_ms) *total_ms = c->t_ms;
  if (upd) *upd = c->t_updates;
  return EDG_OK;
}

int64_t edg_element_updates(const edg_ctx* c) { return c ? c->updates : 0; }

void edg_destroy(edg_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->cfg.device);
  delete c;
}

int edg_reference_matrices(int32_t order, double* K, double* Ft) {
  if (order < 1 || order > 8 || !K || !Ft) return EDG_EINVAL;
  RefMats R = reference_matrices(order);
  std::copy(R.K.begin(), R.K.end(), K);
  std::copy(R.Ft.begin(), R.Ft.end(), Ft);
  return EDG_OK;
}

int edg_cluster_host(int64_t K, const double* dt, const int64_t* nbr, int32_t Nc, double lam_in, int32_t* cluster,
                     double* lam_out, double* speedup_out) {
  if (K <= 0 || !dt || !nbr || !cluster || Nc < 1 || Nc > MAX_CLUSTERS || lam_in > 1.0) return EDG_EINVAL;
  std::vector<int> cl;
  double lam = 1.0, sp = 1.0;
  cluster_all(K, dt, nbr, Nc, lam_in, cl, lam, sp);
  for (int64_t k = 0; k < K; ++k) cluster[k] = cl[k] + 1;
  if (lam_out) *lam_out = lam;
  if (speedup_out) *speedup_out = sp;
  return EDG_OK;
}

}  // extern "C"
