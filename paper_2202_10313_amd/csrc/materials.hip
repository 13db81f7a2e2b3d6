// Device-side material tables: the range check and the material words of the
// per-element parameter table for materials given in device memory
// (edg_upload_materials with on_device = 1), and the scatter of the material
// gradient to the caller's element order (edg_adjoint with on_device = 1).
// The words are the same FP64 expressions as the host's table builder,
// evaluated without contraction into fused multiply-adds, so both routes
// give the same table bit for bit.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace edg {

namespace {

__global__ void k_check_materials(MatIn m, long long K, unsigned* bad) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double rho = m.rho[k], vp = m.vp[k], vs = m.vs[k];
  if (!(rho > 0) || !(vs > 0) || !(vp > sqrt(4.0 / 3.0) * vs)) atomicAdd(bad, 1u);
}

template <class R>
__global__ void k_pack_materials(MatIn m, int M, long long Kp, const long long* i2u, const long long* nbr, R* P,
                                 double* amat) {
#pragma clang fp contract(off)
  const long long ki = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (ki >= Kp) return;
  const long long k = i2u[ki];
  const int mw = 3 + 2 * M;
  double* am = amat + ki * mw;
  if (k < 0) {   // padding slot: zero parameters (left as packed), zero material row
    for (int j = 0; j < mw; ++j) am[j] = 0.0;
    return;
  }
  R* p = P + ki * NPARAM;
  const double rho = m.rho[k], vp = m.vp[k], vs = m.vs[k];
  const double mu = rho * vs * vs, lam = rho * vp * vp - 2.0 * mu;
  p[9] = R(1.0 / rho);
  p[10] = R(lam);
  p[11] = R(mu);
  p[12] = R(rho * vp);
  p[13] = R(rho * vs);
  am[0] = rho;
  am[1] = vp;
  am[2] = vs;
  for (int l = 0; l < M; ++l) {
    const double ypl = m.yp[k * M + l], ysl = m.ys[k * M + l];
    p[14 + 2 * l] = R((lam + 2.0 * mu) * ypl - 2.0 * mu * ysl);
    p[15 + 2 * l] = R(2.0 * mu * ysl);
    am[3 + 2 * l] = ypl;
    am[4 + 2 * l] = ysl;
  }
  for (int i = 0; i < 4; ++i) {
    R* f = p + 20 + 6 * i;
    const long long n = nbr[k * 4 + i];
    if (n >= 0) {
      f[4] = R(m.rho[n] * m.vp[n]);
      f[5] = R(m.rho[n] * m.vs[n]);
    } else {
      f[4] = R(rho * vp);
      f[5] = R(rho * vs);
    }
  }
}

__global__ void k_scatter_gradient(const double* g, const long long* i2u, long long Kp, double* g_rho, double* g_vp,
                                   double* g_vs) {
  const long long ki = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (ki >= Kp) return;
  const long long k = i2u[ki];
  if (k < 0) return;
  if (g_rho) g_rho[k] = g[ki * 3 + 0];
  if (g_vp) g_vp[k] = g[ki * 3 + 1];
  if (g_vs) g_vs[k] = g[ki * 3 + 2];
}

unsigned blocks_of(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int launch_check_materials(const MatIn& m, long long K, unsigned* bad, hipStream_t st) {
  if (K <= 0) return 0;
  hipLaunchKernelGGL(k_check_materials, dim3(blocks_of(K)), dim3(256), 0, st, m, K, bad);
  return (int)hipGetLastError();
}

template <class R>
int launch_pack_materials(const MatIn& m, int M, long long Kp, const long long* i2u, const long long* nbr, R* P,
                          double* amat, hipStream_t st) {
  if (Kp <= 0) return 0;
  hipLaunchKernelGGL((k_pack_materials<R>), dim3(blocks_of(Kp)), dim3(256), 0, st, m, M, Kp, i2u, nbr, P, amat);
  return (int)hipGetLastError();
}
template int launch_pack_materials<float>(const MatIn&, int, long long, const long long*, const long long*, float*,
                                          double*, hipStream_t);
template int launch_pack_materials<double>(const MatIn&, int, long long, const long long*, const long long*, double*,
                                           double*, hipStream_t);

int launch_scatter_gradient(const double* g, const long long* i2u, long long Kp, double* g_rho, double* g_vp,
                            double* g_vs, hipStream_t st) {
  if (Kp <= 0) return 0;
  hipLaunchKernelGGL(k_scatter_gradient, dim3(blocks_of(Kp)), dim3(256), 0, st, g, i2u, Kp, g_rho, g_vp, g_vs);
  return (int)hipGetLastError();
}

}  // namespace edg
