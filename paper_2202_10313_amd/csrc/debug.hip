// Debug aids for the LTS buffer schedule (not on the production path):
//  * NaN poisoning of the B1 / B2 / B3 face traces (Sec. V-B (Buffers and
//    Algorithm): every buffer is consumed by the steps that read it and then
//    rewritten).  After the launch of finest level G each trace slot whose
//    last legal read happened at G is overwritten with NaN, so a read of a
//    stale slot in a later launch turns the DOFs it touches into NaN;
//  * a count of the non-finite DOF words (the check that turns such NaNs, or
//    an unstable run, into an error).
//
// Which slots die at level G.  Element e of cluster l finishes its step n at
// the level (n+1) 2^l, the launch where it also writes the traces of step
// n+1 into the other parity slot:
//  * its B1 of step n (T1[n & 1]) is read at that level only: by e, by its
//    same-cluster neighbours finishing step n and by its finer neighbours
//    finishing their step 2n+1 (as B1 - B2);
//  * its B2 of step n (T2[n & 1]) is read by the finer neighbours finishing
//    their steps 2n and 2n+1, the last of them at that level;
//  * its B3 (T3[k & 1], accumulated over its steps 2k and 2k+1) is read by
//    the coarser neighbour finishing its step k, at the level where e
//    finishes step 2k+1 (odd n only).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "device_common.hpp"
#include "debug.hpp"

namespace edg {

namespace {

// all-ones words: a NaN as FP32 and (in pairs) as FP64
constexpr uint32_t NAN_WORD = 0xFFFFFFFFu;

template <class R>
__global__ __launch_bounds__(256) void k_poison_traces(KPtrs p, LevelArgs a, long long ts, int early) {
  const int run = a.run0 + (int)blockIdx.y;
  select_run<R>(p, run);
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)a.end * ts) return;
  const int e = (int)(idx / ts);
  const long long w = idx % ts;
  const int nfin = step_fin_of(a, cluster_of(a, e));
  const R nan = __builtin_bit_cast(R, ~(typename std::conditional<sizeof(R) == 4, uint32_t, uint64_t>::type)0);
  R* T1 = reinterpret_cast<R*>(p.T1);
  R* T2 = reinterpret_cast<R*>(p.T2);
  R* T3 = reinterpret_cast<R*>(p.T3);
  const int* FI = p.FI + (size_t)e * FI_WORDS;
  if (early) {
    // detector self-test: the slot written by this level's prediction, which
    // a later level still has to read
    T1[((size_t)((nfin + 1) & 1) * p.Kp + e) * ts + w] = nan;
    return;
  }
  T1[((size_t)(nfin & 1) * p.Kp + e) * ts + w] = nan;
  if (FI[13] >= 0) T2[((size_t)(nfin & 1) * p.N2 + FI[13]) * ts + w] = nan;
  if (FI[14] >= 0 && (nfin & 1)) T3[((size_t)((nfin >> 1) & 1) * p.N3 + FI[14]) * ts + w] = nan;
}

__global__ __launch_bounds__(256) void k_fill_words(uint32_t* p, size_t words, uint32_t v) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = v;
}

// out[0] += non-finite words of q [n]; out[1] = min(out[1], their smallest index)
template <class R>
__global__ __launch_bounds__(256) void k_count_nonfinite(const R* q, long long n, unsigned long long* out) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  unsigned long long cnt = 0, first = ~0ull;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (!__builtin_isfinite(q[i])) {
      ++cnt;
      if ((unsigned long long)i < first) first = (unsigned long long)i;
    }
  }
  if (cnt) {
    atomicAdd(&out[0], cnt);
    atomicMin(&out[1], first);
  }
}

}  // namespace

template <class R>
int launch_poison_traces(const KPtrs& p, const LevelArgs& a, int runs, int FP, int early, hipStream_t st) {
  const long long ts = 4LL * LPE * FP;
  const long long total = (long long)a.end * ts;
  if (total <= 0 || runs <= 0) return 0;
  hipLaunchKernelGGL((k_poison_traces<R>), dim3((unsigned)((total + 255) / 256), runs), dim3(256), 0, st, p, a, ts,
                     early);
  return (int)hipGetLastError();
}

int launch_poison_words(void* p, size_t words, hipStream_t st) {
  if (words == 0) return 0;
  const size_t blocks = (words + 255) / 256 < 4096 ? (words + 255) / 256 : 4096;
  hipLaunchKernelGGL(k_fill_words, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t*)p, words, NAN_WORD);
  return (int)hipGetLastError();
}

template <class R>
int launch_count_nonfinite(const void* q, long long n, unsigned long long* out, hipStream_t st) {
  if (n <= 0) return 0;
  const long long blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
  hipLaunchKernelGGL((k_count_nonfinite<R>), dim3((unsigned)blocks), dim3(256), 0, st, (const R*)q, n, out);
  return (int)hipGetLastError();
}

template int launch_poison_traces<float>(const KPtrs&, const LevelArgs&, int, int, int, hipStream_t);
template int launch_poison_traces<double>(const KPtrs&, const LevelArgs&, int, int, int, hipStream_t);
template int launch_count_nonfinite<float>(const void*, long long, unsigned long long*, hipStream_t);
template int launch_count_nonfinite<double>(const void*, long long, unsigned long long*, hipStream_t);

}  // namespace edg
