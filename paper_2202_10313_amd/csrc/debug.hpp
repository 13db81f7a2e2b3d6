// Debug aids of the LTS buffer schedule (internal; see debug.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

#include "kernels.hpp"

namespace edg {

// NaN into every trace slot whose last legal read was at the level of `a`
// (runs a.run0 .. a.run0 + runs - 1; FP: padded face-basis size).  early = 1:
// instead the B1 slot that level's prediction wrote (a self-test of the
// detector: a later read of it must produce NaNs).
template <class R>
int launch_poison_traces(const KPtrs& p, const LevelArgs& a, int runs, int FP, int early, hipStream_t st);
// NaN into `words` 32-bit words at p (a fill kernel: no memset node in a capture)
int launch_poison_words(void* p, size_t words, hipStream_t st);
// out[0] += non-finite words among q [n] (R = float or double); out[1] =
// min(out[1], the smallest such index).  out starts as {0, ~0}.
template <class R>
int launch_count_nonfinite(const void* q, long long n, unsigned long long* out, hipStream_t st);

}  // namespace edg
