// Per-kernel event timing used by the benchmark (see helm_kprof_* in helm.h).
#pragma once

#include <hip/hip_runtime.h>

namespace helm {

enum { KP_STENCIL = 0, KP_MULTIDOT = 1, KP_MULTIAXPY = 2, KP_QT = 3, KP_SKINNY = 4, KP_CGS = 5, KP_MFMA = 6,
       KP_COUNT = 7 };

bool kprof_on();
void kprof_begin(int kind, hipStream_t st);
// bytes: the launch's algorithmic bytes (KP_MFMA: its algorithmic flops)
void kprof_end(int kind, double bytes, hipStream_t st);

}  // namespace helm
