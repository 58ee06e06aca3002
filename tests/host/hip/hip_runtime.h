// Host stand-in for <hip/hip_runtime.h>, used only by the CPU tests that
// compile the device headers (helas.h, helas_adj.h, rambo.h) with the host
// compiler:
// the function qualifiers become plain inline functions and the two gfx950
// builtins the headers use get their exact host meaning (no scheduling
// barrier; a correctly rounded reciprocal instead of the hardware estimate,
// which the Newton steps of recip() leave unchanged).
#pragma once
#include <cmath>
#include <cstdint>
#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
// launcher declarations name the stream type; nothing is launched on the host
typedef struct ihipStream_t* hipStream_t;
