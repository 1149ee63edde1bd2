// Host stand-in for <hip/hip_runtime.h>, for the sanitizer test only: with
// it the per-point device code of the library (geometry, physics and the
// primitive-variable recoveries) compiles as plain C++ on the host.  The
// function qualifiers become nothing and the hardware reciprocals become
// divisions (used only in the reconstruction and face code, which the test
// does not call).
#pragma once
#include <math.h>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline

static inline float host_rcpf(float x) { return 1.0f / x; }
static inline double host_rcp(double x) { return 1.0 / x; }
#define __builtin_amdgcn_rcpf(x) host_rcpf(x)
#define __builtin_amdgcn_rcp(x) host_rcp(x)
