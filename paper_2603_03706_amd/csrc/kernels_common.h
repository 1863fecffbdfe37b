// Small device helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "mm_internal.h"

namespace mmk {

// Stage input m = p0 + c1 * p1 (p1 optional), component-major per instance.
struct Src {
  const float* p0;
  const float* p1;
  float c1;
  __device__ __forceinline__ float ld(int idx) const {
    float v = p0[idx];
    if (p1) v = fmaf(c1, p1[idx], v);
    return v;
  }
};

// Where the input of stage `stage` lives.  RK4: 0/1 state, 2 and 4 buffer
// A, 3 buffer B.  DP45: 1 state, 2 state + h a21 k1 (not stored), 3 and 5
// buffer A, 4 and 6 buffer B, 7 the normalised candidate.
__device__ __forceinline__ Src stage_src(const InstDesc& D, const InstCtl* C, int method, int stage) {
  Src s;
  s.p1 = nullptr;
  s.c1 = 0.f;
  const int cur = C->cur;
  if (method == MMI_RK4) {
    s.p0 = (stage <= 1) ? D.y[cur] : (stage == 3 ? D.st[1] : D.st[0]);
  } else {
    switch (stage) {
      case 1: s.p0 = D.y[cur]; break;
      case 2:
        s.p0 = D.y[cur];
        s.p1 = D.k[C->slot[0]];
        s.c1 = (float)(C->h * DPCoef::a21);
        break;
      case 3: case 5: s.p0 = D.st[0]; break;
      case 4: case 6: s.p0 = D.st[1]; break;
      default: s.p0 = D.y[1 - cur]; break;
    }
  }
  return s;
}

// max that propagates NaN (a NaN anywhere makes the result NaN)
__device__ __forceinline__ double nan_max(double a, double b) {
  return (a != a || b != b) ? (a + b) : fmax(a, b);
}

// wave64 butterfly sum; every lane ends with the same value, the order of
// additions is fixed, so the result is deterministic
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = nan_max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

}  // namespace mmk
