// In-register line FFTs shared by the FFT kernels and the stage kernels.
// A line of length P = 4M whose inputs vanish from 2M on is split over four
// adjacent lanes by the residue r of its frequency index (see k_fft_yzr);
// reg_dft is an unrolled radix-2 DIF DFT of a register array (natural order
// in, bit-reversed out), quad_inverse the 4-point inverse DFT across the
// residue lanes with DPP quad permutations.
#pragma once
#include <hip/hip_runtime.h>
#include "kernels_common.h"
#include "fft_lds.h"

namespace mmk {

__host__ __device__ constexpr int brevc(int p, int lg) {
  int r = 0;
  for (int b = 0; b < lg; ++b) r |= ((p >> b) & 1) << (lg - 1 - b);
  return r;
}
__host__ __device__ constexpr int ilog2c(int m) { return m <= 1 ? 0 : 1 + ilog2c(m >> 1); }

// cos(2 pi j / 16)
__device__ __forceinline__ constexpr float cos16(int j) {
  j &= 15;
  switch (j) {
    case 0: return 1.0f;
    case 1: case 15: return 0.92387953251128674f;
    case 2: case 14: return 0.70710678118654752f;
    case 3: case 13: return 0.38268343236508977f;
    case 4: case 12: return 0.0f;
    case 5: case 11: return -0.38268343236508977f;
    case 6: case 10: return -0.70710678118654752f;
    case 7: case 9: return -0.92387953251128674f;
    default: return -1.0f;
  }
}

// d * W_M^{k} (forward, W_M = e^{-2 pi i / M}) or d * W_M^{-k} (inverse), 0 <= k < M/2, M <= 16
template <int M, bool INV>
__device__ __forceinline__ float2 twc(float2 d, int k) {
  if (k == 0) return d;
  const int j = k * (16 / M);
  if (j == 4) return rot<INV>(d);
  const float c = cos16(j), sn = INV ? cos16(j - 4) : -cos16(j - 4);
  return make_float2(d.x * c - d.y * sn, d.x * sn + d.y * c);
}
// d * W_M^{+-k} for M = 32 (angles on the 32-point circle)
template <bool INV>
__device__ __forceinline__ float2 twc32(float2 d, int k, const float2* tw32) {
  if ((k & 1) == 0) return twc<16, INV>(d, k >> 1);
  const float2 w = tw32[k];
  const float sn = INV ? -w.y : w.y;
  return make_float2(d.x * w.x - d.y * sn, d.x * sn + d.y * w.x);
}

// In-register radix-2 DIF DFT of length M: natural order in, bit-reversed out.
template <int M, bool INV>
__device__ __forceinline__ void reg_dft(float2 (&v)[M], const float2* tw32) {
#pragma unroll
  for (int h = M / 2; h >= 1; h >>= 1) {
#pragma unroll
    for (int g = 0; g < M; g += 2 * h) {
#pragma unroll
      for (int i = 0; i < h; ++i) {
        const float2 a = v[g + i], b = v[g + i + h];
        v[g + i] = cadd(a, b);
        const float2 d = csub(a, b);
        const int k = i * (M / (2 * h));
        if constexpr (M <= 16) v[g + i + h] = twc<M, INV>(d, k);
        else v[g + i + h] = twc32<INV>(d, k, tw32);
      }
    }
  }
}

// quad_perm lane exchange: XOR 1 and XOR 2 within each group of four lanes
__device__ __forceinline__ float dpp_x1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_x2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
}
__device__ __forceinline__ float2 quad_x1(float2 v) { return make_float2(dpp_x1(v.x), dpp_x1(v.y)); }
__device__ __forceinline__ float2 quad_x2(float2 v) { return make_float2(dpp_x2(v.x), dpp_x2(v.y)); }

// Inverse 4-point DFT across the residue lanes r of a quad, keeping the
// outputs jj = 0, 1: lane r returns h[y0 + M (r & 1)] for y0 = i + (M/2)(r >> 1),
// i < M/2, where h[y0 + M jj] = sum_r i^{r jj} w_r[y0].
template <int M>
__device__ __forceinline__ void quad_inverse(const float2 (&w)[M], int r, float2 (&out)[M / 2]) {
  const bool hi = r & 2, odd = r & 1;
#pragma unroll
  for (int i = 0; i < M / 2; ++i) {
    const float2 mine = hi ? w[i + M / 2] : w[i];
    const float2 recv = quad_x2(hi ? w[i] : w[i + M / 2]);
    const float2 sm = cadd(mine, recv);
    const float2 df = hi ? csub(recv, mine) : csub(mine, recv);
    const float2 got = quad_x1(odd ? sm : df);
    out[i] = odd ? cadd(got, rot<true>(df)) : cadd(sm, got);
  }
}

// LDS element or zero: the (always in-bounds) load is unconditional and the
// zero is selected afterwards, so no branch splits the batch of loads
__device__ __forceinline__ float2 lds_or0(const float2* p, bool in) {
  const float2 v = *p;
  return make_float2(in ? v.x : 0.f, in ? v.y : 0.f);
}

// fold for residue r: f[j] = W_P^{rj} (x0 + (-i)^r x1)
__device__ __forceinline__ float2 fold(float2 x0, float2 x1, int r, float2 w) {
  if (r & 1) x1 = make_float2(x1.y, -x1.x);
  if (r & 2) x1 = make_float2(-x1.x, -x1.y);
  return cmul(cadd(x0, x1), w);
}

}  // namespace mmk
