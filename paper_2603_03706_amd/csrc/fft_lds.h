// Line FFTs on LDS shared by the FFT kernels and the stage kernels (which do
// the x passes of the demag convolution for their own rows).  Forward
// transforms run in place by decimation in frequency (natural order in,
// bit-reversed out), inverse ones by decimation in time (bit-reversed in,
// natural out), in radix-2^2 passes; twiddles W_L^m = e^{-2 pi i m / L} come
// from a table in LDS.
#pragma once
#include <hip/hip_runtime.h>
#include "kernels_common.h"

namespace mmk {

// Bit reversal of the low lg bits.
__device__ __forceinline__ int brev(int p, int lg) {
  return lg ? (int)(__brev((unsigned)p) >> (32 - lg)) : 0;
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
template <bool INV>
__device__ __forceinline__ float2 twid(const float2* twl, int m) {
  float2 w = twl[m];
  if (INV) w.y = -w.y;
  return w;
}

__device__ __forceinline__ int ilog2(int L) {
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  return lg;
}

// In-place radix-2^2 butterflies shared by the line FFTs below.
// DIF (forward): elements p0, p0+e1, p0+e2, p0+e2+e1 with e1 = q, e2 = h = 2q.
__device__ __forceinline__ void dif4(float2* lds, int p0, int e1, int e2, float2 w1, float2 w2) {
  const float2 x0 = lds[p0], x1 = lds[p0 + e1], x2 = lds[p0 + e2], x3 = lds[p0 + e2 + e1];
  const float2 a0 = cadd(x0, x2), a1 = cadd(x1, x3);
  const float2 a2 = cmul(csub(x0, x2), w1);
  const float2 a3 = rot<false>(cmul(csub(x1, x3), w1));
  lds[p0] = cadd(a0, a1);
  lds[p0 + e1] = cmul(csub(a0, a1), w2);
  lds[p0 + e2] = cadd(a2, a3);
  lds[p0 + e2 + e1] = cmul(csub(a2, a3), w2);
}
// DIT (inverse): elements p0 + k e1, k = 0..3, conjugate twiddles wA, wB given.
__device__ __forceinline__ void dit4(float2* lds, int p0, int e1, float2 wA, float2 wB) {
  const float2 x0 = lds[p0], x1 = lds[p0 + e1], x2 = lds[p0 + 2 * e1], x3 = lds[p0 + 3 * e1];
  const float2 t1 = cmul(x1, wA), t3 = cmul(x3, wA);
  const float2 a0 = cadd(x0, t1), a1 = csub(x0, t1), a2 = cadd(x2, t3), a3 = csub(x2, t3);
  const float2 u = cmul(a2, wB), v = rot<true>(cmul(a3, wB));
  lds[p0] = cadd(a0, u);
  lds[p0 + 2 * e1] = csub(a0, u);
  lds[p0 + e1] = cadd(a1, v);
  lds[p0 + 3 * e1] = csub(a1, v);
}
__device__ __forceinline__ void bf2(float2* lds, int p, int e) {
  const float2 a = lds[p], b = lds[p + e];
  lds[p] = cadd(a, b);
  lds[p + e] = csub(a, b);
}

// Lines along a contiguous axis (element stride 1), line bases in tab[].
// Consecutive threads take consecutive butterflies of a line.
template <int T, bool DIT>
__device__ void fft_rows(float2* lds, int L, int lg, int NL, const int* tab, const float2* twl) {
  if (lg == 0) return;
  if (!DIT) {
    int s = 0;
    for (; s + 2 <= lg; s += 2) {
      const int h = L >> (s + 1), q = h >> 1, lq = lg - s - 2, lgQ = lg - 2;
      const int NB = NL << lgQ;
      for (int idx = threadIdx.x; idx < NB; idx += T) {
        const int r = idx & ((1 << lgQ) - 1), l = idx >> lgQ;
        const int g = r >> lq, i = r & (q - 1);
        dif4(lds, tab[l] + g * 2 * h + i, q, h, twl[i << s], twl[i << (s + 1)]);
      }
      __syncthreads();
    }
    if (s < lg) {
      const int NB = NL << (lg - 1);
      for (int idx = threadIdx.x; idx < NB; idx += T) {
        const int m = idx & ((1 << (lg - 1)) - 1), l = idx >> (lg - 1);
        bf2(lds, tab[l] + 2 * m, 1);
      }
      __syncthreads();
    }
  } else {
    int t = 0;
    if (lg & 1) {
      const int NB = NL << (lg - 1);
      for (int idx = threadIdx.x; idx < NB; idx += T) {
        const int m = idx & ((1 << (lg - 1)) - 1), l = idx >> (lg - 1);
        bf2(lds, tab[l] + 2 * m, 1);
      }
      __syncthreads();
      t = 1;
    }
    for (; t + 2 <= lg; t += 2) {
      const int q = 1 << t, lgQ = lg - 2;
      const int NB = NL << lgQ;
      for (int idx = threadIdx.x; idx < NB; idx += T) {
        const int r = idx & ((1 << lgQ) - 1), l = idx >> lgQ;
        const int g = r >> t, i = r & (q - 1);
        dit4(lds, tab[l] + g * 4 * q + i, q, twid<true>(twl, i << (lg - t - 1)),
             twid<true>(twl, i << (lg - t - 2)));
      }
      __syncthreads();
    }
  }
}

// Lines along a strided axis: line (c, j) of NC groups of 2^lgJ adjacent
// lines, element stride es, group stride cs.  Consecutive threads take
// adjacent lines.
template <int T, bool DIT>
__device__ void fft_cols(float2* lds, int L, int lg, int NC, int lgJ, int cs, int es, const float2* twl,
                         int s0 = 0, int tmax = -1) {
  if (lg == 0) return;
  const int J = 1 << lgJ;
  if (!DIT) {
    // DIF stages s0 .. lg-1 (stage s has span L >> (s + 1))
    int s = s0;
    for (; s + 2 <= lg; s += 2) {
      const int h = L >> (s + 1), q = h >> 1, lq = lg - s - 2, lgQ = lg - 2;
      const int NB = (NC << lgQ) << lgJ;
      for (int idx = threadIdx.x; idx < NB; idx += T) {
        const int j = idx & (J - 1), rest = idx >> lgJ;
        const int r = rest & ((1 << lgQ) - 1), c = rest >> lgQ;
        const int g = r >> lq, i = r & (q - 1);
        dif4(lds, c * cs + j + (g * 2 * h + i) * es, q * es, h * es, twl[i << s], twl[i << (s + 1)]);
      }
      __syncthreads();
    }
    if (s < lg) {
      const int NB = (NC << (lg - 1)) << lgJ;
      for (int idx = threadIdx.x; idx < NB; idx += T) {
        const int j = idx & (J - 1), rest = idx >> lgJ;
        const int m = rest & ((1 << (lg - 1)) - 1), c = rest >> (lg - 1);
        bf2(lds, c * cs + j + 2 * m * es, es);
      }
      __syncthreads();
    }
  } else {
    // DIT stages 0 .. tmax-1 (stage t has span 1 << t)
    if (tmax < 0) tmax = lg;
    int t = 0;
    if (tmax & 1) {
      const int NB = (NC << (lg - 1)) << lgJ;
      for (int idx = threadIdx.x; idx < NB; idx += T) {
        const int j = idx & (J - 1), rest = idx >> lgJ;
        const int m = rest & ((1 << (lg - 1)) - 1), c = rest >> (lg - 1);
        bf2(lds, c * cs + j + 2 * m * es, es);
      }
      __syncthreads();
      t = 1;
    }
    for (; t + 2 <= tmax; t += 2) {
      const int q = 1 << t, lgQ = lg - 2;
      const int NB = (NC << lgQ) << lgJ;
      for (int idx = threadIdx.x; idx < NB; idx += T) {
        const int j = idx & (J - 1), rest = idx >> lgJ;
        const int r = rest & ((1 << lgQ) - 1), c = rest >> lgQ;
        const int g = r >> t, i = r & (q - 1);
        dit4(lds, c * cs + j + (g * 4 * q + i) * es, q * es, twid<true>(twl, i << (lg - t - 1)),
             twid<true>(twl, i << (lg - t - 2)));
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ void load_twiddles(float2* twl, int L, const float2* __restrict__ tw,
                                              int T) {
  for (int m = threadIdx.x; m < L; m += T) twl[m] = tw[m * (MMI_TW_LEN / L)];
}

}  // namespace mmk
