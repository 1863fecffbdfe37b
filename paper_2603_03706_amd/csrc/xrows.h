// x passes of the demag convolution done by a cell kernel for its own
// x-rows (the stage kernels, and the adjoint stage kernels for the field
// adjoint): C2R of the convolved X rows into a per-cell field, R2C of a
// per-cell vector into the X rows of the next convolution.
#pragma once
#include <hip/hip_runtime.h>
#include "mm_internal.h"
#include "kernels_common.h"
#include "fft_lds.h"

namespace mmk {

// With D.xfused (FFT demag, one sublattice, nx a power of two from 2 to MMI_WG/2),
// a workgroup of MMI_WG cells holds R = MMI_WG/nx whole x-rows of each component.  It
// transforms them itself: the C2R of the convolved X rows gives the demag
// field of its cells in LDS (no B_d round trip), and the R2C of the next
// stage input it computes writes the X rows of the next convolution (no
// separate x-forward pass).  Rows (c, 2j) and (c, 2j+1) share one complex
// line; lines are transformed by the LDS line FFTs in place.
struct XRows {
  int nx, lgnx, R, lgR, J, lgJ, Px, lgx, Kx, es, cs, nyz, rows, yz0, nrow;
  float2 *zb, *twl;
};

__device__ __forceinline__ XRows xrows_setup(const InstDesc& D, int lw, float2* lds) {
  XRows q;
  q.nx = D.nx;
  q.lgnx = ilog2(q.nx);
  q.lgR = MMI_LG_WG - q.lgnx;
  q.R = 1 << q.lgR;
  q.lgJ = q.lgR - 1;
  q.J = 1 << q.lgJ;
  q.Px = D.px;
  q.lgx = q.lgnx + 1;
  q.Kx = D.kx;
  q.es = q.J + 1;
  q.cs = q.Px * q.es;
  q.nyz = D.ny * D.nz;
  q.rows = 3 * q.nyz;
  q.yz0 = lw * q.R;
  q.nrow = min(q.R, q.nyz - q.yz0);     // rows of this workgroup (the last one may hold fewer)
  q.zb = lds;                            // [3][Px][J + 1] lines
  q.twl = lds + 3 * q.cs;                // [Px]
  return q;
}

// demag field [T] of this thread's cell from the convolved X rows
__device__ __forceinline__ void xrows_c2r(const InstDesc& D, const XRows& q, float (&bdv)[3]) {
  const MMG float2* X = gbl(D.fx);
  const int half = q.Px >> 1;
  // Item (k, c, j2), k <= Px/2: the X values a, b of rows 2 j2 and 2 j2 + 1
  // give line entries Z[k] = a + i b and, by Hermitian symmetry,
  // Z[Px - k] = conj(a) + i conj(b); both go to their bit-reversed slots.
  const int n = q.Kx * 3 * q.J;
  for (int e = threadIdx.x; e < n; e += MMI_WG) {
    const int j2 = e & (q.J - 1), rest = e >> q.lgJ;
    const int k = rest / 3, c = rest - 3 * k;
    const int j = 2 * j2;
    const int e0 = k * q.rows + c * q.nyz + q.yz0;
    float2 a = gld2(&gat(X, e0 + min(j, q.nrow - 1))), b = gld2(&gat(X, e0 + min(j + 1, q.nrow - 1)));
    if (j >= q.nrow) a = make_float2(0.f, 0.f);
    if (j + 1 >= q.nrow) b = make_float2(0.f, 0.f);
    const bool edge = k == 0 || k == half;
    if (edge) { a.y = 0.f; b.y = 0.f; }
    float2* line = q.zb + c * q.cs + j2;
    line[brev(k, q.lgx) * q.es] = make_float2(a.x - b.y, a.y + b.x);
    if (!edge) line[brev(q.Px - k, q.lgx) * q.es] = make_float2(a.x + b.y, b.x - a.y);
  }
  __syncthreads();
  fft_cols<MMI_WG, true>(q.zb, q.Px, q.lgx, 3, q.lgJ, q.cs, q.es, q.twl);
  const int j = threadIdx.x >> q.lgnx, x = threadIdx.x & (q.nx - 1);
  const float sc = D.bd_scale;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float2 z = q.zb[c * q.cs + x * q.es + (j >> 1)];
    bdv[c] = sc * ((j & 1) ? z.y : z.x);
  }
}

// X rows of the next stage input v (this thread's cell; zero for cells
// outside the grid).  `synced`: a workgroup barrier already separates the
// C2R's last reads of the lines from here.
__device__ __forceinline__ void xrows_r2c(const InstDesc& D, const XRows& q, const float (&v)[3], bool synced) {
  if (!synced) __syncthreads();
  {
    // line entries x < nx hold the cells; the padding x >= nx is never stored
    const int j = threadIdx.x >> q.lgnx, x = threadIdx.x & (q.nx - 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float* p = reinterpret_cast<float*>(q.zb + c * q.cs + x * q.es + (j >> 1));
      p[j & 1] = v[c];
    }
  }
  __syncthreads();
  {
    // first radix-2^2 DIF stage (span Px/2): its inputs x2, x3 are the zero
    // padding, so it reads only x0 = Z[i] and x1 = Z[i + Px/4] and is done
    // with the arithmetic of the full stage (zeros for x2, x3)
    const int qq = q.Px >> 2, lgq = q.lgx - 2;
    const float2 zero = make_float2(0.f, 0.f);
    for (int e = threadIdx.x; e < 3 * q.J * qq; e += MMI_WG) {
      const int j2 = e & (q.J - 1), rest = e >> q.lgJ;
      const int i = rest & (qq - 1), c = rest >> lgq;
      float2* line = q.zb + c * q.cs + j2;
      const float2 x0 = line[i * q.es], x1 = line[(i + qq) * q.es];
      const float2 w1 = q.twl[i], w2 = q.twl[2 * i];
      const float2 a0 = cadd(x0, zero), a1 = cadd(x1, zero);
      const float2 a2 = cmul(csub(x0, zero), w1);
      const float2 a3 = rot<false>(cmul(csub(x1, zero), w1));
      line[i * q.es] = cadd(a0, a1);
      line[(i + qq) * q.es] = cmul(csub(a0, a1), w2);
      line[(i + 2 * qq) * q.es] = cadd(a2, a3);
      line[(i + 3 * qq) * q.es] = cmul(csub(a2, a3), w2);
    }
  }
  __syncthreads();
  fft_cols<MMI_WG, false>(q.zb, q.Px, q.lgx, 3, q.lgJ, q.cs, q.es, q.twl, 2);
  MMG float2* X = gbl(D.fx);
  // Item (k, c, j2): Z[k] and Z[Px - k] of line j2 separate into the X values
  // of rows 2 j2 (even part) and 2 j2 + 1 (odd part).
  const int n = q.Kx * 3 * q.J;
  for (int e = threadIdx.x; e < n; e += MMI_WG) {
    const int j2 = e & (q.J - 1), rest = e >> q.lgJ;
    const int k = rest / 3, c = rest - 3 * k;
    const int j = 2 * j2;
    if (j >= q.nrow) continue;
    const float2* zc = q.zb + c * q.cs + j2;
    const float2 Z = zc[brev(k & (q.Px - 1), q.lgx) * q.es];
    const float2 Zm = zc[brev((q.Px - k) & (q.Px - 1), q.lgx) * q.es];
    MMG float2* row = &gat(X, k * q.rows + c * q.nyz + q.yz0 + j);
    gst2(row, make_float2(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y)));
    if (j + 1 < q.nrow) gst2(row + 1, make_float2(0.5f * (Z.y + Zm.y), -0.5f * (Z.x - Zm.x)));
  }
}

}  // namespace mmk
