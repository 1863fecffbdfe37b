// Demag field by zero-padded FFT convolution with the cell-averaged tensor.
//
// Per stage, for the stage input m (3 real components on nx*ny*nz cells):
//   x-forward : R2C along x (two real rows packed in one complex line),
//               zero padded to Px, output X[kx][c][z][y], kx <= Px/2
//   yz        : C2C along y (zero padded to Py), C2C along z (zero padded to
//               Pz), multiply by the real symmetric 3x3 kernel spectrum,
//               inverse z, inverse y, crop to z < nz, y < ny (in place on X).
//               One workgroup per (instance, kx) when the padded (y, z) plane
//               of all three components fits in LDS ("fused"), otherwise a
//               y pass into Y[kx][c][z][ky], a z pass with the multiply on
//               tiles of ky, and an inverse y pass back into X ("split").
//   x-inverse : C2R along x, crop to x < nx, scale by -mu0 Ms / (Px Py Pz),
//               output B_d[c][z][y][x] [T].
// Every line FFT runs in LDS with in-place radix-2^2 passes: forward
// transforms by decimation in frequency (bit-reversed output), inverse
// transforms by decimation in time (bit-reversed input), so no reordering
// pass is needed between them.
#include "mm_internal.h"
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

// 3x3 kernel multiply at (kx, ky, kz): H = N M (sign and scale applied later)
__device__ __forceinline__ void kernel_mul(const InstDesc& D, int kx, int ky, int kz, float2& mx,
                                           float2& my, float2& mz) {
  const int hy = D.py / 2, hz = D.pz / 2;
  int ky2 = ky, kz2 = kz;
  float sy = 1.f, sz = 1.f;
  if (ky > hy) { ky2 = D.py - ky; sy = -1.f; }
  if (kz > hz) { kz2 = D.pz - kz; sz = -1.f; }
  const size_t plane = (size_t)(hz + 1) * (hy + 1) * D.kx;
  const size_t o = ((size_t)kz2 * (hy + 1) + ky2) * D.kx + kx;
  const float* K = D.kern;
  const float nxx = K[o], nyy = K[plane + o], nzz = K[2 * plane + o];
  const float nxy = sy * K[3 * plane + o], nxz = sz * K[4 * plane + o], nyz = sy * sz * K[5 * plane + o];
  const float2 a = mx, b = my, c = mz;
  mx = make_float2(nxx * a.x + nxy * b.x + nxz * c.x, nxx * a.y + nxy * b.y + nxz * c.y);
  my = make_float2(nxy * a.x + nyy * b.x + nyz * c.x, nxy * a.y + nyy * b.y + nyz * c.y);
  mz = make_float2(nxz * a.x + nyz * b.x + nzz * c.x, nxz * a.y + nyz * b.y + nzz * c.y);
}

// ------------------------------------------------------------ x forward
// work item = tile of 2W real rows (c, z, y) of one instance
template <int W>
__global__ __launch_bounds__(256) void k_fft_xf(const InstDesc* __restrict__ descs,
                                                const WorkItem* __restrict__ work, int method,
                                                int stage, const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  const WorkItem wi = work[blockIdx.x];
  const InstDesc& D = descs[wi.inst];
  const InstCtl* C = D.ctl;
  if (C->done) return;
  const int Px = D.px, nx = D.nx, ny = D.ny, nz = D.nz, nc = D.ncell;
  const int nyz = ny * nz, rows = 3 * nyz;
  const int r0 = wi.item * 2 * W;
  const Src src = stage_src(D, C, method, stage);
  constexpr int WP = W + 1;                 // padded line stride (bank conflicts)
  float2* buf = lds;
  float2* twl = lds + Px * WP;
  load_twiddles(twl, Px, tw, 256);
  const int lgx = ilog2(Px);
  for (int e = threadIdx.x; e < 2 * W * Px; e += 256) {
    const int rr = e >> lgx, x = e & (Px - 1);
    const int r = r0 + rr;
    float v = 0.f;
    if (x < nx && r < rows) {
      const int c = r / nyz, yz = r - c * nyz;
      v = src.ld(c * nc + yz * nx + x);
    }
    float* p = reinterpret_cast<float*>(&buf[x * WP + (rr >> 1)]);
    p[rr & 1] = v;
  }
  __syncthreads();
  fft_cols<256, false>(buf, Px, lgx, 1, ilog2(W), 0, WP, twl);
  const int Kx = D.kx;
  for (int e = threadIdx.x; e < Kx * 2 * W; e += 256) {
    const int kx = e / (2 * W), rr = e - kx * 2 * W;
    const int r = r0 + rr;
    if (r >= rows) continue;
    const int line = rr >> 1;
    const float2 Z = buf[brev(kx & (Px - 1), lgx) * WP + line];
    const float2 Zm = buf[brev((Px - kx) & (Px - 1), lgx) * WP + line];
    float2 X;
    if ((rr & 1) == 0) X = make_float2(0.5f * (Z.x + Zm.x), 0.5f * (Z.y - Zm.y));
    else X = make_float2(0.5f * (Z.y + Zm.y), -0.5f * (Z.x - Zm.x));
    const int c = r / nyz, yz = r - c * nyz;
    D.fx[((size_t)kx * 3 + c) * nyz + yz] = X;
  }
}

// ------------------------------------------------------------ x inverse
template <int W>
__global__ __launch_bounds__(256) void k_fft_xi(const InstDesc* __restrict__ descs,
                                                const WorkItem* __restrict__ work,
                                                const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  const WorkItem wi = work[blockIdx.x];
  const InstDesc& D = descs[wi.inst];
  if (D.ctl->done) return;
  const int Px = D.px, nx = D.nx, ny = D.ny, nz = D.nz, nc = D.ncell;
  const int nyz = ny * nz, rows = 3 * nyz;
  const int r0 = wi.item * 2 * W;
  const int Kx = D.kx;
  constexpr int WP = W + 1;             // padded line stride (bank conflicts)
  float2* buf = lds;                    // [Px][W + 1]
  float2* stg = lds + Px * WP;          // [Kx][2W]
  float2* twl = stg + Kx * 2 * W;
  load_twiddles(twl, Px, tw, 256);
  for (int e = threadIdx.x; e < Kx * 2 * W; e += 256) {
    const int kx = e / (2 * W), rr = e - kx * 2 * W;
    const int r = r0 + rr;
    float2 X = make_float2(0.f, 0.f);
    if (r < rows) {
      const int c = r / nyz, yz = r - c * nyz;
      X = D.fx[((size_t)kx * 3 + c) * nyz + yz];
    }
    stg[kx * 2 * W + rr] = X;
  }
  __syncthreads();
  const int half = Px / 2;
  const int lgx = ilog2(Px);
  for (int e = threadIdx.x; e < Px * W; e += 256) {
    const int j = e / W, line = e - j * W;
    float2 Z;
    if (j <= half) {
      float2 a = stg[j * 2 * W + 2 * line], b = stg[j * 2 * W + 2 * line + 1];
      if (j == 0 || j == half) { a.y = 0.f; b.y = 0.f; }
      Z = make_float2(a.x - b.y, a.y + b.x);
    } else {
      const int k = Px - j;
      const float2 a = stg[k * 2 * W + 2 * line], b = stg[k * 2 * W + 2 * line + 1];
      Z = make_float2(a.x + b.y, b.x - a.y);
    }
    buf[brev(j, lgx) * WP + line] = Z;
  }
  __syncthreads();
  fft_cols<256, true>(buf, Px, lgx, 1, ilog2(W), 0, WP, twl);
  const float sc = D.bd_scale;
  for (int e = threadIdx.x; e < 2 * W * nx; e += 256) {
    const int rr = e / nx, x = e - rr * nx;
    const int r = r0 + rr;
    if (r >= rows) continue;
    const float2 Z = buf[x * WP + (rr >> 1)];
    const int c = r / nyz, yz = r - c * nyz;
    D.bd[c * nc + yz * nx + x] = sc * ((rr & 1) ? Z.y : Z.x);
  }
}

// ------------------------------------------------------- fused y-z pass
// work item = kx of one instance.
// LDS: Y rows [3][nz][Py+1] (y transforms), a z work tile [3][Pz][TK] for TK
// adjacent ky columns, twiddles, y-line table.  The z transform of a tile
// starts from nz nonzero rows: its first DIF stage (span Pz/2, upper half
// zero) is folded into the copy into the tile, and the last DIT stage is
// folded into the copy back, which keeps only z < nz.
#define MM_YZ_T 512
__global__ __launch_bounds__(MM_YZ_T) void k_fft_yz(const InstDesc* __restrict__ descs,
                                                    const WorkItem* __restrict__ work,
                                                    const float2* __restrict__ tw, int TK) {
  extern __shared__ float2 lds[];
  const WorkItem wi = work[blockIdx.x];
  const InstDesc& D = descs[wi.inst];
  if (D.ctl->done) return;
  const int kx = wi.item;
  const int ny = D.ny, nz = D.nz, Py = D.py, Pz = D.pz;
  const int RP = Py + 1;
  const int yplane = nz * RP;                 // one component of the Y rows
  const int zplane = Pz * TK;                 // one component of the z tile
  float2* ybuf = lds;
  float2* zbuf = ybuf + 3 * yplane;
  float2* twy = zbuf + 3 * zplane;
  float2* twz = twy + Py;
  int* ytab = reinterpret_cast<int*>(twz + Pz);
  load_twiddles(twy, Py, tw, MM_YZ_T);
  load_twiddles(twz, Pz, tw, MM_YZ_T);
  for (int l = threadIdx.x; l < 3 * nz; l += MM_YZ_T) ytab[l] = l * RP;
  const int lgy = ilog2(Py), lgz = ilog2(Pz), lgT = ilog2(TK);
  const int nyz = ny * nz;
  float2* X = D.fx + (size_t)kx * 3 * nyz;
  // load rows, zero-padded in y
  for (int e = threadIdx.x; e < 3 * nz * Py; e += MM_YZ_T) {
    const int l = e >> lgy, y = e & (Py - 1);
    ybuf[l * RP + y] = (y < ny) ? X[l * ny + y] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_rows<MM_YZ_T, false>(ybuf, Py, lgy, 3 * nz, ytab, twy);
  const int hz = Pz >> 1;
  for (int k0 = 0; k0 < Py; k0 += TK) {
    // copy in with the first DIF stage: out[z] = x[z], out[z + Pz/2] = x[z] W^z
    if (Pz == 1) {
      for (int e = threadIdx.x; e < 3 * TK; e += MM_YZ_T) {
        const int c = e >> lgT, t = e & (TK - 1);
        zbuf[c * zplane + t] = ybuf[c * yplane + k0 + t];
      }
    } else {
      for (int e = threadIdx.x; e < 3 * hz * TK; e += MM_YZ_T) {
        const int t = e & (TK - 1), rest = e >> lgT;
        const int z = rest & (hz - 1), c = rest >> (lgz - 1);
        float2 v = make_float2(0.f, 0.f);
        if (z < nz) v = ybuf[c * yplane + z * RP + k0 + t];
        zbuf[c * zplane + z * TK + t] = v;
        zbuf[c * zplane + (z + hz) * TK + t] = cmul(v, twz[z]);
      }
    }
    __syncthreads();
    if (Pz > 1) fft_cols<MM_YZ_T, false>(zbuf, Pz, lgz, 3, lgT, zplane, TK, twz, 1);
    // spectra at bit-reversed positions in y and z
    for (int e = threadIdx.x; e < Pz * TK; e += MM_YZ_T) {
      const int pz_ = e >> lgT, t = e & (TK - 1);
      const int o = pz_ * TK + t;
      float2 mx = zbuf[o], my = zbuf[zplane + o], mz = zbuf[2 * zplane + o];
      kernel_mul(D, kx, brev(k0 + t, lgy), brev(pz_, lgz), mx, my, mz);
      zbuf[o] = mx;
      zbuf[zplane + o] = my;
      zbuf[2 * zplane + o] = mz;
    }
    __syncthreads();
    if (Pz > 1) fft_cols<MM_YZ_T, true>(zbuf, Pz, lgz, 3, lgT, zplane, TK, twz, 0, lgz - 1);
    // copy back with the last DIT stage: out[z] = x[z] + x[z + Pz/2] conj(W^z), z < nz
    for (int e = threadIdx.x; e < 3 * nz * TK; e += MM_YZ_T) {
      const int t = e & (TK - 1), rest = e >> lgT;
      const int c = rest / nz, z = rest - c * nz;
      float2 v = zbuf[c * zplane + z * TK + t];
      if (Pz > 1) v = cadd(v, cmul(zbuf[c * zplane + (z + hz) * TK + t], twid<true>(twz, z)));
      ybuf[c * yplane + z * RP + k0 + t] = v;
    }
    __syncthreads();
  }
  fft_rows<MM_YZ_T, true>(ybuf, Py, lgy, 3 * nz, ytab, twy);
  for (int e = threadIdx.x; e < 3 * nz * Py; e += MM_YZ_T) {
    const int l = e >> lgy, y = e & (Py - 1);
    if (y < ny) X[l * ny + y] = ybuf[l * RP + y];
  }
}

// --------------------------------------------------------- split y passes
// work item = tile of W lines (kx, c, z) of one instance; LDS [Py][W]
template <int DIR>
__global__ __launch_bounds__(256) void k_fft_y(const InstDesc* __restrict__ descs,
                                               const WorkItem* __restrict__ work, int W,
                                               const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  const WorkItem wi = work[blockIdx.x];
  const InstDesc& D = descs[wi.inst];
  if (D.ctl->done) return;
  const int ny = D.ny, Py = D.py;
  const int nlines = D.kx * 3 * D.nz;
  const int l0 = wi.item * W;
  const int WP = W + 1;                   // padded line stride (bank conflicts)
  float2* buf = lds;
  float2* twl = lds + Py * WP;
  load_twiddles(twl, Py, tw, 256);
  const int nin = (DIR < 0) ? ny : Py;
  const int lgy = ilog2(Py);
  for (int e = threadIdx.x; e < W * Py; e += 256) {
    const int ll = e >> lgy, y = e & (Py - 1);
    const int l = l0 + ll;
    float2 v = make_float2(0.f, 0.f);
    if (l < nlines && y < nin) v = (DIR < 0) ? D.fx[(size_t)l * ny + y] : D.fy[(size_t)l * Py + y];
    // forward: natural order in; inverse: bit-reversed order in
    buf[((DIR < 0) ? y : brev(y, lgy)) * WP + ll] = v;
  }
  __syncthreads();
  if (DIR < 0) fft_cols<256, false>(buf, Py, lgy, 1, ilog2(W), 0, WP, twl);
  else fft_cols<256, true>(buf, Py, lgy, 1, ilog2(W), 0, WP, twl);
  const int nout = (DIR < 0) ? Py : ny;
  for (int e = threadIdx.x; e < W * nout; e += 256) {
    const int ll = e / nout, y = e - ll * nout;
    const int l = l0 + ll;
    if (l >= nlines) continue;
    const float2 v = buf[((DIR < 0) ? brev(y, lgy) : y) * WP + ll];
    if (DIR < 0) D.fy[(size_t)l * Py + y] = v;
    else D.fx[(size_t)l * ny + y] = v;
  }
}

// ---------------------------------------------- split z pass with multiply
// work item = (kx, tile of TW ky) of one instance; LDS [Pz][3 TW]
__global__ __launch_bounds__(256) void k_fft_zc(const InstDesc* __restrict__ descs,
                                                const WorkItem* __restrict__ work, int TW,
                                                const float2* __restrict__ tw) {
  extern __shared__ float2 lds[];
  const WorkItem wi = work[blockIdx.x];
  const InstDesc& D = descs[wi.inst];
  if (D.ctl->done) return;
  const int nz = D.nz, Py = D.py, Pz = D.pz;
  const int tiles = (Py + TW - 1) / TW;
  const int kx = wi.item / tiles;
  const int ky0 = (wi.item - kx * tiles) * TW;
  const int NL = 3 * TW;
  float2* buf = lds;
  float2* twl = lds + Pz * NL;
  load_twiddles(twl, Pz, tw, 256);
  for (int e = threadIdx.x; e < Pz * NL; e += 256) {
    const int z = e / NL, l = e - z * NL;
    const int c = l / TW, t = l - c * TW;
    const int ky = ky0 + t;
    float2 v = make_float2(0.f, 0.f);
    if (z < nz && ky < Py) v = D.fy[(((size_t)kx * 3 + c) * nz + z) * Py + ky];
    buf[e] = v;
  }
  __syncthreads();
  const int lgz = ilog2(Pz), lgT = ilog2(TW);
  fft_cols<256, false>(buf, Pz, lgz, 3, lgT, TW, NL, twl);
  for (int e = threadIdx.x; e < Pz * TW; e += 256) {
    const int pz_ = e / TW, t = e - pz_ * TW;
    const int ky = ky0 + t;
    if (ky >= Py) continue;
    float2 mx = buf[pz_ * NL + t], my = buf[pz_ * NL + TW + t], mz = buf[pz_ * NL + 2 * TW + t];
    kernel_mul(D, kx, ky, brev(pz_, lgz), mx, my, mz);
    buf[pz_ * NL + t] = mx;
    buf[pz_ * NL + TW + t] = my;
    buf[pz_ * NL + 2 * TW + t] = mz;
  }
  __syncthreads();
  fft_cols<256, true>(buf, Pz, lgz, 3, lgT, TW, NL, twl);
  for (int e = threadIdx.x; e < nz * NL; e += 256) {
    const int z = e / NL, l = e - z * NL;
    const int c = l / TW, t = l - c * TW;
    const int ky = ky0 + t;
    if (ky < Py) D.fy[(((size_t)kx * 3 + c) * nz + z) * Py + ky] = buf[e];
  }
}

}  // namespace mmk

// ------------------------------------------------------------ launchers
hipError_t mmk_launch_fft_xf(int W, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             int method, int stage, const float2* tw, hipStream_t s) {
  switch (W) {
    case 1: hipLaunchKernelGGL(mmk::k_fft_xf<1>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    case 2: hipLaunchKernelGGL(mmk::k_fft_xf<2>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    case 4: hipLaunchKernelGGL(mmk::k_fft_xf<4>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    case 8: hipLaunchKernelGGL(mmk::k_fft_xf<8>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    case 16: hipLaunchKernelGGL(mmk::k_fft_xf<16>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    case 32: hipLaunchKernelGGL(mmk::k_fft_xf<32>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mmk_launch_fft_xi(int W, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             const float2* tw, hipStream_t s) {
  switch (W) {
    case 1: hipLaunchKernelGGL(mmk::k_fft_xi<1>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    case 2: hipLaunchKernelGGL(mmk::k_fft_xi<2>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    case 4: hipLaunchKernelGGL(mmk::k_fft_xi<4>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    case 8: hipLaunchKernelGGL(mmk::k_fft_xi<8>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    case 16: hipLaunchKernelGGL(mmk::k_fft_xi<16>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    case 32: hipLaunchKernelGGL(mmk::k_fft_xi<32>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mmk_launch_fft_yz(int TK, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             const float2* tw, hipStream_t s) {
  hipLaunchKernelGGL(mmk::k_fft_yz, dim3(nblocks), dim3(MM_YZ_T), lds, s, d, w, tw, TK);
  return hipGetLastError();
}

hipError_t mmk_launch_fft_y(int dir, int W, int nblocks, size_t lds, const InstDesc* d,
                            const WorkItem* w, const float2* tw, hipStream_t s) {
  if (dir < 0) hipLaunchKernelGGL(mmk::k_fft_y<-1>, dim3(nblocks), dim3(256), lds, s, d, w, W, tw);
  else hipLaunchKernelGGL(mmk::k_fft_y<1>, dim3(nblocks), dim3(256), lds, s, d, w, W, tw);
  return hipGetLastError();
}

hipError_t mmk_launch_fft_zc(int TW, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             const float2* tw, hipStream_t s) {
  hipLaunchKernelGGL(mmk::k_fft_zc, dim3(nblocks), dim3(256), lds, s, d, w, TW, tw);
  return hipGetLastError();
}

hipError_t mmk_set_lds_limits() {
  hipError_t e = hipFuncSetAttribute((const void*)mmk::k_fft_yz,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  return e;
}
