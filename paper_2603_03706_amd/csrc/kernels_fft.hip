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
#include <type_traits>
#include "mm_internal.h"
#include "kernels_common.h"
#include "launch.h"
#include "fft_lds.h"
#include "stage_final.h"

namespace mmk {

// 3x3 kernel multiply at (kx, ky, kz): H = N M (sign and scale applied later)
__device__ __forceinline__ void kernel_mul(const InstDesc& D, int kx, int ky, int kz, float2& mx,
                                           float2& my, float2& mz) {
  const int hy = D.py / 2, hz = D.pz / 2;
  int ky2 = ky, kz2 = kz;
  float sy = 1.f, sz = 1.f;
  if (ky > hy) { ky2 = D.py - ky; sy = -1.f; }
  if (kz > hz) { kz2 = D.pz - kz; sz = -1.f; }
  const int plane = (hz + 1) * (hy + 1);
  const int o = kz2 * (hy + 1) + ky2;
  const MMG float* K = gbl(D.kern) + (size_t)kx * 6 * plane;
  const float nxx = K[o], nyy = K[plane + o], nzz = K[2 * plane + o];
  const float nxy = sy * K[3 * plane + o], nxz = sz * K[4 * plane + o], nyz = sy * sz * K[5 * plane + o];
  const float2 a = mx, b = my, c = mz;
  mx = make_float2(nxx * a.x + nxy * b.x + nxz * c.x, nxx * a.y + nxy * b.y + nxz * c.y);
  my = make_float2(nxy * a.x + nyy * b.x + nyz * c.x, nxy * a.y + nyy * b.y + nyz * c.y);
  mz = make_float2(nxz * a.x + nyz * b.x + nzz * c.x, nxz * a.y + nyz * b.y + nzz * c.y);
}

// the same multiply with the kernel slice of one kx staged in LDS as [6][PZ/2+1][PY/2+1]
template <int PY, int PZ>
__device__ __forceinline__ void kernel_mul_lds(const float* Ks, int ky, int kz, float2& mx, float2& my, float2& mz) {
  constexpr int HY = PY / 2, HZ = PZ / 2, PL = (HZ + 1) * (HY + 1);
  int ky2 = ky, kz2 = kz;
  float sy = 1.f, sz = 1.f;
  if (ky > HY) { ky2 = PY - ky; sy = -1.f; }
  if (kz > HZ) { kz2 = PZ - kz; sz = -1.f; }
  const float* K = Ks + kz2 * (HY + 1) + ky2;
  const float nxx = K[0], nyy = K[PL], nzz = K[2 * PL];
  const float nxy = sy * K[3 * PL], nxz = sz * K[4 * PL], nyz = sy * sz * K[5 * PL];
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
  const MMG InstCtl* __restrict__ C = gbl(D.ctl);
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
  // Entries x >= Px/2 are zero padding (nx <= Px/2): with lines of four or
  // more points only the lower half is stored here and the first DIF stage
  // below reads just the two nonzero quarters.
  const bool pruned = Px >= 4;
  const int nl = pruned ? Px >> 1 : Px, lgl = pruned ? lgx - 1 : lgx;
  // batches of 8 loads per thread in flight (clamped addresses, padding selected afterwards)
  const bool two = src.p1 != nullptr;
  for (int e0 = 0; e0 < 2 * W * nl; e0 += 8 * 256) {
    float v[8];
    int idx[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256 + threadIdx.x;
      const int rr = e >> lgl, x = e & (nl - 1);
      const int rc = min(r0 + rr, rows - 1);
      const int c = (rc >= nyz) + (rc >= 2 * nyz), yz = rc - c * nyz;
      idx[u] = c * nc + yz * nx + min(x, nx - 1);
      v[u] = src.p0[idx[u]];
    }
    if (two) {
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = fmaf(src.c1, src.p1[idx[u]], v[u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256 + threadIdx.x;
      const int rr = e >> lgl, x = e & (nl - 1);
      if (!(e < 2 * W * nl && x < nx && r0 + rr < rows)) v[u] = 0.f;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256 + threadIdx.x;
      if (e < 2 * W * nl) {
        const int rr = e >> lgl, x = e & (nl - 1);
        float* p = reinterpret_cast<float*>(&buf[x * WP + (rr >> 1)]);
        p[rr & 1] = v[u];
      }
    }
  }
  __syncthreads();
  if (pruned) {
    // first radix-2^2 DIF stage (span Px/2) with the arithmetic of the full
    // stage, zeros for its inputs x2, x3
    const int q = Px >> 2;
    const float2 zero = make_float2(0.f, 0.f);
    for (int e = threadIdx.x; e < W * q; e += 256) {
      const int ll = e & (W - 1), i = e / W;
      float2* line = buf + ll;
      const float2 x0 = line[i * WP], x1 = line[(i + q) * WP];
      const float2 w1 = twl[i], w2 = twl[2 * i];
      const float2 a0 = cadd(x0, zero), a1 = cadd(x1, zero);
      const float2 a2 = cmul(csub(x0, zero), w1);
      const float2 a3 = rot<false>(cmul(csub(x1, zero), w1));
      line[i * WP] = cadd(a0, a1);
      line[(i + q) * WP] = cmul(csub(a0, a1), w2);
      line[(i + 2 * q) * WP] = cadd(a2, a3);
      line[(i + 3 * q) * WP] = cmul(csub(a2, a3), w2);
    }
    __syncthreads();
  }
  fft_cols<256, false>(buf, Px, lgx, 1, ilog2(W), 0, WP, twl, pruned ? 2 : 0);
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
    // X[kx][c][z][y] with row r = (c, z, y): offset kx * rows + r
    gst2(gbl(D.fx) + (size_t)kx * rows + r, X);
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
  if (gbl(D.ctl)->done) return;
  const int Px = D.px, nx = D.nx, ny = D.ny, nz = D.nz, nc = D.ncell;
  const int nyz = ny * nz, rows = 3 * nyz;
  const int r0 = wi.item * 2 * W;
  const int Kx = D.kx;
  constexpr int WP = W + 1;             // padded line stride (bank conflicts)
  float2* buf = lds;                    // [Px][W + 1]
  float2* stg = lds + Px * WP;          // [Kx][2W]
  float2* twl = stg + Kx * 2 * W;
  load_twiddles(twl, Px, tw, 256);
  // batches of 8 loads per thread in flight (clamped addresses, padding selected afterwards)
  const MMG float2* fx = gbl(D.fx);
  for (int e0 = 0; e0 < Kx * 2 * W; e0 += 8 * 256) {
    float2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256 + threadIdx.x;
      const int kx = min(e / (2 * W), Kx - 1), rr = e - (e / (2 * W)) * 2 * W;
      const int r = r0 + rr;
      const bool in = e < Kx * 2 * W && r < rows;
      const float2 t = gld2(fx + (size_t)kx * rows + min(r, rows - 1));
      v[u] = make_float2(in ? t.x : 0.f, in ? t.y : 0.f);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256 + threadIdx.x;
      if (e < Kx * 2 * W) stg[e] = v[u];
    }
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
    gbl(D.bd)[r * nx + x] = sc * ((rr & 1) ? Z.y : Z.x);
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
  if (gbl(D.ctl)->done) return;
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
  MMG float2* X = gbl(D.fx) + (size_t)kx * 3 * nyz;
  // load rows, zero-padded in y
  for (int e = threadIdx.x; e < 3 * nz * Py; e += MM_YZ_T) {
    const int l = e >> lgy, y = e & (Py - 1);
    ybuf[l * RP + y] = (y < ny) ? gld2(X + l * ny + y) : make_float2(0.f, 0.f);
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
    if (y < ny) gst2(X + l * ny + y, ybuf[l * RP + y]);
  }
}

// ------------------------------------------- fused y-z, lines in registers
// A padded line of length P = 4M whose inputs vanish from index 2M on is
// split by the residue r = k mod 4 of the frequency index k = 4k' + r:
//   X[4k' + r] = sum_j W_M^{k'j} f_r[j],  f_r[j] = W_P^{rj} (x[j] + (-i)^r x[j+M]),
// an M-point DFT of a folded sequence.  The inverse, cropped to outputs
// y = y0 + M jj < 2M, is the 4-point inverse DFT over r of
//   w_r[y0] = W_P^{-r y0} (M-point inverse DFT of X[4k' + r] over k')[y0].
// Each lane keeps one residue of one line (M points) in registers; the four
// residues of a line sit in adjacent lanes of one wavefront, which combine
// the inverse with two quad permutations.  One workgroup per (instance, kx):
//   load X -> LDS rows [3][nz][Py+1];  forward y per row (in place);
//   per ky column: forward z, kernel multiply, inverse z (in place);
//   inverse y per row (in place);  store X.
// Lines are read and written by the four lanes of one quad in program order,
// so only the three phase changes need workgroup barriers.
#define MM_YZR_T 256

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

// d * (1 + hf (W_M^{+-k} - 1)): the twiddle for lanes with hf = 1, the
// identity for hf = 0 (k > 0, M <= 16)
template <int M, bool INV>
__device__ __forceinline__ float2 twh(float2 d, int k, float hf) {
  const int j = k * (16 / M);
  const float c = cos16(j), sn = INV ? cos16(j - 4) : -cos16(j - 4);
  const float tr = fmaf(hf, c - 1.f, 1.f), ti = hf * sn;
  return make_float2(d.x * tr - d.y * ti, d.x * ti + d.y * tr);
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

// (-i)^r of a lane's residue r, as (re, im) in {0, +-1}
struct Root4 {
  float re, im;
  __device__ __forceinline__ explicit Root4(int r)
      : re((r & 1) ? 0.f : ((r & 2) ? -1.f : 1.f)), im((r & 1) ? ((r & 2) ? 1.f : -1.f) : 0.f) {}
};
// the same fold with the residue's root held by the lane: x0 + c x1 by two
// fused multiply-adds per part (c has one nonzero part, so each result is
// rounded once, as the plain sum), then the twiddle
__device__ __forceinline__ float2 fold_c(float2 x0, float2 x1, Root4 c, float2 w) {
  const float2 s = make_float2(fmaf(c.re, x1.x, fmaf(-c.im, x1.y, x0.x)), fmaf(c.re, x1.y, fmaf(c.im, x1.x, x0.y)));
  return cmul(s, w);
}

template <int MY, int MZ>
__global__ __launch_bounds__(MM_YZR_T, 2) void k_fft_yzr(const InstDesc* __restrict__ descs,
                                                         const WorkItem* __restrict__ work,
                                                         const float2* __restrict__ tw) {
  // LDS rows [3][2 MZ][RS]: row (c, z) holds y samples, zero beyond (nz, ny),
  // so every line read below is unconditional with compile-time offsets
  constexpr int PY = 4 * MY, PZ = 4 * MZ, RS = PY + 1, ZR = 2 * MZ, YR = 2 * MY;
  constexpr int lgMY = ilog2c(MY), lgMZ = ilog2c(MZ), lgPY = lgMY + 2;
  extern __shared__ float2 lds[];
  float2* B = lds;
  float2* twy = B + 3 * ZR * RS;
  float2* twz = twy + PY;
  float2* tw32 = twz + PZ;
  float* Ks = reinterpret_cast<float*>(tw32 + 32);   // kernel slice of this kx: [6][PZ/2+1][PY/2+1]
  constexpr int HY1 = PY / 2 + 1, KPL = (PZ / 2 + 1) * HY1;
  constexpr int NK = (6 * KPL + MM_YZR_T - 1) / MM_YZR_T, NXE = 3 * ZR * PY;
  constexpr int NX = (NXE + MM_YZR_T - 1) / MM_YZR_T;
  load_twiddles(twy, PY, tw, MM_YZR_T);
  load_twiddles(twz, PZ, tw, MM_YZR_T);
  load_twiddles(tw32, 32, tw, MM_YZR_T);
  const WorkItem wi = work[blockIdx.x];
  const InstDesc& D = descs[wi.inst];
  if (gbl(D.ctl)->done) return;
  const int kx = wi.item;
  const int ny = D.ny, nz = D.nz;
  const int nrow = 3 * nz;
  MMG float2* X = gbl(D.fx) + (size_t)kx * nrow * ny;
  {
    // all global loads of the prologue are issued before the first wait
    const MMG float* K = gbl(D.kern) + (size_t)kx * 6 * KPL;
    float kv[NK];
    float2 xv[NX];
#pragma unroll
    for (int it = 0; it < NK; ++it) kv[it] = K[min(it * MM_YZR_T + (int)threadIdx.x, 6 * KPL - 1)];
#pragma unroll
    for (int it = 0; it < NX; ++it) {
      // rows z >= nz are read by the z pass at every ky: they are cleared over the full padded width;
      // clamped (in-bounds) address, padding selected afterwards: no branch between the loads
      const int e = it * MM_YZR_T + threadIdx.x;
      const int row = e >> lgPY, y = e & (PY - 1);
      const int c = row / ZR, z = row - c * ZR;
      const bool in = e < NXE && z < nz && y < ny;
      const float2 v = gld2(X + (min(c, 2) * nz + min(z, nz - 1)) * ny + min(y, ny - 1));
      xv[it] = make_float2(in ? v.x : 0.f, in ? v.y : 0.f);
    }
#pragma unroll
    for (int it = 0; it < NK; ++it) {
      const int e = it * MM_YZR_T + threadIdx.x;
      if (e < 6 * KPL) Ks[e] = kv[it];
    }
#pragma unroll
    for (int it = 0; it < NX; ++it) {
      const int e = it * MM_YZR_T + threadIdx.x;
      const int row = e >> lgPY, y = e & (PY - 1);
      const int z = row % ZR;
      if (e < NXE && (z >= nz || y < YR)) B[row * RS + y] = xv[it];
    }
  }
  __syncthreads();
  {
  // forward y.  Up to 64-point rows: two residue lanes per row, 2 MY points
  // each; the upper half of a padded row is zero, so the fold reduces to the
  // twiddle W^{rj}.  Longer rows: four residue lanes as in the z pass.
  if constexpr (MY <= 16) {
    constexpr int M2 = 2 * MY, lg2 = lgMY + 1;
#pragma unroll 1
    for (int t = threadIdx.x; t < 2 * 3 * ZR; t += MM_YZR_T) {
      const int r = t & 1;
      float2* line = B + (t >> 1) * RS;
      float2 f[M2];
#pragma unroll
      for (int j = 0; j < M2; ++j) f[j] = cmul(line[j], twy[r * j]);
      reg_dft<M2, false>(f, tw32);
#pragma unroll
      for (int p = 0; p < M2; ++p) line[2 * brevc(p, lg2) + r] = f[p];
    }
  } else {
#pragma unroll 1
    for (int t = threadIdx.x; t < 4 * 3 * ZR; t += MM_YZR_T) {
      const int r = t & 3;
      float2* line = B + (t >> 2) * RS;
      float2 f[MY];
#pragma unroll
      for (int j = 0; j < MY; ++j) f[j] = fold(line[j], line[j + MY], r, twy[r * j]);
      reg_dft<MY, false>(f, tw32);
#pragma unroll
      for (int p = 0; p < MY; ++p) line[4 * brevc(p, lgMY) + r] = f[p];
    }
  }
  __syncthreads();
  // z per ky column: forward, kernel multiply, inverse
#pragma unroll 1
  for (int t = threadIdx.x; t < 4 * PY; t += MM_YZR_T) {
    const int ky = t >> 2, r = t & 3;
    float2 fx[MZ], fy[MZ], fz[MZ];
    const float2* col = B + ky;
#pragma unroll
    for (int j = 0; j < MZ; ++j) fx[j] = fold(col[j * RS], col[(j + MZ) * RS], r, twz[r * j]);
    reg_dft<MZ, false>(fx, tw32);
    asm volatile("" ::: "memory");
#pragma unroll
    for (int j = 0; j < MZ; ++j) fy[j] = fold(col[(ZR + j) * RS], col[(ZR + j + MZ) * RS], r, twz[r * j]);
    reg_dft<MZ, false>(fy, tw32);
    asm volatile("" ::: "memory");
#pragma unroll
    for (int j = 0; j < MZ; ++j) fz[j] = fold(col[(2 * ZR + j) * RS], col[(2 * ZR + j + MZ) * RS], r, twz[r * j]);
    reg_dft<MZ, false>(fz, tw32);
    asm volatile("" ::: "memory");
#pragma unroll
    for (int p = 0; p < MZ; ++p) {
      kernel_mul_lds<PY, PZ>(Ks, ky, 4 * brevc(p, lgMZ) + r, fx[p], fy[p], fz[p]);
      asm volatile("" ::: "memory");
    }
    const int z0 = (MZ / 2) * (r >> 1) + MZ * (r & 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float2 g[MZ];
#pragma unroll
      for (int k = 0; k < MZ; ++k) g[k] = c == 0 ? fx[brevc(k, lgMZ)] : c == 1 ? fy[brevc(k, lgMZ)] : fz[brevc(k, lgMZ)];
      reg_dft<MZ, true>(g, tw32);
      float2 v[MZ];
#pragma unroll
      for (int y0 = 0; y0 < MZ; ++y0) v[y0] = cmul(g[brevc(y0, lgMZ)], twid<true>(twz, r * y0));
      float2 o[MZ / 2];
      quad_inverse<MZ>(v, r, o);
      float2* out = B + (c * ZR + z0) * RS + ky;
#pragma unroll
      for (int i = 0; i < MZ / 2; ++i)
        if (z0 + i < nz) out[i * RS] = o[i];
      asm volatile("" ::: "memory");
    }
  }
  __syncthreads();
  }
  {
  // inverse y (cropped to y < 2 MY), the same lane split as the forward pass
  if constexpr (MY <= 16) {
    constexpr int M2 = 2 * MY, lg2 = lgMY + 1;
#pragma unroll 1
    for (int t = threadIdx.x; t < 2 * 3 * ZR; t += MM_YZR_T) {
      const int r = t & 1;
      float2* line = B + (t >> 1) * RS;
      float2 g[M2];
#pragma unroll
      for (int k = 0; k < M2; ++k) g[k] = line[2 * k + r];
      reg_dft<M2, true>(g, tw32);
      // h[y0] = w_0[y0] + w_1[y0]; lane r keeps y0 in [r MY, (r + 1) MY)
#pragma unroll
      for (int i = 0; i < MY; ++i) {
        const float2 w0 = cmul(g[brevc(i, lg2)], twid<true>(twy, r * i));
        const float2 w1 = cmul(g[brevc(i + MY, lg2)], twid<true>(twy, r * (i + MY)));
        const float2 got = make_float2(dpp_x1(r ? w0.x : w1.x), dpp_x1(r ? w0.y : w1.y));
        line[r * MY + i] = cadd(r ? w1 : w0, got);
      }
    }
  } else {
#pragma unroll 1
    for (int t = threadIdx.x; t < 4 * 3 * ZR; t += MM_YZR_T) {
      const int r = t & 3;
      float2* line = B + (t >> 2) * RS;
      float2 g[MY];
#pragma unroll
      for (int k = 0; k < MY; ++k) g[k] = line[4 * k + r];
      reg_dft<MY, true>(g, tw32);
      float2 v[MY];
#pragma unroll
      for (int y0 = 0; y0 < MY; ++y0) v[y0] = cmul(g[brevc(y0, lgMY)], twid<true>(twy, r * y0));
      float2 o[MY / 2];
      quad_inverse<MY>(v, r, o);
      const int y0 = (MY / 2) * (r >> 1) + MY * (r & 1);
#pragma unroll
      for (int i = 0; i < MY / 2; ++i) line[y0 + i] = o[i];
    }
  }
  __syncthreads();
#pragma unroll 4
  for (int e = threadIdx.x; e < 3 * ZR * YR; e += MM_YZR_T) {
    const int row = e >> (lgMY + 1), y = e & (YR - 1);
    const int c = row / ZR, z = row & (ZR - 1);
    if (z < nz && y < ny) gst2(X + (c * nz + z) * ny + y, B[row * RS + y]);
  }
  }
}

// ------------------------------ fused y-z, eight lanes per z column (T = 512)
// The same transform as k_fft_yzr, with each residue's z line split again
// over two lanes (h = 0, 1) by one radix-2 stage: the even and odd outputs of
// the residue DFT are (M/2)-point DFTs of f[j] + f[j+M/2] and
// (f[j] - f[j+M/2]) W_M^j, and its inverse recombines the two half-length
// inverses the same way.  Lane l = 2r + h of a group of eight: the half
// exchange is a DPP swap of adjacent lanes, residue pairs r^1 are two lanes
// apart (DPP), r^2 four lanes apart (swizzle).  Half the registers per lane
// of k_fft_yzr, so twice the wavefronts per SIMD; y rows use four lanes.
#define MM_YZ8_T 512

__device__ __forceinline__ float swz_x4(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x101F));
}
__device__ __forceinline__ float2 lane_x4(float2 v) { return make_float2(swz_x4(v.x), swz_x4(v.y)); }
__device__ __forceinline__ float2 lane_x2(float2 v) { return make_float2(dpp_x2(v.x), dpp_x2(v.y)); }
__device__ __forceinline__ float2 lane_x1(float2 v) { return make_float2(dpp_x1(v.x), dpp_x1(v.y)); }

// quad_inverse with residue r^2 four lanes and r^1 two lanes apart
template <int M>
__device__ __forceinline__ void quad_inverse8(const float2 (&w)[M], int r, float2 (&out)[M / 2]) {
  const bool hi = r & 2, odd = r & 1;
#pragma unroll
  for (int i = 0; i < M / 2; ++i) {
    const float2 mine = hi ? w[i + M / 2] : w[i];
    const float2 recv = lane_x4(hi ? w[i] : w[i + M / 2]);
    const float2 sm = cadd(mine, recv);
    const float2 df = hi ? csub(recv, mine) : csub(mine, recv);
    const float2 got = lane_x2(odd ? sm : df);
    out[i] = odd ? cadd(got, rot<true>(df)) : cadd(sm, got);
  }
}

// Workgroups nyz .. nyz + nfinal - 1 of the launch do not transform: each
// runs the finalisation of stage fstage (method fmethod) for instance
// blockIdx.x - nyz.  That work reads only the partial records and control
// blocks of the previous stage kernel, which the transform never touches, so
// the two share one launch and the finalisation fills the last, partly empty
// round of transform workgroups.
static_assert(MM_YZ8_T == MMI_WG, "the finalisation body assumes MMI_WG threads");

template <int MY, int MZ>
__global__ __launch_bounds__(MM_YZ8_T) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_fft_yz8(const InstDesc* __restrict__ descs,
                                                         const WorkItem* __restrict__ work,
                                                         const float2* __restrict__ tw, int nyz,
                                                         int fmethod, int fstage) {
  constexpr int PY = 4 * MY, PZ = 4 * MZ, RS = PY + 1, ZR = 2 * MZ, YR = 2 * MY, MH = MZ / 2;
  constexpr int lgMY = ilog2c(MY), lgMZ = ilog2c(MZ), lgMH = lgMZ - 1, lgPY = lgMY + 2;
  extern __shared__ float2 lds[];
  if ((int)blockIdx.x >= nyz) {
    final_any(fmethod, fstage, descs, (int)blockIdx.x - nyz, reinterpret_cast<double*>(lds));
    return;
  }
  float2* B = lds;
  float2* twy = B + 3 * ZR * RS;
  float2* twz = twy + PY;
  float2* tw32 = twz + PZ;
  float* Ks = reinterpret_cast<float*>(tw32 + 32);
  constexpr int HY1 = PY / 2 + 1, KPL = (PZ / 2 + 1) * HY1;
  constexpr int NK = (6 * KPL + MM_YZ8_T - 1) / MM_YZ8_T, NXE = 3 * ZR * PY;
  constexpr int NX = (NXE + MM_YZ8_T - 1) / MM_YZ8_T;
  load_twiddles(twy, PY, tw, MM_YZ8_T);
  load_twiddles(twz, PZ, tw, MM_YZ8_T);
  load_twiddles(tw32, 32, tw, MM_YZ8_T);
  const WorkItem wi = work[blockIdx.x];
  const InstDesc& D = descs[wi.inst];
  if (gbl(D.ctl)->done) return;
  const int kx = wi.item;
  const int ny = D.ny, nz = D.nz;
  const int nrow = 3 * nz;
  MMG float2* X = gbl(D.fx) + (size_t)kx * nrow * ny;
  {
    const MMG float* K = gbl(D.kern) + (size_t)kx * 6 * KPL;
    float kv[NK];
    float2 xv[NX];
#pragma unroll
    for (int it = 0; it < NK; ++it) kv[it] = K[min(it * MM_YZ8_T + (int)threadIdx.x, 6 * KPL - 1)];
#pragma unroll
    for (int it = 0; it < NX; ++it) {
      const int e = it * MM_YZ8_T + threadIdx.x;
      const int row = e >> lgPY, y = e & (PY - 1);
      const int c = row / ZR, z = row - c * ZR;
      const bool in = e < NXE && z < nz && y < ny;
      const float2 v = gld2(X + (min(c, 2) * nz + min(z, nz - 1)) * ny + min(y, ny - 1));
      xv[it] = make_float2(in ? v.x : 0.f, in ? v.y : 0.f);
    }
#pragma unroll
    for (int it = 0; it < NK; ++it) {
      const int e = it * MM_YZ8_T + threadIdx.x;
      if (e < 6 * KPL) Ks[e] = kv[it];
    }
#pragma unroll
    for (int it = 0; it < NX; ++it) {
      const int e = it * MM_YZ8_T + threadIdx.x;
      const int row = e >> lgPY, y = e & (PY - 1);
      const int z = row % ZR;
      if (e < NXE && (z >= nz || y < YR)) B[row * RS + y] = xv[it];
    }
  }
  __syncthreads();
  // forward y, four residue lanes per row
#pragma unroll 1
  for (int t = threadIdx.x; t < 4 * 3 * ZR; t += MM_YZ8_T) {
    const int r = t & 3;
    const Root4 cr(r);
    float2* line = B + (t >> 2) * RS;
    float2 f[MY];
#pragma unroll
    for (int j = 0; j < MY; ++j) f[j] = fold_c(line[j], line[j + MY], cr, twy[r * j]);
    reg_dft<MY, false>(f, tw32);
#pragma unroll
    for (int p = 0; p < MY; ++p) line[4 * brevc(p, lgMY) + r] = f[p];
  }
  __syncthreads();
  // z per ky column: eight lanes (residue r, half h).  The lane-dependent
  // roles are written as arithmetic with per-lane constants instead of
  // selects: sg = +1 / -1 for h = 0 / 1, and the half-split twiddle is
  // 1 + hf (W - 1) with hf = h.
#pragma unroll 1
  for (int t = threadIdx.x; t < 8 * PY; t += MM_YZ8_T) {
    const int ky = t >> 3, h = t & 1, r = (t >> 1) & 3;
    const Root4 cr(r);
    const float hf = (float)h, sg = 1.f - 2.f * hf;
    const float2* col = B + ky;
    float2 fc[3][MH];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // fold of this half, then the radix-2 stage across the two halves:
      // h = 0 keeps own + recv, h = 1 (recv - own) W_MZ^jj
#pragma unroll
      for (int jj = 0; jj < MH; ++jj) {
        const int j = h * MH + jj;
        fc[c][jj] = fold_c(col[(c * ZR + j) * RS], col[(c * ZR + j + MZ) * RS], cr, twz[r * j]);
      }
#pragma unroll
      for (int jj = 0; jj < MH; ++jj) {
        const float2 own = fc[c][jj];
        const float2 recv = lane_x1(own);
        const float2 d = make_float2(fmaf(sg, own.x, recv.x), fmaf(sg, own.y, recv.y));
        fc[c][jj] = jj == 0 ? d : twh<MZ, false>(d, jj, hf);
      }
      reg_dft<MH, false>(fc[c], tw32);
      asm volatile("" ::: "memory");
    }
    // fc[c][p] = X_r[2 brev(p) + h]
#pragma unroll
    for (int p = 0; p < MH; ++p) {
      kernel_mul_lds<PY, PZ>(Ks, ky, 4 * (2 * brevc(p, lgMH) + h) + r, fc[0][p], fc[1][p], fc[2][p]);
      asm volatile("" ::: "memory");
    }
    const int zb = h * MH;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float2 g[MH];
#pragma unroll
      for (int k = 0; k < MH; ++k) g[k] = fc[c][brevc(k, lgMH)];
      reg_dft<MH, true>(g, tw32);
      // recombine the halves: x[z'] = g0 + W^{-z'} g1, x[z' + MH] = g0 - W^{-z'} g1
      // (selects here: the arithmetic form needs registers this kernel does
      // not have at four wavefronts per SIMD)
      float2 w[MH];
#pragma unroll
      for (int zz = 0; zz < MH; ++zz) {
        const float2 own = g[brevc(zz, lgMH)];
        const float2 t1 = twc<MZ, true>(own, zz);
        const float2 recv = lane_x1(h ? t1 : own);
        const float2 x = h ? csub(recv, t1) : cadd(own, recv);
        w[zz] = cmul(x, twid<true>(twz, r * (zb + zz)));
      }
      float2 o[MH / 2];
      quad_inverse8<MH>(w, r, o);
      const int z0 = zb + (MH / 2) * (r >> 1) + MZ * (r & 1);
#pragma unroll
      for (int i = 0; i < MH / 2; ++i)
        if (z0 + i < nz) B[(c * ZR + z0 + i) * RS + ky] = o[i];
      asm volatile("" ::: "memory");
    }
  }
  __syncthreads();
  // inverse y, four residue lanes per row
#pragma unroll 1
  for (int t = threadIdx.x; t < 4 * 3 * ZR; t += MM_YZ8_T) {
    const int r = t & 3;
    float2* line = B + (t >> 2) * RS;
    float2 g[MY];
#pragma unroll
    for (int k = 0; k < MY; ++k) g[k] = line[4 * k + r];
    reg_dft<MY, true>(g, tw32);
    float2 v[MY];
#pragma unroll
    for (int y0 = 0; y0 < MY; ++y0) v[y0] = cmul(g[brevc(y0, lgMY)], twid<true>(twy, r * y0));
    float2 o[MY / 2];
    quad_inverse<MY>(v, r, o);
    const int y0 = (MY / 2) * (r >> 1) + MY * (r & 1);
#pragma unroll
    for (int i = 0; i < MY / 2; ++i) line[y0 + i] = o[i];
  }
  __syncthreads();
#pragma unroll 4
  for (int e = threadIdx.x; e < 3 * ZR * YR; e += MM_YZ8_T) {
    const int row = e >> (lgMY + 1), y = e & (YR - 1);
    const int c = row / ZR, z = row & (ZR - 1);
    if (z < nz && y < ny) gst2(X + (c * nz + z) * ny + y, B[row * RS + y]);
  }
}

// ------------------------- fused y-z, two register passes per line (T = 512)
// A padded line of length P = L Q whose inputs vanish from P/2 on is
// transformed by L lanes.  With n = L n1 + lam and k = k1 + Q k2,
//   X[k1 + Q k2] = sum_lam W_L^{lam k2} W_P^{lam k1} sum_{n1 < Q/2} x[L n1 + lam] W_Q^{n1 k1}:
// lane lam takes the Q-point DFT of its own decimated sequence (whose upper
// half is zero) and scales it by W_P^{lam k1}; after an exchange through LDS
// lane mu takes the L-point DFTs of k1 = mu + L j, j < Q/L.  The inverse
// runs the same factorisation backwards with n = n1 + L n2: L-point inverse
// DFTs over k2 for each k1 of the lane, the conjugate scale W_P^{-n1 k1},
// exchange, and the Q-point inverse DFTs of which only the outputs n2 < Q/2
// (n < P/2, the cropped half) are formed.  All lanes of a line sit in one
// wavefront, whose LDS accesses complete in program order, so the exchange
// needs no workgroup barrier; the line's own LDS storage is the exchange
// area (a y row holds P slots, a z column of the three components 3P/2).
// One workgroup per (instance, kx):
//   load X -> LDS rows [3][Pz/2][Py + pad];  forward y per row (in place);
//   per ky column: forward z of the three components, kernel multiply,
//   inverse z (in place);  inverse y per row (in place);  store X.
#define MM_YZX_T 512
static_assert(MM_YZX_T == MMI_WG, "the finalisation body in the extra workgroups assumes MMI_WG threads");

// points per lane Q and lanes per line L of a padded length P (Q >= L):
// y rows take up to sixteen points per lane, z columns eight
template <int P, int QMAX>
struct LinePass {
  static constexpr int Q = P / 2 < QMAX ? P / 2 : QMAX, L = P / Q;
  static constexpr int lgQ = ilog2c(Q), lgL = ilog2c(L);
  static_assert(Q >= L && L >= 2, "unsupported padded length");
};

// radix-2 DIF stages h = H0 .. 1 of an in-register M-point DFT (M <= 16):
// natural order in, bit-reversed out when H0 = M/2
template <int M, bool INV, int H0>
__device__ __forceinline__ void dif_stages(float2 (&v)[M]) {
#pragma unroll
  for (int h = H0; h >= 1; h >>= 1) {
#pragma unroll
    for (int g = 0; g < M; g += 2 * h) {
#pragma unroll
      for (int i = 0; i < h; ++i) {
        const float2 a = v[g + i], b = v[g + i + h];
        v[g + i] = cadd(a, b);
        v[g + i + h] = twc<M, INV>(csub(a, b), i * (M / (2 * h)));
      }
    }
  }
}
// the same DFT of a sequence whose entries M/2 .. M-1 are zero (not read):
// the first stage has nothing to add and only scales
template <int M, bool INV>
__device__ __forceinline__ void dif_half(float2 (&v)[M]) {
#pragma unroll
  for (int i = 0; i < M / 2; ++i) v[i + M / 2] = twc<M, INV>(v[i], i);
  if constexpr (M >= 4) dif_stages<M, INV, M / 4>(v);
}

// exchange slot of value k1 from / for lane a: groups of L slots, rotated by
// k1 so that a write of fixed k1 and a read of fixed a both spread over L
// groups (and so over LDS banks)
template <int L>
__device__ __forceinline__ int xslot(int k1, int a) {
  return k1 * L + ((a + k1) & (L - 1));
}

// order the wavefront's LDS accesses across lanes (no instruction: a
// wavefront's LDS operations already complete in issue order)
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// The y transforms of one row held in LDS by N lanes (lane lam).  Forward:
// inputs at slots [0, P/2), afterwards slot k holds X[k].  Inverse: slot k
// holds X[k], afterwards slots [0, P/2) hold the inverse transform (no 1/P).
// wf[k1] = W_P^{lam k1}; wv[j][n1] = W_P^{-n1 (lam + N j)}.
template <int P>
struct YRow {
  using LP = LinePass<P, 16>;
  static constexpr int Q = LP::Q, N = LP::L;
  struct Tw {
    float2 wf[Q], wv[Q / N][N];
  };
  __device__ static void twiddles(Tw& w, const float2* tw, int lam) {
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) w.wf[k1] = tw[lam * k1];
#pragma unroll
    for (int j = 0; j < Q / N; ++j)
#pragma unroll
      for (int n1 = 0; n1 < N; ++n1) w.wv[j][n1] = conjf2(j == 0 ? w.wf[n1] : tw[n1 * (lam + N * j)]);
  }
  __device__ static void forward(float2* line, int lam, const Tw& w) {
    float2 v[Q];
#pragma unroll
    for (int n1 = 0; n1 < Q / 2; ++n1) v[n1] = line[N * n1 + lam];
    dif_half<Q, false>(v);
    wave_lds_order();
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      const int k1 = brevc(p, LP::lgQ);
      line[xslot<N>(k1, lam)] = k1 ? cmul(v[p], w.wf[k1]) : v[p];
    }
    wave_lds_order();
    float2 u[Q / N][N];
#pragma unroll
    for (int j = 0; j < Q / N; ++j) {
#pragma unroll
      for (int a = 0; a < N; ++a) u[j][a] = line[xslot<N>(lam + N * j, a)];
      dif_stages<N, false, N / 2>(u[j]);
    }
    wave_lds_order();
#pragma unroll
    for (int j = 0; j < Q / N; ++j)
#pragma unroll
      for (int p = 0; p < N; ++p) line[lam + N * j + Q * brevc(p, LP::lgL)] = u[j][p];
  }
  // Two real rows A, B transformed as one row A + iB: afterwards slot
  // SM::of(0, k) holds A[k] = (X[k] + conj X[P-k]) / 2 and SM::of(1, k) holds
  // B[k] = (X[k] - conj X[P-k]) / 2i for k < P/2, except that the real values
  // at k = 0 and P/2 share the slots of k = 0: (A[0], A[P/2]) and (B[0], B[P/2]).
  template <class SM>
  __device__ static void split_pair(float2* line, int lam) {
    constexpr int H = P / 2, NI = H / N;
    float2 r[NI], q[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int k = lam + N * i;
      r[i] = line[k];
      q[i] = line[k == 0 ? H : P - k];
    }
    wave_lds_order();
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int k = lam + N * i;
      const bool z = k == 0;
      line[SM::of(0, k)] = z ? make_float2(r[i].x, q[i].x) : make_float2(0.5f * (r[i].x + q[i].x), 0.5f * (r[i].y - q[i].y));
      line[SM::of(1, k)] = z ? make_float2(r[i].y, q[i].y) : make_float2(0.5f * (r[i].y + q[i].y), 0.5f * (q[i].x - r[i].x));
    }
  }
  // The inverse's input at k = k1 + Q k2 from two half spectra laid out as
  // split_pair leaves them (both of real rows, so X[P-k] = conj X[k]):
  // A[k] + i B[k], whose inverse has A's row as real and B's as imaginary part.
  template <class SM>
  __device__ static float2 pair_value(const float2* line, int k1, int k2) {
    constexpr int H = P / 2;
    if (k2 < N / 2) {                            // k < P/2
      const int k = k1 + Q * k2;
      const float2 a = line[SM::of(0, k)], b = line[SM::of(1, k)];
      return k == 0 ? make_float2(a.x, b.x) : make_float2(a.x - b.y, a.y + b.x);
    }
    const int m = P - (k1 + Q * k2);             // 1 .. P/2
    const int i = m == H ? 0 : m;
    const float2 a = line[SM::of(0, i)], b = line[SM::of(1, i)];
    return m == H ? make_float2(a.y, b.y) : make_float2(a.x + b.y, b.x - a.y);
  }
  // SM = void: a plain row; else two half spectra (split_pair's layout)
  template <class SM = void>
  __device__ static void inverse(float2* line, int lam, const Tw& w) {
    float2 g[Q / N][N];
#pragma unroll
    for (int j = 0; j < Q / N; ++j) {
#pragma unroll
      for (int k2 = 0; k2 < N; ++k2) {
        if constexpr (std::is_void_v<SM>) g[j][k2] = line[lam + N * j + Q * k2];
        else g[j][k2] = pair_value<SM>(line, lam + N * j, k2);
      }
      dif_stages<N, true, N / 2>(g[j]);
    }
    wave_lds_order();
#pragma unroll
    for (int j = 0; j < Q / N; ++j)
#pragma unroll
      for (int n1 = 0; n1 < N; ++n1) {
        const float2 zv = g[j][brevc(n1, LP::lgL)];
        line[xslot<N>(lam + N * j, n1)] = n1 == 0 ? zv : cmul(zv, w.wv[j][n1]);
      }
    wave_lds_order();
    float2 v[Q];
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) v[k1] = line[xslot<N>(k1, lam)];
    dif_stages<Q, true, Q / 2>(v);
    wave_lds_order();
#pragma unroll
    for (int n2 = 0; n2 < Q / 2; ++n2) line[lam + N * n2] = v[brevc(n2, LP::lgQ)];
  }
};

// The z convolution of one column held in LDS by N lanes (lane lam): the
// three components at rows c ZR + z (stride RS, ZR = P/2; rows nz .. ZR-1
// zero), forward z, the kernel multiply kmul(kz, x, y, z) at every kz, the
// inverse z; rows z < nz receive the result.  The column's 3 ZR slots serve
// as the exchange area once its inputs are in registers.
template <int P>
struct ZCol {
  using LP = LinePass<P, 8>;
  static constexpr int Q = LP::Q, N = LP::L, ZR = P / 2;
  struct Tw {
    float2 wf[Q], wv[Q / N][N];
  };
  __device__ static void twiddles(Tw& w, const float2* tw, int lam) {
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) w.wf[k1] = tw[lam * k1];
#pragma unroll
    for (int j = 0; j < Q / N; ++j)
#pragma unroll
      for (int n1 = 0; n1 < N; ++n1) w.wv[j][n1] = conjf2(j == 0 ? w.wf[n1] : tw[n1 * (lam + N * j)]);
  }
  using Spec = float2[3][Q / N][N];
  // frequency of sp[c][j][p] after forward(): k1 + Q brev(p), k1 = lam + N j
  __device__ static int kz_of(int lam, int j, int p) { return lam + N * j + Q * brevc(p, LP::lgL); }
  __device__ static void forward(float2* col, int RS, int lam, const Tw& w, Spec& sp) {
    float2 xin[3][Q / 2];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int n1 = 0; n1 < Q / 2; ++n1) xin[c][n1] = col[(c * ZR + N * n1 + lam) * RS];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float2 v[Q];
#pragma unroll
      for (int n1 = 0; n1 < Q / 2; ++n1) v[n1] = xin[c][n1];
      dif_half<Q, false>(v);
      wave_lds_order();
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        const int k1 = brevc(p, LP::lgQ);
        col[xslot<N>(k1, lam) * RS] = k1 ? cmul(v[p], w.wf[k1]) : v[p];
      }
      wave_lds_order();
#pragma unroll
      for (int j = 0; j < Q / N; ++j) {
#pragma unroll
        for (int a = 0; a < N; ++a) sp[c][j][a] = col[xslot<N>(lam + N * j, a) * RS];
        dif_stages<N, false, N / 2>(sp[c][j]);
      }
      wave_lds_order();
    }
  }
  // inverse z of sp (the column's slots are the exchange area); rows z < nz
  // receive the result
  __device__ static void inverse(float2* col, int RS, int nz, int lam, const Tw& w, Spec& sp) {
    float2 res[3][Q / 2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int j = 0; j < Q / N; ++j) {
        float2 g[N];
#pragma unroll
        for (int k2 = 0; k2 < N; ++k2) g[k2] = sp[c][j][brevc(k2, LP::lgL)];
        dif_stages<N, true, N / 2>(g);
        // g[p] = sum_k2 X[k1 + Q k2] W_N^{-n1 k2} at n1 = brev(p)
#pragma unroll
        for (int n1 = 0; n1 < N; ++n1) {
          const float2 zv = g[brevc(n1, LP::lgL)];
          col[xslot<N>(lam + N * j, n1) * RS] = n1 == 0 ? zv : cmul(zv, w.wv[j][n1]);
        }
      }
      wave_lds_order();
      float2 v[Q];
#pragma unroll
      for (int k1 = 0; k1 < Q; ++k1) v[k1] = col[xslot<N>(k1, lam) * RS];
      dif_stages<Q, true, Q / 2>(v);
#pragma unroll
      for (int n2 = 0; n2 < Q / 2; ++n2) res[c][n2] = v[brevc(n2, LP::lgQ)];
      wave_lds_order();
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int n2 = 0; n2 < Q / 2; ++n2) {
        const int z = lam + N * n2;
        if (z < nz) col[(c * ZR + z) * RS] = res[c][n2];
      }
  }
  template <class KMul>
  __device__ static void convolve(float2* col, int RS, int nz, int lam, const Tw& w, KMul&& kmul) {
    Spec sp;
    forward(col, RS, lam, w, sp);
#pragma unroll
    for (int j = 0; j < Q / N; ++j)
#pragma unroll
      for (int p = 0; p < N; ++p) kmul(kz_of(lam, j, p), sp[0][j][p], sp[1][j][p], sp[2][j][p]);
    inverse(col, RS, nz, lam, w, sp);
  }
};

// LDS bank layout shared by the kernels below (64 banks of four bytes; an
// eight-byte access is served 32 lanes per cycle).  Rows are an odd number of
// slots apart.  A y row has N lanes, lane = lam * RPW + r in its wavefront
// (RPW = 64 / N rows), and the wavefront's rows are SY = N / 2 apart, so the
// 32 lanes of a half-wavefront (N / 2 values of lam, RPW rows) fall on
// distinct bank pairs; the rows of SY wavefronts interleave to fill blocks of
// 32 rows.  A z column has N consecutive lanes and the wavefront's columns
// are SZ apart (SZ = N where the tile is wide enough), for the same reason.
// Row of y-lane yrl in block g0 of wavefront `wave`:
template <int N>
__device__ __forceinline__ int yrow_of(int g0, int wave, int yrl) {
  constexpr int SY = N / 2;
  return 32 * g0 + wave % SY + SY * yrl;
}
// Column of thread t in a tile of NCOL columns, N lanes per column:
template <int N, int NCOL>
__device__ __forceinline__ int zcol_of(int t) {
  constexpr int CPW = 64 / N, SZ = N < NCOL / CPW ? N : NCOL / CPW;
  const int wz = t >> 6;
  return wz % SZ + SZ * ((t & 63) / N) + SZ * CPW * (wz / SZ);
}

// Planes kx = 0 and kx = Px/2 of the x transform of real rows are real, and
// in them the tensor components odd in x (xy, xz) vanish, so each plane's y-z
// convolution is real as well.  Where one column per thread covers the padded
// y range (Py NZ = MM_YZX_T), work item 0 of an instance carries both planes,
// as A + iB through the forward y pass, which YRow::split_pair turns into the
// two half spectra (ky <= Py/2 of each; the real columns ky = 0 and Py/2 of a
// plane share one slot).  The z columns are then the columns of the two half
// spectra, placed so that plane 0's fall in the first half of the
// workgroup's wavefronts and plane Px/2's in the second: the first half
// multiplies with the kernel of plane 0, then the second with that of plane
// Px/2.  A shared column holds U + iV of two real columns U (ky = 0) and V
// (ky = Py/2), whose spectra it separates as U[kz] = (Z[kz] + conj Z[-kz]) / 2
// and V[kz] = (Z[kz] - conj Z[-kz]) / 2i, from a copy in LDS worked on by the
// idle half.  The inverse y transforms A + iB rebuilt from the half spectra,
// and the real and imaginary parts go back to the two planes.  An instance
// then has Px/2 work items instead of Px/2 + 1.
template <int PY, int PZ>
struct YzxPairs {
  static constexpr int NZ = ZCol<PZ>::N, NW = MM_YZX_T / 64;
  static constexpr bool on = PY * NZ == MM_YZX_T;
  // zcol_of<NZ, PY> gives wavefront w the columns s with s mod SZ = w mod SZ
  // and s / (SZ CPW) = w / SZ.  Slot of half-spectrum column k of plane hi
  // (0: plane 0, 1: plane Px/2) such that plane 0's columns fall in
  // wavefronts 0 .. NW/2 - 1 and plane Px/2's in the others:
  static constexpr int CPW = 64 / NZ, SZ = NZ < PY / CPW ? NZ : PY / CPW;
  static_assert(!on || SZ == NW || (2 * SZ == NW && SZ * CPW == PY / 2), "column layout");
  __device__ static int of(int hi, int k) {
    if constexpr (SZ == NW) return k % (SZ / 2) + SZ * (k / (SZ / 2)) + hi * (SZ / 2);
    else return k + hi * (PY / 2);
  }
  __device__ static int ky_of(int s) {
    if constexpr (SZ == NW) return s % (SZ / 2) + (SZ / 2) * (s / SZ);
    else return s & (PY / 2 - 1);
  }
};

template <int MY, int MZ, int RPAD, bool PAIR>
__device__ __forceinline__ void yzx_item(const InstDesc& D, int kx, const float2* __restrict__ tw, float2* lds) {
  constexpr int PY = 4 * MY, PZ = 4 * MZ, RS = PY + RPAD, ZR = 2 * MZ, YR = 2 * MY;
  using YR_ = YRow<PY>;
  using ZC = ZCol<PZ>;
  constexpr int NY = YR_::N, NZ = ZC::N;
  constexpr int lgPY = ilog2c(PY);
  constexpr int RPW = 64 / NY;                  // y rows per wavefront
  constexpr int NW = MM_YZX_T / 64;             // wavefronts per workgroup
  constexpr int SY = NY / 2;
  static_assert(!PAIR || YzxPairs<PY, PZ>::on, "paired planes need one z column per thread");
  float2* B = lds;
  float2* twy = B + 3 * ZR * RS;
  float2* twz = twy + PY;
  float* Ks = reinterpret_cast<float*>(twz + PZ);
  constexpr int HY1 = PY / 2 + 1, KPL = (PZ / 2 + 1) * HY1;
  float2* Pk = reinterpret_cast<float2*>(Ks + 6 * KPL);   // PAIR: copies of the two shared columns' spectra
  constexpr int NK = (6 * KPL + MM_YZX_T - 1) / MM_YZX_T, NXE = 3 * ZR * PY;
  constexpr int NX = (NXE + MM_YZX_T - 1) / MM_YZX_T;
  load_twiddles(twy, PY, tw, MM_YZX_T);
  load_twiddles(twz, PZ, tw, MM_YZX_T);
  const int ny = D.ny, nz = D.nz;
  const int nrow = 3 * nz;
  MMG float2* X = gbl(D.fx) + (size_t)kx * nrow * ny;
  MMG float2* X2 = gbl(D.fx) + (size_t)(D.kx - 1) * nrow * ny;   // PAIR: plane Px/2
  // Loads: thread t takes column y = t mod Py of rows it * RPI + t / Py.  The
  // row's (c, z) and the X offset (c nz + z) ny + y are a per-thread part
  // plus a part uniform over the workgroup, so each element costs a compare,
  // a select and an add.
  constexpr int RPI = MM_YZX_T / PY;            // rows per iteration
  {
    const MMG float* K = gbl(D.kern) + (size_t)kx * 6 * KPL;
    float kv[NK];
    float2 xv[NX];
#pragma unroll
    for (int it = 0; it < NK; ++it) kv[it] = K[min(it * MM_YZX_T + (int)threadIdx.x, 6 * KPL - 1)];
    const int y = threadIdx.x & (PY - 1), r0 = threadIdx.x >> lgPY;
    const bool yin = y < ny;
    const int tb = r0 * ny + y;
#pragma unroll
    for (int it = 0; it < NX; ++it) {
      const int row = it * RPI + r0;
      // when the rows of an iteration stay within a component, c and the
      // first z are compile-time and z = z0 + r0
      const int c = (ZR % RPI == 0) ? (it * RPI) / ZR : row / ZR;
      const int z = (ZR % RPI == 0) ? (it * RPI) % ZR + r0 : row % ZR;
      const bool in = row < 3 * ZR && yin && z < nz;
      const int off = (ZR % RPI == 0) ? (c * nz + (it * RPI) % ZR) * ny + tb : (c * nz + z) * ny + y;
      float2 v = gld2(X + (in ? off : 0));
      if constexpr (PAIR) v = make_float2(v.x, gld2(X2 + (in ? off : 0)).x);
      xv[it] = make_float2(in ? v.x : 0.f, in ? v.y : 0.f);
    }
#pragma unroll
    for (int it = 0; it < NK; ++it) {
      const int e = it * MM_YZX_T + threadIdx.x;
      if (e < 6 * KPL) Ks[e] = kv[it];
    }
#pragma unroll
    for (int it = 0; it < NX; ++it) {
      const int row = it * RPI + r0, z = row % ZR;
      if (row < 3 * ZR && (z >= nz || y < YR)) B[row * RS + y] = xv[it];
    }
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ylam = lane / RPW, yrl = lane % RPW;
  typename YR_::Tw wy;
  YR_::twiddles(wy, twy, ylam);
  // forward y of the rows z < nz (rows z >= nz stay zero)
#pragma unroll 1
  for (int g0 = wave / SY; 32 * g0 < 3 * ZR; g0 += NW / SY) {
    const int rho = yrow_of<NY>(g0, wave, yrl);
    if (rho < 3 * ZR && (rho & (ZR - 1)) < nz) {
      YR_::forward(B + rho * RS, ylam, wy);
      if constexpr (PAIR) YR_::template split_pair<YzxPairs<PY, PZ>>(B + rho * RS, ylam);
    }
  }
  __syncthreads();
  // z columns
  {
    const int lam = threadIdx.x & (NZ - 1);
    typename ZC::Tw wz;
    ZC::twiddles(wz, twz, lam);
    if constexpr (!PAIR) {
#pragma unroll 1
      for (int t = threadIdx.x; t < NZ * PY; t += MM_YZX_T) {
        const int ky = zcol_of<NZ, PY>(t);
        ZC::convolve(B + ky, RS, nz, lam, wz, [&](int kz, float2& a, float2& b, float2& c) {
          kernel_mul_lds<PY, PZ>(Ks, ky, kz, a, b, c);
        });
      }
    } else {
      // the kernel of plane Px/2, for the second half of the multiply (its
      // loads complete during the forward z)
      float kv2[NK];
      {
        const MMG float* K2 = gbl(D.kern) + (size_t)(D.kx - 1) * 6 * KPL;
#pragma unroll
        for (int it = 0; it < NK; ++it) kv2[it] = K2[min(it * MM_YZX_T + (int)threadIdx.x, 6 * KPL - 1)];
      }
      using PS = YzxPairs<PY, PZ>;
      const int s = zcol_of<NZ, PY>(threadIdx.x);
      const bool hi = wave >= NW / 2;           // columns of plane Px/2 (uniform per wavefront)
      const int ky = PS::ky_of(s);
      const bool shared = ky == 0;              // the column of ky = 0 and Py/2
      typename ZC::Spec sp;
      ZC::forward(B + s, RS, lam, wz, sp);
      if (shared) {
        float2* pk = Pk + (hi ? 3 * PZ : 0);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int j = 0; j < ZC::Q / NZ; ++j)
#pragma unroll
            for (int p = 0; p < NZ; ++p) pk[c * PZ + ZC::kz_of(lam, j, p)] = sp[c][j][p];
      }
      __syncthreads();
      // Multiply with the kernel in Ks: one half of the workgroup multiplies
      // its columns while lanes kz < Pz of the other half (one wavefront) do
      // the shared column of the same plane on its copy, each forming U[kz]
      // and V[kz] from Z[kz] and Z[-kz].
      auto columns = [&]() {
        if (shared) return;
#pragma unroll
        for (int j = 0; j < ZC::Q / NZ; ++j)
#pragma unroll
          for (int p = 0; p < NZ; ++p)
            kernel_mul_lds<PY, PZ>(Ks, ky, ZC::kz_of(lam, j, p), sp[0][j][p], sp[1][j][p], sp[2][j][p]);
      };
      auto shared_col = [&](float2* pk) {
        const int kz = threadIdx.x & (MM_YZX_T / 2 - 1);
        if (kz >= PZ) return;
        const int mz = (PZ - kz) & (PZ - 1);
        float2 u[3], v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float2 zk = pk[c * PZ + kz], zm = pk[c * PZ + mz];
          u[c] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
          v[c] = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
        }
        wave_lds_order();                       // all of the copy read before it is overwritten
        kernel_mul_lds<PY, PZ>(Ks, 0, kz, u[0], u[1], u[2]);
        kernel_mul_lds<PY, PZ>(Ks, PY / 2, kz, v[0], v[1], v[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) pk[c * PZ + kz] = make_float2(u[c].x - v[c].y, u[c].y + v[c].x);
      };
      auto read_back = [&](const float2* pk) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int j = 0; j < ZC::Q / NZ; ++j)
#pragma unroll
            for (int p = 0; p < NZ; ++p) sp[c][j][p] = pk[c * PZ + ZC::kz_of(lam, j, p)];
      };
      if (!hi) columns(); else shared_col(Pk);                   // kernel of plane 0
      __syncthreads();
      if (!hi && shared) read_back(Pk);
      // the kernel of plane Px/2 replaces it
#pragma unroll
      for (int it = 0; it < NK; ++it) {
        const int e = it * MM_YZX_T + threadIdx.x;
        if (e < 6 * KPL) Ks[e] = kv2[it];
      }
      __syncthreads();
      if (hi) columns(); else shared_col(Pk + 3 * PZ);
      __syncthreads();
      if (hi && shared) read_back(Pk + 3 * PZ);
      ZC::inverse(B + s, RS, nz, lam, wz, sp);
    }
  }
  __syncthreads();
  // inverse y of the rows z < nz, cropped to y < Py/2 (the paired path takes
  // its y twiddles again here: keeping them, or their LDS addresses, through
  // its z pass spills; the empty asm makes the lane index opaque)
  if constexpr (PAIR) {
    int yl = ylam;
    asm volatile("" : "+v"(yl));
    YR_::twiddles(wy, twy, yl);
  }
#pragma unroll 1
  for (int g0 = wave / SY; 32 * g0 < 3 * ZR; g0 += NW / SY) {
    const int rho = yrow_of<NY>(g0, wave, yrl);
    if (rho < 3 * ZR && (rho & (ZR - 1)) < nz)
      YR_::template inverse<std::conditional_t<PAIR, YzxPairs<PY, PZ>, void>>(B + rho * RS, ylam, wy);
  }
  __syncthreads();
  {
    // stores: thread t takes column y = t mod (Py/2) of rows it * RPO + t / (Py/2)
    constexpr int RPO = MM_YZX_T / YR, NO = (3 * ZR + RPO - 1) / RPO;
    const int y = threadIdx.x & (YR - 1), r0 = threadIdx.x / YR;
    const bool yin = y < ny;
    const int tb = r0 * ny + y;
#pragma unroll
    for (int it = 0; it < NO; ++it) {
      const int row = it * RPO + r0;
      const int c = (ZR % RPO == 0) ? (it * RPO) / ZR : row / ZR;
      const int z = (ZR % RPO == 0) ? (it * RPO) % ZR + r0 : row % ZR;
      const int off = (ZR % RPO == 0) ? (c * nz + (it * RPO) % ZR) * ny + tb : (c * nz + z) * ny + y;
      if (row < 3 * ZR && z < nz && yin) {
        const float2 v = B[row * RS + y];
        if constexpr (PAIR) {
          gst2(X + off, make_float2(v.x, 0.f));
          gst2(X2 + off, make_float2(v.y, 0.f));
        } else {
          gst2(X + off, v);
        }
      }
    }
  }
}

template <int MY, int MZ, int RPAD>
__global__ __launch_bounds__(MM_YZX_T) __attribute__((amdgpu_waves_per_eu(MY >= 32 ? 2 : 4, MY >= 32 ? 2 : 4))) void k_fft_yzx(
    const InstDesc* __restrict__ descs, const WorkItem* __restrict__ work, const float2* __restrict__ tw,
    int nyz, int fmethod, int fstage) {
  extern __shared__ float2 lds[];
  if ((int)blockIdx.x >= nyz) {
    final_any(fmethod, fstage, descs, (int)blockIdx.x - nyz, reinterpret_cast<double*>(lds));
    return;
  }
  const WorkItem wi = work[blockIdx.x];
  const InstDesc& D = descs[wi.inst];
  if (gbl(D.ctl)->done) return;
  if constexpr (YzxPairs<4 * MY, 4 * MZ>::on) {
    if (wi.item == 0 && D.kx > 1) {
      yzx_item<MY, MZ, RPAD, true>(D, 0, tw, lds);
      return;
    }
  }
  yzx_item<MY, MZ, RPAD, false>(D, wi.item, tw, lds);
}

// ------------------------ split y passes with the same line transforms (T = 512)
// For padded y planes too large for one workgroup's LDS: the y passes over
// rows (kx, c, z < nz) between X[kx][c][z][y < ny] and Y[kx][c][z][ky < Py]
// (the z pass with the kernel multiply is k_fft_zc, over tiles of ky columns).
#define MM_SX_T 512

// rows per workgroup of the split y pass
template <int PY>
struct SplitY {
  static constexpr int N = YRow<PY>::N, ROWS = 32 * (MM_SX_T / 64) / (N / 2), RS = PY + 1;
};

// Workgroups nwork .. nwork + nfinal - 1 of a forward launch run the
// finalisation of stage fstage instead (as in k_fft_yzx: the y pass reads
// and writes only X and Y, which the finalisation does not touch).
static_assert(MM_SX_T == MMI_WG, "the finalisation body in the extra workgroups assumes MMI_WG threads");
template <int PY, int DIR>
__global__ __launch_bounds__(MM_SX_T) void k_fft_ysx(const InstDesc* __restrict__ descs,
                                                    const WorkItem* __restrict__ work,
                                                    const float2* __restrict__ tw, int nwork,
                                                    int fmethod, int fstage) {
  using YR_ = YRow<PY>;
  using S = SplitY<PY>;
  constexpr int N = S::N, RS = S::RS, ROWS = S::ROWS, RPW = 64 / N, SY = N / 2, NW = MM_SX_T / 64;
  constexpr int HP = PY / 2;
  extern __shared__ float2 lds[];
  if ((int)blockIdx.x >= nwork) {
    final_any(fmethod, fstage, descs, (int)blockIdx.x - nwork, reinterpret_cast<double*>(lds));
    return;
  }
  float2* B = lds;
  float2* twy = B + ROWS * RS;
  load_twiddles(twy, PY, tw, MM_SX_T);
  const WorkItem wi = work[blockIdx.x];
  const InstDesc& D = descs[wi.inst];
  if (gbl(D.ctl)->done) return;
  const int ny = D.ny, nlines = D.kx * 3 * D.nz;
  const int l0 = wi.item * ROWS;
  const int nr = min(ROWS, nlines - l0);
  MMG float2* X = gbl(D.fx) + (size_t)l0 * ny;
  MMG float2* Y = gbl(D.fy) + (size_t)l0 * PY;
  if (DIR < 0) {
    for (int e = threadIdx.x; e < ROWS * HP; e += MM_SX_T) {
      const int r = e / HP, y = e - r * HP;
      float2 v = make_float2(0.f, 0.f);
      if (r < nr && y < ny) v = gld2(X + (size_t)r * ny + y);
      B[r * RS + y] = v;
    }
  } else {
    for (int e = threadIdx.x; e < ROWS * PY; e += MM_SX_T) {
      const int r = e / PY, y = e - r * PY;
      if (r < nr) B[r * RS + y] = gld2(Y + (size_t)r * PY + y);
    }
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ylam = lane / RPW, yrl = lane % RPW;
  typename YR_::Tw w;
  YR_::twiddles(w, twy, ylam);
#pragma unroll 1
  for (int g0 = wave / SY; 32 * g0 < ROWS; g0 += NW / SY) {
    const int r = yrow_of<N>(g0, wave, yrl);
    if (r < nr) {
      if (DIR < 0) YR_::forward(B + r * RS, ylam, w);
      else YR_::inverse(B + r * RS, ylam, w);
    }
  }
  __syncthreads();
  if (DIR < 0) {
    for (int e = threadIdx.x; e < ROWS * PY; e += MM_SX_T) {
      const int r = e / PY, y = e - r * PY;
      if (r < nr) gst2(Y + (size_t)r * PY + y, B[r * RS + y]);
    }
  } else {
    for (int e = threadIdx.x; e < ROWS * HP; e += MM_SX_T) {
      const int r = e / HP, y = e - r * HP;
      if (r < nr && y < ny) gst2(X + (size_t)r * ny + y, B[r * RS + y]);
    }
  }
}

// --------------------------------------------------- x passes, lines in registers
// Work item = 128 consecutive real rows (64 complex lines) of one instance.
// A line packs two real rows (real and imaginary part) and is split over four
// adjacent lanes by frequency residue, as in the fused y-z kernel above.
#define MM_XR_T 256
#define MM_XR_ROWS 128

// forward: rows of the stage input -> X[kx][row] for kx <= Px/2
template <int MX>
__global__ __launch_bounds__(MM_XR_T) void k_fft_xfr(const InstDesc* __restrict__ descs,
                                                     const WorkItem* __restrict__ work, int method,
                                                     int stage, const float2* __restrict__ tw) {
  constexpr int PX = 4 * MX, NXP = 2 * MX, RSX = NXP + 1, lgM = ilog2c(MX), lgN = lgM + 1;
  __shared__ float rowbuf[MM_XR_ROWS * RSX];
  __shared__ float2 twx[PX + 32];
  const WorkItem wi = work[blockIdx.x];
  const InstDesc& D = descs[wi.inst];
  const MMG InstCtl* __restrict__ C = gbl(D.ctl);
  if (C->done) return;
  const int nx = D.nx, rows = 3 * D.ny * D.nz;
  const int r0 = wi.item * MM_XR_ROWS;
  const Src src = stage_src(D, C, method, stage);
  float2* tw32 = twx + PX;
  load_twiddles(twx, PX, tw, MM_XR_T);
  load_twiddles(tw32, 32, tw, MM_XR_T);
  {
    // rows are contiguous x-lines: element (row, x) of the stage input is at row * nx + x
    constexpr int NE = MM_XR_ROWS * NXP, NB = NE / MM_XR_T;
    float v[NB];
    int idx[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = u * MM_XR_T + threadIdx.x;
      const int rr = e >> lgN, x = e & (NXP - 1);
      idx[u] = min(r0 + rr, rows - 1) * nx + min(x, nx - 1);
      v[u] = src.p0[idx[u]];
    }
    if (src.p1) {
#pragma unroll
      for (int u = 0; u < NB; ++u) v[u] = fmaf(src.c1, src.p1[idx[u]], v[u]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = u * MM_XR_T + threadIdx.x;
      const int rr = e >> lgN, x = e & (NXP - 1);
      rowbuf[rr * RSX + x] = (x < nx && r0 + rr < rows) ? v[u] : 0.f;
    }
  }
  __syncthreads();
  const int l = threadIdx.x >> 2, r = threadIdx.x & 3;
  const float* ra = rowbuf + (2 * l) * RSX;
  const float* rb = ra + RSX;
  float2 f[MX];
#pragma unroll
  for (int j = 0; j < MX; ++j)
    f[j] = fold(make_float2(ra[j], rb[j]), make_float2(ra[j + MX], rb[j + MX]), r, twx[r * j]);
  reg_dft<MX, false>(f, tw32);
  // f[brev(k)] = Z[4k + r].  R2C split with the partner Z[Px - kx]: the same
  // lane for r = 0, 2, the lane r ^ 2 for r = 1, 3 (register of k' = MX-1-k).
  MMG float2* X = gbl(D.fx);
  const size_t kstride = (size_t)rows;
  const int ra_row = r0 + 2 * l;
#pragma unroll
  for (int k = 0; k <= MX / 2; ++k) {
    const float2 z = f[brevc(k % MX, lgM)];
    const float2 recv = quad_x2(f[brevc(MX - 1 - k < 0 ? 0 : MX - 1 - k, lgM)]);
    const float2 zm = r == 0 ? f[brevc((MX - k) % MX, lgM)] : r == 2 ? f[brevc(MX - 1 - k < 0 ? 0 : MX - 1 - k, lgM)] : recv;
    const int kx = 4 * k + r;
    if (kx <= NXP) {
      const float2 xa = make_float2(0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y));
      const float2 xb = make_float2(0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x));
      MMG float2* o = X + (size_t)kx * kstride + ra_row;
      if (ra_row < rows) gst2(o, xa);
      if (ra_row + 1 < rows) gst2(o + 1, xb);
    }
  }
}

// inverse: X[kx][row] -> B_d rows (crop x < nx, scale), C2R of two rows per line
template <int MX>
__global__ __launch_bounds__(MM_XR_T) void k_fft_xir(const InstDesc* __restrict__ descs,
                                                     const WorkItem* __restrict__ work,
                                                     const float2* __restrict__ tw) {
  constexpr int PX = 4 * MX, NXP = 2 * MX, RSX = NXP + 1, lgM = ilog2c(MX), lgN = lgM + 1;
  __shared__ float rowbuf[MM_XR_ROWS * RSX];
  __shared__ float2 twx[PX + 32];
  const WorkItem wi = work[blockIdx.x];
  const InstDesc& D = descs[wi.inst];
  if (gbl(D.ctl)->done) return;
  const int nx = D.nx, rows = 3 * D.ny * D.nz;
  const int r0 = wi.item * MM_XR_ROWS;
  float2* tw32 = twx + PX;
  load_twiddles(twx, PX, tw, MM_XR_T);
  load_twiddles(tw32, 32, tw, MM_XR_T);
  const int l = threadIdx.x >> 2, r = threadIdx.x & 3;
  const int ra_row = min(r0 + 2 * l, rows - 1), rb_row = min(r0 + 2 * l + 1, rows - 1);
  const bool b_in = r0 + 2 * l + 1 < rows;
  const MMG float2* X = gbl(D.fx);
  const size_t kstride = (size_t)rows;
  // Z[kx] = Xa[kx] + i Xb[kx] for kx <= Px/2, conj(Xa[Px-kx]) + i conj(Xb[Px-kx]) above
  float2 g[MX];
#pragma unroll
  for (int k = 0; k < MX; ++k) {
    const int kx = 4 * k + r;
    const bool lo = kx <= NXP;
    const int kk = lo ? kx : PX - kx;
    float2 a = gld2(X + (size_t)kk * kstride + ra_row);
    float2 b = gld2(X + (size_t)kk * kstride + rb_row);
    if (!b_in) b = make_float2(0.f, 0.f);
    if (kx == 0 || kx == NXP) { a.y = 0.f; b.y = 0.f; }
    g[k] = lo ? make_float2(a.x - b.y, a.y + b.x) : make_float2(a.x + b.y, b.x - a.y);
  }
  __syncthreads();   // twiddles
  reg_dft<MX, true>(g, tw32);
  float2 w[MX];
#pragma unroll
  for (int y0 = 0; y0 < MX; ++y0) w[y0] = cmul(g[brevc(y0, lgM)], twid<true>(twx, r * y0));
  float2 o[MX / 2];
  quad_inverse<MX>(w, r, o);
  const int x0 = (MX / 2) * (r >> 1) + MX * (r & 1);
  float* pa = rowbuf + (2 * l) * RSX;
#pragma unroll
  for (int i = 0; i < MX / 2; ++i) {
    pa[x0 + i] = o[i].x;
    pa[RSX + x0 + i] = o[i].y;
  }
  __syncthreads();
  const float sc = D.bd_scale;
  MMG float* bd = gbl(D.bd);
  constexpr int NE = MM_XR_ROWS * NXP;
#pragma unroll 4
  for (int e = threadIdx.x; e < NE; e += MM_XR_T) {
    const int rr = e >> lgN, x = e & (NXP - 1);
    if (x < nx && r0 + rr < rows) bd[(r0 + rr) * nx + x] = sc * rowbuf[rr * RSX + x];
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
  if (gbl(D.ctl)->done) return;
  const int ny = D.ny, Py = D.py;
  const int nlines = D.kx * 3 * D.nz;
  const int l0 = wi.item * W;
  const int WP = W + 1;                   // padded line stride (bank conflicts)
  float2* buf = lds;
  float2* twl = lds + Py * WP;
  load_twiddles(twl, Py, tw, 256);
  __syncthreads();   // the pruned forward stage below reads the table
  const int lgy = ilog2(Py), lgW = ilog2(W);
  if (DIR < 0) {
    // The inputs vanish for y >= ny, and ny <= Py/2: the first radix-2^2 DIF
    // stage (span Py/2) reads only x0 = x[y] and x1 = x[y + Py/4] and is done
    // here with the same arithmetic as the full stage (x2 = x3 = 0).
    const int q = Py >> 2;
    if (q == 0) {
      // lines of one or two points: no stage to skip
      for (int e = threadIdx.x; e < W * Py; e += 256) {
        const int ll = e >> lgy, y = e & (Py - 1);
        const int l = l0 + ll;
        float2 v = make_float2(0.f, 0.f);
        if (l < nlines && y < ny) v = gld2(gbl(D.fx) + (size_t)l * ny + y);
        buf[y * WP + ll] = v;
      }
    }
    for (int e = threadIdx.x; e < W * q; e += 256) {
      const int y = e & (q - 1), ll = e >> (lgy - 2);   // consecutive threads: consecutive y
      const int l = l0 + ll;
      const MMG float2* row = gbl(D.fx) + (size_t)min(l, nlines - 1) * ny;
      float2 x0 = gld2(row + min(y, ny - 1)), x1 = gld2(row + min(y + q, ny - 1));
      if (l >= nlines || y >= ny) x0 = make_float2(0.f, 0.f);
      if (l >= nlines || y + q >= ny) x1 = make_float2(0.f, 0.f);
      const float2 z = make_float2(0.f, 0.f);
      const float2 w1 = twl[y], w2 = twl[2 * y];
      const float2 a0 = cadd(x0, z), a1 = cadd(x1, z);
      const float2 a2 = cmul(csub(x0, z), w1);
      const float2 a3 = rot<false>(cmul(csub(x1, z), w1));
      buf[y * WP + ll] = cadd(a0, a1);
      buf[(y + q) * WP + ll] = cmul(csub(a0, a1), w2);
      buf[(y + 2 * q) * WP + ll] = cadd(a2, a3);
      buf[(y + 3 * q) * WP + ll] = cmul(csub(a2, a3), w2);
    }
    __syncthreads();
    fft_cols<256, false>(buf, Py, lgy, 1, lgW, 0, WP, twl, q == 0 ? 0 : 2);
    for (int e = threadIdx.x; e < W * Py; e += 256) {
      const int ll = e >> lgy, y = e & (Py - 1);
      const int l = l0 + ll;
      if (l < nlines) gst2(gbl(D.fy) + (size_t)l * Py + y, buf[brev(y, lgy) * WP + ll]);
    }
  } else {
    // bit-reversed order in, natural order out, cropped to y < ny
    for (int e = threadIdx.x; e < W * Py; e += 256) {
      const int ll = e >> lgy, y = e & (Py - 1);
      const int l = l0 + ll;
      float2 v = make_float2(0.f, 0.f);
      if (l < nlines) v = gld2(gbl(D.fy) + (size_t)l * Py + y);
      buf[brev(y, lgy) * WP + ll] = v;
    }
    __syncthreads();
    const int q = Py >> 2;
    if (q == 0) {
      fft_cols<256, true>(buf, Py, lgy, 1, lgW, 0, WP, twl);
      for (int e = threadIdx.x; e < W * Py; e += 256) {
        const int ll = e >> lgy, y = e & (Py - 1);
        const int l = l0 + ll;
        if (l < nlines && y < ny) gst2(gbl(D.fx) + (size_t)l * ny + y, buf[y * WP + ll]);
      }
    } else {
      // all DIT stages but the last radix-2^2 one (span Py/4); that one is
      // done here for the outputs y < Py/2 only (ny <= Py/2), with the same
      // arithmetic as the full stage
      fft_cols<256, true>(buf, Py, lgy, 1, lgW, 0, WP, twl, 0, lgy - 2);
      for (int e = threadIdx.x; e < W * q; e += 256) {
        const int i = e & (q - 1), ll = e >> (lgy - 2);
        const int l = l0 + ll;
        const float2* x = buf + i * WP + ll;
        const float2 wA = twid<true>(twl, i << 1), wB = twid<true>(twl, i);
        const float2 t1 = cmul(x[q * WP], wA), t3 = cmul(x[3 * q * WP], wA);
        const float2 a0 = cadd(x[0], t1), a1 = csub(x[0], t1), a2 = cadd(x[2 * q * WP], t3),
                     a3 = csub(x[2 * q * WP], t3);
        const float2 u = cmul(a2, wB), v = rot<true>(cmul(a3, wB));
        MMG float2* out = gbl(D.fx) + (size_t)l * ny;
        if (l < nlines && i < ny) gst2(out + i, cadd(a0, u));
        if (l < nlines && i + q < ny) gst2(out + i + q, cadd(a1, v));
      }
    }
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
  if (gbl(D.ctl)->done) return;
  const int nz = D.nz, Py = D.py, Pz = D.pz;
  const int tiles = (Py + TW - 1) / TW;
  const int kx = wi.item / tiles;
  const int ky0 = (wi.item - kx * tiles) * TW;
  const int NL = 3 * TW;
  float2* buf = lds;
  float2* twl = lds + Pz * NL;
  load_twiddles(twl, Pz, tw, 256);
  __syncthreads();
  const int lgz = ilog2(Pz), lgT = ilog2(TW);
  const MMG float2* Yk = gbl(D.fy) + (size_t)kx * 3 * nz * Py;
  // The inputs vanish for z >= nz, and nz <= Pz/2: the first radix-2^2 DIF
  // stage (span Pz/2) reads only x0 = x[z] and x1 = x[z + Pz/4] and is done
  // here with the same arithmetic as the full stage (x2 = x3 = 0).
  const int q = Pz >> 2;
  if (q == 0) {
    for (int e = threadIdx.x; e < Pz * NL; e += 256) {
      const int t = e & (TW - 1), zc = e >> lgT;
      const int z = zc / 3, c = zc - 3 * z;
      const int ky = ky0 + t;
      float2 v = make_float2(0.f, 0.f);
      if (z < nz && ky < Py) v = gld2(Yk + ((size_t)c * nz + z) * Py + ky);
      buf[z * NL + c * TW + t] = v;
    }
  }
  for (int e = threadIdx.x; e < q * NL; e += 256) {
    const int t = e & (TW - 1), zc = e >> lgT;
    const int z = zc / 3, c = zc - 3 * z;
    const int ky = min(ky0 + t, Py - 1);
    const MMG float2* col = Yk + (size_t)c * nz * Py + ky;
    float2 x0 = gld2(col + (size_t)min(z, nz - 1) * Py), x1 = gld2(col + (size_t)min(z + q, nz - 1) * Py);
    if (z >= nz) x0 = make_float2(0.f, 0.f);
    if (z + q >= nz) x1 = make_float2(0.f, 0.f);
    const float2 zero = make_float2(0.f, 0.f);
    const float2 w1 = twl[z], w2 = twl[2 * z];
    const float2 a0 = cadd(x0, zero), a1 = cadd(x1, zero);
    const float2 a2 = cmul(csub(x0, zero), w1);
    const float2 a3 = rot<false>(cmul(csub(x1, zero), w1));
    float2* line = buf + c * TW + t;
    line[z * NL] = cadd(a0, a1);
    line[(z + q) * NL] = cmul(csub(a0, a1), w2);
    line[(z + 2 * q) * NL] = cadd(a2, a3);
    line[(z + 3 * q) * NL] = cmul(csub(a2, a3), w2);
  }
  __syncthreads();
  fft_cols<256, false>(buf, Pz, lgz, 3, lgT, TW, NL, twl, q == 0 ? 0 : 2);
  for (int e = threadIdx.x; e < Pz * TW; e += 256) {
    const int pz_ = e >> lgT, t = e & (TW - 1);
    const int ky = ky0 + t;
    if (ky >= Py) continue;
    float2 mx = buf[pz_ * NL + t], my = buf[pz_ * NL + TW + t], mz = buf[pz_ * NL + 2 * TW + t];
    kernel_mul(D, kx, ky, brev(pz_, lgz), mx, my, mz);
    buf[pz_ * NL + t] = mx;
    buf[pz_ * NL + TW + t] = my;
    buf[pz_ * NL + 2 * TW + t] = mz;
  }
  __syncthreads();
  if (q == 0) {
    fft_cols<256, true>(buf, Pz, lgz, 3, lgT, TW, NL, twl);
    for (int e = threadIdx.x; e < nz * NL; e += 256) {
      const int t = e & (TW - 1), zc = e >> lgT;
      const int z = zc / 3, c = zc - 3 * z;
      const int ky = ky0 + t;
      if (ky < Py) gst2(gbl(D.fy) + (((size_t)kx * 3 + c) * nz + z) * Py + ky, buf[z * NL + c * TW + t]);
    }
    return;
  }
  // all DIT stages but the last radix-2^2 one (span Pz/4); that one is done
  // here for the outputs z < Pz/2 only (nz <= Pz/2), with the same arithmetic
  // as the full stage
  fft_cols<256, true>(buf, Pz, lgz, 3, lgT, TW, NL, twl, 0, lgz - 2);
  for (int e = threadIdx.x; e < q * NL; e += 256) {
    const int t = e & (TW - 1), zc = e >> lgT;
    const int i = zc / 3, c = zc - 3 * i;
    const int ky = ky0 + t;
    const float2* x = buf + i * NL + c * TW + t;
    const float2 wA = twid<true>(twl, i << 1), wB = twid<true>(twl, i);
    const float2 t1 = cmul(x[q * NL], wA), t3 = cmul(x[3 * q * NL], wA);
    const float2 a0 = cadd(x[0], t1), a1 = csub(x[0], t1), a2 = cadd(x[2 * q * NL], t3),
                 a3 = csub(x[2 * q * NL], t3);
    const float2 u = cmul(a2, wB), v = rot<true>(cmul(a3, wB));
    MMG float2* out = gbl(D.fy) + (((size_t)kx * 3 + c) * nz) * Py + ky;
    if (ky < Py && i < nz) gst2(out + (size_t)i * Py, cadd(a0, u));
    if (ky < Py && i + q < nz) gst2(out + (size_t)(i + q) * Py, cadd(a1, v));
  }
}

}  // namespace mmk

// ------------------------------------------------------------ launchers
hipError_t mmk_launch_fft_xf(int W, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             int method, int stage, const float2* tw, hipStream_t s) {
  switch (W) {
    case 1: MM_LAUNCH(mmk::k_fft_xf<1>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    case 2: MM_LAUNCH(mmk::k_fft_xf<2>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    case 4: MM_LAUNCH(mmk::k_fft_xf<4>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    case 8: MM_LAUNCH(mmk::k_fft_xf<8>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    case 16: MM_LAUNCH(mmk::k_fft_xf<16>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    case 32: MM_LAUNCH(mmk::k_fft_xf<32>, dim3(nblocks), dim3(256), lds, s, d, w, method, stage, tw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mmk_launch_fft_xi(int W, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             const float2* tw, hipStream_t s) {
  switch (W) {
    case 1: MM_LAUNCH(mmk::k_fft_xi<1>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    case 2: MM_LAUNCH(mmk::k_fft_xi<2>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    case 4: MM_LAUNCH(mmk::k_fft_xi<4>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    case 8: MM_LAUNCH(mmk::k_fft_xi<8>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    case 16: MM_LAUNCH(mmk::k_fft_xi<16>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    case 32: MM_LAUNCH(mmk::k_fft_xi<32>, dim3(nblocks), dim3(256), lds, s, d, w, tw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t mmk_launch_fft_yz(int TK, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             const float2* tw, hipStream_t s) {
  MM_LAUNCH(mmk::k_fft_yz, dim3(nblocks), dim3(MM_YZ_T), lds, s, d, w, tw, TK);
  return hipGetLastError();
}

#define MM_YZR_CASE(A, B)                                                                        \
  if (MY == A && MZ == B) {                                                                      \
    MM_LAUNCH((mmk::k_fft_yzr<A, B>), dim3(nblocks), dim3(MM_YZR_T), lds, s, d, w, tw); \
    return hipGetLastError();                                                                    \
  }
hipError_t mmk_launch_fft_yzr(int MY, int MZ, int nblocks, size_t lds, const InstDesc* d,
                              const WorkItem* w, const float2* tw, hipStream_t s) {
  MM_YZR_CASE(4, 4) MM_YZR_CASE(8, 4) MM_YZR_CASE(16, 4) MM_YZR_CASE(32, 4)
  MM_YZR_CASE(4, 8) MM_YZR_CASE(8, 8) MM_YZR_CASE(16, 8) MM_YZR_CASE(32, 8)
  MM_YZR_CASE(4, 16) MM_YZR_CASE(8, 16) MM_YZR_CASE(16, 16) MM_YZR_CASE(32, 16)
  return hipErrorInvalidValue;
}

hipError_t mmk_launch_fft_xr(int dir, int MX, int nblocks, const InstDesc* d, const WorkItem* w, int method,
                             int stage, const float2* tw, hipStream_t s) {
  switch (MX * dir) {
    case 4: MM_LAUNCH(mmk::k_fft_xfr<4>, dim3(nblocks), dim3(MM_XR_T), 0, s, d, w, method, stage, tw); break;
    case 8: MM_LAUNCH(mmk::k_fft_xfr<8>, dim3(nblocks), dim3(MM_XR_T), 0, s, d, w, method, stage, tw); break;
    case 16: MM_LAUNCH(mmk::k_fft_xfr<16>, dim3(nblocks), dim3(MM_XR_T), 0, s, d, w, method, stage, tw); break;
    case 32: MM_LAUNCH(mmk::k_fft_xfr<32>, dim3(nblocks), dim3(MM_XR_T), 0, s, d, w, method, stage, tw); break;
    case -4: MM_LAUNCH(mmk::k_fft_xir<4>, dim3(nblocks), dim3(MM_XR_T), 0, s, d, w, tw); break;
    case -8: MM_LAUNCH(mmk::k_fft_xir<8>, dim3(nblocks), dim3(MM_XR_T), 0, s, d, w, tw); break;
    case -16: MM_LAUNCH(mmk::k_fft_xir<16>, dim3(nblocks), dim3(MM_XR_T), 0, s, d, w, tw); break;
    case -32: MM_LAUNCH(mmk::k_fft_xir<32>, dim3(nblocks), dim3(MM_XR_T), 0, s, d, w, tw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define MM_YZ8_CASE(A, B)                                                                        \
  if (MY == A && MZ == B) {                                                                      \
    MM_LAUNCH((mmk::k_fft_yz8<A, B>), dim3(nblocks + nfinal), dim3(MM_YZ8_T), lds, s, d, w, tw, \
                       nblocks, fmethod, fstage);                                                \
    return hipGetLastError();                                                                    \
  }
hipError_t mmk_launch_fft_yz8(int MY, int MZ, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                              const float2* tw, hipStream_t s, int nfinal, int fmethod, int fstage) {
  if (nfinal < 0 || (nfinal > 0 && lds < MMI_PSTRIDE * sizeof(double))) return hipErrorInvalidValue;
  MM_YZ8_CASE(4, 8) MM_YZ8_CASE(8, 8) MM_YZ8_CASE(16, 8) MM_YZ8_CASE(32, 8)
  MM_YZ8_CASE(4, 16) MM_YZ8_CASE(8, 16) MM_YZ8_CASE(16, 16) MM_YZ8_CASE(32, 16)
  return hipErrorInvalidValue;
}

#ifndef MM_YZX_PAD
#define MM_YZX_PAD 1
#endif
#define MM_YZX_CASE(A, B)                                                                          \
  if (MY == A && MZ == B) {                                                                        \
    MM_LAUNCH((mmk::k_fft_yzx<A, B, MM_YZX_PAD>), dim3(nblocks + nfinal), dim3(MM_YZX_T), lds, s, d, w, tw, \
              nblocks, fmethod, fstage);                                                          \
    return hipGetLastError();                                                                      \
  }
hipError_t mmk_launch_fft_yzx(int MY, int MZ, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                              const float2* tw, hipStream_t s, int nfinal, int fmethod, int fstage) {
  if (nfinal < 0 || (nfinal > 0 && lds < MMI_PSTRIDE * sizeof(double))) return hipErrorInvalidValue;
  MM_YZX_CASE(4, 8) MM_YZX_CASE(8, 8) MM_YZX_CASE(16, 8) MM_YZX_CASE(32, 8)
  MM_YZX_CASE(4, 16) MM_YZX_CASE(8, 16) MM_YZX_CASE(16, 16) MM_YZX_CASE(32, 16)
  return hipErrorInvalidValue;
}
int mmk_yzx_pad() { return MM_YZX_PAD; }
bool mmk_yzx_pairs(int py, int pz) {
  return (pz == 32 && mmk::YzxPairs<128, 32>::on && py == 128) || (pz == 64 && mmk::YzxPairs<64, 64>::on && py == 64);
}

hipError_t mmk_launch_fft_ysx(int dir, int py, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                              const float2* tw, hipStream_t s, int nfinal, int fmethod, int fstage) {
  if (nfinal < 0 || (nfinal > 0 && (dir > 0 || lds < MMI_PSTRIDE * sizeof(double)))) return hipErrorInvalidValue;
#define MM_YSX_CASE(P)                                                                                       \
  if (py == P) {                                                                                             \
    if (dir < 0)                                                                                             \
      MM_LAUNCH((mmk::k_fft_ysx<P, -1>), dim3(nblocks + nfinal), dim3(MM_SX_T), lds, s, d, w, tw, nblocks,   \
                fmethod, fstage);                                                                            \
    else                                                                                                     \
      MM_LAUNCH((mmk::k_fft_ysx<P, 1>), dim3(nblocks), dim3(MM_SX_T), lds, s, d, w, tw, nblocks, 0, 0);      \
    return hipGetLastError();                                                                                \
  }
  MM_YSX_CASE(16) MM_YSX_CASE(32) MM_YSX_CASE(64) MM_YSX_CASE(128) MM_YSX_CASE(256)
  return hipErrorInvalidValue;
}
// rows per workgroup of the split y pass
int mmk_sx_rows(int py) {
  switch (py) {
    case 16: return mmk::SplitY<16>::ROWS;
    case 32: return mmk::SplitY<32>::ROWS;
    case 64: return mmk::SplitY<64>::ROWS;
    case 128: return mmk::SplitY<128>::ROWS;
    case 256: return mmk::SplitY<256>::ROWS;
    default: return 0;
  }
}

hipError_t mmk_launch_fft_y(int dir, int W, int nblocks, size_t lds, const InstDesc* d,
                            const WorkItem* w, const float2* tw, hipStream_t s) {
  if (dir < 0) MM_LAUNCH(mmk::k_fft_y<-1>, dim3(nblocks), dim3(256), lds, s, d, w, W, tw);
  else MM_LAUNCH(mmk::k_fft_y<1>, dim3(nblocks), dim3(256), lds, s, d, w, W, tw);
  return hipGetLastError();
}

hipError_t mmk_launch_fft_zc(int TW, int nblocks, size_t lds, const InstDesc* d, const WorkItem* w,
                             const float2* tw, hipStream_t s) {
  MM_LAUNCH(mmk::k_fft_zc, dim3(nblocks), dim3(256), lds, s, d, w, TW, tw);
  return hipGetLastError();
}

hipError_t mmk_set_lds_limits() {
  hipError_t e = hipFuncSetAttribute((const void*)mmk::k_fft_yz,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
#define MM_YZR_ATTR(A, B)                                                                         \
  if (e == hipSuccess)                                                                            \
    e = hipFuncSetAttribute((const void*)mmk::k_fft_yzr<A, B>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                            160 * 1024);
  MM_YZR_ATTR(4, 4) MM_YZR_ATTR(8, 4) MM_YZR_ATTR(16, 4) MM_YZR_ATTR(32, 4)
  MM_YZR_ATTR(4, 8) MM_YZR_ATTR(8, 8) MM_YZR_ATTR(16, 8) MM_YZR_ATTR(32, 8)
  MM_YZR_ATTR(4, 16) MM_YZR_ATTR(8, 16) MM_YZR_ATTR(16, 16) MM_YZR_ATTR(32, 16)
#define MM_YZ8_ATTR(A, B)                                                                         \
  if (e == hipSuccess)                                                                            \
    e = hipFuncSetAttribute((const void*)mmk::k_fft_yz8<A, B>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                            160 * 1024);
  MM_YZ8_ATTR(4, 8) MM_YZ8_ATTR(8, 8) MM_YZ8_ATTR(16, 8) MM_YZ8_ATTR(32, 8)
  MM_YZ8_ATTR(4, 16) MM_YZ8_ATTR(8, 16) MM_YZ8_ATTR(16, 16) MM_YZ8_ATTR(32, 16)
#define MM_YZX_ATTR(A, B)                                                                         \
  if (e == hipSuccess)                                                                            \
    e = hipFuncSetAttribute((const void*)mmk::k_fft_yzx<A, B, MM_YZX_PAD>,                        \
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  MM_YZX_ATTR(4, 8) MM_YZX_ATTR(8, 8) MM_YZX_ATTR(16, 8) MM_YZX_ATTR(32, 8)
  MM_YZX_ATTR(4, 16) MM_YZX_ATTR(8, 16) MM_YZX_ATTR(16, 16) MM_YZX_ATTR(32, 16)
#define MM_SX_ATTR(K)                                                                                      \
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)K, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  MM_SX_ATTR((mmk::k_fft_ysx<16, -1>)) MM_SX_ATTR((mmk::k_fft_ysx<32, -1>)) MM_SX_ATTR((mmk::k_fft_ysx<64, -1>))
  MM_SX_ATTR((mmk::k_fft_ysx<128, -1>)) MM_SX_ATTR((mmk::k_fft_ysx<256, -1>))
  MM_SX_ATTR((mmk::k_fft_ysx<16, 1>)) MM_SX_ATTR((mmk::k_fft_ysx<32, 1>)) MM_SX_ATTR((mmk::k_fft_ysx<64, 1>))
  MM_SX_ATTR((mmk::k_fft_ysx<128, 1>)) MM_SX_ATTR((mmk::k_fft_ysx<256, 1>))
  return e;
}
