// Small device helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "mm_internal.h"

namespace mmk {

// Every buffer reached through the descriptor table lives in global memory.
// Stating the address space lets the compiler emit global loads and stores
// (scalar base + 32-bit offset, vector-memory counter only) instead of flat
// ones, which carry 64-bit addresses and also wait on the LDS counter.
#define MMG __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ MMG T* gbl(T* p) {
  return (MMG T*)p;
}

// float2 through global pointers (the vector type's operators do not take
// address-space qualified operands)
__device__ __forceinline__ float2 gld2(const MMG float2* p) {
  const MMG float* q = (const MMG float*)p;
  return make_float2(q[0], q[1]);
}
__device__ __forceinline__ void gst2(MMG float2* p, float2 v) {
  MMG float* q = (MMG float*)p;
  q[0] = v.x;
  q[1] = v.y;
}

// Element i of a global array through a scalar base and an unsigned 32-bit
// byte offset (i >= 0 and i * sizeof(T) < 2^32; the host bounds instance
// sizes accordingly): with a signed index every lane would form a 64-bit
// address (sign extension and a 64-bit add per access).
template <class T>
__device__ __forceinline__ const MMG T& gat(const MMG T* p, int i) {
  return *(const MMG T*)((const MMG char*)p + (uint32_t)i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ MMG T& gat(MMG T* p, int i) {
  return *(MMG T*)((MMG char*)p + (uint32_t)i * (uint32_t)sizeof(T));
}

// Stage input m = p0 + c1 * p1 (p1 optional), component-major per instance.
struct Src {
  const MMG float* p0;
  const MMG float* p1;
  float c1;
  __device__ __forceinline__ float ld(int idx) const {
    float v = gat(p0, idx);
    if (p1) v = fmaf(c1, gat(p1, idx), v);
    return v;
  }
};

// The same with the presence of p1 fixed at compile time, so that every
// load of a stencil (both fields when TWO) is issued without a test.
template <bool TWO>
struct SrcFixed {
  const MMG float* p0;
  const MMG float* p1;
  float c1;
  __device__ __forceinline__ explicit SrcFixed(const Src& s) : p0(s.p0), p1(s.p1), c1(s.c1) {}
  __device__ __forceinline__ float ld(int idx) const {
    float v = gat(p0, idx);
    if (TWO) v = fmaf(c1, gat(p1, idx), v);
    return v;
  }
};

// Where the input of stage `stage` lives.  RK4: 0/1 state, 2 and 4 buffer
// A, 3 buffer B.  DP45: 1 state, 2 state + h a21 k1 (not stored), 3 and 5
// buffer A, 4 and 6 buffer B, 7 the normalised candidate.
template <class CtlPtr>
__device__ __forceinline__ Src stage_src(const InstDesc& D, CtlPtr C, int method, int stage) {
  Src s;
  s.p1 = nullptr;
  s.c1 = 0.f;
  const int cur = C->cur;
  if (method == MMI_ADJ) {
    // adjoint: stage 1..nstg -> recorded stage input of the current step, 0 -> lambda_B
    const size_t vec = (size_t)3 * D.S * D.ncell;
    s.p0 = gbl((stage == 0) ? D.lam_B : D.rec_m + ((size_t)C->rec_index * D.rec_nstg + (stage - 1)) * vec);
    return s;
  }
  if (method == MMI_RK4) {
    s.p0 = gbl((stage <= 1) ? D.y[cur] : (stage == 3 ? D.st[1] : D.st[0]));
  } else {
    switch (stage) {
      case 1: s.p0 = gbl(D.y[cur]); break;
      case 2:
        s.p0 = gbl(D.y[cur]);
        s.p1 = gbl(D.k[C->slot[0]]);
        s.c1 = (float)(C->h * DPCoef::a21);
        break;
      case 3: case 5: s.p0 = gbl(D.st[0]); break;
      case 4: case 6: s.p0 = gbl(D.st[1]); break;
      default: s.p0 = gbl(D.y[1 - cur]); break;
    }
  }
  return s;
}

// bdv: this cell's demag field already at hand (used when use_bdv; pass a
// pointer fixed at compile time, never one chosen at run time, so that the
// array stays in registers).
// Effective field [T] on sublattice s at cell i (x, y, z its coordinates):
// Zeeman + exchange over magnetic neighbour pairs + uniaxial anisotropy +
// demag (local diagonal, or the FFT result in D.bd) + feedback c_s fb along
// x + intersublattice -B_E m_{s'}.  m holds the cell's own stage input.
template <class SRC>
__device__ __forceinline__ void field_at(const InstDesc& D, const SRC& src, int i, int x, int y,
                                         int z, const float (&m)[2][3], int s, float fb,
                                         bool has_bd, float (&B)[3], const float* bdv = nullptr,
                                         bool use_bdv = true) {
  const int nc = D.ncell;
  const int nx = D.nx, ny = D.ny, nz = D.nz;
  const int base = s * 3 * nc;
  const float m0 = m[s][0], m1 = m[s][1], m2 = m[s][2];
  float bx = D.B0x, by = D.B0y, bz = D.B0z;
  // Neighbour indices: a missing or non-magnetic neighbour is replaced by the
  // cell itself, whose difference m_j - m_i is then exactly zero, so every
  // load below is unconditional and all of them are in flight together.
  const int off[6] = {-1, 1, -nx, nx, -nx * ny, nx * ny};
  const bool has[6] = {x > 0, x < nx - 1, y > 0, y < ny - 1, z > 0, z < nz - 1};
  int jn[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) jn[q] = has[q] ? i + off[q] : i;
  if (D.has_geom) {
    const MMG uint8_t* G = gbl(D.geom);
    uint8_t g[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) g[q] = gat(G, jn[q]);
#pragma unroll
    for (int q = 0; q < 6; ++q) jn[q] = g[q] ? jn[q] : i;
  }
  float nb[6][3];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    nb[q][0] = src.ld(base + jn[q]);
    nb[q][1] = src.ld(base + nc + jn[q]);
    nb[q][2] = src.ld(base + 2 * nc + jn[q]);
  }
  const float cq[6] = {D.cex_x, D.cex_x, D.cex_y, D.cex_y, D.cex_z, D.cex_z};
  float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    sx = fmaf(cq[q], nb[q][0] - m0, sx);
    sy = fmaf(cq[q], nb[q][1] - m1, sy);
    sz = fmaf(cq[q], nb[q][2] - m2, sz);
  }
  bx += sx;
  by += sy;
  bz += sz;
  const float md = m0 * D.ex + m1 * D.ey + m2 * D.ez;
  const float ck = D.cK * md;
  bx = fmaf(ck, D.ex, bx);
  by = fmaf(ck, D.ey, by);
  bz = fmaf(ck, D.ez, bz);
  if (D.demag == 1) {
    float tx = m[0][0], ty = m[0][1], tz = m[0][2];
    if (D.S == 2) { tx += m[1][0]; ty += m[1][1]; tz += m[1][2]; }
    bx = fmaf(D.nlx, tx, bx);
    by = fmaf(D.nly, ty, by);
    bz = fmaf(D.nlz, tz, bz);
  } else if (bdv && use_bdv) {
    bx += bdv[0];
    by += bdv[1];
    bz += bdv[2];
  } else if (has_bd) {
    const MMG float* bd = gbl(D.bd);
    bx += gat(bd, i);
    by += gat(bd, nc + i);
    bz += gat(bd, 2 * nc + i);
  }
  bx = fmaf(D.csign[s], fb, bx);
  if (D.S == 2) {
    const int o = 1 - s;
    bx = fmaf(-D.BE, m[o][0], bx);
    by = fmaf(-D.BE, m[o][1], by);
    bz = fmaf(-D.BE, m[o][2], bz);
  }
  B[0] = bx;
  B[1] = by;
  B[2] = bz;
}

// The workgroups of one dispatch are placed on the eight XCDs round-robin
// (block b on XCD b mod 8) and every XCD has its own L2.  This maps the
// hardware block index to a logical one (a bijection on [0, gridDim.x)) so
// that each XCD works through one contiguous range of logical blocks: cells
// that are neighbours in z, two 512-cell workgroups apart, are then read
// through the same L2 instead of being fetched again by another XCD.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// Workgroup (of MMI_WG cells) that the lw-th workgroup of an instance takes.
// Where a z-plane is a whole number P >= 64 of workgroups, consecutive
// workgroups walk z first (lw = b nz + z takes block b of plane z), so that
// the planes a stencil reads above and below are fetched by workgroups that
// run close together on the same XCD (otherwise P workgroups apart, about
// the span an XCD has resident).  Smaller planes keep the plain order, in
// which z-neighbours are already close.  A bijection on the instance's
// workgroups; the workgroup's cells, x-rows and partial record follow it.
__device__ __forceinline__ int zmajor_wg(const InstDesc& D, int lw) {
  const int plane = D.nx * D.ny;
  if ((plane & (MMI_WG - 1)) || plane < 64 * MMI_WG) return lw;
  const int P = plane >> MMI_LG_WG, b = lw / D.nz;
  return (lw - b * D.nz) * P + b;
}

// Coordinates of cell i = (z ny + y) nx + x: shifts and masks when nx and ny
// are powers of two, integer divisions otherwise.
__device__ __forceinline__ void cell_xyz(const InstDesc& D, int i, int& x, int& y, int& z) {
  if (D.lgnx >= 0 && D.lgny >= 0) {
    x = i & (D.nx - 1);
    const int yz = i >> D.lgnx;
    y = yz & (D.ny - 1);
    z = yz >> D.lgny;
  } else {
    const int yz = i / D.nx;
    x = i - yz * D.nx;
    z = yz / D.ny;
    y = yz - z * D.ny;
  }
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
