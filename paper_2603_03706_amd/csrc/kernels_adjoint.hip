// Discrete adjoint of the fixed-step RK4 map, one reverse step at a time.
//
// Forward step (joint state y = (m, a), f = (torque, cavity RHS)):
//   k1 = f(y1), y2 = y + h/2 k1, k2 = f(y2), y3 = y + h/2 k2, k3 = f(y3),
//   y4 = y + h k3, k4 = f(y4), z = y + h/6 (k1 + 2 k2 + 2 k3 + k4),
//   m' = z_m / |z_m| on magnetic cells, a' = z_a.
// Reverse step, given lambda' = dL/dy':
//   lambda_z = (I - m' m'^T) lambda'_m / |z_m| (a: unchanged),
//   lambda_y = lambda_z, lambda_k4 = h/6 lambda_z, then for s = 4..1:
//   mu_s = J_f(y_s)^T lambda_ks (+ parameter gradients), lambda_y += mu_s,
//   lambda_k(s-1) = h w_(s-1)/6 lambda_z + c_s mu_s  (w = 1,2,2,1; c = h/2, h/2, h).
// The stage inputs y_s, |z_m| and a_s were recorded by the forward kernels
// while the segment was recomputed from its checkpoint.
//
// Adaptive (DP45) runs are reversed as the replay of their accepted steps
// (the step sizes h held): z = y + h sum_{j<=6} b_j k_j with stage inputs
// y_s = y + h sum_{j<s} a_sj k_j.  Reverse: lambda_z as above, lambda_y =
// lambda_z, then for s = 6..1: mu_s = J_f(y_s)^T lambda_ks, lambda_y += mu_s,
// with lambda_ks = h (b_s lambda_z + sum_{q>s} a_qs mu_q); the mu_q of
// stages 3..6 are kept until the earlier stages have used them.
// Stage numbering of the launches: RK4 stages 1..4 and 5 for the step
// start; DP45 stages 1..6 and 7 for the step start.
//
// Per stage the VJP is split in two cell kernels around the demag
// convolution of lambda_B (the tensor is symmetric and even, so the same
// FFT convolution is its own transpose):
//   A: lambda_B = dtorque/dB^T lambda_k, the direct torque term, the m^-
//      term, partial sums for the cavity and the parameters, grad u_n;
//   B: exchange / anisotropy / demag / intersublattice transposes applied
//      to lambda_B, then the RK bookkeeping above.
#include "mm_internal.h"
#include "kernels_common.h"
#include "launch.h"
#include "xrows.h"

namespace mmk {

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int w = 1; w < MMI_WG / 64; ++w) r += sh[w];
  return r;
}

// K block sums with one exchange through LDS (sh: K * MMI_WG / 64 doubles);
// every value is added in the same order as by block_sum.
template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double* sh) {
  constexpr int NW = MMI_WG / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k * NW + wv] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double r = sh[k * NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) r += sh[k * NW + w];
    v[k] = r;
  }
}

__device__ __forceinline__ void cross3(const float* a, const float* b, float* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// size of the step being reversed: fixed (RK4) or the logged one (DP45)
template <class CtlPtr>
__device__ __forceinline__ double adj_step(const InstDesc& D, CtlPtr C) {
  if (D.method != MMI_DP45) return C->adj_h;
  return fabs(gbl(D.hlog)[C->adj_base + C->rec_index]);
}

// ---------------------------------------------------------- step start
// lambda_z from the step-end adjoint (held in lam_y), lambda_y = lambda_z,
// lambda_k4 = h/6 lambda_z.
__global__ __launch_bounds__(MMI_WG) void k_adj_start(const InstDesc* __restrict__ descs,
                                                      const int* __restrict__ wg_inst) {
  const int lblk = xcd_block();
  const InstDesc& D = descs[wg_inst[lblk]];
  const MMG InstCtl* __restrict__ C = gbl(D.ctl);
  if (C->done) return;
  const int nc = D.ncell, S = D.S;
  const int i = (lblk - D.wg0) * MMI_WG + threadIdx.x;
  if (i >= nc) return;
  const bool mag = !D.has_geom || gbl(D.geom)[i];
  const size_t vec = (size_t)3 * S * nc;
  const int ri = C->rec_index;
  const MMG float* Yn = gbl(D.rec_m) + ((size_t)(ri + 1) * D.rec_nstg) * vec;   // state after the step
  MMG float* const lam_y = gbl(D.lam_y);
  MMG float* const lam_z = gbl(D.lam_z);
  MMG float* const lam_k = gbl(D.lam_k);
  // weight of the last stage in the step-end combination: h/6 (RK4), h b_6 (DP45)
  const float c6 = (float)(D.method == MMI_DP45 ? adj_step(D, C) * DPCoef::b6 : C->adj_h / 6.0);
  for (int s = 0; s < S; ++s) {
    float l[3], y[3];
    for (int c = 0; c < 3; ++c) {
      l[c] = lam_y[(s * 3 + c) * nc + i];
      y[c] = Yn[(s * 3 + c) * nc + i];
    }
    float z[3] = {0.f, 0.f, 0.f};
    if (mag) {
      const float inv = 1.0f / gbl(D.rec_norm)[(size_t)ri * S * nc + s * nc + i];
      const float d = l[0] * y[0] + l[1] * y[1] + l[2] * y[2];
      for (int c = 0; c < 3; ++c) z[c] = (l[c] - y[c] * d) * inv;
    }
    for (int c = 0; c < 3; ++c) {
      const int idx = (s * 3 + c) * nc + i;
      lam_z[idx] = z[c];
      lam_y[idx] = z[c];
      lam_k[idx] = c6 * z[c];
    }
  }
}

// ------------------------------------------------------------ stage A
template <int ST>
__global__ __launch_bounds__(MMI_WG) void k_adj_a(const InstDesc* __restrict__ descs,
                                                  const int* __restrict__ wg_inst,
                                                  const float2* __restrict__ tw) {
  __shared__ double sh[4 * (MMI_WG / 64)];
  extern __shared__ float2 xl[];
  const int lblk = xcd_block();
  const InstDesc& D = descs[wg_inst[lblk]];
  const MMG InstCtl* __restrict__ C = gbl(D.ctl);
  if (C->done) return;
  const int lw = lblk - D.wg0;
  const int nc = D.ncell, S = D.S, N = D.N;
  const int i = lw * MMI_WG + threadIdx.x;
  const bool valid = i < nc;
  const bool mag = valid && (!D.has_geom || gbl(D.geom)[i]);
  const int ri = C->rec_index;
  const Src src = stage_src(D, C, MMI_ADJ, ST);
  const MMG double* as = gbl(D.rec_a) + ((size_t)ri * D.rec_nstg + (ST - 1)) * N * 2;
  const MMG float* const u_ = gbl(D.u);
  MMG float* const lam_B = gbl(D.lam_B);
  int x = 0, yy = 0, zz = 0;
  if (valid) cell_xyz(D, i, x, yy, zz);

  float m[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  if (valid)
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (s < S)
#pragma unroll
        for (int c = 0; c < 3; ++c) m[s][c] = src.ld((s * 3 + c) * nc + i);

  // feedback value of this stage: sum_n h0_n u_n Re[e^{-i Phi_n} a_n]
  float fb = 0.f;
  if (mag)
    for (int n = 0; n < N; ++n) {
      const float b = (float)(D.h0[n] * (D.cphi[n] * as[2 * n] + D.sphi[n] * as[2 * n + 1]));
      fb = fmaf(b, D.profiled ? u_[(size_t)n * nc + i] : 1.f, fb);
    }
  const float gl = D.gl, al = D.alpha;
  const float dga = 2.f * al / (1.f + al * al);   // -d ln(gamma')/d alpha
  const float wmm = (float)(D.inv_ngeo / (double)S);
  double galpha = 0.0, gb0x = 0.0, gb0y = 0.0, gb0z = 0.0;
  float lbx[2] = {0.f, 0.f};
  float lb0[3] = {0.f, 0.f, 0.f};   // field adjoint of sublattice 0 (the R2C input)
  float mux[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  // demag field of this stage input: recorded during the segment recompute,
  // else from the convolution just enqueued
  float bdv[3] = {0.f, 0.f, 0.f};
  const bool bd_recorded = D.rec_bd != nullptr;
  if (bd_recorded && valid) {
    const MMG float* RB = gbl(D.rec_bd) + ((size_t)ri * D.rec_nstg + (ST - 1)) * (size_t)(3 * nc);
#pragma unroll
    for (int c = 0; c < 3; ++c) bdv[c] = RB[c * nc + i];
  }
  if (mag) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s >= S) continue;
      float B[3];
      field_at(D, src, i, x, yy, zz, m, s, fb, D.demag == 2, B, bdv, bd_recorded);
      const float* ms = m[s];
      float l[3];
      for (int c = 0; c < 3; ++c) l[c] = gbl(D.lam_k)[(s * 3 + c) * nc + i];
      float P[3], Q[3], lm[3], t1[3], t2[3], t3[3], lB[3];
      cross3(ms, B, P);
      cross3(ms, P, Q);
      cross3(l, ms, lm);          // lambda x m
      cross3(lm, ms, t1);         // (lambda x m) x m
      for (int c = 0; c < 3; ++c) lB[c] = -gl * (lm[c] + al * t1[c]);
      cross3(B, l, t1);           // B x lambda
      cross3(P, l, t2);           // P x lambda
      cross3(B, lm, t3);          // B x (lambda x m)
      for (int c = 0; c < 3; ++c) mux[s][c] = -gl * (t1[c] + al * (t2[c] + t3[c]));
      // dL/dalpha: lambda . (-(2a/(1+a^2)) tau - gamma' Q), tau = -gamma' (P + a Q)
      float ga = 0.f;
      for (int c = 0; c < 3; ++c) {
        const float tau = -gl * (P[c] + al * Q[c]);
        ga += l[c] * (-dga * tau - gl * Q[c]);
      }
      galpha += ga;
      gb0x += lB[0];
      gb0y += lB[1];
      gb0z += lB[2];
      lbx[s] = lB[0];
      for (int c = 0; c < 3; ++c) lam_B[(s * 3 + c) * nc + i] = lB[c];
      if (s == 0)
        for (int c = 0; c < 3; ++c) lb0[c] = lB[c];
    }
  } else if (valid) {
    for (int s = 0; s < S; ++s)
      for (int c = 0; c < 3; ++c) lam_B[(s * 3 + c) * nc + i] = 0.f;
  }
  // m^- transpose and the gradient of the mode profiles
  for (int n = 0; n < N; ++n) {
    const float u = D.profiled ? (valid ? u_[(size_t)n * nc + i] : 0.f) : 1.f;
    const float lr = (float)C->lmm[n][0], li = (float)C->lmm[n][1];
    double fbn = 0.0, mr = 0.0, mi = 0.0, gu = 0.0;
    if (mag) {
      const float arn = (float)as[2 * n], ain = (float)as[2 * n + 1];
      const float fbw = (float)(D.h0[n] * (D.cphi[n] * arn + D.sphi[n] * ain));
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (s >= S) continue;
        const float cs = D.csign[s];
        mux[s][0] += wmm * cs * u * lr;
        mux[s][1] -= wmm * cs * u * li;
        fbn += (double)(cs * lbx[s] * u);
        mr += (double)(cs * m[s][0] * u);
        mi -= (double)(cs * m[s][1] * u);
        gu += (double)(cs * (lbx[s] * fbw + wmm * (lr * m[s][0] - li * m[s][1])));
      }
      if (D.grad_u) gbl(D.grad_u)[(size_t)n * nc + i] += gu;
    }
    double sums[3] = {fbn, mr, mi};
    block_sums<3>(sums, sh);
    if (threadIdx.x == 0) {
      MMG double* rec = gbl(D.partials) + (size_t)lw * MMI_PSTRIDE;
      rec[MMI_ASLOT_FB + n] = sums[0];
      rec[MMI_ASLOT_MM + 2 * n] = sums[1];
      rec[MMI_ASLOT_MM + 2 * n + 1] = sums[2];
    }
  }
  if (valid)
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (s < S)
#pragma unroll
        for (int c = 0; c < 3; ++c) gbl(D.mu)[(s * 3 + c) * nc + i] = mux[s][c];
  double r[4] = {galpha, gb0x, gb0y, gb0z};
  block_sums<4>(r, sh);
  if (threadIdx.x == 0) {
    MMG double* rec = gbl(D.partials) + (size_t)lw * MMI_PSTRIDE;
    rec[MMI_ASLOT_ALPHA] = r[0];
    rec[MMI_ASLOT_B0] = r[1];
    rec[MMI_ASLOT_B0 + 1] = r[2];
    rec[MMI_ASLOT_B0 + 2] = r[3];
  }
  if (D.xfused) {
    // R2C of the field adjoint of this workgroup's x-rows: the X rows of its
    // convolution (no separate x-forward pass)
    const XRows xq = xrows_setup(D, lw, xl);
    load_twiddles(xq.twl, xq.Px, tw, MMI_WG);
    xrows_r2c(D, xq, lb0, false);
  }
}

// ------------------------------------------------------------ stage B
template <int ST>
__global__ __launch_bounds__(MMI_WG) void k_adj_b(const InstDesc* __restrict__ descs,
                                                  const int* __restrict__ wg_inst,
                                                  const float2* __restrict__ tw) {
  extern __shared__ float2 xl[];
  const int lblk = xcd_block();
  const InstDesc& D = descs[wg_inst[lblk]];
  const MMG InstCtl* __restrict__ C = gbl(D.ctl);
  if (C->done) return;
  const int nc = D.ncell, S = D.S;
  const int lw = lblk - D.wg0;
  // convolved field adjoint of this cell: C2R of the workgroup's X rows, or
  // the x-inverse pass's output
  float bdv[3] = {0.f, 0.f, 0.f};
  if (D.xfused) {
    const XRows xq = xrows_setup(D, lw, xl);
    load_twiddles(xq.twl, xq.Px, tw, MMI_WG);
    xrows_c2r(D, xq, bdv);
  }
  const int i = lw * MMI_WG + threadIdx.x;
  if (i >= nc) return;   // no barrier below
  const bool mag = !D.has_geom || gbl(D.geom)[i];
  const int nx = D.nx, ny = D.ny, nz = D.nz;
  int x, y, z;
  cell_xyz(D, i, x, y, z);
  const MMG float* L = gbl(D.lam_B);
  const MMG uint8_t* G = D.has_geom ? gbl(D.geom) : nullptr;
  MMG float* const lam_y = gbl(D.lam_y);
  MMG float* const lam_z = gbl(D.lam_z);
  MMG float* const lam_k = gbl(D.lam_k);
  const bool dp = D.method == MMI_DP45;
  const double h = adj_step(D, C);
  // RK4: coefficient of k_(ST-1) in y_ST and the weight of k_(ST-1)
  const float cst = (float)(ST == 4 ? h : 0.5 * h);
  const float wprev = (float)(h * (ST == 2 ? 1.0 : 2.0) / 6.0);
  // DP45: lambda_k(ST-1) = h (b_(ST-1) lambda_z + sum_{q>=ST} a_(q,ST-1) mu_q)
  const size_t vec = (size_t)3 * S * nc;
  float lb[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  for (int s = 0; s < S; ++s)
    for (int c = 0; c < 3; ++c) lb[s][c] = L[(s * 3 + c) * nc + i];
  for (int s = 0; s < S; ++s) {
    float mu[3];
    for (int c = 0; c < 3; ++c) mu[c] = gbl(D.mu)[(s * 3 + c) * nc + i];
    if (mag) {
      // exchange (a symmetric graph Laplacian over magnetic pairs)
      const int base = s * 3 * nc;
      float ex[3] = {0.f, 0.f, 0.f};
#define MM_NBR(cond, off, coef)                                       \
  if (cond) {                                                         \
    const int j = i + (off);                                          \
    if (!G || G[j]) {                                                 \
      for (int c = 0; c < 3; ++c)                                     \
        ex[c] = fmaf(coef, L[base + c * nc + j] - lb[s][c], ex[c]);   \
    }                                                                 \
  }
      MM_NBR(x > 0, -1, D.cex_x)
      MM_NBR(x < nx - 1, 1, D.cex_x)
      MM_NBR(y > 0, -nx, D.cex_y)
      MM_NBR(y < ny - 1, nx, D.cex_y)
      MM_NBR(z > 0, -nx * ny, D.cex_z)
      MM_NBR(z < nz - 1, nx * ny, D.cex_z)
#undef MM_NBR
      const float e[3] = {D.ex, D.ey, D.ez};
      const float le = lb[s][0] * e[0] + lb[s][1] * e[1] + lb[s][2] * e[2];
      const float nl[3] = {D.nlx, D.nly, D.nlz};
      for (int c = 0; c < 3; ++c) {
        float v = mu[c] + ex[c] + D.cK * le * e[c];
        if (D.demag == 1) {
          float t = lb[0][c];
          if (S == 2) t += lb[1][c];
          v += nl[c] * t;
        } else if (D.demag == 2) {
          v += D.xfused ? bdv[c] : gbl(D.bd)[c * nc + i];
        }
        if (S == 2) v -= D.BE * lb[1 - s][c];
        mu[c] = v;
      }
    } else {
      mu[0] = mu[1] = mu[2] = 0.f;
    }
    for (int c = 0; c < 3; ++c) {
      const int idx = (s * 3 + c) * nc + i;
      lam_y[idx] += mu[c];
      if (!dp) {
        if (ST > 1) lam_k[idx] = fmaf(wprev, lam_z[idx], cst * mu[c]);
      } else if (ST > 1) {
        // keep mu of stages 3..6 for the stages below
        if (ST >= 3) gbl(D.mu_st)[(size_t)(ST - 3) * vec + idx] = mu[c];
        float acc = (float)(DPCoef::b(ST - 1)) * lam_z[idx] + (float)DPCoef::a(ST, ST - 1) * mu[c];
#pragma unroll
        for (int q = ST + 1; q <= 6; ++q)
          acc = fmaf((float)DPCoef::a(q, ST - 1), gbl(D.mu_st)[(size_t)(q - 3) * vec + idx], acc);
        lam_k[idx] = (float)h * acc;
      }
    }
  }
}

// --------------------------------------------------------- cavity part
// RK4 (DP = false): ST = 5 step start, ST = 4..1 after the stage kernels of
// that stage.  DP45 (DP = true): ST = 7 step start, ST = 6..1.
template <bool DP, int ST>
__global__ __launch_bounds__(MMI_WG) void k_adj_cav(const InstDesc* __restrict__ descs, int count) {
  __shared__ double sh[MMI_WG / 64];
  __shared__ double tot[MMI_PSTRIDE];
  constexpr bool kStart = DP ? ST == 7 : ST == 5;
  if ((int)blockIdx.x >= count) return;
  const InstDesc& D = descs[blockIdx.x];
  InstCtl* C = D.ctl;
  if (C->done) return;
  const int N = D.N;
  const double h = adj_step(D, C);
  if (!kStart) {
    for (int q = 0; q < MMI_PSTRIDE; ++q) {
      const bool used = (q < N) || (q >= MMI_ASLOT_MM && q < MMI_ASLOT_MM + 2 * N) ||
                        (q >= MMI_ASLOT_ALPHA && q < MMI_ASLOT_B0 + 3);
      if (!used) continue;
      double v = 0.0;
      for (int w = threadIdx.x; w < D.nwg; w += MMI_WG) v += gbl(D.partials)[(size_t)w * MMI_PSTRIDE + q];
      v = block_sum(v, sh);
      if (threadIdx.x == 0) tot[q] = v;
    }
  }
  if (threadIdx.x != 0) return;
  if (kStart) {
    // a loss on the trace: its derivative at the end of the step being reversed
    if (!DP && D.dla_trace) {
      const double* q = D.dla_trace + (size_t)(C->adj_base + C->rec_index + 1) * N * 2;
      for (int n = 0; n < N; ++n) {
        C->la[n][0] += q[2 * n];
        C->la[n][1] += q[2 * n + 1];
      }
    }
    const double wl = DP ? h * DPCoef::b6 : h / 6.0;
    for (int n = 0; n < N; ++n)
      for (int r = 0; r < 2; ++r) {
        C->lza[n][r] = C->la[n][r];
        C->lka[n][r] = wl * C->la[n][r];
      }
  } else {
    const double* as = D.rec_a + ((size_t)C->rec_index * D.rec_nstg + (ST - 1)) * N * 2;
    const double scale = D.inv_ngeo / (double)D.S;
    C->grad_alpha += tot[MMI_ASLOT_ALPHA];
    for (int c = 0; c < 3; ++c) C->grad_B0[c] += tot[MMI_ASLOT_B0 + c];
    const double cst = (ST == 4) ? h : 0.5 * h;
    const double wprev = h * (ST == 2 ? 1.0 : 2.0) / 6.0;
    // mu_a of every mode first: with direct mode coupling it reads the
    // lambda_ka of all modes, which the update below overwrites
    double mu[MMI_MAX_MODES][2];
    for (int n = 0; n < N; ++n) {
      const double c = D.cphi[n], s = D.sphi[n], g = D.g[n];
      const double lr = C->lka[n][0], li = C->lka[n][1];
      const double fb = tot[MMI_ASLOT_FB + n];
      const double mr = tot[MMI_ASLOT_MM + 2 * n] * scale, mi = tot[MMI_ASLOT_MM + 2 * n + 1] * scale;
      // dF/dg = (s + i c) m^- ; feedback h0 = 2 g / gamma with Re[e^{-i Phi} a] = c ar + s ai
      const double fr = s * mr - c * mi, fi = s * mi + c * mr;
      C->grad_g[n] += lr * fr + li * fi + fb * (2.0 / D.gamma) * (c * as[2 * n] + s * as[2 * n + 1]);
      // mu_a = conj(-kappa - i w) lambda_ka + h0 fb (c, s)
      const double w = D.omega[n], kp = D.kappa[n];
      double mur = -kp * lr - w * li + D.h0[n] * fb * c;
      double mui = w * lr - kp * li + D.h0[n] * fb * s;
      if (D.kerr_on) {
        // transpose of the Jacobian of -i K |a|^2 a at the stage amplitude
        const double ar = as[2 * n], ai = as[2 * n + 1], K = D.kerr[n];
        const double q = K * (ar * ar + ai * ai), x = 2.0 * K * ar * ai;
        mur += lr * x - li * (q + 2.0 * K * ar * ar);
        mui += lr * (q + 2.0 * K * ai * ai) - li * x;
      }
      if (D.param_on) {
        // transpose of the Jacobian of -i Lam conj(a), Lam = lam e^{-2 i wp t}
        // at the stage time: [[Li, -Lr], [-Lr, -Li]] (symmetric)
        const double ts = DP ? gbl(D.rec_t)[C->rec_index] + DPCoef::c(ST) * h
                             : C->adj_t0 + (double)C->rec_index * h + (ST == 1 ? 0.0 : ST == 4 ? h : 0.5 * h);
        double sn, cs;
        sincos(2.0 * D.par_wp[n] * ts, &sn, &cs);
        const double Lr = D.par_re[n] * cs + D.par_im[n] * sn;
        const double Li = D.par_im[n] * cs - D.par_re[n] * sn;
        mur += Li * lr - Lr * li;
        mui -= Lr * lr + Li * li;
      }
      if (D.jcpl_on)
        for (int q = 0; q < N; ++q) {
          // -i sum_q J_qn a_n in the equation of mode q, J symmetric
          mur -= D.jcpl[q][n] * C->lka[q][1];
          mui += D.jcpl[q][n] * C->lka[q][0];
        }
      mu[n][0] = mur;
      mu[n][1] = mui;
    }
    for (int n = 0; n < N; ++n) {
      C->la[n][0] += mu[n][0];
      C->la[n][1] += mu[n][1];
      if (!DP) {
        if (ST > 1) {
          C->lka[n][0] = wprev * C->lza[n][0] + cst * mu[n][0];
          C->lka[n][1] = wprev * C->lza[n][1] + cst * mu[n][1];
        }
      } else if (ST > 1) {
        // lambda_ka(ST-1) = h (b_(ST-1) lambda_za + sum_{q>=ST} a_(q,ST-1) mu_a,q)
        for (int r = 0; r < 2; ++r) {
          if (ST >= 3) C->lmua[ST - 1][n][r] = mu[n][r];
          double acc = DPCoef::b(ST - 1) * C->lza[n][r] + DPCoef::a(ST, ST - 1) * mu[n][r];
          for (int q = ST + 1; q <= 6; ++q) acc += DPCoef::a(q, ST - 1) * C->lmua[q - 1][n][r];
          C->lka[n][r] = h * acc;
        }
      }
    }
    if (ST == 1) C->rec_index -= 1;
  }
  // adjoint of m^- for the next stage kernel A: conj(i g e^{-i Phi}) lambda_ka
  if (ST >= 2) {
    for (int n = 0; n < N; ++n) {
      const double c = D.cphi[n], s = D.sphi[n], g = D.g[n];
      const double lr = C->lka[n][0], li = C->lka[n][1];
      // conj(g (s + i c)) = g (s - i c)
      C->lmm[n][0] = g * (s * lr + c * li);
      C->lmm[n][1] = g * (s * li - c * lr);
    }
  }
}

}  // namespace mmk

hipError_t mmk_launch_adj(int kind, int stage, int nblocks, int count, const InstDesc* d, const int* wg,
                          hipStream_t s, const float2* tw, size_t lds) {
  // kind 0: start, 1: A, 2: B, 3: cavity (RK4), 4: cavity (DP45)
  if (kind == 0) {
    MM_LAUNCH(mmk::k_adj_start, dim3(nblocks), dim3(MMI_WG), 0, s, d, wg);
    return hipGetLastError();
  }
#define MM_ADJ(K, ST)                                                                                  \
  if (kind == K && stage == ST) {                                                                      \
    if (K == 1) MM_LAUNCH(mmk::k_adj_a<ST>, dim3(nblocks), dim3(MMI_WG), lds, s, d, wg, tw);  \
    if (K == 2) MM_LAUNCH(mmk::k_adj_b<ST>, dim3(nblocks), dim3(MMI_WG), lds, s, d, wg, tw);  \
    return hipGetLastError();                                                                          \
  }
  MM_ADJ(1, 1) MM_ADJ(1, 2) MM_ADJ(1, 3) MM_ADJ(1, 4) MM_ADJ(1, 5) MM_ADJ(1, 6)
  MM_ADJ(2, 1) MM_ADJ(2, 2) MM_ADJ(2, 3) MM_ADJ(2, 4) MM_ADJ(2, 5) MM_ADJ(2, 6)
#undef MM_ADJ
  if (kind == 3) {
    switch (stage) {
      case 1: MM_LAUNCH((mmk::k_adj_cav<false, 1>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      case 2: MM_LAUNCH((mmk::k_adj_cav<false, 2>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      case 3: MM_LAUNCH((mmk::k_adj_cav<false, 3>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      case 4: MM_LAUNCH((mmk::k_adj_cav<false, 4>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      case 5: MM_LAUNCH((mmk::k_adj_cav<false, 5>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (kind == 4) {   // DP45 cavity part: stages 1..6, 7 = step start
    switch (stage) {
      case 1: MM_LAUNCH((mmk::k_adj_cav<true, 1>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      case 2: MM_LAUNCH((mmk::k_adj_cav<true, 2>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      case 3: MM_LAUNCH((mmk::k_adj_cav<true, 3>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      case 4: MM_LAUNCH((mmk::k_adj_cav<true, 4>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      case 5: MM_LAUNCH((mmk::k_adj_cav<true, 5>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      case 6: MM_LAUNCH((mmk::k_adj_cav<true, 6>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      case 7: MM_LAUNCH((mmk::k_adj_cav<true, 7>), dim3(count), dim3(MMI_WG), 0, s, d, count); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}
