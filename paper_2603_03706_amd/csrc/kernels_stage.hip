// Fused stage kernels: stage input -> effective field -> LL torque -> next
// stage input, with FP64 mode-weighted reductions and the FP64 cavity step /
// step-size controller done by the last workgroup of each instance.
#include "mm_internal.h"
#include "kernels_common.h"
#include "launch.h"
#include "fft_lds.h"
#include "stage_final.h"
#include "xrows.h"

namespace mmk {

// ---------------------------------------------------------------- helpers

// LL torque on sublattice s at cell i from its effective field.
template <class SRC>
__device__ __forceinline__ void torque_at(const InstDesc& D, const SRC& src, int i, int x, int y,
                                          int z, const float (&m)[2][3], int s, float fb,
                                          bool has_bd, float (&k)[3], const float* bdv = nullptr,
                                          bool use_bdv = true) {
  float B[3];
  field_at(D, src, i, x, y, z, m, s, fb, has_bd, B, bdv, use_bdv);
  const float m0 = m[s][0], m1 = m[s][1], m2 = m[s][2];
  // -gl [m x B + alpha m x (m x B)]
  const float cx = m1 * B[2] - m2 * B[1];
  const float cy = m2 * B[0] - m0 * B[2];
  const float cz = m0 * B[1] - m1 * B[0];
  const float dx = m1 * cz - m2 * cy;
  const float dy = m2 * cx - m0 * cz;
  const float dz = m0 * cy - m1 * cx;
  const float a = D.alpha, gl = -D.gl;
  k[0] = gl * fmaf(a, dx, cx);
  k[1] = gl * fmaf(a, dy, cy);
  k[2] = gl * fmaf(a, dz, cz);
}


// Reduce the per-thread mode sums of a vector field v (complex weight
// sum_s c_s (v_x - i v_y) u_n) and store them in the partial record.
// Modes are reduced CH at a time: the wave sums of up to 2 CH values, one
// exchange through LDS (two barriers), and thread 0 adds the waves' sums in
// wave order (the same order of additions for every value as one block sum
// per value).  sh: MODE_CHUNK * 2 * (MMI_WG / 64) doubles.
#define MODE_CHUNK 4
template <int CH>
__device__ __forceinline__ void reduce_modes_by(const InstDesc& D, int i, bool mag, float vr, float vi,
                                                MMG double* rec, int slot, double* sh) {
  constexpr int NW = MMI_WG / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int NM = D.N;
  for (int n0 = 0; n0 < NM; n0 += CH) {
    double wr[CH], wi[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      wr[q] = 0.0;
      wi[q] = 0.0;
      if (n0 + q < NM) {
        if (mag) {
          const double u = D.profiled ? (double)gbl(D.u)[(size_t)(n0 + q) * D.ncell + i] : 1.0;
          wr[q] = u * (double)vr;
          wi[q] = u * (double)vi;
        }
        wr[q] = wave_sum(wr[q]);
        wi[q] = wave_sum(wi[q]);
      }
    }
    __syncthreads();
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        sh[(2 * q) * NW + wv] = wr[q];
        sh[(2 * q + 1) * NW + wv] = wi[q];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        if (n0 + q >= NM) break;
        double sr = sh[(2 * q) * NW], si = sh[(2 * q + 1) * NW];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
          sr += sh[(2 * q) * NW + w];
          si += sh[(2 * q + 1) * NW + w];
        }
        rec[slot + 2 * (n0 + q)] = sr;
        rec[slot + 2 * (n0 + q) + 1] = si;
      }
    }
  }
}

// one mode: one value pair per exchange; more: MODE_CHUNK modes per exchange
__device__ __forceinline__ void reduce_modes(const InstDesc& D, int i, bool mag, float vr, float vi,
                                             MMG double* rec, int slot, double* sh) {
  if (D.N <= 1) reduce_modes_by<1>(D, i, mag, vr, vi, rec, slot, sh);
  else reduce_modes_by<MODE_CHUNK>(D, i, mag, vr, vi, rec, slot, sh);
}

// --------------------------------------------------------------- the kernel
// METHOD RK4: ST = 0 run start (reductions only), 1..4 stages.
// METHOD DP45: ST = 1 run start (k1), 2..7 stages.
template <int METHOD, int ST>
__global__ __launch_bounds__(MMI_WG) void k_stage(const InstDesc* __restrict__ descs,
                                                  const int* __restrict__ wg_inst,
                                                  const float2* __restrict__ tw) {
  __shared__ double sh[MODE_CHUNK * 2 * (MMI_WG / 64)];
  extern __shared__ float2 xl[];
  const int lblk = xcd_block();
  const InstDesc& D = descs[wg_inst[lblk]];
  // the control block is only read here (the finalisation kernel writes it)
  const MMG InstCtl* __restrict__ C = gbl(D.ctl);
  if (C->done) return;
  const int lw = zmajor_wg(D, lblk - D.wg0);
  const int nc = D.ncell;
  const int i = lw * MMI_WG + threadIdx.x;
  const bool valid = i < nc;
  const bool mag = valid && (!D.has_geom || gat(gbl(D.geom), i));
  const int cur = C->cur;
  const double h = C->h;
  const int S = D.S;
  using P = DPCoef;
  // control values used below, read once (global stores cannot alias them)
  MMG float* K[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) K[j] = gbl(D.k[(METHOD == MMI_DP45) ? C->slot[j] : j]);
  MMG float* const st0 = gbl(D.st[0]);
  MMG float* const st1 = gbl(D.st[1]);
  float fbc[MMI_MAX_MODES];
  const int NM = D.N;
  for (int n = 0; n < MMI_MAX_MODES; ++n)
    fbc[n] = n < NM ? (float)(D.h0[n] * (D.cphi[n] * C->as[n][0] + D.sphi[n] * C->as[n][1])) : 0.f;

  // only the DP45 stage-2 input is formed on the fly from two fields
  const SrcFixed<METHOD == MMI_DP45 && ST == 2> src(stage_src(D, C, METHOD, ST));

  // x passes done here: the C2R of this stage's convolved rows, and (below)
  // the R2C of the next stage input
  constexpr bool kC2R = (METHOD == MMI_RK4) ? (ST >= 1) : (ST >= 2);
  constexpr bool kR2C = (METHOD == MMI_RK4) ? (ST >= 1) : (ST >= 2 && ST <= 6);
  const bool xf = (kC2R || kR2C) && D.xfused;
  XRows xq;
  float bdv[3] = {0.f, 0.f, 0.f};
  if (xf) {
    xq = xrows_setup(D, lw, xl);
    // the barriers inside the passes order these stores before the line FFTs
    load_twiddles(xq.twl, xq.Px, tw, MMI_WG);
    if (kC2R) xrows_c2r(D, xq, bdv);
  }

  int x = 0, yy = 0, zz = 0;
  if (valid) cell_xyz(D, i, x, yy, zz);

  float m[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  float k[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  if (valid) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (s < S)
#pragma unroll
        for (int c = 0; c < 3; ++c) m[s][c] = src.ld((s * 3 + c) * nc + i);
  }
  // recording for the discrete adjoint: keep every stage input of the step
  // (RK4 stages 1..4; DP45 stages 1..6, and the stage-7 input, the
  // normalised candidate, as stage 1 of the next step)
  const int ri = (ST >= 1) ? C->rec_index : -1;
  if (ST >= 1 && ri >= 0 && valid) {
    const int slot = (METHOD == MMI_DP45 && ST == 7) ? (ri + 1) * D.rec_nstg : ri * D.rec_nstg + (ST - 1);
    MMG float* R = gbl(D.rec_m) + (size_t)slot * (size_t)(3 * S * nc);
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (s < S)
#pragma unroll
        for (int c = 0; c < 3; ++c) R[(s * 3 + c) * nc + i] = m[s][c];
    // and the demag field of this stage input (FFT demag: one sublattice);
    // with FSAL, the next step's stage-1 field is the stage-7 one
    if (D.rec_bd) {
      MMG float* RB = gbl(D.rec_bd) + (size_t)slot * (size_t)(3 * nc);
      const MMG float* bd = gbl(D.bd);
#pragma unroll
      for (int c = 0; c < 3; ++c) RB[c * nc + i] = (kC2R && xf) ? bdv[c] : bd[c * nc + i];
    }
  }
  const bool need_torque = !(METHOD == MMI_RK4 && ST == 0);
  if (need_torque && mag) {
    // cavity feedback sum_n h0_n u_n Re[e^{-i Phi_n} a_n]
    float fb = 0.f;
    if (D.profiled) {
      const MMG float* u = gbl(D.u);
      for (int n = 0; n < NM; ++n) fb = fmaf(fbc[n], u[(size_t)n * nc + i], fb);
    } else {
      for (int n = 0; n < NM; ++n) fb += fbc[n];
    }
    const bool has_bd = D.demag == 2;
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (s < S) torque_at(D, src, i, x, yy, zz, m, s, fb, has_bd, k[s], kC2R ? bdv : nullptr, xf);
  }

  // combination and outputs
  float nx_[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};   // next stage input (or candidate)
  float aux[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};   // DP45 stage-2 input values
  float errm = 0.f;
  bool bad = false;
  bool has_next = true;
  if (valid) {
    const MMG float* Y = gbl(D.y[cur]);
    // every earlier-stage value this stage combines is loaded before any store,
    // so the loads of all components are in flight together
    constexpr bool dp = METHOD == MMI_DP45;
    constexpr bool needY = dp ? (ST >= 2 && ST <= 6) : (ST >= 2);
    constexpr unsigned usedK = dp ? (ST == 2 ? 0x1u : ST == 3 ? 0x3u : ST == 4 ? 0x7u : ST == 5 ? 0xFu
                                     : ST == 6 ? 0x1Du : ST == 7 ? 0x3Du : 0u)
                                  : (ST >= 2 ? 0x1u : 0u);
    float yv[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    float kl[6][2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s >= S) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int idx = (s * 3 + c) * nc + i;
        if (needY) yv[s][c] = gat(Y, idx);
#pragma unroll
        for (int j = 0; j < 6; ++j)
          if (usedK & (1u << j)) kl[j][s][c] = gat(K[j], idx);
      }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (s >= S) continue;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int idx = (s * 3 + c) * nc + i;
        const float kk = k[s][c];
        if (METHOD == MMI_RK4) {
          if (ST == 0) {
            nx_[s][c] = m[s][c];
          } else if (ST == 1) {
            gat(K[0], idx) = kk;
            nx_[s][c] = fmaf((float)(0.5 * h), kk, m[s][c]);
            gat(st0, idx) = nx_[s][c];
          } else if (ST == 2 || ST == 3) {
            const float acc = fmaf(2.f, kk, kl[0][s][c]);
            gat(K[0], idx) = acc;
            const float cc = (float)(ST == 3 ? h : 0.5 * h);
            nx_[s][c] = fmaf(cc, kk, yv[s][c]);
            gat(ST == 2 ? st1 : st0, idx) = nx_[s][c];
          } else {  // ST == 4
            nx_[s][c] = fmaf((float)(h / 6.0), kl[0][s][c] + kk, yv[s][c]);
          }
        } else {
          if (ST == 1) {
            gat(K[0], idx) = kk;
            nx_[s][c] = m[s][c];
          } else if (ST == 2) {
            gat(K[1], idx) = kk;
            aux[s][c] = m[s][c];
            nx_[s][c] = yv[s][c] + ((float)(h * P::a31) * kl[0][s][c] + (float)(h * P::a32) * kk);
            gat(st0, idx) = nx_[s][c];
          } else if (ST == 3) {
            gat(K[2], idx) = kk;
            nx_[s][c] = yv[s][c] + ((float)(h * P::a41) * kl[0][s][c] +
                                  (float)(h * P::a42) * kl[1][s][c] +
                                  (float)(h * P::a43) * kk);
            gat(st1, idx) = nx_[s][c];
          } else if (ST == 4) {
            gat(K[3], idx) = kk;
            nx_[s][c] = yv[s][c] + ((float)(h * P::a51) * kl[0][s][c] +
                                  (float)(h * P::a52) * kl[1][s][c] +
                                  (float)(h * P::a53) * kl[2][s][c] +
                                  (float)(h * P::a54) * kk);
            gat(st0, idx) = nx_[s][c];
          } else if (ST == 5) {
            gat(K[4], idx) = kk;
            nx_[s][c] = yv[s][c] + ((float)(h * P::a61) * kl[0][s][c] +
                                  (float)(h * P::a62) * kl[1][s][c] +
                                  (float)(h * P::a63) * kl[2][s][c] +
                                  (float)(h * P::a64) * kl[3][s][c] +
                                  (float)(h * P::a65) * kk);
            gat(st1, idx) = nx_[s][c];
          } else if (ST == 6) {
            gat(K[5], idx) = kk;
            nx_[s][c] = yv[s][c] + ((float)(h * P::b1) * kl[0][s][c] +
                                  (float)(h * P::b3) * kl[2][s][c] +
                                  (float)(h * P::b4) * kl[3][s][c] +
                                  (float)(h * P::b5) * kl[4][s][c] +
                                  (float)(h * P::b6) * kk);
          } else {  // ST == 7
            gat(K[6], idx) = kk;
            const float e = (float)P::e1 * kl[0][s][c] + (float)P::e3 * kl[2][s][c] +
                            (float)P::e4 * kl[3][s][c] +
                            (float)P::e5 * kl[4][s][c] +
                            (float)P::e6 * kl[5][s][c] + (float)P::e7 * kk;
            const float ae = fabsf(e);
            errm = (ae != ae || errm != errm) ? ae + errm : fmaxf(errm, ae);
          }
        }
      }
      // normalise the step-end state
      const bool step_end = (METHOD == MMI_RK4 && ST == 4) || (METHOD == MMI_DP45 && ST == 6);
      if (step_end) {
        float v0 = nx_[s][0], v1 = nx_[s][1], v2 = nx_[s][2];
        if (mag) {
          const float nrm = sqrtf(v0 * v0 + v1 * v1 + v2 * v2);
          if (ri >= 0) gbl(D.rec_norm)[(size_t)ri * S * nc + s * nc + i] = nrm;
          const float inv = 1.0f / nrm;
          v0 *= inv;
          v1 *= inv;
          v2 *= inv;
        }
        if (!(isfinite(v0) && isfinite(v1) && isfinite(v2))) bad = true;
        nx_[s][0] = v0;
        nx_[s][1] = v1;
        nx_[s][2] = v2;
        MMG float* Yn = gbl(D.y[1 - cur]);
        gat(Yn, (s * 3 + 0) * nc + i) = v0;
        gat(Yn, (s * 3 + 1) * nc + i) = v1;
        gat(Yn, (s * 3 + 2) * nc + i) = v2;
      }
    }
  }
  if (METHOD == MMI_DP45 && ST == 7) has_next = false;

  // ---- per-workgroup partials
  MMG double* rec = gbl(D.partials) + (size_t)lw * MMI_PSTRIDE;
  if (has_next) {
    float vr = 0.f, vi = 0.f;
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (s < S) {
        vr = fmaf(D.csign[s], nx_[s][0], vr);
        vi = fmaf(-D.csign[s], nx_[s][1], vi);
      }
    reduce_modes(D, i, mag, vr, vi, rec, MMI_SLOT_MM, sh);
  }
  if (METHOD == MMI_DP45 && (ST == 1 || ST == 7)) {
    float vr = 0.f, vi = 0.f;
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (s < S) {
        vr = fmaf(D.csign[s], k[s][0], vr);
        vi = fmaf(-D.csign[s], k[s][1], vi);
      }
    reduce_modes(D, i, mag, vr, vi, rec, MMI_SLOT_DMM, sh);
  }
  if (METHOD == MMI_DP45 && ST == 2) {
    float vr = 0.f, vi = 0.f;
#pragma unroll
    for (int s = 0; s < 2; ++s)
      if (s < S) {
        vr = fmaf(D.csign[s], aux[s][0], vr);
        vi = fmaf(-D.csign[s], aux[s][1], vi);
      }
    reduce_modes(D, i, mag, vr, vi, rec, MMI_SLOT_DMM, sh);
  }
  if (METHOD == MMI_DP45 && ST == 7) {
    const double r = block_reduce<true>((double)errm * h, sh);
    if (threadIdx.x == 0) rec[MMI_SLOT_ERR] = r;
  }
  if (METHOD == MMI_RK4 && ST == 4) {
    const double r = block_reduce<true>(bad ? 1.0 : 0.0, sh);
    if (threadIdx.x == 0) rec[MMI_SLOT_BAD] = r;
  }
  if (kR2C && xf) {
    const float v[3] = {valid ? nx_[0][0] : 0.f, valid ? nx_[0][1] : 0.f, valid ? nx_[0][2] : 0.f};
    // the mode reductions above end with workgroup barriers
    xrows_r2c(D, xq, v, has_next && NM > 0);
  }
}

// One workgroup per instance: gather the partial records of the stage
// kernel in a fixed order and run the FP64 cavity step / controller.
template <int METHOD, int ST>
__global__ __launch_bounds__(MMI_WG) void k_final(const InstDesc* __restrict__ descs, int count) {
  __shared__ double tot[MMI_PSTRIDE];
  if ((int)blockIdx.x >= count) return;
  final_body<METHOD, ST>(descs, blockIdx.x, tot);
}

}  // namespace mmk

// explicit launch wrappers --------------------------------------------------
#define MM_STAGE_LAUNCH(M, S)                                                                   \
  case S:                                                                                       \
    if (final_pass)                                                                             \
      MM_LAUNCH((mmk::k_final<M, S>), dim3(count), dim3(MMI_WG), 0, stream, descs, count); \
    else                                                                                        \
      MM_LAUNCH((mmk::k_stage<M, S>), dim3(nblocks), dim3(MMI_WG), lds, stream, descs, wg, tw); \
    break;

// final_pass = false: the cell kernel of a stage; true: its per-instance
// finalisation (count instances).
hipError_t mmk_launch_stage(int method, int stage, bool final_pass, int nblocks, int count,
                            const InstDesc* descs, const int* wg, const float2* tw, size_t lds,
                            hipStream_t stream) {
  if (method == MMI_RK4) {
    switch (stage) {
      MM_STAGE_LAUNCH(MMI_RK4, 0)
      MM_STAGE_LAUNCH(MMI_RK4, 1)
      MM_STAGE_LAUNCH(MMI_RK4, 2)
      MM_STAGE_LAUNCH(MMI_RK4, 3)
      MM_STAGE_LAUNCH(MMI_RK4, 4)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (stage) {
      MM_STAGE_LAUNCH(MMI_DP45, 1)
      MM_STAGE_LAUNCH(MMI_DP45, 2)
      MM_STAGE_LAUNCH(MMI_DP45, 3)
      MM_STAGE_LAUNCH(MMI_DP45, 4)
      MM_STAGE_LAUNCH(MMI_DP45, 5)
      MM_STAGE_LAUNCH(MMI_DP45, 6)
      MM_STAGE_LAUNCH(MMI_DP45, 7)
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

namespace mmk {
// x-forward pass of a stage input that no stage kernel produced (the DP45
// stage-2 input y + h a21 k1, the run-start state), for the instances whose
// x passes run inside the stage kernels: each MMI_WG-cell workgroup of the
// stage grid forms its cells' input and writes the X rows of its own x-rows
// with the stage kernels' R2C.  Other instances return at once.
__global__ __launch_bounds__(MMI_WG) void k_xfwd_cells(const InstDesc* __restrict__ descs,
                                                      const int* __restrict__ wg_inst, int method, int stage,
                                                      const float2* __restrict__ tw) {
  extern __shared__ float2 xl[];
  const int lblk = xcd_block();
  const InstDesc& D = descs[wg_inst[lblk]];
  const MMG InstCtl* __restrict__ C = gbl(D.ctl);
  if (C->done || !D.xfused) return;
  const int lw = lblk - D.wg0;
  const int nc = D.ncell;
  const int i = lw * MMI_WG + threadIdx.x;
  const Src src = stage_src(D, C, method, stage);
  const XRows xq = xrows_setup(D, lw, xl);
  load_twiddles(xq.twl, xq.Px, tw, MMI_WG);
  float v[3] = {0.f, 0.f, 0.f};
  if (i < nc) {
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = src.ld(c * nc + i);
  }
  // the barrier at the start of the pass orders the twiddle stores too
  xrows_r2c(D, xq, v, false);
}

__global__ void k_gather_done(const InstDesc* __restrict__ d, int count, int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    const InstCtl* C = d[i].ctl;
    out[2 * i] = C->done;
    out[2 * i + 1] = C->status;
  }
}
}  // namespace mmk

hipError_t mmk_launch_xfwd_cells(int method, int stage, int nblocks, const InstDesc* descs, const int* wg,
                                 const float2* tw, size_t lds, hipStream_t s) {
  if (method != MMI_RK4 && method != MMI_DP45) return hipErrorInvalidValue;
  MM_LAUNCH(mmk::k_xfwd_cells, dim3(nblocks), dim3(MMI_WG), lds, s, descs, wg, method, stage, tw);
  return hipGetLastError();
}

hipError_t mmk_launch_gather_done(int count, const InstDesc* d, int* out, hipStream_t s) {
  MM_LAUNCH(mmk::k_gather_done, dim3((count + 63) / 64), dim3(64), 0, s, d, count, out);
  return hipGetLastError();
}
