// Per-instance finalisation of a stage, shared by the stage kernels' own
// finalisation launch and by the FFT kernels that carry it as extra
// workgroups: gather the partial records of the stage kernel in a fixed
// order and run the FP64 cavity step / step-size controller in thread 0.
#pragma once
#include <hip/hip_runtime.h>
#include "mm_internal.h"
#include "kernels_common.h"

namespace mmk {

// Cavity right-hand side of mode n at stage time t, with the stage
// amplitudes of all modes in A: (-i w - kappa) a + i g e^{-i Phi} m^-
// (Eq. (12) with the phase of Eq. (19)), plus, when set, the self-Kerr term
// -i K |a|^2 a, the direct mode coupling -i sum_m J_nm a_m (the H_13 entry of
// Eq. (14)), the degenerate parametric pump -i lam e^{-2 i wp t} conj(a) and
// the Gaussian drive eta_n(t) of Eq. (1).
__device__ __forceinline__ void cav_rhs(const InstDesc& D, int n, double t, const double (*A)[2],
                                        double mr, double mi, double& fr, double& fi) {
  const double ar = A[n][0], ai = A[n][1];
  const double w = D.omega[n], kp = D.kappa[n], g = D.g[n], c = D.cphi[n], s = D.sphi[n];
  fr = -kp * ar + w * ai + g * (s * mr - c * mi);
  fi = -w * ar - kp * ai + g * (s * mi + c * mr);
  if (D.kerr_on) {
    const double q = D.kerr[n] * (ar * ar + ai * ai);
    fr += q * ai;
    fi -= q * ar;
  }
  if (D.jcpl_on) {
    double jr = 0.0, ji = 0.0;
    for (int m = 0; m < D.N; ++m) {
      jr += D.jcpl[n][m] * A[m][0];
      ji += D.jcpl[n][m] * A[m][1];
    }
    fr += ji;
    fi -= jr;
  }
  if (D.param_on) {
    double sn, cs;
    sincos(2.0 * D.par_wp[n] * t, &sn, &cs);
    // Lam = lam e^{-2 i wp t};  -i Lam conj(a) = (Li ar - Lr ai) - i (Lr ar + Li ai)
    const double lr = D.par_re[n] * cs + D.par_im[n] * sn;
    const double li = D.par_im[n] * cs - D.par_re[n] * sn;
    fr += li * ar - lr * ai;
    fi -= lr * ar + li * ai;
  }
  if (D.drive_on) {
    const double x = (t - D.eta_t0[n]) / D.eta_sigma[n];
    const double e = exp(-0.5 * x * x);
    fr += D.eta_re[n] * e;
    fi += D.eta_im[n] * e;
  }
}

// Block-wide reduction over the workgroup in a fixed order, result valid in
// thread 0.
template <bool MAX>
__device__ __forceinline__ double block_reduce(double v, double* sh) {
  constexpr int NW = MMI_WG / 64;
  v = MAX ? wave_max(v) : wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) r = MAX ? nan_max(r, sh[w]) : r + sh[w];
  return r;
}

// The gathers of one finalisation as one list of tasks: mode sums m^-
// (slots MMI_SLOT_MM + 0 .. nmm-1), stage-derivative sums (MMI_SLOT_DMM +
// 0 .. ndmm-1) and, with has_max, the NaN-propagating max of one slot over
// the workgroups; wave w takes tasks w, w + 8, ...  Every slot is combined in
// a fixed order: lane l takes records l, l + 64, ... (eight in flight) and a
// butterfly joins the lanes.  Results (sums times `scale`) go to tot[slot]
// in LDS; the caller synchronises before reading them.
__device__ __forceinline__ void gather_list(const InstDesc& D, int nmm, int ndmm, bool has_max, int max_slot,
                                            double scale, double* tot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const MMG double* P = gbl(D.partials);
  const int ntask = nmm + ndmm + (has_max ? 1 : 0);
  for (int k = wv; k < ntask; k += MMI_WG / 64) {
    const bool mx = has_max && k == ntask - 1;
    const int slot = mx ? max_slot : (k < nmm ? MMI_SLOT_MM + k : MMI_SLOT_DMM + (k - nmm));
    double v = 0.0;
    int w = lane;
    for (; w + 7 * 64 < D.nwg; w += 8 * 64) {
      double p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) p[u] = P[(size_t)(w + u * 64) * MMI_PSTRIDE + slot];
#pragma unroll
      for (int u = 0; u < 8; ++u) v = mx ? nan_max(v, p[u]) : v + p[u];
    }
    for (; w < D.nwg; w += 64) {
      const double p = P[(size_t)w * MMI_PSTRIDE + slot];
      v = mx ? nan_max(v, p) : v + p;
    }
    v = mx ? wave_max(v) : wave_sum(v);
    if (lane == 0) tot[slot] = mx ? v : v * scale;
  }
}

// Append one trace sample (time, a, m^-) from values held in the control
// block / the gathered sums.
__device__ __forceinline__ void record_sample(const InstDesc& D, InstCtl* C, double t,
                                              const double (*a)[2], const double (*mm)[2]) {
  const long long n = C->trace_n;
  if (n >= C->trace_max) return;
  gbl(D.trace_t)[n] = t;
  MMG double* ta = gbl(D.trace_a);
  MMG double* tm = gbl(D.trace_m);
  for (int q = 0; q < D.N; ++q) {
    ta[(n * D.N + q) * 2] = a[q][0];
    ta[(n * D.N + q) * 2 + 1] = a[q][1];
    tm[(n * D.N + q) * 2] = mm[q][0];
    tm[(n * D.N + q) * 2 + 1] = mm[q][1];
  }
  C->trace_n = n + 1;
}

__device__ __forceinline__ double hermite(double th, double h, double y0, double f0, double y1,
                                          double f1) {
  const double t2 = th * th, t3 = t2 * th;
  return (2 * t3 - 3 * t2 + 1) * y0 + (t3 - 2 * t2 + th) * h * f0 + (-2 * t3 + 3 * t2) * y1 +
         (t3 - t2) * h * f1;
}

// next attempted step: min(dt, t_end - t), clipped to land on t_end
__device__ __forceinline__ void plan_step(InstCtl* C, double dt) {
  const double rem = C->t_end - C->t;
  double h = dt;
  int clipped = 0;
  if (h * (1.0 + 1e-9) >= rem) {
    h = rem;
    clipped = 1;
  }
  C->h = h;
  C->clipped = clipped;
}

// replayed step (adaptive runs): the logged size, negative when the step
// was clipped onto the end time; the host keeps replay_idx below the log's
// filled length
__device__ __forceinline__ void plan_replay(const InstDesc& D, InstCtl* C) {
  const double hs = gbl(D.hlog)[C->replay_idx];
  C->h = fabs(hs);
  C->clipped = hs < 0.0 ? 1 : 0;
}

// Operator-split cavity step (the co-simulation scheme of Sec. III B): one
// RK4 step of the cavity ODE over C->h from C->a with m^- held at mh, into
// C->as, which then feeds every LLG stage of the step.  The stage
// derivatives go to C->ka[0..3].
__device__ __forceinline__ void split_cavity(const InstDesc& D, InstCtl* C, const double (*mh)[2]) {
  const int N = D.N;
  const double h = C->h, t = C->t;
  for (int n = 0; n < N; ++n)
    cav_rhs(D, n, t, C->a, mh[n][0], mh[n][1], C->ka[0][n][0], C->ka[0][n][1]);
  for (int s = 1; s <= 3; ++s) {
    const double c = (s == 3) ? h : 0.5 * h;
    for (int n = 0; n < N; ++n) {
      C->as[n][0] = C->a[n][0] + c * C->ka[s - 1][n][0];
      C->as[n][1] = C->a[n][1] + c * C->ka[s - 1][n][1];
    }
    for (int n = 0; n < N; ++n)
      cav_rhs(D, n, t + c, C->as, mh[n][0], mh[n][1], C->ka[s][n][0], C->ka[s][n][1]);
  }
  const double c6 = h / 6.0;
  for (int n = 0; n < N; ++n)
    for (int r = 0; r < 2; ++r)
      C->as[n][r] = C->a[n][r] + c6 * (C->ka[0][n][r] + 2.0 * C->ka[1][n][r] + 2.0 * C->ka[2][n][r] +
                                       C->ka[3][n][r]);
}

// ------------------------------------------------------------ finalisation
// Runs in thread 0 of the last workgroup of an instance, with the gathered
// sums in tot[] (mode sums already scaled by 1/(S N_geo)).
template <int METHOD, int ST>
__device__ void finalize(const InstDesc& D, InstCtl* C, const double* tot) {
  const int N = D.N;
  const double h = C->h;
  // m^- of the stage input written by this kernel
  const double(*mmv)[2] = reinterpret_cast<const double(*)[2]>(tot + MMI_SLOT_MM);
  if (METHOD == MMI_RK4 && ST >= 1 && C->rec_index >= 0) {
    MMG double* ra = gbl(D.rec_a) + ((size_t)C->rec_index * 4 + (ST - 1)) * N * 2;
    for (int n = 0; n < N; ++n) {
      ra[2 * n] = C->as[n][0];
      ra[2 * n + 1] = C->as[n][1];
    }
  }
  if (METHOD == MMI_RK4) {
    if (ST == 0) {  // run start: m^- of y, first derivative, first step
      for (int n = 0; n < N; ++n) {
        if (!D.split)
          cav_rhs(D, n, C->t, C->a, mmv[n][0], mmv[n][1], C->ka[0][n][0], C->ka[0][n][1]);
        C->mm1[n][0] = mmv[n][0];
        C->mm1[n][1] = mmv[n][1];
        C->as[n][0] = C->a[n][0];
        C->as[n][1] = C->a[n][1];
      }
      if (C->trace_on && !C->trace_started) {
        C->trace_started = 1;
        C->trace_t0 = C->t;
        record_sample(D, C, C->t, C->a, C->mm1);
      }
      plan_step(C, C->dt_fixed);
      if (D.split) split_cavity(D, C, mmv);
      return;
    }
    if (D.split && ST <= 3) return;  // the LLG stages keep the new amplitudes
    if (ST <= 3) {
      const double c = (ST == 3) ? h : 0.5 * h;
      for (int n = 0; n < N; ++n) {
        C->as[n][0] = C->a[n][0] + c * C->ka[ST - 1][n][0];
        C->as[n][1] = C->a[n][1] + c * C->ka[ST - 1][n][1];
      }
      // stage ST + 1 sits at t + c (c = h/2, h/2, h)
      for (int n = 0; n < N; ++n)
        cav_rhs(D, n, C->t + c, C->as, mmv[n][0], mmv[n][1], C->ka[ST][n][0], C->ka[ST][n][1]);
      return;
    }
    // ST == 4: step end; the new amplitudes go to C->as first (the split
    // scheme has them there since the step start)
    bool bad = tot[MMI_SLOT_BAD] != 0.0;
    const double c6 = h / 6.0;
    for (int n = 0; n < N; ++n) {
      for (int r = 0; r < 2; ++r) {
        const double v = D.split ? C->as[n][r]
                                 : C->a[n][r] + c6 * (C->ka[0][n][r] + 2.0 * C->ka[1][n][r] +
                                                      2.0 * C->ka[2][n][r] + C->ka[3][n][r]);
        if (!isfinite(v)) bad = true;
        C->as[n][r] = v;
      }
    }
    if (bad) {
      for (int n = 0; n < N; ++n) {
        C->as[n][0] = C->a[n][0];
        C->as[n][1] = C->a[n][1];
      }
      C->status = -6;
      C->done = 1;
      return;
    }
    C->cur ^= 1;
    C->t = C->clipped ? C->t_end : C->t + h;
    C->accepted += 1;
    if (C->rec_index >= 0) C->rec_index += 1;
    C->dt_min_seen = fmin(C->dt_min_seen, h);
    C->dt_max_seen = fmax(C->dt_max_seen, h);
    for (int n = 0; n < N; ++n) {
      C->a[n][0] = C->as[n][0];
      C->a[n][1] = C->as[n][1];
    }
    for (int n = 0; n < N; ++n) {
      if (!D.split)
        cav_rhs(D, n, C->t, C->a, mmv[n][0], mmv[n][1], C->ka[0][n][0], C->ka[0][n][1]);
      C->mm1[n][0] = mmv[n][0];
      C->mm1[n][1] = mmv[n][1];
    }
    if (C->trace_on) {
      C->trace_steps += 1;
      if (C->trace_steps % C->trace_stride == 0) record_sample(D, C, C->t, C->a, C->mm1);
    }
    if (C->t >= C->t_end) {
      C->done = 1;
      return;
    }
    plan_step(C, C->dt_fixed);
    if (D.split) split_cavity(D, C, mmv);
    return;
  }
  // ------------------------------------------------------------- DP45
  using P = DPCoef;
  if (ST == 1) {  // run start (k1 written by the kernel)
    for (int n = 0; n < N; ++n) {
      if (!D.split)
        cav_rhs(D, n, C->t, C->a, mmv[n][0], mmv[n][1], C->ka[0][n][0], C->ka[0][n][1]);
      C->mm1[n][0] = mmv[n][0];
      C->mm1[n][1] = mmv[n][1];
      C->dmm1[n][0] = tot[MMI_SLOT_DMM + 2 * n];
      C->dmm1[n][1] = tot[MMI_SLOT_DMM + 2 * n + 1];
    }
    if (C->trace_on && !C->trace_started) {
      C->trace_started = 1;
      C->trace_t0 = C->t;
      record_sample(D, C, C->t, C->a, C->mm1);
    }
    if (C->replay) plan_replay(D, C);
    else plan_step(C, C->dt);
    const double hh = C->h;
    for (int n = 0; n < N; ++n) {
      C->as[n][0] = C->a[n][0] + hh * P::a21 * C->ka[0][n][0];
      C->as[n][1] = C->a[n][1] + hh * P::a21 * C->ka[0][n][1];
    }
    return;
  }
  // recording for the adjoint: the cavity stage inputs of the step (stage 1:
  // the step-start amplitude) and the step's start time
  if (C->rec_index >= 0 && ST >= 2 && ST <= 6) {
    const int ri = C->rec_index;
    MMG double* ra = gbl(D.rec_a) + ((size_t)ri * 6 + (ST - 1)) * N * 2;
    for (int n = 0; n < N; ++n) {
      ra[2 * n] = C->as[n][0];
      ra[2 * n + 1] = C->as[n][1];
    }
    if (ST == 2) {
      MMG double* r1 = gbl(D.rec_a) + (size_t)ri * 6 * N * 2;
      for (int n = 0; n < N; ++n) {
        r1[2 * n] = C->a[n][0];
        r1[2 * n + 1] = C->a[n][1];
      }
      gbl(D.rec_t)[ri] = C->t;
    }
  }
  if (ST == 2) {
    // ka2 at (a2, m^-(m2)) [m2 sums in the DMM slot], then ka3 at (a3, m^-(m3))
    for (int n = 0; n < N; ++n)
      cav_rhs(D, n, C->t + P::c2 * h, C->as, tot[MMI_SLOT_DMM + 2 * n],
              tot[MMI_SLOT_DMM + 2 * n + 1], C->ka[1][n][0], C->ka[1][n][1]);
  }
  if (ST >= 2 && ST <= 6) {
    // a_{ST+1} = a + h sum_j A[ST+1][j] ka_j
    double A[6];
    // node of stage ST + 1
    const double cn = ST == 2 ? P::c3 : ST == 3 ? P::c4 : ST == 4 ? P::c5 : 1.0;
    if (ST == 2) { A[0] = P::a31; A[1] = P::a32; }
    if (ST == 3) { A[0] = P::a41; A[1] = P::a42; A[2] = P::a43; }
    if (ST == 4) { A[0] = P::a51; A[1] = P::a52; A[2] = P::a53; A[3] = P::a54; }
    if (ST == 5) { A[0] = P::a61; A[1] = P::a62; A[2] = P::a63; A[3] = P::a64; A[4] = P::a65; }
    if (ST == 6) { A[0] = P::b1; A[1] = 0.0; A[2] = P::b3; A[3] = P::b4; A[4] = P::b5; A[5] = P::b6; }
    for (int n = 0; n < N; ++n) {
      double s0 = 0.0, s1 = 0.0;
      for (int j = 0; j < ST; ++j) {
        s0 += A[j] * C->ka[j][n][0];
        s1 += A[j] * C->ka[j][n][1];
      }
      C->as[n][0] = C->a[n][0] + h * s0;
      C->as[n][1] = C->a[n][1] + h * s1;
    }
    for (int n = 0; n < N; ++n) {
      cav_rhs(D, n, C->t + cn * h, C->as, mmv[n][0], mmv[n][1], C->ka[ST][n][0], C->ka[ST][n][1]);
      if (ST == 6) {
        C->mm7[n][0] = mmv[n][0];
        C->mm7[n][1] = mmv[n][1];
      }
    }
    return;
  }
  // ST == 7: error norm, accept / reject, next step
  double err = tot[MMI_SLOT_ERR];
  const double E[7] = {P::e1, 0.0, P::e3, P::e4, P::e5, P::e6, P::e7};
  for (int n = 0; n < N; ++n) {
    double s0 = 0.0, s1 = 0.0;
    for (int j = 0; j < 7; ++j) {
      s0 += E[j] * C->ka[j][n][0];
      s1 += E[j] * C->ka[j][n][1];
    }
    err = nan_max(err, fabs(h * s0));
    err = nan_max(err, fabs(h * s1));
  }
  const double eps = err / C->tol;
  const bool finite = isfinite(eps);
  double fac = 1.0;
  // a replayed step is accepted whatever its error: the logged sequence
  // holds only accepted steps
  if (C->replay || (finite && eps <= 1.0)) {
    // trace: samples in (t, t + h]
    if (C->trace_on) {
      const double t0 = C->t;
      while (C->trace_n < C->trace_max) {
        const double tk = C->trace_t0 + (double)C->trace_n * C->trace_dt;
        if (tk > t0 + h * (1.0 + 1e-12) || tk <= t0) break;
        const double th = (tk - t0) / h;
        const long long q = C->trace_n;
        D.trace_t[q] = tk;
        for (int n = 0; n < N; ++n)
          for (int r = 0; r < 2; ++r) {
            D.trace_a[(q * N + n) * 2 + r] =
                hermite(th, h, C->a[n][r], C->ka[0][n][r], C->as[n][r], C->ka[6][n][r]);
            D.trace_m[(q * N + n) * 2 + r] = hermite(th, h, C->mm1[n][r], C->dmm1[n][r], C->mm7[n][r],
                                                     tot[MMI_SLOT_DMM + 2 * n + r]);
          }
        C->trace_n = q + 1;
      }
    }
    if (C->hlog_on) {
      if (C->hlog_n < D.hlog_cap) gbl(D.hlog)[C->hlog_n] = C->clipped ? -h : h;
      C->hlog_n += 1;
    }
    if (C->rec_index >= 0) C->rec_index += 1;
    if (C->replay) C->replay_idx += 1;
    C->t = C->clipped ? C->t_end : C->t + h;
    C->accepted += 1;
    C->dt_min_seen = fmin(C->dt_min_seen, h);
    C->dt_max_seen = fmax(C->dt_max_seen, h);
    for (int n = 0; n < N; ++n)
      for (int r = 0; r < 2; ++r) {
        C->a[n][r] = C->as[n][r];          // a_7
        C->ka[0][n][r] = C->ka[6][n][r];   // FSAL
        C->mm1[n][r] = C->mm7[n][r];
        C->dmm1[n][r] = tot[MMI_SLOT_DMM + 2 * n + r];
      }
    C->cur ^= 1;
    const int s0 = C->slot[0];
    C->slot[0] = C->slot[6];
    C->slot[6] = s0;
    if (C->replay) {
      if (C->replay_idx >= C->replay_end || C->t >= C->t_end) {
        C->done = 1;
      } else {
        plan_replay(D, C);
        const double hh = C->h;
        for (int n = 0; n < N; ++n) {
          C->as[n][0] = C->a[n][0] + hh * P::a21 * C->ka[0][n][0];
          C->as[n][1] = C->a[n][1] + hh * P::a21 * C->ka[0][n][1];
        }
      }
      return;
    }
    const double fmx = C->last_rejected ? 1.0 : 5.0;
    fac = (eps == 0.0) ? 5.0 : 0.9 * pow(eps, -0.2);
    fac = fmin(fmx, fmax(0.2, fac));
    C->last_rejected = 0;
  } else {
    C->rejected += 1;
    fac = finite ? fmax(0.2, 0.9 * pow(eps, -0.2)) : 0.2;
    fac = fmin(1.0, fac);
    C->last_rejected = 1;
  }
  double dtn = h * fac;
  if (C->dt_max > 0.0) dtn = fmin(dtn, C->dt_max);
  C->dt = dtn;
  if (C->t >= C->t_end) {
    C->done = 1;
  } else if (dtn < C->dt_min) {
    C->status = finite ? -5 : -6;
    C->done = 1;
  }
  plan_step(C, dtn);
  const double hh = C->h;
  for (int n = 0; n < N; ++n) {
    C->as[n][0] = C->a[n][0] + hh * P::a21 * C->ka[0][n][0];
    C->as[n][1] = C->a[n][1] + hh * P::a21 * C->ka[0][n][1];
  }
}

// Body of the finalisation of stage ST of instance `inst` (all MMI_WG
// threads of the workgroup; tot: MMI_PSTRIDE doubles of LDS).
template <int METHOD, int ST>
__device__ void final_body(const InstDesc* __restrict__ descs, int inst, double* tot) {
  const InstDesc& D = descs[inst];
  InstCtl* C = D.ctl;
  if (C->done) return;
  const bool has_next = !(METHOD == MMI_DP45 && ST == 7);
  const double scale = D.inv_ngeo / (double)D.S;
  // the slots this stage needs, dealt to the waves as one list so that the
  // error (or non-finite) slot runs beside the mode sums, not after them
  const int nmm = has_next ? 2 * D.N : 0;
  const int ndmm = (METHOD == MMI_DP45 && (ST == 1 || ST == 2 || ST == 7)) ? 2 * D.N : 0;
  constexpr bool kMax = (METHOD == MMI_DP45 && ST == 7) || (METHOD == MMI_RK4 && ST == 4);
  constexpr int kMaxSlot = METHOD == MMI_DP45 ? MMI_SLOT_ERR : MMI_SLOT_BAD;
  gather_list(D, nmm, ndmm, kMax, kMaxSlot, scale, tot);
  __syncthreads();
  if (threadIdx.x == 0) finalize<METHOD, ST>(D, C, tot);
}

// the same with the method and stage chosen at run time
__device__ __forceinline__ void final_any(int method, int st, const InstDesc* __restrict__ descs, int inst,
                                          double* tot) {
  if (method == MMI_RK4) {
    switch (st) {
      case 0: final_body<MMI_RK4, 0>(descs, inst, tot); break;
      case 1: final_body<MMI_RK4, 1>(descs, inst, tot); break;
      case 2: final_body<MMI_RK4, 2>(descs, inst, tot); break;
      case 3: final_body<MMI_RK4, 3>(descs, inst, tot); break;
      case 4: final_body<MMI_RK4, 4>(descs, inst, tot); break;
      default: break;
    }
  } else {
    switch (st) {
      case 1: final_body<MMI_DP45, 1>(descs, inst, tot); break;
      case 2: final_body<MMI_DP45, 2>(descs, inst, tot); break;
      case 3: final_body<MMI_DP45, 3>(descs, inst, tot); break;
      case 4: final_body<MMI_DP45, 4>(descs, inst, tot); break;
      case 5: final_body<MMI_DP45, 5>(descs, inst, tot); break;
      case 6: final_body<MMI_DP45, 6>(descs, inst, tot); break;
      case 7: final_body<MMI_DP45, 7>(descs, inst, tot); break;
      default: break;
    }
  }
}

}  // namespace mmk
