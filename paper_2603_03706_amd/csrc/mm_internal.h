// Internal data structures shared by the host runtime and the device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MMI_MAX_MODES 16
#define MMI_WG 512                    // threads (= cells) per workgroup of the cell kernels
#define MMI_LG_WG 9
#define MMI_PSTRIDE 72             // doubles per workgroup partial record
#define MMI_TW_LEN 1024            // length of the twiddle table (max FFT length)

// partial-record slots (doubles)
//   [0, 2N)       sum of u_n * m^- of the next stage input (re, im)
//   [32, 32+2N)   sum of u_n * k^- of this stage's torque (re, im), trace rate
//   [64]          max-norm of the error estimate (NaN-propagating)
//   [65]          non-finite flag of the written state (RK4 step end)
#define MMI_SLOT_MM 0
#define MMI_SLOT_DMM 32
#define MMI_SLOT_ERR 64
#define MMI_SLOT_BAD 65

enum { MMI_RK4 = 0, MMI_DP45 = 1, MMI_ADJ = 2 };

// Mutable per-instance control block (device memory).
struct InstCtl {
  double t, t_end, h;                 // time, end time, step of the current attempt
  double dt;                          // proposed next step (adaptive)
  double dt_fixed, tol, dt_min, dt_max;
  double dt_min_seen, dt_max_seen;
  long long accepted, rejected;
  int status, done, cur, clipped, last_rejected, pad0;
  int slot[8];                        // physical k-buffer of stage derivative j
  double a[MMI_MAX_MODES][2];         // cavity amplitudes at the step start
  double as[MMI_MAX_MODES][2];        // cavity value feeding the next stage kernel
  double ka[7][MMI_MAX_MODES][2];     // stage derivatives of the cavity
  double mm1[MMI_MAX_MODES][2];       // m^- at the step start
  double dmm1[MMI_MAX_MODES][2];      // d m^-/dt at the step start
  double mm7[MMI_MAX_MODES][2];       // m^- at the candidate (DP45)
  // trace
  long long trace_n, trace_max, trace_steps, trace_stride;
  double trace_t0, trace_dt;
  int trace_on, trace_started;
  // discrete adjoint of fixed-step RK4
  int rec_index;                      // recorded step within the segment (-1: not recording)
  int pad1;
  double adj_h;                       // step of the recorded run
  double adj_t0;                      // time at the start of the segment being reversed
  long long adj_base;                 // recorded-run index of the first step of the segment being reversed
  double la[MMI_MAX_MODES][2];        // adjoint of a at the step start (accumulator)
  double lza[MMI_MAX_MODES][2];       // adjoint of a after the step
  double lka[MMI_MAX_MODES][2];       // adjoint of the current stage derivative of a
  double lmm[MMI_MAX_MODES][2];       // adjoint of m^- at the current stage
  double grad_g[MMI_MAX_MODES];
  double grad_alpha;
  double grad_B0[3];
  // adaptive (DP45) runs: log of the accepted step sizes and their replay
  long long hlog_n;                   // accepted steps logged (beyond the capacity: overflow)
  long long replay_idx, replay_end;   // replay: next logged step, end of the replayed range
  int hlog_on;                        // 1: log the size of every accepted step
  int replay;                         // 1: steps take the logged sizes and are all accepted
  double lmua[6][MMI_MAX_MODES][2];   // DP45 adjoint: mu_a of stage s at [s - 1]
};

// Read-only per-instance descriptor (device memory).
struct InstDesc {
  int nx, ny, nz, ncell;
  int lgnx, lgny;                     // log2 of nx, ny when powers of two, else -1
  int S, N, profiled, has_geom;
  int demag, method, nwg, wg0;
  int split, pad_split;               // RK4 in the operator-split scheme (cavity first, m^- held)
  float cex_x, cex_y, cex_z;          // (2A/Ms)/d^2 per axis
  float cK, ex, ey, ez;               // 2K/Ms and the unit axis
  float B0x, B0y, B0z;
  float nlx, nly, nlz;                // -mu0 Ms n_local
  float BE, gl, alpha;                // B_E, gamma/(1+alpha^2), alpha
  float csign[2];
  float bd_scale;                     // -mu0 Ms / (Px Py Pz)
  double inv_ngeo;
  double gamma;                       // gyromagnetic ratio [rad/(s T)]
  double omega[MMI_MAX_MODES], kappa[MMI_MAX_MODES], g[MMI_MAX_MODES];
  double cphi[MMI_MAX_MODES], sphi[MMI_MAX_MODES], h0[MMI_MAX_MODES];
  // self-Kerr term -i K_n |a_n|^2 a_n of the cavity equation
  int kerr_on, pad_kerr;
  double kerr[MMI_MAX_MODES];
  // direct mode coupling -i sum_m J_nm a_m (J symmetric, zero diagonal)
  int jcpl_on, pad_jcpl;
  double jcpl[MMI_MAX_MODES][MMI_MAX_MODES];
  // Gaussian cavity drive eta_n(t) = A_n exp(-((t - t0_n) / sigma_n)^2 / 2)
  int drive_on, pad_drive;
  double eta_re[MMI_MAX_MODES], eta_im[MMI_MAX_MODES];
  double eta_t0[MMI_MAX_MODES], eta_sigma[MMI_MAX_MODES];
  // degenerate parametric pump -i lam_n e^{-2 i wp_n t} conj(a_n)
  int param_on, pad_param;
  double par_re[MMI_MAX_MODES], par_im[MMI_MAX_MODES], par_wp[MMI_MAX_MODES];
  // device buffers
  float* y[2];                        // state [S][3][cells]
  float* k[7];                        // stage derivatives (RK4 uses k[0] as the running sum)
  float* st[2];                       // stage-input ping-pong
  const uint8_t* geom;                // [cells] or null
  const float* u;                     // [N][cells] or null (uniform)
  float* bd;                          // demag field [3][cells] (FFT demag)
  double* partials;                   // [nwg][MMI_PSTRIDE]
  InstCtl* ctl;
  double* trace_t;                    // [max]
  double* trace_a;                    // [max][N][2]
  double* trace_m;                    // [max][N][2]
  // FFT demag
  float2* fx;                         // [Kx][3][nz][ny]
  float2* fy;                         // [Kx][3][nz][Py] (split path)
  const float* kern;                  // [Kx][6][Pz/2+1][Py/2+1]
  int px, py, pz, kx;
  int xfused;                         // x passes done inside the stage kernels (see k_stage)
  // discrete adjoint (RK4): recorded segment and adjoint fields
  float* rec_m;                       // [K+1][4][S*3*cells] stage inputs of each recorded step
  float* rec_norm;                    // [K][S*cells] |z| before the renormalisation
  float* rec_bd;                      // [K][4][3*cells] demag field of each recorded stage input (FFT demag), or null
  double* rec_a;                      // [K][4][N][2] cavity stage inputs
  float* lam_y;                       // adjoint of the step start state
  float* lam_k;                       // adjoint of the current stage derivative
  float* lam_z;                       // adjoint of the pre-normalisation sum
  float* mu;                          // direct part of the stage VJP
  float* lam_B;                       // adjoint of the effective field
  double* grad_u;                     // [N][cells] accumulator (null: not requested)
  const double* dla_trace;            // [steps+1][N][2] dL/da at every step end of the recorded run, or null
  // adaptive runs (DP45): step log, and the adjoint's extra records
  double* hlog;                       // [hlog_cap] accepted step sizes, negative when clipped onto t_end
  long long hlog_cap;
  int rec_nstg, pad_nstg;             // stage inputs recorded per step: 4 (RK4), 6 (DP45)
  double* rec_t;                      // [K] start time of each recorded step (DP45)
  float* mu_st;                       // [4][S*3*cells] DP45 adjoint: mu of stages 3..6
};

// adjoint partial-record slots (doubles), reusing the forward partials
#define MMI_ASLOT_FB 0                // [N]   sum_s,i lambda_Bx c_s u_n
#define MMI_ASLOT_MM 16               // [2N]  sum u_n G c_s (m_x - i m_y) of the stage state
#define MMI_ASLOT_ALPHA 48            // dL/dalpha contribution
#define MMI_ASLOT_B0 49               // [3] dL/dB0 contribution

// Dormand-Prince 5(4) coefficients.
struct DPCoef {
  static constexpr double c2 = 1.0 / 5, c3 = 3.0 / 10, c4 = 4.0 / 5, c5 = 8.0 / 9;
  static constexpr double a21 = 1.0 / 5;
  static constexpr double a31 = 3.0 / 40, a32 = 9.0 / 40;
  static constexpr double a41 = 44.0 / 45, a42 = -56.0 / 15, a43 = 32.0 / 9;
  static constexpr double a51 = 19372.0 / 6561, a52 = -25360.0 / 2187, a53 = 64448.0 / 6561,
                          a54 = -212.0 / 729;
  static constexpr double a61 = 9017.0 / 3168, a62 = -355.0 / 33, a63 = 46732.0 / 5247,
                          a64 = 49.0 / 176, a65 = -5103.0 / 18656;
  static constexpr double b1 = 35.0 / 384, b3 = 500.0 / 1113, b4 = 125.0 / 192,
                          b5 = -2187.0 / 6784, b6 = 11.0 / 84;
  static constexpr double e1 = 71.0 / 57600, e3 = -71.0 / 16695, e4 = 71.0 / 1920,
                          e5 = -17253.0 / 339200, e6 = 22.0 / 525, e7 = -1.0 / 40;
  // a_qj of the tableau (1-based, j < q <= 6), 0 elsewhere
  __host__ __device__ static constexpr double a(int q, int j) {
    return q == 2 ? (j == 1 ? a21 : 0.0)
         : q == 3 ? (j == 1 ? a31 : j == 2 ? a32 : 0.0)
         : q == 4 ? (j == 1 ? a41 : j == 2 ? a42 : j == 3 ? a43 : 0.0)
         : q == 5 ? (j == 1 ? a51 : j == 2 ? a52 : j == 3 ? a53 : j == 4 ? a54 : 0.0)
         : q == 6 ? (j == 1 ? a61 : j == 2 ? a62 : j == 3 ? a63 : j == 4 ? a64 : j == 5 ? a65 : 0.0)
                  : 0.0;
  }
  // b_j of the 5th-order solution (1-based, j <= 6)
  __host__ __device__ static constexpr double b(int j) {
    return j == 1 ? b1 : j == 3 ? b3 : j == 4 ? b4 : j == 5 ? b5 : j == 6 ? b6 : 0.0;
  }
  // node c_s (1-based)
  __host__ __device__ static constexpr double c(int s) {
    return s == 2 ? c2 : s == 3 ? c3 : s == 4 ? c4 : s == 5 ? c5 : s >= 6 ? 1.0 : 0.0;
  }
};

// Work item of the FFT kernels: (instance, item index within the instance).
struct WorkItem {
  int inst, item;
};
