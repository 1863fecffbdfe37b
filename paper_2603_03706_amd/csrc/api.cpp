// C-ABI of the stepper: argument validation, device memory layout, run loop
// (a HIP graph of K steps replayed until every instance is done), batching
// and per-kernel timing.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "mm_host.h"
#include "launch.h"
#include "mmcav.h"

hipEvent_t* mm_launch_events() {
  thread_local hipEvent_t ev[2] = {nullptr, nullptr};
  return ev;
}

namespace {

thread_local std::string g_err = "no error";

mm_status fail(mm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define MM_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(MM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr double kMu0 = 4e-7 * M_PI;

// Error of a context call made while the context is in an open batch run.
mm_status open_error() { return fail(MM_ERR_STATE, "the instance is in an open batch run (mm_batch_end first)"); }

constexpr int kStepsPerGraph = 32;
// Sub-batches (streams) a new batch runs as; mm_batch_tune may choose more.
constexpr int kDefaultParts = 1;
constexpr int kMaxTunedParts = 3;
constexpr long long kMaxCellsSublattices = 1LL << 26;   // cells x sublattices of one instance
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------ device state
float2* g_twiddle = nullptr;  // e^{-2 pi i m / 1024}, m < 1024
int g_cus = 256;               // compute units of the device (set with the twiddles)
std::mutex g_mu;

struct Spectrum {
  int nx, ny, nz;
  double dx, dy, dz;
  float* dev = nullptr;
  size_t count = 0;
  int refs = 0;
};
std::vector<Spectrum*> g_spectra;

mm_status ensure_twiddles() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_twiddle) return MM_OK;
  std::vector<float2> h(MMI_TW_LEN);
  for (int m = 0; m < MMI_TW_LEN; ++m) {
    const double a = -2.0 * M_PI * m / MMI_TW_LEN;
    h[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  MM_HIP(hipMalloc(&g_twiddle, sizeof(float2) * MMI_TW_LEN));
  MM_HIP(hipMemcpy(g_twiddle, h.data(), sizeof(float2) * MMI_TW_LEN, hipMemcpyHostToDevice));
  MM_HIP(mmk_set_lds_limits());
  int dev = 0;
  MM_HIP(hipGetDevice(&dev));
  MM_HIP(hipDeviceGetAttribute(&g_cus, hipDeviceAttributeMultiprocessorCount, dev));
  return MM_OK;
}

mm_status acquire_spectrum(const mm_params& p, Spectrum** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (Spectrum* s : g_spectra)
    if (s->nx == p.nx && s->ny == p.ny && s->nz == p.nz && s->dx == p.dx && s->dy == p.dy &&
        s->dz == p.dz) {
      s->refs++;
      *out = s;
      return MM_OK;
    }
  std::vector<float> h;
  mmh::kernel_spectrum(p.nx, p.ny, p.nz, p.dx, p.dy, p.dz, h);
  auto* s = new Spectrum{p.nx, p.ny, p.nz, p.dx, p.dy, p.dz};
  s->count = h.size();
  hipError_t e = hipMalloc(&s->dev, sizeof(float) * h.size());
  if (e != hipSuccess) {
    delete s;
    return fail(MM_ERR_OOM, "demag kernel allocation failed");
  }
  e = hipMemcpy(s->dev, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(s->dev);
    delete s;
    return fail(MM_ERR_HIP, std::string("demag kernel upload: ") + hipGetErrorString(e));
  }
  s->refs = 1;
  g_spectra.push_back(s);
  *out = s;
  return MM_OK;
}

void release_spectrum(Spectrum* s) {
  if (!s) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (--s->refs == 0) {
    hipFree(s->dev);
    g_spectra.erase(std::find(g_spectra.begin(), g_spectra.end(), s));
    delete s;
  }
}

// --------------------------------------------------------------- layout
struct Layout {
  size_t ctl, y[2], k[7], st[2], geom, partials, bd, fx, fy, u, fixed_end, total;
  int ncell, nwg, S, px, py, pz, kx;
  bool fft, split;
};

size_t fused_lds(int ny, int nz, int py, int pz, int tk) {
  (void)ny;
  return sizeof(float2) * ((size_t)3 * nz * (py + 1) + (size_t)3 * pz * tk + py + pz) + sizeof(int) * 3 * (size_t)nz;
}

// z-tile width of the fused y-z kernel: the widest power of two <= 16 that
// fits, or 0 when even a single column does not
int fused_tile(int ny, int nz, int py, int pz) {
  for (int tk = std::min(16, py); tk >= 1; tk /= 2)
    if (fused_lds(ny, nz, py, pz, tk) <= 160 * 1024) return tk;
  return 0;
}

bool fused_fits(int ny, int nz, int py, int pz) { return fused_tile(ny, nz, py, pz) > 0; }

// fused y-z with lines in registers: padded y in {16..128}, padded z in {16..64}
size_t reg_lds(int nz, int py, int pz) {
  (void)nz;
  return sizeof(float2) * ((size_t)3 * (pz / 2) * (py + 1) + py + pz + 32) +
         sizeof(float) * 6 * (size_t)(pz / 2 + 1) * (py / 2 + 1);
}
bool reg_fits(int ny, int nz, int py, int pz) {
  (void)ny;
  const bool y_ok = py == 16 || py == 32 || py == 64 || py == 128;
  const bool z_ok = pz == 16 || pz == 32 || pz == 64;
  return y_ok && z_ok && reg_lds(nz, py, pz) <= 160 * 1024;
}

enum {
  PATH_FUSED = MM_YZ_FUSED,
  PATH_REG = MM_YZ_REGISTER,
  PATH_SPLIT = MM_YZ_SPLIT,
  PATH_REG8 = MM_YZ_REGISTER8,
  PATH_XCH = MM_YZ_EXCHANGE,
  PATH_SPLITX = MM_YZ_SPLIT_EXCHANGE
};
// eight lanes per z column: padded z of 32 or 64
bool reg8_fits(int ny, int nz, int py, int pz) { return reg_fits(ny, nz, py, pz) && (pz == 32 || pz == 64); }
// two register passes per line with an LDS exchange: padded y of 16..128, padded z of 32 or 64
size_t xch_lds(int py, int pz) {
  return sizeof(float2) * ((size_t)3 * (pz / 2) * (py + mmk_yzx_pad()) + py + pz) +
         sizeof(float) * 6 * (size_t)(pz / 2 + 1) * (py / 2 + 1) +
         (mmk_yzx_pairs(py, pz) ? sizeof(float2) * 6 * (size_t)pz : 0);
}
// split passes with the two-pass y line transforms: padded y of 16..256
bool splitx_fits(int py) { return mmk_sx_rows(py) > 0; }
size_t splitx_lds_y(int py) { return sizeof(float2) * ((size_t)mmk_sx_rows(py) * (py + 1) + py); }
bool xch_fits(int ny, int nz, int py, int pz) {
  (void)ny, (void)nz;
  const bool y_ok = py == 16 || py == 32 || py == 64 || py == 128;
  return y_ok && (pz == 32 || pz == 64) && xch_lds(py, pz) <= 160 * 1024;
}

// x passes with lines in registers (selected by a tile width Wx of 0): padded x of 16..128
bool xreg_fits(int px) { return px == 16 || px == 32 || px == 64 || px == 128; }
constexpr int XR_ROWS = 128;

// x passes inside the stage kernels: a workgroup must hold at least two whole
// x-rows of each component, so nx is a power of two from 2 to MMI_WG / 2
bool xfuse_fits(int nx) { return nx >= 2 && nx <= MMI_WG / 2 && (nx & (nx - 1)) == 0; }
size_t xfuse_lds(int nx) {
  const int R = MMI_WG / nx, J = R / 2, Px = 2 * nx;
  return sizeof(float2) * ((size_t)3 * Px * (J + 1) + Px);
}
const char* path_name(int p) {
  return p == PATH_REG      ? "reg"
         : p == PATH_REG8   ? "reg8"
         : p == PATH_XCH    ? "xch"
         : p == PATH_SPLIT  ? "split"
         : p == PATH_SPLITX ? "splitx"
                            : "fused";
}

Layout make_layout(const mm_params& p, int n_modes) {
  Layout L{};
  L.ncell = p.nx * p.ny * p.nz;
  L.nwg = (L.ncell + MMI_WG - 1) / MMI_WG;
  L.S = p.sublattices;
  L.fft = p.demag == MM_DEMAG_FFT;
  L.px = mmh::padded(p.nx);
  L.py = mmh::padded(p.ny);
  L.pz = mmh::padded(p.nz);
  L.kx = L.px / 2 + 1;
  L.split = L.fft && !fused_fits(p.ny, p.nz, L.py, L.pz);
  const size_t vec = align_up(sizeof(float) * 3 * L.S * (size_t)L.ncell);
  size_t o = 0;
  L.ctl = o; o += align_up(sizeof(InstCtl));
  for (int i = 0; i < 2; ++i) { L.y[i] = o; o += vec; }
  for (int i = 0; i < 7; ++i) { L.k[i] = o; o += vec; }
  for (int i = 0; i < 2; ++i) { L.st[i] = o; o += vec; }
  L.geom = o; o += p.geometry ? align_up(L.ncell) : 0;
  L.partials = o; o += align_up(sizeof(double) * MMI_PSTRIDE * (size_t)L.nwg);
  if (L.fft) {
    L.bd = o; o += align_up(sizeof(float) * 3 * (size_t)L.ncell);
    L.fx = o; o += align_up(sizeof(float2) * (size_t)L.kx * 3 * p.nz * p.ny);
    L.fy = o; o += align_up(sizeof(float2) * (size_t)L.kx * 3 * p.nz * L.py);   // split path (tunable)
  }
  L.fixed_end = o;
  L.u = o;
  o += align_up(sizeof(float) * (size_t)std::max(0, n_modes) * L.ncell);
  L.total = o;
  return L;
}

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

mm_status validate(const mm_params* p) {
  if (!p) return fail(MM_ERR_ARG, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(MM_ERR_ARG, "grid sizes must be >= 1");
  if ((long long)p->nx * p->ny * p->nz > (1LL << 30)) return fail(MM_ERR_ARG, "grid too large");
  if (!(p->dx > 0 && p->dy > 0 && p->dz > 0) || !std::isfinite(p->dx * p->dy * p->dz))
    return fail(MM_ERR_ARG, "cell sizes must be finite and > 0");
  if (!(p->Ms > 0) || !std::isfinite(p->Ms)) return fail(MM_ERR_ARG, "Ms must be > 0");
  if (!(p->gamma > 0) || !std::isfinite(p->gamma)) return fail(MM_ERR_ARG, "gamma must be > 0");
  if (!(p->alpha >= 0) || !std::isfinite(p->alpha)) return fail(MM_ERR_ARG, "alpha must be >= 0");
  if (!std::isfinite(p->Aex) || !std::isfinite(p->Ku) || !finite3(p->ku_axis) || !finite3(p->B0) ||
      !finite3(p->n_local) || !std::isfinite(p->B_E))
    return fail(MM_ERR_ARG, "non-finite material parameter");
  if (p->demag < MM_DEMAG_NONE || p->demag > MM_DEMAG_FFT) return fail(MM_ERR_ARG, "demag mode out of range");
  if (p->sublattices != 1 && p->sublattices != 2) return fail(MM_ERR_ARG, "sublattices must be 1 or 2");
  // the kernels address an instance's fields with unsigned 32-bit byte
  // offsets (at most 48 bytes per cell and sublattice)
  if ((long long)p->nx * p->ny * p->nz * p->sublattices > kMaxCellsSublattices)
    return fail(MM_ERR_ARG, "grid too large: cells x sublattices must be <= 2^26");
  if (p->demag == MM_DEMAG_FFT) {
    if (p->sublattices != 1) return fail(MM_ERR_ARG, "FFT demag needs sublattices == 1");
    if (mmh::padded(p->nx) > MMI_TW_LEN || mmh::padded(p->ny) > MMI_TW_LEN || mmh::padded(p->nz) > MMI_TW_LEN)
      return fail(MM_ERR_ARG, "FFT demag supports grids up to 512 cells per axis");
  }
  if (p->geometry) {
    long long n = 0;
    const long long nc = (long long)p->nx * p->ny * p->nz;
    for (long long i = 0; i < nc; ++i) n += p->geometry[i] != 0;
    if (n == 0) return fail(MM_ERR_ARG, "geometry has no magnetic cell");
  }
  return MM_OK;
}

}  // namespace

// ================================================================== context
struct mm_ctx {
  mm_params p{};
  std::vector<uint8_t> geom;
  long long n_geo = 0;
  int dev = 0;
  Layout L{};
  // modes
  int N = 0;
  bool modes_set = false;
  bool profiled = false;
  std::vector<double> omega, kappa, g, phi;
  int8_t cs[2] = {1, 1};
  bool nonrecip = false;          // backward coupling g_b set (h0 = 2 g_b / gamma)
  bool kerr_on = false;           // self-Kerr term set
  bool jcpl_on = false;           // direct mode coupling set
  std::vector<double> g_back, kerr, jcpl;
  bool drive_on = false;          // Gaussian cavity drive per mode
  bool param_on = false;          // degenerate parametric pump per mode
  std::vector<double> par_re, par_im, par_wp;
  std::vector<double> drive_re, drive_im, drive_t0, drive_sigma;
  // stepper
  int method = MM_RK4;
  bool split = false;             // MM_RK4_SPLIT: RK4 kernels in the operator-split scheme
  double dt0 = 1e-13, dt_min = 1e-18, dt_max = 0.0;
  // sampling
  double dt_sample = 0.0;
  int64_t max_samples = 0;
  bool sampling_changed = false;
  // device memory
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_bound = false;
  bool dev_ready = false;
  int u_cap = 0;
  float* u_own = nullptr;        // library-owned mode profiles (no bound workspace)
  double* trace = nullptr;       // library-owned trace buffer
  int64_t trace_cap = 0;
  Spectrum* spec = nullptr;
  bool m_set = false;
  hipStream_t user_stream = nullptr;
  mm_batch* solo = nullptr;      // batch of one for mm_run
  mm_batch* open_in = nullptr;   // batch with an open run (mm_batch_begin .. mm_batch_end)
  unsigned version = 1;          // bumps when the descriptor changes
  mm_stats stats{};
  InstDesc desc{};
  // discrete adjoint
  int record_next = -1;            // rec_index for the next run (-1: no recording)
  bool rec_have = false;
  int64_t rec_steps = 0;
  int rec_K = 0, rec_nck = 0;
  double rec_h = 0.0;
  float* ck_m = nullptr;           // checkpoints [nck][S*3*cells]
  std::vector<InstCtl> ck_ctl;
  float* adj_f = nullptr;          // rec_m, rec_norm, lam_y, lam_k, lam_z, mu, lam_B
  double* adj_d = nullptr;         // rec_a, grad_u
  int adj_K = -1, adj_N = -1, adj_nstg = 4;
  bool adj_on = false;             // descriptor carries the adjoint pointers
  double* dla_dev = nullptr;       // dL/da at every step end (mm_adjoint_trace), during the call only
  // adaptive recorded runs (DP45): the accepted step sizes on the device,
  // their host copy, and the end time of the recorded run
  double* hlog_dev = nullptr;
  long long hlog_cap = 0;
  std::vector<double> rec_hs;
  int rec_method = MM_RK4;
  double rec_t_end = 0.0;
};

struct mm_batch {
  std::vector<mm_ctx*> ctxs;
  int method = MM_RK4;
  hipStream_t stream = nullptr;
  InstDesc* d_desc = nullptr;
  int* d_wg = nullptr;
  int total_wg = 0;
  int* d_flags = nullptr;
  int* h_flags = nullptr;
  int h_flags_local[2] = {0, 0};   // host flags of a batch without pinned memory (no-allocation run)
  bool arena = false;              // tables and run buffers carved from a fixed region: nothing to free
  // per-run buffers that replace the context's own (no-allocation run)
  struct RunBufs {
    bool on = false;
    float* k[7] = {};
    float* st[2] = {};
    double* partials = nullptr;
    float* bd = nullptr;
    float2* fx = nullptr;
    float2* fy = nullptr;
    char* lo = nullptr;            // byte range to clear before the run
    size_t bytes = 0;
  } rb;
  std::vector<unsigned> versions;
  struct Group {
    int nx, ny, nz, px, py, pz, kx;
    int path;
    bool xfused = false;   // x passes inside the stage kernels
    int Wx, Wy, TW, TK = 1;
    WorkItem *xf = nullptr, *yz = nullptr, *y = nullptr, *zc = nullptr;
    int n_xf = 0, n_yz = 0, n_y = 0, n_zc = 0;
    size_t lds_xf = 0, lds_xi = 0, lds_yz = 0, lds_y = 0, lds_zc = 0;
    std::vector<int> members;
  };
  std::vector<Group> groups;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec_pow[5] = {};   // 1, 2, 4, 8 and 16 steps (step counts below kStepsPerGraph)
  hipGraph_t graph_pow[5] = {};
  bool open = false;                 // between mm_batch_begin and mm_batch_end
  std::chrono::steady_clock::time_point open_t0{};
  hipGraphExec_t exec_rev = nullptr;
  hipGraph_t graph_rev = nullptr;
  hipEvent_t ev = nullptr;
  std::vector<int> xfused;     // per instance: x passes inside the stage kernels
  size_t stage_lds = 0;        // dynamic LDS of the stage kernels (x passes), 0 if none
  // profiling
  bool profiling = false;
  struct Prof { std::string name; long long launches = 0; double ms = 0.0; double bytes = 0.0; };
  std::vector<Prof> prof;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<int> pending_idx;
  // Non-empty: this batch only dispatches to sub-batches over disjoint sets
  // of its instances, each with its own stream, tables and graphs, whose
  // launch sequences the device runs concurrently.
  std::vector<mm_batch*> parts;
};

namespace {

// A batch is busy while it, one of its parts or one of its instances has an
// open run.
bool batch_busy(const mm_batch* b) {
  if (b->open) return true;
  for (const mm_ctx* c : b->ctxs)
    if (c->open_in) return true;
  return false;
}

mm_status upload_desc(mm_ctx* c);

mm_status set_device(mm_ctx* c) {
  MM_HIP(hipSetDevice(c->dev));
  return MM_OK;
}

void init_ctl(mm_ctx* c, InstCtl& h) {
  std::memset(&h, 0, sizeof(h));
  for (int j = 0; j < 8; ++j) h.slot[j] = j;
  h.dt = c->dt0;
  h.dt_fixed = c->dt0;
  h.dt_min = c->dt_min;
  h.dt_max = c->dt_max;
  h.dt_min_seen = INFINITY;
  h.dt_max_seen = 0.0;
  h.rec_index = -1;
}

mm_status ctl_pull(const mm_ctx* c, InstCtl& h) {
  MM_HIP(hipMemcpy(&h, c->ws + c->L.ctl, sizeof(InstCtl), hipMemcpyDeviceToHost));
  return MM_OK;
}

mm_status ctl_push(mm_ctx* c, const InstCtl& h) {
  MM_HIP(hipMemcpy(c->ws + c->L.ctl, &h, sizeof(InstCtl), hipMemcpyHostToDevice));
  return MM_OK;
}

// Allocate (or adopt the bound workspace) and initialise device state.
mm_status ensure_device(mm_ctx* c) {
  if (c->dev_ready) return MM_OK;
  if (mm_status s = set_device(c)) return s;
  if (mm_status s = ensure_twiddles()) return s;
  if (!c->ws_bound) {
    const Layout L = make_layout(c->p, 0);
    void* p = nullptr;
    if (hipMalloc(&p, L.total) != hipSuccess) return fail(MM_ERR_OOM, "device allocation failed");
    c->ws = (char*)p;
    c->ws_bytes = L.total;
  }
  c->L = make_layout(c->p, c->u_cap);
  char* w = c->ws;
  MM_HIP(hipMemset(w, 0, c->L.fixed_end));
  if (c->p.geometry) MM_HIP(hipMemcpy(w + c->L.geom, c->geom.data(), c->geom.size(), hipMemcpyHostToDevice));
  if (c->p.demag == MM_DEMAG_FFT) {
    if (mm_status s = acquire_spectrum(c->p, &c->spec)) return s;
  }
  InstCtl h;
  init_ctl(c, h);
  if (mm_status s = ctl_push(c, h)) return s;
  c->dev_ready = true;
  return upload_desc(c);
}

// Build the host copy of the descriptor (device pointers included).
mm_status upload_desc(mm_ctx* c) {
  InstDesc& d = c->desc;
  std::memset(&d, 0, sizeof(d));
  const mm_params& p = c->p;
  const Layout& L = c->L;
  d.nx = p.nx; d.ny = p.ny; d.nz = p.nz; d.ncell = L.ncell;
  auto lg_pow2 = [](int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return (1 << l) == n ? l : -1;
  };
  d.lgnx = lg_pow2(p.nx);
  d.lgny = lg_pow2(p.ny);
  d.S = p.sublattices; d.N = c->N; d.profiled = c->profiled ? 1 : 0; d.has_geom = p.geometry ? 1 : 0;
  d.demag = p.demag; d.method = c->method; d.nwg = L.nwg; d.wg0 = 0;
  d.split = c->split ? 1 : 0;
  const double cex = 2.0 * p.Aex / p.Ms;
  d.cex_x = p.nx > 1 ? (float)(cex / (p.dx * p.dx)) : 0.f;
  d.cex_y = p.ny > 1 ? (float)(cex / (p.dy * p.dy)) : 0.f;
  d.cex_z = p.nz > 1 ? (float)(cex / (p.dz * p.dz)) : 0.f;
  const double en = std::sqrt(p.ku_axis[0] * p.ku_axis[0] + p.ku_axis[1] * p.ku_axis[1] + p.ku_axis[2] * p.ku_axis[2]);
  d.cK = en > 0 ? (float)(2.0 * p.Ku / p.Ms) : 0.f;
  d.ex = en > 0 ? (float)(p.ku_axis[0] / en) : 0.f;
  d.ey = en > 0 ? (float)(p.ku_axis[1] / en) : 0.f;
  d.ez = en > 0 ? (float)(p.ku_axis[2] / en) : 0.f;
  d.B0x = (float)p.B0[0]; d.B0y = (float)p.B0[1]; d.B0z = (float)p.B0[2];
  d.nlx = (float)(-kMu0 * p.Ms * p.n_local[0]);
  d.nly = (float)(-kMu0 * p.Ms * p.n_local[1]);
  d.nlz = (float)(-kMu0 * p.Ms * p.n_local[2]);
  d.BE = (float)p.B_E;
  d.gl = (float)(p.gamma / (1.0 + p.alpha * p.alpha));
  d.alpha = (float)p.alpha;
  d.csign[0] = c->cs[0];
  d.csign[1] = c->cs[1];
  d.px = L.px; d.py = L.py; d.pz = L.pz; d.kx = L.kx;
  d.bd_scale = (float)(-kMu0 * p.Ms / ((double)L.px * L.py * L.pz));
  d.inv_ngeo = 1.0 / (double)c->n_geo;
  d.gamma = p.gamma;
  for (int n = 0; n < c->N; ++n) {
    d.omega[n] = c->omega[n];
    d.kappa[n] = c->kappa[n];
    d.g[n] = c->g[n];
    d.cphi[n] = std::cos(c->phi[n]);
    d.sphi[n] = std::sin(c->phi[n]);
    d.h0[n] = 2.0 * (c->nonrecip ? c->g_back[n] : c->g[n]) / p.gamma;
  }
  d.kerr_on = c->kerr_on ? 1 : 0;
  if (c->kerr_on)
    for (int n = 0; n < c->N; ++n) d.kerr[n] = c->kerr[n];
  d.jcpl_on = c->jcpl_on ? 1 : 0;
  if (c->jcpl_on)
    for (int n = 0; n < c->N; ++n)
      for (int m = 0; m < c->N; ++m) d.jcpl[n][m] = c->jcpl[(size_t)n * c->N + m];
  d.param_on = c->param_on ? 1 : 0;
  if (c->param_on)
    for (int n = 0; n < c->N; ++n) {
      d.par_re[n] = c->par_re[n];
      d.par_im[n] = c->par_im[n];
      d.par_wp[n] = c->par_wp[n];
    }
  d.drive_on = c->drive_on ? 1 : 0;
  if (c->drive_on)
    for (int n = 0; n < c->N; ++n) {
      d.eta_re[n] = c->drive_re[n];
      d.eta_im[n] = c->drive_im[n];
      d.eta_t0[n] = c->drive_t0[n];
      d.eta_sigma[n] = c->drive_sigma[n];
    }
  char* w = c->ws;
  for (int i = 0; i < 2; ++i) d.y[i] = (float*)(w + L.y[i]);
  for (int i = 0; i < 7; ++i) d.k[i] = (float*)(w + L.k[i]);
  for (int i = 0; i < 2; ++i) d.st[i] = (float*)(w + L.st[i]);
  d.geom = p.geometry ? (const uint8_t*)(w + L.geom) : nullptr;
  d.u = c->profiled ? (c->ws_bound ? (const float*)(w + L.u) : c->u_own) : nullptr;
  d.partials = (double*)(w + L.partials);
  d.ctl = (InstCtl*)(w + L.ctl);
  if (c->trace) {
    d.trace_t = c->trace;
    d.trace_a = c->trace + c->trace_cap;
    d.trace_m = c->trace + c->trace_cap * (1 + 2 * (int64_t)std::max(1, c->N));
  }
  if (L.fft) {
    d.bd = (float*)(w + L.bd);
    d.fx = (float2*)(w + L.fx);
    d.fy = (float2*)(w + L.fy);
    d.kern = c->spec ? c->spec->dev : nullptr;
  }
  d.hlog = c->hlog_dev;
  d.hlog_cap = c->hlog_cap;
  d.rec_nstg = c->method == MM_DP45 ? 6 : 4;
  if (c->adj_on) {
    const size_t vec = (size_t)3 * p.sublattices * L.ncell;
    const int K = c->adj_K, ns = d.rec_nstg;
    const bool dp = c->method == MM_DP45;
    float* f = c->adj_f;
    d.rec_m = f; f += (size_t)(K + 1) * ns * vec;
    d.rec_norm = f; f += (size_t)K * p.sublattices * L.ncell;
    d.lam_y = f; f += vec;
    d.lam_k = f; f += vec;
    d.lam_z = f; f += vec;
    d.mu = f; f += vec;
    d.lam_B = f; f += vec;
    d.rec_bd = L.fft ? f : nullptr;
    if (L.fft) f += (size_t)(K + (dp ? 1 : 0)) * ns * 3 * L.ncell;
    d.mu_st = dp ? f : nullptr;
    d.rec_a = c->adj_d;
    d.grad_u = c->adj_d + (size_t)K * ns * std::max(1, c->N) * 2;
    d.rec_t = dp ? d.grad_u + (size_t)std::max(1, c->N) * L.ncell : nullptr;
    d.dla_trace = c->dla_dev;
  }
  c->version++;
  return MM_OK;
}

// ------------------------------------------------------------- batches
double algorithmic_bytes(const mm_batch* b, const std::string& name);

// Device memory for a batch's tables and per-run buffers: hipMalloc
// (MALLOC), carved in order from a fixed region (CARVE: the no-allocation
// run), or only counted (COUNT: the bytes a carve would take).
struct DevArena {
  enum Mode { MALLOC, CARVE, COUNT } mode = MALLOC;
  char* base = nullptr;
  size_t cap = 0, off = 0;
  mm_status take(size_t bytes, void** out) {
    if (mode == MALLOC) {
      if (hipMalloc(out, bytes) != hipSuccess) return fail(MM_ERR_OOM, "device allocation failed");
      return MM_OK;
    }
    const size_t o = (off + 255) & ~(size_t)255;
    off = o + bytes;
    if (mode == COUNT) {
      *out = (void*)(uintptr_t)256;          // never dereferenced
      return MM_OK;
    }
    if (off > cap) return fail(MM_ERR_ARG, "instance does not fit the no-allocation scratch");
    *out = base + o;
    return MM_OK;
  }
  // take `bytes` and copy `src` there (host to device, synchronous)
  mm_status upload(void** dst, const void* src, size_t bytes) {
    if (mm_status s = take(bytes, dst)) return s;
    if (mode != COUNT) MM_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return MM_OK;
  }
};

// Work tables and LDS sizes of one FFT group for its current tile choice.
mm_status build_group(mm_batch::Group& g, DevArena* arena = nullptr) {
  DevArena heap;
  if (!arena) arena = &heap;
  if (arena->mode == DevArena::MALLOC)
    for (WorkItem** p : {&g.xf, &g.yz, &g.y, &g.zc})
      if (*p) {
        hipFree(*p);
        *p = nullptr;
      }
  const int rows = 3 * g.ny * g.nz;
  const int tiles_x = g.Wx == 0 ? (rows + XR_ROWS - 1) / XR_ROWS : (rows + 2 * g.Wx - 1) / (2 * g.Wx);
  std::vector<WorkItem> xf, yz, yy, zc;
  const int ylines = g.kx * 3 * g.nz;
  const bool sx = g.path == PATH_SPLITX;
  const int wy = sx ? mmk_sx_rows(g.py) : g.Wy;
  const int tiles_y = (ylines + wy - 1) / wy;
  const int ky_tiles = (g.py + g.TW - 1) / g.TW;
  // The two-pass kernel may take planes 0 and Px/2 of an instance as one
  // item (item 0), which takes longer than the others: these items go first,
  // so that none of them starts in the launch's last round.
  const bool pairs = g.path == PATH_XCH && g.kx > 1 && mmk_yzx_pairs(g.py, g.pz);
  if (pairs)
    for (int m : g.members) yz.push_back({m, 0});
  for (int m : g.members) {
    for (int t = 0; t < tiles_x; ++t) xf.push_back({m, t});
    if (g.path != PATH_SPLIT && !sx) {
      for (int k = pairs ? 1 : 0; k < (pairs ? g.kx - 1 : g.kx); ++k) yz.push_back({m, k});
    } else {
      for (int t = 0; t < tiles_y; ++t) yy.push_back({m, t});
      for (int k = 0; k < g.kx * ky_tiles; ++k) zc.push_back({m, k});
    }
  }
  auto up = [&](std::vector<WorkItem>& v, WorkItem** dst, int* cnt) -> mm_status {
    *cnt = (int)v.size();
    if (v.empty()) return MM_OK;
    return arena->upload((void**)dst, v.data(), sizeof(WorkItem) * v.size());
  };
  if (mm_status s = up(xf, &g.xf, &g.n_xf)) return s;
  if (mm_status s = up(yz, &g.yz, &g.n_yz)) return s;
  if (mm_status s = up(yy, &g.y, &g.n_y)) return s;
  if (mm_status s = up(zc, &g.zc, &g.n_zc)) return s;
  g.lds_xf = g.Wx == 0 ? 0 : sizeof(float2) * ((size_t)g.px * (g.Wx + 1) + g.px);
  g.lds_xi = g.Wx == 0 ? 0 : sizeof(float2) * ((size_t)g.px * (g.Wx + 1) + (size_t)g.kx * 2 * g.Wx + g.px);
  g.lds_yz = g.path == PATH_XCH                             ? xch_lds(g.py, g.pz)
             : (g.path == PATH_REG || g.path == PATH_REG8) ? reg_lds(g.nz, g.py, g.pz)
                                                           : fused_lds(g.ny, g.nz, g.py, g.pz, g.TK);
  g.lds_y = sx ? splitx_lds_y(g.py) : sizeof(float2) * ((size_t)g.py * (g.Wy + 1) + g.py);
  g.lds_zc = sizeof(float2) * ((size_t)g.pz * 3 * g.TW + g.pz);
  return MM_OK;
}

// Per-instance x-pass placement and the stage kernels' LDS, from the groups.
void batch_xfused(mm_batch* b) {
  b->xfused.assign(b->ctxs.size(), 0);
  b->stage_lds = 0;
  for (auto& g : b->groups)
    if (g.xfused) {
      for (int m : g.members) b->xfused[m] = 1;
      b->stage_lds = std::max(b->stage_lds, xfuse_lds(g.nx));
    }
}

InstDesc batch_desc(const mm_batch* b, int i) {
  InstDesc d = b->ctxs[i]->desc;
  int wg0 = 0;
  for (int j = 0; j < i; ++j) wg0 += b->ctxs[j]->desc.nwg;
  d.wg0 = wg0;
  d.xfused = b->xfused.empty() ? 0 : b->xfused[i];
  if (b->rb.on) {
    for (int j = 0; j < 7; ++j) d.k[j] = b->rb.k[j];
    for (int j = 0; j < 2; ++j) d.st[j] = b->rb.st[j];
    d.partials = b->rb.partials;
    if (d.bd) d.bd = b->rb.bd;
    if (d.fx) d.fx = b->rb.fx;
    if (d.fy) d.fy = b->rb.fy;
  }
  return d;
}

mm_status upload_batch_descs(mm_batch* b, bool count_only = false) {
  const int n = (int)b->ctxs.size();
  std::vector<InstDesc> descs(n);
  for (int i = 0; i < n; ++i) descs[i] = batch_desc(b, i);
  if (!count_only) MM_HIP(hipMemcpy(b->d_desc, descs.data(), sizeof(InstDesc) * n, hipMemcpyHostToDevice));
  for (int i = 0; i < n; ++i) b->versions[i] = b->ctxs[i]->version;
  return MM_OK;
}

// Per-run buffers of the batch's single instance (stage derivatives, stage
// inputs, workgroup partials and, with FFT demag, the demag field and the
// spectra) carved from the arena instead of the context's workspace.
mm_status carve_run_buffers(mm_batch* b, DevArena* ar) {
  const mm_ctx* c = b->ctxs[0];
  const Layout& L = c->L;
  const size_t vec = sizeof(float) * 3 * L.S * (size_t)L.ncell;
  mm_batch::RunBufs& r = b->rb;
  const size_t start = ar->off;
  for (int j = 0; j < 7; ++j)
    if (mm_status s = ar->take(vec, (void**)&r.k[j])) return s;
  for (int j = 0; j < 2; ++j)
    if (mm_status s = ar->take(vec, (void**)&r.st[j])) return s;
  if (mm_status s = ar->take(sizeof(double) * MMI_PSTRIDE * (size_t)L.nwg, (void**)&r.partials)) return s;
  if (L.fft) {
    const mm_params& p = c->p;
    if (mm_status s = ar->take(sizeof(float) * 3 * (size_t)L.ncell, (void**)&r.bd)) return s;
    if (mm_status s = ar->take(sizeof(float2) * (size_t)L.kx * 3 * p.nz * p.ny, (void**)&r.fx)) return s;
    // the spectra of the y pass exist only on the split y-z paths
    if (!b->groups.empty() && (b->groups[0].path == PATH_SPLIT || b->groups[0].path == PATH_SPLITX))
      if (mm_status s = ar->take(sizeof(float2) * (size_t)L.kx * 3 * p.nz * L.py, (void**)&r.fy)) return s;
  }
  r.on = true;
  r.lo = (char*)r.k[0];
  r.bytes = ar->off - ((start + 255) & ~(size_t)255);
  return MM_OK;
}

// Tables, descriptors and streams of a batch.  With an arena (one instance
// only), every device buffer, the per-run buffers included, is carved from it
// and no stream or event is created: the caller sets b->stream.
mm_status batch_build(mm_batch* b, DevArena* arena = nullptr) {
  DevArena heap;
  DevArena* ar = arena ? arena : &heap;
  const bool counting = ar->mode == DevArena::COUNT;
  const int n = (int)b->ctxs.size();
  std::vector<int> wg;
  for (int i = 0; i < n; ++i)
    for (int w = 0; w < b->ctxs[i]->desc.nwg; ++w) wg.push_back(i);
  b->total_wg = (int)wg.size();
  b->arena = arena != nullptr;
  if (mm_status s = ar->take(sizeof(InstDesc) * n, (void**)&b->d_desc)) return s;
  if (mm_status s = ar->upload((void**)&b->d_wg, wg.data(), sizeof(int) * wg.size())) return s;
  if (mm_status s = ar->take(sizeof(int) * 2 * n, (void**)&b->d_flags)) return s;
  if (arena)
    b->h_flags = b->h_flags_local;
  else
    MM_HIP(hipHostMalloc((void**)&b->h_flags, sizeof(int) * 2 * n, hipHostMallocDefault));
  b->versions.resize(n);
  // FFT groups by grid shape
  for (int i = 0; i < n; ++i) {
    const mm_ctx* c = b->ctxs[i];
    if (c->p.demag != MM_DEMAG_FFT) continue;
    mm_batch::Group* g = nullptr;
    for (auto& q : b->groups)
      if (q.nx == c->p.nx && q.ny == c->p.ny && q.nz == c->p.nz) g = &q;
    if (!g) {
      b->groups.emplace_back();
      g = &b->groups.back();
      g->nx = c->p.nx; g->ny = c->p.ny; g->nz = c->p.nz;
      g->px = c->L.px; g->py = c->L.py; g->pz = c->L.pz; g->kx = c->L.kx;
      g->path = xch_fits(g->ny, g->nz, g->py, g->pz)    ? PATH_XCH
                : reg8_fits(g->ny, g->nz, g->py, g->pz) ? PATH_REG8
                : reg_fits(g->ny, g->nz, g->py, g->pz)  ? PATH_REG
                : c->L.split && splitx_fits(g->py)     ? PATH_SPLITX
                : c->L.split                           ? PATH_SPLIT
                                                       : PATH_FUSED;
    }
    g->members.push_back(i);
  }
  for (auto& g : b->groups) {
    g.Wx = std::max(1, std::min(16, 1024 / g.px));
    g.Wy = std::max(1, std::min(64, 2048 / g.py));
    int tw = 1;
    while (tw * 2 <= 16 && 3 * (tw * 2) * g.pz <= 2048) tw *= 2;
    g.TW = tw;
    g.TK = std::max(1, fused_tile(g.ny, g.nz, g.py, g.pz));
    g.xfused = xfuse_fits(g.nx);
    for (int m : g.members)
      if (b->ctxs[m]->p.sublattices != 1) g.xfused = false;
    if (mm_status s = build_group(g, ar)) return s;
  }
  batch_xfused(b);
  if (arena)
    if (mm_status s = carve_run_buffers(b, ar)) return s;
  if (mm_status s = upload_batch_descs(b, counting)) return s;
  if (arena) return MM_OK;
  MM_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
  MM_HIP(hipEventCreateWithFlags(&b->ev, hipEventDisableTiming));
  return MM_OK;
}

mm_status refresh_descs(mm_batch* b) {
  for (size_t i = 0; i < b->ctxs.size(); ++i) {
    if (b->versions[i] == b->ctxs[i]->version) continue;
    const InstDesc d = batch_desc(b, (int)i);
    MM_HIP(hipMemcpy(b->d_desc + i, &d, sizeof(InstDesc), hipMemcpyHostToDevice));
    b->versions[i] = b->ctxs[i]->version;
  }
  return MM_OK;
}

// Launch wrapper that times the launch when profiling.
template <class F>
mm_status launch(mm_batch* b, const char* name, F&& f) {
  size_t idx = 0;
  if (b->profiling) {
    for (; idx < b->prof.size(); ++idx)
      if (b->prof[idx].name == name) break;
    if (idx == b->prof.size()) {
      b->prof.push_back({name});
      b->prof.back().bytes = algorithmic_bytes(b, name);
    }
    hipEvent_t e0, e1;
    // default events: the system-scope release at the end of the kernel
    // writes its dirty lines back, so per-dispatch write counters see them
    MM_HIP(hipEventCreate(&e0));
    MM_HIP(hipEventCreate(&e1));
    // recorded by the runtime at the kernel's own start and end
    hipEvent_t* ev = mm_launch_events();
    ev[0] = e0;
    ev[1] = e1;
    const hipError_t err = f();
    ev[0] = nullptr;
    ev[1] = nullptr;
    MM_HIP(err);
    b->pending.push_back({e0, e1});
    b->pending_idx.push_back((int)idx);
    return MM_OK;
  }
  MM_HIP(f());
  return MM_OK;
}

bool any_xfused(const mm_batch* b) {
  for (const auto& g : b->groups)
    if (g.xfused) return true;
  return false;
}

// Demag convolution of the given stage's input.  For groups whose x passes
// run inside the stage kernels, the x-forward pass is enqueued only when
// `fwd` (the input was not produced by a stage kernel) and the x-inverse
// pass only when `inv` (the consuming kernel does not transform itself).
// final_st >= 0: the finalisation of that stage of the batch's method rides
// on the first group's y-z launch (see merge_final).
mm_status enqueue_demag(mm_batch* b, int stage, int method = -1, bool fwd = true, bool inv = true,
                        int final_st = -1) {
  if (method < 0) method = b->method;
  const int nfinal = final_st >= 0 ? (int)b->ctxs.size() : 0;
  // x-forward of the instances whose x passes run in the stage kernels: one
  // launch on the stage grid (forward stepping; the adjoint's inputs go
  // through the x kernels of their groups)
  const bool cells_fwd = fwd && method != MMI_ADJ && any_xfused(b);
  if (cells_fwd)
    if (mm_status s = launch(b, "fft_x_forward", [&] {
          return mmk_launch_xfwd_cells(method, stage, b->total_wg, b->d_desc, b->d_wg, g_twiddle, b->stage_lds,
                                       b->stream);
        }))
      return s;
  for (auto& g : b->groups) {
    const bool first = &g == &b->groups[0];
    if (!g.xfused || (fwd && !cells_fwd))
    if (mm_status s = launch(b, "fft_x_forward", [&] {
          if (g.Wx == 0)
            return mmk_launch_fft_xr(1, g.px / 4, g.n_xf, b->d_desc, g.xf, method, stage, g_twiddle, b->stream);
          return mmk_launch_fft_xf(g.Wx, g.n_xf, g.lds_xf, b->d_desc, g.xf, method, stage, g_twiddle, b->stream);
        }))
      return s;
    if (g.path == PATH_REG8 || g.path == PATH_XCH) {
      if (mm_status s = launch(b, "fft_yz_convolve", [&] {
            auto f = g.path == PATH_XCH ? mmk_launch_fft_yzx : mmk_launch_fft_yz8;
            return f(g.py / 4, g.pz / 4, g.n_yz, g.lds_yz, b->d_desc, g.yz, g_twiddle, b->stream,
                     first ? nfinal : 0, b->method, final_st);
          }))
        return s;
    } else if (g.path == PATH_REG) {
      if (mm_status s = launch(b, "fft_yz_convolve", [&] {
            return mmk_launch_fft_yzr(g.py / 4, g.pz / 4, g.n_yz, g.lds_yz, b->d_desc, g.yz, g_twiddle, b->stream);
          }))
        return s;
    } else if (g.path == PATH_FUSED) {
      if (mm_status s = launch(b, "fft_yz_convolve", [&] {
            return mmk_launch_fft_yz(g.TK, g.n_yz, g.lds_yz, b->d_desc, g.yz, g_twiddle, b->stream);
          }))
        return s;
    } else if (g.path == PATH_SPLITX) {
      if (mm_status s = launch(b, "fft_y_forward", [&] {
            return mmk_launch_fft_ysx(-1, g.py, g.n_y, g.lds_y, b->d_desc, g.y, g_twiddle, b->stream,
                                      first ? nfinal : 0, b->method, final_st);
          }))
        return s;
      if (mm_status s = launch(b, "fft_z_convolve", [&] {
            return mmk_launch_fft_zc(g.TW, g.n_zc, g.lds_zc, b->d_desc, g.zc, g_twiddle, b->stream);
          }))
        return s;
      if (mm_status s = launch(b, "fft_y_inverse", [&] {
            return mmk_launch_fft_ysx(1, g.py, g.n_y, g.lds_y, b->d_desc, g.y, g_twiddle, b->stream);
          }))
        return s;
    } else {
      if (mm_status s = launch(b, "fft_y_forward", [&] {
            return mmk_launch_fft_y(-1, g.Wy, g.n_y, g.lds_y, b->d_desc, g.y, g_twiddle, b->stream);
          }))
        return s;
      if (mm_status s = launch(b, "fft_z_convolve", [&] {
            return mmk_launch_fft_zc(g.TW, g.n_zc, g.lds_zc, b->d_desc, g.zc, g_twiddle, b->stream);
          }))
        return s;
      if (mm_status s = launch(b, "fft_y_inverse", [&] {
            return mmk_launch_fft_y(1, g.Wy, g.n_y, g.lds_y, b->d_desc, g.y, g_twiddle, b->stream);
          }))
        return s;
    }
    if (!g.xfused || inv)
    if (mm_status s = launch(b, "fft_x_inverse", [&] {
          if (g.Wx == 0) return mmk_launch_fft_xr(-1, g.px / 4, g.n_xf, b->d_desc, g.xf, 0, 0, g_twiddle, b->stream);
          return mmk_launch_fft_xi(g.Wx, g.n_xf, g.lds_xi, b->d_desc, g.xf, g_twiddle, b->stream);
        }))
      return s;
  }
  return MM_OK;
}

const char* stage_name(int method, int st) {
  static const char* rk[] = {"stage_rk4_start", "stage_rk4_1", "stage_rk4_2", "stage_rk4_3", "stage_rk4_4"};
  static const char* dp[] = {"", "stage_dp45_1", "stage_dp45_2", "stage_dp45_3", "stage_dp45_4",
                             "stage_dp45_5", "stage_dp45_6", "stage_dp45_7"};
  return method == MM_RK4 ? rk[st] : dp[st];
}

const char* final_name(int method, int st) {
  static const char* rk[] = {"final_rk4_start", "final_rk4_1", "final_rk4_2", "final_rk4_3", "final_rk4_4"};
  static const char* dp[] = {"", "final_dp45_1", "final_dp45_2", "final_dp45_3", "final_dp45_4",
                             "final_dp45_5", "final_dp45_6", "final_dp45_7"};
  return method == MM_RK4 ? rk[st] : dp[st];
}

// Stage kernel, then (unless the next y-z launch carries it) its finalisation.
mm_status enqueue_stage(mm_batch* b, int st, bool with_final = true) {
  const int n = (int)b->ctxs.size();
  if (mm_status s = launch(b, stage_name(b->method, st), [&] {
        return mmk_launch_stage(b->method, st, false, b->total_wg, n, b->d_desc, b->d_wg, g_twiddle,
                                b->stage_lds, b->stream);
      }))
    return s;
  if (!with_final) return MM_OK;
  return launch(b, final_name(b->method, st), [&] {
    return mmk_launch_stage(b->method, st, true, b->total_wg, n, b->d_desc, b->d_wg, g_twiddle, 0, b->stream);
  });
}

// x-forward pass of the state for groups whose x passes run in the stage kernels
mm_status enqueue_x_forward(mm_batch* b, int stage) {
  if (!any_xfused(b)) return MM_OK;
  return launch(b, "fft_x_forward", [&] {
    return mmk_launch_xfwd_cells(b->method, stage, b->total_wg, b->d_desc, b->d_wg, g_twiddle, b->stage_lds,
                                 b->stream);
  });
}

// Run start.  RK4: reductions of the state (and, for groups with x passes in
// the stage kernels, the X rows of the state for the first stage).  DP45:
// the full first derivative, whose kernel reads the demag field from memory.
mm_status enqueue_start(mm_batch* b) {
  if (b->method == MM_RK4) {
    if (mm_status s = enqueue_x_forward(b, 1)) return s;
    return enqueue_stage(b, 0);
  }
  if (mm_status s = enqueue_demag(b, 1)) return s;
  return enqueue_stage(b, 1);
}

// One step.  Where the stage kernels do the x passes, each stage's input is
// already in X (written by the previous stage kernel) except the DP45 stage
// 2 input, which depends on the step size chosen after stage 7.
// The finalisation of a stage other than the last of the step runs as extra
// workgroups of the next stage's first y-z launch when that launch is the
// eight-lane, the two-pass or the split two-pass y forward kernel: the
// transform reads and writes only X (and Y), which the finalisation does not
// touch, and the next stage kernel comes after both in stream order.
bool merge_final(const mm_batch* b) {
  if (b->groups.empty()) return false;
  const int p = b->groups[0].path;
  return p == PATH_REG8 || p == PATH_XCH || p == PATH_SPLITX;
}

mm_status enqueue_step(mm_batch* b) {
  const int s0 = b->method == MM_RK4 ? 1 : 2;
  const int s1 = b->method == MM_RK4 ? 4 : 7;
  int pending = -1;
  for (int st = s0; st <= s1; ++st) {
    const bool fwd = b->method == MM_DP45 && st == 2;
    if (mm_status s = enqueue_demag(b, st, -1, fwd, false, pending)) return s;
    const bool merge = st < s1 && merge_final(b);
    if (mm_status s = enqueue_stage(b, st, !merge)) return s;
    pending = merge ? st : -1;
  }
  return MM_OK;
}

// Capture `steps` consecutive steps of the batch into one executable graph.
mm_status capture_steps(mm_batch* b, int steps, hipGraph_t* graph, hipGraphExec_t* exec) {
  MM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  mm_status st = MM_OK;
  for (int k = 0; k < steps && st == MM_OK; ++k) st = enqueue_step(b);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (st != MM_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(MM_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  *graph = g;
  MM_HIP(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
  // move the executable graph to the device now rather than at its first
  // launch, which may fall inside a caller's timed region
  MM_HIP(hipGraphUpload(*exec, b->stream));
  return MM_OK;
}

mm_status ensure_graph(mm_batch* b) {
  if (b->exec) return MM_OK;
  return capture_steps(b, kStepsPerGraph, &b->graph, &b->exec);
}

// Graph of 2^lg steps (lg 0..4).
mm_status ensure_graph_pow(mm_batch* b, int lg) {
  if (b->exec_pow[lg]) return MM_OK;
  return capture_steps(b, 1 << lg, &b->graph_pow[lg], &b->exec_pow[lg]);
}

// Every captured graph of the batch (after a change of work tables or
// strategy they no longer match the launches the batch would make).
void drop_graphs(mm_batch* b) {
  if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { hipGraphDestroy(b->graph); b->graph = nullptr; }
  for (int i = 0; i < 5; ++i) {
    if (b->exec_pow[i]) { hipGraphExecDestroy(b->exec_pow[i]); b->exec_pow[i] = nullptr; }
    if (b->graph_pow[i]) { hipGraphDestroy(b->graph_pow[i]); b->graph_pow[i] = nullptr; }
  }
  if (b->exec_rev) { hipGraphExecDestroy(b->exec_rev); b->exec_rev = nullptr; }
  if (b->graph_rev) { hipGraphDestroy(b->graph_rev); b->graph_rev = nullptr; }
}

// Graph launches for exactly `steps` steps on every part (or the batch
// itself): whole 32-step graphs, then the binary digits of the remainder.
// Graphs are captured on first use.
mm_status launch_steps(mm_batch* b, int64_t steps) {
  std::vector<mm_batch*> seq = b->parts;
  if (seq.empty()) seq.push_back(b);
  for (mm_batch* p : seq) {
    if (mm_status s = ensure_graph(p)) return s;
    for (int lg = 0; lg < 5; ++lg)
      if ((steps % kStepsPerGraph) >> lg & 1)
        if (mm_status s = ensure_graph_pow(p, lg)) return s;
  }
  for (int64_t left = steps; left >= kStepsPerGraph; left -= kStepsPerGraph)
    for (mm_batch* p : seq) MM_HIP(hipGraphLaunch(p->exec, p->stream));
  for (int lg = 4; lg >= 0; --lg)
    if ((steps % kStepsPerGraph) >> lg & 1)
      for (mm_batch* p : seq) MM_HIP(hipGraphLaunch(p->exec_pow[lg], p->stream));
  return MM_OK;
}

// One reverse step of the discrete adjoint for every instance of the batch.
mm_status enqueue_reverse_step_dp(mm_batch* b);
mm_status enqueue_reverse_step(mm_batch* b) {
  if (b->method == MM_DP45) return enqueue_reverse_step_dp(b);
  const int n = (int)b->ctxs.size();
  if (mm_status s = launch(b, "adj_start", [&] { return mmk_launch_adj(0, 0, b->total_wg, n, b->d_desc, b->d_wg, b->stream); }))
    return s;
  if (mm_status s = launch(b, "adj_cavity", [&] { return mmk_launch_adj(3, 5, b->total_wg, n, b->d_desc, b->d_wg, b->stream); }))
    return s;
  // with the demag fields of the stage inputs recorded, only the convolution
  // of the field adjoint remains per stage
  const bool bd_recorded = b->ctxs.size() == 1 && b->ctxs[0]->desc.rec_bd;
  for (int st = 4; st >= 1; --st) {
    if (!bd_recorded)
      if (mm_status s = enqueue_demag(b, st, MMI_ADJ)) return s;
    // for groups with x passes in the cell kernels, the adjoint stage kernels
    // transform the field adjoint themselves (R2C in A, C2R in B)
    if (mm_status s = launch(b, "adj_stage_a", [&] {
          return mmk_launch_adj(1, st, b->total_wg, n, b->d_desc, b->d_wg, b->stream, g_twiddle, b->stage_lds);
        }))
      return s;
    if (mm_status s = enqueue_demag(b, 0, MMI_ADJ, false, false)) return s;
    if (mm_status s = launch(b, "adj_stage_b", [&] {
          return mmk_launch_adj(2, st, b->total_wg, n, b->d_desc, b->d_wg, b->stream, g_twiddle, b->stage_lds);
        }))
      return s;
    if (mm_status s = launch(b, "adj_cavity", [&] { return mmk_launch_adj(3, st, b->total_wg, n, b->d_desc, b->d_wg, b->stream); }))
      return s;
  }
  return MM_OK;
}

// The same for the replayed steps of an adaptive run: stages 6..1 of the
// Dormand-Prince tableau (cavity part: kind 4, stage 7 = step start).
mm_status enqueue_reverse_step_dp(mm_batch* b) {
  const int n = (int)b->ctxs.size();
  if (mm_status s = launch(b, "adj_start", [&] { return mmk_launch_adj(0, 0, b->total_wg, n, b->d_desc, b->d_wg, b->stream); }))
    return s;
  if (mm_status s = launch(b, "adj_cavity", [&] { return mmk_launch_adj(4, 7, b->total_wg, n, b->d_desc, b->d_wg, b->stream); }))
    return s;
  const bool bd_recorded = b->ctxs.size() == 1 && b->ctxs[0]->desc.rec_bd;
  for (int st = 6; st >= 1; --st) {
    if (!bd_recorded)
      if (mm_status s = enqueue_demag(b, st, MMI_ADJ)) return s;
    if (mm_status s = launch(b, "adj_stage_a", [&] {
          return mmk_launch_adj(1, st, b->total_wg, n, b->d_desc, b->d_wg, b->stream, g_twiddle, b->stage_lds);
        }))
      return s;
    if (mm_status s = enqueue_demag(b, 0, MMI_ADJ, false, false)) return s;
    if (mm_status s = launch(b, "adj_stage_b", [&] {
          return mmk_launch_adj(2, st, b->total_wg, n, b->d_desc, b->d_wg, b->stream, g_twiddle, b->stage_lds);
        }))
      return s;
    if (mm_status s = launch(b, "adj_cavity", [&] { return mmk_launch_adj(4, st, b->total_wg, n, b->d_desc, b->d_wg, b->stream); }))
      return s;
  }
  return MM_OK;
}

mm_status ensure_reverse_graph(mm_batch* b) {
  if (b->exec_rev) return MM_OK;
  MM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  mm_status st = enqueue_reverse_step(b);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (st != MM_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(MM_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  b->graph_rev = g;
  MM_HIP(hipGraphInstantiate(&b->exec_rev, g, nullptr, nullptr, 0));
  return MM_OK;
}

mm_status wait_user_streams(mm_batch* b) {
  for (mm_ctx* c : b->ctxs)
    if (c->user_stream && c->user_stream != b->stream) {
      MM_HIP(hipEventRecord(b->ev, c->user_stream));
      MM_HIP(hipStreamWaitEvent(b->stream, b->ev, 0));
    }
  return MM_OK;
}

mm_status check_ready(mm_ctx* c) {
  if (!c->modes_set) return fail(MM_ERR_STATE, "modes not set (mm_set_modes)");
  if (!c->m_set) return fail(MM_ERR_STATE, "magnetisation not set (mm_set_m)");
  return MM_OK;
}

// Set run parameters of every instance; t_end = t + T (T <= 0: unbounded),
// or t_end_abs when that is finite.
mm_status begin_run(mm_batch* b, double T, double tol, double t_end_abs = NAN) {
  for (mm_ctx* c : b->ctxs) {
    InstCtl h;
    if (mm_status s = ctl_pull(c, h)) return s;
    h.t_end = std::isfinite(t_end_abs) ? t_end_abs : T > 0 ? h.t + T : 1e300;
    h.tol = tol;
    h.dt_fixed = c->dt0;
    h.dt_min = c->dt_min;
    h.dt_max = c->dt_max;
    h.done = 0;
    h.status = 0;
    // the run-start stage kernel evaluates the feedback from the stage
    // amplitude: it must be the amplitude of the state the run starts from
    // (a previous run leaves the next stage input there, mm_set_a and
    // mm_set_state set a alone)
    for (int n = 0; n < MMI_MAX_MODES; ++n) {
      h.as[n][0] = h.a[n][0];
      h.as[n][1] = h.a[n][1];
    }
    h.rec_index = c->record_next;
    c->record_next = -1;
    if (c->sampling_changed) {
      c->sampling_changed = false;
      h.trace_on = c->max_samples > 0 ? 1 : 0;
      h.trace_started = 0;
      h.trace_n = 0;
      h.trace_steps = 0;
      h.trace_max = c->max_samples;
      h.trace_dt = c->dt_sample;
      h.trace_stride = c->method == MM_RK4 ? std::max<long long>(1, llround(c->dt_sample / c->dt0)) : 1;
    }
    if (mm_status s = ctl_push(c, h)) return s;
  }
  if (mm_status s = refresh_descs(b)) return s;
  if (mm_status s = wait_user_streams(b)) return s;
  return enqueue_start(b);
}

// The host copy of an instance's statistics from its control block.
void set_stats(mm_ctx* c, const InstCtl& h, double wall) {
  c->stats.accepted = h.accepted;
  c->stats.rejected = h.rejected;
  c->stats.t = h.t;
  c->stats.dt = c->method == MM_RK4 ? h.dt_fixed : h.dt;
  c->stats.dt_min_seen = h.dt_min_seen;
  c->stats.dt_max_seen = h.dt_max_seen;
  c->stats.wall_s = wall;
  c->stats.status = h.status;
}

mm_status end_run(mm_batch* b, double wall) {
  MM_HIP(hipStreamSynchronize(b->stream));
  mm_status first = MM_OK;
  for (mm_ctx* c : b->ctxs) {
    InstCtl h;
    if (mm_status s = ctl_pull(c, h)) return s;
    set_stats(c, h, wall);
    if (h.status != 0 && first == MM_OK) first = (mm_status)h.status;
  }
  if (first == MM_ERR_DT_UNDERFLOW) return fail(first, "adaptive step fell below dt_min");
  if (first == MM_ERR_NONFINITE) return fail(first, "state became non-finite");
  return first;
}

mm_status batch_run(mm_batch* b, double T, double tol, double t_end_abs = NAN) {
  const auto t0 = std::chrono::steady_clock::now();
  if (mm_status s = begin_run(b, T, tol, t_end_abs)) return s;
  if (mm_status s = ensure_graph(b)) return s;
  const int n = (int)b->ctxs.size();
  for (;;) {
    MM_HIP(hipGraphLaunch(b->exec, b->stream));
    MM_HIP(mmk_launch_gather_done(n, b->d_desc, b->d_flags, b->stream));
    MM_HIP(hipMemcpyAsync(b->h_flags, b->d_flags, sizeof(int) * 2 * n, hipMemcpyDeviceToHost, b->stream));
    MM_HIP(hipStreamSynchronize(b->stream));
    bool all = true;
    for (int i = 0; i < n; ++i) all = all && b->h_flags[2 * i] != 0;
    if (all) break;
  }
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return end_run(b, wall);
}

mm_status validate_tol(const mm_batch* b, double tol) {
  if (b->method == MM_DP45 && !(tol > 0 && std::isfinite(tol)))
    return fail(MM_ERR_ARG, "DP45 needs a finite tol > 0");
  return MM_OK;
}

mm_status new_batch(mm_ctx* const* ctxs, int count, mm_batch** out) {
  auto* b = new mm_batch();
  b->ctxs.assign(ctxs, ctxs + count);
  b->method = ctxs[0]->method;
  if (mm_status s = batch_build(b)) {
    mm_batch_destroy(b);
    return s;
  }
  *out = b;
  return MM_OK;
}

// Work of one instance for the partition below: cells times sublattices.
double inst_cells(const mm_ctx* c) { return (double)c->L.ncell * c->p.sublattices; }

// A batch of `parts` sub-batches (parts >= 2) whose cell counts are as even
// as a greedy assignment (largest instance first, to the lightest part) makes
// them; each part keeps the instances in batch order.
mm_status new_split_batch(mm_ctx* const* ctxs, int count, int parts, mm_batch** out) {
  auto* b = new mm_batch();
  b->ctxs.assign(ctxs, ctxs + count);
  b->method = ctxs[0]->method;
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return inst_cells(ctxs[a]) > inst_cells(ctxs[c]); });
  std::vector<double> load(parts, 0.0);
  std::vector<std::vector<int>> sets(parts);
  for (int i : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    sets[k].push_back(i);
    load[k] += inst_cells(ctxs[i]);
  }
  for (auto& set : sets) {
    std::sort(set.begin(), set.end());
    std::vector<mm_ctx*> sub;
    for (int i : set) sub.push_back(ctxs[i]);
    mm_batch* part = nullptr;
    if (mm_status s = new_batch(sub.data(), (int)sub.size(), &part)) {
      mm_batch_destroy(b);
      return s;
    }
    b->parts.push_back(part);
  }
  *out = b;
  return MM_OK;
}

mm_status make_batch(mm_ctx* const* ctxs, int count, int parts, mm_batch** out) {
  parts = std::min(parts, count);
  return parts <= 1 ? new_batch(ctxs, count, out) : new_split_batch(ctxs, count, parts, out);
}

// Run every part to its end time (T as in batch_run), the parts' graphs
// launched round-robin so that their streams overlap.
mm_status parts_run(mm_batch* b, double T, double tol) {
  const auto t0 = std::chrono::steady_clock::now();
  for (mm_batch* p : b->parts) {
    if (mm_status s = begin_run(p, T, tol)) return s;
    if (mm_status s = ensure_graph(p)) return s;
  }
  std::vector<mm_batch*> active = b->parts;
  while (!active.empty()) {
    for (mm_batch* p : active) {
      const int n = (int)p->ctxs.size();
      MM_HIP(hipGraphLaunch(p->exec, p->stream));
      MM_HIP(mmk_launch_gather_done(n, p->d_desc, p->d_flags, p->stream));
      MM_HIP(hipMemcpyAsync(p->h_flags, p->d_flags, sizeof(int) * 2 * n, hipMemcpyDeviceToHost, p->stream));
    }
    std::vector<mm_batch*> still;
    for (mm_batch* p : active) {
      MM_HIP(hipStreamSynchronize(p->stream));
      bool all = true;
      for (size_t i = 0; i < p->ctxs.size(); ++i) all = all && p->h_flags[2 * i] != 0;
      if (!all) still.push_back(p);
    }
    active.swap(still);
  }
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  mm_status first = MM_OK;
  for (mm_batch* p : b->parts) {
    const mm_status s = end_run(p, wall);
    if (s != MM_OK && first == MM_OK) first = s;
  }
  return first;
}

// Begin an open-ended run of every part (or of the batch itself).
mm_status open_run(mm_batch* b, double tol) {
  std::vector<mm_batch*> seq = b->parts;
  if (seq.empty()) seq.push_back(b);
  for (mm_batch* p : seq)
    if (mm_status s = begin_run(p, -1.0, tol)) return s;
  return MM_OK;
}

// Wait for every part and pull the statistics of its instances.
mm_status close_run(mm_batch* b, double wall) {
  std::vector<mm_batch*> seq = b->parts;
  if (seq.empty()) seq.push_back(b);
  for (mm_batch* p : seq) MM_HIP(hipStreamSynchronize(p->stream));
  mm_status first = MM_OK;
  for (mm_batch* p : seq) {
    const mm_status s = end_run(p, wall);
    if (s != MM_OK && first == MM_OK) first = s;
  }
  return first;
}

// FFT strategy of `src`'s groups copied to the groups of `dst` with the same
// grid shape (and the work tables rebuilt).
mm_status copy_fft_settings(mm_batch* dst, const mm_batch* src) {
  for (auto& g : dst->groups)
    for (const auto& h : src->groups)
      if (g.nx == h.nx && g.ny == h.ny && g.nz == h.nz && g.px == h.px && g.py == h.py && g.pz == h.pz) {
        g.path = h.path;
        g.xfused = h.xfused;
        g.Wx = h.Wx;
        g.Wy = h.Wy;
        g.TW = h.TW;
        g.TK = h.TK;
        if (mm_status s = build_group(g)) return s;
        break;
      }
  batch_xfused(dst);
  return upload_batch_descs(dst);
}

double algorithmic_bytes(const mm_batch* b, const std::string& name) {
  double total = 0.0;
  if (name.rfind("final_", 0) == 0) {
    double t = 0.0;   // partial records of every workgroup, read once
    for (const mm_ctx* c : b->ctxs) t += (double)c->L.nwg * MMI_PSTRIDE * sizeof(double);
    return t;
  }
  const bool is_stage = name.rfind("stage_", 0) == 0;
  int st = 0;
  if (is_stage) st = name.back() - '0';
  for (size_t gi = 0; gi < b->groups.size() || is_stage; ++gi) {
    if (is_stage) {
      for (size_t ci = 0; ci < b->ctxs.size(); ++ci) {
        const mm_ctx* c = b->ctxs[ci];
        const double cells = (double)c->L.ncell * c->p.sublattices;
        double rd = 0, wr = 0;
        if (b->method == MM_RK4) {
          if (name == "stage_rk4_start") { rd = 12; wr = 0; }
          else if (st == 1) { rd = 12; wr = 24; }
          else if (st == 2 || st == 3) { rd = 36; wr = 24; }
          else { rd = 36; wr = 12; }
        } else {
          static const double R[8] = {0, 12, 24, 48, 60, 72, 72, 72};
          static const double Wt[8] = {0, 12, 24, 24, 24, 24, 24, 12};
          rd = R[st];
          wr = Wt[st];
        }
        const bool fft = c->p.demag == MM_DEMAG_FFT && name != "stage_rk4_start";
        const bool xin = !b->xfused.empty() && b->xfused[ci];
        // demag field: B_d read, or with the x passes inside, the X rows read
        // (C2R) and the next input's X rows written (R2C)
        double demag = 0.0;
        if (fft && !xin) demag = 12.0;
        if (fft && xin) {
          const bool c2r = b->method == MM_RK4 ? st >= 1 : st >= 2;
          const bool r2c = b->method == MM_RK4 ? st >= 1 : (st >= 2 && st <= 6);
          const double xrow = 24.0 * c->L.kx / c->p.nx;   // X bytes per cell
          demag = (c2r ? xrow : 0.0) + (r2c ? xrow : 0.0);
        }
        double extra = (double)c->L.ncell * ((c->p.geometry ? 1.0 : 0.0) + (c->profiled ? 4.0 * c->N : 0.0) + demag);
        total += cells * (rd + wr) + extra;
      }
      break;
    }
    const auto& g = b->groups[gi];
    const double m = (double)g.members.size();
    const double cells = (double)g.nx * g.ny * g.nz;
    const double X = 8.0 * g.kx * 3.0 * g.ny * g.nz;       // complex after the x pass
    const double Y = 8.0 * g.kx * 3.0 * g.nz * g.py;       // complex after the y pass
    const double kern = 4.0 * 6.0 * (g.pz / 2 + 1) * (g.py / 2 + 1) * g.kx;
    // x-forward: the stage input read once (two fields, y and k1, for the
    // DP45 stage-2 input, the only one left to this pass when the stage
    // kernels do the x passes) and the X rows written
    const double xin = (b->method == MM_DP45 && g.xfused) ? 24.0 : 12.0;
    if (name == "fft_x_forward") total += m * (xin * cells + X);
    if (name == "fft_x_inverse") total += m * (X + 12.0 * cells);
    if (name == "fft_yz_convolve") total += m * 2.0 * X + kern;
    if (name == "fft_y_forward" || name == "fft_y_inverse") total += m * (X + Y);
    if (name == "fft_z_convolve") total += m * 2.0 * Y + kern;
  }
  return total;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

const char* mm_last_error(void) { return g_err.c_str(); }

mm_status mm_demag_tensor(double X, double Y, double Z, double dx, double dy, double dz, double* out6) {
  if (!out6) return fail(MM_ERR_ARG, "out6 is NULL");
  if (!(dx > 0 && dy > 0 && dz > 0)) return fail(MM_ERR_ARG, "cell sizes must be > 0");
  if (!std::isfinite(X) || !std::isfinite(Y) || !std::isfinite(Z)) return fail(MM_ERR_ARG, "non-finite displacement");
  mmh::demag_tensor(X, Y, Z, dx, dy, dz, out6);
  return MM_OK;
}

mm_status mm_create(const mm_params* p, mm_ctx** out) {
  if (!out) return fail(MM_ERR_ARG, "out is NULL");
  if (mm_status s = validate(p)) return s;
  auto* c = new (std::nothrow) mm_ctx();
  if (!c) return fail(MM_ERR_OOM, "host allocation failed");
  c->p = *p;
  const size_t nc = (size_t)p->nx * p->ny * p->nz;
  if (p->geometry) {
    c->geom.assign(p->geometry, p->geometry + nc);
    for (auto& v : c->geom) v = v ? 1 : 0;
    c->p.geometry = c->geom.data();
    c->n_geo = 0;
    for (auto v : c->geom) c->n_geo += v;
  } else {
    c->n_geo = (long long)nc;
  }
  c->L = make_layout(c->p, 0);
  hipError_t e = hipGetDevice(&c->dev);
  if (e != hipSuccess) c->dev = 0;
  c->stats.dt_min_seen = INFINITY;
  *out = c;
  return MM_OK;
}

mm_status mm_destroy(mm_ctx* c) {
  if (c && c->open_in) return open_error();
  if (!c) return MM_OK;
  if (c->solo) mm_batch_destroy(c->solo);
  if (c->dev_ready || c->ws) hipSetDevice(c->dev);
  if (!c->ws_bound && c->ws) hipFree(c->ws);
  if (c->u_own) hipFree(c->u_own);
  if (c->trace) hipFree(c->trace);
  if (c->ck_m) hipFree(c->ck_m);
  if (c->adj_f) hipFree(c->adj_f);
  if (c->adj_d) hipFree(c->adj_d);
  if (c->hlog_dev) hipFree(c->hlog_dev);
  release_spectrum(c->spec);
  delete c;
  return MM_OK;
}

mm_status mm_workspace_bytes(const mm_params* p, int32_t n_modes, size_t* bytes) {
  if (!bytes) return fail(MM_ERR_ARG, "bytes is NULL");
  if (mm_status s = validate(p)) return s;
  if (n_modes < 0 || n_modes > MM_MAX_MODES) return fail(MM_ERR_ARG, "n_modes out of range");
  *bytes = make_layout(*p, n_modes).total;
  return MM_OK;
}

mm_status mm_bind_workspace(mm_ctx* c, void* ptr, size_t bytes) {
  if (c && c->open_in) return open_error();
  if (!c || !ptr) return fail(MM_ERR_ARG, "NULL context or pointer");
  if (c->dev_ready) return fail(MM_ERR_STATE, "device memory already in use; bind before mm_set_modes");
  if (((uintptr_t)ptr) % kAlign) return fail(MM_ERR_ARG, "workspace must be 256-byte aligned");
  const Layout L0 = make_layout(c->p, 0);
  if (bytes < L0.total) return fail(MM_ERR_ARG, "workspace too small");
  c->u_cap = 0;
  while (c->u_cap < MM_MAX_MODES && make_layout(c->p, c->u_cap + 1).total <= bytes) c->u_cap++;
  c->ws = (char*)ptr;
  c->ws_bytes = bytes;
  c->ws_bound = true;
  return MM_OK;
}

mm_status mm_set_stream(mm_ctx* c, void* stream) {
  if (c && c->open_in) return open_error();
  if (!c) return fail(MM_ERR_ARG, "NULL context");
  c->user_stream = (hipStream_t)stream;
  return MM_OK;
}

mm_status mm_set_modes(mm_ctx* c, int32_t n, const double* omega, const double* kappa, const double* g,
                       const float* u, const double* phi, const int8_t* sign) {
  if (c && c->open_in) return open_error();
  if (!c) return fail(MM_ERR_ARG, "NULL context");
  if (n < 0 || n > MM_MAX_MODES) return fail(MM_ERR_ARG, "mode count out of range");
  if (n > 0 && (!omega || !kappa || !g)) return fail(MM_ERR_ARG, "omega, kappa and g are required");
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(omega[i]) || !std::isfinite(g[i]) || !(kappa[i] >= 0) || !std::isfinite(kappa[i]))
      return fail(MM_ERR_ARG, "mode parameters must be finite with kappa >= 0");
    if (phi && !std::isfinite(phi[i])) return fail(MM_ERR_ARG, "non-finite phase");
  }
  const int S = c->p.sublattices;
  if (sign)
    for (int s = 0; s < S; ++s)
      if (sign[s] != 1 && sign[s] != -1) return fail(MM_ERR_ARG, "sublattice signs must be +1 or -1");
  const size_t nc = (size_t)c->L.ncell;
  if (u)
    for (size_t i = 0; i < (size_t)n * nc; ++i)
      if (!std::isfinite(u[i])) return fail(MM_ERR_ARG, "non-finite mode profile");
  if (c->ws_bound && u && n > c->u_cap) return fail(MM_ERR_ARG, "bound workspace has no room for the mode profiles");
  if (mm_status s = ensure_device(c)) return s;
  c->N = n;
  c->drive_on = false;
  c->param_on = false;
  c->nonrecip = false;
  c->kerr_on = false;
  c->jcpl_on = false;
  c->omega.assign(omega, omega + n);
  c->kappa.assign(kappa, kappa + n);
  c->g.assign(g, g + n);
  c->phi.assign(n, 0.0);
  if (phi) c->phi.assign(phi, phi + n);
  c->cs[0] = c->cs[1] = 1;
  if (sign)
    for (int s = 0; s < S; ++s) c->cs[s] = sign[s];
  c->profiled = u != nullptr && n > 0;
  if (c->profiled) {
    float* dst;
    if (c->ws_bound) {
      dst = (float*)(c->ws + c->L.u);
    } else {
      if (c->u_own) hipFree(c->u_own);
      c->u_own = nullptr;
      if (hipMalloc(&c->u_own, sizeof(float) * n * nc) != hipSuccess) return fail(MM_ERR_OOM, "mode profile allocation failed");
      dst = c->u_own;
    }
    MM_HIP(hipMemcpy(dst, u, sizeof(float) * n * nc, hipMemcpyHostToDevice));
  }
  InstCtl h;
  if (mm_status s = ctl_pull(c, h)) return s;
  std::memset(h.a, 0, sizeof(h.a));
  h.trace_n = 0;
  h.trace_started = 0;
  if (mm_status s = ctl_push(c, h)) return s;
  c->modes_set = true;
  if (c->trace) {  // trace layout depends on N
    hipFree(c->trace);
    c->trace = nullptr;
    c->trace_cap = 0;
    if (c->max_samples > 0) {
      const size_t cnt = (size_t)c->max_samples * (1 + 4 * (size_t)std::max(1, n));
      if (hipMalloc(&c->trace, sizeof(double) * cnt) != hipSuccess) return fail(MM_ERR_OOM, "trace allocation failed");
      c->trace_cap = c->max_samples;
      c->sampling_changed = true;
    }
  }
  return upload_desc(c);
}

mm_status mm_set_cavity_model(mm_ctx* c, int32_t n, const double* g_back, const double* kerr,
                              const double* coupling) {
  if (c && c->open_in) return open_error();
  if (!c) return fail(MM_ERR_ARG, "NULL context");
  if (!c->modes_set) return fail(MM_ERR_STATE, "modes not set (mm_set_modes)");
  if (n != 0 && n != c->N) return fail(MM_ERR_ARG, "count must equal the mode count");
  if (n == 0) g_back = kerr = coupling = nullptr;
  for (int i = 0; i < n; ++i)
    if ((g_back && !std::isfinite(g_back[i])) || (kerr && !std::isfinite(kerr[i])))
      return fail(MM_ERR_ARG, "cavity-model parameters must be finite");
  if (coupling)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double v = coupling[(size_t)i * n + j];
        if (!std::isfinite(v)) return fail(MM_ERR_ARG, "cavity-model parameters must be finite");
        if (i == j && v != 0.0) return fail(MM_ERR_ARG, "mode coupling must be zero on the diagonal");
        if (v != coupling[(size_t)j * n + i]) return fail(MM_ERR_ARG, "mode coupling must be symmetric");
      }
  c->nonrecip = g_back != nullptr;
  c->kerr_on = kerr != nullptr;
  c->jcpl_on = coupling != nullptr;
  if (g_back) c->g_back.assign(g_back, g_back + n);
  if (kerr) c->kerr.assign(kerr, kerr + n);
  if (coupling) c->jcpl.assign(coupling, coupling + (size_t)n * n);
  return upload_desc(c);
}

mm_status mm_set_drive(mm_ctx* c, int32_t n, const double* amp, const double* t0, const double* sigma) {
  if (c && c->open_in) return open_error();
  if (!c) return fail(MM_ERR_ARG, "NULL context");
  if (!c->modes_set) return fail(MM_ERR_STATE, "modes not set (mm_set_modes)");
  if (n == 0 || !amp) {
    c->drive_on = false;
    return upload_desc(c);
  }
  if (n != c->N) return fail(MM_ERR_ARG, "drive count must equal the mode count");
  if (!t0 || !sigma) return fail(MM_ERR_ARG, "t0 and sigma are required with an amplitude");
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(amp[2 * i]) || !std::isfinite(amp[2 * i + 1]) || !std::isfinite(t0[i]))
      return fail(MM_ERR_ARG, "drive parameters must be finite");
    if (!(sigma[i] > 0) || !std::isfinite(sigma[i])) return fail(MM_ERR_ARG, "drive width sigma must be > 0");
  }
  c->drive_re.assign(n, 0.0);
  c->drive_im.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    c->drive_re[i] = amp[2 * i];
    c->drive_im[i] = amp[2 * i + 1];
  }
  c->drive_t0.assign(t0, t0 + n);
  c->drive_sigma.assign(sigma, sigma + n);
  c->drive_on = true;
  return upload_desc(c);
}

mm_status mm_set_parametric(mm_ctx* c, int32_t n, const double* lambda, const double* omega_p) {
  if (c && c->open_in) return open_error();
  if (!c) return fail(MM_ERR_ARG, "NULL context");
  if (!c->modes_set) return fail(MM_ERR_STATE, "modes not set (mm_set_modes)");
  if (n == 0 || !lambda) {
    c->param_on = false;
    return upload_desc(c);
  }
  if (n != c->N) return fail(MM_ERR_ARG, "pump count must equal the mode count");
  if (!omega_p) return fail(MM_ERR_ARG, "omega_p is required with a pump strength");
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(lambda[2 * i]) || !std::isfinite(lambda[2 * i + 1]) || !std::isfinite(omega_p[i]))
      return fail(MM_ERR_ARG, "pump parameters must be finite");
  c->par_re.assign(n, 0.0);
  c->par_im.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    c->par_re[i] = lambda[2 * i];
    c->par_im[i] = lambda[2 * i + 1];
  }
  c->par_wp.assign(omega_p, omega_p + n);
  c->param_on = true;
  return upload_desc(c);
}

mm_status mm_set_m(mm_ctx* c, const float* m) {
  if (c && c->open_in) return open_error();
  if (!c || !m) return fail(MM_ERR_ARG, "NULL argument");
  const size_t nc = (size_t)c->L.ncell;
  const int S = c->p.sublattices;
  std::vector<float> h((size_t)3 * S * nc);
  for (int s = 0; s < S; ++s)
    for (size_t i = 0; i < nc; ++i) {
      const bool mag = !c->p.geometry || c->geom[i];
      double v[3];
      for (int q = 0; q < 3; ++q) v[q] = m[((size_t)s * 3 + q) * nc + i];
      if (!mag) {
        for (int q = 0; q < 3; ++q) h[((size_t)s * 3 + q) * nc + i] = 0.f;
        continue;
      }
      const double nrm = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      if (!(nrm > 0) || !std::isfinite(nrm)) return fail(MM_ERR_ARG, "magnetic cell with zero or non-finite m");
      for (int q = 0; q < 3; ++q) h[((size_t)s * 3 + q) * nc + i] = (float)(v[q] / nrm);
    }
  if (mm_status s = ensure_device(c)) return s;
  InstCtl ctl;
  if (mm_status s = ctl_pull(c, ctl)) return s;
  MM_HIP(hipMemcpy(c->ws + c->L.y[ctl.cur], h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice));
  c->m_set = true;
  return MM_OK;
}

mm_status mm_set_a(mm_ctx* c, const double* a) {
  if (c && c->open_in) return open_error();
  if (!c || !a) return fail(MM_ERR_ARG, "NULL argument");
  if (!c->modes_set) return fail(MM_ERR_STATE, "modes not set");
  for (int i = 0; i < 2 * c->N; ++i)
    if (!std::isfinite(a[i])) return fail(MM_ERR_ARG, "non-finite cavity amplitude");
  InstCtl h;
  if (mm_status s = ctl_pull(c, h)) return s;
  for (int n = 0; n < c->N; ++n) {
    h.a[n][0] = a[2 * n];
    h.a[n][1] = a[2 * n + 1];
  }
  return ctl_push(c, h);
}

mm_status mm_set_stepper(mm_ctx* c, int32_t method, double dt0, double dt_min, double dt_max) {
  if (c && c->open_in) return open_error();
  if (!c) return fail(MM_ERR_ARG, "NULL context");
  if (method != MM_RK4 && method != MM_DP45 && method != MM_RK4_SPLIT) return fail(MM_ERR_ARG, "unknown method");
  const bool split = method == MM_RK4_SPLIT;
  if (split) method = MM_RK4;
  if (!(dt0 > 0) || !std::isfinite(dt0)) return fail(MM_ERR_ARG, "dt0 must be > 0");
  if (!(dt_min > 0) || !std::isfinite(dt_min) || dt_min > dt0) return fail(MM_ERR_ARG, "need 0 < dt_min <= dt0");
  if (!std::isfinite(dt_max)) return fail(MM_ERR_ARG, "dt_max must be finite");
  if (c->solo && c->method != method) {
    mm_batch_destroy(c->solo);
    c->solo = nullptr;
  }
  c->method = method;
  c->split = split;
  c->dt0 = dt0;
  c->dt_min = dt_min;
  c->dt_max = dt_max;
  if (c->dev_ready) {
    InstCtl h;
    if (mm_status s = ctl_pull(c, h)) return s;
    h.dt = dt0;
    h.dt_fixed = dt0;
    h.last_rejected = 0;
    if (mm_status s = ctl_push(c, h)) return s;
    c->desc.method = method;
    c->desc.split = split ? 1 : 0;
    c->version++;
  }
  return MM_OK;
}

mm_status mm_set_sampling(mm_ctx* c, double dt_sample, int64_t max_samples) {
  if (c && c->open_in) return open_error();
  if (!c) return fail(MM_ERR_ARG, "NULL context");
  if (max_samples < 0) return fail(MM_ERR_ARG, "max_samples must be >= 0");
  if (max_samples > 0 && !(dt_sample > 0 && std::isfinite(dt_sample))) return fail(MM_ERR_ARG, "dt_sample must be > 0");
  if (max_samples > 0 && c->method == MM_RK4) {
    const double r = dt_sample / c->dt0;
    if (r < 1.0 - 1e-9 || std::fabs(r - std::llround(r)) > 1e-9 * r)
      return fail(MM_ERR_ARG, "RK4 sampling interval must be a whole multiple of dt0");
  }
  if (mm_status s = ensure_device(c)) return s;
  if (c->trace) hipFree(c->trace);
  c->trace = nullptr;
  c->trace_cap = 0;
  if (max_samples > 0) {
    const size_t cnt = (size_t)max_samples * (1 + 4 * (size_t)std::max(1, c->N));
    if (hipMalloc(&c->trace, sizeof(double) * cnt) != hipSuccess) return fail(MM_ERR_OOM, "trace allocation failed");
    c->trace_cap = max_samples;
  }
  c->dt_sample = dt_sample;
  c->max_samples = max_samples;
  c->sampling_changed = true;
  return upload_desc(c);
}

mm_status mm_run(mm_ctx* c, double T, double tol) {
  if (c && c->open_in) return open_error();
  if (!c) return fail(MM_ERR_ARG, "NULL context");
  if (!(T > 0) || !std::isfinite(T)) return fail(MM_ERR_ARG, "T must be finite and > 0");
  if (mm_status s = check_ready(c)) return s;
  if (!c->solo) {
    mm_ctx* one[1] = {c};
    if (mm_status s = new_batch(one, 1, &c->solo)) return s;
  }
  if (mm_status s = validate_tol(c->solo, tol)) return s;
  if (mm_status s = set_device(c)) return s;
  return batch_run(c->solo, T, tol);
}

mm_status mm_run_noalloc(mm_ctx* c, double T, double tol) {
  if (c && c->open_in) return open_error();
  if (!c) return fail(MM_ERR_ARG, "NULL context");
  if (!(T > 0) || !std::isfinite(T)) return fail(MM_ERR_ARG, "T must be finite and > 0");
  if (mm_status s = check_ready(c)) return s;
  if (!c->dev_ready) return fail(MM_ERR_STATE, "device state not set up");
  if (c->method == MM_DP45 && !(tol > 0 && std::isfinite(tol)))
    return fail(MM_ERR_ARG, "DP45 needs a finite tol > 0");
  if (mm_status s = set_device(c)) return s;
  void* base = nullptr;
  size_t cap = 0;
  MM_HIP(mmk_noalloc_scratch(c->dev, &base, &cap));
  mm_ctx* one[1] = {c};
  {
    // bytes the tables and run buffers take, with the same choices as mm_run
    mm_batch probe;
    probe.ctxs.assign(one, one + 1);
    probe.method = c->method;
    DevArena cnt;
    cnt.mode = DevArena::COUNT;
    if (mm_status s = batch_build(&probe, &cnt)) return s;
    if (cnt.off > cap)
      return fail(MM_ERR_ARG, "the instance needs " + std::to_string(cnt.off) + " bytes of scratch; mm_run_noalloc has " +
                                  std::to_string(cap));
  }
  std::lock_guard<std::mutex> lk(mmk_noalloc_lock(c->dev));
  const auto t0 = std::chrono::steady_clock::now();
  mm_batch b;
  b.ctxs.assign(one, one + 1);
  b.method = c->method;
  b.stream = c->user_stream;
  DevArena ar;
  ar.mode = DevArena::CARVE;
  ar.base = (char*)base;
  ar.cap = cap;
  if (mm_status s = batch_build(&b, &ar)) return s;
  // the array keeps the previous call's contents: start from zeros, as the
  // context's own buffers did
  MM_HIP(mmk_launch_fill_zero(b.rb.lo, b.rb.bytes, b.stream));
  if (mm_status s = begin_run(&b, T, tol)) return s;
  for (;;) {
    for (int k = 0; k < kStepsPerGraph; ++k)
      if (mm_status s = enqueue_step(&b)) return s;
    MM_HIP(mmk_launch_gather_done(1, b.d_desc, b.d_flags, b.stream));
    MM_HIP(hipMemcpyAsync(b.h_flags, b.d_flags, sizeof(int) * 2, hipMemcpyDeviceToHost, b.stream));
    MM_HIP(hipStreamSynchronize(b.stream));
    if (b.h_flags[0] != 0) break;
  }
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return end_run(&b, wall);
}

mm_status mm_get_m(const mm_ctx* c, float* out) {
  if (c && c->open_in) return open_error();
  if (!c || !out) return fail(MM_ERR_ARG, "NULL argument");
  if (!c->dev_ready || !c->m_set) return fail(MM_ERR_STATE, "no state on the device");
  InstCtl h;
  if (mm_status s = ctl_pull(c, h)) return s;
  MM_HIP(hipMemcpy(out, c->ws + c->L.y[h.cur], sizeof(float) * 3 * c->p.sublattices * (size_t)c->L.ncell,
                   hipMemcpyDeviceToHost));
  return MM_OK;
}

mm_status mm_get_a(const mm_ctx* c, double* out) {
  if (c && c->open_in) return open_error();
  if (!c || !out) return fail(MM_ERR_ARG, "NULL argument");
  if (!c->dev_ready) return fail(MM_ERR_STATE, "no state on the device");
  InstCtl h;
  if (mm_status s = ctl_pull(c, h)) return s;
  for (int n = 0; n < c->N; ++n) {
    out[2 * n] = h.a[n][0];
    out[2 * n + 1] = h.a[n][1];
  }
  return MM_OK;
}

mm_status mm_get_trace(const mm_ctx* c, double* t, double* a, double* mminus, int64_t* n) {
  if (c && c->open_in) return open_error();
  if (!c || !n) return fail(MM_ERR_ARG, "NULL argument");
  if (!c->dev_ready) return fail(MM_ERR_STATE, "no state on the device");
  InstCtl h;
  if (mm_status s = ctl_pull(c, h)) return s;
  const int64_t have = c->trace ? h.trace_n : 0;
  const int64_t cnt = std::min<int64_t>(have, *n);
  const int N = c->N;
  if (cnt > 0) {
    if (!t || !a || !mminus) return fail(MM_ERR_ARG, "NULL output buffer");
    const int64_t cap = c->trace_cap;
    MM_HIP(hipMemcpy(t, c->trace, sizeof(double) * cnt, hipMemcpyDeviceToHost));
    MM_HIP(hipMemcpy(a, c->trace + cap, sizeof(double) * cnt * 2 * N, hipMemcpyDeviceToHost));
    MM_HIP(hipMemcpy(mminus, c->trace + cap * (1 + 2 * (int64_t)std::max(1, N)), sizeof(double) * cnt * 2 * N,
                     hipMemcpyDeviceToHost));
  }
  *n = cnt;
  return MM_OK;
}

mm_status mm_get_stats(const mm_ctx* c, mm_stats* out) {
  if (c && c->open_in) return open_error();
  if (!c || !out) return fail(MM_ERR_ARG, "NULL argument");
  *out = c->stats;
  return MM_OK;
}

namespace {
struct StateHeader {
  uint64_t magic;
  int32_t S, N, ncell, method;
  uint64_t ctl_bytes, m_bytes;
};
constexpr uint64_t kMagic = 0x6d6d636176310001ULL;
}  // namespace

mm_status mm_get_state(const mm_ctx* c, void* blob, size_t* bytes) {
  if (c && c->open_in) return open_error();
  if (!c || !bytes) return fail(MM_ERR_ARG, "NULL argument");
  const size_t mb = sizeof(float) * 3 * c->p.sublattices * (size_t)c->L.ncell;
  const size_t need = sizeof(StateHeader) + sizeof(InstCtl) + mb;
  if (!blob) {
    *bytes = need;
    return MM_OK;
  }
  if (*bytes < need) return fail(MM_ERR_ARG, "state buffer too small");
  if (!c->dev_ready || !c->m_set) return fail(MM_ERR_STATE, "no state on the device");
  StateHeader hd{kMagic, c->p.sublattices, c->N, c->L.ncell, c->method, sizeof(InstCtl), mb};
  char* o = (char*)blob;
  std::memcpy(o, &hd, sizeof(hd));
  InstCtl h;
  if (mm_status s = ctl_pull(c, h)) return s;
  std::memcpy(o + sizeof(hd), &h, sizeof(h));
  MM_HIP(hipMemcpy(o + sizeof(hd) + sizeof(h), c->ws + c->L.y[h.cur], mb, hipMemcpyDeviceToHost));
  *bytes = need;
  return MM_OK;
}

mm_status mm_set_state(mm_ctx* c, const void* blob, size_t bytes) {
  if (c && c->open_in) return open_error();
  if (!c || !blob) return fail(MM_ERR_ARG, "NULL argument");
  if (bytes < sizeof(StateHeader)) return fail(MM_ERR_ARG, "state blob too small");
  StateHeader hd;
  std::memcpy(&hd, blob, sizeof(hd));
  const size_t mb = sizeof(float) * 3 * c->p.sublattices * (size_t)c->L.ncell;
  if (hd.magic != kMagic || hd.S != c->p.sublattices || hd.N != c->N || hd.ncell != c->L.ncell ||
      hd.ctl_bytes != sizeof(InstCtl) || hd.m_bytes != mb || bytes < sizeof(hd) + sizeof(InstCtl) + mb)
    return fail(MM_ERR_ARG, "state blob does not match this context");
  if (mm_status s = ensure_device(c)) return s;
  InstCtl h;
  std::memcpy(&h, (const char*)blob + sizeof(hd), sizeof(h));
  InstCtl cur;
  if (mm_status s = ctl_pull(c, cur)) return s;
  // keep this context's trace settings
  h.trace_n = cur.trace_n; h.trace_max = cur.trace_max; h.trace_steps = cur.trace_steps;
  h.trace_stride = cur.trace_stride; h.trace_t0 = cur.trace_t0; h.trace_dt = cur.trace_dt;
  h.trace_on = cur.trace_on; h.trace_started = cur.trace_started;
  h.cur = 0;
  h.rec_index = -1;
  for (int j = 0; j < 8; ++j) h.slot[j] = j;
  if (mm_status s = ctl_push(c, h)) return s;
  MM_HIP(hipMemcpy(c->ws + c->L.y[0], (const char*)blob + sizeof(hd) + sizeof(h), mb, hipMemcpyHostToDevice));
  c->m_set = true;
  return MM_OK;
}

namespace {
mm_status ensure_solo(mm_ctx* c) {
  if (c->solo) return MM_OK;
  mm_ctx* one[1] = {c};
  return new_batch(one, 1, &c->solo);
}

// restore the forward part of a checkpointed control block, keeping the
// adjoint accumulators
void restore_forward(InstCtl& dst, const InstCtl& ck) {
  dst.t = ck.t;
  dst.h = ck.h;
  dst.dt = ck.dt;
  dst.clipped = ck.clipped;
  dst.accepted = ck.accepted;
  dst.rejected = ck.rejected;
  std::memcpy(dst.a, ck.a, sizeof(dst.a));
  dst.cur = 0;
  dst.trace_on = 0;               // the recomputation records no trace
}
}  // namespace

mm_status mm_run_record(mm_ctx* c, double T, int32_t every) {
  if (c && c->open_in) return open_error();
  if (!c) return fail(MM_ERR_ARG, "NULL context");
  if (c->method != MM_RK4 || c->split)
    return fail(MM_ERR_STATE, "recording needs the fixed-step RK4 method (DP45: mm_run_record_adaptive)");
  if (c->nonrecip)
    return fail(MM_ERR_STATE, "the adjoint covers reciprocal coupling (g_b = g)");
  if (!(T > 0) || !std::isfinite(T) || every < 1) return fail(MM_ERR_ARG, "need T > 0 and checkpoint_every >= 1");
  if (mm_status s = check_ready(c)) return s;
  const double r = T / c->dt0;
  const long long nsteps = llround(r);
  if (nsteps < 1 || std::fabs(r - (double)nsteps) > 1e-9 * r) return fail(MM_ERR_ARG, "T must be a whole number of steps dt0");
  if (mm_status s = set_device(c)) return s;
  if (mm_status s = ensure_solo(c)) return s;
  const int nck = (int)((nsteps + every - 1) / every);
  const size_t vec = (size_t)3 * c->p.sublattices * c->L.ncell;
  if (c->ck_m) hipFree(c->ck_m);
  c->ck_m = nullptr;
  if (hipMalloc(&c->ck_m, sizeof(float) * vec * nck) != hipSuccess) return fail(MM_ERR_OOM, "checkpoint allocation failed");
  c->ck_ctl.assign(nck, InstCtl{});
  c->rec_have = false;
  long long left = nsteps;
  for (int k = 0; k < nck; ++k) {
    InstCtl h;
    if (mm_status s = ctl_pull(c, h)) return s;
    c->ck_ctl[k] = h;
    MM_HIP(hipMemcpy(c->ck_m + vec * k, c->ws + c->L.y[h.cur], sizeof(float) * vec, hipMemcpyDeviceToDevice));
    const long long steps = std::min<long long>(every, left);
    if (mm_status s = batch_run(c->solo, (double)steps * c->dt0, 0.0)) return s;
    left -= steps;
  }
  c->rec_have = true;
  c->rec_steps = nsteps;
  c->rec_K = every;
  c->rec_nck = nck;
  c->rec_h = c->dt0;
  c->rec_method = MM_RK4;
  return MM_OK;
}

// Replay the logged accepted steps idx0 .. idx_end - 1 of an adaptive
// recorded run from the current state: each step takes its logged size and
// is accepted, and a step logged as clipped lands on the recorded run's own
// end time, so the replay reaches the recorded states bit for bit.
mm_status replay_run(mm_ctx* c, long long idx0, long long idx_end) {
  InstCtl h;
  if (mm_status s = ctl_pull(c, h)) return s;
  h.replay = 1;
  h.replay_idx = idx0;
  h.replay_end = idx_end;
  h.hlog_on = 0;
  h.trace_on = 0;
  if (mm_status s = ctl_push(c, h)) return s;
  const bool sc = c->sampling_changed;
  c->sampling_changed = false;
  const mm_status st = batch_run(c->solo, 0.0, 1.0, c->rec_t_end);
  c->sampling_changed = sc;
  if (st != MM_OK) return st;
  if (mm_status s = ctl_pull(c, h)) return s;
  h.replay = 0;
  return ctl_push(c, h);
}

// (Re)allocate the step log for `cap` accepted steps.
mm_status ensure_step_log(mm_ctx* c, long long cap) {
  if (c->hlog_dev && c->hlog_cap >= cap) return MM_OK;
  if (c->hlog_dev) hipFree(c->hlog_dev);
  c->hlog_dev = nullptr;
  c->hlog_cap = 0;
  if (hipMalloc(&c->hlog_dev, sizeof(double) * (size_t)cap) != hipSuccess) return fail(MM_ERR_OOM, "step log allocation failed");
  c->hlog_cap = cap;
  if (mm_status s = upload_desc(c)) return s;
  return refresh_descs(c->solo);
}

static mm_status adjoint_impl(mm_ctx* c, const double* dL_da, const float* dL_dm, const double* dL_dtrace,
                              float* grad_u, double* grad_g, double* grad_alpha, double* grad_B0,
                              double* grad_a0, float* grad_m0);

mm_status mm_run_record_adaptive(mm_ctx* c, double T, double tol, int32_t every) {
  if (c && c->open_in) return open_error();
  if (!c) return fail(MM_ERR_ARG, "NULL context");
  if (c->method != MM_DP45) return fail(MM_ERR_STATE, "adaptive recording needs the DP45 method");
  if (c->nonrecip) return fail(MM_ERR_STATE, "the adjoint covers reciprocal coupling (g_b = g)");
  if (!(T > 0) || !std::isfinite(T) || every < 1) return fail(MM_ERR_ARG, "need T > 0 and checkpoint_every >= 1");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(MM_ERR_ARG, "DP45 needs a finite tol > 0");
  if (mm_status s = check_ready(c)) return s;
  if (mm_status s = set_device(c)) return s;
  if (mm_status s = ensure_solo(c)) return s;
  const size_t vec = (size_t)3 * c->p.sublattices * c->L.ncell;
  c->rec_have = false;
  // the start state
  InstCtl h0;
  if (mm_status s = ctl_pull(c, h0)) return s;
  std::vector<float> m0(vec);
  MM_HIP(hipMemcpy(m0.data(), c->ws + c->L.y[h0.cur], sizeof(float) * vec, hipMemcpyDeviceToHost));
  // 1. the adaptive run, logging the size of every accepted step (run again
  //    from the start with a larger log if it fills)
  long long cap = std::max<long long>(1024, c->hlog_cap);
  InstCtl hend;
  double wall_run = 0.0;
  for (;;) {
    if (mm_status s = ensure_step_log(c, cap)) return s;
    InstCtl h = h0;
    h.hlog_on = 1;
    h.hlog_n = 0;
    h.replay = 0;
    if (mm_status s = ctl_push(c, h)) return s;
    MM_HIP(hipMemcpy(c->ws + c->L.y[h0.cur], m0.data(), sizeof(float) * vec, hipMemcpyHostToDevice));
    if (mm_status s = batch_run(c->solo, T, tol)) return s;
    wall_run = c->stats.wall_s;
    if (mm_status s = ctl_pull(c, hend)) return s;
    if (hend.hlog_n <= c->hlog_cap) break;
    cap = 2 * hend.hlog_n;
  }
  const long long n = hend.hlog_n;
  if (n < 1) return fail(MM_ERR_STATE, "the run took no step");
  c->rec_hs.assign((size_t)n, 0.0);
  MM_HIP(hipMemcpy(c->rec_hs.data(), c->hlog_dev, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost));
  c->rec_t_end = hend.t_end;
  // 2. checkpoints every `every` steps along the replay of the logged steps
  const int nck = (int)((n + every - 1) / every);
  if (c->ck_m) hipFree(c->ck_m);
  c->ck_m = nullptr;
  if (hipMalloc(&c->ck_m, sizeof(float) * vec * nck) != hipSuccess) return fail(MM_ERR_OOM, "checkpoint allocation failed");
  c->ck_ctl.assign(nck, InstCtl{});
  {
    InstCtl h = h0;
    h.hlog_on = 0;
    if (mm_status s = ctl_push(c, h)) return s;
    MM_HIP(hipMemcpy(c->ws + c->L.y[h0.cur], m0.data(), sizeof(float) * vec, hipMemcpyHostToDevice));
  }
  for (int k = 0; k < nck; ++k) {
    InstCtl h;
    if (mm_status s = ctl_pull(c, h)) return s;
    c->ck_ctl[k] = h;
    MM_HIP(hipMemcpy(c->ck_m + vec * k, c->ws + c->L.y[h.cur], sizeof(float) * vec, hipMemcpyDeviceToDevice));
    if (mm_status s = replay_run(c, (long long)k * every, std::min<long long>((long long)(k + 1) * every, n))) return s;
  }
  // the replay has reached the recorded run's end state; its own control
  // block (step-size controller, counters, trace) comes back
  hend.hlog_on = 0;
  hend.replay = 0;
  if (mm_status s = ctl_push(c, hend)) return s;
  set_stats(c, hend, wall_run);
  c->rec_have = true;
  c->rec_steps = n;
  c->rec_K = every;
  c->rec_nck = nck;
  c->rec_h = 0.0;
  c->rec_method = MM_DP45;
  return MM_OK;
}

mm_status mm_get_step_log(const mm_ctx* c, double* h, int64_t* n) {
  if (c && c->open_in) return open_error();
  if (!c || !n) return fail(MM_ERR_ARG, "NULL argument");
  if (!c->rec_have || c->rec_method != MM_DP45) return fail(MM_ERR_STATE, "no adaptive recorded run (mm_run_record_adaptive)");
  const int64_t cnt = (int64_t)c->rec_hs.size();
  if (h) std::memcpy(h, c->rec_hs.data(), sizeof(double) * (size_t)std::min<int64_t>(*n, cnt));
  *n = cnt;
  return MM_OK;
}

mm_status mm_adjoint(mm_ctx* c, const double* dL_da, const float* dL_dm, float* grad_u, double* grad_g,
                     double* grad_alpha, double* grad_B0, double* grad_a0, float* grad_m0) {
  if (c && c->open_in) return open_error();
  return adjoint_impl(c, dL_da, dL_dm, nullptr, grad_u, grad_g, grad_alpha, grad_B0, grad_a0, grad_m0);
}

mm_status mm_adjoint_trace(mm_ctx* c, const double* dL_dtrace, int64_t count, const double* dL_da,
                           const float* dL_dm, float* grad_u, double* grad_g, double* grad_alpha,
                           double* grad_B0, double* grad_a0, float* grad_m0) {
  if (!c || !dL_dtrace) return fail(MM_ERR_ARG, "NULL context or dL_dtrace");
  if (!c->rec_have) return fail(MM_ERR_STATE, "no recorded run (mm_run_record)");
  if (count != c->rec_steps + 1) return fail(MM_ERR_ARG, "dL_dtrace needs one entry per step end and the start");
  const size_t n = (size_t)count * 2 * std::max(1, c->N);
  for (size_t i = 0; i < (size_t)count * 2 * c->N; ++i)
    if (!std::isfinite(dL_dtrace[i])) return fail(MM_ERR_ARG, "non-finite dL_dtrace");
  if (mm_status s = set_device(c)) return s;
  // the layout [count][N][2] as given, padded to at least one mode
  std::vector<double> hbuf(n, 0.0);
  for (int64_t k = 0; k < count; ++k)
    for (int q = 0; q < 2 * c->N; ++q) hbuf[(size_t)k * 2 * std::max(1, c->N) + q] = dL_dtrace[(size_t)k * 2 * c->N + q];
  double* dev = nullptr;
  if (hipMalloc(&dev, sizeof(double) * n) != hipSuccess) return fail(MM_ERR_OOM, "trace adjoint allocation failed");
  mm_status st = MM_OK;
  if (hipMemcpy(dev, hbuf.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess) {
    st = fail(MM_ERR_HIP, "trace adjoint copy failed");
  } else {
    std::vector<double> zero(2 * std::max(1, c->N), 0.0);
    c->dla_dev = dev;
    st = adjoint_impl(c, dL_da ? dL_da : zero.data(), dL_dm, dL_dtrace, grad_u, grad_g, grad_alpha, grad_B0,
                      grad_a0, grad_m0);
    c->dla_dev = nullptr;
    const mm_status s2 = upload_desc(c);
    if (st == MM_OK) st = s2;
  }
  hipFree(dev);
  return st;
}

static mm_status adjoint_impl(mm_ctx* c, const double* dL_da, const float* dL_dm, const double* dL_dtrace,
                              float* grad_u, double* grad_g, double* grad_alpha, double* grad_B0,
                              double* grad_a0, float* grad_m0) {
  if (!c || !dL_da) return fail(MM_ERR_ARG, "NULL context or dL_da");
  if (!c->rec_have) return fail(MM_ERR_STATE, "no recorded run (mm_run_record)");
  if (c->nonrecip)
    return fail(MM_ERR_STATE, "the adjoint covers reciprocal coupling (g_b = g)");
  if (mm_status s = set_device(c)) return s;
  const int N = c->N, S = c->p.sublattices, K = c->rec_K;
  const size_t nc = (size_t)c->L.ncell, vec = (size_t)3 * S * nc;
  for (int i = 0; i < 2 * N; ++i)
    if (!std::isfinite(dL_da[i])) return fail(MM_ERR_ARG, "non-finite dL_da");
  // adjoint buffers for segments of K steps
  const bool dp = c->rec_method == MM_DP45;
  if (dp && dL_dtrace) return fail(MM_ERR_STATE, "losses on the trace are built for fixed-step RK4 runs");
  if (dp != (c->method == MM_DP45)) return fail(MM_ERR_STATE, "the stepper changed since the run was recorded");
  const int ns = dp ? 6 : 4;
  if (c->adj_K != K || c->adj_N != N || c->adj_nstg != ns) {
    if (c->adj_f) hipFree(c->adj_f);
    if (c->adj_d) hipFree(c->adj_d);
    c->adj_f = nullptr;
    c->adj_d = nullptr;
    c->adj_K = -1;
    // stage inputs, norms, five adjoint vectors and, with FFT demag, the demag
    // field of every recorded stage input (the reverse pass then needs one
    // convolution per stage instead of two); DP45: the mu of stages 3..6 and
    // the start time of every step
    const size_t nf = (size_t)(K + 1) * ns * vec + (size_t)K * S * nc + 5 * vec +
                      (c->L.fft ? (size_t)(K + (dp ? 1 : 0)) * ns * 3 * nc : 0) + (dp ? 4 * vec : 0);
    const size_t nd = (size_t)K * ns * std::max(1, N) * 2 + (size_t)std::max(1, N) * nc + (dp ? (size_t)K : 0);
    if (hipMalloc(&c->adj_f, sizeof(float) * nf) != hipSuccess) return fail(MM_ERR_OOM, "adjoint allocation failed");
    if (hipMalloc(&c->adj_d, sizeof(double) * nd) != hipSuccess) return fail(MM_ERR_OOM, "adjoint allocation failed");
    c->adj_K = K;
    c->adj_N = N;
    c->adj_nstg = ns;
  }
  c->adj_on = true;
  if (mm_status s = upload_desc(c)) return s;
  // the end state, restored afterwards
  InstCtl end;
  if (mm_status s = ctl_pull(c, end)) return s;
  std::vector<float> m_end(vec);
  MM_HIP(hipMemcpy(m_end.data(), c->ws + c->L.y[end.cur], sizeof(float) * vec, hipMemcpyDeviceToHost));
  // initial adjoint
  {
    InstCtl h = end;
    std::memset(h.la, 0, sizeof(h.la));
    for (int n = 0; n < N; ++n) {
      h.la[n][0] = dL_da[2 * n];
      h.la[n][1] = dL_da[2 * n + 1];
    }
    std::memset(h.grad_g, 0, sizeof(h.grad_g));
    h.grad_alpha = 0.0;
    h.grad_B0[0] = h.grad_B0[1] = h.grad_B0[2] = 0.0;
    h.adj_h = c->rec_h;
    if (mm_status s = ctl_push(c, h)) return s;
    std::vector<float> l0(vec, 0.f);
    if (dL_dm) std::memcpy(l0.data(), dL_dm, sizeof(float) * vec);
    MM_HIP(hipMemcpy(c->desc.lam_y, l0.data(), sizeof(float) * vec, hipMemcpyHostToDevice));
    MM_HIP(hipMemset(c->desc.grad_u, 0, sizeof(double) * std::max(1, N) * nc));
  }
  mm_batch* b = c->solo;
  if (mm_status s = refresh_descs(b)) return s;
  if (mm_status s = ensure_reverse_graph(b)) return s;
  const auto t0 = std::chrono::steady_clock::now();
  for (int k = c->rec_nck - 1; k >= 0; --k) {
    const long long steps = std::min<long long>(K, c->rec_steps - (long long)k * K);
    // restore the checkpoint and recompute the segment, keeping its stages
    InstCtl h;
    if (mm_status s = ctl_pull(c, h)) return s;
    restore_forward(h, c->ck_ctl[k]);
    if (mm_status s = ctl_push(c, h)) return s;
    MM_HIP(hipMemcpy(c->ws + c->L.y[0], c->ck_m + vec * k, sizeof(float) * vec, hipMemcpyDeviceToDevice));
    c->record_next = 0;
    if (dp) {
      // the replay records every stage input, the stage-7 one as the next
      // step's first, so the state after the segment is in place too
      if (mm_status s = replay_run(c, (long long)k * K, (long long)k * K + steps)) return s;
      if (mm_status s = ctl_pull(c, h)) return s;
    } else {
      if (mm_status s = batch_run(b, (double)steps * c->rec_h, 0.0)) return s;
      if (mm_status s = ctl_pull(c, h)) return s;
      MM_HIP(hipMemcpy(c->desc.rec_m + (size_t)steps * 4 * vec, c->ws + c->L.y[h.cur], sizeof(float) * vec,
                       hipMemcpyDeviceToDevice));
    }
    // reverse the segment
    h.rec_index = (int)steps - 1;
    h.adj_base = (long long)k * K;
    h.done = 0;
    h.adj_h = c->rec_h;
    h.adj_t0 = c->ck_ctl[k].t;
    if (mm_status s = ctl_push(c, h)) return s;
    for (long long q = 0; q < steps; ++q) MM_HIP(hipGraphLaunch(b->exec_rev, b->stream));
    MM_HIP(hipStreamSynchronize(b->stream));
  }
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  // outputs
  InstCtl h;
  if (mm_status s = ctl_pull(c, h)) return s;
  if (grad_g) for (int n = 0; n < N; ++n) grad_g[n] = h.grad_g[n];
  if (grad_alpha) *grad_alpha = h.grad_alpha;
  if (grad_B0) for (int q = 0; q < 3; ++q) grad_B0[q] = h.grad_B0[q];
  // the trace loss at the start acts on a0 directly
  if (grad_a0)
    for (int n = 0; n < N; ++n) {
      grad_a0[2 * n] = h.la[n][0] + (dL_dtrace ? dL_dtrace[2 * n] : 0.0);
      grad_a0[2 * n + 1] = h.la[n][1] + (dL_dtrace ? dL_dtrace[2 * n + 1] : 0.0);
    }
  if (grad_m0) MM_HIP(hipMemcpy(grad_m0, c->desc.lam_y, sizeof(float) * vec, hipMemcpyDeviceToHost));
  if (grad_u && N > 0) {
    std::vector<double> gu((size_t)N * nc);
    MM_HIP(hipMemcpy(gu.data(), c->desc.grad_u, sizeof(double) * gu.size(), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < gu.size(); ++i) grad_u[i] = (float)gu[i];
  }
  // back to the end state of the recorded run
  InstCtl fin = h;
  restore_forward(fin, end);
  fin.cur = end.cur;
  fin.rec_index = -1;
  fin.status = end.status;
  fin.done = end.done;
  fin.trace_on = end.trace_on;
  if (mm_status s = ctl_push(c, fin)) return s;
  MM_HIP(hipMemcpy(c->ws + c->L.y[end.cur], m_end.data(), sizeof(float) * vec, hipMemcpyHostToDevice));
  c->stats.wall_s = wall;
  return MM_OK;
}

mm_status mm_batch_create(mm_ctx* const* ctxs, int32_t count, mm_batch** out) {
  if (!ctxs || !out || count < 1) return fail(MM_ERR_ARG, "need count >= 1 contexts and an output");
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i]) return fail(MM_ERR_ARG, "NULL context in batch");
    if (ctxs[i]->open_in) return open_error();
    if (mm_status s = check_ready(ctxs[i])) return s;
    if (ctxs[i]->method != ctxs[0]->method) return fail(MM_ERR_ARG, "all instances need the same method");
    if (ctxs[i]->dev != ctxs[0]->dev) return fail(MM_ERR_ARG, "all instances need the same device");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(MM_ERR_ARG, "a context appears twice in the batch");
  }
  if (mm_status s = set_device(ctxs[0])) return s;
  return make_batch(ctxs, count, kDefaultParts, out);
}

mm_status mm_batch_set_streams(mm_batch* b, int32_t parts) {
  if (b && batch_busy(b)) return open_error();
  if (!b) return fail(MM_ERR_ARG, "batch is NULL");
  if (parts < 1 || parts > 8) return fail(MM_ERR_ARG, "parts must be 1..8");
  if (mm_status s = set_device(b->ctxs[0])) return s;
  for (mm_batch* p : b->parts) MM_HIP(hipStreamSynchronize(p->stream));
  if (b->stream) MM_HIP(hipStreamSynchronize(b->stream));
  mm_batch* nb = nullptr;
  if (mm_status s = make_batch(b->ctxs.data(), (int)b->ctxs.size(), parts, &nb)) return s;
  // the handle stays valid: it takes the new contents, the old ones are freed
  std::swap(*b, *nb);
  return mm_batch_destroy(nb);
}

mm_status mm_batch_get_streams(const mm_batch* b, int32_t* parts) {
  if (!b || !parts) return fail(MM_ERR_ARG, "bad arguments");
  *parts = b->parts.empty() ? 1 : (int32_t)b->parts.size();
  return MM_OK;
}

mm_status mm_batch_run(mm_batch* b, double T, double tol) {
  if (b && batch_busy(b)) return open_error();
  if (!b) return fail(MM_ERR_ARG, "NULL batch");
  if (!(T > 0) || !std::isfinite(T)) return fail(MM_ERR_ARG, "T must be finite and > 0");
  if (mm_status s = validate_tol(b, tol)) return s;
  for (mm_ctx* c : b->ctxs)
    if (c->method != b->method) return fail(MM_ERR_STATE, "instance method changed after batch creation");
  if (mm_status s = set_device(b->ctxs[0])) return s;
  if (!b->parts.empty()) return parts_run(b, T, tol);
  return batch_run(b, T, tol);
}

mm_status mm_batch_step(mm_batch* b, int64_t steps, double tol) {
  if (!b || steps < 0) return fail(MM_ERR_ARG, "bad arguments");
  if (b->open) return fail(MM_ERR_STATE, "the batch has an open run (mm_batch_end first)");
  if (mm_status s = validate_tol(b, tol)) return s;
  if (mm_status s = set_device(b->ctxs[0])) return s;
  const auto t0 = std::chrono::steady_clock::now();
  if (mm_status s = open_run(b, tol)) return s;
  if (mm_status s = launch_steps(b, steps)) return s;
  for (mm_batch* p : b->parts) MM_HIP(hipStreamSynchronize(p->stream));
  MM_HIP(hipStreamSynchronize(b->stream));
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return close_run(b, wall);
}

mm_status mm_batch_begin(mm_batch* b, double tol) {
  if (!b) return fail(MM_ERR_ARG, "batch is NULL");
  if (b->open) return fail(MM_ERR_STATE, "the batch already has an open run");
  if (mm_status s = validate_tol(b, tol)) return s;
  for (mm_ctx* c : b->ctxs) {
    if (c->method != b->method) return fail(MM_ERR_STATE, "instance method changed after batch creation");
    if (c->open_in) return fail(MM_ERR_STATE, "an instance of the batch is in another open run");
  }
  if (mm_status s = set_device(b->ctxs[0])) return s;
  if (mm_status s = open_run(b, tol)) return s;
  // capture every step graph now, so that mm_batch_advance only launches
  std::vector<mm_batch*> seq = b->parts;
  if (seq.empty()) seq.push_back(b);
  for (mm_batch* p : seq) {
    if (mm_status s = ensure_graph(p)) return s;
    for (int lg = 0; lg < 5; ++lg)
      if (mm_status s = ensure_graph_pow(p, lg)) return s;
  }
  b->open = true;
  b->open_t0 = std::chrono::steady_clock::now();
  for (mm_ctx* c : b->ctxs) c->open_in = b;
  return MM_OK;
}

mm_status mm_batch_advance(mm_batch* b, int64_t steps) {
  if (!b || steps < 0) return fail(MM_ERR_ARG, "bad arguments");
  if (!b->open) return fail(MM_ERR_STATE, "no open run (mm_batch_begin first)");
  if (mm_status s = set_device(b->ctxs[0])) return s;
  return launch_steps(b, steps);
}

mm_status mm_batch_counts(mm_batch* b, int64_t* accepted, int64_t* rejected) {
  if (!b) return fail(MM_ERR_ARG, "batch is NULL");
  if (mm_status s = set_device(b->ctxs[0])) return s;
  MM_HIP(hipStreamSynchronize(b->stream));
  for (mm_batch* p : b->parts) MM_HIP(hipStreamSynchronize(p->stream));
  int64_t acc = 0, rej = 0;
  for (const mm_ctx* c : b->ctxs) {
    InstCtl h;
    if (mm_status s = ctl_pull(c, h)) return s;
    acc += h.accepted;
    rej += h.rejected;
  }
  if (accepted) *accepted = acc;
  if (rejected) *rejected = rej;
  return MM_OK;
}

mm_status mm_batch_end(mm_batch* b) {
  if (!b) return fail(MM_ERR_ARG, "batch is NULL");
  if (!b->open) return fail(MM_ERR_STATE, "no open run (mm_batch_begin first)");
  if (mm_status s = set_device(b->ctxs[0])) return s;
  b->open = false;
  for (mm_ctx* c : b->ctxs) c->open_in = nullptr;
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - b->open_t0).count();
  return close_run(b, wall);
}

static mm_status check_fft_path(const mm_batch* b, int32_t path) {
  if (path != PATH_FUSED && path != PATH_REG && path != PATH_SPLIT && path != PATH_REG8 && path != PATH_XCH &&
      path != PATH_SPLITX)
    return fail(MM_ERR_ARG, "unknown y-z path");
  for (const mm_batch* p : b->parts)
    if (mm_status s = check_fft_path(p, path)) return s;
  for (auto& g : b->groups) {
    if (path == PATH_REG && !reg_fits(g.ny, g.nz, g.py, g.pz))
      return fail(MM_ERR_ARG, "register y-z path needs padded y in 16..128 and padded z in 16..64");
    if (path == PATH_REG8 && !reg8_fits(g.ny, g.nz, g.py, g.pz))
      return fail(MM_ERR_ARG, "eight-lane register y-z path needs padded y in 16..128 and padded z of 32 or 64");
    if (path == PATH_SPLITX && !splitx_fits(g.py))
      return fail(MM_ERR_ARG, "split exchange y-z path needs padded y in 16..256");
    if (path == PATH_XCH && !xch_fits(g.ny, g.nz, g.py, g.pz))
      return fail(MM_ERR_ARG, "exchange y-z path needs padded y in 16..128 and padded z of 32 or 64");
    if (path == PATH_FUSED && !fused_fits(g.ny, g.nz, g.py, g.pz))
      return fail(MM_ERR_ARG, "fused y-z path does not fit in LDS for this grid");
  }
  return MM_OK;
}

mm_status mm_batch_set_fft_path(mm_batch* b, int32_t path) {
  if (b && batch_busy(b)) return open_error();
  if (!b) return fail(MM_ERR_ARG, "batch is NULL");
  if (mm_status s = check_fft_path(b, path)) return s;
  for (mm_batch* p : b->parts)
    if (mm_status s = mm_batch_set_fft_path(p, path)) return s;
  if (!b->parts.empty()) return MM_OK;
  MM_HIP(hipStreamSynchronize(b->stream));
  for (auto& g : b->groups) {
    g.path = path;
    if (path == PATH_FUSED) g.TK = std::max(1, fused_tile(g.ny, g.nz, g.py, g.pz));
    if (mm_status s = build_group(g)) return s;
  }
  drop_graphs(b);
  return MM_OK;
}

static mm_status check_fft_x(const mm_batch* b, int32_t path) {
  if (path != MM_X_LDS && path != MM_X_REGISTER && path != MM_X_STAGE) return fail(MM_ERR_ARG, "unknown x path");
  for (const mm_batch* p : b->parts)
    if (mm_status s = check_fft_x(p, path)) return s;
  for (auto& g : b->groups) {
    if (path == MM_X_REGISTER && !xreg_fits(g.px))
      return fail(MM_ERR_ARG, "register x path needs a padded x of 16..128 cells");
    if (path == MM_X_STAGE && !g.xfused && !xfuse_fits(g.nx))
      return fail(MM_ERR_ARG, "x passes in the stage kernels need nx a power of two from 2 to 256");
    if (path == MM_X_STAGE)
      for (int m : g.members)
        if (b->ctxs[m]->p.sublattices != 1) return fail(MM_ERR_ARG, "x passes in the stage kernels need one sublattice");
  }
  return MM_OK;
}

mm_status mm_batch_set_fft_x(mm_batch* b, int32_t path) {
  if (b && batch_busy(b)) return open_error();
  if (!b) return fail(MM_ERR_ARG, "batch is NULL");
  if (mm_status s = check_fft_x(b, path)) return s;
  for (mm_batch* p : b->parts)
    if (mm_status s = mm_batch_set_fft_x(p, path)) return s;
  if (!b->parts.empty()) return MM_OK;
  MM_HIP(hipStreamSynchronize(b->stream));
  for (auto& g : b->groups) {
    g.xfused = path == MM_X_STAGE;
    g.Wx = path == MM_X_REGISTER ? 0 : std::max(1, std::min(16, 1024 / g.px));
    if (mm_status s = build_group(g)) return s;
  }
  batch_xfused(b);
  if (mm_status s = upload_batch_descs(b)) return s;
  drop_graphs(b);
  return MM_OK;
}

mm_status mm_batch_profile(mm_batch* b, int64_t steps, double tol, int32_t cap, char* names, int64_t* launches,
                           double* total_ms, double* bytes_per_launch, int32_t* n) {
  if (b && batch_busy(b)) return open_error();
  if (!b || !n || steps < 0 || cap < 0) return fail(MM_ERR_ARG, "bad arguments");
  if (mm_status s = validate_tol(b, tol)) return s;
  if (mm_status s = set_device(b->ctxs[0])) return s;
  if (!b->parts.empty()) {
    // kernels of the whole batch as one launch sequence, one at a time, with
    // the FFT strategies the parts use
    for (mm_batch* p : b->parts) MM_HIP(hipStreamSynchronize(p->stream));
    mm_batch* whole = nullptr;
    if (mm_status s = new_batch(b->ctxs.data(), (int)b->ctxs.size(), &whole)) return s;
    mm_status s = copy_fft_settings(whole, b->parts[0]);
    if (s == MM_OK)
      s = mm_batch_profile(whole, steps, tol, cap, names, launches, total_ms, bytes_per_launch, n);
    mm_batch_destroy(whole);
    return s;
  }
  b->prof.clear();
  if (mm_status s = begin_run(b, -1.0, tol)) return s;
  MM_HIP(hipStreamSynchronize(b->stream));
  b->profiling = true;
  mm_status st = MM_OK;
  for (int64_t k = 0; k < steps && st == MM_OK; ++k) st = enqueue_step(b);
  b->profiling = false;
  hipError_t e = hipStreamSynchronize(b->stream);
  for (size_t q = 0; q < b->pending.size(); ++q) {
    float ms = 0.f;
    if (e == hipSuccess) hipEventElapsedTime(&ms, b->pending[q].first, b->pending[q].second);
    b->prof[b->pending_idx[q]].ms += ms;
    b->prof[b->pending_idx[q]].launches += 1;
    hipEventDestroy(b->pending[q].first);
    hipEventDestroy(b->pending[q].second);
  }
  b->pending.clear();
  b->pending_idx.clear();
  if (st != MM_OK) return st;
  if (e != hipSuccess) return fail(MM_ERR_HIP, std::string("profile: ") + hipGetErrorString(e));
  if (mm_status s = end_run(b, 0.0)) return s;
  const int cnt = (int)std::min<size_t>(cap, b->prof.size());
  for (int i = 0; i < cnt; ++i) {
    if (names) {
      std::memset(names + 48 * i, 0, 48);
      std::strncpy(names + 48 * i, b->prof[i].name.c_str(), 47);
    }
    if (launches) launches[i] = b->prof[i].launches;
    if (total_ms) total_ms[i] = b->prof[i].ms;
    if (bytes_per_launch) bytes_per_launch[i] = b->prof[i].bytes;
  }
  *n = (int)b->prof.size();
  return MM_OK;
}

// Insert `fields` (JSON members) at the start of every top-level object of
// the JSON list `list`.
static std::string add_to_entries(const std::string& list, const std::string& fields) {
  std::string out;
  int depth = 0;
  for (char ch : list) {
    out += ch;
    if (ch == '{') {
      if (depth == 1) out += fields + ", ";
      ++depth;
    } else if (ch == '[') {
      ++depth;
    } else if (ch == ']' || ch == '}') {
      --depth;
    }
  }
  return out;
}

// Everything of a context that a timed run changes: the control block, the
// state vector it points to and the host-side run bookkeeping.
struct SavedRun {
  InstCtl h;
  std::vector<char> y;
  mm_stats stats;
  bool sampling_changed;
  int record_next;
};

static mm_status save_run(mm_ctx* c, SavedRun& sv) {
  if (mm_status s = ctl_pull(c, sv.h)) return s;
  sv.y.resize(sizeof(float) * 3 * c->p.sublattices * (size_t)c->L.ncell);
  MM_HIP(hipMemcpy(sv.y.data(), c->ws + c->L.y[sv.h.cur], sv.y.size(), hipMemcpyDeviceToHost));
  sv.stats = c->stats;
  sv.sampling_changed = c->sampling_changed;
  sv.record_next = c->record_next;
  return MM_OK;
}

static mm_status restore_run(mm_ctx* c, const SavedRun& sv) {
  if (mm_status s = ctl_push(c, sv.h)) return s;
  MM_HIP(hipMemcpy(c->ws + c->L.y[sv.h.cur], sv.y.data(), sv.y.size(), hipMemcpyHostToDevice));
  c->stats = sv.stats;
  c->sampling_changed = sv.sampling_changed;
  c->record_next = sv.record_next;
  return MM_OK;
}

// Choose how many concurrent sub-batches (1 .. kMaxTunedParts) the batch
// runs as by timing whole steps of each candidate partition; the fastest one
// (the very object timed, so its streams stay as measured) replaces b's
// contents.  Every instance's state is restored afterwards.
static mm_status tune_streams(mm_batch* b, std::string& rep) {
  const int count = (int)b->ctxs.size();
  std::vector<SavedRun> saved(count);
  for (int i = 0; i < count; ++i)
    if (mm_status s = save_run(b->ctxs[i], saved[i])) return s;
  const double tol = saved[0].h.tol > 0 ? saved[0].h.tol : 1e-6;
  std::vector<mm_batch*> cand;
  std::vector<double> ms;
  mm_status st = MM_OK;
  for (int parts = 1; parts <= std::min(kMaxTunedParts, count) && st == MM_OK; ++parts) {
    mm_batch* c = nullptr;
    st = make_batch(b->ctxs.data(), count, parts, &c);
    if (st != MM_OK) break;
    cand.push_back(c);
    double best = 1e300;
    st = mm_batch_step(c, kStepsPerGraph, tol);    // captures the graphs
    for (int rep_i = 0; rep_i < 2 && st == MM_OK; ++rep_i) {
      const auto t0 = std::chrono::steady_clock::now();
      st = mm_batch_step(c, 2 * kStepsPerGraph, tol);
      best = std::min(best, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    }
    ms.push_back(best * 1e3 / (2 * kStepsPerGraph));
    for (int i = 0; i < count && st == MM_OK; ++i) st = restore_run(b->ctxs[i], saved[i]);
  }
  if (st == MM_OK) {
    const int k = (int)(std::min_element(ms.begin(), ms.end()) - ms.begin());
    std::swap(*b, *cand[k]);
    rep = "\"streams_ms_per_step\": [";
    for (size_t i = 0; i < ms.size(); ++i) rep += (i ? ", " : "") + std::to_string(ms[i]);
    rep += "], \"streams\": " + std::to_string(k + 1);
  }
  for (mm_batch* c : cand) mm_batch_destroy(c);   // the chosen slot now holds b's old contents
  if (st != MM_OK)
    for (int i = 0; i < count; ++i) restore_run(b->ctxs[i], saved[i]);
  return st;
}

static mm_status tune_fft(mm_batch* b, std::string& rep);

static mm_status tune_all_fft(mm_batch* b, const std::string& srep, char* report, size_t report_len);

mm_status mm_batch_tune(mm_batch* b, char* report, size_t report_len) {
  if (b && batch_busy(b)) return open_error();
  if (!b) return fail(MM_ERR_ARG, "NULL batch");
  if (mm_status s = set_device(b->ctxs[0])) return s;
  std::string srep;
  if (b->ctxs.size() >= 2)
    if (mm_status s = tune_streams(b, srep)) return s;
  return tune_all_fft(b, srep, report, report_len);
}

mm_status mm_batch_tune_fft(mm_batch* b, char* report, size_t report_len) {
  if (b && batch_busy(b)) return open_error();
  if (!b) return fail(MM_ERR_ARG, "NULL batch");
  if (mm_status s = set_device(b->ctxs[0])) return s;
  return tune_all_fft(b, "", report, report_len);
}

static mm_status tune_all_fft(mm_batch* b, const std::string& srep, char* report, size_t report_len) {
  // each part tunes its own launches; the reports are joined into one list
  std::string all;
  std::vector<mm_batch*> leaves = b->parts;
  if (leaves.empty()) leaves.push_back(b);
  for (size_t k = 0; k < leaves.size(); ++k) {
    std::string r;
    if (mm_status s = tune_fft(leaves[k], r)) return s;
    r = add_to_entries(r, "\"part\": " + std::to_string(k));
    if (r.size() >= 2) r = r.substr(1, r.size() - 2);
    if (!r.empty()) all += (all.empty() ? "" : ", ") + r;
  }
  all = "[" + all + "]";
  if (!srep.empty()) all = add_to_entries(all, srep);
  if (report && report_len) {
    std::strncpy(report, all.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return MM_OK;
}

// FFT tiles and paths of one launch sequence (a batch without parts).
static mm_status tune_fft(mm_batch* b, std::string& out) {
  // make every instance runnable without touching its state
  for (mm_ctx* c : b->ctxs) {
    InstCtl h;
    if (mm_status s = ctl_pull(c, h)) return s;
    h.done = 0;
    if (mm_status s = ctl_push(c, h)) return s;
  }
  if (mm_status s = refresh_descs(b)) return s;
  hipEvent_t e0, e1;
  MM_HIP(hipEventCreate(&e0));
  MM_HIP(hipEventCreate(&e1));
  std::string rep = "[";
  const int reps = 3;
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    auto& g = b->groups[gi];
    auto timed = [&](auto&& enqueue, double* us) -> mm_status {
      MM_HIP(enqueue());
      MM_HIP(hipEventRecord(e0, b->stream));
      for (int r = 0; r < reps; ++r) MM_HIP(enqueue());
      MM_HIP(hipEventRecord(e1, b->stream));
      MM_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      MM_HIP(hipEventElapsedTime(&ms, e0, e1));
      *us = 1e3 * ms / reps;
      return MM_OK;
    };
    const size_t lds_cap = 64 * 1024;
    // x passes: tile width
    int bestW = g.Wx;
    double bestT = 1e30;
    std::string xrep;
    for (int W = xreg_fits(g.px) ? 0 : 2; W <= 32; W = W ? 2 * W : 2) {
      if (W && sizeof(float2) * ((size_t)g.px * (W + 1) + (size_t)g.kx * 2 * W + g.px) > lds_cap) continue;
      g.Wx = W;
      if (mm_status s = build_group(g)) return s;
      double us;
      if (mm_status s = timed([&] {
            if (g.Wx == 0) {
              hipError_t e = mmk_launch_fft_xr(1, g.px / 4, g.n_xf, b->d_desc, g.xf, b->method, 1, g_twiddle, b->stream);
              if (e != hipSuccess) return e;
              return mmk_launch_fft_xr(-1, g.px / 4, g.n_xf, b->d_desc, g.xf, 0, 0, g_twiddle, b->stream);
            }
            hipError_t e = mmk_launch_fft_xf(g.Wx, g.n_xf, g.lds_xf, b->d_desc, g.xf, b->method, 1, g_twiddle, b->stream);
            if (e != hipSuccess) return e;
            return mmk_launch_fft_xi(g.Wx, g.n_xf, g.lds_xi, b->d_desc, g.xf, g_twiddle, b->stream);
          }, &us))
        return s;
      xrep += (xrep.empty() ? "" : ", ") + std::string("\"") + (W ? std::to_string(W) : std::string("reg")) + "\": " +
              std::to_string(us);
      if (us < bestT) { bestT = us; bestW = W; }
    }
    g.Wx = bestW;
    // y-z passes: fused vs split with tile widths
    int bestPath = g.path;
    int bestWy = g.Wy, bestTW = g.TW;
    double bestYZ = 1e30;
    std::string yrep;
    int bestTK = g.TK;
    for (int tk = std::min(16, g.py); tk >= 1 && fused_fits(g.ny, g.nz, g.py, g.pz); tk /= 2) {
      if (fused_lds(g.ny, g.nz, g.py, g.pz, tk) > 160 * 1024) continue;
      g.path = PATH_FUSED;
      g.TK = tk;
      if (mm_status s = build_group(g)) return s;
      double us;
      if (mm_status s = timed([&] { return mmk_launch_fft_yz(g.TK, g.n_yz, g.lds_yz, b->d_desc, g.yz, g_twiddle, b->stream); }, &us))
        return s;
      yrep += (yrep.empty() ? "" : ", ") + std::string("\"fused_") + std::to_string(tk) + "\": " + std::to_string(us);
      if (us < bestYZ) { bestYZ = us; bestPath = PATH_FUSED; bestTK = tk; }
      if (tk <= 2) break;
    }
    if (reg_fits(g.ny, g.nz, g.py, g.pz)) {
      g.path = PATH_REG;
      if (mm_status s = build_group(g)) return s;
      double us;
      if (mm_status s = timed([&] {
            return mmk_launch_fft_yzr(g.py / 4, g.pz / 4, g.n_yz, g.lds_yz, b->d_desc, g.yz, g_twiddle, b->stream);
          }, &us))
        return s;
      yrep += (yrep.empty() ? "" : ", ") + std::string("\"reg\": ") + std::to_string(us);
      if (us < bestYZ) { bestYZ = us; bestPath = PATH_REG; }
    }
    if (reg8_fits(g.ny, g.nz, g.py, g.pz)) {
      g.path = PATH_REG8;
      if (mm_status s = build_group(g)) return s;
      double us;
      if (mm_status s = timed([&] {
            return mmk_launch_fft_yz8(g.py / 4, g.pz / 4, g.n_yz, g.lds_yz, b->d_desc, g.yz, g_twiddle, b->stream);
          }, &us))
        return s;
      yrep += (yrep.empty() ? "" : ", ") + std::string("\"reg8\": ") + std::to_string(us);
      if (us < bestYZ) { bestYZ = us; bestPath = PATH_REG8; }
    }
    if (xch_fits(g.ny, g.nz, g.py, g.pz)) {
      g.path = PATH_XCH;
      if (mm_status s = build_group(g)) return s;
      double us;
      if (mm_status s = timed([&] {
            return mmk_launch_fft_yzx(g.py / 4, g.pz / 4, g.n_yz, g.lds_yz, b->d_desc, g.yz, g_twiddle, b->stream);
          }, &us))
        return s;
      yrep += (yrep.empty() ? "" : ", ") + std::string("\"xch\": ") + std::to_string(us);
      if (us < bestYZ) { bestYZ = us; bestPath = PATH_XCH; }
    }
    for (int TW = 1; TW <= 16 && splitx_fits(g.py); TW *= 2) {
      if (sizeof(float2) * ((size_t)g.pz * 3 * TW + g.pz) > lds_cap) continue;
      g.path = PATH_SPLITX;
      g.TW = TW;
      if (mm_status s = build_group(g)) return s;
      double us;
      if (mm_status s = timed([&] {
            hipError_t e = mmk_launch_fft_ysx(-1, g.py, g.n_y, g.lds_y, b->d_desc, g.y, g_twiddle, b->stream);
            if (e != hipSuccess) return e;
            e = mmk_launch_fft_zc(g.TW, g.n_zc, g.lds_zc, b->d_desc, g.zc, g_twiddle, b->stream);
            if (e != hipSuccess) return e;
            return mmk_launch_fft_ysx(1, g.py, g.n_y, g.lds_y, b->d_desc, g.y, g_twiddle, b->stream);
          }, &us))
        return s;
      yrep += (yrep.empty() ? "" : ", ") + std::string("\"splitx_") + std::to_string(TW) + "\": " + std::to_string(us);
      if (us < bestYZ) { bestYZ = us; bestPath = PATH_SPLITX; bestTW = TW; }
    }
    for (int Wy = 4; Wy <= 64; Wy *= 2) {
      if (sizeof(float2) * ((size_t)g.py * (Wy + 1) + g.py) > lds_cap) continue;
      for (int TW = 1; TW <= 16; TW *= 2) {
        if (sizeof(float2) * ((size_t)g.pz * 3 * TW + g.pz) > lds_cap) continue;
        g.path = PATH_SPLIT;
        g.Wy = Wy;
        g.TW = TW;
        if (mm_status s = build_group(g)) return s;
        double us;
        if (mm_status s = timed([&] {
              hipError_t e = mmk_launch_fft_y(-1, g.Wy, g.n_y, g.lds_y, b->d_desc, g.y, g_twiddle, b->stream);
              if (e != hipSuccess) return e;
              e = mmk_launch_fft_zc(g.TW, g.n_zc, g.lds_zc, b->d_desc, g.zc, g_twiddle, b->stream);
              if (e != hipSuccess) return e;
              return mmk_launch_fft_y(1, g.Wy, g.n_y, g.lds_y, b->d_desc, g.y, g_twiddle, b->stream);
            }, &us))
          return s;
        yrep += (yrep.empty() ? "" : ", ") + std::string("\"split_") + std::to_string(Wy) + "_" +
                std::to_string(TW) + "\": " + std::to_string(us);
        if (us < bestYZ) { bestYZ = us; bestPath = PATH_SPLIT; bestWy = Wy; bestTW = TW; }
      }
    }
    g.path = bestPath;
    g.Wy = bestWy;
    g.TW = bestTW;
    g.TK = bestTK;
    if (mm_status s = build_group(g)) return s;
    rep += (gi ? ", " : "") + std::string("{\"grid\": [") + std::to_string(g.nx) + ", " + std::to_string(g.ny) + ", " +
           std::to_string(g.nz) + "], \"instances\": " + std::to_string(g.members.size()) + ", \"Wx\": " +
           std::to_string(g.Wx) + ", \"x_stage\": " + std::string(g.xfused ? "true" : "false") + ", \"path\": \"" + path_name(g.path) + "\", \"Wy\": " +
           std::to_string(g.Wy) + ", \"TW\": " + std::to_string(g.TW) + ", \"TK\": " + std::to_string(g.TK) + ", \"x_us\": {" + xrep +
           "}, \"yz_us\": {" + yrep + "}}";
  }
  rep += "]";
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  // launch sequences changed: recapture on next use
  drop_graphs(b);
  MM_HIP(hipStreamSynchronize(b->stream));
  out = rep;
  return MM_OK;
}

mm_status mm_batch_destroy(mm_batch* b) {
  if (!b) return MM_OK;
  if (!b->ctxs.empty()) hipSetDevice(b->ctxs[0]->dev);
  for (mm_batch* p : b->parts) mm_batch_destroy(p);
  if (b->open) {
    hipStreamSynchronize(b->stream);
    for (mm_ctx* c : b->ctxs) c->open_in = nullptr;
  }
  drop_graphs(b);
  for (auto& g : b->groups) {
    if (g.xf) hipFree(g.xf);
    if (g.yz) hipFree(g.yz);
    if (g.y) hipFree(g.y);
    if (g.zc) hipFree(g.zc);
  }
  if (b->d_desc) hipFree(b->d_desc);
  if (b->d_wg) hipFree(b->d_wg);
  if (b->d_flags) hipFree(b->d_flags);
  if (b->h_flags) hipHostFree(b->h_flags);
  if (b->ev) hipEventDestroy(b->ev);
  if (b->stream) hipStreamDestroy(b->stream);
  delete b;
  return MM_OK;
}

}  // extern "C"
