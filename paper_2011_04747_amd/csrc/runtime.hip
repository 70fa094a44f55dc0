// libmono runtime: the C interface of include/mono.h.
//
// Owns the device buffers of a simulation, derives the time discretisation
// of the DAETI method (paper Sec. 2: Gershgorin step of eq. 3, diffusion
// substep count l, reaction cap k_max) and enqueues the split step
// B(dt/2) A(dt) B(dt/2) on the simulation's stream, replaying a cached HIP
// graph of a chunk of outer steps so that per-launch host overhead is paid
// once per chunk.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "checkpoint_plan.h"
#include "mono_internal.h"

using namespace mono;

namespace {

thread_local std::string t_err;

mono_status fail(mono_status s, const std::string& m) {
  t_err = m;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(MONO_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

// Device memory comes from hipMalloc or from the caller's allocator hook
// (mono_set_allocator), which may only change while no simulation exists.
struct DeviceAllocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free_)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
DeviceAllocator g_alloc;
std::atomic<int64_t> g_live_sims{0};

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  if (g_alloc.alloc) {
    void* q = g_alloc.alloc(count * sizeof(T), g_alloc.ctx);
    if (!q) return hipErrorOutOfMemory;
    *p = (T*)q;
    return hipSuccess;
  }
  return hipMalloc((void**)p, count * sizeof(T));
}

template <typename T>
void dfree(T*& p) {
  if (p) {
    if (g_alloc.free_)
      g_alloc.free_((void*)p, g_alloc.ctx);
    else
      (void)hipFree((void*)p);
  }
  p = nullptr;
}


// published initial values of the TP06 code release (not pre-paced)
const double kTP06Init[19] = {-86.2, 138.3, 7.67, 0.00007, 0.00007, 1.3, 1.0, 0.0, 0.75, 0.75,
                              0.0,   1.0,   0.0,  0.0,     1.0,     0.0, 1.0, 1.0, 1.0};
const double kMSParams[5] = {0.3, 6.0, 120.0, 150.0, 0.13};
// rows 6..8: cell type or node class, fibroblast membrane rate g_f [1/ms] and
// reversal potential E_f [mV]
const double kTP06Params[9] = {5.4, 1.0, 1.0, 1.0, 1.0, 1.0, 0.0, 0.0216, -49.6};

bool is_tp06(int m) {
  return m == MONO_MODEL_TP06_EPI || m == MONO_MODEL_TP06_TYPES || m == MONO_MODEL_TP06_FIBRO;
}
int model_states(int m) { return m == MONO_MODEL_LINEAR ? 1 : (m == MONO_MODEL_MS ? 2 : 19); }
int model_params(int m) {
  switch (m) {
    case MONO_MODEL_LINEAR: return 2;
    case MONO_MODEL_MS: return 5;
    case MONO_MODEL_TP06_EPI: return 6;
    case MONO_MODEL_TP06_TYPES: return 7;
    default: return 9;
  }
}
double default_lat_threshold(int m) {
  return is_tp06(m) ? -40.0 : (m == MONO_MODEL_MS ? 0.5 : 0.0);
}

}  // namespace

struct mono_sim {
  int prec = MONO_F64;
  size_t es = 8;               // bytes per state value
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int dim = 0;
  int64_t n = 0, Np = 0;
  int n_inst = 1;
  std::vector<int64_t> inst_off;
  int32_t* d_inst = nullptr;
  int64_t* d_inst_off = nullptr;
  // operator
  int layout = MONO_LAYOUT_ELL;
  int W = 0, P = 0;
  int32_t* d_col = nullptr;
  void* d_val = nullptr;
  void* d_e = nullptr;
  uint16_t* d_cls = nullptr;       // row classes of a single-instance stencil
  void* d_ctab = nullptr;
  int tw = 0, n_classes = 0;
  int row_pattern = 0;             // stencil offsets are grid row triples
  int grid_nx = 0, grid_nxy = 0;   // their y-row and z-plane offsets
  int grid_ny = 0, grid_nz = 0;    // a 3D grid's rows per plane and planes
  int fuse_ok = 0;                 // the grid admits the fused half-step diffusion
  int n_cu = 0;                    // compute units of the device
  int32_t* d_wcls = nullptr;       // per-wavefront class of the row-sharing diffusion
  void* d_minv = nullptr;
  int32_t* d_off = nullptr;
  int64_t nnz = 0;
  HostCSR K;
  std::vector<double> dt_s, gmax, lambda;
  // cell model
  int model = -1, S = 0, Pm = 0;
  void* d_V[2] = {nullptr, nullptr};
  void* d_st = nullptr;
  void* d_vprev = nullptr;
  double* d_lat = nullptr;
  double* d_apd = nullptr;         // APD90 trackers (5 rows of Np) or nullptr
  uint8_t* d_k = nullptr;
  void* d_par = nullptr;
  uint32_t par_pernode = 0;
  double par_uniform[kMaxParams] = {0};
  double lat_thr = 0.0;
  double dt0 = 0.01;
  StimTable stim{};
  uint8_t* d_mask = nullptr;
  // method and discretisation
  int method = MONO_DAETI, dvdt_src = 0, l_round = 0;
  double dt = -1.0;
  std::vector<int32_t> l;
  std::vector<double> dt_ad;
  int l_max = 1, k_max = 1;
  int32_t* d_l = nullptr;
  double* d_dtad = nullptr;
  int64_t step = 0;
  int64_t* d_base = nullptr;
  int* d_flag = nullptr;
  bool latched = false;
  // graph cache
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool g_valid = false;
  // the same chunk captured with the stimulus test switched off, replayed
  // for chunks in which no stimulus window can open (the diffusion kernels
  // then skip reading the device clock for the window test)
  hipGraph_t graph_q = nullptr;
  hipGraphExec_t gexec_q = nullptr;
  bool quiet = false;              // set while capturing graph_q
  // graph of a shorter run (the remainder of a step count that graph_steps
  // does not divide)
  hipGraph_t graph_r = nullptr;
  hipGraphExec_t gexec_r = nullptr;
  int64_t g_r_steps = 0;
  hipGraph_t graph_rq = nullptr;   // its capture without the stimulus test
  hipGraphExec_t gexec_rq = nullptr;
  LaunchCfg lc;
  // debug
  KTraceArgs kt{};
  int vclamp = 0, force_l = 0;
  unsigned long long* d_stats = nullptr;   // 4 counters, 16 apart
  bool stats_on = false;
  // per-kernel timing of MONO_STEP_TIMED calls: [0] diffusion, [1] reaction
  std::vector<hipEvent_t> ev_pool;
  double ktime_ms[2] = {0.0, 0.0};
  int64_t klaunches[2] = {0, 0};
  // adjoint: conductivity scales, loss sensors, checkpoints and segment tape
  void* d_sigma = nullptr;         // Np, simulation precision
  int sigma_uniform = 0;           // every node has sigma_value (in precision T)
  double sigma_value = 1.0;
  int32_t* d_sens = nullptr;
  int32_t* d_sens_of = nullptr;    // per node: sensor index or -1
  int ns = 0;
  double* d_target = nullptr;      // target_steps x ns
  int64_t target_steps = 0;
  bool taped = false;
  int64_t tape_step0 = 0, tape_steps = 0;
  int ckpt_every = 0;
  // checkpoint schedule of the next taped run: uniform (a snapshot at every
  // segment start) or binomial within ckpt_max_slots snapshot buffers
  int ckpt_schedule = MONO_CKPT_UNIFORM, ckpt_max_slots = 0;
  CkptPlan plan;                   // the binomial plan of the taped run
  int64_t ckpt_advances = 0;       // segment advances of the last reverse sweep
  // parameter scalings of mono_set_param_scalings since the last cell model
  int scal_n = -1;                 // -1: none set
  int scal_rows[kMaxParams] = {};
  double scal_vals[kMaxParams] = {};
  std::vector<void*> d_ckpt;       // state snapshots (segment starts)
  void* d_final = nullptr;         // state after the taped run
  void* d_seg_vsub = nullptr;      // ckpt_every x 2 l_max x Np
  void* d_seg_entry = nullptr;     // ckpt_every x S x Np
  uint8_t* d_seg_k = nullptr;      // ckpt_every x n
  // a second segment tape (the uniform schedule recomputes one segment while
  // the one after it is reversed) and the reverse sweep's own device clock
  void* d_seg_vsub2 = nullptr;
  void* d_seg_entry2 = nullptr;
  uint8_t* d_seg_k2 = nullptr;
  int64_t* d_base_rev = nullptr;
  hipStream_t stream_aux = nullptr;  // library-created, for the recomputes
  void* d_lam = nullptr;           // S x Np adjoint of the state
  void* d_lamV2 = nullptr;         // Np, ping-pong partner of the V adjoint
  double* d_gsig = nullptr;        // Np
  double* d_gpart = nullptr;       // workgroups x kMaxParams
  double* d_loss_steps = nullptr;  // tape_steps
};

namespace {

void drop_graph(mono_sim* s) {
  if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  s->gexec = nullptr;
  s->graph = nullptr;
  s->g_valid = false;
  if (s->gexec_q) (void)hipGraphExecDestroy(s->gexec_q);
  if (s->graph_q) (void)hipGraphDestroy(s->graph_q);
  s->gexec_q = nullptr;
  s->graph_q = nullptr;
  if (s->gexec_r) (void)hipGraphExecDestroy(s->gexec_r);
  if (s->graph_r) (void)hipGraphDestroy(s->graph_r);
  s->gexec_r = nullptr;
  s->graph_r = nullptr;
  s->g_r_steps = 0;
  if (s->gexec_rq) (void)hipGraphExecDestroy(s->gexec_rq);
  if (s->graph_rq) (void)hipGraphDestroy(s->graph_rq);
  s->gexec_rq = nullptr;
  s->graph_rq = nullptr;
}

// upload n_host doubles into a device array of the simulation's precision
// Offsets of a structured grid numbered x fastest: 1 (line); 1, nx-1, nx, nx+1
// (quads); and in 3D the nine x-triples around 0, nx, nxy-nx, nxy, nxy+nx.
bool grid_row_pattern(const std::vector<int32_t>& off) {
  const size_t P = off.size();
  if (P == 1) return off[0] == 1;
  if (P == 4) {
    const int nx = off[2];
    return nx > 2 && off[0] == 1 && off[1] == nx - 1 && off[3] == nx + 1;
  }
  if (P == 13) {
    const int64_t nx = off[2], nxy = off[8];
    const int64_t want[13] = {1,           nx - 1,       nx,       nx + 1,  nxy - nx - 1,
                              nxy - nx,    nxy - nx + 1, nxy - 1,  nxy,     nxy + 1,
                              nxy + nx - 1, nxy + nx,    nxy + nx + 1};
    for (int p = 0; p < 13; ++p)
      if (off[p] != want[p] || (p > 0 && want[p] <= want[p - 1])) return false;
    return true;
  }
  return false;
}

// Whether a single-instance 13-offset grid stencil can take the fused
// half-step diffusion: the n rows are a whole nx x ny x nz grid (32-bit byte
// offsets), and no nonzero weight joins a node to a position outside the grid
// (past a row end, a face): the fused kernel holds 0 there.
bool fused_grid_ok(const StencilHost& sh, int64_t n, int64_t Np, size_t es, int64_t nx,
                   int64_t nxy) {
  if (sh.P != 13 || (int64_t)sh.off.size() != 13 || nx < 1 || nxy < nx || nxy % nx ||
      n % nxy || n * (int64_t)es >= ((int64_t)1 << 31))
    return false;
  const int64_t ny = nxy / nx, nz = n / nxy;
  // grid step of each forward offset (the order of the 13-offset pattern)
  static const int d[13][3] = {{1, 0, 0},  {-1, 1, 0},  {0, 1, 0},  {1, 1, 0},  {-1, -1, 1},
                               {0, -1, 1}, {1, -1, 1},  {-1, 0, 1}, {0, 0, 1},  {1, 0, 1},
                               {-1, 1, 1}, {0, 1, 1},   {1, 1, 1}};
  for (int64_t i = 0; i < n; ++i) {
    const int64_t x = i % nx, y = (i / nx) % ny, z = i / nxy;
    for (int p = 0; p < 13; ++p) {
      const int64_t xj = x + d[p][0], yj = y + d[p][1], zj = z + d[p][2];
      const bool inside = xj >= 0 && xj < nx && yj >= 0 && yj < ny && zj >= 0 && zj < nz;
      if (!inside && sh.e[(size_t)p * Np + i] != 0.0) return false;
    }
  }
  return true;
}

mono_status upload_real(mono_sim* s, void* dst, const double* src, size_t count) {
  if (count == 0) return MONO_OK;
  if (s->prec == MONO_F64) {
    HIP_TRY(hipMemcpy(dst, src, count * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> tmp(count);
    for (size_t i = 0; i < count; ++i) tmp[i] = (float)src[i];
    HIP_TRY(hipMemcpy(dst, tmp.data(), count * 4, hipMemcpyHostToDevice));
  }
  return MONO_OK;
}

mono_status download_real(mono_sim* s, double* dst, const void* src, size_t count) {
  if (count == 0) return MONO_OK;
  if (s->prec == MONO_F64) {
    HIP_TRY(hipMemcpyAsync(dst, src, count * 8, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  } else {
    std::vector<float> tmp(count);
    HIP_TRY(hipMemcpyAsync(tmp.data(), src, count * 4, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (size_t i = 0; i < count; ++i) dst[i] = tmp[i];
  }
  return MONO_OK;
}

mono_status check_flag(mono_sim* s) {
  int f = 0;
  HIP_TRY(hipMemcpyAsync(&f, s->d_flag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (f) {
    s->latched = true;
    return fail(MONO_ENONFINITE, "non-finite membrane potential during stepping");
  }
  return MONO_OK;
}

// Time discretisation for outer step dt (Sec. 2).
mono_status prepare(mono_sim* s, double dt) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(MONO_EINVAL, "dt must be positive");
  std::vector<int32_t> l(s->n_inst);
  std::vector<double> dad(s->n_inst);
  for (int q = 0; q < s->n_inst; ++q) {
    int lq = 1;
    if (0.5 * dt > s->dt_s[q]) {
      const double x = dt / (2.0 * s->dt_s[q]);
      const double r = s->l_round ? std::ceil(x) : std::floor(x);
      lq = r < 1.0 ? 1 : (int)r;
    }
    if (s->method != MONO_DAETI) lq = 1;
    if (s->force_l > 0) lq = s->force_l;
    l[q] = lq;
    dad[q] = dt / (2.0 * lq);
  }
  double km = std::floor(dt / s->dt0);
  int kmax = km < 1.0 ? 1 : (km > 255.0 ? 255 : (int)km);
  if (s->method == MONO_OST) kmax = 1;
  const bool changed = (l != s->l) || (dad != s->dt_ad) || kmax != s->k_max || dt != s->dt;
  if (changed) {
    // kernels already enqueued may still read the per-instance tables
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->l = l;
    s->dt_ad = dad;
    s->k_max = kmax;
    s->dt = dt;
    s->l_max = *std::max_element(l.begin(), l.end());
    HIP_TRY(hipMemcpy(s->d_l, l.data(), l.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->d_dtad, dad.data(), dad.size() * sizeof(double), hipMemcpyHostToDevice));
    drop_graph(s);
  }
  return MONO_OK;
}

// Start time of substep q = (2 step + half) L + m, with the rounding of the
// diffusion kernels' substep clock.
double substep_start(int64_t q, double dt, int L, double dt_ad) {
  const int64_t step = q / (2 * (int64_t)L), r = q % (2 * (int64_t)L);
  double t0 = rn_mul((double)step, dt);
  if (r >= L) t0 = rn_add(t0, rn_mul(0.5, dt));
  return rn_add(t0, rn_mul((double)(r % L), dt_ad));
}
// First substep whose start time is at or after t (start times increase
// with q: within a half step by m dt_ad, across halves and steps by at least
// dt_ad, far above their rounding)
int64_t first_substep_from(double t, double dt, int L, double dt_ad) {
  if (!(t > 0.0)) return 0;
  const double qf = t / dt * 2.0 * L + 4.0;
  if (!(qf < 4.0e18)) return INT64_MAX;
  int64_t lo = 0, hi = (int64_t)qf;          // tau(lo) < t <= tau(hi)
  if (substep_start(hi, dt, L, dt_ad) < t) return INT64_MAX;
  while (hi - lo > 1) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (substep_start(mid, dt, L, dt_ad) >= t)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

template <typename T>
DiffArgs<T> diff_args(mono_sim* s, int pass_in, int half, int m, int64_t g) {
  DiffArgs<T> a{};
  a.n = s->n;
  a.Np = s->Np;
  a.Vin = (const T*)s->d_V[pass_in & 1];
  a.Vout = (T*)s->d_V[(pass_in + 1) & 1];
  a.W = s->W;
  a.col = s->d_col;
  a.val = (const T*)s->d_val;
  a.P = s->P;
  a.cls = s->d_cls;
  a.ctab = (const T*)s->d_ctab;
  a.tw = s->tw;
  a.wcls = s->d_wcls;
  a.nx = s->grid_nx;
  a.nxy = s->grid_nxy;
  a.e = (const T*)s->d_e;
  a.minv = (const T*)s->d_minv;
  a.off = s->d_off;
  a.inst = s->n_inst > 1 ? s->d_inst : nullptr;
  a.inst_off = s->d_inst_off;
  a.l = s->d_l;
  a.dt_ad = s->d_dtad;
  a.stim_mask = s->quiet ? nullptr : s->d_mask;
  a.stim = s->stim;
  a.stim.L = 0;
  if (s->n_inst == 1 && !s->l.empty() && s->l[0] > 0) {
    a.stim.L = s->l[0];
    for (int q = 0; q < a.stim.n; ++q) {
      a.stim.q_on[q] = first_substep_from(a.stim.t_on[q], s->dt, s->l[0], s->dt_ad[0]);
      a.stim.q_end[q] = first_substep_from(a.stim.t_end[q], s->dt, s->l[0], s->dt_ad[0]);
    }
  }
  a.clk.base = s->d_base;
  a.clk.g = g;
  a.clk.dt = s->dt;
  a.half = half;
  a.m = m;
  a.xcd = s->lc.diff_xcd;
  return a;
}

template <typename T>
IonArgs<T> ion_args(mono_sim* s, void* V, int64_t g) {
  IonArgs<T> a{};
  a.n = s->n;
  a.Np = s->Np;
  a.V = (T*)V;
  a.st = (T*)s->d_st;
  a.vprev = (T*)s->d_vprev;
  a.lat = s->d_lat;
  a.lastk = s->d_k;
  a.par = (const T*)s->d_par;
  for (int q = 0; q < kMaxParams; ++q) a.par_uniform[q] = (T)s->par_uniform[q];
  a.par_pernode = s->par_pernode;
  a.clk.base = s->d_base;
  a.clk.g = g;
  a.clk.dt = s->dt;
  a.k_max = s->k_max;
  a.lat_thr = s->lat_thr;
  a.dvdt_src = s->dvdt_src;
  a.vclamp = s->vclamp;
  a.kt = s->kt;
  a.flag = s->d_flag;
  a.stats = s->stats_on ? s->d_stats : nullptr;
  a.apd = s->d_apd;
  // the largest row offset of the state and parameter arrays (plus a
  // workgroup's span) must fit a 32-bit byte offset
  const int64_t rows = std::max<int64_t>(s->S - 1, kMaxParams);
  a.off32 = (rows * s->Np + 1024) * (int64_t)sizeof(T) < ((int64_t)1 << 32) ? 1 : 0;
  return a;
}

// Whether the half steps run fused: a grid that takes it, row classes in
// use, one instance and at least two substeps per half step.
bool use_fused(const mono_sim* s) {
  return s->fuse_ok && s->lc.diff_fuse && s->lc.diff_classes && s->d_cls && s->n_inst == 1 &&
         s->l_max >= 2;
}

// Diffusion launches per half step: ceil(l / 4) fused launches, else l.
int diff_launches_per_half(const mono_sim* s) {
  return use_fused(s) ? (s->l_max + 3) / 4 : s->l_max;
}

// Tiling of a fused launch of L substeps: 64 - 2L x per workgroup, 16 - 2L y
// rows, and z planes as set, else the split of z that minimises the planes
// each compute unit marches (workgroups per compute unit, rounded up, times
// the planes of one tile with its 2L halo planes).
FusedGeom fused_geom(const mono_sim* s, int L) {
  FusedGeom g{};
  g.nx = s->grid_nx;
  g.ny = s->grid_ny;
  g.nz = s->grid_nz;
  g.ty = kFusedRows - 2 * L;
  g.nxs = (g.nx + 63 - 2 * L) / (64 - 2 * L);
  g.nys = (g.ny + g.ty - 1) / g.ty;
  int tz = s->lc.diff_fuse_planes;
  if (tz <= 0) {
    const int64_t xy = (int64_t)g.nxs * g.nys;
    int64_t best = INT64_MAX;
    for (int nzs = 1; nzs <= g.nz; ++nzs) {
      const int t = (g.nz + nzs - 1) / nzs;
      const int64_t blocks = xy * ((g.nz + t - 1) / t);
      const int64_t cost = (blocks + s->n_cu - 1) / s->n_cu * (t + 2 * L);
      if (cost < best) {
        best = cost;
        tz = t;
      }
    }
  }
  g.tz = std::min(tz, g.nz);
  g.nzs = (g.nz + g.tz - 1) / g.tz;
  return g;
}

// One half step's diffusion (half 0 or 1) at clock offset g, reading the
// potential buffer d_V[cur] and leaving cur at the buffer that holds the
// result; mark(0) is called before each launch (kernel timing).
template <typename T, typename Mark>
void enqueue_half(mono_sim* s, int half, int64_t g, int& cur, Mark&& mark) {
  const int L = s->l_max;
  if (use_fused(s)) {
    const int nch = (L + 3) / 4;
    int m = 0;
    for (int c = 0; c < nch; ++c) {
      const int len = (L - m) / (nch - c);
      mark(0);
      launch_diffusion_fused<T>(diff_args<T>(s, cur, half, m, g), len, fused_geom(s, len),
                                s->stream);
      cur ^= 1;
      m += len;
    }
    return;
  }
  for (int m = 0; m < L; ++m) {
    mark(0);
    launch_diffusion<T>(s->layout, diff_args<T>(s, cur, half, m, g), s->lc, s->stream);
    cur ^= 1;
  }
}

// Enqueue `count` outer steps with clock offsets 0..count-1 and advance the
// device clock by count.  With `ev` non-null every step kernel is launched
// with a start/stop event pair (appended as {start, stop, class}).
struct TimedPair {
  hipEvent_t a, b;
  int cls;
};

}  // namespace

thread_local KernelTimer* mono::g_ktimer = nullptr;

namespace {

template <typename T>
void enqueue_steps(mono_sim* s, int64_t count, std::vector<TimedPair>* ev) {
  size_t next = 0;
  KernelTimer kt{};
  auto mark = [&](int cls) {
    if (!ev) return;
    TimedPair p{s->ev_pool[next], s->ev_pool[next + 1], cls};
    next += 2;
    ev->push_back(p);
    kt = KernelTimer{p.a, p.b};
    g_ktimer = &kt;
  };
  for (int64_t g = 0; g < count; ++g) {
    // the step starts in d_V[0] and, after 2 l substeps or twice the same
    // number of fused launches, ends there again
    int cur = 0;
    enqueue_half<T>(s, 0, g, cur, mark);
    mark(1);
    launch_ionic<T>(s->model, ion_args<T>(s, s->d_V[cur], g), s->lc, s->stream);
    enqueue_half<T>(s, 1, g, cur, mark);
  }
  g_ktimer = nullptr;
  launch_advance_clock(s->d_base, count, s->stream);
}

void enqueue(mono_sim* s, int64_t count, std::vector<TimedPair>* ev = nullptr) {
  if (s->prec == MONO_F64)
    enqueue_steps<double>(s, count, ev);
  else
    enqueue_steps<float>(s, count, ev);
}

// Eager steps with every step kernel timed by its own start/stop events
// (synchronising); adds to the per-class totals.
mono_status enqueue_timed(mono_sim* s, int64_t count) {
  const int64_t per_step = 2 * s->l_max + 1;
  const int64_t chunk = 64;
  for (int64_t done = 0; done < count;) {
    const int64_t c = std::min(chunk, count - done);
    const size_t need = (size_t)(2 * per_step * c);
    while (s->ev_pool.size() < need) {
      // timing-only events: no system-scope fence (cache writeback and
      // invalidation) around the kernels they time; the stream is synchronised
      // before they are read
      hipEvent_t e;
      HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      s->ev_pool.push_back(e);
    }
    std::vector<TimedPair> ev;
    ev.reserve(per_step * c);
    // the device clock of this chunk starts at the current time level
    enqueue(s, c, &ev);
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (const TimedPair& p : ev) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, p.a, p.b));
      s->ktime_ms[p.cls] += ms;
      s->klaunches[p.cls] += 1;
    }
    done += c;
  }
  return MONO_OK;
}

// R diffusion substeps alternating between the potential buffers, captured
// in one graph and timed by events around its launch (after one untimed
// launch).  Unfused: R launches of the first substep of the first half step
// (clock offset 0).  Fused: R / l first half steps (at least one), launched
// as stepping launches them; the mean is taken over the substeps they run.
mono_status time_diffusion(mono_sim* s, int64_t R, double& ms_per) {
  HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
  auto none = [](int) {};
  int64_t substeps = R;
  if (use_fused(s)) {
    // an even number of launches, so that the potential ends in d_V[0]
    int64_t H = std::max<int64_t>(1, R / s->l_max);
    if ((H * diff_launches_per_half(s)) & 1) ++H;
    substeps = H * s->l_max;
    int cur = 0;
    for (int64_t h = 0; h < H; ++h) {
      if (s->prec == MONO_F64)
        enqueue_half<double>(s, 0, 0, cur, none);
      else
        enqueue_half<float>(s, 0, 0, cur, none);
    }
  } else {
    for (int64_t r = 0; r < R; ++r) {
      if (s->prec == MONO_F64)
        launch_diffusion<double>(s->layout, diff_args<double>(s, (int)(r & 1), 0, 0, 0), s->lc,
                                 s->stream);
      else
        launch_diffusion<float>(s->layout, diff_args<float>(s, (int)(r & 1), 0, 0, 0), s->lc,
                                s->stream);
    }
  }
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamEndCapture(s->stream, &g));
  hipGraphExec_t ge = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  mono_status st = MONO_OK;
  float ms = 0.f;
  if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      hipGraphLaunch(ge, s->stream) != hipSuccess ||
      hipEventRecord(e0, s->stream) != hipSuccess || hipGraphLaunch(ge, s->stream) != hipSuccess ||
      hipEventRecord(e1, s->stream) != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess ||
      hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
    st = fail(MONO_EDEVICE, "diffusion timing failed");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (ge) (void)hipGraphExecDestroy(ge);
  (void)hipGraphDestroy(g);
  ms_per = (double)ms / (double)substeps;
  return st;
}

mono_status ensure_graph(mono_sim* s) {
  if (s->g_valid) return MONO_OK;
  drop_graph(s);
  HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
  enqueue(s, s->lc.graph_steps);
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamEndCapture(s->stream, &g));
  s->graph = g;
  HIP_TRY(hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0));
  if (s->stim.n > 0) {
    s->quiet = true;
    hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      enqueue(s, s->lc.graph_steps);
      e = hipStreamEndCapture(s->stream, &g);
    }
    s->quiet = false;
    HIP_TRY(e);
    s->graph_q = g;
    HIP_TRY(hipGraphInstantiate(&s->gexec_q, s->graph_q, nullptr, nullptr, 0));
  }
  s->g_valid = true;
  return MONO_OK;
}

// True when no stimulus can be open on any diffusion substep of the outer
// steps [step0, step0 + count): single instance, by the integer substep
// windows the kernels test; several instances (per-instance substep
// lengths), by time with a margin of one outer step on either side.
bool chunk_is_quiet(const mono_sim* s, int64_t step0, int64_t count) {
  if (s->n_inst == 1 && !s->l.empty() && s->l[0] > 0) {
    const int L = s->l[0];
    const int64_t lo = 2 * step0 * (int64_t)L, hi = 2 * (step0 + count) * (int64_t)L;
    for (int q = 0; q < s->stim.n; ++q) {
      const int64_t on = first_substep_from(s->stim.t_on[q], s->dt, L, s->dt_ad[0]);
      const int64_t end = first_substep_from(s->stim.t_end[q], s->dt, L, s->dt_ad[0]);
      if (on < end && on < hi && end > lo) return false;
    }
    return true;
  }
  const double t0 = (double)(step0 - 1) * s->dt, t1 = (double)(step0 + count + 1) * s->dt;
  for (int q = 0; q < s->stim.n; ++q)
    if (s->stim.t_on[q] < t1 && s->stim.t_end[q] > t0) return false;
  return true;
}

// Graph of `steps` outer steps for the remainder of a run (cached while the
// remainder length repeats).
mono_status ensure_rem_graph(mono_sim* s, int64_t steps) {
  if (s->g_r_steps == steps && s->gexec_r) return MONO_OK;
  if (s->gexec_r) (void)hipGraphExecDestroy(s->gexec_r);
  if (s->graph_r) (void)hipGraphDestroy(s->graph_r);
  if (s->gexec_rq) (void)hipGraphExecDestroy(s->gexec_rq);
  if (s->graph_rq) (void)hipGraphDestroy(s->graph_rq);
  s->gexec_r = nullptr;
  s->graph_r = nullptr;
  s->gexec_rq = nullptr;
  s->graph_rq = nullptr;
  s->g_r_steps = 0;
  HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
  enqueue(s, steps);
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamEndCapture(s->stream, &g));
  s->graph_r = g;
  HIP_TRY(hipGraphInstantiate(&s->gexec_r, s->graph_r, nullptr, nullptr, 0));
  if (s->stim.n > 0) {
    s->quiet = true;
    hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      enqueue(s, steps);
      e = hipStreamEndCapture(s->stream, &g);
    }
    s->quiet = false;
    HIP_TRY(e);
    s->graph_rq = g;
    HIP_TRY(hipGraphInstantiate(&s->gexec_rq, s->graph_rq, nullptr, nullptr, 0));
  }
  s->g_r_steps = steps;
  return MONO_OK;
}

mono_status require_model(mono_sim* s) {
  if (!s) return fail(MONO_EINVAL, "NULL simulation");
  if (s->model < 0) return fail(MONO_ESTATE, "no cell model set");
  return MONO_OK;
}

void* field_ptr(mono_sim* s, int field, size_t& es) {
  es = s->es;
  if (field == MONO_FIELD_V || field == MONO_FIELD_STATE0) return s->d_V[0];
  if (field == MONO_FIELD_VPREV) return s->d_vprev;
  if (field == MONO_FIELD_LAT) {
    es = 8;
    return s->d_lat;
  }
  if (field == MONO_FIELD_K) {
    es = 1;
    return s->d_k;
  }
  if (field > MONO_FIELD_STATE0 && field < MONO_FIELD_STATE0 + s->S)
    return (char*)s->d_st + (size_t)(field - MONO_FIELD_STATE0 - 1) * s->Np * s->es;
  return nullptr;
}

void free_model(mono_sim* s) {
  dfree(s->d_V[0]);
  dfree(s->d_V[1]);
  dfree(s->d_st);
  dfree(s->d_vprev);
  dfree(s->d_lat);
  dfree(s->d_apd);
  dfree(s->d_k);
  dfree(s->d_par);
}

void free_tape(mono_sim* s) {
  for (void*& p : s->d_ckpt) dfree(p);
  s->d_ckpt.clear();
  dfree(s->d_final);
  dfree(s->d_seg_vsub);
  dfree(s->d_seg_entry);
  dfree(s->d_seg_k);
  dfree(s->d_seg_vsub2);
  dfree(s->d_seg_entry2);
  dfree(s->d_seg_k2);
  dfree(s->d_base_rev);
  dfree(s->d_lam);
  dfree(s->d_lamV2);
  dfree(s->d_gsig);
  dfree(s->d_gpart);
  dfree(s->d_loss_steps);
  s->taped = false;
}

// snapshot layout: V, the other S-1 states, V_prev (all Np, precision T),
// then the activation times (Np doubles)
size_t snapshot_bytes(const mono_sim* s) { return (size_t)(s->S + 1) * s->Np * s->es + s->Np * 8; }

hipError_t save_state(mono_sim* s, void* dst) {
  const size_t b = s->Np * s->es;
  char* d = (char*)dst;
  hipError_t e = hipMemcpyAsync(d, s->d_V[0], b, hipMemcpyDeviceToDevice, s->stream);
  if (!e && s->S > 1)
    e = hipMemcpyAsync(d + b, s->d_st, (size_t)(s->S - 1) * b, hipMemcpyDeviceToDevice, s->stream);
  if (!e) e = hipMemcpyAsync(d + (size_t)s->S * b, s->d_vprev, b, hipMemcpyDeviceToDevice, s->stream);
  if (!e)
    e = hipMemcpyAsync(d + (size_t)(s->S + 1) * b, s->d_lat, s->Np * 8, hipMemcpyDeviceToDevice,
                       s->stream);
  return e;
}

// V goes to Vdst (default: the simulation's potential)
hipError_t load_state(mono_sim* s, const void* src, void* Vdst = nullptr) {
  const size_t b = s->Np * s->es;
  const char* d = (const char*)src;
  hipError_t e = hipMemcpyAsync(Vdst ? Vdst : s->d_V[0], d, b, hipMemcpyDeviceToDevice, s->stream);
  if (!e && s->S > 1)
    e = hipMemcpyAsync(s->d_st, d + b, (size_t)(s->S - 1) * b, hipMemcpyDeviceToDevice, s->stream);
  if (!e) e = hipMemcpyAsync(s->d_vprev, d + (size_t)s->S * b, b, hipMemcpyDeviceToDevice, s->stream);
  if (!e)
    e = hipMemcpyAsync(s->d_lat, d + (size_t)(s->S + 1) * b, s->Np * 8, hipMemcpyDeviceToDevice,
                       s->stream);
  return e;
}

// Sensor arguments for clock offset g: targets by device step, losses to
// d_loss_steps[step - tape_step0].
SensorArgs sensor_args(mono_sim* s, int64_t g) {
  SensorArgs a{};
  a.sens = s->d_sens;
  a.ns = s->ns;
  a.target = s->d_target;
  a.target_steps = s->target_steps;
  a.clk.base = s->d_base;
  a.clk.g = g;
  a.clk.dt = s->dt;
  a.out = s->d_loss_steps;
  a.out_base = s->tape_step0;
  return a;
}

// One outer step with clock offset g that also stores the loss at reaction
// entry (loss) and/or samples the sensors there (sample).  recompute: a
// repeat of a step already taken (checkpoint advances of the reverse sweep),
// which leaves the APD trackers and the k statistics alone.
template <typename T>
void enqueue_loss_step(mono_sim* s, int64_t g, bool loss, double* sample = nullptr,
                       bool recompute = false) {
  const int L = s->l_max;
  for (int m = 0; m < L; ++m)
    launch_diffusion<T>(s->layout, diff_args<T>(s, m, 0, m, g), s->lc, s->stream);
  T* Vmid = (T*)s->d_V[L & 1];
  if (loss && s->ns > 0) launch_sensor_loss<T>(Vmid, sensor_args(s, g), s->stream);
  if (sample) launch_sensor_sample<T>(Vmid, s->d_sens, s->ns, sample, s->stream);
  IonArgs<T> ia = ion_args<T>(s, Vmid, g);
  if (recompute) {
    ia.apd = nullptr;
    ia.stats = nullptr;
  }
  launch_ionic<T>(s->model, ia, s->lc, s->stream);
  for (int m = 0; m < L; ++m)
    launch_diffusion<T>(s->layout, diff_args<T>(s, L + m, 1, m, g), s->lc, s->stream);
}

// One outer step of a segment recompute writing what the reverse sweep needs
// straight into the segment tape: vs holds the inputs of the 2 l_max diffusion
// substeps (vs[0], the step's starting potential, is already there; every
// substep writes the next slot), entry the reaction-entry state (its V row
// written by the last first-half substep, the other rows by the reaction
// kernel as it loads them), krec the substep counts (row g); the last
// substep writes vnext.
template <typename T>
void enqueue_tape_step(mono_sim* s, int64_t g, T* vs, T* entry, uint8_t* krec, int64_t krec_steps,
                       T* vnext) {
  const int L = s->l_max;
  const size_t Np = s->Np;
  for (int m = 0; m < L; ++m) {
    DiffArgs<T> a = diff_args<T>(s, m, 0, m, g);
    a.Vin = vs + (size_t)m * Np;
    a.Vout = (m + 1 < L) ? vs + (size_t)(m + 1) * Np : entry;
    launch_diffusion<T>(s->layout, a, s->lc, s->stream);
  }
  IonArgs<T> ia = ion_args<T>(s, entry, g);
  ia.apd = nullptr;   // segment recomputes replay earlier steps
  ia.Vout = vs + (size_t)L * Np;
  ia.tape_st = entry + Np;
  ia.kt.mode |= 1;
  ia.kt.rec = krec;
  ia.kt.rec_rel = 1;
  ia.kt.rec_steps = krec_steps;
  launch_ionic<T>(s->model, ia, s->lc, s->stream);
  for (int m = 0; m < L; ++m) {
    DiffArgs<T> a = diff_args<T>(s, L + m, 1, m, g);
    a.Vin = vs + (size_t)(L + m) * Np;
    a.Vout = (m + 1 < L) ? vs + (size_t)(L + m + 1) * Np : vnext;
    launch_diffusion<T>(s->layout, a, s->lc, s->stream);
  }
}

template <typename T>
AdjDiffArgs<T> adj_diff_args(mono_sim* s, const T* lam_in, T* lam_out, const T* V, int m) {
  AdjDiffArgs<T> a{};
  a.n = s->n;
  a.Np = s->Np;
  a.lam_in = lam_in;
  a.lam_out = lam_out;
  a.V = V;
  a.minv = (const T*)s->d_minv;
  a.sigma = (const T*)s->d_sigma;
  a.W = s->W;
  a.col = s->d_col;
  a.val = (const T*)s->d_val;
  a.P = s->P;
  a.e = (const T*)s->d_e;
  a.off = s->d_off;
  a.inst = s->n_inst > 1 ? s->d_inst : nullptr;
  a.inst_off = s->d_inst_off;
  a.l = s->d_l;
  a.dt_ad = s->d_dtad;
  a.m = m;
  a.gsig = s->d_gsig;
  if (s->d_wcls && s->lc.diff_classes && s->lc.diff_wave_rows) {
    a.cls = s->d_cls;
    a.ctab = (const T*)s->d_ctab;
    a.tw = s->tw;
    a.wcls = s->d_wcls;
    a.nx = s->grid_nx;
    a.nxy = s->grid_nxy;
    a.iter = s->lc.diff_rpl >= 2 ? 2 : 1;
    a.sig_uni = s->sigma_uniform;
    a.sig_val = (T)s->sigma_value;
  }
  return a;
}

// Capture the work `body` enqueues on the simulation's stream as a graph.
template <class F>
mono_status capture_graph(mono_sim* s, F body, hipGraphExec_t* out) {
  HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
  body();
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamEndCapture(s->stream, &g));
  const hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(MONO_EDEVICE, "graph instantiation failed");
  return MONO_OK;
}

// Segment graphs of full and remainder length, each also captured with the
// stimulus mask switched off (the *q members, when the simulation has
// stimuli) for segments in which no stimulus window can open.
struct GraphPair {
  hipGraphExec_t full = nullptr, rest = nullptr, fullq = nullptr, restq = nullptr;
  ~GraphPair() {
    for (hipGraphExec_t g : {full, rest, fullq, restq})
      if (g) (void)hipGraphExecDestroy(g);
  }
  // With step0 >= 0 (the run's first step) only the variants that the run's
  // segments will pick are captured (of the segments whose index is
  // seg_rem modulo seg_mod); otherwise all of them.
  template <class MK>
  mono_status capture(mono_sim* s, MK make, int64_t n_steps, int64_t C, bool stimuli = true,
                      int64_t step0 = -1, int seg_mod = 1, int seg_rem = 0) {
    const int64_t rest_n = n_steps % C;
    const bool variants = stimuli && s->stim.n > 0;
    bool need[2][2] = {{n_steps >= C, rest_n > 0}, {variants && n_steps >= C, variants && rest_n > 0}};
    if (step0 >= 0) {
      need[0][0] = need[0][1] = need[1][0] = need[1][1] = false;
      for (int64_t t0 = 0; t0 < n_steps; t0 += C) {
        if ((t0 / C) % seg_mod != seg_rem) continue;
        const int64_t cn = std::min(C, n_steps - t0);
        const bool q = variants && chunk_is_quiet(s, step0 + t0, cn);
        need[q ? 1 : 0][cn == C ? 0 : 1] = true;
      }
    }
    mono_status st = MONO_OK;
    for (int quiet = 0; quiet < 2 && st == MONO_OK; ++quiet) {
      s->quiet = quiet != 0;
      if (need[quiet][0]) st = capture_graph(s, make(C), quiet ? &fullq : &full);
      if (st == MONO_OK && need[quiet][1])
        st = capture_graph(s, make(rest_n), quiet ? &restq : &rest);
    }
    s->quiet = false;
    return st;
  }
  hipGraphExec_t pick(const mono_sim* s, int64_t step0, int64_t cn, int64_t C) const {
    const bool q = (cn == C ? fullq : restq) && chunk_is_quiet(s, step0, cn);
    if (cn == C) return q ? fullq : full;
    return q ? restq : rest;
  }
};

// Taped forward run: the state at every segment start goes to a checkpoint,
// then the segment's steps (with the loss at each reaction entry) replay as
// one graph; the clock advances on the device.
template <typename T>
mono_status forward_taped_t(mono_sim* s, int64_t n_steps, double* loss) {
  const int64_t C = s->ckpt_every;
  const int64_t nck = (n_steps + C - 1) / C;
  GraphPair gp;
  auto segment = [s](int64_t cn) {
    return [s, cn]() {
      for (int64_t t = 0; t < cn; ++t) enqueue_loss_step<T>(s, t, true);
      launch_advance_clock(s->d_base, cn, s->stream);
    };
  };
  mono_status st = gp.capture(s, segment, n_steps, C, true, s->step);
  if (st != MONO_OK) return st;
  // snapshot buffer of each segment start (-1: not stored): every start in
  // the uniform schedule; the binomial plan's first splits otherwise
  std::vector<int> slot_at(nck, -1);
  if (s->ckpt_schedule == MONO_CKPT_UNIFORM) {
    for (int64_t c = 0; c < nck; ++c) slot_at[c] = (int)c;
  } else {
    const CkptPlan& p = s->plan;
    int64_t first = 0, k = nck;
    int f = p.width - 1, slot = 0;
    slot_at[0] = 0;
    while (k > 1) {
      const int64_t m = p.splitA[p.idx(k, f)];
      if (m == 0) break;
      first += m;
      k -= m;
      --f;
      slot_at[first] = ++slot;
    }
  }
  for (int64_t c = 0; c < nck; ++c) {
    if (slot_at[c] >= 0) HIP_TRY(save_state(s, s->d_ckpt[slot_at[c]]));
    const int64_t cn = std::min(C, n_steps - c * C);
    HIP_TRY(hipGraphLaunch(gp.pick(s, s->step, cn, C), s->stream));
    s->step += cn;
  }
  HIP_TRY(save_state(s, s->d_final));
  std::vector<double> ls(n_steps);
  HIP_TRY(hipMemcpyAsync(ls.data(), s->d_loss_steps, n_steps * 8, hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  double L = 0.0;
  for (double v : ls) L += v;
  *loss = L;
  return MONO_OK;
}

// Reverse sweep.  Per segment, from the last: load its checkpoint (the
// potential straight into the tape's first slot) and set the clock, then one
// graph recomputes the segment, taping what the reverse needs, and runs the
// reverse steps: adjoint diffusion substeps (the V adjoint ping-pongs between
// two rows, an even number of times per step), adjoint reaction with the
// sensors' loss gradient added in the same kernel.  Every segment of
// ckpt_every steps replays the same graph.
template <typename T>
mono_status backward_t(mono_sim* s) {
  const int64_t C = s->ckpt_every, N = s->tape_steps;
  const int64_t nck = (N + C - 1) / C;
  const int L = s->l_max, S = s->S;
  const size_t Np = s->Np;
  // segment tape b (0, or 1 when the uniform schedule overlaps segments)
  T* const vsubs[2] = {(T*)s->d_seg_vsub, (T*)s->d_seg_vsub2};
  T* const ents[2] = {(T*)s->d_seg_entry, (T*)s->d_seg_entry2};
  uint8_t* const ks[2] = {s->d_seg_k, s->d_seg_k2};
  // recompute of a segment into tape b: the forward steps, writing what the
  // reverse needs; the last step leaves the potential in the live state
  auto recompute = [=](int b) {
    return [=](int64_t cn) {
      return [=]() {
        for (int64_t t = 0; t < cn; ++t) {
          T* vs = vsubs[b] + (size_t)t * 2 * L * Np;
          T* vnext = (t + 1 < cn) ? vs + 2 * (size_t)L * Np : (T*)s->d_V[0];
          enqueue_tape_step<T>(s, t, vs, ents[b] + (size_t)t * S * Np, ks[b], cn, vnext);
        }
      };
    };
  };
  // reverse of a segment from tape b (the sensors' targets by the reverse's
  // own clock, d_base_rev, so that a recompute can run beside it)
  auto reverse = [=](int b) {
    return [=](int64_t cn) {
      return [=]() {
        T* lamV = (T*)s->d_lam;
        T* lamW = (T*)s->d_lamV2;
        for (int64_t t = cn - 1; t >= 0; --t) {
          const T* vs = vsubs[b] + (size_t)t * 2 * L * Np;
          const T* entry = ents[b] + (size_t)t * S * Np;
          for (int m = L - 1; m >= 0; --m) {
            launch_adj_diffusion<T>(
                s->layout, adj_diff_args<T>(s, lamV, lamW, vs + (size_t)(L + m) * Np, m),
                s->stream);
            std::swap(lamV, lamW);
          }
          AdjIonArgs<T> ai{};
          ai.n = s->n;
          ai.Np = s->Np;
          ai.entry = entry;
          ai.k = ks[b] + (size_t)t * s->n;
          ai.lam = (T*)s->d_lam;
          ai.lamV = lamV;
          ai.par = (const T*)s->d_par;
          for (int q = 0; q < kMaxParams; ++q) ai.par_uniform[q] = (T)s->par_uniform[q];
          ai.par_pernode = s->par_pernode;
          ai.dt = s->dt;
          ai.gpart = s->d_gpart;
          ai.sort = s->lc.react_sort;
          if (s->ns > 0) {
            // the loss gradient at reaction entry goes in with the reaction's
            // adjoint (one launch instead of two)
            SensorArgs sa = sensor_args(s, t);
            sa.clk.base = s->d_base_rev;
            ai.sens_of = s->d_sens_of;
            ai.target = sa.target;
            ai.ns = sa.ns;
            ai.target_steps = sa.target_steps;
            ai.clk = sa.clk;
          }
          launch_adj_ionic<T>(s->model, ai, s->stream);
          for (int m = L - 1; m >= 0; --m) {
            launch_adj_diffusion<T>(
                s->layout, adj_diff_args<T>(s, lamV, lamW, vs + (size_t)m * Np, m), s->stream);
            std::swap(lamV, lamW);
          }
        }
      };
    };
  };
  const bool overlap = s->ckpt_schedule == MONO_CKPT_UNIFORM && s->d_seg_vsub2 && nck > 1;
  const int nbuf = overlap ? 2 : 1;
  GraphPair rec[2], rev[2];
  for (int b = 0; b < nbuf; ++b) {
    // tape b serves the segments c with c % 2 == b when two tapes alternate
    mono_status st = rec[b].capture(s, recompute(b), N, C, true, s->tape_step0, nbuf, b);
    if (st == MONO_OK) st = rev[b].capture(s, reverse(b), N, C, false, s->tape_step0, nbuf, b);
    if (st != MONO_OK) return st;
  }
  // one segment: its state from a snapshot buffer (or the live state), the
  // recompute into tape b, then its reverse; with `aux` the recompute runs on
  // the auxiliary stream (after the reverse that last read tape b) and the
  // reverse on the simulation's stream after it
  hipEvent_t ev[5] = {};
  auto seg = [&](int64_t c, int from, int b, bool aux) -> mono_status {
    const int64_t t0 = c * C, cn = std::min(C, N - t0);
    hipStream_t R = s->stream;
    if (aux) {
      HIP_TRY(hipStreamWaitEvent(s->stream_aux, ev[2 + b], 0));    // tape b free
      s->stream = s->stream_aux;
    }
    hipError_t e = hipSuccess;
    if (from >= 0) {
      e = load_state(s, s->d_ckpt[from], vsubs[b]);
    } else {
      // the live state is the segment's start: its potential to the tape's
      // first slot, the other rows stay where the recompute reads them
      e = hipMemcpyAsync(vsubs[b], s->d_V[0], Np * s->es, hipMemcpyDeviceToDevice, s->stream);
    }
    if (e == hipSuccess) {
      launch_set_clock(s->d_base, s->tape_step0 + t0, s->stream);
      e = hipGraphLaunch(rec[b].pick(s, s->tape_step0 + t0, cn, C), s->stream);
    }
    if (aux) {
      if (e == hipSuccess) e = hipEventRecord(ev[b], s->stream);     // tape b written
      s->stream = R;
      if (e == hipSuccess) e = hipStreamWaitEvent(R, ev[b], 0);
    }
    HIP_TRY(e);
    launch_set_clock(s->d_base_rev, s->tape_step0 + t0, R);
    HIP_TRY(hipGraphLaunch(rev[b].pick(s, s->tape_step0 + t0, cn, C), R));
    if (aux) HIP_TRY(hipEventRecord(ev[2 + b], R));               // tape b read
    return MONO_OK;
  };
  mono_status st = MONO_OK;
  s->ckpt_advances = 0;
  if (overlap) {
    // segments from the last to the first; the recompute of segment c - 1
    // (auxiliary stream, tape (c - 1) % 2) runs while segment c is reversed
    // (tape c % 2); everything before this point on the simulation's stream
    // comes first
    if (!s->stream_aux &&
        hipStreamCreateWithFlags(&s->stream_aux, hipStreamNonBlocking) != hipSuccess)
      return fail(MONO_EDEVICE, "stream creation failed");
    for (hipEvent_t& e : ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        st = fail(MONO_EDEVICE, "event creation failed");
    if (st == MONO_OK) {
      hipError_t e = hipEventRecord(ev[4], s->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(s->stream_aux, ev[4], 0);
      for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipEventRecord(ev[2 + b], s->stream);
      if (e != hipSuccess) st = fail(MONO_EDEVICE, "stream ordering failed");
    }
    for (int64_t c = nck - 1; c >= 0 && st == MONO_OK; --c)
      st = seg(c, (int)c, (int)(c & 1), true);
    // the simulation's stream has waited for the last recompute
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (st != MONO_OK) {
      (void)hipStreamSynchronize(s->stream_aux);
      return st;
    }
  } else {
    // the schedule: segments reversed from the last to the first, each from a
    // snapshot buffer; in the binomial schedule, forward advances of whole
    // segments refill buffers in between
    struct Act {
      bool advance;
      int64_t c;     // segment reversed, or first segment advanced over
      int64_t m;     // segments advanced
      int from, to;  // snapshot buffers (reverse: `from` only; -1: the live state)
    };
    std::vector<Act> acts;
    if (s->ckpt_schedule == MONO_CKPT_UNIFORM) {
      for (int64_t c = nck - 1; c >= 0; --c) acts.push_back({false, c, 0, (int)c, -1});
    } else {
      const CkptPlan& p = s->plan;
      std::function<void(int64_t, int64_t, int, int)> revF = [&](int64_t first, int64_t k,
                                                                  int slot, int f) {
        if (k == 1) {
          acts.push_back({false, first, 0, slot, -1});
          return;
        }
        const int64_t m = p.splitF[p.idx(k, f)];
        if (k - m == 1) {
          // advance to the last segment and reverse it from the live state
          acts.push_back({true, first, m, slot, -1});
          acts.push_back({false, first + m, 0, -1, -1});
        } else {
          acts.push_back({true, first, m, slot, slot + 1});
          revF(first + m, k - m, slot + 1, f - 1);
        }
        revF(first, m, slot, f);
      };
      std::function<void(int64_t, int64_t, int, int)> revA = [&](int64_t first, int64_t k,
                                                                  int slot, int f) {
        if (k == 1) {
          acts.push_back({false, first, 0, slot, -1});
          return;
        }
        const int64_t m = p.splitA[p.idx(k, f)];
        if (m == 0) return revF(first, k, slot, f);
        revA(first + m, k - m, slot + 1, f - 1);
        revF(first, m, slot, f);
      };
      revA(0, nck, 0, p.width - 1);
    }
    // forward advances of whole segments (never the last, possibly shorter,
    // one): plain outer steps, the clock advanced on the device
    GraphPair adv;
    bool have_adv = false;
    for (const Act& a : acts) {
      if (a.advance && !have_adv) {
        auto plain = [s](int64_t cn) {
          return [s, cn]() {
            for (int64_t t = 0; t < cn; ++t) enqueue_loss_step<T>(s, t, false, nullptr, true);
            launch_advance_clock(s->d_base, cn, s->stream);
          };
        };
        st = adv.capture(s, plain, C, C);
        if (st != MONO_OK) return st;
        have_adv = true;
      }
      if (a.advance) {
        HIP_TRY(load_state(s, s->d_ckpt[a.from]));
        launch_set_clock(s->d_base, s->tape_step0 + a.c * C, s->stream);
        for (int64_t q = 0; q < a.m; ++q)
          HIP_TRY(hipGraphLaunch(adv.pick(s, s->tape_step0 + (a.c + q) * C, C, C), s->stream));
        if (a.to >= 0) HIP_TRY(save_state(s, s->d_ckpt[a.to]));
        s->ckpt_advances += a.m;
        continue;
      }
      st = seg(a.c, a.from, 0, false);
      if (st != MONO_OK) return st;
    }
  }
  HIP_TRY(hipGetLastError());
  // leave the simulation where the taped forward run ended
  HIP_TRY(load_state(s, s->d_final));
  launch_set_clock(s->d_base, s->tape_step0 + N, s->stream);
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->step = s->tape_step0 + N;
  return MONO_OK;
}

template <typename T>
void sample_steps(mono_sim* s, int64_t n_steps, double* dbuf) {
  for (int64_t t = 0; t < n_steps; ++t)
    enqueue_loss_step<T>(s, t, false, dbuf + t * s->ns);
  launch_advance_clock(s->d_base, n_steps, s->stream);
}

}  // namespace

// ===========================================================================
extern "C" {

const char* mono_last_error(void) { return t_err.c_str(); }

static mono_status create_mesh(const mono_mesh_desc* d, mono_sim** out);

mono_status mono_create_mesh(const mono_mesh_desc* d, mono_sim** out) {
  if (!d || !out) return fail(MONO_EINVAL, "NULL argument");
  if (!d->sigma_device || !d->sigma_node) return create_mesh(d, out);
  // conductivity scales in device memory: copied to the host, where the FP64
  // assembly runs
  *out = nullptr;
  if (d->n_nodes < 1 || d->n_nodes > (int64_t)INT32_MAX - 1024)
    return fail(MONO_EINVAL, "n_nodes out of range");
  hipPointerAttribute_t attr{};
  if (hipPointerGetAttributes(&attr, d->sigma_node) != hipSuccess ||
      attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(MONO_EINVAL, "sigma_device set but sigma_node is not device memory");
  }
  std::vector<double> sg((size_t)d->n_nodes);
  HIP_TRY(hipMemcpy(sg.data(), d->sigma_node, sg.size() * 8, hipMemcpyDeviceToHost));
  mono_mesh_desc h = *d;
  h.sigma_node = sg.data();
  h.sigma_device = 0;
  return create_mesh(&h, out);
}

static mono_status create_mesh(const mono_mesh_desc* d, mono_sim** out) {
  *out = nullptr;
  if (d->dim < 1 || d->dim > 3) return fail(MONO_EINVAL, "dim must be 1, 2 or 3");
  if (d->etype != (1 << d->dim) && !(d->dim >= 2 && d->etype == d->dim + 1))
    return fail(MONO_EINVAL, "etype does not match dim");
  if (d->n_nodes < 1 || d->n_nodes > (int64_t)INT32_MAX - 1024)
    return fail(MONO_EINVAL, "n_nodes out of range");
  if (d->n_elems < 0) return fail(MONO_EINVAL, "n_elems must be >= 0");
  if (d->prec != MONO_F64 && d->prec != MONO_F32) return fail(MONO_EINVAL, "bad precision");
  if (d->layout < MONO_LAYOUT_AUTO || d->layout > MONO_LAYOUT_STENCIL)
    return fail(MONO_EINVAL, "bad layout");
  const int ni = d->n_instances < 1 ? 1 : d->n_instances;
  std::vector<int64_t> off;
  if (ni == 1 || !d->inst_node_off) {
    if (ni > 1) return fail(MONO_EINVAL, "inst_node_off required for several instances");
    off = {0, d->n_nodes};
  } else {
    off.assign(d->inst_node_off, d->inst_node_off + ni + 1);
    if (off[0] != 0 || off[ni] != d->n_nodes) return fail(MONO_EINVAL, "bad instance offsets");
    for (int q = 0; q < ni; ++q)
      if (off[q + 1] <= off[q]) return fail(MONO_EINVAL, "empty or decreasing instance");
  }
  mono_sim* s = new mono_sim();
  g_live_sims.fetch_add(1);
  s->prec = d->prec;
  s->es = d->prec == MONO_F64 ? 8 : 4;
  s->dim = d->dim;
  s->n = d->n_nodes;
  s->Np = (d->n_nodes + kBlock - 1) / kBlock * kBlock;
  s->n_inst = ni;
  s->inst_off = off;
  auto bail = [&](mono_status st) {
    mono_destroy(s);
    return st;
  };
  std::string err;
  int rc = assemble_fe(d, s->K, err);
  if (rc != MONO_OK) return bail(fail((mono_status)rc, err));
  s->nnz = (int64_t)s->K.col.size();
  // instance ids; elements must not join instances
  std::vector<int32_t> inst(s->n, 0);
  for (int q = 0; q < ni; ++q)
    for (int64_t i = off[q]; i < off[q + 1]; ++i) inst[i] = q;
  if (ni > 1) {
    const int nen = d->etype;
    for (int64_t e = 0; e < d->n_elems; ++e) {
      const int32_t q0 = inst[d->conn[e * nen]];
      for (int a = 1; a < nen; ++a)
        if (inst[d->conn[e * nen + a]] != q0)
          return bail(fail(MONO_EINVAL, "element joins two instances"));
    }
  }
  // stream
  if (d->stream) {
    s->stream = (hipStream_t)d->stream;
  } else {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(MONO_EDEVICE, "hipStreamCreate failed"));
    s->own_stream = true;
  }
  // small per-instance arrays, clock and flags
  if (dalloc(&s->d_base, 1) || dalloc(&s->d_flag, 1) || dalloc(&s->d_l, ni) ||
      dalloc(&s->d_dtad, ni) || dalloc(&s->d_inst_off, ni + 1))
    return bail(fail(MONO_ENOMEM, "device allocation failed"));
  if (hipMemsetAsync(s->d_base, 0, 8, s->stream) ||
      hipMemsetAsync(s->d_flag, 0, sizeof(int), s->stream) || hipStreamSynchronize(s->stream) ||
      hipMemcpy(s->d_inst_off, off.data(), (ni + 1) * 8, hipMemcpyHostToDevice))
    return bail(fail(MONO_EDEVICE, "device initialisation failed"));
  if (ni > 1) {
    std::vector<int32_t> ip(s->Np, ni - 1);
    std::copy(inst.begin(), inst.end(), ip.begin());
    if (dalloc(&s->d_inst, s->Np)) return bail(fail(MONO_ENOMEM, "device allocation failed"));
    if (hipMemcpy(s->d_inst, ip.data(), s->Np * 4, hipMemcpyHostToDevice))
      return bail(fail(MONO_EDEVICE, "upload failed"));
  }
  // eq. (3) in FP64 on the device
  {
    int64_t *rp = nullptr;
    int32_t* col = nullptr;
    double *val = nullptr, *mass = nullptr, *r = nullptr, *g = nullptr, *rmin = nullptr,
           *gmx = nullptr;
    bool ok = !dalloc(&rp, s->n + 1) && !dalloc(&col, s->nnz) && !dalloc(&val, s->nnz) &&
              !dalloc(&mass, s->n) && !dalloc(&r, s->n) && !dalloc(&g, s->n) &&
              !dalloc(&rmin, ni) && !dalloc(&gmx, ni);
    std::vector<double> hr(ni), hg(ni);
    if (ok)
      ok = !hipMemcpy(rp, s->K.rp.data(), (s->n + 1) * 8, hipMemcpyHostToDevice) &&
           !hipMemcpy(col, s->K.col.data(), s->nnz * 4, hipMemcpyHostToDevice) &&
           !hipMemcpy(val, s->K.val.data(), s->nnz * 8, hipMemcpyHostToDevice) &&
           !hipMemcpy(mass, s->K.mass.data(), s->n * 8, hipMemcpyHostToDevice);
    if (ok) {
      launch_gershgorin(s->n, rp, col, val, mass, r, g, s->stream);
      launch_segmented_minmax(ni, s->d_inst_off, r, g, rmin, gmx, s->stream);
      ok = !hipMemcpyAsync(hr.data(), rmin, ni * 8, hipMemcpyDeviceToHost, s->stream) &&
           !hipMemcpyAsync(hg.data(), gmx, ni * 8, hipMemcpyDeviceToHost, s->stream) &&
           !hipStreamSynchronize(s->stream) && !hipGetLastError();
    }
    dfree(rp);
    dfree(col);
    dfree(val);
    dfree(mass);
    dfree(r);
    dfree(g);
    dfree(rmin);
    dfree(gmx);
    if (!ok) return bail(fail(MONO_EDEVICE, "Gershgorin kernel failed"));
    s->dt_s.resize(ni);
    s->gmax = hg;
    s->lambda.assign(ni, 0.0);
    for (int q = 0; q < ni; ++q) {
      if (!(hr[q] > 0.0) || !std::isfinite(hr[q]))
        return bail(fail(MONO_EINVAL, "degenerate stiffness (no diffusion) in an instance"));
      s->dt_s[q] = 0.9 * hr[q];
    }
  }
  // conductivity scales (adjoint) and 1/m in both layouts
  {
    std::vector<double> sg(s->Np, 1.0);
    if (d->sigma_node) std::copy(d->sigma_node, d->sigma_node + s->n, sg.begin());
    {
      // uniform in the simulation precision (padding rows hold 1 and are never read)
      auto rnd = [s](double v) { return s->prec == MONO_F32 ? (double)(float)v : v; };
      s->sigma_value = rnd(sg[0]);
      s->sigma_uniform = 1;
      for (int64_t i = 1; i < s->n && s->sigma_uniform; ++i)
        if (rnd(sg[i]) != s->sigma_value) s->sigma_uniform = 0;
    }
    if (dalloc((char**)&s->d_sigma, s->Np * s->es))
      return bail(fail(MONO_ENOMEM, "device allocation failed"));
    mono_status st = upload_real(s, s->d_sigma, sg.data(), sg.size());
    if (st != MONO_OK) return bail(st);
  }
  // operator layout
  int layout = d->layout;
  StencilHost sh;
  bool stencil_ok = false;
  if (layout != MONO_LAYOUT_ELL) stencil_ok = build_stencil(s->K, off, s->Np, sh);
  if (layout == MONO_LAYOUT_STENCIL && !stencil_ok)
    return bail(fail(MONO_EUNSUPPORTED, "mesh numbering has too many stencil offsets"));
  if (layout == MONO_LAYOUT_AUTO) layout = stencil_ok ? MONO_LAYOUT_STENCIL : MONO_LAYOUT_ELL;
  s->layout = layout;
  if (layout == MONO_LAYOUT_STENCIL) {
    s->P = sh.P;
    if (dalloc((char**)&s->d_e, (size_t)sh.P * s->Np * s->es) ||
        dalloc((char**)&s->d_minv, s->Np * s->es) || dalloc(&s->d_off, sh.off.size()))
      return bail(fail(MONO_ENOMEM, "device allocation failed"));
    mono_status st = upload_real(s, s->d_e, sh.e.data(), sh.e.size());
    if (st == MONO_OK) st = upload_real(s, s->d_minv, sh.minv.data(), sh.minv.size());
    if (st != MONO_OK) return bail(st);
    if (hipMemcpy(s->d_off, sh.off.data(), sh.off.size() * 4, hipMemcpyHostToDevice))
      return bail(fail(MONO_EDEVICE, "upload failed"));
    // the kernels that read rows by class (and the row-sharing and fused
    // forms built on them) index rows with 32-bit byte offsets, so classes are
    // used only where every row array stays below 2 GiB; larger meshes keep
    // the per-row stencil with 64-bit indices
    RowClasses rc;
    const bool narrow = s->Np * (int64_t)s->es < ((int64_t)1 << 31);
    if (narrow && build_row_classes(sh, s->n, s->Np, s->prec == MONO_F32, 65535, rc)) {
      if (dalloc(&s->d_cls, rc.cls.size()) ||
          dalloc((char**)&s->d_ctab, rc.table.size() * s->es))
        return bail(fail(MONO_ENOMEM, "device allocation failed"));
      if (hipMemcpy(s->d_cls, rc.cls.data(), rc.cls.size() * 2, hipMemcpyHostToDevice))
        return bail(fail(MONO_EDEVICE, "upload failed"));
      st = upload_real(s, s->d_ctab, rc.table.data(), rc.table.size());
      if (st != MONO_OK) return bail(st);
      s->tw = rc.tw;
      s->n_classes = rc.n_classes;
      s->row_pattern = grid_row_pattern(sh.off) ? 1 : 0;
      if (s->row_pattern) {
        s->grid_nx = sh.P >= 4 ? sh.off[2] : 0;
        s->grid_nxy = sh.P >= 13 ? sh.off[8] : 0;
        // class shared by all kWaveRows rows of a wavefront, else kNoClass
        const int64_t nw = (s->n + kWaveRows - 1) / kWaveRows;
        std::vector<int32_t> wc(nw);
        for (int64_t w = 0; w < nw; ++w) {
          const int64_t r0 = w * kWaveRows, r1 = std::min<int64_t>(r0 + kWaveRows, s->n);
          int32_t c = rc.cls[r0];
          for (int64_t r = r0 + 1; r < r1 && c != kNoClass; ++r)
            if (rc.cls[r] != c) c = kNoClass;
          wc[w] = c;
        }
        if (dalloc(&s->d_wcls, nw)) return bail(fail(MONO_ENOMEM, "device allocation failed"));
        if (hipMemcpy(s->d_wcls, wc.data(), nw * 4, hipMemcpyHostToDevice))
          return bail(fail(MONO_EDEVICE, "upload failed"));
        if (sh.P == 13 && fused_grid_ok(sh, s->n, s->Np, s->es, s->grid_nx, s->grid_nxy)) {
          int dev = 0, cus = 0;
          if (hipGetDevice(&dev) != hipSuccess ||
              hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                  hipSuccess)
            return bail(fail(MONO_EDEVICE, "device query failed"));
          s->n_cu = std::max(cus, 1);
          s->fuse_ok = 1;
          s->grid_ny = s->grid_nxy / s->grid_nx;
          s->grid_nz = (int)(s->n / s->grid_nxy);
        }
      }
    }
  } else {
    EllHost eh;
    build_ell(s->K, s->Np, eh);
    s->W = eh.width;
    if (dalloc(&s->d_col, eh.col.size()) || dalloc((char**)&s->d_val, eh.val.size() * s->es) ||
        dalloc((char**)&s->d_minv, s->Np * s->es))
      return bail(fail(MONO_ENOMEM, "device allocation failed"));
    {
      std::vector<double> mi(s->Np, 0.0);
      for (int64_t i = 0; i < s->n; ++i) mi[i] = 1.0 / s->K.mass[i];
      mono_status st = upload_real(s, s->d_minv, mi.data(), mi.size());
      if (st != MONO_OK) return bail(st);
    }
    if (hipMemcpy(s->d_col, eh.col.data(), eh.col.size() * 4, hipMemcpyHostToDevice))
      return bail(fail(MONO_EDEVICE, "upload failed"));
    mono_status st = upload_real(s, s->d_val, eh.val.data(), eh.val.size());
    if (st != MONO_OK) return bail(st);
  }
  *out = s;
  return MONO_OK;
}

mono_status mono_set_allocator(void* (*alloc)(size_t, void*), void (*free_)(void*, void*),
                               void* ctx) {
  if ((alloc == nullptr) != (free_ == nullptr))
    return fail(MONO_EINVAL, "give both allocator functions or neither");
  if (g_live_sims.load() != 0)
    return fail(MONO_ESTATE, "the allocator can change only while no simulation exists");
  g_alloc.alloc = alloc;
  g_alloc.free_ = free_;
  g_alloc.ctx = alloc ? ctx : nullptr;
  return MONO_OK;
}

void mono_destroy(mono_sim* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  drop_graph(s);
  free_model(s);
  dfree(s->d_inst);
  dfree(s->d_inst_off);
  dfree(s->d_col);
  dfree(s->d_val);
  dfree(s->d_e);
  dfree(s->d_cls);
  dfree(s->d_ctab);
  dfree(s->d_wcls);
  dfree(s->d_minv);
  dfree(s->d_off);
  dfree(s->d_mask);
  dfree(s->d_l);
  dfree(s->d_dtad);
  dfree(s->d_base);
  dfree(s->d_flag);
  dfree(s->d_stats);
  free_tape(s);
  dfree(s->d_sigma);
  dfree(s->d_sens);
  dfree(s->d_sens_of);
  dfree(s->d_target);
  for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
  if (s->stream_aux) (void)hipStreamDestroy(s->stream_aux);
  delete s;
  g_live_sims.fetch_sub(1);
}

mono_status mono_set_cell_model(mono_sim* s, int32_t model, int32_t n_params,
                                const double* params, const double* init_state, double dt0) {
  if (!s) return fail(MONO_EINVAL, "NULL simulation");
  if (model < MONO_MODEL_LINEAR || model > MONO_MODEL_TP06_FIBRO)
    return fail(MONO_EINVAL, "unknown cell model");
  if (!(dt0 > 0.0)) return fail(MONO_EINVAL, "dt0 must be positive");
  const int S = model_states(model), P = model_params(model);
  if (params && n_params != P) return fail(MONO_EINVAL, "wrong number of parameter rows");
  if (params && model == MONO_MODEL_TP06_TYPES)
    for (int64_t i = 0; i < s->n; ++i) {
      const double c = params[(size_t)6 * s->n + i];
      if (c != 0.0 && c != 1.0 && c != 2.0)
        return fail(MONO_EINVAL, "cell type row must hold 0, 1 or 2");
    }
  if (params && model == MONO_MODEL_TP06_FIBRO)
    for (int64_t i = 0; i < s->n; ++i) {
      const double c = params[(size_t)6 * s->n + i];
      if (c != 0.0 && c != 1.0) return fail(MONO_EINVAL, "node class row must hold 0 or 1");
    }
  HIP_TRY(hipStreamSynchronize(s->stream));
  drop_graph(s);
  free_model(s);
  s->model = model;
  s->S = S;
  s->Pm = P;
  const size_t Np = s->Np, es = s->es;
  if (dalloc((char**)&s->d_V[0], Np * es) || dalloc((char**)&s->d_V[1], Np * es) ||
      dalloc((char**)&s->d_st, (size_t)std::max(S - 1, 1) * Np * es) ||
      dalloc((char**)&s->d_vprev, Np * es) || dalloc(&s->d_lat, Np) || dalloc(&s->d_k, Np))
    return fail(MONO_ENOMEM, "device allocation failed");
  HIP_TRY(hipMemsetAsync(s->d_V[0], 0, Np * es, s->stream));
  HIP_TRY(hipMemsetAsync(s->d_V[1], 0, Np * es, s->stream));
  HIP_TRY(hipMemsetAsync(s->d_st, 0, (size_t)std::max(S - 1, 1) * Np * es, s->stream));
  HIP_TRY(hipMemsetAsync(s->d_k, 0, Np, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));

  // initial state
  std::vector<double> y((size_t)S * s->n);
  if (init_state) {
    std::memcpy(y.data(), init_state, y.size() * 8);
  } else {
    for (int a = 0; a < S; ++a) {
      double v = 0.0;
      if (is_tp06(model)) v = kTP06Init[a];
      if (model == MONO_MODEL_MS) v = (a == 0) ? 0.0 : 1.0;
      std::fill(y.begin() + (size_t)a * s->n, y.begin() + (size_t)(a + 1) * s->n, v);
    }
  }
  mono_status st = upload_real(s, s->d_V[0], y.data(), s->n);
  if (st == MONO_OK) st = upload_real(s, s->d_vprev, y.data(), s->n);
  for (int a = 1; a < S && st == MONO_OK; ++a)
    st = upload_real(s, (char*)s->d_st + (size_t)(a - 1) * Np * es, y.data() + (size_t)a * s->n,
                     s->n);
  if (st != MONO_OK) return st;
  {
    std::vector<double> lat(s->n, -1.0);
    HIP_TRY(hipMemcpy(s->d_lat, lat.data(), s->n * 8, hipMemcpyHostToDevice));
  }
  // parameters: uniform rows are passed by value, the others stored per node
  s->par_pernode = 0;
  std::vector<double> pu(P);
  for (int a = 0; a < P; ++a) {
    double v = model == MONO_MODEL_MS ? kMSParams[a]
                                      : (is_tp06(model) ? kTP06Params[a] : 0.0);
    if (params) {
      const double* row = params + (size_t)a * s->n;
      v = row[0];
      for (int64_t i = 1; i < s->n; ++i)
        if (row[i] != v) {
          s->par_pernode |= 1u << a;
          break;
        }
    }
    s->par_uniform[a] = v;
  }
  if (s->par_pernode) {
    if (dalloc((char**)&s->d_par, (size_t)P * Np * es))
      return fail(MONO_ENOMEM, "device allocation failed");
    HIP_TRY(hipMemsetAsync(s->d_par, 0, (size_t)P * Np * es, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int a = 0; a < P; ++a)
      if (s->par_pernode >> a & 1u) {
        st = upload_real(s, (char*)s->d_par + (size_t)a * Np * es, params + (size_t)a * s->n, s->n);
        if (st != MONO_OK) return st;
      }
  }
  s->dt0 = dt0;
  s->scal_n = -1;
  s->lat_thr = default_lat_threshold(model);
  s->step = 0;
  HIP_TRY(hipMemsetAsync(s->d_base, 0, 8, s->stream));
  HIP_TRY(hipMemsetAsync(s->d_flag, 0, sizeof(int), s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->latched = false;
  if (s->dt > 0.0) {
    const double dt = s->dt;
    s->dt = -1.0;
    return prepare(s, dt);
  }
  return MONO_OK;
}

mono_status mono_set_lat_threshold(mono_sim* s, double v) {
  if (!s || !std::isfinite(v)) return fail(MONO_EINVAL, "bad argument");
  s->lat_thr = v;
  drop_graph(s);
  return MONO_OK;
}

mono_status mono_add_stimulus(mono_sim* s, int64_t n, const int32_t* nodes, double t_on,
                              double duration, double amplitude) {
  if (!s || (n > 0 && !nodes) || n < 0) return fail(MONO_EINVAL, "bad argument");
  if (s->stim.n >= kMaxStim) return fail(MONO_EUNSUPPORTED, "at most 8 stimuli");
  if (!std::isfinite(t_on) || !(duration >= 0.0) || !std::isfinite(amplitude))
    return fail(MONO_EINVAL, "bad stimulus timing or amplitude");
  std::vector<uint8_t> mask(s->Np, 0);
  if (s->d_mask) {
    HIP_TRY(hipStreamSynchronize(s->stream));
    HIP_TRY(hipMemcpy(mask.data(), s->d_mask, s->Np, hipMemcpyDeviceToHost));
  } else if (dalloc(&s->d_mask, s->Np)) {
    return fail(MONO_ENOMEM, "device allocation failed");
  }
  const int b = s->stim.n;
  for (int64_t q = 0; q < n; ++q) {
    if (nodes[q] < 0 || nodes[q] >= s->n) return fail(MONO_EINVAL, "stimulus node out of range");
    mask[nodes[q]] |= (uint8_t)(1u << b);
  }
  HIP_TRY(hipMemcpy(s->d_mask, mask.data(), s->Np, hipMemcpyHostToDevice));
  s->stim.t_on[b] = t_on;
  s->stim.t_end[b] = t_on + duration;
  s->stim.amp[b] = amplitude;
  s->stim.n = b + 1;
  drop_graph(s);
  return MONO_OK;
}

mono_status mono_set_method(mono_sim* s, int32_t method, int32_t dvdt_source, int32_t l_round) {
  if (!s || method < MONO_DAETI || method > MONO_OST || dvdt_source < 0 || dvdt_source > 1 ||
      l_round < 0 || l_round > 1)
    return fail(MONO_EINVAL, "bad method flags");
  s->method = method;
  s->dvdt_src = dvdt_source;
  s->l_round = l_round;
  drop_graph(s);
  if (s->dt > 0.0) {
    const double dt = s->dt;
    s->dt = -1.0;
    return prepare(s, dt);
  }
  return MONO_OK;
}

mono_status mono_prepare(mono_sim* s, double dt) {
  if (!s) return fail(MONO_EINVAL, "NULL simulation");
  return prepare(s, dt);
}

mono_status mono_step(mono_sim* s, int64_t n_steps, double dt, uint32_t flags) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (n_steps < 0) return fail(MONO_EINVAL, "negative step count");
  if (s->latched) return fail(MONO_ESTATE, "simulation latched after a non-finite potential");
  st = prepare(s, dt);
  if (st != MONO_OK) return st;
  int64_t left = n_steps;
  if (flags & 2u) {
    st = enqueue_timed(s, n_steps);
    if (st != MONO_OK) return st;
    HIP_TRY(hipGetLastError());
    s->step += n_steps;
    return MONO_OK;
  }
  const int64_t chunk = s->lc.graph_steps;
  if (flags & 4u) {
    // capture the graphs a graph-mode call of n_steps would replay; run nothing
    if (flags & 1u) return fail(MONO_EINVAL, "capture-only needs graph mode");
    st = ensure_graph(s);
    if (st == MONO_OK && n_steps % chunk) st = ensure_rem_graph(s, n_steps % chunk);
    return st;
  }
  if (!(flags & 1u) && left > 0) {
    // the first graph-mode call captures the graph of graph_steps steps, so
    // later calls launch it without capture work
    st = ensure_graph(s);
    if (st != MONO_OK) return st;
    while (left >= chunk) {
      const int64_t step0 = s->step + (n_steps - left);
      const bool q = s->gexec_q && chunk_is_quiet(s, step0, chunk);
      HIP_TRY(hipGraphLaunch(q ? s->gexec_q : s->gexec, s->stream));
      left -= chunk;
    }
  }
  if (left > 0) {
    if (flags & 1u) {
      enqueue(s, left);
    } else {
      st = ensure_rem_graph(s, left);
      if (st != MONO_OK) return st;
      const bool q = s->gexec_rq && chunk_is_quiet(s, s->step + (n_steps - left), left);
      HIP_TRY(hipGraphLaunch(q ? s->gexec_rq : s->gexec_r, s->stream));
    }
  }
  HIP_TRY(hipGetLastError());
  s->step += n_steps;
  return MONO_OK;
}

mono_status mono_apply_phase(mono_sim* s, int32_t phase, int64_t step, int32_t m) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (s->dt <= 0.0) return fail(MONO_ESTATE, "call mono_prepare first");
  if (phase < 0 || phase > 2 || step < 0 || m < 0 || m >= s->l_max)
    return fail(MONO_EINVAL, "bad phase, step or substep");
  HIP_TRY(hipMemcpyAsync(s->d_base, &step, 8, hipMemcpyHostToDevice, s->stream));
  if (phase == 1) {
    if (s->prec == MONO_F64)
      launch_ionic<double>(s->model, ion_args<double>(s, s->d_V[0], 0), s->lc, s->stream);
    else
      launch_ionic<float>(s->model, ion_args<float>(s, s->d_V[0], 0), s->lc, s->stream);
  } else {
    const int half = phase / 2;
    if (s->prec == MONO_F64)
      launch_diffusion<double>(s->layout, diff_args<double>(s, 0, half, m, 0), s->lc,
                               s->stream);
    else
      launch_diffusion<float>(s->layout, diff_args<float>(s, 0, half, m, 0), s->lc, s->stream);
    HIP_TRY(hipMemcpyAsync(s->d_V[0], s->d_V[1], s->Np * s->es, hipMemcpyDeviceToDevice,
                           s->stream));
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(s->d_base, &s->step, 8, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return check_flag(s);
}

mono_status mono_get_state(mono_sim* s, int32_t field, double* dst, int64_t count) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (!dst || count != s->n) return fail(MONO_EINVAL, "count must equal n_nodes");
  if (field == MONO_FIELD_APD || field == MONO_FIELD_TUP) {
    if (!s->d_apd) return fail(MONO_ESTATE, "APD tracking is off (mono_track_apd)");
    std::vector<double> tup(s->n), trep(s->n);
    HIP_TRY(hipMemcpyAsync(tup.data(), s->d_apd, s->n * 8, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipMemcpyAsync(trep.data(), s->d_apd + 4 * s->Np, s->n * 8, hipMemcpyDeviceToHost,
                           s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int64_t i = 0; i < s->n; ++i)
      dst[i] = field == MONO_FIELD_TUP ? tup[i]
                                       : ((tup[i] >= 0.0 && trep[i] >= 0.0) ? trep[i] - tup[i] : -1.0);
    return check_flag(s);
  }
  size_t es = 0;
  void* src = field_ptr(s, field, es);
  if (!src) return fail(MONO_EINVAL, "unknown field");
  if (field == MONO_FIELD_LAT) {
    HIP_TRY(hipMemcpyAsync(dst, src, s->n * 8, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  } else if (field == MONO_FIELD_K) {
    std::vector<uint8_t> k(s->n);
    HIP_TRY(hipMemcpyAsync(k.data(), src, s->n, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int64_t i = 0; i < s->n; ++i) dst[i] = k[i];
  } else {
    st = download_real(s, dst, src, s->n);
    if (st != MONO_OK) return st;
  }
  return check_flag(s);
}

mono_status mono_get_state_device_async(mono_sim* s, int32_t field, void* dev_dst) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (!dev_dst) return fail(MONO_EINVAL, "NULL destination");
  size_t es = 0;
  void* src = field_ptr(s, field, es);
  if (!src) return fail(MONO_EINVAL, "unknown field");
  HIP_TRY(hipMemcpyAsync(dev_dst, src, s->n * es, hipMemcpyDeviceToDevice, s->stream));
  return MONO_OK;
}

mono_status mono_set_state(mono_sim* s, int32_t field, const double* src, int64_t count) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (!src || count != s->n) return fail(MONO_EINVAL, "count must equal n_nodes");
  if (field == MONO_FIELD_K || field == MONO_FIELD_APD || field == MONO_FIELD_TUP)
    return fail(MONO_EINVAL, "field is read-only");
  size_t es = 0;
  void* dst = field_ptr(s, field, es);
  if (!dst) return fail(MONO_EINVAL, "unknown field");
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (field == MONO_FIELD_LAT) {
    HIP_TRY(hipMemcpy(dst, src, s->n * 8, hipMemcpyHostToDevice));
  } else {
    st = upload_real(s, dst, src, s->n);
    if (st != MONO_OK) return st;
  }
  if (field == MONO_FIELD_V || field == MONO_FIELD_STATE0) {
    HIP_TRY(hipMemsetAsync(s->d_flag, 0, sizeof(int), s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->latched = false;
  }
  return MONO_OK;
}

mono_status mono_track_apd(mono_sim* s, int32_t on) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (on != 0 && on != 1) return fail(MONO_EINVAL, "on must be 0 or 1");
  HIP_TRY(hipStreamSynchronize(s->stream));
  drop_graph(s);
  if (!on) {
    dfree(s->d_apd);
    return MONO_OK;
  }
  if (!s->d_apd && dalloc(&s->d_apd, 5 * s->Np))
    return fail(MONO_ENOMEM, "device allocation failed");
  // upstroke and repolarisation times -1 (not activated), the rest 0
  std::vector<double> init(5 * s->Np, 0.0);
  std::fill(init.begin(), init.begin() + s->Np, -1.0);
  std::fill(init.begin() + 4 * s->Np, init.end(), -1.0);
  HIP_TRY(hipMemcpy(s->d_apd, init.data(), init.size() * 8, hipMemcpyHostToDevice));
  return MONO_OK;
}

mono_status mono_nrmse(const double* u_hat, const double* u, int64_t n, double* out) {
  if (!u_hat || !u || !out || n < 0) return fail(MONO_EINVAL, "bad argument");
  double ss = 0.0, lo = INFINITY, hi = -INFINITY;
  int64_t cnt = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!(u_hat[i] >= 0.0) || !(u[i] >= 0.0)) continue;
    const double e = u_hat[i] - u[i];
    ss += e * e;
    lo = std::min(lo, u[i]);
    hi = std::max(hi, u[i]);
    ++cnt;
  }
  *out = (cnt > 0 && hi > lo) ? std::sqrt(ss / (double)cnt) / (hi - lo) : NAN;
  return MONO_OK;
}

mono_status mono_set_time_level(mono_sim* s, int64_t step) {
  if (!s || step < 0) return fail(MONO_EINVAL, "bad argument");
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->step = step;
  HIP_TRY(hipMemcpy(s->d_base, &step, 8, hipMemcpyHostToDevice));
  return MONO_OK;
}

mono_status mono_get_info(mono_sim* s, int32_t inst, mono_info* out) {
  if (!s || !out) return fail(MONO_EINVAL, "NULL argument");
  if (inst < 0 || inst >= s->n_inst) return fail(MONO_EINVAL, "bad instance index");
  std::memset(out, 0, sizeof(*out));
  out->dt_s = s->dt_s[inst];
  out->G_max = s->gmax[inst];
  out->lambda_est = s->lambda[inst];
  out->dt = s->dt > 0.0 ? s->dt : 0.0;
  if (s->dt > 0.0) {
    out->dt_ad = s->dt_ad[inst];
    out->l = s->l[inst];
    out->k_max = s->k_max;
    out->t = (double)s->step * s->dt;
  }
  out->step = s->step;
  out->nnz = s->nnz;
  out->layout = s->layout;
  out->n_instances = s->n_inst;
  out->n_states = s->S;
  out->ell_width = s->layout == MONO_LAYOUT_ELL ? s->W : s->P;
  out->row_classes = s->n_classes;
  out->grid_rows = s->row_pattern;
  out->diff_fused = s->fuse_ok;
  if (s->dt > 0.0) out->diff_launches = diff_launches_per_half(s);
  return MONO_OK;
}

mono_status mono_estimate_lambda(mono_sim* s, int32_t iters) {
  if (!s || iters < 1) return fail(MONO_EINVAL, "bad argument");
  const int ni = s->n_inst;
  int64_t* rp = nullptr;
  int32_t* col = nullptr;
  double *val = nullptr, *mass = nullptr, *x = nullptr, *kx = nullptr, *xkx = nullptr,
         *xmx = nullptr;
  bool ok = !dalloc(&rp, s->n + 1) && !dalloc(&col, s->nnz) && !dalloc(&val, s->nnz) &&
            !dalloc(&mass, s->n) && !dalloc(&x, s->n) && !dalloc(&kx, s->n) &&
            !dalloc(&xkx, ni) && !dalloc(&xmx, ni);
  std::vector<double> a(ni), b(ni);
  if (ok)
    ok = !hipMemcpy(rp, s->K.rp.data(), (s->n + 1) * 8, hipMemcpyHostToDevice) &&
         !hipMemcpy(col, s->K.col.data(), s->nnz * 4, hipMemcpyHostToDevice) &&
         !hipMemcpy(val, s->K.val.data(), s->nnz * 8, hipMemcpyHostToDevice) &&
         !hipMemcpy(mass, s->K.mass.data(), s->n * 8, hipMemcpyHostToDevice);
  if (ok) {
    const int32_t* inst = ni > 1 ? s->d_inst : nullptr;
    launch_power_init(s->n, x, s->stream);
    for (int it = 0; it < iters; ++it) {
      launch_spmv_csr(s->n, rp, col, val, x, kx, s->stream);
      launch_segmented_dots(ni, s->d_inst_off, x, kx, mass, xkx, xmx, s->stream);
      launch_power_update(s->n, inst, kx, mass, xmx, x, s->stream);
    }
    launch_spmv_csr(s->n, rp, col, val, x, kx, s->stream);
    launch_segmented_dots(ni, s->d_inst_off, x, kx, mass, xkx, xmx, s->stream);
    ok = !hipMemcpyAsync(a.data(), xkx, ni * 8, hipMemcpyDeviceToHost, s->stream) &&
         !hipMemcpyAsync(b.data(), xmx, ni * 8, hipMemcpyDeviceToHost, s->stream) &&
         !hipStreamSynchronize(s->stream) && !hipGetLastError();
  }
  dfree(rp);
  dfree(col);
  dfree(val);
  dfree(mass);
  dfree(x);
  dfree(kx);
  dfree(xkx);
  dfree(xmx);
  if (!ok) return fail(MONO_EDEVICE, "power iteration failed");
  for (int q = 0; q < ni; ++q) {
    s->lambda[q] = a[q] / b[q];
    if (s->dt > 0.0 && !(s->dt_ad[q] < 2.0 / s->lambda[q]))
      return fail(MONO_ESTATE, "dt_ad violates the forward Euler bound 2/lambda_max");
  }
  return MONO_OK;
}

mono_status mono_set_sensors(mono_sim* s, int32_t n, const int32_t* nodes, const double* target,
                             int64_t n_steps) {
  if (!s || n < 0 || (n > 0 && (!nodes || !target)) || n_steps < 0)
    return fail(MONO_EINVAL, "bad argument");
  std::vector<int32_t> v(nodes, nodes + n);
  for (int32_t i : v)
    if (i < 0 || i >= s->n) return fail(MONO_EINVAL, "sensor node out of range");
  std::vector<int32_t> u = v;
  std::sort(u.begin(), u.end());
  if (std::adjacent_find(u.begin(), u.end()) != u.end())
    return fail(MONO_EINVAL, "sensor nodes must be distinct");
  HIP_TRY(hipStreamSynchronize(s->stream));
  drop_graph(s);
  dfree(s->d_sens);
  dfree(s->d_sens_of);
  dfree(s->d_target);
  s->ns = n;
  s->target_steps = n_steps;
  if (n > 0) {
    if (dalloc(&s->d_sens, n) || dalloc(&s->d_target, (size_t)n * std::max<int64_t>(n_steps, 1)) ||
        dalloc(&s->d_sens_of, s->Np))
      return fail(MONO_ENOMEM, "device allocation failed");
    HIP_TRY(hipMemcpy(s->d_sens, v.data(), n * 4, hipMemcpyHostToDevice));
    std::vector<int32_t> of(s->Np, -1);
    for (int32_t q = 0; q < n; ++q) of[v[q]] = q;
    HIP_TRY(hipMemcpy(s->d_sens_of, of.data(), s->Np * 4, hipMemcpyHostToDevice));
    if (n_steps > 0)
      HIP_TRY(hipMemcpy(s->d_target, target, (size_t)n * n_steps * 8, hipMemcpyHostToDevice));
  }
  return MONO_OK;
}

mono_status mono_sample_sensors(mono_sim* s, int64_t n_steps, double dt, double* out) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (n_steps < 0 || (n_steps > 0 && !out)) return fail(MONO_EINVAL, "bad argument");
  if (s->ns <= 0) return fail(MONO_ESTATE, "no sensors set");
  if (s->latched) return fail(MONO_ESTATE, "simulation latched after a non-finite potential");
  st = prepare(s, dt);
  if (st != MONO_OK) return st;
  double* dbuf = nullptr;
  if (dalloc(&dbuf, (size_t)std::max<int64_t>(n_steps, 1) * s->ns))
    return fail(MONO_ENOMEM, "device allocation failed");
  if (s->prec == MONO_F64)
    sample_steps<double>(s, n_steps, dbuf);
  else
    sample_steps<float>(s, n_steps, dbuf);
  hipError_t e = hipGetLastError();
  if (!e) e = hipMemcpyAsync(out, dbuf, (size_t)n_steps * s->ns * 8, hipMemcpyDeviceToHost, s->stream);
  if (!e) e = hipStreamSynchronize(s->stream);
  dfree(dbuf);
  if (e) return fail(MONO_EDEVICE, hipGetErrorString(e));
  s->step += n_steps;
  return check_flag(s);
}

}  // extern "C"

namespace {
// Staging of mono_sample_sensors_noalloc: a file-scope device array (each GPU
// the library runs on holds its own copy until the process ends).  Host code
// never passes the array's name to a kernel or a copy: it takes the address
// of this device's copy from hipGetSymbolAddress once per device and uses
// that pointer.
constexpr int64_t kNoAllocSamples = (int64_t)1 << 19;   // doubles (4 MiB)
__device__ __align__(256) double scratch[kNoAllocSamples];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;   // per device ordinal, nullptr until looked up

// Address of the current device's copy of `scratch`.
hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

mono_status mono_sample_sensors_noalloc(mono_sim* s, int64_t n_steps, double dt, double* out) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (n_steps < 0 || (n_steps > 0 && !out)) return fail(MONO_EINVAL, "bad argument");
  if (s->ns <= 0) return fail(MONO_ESTATE, "no sensors set");
  if (n_steps * (int64_t)s->ns > kNoAllocSamples)
    return fail(MONO_EINVAL, "n_steps x sensors exceeds the 524288 samples of the static buffer");
  if (s->latched) return fail(MONO_ESTATE, "simulation latched after a non-finite potential");
  // a change of dt would rebuild the per-instance tables: not here
  if (s->dt != dt) return fail(MONO_ESTATE, "call mono_prepare with this dt first");
  double* buf = nullptr;
  HIP_TRY(scratch_address(&buf));
  // every sample slot of the n_steps x sensors written is set by the sample
  // kernel before it is copied, so nothing needs clearing
  if (s->prec == MONO_F64)
    sample_steps<double>(s, n_steps, buf);
  else
    sample_steps<float>(s, n_steps, buf);
  hipError_t e = hipGetLastError();
  if (!e && n_steps > 0)
    e = hipMemcpyAsync(out, buf, (size_t)n_steps * s->ns * 8, hipMemcpyDeviceToHost, s->stream);
  if (!e) e = hipStreamSynchronize(s->stream);
  if (e) return fail(MONO_EDEVICE, hipGetErrorString(e));
  s->step += n_steps;
  return check_flag(s);
}

mono_status mono_forward_taped(mono_sim* s, int64_t n_steps, double dt, int32_t ckpt_every,
                               double* loss) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (n_steps < 1 || ckpt_every < 1 || !loss) return fail(MONO_EINVAL, "bad argument");
  if (s->latched) return fail(MONO_ESTATE, "simulation latched after a non-finite potential");
  st = prepare(s, dt);
  if (st != MONO_OK) return st;
  if (s->k_max > kAdjMaxK) return fail(MONO_EUNSUPPORTED, "adjoint needs k_max <= 16");
  if (s->vclamp) return fail(MONO_EUNSUPPORTED, "adjoint with a clamped potential");
  HIP_TRY(hipStreamSynchronize(s->stream));
  free_tape(s);
  const int64_t C = std::min<int64_t>(ckpt_every, n_steps);
  const int64_t nck = (n_steps + C - 1) / C;
  int64_t nslots = nck;
  if (s->ckpt_schedule == MONO_CKPT_BINOMIAL) {
    nslots = std::min<int64_t>(s->ckpt_max_slots, nck);
    if (!make_ckpt_plan(nck, (int)nslots, s->plan))
      return fail(MONO_EUNSUPPORTED, "no binomial plan for this many segments and snapshots");
  }
  const size_t snap = snapshot_bytes(s);
  const size_t nblk = (size_t)((s->n + 255) / 256);
  s->d_ckpt.assign(nslots, nullptr);
  bool ok = true;
  for (int64_t c = 0; c < nslots && ok; ++c) ok = !dalloc((char**)&s->d_ckpt[c], snap);
  ok = ok && !dalloc((char**)&s->d_final, snap) &&
       !dalloc((char**)&s->d_seg_vsub, (size_t)C * 2 * s->l_max * s->Np * s->es) &&
       !dalloc((char**)&s->d_seg_entry, (size_t)C * s->S * s->Np * s->es) &&
       !dalloc(&s->d_seg_k, (size_t)C * s->n) && !dalloc(&s->d_base_rev, 1) &&
       !dalloc((char**)&s->d_lam, (size_t)s->S * s->Np * s->es) &&
       !dalloc((char**)&s->d_lamV2, s->Np * s->es) && !dalloc(&s->d_gsig, s->Np) &&
       !dalloc(&s->d_gpart, nblk * kMaxParams) && !dalloc(&s->d_loss_steps, n_steps);
  if (!ok) {
    free_tape(s);
    return fail(MONO_ENOMEM, "not enough device memory for the checkpoints and tape");
  }
  // the uniform schedule's second segment tape (overlapped recompute); without
  // the memory for it the segments are reversed one after the other
  if (s->ckpt_schedule == MONO_CKPT_UNIFORM && nck > 1 &&
      (dalloc((char**)&s->d_seg_vsub2, (size_t)C * 2 * s->l_max * s->Np * s->es) ||
       dalloc((char**)&s->d_seg_entry2, (size_t)C * s->S * s->Np * s->es) ||
       dalloc(&s->d_seg_k2, (size_t)C * s->n))) {
    dfree(s->d_seg_vsub2);
    dfree(s->d_seg_entry2);
    dfree(s->d_seg_k2);
    (void)hipGetLastError();
  }
  HIP_TRY(hipMemsetAsync(s->d_loss_steps, 0, n_steps * 8, s->stream));
  s->ckpt_every = (int)C;
  s->tape_step0 = s->step;
  s->tape_steps = n_steps;
  st = s->prec == MONO_F64 ? forward_taped_t<double>(s, n_steps, loss)
                           : forward_taped_t<float>(s, n_steps, loss);
  if (st != MONO_OK) return st;
  s->taped = true;
  return check_flag(s);
}

mono_status mono_set_checkpointing(mono_sim* s, int32_t schedule, int32_t max_snapshots) {
  if (!s) return fail(MONO_EINVAL, "NULL simulation");
  if (schedule == MONO_CKPT_UNIFORM) {
    s->ckpt_schedule = schedule;
    s->ckpt_max_slots = 0;
    return MONO_OK;
  }
  if (schedule != MONO_CKPT_BINOMIAL || max_snapshots < 2)
    return fail(MONO_EINVAL, "schedule must be uniform, or binomial with at least 2 snapshots");
  s->ckpt_schedule = schedule;
  s->ckpt_max_slots = max_snapshots;
  return MONO_OK;
}

mono_status mono_checkpoint_info(mono_sim* s, int64_t* out) {
  if (!s || !out) return fail(MONO_EINVAL, "NULL argument");
  if (!s->taped) return fail(MONO_ESTATE, "call mono_forward_taped first");
  const int64_t C = s->ckpt_every;
  const int L = s->l_max;
  out[0] = s->ckpt_schedule;
  out[1] = (int64_t)s->d_ckpt.size();
  out[2] = (s->tape_steps + C - 1) / C;
  out[3] = s->ckpt_advances;
  out[4] = (int64_t)(s->d_ckpt.size() * snapshot_bytes(s));
  out[5] = (int64_t)((s->d_seg_vsub2 ? 2 : 1) *
                     ((size_t)C * (2 * L + s->S) * s->Np * s->es + (size_t)C * s->n));
  return MONO_OK;
}

mono_status mono_checkpoint_plan(int64_t n_segments, int32_t max_snapshots, int64_t* advances) {
  if (!advances || n_segments < 1) return fail(MONO_EINVAL, "bad argument");
  CkptPlan p;
  const int64_t slots = std::min<int64_t>(max_snapshots, n_segments);
  if (!make_ckpt_plan(n_segments, (int)slots, p))
    return fail(MONO_EINVAL, "no plan (fewer than 2 snapshots, or too large a table)");
  *advances = p.advances();
  return MONO_OK;
}

mono_status mono_backward(mono_sim* s, double* grad_sigma, double* grad_params) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (!s->taped) return fail(MONO_ESTATE, "call mono_forward_taped first");
  if (s->step != s->tape_step0 + s->tape_steps)
    return fail(MONO_ESTATE, "the simulation moved since the taped run");
  const size_t nblk = (size_t)((s->n + 255) / 256);
  HIP_TRY(hipMemsetAsync(s->d_lam, 0, (size_t)s->S * s->Np * s->es, s->stream));
  HIP_TRY(hipMemsetAsync(s->d_lamV2, 0, s->Np * s->es, s->stream));
  HIP_TRY(hipMemsetAsync(s->d_gsig, 0, s->Np * 8, s->stream));
  HIP_TRY(hipMemsetAsync(s->d_gpart, 0, nblk * kMaxParams * 8, s->stream));
  st = s->prec == MONO_F64 ? backward_t<double>(s) : backward_t<float>(s);
  if (st != MONO_OK) return st;
  if (grad_sigma)
    HIP_TRY(hipMemcpy(grad_sigma, s->d_gsig, s->n * 8, hipMemcpyDeviceToHost));
  if (grad_params) {
    std::vector<double> gp(nblk * kMaxParams);
    HIP_TRY(hipMemcpy(gp.data(), s->d_gpart, gp.size() * 8, hipMemcpyDeviceToHost));
    for (int b = 0; b < s->Pm; ++b) {
      double acc = 0.0;
      for (size_t q = 0; q < nblk; ++q) acc += gp[q * kMaxParams + b];
      grad_params[b] = acc;
    }
  }
  return check_flag(s);
}

mono_status mono_set_param_scalings(mono_sim* s, int32_t n, const int32_t* rows,
                                    const double* scalings) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (n < 1 || n > s->Pm || !rows || !scalings) return fail(MONO_EINVAL, "bad argument");
  if (s->scal_n >= 0)
    return fail(MONO_ESTATE, "scalings already set since the last mono_set_cell_model");
  const bool label6 = s->model == MONO_MODEL_TP06_TYPES || s->model == MONO_MODEL_TP06_FIBRO;
  for (int j = 0; j < n; ++j) {
    if (rows[j] < 0 || rows[j] >= s->Pm) return fail(MONO_EINVAL, "parameter row out of range");
    if (label6 && rows[j] == 6) return fail(MONO_EINVAL, "the type / class row is a label");
    for (int k = 0; k < j; ++k)
      if (rows[k] == rows[j]) return fail(MONO_EINVAL, "repeated parameter row");
  }
  hipPointerAttribute_t attr{};
  if (hipPointerGetAttributes(&attr, scalings) != hipSuccess ||
      attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(MONO_EINVAL, "scalings must be device memory");
  }
  double c[kMaxParams];
  HIP_TRY(hipMemcpyAsync(c, scalings, (size_t)n * 8, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (int j = 0; j < n; ++j)
    if (!std::isfinite(c[j]) || c[j] == 0.0)
      return fail(MONO_EINVAL, "scalings must be finite and nonzero");
  for (int j = 0; j < n; ++j) {
    const int a = rows[j];
    if (s->par_pernode >> a & 1u) {
      if (s->prec == MONO_F64)
        launch_scale_row<double>((double*)s->d_par + (size_t)a * s->Np, s->n, c[j], s->stream);
      else
        launch_scale_row<float>((float*)s->d_par + (size_t)a * s->Np, s->n, (float)c[j],
                                s->stream);
    } else {
      s->par_uniform[a] *= c[j];
    }
    s->scal_rows[j] = a;
    s->scal_vals[j] = c[j];
  }
  HIP_TRY(hipGetLastError());
  s->scal_n = n;
  drop_graph(s);
  return MONO_OK;
}

mono_status mono_forward_taped_device(mono_sim* s, int64_t n_steps, double dt, int32_t ckpt_every,
                                      double* loss) {
  if (!s || !loss) return fail(MONO_EINVAL, "NULL argument");
  double L = 0.0;
  mono_status st = mono_forward_taped(s, n_steps, dt, ckpt_every, &L);
  if (st != MONO_OK) return st;
  // the per-step losses summed on the device in the host's order
  OrderedSums a{};
  a.count = 1;
  a.col[0] = 0;
  a.div[0] = 1.0;
  launch_ordered_sums(s->d_loss_steps, s->tape_steps, 1, a, loss, s->stream);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s->stream));
  return MONO_OK;
}

mono_status mono_backward_device(mono_sim* s, double* grad_sigma, double* grad_scalings) {
  mono_status st = require_model(s);
  if (st != MONO_OK) return st;
  if (grad_scalings && s->scal_n < 0)
    return fail(MONO_ESTATE, "no scalings set (mono_set_param_scalings)");
  st = mono_backward(s, nullptr, nullptr);
  if (st != MONO_OK) return st;
  if (grad_sigma)
    HIP_TRY(hipMemcpyAsync(grad_sigma, s->d_gsig, s->n * 8, hipMemcpyDeviceToDevice, s->stream));
  if (grad_scalings) {
    // per-workgroup partial sums reduced in the order mono_backward uses,
    // then the chain rule through p = c base
    OrderedSums a{};
    a.count = s->scal_n;
    for (int j = 0; j < s->scal_n; ++j) {
      a.col[j] = s->scal_rows[j];
      a.div[j] = s->scal_vals[j];
    }
    launch_ordered_sums(s->d_gpart, (s->n + 255) / 256, kMaxParams, a, grad_scalings, s->stream);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  return MONO_OK;
}

mono_status mono_set_launch(mono_sim* s, const mono_launch* c) {
  if (!s || !c) return fail(MONO_EINVAL, "NULL argument");
  auto okb = [](int b) { return b == 128 || b == 256 || b == 512; };
  const int maxr = s->prec == MONO_F32 ? 4 : 2;
  if (!okb(c->diff_block) ||
      !(okb(c->react_block) || (c->react_block == 1024 && s->prec == MONO_F32)))
    return fail(MONO_EINVAL, "block sizes must be 128, 256 or 512 (FP32 reaction: also 1024)");
  const int r = c->diff_rows_per_lane;
  const bool by_class = s->layout == MONO_LAYOUT_STENCIL && s->n_classes > 0 && c->diff_classes;
  if (by_class) {
    if (!(r == 1 || r == 2 || r == 4 || r == 8 || r == 16))
      return fail(MONO_EINVAL, "rows per lane must be 1, 2, 4, 8 or 16");
  } else if (!(r == 1 || r == 2 || r == 4) || r > maxr) {
    return fail(MONO_EINVAL, "rows per lane must be 1, 2 or 4 (FP64: 1 or 2)");
  }
  if (c->diff_xcd_remap < 0 || c->diff_xcd_remap > 1) return fail(MONO_EINVAL, "bad remap flag");
  if (c->graph_steps < 1 || c->graph_steps > 8192)
    return fail(MONO_EINVAL, "graph_steps must be in 1..8192");
  if (c->react_sort < 0 || c->react_sort > 1) return fail(MONO_EINVAL, "bad sort flag");
  if (c->diff_classes < 0 || c->diff_classes > 1) return fail(MONO_EINVAL, "bad classes flag");
  if (c->diff_wave_rows < 0 || c->diff_wave_rows > 1) return fail(MONO_EINVAL, "bad rows flag");
  if (c->diff_fuse < 0 || c->diff_fuse > 1) return fail(MONO_EINVAL, "bad fuse flag");
  if (c->diff_fuse_planes < 0 || c->diff_fuse_planes > 4096)
    return fail(MONO_EINVAL, "diff_fuse_planes must be in 0..4096");
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->lc.diff_block = c->diff_block;
  s->lc.diff_rpl = c->diff_rows_per_lane;
  s->lc.diff_xcd = c->diff_xcd_remap;
  s->lc.react_block = c->react_block;
  s->lc.graph_steps = c->graph_steps;
  s->lc.react_sort = c->react_sort;
  s->lc.diff_classes = c->diff_classes;
  s->lc.diff_wave_rows = c->diff_wave_rows;
  s->lc.diff_fuse = c->diff_fuse;
  s->lc.diff_fuse_planes = c->diff_fuse_planes;
  drop_graph(s);
  return MONO_OK;
}

mono_status mono_get_launch(mono_sim* s, mono_launch* c) {
  if (!s || !c) return fail(MONO_EINVAL, "NULL argument");
  c->diff_block = s->lc.diff_block;
  c->diff_rows_per_lane = s->lc.diff_rpl;
  c->diff_xcd_remap = s->lc.diff_xcd;
  c->react_block = s->lc.react_block;
  c->graph_steps = s->lc.graph_steps;
  c->react_sort = s->lc.react_sort;
  c->diff_classes = s->lc.diff_classes;
  c->diff_wave_rows = s->lc.diff_wave_rows;
  c->diff_fuse = s->lc.diff_fuse;
  c->diff_fuse_planes = s->lc.diff_fuse_planes;
  return MONO_OK;
}

mono_status mono_set_stream(mono_sim* s, void* stream) {
  if (!s || !stream) return fail(MONO_EINVAL, "bad argument");
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (s->own_stream) HIP_TRY(hipStreamDestroy(s->stream));
  s->own_stream = false;
  s->stream = (hipStream_t)stream;
  return MONO_OK;
}

mono_status mono_sync(mono_sim* s) {
  if (!s) return fail(MONO_EINVAL, "NULL simulation");
  HIP_TRY(hipStreamSynchronize(s->stream));
  return check_flag(s);
}

mono_status mono_debug(mono_sim* s, int32_t what, void* arg) {
  if (!s) return fail(MONO_EINVAL, "NULL simulation");
  switch (what) {
    case MONO_DEBUG_KTRACE: {
      if (!arg) return fail(MONO_EINVAL, "NULL argument");
      const mono_ktrace* k = (const mono_ktrace*)arg;
      if (k->mode < 0 || k->mode > 3 || ((k->mode & 1) && !k->record) ||
          ((k->mode & 2) && !k->replay) || (k->mode && k->n_steps < 0))
        return fail(MONO_EINVAL, "bad k-trace description");
      s->kt.mode = k->mode;
      s->kt.rec = k->record;
      s->kt.rep = k->replay;
      s->kt.rec_base = s->kt.rep_base = k->base_step;
      s->kt.rec_steps = s->kt.rep_steps = k->mode ? k->n_steps : 0;
      drop_graph(s);
      return MONO_OK;
    }
    case MONO_DEBUG_VCLAMP:
      if (!arg) return fail(MONO_EINVAL, "NULL argument");
      s->vclamp = *(const int32_t*)arg ? 1 : 0;
      drop_graph(s);
      return MONO_OK;
    case MONO_DEBUG_FORCE_L: {
      if (!arg || *(const int32_t*)arg < 0) return fail(MONO_EINVAL, "bad argument");
      s->force_l = *(const int32_t*)arg;
      if (s->dt > 0.0) {
        const double dt = s->dt;
        s->dt = -1.0;
        return prepare(s, dt);
      }
      return MONO_OK;
    }
    case MONO_DEBUG_STATS_ENABLE: {
      if (!arg) return fail(MONO_EINVAL, "NULL argument");
      const bool on = *(const int32_t*)arg != 0;
      if (on && !s->d_stats && dalloc(&s->d_stats, 64)) return fail(MONO_ENOMEM, "allocation failed");
      if (on) {
        HIP_TRY(hipStreamSynchronize(s->stream));
        HIP_TRY(hipMemsetAsync(s->d_stats, 0, 64 * sizeof(unsigned long long), s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
      }
      s->stats_on = on;
      drop_graph(s);
      return MONO_OK;
    }
    case MONO_DEBUG_STATS: {
      if (!arg) return fail(MONO_EINVAL, "NULL argument");
      int64_t* o = (int64_t*)arg;
      if (!s->d_stats) {
        std::memset(o, 0, 4 * sizeof(int64_t));
        return MONO_OK;
      }
      HIP_TRY(hipStreamSynchronize(s->stream));
      unsigned long long h[64];
      HIP_TRY(hipMemcpy(h, s->d_stats, sizeof(h), hipMemcpyDeviceToHost));
      for (int q = 0; q < 4; ++q) o[q] = (int64_t)h[q * 16];
      return MONO_OK;
    }
    case MONO_DEBUG_KTIMES: {
      if (!arg) return fail(MONO_EINVAL, "NULL argument");
      double* o = (double*)arg;
      const bool reset = o[4] != 0.0;
      o[0] = s->ktime_ms[0];
      o[1] = (double)s->klaunches[0];
      o[2] = s->ktime_ms[1];
      o[3] = (double)s->klaunches[1];
      if (reset) {
        s->ktime_ms[0] = s->ktime_ms[1] = 0.0;
        s->klaunches[0] = s->klaunches[1] = 0;
      }
      return MONO_OK;
    }
    case MONO_DEBUG_TIME_DIFFUSION: {
      if (!arg) return fail(MONO_EINVAL, "NULL argument");
      double* o = (double*)arg;
      const int64_t R = (int64_t)o[0];
      if (R < 2 || R % 2 || R > 100000) return fail(MONO_EINVAL, "R must be even, 2..100000");
      const mono_status ms = require_model(s);
      if (ms != MONO_OK) return ms;
      if (s->dt <= 0.0) return fail(MONO_ESTATE, "call mono_prepare first");
      HIP_TRY(hipStreamSynchronize(s->stream));
      return time_diffusion(s, R, o[1]);
    }
    default:
      return fail(MONO_EINVAL, "unknown debug request");
  }
}

}  // extern "C"
