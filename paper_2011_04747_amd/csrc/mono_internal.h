// Internal declarations of libmono (host runtime <-> HIP kernels).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mono.h"

namespace mono {

// FP64 product and sum with one rounding each: never fused into an FMA (HIP
// compiles with contraction on, and the _rn intrinsics are plain operators).
__host__ __device__ __forceinline__ double rn_mul(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}
__host__ __device__ __forceinline__ double rn_add(double a, double b) {
#pragma clang fp contract(off)
  return a + b;
}

// Per-kernel timing of eager steps: when set, the next step kernel is launched
// with a start and a stop event that the command processor records at the
// kernel's own begin and end (no event packets between kernels), then cleared.
struct KernelTimer {
  hipEvent_t start, stop;
};
extern thread_local KernelTimer* g_ktimer;

template <typename F, typename... A>
void launch_step_kernel(F kernel, dim3 grid, dim3 block, hipStream_t s, A... args) {
  if (KernelTimer* t = g_ktimer) {
    g_ktimer = nullptr;
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, t->start, t->stop, 0, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
  }
}

constexpr int kBlock = 256;        // threads per workgroup (4 wavefronts of 64)
constexpr int kMaxStim = 8;        // stimuli per simulation
constexpr int kMaxOffsets = 13;    // positive stencil offsets (27-point hex stencil)
constexpr int kMaxParams = 10;
constexpr int kMaxStates = 19;

// ---------------------------------------------------------------------------
// host-side FE assembly (assembly.cpp)
// ---------------------------------------------------------------------------
struct HostCSR {
  int64_t n = 0;
  std::vector<int64_t> rp;    // n + 1
  std::vector<int32_t> col;   // sorted per row, includes the diagonal
  std::vector<double> val;    // K entries
  std::vector<double> mass;   // row-sum lumped mass
};

// Assemble K (with per-node conductivity scaling) and the lumped mass.
// Returns 0 or a MONO_E* code with a message in err.
int assemble_fe(const mono_mesh_desc* d, HostCSR& K, std::string& err);

struct EllHost {
  int width = 0;
  std::vector<int32_t> col;   // width * Np, slot-major
  std::vector<double> val;    // a_ij = -k_ij / m_i
};
void build_ell(const HostCSR& K, int64_t Np, EllHost& out);

struct StencilHost {
  int P = 0;                   // offsets per instance (padded)
  std::vector<int32_t> off;    // n_inst * P positive offsets
  std::vector<double> e;       // P * Np, e[p][i] = -k(i, i + off_p) or 0
  std::vector<double> minv;    // Np, 1 / m_i
};
// Returns false when some instance needs more than kMaxOffsets offsets.
bool build_stencil(const HostCSR& K, const std::vector<int64_t>& inst_off, int64_t Np,
                   StencilHost& out);

// Rows of a single-instance stencil that repeat exactly: row i is represented
// by class cls[i], a table row holding its P forward weights e[p][i], its P
// backward weights e[p][i - off_p] (0 where that neighbour is absent) and 1/m_i,
// compared after rounding to the simulation precision.  Structured meshes with
// piecewise-uniform conductivity have few classes (boundary type x material).
struct RowClasses {
  int tw = 0;                    // table row width: 2P + 1, padded to even
  int n_classes = 0;
  std::vector<uint16_t> cls;     // Np
  std::vector<double> table;     // n_classes * tw, values exact in the precision
};
// Returns false (no compression) for several instances or when the rows do not
// repeat enough: more than max_classes classes or more than Np / 8.
bool build_row_classes(const StencilHost& sh, int64_t n, int64_t Np, bool fp32,
                       int max_classes, RowClasses& out);

// ---------------------------------------------------------------------------
// kernel argument blocks
// ---------------------------------------------------------------------------
// Launch shapes chosen per simulation (by the autotuner or the caller).
struct LaunchCfg {
  int diff_block = 256;   // 128, 256 or 512 lanes per workgroup
  int diff_rpl = 1;       // stencil rows per lane: 1, 2 or 4 (FP32 only)
  int diff_xcd = 1;       // deal row ranges to XCDs
  int react_block = 256;  // 128, 256 or 512
  int graph_steps = 32;   // outer steps per captured HIP graph
  int react_sort = 0;     // reaction nodes ordered by k within a workgroup
  int diff_classes = 1;   // diffusion from row classes when the mesh has them
  int diff_wave_rows = 1; // class diffusion sharing neighbour rows across lanes
  int diff_fuse = 0;      // up to 4 substeps of a half step per launch (3D grids)
  int diff_fuse_planes = 0;  // z planes per workgroup of the fused kernel, 0 = auto
};

// keys of the in-workgroup ordering of the reaction by k: k = 0..kSortMaxK-1
// each, and every k >= kSortMaxK the last key
constexpr int kSortMaxK = 16;

// rows produced per wavefront by the row-sharing diffusion (lanes 1..62; lanes
// 0 and 63 hold the neighbouring rows)
constexpr int kWaveRows = 62;
// fused half-step diffusion (structured 3D grids): wavefronts (y rows) per
// workgroup and the tiling of the grid
constexpr int kFusedRows = 16;
struct FusedGeom {
  int nx, ny, nz;      // grid
  int ty, tz;          // y rows and z planes each workgroup produces
  int nxs, nys, nzs;   // workgroups along x, y and z
};
constexpr int32_t kNoClass = -1;

struct StimTable {
  int n;
  double t_on[kMaxStim];
  double t_end[kMaxStim];
  double amp[kMaxStim];
  // Single instance: with L > 0 substeps per half step, stimulus s is open
  // on the substeps q = (2 step + half) L + m with q_on[s] <= q < q_end[s],
  // which are exactly those whose start time tau (below) lies in
  // [t_on, t_end); L = 0 leaves the test to tau.
  int L;
  int64_t q_on[kMaxStim];
  int64_t q_end[kMaxStim];
};

struct StepClock {
  const int64_t* base;   // device: index of the first step of this launch sequence
  int64_t g;             // offset of this step within the sequence
  double dt;
};

template <typename T>
struct DiffArgs {
  int64_t n, Np;
  const T* Vin;
  T* Vout;
  // ELL
  int W;
  const int32_t* col;
  const T* val;
  // STENCIL
  int P;
  const T* e;
  const T* minv;
  const int32_t* off;        // n_inst * P
  // STENCIL rows by class (single instance): table row = P forward weights,
  // P backward weights, 1/m
  const uint16_t* cls;       // per row, or nullptr
  const T* ctab;
  int tw;
  const int32_t* wcls;       // grid-row stencils: class of each wavefront's
                             // kWaveRows rows, or kNoClass; nullptr otherwise
  int nx, nxy;               // grid-row stencils: offsets of the y and z rows
  // instances
  const int32_t* inst;       // per node, or nullptr for a single instance
  const int64_t* inst_off;   // n_inst + 1 first nodes of the instances
  const int32_t* l;          // per instance substep counts
  const double* dt_ad;       // per instance
  // stimulus
  const uint8_t* stim_mask;  // per node bit set, or nullptr
  StimTable stim;
  // time of this substep: tau = step*dt (+ dt/2 for the second half) + m*dt_ad
  StepClock clk;
  int half;
  int m;
  int xcd;                   // remap workgroups to contiguous rows per XCD
};

struct KTraceArgs {
  int mode;                  // bit 0 record, bit 1 replay
  uint8_t* rec;              // row (step - rec_base), or row g if rec_rel, n values per row
  int rec_rel;               // record rows by clock offset g (graph-replayed segments)
  const uint8_t* rep;        // row (step - rep_base)
  int64_t rec_base, rec_steps;
  int64_t rep_base, rep_steps;
};

template <typename T>
struct IonArgs {
  int64_t n, Np;
  T* V;                      // potential in (and out unless Vout is set)
  T* Vout;                   // potential out, or nullptr (in place)
  T* tape_st;                // if set: (S - 1) * Np copy of the entry states
  T* st;                     // (S - 1) * Np
  T* vprev;
  double* lat;
  uint8_t* lastk;
  const T* par;              // per-node parameter rows (P * Np) where non-uniform
  T par_uniform[kMaxParams];
  uint32_t par_pernode;      // bit a set: row a is per node
  StepClock clk;
  int k_max;
  double lat_thr;
  int dvdt_src;
  int vclamp;
  KTraceArgs kt;
  int* flag;                 // non-finite latch
  unsigned long long* stats; // 4 counters or nullptr
  double* apd;               // APD90 trackers (rows of Np: upstroke time,
                             // largest slope, V_max, V_rest, repolarisation
                             // time) or nullptr
  int off32;                 // every state, parameter and tape row starts
                             // below 4 GiB from its array (32-bit offsets)
};

// ---------------------------------------------------------------------------
// launchers (kernels_*.hip)
// ---------------------------------------------------------------------------
// adjoint of one diffusion substep (kernels_adjoint.hip)
constexpr int kAdjMaxK = 16;   // largest k the adjoint reaction kernel replays
template <typename T>
struct AdjDiffArgs {
  int64_t n, Np;
  const T* lam_in;           // adjoint of the substep output
  T* lam_out;                // adjoint of the substep input
  const T* V;                // forward input of the substep
  const T* minv;
  const T* sigma;
  int W;
  const int32_t* col;
  const T* val;
  int P;
  const T* e;
  const int32_t* off;
  const int32_t* inst;
  const int64_t* inst_off;
  const int32_t* l;
  const double* dt_ad;
  int m;
  double* gsig;              // += dL/dsigma (FP64)
  // grid-row stencils with row classes (single instance): class table and
  // per-wavefront classes as in DiffArgs, or wcls = nullptr
  const uint16_t* cls;
  const T* ctab;
  int tw;
  const int32_t* wcls;
  int nx, nxy;
  int iter;                  // row groups per wavefront (1 or 2)
  int sig_uni;               // every sigma equals sig_val (no sigma loads)
  T sig_val;
};
template <typename T>
struct AdjIonArgs {
  int64_t n, Np;
  const T* entry;            // S x Np reaction-entry state
  const uint8_t* k;          // n substep counts
  T* lam;                    // S x Np adjoint of the states (row 0 unused)
  T* lamV;                   // Np adjoint of V
  const T* par;
  T par_uniform[kMaxParams];
  uint32_t par_pernode;
  double dt;
  double* gpart;             // per workgroup kMaxParams FP64 partial sums
  int sort;                  // take each workgroup's nodes in order of k
  // loss gradient at reaction entry, added to the adjoint of V where a node
  // is a sensor: sens_of[i] = its sensor index or -1 (nullptr: no sensors)
  const int32_t* sens_of;
  const double* target;      // target_steps x ns
  int ns;
  int64_t target_steps;
  StepClock clk;
};
template <typename T>
void launch_adj_diffusion(int layout, const AdjDiffArgs<T>& a, hipStream_t s);
template <typename T>
void launch_adj_ionic(int model, const AdjIonArgs<T>& a, hipStream_t s);
// sensors of the adjoint loss; the target row and the output slot follow the
// device clock (step = *clk.base + clk.g), so graphs replay them correctly
struct SensorArgs {
  const int32_t* sens;
  int ns;
  const double* target;      // target_steps x ns
  int64_t target_steps;      // steps at or past this have no target (no loss)
  StepClock clk;
  double* out;               // loss of step s goes to out[s - out_base]
  int64_t out_base;
};
template <typename T>
void launch_sensor_loss(const T* V, const SensorArgs& a, hipStream_t s);
// one parameter row scaled in place
template <typename T>
void launch_scale_row(T* x, int64_t n, T c, hipStream_t s);
// out[j] = (sum_{q < n} x[q * stride + col[j]], in order) / div[j]
struct OrderedSums {
  int count;
  int col[kMaxParams];
  double div[kMaxParams];
};
void launch_ordered_sums(const double* x, int64_t n, int stride, const OrderedSums& a,
                         double* out, hipStream_t s);
template <typename T>
void launch_sensor_sample(const T* V, const int32_t* sens, int ns, double* out, hipStream_t s);

template <typename T>
void launch_diffusion(int layout, const DiffArgs<T>& a, const LaunchCfg& c, hipStream_t s);
// L = 2..4 substeps a.m .. a.m+L-1 of a half step in one launch (3D grid
// stencils that the host admitted); Vin and Vout must differ.
template <typename T>
void launch_diffusion_fused(const DiffArgs<T>& a, int L, const FusedGeom& g, hipStream_t s);

template <typename T>
void launch_ionic(int model, const IonArgs<T>& a, const LaunchCfg& c, hipStream_t s);

void launch_advance_clock(int64_t* base, int64_t by, hipStream_t s);
void launch_set_clock(int64_t* base, int64_t to, hipStream_t s);

// Gershgorin rows in FP64 on CSR: r_i = m_i/(k_ii + sum|k_ij|), g_i = 1/r_i,
// then per-instance min r and max g.
void launch_gershgorin(int64_t n, const int64_t* rp, const int32_t* col, const double* val,
                       const double* mass, double* r, double* g, hipStream_t s);
void launch_segmented_minmax(int n_inst, const int64_t* inst_off, const double* r,
                             const double* g, double* rmin, double* gmax, hipStream_t s);

// power iteration helpers (FP64, CSR)
void launch_spmv_csr(int64_t n, const int64_t* rp, const int32_t* col, const double* val,
                     const double* x, double* y, hipStream_t s);
void launch_segmented_dots(int n_inst, const int64_t* inst_off, const double* x,
                           const double* kx, const double* mass, double* xkx, double* xmx,
                           hipStream_t s);
void launch_power_update(int64_t n, const int32_t* inst, const double* kx, const double* mass,
                         const double* xmx, double* x, hipStream_t s);
void launch_power_init(int64_t n, double* x, hipStream_t s);

template <typename T>
void launch_convert(int64_t n, const T* src, double* dst, hipStream_t s);
template <typename T>
void launch_convert_from(int64_t n, const double* src, T* dst, hipStream_t s);

}  // namespace mono
