// Adjoint kernels of the split step: the gradient of a sensor-mismatch loss
// with respect to per-node conductivity scales and the cell-model parameter
// rows, by reverse sweeps over a taped forward run.
//
// Diffusion substep (forward, difference form):
//   V'_i = V_i + dt_ad ( (1/m_i) sum_j e_ij (V_j - V_i) + s_i ),  e = -K.
// Its reverse with u = lam'/m:
//   lam_i = lam'_i + dt_ad sum_j e_ij (u_j - u_i)              (K symmetric)
//   dL/dsigma_i += dt_ad sum_j e_ij/(sigma_i + sigma_j) (u_i - u_j)(V_j - V_i)
// because e_ij = e0_ij (sigma_i + sigma_j)/2 off the diagonal.
// Reaction: every node replays its k substeps from the taped entry state into
// private memory and applies the hand-written reverse substep backwards.
#include "cell_models.h"
#include "cell_models_adjoint.h"
#include "grid_rows.h"
#include "mono_internal.h"
#include "wg_sort.h"

namespace mono {

// --- loss at reaction entry -------------------------------------------------
// out = sum_q (V[sensor_q] - target_q)^2 in FP64 (one workgroup)
template <typename T>
__global__ __launch_bounds__(256) void k_sensor_loss(const T* V, SensorArgs a) {
  const int64_t step = *a.clk.base + a.clk.g;
  const bool on = step < a.target_steps;
  const double* target = a.target + step * a.ns;
  __shared__ double part[4];
  double acc = 0.0;
  if (on)
    for (int q = threadIdx.x; q < a.ns; q += 256) {
      const double e = (double)V[a.sens[q]] - target[q];
      acc += e * e;
    }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) a.out[step - a.out_base] = part[0] + part[1] + part[2] + part[3];
}

// out[q] = V[sensor_q] (FP64)
template <typename T>
__global__ __launch_bounds__(256) void k_sensor_sample(const T* V, const int32_t* sens, int ns,
                                                       double* out) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q < ns) out[q] = (double)V[sens[q]];
}

// --- adjoint diffusion substep ------------------------------------------------
template <typename T, bool BATCHED>
__global__ __launch_bounds__(256) void k_adj_diff_stencil(AdjDiffArgs<T> a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  const int q = BATCHED ? a.inst[i] : 0;
  const T li = a.lam_in[i];
  if (BATCHED && a.m >= a.l[q]) {
    a.lam_out[i] = li;
    return;
  }
  const int np = a.P;
  const int64_t last = a.n - 1;
  const int64_t first = BATCHED ? a.inst_off[q] : 0;
  const T ui = li * a.minv[i];
  const T vi = a.V[i];
  const T si = a.sigma[i];
  T acc = T(0), gs = T(0);
  for (int p = 0; p < np; ++p) {
    const int64_t o = a.off[(int64_t)q * np + p];
    const int64_t jf = i + o;
    const int64_t jb = i - o;
    const int64_t jfc = jf <= last ? jf : last;
    const int64_t jbc = jb >= first ? jb : first;
    const T wf = a.e[(int64_t)p * a.Np + i];
    const T wbl = a.e[(int64_t)p * a.Np + jbc];   // jbc is a row of this instance
    const T wb = (jb >= first) ? wbl : T(0);
    const T uf = a.lam_in[jfc] * a.minv[jfc];
    const T ub = a.lam_in[jbc] * a.minv[jbc];
    acc += wf * (uf - ui) + wb * (ub - ui);
    gs += wf * xrcp(si + a.sigma[jfc]) * (ui - uf) * (a.V[jfc] - vi);
    gs += wb * xrcp(si + a.sigma[jbc]) * (ui - ub) * (a.V[jbc] - vi);
  }
  const double dt_ad = a.dt_ad[q];
  a.lam_out[i] = li + (T)dt_ad * acc;
  a.gsig[i] += dt_ad * (double)gs;
}

// The same substep adjoint on a structured grid with row classes: a
// wavefront loads lambda, 1/m, V and sigma (unless uniform) of each
// neighbouring grid row once and passes x-neighbours between lanes
// (grid_rows.h); the edge weights come from the class table (scalar loads
// when the wavefront's rows share a class).  Each wavefront produces ITER
// consecutive groups of kWaveRows rows, loading all of them first.  Same
// arithmetic, in the same order, as k_adj_diff_stencil.
template <typename T, int P, int ITER, bool SIGU>
__global__ __launch_bounds__(256) void k_adj_diff_rows(AdjDiffArgs<T> a,
                                                       const T* __restrict__ ctab,
                                                       const int32_t* __restrict__ wcls) {
  using RP = RowPattern<P>;
  constexpr int NC = RP::NC;
  constexpr int WR = kWaveRows;
  constexpr int ES = (int)sizeof(T);
  const int n = (int)a.n;
  const int lane = threadIdx.x & 63;
  const int64_t ngroups = (a.n + WR - 1) / WR;
  const int64_t g0 =
      ((int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6)) * ITER;
  if (g0 >= ngroups) return;
  int ctr[NC];
  ctr[0] = 0;
  if constexpr (P == 4) {
    ctr[1] = a.nx;
    ctr[2] = -a.nx;
  } else if constexpr (P == 13) {
    ctr[1] = a.nx;
    ctr[2] = a.nxy - a.nx;
    ctr[3] = a.nxy;
    ctr[4] = a.nxy + a.nx;
    for (int k = 1; k < 5; ++k) ctr[4 + k] = -ctr[k];
  }
  T uc[ITER][NC], vc[ITER][NC], sc[ITER][NC], li[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int i = (int)((g0 + it) * WR) + lane - 1;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const uint32_t bj = (uint32_t)(min(max(i + ctr[k], 0), n - 1) * ES);
      const T lam = ld_bytes(a.lam_in, bj);
      if (k == 0) li[it] = lam;
      uc[it][k] = lam * ld_bytes(a.minv, bj);
      vc[it][k] = ld_bytes(a.V, bj);
      sc[it][k] = SIGU ? a.sig_val : ld_bytes(a.sigma, bj);
    }
  }
  const double dt_ad = a.dt_ad[0];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int64_t g = g0 + it;
    if (g >= ngroups) break;
    const int i = (int)(g * WR) + lane - 1;
    const bool produce = lane >= 1 && lane <= WR && i < n;
    // the x-neighbours are taken from the adjacent lanes where each is used,
    // so that only the row centres stay live through the sweep
    auto pick = [](const T* c, int k, int d) -> T {
      return d > 0 ? lane_shift<1>(c[k]) : (d < 0 ? lane_shift<-1>(c[k]) : c[k]);
    };
    auto pick_s = [&](int k, int d) -> T { return SIGU ? sc[it][k] : pick(sc[it], k, d); };
    const T ui = uc[it][0], vi = vc[it][0], si = sc[it][0];
    T acc = T(0), gs = T(0);
    auto sweep = [&](auto w) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        const int kf = RP::fk(p), df = RP::fd(p), kb = RP::bk(p), db = RP::bd(p);
        const T wf = w[p], wb = w[P + p];
        const T uf = pick(uc[it], kf, df), ub = pick(uc[it], kb, db);
        const T vf = pick(vc[it], kf, df), vb = pick(vc[it], kb, db);
        const T sf = pick_s(kf, df), sb = pick_s(kb, db);
        acc += wf * (uf - ui) + wb * (ub - ui);
        gs += wf * xrcp(si + sf) * (ui - uf) * (vf - vi);
        gs += wb * xrcp(si + sb) * (ui - ub) * (vb - vi);
      }
    };
    const int wc = wcls[g];
    if (wc != kNoClass) {
      using CT = const __attribute__((address_space(4))) T*;
      sweep((CT)(ctab + (uint32_t)(wc * a.tw)));
    } else {
      const int ic = min(max(i, 0), n - 1);
      sweep(ctab + (uint32_t)((int)a.cls[(uint32_t)ic] * a.tw));
    }
    if (produce) {
      a.lam_out[i] = li[it] + (T)dt_ad * acc;
      a.gsig[i] += dt_ad * (double)gs;
    }
  }
}

template <typename T, int P, int ITER>
static void launch_adj_rows_k(const AdjDiffArgs<T>& a, hipStream_t s) {
  const int64_t ngroups = (a.n + kWaveRows - 1) / kWaveRows;
  const dim3 grid((unsigned)((ngroups + 4 * ITER - 1) / (4 * ITER)));
  if (a.sig_uni)
    hipLaunchKernelGGL((k_adj_diff_rows<T, P, ITER, true>), grid, dim3(256), 0, s, a, a.ctab,
                       a.wcls);
  else
    hipLaunchKernelGGL((k_adj_diff_rows<T, P, ITER, false>), grid, dim3(256), 0, s, a, a.ctab,
                       a.wcls);
}
template <typename T, int P>
static void launch_adj_rows_p(const AdjDiffArgs<T>& a, hipStream_t s) {
  if (a.iter >= 2)
    launch_adj_rows_k<T, P, 2>(a, s);
  else
    launch_adj_rows_k<T, P, 1>(a, s);
}

// ELL stores a_ij = e_ij / m_i, so e_ij = a_ij / (1/m_i).
template <typename T, bool BATCHED>
__global__ __launch_bounds__(256) void k_adj_diff_ell(AdjDiffArgs<T> a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  const int q = BATCHED ? a.inst[i] : 0;
  const T li = a.lam_in[i];
  if (BATCHED && a.m >= a.l[q]) {
    a.lam_out[i] = li;
    return;
  }
  const T mi = a.minv[i];
  const T ui = li * mi;
  const T vi = a.V[i];
  const T si = a.sigma[i];
  const T rm = xrcp(mi);
  T acc = T(0), gs = T(0);
  for (int s = 0; s < a.W; ++s) {
    const int64_t k = (int64_t)s * a.Np + i;
    const int32_t j = a.col[k];
    const T e = a.val[k] * rm;
    const T uj = a.lam_in[j] * a.minv[j];
    acc += e * (uj - ui);
    gs += e * xrcp(si + a.sigma[j]) * (ui - uj) * (a.V[j] - vi);
  }
  const double dt_ad = a.dt_ad[q];
  a.lam_out[i] = li + (T)dt_ad * acc;
  a.gsig[i] += dt_ad * (double)gs;
}

template <typename T>
void launch_adj_diffusion(int layout, const AdjDiffArgs<T>& a, hipStream_t s) {
  if (a.n <= 0) return;
  const dim3 grid((unsigned)((a.n + 255) / 256));
  if (layout == MONO_LAYOUT_ELL) {
    if (a.inst)
      hipLaunchKernelGGL((k_adj_diff_ell<T, true>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_adj_diff_ell<T, false>), grid, dim3(256), 0, s, a);
  } else {
    if (a.wcls && !a.inst && (a.P == 1 || a.P == 4 || a.P == 13) &&
        a.n * (int64_t)sizeof(T) < (int64_t(1) << 31)) {
      if (a.P == 1)
        launch_adj_rows_p<T, 1>(a, s);
      else if (a.P == 4)
        launch_adj_rows_p<T, 4>(a, s);
      else
        launch_adj_rows_p<T, 13>(a, s);
      return;
    }
    if (a.inst)
      hipLaunchKernelGGL((k_adj_diff_stencil<T, true>), grid, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_adj_diff_stencil<T, false>), grid, dim3(256), 0, s, a);
  }
}

// --- adjoint reaction step ------------------------------------------------------
struct LinearAdj {
  template <typename T>
  __device__ static void vjp(const T* y, const T* p, T h, T* lam, T* gp) {
    linear_substep_vjp(y, p, h, false, lam, gp);
  }
};
struct MSAdj {
  template <typename T>
  __device__ static void vjp(const T* y, const T* p, T h, T* lam, T* gp) {
    ms_substep_vjp(y, p, h, false, lam, gp);
  }
};
struct TP06Adj {
  template <typename T>
  __device__ static void vjp(const T* y, const T* p, T h, T* lam, T* gp) {
    tp06_substep_vjp(y, p, h, false, lam, gp);
  }
};
struct TP06TypesAdj {
  template <typename T>
  __device__ static void vjp(const T* y, const T* p, T h, T* lam, T* gp) {
    tp06_types_substep_vjp(y, p, h, false, lam, gp);
  }
};
// The myocyte/fibroblast VJP is a call, not inlined: inlined into the
// unsorted FP64 kernel (some 430 registers, accumulation registers used as
// spill space) it returned wrong parameter gradients while the sorted
// instantiation and this out-of-line form match the FP64 oracle adjoint to
// rounding (tested for both orders and precisions).
template <typename T>
__device__ __noinline__ void fibro_vjp_call(const T* y, const T* p, T h, T* lam, T* gp) {
  tp06_fibro_substep_vjp(y, p, h, false, lam, gp);
}
struct TP06FibroAdj {
  template <typename T>
  __device__ static void vjp(const T* y, const T* p, T h, T* lam, T* gp) {
    fibro_vjp_call(y, p, h, lam, gp);
  }
};

// SORT: the workgroup's nodes are taken in order of their substep count k
// (wg_sort.h), so a wavefront replays and reverses one k where it can; the
// per-node arithmetic is unchanged (only the order of the FP64 workgroup sum
// of the parameter gradients differs).
template <typename T, class M, class A, bool SORT>
__global__ __launch_bounds__(256) void k_adj_ionic(AdjIonArgs<T> a) {
  const int64_t b0 = (int64_t)blockIdx.x * 256;
  int64_t i = b0 + threadIdx.x;
  bool live = i < a.n;
  if constexpr (SORT) {
    __shared__ int slot_node[256];
    const bool ordered =
        wg_order_by_key<256, kAdjMaxK + 1>(live ? min((int)a.k[i], kAdjMaxK) : -1,
                                           kAdjMaxK + 1, slot_node);
    live = (int64_t)threadIdx.x < a.n - b0;
    if (live && ordered) i = b0 + slot_node[threadIdx.x];
  }
  double gpd[M::P];
  for (int b = 0; b < M::P; ++b) gpd[b] = 0.0;
  if (live) {
    T p[M::P];
    for (int b = 0; b < M::P; ++b)
      p[b] = (a.par_pernode >> b & 1u) ? a.par[(int64_t)b * a.Np + i] : a.par_uniform[b];
    const int k = a.k[i];
    const T h = (T)(a.dt / (double)k);
    T lam[M::S];
    lam[0] = a.lamV[i];
    for (int s = 1; s < M::S; ++s) lam[s] = a.lam[(int64_t)s * a.Np + i];
    T gp[M::P];
    for (int b = 0; b < M::P; ++b) gp[b] = T(0);
    T v_entry;
    if (k <= 2) {
      // one or two substeps (most nodes outside upstrokes): both substep
      // inputs stay in registers
      T y0[M::S], y1[M::S];
      for (int s = 0; s < M::S; ++s) y0[s] = y1[s] = a.entry[(int64_t)s * a.Np + i];
      if (k == 2) M::substep(y1, p, h, false);
      for (int q = k - 1; q >= 0; --q) {
        T yq[M::S];
        for (int s = 0; s < M::S; ++s) yq[s] = q ? y1[s] : y0[s];
        A::vjp(yq, p, h, lam, gp);
      }
      v_entry = y0[0];
    } else {
      // the inputs of all k substeps, replayed forward, then reversed
      T ys[kAdjMaxK][M::S];
      for (int s = 0; s < M::S; ++s) ys[0][s] = a.entry[(int64_t)s * a.Np + i];
      for (int q = 1; q < k; ++q) {
        for (int s = 0; s < M::S; ++s) ys[q][s] = ys[q - 1][s];
        M::substep(ys[q], p, h, false);
      }
      for (int q = k - 1; q >= 0; --q) A::vjp(ys[q], p, h, lam, gp);
      v_entry = ys[0][0];
    }
    // loss term of a sensor node: lam_V += 2 (V_entry - target)
    if (a.sens_of) {
      const int32_t sq = a.sens_of[i];
      const int64_t step = *a.clk.base + a.clk.g;
      if (sq >= 0 && step < a.target_steps)
        lam[0] = (T)((double)lam[0] +
                     2.0 * ((double)v_entry - a.target[step * a.ns + sq]));
    }
    a.lamV[i] = lam[0];
    for (int s = 1; s < M::S; ++s) a.lam[(int64_t)s * a.Np + i] = lam[s];
    // derivative with respect to a common multiplier of each parameter row
    for (int b = 0; b < M::P; ++b) gpd[b] = (double)p[b] * (double)gp[b];
  }
  // workgroup sum into this workgroup's own FP64 slot (no atomics)
  __shared__ double part[4][M::P];
  for (int b = 0; b < M::P; ++b) {
    double v = gpd[b];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6][b] = v;
  }
  __syncthreads();
  if (threadIdx.x < M::P) {
    const int b = threadIdx.x;
    a.gpart[(int64_t)blockIdx.x * kMaxParams + b] += part[0][b] + part[1][b] + part[2][b] + part[3][b];
  }
}

template <typename T>
void launch_adj_ionic(int model, const AdjIonArgs<T>& a, hipStream_t s) {
  if (a.n <= 0) return;
  const dim3 grid((unsigned)((a.n + 255) / 256));
  if (model == MONO_MODEL_LINEAR)
    hipLaunchKernelGGL((k_adj_ionic<T, LinearModel, LinearAdj, false>), grid, dim3(256), 0, s, a);
  else if (model == MONO_MODEL_MS)
    hipLaunchKernelGGL((k_adj_ionic<T, MSModel, MSAdj, false>), grid, dim3(256), 0, s, a);
  else if (model == MONO_MODEL_TP06_TYPES && a.sort)
    hipLaunchKernelGGL((k_adj_ionic<T, TP06TypesModel, TP06TypesAdj, true>), grid, dim3(256), 0,
                       s, a);
  else if (model == MONO_MODEL_TP06_TYPES)
    hipLaunchKernelGGL((k_adj_ionic<T, TP06TypesModel, TP06TypesAdj, false>), grid, dim3(256), 0,
                       s, a);
  else if (model == MONO_MODEL_TP06_FIBRO && a.sort)
    hipLaunchKernelGGL((k_adj_ionic<T, TP06FibroModel, TP06FibroAdj, true>), grid, dim3(256), 0,
                       s, a);
  else if (model == MONO_MODEL_TP06_FIBRO)
    hipLaunchKernelGGL((k_adj_ionic<T, TP06FibroModel, TP06FibroAdj, false>), grid, dim3(256), 0,
                       s, a);
  else if (a.sort)
    hipLaunchKernelGGL((k_adj_ionic<T, TP06Model, TP06Adj, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_adj_ionic<T, TP06Model, TP06Adj, false>), grid, dim3(256), 0, s, a);
}

template <typename T>
void launch_sensor_loss(const T* V, const SensorArgs& a, hipStream_t s) {
  if (a.ns <= 0) return;
  hipLaunchKernelGGL((k_sensor_loss<T>), dim3(1), dim3(256), 0, s, V, a);
}
template <typename T>
void launch_sensor_sample(const T* V, const int32_t* sens, int ns, double* out, hipStream_t s) {
  if (ns <= 0) return;
  hipLaunchKernelGGL((k_sensor_sample<T>), dim3((ns + 255) / 256), dim3(256), 0, s, V, sens, ns,
                     out);
}
template void launch_sensor_sample<float>(const float*, const int32_t*, int, double*, hipStream_t);
template void launch_sensor_sample<double>(const double*, const int32_t*, int, double*,
                                           hipStream_t);
// x[i] *= c for i < n (one parameter row)
template <typename T>
__global__ void k_scale_row(T* x, int64_t n, T c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= c;
}
template <typename T>
void launch_scale_row(T* x, int64_t n, T c, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_scale_row<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n,
                     c);
}
template void launch_scale_row<float>(float*, int64_t, float, hipStream_t);
template void launch_scale_row<double>(double*, int64_t, double, hipStream_t);

// out[j] = (sum over q = 0, 1, ..., n-1 in that order of x[q * stride + col_j])
// / div_j (div_j = 1: the plain sum), one thread per j: the sums a host loop
// would form, bit for bit.
__global__ void k_ordered_sums(const double* x, int64_t n, int stride, OrderedSums a,
                               double* out) {
  const int j = threadIdx.x;
  if (j >= a.count) return;
  double acc = 0.0;
  for (int64_t q = 0; q < n; ++q) acc += x[q * stride + a.col[j]];
  out[j] = acc / a.div[j];
}
void launch_ordered_sums(const double* x, int64_t n, int stride, const OrderedSums& a,
                         double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_ordered_sums, dim3(1), dim3(64), 0, s, x, n, stride, a, out);
}

template void launch_adj_diffusion<float>(int, const AdjDiffArgs<float>&, hipStream_t);
template void launch_adj_diffusion<double>(int, const AdjDiffArgs<double>&, hipStream_t);
template void launch_adj_ionic<float>(int, const AdjIonArgs<float>&, hipStream_t);
template void launch_adj_ionic<double>(int, const AdjIonArgs<double>&, hipStream_t);
template void launch_sensor_loss<float>(const float*, const SensorArgs&, hipStream_t);
template void launch_sensor_loss<double>(const double*, const SensorArgs&, hipStream_t);
}  // namespace mono
