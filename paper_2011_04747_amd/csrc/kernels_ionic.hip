// Reaction kernel of the DAETI step A (paper Sec. 2): every node advances
// its own cell model over dt in k substeps of dt/k, with
//     k = min(k0 + floor|dV/dt|, k_max),  k0 = 5 if dV/dt > 0 else 1,
// gates by Rush-Larsen (y <- y_inf + (y - y_inf) exp(-h/tau)) and every other
// variable by forward Euler, all rates taken at the substep start.
//
// One node per lane with the whole cell state in registers; states,
// parameters and V are structure-of-arrays so every load and store of a
// wavefront is one contiguous 256 B (FP32) or 512 B (FP64) segment (or, with
// the nodes of a workgroup ordered by k, falls inside the workgroup's own
// segment).  The activation time of
// a node (first upward crossing of a threshold between the V samples taken at
// reaction entry, linearly interpolated) is kept in FP64 in every precision.
#include <type_traits>

#include "cell_models.h"
#include "mono_internal.h"
#include "wg_sort.h"

namespace mono {

// ---------------------------------------------------------------------------
// the reaction kernel
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// APD90 of the first action potential from the reaction-entry samples v0 =
// V_{n-1}, v1 = V_n of outer step n (times in FP64, one rounding per
// operation): the sampled interval of largest slope from activation on gives
// the upstroke time (its midpoint), V_rest is the sample before activation,
// V_max the largest sample since, and repolarisation the first interval
// crossing V_max - 0.9 (V_max - V_rest) downwards, interpolated linearly.
__device__ __forceinline__ void track_apd(double* apd, int64_t Np, int64_t i, int64_t step,
                                          double dt, double v0, double v1, bool first) {
  double* tup = apd;
  double* dmax = apd + Np;
  double* vmax = apd + 2 * Np;
  double* vrest = apd + 3 * Np;
  double* trep = apd + 4 * Np;
  const double t0 = rn_add(rn_add(rn_mul((double)step, dt), rn_mul(0.5, dt)), -dt);
  const double tmid = rn_add(t0, rn_mul(0.5, dt));
  const double d = (v1 - v0) / dt;
  if (first) {
    tup[i] = tmid;
    dmax[i] = d;
    vmax[i] = v1;
    vrest[i] = v0;
    return;
  }
  if (trep[i] >= 0.0 || tup[i] < 0.0) return;   // done, or not activated
  if (d > dmax[i]) {
    dmax[i] = d;
    tup[i] = tmid;
  }
  const double vm = vmax[i];
  const double v90 = rn_add(vm, -rn_mul(0.9, rn_add(vm, -vrest[i])));
  if (v0 >= v90 && v1 < v90) trep[i] = rn_add(t0, rn_mul((v0 - v90) / (v0 - v1), dt));
  if (v1 > vm) vmax[i] = v1;
}

// The substep count of node i at outer step `step`, with the bookkeeping that
// goes with reaction entry: non-finite check, activation time, V_prev, k-trace
// record/replay and the stored k.  y/p are needed only for dvdt_src = 1.
template <typename T, class M>
__device__ __forceinline__ int decide_k(const IonArgs<T>& a, int64_t i, int64_t step, T Vb,
                                        const T* y, const T* p) {
  const double dt = a.clk.dt;
  if (!isfinite(Vb)) atomicOr(a.flag, 1);
  const T vp = a.vprev[i];
  // dV/dt that drives the substep count
  T d;
  if (a.dvdt_src == 0)
    d = (step == 0) ? T(0) : (Vb - vp) / (T)dt;
  else
    d = M::vrate(y, p);
  // activation time: first upward crossing between reaction-entry samples
  if (step > 0) {
    const double thr = a.lat_thr, v0 = (double)vp, v1 = (double)Vb;
    bool first = false;
    if (v0 < thr && v1 >= thr && a.lat[i] < 0.0) {
      const double w = (thr - v0) / (v1 - v0);
      const double tA = rn_add(rn_mul((double)step, dt), rn_mul(0.5, dt));
      a.lat[i] = rn_add(rn_add(tA, -dt), rn_mul(w, dt));
      first = true;
    }
    if (a.apd) track_apd(a.apd, a.Np, i, step, dt, v0, v1, first);
  }
  a.vprev[i] = Vb;
  // k = min(k0 + floor|d|, k_max), k0 = 5 for d > 0 else 1
  const T kd = (d > T(0) ? T(5) : T(1)) + xfloor(fabs(d));
  int k = (kd <= (T)a.k_max) ? (int)kd : a.k_max;
  if (a.kt.mode & 1) {
    const int64_t r = a.kt.rec_rel ? a.clk.g : step - a.kt.rec_base;
    if (r >= 0 && r < a.kt.rec_steps) a.kt.rec[r * a.n + i] = (uint8_t)k;
  }
  if (a.kt.mode & 2) {
    // a replayed count is clamped to [1, k_max] like a decided one (a trace
    // entry of 0 would give h = dt/0, and the adjoint replays at most k_max
    // substeps per node)
    const int64_t r = step - a.kt.rep_base;
    if (r >= 0 && r < a.kt.rep_steps) k = min(max((int)a.kt.rep[r * a.n + i], 1), a.k_max);
  }
  a.lastk[i] = (uint8_t)k;
  return k;
}

// Loads and stores of the state, parameter and potential rows of the node at
// byte offset boff from the workgroup's first node b0.  Fast form (off32):
// through buffer resources whose base (row 0 at node b0) sits in scalar
// registers, with the row as a 32-bit scalar offset and the node as a 32-bit
// lane offset, so an access takes no per-lane address arithmetic and nothing
// address-like stays live across the substep loop; the host selects it when
// every row offset fits in 32 bits.  General form: 64-bit indices.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const T* base) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, -1, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T ld_row(__amdgpu_buffer_rsrc_t r, uint32_t boff, uint32_t soff) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, boff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, boff, soff, 0));
}
template <typename T>
__device__ __forceinline__ void st_row(__amdgpu_buffer_rsrc_t r, uint32_t boff, uint32_t soff,
                                       T v) {
  if constexpr (sizeof(T) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, boff, soff, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(__attribute__((__vector_size__(8))) unsigned int, v), r, boff, soff, 0);
}

template <typename T, class M>
__device__ __forceinline__ void load_cell(const IonArgs<T>& a, int64_t b0, uint32_t lane, T* y,
                                          T* p) {
  if (a.off32) {
    const uint32_t boff = lane * (uint32_t)sizeof(T);
    const uint32_t rs = (uint32_t)(a.Np * (int64_t)sizeof(T));
    y[0] = ld_row<T>(rows_rsrc(a.V + b0), boff, 0u);
    const __amdgpu_buffer_rsrc_t st = rows_rsrc(a.st + b0);
    for (int s = 1; s < M::S; ++s) y[s] = ld_row<T>(st, boff, (uint32_t)(s - 1) * rs);
    const __amdgpu_buffer_rsrc_t pr = rows_rsrc(a.par + b0);
    for (int q = 0; q < M::P; ++q) {
      // the per-node test is uniform: a uniform parameter stays a scalar
      T v = a.par_uniform[q];
      if (a.par_pernode >> q & 1u) v = ld_row<T>(pr, boff, (uint32_t)q * rs);
      p[q] = v;
    }
    return;
  }
  const int64_t i = b0 + lane;
  y[0] = a.V[i];
  for (int s = 1; s < M::S; ++s) y[s] = a.st[(int64_t)(s - 1) * a.Np + i];
  for (int q = 0; q < M::P; ++q) {
    T v = a.par_uniform[q];
    if (a.par_pernode >> q & 1u) v = a.par[(int64_t)q * a.Np + i];
    p[q] = v;
  }
}

template <typename T, class M>
__device__ __forceinline__ void advance_cell(const IonArgs<T>& a, int64_t b0, uint32_t lane, T* y,
                                             const T* p, int k) {
  const uint32_t boff = lane * (uint32_t)sizeof(T);
  const uint32_t rs = (uint32_t)(a.Np * (int64_t)sizeof(T));
  if (a.tape_st) {
    if (a.off32) {
      const __amdgpu_buffer_rsrc_t tp = rows_rsrc(a.tape_st + b0);
      for (int s = 1; s < M::S; ++s) st_row<T>(tp, boff, (uint32_t)(s - 1) * rs, y[s]);
    } else {
      const int64_t i = b0 + lane;
      for (int s = 1; s < M::S; ++s) a.tape_st[(int64_t)(s - 1) * a.Np + i] = y[s];
    }
  }
  const T h = (T)(a.clk.dt / (double)k);
  const bool clamp = a.vclamp != 0;
  for (int s = 0; s < k; ++s) M::substep(y, p, h, clamp);
  T* const vo = a.Vout ? a.Vout : a.V;
  if (a.off32) {
    st_row<T>(rows_rsrc(vo + b0), boff, 0u, y[0]);
    const __amdgpu_buffer_rsrc_t st = rows_rsrc(a.st + b0);
    for (int s = 1; s < M::S; ++s) st_row<T>(st, boff, (uint32_t)(s - 1) * rs, y[s]);
  } else {
    // the node index taken again from the byte offset, which stays live for
    // the 32-bit path anyway, rather than a 64-bit index kept through the
    // substep loop (the empty asm hides that the offset came from the lane,
    // so that the compiler does not reuse an index computed before the loop)
    uint32_t off = boff;
    __asm__ volatile("" : "+v"(off));
    const int64_t i = b0 + (int64_t)(off / (uint32_t)sizeof(T));
    vo[i] = y[0];
    for (int s = 1; s < M::S; ++s) a.st[(int64_t)(s - 1) * a.Np + i] = y[s];
  }
}

// One node per lane.  SORT = false: the lane that decides node i's k advances
// node i, so a wavefront runs as many substeps as its largest k.  SORT = true:
// the workgroup first decides the k of all its nodes, orders them by k in LDS
// (a stable counting sort over k = 0..kSortMaxK, larger k sharing the last
// key), and lane t then advances the t-th node of that order, so a wavefront
// mixes substep counts only where two keys meet.  Each node's arithmetic is
// the same either way, so both give the same bits.
// Occupancy floor for the register allocator: 8 wavefronts per SIMD (at most
// 64 registers) for FP32, so that four 512-lane workgroups fill a compute
// unit; the TP06 substep loop fits in them without spilling (the fallback
// node index is rebuilt after the loop, see advance_cell).  FP64: 2 per SIMD
// (256 registers; without a floor the allocator also takes accumulation
// registers and leaves one), since its substep needs twice the registers per
// value and a floor of three or four makes it spill and run slower.
template <typename T>
constexpr int kIonWavesPerEU = sizeof(T) == 4 ? 8 : 2;

template <typename T, class M, int BLOCK, bool SORT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(kIonWavesPerEU<T>)))
void k_ionic(IonArgs<T> a) {
  const int64_t b0 = (int64_t)blockIdx.x * BLOCK;
  const int64_t i = b0 + threadIdx.x;
  const bool live = i < a.n;
  const int64_t step = *a.clk.base + a.clk.g;
  int k = 0;
  T y[M::S];
  T p[M::P];
  if (live) {
    if (!SORT || a.dvdt_src != 0) {
      load_cell<T, M>(a, b0, threadIdx.x, y, p);
      k = decide_k<T, M>(a, i, step, y[0], y, p);
    } else {
      k = decide_k<T, M>(a, i, step, a.V[i], y, p);
    }
  }
  if (a.stats) {
    // k statistics: wavefront reductions, then one atomic per workgroup and
    // counter (diagnostic path, off by default)
    __shared__ unsigned long long part[4][BLOCK / 64];
    const unsigned long long ks = wave_sum_u64((unsigned long long)k);
    const int kmax = wave_max_i(k);
    const unsigned long long sat = wave_sum_u64((live && k == a.k_max) ? 1ull : 0ull);
    const unsigned long long cnt = wave_sum_u64(live ? 1ull : 0ull);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
      part[0][w] = ks;
      part[1][w] = 64ull * (unsigned long long)kmax;
      part[2][w] = cnt;
      part[3][w] = sat;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
      unsigned long long v = 0;
      for (int q = 0; q < BLOCK / 64; ++q) v += part[threadIdx.x][q];
      atomicAdd(&a.stats[threadIdx.x * 16], v);   // one 128-byte line per counter
    }
  }
  if constexpr (SORT) {
    __shared__ int slot_node[BLOCK];
    __shared__ unsigned char node_k[BLOCK];
    node_k[threadIdx.x] = (unsigned char)k;   // k <= 255 (k_max is capped there)
    // keys 1 .. min(k_max, kSortMaxK) occur; a model with a cheap node class
    // (fibroblasts) gives those nodes key 0, so that they share wavefronts
    int key = live ? min(k, kSortMaxK) : -1;
    if constexpr (std::is_same<M, TP06FibroModel>::value) {
      if (live) {
        const T cls = (a.par_pernode >> 6 & 1u) ? a.par[6 * a.Np + i] : a.par_uniform[6];
        if (cls == T(1)) key = 0;
      }
    }
    const bool ordered = wg_order_by_key<BLOCK, kSortMaxK + 1>(
        key, min(a.k_max, kSortMaxK) + 1, slot_node);
    const int64_t n_here = min((int64_t)BLOCK, a.n - b0);
    if ((int64_t)threadIdx.x >= n_here) return;
    const uint32_t j = ordered ? (uint32_t)slot_node[threadIdx.x] : threadIdx.x;
    load_cell<T, M>(a, b0, j, y, p);
    advance_cell<T, M>(a, b0, j, y, p, node_k[j]);
  } else {
    if (!live) return;
    advance_cell<T, M>(a, b0, threadIdx.x, y, p, k);
  }
}

template <typename T, class M, int BLOCK>
static void launch_ionic_k(const IonArgs<T>& a, bool sort, hipStream_t s) {
  const dim3 grid((unsigned)((a.n + BLOCK - 1) / BLOCK));
  if (sort)
    launch_step_kernel(k_ionic<T, M, BLOCK, true>, grid, dim3(BLOCK), s, a);
  else
    launch_step_kernel(k_ionic<T, M, BLOCK, false>, grid, dim3(BLOCK), s, a);
}
template <typename T, class M>
static void launch_ionic_m(const IonArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  const bool sort = c.react_sort != 0;
  if (c.react_block == 128) return launch_ionic_k<T, M, 128>(a, sort, s);
  if (c.react_block == 512) return launch_ionic_k<T, M, 512>(a, sort, s);
  if constexpr (sizeof(T) == 4) {
    // 16 wavefronts per workgroup fit the register file only in FP32
    if (c.react_block == 1024) return launch_ionic_k<T, M, 1024>(a, sort, s);
  }
  launch_ionic_k<T, M, 256>(a, sort, s);
}

template <typename T>
void launch_ionic(int model, const IonArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  if (a.n <= 0) return;
  if (model == MONO_MODEL_LINEAR)
    launch_ionic_m<T, LinearModel>(a, c, s);
  else if (model == MONO_MODEL_MS)
    launch_ionic_m<T, MSModel>(a, c, s);
  else if (model == MONO_MODEL_TP06_TYPES)
    launch_ionic_m<T, TP06TypesModel>(a, c, s);
  else if (model == MONO_MODEL_TP06_FIBRO)
    launch_ionic_m<T, TP06FibroModel>(a, c, s);
  else
    launch_ionic_m<T, TP06Model>(a, c, s);
}

template void launch_ionic<float>(int, const IonArgs<float>&, const LaunchCfg&, hipStream_t);
template void launch_ionic<double>(int, const IonArgs<double>&, const LaunchCfg&, hipStream_t);

}  // namespace mono
