// Reaction kernel of the DAETI step A (paper Sec. 2): every node advances
// its own cell model over dt in k substeps of dt/k, with
//     k = min(k0 + floor|dV/dt|, k_max),  k0 = 5 if dV/dt > 0 else 1,
// gates by Rush-Larsen (y <- y_inf + (y - y_inf) exp(-h/tau)) and every other
// variable by forward Euler, all rates taken at the substep start.
//
// One node per lane with the whole cell state in registers; states,
// parameters and V are structure-of-arrays so every load and store of a
// wavefront is one contiguous 256 B (FP32) or 512 B (FP64) segment.  A
// wavefront runs as many substeps as its largest k.  The activation time of
// a node (first upward crossing of a threshold between the V samples taken at
// reaction entry, linearly interpolated) is kept in FP64 in every precision.
#include "cell_models.h"
#include "mono_internal.h"

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

template <typename T, class M, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_ionic(IonArgs<T> a) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool live = i < a.n;
  const int64_t step = *a.clk.base + a.clk.g;
  const double dt = a.clk.dt;
  int k = 0;
  T y[M::S];
  T p[M::P];
  if (live) {
    y[0] = a.V[i];
    for (int s = 1; s < M::S; ++s) y[s] = a.st[(int64_t)(s - 1) * a.Np + i];
    for (int q = 0; q < M::P; ++q)
      p[q] = (a.par_pernode >> q & 1u) ? a.par[(int64_t)q * a.Np + i] : a.par_uniform[q];
    const T Vb = y[0];
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
      if (v0 < thr && v1 >= thr && a.lat[i] < 0.0) {
        const double w = (thr - v0) / (v1 - v0);
        const double tA = __dadd_rn(__dmul_rn((double)step, dt), __dmul_rn(0.5, dt));
        a.lat[i] = __dadd_rn(__dadd_rn(tA, -dt), __dmul_rn(w, dt));
      }
    }
    a.vprev[i] = Vb;
    // k = min(k0 + floor|d|, k_max), k0 = 5 for d > 0 else 1
    const T kd = (d > T(0) ? T(5) : T(1)) + xfloor(fabs(d));
    k = (kd <= (T)a.k_max) ? (int)kd : a.k_max;
    if (a.kt.mode & 1) {
      const int64_t r = step - a.kt.rec_base;
      if (r >= 0 && r < a.kt.rec_steps) a.kt.rec[r * a.n + i] = (uint8_t)k;
    }
    if (a.kt.mode & 2) {
      const int64_t r = step - a.kt.rep_base;
      if (r >= 0 && r < a.kt.rep_steps) k = a.kt.rep[r * a.n + i];
    }
    a.lastk[i] = (uint8_t)k;
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
  if (!live) return;
  const T h = (T)(dt / (double)k);
  const bool clamp = a.vclamp != 0;
  for (int s = 0; s < k; ++s) M::substep(y, p, h, clamp);
  a.V[i] = y[0];
  for (int s = 1; s < M::S; ++s) a.st[(int64_t)(s - 1) * a.Np + i] = y[s];
}

template <typename T, class M, int BLOCK>
static void launch_ionic_k(const IonArgs<T>& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.n + BLOCK - 1) / BLOCK));
  hipLaunchKernelGGL((k_ionic<T, M, BLOCK>), grid, dim3(BLOCK), 0, s, a);
}
template <typename T, class M>
static void launch_ionic_m(const IonArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  if (c.react_block == 128) return launch_ionic_k<T, M, 128>(a, s);
  if (c.react_block == 512) return launch_ionic_k<T, M, 512>(a, s);
  launch_ionic_k<T, M, 256>(a, s);
}

template <typename T>
void launch_ionic(int model, const IonArgs<T>& a, const LaunchCfg& c, hipStream_t s) {
  if (a.n <= 0) return;
  if (model == MONO_MODEL_LINEAR)
    launch_ionic_m<T, LinearModel>(a, c, s);
  else if (model == MONO_MODEL_MS)
    launch_ionic_m<T, MSModel>(a, c, s);
  else
    launch_ionic_m<T, TP06Model>(a, c, s);
}

template void launch_ionic<float>(int, const IonArgs<float>&, const LaunchCfg&, hipStream_t);
template void launch_ionic<double>(int, const IonArgs<double>&, const LaunchCfg&, hipStream_t);

}  // namespace mono
