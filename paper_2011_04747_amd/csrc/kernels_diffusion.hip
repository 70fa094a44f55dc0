// Diffusion kernels of the DAETI step B (paper Sec. 2): one forward-Euler
// substep of dt_ad on dV/dt = -M_L^-1 K V + s(tau), fused with the stimulus
// and written Jacobi-style (read Vin, write Vout), plus the FP64 Gershgorin
// bound of eq. (3) and a power iteration for lambda_max(M_L^-1 K).
//
// Both operator layouts use the difference form
//     V'_i = V_i + dt_ad * ( sum_{j != i} a_ij (V_j - V_i) + s_i ),
// with a_ij = -k_ij / m_i, which equals -(M_L^-1 K V)_i because every row
// of K sums to zero; a constant V is therefore reproduced exactly.
//
// Launch shape: one row per lane, 256 lanes per workgroup, 1-D grid.  The
// workgroup index is remapped so that each of the chip's 8 XCDs (which
// receive workgroups round-robin) works on one contiguous slice of rows: the
// neighbour rows a stencil reaches (up to one plane away) then stay in that
// XCD's L2.
#include "mono_internal.h"

namespace mono {

__device__ __forceinline__ int64_t xcd_row_block(int64_t nb) {
  // hardware dispatch: workgroup b runs on XCD b % 8
  const int64_t b = blockIdx.x;
  const int64_t x = b & 7, idx = b >> 3;
  const int64_t per = nb >> 3, rem = nb & 7;
  return x * per + (x < rem ? x : rem) + idx;
}

__device__ __forceinline__ double tmul(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double tadd(double a, double b) { return __dadd_rn(a, b); }

// Start time of this substep, evaluated exactly as t_n (+ dt/2) + m dt_ad
// with one rounding per operation (no contraction), so that stimulus windows
// open and close on the same substeps on every implementation.
__device__ __forceinline__ double substep_time(const StepClock& c, int half, int m,
                                               double dt_ad) {
  const int64_t step = *c.base + c.g;
  double t0 = tmul((double)step, c.dt);
  if (half) t0 = tadd(t0, tmul(0.5, c.dt));
  return tadd(t0, tmul((double)m, dt_ad));
}

template <typename T>
__device__ __forceinline__ T stimulus_rate(const DiffArgs<T>& a, int64_t i, double tau) {
  if (a.stim.n == 0 || a.stim_mask == nullptr) return T(0);
  uint32_t active = 0;
  for (int s = 0; s < a.stim.n; ++s)
    if (a.stim.t_on[s] <= tau && tau < a.stim.t_end[s]) active |= 1u << s;
  if (!active) return T(0);
  const uint32_t mask = a.stim_mask[i] & active;
  T r = T(0);
  for (int s = 0; s < a.stim.n; ++s)
    if (mask & (1u << s)) r += (T)a.stim.amp[s];
  return r;
}

template <typename T, bool BATCHED>
__global__ __launch_bounds__(kBlock) void k_diff_ell(DiffArgs<T> a) {
  const int64_t nb = (a.n + kBlock - 1) / kBlock;
  const int64_t i = xcd_row_block(nb) * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int q = BATCHED ? a.inst[i] : 0;
  const T vi = a.Vin[i];
  if (BATCHED && a.m >= a.l[q]) {   // this instance has finished its substeps
    a.Vout[i] = vi;
    return;
  }
  const double dt_ad = a.dt_ad[q];
  T acc = T(0);
  for (int s = 0; s < a.W; ++s) {
    const int64_t k = (int64_t)s * a.Np + i;
    const int32_t j = a.col[k];
    acc += a.val[k] * (a.Vin[j] - vi);
  }
  const double tau = substep_time(a.clk, a.half, a.m, dt_ad);
  acc += stimulus_rate(a, i, tau);
  a.Vout[i] = vi + (T)dt_ad * acc;
}

// Symmetric stencil: e[p][i] = -k(i, i+off_p) stored once per edge; row i
// gathers its forward edges from e[p][i] and its backward edges from
// e[p][i-off_p] (the edge stored by the neighbour).  Within an instance the
// entries of absent neighbours are zero, so clamping only keeps loads in
// bounds; a backward neighbour before the instance's first node belongs to
// another instance (whose slots mean other offsets) and is skipped.
template <typename T, int P, bool BATCHED>
__global__ __launch_bounds__(kBlock) void k_diff_stencil(DiffArgs<T> a) {
  const int64_t nb = (a.n + kBlock - 1) / kBlock;
  const int64_t i = xcd_row_block(nb) * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int q = BATCHED ? a.inst[i] : 0;
  const T vi = a.Vin[i];
  if (BATCHED && a.m >= a.l[q]) {
    a.Vout[i] = vi;
    return;
  }
  const int32_t* off = a.off + (int64_t)q * P;
  const int64_t last = a.n - 1;
  const int64_t first = BATCHED ? a.inst_off[q] : 0;
  T acc = T(0);
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int64_t o = off[p];
    const int64_t jf = i + o;
    const int64_t jb = i - o;
    const T wf = a.e[(int64_t)p * a.Np + i];
    const int64_t jbc = jb >= first ? jb : first;
    const T wb = (jb >= first) ? a.e[(int64_t)p * a.Np + jbc] : T(0);
    const T vf = a.Vin[jf <= last ? jf : last];
    const T vb = a.Vin[jbc];
    acc += wf * (vf - vi);
    acc += wb * (vb - vi);
  }
  const double dt_ad = a.dt_ad[q];
  const double tau = substep_time(a.clk, a.half, a.m, dt_ad);
  const T r = a.minv[i] * acc + stimulus_rate(a, i, tau);
  a.Vout[i] = vi + (T)dt_ad * r;
}

template <typename T, int P>
static void launch_stencil_p(const DiffArgs<T>& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.n + kBlock - 1) / kBlock));
  if (a.inst)
    hipLaunchKernelGGL((k_diff_stencil<T, P, true>), grid, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_diff_stencil<T, P, false>), grid, dim3(kBlock), 0, s, a);
}

template <typename T>
void launch_diffusion(int layout, const DiffArgs<T>& a, hipStream_t s) {
  if (a.n <= 0) return;
  const dim3 grid((unsigned)((a.n + kBlock - 1) / kBlock));
  if (layout == MONO_LAYOUT_ELL) {
    if (a.inst)
      hipLaunchKernelGGL((k_diff_ell<T, true>), grid, dim3(kBlock), 0, s, a);
    else
      hipLaunchKernelGGL((k_diff_ell<T, false>), grid, dim3(kBlock), 0, s, a);
    return;
  }
  switch (a.P) {
    case 1: launch_stencil_p<T, 1>(a, s); break;
    case 2: launch_stencil_p<T, 2>(a, s); break;
    case 3: launch_stencil_p<T, 3>(a, s); break;
    case 4: launch_stencil_p<T, 4>(a, s); break;
    case 5: launch_stencil_p<T, 5>(a, s); break;
    case 6: launch_stencil_p<T, 6>(a, s); break;
    case 7: launch_stencil_p<T, 7>(a, s); break;
    case 8: launch_stencil_p<T, 8>(a, s); break;
    case 9: launch_stencil_p<T, 9>(a, s); break;
    case 10: launch_stencil_p<T, 10>(a, s); break;
    case 11: launch_stencil_p<T, 11>(a, s); break;
    case 12: launch_stencil_p<T, 12>(a, s); break;
    default: launch_stencil_p<T, 13>(a, s); break;
  }
}

template void launch_diffusion<float>(int, const DiffArgs<float>&, hipStream_t);
template void launch_diffusion<double>(int, const DiffArgs<double>&, hipStream_t);

__global__ void k_advance_clock(int64_t* base, int64_t by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *base += by;
}
void launch_advance_clock(int64_t* base, int64_t by, hipStream_t s) {
  hipLaunchKernelGGL(k_advance_clock, dim3(1), dim3(64), 0, s, base, by);
}

// ---------------------------------------------------------------------------
// eq. (3): Gershgorin rows in FP64
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_gersh_rows(int64_t n, const int64_t* rp,
                                                       const int32_t* col, const double* val,
                                                       const double* mass, double* r,
                                                       double* g) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double kii = 0.0, off = 0.0;
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
    const double v = val[p];
    if (col[p] == i)
      kii += v;
    else
      off += fabs(v);
  }
  const double s = kii + off;
  r[i] = mass[i] / s;
  g[i] = s / mass[i];
}

void launch_gershgorin(int64_t n, const int64_t* rp, const int32_t* col, const double* val,
                       const double* mass, double* r, double* g, hipStream_t s) {
  hipLaunchKernelGGL(k_gersh_rows, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, n, rp, col, val, mass, r, g);
}

// wavefront (64-lane) reductions through cross-lane shuffles
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One workgroup per instance: min of r and max of g over its rows.
__global__ __launch_bounds__(kBlock) void k_seg_minmax(const int64_t* inst_off, const double* r,
                                                       const double* g, double* rmin,
                                                       double* gmax) {
  __shared__ double smin[kBlock / 64], smax[kBlock / 64];
  const int q = blockIdx.x;
  double mn = INFINITY, mx = 0.0;
  for (int64_t i = inst_off[q] + threadIdx.x; i < inst_off[q + 1]; i += kBlock) {
    mn = fmin(mn, r[i]);
    mx = fmax(mx, g[i]);
  }
  mn = wave_min(mn);
  mx = wave_max(mx);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    smin[w] = mn;
    smax[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kBlock / 64; ++k) {
      mn = fmin(mn, smin[k]);
      mx = fmax(mx, smax[k]);
    }
    rmin[q] = mn;
    gmax[q] = mx;
  }
}

void launch_segmented_minmax(int n_inst, const int64_t* inst_off, const double* r,
                             const double* g, double* rmin, double* gmax, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_minmax, dim3(n_inst), dim3(kBlock), 0, s, inst_off, r, g, rmin, gmax);
}

// ---------------------------------------------------------------------------
// power iteration for lambda_max(M_L^-1 K), FP64 (diagnostic)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_spmv_csr(int64_t n, const int64_t* rp,
                                                     const int32_t* col, const double* val,
                                                     const double* x, double* y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += val[p] * x[col[p]];
  y[i] = s;
}
void launch_spmv_csr(int64_t n, const int64_t* rp, const int32_t* col, const double* val,
                     const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv_csr, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     n, rp, col, val, x, y);
}

__global__ __launch_bounds__(kBlock) void k_seg_dots(const int64_t* inst_off, const double* x,
                                                     const double* kx, const double* mass,
                                                     double* xkx, double* xmx) {
  __shared__ double sa[kBlock / 64], sb[kBlock / 64];
  const int q = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = inst_off[q] + threadIdx.x; i < inst_off[q + 1]; i += kBlock) {
    a += x[i] * kx[i];
    b += x[i] * mass[i] * x[i];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    sa[w] = a;
    sb[w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kBlock / 64; ++k) {
      a += sa[k];
      b += sb[k];
    }
    xkx[q] = a;
    xmx[q] = b;
  }
}
void launch_segmented_dots(int n_inst, const int64_t* inst_off, const double* x, const double* kx,
                           const double* mass, double* xkx, double* xmx, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_dots, dim3(n_inst), dim3(kBlock), 0, s, inst_off, x, kx, mass, xkx,
                     xmx);
}

// x <- (M^-1 K x) / ||x||_M of its instance (xmx = x^T M x per instance)
__global__ __launch_bounds__(kBlock) void k_power_update(int64_t n, const int32_t* inst,
                                                         const double* kx, const double* mass,
                                                         const double* xmx, double* x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int q = inst ? inst[i] : 0;
  x[i] = kx[i] / mass[i] / sqrt(xmx[q]);
}
void launch_power_update(int64_t n, const int32_t* inst, const double* kx, const double* mass,
                         const double* xmx, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_power_update, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, n, inst, kx, mass, xmx, x);
}

// deterministic start vector with energy in every mode (integer hash in [-1,1])
__global__ __launch_bounds__(kBlock) void k_power_init(int64_t n, double* x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  uint64_t z = (uint64_t)i + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}
void launch_power_init(int64_t n, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_power_init, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, n, x);
}

// precision conversion helpers
template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_f64(int64_t n, const T* src, double* dst) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_from_f64(int64_t n, const double* src, T* dst) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}
template <typename T>
void launch_convert(int64_t n, const T* src, double* dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_to_f64<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, n, src, dst);
}
template <typename T>
void launch_convert_from(int64_t n, const double* src, T* dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_from_f64<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, n, src, dst);
}
template void launch_convert<float>(int64_t, const float*, double*, hipStream_t);
template void launch_convert<double>(int64_t, const double*, double*, hipStream_t);
template void launch_convert_from<float>(int64_t, const double*, float*, hipStream_t);
template void launch_convert_from<double>(int64_t, const double*, double*, hipStream_t);

}  // namespace mono
