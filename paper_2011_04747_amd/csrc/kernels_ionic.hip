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
#include "mono_internal.h"

namespace mono {

__device__ __forceinline__ float xexp(float x) { return expf(x); }
__device__ __forceinline__ double xexp(double x) { return exp(x); }
__device__ __forceinline__ float xexpm1(float x) { return expm1f(x); }
__device__ __forceinline__ double xexpm1(double x) { return expm1(x); }
__device__ __forceinline__ float xlog(float x) { return logf(x); }
__device__ __forceinline__ double xlog(double x) { return log(x); }
__device__ __forceinline__ float xsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double xsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float xfloor(float x) { return floorf(x); }
__device__ __forceinline__ double xfloor(double x) { return floor(x); }

template <typename T>
__device__ __forceinline__ T rush_larsen(T y, T yinf, T tau, T h) {
  return yinf + (y - yinf) * xexp(-h / tau);
}

// ---------------------------------------------------------------------------
// linear test model: dV/dt = -g (V - E);  p = {g, E}
// ---------------------------------------------------------------------------
struct LinearModel {
  static constexpr int S = 1, P = 2;
  template <typename T>
  __device__ static T vrate(const T* y, const T* p) { return -p[0] * (y[0] - p[1]); }
  template <typename T>
  __device__ static void substep(T* y, const T* p, T h, bool clamp) {
    if (!clamp) y[0] = y[0] + h * (-p[0] * (y[0] - p[1]));
  }
};

// ---------------------------------------------------------------------------
// Mitchell & Schaeffer (2003): v' = h v^2 (1-v)/tau_in - v/tau_out;
// h' = (1-h)/tau_open below v_gate, -h/tau_close from v_gate up.
// p = {tau_in, tau_out, tau_open, tau_close, v_gate}
// ---------------------------------------------------------------------------
struct MSModel {
  static constexpr int S = 2, P = 5;
  template <typename T>
  __device__ static T vrate(const T* y, const T* p) {
    const T v = y[0];
    return y[1] * v * v * (T(1) - v) / p[0] - v / p[1];
  }
  template <typename T>
  __device__ static void substep(T* y, const T* p, T h, bool clamp) {
    const T v = y[0], g = y[1];
    const T dv = g * v * v * (T(1) - v) / p[0] - v / p[1];
    const bool open = v < p[4];
    y[1] = rush_larsen(g, open ? T(1) : T(0), open ? p[2] : p[3], h);
    if (!clamp) y[0] = v + h * dv;
  }
};

// ---------------------------------------------------------------------------
// ten Tusscher & Panfilov (2006), epicardial cell.
// y = {V, Ki, Nai, Cai, Cass, CaSR, Rbar, m, h, j, xr1, xr2, xs, r, s, d, f,
//      f2, fCass};  p = {Ko, gNa, gCaL, gKr, gKs, gK1 scalings}
// Currents in pA/pF, concentrations in mM, time in ms.  Ca_i, Ca_ss and
// Ca_SR are buffered instantaneously: forward Euler moves the total
// (free + bound) amount and the free value is recovered from the quadratic.
// ---------------------------------------------------------------------------
namespace tp06 {
constexpr double kR = 8314.472, kT = 310.0, kF = 96485.3415;
constexpr double kRTF = kR * kT / kF;      // mV
constexpr double kFRT = kF / (kR * kT);    // 1/mV
constexpr double kCap = 0.185;             // cell capacitance (uF)
constexpr double kVc = 0.016404, kVsr = 0.001094, kVss = 0.00005468;
constexpr double kNao = 140.0, kCao = 2.0;
constexpr double kGNa = 14.838, kGK1 = 5.405, kGto = 0.294, kGKr = 0.153, kGKs = 0.392;
constexpr double kPKNa = 0.03, kGCaL = 3.980e-5;
constexpr double kNaCaMax = 1000.0, kNaCaGam = 0.35, kKmCa = 1.38, kKmNai = 87.5;
constexpr double kNaCaSat = 0.1, kNaCaAlpha = 2.5;
constexpr double kPNaK = 2.724, kKmK = 1.0, kKmNa = 40.0;
constexpr double kGpK = 0.0146, kGpCa = 0.1238, kKpCa = 0.0005, kGbNa = 0.00029, kGbCa = 0.000592;
constexpr double kVmaxUp = 0.006375, kKup = 0.00025, kVrel = 0.102;
constexpr double kK1p = 0.15, kK2p = 0.045, kK3 = 0.060, kK4 = 0.005;
constexpr double kEC = 1.5, kMaxSR = 2.5, kMinSR = 1.0, kVleak = 0.00036, kVxfer = 0.0038;
constexpr double kBufc = 0.2, kKbufc = 0.001, kBufsr = 10.0, kKbufsr = 0.3;
constexpr double kBufss = 0.4, kKbufss = 0.00025;
// concentration change per unit current: Cm / (V F)
constexpr double kCurToConc = kCap / (kVc * kF);
}  // namespace tp06

// free concentration c from a new total c_tot = c + B c / (c + K), i.e. the
// positive root of c^2 + (B + K - c_tot) c - K c_tot = 0, in the form that
// avoids cancellation
template <typename T>
__device__ __forceinline__ T free_from_total(T tot, T B, T K) {
  const T b = B + K - tot;
  const T c = K * tot;
  const T disc = xsqrt(b * b + T(4) * c);
  return (b >= T(0)) ? (T(2) * c) / (b + disc) : T(0.5) * (disc - b);
}

template <typename T>
struct TP06Fluxes {
  T Iion, INa, IbNa, INaK, INaCa, IK, ICaL, IbCa, IpCa;   // IK: K+ carrying currents
  T Irel, Iup, Ileak, Ixfer;
};

template <typename T>
__device__ __forceinline__ void tp06_fluxes(const T* y, const T* p, TP06Fluxes<T>& c) {
  using namespace tp06;
  const T V = y[0], Ki = y[1], Nai = y[2], Cai = y[3], Cass = y[4], CaSR = y[5], Rb = y[6];
  const T Ko = p[0];
  const T rtf = T(kRTF), frt = T(kFRT);
  const T EK = rtf * xlog(Ko / Ki);
  const T ENa = rtf * xlog(T(kNao) / Nai);
  const T ECa = T(0.5) * rtf * xlog(T(kCao) / Cai);
  const T EKs = rtf * xlog((Ko + T(kPKNa) * T(kNao)) / (Ki + T(kPKNa) * Nai));
  const T sqKo = xsqrt(Ko / T(5.4));

  const T m = y[7], hh = y[8], jj = y[9];
  c.INa = p[1] * T(kGNa) * m * m * m * hh * jj * (V - ENa);

  const T vk = V - EK;
  const T aK1 = T(0.1) / (T(1) + xexp(T(0.06) * (vk - T(200))));
  const T bK1 = (T(3) * xexp(T(0.0002) * (vk + T(100))) + xexp(T(0.1) * (vk - T(10)))) /
                (T(1) + xexp(T(-0.5) * vk));
  const T IK1 = p[5] * T(kGK1) * sqKo * (aK1 / (aK1 + bK1)) * vk;
  const T Ito = T(kGto) * y[13] * y[14] * vk;
  const T IKr = p[3] * T(kGKr) * sqKo * y[10] * y[11] * vk;
  const T IKs = p[4] * T(kGKs) * y[12] * y[12] * (V - EKs);
  const T IpK = T(kGpK) * vk / (T(1) + xexp((T(25) - V) / T(5.98)));

  // L-type Ca current with the removable singularity at V = 15 mV handled
  // through x / (e^x - 1)
  const T x = T(2) * (V - T(15)) * frt;
  const T xe = (x == T(0)) ? T(1) : x / xexpm1(x);
  c.ICaL = p[2] * T(kGCaL) * y[15] * y[16] * y[17] * y[18] * T(2.0 * kF) * xe *
           (T(0.25) * Cass * xexp(x) - T(kCao));

  const T eg = xexp(T(kNaCaGam) * V * frt);
  const T eg1 = xexp(T(kNaCaGam - 1.0) * V * frt);
  const T denom = T((kKmNai * kKmNai * kKmNai + kNao * kNao * kNao) * (kKmCa + kCao));
  c.INaCa = T(kNaCaMax) *
            (eg * Nai * Nai * Nai * T(kCao) - eg1 * T(kNao * kNao * kNao) * Cai * T(kNaCaAlpha)) /
            (denom * (T(1) + T(kNaCaSat) * eg1));
  c.INaK = T(kPNaK) * Ko * Nai /
           ((Ko + T(kKmK)) * (Nai + T(kKmNa)) *
            (T(1) + T(0.1245) * xexp(T(-0.1) * V * frt) + T(0.0353) * xexp(-V * frt)));
  c.IpCa = T(kGpCa) * Cai / (T(kKpCa) + Cai);
  c.IbNa = T(kGbNa) * (V - ENa);
  c.IbCa = T(kGbCa) * (V - ECa);
  c.IK = IK1 + Ito + IKr + IKs + IpK;
  c.Iion = c.INa + c.IK + c.ICaL + c.INaCa + c.INaK + c.IpCa + c.IbNa + c.IbCa;

  const T r_sr = T(kEC) / CaSR;
  const T kcasr = T(kMaxSR) - T(kMaxSR - kMinSR) / (T(1) + r_sr * r_sr);
  const T k1 = T(kK1p) / kcasr;
  const T cs2 = Cass * Cass;
  c.Irel = T(kVrel) * (k1 * cs2 * Rb / (T(kK3) + k1 * cs2)) * (CaSR - Cass);
  c.Iup = T(kVmaxUp) / (T(1) + T(kKup * kKup) / (Cai * Cai));
  c.Ileak = T(kVleak) * (CaSR - Cai);
  c.Ixfer = T(kVxfer) * (Cass - Cai);
}

struct TP06Model {
  static constexpr int S = 19, P = 6;
  template <typename T>
  __device__ static T vrate(const T* y, const T* p) {
    TP06Fluxes<T> c;
    tp06_fluxes(y, p, c);
    return -c.Iion;
  }
  template <typename T>
  __device__ static void substep(T* y, const T* p, T h, bool clamp) {
    using namespace tp06;
    TP06Fluxes<T> c;
    tp06_fluxes(y, p, c);
    const T V = y[0];
    const T cc = T(kCurToConc);
    // forward Euler: V, Ki, Nai, Rbar; buffered totals of Ca_i, Ca_ss, Ca_SR
    const T dKi = -(c.IK - T(2) * c.INaK) * cc;
    const T dNai = -(c.INa + c.IbNa + T(3) * c.INaK + T(3) * c.INaCa) * cc;
    const T dCai = -(c.IbCa + c.IpCa - T(2) * c.INaCa) * T(0.5) * cc +
                   T(kVsr / kVc) * (c.Ileak - c.Iup) + c.Ixfer;
    const T dCass = -c.ICaL * T(kCap / (2.0 * kVss * kF)) + T(kVsr / kVss) * c.Irel -
                    T(kVc / kVss) * c.Ixfer;
    const T dCaSR = c.Iup - c.Ileak - c.Irel;
    const T r_sr = T(kEC) / y[5];
    const T kcasr = T(kMaxSR) - T(kMaxSR - kMinSR) / (T(1) + r_sr * r_sr);
    const T dRb = -T(kK2p) * kcasr * y[4] * y[6] + T(kK4) * (T(1) - y[6]);

    // gates from the substep-start V (and Ca_ss for fCass)
    T g[12];
    {
      const T e = T(1) / (T(1) + xexp((T(-56.86) - V) / T(9.03)));
      const T am = T(1) / (T(1) + xexp((T(-60) - V) / T(5)));
      const T bm = T(0.1) / (T(1) + xexp((V + T(35)) / T(5))) +
                   T(0.1) / (T(1) + xexp((V - T(50)) / T(200)));
      g[0] = rush_larsen(y[7], e * e, am * bm, h);
    }
    {
      const T e = T(1) / (T(1) + xexp((V + T(71.55)) / T(7.43)));
      const T inf = e * e;
      T ah, bh, aj, bj;
      if (V >= T(-40)) {
        ah = T(0);
        bh = T(0.77) / (T(0.13) * (T(1) + xexp(-(V + T(10.66)) / T(11.1))));
        aj = T(0);
        bj = T(0.6) * xexp(T(0.057) * V) / (T(1) + xexp(T(-0.1) * (V + T(32))));
      } else {
        ah = T(0.057) * xexp(-(V + T(80)) / T(6.8));
        bh = T(2.7) * xexp(T(0.079) * V) + T(3.1e5) * xexp(T(0.3485) * V);
        aj = (T(-2.5428e4) * xexp(T(0.2444) * V) - T(6.948e-6) * xexp(T(-0.04391) * V)) *
             (V + T(37.78)) / (T(1) + xexp(T(0.311) * (V + T(79.23))));
        bj = T(0.02424) * xexp(T(-0.01052) * V) / (T(1) + xexp(T(-0.1378) * (V + T(40.14))));
      }
      g[1] = rush_larsen(y[8], inf, T(1) / (ah + bh), h);
      g[2] = rush_larsen(y[9], inf, T(1) / (aj + bj), h);
    }
    {
      const T a1 = T(450) / (T(1) + xexp((T(-45) - V) / T(10)));
      const T b1 = T(6) / (T(1) + xexp((V + T(30)) / T(11.5)));
      g[3] = rush_larsen(y[10], T(1) / (T(1) + xexp((T(-26) - V) / T(7))), a1 * b1, h);
      const T a2 = T(3) / (T(1) + xexp((T(-60) - V) / T(20)));
      const T b2 = T(1.12) / (T(1) + xexp((V - T(60)) / T(20)));
      g[4] = rush_larsen(y[11], T(1) / (T(1) + xexp((V + T(88)) / T(24))), a2 * b2, h);
    }
    {
      const T a = T(1400) / xsqrt(T(1) + xexp((T(5) - V) / T(6)));
      const T b = T(1) / (T(1) + xexp((V - T(35)) / T(15)));
      g[5] = rush_larsen(y[12], T(1) / (T(1) + xexp((T(-5) - V) / T(14))), a * b + T(80), h);
    }
    {
      const T vr = V + T(40), vs = V + T(45);
      g[6] = rush_larsen(y[13], T(1) / (T(1) + xexp((T(20) - V) / T(6))),
                         T(9.5) * xexp(-vr * vr / T(1800)) + T(0.8), h);
      g[7] = rush_larsen(y[14], T(1) / (T(1) + xexp((V + T(20)) / T(5))),
                         T(85) * xexp(-vs * vs / T(320)) + T(5) / (T(1) + xexp((V - T(20)) / T(5))) +
                             T(3),
                         h);
    }
    {
      const T ad = T(1.4) / (T(1) + xexp((T(-35) - V) / T(13))) + T(0.25);
      const T bd = T(1.4) / (T(1) + xexp((V + T(5)) / T(5)));
      const T gd = T(1) / (T(1) + xexp((T(50) - V) / T(20)));
      g[8] = rush_larsen(y[15], T(1) / (T(1) + xexp((T(-8) - V) / T(7.5))), ad * bd + gd, h);
      const T vf = V + T(27);
      const T tf = T(1102.5) * xexp(-vf * vf / T(225)) + T(200) / (T(1) + xexp((T(13) - V) / T(10))) +
                   T(180) / (T(1) + xexp((V + T(30)) / T(10))) + T(20);
      g[9] = rush_larsen(y[16], T(1) / (T(1) + xexp((V + T(20)) / T(7))), tf, h);
      const T vf2 = V + T(25);
      const T tf2 = T(600) * xexp(-vf2 * vf2 / T(170)) + T(31) / (T(1) + xexp((T(25) - V) / T(10))) +
                    T(16) / (T(1) + xexp((V + T(30)) / T(10)));
      g[10] = rush_larsen(y[17], T(0.67) / (T(1) + xexp((V + T(35)) / T(7))) + T(0.33), tf2, h);
      const T q = (y[4] / T(0.05)) * (y[4] / T(0.05));
      g[11] = rush_larsen(y[18], T(0.6) / (T(1) + q) + T(0.4), T(80) / (T(1) + q) + T(2), h);
    }

    // commit
    const T Cai = y[3], Cass = y[4], CaSR = y[5];
    y[3] = free_from_total(Cai + T(kBufc) * Cai / (Cai + T(kKbufc)) + h * dCai, T(kBufc),
                           T(kKbufc));
    y[4] = free_from_total(Cass + T(kBufss) * Cass / (Cass + T(kKbufss)) + h * dCass, T(kBufss),
                           T(kKbufss));
    y[5] = free_from_total(CaSR + T(kBufsr) * CaSR / (CaSR + T(kKbufsr)) + h * dCaSR, T(kBufsr),
                           T(kKbufsr));
    y[1] = y[1] + h * dKi;
    y[2] = y[2] + h * dNai;
    y[6] = y[6] + h * dRb;
    for (int a = 0; a < 12; ++a) y[7 + a] = g[a];
    if (!clamp) y[0] = V - h * c.Iion;
  }
};

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

template <typename T, class M>
__global__ __launch_bounds__(kBlock) void k_ionic(IonArgs<T> a) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
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
    if (a.kt.mode) {
      const int64_t r = step - a.kt.base;
      if (r >= 0 && r < a.kt.steps) {
        const int64_t at = r * a.n + i;
        if (a.kt.mode & 1) a.kt.rec[at] = (uint8_t)k;
        if (a.kt.mode & 2) k = a.kt.rep[at];
      }
    }
    a.lastk[i] = (uint8_t)k;
  }
  if (a.stats) {
    const unsigned long long ks = wave_sum_u64((unsigned long long)k);
    const int kmax = wave_max_i(k);
    const unsigned long long sat = wave_sum_u64((live && k == a.k_max) ? 1ull : 0ull);
    const unsigned long long cnt = wave_sum_u64(live ? 1ull : 0ull);
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&a.stats[0], ks);
      atomicAdd(&a.stats[1], 64ull * (unsigned long long)kmax);
      atomicAdd(&a.stats[2], cnt);
      atomicAdd(&a.stats[3], sat);
    }
  }
  if (!live) return;
  const T h = (T)(dt / (double)k);
  const bool clamp = a.vclamp != 0;
  for (int s = 0; s < k; ++s) M::substep(y, p, h, clamp);
  a.V[i] = y[0];
  for (int s = 1; s < M::S; ++s) a.st[(int64_t)(s - 1) * a.Np + i] = y[s];
}

template <typename T>
void launch_ionic(int model, const IonArgs<T>& a, hipStream_t s) {
  if (a.n <= 0) return;
  const dim3 grid((unsigned)((a.n + kBlock - 1) / kBlock));
  if (model == MONO_MODEL_LINEAR)
    hipLaunchKernelGGL((k_ionic<T, LinearModel>), grid, dim3(kBlock), 0, s, a);
  else if (model == MONO_MODEL_MS)
    hipLaunchKernelGGL((k_ionic<T, MSModel>), grid, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_ionic<T, TP06Model>), grid, dim3(kBlock), 0, s, a);
}

template void launch_ionic<float>(int, const IonArgs<float>&, hipStream_t);
template void launch_ionic<double>(int, const IonArgs<double>&, hipStream_t);

}  // namespace mono
