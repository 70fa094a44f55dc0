// Cell models of the reaction step (paper Sec. 2, step A), written once as
// templates over the scalar type: the reaction kernel instantiates them in
// FP32 and FP64, and the host instantiates them on a counting type to obtain
// the exact arithmetic of one substep.
//
// Every model advances one substep of length h from the substep-start state:
// gates by Rush-Larsen (y <- y_inf + (y - y_inf) exp(-h/tau)), every other
// variable by forward Euler.  State 0 is V.
#pragma once
#include <type_traits>

#include <hip/hip_runtime.h>

namespace mono {

// --- arithmetic primitives --------------------------------------------------
// FP32 uses the hardware reciprocal, exp2 and log2 instructions (about 1 ulp
// each, no denormals) in place of the correctly rounded multi-instruction
// sequences; the difference is at the 1e-6 relative level, far inside the
// FP32 tolerances, and cuts the substep's instruction count severalfold.
// FP64 on the device forms its reciprocal, exp2 and log2 below (within a few
// ulp for the finite, normal, in-range arguments the models pass, without the
// library's handling of denormals, infinities and NaN); the rest of FP64, and
// the host, use the math library.
__host__ __device__ __forceinline__ double xexp(double x) { return exp(x); }
__host__ __device__ __forceinline__ double xexpm1(double x) { return expm1(x); }
__host__ __device__ __forceinline__ double xlog(double x) { return log(x); }
__host__ __device__ __forceinline__ double xsqrt(double x) { return sqrt(x); }
#if defined(__HIP_DEVICE_COMPILE__)
// 1/b from the hardware estimate and two Newton steps r <- r + r (1 - b r)
// (each squares the relative error; the last leaves about an ulp)
__device__ __forceinline__ double xrcp(double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = __builtin_fma(-b, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-b, r, 1.0);
  return __builtin_fma(r, e, r);
}
#else
__host__ __device__ inline double xrcp(double x) { return 1.0 / x; }
#endif
__host__ __device__ __forceinline__ double xfloor(double x) { return floor(x); }
__host__ __device__ __forceinline__ float xexpm1(float x) { return expm1f(x); }
__host__ __device__ __forceinline__ float xfloor(float x) { return floorf(x); }
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ float xexp(float x) { return __expf(x); }
__device__ __forceinline__ float xlog(float x) { return __logf(x); }
__device__ __forceinline__ float xsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float xrcp(float x) { return __builtin_amdgcn_rcpf(x); }
#else
inline float xexp(float x) { return expf(x); }
inline float xlog(float x) { return logf(x); }
inline float xsqrt(float x) { return sqrtf(x); }
inline float xrcp(float x) { return 1.0f / x; }
#endif

// base-2 exponential and logarithm: e^x = 2^(x log2 e), ln x = ln 2 log2 x.
// Written with the base-2 forms, an exponential of an affine function of V
// is 2^(A V + B) with A, B folded into constants (one fused multiply-add and
// the hardware exp2 in FP32) instead of a subtraction, a scaling and the
// base conversion.
constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;
#if defined(__HIP_DEVICE_COMPILE__)
// coefficients of the Taylor series of 2^f = e^(f ln 2), (ln 2)^k / k!, and of
// the series of atanh(s)/s in s^2, 1/(2k + 1), as compile-time constants
template <int K>
struct Exp2Coef {
  static constexpr double v = Exp2Coef<K - 1>::v * kLn2 / K;
};
template <>
struct Exp2Coef<0> {
  static constexpr double v = 1.0;
};
// sum_{k >= K} c_k f^(k - K) to degree 13 by Horner's rule
template <int K>
__device__ __forceinline__ double exp2_series(double f) {
  if constexpr (K == 13)
    return Exp2Coef<13>::v;
  else
    return __builtin_fma(exp2_series<K + 1>(f), f, Exp2Coef<K>::v);
}
template <int K>
__device__ __forceinline__ double atanh_series(double t) {
  if constexpr (K == 11)
    return 1.0 / 23.0;
  else
    return __builtin_fma(atanh_series<K + 1>(t), t, 1.0 / (2 * K + 1));
}
// 2^x = 2^n 2^f with n = rint(x), |f| <= 1/2: the series to degree 13 (its
// remainder is below 2^-56 of the sum for |f ln 2| <= 0.35), then the
// exponent added to n.
__device__ __forceinline__ double xexp2(double x) {
  const double n = __builtin_rint(x);
  return __builtin_amdgcn_ldexp(exp2_series<0>(x - n), (int)n);
}
// log2 x = e + log2 m with x = m 2^e, m in [sqrt(1/2), sqrt(2)); ln m =
// 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...) with s = (m - 1)/(m + 1),
// |s| <= 0.172, to the term s^23 (the next is below 2^-58 of the sum).
__device__ __forceinline__ double xlog2(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);   // [1/2, 1)
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo = m < 0.7071067811865476;
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const double s = (m - 1.0) * xrcp(m + 1.0);
  return __builtin_fma(s * atanh_series<0>(s * s), 2.0 * kLog2e, (double)e);
}
#else
__host__ __device__ inline double xexp2(double x) { return exp2(x); }
__host__ __device__ inline double xlog2(double x) { return log2(x); }
#endif
// xlog2c: the same for operands that do not change inside the substep loop
// (parameters), in a form the compiler may move out of the loop
__host__ __device__ __forceinline__ double xlog2c(double x) { return log2(x); }
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ float xexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float xlog2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float xlog2c(float x) { return __builtin_log2f(x); }
#else
inline float xexp2(float x) { return exp2f(x); }
inline float xlog2(float x) { return log2f(x); }
inline float xlog2c(float x) { return log2f(x); }
#endif

template <typename T>
__host__ __device__ __forceinline__ T xdiv(T a, T b) {
  return a * xrcp(b);
}
// a V + b with the constants rounded once to T
template <typename T>
__host__ __device__ __forceinline__ T lin(T V, double a, double b) {
  return V * T(a) + T(b);
}
// logistic 1 / (1 + 2^z2), i.e. sig(z) for z2 = z log2 e
template <typename T>
__host__ __device__ __forceinline__ T sig2(T z2) {
  return xrcp(T(1) + xexp2(z2));
}
// logistic 1 / (1 + e^z)
template <typename T>
__host__ __device__ __forceinline__ T sig(T z) {
  return xrcp(T(1) + xexp(z));
}
// Rush-Larsen update with the rate 1/tau given directly
template <typename T>
__host__ __device__ __forceinline__ T rl_rate(T y, T yinf, T rate, T h) {
  return yinf + (y - yinf) * xexp(-h * rate);
}
template <typename T>
__host__ __device__ __forceinline__ T rush_larsen(T y, T yinf, T tau, T h) {
  return rl_rate(y, yinf, xrcp(tau), h);
}
// Rush-Larsen update with hl = -h log2 e taken once per substep
template <typename T>
__host__ __device__ __forceinline__ T rl_rate2(T y, T yinf, T rate, T hl) {
  return yinf + (y - yinf) * xexp2(rate * hl);
}

// ---------------------------------------------------------------------------
// linear test model: dV/dt = -g (V - E);  p = {g, E}
// ---------------------------------------------------------------------------
struct LinearModel {
  static constexpr int S = 1, P = 2;
  template <typename T>
  __host__ __device__ static T vrate(const T* y, const T* p) { return -p[0] * (y[0] - p[1]); }
  template <typename T>
  __host__ __device__ static void substep(T* y, const T* p, T h, bool clamp) {
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
  __host__ __device__ static T vrate(const T* y, const T* p) {
    const T v = y[0];
    return xdiv(y[1] * v * v * (T(1) - v), p[0]) - xdiv(v, p[1]);
  }
  template <typename T>
  __host__ __device__ static void substep(T* y, const T* p, T h, bool clamp) {
    const T v = y[0], g = y[1];
    const T dv = xdiv(g * v * v * (T(1) - v), p[0]) - xdiv(v, p[1]);
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
__host__ __device__ __forceinline__ T free_from_total(T tot, T B, T K) {
  const T b = B + K - tot;
  const T c = K * tot;
  const T disc = xsqrt(b * b + T(4) * c);
  return (b >= T(0)) ? xdiv(T(2) * c, b + disc) : T(0.5) * (disc - b);
}
template <typename T>
__host__ __device__ __forceinline__ T total_from_free(T c, T B, T K) {
  return c + xdiv(B * c, c + K);
}

// SR-calcium dependence of the RyR rates,
// max - (max - min) / (1 + (EC/CaSR)^2) = max - (max - min) CaSR^2 / (CaSR^2 + EC^2)
template <typename T>
__host__ __device__ __forceinline__ T tp06_kcasr(T CaSR) {
  using namespace tp06;
  const T c2 = CaSR * CaSR;
  return T(kMaxSR) - T(kMaxSR - kMinSR) * xdiv(c2, c2 + T(kEC * kEC));
}

template <typename T>
struct TP06Fluxes {
  T Iion, INa, IbNa, INaK, INaCa, IK, ICaL, IbCa, IpCa;   // IK: K+ carrying currents
  T Irel, Iup, Ileak, Ixfer;
};

// gto, gks: maximal I_to and I_Ks conductances (the epicardial values unless
// a cell type says otherwise)
template <typename T>
__host__ __device__ __forceinline__ void tp06_fluxes(const T* y, const T* p, TP06Fluxes<T>& c,
                                                     T gto = T(tp06::kGto),
                                                     T gks = T(tp06::kGKs)) {
  using namespace tp06;
  const T V = y[0], Ki = y[1], Nai = y[2], Cai = y[3], Cass = y[4], CaSR = y[5], Rb = y[6];
  const T Ko = p[0];
  // Nernst potentials as differences of base-2 logarithms (the logarithms
  // of the parameter and constant concentrations do not change between
  // substeps); RT/F ln 2 is one constant
  const T rtf2 = T(kRTF * kLn2);
  const T EK = rtf2 * (xlog2c(Ko) - xlog2(Ki));
  const T ENa = rtf2 * (T(7.129283016944966) - xlog2(Nai));            // log2 140
  const T ECa = T(0.5 * kRTF * kLn2) * (T(1) - xlog2(Cai));            // log2 2
  const T EKs = rtf2 * (xlog2c(Ko + T(kPKNa * kNao)) - xlog2(Ki + T(kPKNa) * Nai));
  const T sqKo = xsqrt(Ko * T(1.0 / 5.4));

  const T m = y[7], hh = y[8], jj = y[9];
  c.INa = p[1] * T(kGNa) * m * m * m * hh * jj * (V - ENa);

  const T vk = V - EK;
  // x_K1 = a/(a + b) with a = 0.1 sig(0.06 (vk - 200)) = 0.1/(1 + e_a):
  // 1/(1 + 10 b (1 + e_a))
  const T ea = xexp2(lin(vk, 0.06 * kLog2e, -12.0 * kLog2e));
  // 3 e^{0.0002 (vk + 100)} = 2^{0.0002 log2e vk + 0.02 log2e + log2 3}
  const T bK1 = (xexp2(lin(vk, 0.0002 * kLog2e, 0.02 * kLog2e + 1.5849625007211563)) +
                 xexp2(lin(vk, 0.1 * kLog2e, -kLog2e))) *
                sig2(vk * T(-0.5 * kLog2e));
  const T IK1 = p[5] * T(kGK1) * sqKo * xrcp(T(1) + T(10) * bK1 * (T(1) + ea)) * vk;
  const T Ito = gto * y[13] * y[14] * vk;
  const T IKr = p[3] * T(kGKr) * sqKo * y[10] * y[11] * vk;
  const T IKs = p[4] * gks * y[12] * y[12] * (V - EKs);
  const T IpK = T(kGpK) * vk * sig2(lin(V, -kLog2e / 5.98, 25.0 * kLog2e / 5.98));

  // L-type Ca current with the removable singularity at V = 15 mV handled
  // through x / (e^x - 1)
  const T x = lin(V, 2.0 * kFRT, -30.0 * kFRT);
  const T ex = xexp2(x * T(kLog2e));
  T xe;
  if constexpr (std::is_same<T, float>::value) {
    // FP32: x / (e^x - 1) from the e^x needed anyway, its Taylor series
    // 1 - x/2 + x^2/12 where e^x - 1 would cancel (|x| < 1e-2)
    xe = (fabsf(x) < 1e-2f) ? 1.0f + x * (-0.5f + x * (1.0f / 12.0f)) : xdiv(x, ex - 1.0f);
  } else {
    xe = (x == T(0)) ? T(1) : xdiv(x, xexpm1(x));
  }
  c.ICaL = p[2] * T(kGCaL * 2.0 * kF) * y[15] * y[16] * y[17] * y[18] * xe *
           (T(0.25) * Cass * ex - T(kCao));

  // e^{-VF/RT} serves the Na/Ca exchanger and the Na/K pump
  const T u = xexp2(V * T(-kFRT * kLog2e));
  const T eg = xexp2(V * T(kNaCaGam * kFRT * kLog2e));
  const T eg1 = eg * u;
  const T denom = T((kKmNai * kKmNai * kKmNai + kNao * kNao * kNao) * (kKmCa + kCao));
  c.INaCa = T(kNaCaMax) *
            xdiv(eg * Nai * Nai * Nai * T(kCao) - eg1 * T(kNao * kNao * kNao * kNaCaAlpha) * Cai,
                 denom * (T(1) + T(kNaCaSat) * eg1));
  c.INaK = T(kPNaK) * xdiv(Ko * Nai, (Ko + T(kKmK)) * (Nai + T(kKmNa)) *
                                         (T(1) + T(0.1245) * xexp2(V * T(-0.1 * kFRT * kLog2e)) +
                                          T(0.0353) * u));
  c.IpCa = T(kGpCa) * xdiv(Cai, T(kKpCa) + Cai);
  c.IbNa = T(kGbNa) * (V - ENa);
  c.IbCa = T(kGbCa) * (V - ECa);
  c.IK = IK1 + Ito + IKr + IKs + IpK;
  c.Iion = c.INa + c.IK + c.ICaL + c.INaCa + c.INaK + c.IpCa + c.IbNa + c.IbCa;

  // open RyR fraction k1 cs^2 Rb / (k3 + k1 cs^2) with k1 = k1'/kcasr, taken
  // with both terms multiplied by kcasr
  const T kcasr = tp06_kcasr(CaSR);
  const T cs2 = Cass * Cass;
  const T k1cs2 = T(kK1p) * cs2;
  c.Irel = T(kVrel) * xdiv(k1cs2 * Rb, T(kK3) * kcasr + k1cs2) * (CaSR - Cass);
  const T ci2 = Cai * Cai;
  c.Iup = T(kVmaxUp) * xdiv(ci2, ci2 + T(kKup * kKup));
  c.Ileak = T(kVleak) * (CaSR - Cai);
  c.Ixfer = T(kVxfer) * (Cass - Cai);
}

// 1 / (1 + ez) for ez = e^z precomputed: the logistic factor sig(z)
template <typename T>
__host__ __device__ __forceinline__ T sig_e(T ez) {
  return xrcp(T(1) + ez);
}

// Steady states and rates (1/tau) of the eleven V-driven TP06 gates, in the
// state order m, h, j, xr1, xr2, xs, r, s, d, f, f2.  Exponentials of V that
// differ only by a constant factor are taken once (e^{a + bV} = e^a e^{bV}:
// five shared powers replace fourteen exponentials), and the rates that are
// reciprocals of products of logistic factors are formed directly as
// products of (1 + e^z) (no reciprocal of a reciprocal).  Same functions as
// the published forms; only the rounding differs.
// endo: the endocardial s gate (steady state half-activation at -28 mV, slow
// recovery) instead of the epicardial / M-cell one
template <typename T>
__host__ __device__ __forceinline__ void tp06_gate_params(T V, T* inf, T* rate,
                                                          bool endo = false) {
  constexpr double L = kLog2e;
  const T P5 = xexp2(V * T(0.2 * L));         // e^{V/5}
  const T N10 = xexp2(V * T(-0.1 * L));       // e^{-V/10}
  const T N20 = xexp2(V * T(-0.05 * L));      // e^{-V/20}
  const T P7 = xexp2(V * T(L / 7.0));         // e^{V/7}
  const T N6 = xexp2(V * T(-L / 6.0));        // e^{-V/6}
  {
    // m: alpha = sig(-(V+60)/5), beta = 0.1 sig((V+35)/5) + 0.1 sig((V-50)/200)
    const T e = sig2(lin(V, -L / 9.03, -56.86 * L / 9.03));
    const T ea = xexp2(lin(V, -0.2 * L, -12.0 * L));                 // e^{-(V+60)/5}
    const T bm = T(0.1) * sig_e(T(1096.6331584284585) * P5) +       // e^7 e^{V/5}
                 T(0.1) * sig2(lin(V, 0.005 * L, -0.25 * L));
    inf[0] = e * e;
    rate[0] = (T(1) + ea) * xrcp(bm);
  }
  {
    const T e = sig2(lin(V, L / 7.43, 71.55 * L / 7.43));
    inf[1] = e * e;
    inf[2] = e * e;
    if (V >= T(-40)) {
      rate[1] = T(0.77 / 0.13) * sig2(lin(V, -L / 11.1, -10.66 * L / 11.1));
      rate[2] = T(0.6) * xexp2(V * T(0.057 * L)) *
                sig_e(T(0.04076220397836621) * N10);                 // e^{-3.2} e^{-V/10}
    } else {
      rate[1] = T(0.057) * xexp2(lin(V, -L / 6.8, -80.0 * L / 6.8)) +
                T(2.7) * xexp2(V * T(0.079 * L)) + T(3.1e5) * xexp2(V * T(0.3485 * L));
      rate[2] = (T(-2.5428e4) * xexp2(V * T(0.2444 * L)) -
                 T(6.948e-6) * xexp2(V * T(-0.04391 * L))) *
                    (V + T(37.78)) * sig2(lin(V, 0.311 * L, 0.311 * 79.23 * L)) +
                T(0.02424) * xexp2(V * T(-0.01052 * L)) *
                    sig2(lin(V, -0.1378 * L, -0.1378 * 40.14 * L));
    }
  }
  const T s30 = sig2(lin(V, 0.1 * L, 3.0 * L));    // sig((V+30)/10), shared by f and f2
  {
    // xr1: 1/(alpha beta), alpha = 450 sig(-(V+45)/10), beta = 6 sig((V+30)/11.5)
    inf[3] = sig2(lin(V, -L / 7.0, -26.0 * L / 7.0));
    rate[3] = (T(1) + T(0.011108996538242306) * N10) *                // e^{-4.5} e^{-V/10}
              (T(1) + xexp2(lin(V, L / 11.5, 30.0 * L / 11.5))) * T(1.0 / 2700.0);
    // xr2: alpha = 3 sig(-(V+60)/20), beta = 1.12 sig((V-60)/20)
    inf[4] = sig2(lin(V, L / 24.0, 88.0 * L / 24.0));
    rate[4] = (T(1) + T(0.049787068367863944) * N20) *                // e^{-3} e^{-V/20}
              (T(1) + xexp2(lin(V, 0.05 * L, -3.0 * L))) * T(1.0 / 3.36);
  }
  {
    const T a = T(1400) * xrcp(xsqrt(T(1) + T(2.300975890892825) * N6));   // e^{5/6} e^{-V/6}
    const T b = sig2(lin(V, L / 15.0, -35.0 * L / 15.0));
    inf[5] = sig2(lin(V, -L / 14.0, -5.0 * L / 14.0));
    rate[5] = xrcp(a * b + T(80));
  }
  {
    const T vr = V + T(40), vs = V + T(45);
    inf[6] = sig_e(T(28.03162489452614) * N6);                        // e^{20/6} e^{-V/6}
    rate[6] = xrcp(T(9.5) * xexp2(vr * vr * T(-L / 1800.0)) + T(0.8));
    if (endo) {
      const T ve = V + T(67);
      inf[7] = sig_e(T(270.42640742615254) * P5);                      // e^5.6 e^{V/5}
      rate[7] = xrcp(T(1000) * xexp2(ve * ve * T(-L / 1000.0)) + T(8));
    } else {
      inf[7] = sig_e(T(54.598150033144236) * P5);                     // e^4 e^{V/5}
      rate[7] = xrcp(T(85) * xexp2(vs * vs * T(-L / 320.0)) +
                     T(5) * sig_e(T(0.01831563888873418) * P5) + T(3));  // e^{-4} e^{V/5}
    }
  }
  {
    const T ad = T(1.4) * sig2(lin(V, -L / 13.0, -35.0 * L / 13.0)) + T(0.25);
    const T bd = T(1.4) * sig_e(T(2.718281828459045) * P5);            // e^1 e^{V/5}
    const T gd = sig_e(T(12.182493960703473) * N20);                   // e^{2.5} e^{-V/20}
    inf[8] = sig2(lin(V, -L / 7.5, -8.0 * L / 7.5));
    rate[8] = xrcp(ad * bd + gd);
    const T vf = V + T(27);
    inf[9] = sig_e(T(17.41170806332765) * P7);                         // e^{20/7} e^{V/7}
    rate[9] = xrcp(T(1102.5) * xexp2(vf * vf * T(-L / 225.0)) +
                   T(200) * sig_e(T(3.6692966676192444) * N10) +        // e^{1.3} e^{-V/10}
                   T(180) * s30 + T(20));
    const T vf2 = V + T(25);
    inf[10] = T(0.67) * sig_e(T(148.4131591025766) * P7) + T(0.33);   // e^5 e^{V/7}
    rate[10] = xrcp(T(600) * xexp2(vf2 * vf2 * T(-L / 170.0)) +
                    T(31) * sig_e(T(12.182493960703473) * N10) +        // e^{2.5} e^{-V/10}
                    T(16) * s30);
  }
}

// fCass gate: steady state and rate from the subspace calcium
template <typename T>
__host__ __device__ __forceinline__ void tp06_fcass_params(T Cass, T& inf, T& rate) {
  const T q = (Cass * T(20)) * (Cass * T(20));
  const T r1q = xrcp(T(1) + q);
  inf = T(0.6) * r1q + T(0.4);
  rate = xrcp(T(80) * r1q + T(2));
}

// One TP06 substep with the cell type's I_to / I_Ks conductances and s gate.
template <typename T>
__host__ __device__ __forceinline__ void tp06_substep(T* y, const T* p, T h, bool clamp, T gto,
                                                      T gks, bool endo) {
  using namespace tp06;
  TP06Fluxes<T> c;
  tp06_fluxes(y, p, c, gto, gks);
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
  const T kcasr = tp06_kcasr(y[5]);
  const T dRb = -T(kK2p) * kcasr * y[4] * y[6] + T(kK4) * (T(1) - y[6]);

  // gates from the substep-start V (and Ca_ss for fCass)
  T inf[12], rate[12];
  tp06_gate_params(V, inf, rate, endo);
  tp06_fcass_params(y[4], inf[11], rate[11]);
  T g[12];
  const T hl = h * T(-kLog2e);
  for (int a = 0; a < 12; ++a) g[a] = rl_rate2(y[7 + a], inf[a], rate[a], hl);

  // commit
  y[3] = free_from_total(total_from_free(y[3], T(kBufc), T(kKbufc)) + h * dCai, T(kBufc),
                         T(kKbufc));
  y[4] = free_from_total(total_from_free(y[4], T(kBufss), T(kKbufss)) + h * dCass, T(kBufss),
                         T(kKbufss));
  y[5] = free_from_total(total_from_free(y[5], T(kBufsr), T(kKbufsr)) + h * dCaSR, T(kBufsr),
                         T(kKbufsr));
  y[1] = y[1] + h * dKi;
  y[2] = y[2] + h * dNai;
  y[6] = y[6] + h * dRb;
  for (int a = 0; a < 12; ++a) y[7 + a] = g[a];
  if (!clamp) y[0] = V - h * c.Iion;
}

struct TP06Model {
  static constexpr int S = 19, P = 6;
  template <typename T>
  __host__ __device__ static T vrate(const T* y, const T* p) {
    TP06Fluxes<T> c;
    tp06_fluxes(y, p, c);
    return -c.Iion;
  }
  template <typename T>
  __host__ __device__ static void substep(T* y, const T* p, T h, bool clamp) {
    tp06_substep(y, p, h, clamp, T(tp06::kGto), T(tp06::kGKs), false);
  }
};

// TP06 with a transmural cell type per node in parameter row 6 (0
// epicardial, 1 endocardial, 2 M cell; ten Tusscher & Panfilov 2006): the
// endocardial cell has G_to = 0.073 and the endocardial s gate, the M cell
// G_Ks = 0.098; everything else is the epicardial model.
struct TP06TypesModel {
  static constexpr int S = 19, P = 7;
  template <typename T>
  __host__ __device__ static void type_constants(const T* p, T& gto, T& gks, bool& endo) {
    endo = p[6] == T(1);
    gto = endo ? T(0.073) : T(tp06::kGto);
    gks = p[6] == T(2) ? T(0.098) : T(tp06::kGKs);
  }
  template <typename T>
  __host__ __device__ static T vrate(const T* y, const T* p) {
    T gto, gks;
    bool endo;
    type_constants(p, gto, gks, endo);
    TP06Fluxes<T> c;
    tp06_fluxes(y, p, c, gto, gks);
    return -c.Iion;
  }
  template <typename T>
  __host__ __device__ static void substep(T* y, const T* p, T h, bool clamp) {
    T gto, gks;
    bool endo;
    type_constants(p, gto, gks, endo);
    tp06_substep(y, p, h, clamp, gto, gks, endo);
  }
};

// Myocytes and fibroblasts in one tissue (the paper's fibrotic sheet, Sec.
// 3.2): parameter row 6 holds the node class, 0 an epicardial TP06 myocyte,
// 1 a fibroblast with a passive (linear) membrane dV/dt = -g_f (V - E_f),
// g_f and E_f in rows 7 and 8.  A fibroblast node keeps its other 18 state
// rows unchanged.
struct TP06FibroModel {
  static constexpr int S = 19, P = 9;
  template <typename T>
  __host__ __device__ static bool fibroblast(const T* p) { return p[6] == T(1); }
  template <typename T>
  __host__ __device__ static T vrate(const T* y, const T* p) {
    if (fibroblast(p)) return -p[7] * (y[0] - p[8]);
    TP06Fluxes<T> c;
    tp06_fluxes(y, p, c);
    return -c.Iion;
  }
  template <typename T>
  __host__ __device__ static void substep(T* y, const T* p, T h, bool clamp) {
    if (fibroblast(p)) {
      if (!clamp) y[0] = y[0] + h * (-p[7] * (y[0] - p[8]));
      return;
    }
    tp06_substep(y, p, h, clamp, T(tp06::kGto), T(tp06::kGKs), false);
  }
};

}  // namespace mono
