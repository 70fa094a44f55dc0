// Reverse-mode derivatives (vector-Jacobian products) of one cell-model
// substep, written by hand from the forward code in cell_models.h.
//
// For a substep y' = F(y, p; h) and the adjoint lam' = dL/dy' of its output,
// vjp() overwrites lam with dL/dy = (dF/dy)^T lam' and adds (dF/dp)^T lam'
// to gp.  Univariate pieces (gate steady states and rates as functions of V,
// the K1 rectification as a function of V - E_K, the L-type driving factor)
// are differentiated with a value/derivative pair type; everything else is
// reversed term by term.
#pragma once

#include <type_traits>

#include "cell_models.h"

namespace mono {

// value and derivative with respect to one scalar input
template <typename S>
struct Dual {
  S v, d;
  __host__ __device__ Dual() : v(0), d(0) {}
  __host__ __device__ Dual(S x, S dx) : v(x), d(dx) {}
  template <typename U, typename = typename std::enable_if<std::is_arithmetic<U>::value>::type>
  __host__ __device__ Dual(U x) : v(S(x)), d(S(0)) {}
};
template <typename S>
__host__ __device__ __forceinline__ Dual<S> operator+(Dual<S> a, Dual<S> b) {
  return Dual<S>(a.v + b.v, a.d + b.d);
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S> operator-(Dual<S> a, Dual<S> b) {
  return Dual<S>(a.v - b.v, a.d - b.d);
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S> operator-(Dual<S> a) {
  return Dual<S>(-a.v, -a.d);
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S> operator*(Dual<S> a, Dual<S> b) {
  return Dual<S>(a.v * b.v, a.d * b.v + a.v * b.d);
}
template <typename S>
__host__ __device__ __forceinline__ bool operator>=(Dual<S> a, Dual<S> b) {
  return a.v >= b.v;
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S> xexp(Dual<S> a) {
  const S e = xexp(a.v);
  return Dual<S>(e, e * a.d);
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S> xexp2(Dual<S> a) {
  const S e = xexp2(a.v);
  return Dual<S>(e, e * S(kLn2) * a.d);
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S> xrcp(Dual<S> a) {
  const S r = xrcp(a.v);
  return Dual<S>(r, -r * r * a.d);
}
template <typename S>
__host__ __device__ __forceinline__ Dual<S> xsqrt(Dual<S> a) {
  const S q = xsqrt(a.v);
  return Dual<S>(q, S(0.5) * a.d * xrcp(q));
}

// ---------------------------------------------------------------------------
template <typename T>
__host__ __device__ void linear_substep_vjp(const T* y, const T* p, T h, bool clamp, T* lam,
                                            T* gp) {
  // V' = V - h g (V - E)
  const T l0 = lam[0];
  if (clamp) return;
  lam[0] = l0 * (T(1) - h * p[0]);
  gp[0] += -l0 * h * (y[0] - p[1]);
  gp[1] += l0 * h * p[0];
}

template <typename T>
__host__ __device__ void ms_substep_vjp(const T* y, const T* p, T h, bool clamp, T* lam, T* gp) {
  const T v = y[0], g = y[1];
  const T tin = p[0], tout = p[1];
  const bool open = v < p[4];
  const T hinf = open ? T(1) : T(0);
  const T tau = open ? p[2] : p[3];
  const T rate = xrcp(tau);
  const T E = xexp(-h * rate);
  const T l0 = lam[0], l1 = lam[1];
  // h' = hinf + (h - hinf) E, with E = exp(-h/tau)
  T ag = l1 * E;
  const T dtau = l1 * (g - hinf) * E * h * rate * rate;
  gp[open ? 2 : 3] += dtau;
  T av = T(0);
  if (clamp) {
    av = l0;
  } else {
    // v' = v + h (g v^2 (1-v)/tin - v/tout)
    const T v2 = v * v;
    av = l0 * (T(1) + h * (g * (T(2) * v - T(3) * v2) * xrcp(tin) - xrcp(tout)));
    ag += l0 * h * v2 * (T(1) - v) * xrcp(tin);
    gp[0] += -l0 * h * g * v2 * (T(1) - v) * xrcp(tin * tin);
    gp[1] += l0 * h * v * xrcp(tout * tout);
  }
  lam[0] = av;
  lam[1] = ag;
}

// ---------------------------------------------------------------------------
// TP06: reverse of tp06_substep.  gp[6] adjoints of {Ko, gNa, gCaL, gKr,
// gKs, gK1}; gto, gks and endo as in the forward substep (the cell type's
// I_to and I_Ks conductances and s gate).
template <typename T>
__host__ __device__ void tp06_substep_vjp(const T* y, const T* p, T h, bool clamp, T* lam,
                                          T* gp, T gto = T(tp06::kGto), T gks = T(tp06::kGKs),
                                          bool endo = false) {
  using namespace tp06;
  using D = Dual<T>;
  // ---- forward intermediates ------------------------------------------------
  const T V = y[0], Ki = y[1], Nai = y[2], Cai = y[3], Cass = y[4], CaSR = y[5], Rb = y[6];
  const T m = y[7], hh = y[8], jj = y[9], xr1 = y[10], xr2 = y[11], xs = y[12];
  const T rg = y[13], sg = y[14], dg = y[15], fg = y[16], f2 = y[17], fc = y[18];
  const T Ko = p[0];
  const T rtf = T(kRTF), frt = T(kFRT);
  const T EK = rtf * xlog(xdiv(Ko, Ki));
  const T ENa = rtf * xlog(xdiv(T(kNao), Nai));
  const T nKs = Ko + T(kPKNa * kNao), dKs = Ki + T(kPKNa) * Nai;
  const T EKs = rtf * xlog(xdiv(nKs, dKs));
  const T sqKo = xsqrt(Ko * T(1.0 / 5.4));
  const T m3 = m * m * m;
  const T vk = V - EK;
  D xK1;
  {
    const D z(vk, T(1));
    const D aK1 = D(0.1) * sig(D(0.06) * (z - D(200)));
    const D bK1 = (D(3) * xexp(D(0.0002) * (z + D(100))) + xexp(D(0.1) * (z - D(10)))) *
                  sig(D(-0.5) * z);
    xK1 = aK1 * xrcp(aK1 + bK1);
  }
  D spk;
  {
    const D Vd(V, T(1));
    spk = sig((D(25) - Vd) * D(1.0 / 5.98));
  }
  const T x = T(2) * (V - T(15)) * frt;
  T xe, xe_d;
  if (x == T(0)) {
    xe = T(1);
    xe_d = T(-0.5);
  } else {
    const T em1 = xexpm1(x);
    const T ex1 = em1 + T(1);
    xe = xdiv(x, em1);
    xe_d = xdiv(em1 - x * ex1, em1 * em1);
  }
  const T ex = xexp(x);
  const T Bc = T(0.25) * Cass * ex - T(kCao);
  const T G2F = T(kGCaL * 2.0 * kF);
  const T u = xexp(-V * frt);
  const T eg = xexp(T(kNaCaGam) * V * frt);
  const T eg1 = eg * u;
  const T c3 = T(kNao * kNao * kNao * kNaCaAlpha);
  const T den = T((kKmNai * kKmNai * kKmNai + kNao * kNao * kNao) * (kKmCa + kCao));
  const T Nai3 = Nai * Nai * Nai;
  const T Nn = eg * Nai3 * T(kCao) - eg1 * c3 * Cai;
  const T Dd = den * (T(1) + T(kNaCaSat) * eg1);
  const T w = xexp(T(-0.1) * V * frt);
  const T Q = T(1) + T(0.1245) * w + T(0.0353) * u;
  const T INaK = T(kPNaK) * xdiv(Ko * Nai, (Ko + T(kKmK)) * (Nai + T(kKmNa)) * Q);
  const T r_sr = xdiv(T(kEC), CaSR);
  const T opr = T(1) + r_sr * r_sr;
  const T kcasr = T(kMaxSR) - T(kMaxSR - kMinSR) * xrcp(opr);
  const T k1 = xdiv(T(kK1p), kcasr);
  const T cs2 = Cass * Cass;
  const T z = k1 * cs2;
  const T O = xdiv(z * Rb, T(kK3) + z);
  const T ci2 = Cai * Cai;
  const T cc = T(kCurToConc);
  // concentration slopes (for the buffered updates)
  TP06Fluxes<T> c;
  tp06_fluxes(y, p, c, gto, gks);
  const T dCai = -(c.IbCa + c.IpCa - T(2) * c.INaCa) * T(0.5) * cc +
                 T(kVsr / kVc) * (c.Ileak - c.Iup) + c.Ixfer;
  const T dCass = -c.ICaL * T(kCap / (2.0 * kVss * kF)) + T(kVsr / kVss) * c.Irel -
                  T(kVc / kVss) * c.Ixfer;
  const T dCaSR = c.Iup - c.Ileak - c.Irel;
  const T Cai_n = free_from_total(total_from_free(Cai, T(kBufc), T(kKbufc)) + h * dCai, T(kBufc),
                                  T(kKbufc));
  const T Cass_n = free_from_total(total_from_free(Cass, T(kBufss), T(kKbufss)) + h * dCass,
                                   T(kBufss), T(kKbufss));
  const T CaSR_n = free_from_total(total_from_free(CaSR, T(kBufsr), T(kKbufsr)) + h * dCaSR,
                                   T(kBufsr), T(kKbufsr));
  // gates: steady states and rates with their derivatives
  D ginf[12], grate[12];
  tp06_gate_params(D(V, T(1)), ginf, grate, endo);
  tp06_fcass_params(D(Cass, T(1)), ginf[11], grate[11]);

  // ---- reverse ----------------------------------------------------------------
  const T lV = lam[0], lKi = lam[1], lNai = lam[2], lCai = lam[3], lCass = lam[4];
  const T lCaSR = lam[5], lRb = lam[6];
  T aV = T(0), aKi = T(0), aNai = T(0), aCai = T(0), aCass = T(0), aCaSR = T(0), aRb = T(0);
  T ag[12];
  for (int a = 0; a < 12; ++a) {
    const T E = xexp(-h * grate[a].v);
    const T lg = lam[7 + a];
    ag[a] = lg * E;
    const T dq = lg * (ginf[a].d * (T(1) - E) - h * (y[7 + a] - ginf[a].v) * E * grate[a].d);
    if (a < 11)
      aV += dq;
    else
      aCass += dq;
  }
  // V' = V - h Iion; Ki' = Ki + h dKi; Nai' = Nai + h dNai; Rb' = Rb + h dRb
  aV += lV;
  const T lIion = clamp ? T(0) : -h * lV;
  aKi += lKi;
  const T ldKi = h * lKi;
  aNai += lNai;
  const T ldNai = h * lNai;
  aRb += lRb;
  const T ldRb = h * lRb;
  // buffered calcium: c' = free(total(c) + h dc)
  auto buffered = [&](T c0, T cn, T B, T K, T lout, T& ac, T& ldc) {
    const T lt = lout * xrcp(T(1) + B * K * xrcp((cn + K) * (cn + K)));
    ac += lt * (T(1) + B * K * xrcp((c0 + K) * (c0 + K)));
    ldc = lt * h;
  };
  T ldCai, ldCass, ldCaSR;
  buffered(Cai, Cai_n, T(kBufc), T(kKbufc), lCai, aCai, ldCai);
  buffered(Cass, Cass_n, T(kBufss), T(kKbufss), lCass, aCass, ldCass);
  buffered(CaSR, CaSR_n, T(kBufsr), T(kKbufsr), lCaSR, aCaSR, ldCaSR);
  // slopes -> currents and fluxes
  T lIK = -cc * ldKi;
  T lINaK = T(2) * cc * ldKi - T(3) * cc * ldNai;
  T lINa = -cc * ldNai;
  T lIbNa = -cc * ldNai;
  T lINaCa = -T(3) * cc * ldNai + cc * ldCai;
  T lIbCa = -T(0.5) * cc * ldCai;
  T lIpCa = -T(0.5) * cc * ldCai;
  T lIleak = T(kVsr / kVc) * ldCai - ldCaSR;
  T lIup = -T(kVsr / kVc) * ldCai + ldCaSR;
  T lIxfer = ldCai - T(kVc / kVss) * ldCass;
  T lICaL = -T(kCap / (2.0 * kVss * kF)) * ldCass;
  T lIrel = T(kVsr / kVss) * ldCass - ldCaSR;
  T lkcasr = -T(kK2p) * Cass * Rb * ldRb;
  aCass += -T(kK2p) * kcasr * Rb * ldRb;
  aRb += (-T(kK2p) * kcasr * Cass - T(kK4)) * ldRb;
  // Iion and IK are sums
  lINa += lIion;
  lIK += lIion;
  lICaL += lIion;
  lINaCa += lIion;
  lINaK += lIion;
  lIpCa += lIion;
  lIbNa += lIion;
  lIbCa += lIion;
  const T lIK1 = lIK, lIto = lIK, lIKr = lIK, lIKs = lIK, lIpK = lIK;
  T lENa = T(0), lEK = T(0), lECa = T(0), lEKs = T(0), lvk = T(0), lsqKo = T(0), lKo = T(0);
  // INa = gNa GNa m^3 h j (V - ENa)
  {
    const T base = T(kGNa) * m3 * hh * jj;
    const T vn = V - ENa;
    gp[1] += lINa * base * vn;
    const T q = lINa * p[1] * T(kGNa) * vn;
    ag[0] += q * T(3) * m * m * hh * jj;
    ag[1] += q * m3 * jj;
    ag[2] += q * m3 * hh;
    aV += lINa * p[1] * base;
    lENa -= lINa * p[1] * base;
  }
  aV += lIbNa * T(kGbNa);
  lENa -= lIbNa * T(kGbNa);
  // IK1 = gK1 GK1 sqKo xK1(vk) vk
  gp[5] += lIK1 * T(kGK1) * sqKo * xK1.v * vk;
  lsqKo += lIK1 * p[5] * T(kGK1) * xK1.v * vk;
  lvk += lIK1 * p[5] * T(kGK1) * sqKo * (xK1.v + xK1.d * vk);
  // Ito = Gto r s vk
  ag[6] += lIto * gto * sg * vk;
  ag[7] += lIto * gto * rg * vk;
  lvk += lIto * gto * rg * sg;
  // IKr = gKr GKr sqKo xr1 xr2 vk
  gp[3] += lIKr * T(kGKr) * sqKo * xr1 * xr2 * vk;
  lsqKo += lIKr * p[3] * T(kGKr) * xr1 * xr2 * vk;
  ag[3] += lIKr * p[3] * T(kGKr) * sqKo * xr2 * vk;
  ag[4] += lIKr * p[3] * T(kGKr) * sqKo * xr1 * vk;
  lvk += lIKr * p[3] * T(kGKr) * sqKo * xr1 * xr2;
  // IKs = gKs GKs xs^2 (V - EKs)
  {
    const T ve = V - EKs;
    gp[4] += lIKs * gks * xs * xs * ve;
    ag[5] += lIKs * p[4] * gks * T(2) * xs * ve;
    aV += lIKs * p[4] * gks * xs * xs;
    lEKs -= lIKs * p[4] * gks * xs * xs;
  }
  // IpK = GpK vk sig((25 - V)/5.98)
  lvk += lIpK * T(kGpK) * spk.v;
  aV += lIpK * T(kGpK) * vk * spk.d;
  // vk = V - EK
  aV += lvk;
  lEK -= lvk;
  // ICaL = gCaL G2F d f f2 fCass xe(x) (0.25 Cass e^x - Cao), x = 2 (V - 15) F/RT
  {
    const T dff = G2F * dg * fg * f2 * fc;
    gp[2] += lICaL * dff * xe * Bc;
    const T pre = lICaL * p[2] * G2F * xe * Bc;
    ag[8] += pre * fg * f2 * fc;
    ag[9] += pre * dg * f2 * fc;
    ag[10] += pre * dg * fg * fc;
    ag[11] += pre * dg * fg * f2;
    const T A = p[2] * dff;
    aCass += lICaL * A * xe * T(0.25) * ex;
    const T lx = lICaL * A * (xe_d * Bc + xe * T(0.25) * Cass * ex);
    aV += lx * T(2) * frt;
  }
  // INaCa = kNaCa Nn / Dd and INaK = PNaK Ko Nai / ((Ko+KmK)(Nai+KmNa) Q)
  {
    const T rD = xrcp(Dd);
    const T lNn = lINaCa * T(kNaCaMax) * rD;
    const T lDd = -lINaCa * T(kNaCaMax) * Nn * rD * rD;
    T leg = lNn * Nai3 * T(kCao);
    aNai += lNn * T(3) * eg * Nai * Nai * T(kCao);
    const T leg1 = -lNn * c3 * Cai + lDd * den * T(kNaCaSat);
    aCai += -lNn * eg1 * c3;
    leg += leg1 * u;
    T lu = leg1 * eg;
    lKo += lINaK * INaK * (xrcp(Ko) - xrcp(Ko + T(kKmK)));
    aNai += lINaK * INaK * (xrcp(Nai) - xrcp(Nai + T(kKmNa)));
    const T lQ = -lINaK * INaK * xrcp(Q);
    const T lw = T(0.1245) * lQ;
    lu += T(0.0353) * lQ;
    aV += leg * eg * T(kNaCaGam) * frt - lu * frt * u - lw * T(0.1) * frt * w;
  }
  // IpCa = GpCa Cai/(KpCa + Cai)
  {
    const T s = T(kKpCa) + Cai;
    aCai += lIpCa * T(kGpCa) * T(kKpCa) * xrcp(s * s);
  }
  // IbCa = GbCa (V - ECa)
  aV += lIbCa * T(kGbCa);
  lECa -= lIbCa * T(kGbCa);
  // Irel = Vrel O (CaSR - Cass), O = z Rb/(K3 + z), z = k1 Cass^2, k1 = K1p/kcasr
  {
    const T lO = lIrel * T(kVrel) * (CaSR - Cass);
    aCaSR += lIrel * T(kVrel) * O;
    aCass -= lIrel * T(kVrel) * O;
    const T rz = xrcp(T(kK3) + z);
    const T lz = lO * Rb * T(kK3) * rz * rz;
    aRb += lO * z * rz;
    const T lk1 = lz * cs2;
    aCass += lz * k1 * T(2) * Cass;
    lkcasr += -lk1 * T(kK1p) * xrcp(kcasr * kcasr);
  }
  // kcasr(CaSR) = maxsr - (maxsr - minsr)/(1 + (EC/CaSR)^2)
  aCaSR += lkcasr * (-T(2.0 * (kMaxSR - kMinSR)) * r_sr * r_sr * xrcp(CaSR * opr * opr));
  // Iup = Vmaxup Cai^2/(Cai^2 + Kup^2)
  {
    const T s = ci2 + T(kKup * kKup);
    aCai += lIup * T(kVmaxUp) * T(2) * Cai * T(kKup * kKup) * xrcp(s * s);
  }
  aCaSR += lIleak * T(kVleak);
  aCai -= lIleak * T(kVleak);
  aCass += lIxfer * T(kVxfer);
  aCai -= lIxfer * T(kVxfer);
  // reversal potentials and sqrt(Ko/5.4)
  aNai += -lENa * rtf * xrcp(Nai);
  lKo += lEK * rtf * xrcp(Ko);
  aKi += -lEK * rtf * xrcp(Ki);
  aCai += -lECa * T(0.5) * rtf * xrcp(Cai);
  lKo += lEKs * rtf * xrcp(nKs);
  aKi -= lEKs * rtf * xrcp(dKs);
  aNai -= lEKs * rtf * T(kPKNa) * xrcp(dKs);
  lKo += lsqKo * T(1.0 / (2.0 * 5.4)) * xrcp(sqKo);
  gp[0] += lKo;

  lam[0] = aV;
  lam[1] = aKi;
  lam[2] = aNai;
  lam[3] = aCai;
  lam[4] = aCass;
  lam[5] = aCaSR;
  lam[6] = aRb;
  for (int a = 0; a < 12; ++a) lam[7 + a] = ag[a];
}

// TP06 with cell types: the type row (p[6]) is a label, its adjoint is zero
template <typename T>
__host__ __device__ void tp06_types_substep_vjp(const T* y, const T* p, T h, bool clamp, T* lam,
                                                T* gp) {
  T gto, gks;
  bool endo;
  TP06TypesModel::type_constants(p, gto, gks, endo);
  tp06_substep_vjp(y, p, h, clamp, lam, gp, gto, gks, endo);
}

// Myocytes and fibroblasts: the class row (p[6]) is a label (adjoint 0); a
// fibroblast's substep V' = V - h g_f (V - E_f) leaves the other states
// (and their adjoints) unchanged and feeds the g_f and E_f rows.
template <typename T>
__host__ __device__ void tp06_fibro_substep_vjp(const T* y, const T* p, T h, bool clamp, T* lam,
                                                T* gp) {
  if (TP06FibroModel::fibroblast(p)) {
    if (clamp) return;
    const T l0 = lam[0];
    lam[0] = l0 * (T(1) - h * p[7]);
    gp[7] += -l0 * h * (y[0] - p[8]);
    gp[8] += l0 * h * p[7];
    return;
  }
  tp06_substep_vjp(y, p, h, clamp, lam, gp);
}

}  // namespace mono
