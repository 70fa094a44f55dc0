// Exact operation count of one cell-model substep: the reaction kernel's own
// model templates instantiated on the host with a scalar type that counts
// every arithmetic operation it takes part in.
#include <cmath>
#include <cstring>

#include "cell_models.h"
#include "cell_models_adjoint.h"
#include "mono_internal.h"

namespace {

struct OpCounts {
  long long add = 0, mul = 0, div = 0, exp = 0, log = 0, sqrt = 0, cmp = 0;
};
thread_local OpCounts* g_ops = nullptr;

struct CF {
  double v;
  constexpr CF() : v(0.0) {}
  constexpr CF(double x) : v(x) {}
  CF& operator+=(CF o) {
    g_ops->add++;
    v += o.v;
    return *this;
  }
};
inline CF operator+(CF a, CF b) { g_ops->add++; return CF(a.v + b.v); }
inline CF operator-(CF a, CF b) { g_ops->add++; return CF(a.v - b.v); }
inline CF operator*(CF a, CF b) { g_ops->mul++; return CF(a.v * b.v); }
inline CF operator/(CF a, CF b) { g_ops->div++; return CF(a.v / b.v); }
inline CF operator-(CF a) { return CF(-a.v); }   // sign flip: an operand modifier
inline bool operator<(CF a, CF b) { g_ops->cmp++; return a.v < b.v; }
inline bool operator>=(CF a, CF b) { g_ops->cmp++; return a.v >= b.v; }
inline bool operator==(CF a, CF b) { g_ops->cmp++; return a.v == b.v; }
// found by argument-dependent lookup from the model templates
inline CF xexp(CF x) { g_ops->exp++; return CF(std::exp(x.v)); }
inline CF xexpm1(CF x) { g_ops->exp++; return CF(std::expm1(x.v)); }
inline CF xlog(CF x) { g_ops->log++; return CF(std::log(x.v)); }
inline CF xexp2(CF x) { g_ops->exp++; return CF(std::exp2(x.v)); }
inline CF xlog2(CF x) { g_ops->log++; return CF(std::log2(x.v)); }
inline CF xlog2c(CF x) { g_ops->log++; return CF(std::log2(x.v)); }
inline CF xsqrt(CF x) { g_ops->sqrt++; return CF(std::sqrt(x.v)); }
inline CF xrcp(CF x) { g_ops->div++; return CF(1.0 / x.v); }

}  // namespace

namespace {
template <class M>
void count_substep(const double* y0, const double* p0, OpCounts& c) {
  CF y[M::S], p[M::P];
  for (int a = 0; a < M::S; ++a) y[a] = CF(y0[a]);
  for (int a = 0; a < M::P; ++a) p[a] = CF(p0[a]);
  g_ops = &c;
  M::substep(y, p, CF(0.02), false);
  g_ops = nullptr;
}
}  // namespace

extern "C" mono_status mono_model_flops(int32_t model, const double* state, const double* params,
                                        int64_t* out) {
  if (!state || !params || !out) return MONO_EINVAL;
  OpCounts c;
  if (model == MONO_MODEL_LINEAR)
    count_substep<mono::LinearModel>(state, params, c);
  else if (model == MONO_MODEL_MS)
    count_substep<mono::MSModel>(state, params, c);
  else if (model == MONO_MODEL_TP06_EPI)
    count_substep<mono::TP06Model>(state, params, c);
  else if (model == MONO_MODEL_TP06_TYPES)
    count_substep<mono::TP06TypesModel>(state, params, c);
  else if (model == MONO_MODEL_TP06_FIBRO)
    count_substep<mono::TP06FibroModel>(state, params, c);
  else
    return MONO_EINVAL;
  const long long v[7] = {c.add, c.mul, c.div, c.exp, c.log, c.sqrt, c.cmp};
  for (int a = 0; a < 7; ++a) out[a] = v[a];
  return MONO_OK;
}

// Host evaluation of the kernel's model code in FP64 (diagnostics and tests).
extern "C" mono_status mono_model_substep_host(int32_t model, double* y, const double* p,
                                               double h, int32_t clamp) {
  if (!y || !p || !(h > 0.0)) return MONO_EINVAL;
  if (model == MONO_MODEL_LINEAR)
    mono::LinearModel::substep(y, p, h, clamp != 0);
  else if (model == MONO_MODEL_MS)
    mono::MSModel::substep(y, p, h, clamp != 0);
  else if (model == MONO_MODEL_TP06_EPI)
    mono::TP06Model::substep(y, p, h, clamp != 0);
  else if (model == MONO_MODEL_TP06_TYPES)
    mono::TP06TypesModel::substep(y, p, h, clamp != 0);
  else if (model == MONO_MODEL_TP06_FIBRO)
    mono::TP06FibroModel::substep(y, p, h, clamp != 0);
  else
    return MONO_EINVAL;
  return MONO_OK;
}

extern "C" mono_status mono_model_vjp_host(int32_t model, const double* y, const double* p,
                                           double h, int32_t clamp, double* lam, double* gp) {
  if (!y || !p || !lam || !gp || !(h > 0.0)) return MONO_EINVAL;
  if (model == MONO_MODEL_LINEAR)
    mono::linear_substep_vjp(y, p, h, clamp != 0, lam, gp);
  else if (model == MONO_MODEL_MS)
    mono::ms_substep_vjp(y, p, h, clamp != 0, lam, gp);
  else if (model == MONO_MODEL_TP06_EPI)
    mono::tp06_substep_vjp(y, p, h, clamp != 0, lam, gp);
  else if (model == MONO_MODEL_TP06_TYPES)
    mono::tp06_types_substep_vjp(y, p, h, clamp != 0, lam, gp);
  else if (model == MONO_MODEL_TP06_FIBRO)
    mono::tp06_fibro_substep_vjp(y, p, h, clamp != 0, lam, gp);
  else
    return MONO_EINVAL;
  return MONO_OK;
}
