// FP64 CPU oracle for the dual adaptive explicit time integration (DAETI)
// method of Mountris & Pueyo, "A dual adaptive explicit time integration
// algorithm for efficiently solving the cardiac monodomain equation".
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
// reference the GPU library is checked against.  Only the test suite, the
// smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
// code, header, table or constant with the GPU library.
//
// What it computes (paper Sec. 2):
//   * FE stiffness K and row-sum lumped mass m of the diffusion problem,
//     eq. (2b)-(2c), on Q1 line / quad / hex elements (2^d Gauss points)
//     and on linear triangles and tetrahedra (constant gradients).
//   * The Gershgorin stable step, eq. (3):
//       dt_s = 0.9 * min_i m_ii / (k_ii + sum_{j!=i} |k_ij|)
//     and the diffusion substep count l and dt_ad = dt/(2l) (Sec. 2).
//   * Strang splitting B(dt/2) A(dt) B(dt/2) per outer step (Sec. 2): B is
//     forward Euler on dV/dt = -M^-1 K V + s(t); A advances every node's cell
//     model with k substeps of dt/k, k = min(k0 + floor|dV/dt|, k_max),
//     k0 = 5 if dV/dt > 0 else 1, k_max = floor(dt/dt0) (Sec. 2).
//   * Gates by Rush-Larsen, everything else by forward Euler.
//   * First upward crossing time of a voltage threshold (local activation
//     time, Sec. 3.3), kept in FP64.
//
// Readings of points the paper leaves open are listed in the project's design
// notes; the ones that change arithmetic are restated where they are used.
//
// Cell models:
//   * linear test model   dV/dt = -g (V - E)
//   * Mitchell & Schaeffer, Bull. Math. Biol. 65:767 (2003), two variables.
//   * ten Tusscher & Panfilov, Am. J. Physiol. Heart Circ. Physiol.
//     291:H1088 (2006), epicardial, 19 state variables, with the current
//     formulations carried over from ten Tusscher et al., Am. J. Physiol.
//     286:H1573 (2004); optionally with the endocardial / M-cell variants
//     per node (a seventh parameter).
//     Parity unpinned: the numerical constants of the TP06 rate equations
//     (half-activation voltages, slopes, time-constant fits, conductances).
//     The publication is not at hand, so only properties pin them (rest
//     stability, upstroke, peak and APD90 ranges; for the cell types, the
//     closed-form differences of dV/dt, the s-gate half points and the APD
//     ordering); the GPU library's independent transcription agreeing with
//     this one checks each against the other, not against the publication.
//     The model's structure is pinned: charge and ion balance (every current
//     moves its own ion; forward Euler keeps that linear invariant), every
//     current's zero at its Nernst potential and its outward sign above it,
//     the L-type flux's reversal and removable singularity, the direction
//     and range of every gate, and the membrane current as the sum of its
//     parts.
//
// Build: g++ -O2 -fopenmp -ffp-contract=off -shared -fPIC (see build.py).

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <string>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
std::string g_err;
int fail(const char* msg) { g_err = msg; return -1; }

// ---------------------------------------------------------------------------
// finite elements: Q1 shape functions on [-1,1]^d, 2-point Gauss rule
// ---------------------------------------------------------------------------
// Reference coordinates of the element nodes, in the ordering of the mesh
// description (line: x-,x+; quad: counter-clockwise; hex: z- face then z+).
const double REF_LINE[2][1] = {{-1}, {1}};
const double REF_QUAD[4][2] = {{-1, -1}, {1, -1}, {1, 1}, {-1, 1}};
const double REF_HEX[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                              {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

double ref_coord(int nen, int a, int d) {
  if (nen == 2) return REF_LINE[a][d];
  if (nen == 4) return REF_QUAD[a][d];
  return REF_HEX[a][d];
}

// N_a(xi) = prod_d (1 + xi_d xa_d)/2 and its xi-gradient.
void shape(int dim, int nen, const double* xi, double* N, double* dN /* nen*dim */) {
  for (int a = 0; a < nen; ++a) {
    double f[3];
    for (int d = 0; d < dim; ++d) f[d] = 0.5 * (1.0 + xi[d] * ref_coord(nen, a, d));
    double p = 1.0;
    for (int d = 0; d < dim; ++d) p *= f[d];
    N[a] = p;
    for (int d = 0; d < dim; ++d) {
      double g = 0.5 * ref_coord(nen, a, d);
      for (int e = 0; e < dim; ++e)
        if (e != d) g *= f[e];
      dN[a * dim + d] = g;
    }
  }
}

// Inverse and determinant of a dim x dim matrix (dim <= 3), row-major.
double invert(int dim, const double* A, double* Ai) {
  if (dim == 1) {
    Ai[0] = 1.0 / A[0];
    return A[0];
  }
  if (dim == 2) {
    double det = A[0] * A[3] - A[1] * A[2];
    Ai[0] = A[3] / det;
    Ai[1] = -A[1] / det;
    Ai[2] = -A[2] / det;
    Ai[3] = A[0] / det;
    return det;
  }
  double c00 = A[4] * A[8] - A[5] * A[7];
  double c01 = A[5] * A[6] - A[3] * A[8];
  double c02 = A[3] * A[7] - A[4] * A[6];
  double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  Ai[0] = c00 / det;
  Ai[1] = (A[2] * A[7] - A[1] * A[8]) / det;
  Ai[2] = (A[1] * A[5] - A[2] * A[4]) / det;
  Ai[3] = c01 / det;
  Ai[4] = (A[0] * A[8] - A[2] * A[6]) / det;
  Ai[5] = (A[2] * A[3] - A[0] * A[5]) / det;
  Ai[6] = c02 / det;
  Ai[7] = (A[1] * A[6] - A[0] * A[7]) / det;
  Ai[8] = (A[0] * A[4] - A[1] * A[3]) / det;
  return det;
}

// Linear simplex (triangle, tetrahedron) with nodes x_0..x_dim: on it
// x - x_0 = E^T lambda for E's rows x_a - x_0 (a = 1..dim), so the gradient
// of the barycentric coordinate lambda_a is column a-1 of E^-1 and that of
// lambda_0 minus their sum; all constant.  Ke[a][b] = vol grad l_a . D
// grad l_b, me[a] = vol / (dim + 1) (int lambda_a over the simplex).
int simplex_matrices(int dim, const double* X, const double* D, double* Ke, double* me) {
  const int nen = dim + 1;
  double E[9], Ei[9];
  for (int r = 0; r < dim; ++r)
    for (int c = 0; c < dim; ++c) E[r * dim + c] = X[(r + 1) * dim + c] - X[c];
  const double det = invert(dim, E, Ei);
  if (!(det > 0.0)) return -1;
  const double vol = det / (dim == 2 ? 2.0 : 6.0);
  double G[4][3];
  for (int c = 0; c < dim; ++c) {
    G[0][c] = 0.0;
    for (int a = 1; a < nen; ++a) {
      G[a][c] = Ei[c * dim + (a - 1)];
      G[0][c] -= G[a][c];
    }
  }
  for (int a = 0; a < nen; ++a) {
    me[a] = vol / nen;
    for (int b = 0; b < nen; ++b) {
      double sum = 0.0;
      for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) sum += G[a][i] * D[i * dim + j] * G[b][j];
      Ke[a * nen + b] = vol * sum;
    }
  }
  return 0;
}

// Element stiffness Ke[a][b] = int grad N_a . D grad N_b and lumped mass
// me[a] = int N_a (the row sum of the consistent mass, since sum_b N_b = 1).
int element_matrices(int dim, int nen, const double* X /* nen*dim */, const double* D,
                     double* Ke, double* me) {
  const double g = 1.0 / std::sqrt(3.0);
  const int nq = 1 << dim;
  for (int i = 0; i < nen * nen; ++i) Ke[i] = 0.0;
  for (int a = 0; a < nen; ++a) me[a] = 0.0;
  for (int q = 0; q < nq; ++q) {
    double xi[3];
    for (int d = 0; d < dim; ++d) xi[d] = ((q >> d) & 1) ? g : -g;
    double N[8], dN[24];
    shape(dim, nen, xi, N, dN);
    // J[d][e] = dx_e / dxi_d
    double J[9] = {0}, Ji[9];
    for (int d = 0; d < dim; ++d)
      for (int e = 0; e < dim; ++e) {
        double s = 0.0;
        for (int a = 0; a < nen; ++a) s += dN[a * dim + d] * X[a * dim + e];
        J[d * dim + e] = s;
      }
    double detJ = invert(dim, J, Ji);
    if (!(detJ > 0.0)) return -1;
    // grad_x N_a = J^-1 grad_xi N_a
    double G[24];
    for (int a = 0; a < nen; ++a)
      for (int e = 0; e < dim; ++e) {
        double s = 0.0;
        for (int d = 0; d < dim; ++d) s += Ji[e * dim + d] * dN[a * dim + d];
        G[a * dim + e] = s;
      }
    for (int a = 0; a < nen; ++a) {
      me[a] += N[a] * detJ;
      for (int b = 0; b < nen; ++b) {
        double s = 0.0;
        for (int d = 0; d < dim; ++d)
          for (int e = 0; e < dim; ++e) s += G[a * dim + d] * D[d * dim + e] * G[b * dim + e];
        Ke[a * nen + b] += s * detJ;
      }
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// forward-mode derivatives: a value and its N partial derivatives
// ---------------------------------------------------------------------------
template <int N>
struct DualN {
  double v;
  double d[N];
  DualN() : v(0.0) {
    for (int k = 0; k < N; ++k) d[k] = 0.0;
  }
  DualN(double x) : v(x) {
    for (int k = 0; k < N; ++k) d[k] = 0.0;
  }
};
template <int N> DualN<N> operator+(const DualN<N>& a, const DualN<N>& b) {
  DualN<N> r(a.v + b.v);
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N> DualN<N> operator-(const DualN<N>& a, const DualN<N>& b) {
  DualN<N> r(a.v - b.v);
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N> DualN<N> operator-(const DualN<N>& a) {
  DualN<N> r(-a.v);
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N> DualN<N> operator*(const DualN<N>& a, const DualN<N>& b) {
  DualN<N> r(a.v * b.v);
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int N> DualN<N> operator/(const DualN<N>& a, const DualN<N>& b) {
  DualN<N> r(a.v / b.v);
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
template <int N> DualN<N> operator+(const DualN<N>& a, double b) { return a + DualN<N>(b); }
template <int N> DualN<N> operator+(double a, const DualN<N>& b) { return DualN<N>(a) + b; }
template <int N> DualN<N> operator-(const DualN<N>& a, double b) { return a - DualN<N>(b); }
template <int N> DualN<N> operator-(double a, const DualN<N>& b) { return DualN<N>(a) - b; }
template <int N> DualN<N> operator*(const DualN<N>& a, double b) { return a * DualN<N>(b); }
template <int N> DualN<N> operator*(double a, const DualN<N>& b) { return DualN<N>(a) * b; }
template <int N> DualN<N> operator/(const DualN<N>& a, double b) { return a / DualN<N>(b); }
template <int N> DualN<N> operator/(double a, const DualN<N>& b) { return DualN<N>(a) / b; }
template <int N> bool operator<(const DualN<N>& a, const DualN<N>& b) { return a.v < b.v; }
template <int N> bool operator<(const DualN<N>& a, double b) { return a.v < b; }
template <int N> bool operator>=(const DualN<N>& a, double b) { return a.v >= b; }
template <int N> bool operator==(const DualN<N>& a, double b) { return a.v == b; }
template <int N> DualN<N> exp(const DualN<N>& a) {
  DualN<N> r(std::exp(a.v));
  for (int k = 0; k < N; ++k) r.d[k] = r.v * a.d[k];
  return r;
}
template <int N> DualN<N> expm1(const DualN<N>& a) {
  DualN<N> r(std::expm1(a.v));
  const double e = std::exp(a.v);
  for (int k = 0; k < N; ++k) r.d[k] = e * a.d[k];
  return r;
}
template <int N> DualN<N> log(const DualN<N>& a) {
  DualN<N> r(std::log(a.v));
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] / a.v;
  return r;
}
template <int N> DualN<N> sqrt(const DualN<N>& a) {
  DualN<N> r(std::sqrt(a.v));
  for (int k = 0; k < N; ++k) r.d[k] = 0.5 * a.d[k] / r.v;
  return r;
}

// ---------------------------------------------------------------------------
// cell models
// ---------------------------------------------------------------------------
// M_TP06T is TP06 with the transmural cell type as a seventh parameter
// (0 epicardial, 1 endocardial, 2 mid-myocardial); M_TP06 is the epicardial
// cell alone.  M_TP06F mixes epicardial myocytes and fibroblasts in one
// tissue (Sec. 3.2): parameter 6 is the node class (0 myocyte, 1
// fibroblast), parameters 7 and 8 the rate g_f and reversal potential E_f of
// the fibroblast's passive membrane.
enum { M_LINEAR = 0, M_MS = 1, M_TP06 = 2, M_TP06T = 3, M_TP06F = 4 };
// largest state and parameter counts over the models (buffer sizes)
constexpr int kMaxStates = 19, kMaxParams = 9;

bool is_tp06(int m) { return m == M_TP06 || m == M_TP06T || m == M_TP06F; }
// cell type stored as a parameter value (checked to be 0, 1 or 2 on input)
int cell_type(double v) { return v == 1.0 ? 1 : (v == 2.0 ? 2 : 0); }
template <int N>
int cell_type(const DualN<N>& v) { return cell_type(v.v); }
int model_nstates(int m) { return m == M_LINEAR ? 1 : (m == M_MS ? 2 : 19); }
int model_nparams(int m) {
  return m == M_LINEAR ? 2 : (m == M_MS ? 5 : (m == M_TP06 ? 6 : (m == M_TP06T ? 7 : 9)));
}

// Rates of one cell.  For every state y the model reports either a forward
// Euler slope (is_gate = 0: rate = dy/dt) or Rush-Larsen data (is_gate = 1:
// inf = y_inf, tau = time constant).  State 0 is always V.
template <typename Num>
struct Rates {
  Num rate[19];
  Num inf[19];
  Num tau[19];
  int is_gate[19];
  // Ca buffering: slopes of the *total* concentrations of states 3,4,5
  int buffered;
};

// Linear test model: dV/dt = -g (V - E).   p = {g, E}
template <typename Num>
void rates_linear(const Num* y, const Num* p, Rates<Num>& r) {
  r.buffered = 0;
  r.is_gate[0] = 0;
  r.rate[0] = -p[0] * (y[0] - p[1]);
}

// Passive fibroblast of the mixed tissue: dV/dt = -g_f (V - E_f) with
// p[7] = g_f, p[8] = E_f; its other (TP06-sized) states do not move.
template <typename Num>
void rates_fibroblast(const Num* y, const Num* p, Rates<Num>& r) {
  r.buffered = 0;
  for (int i = 0; i < 19; ++i) {
    r.is_gate[i] = 0;
    r.rate[i] = 0.0;
  }
  r.rate[0] = -p[7] * (y[0] - p[8]);
}

// Mitchell-Schaeffer: dv/dt = h v^2 (1-v)/tau_in - v/tau_out,
// dh/dt = (1-h)/tau_open if v < v_gate, else -h/tau_close.
// p = {tau_in, tau_out, tau_open, tau_close, v_gate}.  The gate is written in
// Rush-Larsen form: h_inf = 1 (tau_open) below v_gate, 0 (tau_close) at or
// above it.
template <typename Num>
void rates_ms(const Num* y, const Num* p, Rates<Num>& r) {
  using std::exp;
  Num v = y[0], h = y[1];
  r.buffered = 0;
  r.is_gate[0] = 0;
  r.rate[0] = h * v * v * (1.0 - v) / p[0] - v / p[1];
  r.is_gate[1] = 1;
  if (v < p[4]) {
    r.inf[1] = 1.0;
    r.tau[1] = p[2];
  } else {
    r.inf[1] = 0.0;
    r.tau[1] = p[3];
  }
}

// --- ten Tusscher-Panfilov 2006, epicardial --------------------------------
// state order: 0 V, 1 K_i, 2 Na_i, 3 Ca_i, 4 Ca_ss, 5 Ca_SR, 6 Rbar,
//              7 m, 8 h, 9 j, 10 xr1, 11 xr2, 12 xs, 13 r, 14 s,
//              15 d, 16 f, 17 f2, 18 fCass
// p = {Ko, scale gNa, scale gCaL, scale gKr, scale gKs, scale gK1}
namespace tp {
const double R = 8314.472, T = 310.0, F = 96485.3415;
const double Cm = 0.185;                 // uF, cell capacitance
const double Vc = 0.016404, Vsr = 0.001094, Vss = 0.00005468;  // nL
const double Nao = 140.0, Cao = 2.0;
const double GNa = 14.838, GK1 = 5.405, Gto = 0.294, GKr = 0.153, GKs = 0.392;
const double pKNa = 0.03;
const double GCaL = 3.980e-5;
const double kNaCa = 1000.0, gam = 0.35, KmCa = 1.38, KmNai = 87.5, ksat = 0.1, alf = 2.5;
const double PNaK = 2.724, KmK = 1.0, KmNa = 40.0;
const double GpK = 0.0146, GpCa = 0.1238, KpCa = 0.0005;
const double GbNa = 0.00029, GbCa = 0.000592;
const double Vmaxup = 0.006375, Kup = 0.00025;
const double Vrel = 0.102, k1p = 0.15, k2p = 0.045, k3 = 0.060, k4 = 0.005;
const double EC = 1.5, maxsr = 2.5, minsr = 1.0;
const double Vleak = 0.00036, Vxfer = 0.0038;
const double Bufc = 0.2, Kbufc = 0.001;
const double Bufsr = 10.0, Kbufsr = 0.3;
const double Bufss = 0.4, Kbufss = 0.00025;

// Published initial values of the model's code release (not pre-paced).
const double INIT[19] = {-86.2, 138.3, 7.67, 0.00007, 0.00007, 1.3, 1.0,
                         0.0,   0.75,  0.75, 0.0,     1.0,     0.0, 0.0,
                         1.0,   0.0,   1.0,  1.0,     1.0};
}  // namespace tp

// Ionic currents of TP06 (pA/pF) at state y; also used by qualitative tests.
template <typename Num>
struct TPCurrents {
  Num INa, IK1, Ito, IKr, IKs, ICaL, INaCa, INaK, IpCa, IpK, IbNa, IbCa;
  Num Irel, Iup, Ileak, Ixfer;
  Num Iion;
};

template <typename Num>
void tp06_currents(const Num* y, const Num* p, TPCurrents<Num>& c, int type = 0) {
  using std::exp;
  using std::expm1;
  using std::log;
  using std::sqrt;
  using namespace tp;
  const Num V = y[0], Ki = y[1], Nai = y[2], Cai = y[3], Cass = y[4], CaSR = y[5],
               Rb = y[6];
  const Num m = y[7], h = y[8], j = y[9], xr1 = y[10], xr2 = y[11], xs = y[12];
  const Num r = y[13], s = y[14], d = y[15], f = y[16], f2 = y[17], fcass = y[18];
  const Num Ko = p[0];
  const Num RTF = R * T / F;
  const Num EK = RTF * log(Ko / Ki);
  const Num ENa = RTF * log(Nao / Nai);
  const Num ECa = 0.5 * RTF * log(Cao / Cai);
  const Num EKs = RTF * log((Ko + pKNa * Nao) / (Ki + pKNa * Nai));

  c.INa = p[1] * GNa * m * m * m * h * j * (V - ENa);

  const Num aK1 = 0.1 / (1.0 + exp(0.06 * (V - EK - 200.0)));
  const Num bK1 = (3.0 * exp(0.0002 * (V - EK + 100.0)) + exp(0.1 * (V - EK - 10.0))) /
                     (1.0 + exp(-0.5 * (V - EK)));
  const Num xK1 = aK1 / (aK1 + bK1);
  c.IK1 = p[5] * GK1 * sqrt(Ko / 5.4) * xK1 * (V - EK);

  // ten Tusscher-Panfilov 2006 cell types: endocardial cells carry a smaller
  // transient outward current, mid-myocardial cells a smaller slow delayed
  // rectifier; everything else is shared.
  const double gto = type == 1 ? 0.073 : Gto;
  const double gks = type == 2 ? 0.098 : GKs;
  c.Ito = gto * r * s * (V - EK);
  c.IKr = p[3] * GKr * sqrt(Ko / 5.4) * xr1 * xr2 * (V - EK);
  c.IKs = p[4] * gks * xs * xs * (V - EKs);

  // L-type current; x/(e^x - 1) -> 1 at x = 0 (removable singularity at V=15)
  const Num x = 2.0 * (V - 15.0) * F / (R * T);
  const Num xe = (x == 0.0) ? 1.0 : x / expm1(x);
  // 4 (V-15) F^2/(RT) (0.25 Cass e^x - Cao)/(e^x - 1) = 2 F (x/(e^x-1)) (0.25 Cass e^x - Cao)
  c.ICaL = p[2] * GCaL * d * f * f2 * fcass * 2.0 * F * xe * (0.25 * Cass * exp(x) - Cao);

  const Num eg = exp(gam * V * F / (R * T));
  const Num eg1 = exp((gam - 1.0) * V * F / (R * T));
  c.INaCa = kNaCa * (eg * Nai * Nai * Nai * Cao - eg1 * Nao * Nao * Nao * Cai * alf) /
            ((KmNai * KmNai * KmNai + Nao * Nao * Nao) * (KmCa + Cao) * (1.0 + ksat * eg1));
  c.INaK = PNaK * Ko * Nai /
           ((Ko + KmK) * (Nai + KmNa) *
            (1.0 + 0.1245 * exp(-0.1 * V * F / (R * T)) + 0.0353 * exp(-V * F / (R * T))));
  c.IpCa = GpCa * Cai / (KpCa + Cai);
  c.IpK = GpK * (V - EK) / (1.0 + exp((25.0 - V) / 5.98));
  c.IbNa = GbNa * (V - ENa);
  c.IbCa = GbCa * (V - ECa);

  const Num kcasr = maxsr - (maxsr - minsr) / (1.0 + (EC / CaSR) * (EC / CaSR));
  const Num k1 = k1p / kcasr;
  const Num O = k1 * Cass * Cass * Rb / (k3 + k1 * Cass * Cass);
  c.Irel = Vrel * O * (CaSR - Cass);
  c.Iup = Vmaxup / (1.0 + Kup * Kup / (Cai * Cai));
  c.Ileak = Vleak * (CaSR - Cai);
  c.Ixfer = Vxfer * (Cass - Cai);

  c.Iion = c.INa + c.IK1 + c.Ito + c.IKr + c.IKs + c.ICaL + c.INaCa + c.INaK + c.IpCa + c.IpK +
           c.IbNa + c.IbCa;
}

template <typename Num>
void rates_tp06(const Num* y, const Num* p, Rates<Num>& r, int type = 0) {
  using std::exp;
  using std::sqrt;
  using namespace tp;
  TPCurrents<Num> c;
  tp06_currents(y, p, c, type);
  const Num V = y[0], Cass = y[4], CaSR = y[5], Rb = y[6];

  for (int i = 0; i < 7; ++i) r.is_gate[i] = 0;
  for (int i = 7; i < 19; ++i) r.is_gate[i] = 1;
  r.buffered = 1;

  r.rate[0] = -c.Iion;
  r.rate[1] = -(c.IK1 + c.Ito + c.IKr + c.IKs - 2.0 * c.INaK + c.IpK) * Cm / (Vc * F);
  r.rate[2] = -(c.INa + c.IbNa + 3.0 * c.INaK + 3.0 * c.INaCa) * Cm / (Vc * F);
  // slopes of total (free + buffered) calcium in cytosol, subspace and SR
  r.rate[3] = -(c.IbCa + c.IpCa - 2.0 * c.INaCa) * Cm / (2.0 * Vc * F) +
              (Vsr / Vc) * (c.Ileak - c.Iup) + c.Ixfer;
  r.rate[4] = -c.ICaL * Cm / (2.0 * Vss * F) + (Vsr / Vss) * c.Irel - (Vc / Vss) * c.Ixfer;
  r.rate[5] = c.Iup - c.Ileak - c.Irel;
  const Num kcasr = maxsr - (maxsr - minsr) / (1.0 + (EC / CaSR) * (EC / CaSR));
  const Num k2 = k2p * kcasr;
  r.rate[6] = -k2 * Cass * Rb + k4 * (1.0 - Rb);

  // m
  {
    Num e = 1.0 / (1.0 + exp((-56.86 - V) / 9.03));
    r.inf[7] = e * e;
    Num am = 1.0 / (1.0 + exp((-60.0 - V) / 5.0));
    Num bm = 0.1 / (1.0 + exp((V + 35.0) / 5.0)) + 0.10 / (1.0 + exp((V - 50.0) / 200.0));
    r.tau[7] = am * bm;
  }
  // h, j
  {
    Num e = 1.0 / (1.0 + exp((V + 71.55) / 7.43));
    r.inf[8] = e * e;
    r.inf[9] = e * e;
    Num ah, bh, aj, bj;
    if (V >= -40.0) {
      ah = 0.0;
      bh = 0.77 / (0.13 * (1.0 + exp(-(V + 10.66) / 11.1)));
      aj = 0.0;
      bj = 0.6 * exp(0.057 * V) / (1.0 + exp(-0.1 * (V + 32.0)));
    } else {
      ah = 0.057 * exp(-(V + 80.0) / 6.8);
      bh = 2.7 * exp(0.079 * V) + 3.1e5 * exp(0.3485 * V);
      aj = (-2.5428e4 * exp(0.2444 * V) - 6.948e-6 * exp(-0.04391 * V)) * (V + 37.78) /
           (1.0 + exp(0.311 * (V + 79.23)));
      bj = 0.02424 * exp(-0.01052 * V) / (1.0 + exp(-0.1378 * (V + 40.14)));
    }
    r.tau[8] = 1.0 / (ah + bh);
    r.tau[9] = 1.0 / (aj + bj);
  }
  // xr1, xr2
  {
    r.inf[10] = 1.0 / (1.0 + exp((-26.0 - V) / 7.0));
    Num a = 450.0 / (1.0 + exp((-45.0 - V) / 10.0));
    Num b = 6.0 / (1.0 + exp((V + 30.0) / 11.5));
    r.tau[10] = a * b;
    r.inf[11] = 1.0 / (1.0 + exp((V + 88.0) / 24.0));
    a = 3.0 / (1.0 + exp((-60.0 - V) / 20.0));
    b = 1.12 / (1.0 + exp((V - 60.0) / 20.0));
    r.tau[11] = a * b;
  }
  // xs
  {
    r.inf[12] = 1.0 / (1.0 + exp((-5.0 - V) / 14.0));
    Num a = 1400.0 / sqrt(1.0 + exp((5.0 - V) / 6.0));
    Num b = 1.0 / (1.0 + exp((V - 35.0) / 15.0));
    r.tau[12] = a * b + 80.0;
  }
  // r, s (the s gate of endocardial cells inactivates more slowly)
  {
    r.inf[13] = 1.0 / (1.0 + exp((20.0 - V) / 6.0));
    r.tau[13] = 9.5 * exp(-(V + 40.0) * (V + 40.0) / 1800.0) + 0.8;
    if (type == 1) {
      r.inf[14] = 1.0 / (1.0 + exp((V + 28.0) / 5.0));
      r.tau[14] = 1000.0 * exp(-(V + 67.0) * (V + 67.0) / 1000.0) + 8.0;
    } else {
      r.inf[14] = 1.0 / (1.0 + exp((V + 20.0) / 5.0));
      r.tau[14] = 85.0 * exp(-(V + 45.0) * (V + 45.0) / 320.0) +
                  5.0 / (1.0 + exp((V - 20.0) / 5.0)) + 3.0;
    }
  }
  // d, f, f2, fCass
  {
    r.inf[15] = 1.0 / (1.0 + exp((-8.0 - V) / 7.5));
    Num a = 1.4 / (1.0 + exp((-35.0 - V) / 13.0)) + 0.25;
    Num b = 1.4 / (1.0 + exp((V + 5.0) / 5.0));
    Num g = 1.0 / (1.0 + exp((50.0 - V) / 20.0));
    r.tau[15] = a * b + g;

    r.inf[16] = 1.0 / (1.0 + exp((V + 20.0) / 7.0));
    a = 1102.5 * exp(-(V + 27.0) * (V + 27.0) / 225.0);
    b = 200.0 / (1.0 + exp((13.0 - V) / 10.0));
    g = 180.0 / (1.0 + exp((V + 30.0) / 10.0)) + 20.0;
    r.tau[16] = a + b + g;

    r.inf[17] = 0.67 / (1.0 + exp((V + 35.0) / 7.0)) + 0.33;
    a = 600.0 * exp(-(V + 25.0) * (V + 25.0) / 170.0);
    b = 31.0 / (1.0 + exp((25.0 - V) / 10.0));
    g = 16.0 / (1.0 + exp((V + 30.0) / 10.0));
    r.tau[17] = a + b + g;

    Num q = (Cass / 0.05) * (Cass / 0.05);
    r.inf[18] = 0.6 / (1.0 + q) + 0.4;
    r.tau[18] = 80.0 / (1.0 + q) + 2.0;
  }
}

// Free concentration c >= 0 whose total c + B c/(c + K) equals `total`:
// the positive root of c^2 + (B + K - total) c - K total = 0.
template <typename Num>
Num free_from_total(Num total, double B, double K) {
  using std::sqrt;
  Num b = B + K - total;
  return 0.5 * (-b + sqrt(b * b + 4.0 * K * total));
}
template <typename Num>
Num total_from_free(Num c, double B, double K) { return c + B * c / (c + K); }

template <typename Num>
void model_rates(int model, const Num* y, const Num* p, Rates<Num>& r) {
  if (model == M_LINEAR)
    rates_linear(y, p, r);
  else if (model == M_MS)
    rates_ms(y, p, r);
  else if (model == M_TP06)
    rates_tp06(y, p, r);
  else if (model == M_TP06F && cell_type(p[6]) == 1)
    rates_fibroblast(y, p, r);
  else if (model == M_TP06F)
    rates_tp06(y, p, r);
  else
    rates_tp06(y, p, r, cell_type(p[6]));
}

// One substep of length h from y (all rates taken at the substep start):
// Rush-Larsen for gates, forward Euler for the rest (TP06 calcium through its
// buffered totals).  If vclamp, V is held.
template <typename Num>
void cell_substep(int model, Num* y, const Num* p, double h, int vclamp) {
  using std::exp;
  Rates<Num> r;
  model_rates(model, y, p, r);
  const int S = model_nstates(model);
  Num yn[19];
  for (int i = 0; i < S; ++i) {
    if (r.is_gate[i]) {
      yn[i] = r.inf[i] + (y[i] - r.inf[i]) * exp(-h / r.tau[i]);
    } else if (r.buffered && i == 3) {
      yn[i] = free_from_total(total_from_free(y[i], tp::Bufc, tp::Kbufc) + h * r.rate[i], tp::Bufc,
                              tp::Kbufc);
    } else if (r.buffered && i == 4) {
      yn[i] = free_from_total(total_from_free(y[i], tp::Bufss, tp::Kbufss) + h * r.rate[i],
                              tp::Bufss, tp::Kbufss);
    } else if (r.buffered && i == 5) {
      yn[i] = free_from_total(total_from_free(y[i], tp::Bufsr, tp::Kbufsr) + h * r.rate[i],
                              tp::Bufsr, tp::Kbufsr);
    } else {
      yn[i] = y[i] + h * r.rate[i];
    }
  }
  if (vclamp) yn[0] = y[0];
  for (int i = 0; i < S; ++i) y[i] = yn[i];
}

// Reaction substep count (Sec. 2): k0 = 5 for dV/dt > 0, else 1;
// k = k0 + floor|dV/dt|, capped at k_max.
int k_rule(double dvdt, int k_max) {
  double k0 = dvdt > 0.0 ? 5.0 : 1.0;
  double k = k0 + std::floor(std::fabs(dvdt));
  if (!(k <= (double)k_max)) return k_max;   // also catches NaN
  return (int)k;
}

// Diffusion substep count (Sec. 2): l = floor(dt/(2 dt_s)) when dt/2 > dt_s,
// else 1.  l_round = 1 selects the ceiling instead (dt_ad <= dt_s).
int l_rule(double dt, double dt_s, int l_round) {
  if (!(0.5 * dt > dt_s)) return 1;
  double x = dt / (2.0 * dt_s);
  double l = l_round ? std::ceil(x) : std::floor(x);
  if (l < 1.0) l = 1.0;
  return (int)l;
}

// ---------------------------------------------------------------------------
// simulation
// ---------------------------------------------------------------------------
struct Stim {
  std::vector<int32_t> nodes;
  double t_on, dur, amp;
};

struct Sim {
  int dim = 0, nen = 0;
  int64_t n = 0;
  // CSR of K (with diagonal), lumped mass
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  std::vector<double> mass;
  // instances
  std::vector<int64_t> inst_off;   // n_inst + 1
  std::vector<int32_t> inst_of;    // node -> instance
  // model
  int model = -1;
  int S = 0, P = 0;
  std::vector<double> state;       // S * n, SoA (state 0 = V)
  std::vector<double> params;      // P * n, SoA
  std::vector<double> vprev;       // n
  std::vector<double> lat;         // n, -1 = not activated
  std::vector<int32_t> lastk;      // n
  double lat_thr = 0.0;
  double dt0 = 0.01;
  std::vector<Stim> stims;
  std::vector<double> stim_rate;   // n, scratch
  // method
  int method = 0;      // 0 DAETI, 1 OSTAR (l = 1), 2 OST (k = 1, l = 1)
  int dvdt_src = 0;    // 0: (V_b^n - V_b^{n-1})/dt ; 1: reaction rate at A-entry
  int l_round = 0;     // 0 floor, 1 ceil
  int vclamp = 0;
  // time discretisation
  double dt = -1.0;
  std::vector<double> dt_s, gmax;  // per instance
  std::vector<int> l;              // per instance
  std::vector<double> dt_ad;       // per instance
  int k_max = 1;
  int64_t step = 0;
  // k trace
  int ktrace_mode = 0;             // 0 off, 1 record, 2 replay
  uint8_t* ktrace = nullptr;
  double* dtrace = nullptr;
  int64_t ktrace_steps = 0;
  // sensors: record V at A-entry of every step
  std::vector<int32_t> sensors;
  double* sensor_buf = nullptr;
  int64_t sensor_steps = 0;
  std::vector<double> vtmp;
  // adjoint: unscaled stiffness, loss target and the taped forward run
  std::vector<double> val0;        // K before the per-node conductivity scaling
  std::vector<int32_t> tsens;      // loss sensors
  std::vector<double> target;      // n_steps x sensors
  int64_t target_steps = 0;
  bool taped = false;
  int64_t tape_step0 = 0, tape_steps = 0;
  std::vector<double> tape_vsub;   // per step: 2*lmax substep inputs of n values
  std::vector<double> tape_entry;  // per step: S*n reaction-entry states
  std::vector<uint8_t> tape_k;     // per step: n
};

int prepare(Sim* s, double dt) {
  if (!(dt > 0.0)) return fail("dt must be positive");
  int ni = (int)s->inst_off.size() - 1;
  s->dt = dt;
  s->dt_s.assign(ni, 0.0);
  s->gmax.assign(ni, 0.0);
  s->l.assign(ni, 1);
  s->dt_ad.assign(ni, 0.0);
  for (int q = 0; q < ni; ++q) {
    // eq. (3): dt_s = 0.9 min_i m_ii / (k_ii + sum_{j != i} |k_ij|)
    double rmin = INFINITY, gm = 0.0;
    for (int64_t i = s->inst_off[q]; i < s->inst_off[q + 1]; ++i) {
      double kii = 0.0, off = 0.0;
      for (int64_t p = s->rowptr[i]; p < s->rowptr[i + 1]; ++p) {
        if (s->col[p] == i)
          kii += s->val[p];
        else
          off += std::fabs(s->val[p]);
      }
      double r = s->mass[i] / (kii + off);
      if (r < rmin) rmin = r;
      double g = (kii + off) / s->mass[i];
      if (g > gm) gm = g;
    }
    s->dt_s[q] = 0.9 * rmin;
    s->gmax[q] = gm;
    int l = l_rule(dt, s->dt_s[q], s->l_round);
    if (s->method != 0) l = 1;
    s->l[q] = l;
    s->dt_ad[q] = dt / (2.0 * l);
  }
  double km = std::floor(dt / s->dt0);
  s->k_max = km < 1.0 ? 1 : (int)km;
  if (s->method == 2) s->k_max = 1;
  return 0;
}

// Stimulus rate of node i at substep start time tau: the sum of the
// amplitudes of the stimuli that contain i and are on at tau.
double stim_rate_at(const Sim* s, int64_t i, double tau) {
  double r = 0.0;
  for (const Stim& st : s->stims) {
    if (!(st.t_on <= tau && tau < st.t_on + st.dur)) continue;
    if (std::binary_search(st.nodes.begin(), st.nodes.end(), (int32_t)i)) r += st.amp;
  }
  return r;
}

// Row i of diffusion substep m of a half step starting at t0:
// V_i + dt_ad (-(K V)_i / m_i + s_i(tau)), tau = t0 + m dt_ad.
double diffusion_row(const Sim* s, const double* V, int64_t i, int m, double t0,
                     double stim_rate) {
  int q = s->inst_of[i];
  if (m >= s->l[q]) return V[i];
  double kv = 0.0;
  for (int64_t p = s->rowptr[i]; p < s->rowptr[i + 1]; ++p) kv += s->val[p] * V[s->col[p]];
  return V[i] + s->dt_ad[q] * (-kv / s->mass[i] + stim_rate);
}

// One diffusion half step B(dt/2) at time t0: l forward Euler substeps of
// V <- V + dt_ad (-M^-1 K V + s(tau)), tau = t0 + m dt_ad (Jacobi: every row
// reads the V of the previous substep).
void diffusion_half(Sim* s, double t0, double* store = nullptr) {
  const int64_t n = s->n;
  double* V = s->state.data();
  int lmax = 0;
  for (int x : s->l) lmax = std::max(lmax, x);
  for (int m = 0; m < lmax; ++m) {
    if (store) std::memcpy(store + (int64_t)m * n, V, sizeof(double) * n);
    // stimulus rate per node at this substep
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) s->stim_rate[i] = 0.0;
    for (const Stim& st : s->stims) {
      for (int32_t i : st.nodes) {
        int q = s->inst_of[i];
        if (m >= s->l[q]) continue;
        double tau = t0 + m * s->dt_ad[q];
        if (st.t_on <= tau && tau < st.t_on + st.dur) s->stim_rate[i] += st.amp;
      }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) s->vtmp[i] = diffusion_row(s, V, i, m, t0, s->stim_rate[i]);
    std::memcpy(V, s->vtmp.data(), sizeof(double) * n);
  }
}

// Step A for one node at outer step nstep: y (S states) and p (P params) in,
// y out; vprev, lat updated; returns the k used.
int react_node(const Sim* s, int64_t nstep, int64_t i, double* y, const double* p, double& vprev,
               double& lat) {
  const double dt = s->dt;
  const double tA = nstep * dt + 0.5 * dt;   // time of the A-entry sample
  const double Vb = y[0];
  // dV/dt used by the k rule
  double d;
  if (s->dvdt_src == 0) {
    d = (nstep == 0) ? 0.0 : (Vb - vprev) / dt;
  } else {
    Rates<double> r;
    model_rates(s->model, y, p, r);
    d = r.rate[0];
  }
  // activation: first upward crossing of the threshold between samples
  if (nstep > 0 && lat < 0.0 && vprev < s->lat_thr && Vb >= s->lat_thr) {
    double w = (s->lat_thr - vprev) / (Vb - vprev);
    lat = (tA - dt) + w * dt;
  }
  vprev = Vb;
  int k = k_rule(d, s->k_max);
  if (s->ktrace_mode && nstep < s->ktrace_steps) {
    uint8_t* kt = s->ktrace + nstep * s->n + i;
    if (s->ktrace_mode == 1) {
      *kt = (uint8_t)k;
      if (s->dtrace) s->dtrace[nstep * s->n + i] = d;
    } else {
      k = *kt;
    }
  }
  const double h = dt / k;
  for (int sub = 0; sub < k; ++sub) cell_substep(s->model, y, p, h, s->vclamp);
  return k;
}

// Step A at outer step n: every node picks k and advances its cell model by
// dt in k substeps.  Activation time and sensors sample V at A-entry.
void reaction(Sim* s, int64_t nstep) {
  const int64_t n = s->n;
  const int S = s->S, P = s->P;
  if (s->sensor_buf && nstep < s->sensor_steps) {
    for (size_t q = 0; q < s->sensors.size(); ++q)
      s->sensor_buf[nstep * (int64_t)s->sensors.size() + q] = s->state[s->sensors[q]];
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double y[kMaxStates], p[kMaxParams];
    for (int a = 0; a < S; ++a) y[a] = s->state[a * n + i];
    for (int a = 0; a < P; ++a) p[a] = s->params[a * n + i];
    s->lastk[i] = react_node(s, nstep, i, y, p, s->vprev[i], s->lat[i]);
    for (int a = 0; a < S; ++a) s->state[a * n + i] = y[a];
  }
}

// ---------------------------------------------------------------------------
// adjoint of the split step (gradient of a sensor-mismatch loss)
// ---------------------------------------------------------------------------
// Jacobian of one substep at (y, p): J[i][j] = d y'_i / d (y_j for j < S,
// p_{j-S} for j >= S), by forward-mode derivatives through the model code.
constexpr int kJac = 28;   // 19 states + 9 parameters (TP06 with fibroblasts), the largest model
static_assert(kJac >= kMaxStates + kMaxParams, "Jacobian width must hold every model's states and parameters");
void substep_jacobian(int model, const double* y, const double* p, double h, int S, int P,
                      double* J) {
  DualN<kJac> yd[19], pd[kMaxParams];
  for (int a = 0; a < S; ++a) {
    yd[a] = DualN<kJac>(y[a]);
    yd[a].d[a] = 1.0;
  }
  for (int b = 0; b < P; ++b) {
    pd[b] = DualN<kJac>(p[b]);
    pd[b].d[S + b] = 1.0;
  }
  cell_substep(model, yd, pd, h, 0);
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S + P; ++j) J[i * (S + P) + j] = yd[i].d[j];
}

// One taped outer step: stores the inputs of every diffusion substep and the
// reaction-entry state, and adds the loss at reaction entry.
double taped_step(Sim* s, int64_t t) {
  const int64_t n = s->n, nstep = s->step;
  int lmax = 0;
  for (int x : s->l) lmax = std::max(lmax, x);
  double* vs = s->tape_vsub.data() + t * 2 * lmax * n;
  const double tn = nstep * s->dt;
  diffusion_half(s, tn, vs);
  std::memcpy(s->tape_entry.data() + t * s->S * n, s->state.data(), sizeof(double) * s->S * n);
  double loss = 0.0;
  const int64_t ns = (int64_t)s->tsens.size();
  if (nstep < s->target_steps)
    for (int64_t q = 0; q < ns; ++q) {
      const double e = s->state[s->tsens[q]] - s->target[nstep * ns + q];
      loss += e * e;
    }
  reaction(s, nstep);
  for (int64_t i = 0; i < n; ++i) s->tape_k[t * n + i] = (uint8_t)s->lastk[i];
  diffusion_half(s, tn + 0.5 * s->dt, vs + (int64_t)lmax * n);
  s->step = nstep + 1;
  return loss;
}

// Reverse of diffusion substep m (input potential Vin): lam_V <- (I - dt_ad K
// M^-1) lam_V, and the conductivity gradient of lam^T V' through K(sigma).
void adjoint_diffusion(Sim* s, int m, const double* Vin, double* lamV, double* gsig) {
  const int64_t n = s->n;
  std::vector<double> u(n), out(n);
  for (int64_t i = 0; i < n; ++i) u[i] = lamV[i] / s->mass[i];
  for (int64_t i = 0; i < n; ++i) {
    const int q = s->inst_of[i];
    if (m >= s->l[q]) {
      out[i] = lamV[i];
      continue;
    }
    double ku = 0.0;
    for (int64_t p = s->rowptr[i]; p < s->rowptr[i + 1]; ++p) ku += s->val[p] * u[s->col[p]];
    out[i] = lamV[i] - s->dt_ad[q] * ku;
    // d/dsigma of -dt_ad u^T K V, with K_ij = k0_ij (sigma_i + sigma_j)/2 off
    // the diagonal and K_ii = -sum_j K_ij
    for (int64_t p = s->rowptr[i]; p < s->rowptr[i + 1]; ++p) {
      const int32_t j = s->col[p];
      if (j == i) continue;
      const double c = -s->dt_ad[q] * u[i] * 0.5 * s->val0[p] * (Vin[j] - Vin[i]);
      gsig[i] += c;
      gsig[j] += c;
    }
  }
  std::memcpy(lamV, out.data(), sizeof(double) * n);
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface (ctypes)
// ---------------------------------------------------------------------------
extern "C" {

const char* orc_last_error() { return g_err.c_str(); }

void* orc_create(int dim, int64_t n_nodes, const double* xyz, int etype, int64_t n_elems,
                 const int32_t* conn, const double* D_elem, const double* sigma, int32_t n_inst,
                 const int64_t* inst_node_off) {
  const bool simplex = dim >= 2 && etype == dim + 1;
  if (dim < 1 || dim > 3 || n_nodes <= 0 || n_elems < 0 || (etype != (1 << dim) && !simplex)) {
    fail("bad mesh description");
    return nullptr;
  }
  Sim* s = new Sim();
  s->dim = dim;
  s->nen = etype;
  s->n = n_nodes;
  const int nen = etype;
  // assemble row by row into small sorted lists
  std::vector<std::vector<std::pair<int32_t, double>>> rows(n_nodes);
  s->mass.assign(n_nodes, 0.0);
  for (int64_t e = 0; e < n_elems; ++e) {
    double X[24], Ke[64], me[8];
    for (int a = 0; a < nen; ++a) {
      int32_t g = conn[e * nen + a];
      if (g < 0 || g >= n_nodes) {
        delete s;
        fail("connectivity index out of range");
        return nullptr;
      }
      for (int d = 0; d < dim; ++d) X[a * dim + d] = xyz[(int64_t)g * dim + d];
    }
    const int bad = simplex ? simplex_matrices(dim, X, D_elem + e * dim * dim, Ke, me)
                            : element_matrices(dim, nen, X, D_elem + e * dim * dim, Ke, me);
    if (bad != 0) {
      delete s;
      fail("non-positive Jacobian");
      return nullptr;
    }
    for (int a = 0; a < nen; ++a) {
      int32_t ga = conn[e * nen + a];
      s->mass[ga] += me[a];
      for (int b = 0; b < nen; ++b) {
        int32_t gb = conn[e * nen + b];
        auto& row = rows[ga];
        bool found = false;
        for (auto& pr : row)
          if (pr.first == gb) {
            pr.second += Ke[a * nen + b];
            found = true;
            break;
          }
        if (!found) row.push_back({gb, Ke[a * nen + b]});
      }
    }
  }
  // per-node conductivity: off-diagonals scaled by (sigma_i + sigma_j)/2,
  // diagonal reset so that every row sums to zero
  s->rowptr.assign(n_nodes + 1, 0);
  for (int64_t i = 0; i < n_nodes; ++i) {
    auto& row = rows[i];
    std::sort(row.begin(), row.end());
    s->rowptr[i + 1] = s->rowptr[i] + (int64_t)row.size();
  }
  s->col.resize(s->rowptr[n_nodes]);
  s->val.resize(s->rowptr[n_nodes]);
  s->val0.resize(s->rowptr[n_nodes]);
  for (int64_t i = 0; i < n_nodes; ++i) {
    int64_t p = s->rowptr[i];
    double offsum = 0.0;
    int64_t pdiag = -1;
    for (auto& pr : rows[i]) {
      s->col[p] = pr.first;
      double v = pr.second;
      s->val0[p] = v;
      if (pr.first == i) {
        pdiag = p;
      } else if (sigma) {
        v *= 0.5 * (sigma[i] + sigma[pr.first]);
      }
      s->val[p] = v;
      if (pr.first != i) offsum += v;
      ++p;
    }
    if (sigma && pdiag >= 0) s->val[pdiag] = -offsum;
  }
  if (n_inst <= 1 || !inst_node_off) {
    s->inst_off = {0, n_nodes};
  } else {
    s->inst_off.assign(inst_node_off, inst_node_off + n_inst + 1);
  }
  s->inst_of.assign(n_nodes, 0);
  for (size_t q = 0; q + 1 < s->inst_off.size(); ++q)
    for (int64_t i = s->inst_off[q]; i < s->inst_off[q + 1]; ++i) s->inst_of[i] = (int32_t)q;
  s->vtmp.assign(n_nodes, 0.0);
  s->stim_rate.assign(n_nodes, 0.0);
  return s;
}

void orc_destroy(void* h) { delete (Sim*)h; }

int64_t orc_nnz(void* h) { return ((Sim*)h)->rowptr.back(); }

int orc_get_matrix(void* h, int64_t* rowptr, int32_t* col, double* val, double* mass) {
  Sim* s = (Sim*)h;
  std::memcpy(rowptr, s->rowptr.data(), sizeof(int64_t) * (s->n + 1));
  std::memcpy(col, s->col.data(), sizeof(int32_t) * s->col.size());
  std::memcpy(val, s->val.data(), sizeof(double) * s->val.size());
  std::memcpy(mass, s->mass.data(), sizeof(double) * s->n);
  return 0;
}

int orc_set_model(void* h, int model, int n_params, const double* params,
                  const double* init_state, double dt0, double lat_thr) {
  Sim* s = (Sim*)h;
  if (model < 0 || model > 4) return fail("unknown model");
  if (!(dt0 > 0.0)) return fail("dt0 must be positive");
  s->model = model;
  s->S = model_nstates(model);
  s->P = model_nparams(model);
  if (params && n_params != s->P) return fail("wrong parameter count");
  const int64_t n = s->n;
  s->state.assign((size_t)s->S * n, 0.0);
  s->params.assign((size_t)s->P * n, 0.0);
  if (init_state) {
    std::memcpy(s->state.data(), init_state, sizeof(double) * s->S * n);
  } else {
    for (int a = 0; a < s->S; ++a) {
      double v = 0.0;
      if (model == M_MS) v = (a == 0) ? 0.0 : 1.0;
      if (is_tp06(model)) v = tp::INIT[a];
      for (int64_t i = 0; i < n; ++i) s->state[a * n + i] = v;
    }
  }
  if (params) {
    if (model == M_TP06T)
      for (int64_t i = 0; i < n; ++i) {
        const double c = params[6 * n + i];
        if (c != 0.0 && c != 1.0 && c != 2.0) return fail("cell type must be 0, 1 or 2");
      }
    if (model == M_TP06F)
      for (int64_t i = 0; i < n; ++i) {
        const double c = params[6 * n + i];
        if (c != 0.0 && c != 1.0) return fail("node class must be 0 or 1");
      }
    std::memcpy(s->params.data(), params, sizeof(double) * s->P * n);
  } else {
    const double ms[5] = {0.3, 6.0, 120.0, 150.0, 0.13};
    const double tp6[9] = {5.4, 1, 1, 1, 1, 1, 0, 0.0216, -49.6};
    const double lin[2] = {0.0, 0.0};
    for (int a = 0; a < s->P; ++a) {
      double v = model == M_MS ? ms[a] : (is_tp06(model) ? tp6[a] : lin[a]);
      for (int64_t i = 0; i < n; ++i) s->params[a * n + i] = v;
    }
  }
  s->vprev.assign(n, 0.0);
  for (int64_t i = 0; i < n; ++i) s->vprev[i] = s->state[i];
  s->lat.assign(n, -1.0);
  s->lastk.assign(n, 0);
  s->dt0 = dt0;
  s->lat_thr = lat_thr;
  s->step = 0;
  return 0;
}

int orc_add_stimulus(void* h, int64_t n, const int32_t* nodes, double t_on, double dur,
                     double amp) {
  Sim* s = (Sim*)h;
  Stim st;
  for (int64_t q = 0; q < n; ++q) {
    if (nodes[q] < 0 || nodes[q] >= s->n) return fail("stimulus node out of range");
    st.nodes.push_back(nodes[q]);
  }
  std::sort(st.nodes.begin(), st.nodes.end());
  st.nodes.erase(std::unique(st.nodes.begin(), st.nodes.end()), st.nodes.end());
  st.t_on = t_on;
  st.dur = dur;
  st.amp = amp;
  s->stims.push_back(st);
  return 0;
}

int orc_set_method(void* h, int method, int dvdt_src, int l_round) {
  Sim* s = (Sim*)h;
  if (method < 0 || method > 2 || dvdt_src < 0 || dvdt_src > 1 || l_round < 0 || l_round > 1)
    return fail("bad method flags");
  s->method = method;
  s->dvdt_src = dvdt_src;
  s->l_round = l_round;
  if (s->dt > 0.0) return prepare(s, s->dt);
  return 0;
}

int orc_prepare(void* h, double dt) { return prepare((Sim*)h, dt); }

// out: dt_s, G_max, l, dt_ad, k_max, t, step
int orc_info(void* h, int inst, double* out) {
  Sim* s = (Sim*)h;
  if (s->dt <= 0.0) return fail("not prepared");
  if (inst < 0 || inst >= (int)s->l.size()) return fail("bad instance");
  out[0] = s->dt_s[inst];
  out[1] = s->gmax[inst];
  out[2] = s->l[inst];
  out[3] = s->dt_ad[inst];
  out[4] = s->k_max;
  out[5] = s->step * s->dt;
  out[6] = (double)s->step;
  return 0;
}

int orc_step(void* h, int64_t n_steps, double dt) {
  Sim* s = (Sim*)h;
  if (s->model < 0) return fail("no cell model");
  if (s->dt != dt) {
    if (prepare(s, dt) != 0) return -1;
  }
  for (int64_t q = 0; q < n_steps; ++q) {
    const int64_t n = s->step;
    const double tn = n * dt;
    diffusion_half(s, tn);
    reaction(s, n);
    diffusion_half(s, tn + 0.5 * dt);
    s->step = n + 1;
  }
  return 0;
}

// fields: 0 V, 1 V_prev, 2 LAT, 3 last k, 16 + j state j
int orc_get_field(void* h, int field, double* out) {
  Sim* s = (Sim*)h;
  const int64_t n = s->n;
  if (field == 0) std::memcpy(out, s->state.data(), sizeof(double) * n);
  else if (field == 1) std::memcpy(out, s->vprev.data(), sizeof(double) * n);
  else if (field == 2) std::memcpy(out, s->lat.data(), sizeof(double) * n);
  else if (field == 3) for (int64_t i = 0; i < n; ++i) out[i] = s->lastk[i];
  else if (field >= 16 && field < 16 + s->S)
    std::memcpy(out, s->state.data() + (int64_t)(field - 16) * n, sizeof(double) * n);
  else return fail("bad field");
  return 0;
}

int orc_set_field(void* h, int field, const double* in) {
  Sim* s = (Sim*)h;
  const int64_t n = s->n;
  if (field == 0) std::memcpy(s->state.data(), in, sizeof(double) * n);
  else if (field == 1) std::memcpy(s->vprev.data(), in, sizeof(double) * n);
  else if (field == 2) std::memcpy(s->lat.data(), in, sizeof(double) * n);
  else if (field >= 16 && field < 16 + s->S)
    std::memcpy(s->state.data() + (int64_t)(field - 16) * n, in, sizeof(double) * n);
  else return fail("bad field");
  return 0;
}

int orc_set_step(void* h, int64_t step) {
  ((Sim*)h)->step = step;
  return 0;
}

// mode 0 off, 1 record k (and dV/dt if dbuf), 2 replay k.  buf: n_steps * n.
int orc_set_ktrace(void* h, int mode, uint8_t* buf, double* dbuf, int64_t n_steps) {
  Sim* s = (Sim*)h;
  s->ktrace_mode = mode;
  s->ktrace = buf;
  s->dtrace = dbuf;
  s->ktrace_steps = n_steps;
  return 0;
}

int orc_set_sensors(void* h, int32_t n, const int32_t* nodes, double* buf, int64_t n_steps) {
  Sim* s = (Sim*)h;
  s->sensors.assign(nodes, nodes + n);
  s->sensor_buf = buf;
  s->sensor_steps = n_steps;
  return 0;
}

int orc_set_vclamp(void* h, int on) {
  ((Sim*)h)->vclamp = on;
  return 0;
}

// --- adjoint ------------------------------------------------------------------
// Loss = sum over steps n and sensors q of (V_q at reaction entry of step n -
// target[n][q])^2.
int orc_set_target(void* h, int32_t n, const int32_t* nodes, const double* target,
                   int64_t n_steps) {
  Sim* s = (Sim*)h;
  for (int32_t q = 0; q < n; ++q)
    if (nodes[q] < 0 || nodes[q] >= s->n) return fail("sensor out of range");
  s->tsens.assign(nodes, nodes + n);
  s->target.assign(target, target + (int64_t)n * n_steps);
  s->target_steps = n_steps;
  return 0;
}

int orc_forward_taped(void* h, int64_t n_steps, double dt, double* loss) {
  Sim* s = (Sim*)h;
  if (s->model < 0) return fail("no cell model");
  if (s->dt != dt && prepare(s, dt) != 0) return -1;
  int lmax = 0;
  for (int x : s->l) lmax = std::max(lmax, x);
  const int64_t n = s->n;
  s->tape_step0 = s->step;
  s->tape_steps = n_steps;
  s->tape_vsub.assign((size_t)n_steps * 2 * lmax * n, 0.0);
  s->tape_entry.assign((size_t)n_steps * s->S * n, 0.0);
  s->tape_k.assign((size_t)n_steps * n, 0);
  double L = 0.0;
  for (int64_t t = 0; t < n_steps; ++t) L += taped_step(s, t);
  s->taped = true;
  *loss = L;
  return 0;
}

// grad_sigma[n]: dL/dsigma_i.  grad_params[P]: derivative with respect to a
// common multiplier of each parameter row at 1, sum_i p_i[a] dL/dp_i[a].
int orc_backward(void* h, double* grad_sigma, double* grad_params) {
  Sim* s = (Sim*)h;
  if (!s->taped) return fail("no taped forward run");
  const int64_t n = s->n;
  const int S = s->S, P = s->P;
  int lmax = 0;
  for (int x : s->l) lmax = std::max(lmax, x);
  std::vector<double> lam((size_t)S * n, 0.0), gp((size_t)P * n, 0.0);
  for (int64_t i = 0; i < n; ++i) grad_sigma[i] = 0.0;
  const int64_t ns = (int64_t)s->tsens.size();
  for (int64_t t = s->tape_steps - 1; t >= 0; --t) {
    const int64_t nstep = s->tape_step0 + t;
    const double* vs = s->tape_vsub.data() + t * 2 * lmax * n;
    for (int m = lmax - 1; m >= 0; --m)
      adjoint_diffusion(s, m, vs + (int64_t)(lmax + m) * n, lam.data(), grad_sigma);
    // reaction: replay the k substeps from the entry state, then reverse them
    const double* entry = s->tape_entry.data() + t * S * n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const int k = s->tape_k[t * n + i];
      const double hsub = s->dt / k;
      double p[kMaxParams], J[kMaxStates * kJac], li[kMaxStates];
      std::vector<double> ys((size_t)k * S);   // substep start states
      for (int b = 0; b < P; ++b) p[b] = s->params[(int64_t)b * n + i];
      for (int a = 0; a < S; ++a) ys[a] = entry[(int64_t)a * n + i];
      for (int q = 1; q < k; ++q) {
        for (int a = 0; a < S; ++a) ys[(size_t)q * S + a] = ys[(size_t)(q - 1) * S + a];
        cell_substep(s->model, &ys[(size_t)q * S], p, hsub, 0);
      }
      for (int a = 0; a < S; ++a) li[a] = lam[(int64_t)a * n + i];
      for (int q = k - 1; q >= 0; --q) {
        substep_jacobian(s->model, &ys[(size_t)q * S], p, hsub, S, P, J);
        double lo[19];
        for (int j = 0; j < S; ++j) {
          double acc = 0.0;
          for (int a = 0; a < S; ++a) acc += J[a * (S + P) + j] * li[a];
          lo[j] = acc;
        }
        for (int b = 0; b < P; ++b) {
          double acc = 0.0;
          for (int a = 0; a < S; ++a) acc += J[a * (S + P) + S + b] * li[a];
          gp[(int64_t)b * n + i] += acc;
        }
        for (int a = 0; a < S; ++a) li[a] = lo[a];
      }
      for (int a = 0; a < S; ++a) lam[(int64_t)a * n + i] = li[a];
    }
    // loss at reaction entry of this step
    if (nstep < s->target_steps)
      for (int64_t q = 0; q < ns; ++q) {
        const int32_t i = s->tsens[q];
        lam[i] += 2.0 * (entry[i] - s->target[nstep * ns + q]);
      }
    for (int m = lmax - 1; m >= 0; --m) adjoint_diffusion(s, m, vs + (int64_t)m * n, lam.data(), grad_sigma);
  }
  for (int b = 0; b < P; ++b) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += s->params[(int64_t)b * n + i] * gp[(int64_t)b * n + i];
    grad_params[b] = acc;
  }
  return 0;
}

// --- sampled evaluation (rows of one full-size launch) -----------------------
// Substep m of the half step that starts at t0, applied to V_in (all n
// values), evaluated only on `rows`.
int orc_diffusion_rows(void* h, const double* V_in, double t0, int m, int64_t nrows,
                       const int64_t* rows, double* out) {
  Sim* s = (Sim*)h;
  if (s->dt <= 0.0) return fail("not prepared");
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    if (i < 0 || i >= s->n) return fail("row out of range");
    const int q = s->inst_of[i];
    const double tau = t0 + m * s->dt_ad[q];
    out[r] = diffusion_row(s, V_in, i, m, t0, stim_rate_at(s, i, tau));
  }
  return 0;
}

// Step A of outer step nstep on the given nodes: y (S x nrows, SoA), vprev,
// lat in/out, k out.  Uses the simulation's parameters of those nodes.
int orc_reaction_nodes(void* h, int64_t nstep, int64_t nrows, const int64_t* rows, double* y,
                       double* vprev, double* lat, int32_t* k_out) {
  Sim* s = (Sim*)h;
  if (s->dt <= 0.0 || s->model < 0) return fail("not prepared");
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    if (i < 0 || i >= s->n) return fail("node out of range");
    double yy[kMaxStates], p[kMaxParams];
    for (int a = 0; a < s->S; ++a) yy[a] = y[a * nrows + r];
    for (int a = 0; a < s->P; ++a) p[a] = s->params[a * s->n + i];
    k_out[r] = react_node(s, nstep, i, yy, p, vprev[r], lat[r]);
    for (int a = 0; a < s->S; ++a) y[a * nrows + r] = yy[a];
  }
  return 0;
}

// --- cell-level helpers ------------------------------------------------------
// The instantaneous-buffering maps of TP06's calcium pools, exposed so that
// the free-from-total root can be checked against its defining relation.
double orc_free_from_total(double total, double B, double K) { return free_from_total(total, B, K); }
double orc_total_from_free(double c, double B, double K) { return total_from_free(c, B, K); }

int orc_model_nstates(int model) { return model_nstates(model); }
int orc_model_nparams(int model) { return model_nparams(model); }

int orc_model_init(int model, double* y) {
  const int S = model_nstates(model);
  for (int a = 0; a < S; ++a)
    y[a] = is_tp06(model) ? tp::INIT[a] : (model == M_MS ? (a == 0 ? 0.0 : 1.0) : 0.0);
  return 0;
}

// Advance one cell by `dt` in k substeps (k frozen).
int orc_cell_advance(int model, const double* p, double* y, int k, double dt, int vclamp) {
  if (k < 1) return fail("k must be >= 1");
  for (int q = 0; q < k; ++q) cell_substep(model, y, p, dt / k, vclamp);
  return 0;
}

// Rates at a state: out_rate[S], out_inf[S], out_tau[S], out_gate[S]
int orc_cell_rates(int model, const double* p, const double* y, double* rate, double* inf,
                   double* tau, int32_t* gate) {
  Rates<double> r;
  model_rates(model, y, p, r);
  const int S = model_nstates(model);
  for (int a = 0; a < S; ++a) {
    gate[a] = r.is_gate[a];
    rate[a] = r.is_gate[a] ? 0.0 : r.rate[a];
    inf[a] = r.is_gate[a] ? r.inf[a] : 0.0;
    tau[a] = r.is_gate[a] ? r.tau[a] : 0.0;
  }
  return 0;
}

// TP06 currents: INa IK1 Ito IKr IKs ICaL INaCa INaK IpCa IpK IbNa IbCa Irel Iup Ileak Ixfer Iion
int orc_tp06_currents(const double* p, const double* y, double* out) {
  TPCurrents<double> c;
  tp06_currents(y, p, c);
  const double v[17] = {c.INa,  c.IK1,  c.Ito,  c.IKr,  c.IKs, c.ICaL, c.INaCa, c.INaK, c.IpCa,
                        c.IpK,  c.IbNa, c.IbCa, c.Irel, c.Iup, c.Ileak, c.Ixfer, c.Iion};
  for (int a = 0; a < 17; ++a) out[a] = v[a];
  return 0;
}

int orc_k_rule(double dvdt, int k_max) { return k_rule(dvdt, k_max); }
int orc_l_rule(double dt, double dt_s, int l_round) { return l_rule(dt, dt_s, l_round); }


// APD90 of the first action potential of each of ns nodes from its
// reaction-entry samples V[n * ns + q], n = 0..steps-1, taken at
// t_n = (step0 + n) dt + dt/2 (the samples the activation time uses).
// Readings (the paper measures APD90 from the time of the maximum upstroke
// derivative, Sec. 4): activation is the first n with V_{n-1} < thr <= V_n
// and V_rest = V_{n-1} there; repolarisation is the first later interval with
// V_{n-1} >= V_90 > V_n, V_90 = V_max - 0.9 (V_max - V_rest), V_max the
// largest sample from activation to V_{n-1}, its time interpolated linearly;
// the upstroke time is the midpoint of the interval of largest slope
// (V_n - V_{n-1}) / dt from activation to repolarisation (to the last sample
// if there is none), the first one on ties.  apd = -1 where there is no
// repolarisation, tup = -1 where there is no activation.
int orc_apd90(int64_t steps, int64_t ns, const double* V, int64_t step0, double dt, double thr,
              double* apd, double* tup) {
  if (steps < 0 || ns < 0 || (steps * ns > 0 && !V) || !(dt > 0.0) || !apd || !tup)
    return fail("bad argument");
  for (int64_t q = 0; q < ns; ++q) {
    apd[q] = -1.0;
    tup[q] = -1.0;
    auto v = [&](int64_t n) { return V[n * ns + q]; };
    auto t_prev = [&](int64_t n) { return ((step0 + n) * dt + 0.5 * dt) - dt; };
    auto slope = [&](int64_t n) { return (v(n) - v(n - 1)) / dt; };
    int64_t na = -1;
    for (int64_t n = 1; n < steps; ++n)
      if (v(n - 1) < thr && v(n) >= thr) {
        na = n;
        break;
      }
    if (na < 0) continue;
    const double vrest = v(na - 1);
    double vmax = v(na), v90 = 0.0;
    int64_t nr = -1;
    for (int64_t n = na + 1; n < steps; ++n) {
      v90 = vmax - 0.9 * (vmax - vrest);
      if (v(n - 1) >= v90 && v(n) < v90) {
        nr = n;
        break;
      }
      vmax = std::max(vmax, v(n));
    }
    const int64_t nend = nr >= 0 ? nr : steps - 1;
    int64_t best = na;
    for (int64_t n = na + 1; n <= nend; ++n)
      if (slope(n) > slope(best)) best = n;
    tup[q] = t_prev(best) + 0.5 * dt;
    if (nr >= 0) {
      const double w = (v(nr - 1) - v90) / (v(nr - 1) - v(nr));
      apd[q] = (t_prev(nr) + w * dt) - tup[q];
    }
  }
  return 0;
}

}  // extern "C"
