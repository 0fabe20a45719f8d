// Plain FP64 CPU oracle for record-and-replay exact gradients of ODE ensembles.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark do.  It shares no code, header or table with the GPU
// path: every coefficient and formula below is typed here on its own.
//
// What it computes (paper, Sections 2.1 and 3.1):
//  * record  -- the adaptive solve of each trajectory (eq. stages, eq. update,
//               the embedded error estimate and the RMS acceptance test of
//               Section 2.1), keeping the accepted step sizes h_1..h_S and the
//               states at requested save times, each reached by one extra
//               step from the preceding mesh point (Section 3.4).
//  * replay  -- the chain y_i = Phi(y_{i-1}; h_i, theta) of eq. (replay) on a
//               given (frozen) mesh, templated on the scalar type so that the
//               same code runs in double, in forward-mode dual numbers and in
//               complex arithmetic (complex-step derivatives).
//  * adjoint -- the discrete adjoint (reverse sweep) of the replay with the
//               mesh held fixed (the sg[h] convention of Section 3.1), written
//               out by hand stage by stage.
//
// Arithmetic convention.  Every linear combination sum_j c_j v_j is formed in
// index order as acc = c_1 v_1, then acc = fma(c_j, v_j, acc); zero
// coefficients are skipped.  A stage input is fma(h, acc, y).  The right-hand
// sides and their vector-Jacobian products are written with the fma
// placement documented beside each one.  This fixes the rounding of every
// quantity, so an independent implementation that evaluates the same
// formulas in the same order reproduces the oracle bit for bit.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -shared -fPIC.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

namespace orc {

// ---------------------------------------------------------------- scalars --
// Forward-mode dual number with one tangent direction.
struct Dual {
  double v, d;
  Dual(double x = 0.0) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
inline Dual fma(Dual a, Dual b, Dual c) {
  return {std::fma(a.v, b.v, c.v), a.d * b.v + a.v * b.d + c.d};
}
inline Dual tanh(Dual a) {
  double t = std::tanh(a.v);
  return {t, a.d * (1.0 - t * t)};
}

using Cplx = std::complex<double>;
inline Cplx fma(Cplx a, Cplx b, Cplx c) { return a * b + c; }

inline double fma(double a, double b, double c) { return std::fma(a, b, c); }
inline double tanh(double a) { return std::tanh(a); }

inline double value_of(double x) { return x; }
inline double value_of(Dual x) { return x.v; }
inline double value_of(Cplx x) { return x.real(); }

// Operation counter: a double that counts the floating-point operations done
// on it, by the counting rules of the algorithmic work (fma 2; +, -, *, /,
// min, max 1; sqrt, tanh and the controller's root 1; negation, abs and
// comparisons 0).  Instantiating the step routines below on it counts the
// work of one trial step, one reverse step, ... as this file performs it.
//
// Inside the linear algebra of W (factorisation and solves, marked by an
// LuCount scope) an operation whose factor or term is exactly zero is not
// counted, and an fma onto an exact zero counts as the product alone.  At the
// counting point (a small step, so W is dominated by its diagonal and no rows
// are interchanged) W's zeros are the structural zeros of the Jacobian, and
// such operations only add or move a zero: the count is that of the sparse
// factorisation.  The values computed are unchanged.
thread_local int64_t g_ops = 0;
thread_local int g_lu_scope = 0;
struct LuCount {
  LuCount() { ++g_lu_scope; }
  ~LuCount() { --g_lu_scope; }
};
struct OpCount {
  double v;
  OpCount(double x = 0.0) : v(x) {}
};
inline bool lu_zero(double a, double b) { return g_lu_scope > 0 && (a == 0.0 || b == 0.0); }
inline OpCount operator+(OpCount a, OpCount b) { g_ops += lu_zero(a.v, b.v) ? 0 : 1; return a.v + b.v; }
inline OpCount operator-(OpCount a, OpCount b) { g_ops += lu_zero(a.v, b.v) ? 0 : 1; return a.v - b.v; }
inline OpCount operator*(OpCount a, OpCount b) { g_ops += lu_zero(a.v, b.v) ? 0 : 1; return a.v * b.v; }
inline OpCount operator/(OpCount a, OpCount b) { g_ops += lu_zero(a.v, 1.0) ? 0 : 1; return a.v / b.v; }
inline OpCount operator-(OpCount a) { return -a.v; }
inline OpCount& operator+=(OpCount& a, OpCount b) { a = a + b; return a; }
inline bool operator==(OpCount a, OpCount b) { return a.v == b.v; }
inline bool operator!=(OpCount a, OpCount b) { return a.v != b.v; }
inline OpCount fma(OpCount a, OpCount b, OpCount c) {
  g_ops += lu_zero(a.v, b.v) ? 0 : lu_zero(c.v, 1.0) ? 1 : 2;
  return std::fma(a.v, b.v, c.v);
}
inline OpCount tanh(OpCount a) { ++g_ops; return std::tanh(a.v); }
inline double value_of(OpCount x) { return x.v; }

// max, abs and sqrt in every scalar type of the norm and controller (double
// and the counter; the others never reach them)
inline double maxval(double a, double b) { return std::fmax(a, b); }
inline double minval(double a, double b) { return std::fmin(a, b); }
inline double absT(double a) { return std::fabs(a); }
inline double sqrtT(double a) { return std::sqrt(a); }
inline OpCount maxval(OpCount a, OpCount b) { ++g_ops; return std::fmax(a.v, b.v); }
inline OpCount minval(OpCount a, OpCount b) { ++g_ops; return std::fmin(a.v, b.v); }
inline OpCount absT(OpCount a) { return std::fabs(a.v); }
inline OpCount sqrtT(OpCount a) { ++g_ops; return std::sqrt(a.v); }

// --------------------------------------------------------------- tableaux --
// Explicit Runge-Kutta pairs.  c, a (strictly lower), b and ew = b - bhat
// (the weights of the embedded error estimate, up to a sign that the RMS
// norm ignores).
struct ERK {
  int s;        // stages
  int order;    // order of b
  int q_emb;    // order of bhat (controller exponent -1/(q_emb+1))
  bool fsal;    // last stage input equals the new state
  int s_used;   // stages with b_j != 0 (the replay needs only these)
  double c[10];
  double a[10][10];
  double b[10];
  double ew[10];
};

// Tsit5: Tsitouras (2011), 5(4) pair, 7 stages, first-same-as-last.
static ERK make_tsit5() {
  ERK t{};
  t.s = 7; t.order = 5; t.q_emb = 4; t.fsal = true; t.s_used = 6;
  const double c[7] = {0.0, 0.161, 0.327, 0.9, 0.9800255409045097, 1.0, 1.0};
  for (int i = 0; i < 7; ++i) t.c[i] = c[i];
  t.a[1][0] = 0.161;
  t.a[2][0] = -0.008480655492356989;
  t.a[2][1] = 0.335480655492357;
  t.a[3][0] = 2.897153057105493;
  t.a[3][1] = -6.359448489975075;
  t.a[3][2] = 4.3622954328695815;
  t.a[4][0] = 5.325864828439257;
  t.a[4][1] = -11.748883564062828;
  t.a[4][2] = 7.4955393428898365;
  t.a[4][3] = -0.09249506636175525;
  t.a[5][0] = 5.86145544294642;
  t.a[5][1] = -12.92096931784711;
  t.a[5][2] = 8.159367898576159;
  t.a[5][3] = -0.071584973281401;
  t.a[5][4] = -0.028269050394068383;
  t.a[6][0] = 0.09646076681806523;
  t.a[6][1] = 0.01;
  t.a[6][2] = 0.4798896504144996;
  t.a[6][3] = 1.379008574103742;
  t.a[6][4] = -3.290069515436081;
  t.a[6][5] = 2.324710524099774;
  for (int j = 0; j < 6; ++j) t.b[j] = t.a[6][j];
  t.b[6] = 0.0;
  const double ew[7] = {-0.00178001105222577714, -0.0008164344596567469,
                        0.007880878010261995,    -0.1447110071732629,
                        0.5823571654525552,      -0.45808210592918697,
                        0.015151515151515152};
  for (int j = 0; j < 7; ++j) t.ew[j] = ew[j];
  return t;
}

// Vern7: Verner (2010), 7(6) pair, 10 stages, not first-same-as-last.
static ERK make_vern7() {
  ERK t{};
  t.s = 10; t.order = 7; t.q_emb = 6; t.fsal = false; t.s_used = 9;
  const double c[10] = {0.0, 0.005, 0.10888888888888888, 0.16333333333333333,
                        0.4555, 0.6095094489978381, 0.884, 0.925, 1.0, 1.0};
  for (int i = 0; i < 10; ++i) t.c[i] = c[i];
  t.a[1][0] = 0.005;
  t.a[2][0] = -1.07679012345679;
  t.a[2][1] = 1.185679012345679;
  t.a[3][0] = 0.04083333333333333;
  t.a[3][2] = 0.1225;
  t.a[4][0] = 0.6389139236255726;
  t.a[4][2] = -2.455672638223657;
  t.a[4][3] = 2.272258714598084;
  t.a[5][0] = -2.6615773750187572;
  t.a[5][2] = 10.804513886456137;
  t.a[5][3] = -8.3539146573962;
  t.a[5][4] = 0.820487594956657;
  t.a[6][0] = 6.067741434696772;
  t.a[6][2] = -24.711273635911088;
  t.a[6][3] = 20.427517930788895;
  t.a[6][4] = -1.9061579788166472;
  t.a[6][5] = 1.006172249242068;
  t.a[7][0] = 12.054670076253203;
  t.a[7][2] = -49.75478495046899;
  t.a[7][3] = 41.142888638604674;
  t.a[7][4] = -4.461760149974004;
  t.a[7][5] = 2.042334822239175;
  t.a[7][6] = -0.09834843665406107;
  t.a[8][0] = 10.138146522881808;
  t.a[8][2] = -42.6411360317175;
  t.a[8][3] = 35.76384003992257;
  t.a[8][4] = -4.3480228403929075;
  t.a[8][5] = 2.0098622683770357;
  t.a[8][6] = 0.3487490460338272;
  t.a[8][7] = -0.27143900510483127;
  t.a[9][0] = -45.030072034298676;
  t.a[9][2] = 187.3272437654589;
  t.a[9][3] = -154.02882369350186;
  t.a[9][4] = 18.56465306347536;
  t.a[9][5] = -7.141809679295079;
  t.a[9][6] = 1.3088085781613787;
  const double b[10] = {0.04715561848627222, 0.0, 0.0, 0.25750564298434153,
                        0.26216653977412624, 0.15216092656738558,
                        0.4939969170032485, -0.29430311714032503,
                        0.08131747232495111, 0.0};
  for (int j = 0; j < 10; ++j) t.b[j] = b[j];
  const double ew[10] = {0.0025470118799348416, 0.0, 0.0,
                         -0.009658394872807551, 0.04206470975642573,
                         -0.06668224374695614,  0.26500974646213266,
                         -0.29430311714032503,  0.08131747232495111,
                         -0.020295184663355476};
  for (int j = 0; j < 10; ++j) t.ew[j] = ew[j];
  return t;
}

static const ERK TSIT5 = make_tsit5();
static const ERK VERN7 = make_vern7();

static const ERK* erk_of(int method) {
  if (method == 1) return &TSIT5;
  if (method == 2) return &VERN7;
  return nullptr;
}

// ---------------------------------------------------------------- systems --
enum { SYS_LORENZ = 1, SYS_VDP = 2, SYS_ROBERTSON = 3, SYS_HIRES = 4, SYS_LV_UDE = 5,
       SYS_LINEAR = 6 };

// Universal differential equation: Lotka-Volterra plus a multilayer
// perceptron, y' = f_LV(y) + NN(y), with the predator-prey constants fixed,
//   f_LV = (alpha x - beta x y, delta x y - gamma y),
//   (alpha, beta, gamma, delta) = (1.5, 1, 3, 1),
// and NN(y) = W3 tanh(W2 tanh(W1 y + b1) + b2) + b3 with widths 2-32-32-2.
// The parameter vector holds W1 [32][2], b1 [32], W2 [32][32], b2 [32],
// W3 [2][32], b3 [2] in that order, row-major (1218 values).  Plain loops,
// left to right sums; no operation order is shared with any device code.
constexpr int UDE_H = 32;
constexpr int UDE_W1 = 0, UDE_B1 = 64, UDE_W2 = 96, UDE_B2 = 1120, UDE_W3 = 1152,
              UDE_B3 = 1216, UDE_NP = 1218;
constexpr double LV_ALPHA = 1.5, LV_BETA = 1.0, LV_GAMMA = 3.0, LV_DELTA = 1.0;

template <class T, class P>
static void ude_forward(const T* y, const P* p, T* h1, T* h2, T* f) {
  for (int i = 0; i < UDE_H; ++i) {
    T a = T(p[UDE_B1 + i]);
    for (int k = 0; k < 2; ++k) a = a + T(p[UDE_W1 + 2 * i + k]) * y[k];
    h1[i] = tanh(a);
  }
  for (int i = 0; i < UDE_H; ++i) {
    T a = T(p[UDE_B2 + i]);
    for (int j = 0; j < UDE_H; ++j) a = a + T(p[UDE_W2 + UDE_H * i + j]) * h1[j];
    h2[i] = tanh(a);
  }
  for (int o = 0; o < 2; ++o) {
    T a = T(p[UDE_B3 + o]);
    for (int j = 0; j < UDE_H; ++j) a = a + T(p[UDE_W3 + UDE_H * o + j]) * h2[j];
    f[o] = a;
  }
  const T xy = y[0] * y[1];
  f[0] = f[0] + (T(LV_ALPHA) * y[0] - T(LV_BETA) * xy);
  f[1] = f[1] + (T(LV_DELTA) * xy - T(LV_GAMMA) * y[1]);
}

// gy = (df/dy)^T w (overwritten), gp += (df/dp)^T w, by the chain rule
// through the three layers (tanh' = 1 - tanh^2).
template <class T>
static void ude_vjp(const T* y, const T* p, const T* w, T* gy, T* gp) {
  T h1[UDE_H], h2[UDE_H], f[2], d2[UDE_H], d1[UDE_H];
  ude_forward(y, p, h1, h2, f);
  for (int o = 0; o < 2; ++o) {
    gp[UDE_B3 + o] += w[o];
    for (int j = 0; j < UDE_H; ++j) gp[UDE_W3 + UDE_H * o + j] += w[o] * h2[j];
  }
  for (int j = 0; j < UDE_H; ++j) {
    T g = T(0.0);
    for (int o = 0; o < 2; ++o) g += p[UDE_W3 + UDE_H * o + j] * w[o];
    d2[j] = g * (1.0 - h2[j] * h2[j]);
  }
  for (int i = 0; i < UDE_H; ++i) {
    gp[UDE_B2 + i] += d2[i];
    for (int j = 0; j < UDE_H; ++j) gp[UDE_W2 + UDE_H * i + j] += d2[i] * h1[j];
  }
  for (int j = 0; j < UDE_H; ++j) {
    T g = T(0.0);
    for (int i = 0; i < UDE_H; ++i) g += p[UDE_W2 + UDE_H * i + j] * d2[i];
    d1[j] = g * (1.0 - h1[j] * h1[j]);
  }
  for (int i = 0; i < UDE_H; ++i) {
    gp[UDE_B1 + i] += d1[i];
    for (int k = 0; k < 2; ++k) gp[UDE_W1 + 2 * i + k] += d1[i] * y[k];
  }
  for (int k = 0; k < 2; ++k) {
    T g = T(0.0);
    for (int i = 0; i < UDE_H; ++i) g += p[UDE_W1 + 2 * i + k] * d1[i];
    gy[k] = g;
  }
  // Lotka-Volterra part: J_LV = [[alpha - beta y, -beta x], [delta y, delta x - gamma]]
  gy[0] += (LV_ALPHA - LV_BETA * y[1]) * w[0] + LV_DELTA * y[1] * w[1];
  gy[1] += -LV_BETA * y[0] * w[0] + (LV_DELTA * y[0] - LV_GAMMA) * w[1];
}

static int sys_dim(int sys) {
  switch (sys) {
    case SYS_LORENZ: return 3;
    case SYS_VDP: return 2;
    case SYS_ROBERTSON: return 3;
    case SYS_HIRES: return 8;
    case SYS_LV_UDE: return 2;
    case SYS_LINEAR: return 2;
  }
  return -1;
}
static int sys_np(int sys) {
  switch (sys) {
    case SYS_LORENZ: return 3;
    case SYS_VDP: return 1;
    case SYS_ROBERTSON: return 3;
    case SYS_HIRES: return 12;
    case SYS_LV_UDE: return UDE_NP;
    case SYS_LINEAR: return 2;
  }
  return -1;
}

// Right-hand sides f(y, p) of the autonomous systems (paper, Appendix A).
//  Lorenz  p = (sigma, rho, beta):
//    f0 = sigma*(y1 - y0);  f1 = fma(y0, rho - y2, -y1);  f2 = fma(y0, y1, -(beta*y2))
//  Van der Pol  p = (mu):
//    f0 = y1;  f1 = mu * fma(fma(-y0, y0, 1), y1, -y0)
//  Linear (damped rotation y' = A y, A = [[-a, -w], [w, -a]])  p = (a, w):
//    f0 = -fma(a, y0, w*y1);  f1 = fma(w, y0, -(a*y1))
//  Robertson and HIRES: see below (stiff; also Jacobian and its VJP).
template <class T, class P>
static void rhs(int sys, const T* y, const P* p, T* f) {
  switch (sys) {
    case SYS_LORENZ: {
      f[0] = p[0] * (y[1] - y[0]);
      f[1] = fma(y[0], p[1] - y[2], -y[1]);
      f[2] = fma(y[0], y[1], -(p[2] * y[2]));
    } break;
    case SYS_VDP: {
      f[0] = y[1];
      f[1] = p[0] * fma(fma(-y[0], y[0], T(1.0)), y[1], -y[0]);
    } break;
    case SYS_LINEAR: {
      f[0] = -fma(p[0], y[0], p[1] * y[1]);
      f[1] = fma(p[1], y[0], -(p[0] * y[1]));
    } break;
    case SYS_ROBERTSON: {
      // p = (k1, k2, k3): a = k1 y0, b = k3 y1 y2, c = k2 y1^2
      T a = p[0] * y[0];
      T b = (p[2] * y[1]) * y[2];
      T c = (p[1] * y[1]) * y[1];
      f[0] = b - a;
      f[1] = (a - b) - c;
      f[2] = c;
    } break;
    case SYS_LV_UDE: {
      T h1[UDE_H], h2[UDE_H];
      ude_forward(y, p, h1, h2, f);
    } break;
    case SYS_HIRES: {
      // p = the twelve rate literals of Appendix A in order of first appearance
      // (1.71, 0.43, 8.32, 0.0007, 8.75, 10.03, 0.035, 1.12, 1.745, 280, 0.69, 1.81)
      f[0] = fma(p[2], y[2], fma(p[1], y[1], fma(-p[0], y[0], P(p[3]))));
      f[1] = fma(p[0], y[0], -(p[4] * y[1]));
      f[2] = fma(p[6], y[4], fma(p[1], y[3], -(p[5] * y[2])));
      f[3] = fma(p[2], y[1], fma(p[0], y[2], -(p[7] * y[3])));
      f[4] = fma(p[1], y[6], fma(p[1], y[5], -(p[8] * y[4])));
      T z = (p[9] * y[5]) * y[7];
      f[5] = fma(p[10], y[6], fma(-p[1], y[5], fma(p[0], y[4], fma(p[10], y[3], -z))));
      f[6] = fma(-p[11], y[6], z);
      f[7] = -f[6];
    } break;
  }
}

// Jacobian J = df/dy (row-major d x d) of the stiff systems.
template <class T, class P>
static void jac(int sys, const T* y, const P* p, T* J) {
  switch (sys) {
    case SYS_LINEAR: {
      J[0] = -p[0]; J[1] = -p[1];
      J[2] = p[1];  J[3] = -p[0];
    } break;
    case SYS_ROBERTSON: {
      T s2 = p[2] * y[2], s1 = p[2] * y[1], q = p[1] * y[1];
      J[0] = -p[0]; J[1] = s2;            J[2] = s1;
      J[3] = p[0];  J[4] = -s2 - (q + q); J[5] = -s1;
      J[6] = T(0.0); J[7] = q + q;        J[8] = T(0.0);
    } break;
    case SYS_HIRES: {
      for (int i = 0; i < 64; ++i) J[i] = T(0.0);
      T a = p[9] * y[7], b = p[9] * y[5];
      J[0 * 8 + 0] = -p[0]; J[0 * 8 + 1] = p[1]; J[0 * 8 + 2] = p[2];
      J[1 * 8 + 0] = p[0];  J[1 * 8 + 1] = -p[4];
      J[2 * 8 + 2] = -p[5]; J[2 * 8 + 3] = p[1]; J[2 * 8 + 4] = p[6];
      J[3 * 8 + 1] = p[2];  J[3 * 8 + 2] = p[0]; J[3 * 8 + 3] = -p[7];
      J[4 * 8 + 4] = -p[8]; J[4 * 8 + 5] = p[1]; J[4 * 8 + 6] = p[1];
      J[5 * 8 + 3] = p[10]; J[5 * 8 + 4] = p[0]; J[5 * 8 + 5] = -a - p[1];
      J[5 * 8 + 6] = p[10]; J[5 * 8 + 7] = -b;
      J[6 * 8 + 5] = a;     J[6 * 8 + 6] = -p[11]; J[6 * 8 + 7] = b;
      J[7 * 8 + 5] = -a;    J[7 * 8 + 6] = p[11];  J[7 * 8 + 7] = -b;
    } break;
  }
}

// d/d(y, p) of G = u^T J(y, p) v, accumulated into gy and gp.
template <class T>
static void jac_vjp(int sys, const T* y, const T* p, const T* u, const T* v, T* gy, T* gp) {
  switch (sys) {
    case SYS_LINEAR: {
      gp[0] = gp[0] - fma(u[0], v[0], u[1] * v[1]);
      gp[1] = gp[1] + fma(u[1], v[0], -(u[0] * v[1]));
    } break;
    case SYS_ROBERTSON: {
      T du = u[0] - u[1];
      T t = (p[1] + p[1]) * (v[1] * (u[2] - u[1]));
      gy[1] = gy[1] + fma(p[2] * v[2], du, t);
      gy[2] = gy[2] + (p[2] * v[1]) * du;
      gp[0] = gp[0] + v[0] * (u[1] - u[0]);
      gp[1] = gp[1] + (y[1] + y[1]) * (v[1] * (u[2] - u[1]));
      gp[2] = gp[2] + du * fma(y[2], v[1], y[1] * v[2]);
    } break;
    case SYS_HIRES: {
      T du = (u[6] - u[5]) - u[7];
      gy[5] = gy[5] + (p[9] * v[7]) * du;
      gy[7] = gy[7] + (p[9] * v[5]) * du;
      gp[0] = gp[0] + fma(u[5], v[4], fma(u[3], v[2], v[0] * (u[1] - u[0])));
      gp[1] = gp[1] + fma(u[4], v[5] + v[6], fma(u[2], v[3], fma(u[0], v[1], -(u[5] * v[5]))));
      gp[2] = gp[2] + fma(u[0], v[2], u[3] * v[1]);
      gp[4] = gp[4] - u[1] * v[1];
      gp[5] = gp[5] - u[2] * v[2];
      gp[6] = gp[6] + u[2] * v[4];
      gp[7] = gp[7] - u[3] * v[3];
      gp[8] = gp[8] - u[4] * v[4];
      gp[9] = gp[9] + du * fma(y[7], v[5], y[5] * v[7]);
      gp[10] = gp[10] + u[5] * (v[3] + v[6]);
      gp[11] = gp[11] + v[6] * (u[7] - u[6]);
    } break;
  }
}

// Vector-Jacobian products at y: gy = (df/dy)^T w (overwritten) and
// gp += (df/dp)^T w (accumulated).
//  Lorenz:
//    gy0 = fma(y1, w2, fma(rho - y2, w1, -(sigma*w0)))
//    gy1 = fma(y0, w2, fma(sigma, w0, -w1))
//    gy2 = -fma(y0, w1, beta*w2)
//    gp0 = fma(y1 - y0, w0, gp0);  gp1 = fma(y0, w1, gp1);  gp2 = fma(-y2, w2, gp2)
//  Van der Pol (u = mu*w1, q = fma(-y0, y0, 1)):
//    gy0 = u * fma(-2*y0, y1, -1);  gy1 = fma(u, q, w0)
//    gp0 = fma(w1, fma(q, y1, -y0), gp0)
//  Linear:
//    gy0 = fma(w, w1, -(a*w0));  gy1 = -fma(w, w0, a*w1)
//    gp0 = gp0 - fma(y0, w0, y1*w1);  gp1 = gp1 + fma(y0, w1, -(y1*w0))
template <class T>
static void vjp(int sys, const T* y, const T* p, const T* w, T* gy, T* gp) {
  switch (sys) {
    case SYS_LORENZ: {
      gy[0] = fma(y[1], w[2], fma(p[1] - y[2], w[1], -(p[0] * w[0])));
      gy[1] = fma(y[0], w[2], fma(p[0], w[0], -w[1]));
      gy[2] = -fma(y[0], w[1], p[2] * w[2]);
      gp[0] = fma(y[1] - y[0], w[0], gp[0]);
      gp[1] = fma(y[0], w[1], gp[1]);
      gp[2] = fma(-y[2], w[2], gp[2]);
    } break;
    case SYS_VDP: {
      T u = p[0] * w[1];
      T q = fma(-y[0], y[0], T(1.0));
      gy[0] = u * fma(T(-2.0) * y[0], y[1], T(-1.0));
      gy[1] = fma(u, q, w[0]);
      gp[0] = fma(w[1], fma(q, y[1], -y[0]), gp[0]);
    } break;
    case SYS_LINEAR: {
      gy[0] = fma(p[1], w[1], -(p[0] * w[0]));
      gy[1] = -fma(p[1], w[0], p[0] * w[1]);
      gp[0] = gp[0] - fma(y[0], w[0], y[1] * w[1]);
      gp[1] = gp[1] + fma(y[0], w[1], -(y[1] * w[0]));
    } break;
    case SYS_ROBERTSON: {
      T s2 = p[2] * y[2], s1 = p[2] * y[1], q = p[1] * y[1];
      gy[0] = p[0] * (w[1] - w[0]);
      gy[1] = fma(s2, w[0] - w[1], (q + q) * (w[2] - w[1]));
      gy[2] = s1 * (w[0] - w[1]);
      gp[0] = fma(y[0], w[1] - w[0], gp[0]);
      gp[1] = fma(y[1] * y[1], w[2] - w[1], gp[1]);
      gp[2] = fma(y[1] * y[2], w[0] - w[1], gp[2]);
    } break;
    case SYS_LV_UDE: ude_vjp(y, p, w, gy, gp); break;
    case SYS_HIRES: {
      T a = p[9] * y[7], b = p[9] * y[5];
      gy[0] = p[0] * (w[1] - w[0]);
      gy[1] = fma(p[2], w[3], fma(p[1], w[0], -(p[4] * w[1])));
      gy[2] = fma(p[0], w[3], fma(p[2], w[0], -(p[5] * w[2])));
      gy[3] = fma(p[10], w[5], fma(p[1], w[2], -(p[7] * w[3])));
      gy[4] = fma(p[0], w[5], fma(p[6], w[2], -(p[8] * w[4])));
      gy[5] = fma(a, (w[6] - w[7]) - w[5], p[1] * (w[4] - w[5]));
      gy[6] = fma(p[11], w[7] - w[6], fma(p[10], w[5], p[1] * w[4]));
      gy[7] = b * ((w[6] - w[5]) - w[7]);
      gp[0] = gp[0] + fma(y[4], w[5], fma(y[2], w[3], y[0] * (w[1] - w[0])));
      gp[1] = gp[1] + fma(y[5] + y[6], w[4], fma(y[3], w[2], fma(y[1], w[0], -(y[5] * w[5]))));
      gp[2] = gp[2] + fma(y[2], w[0], y[1] * w[3]);
      gp[3] = gp[3] + w[0];
      gp[4] = gp[4] - y[1] * w[1];
      gp[5] = gp[5] - y[2] * w[2];
      gp[6] = gp[6] + y[4] * w[2];
      gp[7] = gp[7] - y[3] * w[3];
      gp[8] = gp[8] - y[4] * w[4];
      gp[9] = gp[9] + (y[5] * y[7]) * ((w[6] - w[5]) - w[7]);
      gp[10] = gp[10] + (y[3] + y[6]) * w[5];
      gp[11] = gp[11] + y[6] * (w[7] - w[6]);
    } break;
  }
}

// ------------------------------------------------------------ one ERK step --
constexpr int DMAX = 8;
constexpr int SMAX = 10;

// Stage values k_1..k_s of one explicit step from y with step h (eq. stages),
// given k_1 = f(y).  Also returns each stage input Y_j.  n_st stages are
// formed (the replay needs only the stages with nonzero b).
template <class T, class P>
static void erk_stages(const ERK& m, int sys, int d, const T* y, const P* p,
                       T h, int n_st, T k[SMAX][DMAX], T Y[SMAX][DMAX]) {
  for (int c = 0; c < d; ++c) Y[0][c] = y[c];
  for (int i = 1; i < n_st; ++i) {
    for (int c = 0; c < d; ++c) {
      T acc = T(0.0);
      bool first = true;
      for (int j = 0; j < i; ++j) {
        if (m.a[i][j] == 0.0) continue;
        if (first) { acc = T(m.a[i][j]) * k[j][c]; first = false; }
        else acc = fma(T(m.a[i][j]), k[j][c], acc);
      }
      Y[i][c] = fma(h, acc, y[c]);
    }
    rhs(sys, Y[i], p, k[i]);
  }
}

// y_new = y + h * sum_j b_j k_j (eq. update), combination over stages with
// nonzero b in index order.
template <class T>
static void erk_update(const ERK& m, int d, const T* y, T h, T k[SMAX][DMAX],
                       T* ynew) {
  for (int c = 0; c < d; ++c) {
    T acc = T(0.0);
    bool first = true;
    for (int j = 0; j < m.s; ++j) {
      if (m.b[j] == 0.0) continue;
      if (first) { acc = T(m.b[j]) * k[j][c]; first = false; }
      else acc = fma(T(m.b[j]), k[j][c], acc);
    }
    ynew[c] = fma(h, acc, y[c]);
  }
}

// One replay step Phi(y; h) (eq. replay).  For a first-same-as-last pair the
// last stage input equals the update, so both are formed by the same
// expression.
template <class T, class P>
static void erk_phi(const ERK& m, int sys, int d, const T* y, const P* p, T h,
                    T* ynew) {
  T k[SMAX][DMAX], Y[SMAX][DMAX];
  rhs(sys, y, p, k[0]);
  erk_stages(m, sys, d, y, p, h, m.s_used, k, Y);
  erk_update(m, d, y, h, k, ynew);
}

// ------------------------------------------------------- controller power --
// x^(-1/k) for the step-size controller and the starting step, k = 4..8,
// from operations that are exactly or correctly rounded (frexp, ldexp, +, *,
// fma) so that any implementation following the same sequence obtains the
// same bits.  x = m 2^e with m in [0.5, 1) and e = k q + j; a linear first
// guess for m^(-1/k) is scaled by 2^(-j/k) 2^(-q), then four Newton steps
// y <- y + (y / k) (1 - x y^k) on f(y) = y^(-k) - x.  Arguments below
// 1e-300 are raised to it (the controller clamps the factor long before).
static const double TWO_NEG_3[3] = {1.0, 0.7937005259840998, 0.6299605249474366};
static const double TWO_NEG_4[4] = {1.0, 0.8408964152537145, 0.7071067811865476,
                                    0.5946035575013605};
static const double TWO_NEG_5[5] = {1.0, 0.8705505632961241, 0.757858283255199,
                                    0.6597539553864471, 0.5743491774985175};
static const double TWO_NEG_6[6] = {1.0, 0.8908987181403393, 0.7937005259840998,
                                    0.7071067811865476, 0.6299605249474366,
                                    0.5612310241546865};
static const double TWO_NEG_7[7] = {1.0, 0.9057236642639067, 0.820335356007638,
                                    0.7429971445684742, 0.6729500963161781,
                                    0.6095068271022377, 0.5520447568369061};
static const double TWO_NEG_8[8] = {1.0, 0.9170040432046712, 0.8408964152537145,
                                    0.7711054127039704, 0.7071067811865476,
                                    0.6484197773255048, 0.5946035575013605,
                                    0.5452538663326288};

static double root_inv(double x, int k) {
  if (std::isnan(x) || x < 0.0) return NAN;
  if (std::isinf(x)) return 0.0;
  if (k < 3 || k > 8) return NAN;
  const double* c = k == 3   ? TWO_NEG_3
                    : k == 4 ? TWO_NEG_4
                    : k == 5 ? TWO_NEG_5
                    : k == 6 ? TWO_NEG_6
                    : k == 7 ? TWO_NEG_7
                             : TWO_NEG_8;
  const double u = 2.0 * c[k - 1];  // 2^(1/k), exactly twice 2^(-(k-1)/k)
  const double inv_k = 1.0 / (double)k;
  x = std::fmax(x, 1e-300);
  int e;
  const double m = std::frexp(x, &e);
  const int q = e >= 0 ? e / k : -((-e + k - 1) / k);
  const int j = e - q * k;
  const double g = fma(-2.0 * (u - 1.0), m - 0.5, u);
  double y = std::ldexp(c[j] * g, -q);
  for (int it = 0; it < 4; ++it) {
    double pw = y;
    for (int i = 1; i < k; ++i) pw = pw * y;
    const double t = fma(-x, pw, 1.0);
    y = fma(y * inv_k, t, y);
  }
  return y;
}

// ----------------------------------------------------------------- record --
enum { ST_OK = 0, ST_MAX_STEPS = 1, ST_DT_UNDERFLOW = 2, ST_NONFINITE = 3,
       ST_NOSPACE = 4 };

struct RecordArgs {
  int sys, method, n, d, np, params_shared;
  const double* y0;      // [n][d]
  const double* p;       // [n][np] or [np]
  double t0, t1, rtol, atol, h0;
  int64_t max_steps;
  int n_save;
  const double* save_t;  // [n_save], ascending, in [t0, t1]
  int64_t cap;           // mesh capacity per lane
  double* h_out;         // [n][cap]
  int32_t* S_out;        // [n]
  int32_t* status_out;   // [n]
  int32_t* save_idx;     // [n][n_save]  base index i(s)
  double* save_dt;       // [n][n_save]  side-step size t_s - t_i(s)
  double* y_save;        // [n][n_save][d]
  int64_t* n_trial;      // [n] trials (accepted + rejected)
  // Refresh of an old mesh (the mesh-drift policy): when follow_h is set,
  // each lane first takes the steps of its old mesh, keeping each one whose
  // error estimate at the new inputs is <= slack; at the first that fails
  // the lane treats that trial as rejected and goes on adaptively from there.
  const double* follow_h;   // [n][follow_cap] or null
  const int32_t* follow_S;  // [n]
  int64_t follow_cap;
  double slack;
  int32_t* drift_at;        // [n] or null: steps kept (= old S if none failed)
};

// Scaled RMS norm of v against the scales sc (paper, Section 2.1):
// sqrt(mean_c (v_c / sc_c)^2), the squares summed with fma in index order.
template <class T>
static T rms_norm(int d, const T* v, const T* sc) {
  T r = v[0] / sc[0];
  T ss = r * r;
  for (int c = 1; c < d; ++c) {
    r = v[c] / sc[c];
    ss = fma(r, r, ss);
  }
  return sqrtT(ss * T(1.0 / (double)d));
}

// The controller's power: x^(-1/k) by root_inv in double; the counter counts
// it as one operation (a pow).
static double root_pow(double x, int k) { return root_inv(x, k); }
static OpCount root_pow(OpCount x, int k) {
  ++g_ops;
  return root_inv(x.v, k);
}

// Error estimate e = h * sum_j ew_j k_j of an explicit pair (index order, fma)
// and its scaled RMS norm against atol + rtol max(|y|, |y_new|) (Section 2.1).
template <class T>
static T erk_err(const ERK& m, int d, T h, const T* y, const T* ynew, T k[SMAX][DMAX],
                 double rtol, double atol) {
  T e[DMAX], sc[DMAX];
  for (int c = 0; c < d; ++c) {
    T acc = T(0.0);
    bool first = true;
    for (int j = 0; j < m.s; ++j) {
      if (m.ew[j] == 0.0) continue;
      if (first) { acc = T(m.ew[j]) * k[j][c]; first = false; }
      else acc = fma(T(m.ew[j]), k[j][c], acc);
    }
    e[c] = h * acc;
    sc[c] = fma(T(rtol), maxval(absT(y[c]), absT(ynew[c])), T(atol));
  }
  return rms_norm(d, e, sc);
}

// Controller (integral, Section 2.1): the proposed factor 0.9 err^(-1/k),
// then the next step after a rejection (factor at least 0.2) or an
// acceptance (factor in [0.2, 10], at most 1 right after a rejection).
template <class T>
static T ctrl_fac0(T err, int k) { return T(0.9) * root_pow(err, k); }
template <class T>
static T ctrl_reject(T h, T fac0) { return h * maxval(T(0.2), fac0); }
template <class T>
static T ctrl_accept(T h, T fac0, bool prev_rejected) {
  return h * maxval(T(0.2), minval(T(prev_rejected ? 1.0 : 10.0), fac0));
}

// Starting step: Hairer, Norsett & Wanner, Solving ODEs I, Sec. II.4, with
// the same scaled RMS norm (scale atol + rtol*|y0|).
static double initial_step(const ERK& m, int sys, int d, const double* y0,
                           const double* p, const double* f0, double t0,
                           double t1, double rtol, double atol) {
  double sc[DMAX] = {}, tmp[DMAX] = {}, y1[DMAX] = {}, f1[DMAX] = {};
  for (int c = 0; c < d; ++c) sc[c] = fma(rtol, std::fabs(y0[c]), atol);
  double d0 = rms_norm(d, y0, sc);
  double d1 = rms_norm(d, f0, sc);
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * (d0 / d1);
  h0 = std::fmin(h0, t1 - t0);
  for (int c = 0; c < d; ++c) y1[c] = fma(h0, f0[c], y0[c]);
  rhs(sys, y1, p, f1);
  for (int c = 0; c < d; ++c) tmp[c] = f1[c] - f0[c];
  double d2 = rms_norm(d, tmp, sc) / h0;
  double dm = std::fmax(d1, d2);
  double h1 = (dm <= 1e-15) ? std::fmax(1e-6, h0 * 1e-3)
                            : root_inv(dm * 100.0, m.order + 1);
  return std::fmin(std::fmin(100.0 * h0, h1), t1 - t0);
}

static void record_lane(const RecordArgs& A, int lane) {
  const ERK& m = *erk_of(A.method);
  const int d = A.d, sys = A.sys;
  const double* p = A.params_shared ? A.p : A.p + (int64_t)lane * A.np;
  double y[DMAX], k1[DMAX];
  for (int c = 0; c < d; ++c) y[c] = A.y0[(int64_t)lane * d + c];
  double* hrow = A.h_out + (int64_t)lane * A.cap;
  int32_t* sidx = A.save_idx + (int64_t)lane * A.n_save;
  double* sdt = A.save_dt + (int64_t)lane * A.n_save;
  double* ysv = A.y_save + (int64_t)lane * A.n_save * d;
  for (int s = 0; s < A.n_save; ++s) {
    sidx[s] = -1;
    sdt[s] = NAN;
    for (int c = 0; c < d; ++c) ysv[s * d + c] = NAN;
  }

  rhs(sys, y, p, k1);
  int status = ST_OK;
  for (int c = 0; c < d; ++c)
    if (!std::isfinite(y[c]) || !std::isfinite(k1[c])) status = ST_NONFINITE;
  double t = A.t0;
  double h = A.h0 > 0.0 ? std::fmin(A.h0, A.t1 - A.t0)
                        : initial_step(m, sys, d, y, p, k1, A.t0, A.t1, A.rtol,
                                       A.atol);
  const int kroot = m.q_emb + 1;  // controller factor 0.9 err^(-1/(q_emb+1))
  int64_t S = 0, trials = 0;
  int next_save = 0;
  bool prev_rejected = false;
  const int64_t S_old = A.follow_h ? A.follow_S[lane] : 0;
  bool following = S_old > 0;
  int64_t kept = S_old;

  while (status == ST_OK && t < A.t1) {
    if (trials >= A.max_steps) { status = ST_MAX_STEPS; break; }
    bool last = false;
    if (following) {  // the old mesh's step, its last one ending at t1
      h = A.follow_h[(int64_t)lane * A.follow_cap + S];
      last = (S == S_old - 1);
    } else {
      // a proposed step too small to advance t ends the lane
      if (h < 16.0 * 2.220446049250313e-16 * std::fmax(std::fabs(t), 1.0)) {
        status = ST_DT_UNDERFLOW;
        break;
      }
      if (t + h >= A.t1) { h = A.t1 - t; last = true; }
    }
    ++trials;

    double k[SMAX][DMAX], Y[SMAX][DMAX], ynew[DMAX];
    for (int c = 0; c < d; ++c) k[0][c] = k1[c];
    erk_stages(m, sys, d, y, p, h, m.s, k, Y);
    if (m.fsal) {
      for (int c = 0; c < d; ++c) ynew[c] = Y[m.s - 1][c];
    } else {
      erk_update(m, d, y, h, k, ynew);
    }
    // error estimate e = h * sum_j ew_j k_j and its scaled RMS norm
    const double err = erk_err(m, d, h, y, ynew, k, A.rtol, A.atol);
    // proposed factor 0.9 err^(-1/(q_emb+1)), bounded below by 0.2 and above
    // by 10 (1 right after a rejection); err = 0 gives the upper bound
    const double fac0 = ctrl_fac0(err, kroot);
    if (following && !(err <= A.slack)) {  // the old mesh ends here: a rejected trial
      following = false;
      kept = S;
      h = ctrl_reject(h, fac0);
      prev_rejected = true;
      continue;
    }

    if (following || err <= 1.0) {
      if (S >= A.cap) { status = ST_NOSPACE; break; }
      hrow[S] = h;
      double tnew = last ? A.t1 : t + h;
      // saves strictly inside this step: one extra step from y (the base
      // state of this step) to each save time.
      while (next_save < A.n_save && A.save_t[next_save] < tnew) {
        double dt = A.save_t[next_save] - t;
        double ys[DMAX];
        double ks[SMAX][DMAX], Ys[SMAX][DMAX];
        for (int c = 0; c < d; ++c) ks[0][c] = k1[c];
        erk_stages(m, sys, d, y, p, dt, m.s_used, ks, Ys);
        erk_update(m, d, y, dt, ks, ys);
        sidx[next_save] = (int32_t)S;
        sdt[next_save] = dt;
        for (int c = 0; c < d; ++c) ysv[next_save * d + c] = ys[c];
        ++next_save;
      }
      ++S;
      t = tnew;
      for (int c = 0; c < d; ++c) y[c] = ynew[c];
      if (m.fsal) {
        for (int c = 0; c < d; ++c) k1[c] = k[m.s - 1][c];
      } else {
        rhs(sys, y, p, k1);
      }
      h = ctrl_accept(h, fac0, prev_rejected);
      prev_rejected = false;
    } else {
      h = ctrl_reject(h, fac0);
      prev_rejected = true;
    }
  }
  // saves at or after the last mesh point (t_s == t_S): side step of size 0,
  // i.e. the state itself.
  if (status == ST_OK) {
    while (next_save < A.n_save) {
      sidx[next_save] = (int32_t)S;
      sdt[next_save] = A.save_t[next_save] - t;
      double ys[DMAX];
      erk_phi(m, sys, d, y, p, sdt[next_save], ys);
      for (int c = 0; c < d; ++c) ysv[next_save * d + c] = ys[c];
      ++next_save;
    }
  }
  A.S_out[lane] = (int32_t)S;
  A.status_out[lane] = status;
  A.n_trial[lane] = trials;
  if (A.drift_at) A.drift_at[lane] = (int32_t)kept;
}

// ----------------------------------------------------------------- replay --
struct MeshArgs {
  int sys, method, n, d, np, params_shared;
  int64_t cap;
  const double* h;        // [n][cap]
  const int32_t* S;       // [n]
  int n_save;
  const int32_t* save_idx;  // [n][n_save]
  const double* save_dt;    // [n][n_save]
  int dense = 0;            // save states by the continuous extension (below)
};

// ------------------------------------------------------------ dense output --
// Dense output (the continuous extension of an accepted step, Section 3.2):
// the state at t_i + theta h inside the step from y_i to y_{i+1} is the cubic
// Hermite interpolant of the two end states and their slopes f_i = f(y_i),
// f_{i+1} = f(y_{i+1}) (Hairer, Norsett & Wanner I, Sec. II.6):
//   y(theta) = a0 y_i + a1 y_{i+1} + h (c0 f_i + c1 f_{i+1}),
//   a0 = (1 - theta)^2 (1 + 2 theta),  a1 = theta^2 (3 - 2 theta),
//   c0 = theta (1 - theta)^2,          c1 = -theta^2 (1 - theta),
// with theta = (t_s - t_i) / h.  It takes the step's end values exactly
// (theta = 0 and 1), is exact for cubic solutions, and its local error is
// O(h^4).  A save at or after the last mesh point is y_S.
struct Hermite {
  double a0, a1, c0, c1;
};
static Hermite hermite(double theta) {
  const double u = 1.0 - theta;
  return Hermite{u * u * (1.0 + 2.0 * theta), theta * theta * (3.0 - 2.0 * theta),
                 theta * u * u, -(theta * theta) * u};
}

// The dense state from (y_i, y_{i+1}) over a step of size h at offset dt.
template <class T, class P>
static void dense_state(int sys, int d, const T* y0, const T* y1, const P* p, double h,
                        double dt, T* out) {
  const Hermite H = hermite(dt / h);
  T f0[DMAX], f1[DMAX];
  rhs(sys, y0, p, f0);
  rhs(sys, y1, p, f1);
  for (int c = 0; c < d; ++c)
    out[c] = T(H.a0) * y0[c] + T(H.a1) * y1[c] + T(h) * (T(H.c0) * f0[c] + T(H.c1) * f1[c]);
}

// Replay one lane in scalar type T; writes the save-time states.
// One replay step Phi(y; h) of the chosen method.
template <class T, class P>
static void phi_any(int method, int sys, int d, const T* y, const P* p, T h, T* ynew);

template <class T>
static void replay_lane(const MeshArgs& M, int lane, const T* y0, const T* p,
                        T* ysave /*[n_save][d]*/) {
  const int d = M.d;
  const double* hrow = M.h + (int64_t)lane * M.cap;
  const int32_t* sidx = M.save_idx + (int64_t)lane * M.n_save;
  const double* sdt = M.save_dt + (int64_t)lane * M.n_save;
  const int S = M.S[lane];
  T y[DMAX];
  for (int c = 0; c < d; ++c) y[c] = y0[c];
  int s = 0;
  for (int i = 0; i <= S; ++i) {
    if (M.dense) {
      if (i == S) {  // saves at the last mesh point: the state itself
        for (; s < M.n_save; ++s)
          for (int c = 0; c < d; ++c) ysave[s * d + c] = y[c];
        break;
      }
      T yn[DMAX];
      phi_any(M.method, M.sys, d, y, p, T(hrow[i]), yn);
      // saves inside this step: the continuous extension
      for (; s < M.n_save && sidx[s] == i; ++s)
        dense_state(M.sys, d, y, yn, p, hrow[i], sdt[s], ysave + s * d);
      for (int c = 0; c < d; ++c) y[c] = yn[c];
      continue;
    }
    // saves whose base is y_i
    while (s < M.n_save && sidx[s] == i) {
      phi_any(M.method, M.sys, d, y, p, T(sdt[s]), ysave + s * d);
      ++s;
    }
    if (i == S) break;
    T yn[DMAX];
    phi_any(M.method, M.sys, d, y, p, T(hrow[i]), yn);
    for (int c = 0; c < d; ++c) y[c] = yn[c];
  }
}

// ---------------------------------------------------------------- adjoint --
enum { LOSS_SUMSQ = 0, LOSS_MSE_TARGET = 1, LOSS_COTANGENT = 2 };

// Reverse sweep through one step Phi(y; h) with output cotangent lam.
// Returns the input cotangent lam + sum_j Ybar_j (accumulated in descending
// j) and accumulates gp += sum_j (df/dp)^T kbar_j, where for j = s'..1
//   kbar_j = h * (b_j lam + sum_{l>j} a_lj Ybar_l),  Ybar_j = (df/dy)^T kbar_j.
template <class T>
static void erk_step_vjp(const ERK& m, int sys, int d, const T* y, const T* p, T h,
                         const T* lam, T* lam_in, T* gp) {
  T k[SMAX][DMAX], Y[SMAX][DMAX];
  rhs(sys, y, p, k[0]);
  const int su = m.s_used;
  erk_stages(m, sys, d, y, p, h, su, k, Y);
  T Yb[SMAX][DMAX];
  for (int c = 0; c < d; ++c) lam_in[c] = lam[c];
  for (int j = su - 1; j >= 0; --j) {
    T kb[DMAX];
    for (int c = 0; c < d; ++c) {
      T acc = T(0.0);
      bool first = true;
      if (m.b[j] != 0.0) { acc = T(m.b[j]) * lam[c]; first = false; }
      for (int l = j + 1; l < su; ++l) {
        if (m.a[l][j] == 0.0) continue;
        if (first) { acc = T(m.a[l][j]) * Yb[l][c]; first = false; }
        else acc = fma(T(m.a[l][j]), Yb[l][c], acc);
      }
      kb[c] = h * acc;
    }
    vjp(sys, Y[j], p, kb, Yb[j], gp);
    for (int c = 0; c < d; ++c) lam_in[c] = lam_in[c] + Yb[j][c];
  }
}

struct LossArgs {
  int kind;
  const double* data;  // [n][n_save][d]: targets (MSE) or cotangents
  double scale;
};

// The reverse of one dense save (the continuous extension of the step from
// y0 to y1 of size h, at offset dt) with cotangent w: the cotangents of the
// two end states, lo = a0 w + f_y(y0)^T (h c0 w) and hi = a1 w +
// f_y(y1)^T (h c1 w), and the parameter terms of both VJPs into gp.
template <class T>
static void dense_save_vjp(int sys, int d, const T* y0, const T* y1, const T* p, double h,
                           double dt, const T* w, T* lo, T* hi, T* gp) {
  const Hermite H = hermite(dt / h);
  T v0[DMAX], v1[DMAX], g0[DMAX], g1[DMAX];
  for (int c = 0; c < d; ++c) {
    v0[c] = T(h * H.c0) * w[c];
    v1[c] = T(h * H.c1) * w[c];
  }
  vjp(sys, y0, p, v0, g0, gp);
  vjp(sys, y1, p, v1, g1, gp);
  for (int c = 0; c < d; ++c) {
    lo[c] = T(H.a0) * w[c] + g0[c];
    hi[c] = T(H.a1) * w[c] + g1[c];
  }
}

// One component's loss cotangent w at a save state's value v and its loss
// term (added into loss): sum of squares v^2 (w = 2 scale v), squared
// difference to a target (v - x)^2 (w = 2 scale (v - x)), or a given
// cotangent x (no loss term).
template <class T>
static void loss_cot(int kind, T v, double x, T two_scale, T& loss, T& w) {
  if (kind == LOSS_SUMSQ) {
    loss = fma(v, v, loss);
    w = two_scale * v;
  } else if (kind == LOSS_MSE_TARGET) {
    T r = v - T(x);
    loss = fma(r, r, loss);
    w = two_scale * r;
  } else {
    w = T(x);
  }
}

// Discrete adjoint of one lane: gradient of the lane's loss with respect to
// its parameters (gp, accumulated) and its initial state (gy0).  Returns the
// lane's loss.
template <class T>
static void step_vjp_any(int method, int sys, int d, const T* y, const T* p, T h,
                         const T* lam, T* lam_in, T* gp);

static double adjoint_lane(const MeshArgs& M, const LossArgs& L, int lane,
                           const double* y0, const double* p, double* gp,
                           double* gy0) {
  const int d = M.d;
  const int S = M.S[lane];
  const double* hrow = M.h + (int64_t)lane * M.cap;
  const int32_t* sidx = M.save_idx + (int64_t)lane * M.n_save;
  const double* sdt = M.save_dt + (int64_t)lane * M.n_save;
  const double* ldat = L.data ? L.data + (int64_t)lane * M.n_save * d : nullptr;

  // forward states y_0..y_S (the replay in double)
  std::vector<double> ys((size_t)(S + 1) * d);
  for (int c = 0; c < d; ++c) ys[c] = y0[c];
  for (int i = 0; i < S; ++i)
    phi_any(M.method, M.sys, d, &ys[(size_t)i * d], p, hrow[i], &ys[(size_t)(i + 1) * d]);

  // save-time states (one extra step from the base mesh point, or the
  // continuous extension of the step that holds the save time)
  std::vector<double> ysave((size_t)M.n_save * d);
  for (int s = 0; s < M.n_save; ++s) {
    if (!M.dense) {
      phi_any(M.method, M.sys, d, &ys[(size_t)sidx[s] * d], p, sdt[s], &ysave[(size_t)s * d]);
    } else if (sidx[s] == S) {
      for (int c = 0; c < d; ++c) ysave[(size_t)s * d + c] = ys[(size_t)S * d + c];
    } else {
      dense_state(M.sys, d, &ys[(size_t)sidx[s] * d], &ys[(size_t)(sidx[s] + 1) * d], p,
                  hrow[sidx[s]], sdt[s], &ysave[(size_t)s * d]);
    }
  }

  // loss and save-time cotangents
  double loss = 0.0;
  std::vector<double> wbar((size_t)M.n_save * d);
  const double two_scale = 2.0 * L.scale;
  for (int s = 0; s < M.n_save; ++s)
    for (int c = 0; c < d; ++c)
      loss_cot(L.kind, ysave[s * d + c], ldat ? ldat[s * d + c] : 0.0, two_scale, loss,
               wbar[s * d + c]);
  loss = L.scale * loss;

  // The save steps first, from the last save to the first: each one's
  // cotangent for its base state (lsave) and its parameter terms (into gp);
  // then the mesh steps from the last, each base state's cotangent taking
  // the saves based there as the sweep reaches it (the order of the sum over
  // steps in gp is not fixed by the method; this one every sweep layout on
  // the device reproduces).
  std::vector<double> lsave((size_t)M.n_save * d);
  // dense output: each save's cotangent reaches both end states of its step;
  // collected per mesh point first, added as the sweep reaches the point
  std::vector<double> lpt(M.dense ? (size_t)(S + 1) * d : 0, 0.0);
  if (M.dense) {
    for (int s2 = M.n_save - 1; s2 >= 0; --s2) {
      const int i = sidx[s2];
      const double* w = &wbar[(size_t)s2 * d];
      if (i == S) {
        for (int c = 0; c < d; ++c) lpt[(size_t)S * d + c] += w[c];
        continue;
      }
      // y(theta) = a0 y_i + a1 y_{i+1} + h (c0 f(y_i) + c1 f(y_{i+1}))
      double lo[DMAX], hi[DMAX];
      dense_save_vjp(M.sys, d, &ys[(size_t)i * d], &ys[(size_t)(i + 1) * d], p, hrow[i],
                     sdt[s2], w, lo, hi, gp);
      for (int c = 0; c < d; ++c) {
        lpt[(size_t)i * d + c] += lo[c];
        lpt[(size_t)(i + 1) * d + c] += hi[c];
      }
    }
  } else {
    for (int s2 = M.n_save - 1; s2 >= 0; --s2)
      step_vjp_any(M.method, M.sys, d, &ys[(size_t)sidx[s2] * d], p, sdt[s2], &wbar[s2 * d],
                   &lsave[(size_t)s2 * d], gp);
  }
  double lam[DMAX];
  for (int c = 0; c < d; ++c) lam[c] = 0.0;
  int s = M.n_save - 1;
  for (int i = S; i >= 0; --i) {
    if (M.dense)
      for (int c = 0; c < d; ++c) lam[c] = lam[c] + lpt[(size_t)i * d + c];
    while (!M.dense && s >= 0 && sidx[s] == i) {
      for (int c = 0; c < d; ++c) lam[c] = lam[c] + lsave[(size_t)s * d + c];
      --s;
    }
    if (i == 0) break;
    double li[DMAX];
    step_vjp_any(M.method, M.sys, d, &ys[(size_t)(i - 1) * d], p, hrow[i - 1], lam, li, gp);
    for (int c = 0; c < d; ++c) lam[c] = li[c];
  }
  for (int c = 0; c < d; ++c) gy0[c] = lam[c];
  return loss;
}

// ============================================================ Rosenbrock ==
// Rodas4 (Hairer & Wanner, Solving ODEs II, Sec. IV.7): a stiffly accurate,
// L-stable Rosenbrock-Wanner method of order 4 with an embedded order-3
// solution, in the transformed form with W = I/(gamma h) - J (J = df/dy at
// the step's start, the systems are autonomous):
//   Y_i = y + sum_{j<i} a_ij u_j,   W u_i = f(Y_i) + (1/h) sum_{j<i} c_ij u_j,
//   y_new = Y_6 + u_6,   error estimate e = u_6.
// Rosenbrock23 (below) is written in the same form.  Fields: s stages, of
// which the first su enter y_new (y_new = y + sum_{j<su} m_j u_j); the error
// estimate is sum_j e_j u_j; new_at_input: y_new is the input Y_s of the
// last stage (formed as that stage's input), otherwise y_new = Y_s + u_s.
struct ROS {
  int s, su, order, q_emb;
  bool new_at_input;
  double gamma;
  double a[6][6];
  double c[6][6];
  double m[6];
  double e[6];
};

static ROS make_rodas4() {
  ROS r{};
  r.s = 6; r.su = 6; r.order = 4; r.q_emb = 3; r.gamma = 0.25;
  r.new_at_input = false;
  r.a[1][0] = 1.544;
  r.a[2][0] = 0.9466785280815826;  r.a[2][1] = 0.2557011698983284;
  r.a[3][0] = 3.314825187068521;   r.a[3][1] = 2.896124015972201;
  r.a[3][2] = 0.9986419139977817;
  r.a[4][0] = 1.221224509226641;   r.a[4][1] = 6.019134481288629;
  r.a[4][2] = 12.53708332932087;   r.a[4][3] = -0.6878860361058950;
  for (int j = 0; j < 4; ++j) r.a[5][j] = r.a[4][j];
  r.a[5][4] = 1.0;
  r.c[1][0] = -5.6688;
  r.c[2][0] = -2.430093356833875;  r.c[2][1] = -0.2063599157091915;
  r.c[3][0] = -0.1073529058151375; r.c[3][1] = -9.594562251023355;
  r.c[3][2] = -20.47028614809616;
  r.c[4][0] = 7.496443313967647;   r.c[4][1] = -10.24680431464352;
  r.c[4][2] = -33.99990352819905;  r.c[4][3] = 11.70890893206160;
  r.c[5][0] = 8.083246795921522;   r.c[5][1] = -7.981132988064893;
  r.c[5][2] = -31.52159432874371;  r.c[5][3] = 16.31930543123136;
  r.c[5][4] = -6.058818238834054;
  for (int j = 0; j < 5; ++j) r.m[j] = r.a[5][j];
  r.m[5] = 1.0;
  r.e[5] = 1.0;
  return r;
}
static const ROS RODAS4 = make_rodas4();

// Rosenbrock23 (Shampine & Reichelt 1997, the method of MATLAB's ode23s) for
// an autonomous f, with d = 1/(2 + sqrt 2) and e32 = 6 + sqrt 2:
//   W = I - h d J,  k1 = W^{-1} f(y),  F1 = f(y + h k1 / 2),
//   k2 = W^{-1}(F1 - k1) + k1,  y_new = y + h k2,  F2 = f(y_new),
//   k3 = W^{-1}(F2 - e32 (k2 - F1) - 2 (k1 - f(y))),
//   error estimate (h/6)(k1 - 2 k2 + k3).
// With W k1 = f(y) and W k2 = F1 - h d J k1 the differences of f-values are
// J-terms, k1 - f(y) = h d J k1 and k2 - F1 = h d J (k2 - k1), so in the
// increments K_i = h k_i it is the Rosenbrock method
//   (I - d h J) K_i = h f(y + sum alpha_ij K_j) + h J sum gamma_ij K_j
// with alpha_21 = 1/2, alpha_32 = 1, gamma_21 = -d,
// gamma_31 = (e32 - 2) d, gamma_32 = -e32 d, b = (0, 1, 0) and error weights
// (1, -2, 1)/6.  The transformed form (u = Gamma K, Gamma = (gamma_ij) with
// d on the diagonal) has Gamma^{-1} = (1/d) [[1,0,0],[1,1,0],[2,e32,1]], so
//   a = alpha Gamma^{-1}:   a_21 = 1/(2d), a_31 = a_32 = 1/d,
//   c = diag(1/d) - Gamma^{-1}:  c_21 = -1/d, c_31 = -2/d, c_32 = -e32/d,
//   m = b Gamma^{-1} = (1/d, 1/d, 0)  (y_new = Y_3, the third stage input),
//   error weights (1, e32 - 2, 1)/(6d).
// Order 2; the error estimate is O(h^3), so the controller's root is the
// third (q_emb = 2).  Values: the doubles nearest the exact numbers.
static ROS make_ros23() {
  ROS r{};
  r.s = 3; r.su = 2; r.order = 2; r.q_emb = 2;
  r.new_at_input = true;
  r.gamma = 0.2928932188134525;
  r.a[1][0] = 1.7071067811865475;
  r.a[2][0] = 3.414213562373095;   r.a[2][1] = 3.414213562373095;
  r.c[1][0] = -3.414213562373095;
  r.c[2][0] = -6.82842712474619;   r.c[2][1] = -25.31370849898476;
  r.m[0] = 3.414213562373095;      r.m[1] = 3.414213562373095;
  r.e[0] = 0.5690355937288492;     r.e[1] = 3.080880229039762;
  r.e[2] = 0.5690355937288492;
  return r;
}
static const ROS ROS23 = make_ros23();

static const ROS* ros_of(int method) {
  return method == 3 ? &RODAS4 : method == 4 ? &ROS23 : nullptr;
}
static bool is_ros(int method) { return ros_of(method) != nullptr; }

inline double absval(double x) { return std::fabs(x); }
inline double absval(Dual x) { return std::fabs(x.v); }
inline double absval(Cplx x) { return std::fabs(x.real()); }
inline double absval(OpCount x) { return std::fabs(x.v); }

// LU factorisation with partial pivoting, in place (row-major d x d).  The
// pivot of column k is the first row i >= k with the largest |W_ik| (ties go
// to the lowest row); the permutation only depends on values, so it is the
// same in every scalar type.  As LAPACK's getf2 scales a column by the
// pivot's reciprocal: r_k = 1 / W_kk, l_ik = W_ik * r_k,
// W_ij = fma(-l_ik, W_kj, W_ij).  The diagonal keeps r_k (not U_kk), and the
// triangular solves multiply by it.
template <class T>
static void lu_factor(int d, T* W, int* perm) {
  const LuCount scope;
  for (int i = 0; i < d; ++i) perm[i] = i;
  for (int k = 0; k < d; ++k) {
    int piv = k;
    double best = absval(W[k * d + k]);
    for (int i = k + 1; i < d; ++i)
      if (absval(W[i * d + k]) > best) { best = absval(W[i * d + k]); piv = i; }
    if (piv != k) {
      for (int j = 0; j < d; ++j) std::swap(W[k * d + j], W[piv * d + j]);
      std::swap(perm[k], perm[piv]);
    }
    const T r = T(1.0) / W[k * d + k];
    W[k * d + k] = r;
    for (int i = k + 1; i < d; ++i) {
      T l = W[i * d + k] * r;
      W[i * d + k] = l;
      for (int j = k + 1; j < d; ++j) W[i * d + j] = fma(-l, W[k * d + j], W[i * d + j]);
    }
  }
}

// Solve W x = b with the factors (x may not alias b; the diagonal holds the
// reciprocals of U's).
template <class T>
static void lu_solve(int d, const T* LU, const int* perm, const T* b, T* x) {
  const LuCount scope;
  for (int i = 0; i < d; ++i) {
    T acc = b[perm[i]];
    for (int j = 0; j < i; ++j) acc = fma(-LU[i * d + j], x[j], acc);
    x[i] = acc;
  }
  for (int i = d - 1; i >= 0; --i) {
    T acc = x[i];
    for (int j = i + 1; j < d; ++j) acc = fma(-LU[i * d + j], x[j], acc);
    x[i] = acc * LU[i * d + i];
  }
}

// Solve W^T z = b with the factors: U^T v = b, L^T w = v, z[perm[i]] = w[i].
template <class T>
static void lu_solve_t(int d, const T* LU, const int* perm, const T* b, T* z) {
  const LuCount scope;
  T v[DMAX];
  for (int i = 0; i < d; ++i) {
    T acc = b[i];
    for (int j = 0; j < i; ++j) acc = fma(-LU[j * d + i], v[j], acc);
    v[i] = acc * LU[i * d + i];
  }
  for (int i = d - 1; i >= 0; --i) {
    T acc = v[i];
    for (int j = i + 1; j < d; ++j) acc = fma(-LU[j * d + i], v[j], acc);
    v[i] = acc;
  }
  for (int i = 0; i < d; ++i) z[perm[i]] = v[i];
}

// One Rosenbrock step of method m from y with step h; stage inputs Y,
// increments u and the factors are returned for the reverse sweep.
// y_new = Y_s + u_s (Rodas4) or Y_s (Rosenbrock23).  The first n_st stages
// are formed: a trial step needs all s; a replay step and its reverse only
// the su that enter y_new (for Rosenbrock23, y_new is then formed as the
// third stage's input without that stage's solve).
template <class T, class P>
static void ros_step(const ROS& m, int sys, int d, const T* y, const P* p, T h, int n_st,
                     T* ynew, T Y[6][DMAX], T u[6][DMAX], T* LU, int* perm) {
  jac(sys, y, p, LU);
  const T dg = T(1.0) / (T(m.gamma) * h);
  for (int i = 0; i < d * d; ++i) LU[i] = -LU[i];
  for (int i = 0; i < d; ++i) LU[i * d + i] = LU[i * d + i] + dg;
  lu_factor(d, LU, perm);
  const T hinv = T(1.0) / h;
  // stage input Y_i = y + sum_{j<i} a_ij u_j
  auto stage_input = [&](int i) {
    for (int c = 0; c < d; ++c) {
      T acc = T(0.0);
      bool first = true;
      for (int j = 0; j < i; ++j) {
        if (m.a[i][j] == 0.0) continue;
        if (first) { acc = T(m.a[i][j]) * u[j][c]; first = false; }
        else acc = fma(T(m.a[i][j]), u[j][c], acc);
      }
      Y[i][c] = first ? y[c] : y[c] + acc;
    }
  };
  for (int i = 0; i < n_st; ++i) {
    T F[DMAX], r[DMAX];
    stage_input(i);
    rhs(sys, Y[i], p, F);
    for (int c = 0; c < d; ++c) {
      T acc = T(0.0);
      bool first = true;
      for (int j = 0; j < i; ++j) {
        if (m.c[i][j] == 0.0) continue;
        if (first) { acc = T(m.c[i][j]) * u[j][c]; first = false; }
        else acc = fma(T(m.c[i][j]), u[j][c], acc);
      }
      r[c] = first ? F[c] : fma(acc, hinv, F[c]);
    }
    lu_solve(d, LU, perm, r, u[i]);
  }
  if (!ynew) return;  // the reverse needs only the stages
  if (m.new_at_input && n_st < m.s) stage_input(m.s - 1);
  for (int c = 0; c < d; ++c)
    ynew[c] = m.new_at_input ? Y[m.s - 1][c] : Y[m.s - 1][c] + u[m.s - 1][c];
}

// Error estimate e = sum_j e_j u_j (Rodas4: u_6 itself).
template <class T>
static void ros_errvec(const ROS& m, int d, const T u[6][DMAX], T* e) {
  for (int c = 0; c < d; ++c) {
    T acc = T(0.0);
    bool first = true;
    for (int j = 0; j < m.s; ++j) {
      if (m.e[j] == 0.0) continue;
      if (first) { acc = T(m.e[j]) * u[j][c]; first = false; }
      else acc = fma(T(m.e[j]), u[j][c], acc);
    }
    e[c] = acc;
  }
}

// The error estimate's scaled RMS norm (as for the explicit pairs).
template <class T>
static T ros_err(const ROS& m, int d, const T* y, const T* ynew, const T u[6][DMAX],
                 double rtol, double atol) {
  T sc[DMAX] = {}, e[DMAX] = {};
  for (int c = 0; c < d; ++c) sc[c] = fma(T(rtol), maxval(absT(y[c]), absT(ynew[c])), T(atol));
  ros_errvec(m, d, u, e);
  return rms_norm(d, e, sc);
}

template <class T, class P>
static void ros_phi(const ROS& m, int sys, int d, const T* y, const P* p, T h, T* ynew) {
  if (value_of(h) == 0.0) {  // a zero-length step is the identity (skipped)
    for (int c = 0; c < d; ++c) ynew[c] = y[c];
    return;
  }
  T Y[6][DMAX], u[6][DMAX], LU[DMAX * DMAX];
  int perm[DMAX];
  ros_step(m, sys, d, y, p, h, m.su, ynew, Y, u, LU, perm);
}

static void ros_record_lane(const RecordArgs& A, int lane) {
  const ROS& m = *ros_of(A.method);
  const int d = A.d, sys = A.sys;
  const double* p = A.params_shared ? A.p : A.p + (int64_t)lane * A.np;
  double y[DMAX], f0[DMAX];
  for (int c = 0; c < d; ++c) y[c] = A.y0[(int64_t)lane * d + c];
  double* hrow = A.h_out + (int64_t)lane * A.cap;
  int32_t* sidx = A.save_idx + (int64_t)lane * A.n_save;
  double* sdt = A.save_dt + (int64_t)lane * A.n_save;
  double* ysv = A.y_save + (int64_t)lane * A.n_save * d;
  for (int s = 0; s < A.n_save; ++s) {
    sidx[s] = -1;
    sdt[s] = NAN;
    for (int c = 0; c < d; ++c) ysv[s * d + c] = NAN;
  }
  rhs(sys, y, p, f0);
  int status = ST_OK;
  for (int c = 0; c < d; ++c)
    if (!std::isfinite(y[c]) || !std::isfinite(f0[c])) status = ST_NONFINITE;
  double t = A.t0;
  // starting step as for the explicit pairs, with the method's order
  ERK pseudo{};
  pseudo.order = m.order;
  double h = A.h0 > 0.0 ? std::fmin(A.h0, A.t1 - A.t0)
                        : initial_step(pseudo, sys, d, y, p, f0, A.t0, A.t1, A.rtol, A.atol);
  const int kroot = m.q_emb + 1;
  int64_t S = 0, trials = 0;
  int next_save = 0;
  bool prev_rejected = false;
  const int64_t S_old = A.follow_h ? A.follow_S[lane] : 0;
  bool following = S_old > 0;
  int64_t kept = S_old;
  while (status == ST_OK && t < A.t1) {
    if (trials >= A.max_steps) { status = ST_MAX_STEPS; break; }
    bool last = false;
    if (following) {
      h = A.follow_h[(int64_t)lane * A.follow_cap + S];
      last = (S == S_old - 1);
    } else {
      if (h < 16.0 * 2.220446049250313e-16 * std::fmax(std::fabs(t), 1.0)) {
        status = ST_DT_UNDERFLOW;
        break;
      }
      if (t + h >= A.t1) { h = A.t1 - t; last = true; }
    }
    ++trials;
    double ynew[DMAX], Y[6][DMAX], u[6][DMAX], LU[DMAX * DMAX];
    int perm[DMAX];
    ros_step(m, sys, d, y, p, h, m.s, ynew, Y, u, LU, perm);
    const double err = ros_err(m, d, y, ynew, u, A.rtol, A.atol);
    const double fac0 = ctrl_fac0(err, kroot);
    if (following && !(err <= A.slack)) {  // the old mesh ends here: a rejected trial
      following = false;
      kept = S;
      h = ctrl_reject(h, fac0);
      prev_rejected = true;
      continue;
    }
    if (following || err <= 1.0) {
      if (S >= A.cap) { status = ST_NOSPACE; break; }
      hrow[S] = h;
      double tnew = last ? A.t1 : t + h;
      while (next_save < A.n_save && A.save_t[next_save] < tnew) {
        double dt = A.save_t[next_save] - t;
        double ys[DMAX];
        ros_phi(m, sys, d, y, p, dt, ys);
        sidx[next_save] = (int32_t)S;
        sdt[next_save] = dt;
        for (int c = 0; c < d; ++c) ysv[next_save * d + c] = ys[c];
        ++next_save;
      }
      ++S;
      t = tnew;
      for (int c = 0; c < d; ++c) y[c] = ynew[c];
      h = ctrl_accept(h, fac0, prev_rejected);
      prev_rejected = false;
    } else {
      h = ctrl_reject(h, fac0);
      prev_rejected = true;
    }
  }
  if (status == ST_OK) {
    while (next_save < A.n_save) {
      sidx[next_save] = (int32_t)S;
      sdt[next_save] = A.save_t[next_save] - t;
      double ys[DMAX];
      ros_phi(m, sys, d, y, p, sdt[next_save], ys);
      for (int c = 0; c < d; ++c) ysv[next_save * d + c] = ys[c];
      ++next_save;
    }
  }
  A.S_out[lane] = (int32_t)S;
  A.status_out[lane] = status;
  A.n_trial[lane] = trials;
  if (A.drift_at) A.drift_at[lane] = (int32_t)kept;
}

// Reverse sweep through one Rosenbrock step with output cotangent lam:
//   ubar_i = m_i lam + sum_{l>i} (a_li Ybar_l + c_li t_l),  t_l = rbar_l / h
// (the sum over l runs from the last stage down, as the sweep forms them)
//   rbar_i = W^{-T} ubar_i,  Ybar_i = J(Y_i)^T rbar_i,  p_bar += f_p(Y_i)^T rbar_i
//   lam_in = lam + sum_i Ybar_i + d/dy sum_i rbar_i^T J(y) u_i  (J is at y)
// with p_bar also receiving d/dp of rbar_i^T J u_i.  Stages run i = 6..1 and
// each stage adds its f_p term, then its J_p term, to p_bar.  Only the su
// stages that enter y_new are reversed: a later stage (Rosenbrock23's third,
// which serves the error estimate alone) has a zero cotangent.
template <class T>
static void ros_step_vjp(const ROS& m, int sys, int d, const T* y, const T* p, T h,
                         const T* lam, T* lam_in, T* gp) {
  if (value_of(h) == 0.0) {
    for (int c = 0; c < d; ++c) lam_in[c] = lam[c];
    return;
  }
  T Y[6][DMAX], u[6][DMAX], LU[DMAX * DMAX];
  int perm[DMAX];
  ros_step(m, sys, d, y, p, h, m.su, (T*)nullptr, Y, u, LU, perm);
  const T hinv = T(1.0) / h;
  T Yb[6][DMAX], rb[6][DMAX], tb[6][DMAX], gJ[DMAX];
  for (int c = 0; c < d; ++c) {
    lam_in[c] = lam[c];
    gJ[c] = T(0.0);
  }
  for (int i = m.su - 1; i >= 0; --i) {
    T ub[DMAX];
    for (int c = 0; c < d; ++c) {
      T acc = T(0.0);
      bool first = true;
      if (m.m[i] != 0.0) { acc = T(m.m[i]) * lam[c]; first = false; }
      for (int l = m.su - 1; l > i; --l) {  // in the order the sweep forms them
        if (m.a[l][i] != 0.0) {
          if (first) { acc = T(m.a[l][i]) * Yb[l][c]; first = false; }
          else acc = fma(T(m.a[l][i]), Yb[l][c], acc);
        }
        if (m.c[l][i] != 0.0) {
          if (first) { acc = T(m.c[l][i]) * tb[l][c]; first = false; }
          else acc = fma(T(m.c[l][i]), tb[l][c], acc);
        }
      }
      ub[c] = acc;
    }
    lu_solve_t(d, LU, perm, ub, rb[i]);
    for (int c = 0; c < d; ++c) tb[i][c] = hinv * rb[i][c];
    vjp(sys, Y[i], p, rb[i], Yb[i], gp);
    for (int c = 0; c < d; ++c) lam_in[c] = lam_in[c] + Yb[i][c];
    jac_vjp(sys, y, p, rb[i], u[i], gJ, gp);
  }
  for (int c = 0; c < d; ++c) lam_in[c] = lam_in[c] + gJ[c];
}

// ------------------------------------------------------- method dispatch --
template <class T, class P>
static void phi_any(int method, int sys, int d, const T* y, const P* p, T h, T* ynew) {
  if (is_ros(method)) ros_phi(*ros_of(method), sys, d, y, p, h, ynew);
  else erk_phi(*erk_of(method), sys, d, y, p, h, ynew);
}

template <class T>
static void step_vjp_any(int method, int sys, int d, const T* y, const T* p, T h,
                         const T* lam, T* lam_in, T* gp) {
  if (is_ros(method)) ros_step_vjp(*ros_of(method), sys, d, y, p, h, lam, lam_in, gp);
  else erk_step_vjp(*erk_of(method), sys, d, y, p, h, lam, lam_in, gp);
}

}  // namespace orc

// ============================================================== C entry ==
using namespace orc;

extern "C" {

int oracle_dims(int sys, int* dim, int* np) {
  *dim = sys_dim(sys);
  *np = sys_np(sys);
  return (*dim > 0) ? 0 : -1;
}

// Export a tableau: c[s], a[s*s] (row-major), b[s], ew[s]; returns s.
int oracle_erk_tableau(int method, double* c, double* a, double* b, double* ew,
                       int* order, int* q_emb) {
  const ERK* m = erk_of(method);
  if (!m) return -1;
  for (int i = 0; i < m->s; ++i) {
    c[i] = m->c[i];
    b[i] = m->b[i];
    ew[i] = m->ew[i];
    for (int j = 0; j < m->s; ++j) a[i * m->s + j] = m->a[i][j];
  }
  *order = m->order;
  *q_emb = m->q_emb;
  return m->s;
}

double oracle_root_inv(double x, int k) { return root_inv(x, k); }

int oracle_rhs(int sys, const double* y, const double* p, double* f) {
  if (sys_dim(sys) < 0) return -1;
  rhs(sys, y, p, f);
  return 0;
}

int oracle_jac(int sys, const double* y, const double* p, double* J) {
  if (sys != SYS_ROBERTSON && sys != SYS_HIRES && sys != SYS_LINEAR) return -1;
  jac(sys, y, p, J);
  return 0;
}

int oracle_jac_vjp(int sys, const double* y, const double* p, const double* u,
                   const double* v, double* gy, double* gp) {
  if (sys != SYS_ROBERTSON && sys != SYS_HIRES && sys != SYS_LINEAR) return -1;
  jac_vjp(sys, y, p, u, v, gy, gp);
  return 0;
}

// A Rosenbrock method (3: Rodas4, 4: Rosenbrock23) in transformed form:
// gamma, a[s*s], c[s*s], m[s], error weights e[s], su; returns s.
int oracle_ros_tableau(int method, double* gamma, double* a, double* c, double* m,
                       double* e, int* order, int* q_emb, int* su) {
  const ROS* rp = ros_of(method);
  if (!rp) return -1;
  const ROS& r = *rp;
  *gamma = r.gamma;
  *su = r.su;
  for (int i = 0; i < r.s; ++i) {
    m[i] = r.m[i];
    e[i] = r.e[i];
    for (int j = 0; j < r.s; ++j) {
      a[i * r.s + j] = r.a[i][j];
      c[i * r.s + j] = r.c[i][j];
    }
  }
  *order = r.order;
  *q_emb = r.q_emb;
  return r.s;
}

// One trial step of a Rosenbrock method from y with step h: y_new and the
// error estimate vector (before scaling).
int oracle_ros_trial(int method, int sys, const double* y, const double* p, double h,
                     double* ynew, double* err) {
  const ROS* rp = ros_of(method);
  const int d = sys_dim(sys);
  if (!rp || d < 0 || (sys != SYS_ROBERTSON && sys != SYS_HIRES && sys != SYS_LINEAR) ||
      h == 0.0)
    return -1;
  double Y[6][DMAX], u[6][DMAX], LU[DMAX * DMAX];
  int perm[DMAX];
  ros_step(*rp, sys, d, y, p, h, rp->s, ynew, Y, u, LU, perm);
  ros_errvec(*rp, d, u, err);
  return 0;
}

int oracle_vjp(int sys, const double* y, const double* p, const double* w,
               double* gy, double* gp) {
  if (sys_dim(sys) < 0) return -1;
  vjp(sys, y, p, w, gy, gp);
  return 0;
}

int oracle_record(int sys, int method, int n, int params_shared,
                  const double* y0, const double* p, double t0, double t1,
                  double rtol, double atol, double h0, int64_t max_steps,
                  int n_save, const double* save_t, int64_t cap, double* h_out,
                  int32_t* S_out, int32_t* status_out, int32_t* save_idx,
                  double* save_dt, double* y_save, int64_t* n_trial) {
  if (sys_dim(sys) < 0 || !(erk_of(method) || is_ros(method)) || n < 0 || n_save < 1 ||
      n_save > 64)
    return -1;
  RecordArgs A{sys, method, n, sys_dim(sys), sys_np(sys), params_shared,
               y0, p, t0, t1, rtol, atol, h0, max_steps, n_save, save_t, cap,
               h_out, S_out, status_out, save_idx, save_dt, y_save, n_trial};
#pragma omp parallel for schedule(dynamic, 64)
  for (int l = 0; l < n; ++l) {
    if (is_ros(method)) ros_record_lane(A, l);
    else record_lane(A, l);
  }
  return 0;
}

// Refresh an old mesh at new inputs (the mesh-drift policy): every lane
// keeps the steps of its old mesh (follow_h [n][follow_cap], follow_S [n])
// while their error estimates stay <= slack, then goes on adaptively; the
// output is a record like oracle_record's, plus drift_at [n] (steps kept).
int oracle_refresh(int sys, int method, int n, int params_shared,
                   const double* y0, const double* p, double t0, double t1,
                   double rtol, double atol, int64_t max_steps,
                   int n_save, const double* save_t, int64_t follow_cap,
                   const double* follow_h, const int32_t* follow_S, double slack,
                   int64_t cap, double* h_out, int32_t* S_out, int32_t* status_out,
                   int32_t* save_idx, double* save_dt, double* y_save, int64_t* n_trial,
                   int32_t* drift_at) {
  if (sys_dim(sys) < 0 || !(erk_of(method) || is_ros(method)) || n < 0 || n_save < 1 ||
      n_save > 64 || !follow_h || !follow_S || follow_cap < 1)
    return -1;
  RecordArgs A{sys, method, n, sys_dim(sys), sys_np(sys), params_shared,
               y0, p, t0, t1, rtol, atol, 0.0, max_steps, n_save, save_t, cap,
               h_out, S_out, status_out, save_idx, save_dt, y_save, n_trial,
               follow_h, follow_S, follow_cap, slack, drift_at};
#pragma omp parallel for schedule(dynamic, 64)
  for (int l = 0; l < n; ++l) {
    if (is_ros(method)) ros_record_lane(A, l);
    else record_lane(A, l);
  }
  return 0;
}

static MeshArgs mesh_args(int sys, int method, int n, int params_shared,
                          int64_t cap, const double* h, const int32_t* S,
                          int n_save, const int32_t* save_idx,
                          const double* save_dt) {
  return MeshArgs{sys, method, n, sys_dim(sys), sys_np(sys), params_shared,
                  cap, h, S, n_save, save_idx, save_dt};
}

// Replay on a frozen mesh in double.
int oracle_replay(int sys, int method, int n, int params_shared,
                  const double* y0, const double* p, int64_t cap,
                  const double* h, const int32_t* S, int n_save,
                  const int32_t* save_idx, const double* save_dt,
                  double* y_save, int dense) {
  if (sys_dim(sys) < 0 || !(erk_of(method) || is_ros(method))) return -1;
  MeshArgs M = mesh_args(sys, method, n, params_shared, cap, h, S, n_save,
                         save_idx, save_dt);
  M.dense = dense;
  const int d = M.d, np = M.np;
#pragma omp parallel for schedule(dynamic, 64)
  for (int l = 0; l < n; ++l) {
    const double* pl = params_shared ? p : p + (int64_t)l * np;
    replay_lane<double>(M, l, y0 + (int64_t)l * d, pl,
                        y_save + (int64_t)l * n_save * d);
  }
  return 0;
}

// Forward-mode (dual number) replay: tangent of the save states along the
// direction (dy0 [n][d], dp [n][np]); per-lane parameters only.
int oracle_replay_dual(int sys, int method, int n, const double* y0,
                       const double* p, const double* dy0, const double* dp,
                       int64_t cap, const double* h, const int32_t* S,
                       int n_save, const int32_t* save_idx,
                       const double* save_dt, double* y_save, double* dy_save, int dense) {
  if (sys_dim(sys) < 0 || !(erk_of(method) || is_ros(method))) return -1;
  MeshArgs M = mesh_args(sys, method, n, 0, cap, h, S, n_save, save_idx, save_dt);
  M.dense = dense;
  const int d = M.d, np = M.np;
#pragma omp parallel for schedule(dynamic, 64)
  for (int l = 0; l < n; ++l) {
    Dual y[DMAX], out[64 * DMAX];
    std::vector<Dual> pp(np);
    for (int c = 0; c < d; ++c)
      y[c] = Dual(y0[(int64_t)l * d + c], dy0[(int64_t)l * d + c]);
    for (int c = 0; c < np; ++c)
      pp[c] = Dual(p[(int64_t)l * np + c], dp[(int64_t)l * np + c]);
    replay_lane<Dual>(M, l, y, pp.data(), out);
    for (int i = 0; i < n_save * d; ++i) {
      y_save[(int64_t)l * n_save * d + i] = out[i].v;
      dy_save[(int64_t)l * n_save * d + i] = out[i].d;
    }
  }
  return 0;
}

// Complex-step replay: inputs y0 + i*eps*dy0, p + i*eps*dp; returns the real
// and imaginary parts of the save states (per-lane parameters only).
int oracle_replay_complex(int sys, int method, int n, const double* y0,
                          const double* p, const double* dy0, const double* dp,
                          double eps, int64_t cap, const double* h,
                          const int32_t* S, int n_save, const int32_t* save_idx,
                          const double* save_dt, double* re, double* im, int dense) {
  if (sys_dim(sys) < 0 || !(erk_of(method) || is_ros(method))) return -1;
  MeshArgs M = mesh_args(sys, method, n, 0, cap, h, S, n_save, save_idx, save_dt);
  M.dense = dense;
  const int d = M.d, np = M.np;
#pragma omp parallel for schedule(dynamic, 64)
  for (int l = 0; l < n; ++l) {
    Cplx y[DMAX], out[64 * DMAX];
    std::vector<Cplx> pp(np);
    for (int c = 0; c < d; ++c)
      y[c] = Cplx(y0[(int64_t)l * d + c], eps * dy0[(int64_t)l * d + c]);
    for (int c = 0; c < np; ++c)
      pp[c] = Cplx(p[(int64_t)l * np + c], eps * dp[(int64_t)l * np + c]);
    replay_lane<Cplx>(M, l, y, pp.data(), out);
    for (int i = 0; i < n_save * d; ++i) {
      re[(int64_t)l * n_save * d + i] = out[i].real();
      im[(int64_t)l * n_save * d + i] = out[i].imag();
    }
  }
  return 0;
}

// Discrete adjoint on a frozen mesh.  grad_p is [n][np] (per lane; for shared
// parameters each lane's contribution is returned separately and the caller
// sums them); grad_y0 is [n][d]; loss_lane is [n].
int oracle_adjoint(int sys, int method, int n, int params_shared,
                   const double* y0, const double* p, int64_t cap,
                   const double* h, const int32_t* S, int n_save,
                   const int32_t* save_idx, const double* save_dt,
                   int loss_kind, const double* loss_data,
                   double loss_scale, double* grad_p, double* grad_y0,
                   double* loss_lane, int dense) {
  if (sys_dim(sys) < 0 || !(erk_of(method) || is_ros(method))) return -1;
  MeshArgs M = mesh_args(sys, method, n, params_shared, cap, h, S, n_save,
                         save_idx, save_dt);
  M.dense = dense;
  LossArgs L{loss_kind, loss_data, loss_scale};
  const int d = M.d, np = M.np;
#pragma omp parallel for schedule(dynamic, 64)
  for (int l = 0; l < n; ++l) {
    const double* pl = params_shared ? p : p + (int64_t)l * np;
    double* gp = grad_p + (int64_t)l * np;
    for (int c = 0; c < np; ++c) gp[c] = 0.0;
    loss_lane[l] = adjoint_lane(M, L, l, y0 + (int64_t)l * d, pl, gp,
                                grad_y0 + (int64_t)l * d);
  }
  return 0;
}

// ------------------------------------------------------- operation counts --
// Floating-point operations of one unit of work, counted by running this
// file's own step routines on the OpCount scalar (the values are irrelevant:
// no routine branches on them except the pivot search, which counts the same
// either way).  out[6] for (method, system):
//   0 trial     one trial step of the record: the stages, y_new, the error
//               estimate and its norm, the controller's proposed factor and
//               the next step size as after a rejection
//   1 accept    what an accepted trial adds: the acceptance bound of the
//               controller, and f(y_new) for a pair without first-same-as-last
//   2 side_fwd  a save-time side step of the record (stages that enter
//               y_new, y_new; the slope at the base point is known)
//   3 adj_step  one mesh step of the reverse sweep (recomputed stages and
//               their vector-Jacobian products)
//   4 adj_side  a save-time side step of the sweep: the step's reverse, its
//               y_new formed from the recomputed stages, the sum-of-squares
//               cotangent and loss term, and the cotangent's addition into
//               the base point's
//   5 adj_zero  a save on a mesh point in the sweep (cotangent, loss term,
//               addition)
//   6 dense_fwd a dense save of the record: the continuous extension from
//               the step's end states (both slopes counted, as evaluated here)
//   7 dense_adj a dense save of the sweep: the extension recomputed, the
//               sum-of-squares cotangent and loss term, its reverse (two
//               VJPs), and both end states' additions
// Time bookkeeping (t + h, the end-of-span clip, the underflow test) is not
// counted.  Returns 0, or -1 for an unknown pair.
int oracle_count_ops(int method, int sys, int64_t* out) {
  const int d = sys_dim(sys), np = sys_np(sys);
  if (d < 0 || !(erk_of(method) || is_ros(method))) return -1;
  std::vector<OpCount> p(np);
  for (int c = 0; c < np; ++c) p[c] = OpCount(0.5 + 0.01 * c);
  OpCount y[DMAX], ynew[DMAX], lam[DMAX], lin[DMAX], w[DMAX];
  std::vector<OpCount> gp(np);
  for (int c = 0; c < d; ++c) {
    y[c] = OpCount(0.3 + 0.1 * c);
    lam[c] = OpCount(1.0);
  }
  const OpCount h(1e-3);
  const int kroot = is_ros(method) ? ros_of(method)->q_emb + 1 : erk_of(method)->q_emb + 1;
  auto count = [&](auto&& fn) {
    g_ops = 0;
    fn();
    return g_ops;
  };
  int64_t update = 0;  // y_new from the stages of a replay step
  if (is_ros(method)) {
    const ROS& m = *ros_of(method);
    OpCount Y[6][DMAX], u[6][DMAX], LU[DMAX * DMAX];
    int perm[DMAX];
    out[0] = count([&] {
      ros_step(m, sys, d, y, p.data(), h, m.s, ynew, Y, u, LU, perm);
      OpCount fac0 = ctrl_fac0(ros_err(m, d, y, ynew, u, 1e-6, 1e-8), kroot);
      ctrl_reject(h, fac0);
    });
    out[1] = count([&] { ctrl_accept(h, OpCount(1.0), false); }) -
             count([&] { ctrl_reject(h, OpCount(1.0)); });
    out[2] = count([&] { ros_step(m, sys, d, y, p.data(), h, m.su, ynew, Y, u, LU, perm); });
    update = out[2] - count([&] {
      ros_step(m, sys, d, y, p.data(), h, m.su, (OpCount*)nullptr, Y, u, LU, perm);
    });
  } else {
    const ERK& m = *erk_of(method);
    OpCount k[SMAX][DMAX], Y[SMAX][DMAX];
    g_ops = 0;
    rhs(sys, y, p.data(), k[0]);  // the slope at the base point is known
    out[0] = count([&] {
      erk_stages(m, sys, d, y, p.data(), h, m.s, k, Y);
      if (m.fsal) {
        for (int c = 0; c < d; ++c) ynew[c] = Y[m.s - 1][c];
      } else {
        erk_update(m, d, y, h, k, ynew);
      }
      OpCount fac0 = ctrl_fac0(erk_err(m, d, h, y, ynew, k, 1e-6, 1e-8), kroot);
      ctrl_reject(h, fac0);
    });
    out[1] = count([&] { ctrl_accept(h, OpCount(1.0), false); }) -
             count([&] { ctrl_reject(h, OpCount(1.0)); }) +
             (m.fsal ? 0 : count([&] { rhs(sys, ynew, p.data(), k[0]); }));
    out[2] = count([&] {
      erk_stages(m, sys, d, y, p.data(), h, m.s_used, k, Y);
      erk_update(m, d, y, h, k, ynew);
    });
    update = count([&] { erk_update(m, d, y, h, k, ynew); });
  }
  out[3] = count([&] { step_vjp_any(method, sys, d, y, p.data(), h, lam, lin, gp.data()); });
  const int64_t cot = count([&] {
    OpCount loss(0.0);
    for (int c = 0; c < d; ++c) loss_cot(LOSS_SUMSQ, y[c], 0.0, OpCount(2.0), loss, w[c]);
  });
  const int64_t add = count([&] {
    for (int c = 0; c < d; ++c) lam[c] = lam[c] + lin[c];
  });
  out[4] = out[3] + update + cot + add;
  out[5] = cot + add;
  OpCount y1[DMAX], lo[DMAX], hi[DMAX];
  for (int c = 0; c < d; ++c) y1[c] = OpCount(0.35 + 0.1 * c);
  out[6] = count([&] { dense_state(sys, d, y, y1, p.data(), 1e-3, 4e-4, w); });
  out[7] = out[6] + cot +
           count([&] { dense_save_vjp(sys, d, y, y1, p.data(), 1e-3, 4e-4, lam, lo, hi, gp.data()); }) +
           2 * add;
  return 0;
}

// Operations of one evaluation of a system's f, its VJP ((df/dy)^T w with
// the parameter terms), its Jacobian and d/d(y, p) of u^T J v (the last two
// for the stiff systems only, else 0): out[4].
int oracle_count_system(int sys, int64_t* out) {
  const int d = sys_dim(sys), np = sys_np(sys);
  if (d < 0) return -1;
  std::vector<OpCount> p(np), gp(np);
  for (int c = 0; c < np; ++c) p[c] = OpCount(0.5 + 0.01 * c);
  OpCount y[DMAX], f[DMAX], w[DMAX], gy[DMAX], J[DMAX * DMAX];
  for (int c = 0; c < d; ++c) {
    y[c] = OpCount(0.3 + 0.1 * c);
    w[c] = OpCount(1.0);
  }
  const bool stiff = sys == SYS_ROBERTSON || sys == SYS_HIRES || sys == SYS_LINEAR;
  g_ops = 0;
  rhs(sys, y, p.data(), f);
  out[0] = g_ops;
  g_ops = 0;
  vjp(sys, y, p.data(), w, gy, gp.data());
  out[1] = g_ops;
  out[2] = out[3] = 0;
  if (stiff) {
    g_ops = 0;
    jac(sys, y, p.data(), J);
    out[2] = g_ops;
    g_ops = 0;
    jac_vjp(sys, y, p.data(), w, f, gy, gp.data());
    out[3] = g_ops;
  }
  return 0;
}

// Operations of the linear algebra of W = I/(gamma h) - J at the counting
// point (h = 1e-3, gamma = 1/4): the factorisation, one solve and one
// transposed solve, counted with the LU rule above.
int oracle_count_lu(int sys, int64_t* out) {
  const int d = sys_dim(sys), np = sys_np(sys);
  if (d < 0 || !(sys == SYS_ROBERTSON || sys == SYS_HIRES || sys == SYS_LINEAR)) return -1;
  std::vector<OpCount> p(np);
  for (int c = 0; c < np; ++c) p[c] = OpCount(0.5 + 0.01 * c);
  OpCount y[DMAX], b[DMAX], x[DMAX], LU[DMAX * DMAX];
  for (int c = 0; c < d; ++c) {
    y[c] = OpCount(0.3 + 0.1 * c);
    b[c] = OpCount(1.0 + 0.1 * c);
  }
  int perm[DMAX];
  jac(sys, y, p.data(), LU);
  const OpCount dg = OpCount(1.0) / (OpCount(0.25) * OpCount(1e-3));
  for (int i = 0; i < d * d; ++i) LU[i] = -LU[i];
  for (int i = 0; i < d; ++i) LU[i * d + i] = LU[i * d + i] + dg;
  g_ops = 0;
  lu_factor(d, LU, perm);
  out[0] = g_ops;
  g_ops = 0;
  lu_solve(d, LU, perm, b, x);
  out[1] = g_ops;
  g_ops = 0;
  lu_solve_t(d, LU, perm, b, x);
  out[2] = g_ops;
  int swaps = 0;
  for (int i = 0; i < d; ++i) swaps += perm[i] != i;
  out[3] = swaps;
  return 0;
}

}  // extern "C"
