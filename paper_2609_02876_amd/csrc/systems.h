// Right-hand sides and vector-Jacobian products of the built-in autonomous
// systems (paper, Appendix A), one trajectory per GPU lane.
//
// rhs(y, p, f)          f = f(y, p)
// vjp(y, p, w, gy, gp)  gy = (df/dy)^T w (overwritten), gp += (df/dp)^T w
//
// The fma placement is part of the definition: it fixes the rounding of
// every result, so these functions agree bit for bit with any other
// implementation that writes the same expressions.
#pragma once
#include "ens_device.h"

namespace ens {

// Lorenz: p = (sigma, rho, beta)
//   f0 = sigma (y1 - y0), f1 = y0 (rho - y2) - y1, f2 = y0 y1 - beta y2
struct Lorenz {
  static constexpr int D = 3, NP = 3, ID = 1;
  template <class T>
  __device__ static inline void rhs(const T* y, const T* p, T* f) {
    f[0] = p[0] * (y[1] - y[0]);
    f[1] = fmaT(y[0], p[1] - y[2], -y[1]);
    f[2] = fmaT(y[0], y[1], -(p[2] * y[2]));
  }
  template <class T>
  __device__ static inline void vjp(const T* y, const T* p, const T* w, T* gy,
                                    T* gp) {
    gy[0] = fmaT(y[1], w[2], fmaT(p[1] - y[2], w[1], -(p[0] * w[0])));
    gy[1] = fmaT(y[0], w[2], fmaT(p[0], w[0], -w[1]));
    gy[2] = -fmaT(y[0], w[1], p[2] * w[2]);
    gp[0] = fmaT(y[1] - y[0], w[0], gp[0]);
    gp[1] = fmaT(y[0], w[1], gp[1]);
    gp[2] = fmaT(-y[2], w[2], gp[2]);
  }
};

// Van der Pol: p = (mu);  f0 = y1,  f1 = mu ((1 - y0^2) y1 - y0)
struct VanDerPol {
  static constexpr int D = 2, NP = 1, ID = 2;
  template <class T>
  __device__ static inline void rhs(const T* y, const T* p, T* f) {
    f[0] = y[1];
    f[1] = p[0] * fmaT(fmaT(-y[0], y[0], T(1)), y[1], -y[0]);
  }
  template <class T>
  __device__ static inline void vjp(const T* y, const T* p, const T* w, T* gy,
                                    T* gp) {
    const T u = p[0] * w[1];
    const T q = fmaT(-y[0], y[0], T(1));
    gy[0] = u * fmaT(T(-2) * y[0], y[1], T(-1));
    gy[1] = fmaT(u, q, w[0]);
    gp[0] = fmaT(w[1], fmaT(q, y[1], -y[0]), gp[0]);
  }
};

// Damped rotation y' = A y, A = [[-a, -w], [w, -a]]: p = (a, w)
// jac(y, p, J)               J = df/dy, row-major (stiff solvers)
// jac_vjp(y, p, u, v, gy, gp) gy, gp += d/d(y, p) of u^T J(y, p) v
struct Linear {
  static constexpr int D = 2, NP = 2, ID = 6;
  template <class T>
  __device__ static inline void jac(const T* y, const T* p, T* J) {
    J[0] = -p[0];
    J[1] = -p[1];
    J[2] = p[1];
    J[3] = -p[0];
  }
  template <class T>
  __device__ static inline void jac_vjp(const T* y, const T* p, const T* u, const T* v,
                                        T* gy, T* gp) {
    gp[0] = gp[0] - fmaT(u[0], v[0], u[1] * v[1]);
    gp[1] = gp[1] + fmaT(u[1], v[0], -(u[0] * v[1]));
  }
  template <class T>
  __device__ static inline void rhs(const T* y, const T* p, T* f) {
    f[0] = -fmaT(p[0], y[0], p[1] * y[1]);
    f[1] = fmaT(p[1], y[0], -(p[0] * y[1]));
  }
  template <class T>
  __device__ static inline void vjp(const T* y, const T* p, const T* w, T* gy,
                                    T* gp) {
    gy[0] = fmaT(p[1], w[1], -(p[0] * w[0]));
    gy[1] = -fmaT(p[1], w[0], p[0] * w[1]);
    gp[0] = gp[0] - fmaT(y[0], w[0], y[1] * w[1]);
    gp[1] = gp[1] + fmaT(y[0], w[1], -(y[1] * w[0]));
  }
};

// Robertson kinetics: p = (k1, k2, k3);  a = k1 y0, b = k3 y1 y2, c = k2 y1^2,
//   f0 = b - a,  f1 = (a - b) - c,  f2 = c.
struct Robertson {
  static constexpr int D = 3, NP = 3, ID = 3;
  // nonzero pattern of the Jacobian, row i: bit j where dF_i/dy_j is not
  // identically zero
  static constexpr unsigned JAC_ROWS[3] = {0x7u, 0x7u, 0x2u};
  template <class T>
  __device__ static inline void rhs(const T* y, const T* p, T* f) {
    const T a = p[0] * y[0];
    const T b = (p[2] * y[1]) * y[2];
    const T c = (p[1] * y[1]) * y[1];
    f[0] = b - a;
    f[1] = (a - b) - c;
    f[2] = c;
  }
  template <class T>
  __device__ static inline void jac(const T* y, const T* p, T* J) {
    const T s2 = p[2] * y[2], s1 = p[2] * y[1], q = p[1] * y[1];
    J[0] = -p[0];
    J[1] = s2;
    J[2] = s1;
    J[3] = p[0];
    J[4] = -s2 - (q + q);
    J[5] = -s1;
    J[6] = T(0);
    J[7] = q + q;
    J[8] = T(0);
  }
  template <class T>
  __device__ static inline void vjp(const T* y, const T* p, const T* w, T* gy, T* gp) {
    const T s2 = p[2] * y[2], s1 = p[2] * y[1], q = p[1] * y[1];
    gy[0] = p[0] * (w[1] - w[0]);
    gy[1] = fmaT(s2, w[0] - w[1], (q + q) * (w[2] - w[1]));
    gy[2] = s1 * (w[0] - w[1]);
    gp[0] = fmaT(y[0], w[1] - w[0], gp[0]);
    gp[1] = fmaT(y[1] * y[1], w[2] - w[1], gp[1]);
    gp[2] = fmaT(y[1] * y[2], w[0] - w[1], gp[2]);
  }
  template <class T>
  __device__ static inline void jac_vjp(const T* y, const T* p, const T* u, const T* v,
                                        T* gy, T* gp) {
    const T du = u[0] - u[1];
    const T t = (p[1] + p[1]) * (v[1] * (u[2] - u[1]));
    gy[1] = gy[1] + fmaT(p[2] * v[2], du, t);
    gy[2] = gy[2] + (p[2] * v[1]) * du;
    gp[0] = gp[0] + v[0] * (u[1] - u[0]);
    gp[1] = gp[1] + (y[1] + y[1]) * (v[1] * (u[2] - u[1]));
    gp[2] = gp[2] + du * fmaT(y[2], v[1], y[1] * v[2]);
  }
};

// HIRES: p = the twelve rate literals of the model in order of first
// appearance (1.71, 0.43, 8.32, 0.0007, 8.75, 10.03, 0.035, 1.12, 1.745, 280,
// 0.69, 1.81); f7 = -f6 keeps y6 + y7 constant to the bit.
struct Hires {
  static constexpr int D = 8, NP = 12, ID = 4;
  // nonzero pattern of the Jacobian (as jac below writes it), row i: bit j
  // where dF_i/dy_j is not identically zero
  static constexpr unsigned JAC_ROWS[8] = {0x07u, 0x03u, 0x1Cu, 0x0Eu, 0x70u, 0xF8u, 0xE0u, 0xE0u};
  template <class T>
  __device__ static inline void rhs(const T* y, const T* p, T* f) {
    f[0] = fmaT(p[2], y[2], fmaT(p[1], y[1], fmaT(-p[0], y[0], p[3])));
    f[1] = fmaT(p[0], y[0], -(p[4] * y[1]));
    f[2] = fmaT(p[6], y[4], fmaT(p[1], y[3], -(p[5] * y[2])));
    f[3] = fmaT(p[2], y[1], fmaT(p[0], y[2], -(p[7] * y[3])));
    f[4] = fmaT(p[1], y[6], fmaT(p[1], y[5], -(p[8] * y[4])));
    const T z = (p[9] * y[5]) * y[7];
    f[5] = fmaT(p[10], y[6], fmaT(-p[1], y[5], fmaT(p[0], y[4], fmaT(p[10], y[3], -z))));
    f[6] = fmaT(-p[11], y[6], z);
    f[7] = -f[6];
  }
  template <class T>
  __device__ static inline void jac(const T* y, const T* p, T* J) {
#pragma unroll
    for (int i = 0; i < 64; ++i) J[i] = T(0);
    const T a = p[9] * y[7], b = p[9] * y[5];
    J[0 * 8 + 0] = -p[0]; J[0 * 8 + 1] = p[1]; J[0 * 8 + 2] = p[2];
    J[1 * 8 + 0] = p[0];  J[1 * 8 + 1] = -p[4];
    J[2 * 8 + 2] = -p[5]; J[2 * 8 + 3] = p[1]; J[2 * 8 + 4] = p[6];
    J[3 * 8 + 1] = p[2];  J[3 * 8 + 2] = p[0]; J[3 * 8 + 3] = -p[7];
    J[4 * 8 + 4] = -p[8]; J[4 * 8 + 5] = p[1]; J[4 * 8 + 6] = p[1];
    J[5 * 8 + 3] = p[10]; J[5 * 8 + 4] = p[0]; J[5 * 8 + 5] = -a - p[1];
    J[5 * 8 + 6] = p[10]; J[5 * 8 + 7] = -b;
    J[6 * 8 + 5] = a;     J[6 * 8 + 6] = -p[11]; J[6 * 8 + 7] = b;
    J[7 * 8 + 5] = -a;    J[7 * 8 + 6] = p[11];  J[7 * 8 + 7] = -b;
  }
  template <class T>
  __device__ static inline void vjp(const T* y, const T* p, const T* w, T* gy, T* gp) {
    const T a = p[9] * y[7], b = p[9] * y[5];
    gy[0] = p[0] * (w[1] - w[0]);
    gy[1] = fmaT(p[2], w[3], fmaT(p[1], w[0], -(p[4] * w[1])));
    gy[2] = fmaT(p[0], w[3], fmaT(p[2], w[0], -(p[5] * w[2])));
    gy[3] = fmaT(p[10], w[5], fmaT(p[1], w[2], -(p[7] * w[3])));
    gy[4] = fmaT(p[0], w[5], fmaT(p[6], w[2], -(p[8] * w[4])));
    gy[5] = fmaT(a, (w[6] - w[7]) - w[5], p[1] * (w[4] - w[5]));
    gy[6] = fmaT(p[11], w[7] - w[6], fmaT(p[10], w[5], p[1] * w[4]));
    gy[7] = b * ((w[6] - w[5]) - w[7]);
    gp[0] = gp[0] + fmaT(y[4], w[5], fmaT(y[2], w[3], y[0] * (w[1] - w[0])));
    gp[1] = gp[1] + fmaT(y[5] + y[6], w[4], fmaT(y[3], w[2], fmaT(y[1], w[0], -(y[5] * w[5]))));
    gp[2] = gp[2] + fmaT(y[2], w[0], y[1] * w[3]);
    gp[3] = gp[3] + w[0];
    gp[4] = gp[4] - y[1] * w[1];
    gp[5] = gp[5] - y[2] * w[2];
    gp[6] = gp[6] + y[4] * w[2];
    gp[7] = gp[7] - y[3] * w[3];
    gp[8] = gp[8] - y[4] * w[4];
    gp[9] = gp[9] + (y[5] * y[7]) * ((w[6] - w[5]) - w[7]);
    gp[10] = gp[10] + (y[3] + y[6]) * w[5];
    gp[11] = gp[11] + y[6] * (w[7] - w[6]);
  }
  template <class T>
  __device__ static inline void jac_vjp(const T* y, const T* p, const T* u, const T* v,
                                        T* gy, T* gp) {
    const T du = (u[6] - u[5]) - u[7];
    gy[5] = gy[5] + (p[9] * v[7]) * du;
    gy[7] = gy[7] + (p[9] * v[5]) * du;
    gp[0] = gp[0] + fmaT(u[5], v[4], fmaT(u[3], v[2], v[0] * (u[1] - u[0])));
    gp[1] = gp[1] + fmaT(u[4], v[5] + v[6], fmaT(u[2], v[3], fmaT(u[0], v[1], -(u[5] * v[5]))));
    gp[2] = gp[2] + fmaT(u[0], v[2], u[3] * v[1]);
    gp[4] = gp[4] - u[1] * v[1];
    gp[5] = gp[5] - u[2] * v[2];
    gp[6] = gp[6] + u[2] * v[4];
    gp[7] = gp[7] - u[3] * v[3];
    gp[8] = gp[8] - u[4] * v[4];
    gp[9] = gp[9] + du * fmaT(y[7], v[5], y[5] * v[7]);
    gp[10] = gp[10] + u[5] * (v[3] + v[6]);
    gp[11] = gp[11] + v[6] * (u[7] - u[6]);
  }
};

}  // namespace ens
