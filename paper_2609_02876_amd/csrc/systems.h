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
struct Linear {
  static constexpr int D = 2, NP = 2, ID = 6;
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

}  // namespace ens
