"""Example sources for binding.register_system: systems given as text and
compiled at run time.  They restate built-in systems with the same
operations, so a registered copy computes the same bits as the built-in one
(which is how the run-time path is tested); a new system is written the same
way."""

# Lorenz, p = (sigma, rho, beta)
LORENZ = """
struct System {
  template <class T>
  __device__ static void rhs(const T* y, const T* p, T* f) {
    f[0] = p[0] * (y[1] - y[0]);
    f[1] = fmaT(y[0], p[1] - y[2], -y[1]);
    f[2] = fmaT(y[0], y[1], -(p[2] * y[2]));
  }
  template <class T>
  __device__ static void vjp(const T* y, const T* p, const T* w, T* gy, T* gp) {
    gy[0] = fmaT(y[1], w[2], fmaT(p[1] - y[2], w[1], -(p[0] * w[0])));
    gy[1] = fmaT(y[0], w[2], fmaT(p[0], w[0], -w[1]));
    gy[2] = -fmaT(y[0], w[1], p[2] * w[2]);
    gp[0] = fmaT(y[1] - y[0], w[0], gp[0]);
    gp[1] = fmaT(y[0], w[1], gp[1]);
    gp[2] = fmaT(-y[2], w[2], gp[2]);
  }
};
"""

# Robertson kinetics, p = (k1, k2, k3), with the Jacobian terms Rodas4 needs
ROBERTSON = """
struct System {
  template <class T>
  __device__ static void rhs(const T* y, const T* p, T* f) {
    const T a = p[0] * y[0];
    const T b = (p[2] * y[1]) * y[2];
    const T c = (p[1] * y[1]) * y[1];
    f[0] = b - a;
    f[1] = (a - b) - c;
    f[2] = c;
  }
  template <class T>
  __device__ static void jac(const T* y, const T* p, T* J) {
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
  __device__ static void vjp(const T* y, const T* p, const T* w, T* gy, T* gp) {
    const T s2 = p[2] * y[2], s1 = p[2] * y[1], q = p[1] * y[1];
    gy[0] = p[0] * (w[1] - w[0]);
    gy[1] = fmaT(s2, w[0] - w[1], (q + q) * (w[2] - w[1]));
    gy[2] = s1 * (w[0] - w[1]);
    gp[0] = fmaT(y[0], w[1] - w[0], gp[0]);
    gp[1] = fmaT(y[1] * y[1], w[2] - w[1], gp[1]);
    gp[2] = fmaT(y[1] * y[2], w[0] - w[1], gp[2]);
  }
  template <class T>
  __device__ static void jac_vjp(const T* y, const T* p, const T* u, const T* v, T* gy, T* gp) {
    const T du = u[0] - u[1];
    const T t = (p[1] + p[1]) * (v[1] * (u[2] - u[1]));
    gy[1] = gy[1] + fmaT(p[2] * v[2], du, t);
    gy[2] = gy[2] + (p[2] * v[1]) * du;
    gp[0] = gp[0] + v[0] * (u[1] - u[0]);
    gp[1] = gp[1] + (y[1] + y[1]) * (v[1] * (u[2] - u[1]));
    gp[2] = gp[2] + du * fmaT(y[2], v[1], y[1] * v[2]);
  }
};
"""
