// Forward-mode replay on a recorded mesh (paper, Section 4: forward mode for
// few inputs; the mesh held fixed as in the reverse sweep, Section 3.1).
//
// One pass carries one tangent direction (dy0, dtheta) per trajectory through
// the replay y_i = Phi(y_{i-1}; h_i, theta) in dual numbers and returns the
// tangents of the save states and of the loss.  Changing the same input of
// every trajectory in one pass gives each trajectory's own derivative with
// respect to that input, so a trajectory with P inputs needs P passes,
// whatever the ensemble size.
#pragma once
#include "erk.h"

namespace ens {

// Dual number v + eps d.  Each operation forms its tangent exactly as written
// here (products left to right, then sums, no fused multiply-add in the
// tangent), which fixes the rounding of every tangent.
template <class R>
struct Dual {
  R v, d;
  Dual() = default;
  __device__ __forceinline__ Dual(R x) : v(x), d(R(0)) {}
  __device__ __forceinline__ Dual(R x, R dx) : v(x), d(dx) {}
  // |x| for pivot search: only its value is ever compared (found by
  // argument-dependent lookup only, so it hides no other fabs)
  friend __device__ __forceinline__ Dual fabs(Dual a) {
    return {a.v < R(0) ? -a.v : a.v, a.v < R(0) ? -a.d : a.d};
  }
};

template <class R>
__device__ __forceinline__ Dual<R> operator+(Dual<R> a, Dual<R> b) {
  return {a.v + b.v, a.d + b.d};
}
template <class R>
__device__ __forceinline__ Dual<R> operator-(Dual<R> a, Dual<R> b) {
  return {a.v - b.v, a.d - b.d};
}
template <class R>
__device__ __forceinline__ Dual<R> operator-(Dual<R> a) {
  return {-a.v, -a.d};
}
template <class R>
__device__ __forceinline__ Dual<R> operator*(Dual<R> a, Dual<R> b) {
  return {a.v * b.v, a.d * b.v + a.v * b.d};
}
template <class R>
__device__ __forceinline__ Dual<R> operator/(Dual<R> a, Dual<R> b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
template <class R>
__device__ __forceinline__ Dual<R> fmaT(Dual<R> a, Dual<R> b, Dual<R> c) {
  return {fmaT(a.v, b.v, c.v), (a.d * b.v + a.v * b.d) + c.d};
}
template <class R>
__device__ __forceinline__ bool operator>(Dual<R> a, Dual<R> b) {
  return a.v > b.v;
}
// A factor without tangent (a method coefficient, the step size or its
// inverse: the mesh is fixed) contributes only its product with the other
// operand's tangent.  These give the same bits as the general operations
// above with that factor's tangent zero, whenever the other operand is finite.
template <class R>
__device__ __forceinline__ Dual<R> cmul(double c, Dual<R> x) {
  return {R(c) * x.v, R(c) * x.d};
}
template <class R>
__device__ __forceinline__ Dual<R> cfma(double c, Dual<R> x, Dual<R> acc) {
  return {fmaT(R(c), x.v, acc.v), R(c) * x.d + acc.d};
}
template <class R>
__device__ __forceinline__ Dual<R> hfma(Dual<R> h, Dual<R> x, Dual<R> acc) {
  return {fmaT(h.v, x.v, acc.v), h.v * x.d + acc.d};
}
template <class R>
__device__ __forceinline__ Dual<R> fmah(Dual<R> x, Dual<R> h, Dual<R> acc) {
  return {fmaT(x.v, h.v, acc.v), x.d * h.v + acc.d};
}

// select part by part (a select of whole structs goes through memory)
template <class R>
__device__ __forceinline__ Dual<R> pick(bool c, Dual<R> a, Dual<R> b) {
  return {c ? a.v : b.v, c ? a.d : b.d};
}

struct JvpArgs {
  IvpArgs ivp;
  RecView rec;
  const void* dy0;        // [D][n] or null (zero)
  const void* dp;         // [NP][n] or null (zero)
  int32_t loss_kind;      // LOSS_* or -1: no loss tangent
  const void* loss_data;  // [n_save][D][n]: targets (MSE) or cotangents
  double scale;
  void* ys_dot;           // [n_save][D][n] or null
  double* loss_dot;       // [n] or null
  int64_t rec_b;          // bytes from one step's h to the next within a page
  int64_t h_off;          // offset of the first h in a page
};

// Phi(y; h) in dual numbers: the replay's step (stages 1..SU, update
// y + h sum_j b_j k_j), or for a Rosenbrock method its transformed stages
// with the factorisation of W = I/(gamma h) - J carried in dual numbers
// (pivots chosen on values); a Rosenbrock step of size 0 is the identity.
template <class Sys, class Tab, class DT>
__device__ __forceinline__ void jvp_phi(const DT* y, const DT* p, double h, DT* yn) {
  constexpr int D = Sys::D;
  if constexpr (Tab::ROS) {
    const bool zero = (h == 0.0);
    DT W[D * D], u[Tab::S][D], ys[D];
    int piv[D];
    ros_step<Sys, Tab, DT, Tab::SU>(y, p, DT(zero ? 1.0 : h), W, piv, u, ys);
#pragma unroll
    for (int c = 0; c < D; ++c) yn[c] = pick(zero, y[c], ys[c]);
  } else {
    DT k0[D], Yd[Tab::SU][D], ylast[D], klast[D];
    Sys::rhs(y, p, k0);
    step_push<Sys, Tab, DT, Tab::SU, false, true, false>(y, k0, p, DT(h), Yd, ylast, klast,
                                                         yn, nullptr);
  }
}

// One trajectory per lane.  Loss tangents, accumulated over saves (in save
// order) and components (in index order) by fma in double:
//   SUMSQ:      2 scale sum y . ydot
//   MSE_TARGET: 2 scale sum (y - target) . ydot
//   COTANGENT:  sum c . ydot
// A trajectory whose record failed gets NaN tangents.
// The FP64 Lorenz / Tsit5 pass is held to 128 VGPRs, four waves per SIMD.
template <class Sys, class Tab, class T>
struct JvpBlocks {
  static constexpr int value =
      (Sys::ID == 1 && Tab::ORDER == 5 && !Tab::ROS && sizeof(T) == 8) ? 4 : 1;
};

template <class Sys, class Tab, class T>
__global__ void __launch_bounds__(256, (JvpBlocks<Sys, Tab, T>::value)) jvp_kernel(const JvpArgs a) {
  using DT = Dual<T>;
  constexpr int D = Sys::D, NP = Sys::NP;
  const int64_t n = a.ivp.n;
  const int64_t tr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tr >= n) return;
  const RecView& R = a.rec;
  const int ns = R.n_save;
  T* ysd = (T*)a.ys_dot;
  if (R.status[tr] != LANE_OK) {
    if (ysd)
      for (int s = 0; s < ns; ++s)
#pragma unroll
        for (int c = 0; c < D; ++c) ysd[((int64_t)s * D + c) * n + tr] = T(NAN);
    if (a.loss_dot) a.loss_dot[tr] = NAN;
    return;
  }
  DT y[D], p[NP];
  const T* y0 = (const T*)a.ivp.y0;
  const T* dy0 = (const T*)a.dy0;
  const T* P = (const T*)a.ivp.params;
  const T* dP = (const T*)a.dp;
#pragma unroll
  for (int c = 0; c < D; ++c) y[c] = DT(y0[c * n + tr], dy0 ? dy0[c * n + tr] : T(0));
#pragma unroll
  for (int c = 0; c < NP; ++c) p[c] = DT(P[c * n + tr], dP ? dP[c * n + tr] : T(0));

  const T* data = (const T*)a.loss_data;
  double ldot = 0.0;
  const int32_t S = R.steps[tr];
  const int K = R.page_steps;
  int32_t page = R.static_pages > 0 ? (int32_t)(tr * R.static_pages) : R.first_page[tr];
  int s = 0;
  int32_t sidx = R.save_idx[tr];
  double sdt = R.save_dt[tr];
  // One step of the dual-number map a trip: a save step (size t_s - t_i from
  // y_i, whose state is an output) while a save's base is y_i, else mesh step
  // i.  Taking either kind through the same call keeps the lanes of a
  // wavefront in one step evaluation whichever kind each needs; a save step
  // taken as a second call beside the mesh step would cost the wavefront two
  // evaluations on nearly every trip, since some lane saves on most of them.
  int32_t i = 0;
  for (;;) {
    const bool save = s < ns && sidx == i;
    if (!save && i >= S) break;
    double hh = sdt;
    if (!save) {
      const int slot = i % K;
      if (i > 0 && slot == 0) page = next_page(R, tr, page);
      hh = *(const double*)(R.pages + (int64_t)page * R.page_bytes + a.h_off + slot * a.rec_b);
    }
    DT yn[D];
    jvp_phi<Sys, Tab, DT>(y, p, hh, yn);
    if (save) {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        if (ysd) ysd[((int64_t)s * D + c) * n + tr] = yn[c].d;
        const double dv = (double)yn[c].d;
        if (a.loss_kind == LOSS_SUMSQ) {
          ldot = fmaT((double)yn[c].v, dv, ldot);
        } else if (a.loss_kind == LOSS_MSE_TARGET) {
          const T r = yn[c].v - data[((int64_t)s * D + c) * n + tr];
          ldot = fmaT((double)r, dv, ldot);
        } else if (a.loss_kind == LOSS_COTANGENT) {
          ldot = fmaT((double)data[((int64_t)s * D + c) * n + tr], dv, ldot);
        }
      }
      ++s;
      if (s < ns) {
        sidx = R.save_idx[(int64_t)s * n + tr];
        sdt = R.save_dt[(int64_t)s * n + tr];
      }
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) y[c] = yn[c];
      ++i;
    }
  }
  if (a.loss_dot)
    a.loss_dot[tr] = a.loss_kind == LOSS_COTANGENT ? ldot : 2.0 * a.scale * ldot;
}

}  // namespace ens
