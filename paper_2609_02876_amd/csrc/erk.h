// Explicit Runge-Kutta ensemble kernels: forward solve, record (adaptive or
// on a given mesh) and the reverse sweep.  One trajectory per lane; the
// state, the parameters and the stage vectors live in registers.
//
// Paper references: trial step eq. (stages)/(update) and the embedded error
// estimate, RMS test and controller of Section 2.1; record and replay of
// Section 3.1 (eq. replay); save states by one extra step (Section 3.4).
//
// Control flow is kept uniform across a wavefront: every loop iteration of a
// lane is one step evaluation Phi(y_base; h) whose base and size are chosen
// by selects -- a trial from the current state, or a side step from the base
// of the last accepted step to a save time.  The reverse sweep is the same:
// one VJP of Phi per iteration, for a mesh step or a save-time side step.
#pragma once
#ifndef __HIPCC_RTC__
#include <math.h>
#endif

#include "ens_device.h"
#include "ros.h"
#include "systems.h"
#include "tableaux.h"

namespace ens {

constexpr double EPS64 = 2.220446049250313e-16;

enum : int { MODE_SOLVE = 0, MODE_RECORD = 1, MODE_FROZEN = 2, MODE_REFRESH = 3 };

// Save times travel by value in the kernel arguments (constant memory).
struct SaveTimes {
  double t[64];
  int n;
};

// t[i] for a lane-varying i without indexing the argument block dynamically.
__device__ __forceinline__ double save_time_at(const SaveTimes& st, int i) {
  return st.t[i];
}

struct IvpArgs {
  int64_t n;
  const void* y0;      // [D][n]
  const void* params;  // [NP][n] or [NP]
  int32_t params_shared;
  double t0, t1, rtol, atol, h0;
  int64_t max_steps;
  int32_t n_save;  // >= 1 (t1 alone when the caller asks for none)
  SaveTimes st;
};

struct FwdArgs {
  IvpArgs ivp;
  RecView rec;
  void* y_save;           // [n_save][D][n]
  int32_t* lane_status;   // [n]
  const double* mesh_h;   // MODE_FROZEN, MODE_REFRESH: [cap][n]
  const int32_t* mesh_S;  // MODE_FROZEN, MODE_REFRESH: [n]
  int64_t cap;
  double slack;           // MODE_REFRESH: an old step is kept while err <= slack
  int32_t* drift_at;      // MODE_REFRESH: [n] old steps kept, or null
};

struct AdjArgs {
  IvpArgs ivp;
  RecView rec;
  int32_t loss_kind;
  const void* loss_data;  // [n_save][D][n]
  double scale;
  void* grad_p;           // [NP][n]
  void* grad_y0;          // [D][n] or null
  double* loss_out;       // [n] or null
  void* workspace;        // shared parameters: [n_blocks][NP] partials
  void* scratch;          // checkpointed tape: [n][page_steps] step records
  void* contrib;          // [n_save][D][n]: each save's cotangent for its base state
                          // (dense output: [2 n_save][D][n], one per event below)
  int32_t* events;        // dense output: [2 n_save][n] mesh point of each cotangent
};

// ------------------------------------------------------------ one step --
// Stage inputs Y_i = y + h * sum_j a_ij k_j (index order, fma) and stage
// values k_i = f(Y_i) for i = 1..NST-1; k[0] = f(y) is given.
template <class Sys, class Tab, class T, int NST>
__device__ __forceinline__ void stages(const T* y, const T* p, T h,
                                       T (&k)[NST][Sys::D],
                                       T (&Y)[NST][Sys::D]) {
  constexpr int D = Sys::D;
#pragma unroll
  for (int c = 0; c < D; ++c) Y[0][c] = y[c];
#pragma unroll
  for (int i = 1; i < NST; ++i) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T acc = T(0);
      bool first = true;
#pragma unroll
      for (int j = 0; j < i; ++j) {
        if (Tab::A[i][j] != 0.0) {
          if (first) {
            acc = T(Tab::A[i][j]) * k[j][c];
            first = false;
          } else {
            acc = fmaT(T(Tab::A[i][j]), k[j][c], acc);
          }
        }
      }
      Y[i][c] = fmaT(h, acc, y[c]);
    }
    Sys::rhs(Y[i], p, k[i]);
  }
}

// y_new = y + h * sum_j b_j k_j over the stages with b_j != 0.
template <class Tab, class T, int D, int NST>
__device__ __forceinline__ void update(const T* y, T h, const T (&k)[NST][D],
                                       T* ynew) {
#pragma unroll
  for (int c = 0; c < D; ++c) {
    T acc = T(0);
    bool first = true;
#pragma unroll
    for (int j = 0; j < NST; ++j) {
      if (Tab::B[j] != 0.0) {
        if (first) {
          acc = T(Tab::B[j]) * k[j][c];
          first = false;
        } else {
          acc = fmaT(T(Tab::B[j]), k[j][c], acc);
        }
      }
    }
    ynew[c] = fmaT(h, acc, y[c]);
  }
}

// First nonzero column of row i of A, of b and of the error weights
// (compile-time).
template <class Tab>
__host__ __device__ constexpr int first_a(int i) {
  for (int j = 0; j < i; ++j)
    if (Tab::A[i][j] != 0.0) return j;
  return -1;
}
template <class Tab>
__host__ __device__ constexpr int first_b() {
  for (int j = 0; j < Tab::S; ++j)
    if (Tab::B[j] != 0.0) return j;
  return -1;
}
template <class Tab>
__host__ __device__ constexpr int first_ew() {
  for (int j = 0; j < Tab::S; ++j)
    if (Tab::EW[j] != 0.0) return j;
  return -1;
}

// Stages 1..NST-1 of one explicit step from y with k_0 given, evaluated in
// "push" order: as soon as a stage value k_l exists it is folded into every
// later running sum (stage inputs, the update, the error estimate), so only
// the running sums stay live.  Each sum still receives its terms in index
// order, as acc = c_0 k_0, then fma(c_l, k_l, acc) -- the same operations as
// forming each sum at once.  Outputs: Y[i] (if KEEP_Y), the last stage input
// and value, the update y + h sum_j b_j k_j (if WANT_B) and the double-precision
// sum sum_j ew_j k_j (if WANT_E).
template <class Sys, class Tab, class T, int NST, bool KEEP_Y, bool WANT_B, bool WANT_E>
__device__ __forceinline__ void step_push(const T* y, const T* k0, const T* p, T h,
                                          T (&Y)[NST][Sys::D], T* ylast, T* klast,
                                          T* yn, double* e) {
  constexpr int D = Sys::D;
  T Z[NST][D];
  T Zb[D];
  T kc[D], Yl[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    kc[c] = k0[c];
    Yl[c] = y[c];
    if (KEEP_Y) Y[0][c] = y[c];
  }
#pragma unroll
  for (int l = 0; l < NST; ++l) {
    if (l > 0) {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        Yl[c] = hfma(h, Z[l][c], y[c]);
        if (KEEP_Y) Y[l][c] = Yl[c];
      }
      Sys::rhs(Yl, p, kc);
    }
#pragma unroll
    for (int j = l + 1; j < NST; ++j) {
      if (Tab::A[j][l] != 0.0) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
          if (first_a<Tab>(j) == l)
            Z[j][c] = cmul(Tab::A[j][l], kc[c]);
          else
            Z[j][c] = cfma(Tab::A[j][l], kc[c], Z[j][c]);
        }
      }
    }
    if (WANT_B && Tab::B[l] != 0.0) {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        if (first_b<Tab>() == l)
          Zb[c] = cmul(Tab::B[l], kc[c]);
        else
          Zb[c] = cfma(Tab::B[l], kc[c], Zb[c]);
      }
    }
    if constexpr (WANT_E) {
      if (Tab::EW[l] != 0.0) {
#pragma unroll
        for (int c = 0; c < D; ++c) {
          if (first_ew<Tab>() == l)
            e[c] = Tab::EW[l] * (double)kc[c];
          else
            e[c] = fmaT(Tab::EW[l], (double)kc[c], e[c]);
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) {
    ylast[c] = Yl[c];
    klast[c] = kc[c];
    if (WANT_B) yn[c] = hfma(h, Zb[c], y[c]);
  }
}

// Scaled RMS norm sqrt(mean (v_c / sc_c)^2) with squares summed by fma (the
// starting step's norm).
template <int D>
__device__ __forceinline__ double rms(const double* v, const double* sc) {
  double r = v[0] / sc[0];
  double ss = r * r;
#pragma unroll
  for (int c = 1; c < D; ++c) {
    r = v[c] / sc[c];
    ss = fmaT(r, r, ss);
  }
  return sqrt(ss * (1.0 / (double)D));
}

// ---------------------------------------------------- trial-step control --
// The acceptance test and the controller of the adaptive loop (Section 2.1)
// work on the mean square ms = err^2 of the scaled error: err <= 1 is
// ms <= 1, and the proposed factor 0.9 err^(-1/k) is 0.9 ms^(-1/(2k)).  No
// square root, no division: each scale's reciprocal is the hardware
// estimate refined by one Newton step (which squares its relative error),
// and the power a single-precision estimate refined by one Newton step in
// double; both land within about 1e-13 of the exact values.  That is far below the
// rounding noise of the error estimate itself (a small difference of large
// stage terms, near 1e-10 relative at rtol 1e-6), which sets how far two
// correct adaptive meshes of the same trajectory may differ; the mesh is
// recorded as taken, and the gradient is exact for it.

// 1/x for x > 0 finite: e = 1 - x r, r <- r + r e, once (relative error
// about the square of the estimate's).
__device__ __forceinline__ double recip(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fmaT(-x, r, 1.0);
  return fmaT(r, e, r);
}

// mean_c (v_c / sc_c)^2, the squares summed by fma in index order
template <int D>
__device__ __forceinline__ double mean_sq(const double* v, const double* sc) {
  double ss = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double r = v[c] * recip(sc[c]);
    ss = c == 0 ? r * r : fmaT(r, r, ss);
  }
  return ss * (1.0 / (double)D);
}

// Mean square of the error estimate e = h * esum against atol + rtol
// max(|y|, |y_new|).
template <class T, int D>
__device__ __forceinline__ double err_ms_sum(const T* y, const T* ynew, double h,
                                             const double* esum, double rtol, double atol) {
  double e[D], sc[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    e[c] = h * esum[c];
    sc[c] = fmaT(rtol, fmax(fabs((double)y[c]), fabs((double)ynew[c])), atol);
  }
  return mean_sq<D>(e, sc);
}

// y^K by repeated squaring (compile-time K >= 1)
template <int K>
__device__ __forceinline__ double ipow(double y) {
  if constexpr (K == 1) {
    return y;
  } else if constexpr (K % 2 == 0) {
    const double h = ipow<K / 2>(y);
    return h * h;
  } else {
    return ipow<K - 1>(y) * y;
  }
}

// The proposed step factor 0.9 ms^(-1/K2), K2 = 2 (q + 1) for an embedded
// order q.  ms is held to [1e-30, 1e30] first: the factor is clamped to
// [0.2, 10] long before either end (with K2 >= 6 the ends give factors
// beyond 90 and below 0.01).  A NaN ms gives 0, so that a trial whose
// error is not a number shrinks h by the lower bound.  The seed
// 2^(-log2(x) / K2) in single precision is within a few 1e-7; one Newton
// step y <- y + (y / K2)(1 - x y^K2) takes it to about 1e-13.
template <int K2>
__device__ __forceinline__ double step_factor(double ms) {
  const double x = fmin(fmax(ms, 1e-30), 1e30);
  const float l2 = __builtin_amdgcn_logf((float)x);
  const double y = (double)__builtin_amdgcn_exp2f(l2 * (-1.0f / (float)K2));
  constexpr double inv_k = 1.0 / (double)K2;
  const double t = fmaT(-x, ipow<K2>(y), 1.0);
  const double yr = fmaT(y * inv_k, t, y);
  return ms >= 0.0 ? 0.9 * yr : 0.0;
}

// x^(-1/K) for the controller and the starting step (K = 3..8), from
// operations that are exactly or correctly rounded on the device and on any
// IEEE host: x = m 2^e (m in [0.5, 1)), e = K q + j, a linear first guess
// for m^(-1/K) times 2^(-j/K) 2^(-q), then four Newton steps
// y <- y + (y / K)(1 - x y^K) on y^(-K) = x.  No division; deterministic to
// the bit.  Arguments below 1e-300 are raised to it.
template <int K>
struct TwoNeg;
template <>
struct TwoNeg<3> {
  static constexpr double c[3] = {1.0, 0.7937005259840998, 0.6299605249474366};
};
template <>
struct TwoNeg<4> {
  static constexpr double c[4] = {1.0, 0.8408964152537145, 0.7071067811865476,
                                  0.5946035575013605};
};
template <>
struct TwoNeg<5> {
  static constexpr double c[5] = {1.0, 0.8705505632961241, 0.757858283255199,
                                  0.6597539553864471, 0.5743491774985175};
};
template <>
struct TwoNeg<6> {
  static constexpr double c[6] = {1.0, 0.8908987181403393, 0.7937005259840998,
                                  0.7071067811865476, 0.6299605249474366,
                                  0.5612310241546865};
};
template <>
struct TwoNeg<7> {
  static constexpr double c[7] = {1.0, 0.9057236642639067, 0.820335356007638,
                                  0.7429971445684742, 0.6729500963161781,
                                  0.6095068271022377, 0.5520447568369061};
};
template <>
struct TwoNeg<8> {
  static constexpr double c[8] = {1.0, 0.9170040432046712, 0.8408964152537145,
                                  0.7711054127039704, 0.7071067811865476,
                                  0.6484197773255048, 0.5946035575013605,
                                  0.5452538663326288};
};

template <int K>
__device__ __forceinline__ double root_inv(double x) {
  if (isnan(x) || x < 0.0) return NAN;
  if (isinf(x)) return 0.0;
  constexpr double u = 2.0 * TwoNeg<K>::c[K - 1];  // 2^(1/K)
  constexpr double inv_k = 1.0 / (double)K;
  x = fmax(x, 1e-300);
  int e;
  const double m = frexp(x, &e);
  const int q = e >= 0 ? e / K : -((-e + K - 1) / K);
  const int j = e - q * K;
  double cj = 1.0;
#pragma unroll
  for (int i = 0; i < K; ++i) cj = (i == j) ? TwoNeg<K>::c[i] : cj;
  const double g = fmaT(-2.0 * (u - 1.0), m - 0.5, u);
  double y = ldexp(cj * g, -q);
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    double pw = y;
#pragma unroll
    for (int i = 1; i < K; ++i) pw = pw * y;
    const double t = fmaT(-x, pw, 1.0);
    y = fmaT(y * inv_k, t, y);
  }
  return y;
}

// Starting step of Hairer, Norsett & Wanner (Solving ODEs I, Sec. II.4).
template <class Sys, class Tab, class T>
__device__ double initial_step(const T* y0, const T* p, const T* f0, double t0,
                               double t1, double rtol, double atol) {
  constexpr int D = Sys::D;
  double sc[D], v[D];
#pragma unroll
  for (int c = 0; c < D; ++c) sc[c] = fmaT(rtol, fabs((double)y0[c]), atol);
#pragma unroll
  for (int c = 0; c < D; ++c) v[c] = (double)y0[c];
  const double d0 = rms<D>(v, sc);
#pragma unroll
  for (int c = 0; c < D; ++c) v[c] = (double)f0[c];
  const double d1 = rms<D>(v, sc);
  double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * (d0 / d1);
  h0 = fmin(h0, t1 - t0);
  T y1[D], f1[D];
#pragma unroll
  for (int c = 0; c < D; ++c) y1[c] = fmaT(T(h0), f0[c], y0[c]);
  Sys::rhs(y1, p, f1);
#pragma unroll
  for (int c = 0; c < D; ++c) v[c] = (double)(f1[c] - f0[c]);
  const double d2 = rms<D>(v, sc) / h0;
  const double dm = fmax(d1, d2);
  const double h1 = (dm <= 1e-15) ? fmax(1e-6, h0 * 1e-3)
                                  : root_inv<Tab::ORDER + 1>(dm * 100.0);
  return fmin(fmin(100.0 * h0, h1), t1 - t0);
}

template <class T, int NP>
__device__ __forceinline__ void load_params(const IvpArgs& a, int64_t tr, T* p) {
  const T* P = (const T*)a.params;
#pragma unroll
  for (int c = 0; c < NP; ++c) p[c] = a.params_shared ? P[c] : P[c * a.n + tr];
}

// One taped step: h then the state, moved as 16-byte chunks (the record
// size is a multiple of 16 and every record starts 16-byte aligned).
template <class T, int D>
struct alignas(16) RecBuf {
  double h;
  T y[D];
};

template <class T, int D>
__device__ __forceinline__ void store_rec(char* rp, double h, const T* y) {
  constexpr int RB = TapeRec<T, D>::BYTES;
  static_assert(sizeof(RecBuf<T, D>) == RB, "record layout");
  RecBuf<T, D> b;
  b.h = h;
#pragma unroll
  for (int c = 0; c < D; ++c) b.y[c] = y[c];
  const uint4* src = reinterpret_cast<const uint4*>(&b);
  uint4* dst = reinterpret_cast<uint4*>(__builtin_assume_aligned(rp, 16));
#pragma unroll
  for (int q = 0; q < RB / 16; ++q) dst[q] = src[q];
}

// Bytes of a checkpoint state (padded to 16).
template <class T, int D>
struct StateBytes {
  static constexpr int BYTES = (D * (int)sizeof(T) + 15) / 16 * 16;
};

template <class T, int D>
struct alignas(16) StateBuf {
  T y[D];
};

template <class T, int D>
__device__ __forceinline__ void store_state(char* rp, const T* y) {
  StateBuf<T, D> b;
#pragma unroll
  for (int c = 0; c < D; ++c) b.y[c] = y[c];
  const uint4* src = reinterpret_cast<const uint4*>(&b);
  uint4* dst = reinterpret_cast<uint4*>(__builtin_assume_aligned(rp, 16));
#pragma unroll
  for (int q = 0; q < (int)sizeof(b) / 16; ++q) dst[q] = src[q];
}

template <class T, int D>
__device__ __forceinline__ void load_state(const char* rp, T* y) {
  StateBuf<T, D> b;
  uint4* dst = reinterpret_cast<uint4*>(&b);
  const uint4* src = reinterpret_cast<const uint4*>(__builtin_assume_aligned(rp, 16));
#pragma unroll
  for (int q = 0; q < (int)sizeof(b) / 16; ++q) dst[q] = src[q];
#pragma unroll
  for (int c = 0; c < D; ++c) y[c] = b.y[c];
}

constexpr int H_GROUP = 16;  // step sizes staged per lane (checkpointed tape)
static_assert((H_GROUP & (H_GROUP - 1)) == 0, "a power of two (slot & (H_GROUP - 1))");

// Write this lane's first `count` staged step sizes to hp (contiguous).
__device__ __forceinline__ void flush_h(const double* s_h, int count, char* hp) {
  double2* dst = reinterpret_cast<double2*>(__builtin_assume_aligned(hp, 16));
  int q = 0;
  for (; q + 1 < count; q += 2)
    dst[q / 2] = make_double2(s_h[q * 256 + threadIdx.x], s_h[(q + 1) * 256 + threadIdx.x]);
  if (q < count) reinterpret_cast<double*>(hp)[q] = s_h[q * 256 + threadIdx.x];
}

constexpr int TAPE_GROUP = 4;  // step records per lane written together
static_assert((TAPE_GROUP & (TAPE_GROUP - 1)) == 0, "a power of two (slot & (TAPE_GROUP - 1))");

// Put one record into this lane's staging slots starting at chunk q0.
template <class T, int D>
__device__ __forceinline__ void stage_rec(uint4* stage, int q0, double h, const T* y) {
  constexpr int CH = TapeRec<T, D>::BYTES / 16;
  RecBuf<T, D> b;
  b.h = h;
#pragma unroll
  for (int c = 0; c < D; ++c) b.y[c] = y[c];
  const uint4* src = reinterpret_cast<const uint4*>(&b);
#pragma unroll
  for (int q = 0; q < CH; ++q) stage[(q0 + q) * 256 + threadIdx.x] = src[q];
}

// Write this lane's first `count` staged records to rp (contiguous).
template <class T, int D>
__device__ __forceinline__ void flush_recs(const uint4* stage, int count, char* rp) {
  constexpr int CH = TapeRec<T, D>::BYTES / 16;
  uint4* dst = reinterpret_cast<uint4*>(__builtin_assume_aligned(rp, 16));
  for (int q = 0; q < count * CH; ++q) dst[q] = stage[q * 256 + threadIdx.x];
}

// Wave-cooperative tape writes (full-tape records of the explicit pairs).
// Every record of a group waits in LDS; chunk c of lane l sits at
// c * 256 + (l ^ (c & 7)), so that the eight chunks of one lane, read by
// eight neighbouring lanes, fall in distinct 16-byte bank groups.  At the end
// of each loop iteration the groups that the wavefront's lanes completed are
// written out together: each group (TAPE_GROUP * CH chunks, one whole cache
// line for 32-byte records) by as many consecutive lanes, so that one store
// instruction writes whole lines, where a lane writing its own group issues
// TAPE_GROUP * CH stores that each touch one line per active lane.
template <class T, int D>
__device__ __forceinline__ void stage_rec_sw(uint4* stage, int q0, double h, const T* y) {
  constexpr int CH = TapeRec<T, D>::BYTES / 16;
  RecBuf<T, D> b;
  b.h = h;
#pragma unroll
  for (int c = 0; c < D; ++c) b.y[c] = y[c];
  const uint4* src = reinterpret_cast<const uint4*>(&b);
  const int l = (int)threadIdx.x;
#pragma unroll
  for (int q = 0; q < CH; ++q) {
    const int c = q0 + q;
    stage[c * 256 + (l ^ (c & 7))] = src[q];
  }
}

template <class T, int D>
__device__ __forceinline__ void flush_recs_sw(const uint4* stage, int count, char* rp) {
  constexpr int CH = TapeRec<T, D>::BYTES / 16;
  uint4* dst = reinterpret_cast<uint4*>(__builtin_assume_aligned(rp, 16));
  const int l = (int)threadIdx.x;
  for (int c = 0; c < count * CH; ++c) dst[c] = stage[c * 256 + (l ^ (c & 7))];
}

typedef unsigned int U32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) U32x4 GlobalU32x4;

// The lanes' parts in flush_groups_wave, fixed for a wavefront whose lanes
// all run the loop: with `per` groups written per store instruction, lane
// rank r among the live lanes writes chunk c = r mod G of the (r / G)-th
// group of a round (G chunks a group); lanes past per * G only wait.
struct WaveFlush {
  int per;      // groups per round (0: each lane writes its own)
  bool helper;  // r < per * G
  int gj;       // r / G: this lane's group in a round
  int qi;       // its queue entry in the first round: wavefront base + gj
  int c;        // r mod G: its chunk
};

template <class T, int D>
__device__ __forceinline__ WaveFlush wave_flush_parts() {
  constexpr int G = TAPE_GROUP * (TapeRec<T, D>::BYTES / 16);
  const uint64_t live = __ballot(1);
  const int r = rank_below(live);
  WaveFlush f;
  f.per = __popcll(live) / G;
  f.helper = r < f.per * G;
  f.gj = r / G;
  f.qi = ((int)threadIdx.x & ~63) + f.gj;
  f.c = r % G;
  return f;
}

// Called by every lane of the wavefront that has not returned (the lanes of
// `f`); `gp` is the address of the lane's completed group or null, and is
// cleared.  `queue` holds 64 16-byte entries per wavefront: (address, thread)
// of each completed group in lane order.
template <class T, int D>
__device__ __forceinline__ void flush_groups_wave(const uint4* stage, uint4* queue,
                                                  const WaveFlush& f, char*& gp) {
  const uint64_t need = __ballot(gp != nullptr);
  if (need == 0) return;
  if (f.per == 0) {
    if (gp != nullptr) flush_recs_sw<T, D>(stage, TAPE_GROUP, gp);
    gp = nullptr;
    return;
  }
  const int cnt = __popcll(need);
  if (gp != nullptr) {
    const uint64_t ad = (uint64_t)gp;
    queue[((int)threadIdx.x & ~63) + rank_below(need)] =
        make_uint4((uint32_t)ad, (uint32_t)(ad >> 32), threadIdx.x, 0u);
  }
  // the entries, and the staged records, were written by other lanes of
  // this wavefront; a wavefront's LDS accesses complete in order
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int c = f.c;
  for (int b = 0; b < cnt; b += f.per) {
    if (f.helper && b + f.gj < cnt) {
      const uint4 e = queue[f.qi + b];
      // a global-memory pointer: a generic (flat) store would also count
      // against the LDS wait of the next round's reads
      GlobalU32x4* dst = (GlobalU32x4*)(((uint64_t)e.y << 32) | (uint64_t)e.x);
      const uint4 v = stage[c * 256 + ((int)e.z ^ (c & 7))];
      dst[c] = U32x4{v.x, v.y, v.z, v.w};
    }
  }
  gp = nullptr;
}

template <class T, int D>
__device__ __forceinline__ void load_rec(const char* rp, double& h, T* y) {
  constexpr int RB = TapeRec<T, D>::BYTES;
  RecBuf<T, D> b;
  uint4* dst = reinterpret_cast<uint4*>(&b);
  const uint4* src = reinterpret_cast<const uint4*>(__builtin_assume_aligned(rp, 16));
#pragma unroll
  for (int q = 0; q < RB / 16; ++q) dst[q] = src[q];
  h = b.h;
#pragma unroll
  for (int c = 0; c < D; ++c) y[c] = b.y[c];
}

// ------------------------------------------------------------ dense output --
// The continuous extension of an accepted step (the dense output of Section
// 3.2): the cubic Hermite interpolant of the step's end states y0, y1 and
// slopes f0 = f(y0), f1 = f(y1), at offset theta = dt / h,
//   y(theta) = a0 y0 + a1 y1 + h (c0 f0 + c1 f1),
//   a0 = (1 - theta)^2 (1 + 2 theta), a1 = theta^2 (3 - 2 theta),
//   c0 = theta (1 - theta)^2,         c1 = -theta^2 (1 - theta).
struct HermiteW {
  double a0, a1, c0, c1;
};
__device__ __forceinline__ HermiteW hermite_weights(double theta) {
  const double u = 1.0 - theta;
  return HermiteW{u * u * fmaT(2.0, theta, 1.0), theta * theta * fmaT(-2.0, theta, 3.0),
                  theta * u * u, -(theta * theta) * u};
}

template <class T, int D>
__device__ __forceinline__ void hermite_state(const T* y0, const T* y1, const T* f0,
                                              const T* f1, double h, double dt, T* out) {
  const HermiteW w = hermite_weights(dt / h);
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const T slope = fmaT(T(w.c1), f1[c], T(w.c0) * f0[c]);
    out[c] = fmaT(T(h), slope, fmaT(T(w.a1), y1[c], T(w.a0) * y0[c]));
  }
}

// ------------------------------------------------------- forward / record --
// MODE_SOLVE: adaptive solve, no tape.  MODE_RECORD: adaptive solve writing
// the tape.  MODE_FROZEN: steps taken from a given mesh, writing the tape.
// MODE_REFRESH: the mesh-drift policy -- the given (old) mesh's steps are
// taken while their error estimates stay <= slack; the first that fails is
// a rejected trial, and the lane goes on adaptively from there.
//
// CKPT (checkpointed tape): a page covers R.page_steps accepted steps and
// holds the state before its first step followed by the step sizes only.
//
// DEFER (MODE_RECORD with the full tape): the loop takes no save-time side
// steps.  It notes, for each save time inside an accepted step, the step's
// index and the offset from its start, and erk_saves_kernel then forms the
// save states from the taped base states, all (trajectory, save) pairs in
// parallel with the same step map: the same values, and a loop with fewer
// iterations and less state.
//
// DENSE (dense output): no side steps either.  A record notes, for each save
// time inside an accepted step, both end states of the step (save_base and
// save_base_hi), its size (save_h) and the save's offset; dense_saves_kernel
// then forms the states from the step's continuous extension, and the sweep
// reads the same notes.  The solve, which keeps nothing, takes the extension
// at once in the loop.
template <class Sys, class Tab, class T, int MODE, bool CKPT, bool DEFER = false,
          bool DENSE = false>
__device__ __forceinline__ void erk_forward_body(const FwdArgs& a, int64_t block) {
  static_assert(!DEFER || (MODE == MODE_RECORD && !CKPT),
                "save steps are deferred only from a full-tape record");
  static_assert(!(DEFER && DENSE), "a dense record forms its save states in the loop");
  constexpr int D = Sys::D, NP = Sys::NP;
  constexpr int RB = TapeRec<T, D>::BYTES;
  constexpr int YB = StateBytes<T, D>::BYTES;
  const int K = CKPT ? a.rec.page_steps : PAGE_STEPS;
  const int64_t n = a.ivp.n;
  const int64_t tr = block * blockDim.x + threadIdx.x;
  // save times in LDS (lane-varying index, short latency); slot n_save holds
  // +inf so that "no save left" needs no branch
  __shared__ double s_times[65];
  // Tape staging.  COOP (full-tape records of the explicit pairs): every
  // record of a group waits here, and the wavefront writes the completed
  // groups together (flush_groups_wave).  Otherwise each lane collects the
  // first GROUP - 1 step records of a group here and writes them, together
  // with the last one straight from registers, as one whole cache line; the
  // Rosenbrock records and the given-mesh modes keep that (their loops hold
  // more state, and the cooperative writes measured slower there).
  // Chunk-major layouts (chunk, lane) keep the 16-byte LDS accesses free of
  // bank conflicts.
  constexpr int CH = TapeRec<T, D>::BYTES / 16;
  constexpr bool COOP = MODE == MODE_RECORD && !CKPT && !Tab::ROS;
  __shared__ uint4 s_tape[(MODE == MODE_SOLVE || CKPT) ? 1
                                                    : (TAPE_GROUP - (COOP ? 0 : 1)) * CH * 256];
  __shared__ uint4 s_wq[COOP ? 256 : 1];
  char* flush_gp = nullptr;  // COOP: this lane's group completed in this iteration
  // checkpointed tape: step sizes staged H_GROUP at a time (one 128-byte line)
  __shared__ double s_h[CKPT ? H_GROUP * 256 : 1];
  if (threadIdx.x < 65)
    s_times[threadIdx.x] = (int)threadIdx.x < a.ivp.n_save ? save_time_at(a.ivp.st, threadIdx.x)
                                                          : INFINITY;
  __syncthreads();
  if (tr >= n) return;
  const double t0 = a.ivp.t0, t1 = a.ivp.t1;
  const double rtol = a.ivp.rtol, atol = a.ivp.atol;
  const int ns = a.ivp.n_save;
  T* ysv = (T*)a.y_save;
  const RecView& R = a.rec;

  T y[D], p[NP], k1[D];
#pragma unroll
  for (int c = 0; c < D; ++c) y[c] = ((const T*)a.ivp.y0)[c * n + tr];
  load_params<T, NP>(a.ivp, tr, p);
  Sys::rhs(y, p, k1);
  int32_t status = LANE_OK;
#pragma unroll
  for (int c = 0; c < D; ++c)
    if (!isfinite(y[c]) || !isfinite(k1[c])) status = LANE_NONFINITE;

  double t = t0, h = 0.0;
  int32_t S_mesh = 0;
  if constexpr (MODE == MODE_FROZEN || MODE == MODE_REFRESH) {
    S_mesh = a.mesh_S[tr];
    // a step count the rectangle cannot hold is refused for this lane
    if (S_mesh < 0 || (int64_t)S_mesh > a.cap) {
      S_mesh = 0;
      status = LANE_MAX_STEPS;
    }
  }
  if constexpr (MODE != MODE_FROZEN) {
    if (status == LANE_OK)
      h = a.ivp.h0 > 0.0 ? fmin(a.ivp.h0, t1 - t0)
                         : initial_step<Sys, Tab, T>(y, p, k1, t0, t1, rtol, atol);
  }
  // MODE_REFRESH: still on the old mesh; old steps kept so far.  An old step
  // is kept while its RMS error is <= slack, i.e. its mean square <= slack^2.
  bool following = (MODE == MODE_REFRESH) && S_mesh > 0;
  const double slack2 = a.slack * a.slack;
  int32_t kept = S_mesh;
  // Given mesh: the size of the next mesh step is loaded one step ahead, so
  // the load's latency is hidden behind a whole step's arithmetic.
  double h_next = 0.0;
  if constexpr (MODE == MODE_FROZEN || MODE == MODE_REFRESH) {
    if (S_mesh > 0) h_next = a.mesh_h[tr];
  }

  // Side steps of the save times.  After a step is accepted whose interval
  // holds save times, the new state is held back (yn, kn at tn) and the
  // following iterations take the side steps from the unchanged base (y, k1
  // at t); the last one commits the new state.  So every evaluation starts
  // from (y, k1), with no per-iteration select between two bases.
  T yn[D], kn[D];
  double tn = t0;
  if constexpr (MODE != MODE_SOLVE) R.first_page[tr] = -1;
  int next_save = 0;
  // running pointers to this lane's next save-state slots
  T* ys_out = ysv + tr;
  // the base state of the save at ys_out, into the record's save_base.  The
  // given-mesh modes on a full tape leave it to a kernel that copies the
  // states from the tape afterwards: their loops load a step size per step,
  // and those loads would wait behind these stores.
  auto put_base = [&](const T* yb, bool valid) {
    if constexpr (MODE == MODE_RECORD || (CKPT && MODE != MODE_SOLVE) ||
                  (DENSE && MODE != MODE_SOLVE)) {
      T* sb = (T*)R.save_base + (ys_out - ysv);
#pragma unroll
      for (int c = 0; c < D; ++c) sb[c * n] = valid ? yb[c] : T(NAN);
    }
  };
  // dense output: the step's end state and its size, beside the base state
  auto put_dense = [&](const T* y1, double hstep) {
    if constexpr (DENSE && MODE != MODE_SOLVE) {
      T* sb = (T*)R.save_base_hi + (ys_out - ysv);
#pragma unroll
      for (int c = 0; c < D; ++c) sb[c * n] = y1[c];
      R.save_h[(int64_t)next_save * n + tr] = hstep;
    }
  };
  int32_t* sidx_out = R.save_idx + tr;
  double* sdt_out = R.save_dt + tr;
  const int64_t ys_stride = (int64_t)D * n;
  double ts = s_times[0];
  bool side = false;
  int32_t S = 0, trials = 0;
  bool prev_rej = false;
  int32_t page = -1;
  char* pg = nullptr;
  int slot = 0, kpage = 0;  // position of the next taped step: S = K kpage + slot
  // the trial budget as a 32-bit count (trials never exceed it)
  const int32_t max_trials =
      a.ivp.max_steps < 0x7fffffff ? (int32_t)a.ivp.max_steps : 0x7fffffff;

  // one iteration of a lane's loop (a `return` ends the iteration)
  auto live = [&]() {
    return status == LANE_OK && (side || (MODE == MODE_FROZEN ? (S < S_mesh) : (t < t1)));
  };
  auto iteration = [&]() {
    double hh;
    bool last = false;
    if (!side) {
      if constexpr (MODE == MODE_FROZEN) {
        hh = h_next;
        last = (S == S_mesh - 1);
        if (!last) h_next = a.mesh_h[(int64_t)(S + 1) * n + tr];
        ++trials;
      } else if constexpr (MODE == MODE_REFRESH) {
        if (trials >= max_trials) {
          status = LANE_MAX_STEPS;
          return;  // the lane's loop ends here
        }
        if (following) {  // the old mesh's step, its last one ending at t1
          h = h_next;
          last = (S == S_mesh - 1);
          if (!last) h_next = a.mesh_h[(int64_t)(S + 1) * n + tr];
        } else {
          if (h < 16.0 * EPS64 * fmax(fabs(t), 1.0)) {
            status = LANE_DT_UNDERFLOW;
            return;  // the lane's loop ends here
          }
          if (t + h >= t1) {
            h = t1 - t;
            last = true;
          }
        }
        ++trials;
        hh = h;
      } else {
        if (trials >= max_trials) {
          status = LANE_MAX_STEPS;
          return;  // the lane's loop ends here
        }
        if (h < 16.0 * EPS64 * fmax(fabs(t), 1.0)) {
          status = LANE_DT_UNDERFLOW;
          return;  // the lane's loop ends here
        }
        ++trials;
        if (t + h >= t1) {
          h = t1 - t;
          last = true;
        }
        hh = h;
      }
    } else {
      hh = ts - t;
    }

    // one evaluation of the step map from the base (y, k1); err is the mean
    // square of the scaled error estimate (the RMS norm squared)
    T ynew[D], klast[D];
    double err = 0.0;
    if constexpr (Tab::ROS) {
      // a side step onto the base point itself is the identity (1/(gamma h)
      // would divide by zero): evaluate at a harmless h and keep y
      const bool zero = (hh == 0.0);
      T W[D * D], u[Tab::S][D];
      int piv[D];
      // a replay on a given mesh forms only the stages that enter y_new
      ros_step<Sys, Tab, T, (MODE == MODE_FROZEN ? Tab::SU : Tab::S)>(
          y, p, T(zero ? 1.0 : hh), W, piv, u, ynew);
#pragma unroll
      for (int c = 0; c < D; ++c) ynew[c] = zero ? y[c] : ynew[c];
      if constexpr (MODE != MODE_FROZEN) {
        T e[D];
        ros_errvec<Tab, D, T>(u, e);
        err = ros_ms<D, T>(y, ynew, e, rtol, atol);
      }
    } else {
      T kb[D];
      if constexpr (Tab::FSAL) {
#pragma unroll
        for (int c = 0; c < D; ++c) kb[c] = k1[c];
      } else {
        Sys::rhs(y, p, kb);
      }
      T Yunused[Tab::S][D];
      T ylast[D];
      double esum[D];
      step_push<Sys, Tab, T, Tab::S, false, !Tab::FSAL, MODE != MODE_FROZEN>(
          y, kb, p, T(hh), Yunused, ylast, klast, ynew, esum);
      if constexpr (Tab::FSAL) {
#pragma unroll
        for (int c = 0; c < D; ++c) ynew[c] = ylast[c];
      }
      if constexpr (MODE != MODE_FROZEN) err = err_ms_sum<T, D>(y, ynew, hh, esum, rtol, atol);
    }

    if (side) {
#pragma unroll
      for (int c = 0; c < D; ++c) ys_out[c * n] = ynew[c];
      put_base(y, true);
      ys_out += ys_stride;
      if constexpr (MODE != MODE_SOLVE) {
        *sidx_out = S - 1;
        *sdt_out = hh;
        sidx_out += n;
        sdt_out += n;
      }
      ++next_save;
      ts = s_times[next_save];
      side = ts < tn;
      if (!side) {  // the last save of the interval: commit the new state
#pragma unroll
        for (int c = 0; c < D; ++c) {
          y[c] = yn[c];
          if constexpr (Tab::FSAL) k1[c] = kn[c];
        }
        t = tn;
      }
      return;
    }

    // proposed factor 0.9 err^(-1/(q+1)), formed once for both outcomes
    double fac0 = 0.0;
    if constexpr (MODE != MODE_FROZEN) fac0 = step_factor<2 * (Tab::QEMB + 1)>(err);
    if constexpr (MODE == MODE_REFRESH) {
      if (following && !(err <= slack2)) {  // the old mesh ends here: a rejected trial
        following = false;
        kept = S;
        h = hh * fmax(0.2, fac0);
        prev_rej = true;
        return;
      }
    }
    if (MODE == MODE_FROZEN || (MODE == MODE_REFRESH && following) || err <= 1.0) {
      if constexpr (MODE != MODE_SOLVE) {
        const bool need = (slot == 0);
        const bool over = need && (kpage >= R.static_pages);
        const uint64_t got = wave_bump(&R.counters[CNT_PAGES], over);
        if (need) {
          int32_t np_;
          if (!over) {
            np_ = (int32_t)(tr * R.static_pages + kpage);
          } else {
            if (got >= (uint64_t)(R.n_pages - R.n_static)) {
              status = LANE_NOSPACE;
              return;  // the lane's loop ends here
            }
            np_ = (int32_t)(R.n_static + (int64_t)got);
            const int64_t li = (int64_t)np_ - R.n_static;
            R.links[2 * li] = page;
            R.links[2 * li + 1] = -1;
            if (page >= R.n_static)
              R.links[2 * ((int64_t)page - R.n_static) + 1] = np_;
            else
              R.first_page[tr] = np_;
          }
          page = np_;
          pg = R.pages + (int64_t)page * R.page_bytes;
        }
        if constexpr (CKPT) {
          if (need) store_state<T, D>(pg, y);
          s_h[(slot & (H_GROUP - 1)) * 256 + threadIdx.x] = hh;
          if ((slot & (H_GROUP - 1)) == H_GROUP - 1)
            flush_h(s_h, H_GROUP, pg + YB + (slot - (H_GROUP - 1)) * 8);
        } else {
          if constexpr (COOP) {
            stage_rec_sw<T, D>(s_tape, (slot & (TAPE_GROUP - 1)) * CH, hh, y);
            if ((slot & (TAPE_GROUP - 1)) == TAPE_GROUP - 1)
              flush_gp = pg + (slot - (TAPE_GROUP - 1)) * RB;
          } else if ((slot & (TAPE_GROUP - 1)) == TAPE_GROUP - 1) {
            char* gp = pg + (slot - (TAPE_GROUP - 1)) * RB;
            flush_recs<T, D>(s_tape, TAPE_GROUP - 1, gp);
            store_rec<T, D>(gp + (TAPE_GROUP - 1) * RB, hh, y);
          } else {
            stage_rec<T, D>(s_tape, (slot & (TAPE_GROUP - 1)) * CH, hh, y);
          }
        }
        if (++slot == K) {
          slot = 0;
          ++kpage;
        }
      }
      ++S;
      const double tnew = last ? t1 : t + hh;
      if constexpr (MODE != MODE_FROZEN) {
        h = hh * fmax(0.2, fmin(prev_rej ? 1.0 : 10.0, fac0));
        prev_rej = false;
      }
      if constexpr (DENSE && MODE != MODE_SOLVE) {
        // saves inside this step: the step's end states, size and the save's
        // offset are noted, and dense_saves_kernel forms the states from
        // them afterwards, all (trajectory, save) pairs in parallel
        while (ts < tnew) {
          *sidx_out = S - 1;
          *sdt_out = ts - t;
          sidx_out += n;
          sdt_out += n;
          put_base(y, true);
          put_dense(ynew, hh);
          ys_out += ys_stride;
          ++next_save;
          ts = s_times[next_save];
        }
#pragma unroll
        for (int c = 0; c < D; ++c) {
          y[c] = ynew[c];
          if constexpr (Tab::FSAL) k1[c] = klast[c];
        }
        t = tnew;
      } else if constexpr (DENSE) {
        // the solve keeps nothing: saves inside this step take the step's
        // continuous extension at once
        if (ts < tnew) {
          T f0[D], f1[D], yd[D];
          if constexpr (Tab::FSAL) {
#pragma unroll
            for (int c = 0; c < D; ++c) {
              f0[c] = k1[c];
              f1[c] = klast[c];
            }
          } else {
            Sys::rhs(y, p, f0);
            Sys::rhs(ynew, p, f1);
          }
          while (ts < tnew) {
            hermite_state<T, D>(y, ynew, f0, f1, hh, ts - t, yd);
#pragma unroll
            for (int c = 0; c < D; ++c) ys_out[c * n] = yd[c];
            if constexpr (MODE != MODE_SOLVE) {
              *sidx_out = S - 1;
              *sdt_out = ts - t;
              sidx_out += n;
              sdt_out += n;
            }
            put_base(y, true);
            put_dense(ynew, hh);
            ys_out += ys_stride;
            ++next_save;
            ts = s_times[next_save];
          }
        }
#pragma unroll
        for (int c = 0; c < D; ++c) {
          y[c] = ynew[c];
          if constexpr (Tab::FSAL) k1[c] = klast[c];
        }
        t = tnew;
      } else if constexpr (DEFER) {
        // saves inside this step: base index S - 1 and offset from its start
        while (ts < tnew) {
          *sidx_out = S - 1;
          *sdt_out = ts - t;
          sidx_out += n;
          sdt_out += n;
          put_base(y, true);
          ys_out += ys_stride;
          ++next_save;
          ts = s_times[next_save];
        }
#pragma unroll
        for (int c = 0; c < D; ++c) {
          y[c] = ynew[c];
          if constexpr (Tab::FSAL) k1[c] = klast[c];
        }
        t = tnew;
      } else {
        side = ts < tnew;
        if (side) {
#pragma unroll
          for (int c = 0; c < D; ++c) {
            yn[c] = ynew[c];
            if constexpr (Tab::FSAL) kn[c] = klast[c];
          }
          tn = tnew;
        } else {
#pragma unroll
          for (int c = 0; c < D; ++c) {
            y[c] = ynew[c];
            if constexpr (Tab::FSAL) k1[c] = klast[c];
          }
          t = tnew;
        }
      }
    } else {
      h = hh * fmax(0.2, fac0);
      prev_rej = true;
    }
  };
  if constexpr (COOP) {
    // the loop runs while any lane of the wavefront is live: lanes that are
    // done stay to help write the groups
    const WaveFlush wf = wave_flush_parts<T, D>();
    for (;;) {
      const bool act = live();
      if (!__any(act)) break;
      if (act) iteration();
      flush_groups_wave<T, D>(s_tape, s_wq, wf, flush_gp);
    }
  } else {
    while (live()) iteration();
  }

  // records of an unfinished group (S = K kpage + slot; groups never
  // straddle a page because K is a multiple of the group size)
  if constexpr (MODE != MODE_SOLVE) {
    if constexpr (CKPT) {
      const int rem = S % H_GROUP;
      if (rem > 0 && pg != nullptr) flush_h(s_h, rem, pg + YB + (slot - rem) * 8);
    } else {
      const int rem = S % TAPE_GROUP;
      if constexpr (COOP) {
        if (rem > 0 && pg != nullptr) flush_recs_sw<T, D>(s_tape, rem, pg + (slot - rem) * RB);
      } else {
        if (rem > 0 && pg != nullptr) flush_recs<T, D>(s_tape, rem, pg + (slot - rem) * RB);
      }
    }
  }

  // saves at the last mesh point (t_s = t1): a side step of size zero
  const bool ok = (status == LANE_OK);
  for (; next_save < ns; ++next_save) {
#pragma unroll
    for (int c = 0; c < D; ++c) ys_out[c * n] = ok ? y[c] : T(NAN);
    put_base(y, ok);
    put_dense(y, 0.0);
    ys_out += ys_stride;
    if constexpr (MODE != MODE_SOLVE) {
      *sidx_out = ok ? S : -1;
      *sdt_out = ok ? s_times[next_save] - t : NAN;
      sidx_out += n;
      sdt_out += n;
    }
  }
  if constexpr (MODE != MODE_SOLVE) {
    R.steps[tr] = S;
    R.n_trial[tr] = trials;
    R.last_page[tr] = page;
    R.status[tr] = status;
#pragma unroll
    for (int c = 0; c < D; ++c) ((T*)R.y_final)[c * n + tr] = y[c];
  }
  if constexpr (MODE == MODE_REFRESH) {
    if (a.drift_at) a.drift_at[tr] = kept;
  }
  if (a.lane_status) a.lane_status[tr] = status;
}

// ------------------------------------------------------------ reverse sweep --
// Loss cotangent at one save state v, accumulating the lane's loss.
template <class T, int D>
__device__ __forceinline__ void save_cotangent(const AdjArgs& a, int s,
                                               int64_t tr, const T* v, T two_scale,
                                               T* w, double& loss) {
  const int64_t n = a.ivp.n;
  const T* data = (const T*)a.loss_data;
  if (a.loss_kind == LOSS_SUMSQ) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      w[c] = two_scale * v[c];
      loss = fmaT((double)v[c], (double)v[c], loss);
    }
  } else if (a.loss_kind == LOSS_MSE_TARGET) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const T r = v[c] - data[((int64_t)s * D + c) * n + tr];
      w[c] = two_scale * r;
      loss = fmaT((double)r, (double)r, loss);
    }
  } else {
#pragma unroll
    for (int c = 0; c < D; ++c) w[c] = data[((int64_t)s * D + c) * n + tr];
  }
}

// Reverse of one explicit step from stage states Y (recomputed by
// step_push) with output cotangent w: lin = d(y_new)/dy^T w and
// g += d(y_new)/dp^T w, stage by stage from the last:
//   kbar_j = h (b_j w + sum_{l>j} a_lj Ybar_l),  Ybar_j = f_y(Y_j)^T kbar_j,
//   g += f_p(Y_j)^T kbar_j,  lin = w + sum_j Ybar_j.
template <class Sys, class Tab, class T>
__device__ __forceinline__ void erk_step_vjp(const T (&Y)[Tab::SU][Sys::D], const T* p,
                                             double hh, const T* w, T* lin, T* g) {
  constexpr int D = Sys::D, SU = Tab::SU;
  T Yb[SU][D];
#pragma unroll
  for (int c = 0; c < D; ++c) lin[c] = w[c];
#pragma unroll
  for (int j = SU - 1; j >= 0; --j) {
    T kb[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T acc = T(0);
      bool first = true;
      if (Tab::B[j] != 0.0) {
        acc = T(Tab::B[j]) * w[c];
        first = false;
      }
#pragma unroll
      for (int l = j + 1; l < SU; ++l) {
        if (Tab::A[l][j] != 0.0) {
          if (first) {
            acc = T(Tab::A[l][j]) * Yb[l][c];
            first = false;
          } else {
            acc = fmaT(T(Tab::A[l][j]), Yb[l][c], acc);
          }
        }
      }
      kb[c] = T(hh) * acc;
    }
    Sys::vjp(Y[j], p, kb, Yb[j], g);
#pragma unroll
    for (int c = 0; c < D; ++c) lin[c] = lin[c] + Yb[j][c];
  }
}

// A save step of size hh != 0 from its base state yb: recompute it, form
// the save's cotangent from the state it reaches (cot(ys, w)), and reverse
// it: lin = d(ys)/dyb^T w, g += d(ys)/dp^T w.  Rosenbrock factors of d >= 6
// go through the lane's LDS slots sW, as in the sweep's loop.
template <class Sys, class Tab, class T, bool W_LDS, class Cot>
__device__ __forceinline__ void save_step_reverse(const T* yb, const T* p, double hh, T* sW,
                                                  Cot&& cot, T* lin, T* g) {
  constexpr int D = Sys::D;
  T ys[D], w[D];
  if constexpr (Tab::ROS) {
    T u[Tab::S][D];
    int piv[D];
    if constexpr (W_LDS) {
      ros_step_lds<Sys, Tab, T, Tab::SU>(yb, p, T(hh), LdsMat<Sys, T>{sW}, piv, u, ys);
    } else {
      T W[D * D];
      ros_step<Sys, Tab, T, Tab::SU>(yb, p, T(hh), W, piv, u, ys);
      cot(ys, w);
      ros_step_vjp<Sys, Tab, T, T[D * D]>(yb, p, T(hh), W, piv, u, w, lin, g);
      return;
    }
    cot(ys, w);
    T ybo[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      ybo[c] = yb[c];
      opaque(ybo[c]);
#pragma unroll
      for (int q = 0; q < Tab::SU; ++q) opaque(u[q][c]);
    }
    ros_step_vjp<Sys, Tab, T, LdsMat<Sys, T>>(ybo, p, T(hh), LdsMat<Sys, T>{sW}, piv, u, w, lin,
                                              g);
  } else {
    T k0[D], Y[Tab::SU][D], ylast[D], klast[D];
    Sys::rhs(yb, p, k0);
    step_push<Sys, Tab, T, Tab::SU, true, true, false>(yb, k0, p, T(hh), Y, ylast, klast, ys,
                                                       nullptr);
    cot(ys, w);
    erk_step_vjp<Sys, Tab, T>(Y, p, hh, w, lin, g);
  }
}

// The save steps of one trajectory's reverse sweep, from the last save to
// the first: each save's cotangent (from the state its side step reaches, or
// from its base state for a save on a mesh point), its loss term and the
// reverse of its side step from the recorded base state, with the parameter
// terms added into g.  The cotangent each save gives its base state goes to
// a.contrib.
template <class Sys, class Tab, class T, bool W_LDS>
__device__ __forceinline__ void save_steps_reverse(const AdjArgs& a, int64_t tr, const T* p,
                                                   T two_scale, T* sW, T* g, double& loss) {
  constexpr int D = Sys::D;
  const RecView& R = a.rec;
  const int64_t n = a.ivp.n;
  T* cb = (T*)a.contrib;
  const T* sbase = (const T*)R.save_base;
  for (int ss = R.n_save - 1; ss >= 0; --ss) {
    const double dt = R.save_dt[(int64_t)ss * n + tr];
    T yb[D], cs[D];
#pragma unroll
    for (int c = 0; c < D; ++c) yb[c] = sbase[((int64_t)ss * D + c) * n + tr];
    if (dt == 0.0) {
      save_cotangent<T, D>(a, ss, tr, yb, two_scale, cs, loss);
    } else {
      auto cot = [&](const T* ys, T* w) {
        save_cotangent<T, D>(a, ss, tr, ys, two_scale, w, loss);
      };
      save_step_reverse<Sys, Tab, T, W_LDS>(yb, p, dt, sW, cot, cs, g);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) cb[((int64_t)ss * D + c) * n + tr] = cs[c];
  }
}

// The dense saves of one trajectory's reverse sweep, from the last save to
// the first: each save's cotangent w (from its state, the continuous
// extension recomputed from the step's end states), its loss term, and the
// reverse of the extension.  With y(theta) = a0 y0 + a1 y1 + h (c0 f(y0) +
// c1 f(y1)), the end states receive a0 w + f_y(y0)^T (h c0 w) and
// a1 w + f_y(y1)^T (h c1 w), and g the parameter terms of both VJPs.  The
// saves of one step are summed (from the last), and the step's two sums
// become two events: (end point, sum for y1), then (start point, sum for
// y0); a save at the last mesh point gives w to y_S alone.  Events are
// written from the top slot of a.events / a.contrib down, so that their
// mesh points increase with the slot, as the save bookkeeping's do; unused
// slots carry point -1.  The sweep then takes them as it takes plain saves,
// so at a mesh point the sums of the step that starts there are added
// before those of the step that ends there.
template <class Sys, class T>
__device__ __forceinline__ void dense_saves_reverse(const AdjArgs& a, int64_t tr, const T* p,
                                                    T two_scale, T* g, double& loss) {
  constexpr int D = Sys::D;
  const RecView& R = a.rec;
  const int64_t n = a.ivp.n;
  T* cb = (T*)a.contrib;
  int32_t* ev = a.events;
  const T* b0 = (const T*)R.save_base;
  const T* b1 = (const T*)R.save_base_hi;
  int slot = 2 * R.n_save - 1;
  auto emit = [&](int32_t point, const T* v) {
    ev[(int64_t)slot * n + tr] = point;
#pragma unroll
    for (int c = 0; c < D; ++c) cb[((int64_t)slot * D + c) * n + tr] = v[c];
    --slot;
  };
  T acc_lo[D], acc_hi[D];
  int32_t gidx = -1;
  double gh = 0.0;
  for (int ss = R.n_save - 1; ss >= 0; --ss) {
    const int32_t idx = R.save_idx[(int64_t)ss * n + tr];
    const double dt = R.save_dt[(int64_t)ss * n + tr];
    const double hs = R.save_h[(int64_t)ss * n + tr];
    T y0[D], lo[D], hi[D];
#pragma unroll
    for (int c = 0; c < D; ++c) y0[c] = b0[((int64_t)ss * D + c) * n + tr];
    if (hs == 0.0) {  // at the last mesh point: the state itself
      save_cotangent<T, D>(a, ss, tr, y0, two_scale, lo, loss);
#pragma unroll
      for (int c = 0; c < D; ++c) hi[c] = T(0);
    } else {
      T y1[D], f0[D], f1[D], ys[D], w[D], v0[D], v1[D], g0[D], g1[D];
#pragma unroll
      for (int c = 0; c < D; ++c) y1[c] = b1[((int64_t)ss * D + c) * n + tr];
      Sys::rhs(y0, p, f0);
      Sys::rhs(y1, p, f1);
      hermite_state<T, D>(y0, y1, f0, f1, hs, dt, ys);
      save_cotangent<T, D>(a, ss, tr, ys, two_scale, w, loss);
      const HermiteW hw = hermite_weights(dt / hs);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        v0[c] = T(hs * hw.c0) * w[c];
        v1[c] = T(hs * hw.c1) * w[c];
      }
      Sys::vjp(y0, p, v0, g0, g);
      Sys::vjp(y1, p, v1, g1, g);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        lo[c] = fmaT(T(hw.a0), w[c], g0[c]);
        hi[c] = fmaT(T(hw.a1), w[c], g1[c]);
      }
    }
    if (gidx >= 0 && idx != gidx) {  // the previous step's saves are complete
      if (gh > 0.0) emit(gidx + 1, acc_hi);
      emit(gidx, acc_lo);
      gidx = -1;
    }
    if (gidx < 0) {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        acc_lo[c] = lo[c];
        acc_hi[c] = hi[c];
      }
      gidx = idx;
      gh = hs;
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        acc_lo[c] = acc_lo[c] + lo[c];
        acc_hi[c] = acc_hi[c] + hi[c];
      }
    }
  }
  if (gidx >= 0) {
    if (gh > 0.0) emit(gidx + 1, acc_hi);
    emit(gidx, acc_lo);
  }
  for (; slot >= 0; --slot) ev[(int64_t)slot * n + tr] = -1;
}

// Slot (trajectory offset in the block) this lane sweeps.  The block's 256
// lanes take its trajectories in increasing order of their step counts (ties
// by index; failed and absent ones first), so each wavefront gets sweeps of
// nearly equal length and few lanes idle while the longest one finishes.  A
// trajectory's results do not depend on the lane that computes it.
__device__ __forceinline__ int sweep_slot(const RecView& R, int64_t base, int64_t n) {
  __shared__ int4 s_key4[64];
  __shared__ int s_slot[256];
  int32_t* s_key = reinterpret_cast<int32_t*>(s_key4);
  const int me = threadIdx.x;
  const int64_t t = base + me;
  const int32_t key = (t < n && R.status[t] == LANE_OK) ? R.steps[t] : -1;
  s_key[me] = key;
  __syncthreads();
  int rank = 0;
  for (int j4 = 0; j4 < 64; ++j4) {
    const int4 v = s_key4[j4];
    const int j = 4 * j4;
    rank += (v.x < key || (v.x == key && j < me)) ? 1 : 0;
    rank += (v.y < key || (v.y == key && j + 1 < me)) ? 1 : 0;
    rank += (v.z < key || (v.z == key && j + 2 < me)) ? 1 : 0;
    rank += (v.w < key || (v.w == key && j + 3 < me)) ? 1 : 0;
  }
  s_slot[rank] = me;
  __syncthreads();
  return s_slot[me];
}

// CKPT: the tape holds one state per page (segment) and the step sizes; the
// sweep first replays each segment forward into this trajectory's scratch
// page (full step records, the same arithmetic as the record, so the same
// bits), then walks it backward.  Replay steps and reverse steps share one
// loop iteration so that lanes at different phases do not serialize, and the
// lanes of a wavefront are aligned by segment (first_gap below).
//
// DENSE: the saves come from the continuous extension of the step holding
// each one (dense_saves_reverse); each save's cotangent reaches both end
// states of its step, and the loop takes the resulting events (a mesh point
// and a cotangent each) as it takes plain saves.
template <class Sys, class Tab, class T, bool SHARED, bool CKPT, bool DENSE = false>
__device__ __forceinline__ void erk_adjoint_body(const AdjArgs& a, int64_t block) {
  constexpr int D = Sys::D, NP = Sys::NP, SU = Tab::SU;
  constexpr int RB = TapeRec<T, D>::BYTES;
  constexpr int YB = StateBytes<T, D>::BYTES;
  constexpr int CH = RB / 16;
  const int K = CKPT ? a.rec.page_steps : PAGE_STEPS;
  const int64_t n = a.ivp.n;
  const int64_t base = block * 256;  // blocks of 256 lanes
  const int slot_in_block = sweep_slot(a.rec, base, n);
  const int64_t tr = base + slot_in_block;
  const bool valid = tr < n;
  // tape lines staged through LDS for records of up to 32 bytes; larger
  // records (their systems run at one wave per SIMD) are read directly
  constexpr bool STAGE = CH <= 2;
  __shared__ uint4 s_rd[STAGE ? TAPE_GROUP * CH * 256 : 1];
  // Rosenbrock factors of d >= 6 held in LDS during the transposed solves
  // (their possible nonzeros, 52 doubles a lane for HIRES, would otherwise
  // push the reverse step past the register file into scratch); one wave
  // per SIMD either way
  constexpr bool W_LDS = Tab::ROS && D >= 6;
  __shared__ T s_W[W_LDS ? lu_nnz<Sys>() * 256 : 1];
  const RecView& R = a.rec;
  const bool ok = valid && R.status[tr] == LANE_OK;
  // CKPT: lanes of a wavefront aligned by segment.  A lane's first segment
  // (the last of its tape) holds r = (S - 1) mod K + 1 steps, its F others K
  // each.  Each lane waits first_gap = L - r trips before replaying its first
  // segment and as many again after reversing it; from then on all its
  // lanes replay their K-step segments in the same trips and reverse them in
  // the same trips, so a replay trip skips the reverse step's work for the
  // whole wavefront.  L = r_max, the wavefront's longest first segment, when
  // that adds no trips to the unaligned 2 S_max (2 (r_max + K F_max) =
  // 2 S_max: the step counts do not straddle a multiple of K); else L = K
  // when the 2 K (F_max + 1) trips that takes are at most a quarter more
  // (half of them replay trips); else the lanes are left unaligned.  (Every
  // lane of the wavefront is here.)
  int first_gap = 0;
  if constexpr (CKPT) {
    const int S0 = ok ? R.steps[tr] : 0;
    const int r = S0 > 0 ? (S0 - 1) % K + 1 : 0;
    const int r_max = wave_max(r);
    const int F_max = wave_max(S0 > 0 ? (S0 - r) / K : 0);
    const int S_max = wave_max(S0);
    if (r_max + K * F_max <= S_max)
      first_gap = r_max - r;
    else if (4 * (int64_t)K * (F_max + 1) <= 5 * (int64_t)S_max)
      first_gap = K - r;
  }
  T* gpo = (T*)a.grad_p;
  T* gyo = (T*)a.grad_y0;
  T lam[D], gp[NP];
#pragma unroll
  for (int c = 0; c < D; ++c) lam[c] = T(0);
#pragma unroll
  for (int c = 0; c < NP; ++c) gp[c] = T(0);
  double loss = 0.0;

  if (ok) {
  T p[NP];
  load_params<T, NP>(a.ivp, tr, p);
  const int32_t S = R.steps[tr];
  int32_t page = R.last_page[tr];
  const T two_scale = T(2.0 * a.scale);

  // The save steps first (save_steps_reverse); the cotangent each save
  // gives its base state is added when the loop below reaches that point.
  if constexpr (DENSE)
    dense_saves_reverse<Sys, T>(a, tr, p, two_scale, gp, loss);
  else
    save_steps_reverse<Sys, Tab, T, W_LDS>(a, tr, p, two_scale, s_W, gp, loss);

  // Save bookkeeping, walked from the last save to the first: the save's
  // base index and its cotangent in a.contrib.
  // (dense output: the events of dense_saves_reverse, in the same layout)
  int s = (DENSE ? 2 * R.n_save : R.n_save) - 1;
  const int32_t* sidx_p = (DENSE ? a.events : R.save_idx) + (int64_t)s * n + tr;
  const T* cb_p = (const T*)a.contrib + (int64_t)s * D * n + tr;
  int32_t sidx = *sidx_p;
  auto next_save = [&]() {
    --s;
    sidx_p -= n;
    cb_p -= D * n;
    if (s >= 0) sidx = *sidx_p;
  };

  // Tape position of the step record of mesh step i (h_i, y_{i-1}).
  int32_t i = S;
  int slot = S > 0 ? (S - 1) % K : 0;
  // Tape reads: the TAPE_GROUP records of a 128-byte line are loaded into
  // LDS together (chunk-major, as in the record) when the sweep enters the
  // line, so each line is fetched once although it serves TAPE_GROUP steps.
  int grp = -1;  // first slot of the staged group; -1: none

  // checkpointed tape: segment replay state
  char* scr = CKPT ? (char*)a.scratch + (int64_t)tr * K * RB : nullptr;
  bool rebuild = false;
  int j_rb = 0, seg_len = 0;
  T y_rb[D];
#pragma unroll
  for (int c = 0; c < D; ++c) y_rb[c] = T(0);
  // the next replay step's size, loaded one step ahead so that its latency
  // hides behind the current step
  double h_rb = 0.0;
  auto start_segment = [&](int len) {
    const char* pgp = R.pages + (int64_t)page * R.page_bytes;
    load_state<T, D>(pgp, y_rb);
    h_rb = ((const double*)(pgp + YB))[0];
    rebuild = true;
    j_rb = 0;
    seg_len = len;
    grp = -1;
  };
  if (CKPT && S > 0) start_segment(slot + 1);

  // the saves based at mesh point i, from the last: their cotangents into lam
  auto take_saves = [&]() {
    while (s >= 0 && sidx == i) {
#pragma unroll
      for (int c = 0; c < D; ++c) lam[c] = lam[c] + cb_p[c * n];
      next_save();
    }
  };
  // Where the loop takes them: on reaching a point, or at the end of the
  // reverse step that reaches it (the six-stage Rodas4).  The same additions
  // in the same order; only the register allocation differs, and measured
  // in opposite directions: at the end, the HIRES Rodas4 sweep spills
  // nothing instead of 92 B a lane and runs 4 % faster, while the FP64
  // Lorenz / Tsit5 sweep needs 146 VGPRs instead of 124 and the HIRES
  // Rosenbrock23 sweep runs 17 % slower.
  constexpr bool AT_END = Tab::ROS && Tab::SU >= 6;
  if constexpr (AT_END) take_saves();

  // CKPT: a wave-uniform loop (the wavefront leaves it when no lane is
  // live).  A lane replaying and a lane reversing then take one step each
  // per trip; with a per-lane loop the compiler made the replay a loop of its
  // own, and a lane reversing waited for every other lane's whole segment.
  bool live = true;
  int wait = first_gap;  // trips this lane idles before its next replay
  while (true) {
    if constexpr (CKPT) {
      if (!__any(live)) break;
      if (!live) continue;
      if (wait > 0) {
        --wait;
        continue;
      }
    }
    if constexpr (!AT_END) {
      if (!rebuild) {
        take_saves();
        if (i == 0) {
          if constexpr (CKPT) {
            live = false;
            continue;
          }
          break;
        }
      }
    } else {
      if (i == 0) {
        if constexpr (CKPT) {
          live = false;
          continue;
        }
        break;
      }
    }

    T yb[D];
    double hh;
    {
      if (CKPT && rebuild) {
        hh = h_rb;
        if (j_rb + 1 < seg_len)
          h_rb = ((const double*)(R.pages + (int64_t)page * R.page_bytes + YB))[j_rb + 1];
#pragma unroll
        for (int c = 0; c < D; ++c) yb[c] = y_rb[c];
      } else if constexpr (!STAGE) {
        load_rec<T, D>((CKPT ? scr : R.pages + (int64_t)page * R.page_bytes) + slot * RB, hh, yb);
      } else {
        const int g0 = slot & ~(TAPE_GROUP - 1);
        if (g0 != grp) {
          const char* base = CKPT ? scr : R.pages + (int64_t)page * R.page_bytes;
          const uint4* src = reinterpret_cast<const uint4*>(
              __builtin_assume_aligned(base + g0 * RB, 16));
#pragma unroll
          for (int q = 0; q < TAPE_GROUP * CH; ++q) s_rd[q * 256 + threadIdx.x] = src[q];
          grp = g0;
        }
        RecBuf<T, D> b;
        uint4* dst = reinterpret_cast<uint4*>(&b);
#pragma unroll
        for (int q = 0; q < CH; ++q) dst[q] = s_rd[((slot - g0) * CH + q) * 256 + threadIdx.x];
        hh = b.h;
#pragma unroll
        for (int c = 0; c < D; ++c) yb[c] = b.y[c];
      }
    }

    // recompute the stages of this step
    constexpr int NW = Tab::ROS ? D * D : 1;
    constexpr int NU = Tab::ROS ? Tab::S : 1;
    constexpr int NY = Tab::ROS ? 1 : SU;
    T W[NW], u[NU][D];
    int piv[D];
    T Y[NY][D], ys[D];
    if constexpr (W_LDS) {
      ros_step_lds<Sys, Tab, T, Tab::SU>(yb, p, T(hh), LdsMat<Sys, T>{s_W}, piv, u, ys);
    } else if constexpr (Tab::ROS) {
      ros_step<Sys, Tab, T, Tab::SU>(yb, p, T(hh), W, piv, u, ys);
    } else {
      T k0[D], ylast[D], klast[D];
      Sys::rhs(yb, p, k0);
      step_push<Sys, Tab, T, SU, true, true, false>(yb, k0, p, T(hh), Y, ylast, klast, ys,
                                                    nullptr);
    }
    if (CKPT && rebuild) {
      // one replay step of the segment: keep its record, move on.  Records
      // of up to 32 bytes wait in this lane's group slots (free while it
      // replays) and go out a whole group (one cache line) at a time; the
      // segment's last group stays there for the reverse steps that follow.
      if constexpr (STAGE) {
        const int q = j_rb & (TAPE_GROUP - 1);
        stage_rec<T, D>(s_rd, q * CH, hh, yb);
        if (q == TAPE_GROUP - 1 || j_rb + 1 == seg_len) {
          flush_recs<T, D>(s_rd, q + 1, scr + (j_rb - q) * RB);
          if (j_rb + 1 == seg_len) grp = j_rb - q;
        }
      } else {
        store_rec<T, D>(scr + j_rb * RB, hh, yb);
      }
#pragma unroll
      for (int c = 0; c < D; ++c) y_rb[c] = ys[c];
      if (++j_rb == seg_len) rebuild = false;
      continue;
    }
    T w[D];
#pragma unroll
    for (int c = 0; c < D; ++c) w[c] = lam[c];

    // reverse through the stages: kbar_j = h (b_j w + sum_{l>j} a_lj Ybar_l)
    T lin[D];
    if constexpr (W_LDS) {
      const LdsMat<Sys, T> Wl{s_W};
      // the reverse recomputes the stage states and Jacobian terms from
      // (y, u) rather than keeping the forward's copies live
#pragma unroll
      for (int c = 0; c < D; ++c) {
        opaque(yb[c]);
#pragma unroll
        for (int q = 0; q < (Tab::ROS ? Tab::SU : 0); ++q) opaque(u[q][c]);
      }
      ros_step_vjp<Sys, Tab, T, LdsMat<Sys, T>>(yb, p, T(hh), Wl, piv, u, w, lin, gp);
    } else if constexpr (Tab::ROS) {
      ros_step_vjp<Sys, Tab, T, T[NW]>(yb, p, T(hh), W, piv, u, w, lin, gp);
    } else {
      erk_step_vjp<Sys, Tab, T>(Y, p, hh, w, lin, gp);
    }

#pragma unroll
    for (int c = 0; c < D; ++c) lam[c] = lin[c];
    --i;
    if constexpr (AT_END) take_saves();
    if (--slot < 0 && i > 0) {
      page = prev_page(R, page);
      slot = K - 1;
      grp = -1;
      if (CKPT) {
        start_segment(K);
        wait = first_gap;
        first_gap = 0;
      }
    }
  }

  if (a.loss_kind != LOSS_COTANGENT) loss = a.scale * loss;
  }  // ok

  // per-trajectory outputs; a trajectory whose record failed gets NaN
  if (valid) {
    if (!SHARED) {
#pragma unroll
      for (int c = 0; c < NP; ++c) gpo[c * n + tr] = ok ? gp[c] : T(NAN);
    }
    if (gyo) {
#pragma unroll
      for (int c = 0; c < D; ++c) gyo[c * n + tr] = ok ? lam[c] : T(NAN);
    }
    if (a.loss_out)
      a.loss_out[tr] = !ok ? NAN : (a.loss_kind == LOSS_COTANGENT ? 0.0 : loss);
  }
  if constexpr (SHARED) {
    // shared parameters: each wavefront sums its lanes by cross-lane
    // exchanges (wave_sum; a failed trajectory contributes nothing), then
    // the block's four wavefront sums are added in wavefront order: one
    // partial per block, in a fixed order
    __shared__ T red[4][NP];
    const int wave = (int)threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NP; ++c) {
      const T sw = wave_sum<T>(ok ? gp[c] : T(0));
      if (lane_id() == 0) red[wave][c] = sw;
    }
    __syncthreads();
    if ((int)threadIdx.x < NP) {
      const int c = (int)threadIdx.x;
      ((T*)a.workspace)[block * NP + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
    }
  }
}

// Blocks per CU the compiler is asked to fit in the record of the FP64
// Lorenz / Tsit5 ensemble (4: four waves per SIMD; five need a 96-register
// budget that spills and runs 50 % slower); no request otherwise.
template <class Sys, class Tab, class T>
struct FwdBlocks {
  static constexpr int value =
      (Sys::ID == 1 && Tab::ORDER == 5 && !Tab::ROS && sizeof(T) == 8) ? 4 : 1;
};

template <class Sys, class Tab, class T, int MODE, bool CKPT, bool DENSE = false>
__global__ void __launch_bounds__(256, (FwdBlocks<Sys, Tab, T>::value))
    erk_forward_kernel(const FwdArgs a) {
  erk_forward_body<Sys, Tab, T, MODE, CKPT, false, DENSE>(a, blockIdx.x);
}

// Full-tape record whose save states are formed afterwards by
// erk_saves_kernel (explicit pairs), with wave-cooperative tape writes.  The
// FP64 Lorenz / Tsit5 record needs 114 VGPRs at four blocks per CU; its 37 KB
// of LDS (a whole group of records per lane and the write queue) admit no
// more.  2^20 trajectories are 16 waves per SIMD: four full rounds.
template <class Sys, class Tab, class T>
struct DeferBlocks {
  static constexpr int value =
      (Sys::ID == 1 && Tab::ORDER == 5 && !Tab::ROS && sizeof(T) == 8) ? 4 : 1;
};

template <class Sys, class Tab, class T>
__global__ void __launch_bounds__(256, (DeferBlocks<Sys, Tab, T>::value))
    erk_record_deferred_kernel(const FwdArgs a) {
  erk_forward_body<Sys, Tab, T, MODE_RECORD, false, true>(a, blockIdx.x);
}

// Save states of a deferred record: for each trajectory and each save time
// noted inside an accepted step (base index i < S), the step map from the
// recorded base state over the noted offset, Phi(y_i; t_s - t_i) -- the side
// step of the paper's extra-step save (Section 3.4), formed as the reverse
// sweep forms it.  Saves at or after the last mesh point were written by
// the record itself.
template <class Sys, class Tab, class T>
__global__ void __launch_bounds__(256) erk_saves_kernel(const FwdArgs a) {
  constexpr int D = Sys::D, NP = Sys::NP, SU = Tab::SU;
  static_assert(!Tab::ROS, "explicit pairs only");
  const int64_t n = a.ivp.n;
  const int64_t tr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tr >= n) return;
  const RecView& R = a.rec;
  const int32_t S = R.steps[tr];
  T p[NP];
  load_params<T, NP>(a.ivp, tr, p);
  T* ysv = (T*)a.y_save;
  const T* sbase = (const T*)R.save_base;
  for (int s = 0; s < a.ivp.n_save; ++s) {
    const int32_t i = R.save_idx[(int64_t)s * n + tr];
    if (i < 0 || i >= S) continue;
    const double dt = R.save_dt[(int64_t)s * n + tr];
    T y[D], k0[D], Yd[SU][D], ylast[D], klast[D], ys[D];
#pragma unroll
    for (int c = 0; c < D; ++c) y[c] = sbase[((int64_t)s * D + c) * n + tr];
    Sys::rhs(y, p, k0);
    step_push<Sys, Tab, T, SU, true, true, false>(y, k0, p, T(dt), Yd, ylast, klast, ys,
                                                  nullptr);
#pragma unroll
    for (int c = 0; c < D; ++c) ysv[((int64_t)s * D + c) * n + tr] = ys[c];
  }
}

// Save states of a dense record: for each trajectory and each save noted
// inside an accepted step (step size h > 0), the step's continuous extension
// from the recorded end states, at the noted offset (saves at the last mesh
// point were written by the record itself).
template <class Sys, class T>
__global__ void __launch_bounds__(256) dense_saves_kernel(const FwdArgs a) {
  constexpr int D = Sys::D, NP = Sys::NP;
  const int64_t n = a.ivp.n;
  const int64_t tr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tr >= n) return;
  const RecView& R = a.rec;
  T p[NP];
  load_params<T, NP>(a.ivp, tr, p);
  T* ysv = (T*)a.y_save;
  const T* b0 = (const T*)R.save_base;
  const T* b1 = (const T*)R.save_base_hi;
  for (int s = 0; s < a.ivp.n_save; ++s) {
    const int32_t i = R.save_idx[(int64_t)s * n + tr];
    const double hs = R.save_h[(int64_t)s * n + tr];
    if (i < 0 || !(hs > 0.0)) continue;
    T y0[D], y1[D], f0[D], f1[D], ys[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      y0[c] = b0[((int64_t)s * D + c) * n + tr];
      y1[c] = b1[((int64_t)s * D + c) * n + tr];
    }
    Sys::rhs(y0, p, f0);
    Sys::rhs(y1, p, f1);
    hermite_state<T, D>(y0, y1, f0, f1, hs, R.save_dt[(int64_t)s * n + tr], ys);
#pragma unroll
    for (int c = 0; c < D; ++c) ysv[((int64_t)s * D + c) * n + tr] = ys[c];
  }
}

// Blocks per CU the compiler is asked to fit in the reverse sweep: 3 for the
// FP64 Lorenz / Tsit5 sweep, which then lands at 124 registers with no
// spill (4 waves per SIMD); asking for 4 gives the same occupancy with a
// spill.  No request for the others.
template <class Sys, class Tab, class T>
struct AdjBlocks {
  static constexpr int value =
      (Sys::ID == 1 && Tab::ORDER == 5 && !Tab::ROS && sizeof(T) == 8) ? 3 : 1;
};

template <class Sys, class Tab, class T, bool SHARED, bool CKPT, bool DENSE = false>
__global__ void __launch_bounds__(256, (AdjBlocks<Sys, Tab, T>::value))
    erk_adjoint_kernel(const AdjArgs a) {
  erk_adjoint_body<Sys, Tab, T, SHARED, CKPT, DENSE>(a, blockIdx.x);
}

// Sum of the per-block partials of shared-parameter gradients, in a fixed
// order: thread k adds blocks k, k+256, ... then a tree over the threads.
template <class T>
__global__ void __launch_bounds__(256) reduce_partials_kernel(const T* part, int64_t nb,
                                                              int np, T* out) {
  __shared__ T red[256];
  const int c = blockIdx.x;
  T acc = T(0);
  for (int64_t b = threadIdx.x; b < nb; b += 256) acc = acc + part[b * np + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

}  // namespace ens
