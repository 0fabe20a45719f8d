// Device-side building blocks shared by the ensemble kernels: scalar fma
// wrappers, wavefront primitives and the device view of a record.
#pragma once
#ifndef __HIPCC_RTC__  // run-time compilation brings its own runtime and types
#include <hip/hip_runtime.h>
#include <stdint.h>
#else
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif
#ifndef INFINITY
#define INFINITY __builtin_inff()
#endif
#ifndef NAN
#define NAN __builtin_nanf("")
#endif

namespace ens {

__device__ __forceinline__ double fmaT(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
__device__ __forceinline__ float fmaT(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// Products and fmas with a factor that is a constant of the method (c) or of
// the step (the step size h and 1/h): the mesh is fixed, so these factors
// carry no tangent in forward mode, where a dual-number type overloads them.
// For plain scalars they are the ordinary operations.
template <class T>
__device__ __forceinline__ T cmul(double c, T x) {
  return T(c) * x;
}
template <class T>
__device__ __forceinline__ T cfma(double c, T x, T acc) {
  return fmaT(T(c), x, acc);
}
template <class T>
__device__ __forceinline__ T hfma(T h, T x, T acc) {  // fma(h, x, acc)
  return fmaT(h, x, acc);
}
template <class T>
__device__ __forceinline__ T fmah(T x, T h, T acc) {  // fma(x, h, acc)
  return fmaT(x, h, acc);
}

enum : int32_t {
  LANE_OK = 0,
  LANE_MAX_STEPS = 1,
  LANE_DT_UNDERFLOW = 2,
  LANE_NONFINITE = 3,
  LANE_NOSPACE = 4,
};

enum : int32_t { LOSS_SUMSQ = 0, LOSS_MSE_TARGET = 1, LOSS_COTANGENT = 2 };

// counters[] slots in the record
enum : int { CNT_PAGES = 0, CNT_ACCEPTED = 1, CNT_TRIALS = 2, CNT_SIDE = 3 };

constexpr int PAGE_STEPS = 16;  // accepted steps per tape page

// Bytes of one taped step: the step size (double) followed by the state
// before the step, padded to 16 bytes so a step is read with vector loads.
template <class T, int D>
struct TapeRec {
  static constexpr int BYTES = ((8 + D * (int)sizeof(T)) + 15) / 16 * 16;
};

// ---------------------------------------------------------- wavefronts --
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane (its rank among them).
__device__ __forceinline__ int rank_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

// Wave-aggregated bump allocation: every active lane with `want` set gets a
// distinct slot of a global counter; one atomic per wave.
__device__ __forceinline__ uint64_t wave_bump(unsigned long long* counter,
                                              bool want) {
  const uint64_t mask = __ballot(want);
  uint64_t base = 0;
  if (mask) {
    const int leader = __ffsll((unsigned long long)mask) - 1;
    if (lane_id() == leader)
      base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
  }
  return base + (uint64_t)rank_below(mask);
}

// Sum over the 64 lanes of a wavefront, by butterfly exchanges: within quads
// (DPP quad_perm, partners lane ^ 1 and lane ^ 2), within rows (DPP
// row_half_mirror, then row_mirror: each exchanges a lane's half-row, then
// its half of the row, with the mirrored one) and across the four rows
// (lane ^ 16 and lane ^ 32).  At every stage a lane and its partner add the
// same two values, so every lane ends with the same, order-fixed sum.  Every
// lane of the wavefront must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = dpp_i32<CTRL>(__double2loint(x));
  const int hi = dpp_i32<CTRL>(__double2hiint(x));
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(dpp_i32<CTRL>(__float_as_int(x)));
}
template <class T>
__device__ __forceinline__ T wave_sum(T x) {
  constexpr int QUAD_XOR1 = 0xB1;   // quad_perm [1, 0, 3, 2]
  constexpr int QUAD_XOR2 = 0x4E;   // quad_perm [2, 3, 0, 1]
  constexpr int ROW_HALF_MIRROR = 0x141;
  constexpr int ROW_MIRROR = 0x140;
  x = x + dpp_move<QUAD_XOR1>(x);
  x = x + dpp_move<QUAD_XOR2>(x);
  x = x + dpp_move<ROW_HALF_MIRROR>(x);
  x = x + dpp_move<ROW_MIRROR>(x);
  x = x + __shfl_xor(x, 16);
  x = x + __shfl_xor(x, 32);
  return x;
}

// Largest value over the 64 lanes of a wavefront, by butterfly exchanges
// (lane ^ 1, ^ 2, ..., ^ 32); every lane of the wavefront must be active.
__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) x = max(x, __shfl_xor(x, m));
  return x;
}

// ----------------------------------------------------------- record view --
// Device view of a record (see ens_record in ensode.h for the meaning).
struct RecView {
  int64_t n;
  int32_t n_save;        // effective, >= 1
  int64_t n_pages;       // reserved + overflow
  int64_t n_static;      // n * static_pages: ids below this are reserved pages
  int32_t static_pages;  // reserved pages per trajectory
  int32_t page_steps;    // accepted steps per page
  int64_t page_bytes;
  int32_t* steps;
  int32_t* n_trial;
  int32_t* first_page;
  int32_t* last_page;
  int32_t* status;
  int32_t* save_idx;     // [n_save][n]
  double* save_dt;       // [n_save][n]
  const double* save_times;
  void* y_final;         // [D][n]
  void* save_base;       // [n_save][D][n] base state of each save's side step
  // dense output: the end state of the step holding each save and its size
  void* save_base_hi;    // [n_save][D][n] or null
  double* save_h;        // [n_save][n] or null
  int32_t* links;        // [overflow pages][2]: previous, next page id
  unsigned long long* counters;
  char* pages;
};

// Page holding the taped step before the first step of `page` (only called
// when such a step exists): reserved pages of a trajectory are consecutive,
// overflow pages are linked.
__device__ __forceinline__ int32_t prev_page(const RecView& R, int32_t page) {
  return page < R.n_static ? page - 1
                           : R.links[2 * ((int64_t)page - R.n_static)];
}

__device__ __forceinline__ int32_t next_page(const RecView& R, int64_t tr,
                                             int32_t page) {
  if (page >= R.n_static) return R.links[2 * ((int64_t)page - R.n_static) + 1];
  const int32_t k = page - (int32_t)(tr * R.static_pages);
  return k + 1 < R.static_pages ? page + 1 : R.first_page[tr];
}

}  // namespace ens
