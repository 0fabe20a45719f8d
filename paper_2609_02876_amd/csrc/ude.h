// Universal differential equation on matrix cores: Lotka-Volterra plus a
// 2-32-32-2 tanh MLP whose weights are shared by every trajectory, FP32 with
// FP32 accumulation.  Record and reverse sweep are the ones of the explicit
// pairs (paper, Sections 2.1, 3.1 and 3.4) with Tsit5; what changes is the
// right-hand side, which is evaluated for a whole wavefront at once.
//
// MLP on MFMA (v_mfma_f32_32x32x2f32).  A wavefront holds 64 trajectories,
// one per lane, as two column blocks of 32.  Every layer is computed in the
// transposed form out[unit][trajectory] = W[unit][k] x[k][trajectory], so
// the trajectories sit on the MFMA's N dimension and the weights are the A
// operand.  In the accumulator layout lane l (half hf = l / 32, column
// c = l % 32) holds, for column block b, trajectory c + 32 b and the 16 units
//   U(r, hf) = 8 (r / 4) + 4 hf + (r % 4),   r = 0..15.
// The next layer takes its B operand for K-step k straight from register k
// (the K index enumerates units in the order U(k, kk), kk = 0, 1), so hidden
// activations never leave registers.  Only the 2-vector input and output of
// the MLP cross between the lane halves (one xor-32 exchange each).
//
// All lanes of a wavefront must run every right-hand side together: a lane
// computes half of the hidden units of two trajectories, its own and its
// partner's.  The kernels below therefore keep finished lanes in the loop
// (doing zero-length steps) until the whole wavefront is done.
//
// Weight gradient.  Per stage the contribution sum over trajectories of
// delta2 h1^T (32 x 32) is one more MFMA chain with the trajectories as the
// K dimension; delta2 and h1 are transposed through a per-wave LDS tile for
// it.  Every other weight gradient is accumulated per lane and reduced over
// the lanes at the end, in a fixed order.
#pragma once
#include <math.h>

#include "erk.h"

namespace ens {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int UDE_NP = 1218;
constexpr int UDE_OW1 = 0, UDE_OB1 = 64, UDE_OW2 = 96, UDE_OB2 = 1120, UDE_OW3 = 1152,
              UDE_OB3 = 1216;
constexpr float LV_A = 1.5f, LV_B = 1.0f, LV_G = 3.0f, LV_D = 1.0f;
constexpr int UDE_STRIDE = 33;                 // LDS row of a transposed tile (no conflicts)
constexpr int UDE_TILE = 64 * UDE_STRIDE;      // one [64 trajectories][32 units] tile
constexpr int UDE_ADJ_WAVES = 4;               // waves per adjoint block

// Per-lane gradient accumulator slots.
enum : int {
  UG_W2 = 0,     // 16: dW2[U(r, hf)][c] (the MFMA accumulator)
  UG_W3 = 16,    // 32: dW3[o][U(r, hf)] at 16 o + r
  UG_B2 = 48,    // 16: db2[U(r, hf)]
  UG_W1 = 64,    // 32: dW1[U(r, hf)][k] at 16 k + r
  UG_B1 = 96,    // 16: db1[U(r, hf)]
  UG_B3 = 112,   // 2:  db3[o]
  UG_N = 114
};

__device__ __forceinline__ int ude_unit(int r, int hf) {
  return 8 * (r >> 2) + 4 * hf + (r & 3);
}

// The weights in the per-lane layouts of the MFMA operands, [slot][lane],
// so that a wavefront reads each slot as 64 consecutive floats.
struct UdeW {
  float a1[64];          // W1[c][hf]
  float a2f[16][64];     // W2[c][U(k, hf)]    (forward layer 2)
  float a2b[16][64];     // W2[U(k, hf)][c]    (transposed, for delta h1)
  float b1[16][64];      // b1[U(r, hf)]
  float b2[16][64];      // b2[U(r, hf)]
  float w3[2][16][64];   // W3[o][U(r, hf)]
  float w1[2][16][64];   // W1[U(r, hf)][k]
  float b3[2];
};

// Weights plus the per-wave transpose tiles of the reverse sweep.
struct UdeAdjLds {
  UdeW w;
  float tile[UDE_ADJ_WAVES][2][UDE_TILE];
};

// Fill the LDS image from the parameter vector (W1, b1, W2, b2, W3, b3).
__device__ __forceinline__ void ude_load_weights(UdeW& s, const float* th) {
  for (int i = threadIdx.x; i < 64; i += blockDim.x) {
    const int hf = i >> 5, c = i & 31;
    s.a1[i] = th[UDE_OW1 + 2 * c + hf];
  }
  for (int i = threadIdx.x; i < 16 * 64; i += blockDim.x) {
    const int k = i >> 6, l = i & 63, hf = l >> 5, c = l & 31;
    const int u = ude_unit(k, hf);
    s.a2f[k][l] = th[UDE_OW2 + 32 * c + u];
    s.a2b[k][l] = th[UDE_OW2 + 32 * u + c];
    s.b1[k][l] = th[UDE_OB1 + u];
    s.b2[k][l] = th[UDE_OB2 + u];
    s.w3[0][k][l] = th[UDE_OW3 + u];
    s.w3[1][k][l] = th[UDE_OW3 + 32 + u];
    s.w1[0][k][l] = th[UDE_OW1 + 2 * u];
    s.w1[1][k][l] = th[UDE_OW1 + 2 * u + 1];
  }
  if (threadIdx.x < 2) s.b3[threadIdx.x] = th[UDE_OB3 + threadIdx.x];
}

__device__ __forceinline__ float xor32(float v) { return __shfl_xor(v, 32); }

// tanh in FP32 (relative error below 5e-7): for |x| < 0.55 the odd series
// x + x^3 P(x^2), P of degree 4 fitted by least squares to (tanh(x)/x - 1)/x^2
// on [0, 0.55]; above, 1 - 2 / (e^{2|x|} + 1) with the hardware exp2 and
// reciprocal (the series avoids that form's cancellation near 0).
__device__ __forceinline__ float ude_tanh(float x) {
  const float ax = fabsf(x);
  const float e = __builtin_amdgcn_exp2f(ax * 2.8853900817779268f);  // 2^(2|x| / ln 2)
  const float big = fmaT(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
  const float x2 = x * x;
  float q = -0.026664944365620613f;
  q = fmaT(q, x2, 0.03440927714109421f);
  q = fmaT(q, x2, -0.05673672631382942f);
  q = fmaT(q, x2, 0.13355417549610138f);
  q = fmaT(q, x2, -0.3333379626274109f);
  const float small = fmaT(x * x2, q, x);
  return ax < 0.55f ? small : copysignf(big, x);
}

__device__ __forceinline__ v16f mfma32(float a, float b, v16f c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Hidden layers for both column blocks: h1 = tanh(W1 x + b1),
// h2 = tanh(W2 h1 + b2), in the accumulator layout.  x0 / x1 are this lane's
// B operands of layer 1 (feature hf of trajectory c + 32 b).
__device__ __forceinline__ void ude_hidden(const UdeW& W, int l, float x0, float x1, v16f& h1a,
                                           v16f& h1b, v16f& h2a, v16f& h2b) {
  v16f c1;
#pragma unroll
  for (int r = 0; r < 16; ++r) c1[r] = W.b1[r][l];
  const float a1 = W.a1[l];
  h1a = mfma32(a1, x0, c1);
  h1b = mfma32(a1, x1, c1);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    h1a[r] = ude_tanh(h1a[r]);
    h1b[r] = ude_tanh(h1b[r]);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) c1[r] = W.b2[r][l];
  h2a = c1;
  h2b = c1;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const float a = W.a2f[k][l];
    h2a = mfma32(a, h1a[k], h2a);
    h2b = mfma32(a, h1b[k], h2b);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    h2a[r] = ude_tanh(h2a[r]);
    h2b[r] = ude_tanh(h2b[r]);
  }
}

// Sum of a lane's half-unit partial with its partner's, low units first:
// the full contraction for this lane's own trajectory.  `mine` is the
// partial for the own trajectory's block, `other` the one for the partner's.
__device__ __forceinline__ float ude_join(int hf, float mine, float other) {
  const float recv = xor32(other);
  return hf == 0 ? mine + recv : recv + mine;
}

struct LvUde {
  static constexpr int D = 2, NP = 0, ID = 5;

  // f(y) = f_LV(y) + W3 h2 + b3 for this lane's trajectory; p is the LDS
  // weight image.  Wave-uniform: every lane of the wavefront must call it.
  __device__ static inline void rhs(const float* y, const float* p, float* f) {
    const UdeW& W = *reinterpret_cast<const UdeW*>(p);
    const int l = __lane_id(), hf = l >> 5;
    const float own = hf ? y[1] : y[0];
    const float recv = xor32(hf ? y[0] : y[1]);
    const float x0 = hf ? recv : own, x1 = hf ? own : recv;
    v16f h1a, h1b, h2a, h2b;
    ude_hidden(W, l, x0, x1, h1a, h1b, h2a, h2b);
    float pa0 = 0.f, pa1 = 0.f, pb0 = 0.f, pb1 = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float u0 = W.w3[0][r][l], u1 = W.w3[1][r][l];
      pa0 = fmaT(u0, h2a[r], pa0);
      pa1 = fmaT(u1, h2a[r], pa1);
      pb0 = fmaT(u0, h2b[r], pb0);
      pb1 = fmaT(u1, h2b[r], pb1);
    }
    const float n0 = ude_join(hf, hf ? pb0 : pa0, hf ? pa0 : pb0);
    const float n1 = ude_join(hf, hf ? pb1 : pa1, hf ? pa1 : pb1);
    const float xy = y[0] * y[1];
    f[0] = (n0 + W.b3[0]) + (LV_A * y[0] - LV_B * xy);
    f[1] = (n1 + W.b3[1]) + (LV_D * xy - LV_G * y[1]);
  }

  // gy = (df/dy)^T w; the weight gradient of w^T f is added to the lane's
  // accumulators g[UG_N].  p is the UdeAdjLds image.  Wave-uniform.
  __device__ static inline void vjp(const float* y, const float* p, const float* w, float* gy,
                                    float* g) {
    const UdeAdjLds& S = *reinterpret_cast<const UdeAdjLds*>(p);
    const UdeW& W = S.w;
    const int l = __lane_id(), hf = l >> 5, c = l & 31;
    const int wave = threadIdx.x >> 6;
    // inputs and cotangents of the two trajectories this lane works on
    const float ry0 = xor32(y[0]), ry1 = xor32(y[1]);
    const float rw0 = xor32(w[0]), rw1 = xor32(w[1]);
    const float ya0 = hf ? ry0 : y[0], ya1 = hf ? ry1 : y[1];   // block a: trajectory c
    const float yb0 = hf ? y[0] : ry0, yb1 = hf ? y[1] : ry1;   // block b: trajectory c + 32
    const float wa0 = hf ? rw0 : w[0], wa1 = hf ? rw1 : w[1];
    const float wb0 = hf ? w[0] : rw0, wb1 = hf ? w[1] : rw1;
    v16f h1a, h1b, h2a, h2b;
    ude_hidden(W, l, hf ? ya1 : ya0, hf ? yb1 : yb0, h1a, h1b, h2a, h2b);

    // output layer: dW3 += w h2^T, db3 += w, delta2 = (W3^T w) (1 - h2^2)
    v16f d2a, d2b;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float u0 = W.w3[0][r][l], u1 = W.w3[1][r][l];
      g[UG_W3 + r] = fmaT(wb0, h2b[r], fmaT(wa0, h2a[r], g[UG_W3 + r]));
      g[UG_W3 + 16 + r] = fmaT(wb1, h2b[r], fmaT(wa1, h2a[r], g[UG_W3 + 16 + r]));
      d2a[r] = fmaT(u1, wa1, u0 * wa0) * fmaT(-h2a[r], h2a[r], 1.f);
      d2b[r] = fmaT(u1, wb1, u0 * wb0) * fmaT(-h2b[r], h2b[r], 1.f);
      g[UG_B2 + r] = (g[UG_B2 + r] + d2a[r]) + d2b[r];
    }
    g[UG_B3] = g[UG_B3] + w[0];
    g[UG_B3 + 1] = g[UG_B3 + 1] + w[1];

    // stage delta2 and h1 as [trajectory][unit] tiles for the weight gradient
    float* td = const_cast<float*>(S.tile[wave][0]);
    float* th = const_cast<float*>(S.tile[wave][1]);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int u = ude_unit(r, hf);
      td[c * UDE_STRIDE + u] = d2a[r];
      td[(c + 32) * UDE_STRIDE + u] = d2b[r];
      th[c * UDE_STRIDE + u] = h1a[r];
      th[(c + 32) * UDE_STRIDE + u] = h1b[r];
    }

    // delta h1 = W2^T delta2 on the matrix cores, delta1 = delta h1 (1 - h1^2)
    v16f e1a = {0}, e1b = {0};
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const float a = W.a2b[k][l];
      e1a = mfma32(a, d2a[k], e1a);
      e1b = mfma32(a, d2b[k], e1b);
    }
    float pa0 = 0.f, pa1 = 0.f, pb0 = 0.f, pb1 = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float da = e1a[r] * fmaT(-h1a[r], h1a[r], 1.f);
      const float db = e1b[r] * fmaT(-h1b[r], h1b[r], 1.f);
      g[UG_B1 + r] = (g[UG_B1 + r] + da) + db;
      g[UG_W1 + r] = fmaT(db, yb0, fmaT(da, ya0, g[UG_W1 + r]));
      g[UG_W1 + 16 + r] = fmaT(db, yb1, fmaT(da, ya1, g[UG_W1 + 16 + r]));
      const float v0 = W.w1[0][r][l], v1 = W.w1[1][r][l];
      pa0 = fmaT(v0, da, pa0);
      pa1 = fmaT(v1, da, pa1);
      pb0 = fmaT(v0, db, pb0);
      pb1 = fmaT(v1, db, pb1);
    }
    const float n0 = ude_join(hf, hf ? pb0 : pa0, hf ? pa0 : pb0);
    const float n1 = ude_join(hf, hf ? pb1 : pa1, hf ? pa1 : pb1);
    // Lotka-Volterra: J = [[a - b y1, -b y0], [d y1, d y0 - g]]
    gy[0] = n0 + fmaT(LV_D * y[1], w[1], (LV_A - LV_B * y[1]) * w[0]);
    gy[1] = n1 + fmaT(LV_D * y[0] - LV_G, w[1], -LV_B * y[0] * w[0]);

    // dW2 += sum over the wave's trajectories of delta2 h1^T: K = trajectories
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = g[UG_W2 + r];
#pragma unroll 8
    for (int k = 0; k < 32; ++k) {
      const int row = (2 * k + hf) * UDE_STRIDE + c;
      acc = mfma32(td[row], th[row], acc);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) g[UG_W2 + r] = acc[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

// ---------------------------------------------------------------- kernels --
constexpr int32_t LANE_IDLE = -1;  // a lane past the end of the ensemble

// Record / solve / frozen-mesh replay of the UDE (Tsit5, FP32): the explicit
// record with a wave-uniform loop -- lanes whose trajectory is done take
// zero-length steps until the whole wavefront is done.
template <int MODE, bool CKPT>
__global__ void __launch_bounds__(256, 2) ude_forward_kernel(const FwdArgs a) {
  using Sys = LvUde;
  using Tab = Tsit5;
  using T = float;
  constexpr int D = 2;
  constexpr int RB = TapeRec<T, D>::BYTES;
  constexpr int YB = StateBytes<T, D>::BYTES;
  constexpr int CH = RB / 16;
  const int K = CKPT ? a.rec.page_steps : PAGE_STEPS;
  const int64_t n = a.ivp.n;
  const int64_t tr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = tr < n;
  __shared__ double s_times[65];
  __shared__ uint4 s_tape[(MODE == MODE_SOLVE || CKPT) ? 1 : TAPE_GROUP * CH * 256];
  __shared__ double s_h[CKPT ? H_GROUP * 256 : 1];
  __shared__ UdeW s_w;
  ude_load_weights(s_w, (const float*)a.ivp.params);
  if (threadIdx.x < 65)
    s_times[threadIdx.x] = (int)threadIdx.x < a.ivp.n_save ? save_time_at(a.ivp.st, threadIdx.x)
                                                          : INFINITY;
  __syncthreads();
  const float* p = reinterpret_cast<const float*>(&s_w);
  const double t0 = a.ivp.t0, t1 = a.ivp.t1;
  const double rtol = a.ivp.rtol, atol = a.ivp.atol;
  const int ns = a.ivp.n_save;
  T* ysv = (T*)a.y_save;
  const RecView& R = a.rec;

  T y[D], k1[D];
#pragma unroll
  for (int c = 0; c < D; ++c) y[c] = valid ? ((const T*)a.ivp.y0)[c * n + tr] : T(1);
  Sys::rhs(y, p, k1);
  int32_t status = valid ? LANE_OK : LANE_IDLE;
  if (valid) {
#pragma unroll
    for (int c = 0; c < D; ++c)
      if (!isfinite(y[c]) || !isfinite(k1[c])) status = LANE_NONFINITE;
  }
  double t = t0, h = 0.0;
  int32_t S_mesh = 0;
  if constexpr (MODE == MODE_FROZEN) {
    if (valid) {
      S_mesh = a.mesh_S[tr];
      if (S_mesh < 0 || (int64_t)S_mesh > a.cap) {
        S_mesh = 0;
        status = LANE_MAX_STEPS;
      }
    }
  } else {
    const double h_init = initial_step<Sys, Tab, T>(y, p, k1, t0, t1, rtol, atol);
    h = a.ivp.h0 > 0.0 ? fmin(a.ivp.h0, t1 - t0) : h_init;
  }

  T yp[D], k1p[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    yp[c] = y[c];
    k1p[c] = k1[c];
  }
  if constexpr (MODE != MODE_SOLVE) {
    if (valid) R.first_page[tr] = -1;
  }
  double tp = t0;
  int next_save = 0;
  T* ys_out = ysv + tr;
  int32_t* sidx_out = R.save_idx + tr;
  double* sdt_out = R.save_dt + tr;
  const int64_t ys_stride = (int64_t)D * n;
  double ts = s_times[0];
  bool side = false;
  int32_t S = 0, trials = 0;
  bool prev_rej = false;
  int32_t page = -1;
  char* pg = nullptr;

  while (true) {
    bool act = status == LANE_OK &&
               (side || (MODE == MODE_FROZEN ? (S < S_mesh) : (t < t1)));
    if (!__any(act)) break;
    double hh = 0.0;
    bool last = false;
    if (act) {
      if (!side) {
        if constexpr (MODE == MODE_FROZEN) {
          hh = a.mesh_h[(int64_t)S * n + tr];
          last = (S == S_mesh - 1);
          ++trials;
        } else {
          if (trials >= a.ivp.max_steps) {
            status = LANE_MAX_STEPS;
            act = false;
          } else if (h < 16.0 * EPS64 * fmax(fabs(t), 1.0)) {
            status = LANE_DT_UNDERFLOW;
            act = false;
          } else {
            ++trials;
            if (t + h >= t1) {
              h = t1 - t;
              last = true;
            }
            hh = h;
          }
        }
      } else {
        hh = ts - tp;
      }
    }

    // one evaluation of the step map by every lane (idle lanes: h = 0)
    T yb[D], kb[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      yb[c] = side ? yp[c] : y[c];
      kb[c] = side ? k1p[c] : k1[c];
    }
    T Yunused[Tab::S][D];
    T ylast[D], klast[D], ynew[D];
    double esum[D];
    step_push<Sys, Tab, T, Tab::S, false, false, MODE != MODE_FROZEN>(
        yb, kb, p, T(hh), Yunused, ylast, klast, ynew, esum);
#pragma unroll
    for (int c = 0; c < D; ++c) ynew[c] = ylast[c];
    double err = 0.0, fac0 = 0.0;
    if constexpr (MODE != MODE_FROZEN) {
      err = err_ms_sum<T, D>(yb, ynew, hh, esum, rtol, atol);  // RMS norm squared
      fac0 = step_factor<2 * (Tab::QEMB + 1)>(err);
    }
    if (!act) continue;

    if (side) {
#pragma unroll
      for (int c = 0; c < D; ++c) ys_out[c * n] = ynew[c];
      ys_out += ys_stride;
      if constexpr (MODE != MODE_SOLVE) {
        *sidx_out = S - 1;
        *sdt_out = hh;
        sidx_out += n;
        sdt_out += n;
      }
      ++next_save;
      ts = s_times[next_save];
      side = ts < t;
      continue;
    }

    if (MODE == MODE_FROZEN || err <= 1.0) {
      if constexpr (MODE != MODE_SOLVE) {
        const int slot = S % K;
        const int kpage = S / K;
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
              continue;
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
          if (need) store_state<T, D>(pg, yb);
          s_h[((slot & (H_GROUP - 1))) * 256 + threadIdx.x] = hh;
          if ((slot & (H_GROUP - 1)) == H_GROUP - 1)
            flush_h(s_h, H_GROUP, pg + YB + (slot - (H_GROUP - 1)) * 8);
        } else {
          stage_rec<T, D>(s_tape, ((slot & (TAPE_GROUP - 1))) * CH, hh, yb);
          if ((slot & (TAPE_GROUP - 1)) == TAPE_GROUP - 1)
            flush_recs<T, D>(s_tape, TAPE_GROUP, pg + (slot - (TAPE_GROUP - 1)) * RB);
        }
      }
      ++S;
      tp = t;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        yp[c] = y[c];
        k1p[c] = k1[c];
        y[c] = ynew[c];
        k1[c] = klast[c];
      }
      t = last ? t1 : t + hh;
      if constexpr (MODE != MODE_FROZEN) {
        h = hh * fmax(0.2, fmin(prev_rej ? 1.0 : 10.0, fac0));
        prev_rej = false;
      }
      side = ts < t;
    } else {
      h = hh * fmax(0.2, fac0);
      prev_rej = true;
    }
  }
  if (!valid) return;

  if constexpr (MODE != MODE_SOLVE) {
    if constexpr (CKPT) {
      const int rem = S % H_GROUP;
      if (rem > 0 && pg != nullptr) flush_h(s_h, rem, pg + YB + ((S - rem) % K) * 8);
    } else {
      const int rem = S % TAPE_GROUP;
      if (rem > 0 && pg != nullptr) {
        const int slot0 = (S - rem) % K;
        flush_recs<T, D>(s_tape, rem, pg + slot0 * RB);
      }
    }
  }
  const bool ok = (status == LANE_OK);
  for (; next_save < ns; ++next_save) {
#pragma unroll
    for (int c = 0; c < D; ++c) ys_out[c * n] = ok ? y[c] : T(NAN);
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
  if (a.lane_status) a.lane_status[tr] = status;
}

// Fixed-order sum over the 32 lanes of this lane's half (result valid in
// the lane with c = 0).
__device__ __forceinline__ float half_sum(float v) {
  v = v + __shfl_xor(v, 16);
  v = v + __shfl_xor(v, 8);
  v = v + __shfl_xor(v, 4);
  v = v + __shfl_xor(v, 2);
  v = v + __shfl_xor(v, 1);
  return v;
}

// Reverse sweep of the UDE with the weight gradient summed over the
// ensemble: one partial [UDE_NP] per wavefront in the workspace, summed by
// reduce_partials_kernel in a fixed order.
template <bool CKPT>
__global__ void __launch_bounds__(64 * UDE_ADJ_WAVES) ude_adjoint_kernel(const AdjArgs a) {
  using Sys = LvUde;
  using Tab = Tsit5;
  using T = float;
  constexpr int D = 2, SU = Tab::SU;
  constexpr int RB = TapeRec<T, D>::BYTES;
  constexpr int YB = StateBytes<T, D>::BYTES;
  const int K = CKPT ? a.rec.page_steps : PAGE_STEPS;
  const int64_t n = a.ivp.n;
  const int64_t tr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = tr < n;
  const RecView& R = a.rec;
  __shared__ UdeAdjLds s_lds;
  ude_load_weights(s_lds.w, (const float*)a.ivp.params);
  __syncthreads();
  const float* p = reinterpret_cast<const float*>(&s_lds);
  const bool ok = valid && R.status[tr] == LANE_OK;
  float g[UG_N];
#pragma unroll
  for (int i = 0; i < UG_N; ++i) g[i] = 0.f;
  T lam[D] = {0.f, 0.f};
  double loss = 0.0;
  const T two_scale = T(2.0 * a.scale);

  const int32_t S = ok ? R.steps[tr] : 0;
  int32_t page = ok ? R.last_page[tr] : -1;
  T ycur[D];
#pragma unroll
  for (int c = 0; c < D; ++c) ycur[c] = ok ? ((const T*)R.y_final)[c * n + tr] : T(1);
  int s = ok ? R.n_save - 1 : -1;
  const int32_t* sidx_p = R.save_idx + (int64_t)(s < 0 ? 0 : s) * n + (valid ? tr : 0);
  const double* sdt_p = R.save_dt + (int64_t)(s < 0 ? 0 : s) * n + (valid ? tr : 0);
  int32_t sidx = ok ? *sidx_p : -1;
  double sdt = ok ? *sdt_p : 0.0;
  auto next_save = [&]() {
    --s;
    sidx_p -= n;
    sdt_p -= n;
    if (s >= 0) {
      sidx = *sidx_p;
      sdt = *sdt_p;
    }
  };
  int32_t i = S;
  int slot = S > 0 ? (S - 1) % K : 0;
  char* scr = CKPT && valid ? (char*)a.scratch + (int64_t)tr * K * RB : nullptr;
  bool rebuild = false;
  int j_rb = 0, seg_len = 0;
  T y_rb[D] = {0.f, 0.f};
  auto start_segment = [&](int len) {
    load_state<T, D>(R.pages + (int64_t)page * R.page_bytes, y_rb);
    rebuild = true;
    j_rb = 0;
    seg_len = len;
  };
  if (CKPT && ok && S > 0) start_segment(slot + 1);

  while (true) {
    while (!rebuild && s >= 0 && sidx == i && sdt == 0.0) {
      T w[D];
      save_cotangent<T, D>(a, s, tr, ycur, two_scale, w, loss);
#pragma unroll
      for (int c = 0; c < D; ++c) lam[c] = lam[c] + w[c];
      next_save();
    }
    const bool side = !rebuild && (s >= 0 && sidx == i);
    const bool act = ok && (rebuild || side || i > 0);
    if (!__any(act)) break;

    T yb[D] = {T(1), T(1)};
    double hh = 0.0;
    if (act) {
      if (side) {
        hh = sdt;
#pragma unroll
        for (int c = 0; c < D; ++c) yb[c] = ycur[c];
      } else if (CKPT && rebuild) {
        hh = ((const double*)(R.pages + (int64_t)page * R.page_bytes + YB))[j_rb];
#pragma unroll
        for (int c = 0; c < D; ++c) yb[c] = y_rb[c];
      } else if (CKPT) {
        load_rec<T, D>(scr + slot * RB, hh, yb);
      } else {
        load_rec<T, D>(R.pages + (int64_t)page * R.page_bytes + slot * RB, hh, yb);
      }
    }

    // stages of this step, recomputed by every lane
    T k0[D], Y[SU][D], ylast[D], klast[D], ys[D];
    Sys::rhs(yb, p, k0);
    step_push<Sys, Tab, T, SU, true, true, false>(yb, k0, p, T(hh), Y, ylast, klast, ys,
                                                  nullptr);
    const bool rb_step = CKPT && act && rebuild;
    if (rb_step) {
      store_rec<T, D>(scr + j_rb * RB, hh, yb);
#pragma unroll
      for (int c = 0; c < D; ++c) y_rb[c] = ys[c];
      if (++j_rb == seg_len) rebuild = false;
    }
    const bool rev = act && !rb_step;
    T w[D] = {T(0), T(0)};
    if (rev && side) {
      save_cotangent<T, D>(a, s, tr, ys, two_scale, w, loss);
    } else if (rev) {
#pragma unroll
      for (int c = 0; c < D; ++c) w[c] = lam[c];
    }

    // reverse through the stages (every lane, zero cotangent where idle);
    // skipped when no lane of the wavefront reverses a step (segment replays)
    T Yb[SU][D], lin[D];
#pragma unroll
    for (int c = 0; c < D; ++c) lin[c] = w[c];
    if (__any(rev)) {
      // One stage per trip of a loop that is not unrolled, so that one copy
      // of the VJP (and its registers) serves all stages; the stage arrays
      // are read and written by selects over the constant stage index.
      // Tsit5's b_j and a_lj (l > j) are all nonzero, so the sum is
      // b_j w + a_{j+1,j} Ybar_{j+1} + ... in index order, as unrolled.
      static_assert(Tab::B[0] != 0.0 && Tab::B[5] != 0.0 && Tab::A[5][4] != 0.0 &&
                        Tab::A[5][0] != 0.0 && Tab::A[4][0] != 0.0,
                    "dense lower triangle expected");
#pragma unroll 1
      for (int j = SU - 1; j >= 0; --j) {
        T kb[D], Yj[D], Ybj[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
          T yj = Y[0][c];
#pragma unroll
          for (int q = 1; q < SU; ++q) yj = (q == j) ? Y[q][c] : yj;
          Yj[c] = yj;
          T acc = T(Tab::B[0]) * w[c];
#pragma unroll
          for (int q = 1; q < SU; ++q) acc = (q == j) ? T(Tab::B[q]) * w[c] : acc;
#pragma unroll
          for (int l2 = 1; l2 < SU; ++l2) {
            T a = T(0);
#pragma unroll
            for (int q = 0; q < l2; ++q) a = (q == j) ? T(Tab::A[l2][q]) : a;
            acc = (l2 > j) ? fmaT(a, Yb[l2][c], acc) : acc;
          }
          kb[c] = T(hh) * acc;
        }
        Sys::vjp(Yj, p, kb, Ybj, g);
#pragma unroll
        for (int c = 0; c < D; ++c) {
          lin[c] = lin[c] + Ybj[c];
#pragma unroll
          for (int q = 0; q < SU; ++q) Yb[q][c] = (q == j) ? Ybj[c] : Yb[q][c];
        }
      }
    }
    if (!rev) continue;

    if (side) {
#pragma unroll
      for (int c = 0; c < D; ++c) lam[c] = lam[c] + lin[c];
      next_save();
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        lam[c] = lin[c];
        ycur[c] = yb[c];
      }
      --i;
      if (--slot < 0 && i > 0) {
        page = prev_page(R, page);
        slot = K - 1;
        if (CKPT) start_segment(K);
      }
    }
  }
  if (a.loss_kind != LOSS_COTANGENT) loss = a.scale * loss;

  if (valid) {
    T* gyo = (T*)a.grad_y0;
    if (gyo) {
#pragma unroll
      for (int c = 0; c < D; ++c) gyo[c * n + tr] = ok ? lam[c] : T(NAN);
    }
    if (a.loss_out) a.loss_out[tr] = !ok ? NAN : (a.loss_kind == LOSS_COTANGENT ? 0.0 : loss);
  }

  // this wavefront's partial of the weight gradient, in parameter order
  const int l = __lane_id(), hf = l >> 5, c = l & 31;
  float* part = (float*)a.workspace + ((int64_t)blockIdx.x * UDE_ADJ_WAVES + (threadIdx.x >> 6)) * UDE_NP;
#pragma unroll
  for (int r = 0; r < 16; ++r) part[UDE_OW2 + 32 * ude_unit(r, hf) + c] = g[UG_W2 + r];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int u = ude_unit(r, hf);
    const float w30 = half_sum(g[UG_W3 + r]), w31 = half_sum(g[UG_W3 + 16 + r]);
    const float b2 = half_sum(g[UG_B2 + r]);
    const float w10 = half_sum(g[UG_W1 + r]), w11 = half_sum(g[UG_W1 + 16 + r]);
    const float b1 = half_sum(g[UG_B1 + r]);
    if (c == 0) {
      part[UDE_OW3 + u] = w30;
      part[UDE_OW3 + 32 + u] = w31;
      part[UDE_OB2 + u] = b2;
      part[UDE_OW1 + 2 * u] = w10;
      part[UDE_OW1 + 2 * u + 1] = w11;
      part[UDE_OB1 + u] = b1;
    }
  }
  // both halves: exchange first (every lane), then add low half first
  float b30 = half_sum(g[UG_B3]), b31 = half_sum(g[UG_B3 + 1]);
  const float o30 = __shfl_xor(b30, 32), o31 = __shfl_xor(b31, 32);
  b30 = hf == 0 ? b30 + o30 : o30 + b30;
  b31 = hf == 0 ? b31 + o31 : o31 + b31;
  if (l == 0) {
    part[UDE_OB3] = b30;
    part[UDE_OB3 + 1] = b31;
  }
}

}  // namespace ens
