// Host side of the C ABI declared in include/ensode.h: argument checks,
// pool layout, kernel dispatch over (system, method, dtype).
#include <hip/hip_runtime.h>

#include <hip/hiprtc.h>

#include <cctype>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "ensode.h"
#include "erk.h"
#include "jvp.h"
#include "ude.h"

using namespace ens;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char* fmt, ...) {
  char buf[2048];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(ENS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

struct SysInfo {
  int d, np;
};

// systems registered at run time (rtc.h)
bool is_rtc(int sys);
bool rtc_info(int sys, int* d, int* np, bool* jac);

bool sys_info(int sys, SysInfo* s) {
  switch (sys) {
    case ENS_SYS_LORENZ: *s = {3, 3}; return true;
    case ENS_SYS_VDP: *s = {2, 1}; return true;
    case ENS_SYS_ROBERTSON: *s = {3, 3}; return true;
    case ENS_SYS_HIRES: *s = {8, 12}; return true;
    case ENS_SYS_LV_UDE: *s = {2, UDE_NP}; return true;
    case ENS_SYS_LINEAR: *s = {2, 2}; return true;
  }
  bool jac;
  return rtc_info(sys, &s->d, &s->np, &jac);
}

size_t elem_size(int dtype) { return dtype == ENS_F32 ? 4 : 8; }

size_t rec_bytes(int dtype, int d) {
  return ((8 + d * elem_size(dtype)) + 15) / 16 * 16;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool is_ros_method(int m) { return m == ENS_RODAS4 || m == ENS_ROS23; }

int check_problem(const ens_problem* p, SysInfo* si) {
  if (!p) return fail(ENS_EINVAL, "problem is NULL");
  if (!sys_info(p->system, si))
    return fail(ENS_EUNSUPPORTED, "unknown system %d", p->system);
  if (p->dim != si->d || p->nparams != si->np)
    return fail(ENS_EINVAL, "system %d has dim %d and %d params (got %d, %d)",
                p->system, si->d, si->np, p->dim, p->nparams);
  if (p->method != ENS_TSIT5 && p->method != ENS_VERN7 && !is_ros_method(p->method))
    return fail(ENS_EUNSUPPORTED, "unknown method %d", p->method);
  if (p->dtype != ENS_F64 && p->dtype != ENS_F32)
    return fail(ENS_EUNSUPPORTED, "unknown dtype %d", p->dtype);
  if (p->system == ENS_SYS_LV_UDE) {
    if (p->method != ENS_TSIT5 || p->dtype != ENS_F32)
      return fail(ENS_EUNSUPPORTED, "the UDE is built for Tsit5 in F32 only");
    if (p->params_shared != 1)
      return fail(ENS_EINVAL, "the UDE's network weights are shared: params_shared must be 1");
    return ENS_OK;
  }
  if (p->system >= ENS_SYS_USER_BASE) {
    int d, np;
    bool jac;
    rtc_info(p->system, &d, &np, &jac);
    if (is_ros_method(p->method) && !jac)
      return fail(ENS_EUNSUPPORTED,
                  "system %d was registered without jac and jac_vjp, which a Rosenbrock "
                  "method needs",
                  p->system);
    if (is_ros_method(p->method) && p->dtype != ENS_F64)
      return fail(ENS_EUNSUPPORTED, "the Rosenbrock methods are built for F64 only");
    if (p->params_shared != 0 && p->params_shared != 1)
      return fail(ENS_EINVAL, "params_shared must be 0 or 1");
    return ENS_OK;
  }
  const bool stiff_sys = p->system == ENS_SYS_ROBERTSON || p->system == ENS_SYS_HIRES;
  if (is_ros_method(p->method)) {
    if (!stiff_sys && p->system != ENS_SYS_LINEAR)
      return fail(ENS_EUNSUPPORTED,
                  "the Rosenbrock methods run on the Robertson, HIRES and linear systems");
    if (p->dtype != ENS_F64)
      return fail(ENS_EUNSUPPORTED, "the Rosenbrock methods are built for F64 only");
  } else if (stiff_sys) {
    return fail(ENS_EUNSUPPORTED, "system %d is stiff: use ENS_RODAS4 or ENS_ROS23",
                p->system);
  }
  if (p->params_shared != 0 && p->params_shared != 1)
    return fail(ENS_EINVAL, "params_shared must be 0 or 1");
  return ENS_OK;
}

int check_ivp(const ens_ivp* v, bool need_ptrs) {
  if (!v) return fail(ENS_EINVAL, "ivp is NULL");
  if (v->n <= 0 || v->n > (int64_t)INT32_MAX * 64)
    return fail(ENS_EINVAL, "n = %lld out of range", (long long)v->n);
  if (need_ptrs && (!v->y0 || !v->params))
    return fail(ENS_EINVAL, "y0 and params must be device pointers");
  if (!(std::isfinite(v->t0) && std::isfinite(v->t1) && v->t1 > v->t0))
    return fail(ENS_EINVAL, "need finite t0 < t1 (got %g, %g)", v->t0, v->t1);
  if (!(v->rtol >= 0.0 && v->atol >= 0.0 && (v->rtol > 0.0 || v->atol > 0.0)) ||
      !std::isfinite(v->rtol) || !std::isfinite(v->atol))
    return fail(ENS_EINVAL, "need rtol >= 0, atol >= 0, not both zero");
  if (!(v->h0 >= 0.0) || !std::isfinite(v->h0))
    return fail(ENS_EINVAL, "h0 must be finite and >= 0");
  if (v->max_steps < 0 || v->max_steps > INT32_MAX)
    return fail(ENS_EINVAL, "max_steps out of range");
  if (v->n_save < 0 || v->n_save > ENS_MAX_SAVE)
    return fail(ENS_EINVAL, "n_save must be in [0, %d]", ENS_MAX_SAVE);
  if (v->dense != 0 && v->dense != 1) return fail(ENS_EINVAL, "dense must be 0 or 1");
  if (v->n_save > 0) {
    if (!v->save_times) return fail(ENS_EINVAL, "save_times is NULL");
    for (int i = 0; i < v->n_save; ++i) {
      const double s = v->save_times[i];
      if (!(s >= v->t0 && s <= v->t1))
        return fail(ENS_EINVAL, "save time %d = %g outside [t0, t1]", i, s);
      if (i > 0 && s < v->save_times[i - 1])
        return fail(ENS_EINVAL, "save times must be nondecreasing");
    }
  }
  return ENS_OK;
}

// Pool layout of a record.
struct Layout {
  size_t counters, save_times, steps, n_trial, first_page, last_page, status,
      save_idx, save_dt, y_final, save_base, save_base_hi, save_h, links, pages;
  size_t fixed;  // bytes before the links array
  size_t page_bytes;
};

size_t state_bytes(int dtype, int d) { return (d * elem_size(dtype) + 15) / 16 * 16; }

// Accepted steps per page: 16 for a full tape, the checkpoint interval otherwise.
int page_steps_of(int ckpt_every) { return ckpt_every > 0 ? ckpt_every : PAGE_STEPS; }

bool ckpt_ok(int ckpt_every) {
  return ckpt_every == 0 || ckpt_every == 16 || ckpt_every == 32 || ckpt_every == 64 ||
         ckpt_every == 128 || ckpt_every == 256;
}

Layout layout(int64_t n, int n_save_eff, int d, int dtype, int ckpt_every, bool dense = false) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  L.counters = take(8 * sizeof(unsigned long long));
  L.save_times = take(ENS_MAX_SAVE * sizeof(double));
  L.steps = take(n * 4);
  L.n_trial = take(n * 4);
  L.first_page = take(n * 4);
  L.last_page = take(n * 4);
  L.status = take(n * 4);
  L.save_idx = take((size_t)n_save_eff * n * 4);
  L.save_dt = take((size_t)n_save_eff * n * 8);
  L.y_final = take((size_t)d * n * elem_size(dtype));
  L.save_base = take((size_t)n_save_eff * d * n * elem_size(dtype));
  // dense output: each save's step end state and step size
  L.save_base_hi = dense ? take((size_t)n_save_eff * d * n * elem_size(dtype)) : 0;
  L.save_h = dense ? take((size_t)n_save_eff * n * 8) : 0;
  L.fixed = off;
  L.links = off;
  L.page_bytes = ckpt_every > 0
                     ? state_bytes(dtype, d) + (size_t)ckpt_every * sizeof(double)
                     : (size_t)PAGE_STEPS * rec_bytes(dtype, d);
  return L;
}

// Split of a pool into reserved pages (static_pages per trajectory) and an
// overflow area whose pages carry 8 bytes of links each.
struct PageSplit {
  int64_t static_pages, n_static, n_over;
};

bool split_pages(const Layout& L, int64_t n, size_t pool_bytes,
                 int32_t steps_per_traj, int page_steps, PageSplit* ps) {
  if (pool_bytes < L.fixed + 512) return false;
  const size_t avail = pool_bytes - L.fixed - 256;
  int64_t sp;
  if (steps_per_traj > 0) {
    sp = (steps_per_traj + page_steps - 1) / page_steps;
  } else {
    sp = (int64_t)((avail / 8 * 7) / ((size_t)n * L.page_bytes));
  }
  const size_t static_bytes = (size_t)n * (size_t)sp * L.page_bytes;
  if (static_bytes > avail) return false;
  ps->static_pages = sp;
  ps->n_static = n * sp;
  ps->n_over = (int64_t)((avail - static_bytes) / (L.page_bytes + 8));
  return true;
}

void fill_record(ens_record* r, const ens_problem* p, const ens_ivp* v,
                 const ens_tape_cfg* tc, const Layout& L, const PageSplit& ps) {
  const int64_t n_pages = ps.n_static + ps.n_over;
  memset(r, 0, sizeof *r);
  char* base = (char*)tc->pool;
  r->n = v->n;
  r->system = p->system;
  r->method = p->method;
  r->dtype = p->dtype;
  r->dim = p->dim;
  r->nparams = p->nparams;
  r->params_shared = p->params_shared;
  r->n_save = v->n_save > 0 ? v->n_save : 1;
  r->page_steps = page_steps_of(tc->ckpt_every);
  r->ckpt_every = tc->ckpt_every;
  r->rec_bytes = (int32_t)rec_bytes(p->dtype, p->dim);
  r->n_pages = n_pages;
  r->page_bytes = (int64_t)L.page_bytes;
  r->static_pages = (int32_t)ps.static_pages;
  r->t0 = v->t0;
  r->t1 = v->t1;
  r->pool = tc->pool;
  r->pool_bytes = tc->pool_bytes;
  r->counters = (unsigned long long*)(base + L.counters);
  r->save_times = (double*)(base + L.save_times);
  r->steps = (int32_t*)(base + L.steps);
  r->n_trial = (int32_t*)(base + L.n_trial);
  r->first_page = (int32_t*)(base + L.first_page);
  r->last_page = (int32_t*)(base + L.last_page);
  r->status = (int32_t*)(base + L.status);
  r->save_idx = (int32_t*)(base + L.save_idx);
  r->save_dt = (double*)(base + L.save_dt);
  r->y_final = base + L.y_final;
  r->save_base = base + L.save_base;
  r->dense = v->dense;
  r->save_base_hi = v->dense ? base + L.save_base_hi : nullptr;
  r->save_h = v->dense ? (double*)(base + L.save_h) : nullptr;
  r->links = (int32_t*)(base + L.links);
  r->pages = base + align256(L.links + (size_t)ps.n_over * 8);
}

RecView view_of(const ens_record* r) {
  RecView v{};
  v.n = r->n;
  v.n_save = r->n_save;
  v.n_pages = r->n_pages;
  v.static_pages = r->static_pages;
  v.page_steps = r->page_steps;
  v.n_static = r->n * (int64_t)r->static_pages;
  v.page_bytes = r->page_bytes;
  v.steps = r->steps;
  v.n_trial = r->n_trial;
  v.first_page = r->first_page;
  v.last_page = r->last_page;
  v.status = r->status;
  v.save_idx = r->save_idx;
  v.save_dt = r->save_dt;
  v.save_times = r->save_times;
  v.y_final = r->y_final;
  v.save_base = r->save_base;
  v.save_base_hi = r->save_base_hi;
  v.save_h = r->save_h;
  v.links = r->links;
  v.counters = r->counters;
  v.pages = (char*)r->pages;
  return v;
}

// Small setup kernel: clears the counters and copies the save times into the
// pool (no memset node, so the sequence stays capturable).
__global__ void setup_kernel(unsigned long long* counters, double* dst,
                             const SaveTimes st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) counters[i] = 0ull;
#pragma unroll
    for (int i = 0; i < ENS_MAX_SAVE; ++i)
      if (i < st.n) dst[i] = st.t[i];
  }
}

SaveTimes save_times_of(const ens_ivp* v) {
  SaveTimes st{};
  if (v->n_save > 0) {
    st.n = v->n_save;
    for (int i = 0; i < v->n_save; ++i) st.t[i] = v->save_times[i];
  } else {
    st.n = 1;
    st.t[0] = v->t1;
  }
  return st;
}

IvpArgs ivp_args(const ens_problem* p, const ens_ivp* v) {
  IvpArgs a{};
  a.n = v->n;
  a.y0 = v->y0;
  a.params = v->params;
  a.params_shared = p->params_shared;
  a.t0 = v->t0;
  a.t1 = v->t1;
  a.rtol = v->rtol;
  a.atol = v->atol;
  a.h0 = v->h0;
  a.max_steps = v->max_steps > 0 ? v->max_steps : 100000;
  a.n_save = v->n_save > 0 ? v->n_save : 1;
  a.st = save_times_of(v);
  return a;
}

// ------------------------------------------------------------- dispatch --
template <class F>
int with_kernels(int sys, int method, int dtype, F&& f) {
  auto by_type = [&](auto sys_tag, auto tab_tag) -> int {
    if (dtype == ENS_F64) return f(sys_tag, tab_tag, double{});
    return f(sys_tag, tab_tag, float{});
  };
  auto by_method = [&](auto sys_tag) -> int {
    if (method == ENS_TSIT5) return by_type(sys_tag, Tsit5{});
    return by_type(sys_tag, Vern7{});
  };
  auto by_ros = [&](auto tab_tag) -> int {
    if (dtype != ENS_F64)
      return fail(ENS_EUNSUPPORTED, "the Rosenbrock methods are built for F64 only");
    switch (sys) {
      case ENS_SYS_ROBERTSON: return f(Robertson{}, tab_tag, double{});
      case ENS_SYS_HIRES: return f(Hires{}, tab_tag, double{});
      case ENS_SYS_LINEAR: return f(Linear{}, tab_tag, double{});
    }
    return fail(ENS_EUNSUPPORTED, "the Rosenbrock methods are not built for system %d", sys);
  };
  if (method == ENS_RODAS4) return by_ros(Rodas4{});
  if (method == ENS_ROS23) return by_ros(Ros23{});
  switch (sys) {
    case ENS_SYS_LORENZ: return by_method(Lorenz{});
    case ENS_SYS_VDP: return by_method(VanDerPol{});
    case ENS_SYS_LINEAR: return by_method(Linear{});
  }
  return fail(ENS_EUNSUPPORTED, "unknown system %d", sys);
}

constexpr int BLOCK = 256;

unsigned grid_of(int64_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }

#include "rtc.h"

// Shared-parameter partials of the reverse sweep: one per block, or one per
// wavefront for the UDE (whose gradient is reduced per wavefront).
size_t partials_bytes(int sys, int64_t n, int np, int dtype) {
  const size_t parts = (size_t)grid_of(n) * (sys == ENS_SYS_LV_UDE ? UDE_ADJ_WAVES : 1);
  return align256(parts * np * elem_size(dtype));
}

int launch_forward_ude(int mode, bool ckpt, const FwdArgs& fa, hipStream_t st) {
  const dim3 g(grid_of(fa.ivp.n)), b(BLOCK);
  if (mode == MODE_SOLVE)
    hipLaunchKernelGGL((ude_forward_kernel<MODE_SOLVE, false>), g, b, 0, st, fa);
  else if (mode == MODE_RECORD && !ckpt)
    hipLaunchKernelGGL((ude_forward_kernel<MODE_RECORD, false>), g, b, 0, st, fa);
  else if (mode == MODE_RECORD)
    hipLaunchKernelGGL((ude_forward_kernel<MODE_RECORD, true>), g, b, 0, st, fa);
  else if (!ckpt)
    hipLaunchKernelGGL((ude_forward_kernel<MODE_FROZEN, false>), g, b, 0, st, fa);
  else
    hipLaunchKernelGGL((ude_forward_kernel<MODE_FROZEN, true>), g, b, 0, st, fa);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ENS_OK : hip_fail(e, "forward launch");
}

// Base states of the saves of a full-tape record made on a given mesh
// (MODE_FROZEN, MODE_REFRESH), which those loops do not store: the state in
// the record of step i + 1 for a save based at mesh point i < S, the final
// state for i = S.  Element size es (4 or 8), dimension d.
__global__ void __launch_bounds__(256) save_bases_kernel(const RecView R, int64_t n, int d,
                                                         int es) {
  const int64_t tr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tr >= n || R.status[tr] != LANE_OK) return;
  const int32_t S = R.steps[tr];
  const int rb = (8 + d * es + 15) / 16 * 16;
  int32_t page = -1, pidx = -1;  // the page last walked to and its index
  for (int s = 0; s < R.n_save; ++s) {
    const int32_t i = R.save_idx[(int64_t)s * n + tr];
    const char* src;
    int64_t sstride;  // bytes between components
    if (i >= S) {
      src = (const char*)R.y_final + tr * es;
      sstride = n * es;
    } else {
      const int32_t q = i / PAGE_STEPS;
      if (q < R.static_pages) {
        page = (int32_t)(tr * R.static_pages + q);
        pidx = q;
      } else {
        if (pidx < R.static_pages || pidx > q) {
          page = R.first_page[tr];
          pidx = R.static_pages;
        }
        for (; pidx < q; ++pidx) page = next_page(R, tr, page);
      }
      src = R.pages + (int64_t)page * R.page_bytes + (i % PAGE_STEPS) * rb + 8;
      sstride = es;
    }
    char* dst = (char*)R.save_base + ((int64_t)s * d * n + tr) * es;
    for (int c = 0; c < d; ++c) {
      if (es == 8)
        *(double*)(dst + (int64_t)c * n * es) = *(const double*)(src + c * sstride);
      else
        *(float*)(dst + (int64_t)c * n * es) = *(const float*)(src + c * sstride);
    }
  }
}

int launch_forward_body(const ens_problem* p, int mode, bool ckpt, const FwdArgs& fa,
                        hipStream_t st, bool dense);

int launch_forward(const ens_problem* p, int mode, bool ckpt, const FwdArgs& fa,
                   hipStream_t st, bool dense = false) {
  int rc = launch_forward_body(p, mode, ckpt, fa, st, dense);
  if (rc != ENS_OK || ckpt || dense || (mode != MODE_FROZEN && mode != MODE_REFRESH) ||
      p->system == ENS_SYS_LV_UDE)
    return rc;
  SysInfo si;
  sys_info(p->system, &si);
  hipLaunchKernelGGL(save_bases_kernel, dim3(grid_of(fa.ivp.n)), dim3(BLOCK), 0, st, fa.rec,
                     fa.ivp.n, si.d, (int)elem_size(p->dtype));
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ENS_OK : hip_fail(e, "save-base launch");
}

int launch_forward_body(const ens_problem* p, int mode, bool ckpt, const FwdArgs& fa,
                        hipStream_t st, bool dense) {
  if (p->system == ENS_SYS_LV_UDE) return launch_forward_ude(mode, ckpt, fa, st);
  if (dense) {
    // dense output: the save states from the continuous extension, formed in
    // the loop (solve, record with either tape, replay of a given mesh)
    return with_kernels(p->system, p->method, p->dtype, [&](auto s, auto m, auto t) {
      using Sys = decltype(s);
      using Tab = decltype(m);
      using T = decltype(t);
      const dim3 g(grid_of(fa.ivp.n)), b(BLOCK);
      if (mode == MODE_SOLVE)
        hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_SOLVE, false, true>), g, b, 0,
                           st, fa);
      else if (mode == MODE_RECORD && !ckpt)
        hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_RECORD, false, true>), g, b,
                           0, st, fa);
      else if (mode == MODE_RECORD)
        hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_RECORD, true, true>), g, b, 0,
                           st, fa);
      else if (mode == MODE_FROZEN && !ckpt)
        hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_FROZEN, false, true>), g, b,
                           0, st, fa);
      else if (mode == MODE_FROZEN)
        hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_FROZEN, true, true>), g, b, 0,
                           st, fa);
      else
        return fail(ENS_EUNSUPPORTED, "dense output is not built for this mode");
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "dense forward launch");
      if (mode == MODE_SOLVE) return ENS_OK;
      // the records note each save's step; the states come from its extension
      hipLaunchKernelGGL((dense_saves_kernel<Sys, T>), g, b, 0, st, fa);
      e = hipGetLastError();
      return e == hipSuccess ? ENS_OK : hip_fail(e, "dense save-state launch");
    });
  }
  if (is_rtc(p->system)) {
    if (mode == MODE_RECORD && !ckpt && (p->method == ENS_TSIT5 || p->method == ENS_VERN7)) {
      // the explicit pairs' full-tape record forms its save states afterwards
      const int rc = rtc_launch(p->system, p->method, p->dtype,
                                deferred_expr(p->method, p->dtype), grid_of(fa.ivp.n), fa, st);
      if (rc != ENS_OK) return rc;
      return rtc_launch(p->system, p->method, p->dtype, saves_expr(p->method, p->dtype),
                        grid_of(fa.ivp.n), fa, st);
    }
    return rtc_launch(p->system, p->method, p->dtype, fwd_expr(p->method, p->dtype, mode, ckpt),
                      grid_of(fa.ivp.n), fa, st);
  }
  return with_kernels(p->system, p->method, p->dtype, [&](auto s, auto m, auto t) {
    using Sys = decltype(s);
    using Tab = decltype(m);
    using T = decltype(t);
    const dim3 g(grid_of(fa.ivp.n)), b(BLOCK);
    if constexpr (!Tab::ROS) {
      if (mode == MODE_RECORD && !ckpt) {
        // the explicit pairs' full-tape record forms its save states afterwards
        hipLaunchKernelGGL((erk_record_deferred_kernel<Sys, Tab, T>), g, b, 0, st, fa);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "record launch");
        hipLaunchKernelGGL((erk_saves_kernel<Sys, Tab, T>), g, b, 0, st, fa);
        e = hipGetLastError();
        return e == hipSuccess ? ENS_OK : hip_fail(e, "save-state launch");
      }
    }
    if (mode == MODE_SOLVE)
      hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_SOLVE, false>), g, b, 0, st, fa);
    else if (mode == MODE_RECORD && !ckpt)
      hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_RECORD, false>), g, b, 0, st, fa);
    else if (mode == MODE_RECORD)
      hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_RECORD, true>), g, b, 0, st, fa);
    else if (mode == MODE_REFRESH && !ckpt)
      hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_REFRESH, false>), g, b, 0, st, fa);
    else if (mode == MODE_REFRESH)
      hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_REFRESH, true>), g, b, 0, st, fa);
    else if (!ckpt)
      hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_FROZEN, false>), g, b, 0, st, fa);
    else
      hipLaunchKernelGGL((erk_forward_kernel<Sys, Tab, T, MODE_FROZEN, true>), g, b, 0, st, fa);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ENS_OK : hip_fail(e, "forward launch");
  });
}

int check_record_matches(const ens_problem* p, const ens_ivp* v,
                         const ens_record* r) {
  if (!r) return fail(ENS_EINVAL, "record is NULL");
  if (r->n != v->n || r->system != p->system || r->method != p->method ||
      r->dtype != p->dtype || r->params_shared != p->params_shared)
    return fail(ENS_EINVAL, "record does not match the problem / ivp");
  if (r->n_save != (v->n_save > 0 ? v->n_save : 1))
    return fail(ENS_EINVAL, "record has %d save times, ivp %d", r->n_save,
                v->n_save);
  if (r->dense != v->dense)
    return fail(ENS_EINVAL, "record and ivp differ in dense output");
  if (!r->pool || !r->pages) return fail(ENS_EINVAL, "record has no pool");
  return ENS_OK;
}

// Dense output is built for the explicit pairs and the Rosenbrock methods on
// the built-in systems other than the UDE, in the solve, the record and the
// replay of a given mesh.
int check_dense(const ens_problem* p, const ens_ivp* v, int mode) {
  if (!v->dense) return ENS_OK;
  if (p->system == ENS_SYS_LV_UDE || is_rtc(p->system))
    return fail(ENS_EUNSUPPORTED, "dense output is not built for the UDE or registered systems");
  if (mode == MODE_REFRESH)
    return fail(ENS_EUNSUPPORTED, "dense output is not built for the mesh refresh");
  return ENS_OK;
}

int record_common(const ens_problem* p, const ens_ivp* v,
                  const ens_tape_cfg* tc, int mode, const double* mesh_h,
                  const int32_t* mesh_S, int64_t cap, ens_record* out,
                  void* y_save, int32_t* lane_status, void* stream, double slack = 1.0,
                  int32_t* drift_at = nullptr) {
  SysInfo si;
  int rc;
  if ((rc = check_problem(p, &si)) != ENS_OK) return rc;
  if ((rc = check_ivp(v, true)) != ENS_OK) return rc;
  if (!tc || !tc->pool) return fail(ENS_EINVAL, "tape pool is NULL");
  if (((uintptr_t)tc->pool & 255) != 0)
    return fail(ENS_EINVAL, "tape pool must be 256-byte aligned");
  if (!ckpt_ok(tc->ckpt_every))
    return fail(ENS_EINVAL, "ckpt_every must be 0, 16, 32, 64, 128 or 256");
  if (!out || !y_save) return fail(ENS_EINVAL, "out and y_save are required");
  const int nse = v->n_save > 0 ? v->n_save : 1;
  if ((rc = check_dense(p, v, mode)) != ENS_OK) return rc;
  Layout L = layout(v->n, nse, si.d, p->dtype, tc->ckpt_every, v->dense != 0);
  if (tc->steps_per_traj < 0) return fail(ENS_EINVAL, "steps_per_traj < 0");
  PageSplit ps;
  if (!split_pages(L, v->n, tc->pool_bytes, tc->steps_per_traj,
                   page_steps_of(tc->ckpt_every), &ps))
    return fail(ENS_ENOSPACE,
                "pool of %zu bytes is below the fixed part (%zu) plus the "
                "reserved pages",
                tc->pool_bytes, L.fixed + 512);
  if (ps.n_static + ps.n_over > INT32_MAX)
    return fail(ENS_EINVAL, "pool holds more than 2^31 pages");
  fill_record(out, p, v, tc, L, ps);
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(setup_kernel, dim3(1), dim3(64), 0, st, out->counters,
                     out->save_times, save_times_of(v));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "setup launch");
  FwdArgs fa{};
  fa.ivp = ivp_args(p, v);
  fa.rec = view_of(out);
  fa.y_save = y_save;
  fa.lane_status = lane_status;
  fa.mesh_h = mesh_h;
  fa.mesh_S = mesh_S;
  fa.cap = cap;
  fa.slack = slack;
  fa.drift_at = drift_at;
  return launch_forward(p, mode, tc->ckpt_every > 0, fa, st, v->dense != 0);
}

// Mesh export: walk each trajectory's pages forward.  The step sizes of
// EXP_GROUP consecutive steps (a group never straddles a page: pages hold a
// multiple of 16 steps) are loaded together, so each tape line is fetched
// once while it is still cached instead of once per step.
constexpr int EXP_GROUP = 16;
static_assert(PAGE_STEPS % EXP_GROUP == 0, "a group of exported steps stays in one page");

__global__ void mesh_export_kernel(const RecView R, int64_t rec_b, int64_t h_off,
                                   double* h, int32_t* steps, int64_t cap) {
  const int64_t n = R.n;
  const int64_t tr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tr >= n) return;
  const int32_t S = R.steps[tr];
  steps[tr] = S;
  int32_t page = R.static_pages > 0 ? (int32_t)(tr * R.static_pages) : R.first_page[tr];
  const int K = R.page_steps;
  const int64_t lim = S < cap ? (int64_t)S : cap;
  for (int64_t i0 = 0; i0 < lim; i0 += EXP_GROUP) {
    const int slot0 = (int)(i0 % K);
    if (i0 > 0 && slot0 == 0) page = next_page(R, tr, page);
    const char* base = R.pages + (int64_t)page * R.page_bytes + h_off + slot0 * rec_b;
    double v[EXP_GROUP];
#pragma unroll
    for (int j = 0; j < EXP_GROUP; ++j)
      v[j] = (i0 + j < lim) ? *(const double*)(base + j * rec_b) : 0.0;
#pragma unroll
    for (int j = 0; j < EXP_GROUP; ++j)
      if (i0 + j < lim) h[(i0 + j) * n + tr] = v[j];
  }
  for (int64_t i = lim; i < cap; ++i) h[i * n + tr] = 0.0;
}

// Totals of a record: pages used, accepted steps, trials, nonzero side steps.
__global__ void stats_kernel(const RecView R, unsigned long long* out) {
  __shared__ unsigned long long red[3][BLOCK];
  const int64_t n = R.n;
  const int64_t tr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long a = 0, b = 0, c = 0;
  if (tr < n) {
    a = (unsigned)R.steps[tr];
    b = (unsigned)R.n_trial[tr];
    for (int s = 0; s < R.n_save; ++s) {
      const double dt = R.save_dt[(int64_t)s * n + tr];
      c += (dt != 0.0 && R.save_idx[(int64_t)s * n + tr] >= 0) ? 1ull : 0ull;
    }
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int off = BLOCK / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
      red[2][threadIdx.x] += red[2][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], red[0][0]);
    atomicAdd(&out[1], red[1][0]);
    atomicAdd(&out[2], red[2][0]);
  }
}

__global__ void zero3_kernel(unsigned long long* p) {
  if (threadIdx.x < 3) p[threadIdx.x] = 0ull;
}

}  // namespace

// ================================================================ C ABI ==
extern "C" {

const char* ensemble_last_error(void) { return g_err.c_str(); }

int ensemble_solve(const ens_problem* p, const ens_ivp* v, void* y_out,
                   int32_t* lane_status, void* stream) {
  SysInfo si;
  int rc;
  if ((rc = check_problem(p, &si)) != ENS_OK) return rc;
  if ((rc = check_ivp(v, true)) != ENS_OK) return rc;
  if (!y_out) return fail(ENS_EINVAL, "y_out is NULL");
  if ((rc = check_dense(p, v, MODE_SOLVE)) != ENS_OK) return rc;
  FwdArgs fa{};
  fa.ivp = ivp_args(p, v);
  fa.y_save = y_out;
  fa.lane_status = lane_status;
  return launch_forward(p, MODE_SOLVE, false, fa, (hipStream_t)stream, v->dense != 0);
}

int ensemble_record_bytes(const ens_problem* p, const ens_ivp* v,
                          int64_t steps_hint, int32_t ckpt_every,
                          size_t* bytes) {
  SysInfo si;
  int rc;
  if ((rc = check_problem(p, &si)) != ENS_OK) return rc;
  if ((rc = check_ivp(v, false)) != ENS_OK) return rc;
  if (!bytes) return fail(ENS_EINVAL, "bytes is NULL");
  if (!ckpt_ok(ckpt_every))
    return fail(ENS_EINVAL, "ckpt_every must be 0, 16, 32, 64, 128 or 256");
  if (steps_hint < 1) return fail(ENS_EINVAL, "steps_hint must be >= 1");
  const int nse = v->n_save > 0 ? v->n_save : 1;
  if ((rc = check_dense(p, v, MODE_RECORD)) != ENS_OK) return rc;
  Layout L = layout(v->n, nse, si.d, p->dtype, ckpt_every, v->dense != 0);
  const int ps = page_steps_of(ckpt_every);
  const int64_t pages_per = (steps_hint + ps - 1) / ps;
  const int64_t n_static = pages_per * v->n;
  const int64_t n_over = n_static / 8 + 64;
  *bytes = L.fixed + 512 + (size_t)n_static * L.page_bytes +
           (size_t)n_over * (L.page_bytes + 8);
  return ENS_OK;
}

int ensemble_record(const ens_problem* p, const ens_ivp* v,
                    const ens_tape_cfg* tc, ens_record* out, void* y_save,
                    int32_t* lane_status, void* stream) {
  return record_common(p, v, tc, MODE_RECORD, nullptr, nullptr, 0, out, y_save,
                       lane_status, stream);
}

int ensemble_replay_mesh(const ens_problem* p, const ens_ivp* v,
                         const ens_tape_cfg* tc, const double* h,
                         const int32_t* steps, int64_t cap, ens_record* out,
                         void* y_save, int32_t* lane_status, void* stream) {
  if (!h || !steps || cap < 1) return fail(ENS_EINVAL, "mesh h / steps / cap");
  return record_common(p, v, tc, MODE_FROZEN, h, steps, cap, out, y_save,
                       lane_status, stream);
}

int ensemble_refresh(const ens_problem* p, const ens_ivp* v, const ens_tape_cfg* tc,
                     const double* h, const int32_t* steps, int64_t cap, double slack,
                     ens_record* out, void* y_save, int32_t* lane_status, int32_t* drift_at,
                     void* stream) {
  if (!h || !steps || cap < 1) return fail(ENS_EINVAL, "mesh h / steps / cap");
  if (!(slack >= 0.0)) return fail(ENS_EINVAL, "slack must be >= 0 (got %g)", slack);
  if (p && p->system == ENS_SYS_LV_UDE)
    return fail(ENS_EUNSUPPORTED, "refresh is not built for the UDE");
  if (p && is_rtc(p->system))
    return fail(ENS_EUNSUPPORTED, "refresh is not built for registered systems");
  return record_common(p, v, tc, MODE_REFRESH, h, steps, cap, out, y_save, lane_status, stream,
                       slack, drift_at);
}

int ensemble_mesh_export(const ens_record* r, double* h, int32_t* steps,
                         int64_t cap, void* stream) {
  if (!r || !h || !steps || cap < 1) return fail(ENS_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  const bool ck = r->ckpt_every > 0;
  hipLaunchKernelGGL(mesh_export_kernel, dim3(grid_of(r->n)), dim3(BLOCK), 0, st, view_of(r),
                     ck ? (int64_t)8 : (int64_t)r->rec_bytes,
                     ck ? (int64_t)state_bytes(r->dtype, r->dim) : (int64_t)0, h, steps, cap);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? ENS_OK : hip_fail(e, "export launch");
}

// Dense output: the mesh point of each of the sweep's 2 n_save events, [2 n_save][n].
size_t events_bytes(const ens_record* r) {
  return align256((size_t)2 * r->n_save * r->n * sizeof(int32_t));
}

// The sweep's per-save cotangents for their base states, [n_save][dim][n].
size_t contrib_bytes(const ens_record* r) {
  return align256((size_t)(r->dense ? 2 : 1) * r->n_save * r->dim * r->n * elem_size(r->dtype));
}

int ensemble_adjoint_workspace_bytes(const ens_record* r, size_t* bytes) {
  if (!r || !bytes) return fail(ENS_EINVAL, "bad arguments");
  SysInfo si;
  if (!sys_info(r->system, &si)) return fail(ENS_EINVAL, "record of unknown system");
  size_t b = 0;
  if (r->params_shared) b = partials_bytes(r->system, r->n, si.np, r->dtype);
  if (r->ckpt_every > 0) b += align256((size_t)r->n * r->page_steps * rec_bytes(r->dtype, r->dim));
  if (r->system != ENS_SYS_LV_UDE) b += contrib_bytes(r);
  if (r->dense) b += events_bytes(r);
  *bytes = b;
  return ENS_OK;
}

namespace {
int adjoint_impl(const ens_problem* p, const ens_ivp* v, const ens_record* r,
                 const ens_loss* loss, void* grad_params, void* grad_y0, double* loss_out,
                 void* workspace, size_t workspace_bytes, void* stream);

// The workspace of ensemble_adjoint_static: one copy of this array on each
// GPU the library runs on.  In host code its name is only a stand-in, never a
// device address; the address comes from hipGetSymbolAddress, taken once per
// device with that device current and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[ENS_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// This device's copy of the scratch array.
int scratch_of_current_device(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(ENS_EUNSUPPORTED, "device %d: the static workspace serves devices 0..%d", dev,
                kMaxDevices - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr || ((uintptr_t)ptr & 255) != 0)
      return fail(ENS_EHIP, "the static workspace has no 256-byte aligned device address");
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return ENS_OK;
}
}  // namespace

int ensemble_adjoint(const ens_problem* p, const ens_ivp* v,
                     const ens_record* r, const ens_loss* loss,
                     void* grad_params, void* grad_y0, double* loss_out,
                     void* workspace, size_t workspace_bytes, void* stream) {
  return adjoint_impl(p, v, r, loss, grad_params, grad_y0, loss_out, workspace,
                      workspace_bytes, stream);
}

int ensemble_adjoint_static(const ens_problem* p, const ens_ivp* v,
                            const ens_record* r, const ens_loss* loss,
                            void* grad_params, void* grad_y0, double* loss_out,
                            void* stream) {
  if (!r) return fail(ENS_EINVAL, "record is NULL");
  size_t need = 0;
  int rc = ensemble_adjoint_workspace_bytes(r, &need);
  if (rc != ENS_OK) return rc;
  if (need > ENS_STATIC_WORKSPACE_BYTES)
    return fail(ENS_EINVAL,
                "this adjoint needs %zu bytes of workspace; the static workspace holds %zu "
                "(use ensemble_adjoint with a caller buffer)",
                need, (size_t)ENS_STATIC_WORKSPACE_BYTES);
  void* ws = nullptr;
  if ((rc = scratch_of_current_device(&ws)) != ENS_OK) return rc;
  return adjoint_impl(p, v, r, loss, grad_params, grad_y0, loss_out, ws,
                      (size_t)ENS_STATIC_WORKSPACE_BYTES, stream);
}

namespace {
int adjoint_impl(const ens_problem* p, const ens_ivp* v, const ens_record* r,
                 const ens_loss* loss, void* grad_params, void* grad_y0, double* loss_out,
                 void* workspace, size_t workspace_bytes, void* stream) {
  SysInfo si;
  int rc;
  if ((rc = check_problem(p, &si)) != ENS_OK) return rc;
  if ((rc = check_ivp(v, true)) != ENS_OK) return rc;
  if ((rc = check_record_matches(p, v, r)) != ENS_OK) return rc;
  if (!loss) return fail(ENS_EINVAL, "loss is NULL");
  if (loss->kind != ENS_LOSS_SUMSQ && loss->kind != ENS_LOSS_MSE_TARGET &&
      loss->kind != ENS_LOSS_COTANGENT)
    return fail(ENS_EINVAL, "unknown loss kind %d", loss->kind);
  if (loss->kind != ENS_LOSS_SUMSQ && !loss->data)
    return fail(ENS_EINVAL, "loss data is NULL");
  if (!grad_params) return fail(ENS_EINVAL, "grad_params is NULL");
  size_t need = 0;
  ensemble_adjoint_workspace_bytes(r, &need);
  if (need > 0 && (!workspace || workspace_bytes < need))
    return fail(ENS_EINVAL, "this adjoint needs a workspace of %zu bytes", need);
  if (((uintptr_t)workspace & 255) != 0)
    return fail(ENS_EINVAL, "workspace must be 256-byte aligned");
  AdjArgs aa{};
  aa.ivp = ivp_args(p, v);
  aa.rec = view_of(r);
  aa.loss_kind = loss->kind;
  aa.loss_data = loss->data;
  aa.scale = loss->scale;
  aa.grad_p = grad_params;
  aa.grad_y0 = grad_y0;
  aa.loss_out = loss_out;
  aa.workspace = workspace;
  const bool shared = p->params_shared != 0;
  const bool ckpt = r->ckpt_every > 0;
  {
    char* w = (char*)workspace;
    if (shared) w += partials_bytes(p->system, v->n, si.np, p->dtype);
    aa.scratch = ckpt ? w : nullptr;
    if (ckpt) w += align256((size_t)r->n * r->page_steps * rec_bytes(r->dtype, r->dim));
    aa.contrib = p->system != ENS_SYS_LV_UDE ? w : nullptr;
    if (p->system != ENS_SYS_LV_UDE) w += contrib_bytes(r);
    aa.events = r->dense ? (int32_t*)w : nullptr;
  }
  hipStream_t st = (hipStream_t)stream;
  if (p->system == ENS_SYS_LV_UDE) {
    const dim3 g(grid_of(v->n)), b(64 * UDE_ADJ_WAVES);
    if (ckpt)
      hipLaunchKernelGGL((ude_adjoint_kernel<true>), g, b, 0, st, aa);
    else
      hipLaunchKernelGGL((ude_adjoint_kernel<false>), g, b, 0, st, aa);
    hipLaunchKernelGGL((reduce_partials_kernel<float>), dim3(UDE_NP), dim3(BLOCK), 0, st,
                       (const float*)workspace, (int64_t)grid_of(v->n) * UDE_ADJ_WAVES, UDE_NP,
                       (float*)grad_params);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ENS_OK : hip_fail(e, "adjoint launch");
  }
  if (is_rtc(p->system)) {
    rc = rtc_launch(p->system, p->method, p->dtype, adj_expr(p->method, p->dtype, shared, ckpt),
                    grid_of(v->n), aa, st);
    if (rc != ENS_OK || !shared) return rc;
    const dim3 b(BLOCK);
    if (p->dtype == ENS_F64)
      hipLaunchKernelGGL((reduce_partials_kernel<double>), dim3(si.np), b, 0, st,
                         (const double*)workspace, (int64_t)grid_of(v->n), si.np,
                         (double*)grad_params);
    else
      hipLaunchKernelGGL((reduce_partials_kernel<float>), dim3(si.np), b, 0, st,
                         (const float*)workspace, (int64_t)grid_of(v->n), si.np,
                         (float*)grad_params);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ENS_OK : hip_fail(e, "adjoint launch");
  }
  return with_kernels(p->system, p->method, p->dtype, [&](auto s, auto m, auto t) {
    using Sys = decltype(s);
    using Tab = decltype(m);
    using T = decltype(t);
    const dim3 g(grid_of(v->n)), b(BLOCK);
    if (r->dense) {
      if (shared && ckpt)
        hipLaunchKernelGGL((erk_adjoint_kernel<Sys, Tab, T, true, true, true>), g, b, 0, st, aa);
      else if (shared)
        hipLaunchKernelGGL((erk_adjoint_kernel<Sys, Tab, T, true, false, true>), g, b, 0, st,
                           aa);
      else if (ckpt)
        hipLaunchKernelGGL((erk_adjoint_kernel<Sys, Tab, T, false, true, true>), g, b, 0, st,
                           aa);
      else
        hipLaunchKernelGGL((erk_adjoint_kernel<Sys, Tab, T, false, false, true>), g, b, 0, st,
                           aa);
    } else if (shared && ckpt)
      hipLaunchKernelGGL((erk_adjoint_kernel<Sys, Tab, T, true, true>), g, b, 0, st, aa);
    else if (shared)
      hipLaunchKernelGGL((erk_adjoint_kernel<Sys, Tab, T, true, false>), g, b, 0, st, aa);
    else if (ckpt)
      hipLaunchKernelGGL((erk_adjoint_kernel<Sys, Tab, T, false, true>), g, b, 0, st, aa);
    else
      hipLaunchKernelGGL((erk_adjoint_kernel<Sys, Tab, T, false, false>), g, b, 0, st, aa);
    if (shared)
      hipLaunchKernelGGL((reduce_partials_kernel<T>), dim3(Sys::NP), b, 0, st,
                         (const T*)workspace, (int64_t)grid_of(v->n), Sys::NP,
                         (T*)grad_params);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? ENS_OK : hip_fail(e, "adjoint launch");
  });
}
}  // namespace

int ensemble_jvp(const ens_problem* p, const ens_ivp* v, const ens_record* r,
                 const void* dy0, const void* dparams, const ens_loss* loss,
                 void* y_save_dot, double* loss_dot, void* stream) {
  SysInfo si;
  int rc;
  if ((rc = check_problem(p, &si)) != ENS_OK) return rc;
  if ((rc = check_ivp(v, true)) != ENS_OK) return rc;
  if ((rc = check_record_matches(p, v, r)) != ENS_OK) return rc;
  if (p->params_shared)
    return fail(ENS_EUNSUPPORTED, "forward mode takes per-trajectory parameters");
  if (r->dense) return fail(ENS_EUNSUPPORTED, "forward mode is not built for dense output");
  if (p->system == ENS_SYS_LV_UDE || p->system == ENS_SYS_HIRES)
    return fail(ENS_EUNSUPPORTED,
                "forward mode is built for the systems with few inputs per trajectory "
                "(not HIRES or the UDE)");
  int kind = -1;
  if (loss_dot) {
    if (!loss) return fail(ENS_EINVAL, "loss_dot needs a loss");
    if (loss->kind != ENS_LOSS_SUMSQ && loss->kind != ENS_LOSS_MSE_TARGET &&
        loss->kind != ENS_LOSS_COTANGENT)
      return fail(ENS_EINVAL, "unknown loss kind %d", loss->kind);
    if (loss->kind != ENS_LOSS_SUMSQ && !loss->data)
      return fail(ENS_EINVAL, "loss data is NULL");
    kind = loss->kind;
  }
  JvpArgs ja{};
  ja.ivp = ivp_args(p, v);
  ja.rec = view_of(r);
  ja.dy0 = dy0;
  ja.dp = dparams;
  ja.loss_kind = kind;
  ja.loss_data = kind >= 0 ? loss->data : nullptr;
  ja.scale = kind >= 0 ? loss->scale : 1.0;
  ja.ys_dot = y_save_dot;
  ja.loss_dot = loss_dot;
  const bool ck = r->ckpt_every > 0;
  ja.rec_b = ck ? (int64_t)8 : (int64_t)r->rec_bytes;
  ja.h_off = ck ? (int64_t)state_bytes(r->dtype, r->dim) : (int64_t)0;
  hipStream_t st = (hipStream_t)stream;
  if (is_rtc(p->system))
    return rtc_launch(p->system, p->method, p->dtype, jvp_expr(p->method, p->dtype),
                      grid_of(v->n), ja, st);
  return with_kernels(p->system, p->method, p->dtype, [&](auto s, auto m, auto t) {
    using Sys = decltype(s);
    using Tab = decltype(m);
    using T = decltype(t);
    if constexpr (Sys::ID == Hires::ID) {
      return fail(ENS_EUNSUPPORTED, "forward mode is not built for HIRES");
    } else {
      hipLaunchKernelGGL((jvp_kernel<Sys, Tab, T>), dim3(grid_of(v->n)), dim3(BLOCK), 0, st, ja);
      hipError_t e = hipGetLastError();
      return e == hipSuccess ? ENS_OK : hip_fail(e, "jvp launch");
    }
  });
}

extern "C" int ensemble_system_register(const char* source, int dim, int nparams,
                                        int has_jacobian, int* system) {
  if (!source || !system) return fail(ENS_EINVAL, "source and system must not be NULL");
  if (dim < 1 || dim > ENS_USER_MAX_DIM)
    return fail(ENS_EINVAL, "dim must be in [1, %d]", ENS_USER_MAX_DIM);
  if (nparams < 1 || nparams > ENS_USER_MAX_PARAMS)
    return fail(ENS_EINVAL, "nparams must be in [1, %d]", ENS_USER_MAX_PARAMS);
  if (has_jacobian && dim > 8)
    return fail(ENS_EINVAL, "a system with a Jacobian (for the Rosenbrock methods) has dim <= 8");
  const std::string src(source);
  const std::string bad = refused_construct(src);
  if (!bad.empty())
    return fail(ENS_EINVAL,
                "a registered system must be straight-line arithmetic (no data-dependent "
                "control flow): found %s",
                bad.c_str());
  auto r = std::make_unique<RtcSystem>();
  r->d = dim;
  r->np = nparams;
  r->jac = has_jacobian != 0;
  std::lock_guard<std::mutex> lk(g_rtc_mu);
  if ((int)g_rtc.size() >= ENS_USER_MAX_SYSTEMS)
    return fail(ENS_EINVAL, "at most %d systems can be registered", ENS_USER_MAX_SYSTEMS);
  const int id = ENS_SYS_USER_BASE + (int)g_rtc.size();
  r->source = "#include \"jvp.h\"\nnamespace ens_user {\nusing ens::fmaT;\n" + src +
              "\n}  // namespace ens_user\nnamespace ens {\nstruct RtcSys : ::ens_user::System {\n"
              "  static constexpr int D = " + std::to_string(dim) +
              ", NP = " + std::to_string(nparams) + ", ID = " + std::to_string(id) +
              ";\n};\n}  // namespace ens\n";
  // compile one variant now, so that a source that does not compile is
  // refused here rather than at its first launch
  const int rc = rtc_compile(*r, ENS_TSIT5, ENS_F64);
  if (rc != ENS_OK) return rc;
  if (r->jac) {
    const int rc2 = rtc_compile(*r, ENS_RODAS4, ENS_F64);
    if (rc2 != ENS_OK) return rc2;
  }
  g_rtc.push_back(std::move(r));
  *system = id;
  return ENS_OK;
}

int ensemble_record_stats(const ens_record* r, ens_stats* out, void* stream) {
  if (!r || !out) return fail(ENS_EINVAL, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  // counters[4..6] of the record receive the step totals
  unsigned long long* tot = r->counters + 4;
  hipLaunchKernelGGL(zero3_kernel, dim3(1), dim3(64), 0, st, tot);
  hipLaunchKernelGGL(stats_kernel, dim3(grid_of(r->n)), dim3(BLOCK), 0, st,
                     view_of(r), tot);
  unsigned long long host[7] = {0};
  hipError_t e = hipMemcpyAsync(host, r->counters, sizeof host,
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "stats");
  const unsigned long long n_over =
      (unsigned long long)(r->n_pages - r->n * (int64_t)r->static_pages);
  out->overflow_pages_used = (host[0] < n_over ? host[0] : n_over);  // overflow pages taken
  out->steps_accepted = host[4];
  out->trials = host[5];
  out->side_steps = host[6];
  return ENS_OK;
}

}  // extern "C"

#include "server.h"
