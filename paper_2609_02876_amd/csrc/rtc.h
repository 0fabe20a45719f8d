// Systems registered at run time: a right-hand side, its vector-Jacobian
// product and, for Rodas4, its Jacobian and the derivative of u^T J v, given
// as source text and compiled with hipRTC against the library's own kernel
// headers.  A registered system runs the same record, reverse-sweep and
// forward-mode kernels as a built-in one (the paper's user-supplied "RHS and
// its VJP", Section 3.4; its translation of a user function into the fused
// kernels refuses data-dependent control flow, Section 3.3, and so does this).
//
// Host code only: included by ensode.hip inside its internal namespace,
// after the launch helpers (ensode.hip includes hiprtc.h and the standard
// headers this needs).
#pragma once

#include "_rtc_sources.inc"

struct RtcSystem {
  std::string source;  // the composed translation unit
  int d = 0, np = 0;
  bool jac = false;
  std::map<int, std::vector<char>> code;                          // per (method, dtype)
  std::map<int, std::map<std::string, std::string>> lowered;      // name expression -> symbol
  std::map<std::pair<int, int>, hipModule_t> module;              // per (key, device)
  std::map<std::pair<std::string, int>, hipFunction_t> function;  // per (expression, device)
};

std::mutex g_rtc_mu;
std::vector<std::unique_ptr<RtcSystem>> g_rtc;

bool is_rtc(int sys) {
  std::lock_guard<std::mutex> lk(g_rtc_mu);
  return sys >= ENS_SYS_USER_BASE && sys < ENS_SYS_USER_BASE + (int)g_rtc.size();
}

bool rtc_info(int sys, int* d, int* np, bool* jac) {
  std::lock_guard<std::mutex> lk(g_rtc_mu);
  if (sys < ENS_SYS_USER_BASE || sys >= ENS_SYS_USER_BASE + (int)g_rtc.size()) return false;
  const RtcSystem& r = *g_rtc[sys - ENS_SYS_USER_BASE];
  *d = r.d;
  *np = r.np;
  *jac = r.jac;
  return true;
}

// The first construct of the source that is not plain arithmetic on the
// arguments (control flow, preprocessor, inline assembly, compiler
// intrinsics, shared memory, synchronisation, atomics, thread or block
// indices), or "" if there is none.  Comments and literals are skipped.
// Identifiers beginning with two underscores are reserved to the compiler
// (its intrinsics among them) and refused, except the two qualifiers a
// device function declaration needs.
std::string refused_construct(const std::string& s) {
  static const char* const kWords[] = {
      "if", "else", "for", "while", "do", "switch", "case", "goto", "break", "continue",
      "asm", "volatile", "extern", "threadIdx", "blockIdx", "blockDim", "gridDim",
      "warpSize"};
  static const char* const kAllowed[] = {"__device__", "__forceinline__"};
  const size_t n = s.size();
  size_t i = 0;
  bool line_start = true;
  while (i < n) {
    const char c = s[i];
    if (c == '/' && i + 1 < n && s[i + 1] == '/') {
      while (i < n && s[i] != '\n') ++i;
      continue;
    }
    if (c == '/' && i + 1 < n && s[i + 1] == '*') {
      const size_t e = s.find("*/", i + 2);
      i = e == std::string::npos ? n : e + 2;
      continue;
    }
    if (c == '"' || c == '\'') {
      ++i;
      while (i < n && s[i] != c) i += (s[i] == '\\') ? 2 : 1;
      ++i;
      continue;
    }
    if (c == '\n') {
      line_start = true;
      ++i;
      continue;
    }
    if (c == ' ' || c == '\t' || c == '\r') {
      ++i;
      continue;
    }
    if (c == '#' && line_start) return "a preprocessor directive";
    line_start = false;
    if (c == '?') return "'?'";
    if ((c == '&' || c == '|') && i + 1 < n && s[i + 1] == c) return std::string(2, c);
    if (std::isalpha((unsigned char)c) || c == '_') {
      size_t j = i;
      while (j < n && (std::isalnum((unsigned char)s[j]) || s[j] == '_')) ++j;
      const std::string w = s.substr(i, j - i);
      for (const char* k : kWords)
        if (w == k) return "'" + w + "'";
      if (w.compare(0, 2, "__") == 0 || w.compare(0, 6, "atomic") == 0) {
        bool ok = false;
        for (const char* k : kAllowed) ok = ok || w == k;
        if (!ok) return "'" + w + "'";
      }
      i = j;
      continue;
    }
    ++i;
  }
  return "";
}

const char* tab_name(int method) {
  return method == ENS_TSIT5   ? "ens::Tsit5"
         : method == ENS_VERN7 ? "ens::Vern7"
         : method == ENS_ROS23 ? "ens::Ros23"
                               : "ens::Rodas4";
}

// Name expressions of every kernel a registered system uses with one method
// and element type.
std::vector<std::string> rtc_exprs(int method, int dtype) {
  const std::string t = dtype == ENS_F64 ? "double" : "float";
  const std::string pre = std::string("ens::RtcSys, ") + tab_name(method) + ", " + t;
  std::vector<std::string> v;
  v.push_back("ens::erk_forward_kernel<" + pre + ", 0, false>");
  for (int mode = 1; mode <= 2; ++mode)
    for (const char* ck : {"false", "true"})
      v.push_back("ens::erk_forward_kernel<" + pre + ", " + std::to_string(mode) + ", " + ck +
                  ">");
  for (const char* sh : {"false", "true"})
    for (const char* ck : {"false", "true"})
      v.push_back("ens::erk_adjoint_kernel<" + pre + ", " + sh + ", " + ck + ">");
  v.push_back("ens::jvp_kernel<" + pre + ">");
  if (method == ENS_TSIT5 || method == ENS_VERN7) {
    // the explicit pairs' full-tape record: the loop, then the save states
    v.push_back("ens::erk_record_deferred_kernel<" + pre + ">");
    v.push_back("ens::erk_saves_kernel<" + pre + ">");
  }
  return v;
}

std::string fwd_expr(int method, int dtype, int mode, bool ckpt) {
  return std::string("ens::erk_forward_kernel<ens::RtcSys, ") + tab_name(method) + ", " +
         (dtype == ENS_F64 ? "double" : "float") + ", " + std::to_string(mode) + ", " +
         (ckpt ? "true" : "false") + ">";
}
std::string adj_expr(int method, int dtype, bool shared, bool ckpt) {
  return std::string("ens::erk_adjoint_kernel<ens::RtcSys, ") + tab_name(method) + ", " +
         (dtype == ENS_F64 ? "double" : "float") + ", " + (shared ? "true" : "false") + ", " +
         (ckpt ? "true" : "false") + ">";
}
std::string deferred_expr(int method, int dtype) {
  return std::string("ens::erk_record_deferred_kernel<ens::RtcSys, ") + tab_name(method) + ", " +
         (dtype == ENS_F64 ? "double" : "float") + ">";
}
std::string saves_expr(int method, int dtype) {
  return std::string("ens::erk_saves_kernel<ens::RtcSys, ") + tab_name(method) + ", " +
         (dtype == ENS_F64 ? "double" : "float") + ">";
}
std::string jvp_expr(int method, int dtype) {
  return std::string("ens::jvp_kernel<ens::RtcSys, ") + tab_name(method) + ", " +
         (dtype == ENS_F64 ? "double" : "float") + ">";
}

// Compile the kernels of one (method, dtype) for a registered system (the
// caller holds g_rtc_mu).
int rtc_compile(RtcSystem& r, int method, int dtype) {
  const int key = method * 16 + dtype;
  if (r.code.count(key)) return ENS_OK;
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, r.source.c_str(), "registered_system.hip", kRtcHeaders,
                          kRtcHeaderBodies, kRtcHeaderNames) != HIPRTC_SUCCESS)
    return fail(ENS_EHIP, "hiprtcCreateProgram failed");
  const std::vector<std::string> exprs = rtc_exprs(method, dtype);
  for (const std::string& e : exprs) hiprtcAddNameExpression(prog, e.c_str());
  // the flags of the library's own build (no contraction of products and
  // sums the source did not fuse; no packed FP32 instructions)
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                        "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops"};
  const hiprtcResult cr = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
  if (cr != HIPRTC_SUCCESS) {
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    std::string log(ls + 1, '\0');
    hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    if (log.size() > 1500) log = log.substr(0, 1500) + " ...";
    return fail(ENS_EINVAL, "the registered system does not compile: %s", log.c_str());
  }
  std::map<std::string, std::string> low;
  for (const std::string& e : exprs) {
    const char* name = nullptr;
    if (hiprtcGetLoweredName(prog, e.c_str(), &name) != HIPRTC_SUCCESS || !name) {
      hiprtcDestroyProgram(&prog);
      return fail(ENS_EHIP, "no symbol for %s", e.c_str());
    }
    low[e] = name;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  std::vector<char> code(cs);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  r.code[key] = std::move(code);
  r.lowered[key] = std::move(low);
  return ENS_OK;
}

// The kernel `expr` of a registered system on the current device, compiling
// and loading on first use.
int rtc_function(int sys, int method, int dtype, const std::string& expr, hipFunction_t* out) {
  std::lock_guard<std::mutex> lk(g_rtc_mu);
  RtcSystem& r = *g_rtc[sys - ENS_SYS_USER_BASE];
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  auto it = r.function.find({expr, dev});
  if (it != r.function.end()) {
    *out = it->second;
    return ENS_OK;
  }
  const int key = method * 16 + dtype;
  int rc = rtc_compile(r, method, dtype);
  if (rc != ENS_OK) return rc;
  auto mk = std::make_pair(key, dev);
  if (!r.module.count(mk)) {
    hipModule_t m;
    e = hipModuleLoadData(&m, r.code[key].data());
    if (e != hipSuccess) return hip_fail(e, "loading a registered system's kernels");
    r.module[mk] = m;
  }
  hipFunction_t f;
  e = hipModuleGetFunction(&f, r.module[mk], r.lowered[key].at(expr).c_str());
  if (e != hipSuccess) return hip_fail(e, "hipModuleGetFunction");
  r.function[{expr, dev}] = f;
  *out = f;
  return ENS_OK;
}

// Launch one kernel of a registered system: BLOCK lanes per block, the
// argument struct passed by value.
template <class Args>
int rtc_launch(int sys, int method, int dtype, const std::string& expr, unsigned grid,
               const Args& args, hipStream_t st) {
  hipFunction_t f;
  const int rc = rtc_function(sys, method, dtype, expr, &f);
  if (rc != ENS_OK) return rc;
  void* params[] = {const_cast<Args*>(&args)};
  const hipError_t e =
      hipModuleLaunchKernel(f, grid, 1, 1, BLOCK, 1, 1, 0, st, params, nullptr);
  return e == hipSuccess ? ENS_OK : hip_fail(e, "launch of a registered system's kernel");
}

