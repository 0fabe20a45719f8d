// Rosenbrock-Wanner (Rodas4) step for one trajectory per lane, and its
// reverse.  Paper references: the Rosenbrock replay with the mesh frozen and
// the transposed linear solve plus the Jacobian's own derivative in the
// reverse sweep (Section 3.2).
//
// Everything lives in registers with compile-time indexing: the d x d
// matrix W = I/(gamma h) - J is factored in place with partial pivoting,
// the row interchanges done by selects, and the pivot row of each column
// kept so that a right-hand side is permuted by the same interchanges in
// the same order (and in reverse order for the transposed solve).
//
// Structural zeros: a system may declare the pattern of its Jacobian
// (JAC_ROWS).  From it the factorisation's possible fill is found at
// compile time, over every pivot order partial pivoting could choose, and
// the factorisation and the solves leave out the operations on entries that
// are zero whatever the values: the rows that cannot hold a column's pivot
// are neither compared nor interchanged, rows with a zero in the pivot
// column are not eliminated, and the solves skip the zeros of L and U.
// Each skipped operation would have added or moved an exact zero, so the
// results are those of the dense factorisation (up to the sign of a zero
// that no result reads).
namespace ens {

// c ? a : b for the values the factorisation moves by selects (a separate
// function so that a scalar type made of several parts can select them part
// by part).
template <class T>
__device__ __forceinline__ T pick(bool c, T a, T b) {
  return c ? a : b;
}

// The nonzero pattern of row i of the Jacobian, bit j for column j: the
// system's JAC_ROWS if it declares one, else every column.
template <class S>
constexpr auto jac_row_of(int i, int) -> decltype(S::JAC_ROWS[0], 0u) {
  return S::JAC_ROWS[i];
}
template <class S>
constexpr unsigned jac_row_of(int, long) {
  return (1u << S::D) - 1u;
}

// What partial pivoting can make of W's pattern, step by step.  Rows are
// bitmasks of the columns that may be nonzero.  Step k: the rows at or
// below k with a possibly nonzero column-k entry are the pivot candidates;
// the interchange may give row k any candidate's pattern and a candidate
// row k's; then each row below k with a possibly nonzero column-k entry is
// eliminated, taking on the pivot row's pattern right of column k.
template <int D>
struct LuPattern {
  unsigned cand[D];    // step k: candidate pivot rows (bit i), row k included
  unsigned before[D][D];  // step k: row patterns before the interchange
  unsigned pivrow[D];  // step k: the pivot row's pattern after the interchange
  unsigned elim[D];    // step k: rows below k that are eliminated
  unsigned fin[D];     // the factors: L below the diagonal, U and 1/U_kk on and above
  int slot[D * D];     // entry -> its place among the factors' possible nonzeros (-1: zero)
  int nnz;             // number of those
};

template <class Sys>
constexpr LuPattern<Sys::D> lu_pattern() {
  constexpr int D = Sys::D;
  LuPattern<D> P{};
  unsigned M[D] = {};
  for (int i = 0; i < D; ++i) M[i] = jac_row_of<Sys>(i, 0) | (1u << i);
  for (int k = 0; k < D; ++k) {
    for (int i = 0; i < D; ++i) P.before[k][i] = M[i];
    unsigned cand = 1u << k, any = M[k];
    for (int i = k + 1; i < D; ++i)
      if ((M[i] >> k) & 1u) {
        cand |= 1u << i;
        any |= M[i];
      }
    const unsigned mk = M[k];
    for (int i = k + 1; i < D; ++i)
      if ((cand >> i) & 1u) M[i] |= mk;
    M[k] = any;
    P.cand[k] = cand;
    P.pivrow[k] = any;
    const unsigned right = any & ~((2u << k) - 1u);
    unsigned el = 0;
    for (int i = k + 1; i < D; ++i)
      if ((M[i] >> k) & 1u) {
        el |= 1u << i;
        M[i] |= right;
      }
    P.elim[k] = el;
  }
  int nz = 0;
  for (int i = 0; i < D; ++i) {
    P.fin[i] = M[i];
    for (int j = 0; j < D; ++j) P.slot[i * D + j] = ((M[i] >> j) & 1u) ? nz++ : -1;
  }
  P.nnz = nz;
  return P;
}

constexpr bool has(unsigned mask, int j) { return ((mask >> j) & 1u) != 0u; }

// W = I/(gamma h) - J(y) factored as P W = L U (unit L below the diagonal,
// U above it).  The pivot of column k is the first row i >= k with the
// largest |W_ik|; piv[k] records it.  The column is scaled by the pivot's
// reciprocal r_k = 1/U_kk (as LAPACK's getf2 does), and the diagonal keeps
// r_k, which the triangular solves multiply by: one division per pivot.
template <class Sys, class Tab, class T>
__device__ __forceinline__ void ros_factor(const T* y, const T* p, T h, T (&W)[Sys::D * Sys::D],
                                           int (&piv)[Sys::D]) {
  constexpr int D = Sys::D;
  constexpr LuPattern<D> P = lu_pattern<Sys>();
  Sys::jac(y, p, W);
  const T dg = T(1.0) / (T(Tab::GAMMA) * h);
#pragma unroll
  for (int i = 0; i < D * D; ++i) W[i] = -W[i];
#pragma unroll
  for (int i = 0; i < D; ++i) W[i * D + i] = W[i * D + i] + dg;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int pk = k;
    T best = fabs(W[k * D + k]);
#pragma unroll
    for (int i = k + 1; i < D; ++i) {
      if (!has(P.cand[k], i)) continue;  // a zero never beats |W_kk| >= 0
      const T v = fabs(W[i * D + k]);
      const bool gt = v > best;
      best = pick(gt, v, best);
      pk = gt ? i : pk;
    }
    piv[k] = pk;
#pragma unroll
    for (int i = k + 1; i < D; ++i) {
      if (!has(P.cand[k], i)) continue;
      const bool sw = (pk == i);
#pragma unroll
      for (int j = 0; j < D; ++j) {
        if (!has(P.before[k][k] | P.before[k][i], j)) continue;  // both zero
        const T a = W[k * D + j], b = W[i * D + j];
        W[k * D + j] = pick(sw, b, a);
        W[i * D + j] = pick(sw, a, b);
      }
    }
    const T r = T(1.0) / W[k * D + k];
    W[k * D + k] = r;
#pragma unroll
    for (int i = k + 1; i < D; ++i) {
      if (!has(P.elim[k], i)) continue;  // its multiplier is zero
      const T l = W[i * D + k] * r;
      W[i * D + k] = l;
#pragma unroll
      for (int j = k + 1; j < D; ++j)
        if (has(P.pivrow[k], j)) W[i * D + j] = fmaT(-l, W[k * D + j], W[i * D + j]);
    }
  }
}

// Apply the interchanges of the factorisation to v, first to last (only
// the candidate rows of each step can have been interchanged).
template <class Sys, class T>
__device__ __forceinline__ void permute_fwd(const int (&piv)[Sys::D], T* v) {
  constexpr int D = Sys::D;
  constexpr LuPattern<D> P = lu_pattern<Sys>();
#pragma unroll
  for (int k = 0; k < D; ++k) {
#pragma unroll
    for (int i = k + 1; i < D; ++i) {
      if (!has(P.cand[k], i)) continue;
      const bool sw = (piv[k] == i);
      const T a = v[k], b = v[i];
      v[k] = pick(sw, b, a);
      v[i] = pick(sw, a, b);
    }
  }
}

// Undo them (last to first): the permutation's transpose.
template <class Sys, class T>
__device__ __forceinline__ void permute_bwd(const int (&piv)[Sys::D], T* v) {
  constexpr int D = Sys::D;
  constexpr LuPattern<D> P = lu_pattern<Sys>();
#pragma unroll
  for (int k = D - 1; k >= 0; --k) {
#pragma unroll
    for (int i = k + 1; i < D; ++i) {
      if (!has(P.cand[k], i)) continue;
      const bool sw = (piv[k] == i);
      const T a = v[k], b = v[i];
      v[k] = pick(sw, b, a);
      v[i] = pick(sw, a, b);
    }
  }
}

// The factors of one lane held in LDS, only the entries that can be
// nonzero: entry e at base[slot(e) * 256 + lane] (consecutive lanes on
// consecutive words, so a wave's access is one conflict-free sweep).
// Indexing as for a register array; an entry that is always zero is never
// read.
template <class Sys, class T>
struct LdsMat {
  T* base;
  __device__ __forceinline__ T operator[](int e) const {
    constexpr LuPattern<Sys::D> P = lu_pattern<Sys>();
    return base[P.slot[e] * 256 + threadIdx.x];
  }
};

// LDS words a lane's factors take.
template <class Sys>
constexpr int lu_nnz() {
  return lu_pattern<Sys>().nnz;
}

// Before each solve from LDS: a compiler memory barrier, so that every solve
// reads the factors afresh instead of the compiler merging the reads of
// successive solves (which would keep all the factors in registers).
template <class Sys, class T>
__device__ __forceinline__ void reload_point(const LdsMat<Sys, T>&) {
  __asm__ __volatile__("" ::: "memory");
}
template <class A>
__device__ __forceinline__ void reload_point(const A&) {}


// After a solve from LDS: its result is taken as new (an optimisation
// barrier per component), which keeps the compiler from interleaving the
// arithmetic of successive solves; without it the 8 x 8 reverse step holds
// too much at once and spills about 2 KB a lane.
template <class Sys, class T>
__device__ __forceinline__ void solved_point(const LdsMat<Sys, T>&, T* x) {
#pragma unroll
  for (int c = 0; c < Sys::D; ++c) __asm__ __volatile__("" : "+v"(x[c]));
}
template <class Sys, class T, class A>
__device__ __forceinline__ void solved_point(const A&, T*) {}

// An optimisation barrier on a value: the compiler must treat x as changed,
// so expressions of it formed afterwards are computed afresh instead of
// reusing (and keeping alive) equal ones formed before.  No instruction.
template <class T>
__device__ __forceinline__ void opaque(T& x) {
  __asm__ __volatile__("" : "+v"(x));
}

// Copy register factors into a lane's LDS slots (the entries that can be
// nonzero).  The empty asm with a memory clobber keeps the compiler from
// forwarding the stored values to the later reads, which would keep the
// factors live in registers after all.
template <class Sys, class T>
__device__ __forceinline__ void put_lds(const T (&W)[Sys::D * Sys::D], const LdsMat<Sys, T>& M) {
  constexpr int D = Sys::D;
  constexpr LuPattern<D> P = lu_pattern<Sys>();
#pragma unroll
  for (int e = 0; e < D * D; ++e)
    if (P.slot[e] >= 0) M.base[P.slot[e] * 256 + threadIdx.x] = W[e];
  __asm__ __volatile__("" ::: "memory");
}

// x = W^{-1} b in place: L z = P b forward, then U x = z backward (the
// diagonal holds 1/U_kk); the zeros of L and U skipped.
template <class Sys, class T, class Mat>
__device__ __forceinline__ void lu_solve(const Mat& W, const int (&piv)[Sys::D], T* x) {
  constexpr int D = Sys::D;
  constexpr LuPattern<D> P = lu_pattern<Sys>();
  reload_point(W);
  permute_fwd<Sys, T>(piv, x);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T acc = x[i];
#pragma unroll
    for (int j = 0; j < i; ++j)
      if (has(P.fin[i], j)) acc = fmaT(-W[i * D + j], x[j], acc);
    x[i] = acc;
  }
#pragma unroll
  for (int i = D - 1; i >= 0; --i) {
    T acc = x[i];
#pragma unroll
    for (int j = i + 1; j < D; ++j)
      if (has(P.fin[i], j)) acc = fmaT(-W[i * D + j], x[j], acc);
    x[i] = acc * W[i * D + i];
  }
}

// z = W^{-T} b in place: U^T v = b forward, L^T w = v backward, z = P^T w.
// W: the factors as a register array or an LdsMat.
template <class Sys, class T, class Mat>
__device__ __forceinline__ void lu_solve_t(const Mat& W, const int (&piv)[Sys::D], T* z) {
  constexpr int D = Sys::D;
  constexpr LuPattern<D> P = lu_pattern<Sys>();
  reload_point(W);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    T acc = z[i];
#pragma unroll
    for (int j = 0; j < i; ++j)
      if (has(P.fin[j], i)) acc = fmaT(-W[j * D + i], z[j], acc);
    z[i] = acc * W[i * D + i];
  }
#pragma unroll
  for (int i = D - 1; i >= 0; --i) {
    T acc = z[i];
#pragma unroll
    for (int j = i + 1; j < D; ++j)
      if (has(P.fin[j], i)) acc = fmaT(-W[j * D + i], z[j], acc);
    z[i] = acc;
  }
  permute_bwd<Sys, T>(piv, z);
}

// Stage input Y_i = y + sum_{j<i} A_ij u_j (index order, first term a
// product, the rest fmas).
template <class Tab, int D, class T>
__device__ __forceinline__ void ros_input(int i, const T* y, const T (&u)[Tab::S][D], T* Yi) {
#pragma unroll
  for (int c = 0; c < D; ++c) {
    T acc = T(0);
    bool first = true;
#pragma unroll
    for (int j = 0; j < Tab::S; ++j) {
      if (j < i && Tab::A[i][j] != 0.0) {
        acc = first ? cmul(Tab::A[i][j], u[j][c]) : cfma(Tab::A[i][j], u[j][c], acc);
        first = false;
      }
    }
    Yi[c] = first ? y[c] : y[c] + acc;
  }
}

// The increments u_1..u_NSC of one step from y with step h (h != 0), the
// factors left in W/piv for the reverse, and y_new: Y_s + u_s, or the last
// stage input Y_s (NEW_AT_INPUT).  NSC = S forms every stage (a trial step
// needs the last for its error estimate); NSC = SU only those that enter
// y_new (a replay).  W: the factors as a register array or an LdsMat.
template <class Sys, class Tab, class T, class Mat, int NSC = Tab::S>
__device__ __forceinline__ void ros_stages(const T* y, const T* p, T h, const Mat& W,
                                           const int (&piv)[Sys::D], T (&u)[Tab::S][Sys::D],
                                           T* ynew) {
  constexpr int D = Sys::D, NS = Tab::S;
  static_assert(NSC == NS || (NSC == Tab::SU && Tab::NEW_AT_INPUT),
                "a step that stops short of the last stage needs y_new at its input");
  const T hinv = T(1.0) / h;
  T Yi[D];
#pragma unroll
  for (int i = 0; i < NSC; ++i) {
    ros_input<Tab, D, T>(i, y, u, Yi);
    T F[D];
    Sys::rhs(Yi, p, F);
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T acc = T(0);
      bool first = true;
#pragma unroll
      for (int j = 0; j < i; ++j) {
        if (Tab::C[i][j] != 0.0) {
          acc = first ? cmul(Tab::C[i][j], u[j][c]) : cfma(Tab::C[i][j], u[j][c], acc);
          first = false;
        }
      }
      u[i][c] = first ? F[c] : fmah(acc, hinv, F[c]);
    }
    lu_solve<Sys, T, Mat>(W, piv, u[i]);
    solved_point<Sys, T>(W, u[i]);
  }
  if constexpr (Tab::NEW_AT_INPUT) {
    ros_input<Tab, D, T>(NS - 1, y, u, ynew);
  } else {
#pragma unroll
    for (int c = 0; c < D; ++c) ynew[c] = Yi[c] + u[NS - 1][c];
  }
}

template <class Sys, class Tab, class T, int NSC = Tab::S>
__device__ __forceinline__ void ros_step(const T* y, const T* p, T h, T (&W)[Sys::D * Sys::D],
                                         int (&piv)[Sys::D], T (&u)[Tab::S][Sys::D], T* ynew) {
  ros_factor<Sys, Tab, T>(y, p, h, W, piv);
  ros_stages<Sys, Tab, T, T[Sys::D * Sys::D], NSC>(y, p, h, W, piv, u, ynew);
}

// Error estimate e = sum_j E_j u_j (Rodas4: u_6 itself).
template <class Tab, int D, class T>
__device__ __forceinline__ void ros_errvec(const T (&u)[Tab::S][D], T* e) {
#pragma unroll
  for (int c = 0; c < D; ++c) {
    T acc = T(0);
    bool first = true;
#pragma unroll
    for (int j = 0; j < Tab::S; ++j) {
      if (Tab::E[j] != 0.0) {
        acc = first ? cmul(Tab::E[j], u[j][c]) : cfma(Tab::E[j], u[j][c], acc);
        first = false;
      }
    }
    e[c] = acc;
  }
}

// The same step with the factors moved to this lane's LDS slots right after
// the factorisation (the same values, so the same results), for systems
// whose factors crowd the registers of the reverse sweep.
template <class Sys, class Tab, class T, int NSC = Tab::S>
__device__ __forceinline__ void ros_step_lds(const T* y, const T* p, T h,
                                             const LdsMat<Sys, T>& Wl,
                                             int (&piv)[Sys::D], T (&u)[Tab::S][Sys::D],
                                             T* ynew) {
  T W[Sys::D * Sys::D];
  ros_factor<Sys, Tab, T>(y, p, h, W, piv);
  put_lds<Sys, T>(W, Wl);
  ros_stages<Sys, Tab, T, LdsMat<Sys, T>, NSC>(y, p, h, Wl, piv, u, ynew);
}

template <class Tab>
constexpr bool m_nonzero_below_su() {
  for (int i = 0; i < Tab::SU; ++i)
    if (Tab::M[i] == 0.0) return false;
  return true;
}

// Reverse of one step (W, piv, u from ros_step at the same y, h; W as a
// register array or an LdsMat): with the
// output cotangent w, lam_in = d(y_new)/dy^T w and gp += d(y_new)/dp^T w.
//   ubar_i = M_i w + sum_{l>i} (A_li Ybar_l + C_li rbar_l / h)   (l from s down)
//   rbar_i = W^{-T} ubar_i,  Ybar_i = f_y(Y_i)^T rbar_i,  gp += f_p(Y_i)^T rbar_i
//   lam_in = w + sum_i Ybar_i + d/dy sum_i rbar_i^T J(y) u_i,
// the last term (and its p part, into gp) from each stage in turn.  Stage
// cotangents are pushed into running sums as they are formed.  Only the SU
// stages that enter y_new are reversed (a stage that serves the error
// estimate alone has a zero cotangent).
template <class Sys, class Tab, class T, class Mat>
__device__ __forceinline__ void ros_step_vjp(const T* y, const T* p, T h, const Mat& W,
                                             const int (&piv)[Sys::D],
                                             const T (&u)[Tab::S][Sys::D], const T* w,
                                             T* lam_in, T* gp) {
  constexpr int D = Sys::D, NS = Tab::SU;
  static_assert(m_nonzero_below_su<Tab>(), "every stage sum starts with its M term");
  const T hinv = T(1.0) / h;
  T ub[NS][D], gJ[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    lam_in[c] = w[c];
    gJ[c] = T(0);
  }
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int c = 0; c < D; ++c) ub[i][c] = T(Tab::M[i]) * w[c];
#pragma unroll
  for (int i = NS - 1; i >= 0; --i) {
    T rb[D], tb[D], Yi[D], Yb[D];
#pragma unroll
    for (int c = 0; c < D; ++c) rb[c] = ub[i][c];
    lu_solve_t<Sys, T, Mat>(W, piv, rb);
    solved_point<Sys, T>(W, rb);
#pragma unroll
    for (int c = 0; c < D; ++c) tb[c] = hinv * rb[c];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      T acc = T(0);
      bool first = true;
#pragma unroll
      for (int j = 0; j < i; ++j) {
        if (Tab::A[i][j] != 0.0) {
          acc = first ? T(Tab::A[i][j]) * u[j][c] : fmaT(T(Tab::A[i][j]), u[j][c], acc);
          first = false;
        }
      }
      Yi[c] = first ? y[c] : y[c] + acc;
    }
    Sys::vjp(Yi, p, rb, Yb, gp);
#pragma unroll
    for (int c = 0; c < D; ++c) lam_in[c] = lam_in[c] + Yb[c];
    Sys::jac_vjp(y, p, rb, u[i], gJ, gp);
#pragma unroll
    for (int j = 0; j < i; ++j) {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        if (Tab::A[i][j] != 0.0) ub[j][c] = fmaT(T(Tab::A[i][j]), Yb[c], ub[j][c]);
        if (Tab::C[i][j] != 0.0) ub[j][c] = fmaT(T(Tab::C[i][j]), tb[c], ub[j][c]);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < D; ++c) lam_in[c] = lam_in[c] + gJ[c];
}

// Mean square (the RMS norm squared) of the scaled error estimate against
// atol + rtol max(|y|, |y_new|); the reciprocal of each scale as the
// explicit pairs' recip (the hardware estimate and one Newton step).
template <int D, class T>
__device__ __forceinline__ double ros_ms(const T* y, const T* ynew, const T* e, double rtol,
                                         double atol) {
  double ss = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const double sc = fmaT(rtol, fmax(fabs((double)y[c]), fabs((double)ynew[c])), atol);
    const double q0 = __builtin_amdgcn_rcp(sc);
    const double q = fmaT(q0, fmaT(-sc, q0, 1.0), q0);
    const double r = (double)e[c] * q;
    ss = c == 0 ? r * r : fmaT(r, r, ss);
  }
  return ss * (1.0 / (double)D);
}

}  // namespace ens
