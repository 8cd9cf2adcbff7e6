// Pointwise algebra of the implicit step on one grid level: the rows of the
// nonlinear system N(g) = S (App. G, typos fixed from Eqs. discrete_a-d), the
// source S, and the point-block Gauss-Seidel update (App. G smoother with its
// damping).  Every function works on one node (i, j) of a periodic n x n
// level, n a power of two, fields row-major with x fastest.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hfz {

// PFC and CDFT: the hydrodynamic step (App. G).  GPFC and GCDFT: the
// gradient-flow variant of the same convex splitting (Thm. thm_grad).  WPFC:
// the hydrodynamic PFC step in a channel, periodic in x with walls in y
// (Sec. 6, sheared-nanocrystal run).
enum { PFC = 0, CDFT = 1, GPFC = 2, GCDFT = 3, WPFC = 4 };

__host__ __device__ constexpr bool gradflow(int m) { return m == GPFC || m == GCDFT; }
__host__ __device__ constexpr bool cdft_like(int m) { return m == CDFT || m == GCDFT; }
__host__ __device__ constexpr bool walls(int m) { return m == WPFC; }
// The model whose rows and block solve a model uses.
__host__ __device__ constexpr int algebra(int m) { return m == WPFC ? PFC : m; }

// Unknowns per node: PFC (rho, u, v, mu, kappa), CDFT (rho, u, v), GPFC
// (rho, mu, kappa), GCDFT (rho, mu).
template <int MODEL> struct NC {
  static constexpr int value =
      algebra(MODEL) == PFC ? 5 : (MODEL == CDFT ? 3 : (MODEL == GPFC ? 3 : 2));
};
// Base fields the correction form is taken about: (rho, u, v), or rho alone
// in the gradient flow (its only nonlinearities are in rho).
template <int MODEL> struct NBase { static constexpr int value = gradflow(MODEL) ? 1 : 3; };
// Frozen-coefficient arrays the rows read (rho^k, omega^k); the gradient-flow
// rows have constant coefficients.
template <int MODEL> struct NCoef { static constexpr int value = gradflow(MODEL) ? 0 : 2; };

__device__ __forceinline__ double flog(double x) { return log(x); }
__device__ __forceinline__ float flog(float x) { return logf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fsqrt(float x) { return sqrtf(x); }

// Physical constants of the step, in the arithmetic type T, and the device
// stop flag of the V-cycle loop (null: none).  A V-cycle kernel whose flag is
// set returns at once: the cycles the host enqueued past convergence do
// nothing.
template <typename T> struct Phys {
  T s, gamma, sigma, alpha, ce, delta, w;
  T ub, ut;  // channel: u on the walls j = 0 and j = n
  const int* halt;
};

__device__ __forceinline__ bool halted(const int* flag) { return flag != nullptr && *flag != 0; }

// The same flag read as a vector load (an agent-scope relaxed atomic load,
// which the compiler never turns into a scalar one), for kernels that issue it
// with their first data loads and test it (stop_set) before their first
// store.  halted() reads it with a scalar load at the kernel's start, and the
// scalar loads are waited for together, so the kernel-argument loads that
// address the data would wait for the flag: one more memory round trip ahead
// of every load of the kernel.
// (A missing flag reads a zero of its own: a select, not a branch, so the
// kernel-argument loads are not split in two rounds either.)
static __device__ int kNoStopFlag = 0;
__device__ __forceinline__ int stop_flag(const int* flag) {
  return __hip_atomic_load(flag != nullptr ? flag : &kNoStopFlag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool stop_set(int v) { return __builtin_amdgcn_readfirstlane(v) != 0; }

// XCD-contiguous numbering of a 2D grid of workgroups (blockIdx.z, if used,
// numbers independent slices): the workgroups of a launch are dealt to the 8
// XCDs in turn, and block tb = (b % 8) (nb / 8) + b / 8 for workgroup b of a
// slice of nb gives each XCD a contiguous band of block rows, whose shared
// halos are then read through one L2.  Returns tb (a bijection of the slice's
// blocks; the index of the block's partial sums) and its coordinates.
__device__ __forceinline__ int xcd_block(int& bx, int& by) {
  const int gx = (int)gridDim.x, nb = gx * (int)gridDim.y;
  const int bid = (int)blockIdx.y * gx + (int)blockIdx.x;
  const int tb = (nb & 7) ? bid : (bid & 7) * (nb >> 3) + (bid >> 3);
  bx = tb % gx;
  by = tb / gx;
  return tb;
}

// Stencil coefficients of one level: s/(4h), s/(2h), 1/h^2.
template <typename T> struct Coef {
  T c4, c2, ih2;
};

// One level of the hierarchy.
template <typename T> struct Lvl {
  T* g[5];    // iterate
  T* f[5];    // right-hand side (level 0: the source S)
  T* g0[5];   // restricted iterate R g (coarse levels)
  T* d[5];    // scratch: residual f - N(g) before restriction
  T* gb[5];   // second buffer of the iterate (double-buffered tiled sweeps)
  T* rk;      // frozen rho^k
  T* om;      // frozen omega^k
  T* bg[3];   // correction form only: base state (rho, u, v) the correction is taken about
  int n;      // grid size n_l (x; and y for the periodic models)
  int ny;     // rows stored: n_l, or n_l + 1 in a channel (node rows 0..n_l, the walls at 0 and n_l)
  int lg;     // log2 n_l (row stride 2^lg)
  T h;        // spacing h_l
  Coef<T> k;  // stencil coefficients of this level
};

// Address-space views.  A pointer loaded from memory (a level descriptor in a
// device array or in LDS) is generic to the compiler, so its loads and stores
// become FLAT instructions, which wait on both the vector-memory and the LDS
// counters.  These views tell the compiler where the data lives so that it
// emits global_* / ds_* instructions: global through an integer round trip
// into an address_space(1) pointer, LDS through an assumption the address
// space inference uses.  Only apply them to pointers that do point there.
// (The host pass of the single-source compile sees only the plain pointer.)
template <typename T> __device__ __forceinline__ T* as_global(T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return (T*)((__attribute__((address_space(1))) T*)(uintptr_t)p);
#else
  return p;
#endif
}
template <typename T> __device__ __forceinline__ T* as_lds(T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_assume(__builtin_amdgcn_is_shared((const void*)p));
#endif
  return p;
}

// A level whose arrays are all in global memory (descriptor loaded from a
// device array); null pointers stay null.
template <typename T> __device__ __forceinline__ Lvl<T> lvl_global(const Lvl<T>& s) {
  Lvl<T> L = s;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    L.g[c] = as_global(s.g[c]);
    L.f[c] = as_global(s.f[c]);
    L.g0[c] = as_global(s.g0[c]);
    L.d[c] = as_global(s.d[c]);
    L.gb[c] = as_global(s.gb[c]);
  }
  L.rk = as_global(s.rk);
  L.om = as_global(s.om);
#pragma unroll
  for (int c = 0; c < 3; ++c) L.bg[c] = as_global(s.bg[c]);
  return L;
}

// Neighbour offsets of node (i, j).
struct Nbr {
  int p, e, w, n, s;
};

__device__ __forceinline__ Nbr nbr(int i, int j, int n, int lg) {
  const int m = n - 1;
  Nbr q;
  const int row = j << lg;
  q.p = row + i;
  q.e = row + ((i + 1) & m);
  q.w = row + ((i - 1) & m);
  q.n = (((j + 1) & m) << lg) + i;
  q.s = (((j - 1) & m) << lg) + i;
  return q;
}

// Neighbours for the model: in a channel y does not wrap (j an interior row,
// 1 <= j <= n - 1, whose neighbours are rows of the (n + 1)-row array).
template <int MODEL> __device__ __forceinline__ Nbr nbr_of(int i, int j, int n, int lg) {
  if constexpr (walls(MODEL)) {
    const int m = n - 1;
    Nbr q;
    const int row = j << lg;
    q.p = row + i;
    q.e = row + ((i + 1) & m);
    q.w = row + ((i - 1) & m);
    q.n = q.p + (1 << lg);
    q.s = q.p - (1 << lg);
    return q;
  } else {
    return nbr(i, j, n, lg);
  }
}

// Channel wall rows: u = u_wall, v = 0 (fixed); rho, mu, kappa copy the
// adjacent interior row (no flux), refreshed whenever that row changes.
__host__ __device__ constexpr bool wall_copied(int c) { return c == 0 || c == 3 || c == 4; }

// M = the part of mu^{k+1} carried by the unknowns: mu (PFC) or
// ln rho + 2 c_e rho (CDFT, Lemma CDFT_ineq).
template <int MODEL, typename T>
__device__ __forceinline__ T potential(const T* const* g, int q, const Phys<T>& P) {
  if constexpr (MODEL == PFC) {
    return g[3][q];
  } else {
    const T r = g[0][q];
    return flog(r) + T(2) * P.ce * r;
  }
}

// ---------------------------------------------------------------------------
// Gradient-flow variant (Thm. thm_grad, Eq. gradient_scheme): rho^{k+1} -
// rho^k = s Delta_h (dF_c[rho^{k+1}] - dF_e[rho^k]) with the discrete
// gradients of Sec. 5.2 / 5.3, written as N(g) = S with mu (and for PFC
// kappa = Delta_h rho) as unknowns:
//   N1 = rho - s Delta_h mu                              S1 = rho^k
//   GPFC:  N2 = mu - phi^3/3 - alpha phi - Delta_h kappa, S2 = 2 Delta_h rho^k
//          N3 = kappa - Delta_h rho,                      S3 = 0
//   GCDFT: N2 = mu - ln rho - 2 c_e rho,   S2 = -(J*rho^k + 2 c_e rho^k)
// The smoother solves the node's block exactly with the neighbours held and
// the nonlinearity linearised about the current iterate (the App. G
// treatment of the cubic), then damps like App. G; GCDFT projects rho^.
// With c = 1/h^2 and sums over the four neighbours the block is
//   rho + 4 s c mu = S1 + s c sum(mu)                                =: b1
//   GPFC:  mu - A rho + 4 c kappa = S2 - 3A/2 - (2/3) phi_l^3 + c sum(kappa) =: b2,
//          A = alpha + phi_l^2;   kappa + 4 c rho = S3 + c sum(rho)  =: b3
//   GCDFT: mu - B rho = S2 + ln rho_l - 1 =: b2,  B = 1/rho_l + 2 c_e
// so rho^ = (b1 - 4sc(b2 - 4c b3)) / (1 + 4sc(A + 16c^2)), kappa^ = b3 - 4c rho^,
// mu^ = b2 + A rho^ - 4c kappa^ (GPFC); rho^ = (b1 - 4sc b2)/(1 + 4sc B),
// projected, mu^ = b2 + B rho^ (GCDFT).

template <typename T> __device__ __forceinline__ T nsum(const T* f, const Nbr& q) {
  return f[q.e] + f[q.w] + f[q.n] + f[q.s];
}

template <int MODEL, typename T>
__device__ __forceinline__ void rows_gf(const T* const* g, const Nbr& q, const Coef<T>& K, const Phys<T>& P,
                                        T* out) {
  const T ih2 = K.ih2;
  const T* rho = g[0];
  const T* mu = g[1];
  const T rP = rho[q.p], mP = mu[q.p];
  out[0] = rP - P.s * ((nsum(mu, q) - T(4) * mP) * ih2);
  if constexpr (MODEL == GPFC) {
    const T* ka = g[2];
    const T phi = rP - T(1.5);
    const T lapk = (nsum(ka, q) - T(4) * ka[q.p]) * ih2;
    const T lapr = (nsum(rho, q) - T(4) * rP) * ih2;
    out[1] = mP - phi * phi * phi * T(1.0 / 3.0) - P.alpha * phi - lapk;
    out[2] = ka[q.p] - lapr;
  } else {
    out[1] = mP - flog(rP) - T(2) * P.ce * rP;
  }
}

template <int MODEL, typename T>
__device__ __forceinline__ void block_update_gf(const T* const* g, const T* const* f, const Nbr& q, int pf,
                                                const Coef<T>& K, const Phys<T>& P, T* out) {
  const T c = K.ih2, sc = P.s * c;
  const T* rho = g[0];
  const T* mu = g[1];
  const T rl = rho[q.p];
  const T b1 = f[0][pf] + sc * nsum(mu, q);
  const T w = P.w, w1 = T(1) - P.w;
  if constexpr (MODEL == GPFC) {
    const T* ka = g[2];
    const T pl = rl - T(1.5);
    const T A = P.alpha + pl * pl;
    const T b2 = f[1][pf] - T(1.5) * A - (T(2) / T(3)) * pl * pl * pl + c * nsum(ka, q);
    const T b3 = f[2][pf] + c * nsum(rho, q);
    const T rh = (b1 - T(4) * sc * (b2 - T(4) * c * b3)) / (T(1) + T(4) * sc * (A + T(16) * c * c));
    const T kh = b3 - T(4) * c * rh;
    const T mh = b2 + A * rh - T(4) * c * kh;
    out[0] = w1 * rh + w * rl;
    out[1] = w1 * mh + w * mu[q.p];
    out[2] = w1 * kh + w * ka[q.p];
  } else {
    const T B = T(1) / rl + T(2) * P.ce;
    const T b2 = f[1][pf] + flog(rl) - T(1);
    T rh = (b1 - T(4) * sc * b2) / (T(1) + T(4) * sc * B);
    rh = fsqrt(rh * rh + P.delta * P.delta);
    const T mh = b2 + B * rh;
    out[0] = w1 * rh + w * rl;
    out[1] = w1 * mh + w * mu[q.p];
  }
}

// Rows of N(g) at node q (App. G, Eqs. MGN_DFT_a-c / MGN_PFC_a-e).  g and rk
// are read at q and its neighbours; om at index pf (which may live in another
// array layout, e.g. a global array while g sits in an LDS tile).
template <int MODEL, typename T, bool PM = false>
__device__ __forceinline__ void rows_hydro(const T* const* g, const T* rk, const T* om, const Nbr& q,
                                           int pf, const Coef<T>& K, const Phys<T>& P, T* out,
                                           const T* pm = nullptr) {
  const T s = P.s;
  const T c4 = K.c4, c2 = K.c2, ih2 = K.ih2;
  const T* rho = g[0];
  const T* u = g[1];
  const T* v = g[2];
  const T rkP = rk[q.p], omP = om[pf];
  const T uP = u[q.p], vP = v[q.p];
  const T uE = u[q.e], uW = u[q.w], uN = u[q.n], uS = u[q.s];
  const T vE = v[q.e], vW = v[q.w], vN = v[q.n], vS = v[q.s];
  out[0] = rho[q.p] + c4 * (rk[q.e] * uE - rk[q.w] * uW + rk[q.n] * vN - rk[q.s] * vS);
  const T qE = uE * uE + vE * vE, qW = uW * uW + vW * vW;
  const T qN = uN * uN + vN * vN, qS = uS * uS + vS * vS;
  const T ME = PM ? pm[q.e] : potential<MODEL>(g, q.e, P), MW = PM ? pm[q.w] : potential<MODEL>(g, q.w, P);
  const T MN = PM ? pm[q.n] : potential<MODEL>(g, q.n, P), MS = PM ? pm[q.s] : potential<MODEL>(g, q.s, P);
  const T lapu = (uE + uW + uN + uS - T(4) * uP) * ih2;
  const T lapv = (vE + vW + vN + vS - T(4) * vP) * ih2;
  const T b = T(0.5) * s * P.sigma * rkP * omP;
  out[1] = rkP * uP - b * vP + c4 * rkP * (qE - qW) + c2 * rkP * (ME - MW) - T(0.5) * s * P.gamma * lapu;
  out[2] = rkP * vP + b * uP + c4 * rkP * (qN - qS) + c2 * rkP * (MN - MS) - T(0.5) * s * P.gamma * lapv;
  if constexpr (MODEL == PFC) {
    const T* mu = g[3];
    const T* ka = g[4];
    const T phi = rho[q.p] - T(1.5);
    const T lapk = (ka[q.e] + ka[q.w] + ka[q.n] + ka[q.s] - T(4) * ka[q.p]) * ih2;
    const T lapr = (rho[q.e] + rho[q.w] + rho[q.n] + rho[q.s] - T(4) * rho[q.p]) * ih2;
    out[3] = mu[q.p] - phi * phi * phi * T(1.0 / 3.0) - P.alpha * phi - lapk;
    out[4] = ka[q.p] - lapr;
  }
}

// Undamped point-block solve at node q from the current neighbour values,
// then the damping x <- (1 - w) x^ + w x_l (App. G).  The block is
// triangular: rho^ from row 1 alone, (u^, v^) from the 2x2 system of rows 2-3,
// kappa^ from row 5 given rho^, mu^ from row 4 given rho^, kappa^ with the
// cubic linearised about the current iterate.  g and rk are read at q and its
// neighbours, f and om at index pf.
template <int MODEL, typename T, bool PM = false>
__device__ __forceinline__ void block_update_hydro(const T* const* g, const T* const* f, const T* rk,
                                                   const T* om, const Nbr& q, int pf, const Coef<T>& K,
                                                   const Phys<T>& P, T* out, const T* pm = nullptr) {
  const T s = P.s;
  const T c4 = K.c4, c2 = K.c2, ih2 = K.ih2;
  const T* rho = g[0];
  const T* u = g[1];
  const T* v = g[2];
  const T rkP = rk[q.p], omP = om[pf];
  const T uE = u[q.e], uW = u[q.w], uN = u[q.n], uS = u[q.s];
  const T vE = v[q.e], vW = v[q.w], vN = v[q.n], vS = v[q.s];
  T rh = f[0][pf] - c4 * (rk[q.e] * uE - rk[q.w] * uW + rk[q.n] * vN - rk[q.s] * vS);
  if constexpr (MODEL == CDFT) rh = fsqrt(rh * rh + P.delta * P.delta);
  const T qE = uE * uE + vE * vE, qW = uW * uW + vW * vW;
  const T qN = uN * uN + vN * vN, qS = uS * uS + vS * vS;
  const T ME = PM ? pm[q.e] : potential<MODEL>(g, q.e, P), MW = PM ? pm[q.w] : potential<MODEL>(g, q.w, P);
  const T MN = PM ? pm[q.n] : potential<MODEL>(g, q.n, P), MS = PM ? pm[q.s] : potential<MODEL>(g, q.s, P);
  const T cg = T(0.5) * s * P.gamma * ih2;
  const T a = rkP + T(4) * cg;
  const T b = T(0.5) * s * P.sigma * rkP * omP;
  const T ru = f[1][pf] - c4 * rkP * (qE - qW) - c2 * rkP * (ME - MW) + cg * (uE + uW + uN + uS);
  const T rv = f[2][pf] - c4 * rkP * (qN - qS) - c2 * rkP * (MN - MS) + cg * (vE + vW + vN + vS);
  const T idet = T(1) / (a * a + b * b);
  const T uh = (a * ru + b * rv) * idet;
  const T vh = (a * rv - b * ru) * idet;
  const T w = P.w, w1 = T(1) - P.w;
  const T rl = rho[q.p];
  out[0] = w1 * rh + w * rl;
  out[1] = w1 * uh + w * u[q.p];
  out[2] = w1 * vh + w * v[q.p];
  if constexpr (MODEL == PFC) {
    const T* mu = g[3];
    const T* ka = g[4];
    const T kh = f[4][pf] + (rho[q.e] + rho[q.w] + rho[q.n] + rho[q.s]) * ih2 - T(4) * rh * ih2;
    const T pl = rl - T(1.5);
    const T mh = f[3][pf] + (P.alpha + pl * pl) * (rh - T(1.5)) - (T(2) / T(3)) * pl * pl * pl +
                 (ka[q.e] + ka[q.w] + ka[q.n] + ka[q.s]) * ih2 - T(4) * kh * ih2;
    out[3] = w1 * mh + w * mu[q.p];
    out[4] = w1 * kh + w * ka[q.p];
  }
}

// ---------------------------------------------------------------------------
// Correction form (the inner FP32 solve of the mixed-precision step).
//
// With the outer FP64 iterate g held fixed as the base b = (rho_b, u_b, v_b),
// the inner unknown is the correction e and the inner operator is
//   N_d(e) = N(b + e) - N(b),
// written so that every term is formed from e directly (no difference of two
// nearly equal FP32 numbers): the linear rows are N's own rows applied to e;
// the nonlinear pieces are
//   |u|^2:  (u_b + e_u)^2 - u_b^2 = e_u (2 u_b + e_u)   (and v)
//   PFC cubic: c(e) = ((phi_b + e)^3 - phi_b^3)/3 = e (phi_b^2 + phi_b e + e^2/3)
//   CDFT potential: ln((rho_b + e)/rho_b) + 2 c_e e = log1p(e/rho_b) + 2 c_e e.
// N_d(e) = d with d = S - N(b) has the root e = g* - b.  The smoother is the
// block solve of the rows above, the cubic linearised about the current
// correction e_l, c(e) ~ c(e_l) + (phi_b + e_l)^2 (e - e_l) (the same
// linearisation as the full form), damped like the full form.

__device__ __forceinline__ float flog1p(float x) { return log1pf(x); }
__device__ __forceinline__ double flog1p(double x) { return log1p(x); }

template <int MODEL, typename T>
__device__ __forceinline__ T potential_d(const T* const* e, const T* const* b, int q, const Phys<T>& P) {
  if constexpr (MODEL == PFC) {
    return e[3][q];
  } else {
    const T x = e[0][q];
    return flog1p(x / b[0][q]) + T(2) * P.ce * x;
  }
}

template <typename T>
__device__ __forceinline__ T dq(const T* const* e, const T* const* b, int q) {
  const T eu = e[1][q], ev = e[2][q];
  return eu * (T(2) * b[1][q] + eu) + ev * (T(2) * b[2][q] + ev);
}

template <int MODEL, typename T, bool PM = false>
__device__ __forceinline__ void rows_Nd_hydro(const T* const* e, const T* const* b, const T* rk, const T* om,
                                              const Nbr& q, int pf, const Coef<T>& K, const Phys<T>& P, T* out,
                                              const T* pm = nullptr) {
  const T s = P.s;
  const T c4 = K.c4, c2 = K.c2, ih2 = K.ih2;
  const T* er = e[0];
  const T* u = e[1];
  const T* v = e[2];
  const T rkP = rk[q.p], omP = om[pf];
  const T uP = u[q.p], vP = v[q.p];
  const T uE = u[q.e], uW = u[q.w], uN = u[q.n], uS = u[q.s];
  const T vE = v[q.e], vW = v[q.w], vN = v[q.n], vS = v[q.s];
  out[0] = er[q.p] + c4 * (rk[q.e] * uE - rk[q.w] * uW + rk[q.n] * vN - rk[q.s] * vS);
  const T qE = dq(e, b, q.e), qW = dq(e, b, q.w), qN = dq(e, b, q.n), qS = dq(e, b, q.s);
  const T ME = PM ? pm[q.e] : potential_d<MODEL>(e, b, q.e, P);
  const T MW = PM ? pm[q.w] : potential_d<MODEL>(e, b, q.w, P);
  const T MN = PM ? pm[q.n] : potential_d<MODEL>(e, b, q.n, P);
  const T MS = PM ? pm[q.s] : potential_d<MODEL>(e, b, q.s, P);
  const T lapu = (uE + uW + uN + uS - T(4) * uP) * ih2;
  const T lapv = (vE + vW + vN + vS - T(4) * vP) * ih2;
  const T bb = T(0.5) * s * P.sigma * rkP * omP;
  out[1] = rkP * uP - bb * vP + c4 * rkP * (qE - qW) + c2 * rkP * (ME - MW) - T(0.5) * s * P.gamma * lapu;
  out[2] = rkP * vP + bb * uP + c4 * rkP * (qN - qS) + c2 * rkP * (MN - MS) - T(0.5) * s * P.gamma * lapv;
  if constexpr (MODEL == PFC) {
    const T* mu = e[3];
    const T* ka = e[4];
    const T x = er[q.p];
    const T pb = b[0][q.p] - T(1.5);
    const T cub = x * (pb * pb + pb * x + x * x * T(1.0 / 3.0));
    const T lapk = (ka[q.e] + ka[q.w] + ka[q.n] + ka[q.s] - T(4) * ka[q.p]) * ih2;
    const T lapr = (er[q.e] + er[q.w] + er[q.n] + er[q.s] - T(4) * x) * ih2;
    out[3] = mu[q.p] - cub - P.alpha * x - lapk;
    out[4] = ka[q.p] - lapr;
  }
}

template <int MODEL, typename T, bool PM = false>
__device__ __forceinline__ void block_update_d_hydro(const T* const* e, const T* const* f, const T* const* b,
                                                     const T* rk, const T* om, const Nbr& q, int pf,
                                                     const Coef<T>& K, const Phys<T>& P, T* out,
                                                     const T* pm = nullptr) {
  const T s = P.s;
  const T c4 = K.c4, c2 = K.c2, ih2 = K.ih2;
  const T* er = e[0];
  const T* u = e[1];
  const T* v = e[2];
  const T rkP = rk[q.p], omP = om[pf];
  const T uE = u[q.e], uW = u[q.w], uN = u[q.n], uS = u[q.s];
  const T vE = v[q.e], vW = v[q.w], vN = v[q.n], vS = v[q.s];
  T rh = f[0][pf] - c4 * (rk[q.e] * uE - rk[q.w] * uW + rk[q.n] * vN - rk[q.s] * vS);
  if constexpr (MODEL == CDFT) {
    // positivity projection of rho = rho_b + e; a no-op in this precision
    // unless rho_b + e is within a few orders of magnitude of delta or below
    const T rb = b[0][q.p];
    const T t = rb + rh;
    if (!(t > T(0) && t * t > T(1e6) * P.delta * P.delta)) rh = fsqrt(t * t + P.delta * P.delta) - rb;
  }
  const T qE = dq(e, b, q.e), qW = dq(e, b, q.w), qN = dq(e, b, q.n), qS = dq(e, b, q.s);
  const T ME = PM ? pm[q.e] : potential_d<MODEL>(e, b, q.e, P);
  const T MW = PM ? pm[q.w] : potential_d<MODEL>(e, b, q.w, P);
  const T MN = PM ? pm[q.n] : potential_d<MODEL>(e, b, q.n, P);
  const T MS = PM ? pm[q.s] : potential_d<MODEL>(e, b, q.s, P);
  const T cg = T(0.5) * s * P.gamma * ih2;
  const T a = rkP + T(4) * cg;
  const T bb = T(0.5) * s * P.sigma * rkP * omP;
  const T ru = f[1][pf] - c4 * rkP * (qE - qW) - c2 * rkP * (ME - MW) + cg * (uE + uW + uN + uS);
  const T rv = f[2][pf] - c4 * rkP * (qN - qS) - c2 * rkP * (MN - MS) + cg * (vE + vW + vN + vS);
  const T idet = T(1) / (a * a + bb * bb);
  const T uh = (a * ru + bb * rv) * idet;
  const T vh = (a * rv - bb * ru) * idet;
  const T w = P.w, w1 = T(1) - P.w;
  const T el = er[q.p];
  out[0] = w1 * rh + w * el;
  out[1] = w1 * uh + w * u[q.p];
  out[2] = w1 * vh + w * v[q.p];
  if constexpr (MODEL == PFC) {
    const T* mu = e[3];
    const T* ka = e[4];
    const T kh = f[4][pf] + (er[q.e] + er[q.w] + er[q.n] + er[q.s]) * ih2 - T(4) * rh * ih2;
    const T pb = b[0][q.p] - T(1.5);
    const T pl = pb + el;
    const T cl = el * (pb * pb + pb * el + el * el * T(1.0 / 3.0));
    const T mh = f[3][pf] + cl + pl * pl * (rh - el) + P.alpha * rh +
                 (ka[q.e] + ka[q.w] + ka[q.n] + ka[q.s]) * ih2 - T(4) * kh * ih2;
    out[3] = w1 * mh + w * mu[q.p];
    out[4] = w1 * kh + w * ka[q.p];
  }
}

// Correction form of the gradient flow about the base density rho_b (b[0]):
// N_d(e) = N(b + e) - N(b) with the cubic difference
// c(e) = e (phi_b^2 + phi_b e + e^2/3) (GPFC) and ln((rho_b + e)/rho_b) =
// log1p(e/rho_b) (GCDFT); the rows are otherwise linear in e.  The block
// solve linearises c(e) ~ c(e_l) + (phi_b + e_l)^2 (e - e_l) and
// log1p(e/rho_b) ~ log1p(e_l/rho_b) + (e - e_l)/(rho_b + e_l), and projects
// rho_b + e^ like the full form.
template <int MODEL, typename T>
__device__ __forceinline__ void rows_gfd(const T* const* e, const T* const* b, const Nbr& q, const Coef<T>& K,
                                         const Phys<T>& P, T* out) {
  const T ih2 = K.ih2;
  const T* er = e[0];
  const T* em = e[1];
  const T x = er[q.p];
  out[0] = x - P.s * ((nsum(em, q) - T(4) * em[q.p]) * ih2);
  if constexpr (MODEL == GPFC) {
    const T* ek = e[2];
    const T pb = b[0][q.p] - T(1.5);
    const T cub = x * (pb * pb + pb * x + x * x * T(1.0 / 3.0));
    const T lapk = (nsum(ek, q) - T(4) * ek[q.p]) * ih2;
    const T lapr = (nsum(er, q) - T(4) * x) * ih2;
    out[1] = em[q.p] - cub - P.alpha * x - lapk;
    out[2] = ek[q.p] - lapr;
  } else {
    out[1] = em[q.p] - flog1p(x / b[0][q.p]) - T(2) * P.ce * x;
  }
}

template <int MODEL, typename T>
__device__ __forceinline__ void block_update_gfd(const T* const* e, const T* const* f, const T* const* b,
                                                 const Nbr& q, int pf, const Coef<T>& K, const Phys<T>& P,
                                                 T* out) {
  const T c = K.ih2, sc = P.s * c;
  const T* er = e[0];
  const T* em = e[1];
  const T el = er[q.p];
  const T b1 = f[0][pf] + sc * nsum(em, q);
  const T w = P.w, w1 = T(1) - P.w;
  if constexpr (MODEL == GPFC) {
    const T* ek = e[2];
    const T pb = b[0][q.p] - T(1.5);
    const T pl = pb + el;
    const T A = P.alpha + pl * pl;
    const T cl = el * (pb * pb + pb * el + el * el * T(1.0 / 3.0));
    const T b2 = f[1][pf] + cl - pl * pl * el + c * nsum(ek, q);
    const T b3 = f[2][pf] + c * nsum(er, q);
    const T rh = (b1 - T(4) * sc * (b2 - T(4) * c * b3)) / (T(1) + T(4) * sc * (A + T(16) * c * c));
    const T kh = b3 - T(4) * c * rh;
    const T mh = b2 + A * rh - T(4) * c * kh;
    out[0] = w1 * rh + w * el;
    out[1] = w1 * mh + w * em[q.p];
    out[2] = w1 * kh + w * ek[q.p];
  } else {
    const T rb = b[0][q.p];
    const T t = rb + el;
    const T B = T(1) / t + T(2) * P.ce;
    const T b2 = f[1][pf] + flog1p(el / rb) - el / t;
    T rh = (b1 - T(4) * sc * b2) / (T(1) + T(4) * sc * B);
    const T tt = rb + rh;
    if (!(tt > T(0) && tt * tt > T(1e6) * P.delta * P.delta)) rh = fsqrt(tt * tt + P.delta * P.delta) - rb;
    const T mh = b2 + B * rh;
    out[0] = w1 * rh + w * el;
    out[1] = w1 * mh + w * em[q.p];
  }
}

// Model dispatch of the rows and the block update: the hydrodynamic system
// or the gradient flow.
template <int MODEL, typename T, bool PM = false>
__device__ __forceinline__ void rows_N(const T* const* g, const T* rk, const T* om, const Nbr& q, int pf,
                                       const Coef<T>& K, const Phys<T>& P, T* out, const T* pm = nullptr) {
  if constexpr (gradflow(MODEL))
    rows_gf<MODEL, T>(g, q, K, P, out);
  else
    rows_hydro<algebra(MODEL), T, PM>(g, rk, om, q, pf, K, P, out, pm);
}

template <int MODEL, typename T, bool PM = false>
__device__ __forceinline__ void block_update(const T* const* g, const T* const* f, const T* rk, const T* om,
                                             const Nbr& q, int pf, const Coef<T>& K, const Phys<T>& P, T* out,
                                             const T* pm = nullptr) {
  if constexpr (gradflow(MODEL))
    block_update_gf<MODEL, T>(g, f, q, pf, K, P, out);
  else
    block_update_hydro<algebra(MODEL), T, PM>(g, f, rk, om, q, pf, K, P, out, pm);
}

template <int MODEL, typename T, bool PM = false>
__device__ __forceinline__ void rows_Nd(const T* const* e, const T* const* b, const T* rk, const T* om,
                                        const Nbr& q, int pf, const Coef<T>& K, const Phys<T>& P, T* out,
                                        const T* pm = nullptr) {
  if constexpr (gradflow(MODEL))
    rows_gfd<MODEL, T>(e, b, q, K, P, out);
  else
    rows_Nd_hydro<algebra(MODEL), T, PM>(e, b, rk, om, q, pf, K, P, out, pm);
}

template <int MODEL, typename T, bool PM = false>
__device__ __forceinline__ void block_update_d(const T* const* e, const T* const* f, const T* const* b,
                                               const T* rk, const T* om, const Nbr& q, int pf, const Coef<T>& K,
                                               const Phys<T>& P, T* out, const T* pm = nullptr) {
  if constexpr (gradflow(MODEL))
    block_update_gfd<MODEL, T>(e, f, b, q, pf, K, P, out);
  else
    block_update_d_hydro<algebra(MODEL), T, PM>(e, f, b, rk, om, q, pf, K, P, out, pm);
}

// Mode dispatch: CORR = false is the full form, CORR = true the correction
// form about the base fields b.  PM = true reads the potential M at the four
// neighbours from pm (same index space as g) instead of evaluating it there.
template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ T potential_any(const T* const* g, const T* const* b, int q, const Phys<T>& P) {
  if constexpr (CORR)
    return potential_d<MODEL, T>(g, b, q, P);
  else
    return potential<MODEL, T>(g, q, P);
}

template <int MODEL, typename T, bool CORR, bool PM = false>
__device__ __forceinline__ void rows_any(const T* const* g, const T* const* b, const T* rk, const T* om,
                                         const Nbr& q, int pf, const Coef<T>& K, const Phys<T>& P, T* out,
                                         const T* pm = nullptr) {
  if constexpr (CORR)
    rows_Nd<MODEL, T, PM>(g, b, rk, om, q, pf, K, P, out, pm);
  else
    rows_N<MODEL, T, PM>(g, rk, om, q, pf, K, P, out, pm);
}

template <int MODEL, typename T, bool CORR, bool PM = false>
__device__ __forceinline__ void update_any(const T* const* g, const T* const* f, const T* const* b, const T* rk,
                                           const T* om, const Nbr& q, int pf, const Coef<T>& K,
                                           const Phys<T>& P, T* out, const T* pm = nullptr) {
  if constexpr (CORR)
    block_update_d<MODEL, T, PM>(g, f, b, rk, om, q, pf, K, P, out, pm);
  else
    block_update<MODEL, T, PM>(g, f, rk, om, q, pf, K, P, out, pm);
}

// CDFT projection of an iterate value after the coarse-grid correction: full
// form rho <- sqrt(rho^2 + delta^2); correction form the same on rho_b + e.
template <typename T, bool CORR>
__device__ __forceinline__ T project_any(T x, T base, T delta) {
  if constexpr (CORR) {
    const T t = base + x;
    if (!(t > T(0) && t * t > T(1e6) * delta * delta)) return fsqrt(t * t + delta * delta) - base;
    return x;
  } else {
    return fsqrt(x * x + delta * delta);
  }
}

}  // namespace hfz
