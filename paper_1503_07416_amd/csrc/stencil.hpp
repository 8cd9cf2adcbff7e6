// Pointwise algebra of the implicit step on one grid level: the rows of the
// nonlinear system N(g) = S (App. G, typos fixed from Eqs. discrete_a-d), the
// source S, and the point-block Gauss-Seidel update (App. G smoother with its
// damping).  Every function works on one node (i, j) of a periodic n x n
// level, n a power of two, fields row-major with x fastest.
#pragma once
#include <hip/hip_runtime.h>

namespace hfz {

enum { PFC = 0, CDFT = 1 };

template <int MODEL> struct NC { static constexpr int value = (MODEL == PFC) ? 5 : 3; };

__device__ __forceinline__ double flog(double x) { return log(x); }
__device__ __forceinline__ float flog(float x) { return logf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fsqrt(float x) { return sqrtf(x); }

// Physical constants of the step, in the arithmetic type T.
template <typename T> struct Phys {
  T s, gamma, sigma, alpha, ce, delta, w;
};

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
  int n;      // grid size n_l
  int lg;     // log2 n_l
  T h;        // spacing h_l
  Coef<T> k;  // stencil coefficients of this level
};

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

// Rows of N(g) at node q (App. G, Eqs. MGN_DFT_a-c / MGN_PFC_a-e).  g and rk
// are read at q and its neighbours; om at index pf (which may live in another
// array layout, e.g. a global array while g sits in an LDS tile).
template <int MODEL, typename T>
__device__ __forceinline__ void rows_N(const T* const* g, const T* rk, const T* om, const Nbr& q,
                                       int pf, const Coef<T>& K, const Phys<T>& P, T* out) {
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
  const T ME = potential<MODEL>(g, q.e, P), MW = potential<MODEL>(g, q.w, P);
  const T MN = potential<MODEL>(g, q.n, P), MS = potential<MODEL>(g, q.s, P);
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
template <int MODEL, typename T>
__device__ __forceinline__ void block_update(const T* const* g, const T* const* f, const T* rk,
                                             const T* om, const Nbr& q, int pf, const Coef<T>& K,
                                             const Phys<T>& P, T* out) {
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
  const T ME = potential<MODEL>(g, q.e, P), MW = potential<MODEL>(g, q.w, P);
  const T MN = potential<MODEL>(g, q.n, P), MS = potential<MODEL>(g, q.s, P);
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

}  // namespace hfz
