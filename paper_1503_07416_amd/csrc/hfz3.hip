// The hydrodynamic PFC step in three dimensions (the extension Sec. 3 calls
// straightforward; the paper works in 2D): the C ABI hfz3_* of include/hfz.h.
//
// Unknowns per node g = (rho, u, v, w, mu, kappa) on a periodic n^3 grid,
// fields stored x fastest, then y, then z (index ((l n) + j) n + i).  The rows
// are the 2D ones of App. G with a third direction: the 7-point Delta_h, the
// wide central differences, the vector vorticity omega^k = curl_h u^k and the
// vector form -rho^k omega^k x u of the advection term.  The smoother keeps
// App. G's triangular block: rho^ from the continuity row, then the 3x3
// velocity block (a I + [b x]) u^ = r, a = rho^k + 3 s gamma / h^2,
// b = (s/2) sigma rho^k omega^k, whose inverse is
//   u^ = (a^2 r - a (b x r) + (b . r) b) / (a (a^2 + |b|^2)),
// then kappa^ and mu^ (the cubic linearised about the current iterate), all
// damped by w; red-black by (i + j + l) mod 2.  FAS V(nu1, nu2) with 27-point
// full weighting and trilinear prolongation, coarsest grid swept a fixed
// number of times, stop on (h^3 sum d^2)^(1/2) <= tol tested on the device.
//
// One thread per node (per node of a colour in the smoother); the levels are
// bandwidth- or latency-bound, the neighbour reads served by the caches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "hfz.h"

namespace hfz3 {

constexpr int NC = 6;

struct Lvl {
  double* g[NC];   // iterate
  double* f[NC];   // right-hand side (level 0: the source S)
  double* g0[NC];  // restricted iterate R g (coarse levels)
  double* d[NC];   // residual f - N(g) before restriction
  double* rk;      // frozen rho^k
  double* om[3];   // frozen omega^k
  int n, lg;       // n = 2^lg nodes per direction
  double h;
};

struct Phys {
  double s, gamma, sigma, alpha, w;
  const int* halt;  // device stop flag of the V-cycle loop (null: none)
};

__device__ __forceinline__ bool halted(const int* f) { return f != nullptr && *f != 0; }

struct Nbr {
  int p, e, w, n, s, u, d;  // node and its neighbours in +x, -x, +y, -y, +z, -z
};

__device__ __forceinline__ Nbr nbr(int i, int j, int l, int lg) {
  const int m = (1 << lg) - 1;
  const int row = (l << lg) + j;
  Nbr q;
  q.p = (row << lg) + i;
  q.e = (row << lg) + ((i + 1) & m);
  q.w = (row << lg) + ((i - 1) & m);
  q.n = (((l << lg) + ((j + 1) & m)) << lg) + i;
  q.s = (((l << lg) + ((j - 1) & m)) << lg) + i;
  q.u = (((((l + 1) & m) << lg) + j) << lg) + i;
  q.d = (((((l - 1) & m) << lg) + j) << lg) + i;
  return q;
}

__device__ __forceinline__ double sum6(const double* f, const Nbr& q) {
  return f[q.e] + f[q.w] + f[q.n] + f[q.s] + f[q.u] + f[q.d];
}

__device__ __forceinline__ double q2(const double* const* g, int p) {
  return g[1][p] * g[1][p] + g[2][p] * g[2][p] + g[3][p] * g[3][p];
}

// Rows of N(g) at node q (module comment).
__device__ __forceinline__ void rows(const Lvl& L, const Phys& P, const double* const* g, const Nbr& q,
                                     double* out) {
  const double h = L.h, s = P.s, c4 = s / (4.0 * h), c2 = s / (2.0 * h), ih2 = 1.0 / (h * h);
  const double* rk = L.rk;
  const double* u = g[1];
  const double* v = g[2];
  const double* w = g[3];
  const double* mu = g[4];
  out[0] = g[0][q.p] + c4 * (rk[q.e] * u[q.e] - rk[q.w] * u[q.w] + rk[q.n] * v[q.n] - rk[q.s] * v[q.s] +
                             rk[q.u] * w[q.u] - rk[q.d] * w[q.d]);
  const double rkP = rk[q.p];
  const double o0 = L.om[0][q.p], o1 = L.om[1][q.p], o2 = L.om[2][q.p];
  const double uP = u[q.p], vP = v[q.p], wP = w[q.p];
  const double cx = o1 * wP - o2 * vP, cy = o2 * uP - o0 * wP, cz = o0 * vP - o1 * uP;
  const double bs = 0.5 * s * P.sigma * rkP, gl = 0.5 * s * P.gamma * ih2;
  out[1] = rkP * uP + bs * cx + c4 * rkP * (q2(g, q.e) - q2(g, q.w)) + c2 * rkP * (mu[q.e] - mu[q.w]) -
           gl * (sum6(u, q) - 6.0 * uP);
  out[2] = rkP * vP + bs * cy + c4 * rkP * (q2(g, q.n) - q2(g, q.s)) + c2 * rkP * (mu[q.n] - mu[q.s]) -
           gl * (sum6(v, q) - 6.0 * vP);
  out[3] = rkP * wP + bs * cz + c4 * rkP * (q2(g, q.u) - q2(g, q.d)) + c2 * rkP * (mu[q.u] - mu[q.d]) -
           gl * (sum6(w, q) - 6.0 * wP);
  const double phi = g[0][q.p] - 1.5;
  out[4] = mu[q.p] - phi * phi * phi * (1.0 / 3.0) - P.alpha * phi - (sum6(g[5], q) - 6.0 * g[5][q.p]) * ih2;
  out[5] = g[5][q.p] - (sum6(g[0], q) - 6.0 * g[0][q.p]) * ih2;
}

// Damped block update at node q (module comment).
__device__ __forceinline__ void block(const Lvl& L, const Phys& P, const Nbr& q, double* out) {
  const double h = L.h, s = P.s, c4 = s / (4.0 * h), c2 = s / (2.0 * h), ih2 = 1.0 / (h * h);
  const double* rk = L.rk;
  double* const* g = L.g;
  const double* u = g[1];
  const double* v = g[2];
  const double* w = g[3];
  const double* mu = g[4];
  const double rh = L.f[0][q.p] - c4 * (rk[q.e] * u[q.e] - rk[q.w] * u[q.w] + rk[q.n] * v[q.n] - rk[q.s] * v[q.s] +
                                        rk[q.u] * w[q.u] - rk[q.d] * w[q.d]);
  const double rkP = rk[q.p];
  const double cg = 0.5 * s * P.gamma * ih2;
  const double a = rkP + 6.0 * cg;
  const double bs = 0.5 * s * P.sigma * rkP;
  const double b0 = bs * L.om[0][q.p], b1 = bs * L.om[1][q.p], b2 = bs * L.om[2][q.p];
  const double r0 = L.f[1][q.p] - c4 * rkP * (q2(g, q.e) - q2(g, q.w)) - c2 * rkP * (mu[q.e] - mu[q.w]) + cg * sum6(u, q);
  const double r1 = L.f[2][q.p] - c4 * rkP * (q2(g, q.n) - q2(g, q.s)) - c2 * rkP * (mu[q.n] - mu[q.s]) + cg * sum6(v, q);
  const double r2 = L.f[3][q.p] - c4 * rkP * (q2(g, q.u) - q2(g, q.d)) - c2 * rkP * (mu[q.u] - mu[q.d]) + cg * sum6(w, q);
  const double bb = b0 * b0 + b1 * b1 + b2 * b2;
  const double br = b0 * r0 + b1 * r1 + b2 * r2;
  const double x0 = b1 * r2 - b2 * r1, x1 = b2 * r0 - b0 * r2, x2 = b0 * r1 - b1 * r0;
  const double den = a * (a * a + bb);
  const double uh = (a * a * r0 - a * x0 + br * b0) / den;
  const double vh = (a * a * r1 - a * x1 + br * b1) / den;
  const double wh = (a * a * r2 - a * x2 + br * b2) / den;
  const double kh = L.f[5][q.p] + sum6(g[0], q) * ih2 - 6.0 * rh * ih2;
  const double pl = g[0][q.p] - 1.5;
  const double mh = L.f[4][q.p] + (P.alpha + pl * pl) * (rh - 1.5) - (2.0 / 3.0) * pl * pl * pl +
                    sum6(g[5], q) * ih2 - 6.0 * kh * ih2;
  const double wd = P.w, w1 = 1.0 - P.w;
  out[0] = w1 * rh + wd * g[0][q.p];
  out[1] = w1 * uh + wd * u[q.p];
  out[2] = w1 * vh + wd * v[q.p];
  out[3] = w1 * wh + wd * w[q.p];
  out[4] = w1 * mh + wd * mu[q.p];
  out[5] = w1 * kh + wd * g[5][q.p];
}

// 27-point full weighting at coarse node (I, J, K) = fine (2I, 2J, 2K).
__device__ __forceinline__ double fw27(const double* f, int I, int J, int K, int lgf) {
  const int m = (1 << lgf) - 1;
  double acc = 0.0;
  for (int dk = -1; dk <= 1; ++dk) {
    const int k = (2 * K + dk) & m;
    const double wk = dk == 0 ? 2.0 : 1.0;
    for (int dj = -1; dj <= 1; ++dj) {
      const int j = (2 * J + dj) & m;
      const double wj = dj == 0 ? 2.0 : 1.0;
      const int row = ((k << lgf) + j) << lgf;
      acc += wk * wj * (f[row + ((2 * I - 1) & m)] + 2.0 * f[row + 2 * I] + f[row + ((2 * I + 1) & m)]);
    }
  }
  return acc * (1.0 / 64.0);
}

struct Idx {
  int i, j, l, ok;
};

// Thread -> node of an n^3 level in 2D launch geometry (x in blockIdx.x, the
// (y, z) rows in blockIdx.y).
__device__ __forceinline__ Idx node(int n, int lg) {
  Idx x;
  x.i = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = blockIdx.y * blockDim.y + threadIdx.y;
  x.j = row & (n - 1);
  x.l = row >> lg;
  x.ok = x.i < n && row < n * n;
  return x;
}

// ---------------------------------------------------------------- kernels --
// omega^k = curl_h u^k and S from the state (rho^k, u^k, v^k, w^k); the iterate
// starts at the state (g = state, mu and kappa from the previous solve).
__global__ void k3_begin(Lvl L, const double* __restrict__ u0, const double* __restrict__ v0,
                         const double* __restrict__ w0, const double* __restrict__ mu0,
                         const double* __restrict__ ka0, Phys P) {
  const Idx x = node(L.n, L.lg);
  if (!x.ok) return;
  const Nbr q = nbr(x.i, x.j, x.l, L.lg);
  const double h = L.h, s = P.s, c4 = s / (4.0 * h), ih2 = 1.0 / (h * h), t2 = 1.0 / (2.0 * h);
  const double* r = L.rk;
  const double o0 = (w0[q.n] - w0[q.s]) * t2 - (v0[q.u] - v0[q.d]) * t2;
  const double o1 = (u0[q.u] - u0[q.d]) * t2 - (w0[q.e] - w0[q.w]) * t2;
  const double o2 = (v0[q.e] - v0[q.w]) * t2 - (u0[q.n] - u0[q.s]) * t2;
  L.om[0][q.p] = o0;
  L.om[1][q.p] = o1;
  L.om[2][q.p] = o2;
  const double rP = r[q.p], uP = u0[q.p], vP = v0[q.p], wP = w0[q.p];
  L.f[0][q.p] = rP - c4 * (r[q.e] * u0[q.e] - r[q.w] * u0[q.w] + r[q.n] * v0[q.n] - r[q.s] * v0[q.s] +
                           r[q.u] * w0[q.u] - r[q.d] * w0[q.d]);
  const double bs = 0.5 * s * P.sigma * rP, gl = 0.5 * s * P.gamma * ih2;
  L.f[1][q.p] = rP * uP - bs * (o1 * wP - o2 * vP) + gl * (sum6(u0, q) - 6.0 * uP);
  L.f[2][q.p] = rP * vP - bs * (o2 * uP - o0 * wP) + gl * (sum6(v0, q) - 6.0 * vP);
  L.f[3][q.p] = rP * wP - bs * (o0 * vP - o1 * uP) + gl * (sum6(w0, q) - 6.0 * wP);
  L.f[4][q.p] = 2.0 * (sum6(r, q) - 6.0 * rP) * ih2;
  L.f[5][q.p] = 0.0;
  L.g[0][q.p] = rP;
  L.g[1][q.p] = uP;
  L.g[2][q.p] = vP;
  L.g[3][q.p] = wP;
  L.g[4][q.p] = mu0[q.p];
  L.g[5][q.p] = ka0[q.p];
}

// rho^k and omega^k onto the next coarser level.
__global__ void k3_restrict_coef(Lvl F, Lvl C) {
  const Idx x = node(C.n, C.lg);
  if (!x.ok) return;
  const int pc = (((x.l << C.lg) + x.j) << C.lg) + x.i;
  C.rk[pc] = fw27(F.rk, x.i, x.j, x.l, F.lg);
  for (int c = 0; c < 3; ++c) C.om[c][pc] = fw27(F.om[c], x.i, x.j, x.l, F.lg);
}

// One colour of a damped red-black sweep: thread t of (y, z) row updates node
// i = 2 t + ((j + l + colour) & 1).
__global__ void k3_smooth(Lvl L, Phys P, int colour) {
  if (halted(P.halt)) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = blockIdx.y * blockDim.y + threadIdx.y;
  const int n = L.n;
  if (t >= (n >> 1) || row >= n * n) return;
  const int j = row & (n - 1), l = row >> L.lg;
  const int i = 2 * t + ((j + l + colour) & 1);
  const Nbr q = nbr(i, j, l, L.lg);
  double out[NC];
  block(L, P, q, out);
#pragma unroll
  for (int c = 0; c < NC; ++c) L.g[c][q.p] = out[c];
}

// d = f - N(g).
__global__ void k3_residual_field(Lvl L, Phys P) {
  if (halted(P.halt)) return;
  const Idx x = node(L.n, L.lg);
  if (!x.ok) return;
  const Nbr q = nbr(x.i, x.j, x.l, L.lg);
  double nv[NC];
  rows(L, P, L.g, q, nv);
#pragma unroll
  for (int c = 0; c < NC; ++c) L.d[c][q.p] = L.f[c][q.p] - nv[c];
}

// g_c = g0_c = R g, f_c = R d.
__global__ void k3_restrict(Lvl F, Lvl C, const int* halt) {
  if (halted(halt)) return;
  const Idx x = node(C.n, C.lg);
  if (!x.ok) return;
  const int pc = (((x.l << C.lg) + x.j) << C.lg) + x.i;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double gr = fw27(F.g[c], x.i, x.j, x.l, F.lg);
    C.g[c][pc] = gr;
    C.g0[c][pc] = gr;
    C.f[c][pc] = fw27(F.d[c], x.i, x.j, x.l, F.lg);
  }
}

// f_c += N_c(R g).
__global__ void k3_fas_rhs(Lvl C, Phys P) {
  if (halted(P.halt)) return;
  const Idx x = node(C.n, C.lg);
  if (!x.ok) return;
  const Nbr q = nbr(x.i, x.j, x.l, C.lg);
  double nv[NC];
  rows(C, P, C.g0, q, nv);
#pragma unroll
  for (int c = 0; c < NC; ++c) C.f[c][q.p] += nv[c];
}

// g += P(g_c - R g), trilinear.
__global__ void k3_prolong(Lvl F, Lvl C, const int* halt) {
  if (halted(halt)) return;
  const Idx x = node(F.n, F.lg);
  if (!x.ok) return;
  const int mc = C.n - 1, lc = C.lg;
  const int I0 = x.i >> 1, J0 = x.j >> 1, K0 = x.l >> 1;
  const int I1 = (I0 + (x.i & 1)) & mc, J1 = (J0 + (x.j & 1)) & mc, K1 = (K0 + (x.l & 1)) & mc;
  auto at = [&](int I, int J, int K) { return (((K << lc) + J) << lc) + I; };
  const int c000 = at(I0, J0, K0), c100 = at(I1, J0, K0), c010 = at(I0, J1, K0), c110 = at(I1, J1, K0);
  const int c001 = at(I0, J0, K1), c101 = at(I1, J0, K1), c011 = at(I0, J1, K1), c111 = at(I1, J1, K1);
  const int pf = (((x.l << F.lg) + x.j) << F.lg) + x.i;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double* gc = C.g[c];
    const double* g0 = C.g0[c];
    auto e = [&](int k) { return gc[k] - g0[k]; };
    // averages along x, then y, then z (a coincident node enters with weight 1)
    const double ex00 = 0.5 * (e(c000) + e(c100)), ex10 = 0.5 * (e(c010) + e(c110));
    const double ex01 = 0.5 * (e(c001) + e(c101)), ex11 = 0.5 * (e(c011) + e(c111));
    const double exy0 = 0.5 * (ex00 + ex10), exy1 = 0.5 * (ex01 + ex11);
    F.g[c][pf] += 0.5 * (exy0 + exy1);
  }
}

// Block sum in a fixed order.
__device__ __forceinline__ double block_sum(double x, double* lds) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  const int tid = threadIdx.y * blockDim.x + threadIdx.x, nth = blockDim.x * blockDim.y;
  if ((tid & 63) == 0) lds[tid >> 6] = x;
  __syncthreads();
  double r = 0.0;
  if (tid == 0)
    for (int k = 0; k < (nth + 63) / 64; ++k) r += lds[k];
  __syncthreads();
  return r;
}

// Per-block partial sums of sum_c (f - N(g))^2 on a level.
__global__ void k3_residual_partial(Lvl L, Phys P, double* __restrict__ partial) {
  if (halted(P.halt)) return;
  __shared__ double lds[16];
  const Idx x = node(L.n, L.lg);
  double acc = 0.0;
  if (x.ok) {
    const Nbr q = nbr(x.i, x.j, x.l, L.lg);
    double nv[NC];
    rows(L, P, L.g, q, nv);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double dd = L.f[c][q.p] - nv[c];
      acc += dd * dd;
    }
  }
  const double r = block_sum(acc, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = r;
}

// result[0..nq) = scale * sums of `count` partials (nq quantities each).
__global__ void k3_reduce(const double* __restrict__ partial, int count, int nq, double scale,
                          double* __restrict__ result) {
  __shared__ double lds[16];
  for (int k = 0; k < nq; ++k) {
    double acc = 0.0;
    for (int t = threadIdx.x; t < count; t += blockDim.x) acc += partial[(size_t)t * nq + k];
    const double r = block_sum(acc, lds);
    if (threadIdx.x == 0) result[k] = scale * r;
  }
}

// The stop test on the device: unless ctl[0] is set, result[0] = the norm^2,
// with `counted` ctl[1] += 1, ctl[0] = 1 when sqrt <= tol, 2 when not finite.
__global__ void k3_reduce_stop(const double* __restrict__ partial, int count, double scale, double tol,
                               double* __restrict__ result, int* ctl, int counted) {
  __shared__ double lds[16];
  if (ctl[0] != 0) return;
  double acc = 0.0;
  for (int t = threadIdx.x; t < count; t += blockDim.x) acc += partial[t];
  const double r = block_sum(acc, lds);
  if (threadIdx.x == 0) {
    const double r2 = scale * r;
    result[0] = r2;
    if (counted) ctl[1] += 1;
    const double nrm = sqrt(r2);
    if (nrm <= tol)
      ctl[0] = 1;
    else if (!isfinite(nrm))
      ctl[0] = 2;
  }
}

__global__ void k3_ctl_reset(int* ctl) {
  if (threadIdx.x < 2) ctl[threadIdx.x] = 0;
}

// End of a step: rho^{k+1} from the continuity row (with fix), the state
// (rho, u, v, w, mu, kappa) <- the iterate.  rho^k (rk) is read at the
// neighbours, so the new rho goes to g[0] here and to rk in k3_state.
__global__ void k3_continuity(Lvl L, Phys P) {
  const Idx x = node(L.n, L.lg);
  if (!x.ok) return;
  const Nbr q = nbr(x.i, x.j, x.l, L.lg);
  const double c4 = P.s / (4.0 * L.h);
  const double* r = L.rk;
  const double* u = L.g[1];
  const double* v = L.g[2];
  const double* w = L.g[3];
  L.g[0][q.p] = L.f[0][q.p] - c4 * (r[q.e] * u[q.e] - r[q.w] * u[q.w] + r[q.n] * v[q.n] - r[q.s] * v[q.s] +
                                    r[q.u] * w[q.u] - r[q.d] * w[q.d]);
}

__global__ void k3_state(Lvl L, double* u0, double* v0, double* w0, double* mu0, double* ka0, size_t count) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  L.rk[t] = L.g[0][t];
  u0[t] = L.g[1][t];
  v0[t] = L.g[2][t];
  w0[t] = L.g[3][t];
  mu0[t] = L.g[4][t];
  ka0[t] = L.g[5][t];
}

// Auxiliaries consistent with rho^{k+1} = rho^k: kappa = Delta_h rho, then
// mu = phi^3/3 + alpha phi + Delta_h kappa + 2 Delta_h rho.
__global__ void k3_kappa(const double* __restrict__ rho, double* __restrict__ ka, int n, int lg, double h) {
  const Idx x = node(n, lg);
  if (!x.ok) return;
  const Nbr q = nbr(x.i, x.j, x.l, lg);
  ka[q.p] = (sum6(rho, q) - 6.0 * rho[q.p]) / (h * h);
}

__global__ void k3_mu(const double* __restrict__ rho, const double* __restrict__ ka, double* __restrict__ mu, int n,
                      int lg, double h, double alpha) {
  const Idx x = node(n, lg);
  if (!x.ok) return;
  const Nbr q = nbr(x.i, x.j, x.l, lg);
  const double phi = rho[q.p] - 1.5;
  mu[q.p] = phi * phi * phi / 3.0 + alpha * phi + (sum6(ka, q) - 6.0 * ka[q.p]) / (h * h) + 2.0 * ka[q.p];
}

// Per-block partials of (KE, F, mass) before the h^3 factor.
__global__ void k3_energy_partial(const double* __restrict__ rho, const double* __restrict__ u,
                                  const double* __restrict__ v, const double* __restrict__ w, int n, int lg,
                                  double h, double alpha, double* __restrict__ partial) {
  __shared__ double lds[16];
  const Idx x = node(n, lg);
  double ke = 0.0, f = 0.0, ms = 0.0;
  if (x.ok) {
    const Nbr q = nbr(x.i, x.j, x.l, lg);
    const double r = rho[q.p];
    ke = 0.5 * r * (u[q.p] * u[q.p] + v[q.p] * v[q.p] + w[q.p] * w[q.p]);
    const double phi = r - 1.5;
    const double L = (sum6(rho, q) - 6.0 * r) / (h * h);
    f = phi * phi * phi * phi / 12.0 + 0.5 * alpha * phi * phi + 0.5 * L * L + r * L;
    ms = r;
  }
  const int b = blockIdx.y * gridDim.x + blockIdx.x;
  double t;
  t = block_sum(ke, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[b * 3 + 0] = t;
  t = block_sum(f, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[b * 3 + 1] = t;
  t = block_sum(ms, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[b * 3 + 2] = t;
}

__global__ void k3_copy(const double* __restrict__ a, double* __restrict__ b, size_t count) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) b[t] = a[t];
}

// ------------------------------------------------------------------ host --
struct Dims {
  dim3 grid, block;
};

// Launch geometry for one thread per node of an n^3 level (nx threads per
// (y, z) row: n, or n/2 for one colour).
Dims dims(int nx, int n) {
  const int bx = std::min(64, nx);
  const int rows = n * n;
  const int by = std::max(1, std::min(256 / bx, rows));
  return {dim3((nx + bx - 1) / bx, (rows + by - 1) / by), dim3(bx, by)};
}

constexpr size_t kAlign = 256;

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T> T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = (off + count * sizeof(T) + kAlign - 1) & ~(kAlign - 1);
    return p;
  }
};

int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

}  // namespace hfz3

using namespace hfz3;

struct hfz3_handle {
  hfz_params p{};
  hipStream_t stream = nullptr;
  std::vector<Lvl> L;  // finest first
  Phys P{};
  double *u = nullptr, *v = nullptr, *w = nullptr, *mu = nullptr, *ka = nullptr;
  double* partial = nullptr;
  size_t partial_cap = 0;
  double* result = nullptr;
  int* ctl = nullptr;
  bool has_state = false;
  int cycle_hint = 4;
  int graph_state = 0;
  hipGraphExec_t cycle_exec = nullptr;
};

namespace {

int validate3(const hfz_params* p) {
  if (!p) return HFZ_EINVAL;
  if (p->model != HFZ_PFC || p->walls != 0 || p->precision != HFZ_FP64) return HFZ_EINVAL;
  if (!is_pow2(p->n) || p->n < 8 || p->n > 512) return HFZ_EINVAL;
  if (!(p->h > 0) || !(p->s > 0) || !(p->gamma > 0) || !std::isfinite(p->alpha)) return HFZ_EINVAL;
  if (!(p->w_damp >= 0.0) || !(p->w_damp < 1.0) || !(p->tol > 0)) return HFZ_EINVAL;
  if (p->nu1 < 0 || p->nu2 < 0 || p->nu1 + p->nu2 < 1 || p->max_cycles < 1 || p->coarse_sweeps < 1)
    return HFZ_EINVAL;
  if (!is_pow2(p->coarsest_n) || p->coarsest_n < 4 || p->coarsest_n > p->n) return HFZ_EINVAL;
  if (p->sigma != 1 && p->sigma != -1) return HFZ_EINVAL;
  return HFZ_OK;
}

size_t layout3(const hfz_params& p, void* ws, hfz3_handle* hd) {
  Carver c{static_cast<char*>(ws)};
  const int n = p.n;
  const size_t N3 = (size_t)n * n * n;
  std::vector<Lvl> L;
  double h = p.h;
  for (int m = n; m >= p.coarsest_n; m >>= 1) {
    Lvl l{};
    l.n = m;
    l.lg = ilog2(m);
    l.h = h;
    h *= 2.0;
    const size_t cnt = (size_t)m * m * m;
    for (int k = 0; k < NC; ++k) l.g[k] = c.take<double>(cnt);
    for (int k = 0; k < NC; ++k) l.f[k] = c.take<double>(cnt);
    if (m != n)
      for (int k = 0; k < NC; ++k) l.g0[k] = c.take<double>(cnt);
    if (m > p.coarsest_n)
      for (int k = 0; k < NC; ++k) l.d[k] = c.take<double>(cnt);
    l.rk = c.take<double>(cnt);
    for (int k = 0; k < 3; ++k) l.om[k] = c.take<double>(cnt);
    L.push_back(l);
  }
  double* u = c.take<double>(N3);
  double* v = c.take<double>(N3);
  double* w = c.take<double>(N3);
  double* mu = c.take<double>(N3);
  double* ka = c.take<double>(N3);
  const size_t pcap = std::max<size_t>(4096, N3 / 64 + 64) * 3;
  double* partial = c.take<double>(pcap);
  double* result = c.take<double>(64);
  if (hd) {
    hd->L = L;
    hd->u = u;
    hd->v = v;
    hd->w = w;
    hd->mu = mu;
    hd->ka = ka;
    hd->partial = partial;
    hd->partial_cap = pcap;
    hd->result = result;
    hd->ctl = reinterpret_cast<int*>(result + 8);
  }
  return c.off;
}

int last_error() { return hipGetLastError() == hipSuccess ? HFZ_OK : HFZ_EHIP; }

void copy_dev(hfz3_handle* hd, const double* a, double* b, size_t count) {
  k3_copy<<<(unsigned)((count + 255) / 256), 256, 0, hd->stream>>>(a, b, count);
}

void smooth(hfz3_handle* hd, int l, int sweeps) {
  const Lvl& L = hd->L[l];
  const Dims d = dims(L.n / 2, L.n);
  for (int k = 0; k < sweeps; ++k)
    for (int colour = 0; colour < 2; ++colour) k3_smooth<<<d.grid, d.block, 0, hd->stream>>>(L, hd->P, colour);
}

void vcycle_rec(hfz3_handle* hd, int l) {
  const int last = (int)hd->L.size() - 1;
  if (l == last) {
    smooth(hd, l, hd->p.coarse_sweeps);
    return;
  }
  const Lvl& F = hd->L[l];
  const Lvl& C = hd->L[l + 1];
  smooth(hd, l, hd->p.nu1);
  const Dims df = dims(F.n, F.n), dc = dims(C.n, C.n);
  k3_residual_field<<<df.grid, df.block, 0, hd->stream>>>(F, hd->P);
  k3_restrict<<<dc.grid, dc.block, 0, hd->stream>>>(F, C, hd->P.halt);
  k3_fas_rhs<<<dc.grid, dc.block, 0, hd->stream>>>(C, hd->P);
  vcycle_rec(hd, l + 1);
  k3_prolong<<<df.grid, df.block, 0, hd->stream>>>(F, C, hd->P.halt);
  smooth(hd, l, hd->p.nu2);
}

void residual_launch(hfz3_handle* hd, bool stop, bool counted) {
  const Lvl& L = hd->L[0];
  const Dims d = dims(L.n, L.n);
  k3_residual_partial<<<d.grid, d.block, 0, hd->stream>>>(L, hd->P, hd->partial);
  const int count = (int)(d.grid.x * d.grid.y);
  const double h3 = L.h * L.h * L.h;
  if (stop)
    k3_reduce_stop<<<1, 1024, 0, hd->stream>>>(hd->partial, count, h3, hd->p.tol, hd->result, hd->ctl,
                                               counted ? 1 : 0);
  else
    k3_reduce<<<1, 1024, 0, hd->stream>>>(hd->partial, count, 1, h3, hd->result);
}

int read_result(hfz3_handle* hd, double* out, int nq) {
  if (hipMemcpyAsync(out, hd->result, nq * sizeof(double), hipMemcpyDeviceToHost, hd->stream) != hipSuccess ||
      hipStreamSynchronize(hd->stream) != hipSuccess)
    return HFZ_EHIP;
  return last_error();
}

int residual(hfz3_handle* hd, double* norm) {
  residual_launch(hd, false, false);
  double r2 = 0.0;
  const int rc = read_result(hd, &r2, 1);
  *norm = std::sqrt(r2);
  return rc;
}

// One V-cycle and its stop-test norm, captured once into a HIP graph on a
// private stream and replayed on the caller's; false when unavailable.
bool cycle_graph(hfz3_handle* hd) {
  if (hd->graph_state == 1) return true;
  if (hd->graph_state < 0) return false;
  hipStream_t cap = nullptr;
  hipGraph_t g = nullptr;
  bool ok = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess;
  if (ok) {
    hipStream_t user = hd->stream;
    hd->stream = cap;
    ok = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
      vcycle_rec(hd, 0);
      residual_launch(hd, true, true);
      ok = hipStreamEndCapture(cap, &g) == hipSuccess;
    }
    hd->stream = user;
  }
  if (ok) ok = hipGraphInstantiate(&hd->cycle_exec, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (cap) (void)hipStreamDestroy(cap);
  (void)hipGetLastError();
  hd->graph_state = ok ? 1 : -1;
  return ok;
}

int begin_step(hfz3_handle* hd) {
  const Lvl& L0 = hd->L[0];
  const Dims d = dims(L0.n, L0.n);
  k3_begin<<<d.grid, d.block, 0, hd->stream>>>(L0, hd->u, hd->v, hd->w, hd->mu, hd->ka, hd->P);
  for (size_t l = 1; l < hd->L.size(); ++l) {
    const Dims dc = dims(hd->L[l].n, hd->L[l].n);
    k3_restrict_coef<<<dc.grid, dc.block, 0, hd->stream>>>(hd->L[l - 1], hd->L[l]);
  }
  return last_error();
}

int finish_step(hfz3_handle* hd) {
  const Lvl& L0 = hd->L[0];
  const Dims d = dims(L0.n, L0.n);
  if (hd->p.continuity_fix) k3_continuity<<<d.grid, d.block, 0, hd->stream>>>(L0, hd->P);
  const size_t N3 = (size_t)L0.n * L0.n * L0.n;
  k3_state<<<(unsigned)((N3 + 255) / 256), 256, 0, hd->stream>>>(L0, hd->u, hd->v, hd->w, hd->mu, hd->ka, N3);
  return last_error();
}

// The solve of one step (the 2D library's scheme): the initial norm and the
// cycle graph run with the device stop test; cycles are enqueued in batches
// (first as many as the previous step needed, then pairs); cycles enqueued
// past the stop return at once.  Without graphs, a host-tested loop.
int solve_step(hfz3_handle* hd, double* r, int* cycles_out) {
  int cycles = 0;
  *cycles_out = 0;
  if (!cycle_graph(hd)) {
    int rc = residual(hd, r);
    while (rc == HFZ_OK && !(*r <= hd->p.tol)) {
      if (!std::isfinite(*r)) return HFZ_ENAN;
      if (cycles >= hd->p.max_cycles) return HFZ_ENOCONV;
      vcycle_rec(hd, 0);
      ++cycles;
      *cycles_out = cycles;
      rc = residual(hd, r);
    }
    return rc;
  }
  k3_ctl_reset<<<1, 64, 0, hd->stream>>>(hd->ctl);
  residual_launch(hd, true, false);
  int rc = HFZ_OK;
  int batch = std::max(1, hd->cycle_hint);
  for (;;) {
    const int nb = std::min(batch, hd->p.max_cycles - cycles);
    for (int i = 0; i < nb && rc == HFZ_OK; ++i)
      if (hipGraphLaunch(hd->cycle_exec, hd->stream) != hipSuccess) rc = HFZ_EHIP;
    if (rc != HFZ_OK) break;
    double hst[10];
    if ((rc = read_result(hd, hst, 10)) != HFZ_OK) break;
    int ctl[2];
    std::memcpy(ctl, &hst[8], sizeof(ctl));
    cycles = ctl[1];
    *r = std::sqrt(hst[0]);
    if (ctl[0] == 1) break;
    if (ctl[0] == 2) {
      rc = HFZ_ENAN;
      break;
    }
    if (cycles >= hd->p.max_cycles) {
      rc = HFZ_ENOCONV;
      break;
    }
    batch = 2;
  }
  k3_ctl_reset<<<1, 64, 0, hd->stream>>>(hd->ctl);
  if (rc == HFZ_OK) hd->cycle_hint = std::max(1, cycles);
  *cycles_out = cycles;
  return rc == HFZ_OK ? last_error() : rc;
}

}  // namespace

extern "C" {

int hfz3_workspace_bytes(const hfz_params* p, size_t* bytes) {
  const int rc = validate3(p);
  if (rc != HFZ_OK) return rc;
  if (!bytes) return HFZ_EINVAL;
  *bytes = layout3(*p, nullptr, nullptr);
  return HFZ_OK;
}

int hfz3_init(const hfz_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, hfz3_handle** out) {
  if (!out) return HFZ_EINVAL;
  *out = nullptr;
  const int rc = validate3(p);
  if (rc != HFZ_OK) return rc;
  if (!dev_ws || ws_bytes < layout3(*p, nullptr, nullptr)) return HFZ_ENOMEM;
  if (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) return HFZ_EINVAL;
  hfz3_handle* hd = new (std::nothrow) hfz3_handle();
  if (!hd) return HFZ_ENOMEM;
  hd->p = *p;
  hd->stream = static_cast<hipStream_t>(hip_stream);
  layout3(*p, dev_ws, hd);
  hd->P.s = p->s;
  hd->P.gamma = p->gamma;
  hd->P.sigma = (double)p->sigma;
  hd->P.alpha = p->alpha;
  hd->P.w = p->w_damp;
  hd->P.halt = hd->ctl;
  k3_ctl_reset<<<1, 64, 0, hd->stream>>>(hd->ctl);
  if (hipStreamSynchronize(hd->stream) != hipSuccess || last_error() != HFZ_OK) {
    delete hd;
    return HFZ_EHIP;
  }
  *out = hd;
  return HFZ_OK;
}

int hfz3_set_state(hfz3_handle* hd, const double* rho, const double* u, const double* v, const double* w) {
  if (!hd || !rho || !u || !v || !w) return HFZ_EINVAL;
  const Lvl& L0 = hd->L[0];
  const size_t N3 = (size_t)L0.n * L0.n * L0.n;
  copy_dev(hd, rho, L0.rk, N3);
  copy_dev(hd, u, hd->u, N3);
  copy_dev(hd, v, hd->v, N3);
  copy_dev(hd, w, hd->w, N3);
  const Dims d = dims(L0.n, L0.n);
  k3_kappa<<<d.grid, d.block, 0, hd->stream>>>(L0.rk, hd->ka, L0.n, L0.lg, L0.h);
  k3_mu<<<d.grid, d.block, 0, hd->stream>>>(L0.rk, hd->ka, hd->mu, L0.n, L0.lg, L0.h, hd->p.alpha);
  if (hipStreamSynchronize(hd->stream) != hipSuccess) return HFZ_EHIP;
  hd->has_state = true;
  return last_error();
}

int hfz3_get_state(hfz3_handle* hd, double* rho, double* u, double* v, double* w) {
  if (!hd || !rho || !u || !v || !w) return HFZ_EINVAL;
  if (!hd->has_state) return HFZ_ESTATE;
  const Lvl& L0 = hd->L[0];
  const size_t N3 = (size_t)L0.n * L0.n * L0.n;
  copy_dev(hd, L0.rk, rho, N3);
  copy_dev(hd, hd->u, u, N3);
  copy_dev(hd, hd->v, v, N3);
  copy_dev(hd, hd->w, w, N3);
  if (hipStreamSynchronize(hd->stream) != hipSuccess) return HFZ_EHIP;
  return last_error();
}

int hfz3_step(hfz3_handle* hd, int nsteps, hfz_stats* stats) {
  if (!hd || nsteps < 0) return HFZ_EINVAL;
  if (!hd->has_state) return HFZ_ESTATE;
  hfz_stats st{};
  int rc = HFZ_OK;
  for (int k = 0; k < nsteps; ++k) {
    if ((rc = begin_step(hd)) != HFZ_OK) break;
    double r = 0.0;
    int cycles = 0;
    rc = solve_step(hd, &r, &cycles);
    st.cycles_last = cycles;
    st.residual_last = r;
    if (rc != HFZ_OK) break;
    if ((rc = finish_step(hd)) != HFZ_OK) break;
    st.steps_done++;
    st.cycles_total += cycles;
  }
  if (rc == HFZ_OK && hipStreamSynchronize(hd->stream) != hipSuccess) rc = HFZ_EHIP;
  if (stats) *stats = st;
  return rc;
}

int hfz3_energy(hfz3_handle* hd, double* out3) {
  if (!hd || !out3) return HFZ_EINVAL;
  if (!hd->has_state) return HFZ_ESTATE;
  const Lvl& L0 = hd->L[0];
  const Dims d = dims(L0.n, L0.n);
  k3_energy_partial<<<d.grid, d.block, 0, hd->stream>>>(L0.rk, hd->u, hd->v, hd->w, L0.n, L0.lg, L0.h,
                                                         hd->p.alpha, hd->partial);
  const double h3 = L0.h * L0.h * L0.h;
  k3_reduce<<<1, 1024, 0, hd->stream>>>(hd->partial, (int)(d.grid.x * d.grid.y), 3, h3, hd->result);
  double q[3];
  const int rc = read_result(hd, q, 3);
  if (rc != HFZ_OK) return rc;
  out3[0] = q[0] + q[1];
  out3[1] = q[0];
  out3[2] = q[1];
  return std::isfinite(out3[0]) ? HFZ_OK : HFZ_ENAN;
}

int hfz3_mass(hfz3_handle* hd, double* mass) {
  if (!hd || !mass) return HFZ_EINVAL;
  if (!hd->has_state) return HFZ_ESTATE;
  const Lvl& L0 = hd->L[0];
  const Dims d = dims(L0.n, L0.n);
  k3_energy_partial<<<d.grid, d.block, 0, hd->stream>>>(L0.rk, hd->u, hd->v, hd->w, L0.n, L0.lg, L0.h,
                                                         hd->p.alpha, hd->partial);
  const double h3 = L0.h * L0.h * L0.h;
  k3_reduce<<<1, 1024, 0, hd->stream>>>(hd->partial, (int)(d.grid.x * d.grid.y), 3, h3, hd->result);
  double q[3];
  const int rc = read_result(hd, q, 3);
  *mass = q[2];
  return rc;
}

int hfz3_begin_step(hfz3_handle* hd) {
  if (!hd) return HFZ_EINVAL;
  if (!hd->has_state) return HFZ_ESTATE;
  return begin_step(hd);
}

int hfz3_smooth(hfz3_handle* hd, int level, int sweeps) {
  if (!hd || level < 0 || level >= (int)hd->L.size() || sweeps < 0) return HFZ_EINVAL;
  smooth(hd, level, sweeps);
  return last_error();
}

int hfz3_vcycle(hfz3_handle* hd, int count) {
  if (!hd || count < 0) return HFZ_EINVAL;
  for (int k = 0; k < count; ++k) vcycle_rec(hd, 0);
  return last_error();
}

int hfz3_residual(hfz3_handle* hd, double* norm) {
  if (!hd || !norm) return HFZ_EINVAL;
  return residual(hd, norm);
}

int hfz3_finish_step(hfz3_handle* hd) {
  if (!hd) return HFZ_EINVAL;
  return finish_step(hd);
}

int hfz3_read_field(hfz3_handle* hd, int which, int level, int comp, double* dst) {
  if (!hd || !dst || level < 0 || level >= (int)hd->L.size()) return HFZ_EINVAL;
  const Lvl& L = hd->L[level];
  const double* src = nullptr;
  if (which == 0 && comp >= 0 && comp < NC) src = L.g[comp];
  if (which == 1 && comp >= 0 && comp < NC) src = L.f[comp];
  if (which == 3 && comp == 0) src = L.rk;
  if (which == 3 && comp >= 1 && comp <= 3) src = L.om[comp - 1];
  if (which == 5 && level == 0 && comp == 0) src = hd->mu;
  if (which == 5 && level == 0 && comp == 1) src = hd->ka;
  if (!src) return HFZ_EINVAL;
  copy_dev(hd, src, dst, (size_t)L.n * L.n * L.n);
  if (hipStreamSynchronize(hd->stream) != hipSuccess) return HFZ_EHIP;
  return last_error();
}

int hfz3_levels(hfz3_handle* hd, int* levels) {
  if (!hd || !levels) return HFZ_EINVAL;
  *levels = (int)hd->L.size();
  return HFZ_OK;
}

int hfz3_destroy(hfz3_handle* hd) {
  if (!hd) return HFZ_EINVAL;
  if (hd->cycle_exec) (void)hipGraphExecDestroy(hd->cycle_exec);
  delete hd;
  return HFZ_OK;
}

}  // extern "C"
