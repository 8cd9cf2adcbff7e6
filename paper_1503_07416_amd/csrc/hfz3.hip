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
// One thread per node in the per-level kernels (per node of a colour in the
// small levels' smoother); on the large levels one launch of a z-marching
// tiled kernel does a whole sweep through an LDS window (k3_sweep_tile).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "hfz.h"

namespace hfz3 {

constexpr int NC = 6;

struct Lvl {
  double* g[NC];   // iterate
  double* f[NC];   // right-hand side (level 0: the source S)
  double* g0[NC];  // restricted iterate R g (coarse levels)
  double* d[NC];   // residual f - N(g) before restriction
  double* gb[NC];  // second iterate buffer of the tiled sweep (levels it runs on)
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

// rho^k on the 7-point stencil, omega^k and f at one node.
struct Coef {
  double rk[7];
  double om[3];
  double f[NC];
};

__device__ __forceinline__ void load_coef(const Lvl& L, const Nbr& q, Coef& C) {
  const int k[7] = {q.p, q.e, q.w, q.n, q.s, q.u, q.d};
#pragma unroll
  for (int t = 0; t < 7; ++t) C.rk[t] = L.rk[k[t]];
#pragma unroll
  for (int c = 0; c < 3; ++c) C.om[c] = L.om[c][q.p];
#pragma unroll
  for (int c = 0; c < NC; ++c) C.f[c] = L.f[c][q.p];
}

// The values a block update reads, gathered: v[c][k] is component c at the
// node (k = 0) and its neighbours +x, -x, +y, -y, +z, -z (k = 1..6); rk the
// same for rho^k; om and f at the node.
struct Gath {
  double v[NC][7];
  double rk[7];
  double om[3];
  double f[NC];
};

__device__ __forceinline__ double s6(const double* a) { return a[1] + a[2] + a[3] + a[4] + a[5] + a[6]; }

__device__ __forceinline__ double q2v(const Gath& G, int k) {
  return G.v[1][k] * G.v[1][k] + G.v[2][k] * G.v[2][k] + G.v[3][k] * G.v[3][k];
}

// Damped block update from gathered values (module comment).
__device__ __forceinline__ void block_vals(const Gath& G, double h, const Phys& P, double* out) {
  const double s = P.s, c4 = s / (4.0 * h), c2 = s / (2.0 * h), ih2 = 1.0 / (h * h);
  const double* rk = G.rk;
  const double* u = G.v[1];
  const double* v = G.v[2];
  const double* w = G.v[3];
  const double* mu = G.v[4];
  const double rh = G.f[0] - c4 * (rk[1] * u[1] - rk[2] * u[2] + rk[3] * v[3] - rk[4] * v[4] + rk[5] * w[5] -
                                   rk[6] * w[6]);
  const double rkP = rk[0];
  const double cg = 0.5 * s * P.gamma * ih2;
  const double a = rkP + 6.0 * cg;
  const double bs = 0.5 * s * P.sigma * rkP;
  const double b0 = bs * G.om[0], b1 = bs * G.om[1], b2 = bs * G.om[2];
  const double r0 = G.f[1] - c4 * rkP * (q2v(G, 1) - q2v(G, 2)) - c2 * rkP * (mu[1] - mu[2]) + cg * s6(u);
  const double r1 = G.f[2] - c4 * rkP * (q2v(G, 3) - q2v(G, 4)) - c2 * rkP * (mu[3] - mu[4]) + cg * s6(v);
  const double r2 = G.f[3] - c4 * rkP * (q2v(G, 5) - q2v(G, 6)) - c2 * rkP * (mu[5] - mu[6]) + cg * s6(w);
  const double bb = b0 * b0 + b1 * b1 + b2 * b2;
  const double br = b0 * r0 + b1 * r1 + b2 * r2;
  const double x0 = b1 * r2 - b2 * r1, x1 = b2 * r0 - b0 * r2, x2 = b0 * r1 - b1 * r0;
  const double den = a * (a * a + bb);
  const double uh = (a * a * r0 - a * x0 + br * b0) / den;
  const double vh = (a * a * r1 - a * x1 + br * b1) / den;
  const double wh = (a * a * r2 - a * x2 + br * b2) / den;
  const double kh = G.f[5] + s6(G.v[0]) * ih2 - 6.0 * rh * ih2;
  const double pl = G.v[0][0] - 1.5;
  const double mh = G.f[4] + (P.alpha + pl * pl) * (rh - 1.5) - (2.0 / 3.0) * pl * pl * pl + s6(G.v[5]) * ih2 -
                    6.0 * kh * ih2;
  const double wd = P.w, w1 = 1.0 - P.w;
  out[0] = w1 * rh + wd * G.v[0][0];
  out[1] = w1 * uh + wd * u[0];
  out[2] = w1 * vh + wd * v[0];
  out[3] = w1 * wh + wd * w[0];
  out[4] = w1 * mh + wd * mu[0];
  out[5] = w1 * kh + wd * G.v[5][0];
}

__device__ __forceinline__ void put_coef(const Coef& C, Gath& G) {
#pragma unroll
  for (int k = 0; k < 7; ++k) G.rk[k] = C.rk[k];
#pragma unroll
  for (int c = 0; c < 3; ++c) G.om[c] = C.om[c];
#pragma unroll
  for (int c = 0; c < NC; ++c) G.f[c] = C.f[c];
}

// Rows of N(g) from gathered values (same arithmetic as rows()).
__device__ __forceinline__ void rows_vals(const Gath& G, double h, const Phys& P, double* out) {
  const double s = P.s, c4 = s / (4.0 * h), c2 = s / (2.0 * h), ih2 = 1.0 / (h * h);
  const double* rk = G.rk;
  const double* u = G.v[1];
  const double* v = G.v[2];
  const double* w = G.v[3];
  const double* mu = G.v[4];
  out[0] = G.v[0][0] + c4 * (rk[1] * u[1] - rk[2] * u[2] + rk[3] * v[3] - rk[4] * v[4] + rk[5] * w[5] - rk[6] * w[6]);
  const double rkP = rk[0];
  const double o0 = G.om[0], o1 = G.om[1], o2 = G.om[2];
  const double uP = u[0], vP = v[0], wP = w[0];
  const double cx = o1 * wP - o2 * vP, cy = o2 * uP - o0 * wP, cz = o0 * vP - o1 * uP;
  const double bs = 0.5 * s * P.sigma * rkP, gl = 0.5 * s * P.gamma * ih2;
  out[1] = rkP * uP + bs * cx + c4 * rkP * (q2v(G, 1) - q2v(G, 2)) + c2 * rkP * (mu[1] - mu[2]) - gl * (s6(u) - 6.0 * uP);
  out[2] = rkP * vP + bs * cy + c4 * rkP * (q2v(G, 3) - q2v(G, 4)) + c2 * rkP * (mu[3] - mu[4]) - gl * (s6(v) - 6.0 * vP);
  out[3] = rkP * wP + bs * cz + c4 * rkP * (q2v(G, 5) - q2v(G, 6)) + c2 * rkP * (mu[5] - mu[6]) - gl * (s6(w) - 6.0 * wP);
  const double phi = G.v[0][0] - 1.5;
  out[4] = mu[0] - phi * phi * phi * (1.0 / 3.0) - P.alpha * phi - (s6(G.v[5]) - 6.0 * G.v[5][0]) * ih2;
  out[5] = G.v[5][0] - (s6(G.v[0]) - 6.0 * G.v[0][0]) * ih2;
}

// The 7-point values of field f at the x pair (i0, i0 + 1) (i0 even) of the
// row at `row` (its j-neighbour rows yn, ys and l-neighbour rows zu, zd):
// seven aligned 16-byte loads give both nodes' stencils, a for i0, b for i0 + 1.
__device__ __forceinline__ void pair7(const double* f, int row, int yn, int ys, int zu, int zd, int i0, int m,
                                      double* a, double* b) {
  const double2 P0 = *reinterpret_cast<const double2*>(f + row + i0);
  const double2 PL = *reinterpret_cast<const double2*>(f + row + ((i0 - 2) & m));
  const double2 PR = *reinterpret_cast<const double2*>(f + row + ((i0 + 2) & m));
  const double2 N = *reinterpret_cast<const double2*>(f + yn + i0);
  const double2 S = *reinterpret_cast<const double2*>(f + ys + i0);
  const double2 U = *reinterpret_cast<const double2*>(f + zu + i0);
  const double2 D = *reinterpret_cast<const double2*>(f + zd + i0);
  a[0] = P0.x, a[1] = P0.y, a[2] = PL.y, a[3] = N.x, a[4] = S.x, a[5] = U.x, a[6] = D.x;
  b[0] = P0.y, b[1] = PR.x, b[2] = P0.x, b[3] = N.y, b[4] = S.y, b[5] = U.y, b[6] = D.y;
}

// Rows of N(g) at the x pair (i0, i0 + 1) of row (j, l), from 16-byte loads.
__device__ __forceinline__ void rows_pair(const Lvl& L, const Phys& P, double* const* g, int i0, int j, int l,
                                          double* na, double* nb, int& pa) {
  const int n = L.n, m = n - 1, lg = L.lg;
  const int row = ((l << lg) + j) << lg;
  const int yn = ((l << lg) + ((j + 1) & m)) << lg, ys = ((l << lg) + ((j - 1) & m)) << lg;
  const int zu = ((((l + 1) & m) << lg) + j) << lg, zd = ((((l - 1) & m) << lg) + j) << lg;
  Gath A, B;
#pragma unroll
  for (int c = 0; c < NC; ++c) pair7(g[c], row, yn, ys, zu, zd, i0, m, A.v[c], B.v[c]);
  pair7(L.rk, row, yn, ys, zu, zd, i0, m, A.rk, B.rk);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double2 o = *reinterpret_cast<const double2*>(L.om[c] + row + i0);
    A.om[c] = o.x;
    B.om[c] = o.y;
  }
  rows_vals(A, L.h, P, na);
  rows_vals(B, L.h, P, nb);
  pa = row + i0;
}

// Damped block update at node q of the iterate g.
__device__ __forceinline__ void block(const Lvl& L, const Phys& P, double* const* g, const Nbr& q, double* out) {
  Coef C;
  load_coef(L, q, C);
  Gath G;
  put_coef(C, G);
  const int k[7] = {q.p, q.e, q.w, q.n, q.s, q.u, q.d};
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int t = 0; t < 7; ++t) G.v[c][t] = g[c][k[t]];
  block_vals(G, L.h, P, out);
}

// 27-point full weighting at coarse node (I, J, K) = fine (2I, 2J, 2K).  Each
// fine row's values 2I - 1, 2I, 2I + 1 come from two aligned 16-byte vectors,
// the pairs (2I - 2, 2I - 1) and (2I, 2I + 1).
__device__ __forceinline__ double fw27(const double* f, int I, int J, int K, int lgf) {
  const int m = (1 << lgf) - 1;
  double acc = 0.0;
#pragma unroll
  for (int dk = -1; dk <= 1; ++dk) {
    const int k = (2 * K + dk) & m;
    const double wk = dk == 0 ? 2.0 : 1.0;
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const int j = (2 * J + dj) & m;
      const double wj = dj == 0 ? 2.0 : 1.0;
      const int row = ((k << lgf) + j) << lgf;
      const double2 a = *reinterpret_cast<const double2*>(f + row + ((2 * I - 2) & m));
      const double2 v = *reinterpret_cast<const double2*>(f + row + 2 * I);
      acc += wk * wj * (a.y + 2.0 * v.x + v.y);
    }
  }
  return acc * (1.0 / 64.0);
}

struct Idx {
  int i, j, l, ok;
};

// Thread -> node of an n^3 level in 2D launch geometry (x in blockIdx.x, the
// (y, z) rows in blockIdx.y).  Workgroups are renumbered so that each XCD
// (workgroups are dealt to the 8 XCDs in turn) takes a contiguous range of
// rows, whose y and z neighbour rows then mostly sit in that XCD's L2.
// (node_x: nx nodes per row, n^2 rows.)
__device__ __forceinline__ Idx node_x(int nx, int n, int lg) {
  Idx x;
  const int nbx = (int)gridDim.x, nb = nbx * (int)gridDim.y;
  const int bid = (int)blockIdx.y * nbx + (int)blockIdx.x;
  const int b = (nb & 7) ? bid : (bid & 7) * (nb >> 3) + (bid >> 3);
  x.i = (b % nbx) * blockDim.x + threadIdx.x;
  const int row = (b / nbx) * blockDim.y + threadIdx.y;
  x.j = row & (n - 1);
  x.l = row >> lg;
  x.ok = x.i < nx && row < n * n;
  return x;
}

__device__ __forceinline__ Idx node(int n, int lg) { return node_x(n, n, lg); }

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
#pragma unroll
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
  block(L, P, L.g, q, out);
#pragma unroll
  for (int c = 0; c < NC; ++c) L.g[c][q.p] = out[c];
}

// One damped red-black sweep in one launch (levels from 128^3 up by default).
//
// A workgroup owns a TX x TY tile of the x-y plane and ZC planes in z and
// marches up them.  The sweep's starting iterate gin passes through a
// four-plane LDS window over the tile plus a two-node ring; each window plane
// is read from gin once.  At plane l the workgroup
//   * updates the red nodes (i + j + l + 1 even) of plane l + 1 over the tile
//     and a one-node ring, in place in the window: a red update reads only
//     black values of its own plane and of planes l and l + 2, and its own old
//     value, so in-place writes race with no other red update;
//   * updates the black nodes of plane l over the tile from the window (their
//     neighbours are red, now new) and their own old value, and writes plane
//     l of the tile, red and black, to gout.
// Before its first plane it updates the red nodes of planes z0 - 1 and z0.
// The ring's red nodes are recomputed by the workgroups on both sides; gin is
// never written, so all of them read the same starting iterate.  The next
// window plane is loaded into registers one plane ahead, each phase's
// coefficients (rho^k at the 7-point stencil, omega^k, f) one phase ahead.
// Workgroups are numbered so that each XCD (workgroups are dealt to the 8
// XCDs in turn) takes a contiguous range of tiles, whose rings then overlap
// in that XCD's L2.
constexpr int TX3 = 32, TY3 = 16, ZC3 = 16, NT3 = 512;
constexpr int WX3 = TX3 + 4, WY3 = TY3 + 4, WP3 = WX3 * WY3;  // window plane (tile + 2-node ring)
constexpr int RX3 = TX3 + 2, RY3 = TY3 + 2;                    // red region (tile + 1-node ring)
constexpr int NRED3 = RX3 * RY3 / 2, NBLK3 = TX3 * TY3 / 2;   // red region nodes, tile nodes of a colour
constexpr int LDPT3 = (WP3 + NT3 - 1) / NT3;                   // window nodes per thread
static_assert(NRED3 <= NT3 && 2 * NBLK3 == NT3 && RX3 % 2 == 0 && TX3 % 2 == 0, "tile shape");

struct G6 {
  double* c[NC];
};

// Window coordinates (a, b) of the red node r (x + y + p even, par = x0 + y0 +
// p) of the tile plus one-node ring; the ring offsets are even and n is even,
// so the periodic wrap keeps parities.
__device__ __forceinline__ void red_pos(int r, int par, int& a, int& b) {
  b = r / (RX3 / 2);
  a = 2 * (r - b * (RX3 / 2)) + ((par + b) & 1);
  a += 1;
  b += 1;
}

// Window coordinates of the tile node r whose x + y + p has the parity of par.
__device__ __forceinline__ void tile_pos(int r, int par, int& a, int& b) {
  b = r / (TX3 / 2);
  a = 2 * (r - b * (TX3 / 2)) + ((par + b) & 1);
  a += 2;
  b += 2;
}

__global__ __launch_bounds__(NT3) void k3_sweep_tile(Lvl L, G6 gin, G6 gout, Phys P) {
  if (halted(P.halt)) return;
  __shared__ double win[4][NC][WP3];
  const int m = L.n - 1, lg = L.lg;
  // XCD-contiguous tile numbering
  const int ntx = L.n / TX3, nty = L.n / TY3, nb = ntx * nty * (L.n / ZC3);
  const int bid = (int)blockIdx.x;
  const int tid = (nb & 7) ? bid : (bid & 7) * (nb >> 3) + (bid >> 3);
  const int tx = tid % ntx, ty = (tid / ntx) % nty, tz = tid / (ntx * nty);
  const int x0 = tx * TX3, y0 = ty * TY3, z0 = tz * ZC3;
  const int t = threadIdx.x;
  auto slot = [&](int p) { return (p - z0 + 8) & 3; };
  auto gidx = [&](int a, int b, int p) { return ((((p & m) << lg) + ((y0 - 2 + b) & m)) << lg) + ((x0 - 2 + a) & m); };
  auto gnbr = [&](int a, int b, int p) { return nbr((x0 - 2 + a) & m, (y0 - 2 + b) & m, p & m, lg); };
  // window loads through registers
  double pre[LDPT3][NC];
  auto fetch = [&](int p) {
#pragma unroll
    for (int k = 0; k < LDPT3; ++k) {
      const int w = t + k * NT3;
      if (w < WP3) {
        const int b = w / WX3, a = w - b * WX3;
        const int gi = gidx(a, b, p);
#pragma unroll
        for (int c = 0; c < NC; ++c) pre[k][c] = gin.c[c][gi];
      }
    }
  };
  auto store = [&](int p) {
    const int sl = slot(p);
#pragma unroll
    for (int k = 0; k < LDPT3; ++k) {
      const int w = t + k * NT3;
      if (w < WP3) {
#pragma unroll
        for (int c = 0; c < NC; ++c) win[sl][c][w] = pre[k][c];
      }
    }
  };
  // the update of the node at window (a, b) of plane p from the window
  auto update = [&](int a, int b, int p, const Coef& C, double* out) {
    const int w = b * WX3 + a, sc = slot(p), su = slot(p + 1), sd = slot(p - 1);
    Gath G;
    put_coef(C, G);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      G.v[c][0] = win[sc][c][w];
      G.v[c][1] = win[sc][c][w + 1];
      G.v[c][2] = win[sc][c][w - 1];
      G.v[c][3] = win[sc][c][w + WX3];
      G.v[c][4] = win[sc][c][w - WX3];
      G.v[c][5] = win[su][c][w];
      G.v[c][6] = win[sd][c][w];
    }
    block_vals(G, L.h, P, out);
  };
  // red node of this thread at plane p: coefficients, then the in-place update
  const bool has_red = t < NRED3;
  auto red_coef = [&](int p, Coef& C) {
    if (has_red) {
      int a, b;
      red_pos(t, x0 + y0 + p, a, b);
      load_coef(L, gnbr(a, b, p), C);
    }
  };
  auto red_update = [&](int p, const Coef& C) {
    if (has_red) {
      int a, b;
      red_pos(t, x0 + y0 + p, a, b);
      double out[NC];
      update(a, b, p, C, out);
      const int w = b * WX3 + a, sc = slot(p);
#pragma unroll
      for (int c = 0; c < NC; ++c) win[sc][c][w] = out[c];
    }
  };
  // black half of the threads: the black tile nodes; red half: copies the red tile nodes
  const bool is_black = t < NBLK3;
  const int r = is_black ? t : t - NBLK3;
  auto black_coef = [&](int p, Coef& C) {
    if (is_black) {
      int a, b;
      tile_pos(r, x0 + y0 + p + 1, a, b);
      load_coef(L, gnbr(a, b, p), C);
    }
  };
  auto finish_plane = [&](int p, const Coef& C) {
    int a, b;
    tile_pos(r, x0 + y0 + p + (is_black ? 1 : 0), a, b);
    double out[NC];
    if (is_black) {
      update(a, b, p, C, out);
    } else {
      const int w = b * WX3 + a, sc = slot(p);
#pragma unroll
      for (int c = 0; c < NC; ++c) out[c] = win[sc][c][w];
    }
    const int gi = gidx(a, b, p);
#pragma unroll
    for (int c = 0; c < NC; ++c) gout.c[c][gi] = out[c];
  };

  // prologue: planes z0 - 2 .. z0 + 1, red of planes z0 - 1 and z0
  Coef cr, cb;
  {
    Coef c0, c1;
    red_coef(z0 - 1, c0);
    red_coef(z0, c1);
    for (int p = z0 - 2; p <= z0 + 1; ++p) {
      fetch(p);
      store(p);
    }
    __syncthreads();
    red_update(z0 - 1, c0);
    red_update(z0, c1);
  }
  red_coef(z0 + 1, cr);
  fetch(z0 + 2);
  __syncthreads();
  // each phase's coefficients are loaded during the phase before it
  for (int k = 0; k < ZC3; ++k) {
    const int l = z0 + k;
    store(l + 2);  // its slot held plane l - 2, last read before the previous barrier
    if (k + 1 < ZC3) fetch(l + 3);
    black_coef(l, cb);
    __syncthreads();
    red_update(l + 1, cr);
    if (k + 1 < ZC3) red_coef(l + 2, cr);
    __syncthreads();
    finish_plane(l, cb);
    __syncthreads();
  }
}

// d = f - N(g).
__device__ __forceinline__ void residual_node(const Lvl& L, const Phys& P, int i, int j, int l) {
  const Nbr q = nbr(i, j, l, L.lg);
  double nv[NC];
  rows(L, P, L.g, q, nv);
#pragma unroll
  for (int c = 0; c < NC; ++c) L.d[c][q.p] = L.f[c][q.p] - nv[c];
}

// d = f - N(g), one thread per x pair of nodes (launch geometry of n/2 x n^2).
__global__ __launch_bounds__(256) void k3_residual_field(Lvl L, Phys P) {
  if (halted(P.halt)) return;
  const Idx x = node_x(L.n >> 1, L.n, L.lg);
  if (!x.ok) return;
  double na[NC], nb[NC];
  int pa;
  rows_pair(L, P, L.g, 2 * x.i, x.j, x.l, na, nb, pa);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double2 f = *reinterpret_cast<const double2*>(L.f[c] + pa);
    *reinterpret_cast<double2*>(L.d[c] + pa) = make_double2(f.x - na[c], f.y - nb[c]);
  }
}

// g_c = g0_c = R g, f_c = R d at coarse node (I, J, K).
__device__ __forceinline__ void restrict_node(const Lvl& F, const Lvl& C, int I, int J, int K) {
  const int pc = (((K << C.lg) + J) << C.lg) + I;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double gr = fw27(F.g[c], I, J, K, F.lg);
    C.g[c][pc] = gr;
    C.g0[c][pc] = gr;
    C.f[c][pc] = fw27(F.d[c], I, J, K, F.lg);
  }
}

__global__ void k3_restrict(Lvl F, Lvl C, const int* halt) {
  if (halted(halt)) return;
  const Idx x = node(C.n, C.lg);
  if (!x.ok) return;
  restrict_node(F, C, x.i, x.j, x.l);
}

// f_c += N_c(R g).
__device__ __forceinline__ void fas_rhs_node(const Lvl& C, const Phys& P, int i, int j, int l) {
  const Nbr q = nbr(i, j, l, C.lg);
  double nv[NC];
  rows(C, P, C.g0, q, nv);
#pragma unroll
  for (int c = 0; c < NC; ++c) C.f[c][q.p] += nv[c];
}

__global__ void k3_fas_rhs(Lvl C, Phys P) {
  if (halted(P.halt)) return;
  const Idx x = node(C.n, C.lg);
  if (!x.ok) return;
  fas_rhs_node(C, P, x.i, x.j, x.l);
}

// g += P (g_c - g0), trilinear.  One thread per coarse node (I, J, K) adds the
// interpolated correction at the eight fine nodes (2I + a, 2J + b, 2K + c),
// a, b, c in {0, 1}, whose stencils lie in the coarse cell from (I, J, K) to
// (I + 1, J + 1, K + 1): averages along x, then y, then z, with the second
// corner equal to the first where the offset is 0 (a coincident node enters
// with weight 1).  The x pairs are read and written as 16-byte vectors.
__device__ __forceinline__ void prolong_cell(const Lvl& F, const Lvl& C, int I, int J, int K) {
  const int mc = C.n - 1, lc = C.lg, lf = F.lg;
  const int I1 = (I + 1) & mc, J1 = (J + 1) & mc, K1 = (K + 1) & mc;
  auto at = [&](int ii, int jj, int kk) { return (((kk << lc) + jj) << lc) + ii; };
  // corner (di, dj, dk) at index di + 2 dj + 4 dk
  const int cc[8] = {at(I, J, K), at(I1, J, K), at(I, J1, K), at(I1, J1, K),
                     at(I, J, K1),  at(I1, J, K1),  at(I, J1, K1),  at(I1, J1, K1)};
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double e[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) e[k] = C.g[c][cc[k]] - C.g0[c][cc[k]];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int cz = 0; cz < 2; ++cz) {
        double v[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const double ex00 = 0.5 * (e[0] + e[a]), ex10 = 0.5 * (e[2 * b] + e[a + 2 * b]);
          const double ex01 = 0.5 * (e[4 * cz] + e[a + 4 * cz]), ex11 = 0.5 * (e[2 * b + 4 * cz] + e[a + 2 * b + 4 * cz]);
          const double exy0 = 0.5 * (ex00 + ex10), exy1 = 0.5 * (ex01 + ex11);
          v[a] = 0.5 * (exy0 + exy1);
        }
        const int pf = ((((2 * K + cz) << lf) + 2 * J + b) << lf) + 2 * I;
        double2* q = reinterpret_cast<double2*>(F.g[c] + pf);
        double2 o = *q;
        o.x += v[0];
        o.y += v[1];
        *q = o;
      }
  }
}

__global__ void k3_prolong(Lvl F, Lvl C, const int* halt) {
  if (halted(halt)) return;
  const Idx x = node(C.n, C.lg);
  if (!x.ok) return;
  prolong_cell(F, C, x.i, x.j, x.l);
}

// The coarse end of the V-cycle in one workgroup: from the tail top (8^3 or
// smaller) down to the coarsest grid and back, every phase (a smoother
// colour, the residual, restriction, the coarse right-hand side, the
// coarsest sweeps, prolongation) runs over the level's nodes in a loop of
// the workgroup's threads, with a workgroup barrier between phases instead
// of a kernel boundary.  Every tail level lives in LDS for the kernel's
// duration: the top level's g, f and every level's rho^k, omega^k are loaded
// once, the top level's g is written back at the end.  The per-node
// arithmetic is that of the per-level kernels (the same expressions), so the
// results agree with theirs to rounding.
constexpr int TAIL3_TOP = 8, TAIL3_THREADS = 512, TAIL3_MAX = 4;
constexpr int TAIL3_LDS = 13312;  // doubles: an 8^3 top and two coarser levels need 13232

// LDS doubles of tail level l of nt (size n): g, f, rho^k, omega^k; g0 below
// the top; d above the coarsest.
__host__ __device__ inline int tail3_count(int n, int l, int nt) {
  return n * n * n * (2 * NC + 4 + (l > 0 ? NC : 0) + (l < nt - 1 ? NC : 0));
}

struct Tail3 {
  const Lvl* L;  // device array: the tail's levels (global arrays), top first
  int nt, nu1, nu2, coarse_sweeps;
};

__device__ __forceinline__ double* lds_ptr(double* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_assume(__builtin_amdgcn_is_shared((const void*)p));
#endif
  return p;
}

__device__ __forceinline__ double* glb_ptr(double* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return (double*)((__attribute__((address_space(1))) double*)(uintptr_t)p);
#else
  return p;
#endif
}

// The LDS view of a tail level built by k3_tail.
__device__ __forceinline__ Lvl lds_view(const Lvl& s) {
  Lvl L = s;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    L.g[c] = lds_ptr(s.g[c]);
    L.f[c] = lds_ptr(s.f[c]);
    L.g0[c] = lds_ptr(s.g0[c]);
    L.d[c] = lds_ptr(s.d[c]);
  }
  L.rk = lds_ptr(s.rk);
#pragma unroll
  for (int c = 0; c < 3; ++c) L.om[c] = lds_ptr(s.om[c]);
  return L;
}

__device__ void t3_colour(const Lvl& L, const Phys& P, int colour) {
  const int n = L.n, cnt = (n >> 1) * n * n, lh = L.lg - 1;
  for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
    const int t = w & ((1 << lh) - 1), row = w >> lh;
    const int j = row & (n - 1), l = row >> L.lg;
    const Nbr q = nbr(2 * t + ((j + l + colour) & 1), j, l, L.lg);
    double out[NC];
    block(L, P, L.g, q, out);
#pragma unroll
    for (int c = 0; c < NC; ++c) L.g[c][q.p] = out[c];
  }
  __syncthreads();
}

__device__ void t3_sweeps(const Lvl& L, const Phys& P, int sweeps) {
  for (int k = 0; k < sweeps; ++k) {
    t3_colour(L, P, 0);
    t3_colour(L, P, 1);
  }
}

// each loop covers the nodes i fastest, then j, then l
#define T3_NODES(L_, i_, j_, l_, body)                                         \
  for (int w_ = threadIdx.x; w_ < (L_).n * (L_).n * (L_).n; w_ += blockDim.x) { \
    const int i_ = w_ & ((L_).n - 1), j_ = (w_ >> (L_).lg) & ((L_).n - 1);     \
    const int l_ = w_ >> (2 * (L_).lg);                                        \
    body;                                                                      \
  }                                                                            \
  __syncthreads();

__global__ __launch_bounds__(TAIL3_THREADS) void k3_tail(Tail3 T, Phys P) {
  if (halted(P.halt)) return;
  __shared__ __align__(16) double smem[TAIL3_LDS];
  __shared__ Lvl S[TAIL3_MAX];
  const int t = threadIdx.x;
  if (t < T.nt) {
    // thread t lays out level t's LDS arrays (in the order of tail3_count)
    Lvl s = T.L[t];
    int off = 0;
    for (int l = 0; l < t; ++l) off += tail3_count(T.L[l].n, l, T.nt);
    double* p = smem + off;
    const int cnt = s.n * s.n * s.n;
    for (int c = 0; c < NC; ++c, p += cnt) s.g[c] = p;
    for (int c = 0; c < NC; ++c, p += cnt) s.f[c] = p;
    s.rk = p;
    p += cnt;
    for (int c = 0; c < 3; ++c, p += cnt) s.om[c] = p;
    // arrays a level does not have point at the LDS base (lds_view assumes
    // every pointer is in LDS; they are never accessed)
    for (int c = 0; c < NC; ++c) {
      s.g0[c] = t > 0 ? p + c * cnt : smem;
      s.gb[c] = smem;
    }
    if (t > 0) p += NC * cnt;
    for (int c = 0; c < NC; ++c) s.d[c] = t < T.nt - 1 ? p + c * cnt : smem;
    S[t] = s;
  }
  __syncthreads();
  // load: the top level's g and f, every level's rho^k and omega^k
  for (int l = 0; l < T.nt; ++l) {
    const Lvl G = T.L[l], V = lds_view(S[l]);
    const int cnt = G.n * G.n * G.n;
    for (int w = t; w < cnt; w += blockDim.x) {
      V.rk[w] = glb_ptr(G.rk)[w];
#pragma unroll
      for (int c = 0; c < 3; ++c) V.om[c][w] = glb_ptr(G.om[c])[w];
      if (l == 0) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          V.g[c][w] = glb_ptr(G.g[c])[w];
          V.f[c][w] = glb_ptr(G.f[c])[w];
        }
      }
    }
  }
  __syncthreads();
  const int last = T.nt - 1;
  for (int l = 0; l < last; ++l) {
    const Lvl F = lds_view(S[l]), C = lds_view(S[l + 1]);
    t3_sweeps(F, P, T.nu1);
    T3_NODES(F, i, j, k, residual_node(F, P, i, j, k));
    T3_NODES(C, i, j, k, restrict_node(F, C, i, j, k));
    T3_NODES(C, i, j, k, fas_rhs_node(C, P, i, j, k));
  }
  t3_sweeps(lds_view(S[last]), P, T.coarse_sweeps);
  for (int l = last - 1; l >= 0; --l) {
    const Lvl F = lds_view(S[l]), C = lds_view(S[l + 1]);
    T3_NODES(C, i, j, k, prolong_cell(F, C, i, j, k));
    t3_sweeps(F, P, T.nu2);
  }
  {
    const Lvl G = T.L[0], V = lds_view(S[0]);
    const int cnt = G.n * G.n * G.n;
    for (int w = t; w < cnt; w += blockDim.x)
#pragma unroll
      for (int c = 0; c < NC; ++c) glb_ptr(G.g[c])[w] = V.g[c][w];
  }
}
#undef T3_NODES

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
// (One thread per x pair of nodes, launch geometry of n/2 x n^2.)
__global__ __launch_bounds__(256) void k3_residual_partial(Lvl L, Phys P, double* __restrict__ partial) {
  if (halted(P.halt)) return;
  __shared__ double lds[16];
  const Idx x = node_x(L.n >> 1, L.n, L.lg);
  double acc = 0.0;
  if (x.ok) {
    double na[NC], nb[NC];
    int pa;
    rows_pair(L, P, L.g, 2 * x.i, x.j, x.l, na, nb, pa);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double2 f = *reinterpret_cast<const double2*>(L.f[c] + pa);
      const double da = f.x - na[c], db = f.y - nb[c];
      acc += da * da;
      acc += db * db;
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

// Copies the six components back after an odd number of tiled sweeps; a
// no-op once the stop flag is set (the sweeps were then no-ops too).
__global__ void k3_copy_back(G6 a, G6 b, size_t count, const int* halt) {
  if (halted(halt)) return;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
#pragma unroll
  for (int c = 0; c < NC; ++c) b.c[c][t] = a.c[c][t];
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
  int graph_state[4] = {};  // graphs of 1, 2, 4, 8 V-cycles: 0 not built, 1 built, -1 unavailable
  hipGraphExec_t cycle_exec[4] = {};
  // smallest level swept by the z-marching tiled kernel (below: the two
  // per-colour kernels, which fill the device better on small grids); the
  // environment variable HFZ3_TILES overrides it (0: never)
  int tile_from = 128;
  // first level of the one-workgroup tail (-1: none; HFZ3_TAIL=0 switches it off)
  int tail_top = -1;
  Lvl* tail_desc = nullptr;  // device copies of the tail's level descriptors
};

namespace {

// Levels the tiled sweep covers exactly (n a multiple of its tile and chunk).
bool tiled_shape(int n) { return n >= 32 && n % TX3 == 0 && n % TY3 == 0 && n % ZC3 == 0; }

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
    if (tiled_shape(m))
      for (int k = 0; k < NC; ++k) l.gb[k] = c.take<double>(cnt);
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
  Lvl* tail_desc = c.take<Lvl>(TAIL3_MAX);
  if (hd) {
    hd->tail_desc = tail_desc;
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
  if (tiled_shape(L.n) && L.n >= hd->tile_from) {
    // one launch per sweep, g -> gb -> g ...; an odd count copies back
    G6 home{}, other{};
    for (int c = 0; c < NC; ++c) {
      home.c[c] = L.g[c];
      other.c[c] = L.gb[c];
    }
    G6 cur = home, nxt = other;
    const unsigned grid = (unsigned)((L.n / TX3) * (L.n / TY3) * (L.n / ZC3));
    for (int k = 0; k < sweeps; ++k) {
      k3_sweep_tile<<<grid, NT3, 0, hd->stream>>>(L, cur, nxt, hd->P);
      std::swap(cur, nxt);
    }
    if (cur.c[0] != home.c[0]) {
      const size_t cnt = (size_t)L.n * L.n * L.n;
      k3_copy_back<<<(unsigned)((cnt + 255) / 256), 256, 0, hd->stream>>>(cur, home, cnt, hd->P.halt);
    }
    return;
  }
  const Dims d = dims(L.n / 2, L.n);
  for (int k = 0; k < sweeps; ++k)
    for (int colour = 0; colour < 2; ++colour) k3_smooth<<<d.grid, d.block, 0, hd->stream>>>(L, hd->P, colour);
}

void vcycle_rec(hfz3_handle* hd, int l) {
  const int last = (int)hd->L.size() - 1;
  if (l == hd->tail_top) {
    const Tail3 T{hd->tail_desc, last - l + 1, hd->p.nu1, hd->p.nu2, hd->p.coarse_sweeps};
    k3_tail<<<1, TAIL3_THREADS, 0, hd->stream>>>(T, hd->P);
    return;
  }
  if (l == last) {
    smooth(hd, l, hd->p.coarse_sweeps);
    return;
  }
  const Lvl& F = hd->L[l];
  const Lvl& C = hd->L[l + 1];
  smooth(hd, l, hd->p.nu1);
  const Dims dp = dims(F.n / 2, F.n), dc = dims(C.n, C.n);  // dp: one thread per x pair
  k3_residual_field<<<dp.grid, dp.block, 0, hd->stream>>>(F, hd->P);
  k3_restrict<<<dc.grid, dc.block, 0, hd->stream>>>(F, C, hd->P.halt);
  k3_fas_rhs<<<dc.grid, dc.block, 0, hd->stream>>>(C, hd->P);
  vcycle_rec(hd, l + 1);
  k3_prolong<<<dc.grid, dc.block, 0, hd->stream>>>(F, C, hd->P.halt);
  smooth(hd, l, hd->p.nu2);
}

void residual_launch(hfz3_handle* hd, bool stop, bool counted) {
  const Lvl& L = hd->L[0];
  const Dims d = dims(L.n / 2, L.n);  // one thread per x pair
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
// 2^k V-cycles, each with its stop-test norm, in one HIP graph (k < 4): a
// batch of cycles is launched as graphs of 8, 4, 2 and 1, since the device
// idles some microseconds between two graph launches.
bool cycle_graph(hfz3_handle* hd, int k = 0) {
  if (hd->graph_state[k] == 1) return true;
  if (hd->graph_state[k] < 0) return false;
  hipStream_t cap = nullptr;
  hipGraph_t g = nullptr;
  bool ok = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess;
  if (ok) {
    hipStream_t user = hd->stream;
    hd->stream = cap;
    ok = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
      for (int i = 0; i < (1 << k); ++i) {
        vcycle_rec(hd, 0);
        residual_launch(hd, true, true);
      }
      ok = hipStreamEndCapture(cap, &g) == hipSuccess;
    }
    hd->stream = user;
  }
  if (ok) ok = hipGraphInstantiate(&hd->cycle_exec[k], g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (cap) (void)hipStreamDestroy(cap);
  (void)hipGetLastError();
  hd->graph_state[k] = ok ? 1 : -1;
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
    int nb = std::min(batch, hd->p.max_cycles - cycles);
    for (int k = 3; k >= 0 && rc == HFZ_OK; --k) {
      if (k > 0 && !cycle_graph(hd, k)) continue;
      for (; nb >= (1 << k) && rc == HFZ_OK; nb -= 1 << k)
        if (hipGraphLaunch(hd->cycle_exec[k], hd->stream) != hipSuccess) rc = HFZ_EHIP;
    }
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
  if (const char* e = std::getenv("HFZ3_TILES")) {
    const int v = std::atoi(e);
    hd->tile_from = v > 0 ? v : INT32_MAX;
  }
  // the tail starts at the first level of at most 8^3, if its levels fit
  const char* te = std::getenv("HFZ3_TAIL");
  if (!(te && std::atoi(te) == 0)) {
    const int nl = (int)hd->L.size();
    for (int l = 0; l < nl; ++l)
      if (hd->L[l].n <= TAIL3_TOP) {
        const int nt = nl - l;
        int need = 0;
        for (int k = 0; k < nt; ++k) need += tail3_count(hd->L[l + k].n, k, nt);
        if (nt <= TAIL3_MAX && need <= TAIL3_LDS) hd->tail_top = l;
        break;
      }
  }
  if (hd->tail_top >= 0 &&
      hipMemcpyAsync(hd->tail_desc, hd->L.data() + hd->tail_top, (hd->L.size() - hd->tail_top) * sizeof(Lvl),
                     hipMemcpyHostToDevice, hd->stream) != hipSuccess) {
    delete hd;
    return HFZ_EHIP;
  }
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
  for (int k = 0; k < 4; ++k)
    if (hd->cycle_exec[k]) (void)hipGraphExecDestroy(hd->cycle_exec[k]);
  delete hd;
  return HFZ_OK;
}

}  // extern "C"
