// Grid kernels of the FAS step.  One thread per node (per node of one colour
// for the smoother); rows of a level are contiguous so a wavefront of 64
// threads reads 64 consecutive doubles of a row.
#pragma once
#include "stencil.hpp"

namespace hfz {

constexpr int RED_BLOCK = 256;  // threads per block of the reduction kernels

// ---------------------------------------------------------------- source --
// K1: omega^k = curl_h u^k (Eq. MG_DFT_d) and the source S of App. G
// (Eqs. MGS_DFT_a-c, MGS_PFC_a-e).  E is the explicit potential dF_e[rho^k]:
// 0 for PFC (its explicit part sits in S4 = 2 Delta_h rho^k), J*rho^k +
// 2 c_e rho^k for CDFT.
template <int MODEL>
__device__ __forceinline__ void source_node(const double* __restrict__ rho, const double* __restrict__ u,
                                            const double* __restrict__ v, const double* __restrict__ jrho,
                                            double* __restrict__ om, double* S0, double* S1, double* S2,
                                            double* S3, double* S4, int i, int j, int n, int lg, double h,
                                            const Phys<double>& P) {
  const Nbr q = nbr_of<MODEL>(i, j, n, lg);
  const double s = P.s, c4 = s / (4.0 * h), c2 = s / (2.0 * h), ih2 = 1.0 / (h * h);
  const double r = rho[q.p], uP = u[q.p], vP = v[q.p];
  const double w2 = 1.0 / (2.0 * h);
  const double o = (v[q.e] - v[q.w]) * w2 - (u[q.n] - u[q.s]) * w2;
  om[q.p] = o;
  S0[q.p] = r - c4 * (rho[q.e] * u[q.e] - rho[q.w] * u[q.w] + rho[q.n] * v[q.n] - rho[q.s] * v[q.s]);
  const double lapu = (u[q.e] + u[q.w] + u[q.n] + u[q.s] - 4.0 * uP) * ih2;
  const double lapv = (v[q.e] + v[q.w] + v[q.n] + v[q.s] - 4.0 * vP) * ih2;
  const double b = 0.5 * s * P.sigma * r * o;
  double s2 = r * uP + b * vP + 0.5 * s * P.gamma * lapu;
  double s3 = r * vP - b * uP + 0.5 * s * P.gamma * lapv;
  if constexpr (algebra(MODEL) == CDFT) {
    const double tc = 2.0 * P.ce;
    const double EE = jrho[q.e] + tc * rho[q.e], EW = jrho[q.w] + tc * rho[q.w];
    const double EN = jrho[q.n] + tc * rho[q.n], ES = jrho[q.s] + tc * rho[q.s];
    s2 += c2 * r * (EE - EW);
    s3 += c2 * r * (EN - ES);
  }
  S1[q.p] = s2;
  S2[q.p] = s3;
  if constexpr (algebra(MODEL) == PFC) {
    S3[q.p] = 2.0 * (rho[q.e] + rho[q.w] + rho[q.n] + rho[q.s] - 4.0 * r) * ih2;
    S4[q.p] = 0.0;
  }
}

template <int MODEL>
__global__ void k_source(const double* __restrict__ rho, const double* __restrict__ u,
                         const double* __restrict__ v, const double* __restrict__ jrho,
                         double* __restrict__ om, double* S0, double* S1, double* S2, double* S3,
                         double* S4, int n, int lg, double h, Phys<double> P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= n || j >= n) return;
  source_node<MODEL>(rho, u, v, jrho, om, S0, S1, S2, S3, S4, i, j, n, lg, h, P);
}

// ----------------------------------------------------- full weighting -----
// Coarse node (I, J) sits on fine node (2I, 2J); weights (1/16)[1 2 1; 2 4 2; 1 2 1].
template <typename T>
__device__ __forceinline__ T fw9(const T* f, int i, int j, int n, int lg) {
  const int m = n - 1;
  const int ie = (i + 1) & m, iw = (i - 1) & m;
  const int rc = j << lg, rn = ((j + 1) & m) << lg, rs = ((j - 1) & m) << lg;
  return (T(4) * f[rc + i] + T(2) * (f[rc + ie] + f[rc + iw] + f[rn + i] + f[rs + i]) +
          (f[rn + ie] + f[rn + iw] + f[rs + ie] + f[rs + iw])) *
         T(0.0625);
}

// K12: frozen coefficients rho^k, omega^k onto the next coarser level.
template <typename T>
__global__ void k_restrict_coef(const T* __restrict__ rf, const T* __restrict__ of,
                                T* __restrict__ rc, T* __restrict__ oc, int nc, int lgc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  if (I >= nc || J >= nc) return;
  const int nf = nc * 2, lgf = lgc + 1;
  rc[(J << lgc) + I] = fw9(rf, 2 * I, 2 * J, nf, lgf);
  oc[(J << lgc) + I] = fw9(of, 2 * I, 2 * J, nf, lgf);
}

// ---------------------------------------------------------- smoother ------
// K4: one colour of a damped red-black point-block sweep.  Thread t of row j
// updates node i = 2 t + ((j + colour) & 1); all its neighbours have the
// other colour, so the update is a simultaneous one.  FINE = 1 instantiates
// a separate symbol for the finest level, so profiles report it apart from
// the coarse levels.
template <int MODEL, typename T, int FINE>
__global__ void k_smooth_colour(Lvl<T> L, Phys<T> P, int colour) {
  if (halted(P.halt)) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int n = L.n;
  if (t >= (n >> 1) || j >= L.ny) return;
  if (walls(MODEL) && (j == 0 || j == n)) return;  // the wall rows are boundary values
  const int i = 2 * t + ((j + colour) & 1);
  const Nbr q = nbr_of<MODEL>(i, j, n, L.lg);
  T out[NC<MODEL>::value];
  block_update<MODEL, T>(L.g, L.f, L.rk, L.om, q, q.p, L.k, P, out);
#pragma unroll
  for (int c = 0; c < NC<MODEL>::value; ++c) L.g[c][q.p] = out[c];
}

// ------------------------------------------------------ FAS transfers -----
// K6a: g_c = g0_c = R g and f_c = R (f - N(g)) (the residual recomputed at
// the nine fine nodes of the full-weighting footprint).
template <int MODEL, typename T>
__global__ void k_fas_restrict(Lvl<T> F, Lvl<T> C, Phys<T> P) {
  if (halted(P.halt)) return;
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  if (I >= C.n || J >= C.n) return;
  constexpr int NCm = NC<MODEL>::value;
  const int m = F.n - 1;
  T accg[NCm], accd[NCm];
#pragma unroll
  for (int c = 0; c < NCm; ++c) accg[c] = accd[c] = T(0);
  for (int dj = -1; dj <= 1; ++dj) {
    for (int di = -1; di <= 1; ++di) {
      const T wgt = T((2 - (di < 0 ? -di : di)) * (2 - (dj < 0 ? -dj : dj))) * T(0.0625);
      const int fi = (2 * I + di) & m, fj = (2 * J + dj) & m;
      const Nbr q = nbr(fi, fj, F.n, F.lg);
      T nv[NCm];
      rows_N<MODEL, T>(F.g, F.rk, F.om, q, q.p, F.k, P, nv);
#pragma unroll
      for (int c = 0; c < NCm; ++c) {
        accg[c] += wgt * F.g[c][q.p];
        accd[c] += wgt * (F.f[c][q.p] - nv[c]);
      }
    }
  }
  const int pc = (J << C.lg) + I;
#pragma unroll
  for (int c = 0; c < NCm; ++c) {
    C.g[c][pc] = accg[c];
    C.g0[c][pc] = accg[c];
    C.f[c][pc] = accd[c];
  }
}

// K6a, split form for large levels: d = f - N(g) on the fine grid (one row
// evaluation per node) ...
template <int MODEL, typename T>
__global__ void k_residual_field(Lvl<T> F, Phys<T> P) {
  if (halted(P.halt)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= F.n || j >= F.n) return;
  constexpr int NCm = NC<MODEL>::value;
  const Nbr q = nbr(i, j, F.n, F.lg);
  T nv[NCm];
  rows_N<MODEL, T>(F.g, F.rk, F.om, q, q.p, F.k, P, nv);
#pragma unroll
  for (int c = 0; c < NCm; ++c) F.d[c][q.p] = F.f[c][q.p] - nv[c];
}

// ... then g_c = g0_c = R g and f_c = R d on the coarse grid.
template <int MODEL, typename T>
__global__ void k_restrict_gd(Lvl<T> F, Lvl<T> C, const int* halt) {
  if (halted(halt)) return;
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  if (I >= C.n || J >= C.n) return;
  constexpr int NCm = NC<MODEL>::value;
  const int pc = (J << C.lg) + I;
#pragma unroll
  for (int c = 0; c < NCm; ++c) {
    const T gr = fw9(F.g[c], 2 * I, 2 * J, F.n, F.lg);
    C.g[c][pc] = gr;
    C.g0[c][pc] = gr;
    C.f[c][pc] = fw9(F.d[c], 2 * I, 2 * J, F.n, F.lg);
  }
}

// K6b: f_c += N_c(R g), the FAS coarse right-hand side (C.f holds R d; the
// correction form evaluates N_d about the restricted base C.bg).
template <int MODEL, typename T, bool CORR = false>
__global__ void k_fas_rhs(Lvl<T> C, Phys<T> P) {
  if (halted(P.halt)) return;
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  if (I >= C.n || J >= C.n) return;
  constexpr int NCm = NC<MODEL>::value;
  const Nbr q = nbr(I, J, C.n, C.lg);
  T nv[NCm];
  rows_any<MODEL, T, CORR>(C.g0, C.bg, C.rk, C.om, q, q.p, C.k, P, nv);
#pragma unroll
  for (int c = 0; c < NCm; ++c) C.f[c][q.p] += nv[c];
}

// K7: g += P(g_c - R g), bilinear; CDFT (both variants) re-projects rho.
template <int MODEL, typename T>
__global__ void k_prolong(Lvl<T> F, Lvl<T> C, Phys<T> P) {
  if (halted(P.halt)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= F.n || j >= F.n) return;
  constexpr int NCm = NC<MODEL>::value;
  const int mc = C.n - 1;
  const int I = i >> 1, J = j >> 1, I1 = (I + 1) & mc, J1 = (J + 1) & mc;
  const int p00 = (J << C.lg) + I, p10 = (J << C.lg) + I1;
  const int p01 = (J1 << C.lg) + I, p11 = (J1 << C.lg) + I1;
  const int pi = i & 1, pj = j & 1;
  const int pf = (j << F.lg) + i;
#pragma unroll
  for (int c = 0; c < NCm; ++c) {
    const T e00 = C.g[c][p00] - C.g0[c][p00];
    T e;
    if (!pi && !pj) {
      e = e00;
    } else if (pi && !pj) {
      e = T(0.5) * (e00 + (C.g[c][p10] - C.g0[c][p10]));
    } else if (!pi && pj) {
      e = T(0.5) * (e00 + (C.g[c][p01] - C.g0[c][p01]));
    } else {
      e = T(0.25) * (e00 + (C.g[c][p10] - C.g0[c][p10]) + (C.g[c][p01] - C.g0[c][p01]) +
                     (C.g[c][p11] - C.g0[c][p11]));
    }
    T x = F.g[c][pf] + e;
    if constexpr (cdft_like(MODEL)) {
      if (c == 0) x = fsqrt(x * x + P.delta * P.delta);
    }
    F.g[c][pf] = x;
  }
}

// ------------------------------------------------------- reductions ------
// Block sum of a double into lds, fixed order (wavefront shuffles, then the
// wave partials in index order).
__device__ __forceinline__ double block_sum(double x, double* lds) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nth = blockDim.x * blockDim.y;
  const int wid = tid >> 6;
  if ((tid & 63) == 0) lds[wid] = x;
  __syncthreads();
  double r = 0.0;
  if (tid == 0) {
    for (int k = 0; k < (nth + 63) / 64; ++k) r += lds[k];
  }
  __syncthreads();
  return r;
}

// K5: per-block partial sums of sum_c (f - N(g))^2.
template <int MODEL, typename T>
__global__ void k_residual_partial(Lvl<T> L, Phys<T> P, double* __restrict__ partial) {
  if (halted(P.halt)) return;
  __shared__ double lds[16];
  int bx, by;
  const int tb = xcd_block(bx, by);  // XCD-contiguous block numbering
  const int i = bx * blockDim.x + threadIdx.x;
  const int j = by * blockDim.y + threadIdx.y;
  double acc = 0.0;
  if (i < L.n && j < L.ny && !(walls(MODEL) && (j == 0 || j == L.n))) {
    constexpr int NCm = NC<MODEL>::value;
    const Nbr q = nbr_of<MODEL>(i, j, L.n, L.lg);
    T nv[NCm];
    rows_N<MODEL, T>(L.g, L.rk, L.om, q, q.p, L.k, P, nv);
#pragma unroll
    for (int c = 0; c < NCm; ++c) {
      const double d = double(L.f[c][q.p]) - double(nv[c]);
      acc += d * d;
    }
  }
  const double r = block_sum(acc, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[tb] = r;
}

// Sums `count` partials (stride `stride` doubles apart, `nq` quantities laid
// out contiguously per partial) in a fixed order; out[k] = scale * sum.
__global__ void k_reduce_final(const double* __restrict__ partial, int count, int nq,
                               double scale, double* __restrict__ out) {
  __shared__ double lds[16];
  for (int k = 0; k < nq; ++k) {
    double acc = 0.0;
    for (int t = threadIdx.x; t < count; t += blockDim.x) acc += partial[(size_t)t * nq + k];
    const double r = block_sum(acc, lds);
    if (threadIdx.x == 0) out[k] = scale * r;
  }
}

// The stop test of a V-cycle on the device: unless the flag ctl[0] is already
// set, result[0] = scale * (sum of the partials, in k_reduce_final's order),
// with `counted` ctl[1] += 1 (cycles run; not for the norm before the first
// cycle), and ctl[0] = 1 if sqrt(result[0]) <= tol, 2 if it is not finite.
// One workgroup of 1024 threads.
__global__ void k_reduce_stop(const double* __restrict__ partial, int count, double scale, double tol,
                              double* __restrict__ result, int* ctl, int counted) {
  __shared__ double lds[16];
  // the flag is read with the partials (a vector load) and tested after the sum
  const int stopped = stop_flag(ctl);
  double acc = 0.0;
  for (int t = threadIdx.x; t < count; t += blockDim.x) acc += partial[t];
  const double r = block_sum(acc, lds);
  if (stop_set(stopped)) return;
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

// Channel wall rows of an iterate: rho, mu, kappa copy the adjacent interior
// row (u, v on the walls are fixed and stay as they are).  One thread per
// column.
template <typename T> __global__ void k_wall_rows(Lvl<T> L, const int* halt) {
  if (halted(halt)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  const int top = L.n << L.lg, stride = 1 << L.lg;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    if (!wall_copied(c) || L.g[c] == nullptr) continue;
    L.g[c][i] = L.g[c][stride + i];
    L.g[c][top + i] = L.g[c][top - stride + i];
  }
}

// Clears the stop flag and the cycle counter.
__global__ void k_ctl_reset(int* ctl) {
  if (threadIdx.x < 2) ctl[threadIdx.x] = 0;
}

// Stores one value of a trivially copyable type (a level descriptor, the
// physics block) into device memory: an upload from the host through the
// kernel's arguments, with no host-to-device copy.
template <typename T> __global__ void k_put(T* dst, T val) {
  if (threadIdx.x == 0) *dst = val;
}

// dst[0..count) = x.
__global__ void k_fill(double* __restrict__ dst, double x, size_t count) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) dst[t] = x;
}

// --------------------------------------------------------- post-step -----
// K10: rho^{k+1} = S1 - s/(4h)[(rho^k u)_E - (rho^k u)_W + (rho^k v)_N - (rho^k v)_S]
// with the converged velocity (Eq. discrete_a), written into dst.
__device__ __forceinline__ double continuity_node(const double* __restrict__ S0, const double* __restrict__ rk,
                                                  const double* __restrict__ u, const double* __restrict__ v,
                                                  const Nbr& q, double h, double s) {
  const double c4 = s / (4.0 * h);
  return S0[q.p] - c4 * (rk[q.e] * u[q.e] - rk[q.w] * u[q.w] + rk[q.n] * v[q.n] - rk[q.s] * v[q.s]);
}

__global__ void k_continuity(const double* __restrict__ S0, const double* __restrict__ rk,
                             const double* __restrict__ u, const double* __restrict__ v,
                             double* __restrict__ dst, int n, int lg, double h, double s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= n || j >= n) return;
  const Nbr q = nbr(i, j, n, lg);
  dst[q.p] = continuity_node(S0, rk, u, v, q, h, s);
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, size_t count) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) b[t] = a[t];
}

template <typename T>
__global__ void k_copy_t(const T* __restrict__ a, T* __restrict__ b, size_t count, const int* halt) {
  if (halted(halt)) return;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) b[t] = a[t];
}

__global__ void k_cast(const double* __restrict__ a, float* __restrict__ b, size_t count) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) b[t] = (float)a[t];
}

// ------------------------------------------- mixed precision, outer loop --
// Before each inner FP32 V-cycle: d = S - N(g) in FP64 on the finest level
// becomes the inner right-hand side (FP32), the current FP64 iterate's
// (rho, u, v) (gradient flow: rho) the inner base state, the inner
// correction starts at 0; the
// per-block partial sums of |d|^2 are the outer stop test.
template <int MODEL>
__global__ void k_mp_prepare(Lvl<double> L, Phys<double> P, Lvl<float> E, double* __restrict__ partial) {
  if (halted(P.halt)) return;
  __shared__ double lds[16];
  int bx, by;
  const int tb = xcd_block(bx, by);  // XCD-contiguous block numbering
  const int i = bx * blockDim.x + threadIdx.x;
  const int j = by * blockDim.y + threadIdx.y;
  double acc = 0.0;
  if (i < L.n && j < L.n) {
    constexpr int NCm = NC<MODEL>::value;
    const Nbr q = nbr(i, j, L.n, L.lg);
    double nv[NCm];
    rows_N<MODEL, double>(L.g, L.rk, L.om, q, q.p, L.k, P, nv);
#pragma unroll
    for (int c = 0; c < NCm; ++c) {
      const double d = L.f[c][q.p] - nv[c];
      acc += d * d;
      E.f[c][q.p] = (float)d;
      E.g[c][q.p] = 0.0f;
    }
#pragma unroll
    for (int c = 0; c < NBase<MODEL>::value; ++c) E.bg[c][q.p] = (float)L.g[c][q.p];
  }
  const double r = block_sum(acc, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[tb] = r;
}

// After the inner V-cycle: g += e (the FP32 correction added in FP64).
template <int MODEL>
__global__ void k_mp_update(Lvl<double> L, Lvl<float> E, const int* halt) {
  if (halted(halt)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= L.n || j >= L.n) return;
  const int p = (j << L.lg) + i;
#pragma unroll
  for (int c = 0; c < NC<MODEL>::value; ++c) L.g[c][p] += (double)E.g[c][p];
}

// K9: per-block partials of (KE, F part 1, F part 2, mass, min rho) before the
// h^2 factor.  PFC: part 1 = phi^4/12 + alpha phi^2/2 + (Delta_h rho)^2/2 +
// rho Delta_h rho, part 2 = 0.  CDFT: part 1 = rho (ln rho - 1) (F_id),
// part 2 = -rho (J*rho)/2 (F_ex).
template <int MODEL>
__global__ void k_energy_partial(const double* __restrict__ rho, const double* __restrict__ u,
                                 const double* __restrict__ v, const double* __restrict__ jrho,
                                 int n, int lg, double h, double alpha, double* __restrict__ partial) {
  __shared__ double lds[16];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  double ke = 0.0, f1 = 0.0, f2 = 0.0, ms = 0.0;
  // a channel sums its interior rows 1..n-1 (the grid then has n + 1 rows)
  if (i < n && j < n + (walls(MODEL) ? 1 : 0) && !(walls(MODEL) && (j == 0 || j == n))) {
    const Nbr q = nbr_of<MODEL>(i, j, n, lg);
    const double r = rho[q.p];
    ke = 0.5 * r * (u[q.p] * u[q.p] + v[q.p] * v[q.p]);
    ms = r;
    if constexpr (!cdft_like(MODEL)) {
      const double phi = r - 1.5;
      const double L = (rho[q.e] + rho[q.w] + rho[q.n] + rho[q.s] - 4.0 * r) / (h * h);
      f1 = phi * phi * phi * phi / 12.0 + 0.5 * alpha * phi * phi + 0.5 * L * L + r * L;
    } else {
      f1 = r * (log(r) - 1.0);
      f2 = -0.5 * r * jrho[q.p];
    }
  }
  const int b = blockIdx.y * gridDim.x + blockIdx.x;
  double t;
  t = block_sum(ke, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[b * 4 + 0] = t;
  t = block_sum(f1, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[b * 4 + 1] = t;
  t = block_sum(f2, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[b * 4 + 2] = t;
  t = block_sum(ms, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[b * 4 + 3] = t;
}

// Per-block minimum of rho (CDFT domain check) as a partial.
__global__ void k_min_partial(const double* __restrict__ rho, size_t count, double* __restrict__ partial) {
  __shared__ double lds[16];
  double x = 1e300;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x)
    x = fmin(x, rho[t]);
  for (int off = 32; off > 0; off >>= 1) x = fmin(x, __shfl_xor(x, off, 64));
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = lds[0];
    for (int k = 1; k < (int)(blockDim.x + 63) / 64; ++k) r = fmin(r, lds[k]);
    partial[blockIdx.x] = r;
  }
}

// PFC initial guess of the auxiliary unknowns for rho^{k+1} = rho^k:
// kappa = Delta_h rho, then (second launch) mu = phi^3/3 + alpha phi +
// Delta_h kappa + 2 Delta_h rho.  WL: a channel (n + 1 rows); a wall row
// takes its adjacent interior row's value (no flux), computed in place.
template <bool WL = false>
__global__ void k_pfc_kappa(const double* __restrict__ rho, double* __restrict__ ka, int n, int lg, double h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= n || j >= n + (WL ? 1 : 0)) return;
  const int jr = !WL ? j : (j == 0 ? 1 : (j == n ? n - 1 : j));
  const Nbr q = WL ? nbr_of<WPFC>(i, jr, n, lg) : nbr(i, j, n, lg);
  ka[(j << lg) + i] = (rho[q.e] + rho[q.w] + rho[q.n] + rho[q.s] - 4.0 * rho[q.p]) / (h * h);
}

template <bool WL = false>
__global__ void k_pfc_mu(const double* __restrict__ rho, const double* __restrict__ ka,
                         double* __restrict__ mu, int n, int lg, double h, double alpha) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= n || j >= n + (WL ? 1 : 0)) return;
  const int jr = !WL ? j : (j == 0 ? 1 : (j == n ? n - 1 : j));
  const Nbr q = WL ? nbr_of<WPFC>(i, jr, n, lg) : nbr(i, j, n, lg);
  const double phi = rho[q.p] - 1.5;
  const double lk = (ka[q.e] + ka[q.w] + ka[q.n] + ka[q.s] - 4.0 * ka[q.p]) / (h * h);
  mu[(j << lg) + i] = phi * phi * phi / 3.0 + alpha * phi + lk + 2.0 * ka[q.p];
}

// Channel state: u = u_wall and v = 0 on the wall rows, rho on them copied
// from the adjacent interior rows.  One thread per column.
__global__ void k_wall_state(double* __restrict__ rho, double* __restrict__ u, double* __restrict__ v, int n,
                             int lg, double ub, double ut) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int top = n << lg, stride = 1 << lg;
  rho[i] = rho[stride + i];
  rho[top + i] = rho[top - stride + i];
  u[i] = ub;
  u[top + i] = ut;
  v[i] = 0.0;
  v[top + i] = 0.0;
}

// CDFT kernel of Sec. 6 on the periodic grid, minimum-image displacement:
// J = sqrt2 exp(-pi^2 r^2/(2 nu^2)) - exp(-pi^2 r^2/(4 nu^2)); also
// J_e = max(-J, 0) for the (J_e * 1) reduction.
__global__ void k_kernel_table(double* __restrict__ J, double* __restrict__ Je, int n, int lg,
                               double h, double nu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= n || j >= n) return;
  const int di = (i <= n / 2) ? i : i - n;
  const int dj = (j <= n / 2) ? j : j - n;
  const double x = di * h, y = dj * h;
  const double r2 = x * x + y * y;
  const double c = M_PI * M_PI / (nu * nu);
  const double val = sqrt(2.0) * exp(-0.5 * c * r2) - exp(-0.25 * c * r2);
  J[(j << lg) + i] = val;
  Je[(j << lg) + i] = (val <= 0.0) ? -val : 0.0;
}

}  // namespace hfz
