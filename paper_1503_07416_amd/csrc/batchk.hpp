// Kernels of the batched solve: many instances per launch, instance =
// blockIdx.z (or blockIdx.x for one workgroup per instance), descriptors in
// device arrays, instances whose flag in `active` is 0 skipped.  Instances may
// differ in grid size: a launch over each instance's finest level is sized
// for the largest, and every thread outside its own instance's grid returns
// (or adds nothing to the partial sums).  The arithmetic is the
// single-instance device code.
#pragma once
#include "kernels.hpp"
#include "stencil.hpp"

namespace hfz {

// Per-block partial sums of sum_c (f - N(g))^2 on each instance's finest level.
template <int MODEL>
__global__ void k_residual_partial_b(const Lvl<double>* Ls, const Phys<double>* Ps, const int* active,
                                     double* __restrict__ partial, int pstride) {
  __shared__ double lds[16];
  const int z = blockIdx.z;
  if (!active[z]) return;
  const Lvl<double> L = lvl_global(Ls[z]);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  double acc = 0.0;
  if (i < L.n && j < L.n) {
    constexpr int NCm = NC<MODEL>::value;
    const Nbr q = nbr(i, j, L.n, L.lg);
    double nv[NCm];
    rows_N<MODEL, double>(L.g, L.rk, L.om, q, q.p, L.k, Ps[z], nv);
#pragma unroll
    for (int c = 0; c < NCm; ++c) {
      const double d = L.f[c][q.p] - nv[c];
      acc += d * d;
    }
  }
  const double r = block_sum(acc, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[(size_t)z * pstride + blockIdx.y * gridDim.x + blockIdx.x] = r;
}

// Mixed precision: k_mp_prepare per instance (the outer FP64 residual into
// the inner right-hand side, base state, e = 0, partial sums).
template <int MODEL>
__global__ void k_mp_prepare_b(const Lvl<double>* Ls, const Phys<double>* Ps, const Lvl<float>* Es,
                               const int* active, double* __restrict__ partial, int pstride) {
  __shared__ double lds[16];
  const int z = blockIdx.z;
  if (!active[z]) return;
  const Lvl<double> L = lvl_global(Ls[z]);
  const Lvl<float> E = lvl_global(Es[z]);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  double acc = 0.0;
  if (i < L.n && j < L.n) {
    constexpr int NCm = NC<MODEL>::value;
    const Nbr q = nbr(i, j, L.n, L.lg);
    double nv[NCm];
    rows_N<MODEL, double>(L.g, L.rk, L.om, q, q.p, L.k, Ps[z], nv);
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
  if (threadIdx.x == 0 && threadIdx.y == 0) partial[(size_t)z * pstride + blockIdx.y * gridDim.x + blockIdx.x] = r;
}

template <int MODEL>
__global__ void k_mp_update_b(const Lvl<double>* Ls, const Lvl<float>* Es, const int* active) {
  const int z = blockIdx.z;
  if (!active[z]) return;
  const Lvl<double> L = lvl_global(Ls[z]);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= L.n || j >= L.n) return;
  const int p = (j << L.lg) + i;
  const Lvl<float> E = lvl_global(Es[z]);
#pragma unroll
  for (int c = 0; c < NC<MODEL>::value; ++c) L.g[c][p] += (double)E.g[c][p];
}

// g <- gb for every component (the iterate ended in the second buffer).
template <typename T>
__global__ void k_swap_back_b(const Lvl<T>* Ls, const int* active, int nc) {
  const int z = blockIdx.z;
  if (!active[z]) return;
  const Lvl<T> L = lvl_global(Ls[z]);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.n * L.n) return;
#pragma unroll
  for (int c = 0; c < 5; ++c)
    if (c < nc) L.g[c][t] = L.gb[c][t];
}

// norm2[z] = h_z^2 * (sum of instance z's `count` partials), fixed order;
// one workgroup per instance.
__global__ void k_reduce_b(const double* __restrict__ partial, int count, int pstride, const Lvl<double>* Ls,
                           const int* active, double* __restrict__ norm2) {
  __shared__ double lds[16];
  const int z = blockIdx.x;
  if (!active[z]) return;
  double acc = 0.0;
  for (int t = threadIdx.x; t < count; t += blockDim.x) acc += partial[(size_t)z * pstride + t];
  const double r = block_sum(acc, lds);
  if (threadIdx.x == 0) {
    const double h = Ls[z].h;
    norm2[z] = h * h * r;
  }
}

// The per-instance stop test on the device: for each active instance z,
// norm2[z] = h_z^2 * (sum of its partials, in k_reduce_b's order: `count` of
// them, or counts[z] when counts is not null); with
// `counted` the cycle that produced it is counted in cyc[z]; the instance
// leaves the batch with stat[z] = 1 once sqrt(norm2) <= tol[z], 2 if the norm
// is not finite, 3 if cyc[z] reached maxc[z].  One workgroup per instance.
__global__ void k_reduce_stop_b(const double* __restrict__ partial, int count, const int* __restrict__ counts,
                                int pstride, const Lvl<double>* Ls, int* active, double* __restrict__ norm2,
                                int* cyc, int* stat, const double* __restrict__ tol, const int* __restrict__ maxc,
                                int counted) {
  __shared__ double lds[16];
  const int z = blockIdx.x;
  if (!active[z]) return;
  if (counts) count = counts[z];
  double acc = 0.0;
  for (int t = threadIdx.x; t < count; t += blockDim.x) acc += partial[(size_t)z * pstride + t];
  const double r = block_sum(acc, lds);
  if (threadIdx.x == 0) {
    const double h = Ls[z].h;
    const double n2 = h * h * r;
    norm2[z] = n2;
    if (counted) cyc[z] += 1;
    const double nrm = sqrt(n2);
    int s = 0;
    if (nrm <= tol[z])
      s = 1;
    else if (!isfinite(nrm))
      s = 2;
    else if (cyc[z] >= maxc[z])
      s = 3;
    if (s != 0) {
      stat[z] = s;
      active[z] = 0;
    }
  }
}

// a[0..count) = 0.
__global__ void k_zero_ints(int* a, int count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) a[t] = 0;
}

// Per-instance state arrays of the batched begin / finish kernels.
struct StateB {
  double* u;
  double* v;
  double* mu;
  double* ka;
  double* jrho;
};

// Start of a step for every instance z with on[z]: omega^k and the source S
// (the single-instance k_source arithmetic), the iterate g = state, and in
// mixed precision the FP32 copies of rho^k and omega^k (E0s non-null).
template <int MODEL>
__global__ void k_begin_b(const Lvl<double>* L0s, const StateB* Ss, const Phys<double>* Ps, const int* on,
                          const Lvl<float>* E0s) {
  const int z = blockIdx.z;
  if (!on[z]) return;
  const Lvl<double> L = lvl_global(L0s[z]);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= L.n || j >= L.ny) return;
  const StateB S = Ss[z];
  double* u = as_global(S.u);
  double* v = as_global(S.v);
  const int p = (j << L.lg) + i;
  constexpr bool PF = algebra(MODEL) == PFC;
  if (walls(MODEL) && (j == 0 || j == L.n)) {
    // channel wall rows: no equation (S = 0, omega^k = 0); the iterate keeps
    // the state's boundary values
#pragma unroll
    for (int c = 0; c < NC<MODEL>::value; ++c) L.f[c][p] = 0.0;
    L.om[p] = 0.0;
  } else {
    source_node<MODEL>(L.rk, u, v, algebra(MODEL) == CDFT ? as_global(S.jrho) : nullptr, L.om, L.f[0], L.f[1],
                       L.f[2], PF ? L.f[3] : nullptr, PF ? L.f[4] : nullptr, i, j, L.n, L.lg, L.h, Ps[z]);
  }
  L.g[0][p] = L.rk[p];
  L.g[1][p] = u[p];
  L.g[2][p] = v[p];
  if constexpr (PF) {
    L.g[3][p] = as_global(S.mu)[p];
    L.g[4][p] = as_global(S.ka)[p];
  }
  if (E0s) {
    const Lvl<float> E = lvl_global(E0s[z]);
    E.rk[p] = (float)L.rk[p];
    E.om[p] = (float)L.om[p];
  }
}

// rho^k, omega^k of every instance onto its next coarser level (and their FP32
// copies in mixed precision, Es non-null).  WL: a channel, whose coarse wall
// rows take rho^k of the adjacent interior row (no flux) and omega^k = 0;
// the interior rows' footprints lie on fine interior rows.
template <bool WL = false>
__global__ void k_restrict_coef_b(const Lvl<double>* Fs, const Lvl<double>* Cs, const int* on,
                                  const Lvl<float>* Es) {
  const int z = blockIdx.z;
  if (!on[z]) return;
  const Lvl<double> F = lvl_global(Fs[z]);
  const Lvl<double> C = lvl_global(Cs[z]);
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  const int J = blockIdx.y * blockDim.y + threadIdx.y;
  if (I >= C.n || J >= C.ny) return;
  const int pc = (J << C.lg) + I;
  const bool wall = WL && (J == 0 || J == C.n);
  const int Jr = !wall ? J : (J == 0 ? 1 : C.n - 1);
  const double r = fw9(F.rk, 2 * I, 2 * Jr, F.n, F.lg);
  const double o = wall ? 0.0 : fw9(F.om, 2 * I, 2 * J, F.n, F.lg);
  C.rk[pc] = r;
  C.om[pc] = o;
  if (Es) {
    const Lvl<float> E = lvl_global(Es[z]);
    E.rk[pc] = (float)r;
    E.om[pc] = (float)o;
  }
}

// End of a step, first half: rho^{k+1} from the continuity row into g[0]
// (the single-instance k_continuity arithmetic).  WL: a channel; a wall row
// takes the value of its adjacent interior row (each thread reads only rk,
// f and the velocity, so the copy needs no second pass).
template <bool WL = false>
__global__ void k_continuity_b(const Lvl<double>* L0s, const Phys<double>* Ps, const int* on) {
  const int z = blockIdx.z;
  if (!on[z]) return;
  const Lvl<double> L = lvl_global(L0s[z]);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= L.n || j >= L.ny) return;
  const int jr = !WL ? j : (j == 0 ? 1 : (j == L.n ? L.n - 1 : j));
  const Nbr q = WL ? nbr_of<WPFC>(i, jr, L.n, L.lg) : nbr(i, j, L.n, L.lg);
  L.g[0][(j << L.lg) + i] = continuity_node(L.f[0], L.rk, L.g[1], L.g[2], q, L.h, Ps[z].s);
}

// End of a step, second half: state <- g.
template <int MODEL> __global__ void k_state_b(const Lvl<double>* L0s, const StateB* Ss, const int* on) {
  const int z = blockIdx.z;
  if (!on[z]) return;
  const Lvl<double> L = lvl_global(L0s[z]);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= L.n * L.ny) return;
  const StateB S = Ss[z];
  L.rk[t] = L.g[0][t];
  as_global(S.u)[t] = L.g[1][t];
  as_global(S.v)[t] = L.g[2][t];
  if constexpr (algebra(MODEL) == PFC) {
    as_global(S.mu)[t] = L.g[3][t];
    as_global(S.ka)[t] = L.g[4][t];
  }
}

// ------------------------------------------------ gradient-flow variant --
// Start of a gradient-flow step (Thm. thm_grad) on level 0 (its rows have no
// frozen coefficients, so no coarse level needs anything): the source
//   S1 = rho^k;  GPFC: S2 = 2 Delta_h rho^k, S3 = 0;  GCDFT: S2 = -(J*rho^k + 2 c_e rho^k)
// and the initial guess g = (rho^k, dF[rho^k] (, Delta_h rho^k)) with
// dF = dF_c - dF_e of Sec. 5.3 / 5.2: GPFC (phi^3/3 + alpha phi +
// Delta_h^2 rho) + 2 Delta_h rho, GCDFT (ln rho + 2 c_e rho) - (2 c_e rho + J*rho).
// rho^k is level 0's rk; J*rho^k the state's jrho.
template <int MODEL>
__global__ void k_begin_gf(const Lvl<double>* L0s, const StateB* Ss, const Phys<double>* Ps, const int* on) {
  const int z = blockIdx.z;
  if (!on[z]) return;
  const Lvl<double> L = lvl_global(L0s[z]);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= L.n || j >= L.n) return;
  const Phys<double> P = Ps[z];
  const double* rho = L.rk;
  const Nbr q = nbr(i, j, L.n, L.lg);
  const double r = rho[q.p];
  L.f[0][q.p] = r;
  L.g[0][q.p] = r;
  if constexpr (MODEL == GPFC) {
    const double ih2 = 1.0 / (L.h * L.h);
    const int m = L.n - 1;
    // Delta_h rho at (a, b)
    auto lap = [&](int a, int b) {
      const Nbr t = nbr(a & m, b & m, L.n, L.lg);
      return (rho[t.e] + rho[t.w] + rho[t.n] + rho[t.s] - 4.0 * rho[t.p]) * ih2;
    };
    const double lP = lap(i, j);
    const double l2 = (lap(i + 1, j) + lap(i - 1, j) + lap(i, j + 1) + lap(i, j - 1) - 4.0 * lP) * ih2;
    const double phi = r - 1.5;
    L.f[1][q.p] = 2.0 * lP;
    L.f[2][q.p] = 0.0;
    L.g[1][q.p] = (phi * phi * phi / 3.0 + P.alpha * phi + l2) + 2.0 * lP;
    L.g[2][q.p] = lP;
  } else {
    const double jr = as_global(Ss[z].jrho)[q.p];
    const double tc = 2.0 * P.ce;
    L.f[1][q.p] = -(jr + tc * r);
    L.g[1][q.p] = (log(r) + tc * r) - (tc * r + jr);
  }
}

// End of a gradient-flow step: with `fix`, rho^{k+1} = rho^k + s Delta_h mu
// from the converged mu (row 1 exactly, so that the mass is conserved to
// round-off), else the solve's rho; into g[0] and the state (level 0's rk),
// and mu (GPFC: and kappa) into the state's auxiliaries.  Each thread reads
// only its own rk and g[0] and the other threads' mu, so one pass is safe.
template <int MODEL>
__global__ void k_finish_gf(const Lvl<double>* L0s, const StateB* Ss, const Phys<double>* Ps, const int* on,
                            int fix) {
  const int z = blockIdx.z;
  if (!on[z]) return;
  const Lvl<double> L = lvl_global(L0s[z]);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= L.n || j >= L.n) return;
  const Nbr q = nbr(i, j, L.n, L.lg);
  const double* mu = L.g[1];
  double r = L.g[0][q.p];
  if (fix) r = L.rk[q.p] + Ps[z].s * ((nsum(mu, q) - 4.0 * mu[q.p]) / (L.h * L.h));
  L.g[0][q.p] = r;
  L.rk[q.p] = r;
  const StateB S = Ss[z];
  as_global(S.mu)[q.p] = mu[q.p];
  if constexpr (MODEL == GPFC) as_global(S.ka)[q.p] = L.g[2][q.p];
}

// mu = dF[rho] of GCDFT, (ln rho + 2 c_e rho) - (2 c_e rho + J*rho): the
// auxiliary consistent with the state before its first step.
__global__ void k_gcdft_mu0(const double* __restrict__ rho, const double* __restrict__ jrho,
                            double* __restrict__ mu, size_t count, double ce) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const double r = rho[t], tc = 2.0 * ce;
  mu[t] = (log(r) + tc * r) - (tc * r + jrho[t]);
}

}  // namespace hfz
