// K8: the coarse end of the V-cycle in one workgroup.  From the tail top
// level (a small grid) down to the coarsest grid and back, every phase of the
// FAS V-cycle (smoother colours, restriction, coarse right-hand side, the
// coarsest sweeps, prolongation) runs inside a single kernel, with a
// workgroup barrier between phases instead of a kernel boundary.  All tail
// levels live in LDS for the duration of the kernel: the top level's g and f
// and every level's frozen coefficients are loaded once, the top level's g is
// written back at the end.  The arithmetic is the same device code the
// per-level kernels use.
#pragma once
#include "kernels.hpp"
#include "stencil.hpp"

namespace hfz {

constexpr int TAIL_MAX_LEVELS = 8;
constexpr int TAIL_THREADS = 512;

template <typename T> struct TailArgs {
  const Lvl<T>* Lg;  // device array of the tail's level descriptors; [0] = tail top
  int nt;            // levels in the tail, all held in LDS
  int top_n;         // size of the tail top
  int nu1, nu2, coarse_sweeps;
};

// T values of LDS that `nt` tail levels need (top size top_n): g, f, rk, om
// per level, plus g0 for all but the tail top.  NB = 3 in the correction form
// (the base state rho, u, v), else 0.
template <int NCm, int NB = 0>
__host__ __device__ inline size_t tail_lds_count(int top_n, int nt) {
  size_t tot = 0;
  int n = top_n;
  for (int l = 0; l < nt; ++l) {
    tot += (size_t)n * n * (2 * NCm + 2 + NB + (l > 0 ? NCm : 0));
    n >>= 1;
  }
  return tot;
}

// Level descriptors of the tail: S = the LDS arrays the phases use, G = the
// global arrays.  Thread t builds level t (same LDS order as tail_lds_count).
template <int NCm, int NB, typename T>
__device__ inline void tail_lds_levels(const TailArgs<T>& A, T* base, Lvl<T>* S, Lvl<T>* G) {
  const int t = threadIdx.x;
  if (t >= A.nt) return;
  Lvl<T> s = A.Lg[t];
  G[t] = s;
  size_t off = 0;
  for (int l = 0; l < t; ++l) {
    const size_t nl = (size_t)(A.top_n >> l);
    off += nl * nl * (2 * NCm + 2 + NB + (l > 0 ? NCm : 0));
  }
  T* p = base + off;
  const int cnt = s.n * s.n;
#pragma unroll
  for (int c = 0; c < NCm; ++c) s.g[c] = p + c * cnt;
  p += NCm * cnt;
#pragma unroll
  for (int c = 0; c < NCm; ++c) s.f[c] = p + c * cnt;
  p += NCm * cnt;
  if (t > 0) {
#pragma unroll
    for (int c = 0; c < NCm; ++c) s.g0[c] = p + c * cnt;
    p += NCm * cnt;
  }
  s.rk = p;
  s.om = p + cnt;
  p += 2 * cnt;
#pragma unroll
  for (int c = 0; c < NB; ++c) s.bg[c] = p + c * cnt;
  S[t] = s;
}

// The view the phases use of a tail level built by tail_lds_levels: its
// arrays in LDS (g0 only below the top, G0 = true), the residual scratch d in
// global memory.
template <int NCm, int NB, bool G0, typename T> __device__ __forceinline__ Lvl<T> tail_view(const Lvl<T>& s) {
  Lvl<T> L = s;
#pragma unroll
  for (int c = 0; c < NCm; ++c) {
    L.g[c] = as_lds(s.g[c]);
    L.f[c] = as_lds(s.f[c]);
    if constexpr (G0) L.g0[c] = as_lds(s.g0[c]);
    L.d[c] = as_global(s.d[c]);
  }
  L.rk = as_lds(s.rk);
  L.om = as_lds(s.om);
#pragma unroll
  for (int c = 0; c < NB; ++c) L.bg[c] = as_lds(s.bg[c]);
  return L;
}

template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void tail_smooth(const Lvl<T> L, const Phys<T>& P, int colour) {
  const int n = L.n, half = n >> 1, cnt = half * n;
  for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
    const int j = w / half, t = w - j * half;
    const int i = 2 * t + ((j + colour) & 1);
    const Nbr q = nbr(i, j, n, L.lg);
    T out[NC<MODEL>::value];
    update_any<MODEL, T, CORR>(L.g, L.f, L.bg, L.rk, L.om, q, q.p, L.k, P, out);
#pragma unroll
    for (int c = 0; c < NC<MODEL>::value; ++c) L.g[c][q.p] = out[c];
  }
  __syncthreads();
}

template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void tail_sweeps(const Lvl<T> L, const Phys<T>& P, int sweeps) {
  for (int k = 0; k < sweeps; ++k) {
    tail_smooth<MODEL, T, CORR>(L, P, 0);
    tail_smooth<MODEL, T, CORR>(L, P, 1);
  }
}

template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void tail_restrict(const Lvl<T> F, const Lvl<T> C, const Phys<T>& P) {
  constexpr int NCm = NC<MODEL>::value;
  // d = f - N(g) on the fine level (into F.d, a global scratch array) ...
  const int fcnt = F.n * F.n;
  for (int w = threadIdx.x; w < fcnt; w += blockDim.x) {
    const Nbr q = nbr(w & (F.n - 1), w >> F.lg, F.n, F.lg);
    T nv[NCm];
    rows_any<MODEL, T, CORR>(F.g, F.bg, F.rk, F.om, q, q.p, F.k, P, nv);
#pragma unroll
    for (int c = 0; c < NCm; ++c) F.d[c][q.p] = F.f[c][q.p] - nv[c];
  }
  __syncthreads();
  // ... then g_c = g0_c = R g and f_c = R d ...
  const int cnt = C.n * C.n;
  for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
    const int J = w >> C.lg, I = w & (C.n - 1);
#pragma unroll
    for (int c = 0; c < NCm; ++c) {
      const T gr = fw9(F.g[c], 2 * I, 2 * J, F.n, F.lg);
      C.g[c][w] = gr;
      C.g0[c][w] = gr;
      C.f[c][w] = fw9(F.d[c], 2 * I, 2 * J, F.n, F.lg);
    }
    if constexpr (CORR) {
#pragma unroll
      for (int c = 0; c < 3; ++c) C.bg[c][w] = fw9(F.bg[c], 2 * I, 2 * J, F.n, F.lg);
    }
  }
  __syncthreads();
  // ... and f_c += N_c(R g)
  for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
    const int J = w >> C.lg, I = w & (C.n - 1);
    const Nbr q = nbr(I, J, C.n, C.lg);
    T nv[NCm];
    rows_any<MODEL, T, CORR>(C.g0, C.bg, C.rk, C.om, q, q.p, C.k, P, nv);
#pragma unroll
    for (int c = 0; c < NCm; ++c) C.f[c][w] += nv[c];
  }
  __syncthreads();
}

template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void tail_prolong(const Lvl<T> F, const Lvl<T> C, const Phys<T>& P) {
  constexpr int NCm = NC<MODEL>::value;
  const int cnt = F.n * F.n, mc = C.n - 1;
  for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
    const int j = w >> F.lg, i = w & (F.n - 1);
    const int I = i >> 1, J = j >> 1, I1 = (I + 1) & mc, J1 = (J + 1) & mc;
    const int p00 = (J << C.lg) + I, p10 = (J << C.lg) + I1;
    const int p01 = (J1 << C.lg) + I, p11 = (J1 << C.lg) + I1;
    const int pi = i & 1, pj = j & 1;
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
      T x = F.g[c][w] + e;
      if constexpr (MODEL == CDFT) {
        if (c == 0) x = project_any<T, CORR>(x, CORR ? F.bg[0][w] : T(0), P.delta);
      }
      F.g[c][w] = x;
    }
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ void tail_copy(T* dst, const T* src, int cnt) {
  for (int w = threadIdx.x; w < cnt; w += blockDim.x) dst[w] = src[w];
}

template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void tail_body(const TailArgs<T>& A, const Phys<T>& P) {
  constexpr int NCm = NC<MODEL>::value;
  constexpr int NB = CORR ? 3 : 0;
  extern __shared__ __align__(16) unsigned char tail_smem[];
  // level descriptors in LDS: S = LDS copies, G = the global arrays
  __shared__ Lvl<T> S[TAIL_MAX_LEVELS];
  __shared__ Lvl<T> G[TAIL_MAX_LEVELS];
  tail_lds_levels<NCm, NB, T>(A, reinterpret_cast<T*>(tail_smem), S, G);
  __syncthreads();
  {
    const Lvl<T> s = tail_view<NCm, NB, false>(S[0]);
    const Lvl<T> g = lvl_global(G[0]);
    const int cnt = g.n * g.n;
#pragma unroll
    for (int c = 0; c < NCm; ++c) {
      tail_copy(s.g[c], g.g[c], cnt);
      tail_copy(s.f[c], g.f[c], cnt);
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) tail_copy(s.bg[c], g.bg[c], cnt);
  }
  for (int l = 0; l < A.nt; ++l) {
    const Lvl<T> s = tail_view<NCm, NB, false>(S[l]);
    const Lvl<T> g = lvl_global(G[l]);
    const int cnt = g.n * g.n;
    tail_copy(s.rk, g.rk, cnt);
    tail_copy(s.om, g.om, cnt);
  }
  __syncthreads();
  const int last = A.nt - 1;
  for (int l = 0; l < last; ++l) {
    const Lvl<T> F = tail_view<NCm, NB, false>(S[l]);
    tail_sweeps<MODEL, T, CORR>(F, P, A.nu1);
    tail_restrict<MODEL, T, CORR>(F, tail_view<NCm, NB, true>(S[l + 1]), P);
  }
  tail_sweeps<MODEL, T, CORR>(tail_view<NCm, NB, false>(S[last]), P, A.coarse_sweeps);
  for (int l = last - 1; l >= 0; --l) {
    const Lvl<T> F = tail_view<NCm, NB, false>(S[l]);
    tail_prolong<MODEL, T, CORR>(F, tail_view<NCm, NB, true>(S[l + 1]), P);
    tail_sweeps<MODEL, T, CORR>(F, P, A.nu2);
  }
  {
    const Lvl<T> s = tail_view<NCm, NB, false>(S[0]);
    const Lvl<T> g = lvl_global(G[0]);
    const int cnt = g.n * g.n;
#pragma unroll
    for (int c = 0; c < NCm; ++c) tail_copy(g.g[c], s.g[c], cnt);
  }
}

template <int MODEL, typename T, bool CORR>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail(TailArgs<T> A, Phys<T> P) {
  tail_body<MODEL, T, CORR>(A, P);
}

// Batched form: workgroup z runs the tail of instance z, whose level
// descriptors start at A.Lg + z * stride.
template <int MODEL, typename T, bool CORR>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail_b(TailArgs<T> A, int stride, const Phys<T>* Ps,
                                                         const int* active) {
  const int z = blockIdx.x;
  if (!active[z]) return;
  TailArgs<T> B = A;
  B.Lg = as_global(A.Lg + (size_t)z * stride);
  tail_body<MODEL, T, CORR>(B, Ps[z]);
}

}  // namespace hfz
