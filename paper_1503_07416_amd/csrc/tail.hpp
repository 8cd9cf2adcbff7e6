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
  int d_from;        // levels l >= d_from keep the residual scratch d in LDS, the others in global memory
  int fc;            // 1: the top level's right-hand side is still R d; the kernel completes
                     // f = R d + N(g) after loading g = R g (the restriction folded into the sweeps)
};

// T values of LDS per level l of nt (size n): g, f, the NR frozen
// coefficients (rk, om; none in the gradient flow), g0 below the top, the NB
// base fields of the correction form, and d where it is held in LDS
// (l >= d_from; the coarsest level needs none).
// WR = 1 for a channel, whose levels hold n + 1 rows.
template <int NCm, int NB, int NR, int WR = 0>
__host__ __device__ inline size_t tail_level_count(int n, int l, int nt, int d_from) {
  const bool dl = l >= d_from && l < nt - 1;
  return (size_t)n * (n + WR) * (2 * NCm + NR + NB + (l > 0 ? NCm : 0) + (dl ? NCm : 0));
}

// PMA: scratch arrays of the top level's size after the levels (one for the
// CDFT potential M, see tail_smooth).
template <int NCm, int NB, int NR, int WR = 0, int PMA = 0>
__host__ __device__ inline size_t tail_lds_count(int top_n, int nt, int d_from) {
  size_t tot = 0;
  for (int l = 0; l < nt; ++l) tot += tail_level_count<NCm, NB, NR, WR>(top_n >> l, l, nt, d_from);
  return tot + (size_t)PMA * top_n * (top_n + WR);
}

// Scratch arrays the tail of MODEL needs (tail_lds_count's PMA).
template <int MODEL> constexpr int tail_pm() { return MODEL == CDFT ? 1 : 0; }

// Level descriptors of the tail: S = the LDS arrays the phases use, G = the
// global arrays.  Thread t builds level t (same LDS order as tail_lds_count).
template <int NCm, int NB, int NR, int WR, typename T>
__device__ inline void tail_lds_levels(const TailArgs<T>& A, T* base, Lvl<T>* S, Lvl<T>* G) {
  const int t = threadIdx.x;
  if (t >= A.nt) return;
  Lvl<T> s = A.Lg[t];
  G[t] = s;
  size_t off = 0;
  for (int l = 0; l < t; ++l) off += tail_level_count<NCm, NB, NR, WR>(A.top_n >> l, l, A.nt, A.d_from);
  T* p = base + off;
  const int cnt = s.n * s.ny;
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
  if constexpr (NR == 2) {
    s.rk = p;
    s.om = p + cnt;
    p += 2 * cnt;
  } else {
    s.rk = nullptr;
    s.om = nullptr;
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) s.bg[c] = p + c * cnt;
  p += NB * cnt;
  if (t >= A.d_from && t < A.nt - 1) {
#pragma unroll
    for (int c = 0; c < NCm; ++c) s.d[c] = p + c * cnt;
  }
  S[t] = s;
}

// The view the phases use of a tail level built by tail_lds_levels: its
// arrays in LDS (g0 only below the top, G0 = true), the residual scratch d in
// LDS (DL = true) or global memory.
template <int NCm, int NB, int NR, bool G0, bool DL = false, typename T>
__device__ __forceinline__ Lvl<T> tail_view(const Lvl<T>& s) {
  Lvl<T> L = s;
#pragma unroll
  for (int c = 0; c < NCm; ++c) {
    L.g[c] = as_lds(s.g[c]);
    L.f[c] = as_lds(s.f[c]);
    if constexpr (G0) L.g0[c] = as_lds(s.g0[c]);
    L.d[c] = DL ? as_lds(s.d[c]) : as_global(s.d[c]);
  }
  if constexpr (NR == 2) {
    L.rk = as_lds(s.rk);
    L.om = as_lds(s.om);
  }
#pragma unroll
  for (int c = 0; c < NB; ++c) L.bg[c] = as_lds(s.bg[c]);
  return L;
}

// Channel: rho, mu, kappa on the wall rows 0 and n <- the adjacent rows.
template <int MODEL, typename T> __device__ __forceinline__ void tail_wall_rows(const Lvl<T> L) {
  if constexpr (walls(MODEL)) {
    const int top = L.n << L.lg, stride = 1 << L.lg;
    for (int i = threadIdx.x; i < L.n; i += blockDim.x) {
#pragma unroll
      for (int c = 0; c < NC<MODEL>::value; ++c) {
        if (!wall_copied(c)) continue;
        L.g[c][i] = L.g[c][stride + i];
        L.g[c][top + i] = L.g[c][top - stride + i];
      }
    }
    __syncthreads();
  }
}

// One colour of a damped red-black sweep.  CDFT: the potential M (a logarithm
// per node) is first evaluated once at each node of the other colour into sm
// (its values are final for this half sweep), instead of at the four
// neighbours of every updated node.
//
// A channel updates its interior rows 1..n-1; the updater of a node on row 1
// (n - 1) also writes the wall copies of rho, mu, kappa on row 0 (n) below
// (above) it.  No other update of the half sweep reads that wall node, and a
// wall node next to a node of the other colour already holds its value, so
// the wall rows end the half sweep as a refresh of them would leave them.
template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void tail_smooth(const Lvl<T> L, const Phys<T>& P, int colour, T* sm) {
  constexpr int J0 = walls(MODEL) ? 1 : 0;
  constexpr bool PM = tail_pm<MODEL>() > 0;
  const int n = L.n, cnt = (n >> 1) * (n - J0), lgh = L.lg - 1;
  if constexpr (PM) {
    for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
      const int j = w >> lgh, t = w & ((1 << lgh) - 1);
      const int p = (j << L.lg) + 2 * t + ((j + colour + 1) & 1);
      sm[p] = potential_any<MODEL, T, CORR>(L.g, L.bg, p, P);
    }
    __syncthreads();
  }
  for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
    const int j = J0 + (w >> lgh), t = w & ((1 << lgh) - 1);
    const int i = 2 * t + ((j + colour) & 1);
    const Nbr q = nbr_of<MODEL>(i, j, n, L.lg);
    T out[NC<MODEL>::value];
    update_any<MODEL, T, CORR, PM>(L.g, L.f, L.bg, L.rk, L.om, q, q.p, L.k, P, out, sm);
#pragma unroll
    for (int c = 0; c < NC<MODEL>::value; ++c) L.g[c][q.p] = out[c];
    if constexpr (walls(MODEL)) {
      if (j == 1 || j == n - 1) {
        const int wp = (j == 1 ? 0 : n << L.lg) + i;
#pragma unroll
        for (int c = 0; c < NC<MODEL>::value; ++c)
          if (wall_copied(c)) L.g[c][wp] = out[c];
      }
    }
  }
  __syncthreads();
}

template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void tail_sweeps(const Lvl<T> L, const Phys<T>& P, int sweeps, T* sm) {
  for (int k = 0; k < sweeps; ++k) {
    tail_smooth<MODEL, T, CORR>(L, P, 0, sm);
    tail_smooth<MODEL, T, CORR>(L, P, 1, sm);
  }
}

// FAS restriction in two phases: d = f - N(g) on the fine level and
// g_c = g0_c = R g (correction form: also the coarse base R bg), then
// f_c = R d + N_c(R g).  CDFT: the potential M of g (then of R g) is evaluated
// once per node into sm before the rows that read it at four neighbours.
template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void tail_restrict(const Lvl<T> F, const Lvl<T> C, const Phys<T>& P, T* sm) {
  // channel: d on the fine interior rows; R g on the coarse interior rows (their
  // footprints are fine interior rows) and the boundary values on the coarse
  // wall rows; f_c on the coarse interior rows
  constexpr int NCm = NC<MODEL>::value;
  constexpr bool WL = walls(MODEL);
  constexpr bool PM = tail_pm<MODEL>() > 0;
  const int fcnt = F.n * F.ny;
  if constexpr (PM) {
    for (int w = threadIdx.x; w < fcnt; w += blockDim.x) sm[w] = potential_any<MODEL, T, CORR>(F.g, F.bg, w, P);
    __syncthreads();
  }
  for (int w = threadIdx.x; w < fcnt; w += blockDim.x) {
    const int j = w >> F.lg;
    if (WL && (j == 0 || j == F.n)) continue;
    const Nbr q = nbr_of<MODEL>(w & (F.n - 1), j, F.n, F.lg);
    T nv[NCm];
    rows_any<MODEL, T, CORR, PM>(F.g, F.bg, F.rk, F.om, q, q.p, F.k, P, nv, sm);
#pragma unroll
    for (int c = 0; c < NCm; ++c) F.d[c][q.p] = F.f[c][q.p] - nv[c];
  }
  const int cnt = C.n * C.ny;
  for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
    const int J = w >> C.lg, I = w & (C.n - 1);
    if (WL && (J == 0 || J == C.n)) {
#pragma unroll
      for (int c = 0; c < NCm; ++c) {
        if (wall_copied(c)) continue;  // after the interior rows, below
        const T b = (c == 1) ? (J == 0 ? P.ub : P.ut) : T(0);
        C.g[c][w] = b;
        C.g0[c][w] = b;
      }
      continue;
    }
#pragma unroll
    for (int c = 0; c < NCm; ++c) {
      const T gr = fw9(F.g[c], 2 * I, 2 * J, F.n, F.lg);
      C.g[c][w] = gr;
      C.g0[c][w] = gr;
    }
    if constexpr (CORR) {
#pragma unroll
      for (int c = 0; c < NBase<MODEL>::value; ++c) C.bg[c][w] = fw9(F.bg[c], 2 * I, 2 * J, F.n, F.lg);
    }
  }
  __syncthreads();
  if constexpr (WL) {
    const int top = C.n << C.lg, stride = 1 << C.lg;
    for (int i = threadIdx.x; i < C.n; i += blockDim.x) {
#pragma unroll
      for (int c = 0; c < NCm; ++c) {
        if (!wall_copied(c)) continue;
        C.g[c][i] = C.g0[c][i] = C.g0[c][stride + i];
        C.g[c][top + i] = C.g0[c][top + i] = C.g0[c][top - stride + i];
      }
    }
    __syncthreads();
  }
  if constexpr (PM) {
    for (int w = threadIdx.x; w < cnt; w += blockDim.x) sm[w] = potential_any<MODEL, T, CORR>(C.g0, C.bg, w, P);
    __syncthreads();
  }
  for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
    const int J = w >> C.lg, I = w & (C.n - 1);
    if (WL && (J == 0 || J == C.n)) continue;
    const Nbr q = nbr_of<MODEL>(I, J, C.n, C.lg);
    T nv[NCm];
    rows_any<MODEL, T, CORR, PM>(C.g0, C.bg, C.rk, C.om, q, q.p, C.k, P, nv, sm);
#pragma unroll
    for (int c = 0; c < NCm; ++c) C.f[c][w] = fw9(F.d[c], 2 * I, 2 * J, F.n, F.lg) + nv[c];
  }
  __syncthreads();
}

// The top level's right-hand side completed in LDS: f (loaded: R d) +=
// N(g) of the loaded iterate (R g), the coarse right-hand side of
// tail_restrict formed for the tail's top.
template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void tail_complete_rhs(const Lvl<T> F, const Phys<T>& P, T* sm) {
  constexpr int NCm = NC<MODEL>::value;
  constexpr bool PM = tail_pm<MODEL>() > 0;
  const int cnt = F.n * F.ny;
  if constexpr (PM) {
    for (int w = threadIdx.x; w < cnt; w += blockDim.x) sm[w] = potential_any<MODEL, T, CORR>(F.g, F.bg, w, P);
    __syncthreads();
  }
  for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
    const Nbr q = nbr_of<MODEL>(w & (F.n - 1), w >> F.lg, F.n, F.lg);
    T nv[NCm];
    rows_any<MODEL, T, CORR, PM>(F.g, F.bg, F.rk, F.om, q, q.p, F.k, P, nv, sm);
#pragma unroll
    for (int c = 0; c < NCm; ++c) F.f[c][w] = F.f[c][w] + nv[c];
  }
  __syncthreads();
}

template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void tail_prolong(const Lvl<T> F, const Lvl<T> C, const Phys<T>& P) {
  // channel: the interior fine rows take the correction (the coarse wall rows
  // hold zero correction for u, v and the adjacent row's for rho, mu, kappa),
  // then the fine wall rows are refreshed
  constexpr int NCm = NC<MODEL>::value;
  constexpr bool WL = walls(MODEL);
  const int cnt = F.n * F.ny, mc = C.n - 1;
  for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
    const int j = w >> F.lg, i = w & (F.n - 1);
    if (WL && (j == 0 || j == F.n)) continue;
    const int I = i >> 1, J = j >> 1, I1 = (I + 1) & mc, J1 = WL ? (J + 1) : ((J + 1) & mc);
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
      if constexpr (cdft_like(MODEL)) {
        if (c == 0) x = project_any<T, CORR>(x, CORR ? F.bg[0][w] : T(0), P.delta);
      }
      F.g[c][w] = x;
    }
  }
  __syncthreads();
  tail_wall_rows<MODEL, T>(F);
}

template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void tail_body(const TailArgs<T>& A, const Phys<T>& P, const int* halt = nullptr) {
  // the V-cycle loop's stop flag, read with the loads below and tested after
  // them (nothing is stored before)
  const int hv = stop_flag(halt);
  constexpr int NCm = NC<MODEL>::value;
  constexpr int NB = CORR ? NBase<MODEL>::value : 0;
  constexpr int NR = NCoef<MODEL>::value;
  constexpr int WR = walls(MODEL) ? 1 : 0;
  extern __shared__ __align__(16) unsigned char tail_smem[];
  // level descriptors in LDS: S = LDS copies, G = the global arrays
  __shared__ Lvl<T> S[TAIL_MAX_LEVELS];
  __shared__ Lvl<T> G[TAIL_MAX_LEVELS];
  tail_lds_levels<NCm, NB, NR, WR, T>(A, reinterpret_cast<T*>(tail_smem), S, G);
  // the scratch array after the levels (CDFT potential)
  T* sm = tail_pm<MODEL>() ? as_lds(reinterpret_cast<T*>(tail_smem) + tail_lds_count<NCm, NB, NR, WR>(A.top_n, A.nt, A.d_from))
                           : nullptr;
  __syncthreads();
  // load: every global value a thread moves is read before it is stored
  for (int l = 0; l < A.nt; ++l) {
    const Lvl<T> s = tail_view<NCm, NB, NR, false>(S[l]);
    const Lvl<T> g = lvl_global(G[l]);
    const int cnt = g.n * g.ny;
    if (NR == 0 && l > 0) break;  // only the top level has anything to load
    for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
      T x[2 * NCm + NB + 2];
      if constexpr (NR == 2) {
        x[0] = g.rk[w];
        x[1] = g.om[w];
      }
      if (l == 0) {
#pragma unroll
        for (int c = 0; c < NCm; ++c) {
          x[2 + c] = g.g[c][w];
          x[2 + NCm + c] = g.f[c][w];
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) x[2 + 2 * NCm + c] = g.bg[c][w];
      }
      if constexpr (NR == 2) {
        s.rk[w] = x[0];
        s.om[w] = x[1];
      }
      if (l == 0) {
#pragma unroll
        for (int c = 0; c < NCm; ++c) {
          s.g[c][w] = x[2 + c];
          s.f[c][w] = x[2 + NCm + c];
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) s.bg[c][w] = x[2 + 2 * NCm + c];
      }
    }
  }
  __syncthreads();
  if (stop_set(hv)) return;
  if constexpr (!walls(MODEL)) {
    if (A.fc) tail_complete_rhs<MODEL, T, CORR>(tail_view<NCm, NB, NR, false>(S[0]), P, sm);
  }
  const int last = A.nt - 1;
  for (int l = 0; l < last; ++l) {
    const Lvl<T> F = tail_view<NCm, NB, NR, false>(S[l]);
    tail_sweeps<MODEL, T, CORR>(F, P, A.nu1, sm);
    if (l >= A.d_from)
      tail_restrict<MODEL, T, CORR>(tail_view<NCm, NB, NR, false, true>(S[l]), tail_view<NCm, NB, NR, true>(S[l + 1]), P, sm);
    else
      tail_restrict<MODEL, T, CORR>(F, tail_view<NCm, NB, NR, true>(S[l + 1]), P, sm);
  }
  tail_sweeps<MODEL, T, CORR>(tail_view<NCm, NB, NR, false>(S[last]), P, A.coarse_sweeps, sm);
  for (int l = last - 1; l >= 0; --l) {
    const Lvl<T> F = tail_view<NCm, NB, NR, false>(S[l]);
    tail_prolong<MODEL, T, CORR>(F, tail_view<NCm, NB, NR, true>(S[l + 1]), P);
    tail_sweeps<MODEL, T, CORR>(F, P, A.nu2, sm);
  }
  {
    const Lvl<T> s = tail_view<NCm, NB, NR, false>(S[0]);
    const Lvl<T> g = lvl_global(G[0]);
    const int cnt = g.n * g.ny;
    for (int w = threadIdx.x; w < cnt; w += blockDim.x) {
      T x[NCm];
#pragma unroll
      for (int c = 0; c < NCm; ++c) x[c] = s.g[c][w];
#pragma unroll
      for (int c = 0; c < NCm; ++c) g.g[c][w] = x[c];
    }
  }
}

template <int MODEL, typename T, bool CORR>
__global__ __launch_bounds__(TAIL_THREADS) void k_tail(TailArgs<T> A, Phys<T> P) {
  tail_body<MODEL, T, CORR>(A, P, P.halt);
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
