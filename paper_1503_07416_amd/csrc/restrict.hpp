// k_restrict_fas_tile: the FAS coarse problem of one level in one launch:
// R g on a coarse tile plus a one-node halo (into LDS), then
// f_c = N_c(R g) + R d with d = f - N(g) precomputed on the fine grid
// (9-point full weighting R, App. G's FAS scheme).  CORR = true restricts the
// correction form of the mixed-precision inner solve: the base state is
// restricted along with the iterate.
#pragma once
#include "kernels.hpp"
#include "stencil.hpp"

namespace hfz {

constexpr int RTILE = 16;  // coarse tile edge of the restriction kernel

template <typename T>
__device__ __forceinline__ T fw9g(const T* f, int i, int j, int n, int lg) {
  const int m = n - 1;
  const int ie = (i + 1) & m, iw = (i - 1) & m;
  const int rc = j << lg, rn = ((j + 1) & m) << lg, rs = ((j - 1) & m) << lg;
  return (T(4) * f[rc + i] + T(2) * (f[rc + ie] + f[rc + iw] + f[rn + i] + f[rs + i]) +
          (f[rn + ie] + f[rn + iw] + f[rs + ie] + f[rs + iw])) *
         T(0.0625);
}

// F.g must point at the current fine iterate and F.d at f - N(g) of it.  In
// the correction form the coarse base C.bg = R F.bg is written here too.
template <int MODEL, typename T, bool CORR>
__device__ __forceinline__ void restrict_fas_body(const Lvl<T>& F, const Lvl<T>& C, const Phys<T>& P) {
  constexpr int NCm = NC<MODEL>::value;
  constexpr int NB = CORR ? 3 : 1;
  constexpr int RX = RTILE + 2, RN = RX * RX;
  __shared__ T sg[NCm][RN];
  __shared__ T srk[RN];
  __shared__ T sb[NB][CORR ? RN : 1];
  const int mc = C.n - 1;
  const int X0 = (int)blockIdx.x * RTILE - 1, Y0 = (int)blockIdx.y * RTILE - 1;
  for (int w = threadIdx.x; w < RN; w += RTILE * RTILE) {
    const int ly = w / RX, lx = w - ly * RX;
    const int I = (X0 + lx) & mc, J = (Y0 + ly) & mc;
    srk[w] = C.rk[(J << C.lg) + I];
#pragma unroll
    for (int c = 0; c < NCm; ++c) sg[c][w] = fw9g(F.g[c], 2 * I, 2 * J, F.n, F.lg);
    if constexpr (CORR) {
#pragma unroll
      for (int c = 0; c < 3; ++c) sb[c][w] = fw9g(F.bg[c], 2 * I, 2 * J, F.n, F.lg);
    }
  }
  __syncthreads();
  const T* gl[NCm];
#pragma unroll
  for (int c = 0; c < NCm; ++c) gl[c] = sg[c];
  const T* bl[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) bl[c] = sb[CORR ? c : 0];
  const int ty = threadIdx.x / RTILE, tx = threadIdx.x - ty * RTILE;
  const int ly = ty + 1, lx = tx + 1;
  const int I = (X0 + lx) & mc, J = (Y0 + ly) & mc;
  const int pc = (J << C.lg) + I;
  Nbr q;
  q.p = ly * RX + lx;
  q.e = q.p + 1;
  q.w = q.p - 1;
  q.n = q.p + RX;
  q.s = q.p - RX;
  T nv[NCm];
  rows_any<MODEL, T, CORR>(gl, bl, srk, C.om, q, pc, C.k, P, nv);
#pragma unroll
  for (int c = 0; c < NCm; ++c) {
    const T gr = sg[c][q.p];
    C.g[c][pc] = gr;
    C.g0[c][pc] = gr;
    C.f[c][pc] = fw9g(F.d[c], 2 * I, 2 * J, F.n, F.lg) + nv[c];
  }
  if constexpr (CORR) {
#pragma unroll
    for (int c = 0; c < 3; ++c) C.bg[c][pc] = sb[c][q.p];
  }
}

template <int MODEL, typename T, bool CORR>
__global__ __launch_bounds__(RTILE* RTILE) void k_restrict_fas_tile(Lvl<T> F, Lvl<T> C, Phys<T> P) {
  restrict_fas_body<MODEL, T, CORR>(F, C, P);
}

// Batched form (instance blockIdx.z); the fine iterate is in g (inb = 0) or gb.
template <int MODEL, typename T, bool CORR>
__global__ __launch_bounds__(RTILE* RTILE) void k_restrict_fas_tile_b(const Lvl<T>* Fs, const Lvl<T>* Cs,
                                                                      const Phys<T>* Ps, const int* active,
                                                                      int inb) {
  const int z = blockIdx.z;
  if (!active[z]) return;
  Lvl<T> F = lvl_global(Fs[z]);
  if (inb) {
#pragma unroll
    for (int c = 0; c < 5; ++c) F.g[c] = F.gb[c];
  }
  restrict_fas_body<MODEL, T, CORR>(F, lvl_global(Cs[z]), Ps[z]);
}

}  // namespace hfz
