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
__device__ __forceinline__ void restrict_fas_body(const Lvl<T>& F, const Lvl<T>& C, const Phys<T>& P,
                                                  bool remap = true) {
  constexpr int NCm = NC<MODEL>::value;
  constexpr int NB = CORR ? NBase<MODEL>::value : 1;
  constexpr bool RK = NCoef<MODEL>::value > 0;
  constexpr int RX = RTILE + 2, RN = RX * RX;
  __shared__ T sg[NCm][RN];
  __shared__ T srk[RK ? RN : 1];
  __shared__ T sb[NB][CORR ? RN : 1];
  // channel (walls in y): coarse wall rows 0 and C.n take the boundary values
  // (u = u_wall, v = 0; rho, mu, kappa copy the adjacent coarse row), R g is
  // formed on the interior coarse rows, whose footprints lie on fine rows
  // 1..F.n-1, and f_c only there
  constexpr bool WL = walls(MODEL);
  const int mc = C.n - 1;
  int bx = (int)blockIdx.x, by = (int)blockIdx.y;
  if (remap) xcd_block(bx, by);  // XCD-contiguous block numbering
  const int X0 = bx * RTILE - 1, Y0 = by * RTILE - 1;
  for (int w = threadIdx.x; w < RN; w += RTILE * RTILE) {
    const int ly = w / RX, lx = w - ly * RX;
    const int I = (X0 + lx) & mc;
    int J = Y0 + ly;
    if constexpr (WL) {
      if (J < 0 || J > C.n) continue;  // beyond the walls: never read
    } else {
      J &= mc;
    }
    if constexpr (RK) srk[w] = C.rk[(J << C.lg) + I];
    if (WL && (J == 0 || J == C.n)) {
#pragma unroll
      for (int c = 0; c < NCm; ++c)
        if (!wall_copied(c)) sg[c][w] = (c == 1) ? (J == 0 ? P.ub : P.ut) : T(0);
      continue;
    }
#pragma unroll
    for (int c = 0; c < NCm; ++c) sg[c][w] = fw9g(F.g[c], 2 * I, 2 * J, F.n, F.lg);
    if constexpr (CORR) {
#pragma unroll
      for (int c = 0; c < NB; ++c) sb[c][w] = fw9g(F.bg[c], 2 * I, 2 * J, F.n, F.lg);
    }
  }
  __syncthreads();
  if constexpr (WL) {
    const int r0 = -Y0, rn = C.n - Y0;  // LDS rows of the coarse walls
    for (int w = threadIdx.x; w < RX; w += RTILE * RTILE) {
#pragma unroll
      for (int c = 0; c < NCm; ++c) {
        if (!wall_copied(c)) continue;
        if (r0 >= 0 && r0 + 1 < RX) sg[c][r0 * RX + w] = sg[c][(r0 + 1) * RX + w];
        if (rn >= 1 && rn < RX) sg[c][rn * RX + w] = sg[c][(rn - 1) * RX + w];
      }
    }
    __syncthreads();
  }
  const T* gl[NCm];
#pragma unroll
  for (int c = 0; c < NCm; ++c) gl[c] = sg[c];
  const T* bl[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) bl[c] = sb[(CORR && c < NB) ? c : 0];
  const int ty = threadIdx.x / RTILE, tx = threadIdx.x - ty * RTILE;
  const int ly = ty + 1, lx = tx + 1;
  const int I = (X0 + lx) & mc, J = WL ? (Y0 + ly) : ((Y0 + ly) & mc);
  const int pc = (J << C.lg) + I;
  Nbr q;
  q.p = ly * RX + lx;
  q.e = q.p + 1;
  q.w = q.p - 1;
  q.n = q.p + RX;
  q.s = q.p - RX;
  if constexpr (WL) {
    // the wall rows: R g (boundary values) only; the block owning row C.n - 1
    // also writes the top wall row, which belongs to no block
    if (J == C.n - 1) {
#pragma unroll
      for (int c = 0; c < NCm; ++c) {
        C.g[c][pc + (1 << C.lg)] = sg[c][q.n];
        C.g0[c][pc + (1 << C.lg)] = sg[c][q.n];
      }
    }
    if (J == 0) {
#pragma unroll
      for (int c = 0; c < NCm; ++c) {
        C.g[c][pc] = sg[c][q.p];
        C.g0[c][pc] = sg[c][q.p];
      }
      return;
    }
  }
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
    for (int c = 0; c < NB; ++c) C.bg[c][pc] = sb[c][q.p];
  }
}

template <int MODEL, typename T, bool CORR>
__global__ __launch_bounds__(RTILE* RTILE) void k_restrict_fas_tile(Lvl<T> F, Lvl<T> C, Phys<T> P) {
  if (halted(P.halt)) return;
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
  restrict_fas_body<MODEL, T, CORR>(F, lvl_global(Cs[z]), Ps[z], false);
}

// Staged form: the fine iterate under the stencils of a coarse tile and its
// ring, and the fine residual under the tile's own stencils, are read into LDS
// in one coalesced phase; R g, N_c(R g) and R d are then formed from LDS.  RT is
// the coarse tile edge, NT the workgroup size.  Same arithmetic, in the same
// order, as restrict_fas_body.
template <typename T> __device__ __forceinline__ T fw9l(const T* f, int p, int stride) {
  return (T(4) * f[p] + T(2) * (f[p + 1] + f[p - 1] + f[p + stride] + f[p - stride]) +
          (f[p + stride + 1] + f[p + stride - 1] + f[p - stride + 1] + f[p - stride - 1])) *
         T(0.0625);
}

template <int MODEL, typename T, bool CORR, int RT, int NT>
__device__ __forceinline__ void restrict_fas_staged(const Lvl<T>& F, const Lvl<T>& C, const Phys<T>& P,
                                                    const int* halt = nullptr, bool remap = true) {
  const int hv = stop_flag(halt);  // tested after the load phase (nothing is stored before)
  constexpr int NCm = NC<MODEL>::value;
  constexpr int NB = CORR ? NBase<MODEL>::value : 1;
  constexpr bool RK = NCoef<MODEL>::value > 0;
  constexpr int CX = RT + 2, CN = CX * CX;      // coarse tile and its ring
  constexpr int FX = 2 * RT + 5, FN = FX * FX;  // fine nodes under the ring's stencils
  constexpr int DX = 2 * RT + 1, DN = DX * DX;  // fine nodes under the tile's stencils
  __shared__ T fg[NCm][FN];
  __shared__ T fb[NB][CORR ? FN : 1];
  __shared__ T fd[NCm][DN];
  __shared__ T sg[NCm][CN];
  __shared__ T sb[NB][CORR ? CN : 1];
  __shared__ T srk[RK ? CN : 1];
  const int mc = C.n - 1, mf = F.n - 1;
  int bx = (int)blockIdx.x, by = (int)blockIdx.y;
  if (remap) xcd_block(bx, by);                  // XCD-contiguous block numbering
  const int X0 = bx * RT - 1, Y0 = by * RT - 1;  // coarse ring origin
  const int fx0 = 2 * X0 - 1, fy0 = 2 * Y0 - 1;                              // fine origin of fg
  for (int w = threadIdx.x; w < FN; w += NT) {
    const int ly = w / FX, lx = w - ly * FX;
    const int p = (((fy0 + ly) & mf) << F.lg) + ((fx0 + lx) & mf);
#pragma unroll
    for (int c = 0; c < NCm; ++c) fg[c][w] = F.g[c][p];
    if constexpr (CORR) {
#pragma unroll
      for (int c = 0; c < NB; ++c) fb[c][w] = F.bg[c][p];
    }
  }
  for (int w = threadIdx.x; w < DN; w += NT) {
    const int ly = w / DX, lx = w - ly * DX;
    const int p = (((fy0 + 2 + ly) & mf) << F.lg) + ((fx0 + 2 + lx) & mf);
#pragma unroll
    for (int c = 0; c < NCm; ++c) fd[c][w] = F.d[c][p];
  }
  if constexpr (RK) {
    for (int w = threadIdx.x; w < CN; w += NT) {
      const int ly = w / CX, lx = w - ly * CX;
      srk[w] = C.rk[(((Y0 + ly) & mc) << C.lg) + ((X0 + lx) & mc)];
    }
  }
  __syncthreads();
  if (stop_set(hv)) return;
  for (int w = threadIdx.x; w < CN; w += NT) {
    const int ly = w / CX, lx = w - ly * CX;
    const int fl = (1 + 2 * ly) * FX + 1 + 2 * lx;  // fine node under coarse (X0 + lx, Y0 + ly)
#pragma unroll
    for (int c = 0; c < NCm; ++c) sg[c][w] = fw9l(fg[c], fl, FX);
    if constexpr (CORR) {
#pragma unroll
      for (int c = 0; c < NB; ++c) sb[c][w] = fw9l(fb[c], fl, FX);
    }
  }
  __syncthreads();
  const T* gl[NCm];
#pragma unroll
  for (int c = 0; c < NCm; ++c) gl[c] = sg[c];
  const T* bl[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) bl[c] = sb[(CORR && c < NB) ? c : 0];
  for (int w = threadIdx.x; w < RT * RT; w += NT) {
    const int ty = w / RT, tx = w - ty * RT;
    const int ly = ty + 1, lx = tx + 1;
    const int pc = (((Y0 + ly) & mc) << C.lg) + ((X0 + lx) & mc);
    Nbr q;
    q.p = ly * CX + lx;
    q.e = q.p + 1;
    q.w = q.p - 1;
    q.n = q.p + CX;
    q.s = q.p - CX;
    T nv[NCm];
    rows_any<MODEL, T, CORR>(gl, bl, srk, C.om, q, pc, C.k, P, nv);
    const int fl = (1 + 2 * ty) * DX + 1 + 2 * tx;
#pragma unroll
    for (int c = 0; c < NCm; ++c) {
      const T gr = sg[c][q.p];
      C.g[c][pc] = gr;
      C.g0[c][pc] = gr;
      C.f[c][pc] = fw9l(fd[c], fl, DX) + nv[c];
    }
    if constexpr (CORR) {
#pragma unroll
      for (int c = 0; c < NB; ++c) C.bg[c][pc] = sb[c][q.p];
    }
  }
}

template <int MODEL, typename T, bool CORR, int RT, int NT>
__global__ __launch_bounds__(NT) void k_restrict_fas_staged(Lvl<T> F, Lvl<T> C, Phys<T> P) {
  restrict_fas_staged<MODEL, T, CORR, RT, NT>(F, C, P, P.halt);
}

// Batched staged form (instance blockIdx.z; the fine iterate in g, inb = 0,
// or gb).
template <int MODEL, typename T, bool CORR, int RT, int NT>
__global__ __launch_bounds__(NT) void k_restrict_fas_staged_b(const Lvl<T>* Fs, const Lvl<T>* Cs,
                                                             const Phys<T>* Ps, const int* active, int inb) {
  const int z = blockIdx.z;
  if (!active[z]) return;
  Lvl<T> F = lvl_global(Fs[z]);
  if (inb) {
#pragma unroll
    for (int c = 0; c < 5; ++c) F.g[c] = F.gb[c];
  }
  restrict_fas_staged<MODEL, T, CORR, RT, NT>(F, lvl_global(Cs[z]), Ps[z], nullptr, false);
}

// Restriction variants the tuner chooses from: 0 the direct kernel (coarse
// tile 16), 1 the staged kernel with coarse tile 8, 2 with coarse tile 16,
// 3 with coarse tile 16 and 512 threads.
constexpr int NUM_RESTRICT_SHAPES = 4;
constexpr int kRestrictTile[NUM_RESTRICT_SHAPES] = {16, 8, 16, 16};

}  // namespace hfz
