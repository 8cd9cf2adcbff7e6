// LDS-tiled kernels for the large grid levels.
//
// k_sweeps_tile: NSW damped red-black sweeps in one launch.  A workgroup owns a
// TILE_X x TILE_Y block of nodes and loads it with a halo of 2 NSW nodes (the
// iterate g and, for the hydrodynamic rows, the frozen rho^k into LDS).  Each half sweep updates the
// nodes of one colour in a box that shrinks by one node per half sweep, so
// after 2 NSW half sweeps the owned block holds exactly the values the
// whole-grid sweeps produce; the halo work is recomputed, not exchanged.  The
// iterate is double-buffered in global memory (read gin, write gout) so that
// no workgroup reads a neighbour's halo after that neighbour wrote it.  With
// PRO the FAS coarse-grid correction g += P(g_c - R g) is applied to every
// node as it is loaded (the prolongation fused into the first post-sweep).
//
// CORR = true runs the same kernel on the correction form of the
// mixed-precision inner solve (stencil.hpp); the base state is then staged
// in LDS beside the iterate.
//
// The V-cycle can fold the FAS restriction into these launches (RES = 3
// below): the last pre-smoothing launch of a level also forms R g and R d on
// the coarse nodes under its block; f_c = R d + N_c(R g) is then completed
// on the coarse grid (k_fas_rhs, or the tail kernel as it loads), or by the
// coarse level's own pre-smoothing launch (RES = 4) when that launch folds
// its restriction too.  The arithmetic is the restriction kernels'
// (restrict.hpp) and k_fas_rhs's.
#pragma once
#include "kernels.hpp"
#include "restrict.hpp"
#include "stencil.hpp"

namespace hfz {

// Tile shapes of the sweep kernel: TX x TY owned nodes per workgroup of NT
// threads.  Shape 0 is the default (the batched kernels use shapes 0 and 2);
// the tuner (tune.hpp) picks a shape per level by timing.  The small shapes
// (4-6) are for the latency-bound levels, where a 16 x 16 tiling leaves most
// compute units idle (64^2: 16 workgroups): more, smaller workgroups split
// each half sweep's updates over more units at the price of more recomputed
// halo.  The large ones (7-9) are for the large levels: a square tile
// recomputes less halo per owned node than a 64 x 16 one, and 1024 threads
// give each node of a half sweep its own thread.  The swept values do not
// depend on the shape; only the grouping of the stop-test partial sums does.
struct TileShape {
  int tx, ty, nt;
};
constexpr int NUM_TILE_SHAPES = 10;
constexpr TileShape kTileShapes[NUM_TILE_SHAPES] = {{32, 16, 256}, {32, 16, 512}, {64, 16, 512}, {16, 16, 256},
                                                    {16, 16, 512}, {16, 8, 256},  {8, 8, 256},   {32, 32, 512},
                                                    {32, 32, 1024}, {64, 16, 1024}};
constexpr int TILE_X = kTileShapes[0].tx;
constexpr int TILE_Y = kTileShapes[0].ty;
constexpr int TILE_THREADS = kTileShapes[0].nt;

template <typename T> struct Fld {
  T* c[5];
};

// RES selects what follows the sweeps on the owned block: 0 nothing, 1 the
// residual d = f - N(g) written to L.d (the input of the FAS restriction),
// 2 the block's partial sum of |d|^2 written to partial[block] (the stop test),
// 3 the FAS restriction of the block: R g into the coarse C.g and C.g0 and
// R d into C.f (to which N_c(R g) is added on the coarse grid afterwards; the
// correction form also restricts its base state into C.bg).  A residual
// needs the swept values one node beyond the block, hence the extra halo
// node; R d needs d one node below and left of the block as well, hence two
// for RES = 3.  RES = 4 is RES = 3 on a level whose right-hand side still holds
// R d from the restriction into it: the launch first completes f = R d + N(g)
// (g is R g before the first half sweep, so this is k_fas_rhs's value) in LDS
// over the nodes it updates, sweeps and restricts with that f, and writes the
// completed f of its block to L.d, from which the level's post-smoothing
// launch reads it (L.f itself stays R d: the neighbouring workgroups read their
// halo of it in the same launch).
// res_on false skips the residual (a batched launch whose instance has this
// level below its finest; uniform over the workgroup).  halt: the V-cycle
// loop's stop flag, read with the first loads and tested after the load phase
// (nothing is stored before it).
template <int MODEL, typename T, int NSW, bool PRO, int RES, bool CORR, int TS = 0>
__device__ __forceinline__ void sweeps_tile_body(const Lvl<T>& L, const Fld<T>& gin, const Fld<T>& gout,
                                                 const Lvl<T>& C, const Phys<T>& P, double* partial,
                                                 bool res_on = true, const int* halt = nullptr) {
  const int hv = stop_flag(halt);
  constexpr int NCm = NC<MODEL>::value;
  constexpr int NB = CORR ? NBase<MODEL>::value : 1;
  constexpr bool RK = NCoef<MODEL>::value > 0;  // the rows read rho^k
  constexpr int TILE_X = kTileShapes[TS].tx, TILE_Y = kTileShapes[TS].ty, TILE_THREADS = kTileShapes[TS].nt;
  constexpr bool FR = RES == 3 || RES == 4;  // the FAS restriction folded in
  constexpr bool FC = RES == 4;              // and this level's f completed first
  static_assert(!(FR && (walls(MODEL) || PRO)), "fused restriction: periodic pre-sweeps");
  constexpr int H = 2 * NSW + (FR ? 2 : (RES ? 1 : 0));
  constexpr int RX = TILE_X + 2 * H, RY = TILE_Y + 2 * H, RN = RX * RY;
  // coarse patch under the region (prolongation staging)
  constexpr int CRX = RX / 2 + 2, CRY = RY / 2 + 2, CRN = CRX * CRY;
  // CDFT: the potential M (a logarithm per node) is evaluated once per node
  // and half sweep into sm, for the nodes of the colour not being updated,
  // instead of at each of their four neighbours.
  constexpr bool PM = MODEL == CDFT;
  // channel (walls in y): rows outside 0..n are not loaded, only interior rows
  // are updated, and the wall rows of rho, mu, kappa in LDS follow the
  // adjacent rows: refreshed after the fused prolongation, and written by the
  // updaters of rows 1 and n - 1 in each half sweep (the block touching a
  // wall holds both it and the adjacent row: its region spans H >= 2 rows
  // beyond its owned block)
  constexpr bool WL = walls(MODEL);
  __shared__ T sg[NCm][RN];
  __shared__ T srk[RK ? RN : 1];
  __shared__ T sb[NB][CORR ? RN : 1];
  // RES = 3: d on the block and one node below and left of it
  constexpr int DX = TILE_X + 1, DN = DX * (TILE_Y + 1);
  __shared__ T sd[NCm][FR ? DN : 1];
  // RES = 4: the completed f and omega^k over the region (the sweeps read
  // them from LDS, indexed like g)
  __shared__ T sf[NCm][FC ? RN : 1];
  __shared__ T som[(FC && RK) ? RN : 1];
  // se (the coarse correction, read only while loading) and sm (the
  // potential, written only after the load) share one LDS array
  constexpr int SE = PRO ? NCm * CRN : 0, SM = PM ? RN : 0;
  __shared__ T sx[(SE > SM ? SE : SM) > 0 ? (SE > SM ? SE : SM) : 1];
  T(*se)[CRN] = reinterpret_cast<T(*)[CRN]>(sx);
  T* sm = sx;
  const int m = L.n - 1, lg = L.lg, nn = L.n;
  // XCD-contiguous tile numbering (tb also indexes the stop-test partial sum)
  int bx, by;
  const int tb = xcd_block(bx, by);
  // x0 + y0 is even for any H, so the colour of region node (lx, ly) is (lx + ly) & 1
  const int x0 = bx * TILE_X - H, y0 = by * TILE_Y - H;
  const int X0c = x0 >> 1, Y0c = y0 >> 1;  // floor halves (arithmetic shift)
  if constexpr (PRO) {
    const int mc = C.n - 1;
    for (int w = threadIdx.x; w < CRN; w += TILE_THREADS) {
      const int cy = w / CRX, cx = w - cy * CRX;
      int cj = Y0c + cy;
      if constexpr (WL) {
        if (cj < 0 || cj > C.n) continue;  // beyond the coarse walls: never read
      } else {
        cj &= mc;
      }
      const int pc = (cj << C.lg) + ((X0c + cx) & mc);
#pragma unroll
      for (int c = 0; c < NCm; ++c) se[c][w] = C.g[c][pc] - C.g0[c][pc];
    }
    __syncthreads();
  }
  for (int w = threadIdx.x; w < RN; w += TILE_THREADS) {
    const int ly = w / RX, lx = w - ly * RX;
    const int gi = (x0 + lx) & m;
    int gj = y0 + ly;
    if constexpr (WL) {
      if (gj < 0 || gj > nn) continue;  // beyond the walls: never read
    } else {
      gj &= m;
    }
    const int gp = (gj << lg) + gi;
    if constexpr (RK) srk[w] = L.rk[gp];
    if constexpr (FC && RK) som[w] = L.om[gp];
    if constexpr (CORR) {
#pragma unroll
      for (int c = 0; c < NB; ++c) sb[c][w] = L.bg[c][gp];
    }
#pragma unroll
    for (int c = 0; c < NCm; ++c) {
      T x = gin.c[c][gp];
      if constexpr (PRO) {
        if (WL && (gj == 0 || gj == nn)) {  // wall rows: refreshed below
          sg[c][w] = x;
          continue;
        }
        // bilinear prolongation of e (same arithmetic as k_prolong)
        const int gu = x0 + lx, gv = y0 + ly;
        const int cp = ((gv >> 1) - Y0c) * CRX + ((gu >> 1) - X0c);
        const int pi = gu & 1, pj = gv & 1;
        const T e00 = se[c][cp];
        T e;
        if (!pi && !pj)
          e = e00;
        else if (pi && !pj)
          e = T(0.5) * (e00 + se[c][cp + 1]);
        else if (!pi && pj)
          e = T(0.5) * (e00 + se[c][cp + CRX]);
        else
          e = T(0.25) * (e00 + se[c][cp + 1] + se[c][cp + CRX] + se[c][cp + CRX + 1]);
        x += e;
        if constexpr (cdft_like(MODEL)) {
          if (c == 0) x = project_any<T, CORR>(x, CORR ? L.bg[0][gp] : T(0), P.delta);
        }
      }
      sg[c][w] = x;
    }
  }
  __syncthreads();
  if (stop_set(hv)) return;
  // LDS rows of the channel's walls (valid when inside 0..RY-1)
  const int r0 = -y0, rn = nn - y0;
  auto wall_refresh = [&]() {
    for (int w = threadIdx.x; w < RX; w += TILE_THREADS) {
#pragma unroll
      for (int c = 0; c < NCm; ++c) {
        if (!wall_copied(c)) continue;
        if (r0 >= 0 && r0 + 1 < RY) sg[c][r0 * RX + w] = sg[c][(r0 + 1) * RX + w];
        if (rn >= 1 && rn < RY) sg[c][rn * RX + w] = sg[c][(rn - 1) * RX + w];
      }
    }
    __syncthreads();
  };
  if constexpr (WL && PRO) wall_refresh();
  const T* gl[NCm];
#pragma unroll
  for (int c = 0; c < NCm; ++c) gl[c] = sg[c];
  const T* bl[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) bl[c] = sb[(CORR && c < NB) ? c : 0];
  const T* fl[NCm];
#pragma unroll
  for (int c = 0; c < NCm; ++c) fl[c] = sf[c];
  if constexpr (FC) {
    // f = R d + N(R g) on the region less its outer ring (the nodes the first
    // half sweep may update), with k_fas_rhs's rows and operand order
    constexpr int BX = RX - 2, BN = BX * (RY - 2);
    for (int w = threadIdx.x; w < BN; w += TILE_THREADS) {
      const int r = w / BX, t = w - r * BX;
      const int lp = (1 + r) * RX + 1 + t;
      const int gp = (((y0 + 1 + r) & m) << lg) + ((x0 + 1 + t) & m);
      Nbr q;
      q.p = lp;
      q.e = lp + 1;
      q.w = lp - 1;
      q.n = lp + RX;
      q.s = lp - RX;
      T nv[NCm];
      rows_any<MODEL, T, CORR>(gl, bl, srk, som, q, lp, L.k, P, nv);
#pragma unroll
      for (int c = 0; c < NCm; ++c) sf[c][lp] = L.f[c][gp] + nv[c];
    }
    __syncthreads();
  }
  for (int k = 1; k <= 2 * NSW; ++k) {
    const int colour = (k - 1) & 1;
    if constexpr (PM) {
      // M at the other colour's nodes of the box one node wider than the
      // one updated below (their values are final for this half sweep)
      const int hm = (RX - 2 * k + 2) >> 1, cm = hm * (RY - 2 * k + 2);
      for (int w = threadIdx.x; w < cm; w += TILE_THREADS) {
        const int r = w / hm, t = w - r * hm;
        const int ly = k - 1 + r;
        const int lx = k - 1 + 2 * t + ((k - 1 + ly + colour + 1) & 1);
        const int lp = ly * RX + lx;
        sm[lp] = potential_any<MODEL, T, CORR>(gl, bl, lp, P);
      }
      __syncthreads();
    }
    const int half = (RX - 2 * k) >> 1, cnt = half * (RY - 2 * k);
    for (int w = threadIdx.x; w < cnt; w += TILE_THREADS) {
      const int r = w / half, t = w - r * half;
      const int ly = k + r;
      const int lx = k + 2 * t + ((k + ly + colour) & 1);
      if constexpr (WL) {
        if (y0 + ly < 1 || y0 + ly > nn - 1) continue;
      }
      Nbr q;
      q.p = ly * RX + lx;
      q.e = q.p + 1;
      q.w = q.p - 1;
      q.n = q.p + RX;
      q.s = q.p - RX;
      const int pf = ((WL ? (y0 + ly) : ((y0 + ly) & m)) << lg) + ((x0 + lx) & m);
      T out[NCm];
      if constexpr (FC)
        update_any<MODEL, T, CORR, PM>(gl, fl, bl, srk, som, q, q.p, L.k, P, out, sm);
      else
        update_any<MODEL, T, CORR, PM>(gl, L.f, bl, srk, L.om, q, pf, L.k, P, out, sm);
#pragma unroll
      for (int c = 0; c < NCm; ++c) sg[c][q.p] = out[c];
      if constexpr (WL) {
        // the wall copies of rho, mu, kappa next to a node on row 1 or n - 1:
        // no other update of this half sweep reads them, and the wall nodes
        // next to nodes not updated here already hold their values
        if (y0 + ly == 1 || y0 + ly == nn - 1) {
          const int wp = q.p + (y0 + ly == 1 ? -RX : RX);
#pragma unroll
          for (int c = 0; c < NCm; ++c)
            if (wall_copied(c)) sg[c][wp] = out[c];
        }
      }
    }
    __syncthreads();
  }
  if constexpr (PM && RES != 0) {
    if (res_on) {
      // M on the nodes the residual rows read: the owned block and its
      // one-node ring (RES = 3, 4: the block of d and its ring)
      constexpr int E0 = FR ? 2 : 1, BX = TILE_X + E0 + 1, BN = BX * (TILE_Y + E0 + 1);
      for (int w = threadIdx.x; w < BN; w += TILE_THREADS) {
        const int r = w / BX, t = w - r * BX;
        const int lp = (H - E0 + r) * RX + H - E0 + t;
        sm[lp] = potential_any<MODEL, T, CORR>(gl, bl, lp, P);
      }
      __syncthreads();
    }
  }
  double acc = 0.0;
  for (int w = threadIdx.x; w < TILE_X * TILE_Y; w += TILE_THREADS) {
    const int ty = w / TILE_X, tx = w - ty * TILE_X;
    const int lp = (ty + H) * RX + tx + H;
    const int gy = WL ? (y0 + H + ty) : ((y0 + H + ty) & m);
    const int gp = (gy << lg) + ((x0 + H + tx) & m);
#pragma unroll
    for (int c = 0; c < NCm; ++c) gout.c[c][gp] = sg[c][lp];
    if constexpr (FC) {
#pragma unroll
      for (int c = 0; c < NCm; ++c) L.d[c][gp] = sf[c][lp];
    }
    if constexpr (WL) {
      // the top wall row n belongs to no block: the block owning row n - 1 writes it
      if (gy == nn - 1) {
#pragma unroll
        for (int c = 0; c < NCm; ++c) gout.c[c][gp + (1 << lg)] = sg[c][lp + RX];
      }
      if (gy == 0) continue;  // the bottom wall row: no equation
    }
    if constexpr (RES == 1 || RES == 2) {
      if (!res_on) continue;
      Nbr q;
      q.p = lp;
      q.e = lp + 1;
      q.w = lp - 1;
      q.n = lp + RX;
      q.s = lp - RX;
      T nv[NCm];
      rows_any<MODEL, T, CORR, PM>(gl, bl, srk, L.om, q, gp, L.k, P, nv, sm);
#pragma unroll
      for (int c = 0; c < NCm; ++c) {
        const T d = L.f[c][gp] - nv[c];
        if constexpr (RES == 1) {
          L.d[c][gp] = d;
        } else {
          acc += double(d) * double(d);
        }
      }
    }
  }
  if constexpr (RES == 2) {
    if (res_on) {
      __shared__ double red[TILE_THREADS / 64];
      const double r = block_sum(acc, red);
      if (threadIdx.x == 0) partial[tb] = r;
    }
  }
  if constexpr (FR) {
    // d = f - N(g) on the block and one node below and left of it (the fine
    // nodes under the 9-point stencils of the block's coarse nodes)
    for (int w = threadIdx.x; w < DN; w += TILE_THREADS) {
      const int r = w / DX, t = w - r * DX;
      const int lp = (H - 1 + r) * RX + H - 1 + t;
      const int gp = (((y0 + H - 1 + r) & m) << lg) + ((x0 + H - 1 + t) & m);
      Nbr q;
      q.p = lp;
      q.e = lp + 1;
      q.w = lp - 1;
      q.n = lp + RX;
      q.s = lp - RX;
      T nv[NCm];
      if constexpr (FC) {
        rows_any<MODEL, T, CORR, PM>(gl, bl, srk, som, q, lp, L.k, P, nv, sm);
#pragma unroll
        for (int c = 0; c < NCm; ++c) sd[c][w] = sf[c][lp] - nv[c];
      } else {
        rows_any<MODEL, T, CORR, PM>(gl, bl, srk, L.om, q, gp, L.k, P, nv, sm);
#pragma unroll
        for (int c = 0; c < NCm; ++c) sd[c][w] = L.f[c][gp] - nv[c];
      }
    }
    __syncthreads();
    // the block's coarse nodes: R g into C.g and C.g0, R d into C.f
    constexpr int CX = TILE_X / 2, CN = CX * (TILE_Y / 2);
    const int I0 = bx * CX, J0 = by * (TILE_Y / 2);
    for (int w = threadIdx.x; w < CN; w += TILE_THREADS) {
      const int cy = w / CX, cx = w - cy * CX;
      const int pc = ((J0 + cy) << C.lg) + I0 + cx;
      const int lg2 = (H + 2 * cy) * RX + H + 2 * cx;
      const int ld2 = (2 * cy + 1) * DX + 2 * cx + 1;
#pragma unroll
      for (int c = 0; c < NCm; ++c) {
        const T gr = fw9l(sg[c], lg2, RX);
        C.g[c][pc] = gr;
        C.g0[c][pc] = gr;
        C.f[c][pc] = fw9l(sd[c], ld2, DX);
      }
      if constexpr (CORR) {
        // the correction form's base state restricted with the iterate
#pragma unroll
        for (int c = 0; c < NB; ++c) C.bg[c][pc] = fw9l(sb[c], lg2, RX);
      }
    }
  }
}

// Whether the RES = 4 form of two fused sweeps in tile shape TS fits the LDS
// of a compute unit (160 KiB): the kernel body's arrays for NSW = 2, PRO =
// false, RES = 4 (large tiles do not fit; there k_fas_rhs completes f).
template <int MODEL, typename T, bool CORR, int TS> constexpr bool fold_rhs_fits() {
  constexpr int NCm = NC<MODEL>::value, NB = CORR ? NBase<MODEL>::value : 1;
  constexpr bool RK = NCoef<MODEL>::value > 0, PM = MODEL == CDFT;
  constexpr int H = 2 * 2 + 2, TX = kTileShapes[TS].tx, TY = kTileShapes[TS].ty;
  constexpr size_t RN = (size_t)(TX + 2 * H) * (TY + 2 * H), DN = (size_t)(TX + 1) * (TY + 1);
  constexpr size_t vals = NCm * RN + (RK ? RN : 1) + NB * (CORR ? RN : 1) + NCm * DN + NCm * RN +
                          (RK ? RN : 1) + (PM ? RN : 1);
  return vals * sizeof(T) <= 160 * 1024;
}

template <int MODEL, typename T, bool CORR> bool fold_rhs_fits_shape(int ts) {
  constexpr bool fits[NUM_TILE_SHAPES] = {
      fold_rhs_fits<MODEL, T, CORR, 0>(), fold_rhs_fits<MODEL, T, CORR, 1>(), fold_rhs_fits<MODEL, T, CORR, 2>(),
      fold_rhs_fits<MODEL, T, CORR, 3>(), fold_rhs_fits<MODEL, T, CORR, 4>(), fold_rhs_fits<MODEL, T, CORR, 5>(),
      fold_rhs_fits<MODEL, T, CORR, 6>(), fold_rhs_fits<MODEL, T, CORR, 7>(), fold_rhs_fits<MODEL, T, CORR, 8>(),
      fold_rhs_fits<MODEL, T, CORR, 9>()};
  return ts >= 0 && ts < NUM_TILE_SHAPES && fits[ts];
}

template <int MODEL, typename T, int NSW, bool PRO, int RES, bool CORR, int TS = 0>
__global__ __launch_bounds__(kTileShapes[TS].nt) void k_sweeps_tile(Lvl<T> L, Fld<T> gin, Fld<T> gout, Lvl<T> C,
                                                                    Phys<T> P, double* partial) {
  sweeps_tile_body<MODEL, T, NSW, PRO, RES, CORR, TS>(L, gin, gout, C, P, partial, true, P.halt);
}

// Batched form: instance blockIdx.z of the instances that have a level of this
// size (all of the same size), descriptors in device arrays, skipped when not
// active.  The iterate is read from g (inb = 0) or gb (inb = 1) and written to
// the other buffer; partial sums go to partial + z * pstride, RES = 2 only for
// the instances whose finest level is at depth `depth` (topd[z]; the others
// are inside their V-cycle).  TS: tile shape (0 or 2).
template <int MODEL, typename T, int NSW, bool PRO, int RES, bool CORR, int TS = 0>
__global__ __launch_bounds__(kTileShapes[TS].nt) void k_sweeps_tile_b(const Lvl<T>* Ls, const Lvl<T>* Cs,
                                                                const Phys<T>* Ps, const int* active, int inb,
                                                                double* partial, int pstride, const int* topd,
                                                                int depth) {
  const int z = blockIdx.z;
  if (!active[z]) return;
  const Lvl<T> L = lvl_global(Ls[z]);
  Fld<T> a{}, b{};
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    a.c[c] = L.g[c];
    b.c[c] = L.gb[c];
  }
  const Lvl<T> C = PRO ? lvl_global(Cs[z]) : L;
  sweeps_tile_body<MODEL, T, NSW, PRO, RES, CORR, TS>(L, inb ? b : a, inb ? a : b, C, Ps[z],
                                                      partial + (size_t)z * pstride, RES != 2 || topd[z] == depth);
}

}  // namespace hfz
