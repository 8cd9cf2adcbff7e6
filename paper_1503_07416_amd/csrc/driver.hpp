// Host-side FAS V-cycle driver: enqueues one V(nu1, nu2) cycle over a level
// hierarchy.  Large levels use the LDS-tiled kernels (tile.hpp), the small
// levels at the bottom the one-workgroup tail kernel (tail.hpp); the plain
// per-level kernels (kernels.hpp) remain for configurations the tiled ones do
// not cover (full form only).  The same driver runs the FP64 solve
// (T = double, full form) and the FP32 inner solve of the mixed-precision
// step (T = float, correction form).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "kernels.hpp"
#include "tail.hpp"
#include "restrict.hpp"
#include "tile.hpp"

namespace hfz {

template <typename T> struct Hier {
  std::vector<Lvl<T>> L;    // finest first
  Lvl<T>* desc = nullptr;   // device copy of L (the tail kernel reads it)
  size_t tail_lds_max = 0;  // dynamic LDS the tail kernel may use
  std::vector<int> tile_shape;      // tile shape of the sweep kernel per level (tile.hpp)
  std::vector<int> restrict_shape;  // restriction variant per fine level (restrict.hpp)
  std::vector<int> sweep_fuse;      // sweeps per tiled launch per level (2 fused, or 1)
  std::vector<char> fused;          // per level: the FAS restriction folded into the pre-sweep launch
  bool fold_rhs = true;             // a folded level completes its own coarse right-hand side (RES = 4)
  Phys<T> P{};
};

struct Cycle {
  hipStream_t stream = nullptr;
  int nu1 = 2, nu2 = 2, coarse_sweeps = 4;
  int tail_n = 32;
  bool use_tiles = true;
  double* partial = nullptr;  // stop-test partial sums of the finest level
  const int* halt = nullptr;  // device stop flag of the V-cycle loop (the kernels' Phys carry it too)
  int norm_partials = 0;      // out: > 0 when the last post-sweep left that many partials
};

inline dim3 grid2(int nx, int ny, dim3 b) { return dim3((nx + b.x - 1) / b.x, (ny + b.y - 1) / b.y); }
inline dim3 block2(int nx, int ny) {
  const int bx = std::min(64, nx);
  return dim3(bx, std::max(1, std::min(256 / bx, ny)));
}

template <typename T> Fld<T> fld(T* const* p) {
  Fld<T> f{};
  for (int c = 0; c < 5; ++c) f.c[c] = p[c];
  return f;
}

// Damped red-black sweeps with the per-colour kernels (full form).
template <int MODEL, typename T> void smooth_level(Hier<T>& H, Cycle& K, int l, int sweeps) {
  const Lvl<T>& L = H.L[l];
  const dim3 b = block2(L.n / 2, L.ny), g = grid2(L.n / 2, L.ny, b);
  for (int k = 0; k < sweeps; ++k) {
    for (int colour = 0; colour < 2; ++colour) {
      if (l == 0)
        k_smooth_colour<MODEL, T, 1><<<g, b, 0, K.stream>>>(L, H.P, colour);
      else
        k_smooth_colour<MODEL, T, 0><<<g, b, 0, K.stream>>>(L, H.P, colour);
      if constexpr (walls(MODEL)) {
        const dim3 bw = block2(L.n, 1);
        k_wall_rows<T><<<grid2(L.n, 1, bw), bw, 0, K.stream>>>(L, K.halt);
      }
    }
  }
}

// LDS plan of the tail from a level of size top_n with nt levels: whether
// every level fits in the LDS the tail kernel may use, and from which level
// down the residual scratch d fits in LDS too (d_from = nt: none).  Grids of
// 16^2 and below always fit.
template <int MODEL, typename T, bool CORR> bool tail_plan(int top_n, int nt, size_t lds_max, int* d_from) {
  constexpr int NCm = NC<MODEL>::value, NB = CORR ? NBase<MODEL>::value : 0, NR = NCoef<MODEL>::value;
  constexpr int WR = walls(MODEL) ? 1 : 0;
  constexpr int PMA = tail_pm<MODEL>();
  if (nt > TAIL_MAX_LEVELS || tail_lds_count<NCm, NB, NR, WR, PMA>(top_n, nt, nt) * sizeof(T) > lds_max) return false;
  int df = nt;
  while (df > 0 && tail_lds_count<NCm, NB, NR, WR, PMA>(top_n, nt, df - 1) * sizeof(T) <= lds_max) --df;
  if (d_from) *d_from = df;
  return true;
}

template <int MODEL, typename T, bool CORR> void tail_launch(Hier<T>& H, Cycle& K, int l, bool fc = false) {
  constexpr int NCm = NC<MODEL>::value, NB = CORR ? NBase<MODEL>::value : 0, NR = NCoef<MODEL>::value;
  TailArgs<T> A{};
  A.nt = (int)H.L.size() - l;
  A.Lg = H.desc + l;
  A.top_n = H.L[l].n;
  A.nu1 = K.nu1;
  A.nu2 = K.nu2;
  A.coarse_sweeps = K.coarse_sweeps;
  A.fc = fc ? 1 : 0;
  tail_plan<MODEL, T, CORR>(A.top_n, A.nt, H.tail_lds_max, &A.d_from);
  const size_t sh =
      tail_lds_count<NCm, NB, NR, walls(MODEL) ? 1 : 0, tail_pm<MODEL>()>(A.top_n, A.nt, A.d_from) * sizeof(T);
  k_tail<MODEL, T, CORR><<<1, TAIL_THREADS, sh, K.stream>>>(A, H.P);
}

// Launches the tiled sweep kernel of shape ts on level L; returns its
// number of workgroups (= stop-test partial sums when res == 2).  res 3 (the
// restriction into C folded in) only without PRO and walls; res 4 (the same
// after completing L's own right-hand side) also only with two sweeps in a
// shape whose arrays fit the LDS (fold_rhs_fits; returns 0 and launches
// nothing otherwise).
template <int MODEL, typename T, bool CORR, int NSW, bool PRO, int TS>
int tile_launch_shape(Hier<T>& H, Cycle& K, const Lvl<T>& L, const Fld<T>& in, const Fld<T>& out,
                      const Lvl<T>& C, int res) {
  constexpr TileShape S = kTileShapes[TS];
  const dim3 grid(L.n / S.tx, L.n / S.ty);
  if constexpr (!PRO && !walls(MODEL)) {
    if (res == 3) {
      k_sweeps_tile<MODEL, T, NSW, false, 3, CORR, TS><<<grid, S.nt, 0, K.stream>>>(L, in, out, C, H.P, K.partial);
      return (int)(grid.x * grid.y);
    }
    if (res == 4) {
      if constexpr (NSW == 2 && fold_rhs_fits<MODEL, T, CORR, TS>()) {
        k_sweeps_tile<MODEL, T, 2, false, 4, CORR, TS><<<grid, S.nt, 0, K.stream>>>(L, in, out, C, H.P, K.partial);
        return (int)(grid.x * grid.y);
      }
      return 0;
    }
  }
  if (res == 1)
    k_sweeps_tile<MODEL, T, NSW, PRO, 1, CORR, TS><<<grid, S.nt, 0, K.stream>>>(L, in, out, C, H.P, K.partial);
  else if (res == 2)
    k_sweeps_tile<MODEL, T, NSW, PRO, 2, CORR, TS><<<grid, S.nt, 0, K.stream>>>(L, in, out, C, H.P, K.partial);
  else
    k_sweeps_tile<MODEL, T, NSW, PRO, 0, CORR, TS><<<grid, S.nt, 0, K.stream>>>(L, in, out, C, H.P, K.partial);
  return (int)(grid.x * grid.y);
}

// The FAS restriction from fine level F (iterate in F.g, residual in F.d) to
// C in variant rs (restrict.hpp).
template <int MODEL, typename T, bool CORR>
void restrict_launch(Hier<T>& H, Cycle& K, const Lvl<T>& F, const Lvl<T>& C, int rs) {
  if (rs < 0 || rs >= NUM_RESTRICT_SHAPES || C.n % kRestrictTile[rs] != 0) rs = 0;
  if constexpr (walls(MODEL)) rs = 0;  // the channel's wall rows are handled by the direct kernel
  const int rt = kRestrictTile[rs];
  const dim3 grid(C.n / rt, C.n / rt);
  if (rs == 1)
    k_restrict_fas_staged<MODEL, T, CORR, 8, 256><<<grid, 256, 0, K.stream>>>(F, C, H.P);
  else if (rs == 2)
    k_restrict_fas_staged<MODEL, T, CORR, 16, 256><<<grid, 256, 0, K.stream>>>(F, C, H.P);
  else if (rs == 3)
    k_restrict_fas_staged<MODEL, T, CORR, 16, 512><<<grid, 512, 0, K.stream>>>(F, C, H.P);
  else
    k_restrict_fas_tile<MODEL, T, CORR><<<grid, RTILE * RTILE, 0, K.stream>>>(F, C, H.P);
}

// Whether tile shape ts covers an n x n level exactly.
inline bool tile_shape_fits(int ts, int n) {
  return ts >= 0 && ts < NUM_TILE_SHAPES && n % kTileShapes[ts].tx == 0 && n % kTileShapes[ts].ty == 0;
}

template <int MODEL, typename T, bool CORR, int NSW, bool PRO>
int tile_launch(Hier<T>& H, Cycle& K, const Lvl<T>& L, const Fld<T>& in, const Fld<T>& out, const Lvl<T>& C,
                int res, int ts) {
  if (!tile_shape_fits(ts, L.n)) ts = 0;
  switch (ts) {
    case 1: return tile_launch_shape<MODEL, T, CORR, NSW, PRO, 1>(H, K, L, in, out, C, res);
    case 2: return tile_launch_shape<MODEL, T, CORR, NSW, PRO, 2>(H, K, L, in, out, C, res);
    case 3: return tile_launch_shape<MODEL, T, CORR, NSW, PRO, 3>(H, K, L, in, out, C, res);
    case 4: return tile_launch_shape<MODEL, T, CORR, NSW, PRO, 4>(H, K, L, in, out, C, res);
    case 5: return tile_launch_shape<MODEL, T, CORR, NSW, PRO, 5>(H, K, L, in, out, C, res);
    case 6: return tile_launch_shape<MODEL, T, CORR, NSW, PRO, 6>(H, K, L, in, out, C, res);
    case 7: return tile_launch_shape<MODEL, T, CORR, NSW, PRO, 7>(H, K, L, in, out, C, res);
    case 8: return tile_launch_shape<MODEL, T, CORR, NSW, PRO, 8>(H, K, L, in, out, C, res);
    case 9: return tile_launch_shape<MODEL, T, CORR, NSW, PRO, 9>(H, K, L, in, out, C, res);
    default: return tile_launch_shape<MODEL, T, CORR, NSW, PRO, 0>(H, K, L, in, out, C, res);
  }
}

// `sweeps` tiled sweeps of level l from cur into the other buffer and back
// (two per launch, or one where the level's sweep schedule says so).  The first launch applies the coarse-grid correction from
// level l+1 when pro is set; the last launch also computes the residual
// (res_last: 1 the field d, 2 stop-test partial sums, 3 and 4 the folded
// restriction).  f_in_d: the level's right-hand side is in L.d (left there by
// its RES = 4 pre-sweep launch).  On return cur names the buffer holding the
// iterate.
template <int MODEL, typename T, bool CORR>
int tiled_sweeps(Hier<T>& H, Cycle& K, int l, int sweeps, bool pro, Fld<T>& cur, Fld<T>& other,
                 int res_last = 0, bool f_in_d = false) {
  Lvl<T> L = H.L[l];
  if (f_in_d)
    for (int c = 0; c < 5; ++c) L.f[c] = L.d[c];
  const Lvl<T>& C = H.L[std::min<size_t>(l + 1, H.L.size() - 1)];
  const int ts = l < (int)H.tile_shape.size() ? H.tile_shape[l] : 0;
  const int fuse = l < (int)H.sweep_fuse.size() ? H.sweep_fuse[l] : 2;
  int blocks = 0;
  while (sweeps > 0) {
    const int nsw = (sweeps >= 2 && fuse >= 2) ? 2 : 1;
    const int res = (sweeps == nsw) ? res_last : 0;
    if (nsw == 2) {
      if (pro)
        blocks = tile_launch<MODEL, T, CORR, 2, true>(H, K, L, cur, other, C, res, ts);
      else
        blocks = tile_launch<MODEL, T, CORR, 2, false>(H, K, L, cur, other, C, res, ts);
    } else {
      if (pro)
        blocks = tile_launch<MODEL, T, CORR, 1, true>(H, K, L, cur, other, C, res, ts);
      else
        blocks = tile_launch<MODEL, T, CORR, 1, false>(H, K, L, cur, other, C, res, ts);
    }
    std::swap(cur, other);
    sweeps -= nsw;
    pro = false;
  }
  return blocks;  // workgroups of the last launch
}

template <typename T> void copy_fields(Cycle& K, const Fld<T>& a, const Fld<T>& b, int nc, size_t cnt) {
  for (int c = 0; c < nc; ++c)
    k_copy_t<T><<<(unsigned)((cnt + 255) / 256), 256, 0, K.stream>>>(a.c[c], b.c[c], cnt, K.halt);
}

template <int MODEL, typename T, bool CORR> void vcycle_rec(Hier<T>& H, Cycle& K, int l, bool fc = false);

// Whether level l folds its FAS restriction into its last pre-sweep launch.
template <typename T> bool level_fused(const Hier<T>& H, const Cycle& K, int l) {
  return K.nu1 >= 1 && l < (int)H.fused.size() && H.fused[l];
}

// Whether the V-cycle visits level l with the tail kernel, or with the tiled
// kernels (vcycle_tiled).
template <int MODEL, typename T, bool CORR> bool level_in_tail(const Hier<T>& H, const Cycle& K, int l) {
  return H.L[l].n <= K.tail_n && tail_plan<MODEL, T, CORR>(H.L[l].n, (int)H.L.size() - l, H.tail_lds_max, nullptr);
}
template <int MODEL, typename T, bool CORR> bool level_tiled(const Hier<T>& H, const Cycle& K, int l) {
  return !level_in_tail<MODEL, T, CORR>(H, K, l) && K.use_tiles && l + 1 < (int)H.L.size() &&
         H.L[l].n >= TILE_X && H.L[l + 1].n >= RTILE;
}

// Whether tiled level l (below the finest), given its right-hand side as R d,
// could complete it in its own pre-sweep launch if that launch folded its
// restriction too: one launch of two sweeps (nu1 = 2) in a tile shape whose
// RES = 4 arrays fit the LDS.
template <int MODEL, typename T, bool CORR> bool fold_rhs_capable(const Hier<T>& H, const Cycle& K, int l) {
  if constexpr (walls(MODEL)) return false;
  if (!H.fold_rhs || l < 1 || !level_tiled<MODEL, T, CORR>(H, K, l)) return false;
  const int fuse = l < (int)H.sweep_fuse.size() ? H.sweep_fuse[l] : 2;
  int ts = l < (int)H.tile_shape.size() ? H.tile_shape[l] : 0;
  if (!tile_shape_fits(ts, H.L[l].n)) ts = 0;
  return K.nu1 == 2 && fuse >= 2 && fold_rhs_fits_shape<MODEL, T, CORR>(ts);
}
// ... and whether it gets it as R d: the restriction into it is folded.
template <int MODEL, typename T, bool CORR> bool fold_rhs_possible(const Hier<T>& H, const Cycle& K, int l) {
  return fold_rhs_capable<MODEL, T, CORR>(H, K, l) && level_fused(H, K, l - 1);
}
template <int MODEL, typename T, bool CORR> bool level_fold_rhs(const Hier<T>& H, const Cycle& K, int l) {
  return level_fused(H, K, l) && fold_rhs_possible<MODEL, T, CORR>(H, K, l);
}

// After a folded restriction from level l: f_c = R d + N_c(R g) on level
// l + 1, by the tail kernel as it loads or by the coarse level's own
// pre-sweep launch (returns true: the caller passes fc), or by k_fas_rhs.
template <int MODEL, typename T, bool CORR> bool complete_coarse_rhs(Hier<T>& H, Cycle& K, int l) {
  const int c = l + 1;
  if (level_in_tail<MODEL, T, CORR>(H, K, c) || level_fold_rhs<MODEL, T, CORR>(H, K, c)) return true;
  const Lvl<T>& C = H.L[c];
  const dim3 b = block2(C.n, C.n);
  k_fas_rhs<MODEL, T, CORR><<<grid2(C.n, C.n, b), b, 0, K.stream>>>(C, H.P);
  return false;
}

// One visit to a large level with the tiled kernels: pre-sweeps (the last also
// writes d = f - N(g)), the fused FAS restriction, the coarser levels, the
// prolongation fused into the first post-sweep, post-sweeps.  The iterate
// starts and ends in L.g.  fc: f still holds R d (level_fold_rhs), completed
// by the pre-sweep launch into L.d, where the post-sweeps read it.
template <int MODEL, typename T, bool CORR> void vcycle_tiled(Hier<T>& H, Cycle& K, int l, bool fc_here = false) {
  constexpr int NCm = NC<MODEL>::value;
  const Lvl<T>& L = H.L[l];
  const Lvl<T>& C = H.L[l + 1];
  const Fld<T> home = fld<T>(L.g);
  Fld<T> cur = home, other = fld<T>(L.gb);
  bool fc = false;
  if (level_fused(H, K, l)) {
    // the last pre-sweep launch restricts g and d into the coarse level
    tiled_sweeps<MODEL, T, CORR>(H, K, l, K.nu1, false, cur, other, fc_here ? 4 : 3);
    fc = complete_coarse_rhs<MODEL, T, CORR>(H, K, l);
  } else {
    tiled_sweeps<MODEL, T, CORR>(H, K, l, K.nu1, false, cur, other, 1);
    Lvl<T> F = L;  // descriptor of the buffer holding the iterate
    for (int c = 0; c < 5; ++c) F.g[c] = cur.c[c];
    if (K.nu1 == 0) {
      if constexpr (!CORR && !walls(MODEL)) {
        const dim3 b = block2(F.n, F.n);
        k_residual_field<MODEL, T><<<grid2(F.n, F.n, b), b, 0, K.stream>>>(F, H.P);
      }
    }
    restrict_launch<MODEL, T, CORR>(H, K, F, C, l < (int)H.restrict_shape.size() ? H.restrict_shape[l] : 0);
  }
  vcycle_rec<MODEL, T, CORR>(H, K, l + 1, fc);
  if (K.nu2 > 0) {
    // post-sweeps; on the finest level of the FP64 solve the last one also
    // leaves the partial sums of the stop-test residual
    const bool norm = (l == 0 && !CORR);
    const int blocks = tiled_sweeps<MODEL, T, CORR>(H, K, l, K.nu2, true, cur, other, norm ? 2 : 0, fc_here);
    if (norm) K.norm_partials = blocks;
  } else {
    if constexpr (!CORR && !walls(MODEL)) {
      Lvl<T> F = L;  // descriptor of the buffer holding the iterate
      for (int c = 0; c < 5; ++c) F.g[c] = cur.c[c];
      const dim3 b = block2(F.n, F.n);
      k_prolong<MODEL, T><<<grid2(F.n, F.n, b), b, 0, K.stream>>>(F, C, H.P);
    }
  }
  if (cur.c[0] != home.c[0]) copy_fields<T>(K, cur, home, NCm, (size_t)L.n * L.ny);
}

template <int MODEL, typename T, bool CORR> void vcycle_rec(Hier<T>& H, Cycle& K, int l, bool fc) {
  const int nlev = (int)H.L.size(), last = nlev - 1;
  if (level_in_tail<MODEL, T, CORR>(H, K, l)) {
    tail_launch<MODEL, T, CORR>(H, K, l, fc);
    return;
  }
  if (level_tiled<MODEL, T, CORR>(H, K, l)) {
    vcycle_tiled<MODEL, T, CORR>(H, K, l, fc);
    return;
  }
  // (a channel always runs the tiled kernels and the tail: its hierarchy is
  // built so, and the plain per-level path below is periodic)
  if constexpr (!CORR && !walls(MODEL)) {
    if (l == last) {
      smooth_level<MODEL, T>(H, K, l, K.coarse_sweeps);
      return;
    }
    smooth_level<MODEL, T>(H, K, l, K.nu1);
    const Lvl<T>& F = H.L[l];
    const Lvl<T>& C = H.L[l + 1];
    const dim3 bc = block2(C.n, C.n), bf = block2(F.n, F.n);
    k_residual_field<MODEL, T><<<grid2(F.n, F.n, bf), bf, 0, K.stream>>>(F, H.P);
    k_restrict_gd<MODEL, T><<<grid2(C.n, C.n, bc), bc, 0, K.stream>>>(F, C, K.halt);
    k_fas_rhs<MODEL, T><<<grid2(C.n, C.n, bc), bc, 0, K.stream>>>(C, H.P);
    vcycle_rec<MODEL, T, CORR>(H, K, l + 1);
    k_prolong<MODEL, T><<<grid2(F.n, F.n, bf), bf, 0, K.stream>>>(F, C, H.P);
    smooth_level<MODEL, T>(H, K, l, K.nu2);
  }
}

// One V-cycle from the finest level.
template <int MODEL, typename T, bool CORR> void vcycle(Hier<T>& H, Cycle& K) {
  K.norm_partials = 0;
  vcycle_rec<MODEL, T, CORR>(H, K, 0);
}

}  // namespace hfz
