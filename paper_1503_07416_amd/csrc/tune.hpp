// Tuner of the tiled sweep kernel's tile shape and the restriction variant.
//
// The best tile shape depends on the level size: small levels have too few
// workgroups to fill the device and want small, quick tiles; large levels want
// wide tiles (less recomputed halo per owned node) and more threads per
// workgroup.  For every level the V-cycle sweeps with the tiled kernel, the
// tuner times the level's pre-smoothing launch (two sweeps and the residual
// field) and post-smoothing launch (the prolongation and two sweeps) in every
// tile shape that covers the level, with HIP events on the handle's stream,
// and keeps the fastest pair (the two can favour different shapes: with the
// CDFT potential the prolongation launch is slower in 1024-thread tiles).  The kernels' speed does not depend
// on the values they sweep, so the tuner runs on the workspace as it is; it
// writes only the second iterate buffer and the residual scratch of the level.
// The restriction variants (restrict.hpp) are timed the same way per level,
// and so is the sweep schedule: two sweeps fused per launch or one per launch.
// Whether each level folds its restriction into its pre-sweep launch is then
// chosen for all levels together (tune_fold_chain), since a folded
// restriction leaves the next level's right-hand side to complete.
// Choices are cached per (model, arithmetic type, form, level size) for the
// life of the process.  HFZ_TILE=<shape> forces one shape where it fits,
// HFZ_RESTRICT=<variant> one restriction variant, HFZ_SWEEPS=1 one sweep per
// launch (2: fused), HFZ_TUNE=0 keeps shape 0, variant 0 and fused sweeps.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "driver.hpp"

namespace hfz {

inline std::mutex& tune_mutex() {
  static std::mutex m;
  return m;
}
inline std::map<std::tuple<int, int, int, int>, std::tuple<int, int, int, int>>& tune_cache() {
  static std::map<std::tuple<int, int, int, int>, std::tuple<int, int, int, int>> c;
  return c;
}

// HFZ_TUNE_CACHE=<file>: the choices are read from the file when it exists
// (one line per level size: model, bytes per value, form, n, shape, variant,
// sweeps per launch, restriction folded) and written to it after timing, so
// that another process (a profiled run, whose timings the profiler distorts)
// takes the same kernels.  Call with tune_mutex held.
inline void tune_cache_load() {
  static bool loaded = false;
  if (loaded) return;
  loaded = true;
  const char* path = std::getenv("HFZ_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  int k[8];
  while (std::fscanf(f, "%d %d %d %d %d %d %d %d", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &k[6], &k[7]) == 8)
    tune_cache()[std::make_tuple(k[0], k[1], k[2], k[3])] = std::make_tuple(k[4], k[5], k[6], k[7]);
  std::fclose(f);
}

inline void tune_cache_save() {
  const char* path = std::getenv("HFZ_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  for (const auto& kv : tune_cache())
    std::fprintf(f, "%d %d %d %d %d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                 std::get<3>(kv.first), std::get<0>(kv.second), std::get<1>(kv.second), std::get<2>(kv.second),
                 std::get<3>(kv.second));
  std::fclose(f);
}

// Average time (ms) of `reps` pairs of a pre-smoothing launch (two sweeps and
// the residual field) and a post-smoothing launch (the prolongation from
// level l + 1, two sweeps, on the finest level of the FP64 solve the
// stop-test partial sums) of shape ts on level l, after one untimed pair;
// negative on a HIP error.  The pre-sweep writes the second iterate buffer,
// the post-sweep reads it and writes the first: the tuner runs before any
// state is set.
template <int MODEL, typename T, bool CORR>
float time_shape(Hier<T>& H, Cycle& K, int l, int ts, int reps) {
  const Lvl<T>& L = H.L[l];
  const Lvl<T>& C = H.L[l + 1];
  const Fld<T> a = fld<T>(L.g), b = fld<T>(L.gb);
  const int res_post = (l == 0 && !CORR) ? 2 : 0;
  auto pass = [&]() {
    tile_launch<MODEL, T, CORR, 2, false>(H, K, L, a, b, C, 1, ts);
    tile_launch<MODEL, T, CORR, 2, true>(H, K, L, b, a, C, res_post, ts);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = -1.0f;
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    pass();
    bool ok = hipEventRecord(e0, K.stream) == hipSuccess;
    for (int r = 0; r < reps && ok; ++r) pass();
    ok = ok && hipEventRecord(e1, K.stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipGetLastError() == hipSuccess;
    if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
      ms /= (float)reps;
    else
      ms = -1.0f;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipGetLastError();
  return ms;
}

// Average time (ms) of `reps` restriction launches of variant rs from level
// l to l + 1, after one untimed launch; negative on a HIP error.
template <int MODEL, typename T, bool CORR>
float time_restrict(Hier<T>& H, Cycle& K, int l, int rs, int reps) {
  const Lvl<T>& F = H.L[l];
  const Lvl<T>& C = H.L[l + 1];
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = -1.0f;
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    restrict_launch<MODEL, T, CORR>(H, K, F, C, rs);
    bool ok = hipEventRecord(e0, K.stream) == hipSuccess;
    for (int r = 0; r < reps && ok; ++r) restrict_launch<MODEL, T, CORR>(H, K, F, C, rs);
    ok = ok && hipEventRecord(e1, K.stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipGetLastError() == hipSuccess;
    if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
      ms /= (float)reps;
    else
      ms = -1.0f;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipGetLastError();
  return ms;
}

// Average time (ms) of `reps` pre-smoothing passes (two sweeps and the
// residual field) on level l with `fuse` sweeps per launch.
template <int MODEL, typename T, bool CORR>
float time_schedule(Hier<T>& H, Cycle& K, int l, int fuse, int reps) {
  const int keep = H.sweep_fuse[l];
  H.sweep_fuse[l] = fuse;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = -1.0f;
  auto pass = [&]() {
    Fld<T> cur = fld<T>(H.L[l].g), other = fld<T>(H.L[l].gb);
    tiled_sweeps<MODEL, T, CORR>(H, K, l, 2, false, cur, other, 1);
  };
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    pass();
    bool ok = hipEventRecord(e0, K.stream) == hipSuccess;
    for (int r = 0; r < reps && ok; ++r) pass();
    ok = ok && hipEventRecord(e1, K.stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipGetLastError() == hipSuccess;
    if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
      ms /= (float)reps;
    else
      ms = -1.0f;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipGetLastError();
  H.sweep_fuse[l] = keep;
  return ms;
}

// Average time (ms) of `reps` launches of what level l's pre-smoothing and
// restriction can cost (two sweeps per launch), after one untimed launch:
// what 0 the pre-sweep launch with the restriction folded in (RES = 3),
// 1 the same after completing the level's own right-hand side (RES = 4),
// 2 the pre-sweep launch with the residual field and the restriction launch
// of variant rs, 3 k_fas_rhs completing level l's right-hand side.  Negative
// on a HIP error.
template <int MODEL, typename T, bool CORR>
float time_restriction_part(Hier<T>& H, Cycle& K, int l, int what, int rs, int reps) {
  const Lvl<T>& L = H.L[l];
  const Lvl<T>& C = H.L[l + 1];
  const Fld<T> a = fld<T>(L.g), b = fld<T>(L.gb);
  const int ts = H.tile_shape[l];
  auto pass = [&]() {
    if (what == 0 || what == 1) {
      tile_launch<MODEL, T, CORR, 2, false>(H, K, L, a, b, C, what == 0 ? 3 : 4, ts);
    } else if (what == 2) {
      tile_launch<MODEL, T, CORR, 2, false>(H, K, L, a, b, C, 1, ts);
      Lvl<T> F = L;
      for (int c = 0; c < 5; ++c) F.g[c] = b.c[c];
      restrict_launch<MODEL, T, CORR>(H, K, F, C, rs);
    } else {
      const dim3 bl = block2(L.n, L.n);
      k_fas_rhs<MODEL, T, CORR><<<grid2(L.n, L.n, bl), bl, 0, K.stream>>>(L, H.P);
    }
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = -1.0f;
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    pass();
    bool ok = hipEventRecord(e0, K.stream) == hipSuccess;
    for (int r = 0; r < reps && ok; ++r) pass();
    ok = ok && hipEventRecord(e1, K.stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipGetLastError() == hipSuccess;
    if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
      ms /= (float)reps;
    else
      ms = -1.0f;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipGetLastError();
  return ms;
}

// Best of three rounds of time_restriction_part (a large value if it fails).
template <int MODEL, typename T, bool CORR>
float restriction_cost(Hier<T>& H, Cycle& K, int l, int what) {
  float best = -1.0f;
  for (int round = 0; round < 3; ++round) {
    const float t = time_restriction_part<MODEL, T, CORR>(H, K, l, what, H.restrict_shape[l], 8);
    if (t > 0.0f && (best < 0.0f || t < best)) best = t;
  }
  return best > 0.0f ? best : 1e9f;
}

// The restriction of every tiled level folded or not, chosen jointly: level
// l's cost depends on its own choice and on whether the level above folded
// (then l's right-hand side arrives as R d, completed by l's RES = 4 launch
// if l folds and can, else by k_fas_rhs), so the cheapest assignment is a
// shortest path over the levels with two states.  Levels whose choice is
// fixed (fixed[l]) keep H.fused[l].
template <int MODEL, typename T, bool CORR>
void tune_fold_chain(Hier<T>& H, Cycle& K, const std::vector<char>& fixed, int verbose) {
  int nt = 0;
  while (nt + 1 < (int)H.L.size() && level_tiled<MODEL, T, CORR>(H, K, nt)) ++nt;
  if (nt == 0) return;
  // cost[l][s][p]: level l folds (s = 1) or not, the level above folded (p = 1) or not
  std::vector<float> c3(nt), c4(nt, 1e9f), csep(nt), crhs(nt, 0.0f);
  std::vector<char> cap(nt, 0);
  for (int l = 0; l < nt; ++l) {
    c3[l] = restriction_cost<MODEL, T, CORR>(H, K, l, 0);
    csep[l] = restriction_cost<MODEL, T, CORR>(H, K, l, 2);
    if (l > 0) crhs[l] = restriction_cost<MODEL, T, CORR>(H, K, l, 3);
    cap[l] = (char)fold_rhs_capable<MODEL, T, CORR>(H, K, l);
    if (cap[l]) c4[l] = restriction_cost<MODEL, T, CORR>(H, K, l, 1);
  }
  auto cost = [&](int l, int s, int p) -> float {
    if (s == 1) return p ? (cap[l] ? c4[l] : crhs[l] + c3[l]) : c3[l];
    return (p ? crhs[l] : 0.0f) + csep[l];
  };
  std::vector<float> best(2 * nt);
  std::vector<int> from(2 * nt, 0);
  for (int l = 0; l < nt; ++l)
    for (int s = 0; s < 2; ++s) {
      float b = 1e30f;
      if (!(fixed[l] && H.fused[l] != s)) {
        if (l == 0) {
          b = cost(0, s, 0);
        } else {
          for (int p = 0; p < 2; ++p) {
            const float v = best[2 * (l - 1) + p] + cost(l, s, p);
            if (v < b) {
              b = v;
              from[2 * l + s] = p;
            }
          }
        }
      }
      best[2 * l + s] = b;
    }
  int s = best[2 * (nt - 1) + 1] < best[2 * (nt - 1)] ? 1 : 0;
  for (int l = nt - 1; l >= 0; --l) {
    H.fused[l] = (char)s;
    s = from[2 * l + s];
  }
  if (verbose) {
    std::fprintf(stderr, "hfz tune restriction folded (us: RES3 / RES4 / separate / rhs):");
    for (int l = 0; l < nt; ++l)
      std::fprintf(stderr, " n=%d %.2f/%.2f/%.2f/%.2f->%d", H.L[l].n, c3[l] * 1e3f, cap[l] ? c4[l] * 1e3f : -1.0f,
                   csep[l] * 1e3f, crhs[l] * 1e3f, (int)H.fused[l]);
    std::fprintf(stderr, "\n");
  }
}

// Index of the fastest of `count` candidates timed by `time(k)` (best of
// three rounds; a later candidate must win by 2%, so near-ties resolve the
// same way every run); 0 if none could be timed.
template <typename F> int pick_fastest(int count, F&& time, const char* what = nullptr, int n = 0) {
  std::vector<float> ms((size_t)count, -1.0f);
  for (int round = 0; round < 3; ++round)
    for (int k = 0; k < count; ++k) {
      const float t = time(k);
      if (t > 0.0f && (ms[k] < 0.0f || t < ms[k])) ms[k] = t;
    }
  int best = 0;
  for (int k = 1; k < count; ++k)
    if (ms[k] > 0.0f && (ms[best] < 0.0f || ms[k] < 0.98f * ms[best])) best = k;
  if (what && std::getenv("HFZ_VERBOSE")) {
    std::fprintf(stderr, "hfz tune %s n=%d:", what, n);
    for (int k = 0; k < count; ++k) std::fprintf(stderr, " %.2f", ms[k] * 1e3f);
    std::fprintf(stderr, " us -> %d\n", best);
  }
  return best;
}

// Fills H.tile_shape, H.restrict_shape, H.sweep_fuse and H.fused for the
// levels the tiled V-cycle visits (size >= 32 with a coarser level of >= 16,
// above the tail).  HFZ_RESTRICT=<variant> forces a restriction variant where
// it fits; HFZ_FUSE=0 / 1 keeps the restriction launches separate / folds
// them into the sweeps wherever it can (default: the cheapest assignment over
// all levels, tune_fold_chain).
// HFZ_FOLD_RHS=0 leaves the completion of a folded level's coarse right-hand
// side to k_fas_rhs everywhere (default: the coarse level's RES = 4 launch
// where level_fold_rhs allows it).
// With time_them false nothing is launched: a level takes the choices cached
// for its size in this process, else shape 0, variant 0, fused sweeps and a
// separate restriction.
template <int MODEL, typename T, bool CORR> void tune_tile_shapes(Hier<T>& H, Cycle K, bool time_them = true) {
  const int nlev = (int)H.L.size();
  H.tile_shape.assign(nlev, 0);
  H.restrict_shape.assign(nlev, 0);
  H.sweep_fuse.assign(nlev, 2);
  H.fused.assign(nlev, 0);
  H.fold_rhs = true;
  if (const char* e = std::getenv("HFZ_FOLD_RHS")) H.fold_rhs = std::atoi(e) != 0;
  int forced_r = -1, forced_f = -1, forced_x = -1;
  if (const char* e = std::getenv("HFZ_FUSE")) forced_x = std::atoi(e) != 0 ? 1 : 0;
  if constexpr (walls(MODEL)) forced_x = 0;  // the channel's wall rows: the direct restriction kernel
  if (const char* e = std::getenv("HFZ_RESTRICT")) forced_r = std::atoi(e);
  if (const char* e = std::getenv("HFZ_SWEEPS")) forced_f = std::atoi(e) == 1 ? 1 : 2;
  int forced = -1;
  if (const char* e = std::getenv("HFZ_TILE")) forced = std::atoi(e);
  bool tune = true;
  if (const char* e = std::getenv("HFZ_TUNE")) tune = std::atoi(e) != 0;
  std::vector<char> pending(nlev, 0);  // levels whose fold choice is timed (tune_fold_chain)
  for (int l = 0; l + 1 < nlev; ++l) {
    const int n = H.L[l].n, nc = H.L[l + 1].n;
    if (n < TILE_X || nc < RTILE || H.L[l].gb[0] == nullptr) continue;
    if (forced >= 0) H.tile_shape[l] = tile_shape_fits(forced, n) ? forced : 0;
    if (forced_r >= 0)
      H.restrict_shape[l] = (forced_r < NUM_RESTRICT_SHAPES && nc % kRestrictTile[forced_r] == 0) ? forced_r : 0;
    if (forced_f > 0) H.sweep_fuse[l] = forced_f;
    if (forced_x >= 0) H.fused[l] = (char)forced_x;
    if (!tune || n <= K.tail_n || (forced >= 0 && forced_r >= 0 && forced_f > 0 && forced_x >= 0)) continue;
    const auto key = std::make_tuple(MODEL, (int)sizeof(T), (int)CORR, n);
    {
      std::lock_guard<std::mutex> g(tune_mutex());
      tune_cache_load();
      auto it = tune_cache().find(key);
      if (it != tune_cache().end()) {
        if (forced < 0) H.tile_shape[l] = std::get<0>(it->second);
        if (forced_r < 0) H.restrict_shape[l] = std::get<1>(it->second);
        if (forced_f < 0) H.sweep_fuse[l] = std::get<2>(it->second);
        if (forced_x < 0) H.fused[l] = (char)std::get<3>(it->second);
        continue;
      }
    }
    if (!time_them) continue;
    const int ts = pick_fastest(NUM_TILE_SHAPES, [&](int k) {
      return tile_shape_fits(k, n) ? time_shape<MODEL, T, CORR>(H, K, l, k, 8) : -1.0f;
    }, "tile shape", n);
    if (forced < 0) H.tile_shape[l] = ts;
    const int rs = pick_fastest(NUM_RESTRICT_SHAPES, [&](int k) {
      return nc % kRestrictTile[k] == 0 ? time_restrict<MODEL, T, CORR>(H, K, l, k, 8) : -1.0f;
    }, "restriction", n);
    if (forced_r < 0) H.restrict_shape[l] = rs;
    // sweep schedule in the chosen shape: candidate 0 fuses two sweeps per
    // launch, candidate 1 launches one sweep at a time
    const int fs = pick_fastest(
        2, [&](int k) { return time_schedule<MODEL, T, CORR>(H, K, l, k == 0 ? 2 : 1, 8); }, "sweeps", n);
    if (forced_f < 0) H.sweep_fuse[l] = fs == 0 ? 2 : 1;
    // the restriction folded or not: decided for all timed levels together
    // below (never folded for the channel)
    if (forced_x < 0) pending[l] = 1;
  }
  bool any = false;
  for (int l = 0; l < nlev; ++l) any = any || pending[l];
  if (any) {
    if constexpr (!walls(MODEL)) {
      std::vector<char> fixed(nlev);
      for (int l = 0; l < nlev; ++l) fixed[l] = !pending[l];
      tune_fold_chain<MODEL, T, CORR>(H, K, fixed, std::getenv("HFZ_VERBOSE") != nullptr);
    }
    std::lock_guard<std::mutex> g(tune_mutex());
    for (int l = 0; l < nlev; ++l) {
      if (!pending[l]) continue;
      tune_cache()[std::make_tuple(MODEL, (int)sizeof(T), (int)CORR, H.L[l].n)] =
          std::make_tuple(H.tile_shape[l], H.restrict_shape[l], H.sweep_fuse[l], (int)H.fused[l]);
    }
    tune_cache_save();
  }
}

}  // namespace hfz
