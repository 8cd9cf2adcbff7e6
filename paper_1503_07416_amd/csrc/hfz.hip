// Host side of the hfz library: parameter checks, workspace layout, the FAS
// driver (V-cycles, stop test, step roll-back), the CDFT convolution set-up,
// diagnostics and the C ABI declared in include/hfz.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "hfz.h"
#include "fft.hpp"
#include "kernels.hpp"
#include "batchk.hpp"
#include "driver.hpp"
#include "tune.hpp"

using namespace hfz;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kTailLdsMax = 160 * 1024;
constexpr int kTailNMax = 32;  // largest level the one-workgroup tail kernel takes

inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

// The kernels' model: the ABI model, or WPFC for the PFC step in a channel.
int kernel_model(const hfz_params& p) { return p.walls ? WPFC : p.model; }

// Calls f with the kernels' model (kernel_model) as a compile-time constant
// (std::integral_constant).
template <class F> auto by_model(int km, F&& f) {
  switch (km) {
    case PFC:
      return f(std::integral_constant<int, PFC>());
    case CDFT:
      return f(std::integral_constant<int, CDFT>());
    case GPFC:
      return f(std::integral_constant<int, GPFC>());
    case WPFC:
      return f(std::integral_constant<int, WPFC>());
    default:
      return f(std::integral_constant<int, GCDFT>());
  }
}

bool model_cdft(int model) { return model == HFZ_CDFT || model == HFZ_CDFT_GF; }
bool model_gf(int model) { return model == HFZ_PFC_GF || model == HFZ_CDFT_GF; }
int model_nc(int model) {
  return model == HFZ_PFC ? 5 : (model == HFZ_CDFT ? 3 : (model == HFZ_PFC_GF ? 3 : 2));
}

int validate(const hfz_params* p) {
  if (!p) return HFZ_EINVAL;
  if (p->model < HFZ_PFC || p->model > HFZ_CDFT_GF) return HFZ_EINVAL;
  if (!is_pow2(p->n) || p->n < 8 || p->n > 8192) return HFZ_EINVAL;
  if (model_cdft(p->model) && p->n > 2048) return HFZ_EINVAL;  // LDS row FFT: 2 x 2048 complex doubles
  if (!(p->h > 0) || !(p->s > 0) || !(p->gamma > 0)) return HFZ_EINVAL;
  if (!(p->w_damp >= 0.0) || !(p->w_damp < 1.0)) return HFZ_EINVAL;
  if (!(p->tol > 0)) return HFZ_EINVAL;
  if (p->nu1 < 0 || p->nu2 < 0 || p->nu1 + p->nu2 < 1) return HFZ_EINVAL;
  if (p->max_cycles < 1 || p->coarse_sweeps < 1) return HFZ_EINVAL;
  if (!is_pow2(p->coarsest_n) || p->coarsest_n < 4 || p->coarsest_n > p->n) return HFZ_EINVAL;
  if (p->sigma != 1 && p->sigma != -1) return HFZ_EINVAL;
  if (p->precision != HFZ_FP64 && p->precision != HFZ_MIXED) return HFZ_EINVAL;
  if (model_cdft(p->model) && (!(p->nu > 0) || !(p->delta >= 0))) return HFZ_EINVAL;
  if (!model_cdft(p->model) && !std::isfinite(p->alpha)) return HFZ_EINVAL;
  if (p->walls != 0 && p->walls != 1) return HFZ_EINVAL;
  if (p->walls && (p->model != HFZ_PFC || p->precision != HFZ_FP64 || p->nu1 < 1 || p->nu2 < 1 ||
                   !std::isfinite(p->u_wall_bottom) || !std::isfinite(p->u_wall_top)))
    return HFZ_EINVAL;
  // The FP32 correction-form inner solve and the channel run only on the
  // tiled kernels, whose pre-sweep launch leaves the residual field and whose
  // first post-sweep launch applies the coarse-grid correction, and on the
  // one-workgroup tail, which must hold the coarsest level.
  if ((p->precision == HFZ_MIXED || p->walls) && (p->nu1 < 1 || p->nu2 < 1 || p->coarsest_n > kTailNMax))
    return HFZ_EINVAL;
  return HFZ_OK;
}

// Workspace carving: a bump allocator over the caller's buffer.  Run once
// with base == nullptr to size the workspace.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T> T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

struct Dims {
  dim3 grid, block;
};

Dims dims2(int nx, int ny) {
  const int bx = std::min(64, nx);
  const int by = std::max(1, std::min(256 / bx, ny));
  return {dim3((nx + bx - 1) / bx, (ny + by - 1) / by), dim3(bx, by)};
}

}  // namespace

constexpr int kGraphSizes = 4;  // graphs of 1, 2, 4, 8 V-cycles

struct hfz_handle {
  hfz_params p{};
  int km = 0;  // the kernels' model (kernel_model)
  hipStream_t stream = nullptr;
  int nlev = 0;
  int nc = 0;
  double ce = 0.0;
  bool has_state = false;
  Hier<double> H;   // FP64 hierarchy (H.L[0].rk is the state rho^k)
  Hier<float> H32;  // FP32 correction hierarchy of the mixed-precision step
  double* u = nullptr;
  double* v = nullptr;
  double* mu = nullptr;
  double* ka = nullptr;
  // CDFT
  double* jrho = nullptr;
  double* mult = nullptr;
  double2* fa = nullptr;
  double2* fb = nullptr;
  // reductions
  double* partial = nullptr;
  double* result = nullptr;
  int* ctl = nullptr;  // device stop flag and cycle counter of the V-cycle loop (inside result)
  StateB* state1 = nullptr;      // device copies of the state pointers, the physics and an "on" flag, so
  Phys<double>* phys1 = nullptr;  // that the batched begin / end kernels serve this handle (count 1)
  int* on1 = nullptr;
  int cycle_hint = 4;  // V-cycles (mixed: outer iterations) the previous step needed
  size_t partial_cap = 0;
  int tail_n = 32;  // levels of this size and below run in the one-workgroup tail kernel
  bool use_graph = true;
  int mp_inner = 3;  // FP32 V-cycles per outer defect-correction iteration
  bool use_tiles = true;  // LDS-tiled kernels on levels >= 32
  int norm_partials = 0;  // > 0: the last V-cycle's post-sweep left this many residual partials
  // HIP graphs of 1, 2, 4 and 8 V-cycles (each with its stop test): state 0
  // not built, 1 built, -1 unavailable
  int graph_state[kGraphSizes] = {};
  hipGraphExec_t cycle_exec[kGraphSizes] = {};
  int mp_graph_state[kGraphSizes] = {};  // the same for the mixed-precision outer iteration
  hipGraphExec_t mp_exec[kGraphSizes] = {};
};

namespace {

// Lays out every buffer of the handle; with ws == nullptr only sizes.
size_t layout(const hfz_params& p, void* ws, hfz_handle* hd) {
  Carver c{static_cast<char*>(ws)};
  const int nc = model_nc(p.model);
  const int n = p.n;
  const int wr = p.walls ? 1 : 0;  // a channel's levels hold the wall rows too
  const size_t N2 = (size_t)n * (n + wr);
  std::vector<Lvl<double>> L;
  for (int m = n; m >= p.coarsest_n; m >>= 1) {
    Lvl<double> l{};
    l.n = m;
    l.ny = m + wr;
    l.lg = ilog2(m);
    const size_t cnt = (size_t)m * (m + wr);
    for (int k = 0; k < nc; ++k) l.g[k] = c.take<double>(cnt);
    for (int k = 0; k < nc; ++k) l.f[k] = c.take<double>(cnt);
    if (m != n)
      for (int k = 0; k < nc; ++k) l.g0[k] = c.take<double>(cnt);
    // d: the residual scratch, and on coarse levels the restricted residual R d
    // the fused restriction leaves there (the coarsest level's too)
    if (m > p.coarsest_n || m != n)
      for (int k = 0; k < nc; ++k) l.d[k] = c.take<double>(cnt);
    if (m >= TILE_X && m > p.coarsest_n)
      for (int k = 0; k < nc; ++k) l.gb[k] = c.take<double>(cnt);
    l.rk = c.take<double>(cnt);
    l.om = c.take<double>(cnt);
    L.push_back(l);
  }
  double* u = c.take<double>(N2);
  double* v = c.take<double>(N2);
  double *mu = nullptr, *ka = nullptr;
  if (p.model != HFZ_CDFT) mu = c.take<double>(N2);  // the auxiliaries (PFC: mu, kappa; CDFT gradient flow: mu)
  if (p.model == HFZ_PFC || p.model == HFZ_PFC_GF) ka = c.take<double>(N2);
  double *jrho = nullptr, *mult = nullptr;
  double2 *fa = nullptr, *fb = nullptr;
  if (model_cdft(p.model)) {
    jrho = c.take<double>(N2);
    mult = c.take<double>(N2);
    fa = c.take<double2>(N2);
    fb = c.take<double2>(N2);
  }
  const size_t pcap = std::max<size_t>(4096, N2 / 64 + 64);
  double* partial = c.take<double>(pcap * 4);
  double* result = c.take<double>(64);
  Lvl<double>* desc = c.take<Lvl<double>>(L.size());
  StateB* state1 = c.take<StateB>(1);
  Phys<double>* phys1 = c.take<Phys<double>>(1);
  int* on1 = c.take<int>(64);
  if (hd) {
    hd->nc = nc;
    hd->nlev = (int)L.size();
    double h = p.h;
    for (auto& l : L) {
      l.h = h;
      l.k.c4 = p.s / (4.0 * h);
      l.k.c2 = p.s / (2.0 * h);
      l.k.ih2 = 1.0 / (h * h);
      h *= 2.0;
    }
    hd->H.L = L;
    hd->u = u;
    hd->v = v;
    hd->mu = mu;
    hd->ka = ka;
    hd->jrho = jrho;
    hd->mult = mult;
    hd->fa = fa;
    hd->fb = fb;
    hd->partial = partial;
    hd->result = result;
    hd->ctl = reinterpret_cast<int*>(result + 8);
    hd->partial_cap = pcap;
    hd->H.desc = desc;
    hd->state1 = state1;
    hd->phys1 = phys1;
    hd->on1 = on1;
  }
  if (p.precision == HFZ_MIXED) {
    // FP32 correction hierarchy: e (the iterate), f, R e, d, the second sweep
    // buffer, FP32 copies of rho^k and omega^k, and the base state (rho, u, v)
    std::vector<Lvl<float>> E;
    for (int m = n; m >= p.coarsest_n; m >>= 1) {
      Lvl<float> l{};
      l.n = m;
      l.ny = m + wr;
      l.lg = ilog2(m);
      const size_t cnt = (size_t)m * (m + wr);
      for (int k = 0; k < nc; ++k) l.g[k] = c.take<float>(cnt);
      for (int k = 0; k < nc; ++k) l.f[k] = c.take<float>(cnt);
      for (int k = 0; k < nc; ++k) l.g0[k] = c.take<float>(cnt);
      if (m > p.coarsest_n || m != n)
        for (int k = 0; k < nc; ++k) l.d[k] = c.take<float>(cnt);
      if (m >= TILE_X && m > p.coarsest_n)
        for (int k = 0; k < nc; ++k) l.gb[k] = c.take<float>(cnt);
      l.rk = c.take<float>(cnt);
      l.om = c.take<float>(cnt);
      for (int k = 0; k < 3; ++k) l.bg[k] = c.take<float>(cnt);
      E.push_back(l);
    }
    Lvl<float>* desc32 = c.take<Lvl<float>>(E.size());
    if (hd) {
      double h = p.h;
      for (auto& l : E) {
        l.h = (float)h;
        l.k.c4 = (float)(p.s / (4.0 * h));
        l.k.c2 = (float)(p.s / (2.0 * h));
        l.k.ih2 = (float)(1.0 / (h * h));
        h *= 2.0;
      }
      hd->H32.L = E;
      hd->H32.desc = desc32;
    }
  }
  return c.off;
}

#define HIPCHK(x)                         \
  do {                                    \
    if ((x) != hipSuccess) return HFZ_EHIP; \
  } while (0)

int last_error() { return hipGetLastError() == hipSuccess ? HFZ_OK : HFZ_EHIP; }

// Raises a kernel's dynamic LDS limit to what a gfx950 CU offers (minus the
// kernel's static LDS); returns the limit in force.
size_t lds_optin(const void* kernel) {
  int dev = 0, optin = 0;
  hipFuncAttributes fa{};
  size_t static_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess)
    optin = 0;
  if (hipFuncGetAttributes(&fa, kernel) == hipSuccess) static_lds = fa.sharedSizeBytes;
  const size_t want = std::min<size_t>(kTailLdsMax, optin > 0 ? (size_t)optin : 65536) - static_lds - 256;
  size_t got = 0;
  for (size_t lim : {want, (size_t)65536 - static_lds - 256}) {
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) == hipSuccess) {
      got = lim;
      break;
    }
  }
  (void)hipGetLastError();
  return got;
}

// Whether the one-workgroup tail holds every level from the first one of
// size <= tail_n down to the coarsest: the tiled V-cycle path has no
// coarsest-level smoother, so the correction form, the channel and the batch
// need the coarsest level in the tail.
template <int MODEL, typename T, bool CORR> bool tail_holds_bottom(const std::vector<Lvl<T>>& L, int tail_n,
                                                                   size_t lds_max) {
  const int nlev = (int)L.size();
  for (int l = 0; l < nlev; ++l)
    if (L[l].n <= tail_n) return tail_plan<MODEL, T, CORR>(L[l].n, nlev - l, lds_max, nullptr);
  return false;
}

// ---- V-cycle entry points (driver.hpp) -------------------------------------

Cycle cycle_ctx(hfz_handle* hd) {
  Cycle K;
  K.stream = hd->stream;
  K.nu1 = hd->p.nu1;
  K.nu2 = hd->p.nu2;
  K.coarse_sweeps = hd->p.coarse_sweeps;
  K.tail_n = hd->tail_n;
  K.use_tiles = hd->use_tiles;
  K.partial = hd->partial;
  K.halt = hd->ctl;
  return K;
}

// Enqueues h^2 sum (f - N(g))^2 on level 0 into result[0].
// The final reduction of `count` stop-test partials into result[0]; with
// `stop`, the device stop test of the V-cycle loop as well (k_reduce_stop).
void reduce_launch(hfz_handle* hd, int count, bool stop, bool counted = true) {
  const double h2 = hd->H.L[0].h * hd->H.L[0].h;
  if (stop)
    k_reduce_stop<<<1, 1024, 0, hd->stream>>>(hd->partial, count, h2, hd->p.tol, hd->result, hd->ctl,
                                              counted ? 1 : 0);
  else
    k_reduce_final<<<1, 1024, 0, hd->stream>>>(hd->partial, count, 1, h2, hd->result);
}

template <int MODEL> void residual_launch_t(hfz_handle* hd, bool stop, bool counted) {
  const Lvl<double>& L = hd->H.L[0];
  const Dims d = dims2(L.n, L.ny);
  k_residual_partial<MODEL, double><<<d.grid, d.block, 0, hd->stream>>>(L, hd->H.P, hd->partial);
  reduce_launch(hd, (int)(d.grid.x * d.grid.y), stop, counted);
}

void residual_launch(hfz_handle* hd, bool stop = false, bool counted = true) {
  by_model(hd->km, [&](auto m) { residual_launch_t<decltype(m)::value>(hd, stop, counted); });
}

int residual_read(hfz_handle* hd, double* norm) {
  double r2 = 0.0;
  HIPCHK(hipMemcpyAsync(&r2, hd->result, sizeof(double), hipMemcpyDeviceToHost, hd->stream));
  HIPCHK(hipStreamSynchronize(hd->stream));
  *norm = std::sqrt(r2);
  return last_error();
}

int residual(hfz_handle* hd, double* norm) {
  residual_launch(hd);
  return residual_read(hd, norm);
}

void vcycle(hfz_handle* hd) {
  Cycle K = cycle_ctx(hd);
  by_model(hd->km, [&](auto m) { hfz::vcycle<decltype(m)::value, double, false>(hd->H, K); });
  hd->norm_partials = K.norm_partials;
}

// A V-cycle and the stop-test residual norm after it (the last post-sweep
// may already have left the partial sums).
void vcycle_and_norm(hfz_handle* hd, bool stop) {
  vcycle(hd);
  if (hd->norm_partials > 0)
    reduce_launch(hd, hd->norm_partials, stop);
  else
    residual_launch(hd, stop);
}

// 2^k V-cycles, each followed by the residual norm and the device stop test,
// captured once into a HIP graph (on a private stream: capture records, it
// does not execute) and replayed on the caller's stream.  A batch of cycles
// is launched as graphs of 8, 4, 2 and 1 cycles: the device idles for some
// microseconds between two graph launches, against under one between two
// kernels of a graph.  `body` enqueues one cycle.  Returns false when graphs
// are unavailable; callers then launch the kernels one by one and test on the
// host.
template <typename F>
bool capture_graph(hfz_handle* hd, int* state, hipGraphExec_t* exec, int k, F&& body) {
  if (state[k] == 1) return true;
  if (state[k] < 0) return false;
  hipStream_t cap = nullptr;
  hipGraph_t g = nullptr;
  bool ok = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess;
  if (ok) {
    hipStream_t user = hd->stream;
    hd->stream = cap;
    ok = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
      for (int i = 0; i < (1 << k); ++i) body();
      ok = hipStreamEndCapture(cap, &g) == hipSuccess;
    }
    hd->stream = user;
  }
  if (ok) ok = hipGraphInstantiate(&exec[k], g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (cap) (void)hipStreamDestroy(cap);
  (void)hipGetLastError();
  state[k] = ok ? 1 : -1;
  return ok;
}

bool cycle_graph(hfz_handle* hd, int k = 0) {
  return capture_graph(hd, hd->graph_state, hd->cycle_exec, k, [&]() { vcycle_and_norm(hd, true); });
}

// One V-cycle and the residual norm that follows it, launched kernel by
// kernel (the host-tested loop).
int cycle_and_residual(hfz_handle* hd, double* norm) {
  vcycle_and_norm(hd, false);
  return residual_read(hd, norm);
}

// ---- mixed precision: FP32 correction V-cycles inside FP64 defect correction

// d = S - N(g) in FP64 -> inner right-hand side, base state, e = 0, and the
// outer stop-test norm into result[0].
void mp_prepare_launch(hfz_handle* hd, bool stop = false, bool counted = true) {
  const Lvl<double>& L = hd->H.L[0];
  const dim3 b = block2(L.n, L.n), g = grid2(L.n, L.n, b);
  by_model(hd->km, [&](auto m) {
    k_mp_prepare<decltype(m)::value><<<g, b, 0, hd->stream>>>(L, hd->H.P, hd->H32.L[0], hd->partial);
  });
  reduce_launch(hd, (int)(g.x * g.y), stop, counted);
}

// One outer iteration: mp_inner FP32 V-cycles on the correction problem
// (three by default: the FP32 solve is cheap next to the FP64 residual and
// the host stop test each outer iteration costs; HFZ_MP_INNER overrides),
// g += e, and the next outer residual.
void mp_cycle(hfz_handle* hd, bool stop) {
  Cycle K = cycle_ctx(hd);
  const Lvl<double>& L = hd->H.L[0];
  const dim3 b = block2(L.n, L.n), g = grid2(L.n, L.n, b);
  by_model(hd->km, [&](auto m) {
    constexpr int M = decltype(m)::value;
    for (int i = 0; i < hd->mp_inner; ++i) hfz::vcycle<M, float, true>(hd->H32, K);
    k_mp_update<M><<<g, b, 0, hd->stream>>>(L, hd->H32.L[0], hd->ctl);
  });
  mp_prepare_launch(hd, stop);
}

bool mp_graph(hfz_handle* hd, int k = 0) {
  return capture_graph(hd, hd->mp_graph_state, hd->mp_exec, k, [&]() { mp_cycle(hd, true); });
}

int mp_cycle_and_residual(hfz_handle* hd, double* norm) {
  mp_cycle(hd, false);
  return residual_read(hd, norm);
}

// The solve of one step: the initial residual and the V-cycles (mixed: outer
// iterations).  On the device-tested path the initial norm and the cycle
// graph run with k_reduce_stop, which raises the stop flag once
// ||S - N(g)|| <= tol or is not finite; the cycles are enqueued in batches
// (the first as long as the previous step needed, then pairs) and the kernels
// of cycles enqueued past the stop return at once, so the cycles that run,
// their count and the final norm are those of the host-tested loop, at one
// host round trip per batch.  Without graphs every cycle is tested on the host.
int solve_step(hfz_handle* hd, bool mixed, double* r, int* cycles_out) {
  int cycles = 0;
  *cycles_out = 0;
  const bool graph = hd->use_graph && (mixed ? mp_graph(hd) : cycle_graph(hd));
  if (!graph) {
    int rc;
    if (mixed) {
      mp_prepare_launch(hd);
      rc = residual_read(hd, r);
    } else {
      rc = residual(hd, r);
    }
    while (rc == HFZ_OK && !(*r <= hd->p.tol)) {
      if (!std::isfinite(*r)) {
        rc = HFZ_ENAN;
        break;
      }
      if (cycles >= hd->p.max_cycles) {
        rc = HFZ_ENOCONV;
        break;
      }
      ++cycles;
      rc = mixed ? mp_cycle_and_residual(hd, r) : cycle_and_residual(hd, r);
    }
    *cycles_out = cycles;
    return rc;
  }
  // `count` cycles as graphs of 8, 4, 2 and 1 (a size whose graph cannot be
  // built is covered by smaller ones)
  auto launch_cycles = [&](int count) -> bool {
    for (int k = kGraphSizes - 1; k >= 0; --k) {
      const bool have = k == 0 || (mixed ? mp_graph(hd, k) : cycle_graph(hd, k));
      if (!have) continue;
      hipGraphExec_t exec = mixed ? hd->mp_exec[k] : hd->cycle_exec[k];
      for (; count >= (1 << k); count -= 1 << k)
        if (hipGraphLaunch(exec, hd->stream) != hipSuccess) return false;
    }
    return true;
  };
  k_ctl_reset<<<1, 64, 0, hd->stream>>>(hd->ctl);
  if (mixed)
    mp_prepare_launch(hd, true, false);
  else
    residual_launch(hd, true, false);
  int rc = HFZ_OK;
  int batch = std::max(1, hd->cycle_hint);
  for (;;) {
    const int remaining = hd->p.max_cycles - cycles;
    const int nb = std::min(batch, remaining);
    if (!launch_cycles(nb)) {
      rc = HFZ_EHIP;
      break;
    }
    double h[10];
    if (hipMemcpyAsync(h, hd->result, sizeof(h), hipMemcpyDeviceToHost, hd->stream) != hipSuccess ||
        hipStreamSynchronize(hd->stream) != hipSuccess) {
      rc = HFZ_EHIP;
      break;
    }
    int ctl[2];
    std::memcpy(ctl, &h[8], sizeof(ctl));
    cycles = ctl[1];
    *r = std::sqrt(h[0]);
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
  k_ctl_reset<<<1, 64, 0, hd->stream>>>(hd->ctl);
  if (rc == HFZ_OK) hd->cycle_hint = std::max(1, cycles);
  *cycles_out = cycles;
  return rc == HFZ_OK ? last_error() : rc;
}

// (J * rho) of Eq. discrete_convolution: jrho = IDFT(mult . DFT(rho)) / n^2.
void convolve(hfz_handle* hd, const double* rho, double* out) {
  const int n = hd->p.n, hx = n / 2 + 1;
  const int thr = std::min(256, n / 2);
  const size_t sh = 2 * (size_t)n * sizeof(double2);
  const dim3 tb(32, 8);
  // rows (two real rows per transform) -> n x hx; columns of the hx kept x
  // frequencies (rows of the transposed hx x n grid; mult's first hx rows are
  // those frequencies) -> back
  k_fft_rows_r2c<<<n / 2, thr, sh, hd->stream>>>(rho, hd->fa, n);
  k_transpose_rect<<<dim3((hx + 31) / 32, (n + 31) / 32), tb, 0, hd->stream>>>(hd->fa, hd->fb, n, hx);
  k_fft_rows_conv<<<hx, thr, sh, hd->stream>>>(hd->fb, hd->mult, n);
  k_transpose_rect<<<dim3((n + 31) / 32, (hx + 31) / 32), tb, 0, hd->stream>>>(hd->fb, hd->fa, hx, n);
  k_fft_rows_c2r<<<n / 2, thr, sh, hd->stream>>>(hd->fa, out, n, 1.0 / ((double)n * n));
}

// CDFT set-up: J on the grid, c_e = h^2 sum J_e, mult = h^2 Re DFT(J) in the
// transposed spectral layout that `convolve` multiplies in.
int cdft_setup(hfz_handle* hd) {
  const int n = hd->p.n;
  const size_t N2 = (size_t)n * n;
  const double h = hd->p.h;
  double* J = reinterpret_cast<double*>(hd->fb);
  double* Je = J + N2;
  const Dims d = dims2(n, n);
  k_kernel_table<<<d.grid, d.block, 0, hd->stream>>>(J, Je, n, ilog2(n), h, hd->p.nu);
  // deterministic sum of J_e: reuse the energy partial layout via a copy-free pass
  const int nb = 256;
  {
    // sum in fixed order: k_reduce_final over N2 "partials" with nq = 1
    k_reduce_final<<<1, 1024, 0, hd->stream>>>(Je, (int)N2, 1, h * h, hd->result);
  }
  double ce = 0.0;
  HIPCHK(hipMemcpyAsync(&ce, hd->result, sizeof(double), hipMemcpyDeviceToHost, hd->stream));
  const int thr = std::min(256, n / 2);
  const size_t sh = 2 * (size_t)n * sizeof(double2);
  const dim3 tg((n + 31) / 32, (n + 31) / 32), tb(32, 8);
  k_fft_rows_real_fwd<<<n, thr, sh, hd->stream>>>(J, hd->fa, n);
  k_transpose<<<tg, tb, 0, hd->stream>>>(hd->fa, hd->fb, n);
  k_fft_rows_fwd<<<n, thr, sh, hd->stream>>>(hd->fb, n);
  k_real_part<<<(unsigned)((N2 + 255) / 256), 256, 0, hd->stream>>>(hd->fb, hd->mult, N2, h * h);
  (void)nb;
  HIPCHK(hipStreamSynchronize(hd->stream));
  hd->ce = ce;
  hd->H.P.ce = ce;
  hd->H32.P.ce = (float)ce;
  return last_error();
}

void copy_dev(hfz_handle* hd, const double* a, double* b, size_t count) {
  k_copy<<<(unsigned)((count + 255) / 256), 256, 0, hd->stream>>>(a, b, count);
}

// Start of a step: omega^k and the source S, the iterate g = state, rho^k and
// omega^k on every level (and their FP32 copies in mixed precision), with
// the batched kernels over this one instance.  Gradient flow: S and the
// initial guess on level 0 (no frozen coefficients).
template <int MODEL> int begin_step_t(hfz_handle* hd) {
  if constexpr (gradflow(MODEL)) {
    const int n = hd->p.n;
    const dim3 b = block2(n, n), g = grid2(n, n, b);
    k_begin_gf<MODEL><<<g, b, 0, hd->stream>>>(hd->H.desc, hd->state1, hd->phys1, hd->on1);
    return last_error();
  }
  const bool mixed = hd->p.precision == HFZ_MIXED;
  for (int l = 0; l < hd->nlev; ++l) {
    const int n = hd->H.L[l].n, ny = hd->H.L[l].ny;
    const dim3 b = block2(n, ny), g = grid2(n, ny, b);
    const Lvl<float>* E = mixed ? hd->H32.desc + l : nullptr;
    if (l == 0)
      k_begin_b<MODEL><<<g, b, 0, hd->stream>>>(hd->H.desc, hd->state1, hd->phys1, hd->on1, E);
    else
      k_restrict_coef_b<walls(MODEL)><<<g, b, 0, hd->stream>>>(hd->H.desc + (l - 1), hd->H.desc + l, hd->on1, E);
  }
  return last_error();
}

int begin_step(hfz_handle* hd) {
  return by_model(hd->km, [&](auto m) { return begin_step_t<decltype(m)::value>(hd); });
}

// End of a step: continuity update, state <- g, the next CDFT convolution.
int finish_step(hfz_handle* hd) {
  const int n = hd->p.n;
  const dim3 b = block2(n, n), g = grid2(n, n, b);
  if (model_gf(hd->p.model)) {
    const int fix = hd->p.continuity_fix ? 1 : 0;
    if (hd->p.model == HFZ_PFC_GF) {
      k_finish_gf<GPFC><<<g, b, 0, hd->stream>>>(hd->H.desc, hd->state1, hd->phys1, hd->on1, fix);
    } else {
      k_finish_gf<GCDFT><<<g, b, 0, hd->stream>>>(hd->H.desc, hd->state1, hd->phys1, hd->on1, fix);
      convolve(hd, hd->H.L[0].rk, hd->jrho);
    }
    return last_error();
  }
  if (hd->km == WPFC) {
    const dim3 bw = block2(n, n + 1), gw = grid2(n, n + 1, bw);
    if (hd->p.continuity_fix) k_continuity_b<true><<<gw, bw, 0, hd->stream>>>(hd->H.desc, hd->phys1, hd->on1);
    const dim3 gs((unsigned)(((size_t)n * (n + 1) + 255) / 256));
    k_state_b<WPFC><<<gs, 256, 0, hd->stream>>>(hd->H.desc, hd->state1, hd->on1);
    return last_error();
  }
  if (hd->p.continuity_fix) k_continuity_b<<<g, b, 0, hd->stream>>>(hd->H.desc, hd->phys1, hd->on1);
  const dim3 gs((unsigned)(((size_t)n * n + 255) / 256));
  if (hd->p.model == HFZ_PFC) {
    k_state_b<PFC><<<gs, 256, 0, hd->stream>>>(hd->H.desc, hd->state1, hd->on1);
  } else {
    k_state_b<CDFT><<<gs, 256, 0, hd->stream>>>(hd->H.desc, hd->state1, hd->on1);
    convolve(hd, hd->H.L[0].rk, hd->jrho);
  }
  return last_error();
}

int energy_impl(hfz_handle* hd, double* out4) {
  const int n = hd->p.n;
  const Lvl<double>& L0 = hd->H.L[0];
  const Dims d = dims2(n, L0.ny);
  const int nb = d.grid.x * d.grid.y;
  if (hd->km == WPFC)
    k_energy_partial<WPFC><<<d.grid, d.block, 0, hd->stream>>>(L0.rk, hd->u, hd->v, nullptr, n, L0.lg, L0.h,
                                                              hd->p.alpha, hd->partial);
  else if (!model_cdft(hd->p.model))
    k_energy_partial<PFC><<<d.grid, d.block, 0, hd->stream>>>(L0.rk, hd->u, hd->v, nullptr, n, L0.lg, L0.h,
                                                             hd->p.alpha, hd->partial);
  else
    k_energy_partial<CDFT><<<d.grid, d.block, 0, hd->stream>>>(L0.rk, hd->u, hd->v, hd->jrho, n, L0.lg, L0.h,
                                                              0.0, hd->partial);
  k_reduce_final<<<1, 1024, 0, hd->stream>>>(hd->partial, nb, 4, L0.h * L0.h, hd->result);
  HIPCHK(hipMemcpyAsync(out4, hd->result, 4 * sizeof(double), hipMemcpyDeviceToHost, hd->stream));
  HIPCHK(hipStreamSynchronize(hd->stream));
  return last_error();
}

double* field_ptr(hfz_handle* hd, int which, int level, int comp) {
  if (level < 0 || level >= hd->nlev) return nullptr;
  Lvl<double>& L = hd->H.L[level];
  switch (which) {
    case 0:
      return (comp >= 0 && comp < hd->nc) ? L.g[comp] : nullptr;
    case 1:
      return (comp >= 0 && comp < hd->nc) ? L.f[comp] : nullptr;
    case 2:
      return (level > 0 && comp >= 0 && comp < hd->nc) ? L.g0[comp] : nullptr;
    case 3:
      return comp == 0 ? L.rk : (comp == 1 ? L.om : nullptr);
    case 4:
      return (level == 0 && comp == 0) ? hd->jrho : nullptr;
    default:
      return nullptr;
  }
}

// Uploads count values from host to device memory on `stream`: with
// by_kernel one small kernel per value carries it in its arguments (no
// host-to-device copy), else one hipMemcpyAsync.
template <typename T> bool upload(T* dst, const T* src, size_t count, hipStream_t stream, bool by_kernel) {
  if (!by_kernel)
    return hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, stream) == hipSuccess;
  for (size_t k = 0; k < count; ++k) k_put<T><<<1, 64, 0, stream>>>(dst + k, src[k]);
  return hipGetLastError() == hipSuccess;
}

// Sets up a handle over the workspace dev_ws (validated and large enough):
// layout, level descriptors on the device, physics, kernel choices, the CDFT
// kernel table.  by_kernel (hfz_step_noalloc): uploads by kernel arguments,
// no timing of kernel candidates (the choices cached in this process, else
// the defaults) and no HIP graphs.
int init_handle(hfz_handle* hd, const hfz_params& p, void* dev_ws, void* hip_stream, bool by_kernel) {
  hd->p = p;
  hd->km = kernel_model(p);
  hd->stream = static_cast<hipStream_t>(hip_stream);
  layout(p, dev_ws, hd);
  bool ok = upload(hd->H.desc, hd->H.L.data(), hd->H.L.size(), hd->stream, by_kernel);
  if (ok && p.precision == HFZ_MIXED) ok = upload(hd->H32.desc, hd->H32.L.data(), hd->H32.L.size(), hd->stream, by_kernel);
  if (!ok || hipStreamSynchronize(hd->stream) != hipSuccess) return HFZ_EHIP;
  hd->H.P.s = p.s;
  hd->H.P.gamma = p.gamma;
  hd->H.P.sigma = (double)p.sigma;
  hd->H.P.alpha = p.alpha;
  hd->H.P.delta = p.delta;
  hd->H.P.w = p.w_damp;
  hd->H.P.ce = 0.0;
  hd->H.P.ub = p.u_wall_bottom;
  hd->H.P.ut = p.u_wall_top;
  hd->H32.P.s = (float)p.s;
  hd->H32.P.gamma = (float)p.gamma;
  hd->H32.P.sigma = (float)p.sigma;
  hd->H32.P.alpha = (float)p.alpha;
  hd->H32.P.delta = (float)p.delta;
  hd->H32.P.w = (float)p.w_damp;
  hd->H32.P.ce = 0.0f;
  hd->H32.P.ub = (float)p.u_wall_bottom;
  hd->H32.P.ut = (float)p.u_wall_top;
  hd->H.P.halt = hd->ctl;
  hd->H32.P.halt = hd->ctl;
  k_ctl_reset<<<1, 64, 0, hd->stream>>>(hd->ctl);
  // opt in to the large LDS of a gfx950 CU for the tail kernels
  by_model(hd->km, [&](auto m) {
    constexpr int M = decltype(m)::value;
    hd->H.tail_lds_max = lds_optin(reinterpret_cast<const void*>(&k_tail<M, double, false>));
    hd->H32.tail_lds_max = lds_optin(reinterpret_cast<const void*>(&k_tail<M, float, true>));
  });
  if (const char* e = std::getenv("HFZ_TAIL_N")) {
    const int t = std::atoi(e);
    if (t == 0 || is_pow2(t)) hd->tail_n = t;
  }
  if (const char* e = std::getenv("HFZ_GRAPH")) hd->use_graph = std::atoi(e) != 0;
  if (const char* e = std::getenv("HFZ_TILES")) hd->use_tiles = std::atoi(e) != 0;
  if (p.precision == HFZ_MIXED || p.walls) {
    // the correction-form inner solve, and a channel, run only on the tiled
    // and tail kernels: every level above the tail must be tileable (>= 32
    // with a >= 16 coarse), and the coarsest level (<= 32, validate()) must
    // be a tail level
    hd->use_tiles = true;
    if (hd->tail_n < 16) hd->tail_n = kTailNMax;
    hd->tail_n = std::max(hd->tail_n, p.coarsest_n);
    const bool held = by_model(hd->km, [&](auto m) {
      constexpr int M = decltype(m)::value;
      return p.precision == HFZ_MIXED ? tail_holds_bottom<M, float, true>(hd->H32.L, hd->tail_n, hd->H32.tail_lds_max)
                                       : tail_holds_bottom<M, double, false>(hd->H.L, hd->tail_n, hd->H.tail_lds_max);
    });
    if (!held) return HFZ_EINVAL;
  }
  if (by_kernel) hd->use_graph = false;
  if (hd->use_tiles) {
    const Cycle K = cycle_ctx(hd);
    by_model(hd->km, [&](auto m) {
      constexpr int M = decltype(m)::value;
      tune_tile_shapes<M, double, false>(hd->H, K, !by_kernel);
      if (p.precision == HFZ_MIXED) tune_tile_shapes<M, float, true>(hd->H32, K, !by_kernel);
      if (std::getenv("HFZ_VERBOSE")) {
        std::fprintf(stderr, "hfz: right-hand side completed by the pre-sweep launch:");
        for (int l = 0; l < (int)hd->H.L.size(); ++l)
          std::fprintf(stderr, " %d", (int)level_fold_rhs<M, double, false>(hd->H, K, l));
        std::fprintf(stderr, "\n");
      }
    });
  }
  if (const char* e = std::getenv("HFZ_MP_INNER")) hd->mp_inner = std::max(1, std::min(8, std::atoi(e)));
  if (std::getenv("HFZ_VERBOSE")) {
    std::fprintf(stderr, "hfz: n=%d levels=%d tail_n=%d tail_lds_max=%zu graph=%d tile shapes:", p.n, hd->nlev,
                 hd->tail_n, hd->H.tail_lds_max, (int)hd->use_graph);
    for (size_t l = 0; l < hd->H.tile_shape.size(); ++l) std::fprintf(stderr, " %d", hd->H.tile_shape[l]);
    std::fprintf(stderr, " restriction:");
    for (size_t l = 0; l < hd->H.restrict_shape.size(); ++l) std::fprintf(stderr, " %d", hd->H.restrict_shape[l]);
    std::fprintf(stderr, " sweeps/launch:");
    for (size_t l = 0; l < hd->H.sweep_fuse.size(); ++l) std::fprintf(stderr, " %d", hd->H.sweep_fuse[l]);
    std::fprintf(stderr, " restriction folded:");
    for (size_t l = 0; l < hd->H.fused.size(); ++l) std::fprintf(stderr, " %d", (int)hd->H.fused[l]);
    for (size_t l = 0; l < hd->H32.tile_shape.size(); ++l) std::fprintf(stderr, "%s%d", l ? " " : " | ", hd->H32.tile_shape[l]);
    std::fprintf(stderr, "\n");
  }
  if (model_cdft(p.model)) {
    const int rc = cdft_setup(hd);
    if (rc != HFZ_OK) return rc;
  }
  {
    const StateB sb{hd->u, hd->v, hd->mu, hd->ka, hd->jrho};
    const int one = 1;
    const bool up = upload(hd->state1, &sb, 1, hd->stream, by_kernel) &&
                    upload(hd->phys1, &hd->H.P, 1, hd->stream, by_kernel) &&
                    upload(hd->on1, &one, 1, hd->stream, by_kernel) && hipStreamSynchronize(hd->stream) == hipSuccess;
    if (!up) return HFZ_EHIP;
  }
  return HFZ_OK;
}

}  // namespace

extern "C" {

int hfz_default_params(int model, hfz_params* p) {
  if (!p || model < HFZ_PFC || model > HFZ_CDFT_GF) return HFZ_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->model = model;
  p->n = 32;
  p->h = 0.25;
  p->s = 0.01;
  p->gamma = 2.0;
  p->alpha = 0.975;
  p->nu = 2.362;
  p->delta = model_cdft(model) ? 1e-10 : 0.0;
  p->w_damp = 0.5;
  p->tol = 1e-10;
  p->nu1 = 2;
  p->nu2 = 2;
  p->max_cycles = 200;
  p->coarsest_n = 4;
  p->coarse_sweeps = 4;
  p->precision = HFZ_FP64;
  p->sigma = 1;
  p->continuity_fix = 1;
  return HFZ_OK;
}

int hfz_workspace_bytes(const hfz_params* p, size_t* bytes) {
  const int rc = validate(p);
  if (rc != HFZ_OK) return rc;
  if (!bytes) return HFZ_EINVAL;
  *bytes = layout(*p, nullptr, nullptr);
  return HFZ_OK;
}

int hfz_init(const hfz_params* p, void* dev_ws, size_t ws_bytes, void* hip_stream, hfz_handle** out) {
  if (!out) return HFZ_EINVAL;
  *out = nullptr;
  int rc = validate(p);
  if (rc != HFZ_OK) return rc;
  const size_t need = layout(*p, nullptr, nullptr);
  if (!dev_ws || ws_bytes < need) return HFZ_ENOMEM;
  if (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) return HFZ_EINVAL;
  hfz_handle* hd = new (std::nothrow) hfz_handle();
  if (!hd) return HFZ_ENOMEM;
  rc = init_handle(hd, *p, dev_ws, hip_stream, false);
  if (rc != HFZ_OK) {
    delete hd;
    return rc;
  }
  *out = hd;
  return HFZ_OK;
}

int hfz_set_state(hfz_handle* hd, const double* rho, const double* u, const double* v) {
  if (!hd || !rho) return HFZ_EINVAL;
  const bool gf = model_gf(hd->p.model);
  if (!gf && (!u || !v)) return HFZ_EINVAL;
  const int n = hd->p.n;
  const size_t N2 = (size_t)n * hd->H.L[0].ny;
  Lvl<double>& L0 = hd->H.L[0];
  if (model_cdft(hd->p.model)) {
    k_min_partial<<<256, 256, 0, hd->stream>>>(rho, N2, hd->partial);
    double mins[256];
    HIPCHK(hipMemcpyAsync(mins, hd->partial, sizeof(mins), hipMemcpyDeviceToHost, hd->stream));
    HIPCHK(hipStreamSynchronize(hd->stream));
    double mn = mins[0];
    for (double x : mins) mn = std::min(mn, x);
    if (!(mn > 0.0)) return HFZ_EDOMAIN;
  }
  copy_dev(hd, rho, L0.rk, N2);
  if (gf) {
    // the gradient flow has no velocity: u = v = 0 (KE = 0 in the energy)
    k_fill<<<(unsigned)((N2 + 255) / 256), 256, 0, hd->stream>>>(hd->u, 0.0, N2);
    k_fill<<<(unsigned)((N2 + 255) / 256), 256, 0, hd->stream>>>(hd->v, 0.0, N2);
  } else {
    copy_dev(hd, u, hd->u, N2);
    copy_dev(hd, v, hd->v, N2);
  }
  const Dims d = dims2(n, n);
  if (hd->km == WPFC) {
    const Dims dw = dims2(n, n + 1);
    k_wall_state<<<(n + 63) / 64, 64, 0, hd->stream>>>(L0.rk, hd->u, hd->v, n, L0.lg, hd->p.u_wall_bottom,
                                                       hd->p.u_wall_top);
    k_pfc_kappa<true><<<dw.grid, dw.block, 0, hd->stream>>>(L0.rk, hd->ka, n, L0.lg, L0.h);
    k_pfc_mu<true><<<dw.grid, dw.block, 0, hd->stream>>>(L0.rk, hd->ka, hd->mu, n, L0.lg, L0.h, hd->p.alpha);
  } else if (!model_cdft(hd->p.model)) {
    k_pfc_kappa<<<d.grid, d.block, 0, hd->stream>>>(L0.rk, hd->ka, n, L0.lg, L0.h);
    k_pfc_mu<<<d.grid, d.block, 0, hd->stream>>>(L0.rk, hd->ka, hd->mu, n, L0.lg, L0.h, hd->p.alpha);
  } else {
    convolve(hd, L0.rk, hd->jrho);
    if (gf) k_gcdft_mu0<<<(unsigned)((N2 + 255) / 256), 256, 0, hd->stream>>>(L0.rk, hd->jrho, hd->mu, N2, hd->ce);
  }
  HIPCHK(hipStreamSynchronize(hd->stream));
  hd->has_state = true;
  return last_error();
}

int hfz_get_state(hfz_handle* hd, double* rho, double* u, double* v) {
  if (!hd || !rho) return HFZ_EINVAL;
  if (!model_gf(hd->p.model) && (!u || !v)) return HFZ_EINVAL;
  if (!hd->has_state) return HFZ_ESTATE;
  const size_t N2 = (size_t)hd->p.n * hd->H.L[0].ny;
  copy_dev(hd, hd->H.L[0].rk, rho, N2);
  if (u) copy_dev(hd, hd->u, u, N2);
  if (v) copy_dev(hd, hd->v, v, N2);
  HIPCHK(hipStreamSynchronize(hd->stream));
  return last_error();
}

int hfz_get_aux(hfz_handle* hd, double* mu, double* kappa) {
  if (!hd || !mu || hd->p.model == HFZ_CDFT) return HFZ_EINVAL;
  const bool has_kappa = hd->ka != nullptr;
  if (has_kappa && !kappa) return HFZ_EINVAL;
  if (!hd->has_state) return HFZ_ESTATE;
  const size_t N2 = (size_t)hd->p.n * hd->H.L[0].ny;
  copy_dev(hd, hd->mu, mu, N2);
  if (has_kappa) copy_dev(hd, hd->ka, kappa, N2);
  HIPCHK(hipStreamSynchronize(hd->stream));
  return last_error();
}

int hfz_begin_step(hfz_handle* hd) {
  if (!hd) return HFZ_EINVAL;
  if (!hd->has_state) return HFZ_ESTATE;
  return begin_step(hd);
}

int hfz_smooth(hfz_handle* hd, int level, int sweeps) {
  if (!hd || level < 0 || level >= hd->nlev || sweeps < 0) return HFZ_EINVAL;
  Cycle K = cycle_ctx(hd);
  if (hd->use_tiles && hd->H.L[level].gb[0] != nullptr) {
    // the sweeps the V-cycle runs on this level (tiled, double-buffered)
    const Lvl<double>& L = hd->H.L[level];
    const Fld<double> home = fld<double>(L.g);
    Fld<double> cur = home, other = fld<double>(L.gb);
    by_model(hd->km, [&](auto m) {
      tiled_sweeps<decltype(m)::value, double, false>(hd->H, K, level, sweeps, false, cur, other);
    });
    if (cur.c[0] != home.c[0]) copy_fields<double>(K, cur, home, hd->nc, (size_t)L.n * L.ny);
  } else {
    by_model(hd->km, [&](auto m) { smooth_level<decltype(m)::value, double>(hd->H, K, level, sweeps); });
  }
  return last_error();
}

int hfz_vcycle(hfz_handle* hd, int count) {
  if (!hd || count < 0) return HFZ_EINVAL;
  for (int k = 0; k < count; ++k) vcycle(hd);
  return last_error();
}

int hfz_residual(hfz_handle* hd, double* norm) {
  if (!hd || !norm) return HFZ_EINVAL;
  return residual(hd, norm);
}

int hfz_finish_step(hfz_handle* hd) {
  if (!hd) return HFZ_EINVAL;
  return finish_step(hd);
}

int hfz_step(hfz_handle* hd, int nsteps, hfz_stats* stats) {
  if (!hd || nsteps < 0) return HFZ_EINVAL;
  if (!hd->has_state) return HFZ_ESTATE;
  hfz_stats st{};
  int rc = HFZ_OK;
  for (int k = 0; k < nsteps; ++k) {
    rc = begin_step(hd);
    if (rc != HFZ_OK) break;
    const bool mixed = hd->p.precision == HFZ_MIXED;
    double r = 0.0;
    int cycles = 0;
    rc = solve_step(hd, mixed, &r, &cycles);
    st.cycles_last = cycles;
    st.residual_last = r;
    if (rc != HFZ_OK) break;
    rc = finish_step(hd);
    if (rc != HFZ_OK) break;
    st.steps_done++;
    st.cycles_total += cycles;
  }
  if (rc == HFZ_OK) {
    if (hipStreamSynchronize(hd->stream) != hipSuccess) rc = HFZ_EHIP;
  }
  if (stats) *stats = st;
  return rc;
}

int hfz_energy(hfz_handle* hd, double* out5) {
  if (!hd || !out5) return HFZ_EINVAL;
  if (!hd->has_state) return HFZ_ESTATE;
  double q[4];
  const int rc = energy_impl(hd, q);
  if (rc != HFZ_OK) return rc;
  const double F = q[1] + q[2];
  out5[0] = q[0] + F;
  out5[1] = q[0];
  out5[2] = F;
  out5[3] = model_cdft(hd->p.model) ? q[1] : 0.0;
  out5[4] = model_cdft(hd->p.model) ? q[2] : 0.0;
  if (!std::isfinite(out5[0])) return HFZ_ENAN;
  return HFZ_OK;
}

int hfz_mass(hfz_handle* hd, double* mass) {
  if (!hd || !mass) return HFZ_EINVAL;
  if (!hd->has_state) return HFZ_ESTATE;
  double q[4];
  const int rc = energy_impl(hd, q);
  if (rc != HFZ_OK) return rc;
  *mass = q[3];
  return HFZ_OK;
}

int hfz_read_field(hfz_handle* hd, int which, int level, int comp, double* dst) {
  if (!hd || !dst) return HFZ_EINVAL;
  double* src = field_ptr(hd, which, level, comp);
  if (!src) return HFZ_EINVAL;
  const size_t cnt = (size_t)hd->H.L[level].n * hd->H.L[level].ny;
  copy_dev(hd, src, dst, cnt);
  HIPCHK(hipStreamSynchronize(hd->stream));
  return last_error();
}

int hfz_write_field(hfz_handle* hd, int which, int level, int comp, const double* src) {
  if (!hd || !src) return HFZ_EINVAL;
  double* dst = field_ptr(hd, which, level, comp);
  if (!dst) return HFZ_EINVAL;
  const size_t cnt = (size_t)hd->H.L[level].n * hd->H.L[level].ny;
  copy_dev(hd, src, dst, cnt);
  HIPCHK(hipStreamSynchronize(hd->stream));
  return last_error();
}

int hfz_info(hfz_handle* hd, int* levels, double* ce) {
  if (!hd) return HFZ_EINVAL;
  if (levels) *levels = hd->nlev;
  if (ce) *ce = hd->ce;
  return HFZ_OK;
}

int hfz_tile_shape(hfz_handle* hd, int level, int* tx, int* ty, int* threads) {
  if (!hd || !tx || !ty || !threads || level < 0 || level >= (int)hd->H.tile_shape.size()) return HFZ_EINVAL;
  const int n = hd->H.L[level].n;
  if (!hd->use_tiles || level + 1 >= hd->nlev || n < TILE_X || hd->H.L[level + 1].n < RTILE || n <= hd->tail_n)
    return HFZ_EINVAL;
  int ts = hd->H.tile_shape[level];
  if (!tile_shape_fits(ts, n)) ts = 0;
  *tx = kTileShapes[ts].tx;
  *ty = kTileShapes[ts].ty;
  *threads = kTileShapes[ts].nt;
  return HFZ_OK;
}

int hfz_destroy(hfz_handle* hd) {
  if (!hd) return HFZ_EINVAL;
  for (int k = 0; k < kGraphSizes; ++k) {
    if (hd->cycle_exec[k]) (void)hipGraphExecDestroy(hd->cycle_exec[k]);
    if (hd->mp_exec[k]) (void)hipGraphExecDestroy(hd->mp_exec[k]);
  }
  delete hd;
  return HFZ_OK;
}

const char* hfz_strerror(int code) {
  switch (code) {
    case HFZ_OK:
      return "ok";
    case HFZ_EINVAL:
      return "invalid argument";
    case HFZ_ENOMEM:
      return "workspace too small";
    case HFZ_EDOMAIN:
      return "density must be positive for the CDFT model";
    case HFZ_ENOCONV:
      return "FAS did not reach the tolerance within max_cycles";
    case HFZ_ENAN:
      return "non-finite residual or energy";
    case HFZ_EHIP:
      return "HIP runtime error";
    case HFZ_ESTATE:
      return "no state loaded";
    case HFZ_ESCRATCH:
      return "problem needs more device memory than the static scratch of hfz_step_noalloc holds";
    default:
      return "unknown error";
  }
}

}  // extern "C"

// ===========================================================================
// The step without device allocation (hfz_step_noalloc): the handle's
// workspace is the file-scope device array `scratch`, of which every GPU the
// library runs on holds its own copy until the process ends.  Host code never
// passes `scratch` itself to a kernel or a copy (in host code the name is a
// host-side stand-in, not the device address): the address of each device's
// copy is queried once per device with hipGetSymbolAddress, with that device
// current, and kept in scratch_addr.
// ===========================================================================

static __device__ __align__(256) unsigned char scratch[HFZ_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of the current device's scratch (nullptr on a HIP error).
void* scratch_addr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mutex);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_addr[dev] = ptr;
  }
  return g_scratch_addr[dev];
}

}  // namespace

extern "C" int hfz_step_noalloc(const hfz_params* p, double* rho, double* u, double* v, int nsteps,
                                void* hip_stream, hfz_stats* stats) {
  if (stats) *stats = hfz_stats{};
  int rc = validate(p);
  if (rc != HFZ_OK) return rc;
  if (!rho || nsteps < 0 || (!model_gf(p->model) && (!u || !v))) return HFZ_EINVAL;
  if (layout(*p, nullptr, nullptr) > HFZ_NOALLOC_SCRATCH_BYTES) return HFZ_ESCRATCH;
  void* ws = scratch_addr();
  if (!ws) return HFZ_EHIP;
  hfz_handle hd;
  rc = init_handle(&hd, *p, ws, hip_stream, true);
  if (rc == HFZ_OK) rc = hfz_set_state(&hd, rho, u, v);
  if (rc != HFZ_OK) return rc;
  rc = hfz_step(&hd, nsteps, stats);
  // the state after the last completed step (a failing step is rolled back)
  const int rc_get = hfz_get_state(&hd, rho, model_gf(p->model) ? nullptr : u, model_gf(p->model) ? nullptr : v);
  return rc != HFZ_OK ? rc : rc_get;
}

// ===========================================================================
// Batched solve: many independent instances of one model and precision
// advance together; their grid sizes may differ.  Every instance is an
// ordinary handle over its own slice of the batch workspace (so set/get
// state, energy and the per-step kernels are the single-instance ones).  The
// instances are kept sorted by grid size, largest first (the slot order), and
// their multigrid levels are aligned from the coarsest grid, which all share:
// at depth d (d = 0 the coarsest level) every instance that has a level there
// has a grid of size coarsest_n * 2^d, and those instances are the first
// cnt[d] slots.  Each V-cycle phase of one depth is then one launch over those
// instances (instance in blockIdx.z; the coarse tail one workgroup per
// instance, one launch per tail size), and each instance's phases run in the
// order of its own V-cycle, so it gets the result it gets alone.  Each
// instance keeps its own stop test; converged instances drop out of the
// launches.
// ===========================================================================

struct hfz_batch {
  int count = 0;
  hfz_params p{};  // model, precision, nu1, nu2, coarsest_n, coarse_sweeps, continuity_fix: shared
  int tile_force = -1;  // smoother tile shape forced by HFZ_BATCH_TILE at init (-1: by level size)
  // FAS restriction (HFZ_BATCH_RESTRICT): 3 the staged kernel with coarse
  // tiles of 16 and 512 threads; 2 the same with 256 threads, 1 with tiles of
  // 8 and 256 threads; 0 the direct kernel
  int restrict_mode = 3;
  hipStream_t stream = nullptr;
  std::vector<hfz_handle*> inst;  // by slot
  std::vector<int> slot_of;       // user index -> slot
  int nmax = 0;                   // largest grid
  int depths = 0;                 // levels of the largest instance
  std::vector<int> cnt;           // [depth] instances with a level there (slots 0 .. cnt - 1)
  std::vector<int> size_at;       // [depth] grid size there
  std::vector<int> h_top;         // [slot] depth of the instance's finest level
  int tail_depth = 0;             // depth of the tail's top level (tail_n) for instances that large
  std::vector<int> tail_first, tail_count, tail_top;  // tail launches: first slot, slots, top depth
  int tiled_count = 0;            // slots whose finest level is above the tail (the first ones)
  std::vector<size_t> doff;       // start of depth d in D64 / D32
  // device arrays
  Lvl<double>* D64 = nullptr;  // [depth][slot < cnt[depth]]
  Lvl<float>* D32 = nullptr;
  Lvl<double>* L064 = nullptr;  // [slot] the finest level
  Lvl<float>* L032 = nullptr;
  Lvl<double>* T64 = nullptr;  // [slot][k] the tail's levels from its top down (TAIL_MAX_LEVELS per slot)
  Lvl<float>* T32 = nullptr;
  Phys<double>* P64 = nullptr;  // [slot]
  Phys<float>* P32 = nullptr;
  int* active = nullptr;
  double* norm2 = nullptr;
  StateB* S = nullptr;   // [slot] state arrays of each instance
  int* on = nullptr;     // [slot] instances the batched begin / finish kernels treat
  std::vector<int> h_on;
  int* cyc = nullptr;     // [slot] V-cycles (mixed: outer iterations) of the current step
  int* stat = nullptr;    // [slot] 0 running, 1 converged, 2 not finite, 3 max_cycles reached
  double* tol = nullptr;  // [slot]
  int* maxc = nullptr;    // [slot]
  int* topd = nullptr;    // [slot] depth of the finest level
  int* npart = nullptr;   // [slot] stop-test partial sums a V-cycle leaves for the instance
  double* partial = nullptr;
  int pstride = 0;
  int cycle_hint = 4;  // most cycles an instance needed in the previous step
  size_t lds64 = 0, lds32 = 0;
  std::vector<int> h_active;
  std::vector<double> h_norm2;
  int graph_state = 0;
  hipGraphExec_t exec = nullptr;
  bool use_graph = true;
};

namespace {

bool batch_compatible(const hfz_params& a, const hfz_params& b) {
  return a.model == b.model && a.precision == b.precision && a.nu1 == b.nu1 && a.nu2 == b.nu2 &&
         a.coarsest_n == b.coarsest_n && a.coarse_sweeps == b.coarse_sweeps && a.continuity_fix == b.continuity_fix;
}

// Host-side geometry of a batch: slot order, the instances' workspace slices,
// the per-depth counts and the offsets of the batch arrays.
struct BatchGeom {
  std::vector<int> order;  // slot -> user index (grid size descending, stable)
  std::vector<int> n, nlev;
  std::vector<size_t> ws_off, ws_bytes;
  int depths = 0;
  std::vector<int> cnt;
  size_t ndesc = 0;
  int pstride = 0;
  size_t off_arrays = 0, total = 0;
};

BatchGeom batch_geom(const hfz_params* ps, int count) {
  BatchGeom G;
  G.order.resize(count);
  for (int i = 0; i < count; ++i) G.order[i] = i;
  std::stable_sort(G.order.begin(), G.order.end(), [&](int a, int b) { return ps[a].n > ps[b].n; });
  size_t off = 0;
  for (int k = 0; k < count; ++k) {
    const hfz_params& p = ps[G.order[k]];
    G.n.push_back(p.n);
    G.nlev.push_back(ilog2(p.n) - ilog2(p.coarsest_n) + 1);
    const size_t b = align_up(layout(p, nullptr, nullptr));
    G.ws_off.push_back(off);
    G.ws_bytes.push_back(b);
    off += b;
    G.ndesc += G.nlev.back();
  }
  G.depths = G.nlev[0];
  G.cnt.assign(G.depths, 0);
  for (int k = 0; k < count; ++k)
    for (int d = 0; d < G.nlev[k]; ++d) G.cnt[d]++;
  G.off_arrays = off;
  G.pstride = (int)((size_t)G.n[0] * G.n[0] / 256 + 64);
  Carver c{nullptr};
  c.take<Lvl<double>>(G.ndesc);
  c.take<Lvl<float>>(G.ndesc);
  c.take<Lvl<double>>(count);
  c.take<Lvl<float>>(count);
  c.take<Lvl<double>>((size_t)count * TAIL_MAX_LEVELS);
  c.take<Lvl<float>>((size_t)count * TAIL_MAX_LEVELS);
  c.take<Phys<double>>(count);
  c.take<Phys<float>>(count);
  c.take<int>(count);
  c.take<double>(count);
  c.take<int>((size_t)count * 5);
  c.take<double>(count);
  c.take<StateB>(count);
  c.take<int>(count);
  c.take<double>((size_t)G.pstride * count);
  G.total = G.off_arrays + c.off;
  return G;
}

// Tile shape of the batched smoother on an n x n level: 64x16 tiles of 512
// threads (shape 2) where they divide n, else 32x16 of 256 (shape 0); forced
// (0 or 2, from the environment variable HFZ_BATCH_TILE at hfz_batch_init)
// overrides it where the shape divides n.  (With many instances per launch
// the workgroups fill the device at any level size, and the wider tile
// recomputes less halo; the 1024-thread shapes time slower here.)
int batch_tile_shape(int n, int forced) {
  const auto fits = [n](int ts) { return n % kTileShapes[ts].tx == 0 && n % kTileShapes[ts].ty == 0; };
  if ((forced == 0 || forced == 2) && fits(forced)) return forced;
  return fits(2) ? 2 : 0;
}

// Launch grid over each instance's finest level (sized for the largest; the
// kernels' threads outside their own instance's grid return).
void batch_top_grid(const hfz_batch* B, int n, int count, dim3* g, dim3* b) {
  *b = block2(n, n);
  const dim3 g2 = grid2(n, n, *b);
  *g = dim3(g2.x, g2.y, count);
}

// One batched V-cycle from depth d down: a tiled level launched over the
// first cnt[d] slots, or, at the tail's depth, the tails of all instances.
template <int MODEL, typename T, bool CORR>
void bvcycle_depth(hfz_batch* B, Lvl<T>* D, Lvl<T>* Tl, Phys<T>* Ps, size_t lds_max, const Cycle& K, int d) {
  constexpr int NCm = NC<MODEL>::value, NB = CORR ? NBase<MODEL>::value : 0, NR = NCoef<MODEL>::value;
  if (d <= B->tail_depth) {
    for (size_t t = 0; t < B->tail_first.size(); ++t) {
      const int first = B->tail_first[t], td = B->tail_top[t];
      TailArgs<T> A{};
      A.Lg = Tl + (size_t)first * TAIL_MAX_LEVELS;
      A.nt = td + 1;
      A.top_n = B->size_at[td];
      A.nu1 = K.nu1;
      A.nu2 = K.nu2;
      A.coarse_sweeps = K.coarse_sweeps;
      tail_plan<MODEL, T, CORR>(A.top_n, A.nt, lds_max, &A.d_from);
      const size_t sh = tail_lds_count<NCm, NB, NR, 0, tail_pm<MODEL>()>(A.top_n, A.nt, A.d_from) * sizeof(T);
      k_tail_b<MODEL, T, CORR><<<B->tail_count[t], TAIL_THREADS, sh, K.stream>>>(A, TAIL_MAX_LEVELS, Ps + first,
                                                                                 B->active + first);
    }
    return;
  }
  Lvl<T>* Dl = D + B->doff[d];
  Lvl<T>* Dc = D + B->doff[d - 1];
  const int n = B->size_at[d], nc = B->size_at[d - 1], cz = B->cnt[d];
  const int ts = batch_tile_shape(n, B->tile_force);
  const dim3 grid(n / kTileShapes[ts].tx, n / kTileShapes[ts].ty, cz);
  int inb = 0;
  auto sweeps = [&](int total, bool pro, int res_last) {
    while (total > 0) {
      const int nsw = total >= 2 ? 2 : 1;
      const int res = (total == nsw) ? res_last : 0;
#define HFZ_BT(NSW, PRO, RES)                                                                                  \
  do {                                                                                                         \
    if (ts == 2)                                                                                               \
      k_sweeps_tile_b<MODEL, T, NSW, PRO, RES, CORR, 2><<<grid, kTileShapes[2].nt, 0, K.stream>>>(             \
          Dl, Dc, Ps, B->active, inb, B->partial, B->pstride, B->topd, d);                                      \
    else                                                                                                       \
      k_sweeps_tile_b<MODEL, T, NSW, PRO, RES, CORR, 0><<<grid, kTileShapes[0].nt, 0, K.stream>>>(             \
          Dl, Dc, Ps, B->active, inb, B->partial, B->pstride, B->topd, d);                                      \
  } while (0)
      if (nsw == 2) {
        if (pro) {
          if (res == 2) HFZ_BT(2, true, 2); else if (res == 1) HFZ_BT(2, true, 1); else HFZ_BT(2, true, 0);
        } else {
          if (res == 2) HFZ_BT(2, false, 2); else if (res == 1) HFZ_BT(2, false, 1); else HFZ_BT(2, false, 0);
        }
      } else {
        if (pro) {
          if (res == 2) HFZ_BT(1, true, 2); else if (res == 1) HFZ_BT(1, true, 1); else HFZ_BT(1, true, 0);
        } else {
          if (res == 2) HFZ_BT(1, false, 2); else if (res == 1) HFZ_BT(1, false, 1); else HFZ_BT(1, false, 0);
        }
      }
#undef HFZ_BT
      inb ^= 1;
      total -= nsw;
      pro = false;
    }
  };
  sweeps(K.nu1, false, 1);
  // the FAS restriction: the staged kernel (coarse tiles through LDS), or the
  // direct one (HFZ_BATCH_RESTRICT=0)
  if (B->restrict_mode == 2 && nc % 16 == 0)
    k_restrict_fas_staged_b<MODEL, T, CORR, 16, 256><<<dim3(nc / 16, nc / 16, cz), 256, 0, K.stream>>>(
        Dl, Dc, Ps, B->active, inb);
  else if (B->restrict_mode == 3 && nc % 16 == 0)
    k_restrict_fas_staged_b<MODEL, T, CORR, 16, 512><<<dim3(nc / 16, nc / 16, cz), 512, 0, K.stream>>>(
        Dl, Dc, Ps, B->active, inb);
  else if (B->restrict_mode != 0 && nc % 8 == 0)
    k_restrict_fas_staged_b<MODEL, T, CORR, 8, 256><<<dim3(nc / 8, nc / 8, cz), 256, 0, K.stream>>>(
        Dl, Dc, Ps, B->active, inb);
  else
    k_restrict_fas_tile_b<MODEL, T, CORR><<<dim3(nc / RTILE, nc / RTILE, cz), RTILE * RTILE, 0, K.stream>>>(
        Dl, Dc, Ps, B->active, inb);
  bvcycle_depth<MODEL, T, CORR>(B, D, Tl, Ps, lds_max, K, d - 1);
  // the post-sweeps leave stop-test partial sums for the instances whose
  // finest level this is (FP64 solve)
  sweeps(K.nu2, true, CORR ? 0 : 2);
  if (inb) k_swap_back_b<T><<<dim3((n * n + 255) / 256, 1, cz), 256, 0, K.stream>>>(Dl, B->active, NCm);
}

// Enqueues one batched V-cycle (mixed: one outer iteration), the
// per-instance stop-test norms into B->norm2 and the device stop test.
template <int MODEL> void batch_cycle(hfz_batch* B, hipStream_t stream) {
  hfz_handle* h0 = B->inst[0];
  Cycle K = cycle_ctx(h0);
  K.stream = stream;
  K.partial = B->partial;
  dim3 g, b;
  batch_top_grid(B, B->nmax, B->count, &g, &b);
  if (B->p.precision == HFZ_MIXED) {
    for (int i = 0; i < h0->mp_inner; ++i)
      bvcycle_depth<MODEL, float, true>(B, B->D32, B->T32, B->P32, B->lds32, K, B->depths - 1);
    k_mp_update_b<MODEL><<<g, b, 0, stream>>>(B->L064, B->L032, B->active);
    k_mp_prepare_b<MODEL><<<g, b, 0, stream>>>(B->L064, B->P64, B->L032, B->active, B->partial, B->pstride);
    k_reduce_stop_b<<<B->count, 1024, 0, stream>>>(B->partial, (int)(g.x * g.y), nullptr, B->pstride, B->L064,
                                                   B->active, B->norm2, B->cyc, B->stat, B->tol, B->maxc, 1);
  } else {
    bvcycle_depth<MODEL, double, false>(B, B->D64, B->T64, B->P64, B->lds64, K, B->depths - 1);
    if (B->tiled_count < B->count) {
      // instances whose finest level is in the tail: their residual in its own pass
      const int first = B->tiled_count;
      dim3 gt, bt;
      batch_top_grid(B, B->inst[first]->p.n, B->count - first, &gt, &bt);
      k_residual_partial_b<MODEL><<<gt, bt, 0, stream>>>(B->L064 + first, B->P64 + first, B->active + first,
                                                         B->partial + (size_t)first * B->pstride, B->pstride);
    }
    k_reduce_stop_b<<<B->count, 1024, 0, stream>>>(B->partial, 0, B->npart, B->pstride, B->L064, B->active,
                                                   B->norm2, B->cyc, B->stat, B->tol, B->maxc, 1);
  }
}

// The first stop test of a step (before any V-cycle).
template <int MODEL> void batch_first_norm(hfz_batch* B) {
  dim3 g, b;
  batch_top_grid(B, B->nmax, B->count, &g, &b);
  if (B->p.precision == HFZ_MIXED)
    k_mp_prepare_b<MODEL><<<g, b, 0, B->stream>>>(B->L064, B->P64, B->L032, B->active, B->partial, B->pstride);
  else
    k_residual_partial_b<MODEL><<<g, b, 0, B->stream>>>(B->L064, B->P64, B->active, B->partial, B->pstride);
  k_reduce_stop_b<<<B->count, 1024, 0, B->stream>>>(B->partial, (int)(g.x * g.y), nullptr, B->pstride, B->L064,
                                                    B->active, B->norm2, B->cyc, B->stat, B->tol, B->maxc, 0);
}

void batch_cycle_any(hfz_batch* B, hipStream_t s) {
  if (B->p.model == HFZ_PFC)
    batch_cycle<PFC>(B, s);
  else
    batch_cycle<CDFT>(B, s);
}

int batch_launch_cycle(hfz_batch* B) {
  if (B->use_graph && B->graph_state == 0) {
    hipStream_t cap = nullptr;
    hipGraph_t g = nullptr;
    bool ok = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess;
    if (ok) ok = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
      batch_cycle_any(B, cap);
      ok = hipStreamEndCapture(cap, &g) == hipSuccess;
    }
    if (ok) ok = hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (cap) (void)hipStreamDestroy(cap);
    (void)hipGetLastError();
    B->graph_state = ok ? 1 : -1;
  }
  if (B->graph_state == 1) return hipGraphLaunch(B->exec, B->stream) == hipSuccess ? HFZ_OK : HFZ_EHIP;
  batch_cycle_any(B, B->stream);
  return last_error();
}

// The batched begin of a step for the instances with h_on set: source and
// iterate on each finest level, then the frozen coefficients restricted
// depth by depth (and their FP32 copies).
template <int MODEL> int batch_begin(hfz_batch* B) {
  HIPCHK(hipMemcpyAsync(B->on, B->h_on.data(), B->count * sizeof(int), hipMemcpyHostToDevice, B->stream));
  const bool mixed = B->p.precision == HFZ_MIXED;
  dim3 g, b;
  batch_top_grid(B, B->nmax, B->count, &g, &b);
  k_begin_b<MODEL><<<g, b, 0, B->stream>>>(B->L064, B->S, B->P64, B->on, mixed ? B->L032 : nullptr);
  for (int d = B->depths - 1; d >= 1; --d) {
    const int nc = B->size_at[d - 1];
    const dim3 bc = block2(nc, nc);
    const dim3 gc(grid2(nc, nc, bc).x, grid2(nc, nc, bc).y, B->cnt[d]);
    k_restrict_coef_b<<<gc, bc, 0, B->stream>>>(B->D64 + B->doff[d], B->D64 + B->doff[d - 1], B->on,
                                                 mixed ? B->D32 + B->doff[d - 1] : nullptr);
  }
  return last_error();
}

// The batched end of a step for the instances with h_on set: continuity
// update, state <- g, and for CDFT the next convolution (per instance).
template <int MODEL> int batch_finish(hfz_batch* B) {
  HIPCHK(hipMemcpyAsync(B->on, B->h_on.data(), B->count * sizeof(int), hipMemcpyHostToDevice, B->stream));
  dim3 g, b;
  batch_top_grid(B, B->nmax, B->count, &g, &b);
  if (B->p.continuity_fix) k_continuity_b<<<g, b, 0, B->stream>>>(B->L064, B->P64, B->on);
  const size_t nn = (size_t)B->nmax * B->nmax;
  k_state_b<MODEL><<<dim3((unsigned)((nn + 255) / 256), 1, B->count), 256, 0, B->stream>>>(B->L064, B->S, B->on);
  if constexpr (MODEL == CDFT) {
    for (int k = 0; k < B->count; ++k)
      if (B->h_on[k]) convolve(B->inst[k], B->inst[k]->H.L[0].rk, B->inst[k]->jrho);
  }
  return last_error();
}

int batch_write_active(hfz_batch* B) {
  HIPCHK(hipMemcpyAsync(B->active, B->h_active.data(), B->count * sizeof(int), hipMemcpyHostToDevice, B->stream));
  return HFZ_OK;
}

}  // namespace

extern "C" {

int hfz_batch_workspace_bytes(const hfz_params* params, int count, size_t* bytes) {
  if (!params || count < 1 || !bytes) return HFZ_EINVAL;
  for (int i = 0; i < count; ++i) {
    const int rc = validate(&params[i]);
    if (rc != HFZ_OK) return rc;
    // the batched solve covers the periodic hydrodynamic models
    if (model_gf(params[i].model) || params[i].walls) return HFZ_EINVAL;
    if (!batch_compatible(params[0], params[i])) return HFZ_EINVAL;
  }
  // the batched V-cycle runs the tiled kernels above the one-workgroup tail,
  // which takes the coarsest level
  if (params[0].nu1 < 1 || params[0].nu2 < 1 || params[0].coarsest_n > kTailNMax) return HFZ_EINVAL;
  *bytes = batch_geom(params, count).total;
  return HFZ_OK;
}

int hfz_batch_init(const hfz_params* params, int count, void* dev_ws, size_t ws_bytes, void* hip_stream,
                   hfz_batch** out) {
  if (!out) return HFZ_EINVAL;
  *out = nullptr;
  size_t need = 0;
  int rc = hfz_batch_workspace_bytes(params, count, &need);
  if (rc != HFZ_OK) return rc;
  if (!dev_ws || ws_bytes < need) return HFZ_ENOMEM;
  if (reinterpret_cast<uintptr_t>(dev_ws) % kAlign) return HFZ_EINVAL;
  hfz_batch* B = new (std::nothrow) hfz_batch();
  if (!B) return HFZ_ENOMEM;
  const BatchGeom G = batch_geom(params, count);
  B->count = count;
  B->p = params[G.order[0]];
  if (const char* e = std::getenv("HFZ_BATCH_TILE")) B->tile_force = std::atoi(e);
  if (const char* e = std::getenv("HFZ_BATCH_RESTRICT")) B->restrict_mode = std::max(0, std::min(3, std::atoi(e)));
  B->stream = static_cast<hipStream_t>(hip_stream);
  char* base = static_cast<char*>(dev_ws);
  B->slot_of.assign(count, 0);
  for (int k = 0; k < count; ++k) {
    const int i = G.order[k];
    hfz_handle* h = nullptr;
    rc = hfz_init(&params[i], base + G.ws_off[k], G.ws_bytes[k], hip_stream, &h);
    if (rc != HFZ_OK) {
      hfz_batch_destroy(B);
      return rc;
    }
    // the batched cycle needs every level above the tail tileable and the
    // coarsest level (<= 32, hfz_batch_workspace_bytes) in the tail
    if (h->tail_n < 16) h->tail_n = kTailNMax;
    h->tail_n = std::max(h->tail_n, params[i].coarsest_n);
    h->use_tiles = true;
    B->inst.push_back(h);
    B->slot_of[i] = k;
  }
  const int cn = B->p.coarsest_n;
  B->nmax = G.n[0];
  B->depths = G.depths;
  B->cnt = G.cnt;
  B->size_at.resize(B->depths);
  for (int d = 0; d < B->depths; ++d) B->size_at[d] = cn << d;
  B->h_top.resize(count);
  for (int k = 0; k < count; ++k) B->h_top[k] = G.nlev[k] - 1;
  B->tail_depth = ilog2(B->inst[0]->tail_n) - ilog2(cn);
  // tail launches: consecutive slots whose tails start at the same depth
  for (int k = 0; k < count; ++k) {
    const int td = std::min(B->h_top[k], B->tail_depth);
    if (B->tail_first.empty() || B->tail_top.back() != td) {
      B->tail_first.push_back(k);
      B->tail_count.push_back(0);
      B->tail_top.push_back(td);
    }
    B->tail_count.back()++;
    if (B->h_top[k] > B->tail_depth) B->tiled_count = k + 1;
  }
  Carver c{base + G.off_arrays};
  B->D64 = c.take<Lvl<double>>(G.ndesc);
  B->D32 = c.take<Lvl<float>>(G.ndesc);
  B->L064 = c.take<Lvl<double>>(count);
  B->L032 = c.take<Lvl<float>>(count);
  B->T64 = c.take<Lvl<double>>((size_t)count * TAIL_MAX_LEVELS);
  B->T32 = c.take<Lvl<float>>((size_t)count * TAIL_MAX_LEVELS);
  B->P64 = c.take<Phys<double>>(count);
  B->P32 = c.take<Phys<float>>(count);
  B->active = c.take<int>(count);
  B->norm2 = c.take<double>(count);
  int* ints = c.take<int>((size_t)count * 5);
  B->cyc = ints;
  B->stat = ints + count;
  B->maxc = ints + 2 * count;
  B->topd = ints + 3 * count;
  B->npart = ints + 4 * count;
  B->tol = c.take<double>(count);
  B->S = c.take<StateB>(count);
  B->on = c.take<int>(count);
  B->h_on.assign(count, 0);
  B->pstride = G.pstride;
  B->partial = c.take<double>((size_t)B->pstride * count);
  const bool mixed = B->p.precision == HFZ_MIXED;
  std::vector<Lvl<double>> d64(G.ndesc), t64((size_t)count * TAIL_MAX_LEVELS), l064(count);
  std::vector<Lvl<float>> d32(G.ndesc), t32((size_t)count * TAIL_MAX_LEVELS), l032(count);
  std::vector<Phys<double>> p64(count);
  std::vector<Phys<float>> p32(count);
  B->doff.assign(B->depths, 0);
  for (int d = 1; d < B->depths; ++d) B->doff[d] = B->doff[d - 1] + B->cnt[d - 1];
  for (int k = 0; k < count; ++k) {
    hfz_handle* h = B->inst[k];
    const int top = B->h_top[k];
    for (int l = 0; l <= top; ++l) {
      const int d = top - l;  // level l of this instance sits at depth d
      d64[B->doff[d] + k] = h->H.L[l];
      if (mixed) d32[B->doff[d] + k] = h->H32.L[l];
    }
    const int td = std::min(top, B->tail_depth);
    for (int j = 0; j <= td; ++j) {
      t64[(size_t)k * TAIL_MAX_LEVELS + j] = h->H.L[top - td + j];
      if (mixed) t32[(size_t)k * TAIL_MAX_LEVELS + j] = h->H32.L[top - td + j];
    }
    l064[k] = h->H.L[0];
    if (mixed) l032[k] = h->H32.L[0];
    p64[k] = h->H.P;
    p32[k] = h->H32.P;
  }
  if (B->p.model == HFZ_PFC) {
    B->lds64 = lds_optin(reinterpret_cast<const void*>(&k_tail_b<PFC, double, false>));
    B->lds32 = lds_optin(reinterpret_cast<const void*>(&k_tail_b<PFC, float, true>));
  } else {
    B->lds64 = lds_optin(reinterpret_cast<const void*>(&k_tail_b<CDFT, double, false>));
    B->lds32 = lds_optin(reinterpret_cast<const void*>(&k_tail_b<CDFT, float, true>));
  }
  // every tail launch must hold its levels in LDS (the tiled path has no
  // coarsest-level smoother)
  for (size_t t = 0; t < B->tail_first.size(); ++t) {
    const int td = B->tail_top[t], nt = td + 1, top_n = B->size_at[td];
    const bool held =
        nt <= TAIL_MAX_LEVELS &&
        (B->p.model == HFZ_PFC
             ? (mixed ? tail_plan<PFC, float, true>(top_n, nt, B->lds32, nullptr)
                      : tail_plan<PFC, double, false>(top_n, nt, B->lds64, nullptr))
             : (mixed ? tail_plan<CDFT, float, true>(top_n, nt, B->lds32, nullptr)
                      : tail_plan<CDFT, double, false>(top_n, nt, B->lds64, nullptr)));
    if (!held) {
      hfz_batch_destroy(B);
      return HFZ_EINVAL;
    }
  }
  // stop-test partial sums per instance: the tiles of its finest level's
  // post-sweep launch, or the blocks of the tail-only instances' residual pass
  std::vector<int> tops(count), nparts(count);
  {
    const int first = B->tiled_count;
    dim3 gt(1, 1, 1), bt;
    if (first < count) batch_top_grid(B, B->inst[first]->p.n, count - first, &gt, &bt);
    for (int k = 0; k < count; ++k) {
      const int n = B->inst[k]->p.n;
      tops[k] = B->h_top[k];
      if (k < first) {
        const int ts = batch_tile_shape(n, B->tile_force);
        nparts[k] = (n / kTileShapes[ts].tx) * (n / kTileShapes[ts].ty);
      } else {
        nparts[k] = (int)(gt.x * gt.y);
      }
    }
  }
  B->h_active.assign(count, 1);
  B->h_norm2.assign(count, 0.0);
  bool ok = hipMemcpyAsync(B->D64, d64.data(), d64.size() * sizeof(Lvl<double>), hipMemcpyHostToDevice,
                           B->stream) == hipSuccess;
  ok = ok && hipMemcpyAsync(B->T64, t64.data(), t64.size() * sizeof(Lvl<double>), hipMemcpyHostToDevice,
                            B->stream) == hipSuccess;
  ok = ok && hipMemcpyAsync(B->L064, l064.data(), l064.size() * sizeof(Lvl<double>), hipMemcpyHostToDevice,
                            B->stream) == hipSuccess;
  if (mixed) {
    ok = ok && hipMemcpyAsync(B->D32, d32.data(), d32.size() * sizeof(Lvl<float>), hipMemcpyHostToDevice,
                              B->stream) == hipSuccess;
    ok = ok && hipMemcpyAsync(B->T32, t32.data(), t32.size() * sizeof(Lvl<float>), hipMemcpyHostToDevice,
                              B->stream) == hipSuccess;
    ok = ok && hipMemcpyAsync(B->L032, l032.data(), l032.size() * sizeof(Lvl<float>), hipMemcpyHostToDevice,
                              B->stream) == hipSuccess;
  }
  ok = ok && hipMemcpyAsync(B->P64, p64.data(), count * sizeof(Phys<double>), hipMemcpyHostToDevice, B->stream) ==
                 hipSuccess;
  ok = ok && hipMemcpyAsync(B->P32, p32.data(), count * sizeof(Phys<float>), hipMemcpyHostToDevice, B->stream) ==
                 hipSuccess;
  std::vector<StateB> sts(count);
  std::vector<double> tols(count);
  std::vector<int> maxcs(count);
  for (int k = 0; k < count; ++k) {
    hfz_handle* h = B->inst[k];
    sts[k] = StateB{h->u, h->v, h->mu, h->ka, h->jrho};
    tols[k] = h->p.tol;
    maxcs[k] = h->p.max_cycles;
  }
  ok = ok && hipMemcpyAsync(B->S, sts.data(), count * sizeof(StateB), hipMemcpyHostToDevice, B->stream) ==
                 hipSuccess;
  ok = ok && hipMemcpyAsync(B->tol, tols.data(), count * sizeof(double), hipMemcpyHostToDevice, B->stream) ==
                 hipSuccess;
  ok = ok && hipMemcpyAsync(B->maxc, maxcs.data(), count * sizeof(int), hipMemcpyHostToDevice, B->stream) ==
                 hipSuccess;
  ok = ok && hipMemcpyAsync(B->topd, tops.data(), count * sizeof(int), hipMemcpyHostToDevice, B->stream) ==
                 hipSuccess;
  ok = ok && hipMemcpyAsync(B->npart, nparts.data(), count * sizeof(int), hipMemcpyHostToDevice, B->stream) ==
                 hipSuccess;
  ok = ok && hipStreamSynchronize(B->stream) == hipSuccess;
  if (!ok) {
    hfz_batch_destroy(B);
    return HFZ_EHIP;
  }
  if (const char* e = std::getenv("HFZ_GRAPH")) B->use_graph = std::atoi(e) != 0;
  *out = B;
  return HFZ_OK;
}

int hfz_batch_set_state(hfz_batch* B, int i, const double* rho, const double* u, const double* v) {
  if (!B || i < 0 || i >= B->count) return HFZ_EINVAL;
  return hfz_set_state(B->inst[B->slot_of[i]], rho, u, v);
}

int hfz_batch_get_state(hfz_batch* B, int i, double* rho, double* u, double* v) {
  if (!B || i < 0 || i >= B->count) return HFZ_EINVAL;
  return hfz_get_state(B->inst[B->slot_of[i]], rho, u, v);
}

int hfz_batch_energy(hfz_batch* B, int i, double* out5) {
  if (!B || i < 0 || i >= B->count) return HFZ_EINVAL;
  return hfz_energy(B->inst[B->slot_of[i]], out5);
}

int hfz_batch_release(hfz_batch* B, int i) {
  if (!B || i < 0 || i >= B->count) return HFZ_EINVAL;
  B->inst[B->slot_of[i]]->has_state = false;
  return HFZ_OK;
}

int hfz_batch_step(hfz_batch* B, int nsteps, hfz_stats* stats) {
  if (!B || nsteps < 0) return HFZ_EINVAL;
  const int count = B->count;
  std::vector<char> filled(count);  // by slot
  int nfilled = 0;
  for (int k = 0; k < count; ++k) nfilled += filled[k] = B->inst[k]->has_state ? 1 : 0;
  if (stats)
    for (int i = 0; i < count; ++i) stats[i] = hfz_stats{};
  if (nfilled == 0) return HFZ_OK;
  std::vector<hfz_stats> st(count);  // by slot
  std::vector<int> h_cyc(count), h_stat(count);
  int rc = HFZ_OK;
  for (int s = 0; s < nsteps && rc == HFZ_OK; ++s) {
    for (int k = 0; k < count; ++k) B->h_on[k] = filled[k];
    rc = B->p.model == HFZ_PFC ? batch_begin<PFC>(B) : batch_begin<CDFT>(B);
    if (rc != HFZ_OK) break;
    // every instance runs until its own stop test ends it (on the device);
    // the host enqueues cycles in batches and reads the states once a batch
    for (int k = 0; k < count; ++k) B->h_active[k] = filled[k];
    rc = batch_write_active(B);
    if (rc != HFZ_OK) break;
    k_zero_ints<<<(2 * count + 255) / 256, 256, 0, B->stream>>>(B->cyc, 2 * count);
    if (B->p.model == HFZ_PFC)
      batch_first_norm<PFC>(B);
    else
      batch_first_norm<CDFT>(B);
    int batch = std::max(1, B->cycle_hint);
    for (;;) {
      for (int c = 0; c < batch && rc == HFZ_OK; ++c) rc = batch_launch_cycle(B);
      if (rc != HFZ_OK) break;
      if (hipMemcpyAsync(h_cyc.data(), B->cyc, count * sizeof(int), hipMemcpyDeviceToHost, B->stream) != hipSuccess ||
          hipMemcpyAsync(h_stat.data(), B->stat, count * sizeof(int), hipMemcpyDeviceToHost, B->stream) !=
              hipSuccess ||
          hipMemcpyAsync(B->h_norm2.data(), B->norm2, count * sizeof(double), hipMemcpyDeviceToHost, B->stream) !=
              hipSuccess ||
          hipStreamSynchronize(B->stream) != hipSuccess) {
        rc = HFZ_EHIP;
        break;
      }
      bool running = false;
      for (int k = 0; k < count; ++k) running = running || (filled[k] && h_stat[k] == 0);
      if (!running) break;
      batch = 2;
    }
    if (rc != HFZ_OK) break;
    int most = 0;
    std::vector<int> failed(count, 0);
    for (int k = 0; k < count; ++k) {
      if (!filled[k]) continue;
      st[k].cycles_last = h_cyc[k];
      st[k].residual_last = std::sqrt(B->h_norm2[k]);
      failed[k] = h_stat[k] == 2 ? HFZ_ENAN : h_stat[k] == 3 ? HFZ_ENOCONV : 0;
      most = std::max(most, h_cyc[k]);
    }
    B->cycle_hint = most;
    // failed instances are rolled back: their state stays that of the previous step
    for (int k = 0; k < count; ++k) B->h_on[k] = filled[k] && !failed[k];
    rc = B->p.model == HFZ_PFC ? batch_finish<PFC>(B) : batch_finish<CDFT>(B);
    if (rc != HFZ_OK) break;
    for (int k = 0; k < count; ++k) {
      if (!B->h_on[k]) continue;
      st[k].steps_done++;
      st[k].cycles_total += h_cyc[k];
    }
    for (int k = 0; k < count; ++k)
      if (failed[k] && rc == HFZ_OK) rc = failed[k];
  }
  if (rc == HFZ_OK && hipStreamSynchronize(B->stream) != hipSuccess) rc = HFZ_EHIP;
  if (stats)
    for (int i = 0; i < count; ++i) stats[i] = st[B->slot_of[i]];
  return rc;
}

int hfz_batch_destroy(hfz_batch* B) {
  if (!B) return HFZ_EINVAL;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  for (auto* h : B->inst) hfz_destroy(h);
  delete B;
  return HFZ_OK;
}

}  // extern "C"
