// Batched solves: a problem table on the device, one persistent launch that
// pulls (problem, block-of-points) tiles from an atomic counter, captured as a
// hipGraph, and an autotuner for the launch shape.
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <functional>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace wobi;

struct wob_batch_s {
  int32_t dim = 0, precision = 0, device = 0;
  std::vector<wob_problem> probs;  // caller's problems
  std::vector<int32_t> order;      // execution order: decreasing cost per tile
  wob_tune tune{256, 4};
  int32_t n_cu = 0;
  void* d_args = nullptr;
  int64_t* d_tile_off = nullptr;
  unsigned long long* d_counter = nullptr;
  int64_t n_tiles = 0;
  int32_t stack_cap = 1;  // largest traversal stack of the problems' scenes
  int32_t max_lds = 0;    // LDS bytes a workgroup may use on the device
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string signature;
};

namespace {

// Resets the tile counter inside the captured graph (a kernel node rather than
// a memset node).
__global__ void zero_counter(unsigned long long* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0ull;
}

// Whether a workgroup of `block` threads fits the device's LDS with the
// traversal stacks of the deepest scene (and the kernel's small static LDS).
bool fits_lds(const wob_batch_s* b, int block) {
  return wob::walk_lds_bytes(b->stack_cap, block) + 1024 <= (size_t)b->max_lds;
}

bool valid_tune(const wob_tune& t) {
  return (t.block == 128 || t.block == 256 || t.block == 512) && t.blocks_per_cu >= 1 &&
         t.blocks_per_cu <= 16;
}

// Problem table for one block size (lanes per point and tiles depend on it).
template <typename R, int D>
wob_status upload_table(wob_batch_s* b, int block) {
  const int n = (int)b->probs.size();
  std::vector<wob::WalkArgs<R, D>> args(n);
  std::vector<int64_t> off(n + 1, 0);
  b->stack_cap = 1;
  for (int i = 0; i < n; ++i) {
    const wob_problem& p = b->probs[b->order[i]];
    Plan pl;
    if (plan_walk(p.scene, &p.bc, p.samples, p.walk_len, &pl) != WOB_OK) return WOB_E_ARG;
    b->stack_cap = std::max(b->stack_cap, p.scene->stack_cap);
    auto a = make_args<R, D>(p.scene, pl, p.points, p.point_prim, p.n_points, &p.bc, p.samples,
                             p.walk_len, p.seed);
    a.problem = p.stream_id;
    a.lpp_shift = lpp_shift_for(p.samples, block);
    a.mean_out = (R*)p.mean_out;
    a.var_out = (R*)p.var_out;
    args[i] = a;
    const int64_t ppt = block >> a.lpp_shift;
    off[i + 1] = off[i] + (p.n_points + ppt - 1) / ppt;
  }
  if (!b->d_args && hipMalloc(&b->d_args, sizeof(wob::WalkArgs<R, D>) * n) != hipSuccess)
    return WOB_E_ALLOC;
  if (!b->d_tile_off && hipMalloc((void**)&b->d_tile_off, sizeof(int64_t) * (n + 1)) != hipSuccess)
    return WOB_E_ALLOC;
  if (hipMemcpy(b->d_args, args.data(), sizeof(wob::WalkArgs<R, D>) * n, hipMemcpyHostToDevice) !=
      hipSuccess)
    return WOB_E_DEVICE;
  if (hipMemcpy(b->d_tile_off, off.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice) !=
      hipSuccess)
    return WOB_E_DEVICE;
  b->n_tiles = off[n];
  return WOB_OK;
}

wob_status upload(wob_batch_s* b, int block) {
  if (b->precision == WOB_F32)
    return b->dim == 3 ? upload_table<float, 3>(b, block) : upload_table<float, 2>(b, block);
  return b->dim == 3 ? upload_table<double, 3>(b, block) : upload_table<double, 2>(b, block);
}

template <typename R, int D, int BLOCK>
void launch_persistent_t(wob_batch_s* b, int bpc, int64_t stride, hipStream_t st) {
  hipLaunchKernelGGL(zero_counter, dim3(1), dim3(64), 0, st, b->d_counter);
  const dim3 grid((unsigned)(b->n_cu * bpc)), block(BLOCK);
  hipLaunchKernelGGL((wob::batch_kernel<R, D, BLOCK>), grid, block,
                     wob::walk_lds_bytes(b->stack_cap, BLOCK), st,
                     (const wob::WalkArgs<R, D>*)b->d_args, (const int64_t*)b->d_tile_off,
                     (int32_t)b->probs.size(), stride, b->d_counter);
}

template <typename R, int D>
void launch_persistent_rd(wob_batch_s* b, const wob_tune& t, int64_t stride, hipStream_t st) {
  if (t.block == 128) launch_persistent_t<R, D, 128>(b, t.blocks_per_cu, stride, st);
  else if (t.block == 256) launch_persistent_t<R, D, 256>(b, t.blocks_per_cu, stride, st);
  else launch_persistent_t<R, D, 512>(b, t.blocks_per_cu, stride, st);
}

void launch_persistent(wob_batch_s* b, const wob_tune& t, int64_t stride, hipStream_t st) {
  if (b->precision == WOB_F32) {
    if (b->dim == 3) launch_persistent_rd<float, 3>(b, t, stride, st);
    else launch_persistent_rd<float, 2>(b, t, stride, st);
  } else {
    if (b->dim == 3) launch_persistent_rd<double, 3>(b, t, stride, st);
    else launch_persistent_rd<double, 2>(b, t, stride, st);
  }
}

void drop_graph(wob_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Capture {zero the tile counter (a kernel, not a memset node), persistent solve}.
wob_status capture(wob_batch_s* b) {
  drop_graph(b);
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return WOB_E_DEVICE;
  launch_persistent(b, b->tune, 1, b->cap);
  if (hipStreamEndCapture(b->cap, &b->graph) != hipSuccess) return WOB_E_DEVICE;
  if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return WOB_E_DEVICE;
  return WOB_OK;
}

std::string signature(const wob_batch_s* b) {
  std::ostringstream s;
  s << "d" << b->dim << "p" << b->precision << "n" << b->probs.size() << "cu" << b->n_cu;
  for (const auto& p : b->probs) {
    Plan pl;
    plan_walk(p.scene, &p.bc, p.samples, p.walk_len, &pl);
    s << ":" << p.n_points << "," << p.samples << "," << pl.L << "," << pl.form << ","
      << p.scene->n_prims;
  }
  char hex[32];
  std::snprintf(hex, sizeof(hex), "%016zx", std::hash<std::string>()(s.str()));
  return std::string(hex);
}

void destroy(wob_batch_s* b) {
  if (!b) return;
  drop_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->d_args) (void)hipFree(b->d_args);
  if (b->d_tile_off) (void)hipFree(b->d_tile_off);
  if (b->d_counter) (void)hipFree(b->d_counter);
  delete b;
}

}  // namespace

extern "C" {

wob_status wob_batch_create(const wob_problem* problems, int32_t n, const wob_tune* tune,
                            wob_batch* out) {
  if (!out) return WOB_E_ARG;
  *out = nullptr;
  if (!problems || n <= 0) return WOB_E_ARG;
  if (tune && !valid_tune(*tune)) return WOB_E_ARG;
  const wob_scene_s* s0 = problems[0].scene;
  if (!s0) return WOB_E_ARG;
  std::vector<double> cost(n);
  for (int i = 0; i < n; ++i) {
    const wob_problem& p = problems[i];
    if (!p.scene || p.scene->dim != s0->dim || p.scene->precision != s0->precision ||
        p.scene->device != s0->device)
      return WOB_E_ARG;
    Plan pl;
    const wob_status st = plan_walk(p.scene, &p.bc, p.samples, p.walk_len, &pl);
    if (st != WOB_OK) return st;
    if (p.samples < 2 && p.var_out) return WOB_E_ARG;
    if (p.n_points < 0 || p.n_points >= ((int64_t)1 << 32)) return WOB_E_ARG;
    if (p.n_points > 0 && (!p.points || !p.mean_out)) return WOB_E_ARG;
    if (p.stream_id >= 256 || p.reserved != 0) return WOB_E_ARG;
    // relative cost of one tile: paths x lines x log2(primitives)
    cost[i] = (double)p.samples * pl.L * std::log2(2.0 + (double)p.scene->n_prims);
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != s0->device) return WOB_E_DEVICE;
  wob_batch_s* b = new (std::nothrow) wob_batch_s();
  if (!b) return WOB_E_ALLOC;
  b->dim = s0->dim;
  b->precision = s0->precision;
  b->device = dev;
  b->probs.assign(problems, problems + n);
  b->order.resize(n);
  for (int i = 0; i < n; ++i) b->order[i] = i;
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int x, int y) { return cost[x] > cost[y]; });
  if (tune) b->tune = *tune;
  if (hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      b->n_cu <= 0 ||
      hipDeviceGetAttribute(&b->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    destroy(b);
    return WOB_E_DEVICE;
  }
  if (hipMalloc((void**)&b->d_counter, sizeof(unsigned long long)) != hipSuccess) {
    destroy(b);
    return WOB_E_ALLOC;
  }
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    destroy(b);
    return WOB_E_DEVICE;
  }
  wob_status st = upload(b, b->tune.block);
  if (st == WOB_OK && !fits_lds(b, b->tune.block)) {
    // very deep trees: a caller's shape that does not fit is an error; the
    // default falls back to the smallest workgroup
    if (tune) st = WOB_E_ARG;
    else {
      b->tune = wob_tune{128, 8};
      st = upload(b, b->tune.block);
      if (st == WOB_OK && !fits_lds(b, b->tune.block)) st = WOB_E_ARG;
    }
  }
  if (st == WOB_OK) st = capture(b);
  if (st != WOB_OK) {
    destroy(b);
    return st;
  }
  b->signature = signature(b);
  *out = b;
  return WOB_OK;
}

wob_status wob_batch_launch(wob_batch b, void* stream) {
  if (!b || !b->exec) return WOB_E_ARG;
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

wob_status wob_batch_get_tune(wob_batch b, wob_tune* tune, int64_t* n_tiles) {
  if (!b) return WOB_E_ARG;
  if (tune) *tune = b->tune;
  if (n_tiles) *n_tiles = b->n_tiles;
  return WOB_OK;
}

wob_status wob_batch_autotune(wob_batch b, int32_t sample_stride, const char* cache_path,
                              wob_tune* chosen, void* stream) {
  if (!b || sample_stride < 1) return WOB_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  wob_tune best = b->tune;
  bool have = false;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string key;
    wob_tune t;
    while (in >> key >> t.block >> t.blocks_per_cu) {
      if (key == b->signature && valid_tune(t) && fits_lds(b, t.block)) {
        best = t;
        have = true;
      }
    }
  }
  if (!have) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return WOB_E_DEVICE;
    float best_ms = 1e30f;
    const int blocks[3] = {128, 256, 512};
    const int bpcs[6] = {1, 2, 3, 4, 6, 8};
    for (int bi = 0; bi < 3; ++bi) {
      // the table is rewritten synchronously: wait for the kernels that read it
      if (hipStreamSynchronize(st) != hipSuccess) return WOB_E_DEVICE;
      if (upload(b, blocks[bi]) != WOB_OK) return WOB_E_DEVICE;
      if (!fits_lds(b, blocks[bi])) continue;
      for (int ci = 0; ci < 6; ++ci) {
        const wob_tune t{blocks[bi], bpcs[ci]};
        if (t.blocks_per_cu * t.block / 64 > 24) continue;  // beyond what a CU can hold
        launch_persistent(b, t, sample_stride, st);  // warm-up
        (void)hipEventRecord(e0, st);
        launch_persistent(b, t, sample_stride, st);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) return WOB_E_DEVICE;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (hipGetLastError() != hipSuccess) return WOB_E_DEVICE;
    if (cache_path) {
      std::ofstream o(cache_path, std::ios::app);
      o << b->signature << " " << best.block << " " << best.blocks_per_cu << "\n";
    }
  }
  b->tune = best;
  if (hipStreamSynchronize(st) != hipSuccess) return WOB_E_DEVICE;
  wob_status s = upload(b, best.block);
  if (s == WOB_OK) s = capture(b);
  if (s == WOB_OK && chosen) *chosen = best;
  return s;
}

void wob_batch_free(wob_batch b) { destroy(b); }

wob_status wob_solve_batched(const wob_problem* problems, int32_t n, const wob_tune* tune,
                             void* stream) {
  wob_batch b = nullptr;
  wob_status s = wob_batch_create(problems, n, tune, &b);
  if (s != WOB_OK) return s;
  s = wob_batch_launch(b, stream);
  if (s == WOB_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) s = WOB_E_DEVICE;
  wob_batch_free(b);
  return s;
}

}  // extern "C"
