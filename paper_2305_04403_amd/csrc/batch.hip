// Batched solves: a problem table on the device, one persistent launch that
// pulls (problem, block-of-points) tiles from an atomic counter, captured as a
// hipGraph, and an autotuner for the launch shape.
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <functional>
#include <mutex>
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
bool fits_lds_cap(int32_t stack_cap, int32_t max_lds, int block) {
  return wob::walk_lds_bytes(stack_cap, block) + 1024 <= (size_t)max_lds;
}
bool fits_lds(const wob_batch_s* b, int block) { return fits_lds_cap(b->stack_cap, b->max_lds, block); }

bool valid_tune(const wob_tune& t) {
  return (t.block == 64 || t.block == 128 || t.block == 256 || t.block == 512) && t.blocks_per_cu >= 1 &&
         t.blocks_per_cu <= 32;
}

// Whether any problem gives its boundary data per vertex (then the batch runs
// the kernel instantiated for it).
inline bool any_vertex_data(const wob_problem* p, int32_t n) {
  for (int32_t i = 0; i < n; ++i)
    if (p[i].bc.data_mode == WOB_DATA_VERTEX) return true;
  return false;
}

// Problem table for one block size (lanes per point and tiles depend on it):
// the walk arguments of problem order[i] at args[i], tile offsets off[0..n],
// and the deepest traversal stack of the problems' scenes.
template <typename R, int D>
wob_status fill_table(const wob_problem* probs, const int32_t* order, int n, int block,
                      wob::WalkArgs<R, D>* args, int64_t* off, int32_t* stack_cap) {
  off[0] = 0;
  *stack_cap = 1;
  const bool vdata = any_vertex_data(probs, n);
  for (int i = 0; i < n; ++i) {
    const wob_problem& p = probs[order[i]];
    Plan pl;
    if (plan_walk(p.scene, &p.bc, p.samples, p.walk_len, &pl) != WOB_OK) return WOB_E_ARG;
    *stack_cap = std::max(*stack_cap, p.scene->stack_cap);
    auto a = make_args<R, D>(p.scene, pl, p.points, p.point_prim, p.n_points, &p.bc, p.samples,
                             p.walk_len, p.seed);
    a.problem = p.stream_id;
    // the kernel runs the X_VDATA instantiation for every problem when one
    // gives its data per vertex; the plain single-layer forms pool two points
    // per lane group in the other (the same rule as the kernel's)
    a.lpp_shift = lpp_shift_for(p.samples, block,
                                wob::pools_points(a.form, vdata ? wob::X_VDATA : wob::X_NONE, false, false));
    a.mean_out = (R*)p.mean_out;
    a.var_out = (R*)p.var_out;
    args[i] = a;
    const int64_t ppt = block >> a.lpp_shift;
    off[i + 1] = off[i] + (p.n_points + ppt - 1) / ppt;
  }
  return WOB_OK;
}

template <typename R, int D>
wob_status upload_table(wob_batch_s* b, int block) {
  const int n = (int)b->probs.size();
  std::vector<wob::WalkArgs<R, D>> args(n);
  std::vector<int64_t> off(n + 1, 0);
  const wob_status fs = fill_table<R, D>(b->probs.data(), b->order.data(), n, block, args.data(), off.data(),
                                         &b->stack_cap);
  if (fs != WOB_OK) return fs;
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

// Where a persistent launch finds its table and counter, and its shape.
struct LaunchBufs {
  const void* args;
  const int64_t* tile_off;
  unsigned long long* counter;
  int32_t n_probs, stack_cap, n_cu;
  bool vdata;  // some problem gives its boundary data per vertex
};


template <typename R, int D, int BLOCK>
void launch_persistent_t(const LaunchBufs& lb, int bpc, int64_t stride, hipStream_t st) {
  hipLaunchKernelGGL(zero_counter, dim3(1), dim3(64), 0, st, lb.counter);
  const dim3 grid((unsigned)(lb.n_cu * bpc)), block(BLOCK);
  const size_t lds = wob::walk_lds_bytes(lb.stack_cap, BLOCK);
  const auto* args = (const wob::WalkArgs<R, D>*)lb.args;
  if (lb.vdata)
    hipLaunchKernelGGL((wob::batch_kernel<R, D, BLOCK, wob::X_VDATA>), grid, block, lds, st, args, lb.tile_off,
                       lb.n_probs, stride, lb.counter);
  else
    hipLaunchKernelGGL((wob::batch_kernel<R, D, BLOCK>), grid, block, lds, st, args, lb.tile_off, lb.n_probs,
                       stride, lb.counter);
}

template <typename R, int D>
void launch_persistent_rd(const LaunchBufs& lb, const wob_tune& t, int64_t stride, hipStream_t st) {
  if (t.block == 64) launch_persistent_t<R, D, 64>(lb, t.blocks_per_cu, stride, st);
  else if (t.block == 128) launch_persistent_t<R, D, 128>(lb, t.blocks_per_cu, stride, st);
  else if (t.block == 256) launch_persistent_t<R, D, 256>(lb, t.blocks_per_cu, stride, st);
  else launch_persistent_t<R, D, 512>(lb, t.blocks_per_cu, stride, st);
}

void launch_persistent_buf(int precision, int dim, const LaunchBufs& lb, const wob_tune& t, int64_t stride,
                           hipStream_t st) {
  if (precision == WOB_F32) {
    if (dim == 3) launch_persistent_rd<float, 3>(lb, t, stride, st);
    else launch_persistent_rd<float, 2>(lb, t, stride, st);
  } else {
    if (dim == 3) launch_persistent_rd<double, 3>(lb, t, stride, st);
    else launch_persistent_rd<double, 2>(lb, t, stride, st);
  }
}

void launch_persistent(wob_batch_s* b, const wob_tune& t, int64_t stride, hipStream_t st) {
  const LaunchBufs lb{b->d_args, b->d_tile_off, b->d_counter, (int32_t)b->probs.size(), b->stack_cap, b->n_cu,
                      any_vertex_data(b->probs.data(), (int32_t)b->probs.size())};
  launch_persistent_buf(b->precision, b->dim, lb, t, stride, st);
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

// Checks every problem against the first one's scene kind and its own plan;
// cost[i] = the relative cost of one of its tiles (paths x lines x
// log2(primitives)).
wob_status check_problems(const wob_problem* problems, int32_t n, double* cost) {
  const wob_scene_s* s0 = problems[0].scene;
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
    cost[i] = (double)p.samples * pl.L * std::log2(2.0 + (double)p.scene->n_prims);
  }
  return WOB_OK;
}

// Execution order: problems by decreasing cost per tile (stable).
void cost_order(const double* cost, int32_t n, int32_t* order) {
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order, order + n, [&](int x, int y) { return cost[x] > cost[y]; });
}

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free batched solve: the problem table, the
// tile offsets and the tile counter, in one file-scope array per device (every
// device the library runs on holds it until the process ends).  Host code uses
// the address hipGetSymbolAddress returns for the current device, never the
// array's name (a host-side stand-in).
constexpr size_t kStaticArgsBytes =
    (std::max(std::max(sizeof(wob::WalkArgs<float, 3>), sizeof(wob::WalkArgs<float, 2>)),
              std::max(sizeof(wob::WalkArgs<double, 3>), sizeof(wob::WalkArgs<double, 2>))) *
         WOB_STATIC_MAX_PROBLEMS + 255) / 256 * 256;
constexpr size_t kStaticOffBytes = (sizeof(int64_t) * (WOB_STATIC_MAX_PROBLEMS + 1) + 255) / 256 * 256;
constexpr size_t kStaticBytes = kStaticArgsBytes + kStaticOffBytes + 256;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;

// The scratch array's device address on device `dev` (the current device),
// looked up once per device.
wob_status scratch_address(int dev, unsigned char** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) return WOB_E_DEVICE;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return WOB_E_DEVICE;
    addr[dev] = p;
  }
  *out = (unsigned char*)addr[dev];
  return WOB_OK;
}

template <typename R, int D>
wob_status solve_static(const wob_problem* problems, int32_t n, const int32_t* order, const wob_tune* given,
                        int32_t n_cu, int32_t max_lds, unsigned char* base, hipStream_t st) {
  // the table is staged in host memory the call owns until it returns (the
  // call waits for the stream, like wob_solve_batched)
  wob::WalkArgs<R, D> args[WOB_STATIC_MAX_PROBLEMS];
  int64_t off[WOB_STATIC_MAX_PROBLEMS + 1];
  int32_t stack_cap = 1;
  wob_tune tune = given ? *given : wob_tune{256, 4};
  wob_status s = fill_table<R, D>(problems, order, n, tune.block, args, off, &stack_cap);
  if (s != WOB_OK) return s;
  if (!fits_lds_cap(stack_cap, max_lds, tune.block)) {
    // as wob_batch_create: the default shape falls back to the smallest workgroup
    if (given) return WOB_E_ARG;
    tune = wob_tune{128, 8};
    s = fill_table<R, D>(problems, order, n, tune.block, args, off, &stack_cap);
    if (s != WOB_OK) return s;
    if (!fits_lds_cap(stack_cap, max_lds, tune.block)) return WOB_E_ARG;
  }
  int64_t* d_off = (int64_t*)(base + kStaticArgsBytes);
  unsigned long long* d_counter = (unsigned long long*)(base + kStaticArgsBytes + kStaticOffBytes);
  if (hipMemcpyAsync(base, args, sizeof(wob::WalkArgs<R, D>) * n, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(d_off, off, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st) != hipSuccess)
    return WOB_E_DEVICE;
  const LaunchBufs lb{base, d_off, d_counter, n, stack_cap, n_cu, any_vertex_data(problems, n)};
  launch_persistent_buf(sizeof(R) == 4 ? WOB_F32 : WOB_F64, D, lb, tune, 1, st);
  if (hipGetLastError() != hipSuccess) return WOB_E_DEVICE;
  return hipStreamSynchronize(st) == hipSuccess ? WOB_OK : WOB_E_DEVICE;
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
  const wob_status vs = check_problems(problems, n, cost.data());
  if (vs != WOB_OK) return vs;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != s0->device) return WOB_E_DEVICE;
  wob_batch_s* b = new (std::nothrow) wob_batch_s();
  if (!b) return WOB_E_ALLOC;
  b->dim = s0->dim;
  b->precision = s0->precision;
  b->device = dev;
  b->probs.assign(problems, problems + n);
  b->order.resize(n);
  cost_order(cost.data(), n, b->order.data());
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
    const int blocks[4] = {64, 128, 256, 512};
    // resident wavefronts per CU to try (4 SIMDs)
    const int waves[6] = {4, 8, 12, 16, 20, 24};
    for (int bi = 0; bi < 4; ++bi) {
      // the table is rewritten synchronously: wait for the kernels that read it
      if (hipStreamSynchronize(st) != hipSuccess) return WOB_E_DEVICE;
      if (upload(b, blocks[bi]) != WOB_OK) return WOB_E_DEVICE;
      if (!fits_lds(b, blocks[bi])) continue;
      for (int ci = 0; ci < 6; ++ci) {
        const int per_block = blocks[bi] / 64;
        if (waves[ci] % per_block != 0) continue;
        const wob_tune t{blocks[bi], waves[ci] / per_block};
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

wob_status wob_solve_batched_static(const wob_problem* problems, int32_t n, const wob_tune* tune,
                                    void* stream) {
  if (!problems || n <= 0) return WOB_E_ARG;
  if (n > WOB_STATIC_MAX_PROBLEMS) return WOB_E_TOO_LARGE;
  if (tune && !valid_tune(*tune)) return WOB_E_ARG;
  const wob_scene_s* s0 = problems[0].scene;
  if (!s0) return WOB_E_ARG;
  double cost[WOB_STATIC_MAX_PROBLEMS];
  int32_t order[WOB_STATIC_MAX_PROBLEMS];
  const wob_status vs = check_problems(problems, n, cost);
  if (vs != WOB_OK) return vs;
  cost_order(cost, n, order);
  int dev = 0, n_cu = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev != s0->device) return WOB_E_DEVICE;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0 ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return WOB_E_DEVICE;
  unsigned char* base = nullptr;
  const wob_status as = scratch_address(dev, &base);
  if (as != WOB_OK) return as;
  hipStream_t st = (hipStream_t)stream;
  if (s0->precision == WOB_F32)
    return s0->dim == 3 ? solve_static<float, 3>(problems, n, order, tune, n_cu, max_lds, base, st)
                        : solve_static<float, 2>(problems, n, order, tune, n_cu, max_lds, base, st);
  return s0->dim == 3 ? solve_static<double, 3>(problems, n, order, tune, n_cu, max_lds, base, st)
                      : solve_static<double, 2>(problems, n, order, tune, n_cu, max_lds, base, st);
}

}  // extern "C"
