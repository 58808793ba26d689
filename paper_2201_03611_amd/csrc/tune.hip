// Autotuner and tune cache of the one-problem GEMM and stencil.
//
// The paper keeps every implementation choice (tile sizes from splitJoinMap,
// which map runs on workgroups, where reduceSeq accumulates) outside the
// program, in a strategy chosen by a user or a search (Sec. IV-B/C).  Here the
// choice is the tile of rise_gemm and the schedule of rise_stencil2d; the
// tuner times every supported candidate on the current device and records the
// fastest in a text cache keyed by (sizes, mode, GPU architecture).  Calls that
// leave the choice to the library (tile / sched = NULL) consult the cache
// named by rise_set_tune_cache() or, if none was set, by the RISE_TUNE_CACHE
// environment variable; without an entry they take the built-in default.
//
// Cache lines (one per key, later lines win):
//   gemm <arch> <M> <N> <K> <mode> <bm> <bn> <bk> <microseconds>
//   stencil <arch> <H> <W> <k> <variant> <rows> <microseconds>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "tune.h"

namespace rise {
namespace {

struct GemmEntry {
  std::string arch;
  int64_t M, N, K;
  int mode;
  rise_tile tile;
  double us;
};
struct StencilEntry {
  std::string arch;
  int64_t H, W;
  int k;
  rise_stencil_schedule sched;
  double us;
};

struct Cache {
  std::mutex mu;
  bool configured = false;  // a path was set (or the environment was read)
  std::string path;
  std::vector<GemmEntry> gemm;
  std::vector<StencilEntry> stencil;
};
Cache& cache() {
  static Cache c;
  return c;
}

// Parse the file at `path` into the entry lists (a missing file is empty).
void load_locked(Cache& c) {
  c.gemm.clear();
  c.stencil.clear();
  if (c.path.empty()) return;
  FILE* f = fopen(c.path.c_str(), "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    char kind[16], arch[64];
    if (sscanf(line, "%15s %63s", kind, arch) != 2) continue;
    if (!strcmp(kind, "gemm")) {
      GemmEntry e;
      long long M, N, K;
      if (sscanf(line, "%*s %*s %lld %lld %lld %d %d %d %d %lf", &M, &N, &K, &e.mode, &e.tile.bm,
                 &e.tile.bn, &e.tile.bk, &e.us) != 8)
        continue;
      e.arch = arch;
      e.M = M, e.N = N, e.K = K;
      c.gemm.push_back(e);
    } else if (!strcmp(kind, "stencil")) {
      StencilEntry e;
      long long H, W;
      if (sscanf(line, "%*s %*s %lld %lld %d %d %d %lf", &H, &W, &e.k, &e.sched.variant,
                 &e.sched.rows, &e.us) != 6)
        continue;
      e.arch = arch;
      e.H = H, e.W = W;
      c.stencil.push_back(e);
    }
  }
  fclose(f);
}

void configure_locked(Cache& c) {
  if (c.configured) return;
  c.configured = true;
  const char* env = getenv("RISE_TUNE_CACHE");
  c.path = env ? env : "";
  load_locked(c);
}

// Write every entry back to `path` (the cache file is rewritten whole).
bool save(const std::string& path, const std::vector<GemmEntry>& g,
          const std::vector<StencilEntry>& s) {
  const std::string tmp = path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  for (const auto& e : g)
    fprintf(f, "gemm %s %lld %lld %lld %d %d %d %d %.3f\n", e.arch.c_str(), (long long)e.M,
            (long long)e.N, (long long)e.K, e.mode, e.tile.bm, e.tile.bn, e.tile.bk, e.us);
  for (const auto& e : s)
    fprintf(f, "stencil %s %lld %lld %d %d %d %.3f\n", e.arch.c_str(), (long long)e.H,
            (long long)e.W, e.k, e.sched.variant, e.sched.rows, e.us);
  const bool ok = fclose(f) == 0;
  return ok && rename(tmp.c_str(), path.c_str()) == 0;
}

// Entries of the file at `path` (read afresh, so concurrent tuners of other
// shapes are not lost), with `add` replacing an entry of the same key.
template <class E, class Same>
void merge(std::vector<E>& list, const E& add, Same same) {
  list.erase(std::remove_if(list.begin(), list.end(), [&](const E& e) { return same(e, add); }),
             list.end());
  list.push_back(add);
}

// Architecture name of the current device up to the first ':' ("gfx950");
// empty when there is no device.
std::string device_arch() {
  static std::mutex mu;
  static std::string names[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return "";
  }
  std::lock_guard<std::mutex> lock(mu);
  if (names[dev].empty()) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
      (void)hipGetLastError();
      return "";
    }
    std::string a = p.gcnArchName;
    names[dev] = a.substr(0, a.find(':'));
  }
  return names[dev];
}

__global__ void fill_uniform(float* p, int64_t n, uint32_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    // a 32-bit integer hash of the index, mapped to [-1, 1)
    uint32_t h = (uint32_t)i * 0x9E3779B1u ^ seed;
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    p[i] = (float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f;
  }
}

struct DeviceBuffers {
  std::vector<void*> ptrs;
  ~DeviceBuffers() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  void* alloc(size_t bytes, hipError_t* e) {
    void* p = nullptr;
    *e = hipMalloc(&p, std::max<size_t>(bytes, 256));
    if (*e == hipSuccess) ptrs.push_back(p);
    return p;
  }
};

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  Events() {
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
  }
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Mean microseconds of one call of `run` on stream s: one warm-up call, then as
// many calls as fill about 20 ms (3 to 50) between two events.
template <class Run>
rise_status time_calls(Run run, hipStream_t s, const Events& ev, double* us) {
  rise_status st = run();
  if (st != RISE_OK) return st;
  hipError_t e = hipEventRecord(ev.a, s);
  if (e == hipSuccess) st = run();
  if (e == hipSuccess) e = hipEventRecord(ev.b, s);
  if (e == hipSuccess) e = hipEventSynchronize(ev.b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.a, ev.b);
  if (e != hipSuccess) return fail(RISE_ERR_HIP, std::string("autotune: ") + hipGetErrorString(e));
  if (st != RISE_OK) return st;
  const int reps = std::max(3, std::min(50, (int)(20.0 / std::max(ms, 1e-3f))));
  e = hipEventRecord(ev.a, s);
  for (int i = 0; i < reps && st == RISE_OK && e == hipSuccess; i++) st = run();
  if (e == hipSuccess) e = hipEventRecord(ev.b, s);
  if (e == hipSuccess) e = hipEventSynchronize(ev.b);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.a, ev.b);
  if (e != hipSuccess) return fail(RISE_ERR_HIP, std::string("autotune: ") + hipGetErrorString(e));
  *us = 1e3 * ms / reps;
  return st;
}

}  // namespace

bool tune_lookup_gemm(int64_t M, int64_t N, int64_t K, int mode, rise_tile* out) {
  Cache& c = cache();
  std::string arch;
  {
    std::lock_guard<std::mutex> lock(c.mu);
    configure_locked(c);
    if (c.gemm.empty()) return false;
  }
  arch = device_arch();
  if (arch.empty()) return false;
  std::lock_guard<std::mutex> lock(c.mu);
  for (auto it = c.gemm.rbegin(); it != c.gemm.rend(); ++it)
    if (it->M == M && it->N == N && it->K == K && it->mode == mode && it->arch == arch) {
      *out = it->tile;
      return true;
    }
  return false;
}

bool tune_lookup_stencil(int64_t H, int64_t W, int k, rise_stencil_schedule* out) {
  Cache& c = cache();
  {
    std::lock_guard<std::mutex> lock(c.mu);
    configure_locked(c);
    if (c.stencil.empty()) return false;
  }
  const std::string arch = device_arch();
  if (arch.empty()) return false;
  std::lock_guard<std::mutex> lock(c.mu);
  for (auto it = c.stencil.rbegin(); it != c.stencil.rend(); ++it)
    if (it->H == H && it->W == W && it->k == k && it->arch == arch) {
      *out = it->sched;
      return true;
    }
  return false;
}

}  // namespace rise

using namespace rise;

extern "C" {

rise_status rise_set_tune_cache(const char* path) {
  clear_error();
  Cache& c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  c.configured = true;
  c.path = path ? path : "";
  load_locked(c);
  return RISE_OK;
}

rise_status rise_autotune_gemm(const char* cache_path, int64_t M, int64_t N, int64_t K,
                               rise_mode mode, void* stream) {
  clear_error();
  if (!cache_path) return fail(RISE_ERR_NULL, "rise_autotune_gemm: cache_path is NULL");
  if (M <= 0 || N <= 0 || K <= 0 || M >= (1LL << 31) || N >= (1LL << 31) || K >= (1LL << 31))
    return fail(RISE_ERR_SHAPE, "rise_autotune_gemm: sizes must be in [1, 2^31)");
  if (mode < RISE_MODE_F32 || mode > RISE_MODE_FP8)
    return fail(RISE_ERR_UNSUPPORTED, "rise_autotune_gemm: unknown mode");
  if ((double)M * K + (double)K * N + (double)M * N > (double)(1LL << 32))
    return fail(RISE_ERR_SHAPE, "rise_autotune_gemm: operands above 16 GiB");
  const std::string arch = device_arch();
  if (arch.empty()) return fail(RISE_ERR_HIP, "rise_autotune_gemm: no current device");
  hipStream_t s = (hipStream_t)stream;
  const int n = rise_gemm_tiles(mode, nullptr, 0);
  std::vector<rise_tile> tiles(n);
  rise_gemm_tiles(mode, tiles.data(), n);
  size_t ws_bytes = 0;
  for (const auto& t : tiles) ws_bytes = std::max(ws_bytes, rise_gemm_workspace(M, N, K, mode, &t));
  DeviceBuffers buf;
  hipError_t e = hipSuccess;
  float* A = (float*)buf.alloc((size_t)M * K * 4, &e);
  float* B = e == hipSuccess ? (float*)buf.alloc((size_t)K * N * 4, &e) : nullptr;
  float* C = e == hipSuccess ? (float*)buf.alloc((size_t)M * N * 4, &e) : nullptr;
  void* ws = e == hipSuccess && ws_bytes ? buf.alloc(ws_bytes, &e) : nullptr;
  if (e != hipSuccess)
    return fail(RISE_ERR_HIP, std::string("rise_autotune_gemm: ") + hipGetErrorString(e));
  hipLaunchKernelGGL(fill_uniform, dim3(1024), dim3(256), 0, s, A, M * K, 1u);
  hipLaunchKernelGGL(fill_uniform, dim3(1024), dim3(256), 0, s, B, K * N, 2u);
  rise_status st = check_launch("rise_autotune_gemm: fill");
  if (st != RISE_OK) return st;
  Events ev;
  GemmEntry best{arch, M, N, K, (int)mode, rise_tile{0, 0, 0}, 0.0};
  for (const auto& t : tiles) {
    double us = 0;
    st = time_calls(
        [&] {
          return rise_gemm(C, N, A, RISE_F32, K, RISE_OP_N, B, RISE_F32, N, RISE_OP_N, M, N, K,
                           mode, &t, ws, ws_bytes, stream);
        },
        s, ev, &us);
    if (st != RISE_OK) return st;
    if (best.tile.bm == 0 || us < best.us) best.tile = t, best.us = us;
  }
  Cache& c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  Cache file;
  file.path = cache_path;
  load_locked(file);
  merge(file.gemm, best, [](const GemmEntry& a, const GemmEntry& b) {
    return a.arch == b.arch && a.M == b.M && a.N == b.N && a.K == b.K && a.mode == b.mode;
  });
  if (!save(cache_path, file.gemm, file.stencil))
    return fail(RISE_ERR_UNSUPPORTED, "rise_autotune_gemm: cannot write the cache file");
  if (c.configured && c.path == cache_path) load_locked(c);
  return RISE_OK;
}

rise_status rise_autotune_stencil(const char* cache_path, int64_t H, int64_t W, int32_t k,
                                  void* stream) {
  clear_error();
  if (!cache_path) return fail(RISE_ERR_NULL, "rise_autotune_stencil: cache_path is NULL");
  if (H <= 0 || W <= 0 || H >= (1LL << 31) || W >= (1LL << 31) || (double)H * W > (double)(1LL << 32))
    return fail(RISE_ERR_SHAPE, "rise_autotune_stencil: sizes must be in [1, 2^31), H*W <= 2^32");
  if (k != 1 && k != 3 && k != 5 && k != 7)
    return fail(RISE_ERR_UNSUPPORTED,
                "rise_autotune_stencil: scheduled windows are square 1, 3, 5 and 7");
  const std::string arch = device_arch();
  if (arch.empty()) return fail(RISE_ERR_HIP, "rise_autotune_stencil: no current device");
  hipStream_t s = (hipStream_t)stream;
  const int n = rise_stencil_schedules(nullptr, 0);
  std::vector<rise_stencil_schedule> scheds(n);
  rise_stencil_schedules(scheds.data(), n);
  DeviceBuffers buf;
  hipError_t e = hipSuccess;
  float* in = (float*)buf.alloc((size_t)H * W * 4, &e);
  float* out = e == hipSuccess ? (float*)buf.alloc((size_t)H * W * 4, &e) : nullptr;
  float* w = e == hipSuccess ? (float*)buf.alloc(256, &e) : nullptr;
  if (e != hipSuccess)
    return fail(RISE_ERR_HIP, std::string("rise_autotune_stencil: ") + hipGetErrorString(e));
  hipLaunchKernelGGL(fill_uniform, dim3(1024), dim3(256), 0, s, in, H * W, 3u);
  hipLaunchKernelGGL(fill_uniform, dim3(1), dim3(64), 0, s, w, (int64_t)k * k, 4u);
  rise_status st = check_launch("rise_autotune_stencil: fill");
  if (st != RISE_OK) return st;
  Events ev;
  StencilEntry best{arch, H, W, k, rise_stencil_schedule{-1, 0}, 0.0};
  for (const auto& sc : scheds) {
    double us = 0;
    st = time_calls(
        [&] {
          return rise_stencil2d(out, W, in, W, H, W, w, k, k, RISE_PAD_CLAMP, &sc, stream);
        },
        s, ev, &us);
    if (st != RISE_OK) return st;
    if (best.sched.variant < 0 || us < best.us) best.sched = sc, best.us = us;
  }
  Cache& c = cache();
  std::lock_guard<std::mutex> lock(c.mu);
  Cache file;
  file.path = cache_path;
  load_locked(file);
  merge(file.stencil, best, [](const StencilEntry& a, const StencilEntry& b) {
    return a.arch == b.arch && a.H == b.H && a.W == b.W && a.k == b.k;
  });
  if (!save(cache_path, file.gemm, file.stencil))
    return fail(RISE_ERR_UNSUPPORTED, "rise_autotune_stencil: cannot write the cache file");
  if (c.configured && c.path == cache_path) load_locked(c);
  return RISE_OK;
}

}  // extern "C"
