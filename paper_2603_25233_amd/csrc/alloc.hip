// Device memory for the library's temporaries, kept for reuse between calls.
//
// A solve allocates some forty buffers (sweep workspace, diffusion hierarchy, basis) and
// hipMalloc / hipFree cost 0.1-0.6 ms each (hipFree waits for the device), so a
// repeated call spent ~15 ms on them at 1024 x 1024.  Buffers allocated inside a call
// that names a stream (StreamScope) come from a cache of idle blocks of the same rounded
// size; at the end of the outermost scope the call's stream is synchronised once and the
// buffers it released become idle blocks, usable by any later call on any stream.
// Buffers allocated outside a scope (the sweep plans, which outlive calls) go straight to
// hipMalloc / hipFree.  The cache is bounded (an eighth of the device's memory) and is
// emptied by rte_release_cached_memory or when a hipMalloc runs out of memory.
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.h"

namespace rte {
namespace {

struct Block {
  void* p;
  size_t bytes;
  int dev;
};

std::mutex mu;
std::multimap<std::pair<int, size_t>, void*> idle;  // (device, rounded bytes) -> block
size_t idle_bytes = 0;
size_t cap_bytes = 0;  // set on first use

thread_local int scope_depth = 0;
thread_local hipStream_t scope_stream = nullptr;
thread_local std::vector<Block> released;  // released inside the current outermost scope

size_t rounded(size_t bytes) {
  const size_t g = bytes < (1u << 20) ? 512 : (2u << 20);
  return (bytes + g - 1) / g * g;
}

size_t cache_cap() {
  if (cap_bytes == 0) {
    size_t fr = 0, tot = 0;
    cap_bytes = hipMemGetInfo(&fr, &tot) == hipSuccess && tot > 0 ? tot / 8 : (size_t)8 << 30;
  }
  return cap_bytes;
}

// frees every idle block (mu held)
void drop_idle() {
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : idle) {
    (void)hipSetDevice(kv.first.first);
    (void)hipFree(kv.second);
  }
  (void)hipSetDevice(cur);
  idle.clear();
  idle_bytes = 0;
}

}  // namespace

void* pool_alloc(size_t bytes, bool* pooled) {
  *pooled = false;
  if (bytes == 0) return nullptr;
  void* p = nullptr;
  if (scope_depth == 0) {
    RTE_CHECK_HIP(hipMalloc(&p, bytes));
    return p;
  }
  int dev = 0;
  RTE_CHECK_HIP(hipGetDevice(&dev));
  const size_t rb = rounded(bytes);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = idle.find({dev, rb});
    if (it != idle.end()) {
      p = it->second;
      idle.erase(it);
      idle_bytes -= rb;
      *pooled = true;
      return p;
    }
  }
  hipError_t e = hipMalloc(&p, rb);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(mu);
      drop_idle();
    }
    e = hipMalloc(&p, rb);
  }
  RTE_CHECK_HIP(e);
  *pooled = true;
  return p;
}

void pool_free(void* p, size_t bytes, bool pooled) {
  if (!p) return;
  if (!pooled || scope_depth == 0) {
    (void)hipFree(p);
    return;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  released.push_back(Block{p, rounded(bytes), dev});
}

StreamScope::StreamScope(hipStream_t st) {
  if (scope_depth++ == 0) scope_stream = st;
}

StreamScope::~StreamScope() {
  if (--scope_depth != 0 || released.empty()) return;
  // the call's work on its stream has finished with the released buffers once this
  // returns; if it fails (a faulted stream), the buffers are freed instead of kept
  const bool ok = hipStreamSynchronize(scope_stream) == hipSuccess;
  std::lock_guard<std::mutex> lk(mu);
  const size_t cap = cache_cap();
  for (const Block& b : released) {
    if (ok && idle_bytes + b.bytes <= cap) {
      idle.insert({{b.dev, b.bytes}, b.p});
      idle_bytes += b.bytes;
    } else {
      (void)hipFree(b.p);
    }
  }
  released.clear();
}

void pool_release_all() {
  std::lock_guard<std::mutex> lk(mu);
  drop_idle();
}

}  // namespace rte

extern "C" rte_status rte_release_cached_memory(void) {
  rte::pool_release_all();
  return RTE_OK;
}
