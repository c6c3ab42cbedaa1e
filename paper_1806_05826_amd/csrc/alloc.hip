// Device memory of the library.  Every device allocation and free of the
// library goes through dev_malloc / dev_free, which serve them from the
// memory context current on the calling thread (MemScope, set by each entry
// point to the context of the handle it works on):
//   * kBump: a handle set up on a caller workspace (rr_setup_ws): a bump
//     arena over that buffer, 256-byte aligned; frees return nothing, the
//     caller owns the memory and releases it after rr_destroy;
//   * kHook: the caller's allocator (rr_set_allocator) as installed when the
//     handle was set up (the Python binding installs PyTorch's caching
//     allocator, so PyTorch supplies the device memory);
//   * kCount: hipMalloc, counting the arena bytes an identical setup needs
//     (rr_setup_workspace_size: setup is deterministic, so an identical call
//     requests the same sizes in the same order);
//   * kHip: hipMalloc / hipFree.
#include <mutex>

#include "rr_device.h"

namespace rr {

namespace {
std::mutex g_hook_mu;
rr_alloc_fn g_alloc = nullptr;
rr_free_fn g_free = nullptr;
void* g_ctx = nullptr;
thread_local MemCtx* t_mem = nullptr;
constexpr size_t kAlign = 256;

size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }
}  // namespace

MemScope::MemScope(MemCtx* m) : saved_(t_mem) { t_mem = m; }
MemScope::~MemScope() { t_mem = saved_; }

MemCtx default_mem() {
  MemCtx m;
  std::lock_guard<std::mutex> lk(g_hook_mu);
  if (g_alloc) {
    m.mode = MemCtx::kHook;
    m.alloc = g_alloc;
    m.free = g_free;
    m.ctx = g_ctx;
  }
  return m;
}

hipError_t dev_malloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  MemCtx* m = t_mem;
  if (!m || m->mode == MemCtx::kHip) return hipMalloc(p, bytes);
  switch (m->mode) {
    case MemCtx::kBump: {
      const size_t need = round_up(bytes);
      if (m->used + need > m->cap) {
        m->overflow = true;
        return hipErrorOutOfMemory;
      }
      *p = m->base + m->used;
      m->used += need;
      return hipSuccess;
    }
    case MemCtx::kCount:
      m->used += round_up(bytes);
      return hipMalloc(p, bytes);
    case MemCtx::kHook: {
      int dev = 0;
      (void)hipGetDevice(&dev);
      *p = m->alloc(bytes, dev, m->ctx);
      return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    default:
      return hipMalloc(p, bytes);
  }
}

hipError_t dev_free(void* p) {
  if (!p) return hipSuccess;
  MemCtx* m = t_mem;
  if (!m || m->mode == MemCtx::kHip || m->mode == MemCtx::kCount) return hipFree(p);
  if (m->mode == MemCtx::kBump) return hipSuccess;   // the caller owns the workspace
  // the caller's allocator may hand the block out again at once: nothing
  // queued on any stream may still use it
  (void)hipDeviceSynchronize();
  int dev = 0;
  (void)hipGetDevice(&dev);
  m->free(p, dev, m->ctx);
  return hipSuccess;
}

}  // namespace rr

extern "C" rr_status rr_set_allocator(rr_alloc_fn alloc, rr_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return rr::fail(RR_ERR_INVALID_ARG, "rr_set_allocator: give both functions or neither");
  std::lock_guard<std::mutex> lk(rr::g_hook_mu);
  rr::g_alloc = alloc;
  rr::g_free = free_fn;
  rr::g_ctx = ctx;
  return RR_OK;
}
