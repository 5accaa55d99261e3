// TEST INFRASTRUCTURE: runtime and launcher of the CPU emulation (see hip/hip_runtime.h).
#include "hip/hip_runtime.h"

#include <condition_variable>
#include <cstdio>
#include <deque>
#include <memory>
#include <mutex>

thread_local dim3 threadIdx, blockIdx;
dim3 blockDim, gridDim;

namespace {
struct BlockCtx {
  std::unique_ptr<std::barrier<>> block;
  std::vector<std::unique_ptr<std::barrier<>>> waves;
  std::vector<unsigned long long> xbuf;  // [wave][64]
  std::vector<unsigned char> lds;
};
BlockCtx g_ctx;
thread_local int t_lane = 0, t_wave = 0;
std::chrono::steady_clock::time_point g_t0 = std::chrono::steady_clock::now();
}  // namespace

long long wall_clock64() {
  return (long long)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now() - g_t0).count() / 10;  // 100 MHz
}
void __syncthreads() { g_ctx.block->arrive_and_wait(); }
int emu_lane() { return t_lane; }
void __builtin_amdgcn_wave_barrier() { g_ctx.waves[t_wave]->arrive_and_wait(); }
unsigned long long emu_wave_exchange(unsigned long long mine, int src) {
  auto& b = *g_ctx.waves[t_wave];
  unsigned long long* buf = &g_ctx.xbuf[(size_t)t_wave * 64];
  buf[t_lane] = mine;
  b.arrive_and_wait();
  const unsigned long long v = buf[src & 63];
  b.arrive_and_wait();
  return v;
}
unsigned long long __ballot(int pred) {
  auto& b = *g_ctx.waves[t_wave];
  unsigned long long* buf = &g_ctx.xbuf[(size_t)t_wave * 64];
  buf[t_lane] = pred ? 1ull : 0ull;
  b.arrive_and_wait();
  unsigned long long m = 0;
  for (int l = 0; l < 64; ++l) if (buf[l]) m |= 1ull << l;
  b.arrive_and_wait();
  return m;
}
void* emu_dyn_lds() { return g_ctx.lds.data(); }

// A pool of worker threads, one per thread of the largest workgroup seen, reused for every
// workgroup of every launch (creating threads per workgroup dominates the run time otherwise).
namespace {
struct Pool {
  std::vector<std::thread> workers;
  std::mutex m;
  std::condition_variable cv_go, cv_done;
  long gen = 0;
  int done = 0;
  bool quit = false;
  const std::function<void()>* body = nullptr;
  unsigned nt = 0;
  dim3 bidx, bdim;
  ~Pool() {
    {
      std::lock_guard<std::mutex> g(m);
      quit = true;
      ++gen;
    }
    cv_go.notify_all();
    for (auto& w : workers) w.join();
  }
  void grow(unsigned n) {
    while (workers.size() < n) {
      const unsigned t = (unsigned)workers.size();
      workers.emplace_back([this, t]() {
        long seen = 0;
        for (;;) {
          {
            std::unique_lock<std::mutex> lk(m);
            cv_go.wait(lk, [&] { return gen != seen; });
            seen = gen;
            if (quit) return;
          }
          if (t < nt) {
            threadIdx = dim3(t % bdim.x, (t / bdim.x) % bdim.y, t / (bdim.x * bdim.y));
            blockIdx = bidx;
            t_lane = t & 63;
            t_wave = t >> 6;
            (*body)();
            g_ctx.waves[t_wave]->arrive_and_drop();
            g_ctx.block->arrive_and_drop();
          }
          {
            std::lock_guard<std::mutex> g(m);
            ++done;
          }
          cv_done.notify_one();
        }
      });
    }
  }
};
Pool g_pool;
}  // namespace

void emu_launch(dim3 grid, dim3 block, size_t shmem, const std::function<void()>& body) {
  const unsigned nt = block.x * block.y * block.z;
  gridDim = grid;
  blockDim = block;
  g_pool.grow(nt);
  const int nworkers = (int)g_pool.workers.size();
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) {
        g_ctx.block = std::make_unique<std::barrier<>>(nt);
        const unsigned nw = (nt + 63) / 64;
        g_ctx.waves.clear();
        for (unsigned w = 0; w < nw; ++w)
          g_ctx.waves.push_back(std::make_unique<std::barrier<>>(std::min(64u, nt - 64 * w)));
        g_ctx.xbuf.assign((size_t)nw * 64, 0);
        g_ctx.lds.assign(shmem + 64, 0xCD);  // poisoned dynamic LDS
        {
          std::lock_guard<std::mutex> g(g_pool.m);
          g_pool.body = &body;
          g_pool.nt = nt;
          g_pool.bidx = dim3(bx, by, bz);
          g_pool.bdim = block;
          g_pool.done = 0;
          ++g_pool.gen;
        }
        g_pool.cv_go.notify_all();
        std::unique_lock<std::mutex> lk(g_pool.m);
        g_pool.cv_done.wait(lk, [&] { return g_pool.done == nworkers; });
      }
}

// ---- runtime
hipError_t hipMalloc(void** p, size_t n) {
  *p = std::aligned_alloc(256, (n + 255) / 256 * 256 + 256);
  if (*p) std::memset(*p, 0xAB, (n + 255) / 256 * 256);
  return *p ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { std::memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) { return hipMemcpy(d, s, n, k); }
struct emu_stream {
  std::deque<std::function<void()>> pending;  // deferred launches, in order
  long long queued = 0, done = 0;
};
static void emu_flush(hipStream_t s, long long upto) {
  while (s && s->done < upto && !s->pending.empty()) {
    std::function<void()> f = std::move(s->pending.front());
    s->pending.pop_front();
    ++s->done;
    f();
  }
}
void emu_launch_on(hipStream_t st, dim3 grid, dim3 block, size_t shmem,
                   const std::function<void()>& body) {
  if (!st) {
    emu_launch(grid, block, shmem, body);
    return;
  }
  st->pending.push_back([=]() { emu_launch(grid, block, shmem, body); });
  ++st->queued;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  if (s) emu_flush(s, s->queued);
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new emu_stream{}; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) {
  if (s) emu_flush(s, s->queued);
  delete s;
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*) { return hipErrorNotSupported; }
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, char*, size_t) { return hipErrorNotSupported; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphUpload(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGetDevice(int* device) {
  *device = 0;
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol) {
  *ptr = const_cast<void*>(symbol);
  return hipSuccess;
}
struct emu_event {
  std::chrono::steady_clock::time_point t;
  hipStream_t st = nullptr;  // deferring stream it was recorded on, and its launch count then
  long long mark = 0;
};
hipError_t hipEventCreate(hipEvent_t* e) { *e = new emu_event{}; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new emu_event{}; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  e->t = std::chrono::steady_clock::now();
  e->st = s;
  e->mark = s ? s->queued : 0;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) {
  emu_flush(e->st, e->mark);
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count(); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "emulated error"; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  *v = a == hipDeviceAttributeMultiprocessorCount ? 1 : 100000; return hipSuccess; }
