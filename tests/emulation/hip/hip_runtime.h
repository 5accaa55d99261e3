// TEST INFRASTRUCTURE: a CPU emulation of the HIP subset the kernels of libimb use, so that the
// unmodified kernel sources can run on the host under AddressSanitizer (bounds checking of every
// index) and be compared with the oracle without a GPU.  Workgroups run one at a time, their
// threads as std::threads; __syncthreads is a std::barrier; 64-lane wavefront operations
// (ballot, shuffles, DPP row rotations, readlane) exchange values through per-wavefront buffers.
// Graph capture reports "not supported", so the library falls back to direct launches.  Never
// part of the product library.
#pragma once
#include <atomic>
#include <barrier>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <thread>
#include <algorithm>
#include <vector>

using std::fabs; using std::sqrt; using std::atan2; using std::sin; using std::cos; using std::fmin;
using std::fmax; using std::floor; using std::ceil; using std::asin; using std::isfinite;

#define __host__
#define __device__
#define __global__
#define __noinline__ __attribute__((noinline))
#define __forceinline__ inline __attribute__((always_inline))
#define __restrict__ __restrict
#define __shared__ static
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define __builtin_nontemporal_load(p) (*(p))
#define __builtin_nontemporal_store(v, p) (*(p) = (v))

struct dim3 {
  unsigned x = 1, y = 1, z = 1;
  dim3() = default;
  dim3(unsigned a, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
extern thread_local dim3 threadIdx, blockIdx;
extern dim3 blockDim, gridDim;

#define EMU_VEC2(N, T) struct N { T x, y; }; inline N make_##N(T a, T b) { return N{a, b}; }
#define EMU_VEC4(N, T) struct N { T x, y, z, w; }; inline N make_##N(T a, T b, T c, T d) { return N{a, b, c, d}; }
EMU_VEC2(int2, int) EMU_VEC2(double2, double) EMU_VEC2(float2, float)
EMU_VEC4(int4, int) EMU_VEC4(double4, double) EMU_VEC4(uint4, unsigned) EMU_VEC4(float4, float)

// ---- atomics / fences
template <class T, class U> inline T atomicAdd(T* p, U v) { return __atomic_fetch_add(p, (T)v, __ATOMIC_SEQ_CST); }
template <class T, class U> inline T atomicOr(T* p, U v) { return __atomic_fetch_or(p, (T)v, __ATOMIC_SEQ_CST); }
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
#define __HIP_MEMORY_SCOPE_AGENT 0
#define __HIP_MEMORY_SCOPE_WORKGROUP 0
#define __hip_atomic_load(p, o, s) __atomic_load_n((p), __ATOMIC_SEQ_CST)
#define __hip_atomic_store(p, v, o, s) __atomic_store_n((p), (v), __ATOMIC_SEQ_CST)
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
#define __builtin_amdgcn_fence(a, b) std::atomic_thread_fence(std::memory_order_seq_cst)
void __builtin_amdgcn_wave_barrier();  // every lane of the wavefront must reach it
#define __builtin_amdgcn_s_sleep(n) std::this_thread::yield()
#define __builtin_amdgcn_s_waitcnt(n) std::atomic_thread_fence(std::memory_order_seq_cst)
long long wall_clock64();
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }

// ---- bit casts
inline int __float_as_int(float f) { int i; std::memcpy(&i, &f, 4); return i; }
inline float __int_as_float(int i) { float f; std::memcpy(&f, &i, 4); return f; }
inline unsigned __float_as_uint(float f) { unsigned i; std::memcpy(&i, &f, 4); return i; }
inline float __uint_as_float(unsigned i) { float f; std::memcpy(&f, &i, 4); return f; }
inline long long __double_as_longlong(double d) { long long i; std::memcpy(&i, &d, 8); return i; }
inline double __longlong_as_double(long long i) { double d; std::memcpy(&d, &i, 8); return d; }

// ---- block / wave synchronisation
void __syncthreads();
unsigned long long emu_wave_exchange(unsigned long long mine, int src_lane);  // value of src_lane
unsigned long long __ballot(int pred);
int emu_lane();
template <class T> inline T emu_from_bits(unsigned long long b) { T v; std::memcpy(&v, &b, sizeof(T)); return v; }
template <class T> inline unsigned long long emu_to_bits(T v) { unsigned long long b = 0; std::memcpy(&b, &v, sizeof(T)); return b; }
template <class T> inline T __shfl_xor(T v, int mask, int width = 64) {
  const int l = emu_lane();
  const int src = (l & ~(width - 1)) | ((l ^ mask) & (width - 1));
  return emu_from_bits<T>(emu_wave_exchange(emu_to_bits(v), src));
}
template <class T> inline T __shfl_up(T v, unsigned delta, int width = 64) {
  const int l = emu_lane();
  const int lw = l & (width - 1);
  const int src = lw >= (int)delta ? l - (int)delta : l;
  return emu_from_bits<T>(emu_wave_exchange(emu_to_bits(v), src));
}
template <class T> inline T __shfl_down(T v, unsigned delta, int width = 64) {
  const int l = emu_lane();
  const int lw = l & (width - 1);
  const int src = lw + (int)delta < width ? l + (int)delta : l;
  return emu_from_bits<T>(emu_wave_exchange(emu_to_bits(v), src));
}
inline int __builtin_amdgcn_readfirstlane(int v) {  // every lane of the wave is active
  return (int)emu_wave_exchange(emu_to_bits(v), 0);
}
inline int __builtin_amdgcn_readlane(int v, int lane) {
  return (int)emu_wave_exchange(emu_to_bits(v), lane);
}
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int, int, bool) {
  (void)old;
  const int l = emu_lane();
  int from = l;
  if (ctrl >= 0x121 && ctrl <= 0x12F) {  // row_ror:N
    const int n = ctrl & 0xF;
    from = (l & ~15) | ((l - n) & 15);
  }
  return (int)emu_wave_exchange(emu_to_bits(src), from);
}

// ---- dynamic LDS
void* emu_dyn_lds();

// ---- runtime API
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorNotSupported = 801, hipErrorInvalidValue = 1 };
typedef struct emu_stream* hipStream_t;
typedef struct emu_event* hipEvent_t;
typedef struct emu_graph* hipGraph_t;
typedef struct emu_graph_exec* hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost,
                     hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum { hipStreamNonBlocking = 1 };
enum { hipEventDisableTiming = 2 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount, hipDeviceAttributeWallClockRate };
hipError_t hipMalloc(void** p, size_t n);
template <class T> inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
hipError_t hipFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned);
hipError_t hipStreamDestroy(hipStream_t);
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode);
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*);
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, char*, size_t);
hipError_t hipGraphDestroy(hipGraph_t);
hipError_t hipGraphExecDestroy(hipGraphExec_t);
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t);
hipError_t hipGraphUpload(hipGraphExec_t, hipStream_t);
hipError_t hipGetDevice(int* device);
// a device variable's address: in the emulation, its host address
#define HIP_SYMBOL(sym) ((const void*)&(sym))
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol);
hipError_t hipEventCreate(hipEvent_t*);
hipError_t hipEventCreateWithFlags(hipEvent_t*, unsigned);
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned);
hipError_t hipEventRecord(hipEvent_t, hipStream_t);
hipError_t hipEventElapsedTime(float*, hipEvent_t, hipEvent_t);
hipError_t hipEventDestroy(hipEvent_t);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t);
hipError_t hipDeviceGetAttribute(int*, hipDeviceAttribute_t, int);
template <class K> inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, K, int, size_t) { *n = 1; return hipSuccess; }

void emu_launch(dim3 grid, dim3 block, size_t shmem, const std::function<void()>& body);
// A launch on a stream the library created (hipStreamCreateWithFlags) is deferred: it runs only
// when another stream waits for an event recorded after it, or that stream is synchronised or
// destroyed.  Work such a stream overlaps with on the GPU thus runs after, not before, what the
// other stream queued meanwhile -- the order the GPU is least likely to produce, which exposes a
// missing dependency.  Launches on the caller's stream run at once.
void emu_launch_on(hipStream_t st, dim3 grid, dim3 block, size_t shmem,
                   const std::function<void()>& body);
#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  emu_launch_on(stream, dim3(grid), dim3(block), (size_t)(shmem), [=]() { kernel(__VA_ARGS__); })
