// CPU emulation of the small HIP subset librmx uses, so that the library (host core AND
// kernels) can be compiled for the host and run under AddressSanitizer on tiny inputs.
// Test infrastructure only.  A block's threads are host threads; __syncthreads and the
// cross-lane operations are barriers over the block, the 64-lane wave or the shuffle
// group.  Blocks of a launch run one after another, so a kernel's __shared__ variables can
// be statics; device memory is host memory.  The persistent kernel, whose blocks wait on
// each other, runs all its blocks at once (see hipLaunchKernelGGL below).
#pragma once
#include <algorithm>
#include <atomic>
#include <barrier>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __noinline__
#define __constant__
#define __shared__ static
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define RMX_GLOBAL_AS   // host memory is the only address space here
inline void __builtin_amdgcn_sched_barrier(int) {}   // instruction scheduling: nothing to do
#define __builtin_amdgcn_fence(order, scope) std::atomic_thread_fence(std::memory_order_seq_cst)
#define HIP_DYNAMIC_SHARED(type, var) type* var = reinterpret_cast<type*>(rmx_emu::dyn_lds());

struct alignas(16) uint4 {
    unsigned x, y, z, w;
};
inline uint4 make_uint4(unsigned x, unsigned y, unsigned z, unsigned w) { return {x, y, z, w}; }

struct dim3 {
    unsigned x = 1, y = 1, z = 1;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

using std::max;
using std::min;

namespace rmx_emu {
struct Block;
extern thread_local dim3 threadIdx_, blockIdx_;
extern dim3 blockDim_, gridDim_;
extern thread_local Block* block_;
unsigned char* dyn_lds();
void sync_block();
// exchange of one 64-bit value among `width` consecutive lanes of the caller's group
uint64_t* group_exchange(uint64_t v, int width);
void group_done(int width);
}  // namespace rmx_emu

#define threadIdx rmx_emu::threadIdx_
#define blockIdx rmx_emu::blockIdx_
#define blockDim rmx_emu::blockDim_
#define gridDim rmx_emu::gridDim_

inline void __syncthreads() { rmx_emu::sync_block(); }
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
int __syncthreads_or(int p);

template <typename T>
inline uint64_t rmx_emu_bits(T v) {
    uint64_t u = 0;
    std::memcpy(&u, &v, sizeof(T));
    return u;
}
template <typename T>
inline T rmx_emu_from(uint64_t u) {
    T v;
    std::memcpy(&v, &u, sizeof(T));
    return v;
}

inline unsigned long long __ballot(int pred) {
    uint64_t* s = rmx_emu::group_exchange(pred ? 1 : 0, 64);
    unsigned long long m = 0;
    for (int i = 0; i < 64; ++i)
        if (s[i]) m |= 1ull << i;
    rmx_emu::group_done(64);
    return m;
}
template <typename T>
inline T __shfl_xor(T v, int o, int width = 64) {
    const int lane = threadIdx.x % width;
    uint64_t* s = rmx_emu::group_exchange(rmx_emu_bits(v), width);
    const T r = rmx_emu_from<T>(s[lane ^ o]);
    rmx_emu::group_done(width);
    return r;
}
template <typename T>
inline T __shfl(T v, int src, int width = 64) {
    uint64_t* s = rmx_emu::group_exchange(rmx_emu_bits(v), width);
    const T r = rmx_emu_from<T>(s[((src % width) + width) % width]);
    rmx_emu::group_done(width);
    return r;
}
template <typename T>
inline T __shfl_up(T v, int o, int width = 64) {
    const int lane = threadIdx.x % width;
    uint64_t* s = rmx_emu::group_exchange(rmx_emu_bits(v), width);
    const T r = lane >= o ? rmx_emu_from<T>(s[lane - o]) : v;
    rmx_emu::group_done(width);
    return r;
}
inline long long __double_as_longlong(double v) { return rmx_emu_from<long long>(rmx_emu_bits(v)); }
inline double __longlong_as_double(long long v) { return rmx_emu_from<double>(rmx_emu_bits(v)); }
inline int __float_as_int(float v) { return rmx_emu_from<int>(rmx_emu_bits(v)); }
inline float __int_as_float(int v) { return rmx_emu_from<float>(rmx_emu_bits(v)); }
// DPP moves used by the library, within the aligned group that holds every source lane:
// quad_perm (0x00-0xff, groups of 4), row_half_mirror (0x141, 8), row_mirror (0x140, 16).
inline int __builtin_amdgcn_update_dpp(int old, int src, int ctrl, int, int, bool) {
    const int w = ctrl <= 0xff ? 4 : (ctrl == 0x141 ? 8 : (ctrl == 0x140 ? 16 : 0));
    if (w == 0) std::abort();
    const int lane = threadIdx.x % w;
    int from = 0;
    if (w == 4) from = (ctrl >> (2 * lane)) & 3;
    else from = w - 1 - lane;
    uint64_t* s = rmx_emu::group_exchange((uint64_t)(uint32_t)src, w);
    const int r = (int)(uint32_t)s[from];
    rmx_emu::group_done(w);
    (void)old;
    return r;
}
// Reciprocal: the hardware's is approximate; the quotient it seeds is refined to the
// correctly rounded one, so an exact reciprocal serves.
inline double __builtin_amdgcn_rcp(double x) { return 1.0 / x; }
inline double __builtin_amdgcn_rsq(double x) { return 1.0 / std::sqrt(x); }
// The value of lane `src` of the wave (every lane active; a 64-lane collective here).
inline int __builtin_amdgcn_readlane(int v, int src) {
    if (src < 0 || src > 63) std::abort();
    uint64_t* s = rmx_emu::group_exchange((uint64_t)(uint32_t)v, 64);
    const int r = (int)(uint32_t)s[src];
    rmx_emu::group_done(64);
    return r;
}
inline int __builtin_amdgcn_readfirstlane(int v) {
    uint64_t* s = rmx_emu::group_exchange((uint64_t)(uint32_t)v, 64);
    const int r = (int)(uint32_t)s[0];
    rmx_emu::group_done(64);
    return r;
}
// A poll's pause.  The bounded waits of the persistent kernel count polls; emulated blocks
// run thousands of host threads under the sanitizers, so a pause of 20 us (about 20 s over
// the bound) keeps a slow but progressing wait from running out, and frees the CPU for the
// blocks that do the work.
inline void __builtin_amdgcn_s_sleep(int) { std::this_thread::sleep_for(std::chrono::microseconds(20)); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __ffsll(long long x) { return __builtin_ffsll(x); }

template <typename T>
inline T atomicAdd(T* p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
template <typename T>
inline T atomicOr(T* p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
#define __HIP_MEMORY_SCOPE_AGENT 0
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), __ATOMIC_SEQ_CST)

// ---- host API ------------------------------------------------------------------------
typedef enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 } hipError_t;
typedef struct rmx_emu_stream* hipStream_t;
typedef struct rmx_emu_event* hipEvent_t;
typedef struct rmx_emu_graph* hipGraph_t;
typedef struct rmx_emu_graph* hipGraphExec_t;
typedef struct rmx_emu_graph_node* hipGraphNode_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum hipDeviceAttribute_t { hipDeviceAttributeMaxSharedMemoryPerBlock,
                            hipDeviceAttributeMultiprocessorCount };
enum hipStreamCaptureMode { hipStreamCaptureModeThreadLocal };
#define hipHostMallocDefault 0
#define hipEventDisableTiming 0
#define hipStreamNonBlocking 0

hipError_t hipGetDeviceCount(int* n);
hipError_t hipSetDevice(int d);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int d);
hipError_t hipMalloc(void** p, size_t n);
template <typename T>
inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc(reinterpret_cast<void**>(p), n); }
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags);
// Blocks resident per compute unit: one (a concurrent launch runs 256 host threads per
// block).
template <typename F>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, F, int, size_t) {
    *n = 1;
    return hipSuccess;
}
// A __device__ variable is host storage here: its address is the symbol's own.
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
    *p = const_cast<void*>(sym);
    return hipSuccess;
}
template <typename T>
inline hipError_t hipHostMalloc(T** p, size_t n, unsigned flags) {
    return hipHostMalloc(reinterpret_cast<void**>(p), n, flags);
}
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t st);
hipError_t hipMemset(void* d, int v, size_t n);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned f);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned f);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* n, char* l,
                               size_t ln);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphDestroy(hipGraph_t g);
namespace rmx_emu {
// Blocks run one after another (static __shared__ variables are one copy), or all at once
// for `concurrent` launches; the threads of a block run concurrently.
void launch(dim3 grid, dim3 block, size_t lds, hipStream_t st, std::function<void()> body,
            bool concurrent = false);
}
// The persistent band kernel (k_band<...>) keeps its whole block state in dynamic LDS and
// its blocks wait on each other: its launches run every block concurrently, each with its
// own LDS.  Other kernels run their blocks in turn.
#define hipLaunchKernelGGL(K, G, B, L, S, ...)                                          \
    rmx_emu::launch((G), (B), (L), (S), [=]() { K(__VA_ARGS__); },                      \
                    std::strncmp(#K, "k_band", 6) == 0)
