// Host implementation of the HIP emulation shim (see hip/hip_runtime.h).  Test
// infrastructure only.
#include "hip/hip_runtime.h"

#include <map>

namespace rmx_emu {

thread_local dim3 threadIdx_, blockIdx_;
dim3 blockDim_, gridDim_;
thread_local Block* block_ = nullptr;


struct Block {
    int n = 0;
    std::unique_ptr<std::barrier<>> all;
    std::map<int, std::vector<std::unique_ptr<std::barrier<>>>> groups;
    std::map<int, std::vector<uint64_t>> slots;
    std::vector<int> orv;
    std::vector<unsigned char> lds;
};

unsigned char* dyn_lds() { return block_->lds.empty() ? nullptr : block_->lds.data(); }

void sync_block() { block_->all->arrive_and_wait(); }

uint64_t* group_exchange(uint64_t v, int width) {
    Block* b = block_;
    const int t = threadIdx_.x;
    auto& s = b->slots[width];
    s[t] = v;
    b->groups[width][t / width]->arrive_and_wait();
    return &s[(t / width) * width];
}

void group_done(int width) { block_->groups[width][threadIdx_.x / width]->arrive_and_wait(); }

namespace {
struct Capture {
    dim3 grid, block;
    size_t lds;
    std::function<void()> body;
    bool concurrent;
};
hipStream_t g_capturing = nullptr;
std::vector<Capture> g_captured;
}  // namespace

// Fresh allocations and LDS hold garbage, like device memory (RMX_EMU_FILL: a byte value,
// or "random").
static void fill_garbage(void* p, size_t n) {
    static uint64_t state = 0x9E3779B97F4A7C15ull;
    const char* e = std::getenv("RMX_EMU_FILL");
    if (n == 0) return;
    unsigned char* c = static_cast<unsigned char*>(p);
    if (e && std::strcmp(e, "random") == 0) {
        for (size_t i = 0; i < n; ++i) {
            state ^= state << 13;
            state ^= state >> 7;
            state ^= state << 17;
            c[i] = (unsigned char)state;
        }
    } else {
        std::memset(c, e ? std::atoi(e) : 0x5A, n);
    }
}


static void init_block(Block& blk, int n, size_t lds) {
    blk.n = n;
    blk.all = std::make_unique<std::barrier<>>(blk.n);
    for (int w : {2, 4, 8, 16, 32, 64}) {
        if (blk.n % w) continue;
        for (int g = 0; g < blk.n / w; ++g)
            blk.groups[w].push_back(std::make_unique<std::barrier<>>(w));
        blk.slots[w].assign(blk.n, 0);
    }
    blk.orv.assign(blk.n, 0);
    blk.lds.assign(lds, 0);
    fill_garbage(blk.lds.data(), lds);
}

static void run(dim3 grid, dim3 block, size_t lds, const std::function<void()>& body) {
    gridDim_ = grid;
    blockDim_ = block;
    Block blk;
    init_block(blk, (int)block.x, lds);
    std::vector<std::thread> th;
    for (int t = 0; t < (int)block.x; ++t) {
        th.emplace_back([&, t]() {
            block_ = &blk;
            threadIdx_ = dim3(t);
            for (unsigned b = 0; b < grid.x; ++b) {
                blockIdx_ = dim3(b);
                body();
                blk.all->arrive_and_wait();
            }
        });
    }
    for (auto& x : th) x.join();
}

// Every block of the launch at once (grid.x * block.x host threads), each block with its
// own barriers and LDS: for kernels whose blocks wait on each other.
static void run_concurrent(dim3 grid, dim3 block, size_t lds,
                           const std::function<void()>& body) {
    gridDim_ = grid;
    blockDim_ = block;
    std::vector<std::unique_ptr<Block>> blks(grid.x);
    for (auto& b : blks) {
        b = std::make_unique<Block>();
        init_block(*b, (int)block.x, lds);
    }
    std::vector<std::thread> th;
    for (unsigned g = 0; g < grid.x; ++g)
        for (int t = 0; t < (int)block.x; ++t)
            th.emplace_back([&, g, t]() {
                block_ = blks[g].get();
                threadIdx_ = dim3(t);
                blockIdx_ = dim3(g);
                body();
            });
    for (auto& x : th) x.join();
}

void launch(dim3 grid, dim3 block, size_t lds, hipStream_t st, std::function<void()> body,
            bool concurrent) {
    if (st && st == g_capturing) {
        g_captured.push_back(Capture{grid, block, lds, body, concurrent});
        return;
    }
    if (concurrent)
        run_concurrent(grid, block, lds, body);
    else
        run(grid, block, lds, body);
}

struct Graph {
    std::vector<Capture> nodes;
};

hipError_t begin_capture(hipStream_t s) {
    g_capturing = s;
    g_captured.clear();
    return hipSuccess;
}
hipError_t end_capture(hipStream_t, hipGraph_t* g) {
    auto* gr = new Graph{g_captured};
    g_captured.clear();
    g_capturing = nullptr;
    *g = reinterpret_cast<hipGraph_t>(gr);
    return hipSuccess;
}
void replay(hipGraph_t g) {
    for (auto& c : reinterpret_cast<Graph*>(g)->nodes) {
        if (c.concurrent)
            run_concurrent(c.grid, c.block, c.lds, c.body);
        else
            run(c.grid, c.block, c.lds, c.body);
    }
}
void destroy(hipGraph_t g) { delete reinterpret_cast<Graph*>(g); }

}  // namespace rmx_emu

int __syncthreads_or(int p) {
    auto* b = rmx_emu::block_;
    b->orv[threadIdx.x] = p ? 1 : 0;
    __syncthreads();
    int r = 0;
    for (int v : b->orv) r |= v;
    __syncthreads();
    return r;
}

struct rmx_emu_stream { int dummy; };
struct rmx_emu_event { std::chrono::steady_clock::time_point t; };

hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
    // compute units: 1, or RMX_EMU_CUS (to exercise grids spread over several XCDs)
    const char* cus = std::getenv("RMX_EMU_CUS");
    *v = a == hipDeviceAttributeMaxSharedMemoryPerBlock ? 160 * 1024 : (cus ? std::atoi(cus) : 1);
    return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
    *p = std::malloc(n ? n : 1);
    if (*p) rmx_emu::fill_garbage(*p, n);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
    std::memcpy(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) {
    return hipMemcpy(d, s, n, k);
}
hipError_t hipMemset(void* d, int v, size_t n) { std::memset(d, v, n); return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    *s = new rmx_emu_stream{0};
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new rmx_emu_event{}; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    e->t = std::chrono::steady_clock::now();
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }   // emulated work is synchronous
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    return rmx_emu::begin_capture(s);
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) { return rmx_emu::end_capture(s, g); }
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    *e = g;
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) { rmx_emu::replay(e); return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { rmx_emu::destroy(g); return hipSuccess; }

// Red zones between workspace regions (the emulation build of the host core records
// them): the whole workspace is made addressable, then each zone is poisoned.
#include <sanitizer/asan_interface.h>
#include <utility>
namespace rmx {
void rmx_emu_poison_gaps(void* ws, size_t ws_bytes,
                         const std::vector<std::pair<size_t, size_t>>& gaps) {
    char* base = static_cast<char*>(ws);
    ASAN_UNPOISON_MEMORY_REGION(base, ws_bytes);
    for (const auto& g : gaps)
        if (g.first + g.second <= ws_bytes) ASAN_POISON_MEMORY_REGION(base + g.first, g.second);
}
}  // namespace rmx
