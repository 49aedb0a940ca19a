// Host runtime pieces: error state, pooled allocation, scans, small helpers.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <unordered_map>
#include <utility>

#include "common.hpp"

namespace eb {

static thread_local char g_last_error[1024] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

void clear_error() { g_last_error[0] = 0; }

// ------------------------------------------------------- caching allocator
// Device blocks come from hipMalloc once and are then recycled by size inside
// the library: freeing a block returns it to a per-device free list, and an
// allocation reuses the smallest cached block that is large enough (at most
// twice the request).  The driver's own alloc/free calls cost tens to
// hundreds of microseconds each, which would dominate a setup that builds and
// frees dozens of arrays.  Reuse is stream ordered: a block freed on stream s
// is handed out again on s at once; on another stream the device is
// synchronised first (rare: callers normally keep one stream).
namespace {

struct CachedBlock {
    size_t bytes;
    hipStream_t stream;
};

struct DeviceCache {
    std::multimap<size_t, std::pair<void*, hipStream_t>> free_blocks;
    std::unordered_map<void*, size_t> live;
    size_t cached_bytes = 0;
};

std::mutex g_cache_mutex;
DeviceCache g_cache[64];

// caller-supplied allocator of the innermost AllocScope on this thread, and
// the blocks taken from such allocators (keyed by pointer)
thread_local const amg_params_t* g_alloc_scope = nullptr;
struct UserBlock {
    eb_free_fn free_fn;
    void* ctx;
};
std::unordered_map<void*, UserBlock> g_user_live;

size_t round_bytes(size_t b) {
    const size_t g = b <= (1 << 20) ? 256 : (1 << 16);
    return (b + g - 1) / g * g;
}

}  // namespace

AllocScope::AllocScope(const amg_params_t* p) : prev_(g_alloc_scope) {
    if (p && p->alloc && p->free) g_alloc_scope = p;
}

AllocScope::~AllocScope() { g_alloc_scope = prev_; }

int dalloc(void** p, size_t bytes, hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        set_error("dalloc: no current device");
        return EB_EHIP;
    }
    const size_t want = round_bytes(bytes);
    if (const amg_params_t* u = g_alloc_scope) {
        void* ptr = u->alloc(want, (void*)s, u->alloc_ctx);
        if (!ptr) {
            set_error("the caller's allocator returned NULL for %zu bytes", want);
            *p = nullptr;
            return EB_EHIP;
        }
        std::lock_guard<std::mutex> lock(g_cache_mutex);
        g_user_live[ptr] = UserBlock{u->free, u->alloc_ctx};
        *p = ptr;
        return EB_OK;
    }
    {
        std::lock_guard<std::mutex> lock(g_cache_mutex);
        DeviceCache& C = g_cache[dev];
        auto it = C.free_blocks.lower_bound(want);
        if (it != C.free_blocks.end() && it->first <= 2 * want) {
            void* ptr = it->second.first;
            hipStream_t old = it->second.second;
            const size_t sz = it->first;
            C.free_blocks.erase(it);
            C.cached_bytes -= sz;
            C.live[ptr] = sz;
            if (old != s) (void)hipDeviceSynchronize();
            *p = ptr;
            return EB_OK;
        }
    }
    void* ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        // release cached blocks and retry once
        (void)hipGetLastError();
        eb_cache_release_all();
        e = hipMalloc(&ptr, want);
    }
    if (e != hipSuccess) {
        set_error("hipMalloc(%zu bytes) failed: %s", want, hipGetErrorString(e));
        *p = nullptr;
        return EB_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    g_cache[dev].live[ptr] = want;
    *p = ptr;
    return EB_OK;
}

int dfree(void* p, hipStream_t s) {
    if (!p) return EB_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        set_error("dfree: no current device");
        return EB_EHIP;
    }
    std::unique_lock<std::mutex> lock(g_cache_mutex);
    auto ub = g_user_live.find(p);
    if (ub != g_user_live.end()) {
        const UserBlock blk = ub->second;
        g_user_live.erase(ub);
        lock.unlock();
        blk.free_fn(p, (void*)s, blk.ctx);
        return EB_OK;
    }
    DeviceCache& C = g_cache[dev];
    auto it = C.live.find(p);
    if (it == C.live.end()) {
        set_error("dfree: pointer not owned by the library");
        return EB_EINVAL;
    }
    const size_t sz = it->second;
    C.live.erase(it);
    C.free_blocks.emplace(sz, std::make_pair(p, s));
    C.cached_bytes += sz;
    return EB_OK;
}

void eb_cache_release_all() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> lock(g_cache_mutex);
    DeviceCache& C = g_cache[dev];
    for (auto& kv : C.free_blocks) (void)hipFree(kv.second.first);
    C.free_blocks.clear();
    C.cached_bytes = 0;
}

int read_device_i32(const int32_t* dptr, int32_t* host, hipStream_t s) {
    EB_HIP(hipMemcpyAsync(host, dptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    EB_HIP(hipStreamSynchronize(s));
    return EB_OK;
}

int read_device_i64(const int64_t* dptr, int64_t* host, hipStream_t s) {
    EB_HIP(hipMemcpyAsync(host, dptr, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    EB_HIP(hipStreamSynchronize(s));
    return EB_OK;
}

int make_dims(const eb_grid_t* g, GridDims* d) {
    if (!g || (g->dim != 2 && g->dim != 3) || !(g->h > 0.0)) {
        set_error("invalid grid (dim must be 2 or 3, h > 0)");
        return EB_EINVAL;
    }
    for (int a = 0; a < g->dim; ++a) {
        if (g->n[a] < 2 || g->n[a] > (1 << 20)) {
            set_error("invalid grid: n[%d] = %d", a, g->n[a]);
            return EB_EINVAL;
        }
    }
    d->dim = g->dim;
    d->nx = g->n[0] + 1;
    d->ny = g->n[1] + 1;
    d->nz = g->dim == 3 ? g->n[2] + 1 : 1;
    int64_t total = (int64_t)d->nx * d->ny * d->nz;
    if (total >= ((int64_t)1 << 31)) {
        set_error("grid has %lld nodes; at most 2^31 - 1 are supported", (long long)total);
        return EB_EINVAL;
    }
    d->sy = d->nx;
    d->sz = (int64_t)d->nx * d->ny;
    d->x0 = g->x0[0];
    d->y0 = g->x0[1];
    d->z0 = g->dim == 3 ? g->x0[2] : 0.0;
    d->h = g->h;
    d->s = 1.0 / (g->h * g->h);
    return EB_OK;
}

// ------------------------------------------------------------ side stream
namespace {
std::mutex g_side_mutex;
hipStream_t g_side[64] = {};
}  // namespace

int side_stream(hipStream_t* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        set_error("side_stream: no current device");
        return EB_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_side_mutex);
    if (!g_side[dev]) EB_HIP(hipStreamCreateWithFlags(&g_side[dev], hipStreamNonBlocking));
    *out = g_side[dev];
    return EB_OK;
}

// ------------------------------------------------------------------- fill
struct FillList {
    uint32_t* p[FILL_MAX];
    int64_t words[FILL_MAX];
    uint32_t word[FILL_MAX];
};

// blockIdx.y = buffer; 16-byte stores where the buffer is 16-byte aligned.
__global__ void __launch_bounds__(BLOCK) k_fill_many(FillList L) {
    const int b = blockIdx.y;
    uint32_t* p = L.p[b];
    const int64_t nw = L.words[b];
    const uint32_t w = L.word[b];
    const int64_t stride = (int64_t)gridDim.x * BLOCK;
    const int64_t t0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    int64_t head = 0;
    if (((uintptr_t)p & 15) == 0) {
        const int64_t n4 = nw / 4;
        uint4* q = reinterpret_cast<uint4*>(p);
        const uint4 v = make_uint4(w, w, w, w);
        for (int64_t i = t0; i < n4; i += stride) q[i] = v;
        head = n4 * 4;
    }
    for (int64_t i = head + t0; i < nw; i += stride) p[i] = w;
}

int fill_words(const FillSpec* items, int count, hipStream_t s) {
    if (count <= 0) return EB_OK;
    if (count > FILL_MAX) {
        set_error("fill_words: %d buffers (limit %d)", count, FILL_MAX);
        return EB_EINVAL;
    }
    FillList L;
    memset(&L, 0, sizeof(L));
    int64_t most = 0;
    for (int i = 0; i < count; ++i) {
        if (items[i].bytes % 4 != 0 || (items[i].bytes > 0 && !items[i].p)) {
            set_error("fill_words: bad buffer %d", i);
            return EB_EINVAL;
        }
        L.p[i] = static_cast<uint32_t*>(items[i].p);
        L.words[i] = (int64_t)(items[i].bytes / 4);
        L.word[i] = items[i].word;
        if (L.words[i] > most) most = L.words[i];
    }
    int64_t gx = (most / 4 + BLOCK - 1) / BLOCK;
    if (gx < 1) gx = 1;
    if (gx > 2048) gx = 2048;
    hipLaunchKernelGGL(k_fill_many, dim3((unsigned)gx, (unsigned)count), dim3(BLOCK), 0, s, L);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// ------------------------------------------------------------------- scan
// Exclusive scan of integers (exact, so any summation order gives the same
// result).  Tiles of SCAN_TILE elements: a first pass writes each tile's sum;
// the second pass scans each tile and adds the sum of all earlier tiles,
// which every workgroup adds up itself while there are at most
// SCAN_DIRECT_TILES tiles (two launches, no flags, no extra pass over the
// output); above that the tile sums are scanned recursively first.  A single
// tile is one launch.
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;
constexpr int64_t SCAN_DIRECT_TILES = 4096;

constexpr int SCAN_WAVES = BLOCK / WAVE;

// Sum over the block (integers: exact in any order): within each wavefront
// by lane exchanges, then the wavefront totals through LDS (one barrier).
template <class T>
__device__ __forceinline__ T block_sum(T v, T* lds) {
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) lds[threadIdx.x / WAVE] = v;
    __syncthreads();
    T r = 0;
#pragma unroll
    for (int w = 0; w < SCAN_WAVES; ++w) r += lds[w];
    __syncthreads();
    return r;
}

template <class TI, class TO>
__global__ void __launch_bounds__(BLOCK) k_scan_reduce(const TI* __restrict__ in, int64_t n, TO* __restrict__ sums) {
    __shared__ TO lds[SCAN_WAVES];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    TO acc = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t idx = base + (int64_t)i * BLOCK + threadIdx.x;
        if (idx < n) acc += (TO)in[idx];
    }
    acc = block_sum(acc, lds);
    if (threadIdx.x == 0) sums[blockIdx.x] = acc;
}

// MODE 0: single tile (offset 0); 1: offset = sum of tile_val[0 .. tile);
// 2: offset = tile_val[tile] (already an exclusive scan of the tile sums).
template <class TI, class TO, int MODE>
__global__ void __launch_bounds__(BLOCK) k_scan_tiles(const TI* __restrict__ in, TO* __restrict__ out, int64_t n,
                                                      const TO* __restrict__ tile_val, int64_t ntiles,
                                                      TO* __restrict__ total) {
    __shared__ TO lds[SCAN_WAVES];
    TO offset = 0;
    if (MODE == 1) {
        TO acc = 0;
        for (int64_t t = threadIdx.x; t < (int64_t)blockIdx.x; t += BLOCK) acc += tile_val[t];
        offset = block_sum(acc, lds);
    } else if (MODE == 2) {
        offset = tile_val[blockIdx.x];
    }
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    TO v[SCAN_ITEMS];
    TO run = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t idx = base + i;
        const TO x = idx < n ? (TO)in[idx] : (TO)0;
        v[i] = run;
        run += x;
    }
    // inclusive scan of the thread totals within the wavefront (lane
    // exchanges), then the wavefront totals through LDS
    const int lane = (int)(threadIdx.x & (WAVE - 1)), wv = (int)(threadIdx.x / WAVE);
    TO inc = run;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const TO y = __shfl_up(inc, off, WAVE);
        if (lane >= off) inc += y;
    }
    if (lane == WAVE - 1) lds[wv] = inc;
    __syncthreads();
    TO before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < SCAN_WAVES; ++w) {
        if (w < wv) before += lds[w];
        all += lds[w];
    }
    const TO prefix = offset + before + (inc - run);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const int64_t idx = base + i;
        if (idx < n) out[idx] = v[i] + prefix;
    }
    if (threadIdx.x == BLOCK - 1 && (int64_t)blockIdx.x == ntiles - 1) *total = offset + all;
}

template <class TI, class TO>
static int scan_impl(const TI* in, TO* out, int64_t n, TO* total_dev, hipStream_t s) {
    if (n <= 0) {
        EB_HIP(hipMemsetAsync(total_dev, 0, sizeof(TO), s));
        return EB_OK;
    }
    const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles == 1) {
        hipLaunchKernelGGL((k_scan_tiles<TI, TO, 0>), dim3(1), dim3(BLOCK), 0, s, in, out, n, (const TO*)nullptr,
                           ntiles, total_dev);
        EB_LAUNCH_CHECK();
        return EB_OK;
    }
    TO* sums = nullptr;
    EB_TRY(dalloc_n(&sums, ntiles, s));
    hipLaunchKernelGGL((k_scan_reduce<TI, TO>), dim3((unsigned)ntiles), dim3(BLOCK), 0, s, in, n, sums);
    EB_LAUNCH_CHECK();
    if (ntiles <= SCAN_DIRECT_TILES) {
        hipLaunchKernelGGL((k_scan_tiles<TI, TO, 1>), dim3((unsigned)ntiles), dim3(BLOCK), 0, s, in, out, n,
                           (const TO*)sums, ntiles, total_dev);
        EB_LAUNCH_CHECK();
    } else {
        TO* sums_scan = nullptr;
        TO* dummy_total = nullptr;
        EB_TRY(dalloc_n(&sums_scan, ntiles, s));
        EB_TRY(dalloc_n(&dummy_total, 1, s));
        EB_TRY((scan_impl<TO, TO>(sums, sums_scan, ntiles, dummy_total, s)));
        hipLaunchKernelGGL((k_scan_tiles<TI, TO, 2>), dim3((unsigned)ntiles), dim3(BLOCK), 0, s, in, out, n,
                           (const TO*)sums_scan, ntiles, total_dev);
        EB_LAUNCH_CHECK();
        EB_TRY(dfree(dummy_total, s));
        EB_TRY(dfree(sums_scan, s));
    }
    EB_TRY(dfree(sums, s));
    return EB_OK;
}

int scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* total_host, hipStream_t s) {
    int64_t* tot = nullptr;
    EB_TRY(dalloc_n(&tot, 1, s));
    EB_TRY((scan_impl<int32_t, int64_t>(in, out, n, tot, s)));
    if (total_host) EB_TRY(read_device_i64(tot, total_host, s));
    EB_TRY(dfree(tot, s));
    return EB_OK;
}

int scan_i32(const int32_t* in, int32_t* out, int64_t n, int64_t* total_host, hipStream_t s) {
    int32_t* tot = nullptr;
    EB_TRY(dalloc_n(&tot, 1, s));
    EB_TRY((scan_impl<int32_t, int32_t>(in, out, n, tot, s)));
    if (total_host) {
        int32_t t = 0;
        EB_TRY(read_device_i32(tot, &t, s));
        *total_host = t;
    }
    EB_TRY(dfree(tot, s));
    return EB_OK;
}

int scan_i32_dev(const int32_t* in, int32_t* out, int64_t n, int32_t* total_dev, hipStream_t s) {
    return scan_impl<int32_t, int32_t>(in, out, n, total_dev, s);
}

int scan_i32_to_i64_dev(const int32_t* in, int64_t* out, int64_t n, int64_t* total_dev, hipStream_t s) {
    return scan_impl<int32_t, int64_t>(in, out, n, total_dev, s);
}

}  // namespace eb

extern "C" {

const char* eb_last_error(void) { return eb::g_last_error; }

const char* eb_strerror(int code) {
    switch (code) {
        case EB_OK: return "success";
        case EB_EINVAL: return "invalid argument";
        case EB_EDOMAIN: return "domain reaches the outermost node layer";
        case EB_ENOSPC: return "output capacity too small";
        case EB_ENOTSPD: return "operator is not symmetric positive definite";
        case EB_ENAN: return "NaN or Inf in the solve";
        case EB_ENOCONV: return "iteration limit reached";
        case EB_EHIP: return "HIP runtime error";
        case EB_ENOTIMPL: return "not implemented";
        case EB_EGEOM: return "boundary points for an RBF row not found (collinear interpolation points)";
        default: return "unknown error";
    }
}

int eb_abi_version(void) { return EBAMG_ABI_VERSION; }

void eb_release_cached_memory(void) { eb::eb_cache_release_all(); }

}  // extern "C"
