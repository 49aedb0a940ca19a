// Shared internals of the ebamg library: error state, allocation, launch
// helpers, deterministic wave/block reductions and the device-wide scan.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "ebamg.h"

namespace eb {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

#define EB_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::eb::set_error("%s:%d: %s failed: %s", __FILE__, __LINE__, #call,   \
                            hipGetErrorString(e_));                               \
            return EB_EHIP;                                                       \
        }                                                                         \
    } while (0)

#define EB_TRY(expr)                                                              \
    do {                                                                          \
        int rc_ = (expr);                                                         \
        if (rc_ != EB_OK) return rc_;                                             \
    } while (0)

#define EB_LAUNCH_CHECK() EB_HIP(hipGetLastError())

// ------------------------------------------------------------- allocation
// Device memory from the library's caching allocator (runtime.hip): blocks
// are recycled by size, so repeated setup/free cycles make no driver calls.
int dalloc(void** p, size_t bytes, hipStream_t s);
int dfree(void* p, hipStream_t s);
void eb_cache_release_all();   // synchronise the device, return cached blocks

// While an AllocScope with a caller-supplied allocator (amg_params_t alloc /
// free) is alive on this thread, dalloc takes blocks from it and dfree hands
// them back to it; otherwise both use the caching allocator.
class AllocScope {
  public:
    explicit AllocScope(const amg_params_t* p);
    ~AllocScope();
    AllocScope(const AllocScope&) = delete;
    AllocScope& operator=(const AllocScope&) = delete;

  private:
    const amg_params_t* prev_;
};

template <class T>
int dalloc_n(T** p, int64_t count, hipStream_t s) {
    return dalloc(reinterpret_cast<void**>(p), (size_t)(count > 0 ? count : 1) * sizeof(T), s);
}

// Device error word: kernels OR in flags, host reads at sync points.
enum : int32_t {
    DEVERR_DOMAIN = 1,
    DEVERR_NOSPC = 2,
    DEVERR_NOTSPD = 4,
    DEVERR_NAN = 8,
    DEVERR_CAP = 16,
    DEVERR_GEOM = 32,
};

constexpr int WAVE = 64;
constexpr int BLOCK = 256;

// The GPU hands out workgroups round-robin over its 8 XCDs, each with its own
// L2.  Renumbering blocks so that XCD x owns the contiguous block range
// [x G/8, (x+1) G/8) (G a multiple of 8) keeps neighbouring grid rows, which
// the stencil kernels read from adjacent strips, inside one L2.
constexpr int NUM_XCD = 8;

// A grid rounded up to whole groups of NUM_XCD blocks, so that xcd_block()
// applies (the extra blocks find no row and return).
inline unsigned xcd_grid(unsigned g) { return (g + NUM_XCD - 1) / NUM_XCD * NUM_XCD; }

__device__ inline int64_t xcd_block() {
    const int64_t per = gridDim.x / NUM_XCD;
    if (per == 0 || (gridDim.x % NUM_XCD) != 0) return blockIdx.x;
    return (int64_t)(blockIdx.x % NUM_XCD) * per + blockIdx.x / NUM_XCD;
}

// Value of the lane to the left (lane - 1; 0 in lane 0) and to the right
// (lane + 1; 0 in lane 63): whole-wave DPP shifts, executed by all lanes.
__device__ inline int dpp_from_left(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }
__device__ inline int dpp_from_right(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true); }
__device__ inline double from_left(double v) {
    return __hiloint2double(dpp_from_left(__double2hiint(v)), dpp_from_left(__double2loint(v)));
}
__device__ inline double from_right(double v) {
    return __hiloint2double(dpp_from_right(__double2hiint(v)), dpp_from_right(__double2loint(v)));
}
__device__ inline float from_left(float v) { return __int_as_float(dpp_from_left(__float_as_int(v))); }
__device__ inline float from_right(float v) { return __int_as_float(dpp_from_right(__float_as_int(v))); }

inline unsigned grid_for(int64_t n, int block = BLOCK) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)(g > 0 ? g : 1);
}

// ------------------------------------------------------------- reductions
// Butterfly sum over the 64 lanes of a wavefront; every lane gets the total.
// The pairing order is fixed, so results are reproducible run to run.
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
    return v;
}

// Block sum for blockDim.x == NT (multiple of 64).  Result valid in thread 0.
template <int NT>
__device__ inline double block_sum(double v, double* lds /* NT/64 */) {
    v = wave_sum(v);
    const int lane = threadIdx.x & (WAVE - 1);
    const int w = threadIdx.x / WAVE;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / WAVE; ++i) t += lds[i];
    }
    return t;
}

// ---------------------------------------------------------------- scans
// Exclusive prefix sum of n counts (int32 in, int64 or int32 out).  If
// `total_host` is non-null the grand total is copied back and the stream is
// synchronised.
int scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* total_host, hipStream_t s);
int scan_i32(const int32_t* in, int32_t* out, int64_t n, int64_t* total_host, hipStream_t s);
// Same scans, grand total written to device memory (no synchronisation).
int scan_i32_dev(const int32_t* in, int32_t* out, int64_t n, int32_t* total_dev, hipStream_t s);

// Set several device buffers to a repeated 32-bit word in one launch (bytes a
// multiple of 4; at most FILL_MAX buffers).  Stands in for a run of
// hipMemsetAsync calls, each of which is a launch of its own.
constexpr int FILL_MAX = 12;
struct FillSpec {
    void* p;
    size_t bytes;
    uint32_t word;
};
int fill_words(const FillSpec* items, int count, hipStream_t s);

// A second stream on the current device (non-blocking, default priority,
// created on first use and kept until the process ends) for work that can
// overlap the caller's stream; ordering with it goes through events.
int side_stream(hipStream_t* out);
int scan_i32_to_i64_dev(const int32_t* in, int64_t* out, int64_t n, int64_t* total_dev, hipStream_t s);

// Small helpers used by several translation units.
int read_device_i32(const int32_t* dptr, int32_t* host, hipStream_t s);
int read_device_i64(const int64_t* dptr, int64_t* host, hipStream_t s);

// Geometry of the node grid as seen by kernels.
struct GridDims {
    int dim;
    int nx, ny, nz;          // nodes per axis (nz = 1 in 2-D)
    int64_t sy, sz;          // strides of y and z in the dense user layout
    double x0, y0, z0, h, s; // s = 1/h^2
};

int make_dims(const eb_grid_t* g, GridDims* d);

// Matrix-free operator passes over node fields (field_ops.hip): op 0 applies
// A + sigma I to f0; op 1 forms the wave theta-scheme right-hand side
// scale (2 f0 - f1 - dt2 A (c0 f0 + c1 f1)); op 2 forms
// alpha (A + sigma I) f0 + beta g0 + gamma g1 (g0, g1 may be null).  cond: the
// face conductivities (dim fields back to back) or null.  out is written at
// every node (0 off computational points) and must not overlap f0 or f1.
struct FieldCoefs {
    double c0 = 1.0, c1 = 0.0, sigma = 0.0, alpha = 1.0, beta = 0.0, gamma = 0.0, scale = 1.0, dt2 = 0.0;
};
int launch_field_op(int op, const GridDims& d, const int8_t* kind, const double* a, const double* cond,
                    const double* f0, const double* f1, const double* g0, const double* g1, double* out,
                    const FieldCoefs& co, hipStream_t s);

// Node coordinates of a flat index in the dense user layout.
struct NodePos {
    int i, j, k;
};

__device__ inline NodePos node_pos(int64_t n, const GridDims& d) {
    NodePos p;
    if (n <= 0x7fffffff) {
        // 32-bit division (the usual case: far fewer than 2^31 nodes)
        const uint32_t u = (uint32_t)n, nx = (uint32_t)d.nx, ny = (uint32_t)d.ny;
        const uint32_t r = u / nx;
        p.i = (int)(u - r * nx);
        const uint32_t k = r / ny;
        p.j = (int)(r - k * ny);
        p.k = (int)k;
        return p;
    }
    p.i = (int)(n % d.nx);
    int64_t r = n / d.nx;
    p.j = (int)(r % d.ny);
    p.k = (int)(r / d.ny);
    return p;
}

__device__ inline int axis_coord(const NodePos& p, int axis) {
    return axis == 0 ? p.i : (axis == 1 ? p.j : p.k);
}

__device__ inline int axis_len(const GridDims& d, int axis) {
    return axis == 0 ? d.nx : (axis == 1 ? d.ny : d.nz);
}

__device__ inline int64_t axis_stride(const GridDims& d, int axis) {
    return axis == 0 ? 1 : (axis == 1 ? d.sy : d.sz);
}

// A node of the outermost layer (never an unknown: it has no full stencil).
__device__ inline bool on_outer_layer(const NodePos& p, const GridDims& d) {
    return p.i == 0 || p.i == d.nx - 1 || p.j == 0 || p.j == d.ny - 1 ||
           (d.dim == 3 && (p.k == 0 || p.k == d.nz - 1));
}

}  // namespace eb
