// Right-hand sides of the time steppers that carry the line-by-line operator
// (the paper's heat example, Sec. 3.4, and wave example, Sec. 3.5), each one
// matrix-free pass over the node fields (the band-tile kernel of
// field_ops.hip), and the per-island weighted sums of the quantity-of-interest
// studies (Sec. 3.6).
#include <math.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace eb {

// ------------------------------------------------ per-island weighted sums
// Linear quantities of interest w . u of several solutions over the islands
// of a canvas (Sec. 3.6: the value at a node, the integral over a region).
// Pass 1: block (c, s, j) sums w * x over chunk c (SEG_CHUNK consecutive
// nodes) of segment s of field j; pass 2: one block per (j, s) adds its
// chunks' partials.  Every sum is taken in a fixed order.
constexpr int SEG_NT = 256;
constexpr int SEG_PER_THREAD = 8;
constexpr int64_t SEG_CHUNK = (int64_t)SEG_NT * SEG_PER_THREAD;

__global__ void __launch_bounds__(SEG_NT) k_seg_partials(const double* __restrict__ w, const double* __restrict__ x,
                                                         int64_t field_nodes, const int64_t* __restrict__ seg_lo,
                                                         const int64_t* __restrict__ seg_hi, int nseg, int nchunk,
                                                         double* __restrict__ part) {
    __shared__ double lds[SEG_NT / WAVE];
    const int c = blockIdx.x, sg = blockIdx.y, j = blockIdx.z;
    const int64_t lo = seg_lo[sg] + (int64_t)c * SEG_CHUNK;
    const int64_t hi = min(seg_hi[sg], lo + SEG_CHUNK);
    const double* xj = x + (int64_t)j * field_nodes;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < SEG_PER_THREAD; ++k) {
        const int64_t n = lo + (int64_t)k * SEG_NT + threadIdx.x;
        if (n < hi) v = fma(w[n], xj[n], v);
    }
    const double t = block_sum<SEG_NT>(v, lds);
    if (threadIdx.x == 0) part[((int64_t)j * nseg + sg) * nchunk + c] = t;
}

__global__ void __launch_bounds__(SEG_NT) k_seg_final(const double* __restrict__ part, int nchunk,
                                                      double* __restrict__ out) {
    __shared__ double lds[SEG_NT / WAVE];
    const int64_t js = blockIdx.x;
    double v = 0.0;
    for (int c = threadIdx.x; c < nchunk; c += SEG_NT) v += part[js * nchunk + c];
    const double t = block_sum<SEG_NT>(v, lds);
    if (threadIdx.x == 0) out[js] = t;
}

}  // namespace eb

using namespace eb;

namespace eb {

// Fixed scratch of eb_segment_dots_noalloc: segment bounds, chunk partials
// and results of one call.  Each GPU that runs the call holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in there).
constexpr size_t SEG_SCRATCH_BYTES = (size_t)8 << 20;
static __device__ __align__(256) double scratch[SEG_SCRATCH_BYTES / sizeof(double)];

static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[64] = {nullptr};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current).
static int scratch_address(void** out) {
    int dev = 0;
    EB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("eb_segment_dots_noalloc: device id %d out of range", dev);
        return EB_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        EB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return EB_OK;
}

// Argument checks and per-segment node bounds (lo for every segment, then hi).
static int segment_bounds(const char* name, const double* w, const double* x, int32_t nfields, int64_t field_nodes,
                          int64_t row_len, int32_t nseg, const int32_t* seg_rows, const double* out,
                          std::vector<int64_t>* lohi, int* nchunk) {
    if (!w || !x || !seg_rows || !out) {
        set_error("%s: null pointer", name);
        return EB_EINVAL;
    }
    if (nfields < 1 || nfields > 65535 || nseg < 1 || nseg > 65535 || row_len < 1 || field_nodes < 1) {
        set_error("%s: need 1 <= nfields, nseg <= 65535 and positive row_len, field_nodes", name);
        return EB_EINVAL;
    }
    lohi->assign(2 * (size_t)nseg, 0);
    int64_t longest = 0;
    for (int s = 0; s < nseg; ++s) {
        const int64_t r0 = seg_rows[s], r1 = seg_rows[s + 1];
        if (r0 < 0 || r1 < r0 || r1 * row_len > field_nodes) {
            set_error("%s: segment %d rows [%lld, %lld) outside the field", name, s, (long long)r0, (long long)r1);
            return EB_EINVAL;
        }
        (*lohi)[s] = r0 * row_len;
        (*lohi)[nseg + s] = r1 * row_len;
        longest = std::max(longest, (r1 - r0) * row_len);
    }
    const int64_t nchunk64 = std::max<int64_t>(1, (longest + SEG_CHUNK - 1) / SEG_CHUNK);
    if (nchunk64 > INT32_MAX) {
        set_error("%s: segment too long", name);
        return EB_EINVAL;
    }
    *nchunk = (int)nchunk64;
    return EB_OK;
}

// The two passes on caller-provided device buffers: dlohi (2 nseg int64),
// part (nfields nseg nchunk doubles), dout (nfields nseg doubles); then the
// results to the host.  Every element of part and dout is written before it
// is read.
static int segment_dots_run(const char* name, const double* w, const double* x, int32_t nfields,
                            int64_t field_nodes, int32_t nseg, const std::vector<int64_t>& lohi, int nchunk,
                            int64_t* dlohi, double* part, double* dout, double* out, hipStream_t s) {
    const int64_t nout = (int64_t)nfields * nseg;
    if (hipMemcpyAsync(dlohi, lohi.data(), sizeof(int64_t) * lohi.size(), hipMemcpyHostToDevice, s) != hipSuccess) {
        set_error("%s: copy to the device failed", name);
        return EB_EHIP;
    }
    hipLaunchKernelGGL(k_seg_partials, dim3(nchunk, nseg, nfields), dim3(SEG_NT), 0, s, w, x, field_nodes, dlohi,
                       dlohi + nseg, nseg, nchunk, part);
    hipLaunchKernelGGL(k_seg_final, dim3((unsigned)nout), dim3(SEG_NT), 0, s, part, nchunk, dout);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(out, dout, sizeof(double) * nout, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("%s: kernel launch or copy failed", name);
        return EB_EHIP;
    }
    return EB_OK;
}

}  // namespace eb

extern "C" int eb_segment_dots(const double* w, const double* x, int32_t nfields, int64_t field_nodes,
                               int64_t row_len, int32_t nseg, const int32_t* seg_rows, double* out, void* stream) {
    clear_error();
    std::vector<int64_t> lohi;
    int nchunk = 0;
    EB_TRY(segment_bounds("eb_segment_dots", w, x, nfields, field_nodes, row_len, nseg, seg_rows, out, &lohi,
                          &nchunk));
    hipStream_t s = (hipStream_t)stream;
    const int64_t nout = (int64_t)nfields * nseg;
    int64_t* dlohi = nullptr;
    double* part = nullptr;
    EB_TRY(dalloc_n(&dlohi, 2 * (int64_t)nseg, s));
    int rc = dalloc_n(&part, nout * nchunk + nout, s);
    if (rc == EB_OK)
        rc = segment_dots_run("eb_segment_dots", w, x, nfields, field_nodes, nseg, lohi, nchunk, dlohi, part,
                              part + nout * nchunk, out, s);
    (void)dfree(part, s);
    (void)dfree(dlohi, s);
    return rc;
}

extern "C" int eb_segment_dots_noalloc(const double* w, const double* x, int32_t nfields, int64_t field_nodes,
                                       int64_t row_len, int32_t nseg, const int32_t* seg_rows, double* out,
                                       void* stream) {
    clear_error();
    std::vector<int64_t> lohi;
    int nchunk = 0;
    EB_TRY(segment_bounds("eb_segment_dots_noalloc", w, x, nfields, field_nodes, row_len, nseg, seg_rows, out,
                          &lohi, &nchunk));
    const int64_t nout = (int64_t)nfields * nseg;
    // scratch layout: bounds (2 nseg int64), partials, results
    const int64_t need = (int64_t)sizeof(int64_t) * 2 * nseg + (int64_t)sizeof(double) * (nout * nchunk + nout);
    if (need > (int64_t)SEG_SCRATCH_BYTES) {
        set_error("eb_segment_dots_noalloc: needs %lld bytes of scratch, more than its fixed %zu (fewer fields, "
                  "segments or shorter segments; or use eb_segment_dots)", (long long)need, SEG_SCRATCH_BYTES);
        return EB_ENOSPC;
    }
    void* base = nullptr;
    EB_TRY(scratch_address(&base));
    int64_t* dlohi = (int64_t*)base;
    double* part = (double*)base + 2 * (int64_t)nseg;
    return segment_dots_run("eb_segment_dots_noalloc", w, x, nfields, field_nodes, nseg, lohi, nchunk, dlohi, part,
                            part + nout * nchunk, out, (hipStream_t)stream);
}

static int wave_rhs_impl(const eb_grid_t* g, const int8_t* kind, const double* a, const double* cond, double theta,
                         double dt, double scale, const double* un, const double* unm1, double* out, void* stream) {
    clear_error();
    GridDims d;
    EB_TRY(make_dims(g, &d));
    if (!kind || !a || !un || !unm1 || !out) {
        set_error("eb_wave_rhs: null pointer");
        return EB_EINVAL;
    }
    if (!(theta >= 0.0) || !(dt > 0.0) || !isfinite(scale)) {
        set_error("eb_wave_rhs: theta must be >= 0, dt > 0 and scale finite");
        return EB_EINVAL;
    }
    if (out == un || out == unm1) {
        set_error("eb_wave_rhs: out must not overlap un or unm1");
        return EB_EINVAL;
    }
    FieldCoefs co;
    co.c0 = 1.0 - 2.0 * theta;
    co.c1 = theta;
    co.scale = scale;
    co.dt2 = dt * dt;
    return launch_field_op(1, d, kind, a, cond, un, unm1, nullptr, nullptr, out, co, (hipStream_t)stream);
}

extern "C" int eb_wave_rhs(const eb_grid_t* g, const int8_t* kind, const double* a, double theta, double dt,
                           double scale, const double* un, const double* unm1, double* out, void* stream) {
    return wave_rhs_impl(g, kind, a, nullptr, theta, dt, scale, un, unm1, out, stream);
}

extern "C" int eb_wave_rhs_beta(const eb_grid_t* g, const int8_t* kind, const double* a, const double* cond,
                                double theta, double dt, double scale, const double* un, const double* unm1,
                                double* out, void* stream) {
    if (!cond) {
        set_error("eb_wave_rhs_beta: null conductivity");
        return EB_EINVAL;
    }
    return wave_rhs_impl(g, kind, a, cond, theta, dt, scale, un, unm1, out, stream);
}

static int combine_impl(const eb_grid_t* g, const int8_t* kind, const double* a, const double* cond, double sigma,
                        double alpha, const double* x, double beta, const double* y, double gamma, const double* z,
                        double* out, void* stream) {
    clear_error();
    GridDims d;
    EB_TRY(make_dims(g, &d));
    if (!kind || !a || !x || !out || (beta != 0.0 && !y) || (gamma != 0.0 && !z)) {
        set_error("eb_stencil_combine: null pointer");
        return EB_EINVAL;
    }
    if (out == x) {
        set_error("eb_stencil_combine: out must not overlap x");
        return EB_EINVAL;
    }
    FieldCoefs co;
    co.sigma = sigma;
    co.alpha = alpha;
    co.beta = beta;
    co.gamma = gamma;
    return launch_field_op(2, d, kind, a, cond, x, nullptr, beta != 0.0 ? y : nullptr, gamma != 0.0 ? z : nullptr,
                           out, co, (hipStream_t)stream);
}

extern "C" int eb_stencil_combine(const eb_grid_t* g, const int8_t* kind, const double* a, double sigma,
                                  double alpha, const double* x, double beta, const double* y, double gamma,
                                  const double* z, double* out, void* stream) {
    return combine_impl(g, kind, a, nullptr, sigma, alpha, x, beta, y, gamma, z, out, stream);
}

extern "C" int eb_stencil_combine_beta(const eb_grid_t* g, const int8_t* kind, const double* a, const double* cond,
                                       double sigma, double alpha, const double* x, double beta, const double* y,
                                       double gamma, const double* z, double* out, void* stream) {
    if (!cond) {
        set_error("eb_stencil_combine_beta: null conductivity");
        return EB_EINVAL;
    }
    return combine_impl(g, kind, a, cond, sigma, alpha, x, beta, y, gamma, z, out, stream);
}
