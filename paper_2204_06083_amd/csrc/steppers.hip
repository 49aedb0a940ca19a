// Right-hand sides of the time steppers that carry the line-by-line operator
// (the paper's heat example, Sec. 3.4, and wave example, Sec. 3.5): one pass
// over the node fields each, with the operator applied matrix-free as in
// stencil_apply, A v = (1/h^2)(a v - sum of v over computational neighbours).
#include <math.h>

#include "common.hpp"

namespace eb {

// out = scale (2 un - unm1 - dt^2 A v), v = (1 - 2 theta) un + theta unm1,
// at computational points; 0 elsewhere.
__global__ void __launch_bounds__(BLOCK) k_wave_rhs(const int8_t* __restrict__ kind, const double* __restrict__ a,
                                                    GridDims d, int64_t nnodes, double theta, double dt2,
                                                    double scale, const double* __restrict__ un,
                                                    const double* __restrict__ unm1, double* __restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= nnodes) return;
    const NodePos p = node_pos(n, d);
    if (kind[n] != 2 || on_outer_layer(p, d)) {
        out[n] = 0.0;
        return;
    }
    const double c0 = 1.0 - 2.0 * theta;
    auto v = [&](int64_t m) { return c0 * un[m] + theta * unm1[m]; };
    double nb = 0.0;
    for (int axis = 0; axis < d.dim; ++axis) {
        const int64_t st = axis_stride(d, axis);
        if (kind[n - st] == 2) nb = nb + v(n - st);
        if (kind[n + st] == 2) nb = nb + v(n + st);
    }
    const double av = (a[n] * d.s) * v(n) - d.s * nb;
    out[n] = scale * ((2.0 * un[n] - unm1[n]) - dt2 * av);
}

// out = alpha ((A + sigma I) x) + beta y + gamma z at computational points; 0
// elsewhere (y or z may be null when their coefficient is 0).
__global__ void __launch_bounds__(BLOCK) k_stencil_combine(const int8_t* __restrict__ kind,
                                                           const double* __restrict__ a, GridDims d, int64_t nnodes,
                                                           double sigma, double alpha, const double* __restrict__ x,
                                                           double beta, const double* __restrict__ y, double gamma,
                                                           const double* __restrict__ z, double* __restrict__ out) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= nnodes) return;
    const NodePos p = node_pos(n, d);
    if (kind[n] != 2 || on_outer_layer(p, d)) {
        out[n] = 0.0;
        return;
    }
    double nb = 0.0;
    for (int axis = 0; axis < d.dim; ++axis) {
        const int64_t st = axis_stride(d, axis);
        if (kind[n - st] == 2) nb = nb + x[n - st];
        if (kind[n + st] == 2) nb = nb + x[n + st];
    }
    const double ax = (a[n] * d.s + sigma) * x[n] - d.s * nb;
    double r = alpha * ax;
    if (y) r += beta * y[n];
    if (z) r += gamma * z[n];
    out[n] = r;
}

}  // namespace eb

using namespace eb;

extern "C" int eb_wave_rhs(const eb_grid_t* g, const int8_t* kind, const double* a, double theta, double dt,
                           double scale, const double* un, const double* unm1, double* out, void* stream) {
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
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    hipLaunchKernelGGL(k_wave_rhs, dim3(grid_for(nn)), dim3(BLOCK), 0, (hipStream_t)stream, kind, a, d, nn, theta,
                       dt * dt, scale, un, unm1, out);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

extern "C" int eb_stencil_combine(const eb_grid_t* g, const int8_t* kind, const double* a, double sigma,
                                  double alpha, const double* x, double beta, const double* y, double gamma,
                                  const double* z, double* out, void* stream) {
    clear_error();
    GridDims d;
    EB_TRY(make_dims(g, &d));
    if (!kind || !a || !x || !out || (beta != 0.0 && !y) || (gamma != 0.0 && !z)) {
        set_error("eb_stencil_combine: null pointer");
        return EB_EINVAL;
    }
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    hipLaunchKernelGGL(k_stencil_combine, dim3(grid_for(nn)), dim3(BLOCK), 0, (hipStream_t)stream, kind, a, d, nn,
                       sigma, alpha, x, beta, beta != 0.0 ? y : nullptr, gamma, gamma != 0.0 ? z : nullptr, out);
    EB_LAUNCH_CHECK();
    return EB_OK;
}
