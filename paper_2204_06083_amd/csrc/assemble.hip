// Embedded-boundary assembly kernels: classification, the line-by-line
// diagonal with its cut records, the right-hand side and the matrix-free
// operator on dense node fields.
//
// Built with -ffp-contract=off: the diagonal a_k, q, c and the crossing
// coordinates are evaluated in a fixed order with separately rounded
// operations, so an independent FP64 implementation can reproduce them bit
// for bit (t = psi_in / (psi_in - psi_out); q = (j-1) + t; c = 1/q;
// a_k = n_regular, then a_k += c side by side in the order -x,+x,-y,+y,-z,+z).
#include "common.hpp"

namespace eb {

// ------------------------------------------------------------ classification
// Sec. 2: mask m = [psi < 0]; boundary point = inside with an outside nearest
// neighbour; computational point = inside with all 2d neighbours inside.
__global__ void __launch_bounds__(BLOCK) k_classify(const double* __restrict__ psi, int8_t* __restrict__ kind,
                                                    GridDims d, int64_t nnodes, int32_t* __restrict__ err,
                                                    int32_t* __restrict__ block_unknowns,
                                                    int32_t* __restrict__ ncut) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool active = n < nnodes;
    int8_t kd = 0;
    if (active) {
        const NodePos p = node_pos(n, d);
        const bool inside = psi[n] < 0.0;
        const bool edge = p.i == 0 || p.i == d.nx - 1 || p.j == 0 || p.j == d.ny - 1 ||
                          (d.dim == 3 && (p.k == 0 || p.k == d.nz - 1));
        if (inside) {
            if (edge) {
                atomicOr(err, DEVERR_DOMAIN);
                kd = 1;
            } else {
                int n_in = 0;
                for (int axis = 0; axis < d.dim; ++axis) {
                    const int64_t st = axis_stride(d, axis);
                    n_in += psi[n - st] < 0.0;
                    n_in += psi[n + st] < 0.0;
                }
                kd = n_in == 2 * d.dim ? 2 : 1;
            }
        }
        kind[n] = kd;
        ncut[n] = 0;  // sides are counted once kinds are known (k_count_cuts)
    }
    // unknowns per workgroup, summed afterwards by k_sum_counts (no atomics)
    __shared__ int32_t wcount[BLOCK / WAVE];
    const unsigned long long bal = __ballot(active && kd == 2);
    if ((threadIdx.x & (WAVE - 1)) == 0) wcount[threadIdx.x / WAVE] = (int32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t c = 0;
        for (int w = 0; w < BLOCK / WAVE; ++w) c += wcount[w];
        block_unknowns[blockIdx.x] = c;
    }
}

// total = sum of n counts, one workgroup (integer: exact in any order).
__global__ void __launch_bounds__(1024) k_sum_counts(const int32_t* __restrict__ v, int64_t n,
                                                     unsigned long long* __restrict__ total) {
    __shared__ unsigned long long part[1024 / WAVE];
    unsigned long long acc = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) acc += (unsigned long long)v[i];
    for (int off = WAVE / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < 1024 / WAVE; ++w) t += part[w];
        *total = t;
    }
}

__global__ void __launch_bounds__(BLOCK) k_count_cuts(const int8_t* __restrict__ kind, GridDims d, int64_t nnodes,
                                                      int32_t* __restrict__ ncut) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= nnodes) return;
    int c = 0;
    if (kind[n] == 2) {
        for (int axis = 0; axis < d.dim; ++axis) {
            const int64_t st = axis_stride(d, axis);
            c += kind[n - st] != 2;
            c += kind[n + st] != 2;
        }
    }
    ncut[n] = c;
}

// ------------------------------------------------- diagonal and cut records
// Sec. 2.1.1: the BP value is the linear interpolant between the computational
// point (xi_1 = 0) and the boundary crossing (xi_Gamma = q h) evaluated at the
// BP (xi = h): u_BP = u_Gamma / q + (1 - 1/q) u_1.  Substituted into the
// central difference, the side adds c = 1/q to the diagonal of -L_h h^2 and
// u_Gamma c / h^2 to the right-hand side.  The crossing is located by linear
// interpolation of psi between the last inside and first outside node on the
// grid line (Sec. 3.3); when the node two steps out is still inside, the line
// is followed to the first outside node.
__global__ void __launch_bounds__(BLOCK) k_diag_cuts(const double* __restrict__ psi, const int8_t* __restrict__ kind,
                                                     GridDims d, int64_t nnodes, const int64_t* __restrict__ cut_off,
                                                     double* __restrict__ a, eb_cut_t* __restrict__ cuts,
                                                     int64_t cap, int32_t* __restrict__ err) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= nnodes) return;
    // A domain that reaches the outer layer (flagged by k_classify, final by
    // now) makes unknowns next to that layer, whose walks would step past it:
    // nothing to do, the call fails.  This kernel only adds the flag where
    // k_classify has already set it.
    if (*err & DEVERR_DOMAIN) return;
    if (kind[n] != 2) {
        a[n] = 0.0;
        return;
    }
    const NodePos p = node_pos(n, d);
    int nreg = 0;
    for (int axis = 0; axis < d.dim; ++axis) {
        const int64_t st = axis_stride(d, axis);
        nreg += kind[n - st] == 2;
        nreg += kind[n + st] == 2;
    }
    double acc = (double)nreg;
    int64_t m = cut_off[n];
    for (int side = 0; side < 2 * d.dim; ++side) {
        const int axis = side >> 1;
        const int step = (side & 1) ? 1 : -1;
        const int64_t st = axis_stride(d, axis) * step;
        if (kind[n + st] == 2) continue;
        const int pos = axis_coord(p, axis);
        const int len = axis_len(d, axis);
        // walk to the first outside node; the outermost layer is outside.
        // Where the boundary runs almost along the line the walk is long, so
        // the nodes are read WALK at a time (all loads in flight, none past
        // the outer layer) and then examined in order.
        constexpr int WALK = 8;
        int j = 2;
        bool found = false;
        while (!found) {
            double v[WALK];
#pragma unroll
            for (int u = 0; u < WALK; ++u) {
                // clamped to the outer layer: the examination below stops there
                const int at = min(max(pos + (j + u) * step, 0), len - 1);
                v[u] = psi[n + (int64_t)(at - pos) * axis_stride(d, axis)];
            }
#pragma unroll
            for (int u = 0; u < WALK; ++u) {
                if (found) continue;
                const int at = pos + (j + u) * step;
                if (at <= 0 || at >= len - 1) {
                    if (v[u] < 0.0) atomicOr(err, DEVERR_DOMAIN);
                    j += u;
                    found = true;
                } else if (!(v[u] < 0.0)) {
                    j += u;
                    found = true;
                }
            }
            if (!found) j += WALK;
        }
        const double psi_in = psi[n + (int64_t)(j - 1) * st];
        const double psi_out = psi[n + (int64_t)j * st];
        const double t = psi_in / (psi_in - psi_out);
        const double q = (double)(j - 1) + t;
        const double c = 1.0 / q;
        acc = acc + c;
        if (m < cap) {
            eb_cut_t rec;
            rec.node = n;
            rec.dir = side;
            rec.steps = j;
            rec.q = q;
            rec.c = c;
            double xg[3];
            xg[0] = d.x0 + (double)p.i * d.h;
            xg[1] = d.y0 + (double)p.j * d.h;
            xg[2] = d.dim == 3 ? d.z0 + (double)p.k * d.h : 0.0;
            const double qh = q * d.h;
            xg[axis] = step > 0 ? xg[axis] + qh : xg[axis] - qh;
            rec.xg[0] = xg[0];
            rec.xg[1] = xg[1];
            rec.xg[2] = xg[2];
            cuts[m] = rec;
        }
        ++m;
    }
    a[n] = acc;
}

// ------------------------------------------------------------ right-hand side
// b_k = f_k + sum over the cuts of k (ascending side) of u_Gamma * (c / h^2).
__global__ void __launch_bounds__(BLOCK) k_rhs(const int8_t* __restrict__ kind, const double* __restrict__ f,
                                               const eb_cut_t* __restrict__ cuts, int64_t ncuts,
                                               const double* __restrict__ u, double* __restrict__ b,
                                               int64_t nnodes, double s) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= nnodes) return;
    if (kind[n] != 2) {
        b[n] = 0.0;
        return;
    }
    double v = f[n];
    // lower_bound of node n in the (node, dir)-sorted records
    int64_t lo = 0, hi = ncuts;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cuts[mid].node < n) lo = mid + 1; else hi = mid;
    }
    for (int64_t m = lo; m < ncuts && cuts[m].node == n; ++m) {
        const double w = cuts[m].c * s;
        v = v + u[m] * w;
    }
    b[n] = v;
}

// -------------------------------------------------------- operator on fields
__global__ void __launch_bounds__(BLOCK) k_stencil_dense(const int8_t* __restrict__ kind, const double* __restrict__ a,
                                                         double sigma, const double* __restrict__ x,
                                                         double* __restrict__ y, GridDims d, int64_t nnodes) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= nnodes) return;
    const NodePos p = node_pos(n, d);
    // a node on the outermost layer has no full stencil: never treated as an unknown
    const bool edge = p.i == 0 || p.i == d.nx - 1 || p.j == 0 || p.j == d.ny - 1 ||
                      (d.dim == 3 && (p.k == 0 || p.k == d.nz - 1));
    if (kind[n] != 2 || edge) {
        y[n] = 0.0;
        return;
    }
    double nb = 0.0;
    for (int axis = 0; axis < d.dim; ++axis) {
        const int64_t st = axis_stride(d, axis);
        if (kind[n - st] == 2) nb = nb + x[n - st];
        if (kind[n + st] == 2) nb = nb + x[n + st];
    }
    const double diag = a[n] * d.s + sigma;
    y[n] = diag * x[n] - d.s * nb;
}

// Device status of one assembly, read back once at the end.
struct AsmStat {
    int32_t err;
    int32_t pad;
    int64_t cuts;                 // total cut records (scan total)
    unsigned long long unknowns;  // interior nodes
};

}  // namespace eb

using namespace eb;

extern "C" int eb_assemble_diag(const eb_grid_t* g, const double* psi, int8_t* kind, double* a,
                                eb_cut_t* cuts, int64_t cuts_cap, int64_t* n_unknowns,
                                int64_t* n_cuts, void* stream) {
    clear_error();
    GridDims d;
    EB_TRY(make_dims(g, &d));
    if (!psi || !kind || !a || !n_unknowns || !n_cuts || cuts_cap < 0 || (cuts_cap > 0 && !cuts)) {
        set_error("eb_assemble_diag: null pointer or negative capacity");
        return EB_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    // No host round trip until the end: with a domain error k_count_cuts only
    // reads neighbours of unknowns (never on the outer layer) and k_diag_cuts
    // returns at once; the cut records are bounded by cuts_cap on the device;
    // status, totals and errors come back in one read.
    AsmStat* st = nullptr;
    int32_t* ncut = nullptr;
    int64_t* off = nullptr;
    int32_t* blk_unk = nullptr;
    const unsigned nblk = grid_for(nn);
    EB_TRY(dalloc_n(&st, 1, s));
    EB_TRY(dalloc_n(&ncut, nn, s));
    EB_TRY(dalloc_n(&off, nn, s));
    EB_TRY(dalloc_n(&blk_unk, nblk, s));
    {
        const FillSpec f[] = {{st, sizeof(AsmStat), 0u}};
        EB_TRY(fill_words(f, 1, s));
    }
    hipLaunchKernelGGL(k_classify, dim3(nblk), dim3(BLOCK), 0, s, psi, kind, d, nn, &st->err, blk_unk, ncut);
    EB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(1024), 0, s, blk_unk, (int64_t)nblk, &st->unknowns);
    EB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_count_cuts, dim3(grid_for(nn)), dim3(BLOCK), 0, s, kind, d, nn, ncut);
    EB_LAUNCH_CHECK();
    EB_TRY(scan_i32_to_i64_dev(ncut, off, nn, &st->cuts, s));
    hipLaunchKernelGGL(k_diag_cuts, dim3(grid_for(nn)), dim3(BLOCK), 0, s, psi, kind, d, nn, off, a, cuts, cuts_cap,
                       &st->err);
    EB_LAUNCH_CHECK();
    AsmStat h;
    EB_HIP(hipMemcpyAsync(&h, st, sizeof(AsmStat), hipMemcpyDeviceToHost, s));
    EB_TRY(dfree(st, s));
    EB_TRY(dfree(ncut, s));
    EB_TRY(dfree(off, s));
    EB_TRY(dfree(blk_unk, s));
    EB_HIP(hipStreamSynchronize(s));
    if (h.err & DEVERR_DOMAIN) {
        set_error("the domain reaches the outermost node layer (psi < 0 there)");
        return EB_EDOMAIN;
    }
    *n_unknowns = (int64_t)h.unknowns;
    *n_cuts = h.cuts;
    if (h.cuts > cuts_cap) {
        set_error("cut-record capacity %lld < required %lld", (long long)cuts_cap, (long long)h.cuts);
        return EB_ENOSPC;
    }
    return EB_OK;
}

extern "C" int eb_assemble_rhs(const eb_grid_t* g, const int8_t* kind, const double* f, const eb_cut_t* cuts,
                               int64_t n_cuts, const double* u_at_cuts, double* b, void* stream) {
    clear_error();
    GridDims d;
    EB_TRY(make_dims(g, &d));
    if (!kind || !f || !b || n_cuts < 0 || (n_cuts > 0 && (!cuts || !u_at_cuts))) {
        set_error("eb_assemble_rhs: null pointer or negative count");
        return EB_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    hipLaunchKernelGGL(k_rhs, dim3(grid_for(nn)), dim3(BLOCK), 0, s, kind, f, cuts, n_cuts, u_at_cuts, b, nn, d.s);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

extern "C" int stencil_apply(const eb_grid_t* g, const int8_t* kind, const double* a, double sigma,
                             const double* x, double* y, void* stream) {
    clear_error();
    GridDims d;
    EB_TRY(make_dims(g, &d));
    if (!kind || !a || !x || !y) {
        set_error("stencil_apply: null pointer");
        return EB_EINVAL;
    }
    if (!(sigma >= 0.0)) {
        set_error("stencil_apply: sigma must be >= 0");
        return EB_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    hipLaunchKernelGGL(k_stencil_dense, dim3(grid_for(nn)), dim3(BLOCK), 0, s, kind, a, sigma, x, y, d, nn);
    EB_LAUNCH_CHECK();
    return EB_OK;
}
