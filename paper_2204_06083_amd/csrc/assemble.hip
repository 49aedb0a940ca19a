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
                                                    int32_t* __restrict__ block_unknowns) {
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

// Cut sides of an unknown (neighbours that are not unknowns); 0 elsewhere.
__device__ inline int node_cuts(const int8_t* __restrict__ kind, int64_t n, const GridDims& d) {
    int c = 0;
    if (kind[n] == 2) {
        for (int axis = 0; axis < d.dim; ++axis) {
            const int64_t st = axis_stride(d, axis);
            c += kind[n - st] != 2;
            c += kind[n + st] != 2;
        }
    }
    return c;
}

// Cut sides per workgroup (the same node-to-workgroup map as k_diag_cuts,
// which places each node's records after those of the workgroups before it
// and of the nodes before it in its own).
__global__ void __launch_bounds__(BLOCK) k_count_cuts(const int8_t* __restrict__ kind, GridDims d, int64_t nnodes,
                                                      int32_t* __restrict__ block_cuts) {
    __shared__ int32_t wcount[BLOCK / WAVE];
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    int c = n < nnodes ? node_cuts(kind, n, d) : 0;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) c += __shfl_xor(c, off, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) wcount[threadIdx.x / WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < BLOCK / WAVE; ++w) t += wcount[w];
        block_cuts[blockIdx.x] = t;
    }
}

// ------------------------------------------------- diagonal and cut records
// Sec. 2.1.1: the BP value is the linear interpolant between the computational
// point (xi_1 = 0) and the boundary crossing (xi_Gamma = q h) evaluated at the
// BP (xi = h): u_BP = u_Gamma / q + (1 - 1/q) u_1.  Substituted into the
// central difference, the side adds c = 1/q to the diagonal of -L_h h^2 and
// u_Gamma c / h^2 to the right-hand side.  The crossing is the root of psi on
// the grid line (Sec. 2.1.1); this library locates it by linear interpolation
// of psi between the last inside and first outside node (a reading: the
// paper names a root finder there and uses this second-order approximation
// for its parametric geometries, Sec. 3.3); when the node two steps out is
// still inside, the line is followed to the first outside node.
// Walks that do not end within the first DIAG_SHORT nodes (a boundary running
// almost along the grid line: up to about a thousand nodes on the 2048^2
// star) would leave one thread walking long after the rest of the grid is
// done, so k_diag_cuts hands such nodes to k_diag_long, where a workgroup
// examines DIAG_LONG_NT nodes of the line per round.  Both kernels compute the
// node's diagonal and records with the same expressions in the same side
// order (diag_side), so the result does not depend on which one did it.
constexpr int DIAG_WALK = 8;                  // nodes read together per round
constexpr int DIAG_SHORT = 2 * DIAG_WALK;     // nodes a thread examines before deferring
constexpr int DIAG_DEFER_CAP = 4096;          // deferred nodes (more: walked in place)
constexpr int DIAG_LONG_NT = 1024;
constexpr int DIAG_LONG_BLOCKS = 64;

// The side's interpolation coefficient c = 1/q from the walk's end j (first
// outside node, j >= 2), and its cut record m (if below the capacity).
__device__ inline double diag_side(const double* __restrict__ psi, int64_t n, const NodePos& p, const GridDims& d,
                                   int side, int j, int64_t m, eb_cut_t* __restrict__ cuts, int64_t cap) {
    const int axis = side >> 1;
    const int step = (side & 1) ? 1 : -1;
    const int64_t st = axis_stride(d, axis) * step;
    const double psi_in = psi[n + (int64_t)(j - 1) * st];
    const double psi_out = psi[n + (int64_t)j * st];
    const double t = psi_in / (psi_in - psi_out);
    const double q = (double)(j - 1) + t;
    const double c = 1.0 / q;
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
    return c;
}

__device__ inline int diag_regular(const int8_t* __restrict__ kind, int64_t n, const GridDims& d) {
    int nreg = 0;
    for (int axis = 0; axis < d.dim; ++axis) {
        const int64_t st = axis_stride(d, axis);
        nreg += kind[n - st] == 2;
        nreg += kind[n + st] == 2;
    }
    return nreg;
}

__global__ void __launch_bounds__(BLOCK) k_diag_cuts(const double* __restrict__ psi, const int8_t* __restrict__ kind,
                                                     GridDims d, int64_t nnodes, const int64_t* __restrict__ block_off,
                                                     double* __restrict__ a, eb_cut_t* __restrict__ cuts,
                                                     int64_t cap, int32_t* __restrict__ err,
                                                     int32_t* __restrict__ ndefer, int64_t* __restrict__ defer) {
    __shared__ int32_t wsum[BLOCK / WAVE];
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool unknown = n < nnodes && kind[n] == 2;
    // first record of the node: the workgroup's offset plus the cut sides of
    // the nodes before it in the workgroup (exclusive scan)
    const int cnt = n < nnodes ? node_cuts(kind, n, d) : 0;
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    int inc = cnt;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const int t = __shfl_up(inc, off, WAVE);
        if (lane >= off) inc += t;
    }
    if (lane == WAVE - 1) wsum[wv] = inc;
    __syncthreads();
    int before = inc - cnt;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    if (n >= nnodes) return;
    // A domain that reaches the outer layer (flagged by k_classify, final by
    // now) makes unknowns next to that layer, whose walks would step past it:
    // nothing to do, the call fails.  This kernel only adds the flag where
    // k_classify has already set it.
    if (*err & DEVERR_DOMAIN) return;
    if (!unknown) {
        a[n] = 0.0;
        return;
    }
    const NodePos p = node_pos(n, d);
    double acc = (double)(2 * d.dim - cnt);     // regular sides: the others are cut
    const int64_t m_first = block_off[blockIdx.x] + before;
    int64_t m = m_first;
    for (int side = 0; side < 2 * d.dim; ++side) {
        const int axis = side >> 1;
        const int step = (side & 1) ? 1 : -1;
        const int64_t st = axis_stride(d, axis) * step;
        if (kind[n + st] == 2) continue;
        const int pos = axis_coord(p, axis);
        const int len = axis_len(d, axis);
        // walk to the first outside node (the outermost layer is outside),
        // DIAG_WALK nodes at a time: all loads in flight, none past the outer
        // layer, then examined in order
        int j = 2;
        bool found = false;
        bool deferred = false;
        while (!found) {
            if (j >= 2 + DIAG_SHORT && !deferred) {
                deferred = true;              // once only; list full: keep walking here
                // (the count stops growing once the list is full)
                if (*(volatile int32_t*)ndefer < DIAG_DEFER_CAP) {
                    const int slot = atomicAdd(ndefer, 1);
                    if (slot < DIAG_DEFER_CAP) {
                        defer[2 * slot] = n;  // the whole node is redone there
                        defer[2 * slot + 1] = m_first;
                        return;
                    }
                }
            }
            double v[DIAG_WALK];
#pragma unroll
            for (int u = 0; u < DIAG_WALK; ++u) {
                // clamped to the outer layer: the examination below stops there
                const int at = min(max(pos + (j + u) * step, 0), len - 1);
                v[u] = psi[n + (int64_t)(at - pos) * axis_stride(d, axis)];
            }
#pragma unroll
            for (int u = 0; u < DIAG_WALK; ++u) {
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
            if (!found) j += DIAG_WALK;
        }
        acc = acc + diag_side(psi, n, p, d, side, j, m, cuts, cap);
        ++m;
    }
    a[n] = acc;
}

// The deferred nodes, one workgroup each at a time: per side, the workgroup
// reads DIAG_LONG_NT consecutive nodes of the line per round and takes the
// first that ends the walk (the same test as the thread's walk: an outside
// node, or the outer layer); thread 0 then adds the sides in order.
__global__ void __launch_bounds__(DIAG_LONG_NT) k_diag_long(const double* __restrict__ psi,
                                                            const int8_t* __restrict__ kind, GridDims d,
                                                            double* __restrict__ a, eb_cut_t* __restrict__ cuts,
                                                            int64_t cap, int32_t* __restrict__ err,
                                                            const int32_t* __restrict__ ndefer,
                                                            const int64_t* __restrict__ defer) {
    __shared__ int first;
    if (*err & DEVERR_DOMAIN) return;
    const int count = min(*ndefer, DIAG_DEFER_CAP);
    const int tid = threadIdx.x;
    for (int i = blockIdx.x; i < count; i += gridDim.x) {
        const int64_t n = defer[2 * i];
        const NodePos p = node_pos(n, d);
        double acc = (double)diag_regular(kind, n, d);
        int64_t m = defer[2 * i + 1];
        for (int side = 0; side < 2 * d.dim; ++side) {
            const int axis = side >> 1;
            const int step = (side & 1) ? 1 : -1;
            const int64_t st = axis_stride(d, axis) * step;
            if (kind[n + st] == 2) continue;
            const int pos = axis_coord(p, axis);
            const int len = axis_len(d, axis);
            int j0 = 2;
            int f;
            bool edge = false;
            double v = 0.0;
            while (true) {
                const int at = pos + (j0 + tid) * step;
                const int atc = min(max(at, 0), len - 1);
                v = psi[n + (int64_t)(atc - pos) * axis_stride(d, axis)];
                edge = at <= 0 || at >= len - 1;
                const bool hit = edge || !(v < 0.0);
                if (tid == 0) first = DIAG_LONG_NT;
                __syncthreads();
                if (hit) atomicMin(&first, tid);
                __syncthreads();
                f = first;
                __syncthreads();
                if (f < DIAG_LONG_NT) break;   // the outer layer ends every line: reached within len rounds
                j0 += DIAG_LONG_NT;
            }
            if (tid == f && edge && v < 0.0) atomicOr(err, DEVERR_DOMAIN);
            if (tid == 0) acc = acc + diag_side(psi, n, p, d, side, j0 + f, m, cuts, cap);
            ++m;
        }
        if (tid == 0) a[n] = acc;
    }
}

// ------------------------------------------------------------ right-hand side
// b_k = f_k + sum over the cuts of k (ascending side) of u_Gamma * (c / h^2).
__global__ void __launch_bounds__(BLOCK) k_rhs(const int8_t* __restrict__ kind, const double* __restrict__ f,
                                               const eb_cut_t* __restrict__ cuts, int64_t ncuts,
                                               const double* __restrict__ u, double* __restrict__ b,
                                               int64_t nnodes, double s, GridDims d) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= nnodes) return;
    if (kind[n] != 2) {
        b[n] = 0.0;
        return;
    }
    double v = f[n];
    // only an unknown with a non-computational neighbour has records (an
    // unknown is never on the outer layer, so its neighbours exist)
    bool cut = false;
    for (int axis = 0; axis < d.dim; ++axis) {
        const int64_t st = axis_stride(d, axis);
        cut = cut || kind[n - st] != 2 || kind[n + st] != 2;
    }
    if (!cut) {
        b[n] = v;
        return;
    }
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

// ------------------------------------------------------------ SPD test
// The a-priori test of Sec. 2.4: along every axis, each maximal run of
// computational points on a grid line is one segment of the 1-D matrix
// D^(n)(a, b) (Eq. (tridiag)), whose end entries a, b are the part of the
// diagonal contributed by the two sides along that axis (1 per computational
// neighbour, c per cut side; minus side first).  Lemma 2.1's conditions on
// every segment make the operator SPD (Theorems 1-2).  The comparisons use
// the same FP64 operations, without contraction, as a plain evaluation.
__device__ inline bool lemma_2_1(int64_t n, double a, double b) {
    if (n == 1) return a > 0.0;
    if (n == 2) return a > 0.0 && a * b > 1.0;
    const double lo = (double)(n - 2) / (double)(n - 1);
    if (!(a > lo && b > lo)) return false;
    return a > ((double)(n - 2) * b - (double)(n - 3)) / ((double)(n - 1) * b - (double)(n - 2));
}

// c of the record (node, side); records are sorted by node, a node's records
// by side.  *miss is set when there is none.
__device__ inline double cut_c_of(const eb_cut_t* __restrict__ cuts, int64_t n_cuts, int64_t node, int side,
                                  int* miss) {
    int64_t lo = 0, hi = n_cuts;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (cuts[mid].node < node) lo = mid + 1;
        else hi = mid;
    }
    for (int64_t m = lo; m < n_cuts && cuts[m].node == node; ++m)
        if (cuts[m].dir == side) return cuts[m].c;
    *miss = 1;
    return 0.0;
}

// One thread per grid line along `axis`; out = {segments, failing, missing}.
__global__ void __launch_bounds__(BLOCK) k_spd_lines(const int8_t* __restrict__ kind, GridDims d, int axis,
                                                     const eb_cut_t* __restrict__ cuts, int64_t n_cuts,
                                                     unsigned long long* __restrict__ out) {
    const int64_t line = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t nx = d.nx, ny = d.ny, nz = d.nz;
    const int64_t sy = d.sy, sz = d.sz;
    int64_t nlines, len, step, base = 0;
    if (axis == 0) {
        nlines = ny * nz;
        len = nx;
        step = 1;
        if (line < nlines) base = sy * (line % ny) + sz * (line / ny);
    } else if (axis == 1) {
        nlines = nx * nz;
        len = ny;
        step = sy;
        if (line < nlines) base = (line % nx) + sz * (line / nx);
    } else {
        nlines = nx * ny;
        len = nz;
        step = sz;
        if (line < nlines) base = line;
    }
    unsigned long long segs = 0, fails = 0;
    int miss = 0;
    if (line < nlines) {
        int64_t run = 0;
        double a = 0.0, last = 0.0;
        for (int64_t t = 0; t <= len; ++t) {
            const int64_t node = base + t * step;
            if (t < len && kind[node] == 2) {
                // 0 + (minus side) + (plus side).  An assembly never has an
                // unknown on the outer layer; a field that does is refused
                // (counted as missing) rather than read past the line
                if (t == 0 || t == len - 1) {
                    miss = 1;
                    run = 0;
                    continue;
                }
                double v = 0.0;
                v = v + (kind[node - step] == 2 ? 1.0 : cut_c_of(cuts, n_cuts, node, 2 * axis, &miss));
                v = v + (kind[node + step] == 2 ? 1.0 : cut_c_of(cuts, n_cuts, node, 2 * axis + 1, &miss));
                if (run == 0) a = v;
                last = v;
                ++run;
                continue;
            }
            if (run > 0) {
                ++segs;
                if (!lemma_2_1(run, a, last)) ++fails;
                run = 0;
            }
        }
    }
    // integer sums: the same in any order
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        segs += __shfl_xor(segs, off);
        fails += __shfl_xor(fails, off);
        miss += __shfl_xor(miss, off);
    }
    if ((threadIdx.x & (WAVE - 1)) == 0 && (segs || fails || miss)) {
        atomicAdd(&out[0], segs);
        atomicAdd(&out[1], fails);
        atomicAdd(&out[2], (unsigned long long)miss);
    }
}

// Device status of one assembly, read back once at the end.
struct AsmStat {
    int32_t err;
    int32_t ndefer;               // nodes handed from k_diag_cuts to k_diag_long
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
    // returns after its offset scan (which reads the same); the cut records
    // are bounded by cuts_cap on the device;
    // status, totals and errors come back in one read.
    AsmStat* st = nullptr;
    int32_t* blk_cuts = nullptr;
    int64_t* blk_off = nullptr;
    int32_t* blk_unk = nullptr;
    int64_t* defer = nullptr;
    const unsigned nblk = grid_for(nn);
    EB_TRY(dalloc_n(&st, 1, s));
    EB_TRY(dalloc_n(&defer, 2 * DIAG_DEFER_CAP, s));
    EB_TRY(dalloc_n(&blk_cuts, nblk, s));
    EB_TRY(dalloc_n(&blk_off, nblk, s));
    EB_TRY(dalloc_n(&blk_unk, nblk, s));
    {
        const FillSpec f[] = {{st, sizeof(AsmStat), 0u}};
        EB_TRY(fill_words(f, 1, s));
    }
    hipLaunchKernelGGL(k_classify, dim3(nblk), dim3(BLOCK), 0, s, psi, kind, d, nn, &st->err, blk_unk);
    EB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(1024), 0, s, blk_unk, (int64_t)nblk, &st->unknowns);
    EB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_count_cuts, dim3(nblk), dim3(BLOCK), 0, s, kind, d, nn, blk_cuts);
    EB_LAUNCH_CHECK();
    EB_TRY(scan_i32_to_i64_dev(blk_cuts, blk_off, nblk, &st->cuts, s));
    hipLaunchKernelGGL(k_diag_cuts, dim3(nblk), dim3(BLOCK), 0, s, psi, kind, d, nn, blk_off, a, cuts, cuts_cap,
                       &st->err, &st->ndefer, defer);
    hipLaunchKernelGGL(k_diag_long, dim3(DIAG_LONG_BLOCKS), dim3(DIAG_LONG_NT), 0, s, psi, kind, d, a, cuts,
                       cuts_cap, &st->err, &st->ndefer, defer);
    EB_LAUNCH_CHECK();
    AsmStat h;
    EB_HIP(hipMemcpyAsync(&h, st, sizeof(AsmStat), hipMemcpyDeviceToHost, s));
    EB_TRY(dfree(st, s));
    EB_TRY(dfree(blk_cuts, s));
    EB_TRY(dfree(blk_off, s));
    EB_TRY(dfree(blk_unk, s));
    EB_TRY(dfree(defer, s));
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

extern "C" int eb_check_spd(const eb_grid_t* g, const int8_t* kind, const eb_cut_t* cuts, int64_t n_cuts,
                            int64_t* n_segments, int64_t* n_failing, void* stream) {
    clear_error();
    GridDims d;
    EB_TRY(make_dims(g, &d));
    if (!kind || !n_segments || !n_failing || n_cuts < 0 || (n_cuts > 0 && !cuts)) {
        set_error("eb_check_spd: null pointer or negative count");
        return EB_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* out = nullptr;
    EB_TRY(dalloc_n(&out, 3, s));
    {
        const FillSpec f[] = {{out, 3 * sizeof(unsigned long long), 0u}};
        EB_TRY(fill_words(f, 1, s));
    }
    for (int axis = 0; axis < d.dim; ++axis) {
        const int64_t nlines = axis == 0 ? (int64_t)d.ny * d.nz : axis == 1 ? (int64_t)d.nx * d.nz : (int64_t)d.nx * d.ny;
        hipLaunchKernelGGL(k_spd_lines, dim3(grid_for(nlines)), dim3(BLOCK), 0, s, kind, d, axis, cuts, n_cuts, out);
        EB_LAUNCH_CHECK();
    }
    unsigned long long h[3] = {0, 0, 0};
    EB_HIP(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
    EB_TRY(dfree(out, s));
    EB_HIP(hipStreamSynchronize(s));
    if (h[2] > 0) {
        set_error("eb_check_spd: %llu cut sides without a record or unknowns on the outer layer (pass the assembly's kind field and all its records)", h[2]);
        return EB_EINVAL;
    }
    *n_segments = (int64_t)h[0];
    *n_failing = (int64_t)h[1];
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
    hipLaunchKernelGGL(k_rhs, dim3(grid_for(nn)), dim3(BLOCK), 0, s, kind, f, cuts, n_cuts, u_at_cuts, b, nn, d.s, d);
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
