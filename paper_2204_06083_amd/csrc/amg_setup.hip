// Aggregation AMG setup on the device.
//
// Level l -> l+1 (every unknown carries integer grid coordinates; the fine
// level uses node indices, a coarse unknown the box it was formed in):
//   aggregates   connected components, in the graph of A_l, of the unknowns of
//                one 3^d coordinate box; coarse order = (box lexicographic,
//                smallest member), which is the order a prefix sum over the
//                box grid produces when each box numbers its components by
//                smallest member;
//   rho          max_i sum_j |a_ij| / a_ii (Gershgorin), omega = 4 / (3 rho);
//   P            (I - omega D^-1 A) P_tent with the structural pattern;
//   R            P^T;
//   A_{l+1}      R (A P), structural patterns, sorted columns.
// Coarsest level: dense Cholesky factorisation and the explicit inverse, so
// the solve phase applies it as one matrix-vector product.
//
// Every edge of A_l joins unknowns whose coordinates differ by at most one
// per axis (true for the stencil; kept by the Galerkin product because boxes
// are 3 wide), so every row of P, A P and A_{l+1} has its columns in the 3^d
// boxes around one centre box.  The products therefore accumulate into a
// small dense slot array per row (slot = neighbour box x rank within box),
// visited in slot order, which is ascending column order.  No floating-point
// atomics: accumulation order per entry is ascending k, then ascending j.
//
// Built with -ffp-contract=off so that separately rounded products and sums
// follow the order stated above.
#include <math.h>
#include <string.h>

#include <utility>
#include <vector>

#include "handle.hpp"

namespace eb {

__device__ inline int box_of(int c) { return c / 3; }

__device__ inline int64_t box_lin(int bx, int by, int bz, const int* nb) {
    return (int64_t)bx + (int64_t)nb[0] * ((int64_t)by + (int64_t)nb[1] * bz);
}

struct NB3 {
    int v[3];
};

__global__ void k_set_i32(int32_t* p, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void __launch_bounds__(BLOCK) k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(BLOCK) k_fill_i8(int8_t* p, int64_t n, int8_t v) {
    int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(BLOCK) k_fill_f64(double* p, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------ fine level CSR
__global__ void __launch_bounds__(BLOCK) k_fine_flags(const int8_t* __restrict__ kind, GridDims d, int64_t nn,
                                                      int32_t* __restrict__ flag, int32_t* __restrict__ err) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= nn) return;
    int f = kind[n] == 2;
    if (f) {
        const int i = (int)(n % d.nx);
        const int64_t r = n / d.nx;
        const int j = (int)(r % d.ny);
        const int k = (int)(r / d.ny);
        const bool edge = i == 0 || i == d.nx - 1 || j == 0 || j == d.ny - 1 ||
                          (d.dim == 3 && (k == 0 || k == d.nz - 1));
        if (edge) {
            atomicOr(err, DEVERR_DOMAIN);
            f = 0;
        }
    }
    flag[n] = f;
}

__global__ void __launch_bounds__(BLOCK) k_fine_rows(const int8_t* __restrict__ kind, GridDims d, int64_t nn,
                                                     const int32_t* __restrict__ flag,
                                                     const int32_t* __restrict__ unk_off,
                                                     int32_t* __restrict__ rowcnt, int64_t* __restrict__ fine_nodes,
                                                     int32_t* __restrict__ coords) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= nn || !flag[n]) return;
    const int32_t k = unk_off[n];
    fine_nodes[k] = n;
    const int i = (int)(n % d.nx);
    const int64_t r = n / d.nx;
    coords[3 * (int64_t)k + 0] = i;
    coords[3 * (int64_t)k + 1] = (int)(r % d.ny);
    coords[3 * (int64_t)k + 2] = (int)(r / d.ny);
    int c = 1;
    c += kind[n - 1] == 2;
    c += kind[n + 1] == 2;
    c += kind[n - d.sy] == 2;
    c += kind[n + d.sy] == 2;
    if (d.dim == 3) {
        c += kind[n - d.sz] == 2;
        c += kind[n + d.sz] == 2;
    }
    rowcnt[k] = c;
}

// Row k in ascending column order: -z, -y, -x, self, +x, +y, +z.  The
// workgroup's rows are one contiguous CSR range: each thread builds its row in
// LDS, then the range is written with consecutive threads on consecutive
// entries.
constexpr int FILL_ROW_MAX = 7;

// With beta (variable conductivity), the entry toward a neighbour is
// -beta_face / h^2 with the face between the two nodes.
__global__ void __launch_bounds__(BLOCK) k_fine_fill(const int8_t* __restrict__ kind, const double* __restrict__ a,
                                                     const double* __restrict__ beta, double sigma, GridDims d,
                                                     int64_t nunk,
                                                     const int64_t* __restrict__ fine_nodes,
                                                     const int32_t* __restrict__ unk_off,
                                                     const int32_t* __restrict__ rowptr, int32_t* __restrict__ col,
                                                     double* __restrict__ val, double* __restrict__ diag) {
    __shared__ int32_t col_s[BLOCK * FILL_ROW_MAX];
    __shared__ double val_s[BLOCK * FILL_ROW_MAX];
    const int64_t k0 = (int64_t)blockIdx.x * BLOCK;
    const int64_t k = k0 + threadIdx.x;
    const int64_t kend = k0 + BLOCK < nunk ? k0 + BLOCK : nunk;
    const int32_t base = rowptr[k0];
    if (k < nunk) {
        const int64_t n = fine_nodes[k];
        int32_t pos = rowptr[k] - base;
        const double off = -d.s;
        const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
        int64_t nbrs[7], faces[7];
        int cnt = 0;
        if (d.dim == 3) { nbrs[cnt] = n - d.sz; faces[cnt++] = 2 * nn + n - d.sz; }
        nbrs[cnt] = n - d.sy; faces[cnt++] = nn + n - d.sy;
        nbrs[cnt] = n - 1; faces[cnt++] = n - 1;
        const int self = cnt;
        nbrs[cnt] = n; faces[cnt++] = 0;
        nbrs[cnt] = n + 1; faces[cnt++] = n;
        nbrs[cnt] = n + d.sy; faces[cnt++] = nn + n;
        if (d.dim == 3) { nbrs[cnt] = n + d.sz; faces[cnt++] = 2 * nn + n; }
        for (int e = 0; e < cnt; ++e) {
            if (e == self) {
                const double dg = a[n] * d.s + sigma;
                col_s[pos] = (int32_t)k;
                val_s[pos] = dg;
                diag[k] = dg;
                ++pos;
            } else if (kind[nbrs[e]] == 2) {
                col_s[pos] = unk_off[nbrs[e]];
                val_s[pos] = beta ? -(beta[faces[e]] * d.s) : off;
                ++pos;
            }
        }
    }
    __syncthreads();
    const int32_t len = rowptr[kend] - base;
    for (int32_t e = threadIdx.x; e < len; e += BLOCK) {
        col[base + e] = col_s[e];
        val[base + e] = val_s[e];
    }
}

// ---------------------------------------------------------------- aggregation
// frz (island hierarchies, may be null): unknowns of islands that end at
// this level belong to no box and form no aggregate
__global__ void __launch_bounds__(BLOCK) k_box_count(const int32_t* __restrict__ coords, int64_t n, NB3 nb,
                                                     const int8_t* __restrict__ frz, int32_t* __restrict__ cnt,
                                                     int32_t* __restrict__ boxid) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    if (frz && frz[i]) {
        boxid[i] = -1;
        return;
    }
    const int64_t b = box_lin(box_of(coords[3 * i]), box_of(coords[3 * i + 1]), box_of(coords[3 * i + 2]), nb.v);
    boxid[i] = (int32_t)b;
    atomicAdd(&cnt[b], 1);
}

__global__ void __launch_bounds__(BLOCK) k_box_fill(const int32_t* __restrict__ boxid, int64_t n,
                                                    const int32_t* __restrict__ boff, int32_t* __restrict__ fillpos,
                                                    int32_t* __restrict__ members) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int32_t b = boxid[i];
    if (b < 0) return;
    const int32_t slot = atomicAdd(&fillpos[b], 1);
    members[boff[b] + slot] = (int32_t)i;
}

// Level 0: a box covers at most 3^d grid nodes and the graph of A_0 inside it
// is the grid adjacency among its unknowns, so its components come from bit
// masks: node offset (ii, jj, kk) is bit (kk * 3 + jj) * 3 + ii.  Bit order is
// node order, which is unknown order, so the lowest bit of a component is its
// smallest member and components numbered in lowest-bit order follow the
// smallest-member rule.
__device__ inline uint32_t grow27(uint32_t c) {
    constexpr uint32_t X0 = 0x1249249u;   // ii == 0
    constexpr uint32_t X2 = X0 << 2;      // ii == 2
    constexpr uint32_t Y0 = 0x01C0E07u;   // jj == 0
    constexpr uint32_t Y2 = Y0 << 6;      // jj == 2
    return c | ((c << 1) & ~X0) | ((c >> 1) & ~X2) | ((c << 3) & ~Y0) | ((c >> 3) & ~Y2) | (c << 9) | (c >> 9);
}

__global__ void __launch_bounds__(BLOCK) k_box_components0(const int8_t* __restrict__ kind, GridDims d, NB3 nb,
                                                           int64_t nboxes, const int32_t* __restrict__ unk_off,
                                                           int32_t* __restrict__ lrank,
                                                           int32_t* __restrict__ ncomp) {
    const int64_t b = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (b >= nboxes) return;
    const int bx = (int)(b % nb.v[0]);
    const int64_t rq = b / nb.v[0];
    const int by = (int)(rq % nb.v[1]);
    const int bz = (int)(rq / nb.v[1]);
    const int kz = d.dim == 3 ? 3 : 1;
    uint32_t mask = 0;
    for (int kk = 0; kk < kz; ++kk) {
        const int k = 3 * bz + kk;
        if (d.dim == 3 && (k < 1 || k > d.nz - 2)) continue;
        for (int jj = 0; jj < 3; ++jj) {
            const int j = 3 * by + jj;
            if (j < 1 || j > d.ny - 2) continue;
            for (int ii = 0; ii < 3; ++ii) {
                const int i = 3 * bx + ii;
                if (i < 1 || i > d.nx - 2) continue;
                if (kind[(int64_t)i + d.sy * j + d.sz * k] == 2) mask |= 1u << ((kk * 3 + jj) * 3 + ii);
            }
        }
    }
    int rank = 0;
    uint32_t rem = mask;
    while (rem) {
        uint32_t comp = rem & (~rem + 1u);
        for (;;) {
            const uint32_t g = grow27(comp) & mask;
            if (g == comp) break;
            comp = g;
        }
        rem &= ~comp;
        for (uint32_t w = comp; w; w &= w - 1u) {
            const int p = __ffs(w) - 1;
            const int ii = p % 3, jj = (p / 3) % 3, kk = p / 9;
            const int64_t node = (int64_t)(3 * bx + ii) + d.sy * (3 * by + jj) + d.sz * (3 * bz + kk);
            lrank[unk_off[node]] = rank;
        }
        ++rank;
    }
    ncomp[b] = rank;
}

constexpr int MAX_BOX_MEMBERS = 128;
constexpr int BOX_WAVES = 4;    // boxes (one wavefront each) per workgroup

__device__ inline int uf_root(volatile int32_t* parent, int x) {
    int p = parent[x];
    while (p != x) {
        x = p;
        p = parent[x];
    }
    return x;
}

// Levels >= 1: one wavefront per box.  The members are ranked by value in
// LDS, the edges of A that stay inside the box are spread over the lanes and
// merged with a lock-free union-find (a root is only ever attached below a
// smaller root, so each component ends rooted at its smallest member), and
// the roots are numbered in member order with a ballot prefix count.
__global__ void __launch_bounds__(BOX_WAVES * WAVE) k_box_components(const int32_t* __restrict__ boff,
                                                                     const int32_t* __restrict__ cnt,
                                                                     const int32_t* __restrict__ members,
                                                                     const int32_t* __restrict__ rowptr,
                                                                     const int32_t* __restrict__ col,
                                                                     const int32_t* __restrict__ boxid,
                                                                     int64_t nboxes, int32_t* __restrict__ lrank,
                                                                     int32_t* __restrict__ ncomp,
                                                                     int32_t* __restrict__ err) {
    __shared__ int32_t raw_s[BOX_WAVES][MAX_BOX_MEMBERS];
    __shared__ int32_t srt_s[BOX_WAVES][MAX_BOX_MEMBERS];
    __shared__ int32_t par_s[BOX_WAVES][MAX_BOX_MEMBERS];
    __shared__ int32_t eoff_s[BOX_WAVES][MAX_BOX_MEMBERS + 1];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t b = (int64_t)blockIdx.x * BOX_WAVES + w;
    int m = b < nboxes ? cnt[b] : 0;
    if (m > MAX_BOX_MEMBERS) {
        if (lane == 0) {
            atomicOr(err, DEVERR_CAP);
            ncomp[b] = 0;
        }
        m = 0;
    }
    const int32_t base = m > 0 ? boff[b] : 0;
    int32_t* raw = raw_s[w];
    int32_t* srt = srt_s[w];
    int32_t* par = par_s[w];
    int32_t* eoff = eoff_s[w];
    for (int t = lane; t < m; t += WAVE) raw[t] = members[base + t];
    __syncthreads();
    // rank by value (members are distinct); row lengths for the edge offsets
    int len[2] = {0, 0};
    for (int h = 0; h < 2; ++h) {
        const int t = lane + h * WAVE;
        if (t < m) {
            const int32_t v = raw[t];
            int r = 0;
            for (int u = 0; u < m; ++u) r += raw[u] < v;
            srt[r] = v;
        }
    }
    __syncthreads();
    for (int h = 0; h < 2; ++h) {
        const int t = lane + h * WAVE;
        if (t < m) {
            len[h] = rowptr[srt[t] + 1] - rowptr[srt[t]];
            par[t] = t;
        }
    }
    // inclusive wave scans of the two halves
    int carry = 0;
    for (int h = 0; h < 2; ++h) {
        int v = len[h];
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            const int u = __shfl_up(v, off, WAVE);
            if (lane >= off) v += u;
        }
        const int t = lane + h * WAVE;
        if (t < m) eoff[t + 1] = carry + v;
        carry += __shfl(v, WAVE - 1, WAVE);
    }
    if (lane == 0) eoff[0] = 0;
    __syncthreads();
    const int ne = m > 0 ? eoff[m] : 0;
    for (int e = lane; e < ne; e += WAVE) {
        int lo = 0, hi = m - 1;          // member li with eoff[li] <= e < eoff[li + 1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (eoff[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const int li = lo;
        const int32_t i = srt[li];
        const int32_t j = col[rowptr[i] + (e - eoff[li])];
        if (j == i || boxid[j] != (int32_t)b) continue;
        int a0 = 0, a1 = m - 1;          // local index of j
        while (a0 < a1) {
            const int mid = (a0 + a1) >> 1;
            if (srt[mid] < j) a0 = mid + 1; else a1 = mid;
        }
        const int lj = a0;
        for (;;) {
            int ra = uf_root(par, li), rb = uf_root(par, lj);
            if (ra == rb) break;
            if (ra > rb) { const int tmp = ra; ra = rb; rb = tmp; }
            if (atomicCAS(&par[rb], rb, ra) == rb) break;
        }
    }
    __syncthreads();
    int root[2] = {0, 0};
    unsigned long long rmask[2];
    for (int h = 0; h < 2; ++h) {
        const int t = lane + h * WAVE;
        if (t < m) root[h] = uf_root(par, t);
        rmask[h] = __ballot(t < m && root[h] == t);
    }
    __syncthreads();
    // par now holds the rank of each root (roots only)
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    for (int h = 0; h < 2; ++h) {
        const int t = lane + h * WAVE;
        if (t < m && root[h] == t) par[t] = __popcll(rmask[h] & below) + (h ? __popcll(rmask[0]) : 0);
    }
    __syncthreads();
    for (int h = 0; h < 2; ++h) {
        const int t = lane + h * WAVE;
        if (t < m) lrank[srt[t]] = par[root[h]];
    }
    if (lane == 0 && b < nboxes && m > 0) ncomp[b] = __popcll(rmask[0]) + __popcll(rmask[1]);
    if (lane == 0 && b < nboxes && m == 0 && cnt[b] == 0) ncomp[b] = 0;
}

__global__ void __launch_bounds__(BLOCK) k_assign_agg(const int32_t* __restrict__ coords, int64_t n, NB3 nb,
                                                      const int32_t* __restrict__ cstart,
                                                      const int32_t* __restrict__ lrank, const int8_t* __restrict__ frz,
                                                      int32_t* __restrict__ agg) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    if (frz && frz[i]) {
        agg[i] = -1;
        return;
    }
    const int64_t b = box_lin(box_of(coords[3 * i]), box_of(coords[3 * i + 1]), box_of(coords[3 * i + 2]), nb.v);
    agg[i] = cstart[b] + lrank[i];
}

__global__ void __launch_bounds__(BLOCK) k_coarse_coords(const int32_t* __restrict__ ncomp,
                                                         const int32_t* __restrict__ cstart, NB3 nb, int64_t nboxes,
                                                         int32_t* __restrict__ ccoords, int4* __restrict__ cinfo) {
    const int64_t b = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (b >= nboxes) return;
    const int m = ncomp[b];
    if (m == 0) return;
    const int bx = (int)(b % nb.v[0]);
    const int64_t r = b / nb.v[0];
    const int by = (int)(r % nb.v[1]);
    const int bz = (int)(r / nb.v[1]);
    const int32_t c0 = cstart[b];
    for (int t = 0; t < m; ++t) {
        ccoords[3 * (int64_t)(c0 + t) + 0] = bx;
        ccoords[3 * (int64_t)(c0 + t) + 1] = by;
        ccoords[3 * (int64_t)(c0 + t) + 2] = bz;
        cinfo[c0 + t] = make_int4(bx, by, bz, t);
    }
}

// Maximum of n non-negative int32 values into *out (pre-zeroed); integer
// atomicMax is order independent, so the result is deterministic.
__global__ void __launch_bounds__(BLOCK) k_max_i32(const int32_t* __restrict__ v, int64_t n, int32_t* __restrict__ out) {
    __shared__ int32_t lds[BLOCK];
    int32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        m = max(m, v[i]);
    lds[threadIdx.x] = m;
    __syncthreads();
    for (int off = BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) lds[threadIdx.x] = max(lds[threadIdx.x], lds[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, lds[0]);
}

// ----------------------------------------------------------------- Gershgorin
__global__ void __launch_bounds__(BLOCK) k_gershgorin_rows(const int32_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           const double* __restrict__ diag, int64_t n,
                                                           const int8_t* __restrict__ frz, double* __restrict__ rowv) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    if (frz && frz[i]) {
        rowv[i] = 1.0;      // no part in this level's weight (every row's bound is >= 1)
        return;
    }
    double s = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) s = s + fabs(val[e]);
    rowv[i] = s / diag[i];
}

// Maximum of n positive doubles into *out (pre-zeroed bit pattern): for
// non-negative IEEE doubles the bit patterns order like the values, so an
// unsigned 64-bit atomicMax gives the exact, order-independent maximum.
// Non-positive, NaN or infinite entries raise DEVERR_NOTSPD.
__global__ void __launch_bounds__(BLOCK) k_max_f64(const double* __restrict__ v, int64_t n,
                                                   unsigned long long* __restrict__ out, int32_t* __restrict__ err) {
    __shared__ double lds[BLOCK];
    double m = 0.0;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK) {
        const double x = v[i];
        if (!(x > 0.0) || isinf(x)) bad = true;
        else m = fmax(m, x);
    }
    lds[threadIdx.x] = m;
    if (bad) atomicOr(err, DEVERR_NOTSPD);
    __syncthreads();
    for (int off = BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(lds[0]));
}

// ------------------------------------------------------- slot accumulators
// Slot of coarse unknown J relative to centre box (bx, by, bz): neighbour box
// offset in {-1,0,1}^d (lexicographic, x fastest) times maxc, plus the rank of
// J within its box.  Ascending slot = ascending J.
struct SlotMap {
    int dim;
    int maxc;
    int nslots;
    const int4* cinfo;        // per coarse unknown: box coordinates and rank within its box
    const int32_t* cstart;    // first coarse unknown of each box
    NB3 nb;                   // box grid of the fine level = coarse extents

    __device__ int slot(int32_t J, int bx, int by, int bz) const {
        const int4 ci = cinfo[J];
        const int ox = ci.x - bx + 1;
        const int oy = ci.y - by + 1;
        const int oz = dim == 3 ? ci.z - bz + 1 : 1;
        const int r = ci.w;
        if (ox < 0 || ox > 2 || oy < 0 || oy > 2 || oz < 0 || oz > 2 || r >= maxc) return -1;
        const int o = dim == 3 ? (oz * 3 + oy) * 3 + ox : oy * 3 + ox;
        return o * maxc + r;
    }
    __device__ int32_t column(int s, int bx, int by, int bz) const {
        const int o = s / maxc;
        const int r = s - o * maxc;
        const int ox = o % 3;
        const int oy = (o / 3) % 3;
        const int oz = dim == 3 ? o / 9 : 1;
        const int64_t b = box_lin(bx + ox - 1, by + oy - 1, bz + oz - 1, nb.v);
        return cstart[b] + r;
    }
};

enum { ACC_P = 0, ACC_AP = 1, ACC_RAP = 2 };
constexpr int ACC_XB = 4;   // first-operand entries a lane reads at once

struct AccArgs {
    SlotMap sm;
    int64_t nrows;
    // centre coordinates per row: level-l coordinates (P, AP: centre = coords / 3)
    // or coarse coordinates (RAP: centre = ccoords)
    const int32_t* row_coords;
    int centre_div;           // 3 for P/AP rows, 1 for RAP rows
    // first operand (rows): A_l for P/AP, R for RAP
    const int32_t* x_rowptr; const int32_t* x_col; const double* x_val;
    // second operand: P (for AP) or AP (for RAP); for ACC_P the agg map.
    // y_start != nullptr: row k holds y_cnt[k] entries from y_start[k] on
    // (the compacted scratch of a product) instead of CSR.
    const int32_t* y_rowptr; const int32_t* y_col; const double* y_val;
    const int32_t* y_start; const int32_t* y_cnt;
    const int32_t* agg;       // ACC_P only
    const double* diag;       // ACC_P only
    const double* omega;      // ACC_P only (device scalar)
    int32_t* out_cnt;         // entries per row
    int32_t* out_start;       // first entry of the row in the scratch
    int32_t* ell_col;         // scratch: workgroup b owns [b * rows * ell_stride, ...)
    double* ell_val;          // and packs its rows there back to back
    int ell_stride;           // bound on the entries of one row
    int32_t* err;
};

// One pass per row: accumulate into slot arrays in LDS, then write the
// occupied slots, in slot = column order, to the row's ELL scratch and count.
// G lanes share a row (blockDim.x = rows per block x G): lane g takes the
// first operand's entries g, g + G, ... in order into a slot array of its
// own; the G arrays are then added slot by slot in lane order.  The order of
// the sums is fixed, so the result is deterministic (for G = 1 it is the
// plain row-by-row accumulation).  LDS: vals[t * ns + s], flags likewise.
template <int MODE>
__global__ void k_accumulate(AccArgs A, int G) {
    extern __shared__ char smem[];
    const int ns = A.sm.nslots;
    const int nt = blockDim.x;
    const int t = threadIdx.x;
    const int g = t % G;
    const int rl = t / G;
    double* vals = reinterpret_cast<double*>(smem);
    uint8_t* flags = reinterpret_cast<uint8_t*>(smem + sizeof(double) * (size_t)ns * nt);
    const int64_t row = (int64_t)blockIdx.x * (nt / G) + rl;
    const bool active = row < A.nrows;
    for (int sl = 0; sl < ns; ++sl) {
        flags[t * ns + sl] = 0;
        vals[t * ns + sl] = 0.0;
    }
    int bx = 0, by = 0, bz = 0;
    bool bad = false;
    if (active) {
        bx = A.row_coords[3 * row] / A.centre_div;
        by = A.row_coords[3 * row + 1] / A.centre_div;
        bz = A.row_coords[3 * row + 2] / A.centre_div;
        double* v = vals + (size_t)t * ns;
        uint8_t* fl = flags + (size_t)t * ns;
        if (MODE == ACC_P && A.agg[row] < 0) {
            // a row of an island that ends at this level: no prolongator entries
        } else if (MODE == ACC_P) {
            const double dii = A.diag[row];
            const double omega = *A.omega;
            if (g == 0) {
                const int s0 = A.sm.slot(A.agg[row], bx, by, bz);
                if (s0 < 0) {
                    bad = true;
                } else {
                    fl[s0] = 1;
                    v[s0] = 1.0;
                }
            }
            // entries in groups of ACC_XB: columns and values, then their
            // aggregates, read a group at a time; added in entry order
            const int e0 = A.x_rowptr[row] + g, e1 = A.x_rowptr[row + 1];
            for (int eb = e0; eb < e1; eb += G * ACC_XB) {
                int gs[ACC_XB];
                double xvs[ACC_XB];
#pragma unroll
                for (int u = 0; u < ACC_XB; ++u) {
                    const int e = eb + u * G;
                    const int ei = e < e1 ? e : 0;
                    const int j = A.x_col[ei];
                    xvs[u] = A.x_val[ei];
                    gs[u] = j;
                }
#pragma unroll
                for (int u = 0; u < ACC_XB; ++u) {
                    const int a = A.agg[gs[u]];
                    gs[u] = eb + u * G < e1 ? a : -1;
                }
#pragma unroll
                for (int u = 0; u < ACC_XB; ++u) {
                    if (gs[u] < 0) continue;   // past the row; or never: no edge joins two islands
                    const int sl = A.sm.slot(gs[u], bx, by, bz);
                    if (sl < 0) { bad = true; continue; }
                    fl[sl] = 1;
                    const double w = omega * (xvs[u] / dii);
                    v[sl] = v[sl] - w;
                }
            }
        } else {
            // the lane's first-operand entries in groups of ACC_XB: their
            // columns and values, then the extents of the second operand's
            // rows they select, are read a group at a time (two round trips
            // per group instead of two per entry); the products are then
            // added in entry order, as one entry at a time would add them.
            // A slot past the row reads entry 0 / row 0 and is not used.
            const int e0 = A.x_rowptr[row] + g, e1 = A.x_rowptr[row + 1];
            for (int eb = e0; eb < e1; eb += G * ACC_XB) {
                int ks[ACC_XB], f0s[ACC_XB], f1s[ACC_XB];
                double xvs[ACC_XB];
#pragma unroll
                for (int u = 0; u < ACC_XB; ++u) {
                    const int e = eb + u * G;
                    const int ei = e < e1 ? e : 0;
                    ks[u] = A.x_col[ei];
                    xvs[u] = A.x_val[ei];
                }
#pragma unroll
                for (int u = 0; u < ACC_XB; ++u) {
                    const int k = eb + u * G < e1 ? ks[u] : 0;
                    const int a = A.y_start ? A.y_start[k] : A.y_rowptr[k];
                    const int b = A.y_start ? a + A.y_cnt[k] : A.y_rowptr[k + 1];
                    f0s[u] = a;
                    f1s[u] = eb + u * G < e1 ? b : a;
                }
#pragma unroll
                for (int u = 0; u < ACC_XB; ++u) {
                    const double xv = xvs[u];
                    for (int f = f0s[u]; f < f1s[u]; ++f) {
                        const int sl = A.sm.slot(A.y_col[f], bx, by, bz);
                        if (sl < 0) { bad = true; continue; }
                        fl[sl] = 1;
                        const double pr = xv * A.y_val[f];
                        v[sl] = v[sl] + pr;
                    }
                }
            }
        }
    }
    if (bad) atomicOr(A.err, DEVERR_CAP);
    if (G > 1) {
        __syncthreads();
        // lane g owns slots g, g + G, ...: sum the G arrays in lane order into
        // the row's first array
        const int t0 = rl * G;
        for (int sl = g; sl < ns; sl += G) {
            double acc = 0.0;
            uint8_t f = 0;
            for (int h = 0; h < G; ++h) {
                acc += vals[(size_t)(t0 + h) * ns + sl];
                f |= flags[(size_t)(t0 + h) * ns + sl];
            }
            vals[(size_t)t0 * ns + sl] = acc;
            flags[(size_t)t0 * ns + sl] = f;
        }
        __syncthreads();
    }
    // pack the block's rows back to back: count, exclusive scan over the
    // block's rows, then write each row's occupied slots in slot = column order
    __shared__ int32_t offs[256];                 // rows per block <= 256
    const int rb = nt / G;
    const double* v = vals + (size_t)t * ns;
    const uint8_t* fl = flags + (size_t)t * ns;
    int c = 0;
    if (active && g == 0)
        for (int sl = 0; sl < ns; ++sl) c += fl[sl] ? 1 : 0;
    if (c > A.ell_stride) {
        atomicOr(A.err, DEVERR_CAP);
        c = A.ell_stride;
    }
    if (g == 0) offs[rl] = c;
    __syncthreads();
    for (int off = 1; off < rb; off <<= 1) {
        const int32_t add = (t < rb && t >= off) ? offs[t - off] : 0;
        __syncthreads();
        if (t < rb) offs[t] += add;
        __syncthreads();
    }
    if (!active || g != 0) return;
    const int32_t start = (int32_t)((int64_t)blockIdx.x * rb * A.ell_stride) + (rl > 0 ? offs[rl - 1] : 0);
    int w = 0;
    for (int sl = 0; sl < ns && w < c; ++sl) {
        if (fl[sl]) {
            A.ell_col[start + w] = A.sm.column(sl, bx, by, bz);
            A.ell_val[start + w] = v[sl];
            ++w;
        }
    }
    A.out_cnt[row] = c;
    A.out_start[row] = start;
}

// Packed product scratch -> CSR (rows keep their order).
__global__ void __launch_bounds__(BLOCK) k_ell_to_csr(const int32_t* __restrict__ ell_col,
                                                      const double* __restrict__ ell_val,
                                                      const int32_t* __restrict__ start, int64_t nrows,
                                                      const int32_t* __restrict__ rowptr, int32_t* __restrict__ col,
                                                      double* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= nrows) return;
    const int32_t b = rowptr[i], e = rowptr[i + 1];
    const int32_t s0 = start[i];
    for (int32_t k = 0; k < e - b; ++k) {
        col[b + k] = ell_col[s0 + k];
        val[b + k] = ell_val[s0 + k];
    }
}

// -------------------------------------------------------------- transpose
__global__ void __launch_bounds__(BLOCK) k_tr_count(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                    int64_t nrows, int32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= nrows) return;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) atomicAdd(&cnt[col[e]], 1);
}

__global__ void __launch_bounds__(BLOCK) k_tr_fill(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                   const double* __restrict__ val, int64_t nrows,
                                                   const int32_t* __restrict__ t_rowptr, int32_t* __restrict__ fill,
                                                   int32_t* __restrict__ t_col, double* __restrict__ t_val) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= nrows) return;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int c = col[e];
        const int32_t pos = t_rowptr[c] + atomicAdd(&fill[c], 1);
        t_col[pos] = (int32_t)i;
        t_val[pos] = val[e];
    }
}

// Level-0 transpose by pulling: P_iI != 0 only for fine unknowns i within one
// node of aggregate I's box, i.e. in the (3+2)^d nodes [3B-1, 3B+3]^d around
// box B.  Listing them in lexicographic order lists rows in ascending unknown
// order, so R = P^T comes out sorted without atomics.  TR_G lanes share a
// row: lane q checks window nodes q, q + TR_G, ...; a ballot prefix over the
// row's lanes keeps the lexicographic order when they write.
constexpr int TR_G = 32;

template <bool FILL>
__global__ void __launch_bounds__(BLOCK) k_tr0_pull(int64_t nc, const int4* __restrict__ cinfo,
                                                    const int8_t* __restrict__ kind, GridDims d,
                                                    const int32_t* __restrict__ unk_off,
                                                    const int32_t* __restrict__ p_rowptr,
                                                    const int32_t* __restrict__ p_col,
                                                    const double* __restrict__ p_val, int32_t* __restrict__ cnt,
                                                    const int32_t* __restrict__ r_rowptr, int32_t* __restrict__ r_col,
                                                    double* __restrict__ r_val) {
    const int64_t I = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) / TR_G;
    const int q = threadIdx.x % TR_G;
    const int gshift = (threadIdx.x % WAVE) / TR_G * TR_G;    // first lane of the row in the wave
    const bool rowok = I < nc;
    int xlo = 0, ylo = 0, zlo = 0, wx = 1, wy = 1, nwin = 0;
    int32_t pos = 0;
    if (rowok) {
        const int4 ci = cinfo[I];
        // unknowns never sit on the outer ring of nodes, so the window stays inside it
        zlo = d.dim == 3 ? max(3 * ci.z - 1, 1) : 0;
        const int zhi = d.dim == 3 ? min(3 * ci.z + 3, d.nz - 2) : 0;
        ylo = max(3 * ci.y - 1, 1);
        const int yhi = min(3 * ci.y + 3, d.ny - 2);
        xlo = max(3 * ci.x - 1, 1);
        const int xhi = min(3 * ci.x + 3, d.nx - 2);
        wx = xhi - xlo + 1;
        wy = yhi - ylo + 1;
        nwin = wx * wy * (zhi - zlo + 1);
        if (wx <= 0 || wy <= 0 || zhi < zlo) nwin = 0;
        if (FILL) pos = r_rowptr[I];
    }
    const int wmax = d.dim == 3 ? 125 : 25;        // the same trip count for every lane
    int c = 0;
    for (int base = 0; base < wmax; base += TR_G) {
        const int w = base + q;
        bool hit = false;
        int32_t u = 0;
        double pv = 0.0;
        if (w < nwin) {
            const int i = xlo + w % wx;
            const int j = ylo + (w / wx) % wy;
            const int k = zlo + w / (wx * wy);
            const int64_t node = (int64_t)i + d.sy * j + d.sz * k;
            if (kind[node] == 2) {
                u = unk_off[node];
                for (int e = p_rowptr[u]; e < p_rowptr[u + 1]; ++e) {
                    if (p_col[e] == (int32_t)I) {
                        hit = true;
                        pv = p_val[e];
                        break;
                    }
                }
            }
        }
        const unsigned long long mask = (__ballot(hit) >> gshift) & ((TR_G == 64) ? ~0ull : ((1ull << TR_G) - 1));
        if (FILL && hit) {
            const int before = __popcll(mask & ((1ull << q) - 1));
            r_col[pos + before] = u;
            r_val[pos + before] = pv;
        }
        const int m = __popcll(mask);
        pos += m;
        c += m;
    }
    if (!FILL && rowok && q == 0) cnt[I] = c;
}

// Sort each row by column: one workgroup of NT threads per row, bitonic
// network in LDS for rows of up to MAXM entries (keys are unique column
// indices), insertion sort by thread 0 beyond that.  R = P^T rows hold up to
// 5^d entries, R A rows up to 7^d (343 in 3-D).
template <int NT, int MAXM>
__global__ void __launch_bounds__(NT) k_sort_rows(const int32_t* __restrict__ rowptr, int32_t* __restrict__ col,
                                                  double* __restrict__ val, int64_t nrows) {
    __shared__ int32_t key[MAXM];
    __shared__ double v[MAXM];
    const int64_t i = blockIdx.x;
    if (i >= nrows) return;
    const int b = rowptr[i], e = rowptr[i + 1];
    const int m = e - b;
    const int tid = threadIdx.x;
    if (m <= 1) return;
    if (m > MAXM) {
        if (tid == 0) {
            for (int u = b + 1; u < e; ++u) {
                const int32_t c = col[u];
                const double x = val[u];
                int w = u;
                while (w > b && col[w - 1] > c) {
                    col[w] = col[w - 1];
                    val[w] = val[w - 1];
                    --w;
                }
                col[w] = c;
                val[w] = x;
            }
        }
        return;
    }
    int p2 = 2;
    while (p2 < m) p2 <<= 1;
    for (int t = tid; t < p2; t += NT) {
        key[t] = t < m ? col[b + t] : INT32_MAX;
        v[t] = t < m ? val[b + t] : 0.0;
    }
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = tid; t < p2; t += NT) {
                const int u = t ^ j;
                if (u > t) {
                    const bool up = (t & k) == 0;
                    const int32_t kt = key[t], ku = key[u];
                    if ((kt > ku) == up) {
                        key[t] = ku;
                        key[u] = kt;
                        const double vt = v[t];
                        v[t] = v[u];
                        v[u] = vt;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int t = tid; t < m; t += NT) {
        col[b + t] = key[t];
        val[b + t] = v[t];
    }
}

__global__ void __launch_bounds__(BLOCK) k_extract_diag(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val, int64_t n,
                                                        double* __restrict__ diag, int32_t* __restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    double dg = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e)
        if (col[e] == (int32_t)i) dg = val[e];
    if (!(dg > 0.0)) atomicOr(err, DEVERR_NOTSPD);
    diag[i] = dg;
}

// ------------------------------------------------------------ coarsest level
__global__ void __launch_bounds__(BLOCK) k_csr_to_dense(const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const double* __restrict__ val, int64_t n,
                                                        double* __restrict__ dense) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    for (int64_t j = 0; j < n; ++j) dense[i * n + j] = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) dense[i * n + col[e]] = val[e];
}

// Blocked right-looking Cholesky in place (lower triangle of the row-major
// n x n matrix).  Per 16-column panel: k_chol_panel (one workgroup) factors
// the panel rows [k0, n) in LDS and writes them back; k_chol_trailing (many
// workgroups) applies A[i][j] -= sum_c L[i][c] L[j][c] to the trailing lower
// triangle, each workgroup a 64 x 64 block with its panel rows staged in LDS
// and each thread a 4 x 4 tile.
constexpr int CHOL_NB = 16;
constexpr int CHOL_THREADS = 256;
constexpr int CHOL_TB = 64;     // trailing block edge

// Panel factorisation: each thread keeps RPT panel rows (16 values each) in
// registers; per column the pivot row's owner takes the square root, every
// row is scaled, the top-block rows publish their scaled entry through LDS and
// every row applies the rank-1 update to its remaining panel columns.
template <int RPT>
__global__ void __launch_bounds__(CHOL_THREADS) k_chol_panel(double* __restrict__ Ad, int n, int k0,
                                                             int32_t* __restrict__ err) {
    __shared__ double piv_s[CHOL_NB];
    __shared__ double col_s[CHOL_NB][CHOL_NB];   // col_s[c][c2] = L[k0+c2][k0+c]
    const int kb = min(CHOL_NB, n - k0);
    const int rows = n - k0;
    const int t = threadIdx.x;
    double x[RPT][CHOL_NB];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = t + q * CHOL_THREADS;
#pragma unroll
        for (int c = 0; c < CHOL_NB; ++c)
            x[q][c] = (r < rows && c < kb) ? Ad[(int64_t)(k0 + r) * n + k0 + c] : 0.0;
    }
    bool fail = false;
#pragma unroll
    for (int c = 0; c < CHOL_NB; ++c) {
        if (c < kb) {   // uniform across the workgroup
        if (t == c) {
            const double d = x[0][c];
            if (!(d > 0.0)) fail = true;
            const double p = d > 0.0 ? sqrt(d) : 1.0;
            x[0][c] = p;
            piv_s[c] = p;
        }
        __syncthreads();
        const double p = piv_s[c];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = t + q * CHOL_THREADS;
            if (r > c && r < rows) x[q][c] = x[q][c] / p;
        }
        if (t > c && t < kb) col_s[c][t] = x[0][c];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = t + q * CHOL_THREADS;
            if (r > c && r < rows) {
#pragma unroll
                for (int c2 = c + 1; c2 < CHOL_NB; ++c2)
                    if (c2 < kb && c2 <= r) x[q][c2] = x[q][c2] - x[q][c] * col_s[c][c2];
            }
        }
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = t + q * CHOL_THREADS;
        if (r < rows) {
#pragma unroll
            for (int c = 0; c < CHOL_NB; ++c)
                if (c < kb && c <= r) Ad[(int64_t)(k0 + r) * n + k0 + c] = x[q][c];
        }
    }
    if (fail) atomicOr(err, DEVERR_NOTSPD);
}

__global__ void __launch_bounds__(CHOL_THREADS) k_chol_trailing(double* __restrict__ Ad, int n, int k0) {
    __shared__ double pi_s[CHOL_TB * CHOL_NB];
    __shared__ double pj_s[CHOL_TB * CHOL_NB];
    const int t0 = k0 + CHOL_NB;
    const int m = n - t0;
    if (m <= 0) return;
    const int nbk = (m + CHOL_TB - 1) / CHOL_TB;
    // lower-triangular block index -> (bi, bj), bj <= bi
    int bi = (int)((sqrt(8.0 * (double)blockIdx.x + 1.0) - 1.0) * 0.5);
    while ((bi + 1) * (bi + 2) / 2 <= (int)blockIdx.x) ++bi;
    while (bi * (bi + 1) / 2 > (int)blockIdx.x) --bi;
    const int bj = blockIdx.x - bi * (bi + 1) / 2;
    if (bi >= nbk) return;
    const int i_base = t0 + bi * CHOL_TB, j_base = t0 + bj * CHOL_TB;
    for (int e = threadIdx.x; e < CHOL_TB * CHOL_NB; e += blockDim.x) {
        const int r = e / CHOL_NB, c = e % CHOL_NB;
        pi_s[e] = i_base + r < n ? Ad[(int64_t)(i_base + r) * n + k0 + c] : 0.0;
        pj_s[e] = j_base + r < n ? Ad[(int64_t)(j_base + r) * n + k0 + c] : 0.0;
    }
    __syncthreads();
    const int ti = threadIdx.x / (CHOL_TB / 4), tj = threadIdx.x % (CHOL_TB / 4);
    const int i0 = i_base + 4 * ti, j0 = j_base + 4 * tj;
    if (i0 >= n || j0 >= n || j0 > i0 + 3) return;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 4
    for (int c = 0; c < CHOL_NB; ++c) {
        double pi[4], pj[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            pi[a] = pi_s[(4 * ti + a) * CHOL_NB + c];
            pj[a] = pj_s[(4 * tj + a) * CHOL_NB + c];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += pi[a] * pj[b];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + a, j = j0 + b;
            if (i < n && j <= i) Ad[(int64_t)i * n + j] -= acc[a][b];
        }
}

// Linv = L^-1 by forward substitution on identity columns, 16 columns per
// workgroup in LDS (n x 16).  Rows go in blocks of 16: the part of each dot
// product that reaches back before the block is one independent sum per
// (row, column) over all 256 threads, then 16 threads (one per column)
// finish the block's lower-triangular solve.  Column c is zero above row c.
constexpr int TRI_NB = 16;
constexpr int TRI_THREADS = TRI_NB * TRI_NB;

__global__ void __launch_bounds__(TRI_THREADS) k_tri_inverse(const double* __restrict__ Lf, int n,
                                                             double* __restrict__ Li) {
    extern __shared__ double ycol[];               // n x TRI_NB, ycol[i * TRI_NB + c]
    __shared__ double t_s[TRI_NB][TRI_NB];
    __shared__ double ld[TRI_NB][TRI_NB];          // diagonal block of L
    const int c0 = blockIdx.x * TRI_NB;
    const int tid = threadIdx.x;
    const int ri = tid / TRI_NB, ci = tid % TRI_NB;
    const int c = c0 + ci;
    for (int r0 = c0; r0 < n; r0 += TRI_NB) {
        const int i = r0 + ri;
        if (i < n) {
            const double* lrow = Lf + (int64_t)i * n;
            double acc = 0.0;
            for (int k = c0; k < r0; ++k) acc = acc + lrow[k] * ycol[k * TRI_NB + ci];
            ld[ri][ci] = r0 + ci < n ? lrow[r0 + ci] : 0.0;
            t_s[ri][ci] = (i == c ? 1.0 : 0.0) - acc;
        }
        __syncthreads();
        if (ri == 0) {
            for (int rr = 0; rr < TRI_NB && r0 + rr < n; ++rr) {
                double v = t_s[rr][ci];
                for (int k = 0; k < rr; ++k) v = v - ld[rr][k] * ycol[(r0 + k) * TRI_NB + ci];
                ycol[(r0 + rr) * TRI_NB + ci] = (c < n && r0 + rr >= c) ? v / ld[rr][rr] : 0.0;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < n * TRI_NB; e += TRI_THREADS) {
        const int i = e / TRI_NB, cc = e % TRI_NB;
        if (c0 + cc < n) Li[(int64_t)i * n + c0 + cc] = i >= c0 ? ycol[i * TRI_NB + cc] : 0.0;
    }
}

// W = Linv^T Linv (the inverse of A_coarsest); same summation order for (i,j)
// and (j,i), so W is exactly symmetric.
__global__ void __launch_bounds__(BLOCK) k_gram(const double* __restrict__ Li, int n, double* __restrict__ W) {
    const int64_t id = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (id >= (int64_t)n * n) return;
    const int i = (int)(id / n), j = (int)(id % n);
    const int k0 = i > j ? i : j;
    double s = 0.0;
    for (int k = k0; k < n; ++k) s = s + Li[(int64_t)k * n + i] * Li[(int64_t)k * n + j];
    W[id] = s;
}

// Small coarsest levels (n <= SW_NMAX): the inverse in one workgroup by the
// symmetric sweep operator.  Sweeping pivot k of a symmetric M maps
//   M_kk -> -1/d,  M_ik -> M_ik/d,  M_kj -> M_kj/d,  M_ij -> M_ij - M_ik M_kj/d
// (d = M_kk, i, j != k); sweeping every pivot of an SPD matrix (no pivoting
// needed: each d is a Schur-complement pivot, positive) leaves -A^-1.  The
// n^3/2 multiply-adds are the least an explicit inverse costs, and the n
// sequential pivots need one barrier each instead of one launch chain per
// panel.  The lower triangle lives in registers as T x T tiles, one per
// thread (diagonal tiles keep the whole block; only their lower half is ever
// read); pivot column k goes through LDS, double-buffered, written by the
// tiles that hold row k and column k of the lower triangle.
// 6 x 6 tiles on 1024 threads: 43 * 44 / 2 = 946 tiles, n <= 258.  Per pivot
// the step is bound by the LDS reads of the pivot column (2T values per T^2
// updates) and the barrier; 8 x 8 tiles on 512 threads read less but hide
// less latency and measure slower.
constexpr int SW_T = 6;
constexpr int SW_THREADS = 1024;
constexpr int SW_NMAX = 43 * SW_T;                // 258
constexpr int SW_NPAD = 264;                      // pivot buffer length (16-byte multiple)

template <int T>
__device__ __forceinline__ void sweep_publish(double (&m)[T][T], double* __restrict__ buf, double* __restrict__ rpiv,
                                              int TI, int TJ, int kb, int kk, bool& fail) {
    // column kb*T + kk of the symmetric matrix, read from lower-triangle
    // positions: rows >= k from tile column kb, rows < k from tile row kb.
    // The tile holding the pivot also publishes its reciprocal.  kk is a
    // compile-time constant at every call, so register indices stay static.
    const bool diag = TI == TJ;
    if (TJ == kb) {
#pragma unroll
        for (int a = 0; a < T; ++a)
            if (!diag || a >= kk) buf[TI * T + a] = m[a][kk];
    }
    if (TI == kb) {
#pragma unroll
        for (int b = 0; b < T; ++b)
            if (!diag || b < kk) buf[TJ * T + b] = m[kk][b];
        if (diag) {
            const double d = m[kk][kk];
            if (!(d > 0.0)) fail = true;
            *rpiv = d > 0.0 ? -1.0 / d : -1.0;     // minus the reciprocal
        }
    }
}

// blk (may be null): workgroup b inverts the diagonal block of blk[2b + 1]
// rows from row blk[2b] on (a contiguous island) into W + woff[b]; without
// it the one workgroup inverts the whole matrix of n rows.
template <int T, int NT>
__global__ void __launch_bounds__(NT) k_dense_sweep(const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val, int n,
                                                    double* __restrict__ W, int32_t* __restrict__ err,
                                                    const int32_t* __restrict__ blk = nullptr,
                                                    const int64_t* __restrict__ woff = nullptr) {
    __shared__ __align__(16) double cb[2][SW_NPAD];
    __shared__ double rp[2];
    int r0 = 0;
    if (blk) {
        r0 = blk[2 * blockIdx.x];
        n = blk[2 * blockIdx.x + 1];
        W += woff[blockIdx.x];
    }
    const int nb = (n + T - 1) / T;
    const int ntiles = nb * (nb + 1) / 2;
    const int tid = threadIdx.x;
    const bool active = tid < ntiles;
    int TI = -1, TJ = -1;      // inactive threads own nothing and publish nothing
    if (active) {
        TI = (int)((sqrt(8.0 * (double)tid + 1.0) - 1.0) * 0.5);
        while ((TI + 1) * (TI + 2) / 2 <= tid) ++TI;
        while (TI * (TI + 1) / 2 > tid) --TI;
        TJ = tid - TI * (TI + 1) / 2;
    }
    const int i0 = active ? TI * T : 0, j0 = active ? TJ * T : 0;
    double m[T][T];
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b) m[a][b] = 0.0;
    if (active) {
#pragma unroll
        for (int a = 0; a < T; ++a) {
            const int i = i0 + a;
            if (i < n) {
                for (int e = rowptr[r0 + i]; e < rowptr[r0 + i + 1]; ++e) {
                    const int c = col[e] - r0 - j0;
                    const double v = val[e];
#pragma unroll
                    for (int b = 0; b < T; ++b)
                        if (c == b) m[a][b] = v;
                }
            }
        }
    }
    bool fail = false;
    sweep_publish<T>(m, cb[0], &rp[0], TI, TJ, 0, 0, fail);
    __syncthreads();
    int p = 0;
    for (int kb = 0; kb < nb; ++kb) {
#pragma unroll
        for (int kk = 0; kk < T; ++kk) {
            const int k = kb * T + kk;
            if (k < n) {     // uniform across the workgroup
                const double nr = rp[p];           // -1/d
                double ci[T], cj[T], si[T];
#pragma unroll
                for (int a = 0; a < T; ++a) {
                    ci[a] = cb[p][i0 + a];
                    cj[a] = cb[p][j0 + a];
                }
                // M_ij - M_ik M_kj / d everywhere, then row and column k
#pragma unroll
                for (int a = 0; a < T; ++a) {
                    si[a] = ci[a] * nr;
#pragma unroll
                    for (int b = 0; b < T; ++b) m[a][b] = fma(si[a], cj[b], m[a][b]);
                }
                if (TJ == kb) {
#pragma unroll
                    for (int a = 0; a < T; ++a) m[a][kk] = -si[a];
                }
                if (TI == kb) {
#pragma unroll
                    for (int b = 0; b < T; ++b) m[kk][b] = -(cj[b] * nr);
                    if (TJ == kb) m[kk][kk] = nr;
                }
                if (k + 1 < n) {     // the next pivot, (kb, kk + 1) or (kb + 1, 0)
                    const int kk_next = kk + 1 < T ? kk + 1 : 0;
                    sweep_publish<T>(m, cb[p ^ 1], &rp[p ^ 1], TI, TJ, kk + 1 < T ? kb : kb + 1, kk_next, fail);
                }
                __syncthreads();
                p ^= 1;
            }
        }
    }
    if (fail) atomicOr(err, DEVERR_NOTSPD);
    if (active) {
#pragma unroll
        for (int a = 0; a < T; ++a)
#pragma unroll
            for (int b = 0; b < T; ++b) {
                const int i = i0 + a, j = j0 + b;
                if (i < n && j < n && (TI != TJ || a >= b)) {
                    W[(int64_t)i * n + j] = -m[a][b];
                    W[(int64_t)j * n + i] = -m[a][b];
                }
            }
    }
}

// ------------------------------------------------------ island hierarchies
// Island of each fine unknown from its node row (rows: the islands' first
// node rows, then the total).
__global__ void __launch_bounds__(BLOCK) k_island0(const int64_t* __restrict__ nodes, int64_t n, int nx,
                                                   const int32_t* __restrict__ rows, int nisl,
                                                   int32_t* __restrict__ isl) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int32_t j = (int32_t)(nodes[i] / nx);
    int lo = 0, hi = nisl - 1;            // last island with rows[island] <= j
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rows[mid] <= j) lo = mid; else hi = mid - 1;
    }
    isl[i] = lo;
}

// Per island: row count, first and last row of this level (cnt, first, last
// pre-set to 0, INT_MAX, -1).  Islands are row ranges, so nearly every wave
// lies in one island: such a wave makes one update per counter instead of 64
// on the same address.
__global__ void __launch_bounds__(BLOCK) k_island_stats(const int32_t* __restrict__ isl, int64_t n,
                                                        int32_t* __restrict__ cnt, int32_t* __restrict__ first,
                                                        int32_t* __restrict__ last) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int lane = (int)(threadIdx.x & 63);
    const int64_t i0 = i - lane;                      // the wave's first row
    if (i0 >= n) return;                              // the whole wave is past the end
    const bool ok = i < n;                            // a prefix of the wave's lanes
    const int32_t b = ok ? isl[i] : -1;
    const int32_t b0 = __shfl(b, 0);
    if (__all(!ok || b == b0)) {
        if (lane == 0) {
            const int32_t k = (int32_t)(n - i0 < 64 ? n - i0 : 64);
            atomicAdd(&cnt[b0], k);
            atomicMin(&first[b0], (int32_t)i0);
            atomicMax(&last[b0], (int32_t)i0 + k - 1);
        }
        return;
    }
    if (!ok) return;
    atomicAdd(&cnt[b], 1);
    atomicMin(&first[b], (int32_t)i);
    atomicMax(&last[b], (int32_t)i);
}

// Island of each coarse unknown: that of its members.
__global__ void __launch_bounds__(BLOCK) k_island_next(const int32_t* __restrict__ agg,
                                                       const int32_t* __restrict__ isl, int64_t n,
                                                       int32_t* __restrict__ isl_next) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    if (agg[i] >= 0) isl_next[agg[i]] = isl[i];
}

// Each island's own Gershgorin bound on this level: the largest row bound of
// its rows (bit patterns of non-negative doubles order like the values).  A
// wave whose rows all lie in one island takes its maximum in registers and
// makes one update.
__global__ void __launch_bounds__(BLOCK) k_island_rho(const double* __restrict__ rowv,
                                                      const int32_t* __restrict__ isl,
                                                      const int8_t* __restrict__ frz, int64_t n,
                                                      unsigned long long* __restrict__ rho_isl) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int lane = (int)(threadIdx.x & 63);
    if (i - lane >= n) return;                        // the whole wave is past the end
    const bool ok = i < n && !(frz && frz[i]);
    const int32_t b = ok ? isl[i] : -1;
    double v = ok ? rowv[i] : 0.0;
    const unsigned long long m = __ballot(ok);
    if (m == 0) return;
    const int lead = __ffsll((long long)m) - 1;       // the first lane with a row
    const int32_t bl = __shfl(b, lead);
    if (__all(!ok || b == bl)) {
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
        if (lane == lead) atomicMax(&rho_isl[bl], (unsigned long long)__double_as_longlong(v));
        return;
    }
    if (ok) atomicMax(&rho_isl[b], (unsigned long long)__double_as_longlong(v));
}

// The smoothers and the prolongator of a level take omega / d: scaling the
// stored diagonal of island k's rows by rho_k / rho (rho the level's bound,
// omega = 4 / (3 rho)) gives those rows the weight 4 / (3 rho_k) that the
// island's own hierarchy has (the operator's values keep the true diagonal).
__global__ void __launch_bounds__(BLOCK) k_island_diag(double* __restrict__ diag, const int32_t* __restrict__ isl,
                                                       const int8_t* __restrict__ frz, int64_t n,
                                                       const unsigned long long* __restrict__ rho_isl,
                                                       const unsigned long long* __restrict__ rho_level) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n || (frz && frz[i])) return;
    const double rk = __longlong_as_double((long long)rho_isl[isl[i]]);
    const double r = __longlong_as_double((long long)*rho_level);
    diag[i] = diag[i] * (rk / r);
}

// Rows of the islands that end at this level, and each row's block (-1
// outside the blocks); ending[island] is the island's block or -1.
__global__ void __launch_bounds__(BLOCK) k_island_rows(const int32_t* __restrict__ isl, int64_t n,
                                                       const int32_t* __restrict__ ending, int8_t* __restrict__ frz,
                                                       int32_t* __restrict__ blk) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int32_t b = ending[isl[i]];
    if (frz) frz[i] = b >= 0 ? 1 : 0;
    blk[i] = b;
}

__global__ void __launch_bounds__(BLOCK) k_compact(const int32_t* __restrict__ flag, const int32_t* __restrict__ off,
                                                   int64_t n, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n && flag[i]) out[off[i]] = (int32_t)i;
}

// omega = 4 / (3 rho) from the bit pattern left by k_max_f64.
__global__ void k_omega(const unsigned long long* __restrict__ rho_bits, double* __restrict__ scal) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double rho = __longlong_as_double((long long)*rho_bits);
    scal[0] = rho;
    scal[1] = 4.0 / (3.0 * rho);
}

// Gather the sizes the host reports (nnz per level) into one array.
// Everything the setup reads back, gathered into one block for one copy:
// nnz of A, P, R per level, (rho, omega) per level, the fine strip and box
// counts, and the status words.
struct ReportArgs {
    int nlev;
    const int32_t* a_tot[MAX_LEVELS];
    const int32_t* p_tot[MAX_LEVELS];
    const int32_t* r_tot[MAX_LEVELS];
    const int32_t* ra_tot[MAX_LEVELS];
    const int32_t* sell_w[3 * MAX_LEVELS];   // widths of the sliced A, P, A P
    const double* scal;      // 2 * MAX_LEVELS
    const int32_t* counts;   // 3
    const int32_t* stat;     // 4 (SetupStat)
};

struct ReportBlock {
    int64_t nnz[4 * MAX_LEVELS];
    int32_t sell_w[3 * MAX_LEVELS];
    double scal[2 * MAX_LEVELS];
    int32_t counts[3];
    int32_t stat[4];
};

__global__ void k_report(ReportArgs R, ReportBlock* __restrict__ out) {
    const int l = threadIdx.x;
    if (l < R.nlev) {
        out->nnz[4 * l + 0] = R.a_tot[l] ? *R.a_tot[l] : 0;
        out->nnz[4 * l + 1] = R.p_tot[l] ? *R.p_tot[l] : 0;
        out->nnz[4 * l + 2] = R.r_tot[l] ? *R.r_tot[l] : 0;
        out->nnz[4 * l + 3] = R.ra_tot[l] ? *R.ra_tot[l] : 0;
        for (int m = 0; m < 3; ++m) out->sell_w[3 * l + m] = R.sell_w[3 * l + m] ? *R.sell_w[3 * l + m] : 0;
    }
    if (l < 2 * MAX_LEVELS) out->scal[l] = R.scal[l];
    if (l < 3) out->counts[l] = R.counts[l];
    if (l < 4) out->stat[l] = R.stat[l];
}

// ------------------------------------------------------------- host helpers
static unsigned max_grid(int64_t n) {
    int64_t g = (n + BLOCK - 1) / BLOCK;
    if (g > 1024) g = 1024;
    return (unsigned)(g > 0 ? g : 1);
}

// Device status words of one setup: [0] error flags, [1] count, [2] max.
struct SetupStat {
    int32_t err;
    int32_t count;
    int32_t maxv;
    int32_t pad;
};

// Pinned host copy of the status words for reads that let the device go on
// working (one per host thread, kept until the process ends); null if pinned
// memory cannot be had, and the plain read is used.
static SetupStat* pinned_stat() {
    thread_local SetupStat* p = nullptr;
    thread_local bool tried = false;
    if (!tried) {
        tried = true;
        if (hipHostMalloc((void**)&p, sizeof(SetupStat), hipHostMallocPortable) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
    }
    return p;
}

static int read_stat(const int32_t* dstat, SetupStat* h, hipStream_t s);

// The status read of a level with work enqueued behind it: the words are
// copied to pinned memory and an event is recorded, then `more` enqueues
// work that does not depend on them, and the host waits for the event only,
// so the device has that work to do while the host reads the words and
// issues the next launches.
template <class F>
static int read_stat_then(amg_handle* H, const int32_t* dstat, SetupStat* h, hipStream_t s, F&& more) {
    SetupStat* ps = pinned_stat();
    if (!ps) {
        EB_TRY(more());
        return read_stat(dstat, h, s);
    }
    if (!H->ev_stat) EB_HIP(hipEventCreateWithFlags(&H->ev_stat, hipEventDisableTiming));
    EB_HIP(hipMemcpyAsync(ps, dstat, sizeof(SetupStat), hipMemcpyDeviceToHost, s));
    EB_HIP(hipEventRecord(H->ev_stat, s));
    const int rc = more();
    // wait even when `more` failed: the copy into the shared pinned words
    // must be complete before they are read or written again
    EB_HIP(hipEventSynchronize(H->ev_stat));
    if (rc != EB_OK) return rc;
    *h = *ps;
    return EB_OK;
}

static int read_stat(const int32_t* dstat, SetupStat* h, hipStream_t s) {
    EB_HIP(hipMemcpyAsync(h, dstat, sizeof(SetupStat), hipMemcpyDeviceToHost, s));
    EB_HIP(hipStreamSynchronize(s));
    return EB_OK;
}

static int err_code(int32_t e, const char* where) {
    if (e & DEVERR_DOMAIN) {
        set_error("%s: a computational point lies on the outermost node layer", where);
        return EB_EDOMAIN;
    }
    if (e & DEVERR_CAP) {
        set_error("%s: a box or accumulator capacity was exceeded", where);
        return EB_ENOSPC;
    }
    if (e & DEVERR_NOTSPD) {
        set_error("%s: non-positive diagonal or Cholesky pivot (operator not SPD)", where);
        return EB_ENOTSPD;
    }
    return EB_OK;
}

// rowptr (n+1 entries) from per-row counts; nnz stays on the device in rowptr[n].
static int rowptr_from_counts(const int32_t* cnt, int64_t n, int32_t** rowptr, hipStream_t s) {
    EB_TRY(dalloc_n(rowptr, n + 1, s));
    EB_TRY(scan_i32_dev(cnt, *rowptr, n, *rowptr + n, s));
    return EB_OK;
}

// Lanes per row: enough (row x lane) threads to fill the GPU when the level
// has few rows (their chains of products are the long ones), within an LDS
// budget per row; P rows (a handful of entries each) keep one lane.
static int launch_accumulate(int mode, AccArgs& args, hipStream_t s) {
    const int ns = args.sm.nslots;
    const size_t per_lane = (size_t)ns * (sizeof(double) + 1);
    int G = 1;
    // (row x lane) thread budget: RAP rows (coarse, long product chains) gain
    // from more lanes than AP rows (measured on the star 2048^2 hierarchy)
    const int64_t cap_thr = mode == ACC_RAP ? 2 * 1024 * 1024 : 512 * 1024;
    if (mode != ACC_P)
        while (G < 64 && args.nrows * (int64_t)(2 * G) <= cap_thr && per_lane * (2 * G) <= 32 * 1024) G *= 2;
    int rows = 256 / G;
    while (rows > 1 && per_lane * G * rows > 64 * 1024) rows >>= 1;
    if (per_lane * G * rows > 150 * 1024) {
        set_error("accumulator needs %zu bytes of LDS per row", per_lane * G);
        return EB_ENOSPC;
    }
    const int nt = rows * G;
    const size_t lds = per_lane * nt + 16;
    const dim3 grid((unsigned)((args.nrows + rows - 1) / rows > 0 ? (args.nrows + rows - 1) / rows : 1));
    if (mode == ACC_P) hipLaunchKernelGGL((k_accumulate<ACC_P>), grid, dim3(nt), lds, s, args, G);
    else if (mode == ACC_AP) hipLaunchKernelGGL((k_accumulate<ACC_AP>), grid, dim3(nt), lds, s, args, G);
    else hipLaunchKernelGGL((k_accumulate<ACC_RAP>), grid, dim3(nt), lds, s, args, G);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// Sparse product via the slot accumulator: one accumulation pass into a
// bounded scratch (row_bound entries per row reserved, each workgroup's rows
// packed at the front of its part), giving per-row counts and starts.  Sized
// by the proven bound, so no host synchronisation is needed.
struct PackedRows {
    int32_t* cnt = nullptr;
    int32_t* start = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
};

static int free_packed(PackedRows& R, hipStream_t s) {
    EB_TRY(dfree(R.cnt, s));
    EB_TRY(dfree(R.start, s));
    EB_TRY(dfree(R.col, s));
    EB_TRY(dfree(R.val, s));
    R = PackedRows();
    return EB_OK;
}

static int accumulate_packed(int mode, AccArgs args, int64_t nrows, int64_t row_bound, PackedRows* out,
                             hipStream_t s) {
    const int64_t cap = nrows * row_bound;
    if (cap >= ((int64_t)1 << 31)) {
        set_error("a sparse matrix bound exceeds 2^31 entries");
        return EB_ENOSPC;
    }
    EB_TRY(dalloc_n(&out->cnt, nrows, s));
    EB_TRY(dalloc_n(&out->start, nrows, s));
    EB_TRY(dalloc_n(&out->col, cap, s));
    EB_TRY(dalloc_n(&out->val, cap, s));
    args.nrows = nrows;
    args.out_cnt = out->cnt;
    args.out_start = out->start;
    args.ell_col = out->col;
    args.ell_val = out->val;
    args.ell_stride = (int)row_bound;
    return launch_accumulate(mode, args, s);
}

// The same, then a prefix sum of the row counts and a copy into CSR (the
// exact nnz stays in rowptr[nrows]).
static int accumulate_product(int mode, AccArgs args, int64_t nrows, int64_t row_bound, int32_t** rowptr,
                              int32_t** col, double** val, hipStream_t s) {
    PackedRows R;
    EB_TRY(accumulate_packed(mode, args, nrows, row_bound, &R, s));
    EB_TRY(rowptr_from_counts(R.cnt, nrows, rowptr, s));
    EB_TRY(dalloc_n(col, nrows * row_bound, s));
    EB_TRY(dalloc_n(val, nrows * row_bound, s));
    hipLaunchKernelGGL(k_ell_to_csr, dim3(grid_for(nrows)), dim3(BLOCK), 0, s, R.col, R.val, R.start, nrows,
                       *rowptr, *col, *val);
    EB_LAUNCH_CHECK();
    return free_packed(R, s);
}

// ---------------------------------------------------------- sliced ELL
// Rows of the source: CSR (rowptr) or packed product rows (start, cnt).
struct RowSrc {
    const int32_t* rowptr;
    const int32_t* start;
    const int32_t* cnt;
    const int32_t* col;
    const double* val;
    __device__ int32_t first(int64_t r) const { return rowptr ? rowptr[r] : start[r]; }
    __device__ int32_t len(int64_t r) const { return rowptr ? rowptr[r + 1] - rowptr[r] : cnt[r]; }
};

// The longest row of each of three matrices with the same rows (width[0..2]
// pre-set to 0): each wavefront's maxima, then an atomic only where a
// maximum exceeds the width already recorded (rows of a level are nearly
// uniform, so after the first wavefronts hardly any atomic is left: one
// address taking an atomic from every wavefront serialises them).
__global__ void __launch_bounds__(BLOCK) k_sell_width3(RowSrc A, RowSrc B, RowSrc C, int64_t n,
                                                       int32_t* __restrict__ width) {
    const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    int32_t w[3] = {r < n ? A.len(r) : 0, r < n ? B.len(r) : 0, r < n ? C.len(r) : 0};
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) w[m] = max(w[m], __shfl_xor(w[m], off, WAVE));
    if ((threadIdx.x & (WAVE - 1)) == 0) {
#pragma unroll
        for (int m = 0; m < 3; ++m)
            if (w[m] > __atomic_load_n(&width[m], __ATOMIC_RELAXED)) atomicMax(&width[m], w[m]);
    }
}

// Row r of a sliced matrix of width w from its source rows (padding: value 0
// and the row's last column, column 0 for an empty row).
__device__ inline void sell_fill_row(const RowSrc& M, int64_t r, int32_t w, int32_t* __restrict__ col,
                                     double* __restrict__ val) {
    const int32_t base = (int32_t)(r / 64) * 64 * w + (int32_t)(r % 64);
    const int32_t f = M.first(r), m = M.len(r);
    int32_t last = 0;
    for (int32_t k = 0; k < w; ++k) {
        if (k < m) {
            last = M.col[f + k];
            col[base + 64 * k] = last;
            val[base + 64 * k] = M.val[f + k];
        } else {
            col[base + 64 * k] = last;
            val[base + 64 * k] = 0.0;
        }
    }
}

// The three sliced matrices of a level in one pass over its rows.
__global__ void __launch_bounds__(BLOCK) k_sell_fill3(RowSrc A, RowSrc B, RowSrc C, int64_t n,
                                                      const int32_t* __restrict__ width, int32_t* __restrict__ ca,
                                                      double* __restrict__ va, int32_t* __restrict__ cb,
                                                      double* __restrict__ vb, int32_t* __restrict__ cc,
                                                      double* __restrict__ vc) {
    const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r >= n) return;
    sell_fill_row(A, r, width[0], ca, va);
    sell_fill_row(B, r, width[1], cb, vb);
    sell_fill_row(C, r, width[2], cc, vc);
}

// Transpose of a matrix given by rows (CSR or packed), into CSR: counts per
// column, then each entry placed by an atomic slot (rows sorted afterwards).
__global__ void __launch_bounds__(BLOCK) k_trs_count(RowSrc M, int64_t n, int32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int32_t f = M.first(i), m = M.len(i);
    for (int32_t k = 0; k < m; ++k) atomicAdd(&cnt[M.col[f + k]], 1);
}

__global__ void __launch_bounds__(BLOCK) k_trs_fill(RowSrc M, int64_t n, const int32_t* __restrict__ t_rowptr,
                                                    int32_t* __restrict__ fill, int32_t* __restrict__ t_col,
                                                    double* __restrict__ t_val) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int32_t f = M.first(i), m = M.len(i);
    for (int32_t k = 0; k < m; ++k) {
        const int32_t c = M.col[f + k];
        const int32_t pos = t_rowptr[c] + atomicAdd(&fill[c], 1);
        t_col[pos] = (int32_t)i;
        t_val[pos] = M.val[f + k];
    }
}

// Sliced ELL copies of the level's A, P and A P (n rows each, at most
// bound[m] entries per row): storage sized by the bounds, the widths found
// on the device (no host synchronisation; the host learns them from the
// setup's final report).  Three launches for the three matrices.
static int build_sells(Level& L, const RowSrc (&M)[3], int64_t n, const int64_t (&bound)[3], hipStream_t s) {
    Sell* out[3] = {&L.sa, &L.sp, &L.sap};
    const int64_t nslices = (n + 63) / 64;
    EB_TRY(dalloc_n(&L.sell_w, 4, s));
    for (int m = 0; m < 3; ++m) {
        out[m]->cap = nslices * 64 * (bound[m] > 0 ? bound[m] : 1);
        if (out[m]->cap >= ((int64_t)1 << 31)) {
            set_error("a sliced matrix bound exceeds 2^31 entries");
            return EB_ENOSPC;
        }
        out[m]->wdev = L.sell_w + m;
        EB_TRY(dalloc_n(&out[m]->col, out[m]->cap, s));
        EB_TRY(dalloc_n(&out[m]->val, out[m]->cap, s));
    }
    {
        const FillSpec f[] = {{L.sell_w, 4 * sizeof(int32_t), 0u}};
        EB_TRY(fill_words(f, 1, s));
    }
    if (n > 0) {
        hipLaunchKernelGGL(k_sell_width3, dim3(grid_for(n)), dim3(BLOCK), 0, s, M[0], M[1], M[2], n, L.sell_w);
        hipLaunchKernelGGL(k_sell_fill3, dim3(grid_for(n)), dim3(BLOCK), 0, s, M[0], M[1], M[2], n,
                           (const int32_t*)L.sell_w, L.sa.col, L.sa.val, L.sp.col, L.sp.val, L.sap.col, L.sap.val);
        EB_LAUNCH_CHECK();
    }
    return EB_OK;
}

// V-cycle copies of level l >= 1 (not the coarsest): sliced A, P and A P for
// the up pass and R A for the down pass, from the A P kept by build_next.
// They feed neither the coarsening nor the coarsest inverse, so setup builds
// them after launching that inverse on the side stream, where they overlap it.
static int build_cycle_copies(amg_handle* H, int l, hipStream_t s) {
    Level& L = H->lev[l];
    if (!L.apk_col) return EB_OK;
    const int64_t n = L.n, nc = H->lev[l + 1].n;
    const int slots = L.apk_slots;
    RowSrc map = {nullptr, L.apk_start, L.apk_cnt, L.apk_col, L.apk_val};
    // sliced copies of A, P and A P for the coarse V-cycle kernels
    const RowSrc ms[3] = {{L.a_rowptr, nullptr, nullptr, L.a_col, L.a_val},
                          {L.p_rowptr, nullptr, nullptr, L.p_col, L.p_val}, map};
    const int64_t bounds[3] = {L.row_bound, L.apk_pbound, slots};
    EB_TRY(build_sells(L, ms, n, bounds, s));
    // R A = P^T A = (A P)^T (A symmetric): rows of level l + 1 over level-l
    // columns, sorted, for the one-pass residual and restriction
    L.ra_cap = n * slots;
    int32_t* tcnt = nullptr;
    int32_t* tfill = nullptr;
    EB_TRY(dalloc_n(&tcnt, nc, s));
    EB_TRY(dalloc_n(&tfill, nc, s));
    {
        const FillSpec f[] = {{tcnt, sizeof(int32_t) * nc, 0u}, {tfill, sizeof(int32_t) * nc, 0u}};
        EB_TRY(fill_words(f, 2, s));
    }
    hipLaunchKernelGGL(k_trs_count, dim3(grid_for(n)), dim3(BLOCK), 0, s, map, n, tcnt);
    EB_LAUNCH_CHECK();
    EB_TRY(rowptr_from_counts(tcnt, nc, &L.ra_rowptr, s));
    EB_TRY(dalloc_n(&L.ra_col, L.ra_cap, s));
    EB_TRY(dalloc_n(&L.ra_val, L.ra_cap, s));
    hipLaunchKernelGGL(k_trs_fill, dim3(grid_for(n)), dim3(BLOCK), 0, s, map, n, (const int32_t*)L.ra_rowptr,
                       tfill, L.ra_col, L.ra_val);
    EB_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sort_rows<BLOCK, 2048>), dim3((unsigned)nc), dim3(BLOCK), 0, s,
                       (const int32_t*)L.ra_rowptr, L.ra_col, L.ra_val, nc);
    EB_LAUNCH_CHECK();
    EB_TRY(dfree(tcnt, s));
    EB_TRY(dfree(tfill, s));
    void* q[] = {L.apk_cnt, L.apk_start, L.apk_col, L.apk_val};
    for (void* p : q) EB_TRY(dfree(p, s));
    L.apk_cnt = L.apk_start = L.apk_col = nullptr;
    L.apk_val = nullptr;
    return EB_OK;
}

static int make_coarsest(amg_handle* H, int l, hipStream_t s, int32_t* err) {
    Level& L = H->lev[l];
    L.is_coarsest = 1;
    const int64_t n = L.n;
    if (n == 0) return EB_OK;
    if (n > H->params.dense_limit) {
        set_error("coarsest level has %lld unknowns, above the dense limit %d (coarsening stalled)",
                  (long long)n, H->params.dense_limit);
        return EB_ENOSPC;
    }
    EB_TRY(dalloc_n(&L.dense_inv, n * n, s));
    if (n <= SW_NMAX) {
        // one workgroup on one CU: run it on the side stream so that the fine
        // solve layout, built next on s, overlaps it; setup_impl joins before
        // its read-back (the kernel reads this level's A and writes dense_inv
        // and the error word, none of which s frees or rewrites meanwhile)
        hipStream_t side = nullptr;
        EB_TRY(side_stream(&side));
        if (!H->ev_fork) EB_HIP(hipEventCreateWithFlags(&H->ev_fork, hipEventDisableTiming));
        if (!H->ev_join) EB_HIP(hipEventCreateWithFlags(&H->ev_join, hipEventDisableTiming));
        EB_HIP(hipEventRecord(H->ev_fork, s));
        EB_HIP(hipStreamWaitEvent(side, H->ev_fork, 0));
        hipLaunchKernelGGL((k_dense_sweep<SW_T, SW_THREADS>), dim3(1), dim3(SW_THREADS), 0, side, L.a_rowptr,
                           L.a_col, L.a_val, (int)n, L.dense_inv, err);
        EB_LAUNCH_CHECK();
        EB_HIP(hipEventRecord(H->ev_join, side));
        H->join_pending = 1;
        return EB_OK;
    }
    // larger levels (coarsening stalled): blocked Cholesky, L^-1, L^-T L^-1
    double* dense = nullptr;
    double* linv = nullptr;
    EB_TRY(dalloc_n(&dense, n * n, s));
    EB_TRY(dalloc_n(&linv, n * n, s));
    hipLaunchKernelGGL(k_csr_to_dense, dim3(grid_for(n)), dim3(BLOCK), 0, s, L.a_rowptr, L.a_col, L.a_val, n, dense);
    EB_LAUNCH_CHECK();
    for (int k0 = 0; k0 < n; k0 += CHOL_NB) {
        const int rpt = (int)((n - k0 + CHOL_THREADS - 1) / CHOL_THREADS);
        switch (rpt) {
            case 1: hipLaunchKernelGGL(k_chol_panel<1>, dim3(1), dim3(CHOL_THREADS), 0, s, dense, (int)n, k0, err); break;
            case 2: hipLaunchKernelGGL(k_chol_panel<2>, dim3(1), dim3(CHOL_THREADS), 0, s, dense, (int)n, k0, err); break;
            case 3: hipLaunchKernelGGL(k_chol_panel<3>, dim3(1), dim3(CHOL_THREADS), 0, s, dense, (int)n, k0, err); break;
            case 4: hipLaunchKernelGGL(k_chol_panel<4>, dim3(1), dim3(CHOL_THREADS), 0, s, dense, (int)n, k0, err); break;
            case 5: hipLaunchKernelGGL(k_chol_panel<5>, dim3(1), dim3(CHOL_THREADS), 0, s, dense, (int)n, k0, err); break;
            default:
                set_error("dense coarsest level of %lld unknowns exceeds the panel kernel", (long long)n);
                return EB_EINVAL;
        }
        const int64_t m = n - k0 - CHOL_NB;
        if (m > 0) {
            const int64_t nbk = (m + CHOL_TB - 1) / CHOL_TB;
            hipLaunchKernelGGL(k_chol_trailing, dim3((unsigned)(nbk * (nbk + 1) / 2)), dim3(CHOL_THREADS), 0, s,
                               dense, (int)n, k0);
        }
    }
    EB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_tri_inverse, dim3((unsigned)((n + TRI_NB - 1) / TRI_NB)), dim3(TRI_THREADS),
                       sizeof(double) * TRI_NB * n, s, dense, (int)n, linv);
    EB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_gram, dim3(grid_for(n * n)), dim3(BLOCK), 0, s, linv, (int)n, L.dense_inv);
    EB_LAUNCH_CHECK();
    EB_TRY(dfree(dense, s));
    EB_TRY(dfree(linv, s));
    return EB_OK;
}

// Aggregate level l and build level l+1; *stop = 1 if level l becomes the
// coarsest.  One host synchronisation (coarse count, box maximum, errors).
// frz (island hierarchies from level 1 on): rows of the islands that end at
// this level, n_act the other rows; they are left out of the aggregation, so
// the coarser levels hold only the islands that go on.
static int build_next(amg_handle* H, int l, hipStream_t s, int32_t* dstat, const int8_t* frz, int64_t n_act,
                      const int32_t* isl, int* stop) {
    Level& L = H->lev[l];
    *stop = 0;
    const int64_t n = L.n;
    const int dim = H->d.dim;
    const bool island_rule = H->nisl > 0 && l >= 1;   // the per-island size rule decides instead
    if ((!island_rule && n <= H->params.coarse_max) || l + 1 >= H->params.max_levels || l + 1 >= MAX_LEVELS) {
        *stop = 1;
        return EB_OK;
    }
    int32_t* err = dstat;
    NB3 nb;
    for (int a = 0; a < 3; ++a) {
        L.nb[a] = (L.ext[a] + 2) / 3;
        nb.v[a] = L.nb[a];
    }
    const int64_t nboxes = (int64_t)nb.v[0] * nb.v[1] * nb.v[2];
    L.nboxes = nboxes;
    int32_t *cnt = nullptr, *boff = nullptr, *fillpos = nullptr, *members = nullptr, *lrank = nullptr;
    int32_t* boxid = nullptr;
    EB_TRY(dalloc_n(&lrank, n, s));
    EB_TRY(dalloc_n(&L.box_ncomp, nboxes, s));
    EB_TRY(dalloc_n(&L.box_cstart, nboxes, s));
    const bool pull0 = l == 0 && H->unk_off_tmp && H->kind_tmp;
    if (!pull0) {
        EB_TRY(dalloc_n(&cnt, nboxes, s));
        EB_TRY(dalloc_n(&fillpos, nboxes, s));
    }
    {
        const FillSpec f[] = {{dstat + 2, sizeof(int32_t), 0u},
                              {cnt, pull0 ? 0 : sizeof(int32_t) * nboxes, 0u},
                              {fillpos, pull0 ? 0 : sizeof(int32_t) * nboxes, 0u}};
        EB_TRY(fill_words(f, pull0 ? 1 : 3, s));
    }
    if (pull0) {
        hipLaunchKernelGGL(k_box_components0, dim3(grid_for(nboxes)), dim3(BLOCK), 0, s, H->kind_tmp, H->d, nb,
                           nboxes, H->unk_off_tmp, lrank, L.box_ncomp);
        EB_LAUNCH_CHECK();
    } else {
        EB_TRY(dalloc_n(&boff, nboxes, s));
        EB_TRY(dalloc_n(&members, n, s));
        EB_TRY(dalloc_n(&boxid, n, s));
        hipLaunchKernelGGL(k_box_count, dim3(grid_for(n)), dim3(BLOCK), 0, s, L.coords, n, nb, (const int8_t*)frz, cnt,
                           boxid);
        EB_LAUNCH_CHECK();
        EB_TRY(scan_i32_dev(cnt, boff, nboxes, dstat + 3, s));     // total (= n) unused
        hipLaunchKernelGGL(k_box_fill, dim3(grid_for(n)), dim3(BLOCK), 0, s, boxid, n, boff, fillpos, members);
        EB_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_box_components, dim3(grid_for(nboxes, BOX_WAVES)), dim3(BOX_WAVES * WAVE), 0, s, boff,
                           cnt, members, L.a_rowptr, L.a_col, boxid, nboxes, lrank, L.box_ncomp, err);
        EB_LAUNCH_CHECK();
    }
    EB_TRY(scan_i32_dev(L.box_ncomp, L.box_cstart, nboxes, dstat + 1, s));
    hipLaunchKernelGGL(k_max_i32, dim3(max_grid(nboxes)), dim3(BLOCK), 0, s, L.box_ncomp, nboxes, dstat + 2);
    EB_LAUNCH_CHECK();
    EB_TRY(dfree(cnt, s));
    EB_TRY(dfree(boff, s));
    EB_TRY(dfree(fillpos, s));
    EB_TRY(dfree(members, s));
    EB_TRY(dfree(boxid, s));
    SetupStat st;
    // the V-cycle copies of the level above (they need this level's size,
    // not these words) keep the device busy while the host reads them
    EB_TRY(read_stat_then(H, dstat, &st, s, [&]() { return l >= 2 ? build_cycle_copies(H, l - 1, s) : EB_OK; }));
    EB_TRY(err_code(st.err, "aggregation"));
    const int64_t nc = st.count;
    const int maxc = st.maxv;
    if ((double)nc > H->params.min_reduction * (double)(frz ? n_act : n) || nc == 0) {
        EB_TRY(dfree(lrank, s));
        *stop = 1;
        return EB_OK;
    }
    L.max_comp = maxc;
    EB_TRY(dalloc_n(&L.agg, n, s));
    hipLaunchKernelGGL(k_assign_agg, dim3(grid_for(n)), dim3(BLOCK), 0, s, L.coords, n, nb, L.box_cstart, lrank,
                       (const int8_t*)frz, L.agg);
    EB_LAUNCH_CHECK();
    EB_TRY(dfree(lrank, s));

    Level& C = H->lev[l + 1];
    C = Level();
    C.n = nc;
    for (int a = 0; a < 3; ++a) C.ext[a] = nb.v[a];
    EB_TRY(dalloc_n(&C.coords, 3 * nc, s));
    EB_TRY(dalloc_n(&C.cinfo, nc, s));
    hipLaunchKernelGGL(k_coarse_coords, dim3(grid_for(nboxes)), dim3(BLOCK), 0, s, L.box_ncomp, L.box_cstart, nb,
                       nboxes, C.coords, C.cinfo);
    EB_LAUNCH_CHECK();

    // Gershgorin bound and smoothing weight, kept on the device
    double* rowv = nullptr;
    unsigned long long* drho = nullptr;
    EB_TRY(dalloc_n(&rowv, n, s));
    EB_TRY(dalloc_n(&drho, 1, s));
    EB_HIP(hipMemsetAsync(drho, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_gershgorin_rows, dim3(grid_for(n)), dim3(BLOCK), 0, s, L.a_rowptr, L.a_col, L.a_val, L.diag,
                       n, (const int8_t*)frz, rowv);
    hipLaunchKernelGGL(k_max_f64, dim3(max_grid(n)), dim3(BLOCK), 0, s, rowv, n, drho, err);
    hipLaunchKernelGGL(k_omega, dim3(1), dim3(1), 0, s, drho, H->dscal + 2 * l);
    EB_LAUNCH_CHECK();
    if (isl) {
        // island hierarchies: every island smooths with its own weight
        unsigned long long* rho_isl = nullptr;
        EB_TRY(dalloc_n(&rho_isl, (int64_t)H->nisl, s));
        EB_HIP(hipMemsetAsync(rho_isl, 0, sizeof(unsigned long long) * (size_t)H->nisl, s));
        hipLaunchKernelGGL(k_island_rho, dim3(grid_for(n)), dim3(BLOCK), 0, s, (const double*)rowv, isl, frz, n,
                           rho_isl);
        hipLaunchKernelGGL(k_island_diag, dim3(grid_for(n)), dim3(BLOCK), 0, s, L.diag, isl, frz, n,
                           (const unsigned long long*)rho_isl, (const unsigned long long*)drho);
        EB_LAUNCH_CHECK();
        EB_TRY(dfree(rho_isl, s));
    }
    EB_TRY(dfree(rowv, s));
    EB_TRY(dfree(drho, s));

    const int slots = (dim == 3 ? 27 : 9) * maxc;
    AccArgs args;
    memset(&args, 0, sizeof(args));
    args.sm.dim = dim;
    args.sm.maxc = maxc;
    args.sm.nslots = slots;
    args.sm.cinfo = C.cinfo;
    args.sm.cstart = L.box_cstart;
    args.sm.nb = nb;
    args.err = err;

    // P = (I - omega D^-1 A) P_tent; a row has at most min(row of A, slots) entries
    const int64_t p_bound = L.row_bound < slots ? L.row_bound : slots;
    args.row_coords = L.coords;
    args.centre_div = 3;
    args.x_rowptr = L.a_rowptr; args.x_col = L.a_col; args.x_val = L.a_val;
    args.agg = L.agg; args.diag = L.diag; args.omega = H->dscal + 2 * l + 1;
    EB_TRY(accumulate_product(ACC_P, args, n, p_bound, &L.p_rowptr, &L.p_col, &L.p_val, s));

    // R = P^T (same number of entries)
    if (l == 0 && H->unk_off_tmp) {
        int32_t* tcnt = nullptr;
        EB_TRY(dalloc_n(&tcnt, nc, s));
        hipLaunchKernelGGL((k_tr0_pull<false>), dim3(grid_for(nc * TR_G)), dim3(BLOCK), 0, s, nc, C.cinfo, H->kind_tmp, H->d,
                           H->unk_off_tmp, L.p_rowptr, L.p_col, L.p_val, tcnt, nullptr, nullptr, nullptr);
        EB_LAUNCH_CHECK();
        EB_TRY(rowptr_from_counts(tcnt, nc, &L.r_rowptr, s));
        EB_TRY(dalloc_n(&L.r_col, n * p_bound, s));
        EB_TRY(dalloc_n(&L.r_val, n * p_bound, s));
        hipLaunchKernelGGL((k_tr0_pull<true>), dim3(grid_for(nc * TR_G)), dim3(BLOCK), 0, s, nc, C.cinfo, H->kind_tmp, H->d,
                           H->unk_off_tmp, L.p_rowptr, L.p_col, L.p_val, nullptr, L.r_rowptr, L.r_col, L.r_val);
        EB_LAUNCH_CHECK();
        EB_TRY(dfree(tcnt, s));
    } else {
        int32_t* tcnt = nullptr;
        int32_t* tfill = nullptr;
        EB_TRY(dalloc_n(&tcnt, nc, s));
        EB_TRY(dalloc_n(&tfill, nc, s));
        {
            const FillSpec f[] = {{tcnt, sizeof(int32_t) * nc, 0u}, {tfill, sizeof(int32_t) * nc, 0u}};
            EB_TRY(fill_words(f, 2, s));
        }
        hipLaunchKernelGGL(k_tr_count, dim3(grid_for(n)), dim3(BLOCK), 0, s, L.p_rowptr, L.p_col, n, tcnt);
        EB_LAUNCH_CHECK();
        EB_TRY(rowptr_from_counts(tcnt, nc, &L.r_rowptr, s));
        EB_TRY(dalloc_n(&L.r_col, n * p_bound, s));
        EB_TRY(dalloc_n(&L.r_val, n * p_bound, s));
        hipLaunchKernelGGL(k_tr_fill, dim3(grid_for(n)), dim3(BLOCK), 0, s, L.p_rowptr, L.p_col, L.p_val, n,
                           L.r_rowptr, tfill, L.r_col, L.r_val);
        EB_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_sort_rows<WAVE, 256>), dim3((unsigned)nc), dim3(WAVE), 0, s, L.r_rowptr, L.r_col, L.r_val,
                           nc);
        EB_LAUNCH_CHECK();
        EB_TRY(dfree(tcnt, s));
        EB_TRY(dfree(tfill, s));
    }

    // AP = A P (left in its packed scratch, read only by the next pass), then
    // A_c = R (A P); rows of both have at most `slots` entries
    PackedRows ap;
    args.x_rowptr = L.a_rowptr; args.x_col = L.a_col; args.x_val = L.a_val;
    args.y_rowptr = L.p_rowptr; args.y_col = L.p_col; args.y_val = L.p_val;
    args.y_start = nullptr; args.y_cnt = nullptr;
    args.row_coords = L.coords;
    args.centre_div = 3;
    EB_TRY(accumulate_packed(ACC_AP, args, n, slots, &ap, s));
    args.x_rowptr = L.r_rowptr; args.x_col = L.r_col; args.x_val = L.r_val;
    args.y_rowptr = nullptr; args.y_col = ap.col; args.y_val = ap.val;
    args.y_start = ap.start; args.y_cnt = ap.cnt;
    args.row_coords = C.coords;
    args.centre_div = 1;
    EB_TRY(accumulate_product(ACC_RAP, args, nc, slots, &C.a_rowptr, &C.a_col, &C.a_val, s));
    C.row_bound = slots;
    if (l >= 1) {
        // kept for the V-cycle copies, built once the coarsest inverse runs
        L.apk_cnt = ap.cnt;
        L.apk_start = ap.start;
        L.apk_col = ap.col;
        L.apk_val = ap.val;
        L.apk_slots = slots;
        L.apk_pbound = p_bound;
        ap = PackedRows();
    } else {
        EB_TRY(free_packed(ap, s));
    }
    EB_TRY(dalloc_n(&C.diag, nc, s));
    hipLaunchKernelGGL(k_extract_diag, dim3(grid_for(nc)), dim3(BLOCK), 0, s, C.a_rowptr, C.a_col, C.a_val, nc,
                       C.diag, err);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

static void free_level(Level& L, hipStream_t s) {
    void* ptrs[] = {L.a_rowptr, L.a_col, L.a_val, L.diag, L.p_rowptr, L.p_col, L.p_val, L.r_rowptr, L.r_col,
                    L.r_val, L.agg, L.coords, L.cinfo, L.box_cstart, L.box_ncomp, L.dense_inv, L.fz_off, L.fz_woff,
                    L.fz_inv, L.fz_blk, L.sell_w, L.apk_cnt, L.apk_start, L.apk_col, L.apk_val, L.rv, L.ev, L.tmp,
                    L.sv, L.a_val32, L.p_val32, L.r_val32, L.diag32, L.rv32, L.ev32, L.tmp32, L.sv32};
    for (void* p : ptrs) (void)dfree(p, s);
    for (Sell* m : {&L.sa, &L.sp, &L.sap}) {
        void* q[] = {m->col, m->val, m->val32};
        for (void* p : q) (void)dfree(p, s);
    }
    {
        void* q[] = {L.ra_rowptr, L.ra_col, L.ra_val, L.ra_val32};
        for (void* p : q) (void)dfree(p, s);
    }
    L = Level();
}

int free_handle_memory(amg_handle* H) {
    hipStream_t s = H->stream;
    // a setup that failed between fork and join may leave the coarsest
    // inverse running on the side stream
    if (H->join_pending && H->ev_join) (void)hipEventSynchronize(H->ev_join);
    H->join_pending = 0;
    // blocks go back to the library cache tagged with the setup stream: wait
    // for any solve still running on another stream first
    if (H->last_stream && H->last_stream != s) (void)hipStreamSynchronize(H->last_stream);
    free_batch(H, s);
    drop_iteration_graphs(H);
    for (int l = 0; l < MAX_LEVELS; ++l) free_level(H->lev[l], s);
    void* ptrs[] = {H->unk_off_tmp, H->strips, H->tiles, H->box_map0, H->box_w0, H->box_w0_32, H->dcount, H->boxes0, H->fine_nodes, H->fine_pad, H->diag_p, H->dinv_p, H->agg_p, H->x, H->rr[0], H->rr[1],
                    H->z, H->zt, H->p[0], H->p[1], H->q, H->res, H->bvec, H->sc, H->dscal, H->red.pq, H->red.rr,
                    H->red.rz[0], H->red.rz[1], H->red.aux, H->red.aux2, H->diag_p32, H->dinv_p32, H->res32, H->zt32, H->z32,
                    H->wf, H->wf32, H->dinv_p16, H->z16, H->bf_p[0], H->bf_p[1], H->bf_p[2]};
    for (void* p : ptrs) (void)dfree(p, s);
    H->sc_host = nullptr;
    H->tim_ev = nullptr;    // process-wide event pool, not owned
    if (H->ev0) (void)hipEventDestroy(H->ev0);
    if (H->ev1) (void)hipEventDestroy(H->ev1);
    if (H->ev_fork) (void)hipEventDestroy(H->ev_fork);
    if (H->ev_join) (void)hipEventDestroy(H->ev_join);
    if (H->ev_stat) (void)hipEventDestroy(H->ev_stat);
    H->ev_fork = H->ev_join = nullptr;
    return EB_OK;
}

// A device int32 buffer freed when it goes out of scope (setup temporaries).
struct TmpI32 {
    int32_t* p = nullptr;
    hipStream_t s = nullptr;
    explicit TmpI32(hipStream_t st) : s(st) {}
    ~TmpI32() {
        if (p) (void)dfree(p, s);
    }
};

// Island hierarchies: per island, its row count, first and last row on level
// l (isl: the island of each row), read back to the host.
static int island_stats(amg_handle* H, const int32_t* isl, int64_t n, std::vector<int32_t>* cnt,
                        std::vector<int32_t>* first, std::vector<int32_t>* last, hipStream_t s) {
    const int m = H->nisl;
    TmpI32 d(s);
    EB_TRY(dalloc_n(&d.p, 3 * (int64_t)m, s));
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(m)), dim3(BLOCK), 0, s, d.p, (int64_t)m, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(m)), dim3(BLOCK), 0, s, d.p + m, (int64_t)m, 0x7fffffff);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(m)), dim3(BLOCK), 0, s, d.p + 2 * m, (int64_t)m, -1);
    if (n > 0)
        hipLaunchKernelGGL(k_island_stats, dim3(grid_for(n)), dim3(BLOCK), 0, s, isl, n, d.p, d.p + m, d.p + 2 * m);
    EB_LAUNCH_CHECK();
    std::vector<int32_t> h(3 * (size_t)m);
    EB_HIP(hipMemcpyAsync(h.data(), d.p, sizeof(int32_t) * 3 * (size_t)m, hipMemcpyDeviceToHost, s));
    EB_HIP(hipStreamSynchronize(s));
    cnt->assign(h.begin(), h.begin() + m);
    first->assign(h.begin() + m, h.begin() + 2 * m);
    last->assign(h.begin() + 2 * m, h.end());
    return EB_OK;
}

// The diagonal blocks of the islands `ending` on level l (their rows must be
// contiguous), each inverted by one workgroup of the sweep kernel; the block
// of every row goes to L.fz_blk and, unless `all` (the blocks cover the
// level: it is the coarsest), the rows of those islands to *frz.
static int make_island_blocks(amg_handle* H, int l, const int32_t* isl, const std::vector<int>& ending,
                              const std::vector<int32_t>& cnt, const std::vector<int32_t>& first,
                              const std::vector<int32_t>& last, bool all, int8_t** frz, int32_t* err,
                              hipStream_t s) {
    Level& L = H->lev[l];
    const int nb = (int)ending.size();
    std::vector<int32_t> blk(2 * (size_t)nb), map((size_t)H->nisl, -1);
    std::vector<int64_t> woff((size_t)nb);
    int64_t tot = 0;
    for (int k = 0; k < nb; ++k) {
        const int i = ending[k];
        if (last[i] - first[i] + 1 != cnt[i]) {
            set_error("amg_setup_islands: island %d is not one row range on level %d (place the islands on node "
                      "rows that are multiples of 3^%d)", i, l, l);
            return EB_EINVAL;
        }
        if (cnt[i] > SW_NMAX) {
            set_error("amg_setup_islands: island %d ends with %d unknowns, more than %d", i, cnt[i], SW_NMAX);
            return EB_ENOSPC;
        }
        blk[2 * k] = first[i];
        blk[2 * k + 1] = cnt[i];
        woff[k] = tot;
        tot += (int64_t)cnt[i] * cnt[i];
        map[i] = k;
    }
    TmpI32 dmap(s);
    EB_TRY(dalloc_n(&L.fz_off, 2 * (int64_t)nb, s));
    EB_TRY(dalloc_n(&L.fz_woff, (int64_t)nb, s));
    EB_TRY(dalloc_n(&L.fz_inv, tot > 0 ? tot : 1, s));
    EB_TRY(dalloc_n(&L.fz_blk, L.n, s));
    EB_TRY(dalloc_n(&dmap.p, (int64_t)H->nisl, s));
    EB_HIP(hipMemcpyAsync(L.fz_off, blk.data(), sizeof(int32_t) * blk.size(), hipMemcpyHostToDevice, s));
    EB_HIP(hipMemcpyAsync(L.fz_woff, woff.data(), sizeof(int64_t) * woff.size(), hipMemcpyHostToDevice, s));
    EB_HIP(hipMemcpyAsync(dmap.p, map.data(), sizeof(int32_t) * map.size(), hipMemcpyHostToDevice, s));
    if (!all) EB_TRY(dalloc_n(frz, L.n, s));
    hipLaunchKernelGGL(k_island_rows, dim3(grid_for(L.n)), dim3(BLOCK), 0, s, isl, L.n, (const int32_t*)dmap.p,
                       all ? nullptr : *frz, L.fz_blk);
    hipLaunchKernelGGL((k_dense_sweep<SW_T, SW_THREADS>), dim3((unsigned)nb), dim3(SW_THREADS), 0, s, L.a_rowptr,
                       L.a_col, L.a_val, 0, L.fz_inv, err, (const int32_t*)L.fz_off, (const int64_t*)L.fz_woff);
    EB_LAUNCH_CHECK();
    // the host vectors above are read by the copies: wait before they go
    EB_HIP(hipStreamSynchronize(s));
    L.nfz = nb;
    L.fz_all = all ? 1 : 0;
    return EB_OK;
}

int solve_layout_alloc(amg_handle* H, hipStream_t s);    // solve.hip
int solve_layout_finish(amg_handle* H, hipStream_t s);   // solve.hip

static int setup_impl(amg_handle* H, const int8_t* kind, const double* a, hipStream_t s) {
    const GridDims& d = H->d;
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    int32_t* dstat = nullptr;
    int32_t* flag = nullptr;
    int32_t* unk_off = nullptr;
    EB_TRY(dalloc_n(&dstat, 4, s));
    EB_TRY(dalloc_n(&H->dscal, 2 * MAX_LEVELS, s));
    {
        const FillSpec f[] = {{dstat, sizeof(SetupStat), 0u}, {H->dscal, sizeof(double) * 2 * MAX_LEVELS, 0u}};
        EB_TRY(fill_words(f, 2, s));
    }
    EB_TRY(dalloc_n(&flag, nn, s));
    EB_TRY(dalloc_n(&unk_off, nn, s));
    hipLaunchKernelGGL(k_fine_flags, dim3(grid_for(nn)), dim3(BLOCK), 0, s, kind, d, nn, flag, dstat);
    EB_LAUNCH_CHECK();
    EB_TRY(scan_i32_dev(flag, unk_off, nn, dstat + 1, s));
    SetupStat st;
    EB_TRY(read_stat(dstat, &st, s));
    EB_TRY(err_code(st.err, "amg_setup"));
    const int64_t nunk = st.count;
    H->n_fine = nunk;
    Level& L0 = H->lev[0];
    L0 = Level();
    L0.n = nunk;
    L0.ext[0] = d.nx;
    L0.ext[1] = d.ny;
    L0.ext[2] = d.nz;
    L0.row_bound = 2 * d.dim + 1;
    EB_TRY(dalloc_n(&H->fine_nodes, nunk, s));
    EB_TRY(dalloc_n(&L0.coords, 3 * nunk, s));
    EB_TRY(dalloc_n(&L0.diag, nunk, s));
    int32_t* rowcnt = nullptr;
    EB_TRY(dalloc_n(&rowcnt, nunk, s));
    hipLaunchKernelGGL(k_fine_rows, dim3(grid_for(nn)), dim3(BLOCK), 0, s, kind, d, nn, flag, unk_off, rowcnt,
                       H->fine_nodes, L0.coords);
    EB_LAUNCH_CHECK();
    EB_TRY(rowptr_from_counts(rowcnt, nunk, &L0.a_rowptr, s));
    EB_TRY(dalloc_n(&L0.a_col, nunk * L0.row_bound, s));
    EB_TRY(dalloc_n(&L0.a_val, nunk * L0.row_bound, s));
    hipLaunchKernelGGL(k_fine_fill, dim3(grid_for(nunk)), dim3(BLOCK), 0, s, kind, a, H->beta_tmp, H->sigma, d,
                       nunk, H->fine_nodes, unk_off, L0.a_rowptr, L0.a_col, L0.a_val, L0.diag);
    EB_LAUNCH_CHECK();
    EB_TRY(dfree(rowcnt, s));
    EB_TRY(dfree(flag, s));
    H->unk_off_tmp = unk_off;   // node -> unknown map, used by the level-0 transpose
    H->kind_tmp = kind;

    // island hierarchies: the island of each row of the current level
    TmpI32 isl(s);
    std::vector<char> going_on;
    if (H->nisl > 0) {
        EB_TRY(dalloc_n(&isl.p, nunk > 0 ? nunk : 1, s));
        if (nunk > 0)
            hipLaunchKernelGGL(k_island0, dim3(grid_for(nunk)), dim3(BLOCK), 0, s, H->fine_nodes, nunk, d.nx,
                               (const int32_t*)H->isl_rows, H->nisl, isl.p);
        EB_LAUNCH_CHECK();
        going_on.assign((size_t)H->nisl, 1);
    }
    int l = 0;
    while (true) {
        if (H->lev[l].n == 0) {
            H->lev[l].is_coarsest = 1;
            break;
        }
        // an island whose rows on this level number at most coarse_max ends
        // here (as its own hierarchy would); once no island goes on, this
        // level is the coarsest and its blocks are every island's exact solve
        int8_t* frz = nullptr;
        int64_t n_act = H->lev[l].n;
        if (H->nisl > 0 && l >= 1) {
            std::vector<int32_t> cnt, first, last;
            EB_TRY(island_stats(H, isl.p, H->lev[l].n, &cnt, &first, &last, s));
            std::vector<int> ending, present;
            bool any_left = false;
            for (int i = 0; i < H->nisl; ++i) {
                if (cnt[i] == 0) continue;
                present.push_back(i);
                if (cnt[i] <= H->params.coarse_max) ending.push_back(i);
                else any_left = true;
            }
            if (!any_left) {
                EB_TRY(make_island_blocks(H, l, isl.p, present, cnt, first, last, true, nullptr, dstat, s));
                H->lev[l].is_coarsest = 1;
                break;
            }
            if (!ending.empty()) {
                EB_TRY(make_island_blocks(H, l, isl.p, ending, cnt, first, last, false, &frz, dstat, s));
                for (int i : ending) n_act -= cnt[i];
            }
        }
        int stop = 0;
        const int rc = build_next(H, l, s, dstat, frz, n_act, H->nisl > 0 && l >= 1 ? isl.p : nullptr, &stop);
        if (rc != EB_OK) {
            if (frz) (void)dfree(frz, s);
            return rc;
        }
        if (frz) EB_TRY(dfree(frz, s));
        if (H->unk_off_tmp) {
            EB_TRY(dfree(H->unk_off_tmp, s));
            H->unk_off_tmp = nullptr;
        }
        if (stop) {
            EB_TRY(make_coarsest(H, l, s, dstat));
            break;
        }
        if (H->nisl > 0) {
            TmpI32 next(s);
            const int64_t nc = H->lev[l + 1].n;
            EB_TRY(dalloc_n(&next.p, nc > 0 ? nc : 1, s));
            hipLaunchKernelGGL(k_island_next, dim3(grid_for(H->lev[l].n)), dim3(BLOCK), 0, s, H->lev[l].agg, isl.p,
                               H->lev[l].n, next.p);
            EB_LAUNCH_CHECK();
            std::swap(isl.p, next.p);
        }
        ++l;
    }
    H->nlev = l + 1;
    // V-cycle copies of the middle levels: after the coarsest inverse was
    // launched on the side stream, so that they run beside it
    for (int k = 1; k < H->nlev - 1; ++k) EB_TRY(build_cycle_copies(H, k, s));
    EB_TRY(solve_layout_alloc(H, s));
    if (H->join_pending) {      // the coarsest inverse (side stream)
        EB_HIP(hipStreamWaitEvent(s, H->ev_join, 0));
        H->join_pending = 0;
    }

    // one read-back: sizes of every level, smoothing weights, errors
    ReportArgs R;
    memset(&R, 0, sizeof(R));
    R.nlev = H->nlev;
    for (int k = 0; k < H->nlev; ++k) {
        const Level& L = H->lev[k];
        R.a_tot[k] = L.a_rowptr ? L.a_rowptr + L.n : nullptr;
        if (!L.is_coarsest && L.p_rowptr) {
            R.p_tot[k] = L.p_rowptr + L.n;
            R.r_tot[k] = L.r_rowptr + H->lev[k + 1].n;
            if (L.ra_rowptr) R.ra_tot[k] = L.ra_rowptr + H->lev[k + 1].n;
        }
        R.sell_w[3 * k + 0] = L.sa.wdev;
        R.sell_w[3 * k + 1] = L.sp.wdev;
        R.sell_w[3 * k + 2] = L.sap.wdev;
    }
    R.scal = H->dscal;
    R.counts = H->dcount;
    R.stat = dstat;
    static_assert(2 * MAX_LEVELS <= 64, "k_report runs one 64-thread block");
    ReportBlock* drep = nullptr;
    EB_TRY(dalloc_n(&drep, 1, s));
    hipLaunchKernelGGL(k_report, dim3(1), dim3(64), 0, s, R, drep);
    EB_LAUNCH_CHECK();
    ReportBlock rep;
    EB_HIP(hipMemcpyAsync(&rep, drep, sizeof(ReportBlock), hipMemcpyDeviceToHost, s));
    EB_HIP(hipStreamSynchronize(s));
    memcpy(&st, rep.stat, sizeof(st));
    H->nstrips = rep.counts[0];
    H->nboxes0 = rep.counts[1];
    H->ntiles = rep.counts[2];
    EB_TRY(dfree(drep, s));
    for (int k = 0; k < H->nlev; ++k) {
        Level& L = H->lev[k];
        L.nnz_a = rep.nnz[4 * k];
        L.nnz_p = rep.nnz[4 * k + 1];
        L.nnz_r = rep.nnz[4 * k + 2];
        L.nnz_ap = rep.nnz[4 * k + 3];
        L.sa.width = rep.sell_w[3 * k + 0];
        L.sp.width = rep.sell_w[3 * k + 1];
        L.sap.width = rep.sell_w[3 * k + 2];
        if (!L.is_coarsest) {
            L.rho = rep.scal[2 * k];
            L.omega = rep.scal[2 * k + 1];
            L.omega_setup = L.omega;
        }
    }
    EB_TRY(err_code(st.err, "amg_setup"));
    EB_TRY(solve_layout_finish(H, s));
    EB_TRY(dfree(dstat, s));
    return EB_OK;
}

}  // namespace eb

using namespace eb;

static int amg_setup_impl(const eb_grid_t* g, const int8_t* kind, const double* a, const double* beta,
                          double sigma, const amg_params_t* p, amg_handle_t** Hout, void* stream, int32_t nisl = 0,
                          const int32_t* isl_rows = nullptr) {
    clear_error();
    if (!Hout || !kind || !a) {
        set_error("amg_setup: null pointer");
        return EB_EINVAL;
    }
    *Hout = nullptr;
    GridDims d;
    EB_TRY(make_dims(g, &d));
    if (!(sigma >= 0.0) || isinf(sigma)) {
        set_error("amg_setup: sigma must be finite and >= 0");
        return EB_EINVAL;
    }
    amg_params_t prm;
    prm.coarse_max = 256;
    prm.max_levels = 16;
    prm.min_reduction = 0.6;
    prm.dense_limit = 1200;
    prm.reserved = 0;
    prm.alloc = nullptr;
    prm.free = nullptr;
    prm.alloc_ctx = nullptr;
    if (p) {
        prm = *p;
        if (prm.coarse_max < 1 || prm.max_levels < 1 || !(prm.min_reduction > 0.0 && prm.min_reduction <= 1.0) ||
            prm.dense_limit < 1) {
            set_error("amg_setup: invalid parameters");
            return EB_EINVAL;
        }
        if ((prm.alloc == nullptr) != (prm.free == nullptr)) {
            set_error("amg_setup: alloc and free must be given together");
            return EB_EINVAL;
        }
        if (prm.dense_limit > 1200) prm.dense_limit = 1200;
    }
    amg_handle* H = new (std::nothrow) amg_handle();
    if (!H) {
        set_error("amg_setup: out of host memory");
        return EB_EINVAL;
    }
    H->d = d;
    H->sigma = sigma;
    H->stream = (hipStream_t)stream;
    H->params = prm;
    H->beta_tmp = beta;
    H->beta_on = beta != nullptr;
    AllocScope scope(&H->params);
    int rc = EB_OK;
    if (nisl > 0) {
        H->nisl = nisl;
        rc = dalloc_n(&H->isl_rows, (int64_t)nisl + 1, H->stream);
        if (rc == EB_OK && hipMemcpyAsync(H->isl_rows, isl_rows, sizeof(int32_t) * ((size_t)nisl + 1),
                                          hipMemcpyHostToDevice, H->stream) != hipSuccess) {
            set_error("amg_setup_islands: copy of the island rows failed");
            rc = EB_EHIP;
        }
    }
    if (rc == EB_OK) rc = setup_impl(H, kind, a, H->stream);
    if (H->isl_rows) {
        (void)hipStreamSynchronize(H->stream);
        (void)dfree(H->isl_rows, H->stream);
        H->isl_rows = nullptr;
    }
    H->beta_tmp = nullptr;
    if (rc != EB_OK) {
        char msg[1024];
        snprintf(msg, sizeof(msg), "%s", eb_last_error());
        (void)free_handle_memory(H);
        delete H;
        set_error("%s", msg);
        return rc;
    }
    *Hout = H;
    return EB_OK;
}

extern "C" int amg_setup(const eb_grid_t* g, const int8_t* kind, const double* a, double sigma,
                         const amg_params_t* p, amg_handle_t** Hout, void* stream) {
    return amg_setup_impl(g, kind, a, nullptr, sigma, p, Hout, stream);
}

extern "C" int amg_setup_beta(const eb_grid_t* g, const int8_t* kind, const double* a, const double* beta,
                              double sigma, const amg_params_t* p, amg_handle_t** Hout, void* stream) {
    if (!beta) {
        set_error("amg_setup_beta: null beta");
        return EB_EINVAL;
    }
    return amg_setup_impl(g, kind, a, beta, sigma, p, Hout, stream);
}

extern "C" int amg_setup_islands(const eb_grid_t* g, const int8_t* kind, const double* a, double sigma,
                                 int32_t nseg, const int32_t* seg_rows, const amg_params_t* p, amg_handle_t** H,
                                 void* stream) {
    clear_error();
    if (!g || g->dim != 2) {
        set_error("amg_setup_islands: 2-D grids only");
        return EB_EINVAL;
    }
    if (nseg < 1 || !seg_rows) {
        set_error("amg_setup_islands: need at least one island and its rows");
        return EB_EINVAL;
    }
    if (seg_rows[0] != 0 || seg_rows[nseg] != g->n[1] + 1) {
        set_error("amg_setup_islands: island rows must start at 0 and end at the node rows (%d)", g->n[1] + 1);
        return EB_EINVAL;
    }
    for (int i = 0; i < nseg; ++i) {
        if (seg_rows[i + 1] <= seg_rows[i]) {
            set_error("amg_setup_islands: island rows must increase");
            return EB_EINVAL;
        }
    }
    return amg_setup_impl(g, kind, a, nullptr, sigma, p, H, stream, nseg, seg_rows);
}

extern "C" void amg_free(amg_handle_t* H) {
    if (!H) return;
    {
        AllocScope scope(&H->params);
        (void)free_handle_memory(H);
    }
    delete H;
}

extern "C" int amg_num_levels(const amg_handle_t* H) { return H ? H->nlev : 0; }

extern "C" const int64_t* amg_fine_nodes(const amg_handle_t* H) { return H ? H->fine_nodes : nullptr; }

extern "C" int amg_level_info(const amg_handle_t* H, int level, amg_level_info_t* out) {
    if (!H || !out || level < 0 || level >= H->nlev) {
        set_error("amg_level_info: bad handle or level");
        return EB_EINVAL;
    }
    const Level& L = H->lev[level];
    memset(out, 0, sizeof(*out));
    out->n = L.n;
    out->nnz_a = L.nnz_a;
    out->nnz_p = L.nnz_p;
    out->nnz_r = L.nnz_r;
    out->rho = L.rho;
    out->omega = L.omega;
    out->is_coarsest = L.is_coarsest;
    out->max_comp = L.max_comp;
    out->nnz_ap = (int32_t)L.nnz_ap;
    for (int a = 0; a < 3; ++a) out->ext[a] = L.ext[a];
    out->a_rowptr = L.a_rowptr; out->a_col = L.a_col; out->a_val = L.a_val;
    out->p_rowptr = L.p_rowptr; out->p_col = L.p_col; out->p_val = L.p_val;
    out->r_rowptr = L.r_rowptr; out->r_col = L.r_col; out->r_val = L.r_val;
    out->agg = L.agg;
    out->coords = L.coords;
    out->dense_inv = L.dense_inv;
    return EB_OK;
}
