// Embedded-boundary assembly kernels: classification, the diagonal with its
// cut records (line-by-line and RBF rows), the right-hand side and the
// matrix-free operator on dense node fields.
//
// Built with -ffp-contract=off: the diagonal a_k, q, c and the crossing
// coordinates are evaluated in a fixed order with separately rounded
// operations, so an independent FP64 implementation can reproduce them bit
// for bit (t = psi_in / (psi_in - psi_out); q = (j-1) + t; c = 1/q;
// a_k = n_regular, then a_k += c side by side in the order -x,+x,-y,+y,-z,+z).
#include <vector>

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

// Whether the boundary-point side of unknown n at offset st takes an RBF row
// (Sec. 2.3; Algorithm 2 step 3: in the mixed strategy, when the node two
// steps out is inside; a computational point is at least two nodes from the
// outer layer, so that node exists).
__device__ inline bool rbf_side(const double* __restrict__ psi, int64_t n, int64_t st, int mode) {
    return mode == EB_BC_RBF || (mode == EB_BC_MIXED && psi[n + 2 * st] < 0.0);
}

// Records of an unknown: one per line-by-line side, two per RBF side.
__device__ inline int node_records(const int8_t* __restrict__ kind, const double* __restrict__ psi, int64_t n,
                                   const GridDims& d, int mode) {
    int c = 0;
    if (kind[n] == 2) {
        for (int axis = 0; axis < d.dim; ++axis) {
            const int64_t st = axis_stride(d, axis);
            if (kind[n - st] != 2) c += mode != EB_BC_LINE && rbf_side(psi, n, -st, mode) ? 2 : 1;
            if (kind[n + st] != 2) c += mode != EB_BC_LINE && rbf_side(psi, n, st, mode) ? 2 : 1;
        }
    }
    return c;
}

// Whether unknown n has a side that takes an RBF row.
__device__ inline bool node_has_rbf(const int8_t* __restrict__ kind, const double* __restrict__ psi, int64_t n,
                                    const GridDims& d, int mode) {
    for (int axis = 0; axis < d.dim; ++axis) {
        const int64_t st = axis_stride(d, axis);
        if (kind[n - st] != 2 && rbf_side(psi, n, -st, mode)) return true;
        if (kind[n + st] != 2 && rbf_side(psi, n, st, mode)) return true;
    }
    return false;
}

// Cut records per workgroup (the same node-to-workgroup map as k_diag_cuts,
// which places each node's records after those of the workgroups before it
// and of the nodes before it in its own).
__global__ void __launch_bounds__(BLOCK) k_count_cuts(const int8_t* __restrict__ kind, const double* __restrict__ psi,
                                                      GridDims d, int64_t nnodes, int mode,
                                                      int32_t* __restrict__ block_cuts) {
    __shared__ int32_t wcount[BLOCK / WAVE];
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    int c = n < nnodes ? node_records(kind, psi, n, d, mode) : 0;
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

// Variable conductivity (Eq. (1)): beta holds dim node fields back to back,
// field `axis` giving beta at the face between each node and its neighbour in
// +axis; the face on the minus side of node n is that of n - e_axis.  NULL
// means beta = 1.
__device__ inline double face_beta(const double* __restrict__ beta, int64_t n, const GridDims& d, int side) {
    const int axis = side >> 1;
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    const int64_t face = (side & 1) ? n : n - axis_stride(d, axis);
    return beta[(int64_t)axis * nn + face];
}

// The side's interpolation coefficient c = 1/q from the walk's end j (first
// outside node, j >= 2), and its cut record m (if below the capacity).
// With beta, c = beta_face / q (the face's conductivity times the weight).
__device__ inline double diag_side(const double* __restrict__ psi, int64_t n, const NodePos& p, const GridDims& d,
                                   int side, int j, int64_t m, eb_cut_t* __restrict__ cuts, int64_t cap,
                                   const double* __restrict__ beta) {
    const int axis = side >> 1;
    const int step = (side & 1) ? 1 : -1;
    const int64_t st = axis_stride(d, axis) * step;
    const double psi_in = psi[n + (int64_t)(j - 1) * st];
    const double psi_out = psi[n + (int64_t)j * st];
    const double t = psi_in / (psi_in - psi_out);
    const double q = (double)(j - 1) + t;
    const double c = beta ? face_beta(beta, n, d, side) * (1.0 / q) : 1.0 / q;
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


// ------------------------------------------------------------- RBF rows
// Sec. 2.2: the BP value is interpolated through the computational point and
// two boundary points by the r^3 spline with linear polynomials (Eq. (rbf),
// (rbf_ubp)); with three points the polynomial condition Pi lambda = 0 leaves
// lambda = 0, so the interpolant is the linear one through the three points
// and the weights are barycentric coordinates.  The boundary points follow
// Algorithm 1 on Gamma = the zero set of the piecewise-linear interpolant of
// psi on the triangles that split each cell along its (i,j)-(i+1,j+1)
// diagonal.  Everything is computed relative to the computational point in
// units of h, so node offsets are exact small integers, and each quantity
// with the same separately rounded operations in the same order as a plain
// evaluation (the file is built without contraction): the points come out
// bit for bit equal to such an evaluation.
struct Pt2 {
    double x, y;
};

constexpr double RBF_EPS = 0.025;                 // distinctness tolerance of Algorithm 1 (Sec. 2.3)
constexpr double RBF_COS45 = 0.7071067811865476;  // cos(pi/4) = sin(pi/4)
constexpr int RBF_WLO = -3, RBF_WHI = 2;          // window of cells (lower-left corner offsets)

// Gamma's segment in the lower (v (0,0),(1,0),(1,1)) or upper ((0,0),(1,1),
// (0,1)) triangle of the cell at offset (oi, oj) from node (i, j): from the
// first to the second crossed edge in the order (v0 v1), (v1 v2), (v2 v0);
// the crossing on an edge is v_in + t (v_out - v_in), t = psi_in / (psi_in -
// psi_out).  False if the cell is off the grid or the triangle not crossed.
__device__ inline bool tri_segment(const double* __restrict__ psi, const GridDims& d, int i, int j, int oi, int oj,
                                   bool upper, Pt2& S0, Pt2& S1) {
    const int ci = i + oi, cj = j + oj;
    if (ci < 0 || ci + 1 > d.nx - 1 || cj < 0 || cj + 1 > d.ny - 1) return false;
    const int vx[3] = {0, 1, upper ? 0 : 1};
    const int vy[3] = {0, upper ? 1 : 0, 1};
    double vp[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) vp[k] = psi[(int64_t)(cj + vy[k]) * d.sy + (ci + vx[k])];
    bool cr[3];
    Pt2 pt[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int a = e, b = e == 2 ? 0 : e + 1;
        const bool ina = vp[a] < 0.0, inb = vp[b] < 0.0;
        cr[e] = ina != inb;
        const int vi = ina ? a : b, vo = ina ? b : a;
        const double pin = vp[vi], pout = vp[vo];
        const double t = cr[e] ? pin / (pin - pout) : 0.0;
        pt[e].x = (double)(oi + vx[vi]) + t * (double)(vx[vo] - vx[vi]);
        pt[e].y = (double)(oj + vy[vi]) + t * (double)(vy[vo] - vy[vi]);
    }
    if (!(cr[0] || cr[1] || cr[2])) return false;
    S0 = cr[0] ? pt[0] : pt[1];
    S1 = cr[2] ? pt[2] : pt[1];
    return true;
}

// Point of [S0, S1] nearest to P and its squared distance.
__device__ inline void seg_closest(const Pt2& P, const Pt2& S0, const Pt2& S1, Pt2& Q, double& d2) {
    const double ex = S1.x - S0.x, ey = S1.y - S0.y;
    const double wx = P.x - S0.x, wy = P.y - S0.y;
    const double den = ex * ex + ey * ey;
    const double num = wx * ex + wy * ey;
    double tau = den > 0.0 ? num / den : 0.0;
    tau = tau < 0.0 ? 0.0 : (tau > 1.0 ? 1.0 : tau);
    Q.x = S0.x + tau * ex;
    Q.y = S0.y + tau * ey;
    const double dx = P.x - Q.x, dy = P.y - Q.y;
    d2 = dx * dx + dy * dy;
}

// Ray O + tau D, tau > 0, against [S0, S1]: keeps the nearest hit.
__device__ inline void seg_ray(const Pt2& O, const Pt2& D, const Pt2& S0, const Pt2& S1, double& best, Pt2& X) {
    const double ex = S1.x - S0.x, ey = S1.y - S0.y;
    const double wx = S0.x - O.x, wy = S0.y - O.y;
    const double denom = D.x * ey - D.y * ex;
    if (denom == 0.0) return;
    const double tau = (wx * ey - wy * ex) / denom;
    const double mu = (wx * D.y - wy * D.x) / denom;
    if (tau > 0.0 && mu >= 0.0 && mu <= 1.0 && tau < best) {
        best = tau;
        X.x = S0.x + mu * ex;
        X.y = S0.y + mu * ey;
    }
}

// First crossing of Gamma by the ray from O along D (relative to node (i, j)).
// The cells are visited column by column along the ray's major axis; in each
// column the ray spans at most two cells of the minor axis, examined with a
// margin of one cell on either side.  Once a hit lies before the far end of
// the current column, no later column can hold a nearer one.  The ray starts
// inside (psi < 0 at the BP) and the outer layer is outside, so it meets
// Gamma before leaving the grid.
__device__ inline bool ray_first_hit(const double* __restrict__ psi, const GridDims& d, int i, int j, const Pt2& O,
                                     const Pt2& D, Pt2& X) {
    const bool xmaj = fabs(D.x) >= fabs(D.y);
    const double o_maj = xmaj ? O.x : O.y, d_maj = xmaj ? D.x : D.y;
    const double o_min = xmaj ? O.y : O.x, d_min = xmaj ? D.y : D.x;
    const int dir = d_maj > 0.0 ? 1 : -1;
    const int base = xmaj ? i : j;
    const int len = xmaj ? d.nx : d.ny;
    double best = INFINITY;
    int c = (int)o_maj + (dir > 0 ? 0 : -1);       // O is a node: integer coordinates
    for (;; c += dir) {
        if (base + c < 0 || base + c + 1 > len - 1) break;
        const double ta = ((double)c - o_maj) / d_maj;
        const double tb = ((double)(c + 1) - o_maj) / d_maj;
        const double t0 = fmax(0.0, fmin(ta, tb)), t1 = fmax(ta, tb);
        const double ya = o_min + t0 * d_min, yb = o_min + t1 * d_min;
        const int m0 = (int)floor(fmin(ya, yb)) - 1, m1 = (int)floor(fmax(ya, yb)) + 1;
        for (int m = m0; m <= m1; ++m) {
            for (int up = 0; up < 2; ++up) {
                Pt2 S0, S1;
                const int oi = xmaj ? c : m, oj = xmaj ? m : c;
                if (tri_segment(psi, d, i, j, oi, oj, up != 0, S0, S1)) seg_ray(O, D, S0, S1, best, X);
            }
        }
        if (best < t1) return true;
    }
    return best < INFINITY;
}

// Algorithm 1 and the weights for the BP side `side` of node n = (i, j):
// boundary points G1, G2 (relative, units of h) and their weights w1, w2 in
// u_BP = w_ij u_ij + w1 u(G1) + w2 u(G2).  False when the three points are
// collinear.
__device__ inline bool rbf_points(const double* __restrict__ psi, const GridDims& d, int i, int j, int side, Pt2& G1,
                                  Pt2& G2, double& w1, double& w2) {
    const Pt2 P = {side == 0 ? -1.0 : side == 1 ? 1.0 : 0.0, side == 2 ? -1.0 : side == 3 ? 1.0 : 0.0};
    const Pt2 Z = {0.0, 0.0};
    double b1 = INFINITY, b2 = INFINITY;
    Pt2 G20 = {0.0, 0.0};
    G1 = G20;
    for (int oj = RBF_WLO; oj <= RBF_WHI; ++oj) {
        for (int oi = RBF_WLO; oi <= RBF_WHI; ++oi) {
            for (int up = 0; up < 2; ++up) {
                Pt2 S0, S1, Q;
                double d2;
                if (!tri_segment(psi, d, i, j, oi, oj, up != 0, S0, S1)) continue;
                seg_closest(P, S0, S1, Q, d2);
                if (d2 < b1) {
                    b1 = d2;
                    G1 = Q;
                }
                seg_closest(Z, S0, S1, Q, d2);
                if (d2 < b2) {
                    b2 = d2;
                    G20 = Q;
                }
            }
        }
    }
    const double dx = G1.x - G20.x, dy = G1.y - G20.y;
    if (dx * dx + dy * dy > RBF_EPS * RBF_EPS) {
        G2 = G20;
    } else {
        // rotate x_BP -> x_G1 counterclockwise by pi/4 and meet Gamma
        const double vx = G1.x - P.x, vy = G1.y - P.y;
        const Pt2 D = {RBF_COS45 * vx - RBF_COS45 * vy, RBF_COS45 * vx + RBF_COS45 * vy};
        if (!ray_first_hit(psi, d, i, j, P, D, G2)) return false;
    }
    const double den = G1.x * G2.y - G1.y * G2.x;
    if (den == 0.0) return false;
    w1 = (P.x * G2.y - P.y * G2.x) / den;
    w2 = (G1.x * P.y - G1.y * P.x) / den;
    return true;
}

// The two records of an RBF side (if below the capacity); returns the side's
// diagonal contribution w1 + w2 added in record order to acc.
__device__ inline double rbf_side_records(const double* __restrict__ psi, int64_t n, const NodePos& p,
                                          const GridDims& d, int side, int64_t m, eb_cut_t* __restrict__ cuts,
                                          int64_t cap, double acc, int32_t* __restrict__ err,
                                          const double* __restrict__ beta) {
    Pt2 G[2];
    double w[2];
    if (!rbf_points(psi, d, p.i, p.j, side, G[0], G[1], w[0], w[1])) {
        atomicOr(err, DEVERR_GEOM);
        return acc;
    }
    if (beta) {
        const double bf = face_beta(beta, n, d, side);
        w[0] = bf * w[0];
        w[1] = bf * w[1];
    }
    const double bx = d.x0 + (double)p.i * d.h, by = d.y0 + (double)p.j * d.h;
    for (int k = 0; k < 2; ++k) {
        if (m + k < cap) {
            eb_cut_t rec;
            rec.node = n;
            rec.dir = side;
            rec.steps = -1 - k;
            rec.q = 0.0;
            rec.c = w[k];
            rec.xg[0] = bx + G[k].x * d.h;
            rec.xg[1] = by + G[k].y * d.h;
            rec.xg[2] = 0.0;
            cuts[m + k] = rec;
        }
        acc = acc + w[k];
    }
    return acc;
}

// The regular sides' part of a_k: their count, or with beta the sum of
// their face values in side order (-x, +x, -y, +y, -z, +z) from 0.
__device__ inline double diag_regular_beta(const int8_t* __restrict__ kind, const double* __restrict__ beta, int64_t n,
                                           const GridDims& d);

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
                                                     const double* __restrict__ beta, GridDims d, int64_t nnodes, int mode,
                                                     const int64_t* __restrict__ block_off,
                                                     double* __restrict__ a, eb_cut_t* __restrict__ cuts,
                                                     int64_t cap, int32_t* __restrict__ err,
                                                     int32_t* __restrict__ ndefer, int64_t* __restrict__ defer) {
    __shared__ int32_t wsum[BLOCK / WAVE];
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const bool unknown = n < nnodes && kind[n] == 2;
    // first record of the node: the workgroup's offset plus the cut sides of
    // the nodes before it in the workgroup (exclusive scan)
    const int cnt = n < nnodes ? node_records(kind, psi, n, d, mode) : 0;
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
    // nodes with an RBF side are done by k_diag_rbf (their records use far more
    // registers than a line walk; kept out of this kernel)
    if (mode != EB_BC_LINE && node_has_rbf(kind, psi, n, d, mode)) return;
    const NodePos p = node_pos(n, d);
    double acc = diag_regular_beta(kind, beta, n, d);
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
        acc = acc + diag_side(psi, n, p, d, side, j, m, cuts, cap, beta);
        ++m;
    }
    a[n] = acc;
}

// The deferred nodes, one workgroup each at a time: per side, the workgroup
// reads DIAG_LONG_NT consecutive nodes of the line per round and takes the
// first that ends the walk (the same test as the thread's walk: an outside
// node, or the outer layer); thread 0 then adds the sides in order.
__global__ void __launch_bounds__(DIAG_LONG_NT) k_diag_long(const double* __restrict__ psi,
                                                            const int8_t* __restrict__ kind,
                                                            const double* __restrict__ beta, GridDims d,
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
        double acc = diag_regular_beta(kind, beta, n, d);
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
            if (tid == 0) acc = acc + diag_side(psi, n, p, d, side, j0 + f, m, cuts, cap, beta);
            ++m;
        }
        if (tid == 0) a[n] = acc;
    }
}

__device__ inline double diag_regular_beta(const int8_t* __restrict__ kind, const double* __restrict__ beta, int64_t n,
                                           const GridDims& d) {
    if (!beta) return (double)diag_regular(kind, n, d);
    double acc = 0.0;
    for (int side = 0; side < 2 * d.dim; ++side) {
        const int64_t st = axis_stride(d, side >> 1) * ((side & 1) ? 1 : -1);
        if (kind[n + st] == 2) acc = acc + face_beta(beta, n, d, side);
    }
    return acc;
}

// The unknowns with an RBF side (mixed and RBF-based strategies, 2-D): the
// same node-to-workgroup map and in-workgroup scan of record counts as
// k_diag_cuts, which skipped them.  Line-by-line sides of such a node end at
// j = 2 (in the mixed strategy a line side has its node two steps out
// outside; the RBF-based one has none), so no walk is needed.
__global__ void __launch_bounds__(BLOCK) k_diag_rbf(const double* __restrict__ psi, const int8_t* __restrict__ kind,
                                                    const double* __restrict__ beta, GridDims d, int64_t nnodes,
                                                    int mode,
                                                    const int64_t* __restrict__ block_off, double* __restrict__ a,
                                                    eb_cut_t* __restrict__ cuts, int64_t cap,
                                                    int32_t* __restrict__ err) {
    __shared__ int32_t wsum[BLOCK / WAVE];
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int cnt = n < nnodes ? node_records(kind, psi, n, d, mode) : 0;
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
    if (n >= nnodes || (*err & DEVERR_DOMAIN)) return;
    if (kind[n] != 2 || !node_has_rbf(kind, psi, n, d, mode)) return;
    const NodePos p = node_pos(n, d);
    double acc = diag_regular_beta(kind, beta, n, d);
    int64_t m = block_off[blockIdx.x] + before;
    for (int side = 0; side < 2 * d.dim; ++side) {
        const int axis = side >> 1;
        const int step = (side & 1) ? 1 : -1;
        const int64_t st = axis_stride(d, axis) * step;
        if (kind[n + st] == 2) continue;
        if (rbf_side(psi, n, st, mode)) {
            acc = rbf_side_records(psi, n, p, d, side, m, cuts, cap, acc, err, beta);
            m += 2;
        } else {
            acc = acc + diag_side(psi, n, p, d, side, 2, m, cuts, cap, beta);
            ++m;
        }
    }
    a[n] = acc;
}

// ------------------------------------------------------------ right-hand side
// b_k = f_k + sum over the cuts of k (ascending side) of u_Gamma * (c / h^2).
// row_scale (optional): f at a node of grid row r (the last axis) is taken
// times row_scale[r] (island canvases: each island's h^2).
__global__ void __launch_bounds__(BLOCK) k_rhs(const int8_t* __restrict__ kind, const double* __restrict__ f,
                                               const eb_cut_t* __restrict__ cuts, int64_t ncuts,
                                               const double* __restrict__ u, double* __restrict__ b,
                                               int64_t nnodes, double s, GridDims d,
                                               const double* __restrict__ row_scale) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= nnodes) return;
    if (kind[n] != 2) {
        b[n] = 0.0;
        return;
    }
    double v = f[n];
    if (row_scale) {
        const NodePos p = node_pos(n, d);
        v = v * row_scale[d.dim == 3 ? p.k : p.j];
    }
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

// The side's contribution from its records: 0 + c of each record (node,
// side) in record order (one on a line-by-line side, two on an RBF side);
// records are sorted by node, a node's records by side.  *miss is set when
// there is none.
__device__ inline double cut_c_of(const eb_cut_t* __restrict__ cuts, int64_t n_cuts, int64_t node, int side,
                                  int* miss) {
    int64_t lo = 0, hi = n_cuts;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (cuts[mid].node < node) lo = mid + 1;
        else hi = mid;
    }
    double v = 0.0;
    bool any = false;
    for (int64_t m = lo; m < n_cuts && cuts[m].node == node; ++m) {
        if (cuts[m].dir == side) {
            v = v + cuts[m].c;
            any = true;
        }
    }
    if (!any) *miss = 1;
    return v;
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

static int assemble_diag_impl(const eb_grid_t* g, const double* psi, const double* beta, int32_t mode,
                              int8_t* kind, double* a, eb_cut_t* cuts, int64_t cuts_cap, int64_t* n_unknowns,
                              int64_t* n_cuts, void* stream) {
    clear_error();
    GridDims d;
    EB_TRY(make_dims(g, &d));
    if (!psi || !kind || !a || !n_unknowns || !n_cuts || cuts_cap < 0 || (cuts_cap > 0 && !cuts)) {
        set_error("eb_assemble_diag: null pointer or negative capacity");
        return EB_EINVAL;
    }
    if (mode != EB_BC_LINE && mode != EB_BC_MIXED && mode != EB_BC_RBF) {
        set_error("eb_assemble_diag_mode: unknown mode %d", (int)mode);
        return EB_EINVAL;
    }
    if (mode != EB_BC_LINE && d.dim != 2) {
        set_error("eb_assemble_diag_mode: RBF rows are defined for 2-D grids only");
        return EB_ENOTIMPL;
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
    hipLaunchKernelGGL(k_count_cuts, dim3(nblk), dim3(BLOCK), 0, s, kind, psi, d, nn, (int)mode, blk_cuts);
    EB_LAUNCH_CHECK();
    EB_TRY(scan_i32_to_i64_dev(blk_cuts, blk_off, nblk, &st->cuts, s));
    hipLaunchKernelGGL(k_diag_cuts, dim3(nblk), dim3(BLOCK), 0, s, psi, kind, beta, d, nn, (int)mode, blk_off, a,
                       cuts, cuts_cap, &st->err, &st->ndefer, defer);
    hipLaunchKernelGGL(k_diag_long, dim3(DIAG_LONG_BLOCKS), dim3(DIAG_LONG_NT), 0, s, psi, kind, beta, d, a,
                       cuts, cuts_cap, &st->err, &st->ndefer, defer);
    if (mode != EB_BC_LINE)
        hipLaunchKernelGGL(k_diag_rbf, dim3(nblk), dim3(BLOCK), 0, s, psi, kind, beta, d, nn, (int)mode, blk_off, a,
                           cuts, cuts_cap, &st->err);
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
    if (h.err & DEVERR_GEOM) {
        set_error("an RBF row's three interpolation points are collinear");
        return EB_EGEOM;
    }
    *n_unknowns = (int64_t)h.unknowns;
    *n_cuts = h.cuts;
    if (h.cuts > cuts_cap) {
        set_error("cut-record capacity %lld < required %lld", (long long)cuts_cap, (long long)h.cuts);
        return EB_ENOSPC;
    }
    return EB_OK;
}

extern "C" int eb_assemble_diag_mode(const eb_grid_t* g, const double* psi, int32_t mode, int8_t* kind,
                                     double* a, eb_cut_t* cuts, int64_t cuts_cap, int64_t* n_unknowns,
                                     int64_t* n_cuts, void* stream) {
    return assemble_diag_impl(g, psi, nullptr, mode, kind, a, cuts, cuts_cap, n_unknowns, n_cuts, stream);
}

extern "C" int eb_assemble_diag_beta(const eb_grid_t* g, const double* psi, const double* beta, int32_t mode,
                                     int8_t* kind, double* a, eb_cut_t* cuts, int64_t cuts_cap,
                                     int64_t* n_unknowns, int64_t* n_cuts, void* stream) {
    return assemble_diag_impl(g, psi, beta, mode, kind, a, cuts, cuts_cap, n_unknowns, n_cuts, stream);
}

extern "C" int eb_assemble_diag(const eb_grid_t* g, const double* psi, int8_t* kind, double* a,
                                eb_cut_t* cuts, int64_t cuts_cap, int64_t* n_unknowns,
                                int64_t* n_cuts, void* stream) {
    return assemble_diag_impl(g, psi, nullptr, EB_BC_LINE, kind, a, cuts, cuts_cap, n_unknowns, n_cuts, stream);
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
    hipLaunchKernelGGL(k_rhs, dim3(grid_for(nn)), dim3(BLOCK), 0, s, kind, f, cuts, n_cuts, u_at_cuts, b, nn, d.s, d,
                       (const double*)nullptr);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

extern "C" int eb_assemble_rhs_islands(const eb_grid_t* g, const int8_t* kind, const double* f,
                                       const eb_cut_t* cuts, int64_t n_cuts, const double* u_at_cuts,
                                       int32_t nseg, const int32_t* seg_rows, const double* seg_h, double* b,
                                       void* stream) {
    clear_error();
    GridDims d;
    EB_TRY(make_dims(g, &d));
    if (!kind || !f || !b || !seg_rows || !seg_h || nseg < 1 || n_cuts < 0 || (n_cuts > 0 && (!cuts || !u_at_cuts))) {
        set_error("eb_assemble_rhs_islands: null pointer or bad count");
        return EB_EINVAL;
    }
    const int nrows = d.dim == 3 ? d.nz : d.ny;
    if (seg_rows[0] != 0 || seg_rows[nseg] != nrows) {
        set_error("eb_assemble_rhs_islands: segments must cover the %d node rows", nrows);
        return EB_EINVAL;
    }
    std::vector<double> sc((size_t)nrows);
    for (int k = 0; k < nseg; ++k) {
        if (seg_rows[k + 1] < seg_rows[k] || !(seg_h[k] > 0.0)) {
            set_error("eb_assemble_rhs_islands: segment %d has decreasing rows or h <= 0", k);
            return EB_EINVAL;
        }
        const double h2 = seg_h[k] * seg_h[k];
        for (int r = seg_rows[k]; r < seg_rows[k + 1]; ++r) sc[(size_t)r] = h2;
    }
    hipStream_t s = (hipStream_t)stream;
    double* dsc = nullptr;
    EB_TRY(dalloc_n(&dsc, nrows, s));
    EB_HIP(hipMemcpyAsync(dsc, sc.data(), sizeof(double) * (size_t)nrows, hipMemcpyHostToDevice, s));
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    hipLaunchKernelGGL(k_rhs, dim3(grid_for(nn)), dim3(BLOCK), 0, s, kind, f, cuts, n_cuts, u_at_cuts, b, nn, d.s, d,
                       (const double*)dsc);
    EB_LAUNCH_CHECK();
    // the copy above reads pageable host memory: wait for it before sc goes away
    EB_HIP(hipStreamSynchronize(s));
    EB_TRY(dfree(dsc, s));
    return EB_OK;
}

static int stencil_apply_impl(const eb_grid_t* g, const int8_t* kind, const double* a, const double* beta,
                              double sigma, const double* x, double* y, void* stream) {
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
    if (x == y) {
        set_error("stencil_apply: y must not overlap x");
        return EB_EINVAL;
    }
    FieldCoefs co;
    co.sigma = sigma;
    return launch_field_op(0, d, kind, a, beta, x, nullptr, nullptr, nullptr, y, co, (hipStream_t)stream);
}

extern "C" int stencil_apply(const eb_grid_t* g, const int8_t* kind, const double* a, double sigma,
                             const double* x, double* y, void* stream) {
    return stencil_apply_impl(g, kind, a, nullptr, sigma, x, y, stream);
}

extern "C" int stencil_apply_beta(const eb_grid_t* g, const int8_t* kind, const double* a, const double* beta,
                                  double sigma, const double* x, double* y, void* stream) {
    if (!beta) {
        set_error("stencil_apply_beta: null beta");
        return EB_EINVAL;
    }
    return stencil_apply_impl(g, kind, a, beta, sigma, x, y, stream);
}
