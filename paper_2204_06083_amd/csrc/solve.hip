// Solve phase: PCG (Algorithm 2 step 4) preconditioned by one V(1,1) cycle
// of the aggregation hierarchy.
//
// Fine level: row-padded node fields (pitch px, a multiple of 64 doubles) and
// a list of active strips (runs of strip_w consecutive x-nodes holding at
// least one unknown), so sweeps touch only the domain.  The operator is
// matrix-free: (A v)_p = d_p v_p - (1/h^2) sum of v over the 2d neighbours,
// with every vector zero off unknowns, so boundary-point neighbours drop out.
// The fine prolongator P = (I - omega D^-1 A) P_tent and its transpose are
// applied matrix-free from the aggregate map.  Coarse levels use CSR; the
// coarsest applies its dense inverse.
//
// Reductions: every reducing fine kernel runs a fixed grid of `nparts` blocks
// (grid-stride over the strips) and writes one partial per block.  The kernel
// that needs the scalar sums those partials itself, in a fixed order, in every
// block, so all blocks agree bit for bit and no cross-block synchronisation,
// fence or atomic is needed.  PCG scalars (alpha, beta, convergence) are thus
// formed on the device; block 0 records them for the host, which polls the
// `done` flag every few iterations.  Once `done` is set, every queued kernel
// returns at once.
#include <math.h>
#include <string.h>

#include <hip/hip_ext.h>

#include <atomic>

#include <type_traits>

#include "handle.hpp"

namespace eb {

constexpr int NT = 512;        // threads per block of the solve kernels
// The fixed-grid reducing kernels ask for 8 waves per SIMD (<= 64 VGPRs) so
// that their whole grid is resident at once.
constexpr int RNT = 256;       // threads per block of the box-per-thread restriction
constexpr int MAX_PARTS = 1024;       // partials of the strip kernels' fixed grid
constexpr int MAX_TILE_PARTS = 2048;  // blocks of the 2-D tile kernels (one partial each)
constexpr int PART_CAP = MAX_TILE_PARTS;

struct FineArgs {
    const int32_t* strips;
    int64_t nstrips;
    int64_t spb;          // strips per block (contiguous range per block)
    int strip_w;
    int64_t sy, sz;       // padded strides
    int dim;
    double s;             // 1/h^2
    const double* diag;   // padded, 0 off unknowns
    const float* diag32;  // the same in FP32 (single-precision V-cycle only)
    const double* wf;     // per-point smoother weights omega_k / d_k (learned weights; 0 off unknowns)
    const float* wf32;
    const void* dinv16;   // BF16 1 / diag (BF16 smoother only)
    const double* bf[3];  // variable beta: beta of the +axis face of each node (padded), else null
};

// BF16 storage of the fine smoother's operands (precision EB_PREC_BF16): the
// top 16 bits of an FP32 value, rounded to nearest with ties to even;
// arithmetic stays FP32.
struct bf16 {
    uint16_t u;
};
__device__ inline float bf16_to_f32(bf16 v) { return __uint_as_float((uint32_t)v.u << 16); }
__device__ inline bf16 f32_to_bf16(float f) {
    uint32_t x = __float_as_uint(f);
    if ((x & 0x7f800000u) == 0x7f800000u)              // Inf stays Inf, NaN stays NaN
        return bf16{(uint16_t)((x >> 16) | ((x & 0xffffu) ? 0x40u : 0u))};
    x += 0x7fffu + ((x >> 16) & 1u);
    return bf16{(uint16_t)(x >> 16)};
}
__device__ inline double to_f64(double v) { return v; }
__device__ inline double to_f64(float v) { return (double)v; }
__device__ inline double to_f64(bf16 v) { return (double)bf16_to_f32(v); }

// Diagonal in the precision of the V-cycle.
template <class V> __device__ inline const V* vdiag(const FineArgs& f);
template <> __device__ inline const double* vdiag<double>(const FineArgs& f) { return f.diag; }
template <> __device__ inline const float* vdiag<float>(const FineArgs& f) { return f.diag32; }
template <class V> __device__ inline const V* vwf(const FineArgs& f);
template <> __device__ inline const double* vwf<double>(const FineArgs& f) { return f.wf; }
template <> __device__ inline const float* vwf<float>(const FineArgs& f) { return f.wf32; }

// Each block sweeps its own contiguous range of strips, NT / strip_w strips
// at a time; p is the padded node index of this thread's node.
#define FINE_LOOP(f, p)                                                                          \
    for (int64_t s0_ = xcd_block() * (f).spb, s1_ = min(s0_ + (f).spb, (f).nstrips),              \
                 sidx_ = s0_ + threadIdx.x / (f).strip_w;                                          \
         sidx_ < s1_; sidx_ += NT / (f).strip_w)                                                   \
        for (int64_t p = (int64_t)(f).strips[sidx_] * (f).strip_w + threadIdx.x % (f).strip_w,     \
                     once_ = 0;                                                                    \
             once_ < 1; ++once_)

template <class V>
__device__ inline V nbr_sum(const V* __restrict__ v, int64_t p, const FineArgs& f) {
    V t = v[p - 1] + v[p + 1];
    t += v[p - f.sy] + v[p + f.sy];
    if (f.dim == 3) t += v[p - f.sz] + v[p + f.sz];
    return t;
}

template <class V>
__device__ inline V safe_div(V x, V d) { return d != V(0) ? x / d : V(0); }

// sum over neighbours of v / d (zero where d == 0, i.e. off unknowns)
template <class V>
__device__ inline V nbr_sum_scaled(const V* __restrict__ v, const V* __restrict__ dg, int64_t p, const FineArgs& f) {
    V t = safe_div(v[p - 1], dg[p - 1]) + safe_div(v[p + 1], dg[p + 1]);
    t += safe_div(v[p - f.sy], dg[p - f.sy]) + safe_div(v[p + f.sy], dg[p + f.sy]);
    if (f.dim == 3) t += safe_div(v[p - f.sz], dg[p - f.sz]) + safe_div(v[p + f.sz], dg[p + f.sz]);
    return t;
}

// Variable conductivity (VB): the same sums with each neighbour weighted by
// the beta of the face toward it (bf[a][p] is the face between p and p + e_a).
template <class V>
__device__ inline V nbr_sum_b(const V* __restrict__ v, int64_t p, const FineArgs& f) {
    V t = (V)f.bf[0][p - 1] * v[p - 1] + (V)f.bf[0][p] * v[p + 1];
    t += (V)f.bf[1][p - f.sy] * v[p - f.sy] + (V)f.bf[1][p] * v[p + f.sy];
    if (f.dim == 3) t += (V)f.bf[2][p - f.sz] * v[p - f.sz] + (V)f.bf[2][p] * v[p + f.sz];
    return t;
}

template <class V>
__device__ inline V nbr_sum_scaled_b(const V* __restrict__ v, const V* __restrict__ dg, int64_t p,
                                     const FineArgs& f) {
    V t = (V)f.bf[0][p - 1] * safe_div(v[p - 1], dg[p - 1]) + (V)f.bf[0][p] * safe_div(v[p + 1], dg[p + 1]);
    t += (V)f.bf[1][p - f.sy] * safe_div(v[p - f.sy], dg[p - f.sy]) + (V)f.bf[1][p] * safe_div(v[p + f.sy], dg[p + f.sy]);
    if (f.dim == 3)
        t += (V)f.bf[2][p - f.sz] * safe_div(v[p - f.sz], dg[p - f.sz]) +
             (V)f.bf[2][p] * safe_div(v[p + f.sz], dg[p + f.sz]);
    return t;
}

template <bool VB, class V>
__device__ inline V nsum(const V* __restrict__ v, int64_t p, const FineArgs& f) {
    if constexpr (VB) return nbr_sum_b(v, p, f);
    else return nbr_sum(v, p, f);
}

template <bool VB, class V>
__device__ inline V nsum_scaled(const V* __restrict__ v, const V* __restrict__ dg, int64_t p, const FineArgs& f) {
    if constexpr (VB) return nbr_sum_scaled_b(v, dg, p, f);
    else return nbr_sum_scaled(v, dg, p, f);
}

// beta of the face on side (axis, +/-) of node p (1 without VB)
template <bool VB>
__device__ inline double fbeta(const FineArgs& f, int axis, int64_t p, int64_t st, bool plus) {
    if constexpr (VB) return plus ? f.bf[axis][p] : f.bf[axis][p - st];
    else return 1.0;
}

// ------------------------------------------------------------ reductions
// BS is the block size of the calling kernel.
template <int BS = NT>
__device__ inline void block_partial(double v, double* __restrict__ part) {
    __shared__ double lds[BS / WAVE];
    const double s = block_sum<BS>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Sum of np partials in a fixed order; every thread of the block gets it.
// Thread t adds part[t], part[t + BS], ... in that order; the loads of a
// round of TOT_U of them are issued together (one memory latency per round,
// not per partial), without a branch (an index past np reads part[0] and is
// not added), so they also go out together with reads issued before them.
constexpr int TOT_U = 4;

template <int BS>
__device__ inline double thread_partials(const double* __restrict__ part, int np) {
    double a = 0.0;
    for (int i0 = 0; i0 < np; i0 += BS * TOT_U) {
        double v[TOT_U];
#pragma unroll
        for (int u = 0; u < TOT_U; ++u) {
            const int i = i0 + u * BS + (int)threadIdx.x;
            v[u] = part[i < np ? i : 0];
        }
#pragma unroll
        for (int u = 0; u < TOT_U; ++u) {
            const double t = a + v[u];
            a = i0 + u * BS + (int)threadIdx.x < np ? t : a;
        }
    }
    return a;
}

// The same for two arrays of np partials, their reads issued together.
template <int BS>
__device__ inline void thread_partials2(const double* __restrict__ pa, const double* __restrict__ pb, int np,
                                        double* a, double* b) {
    double sa = 0.0, sb = 0.0;
    for (int i0 = 0; i0 < np; i0 += BS * TOT_U) {
        double va[TOT_U], vb[TOT_U];
#pragma unroll
        for (int u = 0; u < TOT_U; ++u) {
            const int i = i0 + u * BS + (int)threadIdx.x;
            va[u] = pa[i < np ? i : 0];
            vb[u] = pb[i < np ? i : 0];
        }
#pragma unroll
        for (int u = 0; u < TOT_U; ++u) {
            const bool in = i0 + u * BS + (int)threadIdx.x < np;
            const double ta = sa + va[u], tb = sb + vb[u];
            sa = in ? ta : sa;
            sb = in ? tb : sb;
        }
    }
    *a = sa;
    *b = sb;
}

// The block's total: wavefront sums, then every thread adds the wavefront
// sums in wavefront order (the same value in every thread, one barrier
// before and one after).
template <int BS = NT>
__device__ inline double block_total(const double* __restrict__ part, int np) {
    __shared__ double lds[BS / WAVE];
    const double a = wave_sum(thread_partials<BS>(part, np));
    if ((threadIdx.x & (WAVE - 1)) == 0) lds[threadIdx.x / WAVE] = a;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < BS / WAVE; ++i) r += lds[i];
    __syncthreads();
    return r;
}

// Two totals at once (same order as two block_total calls, one pass of loads
// and barriers).
template <int BS = NT>
__device__ inline void block_total2(const double* __restrict__ pa, const double* __restrict__ pb, int np,
                                    double* ta, double* tb) {
    __shared__ double lds[2][BS / WAVE];
    double a, b;
    thread_partials2<BS>(pa, pb, np, &a, &b);
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        lds[0][w] = a;
        lds[1][w] = b;
    }
    __syncthreads();
    double x = 0.0, y = 0.0;
#pragma unroll
    for (int i = 0; i < BS / WAVE; ++i) {
        x += lds[0][i];
        y += lds[1][i];
    }
    __syncthreads();
    *ta = x;
    *tb = y;
}

__device__ inline bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }

__device__ inline bool bad_value(double v) { return isnan(v) || isinf(v); }

// ------------------------------------------------------------ PCG kernels
// V is the storage type of the preconditioned residual z (the V-cycle's
// precision); the CG vectors and scalars are always FP64.
//
// p_new = z + beta p_old; q = A p_new; partial (p_new, q).
// rho = (r, z) of the latest V-cycle, beta = rho / rho_prev (0 on the first).
template <class V, bool VB = false>
__global__ void __launch_bounds__(NT, 8) k_pcg_p_spmv(FineArgs f, const V* __restrict__ z,
                                                   const double* __restrict__ pold, double* __restrict__ pnew,
                                                   double* __restrict__ q, const double* __restrict__ rz_cur,
                                                   const double* __restrict__ rz_prev, int np,
                                                   double* __restrict__ part_pq, PcgScalars* sc) {
    const int32_t done = sc->done;   // read with the partials; nothing is stored once done
    double rho, rho_prev = 0.0;
    if (rz_prev) block_total2(rz_cur, rz_prev, np, &rho, &rho_prev);
    else rho = block_total(rz_cur, np);
    if (done) return;
    const double beta = rz_prev ? rho / rho_prev : 0.0;
    if (!(rho > 0.0) || bad_value(rho) || bad_value(beta)) {
        if (lead()) {
            sc->status = (bad_value(rho) || bad_value(beta)) ? EB_ENAN : EB_ENOTSPD;
            sc->done = 1;
        }
        return;
    }
    double part = 0.0;
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double pc = to_f64(z[p]) + beta * pold[p];
            double nb;
            if constexpr (VB) {
                nb = f.bf[0][p - 1] * (to_f64(z[p - 1]) + beta * pold[p - 1]);
                nb += f.bf[0][p] * (to_f64(z[p + 1]) + beta * pold[p + 1]);
                nb += f.bf[1][p - f.sy] * (to_f64(z[p - f.sy]) + beta * pold[p - f.sy]);
                nb += f.bf[1][p] * (to_f64(z[p + f.sy]) + beta * pold[p + f.sy]);
                if (f.dim == 3) {
                    nb += f.bf[2][p - f.sz] * (to_f64(z[p - f.sz]) + beta * pold[p - f.sz]);
                    nb += f.bf[2][p] * (to_f64(z[p + f.sz]) + beta * pold[p + f.sz]);
                }
            } else {
                nb = to_f64(z[p - 1]) + beta * pold[p - 1];
                nb += to_f64(z[p + 1]) + beta * pold[p + 1];
                nb += to_f64(z[p - f.sy]) + beta * pold[p - f.sy];
                nb += to_f64(z[p + f.sy]) + beta * pold[p + f.sy];
                if (f.dim == 3) {
                    nb += to_f64(z[p - f.sz]) + beta * pold[p - f.sz];
                    nb += to_f64(z[p + f.sz]) + beta * pold[p + f.sz];
                }
            }
            const double qv = d * pc - f.s * nb;
            pnew[p] = pc;
            q[p] = qv;
            part += pc * qv;
        }
    }
    block_partial(part, part_pq);
}

// alpha = rho / (p, q); x += alpha p; r -= alpha q; partial ||r||^2.
__global__ void __launch_bounds__(NT) k_pcg_xr(FineArgs f, double* __restrict__ x, double* __restrict__ r,
                                               const double* __restrict__ pv, const double* __restrict__ q,
                                               const double* __restrict__ rz_cur, const double* __restrict__ part_pq,
                                               int np, double* __restrict__ part_rr, PcgScalars* sc) {
    if (sc->done) return;
    double rho, pq;
    block_total2(rz_cur, part_pq, np, &rho, &pq);
    if (!(pq > 0.0) || bad_value(pq)) {
        if (lead()) {
            sc->status = bad_value(pq) ? EB_ENAN : EB_ENOTSPD;
            sc->done = 1;
        }
        return;
    }
    const double alpha = rho / pq;
    if (lead()) {
        sc->iters = sc->iters + 1;   // counted on the device: a captured iteration carries no number
        sc->pq = pq;
    }
    double part = 0.0;
    FINE_LOOP(f, p) {
        if (f.diag[p] != 0.0) {
            x[p] = x[p] + alpha * pv[p];
            const double rv = r[p] - alpha * q[p];
            r[p] = rv;
            part += rv * rv;
        }
    }
    block_partial(part, part_rr);
}

// Convergence test on a total ||r||^2 already formed; true if the caller
// must return.
__device__ inline bool converged_or_failed_total(double rr, PcgScalars* sc) {
    if (bad_value(rr)) {
        if (lead()) {
            sc->status = EB_ENAN;
            sc->done = 1;
        }
        return true;
    }
    if (lead()) sc->rr = rr;
    if (rr <= sc->tol2bb) {
        if (lead()) sc->done = 1;
        return true;
    }
    return false;
}

// Convergence test on ||r||^2 (partials of the previous kernel); true if the
// caller must return.  BS is the caller's block size.
template <int BS = NT>
__device__ inline bool converged_or_failed(const double* __restrict__ part_rr, int np, PcgScalars* sc) {
    const double rr = block_total<BS>(part_rr, np);
    return converged_or_failed_total(rr, sc);
}

// ------------------------------------------------------------ fine V-cycle
// Pre-smoothing and residual: z1 = omega r / d (not stored), res = r - A z1,
// formed from the FP64 residual and stored in the V-cycle precision.
// With `check`, first test convergence of the iterate that produced r.
// LW: the smoother uses the per-point weights f.wf (z1 = wf r) instead of
// omega / d; the prolongator always keeps omega.
template <class V, bool LW, bool VB = false>
__global__ void __launch_bounds__(NT) k_fine_down(FineArgs f, double omega, const double* __restrict__ r,
                                                  V* __restrict__ res, PcgScalars* sc, int check,
                                                  const double* __restrict__ part_rr, int np) {
    const int32_t done = sc->done;   // read with the partials; nothing is stored once done
    if (check) {
        const double rr = block_total(part_rr, np);
        if (done || converged_or_failed_total(rr, sc)) return;
    } else if (done) {
        return;
    }
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            if (LW) {
                const double z1 = f.wf[p] * r[p];
                double nb = f.wf[p - 1] * r[p - 1] + f.wf[p + 1] * r[p + 1];
                nb += f.wf[p - f.sy] * r[p - f.sy] + f.wf[p + f.sy] * r[p + f.sy];
                if (f.dim == 3) nb += f.wf[p - f.sz] * r[p - f.sz] + f.wf[p + f.sz] * r[p + f.sz];
                res[p] = (V)(r[p] - (d * z1 - f.s * nb));
            } else {
                const double z1 = omega * r[p] / d;
                const double nb = omega * nsum_scaled<VB>(r, f.diag, p, f);
                res[p] = (V)(r[p] - (d * z1 - f.s * nb));
            }
        }
    }
}

// Restriction r_c = P^T res = P_tent^T (I - omega A D^-1) res over the
// level-0 boxes (2-D: one thread per box; 3-D: restrict_box3); the box's
// coarse unknowns are consecutive from box_cstart.
constexpr int MAX_FINE_COMP = 16;

struct BoxArgs {
    const int32_t* boxes;
    int64_t nboxes;
    int nbx, nby;
    int nx, ny, nz;       // node extents
    const int32_t* cstart;
    const int32_t* ncomp;
    const int32_t* agg;   // padded
    const int32_t* map;   // 2-D: per box, the aggregate of node n (0..8) minus cstart in bits 3n..3n+2 (7: none)
    const double* w0;     // 2-D: per box, omega_1 / d_1 of its first aggregate (0 without aggregates)
    const float* w0_32;
};

template <class V> __device__ inline const V* vbw0(const BoxArgs& b);
template <> __device__ inline const double* vbw0<double>(const BoxArgs& b) { return b.w0; }
template <> __device__ inline const float* vbw0<float>(const BoxArgs& b) { return b.w0_32; }

// 3-D restriction: 9 threads per level-0 box, each the smoothed residual
// u = (I - omega A D^-1) res of a 3-node x-run (one (oy, oz) row of the box),
// staged in LDS; then each aggregate's sum over the box in node order
// (oz, oy, ox), one thread per aggregate.
constexpr int R3_BOXES = RNT / 9;   // boxes per block

template <class V, bool VB = false>
__device__ inline void restrict_box3(const FineArgs& f, const BoxArgs& b, const V* __restrict__ dg, V omega, V sh,
                                     const V* __restrict__ res, V* __restrict__ rc, const V* __restrict__ dg_c,
                                     double omega_c, V* __restrict__ sv_c) {
    __shared__ V us[R3_BOXES][27];
    __shared__ int8_t cs[R3_BOXES][27];
    const int lb = threadIdx.x / 9, q = threadIdx.x % 9;
    const int64_t t = xcd_block() * R3_BOXES + lb;
    const bool active = lb < R3_BOXES && t < b.nboxes;
    int32_t c0 = 0;
    int m = 0;
    if (active) {
        const int64_t box = b.boxes[t];
        const int bx = (int)(box % b.nbx);
        const int64_t rr = box / b.nbx;
        const int by = (int)(rr % b.nby);
        const int bz = (int)(rr / b.nby);
        c0 = b.cstart[box];
        m = b.ncomp[box];
        const int oy = q % 3, oz = q / 3;
        const int j = 3 * by + oy, k = 3 * bz + oz;
#pragma unroll
        for (int ox = 0; ox < 3; ++ox) {
            const int i = 3 * bx + ox;
            V u = V(0);
            int c = -1;
            if (i < b.nx && j < b.ny && k < b.nz) {
                const int64_t p = (int64_t)i + f.sy * j + f.sz * k;
                const V d = dg[p];
                if (d != V(0)) {
                    const V rp = res[p];
                    const V aw = d * (rp / d) - sh * nsum_scaled<VB>(res, dg, p, f);
                    u = rp - omega * aw;
                    c = m == 1 ? 0 : b.agg[p] - c0;
                }
            }
            us[lb][9 * oz + 3 * oy + ox] = u;
            cs[lb][9 * oz + 3 * oy + ox] = (int8_t)(c >= 0 && c < MAX_FINE_COMP ? c : -1);
        }
    }
    __syncthreads();
    if (!active) return;
    for (int c = q; c < m && c < MAX_FINE_COMP; c += 9) {
        V acc = V(0);
        for (int n = 0; n < 27; ++n)
            if (cs[lb][n] == c) acc += us[lb][n];
        rc[c0 + c] = acc;
        if (sv_c) sv_c[c0 + c] = (V)omega_c * acc / dg_c[c0 + c];
    }
}

template <class V, int DIM, bool VB = false>
__global__ void __launch_bounds__(RNT) k_fine_restrict(FineArgs f, BoxArgs b, double omega_d,
                                                      const V* __restrict__ res, V* __restrict__ rc,
                                                      const V* __restrict__ dg_c, double omega_c,
                                                      V* __restrict__ sv_c, PcgScalars* sc, int check,
                                                      const double* __restrict__ part_rr, int np) {
    const int32_t done = sc->done;   // read with the partials; nothing is stored once done
    if (check) {
        const double rr = block_total<RNT>(part_rr, np);
        if (done || converged_or_failed_total(rr, sc)) return;
    } else if (done) {
        return;
    }
    const V* __restrict__ dg = vdiag<V>(f);
    const V omega = (V)omega_d;
    const V sh = (V)f.s;
    if (DIM == 3) {
        restrict_box3<V, VB>(f, b, dg, omega, sh, res, rc, dg_c, omega_c, sv_c);
        return;
    }
    const int64_t t = xcd_block() * RNT + threadIdx.x;
    if (t >= b.nboxes) return;
    const int64_t box = b.boxes[t];
    const int bx = (int)(box % b.nbx);
    const int64_t rr = box / b.nbx;
    const int by = (int)(rr % b.nby);
    const int bz = (int)(rr / b.nby);
    const int32_t c0 = b.cstart[box];
    const int m = b.ncomp[box];
    if (DIM == 2) {
        // The box's 3 x 3 nodes and their neighbours (a 5 x 5 window without
        // its corners) are loaded first; window points off the node grid read
        // as 0 (they neighbour no unknown: the outer node layer is outside).
        // Each node's contribution goes to its component; the components'
        // sums are then formed in node order.
        V rw[5][5], dw[5][5];
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                rw[a][c] = V(0);
                dw[a][c] = V(0);
                if ((a == 0 || a == 4) && (c == 0 || c == 4)) continue;
                const int i = 3 * bx - 1 + c, j = 3 * by - 1 + a;
                if (i < 0 || i >= b.nx || j < 0 || j >= b.ny) continue;
                const int64_t p = (int64_t)i + f.sy * j;
                dw[a][c] = dg[p];
                rw[a][c] = res[p];
            }
        V u[9];
        int comp[9];
#pragma unroll
        for (int oy = 0; oy < 3; ++oy)
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                const int a = oy + 1, c = ox + 1, n = 3 * oy + ox;
                const V d = dw[a][c];
                u[n] = V(0);
                comp[n] = -1;
                if (d == V(0)) continue;
                const V rp = rw[a][c];
                V nb;
                if constexpr (VB) {
                    nb = nbr_sum_scaled_b(res, dg, (int64_t)(3 * bx + ox) + f.sy * (3 * by + oy), f);
                } else {
                    nb = safe_div(rw[a][c - 1], dw[a][c - 1]) + safe_div(rw[a][c + 1], dw[a][c + 1]);
                    nb += safe_div(rw[a - 1][c], dw[a - 1][c]) + safe_div(rw[a + 1][c], dw[a + 1][c]);
                }
                const V aw = d * (rp / d) - sh * nb;
                u[n] = rp - omega * aw;
                comp[n] = m == 1 ? 0 : b.agg[(int64_t)(3 * bx + ox) + f.sy * (3 * by + oy)] - c0;
            }
        for (int c = 0; c < m && c < MAX_FINE_COMP; ++c) {
            V acc = V(0);
#pragma unroll
            for (int n = 0; n < 9; ++n)
                if (comp[n] == c) acc += u[n];
            rc[c0 + c] = acc;
            if (sv_c) sv_c[c0 + c] = (V)omega_c * acc / dg_c[c0 + c];
        }
    }
}

// PCG update fused with the fine pre-smoothing and residual:
//   alpha = rho / (p, q); x += alpha p; r_out = r_in - alpha q;
//   res = r_out - A (omega D^-1 r_out), with r_out at the neighbours recomputed
//   from r_in and q (r_in and r_out are different buffers).
// The CG part is FP64; res is stored in the V-cycle precision.
// The convergence test on ||r_out||^2 happens in the next kernel.
template <class V, bool LW, bool VB = false>
__global__ void __launch_bounds__(NT, 8) k_pcg_xr_down(FineArgs f, double* __restrict__ x, const double* __restrict__ rin,
                                                    double* __restrict__ rout, const double* __restrict__ pv,
                                                    const double* __restrict__ q, V* __restrict__ res,
                                                    double omega, const double* __restrict__ rz_cur,
                                                    const double* __restrict__ part_pq, int np,
                                                    double* __restrict__ part_rr, PcgScalars* sc) {
    const int32_t done = sc->done;   // read with the partials; nothing is stored once done
    double rho, pq;
    block_total2(rz_cur, part_pq, np, &rho, &pq);
    if (done) return;
    if (!(pq > 0.0) || bad_value(pq)) {
        if (lead()) {
            sc->status = bad_value(pq) ? EB_ENAN : EB_ENOTSPD;
            sc->done = 1;
        }
        return;
    }
    const double alpha = rho / pq;
    if (lead()) {
        sc->iters = sc->iters + 1;   // counted on the device: a captured iteration carries no number
        sc->pq = pq;
    }
    double part = 0.0;
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            x[p] = x[p] + alpha * pv[p];
            const double rn = rin[p] - alpha * q[p];
            rout[p] = rn;
            part += rn * rn;
            if (LW) {
                double nb = f.wf[p - 1] * (rin[p - 1] - alpha * q[p - 1]);
                nb += f.wf[p + 1] * (rin[p + 1] - alpha * q[p + 1]);
                nb += f.wf[p - f.sy] * (rin[p - f.sy] - alpha * q[p - f.sy]);
                nb += f.wf[p + f.sy] * (rin[p + f.sy] - alpha * q[p + f.sy]);
                if (f.dim == 3) {
                    nb += f.wf[p - f.sz] * (rin[p - f.sz] - alpha * q[p - f.sz]);
                    nb += f.wf[p + f.sz] * (rin[p + f.sz] - alpha * q[p + f.sz]);
                }
                const double z1 = f.wf[p] * rn;
                res[p] = (V)(rn - (d * z1 - f.s * nb));
            } else {
                double nb = fbeta<VB>(f, 0, p, 1, false) * safe_div(rin[p - 1] - alpha * q[p - 1], f.diag[p - 1]);
                nb += fbeta<VB>(f, 0, p, 1, true) * safe_div(rin[p + 1] - alpha * q[p + 1], f.diag[p + 1]);
                nb += fbeta<VB>(f, 1, p, f.sy, false) * safe_div(rin[p - f.sy] - alpha * q[p - f.sy], f.diag[p - f.sy]);
                nb += fbeta<VB>(f, 1, p, f.sy, true) * safe_div(rin[p + f.sy] - alpha * q[p + f.sy], f.diag[p + f.sy]);
                if (f.dim == 3) {
                    nb += fbeta<VB>(f, 2, p, f.sz, false) *
                          safe_div(rin[p - f.sz] - alpha * q[p - f.sz], f.diag[p - f.sz]);
                    nb += fbeta<VB>(f, 2, p, f.sz, true) *
                          safe_div(rin[p + f.sz] - alpha * q[p + f.sz], f.diag[p + f.sz]);
                }
                const double z1 = omega * rn / d;
                res[p] = (V)(rn - (d * z1 - f.s * (omega * nb)));
            }
        }
    }
    block_partial(part, part_rr);
}

// Coarse-grid correction value t = e_c[agg] at node p (0 off unknowns).
template <class V>
__device__ inline V corr_at(const int32_t* __restrict__ agg, const V* __restrict__ ec, int64_t p) {
    const int32_t g = agg[p];
    return g >= 0 ? ec[g] : V(0);
}

// Pre-smoothed iterate after prolongation at node p:
//   zt = omega r / d + t - omega (A t) / d,  t = e_c[agg].
template <class V, bool LW, bool VB = false>
__device__ inline V zt_at(const FineArgs& f, V omega, const int32_t* __restrict__ agg, const V* __restrict__ ec,
                          const double* __restrict__ r, int64_t p) {
    const V d = vdiag<V>(f)[p];
    if (d == V(0)) return V(0);
    const V tp = corr_at(agg, ec, p);
    V nb;
    if constexpr (VB) {
        nb = (V)f.bf[0][p - 1] * corr_at(agg, ec, p - 1) + (V)f.bf[0][p] * corr_at(agg, ec, p + 1);
        nb += (V)f.bf[1][p - f.sy] * corr_at(agg, ec, p - f.sy) + (V)f.bf[1][p] * corr_at(agg, ec, p + f.sy);
        if (f.dim == 3)
            nb += (V)f.bf[2][p - f.sz] * corr_at(agg, ec, p - f.sz) + (V)f.bf[2][p] * corr_at(agg, ec, p + f.sz);
    } else {
        nb = corr_at(agg, ec, p - 1) + corr_at(agg, ec, p + 1);
        nb += corr_at(agg, ec, p - f.sy) + corr_at(agg, ec, p + f.sy);
        if (f.dim == 3) nb += corr_at(agg, ec, p - f.sz) + corr_at(agg, ec, p + f.sz);
    }
    const V at = d * tp - (V)f.s * nb;
    const V z1 = LW ? vwf<V>(f)[p] * (V)r[p] : omega * (V)r[p] / d;
    return z1 + (tp - omega * at / d);
}

// Prolongation and pre-smoothed correction: zt = omega r / d + t - omega (A t) / d,
// t = e_c[agg].
template <class V, bool LW, bool VB = false>
__global__ void __launch_bounds__(NT) k_fine_up(FineArgs f, double omega, const int32_t* __restrict__ agg,
                                                const V* __restrict__ ec, const double* __restrict__ r,
                                                V* __restrict__ zt, const PcgScalars* sc) {
    if (sc->done) return;
    const V w = (V)omega;
    FINE_LOOP(f, p) {
        if (f.diag[p] != 0.0) zt[p] = zt_at<V, LW, VB>(f, w, agg, ec, r, p);
    }
}

// Post-smoothing: z = zt + omega (r - A zt) / d; partial (r, z) in FP64.
// B16 (BF16 smoother): scaled by the BF16 1 / d and z stored in BF16 (the
// partial uses the stored value).
template <class V, bool LW, bool B16 = false, bool VB = false>
__global__ void __launch_bounds__(NT, 8) k_fine_post(FineArgs f, double omega, const V* __restrict__ zt,
                                                  const double* __restrict__ r,
                                                  std::conditional_t<B16, bf16, V>* __restrict__ z,
                                                  double* __restrict__ part_rz, const PcgScalars* sc) {
    if (sc->done) return;
    const V* __restrict__ dg = vdiag<V>(f);
    const bf16* __restrict__ di16 = (const bf16*)f.dinv16;
    const V w = (V)omega;
    const V sh = (V)f.s;
    double part = 0.0;
    FINE_LOOP(f, p) {
        const V d = dg[p];
        if (d != V(0)) {
            const V az = d * zt[p] - sh * nsum<VB>(zt, p, f);
            if constexpr (B16) {
                const V zv = zt[p] + w * ((V)r[p] - az) * (V)bf16_to_f32(di16[p]);
                const bf16 zb = f32_to_bf16((float)zv);
                z[p] = zb;
                part += r[p] * to_f64(zb);
            } else {
                const V zv = LW ? zt[p] + vwf<V>(f)[p] * ((V)r[p] - az) : zt[p] + w * ((V)r[p] - az) / d;
                z[p] = zv;
                part += r[p] * (double)zv;
            }
        }
    }
    block_partial(part, part_rz);
}

// ------------------------------------------------- 2-D fine band tiles
// In 2-D the fine level of an iteration runs as three kernels:
//   k_t2_pspmv:        p = z + beta p_old; q = A p; (p, q)
//   k_t2_xr_restrict:  x += alpha p; r = r - alpha q; ||r||^2; the
//                      pre-smoothing residual res = r - A z1 (z1 = omega r/d)
//                      and the restriction P^T res, summed per box
//   k_t2_up_post:      t = e_c[agg]; zt = z1 + (I - omega D^-1 A) t;
//                      z = zt + omega D^-1 (r - A zt); (r, z)
// The residual res and the prolongated iterate zt never leave registers, so
// per unknown and iteration the fine level moves 40 + 56 + 28 bytes (plus the
// coarse vector) instead of the 184 of the strip kernels.
//
// Work is cut into band tiles of TX = 60 columns x TY rows (origins multiples
// of 3, so a tile holds whole level-0 boxes), one wavefront per tile: lane l
// owns column x0 - 2 + l (lanes 0, 1, 62, 63 are the two-column halo), and the
// wavefront marches down the rows of the tile and of its halo, keeping the
// last few rows of every quantity in registers.  The left and right
// neighbours of a value come from the adjacent lanes by a whole-wave DPP
// shift, the rows above and below from the registers, so there is no LDS and
// no barrier; the reads of the next two rows are issued before the current
// row is computed.  Fields are zero off unknowns, so no read waits for the
// diagonal.  The smoother and prolongator scale by omega / d through the
// stored 1 / d, with no division.
constexpr int TX = 60, TY = 12;   // band tile: 20 x 4 level-0 boxes
constexpr int TWB = 4;            // wavefronts (tiles) per block
// rows each wavefront has in flight while it marches down its tile (on the
// star 2048^2 solve: 2 rows 2.035 ms, 3 rows 2.023 ms, 4 rows 2.029 ms)
constexpr int T2_AHEAD = 3;
constexpr int TNT = TWB * WAVE;   // threads per block

struct TileArgs {
    const int32_t* tiles;   // active tiles (ty * ntx + tx), row-major order
    int64_t ntiles;
    int tpw;                // tiles per wavefront (a contiguous range per wavefront)
    int ntx;                // tiles per row of the tile grid
    int nx, ny;             // node extents
    int sy;                 // padded row pitch (padded node fields stay below 2^31 entries)
    double s;               // 1/h^2
    const double* diag;     // padded, 0 off unknowns
    const float* diag32;
    const double* dinv;     // padded 1 / diag, 0 off unknowns
    const float* dinv32;
    const double* wf;       // per-point smoother weights omega_k / d_k (learned), else null
    const float* wf32;
    const bf16* dinv16;     // BF16 1 / diag (BF16 smoother only)
};

template <class V> __device__ inline const V* tdiag(const TileArgs& t);
template <> __device__ inline const double* tdiag<double>(const TileArgs& t) { return t.diag; }
template <> __device__ inline const float* tdiag<float>(const TileArgs& t) { return t.diag32; }
template <class V> __device__ inline const V* tdinv(const TileArgs& t);
template <> __device__ inline const double* tdinv<double>(const TileArgs& t) { return t.dinv; }
template <> __device__ inline const float* tdinv<float>(const TileArgs& t) { return t.dinv32; }
template <class V> __device__ inline const V* twf(const TileArgs& t);
template <> __device__ inline const double* twf<double>(const TileArgs& t) { return t.wf; }
template <> __device__ inline const float* twf<float>(const TileArgs& t) { return t.wf32; }

// Element i of a padded field through a 32-bit byte offset from the field's
// base (the tile kernels run only while a padded field spans less than
// 4 GiB): one VGPR per node serves every field.
template <class T>
__device__ inline T ld(const T* __restrict__ base, uint32_t i) {
    return *(const T*)((const char*)base + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ inline void st(T* __restrict__ base, uint32_t i, T v) {
    *(T*)((char*)base + i * (uint32_t)sizeof(T)) = v;
}

// A read without a branch: a lane whose node is off the grid (or not wanted)
// reads element 0 instead and takes `none`, so every read of a row is issued
// at once and stays in flight together.
template <class T>
__device__ inline T ldz(const T* __restrict__ base, bool ok, uint32_t i, T none = T{}) {
    const T v = ld(base, ok ? i : 0u);
    return ok ? v : none;
}

// The tiles of this block's wavefront (block-uniform grid, one range per
// wavefront) and the lane's column.
struct TileLane {
    int lane;
    int64_t t0, t1;   // tile range of this wavefront
};

__device__ inline TileLane tile_lane(const TileArgs& t) {
    TileLane L;
    L.lane = threadIdx.x & (WAVE - 1);
    const int64_t gw = xcd_block() * (int64_t)TWB + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    L.t0 = gw * t.tpw;
    L.t1 = min(L.t0 + (int64_t)t.tpw, t.ntiles);
    return L;
}

__device__ inline void tile_origin_of(const TileArgs& t, int tid, int* x0, int* y0) {
    tid = __builtin_amdgcn_readfirstlane(tid);
    *x0 = (tid % t.ntx) * TX;
    *y0 = (tid / t.ntx) * TY;
}

__device__ inline void tile_origin(const TileArgs& t, int64_t tix, int* x0, int* y0) {
    tile_origin_of(t, t.tiles[tix], x0, y0);
}

// The wavefront's first tile id, read at the kernel's start beside the
// partial sums it reduces (0 when the wavefront has no tile).
__device__ inline int first_tile(const TileArgs& t, const TileLane& L) {
    return L.t0 < L.t1 ? t.tiles[L.t0] : 0;
}

// p = z + beta p_old on the tile and its halo rows, q = A p on the tile;
// partial (p, q).
template <class V>
__global__ void __launch_bounds__(TNT) k_t2_pspmv(TileArgs t, const V* __restrict__ z,
                                                  const double* __restrict__ pold, double* __restrict__ pnew,
                                                  double* __restrict__ q, const double* __restrict__ rz_cur,
                                                  const double* __restrict__ rz_prev, int np,
                                                  double* __restrict__ part_pq, PcgScalars* sc) {
    // the flag and the first tile are read with the partials; the first
    // tile's first rows (T2_AHEAD of them) are read before the partials are
    // reduced, so their latency overlaps the reduction (a wavefront without
    // a tile reads tile 0's and drops them); nothing is stored once the
    // solve is done
    const int32_t done = sc->done;
    const TileLane L = tile_lane(t);
    int x0, y0;
    tile_origin_of(t, first_tile(t, L), &x0, &y0);
    int xc = x0 - 2 + L.lane;
    bool xin = xc >= 0 && xc < t.nx;
    auto row = [&](int j, double& d, double& zz, double& pp) {
        const bool ok = xin && j >= 0 && j < t.ny && j <= y0 + TY;
        const uint32_t pn = xc + t.sy * j;
        d = ldz(t.diag, ok, pn);
        zz = to_f64(ldz(z, ok, pn));
        pp = ldz(pold, ok, pn);
    };
    // rows j .. j + T2_AHEAD - 1 in flight (read ahead)
    double dq[T2_AHEAD], zq[T2_AHEAD], oq[T2_AHEAD];
#pragma unroll
    for (int k = 0; k < T2_AHEAD; ++k) row(y0 - 1 + k, dq[k], zq[k], oq[k]);
    // the tile's last row and its halo row below are the first rows of the
    // tile below, which reads them at its start: read here at the start too
    // (so the second read finds them in L2) and taken by the march from here
    double dt[2], zt2[2], ot[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) row(y0 + TY - 1 + k, dt[k], zt2[k], ot[k]);
    double rho, rho_prev = 0.0;
    if (rz_prev) block_total2<TNT>(rz_cur, rz_prev, np, &rho, &rho_prev);
    else rho = block_total<TNT>(rz_cur, np);
    if (done) return;
    const double beta = rz_prev ? rho / rho_prev : 0.0;
    if (!(rho > 0.0) || bad_value(rho) || bad_value(beta)) {
        if (lead()) {
            sc->status = (bad_value(rho) || bad_value(beta)) ? EB_ENAN : EB_ENOTSPD;
            sc->done = 1;
        }
        return;
    }
    double part = 0.0;
    for (int64_t ti = L.t0; ti < L.t1; ++ti) {
        if (ti > L.t0) {
            tile_origin(t, ti, &x0, &y0);
            xc = x0 - 2 + L.lane;
            xin = xc >= 0 && xc < t.nx;
#pragma unroll
            for (int k = 0; k < T2_AHEAD; ++k) row(y0 - 1 + k, dq[k], zq[k], oq[k]);
#pragma unroll
            for (int k = 0; k < 2; ++k) row(y0 + TY - 1 + k, dt[k], zt2[k], ot[k]);
        }
        const bool inner = xin && L.lane >= 2 && L.lane < 2 + TX;
        double pa = 0.0, pb = 0.0, da = 0.0;   // p of rows j - 2, j - 1; d of row j - 1
        // fully unrolled: the rows in flight are never copied between
        // registers, so no read waits before the row that uses it
#pragma unroll
        for (int jj = 0; jj < TY + 2; ++jj) {
            const int j = y0 - 1 + jj;
            double dn, zn, on;
            // row y0 - 1 + jj + T2_AHEAD: one of the last two (read at the
            // start) or a row of the march (jj is a compile-time constant)
            const int ahead = jj - 1 + T2_AHEAD;
            if (ahead >= TY - 1 && ahead <= TY) {
                dn = dt[ahead - (TY - 1)];
                zn = zt2[ahead - (TY - 1)];
                on = ot[ahead - (TY - 1)];
            } else {
                row(j + T2_AHEAD, dn, zn, on);
            }
            const double d0 = dq[0];
            const double pc = d0 != 0.0 ? zq[0] + beta * oq[0] : 0.0;
            // row j - 1: q = A p
            const double lr = from_left(pb) + from_right(pb);
            if (j > y0 && inner && da != 0.0) {
                const double qv = da * pb - t.s * (lr + (pa + pc));
                const uint32_t pn = xc + t.sy * (j - 1);
                st(pnew, pn, pb);
                st(q, pn, qv);
                part += pb * qv;
            }
            pa = pb;
            pb = pc;
            da = d0;
#pragma unroll
            for (int k = 0; k + 1 < T2_AHEAD; ++k) {
                dq[k] = dq[k + 1];
                zq[k] = zq[k + 1];
                oq[k] = oq[k + 1];
            }
            dq[T2_AHEAD - 1] = dn;
            zq[T2_AHEAD - 1] = zn;
            oq[T2_AHEAD - 1] = on;
        }
    }
    block_partial<TNT>(part, part_pq);
}

// UPD: alpha = rho / (p, q); x += alpha p; r_out = r_in - alpha q and its
// partial ||r_out||^2 (without UPD, r = r_in: the first V-cycle).  Then, with
// r in the halo recomputed from r_in and q, the pre-smoothing residual
// res = r - A z1 = (1 - omega) r + omega s sum (r / d)_nbr (LW: z1 = wf r,
// res = r - d z1 + s sum z1_nbr) on the tile and its first halo, the
// restriction's u = (I - omega A D^-1) res = (1 - omega) res +
// omega s sum (res / d)_nbr on the tile (the prolongator keeps omega), and per
// level-0 box the sum of u over each of its aggregates (each column's three
// rows, then the three columns): r_c = P^T res.  The CG update and res are
// FP64; res is rounded to V, the restriction runs in V.
template <class V, bool LW, bool UPD>
__global__ void __launch_bounds__(TNT) k_t2_xr_restrict(TileArgs t, BoxArgs b, double* __restrict__ x,
                                                        const double* __restrict__ rin, double* __restrict__ rout,
                                                        const double* __restrict__ pv,
                                                        const double* __restrict__ q, double omega,
                                                        const double* __restrict__ rz_cur,
                                                        const double* __restrict__ part_pq, int np,
                                                        double* __restrict__ part_rr, V* __restrict__ rc,
                                                        const V* __restrict__ dg_c, double omega_c,
                                                        V* __restrict__ sv_c, PcgScalars* sc) {
    // the flag and the first tile are read with the partials; the first
    // tile's first rows and box row are read before the partials are
    // reduced, so their latency overlaps the reduction (a wavefront without a
    // tile reads tile 0's and drops them); nothing is stored once the solve
    // is done
    const int32_t done = sc->done;
    const TileLane L = tile_lane(t);
    // a box's lead lane is its left column; lanes 2 .. 61 hold the tile's 20 boxes
    const int bl = L.lane - 2;
    const bool box_lead = bl >= 0 && bl < TX && bl % 3 == 0;
    const int ox = bl >= 0 ? bl % 3 : 0;
    int x0, y0;
    tile_origin_of(t, first_tile(t, L), &x0, &y0);
    int xc = x0 - 2 + L.lane;
    bool xin = xc >= 0 && xc < t.nx;
    bool inner = xin && bl >= 0 && bl < TX;
    int bx = xc >= 0 ? xc / 3 : 0;
    // one row of a lane: 1 / d, r_in, q (UPD); LW: weight, d; the tile's
    // own rows also x and p (UPD)
    struct Row { double iv, r, q, w, d, x, p; };
    auto row = [&](int j, Row& R) {
        const bool ok = xin && j >= 0 && j < t.ny && j <= y0 + TY + 1;
        const bool own = ok && inner && j >= y0 && j < y0 + TY;
        const uint32_t pn = xc + t.sy * j;
        R.iv = ldz(t.dinv, ok, pn);
        R.r = ldz(rin, ok, pn);
        R.q = UPD ? ldz(q, ok, pn) : 0.0;
        R.w = LW ? ldz(t.wf, ok, pn) : 0.0;
        R.d = LW ? ldz(t.diag, ok, pn) : 0.0;
        R.x = UPD ? ldz((const double*)x, own, pn) : 0.0;
        R.p = UPD ? ldz(pv, own, pn) : 0.0;
    };
    // box row of the lane's box: aggregate count, first aggregate, node
    // map and omega_c / d_c of the first aggregate (read a box row ahead)
    auto boxrow = [&](int by, int& m, int& c0, int& map, V& w0) {
        const bool ok = inner && by < b.nby && bx < b.nbx;
        const uint32_t box = by * b.nbx + bx;
        m = ldz(b.ncomp, ok, box);
        c0 = ldz(b.cstart, ok, box);
        map = ldz(b.map, ok, box);
        w0 = ldz(vbw0<V>(b), ok, box);
    };
    Row Rq[T2_AHEAD];                    // rows j .. j + T2_AHEAD - 1 (read ahead)
#pragma unroll
    for (int k = 0; k < T2_AHEAD; ++k) row(y0 - 2 + k, Rq[k]);
    // the tile's last two rows and its two halo rows below are the first
    // rows of the tile below, which reads them at its start: reading them at
    // the start here too lets the second read find them in L2 (read at the
    // end of the march, some 15 us later, they were mostly fetched again)
    Row Rt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) row(y0 + TY - 2 + k, Rt[k]);
    int bm, bc0, bmap;
    V bw0;
    boxrow(y0 / 3, bm, bc0, bmap, bw0);
    double alpha = 0.0;
    if (!UPD && done) return;
    if (UPD) {
        double rho, pq;
        block_total2<TNT>(rz_cur, part_pq, np, &rho, &pq);
        if (done) return;
        if (!(pq > 0.0) || bad_value(pq)) {
            if (lead()) {
                sc->status = bad_value(pq) ? EB_ENAN : EB_ENOTSPD;
                sc->done = 1;
            }
            return;
        }
        alpha = rho / pq;
        if (lead()) {
            sc->iters = sc->iters + 1;   // counted on the device: a captured iteration carries no number
            sc->pq = pq;
        }
    }
    const double sw = omega * t.s;
    const V wV = (V)omega, swV = (V)sw;
    double part = 0.0;
    for (int64_t ti = L.t0; ti < L.t1; ++ti) {
        if (ti > L.t0) {
            tile_origin(t, ti, &x0, &y0);
            xc = x0 - 2 + L.lane;
            xin = xc >= 0 && xc < t.nx;
            inner = xin && bl >= 0 && bl < TX;
            bx = xc >= 0 ? xc / 3 : 0;
#pragma unroll
            for (int k = 0; k < T2_AHEAD; ++k) row(y0 - 2 + k, Rq[k]);
#pragma unroll
            for (int k = 0; k < 4; ++k) row(y0 + TY - 2 + k, Rt[k]);
            boxrow(y0 / 3, bm, bc0, bmap, bw0);
        }
        // rolling rows: z1 (j-2, j-1), r (j-1), 1 / d (j-2, j-1), d (j-1),
        // res (j-2), v (j-3, j-2), column sums per aggregate of the box row
        double za = 0.0, zb = 0.0, rb = 0.0, ia = 0.0, ib = 0.0, dbb = 0.0;
        V resa = V(0), va = V(0), vb = V(0);
        V acc[5] = {V(0), V(0), V(0), V(0), V(0)};
#pragma unroll
        for (int jj = 0; jj < TY + 4; ++jj) {
            const int j = y0 - 2 + jj;
            Row Rn;
            // row y0 - 2 + jj + T2_AHEAD: one of the last four (read at the
            // start) or a row of the march (jj is a compile-time constant)
            const int ahead = jj - 2 + T2_AHEAD;
            if (ahead >= TY - 2 && ahead <= TY + 1) Rn = Rt[ahead - (TY - 2)];
            else row(j + T2_AHEAD, Rn);
            const Row R0 = Rq[0];
            // row j: r, z1 (and the CG update of the tile's own rows)
            double rj = 0.0, zj = 0.0;
            if (R0.iv != 0.0) {
                rj = UPD ? R0.r - alpha * R0.q : R0.r;
                zj = LW ? R0.w * rj : rj * R0.iv;      // LW: z1; else r / d (omega applied below)
                if (UPD && inner && j >= y0 && j < y0 + TY) {
                    const uint32_t pn = xc + t.sy * j;
                    st(x, pn, R0.x + alpha * R0.p);
                    st(rout, pn, rj);
                    part += rj * rj;
                }
            }
            // row j - 1: res and res / d
            const double zlr = from_left(zb) + from_right(zb);
            V resb = V(0), vc = V(0);
            if (j >= y0 && ib != 0.0) {
                const double nb = zlr + (za + zj);
                const double rs = LW ? rb - (dbb * zb - t.s * nb) : (1.0 - omega) * rb + sw * nb;
                resb = (V)rs;
                vc = resb * (V)ib;
            }
            // row j - 2: u, added to its box row's column sums
            const V vlr = from_left(vb) + from_right(vb);
            if (j >= y0 + 2) {
                V u = V(0);
                if (ia != 0.0) u = (V(1) - wV) * resa + swV * (vlr + (va + vc));
                const int oy = (j - 2 - y0) % 3;
                if (bm == 1) {
                    acc[0] += u;
                } else if (bm > 1) {
                    const int c = (bmap >> (3 * (3 * oy + ox))) & 7;
#pragma unroll
                    for (int k = 0; k < 5; ++k)
                        if (c == k) acc[k] += u;
                }
                if (oy == 2) {
                    // box row complete: sum the three columns at the lead lane
                    const int cm = __reduce_max_sync(~0ull, bm);   // wave-uniform bound
                    for (int c = 0; c < cm && c < 5; ++c) {
                        const V a1 = from_right(acc[c]);
                        const V a2 = from_right(a1);
                        const V tot = (acc[c] + a1) + a2;
                        if (box_lead && c < bm) {
                            st(rc, (uint32_t)(bc0 + c), tot);
                            if (sv_c)
                                st(sv_c, (uint32_t)(bc0 + c),
                                   c == 0 ? tot * bw0 : (V)omega_c * tot / ld(dg_c, (uint32_t)(bc0 + c)));
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 5; ++k) acc[k] = V(0);
                    const int nby = (j + 1 - y0) / 3 + y0 / 3;   // next box row
                    if (nby < (y0 + TY) / 3) boxrow(nby, bm, bc0, bmap, bw0);
                }
            }
            za = zb; zb = zj; rb = rj;
            ia = ib; ib = R0.iv; dbb = R0.d;
            resa = resb; va = vb; vb = vc;
#pragma unroll
            for (int k = 0; k + 1 < T2_AHEAD; ++k) Rq[k] = Rq[k + 1];
            Rq[T2_AHEAD - 1] = Rn;
        }
    }
    if (UPD) block_partial<TNT>(part, part_rr);
}

// Prolongation and both halves of the fine smoothing that follow it:
// t = e_c[agg] on the tile and two halo rows,
// zt = z1 + (I - omega D^-1 A) t = z1 + (1 - omega) t + omega s (sum t_nbr) / d
// with z1 = omega r / d (LW: wf r) on the tile and one halo row,
// z = zt + omega (r - A zt) / d = (1 - omega) zt + omega (r + s sum zt_nbr) / d
// (LW: zt + wf (r - A zt)) on the tile; partial (r, z) in FP64.
// With part_rr, first the convergence test of the iterate r belongs to (the
// x/r kernel of this iteration wrote its ||r||^2 partials): once it holds,
// the remaining kernels of the chunk return at once.
// B16 (BF16 smoother): 1 / d read from its BF16 copy, z stored in BF16 (the
// partial uses the stored value).
template <class V, bool LW, bool B16 = false>
__global__ void __launch_bounds__(TNT) k_t2_up_post(TileArgs t, double omega, const int32_t* __restrict__ agg,
                                                    const V* __restrict__ ec, const double* __restrict__ r,
                                                    std::conditional_t<B16, bf16, V>* __restrict__ z,
                                                    double* __restrict__ part_rz,
                                                    const double* __restrict__ part_rr, int np, PcgScalars* sc) {
    // the flag and the first tile are read with the partials; the first
    // tile's first rows (T2_AHEAD of them) are read before the partials are
    // reduced, so their latency overlaps the reduction (a wavefront without
    // a tile reads tile 0's and drops them); nothing is stored once the
    // solve is done
    const int32_t done = sc->done;
    const TileLane L = tile_lane(t);
    const V* __restrict__ dinv = tdinv<V>(t);
    int x0, y0;
    tile_origin_of(t, first_tile(t, L), &x0, &y0);
    int xc = x0 - 2 + L.lane;
    bool xin = xc >= 0 && xc < t.nx;
    bool inner = xin && L.lane >= 2 && L.lane < 2 + TX;
    // one row of a lane: aggregate, 1 / d, r; LW: weight, d
    struct Row { int32_t g; V iv, w, d; double r; };
    auto row = [&](int j, Row& R) {
        const bool ok = xin && j >= 0 && j < t.ny && j <= y0 + TY + 1;
        const bool mid = ok && j >= y0 - 1 && j <= y0 + TY;
        const uint32_t pn = xc + t.sy * j;
        R.g = ldz(agg, ok, pn, -1);
        if constexpr (B16) R.iv = (V)bf16_to_f32(ldz(t.dinv16, mid, pn));
        else R.iv = ldz(dinv, mid, pn);
        R.r = ldz(r, mid, pn);
        R.w = LW ? ldz(twf<V>(t), mid, pn) : V(0);
        R.d = LW ? ldz(tdiag<V>(t), mid, pn) : V(0);
    };
    // e_c at a node's aggregate (0 where it has none)
    auto gather = [&](int32_t g) { return ldz(ec, g >= 0, (uint32_t)g); };
    Row Rq[T2_AHEAD];                    // rows j .. j + T2_AHEAD - 1 (read ahead)
#pragma unroll
    for (int k = 0; k < T2_AHEAD; ++k) row(y0 - 2 + k, Rq[k]);
    // the tile's last two rows and its two halo rows below are the first
    // rows of the tile below, which reads them at its start: read here at
    // the start too (so the second read finds them in L2)
    Row Rt[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) row(y0 + TY - 2 + k, Rt[k]);
    if (part_rr) {
        const double rr = block_total<TNT>(part_rr, np);
        if (done || converged_or_failed_total(rr, sc)) return;
    } else if (done) {
        return;
    }
    const V wV = (V)omega, sV = (V)t.s, swV = (V)(omega * t.s);
    double part = 0.0;
    for (int64_t ti = L.t0; ti < L.t1; ++ti) {
        if (ti > L.t0) {
            tile_origin(t, ti, &x0, &y0);
            xc = x0 - 2 + L.lane;
            xin = xc >= 0 && xc < t.nx;
            inner = xin && L.lane >= 2 && L.lane < 2 + TX;
#pragma unroll
            for (int k = 0; k < T2_AHEAD; ++k) row(y0 - 2 + k, Rq[k]);
#pragma unroll
            for (int k = 0; k < 4; ++k) row(y0 + TY - 2 + k, Rt[k]);
        }
        // e_c gathered two rows ahead (the aggregate of row j + 2 was read
        // one march step earlier, so the gather does not wait for it)
        V t0v = gather(Rq[0].g);
        V t1v = gather(Rq[1].g);
        // rolling rows: t (j-2, j-1), zt (j-3, j-2), 1 / d and r and LW
        // weights of rows j-2, j-1
        V ta = V(0), tb = V(0), zta = V(0), ztb = V(0);
        V iva = V(0), ivb = V(0), wa = V(0), wb = V(0), da = V(0), db = V(0);
        double ra = 0.0, rb = 0.0;
#pragma unroll
        for (int jj = 0; jj < TY + 4; ++jj) {
            const int j = y0 - 2 + jj;
            Row Rn;
            // row y0 - 2 + jj + T2_AHEAD: one of the last four (read at the
            // start) or a row of the march (jj is a compile-time constant)
            const int ahead = jj - 2 + T2_AHEAD;
            if (ahead >= TY - 2 && ahead <= TY + 1) Rn = Rt[ahead - (TY - 2)];
            else row(j + T2_AHEAD, Rn);
            const Row R0 = Rq[0];
            const V t2v = gather(Rq[2].g);
            // row j - 1: zt
            const V tlr = from_left(tb) + from_right(tb);
            V ztc = V(0);
            if (j >= y0 && ivb != V(0)) {
                const V z1 = LW ? wb * (V)rb : wV * (V)rb * ivb;
                ztc = z1 + ((V(1) - wV) * tb + swV * (tlr + (ta + t0v)) * ivb);
            }
            // row j - 2: z
            const V zlr = from_left(ztb) + from_right(ztb);
            if (j >= y0 + 2 && inner && iva != V(0)) {
                const V nb = zlr + (zta + ztc);
                const V rr = (V)ra;
                const V zv = LW ? ztb + wa * (rr - (da * ztb - sV * nb)) : (V(1) - wV) * ztb + wV * (rr + sV * nb) * iva;
                if constexpr (B16) {
                    const bf16 zb = f32_to_bf16((float)zv);
                    st(z, (uint32_t)(xc + t.sy * (j - 2)), zb);
                    part += ra * to_f64(zb);
                } else {
                    st(z, (uint32_t)(xc + t.sy * (j - 2)), zv);
                    part += ra * (double)zv;
                }
            }
            ta = tb; tb = t0v;
            zta = ztb; ztb = ztc;
            iva = ivb; ivb = R0.iv;
            ra = rb; rb = R0.r;
            wa = wb; wb = R0.w;
            da = db; db = R0.d;
            t0v = t1v;
            t1v = t2v;
#pragma unroll
            for (int k = 0; k + 1 < T2_AHEAD; ++k) Rq[k] = Rq[k + 1];
            Rq[T2_AHEAD - 1] = Rn;
        }
    }
    block_partial<TNT>(part, part_rz);
}

// out = b - A x (padded fields), partial ||out||^2.
template <bool VB = false>
__global__ void __launch_bounds__(NT) k_fine_resid(FineArgs f, const double* __restrict__ bp,
                                                   const double* __restrict__ x, double* __restrict__ out,
                                                   double* __restrict__ part) {
    double acc = 0.0;
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double ax = d * x[p] - f.s * nsum<VB>(x, p, f);
            const double rv = bp[p] - ax;
            out[p] = rv;
            acc += rv * rv;
        }
    }
    block_partial(acc, part);
}

__global__ void __launch_bounds__(NT) k_fine_norm2(FineArgs f, const double* __restrict__ v,
                                                   double* __restrict__ part) {
    double acc = 0.0;
    FINE_LOOP(f, p) {
        if (f.diag[p] != 0.0) acc += v[p] * v[p];
    }
    block_partial(acc, part);
}

// One block: ||b||^2, ||r0||^2, tolerance and the initial convergence test.
__global__ void __launch_bounds__(NT) k_finalize_init(PcgScalars* sc, const double* __restrict__ part_bb,
                                                      const double* __restrict__ part_rr, int np, double tol,
                                                      int iters) {
    double bb, rr;
    block_total2(part_bb, part_rr, np, &bb, &rr);
    if (threadIdx.x == 0) {
        sc->bb = bb;
        sc->rr = rr;
        sc->rr0 = rr;
        sc->tol2bb = tol * tol * bb;
        sc->status = (bad_value(bb) || bad_value(rr)) ? EB_ENAN : EB_OK;
        sc->done = (bb == 0.0 || rr <= tol * tol * bb || sc->status != EB_OK) ? 1 : 0;
        sc->iters = iters;
        sc->pq = 0.0;
    }
}

__global__ void __launch_bounds__(NT) k_finalize_true(PcgScalars* sc, const double* __restrict__ part, int np) {
    const double rr = block_total(part, np);
    if (threadIdx.x == 0) sc->rr_true = rr;
}

// ------------------------------------------------------------ coarse kernels
// Arithmetic and storage in the V-cycle precision V.  LPR lanes share one CSR
// row (strided over its entries) and combine their partial sums with
// butterfly shuffles inside the LPR-lane segment.
template <int LPR, class V>
__device__ inline V segment_sum(V v) {
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, LPR);
    return v;
}

template <class V>
struct Csr {
    const int32_t* rowptr;
    const int32_t* col;
    const V* val;
};

// Large coarse levels, two light passes each way:
//   res_j = rv_j - sum_e a_je omega rv_e / d_e;   rv_c[I] = sum_j R_Ij res_j;
//   zt_j = omega rv_j / d_j + sum_J P_jJ ev_c[J]; ev_i = zt_i + omega (rv_i - (A zt)_i) / d_i.
template <int LPR, class V>
__global__ void __launch_bounds__(NT) k_csr_resid(int64_t n, Csr<V> A, const V* __restrict__ sv,
                                                  const V* __restrict__ rv, V* __restrict__ res,
                                                  const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t row = ((int64_t)blockIdx.x * NT + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= n) return;
    V az = V(0);
    for (int e = A.rowptr[row] + lane; e < A.rowptr[row + 1]; e += LPR) {
        const int k = A.col[e];
        az += A.val[e] * sv[k];
    }
    az = segment_sum<LPR>(az);
    if (lane == 0) res[row] = rv[row] - az;
}

template <int LPR, class V>
__global__ void __launch_bounds__(NT) k_csr_matvec(int64_t n, Csr<V> M, const V* __restrict__ x,
                                                   V* __restrict__ y, const V* __restrict__ dg_y, V omega_y,
                                                   V* __restrict__ sv_y, const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t row = ((int64_t)blockIdx.x * NT + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= n) return;
    V acc = V(0);
    for (int e = M.rowptr[row] + lane; e < M.rowptr[row + 1]; e += LPR) acc += M.val[e] * x[M.col[e]];
    acc = segment_sum<LPR>(acc);
    if (lane == 0) {
        y[row] = acc;
        if (sv_y) sv_y[row] = omega_y * acc / dg_y[row];
    }
}

template <int LPR, class V>
__global__ void __launch_bounds__(NT) k_csr_prolong(int64_t n, Csr<V> P, const V* __restrict__ sv,
                                                    const V* __restrict__ ev_c, V* __restrict__ zt,
                                                    const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t row = ((int64_t)blockIdx.x * NT + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= n) return;
    V acc = V(0);
    for (int e = P.rowptr[row] + lane; e < P.rowptr[row + 1]; e += LPR) acc += P.val[e] * ev_c[P.col[e]];
    acc = segment_sum<LPR>(acc);
    if (lane == 0) zt[row] = sv[row] + acc;
}

template <int LPR, class V>
__global__ void __launch_bounds__(NT) k_csr_post(int64_t n, Csr<V> A, const V* __restrict__ diag, V omega,
                                                 const V* __restrict__ rv, const V* __restrict__ zt,
                                                 V* __restrict__ ev, const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t row = ((int64_t)blockIdx.x * NT + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= n) return;
    V az = V(0);
    for (int e = A.rowptr[row] + lane; e < A.rowptr[row + 1]; e += LPR) az += A.val[e] * zt[A.col[e]];
    az = segment_sum<LPR>(az);
    if (lane == 0) ev[row] = zt[row] + omega * (rv[row] - az) / diag[row];
}

// Residual and restriction in one pass:
//   rv_c[I] = sum_{j in R row I} R_Ij (rv_j - sum_e a_je omega rv_e / d_e).
// The inner row of A is read GB entries at a time (their columns and values,
// then their gathers, then the sums in entry order), so a row costs a few
// memory round trips instead of one per entry.
constexpr int GB = 8;

template <class V>
__device__ inline V row_dot(const Csr<V>& M, int e0, int e1, const V* __restrict__ x) {
    V acc = V(0);
    for (int f0 = e0; f0 < e1; f0 += GB) {
        int k[GB];
        V a[GB], xv[GB];
#pragma unroll
        for (int u = 0; u < GB; ++u) {
            k[u] = f0 + u < e1 ? M.col[f0 + u] : -1;
            a[u] = f0 + u < e1 ? M.val[f0 + u] : V(0);
        }
#pragma unroll
        for (int u = 0; u < GB; ++u) xv[u] = k[u] >= 0 ? x[k[u]] : V(0);
#pragma unroll
        for (int u = 0; u < GB; ++u)
            if (f0 + u < e1) acc += a[u] * xv[u];
    }
    return acc;
}

template <int LPR, class V>
__global__ void __launch_bounds__(NT) k_coarse_down(int64_t nc, Csr<V> R, Csr<V> A, const V* __restrict__ sv,
                                                    const V* __restrict__ rv, V* __restrict__ rv_c,
                                                    const V* __restrict__ dg_c, V omega_c, V* __restrict__ sv_c,
                                                    const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t row = ((int64_t)blockIdx.x * NT + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= nc) return;
    V acc = V(0);
    for (int e = R.rowptr[row] + lane; e < R.rowptr[row + 1]; e += LPR) {
        const int j = R.col[e];
        const V az = row_dot(A, A.rowptr[j], A.rowptr[j + 1], sv);
        acc += R.val[e] * (rv[j] - az);
    }
    acc = segment_sum<LPR>(acc);
    if (lane == 0) {
        rv_c[row] = acc;
        if (sv_c) sv_c[row] = omega_c * acc / dg_c[row];
    }
}

// Prolongation and post-smoothing in one pass:
//   zt_j = omega rv_j / d_j + sum_{P row j} P_jJ ev_c[J];
//   ev[i] = zt_i + omega (rv_i - sum_{A row i} a_ij zt_j) / d_i.
// (rows of P read as in k_coarse_down, GB entries at a time)
template <int LPR, class V>
__global__ void __launch_bounds__(NT) k_coarse_up(int64_t n, Csr<V> A, Csr<V> P, const V* __restrict__ diag,
                                                  V omega, const V* __restrict__ rv, const V* __restrict__ sv,
                                                  const V* __restrict__ ev_c, V* __restrict__ ev,
                                                  const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t row = ((int64_t)blockIdx.x * NT + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= n) return;
    V acc = V(0);
    for (int e = A.rowptr[row] + lane; e < A.rowptr[row + 1]; e += LPR) {
        const int j = A.col[e];
        const V zt = sv[j] + row_dot(P, P.rowptr[j], P.rowptr[j + 1], ev_c);
        acc += A.val[e] * zt;
    }
    acc = segment_sum<LPR>(acc);
    if (lane == 0) {
        const V zi = sv[row] + row_dot(P, P.rowptr[row], P.rowptr[row + 1], ev_c);
        ev[row] = zi + omega * (rv[row] - acc) / diag[row];
    }
}

// Coarse levels in sliced ELL (one lane per row, slot-major slices of 64
// rows): a row's entries are read as coalesced slots, GB at a time, then
// gathered, then summed in column order.
template <class V>
struct SellV {
    int w;   // slots per row (the matrix's longest row)
    const int32_t* col;
    const V* val;
};

// Residual after pre-smoothing and restriction in one pass, with R A stored:
//   rv_c = R (rv - A sv) = R rv - (R A) sv,  sv = omega rv / d.
// LPR lanes share a coarse row; a lane issues the reads of UR entries of R
// and UQ of R A (columns and values, then the gathers) before it adds them.
template <int LPR, class V>
__global__ void __launch_bounds__(NT) k_down_ra(int64_t nc, Csr<V> R, Csr<V> RA, const V* __restrict__ rv,
                                                const V* __restrict__ sv, V* __restrict__ rv_c,
                                                const V* __restrict__ dg_c, V omega_c, V* __restrict__ sv_c,
                                                const PcgScalars* sc) {
    const int32_t done = sc->done;   // read beside the row pointers; tested before the stores
    // consecutive rows on one XCD (grid a multiple of 8): neighbouring coarse
    // rows gather overlapping fine entries, which then come from one L2
    const int64_t row = (xcd_block() * NT + threadIdx.x) / LPR;
    const int lane = threadIdx.x % LPR;
    if (row >= nc) return;
    constexpr int UR = 2, UQ = 2;
    const int r0 = R.rowptr[row], r1 = R.rowptr[row + 1];
    const int q0 = RA.rowptr[row], q1 = RA.rowptr[row + 1];
    V acc = V(0);
    for (int br = r0 + lane, bq = q0 + lane; br < r1 || bq < q1; br += UR * LPR, bq += UQ * LPR) {
        int kr[UR], kq[UQ];
        V ar[UR], aq[UQ], xr[UR], xq[UQ];
        // entries past a row's end read entry 0 and are dropped (column -1),
        // so the reads carry no branch and go out together
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const int e = br + u * LPR;
            const int ei = e < r1 ? e : 0;
            const int k = R.col[ei];
            const V a = R.val[ei];
            kr[u] = e < r1 ? k : -1;
            ar[u] = e < r1 ? a : V(0);
        }
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
            const int e = bq + u * LPR;
            const int ei = e < q1 ? e : 0;
            const int k = RA.col[ei];
            const V a = RA.val[ei];
            kq[u] = e < q1 ? k : -1;
            aq[u] = e < q1 ? a : V(0);
        }
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const V v = rv[kr[u] >= 0 ? kr[u] : 0];
            xr[u] = kr[u] >= 0 ? v : V(0);
        }
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
            const V v = sv[kq[u] >= 0 ? kq[u] : 0];
            xq[u] = kq[u] >= 0 ? v : V(0);
        }
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const V t = acc + ar[u] * xr[u];
            acc = kr[u] >= 0 ? t : acc;
        }
#pragma unroll
        for (int u = 0; u < UQ; ++u) {
            const V t = acc - aq[u] * xq[u];
            acc = kq[u] >= 0 ? t : acc;
        }
    }
    acc = segment_sum<LPR>(acc);
    if (done) return;
    if (lane == 0) {
        rv_c[row] = acc;
        if (sv_c) sv_c[row] = omega_c * acc / dg_c[row];
    }
}

// One row of a sliced matrix in chunks of W slots: slot u of the row is
// entry 64 (w slice + u) + lane, with w the matrix's width (a launch
// argument, so no offset is read before the entries).  A chunk's column and
// value reads are issued together, then its gathers, so a row costs one
// round trip per chunk rather than per entry.
template <class V, int W>
struct SellRow {
    int k[W];
    V a[W];
};

struct SellSpan {
    int e0;     // first entry of the lane's row
    int slots;  // slots of the slice
};

template <class V>
__device__ inline SellSpan sell_span(const SellV<V>& M, int slice, int lane) {
    return {slice * 64 * M.w + lane, M.w};
}

// A slot past the slice's width reads entry 0 and is dropped (column -1):
// no branch, so the reads of all matrices of a pass stay in one block and
// are issued together (a branch per slot let the compiler defer a matrix's
// slice pointer until the previous matrix's reads were out).
template <class V, int W>
__device__ inline void sell_load(const SellV<V>& M, const SellSpan& sp, int u0, SellRow<V, W>& r) {
#pragma unroll
    for (int u = 0; u < W; ++u) {
        const bool in = u0 + u < sp.slots;
        const int e = in ? sp.e0 + 64 * (u0 + u) : 0;
        const int k = M.col[e];
        const V a = M.val[e];
        r.k[u] = in ? k : -1;
        r.a[u] = in ? a : V(0);
    }
}

// x at the chunk's columns (a dropped slot reads x[0] and takes 0)
template <class V, int W>
__device__ inline void sell_gather(const SellRow<V, W>& r, const V* __restrict__ x, V* xv) {
#pragma unroll
    for (int u = 0; u < W; ++u) {
        const V v = x[r.k[u] >= 0 ? r.k[u] : 0];
        xv[u] = r.k[u] >= 0 ? v : V(0);
    }
}

// acc + the chunk's products, in slot (column) order; dropped slots leave acc
// as it is
template <class V, int W>
__device__ inline V sell_acc(V acc, const SellRow<V, W>& r, const V* xv) {
#pragma unroll
    for (int u = 0; u < W; ++u) {
        const V t = acc + r.a[u] * xv[u];
        acc = r.k[u] >= 0 ? t : acc;
    }
    return acc;
}

// Prolongation and post-smoothing in one pass, with A P stored:
//   zt = sv + P ev_c,  ev = zt + omega (rv - A zt) / d
//      = sv + P ev_c + omega (rv - A sv - (A P) ev_c) / d.
// The first chunks of P, A and A P are read together; rows of A and A P
// longer than WA slots (3-D: 27) continue in further chunks of both.
template <class V, int WP, int WA>
__global__ void __launch_bounds__(NT) k_sell_up(int64_t n, SellV<V> A, SellV<V> P, SellV<V> AP,
                                                const V* __restrict__ diag, V omega, const V* __restrict__ rv,
                                                const V* __restrict__ sv, const V* __restrict__ ev_c,
                                                V* __restrict__ ev, const PcgScalars* sc) {
    const int32_t done = sc->done;   // read beside the first reads; tested before the store
    const int64_t row = xcd_block() * NT + threadIdx.x;   // consecutive rows on one XCD
    const int slice = __builtin_amdgcn_readfirstlane((int)(row >> 6));
    if (row >= n) return;
    const int lane = (int)(row & 63);
    const SellSpan sp = sell_span(P, slice, lane), sa = sell_span(A, slice, lane), sq = sell_span(AP, slice, lane);
    SellRow<V, WP> rp;
    SellRow<V, WA> ra, rq;
    sell_load(P, sp, 0, rp);
    sell_load(A, sa, 0, ra);
    sell_load(AP, sq, 0, rq);
    const V svr = sv[row], rvr = rv[row], dr = diag[row];
    V xp[WP], xa[WA], xq[WA];
    sell_gather(rp, ev_c, xp);
    sell_gather(ra, sv, xa);
    sell_gather(rq, ev_c, xq);
    V pe = sell_acc(V(0), rp, xp);
    V as = sell_acc(V(0), ra, xa);
    V ape = sell_acc(V(0), rq, xq);
    for (int u0 = WA; u0 < max(sa.slots, sq.slots); u0 += WA) {
        sell_load(A, sa, u0, ra);
        sell_load(AP, sq, u0, rq);
        sell_gather(ra, sv, xa);
        sell_gather(rq, ev_c, xq);
        as = sell_acc(as, ra, xa);
        ape = sell_acc(ape, rq, xq);
    }
    for (int u0 = WP; u0 < sp.slots; u0 += WP) {
        sell_load(P, sp, u0, rp);
        sell_gather(rp, ev_c, xp);
        pe = sell_acc(pe, rp, xp);
    }
    if (done) return;
    ev[row] = svr + pe + omega * (rvr - as - ape) / dr;
}

// Coarsest: ev = W rv with W the dense inverse (FP64 in either precision);
// one wavefront per row.
template <class V>
__global__ void __launch_bounds__(NT) k_dense_apply(int64_t n, const double* __restrict__ W,
                                                    const V* __restrict__ rv, V* __restrict__ ev,
                                                    const PcgScalars* sc) {
    const int32_t done = sc->done;   // read beside the first loads; tested before the store
    const int64_t row = (int64_t)blockIdx.x * (NT / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (row >= n) return;
    double acc = 0.0;
    for (int64_t j = lane; j < n; j += WAVE) acc += W[row * n + j] * (double)rv[j];
    acc = wave_sum(acc);
    if (done) return;
    if (lane == 0) ev[row] = (V)acc;
}

// Island hierarchies: ev = W_b rv on the rows of each island that ends on
// this level (W_b the inverse of its diagonal block; FP64 in either
// precision), one wavefront per row; rows outside the blocks keep their ev.
template <class V>
__global__ void __launch_bounds__(NT) k_block_apply(int64_t n, const int32_t* __restrict__ blk_of,
                                                    const int32_t* __restrict__ blk, const int64_t* __restrict__ woff,
                                                    const double* __restrict__ W, const V* __restrict__ rv,
                                                    V* __restrict__ ev, const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t row = (int64_t)blockIdx.x * (NT / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (row >= n) return;
    const int b = blk_of[row];
    if (b < 0) return;
    const int o = blk[2 * b], m = blk[2 * b + 1];
    const double* Wr = W + woff[b] + (int64_t)(row - o) * m;
    double acc = 0.0;
    for (int j = lane; j < m; j += WAVE) acc += Wr[j] * (double)rv[o + j];
    acc = wave_sum(acc);
    if (lane == 0) ev[row] = (V)acc;
}

// One-level hierarchies (fine level = coarsest): gather r into compact order
// (after the convergence test) and scatter z back with the (r, z) partials.
__global__ void __launch_bounds__(NT) k_gather(int64_t n, const int32_t* __restrict__ pad,
                                               const double* __restrict__ src, double* __restrict__ dst,
                                               PcgScalars* sc, int check, const double* __restrict__ part_rr,
                                               int np) {
    if (sc->done) return;
    if (check && converged_or_failed(part_rr, np, sc)) return;
    for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < n; k += (int64_t)gridDim.x * NT)
        dst[k] = src[pad[k]];
}

__global__ void __launch_bounds__(NT) k_scatter_dot(int64_t n, const int32_t* __restrict__ pad,
                                                    const double* __restrict__ ev, const double* __restrict__ r,
                                                    double* __restrict__ z, double* __restrict__ part_rz,
                                                    const PcgScalars* sc) {
    if (sc->done) return;
    double part = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < n; k += (int64_t)gridDim.x * NT) {
        const int32_t p = pad[k];
        z[p] = ev[k];
        part += r[p] * ev[k];
    }
    block_partial(part, part_rz);
}

// ---------------------------------------------------- layout conversion
__global__ void __launch_bounds__(NT) k_load_field(int64_t n, const int64_t* __restrict__ nodes,
                                                   const int32_t* __restrict__ pad, const double* __restrict__ src,
                                                   double* __restrict__ dst) {
    const int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (k < n) dst[pad[k]] = src[nodes[k]];
}

// Zero initial guess: b goes into the padded layout twice, as b and as
// r0 = b - A 0 = b, x is cleared at the unknowns (every store to x is guarded
// by a non-zero diagonal, so the other slots hold the zero set at setup), and
// each block of the fixed reduction grid leaves its partial of ||b||^2, which
// is also ||r0||^2.  One pass over b instead of a load, a clear of all of x
// and two reductions over the strips.
__global__ void __launch_bounds__(NT) k_init_zero_guess(int64_t n, const int64_t* __restrict__ nodes,
                                                        const int32_t* __restrict__ pad,
                                                        const double* __restrict__ src, double* __restrict__ bvec,
                                                        double* __restrict__ x, double* __restrict__ r0,
                                                        double* __restrict__ part) {
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < n; k += (int64_t)gridDim.x * NT) {
        const int32_t q = pad[k];
        const double v = src[nodes[k]];
        bvec[q] = v;
        r0[q] = v;
        x[q] = 0.0;
        acc += v * v;
    }
    block_partial(acc, part);
}

template <class V>
__global__ void __launch_bounds__(NT) k_store_field(int64_t n, const int64_t* __restrict__ nodes,
                                                    const int32_t* __restrict__ pad, const V* __restrict__ src,
                                                    double* __restrict__ dst) {
    const int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (k < n) dst[nodes[k]] = to_f64(src[pad[k]]);
}

__global__ void k_mark_running(PcgScalars* sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->done = 0;
        sc->status = EB_OK;
    }
}

__global__ void __launch_bounds__(NT) k_copy_f64(int64_t n, const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------- fine solve layout
__global__ void __launch_bounds__(BLOCK) k_fine_layout(const int64_t* __restrict__ fine_nodes, int64_t nunk,
                                                       GridDims d, int px, const double* __restrict__ diag0,
                                                       const int32_t* __restrict__ agg0, int has_agg,
                                                       int32_t* __restrict__ fine_pad,
                                                       double* __restrict__ diag_p, double* __restrict__ dinv_p,
                                                       int32_t* __restrict__ agg_p,
                                                       int32_t* __restrict__ strip_flag, int strip_w,
                                                       int32_t* __restrict__ tile_flag, int tile_ntx) {
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= nunk) return;
    const int64_t n = fine_nodes[k];
    const int64_t i = n % d.nx;
    const int64_t row = n / d.nx;
    const int64_t pidx = i + (int64_t)px * row;
    fine_pad[k] = (int32_t)pidx;
    diag_p[pidx] = diag0[k];
    dinv_p[pidx] = 1.0 / diag0[k];
    agg_p[pidx] = has_agg ? agg0[k] : -1;
    strip_flag[pidx / strip_w] = 1;
    if (tile_flag) tile_flag[(row / TY) * tile_ntx + i / TX] = 1;   // 2-D: row is j
}

// A dense node field copied into the padded layout.
__global__ void __launch_bounds__(BLOCK) k_pad_field(int64_t nn, GridDims d, int px, const double* __restrict__ src,
                                                     double* __restrict__ dst) {
    const int64_t n = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (n >= nn) return;
    dst[n % d.nx + (int64_t)px * (n / d.nx)] = src[n];
}

// 2-D level-0 boxes: the aggregate of each of the 9 nodes, relative to the
// box's first aggregate, 3 bits per node (7: not an unknown or off the grid).
__global__ void __launch_bounds__(BLOCK) k_box_map2(int nbx, int nby, int nx, int ny, int px,
                                                   const int32_t* __restrict__ cstart,
                                                   const int32_t* __restrict__ agg_p, int32_t* __restrict__ map) {
    const int64_t box = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (box >= (int64_t)nbx * nby) return;
    const int bx = (int)(box % nbx), by = (int)(box / nbx);
    const int32_t c0 = cstart[box];
    int32_t m = 0;
    for (int n = 0; n < 9; ++n) {
        const int i = 3 * bx + n % 3, j = 3 * by + n / 3;
        int32_t c = 7;
        if (i < nx && j < ny) {
            const int32_t a = agg_p[(int64_t)i + (int64_t)px * j];
            if (a >= 0) c = a - c0;
        }
        m |= (c & 7) << (3 * n);
    }
    map[box] = m;
}

// 2-D level-0 boxes: omega_1 / d_1 of the box's first aggregate (the level-1
// smoother weight that the restriction applies to its sum), 0 for a box
// without aggregates.  omega_1 comes from the device copy of the level's
// scalars (rho, omega per level).
__global__ void __launch_bounds__(BLOCK) k_box_w0(int64_t nb, const int32_t* __restrict__ cstart,
                                                 const int32_t* __restrict__ ncomp, const double* __restrict__ d1,
                                                 const double* __restrict__ scal, double* __restrict__ w0) {
    const int64_t box = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (box >= nb) return;
    w0[box] = ncomp[box] > 0 ? scal[2 * 1 + 1] / d1[cstart[box]] : 0.0;
}

__global__ void __launch_bounds__(BLOCK) k_flag_nonzero(const int32_t* __restrict__ v, int64_t n,
                                                        int32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) flag[i] = v[i] > 0;
}

__global__ void __launch_bounds__(BLOCK) k_compact_list(const int32_t* __restrict__ flag, const int32_t* __restrict__ off,
                                                   int64_t n, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n && flag[i]) out[off[i]] = (int32_t)i;
}


// ------------------------------------------------------------- host side
// Kernel timing hook: harvest completed event pairs into the accumulators.
static int timing_harvest(amg_handle* H) {
    if (H->tim_used == 0) return EB_OK;
    EB_HIP(hipStreamSynchronize(H->tim_stream));
    for (int i = 0; i < H->tim_used; ++i) {
        float ms = 0.f;
        EB_HIP(hipEventElapsedTime(&ms, H->tim_ev[2 * i], H->tim_ev[2 * i + 1]));
        H->tim_ms += ms;
        H->tim_launches += 1;
    }
    H->tim_used = 0;
    return EB_OK;
}

// Events for the next timed launch of kernel `id` (null when not timed).
// The launch records them at the kernel's own start and end
// (hipExtLaunchKernel), so the durations match a kernel trace.
static int timing_slot(amg_handle* H, int id, hipStream_t s, hipEvent_t* e0, hipEvent_t* e1) {
    *e0 = *e1 = nullptr;
    if (H->tim_kernel != id) return EB_OK;
    if (H->tim_used == H->tim_cap) EB_TRY(timing_harvest(H));
    H->tim_stream = s;
    *e0 = H->tim_ev[2 * H->tim_used];
    *e1 = H->tim_ev[2 * H->tim_used + 1];
    H->tim_used += 1;
    return EB_OK;
}

#define EB_TIMED_LAUNCH(H, id, s, KERNEL, GRID, BLOCKDIM, SHMEM, ...)                          \
    do {                                                                                      \
        hipEvent_t e0_, e1_;                                                                  \
        EB_TRY(timing_slot((H), (id), (s), &e0_, &e1_));                                      \
        if (e0_)                                                                              \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCKDIM, SHMEM, s, e0_, e1_, 0, __VA_ARGS__); \
        else                                                                                  \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCKDIM, SHMEM, s, __VA_ARGS__);                \
    } while (0)

// grid of `bs`-thread blocks covering n items, rounded up to whole XCD groups
static unsigned xcd_grid(int64_t n, int bs) {
    int64_t g = (n + bs - 1) / bs;
    g = (g + NUM_XCD - 1) / NUM_XCD * NUM_XCD;
    return (unsigned)(g > 0 ? g : NUM_XCD);
}

// the box restriction: a box per thread in 2-D, R3_BOXES boxes per block in 3-D
static unsigned restrict_grid(const amg_handle* H) {
    return xcd_grid(H->nboxes0, H->d.dim == 2 ? RNT : R3_BOXES);
}

static FineArgs fine_args(const amg_handle* H) {
    FineArgs f;
    f.strips = H->strips;
    f.nstrips = H->nstrips;
    const int64_t np = H->red.nparts;
    f.spb = (H->nstrips + np - 1) / np;
    f.strip_w = H->strip_w;
    f.sy = H->px;
    f.sz = (int64_t)H->px * H->d.ny;
    f.dim = H->d.dim;
    f.s = H->d.s;
    f.diag = H->diag_p;
    f.diag32 = H->diag_p32;
    f.wf = H->wf_on ? H->wf : nullptr;
    f.wf32 = H->wf_on ? H->wf32 : nullptr;
    f.dinv16 = H->dinv_p16;
    for (int a = 0; a < 3; ++a) f.bf[a] = H->beta_on ? H->bf_p[a] : nullptr;
    return f;
}

// Non-reducing fine kernels: one node per thread over the whole strip list
// (no fixed partial count to respect).
static FineArgs fine_args_full(const amg_handle* H, unsigned* grid) {
    FineArgs f = fine_args(H);
    f.spb = NT / H->strip_w;
    *grid = xcd_grid(H->nstrips * (int64_t)H->strip_w, NT);
    return f;
}

static TileArgs tile_args(const amg_handle* H) {
    TileArgs t;
    t.tiles = H->tiles;
    t.ntiles = H->ntiles;
    t.tpw = H->tile_tpw;
    t.ntx = H->tile_ntx;
    t.nx = H->d.nx;
    t.ny = H->d.ny;
    t.sy = H->px;
    t.s = H->d.s;
    t.diag = H->diag_p;
    t.diag32 = H->diag_p32;
    t.dinv = H->dinv_p;
    t.dinv32 = H->dinv_p32;
    t.wf = H->wf_on ? H->wf : nullptr;
    t.wf32 = H->wf_on ? H->wf32 : nullptr;
    t.dinv16 = (const bf16*)H->dinv_p16;
    return t;
}

// The 2-D fine level of hierarchies with a coarse level runs on tiles.
static bool use_tiles(const amg_handle* H) {
    return H->ntiles > 0 && H->d.dim == 2 && H->nlev > 1 && !H->beta_on;
}

static BoxArgs box_args(const amg_handle* H) {
    BoxArgs b;
    const Level& L0 = H->lev[0];
    b.boxes = H->boxes0;
    b.nboxes = H->nboxes0;
    b.nbx = L0.nb[0];
    b.nby = L0.nb[1];
    b.nx = H->d.nx;
    b.ny = H->d.ny;
    b.nz = H->d.nz;
    b.cstart = L0.box_cstart;
    b.ncomp = L0.box_ncomp;
    b.agg = H->agg_p;
    b.map = H->box_map0;
    b.w0 = H->box_w0;
    b.w0_32 = H->box_w0_32;
    return b;
}

// FP64 fine restriction without convergence check (learned-smoother paths).
static int launch_fine_restrict64(amg_handle* H, const FineArgs& f, double w0, const double* res, double* rc, int np,
                                  hipStream_t s) {
    const dim3 g(restrict_grid(H));
    const Level& L1 = H->lev[1];
    double* sv1 = H->nlev > 2 ? L1.sv : nullptr;
    if (H->d.dim == 2)
        hipLaunchKernelGGL((k_fine_restrict<double, 2>), g, dim3(RNT), 0, s, f, box_args(H), w0, res, rc,
                           (const double*)L1.diag, L1.omega, sv1, H->sc, 0, H->red.rr, np);
    else
        hipLaunchKernelGGL((k_fine_restrict<double, 3>), g, dim3(RNT), 0, s, f, box_args(H), w0, res, rc,
                           (const double*)L1.diag, L1.omega, sv1, H->sc, 0, H->red.rr, np);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// Arrays of one level, and the fine V-cycle vectors, in the V-cycle precision.
template <class V>
struct LevelView {
    Csr<V> A, P, R;
    const V* diag;
    V* rv;
    V* ev;
    V* tmp;
    V* sv;
    SellV<V> sa, sp, sap;
    Csr<V> RA;
};

template <class V> static LevelView<V> view(const Level& L);
template <> LevelView<double> view<double>(const Level& L) {
    return {{L.a_rowptr, L.a_col, L.a_val}, {L.p_rowptr, L.p_col, L.p_val}, {L.r_rowptr, L.r_col, L.r_val},
            L.diag, L.rv, L.ev, L.tmp, L.sv,
            {L.sa.width, L.sa.col, L.sa.val}, {L.sp.width, L.sp.col, L.sp.val}, {L.sap.width, L.sap.col, L.sap.val},
            {L.ra_rowptr, L.ra_col, L.ra_val}};
}
template <> LevelView<float> view<float>(const Level& L) {
    return {{L.a_rowptr, L.a_col, L.a_val32}, {L.p_rowptr, L.p_col, L.p_val32}, {L.r_rowptr, L.r_col, L.r_val32},
            L.diag32, L.rv32, L.ev32, L.tmp32, L.sv32,
            {L.sa.width, L.sa.col, L.sa.val32}, {L.sp.width, L.sp.col, L.sp.val32},
            {L.sap.width, L.sap.col, L.sap.val32}, {L.ra_rowptr, L.ra_col, L.ra_val32}};
}

template <class V>
struct FineBufs {
    V* res;
    V* zt;
    V* z;
};

template <class V> static FineBufs<V> fine_bufs(const amg_handle* H);
template <> FineBufs<double> fine_bufs<double>(const amg_handle* H) { return {H->res, H->zt, H->z}; }
template <> FineBufs<float> fine_bufs<float>(const amg_handle* H) { return {H->res32, H->zt32, H->z32}; }

static int lanes_for(double avg_row) {
    int l = 4;
    while (l < 32 && l < avg_row * 0.75) l <<= 1;
    return l;
}

#define EB_LPR_LAUNCH(KERNEL, V, lpr, rows, ...)                                                         \
    do {                                                                                                 \
        const unsigned g_ = grid_for((rows) * (int64_t)(lpr), NT);                                      \
        switch (lpr) {                                                                                   \
            case 4: hipLaunchKernelGGL((KERNEL<4, V>), dim3(g_), dim3(NT), 0, s, __VA_ARGS__); break;   \
            case 8: hipLaunchKernelGGL((KERNEL<8, V>), dim3(g_), dim3(NT), 0, s, __VA_ARGS__); break;   \
            case 16: hipLaunchKernelGGL((KERNEL<16, V>), dim3(g_), dim3(NT), 0, s, __VA_ARGS__); break; \
            default: hipLaunchKernelGGL((KERNEL<32, V>), dim3(g_), dim3(NT), 0, s, __VA_ARGS__); break; \
        }                                                                                                \
    } while (0)

// Coarse levels with more unknowns than this take two light passes each way;
// smaller ones (launch bound) take one fused pass that recomputes the residual
// or the prolongated correction at the neighbours.  Going down, the fused
// pass costs about (entries per R row) x (entries per A row) products per
// coarse row in sequence; above FUSE_DOWN_WORK (3-D levels: a few thousand)
// the two passes are faster.
constexpr int64_t FUSE_BELOW = 20000;
constexpr double FUSE_DOWN_WORK = 600.0;

static bool fuse_down(const Level& L, const Level& C) {
    if (L.n >= FUSE_BELOW) return false;
    const double ra = (double)L.nnz_a / (double)(L.n > 0 ? L.n : 1);
    const double rr = (double)L.nnz_r / (double)(C.n > 0 ? C.n : 1);
    return ra * rr <= FUSE_DOWN_WORK;
}

// Coarse part of the V-cycle, levels 1 .. nlev-1: rv_1 -> ev_1.  Going down,
// each level forms its residual after pre-smoothing (sliced ELL, one lane
// per row) and restricts it (CSR, several lanes per long row of R); going up,
// one pass per level prolongates and post-smooths with the stored A P.
template <class V>
static int enqueue_coarse(amg_handle* H, hipStream_t s) {
    const PcgScalars* sc = H->sc;
    for (int l = 1; l < H->nlev - 1; ++l) {
        const Level& L = H->lev[l];
        const Level& C = H->lev[l + 1];
        const LevelView<V> Lv = view<V>(L), Cv = view<V>(C);
        const int lpr_r = lanes_for((double)L.nnz_r / (double)(C.n > 0 ? C.n : 1));
        // omega rv / diag of the coarse level, for its own kernels (none on the coarsest)
        const V wc = (V)C.omega;
        V* svc = l + 1 < H->nlev - 1 ? Cv.sv : nullptr;
        (void)lpr_r;
        const int lpr_d = lanes_for((double)(2 * L.nnz_r) / (double)(C.n > 0 ? C.n : 1));
        {
            const unsigned g_ = xcd_grid(grid_for(C.n * (int64_t)lpr_d, NT));
            const dim3 gd(g_), bd(NT);
            switch (lpr_d) {
                case 4: hipLaunchKernelGGL((k_down_ra<4, V>), gd, bd, 0, s, C.n, Lv.R, Lv.RA, (const V*)Lv.rv,
                                           (const V*)Lv.sv, Cv.rv, (const V*)Cv.diag, wc, svc, sc); break;
                case 8: hipLaunchKernelGGL((k_down_ra<8, V>), gd, bd, 0, s, C.n, Lv.R, Lv.RA, (const V*)Lv.rv,
                                           (const V*)Lv.sv, Cv.rv, (const V*)Cv.diag, wc, svc, sc); break;
                case 16: hipLaunchKernelGGL((k_down_ra<16, V>), gd, bd, 0, s, C.n, Lv.R, Lv.RA, (const V*)Lv.rv,
                                            (const V*)Lv.sv, Cv.rv, (const V*)Cv.diag, wc, svc, sc); break;
                default: hipLaunchKernelGGL((k_down_ra<32, V>), gd, bd, 0, s, C.n, Lv.R, Lv.RA, (const V*)Lv.rv,
                                            (const V*)Lv.sv, Cv.rv, (const V*)Cv.diag, wc, svc, sc); break;
            }
        }
    }
    {
        const Level& Lc = H->lev[H->nlev - 1];
        const LevelView<V> Lcv = view<V>(Lc);
        if (Lc.fz_all)
            hipLaunchKernelGGL(k_block_apply<V>, dim3(grid_for(Lc.n, NT / WAVE)), dim3(NT), 0, s, Lc.n,
                               (const int32_t*)Lc.fz_blk, (const int32_t*)Lc.fz_off, (const int64_t*)Lc.fz_woff,
                               (const double*)Lc.fz_inv, (const V*)Lcv.rv, Lcv.ev, sc);
        else
            hipLaunchKernelGGL(k_dense_apply<V>, dim3(grid_for(Lc.n, NT / WAVE)), dim3(NT), 0, s, Lc.n, Lc.dense_inv,
                               Lcv.rv, Lcv.ev, sc);
    }
    for (int l = H->nlev - 2; l >= 1; --l) {
        const Level& L = H->lev[l];
        const Level& C = H->lev[l + 1];
        const LevelView<V> Lv = view<V>(L), Cv = view<V>(C);
        if (H->d.dim == 2)
            hipLaunchKernelGGL((k_sell_up<V, 4, 9>), dim3(xcd_grid(grid_for(L.n, NT))), dim3(NT), 0, s, L.n, Lv.sa, Lv.sp,
                               Lv.sap, Lv.diag, (V)L.omega, (const V*)Lv.rv, (const V*)Lv.sv, (const V*)Cv.ev, Lv.ev,
                               sc);
        else
            hipLaunchKernelGGL((k_sell_up<V, 8, 14>), dim3(xcd_grid(grid_for(L.n, NT))), dim3(NT), 0, s, L.n, Lv.sa, Lv.sp,
                               Lv.sap, Lv.diag, (V)L.omega, (const V*)Lv.rv, (const V*)Lv.sv, (const V*)Cv.ev, Lv.ev,
                               sc);
        // islands ending on this level: their exact block solve replaces the
        // smoothing-only value the up pass left on their rows
        if (L.nfz > 0)
            hipLaunchKernelGGL(k_block_apply<V>, dim3(grid_for(L.n, NT / WAVE)), dim3(NT), 0, s, L.n,
                               (const int32_t*)L.fz_blk, (const int32_t*)L.fz_off, (const int64_t*)L.fz_woff,
                               (const double*)L.fz_inv, (const V*)Lv.rv, Lv.ev, sc);
    }
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// One-level hierarchy (the fine level is the coarsest): z = W r in FP64.
static int enqueue_vcycle_one_level(amg_handle* H, const double* r, double* z, double* rz_out, int check,
                                    hipStream_t s) {
    PcgScalars* sc = H->sc;
    const int np = H->red.nparts;
    const dim3 G((unsigned)np);
    Level& L = H->lev[0];
    const int64_t n = L.n;
    hipLaunchKernelGGL(k_gather, G, dim3(NT), 0, s, n, H->fine_pad, r, L.rv, sc, check, H->red.rr, np);
    hipLaunchKernelGGL(k_dense_apply<double>, dim3(grid_for(n, NT / WAVE)), dim3(NT), 0, s, n, L.dense_inv, L.rv,
                       L.ev, (const PcgScalars*)sc);
    hipLaunchKernelGGL(k_scatter_dot, G, dim3(NT), 0, s, n, H->fine_pad, L.ev, r, z, rz_out, (const PcgScalars*)sc);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// z = M r for the initial residual (or a standalone V-cycle), hierarchies of
// two or more levels: fine pre-smoothing, restriction, coarse levels,
// prolongation and post-smoothing; the last kernel writes the (r, z)
// partials to rz_out.
// B16: the BF16 smoother (V = float; z is the BF16 copy).
// VB: variable conductivity (strip kernels with face weights; the 2-D tile
// kernels are not used then).
template <class V, bool LW, bool B16 = false, bool VB = false>
static int enqueue_vcycle(amg_handle* H, const double* r, std::conditional_t<B16, bf16, V>* z, double* rz_out,
                          hipStream_t s) {
    PcgScalars* sc = H->sc;
    const int np = H->red.nparts;
    const dim3 G((unsigned)np);
    const FineArgs f = fine_args(H);
    const FineBufs<V> fb = fine_bufs<V>(H);
    const LevelView<V> L1 = view<V>(H->lev[1]);
    const double w0 = H->lev[0].omega;
    if (use_tiles(H)) {
        const TileArgs t = tile_args(H);
        V* sv1 = H->nlev > 2 ? L1.sv : nullptr;
        EB_TIMED_LAUNCH(H, EB_K_FINE_DOWN, s, (k_t2_xr_restrict<V, LW, false>), G, dim3(TNT), 0, t, box_args(H),
                        (double*)nullptr, r, (double*)nullptr, (const double*)nullptr, (const double*)nullptr, w0,
                        (const double*)nullptr, (const double*)nullptr, np, (double*)nullptr, L1.rv,
                        (const V*)L1.diag, H->lev[1].omega, sv1, sc);
        EB_TRY(enqueue_coarse<V>(H, s));
        EB_TIMED_LAUNCH(H, EB_K_FINE_POST, s, (k_t2_up_post<V, LW, B16>), G, dim3(TNT), 0, t, w0,
                        (const int32_t*)H->agg_p, (const V*)L1.ev, r, z, rz_out, (const double*)nullptr, np, sc);
        EB_LAUNCH_CHECK();
        return EB_OK;
    }
    EB_TIMED_LAUNCH(H, EB_K_FINE_DOWN, s, (k_fine_down<V, LW, VB>), G, dim3(NT), 0, f, w0, r, fb.res, sc, 0,
                    H->red.rr, np);
    if (H->d.dim == 2)
        EB_TIMED_LAUNCH(H, EB_K_FINE_RESTRICT, s, (k_fine_restrict<V, 2, VB>), dim3(xcd_grid(H->nboxes0, RNT)),
                        dim3(RNT), 0, f, box_args(H), w0, fb.res, L1.rv, (const V*)L1.diag,
                        H->lev[1].omega, H->nlev > 2 ? L1.sv : nullptr, sc, 0, H->red.rr, np);
    else
        EB_TIMED_LAUNCH(H, EB_K_FINE_RESTRICT, s, (k_fine_restrict<V, 3, VB>), dim3(restrict_grid(H)),
                        dim3(RNT), 0, f, box_args(H), w0, fb.res, L1.rv, (const V*)L1.diag,
                        H->lev[1].omega, H->nlev > 2 ? L1.sv : nullptr, sc, 0, H->red.rr, np);
    EB_TRY(enqueue_coarse<V>(H, s));
    unsigned gu = 0;
    const FineArgs fu = fine_args_full(H, &gu);
    EB_TIMED_LAUNCH(H, EB_K_FINE_UP, s, (k_fine_up<V, LW, VB>), dim3(gu), dim3(NT), 0, fu, w0, H->agg_p, L1.ev, r,
                    fb.zt, (const PcgScalars*)sc);
    EB_TIMED_LAUNCH(H, EB_K_FINE_POST, s, (k_fine_post<V, LW, B16, VB>), G, dim3(NT), 0, f, w0, fb.zt, r, z, rz_out,
                    (const PcgScalars*)sc);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// Iteration k >= 1 of a run.  The V-cycle before it (number k-1) wrote
// rz[(k-1) % 2] from r[(k-1) % 2]; this iteration reads r[(k-1) % 2], writes
// r[k % 2] and its V-cycle writes rz[k % 2].
template <class V, bool LW, bool B16 = false, bool VB = false>
static int enqueue_iteration(amg_handle* H, int k, hipStream_t s) {
    const FineArgs f = fine_args(H);
    const int np = H->red.nparts;
    const dim3 G((unsigned)np);
    const FineBufs<V> fb = fine_bufs<V>(H);
    using ZT = std::conditional_t<B16, bf16, V>;
    ZT* zb;
    if constexpr (B16) zb = (bf16*)H->z16;
    else zb = fb.z;
    double* pold = H->p[k & 1];
    double* pnew = H->p[(k + 1) & 1];
    double* rin = H->rr[(k - 1) & 1];
    double* rout = H->rr[k & 1];
    const double* rz_cur = H->red.rz[(k - 1) & 1];
    const double* rz_prev = k >= 2 ? H->red.rz[k & 1] : nullptr;
    double* rz_out = H->red.rz[k & 1];
    PcgScalars* sc = H->sc;
    const double w0 = H->lev[0].omega;
    const LevelView<V> L1 = view<V>(H->lev[1]);
    if (use_tiles(H)) {
        const TileArgs t = tile_args(H);
        V* sv1 = H->nlev > 2 ? L1.sv : nullptr;
        EB_TIMED_LAUNCH(H, EB_K_PCG_SPMV, s, k_t2_pspmv<ZT>, G, dim3(TNT), 0, t, (const ZT*)zb, (const double*)pold,
                        pnew, H->q, rz_cur, rz_prev, np, H->red.pq, sc);
        EB_TIMED_LAUNCH(H, EB_K_PCG_XR, s, (k_t2_xr_restrict<V, LW, true>), G, dim3(TNT), 0, t, box_args(H), H->x,
                        (const double*)rin, rout, (const double*)pnew, (const double*)H->q, w0, rz_cur,
                        (const double*)H->red.pq, np, H->red.rr, L1.rv, (const V*)L1.diag, H->lev[1].omega, sv1,
                        sc);
        EB_TRY(enqueue_coarse<V>(H, s));
        EB_TIMED_LAUNCH(H, EB_K_FINE_POST, s, (k_t2_up_post<V, LW, B16>), G, dim3(TNT), 0, t, w0,
                        (const int32_t*)H->agg_p, (const V*)L1.ev, (const double*)rout, zb, rz_out,
                        (const double*)H->red.rr, np, sc);
        EB_LAUNCH_CHECK();
        return EB_OK;
    }
    EB_TIMED_LAUNCH(H, EB_K_PCG_SPMV, s, (k_pcg_p_spmv<ZT, VB>), G, dim3(NT), 0, f, (const ZT*)zb, pold, pnew, H->q,
                    rz_cur, rz_prev, np, H->red.pq, sc);
    EB_TIMED_LAUNCH(H, EB_K_PCG_XR, s, (k_pcg_xr_down<V, LW, VB>), G, dim3(NT), 0, f, H->x, rin, rout, pnew, H->q, fb.res,
                    w0, rz_cur, H->red.pq, np, H->red.rr, sc);
    if (H->d.dim == 2)
        EB_TIMED_LAUNCH(H, EB_K_FINE_RESTRICT, s, (k_fine_restrict<V, 2, VB>), dim3(xcd_grid(H->nboxes0, RNT)),
                        dim3(RNT), 0, f, box_args(H), w0, fb.res, L1.rv, (const V*)L1.diag,
                        H->lev[1].omega, H->nlev > 2 ? L1.sv : nullptr, sc, 1, H->red.rr, np);
    else
        EB_TIMED_LAUNCH(H, EB_K_FINE_RESTRICT, s, (k_fine_restrict<V, 3, VB>), dim3(restrict_grid(H)),
                        dim3(RNT), 0, f, box_args(H), w0, fb.res, L1.rv, (const V*)L1.diag,
                        H->lev[1].omega, H->nlev > 2 ? L1.sv : nullptr, sc, 1, H->red.rr, np);
    EB_TRY(enqueue_coarse<V>(H, s));
    unsigned gu = 0;
    const FineArgs fu = fine_args_full(H, &gu);
    EB_TIMED_LAUNCH(H, EB_K_FINE_UP, s, (k_fine_up<V, LW, VB>), dim3(gu), dim3(NT), 0, fu, w0, H->agg_p, L1.ev, rout,
                    fb.zt, (const PcgScalars*)sc);
    EB_TIMED_LAUNCH(H, EB_K_FINE_POST, s, (k_fine_post<V, LW, B16, VB>), G, dim3(NT), 0, f, w0, fb.zt, rout, zb, rz_out,
                    (const PcgScalars*)sc);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// The same for a one-level hierarchy (FP64 dense solve of the fine level).
static int enqueue_iteration_one_level(amg_handle* H, int k, hipStream_t s) {
    const FineArgs f = fine_args(H);
    const int np = H->red.nparts;
    const dim3 G((unsigned)np);
    double* pold = H->p[k & 1];
    double* pnew = H->p[(k + 1) & 1];
    double* rin = H->rr[(k - 1) & 1];
    double* rout = H->rr[k & 1];
    const double* rz_cur = H->red.rz[(k - 1) & 1];
    const double* rz_prev = k >= 2 ? H->red.rz[k & 1] : nullptr;
    double* rz_out = H->red.rz[k & 1];
    PcgScalars* sc = H->sc;
    if (H->beta_on)
        EB_TIMED_LAUNCH(H, EB_K_PCG_SPMV, s, (k_pcg_p_spmv<double, true>), G, dim3(NT), 0, f, H->z, pold, pnew, H->q,
                        rz_cur, rz_prev, np, H->red.pq, sc);
    else
        EB_TIMED_LAUNCH(H, EB_K_PCG_SPMV, s, k_pcg_p_spmv<double>, G, dim3(NT), 0, f, H->z, pold, pnew, H->q, rz_cur,
                        rz_prev, np, H->red.pq, sc);
    EB_TIMED_LAUNCH(H, EB_K_PCG_XR, s, k_pcg_xr, G, dim3(NT), 0, f, H->x, rin, pnew, H->q, rz_cur, H->red.pq, np,
                    H->red.rr, sc);
    // k_pcg_xr updates r in place: keep both buffers equal
    hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(H->npad, NT)), dim3(NT), 0, s, H->npad, rin, rout);
    EB_LAUNCH_CHECK();
    return enqueue_vcycle_one_level(H, rout, H->z, rz_out, 1, s);
}

// V-cycle / iteration with or without the per-point smoother weights.
// (the BF16 smoother takes no per-point weights: refused before this point)
// (variable conductivity likewise: refused with per-point weights or BF16)
template <class V, bool B16 = false>
static int enqueue_vcycle_any(amg_handle* H, const double* r, std::conditional_t<B16, bf16, V>* z, double* rz_out,
                              hipStream_t s) {
    if constexpr (B16) return enqueue_vcycle<V, false, true>(H, r, z, rz_out, s);
    else {
        if (H->beta_on) return enqueue_vcycle<V, false, false, true>(H, r, z, rz_out, s);
        return H->wf_on ? enqueue_vcycle<V, true>(H, r, z, rz_out, s) : enqueue_vcycle<V, false>(H, r, z, rz_out, s);
    }
}

template <class V, bool B16 = false>
static int enqueue_iteration_any(amg_handle* H, int k, hipStream_t s) {
    if constexpr (B16) return enqueue_iteration<V, false, true>(H, k, s);
    else {
        if (H->beta_on) return enqueue_iteration<V, false, false, true>(H, k, s);
        return H->wf_on ? enqueue_iteration<V, true>(H, k, s) : enqueue_iteration<V, false>(H, k, s);
    }
}

// True residual out = b - A x with its partials.
static void launch_resid(amg_handle* H, const FineArgs& f, unsigned np, double* out, double* part, hipStream_t s) {
    if (H->beta_on)
        hipLaunchKernelGGL(k_fine_resid<true>, dim3(np), dim3(NT), 0, s, f, H->bvec, H->x, out, part);
    else
        hipLaunchKernelGGL(k_fine_resid<false>, dim3(np), dim3(NT), 0, s, f, H->bvec, H->x, out, part);
}

// Steady-state iterations as a HIP graph.  From iteration 3 on, iterations
// k and k + 2 launch the same kernels with the same arguments (buffers
// alternate with the parity of k, the iteration count lives on the device),
// so one captured pair (k odd, k + 1) is replayed for every later pair; the
// host then submits one graph per two iterations instead of about twenty
// kernels.  The graph holds kernel nodes only (no memset or copy nodes) and
// is kept on the handle, per V-cycle precision and fine-weight switch.
static std::atomic<int> g_use_graphs{1};

bool iteration_graphs_enabled() { return g_use_graphs.load() != 0; }

void drop_iteration_graphs(amg_handle* H) {
    for (int i = 0; i < 3; ++i) {
        if (H->it_graph[i]) (void)hipGraphExecDestroy(H->it_graph[i]);
        H->it_graph[i] = nullptr;
        H->it_graph_wf[i] = -1;
    }
    if (H->cap_stream) (void)hipStreamDestroy(H->cap_stream);
    H->cap_stream = nullptr;
}

template <class V, bool B16 = false>
static int launch_iteration_pair(amg_handle* H, hipStream_t s) {
    const int slot = B16 ? 2 : sizeof(V) == sizeof(float) ? 1 : 0;
    if (!H->it_graph[slot] || H->it_graph_wf[slot] != H->wf_on) {
        if (H->it_graph[slot]) (void)hipGraphExecDestroy(H->it_graph[slot]);
        H->it_graph[slot] = nullptr;
        // captured on a private stream (the solve stream may be the null
        // stream, which cannot capture); nothing runs during capture
        if (!H->cap_stream) EB_HIP(hipStreamCreateWithFlags(&H->cap_stream, hipStreamNonBlocking));
        hipStream_t cs = H->cap_stream;
        hipGraph_t g = nullptr;
        EB_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        const int rc1 = enqueue_iteration_any<V, B16>(H, 3, cs);
        const int rc2 = rc1 == EB_OK ? enqueue_iteration_any<V, B16>(H, 4, cs) : rc1;
        const hipError_t ec = hipStreamEndCapture(cs, &g);
        if (rc2 != EB_OK || ec != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            if (rc2 != EB_OK) return rc2;
            set_error("iteration graph capture failed: %s", hipGetErrorString(ec));
            return EB_EHIP;
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            set_error("iteration graph instantiation failed: %s", hipGetErrorString(ei));
            return EB_EHIP;
        }
        H->it_graph[slot] = ex;
        H->it_graph_wf[slot] = H->wf_on;
    }
    EB_HIP(hipGraphLaunch(H->it_graph[slot], s));
    return EB_OK;
}

// FP32 copies of the hierarchy for the single-precision V-cycle, made once
// per handle on first use.
__global__ void __launch_bounds__(NT) k_to_f32(int64_t n, const double* __restrict__ src, float* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}

static int copy_to_f32(const double* src, int64_t n, float** dst, hipStream_t s) {
    EB_TRY(dalloc_n(dst, n, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n, NT)), dim3(NT), 0, s, n, src, *dst);
        EB_LAUNCH_CHECK();
    }
    return EB_OK;
}

int ensure_fp32(amg_handle* H, hipStream_t s) {
    if (H->fp32_ready) return EB_OK;
    EB_TRY(copy_to_f32(H->diag_p, H->npad, &H->diag_p32, s));
    EB_TRY(copy_to_f32(H->dinv_p, H->npad, &H->dinv_p32, s));
    if (H->box_w0) EB_TRY(copy_to_f32(H->box_w0, (int64_t)H->lev[0].nb[0] * H->lev[0].nb[1], &H->box_w0_32, s));
    EB_TRY(dalloc_n(&H->res32, H->npad, s));
    EB_TRY(dalloc_n(&H->zt32, H->npad, s));
    EB_TRY(dalloc_n(&H->z32, H->npad, s));
    {
        const FillSpec f[] = {{H->zt32, sizeof(float) * H->npad, 0u}, {H->z32, sizeof(float) * H->npad, 0u}};
        EB_TRY(fill_words(f, 2, s));
    }
    for (int l = 1; l < H->nlev; ++l) {
        Level& L = H->lev[l];
        const int64_t n = L.n > 0 ? L.n : 1;
        if (!L.is_coarsest) {
            EB_TRY(copy_to_f32(L.a_val, L.nnz_a, &L.a_val32, s));
            EB_TRY(copy_to_f32(L.diag, L.n, &L.diag32, s));
            EB_TRY(copy_to_f32(L.p_val, L.nnz_p, &L.p_val32, s));
            EB_TRY(copy_to_f32(L.r_val, L.nnz_r, &L.r_val32, s));
            for (Sell* m : {&L.sa, &L.sp, &L.sap})
                if (m->val) EB_TRY(copy_to_f32(m->val, m->cap, &m->val32, s));
            if (L.ra_val) EB_TRY(copy_to_f32(L.ra_val, L.ra_cap, &L.ra_val32, s));
        }
        EB_TRY(dalloc_n(&L.rv32, n, s));
        EB_TRY(dalloc_n(&L.sv32, n, s));
        EB_TRY(dalloc_n(&L.ev32, n, s));
        EB_TRY(dalloc_n(&L.tmp32, n, s));
    }
    H->fp32_ready = 1;
    return EB_OK;
}

// BF16 copies for the BF16 smoother: 1 / d (from the FP64 field, rounded
// once to FP32 and then to BF16) and the z buffer; made once per handle.
__global__ void __launch_bounds__(NT) k_to_bf16(int64_t n, const double* __restrict__ src, bf16* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) dst[i] = f32_to_bf16((float)src[i]);
}

int ensure_bf16(amg_handle* H, hipStream_t s) {
    if (H->bf16_ready) return EB_OK;
    EB_TRY(dalloc(&H->dinv_p16, sizeof(bf16) * (size_t)H->npad, s));
    EB_TRY(dalloc(&H->z16, sizeof(bf16) * (size_t)H->npad, s));
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(H->npad, NT)), dim3(NT), 0, s, H->npad, H->dinv_p,
                       (bf16*)H->dinv_p16);
    EB_LAUNCH_CHECK();
    {
        // npad is a multiple of 64 nodes: whole 32-bit words
        const FillSpec f[] = {{H->z16, sizeof(bf16) * (size_t)H->npad, 0u}};
        EB_TRY(fill_words(f, 1, s));
    }
    H->bf16_ready = 1;
    return EB_OK;
}

// b, x0 -> r0 = b - A x0; ||b||^2, ||r0||^2, tolerance, initial convergence test.
static int enqueue_init(amg_handle* H, double tol, int iters, hipStream_t s) {
    const FineArgs f = fine_args(H);
    const int np = H->red.nparts;
    const dim3 G((unsigned)np);
    hipLaunchKernelGGL(k_fine_norm2, G, dim3(NT), 0, s, f, H->bvec, H->red.aux);
    launch_resid(H, f, (unsigned)np, H->rr[0], H->red.rr, s);
    hipLaunchKernelGGL(k_finalize_init, dim3(1), dim3(NT), 0, s, H->sc, H->red.aux, H->red.rr, np, tol, iters);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// The same for a zero initial guess, b read from the caller's field: one
// kernel in place of the load of b, the clear of x and both reductions.
static int enqueue_init_zero_guess(amg_handle* H, const double* b, int64_t nunk, double tol, hipStream_t s) {
    const int np = H->red.nparts;
    hipLaunchKernelGGL(k_init_zero_guess, dim3((unsigned)np), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, b,
                       H->bvec, H->x, H->rr[0], H->red.aux);
    hipLaunchKernelGGL(k_finalize_init, dim3(1), dim3(NT), 0, s, H->sc, H->red.aux, H->red.aux, np, tol, 0);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// Fine solve layout, part 1 (no synchronisation): padded fields, active
// strip and box lists sized by their bounds, vectors and partial buffers.
int solve_layout_alloc(amg_handle* H, hipStream_t s) {
    const GridDims& d = H->d;
    H->px = (d.nx + 63) / 64 * 64;
    H->npad = (int64_t)H->px * d.ny * d.nz;
    H->strip_w = d.dim == 2 ? 64 : 32;
    const int64_t npad = H->npad;
    const int64_t nunk = H->n_fine;
    EB_TRY(dalloc_n(&H->dcount, 3, s));
    EB_TRY(dalloc_n(&H->fine_pad, nunk, s));
    EB_TRY(dalloc_n(&H->diag_p, npad, s));
    EB_TRY(dalloc_n(&H->dinv_p, npad, s));
    EB_TRY(dalloc_n(&H->agg_p, npad, s));
    const int64_t nstrip_all = npad / H->strip_w;
    int32_t* sflag = nullptr;
    EB_TRY(dalloc_n(&sflag, nstrip_all, s));
    // 2-D: tiles of the tile kernels (their origins are multiples of 3, so
    // a tile holds whole level-0 boxes)
    // (the tile kernels address padded fields by 32-bit byte offsets)
    const bool tiled = d.dim == 2 && H->nlev > 1 && npad < ((int64_t)1 << 29) && !H->beta_on;
    H->tile_ntx = tiled ? (d.nx + TX - 1) / TX : 0;
    const int64_t ntile_all = tiled ? (int64_t)H->tile_ntx * ((d.ny + TY - 1) / TY) : 0;
    int32_t* tflag = nullptr;
    if (tiled) EB_TRY(dalloc_n(&tflag, ntile_all, s));
    // Fields read at neighbours without a guard must be zero off unknowns
    // (kernels only ever write unknowns); the others are fully written first
    // or read only where the diagonal is non-zero.
    // The residuals and q are among them: the per-point smoother weights
    // multiply neighbour values by a weight that is 0 off unknowns, and a
    // recycled block could hold NaN there (0 * NaN = NaN).
    double** zeroed[] = {&H->x, &H->z, &H->zt, &H->p[0], &H->p[1], &H->rr[0], &H->rr[1], &H->q};
    for (double** v : zeroed) EB_TRY(dalloc_n(v, npad, s));
    {
        const FillSpec f[] = {{H->dcount, 3 * sizeof(int32_t), 0u},
                              {H->diag_p, sizeof(double) * npad, 0u},
                              {H->agg_p, sizeof(int32_t) * npad, 0xffffffffu},    // -1
                              {sflag, sizeof(int32_t) * nstrip_all, 0u},
                              {H->x, sizeof(double) * npad, 0u},
                              {H->z, sizeof(double) * npad, 0u},
                              {H->zt, sizeof(double) * npad, 0u},
                              {H->p[0], sizeof(double) * npad, 0u},
                              {H->p[1], sizeof(double) * npad, 0u},
                              {H->rr[0], sizeof(double) * npad, 0u},
                              {H->rr[1], sizeof(double) * npad, 0u},
                              {H->q, sizeof(double) * npad, 0u}};
        EB_TRY(fill_words(f, 12, s));
        const FillSpec ft[] = {{H->dinv_p, sizeof(double) * npad, 0u},
                               {tflag, sizeof(int32_t) * ntile_all, 0u}};
        EB_TRY(fill_words(ft, tiled ? 2 : 1, s));
    }
    if (H->beta_on) {
        // the caller's face conductivities in the padded layout (every node,
        // so that the faces toward non-unknown neighbours are finite)
        const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
        for (int a = 0; a < d.dim; ++a) {
            EB_TRY(dalloc_n(&H->bf_p[a], npad, s));
            const FillSpec fb[] = {{H->bf_p[a], sizeof(double) * npad, 0u}};
            EB_TRY(fill_words(fb, 1, s));
            hipLaunchKernelGGL(k_pad_field, dim3(grid_for(nn)), dim3(BLOCK), 0, s, nn, d, H->px,
                               H->beta_tmp + (int64_t)a * nn, H->bf_p[a]);
        }
        EB_LAUNCH_CHECK();
    }
    Level& L0 = H->lev[0];
    hipLaunchKernelGGL(k_fine_layout, dim3(grid_for(nunk)), dim3(BLOCK), 0, s, H->fine_nodes, nunk, d, H->px, L0.diag,
                       L0.agg, L0.agg != nullptr ? 1 : 0, H->fine_pad, H->diag_p, H->dinv_p, H->agg_p, sflag,
                       H->strip_w, tflag, H->tile_ntx);
    EB_LAUNCH_CHECK();
    if (tiled) {
        const Level& B0 = H->lev[0];
        const int64_t nb = (int64_t)B0.nb[0] * B0.nb[1];
        EB_TRY(dalloc_n(&H->box_map0, nb, s));
        EB_TRY(dalloc_n(&H->box_w0, nb, s));
        hipLaunchKernelGGL(k_box_map2, dim3(grid_for(nb)), dim3(BLOCK), 0, s, B0.nb[0], B0.nb[1], d.nx, d.ny, H->px,
                           (const int32_t*)B0.box_cstart, (const int32_t*)H->agg_p, H->box_map0);
        hipLaunchKernelGGL(k_box_w0, dim3(grid_for(nb)), dim3(BLOCK), 0, s, nb, (const int32_t*)B0.box_cstart,
                           (const int32_t*)B0.box_ncomp, (const double*)H->lev[1].diag, (const double*)H->dscal,
                           H->box_w0);
        EB_LAUNCH_CHECK();
        int32_t* off = nullptr;
        EB_TRY(dalloc_n(&off, ntile_all, s));
        EB_TRY(scan_i32_dev(tflag, off, ntile_all, H->dcount + 2, s));
        EB_TRY(dalloc_n(&H->tiles, ntile_all, s));
        hipLaunchKernelGGL(k_compact_list, dim3(grid_for(ntile_all)), dim3(BLOCK), 0, s, tflag, off, ntile_all,
                           H->tiles);
        EB_LAUNCH_CHECK();
        EB_TRY(dfree(off, s));
        EB_TRY(dfree(tflag, s));
    }
    {
        int32_t* off = nullptr;
        EB_TRY(dalloc_n(&off, nstrip_all, s));
        EB_TRY(scan_i32_dev(sflag, off, nstrip_all, H->dcount + 0, s));
        EB_TRY(dalloc_n(&H->strips, nstrip_all, s));
        hipLaunchKernelGGL(k_compact_list, dim3(grid_for(nstrip_all)), dim3(BLOCK), 0, s, sflag, off, nstrip_all,
                           H->strips);
        EB_LAUNCH_CHECK();
        EB_TRY(dfree(off, s));
    }
    EB_TRY(dfree(sflag, s));
    if (H->nlev > 1) {
        const int64_t nb = L0.nboxes;
        int32_t* bflag = nullptr;
        int32_t* off = nullptr;
        EB_TRY(dalloc_n(&bflag, nb, s));
        EB_TRY(dalloc_n(&off, nb, s));
        hipLaunchKernelGGL(k_flag_nonzero, dim3(grid_for(nb)), dim3(BLOCK), 0, s, L0.box_ncomp, nb, bflag);
        EB_TRY(scan_i32_dev(bflag, off, nb, H->dcount + 1, s));
        EB_TRY(dalloc_n(&H->boxes0, nb, s));
        hipLaunchKernelGGL(k_compact_list, dim3(grid_for(nb)), dim3(BLOCK), 0, s, bflag, off, nb, H->boxes0);
        EB_LAUNCH_CHECK();
        EB_TRY(dfree(bflag, s));
        EB_TRY(dfree(off, s));
        if (L0.max_comp > MAX_FINE_COMP) {
            set_error("a fine-level box holds %d aggregates (limit %d)", L0.max_comp, MAX_FINE_COMP);
            return EB_ENOSPC;
        }
    }
    double** plain[] = {&H->res, &H->bvec};
    for (double** v : plain) EB_TRY(dalloc_n(v, npad, s));
    for (int l = 0; l < H->nlev; ++l) {
        Level& L = H->lev[l];
        if (l == 0 && H->nlev > 1) continue;
        const int64_t n = L.n > 0 ? L.n : 1;
        EB_TRY(dalloc_n(&L.rv, n, s));
        EB_TRY(dalloc_n(&L.sv, n, s));
        EB_TRY(dalloc_n(&L.ev, n, s));
        EB_TRY(dalloc_n(&L.tmp, n, s));
    }
    EB_TRY(dalloc_n(&H->sc, 1, s));
    H->sc_host = &H->sc_mirror;   // pageable, per handle (polled a few times per solve)
    double** parts[] = {&H->red.pq, &H->red.rr, &H->red.rz[0], &H->red.rz[1], &H->red.aux, &H->red.aux2};
    for (double** v : parts) EB_TRY(dalloc_n(v, PART_CAP, s));
    EB_HIP(hipEventCreate(&H->ev0));
    EB_HIP(hipEventCreate(&H->ev1));
    return EB_OK;
}

// Part 2, after the device totals have been read back (dcount copied into
// H->nstrips / H->nboxes0 by the caller's single synchronisation).
int solve_layout_finish(amg_handle* H, hipStream_t s) {
    (void)s;
    int64_t np;
    if (H->ntiles > 0) {
        // the tile kernels' fixed grid: TWB wavefronts per block, each a
        // contiguous range of tile_tpw tiles; the strip kernels share the
        // same partial count
        const int64_t tpw = (H->ntiles + (int64_t)TWB * MAX_TILE_PARTS - 1) / ((int64_t)TWB * MAX_TILE_PARTS);
        H->tile_tpw = (int)tpw;
        np = (H->ntiles + tpw * TWB - 1) / (tpw * TWB);
    } else {
        const int64_t nthreads = H->nlev == 1 ? H->n_fine : H->nstrips * H->strip_w;
        np = (nthreads + NT - 1) / NT;
        if (np > MAX_PARTS) np = MAX_PARTS;
    }
    np = (np + NUM_XCD - 1) / NUM_XCD * NUM_XCD;   // whole XCD groups
    if (np < NUM_XCD) np = NUM_XCD;
    H->red.nparts = (int)np;
    return EB_OK;
}

static int poll_scalars(amg_handle* H, hipStream_t s) {
    EB_HIP(hipMemcpyAsync(H->sc_host, H->sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
    EB_HIP(hipStreamSynchronize(s));
    if (H->tim_used > 0) EB_TRY(timing_harvest(H));
    return EB_OK;
}

// ------------------------------------------------- learned smoother weights
// Per-point fine smoother weights and the training quantities of the learned
// smoother (the network itself is in learned.hip).  Loss for error samples e:
// L = mean (e'^T A e') / (2 e^T A e), e' = e - M A e, M the V(1,1) cycle with
// W = diag(omega_k / d_k) on the fine level.  With r = A e, z1 = W r,
// z2 = z1 + P E_c R (r - A z1), t2 = r - A z2, z = z2 + W t2:
//   g = -A e' / (e^T A e),  u = g - A (W g),  v = u - A P E_c R u,
//   dL/dW = g t2 + v r  (A and E_c symmetric, R = P^T).

__global__ void __launch_bounds__(BLOCK) k_set_wf(int64_t n, const int64_t* __restrict__ nodes,
                                                  const int32_t* __restrict__ pad, const double* __restrict__ diag_p,
                                                  const double* __restrict__ om, double* __restrict__ wf,
                                                  float* __restrict__ wf32, int32_t* __restrict__ bad) {
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= n) return;
    const int32_t p = pad[k];
    const double o = om[nodes[k]];
    if (!(o > 0.0) || isinf(o)) atomicOr(bad, 1);
    const double w = o / diag_p[p];
    wf[p] = w;
    wf32[p] = (float)w;
}

// y = A x on the padded fine layout (0 off unknowns).
__global__ void __launch_bounds__(NT) k_lg_apply(FineArgs f, const double* __restrict__ x, double* __restrict__ y) {
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) y[p] = d * x[p] - f.s * nbr_sum(x, p, f);
    }
}

// partial sums of a . b
__global__ void __launch_bounds__(NT) k_lg_dot(FineArgs f, const double* __restrict__ a, const double* __restrict__ b,
                                               double* __restrict__ part) {
    double acc = 0.0;
    FINE_LOOP(f, p) {
        if (f.diag[p] != 0.0) acc += a[p] * b[p];
    }
    block_partial(acc, part);
}

// e = (e - z) / ||e - z||, the norm from the partials of (e - z, e - z) taken
// by k_lg_diffnorm.
__global__ void __launch_bounds__(NT) k_lg_diffnorm(FineArgs f, const double* __restrict__ e,
                                                    const double* __restrict__ z, double* __restrict__ part) {
    double acc = 0.0;
    FINE_LOOP(f, p) {
        if (f.diag[p] != 0.0) {
            const double t = e[p] - z[p];
            acc += t * t;
        }
    }
    block_partial(acc, part);
}

__global__ void __launch_bounds__(NT) k_lg_diffscale(FineArgs f, double* __restrict__ e, const double* __restrict__ z,
                                                     const double* __restrict__ part, int np) {
    const double nrm = sqrt(block_total(part, np));
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    FINE_LOOP(f, p) {
        if (f.diag[p] != 0.0) e[p] = (e[p] - z[p]) * inv;
    }
}

// From z2 (the prolongated pre-smoothed iterate) and r: t2 = r - A z2,
// e' = e - (z2 + W t2).
__global__ void __launch_bounds__(NT) k_lg_post(FineArgs f, const double* __restrict__ e, const double* __restrict__ r,
                                                const double* __restrict__ z2, double omega,
                                                double* __restrict__ t2, double* __restrict__ ep) {
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double tt = r[p] - (d * z2[p] - f.s * nbr_sum(z2, p, f));
            const double w = f.wf ? f.wf[p] : omega / d;
            t2[p] = tt;
            ep[p] = e[p] - (z2[p] + w * tt);
        }
    }
}

// g = -(A e') / (e^T A e) and wg = W g; the denominator from its partials.
__global__ void __launch_bounds__(NT) k_lg_g(FineArgs f, const double* __restrict__ aep,
                                             const double* __restrict__ part_den, int np, double omega,
                                             double* __restrict__ g, double* __restrict__ wg) {
    const double den = block_total(part_den, np);
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double gg = -aep[p] / den;
            g[p] = gg;
            wg[p] = (f.wf ? f.wf[p] : omega / d) * gg;
        }
    }
}

// u = g - A wg
__global__ void __launch_bounds__(NT) k_lg_u(FineArgs f, const double* __restrict__ g, const double* __restrict__ wg,
                                             double* __restrict__ u) {
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) u[p] = g[p] - (d * wg[p] - f.s * nbr_sum(wg, p, f));
    }
}

// Prolongation only: y = P e_c = t - omega (A t) / d, t = e_c[agg].
__global__ void __launch_bounds__(NT) k_lg_prolong(FineArgs f, double omega, const int32_t* __restrict__ agg,
                                                   const double* __restrict__ ec, double* __restrict__ y) {
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double tp = corr_at(agg, ec, p);
            double nb = corr_at(agg, ec, p - 1) + corr_at(agg, ec, p + 1);
            nb += corr_at(agg, ec, p - f.sy) + corr_at(agg, ec, p + f.sy);
            if (f.dim == 3) nb += corr_at(agg, ec, p - f.sz) + corr_at(agg, ec, p + f.sz);
            y[p] = tp - omega * (d * tp - f.s * nb) / d;
        }
    }
}

// gw += g t2 + (u - A pe) r
__global__ void __launch_bounds__(NT) k_lg_acc(FineArgs f, const double* __restrict__ g, const double* __restrict__ t2,
                                               const double* __restrict__ u, const double* __restrict__ pe,
                                               const double* __restrict__ r, double* __restrict__ gw) {
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double v = u[p] - (d * pe[p] - f.s * nbr_sum(pe, p, f));
            gw[p] += g[p] * t2[p] + v * r[p];
        }
    }
}

// loss += (e'^T A e') / (2 e^T A e)   (one block)
__global__ void __launch_bounds__(NT) k_lg_loss(const double* __restrict__ part_num, const double* __restrict__ part_den,
                                                int np, double* __restrict__ loss) {
    const double num = block_total(part_num, np);
    const double den = block_total(part_den, np);
    if (threadIdx.x == 0) loss[0] += 0.5 * num / den;
}

// dL/domega at the nodes: gw / d / m.
__global__ void __launch_bounds__(NT) k_lg_store_grad(int64_t n, const int64_t* __restrict__ nodes,
                                                      const int32_t* __restrict__ pad, const double* __restrict__ gw,
                                                      const double* __restrict__ diag_p, double inv_m,
                                                      double* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (k >= n) return;
    const int32_t p = pad[k];
    out[nodes[k]] = gw[p] / diag_p[p] * inv_m;
}

// fine pre-smoothing, restriction, coarse cycle, prolongation: z2 from r.
static int lg_cycle_to_z2(amg_handle* H, const double* r, hipStream_t s) {
    const FineArgs f = fine_args(H);
    const int np = H->red.nparts;
    const double w0 = H->lev[0].omega;
    if (H->wf_on)
        hipLaunchKernelGGL((k_fine_down<double, true>), dim3(np), dim3(NT), 0, s, f, w0, r, H->res, H->sc, 0,
                           H->red.rr, np);
    else
        hipLaunchKernelGGL((k_fine_down<double, false>), dim3(np), dim3(NT), 0, s, f, w0, r, H->res, H->sc, 0,
                           H->red.rr, np);
    EB_TRY(launch_fine_restrict64(H, f, w0, (const double*)H->res, H->lev[1].rv, np, s));
    EB_TRY(enqueue_coarse<double>(H, s));
    unsigned gu = 0;
    const FineArgs fu = fine_args_full(H, &gu);
    if (H->wf_on)
        hipLaunchKernelGGL((k_fine_up<double, true>), dim3(gu), dim3(NT), 0, s, fu, w0, H->agg_p,
                           (const double*)H->lev[1].ev, r, H->zt, (const PcgScalars*)H->sc);
    else
        hipLaunchKernelGGL((k_fine_up<double, false>), dim3(gu), dim3(NT), 0, s, fu, w0, H->agg_p,
                           (const double*)H->lev[1].ev, r, H->zt, (const PcgScalars*)H->sc);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

static int lg_check(amg_handle* H, const char* name) {
    if (H->nlev < 2) {
        set_error("%s: the hierarchy has a single level (no fine smoother)", name);
        return EB_EINVAL;
    }
    if (H->beta_on) {
        set_error("%s: the learned smoother is not available with variable conductivity", name);
        return EB_ENOTIMPL;
    }
    return EB_OK;
}

}  // namespace eb

using namespace eb;

extern "C" int amg_set_fine_weights(amg_handle_t* H, const double* omega, void* stream) {
    clear_error();
    AllocScope scope(H ? &H->params : nullptr);
    if (!H || !omega) {
        set_error("amg_set_fine_weights: null pointer");
        return EB_EINVAL;
    }
    if (H->beta_on) {
        set_error("amg_set_fine_weights: per-point weights are not available with variable conductivity");
        return EB_ENOTIMPL;
    }
    hipStream_t s = stream ? (hipStream_t)stream : H->stream;
    H->last_stream = s;
    if (!H->wf) {
        EB_TRY(dalloc_n(&H->wf, H->npad, s));
        EB_TRY(dalloc_n(&H->wf32, H->npad, s));
        EB_HIP(hipMemsetAsync(H->wf, 0, sizeof(double) * H->npad, s));
        EB_HIP(hipMemsetAsync(H->wf32, 0, sizeof(float) * H->npad, s));
    }
    int32_t* bad = nullptr;
    EB_TRY(dalloc_n(&bad, 1, s));
    EB_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
    if (H->n_fine > 0)
        hipLaunchKernelGGL(k_set_wf, dim3(grid_for(H->n_fine)), dim3(BLOCK), 0, s, H->n_fine, H->fine_nodes,
                           H->fine_pad, H->diag_p, omega, H->wf, H->wf32, bad);
    EB_LAUNCH_CHECK();
    int32_t hb = 0;
    EB_TRY(read_device_i32(bad, &hb, s));
    EB_TRY(dfree(bad, s));
    if (hb) {
        H->wf_on = 0;
        set_error("amg_set_fine_weights: weights must be positive and finite at every computational point");
        return EB_EINVAL;
    }
    H->wf_on = H->nlev > 1 ? 1 : 0;
    return EB_OK;
}

extern "C" int amg_clear_fine_weights(amg_handle_t* H) {
    clear_error();
    AllocScope scope(H ? &H->params : nullptr);
    if (!H) {
        set_error("amg_clear_fine_weights: null pointer");
        return EB_EINVAL;
    }
    H->wf_on = 0;
    return EB_OK;
}

extern "C" int amg_smoother_samples(amg_handle_t* H, int32_t m, int32_t sweeps, const double* xi, double* e,
                                    void* stream) {
    clear_error();
    AllocScope scope(H ? &H->params : nullptr);
    if (!H || !xi || !e || m < 1 || sweeps < 0) {
        set_error("amg_smoother_samples: invalid arguments");
        return EB_EINVAL;
    }
    EB_TRY(lg_check(H, "amg_smoother_samples"));
    hipStream_t s = stream ? (hipStream_t)stream : H->stream;
    H->last_stream = s;
    const GridDims& d = H->d;
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    const int64_t nunk = H->n_fine;
    const FineArgs f = fine_args(H);
    const int np = H->red.nparts;
    const unsigned ug = grid_for(nunk, NT);
    double *ev = nullptr, *rv = nullptr;
    EB_TRY(dalloc_n(&ev, H->npad, s));
    EB_TRY(dalloc_n(&rv, H->npad, s));
    EB_HIP(hipMemsetAsync(ev, 0, sizeof(double) * H->npad, s));
    EB_HIP(hipMemsetAsync(rv, 0, sizeof(double) * H->npad, s));
    EB_HIP(hipMemsetAsync(e, 0, sizeof(double) * nn * m, s));
    hipLaunchKernelGGL(k_mark_running, dim3(1), dim3(1), 0, s, H->sc);
    for (int j = 0; j < m; ++j) {
        hipLaunchKernelGGL(k_load_field, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, xi + j * nn, ev);
        for (int k = 0; k < sweeps; ++k) {
            hipLaunchKernelGGL(k_lg_apply, dim3(np), dim3(NT), 0, s, f, (const double*)ev, rv);
            EB_TRY(enqueue_vcycle_any<double>(H, rv, H->z, H->red.aux2, s));
            hipLaunchKernelGGL(k_lg_diffnorm, dim3(np), dim3(NT), 0, s, f, (const double*)ev, (const double*)H->z,
                               H->red.aux);
            hipLaunchKernelGGL(k_lg_diffscale, dim3(np), dim3(NT), 0, s, f, ev, (const double*)H->z,
                               (const double*)H->red.aux, np);
        }
        hipLaunchKernelGGL(k_store_field<double>, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad,
                           (const double*)ev, e + j * nn);
        EB_LAUNCH_CHECK();
    }
    EB_TRY(dfree(ev, s));
    EB_TRY(dfree(rv, s));
    EB_HIP(hipStreamSynchronize(s));
    return EB_OK;
}

extern "C" int amg_smoother_loss_grad(amg_handle_t* H, int32_t m, const double* e, double* loss, double* grad_omega,
                                      void* stream) {
    clear_error();
    AllocScope scope(H ? &H->params : nullptr);
    if (!H || !e || !loss || !grad_omega || m < 1) {
        set_error("amg_smoother_loss_grad: invalid arguments");
        return EB_EINVAL;
    }
    EB_TRY(lg_check(H, "amg_smoother_loss_grad"));
    hipStream_t s = stream ? (hipStream_t)stream : H->stream;
    H->last_stream = s;
    const GridDims& d = H->d;
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    const int64_t nunk = H->n_fine;
    const FineArgs f = fine_args(H);
    const int np = H->red.nparts;
    const unsigned ug = grid_for(nunk, NT);
    const double w0 = H->lev[0].omega;
    // padded vectors: e, r, t2, ep / Aep, g, wg / pe, u, gw, scratch
    double* v[9] = {};
    for (double*& p : v) {
        EB_TRY(dalloc_n(&p, H->npad, s));
        EB_HIP(hipMemsetAsync(p, 0, sizeof(double) * H->npad, s));
    }
    double *ev = v[0], *rv = v[1], *t2 = v[2], *ep = v[3], *g = v[4], *wg = v[5], *u = v[6], *gw = v[7],
           *aep = v[8];
    double* dloss = nullptr;
    double* part_den = nullptr;
    EB_TRY(dalloc_n(&dloss, 1, s));
    EB_TRY(dalloc_n(&part_den, PART_CAP, s));
    EB_HIP(hipMemsetAsync(dloss, 0, sizeof(double), s));
    hipLaunchKernelGGL(k_mark_running, dim3(1), dim3(1), 0, s, H->sc);
    for (int j = 0; j < m; ++j) {
        hipLaunchKernelGGL(k_load_field, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, e + j * nn, ev);
        hipLaunchKernelGGL(k_lg_apply, dim3(np), dim3(NT), 0, s, f, (const double*)ev, rv);
        hipLaunchKernelGGL(k_lg_dot, dim3(np), dim3(NT), 0, s, f, (const double*)ev, (const double*)rv, part_den);
        EB_TRY(lg_cycle_to_z2(H, rv, s));                                   // H->zt = z2
        hipLaunchKernelGGL(k_lg_post, dim3(np), dim3(NT), 0, s, f, (const double*)ev, (const double*)rv,
                           (const double*)H->zt, w0, t2, ep);
        hipLaunchKernelGGL(k_lg_apply, dim3(np), dim3(NT), 0, s, f, (const double*)ep, aep);
        hipLaunchKernelGGL(k_lg_dot, dim3(np), dim3(NT), 0, s, f, (const double*)ep, (const double*)aep, H->red.aux);
        hipLaunchKernelGGL(k_lg_loss, dim3(1), dim3(NT), 0, s, (const double*)H->red.aux, (const double*)part_den, np,
                           dloss);
        hipLaunchKernelGGL(k_lg_g, dim3(np), dim3(NT), 0, s, f, (const double*)aep, (const double*)part_den, np, w0,
                           g, wg);
        hipLaunchKernelGGL(k_lg_u, dim3(np), dim3(NT), 0, s, f, (const double*)g, (const double*)wg, u);
        // R u -> coarse cycle -> P e_c
        EB_TRY(launch_fine_restrict64(H, f, w0, (const double*)u, H->lev[1].rv, np, s));
        EB_TRY(enqueue_coarse<double>(H, s));
        hipLaunchKernelGGL(k_lg_prolong, dim3(np), dim3(NT), 0, s, f, w0, H->agg_p, (const double*)H->lev[1].ev, wg);
        hipLaunchKernelGGL(k_lg_acc, dim3(np), dim3(NT), 0, s, f, (const double*)g, (const double*)t2,
                           (const double*)u, (const double*)wg, (const double*)rv, gw);
        EB_LAUNCH_CHECK();
    }
    const int64_t nnode = nn;
    EB_HIP(hipMemsetAsync(grad_omega, 0, sizeof(double) * nnode, s));
    hipLaunchKernelGGL(k_lg_store_grad, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad,
                       (const double*)gw, H->diag_p, 1.0 / m, grad_omega);
    EB_LAUNCH_CHECK();
    double hl = 0.0;
    EB_HIP(hipMemcpyAsync(&hl, dloss, sizeof(double), hipMemcpyDeviceToHost, s));
    EB_HIP(hipStreamSynchronize(s));
    *loss = hl / m;
    for (double* p : v) EB_TRY(dfree(p, s));
    EB_TRY(dfree(dloss, s));
    EB_TRY(dfree(part_den, s));
    return EB_OK;
}

namespace eb {

}  // namespace eb

using namespace eb;

extern "C" int pcg_solve(amg_handle_t* H, const double* b, double* x, const pcg_params_t* prm, pcg_result_t* res,
                         void* stream) {
    clear_error();
    AllocScope scope(H ? &H->params : nullptr);
    if (!H || !b || !x || !res) {
        set_error("pcg_solve: null pointer");
        return EB_EINVAL;
    }
    pcg_params_t p;
    p.tol = 1e-8;
    p.maxit = 1000;
    p.x0_given = 0;
    p.check_every = 8;
    p.precision = EB_PREC_FP64;
    if (prm) p = *prm;
    if (!(p.tol > 0.0) || p.maxit < 0 || p.check_every < 1 ||
        (p.precision != EB_PREC_FP64 && p.precision != EB_PREC_FP32 && p.precision != EB_PREC_BF16)) {
        set_error("pcg_solve: invalid parameters (tol > 0, maxit >= 0, check_every >= 1, precision 0, 1 or 2)");
        return EB_EINVAL;
    }
    if (p.precision == EB_PREC_BF16 && H->wf_on) {
        set_error("pcg_solve: the BF16 smoother takes no per-point smoother weights");
        return EB_ENOTIMPL;
    }
    if (H->beta_on && p.precision == EB_PREC_BF16) {
        set_error("pcg_solve: the BF16 smoother is not available with variable conductivity");
        return EB_ENOTIMPL;
    }
    memset(res, 0, sizeof(*res));
    res->levels = H->nlev;
    hipStream_t s = stream ? (hipStream_t)stream : H->stream;
    H->last_stream = s;
    const GridDims& d = H->d;
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    const int64_t nunk = H->n_fine;
    EB_HIP(hipEventRecord(H->ev0, s));
    if (nunk == 0) {
        EB_HIP(hipMemsetAsync(x, 0, sizeof(double) * nn, s));
        EB_HIP(hipEventRecord(H->ev1, s));
        EB_HIP(hipStreamSynchronize(s));
        res->status = EB_OK;
        return EB_OK;
    }
    // the single-precision V-cycle (and the BF16 smoother inside it) needs a
    // hierarchy below the fine level
    const bool b16 = p.precision == EB_PREC_BF16 && H->nlev > 1;
    const bool fp32 = (p.precision == EB_PREC_FP32 || p.precision == EB_PREC_BF16) && H->nlev > 1;
    if (fp32) EB_TRY(ensure_fp32(H, s));
    if (b16) EB_TRY(ensure_bf16(H, s));
    const FineArgs f = fine_args(H);
    const int np = H->red.nparts;
    const unsigned ug = grid_for(nunk, NT);
    if (p.x0_given) {
        hipLaunchKernelGGL(k_load_field, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, b, H->bvec);
        hipLaunchKernelGGL(k_load_field, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, x, H->x);
        EB_LAUNCH_CHECK();
    }

    int restarts = 0;
    int enqueued = 0;
    int iter_base = 0;
    int rc = EB_OK;
    while (true) {
        if (!p.x0_given && restarts == 0) EB_TRY(enqueue_init_zero_guess(H, b, nunk, p.tol, s));
        else EB_TRY(enqueue_init(H, p.tol, iter_base, s));
        // V-cycle 0 -> rz[0]
        if (H->nlev == 1) EB_TRY(enqueue_vcycle_one_level(H, H->rr[0], H->z, H->red.rz[0], 0, s));
        else if (b16) EB_TRY((enqueue_vcycle_any<float, true>(H, H->rr[0], (bf16*)H->z16, H->red.rz[0], s)));
        else if (fp32) EB_TRY(enqueue_vcycle_any<float>(H, H->rr[0], H->z32, H->red.rz[0], s));
        else EB_TRY(enqueue_vcycle_any<double>(H, H->rr[0], H->z, H->red.rz[0], s));
        // Iterations go out in chunks between polls of the device scalars.
        // The first chunk is queued without a poll (a system that is already
        // converged is marked done by the init kernel and every later kernel
        // returns at once); later chunks end one iteration past the point
        // where the residual, reduced at the rate seen so far, reaches the
        // tolerance.  A chunk expected to finish is followed by the true
        // residual, so that one poll serves both.
        int k = 0;
        int chunk = p.check_every < p.maxit - iter_base ? p.check_every : p.maxit - iter_base;
        bool predicted = false;    // the chunk was sized to end at convergence
        bool true_done = false;
        while (true) {
            const bool graphs = g_use_graphs.load() && H->nlev > 1 && H->tim_kernel < 0;
            for (int c = 0; c < chunk;) {
                // graphs: not with a one-level hierarchy or while a kernel is being timed
                if (graphs && k + 1 >= 3 && ((k + 1) & 1) && chunk - c >= 2) {
                    if (b16) EB_TRY((launch_iteration_pair<float, true>(H, s)));
                    else if (fp32) EB_TRY(launch_iteration_pair<float>(H, s));
                    else EB_TRY(launch_iteration_pair<double>(H, s));
                    k += 2;
                    c += 2;
                    enqueued += 2;
                    continue;
                }
                ++k;
                ++c;
                ++enqueued;
                if (H->nlev == 1) EB_TRY(enqueue_iteration_one_level(H, k, s));
                else if (b16) EB_TRY((enqueue_iteration_any<float, true>(H, k, s)));
                else if (fp32) EB_TRY(enqueue_iteration_any<float>(H, k, s));
                else EB_TRY(enqueue_iteration_any<double>(H, k, s));
            }
            const bool expect_end = predicted || k >= p.maxit - iter_base;
            if (expect_end) {
                // true residual ||b - A x|| behind the chunk (recomputed below if
                // the chunk turns out not to finish)
                launch_resid(H, f, (unsigned)np, H->res, H->red.aux, s);
                hipLaunchKernelGGL(k_finalize_true, dim3(1), dim3(NT), 0, s, H->sc, H->red.aux, np);
                EB_LAUNCH_CHECK();
            }
            EB_TRY(poll_scalars(H, s));
            const PcgScalars& ph = *H->sc_host;
            if (ph.done || ph.iters >= p.maxit) {
                true_done = expect_end;
                break;
            }
            if (enqueued > 2 * p.maxit + 2 * p.check_every) {
                set_error("pcg_solve: iteration counter stalled");
                return EB_EHIP;
            }
            const int left = p.maxit - ph.iters;
            int next = p.check_every;
            predicted = false;
            const int done_its = ph.iters - iter_base;
            if (done_its >= 2 && ph.rr > 0.0 && ph.rr < ph.rr0 && ph.tol2bb > 0.0) {
                // log(rr_k / rr_0) / k per iteration; iterations to tol^2 bb, plus one
                const double rate = log(ph.rr / ph.rr0) / (double)done_its;
                const double need = log(ph.tol2bb / ph.rr) / rate;
                if (need > 0.0 && need < 2.0 * (double)p.check_every) {
                    next = (int)ceil(need) + 1;
                    predicted = true;
                }
            }
            chunk = next < left ? next : left;
        }
        if (!true_done) {
            // true residual ||b - A x||
            launch_resid(H, f, (unsigned)np, H->res, H->red.aux, s);
            hipLaunchKernelGGL(k_finalize_true, dim3(1), dim3(NT), 0, s, H->sc, H->red.aux, np);
            EB_LAUNCH_CHECK();
            EB_TRY(poll_scalars(H, s));
        }
        const PcgScalars& sh = *H->sc_host;
        const double bb = sh.bb;
        const double true_rel = bb > 0.0 ? sqrt(sh.rr_true / bb) : 0.0;
        res->rel_res_true = true_rel;
        res->rel_res_recursive = bb > 0.0 ? sqrt(sh.rr / bb) : 0.0;
        res->iterations = sh.iters;
        if (sh.status != EB_OK) {
            rc = sh.status;
            break;
        }
        if (true_rel <= p.tol || bb == 0.0) {
            rc = EB_OK;
            break;
        }
        if (restarts == 0 && sh.iters < p.maxit) {
            restarts = 1;          // drift: restart from the current iterate
            iter_base = sh.iters;
            continue;
        }
        rc = EB_ENOCONV;
        break;
    }
    res->restarts = restarts;
    res->status = rc;
    EB_HIP(hipMemsetAsync(x, 0, sizeof(double) * nn, s));
    hipLaunchKernelGGL(k_store_field<double>, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, H->x, x);
    EB_LAUNCH_CHECK();
    EB_HIP(hipEventRecord(H->ev1, s));
    EB_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    EB_HIP(hipEventElapsedTime(&ms, H->ev0, H->ev1));
    res->solve_ms = ms;
    if (rc == EB_ENOCONV) set_error("pcg_solve: no convergence within %d iterations", p.maxit);
    if (rc == EB_ENOTSPD) set_error("pcg_solve: non-positive curvature (operator or preconditioner not SPD)");
    if (rc == EB_ENAN) set_error("pcg_solve: NaN or Inf in the iteration");
    return rc;
}

static int vcycle_apply(amg_handle_t* H, const double* r, double* z, int precision, void* stream,
                        const char* name) {
    clear_error();
    AllocScope scope(H ? &H->params : nullptr);
    if (!H || !r || !z) {
        set_error("%s: null pointer", name);
        return EB_EINVAL;
    }
    hipStream_t s = stream ? (hipStream_t)stream : H->stream;
    H->last_stream = s;
    const GridDims& d = H->d;
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    const int64_t nunk = H->n_fine;
    EB_HIP(hipMemsetAsync(z, 0, sizeof(double) * nn, s));
    if (nunk == 0) return EB_OK;
    if (precision != EB_PREC_FP64 && precision != EB_PREC_FP32 && precision != EB_PREC_BF16) {
        set_error("%s: precision must be 0, 1 or 2", name);
        return EB_EINVAL;
    }
    if (precision == EB_PREC_BF16 && H->wf_on) {
        set_error("%s: the BF16 smoother takes no per-point smoother weights", name);
        return EB_ENOTIMPL;
    }
    if (H->beta_on && precision == EB_PREC_BF16) {
        set_error("%s: the BF16 smoother is not available with variable conductivity", name);
        return EB_ENOTIMPL;
    }
    const bool b16 = precision == EB_PREC_BF16 && H->nlev > 1;
    const bool fp32 = (precision == EB_PREC_FP32 || precision == EB_PREC_BF16) && H->nlev > 1;
    if (fp32) EB_TRY(ensure_fp32(H, s));
    if (b16) EB_TRY(ensure_bf16(H, s));
    const unsigned ug = grid_for(nunk, NT);
    hipLaunchKernelGGL(k_mark_running, dim3(1), dim3(1), 0, s, H->sc);
    hipLaunchKernelGGL(k_load_field, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, r, H->rr[0]);
    EB_LAUNCH_CHECK();
    if (H->nlev == 1) {
        EB_TRY(enqueue_vcycle_one_level(H, H->rr[0], H->z, H->red.aux2, 0, s));
    } else if (b16) {
        EB_TRY((enqueue_vcycle_any<float, true>(H, H->rr[0], (bf16*)H->z16, H->red.aux2, s)));
    } else if (fp32) {
        EB_TRY(enqueue_vcycle_any<float>(H, H->rr[0], H->z32, H->red.aux2, s));
    } else {
        EB_TRY(enqueue_vcycle_any<double>(H, H->rr[0], H->z, H->red.aux2, s));
    }
    if (b16) {
        hipLaunchKernelGGL(k_store_field<bf16>, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad,
                           (const bf16*)H->z16, z);
    } else if (fp32) {
        hipLaunchKernelGGL(k_store_field<float>, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, H->z32,
                           z);
    } else {
        hipLaunchKernelGGL(k_store_field<double>, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, H->z,
                           z);
    }
    EB_LAUNCH_CHECK();
    EB_HIP(hipStreamSynchronize(s));
    return EB_OK;
}

extern "C" int amg_vcycle_apply(amg_handle_t* H, const double* r, double* z, void* stream) {
    return vcycle_apply(H, r, z, EB_PREC_FP64, stream, "amg_vcycle_apply");
}

extern "C" int amg_vcycle_apply_fp32(amg_handle_t* H, const double* r, double* z, void* stream) {
    return vcycle_apply(H, r, z, EB_PREC_FP32, stream, "amg_vcycle_apply_fp32");
}

__global__ void k_set_f64(double* p, double v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

extern "C" int amg_set_level_weight(amg_handle_t* H, int32_t level, double factor, void* stream) {
    clear_error();
    AllocScope scope(H ? &H->params : nullptr);
    if (!H || level < 1 || level >= H->nlev || H->lev[level].is_coarsest || !(factor > 0.0) || isinf(factor)) {
        set_error("amg_set_level_weight: a coarse level with a smoother (1 <= level < levels - 1) and a factor > 0");
        return EB_EINVAL;
    }
    hipStream_t s = stream ? (hipStream_t)stream : H->stream;
    Level& L = H->lev[level];
    const double w = factor == 1.0 ? L.omega_setup : factor * L.omega_setup;
    if (w == L.omega) return EB_OK;
    L.omega = w;
    // captured iterations carry the weight as a kernel argument
    drop_iteration_graphs(H);
    drop_batch_graph(H);
    if (level == 1 && H->box_w0) {
        // the 2-D restriction's per-box omega_1 / d_1
        const Level& B0 = H->lev[0];
        const int64_t nb = (int64_t)B0.nb[0] * B0.nb[1];
        hipLaunchKernelGGL(k_set_f64, dim3(1), dim3(1), 0, s, H->dscal + 2 * 1 + 1, w);
        hipLaunchKernelGGL(k_box_w0, dim3(grid_for(nb)), dim3(BLOCK), 0, s, nb, (const int32_t*)B0.box_cstart,
                           (const int32_t*)B0.box_ncomp, (const double*)L.diag, (const double*)H->dscal, H->box_w0);
        if (H->box_w0_32)
            hipLaunchKernelGGL(k_to_f32, dim3(grid_for(nb, NT)), dim3(NT), 0, s, nb, (const double*)H->box_w0,
                               H->box_w0_32);
        EB_LAUNCH_CHECK();
    }
    H->last_stream = s;
    return EB_OK;
}

extern "C" int amg_vcycle_apply_prec(amg_handle_t* H, const double* r, double* z, int32_t precision, void* stream) {
    return vcycle_apply(H, r, z, precision, stream, "amg_vcycle_apply_prec");
}

extern "C" int eb_timing_select(amg_handle_t* H, int kernel_id) {
    clear_error();
    if (!H || kernel_id >= EB_K_COUNT) {
        set_error("eb_timing_select: bad handle or kernel id");
        return EB_EINVAL;
    }
    if (kernel_id >= 0 && !H->tim_ev) {
        // one event pool per process and device, shared by handles that time
        // kernels (the hook is a measurement aid: not for concurrent solves)
        static hipEvent_t* pools[64] = {nullptr};
        int dev = 0;
        EB_HIP(hipGetDevice(&dev));
        if (dev < 0 || dev >= 64) {
            set_error("eb_timing_select: device id out of range");
            return EB_EINVAL;
        }
        if (!pools[dev]) {
            hipEvent_t* pool = new hipEvent_t[2 * 256];
            for (int i = 0; i < 2 * 256; ++i) EB_HIP(hipEventCreate(&pool[i]));
            pools[dev] = pool;
        }
        H->tim_cap = 256;
        H->tim_ev = pools[dev];
    }
    EB_TRY(timing_harvest(H));
    H->tim_kernel = kernel_id;
    return EB_OK;
}

extern "C" int eb_timing_read(amg_handle_t* H, int64_t* launches, double* total_ms) {
    clear_error();
    if (!H || !launches || !total_ms) {
        set_error("eb_timing_read: null pointer");
        return EB_EINVAL;
    }
    EB_TRY(timing_harvest(H));
    *launches = H->tim_launches;
    *total_ms = H->tim_ms;
    H->tim_launches = 0;
    H->tim_ms = 0.0;
    return EB_OK;
}

extern "C" int eb_set_iteration_graphs(int32_t enabled) {
    clear_error();
    g_use_graphs.store(enabled ? 1 : 0);
    return EB_OK;
}
