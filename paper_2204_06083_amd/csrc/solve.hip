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

#include "handle.hpp"

namespace eb {

constexpr int NT = 256;        // threads per block of every solve kernel
constexpr int MAX_PARTS = 1024;

struct FineArgs {
    const int32_t* strips;
    int64_t nthreads;     // nstrips * strip_w virtual threads
    int strip_w;
    int64_t sy, sz;       // padded strides
    int dim;
    double s;             // 1/h^2
    const double* diag;   // padded, 0 off unknowns
};

__device__ inline int64_t strip_node(const FineArgs& f, int64_t gid) {
    const int64_t sidx = gid / f.strip_w;
    return (int64_t)f.strips[sidx] * f.strip_w + (gid - sidx * f.strip_w);
}

#define FINE_LOOP(f, p)                                                                         \
    for (int64_t gid_ = (int64_t)blockIdx.x * NT + threadIdx.x; gid_ < (f).nthreads;            \
         gid_ += (int64_t)gridDim.x * NT)                                                        \
        for (int64_t p = strip_node((f), gid_), once_ = 0; once_ < 1; ++once_)

__device__ inline double nbr_sum(const double* __restrict__ v, int64_t p, const FineArgs& f) {
    double t = v[p - 1] + v[p + 1];
    t += v[p - f.sy] + v[p + f.sy];
    if (f.dim == 3) t += v[p - f.sz] + v[p + f.sz];
    return t;
}

__device__ inline double safe_div(double x, double d) { return d != 0.0 ? x / d : 0.0; }

// sum over neighbours of v / d (zero where d == 0, i.e. off unknowns)
__device__ inline double nbr_sum_scaled(const double* __restrict__ v, int64_t p, const FineArgs& f) {
    double t = safe_div(v[p - 1], f.diag[p - 1]) + safe_div(v[p + 1], f.diag[p + 1]);
    t += safe_div(v[p - f.sy], f.diag[p - f.sy]) + safe_div(v[p + f.sy], f.diag[p + f.sy]);
    if (f.dim == 3) t += safe_div(v[p - f.sz], f.diag[p - f.sz]) + safe_div(v[p + f.sz], f.diag[p + f.sz]);
    return t;
}

// ------------------------------------------------------------ reductions
__device__ inline void block_partial(double v, double* __restrict__ part) {
    __shared__ double lds[NT / WAVE];
    const double s = block_sum<NT>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Sum of np partials in a fixed order; every thread of the block gets it.
__device__ inline double block_total(const double* __restrict__ part, int np) {
    __shared__ double lds[NT / WAVE];
    __shared__ double tot;
    double a = 0.0;
    for (int i = threadIdx.x; i < np; i += NT) a += part[i];
    a = block_sum<NT>(a, lds);
    if (threadIdx.x == 0) tot = a;
    __syncthreads();
    const double r = tot;
    __syncthreads();
    return r;
}

__device__ inline bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }

__device__ inline bool bad_value(double v) { return isnan(v) || isinf(v); }

// ------------------------------------------------------------ PCG kernels
// p_new = z + beta p_old; q = A p_new; partial (p_new, q).
// rho = (r, z) of the latest V-cycle, beta = rho / rho_prev (0 on the first).
__global__ void __launch_bounds__(NT) k_pcg_p_spmv(FineArgs f, const double* __restrict__ z,
                                                   const double* __restrict__ pold, double* __restrict__ pnew,
                                                   double* __restrict__ q, const double* __restrict__ rz_cur,
                                                   const double* __restrict__ rz_prev, int np,
                                                   double* __restrict__ part_pq, PcgScalars* sc) {
    if (sc->done) return;
    const double rho = block_total(rz_cur, np);
    double beta = 0.0;
    if (rz_prev) beta = rho / block_total(rz_prev, np);
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
            const double pc = z[p] + beta * pold[p];
            double nb = z[p - 1] + beta * pold[p - 1];
            nb += z[p + 1] + beta * pold[p + 1];
            nb += z[p - f.sy] + beta * pold[p - f.sy];
            nb += z[p + f.sy] + beta * pold[p + f.sy];
            if (f.dim == 3) {
                nb += z[p - f.sz] + beta * pold[p - f.sz];
                nb += z[p + f.sz] + beta * pold[p + f.sz];
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
                                               int np, double* __restrict__ part_rr, PcgScalars* sc, int iter) {
    if (sc->done) return;
    const double rho = block_total(rz_cur, np);
    const double pq = block_total(part_pq, np);
    if (!(pq > 0.0) || bad_value(pq)) {
        if (lead()) {
            sc->status = bad_value(pq) ? EB_ENAN : EB_ENOTSPD;
            sc->done = 1;
        }
        return;
    }
    const double alpha = rho / pq;
    if (lead()) {
        sc->iters = iter;
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

// Convergence test on ||r||^2 (partials of the previous kernel); true if the
// caller must return.
__device__ inline bool converged_or_failed(const double* __restrict__ part_rr, int np, PcgScalars* sc) {
    const double rr = block_total(part_rr, np);
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

// ------------------------------------------------------------ fine V-cycle
// Pre-smoothing and residual: z1 = omega r / d (not stored), res = r - A z1.
// With `check`, first test convergence of the iterate that produced r.
__global__ void __launch_bounds__(NT) k_fine_down(FineArgs f, double omega, const double* __restrict__ r,
                                                  double* __restrict__ res, PcgScalars* sc, int check,
                                                  const double* __restrict__ part_rr, int np) {
    if (sc->done) return;
    if (check && converged_or_failed(part_rr, np, sc)) return;
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double z1 = omega * r[p] / d;
            const double nb = omega * nbr_sum_scaled(r, p, f);
            res[p] = r[p] - (d * z1 - f.s * nb);
        }
    }
}

// Restriction r_c = P^T res = P_tent^T (I - omega A D^-1) res, one thread per
// level-0 box; the box's coarse unknowns are consecutive from box_cstart.
constexpr int MAX_FINE_COMP = 16;

struct BoxArgs {
    const int32_t* boxes;
    int64_t nboxes;
    int nbx, nby;
    int nx, ny, nz;       // node extents
    const int32_t* cstart;
    const int32_t* ncomp;
    const int32_t* agg;   // padded
};

__global__ void __launch_bounds__(NT) k_fine_restrict(FineArgs f, BoxArgs b, double omega,
                                                      const double* __restrict__ res, double* __restrict__ rc,
                                                      const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (t >= b.nboxes) return;
    const int64_t box = b.boxes[t];
    const int bx = (int)(box % b.nbx);
    const int64_t rr = box / b.nbx;
    const int by = (int)(rr % b.nby);
    const int bz = (int)(rr / b.nby);
    const int32_t c0 = b.cstart[box];
    const int m = b.ncomp[box];
    double acc[MAX_FINE_COMP];
#pragma unroll
    for (int c = 0; c < MAX_FINE_COMP; ++c) acc[c] = 0.0;
    const int z_hi = f.dim == 3 ? 3 : 1;
    for (int oz = 0; oz < z_hi; ++oz) {
        const int k = f.dim == 3 ? 3 * bz + oz : 0;
        if (k >= b.nz) break;
        for (int oy = 0; oy < 3; ++oy) {
            const int j = 3 * by + oy;
            if (j >= b.ny) break;
            for (int ox = 0; ox < 3; ++ox) {
                const int i = 3 * bx + ox;
                if (i >= b.nx) break;
                const int64_t p = (int64_t)i + f.sy * j + f.sz * k;
                const double d = f.diag[p];
                if (d == 0.0) continue;
                const double rp = res[p];
                const double aw = d * (rp / d) - f.s * nbr_sum_scaled(res, p, f);
                const double u = rp - omega * aw;
                const int c = b.agg[p] - c0;
                if (c >= 0 && c < MAX_FINE_COMP) acc[c] += u;
            }
        }
    }
    for (int c = 0; c < m && c < MAX_FINE_COMP; ++c) rc[c0 + c] = acc[c];
}

// Prolongation and pre-smoothed correction: t = e_c[agg]; z = omega r / d +
// t - omega (A t) / d.
__global__ void __launch_bounds__(NT) k_fine_up(FineArgs f, double omega, const int32_t* __restrict__ agg,
                                                const double* __restrict__ ec, const double* __restrict__ r,
                                                double* __restrict__ zt, const PcgScalars* sc) {
    if (sc->done) return;
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double tp = ec[agg[p]];
            int32_t g;
            double nb = 0.0;
            g = agg[p - 1];      nb += g >= 0 ? ec[g] : 0.0;
            g = agg[p + 1];      nb += g >= 0 ? ec[g] : 0.0;
            g = agg[p - f.sy];   nb += g >= 0 ? ec[g] : 0.0;
            g = agg[p + f.sy];   nb += g >= 0 ? ec[g] : 0.0;
            if (f.dim == 3) {
                g = agg[p - f.sz]; nb += g >= 0 ? ec[g] : 0.0;
                g = agg[p + f.sz]; nb += g >= 0 ? ec[g] : 0.0;
            }
            const double at = d * tp - f.s * nb;
            zt[p] = omega * r[p] / d + (tp - omega * at / d);
        }
    }
}

// Post-smoothing: z = zt + omega (r - A zt) / d; partial (r, z).
__global__ void __launch_bounds__(NT) k_fine_post(FineArgs f, double omega, const double* __restrict__ zt,
                                                  const double* __restrict__ r, double* __restrict__ z,
                                                  double* __restrict__ part_rz, const PcgScalars* sc) {
    if (sc->done) return;
    double part = 0.0;
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double az = d * zt[p] - f.s * nbr_sum(zt, p, f);
            const double zv = zt[p] + omega * (r[p] - az) / d;
            z[p] = zv;
            part += r[p] * zv;
        }
    }
    block_partial(part, part_rz);
}

// out = b - A x (padded fields), partial ||out||^2.
__global__ void __launch_bounds__(NT) k_fine_resid(FineArgs f, const double* __restrict__ bp,
                                                   const double* __restrict__ x, double* __restrict__ out,
                                                   double* __restrict__ part) {
    double acc = 0.0;
    FINE_LOOP(f, p) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double ax = d * x[p] - f.s * nbr_sum(x, p, f);
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
    const double bb = block_total(part_bb, np);
    const double rr = block_total(part_rr, np);
    if (threadIdx.x == 0) {
        sc->bb = bb;
        sc->rr = rr;
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
__global__ void __launch_bounds__(NT) k_csr_down(int64_t n, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col, const double* __restrict__ val,
                                                 const double* __restrict__ diag, double omega,
                                                 const double* __restrict__ rv, double* __restrict__ res,
                                                 const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    double az = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int j = col[e];
        az += val[e] * (omega * rv[j] / diag[j]);
    }
    res[i] = rv[i] - az;
}

__global__ void __launch_bounds__(NT) k_csr_spmv(int64_t n, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col, const double* __restrict__ val,
                                                 const double* __restrict__ x, double* __restrict__ y,
                                                 const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) acc += val[e] * x[col[e]];
    y[i] = acc;
}

// zt = omega rv / d + P e_c
__global__ void __launch_bounds__(NT) k_csr_up(int64_t n, const int32_t* __restrict__ rowptr,
                                               const int32_t* __restrict__ col, const double* __restrict__ val,
                                               const double* __restrict__ diag, double omega,
                                               const double* __restrict__ rv, const double* __restrict__ ec,
                                               double* __restrict__ zt, const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) acc += val[e] * ec[col[e]];
    zt[i] = omega * rv[i] / diag[i] + acc;
}

// ev = zt + omega (rv - A zt) / d
__global__ void __launch_bounds__(NT) k_csr_post(int64_t n, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col, const double* __restrict__ val,
                                                 const double* __restrict__ diag, double omega,
                                                 const double* __restrict__ rv, const double* __restrict__ zt,
                                                 double* __restrict__ ev, const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    double az = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) az += val[e] * zt[col[e]];
    ev[i] = zt[i] + omega * (rv[i] - az) / diag[i];
}

// Coarsest: ev = W rv with W the dense inverse; one wavefront per row.
__global__ void __launch_bounds__(NT) k_dense_apply(int64_t n, const double* __restrict__ W,
                                                    const double* __restrict__ rv, double* __restrict__ ev,
                                                    const PcgScalars* sc) {
    if (sc->done) return;
    const int64_t row = (int64_t)blockIdx.x * (NT / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (row >= n) return;
    double acc = 0.0;
    for (int64_t j = lane; j < n; j += WAVE) acc += W[row * n + j] * rv[j];
    acc = wave_sum(acc);
    if (lane == 0) ev[row] = acc;
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

__global__ void __launch_bounds__(NT) k_store_field(int64_t n, const int64_t* __restrict__ nodes,
                                                    const int32_t* __restrict__ pad, const double* __restrict__ src,
                                                    double* __restrict__ dst) {
    const int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (k < n) dst[nodes[k]] = src[pad[k]];
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
                                                       int32_t* __restrict__ fine_pad, int8_t* __restrict__ kind_p,
                                                       double* __restrict__ diag_p, int32_t* __restrict__ agg_p,
                                                       int32_t* __restrict__ strip_flag, int strip_w) {
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= nunk) return;
    const int64_t n = fine_nodes[k];
    const int64_t i = n % d.nx;
    const int64_t row = n / d.nx;
    const int64_t pidx = i + (int64_t)px * row;
    fine_pad[k] = (int32_t)pidx;
    kind_p[pidx] = 2;
    diag_p[pidx] = diag0[k];
    agg_p[pidx] = has_agg ? agg0[k] : -1;
    strip_flag[pidx / strip_w] = 1;
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

static int timing_begin(amg_handle* H, int id, hipStream_t s, bool* on) {
    *on = H->tim_kernel == id;
    if (!*on) return EB_OK;
    if (H->tim_used == H->tim_cap) EB_TRY(timing_harvest(H));
    H->tim_stream = s;
    EB_HIP(hipEventRecord(H->tim_ev[2 * H->tim_used], s));
    return EB_OK;
}

static int timing_end(amg_handle* H, bool on, hipStream_t s) {
    if (!on) return EB_OK;
    EB_HIP(hipEventRecord(H->tim_ev[2 * H->tim_used + 1], s));
    H->tim_used += 1;
    return EB_OK;
}

#define EB_TIMED(H, id, s, launch)                    \
    do {                                             \
        bool on_;                                    \
        EB_TRY(timing_begin((H), (id), (s), &on_));  \
        launch;                                      \
        EB_TRY(timing_end((H), on_, (s)));           \
    } while (0)

static FineArgs fine_args(const amg_handle* H) {
    FineArgs f;
    f.strips = H->strips;
    f.nthreads = H->nstrips * H->strip_w;
    f.strip_w = H->strip_w;
    f.sy = H->px;
    f.sz = (int64_t)H->px * H->d.ny;
    f.dim = H->d.dim;
    f.s = H->d.s;
    f.diag = H->diag_p;
    return f;
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
    return b;
}

// z = M r on padded fine fields; the last kernel writes the (r, z) partials
// to rz_out.  With `check`, the first kernel tests convergence of r first.
static int enqueue_vcycle(amg_handle* H, const double* r, double* z, double* rz_out, int check, hipStream_t s) {
    PcgScalars* sc = H->sc;
    const int np = H->red.nparts;
    const dim3 G((unsigned)np);
    if (H->nlev == 1) {
        Level& L = H->lev[0];
        const int64_t n = L.n;
        hipLaunchKernelGGL(k_gather, G, dim3(NT), 0, s, n, H->fine_pad, r, L.rv, sc, check, H->red.rr, np);
        hipLaunchKernelGGL(k_dense_apply, dim3(grid_for(n, NT / WAVE)), dim3(NT), 0, s, n, L.dense_inv, L.rv, L.ev,
                           (const PcgScalars*)sc);
        hipLaunchKernelGGL(k_scatter_dot, G, dim3(NT), 0, s, n, H->fine_pad, L.ev, r, z, rz_out,
                           (const PcgScalars*)sc);
        EB_LAUNCH_CHECK();
        return EB_OK;
    }
    const FineArgs f = fine_args(H);
    const double w0 = H->lev[0].omega;
    EB_TIMED(H, EB_K_FINE_DOWN, s,
             hipLaunchKernelGGL(k_fine_down, G, dim3(NT), 0, s, f, w0, r, H->res, sc, check, H->red.rr, np));
    EB_TIMED(H, EB_K_FINE_RESTRICT, s,
             hipLaunchKernelGGL(k_fine_restrict, dim3(grid_for(H->nboxes0, NT)), dim3(NT), 0, s, f, box_args(H), w0,
                                H->res, H->lev[1].rv, (const PcgScalars*)sc));
    for (int l = 1; l < H->nlev - 1; ++l) {
        Level& L = H->lev[l];
        Level& C = H->lev[l + 1];
        hipLaunchKernelGGL(k_csr_down, dim3(grid_for(L.n, NT)), dim3(NT), 0, s, L.n, L.a_rowptr, L.a_col, L.a_val,
                           L.diag, L.omega, L.rv, L.res, (const PcgScalars*)sc);
        hipLaunchKernelGGL(k_csr_spmv, dim3(grid_for(C.n, NT)), dim3(NT), 0, s, C.n, L.r_rowptr, L.r_col, L.r_val,
                           L.res, C.rv, (const PcgScalars*)sc);
    }
    {
        Level& Lc = H->lev[H->nlev - 1];
        hipLaunchKernelGGL(k_dense_apply, dim3(grid_for(Lc.n, NT / WAVE)), dim3(NT), 0, s, Lc.n, Lc.dense_inv, Lc.rv,
                           Lc.ev, (const PcgScalars*)sc);
    }
    for (int l = H->nlev - 2; l >= 1; --l) {
        Level& L = H->lev[l];
        Level& C = H->lev[l + 1];
        hipLaunchKernelGGL(k_csr_up, dim3(grid_for(L.n, NT)), dim3(NT), 0, s, L.n, L.p_rowptr, L.p_col, L.p_val,
                           L.diag, L.omega, L.rv, C.ev, L.zt, (const PcgScalars*)sc);
        hipLaunchKernelGGL(k_csr_post, dim3(grid_for(L.n, NT)), dim3(NT), 0, s, L.n, L.a_rowptr, L.a_col, L.a_val,
                           L.diag, L.omega, L.rv, L.zt, L.ev, (const PcgScalars*)sc);
    }
    EB_TIMED(H, EB_K_FINE_UP, s,
             hipLaunchKernelGGL(k_fine_up, G, dim3(NT), 0, s, f, w0, H->agg_p, H->lev[1].ev, r, H->zt,
                                (const PcgScalars*)sc));
    EB_TIMED(H, EB_K_FINE_POST, s,
             hipLaunchKernelGGL(k_fine_post, G, dim3(NT), 0, s, f, w0, H->zt, r, z, rz_out, (const PcgScalars*)sc));
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// Iteration k >= 1 of a run: the V-cycle before it (number k-1) wrote
// rz[(k-1) % 2]; this iteration's V-cycle writes rz[k % 2].
static int enqueue_iteration(amg_handle* H, int k, int iter_global, hipStream_t s) {
    const FineArgs f = fine_args(H);
    const int np = H->red.nparts;
    const dim3 G((unsigned)np);
    double* pold = H->p[k & 1];
    double* pnew = H->p[(k + 1) & 1];
    const double* rz_cur = H->red.rz[(k - 1) & 1];
    const double* rz_prev = k >= 2 ? H->red.rz[k & 1] : nullptr;
    EB_TIMED(H, EB_K_PCG_SPMV, s,
             hipLaunchKernelGGL(k_pcg_p_spmv, G, dim3(NT), 0, s, f, H->z, pold, pnew, H->q, rz_cur, rz_prev, np,
                                H->red.pq, H->sc));
    EB_TIMED(H, EB_K_PCG_XR, s,
             hipLaunchKernelGGL(k_pcg_xr, G, dim3(NT), 0, s, f, H->x, H->r, pnew, H->q, rz_cur, H->red.pq, np,
                                H->red.rr, H->sc, iter_global));
    EB_LAUNCH_CHECK();
    return enqueue_vcycle(H, H->r, H->z, H->red.rz[k & 1], 1, s);
}

// b, x0 -> r0 = b - A x0; ||b||^2, ||r0||^2, tolerance, initial convergence test.
static int enqueue_init(amg_handle* H, double tol, int iters, hipStream_t s) {
    const FineArgs f = fine_args(H);
    const int np = H->red.nparts;
    const dim3 G((unsigned)np);
    hipLaunchKernelGGL(k_fine_norm2, G, dim3(NT), 0, s, f, H->bvec, H->red.aux);
    hipLaunchKernelGGL(k_fine_resid, G, dim3(NT), 0, s, f, H->bvec, H->x, H->r, H->red.rr);
    hipLaunchKernelGGL(k_finalize_init, dim3(1), dim3(NT), 0, s, H->sc, H->red.aux, H->red.rr, np, tol, iters);
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
    EB_TRY(dalloc_n(&H->dcount, 2, s));
    EB_HIP(hipMemsetAsync(H->dcount, 0, 2 * sizeof(int32_t), s));
    EB_TRY(dalloc_n(&H->fine_pad, nunk, s));
    EB_TRY(dalloc_n(&H->kind_p, npad, s));
    EB_TRY(dalloc_n(&H->diag_p, npad, s));
    EB_TRY(dalloc_n(&H->agg_p, npad, s));
    EB_HIP(hipMemsetAsync(H->kind_p, 0, npad, s));
    EB_HIP(hipMemsetAsync(H->diag_p, 0, sizeof(double) * npad, s));
    EB_HIP(hipMemsetAsync(H->agg_p, 0xff, sizeof(int32_t) * npad, s));   // -1
    const int64_t nstrip_all = npad / H->strip_w;
    int32_t* sflag = nullptr;
    EB_TRY(dalloc_n(&sflag, nstrip_all, s));
    EB_HIP(hipMemsetAsync(sflag, 0, sizeof(int32_t) * nstrip_all, s));
    Level& L0 = H->lev[0];
    hipLaunchKernelGGL(k_fine_layout, dim3(grid_for(nunk)), dim3(BLOCK), 0, s, H->fine_nodes, nunk, d, H->px, L0.diag,
                       L0.agg, L0.agg != nullptr ? 1 : 0, H->fine_pad, H->kind_p, H->diag_p, H->agg_p, sflag,
                       H->strip_w);
    EB_LAUNCH_CHECK();
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
    double** vecs[] = {&H->x, &H->r, &H->z, &H->p[0], &H->p[1], &H->q, &H->res, &H->zt, &H->bvec};
    for (double** v : vecs) {
        EB_TRY(dalloc_n(v, npad, s));
        EB_HIP(hipMemsetAsync(*v, 0, sizeof(double) * npad, s));
    }
    for (int l = 0; l < H->nlev; ++l) {
        Level& L = H->lev[l];
        if (l == 0 && H->nlev > 1) continue;
        const int64_t n = L.n > 0 ? L.n : 1;
        EB_TRY(dalloc_n(&L.rv, n, s));
        EB_TRY(dalloc_n(&L.res, n, s));
        EB_TRY(dalloc_n(&L.zt, n, s));
        EB_TRY(dalloc_n(&L.ev, n, s));
        EB_HIP(hipMemsetAsync(L.rv, 0, sizeof(double) * n, s));
        EB_HIP(hipMemsetAsync(L.ev, 0, sizeof(double) * n, s));
    }
    EB_TRY(dalloc_n(&H->sc, 1, s));
    EB_HIP(hipMemsetAsync(H->sc, 0, sizeof(PcgScalars), s));
    H->sc_host = &H->sc_mirror;   // pageable, per handle (polled a few times per solve)
    double** parts[] = {&H->red.pq, &H->red.rr, &H->red.rz[0], &H->red.rz[1], &H->red.aux, &H->red.aux2};
    for (double** v : parts) {
        EB_TRY(dalloc_n(v, MAX_PARTS, s));
        EB_HIP(hipMemsetAsync(*v, 0, sizeof(double) * MAX_PARTS, s));
    }
    EB_HIP(hipEventCreate(&H->ev0));
    EB_HIP(hipEventCreate(&H->ev1));
    return EB_OK;
}

// Part 2, after the device totals have been read back (dcount copied into
// H->nstrips / H->nboxes0 by the caller's single synchronisation).
int solve_layout_finish(amg_handle* H, hipStream_t s) {
    (void)s;
    const int64_t nthreads = H->nlev == 1 ? H->n_fine : H->nstrips * H->strip_w;
    int64_t np = (nthreads + NT - 1) / NT;
    if (np < 1) np = 1;
    if (np > MAX_PARTS) np = MAX_PARTS;
    H->red.nparts = (int)np;
    return EB_OK;
}

static int poll_scalars(amg_handle* H, hipStream_t s) {
    EB_HIP(hipMemcpyAsync(H->sc_host, H->sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
    EB_HIP(hipStreamSynchronize(s));
    if (H->tim_used > 0) EB_TRY(timing_harvest(H));
    return EB_OK;
}

}  // namespace eb

using namespace eb;

extern "C" int pcg_solve(amg_handle_t* H, const double* b, double* x, const pcg_params_t* prm, pcg_result_t* res,
                         void* stream) {
    clear_error();
    if (!H || !b || !x || !res) {
        set_error("pcg_solve: null pointer");
        return EB_EINVAL;
    }
    pcg_params_t p;
    p.tol = 1e-8;
    p.maxit = 1000;
    p.x0_given = 0;
    p.check_every = 8;
    p.reserved = 0;
    if (prm) p = *prm;
    if (!(p.tol > 0.0) || p.maxit < 0 || p.check_every < 1) {
        set_error("pcg_solve: invalid parameters (tol > 0, maxit >= 0, check_every >= 1)");
        return EB_EINVAL;
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
    const FineArgs f = fine_args(H);
    const int np = H->red.nparts;
    const unsigned ug = grid_for(nunk, NT);
    hipLaunchKernelGGL(k_load_field, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, b, H->bvec);
    if (p.x0_given) {
        hipLaunchKernelGGL(k_load_field, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, x, H->x);
    } else {
        EB_HIP(hipMemsetAsync(H->x, 0, sizeof(double) * H->npad, s));
    }
    EB_LAUNCH_CHECK();

    int restarts = 0;
    int enqueued = 0;
    int iter_base = 0;
    int rc = EB_OK;
    while (true) {
        EB_TRY(enqueue_init(H, p.tol, iter_base, s));
        EB_TRY(enqueue_vcycle(H, H->r, H->z, H->red.rz[0], 0, s));   // V-cycle 0: rz[0]
        int k = 0;
        while (true) {
            EB_TRY(poll_scalars(H, s));
            if (H->sc_host->done || H->sc_host->iters >= p.maxit) break;
            if (enqueued > 2 * p.maxit + 2 * p.check_every) {
                set_error("pcg_solve: iteration counter stalled");
                return EB_EHIP;
            }
            const int left = p.maxit - H->sc_host->iters;
            const int chunk = left < p.check_every ? left : p.check_every;
            for (int c = 0; c < chunk; ++c, ++enqueued) {
                ++k;
                EB_TRY(enqueue_iteration(H, k, iter_base + k, s));
            }
        }
        // true residual ||b - A x||
        hipLaunchKernelGGL(k_fine_resid, dim3((unsigned)np), dim3(NT), 0, s, f, H->bvec, H->x, H->res, H->red.aux);
        hipLaunchKernelGGL(k_finalize_true, dim3(1), dim3(NT), 0, s, H->sc, H->red.aux, np);
        EB_LAUNCH_CHECK();
        EB_TRY(poll_scalars(H, s));
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
    hipLaunchKernelGGL(k_store_field, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, H->x, x);
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

extern "C" int amg_vcycle_apply(amg_handle_t* H, const double* r, double* z, void* stream) {
    clear_error();
    if (!H || !r || !z) {
        set_error("amg_vcycle_apply: null pointer");
        return EB_EINVAL;
    }
    hipStream_t s = stream ? (hipStream_t)stream : H->stream;
    H->last_stream = s;
    const GridDims& d = H->d;
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    const int64_t nunk = H->n_fine;
    EB_HIP(hipMemsetAsync(z, 0, sizeof(double) * nn, s));
    if (nunk == 0) return EB_OK;
    const unsigned ug = grid_for(nunk, NT);
    hipLaunchKernelGGL(k_mark_running, dim3(1), dim3(1), 0, s, H->sc);
    hipLaunchKernelGGL(k_load_field, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, r, H->r);
    EB_LAUNCH_CHECK();
    EB_TRY(enqueue_vcycle(H, H->r, H->z, H->red.aux2, 0, s));
    hipLaunchKernelGGL(k_store_field, dim3(ug), dim3(NT), 0, s, nunk, H->fine_nodes, H->fine_pad, H->z, z);
    EB_LAUNCH_CHECK();
    EB_HIP(hipStreamSynchronize(s));
    return EB_OK;
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
