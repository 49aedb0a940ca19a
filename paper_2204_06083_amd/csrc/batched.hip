// Batched PCG: up to 64 right-hand sides share the hierarchy and one launch
// sequence (Algorithm 2 step 4 applied to several b at once, as in the heat
// steps of Sec. 3.4 and the repeated solves of shape optimisation).
//
// Layout: kp slots (a power of two >= nrhs).  Fine-level vectors are planes
// of kb = min(kp, 8) right-hand sides, node-major inside a plane:
// v[(j / kb) * npad * kb + node * kb + j % kb], so a wavefront reads 8 nodes x
// 8 right-hand sides contiguously, every diagonal or aggregate read serves kb
// right-hand sides, and a grid row of one plane (npad-row x 64 B) stays small
// enough for the rows above and below to be reused from L2.  Coarse-level
// vectors interleave all slots per row, v[row * kp + j], so every matrix entry
// read serves all kp right-hand sides.  The fine level keeps the single
// solve's padded strips; coarse levels keep their CSR.
//
// Each right-hand side runs its own PCG (its own alpha, beta, convergence and
// iteration count); a converged one is skipped by every later kernel.  The
// per-RHS sums are formed deterministically: each reducing kernel runs a fixed
// grid and writes one partial per (block, rhs); a one-block finaliser sums
// them in a fixed order and updates the per-RHS scalars.
#include <math.h>
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>


#include "handle.hpp"

namespace eb {

constexpr int BNT = 512;          // threads per block
constexpr int BMAX_RHS = 64;
constexpr int BPARTS = 512;       // blocks of the reducing fine kernels (multiple of 8)
constexpr int BFIN = 1024;        // threads of the finaliser
constexpr int BMAX_FINE_COMP = 16;
constexpr int BMAX_SLOTS = 4096;  // segments x slots
constexpr int BMAX_SEG = 1024;

// Per-system scalars on the device (one allocation).  A system is a
// (segment, slot) pair, index seg * kp + j: segments are the separate
// geometries of an island batch (one segment otherwise).  The two counters
// come first so that polling copies 16 bytes.
struct BatchState {
    int32_t ndone;             // finished systems
    int32_t maxiter;           // largest iteration count
    int32_t nsys;              // segments x kp
    int32_t pad;
    double rz[BMAX_SLOTS];     // (r, z) of the latest V-cycle
    double beta[BMAX_SLOTS];   // rz_new / rz_old for the next p-update (0 first)
    double alpha[BMAX_SLOTS];
    double pq[BMAX_SLOTS];
    double rr[BMAX_SLOTS];     // ||r||^2 of the latest iterate
    double bb[BMAX_SLOTS];
    double tol2bb[BMAX_SLOTS];
    double rr_true[BMAX_SLOTS];
    int32_t done[BMAX_SLOTS];  // 1: converged, failed or an unused slot
    int32_t status[BMAX_SLOTS];
    int32_t iters[BMAX_SLOTS];
    int32_t mask[BMAX_SLOTS];  // host-set: systems (re)started by the next init
};

struct BatchBufs {
    int kp = 0;
    int prec = -1;                        // precision of the V-typed arrays
    double* x = nullptr;
    double* rr[2] = {nullptr, nullptr};
    double* p[2] = {nullptr, nullptr};
    double* q = nullptr;
    double* bvec = nullptr;
    double* tres = nullptr;               // true residual scratch
    void* res = nullptr;                  // V-typed fine vectors
    void* zt = nullptr;
    void* z = nullptr;
    void* rv[MAX_LEVELS] = {};            // V-typed level vectors (levels >= 1; level 0 if one level)
    void* ev[MAX_LEVELS] = {};
    void* tmp[MAX_LEVELS] = {};
    double* part[3] = {nullptr, nullptr, nullptr};   // [BPARTS][kp]: (p,q), ||r||^2, (r,z)
    double* part_aux = nullptr;
    BatchState* st = nullptr;
    BatchState* host = nullptr;           // host copy (new-allocated: large)
    // segments (island batches): fine blocks never straddle a segment;
    // blk_start[b] .. blk_start[b + 1] are block b's strips, blk_seg[b] its
    // segment, seg_blk[s] .. seg_blk[s + 1] the blocks of segment s
    int nseg = 1;
    int nblk = 0;
    std::vector<int32_t> seg_rows;        // the segmentation these tables are for
    int32_t* blk_start = nullptr;
    int32_t* blk_seg = nullptr;
    int32_t* seg_blk = nullptr;
    // layout and launch shape of the fine kernels: plane width (slots per
    // plane, node-major inside a plane) and planes per block (the grid's y
    // dimension covers the rest); set by the autotuner on the first solve
    int kbw = 8;
    int npb = 2;
    bool tuned = false;
    int ncand = 0;
    int cand_w[8] = {}, cand_n[8] = {};
    float cand_ms[8] = {};
    // a captured pair of iterations (k odd >= 3, k + 1: the same launches for
    // every such k), for the launch shape it was captured with
    hipGraphExec_t it_graph = nullptr;
    int it_graph_kbw = 0, it_graph_npb = 0;
    hipStream_t cap_stream = nullptr;
};

// ------------------------------------------------------------------ helpers
struct BFine {
    const int32_t* strips;
    int64_t nstrips;
    int64_t spb;          // strips per block
    int strip_w;
    int lsw0;             // log2(strip_w)
    int lsw;              // log2(strip_w * kp)
    int lkp;              // log2(kp)
    int kp;
    int kb, lkb;          // plane width min(kp, 8) and its log2
    int64_t plane;        // npad * kb
    int64_t sy, sz;       // padded node strides
    int dim;
    double s;             // 1/h^2
    const double* diag;
    const float* diag32;
    const int32_t* done;  // per-system skip flags
    const int32_t* blk_start;   // segmented block ranges (null: spb strips per block)
    const int32_t* blk_seg;
};

// Index of the first system of this block's segment.
__device__ inline int bseg_base(const BFine& f) { return f.blk_seg ? f.blk_seg[xcd_block()] * f.kp : 0; }

template <class V> __device__ inline const V* bdiag(const BFine& f);
template <> __device__ inline const double* bdiag<double>(const BFine& f) { return f.diag; }
template <> __device__ inline const float* bdiag<float>(const BFine& f) { return f.diag32; }

// Fine index of (node p, slot j).
__device__ inline int64_t bvidx(const BFine& f, int64_t p, int j) {
    return (int64_t)(j >> f.lkb) * f.plane + p * f.kb + (j & (f.kb - 1));
}

template <class V>
__device__ inline V bsafe_div(V x, V d) { return d != V(0) ? x / d : V(0); }

// Per-RHS block partial for plane jb: thread t carries the sum for slot
// jb * kb + t % kb; the block's threads with the same slot are summed in
// thread order.
__device__ inline void bpartial(double v, double* __restrict__ part, int kp, int kb, int jb) {
    __shared__ double lds[BNT];
    lds[threadIdx.x] = v;
    __syncthreads();
    if ((int)threadIdx.x < kb) {
        double a = 0.0;
        for (int t = threadIdx.x; t < BNT; t += kb) a += lds[t];
        part[xcd_block() * kp + jb * kb + threadIdx.x] = a;
    }
    __syncthreads();
}

// The same with the slot t % kp (kernels over interleaved compact vectors).
__device__ inline void bpartial_kp(double v, double* __restrict__ part, int kp) { bpartial(v, part, kp, kp, 0); }

// Finaliser sum for slot j over the block partials b0 .. b1 - 1 (at most
// BPARTS): BFIN / kp threads per slot take block-strided partials, then are
// combined in a fixed order.  Every thread with slot j returns the total
// (threads t with t % kp == j).
__device__ inline double bfin_sum(const double* __restrict__ part, int b0, int b1, int kp) {
    __shared__ double lds[BFIN];
    const int j = threadIdx.x & (kp - 1);
    const int u = threadIdx.x / kp;
    const int g = BFIN / kp;
    // all of a thread's partials are loaded before they are added (in order)
    constexpr int MAXL = BPARTS * BMAX_RHS / BFIN;
    double v[MAXL];
#pragma unroll
    for (int i = 0; i < MAXL; ++i) {
        const int b = b0 + u + i * g;
        v[i] = b < b1 ? part[(int64_t)b * kp + j] : 0.0;
    }
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < MAXL; ++i) a += v[i];
    lds[threadIdx.x] = a;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < g; ++w) t += lds[w * kp + j];
    __syncthreads();
    return t;
}

__device__ inline bool bbad(double v) { return isnan(v) || isinf(v); }

// ------------------------------------------------------------- finalisers
// One block per segment (blockIdx.x); thread j < kp updates system
// seg * kp + j from the sums over the segment's blocks seg_blk[seg] ..
// seg_blk[seg + 1] - 1.  With one segment the block also recounts ndone and
// maxiter; with several, kb_fin_count does it after the finaliser.
#define BFIN_SEG                                              \
    const int seg_ = blockIdx.x;                              \
    const int b0_ = seg_blk[seg_], b1_ = seg_blk[seg_ + 1];   \
    const int j = threadIdx.x;                                \
    const int sj = seg_ * kp + j;

__device__ inline void bfin_count(BatchState* st) {
    if (gridDim.x != 1) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        int nd = 0, mx = 0;
        for (int i = 0; i < st->nsys; ++i) {
            nd += st->done[i] != 0;
            mx = max(mx, st->iters[i]);
        }
        st->ndone = nd;
        st->maxiter = mx;
    }
}

// ndone and maxiter over every system (several segments).
__global__ void __launch_bounds__(BFIN) kb_fin_count(BatchState* st) {
    __shared__ int nd_s[BFIN], mx_s[BFIN];
    int nd = 0, mx = 0;
    for (int i = threadIdx.x; i < st->nsys; i += BFIN) {
        nd += st->done[i] != 0;
        mx = max(mx, st->iters[i]);
    }
    nd_s[threadIdx.x] = nd;
    mx_s[threadIdx.x] = mx;
    __syncthreads();
    for (int h = BFIN / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            nd_s[threadIdx.x] += nd_s[threadIdx.x + h];
            mx_s[threadIdx.x] = max(mx_s[threadIdx.x], mx_s[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->ndone = nd_s[0];
        st->maxiter = mx_s[0];
    }
}

// (Re)start: ||b||^2 and ||r0||^2 per system; systems with mask = 0 are left done.
__global__ void __launch_bounds__(BFIN) kb_fin_init(BatchState* st, const double* __restrict__ part_bb,
                                                    const double* __restrict__ part_rr,
                                                    const int32_t* __restrict__ seg_blk, int kp, double tol) {
    BFIN_SEG
    const double bb = bfin_sum(part_bb, b0_, b1_, kp);
    const double rr = bfin_sum(part_rr, b0_, b1_, kp);
    if (j < kp && st->mask[sj]) {
        st->bb[sj] = bb;
        st->rr[sj] = rr;
        st->tol2bb[sj] = tol * tol * bb;
        st->status[sj] = (bbad(bb) || bbad(rr)) ? EB_ENAN : EB_OK;
        st->done[sj] = (bb == 0.0 || rr <= tol * tol * bb || st->status[sj] != EB_OK) ? 1 : 0;
        st->beta[sj] = 0.0;
    }
    bfin_count(st);
}

// (r, z) after a V-cycle: beta for the next p-update, curvature check.
__global__ void __launch_bounds__(BFIN) kb_fin_rz(BatchState* st, const double* __restrict__ part,
                                                  const int32_t* __restrict__ seg_blk, int kp, int first) {
    BFIN_SEG
    const double rz = bfin_sum(part, b0_, b1_, kp);
    if (j < kp && !st->done[sj]) {
        if (!(rz > 0.0) || bbad(rz)) {
            st->status[sj] = bbad(rz) ? EB_ENAN : EB_ENOTSPD;
            st->done[sj] = 1;
        } else {
            st->beta[sj] = first ? 0.0 : rz / st->rz[sj];
            st->rz[sj] = rz;
        }
    }
}

// (p, q): alpha = rz / (p, q).
__global__ void __launch_bounds__(BFIN) kb_fin_pq(BatchState* st, const double* __restrict__ part,
                                                  const int32_t* __restrict__ seg_blk, int kp) {
    BFIN_SEG
    const double pq = bfin_sum(part, b0_, b1_, kp);
    if (j < kp && !st->done[sj]) {
        st->pq[sj] = pq;
        if (!(pq > 0.0) || bbad(pq)) {
            st->status[sj] = bbad(pq) ? EB_ENAN : EB_ENOTSPD;
            st->done[sj] = 1;
        } else {
            st->alpha[sj] = st->rz[sj] / pq;
        }
    }
}

// ||r||^2 after the update: iteration count and convergence.
__global__ void __launch_bounds__(BFIN) kb_fin_rr(BatchState* st, const double* __restrict__ part,
                                                  const int32_t* __restrict__ seg_blk, int kp) {
    BFIN_SEG
    const double rr = bfin_sum(part, b0_, b1_, kp);
    if (j < kp && !st->done[sj]) {
        st->iters[sj] += 1;
        st->rr[sj] = rr;
        if (bbad(rr)) {
            st->status[sj] = EB_ENAN;
            st->done[sj] = 1;
        } else if (rr <= st->tol2bb[sj]) {
            st->done[sj] = 1;
        }
    }
    bfin_count(st);
}

__global__ void __launch_bounds__(BFIN) kb_fin_true(BatchState* st, const double* __restrict__ part,
                                                    const int32_t* __restrict__ seg_blk, int kp) {
    BFIN_SEG
    const double rr = bfin_sum(part, b0_, b1_, kp);
    if (j < kp) st->rr_true[sj] = rr;
}

// ------------------------------------------------------------ fine kernels
// Each thread takes one (node, j % kb) element of a plane and handles it in
// all NPL = kp / kb planes in one unrolled body, so the loads of the planes
// are independent and in flight together.  v0 is the element's index in
// plane 0; plane jb adds jb * plane.
#define BNODE_LOOP(f, p, jj, v0)                                                                         \
    for (int64_t xb_ = xcd_block(), s0_ = (f).blk_start ? (int64_t)(f).blk_start[xb_] : xb_ * (f).spb,       \
                 s1_ = (f).blk_start ? (int64_t)(f).blk_start[xb_ + 1] : min(s0_ + (f).spb, (f).nstrips),     \
                 e_ = (int64_t)threadIdx.x, eend_ = (s1_ - s0_) * ((int64_t)(f).strip_w << (f).lkb);       \
         e_ < eend_; e_ += BNT)                                                                            \
        for (int64_t p = (int64_t)(f).strips[s0_ + (e_ >> ((f).lsw0 + (f).lkb))] * (f).strip_w +           \
                         ((e_ >> (f).lkb) & ((f).strip_w - 1)),                                            \
                     jj = e_ & ((f).kb - 1), v0 = p * (f).kb + jj, once_ = 0;                              \
             once_ < 1; ++once_)

template <int NPL>
__device__ inline void bpartials(const double (&acc)[NPL], double* __restrict__ part, const BFine& f) {
#pragma unroll
    for (int jb = 0; jb < NPL; ++jb) bpartial(acc[jb], part, f.kp, f.kb, (int)blockIdx.y * NPL + jb);
}

// out = b - A x, partial ||out||^2 per rhs (FP64; every slot).
template <int NPL>
__global__ void __launch_bounds__(BNT) kb_resid(BFine f, const double* __restrict__ b, const double* __restrict__ x,
                                                double* __restrict__ out, double* __restrict__ part) {
    const int pb = (int)blockIdx.y * NPL;   // first plane of this block
    double acc[NPL];
#pragma unroll
    for (int jb = 0; jb < NPL; ++jb) acc[jb] = 0.0;
    const int64_t ox = f.kb, sy = f.sy * f.kb, sz = f.sz * f.kb;
    BNODE_LOOP(f, p, jj, v0) {
        const double d = f.diag[p];
        if (d != 0.0) {
#pragma unroll
            for (int jb = 0; jb < NPL; ++jb) {
                const int64_t v = v0 + (pb + jb) * f.plane;
                double nb = x[v - ox] + x[v + ox] + x[v - sy] + x[v + sy];
                if (f.dim == 3) nb += x[v - sz] + x[v + sz];
                const double rv = b[v] - (d * x[v] - f.s * nb);
                out[v] = rv;
                acc[jb] += rv * rv;
            }
        }
    }
    bpartials<NPL>(acc, part, f);
}

template <int NPL>
__global__ void __launch_bounds__(BNT) kb_norm2(BFine f, const double* __restrict__ a, double* __restrict__ part) {
    const int pb = (int)blockIdx.y * NPL;   // first plane of this block
    double acc[NPL];
#pragma unroll
    for (int jb = 0; jb < NPL; ++jb) acc[jb] = 0.0;
    BNODE_LOOP(f, p, jj, v0) {
        if (f.diag[p] != 0.0) {
#pragma unroll
            for (int jb = 0; jb < NPL; ++jb) {
                const double t = a[v0 + (pb + jb) * f.plane];
                acc[jb] += t * t;
            }
        }
    }
    bpartials<NPL>(acc, part, f);
}

// Initial pre-smoothing residual res = r - A (omega D^-1 r).
template <class V, int NPL>
__global__ void __launch_bounds__(BNT) kb_fine_down(BFine f, double omega, const double* __restrict__ r,
                                                    V* __restrict__ res) {
    const int pb = (int)blockIdx.y * NPL;   // first plane of this block
    const int sb = bseg_base(f);             // first system of this block's segment
    const int64_t ox = f.kb, sy = f.sy * f.kb, sz = f.sz * f.kb;
    BNODE_LOOP(f, p, jj, v0) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double dxm = f.diag[p - 1], dxp = f.diag[p + 1], dym = f.diag[p - f.sy], dyp = f.diag[p + f.sy];
            const double dzm = f.dim == 3 ? f.diag[p - f.sz] : 0.0, dzp = f.dim == 3 ? f.diag[p + f.sz] : 0.0;
#pragma unroll
            for (int jb = 0; jb < NPL; ++jb) {
                if (f.done[sb + ((pb + jb) << f.lkb) + jj]) continue;
                const int64_t v = v0 + (pb + jb) * f.plane;
                double nb = bsafe_div(r[v - ox], dxm) + bsafe_div(r[v + ox], dxp);
                nb += bsafe_div(r[v - sy], dym) + bsafe_div(r[v + sy], dyp);
                if (f.dim == 3) nb += bsafe_div(r[v - sz], dzm) + bsafe_div(r[v + sz], dzp);
                const double z1 = omega * r[v] / d;
                res[v] = (V)(r[v] - (d * z1 - f.s * (omega * nb)));
            }
        }
    }
}

// The per-iteration fine kernels below first read a thread's slot state
// (fixed for the whole kernel: BNT is a multiple of kb), then, per node, issue
// the loads of all its planes before any arithmetic or store, so that the
// planes' loads are in flight together.
template <class T>
struct St {
    T c, xm, xp, ym, yp, zm, zp;
};

template <class T>
__device__ inline St<T> ld_st(const T* __restrict__ a, int64_t v, int64_t ox, int64_t sy, int64_t sz, bool d3) {
    St<T> r;
    r.c = a[v];
    r.xm = a[v - ox];
    r.xp = a[v + ox];
    r.ym = a[v - sy];
    r.yp = a[v + sy];
    r.zm = d3 ? a[v - sz] : T(0);
    r.zp = d3 ? a[v + sz] : T(0);
    return r;
}

template <class T>
__device__ inline St<T> st_zero() {
    return {T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
}

// p_new = z + beta p_old; q = A p_new; partial (p_new, q).
template <class V, int NPL>
__global__ void __launch_bounds__(BNT) kb_pspmv(BFine f, const V* __restrict__ z, const double* __restrict__ pold,
                                                double* __restrict__ pnew, double* __restrict__ q,
                                                const BatchState* __restrict__ st, double* __restrict__ part) {
    const int pb = (int)blockIdx.y * NPL;   // first plane of this block
    const int sb = bseg_base(f);             // first system of this block's segment
    const int jt = (int)threadIdx.x & (f.kb - 1);
    bool act[NPL];
    double beta[NPL], acc[NPL];
#pragma unroll
    for (int jb = 0; jb < NPL; ++jb) {
        const int j = sb + ((pb + jb) << f.lkb) + jt;
        act[jb] = f.done[j] == 0;
        beta[jb] = st->beta[j];
        acc[jb] = 0.0;
    }
    const int64_t ox = f.kb, sy = f.sy * f.kb, sz = f.sz * f.kb;
    const bool d3 = f.dim == 3;
    BNODE_LOOP(f, p, jj, v0) {
        const double d = f.diag[p];
        if (d != 0.0) {
            St<V> zs[NPL];
            St<double> ps[NPL];
#pragma unroll
            for (int jb = 0; jb < NPL; ++jb) {
                zs[jb] = st_zero<V>();
                ps[jb] = st_zero<double>();
                if (!act[jb]) continue;
                const int64_t v = v0 + (pb + jb) * f.plane;
                zs[jb] = ld_st(z, v, ox, sy, sz, d3);
                if (beta[jb] != 0.0) ps[jb] = ld_st(pold, v, ox, sy, sz, d3);
            }
#pragma unroll
            for (int jb = 0; jb < NPL; ++jb) {
                if (!act[jb]) continue;
                const double be = beta[jb];
                auto pv = [&](V zz, double pp) { return be != 0.0 ? (double)zz + be * pp : (double)zz; };
                const St<V>& a = zs[jb];
                const St<double>& b = ps[jb];
                const double pc = pv(a.c, b.c);
                double nb = pv(a.xm, b.xm) + pv(a.xp, b.xp) + pv(a.ym, b.ym) + pv(a.yp, b.yp);
                if (d3) nb += pv(a.zm, b.zm) + pv(a.zp, b.zp);
                const double qv = d * pc - f.s * nb;
                const int64_t v = v0 + (pb + jb) * f.plane;
                pnew[v] = pc;
                q[v] = qv;
                acc[jb] += pc * qv;
            }
        }
    }
    bpartials<NPL>(acc, part, f);
}

// x += alpha p; r_out = r_in - alpha q; res = r_out - A (omega D^-1 r_out).
template <class V, int NPL>
__global__ void __launch_bounds__(BNT) kb_xr_down(BFine f, double* __restrict__ x, const double* __restrict__ rin,
                                                  double* __restrict__ rout, const double* __restrict__ pv,
                                                  const double* __restrict__ q, V* __restrict__ res, double omega,
                                                  const BatchState* __restrict__ st, double* __restrict__ part) {
    const int pb = (int)blockIdx.y * NPL;   // first plane of this block
    const int sb = bseg_base(f);             // first system of this block's segment
    const int jt = (int)threadIdx.x & (f.kb - 1);
    bool act[NPL];
    double alpha[NPL], acc[NPL];
#pragma unroll
    for (int jb = 0; jb < NPL; ++jb) {
        const int j = sb + ((pb + jb) << f.lkb) + jt;
        act[jb] = f.done[j] == 0;
        alpha[jb] = st->alpha[j];
        acc[jb] = 0.0;
    }
    const int64_t ox = f.kb, sy = f.sy * f.kb, sz = f.sz * f.kb;
    const bool d3 = f.dim == 3;
    BNODE_LOOP(f, p, jj, v0) {
        const double d = f.diag[p];
        if (d != 0.0) {
            const double dxm = f.diag[p - 1], dxp = f.diag[p + 1], dym = f.diag[p - f.sy], dyp = f.diag[p + f.sy];
            const double dzm = d3 ? f.diag[p - f.sz] : 0.0, dzp = d3 ? f.diag[p + f.sz] : 0.0;
            St<double> rs[NPL], qs[NPL];
            double xc[NPL], pc[NPL];
#pragma unroll
            for (int jb = 0; jb < NPL; ++jb) {
                rs[jb] = st_zero<double>();
                qs[jb] = st_zero<double>();
                xc[jb] = 0.0;
                pc[jb] = 0.0;
                if (!act[jb]) continue;
                const int64_t v = v0 + (pb + jb) * f.plane;
                xc[jb] = x[v];
                pc[jb] = pv[v];
                rs[jb] = ld_st(rin, v, ox, sy, sz, d3);
                qs[jb] = ld_st(q, v, ox, sy, sz, d3);
            }
#pragma unroll
            for (int jb = 0; jb < NPL; ++jb) {
                if (!act[jb]) continue;
                const double al = alpha[jb];
                const St<double>& a = rs[jb];
                const St<double>& b = qs[jb];
                const int64_t v = v0 + (pb + jb) * f.plane;
                x[v] = xc[jb] + al * pc[jb];
                const double rn = a.c - al * b.c;
                rout[v] = rn;
                acc[jb] += rn * rn;
                double nb = bsafe_div(a.xm - al * b.xm, dxm);
                nb += bsafe_div(a.xp - al * b.xp, dxp);
                nb += bsafe_div(a.ym - al * b.ym, dym);
                nb += bsafe_div(a.yp - al * b.yp, dyp);
                if (d3) {
                    nb += bsafe_div(a.zm - al * b.zm, dzm);
                    nb += bsafe_div(a.zp - al * b.zp, dzp);
                }
                const double z1 = omega * rn / d;
                res[v] = (V)(rn - (d * z1 - f.s * (omega * nb)));
            }
        }
    }
    bpartials<NPL>(acc, part, f);
}

// Restriction r_c = P_tent^T (I - omega A D^-1) res: one thread per
// (level-0 box, rhs).
struct BBox {
    const int32_t* boxes;
    int64_t nboxes;
    int nbx, nby;
    int nx, ny, nz;
    const int32_t* cstart;
    const int32_t* ncomp;
    const int32_t* agg;
};

template <class V, int DIM>
__global__ void __launch_bounds__(256) kb_restrict(BFine f, BBox b, double omega_d, const V* __restrict__ res,
                                                   V* __restrict__ rc) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t bi = t >> f.lkp;
    const int j = (int)(t & (f.kp - 1));
    if (bi >= b.nboxes || (!f.blk_seg && f.done[j])) return;   // (segmented: a box may hold two segments)
    const V* __restrict__ dg = bdiag<V>(f);
    const V omega = (V)omega_d;
    const V sh = (V)f.s;
    const int64_t kp = f.kp;
    const int64_t box = b.boxes[bi];
    const int bx = (int)(box % b.nbx);
    const int64_t rq = box / b.nbx;
    const int by = (int)(rq % b.nby);
    const int bz = (int)(rq / b.nby);
    const int32_t c0 = b.cstart[box];
    const int m = b.ncomp[box];
    if (DIM == 2) {
        // The box's 3 x 3 nodes and their neighbours (a 5 x 5 window without
        // its corners) are loaded first; window points off the node grid read
        // as 0 (they neighbour no unknown: the outer node layer is outside).
        // Each node's contribution u goes to its component; the components'
        // sums are then formed in node order.
        V rw[5][5], dw[5][5];
#pragma unroll
        for (int a = 0; a < 5; ++a)
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                rw[a][c] = V(0);
                dw[a][c] = V(0);
                if ((a == 0 || a == 4) && (c == 0 || c == 4)) continue;
                const int i = 3 * bx - 1 + c, jj = 3 * by - 1 + a;
                if (i < 0 || i >= b.nx || jj < 0 || jj >= b.ny) continue;
                const int64_t p = (int64_t)i + f.sy * jj;
                dw[a][c] = dg[p];
                rw[a][c] = res[bvidx(f, p, j)];
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
                V nb = bsafe_div(rw[a][c - 1], dw[a][c - 1]) + bsafe_div(rw[a][c + 1], dw[a][c + 1]);
                nb += bsafe_div(rw[a - 1][c], dw[a - 1][c]) + bsafe_div(rw[a + 1][c], dw[a + 1][c]);
                const V aw = d * (rp / d) - sh * nb;
                u[n] = rp - omega * aw;
                comp[n] = m == 1 ? 0 : b.agg[(int64_t)(3 * bx + ox) + f.sy * (3 * by + oy)] - c0;
            }
        for (int c = 0; c < m && c < BMAX_FINE_COMP; ++c) {
            V a = V(0);
#pragma unroll
            for (int n = 0; n < 9; ++n)
                if (comp[n] == c) a += u[n];
            rc[(int64_t)(c0 + c) * kp + j] = a;
        }
    } else {
        const int64_t dx = f.kb, dy = f.sy * f.kb, dz = f.sz * f.kb;   // fine-index strides
        V acc[BMAX_FINE_COMP];
#pragma unroll
        for (int c = 0; c < BMAX_FINE_COMP; ++c) acc[c] = V(0);
        for (int oz = 0; oz < 3; ++oz) {
            const int k = 3 * bz + oz;
            if (k >= b.nz) break;
            for (int oy = 0; oy < 3; ++oy) {
                const int jj = 3 * by + oy;
                if (jj >= b.ny) break;
                for (int ox = 0; ox < 3; ++ox) {
                    const int i = 3 * bx + ox;
                    if (i >= b.nx) break;
                    const int64_t p = (int64_t)i + f.sy * jj + f.sz * k;
                    const V d = dg[p];
                    if (d == V(0)) continue;
                    const int64_t v = bvidx(f, p, j);
                    const V rp = res[v];
                    V nb = bsafe_div(res[v - dx], dg[p - 1]) + bsafe_div(res[v + dx], dg[p + 1]);
                    nb += bsafe_div(res[v - dy], dg[p - f.sy]) + bsafe_div(res[v + dy], dg[p + f.sy]);
                    nb += bsafe_div(res[v - dz], dg[p - f.sz]) + bsafe_div(res[v + dz], dg[p + f.sz]);
                    const V aw = d * (rp / d) - sh * nb;
                    const V uu = rp - omega * aw;
                    if (m == 1) {
                        acc[0] += uu;
                    } else {
                        const int c = b.agg[p] - c0;
                        if (c >= 0 && c < BMAX_FINE_COMP) acc[c] += uu;
                    }
                }
            }
        }
        for (int c = 0; c < m && c < BMAX_FINE_COMP; ++c) rc[(int64_t)(c0 + c) * kp + j] = acc[c];
    }
}

// zt = omega r / d + t - omega (A t) / d, t = e_c[agg]; the aggregate ids of
// the five (seven) stencil points are read once for all planes.
template <class V, int NPL>
__global__ void __launch_bounds__(BNT) kb_fine_up(BFine f, double omega_d, const int32_t* __restrict__ agg,
                                                  const V* __restrict__ ec, const double* __restrict__ r,
                                                  V* __restrict__ zt) {
    const int pb = (int)blockIdx.y * NPL;   // first plane of this block
    const int sb = bseg_base(f);             // first system of this block's segment
    const int jt = (int)threadIdx.x & (f.kb - 1);
    const V* __restrict__ dg = bdiag<V>(f);
    const V omega = (V)omega_d;
    const int64_t kp = f.kp;
    const bool d3 = f.dim == 3;
    bool act[NPL];
#pragma unroll
    for (int jb = 0; jb < NPL; ++jb) act[jb] = f.done[sb + ((pb + jb) << f.lkb) + jt] == 0;
    BNODE_LOOP(f, p, jj, v0) {
        const V d = dg[p];
        if (d != V(0)) {
            const int32_t g0 = agg[p], g1 = agg[p - 1], g2 = agg[p + 1], g3 = agg[p - f.sy], g4 = agg[p + f.sy];
            const int32_t g5 = d3 ? agg[p - f.sz] : -1, g6 = d3 ? agg[p + f.sz] : -1;
            St<V> ts[NPL];
            double rv[NPL];
#pragma unroll
            for (int jb = 0; jb < NPL; ++jb) {
                ts[jb] = st_zero<V>();
                rv[jb] = 0.0;
                if (!act[jb]) continue;
                const int j = ((pb + jb) << f.lkb) + jt;
                auto t_at = [&](int32_t g) { return g >= 0 ? ec[(int64_t)g * kp + j] : V(0); };
                ts[jb] = {t_at(g0), t_at(g1), t_at(g2), t_at(g3), t_at(g4), t_at(g5), t_at(g6)};
                rv[jb] = r[v0 + (pb + jb) * f.plane];
            }
#pragma unroll
            for (int jb = 0; jb < NPL; ++jb) {
                if (!act[jb]) continue;
                const St<V>& t = ts[jb];
                V nb = t.xm + t.xp + t.ym + t.yp;
                if (d3) nb += t.zm + t.zp;
                const V at = d * t.c - (V)f.s * nb;
                zt[v0 + (pb + jb) * f.plane] = omega * (V)rv[jb] / d + (t.c - omega * at / d);
            }
        }
    }
}

// z = zt + omega (r - A zt) / d; partial (r, z) per rhs.
template <class V, int NPL>
__global__ void __launch_bounds__(BNT) kb_fine_post(BFine f, double omega_d, const V* __restrict__ zt,
                                                    const double* __restrict__ r, V* __restrict__ z,
                                                    double* __restrict__ part) {
    const int pb = (int)blockIdx.y * NPL;   // first plane of this block
    const int sb = bseg_base(f);             // first system of this block's segment
    const int jt = (int)threadIdx.x & (f.kb - 1);
    const V* __restrict__ dg = bdiag<V>(f);
    const V omega = (V)omega_d;
    const V sh = (V)f.s;
    const int64_t ox = f.kb, sy = f.sy * f.kb, sz = f.sz * f.kb;
    const bool d3 = f.dim == 3;
    bool act[NPL];
    double acc[NPL];
#pragma unroll
    for (int jb = 0; jb < NPL; ++jb) {
        act[jb] = f.done[sb + ((pb + jb) << f.lkb) + jt] == 0;
        acc[jb] = 0.0;
    }
    BNODE_LOOP(f, p, jj, v0) {
        const V d = dg[p];
        if (d != V(0)) {
            St<V> zs[NPL];
            double rv[NPL];
#pragma unroll
            for (int jb = 0; jb < NPL; ++jb) {
                zs[jb] = st_zero<V>();
                rv[jb] = 0.0;
                if (!act[jb]) continue;
                const int64_t v = v0 + (pb + jb) * f.plane;
                zs[jb] = ld_st(zt, v, ox, sy, sz, d3);
                rv[jb] = r[v];
            }
#pragma unroll
            for (int jb = 0; jb < NPL; ++jb) {
                if (!act[jb]) continue;
                const St<V>& a = zs[jb];
                V nb = a.xm + a.xp + a.ym + a.yp;
                if (d3) nb += a.zm + a.zp;
                const V az = d * a.c - sh * nb;
                const V zv = a.c + omega * ((V)rv[jb] - az) / d;
                z[v0 + (pb + jb) * f.plane] = zv;
                acc[jb] += rv[jb] * (double)zv;
            }
        }
    }
    bpartials<NPL>(acc, part, f);
}

// ---------------------------------------------------------- coarse kernels
// One thread per (row, rhs); the lanes of a wavefront share the row's entries.
template <class V>
struct BCsr {
    const int32_t* rowptr;
    const int32_t* col;
    const V* val;
};

#define BROW(n, lkp, kp, done, row, j)                          \
    const int64_t t_ = (int64_t)blockIdx.x * BNT + threadIdx.x;   \
    const int64_t row = t_ >> (lkp);                              \
    const int j = (int)(t_ & ((kp) - 1));                         \
    if (row >= (n) || ((done) && (done)[j])) return;

template <class V>
__global__ void __launch_bounds__(BNT) kb_csr_resid(int64_t n, int lkp, int kp, const int32_t* __restrict__ done,
                                                    BCsr<V> A, const V* __restrict__ diag, V omega,
                                                    const V* __restrict__ rv, V* __restrict__ res) {
    BROW(n, lkp, kp, done, row, j)
    V az = V(0);
    for (int e = A.rowptr[row]; e < A.rowptr[row + 1]; ++e) {
        const int k = A.col[e];
        az += A.val[e] * (omega * rv[(int64_t)k * kp + j] / diag[k]);
    }
    res[row * kp + j] = rv[row * kp + j] - az;
}

template <class V>
__global__ void __launch_bounds__(BNT) kb_csr_matvec(int64_t n, int lkp, int kp, const int32_t* __restrict__ done,
                                                     BCsr<V> M, const V* __restrict__ x, V* __restrict__ y) {
    BROW(n, lkp, kp, done, row, j)
    V acc = V(0);
    for (int e = M.rowptr[row]; e < M.rowptr[row + 1]; ++e) acc += M.val[e] * x[(int64_t)M.col[e] * kp + j];
    y[row * kp + j] = acc;
}

template <class V>
__global__ void __launch_bounds__(BNT) kb_csr_prolong(int64_t n, int lkp, int kp, const int32_t* __restrict__ done,
                                                      BCsr<V> P, const V* __restrict__ diag, V omega,
                                                      const V* __restrict__ rv, const V* __restrict__ ev_c,
                                                      V* __restrict__ zt) {
    BROW(n, lkp, kp, done, row, j)
    V acc = V(0);
    for (int e = P.rowptr[row]; e < P.rowptr[row + 1]; ++e) acc += P.val[e] * ev_c[(int64_t)P.col[e] * kp + j];
    zt[row * kp + j] = omega * rv[row * kp + j] / diag[row] + acc;
}

template <class V>
__global__ void __launch_bounds__(BNT) kb_csr_post(int64_t n, int lkp, int kp, const int32_t* __restrict__ done,
                                                   BCsr<V> A, const V* __restrict__ diag, V omega,
                                                   const V* __restrict__ rv, const V* __restrict__ zt,
                                                   V* __restrict__ ev) {
    BROW(n, lkp, kp, done, row, j)
    V az = V(0);
    for (int e = A.rowptr[row]; e < A.rowptr[row + 1]; ++e) az += A.val[e] * zt[(int64_t)A.col[e] * kp + j];
    ev[row * kp + j] = zt[row * kp + j] + omega * (rv[row * kp + j] - az) / diag[row];
}

// Coarsest: ev = W rv (W FP64, FP64 accumulation).
// Island hierarchies: ev = W_b rv on the rows of each island that ends on
// this level (the single solve's k_block_apply, every rhs).
template <class V>
__global__ void __launch_bounds__(BNT) kb_block(int64_t n, int lkp, int kp, const int32_t* __restrict__ done,
                                                const int32_t* __restrict__ blk_of, const int32_t* __restrict__ blk,
                                                const int64_t* __restrict__ woff, const double* __restrict__ W,
                                                const V* __restrict__ rv, V* __restrict__ ev) {
    BROW(n, lkp, kp, done, row, j)
    const int b = blk_of[row];
    if (b < 0) return;
    const int o = blk[2 * b], m = blk[2 * b + 1];
    const double* Wr = W + woff[b] + (int64_t)(row - o) * m;
    double acc = 0.0;
    for (int c = 0; c < m; ++c) acc += Wr[c] * (double)rv[(int64_t)(o + c) * kp + j];
    ev[row * kp + j] = (V)acc;
}

template <class V>
__global__ void __launch_bounds__(BNT) kb_dense(int64_t n, int lkp, int kp, const int32_t* __restrict__ done,
                                                const double* __restrict__ W, const V* __restrict__ rv,
                                                V* __restrict__ ev) {
    BROW(n, lkp, kp, done, row, j)
    double acc = 0.0;
    for (int64_t m = 0; m < n; ++m) acc += W[row * n + m] * (double)rv[m * kp + j];
    ev[row * kp + j] = (V)acc;
}

// One-level hierarchies: gather r to compact order and scatter z back.
template <class V>
__global__ void __launch_bounds__(BNT) kb_gather(BFine f, int64_t n, int lkp, int kp, const int32_t* __restrict__ done,
                                                 const int32_t* __restrict__ pad, const double* __restrict__ src,
                                                 V* __restrict__ dst) {
    BROW(n, lkp, kp, done, k, j)
    dst[k * kp + j] = (V)src[bvidx(f, pad[k], j)];
}

template <class V>
__global__ void __launch_bounds__(BNT) kb_scatter_dot(BFine f, int64_t n, int lkp, int kp,
                                                      const int32_t* __restrict__ done,
                                                      const int32_t* __restrict__ pad, const V* __restrict__ ev,
                                                      const double* __restrict__ r, V* __restrict__ z,
                                                      double* __restrict__ part) {
    // fixed grid: each block strides over the (unknown, rhs) pairs
    double acc = 0.0;
    const int64_t total = n << lkp;
    for (int64_t t = (int64_t)blockIdx.x * BNT + threadIdx.x; t < total; t += (int64_t)gridDim.x * BNT) {
        const int64_t k = t >> lkp;
        const int j = (int)(t & (kp - 1));
        if (done[j]) continue;
        const int64_t v = bvidx(f, pad[k], j);
        z[v] = ev[k * kp + j];
        acc += r[v] * (double)ev[k * kp + j];
    }
    bpartial_kp(acc, part, kp);
}

// Node fields <-> interleaved padded layout.
__global__ void __launch_bounds__(BNT) kb_load(BFine f, int64_t nunk, int lkp, int kp, int nrhs, int64_t nn,
                                               const int64_t* __restrict__ nodes, const int32_t* __restrict__ pad,
                                               const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * BNT + threadIdx.x;
    const int64_t k = t >> lkp;
    const int j = (int)(t & (kp - 1));
    if (k >= nunk) return;
    dst[bvidx(f, pad[k], j)] = j < nrhs ? src[(int64_t)j * nn + nodes[k]] : 0.0;
}

__global__ void __launch_bounds__(BNT) kb_store(BFine f, int64_t nunk, int lkp, int kp, int nrhs, int64_t nn,
                                                const int64_t* __restrict__ nodes, const int32_t* __restrict__ pad,
                                                const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * BNT + threadIdx.x;
    const int64_t k = t >> lkp;
    const int j = (int)(t & (kp - 1));
    if (k >= nunk || j >= nrhs) return;
    dst[(int64_t)j * nn + nodes[k]] = src[bvidx(f, pad[k], j)];
}

// ---------------------------------------------------------------- host side
// Device addresses of BatchState members (no host dereference of B->st).
static int32_t* st_done(BatchBufs* B) {
    return reinterpret_cast<int32_t*>(reinterpret_cast<char*>(B->st) + offsetof(BatchState, done));
}
static int32_t* st_mask(BatchBufs* B) {
    return reinterpret_cast<int32_t*>(reinterpret_cast<char*>(B->st) + offsetof(BatchState, mask));
}

static int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

void drop_batch_graph(amg_handle* H) {
    BatchBufs* B = H->batch;
    if (B && B->it_graph) {
        (void)hipGraphExecDestroy(B->it_graph);
        B->it_graph = nullptr;
    }
}

void free_batch(amg_handle* H, hipStream_t s) {
    BatchBufs* B = H->batch;
    if (!B) return;
    void* ptrs[] = {B->x, B->rr[0], B->rr[1], B->p[0], B->p[1], B->q, B->bvec, B->tres, B->res, B->zt, B->z,
                    B->part[0], B->part[1], B->part[2], B->part_aux, B->st, B->blk_start, B->blk_seg, B->seg_blk};
    for (void* p : ptrs) (void)dfree(p, s);
    for (int l = 0; l < MAX_LEVELS; ++l) {
        (void)dfree(B->rv[l], s);
        (void)dfree(B->ev[l], s);
        (void)dfree(B->tmp[l], s);
    }
    if (B->it_graph) (void)hipGraphExecDestroy(B->it_graph);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    delete B->host;
    delete B;
    H->batch = nullptr;
}

// Segment tables.  The fine strips are sorted by node, hence by node row, so
// each segment (a run of node rows) owns a contiguous run of strips.  Every
// segment gets a share of about BPARTS blocks proportional to its strips (at
// least one, at most BPARTS), its strips split evenly among them; the block
// count is padded to a multiple of the XCD count with empty blocks of the
// last segment.  rows: nseg + 1 increasing node-row bounds (host).
static int make_segments(amg_handle* H, BatchBufs* B, int nseg, const int32_t* rows, hipStream_t s) {
    std::vector<int32_t> seg_blk((size_t)nseg + 1);
    if (nseg == 1 && !rows) {
        B->nblk = BPARTS;
        seg_blk[0] = 0;
        seg_blk[1] = BPARTS;
    } else {
        const int64_t n = H->nstrips;
        std::vector<int32_t> ids((size_t)(n > 0 ? n : 1));
        if (n > 0) {
            EB_HIP(hipMemcpyAsync(ids.data(), H->strips, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
            EB_HIP(hipStreamSynchronize(s));
        }
        const int64_t per_row = H->px / H->strip_w;
        std::vector<int64_t> first((size_t)nseg + 1, n);
        int sg = 0;
        for (int64_t k = 0; k < n; ++k) {
            const int64_t row = ids[k] / per_row;
            if (row < rows[0] || row >= rows[nseg]) {
                set_error("pcg_solve_islands: an unknown lies in node row %lld, outside the segments",
                          (long long)row);
                return EB_EINVAL;
            }
            while (row >= rows[sg + 1]) ++sg;
            for (int t = sg; t >= 0 && first[t] == n; --t) first[t] = k;
        }
        for (int t = nseg - 1; t >= 0; --t)
            if (first[t] > first[t + 1]) first[t] = first[t + 1];
        std::vector<int32_t> bstart, bseg;
        for (int t = 0; t < nseg; ++t) {
            const int64_t k0 = first[t], k1 = first[t + 1], cnt = k1 - k0;
            int64_t nb = n > 0 ? (int64_t)BPARTS * cnt / n : 1;
            // at most BPARTS - NUM_XCD, so that with the padding blocks a
            // segment never exceeds the BPARTS partials a finaliser sums
            nb = nb < 1 ? 1 : (nb > BPARTS - NUM_XCD ? BPARTS - NUM_XCD : nb);
            seg_blk[t] = (int32_t)bstart.size();
            for (int64_t i = 0; i < nb; ++i) {
                bstart.push_back((int32_t)(k0 + i * cnt / nb));
                bseg.push_back(t);
            }
        }
        while (bstart.size() % NUM_XCD != 0 || bstart.empty()) {
            bstart.push_back((int32_t)n);
            bseg.push_back(nseg - 1);
        }
        seg_blk[nseg] = (int32_t)bstart.size();
        B->nblk = (int)bstart.size();
        bstart.push_back((int32_t)n);
        EB_TRY(dalloc_n(&B->blk_start, (int64_t)bstart.size(), s));
        EB_TRY(dalloc_n(&B->blk_seg, (int64_t)bseg.size(), s));
        EB_HIP(hipMemcpyAsync(B->blk_start, bstart.data(), sizeof(int32_t) * bstart.size(), hipMemcpyHostToDevice, s));
        EB_HIP(hipMemcpyAsync(B->blk_seg, bseg.data(), sizeof(int32_t) * bseg.size(), hipMemcpyHostToDevice, s));
        EB_HIP(hipStreamSynchronize(s));   // the host vectors are freed on return
    }
    EB_TRY(dalloc_n(&B->seg_blk, (int64_t)nseg + 1, s));
    EB_HIP(hipMemcpyAsync(B->seg_blk, seg_blk.data(), sizeof(int32_t) * (nseg + 1), hipMemcpyHostToDevice, s));
    EB_HIP(hipStreamSynchronize(s));
    B->nseg = nseg;
    B->seg_rows.assign(rows ? rows : seg_blk.data(), rows ? rows + nseg + 1 : seg_blk.data());
    return EB_OK;
}

// Buffers for kp slots with V-cycle element size vb (8 or 4 bytes) and the
// given segmentation (nseg = 1, rows = null: no segments).
static int ensure_batch(amg_handle* H, int kp, int prec, int nseg, const int32_t* rows, hipStream_t s) {
    if (H->batch && H->batch->kp == kp && H->batch->prec == prec && H->batch->nseg == nseg) {
        const std::vector<int32_t>& have = H->batch->seg_rows;
        if (!rows ? have.empty() : (have.size() == (size_t)nseg + 1 && std::equal(have.begin(), have.end(), rows)))
            return EB_OK;
    }
    free_batch(H, s);
    BatchBufs* B = new BatchBufs();
    H->batch = B;
    B->kp = kp;
    B->prec = prec;
    B->host = new BatchState();
    EB_TRY(make_segments(H, B, nseg, rows, s));
    const int64_t nv = H->npad * kp;
    const size_t vb = prec == EB_PREC_FP32 ? sizeof(float) : sizeof(double);
    // read at neighbours without a guard: zero off unknowns
    double** zeroed[] = {&B->x, &B->p[0], &B->p[1], &B->rr[0], &B->rr[1]};
    for (double** v : zeroed) {
        EB_TRY(dalloc_n(v, nv, s));
        EB_HIP(hipMemsetAsync(*v, 0, sizeof(double) * nv, s));
    }
    EB_TRY(dalloc_n(&B->q, nv, s));
    EB_HIP(hipMemsetAsync(B->q, 0, sizeof(double) * nv, s));
    EB_TRY(dalloc_n(&B->bvec, nv, s));
    EB_HIP(hipMemsetAsync(B->bvec, 0, sizeof(double) * nv, s));
    EB_TRY(dalloc_n(&B->tres, nv, s));
    void** vzeroed[] = {&B->zt, &B->z, &B->res};
    for (void** v : vzeroed) {
        EB_TRY(dalloc(v, vb * (size_t)nv, s));
        EB_HIP(hipMemsetAsync(*v, 0, vb * (size_t)nv, s));
    }
    for (int l = (H->nlev > 1 ? 1 : 0); l < H->nlev; ++l) {
        const int64_t n = (H->lev[l].n > 0 ? H->lev[l].n : 1) * kp;
        EB_TRY(dalloc(&B->rv[l], vb * (size_t)n, s));
        EB_TRY(dalloc(&B->ev[l], vb * (size_t)n, s));
        EB_TRY(dalloc(&B->tmp[l], vb * (size_t)n, s));
    }
    const int64_t nparts = (int64_t)(B->nblk > BPARTS ? B->nblk : BPARTS) * kp;
    for (int i = 0; i < 3; ++i) EB_TRY(dalloc_n(&B->part[i], nparts, s));
    EB_TRY(dalloc_n(&B->part_aux, nparts, s));
    EB_TRY(dalloc_n(&B->st, 1, s));
    EB_HIP(hipMemsetAsync(B->st, 0, sizeof(BatchState), s));
    return EB_OK;
}

static BFine bfine(const amg_handle* H, const BatchBufs* B, bool full, unsigned* grid) {
    BFine f;
    f.strips = H->strips;
    f.nstrips = H->nstrips;
    f.strip_w = H->strip_w;
    f.kp = B->kp;
    f.lkp = ilog2(B->kp);
    f.kb = B->kp < B->kbw ? B->kp : B->kbw;
    f.lkb = ilog2(f.kb);
    f.plane = H->npad * f.kb;
    f.lsw0 = ilog2(H->strip_w);
    f.lsw = f.lsw0 + f.lkp;
    f.sy = H->px;
    f.sz = (int64_t)H->px * H->d.ny;
    f.dim = H->d.dim;
    f.s = H->d.s;
    f.diag = H->diag_p;
    f.diag32 = H->diag_p32;
    f.done = st_done(const_cast<BatchBufs*>(B));
    f.blk_start = nullptr;
    f.blk_seg = nullptr;
    if (B->blk_start) {
        f.blk_start = B->blk_start;
        f.blk_seg = B->blk_seg;
        f.spb = 0;
        *grid = (unsigned)B->nblk;
        return f;
    }
    if (full) {
        // one element per thread
        const int64_t per_block = BNT / ((int64_t)H->strip_w * f.kb);
        if (per_block >= 1) {
            f.spb = per_block;
            int64_t g = (H->nstrips + per_block - 1) / per_block;
            g = (g + NUM_XCD - 1) / NUM_XCD * NUM_XCD;
            *grid = (unsigned)(g > 0 ? g : NUM_XCD);
            return f;
        }
    }
    f.spb = (H->nstrips + BPARTS - 1) / BPARTS;
    *grid = BPARTS;
    return f;
}

static BBox bbox(const amg_handle* H) {
    BBox b;
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

template <class V> static BCsr<V> bcsr_a(const Level& L);
template <class V> static BCsr<V> bcsr_p(const Level& L);
template <class V> static BCsr<V> bcsr_r(const Level& L);
template <class V> static const V* bldiag(const Level& L);
template <> BCsr<double> bcsr_a<double>(const Level& L) { return {L.a_rowptr, L.a_col, L.a_val}; }
template <> BCsr<double> bcsr_p<double>(const Level& L) { return {L.p_rowptr, L.p_col, L.p_val}; }
template <> BCsr<double> bcsr_r<double>(const Level& L) { return {L.r_rowptr, L.r_col, L.r_val}; }
template <> const double* bldiag<double>(const Level& L) { return L.diag; }
template <> BCsr<float> bcsr_a<float>(const Level& L) { return {L.a_rowptr, L.a_col, L.a_val32}; }
template <> BCsr<float> bcsr_p<float>(const Level& L) { return {L.p_rowptr, L.p_col, L.p_val32}; }
template <> BCsr<float> bcsr_r<float>(const Level& L) { return {L.r_rowptr, L.r_col, L.r_val32}; }
template <> const float* bldiag<float>(const Level& L) { return L.diag32; }

// Launch a fine kernel instantiated for NPL planes per block (1, 2 or 4;
// the grid's y dimension covers the other planes).
constexpr int BMAX_NPB = 4;
#define BLAUNCH_V(KERNEL, V, npl, grid, ...)                                                       \
    do {                                                                                           \
        switch (npl) {                                                                             \
            case 1: hipLaunchKernelGGL((KERNEL<V, 1>), grid, dim3(BNT), 0, s, __VA_ARGS__); break; \
            case 2: hipLaunchKernelGGL((KERNEL<V, 2>), grid, dim3(BNT), 0, s, __VA_ARGS__); break; \
            default: hipLaunchKernelGGL((KERNEL<V, 4>), grid, dim3(BNT), 0, s, __VA_ARGS__); break; \
        }                                                                                          \
    } while (0)
#define BLAUNCH_N(KERNEL, npl, grid, ...)                                                       \
    do {                                                                                        \
        switch (npl) {                                                                          \
            case 1: hipLaunchKernelGGL((KERNEL<1>), grid, dim3(BNT), 0, s, __VA_ARGS__); break; \
            case 2: hipLaunchKernelGGL((KERNEL<2>), grid, dim3(BNT), 0, s, __VA_ARGS__); break; \
            default: hipLaunchKernelGGL((KERNEL<4>), grid, dim3(BNT), 0, s, __VA_ARGS__); break; \
        }                                                                                       \
    } while (0)

// Planes per block and the grid of a fine kernel (y: plane groups).
static int npl_of(const BFine& f, const BatchBufs* B) {
    int n = f.kp / f.kb;
    if (B->npb < n) n = B->npb;
    return n < BMAX_NPB ? n : BMAX_NPB;
}
static dim3 bgrid(unsigned gx, const BFine& f, const BatchBufs* B) {
    return dim3(gx, (unsigned)((f.kp / f.kb) / npl_of(f, B)));
}

static unsigned rows_grid(int64_t rows, int kp) {
    const int64_t t = rows * kp;
    return (unsigned)((t + BNT - 1) / BNT > 0 ? (t + BNT - 1) / BNT : 1);
}

// z = M r for every active rhs; the (r, z) partials go to part.
template <class V>
static int benqueue_vcycle(amg_handle* H, BatchBufs* B, const double* r, int initial, double* part, hipStream_t s) {
    const int kp = B->kp, lkp = ilog2(kp);
    // coarse vectors hold every segment's rows: with segments nothing is skipped there
    const int32_t* done = B->blk_seg ? nullptr : st_done(B);
    V* z = (V*)B->z;
    if (H->nlev == 1) {
        const Level& L = H->lev[0];
        V* rv = (V*)B->rv[0];
        V* ev = (V*)B->ev[0];
        unsigned gq = 0;
        const BFine fq = bfine(H, B, false, &gq);
        hipLaunchKernelGGL(kb_gather<V>, dim3(rows_grid(L.n, kp)), dim3(BNT), 0, s, fq, L.n, lkp, kp, done,
                           H->fine_pad, r, rv);
        hipLaunchKernelGGL(kb_dense<V>, dim3(rows_grid(L.n, kp)), dim3(BNT), 0, s, L.n, lkp, kp, done, L.dense_inv,
                           (const V*)rv, ev);
        hipLaunchKernelGGL(kb_scatter_dot<V>, dim3(BPARTS), dim3(BNT), 0, s, fq, L.n, lkp, kp, done, H->fine_pad,
                           (const V*)ev, r, z, part);
        EB_LAUNCH_CHECK();
        return EB_OK;
    }
    unsigned gfull = 0;
    const BFine ff = bfine(H, B, true, &gfull);
    unsigned gfix = 0;
    const BFine fr = bfine(H, B, false, &gfix);
    const double w0 = H->lev[0].omega;
    if (initial) {
        BLAUNCH_V(kb_fine_down, V, npl_of(ff, B), bgrid(gfull, ff, B), ff, w0, r, (V*)B->res);
    }
    const BBox bx = bbox(H);
    const int64_t nbt = H->nboxes0 * kp;
    const dim3 grx((unsigned)((nbt + 255) / 256 > 0 ? (nbt + 255) / 256 : 1));
    if (H->d.dim == 2)
        hipLaunchKernelGGL((kb_restrict<V, 2>), grx, dim3(256), 0, s, ff, bx, w0, (const V*)B->res, (V*)B->rv[1]);
    else
        hipLaunchKernelGGL((kb_restrict<V, 3>), grx, dim3(256), 0, s, ff, bx, w0, (const V*)B->res, (V*)B->rv[1]);
    for (int l = 1; l < H->nlev - 1; ++l) {
        const Level& L = H->lev[l];
        const Level& C = H->lev[l + 1];
        const V w = (V)L.omega;
        hipLaunchKernelGGL(kb_csr_resid<V>, dim3(rows_grid(L.n, kp)), dim3(BNT), 0, s, L.n, lkp, kp, done,
                           bcsr_a<V>(L), bldiag<V>(L), w, (const V*)B->rv[l], (V*)B->tmp[l]);
        hipLaunchKernelGGL(kb_csr_matvec<V>, dim3(rows_grid(C.n, kp)), dim3(BNT), 0, s, C.n, lkp, kp, done,
                           bcsr_r<V>(L), (const V*)B->tmp[l], (V*)B->rv[l + 1]);
    }
    {
        const Level& Lc = H->lev[H->nlev - 1];
        if (Lc.fz_all)
            hipLaunchKernelGGL(kb_block<V>, dim3(rows_grid(Lc.n, kp)), dim3(BNT), 0, s, Lc.n, lkp, kp, done,
                               (const int32_t*)Lc.fz_blk, (const int32_t*)Lc.fz_off, (const int64_t*)Lc.fz_woff,
                               (const double*)Lc.fz_inv, (const V*)B->rv[H->nlev - 1], (V*)B->ev[H->nlev - 1]);
        else
            hipLaunchKernelGGL(kb_dense<V>, dim3(rows_grid(Lc.n, kp)), dim3(BNT), 0, s, Lc.n, lkp, kp, done,
                               Lc.dense_inv, (const V*)B->rv[H->nlev - 1], (V*)B->ev[H->nlev - 1]);
    }
    for (int l = H->nlev - 2; l >= 1; --l) {
        const Level& L = H->lev[l];
        const V w = (V)L.omega;
        hipLaunchKernelGGL(kb_csr_prolong<V>, dim3(rows_grid(L.n, kp)), dim3(BNT), 0, s, L.n, lkp, kp, done,
                           bcsr_p<V>(L), bldiag<V>(L), w, (const V*)B->rv[l], (const V*)B->ev[l + 1], (V*)B->tmp[l]);
        hipLaunchKernelGGL(kb_csr_post<V>, dim3(rows_grid(L.n, kp)), dim3(BNT), 0, s, L.n, lkp, kp, done,
                           bcsr_a<V>(L), bldiag<V>(L), w, (const V*)B->rv[l], (const V*)B->tmp[l], (V*)B->ev[l]);
        if (L.nfz > 0)
            hipLaunchKernelGGL(kb_block<V>, dim3(rows_grid(L.n, kp)), dim3(BNT), 0, s, L.n, lkp, kp, done,
                               (const int32_t*)L.fz_blk, (const int32_t*)L.fz_off, (const int64_t*)L.fz_woff,
                               (const double*)L.fz_inv, (const V*)B->rv[l], (V*)B->ev[l]);
    }
    BLAUNCH_V(kb_fine_up, V, npl_of(ff, B), bgrid(gfull, ff, B), ff, w0, H->agg_p, (const V*)B->ev[1], r, (V*)B->zt);
    BLAUNCH_V(kb_fine_post, V, npl_of(fr, B), bgrid(gfix, fr, B), fr, w0, (const V*)B->zt, r, z, part);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// Iteration k >= 1 (ping-pong as in the single solve).
template <class V>
static int benqueue_iteration(amg_handle* H, BatchBufs* B, int k, hipStream_t s) {
    const int kp = B->kp;
    unsigned gfix = 0;
    const BFine fr = bfine(H, B, false, &gfix);
    double* pold = B->p[k & 1];
    double* pnew = B->p[(k + 1) & 1];
    double* rin = B->rr[(k - 1) & 1];
    double* rout = B->rr[k & 1];
    BLAUNCH_V(kb_pspmv, V, npl_of(fr, B), bgrid(gfix, fr, B), fr, (const V*)B->z, pold, pnew, B->q, (const BatchState*)B->st,
              B->part[0]);
    hipLaunchKernelGGL(kb_fin_pq, dim3(B->nseg), dim3(BFIN), 0, s, B->st, B->part[0], B->seg_blk, kp);
    // (with one level the fused pre-smoothing residual is formed but not used)
    BLAUNCH_V(kb_xr_down, V, npl_of(fr, B), bgrid(gfix, fr, B), fr, B->x, rin, rout, pnew, B->q, (V*)B->res, H->lev[0].omega,
              (const BatchState*)B->st, B->part[1]);
    hipLaunchKernelGGL(kb_fin_rr, dim3(B->nseg), dim3(BFIN), 0, s, B->st, B->part[1], B->seg_blk, kp);
    if (B->nseg > 1) hipLaunchKernelGGL(kb_fin_count, dim3(1), dim3(BFIN), 0, s, B->st);
    EB_LAUNCH_CHECK();
    EB_TRY(benqueue_vcycle<V>(H, B, rout, 0, B->part[2], s));
    hipLaunchKernelGGL(kb_fin_rz, dim3(B->nseg), dim3(BFIN), 0, s, B->st, B->part[2], B->seg_blk, kp, 0);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// Iterations k and k + 1 (k odd, k >= 3) as one replay of a captured graph;
// captured on the first use and again after a change of launch shape, on a
// private stream (the solve stream may be the null stream, which cannot
// capture).  Kernel nodes only.
template <class V>
static int blaunch_iteration_pair(amg_handle* H, BatchBufs* B, hipStream_t s) {
    if (!B->it_graph || B->it_graph_kbw != B->kbw || B->it_graph_npb != B->npb) {
        if (B->it_graph) (void)hipGraphExecDestroy(B->it_graph);
        B->it_graph = nullptr;
        if (!B->cap_stream) EB_HIP(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
        hipStream_t cs = B->cap_stream;
        hipGraph_t g = nullptr;
        EB_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        const int rc1 = benqueue_iteration<V>(H, B, 3, cs);
        const int rc2 = rc1 == EB_OK ? benqueue_iteration<V>(H, B, 4, cs) : rc1;
        const hipError_t ec = hipStreamEndCapture(cs, &g);
        if (rc2 != EB_OK || ec != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            if (rc2 != EB_OK) return rc2;
            set_error("batched iteration graph capture failed: %s", hipGetErrorString(ec));
            return EB_EHIP;
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            set_error("batched iteration graph instantiation failed: %s", hipGetErrorString(ei));
            return EB_EHIP;
        }
        B->it_graph = ex;
        B->it_graph_kbw = B->kbw;
        B->it_graph_npb = B->npb;
    }
    EB_HIP(hipGraphLaunch(B->it_graph, s));
    return EB_OK;
}

// (Re)start for the slots whose mask is set: r0 = b - A x, norms, first V-cycle.
template <class V>
static int benqueue_start(amg_handle* H, BatchBufs* B, double tol, hipStream_t s) {
    const int kp = B->kp;
    unsigned gfix = 0;
    const BFine fr = bfine(H, B, false, &gfix);
    BLAUNCH_N(kb_norm2, npl_of(fr, B), bgrid(gfix, fr, B), fr, B->bvec, B->part_aux);
    BLAUNCH_N(kb_resid, npl_of(fr, B), bgrid(gfix, fr, B), fr, B->bvec, B->x, B->rr[0], B->part[1]);
    hipLaunchKernelGGL(kb_fin_init, dim3(B->nseg), dim3(BFIN), 0, s, B->st, B->part_aux, B->part[1], B->seg_blk, kp,
                       tol);
    if (B->nseg > 1) hipLaunchKernelGGL(kb_fin_count, dim3(1), dim3(BFIN), 0, s, B->st);
    EB_LAUNCH_CHECK();
    EB_TRY(benqueue_vcycle<V>(H, B, B->rr[0], 1, B->part[2], s));
    hipLaunchKernelGGL(kb_fin_rz, dim3(B->nseg), dim3(BFIN), 0, s, B->st, B->part[2], B->seg_blk, kp, 1);
    EB_LAUNCH_CHECK();
    return EB_OK;
}

// Polling reads the two counters; bstate_get / bstate_put move the whole state.
static int bpoll(BatchBufs* B, hipStream_t s) {
    EB_HIP(hipMemcpyAsync(B->host, B->st, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    EB_HIP(hipStreamSynchronize(s));
    return EB_OK;
}
static int bstate_get(BatchBufs* B, hipStream_t s) {
    EB_HIP(hipMemcpyAsync(B->host, B->st, sizeof(BatchState), hipMemcpyDeviceToHost, s));
    EB_HIP(hipStreamSynchronize(s));
    return EB_OK;
}
static int bstate_put(BatchBufs* B, hipStream_t s) {
    EB_HIP(hipMemcpyAsync(B->st, B->host, sizeof(BatchState), hipMemcpyHostToDevice, s));
    EB_HIP(hipStreamSynchronize(s));   // the host copy is reused
    return EB_OK;
}

// Systems (seg, j): slots j < nrhs of every segment; results in
// res[seg * nrhs + j].
template <class V>
static int batched_run(amg_handle* H, BatchBufs* B, int nrhs, const pcg_params_t& p, pcg_result_t* res,
                       hipStream_t s) {
    const int kp = B->kp;
    const int nsys = B->nseg * kp;
    BatchState& h = *B->host;
    memset(&h, 0, sizeof(h));
    h.nsys = nsys;
    for (int i = 0; i < nsys; ++i) {
        const bool used = (i % kp) < nrhs;
        h.done[i] = used ? 0 : 1;      // unused slots: done from the start
        h.mask[i] = used ? 1 : 0;
    }
    EB_TRY(bstate_put(B, s));
    std::vector<int> restarts((size_t)nsys, 0);
    int enqueued = 0;
    while (true) {
        EB_TRY(benqueue_start<V>(H, B, p.tol, s));
        int k = 0;
        while (true) {
            EB_TRY(bpoll(B, s));
            if (h.ndone >= nsys || h.maxiter >= p.maxit) break;
            if (enqueued > 4 * p.maxit + 4 * p.check_every) {
                set_error("pcg_solve_batched: iteration counter stalled");
                return EB_EHIP;
            }
            const int left = p.maxit - h.maxiter;
            const int chunk = left < p.check_every ? left : p.check_every;
            const bool graphs = iteration_graphs_enabled();
            for (int c = 0; c < chunk;) {
                if (graphs && k + 1 >= 3 && ((k + 1) & 1) && chunk - c >= 2) {
                    EB_TRY(blaunch_iteration_pair<V>(H, B, s));
                    k += 2;
                    c += 2;
                    enqueued += 2;
                    continue;
                }
                ++k;
                ++c;
                ++enqueued;
                EB_TRY(benqueue_iteration<V>(H, B, k, s));
            }
        }
        // true residual ||b - A x|| per system (FP64)
        unsigned gfix = 0;
        const BFine fr = bfine(H, B, false, &gfix);
        BLAUNCH_N(kb_resid, npl_of(fr, B), bgrid(gfix, fr, B), fr, B->bvec, B->x, B->tres, B->part_aux);
        hipLaunchKernelGGL(kb_fin_true, dim3(B->nseg), dim3(BFIN), 0, s, B->st, B->part_aux, B->seg_blk, kp);
        EB_LAUNCH_CHECK();
        EB_TRY(bstate_get(B, s));
        bool again = false;
        for (int i = 0; i < nsys; ++i) {
            h.mask[i] = 0;
            if ((i % kp) >= nrhs) continue;
            const double tr = h.bb[i] > 0.0 ? sqrt(h.rr_true[i] / h.bb[i]) : 0.0;
            const bool drift = h.status[i] == EB_OK && h.bb[i] > 0.0 && tr > p.tol;
            if (drift && restarts[i] == 0 && h.iters[i] < p.maxit) {
                restarts[i] = 1;
                h.mask[i] = 1;
                h.done[i] = 0;   // the start kernels treat it as active again
                again = true;
            }
        }
        if (!again) break;
        // restart the drifted systems from their current iterate
        EB_TRY(bstate_put(B, s));
    }
    int rc = EB_OK;
    for (int sg = 0; sg < B->nseg; ++sg)
        for (int j = 0; j < nrhs; ++j) {
            const int i = sg * kp + j;
            pcg_result_t& r = res[sg * nrhs + j];
            memset(&r, 0, sizeof(r));
            r.iterations = h.iters[i];
            r.restarts = restarts[i];
            r.levels = H->nlev;
            r.rel_res_true = h.bb[i] > 0.0 ? sqrt(h.rr_true[i] / h.bb[i]) : 0.0;
            r.rel_res_recursive = h.bb[i] > 0.0 ? sqrt(h.rr[i] / h.bb[i]) : 0.0;
            int st = h.status[i];
            if (st == EB_OK && h.bb[i] > 0.0 && r.rel_res_true > p.tol) st = EB_ENOCONV;
            r.status = st;
            if (st != EB_OK && rc == EB_OK) rc = st;
        }
    return rc;
}

// ------------------------------------------------------------- autotuner
// Launch shape of the fine kernels, chosen by timing: on the first solve with
// a new set of batch buffers, before that solve's timed window opens and
// before its right-hand sides are loaded, each candidate (plane width 8 or 16,
// planes per block 1, 2 or 4, within the plane count) runs the fine kernels
// that take the shape (p-update, x/r update, prolongation, post-smoothing)
// once untimed and TUNE_REPS times between HIP events on the batch buffers;
// the median run decides.  (Timing the first two alone once chose a shape
// that made the other two, and the whole FP64 batch, 40 % slower.)  Every
// system is marked active (alpha = beta = 1) for the timing, so the kernels
// read and write every slot, as in a solve: their traffic does not depend on
// the values the buffers hold.  The choice is kept with the buffers and in a
// process-wide table keyed by the strip count, the slot count, the precision
// and the segment count, so later handles of the same shape skip the timing.
// A shape set by pcg_batched_set_launch_shape is used as it is.
struct TuneEntry {
    int64_t nstrips;
    int kp, prec, nseg, kbw, npb;
};
static std::mutex g_tune_mutex;
static std::vector<TuneEntry> g_tune_table;
static int g_forced_kbw = 0, g_forced_npb = 0;

template <class V>
static int autotune_batch(amg_handle* H, BatchBufs* B, hipStream_t s) {
    B->tuned = true;
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        if (g_forced_kbw > 0) {
            B->kbw = g_forced_kbw;
            B->npb = g_forced_npb;
            B->ncand = 0;
            return EB_OK;
        }
        for (const TuneEntry& e : g_tune_table)
            if (e.nstrips == H->nstrips && e.kp == B->kp && e.prec == B->prec && e.nseg == B->nseg) {
                B->kbw = e.kbw;
                B->npb = e.npb;
                return EB_OK;
            }
    }
    BatchState& h = *B->host;
    memset(&h, 0, sizeof(h));
    h.nsys = B->nseg * B->kp;
    for (int i = 0; i < h.nsys; ++i) h.alpha[i] = h.beta[i] = 1.0;
    EB_TRY(bstate_put(B, s));
    hipEvent_t a = nullptr, b = nullptr;
    EB_HIP(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        set_error("hipEventCreate failed");
        return EB_EHIP;
    }
    constexpr int TUNE_REPS = 5;
    const int widths[2] = {8, 16}, npbs[3] = {1, 2, 4};
    int best_w = B->kbw, best_n = B->npb;
    float best = 1e30f;
    int rc = EB_OK;
    B->ncand = 0;
    for (int wi = 0; wi < 2 && rc == EB_OK; ++wi) {
        const int w = widths[wi];
        if (w > B->kp && wi > 0) break;                 // the plane width is min(kp, w)
        const int planes = B->kp / (B->kp < w ? B->kp : w);
        for (int ni = 0; ni < 3 && rc == EB_OK; ++ni) {
            const int n = npbs[ni];
            if (n > planes && ni > 0) break;
            B->kbw = w;
            B->npb = n;
            float runs[TUNE_REPS + 1];
            for (int rep = 0; rep <= TUNE_REPS && rc == EB_OK; ++rep) {
                unsigned gfix = 0;
                const BFine fr = bfine(H, B, false, &gfix);
                if (hipEventRecord(a, s) != hipSuccess) rc = EB_EHIP;
                BLAUNCH_V(kb_pspmv, V, npl_of(fr, B), bgrid(gfix, fr, B), fr, (const V*)B->z, B->p[1], B->p[0], B->q,
                          (const BatchState*)B->st, B->part[0]);
                BLAUNCH_V(kb_xr_down, V, npl_of(fr, B), bgrid(gfix, fr, B), fr, B->x, B->rr[0], B->rr[1], B->p[0],
                          B->q, (V*)B->res, H->lev[0].omega, (const BatchState*)B->st, B->part[1]);
                if (H->nlev > 1) {
                    // the prolongation and post-smoothing passes take the same shape
                    unsigned gfull = 0;
                    const BFine ff = bfine(H, B, true, &gfull);
                    BLAUNCH_V(kb_fine_up, V, npl_of(ff, B), bgrid(gfull, ff, B), ff, H->lev[0].omega, H->agg_p,
                              (const V*)B->ev[1], B->rr[1], (V*)B->zt);
                    BLAUNCH_V(kb_fine_post, V, npl_of(fr, B), bgrid(gfix, fr, B), fr, H->lev[0].omega,
                              (const V*)B->zt, B->rr[1], (V*)B->z, B->part[2]);
                }
                if (hipGetLastError() != hipSuccess || hipEventRecord(b, s) != hipSuccess ||
                    hipEventSynchronize(b) != hipSuccess) {
                    rc = EB_EHIP;
                    break;
                }
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, a, b) != hipSuccess) rc = EB_EHIP;
                runs[rep] = ms;                           // run 0 is a warm-up
            }
            float t = 1e30f;
            if (rc == EB_OK) {
                std::sort(runs + 1, runs + 1 + TUNE_REPS);
                t = runs[1 + TUNE_REPS / 2];
            }
            if (B->ncand < 8) {
                B->cand_w[B->ncand] = w;
                B->cand_n[B->ncand] = n;
                B->cand_ms[B->ncand] = t;
                ++B->ncand;
            }
            if (t < best) {
                best = t;
                best_w = w;
                best_n = n;
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != EB_OK) {
        set_error("batched launch-shape autotuner: HIP error");
        return rc;
    }
    // The fine kernels read neighbours without a guard and rely on zeros off
    // the unknowns, but where a slot lies depends on the plane width: values
    // a candidate wrote at its unknowns can sit off the unknowns of another
    // width.  Every vector the timed kernels wrote goes back to zero.
    {
        const int64_t nv = H->npad * B->kp;
        const size_t vb = B->prec == EB_PREC_FP32 ? sizeof(float) : sizeof(double);
        double* dv[] = {B->x, B->p[0], B->p[1], B->rr[0], B->rr[1], B->q};
        for (double* v : dv) EB_HIP(hipMemsetAsync(v, 0, sizeof(double) * nv, s));
        void* vv[] = {B->zt, B->z, B->res};
        for (void* v : vv) EB_HIP(hipMemsetAsync(v, 0, vb * (size_t)nv, s));
    }
    B->kbw = best_w;
    B->npb = best_n;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_table.push_back({H->nstrips, B->kp, B->prec, B->nseg, best_w, best_n});
    return EB_OK;
}

// Shared body of pcg_solve_batched (nseg = 1, rows = null) and
// pcg_solve_islands.
static int solve_systems(amg_handle_t* H, int32_t nrhs, int nseg, const int32_t* rows, const double* b, double* x,
                         const pcg_params_t* prm, pcg_result_t* res, void* stream, const char* who) {
    if (!H || !b || !x || !res) {
        set_error("%s: null pointer", who);
        return EB_EINVAL;
    }
    if (nrhs < 1 || nrhs > BMAX_RHS) {
        set_error("%s: nrhs = %d outside 1..%d", who, nrhs, BMAX_RHS);
        return EB_EINVAL;
    }
    if (H->beta_on) {
        set_error("%s: batched solves are not available with variable conductivity (solve each right-hand side "
                  "with pcg_solve)", who);
        return EB_ENOTIMPL;
    }
    pcg_params_t p;
    p.tol = 1e-8;
    p.maxit = 1000;
    p.x0_given = 0;
    p.check_every = 8;
    p.precision = EB_PREC_FP64;
    if (prm) p = *prm;
    if (!(p.tol > 0.0) || p.maxit < 0 || p.check_every < 1 ||
        (p.precision != EB_PREC_FP64 && p.precision != EB_PREC_FP32)) {
        set_error("%s: invalid parameters (tol > 0, maxit >= 0, check_every >= 1, precision 0 or 1)", who);
        return EB_EINVAL;
    }
    int kp = 1;
    while (kp < nrhs) kp <<= 1;
    if (rows) {
        const int64_t nrows = (int64_t)H->d.ny * H->d.nz;
        if (nseg < 1 || nseg > BMAX_SEG || (int64_t)nseg * kp > BMAX_SLOTS) {
            set_error("%s: nseg = %d outside 1..%d or nseg x %d slots above %d", who, nseg, BMAX_SEG, kp,
                      BMAX_SLOTS);
            return EB_EINVAL;
        }
        for (int t = 0; t < nseg; ++t)
            if (rows[t] < 0 || rows[t] >= rows[t + 1] || rows[t + 1] > nrows) {
                set_error("%s: segment rows must increase within 0..%lld", who, (long long)nrows);
                return EB_EINVAL;
            }
        if (H->nlev < 2 && H->n_fine > 0) {
            set_error("%s: segments need a hierarchy of two or more levels", who);
            return EB_ENOTIMPL;
        }
    }
    hipStream_t s = stream ? (hipStream_t)stream : H->stream;
    H->last_stream = s;
    const GridDims& d = H->d;
    const int64_t nn = (int64_t)d.nx * d.ny * d.nz;
    const int64_t nunk = H->n_fine;
    hipEvent_t e0 = H->ev0, e1 = H->ev1;
    if (nunk == 0) {
        EB_HIP(hipMemsetAsync(x, 0, sizeof(double) * nn * nrhs, s));
        EB_HIP(hipStreamSynchronize(s));
        for (int j = 0; j < nrhs * nseg; ++j) {
            memset(&res[j], 0, sizeof(res[j]));
            res[j].levels = H->nlev;
        }
        return EB_OK;
    }
    const bool fp32 = p.precision == EB_PREC_FP32;
    if (fp32) EB_TRY(ensure_fp32(H, s));
    EB_TRY(ensure_batch(H, kp, fp32 ? EB_PREC_FP32 : EB_PREC_FP64, nseg, rows, s));
    BatchBufs* B = H->batch;
    if (!B->tuned) EB_TRY(fp32 ? autotune_batch<float>(H, B, s) : autotune_batch<double>(H, B, s));
    // the solve's timed window (solve_ms) opens after any tuning
    EB_HIP(hipEventRecord(e0, s));
    const int lkp = ilog2(kp);
    const unsigned ug = (unsigned)(((nunk << lkp) + BNT - 1) / BNT);
    unsigned gdummy = 0;
    const BFine fl = bfine(H, B, false, &gdummy);
    hipLaunchKernelGGL(kb_load, dim3(ug), dim3(BNT), 0, s, fl, nunk, lkp, kp, nrhs, nn, H->fine_nodes, H->fine_pad, b,
                       B->bvec);
    if (p.x0_given) {
        hipLaunchKernelGGL(kb_load, dim3(ug), dim3(BNT), 0, s, fl, nunk, lkp, kp, nrhs, nn, H->fine_nodes, H->fine_pad,
                           x, B->x);
    } else {
        EB_HIP(hipMemsetAsync(B->x, 0, sizeof(double) * H->npad * kp, s));
    }
    EB_LAUNCH_CHECK();
    const int rc = fp32 ? batched_run<float>(H, B, nrhs, p, res, s) : batched_run<double>(H, B, nrhs, p, res, s);
    if (rc == EB_EHIP || rc == EB_EINVAL) return rc;
    EB_HIP(hipMemsetAsync(x, 0, sizeof(double) * nn * nrhs, s));
    hipLaunchKernelGGL(kb_store, dim3(ug), dim3(BNT), 0, s, fl, nunk, lkp, kp, nrhs, nn, H->fine_nodes, H->fine_pad,
                       B->x, x);
    EB_LAUNCH_CHECK();
    EB_HIP(hipEventRecord(e1, s));
    EB_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    EB_HIP(hipEventElapsedTime(&ms, e0, e1));
    for (int j = 0; j < nrhs * nseg; ++j) res[j].solve_ms = ms;
    if (rc == EB_ENOCONV) set_error("%s: a system did not converge within %d iterations", who, p.maxit);
    if (rc == EB_ENOTSPD) set_error("%s: non-positive curvature in a system", who);
    if (rc == EB_ENAN) set_error("%s: NaN or Inf in a system", who);
    return rc;
}

}  // namespace eb

using namespace eb;

extern "C" int pcg_solve_batched(amg_handle_t* H, int32_t nrhs, const double* b, double* x, const pcg_params_t* prm,
                                 pcg_result_t* res, void* stream) {
    clear_error();
    AllocScope scope(H ? &H->params : nullptr);
    return solve_systems(H, nrhs, 1, nullptr, b, x, prm, res, stream, "pcg_solve_batched");
}

extern "C" int pcg_solve_islands(amg_handle_t* H, int32_t nrhs, int32_t nseg, const int32_t* seg_rows,
                                 const double* b, double* x, const pcg_params_t* prm, pcg_result_t* res,
                                 void* stream) {
    clear_error();
    AllocScope scope(H ? &H->params : nullptr);
    if (!seg_rows) {
        set_error("pcg_solve_islands: null seg_rows");
        return EB_EINVAL;
    }
    return solve_systems(H, nrhs, nseg, seg_rows, b, x, prm, res, stream, "pcg_solve_islands");
}

extern "C" int pcg_batched_set_launch_shape(int32_t plane_width, int32_t planes_per_block) {
    clear_error();
    const bool autom = plane_width == 0 && planes_per_block == 0;
    const bool ok = (plane_width == 8 || plane_width == 16 || plane_width == 32 || plane_width == 64) &&
                    (planes_per_block == 1 || planes_per_block == 2 || planes_per_block == 4);
    if (!autom && !ok) {
        set_error("pcg_batched_set_launch_shape: plane width 8/16/32/64 and 1/2/4 planes per block, or 0, 0");
        return EB_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_forced_kbw = plane_width;
    g_forced_npb = planes_per_block;
    return EB_OK;
}

extern "C" int pcg_batched_launch_shape(const amg_handle_t* H, int32_t* plane_width, int32_t* planes_per_block,
                                        int32_t* ncand, int32_t* cand_width, int32_t* cand_planes, float* cand_ms) {
    clear_error();
    if (!H || !plane_width || !planes_per_block) {
        set_error("pcg_batched_launch_shape: null pointer");
        return EB_EINVAL;
    }
    const BatchBufs* B = H->batch;
    if (!B || !B->tuned) {
        set_error("pcg_batched_launch_shape: no batched solve on this handle yet");
        return EB_EINVAL;
    }
    *plane_width = B->kp < B->kbw ? B->kp : B->kbw;
    *planes_per_block = B->npb;
    if (ncand) {
        *ncand = B->ncand;
        for (int i = 0; i < B->ncand; ++i) {
            if (cand_width) cand_width[i] = B->cand_w[i];
            if (cand_planes) cand_planes[i] = B->cand_n[i];
            if (cand_ms) cand_ms[i] = B->cand_ms[i];
        }
    }
    return EB_OK;
}
