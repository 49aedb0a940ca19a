// Matrix-free operator passes over node fields in the dense user layout:
//   apply    y = (A + sigma I) x                                  (stencil_apply)
//   wave     out = scale (2 u^n - u^{n-1} - dt^2 A v),
//            v = (1 - 2 theta) u^n + theta u^{n-1}                (the theta-scheme, Sec. 3.5)
//   combine  out = alpha (A + sigma I) x + beta y + gamma z       (the Crank-Nicolson
//                                                                  right-hand side, Sec. 3.4)
// A is the operator of Eq. (central_difference): h^2 A_kk = a_k (the boundary
// rows' diagonal), -1/h^2 for each computational neighbour, or with a
// variable conductivity -beta_face/h^2 with the beta of the face between the
// two nodes (Eq. (1)).  Outputs are 0 off computational points; operand
// values there are never read.
//
// Work is cut into band tiles of FX = 62 columns x FY rows of one plane (8
// rows with a conductivity or in 3-D), one wavefront per tile.  Lane l holds column x0 - 1 + l (lanes 0 and 63 are the
// halo columns and store nothing).  The wavefront first reads the kinds of
// its FY rows and of the rows above and below (and, in 3-D, of the planes
// k - 1 and k + 1 beside each row), then marches down the rows with three rows
// of the operand in registers: left and right neighbours come from the
// adjacent lanes by DPP shifts, the planes k +- 1 from their own reads.
// Operands, a, the face conductivities and the extra fields are read only at
// computational points, so per node a pass moves the kind (1 B) and the
// output (8 B), and per computational node its operand and coefficient
// fields.  Block b's four wavefronts take four adjacent tiles of one band
// (2-D: each row is read as one run of 4 x 62 columns) or four consecutive
// planes of one tile (3-D), and the blocks are renumbered so that each XCD
// owns a contiguous range: the halo rows and neighbouring planes a tile
// re-reads were just read by its neighbours on the same L2.
#include "common.hpp"

namespace eb {

constexpr int FX = WAVE - 2;    // columns stored per tile
constexpr int FY = 16;          // rows per tile (the plain 2-D passes)
constexpr int FY_SMALL = 8;     // rows per tile with a conductivity or in 3-D (more values per row)

constexpr int rows_per_tile(bool cb, int dim) { return (cb || dim == 3) ? FY_SMALL : FY; }
constexpr int FWB = 4;          // wavefronts (tiles) per block
constexpr int FNT = FWB * WAVE;

enum FieldOp { FOP_APPLY = 0, FOP_WAVE = 1, FOP_COMBINE = 2 };

struct FieldArgs {
    const int8_t* kind;
    const double* a;
    const double* cond;   // dim face fields back to back (field `axis` at the face toward +axis), or null
    const double* f0;     // apply, combine: x; wave: u^n
    const double* f1;     // wave: u^{n-1}
    const double* g0;     // combine: y (null when beta = 0)
    const double* g1;     // combine: z (null when gamma = 0)
    double* out;
    double c0, c1;        // wave: v = c0 u^n + c1 u^{n-1}
    double sigma;         // apply, combine
    double alpha, beta, gamma;   // combine
    double scale, dt2;    // wave
    int nx, ny, nz;
    int64_t sy, sz, nn;
    double s;             // 1/h^2
    int ntx, nty;         // tiles per row, bands per plane
    int64_t nwaves;
};

// Buffer windows.  Each wavefront reads and writes through buffer resources
// based at the first node it may touch, so offsets are 32-bit byte offsets;
// an access that is not wanted (a masked lane, a node off the computational
// points) is given an offset beyond the window: the load returns 0 and the
// store is dropped by the hardware's range check, without a memory access
// and without a branch.  The fourth descriptor word is the gfx9 raw-buffer
// format word.
constexpr uint32_t OOB = 0x80000000u;
constexpr int BUF_WORD3 = 0x00020000;

__device__ inline __amdgpu_buffer_rsrc_t window(const void* base, int64_t lo, int64_t count, int esize) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)((const char*)base + lo * esize), (short)0,
                                             (int)(count * esize), BUF_WORD3);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Element e of a window when ok, else an offset beyond it (0 returned,
// nothing stored).
__device__ inline double bload(__amdgpu_buffer_rsrc_t r, bool ok, uint32_t e) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, ok ? e * 8u : OOB, 0, 0));
}

__device__ inline int bload_kind(__amdgpu_buffer_rsrc_t r, bool ok, uint32_t e) {
    return (int)(signed char)__builtin_amdgcn_raw_buffer_load_b8(r, ok ? e : OOB, 0, 0);
}

__device__ inline void bstore(__amdgpu_buffer_rsrc_t r, bool ok, uint32_t e, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, ok ? e * 8u : OOB, 0, 0);
}

// The operand at a node (wave: from u^n and u^{n-1}, both kept for the
// right-hand side's own terms); 0 where the offset is out of the window.
struct Opd {
    double v, u, um;
};

// Values of a centre row read one row ahead: a, the extra fields, the face
// conductivities toward +x, +y (and +-z), the operand on the planes k +- 1.
struct Cen {
    double a, e0, e1, wr, wup, wzb, wzf, zb, zf;
};

template <int OP, bool CB, int DIM>
__global__ void __launch_bounds__(FNT) k_field_op(FieldArgs p) {
    constexpr int TY = rows_per_tile(CB, DIM);
    const int lane = threadIdx.x & (WAVE - 1);
    // the wavefront's index, in scalar registers (the buffer descriptors built
    // from it must be wave-uniform)
    const int wib = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int64_t gw = xcd_block() * (int64_t)FWB + wib;
    if (gw >= p.nwaves) return;
    int64_t t = gw;
    int k = 0;
    if (DIM == 3) {
        k = (int)(t % p.nz);
        t /= p.nz;
    }
    // 2-D: the tiles of a band are consecutive (a block's four wavefronts read
    // four adjacent column ranges of the same rows); 3-D: the planes are
    const int x0 = (int)(t % p.ntx) * FX;
    const int band = (int)(t / p.ntx);
    const int i = x0 - 1 + lane;
    const int y0 = band * TY;
    const bool col_in = i >= 0 && i < p.nx;
    const bool col_inner = i >= 1 && i < p.nx - 1;
    const bool owner = lane >= 1 && lane <= FX && col_in;
    const bool plane_inner = DIM == 2 || (k >= 1 && k < p.nz - 1);
    const bool zm_inner = DIM == 3 && k - 1 >= 1;
    const bool zp_inner = DIM == 3 && k + 1 < p.nz - 1;
    const int64_t kb = (int64_t)k * p.sz;
    const int64_t zs = DIM == 3 ? p.sz : 0;

    // the nodes this wavefront may touch: rows y0 - 1 .. y0 + TY of columns
    // x0 - 1 .. x0 + FX, and the planes k +- 1 beside them
    int64_t lo = kb - zs + (int64_t)(y0 - 1) * p.sy + (x0 - 1);
    int64_t hi = kb + zs + (int64_t)(y0 + TY) * p.sy + (x0 + FX);
    lo = lo < 0 ? 0 : lo;
    hi = hi > p.nn - 1 ? p.nn - 1 : hi;
    const int64_t cnt = hi - lo + 1;
    const __amdgpu_buffer_rsrc_t rk = window(p.kind, lo, cnt, 1);
    const __amdgpu_buffer_rsrc_t ra = window(p.a, lo, cnt, 8);
    const __amdgpu_buffer_rsrc_t rf0 = window(p.f0, lo, cnt, 8);
    const __amdgpu_buffer_rsrc_t rf1 = window(OP == FOP_WAVE ? p.f1 : p.f0, lo, cnt, 8);
    const __amdgpu_buffer_rsrc_t rg0 = window(p.g0 ? p.g0 : p.f0, lo, p.g0 ? cnt : 0, 8);
    const __amdgpu_buffer_rsrc_t rg1 = window(p.g1 ? p.g1 : p.f0, lo, p.g1 ? cnt : 0, 8);
    const __amdgpu_buffer_rsrc_t rc0 = window(CB ? p.cond : p.a, lo, CB ? cnt : 0, 8);
    const __amdgpu_buffer_rsrc_t rc1 = window(CB ? p.cond + p.nn : p.a, lo, CB ? cnt : 0, 8);
    const __amdgpu_buffer_rsrc_t rc2 = window(CB && DIM == 3 ? p.cond + 2 * p.nn : p.a, lo,
                                              CB && DIM == 3 ? cnt : 0, 8);
    const __amdgpu_buffer_rsrc_t ro = window(p.out, lo, cnt, 8);

    // element offset of row q's node in the windows (rows q = 0 .. TY + 1 are
    // grid rows y0 - 1 .. y0 + TY)
    const int64_t n0 = kb + (int64_t)(y0 - 1) * p.sy + i - lo;
    auto rel = [&](int q) { return (uint32_t)(n0 + (int64_t)q * p.sy); };
    auto row_inner = [&](int q) { return y0 - 1 + q >= 1 && y0 - 1 + q < p.ny - 1; };
    const uint32_t zsb = (uint32_t)zs;

    // computational flags of the rows, and in 3-D of the planes k - 1, k + 1
    bool cm[TY + 2], czm[TY + 2], czp[TY + 2];
#pragma unroll
    for (int q = 0; q < TY + 2; ++q) {
        const bool in = col_inner && row_inner(q);
        cm[q] = bload_kind(rk, in && plane_inner, rel(q)) == 2;
        czm[q] = czp[q] = false;
        if (DIM == 3 && q >= 1 && q <= TY) {
            czm[q] = bload_kind(rk, in && zm_inner, rel(q) - zsb) == 2;
            czp[q] = bload_kind(rk, in && zp_inner, rel(q) + zsb) == 2;
        }
    }

    auto opload = [&](bool ok, uint32_t e) {
        Opd o;
        o.u = bload(rf0, ok, e);
        o.um = OP == FOP_WAVE ? bload(rf1, ok, e) : 0.0;
        o.v = OP == FOP_WAVE ? p.c0 * o.u + p.c1 * o.um : o.u;
        return o;
    };
    auto cenload = [&](int q) {
        Cen c;
        const bool ok = cm[q];
        const uint32_t e = rel(q);
        c.a = bload(ra, ok, e);
        c.e0 = c.e1 = 0.0;
        if (OP == FOP_COMBINE) {
            c.e0 = bload(rg0, ok && owner, e);
            c.e1 = bload(rg1, ok && owner, e);
        }
        c.wr = c.wup = c.wzb = c.wzf = c.zb = c.zf = 0.0;
        if (CB) {
            c.wr = bload(rc0, ok, e);
            c.wup = bload(rc1, ok, e);
            if (DIM == 3) {
                c.wzb = bload(rc2, ok, e - zsb);
                c.wzf = bload(rc2, ok, e);
            }
        }
        if (DIM == 3) {
            c.zb = opload(czm[q], e - zsb).v;
            c.zf = opload(czp[q], e + zsb).v;
        }
        return c;
    };

    // every operand row and every centre row of the tile is read before the
    // first row is formed, so each wavefront keeps all its reads in flight
    Opd o[TY + 2];
    Cen c[TY + 2];
#pragma unroll
    for (int q = 0; q < TY + 2; ++q) o[q] = opload(cm[q], rel(q));
    const double wdn0 = CB ? bload(rc1, cm[0], rel(0)) : 0.0;
#pragma unroll
    for (int q = 1; q <= TY; ++q) c[q] = cenload(q);

#pragma unroll
    for (int q = 1; q <= TY; ++q) {
        const Cen& cc = c[q];
        const double vm = o[q - 1].v, vc = o[q].v, vp = o[q + 1].v;
        const double wdn = q == 1 ? wdn0 : c[q - 1].wup;
        // every lane takes part in the shifts
        const double vl = from_left(vc), vr = from_right(vc);
        const double wl = CB ? from_left(cc.wr) : 0.0;
        double nb = 0.0;
        if (CB) {
            nb = nb + wl * vl;
            nb = nb + cc.wr * vr;
            nb = nb + wdn * vm;
            nb = nb + cc.wup * vp;
            if (DIM == 3) {
                nb = nb + cc.wzb * cc.zb;
                nb = nb + cc.wzf * cc.zf;
            }
        } else {
            nb = nb + vl;
            nb = nb + vr;
            nb = nb + vm;
            nb = nb + vp;
            if (DIM == 3) {
                nb = nb + cc.zb;
                nb = nb + cc.zf;
            }
        }
        double r;
        if (OP == FOP_APPLY) {
            const double diag = cc.a * p.s + p.sigma;
            r = diag * vc - p.s * nb;
        } else if (OP == FOP_WAVE) {
            const double av = (cc.a * p.s) * vc - p.s * nb;
            r = p.scale * ((2.0 * o[q].u - o[q].um) - p.dt2 * av);
        } else {
            const double ax = (cc.a * p.s + p.sigma) * vc - p.s * nb;
            r = p.alpha * ax;
            if (p.g0) r += p.beta * cc.e0;
            if (p.g1) r += p.gamma * cc.e1;
        }
        // exactly 0 off computational points
        r = cm[q] ? r : 0.0;
        bstore(ro, owner && y0 - 1 + q < p.ny, rel(q), r);
    }
}

template <int OP, bool CB>
static void launch_dim(const FieldArgs& p, int dim, hipStream_t s) {
    const int64_t blocks = ((p.nwaves + FWB - 1) / FWB + NUM_XCD - 1) / NUM_XCD * NUM_XCD;
    if (dim == 2)
        hipLaunchKernelGGL((k_field_op<OP, CB, 2>), dim3((unsigned)blocks), dim3(FNT), 0, s, p);
    else
        hipLaunchKernelGGL((k_field_op<OP, CB, 3>), dim3((unsigned)blocks), dim3(FNT), 0, s, p);
}

int launch_field_op(int op, const GridDims& d, const int8_t* kind, const double* a, const double* cond,
                    const double* f0, const double* f1, const double* g0, const double* g1, double* out,
                    const FieldCoefs& co, hipStream_t s) {
    FieldArgs p;
    p.kind = kind;
    p.a = a;
    p.cond = cond;
    p.f0 = f0;
    p.f1 = f1;
    p.g0 = g0;
    p.g1 = g1;
    p.out = out;
    p.c0 = co.c0;
    p.c1 = co.c1;
    p.sigma = co.sigma;
    p.alpha = co.alpha;
    p.beta = co.beta;
    p.gamma = co.gamma;
    p.scale = co.scale;
    p.dt2 = co.dt2;
    p.nx = d.nx;
    p.ny = d.ny;
    p.nz = d.dim == 3 ? d.nz : 1;
    p.sy = d.sy;
    p.sz = d.dim == 3 ? d.sz : (int64_t)d.nx * d.ny;
    p.nn = (int64_t)d.nx * d.ny * p.nz;
    p.s = d.s;
    p.ntx = (d.nx + FX - 1) / FX;
    p.nty = (d.ny + rows_per_tile(cond != nullptr, d.dim) - 1) / rows_per_tile(cond != nullptr, d.dim);
    p.nwaves = (int64_t)p.ntx * p.nty * p.nz;
    const int64_t blocks = ((p.nwaves + FWB - 1) / FWB + NUM_XCD - 1) / NUM_XCD * NUM_XCD;
    // a wavefront's buffer window spans two planes and FY + 2 rows: its byte
    // size must stay below 2^31
    const int64_t span = (d.dim == 3 ? 2 * p.sz : 0) + (int64_t)(FY + 2) * p.sy + FX + 2;
    if (blocks > 0x7fffffffLL || span * (int64_t)sizeof(double) >= (int64_t)OOB) {
        set_error("operator pass: grid too large (planes of at most about 1.3e8 nodes)");
        return EB_EINVAL;
    }
    const bool cb = cond != nullptr;
    switch (op) {
        case FOP_APPLY:
            cb ? launch_dim<FOP_APPLY, true>(p, d.dim, s) : launch_dim<FOP_APPLY, false>(p, d.dim, s);
            break;
        case FOP_WAVE:
            cb ? launch_dim<FOP_WAVE, true>(p, d.dim, s) : launch_dim<FOP_WAVE, false>(p, d.dim, s);
            break;
        default:
            cb ? launch_dim<FOP_COMBINE, true>(p, d.dim, s) : launch_dim<FOP_COMBINE, false>(p, d.dim, s);
            break;
    }
    EB_LAUNCH_CHECK();
    return EB_OK;
}

}  // namespace eb
