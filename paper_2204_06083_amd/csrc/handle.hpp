// Internal layout of an amg_handle_t: the device hierarchy plus the fine-level
// solve layout (row-padded node fields and active strip / box lists).
#pragma once

#include "common.hpp"

namespace eb {

constexpr int MAX_LEVELS = 24;

// ELL copy of a sparse matrix for the V-cycle in slices of 64 consecutive
// rows (one wavefront, one lane per row), each stored slot-major, every row
// padded to the width w of the matrix's longest row: entry k of row r sits at
// 64 (w (r / 64) + k) + r % 64, so a kernel finds it from r and w alone (no
// offset table to read first).  Padding has value 0 and the row's last column
// (column 0 for an empty row), so every read is in bounds and adds nothing.
// On the coarse levels of the box aggregation the widths are nearly uniform
// (2-D: A 9, P 4, A P 9 on most rows).
struct Sell {
    int32_t* wdev = nullptr;   // w on the device (set by the setup kernels; in the level's sell_w)
    int32_t* col = nullptr;
    double* val = nullptr;
    float* val32 = nullptr;    // single-precision V-cycle copy (made on first use)
    int64_t cap = 0;           // entries allocated (a bound on 64 w nslices)
    int width = 0;             // w on the host (read back at the end of setup)
};

struct Level {
    int64_t n = 0, nnz_a = 0, nnz_p = 0, nnz_r = 0, nnz_ap = 0;
    double rho = 0.0, omega = 0.0;
    double omega_setup = 0.0;    // 4 / (3 rho) as set up (omega may be overridden for the V-cycle)
    int is_coarsest = 0;
    int max_comp = 0;            // most coarse unknowns sharing one box of this level
    int ext[3] = {1, 1, 1};      // coordinate extents
    int64_t row_bound = 0;       // upper bound on entries per row of A
    int nb[3] = {1, 1, 1};       // box-grid extents (ceil(ext / 3))
    int64_t nboxes = 0;
    // operator (CSR, sorted columns) and its diagonal
    int32_t* a_rowptr = nullptr; int32_t* a_col = nullptr; double* a_val = nullptr;
    double* diag = nullptr;
    // transfer operators to/from level + 1
    int32_t* p_rowptr = nullptr; int32_t* p_col = nullptr; double* p_val = nullptr;
    int32_t* r_rowptr = nullptr; int32_t* r_col = nullptr; double* r_val = nullptr;
    int32_t* agg = nullptr;      // n: coarse unknown of each unknown
    int32_t* coords = nullptr;   // 3n
    int4* cinfo = nullptr;       // n: box coordinates and rank within the box (levels >= 1)
    int32_t* box_cstart = nullptr;  // nboxes: first coarse unknown of each box
    int32_t* box_ncomp = nullptr;   // nboxes: coarse unknowns formed in each box
    double* dense_inv = nullptr; // coarsest: n x n
    // island hierarchies: the islands whose own hierarchy ends at this level
    // (at most coarse_max unknowns here) take no part in the coarser levels;
    // their correction on this level is the exact solve with their diagonal
    // block of A, kept inverted.  Blocks are contiguous row ranges.
    int nfz = 0;                 // blocks (islands) ending here
    int fz_all = 0;              // 1: every row belongs to a block (the coarsest level of an island hierarchy)
    int32_t* fz_off = nullptr;   // nfz + 1 row offsets (device)
    int64_t* fz_woff = nullptr;  // nfz offsets of the inverses in fz_inv (device)
    double* fz_inv = nullptr;    // the blocks' inverses, row-major, back to back
    int32_t* fz_blk = nullptr;   // n: block of each row, -1 outside the blocks
    // sliced ELL copies of A, P and A P for the V-cycle (levels >= 1 with a
    // coarser level), and R A = (A P)^T in CSR (rows sorted)
    Sell sa, sp, sap;
    int32_t* sell_w = nullptr;   // widths of sa, sp, sap on the device (one allocation)
    // the packed A P of the Galerkin step, kept until the V-cycle copies
    // (sliced A, P, A P and R A) are built at the end of setup
    int32_t* apk_cnt = nullptr;
    int32_t* apk_start = nullptr;
    int32_t* apk_col = nullptr;
    double* apk_val = nullptr;
    int apk_slots = 0;
    int64_t apk_pbound = 0;
    int32_t* ra_rowptr = nullptr; int32_t* ra_col = nullptr; double* ra_val = nullptr; float* ra_val32 = nullptr;
    int64_t ra_cap = 0;
    // solve vectors (levels >= 1); sv = omega rv / diag, written with rv by the
    // restriction that produces it (each consumer then gathers one value
    // instead of two and divides no more)
    double* rv = nullptr; double* ev = nullptr; double* tmp = nullptr; double* sv = nullptr;
    // FP32 copies for the single-precision V-cycle (made on first use)
    float* a_val32 = nullptr; float* p_val32 = nullptr; float* r_val32 = nullptr; float* diag32 = nullptr;
    float* rv32 = nullptr; float* ev32 = nullptr; float* tmp32 = nullptr; float* sv32 = nullptr;
};

// Device scalars of one PCG solve.  Written only by block 0 of the kernel
// that owns each field (or by a one-block finaliser) and read by later kernels.
struct PcgScalars {
    double rr;         // ||r||^2 of the latest iterate
    double bb;         // ||b||^2
    double tol2bb;     // tol^2 ||b||^2
    double pq;         // (p, q) of the latest iteration
    double rr_true;    // ||b - A x||^2 recomputed at exit
    double rr0;        // ||r||^2 at the start (or restart): the host predicts
                       // the remaining iterations from rr / rr0
    int32_t done;      // 1: converged / failed, later kernels return at once
    int32_t status;    // EB_OK or failure code
    int32_t iters;
    int32_t pad;
};

// One partial sum per block of the fixed-size fine grid; consumers sum them
// in a fixed order (every block of the consumer gets the same total).
struct Reduction {
    int nparts = 0;             // blocks of every reducing fine kernel
    double* pq = nullptr;
    double* rr = nullptr;
    double* rz[2] = {nullptr, nullptr};
    double* aux = nullptr;
    double* aux2 = nullptr;
};

struct BatchBufs;    // batched solve state (batched.hip)

}  // namespace eb

struct amg_handle {
    eb::GridDims d;
    double sigma = 0.0;
    hipStream_t stream = nullptr;
    hipStream_t last_stream = nullptr;   // stream of the latest solve / V-cycle call
    amg_params_t params;
    int64_t n_fine = 0;
    int nlev = 0;
    eb::Level lev[eb::MAX_LEVELS];
    // fine-level solve layout: node fields with x rows padded to `px` (multiple of 64)
    int px = 0;
    int64_t npad = 0;
    int strip_w = 64;
    int64_t nstrips = 0;
    int32_t* strips = nullptr;      // active strips (ids: padded index / strip_w)
    int32_t* dcount = nullptr;      // device totals: [0] strips, [1] level-0 boxes, [2] tiles
    int64_t nboxes0 = 0;
    // 2-D fine band tiles (TX x TY nodes) holding unknowns, row-major;
    // tile_tpw tiles per wavefront of the tile kernels
    int64_t ntiles = 0;
    int32_t* tiles = nullptr;
    int tile_ntx = 0;
    int tile_tpw = 1;
    int32_t* box_map0 = nullptr;    // 2-D: aggregate of each node of a level-0 box (3 bits per node)
    double* box_w0 = nullptr;       // 2-D: omega_1 / d_1 of the first aggregate of each level-0 box
    float* box_w0_32 = nullptr;
    int32_t* boxes0 = nullptr;      // level-0 boxes holding unknowns
    int64_t* fine_nodes = nullptr;  // unknown -> dense node index
    int32_t* unk_off_tmp = nullptr; // setup only: dense node -> unknown index
    const int8_t* kind_tmp = nullptr;  // setup only: the caller's kind field
    const double* beta_tmp = nullptr;  // setup only: the caller's face conductivities (variable beta)
    // variable conductivity: beta at the +axis face of every node, padded
    // layout (fine strip kernels take them; the 2-D tile kernels are off)
    int beta_on = 0;
    double* bf_p[3] = {nullptr, nullptr, nullptr};
    int32_t* fine_pad = nullptr;    // unknown -> padded node index
    double* diag_p = nullptr;       // padded diagonal (0 off unknowns)
    double* dinv_p = nullptr;       // padded 1 / diagonal (0 off unknowns): the fine smoother and
                                    // prolongator scale by omega / d
    // single-precision V-cycle: padded FP32 diagonal and V-cycle vectors
    int fp32_ready = 0;
    float* diag_p32 = nullptr;
    float* dinv_p32 = nullptr;
    float* res32 = nullptr;
    float* zt32 = nullptr;
    float* z32 = nullptr;
    // BF16 smoother (EB_PREC_BF16): BF16 copies of the padded 1 / diagonal and
    // of the preconditioned residual z (2 bytes per node each)
    int bf16_ready = 0;
    void* dinv_p16 = nullptr;
    void* z16 = nullptr;
    int32_t* agg_p = nullptr;       // padded level-0 aggregate (-1 off unknowns)
    // per-point fine smoother weights omega_k / d_k (padded; 0 off unknowns)
    int wf_on = 0;
    double* wf = nullptr;
    float* wf32 = nullptr;
    // PCG state (padded node fields)
    double* x = nullptr; double* z = nullptr;
    double* rr[2] = {nullptr, nullptr};   // residual, alternating between iterations
    double* p[2] = {nullptr, nullptr};
    double* q = nullptr; double* res = nullptr; double* zt = nullptr;
    double* bvec = nullptr;         // right-hand side in the padded layout
    eb::PcgScalars* sc = nullptr;
    double* dscal = nullptr;        // per level: rho, omega (device)
    eb::PcgScalars* sc_host = nullptr;   // host mirror (points at sc_mirror)
    eb::PcgScalars sc_mirror;
    eb::Reduction red;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // captured pair of steady-state PCG iterations (k odd, then k + 1) per
    // V-cycle precision, with the fine-weight switch it was captured under
    hipGraphExec_t it_graph[3] = {nullptr, nullptr, nullptr};   // FP64, FP32, BF16 smoother
    int it_graph_wf[3] = {-1, -1, -1};
    hipStream_t cap_stream = nullptr;   // private stream the graphs are captured on
    // the coarsest inverse runs on the device's side stream during setup
    // (forked after the coarsest level is built, joined before the setup's
    // read-back); join_pending while that work may still be in flight
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join = nullptr;
    hipEvent_t ev_stat = nullptr;   // setup: the per-level status read has arrived
    int join_pending = 0;
    // kernel timing hook (eb_timing_select / eb_timing_read)
    int tim_kernel = -1;
    int tim_cap = 0;
    int tim_used = 0;
    hipEvent_t* tim_ev = nullptr;     // 2 * tim_cap events
    hipStream_t tim_stream = nullptr;
    int64_t tim_launches = 0;
    double tim_ms = 0.0;
    // batched solves (made on the first pcg_solve_batched call)
    eb::BatchBufs* batch = nullptr;
    // island hierarchy (amg_setup_islands): node-row bounds of the islands
    int nisl = 0;
    int32_t* isl_rows = nullptr;    // nisl + 1 (device, setup only)
};

namespace eb {
int ensure_fp32(amg_handle* H, hipStream_t s);   // FP32 hierarchy copies (solve.hip)
int ensure_bf16(amg_handle* H, hipStream_t s);   // BF16 smoother operands (solve.hip)
void free_batch(amg_handle* H, hipStream_t s);   // batched.hip
void drop_batch_graph(amg_handle* H);            // batched.hip: the captured batched iterations
// Destroys the captured iteration graphs of a handle (solve.hip).
void drop_iteration_graphs(amg_handle* H);
// The eb_set_iteration_graphs switch, read by single and batched solves (solve.hip).
bool iteration_graphs_enabled();
}  // namespace eb
