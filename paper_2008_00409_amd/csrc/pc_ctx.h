// Host-side context of the library: device buffers and launch helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <unordered_map>
#include <utility>
#include <algorithm>
#include <vector>

#include "pc_common.h"
#include "pcloth.h"

namespace pc {

// CG scalars of one instance.  rz is double-buffered by iteration parity:
// the iteration of parity P reads rzp[P] and its direction kernel, in which
// every block computes beta itself, writes rzp[1 - P], so no block reads a
// value another block of the same launch is writing.
struct PcgState {
    double rzp[2], alpha, rr, bb, tol2, rz0;
    double rho2;     // inner reduction factor squared (refinement sweeps)
    double thresh;   // stop when ||r||^2 <= thresh = max(tol^2 ||b||^2, rho^2 ||r_0||^2)
    double rr0;      // ||r_0||^2 of this sweep
    double rzd;      // r.P^-1 r of the residual the current direction was built from
    // single-reduction (Chronopoulos-Gear) form: beta of the iteration being
    // applied, gamma and alpha of the previous one
    double beta, gprev, aprev;
    int iters, maxit, done, flags;   // flags: 1 breakdown (p.Ap <= 0), 2 non-finite
    int kc, pad_;                    // iterations of the current sweep (single-reduction form)
    // textbook form: live[par] = 1 when the update of the iteration of parity
    // par ran (its alpha is in `alpha`); the direction kernel of that iteration
    // clears the other slot for the next one
    int live[2];
};

// Sampled kernel timing with HIP events on the launch stream: every
// `every`-th launch of a timed kind is bracketed by an event pair; pairs are
// read back at the next synchronisation point.
enum ProfKind { PK_SPMV = 0, PK_UPDATE = 1, PK_DIR = 2, PK_ROW_ASM = 3, PK_ROW_PAT = 4, PK_ASM_ALL = 5,
                PK_ELEMENTS = 6, PK_NKINDS = 8 };

struct Prof {
    int every = 0;
    long long tick[PK_NKINDS] = {};
    std::vector<hipEvent_t> pool;      // 2 events per slot
    std::vector<int> free_slots;
    std::vector<std::pair<int, int>> pending;  // (kind, slot)
    double sum_ms[PK_NKINDS] = {}, min_ms[PK_NKINDS] = {}, max_ms[PK_NKINDS] = {};
    long long count[PK_NKINDS] = {};
    std::vector<float> kept[PK_NKINDS];   // up to 1 << 16 samples per kind, for the median

    void init(int nslots) {
        if (!pool.empty()) return;
        pool.resize(2 * (size_t)nslots);
        for (auto &e : pool) (void)hipEventCreate(&e);
        for (int k = nslots - 1; k >= 0; --k) free_slots.push_back(k);
    }
    void destroy() {
        for (auto &e : pool) (void)hipEventDestroy(e);
        pool.clear();
        free_slots.clear();
        pending.clear();
    }
    void reset() {
        for (int k = 0; k < PK_NKINDS; ++k) {
            sum_ms[k] = min_ms[k] = max_ms[k] = 0.0;
            count[k] = 0;
            tick[k] = 0;
            kept[k].clear();
        }
    }
    // returns a slot (>= 0) when this launch is sampled; records the start event
    int begin(int kind, hipStream_t s) {
        if (every <= 0) return -1;
        if ((tick[kind]++ % every) != 0 || free_slots.empty()) return -1;
        const int slot = free_slots.back();
        free_slots.pop_back();
        (void)hipEventRecord(pool[2 * (size_t)slot], s);
        pending.emplace_back(kind, slot);
        return slot;
    }
    void end(int slot, hipStream_t s) {
        if (slot >= 0) (void)hipEventRecord(pool[2 * (size_t)slot + 1], s);
    }
    // call after the stream has been synchronised
    void harvest() {
        for (auto &kp : pending) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, pool[2 * (size_t)kp.second], pool[2 * (size_t)kp.second + 1]) ==
                hipSuccess) {
                const int k = kp.first;
                if (count[k] == 0 || ms < min_ms[k]) min_ms[k] = ms;
                if (count[k] == 0 || ms > max_ms[k]) max_ms[k] = ms;
                sum_ms[k] += ms;
                count[k] += 1;
                if (kept[k].size() < (1u << 16)) kept[k].push_back(ms);
            }
            free_slots.push_back(kp.second);
        }
        pending.clear();
    }
    double median(int k) const {
        if (kept[k].empty()) return 0.0;
        std::vector<float> v = kept[k];
        std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
        return v[v.size() / 2];
    }
};

struct MlpState;

// The paper's sparse-matrix filling and BELL layout (built beside the
// solver's assembly for comparison): index table (nv x Wi), compacted
// column table and value planes (slot k of row i at k nv + i).
struct BellState {
    int *cnt = nullptr;     // nv + 4: slot counts / fill pointers, then the two widths
    int *len = nullptr;     // nv: compacted row lengths
    double *f = nullptr;    // 6 nv: element forces, then c K v
    int *idx = nullptr;     // nv x Wi index table
    int *col = nullptr;     // Wv x nv columns
    void *val = nullptr;    // 9 x Wv x nv values (FP32 or FP64)
    float4 *x4 = nullptr;   // nv: SpMV input as float4
    size_t cnt_bytes = 0, len_bytes = 0, f_bytes = 0, idx_bytes = 0, col_bytes = 0, val_bytes = 0;
    int Wi = 0, Wv = 0;
    pc_dtype dtype = PC_F32;
    bool valid = false;
};

// Where a device block came from: free_fn == nullptr means hipMalloc.
struct AllocRec {
    pc_free_fn free_fn;
    void *user;
};

struct Ctx {
    std::string err;
    // device allocator of the following allocations (nullptr: hipMalloc) and
    // the origin of every live block
    pc_alloc_fn alloc_fn = nullptr;
    pc_free_fn free_fn = nullptr;
    void *alloc_user = nullptr;
    std::unordered_map<void *, AllocRec> blocks;
    Prof prof;
    double ell = 0.0;          // mean rest edge length (over the 3 edges of every triangle)
    const double *last_x = nullptr, *last_v = nullptr;  // state of the last assembly (caller's buffers)
    MlpState *mlp = nullptr;   // learned warm start (allocated on first use)
    void *ws_scratch = nullptr;   // this GPU's scratch of pc_ws_predict_noalloc (device address)
    int nv = 0, nt = 0, nh = 0;
    int nslices = 0;          // ceil(nv / 64)
    int64_t cap = 0;          // block capacity (upper bound of nnzb)
    int64_t ninc = 0;         // 3 nt + 4 nh + 4 nc incidences
    int64_t ninc_cap = 0;     // incidences inc can hold
    int64_t cap_base = 0;     // block capacity without contacts

    // proximity (contact) elements of the following assemblies
    int nc = 0;
    int64_t nc_cap = 0;
    int *cverts = nullptr;    // nc x 4
    double *cw = nullptr;     // nc x 4 weights (sum zero)
    double *cn = nullptr;     // nc x 3 unit normals
    double ceta = 0.0, ckc = 0.0;
    DevParams prm{};
    pc_params user_prm{};

    // static topology / rest data (device)
    int *tri = nullptr;       // 3 planes of nt
    double *Bm = nullptr;     // 4 planes of nt (inverse rest frame, row major)
    double *A0 = nullptr;     // nt
    int *hinge = nullptr;     // 4 planes of nh
    double *hcoef = nullptr;  // nh, 3|e|^2 / (A1 + A2)
    double *htbar = nullptr;  // nh, rest angle
    double *mass = nullptr;   // nv
    uint8_t *pinned = nullptr;
    int *status = nullptr;    // device error bits

    // per-step pattern
    int *inc_cnt = nullptr;   // nv (kept at zero between uses)
    int *inc_ptr = nullptr;   // nv + 1
    int *inc = nullptr;       // ninc
    int *rowlen = nullptr;    // nv
    int *rowptr = nullptr;    // nv + 1
    int *colidx = nullptr;    // cap (block-CSR order)
    int *jcol = nullptr;      // cap (solver layout)
    int16_t *jdel = nullptr;  // the same columns as offsets from each slice's first row
    bool narrow = false;      // every offset fits in 16 bits (decided with the windows)
    bool use_narrow = true;   // PC_OPT_NARROW_COLUMNS
    int *lane_row = nullptr;  // nslices * 64 (row of each lane, -1 padding)
    int *row_lane = nullptr;  // nv
    uint8_t *slot_cnt = nullptr;  // nslices * 64
    int *slot_off = nullptr;      // nslices * 64: first stored block of each slot, from the slice's first
    uint8_t *row_state = nullptr; // nv: which assembly pass handles each row
    int *rowlen_s = nullptr;
    // FP16 storage: per slice, f16_scale[2 s] = S of the slice's instance
    // (its blocks are stored as S a) and f16_scale[2 s + 1] = 1 / S;
    // f16_part: per-slice maxima of |a|
    double *f16_scale = nullptr;
    double *f16_part = nullptr;
    int f16_cap = 0;                  // slices the two arrays can hold
    int *inst_slice0 = nullptr;       // ninst + 1 instance slice ranges (device)      // nv: blocks of each row in the solver layout (a zero diagonal left out)
    int *wide_rows = nullptr;     // nv: rows of the wide-row passes
    int *row_npairs = nullptr;    // nv: (incidence, corner) pairs of each row
    int *cols_tmp = nullptr;      // 3 ninc + nv: each row's columns, pattern pass -> value pass
    int *pairs_tmp = nullptr;     // 3 ninc: each row's pairs grouped by column slot
    int64_t pair_incs = 0;        // incidences the two buffers above can hold
    // element records of the last assembly (FP64 SoA planes; sizes in doubles)
    double *trec = nullptr, *hrec = nullptr, *crec = nullptr;
    size_t trec_elems = 0, hrec_elems = 0, crec_elems = 0;
    int *slice_row0 = nullptr;    // nslices + 1: first row of each slice
    int *row_slice = nullptr;     // nv: slice of each row
    int *slice_psize = nullptr;   // nslices: stored (padded) blocks of each slice
    int *slice_vbase = nullptr;   // nslices + 1: first stored block of each slice
    int slice_cap = 0;            // slices the layout arrays can hold
    int64_t vcap = 0;             // stored-block capacity: cap + padding bound of the slices
    int64_t jcol_blocks = 0;      // blocks jcol can hold
    int64_t hi_blocks = 0;        // blocks jval_hi can hold

    // instances and work schedules (one instance unless pc_set_instances)
    int ninst = 1;
    std::vector<int> inst_row0_h;     // ninst + 1 instance row ranges
    int spb = 8;                      // slices per SpMV work item (wavefronts per block)
    int rpb = 2048;                   // rows per vector work item
    int n_sitems = 0, n_vitems = 0;
    int4 *sitem = nullptr, *vitem = nullptr;
    int *inst_sitem0 = nullptr, *inst_vitem0 = nullptr;
    uint8_t *restart = nullptr;       // per-instance flags (device)
    uint8_t *restart_h = nullptr;     // pinned host staging
    int *maxit_d = nullptr;           // per-instance iteration budget
    int sched_version = 0;
    std::vector<pc_solve_info> inst_info;
    void *jval = nullptr;     // cap * 9 values of dtype (solver copy)
    size_t jval_bytes = 0;
    double *jval_hi = nullptr;  // cap * 9 FP64 values (refinement residual), when dtype != PC_F64
    bool hi_valid = false;
    pc_dtype dtype = PC_F32;
    bool assembled = false;
    bool have_prev_dv = false;  // ctx->tmp holds the previous step's dv
    double *diag = nullptr;   // nv * 3
    float *dinv = nullptr;    // nv * 3: 1 / diag(A)
    float *binv = nullptr;    // nv * 6: inverse of the diagonal block A_ii (xx, xy, xz, yy, yz, zz)

    // solver vectors
    double *x = nullptr, *r = nullptr, *q = nullptr, *tmp = nullptr, *bbuf = nullptr;
    float *p = nullptr;           // nv * 3: search direction (FP32, packed)
    float *zb = nullptr;          // nv * 3: preconditioned residual (block Jacobi; FP32, packed)
    int precond = 0;              // preconditioner of the current / last solve
    int method = 0;               // 0 textbook PCG, 1 single-reduction (Chronopoulos-Gear) form
    double *cg_pd = nullptr;      // nv * 3: direction of the single-reduction form (FP64)
    double *cg_s = nullptr;       // nv * 3: its product s = A p, by recurrence
    bool inner32 = false;         // inner CG vectors (correction, residual, product) in FP32
    bool use_inner32 = true;      // PC_OPT_INNER_FP32
    bool use_keep_dir = false;    // PC_OPT_KEEP_DIRECTION
    float *e32 = nullptr, *r32 = nullptr, *q32 = nullptr;   // nv * 3 each
    double *partials = nullptr;   // per-block partial sums (4 doubles per block): SpMV, starts, checks
    double *partials_u = nullptr; // per-block partial sums of the CG update (2 doubles per block)
    int cg_par = 0;               // parity of the next CG iteration launched
    double *res2 = nullptr;       // 2 doubles per instance: true-residual check
    unsigned *counter = nullptr;
    PcgState *st = nullptr;       // device, one per instance
    PcgState *st_host = nullptr;  // pinned host, one per instance
    int *status_host = nullptr;   // pinned host

    // scan scratch
    int *scan_tmp = nullptr;
    size_t scan_tmp_elems = 0;

    // CG iterations captured as HIP graphs: one per inner operator (0: the
    // solver copy, 1: the FP64 blocks), each `graph_chunk` iterations long.
    int graph_chunk = 0;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    const void *gkey[2] = {nullptr, nullptr};
    int gkey_dtype[2] = {-1, -1};
    int gkey_chunk[2] = {0, 0};
    int gkey_sched[2] = {-1, -1};
    int gkey_pre[2] = {-1, -1};
    int gkey_win[2] = {-1, -1};
    int gkey_narrow[2] = {-1, -1};
    int gkey_method[2] = {-1, -1};
    int gkey_inner32[2] = {-1, -1};

    // column windows of the SpMV work items (p staged in LDS)
    int2 *sitem_win = nullptr;
    int win_items = 0;            // items sitem_win can hold
    bool win_valid = false;
    bool use_win = true;          // PC_OPT_LDS_WINDOW
    int win_cap = 0;              // LDS window rows of the SpMV launches (0: global gathers)

    BellState bell;
};

// Error helpers (host)
#define PC_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);            \
            return PC_ERR_HIP;                                                       \
        }                                                                            \
    } while (0)

// launch-side entry points implemented in the .hip files
pc_status topo_build(Ctx *ctx, const pc_mesh *mesh, hipStream_t s);
pc_status assemble_run(Ctx *ctx, const double *x, const double *v, pc_dtype dtype, double *b,
                       double *diag_out, hipStream_t s);
pc_status export_blocks(Ctx *ctx, double *vals, double *D, bool solver, hipStream_t s);
pc_status spmv_run(Ctx *ctx, const double *xin, double *y, bool solver, hipStream_t s);
pc_status pcg_run(Ctx *ctx, const double *b, double *dv, const pc_solve_opts *o, pc_solve_info *info,
                  hipStream_t s);
pc_status update_run(Ctx *ctx, const double *dv, double *x, double *v, hipStream_t s);
pc_status scan_excl(Ctx *ctx, const int *in, int *out, int n, hipStream_t s);
// Device memory of the library: through the context's allocator
// (pc_set_allocator) when one is installed, else hipMalloc.  Every block is
// returned by dev_free to the routine that allocated it.
pc_status dev_alloc(Ctx *ctx, void **p, size_t bytes);
void dev_free(Ctx *ctx, void *p);
pc_status read_status(Ctx *ctx, hipStream_t s, int *bits);
pc_status build_schedule(Ctx *ctx);
pc_status check_contacts(Ctx *ctx, int nc, int *bad, hipStream_t s);
pc_status bell_assemble(Ctx *ctx, const double *x, const double *v, pc_dtype dtype, double *b, hipStream_t s);
pc_status bell_spmv(Ctx *ctx, const double *x, double *y, hipStream_t s);
pc_status bell_export(Ctx *ctx, int32_t *width, int32_t *cols, double *vals, hipStream_t s);
void bell_free(Ctx *ctx, BellState &Bs);
pc_status set_inner_vectors(Ctx *ctx);
pc_status autotune_run(Ctx *ctx, const double *b, int iters, int64_t *chosen, float *best_ms, hipStream_t s);

}  // namespace pc
