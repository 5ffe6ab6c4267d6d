// C ABI entry points: argument checks, context lifetime, orchestration of
// the assembly / solve / update launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pc_mlp.h"

using namespace pc;

struct pc_ctx {
    Ctx c;
};

static thread_local std::string g_create_err;

// Allocator installed with pc_set_allocator(NULL, ...): contexts created
// afterwards start with it, so their pc_create buffers come from it too.
static std::mutex g_alloc_mu;
static pc_alloc_fn g_alloc_fn = nullptr;
static pc_free_fn g_free_fn = nullptr;
static void *g_alloc_user = nullptr;

namespace pc {

pc_status dev_alloc(Ctx *ctx, void **p, size_t bytes) {
    if (bytes == 0) bytes = 8;
    *p = nullptr;
    if (ctx->alloc_fn) {
        void *q = ctx->alloc_fn(bytes, ctx->alloc_user);
        if (!q) {
            ctx->err = "allocator returned NULL for " + std::to_string(bytes) + " bytes";
            return PC_ERR_OOM;
        }
        if ((reinterpret_cast<uintptr_t>(q) & 255u) != 0) {
            // kernels read every buffer with 16-byte vector loads and rely on
            // the alignment hipMalloc gives
            ctx->free_fn(q, ctx->alloc_user);
            ctx->err = "allocator returned a block that is not 256-byte aligned";
            return PC_ERR_ARG;
        }
        ctx->blocks[q] = AllocRec{ctx->free_fn, ctx->alloc_user};
        *p = q;
        return PC_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        ctx->err = "hipMalloc(" + std::to_string(bytes) + " bytes): " + hipGetErrorString(e);
        return e == hipErrorOutOfMemory ? PC_ERR_OOM : PC_ERR_HIP;
    }
    ctx->blocks[*p] = AllocRec{nullptr, nullptr};
    return PC_OK;
}

// A block from a caller's allocator may be handed out again as soon as it is
// returned, so the device is drained first (frees happen only when a buffer
// grows and at pc_destroy).
void dev_free(Ctx *ctx, void *p) {
    if (!p) return;
    auto it = ctx->blocks.find(p);
    const AllocRec r = it != ctx->blocks.end() ? it->second : AllocRec{nullptr, nullptr};
    if (it != ctx->blocks.end()) ctx->blocks.erase(it);
    if (r.free_fn) {
        (void)hipDeviceSynchronize();
        r.free_fn(p, r.user);
    } else {
        (void)hipFree(p);
    }
}

}  // namespace pc

static DevParams make_params(const pc_params &u) {
    DevParams d;
    d.h = u.h;
    d.mu = u.mu;
    d.lam = u.lambda;
    d.kb = u.k_bend;
    d.beta = u.beta;
    d.g[0] = u.gravity[0];
    d.g[1] = u.gravity[1];
    d.g[2] = u.gravity[2];
    d.c = u.h * (u.h + u.beta);
    d.s_look = u.rhs_mode == 0 ? 1.0 : 0.0;
    d.kv_coef = u.rhs_mode == 0 ? u.beta : u.h + u.beta;
    return d;
}

static bool params_ok(const pc_params *p, std::string &err) {
    if (!p) { err = "params is NULL"; return false; }
    if (!(p->h > 0.0) || !std::isfinite(p->h)) { err = "h must be > 0"; return false; }
    if (!(p->mu >= 0.0) || !(p->lambda >= 0.0) || !(p->k_bend >= 0.0) || !(p->beta >= 0.0)) {
        err = "material constants must be >= 0";
        return false;
    }
    if (p->rhs_mode != 0 && p->rhs_mode != 1) { err = "rhs_mode must be 0 or 1"; return false; }
    return true;
}

static void free_all(Ctx *c) {
    void *ptrs[] = {c->tri, c->Bm, c->A0, c->hinge, c->hcoef, c->htbar, c->mass, c->pinned, c->status,
                    c->inc_cnt, c->inc_ptr, c->inc, c->rowlen, c->rowptr, c->colidx, c->jcol, c->lane_row,
                    c->row_lane, c->slot_cnt, c->jval, c->diag, c->dinv, c->binv, c->zb, c->x, c->r, c->q, c->tmp, c->bbuf,
                    c->p, c->partials, c->partials_u, c->res2, c->counter, c->st, c->scan_tmp, c->jval_hi, c->slice_row0, c->slice_psize, c->slice_vbase, c->sitem_win, c->cverts, c->cw, c->cn, c->jdel, c->cg_pd, c->cg_s, c->e32, c->r32, c->q32,
                    c->row_slice, c->sitem, c->vitem, c->inst_sitem0, c->inst_vitem0, c->restart, c->maxit_d,
                    c->slot_off, c->rowlen_s, c->f16_scale, c->f16_part, c->inst_slice0, c->row_state, c->wide_rows, c->trec, c->hrec, c->crec, c->row_npairs,
                    c->cols_tmp, c->pairs_tmp};
    for (void *p : ptrs) dev_free(c, p);
    if (c->st_host) (void)hipHostFree(c->st_host);
    if (c->restart_h) (void)hipHostFree(c->restart_h);
    if (c->status_host) (void)hipHostFree(c->status_host);
    bell_free(c, c->bell);
}

extern "C" {

const char *pc_last_error(const pc_ctx *ctx) { return ctx ? ctx->c.err.c_str() : g_create_err.c_str(); }

pc_status pc_create(const pc_mesh *mesh, const pc_params *params, pc_ctx **out) {
    g_create_err.clear();
    if (!out) { g_create_err = "out is NULL"; return PC_ERR_ARG; }
    *out = nullptr;
    if (!mesh || !mesh->tris || !mesh->rest || !mesh->mass) { g_create_err = "mesh arrays are NULL"; return PC_ERR_ARG; }
    if (mesh->nv <= 0 || mesh->nt <= 0) { g_create_err = "nv and nt must be > 0"; return PC_ERR_ARG; }
    if (mesh->nt >= (1 << 29) - 1 || mesh->nv >= (1 << 30)) { g_create_err = "mesh too large"; return PC_ERR_ARG; }
    if (!params_ok(params, g_create_err)) return PC_ERR_ARG;
    const int nv = mesh->nv, nt = mesh->nt;
    for (int i = 0; i < nv; ++i)
        if (!(mesh->mass[i] > 0.0) || !std::isfinite(mesh->mass[i])) {
            g_create_err = "mass must be finite and > 0 (vertex " + std::to_string(i) + ")";
            return PC_ERR_ARG;
        }
    for (int64_t k = 0; k < 3 * (int64_t)nt; ++k)
        if (mesh->tris[k] < 0 || mesh->tris[k] >= nv) {
            g_create_err = "triangle index out of range";
            return PC_ERR_MESH;
        }
    pc_ctx *h = new (std::nothrow) pc_ctx();
    if (!h) { g_create_err = "host allocation failed"; return PC_ERR_OOM; }
    Ctx *ctx = &h->c;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        ctx->alloc_fn = g_alloc_fn;
        ctx->free_fn = g_free_fn;
        ctx->alloc_user = g_alloc_user;
    }
    ctx->nv = nv;
    ctx->nt = nt;
    ctx->nslices = (nv + WAVE - 1) / WAVE;
    ctx->user_prm = *params;
    ctx->prm = make_params(*params);
    hipStream_t s = nullptr;
    pc_status st = PC_OK;
    auto fail = [&](pc_status code) {
        g_create_err = ctx->err;
        free_all(ctx);
        delete h;
        return code;
    };
#define ALLOC(ptr, bytes) \
    if ((st = dev_alloc(ctx, (void **)&(ptr), (bytes)))) return fail(st)
    // static data
    ALLOC(ctx->tri, sizeof(int) * 3 * (size_t)nt);
    ALLOC(ctx->Bm, sizeof(double) * 4 * (size_t)nt);
    ALLOC(ctx->A0, sizeof(double) * (size_t)nt);
    ALLOC(ctx->mass, sizeof(double) * (size_t)nv);
    ALLOC(ctx->pinned, (size_t)nv);
    ALLOC(ctx->status, sizeof(int));
    ALLOC(ctx->inc_cnt, sizeof(int) * (size_t)nv);
    ALLOC(ctx->inc_ptr, sizeof(int) * (size_t)(nv + 1));
    ALLOC(ctx->tmp, sizeof(double) * 3 * (size_t)nv);
    {
        std::vector<int> soa(3 * (size_t)nt);
        for (int t = 0; t < nt; ++t)
            for (int k = 0; k < 3; ++k) soa[(size_t)k * nt + t] = mesh->tris[3 * (size_t)t + k];
        if (hipMemcpy(ctx->tri, soa.data(), sizeof(int) * soa.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ctx->tmp, mesh->rest, sizeof(double) * 3 * (size_t)nv, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ctx->mass, mesh->mass, sizeof(double) * (size_t)nv, hipMemcpyHostToDevice) != hipSuccess) {
            ctx->err = "upload failed";
            return fail(PC_ERR_HIP);
        }
        std::vector<uint8_t> pin((size_t)nv, 0);
        if (mesh->pinned)
            for (int i = 0; i < nv; ++i) pin[i] = mesh->pinned[i] ? 1 : 0;
        if (hipMemcpy(ctx->pinned, pin.data(), (size_t)nv, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemset(ctx->status, 0, sizeof(int)) != hipSuccess ||
            hipMemset(ctx->inc_cnt, 0, sizeof(int) * (size_t)nv) != hipSuccess) {
            ctx->err = "upload failed";
            return fail(PC_ERR_HIP);
        }
    }
    {
        double sum = 0.0;
        for (int t = 0; t < nt; ++t)
            for (int k = 0; k < 3; ++k) {
                const double *a = mesh->rest + 3 * (size_t)mesh->tris[3 * (size_t)t + k];
                const double *b = mesh->rest + 3 * (size_t)mesh->tris[3 * (size_t)t + (k + 1) % 3];
                sum += std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) +
                                 (a[2] - b[2]) * (a[2] - b[2]));
            }
        ctx->ell = sum / (3.0 * nt);
    }
    if ((st = topo_build(ctx, mesh, s))) return fail(st);
    const int nh = ctx->nh;
    if (nt >= MAX_ELEMS || nh >= MAX_ELEMS) {
        ctx->err = "more than 2^28 triangles or hinges";
        return fail(PC_ERR_ARG);
    }
    // element records are indexed with 32-bit plane offsets (36 planes per
    // triangle, up to 25 per hinge)
    if ((int64_t)36 * nt >= ((int64_t)1 << 31) || (int64_t)25 * nh >= ((int64_t)1 << 31)) {
        ctx->err = "more than 59,652,323 triangles or 85,899,345 hinges";
        return fail(PC_ERR_ARG);
    }
    ctx->ninc = 3 * (int64_t)nt + 4 * (int64_t)nh;
    ctx->ninc_cap = ctx->ninc;
    // block capacity: diagonal + both directions of every triangle edge (6
    // per triangle, duplicates included) + both wing pairs of every hinge
    ctx->cap = (int64_t)nv + 6 * (int64_t)nt + 2 * (int64_t)nh;
    ctx->cap_base = ctx->cap;
    if (ctx->cap >= (int64_t)1 << 31) {
        ctx->err = "block capacity exceeds int32 indexing";
        return fail(PC_ERR_ARG);
    }
    const size_t nsl = (size_t)ctx->nslices;
    ALLOC(ctx->inc, sizeof(int) * (size_t)ctx->ninc);
    ALLOC(ctx->rowlen, sizeof(int) * (size_t)nv);
    ALLOC(ctx->rowptr, sizeof(int) * (size_t)(nv + 1));
    ALLOC(ctx->colidx, sizeof(int) * (size_t)ctx->cap);
    ALLOC(ctx->row_lane, sizeof(int) * (size_t)nv);
    ALLOC(ctx->diag, sizeof(double) * 3 * (size_t)nv);
    ALLOC(ctx->dinv, sizeof(float) * 3 * (size_t)nv);
    ALLOC(ctx->binv, sizeof(float) * 6 * (size_t)nv);
    ALLOC(ctx->zb, sizeof(float) * 3 * (size_t)nv);
    ALLOC(ctx->x, sizeof(double) * 3 * (size_t)nv);
    ALLOC(ctx->r, sizeof(double) * 3 * (size_t)nv);
    ALLOC(ctx->q, sizeof(double) * 3 * (size_t)nv);
    ALLOC(ctx->bbuf, sizeof(double) * 3 * (size_t)nv);
    ALLOC(ctx->p, sizeof(float) * 3 * (size_t)nv);
    ALLOC(ctx->counter, sizeof(unsigned) * 4);
#undef ALLOC
    (void)nsl;
    if (hipHostMalloc((void **)&ctx->status_host, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        ctx->err = "pinned host allocation failed";
        return fail(PC_ERR_OOM);
    }
    ctx->inst_row0_h = {0, nv};
    ctx->ninst = 0;  // forces the per-instance buffers to be allocated
    if ((st = build_schedule(ctx))) return fail(st);
    if ((st = mlp_scratch_init(ctx))) return fail(st);
    if (hipMemset(ctx->counter, 0, sizeof(unsigned) * 4) != hipSuccess ||
        hipMemset(ctx->tmp, 0, sizeof(double) * 3 * (size_t)nv) != hipSuccess ||
        hipMemset(ctx->p, 0, sizeof(float) * 3 * (size_t)nv) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        ctx->err = "initialisation failed";
        return fail(PC_ERR_HIP);
    }
    *out = h;
    return PC_OK;
}

pc_status pc_set_allocator(pc_ctx *h, pc_alloc_fn alloc, pc_free_fn free_fn, void *user) {
    if ((alloc == nullptr) != (free_fn == nullptr)) {
        if (h) h->c.err = "pc_set_allocator: give both routines or neither";
        else g_create_err = "pc_set_allocator: give both routines or neither";
        return PC_ERR_ARG;
    }
    if (!h) {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        g_alloc_fn = alloc;
        g_free_fn = free_fn;
        g_alloc_user = alloc ? user : nullptr;
        return PC_OK;
    }
    h->c.alloc_fn = alloc;
    h->c.free_fn = free_fn;
    h->c.alloc_user = alloc ? user : nullptr;
    return PC_OK;
}

pc_status pc_profile(pc_ctx *h, int32_t every) {
    if (!h || every < 0) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    (void)hipDeviceSynchronize();
    ctx->prof.harvest();
    ctx->prof.init(512);
    ctx->prof.reset();
    ctx->prof.every = every;
    return PC_OK;
}

pc_status pc_profile_read(pc_ctx *h, double *out) {
    if (!h || !out) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    PC_HIP(hipDeviceSynchronize());
    ctx->prof.harvest();
    for (int k = 0; k < PK_NKINDS; ++k) {
        const long long n = ctx->prof.count[k];
        out[5 * k] = (double)n;
        out[5 * k + 1] = n ? ctx->prof.sum_ms[k] / n : 0.0;
        out[5 * k + 2] = ctx->prof.min_ms[k];
        out[5 * k + 3] = ctx->prof.max_ms[k];
        out[5 * k + 4] = ctx->prof.median(k);
    }
    return PC_OK;
}

pc_status pc_set_option(pc_ctx *h, int32_t option, int64_t value) {
    if (!h) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    switch (option) {
        case PC_OPT_GRAPH_CHUNK:
            if (value < 0 || value > 4096) {
                ctx->err = "graph chunk must be in [0, 4096]";
                return PC_ERR_ARG;
            }
            ctx->graph_chunk = (int)((value + 1) & ~1LL);   // even: a replay keeps the iteration parity
            return PC_OK;
        case PC_OPT_LDS_WINDOW:
            if (value != 0 && value != 1) {
                ctx->err = "LDS window option must be 0 or 1";
                return PC_ERR_ARG;
            }
            ctx->use_win = value != 0;
            ctx->win_valid = false;
            return PC_OK;
        case PC_OPT_NARROW_COLUMNS:
            if (value != 0 && value != 1) {
                ctx->err = "narrow column option must be 0 or 1";
                return PC_ERR_ARG;
            }
            ctx->use_narrow = value != 0;
            return PC_OK;
        case PC_OPT_INNER_FP32:
            if (value != 0 && value != 1) {
                ctx->err = "inner FP32 option must be 0 or 1";
                return PC_ERR_ARG;
            }
            ctx->use_inner32 = value != 0;
            return PC_OK;
        case PC_OPT_KEEP_DIRECTION:
            if (value != 0 && value != 1) {
                ctx->err = "keep-direction option must be 0 or 1";
                return PC_ERR_ARG;
            }
            ctx->use_keep_dir = value != 0;
            return PC_OK;
        case PC_OPT_SPMV_SLICES_PER_BLOCK: {
            if (value != 1 && value != 2 && value != 4 && value != 8 && value != 16) {
                ctx->err = "slices per block must be 1, 2, 4, 8 or 16";
                return PC_ERR_ARG;
            }
            const bool was = ctx->assembled;
            ctx->spb = (int)value;
            pc_status st = build_schedule(ctx);
            ctx->assembled = was;  // the slices themselves are unchanged
            return st;
        }
        case PC_OPT_VECTOR_ROWS_PER_BLOCK: {
            if (value < 64 || value > 4096 || (value % 64)) {
                ctx->err = "rows per block must be a multiple of 64 in [64, 4096]";
                return PC_ERR_ARG;
            }
            const bool was = ctx->assembled;
            ctx->rpb = (int)value;
            pc_status st = build_schedule(ctx);
            ctx->assembled = was;
            return st;
        }
        default:
            ctx->err = "unknown option";
            return PC_ERR_ARG;
    }
}

pc_status pc_get_option(pc_ctx *h, int32_t option, int64_t *value) {
    if (!h || !value) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    switch (option) {
        case PC_OPT_GRAPH_CHUNK: *value = ctx->graph_chunk; return PC_OK;
        case PC_OPT_SPMV_SLICES_PER_BLOCK: *value = ctx->spb; return PC_OK;
        case PC_OPT_VECTOR_ROWS_PER_BLOCK: *value = ctx->rpb; return PC_OK;
        case PC_OPT_LDS_WINDOW: *value = ctx->use_win ? 1 : 0; return PC_OK;
        case PC_OPT_NARROW_COLUMNS: *value = ctx->use_narrow ? 1 : 0; return PC_OK;
        case PC_OPT_SPMV_NARROW_ACTIVE:
            *value = (ctx->use_narrow && ctx->narrow && ctx->win_valid) ? 1 : 0;
            return PC_OK;
        case PC_OPT_INNER_FP32: *value = ctx->use_inner32 ? 1 : 0; return PC_OK;
        case PC_OPT_KEEP_DIRECTION: *value = ctx->use_keep_dir ? 1 : 0; return PC_OK;
        default: ctx->err = "unknown option"; return PC_ERR_ARG;
    }
}

pc_status pc_autotune(pc_ctx *h, const double *b, int32_t iters, int32_t precond, int64_t *chosen,
                      double *ms_per_iter, void *stream) {
    if (!h || !b || iters < 1 || precond < 0 || precond > 1) return PC_ERR_ARG;
    h->c.precond = precond;
    h->c.method = 0;   // the schedule is timed on the textbook iteration
    pc_status ist = set_inner_vectors(&h->c);
    if (ist) return ist;
    float ms = 0.0f;
    pc_status st = autotune_run(&h->c, b, iters, chosen, &ms, (hipStream_t)stream);
    if (ms_per_iter) *ms_per_iter = ms;
    return st;
}

// True when some contact pair has vertices in two instances (bounds: ninst + 1
// first rows).  Reads the context's contact vertices back to the host.
static pc_status contacts_cross(Ctx *ctx, const int32_t *bounds, int ninst, bool *cross) {
    *cross = false;
    if (ctx->nc == 0 || ninst <= 1) return PC_OK;
    std::vector<int> cv((size_t)4 * ctx->nc);
    PC_HIP(hipMemcpy(cv.data(), ctx->cverts, sizeof(int) * cv.size(), hipMemcpyDeviceToHost));
    auto inst = [&](int v) { return (int)(std::upper_bound(bounds, bounds + ninst + 1, v) - bounds) - 1; };
    for (int e = 0; e < ctx->nc && !*cross; ++e) {
        const int i0 = inst(cv[4 * (size_t)e]);
        for (int k = 1; k < 4; ++k)
            if (inst(cv[4 * (size_t)e + k]) != i0) *cross = true;
    }
    return PC_OK;
}

pc_status pc_set_instances(pc_ctx *h, const int32_t *vertex_begin, int32_t ninst) {
    if (!h || !vertex_begin || ninst < 1) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    if (vertex_begin[0] != 0 || vertex_begin[ninst] != ctx->nv) {
        ctx->err = "instance ranges must start at 0 and end at nv";
        return PC_ERR_ARG;
    }
    for (int i = 0; i < ninst; ++i)
        if (vertex_begin[i + 1] <= vertex_begin[i]) {
            ctx->err = "instance ranges must be non-empty and increasing";
            return PC_ERR_ARG;
        }
    // no triangle may join two instances
    std::vector<int> tri((size_t)3 * ctx->nt);
    PC_HIP(hipMemcpy(tri.data(), ctx->tri, sizeof(int) * tri.size(), hipMemcpyDeviceToHost));
    std::vector<int> inst_of(ctx->nv);
    for (int i = 0; i < ninst; ++i)
        for (int v = vertex_begin[i]; v < vertex_begin[i + 1]; ++v) inst_of[v] = i;
    for (int t = 0; t < ctx->nt; ++t) {
        const int a = inst_of[tri[t]], b = inst_of[tri[(size_t)ctx->nt + t]], c = inst_of[tri[2 * (size_t)ctx->nt + t]];
        if (a != b || b != c) {
            ctx->err = "triangle " + std::to_string(t) + " joins two instances";
            return PC_ERR_MESH;
        }
    }
    bool cross = false;
    pc_status cst = contacts_cross(ctx, vertex_begin, ninst, &cross);
    if (cst) return cst;
    if (cross) {
        ctx->err = "a contact pair joins two instances";
        return PC_ERR_ARG;
    }
    ctx->inst_row0_h.assign(vertex_begin, vertex_begin + ninst + 1);
    return build_schedule(ctx);
}

pc_status pc_get_instance_info(pc_ctx *h, pc_solve_info *infos, int32_t n) {
    if (!h || !infos || n != h->c.ninst) return PC_ERR_ARG;
    for (int i = 0; i < n; ++i) infos[i] = h->c.inst_info[i];
    return PC_OK;
}

static MlpState *mlp_of(Ctx *ctx) {
    if (!ctx->mlp) ctx->mlp = new (std::nothrow) MlpState();
    return ctx->mlp;
}

pc_status pc_ws_set_params(pc_ctx *h, const float *params_host, int32_t n) {
    if (!h || !params_host || n != PC_WS_PARAMS) return PC_ERR_ARG;
    MlpState *M = mlp_of(&h->c);
    if (!M) return PC_ERR_OOM;
    return mlp_set_params(&h->c, M, params_host);
}

pc_status pc_ws_get_params(pc_ctx *h, float *params_host, int32_t n) {
    if (!h || !params_host || n != PC_WS_PARAMS) return PC_ERR_ARG;
    if (!h->c.mlp) { h->c.err = "no warm-start parameters set"; return PC_ERR_ARG; }
    return mlp_get_params(&h->c, h->c.mlp, params_host);
}

static bool ws_args(Ctx *ctx, const void *x, const void *v, const void *b, const void *dvp) {
    if (!x || !v || !b || !dvp) { ctx->err = "warm start: x, v, b, dv_prev must be device pointers"; return false; }
    if (!ctx->assembled) { ctx->err = "warm start: nothing assembled"; return false; }
    return true;
}

pc_status pc_ws_features(pc_ctx *h, const double *x, const double *v, const double *b, const double *dv_prev,
                         uint16_t *feat_out, void *stream) {
    if (!h || !feat_out || !ws_args(&h->c, x, v, b, dv_prev)) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    MlpState *M = mlp_of(ctx);
    if (!M) return PC_ERR_OOM;
    hipStream_t s = (hipStream_t)stream;
    pc_status st = mlp_features(ctx, M, x, v, b, dv_prev, s);
    if (st) return st;
    PC_HIP(hipMemcpyAsync(feat_out, M->X, sizeof(short) * 32 * (size_t)ctx->nv, hipMemcpyDeviceToDevice, s));
    return PC_OK;
}

pc_status pc_ws_predict(pc_ctx *h, const double *x, const double *v, const double *b, const double *dv_prev,
                        double *dv0_out, void *stream) {
    if (!h || !dv0_out || !ws_args(&h->c, x, v, b, dv_prev)) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    if (!ctx->mlp || !ctx->mlp->has_params) { ctx->err = "no warm-start parameters set"; return PC_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    pc_status st = mlp_features(ctx, ctx->mlp, x, v, b, dv_prev, s);
    if (st) return st;
    return mlp_forward(ctx, ctx->mlp, dv_prev, dv0_out, false, s);
}

pc_status pc_ws_predict_noalloc(pc_ctx *h, const double *x, const double *v, const double *b,
                                const double *dv_prev, double *dv0_out, void *stream) {
    if (!h) return PC_ERR_ARG;
    if (!x || !v || !b || !dv_prev || !dv0_out) {
        h->c.err = "pc_ws_predict_noalloc: x, v, b, dv_prev and dv0_out must be device pointers";
        return PC_ERR_ARG;
    }
    return mlp_predict_noalloc(&h->c, x, v, b, dv_prev, dv0_out, (hipStream_t)stream);
}

pc_status pc_ws_start(pc_ctx *h, const double *x, const double *v, const double *b, const double *dv_prev,
                      double *dv0_out, double *step_host, void *stream) {
    if (!h || !dv0_out || !ws_args(&h->c, x, v, b, dv_prev)) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    if (!ctx->mlp || !ctx->mlp->has_params) { ctx->err = "no warm-start parameters set"; return PC_ERR_ARG; }
    if (!ctx->assembled) { ctx->err = "pc_ws_start: nothing assembled"; return PC_ERR_ARG; }
    int used = 0;
    pc_status st = mlp_start(ctx, ctx->mlp, x, v, b, dv_prev, dv0_out, ctx->q, &used, (hipStream_t)stream);
    if (st) return st;
    if (step_host) *step_host = ctx->mlp->last_scale;
    return PC_OK;
}

pc_status pc_ws_gradient(pc_ctx *h, const double *x, const double *v, const double *b, const double *dv_prev,
                         float *grad_host, double *loss_host, void *stream) {
    if (!h || !ws_args(&h->c, x, v, b, dv_prev)) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    if (!ctx->mlp || !ctx->mlp->has_params) { ctx->err = "no warm-start parameters set"; return PC_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    double loss = 0.0;
    pc_status st = mlp_gradient(ctx, ctx->mlp, x, v, b, dv_prev, &loss, s);
    if (st) return st;
    PC_HIP(hipStreamSynchronize(s));
    if (loss_host) *loss_host = loss;
    if (grad_host) return mlp_get_grads(ctx, ctx->mlp, grad_host);
    return PC_OK;
}

pc_status pc_ws_train_step(pc_ctx *h, const double *x, const double *v, const double *b, const double *dv_prev,
                           double lr, double *loss_host, void *stream) {
    if (!h || !ws_args(&h->c, x, v, b, dv_prev) || !(lr >= 0.0)) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    if (!ctx->mlp || !ctx->mlp->has_params) { ctx->err = "no warm-start parameters set"; return PC_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    pc_status st = mlp_gradient(ctx, ctx->mlp, x, v, b, dv_prev, loss_host, s);
    if (st) return st;
    return mlp_adam(ctx, ctx->mlp, lr, s);
}

pc_status pc_mfma_probe(pc_ctx *h, float *out_host) {
    if (!h || !out_host) return PC_ERR_ARG;
    return mlp_probe(&h->c, out_host);
}

pc_status pc_destroy(pc_ctx *h) {
    if (!h) return PC_ERR_ARG;
    (void)hipDeviceSynchronize();
    if (h->c.mlp) {
        mlp_free(&h->c, h->c.mlp);
        delete h->c.mlp;
        h->c.mlp = nullptr;
    }
    h->c.prof.destroy();
    for (int v = 0; v < 2; ++v)
        if (h->c.gexec[v]) (void)hipGraphExecDestroy(h->c.gexec[v]);
    if (h->c.cap_stream) (void)hipStreamDestroy(h->c.cap_stream);
    free_all(&h->c);
    delete h;
    return PC_OK;
}

pc_status pc_set_params(pc_ctx *h, const pc_params *params) {
    if (!h) return PC_ERR_ARG;
    if (!params_ok(params, h->c.err)) return PC_ERR_ARG;
    h->c.user_prm = *params;
    h->c.prm = make_params(*params);
    return PC_OK;
}

pc_status pc_sizes(const pc_ctx *h, int64_t out[4]) {
    if (!h || !out) return PC_ERR_ARG;
    out[0] = h->c.nv;
    out[1] = h->c.nt;
    out[2] = h->c.nh;
    out[3] = h->c.cap;
    return PC_OK;
}

pc_status pc_get_hinges(pc_ctx *h, int32_t *hinges_host, double *coef_host) {
    if (!h) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    const int nh = ctx->nh;
    if (nh == 0) return PC_OK;
    if (hinges_host) {
        std::vector<int> soa(4 * (size_t)nh);
        PC_HIP(hipMemcpy(soa.data(), ctx->hinge, sizeof(int) * soa.size(), hipMemcpyDeviceToHost));
        for (int e = 0; e < nh; ++e)
            for (int k = 0; k < 4; ++k) hinges_host[4 * (size_t)e + k] = soa[(size_t)k * nh + e];
    }
    if (coef_host) {
        std::vector<double> c(nh), t(nh);
        PC_HIP(hipMemcpy(c.data(), ctx->hcoef, sizeof(double) * nh, hipMemcpyDeviceToHost));
        PC_HIP(hipMemcpy(t.data(), ctx->htbar, sizeof(double) * nh, hipMemcpyDeviceToHost));
        for (int e = 0; e < nh; ++e) {
            coef_host[2 * (size_t)e] = c[e];
            coef_host[2 * (size_t)e + 1] = t[e];
        }
    }
    return PC_OK;
}

static bool dtype_ok(Ctx *ctx, pc_dtype dtype) {
    if (dtype == PC_F64 || dtype == PC_F32 || dtype == PC_BF16 || dtype == PC_F16) return true;
    ctx->err = "bad dtype " + std::to_string((int)dtype);
    return false;
}

pc_status cloth_assemble(pc_ctx *h, const double *x, const double *v, pc_dtype dtype, pc_bsr3 *A_out, double *b,
                         double *diag_out, void *stream) {
    if (!h) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    if (!x || !v || !b) { ctx->err = "cloth_assemble: x, v and b must be device pointers"; return PC_ERR_ARG; }
    if (!dtype_ok(ctx, dtype)) return PC_ERR_ARG;
    pc_status st = assemble_run(ctx, x, v, dtype, b, diag_out, (hipStream_t)stream);
    if (st) return st;
    if (A_out) {
        A_out->rowptr = ctx->rowptr;
        A_out->colidx = ctx->colidx;
        A_out->dtype = dtype;
        A_out->nrows = ctx->nv;
        A_out->nnzb = -1;  // known after synchronisation: rowptr[nrows]
    }
    return PC_OK;
}

pc_status pc_check(pc_ctx *h, void *stream) {
    if (!h) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    int bits = 0;
    pc_status st = read_status(ctx, (hipStream_t)stream, &bits);
    if (st) return st;
    if (bits & (ST_INC_OVERFLOW | ST_COL_OVERFLOW | ST_BUCKET_OVERFLOW)) {
        ctx->err = "a vertex exceeds the per-row limits (512 incident element corners, 64 block columns; at pc_create: 64 directed edges from a lower-numbered vertex)";
        return PC_ERR_CAPACITY;
    }
    if (bits & ST_NONFINITE) {
        ctx->err = "non-finite right-hand side";
        PC_HIP(hipMemsetAsync(ctx->status, 0, sizeof(int), (hipStream_t)stream));
        return PC_ERR_NONFINITE;
    }
    if (bits) {
        ctx->err = "device check bits " + std::to_string(bits);
        return PC_ERR_MESH;
    }
    return PC_OK;
}

static bool opts_ok(Ctx *ctx, const pc_solve_opts *o) {
    if (o && (!(o->tol >= 0.0) || o->warm < 0 || o->warm > 2 || !(o->inner_rho >= 0.0) || o->inner_rho >= 1.0 ||
              o->precond < 0 || o->precond > 1 || o->method < 0 || o->method > 1)) {
        ctx->err = "bad solve options";
        return false;
    }
    return true;
}

pc_status cloth_pcg_solve(pc_ctx *h, const double *b, double *dv, const pc_solve_opts *opts, pc_solve_info *info,
                          void *stream) {
    if (!h) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    if (!b || !dv) { ctx->err = "cloth_pcg_solve: b and dv must be device pointers"; return PC_ERR_ARG; }
    if (!opts_ok(ctx, opts)) return PC_ERR_ARG;
    pc_status st = pc_check(h, stream);
    if (st) return st;
    return pcg_run(ctx, b, dv, opts, info, (hipStream_t)stream);
}

pc_status cloth_spmv(pc_ctx *h, const double *x, double *y, int32_t solver_blocks, void *stream) {
    if (!h || !x || !y) return PC_ERR_ARG;
    return spmv_run(&h->c, x, y, solver_blocks != 0, (hipStream_t)stream);
}

pc_status cloth_export_pattern(pc_ctx *h, int32_t *rowptr_out, int32_t *colidx_out, int64_t *nnzb_out,
                               void *stream) {
    if (!h) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    if (!ctx->assembled) { ctx->err = "cloth_export_pattern: nothing assembled"; return PC_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    pc_status st = pc_check(h, stream);
    if (st) return st;
    int nnzb = 0;
    PC_HIP(hipMemcpyAsync(ctx->status_host, ctx->rowptr + ctx->nv, sizeof(int), hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
    nnzb = *ctx->status_host;
    if (nnzb_out) *nnzb_out = nnzb;
    if (rowptr_out)
        PC_HIP(hipMemcpyAsync(rowptr_out, ctx->rowptr, sizeof(int) * (size_t)(ctx->nv + 1), hipMemcpyDeviceToDevice, s));
    if (colidx_out && nnzb > 0)
        PC_HIP(hipMemcpyAsync(colidx_out, ctx->colidx, sizeof(int) * (size_t)nnzb, hipMemcpyDeviceToDevice, s));
    return PC_OK;
}

pc_status cloth_export_blocks(pc_ctx *h, double *vals_out, double *D_out, int32_t solver_blocks, void *stream) {
    if (!h || !vals_out) return PC_ERR_ARG;
    return export_blocks(&h->c, vals_out, D_out, solver_blocks != 0, (hipStream_t)stream);
}

pc_status cloth_assemble_bell(pc_ctx *h, const double *x, const double *v, pc_dtype dtype, double *b,
                              int32_t *width_out, void *stream) {
    if (!h) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    if (!x || !v || !b) { ctx->err = "cloth_assemble_bell: x, v and b must be device pointers"; return PC_ERR_ARG; }
    pc_status st = bell_assemble(ctx, x, v, dtype, b, (hipStream_t)stream);
    if (st) return st;
    if ((st = pc_check(h, stream))) return st;
    if (width_out) *width_out = ctx->bell.Wv;
    return PC_OK;
}

pc_status cloth_spmv_bell(pc_ctx *h, const double *x, double *y, void *stream) {
    if (!h) return PC_ERR_ARG;
    if (!x || !y) { h->c.err = "cloth_spmv_bell: x and y must be device pointers"; return PC_ERR_ARG; }
    return bell_spmv(&h->c, x, y, (hipStream_t)stream);
}

pc_status cloth_export_bell(pc_ctx *h, int32_t *width_out, int32_t *cols_out, double *vals_out, void *stream) {
    if (!h) return PC_ERR_ARG;
    return bell_export(&h->c, width_out, cols_out, vals_out, (hipStream_t)stream);
}

pc_status cloth_set_contacts(pc_ctx *h, int32_t ncontacts, const int32_t *verts, const double *weights,
                             const double *normals, double thickness, double stiffness, void *stream) {
    if (!h) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    hipStream_t s = (hipStream_t)stream;
    if (ncontacts < 0 || ncontacts >= MAX_ELEMS) { ctx->err = "bad contact count"; return PC_ERR_ARG; }
    if (ncontacts > 0 && (!verts || !weights || !normals)) {
        ctx->err = "cloth_set_contacts: null contact arrays";
        return PC_ERR_ARG;
    }
    if (ncontacts > 0 && (!(thickness > 0.0) || !(stiffness >= 0.0) || !std::isfinite(thickness) ||
                          !std::isfinite(stiffness))) {
        ctx->err = "cloth_set_contacts: thickness must be > 0 and stiffness >= 0";
        return PC_ERR_ARG;
    }
    pc_status st;
    const int64_t nc = ncontacts;
    if (nc > ctx->nc_cap) {
        void **bufs[] = {(void **)&ctx->cverts, (void **)&ctx->cw, (void **)&ctx->cn};
        const size_t sizes[] = {sizeof(int) * 4 * (size_t)nc, sizeof(double) * 4 * (size_t)nc,
                                sizeof(double) * 3 * (size_t)nc};
        for (int k = 0; k < 3; ++k) {
            dev_free(ctx, *bufs[k]);
            *bufs[k] = nullptr;
        }
        ctx->nc_cap = 0;
        for (int k = 0; k < 3; ++k)
            if ((st = dev_alloc(ctx, bufs[k], sizes[k]))) return st;
        ctx->nc_cap = nc;
    }
    if (nc > 0) {
        PC_HIP(hipMemcpyAsync(ctx->cverts, verts, sizeof(int) * 4 * (size_t)nc, hipMemcpyDeviceToDevice, s));
        PC_HIP(hipMemcpyAsync(ctx->cw, weights, sizeof(double) * 4 * (size_t)nc, hipMemcpyDeviceToDevice, s));
        PC_HIP(hipMemcpyAsync(ctx->cn, normals, sizeof(double) * 3 * (size_t)nc, hipMemcpyDeviceToDevice, s));
        int bad = 0;
        if ((st = check_contacts(ctx, (int)nc, &bad, s))) return st;
        if (bad) {
            ctx->nc = 0;
            ctx->assembled = false;
            ctx->err = "cloth_set_contacts: a contact has an index out of range, repeated vertices, weights "
                       "not summing to zero or a normal that is not unit length";
            return PC_ERR_ARG;
        }
    }
    // capacities: 4 incidences and at most 12 more blocks per contact
    const int64_t ninc = 3 * (int64_t)ctx->nt + 4 * (int64_t)ctx->nh + 4 * nc;
    if (ninc > ctx->ninc_cap) {
        dev_free(ctx, ctx->inc);
        ctx->inc = nullptr;
        ctx->ninc_cap = 0;
        if ((st = dev_alloc(ctx, (void **)&ctx->inc, sizeof(int) * (size_t)ninc))) return st;
        ctx->ninc_cap = ninc;
    }
    ctx->ninc = ninc;
    const int64_t cap = ctx->cap_base + 12 * nc;
    if (cap >= (int64_t)1 << 31) {
        ctx->err = "block capacity exceeds int32 indexing";
        return PC_ERR_CAPACITY;
    }
    if (cap > ctx->cap) {
        dev_free(ctx, ctx->colidx);
        ctx->colidx = nullptr;
        if ((st = dev_alloc(ctx, (void **)&ctx->colidx, sizeof(int) * (size_t)cap))) return st;
        ctx->cap = cap;
        if ((st = build_schedule(ctx))) return st;   // stored-block capacity follows cap
    }
    ctx->nc = (int)nc;
    ctx->ceta = thickness;
    ctx->ckc = stiffness;
    ctx->assembled = false;   // the pattern changes with the contacts
    bool cross = false;
    if ((st = contacts_cross(ctx, ctx->inst_row0_h.data(), ctx->ninst, &cross))) return st;
    if (cross) {
        ctx->nc = 0;
        ctx->err = "cloth_set_contacts: a contact pair joins two instances";
        return PC_ERR_ARG;
    }
    return PC_OK;
}

pc_status cloth_export_precond(pc_ctx *h, float *inv_diag_out, float *inv_blocks_out, void *stream) {
    if (!h) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    if (!ctx->assembled) { ctx->err = "cloth_export_precond: nothing assembled"; return PC_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    const size_t nv = (size_t)ctx->nv;
    if (inv_diag_out)
        PC_HIP(hipMemcpyAsync(inv_diag_out, ctx->dinv, sizeof(float) * 3 * nv, hipMemcpyDeviceToDevice, s));
    if (inv_blocks_out)
        PC_HIP(hipMemcpyAsync(inv_blocks_out, ctx->binv, sizeof(float) * 6 * nv, hipMemcpyDeviceToDevice, s));
    return PC_OK;
}

pc_status cloth_step(pc_ctx *h, double *x, double *v, int32_t nsteps, pc_dtype dtype, const pc_solve_opts *opts,
                     pc_solve_info *infos, void *stream) {
    if (!h) return PC_ERR_ARG;
    Ctx *ctx = &h->c;
    if (!x || !v || nsteps < 0) { ctx->err = "cloth_step: bad arguments"; return PC_ERR_ARG; }
    if (!opts_ok(ctx, opts) || !dtype_ok(ctx, dtype)) return PC_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    pc_solve_opts o = opts ? *opts : pc_solve_opts{1e-6, 0.0, 20000, 0, 0, 0, 0, 0};
    // dv lives in ctx->tmp between steps (previous-step start when warm = 1)
    for (int k = 0; k < nsteps; ++k) {
        pc_status st = assemble_run(ctx, x, v, dtype, ctx->bbuf, nullptr, s);
        if (st) return st;
        pc_solve_info info{};
        if ((st = pc_check(h, stream))) return st;
        pc_solve_opts ok = o;
        if (!ctx->have_prev_dv && ok.warm == 1) ok.warm = 0;  // the learned start accepts dv_prev = 0
        st = pcg_run(ctx, ctx->bbuf, ctx->tmp, &ok, &info, s);
        if (infos) infos[k] = info;
        if (st) return st;
        if ((st = update_run(ctx, ctx->tmp, x, v, s))) return st;
        ctx->have_prev_dv = true;
    }
    PC_HIP(hipStreamSynchronize(s));
    return PC_OK;
}

}  // extern "C"
