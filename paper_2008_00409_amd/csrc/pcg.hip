// Block SpMV and Jacobi-preconditioned CG (paper Sec. 2.5: the linear system
// of Eq. 3 is solved by PCG each step; Sec. 3.1: SpMV is the dominant
// operator, vector operations are element-wise).
//
// Solver layout: rows are grouped in slices of 64 (one wavefront); inside a
// slice they are ordered by decreasing length, and block k of every row with
// more than k blocks is stored contiguously (column index plane, then 9 value
// planes), so each load instruction of the wavefront reads consecutive
// addresses and no padding is stored.
//
// The operator is applied in difference form
//   y_i = m_i x_i + D_i x_i + sum_{j != i} A_ij (x_j - x_i),
// where the diagonal slot stores the remainder D_i, so that rounding of the
// stored (FP32/BF16) blocks leaves the mass term and the exact null space of
// the stiffness intact.  All arithmetic is FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "pc_ctx.h"

namespace pc {

struct SpmvArgs {
    int nv, nslices;
    const int *rowptr;
    const uint8_t *slot_cnt;
    const int *lane_row;
    const int *jcol;
    const void *jval;
    const double *mass;
};

// Streamed (read-once per product) loads bypass cache retention so that the
// gathered vector stays resident.
__device__ __forceinline__ double ld_stream(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_stream(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ bf16_t ld_stream(const bf16_t *p) {
    return bf16_t{__builtin_nontemporal_load(&p->bits)};
}

struct VecF4 {
    const float4 *p;
    __device__ __forceinline__ void load(int i, double &a, double &b, double &c) const {
        const float4 v = p[i];
        a = v.x; b = v.y; c = v.z;
    }
};
struct VecD3 {
    const double *p;
    __device__ __forceinline__ void load(int i, double &a, double &b, double &c) const {
        a = p[3 * i]; b = p[3 * i + 1]; c = p[3 * i + 2];
    }
};

// One row of the difference-form product for the lane's row of `slice`.
// Lane k of the wavefront holds slot k's row count and start offset, so the
// per-slot values are read with readlane instead of memory loads; slots are
// processed UNROLL at a time with all column-index and value loads of the
// group issued before the gathers of x, to keep several loads in flight.
template <typename TB, typename V, int UNROLL = 4>
__device__ __forceinline__ int spmv_row(const SpmvArgs &M, int slice, int lane, const V &x, double y[3],
                                        double xi[3]) {
    const int row = M.lane_row[slice * WAVE + lane];
    const int base = M.rowptr[slice * WAVE];
    const int my_cnt = (int)M.slot_cnt[slice * WAVE + lane];
    const int my_off = base + wave_excl_scan(my_cnt);
    const int nslots = __popcll(__ballot(my_cnt > 0));  // counts are non-increasing in the slot
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    if (row >= 0) x.load(row, x0, x1, x2);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int k = 0; k < nslots; k += UNROLL) {
        int jc[UNROLL];
        TB v[UNROLL][9];
        bool act[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int kk = min(k + u, WAVE - 1);
            const int c = __builtin_amdgcn_readlane(my_cnt, kk);
            const int off = __builtin_amdgcn_readlane(my_off, kk);
            act[u] = (k + u < nslots) && lane < c;
            jc[u] = row;
            if (act[u]) {
                jc[u] = __builtin_nontemporal_load(M.jcol + off + lane);
                const TB *vp = (const TB *)M.jval + 9 * (int64_t)off + lane;
#pragma unroll
                for (int e = 0; e < 9; ++e) v[u][e] = ld_stream(vp + (int64_t)e * c);
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (!act[u]) continue;
            double d0, d1, d2;
            if (jc[u] == row) {
                d0 = x0; d1 = x1; d2 = x2;
            } else {
                x.load(jc[u], d0, d1, d2);
                d0 -= x0; d1 -= x1; d2 -= x2;
            }
            a0 += to_f64(v[u][0]) * d0 + to_f64(v[u][1]) * d1 + to_f64(v[u][2]) * d2;
            a1 += to_f64(v[u][3]) * d0 + to_f64(v[u][4]) * d1 + to_f64(v[u][5]) * d2;
            a2 += to_f64(v[u][6]) * d0 + to_f64(v[u][7]) * d1 + to_f64(v[u][8]) * d2;
        }
    }
    if (row >= 0) {
        const double m = M.mass[row];
        y[0] = a0 + m * x0;
        y[1] = a1 + m * x1;
        y[2] = a2 + m * x2;
    } else {
        y[0] = y[1] = y[2] = 0.0;
    }
    xi[0] = x0; xi[1] = x1; xi[2] = x2;
    return row;
}

__device__ __forceinline__ int slice_of_thread(int nslices) {
    const int wpb = blockDim.x / WAVE;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    return __builtin_amdgcn_readfirstlane(b * wpb + (int)(threadIdx.x / WAVE));
}

__device__ __forceinline__ int row_of_thread() {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    return b * blockDim.x + threadIdx.x;
}

// ---------------------------------------------------------------- reductions
// Deterministic two-stage sums without device-scope fences: every block of a
// producing kernel writes its NV partial sums (plain stores, block order), and
// a one-block finalize kernel launched next adds them in block order; the
// kernel boundary makes the partials visible.  partials layout: [q][block].
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double *partials) {
    __shared__ double sh[NV][16];
    const int lane = lane_id(), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) sh[q][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int q = threadIdx.x;
        double s = 0.0;
        for (int k = 0; k < nw; ++k) s += sh[q][k];
        partials[(size_t)q * gridDim.x + blockIdx.x] = s;
    }
}

// Sum of partials[q][0..n) in a fixed order, valid in every thread of a
// single 1024-thread block.
template <int NV>
__device__ __forceinline__ void finalize_sum(const double *partials, int n, double (&tot)[NV]) {
    __shared__ double sh[NV][16];
    const int lane = lane_id(), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    double loc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) loc[q] = 0.0;
    for (int b = threadIdx.x; b < n; b += blockDim.x)
#pragma unroll
        for (int q = 0; q < NV; ++q) loc[q] += partials[(size_t)q * n + b];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double s = wave_sum(loc[q]);
        if (lane == 0) sh[q][w] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
        for (int k = 0; k < nw; ++k) s += sh[q][k];
        tot[q] = s;
    }
}

// ---------------------------------------------------------------- kernels
__global__ void k_state_init(PcgState *st, double tol, double rho, int maxit) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->rz = st->pq = st->alpha = st->beta = st->rr = st->bb = 0.0;
        st->tol2 = tol * tol;
        st->rho2 = rho * rho;
        st->thresh = 0.0;
        st->rr0 = 0.0;
        st->rz0 = 0.0;
        st->iters = 0;
        st->maxit = maxit;
        st->done = 0;
        st->flags = 0;
    }
}

// q = A p and per-block partials of p.q.
template <typename TB>
__global__ void __launch_bounds__(256) k_pcg_spmv(SpmvArgs M, const float4 *p, double *q, const PcgState *st,
                                                  double *partials) {
    if (st->done) return;
    const int slice = slice_of_thread(M.nslices);
    const int lane = lane_id();
    double pq = 0.0;
    if (slice < M.nslices) {
        double y[3], xi[3];
        const int row = spmv_row<TB>(M, slice, lane, VecF4{p}, y, xi);
        if (row >= 0) {
            q[3 * row] = y[0];
            q[3 * row + 1] = y[1];
            q[3 * row + 2] = y[2];
            pq = xi[0] * y[0] + xi[1] * y[1] + xi[2] * y[2];
        }
    }
    double v[1] = {pq};
    block_partials<1>(v, partials);
}

// alpha = rz / p.q; a non-positive or non-finite p.q ends the sweep.
__global__ void __launch_bounds__(1024) k_fin_alpha(const double *partials, int n, PcgState *st) {
    if (st->done) return;
    double tot[1];
    finalize_sum<1>(partials, n, tot);
    if (threadIdx.x == 0) {
        const double a = st->rz / tot[0];
        st->pq = tot[0];
        st->alpha = a;
        if (!(tot[0] > 0.0) || !isfinite(a)) {
            st->flags |= isfinite(tot[0]) ? 1 : 2;
            st->done = 1;
        }
    }
}

// x += alpha p, r -= alpha q; partials of r.z (z = D^-1 r) and r.r.
// Flat indexing over the 3 nv components: each thread handles UPD_PER
// components spaced by the block size, so every load instruction of a
// wavefront covers consecutive 8-byte elements.
constexpr int UPD_PER = 4;
__global__ void __launch_bounds__(256) k_pcg_update(int n3, double *x, double *r, const float *pf,
                                                    const double *q, const float *dinv, const PcgState *st,
                                                    double *partials) {
    if (st->done) return;
    const double alpha = st->alpha;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int base = b * (256 * UPD_PER) + threadIdx.x;
    double rz = 0.0, rr = 0.0;
#pragma unroll
    for (int u = 0; u < UPD_PER; ++u) {
        const int k = base + u * 256;
        if (k < n3) {
            const int i = k / 3;
            const double pk = pf[4 * i + (k - 3 * i)];
            x[k] += alpha * pk;
            const double rk = r[k] - alpha * q[k];
            r[k] = rk;
            rz += rk * rk * (double)dinv[k];
            rr += rk * rk;
        }
    }
    double v[2] = {rz, rr};
    block_partials<2>(v, partials);
}

// beta = rz_new / rz; convergence test ||r||^2 <= thresh; iteration count.
__global__ void __launch_bounds__(1024) k_fin_beta(const double *partials, int n, PcgState *st) {
    if (st->done) return;
    double tot[2];
    finalize_sum<2>(partials, n, tot);
    if (threadIdx.x == 0) {
        st->beta = tot[0] / st->rz;
        st->rz = tot[0];
        st->rr = tot[1];
        st->iters += 1;
        if (!isfinite(tot[1]) || !isfinite(tot[0])) {
            st->flags |= 2;
            st->done = 1;
        } else if (tot[1] <= st->thresh || st->iters >= st->maxit) {
            st->done = 1;
        }
    }
}

// p = D^-1 r + beta p
__global__ void __launch_bounds__(256) k_pcg_dir(int nv, const double *r, float4 *p, const float *dinv,
                                                 const PcgState *st) {
    if (st->done) return;
    const double beta = st->beta;
    const int i = row_of_thread();
    if (i >= nv) return;
    const float4 pv = p[i];
    float4 o;
    o.x = (float)(r[3 * i] * (double)dinv[3 * i] + beta * pv.x);
    o.y = (float)(r[3 * i + 1] * (double)dinv[3 * i + 1] + beta * pv.y);
    o.z = (float)(r[3 * i + 2] * (double)dinv[3 * i + 2] + beta * pv.z);
    o.w = 0.0f;
    p[i] = o;
}

// Zero start: x = 0, r = b, p = D^-1 r; partials of r.z and ||b||^2.
__global__ void __launch_bounds__(256) k_pcg_start_zero(int nv, const double *b, double *x, double *r,
                                                        float4 *p, const float *dinv, double *partials) {
    const int i = row_of_thread();
    double rz = 0.0, rr = 0.0;
    if (i < nv) {
        float4 o;
        float *op = &o.x;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double ra = b[3 * i + a];
            x[3 * i + a] = 0.0;
            r[3 * i + a] = ra;
            const double z = ra * (double)dinv[3 * i + a];
            op[a] = (float)z;
            rz += ra * z;
            rr += ra * ra;
        }
        o.w = 0.0f;
        p[i] = o;
    }
    double v[3] = {rz, rr, rr};
    block_partials<3>(v, partials);
}

// Residual t = b - A x for FP64 x.  MODE 0 (sweep start): r = t, p = D^-1 r;
// partials of r.z, ||r||^2, ||b||^2.  MODE 1 (check): partials of ||t||^2,
// ||b||^2 only.
template <typename TB, int MODE>
__global__ void __launch_bounds__(256) k_residual(SpmvArgs M, const double *b, const double *x, double *r,
                                                  float4 *p, const float *dinv, double *partials) {
    const int slice = slice_of_thread(M.nslices);
    const int lane = lane_id();
    double rz = 0.0, rr = 0.0, bb = 0.0;
    if (slice < M.nslices) {
        double y[3], xi[3];
        const int row = spmv_row<TB>(M, slice, lane, VecD3{x}, y, xi);
        if (row >= 0) {
            float4 o;
            float *op = &o.x;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double ba = b[3 * row + a];
                const double ta = ba - y[a];
                rr += ta * ta;
                bb += ba * ba;
                if (MODE == 0) {
                    r[3 * row + a] = ta;
                    const double z = ta * (double)dinv[3 * row + a];
                    op[a] = (float)z;
                    rz += ta * z;
                }
            }
            if (MODE == 0) {
                o.w = 0.0f;
                p[row] = o;
            }
        }
    }
    double v[3] = {rz, rr, bb};
    block_partials<3>(v, partials);
}

// Sweep start: rz, ||r_0||^2, ||b||^2 -> state (threshold, early exit).
__global__ void __launch_bounds__(1024) k_fin_start(const double *partials, int n, PcgState *st) {
    double tot[3];
    finalize_sum<3>(partials, n, tot);
    if (threadIdx.x == 0) {
        st->rz = tot[0];
        st->rz0 = tot[0];
        st->rr = tot[1];
        st->bb = tot[2];
        st->rr0 = tot[1];
        st->thresh = fmax(st->tol2 * tot[2], st->rho2 * tot[1]);
        if (!isfinite(tot[1]) || !isfinite(tot[2])) {
            st->flags |= 2;
            st->done = 1;
        } else if (tot[1] <= st->tol2 * tot[2] || tot[2] == 0.0) {
            st->done = 1;
        }
    }
}

// Residual check: ||t||^2, ||b||^2 -> out2.
__global__ void __launch_bounds__(1024) k_fin_check(const double *partials, int n, double *out2) {
    double tot[3];
    finalize_sum<3>(partials, n, tot);
    if (threadIdx.x == 0) {
        out2[0] = tot[1];
        out2[1] = tot[2];
    }
}

// y = A x (FP64 in and out).
template <typename TB>
__global__ void __launch_bounds__(256) k_spmv_apply(SpmvArgs M, const double *x, double *yout) {
    const int slice = slice_of_thread(M.nslices);
    if (slice >= M.nslices) return;
    double y[3], xi[3];
    const int row = spmv_row<TB>(M, slice, lane_id(), VecD3{x}, y, xi);
    if (row >= 0) {
        yout[3 * row] = y[0];
        yout[3 * row + 1] = y[1];
        yout[3 * row + 2] = y[2];
    }
}

__global__ void k_copy_d(int64_t n, const double *src, double *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// v += dv, x += h v; pinned vertices keep x and get v = 0.
__global__ void k_update(int nv, const double *dv, double *x, double *v, const uint8_t *pinned, double h) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    if (pinned[i]) {
        v[3 * i] = v[3 * i + 1] = v[3 * i + 2] = 0.0;
        return;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double nvv = v[3 * i + a] + dv[3 * i + a];
        v[3 * i + a] = nvv;
        x[3 * i + a] += h * nvv;
    }
}

// ---------------------------------------------------------------- host side
// hi = false: the solver copy (ctx->dtype); hi = true: the FP64 blocks.
static SpmvArgs spmv_args(Ctx *ctx, bool hi) {
    SpmvArgs M;
    M.nv = ctx->nv;
    M.nslices = ctx->nslices;
    M.rowptr = ctx->rowptr;
    M.slot_cnt = ctx->slot_cnt;
    M.lane_row = ctx->lane_row;
    M.jcol = ctx->jcol;
    M.jval = (hi && ctx->hi_valid) ? (const void *)ctx->jval_hi : ctx->jval;
    M.mass = ctx->mass;
    return M;
}

static inline int pad8(int n) { return ((n + 7) / 8) * 8; }

struct Grids {
    int slice_blocks;  // 4 slices per 256-thread block
    int row_blocks;    // 256 rows per block
    int upd_blocks;    // 256 * UPD_PER components per block
};

static Grids grids(Ctx *ctx) {
    Grids g;
    g.slice_blocks = pad8((ctx->nslices + 3) / 4);
    g.row_blocks = pad8((ctx->nv + 255) / 256);
    g.upd_blocks = pad8((3 * ctx->nv + 256 * UPD_PER - 1) / (256 * UPD_PER));
    return g;
}

// One CG iteration.  With `ev` (graph capture) the three main kernels are
// bracketed by the given event pairs instead of the sampled profiler.
template <typename TB>
static void launch_iter(Ctx *ctx, const SpmvArgs &M, const Grids &g, hipStream_t s, hipEvent_t *ev = nullptr) {
    if (ev) {
        (void)hipEventRecord(ev[0], s);
        hipLaunchKernelGGL(k_pcg_spmv<TB>, dim3(g.slice_blocks), dim3(256), 0, s, M, ctx->p, ctx->q, ctx->st,
                           ctx->partials);
        (void)hipEventRecord(ev[1], s);
        hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(1024), 0, s, ctx->partials, g.slice_blocks, ctx->st);
        (void)hipEventRecord(ev[2], s);
        hipLaunchKernelGGL(k_pcg_update, dim3(g.upd_blocks), dim3(256), 0, s, 3 * ctx->nv, ctx->x, ctx->r,
                           (const float *)ctx->p, ctx->q, ctx->dinv, ctx->st, ctx->partials);
        (void)hipEventRecord(ev[3], s);
        hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(1024), 0, s, ctx->partials, g.upd_blocks, ctx->st);
        (void)hipEventRecord(ev[4], s);
        hipLaunchKernelGGL(k_pcg_dir, dim3(g.row_blocks), dim3(256), 0, s, ctx->nv, ctx->r, ctx->p, ctx->dinv,
                           ctx->st);
        (void)hipEventRecord(ev[5], s);
        return;
    }
    int slot = ctx->prof.begin(PK_SPMV, s);
    hipLaunchKernelGGL(k_pcg_spmv<TB>, dim3(g.slice_blocks), dim3(256), 0, s, M, ctx->p, ctx->q, ctx->st,
                       ctx->partials);
    ctx->prof.end(slot, s);
    hipLaunchKernelGGL(k_fin_alpha, dim3(1), dim3(1024), 0, s, ctx->partials, g.slice_blocks, ctx->st);
    slot = ctx->prof.begin(PK_UPDATE, s);
    hipLaunchKernelGGL(k_pcg_update, dim3(g.upd_blocks), dim3(256), 0, s, 3 * ctx->nv, ctx->x, ctx->r,
                       (const float *)ctx->p, ctx->q, ctx->dinv, ctx->st, ctx->partials);
    ctx->prof.end(slot, s);
    hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(1024), 0, s, ctx->partials, g.upd_blocks, ctx->st);
    slot = ctx->prof.begin(PK_DIR, s);
    hipLaunchKernelGGL(k_pcg_dir, dim3(g.row_blocks), dim3(256), 0, s, ctx->nv, ctx->r, ctx->p, ctx->dinv,
                       ctx->st);
    ctx->prof.end(slot, s);
}

// Residuals always use the FP64 blocks.  mode 0 starts a sweep from x,
// mode 1 writes ||b - A x||^2 and ||b||^2 to out2.
static void launch_residual(Ctx *ctx, const SpmvArgs &M, const Grids &g, const double *b, const double *x,
                            int mode, double *out2, hipStream_t s) {
    using TB = double;
    if (mode == 0) {
        hipLaunchKernelGGL((k_residual<TB, 0>), dim3(g.slice_blocks), dim3(256), 0, s, M, b, x, ctx->r, ctx->p,
                           ctx->dinv, ctx->partials);
        hipLaunchKernelGGL(k_fin_start, dim3(1), dim3(1024), 0, s, ctx->partials, g.slice_blocks, ctx->st);
    } else {
        hipLaunchKernelGGL((k_residual<TB, 1>), dim3(g.slice_blocks), dim3(256), 0, s, M, b, x, ctx->r, ctx->p,
                           ctx->dinv, ctx->partials);
        hipLaunchKernelGGL(k_fin_check, dim3(1), dim3(1024), 0, s, ctx->partials, g.slice_blocks, out2);
    }
}

// Capture `chunk` iterations on the context's capture stream.
template <typename TB>
static pc_status capture_chunk(Ctx *ctx, const SpmvArgs &M, const Grids &g, int chunk, int variant) {
    if (!ctx->cap_stream) PC_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    if (!ctx->gev[variant][0])
        for (int k = 0; k < 6; ++k) PC_HIP(hipEventCreate(&ctx->gev[variant][k]));
    if (ctx->gexec[variant]) {
        (void)hipGraphExecDestroy(ctx->gexec[variant]);
        ctx->gexec[variant] = nullptr;
    }
    hipStream_t cs = ctx->cap_stream;
    PC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int c = 0; c < chunk; ++c) launch_iter<TB>(ctx, M, g, cs, c == 0 ? ctx->gev[variant] : nullptr);
    hipGraph_t graph = nullptr;
    PC_HIP(hipStreamEndCapture(cs, &graph));
    hipError_t e = hipGraphInstantiate(&ctx->gexec[variant], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        ctx->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
        ctx->gexec[variant] = nullptr;
        return PC_ERR_HIP;
    }
    ctx->gkey[variant] = M.jval;
    ctx->gkey_dtype[variant] = (int)sizeof(TB);
    ctx->gkey_chunk[variant] = chunk;
    return PC_OK;
}

// Add the graph's event-pair timings (first iteration of the chunk) to the
// profiler statistics; call after the stream has been synchronised.
static void harvest_graph_events(Ctx *ctx, int variant) {
    if (ctx->prof.every <= 0) return;
    const int kinds[3] = {PK_SPMV, PK_UPDATE, PK_DIR};
    for (int q = 0; q < 3; ++q) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ctx->gev[variant][2 * q], ctx->gev[variant][2 * q + 1]) != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        Prof &P = ctx->prof;
        const int k = kinds[q];
        if (P.count[k] == 0 || ms < P.min_ms[k]) P.min_ms[k] = ms;
        if (P.count[k] == 0 || ms > P.max_ms[k]) P.max_ms[k] = ms;
        P.sum_ms[k] += ms;
        P.count[k] += 1;
    }
}

pc_status spmv_run(Ctx *ctx, const double *xin, double *y, bool solver, hipStream_t s) {
    if (!ctx->assembled) {
        ctx->err = "cloth_spmv: nothing assembled";
        return PC_ERR_ARG;
    }
    const SpmvArgs M = spmv_args(ctx, !solver);
    const Grids g = grids(ctx);
    switch (solver ? ctx->dtype : PC_F64) {
        case PC_F64: hipLaunchKernelGGL(k_spmv_apply<double>, dim3(g.slice_blocks), dim3(256), 0, s, M, xin, y); break;
        case PC_F32: hipLaunchKernelGGL(k_spmv_apply<float>, dim3(g.slice_blocks), dim3(256), 0, s, M, xin, y); break;
        case PC_BF16: hipLaunchKernelGGL(k_spmv_apply<bf16_t>, dim3(g.slice_blocks), dim3(256), 0, s, M, xin, y); break;
    }
    PC_HIP(hipGetLastError());
    return PC_OK;
}

pc_status read_status(Ctx *ctx, hipStream_t s, int *bits) {
    PC_HIP(hipMemcpyAsync(ctx->status_host, ctx->status, sizeof(int), hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
    *bits = *ctx->status_host;
    return PC_OK;
}

// CG from the start in ctx->x (warm) or from zero, until the recursive
// residual meets the tolerance; then the residual is recomputed from x with
// FP64 accumulation, and if that true residual misses the tolerance (rounding
// drift of the recurrence) CG restarts from x with the true residual, up to
// max_sweeps times.
template <typename TB>
static pc_status pcg_typed(Ctx *ctx, const double *b, double *dv, const pc_solve_opts *o, pc_solve_info *info,
                           hipStream_t s) {
    const SpmvArgs M = spmv_args(ctx, false);
    const SpmvArgs Mhi = spmv_args(ctx, true);
    const Grids g = grids(ctx);
    const int nv = ctx->nv;
    const double tol = o ? o->tol : 1e-6;
    const int maxit = (o && o->maxit > 0) ? o->maxit : 20000;
    int warm = o ? o->warm : 0;
    const int check = (o && o->check_every > 0) ? o->check_every : 0;
    const bool lowp = ctx->dtype == PC_BF16;
    const double rho = (o && o->inner_rho > 0.0) ? o->inner_rho : (lowp ? 1e-2 : 0.0);
    const int max_sweeps = (o && o->max_sweeps > 0) ? o->max_sweeps : (lowp ? 40 : 4);
    const int64_t n3 = 3 * (int64_t)nv;

    if (warm)
        hipLaunchKernelGGL(k_copy_d, dim3((n3 + 255) / 256), dim3(256), 0, s, n3, dv, ctx->x);
    int total_iters = 0, sweeps = 0, fallback = 0;
    bool inner_hi = false;
    PcgState h{};
    double res2[2] = {0.0, 0.0};
    double *out2 = ctx->res2;
    for (;;) {
        hipLaunchKernelGGL(k_state_init, dim3(1), dim3(64), 0, s, ctx->st, tol, rho, maxit - total_iters);
        if (warm)
            launch_residual(ctx, Mhi, g, b, ctx->x, 0, nullptr, s);
        else {
            hipLaunchKernelGGL(k_pcg_start_zero, dim3(g.row_blocks), dim3(256), 0, s, nv, b, ctx->x, ctx->r,
                               ctx->p, ctx->dinv, ctx->partials);
            hipLaunchKernelGGL(k_fin_start, dim3(1), dim3(1024), 0, s, ctx->partials, g.row_blocks, ctx->st);
        }
        PC_HIP(hipGetLastError());
        PC_HIP(hipMemcpyAsync(ctx->st_host, ctx->st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
        PC_HIP(hipStreamSynchronize(s));
        h = *ctx->st_host;
        ++sweeps;
        const int variant = inner_hi ? 1 : 0;
        const bool graph = ctx->graph_chunk > 0;
        if (graph) {
            const SpmvArgs &Mv = inner_hi ? Mhi : M;
            const int want_size = inner_hi ? (int)sizeof(double) : (int)sizeof(TB);
            if (!ctx->gexec[variant] || ctx->gkey[variant] != Mv.jval || ctx->gkey_dtype[variant] != want_size ||
                ctx->gkey_chunk[variant] != ctx->graph_chunk) {
                pc_status cst = inner_hi ? capture_chunk<double>(ctx, Mhi, g, ctx->graph_chunk, variant)
                                         : capture_chunk<TB>(ctx, M, g, ctx->graph_chunk, variant);
                if (cst) return cst;
            }
        }
        while (!h.done && h.iters < h.maxit) {
            if (graph) {
                PC_HIP(hipGraphLaunch(ctx->gexec[variant], s));
            } else {
                int chunk = check > 0 ? check : std::min(256, std::max(16, (total_iters + h.iters) / 4));
                chunk = std::min(chunk, h.maxit - h.iters);
                for (int c = 0; c < chunk; ++c) {
                    if (inner_hi)
                        launch_iter<double>(ctx, Mhi, g, s);
                    else
                        launch_iter<TB>(ctx, M, g, s);
                }
            }
            PC_HIP(hipGetLastError());
            PC_HIP(hipMemcpyAsync(ctx->st_host, ctx->st, sizeof(PcgState), hipMemcpyDeviceToHost, s));
            PC_HIP(hipStreamSynchronize(s));
            if (graph)
                harvest_graph_events(ctx, variant);
            else
                ctx->prof.harvest();
            h = *ctx->st_host;
        }
        total_iters += h.iters;
        // true residual of the current iterate
        launch_residual(ctx, Mhi, g, b, ctx->x, 1, out2, s);
        PC_HIP(hipGetLastError());
        PC_HIP(hipMemcpyAsync(res2, out2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        PC_HIP(hipStreamSynchronize(s));
        const bool true_ok = res2[0] <= tol * tol * res2[1];
        if ((h.flags & 1) && !inner_hi && ctx->hi_valid && !true_ok) {
            // rounding of the stored blocks made the inner operator lose
            // definiteness: continue the sweeps on the FP64 blocks
            inner_hi = true;
            fallback = 1;
            h.flags = 0;
            warm = 1;
            continue;
        }
        if (h.flags || true_ok || res2[1] == 0.0 || total_iters >= maxit || sweeps >= max_sweeps) break;
        warm = 1;
    }
    hipLaunchKernelGGL(k_copy_d, dim3((n3 + 255) / 256), dim3(256), 0, s, n3, ctx->x, dv);
    const double bnorm = sqrt(res2[1]);
    if (res2[1] == 0.0 && !(h.flags & 2)) {  // b = 0: the solution is 0 whatever the start
        PC_HIP(hipMemsetAsync(dv, 0, sizeof(double) * (size_t)n3, s));
        res2[0] = 0.0;
    }
    PC_HIP(hipStreamSynchronize(s));
    const double rel_true = bnorm > 0 ? sqrt(res2[0]) / bnorm : sqrt(res2[0]);
    if (info) {
        info->iters = total_iters;
        info->sweeps = sweeps;
        info->bnorm = bnorm;
        info->rel_res_recursive = bnorm > 0 ? sqrt(h.rr) / bnorm : 0.0;
        info->rel_res_true = rel_true;
        info->fallback = fallback;
    }
    if (h.flags & 2) {
        ctx->err = "non-finite value in the CG recurrence";
        return PC_ERR_NONFINITE;
    }
    if (h.flags & 1) {
        ctx->err = "CG breakdown: p.Ap <= 0 (matrix not positive definite)";
        return PC_ERR_NOT_CONVERGED;
    }
    if (!(rel_true <= tol) && bnorm > 0) {
        ctx->err = "CG did not reach the tolerance within maxit iterations";
        return PC_ERR_NOT_CONVERGED;
    }
    return PC_OK;
}

pc_status pcg_run(Ctx *ctx, const double *b, double *dv, const pc_solve_opts *o, pc_solve_info *info,
                  hipStream_t s) {
    if (!ctx->assembled) {
        ctx->err = "cloth_pcg_solve: nothing assembled";
        return PC_ERR_ARG;
    }
    switch (ctx->dtype) {
        case PC_F64: return pcg_typed<double>(ctx, b, dv, o, info, s);
        case PC_F32: return pcg_typed<float>(ctx, b, dv, o, info, s);
        case PC_BF16: return pcg_typed<bf16_t>(ctx, b, dv, o, info, s);
    }
    return PC_ERR_ARG;
}

pc_status update_run(Ctx *ctx, const double *dv, double *x, double *v, hipStream_t s) {
    hipLaunchKernelGGL(k_update, dim3((ctx->nv + 255) / 256), dim3(256), 0, s, ctx->nv, dv, x, v, ctx->pinned,
                       ctx->prm.h);
    PC_HIP(hipGetLastError());
    return PC_OK;
}

}  // namespace pc
