// Preconditioned CG on the block SpMV (paper Sec. 2.5: the linear system of
// Eq. 3 is solved by PCG each step; Sec. 3.1: SpMV is the dominant operator,
// vector operations are element-wise): Jacobi or block-Jacobi
// preconditioning, the textbook recurrences or the single-reduction form,
// FP64 refinement sweeps around a low-precision inner solve.  The SpMV kernel
// itself is in pc_spmv.h.
//
// Solver layout: rows are grouped in slices of up to 64 (one wavefront),
// never across instances; inside a slice rows are ordered by decreasing
// length, and block k of every row with more than k blocks is stored
// contiguously (column index plane, then 9 value planes), so each load
// instruction of the wavefront reads consecutive addresses and no padding is
// stored.
//
// Several independent cloths (instances) can share one context: every kernel
// works on a schedule of work items that never straddle instances, and each
// instance has its own CG scalars, convergence flag and refinement sweeps,
// so all instances advance in the same launches.
//
// The operator is applied in difference form
//   y_i = m_i x_i + D_i x_i + sum_{j != i} A_ij (x_j - x_i),
// where the diagonal slot stores the remainder D_i, so that rounding of the
// stored (FP32/BF16) blocks leaves the mass term and the exact null space of
// the stiffness intact.  Arithmetic is FP64, except the BF16 SpMV's row sums
// (FP32, see pc_spmv.h) and the FP32 inner vectors of BF16 sweeps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "pc_mlp.h"
#include "pc_spmv.h"

namespace pc {

// Threads per block of the vector kernels (one block per vector work item;
// the single-reduction vector kernel stages VT rows of r at a time in LDS).
constexpr int VT = 1024;

// Preconditioner z = P^-1 r: kind 0 Jacobi (dinv, 3 per row), kind 1 block
// Jacobi (binv, the inverse diagonal block, 6 per row: xx, xy, xz, yy, yz,
// zz).  z holds the block-Jacobi z of the current residual (FP32).
struct PreArgs {
    int kind;
    const float *dinv;
    const float *binv;
    float *z;   // packed, 3 per row (st3 / ld3)
};

__device__ __forceinline__ void precond3(const PreArgs &P, int i, double r0, double r1, double r2, double z[3]) {
    if (P.kind == 0) {
        z[0] = r0 * (double)P.dinv[3 * i];
        z[1] = r1 * (double)P.dinv[3 * i + 1];
        z[2] = r2 * (double)P.dinv[3 * i + 2];
    } else {
        const float2 *b = (const float2 *)(P.binv + 6 * (int64_t)i);
        const float2 b01 = b[0], b23 = b[1], b45 = b[2];
        const double xx = b01.x, xy = b01.y, xz = b23.x, yy = b23.y, yz = b45.x, zz = b45.y;
        z[0] = xx * r0 + xy * r1 + xz * r2;
        z[1] = xy * r0 + yy * r1 + yz * r2;
        z[2] = xz * r0 + yz * r1 + zz * r2;
    }
}

// Sum of partials[q][i0..i1) in a fixed order, valid in every thread of the
// block (up to 1024 threads).
template <int NV>
__device__ __forceinline__ void instance_sum(const double *partials, int nitems, int i0, int i1, double (&tot)[NV]) {
    __shared__ double sh[NV][16];
    const int lane = lane_id(), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    double loc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) loc[q] = 0.0;
    for (int b = i0 + threadIdx.x; b < i1; b += blockDim.x)
#pragma unroll
        for (int q = 0; q < NV; ++q) loc[q] += partials[(size_t)q * nitems + b];
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
// Reset the state of every instance (restart == nullptr) or of the flagged ones.
__global__ void k_state_init(int ninst, PcgState *st, const uint8_t *restart, double tol, double rho,
                             const int *maxit) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst || (restart && !restart[i])) return;
    PcgState &S = st[i];
    S.rzp[0] = S.rzp[1] = S.alpha = S.rr = S.bb = 0.0;
    S.tol2 = tol * tol;
    S.rho2 = rho * rho;
    S.thresh = 0.0;
    S.rr0 = 0.0;
    S.rz0 = 0.0;
    S.beta = S.gprev = S.aprev = 0.0;
    S.kc = 0;
    S.live[0] = S.live[1] = 0;
    S.iters = 0;
    S.maxit = maxit[i];
    S.done = 0;
    S.flags = 0;
}

// Column window of every SpMV work item: the smallest and largest block
// column of its rows (block-CSR columns are ascending, so the first and last
// of each row suffice).  One block per item.
__global__ void __launch_bounds__(256) k_item_windows(Sched S, const int *slice_row0, const int *rowptr,
                                                      const int *colidx, int2 *win) {
    __shared__ int sh[2][4];
    const int it = blockIdx.x;
    if (it >= S.n_sitems) return;
    const int4 I = S.sitem[it];
    const int r0 = slice_row0[I.y], r1 = slice_row0[I.y + I.z];
    int lo = 0x7fffffff, hi = -1;
    for (int i = r0 + (int)threadIdx.x; i < r1; i += blockDim.x) {
        lo = min(lo, colidx[rowptr[i]]);
        hi = max(hi, colidx[rowptr[i + 1] - 1]);
    }
    for (int m = 32; m >= 1; m >>= 1) {
        lo = min(lo, __shfl_xor(lo, m, WAVE));
        hi = max(hi, __shfl_xor(hi, m, WAVE));
    }
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        sh[0][w] = lo;
        sh[1][w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)blockDim.x / WAVE; ++k) {
            lo = min(lo, sh[0][k]);
            hi = max(hi, sh[1][k]);
        }
        win[it] = make_int2(lo, hi);
    }
}

// Rows i0 + t + u VT (u < U) of an update item, as thread t sees them: the
// row's three components of r and q and its preconditioner entries.
template <typename TV>
struct UpdRows {
    static constexpr int U = 1;   // rows per thread in flight (2 needs more than 64 VGPRs)
    TV r[U][3], q[U][3];
    float d[U][3];
    float2 b[U][3];

    __device__ __forceinline__ void load(int i0, int i1, const TV *r_, const TV *q_, const PreArgs &P) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + (int)threadIdx.x + u * VT;
            if (i < i1) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    r[u][c] = r_[3 * i + c];
                    q[u][c] = q_[3 * i + c];
                }
                if (P.kind == 0) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) d[u][c] = P.dinv[3 * i + c];
                } else {
                    const float2 *bb = (const float2 *)(P.binv + 6 * (int64_t)i);
                    b[u][0] = bb[0]; b[u][1] = bb[1]; b[u][2] = bb[2];
                }
            }
        }
    }
};

// alpha, then r -= alpha q over the item's rows; partials of r.z
// (z = P^-1 r) and r.r with r as stored; block Jacobi stores z.  x += alpha p
// is left to the direction kernel, which reads p anyway.  TV: FP64 vectors,
// or FP32 for the correction, residual and product inside a refinement
// sweep.  One thread per row (all of a row's operands are then in one thread,
// so neither Jacobi form needs LDS or a barrier); the first rows' operands
// are loaded before alpha is formed, so that their latency overlaps the read
// of the SpMV's partials.  alpha = rz / p.q comes from the SpMV's partials
// (every block sums its instance's in the same order, so all blocks agree bit
// for bit); a non-positive or non-finite p.q ends the sweep (the first block
// records it), otherwise the first block hands alpha to the direction kernel.
template <typename TV>
__global__ void __launch_bounds__(VT) k_pcg_update(Sched S, int par, TV *r, const TV *q, PreArgs P, PcgState *st,
                                                    const double *part_s, double *part_u) {
    const int it = item_of_block(S.n_vitems);
    if (it < 0) return;
    const int4 I = S.vitem[it];
    if (st[I.x].done) return;
    const int t = threadIdx.x;
    constexpr int G = UpdRows<TV>::U * VT;
    UpdRows<TV> cur;
    cur.load(I.y, I.z, r, q, P);
    double pq[1];
    instance_sum<1>(part_s, S.n_sitems, S.inst_sitem0[I.x], S.inst_sitem0[I.x + 1], pq);
    const double alpha = st[I.x].rzp[par] / pq[0];
    const bool first = it == S.inst_vitem0[I.x] && t == 0;
    if (!(pq[0] > 0.0) || !isfinite(alpha)) {
        if (first) {
            st[I.x].flags |= isfinite(pq[0]) ? 1 : 2;
            st[I.x].done = 1;
        }
        return;
    }
    if (first) {
        st[I.x].alpha = alpha;
        st[I.x].live[par] = 1;
    }
    double rz = 0.0, rr = 0.0;
    for (int i0 = I.y; i0 < I.z; i0 += G) {
        if (i0 != I.y) cur.load(i0, I.z, r, q, P);
#pragma unroll
        for (int u = 0; u < UpdRows<TV>::U; ++u) {
            const int i = i0 + t + u * VT;
            if (i < I.z) {
                TV rv[3];
                double rk[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    rv[c] = (TV)((double)cur.r[u][c] - alpha * (double)cur.q[u][c]);
                    rk[c] = rv[c];
                    rr += rk[c] * rk[c];
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) r[3 * i + c] = rv[c];
                if (P.kind == 0) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) rz += rk[c] * rk[c] * (double)cur.d[u][c];
                } else {
                    const double xx = cur.b[u][0].x, xy = cur.b[u][0].y, xz = cur.b[u][1].x;
                    const double yy = cur.b[u][1].y, yz = cur.b[u][2].x, zz = cur.b[u][2].y;
                    const double z0 = xx * rk[0] + xy * rk[1] + xz * rk[2];
                    const double z1 = xy * rk[0] + yy * rk[1] + yz * rk[2];
                    const double z2 = xz * rk[0] + yz * rk[1] + zz * rk[2];
                    rz += rk[0] * z0 + rk[1] * z1 + rk[2] * z2;
                    st3(P.z, i, (float)z0, (float)z1, (float)z2);
                }
            }
        }
    }
    double v[2] = {rz, rr};
    block_partials<2>(v, part_u, it, S.n_vitems);
}

// x += alpha p with the update's alpha, then beta = rz_new / rz (every block
// from the update's partials, fixed order) and p = P^-1 r + beta p over the
// item's rows (Jacobi: from r and dinv; block Jacobi: from the z stored by
// the update).  The first block of each instance advances the instance
// state: rzp[1 - par] = rz_new, ||r||^2, the iteration count and the
// convergence test ||r||^2 <= thresh.  Blocks that see the instance
// converged skip the direction (it is not used again) but not x.  Whether
// the iteration is live comes from live[par], which only the update wrote;
// `done` may be set by this launch's first block while others still read it.
// One thread per row; the first row's operands are loaded before the
// partial sums are read.
template <typename TV>
struct DirRow {
    float4 p, z;   // z: block Jacobi's stored P^-1 r
    TV x[3];
    TV r[3];       // Jacobi: r and dinv
    float d[3];

    __device__ __forceinline__ void load(int i, const TV *x_, const TV *r_, const float *p_, const PreArgs &P) {
        p = ld3(p_, i);
#pragma unroll
        for (int c = 0; c < 3; ++c) x[c] = x_[3 * i + c];
        if (P.kind == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                r[c] = r_[3 * i + c];
                d[c] = P.dinv[3 * i + c];
            }
        } else {
            z = ld3(P.z, i);
        }
    }
};

template <typename TV>
__global__ void __launch_bounds__(VT) k_pcg_dir(Sched S, int par, TV *x, const TV *r, float *p, PreArgs P,
                                                 PcgState *st, const double *part_u) {
    const int it = item_of_block(S.n_vitems);
    if (it < 0) return;
    const int4 I = S.vitem[it];
    const bool first = it == S.inst_vitem0[I.x] && threadIdx.x == 0;
    if (first) st[I.x].live[1 - par] = 0;
    if (!st[I.x].live[par]) return;
    DirRow<TV> row;
    int i = I.y + (int)threadIdx.x;
    if (i < I.z) row.load(i, x, r, p, P);
    const double alpha = st[I.x].alpha;
    double tot[2];
    instance_sum<2>(part_u, S.n_vitems, S.inst_vitem0[I.x], S.inst_vitem0[I.x + 1], tot);
    const double beta = tot[0] / st[I.x].rzp[par];
    const bool bad = !isfinite(tot[1]) || !isfinite(tot[0]);
    const bool conv = tot[1] <= st[I.x].thresh;
    const bool new_dir = !(bad || conv);
    if (first) {
        PcgState &T = st[I.x];
        T.rzp[1 - par] = tot[0];
        T.rr = tot[1];
        T.iters += 1;
        if (new_dir) T.rzd = tot[0];
        if (bad) {
            T.flags |= 2;
            T.done = 1;
        } else if (conv || T.iters >= T.maxit) {
            T.done = 1;
        }
    }
    for (; i < I.z; i += VT) {
        if (i != I.y + (int)threadIdx.x) row.load(i, x, r, p, P);
        const float4 pv = row.p;
        x[3 * i] = (TV)((double)row.x[0] + alpha * (double)pv.x);
        x[3 * i + 1] = (TV)((double)row.x[1] + alpha * (double)pv.y);
        x[3 * i + 2] = (TV)((double)row.x[2] + alpha * (double)pv.z);
        if (new_dir) {
            double z[3];
            if (P.kind == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) z[c] = (double)row.r[c] * (double)row.d[c];
            } else {
                z[0] = row.z.x; z[1] = row.z.y; z[2] = row.z.z;
            }
            st3(p, i, (float)(z[0] + beta * pv.x), (float)(z[1] + beta * pv.y), (float)(z[2] + beta * pv.z));
        }
    }
}

// ---- single-reduction form (Chronopoulos and Gear, 1989; s = 1) ----
// Iteration k: w = A u_k (the SpMV above, with u_k in the direction buffer
// and partials of delta_k = u_k.w), then one block per instance sums
// delta_k and the vector kernel's partials of gamma_k = r_k.z_k and
// ||r_k||^2 (z = P^-1 r before rounding; at k = 0 the sweep start's values),
// tests convergence, and forms
//   beta_k = gamma_k / gamma_{k-1} (0 at k = 0),
//   alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1}),
// which equals gamma_k / p_k.A p_k in exact arithmetic; a non-positive
// denominator ends the sweep as a breakdown.
__global__ void __launch_bounds__(1024) k_fin_cgcg(Sched S, const double *partials, const double *part_u,
                                                  PcgState *st) {
    const int inst = blockIdx.x;
    if (inst >= S.ninst || st[inst].done) return;
    double d[1], gu[2];
    instance_sum<1>(partials, S.n_sitems, S.inst_sitem0[inst], S.inst_sitem0[inst + 1], d);
    instance_sum<2>(part_u, S.n_vitems, S.inst_vitem0[inst], S.inst_vitem0[inst + 1], gu);
    if (threadIdx.x != 0) return;
    PcgState &T = st[inst];
    double gamma;
    if (T.kc == 0) {
        gamma = T.rz0;
    } else {
        gamma = gu[0];
        T.rr = gu[1];
        if (!isfinite(gu[0]) || !isfinite(gu[1])) {
            T.flags |= 2;
            T.done = 1;
            return;
        }
        if (gu[1] <= T.thresh) {
            T.done = 1;
            return;
        }
    }
    if (T.iters >= T.maxit) {
        T.done = 1;
        return;
    }
    const double beta = T.kc == 0 ? 0.0 : gamma / T.gprev;
    const double den = T.kc == 0 ? d[0] : d[0] - beta * gamma / T.aprev;
    const double a = gamma / den;
    if (!(den > 0.0) || !isfinite(a)) {
        T.flags |= isfinite(den) ? 1 : 2;
        T.done = 1;
        return;
    }
    T.alpha = a;
    T.beta = beta;
    T.gprev = gamma;
    T.aprev = a;
    T.kc += 1;
    T.iters += 1;
}

// p = u + beta p, s = w + beta s (p = u, s = w in the first iteration of a
// sweep), x += alpha p, r -= alpha s over the item's rows with flat
// component indexing (consecutive threads touch consecutive 8-byte
// elements), each VT-row chunk of the new r staged in LDS; then one thread
// per row forms u = P^-1 r, stores it as packed FP32 for the next product and
// adds to the partials of r.u (with the stored, rounded u, the vector the
// product and the direction use) and ||r||^2.
__global__ void __launch_bounds__(VT) k_cgcg_vec(Sched S, double *x, double *r, float *u, const double *w,
                                                  double *pd, double *sv, PreArgs P, const PcgState *st,
                                                  double *part_u) {
    __shared__ double rs[3 * VT];
    const int it = item_of_block(S.n_vitems);
    if (it < 0) return;
    const int4 I = S.vitem[it];
    const PcgState &T = st[I.x];
    if (T.done) return;
    const double alpha = T.alpha, beta = T.beta;
    const bool first = T.kc == 1;
    double gz = 0.0, rr = 0.0;
    for (int r0 = I.y; r0 < I.z; r0 += VT) {
        const int nr = min(VT, I.z - r0);
        for (int k = threadIdx.x; k < 3 * nr; k += blockDim.x) {
            const int64_t kk = 3 * (int64_t)r0 + k;
            const double uk = u[kk];
            const double pk = first ? uk : uk + beta * pd[kk];
            const double sk = first ? w[kk] : w[kk] + beta * sv[kk];
            pd[kk] = pk;
            sv[kk] = sk;
            x[kk] += alpha * pk;
            const double rk = r[kk] - alpha * sk;
            r[kk] = rk;
            rs[k] = rk;
            rr += rk * rk;
        }
        __syncthreads();
        if ((int)threadIdx.x < nr) {
            const int t = threadIdx.x, i = r0 + t;
            const double a0 = rs[3 * t], a1 = rs[3 * t + 1], a2 = rs[3 * t + 2];
            double z[3];
            precond3(P, i, a0, a1, a2, z);
            const float4 zf = make_float4((float)z[0], (float)z[1], (float)z[2], 0.0f);
            gz += a0 * (double)zf.x + a1 * (double)zf.y + a2 * (double)zf.z;
            st3(u, i, zf.x, zf.y, zf.z);
        }
        __syncthreads();
    }
    double v[2] = {gz, rr};
    block_partials<2>(v, part_u, it, S.n_vitems);
}

// Zero start of the flagged instances (all when restart == nullptr):
// x = 0, r = b, p = P^-1 r (and the sweep's correction e = 0 when the inner
// vectors are FP32); partials of r.z, ||r||^2 and ||b||^2.
template <typename TV>
__global__ void __launch_bounds__(VT) k_pcg_start_zero(Sched S, const uint8_t *restart, const double *b, double *x,
                                                        TV *r, float *p, PreArgs P, double *partials, TV *e) {
    const int it = item_of_block(S.n_vitems);
    if (it < 0) return;
    const int4 I = S.vitem[it];
    if (restart && !restart[I.x]) return;
    double rz = 0.0, rr = 0.0;
    for (int i = I.y + threadIdx.x; i < I.z; i += blockDim.x) {
        const double r0 = b[3 * i], r1 = b[3 * i + 1], r2 = b[3 * i + 2];
        double z[3];
        precond3(P, i, r0, r1, r2, z);
        x[3 * i] = 0.0; x[3 * i + 1] = 0.0; x[3 * i + 2] = 0.0;
        r[3 * i] = (TV)r0; r[3 * i + 1] = (TV)r1; r[3 * i + 2] = (TV)r2;
        if (e) {
            e[3 * i] = TV(0); e[3 * i + 1] = TV(0); e[3 * i + 2] = TV(0);
        }
        rz += r0 * z[0] + r1 * z[1] + r2 * z[2];
        rr += r0 * r0 + r1 * r1 + r2 * r2;
        st3(p, i, (float)z[0], (float)z[1], (float)z[2]);
    }
    double v[3] = {rz, rr, rr};
    block_partials<3>(v, partials, it, S.n_vitems);
}

// Residual t = b - A x for FP64 x over the item's slices.  MODE 0 (sweep
// start of the flagged instances): r = t, p = P^-1 r, e = 0 (FP32 inner
// vectors); partials of r.z, ||r||^2, ||b||^2.  MODE 2 (sweep start that
// keeps the direction): the same, except that p is left alone and block
// Jacobi's z = P^-1 r is stored for k_pcg_redirect.  MODE 1 (check, all
// instances): partials of ||t||^2, ||b||^2.
template <typename TB, int MODE, typename TV>
__global__ void __launch_bounds__(1024) k_residual(SpmvArgs M, Sched S, const uint8_t *restart, const double *b,
                                                  const double *x, TV *r, float *p, PreArgs P,
                                                  double *partials, TV *e) {
    const int it = item_of_block(S.n_sitems);
    if (it < 0) return;
    const int4 I = S.sitem[it];
    if (MODE != 1 && restart && !restart[I.x]) return;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int lane = lane_id();
    double rz = 0.0, rr = 0.0, bb = 0.0;
    if (w < I.z) {
        double y[3], xi[3];
        const int row = spmv_row<TB>(M, I.y + w, lane, VecD3{x}, y, xi);
        if (row >= 0) {
            double t[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double ba = b[3 * row + a];
                t[a] = ba - y[a];
                rr += t[a] * t[a];
                bb += ba * ba;
            }
            if (MODE != 1) {
                double z[3];
                precond3(P, row, t[0], t[1], t[2], z);
                r[3 * row] = (TV)t[0]; r[3 * row + 1] = (TV)t[1]; r[3 * row + 2] = (TV)t[2];
                if (e) {
                    e[3 * row] = TV(0); e[3 * row + 1] = TV(0); e[3 * row + 2] = TV(0);
                }
                rz += t[0] * z[0] + t[1] * z[1] + t[2] * z[2];
                if (MODE == 0)
                    st3(p, row, (float)z[0], (float)z[1], (float)z[2]);
                else if (P.kind != 0)
                    st3(P.z, row, (float)z[0], (float)z[1], (float)z[2]);
            }
        }
    }
    double v[3] = {rz, rr, bb};
    block_partials<3>(v, partials, it, S.n_sitems);
}

// Sweep start that keeps the direction (residual replacement), after
// k_residual MODE 2: beta = r.z / rzd from the residual's partials (rzd:
// r.z of the residual the current direction was built from; beta = 0, a
// plain restart, when it is not positive), then p = z + beta p with z as the
// direction kernel forms it (Jacobi: the stored r times P^-1; block Jacobi:
// the stored z).  Every block sums its instance's partials in the same order.
template <typename TV>
__global__ void __launch_bounds__(VT) k_pcg_redirect(Sched S, const uint8_t *restart, const TV *r, float *p,
                                                      PreArgs P, const PcgState *st, const double *partials) {
    const int it = item_of_block(S.n_vitems);
    if (it < 0) return;
    const int4 I = S.vitem[it];
    if (restart && !restart[I.x]) return;
    double tot[3];
    instance_sum<3>(partials, S.n_sitems, S.inst_sitem0[I.x], S.inst_sitem0[I.x + 1], tot);
    const double rzd = st[I.x].rzd;
    const double q = tot[0] / rzd;
    const double beta = (rzd > 0.0 && isfinite(q) && q >= 0.0) ? q : 0.0;
    for (int i = I.y + (int)threadIdx.x; i < I.z; i += VT) {
        double z[3];
        if (P.kind == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) z[c] = (double)r[3 * i + c] * (double)P.dinv[3 * i + c];
        } else {
            const float4 zv = ld3(P.z, i);
            z[0] = zv.x; z[1] = zv.y; z[2] = zv.z;
        }
        const float4 pv = ld3(p, i);
        st3(p, i, (float)(z[0] + beta * pv.x), (float)(z[1] + beta * pv.y), (float)(z[2] + beta * pv.z));
    }
}

// Sweep start of the flagged instances: rz, ||r_0||^2, ||b||^2 -> state
// (threshold, early exit when the start already meets the tolerance).
__global__ void __launch_bounds__(256) k_fin_start(Sched S, int use_sitems, int par, const uint8_t *restart,
                                                   const double *partials, PcgState *st) {
    const int inst = blockIdx.x;
    if (inst >= S.ninst || (restart && !restart[inst])) return;
    double tot[3];
    if (use_sitems)
        instance_sum<3>(partials, S.n_sitems, S.inst_sitem0[inst], S.inst_sitem0[inst + 1], tot);
    else
        instance_sum<3>(partials, S.n_vitems, S.inst_vitem0[inst], S.inst_vitem0[inst + 1], tot);
    if (threadIdx.x == 0) {
        PcgState &T = st[inst];
        T.rzp[par] = tot[0];
        T.rz0 = tot[0];
        T.rzd = tot[0];
        T.rr = tot[1];
        T.bb = tot[2];
        T.rr0 = tot[1];
        T.live[0] = T.live[1] = 0;
        T.thresh = fmax(T.tol2 * tot[2], T.rho2 * tot[1]);
        if (!isfinite(tot[1]) || !isfinite(tot[2])) {
            T.flags |= 2;
            T.done = 1;
        } else if (tot[1] <= T.tol2 * tot[2] || tot[2] == 0.0) {
            T.done = 1;
        }
    }
}

// Residual check: ||t||^2, ||b||^2 of every instance -> out2[2 inst + {0,1}].
__global__ void __launch_bounds__(256) k_fin_check(Sched S, const double *partials, double *out2) {
    const int inst = blockIdx.x;
    if (inst >= S.ninst) return;
    double tot[3];
    instance_sum<3>(partials, S.n_sitems, S.inst_sitem0[inst], S.inst_sitem0[inst + 1], tot);
    if (threadIdx.x == 0) {
        out2[2 * inst] = tot[1];
        out2[2 * inst + 1] = tot[2];
    }
}

// y = A x (FP64 in and out).
template <typename TB>
__global__ void __launch_bounds__(1024) k_spmv_apply(SpmvArgs M, Sched S, const double *x, double *yout) {
    const int it = item_of_block(S.n_sitems);
    if (it < 0) return;
    const int4 I = S.sitem[it];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    if (w >= I.z) return;
    double y[3], xi[3];
    const int row = spmv_row<TB>(M, I.y + w, lane_id(), VecD3{x}, y, xi);
    if (row >= 0) {
        yout[3 * row] = y[0];
        yout[3 * row + 1] = y[1];
        yout[3 * row + 2] = y[2];
    }
}

// End of a refinement sweep with FP32 inner vectors: x += e, e = 0.
__global__ void k_fold(int64_t n, double *x, float *e) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) {
        x[k] += (double)e[k];
        e[k] = 0.0f;
    }
}

__global__ void k_copy_d(int64_t n, const double *src, double *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Zero the rows of the flagged instances (b = 0 result).
__global__ void k_zero_rows(Sched S, const uint8_t *flag, double *x) {
    const int it = item_of_block(S.n_vitems);
    if (it < 0) return;
    const int4 I = S.vitem[it];
    if (!flag[I.x]) return;
    for (int k = 3 * I.y + threadIdx.x; k < 3 * I.z; k += blockDim.x) x[k] = 0.0;
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
    M.slice_vbase = ctx->slice_vbase;
    M.slice_row0 = ctx->slice_row0;
    M.slot_cnt = ctx->slot_cnt;
    M.lane_row = ctx->lane_row;
    M.jcol = ctx->jcol;
    M.jdel = ctx->use_narrow ? ctx->jdel : nullptr;
    M.jval = (hi && ctx->hi_valid) ? (const void *)ctx->jval_hi : ctx->jval;
    M.mass = ctx->mass;
    M.vscale = ctx->f16_scale;
    return M;
}

static Sched sched_args(Ctx *ctx) {
    Sched S;
    S.n_sitems = ctx->n_sitems;
    S.n_vitems = ctx->n_vitems;
    S.ninst = ctx->ninst;
    S.sitem = ctx->sitem;
    S.vitem = ctx->vitem;
    S.inst_sitem0 = ctx->inst_sitem0;
    S.inst_vitem0 = ctx->inst_vitem0;
    return S;
}

static inline int pad8(int n) { return ((n + 7) / 8) * 8; }

static PreArgs pre_args(Ctx *ctx) {
    PreArgs P;
    P.kind = ctx->precond;
    P.dinv = ctx->dinv;
    P.binv = ctx->binv;
    P.z = ctx->zb;
    return P;
}

// Slices (up to 64 rows, never across instances) and work items from the
// instance row ranges and the current spb / rpb.
pc_status build_schedule(Ctx *ctx) {
    const int ninst = (int)ctx->inst_row0_h.size() - 1;
    std::vector<int> slice_row0, row_slice(ctx->nv);
    std::vector<int4> sitems, vitems;
    std::vector<int> isit(ninst + 1), ivit(ninst + 1), islc(ninst + 1);
    for (int i = 0; i < ninst; ++i) {
        const int r0 = ctx->inst_row0_h[i], r1 = ctx->inst_row0_h[i + 1];
        const int s0 = (int)slice_row0.size();
        islc[i] = s0;
        for (int r = r0; r < r1; r += WAVE) {
            for (int q = r; q < std::min(r + WAVE, r1); ++q) row_slice[q] = (int)slice_row0.size();
            slice_row0.push_back(r);
        }
        const int s1 = (int)slice_row0.size();
        isit[i] = (int)sitems.size();
        for (int sl = s0; sl < s1; sl += ctx->spb) sitems.push_back(int4{i, sl, std::min(ctx->spb, s1 - sl), 0});
        ivit[i] = (int)vitems.size();
        for (int r = r0; r < r1; r += ctx->rpb) vitems.push_back(int4{i, r, std::min(r + ctx->rpb, r1), 0});
    }
    slice_row0.push_back(ctx->nv);
    isit[ninst] = (int)sitems.size();
    ivit[ninst] = (int)vitems.size();
    const int nslices = (int)slice_row0.size() - 1;
    islc[ninst] = nslices;
    pc_status st;
    auto realloc = [&](void **p, size_t bytes) -> pc_status {
        if (*p) dev_free(ctx, *p);
        *p = nullptr;
        return dev_alloc(ctx, p, bytes);
    };
    if (nslices > ctx->slice_cap) {
        if ((st = realloc((void **)&ctx->lane_row, sizeof(int) * (size_t)nslices * WAVE))) return st;
        if ((st = realloc((void **)&ctx->slot_cnt, (size_t)nslices * WAVE))) return st;
        if ((st = realloc((void **)&ctx->slot_off, sizeof(int) * (size_t)nslices * WAVE))) return st;
        if ((st = realloc((void **)&ctx->slice_row0, sizeof(int) * (size_t)(nslices + 1)))) return st;
        if ((st = realloc((void **)&ctx->slice_psize, sizeof(int) * (size_t)nslices))) return st;
        if ((st = realloc((void **)&ctx->slice_vbase, sizeof(int) * (size_t)(nslices + 1)))) return st;
        ctx->slice_cap = nslices;
    }
    // stored blocks: the pattern's blocks plus at most 7 padding lanes in each
    // of the (at most 64) slots of every slice
    const int64_t vcap = ctx->cap + (int64_t)7 * WAVE * nslices;
    if (vcap >= ((int64_t)1 << 31) / 9) {
        ctx->err = "stored block capacity exceeds int32 indexing";
        return PC_ERR_CAPACITY;
    }
    ctx->vcap = vcap;
    if (vcap > ctx->jcol_blocks) {
        if ((st = realloc((void **)&ctx->jcol, sizeof(int) * (size_t)vcap))) return st;
        if ((st = realloc((void **)&ctx->jdel, sizeof(int16_t) * (size_t)vcap))) return st;
        ctx->jcol_blocks = vcap;
    }
    if ((st = realloc((void **)&ctx->sitem, sizeof(int4) * sitems.size()))) return st;
    if ((st = realloc((void **)&ctx->vitem, sizeof(int4) * vitems.size()))) return st;
    if ((st = realloc((void **)&ctx->inst_sitem0, sizeof(int) * (ninst + 1)))) return st;
    if ((st = realloc((void **)&ctx->inst_vitem0, sizeof(int) * (ninst + 1)))) return st;
    if ((st = realloc((void **)&ctx->inst_slice0, sizeof(int) * (ninst + 1)))) return st;
    const size_t nitems = std::max(sitems.size(), vitems.size()) + 16;
    if ((st = realloc((void **)&ctx->partials, sizeof(double) * 4 * nitems))) return st;
    if ((st = realloc((void **)&ctx->partials_u, sizeof(double) * 2 * nitems))) return st;
    if (ninst != ctx->ninst || !ctx->st) {
        if ((st = realloc((void **)&ctx->st, sizeof(PcgState) * ninst))) return st;
        if ((st = realloc((void **)&ctx->res2, sizeof(double) * 2 * ninst))) return st;
        if ((st = realloc((void **)&ctx->restart, (size_t)ninst))) return st;
        if ((st = realloc((void **)&ctx->maxit_d, sizeof(int) * ninst))) return st;
        if (ctx->st_host) (void)hipHostFree(ctx->st_host);
        if (ctx->restart_h) (void)hipHostFree(ctx->restart_h);
        ctx->st_host = nullptr;
        ctx->restart_h = nullptr;
        PC_HIP(hipHostMalloc((void **)&ctx->st_host, sizeof(PcgState) * ninst, hipHostMallocDefault));
        PC_HIP(hipHostMalloc((void **)&ctx->restart_h, (size_t)ninst, hipHostMallocDefault));
    }
    if (!ctx->row_slice && (st = dev_alloc(ctx, (void **)&ctx->row_slice, sizeof(int) * (size_t)ctx->nv))) return st;
    PC_HIP(hipMemcpy(ctx->slice_row0, slice_row0.data(), sizeof(int) * slice_row0.size(), hipMemcpyHostToDevice));
    PC_HIP(hipMemcpy(ctx->row_slice, row_slice.data(), sizeof(int) * row_slice.size(), hipMemcpyHostToDevice));
    PC_HIP(hipMemcpy(ctx->sitem, sitems.data(), sizeof(int4) * sitems.size(), hipMemcpyHostToDevice));
    PC_HIP(hipMemcpy(ctx->vitem, vitems.data(), sizeof(int4) * vitems.size(), hipMemcpyHostToDevice));
    PC_HIP(hipMemcpy(ctx->inst_sitem0, isit.data(), sizeof(int) * isit.size(), hipMemcpyHostToDevice));
    PC_HIP(hipMemcpy(ctx->inst_vitem0, ivit.data(), sizeof(int) * ivit.size(), hipMemcpyHostToDevice));
    PC_HIP(hipMemcpy(ctx->inst_slice0, islc.data(), sizeof(int) * islc.size(), hipMemcpyHostToDevice));
    ctx->nslices = nslices;
    ctx->ninst = ninst;
    ctx->n_sitems = (int)sitems.size();
    ctx->n_vitems = (int)vitems.size();
    ctx->inst_info.assign(ninst, pc_solve_info{});
    ctx->sched_version += 1;
    ctx->win_valid = false;
    ctx->assembled = false;  // the solver layout depends on the slices
    return PC_OK;
}

struct Grids {
    int sblocks, sthreads;  // SpMV items: spb wavefronts each
    int vblocks;            // vector items: VT threads each
};

static Grids grids(Ctx *ctx) {
    Grids g;
    g.sblocks = pad8(ctx->n_sitems);
    g.sthreads = WAVE * ctx->spb;
    g.vblocks = pad8(ctx->n_vitems);
    return g;
}

// Column windows of the SpMV items (after an assembly or a schedule change)
// and the LDS window capacity: the largest window up to PC_WIN_MAX rows;
// items with wider windows gather from global memory.  Synchronises.
#ifndef PC_WIN_MAX
#define PC_WIN_MAX 4096
#endif
static pc_status ensure_windows(Ctx *ctx, hipStream_t s) {
    if (ctx->win_valid) return PC_OK;
    if (ctx->win_items < ctx->n_sitems) {
        if (ctx->sitem_win) dev_free(ctx, ctx->sitem_win);
        ctx->sitem_win = nullptr;
        ctx->win_items = 0;
        pc_status st = dev_alloc(ctx, (void **)&ctx->sitem_win, sizeof(int2) * (size_t)ctx->n_sitems);
        if (st) return st;
        ctx->win_items = ctx->n_sitems;
    }
    const Sched S = sched_args(ctx);
    hipLaunchKernelGGL(k_item_windows, dim3(ctx->n_sitems), dim3(256), 0, s, S, ctx->slice_row0, ctx->rowptr,
                       ctx->colidx, ctx->sitem_win);
    PC_HIP(hipGetLastError());
    std::vector<int2> w(ctx->n_sitems);
    PC_HIP(hipMemcpyAsync(w.data(), ctx->sitem_win, sizeof(int2) * w.size(), hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
    int cap = 0;
    for (const int2 &v : w) {
        const int n = v.y - v.x + 1;
        if (n <= PC_WIN_MAX) cap = std::max(cap, n);
    }
    ctx->win_cap = ctx->use_win ? cap : 0;
    // 16-bit column offsets: every column of an item's slices lies in
    // [lo, hi], and the slices' first rows in [first row, first row + 64 spb)
    bool narrow = true;
    std::vector<int4> items(ctx->n_sitems);
    std::vector<int> row0(ctx->nslices + 1);
    PC_HIP(hipMemcpy(items.data(), ctx->sitem, sizeof(int4) * items.size(), hipMemcpyDeviceToHost));
    PC_HIP(hipMemcpy(row0.data(), ctx->slice_row0, sizeof(int) * row0.size(), hipMemcpyDeviceToHost));
    for (size_t k = 0; k < items.size() && narrow; ++k) {
        const int r_first = row0[items[k].y], r_last = row0[items[k].y + items[k].z - 1];
        narrow = (long long)w[k].y - r_first <= 32767 && (long long)w[k].x - r_last >= -32768;
    }
    ctx->narrow = narrow;
    ctx->win_valid = true;
    return PC_OK;
}

// SpMV of p into q (stored as TQ) with partials of p.q.
template <typename TB, typename TQ>
static void launch_spmv(Ctx *ctx, const SpmvArgs &M, const Sched &S, const Grids &g, hipStream_t s, TQ *q) {
    if (ctx->narrow && M.jdel)
        hipLaunchKernelGGL((k_pcg_spmv<TB, true, TQ>), dim3(g.sblocks), dim3(g.sthreads),
                           sizeof(float4) * (size_t)ctx->win_cap, s, M, S, ctx->p, q, ctx->st, ctx->partials,
                           ctx->sitem_win, ctx->win_cap);
    else
        hipLaunchKernelGGL((k_pcg_spmv<TB, false, TQ>), dim3(g.sblocks), dim3(g.sthreads),
                           sizeof(float4) * (size_t)ctx->win_cap, s, M, S, ctx->p, q, ctx->st, ctx->partials,
                           ctx->sitem_win, ctx->win_cap);
}

// One CG iteration of parity par (the parity selects the rz slot, see
// PcgState): SpMV with its partials; update (alpha, r, z); direction
// (x += alpha p, beta from the update partials, p, state advance).  TV: type
// of the iterate, residual
// and product (FP64, or FP32 inside a refinement sweep, where the iterate
// is the sweep's correction e).
template <typename TB, typename TV>
static void launch_iter_v(Ctx *ctx, const SpmvArgs &M, const Sched &S, const Grids &g, hipStream_t s, int par,
                          TV *x, TV *r, TV *q) {
    int slot = ctx->prof.begin(PK_SPMV, s);
    launch_spmv<TB, TV>(ctx, M, S, g, s, q);
    ctx->prof.end(slot, s);
    slot = ctx->prof.begin(PK_UPDATE, s);
    hipLaunchKernelGGL(k_pcg_update<TV>, dim3(g.vblocks), dim3(VT), 0, s, S, par, r, (const TV *)q, pre_args(ctx),
                       ctx->st, (const double *)ctx->partials, ctx->partials_u);
    ctx->prof.end(slot, s);
    slot = ctx->prof.begin(PK_DIR, s);
    hipLaunchKernelGGL(k_pcg_dir<TV>, dim3(g.vblocks), dim3(VT), 0, s, S, par, x, (const TV *)r, ctx->p,
                       pre_args(ctx), ctx->st, ctx->partials_u);
    ctx->prof.end(slot, s);
}

template <typename TB>
static void launch_iter(Ctx *ctx, const SpmvArgs &M, const Sched &S, const Grids &g, hipStream_t s, int par) {
    if (ctx->inner32)
        launch_iter_v<TB, float>(ctx, M, S, g, s, par, ctx->e32, ctx->r32, ctx->q32);
    else
        launch_iter_v<TB, double>(ctx, M, S, g, s, par, ctx->x, ctx->r, ctx->q);
}

// One iteration of the single-reduction form: SpMV of u with partials of
// u.w, the per-instance scalars, the fused vector update.
template <typename TB>
static void launch_iter_cgcg(Ctx *ctx, const SpmvArgs &M, const Sched &S, const Grids &g, hipStream_t s) {
    int slot = ctx->prof.begin(PK_SPMV, s);
    launch_spmv<TB, double>(ctx, M, S, g, s, ctx->q);
    ctx->prof.end(slot, s);
    hipLaunchKernelGGL(k_fin_cgcg, dim3(ctx->ninst), dim3(1024), 0, s, S, ctx->partials, ctx->partials_u, ctx->st);
    slot = ctx->prof.begin(PK_UPDATE, s);
    hipLaunchKernelGGL(k_cgcg_vec, dim3(g.vblocks), dim3(VT), 0, s, S, ctx->x, ctx->r, ctx->p, ctx->q, ctx->cg_pd,
                       ctx->cg_s, pre_args(ctx), ctx->st, ctx->partials_u);
    ctx->prof.end(slot, s);
}

template <typename TB>
static void launch_one(Ctx *ctx, const SpmvArgs &M, const Sched &S, const Grids &g, hipStream_t s, int par) {
    if (ctx->method == 1)
        launch_iter_cgcg<TB>(ctx, M, S, g, s);
    else
        launch_iter<TB>(ctx, M, S, g, s, par);
}

// Plain launches of n iterations continuing the context's parity.
template <typename TB>
static void launch_iters(Ctx *ctx, const SpmvArgs &M, const Sched &S, const Grids &g, hipStream_t s, int n) {
    for (int c = 0; c < n; ++c) {
        launch_one<TB>(ctx, M, S, g, s, ctx->cg_par);
        ctx->cg_par ^= 1;
    }
}

// Residuals always use the FP64 blocks.  mode 0 starts a sweep from x for
// the flagged instances (restart == nullptr: all), mode 2 does the same but
// keeps the search direction (residual replacement), mode 1 writes
// ||b - A x||^2 and ||b||^2 of every instance to out2.
static void launch_residual(Ctx *ctx, const SpmvArgs &M, const Sched &S, const Grids &g, const uint8_t *restart,
                            const double *b, const double *x, int mode, double *out2, hipStream_t s) {
    using TB = double;
    if (mode == 0) {
        if (ctx->inner32)
            hipLaunchKernelGGL((k_residual<TB, 0, float>), dim3(g.sblocks), dim3(g.sthreads), 0, s, M, S, restart, b,
                               x, ctx->r32, ctx->p, pre_args(ctx), ctx->partials, ctx->e32);
        else
            hipLaunchKernelGGL((k_residual<TB, 0, double>), dim3(g.sblocks), dim3(g.sthreads), 0, s, M, S, restart,
                               b, x, ctx->r, ctx->p, pre_args(ctx), ctx->partials, (double *)nullptr);
        hipLaunchKernelGGL(k_fin_start, dim3(ctx->ninst), dim3(256), 0, s, S, 1, ctx->cg_par, restart, ctx->partials,
                           ctx->st);
    } else if (mode == 2) {
        if (ctx->inner32) {
            hipLaunchKernelGGL((k_residual<TB, 2, float>), dim3(g.sblocks), dim3(g.sthreads), 0, s, M, S, restart, b,
                               x, ctx->r32, ctx->p, pre_args(ctx), ctx->partials, ctx->e32);
            hipLaunchKernelGGL(k_pcg_redirect<float>, dim3(g.vblocks), dim3(VT), 0, s, S, restart,
                               (const float *)ctx->r32, ctx->p, pre_args(ctx), (const PcgState *)ctx->st,
                               (const double *)ctx->partials);
        } else {
            hipLaunchKernelGGL((k_residual<TB, 2, double>), dim3(g.sblocks), dim3(g.sthreads), 0, s, M, S, restart,
                               b, x, ctx->r, ctx->p, pre_args(ctx), ctx->partials, (double *)nullptr);
            hipLaunchKernelGGL(k_pcg_redirect<double>, dim3(g.vblocks), dim3(VT), 0, s, S, restart,
                               (const double *)ctx->r, ctx->p, pre_args(ctx), (const PcgState *)ctx->st,
                               (const double *)ctx->partials);
        }
        hipLaunchKernelGGL(k_fin_start, dim3(ctx->ninst), dim3(256), 0, s, S, 1, ctx->cg_par, restart, ctx->partials,
                           ctx->st);
    } else {
        hipLaunchKernelGGL((k_residual<TB, 1, double>), dim3(g.sblocks), dim3(g.sthreads), 0, s, M, S, restart, b, x,
                           ctx->r, ctx->p, pre_args(ctx), ctx->partials, (double *)nullptr);
        hipLaunchKernelGGL(k_fin_check, dim3(ctx->ninst), dim3(256), 0, s, S, ctx->partials, out2);
    }
}

static void launch_start_zero(Ctx *ctx, const Sched &S, const Grids &g, const uint8_t *restart, const double *b,
                              hipStream_t s) {
    if (ctx->inner32)
        hipLaunchKernelGGL(k_pcg_start_zero<float>, dim3(g.vblocks), dim3(VT), 0, s, S, restart, b, ctx->x,
                           ctx->r32, ctx->p, pre_args(ctx), ctx->partials, ctx->e32);
    else
        hipLaunchKernelGGL(k_pcg_start_zero<double>, dim3(g.vblocks), dim3(VT), 0, s, S, restart, b, ctx->x,
                           ctx->r, ctx->p, pre_args(ctx), ctx->partials, (double *)nullptr);
    hipLaunchKernelGGL(k_fin_start, dim3(ctx->ninst), dim3(256), 0, s, S, 0, ctx->cg_par, restart, ctx->partials,
                       ctx->st);
}

// With FP32 inner vectors the sweep's correction is added to x at its end.
static void launch_fold(Ctx *ctx, hipStream_t s) {
    if (!ctx->inner32) return;
    const int64_t n3 = 3 * (int64_t)ctx->nv;
    hipLaunchKernelGGL(k_fold, dim3((n3 + 255) / 256), dim3(256), 0, s, n3, ctx->x, ctx->e32);
}

// FP32 inner vectors apply to BF16 and FP16 blocks with the textbook
// recurrences (the refinement sweeps only ask 1e-2 of each inner solve there).
pc_status set_inner_vectors(Ctx *ctx) {
    ctx->inner32 = ctx->use_inner32 && (ctx->dtype == PC_BF16 || ctx->dtype == PC_F16) && ctx->method == 0;
    if (ctx->inner32 && !ctx->e32) {
        const size_t bytes = sizeof(float) * 3 * (size_t)ctx->nv;
        pc_status st;
        if ((st = dev_alloc(ctx, (void **)&ctx->e32, bytes))) return st;
        if ((st = dev_alloc(ctx, (void **)&ctx->r32, bytes))) return st;
        if ((st = dev_alloc(ctx, (void **)&ctx->q32, bytes))) return st;
        PC_HIP(hipMemset(ctx->e32, 0, bytes));
    }
    return PC_OK;
}

// storage type of a block template, as its pc_dtype (graph keys)
template <typename TB> constexpr int dtype_code();
template <> constexpr int dtype_code<double>() { return PC_F64; }
template <> constexpr int dtype_code<float>() { return PC_F32; }
template <> constexpr int dtype_code<bf16_t>() { return PC_BF16; }
template <> constexpr int dtype_code<f16_t>() { return PC_F16; }

static bool graph_stale(const Ctx *ctx, int variant, const SpmvArgs &M, int code) {
    return !ctx->gexec[variant] || ctx->gkey[variant] != M.jval || ctx->gkey_dtype[variant] != code ||
           ctx->gkey_chunk[variant] != ctx->graph_chunk || ctx->gkey_sched[variant] != ctx->sched_version ||
           ctx->gkey_pre[variant] != ctx->precond || ctx->gkey_win[variant] != ctx->win_cap ||
           ctx->gkey_narrow[variant] != (int)ctx->narrow || ctx->gkey_method[variant] != ctx->method ||
           ctx->gkey_inner32[variant] != (int)ctx->inner32;
}

// Capture `chunk` (even) iterations on the context's capture stream; the
// captured parities start at 0, so a replay must start at parity 0 and
// leaves the parity unchanged.
template <typename TB>
static pc_status capture_chunk(Ctx *ctx, const SpmvArgs &M, const Sched &S, const Grids &g, int chunk,
                               int variant) {
    if (!ctx->cap_stream) PC_HIP(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    if (ctx->gexec[variant]) {
        (void)hipGraphExecDestroy(ctx->gexec[variant]);
        ctx->gexec[variant] = nullptr;
    }
    const int saved = ctx->prof.every;
    ctx->prof.every = 0;  // no profiler events inside the graph
    hipStream_t cs = ctx->cap_stream;
    PC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int c = 0; c < chunk; ++c) launch_one<TB>(ctx, M, S, g, cs, c & 1);
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(cs, &graph);
    ctx->prof.every = saved;
    if (ec != hipSuccess) {
        ctx->err = std::string("hipStreamEndCapture: ") + hipGetErrorString(ec);
        return PC_ERR_HIP;
    }
    hipError_t e = hipGraphInstantiate(&ctx->gexec[variant], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        ctx->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
        ctx->gexec[variant] = nullptr;
        return PC_ERR_HIP;
    }
    ctx->gkey[variant] = M.jval;
    ctx->gkey_dtype[variant] = dtype_code<TB>();
    ctx->gkey_chunk[variant] = chunk;
    ctx->gkey_sched[variant] = ctx->sched_version;
    ctx->gkey_pre[variant] = ctx->precond;
    ctx->gkey_win[variant] = ctx->win_cap;
    ctx->gkey_narrow[variant] = (int)ctx->narrow;
    ctx->gkey_method[variant] = ctx->method;
    ctx->gkey_inner32[variant] = (int)ctx->inner32;
    return PC_OK;
}

pc_status spmv_run(Ctx *ctx, const double *xin, double *y, bool solver, hipStream_t s) {
    if (!ctx->assembled) {
        ctx->err = "cloth_spmv: nothing assembled";
        return PC_ERR_ARG;
    }
    const SpmvArgs M = spmv_args(ctx, !solver);
    const Sched S = sched_args(ctx);
    const Grids g = grids(ctx);
    switch (solver ? ctx->dtype : PC_F64) {
        case PC_F64:
            hipLaunchKernelGGL(k_spmv_apply<double>, dim3(g.sblocks), dim3(g.sthreads), 0, s, M, S, xin, y);
            break;
        case PC_F32:
            hipLaunchKernelGGL(k_spmv_apply<float>, dim3(g.sblocks), dim3(g.sthreads), 0, s, M, S, xin, y);
            break;
        case PC_BF16:
            hipLaunchKernelGGL(k_spmv_apply<bf16_t>, dim3(g.sblocks), dim3(g.sthreads), 0, s, M, S, xin, y);
            break;
        case PC_F16:
            hipLaunchKernelGGL(k_spmv_apply<f16_t>, dim3(g.sblocks), dim3(g.sthreads), 0, s, M, S, xin, y);
            break;
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

static pc_status read_states(Ctx *ctx, hipStream_t s) {
    PC_HIP(hipMemcpyAsync(ctx->st_host, ctx->st, sizeof(PcgState) * ctx->ninst, hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
    return PC_OK;
}

static pc_status upload_flags(Ctx *ctx, const std::vector<uint8_t> &f, hipStream_t s) {
    for (int i = 0; i < ctx->ninst; ++i) ctx->restart_h[i] = f[i];
    PC_HIP(hipMemcpyAsync(ctx->restart, ctx->restart_h, (size_t)ctx->ninst, hipMemcpyHostToDevice, s));
    return PC_OK;
}

// CG on every instance from the start in ctx->x (warm) or from zero, until
// each instance's recursive residual meets its threshold; then the residual
// of every instance is recomputed with the FP64 blocks, and instances whose
// true residual misses the tolerance restart from x (iterative refinement),
// up to max_sweeps sweeps.  Per-instance results go to ctx->inst_info; info
// receives the aggregate (total iterations of the slowest instance, largest
// residuals).
template <typename TB>
static pc_status pcg_typed(Ctx *ctx, const double *b, double *dv, const pc_solve_opts *o, pc_solve_info *info,
                           hipStream_t s) {
    const SpmvArgs M = spmv_args(ctx, false);
    const SpmvArgs Mhi = spmv_args(ctx, true);
    const Sched S = sched_args(ctx);
    const Grids g = grids(ctx);
    const int nv = ctx->nv, ninst = ctx->ninst;
    const double tol = o ? o->tol : 1e-6;
    const int maxit = (o && o->maxit > 0) ? o->maxit : 20000;
    int warm = o ? o->warm : 0;
    const int check = (o && o->check_every > 0) ? o->check_every : 0;
    const bool lowp = ctx->dtype == PC_BF16 || ctx->dtype == PC_F16;
    // With PC_OPT_KEEP_DIRECTION, FP16 sweeps keep the search direction
    // (residual replacement: the FP64 residual replaces the recursive one and
    // CG goes on), each ending when the recursive residual has halved; BF16's
    // coarser rounding does not let the continued recurrence converge
    const bool keep = ctx->use_keep_dir && ctx->dtype == PC_F16 && ctx->method == 0;
    pc_status wst = ensure_windows(ctx, s);
    if (wst) return wst;
    const double rho = (o && o->inner_rho > 0.0) ? o->inner_rho : (lowp ? (keep ? 0.5 : 1e-2) : 0.0);
    const int max_sweeps = (o && o->max_sweeps > 0) ? o->max_sweeps : (keep ? 400 : (lowp ? 40 : 4));
    // a low-precision sweep must bring the FP64 residual below this factor of
    // its start: half for restarted sweeps, halfway between 1 and rho when
    // sweeps keep the direction (each asks only for a reduction by rho)
    const double contract = keep ? 0.5 * (1.0 + std::min(rho, 1.0)) : 0.5;
    const int64_t n3 = 3 * (int64_t)nv;

    std::vector<int> iters(ninst, 0), sweeps(ninst, 0), fallback(ninst, 0), wused(ninst, 0);
    std::vector<uint8_t> active(ninst, 1);
    std::vector<double> res2(2 * ninst, 0.0);
    // Refinement sweeps on the low-precision copy (inner reduction rho > 0)
    // have an iteration budget: half of maxit for the first, three times the
    // instance's longest earlier sweep (at least 256) for the others.  For
    // some states the copy's rounding leaves CG on it diverging or stalled,
    // which no per-iteration test sees while p.Ap stays positive; a sweep
    // that reaches its budget ends like any other, and the contraction check
    // below then moves the instance to the FP64 blocks.
    const bool sweep_budget = rho > 0.0 && ctx->hi_valid;
    std::vector<int> longest(ninst, 0);
    std::vector<int> maxit_h(ninst, sweep_budget ? std::max(1, maxit / 2) : maxit);
    pc_status st;

    ctx->cg_par = 0;
    int warm_kind = 0;
    if (warm == 2) {
        // learned start from the previous increment held in dv
        if (!ctx->mlp || !ctx->last_x) {
            ctx->err = "learned warm start requested without parameters or an assembled state";
            return PC_ERR_ARG;
        }
        int used = 0;
        if ((st = mlp_start(ctx, ctx->mlp, ctx->last_x, ctx->last_v, b, dv, ctx->x, ctx->q, &used, s))) return st;
        warm_kind = used;
    } else if (warm) {
        hipLaunchKernelGGL(k_copy_d, dim3((n3 + 255) / 256), dim3(256), 0, s, n3, dv, ctx->x);
        warm_kind = 1;
    }
    for (int i = 0; i < ninst; ++i) wused[i] = warm_kind;

    // first start of every instance
    PC_HIP(hipMemcpyAsync(ctx->maxit_d, maxit_h.data(), sizeof(int) * ninst, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_state_init, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, ctx->st,
                       (const uint8_t *)nullptr, tol, rho, ctx->maxit_d);
    if (warm_kind) {
        // the start is used as given: its residual norm is no guide to the
        // CG iterations it saves (a start accurate in the slowly converging
        // smooth modes can have a residual above ||b||)
        launch_residual(ctx, Mhi, S, g, nullptr, b, ctx->x, 0, nullptr, s);
    } else {
        launch_start_zero(ctx, S, g, nullptr, b, s);
    }
    PC_HIP(hipGetLastError());
    for (int i = 0; i < ninst; ++i) sweeps[i] = 1;
    bool inner_hi = false;
    int guard = 0;
    long long nchunk = 0;
    for (;;) {
        if ((st = read_states(ctx, s))) return st;
        // iterate until every instance is done
        const int variant = inner_hi ? 1 : 0;
        const bool graph = ctx->graph_chunk > 0;
        if (graph) {
            const SpmvArgs &Mv = inner_hi ? Mhi : M;
            const int want_code = inner_hi ? dtype_code<double>() : dtype_code<TB>();
            if (graph_stale(ctx, variant, Mv, want_code)) {
                st = inner_hi ? capture_chunk<double>(ctx, Mhi, S, g, ctx->graph_chunk, variant)
                              : capture_chunk<TB>(ctx, M, S, g, ctx->graph_chunk, variant);
                if (st) return st;
            }
        }
        for (;;) {
            bool all_done = true;
            int most = 0;
            for (int i = 0; i < ninst; ++i) {
                const PcgState &h = ctx->st_host[i];
                if (!h.done) {
                    all_done = false;
                    most = std::max(most, h.iters);
                }
            }
            if (all_done) break;
            // with profiling on, events are recorded in one chunk in 8 only, so
            // that they add little to the solve's time; with graph replay that
            // chunk runs as plain launches, which the events time
            const bool sample = ctx->prof.every > 0 && (nchunk++ % 8) == 0;
            if (graph && !sample && ctx->cg_par == 0) {
                PC_HIP(hipGraphLaunch(ctx->gexec[variant], s));
            } else {
                int chunk = graph ? ctx->graph_chunk : (check > 0 ? check : std::min(256, std::max(16, most / 4)));
                if (graph && ctx->cg_par != 0) chunk = 1;   // back to even parity for the graph
                const int every = ctx->prof.every;
                if (!sample) ctx->prof.every = 0;
                if (inner_hi)
                    launch_iters<double>(ctx, Mhi, S, g, s, chunk);
                else
                    launch_iters<TB>(ctx, M, S, g, s, chunk);
                ctx->prof.every = every;
            }
            PC_HIP(hipGetLastError());
            if ((st = read_states(ctx, s))) return st;
            ctx->prof.harvest();
        }
        for (int i = 0; i < ninst; ++i)
            if (active[i]) {
                iters[i] += ctx->st_host[i].iters;
                longest[i] = std::max(longest[i], ctx->st_host[i].iters);
            }
        launch_fold(ctx, s);
        // true residual of every instance
        launch_residual(ctx, Mhi, S, g, nullptr, b, ctx->x, 1, ctx->res2, s);
        PC_HIP(hipGetLastError());
        PC_HIP(hipMemcpyAsync(res2.data(), ctx->res2, sizeof(double) * 2 * ninst, hipMemcpyDeviceToHost, s));
        PC_HIP(hipStreamSynchronize(s));
        std::vector<uint8_t> again(ninst, 0);
        bool any = false, any_breakdown = false;
        for (int i = 0; i < ninst; ++i) {
            const PcgState &h = ctx->st_host[i];
            const bool was_active = active[i] != 0;
            active[i] = 0;
            const bool ok = res2[2 * i] <= tol * tol * res2[2 * i + 1];
            if (ok || res2[2 * i + 1] == 0.0 || (h.flags & 2) || iters[i] >= maxit) continue;
            if (h.flags & 1) {
                if (!inner_hi && ctx->hi_valid) {
                    any_breakdown = true;
                    fallback[i] = 1;
                } else {
                    continue;
                }
            } else if (!inner_hi && ctx->hi_valid && was_active &&
                       !(res2[2 * i] <= contract * contract * h.rr0)) {
                // the sweep on the low-precision copy did not bring the FP64
                // residual it started from below the contraction factor:
                // refinement with that operator is not contracting for this
                // system (its rounding is too coarse for the conditioning); FP64
                // blocks from here on
                any_breakdown = true;
                fallback[i] = 1;
            } else if (sweeps[i] >= max_sweeps) {
                continue;
            }
            again[i] = 1;
            active[i] = 1;
            any = true;
        }
        if (!any || ++guard > max_sweeps + 8) break;
        if (any_breakdown) inner_hi = true;  // low-precision operator lost definiteness or stopped contracting: FP64 blocks from here on
        for (int i = 0; i < ninst; ++i) {
            if (again[i]) {
                sweeps[i] += 1;
                maxit_h[i] = maxit - iters[i];
                if (sweep_budget && !inner_hi) maxit_h[i] = std::min(maxit_h[i], std::max(256, 3 * longest[i]));
            }
        }
        PC_HIP(hipMemcpyAsync(ctx->maxit_d, maxit_h.data(), sizeof(int) * ninst, hipMemcpyHostToDevice, s));
        if ((st = upload_flags(ctx, again, s))) return st;
        hipLaunchKernelGGL(k_state_init, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, ctx->st, ctx->restart, tol,
                           rho, ctx->maxit_d);
        // a breakdown or the switch to the FP64 blocks restarts from P^-1 r
        launch_residual(ctx, Mhi, S, g, ctx->restart, b, ctx->x, (keep && !any_breakdown) ? 2 : 0, nullptr, s);
        PC_HIP(hipGetLastError());
    }
    // b = 0: the solution is 0 whatever the start
    std::vector<uint8_t> zero(ninst, 0);
    bool anyzero = false;
    for (int i = 0; i < ninst; ++i)
        if (res2[2 * i + 1] == 0.0 && !(ctx->st_host[i].flags & 2)) {
            zero[i] = 1;
            anyzero = true;
            res2[2 * i] = 0.0;
        }
    if (anyzero) {
        if ((st = upload_flags(ctx, zero, s))) return st;
        hipLaunchKernelGGL(k_zero_rows, dim3(g.vblocks), dim3(VT), 0, s, S, ctx->restart, ctx->x);
    }
    hipLaunchKernelGGL(k_copy_d, dim3((n3 + 255) / 256), dim3(256), 0, s, n3, ctx->x, dv);
    PC_HIP(hipGetLastError());
    PC_HIP(hipStreamSynchronize(s));
    pc_status ret = PC_OK;
    pc_solve_info agg{};
    double bb_all = 0.0, tt_all = 0.0;
    for (int i = 0; i < ninst; ++i) {
        const PcgState &h = ctx->st_host[i];
        pc_solve_info &I = ctx->inst_info[i];
        const double bn = sqrt(res2[2 * i + 1]);
        I.iters = iters[i];
        I.sweeps = sweeps[i];
        I.bnorm = bn;
        I.rel_res_recursive = bn > 0 ? sqrt(h.rr) / bn : 0.0;
        I.rel_res_true = bn > 0 ? sqrt(res2[2 * i]) / bn : sqrt(res2[2 * i]);
        I.fallback = fallback[i];
        I.warm_used = wused[i];
        agg.iters = std::max(agg.iters, I.iters);
        agg.sweeps = std::max(agg.sweeps, I.sweeps);
        agg.rel_res_recursive = std::max(agg.rel_res_recursive, I.rel_res_recursive);
        agg.rel_res_true = std::max(agg.rel_res_true, I.rel_res_true);
        agg.fallback |= I.fallback;
        agg.warm_used = std::max(agg.warm_used, I.warm_used);
        bb_all += res2[2 * i + 1];
        tt_all += res2[2 * i];
        if (ret == PC_OK) {
            if (h.flags & 2) {
                ctx->err = "non-finite value in the CG recurrence";
                ret = PC_ERR_NONFINITE;
            } else if ((h.flags & 1) && !(I.rel_res_true <= tol)) {
                ctx->err = "CG breakdown: p.Ap <= 0 (matrix not positive definite)";
                ret = PC_ERR_NOT_CONVERGED;
            } else if (!(I.rel_res_true <= tol) && bn > 0) {
                ctx->err = "CG did not reach the tolerance within maxit iterations";
                ret = PC_ERR_NOT_CONVERGED;
            }
        }
    }
    agg.bnorm = sqrt(bb_all);
    if (ninst == 1) agg = ctx->inst_info[0];
    if (info) *info = agg;
    (void)tt_all;
    return ret;
}

// Time `iters` CG iterations from the zero start on the assembled system
// with the current schedule (milliseconds, HIP events on the stream).
template <typename TB>
static pc_status time_iters(Ctx *ctx, const double *b, int iters, float *ms, hipStream_t s) {
    const SpmvArgs M = spmv_args(ctx, false);
    const Sched S = sched_args(ctx);
    const Grids g = grids(ctx);
    const int ninst = ctx->ninst;
    std::vector<int> big(ninst, 1 << 30);
    PC_HIP(hipMemcpyAsync(ctx->maxit_d, big.data(), sizeof(int) * ninst, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_state_init, dim3((ninst + 63) / 64), dim3(64), 0, s, ninst, ctx->st,
                       (const uint8_t *)nullptr, 0.0, 0.0, ctx->maxit_d);
    pc_status wst = ensure_windows(ctx, s);
    if (wst) return wst;
    ctx->cg_par = 0;
    launch_start_zero(ctx, S, g, nullptr, b, s);
    if (ctx->graph_chunk > 0 && graph_stale(ctx, 0, M, dtype_code<TB>())) {
        pc_status st = capture_chunk<TB>(ctx, M, S, g, ctx->graph_chunk, 0);
        if (st) return st;
    }
    hipEvent_t e0, e1;
    PC_HIP(hipEventCreate(&e0));
    PC_HIP(hipEventCreate(&e1));
    PC_HIP(hipEventRecord(e0, s));
    if (ctx->graph_chunk > 0) {
        for (int done = 0; done < iters; done += ctx->graph_chunk) PC_HIP(hipGraphLaunch(ctx->gexec[0], s));
    } else {
        const int saved = ctx->prof.every;
        ctx->prof.every = 0;
        launch_iters<TB>(ctx, M, S, g, s, iters);
        ctx->prof.every = saved;
    }
    PC_HIP(hipEventRecord(e1, s));
    PC_HIP(hipEventSynchronize(e1));
    PC_HIP(hipEventElapsedTime(ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return PC_OK;
}

// Autotuner: try every (slices per SpMV block, rows per vector block, graph
// chunk) candidate on the assembled system, keep the fastest per iteration.
pc_status autotune_run(Ctx *ctx, const double *b, int iters, int64_t *chosen, float *best_ms, hipStream_t s) {
    if (!ctx->assembled) {
        ctx->err = "pc_autotune: nothing assembled";
        return PC_ERR_ARG;
    }
    const int spbs[4] = {2, 4, 8, 16};
    const int chunks[2] = {0, 32};
    // rows per vector block: fixed sizes, plus for k = 1, 2 the smallest
    // multiple of 64 that gives at most k work items per compute unit over all
    // instances.  The vector kernels then run in one round with every CU
    // holding k blocks, so no CU still runs an extra block at the end of the
    // launch (at 1.65M rows 2,048-row items leave 149 of 256 CUs with two).
    std::vector<int> rpbs = {1024, 2048, 4096};
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0) {
        for (int k = 1; k <= 2; ++k) {
            for (int rp = 64; rp <= 4096; rp += 64) {
                int64_t n = 0;
                for (size_t i = 0; i + 1 < ctx->inst_row0_h.size(); ++i)
                    n += (ctx->inst_row0_h[i + 1] - ctx->inst_row0_h[i] + rp - 1) / rp;
                if (n <= (int64_t)k * ncu) {
                    if (std::find(rpbs.begin(), rpbs.end(), rp) == rpbs.end()) rpbs.push_back(rp);
                    break;
                }
            }
        }
    }
    float best = 1e30f;
    int bs = ctx->spb, br = ctx->rpb, bc = ctx->graph_chunk;
    const bool was = ctx->assembled;
    for (int c : chunks)
        for (int sp : spbs)
            for (int rp : rpbs) {
                ctx->spb = sp;
                ctx->rpb = rp;
                ctx->graph_chunk = c;
                pc_status st = build_schedule(ctx);
                ctx->assembled = was;
                if (st) return st;
                float ms = 0.0f;
                switch (ctx->dtype) {
                    case PC_F64: st = time_iters<double>(ctx, b, iters, &ms, s); break;
                    case PC_F32: st = time_iters<float>(ctx, b, iters, &ms, s); break;
                    case PC_BF16: st = time_iters<bf16_t>(ctx, b, iters, &ms, s); break;
                    case PC_F16: st = time_iters<f16_t>(ctx, b, iters, &ms, s); break;
                }
                if (st) return st;
                if (ms < best) {
                    best = ms;
                    bs = sp;
                    br = rp;
                    bc = c;
                }
            }
    ctx->spb = bs;
    ctx->rpb = br;
    ctx->graph_chunk = bc;
    pc_status st = build_schedule(ctx);
    ctx->assembled = was;
    if (st) return st;
    if (chosen) {
        chosen[0] = bs;
        chosen[1] = br;
        chosen[2] = bc;
    }
    if (best_ms) *best_ms = best / (float)iters;
    return PC_OK;
}

pc_status pcg_run(Ctx *ctx, const double *b, double *dv, const pc_solve_opts *o, pc_solve_info *info,
                  hipStream_t s) {
    if (!ctx->assembled) {
        ctx->err = "cloth_pcg_solve: nothing assembled";
        return PC_ERR_ARG;
    }
    ctx->precond = o ? o->precond : 0;
    ctx->method = o ? o->method : 0;
    if (ctx->method == 1 && !ctx->cg_pd) {
        pc_status st = dev_alloc(ctx, (void **)&ctx->cg_pd, sizeof(double) * 3 * (size_t)ctx->nv);
        if (st) return st;
        if ((st = dev_alloc(ctx, (void **)&ctx->cg_s, sizeof(double) * 3 * (size_t)ctx->nv))) return st;
    }
    pc_status ist = set_inner_vectors(ctx);
    if (ist) return ist;
    switch (ctx->dtype) {
        case PC_F64: return pcg_typed<double>(ctx, b, dv, o, info, s);
        case PC_F32: return pcg_typed<float>(ctx, b, dv, o, info, s);
        case PC_BF16: return pcg_typed<bf16_t>(ctx, b, dv, o, info, s);
        case PC_F16: return pcg_typed<f16_t>(ctx, b, dv, o, info, s);
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
