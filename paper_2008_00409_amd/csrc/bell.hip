// The paper's own sparse-matrix filling and BELL SpMV (Sec. 3.2.2), built
// beside the solver's assembly for an A/B comparison on the same system:
//   1. Index table allocating: count every row's index-table slots (each
//      element corner contributes one slot per vertex of its element);
//   2. Index filling: every element writes the (row, column) pairs of its
//      corners into the rows' index tables, slots taken with integer atomics;
//   3. Index compacting: one thread per row sorts its slots and removes
//      duplicates;
//   4. Value table allocating: BELL with the largest compacted row length;
//   5. Value filling: every element adds its 3x3 stiffness blocks into the
//      value table with floating-point atomics.
// Values are A = M + h (h + beta) K with pinned rows and columns eliminated
// and b as in Eq. 3 (the same system as the solver's assembly).  Layout:
// slot k of row i at k nv + i (a thread per row reads consecutive
// addresses), 9 value planes, padded slots with column i and zero blocks.
// The summation order of the atomics, and with it the last bits of A and b,
// varies from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pc_ctx.h"
#include "pc_elements.h"

namespace pc {

// 1. index-table slots per row: every element corner adds one slot per
// vertex of its element; every row also gets one slot for its own diagonal
// block (so that a vertex outside every element still holds its mass).
__global__ void k_bell_count(int nv, int nt, int nh, int nc, const int *tri, const int *hinge, const int *cverts,
                             int *cnt) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntc = 3 * (int64_t)nt, nhc = 4 * (int64_t)nh, ncc = 4 * (int64_t)nc;
    if (idx < ntc) atomicAdd(&cnt[tri[idx]], 3);
    else if (idx < ntc + nhc) atomicAdd(&cnt[hinge[idx - ntc]], 4);
    else if (idx < ntc + nhc + ncc) atomicAdd(&cnt[cverts[idx - ntc - nhc]], 4);
    else if (idx < ntc + nhc + ncc + nv) atomicAdd(&cnt[idx - ntc - nhc - ncc], 1);
}

__global__ void k_max_int(const int *a, int n, int *out) {
    int m = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) m = max(m, a[i]);
    for (int d = 32; d >= 1; d >>= 1) m = max(m, __shfl_xor(m, d, WAVE));
    if (lane_id() == 0) atomicMax(out, m);
}

// Vertices of element corner `idx` (as in k_bell_count's numbering): the
// corner's own vertex, the element's vertex count and its vertices.
__device__ __forceinline__ int bell_element(int64_t idx, int nt, int nh, const int *tri, const int *hinge,
                                            const int *cverts, int &self, int ev[4]) {
    const int64_t ntc = 3 * (int64_t)nt, nhc = 4 * (int64_t)nh;
    if (idx < ntc) {
        const int t = (int)(idx % nt);
#pragma unroll
        for (int q = 0; q < 3; ++q) ev[q] = tri[q * nt + t];
        self = tri[idx];
        return 3;
    }
    if (idx < ntc + nhc) {
        const int64_t j = idx - ntc;
        const int h = (int)(j % nh);
#pragma unroll
        for (int q = 0; q < 4; ++q) ev[q] = hinge[q * nh + h];
        self = hinge[j];
        return 4;
    }
    const int64_t j = idx - ntc - nhc;
    const int e = (int)(j >> 2);
#pragma unroll
    for (int q = 0; q < 4; ++q) ev[q] = cverts[4 * e + q];
    self = cverts[j];
    return 4;
}

// 2. index filling
__global__ void k_bell_index_fill(int nv, int nt, int nh, int nc, const int *tri, const int *hinge,
                                  const int *cverts, int Wi, int *fill, int *idxtab) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ncorner = 3 * (int64_t)nt + 4 * (int64_t)nh + 4 * (int64_t)nc;
    if (idx >= ncorner + nv) return;
    if (idx >= ncorner) {
        const int i = (int)(idx - ncorner);
        const int slot = atomicAdd(&fill[i], 1);
        idxtab[(int64_t)i * Wi + slot] = i;
        return;
    }
    int self, ev[4];
    const int m = bell_element(idx, nt, nh, tri, hinge, cverts, self, ev);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        if (l >= m) break;
        const int slot = atomicAdd(&fill[self], 1);
        idxtab[(int64_t)self * Wi + slot] = ev[l];
    }
}

// 3. compacting: one thread per row sorts its slots (insertion sort) and
// removes duplicates; the row is staged in LDS (slot a of the block's
// thread t at a * 64 + t, so a wavefront's accesses hit distinct banks).
__global__ void __launch_bounds__(64) k_bell_compact(int nv, int Wi, int *idxtab, const int *fill, int *len,
                                                      int *maxlen) {
    extern __shared__ int stage[];
    const int t = threadIdx.x;
    const int i = blockIdx.x * 64 + t;
    if (i >= nv) return;
    int *r = stage + t;
    int *g = idxtab + (int64_t)i * Wi;
    const int n = fill[i];
    for (int a = 0; a < n; ++a) r[64 * a] = g[a];
    for (int a = 1; a < n; ++a) {
        const int key = r[64 * a];
        int b = a - 1;
        while (b >= 0 && r[64 * b] > key) {
            r[64 * (b + 1)] = r[64 * b];
            --b;
        }
        r[64 * (b + 1)] = key;
    }
    int m = 0, last = -1;
    for (int a = 0; a < n; ++a) {
        const int c = r[64 * a];
        if (c != last) g[m++] = c;
        last = c;
    }
    len[i] = m;
    atomicMax(maxlen, m);
}

// The same without LDS, for rows longer than the stage holds.
__global__ void k_bell_compact_global(int nv, int Wi, int *idxtab, const int *fill, int *len, int *maxlen) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    int *r = idxtab + (int64_t)i * Wi;
    const int n = fill[i];
    for (int a = 1; a < n; ++a) {
        const int key = r[a];
        int b = a - 1;
        while (b >= 0 && r[b] > key) {
            r[b + 1] = r[b];
            --b;
        }
        r[b + 1] = key;
    }
    int m = 0;
    for (int a = 0; a < n; ++a)
        if (m == 0 || r[a] != r[m - 1]) r[m++] = r[a];
    len[i] = m;
    atomicMax(maxlen, m);
}

// 4. column table (column-major, padded with the row itself)
__global__ void k_bell_layout(int nv, int Wi, int Wv, const int *idxtab, const int *len, int *col) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    for (int k = 0; k < Wv; ++k) col[(int64_t)k * nv + i] = k < len[i] ? idxtab[(int64_t)i * Wi + k] : i;
}

template <typename T>
__global__ void k_bell_zero(int64_t n, T *p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = T(0);
}

__device__ __forceinline__ int bell_find(const int *row, int n, int col) {
    int lo = 0, hi = n - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        if (row[mid] == col) return mid;
        if (row[mid] < col) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

struct BellArgs {
    int nv, nt, nh, nc, Wi, Wv;
    const int *tri, *hinge, *cverts;
    const double *Bm, *A0, *hcoef, *htbar, *cw, *cn;
    double ceta, ckc;
    const double *x, *v;
    DevParams prm;
    const int *idxtab, *len;
    double *f;   // element forces (nv x 3, FP64 atomics)
    int *status;
};

template <typename TB>
__device__ __forceinline__ void bell_add(const BellArgs &A, TB *val, int row, int colv, const double blk[9]) {
    const int pos = bell_find(A.idxtab + (int64_t)row * A.Wi, A.len[row], colv);
    if (pos < 0) {
        atomicOr(A.status, ST_BADINDEX);
        return;
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) atomicAdd(&val[((int64_t)q * A.Wv + pos) * A.nv + row], (TB)(A.prm.c * blk[q]));
}

// 5. value filling: one thread per element (triangles, then hinges, then
// contacts), stiffness blocks at x, forces at the force state.
template <typename TB>
__global__ void __launch_bounds__(256) k_bell_values(BellArgs A, TB *val) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const DevParams &P = A.prm;
    if (e < A.nt) {
        const int t = (int)e;
        int vv[3];
        TriShape sh;
        const double B0 = A.Bm[t], B1 = A.Bm[A.nt + t], B2 = A.Bm[2 * A.nt + t], B3 = A.Bm[3 * A.nt + t];
        sh.b[1][0] = B0; sh.b[1][1] = B1;
        sh.b[2][0] = B2; sh.b[2][1] = B3;
        sh.b[0][0] = -B0 - B2; sh.b[0][1] = -B1 - B3;
        const double a0 = A.A0[t];
        d3 xs[3], ys[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            vv[q] = A.tri[q * A.nt + t];
            xs[q] = ld3(A.x, vv[q]);
            ys[q] = xs[q] + (P.s_look * P.h) * ld3(A.v, vv[q]);
        }
        double F[3][2], S[3], Sp[3];
        tri_F(xs, sh, F);
        tri_stress(F, P.mu, P.lam, S);
        psd_part(S, Sp);
        double u[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int a = 0; a < 3; ++a) u[k][a] = F[a][0] * sh.b[k][0] + F[a][1] * sh.b[k][1];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const double bb = sh.b[k][0] * sh.b[l][0] + sh.b[k][1] * sh.b[l][1];
                const double bSb = sh.b[k][0] * (Sp[0] * sh.b[l][0] + Sp[1] * sh.b[l][1]) +
                                   sh.b[k][1] * (Sp[1] * sh.b[l][0] + Sp[2] * sh.b[l][1]);
                double blk[9];
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const double fft = F[a][0] * F[b][0] + F[a][1] * F[b][1];
                        double val2 = P.mu * bb * fft + P.mu * u[l][a] * u[k][b] + P.lam * u[k][a] * u[l][b];
                        if (a == b) val2 += bSb;
                        blk[3 * a + b] = a0 * val2;
                    }
                bell_add<TB>(A, val, vv[k], vv[l], blk);
            }
        double Fy[3][2], Sy[3];
        tri_F(ys, sh, Fy);
        tri_stress(Fy, P.mu, P.lam, Sy);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double sb0 = Sy[0] * sh.b[k][0] + Sy[1] * sh.b[k][1];
            const double sb1 = Sy[1] * sh.b[k][0] + Sy[2] * sh.b[k][1];
#pragma unroll
            for (int a = 0; a < 3; ++a) atomicAdd(&A.f[3 * vv[k] + a], -a0 * (Fy[a][0] * sb0 + Fy[a][1] * sb1));
        }
        return;
    }
    if (e < (int64_t)A.nt + A.nh) {
        const int h = (int)(e - A.nt);
        int vv[4];
        d3 xs[4], ys[4], g[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            vv[q] = A.hinge[q * A.nh + h];
            xs[q] = ld3(A.x, vv[q]);
            ys[q] = xs[q] + (P.s_look * P.h) * ld3(A.v, vv[q]);
        }
        const double ch = A.hcoef[h], tb = A.htbar[h];
        double th;
        if (hinge_eval(xs, th, g)) {
            const double sc = 2.0 * P.kb * ch;
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    const double gk[3] = {g[k].x, g[k].y, g[k].z}, gl[3] = {g[l].x, g[l].y, g[l].z};
                    double blk[9];
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) blk[3 * a + b] = sc * gk[a] * gl[b];
                    bell_add<TB>(A, val, vv[k], vv[l], blk);
                }
        }
        if (hinge_eval(ys, th, g)) {
            const double s = -2.0 * P.kb * ch * (th - tb);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                atomicAdd(&A.f[3 * vv[k]], s * g[k].x);
                atomicAdd(&A.f[3 * vv[k] + 1], s * g[k].y);
                atomicAdd(&A.f[3 * vv[k] + 2], s * g[k].z);
            }
        }
        return;
    }
    if (e < (int64_t)A.nt + A.nh + A.nc) {
        const int c = (int)(e - A.nt - A.nh);
        int vv[4];
        double cw[4], gx = 0.0, gy = 0.0;
        const double n[3] = {A.cn[3 * c], A.cn[3 * c + 1], A.cn[3 * c + 2]};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            vv[q] = A.cverts[4 * c + q];
            cw[q] = A.cw[4 * c + q];
            const d3 xq = ld3(A.x, vv[q]);
            const d3 yq = xq + (P.s_look * P.h) * ld3(A.v, vv[q]);
            gx += cw[q] * (n[0] * xq.x + n[1] * xq.y + n[2] * xq.z);
            gy += cw[q] * (n[0] * yq.x + n[1] * yq.y + n[2] * yq.z);
        }
        if (gx < A.ceta)
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    double blk[9];
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) blk[3 * a + b] = A.ckc * cw[k] * cw[l] * n[a] * n[b];
                    bell_add<TB>(A, val, vv[k], vv[l], blk);
                }
        if (gy < A.ceta)
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int a = 0; a < 3; ++a) atomicAdd(&A.f[3 * vv[k] + a], A.ckc * (A.ceta - gy) * cw[k] * n[a]);
    }
}

// y = V x over the BELL table, one thread per row, FP64 accumulation; x as
// float4 (the search direction's storage in the solver) or as the caller's
// FP64 triples.
__device__ __forceinline__ void bell_ldx(const float4 *x, int j, double &a, double &b, double &c) {
    const float4 v = x[j];
    a = v.x; b = v.y; c = v.z;
}
__device__ __forceinline__ void bell_ldx(const double *x, int j, double &a, double &b, double &c) {
    a = x[3 * j]; b = x[3 * j + 1]; c = x[3 * j + 2];
}

template <typename TB, typename TX>
__global__ void __launch_bounds__(256) k_bell_spmv(int nv, int Wv, const int *col, const TB *val, const TX *x,
                                                   double *y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int k = 0; k < Wv; ++k) {
        const int j = col[(int64_t)k * nv + i];
        double x0, x1, x2;
        bell_ldx(x, j, x0, x1, x2);
        double b[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) b[q] = (double)val[((int64_t)q * Wv + k) * nv + i];
        a0 += b[0] * x0 + b[1] * x1 + b[2] * x2;
        a1 += b[3] * x0 + b[4] * x1 + b[5] * x2;
        a2 += b[6] * x0 + b[7] * x1 + b[8] * x2;
    }
    y[3 * i] = a0;
    y[3 * i + 1] = a1;
    y[3 * i + 2] = a2;
}

__global__ void k_to_f4(int nv, const double *x, float4 *x4) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nv) x4[i] = make_float4((float)x[3 * i], (float)x[3 * i + 1], (float)x[3 * i + 2], 0.0f);
}

// b = h (f + m g) - kvh (c K v) for free rows (kvh = h kv_coef / c), 0 for
// pinned rows; then the mass on the diagonal and the Dirichlet elimination.
template <typename TB>
__global__ void k_bell_finish(int nv, int Wv, const int *col, const int *len, TB *val, const double *mass,
                              const uint8_t *pinned, const double *f, const double *cKv, DevParams P, double kvh,
                              double *b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const bool pi = pinned[i] != 0;
    const double mi = mass[i];
    for (int a = 0; a < 3; ++a) b[3 * i + a] = pi ? 0.0 : P.h * (f[3 * i + a] + mi * P.g[a]) - kvh * cKv[3 * i + a];
    for (int k = 0; k < len[i]; ++k) {
        const int j = col[(int64_t)k * nv + i];
        const bool elim = pi || pinned[j] != 0;
        for (int q = 0; q < 9; ++q) {
            TB &e = val[((int64_t)q * Wv + k) * nv + i];
            if (elim) e = TB(0);
            if (j == i && (q == 0 || q == 4 || q == 8)) e = e + (TB)mi;
        }
    }
}

template <typename TB>
__global__ void k_bell_export(int nv, int Wv, const TB *val, double *out) {
    const int64_t n = 9 * (int64_t)Wv * nv;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)val[i];
}

// ---------------------------------------------------------------- host
constexpr int BELL_STAGE_SLOTS = 256;   // 64 rows x 256 slots x 4 B = 64 KiB of LDS
static pc_status grow(Ctx *ctx, void **p, size_t *have, size_t bytes) {
    if (bytes <= *have) return PC_OK;
    if (*p) dev_free(ctx, *p);
    *p = nullptr;
    *have = 0;
    pc_status st = dev_alloc(ctx, p, bytes);
    if (st) return st;
    *have = bytes;
    return PC_OK;
}

pc_status bell_assemble(Ctx *ctx, const double *x, const double *v, pc_dtype dtype, double *b, hipStream_t s) {
    if (dtype != PC_F32 && dtype != PC_F64) {
        ctx->err = "the paper-layout assembly stores FP32 or FP64 values";
        return PC_ERR_ARG;
    }
    BellState &Bs = ctx->bell;
    const int nv = ctx->nv, nt = ctx->nt, nh = ctx->nh, nc = ctx->nc;
    const int64_t nslot = 3 * (int64_t)nt + 4 * (int64_t)nh + 4 * (int64_t)nc + nv;   // threads of steps 1, 2
    const int TBK = 256;
    pc_status st;
    Bs.valid = false;
    if (nv == 0) {
        Bs.Wi = Bs.Wv = 0;
        Bs.dtype = dtype;
        Bs.valid = true;
        return PC_OK;
    }
    if ((st = grow(ctx, (void **)&Bs.cnt, &Bs.cnt_bytes, sizeof(int) * (size_t)(nv + 4)))) return st;
    if ((st = grow(ctx, (void **)&Bs.len, &Bs.len_bytes, sizeof(int) * (size_t)nv))) return st;
    if ((st = grow(ctx, (void **)&Bs.f, &Bs.f_bytes, sizeof(double) * 6 * (size_t)nv))) return st;
    int *maxv = Bs.cnt + nv;   // two scalars after the counts
    const int *cv = ctx->cverts;
    // 1. counts and the index-table width
    hipLaunchKernelGGL(k_bell_zero<int>, dim3((nv + 4 + 255) / 256), dim3(256), 0, s, (int64_t)(nv + 4), Bs.cnt);
    hipLaunchKernelGGL(k_bell_count, dim3((nslot + TBK - 1) / TBK), dim3(TBK), 0, s, nv, nt, nh, nc, ctx->tri,
                       ctx->hinge, cv, Bs.cnt);
    hipLaunchKernelGGL(k_max_int, dim3(256), dim3(256), 0, s, Bs.cnt, nv, maxv);
    int hostv[2] = {0, 0};
    PC_HIP(hipMemcpyAsync(hostv, maxv, sizeof(int), hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
    const int Wi = hostv[0];
    if ((st = grow(ctx, (void **)&Bs.idx, &Bs.idx_bytes, sizeof(int) * (size_t)nv * Wi))) return st;
    // 2. index filling (the counts are reused as fill pointers)
    hipLaunchKernelGGL(k_bell_zero<int>, dim3((nv + 4 + 255) / 256), dim3(256), 0, s, (int64_t)(nv + 4), Bs.cnt);
    hipLaunchKernelGGL(k_bell_index_fill, dim3((nslot + TBK - 1) / TBK), dim3(TBK), 0, s, nv, nt, nh, nc,
                       ctx->tri, ctx->hinge, cv, Wi, Bs.cnt, Bs.idx);
    // 3. compacting
    if (Wi <= BELL_STAGE_SLOTS)
        hipLaunchKernelGGL(k_bell_compact, dim3((nv + 63) / 64), dim3(64), sizeof(int) * 64 * (size_t)Wi, s, nv, Wi,
                           Bs.idx, Bs.cnt, Bs.len, maxv + 1);
    else
        hipLaunchKernelGGL(k_bell_compact_global, dim3((nv + 255) / 256), dim3(256), 0, s, nv, Wi, Bs.idx, Bs.cnt,
                           Bs.len, maxv + 1);
    PC_HIP(hipMemcpyAsync(hostv + 1, maxv + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
    const int Wv = hostv[1];
    // 4. value table
    const size_t esz = dtype == PC_F64 ? 8 : 4;
    if ((st = grow(ctx, (void **)&Bs.col, &Bs.col_bytes, sizeof(int) * (size_t)nv * Wv))) return st;
    if ((st = grow(ctx, &Bs.val, &Bs.val_bytes, esz * 9 * (size_t)nv * Wv))) return st;
    hipLaunchKernelGGL(k_bell_layout, dim3((nv + 255) / 256), dim3(256), 0, s, nv, Wi, Wv, Bs.idx, Bs.len, Bs.col);
    const int64_t nval = 9 * (int64_t)nv * Wv;
    // 5. values and forces
    BellArgs a;
    a.nv = nv; a.nt = nt; a.nh = nh; a.nc = nc; a.Wi = Wi; a.Wv = Wv;
    a.tri = ctx->tri; a.hinge = ctx->hinge; a.cverts = cv;
    a.Bm = ctx->Bm; a.A0 = ctx->A0; a.hcoef = ctx->hcoef; a.htbar = ctx->htbar; a.cw = ctx->cw; a.cn = ctx->cn;
    a.ceta = ctx->ceta; a.ckc = ctx->ckc; a.x = x; a.v = v; a.prm = ctx->prm;
    a.idxtab = Bs.idx; a.len = Bs.len; a.f = Bs.f; a.status = ctx->status;
    const int64_t nel = (int64_t)nt + nh + nc;
    hipLaunchKernelGGL(k_bell_zero<double>, dim3((6 * (int64_t)nv + 255) / 256), dim3(256), 0, s, 6 * (int64_t)nv,
                       Bs.f);
    if (!Bs.x4 && (st = dev_alloc(ctx, (void **)&Bs.x4, sizeof(float4) * (size_t)nv))) return st;
    if (dtype == PC_F64) {
        hipLaunchKernelGGL(k_bell_zero<double>, dim3((nval + 255) / 256), dim3(256), 0, s, nval, (double *)Bs.val);
        hipLaunchKernelGGL(k_bell_values<double>, dim3((nel + 255) / 256), dim3(256), 0, s, a, (double *)Bs.val);
    } else {
        hipLaunchKernelGGL(k_bell_zero<float>, dim3((nval + 255) / 256), dim3(256), 0, s, nval, (float *)Bs.val);
        hipLaunchKernelGGL(k_bell_values<float>, dim3((nel + 255) / 256), dim3(256), 0, s, a, (float *)Bs.val);
    }
    // c K v for the right-hand side (before the mass and the elimination)
    double *cKv = Bs.f + 3 * (size_t)nv;
    if (dtype == PC_F64)
        hipLaunchKernelGGL((k_bell_spmv<double, double>), dim3((nv + 255) / 256), dim3(256), 0, s, nv, Wv, Bs.col,
                           (const double *)Bs.val, v, cKv);
    else
        hipLaunchKernelGGL((k_bell_spmv<float, double>), dim3((nv + 255) / 256), dim3(256), 0, s, nv, Wv, Bs.col,
                           (const float *)Bs.val, v, cKv);
    const double kvh = ctx->prm.c > 0.0 ? ctx->prm.h * ctx->prm.kv_coef / ctx->prm.c : 0.0;
    if (dtype == PC_F64)
        hipLaunchKernelGGL(k_bell_finish<double>, dim3((nv + 255) / 256), dim3(256), 0, s, nv, Wv, Bs.col, Bs.len,
                           (double *)Bs.val, ctx->mass, ctx->pinned, Bs.f, cKv, ctx->prm, kvh, b);
    else
        hipLaunchKernelGGL(k_bell_finish<float>, dim3((nv + 255) / 256), dim3(256), 0, s, nv, Wv, Bs.col, Bs.len,
                           (float *)Bs.val, ctx->mass, ctx->pinned, Bs.f, cKv, ctx->prm, kvh, b);
    PC_HIP(hipGetLastError());
    Bs.Wi = Wi;
    Bs.Wv = Wv;
    Bs.dtype = dtype;
    Bs.valid = true;
    return PC_OK;
}

pc_status bell_spmv(Ctx *ctx, const double *x, double *y, hipStream_t s) {
    BellState &Bs = ctx->bell;
    if (!Bs.valid) {
        ctx->err = "cloth_spmv_bell: nothing assembled in the paper layout";
        return PC_ERR_ARG;
    }
    const int nv = ctx->nv;
    if (nv == 0) return PC_OK;
    hipLaunchKernelGGL(k_to_f4, dim3((nv + 255) / 256), dim3(256), 0, s, nv, x, Bs.x4);
    if (Bs.dtype == PC_F64)
        hipLaunchKernelGGL((k_bell_spmv<double, float4>), dim3((nv + 255) / 256), dim3(256), 0, s, nv, Bs.Wv,
                           Bs.col, (const double *)Bs.val, (const float4 *)Bs.x4, y);
    else
        hipLaunchKernelGGL((k_bell_spmv<float, float4>), dim3((nv + 255) / 256), dim3(256), 0, s, nv, Bs.Wv,
                           Bs.col, (const float *)Bs.val, (const float4 *)Bs.x4, y);
    PC_HIP(hipGetLastError());
    return PC_OK;
}

pc_status bell_export(Ctx *ctx, int32_t *width, int32_t *cols, double *vals, hipStream_t s) {
    BellState &Bs = ctx->bell;
    if (!Bs.valid) {
        ctx->err = "cloth_export_bell: nothing assembled in the paper layout";
        return PC_ERR_ARG;
    }
    if (width) *width = Bs.Wv;
    const int64_t n = (int64_t)ctx->nv * Bs.Wv;
    if (cols && n > 0) PC_HIP(hipMemcpyAsync(cols, Bs.col, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, s));
    if (vals && n > 0) {
        if (Bs.dtype == PC_F64)
            hipLaunchKernelGGL(k_bell_export<double>, dim3((9 * n + 255) / 256), dim3(256), 0, s, ctx->nv, Bs.Wv,
                               (const double *)Bs.val, vals);
        else
            hipLaunchKernelGGL(k_bell_export<float>, dim3((9 * n + 255) / 256), dim3(256), 0, s, ctx->nv, Bs.Wv,
                               (const float *)Bs.val, vals);
        PC_HIP(hipGetLastError());
    }
    return PC_OK;
}

void bell_free(Ctx *ctx, BellState &Bs) {
    void *ptrs[] = {Bs.cnt, Bs.len, Bs.f, Bs.idx, Bs.col, Bs.val, Bs.x4};
    for (void *p : ptrs)
        if (p) dev_free(ctx, p);
    Bs = BellState{};
}

}  // namespace pc
