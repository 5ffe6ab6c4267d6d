// Topology, rest data and per-step assembly of A and b (paper Sec. 2.5, Eq. 3;
// Sec. 3.2.2 for the dynamic block pattern and value filling).
//
// Per step, from the element list (triangles and hinges):
//   1. count the element corners incident to each vertex, scan, and fill the
//      per-vertex incidence buckets (integer atomics only: the contents of a
//      bucket are fixed, their order is not);
//   2. one wavefront per row sorts its incidences (type, element, corner),
//      derives the row's distinct block columns (sort + unique of the element
//      neighbours) and its length; a scan gives the block-CSR row pointers;
//   3. per 64-row slice, rows are ordered by length for the solver layout;
//   4. one wavefront per row evaluates its incident elements (one lane each),
//      then lane s sums, in incidence order, the contributions of every
//      element to block (i, cols[s]), in FP64 -- a deterministic segmented
//      reduce with no floating-point atomics -- and writes the row's blocks,
//      b_i, diag(A)_i and the pinned-neighbour remainder D_i.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pc_ctx.h"
#include "pc_elements.h"

namespace pc {

// ---------------------------------------------------------------- utilities
__global__ void k_fill_int(int *p, int v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Exclusive scan, 1024 elements per block (256 threads x 4).
constexpr int SCAN_TILE = 1024;

__global__ void k_scan_tiles(const int *in, int *out, int *tile_sums, int n) {
    __shared__ int sh[256];
    const int t = threadIdx.x;
    const int base = blockIdx.x * SCAN_TILE + t * 4;
    int v[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    sh[t] = s;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        int y = (t >= d) ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    int run = sh[t] - s;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (t == 255) tile_sums[blockIdx.x] = sh[255];
}

__global__ void k_scan_sums(int *tile_sums, int ntiles, int *total_out) {
    __shared__ int sh[1024];
    __shared__ int carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < ntiles; base += 1024) {
        int v = (base + t < ntiles) ? tile_sums[base + t] : 0;
        sh[t] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            int y = (t >= d) ? sh[t - d] : 0;
            __syncthreads();
            sh[t] += y;
            __syncthreads();
        }
        if (base + t < ntiles) tile_sums[base + t] = carry + sh[t] - v;
        __syncthreads();
        if (t == 1023) carry += sh[1023];
        __syncthreads();
    }
    if (t == 0) *total_out = carry;
}

__global__ void k_scan_add(int *out, const int *tile_sums, int n) {
    const int i = blockIdx.x * SCAN_TILE + threadIdx.x;
    const int add = tile_sums[blockIdx.x];
    for (int k = 0; k < 4; ++k) {
        int j = i + k * 256;
        if (j < n) out[j] += add;
    }
}

pc_status scan_excl(Ctx *ctx, const int *in, int *out, int n, hipStream_t s) {
    const int ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if ((size_t)ntiles > ctx->scan_tmp_elems) {
        if (ctx->scan_tmp) dev_free(ctx, ctx->scan_tmp);
        ctx->scan_tmp = nullptr;
        pc_status st = dev_alloc(ctx, (void **)&ctx->scan_tmp, sizeof(int) * (size_t)(ntiles + 1));
        if (st) return st;
        ctx->scan_tmp_elems = ntiles;
    }
    if (n > 0) hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(256), 0, s, in, out, ctx->scan_tmp, n);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, ctx->scan_tmp, ntiles, out + n);
    if (n > 0) hipLaunchKernelGGL(k_scan_add, dim3(ntiles), dim3(256), 0, s, out, ctx->scan_tmp, n);
    PC_HIP(hipGetLastError());
    return PC_OK;
}

// ---------------------------------------------------------------- rest data
// Orthonormal rest frame per triangle: e1 along X1-X0, n the unit normal,
// e2 = n x e1; Dm = [[|X1-X0|, (X2-X0).e1], [0, (X2-X0).e2]], B = Dm^-1,
// A0 = det(Dm)/2.
__global__ void k_rest_tri(int nt, int nv, const int *tri, const double *X, double *Bm, double *A0,
                           int *status) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int v0 = tri[t], v1 = tri[nt + t], v2 = tri[2 * nt + t];
    if (v0 < 0 || v1 < 0 || v2 < 0 || v0 >= nv || v1 >= nv || v2 >= nv || v0 == v1 || v1 == v2 ||
        v0 == v2) {
        atomicOr(status, ST_BADINDEX);
        return;
    }
    const d3 X0 = ld3(X, v0), E1 = ld3(X, v1) - X0, E2 = ld3(X, v2) - X0;
    const double l1 = sqrt(dot(E1, E1));
    d3 n = cross(E1, E2);
    const double ln = sqrt(dot(n, n));
    if (!(l1 > 0.0) || !(ln > 0.0)) {
        atomicOr(status, ST_DEGENERATE);
        return;
    }
    const d3 e1 = (1.0 / l1) * E1;
    n = (1.0 / ln) * n;
    const d3 e2 = cross(n, e1);
    const double d00 = l1, d01 = dot(E2, e1), d11 = dot(E2, e2);
    const double det = d00 * d11;
    if (!(det > 0.0)) {
        atomicOr(status, ST_DEGENERATE);
        return;
    }
    Bm[t] = 1.0 / d00;
    Bm[nt + t] = -d01 / det;
    Bm[2 * nt + t] = 0.0;
    Bm[3 * nt + t] = 1.0 / d11;
    A0[t] = 0.5 * det;
}

// ---------------------------------------------------------------- hinges
// Directed triangle edges bucketed by their lower vertex; code = t << 2 | k.
__global__ void k_edge_count(int nt, const int *tri, int *cnt) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 3 * (int64_t)nt) return;
    const int k = (int)(idx / nt), t = (int)(idx % nt);
    const int p = tri[k * nt + t], q = tri[((k + 1) % 3) * nt + t];
    atomicAdd(&cnt[min(p, q)], 1);
}

__global__ void k_edge_fill(int nt, const int *tri, int *cnt, const int *ptr, int *list) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 3 * (int64_t)nt) return;
    const int k = (int)(idx / nt), t = (int)(idx % nt);
    const int p = tri[k * nt + t], q = tri[((k + 1) % 3) * nt + t];
    const int lo = min(p, q);
    const int slot = atomicSub(&cnt[lo], 1) - 1;
    list[ptr[lo] + slot] = (t << 2) | k;
}

// One wavefront per lower vertex: sort its directed edges by (upper vertex,
// triangle), pair them into hinges.  WRITE = false counts, true writes.
template <bool WRITE>
__global__ void __launch_bounds__(64) k_hinge_rows(int nv, int nt, const int *tri, const int *ptr,
                                                   const int *list, int *hcnt, const int *hptr,
                                                   int *hinge, int nh, int *status) {
    __shared__ unsigned long long key[64];
    const int lo = xcd_remap(blockIdx.x, gridDim.x);
    if (lo >= nv) return;
    const int t = threadIdx.x;
    const int p0 = ptr[lo], n = ptr[lo + 1] - p0;
    if (n > 64) {
        if (t == 0) atomicOr(status, ST_BUCKET_OVERFLOW);
        return;
    }
    unsigned long long kk = ~0ull;
    if (t < n) {
        const int code = list[p0 + t];
        const int tr = code >> 2, k = code & 3;
        const int p = tri[k * nt + tr], q = tri[((k + 1) % 3) * nt + tr];
        const int hi = max(p, q);
        kk = ((unsigned long long)(unsigned)hi << 32) | (unsigned)code;
    }
    key[t] = kk;
    __syncthreads();
    bitonic_lds<64>(key);
    const unsigned long long me = key[t];
    const bool valid = me != ~0ull;
    const unsigned hi = (unsigned)(me >> 32);
    const bool start = valid && (t == 0 || (unsigned)(key[t - 1] >> 32) != hi);
    int run = 0;
    if (start) {
        while (t + run < 64 && key[t + run] != ~0ull && (unsigned)(key[t + run] >> 32) == hi) ++run;
    }
    const bool is_h = start && run == 2;
    if (start && run > 2) atomicOr(status, ST_NONMANIFOLD);
    const int nh_here = wave_sum_int(is_h ? 1 : 0);
    if (!WRITE) {
        if (t == 0) hcnt[lo] = nh_here;
        return;
    }
    const int rank = wave_excl_scan(is_h ? 1 : 0);
    if (!is_h) return;
    // key[t] holds the lower-numbered triangle (codes sort by triangle id)
    const int c1 = (int)(unsigned)key[t], c2 = (int)(unsigned)key[t + 1];
    const int t1 = c1 >> 2, k1 = c1 & 3, t2 = c2 >> 2, k2 = c2 & 3;
    const int a = tri[k1 * nt + t1], b = tri[((k1 + 1) % 3) * nt + t1], c = tri[((k1 + 2) % 3) * nt + t1];
    const int pp = tri[k2 * nt + t2], qq = tri[((k2 + 1) % 3) * nt + t2], d = tri[((k2 + 2) % 3) * nt + t2];
    if (!(pp == b && qq == a) || c == d) atomicOr(status, ST_ORIENT);
    const int h = hptr[lo] + rank;
    hinge[h] = a;
    hinge[nh + h] = b;
    hinge[2 * nh + h] = c;
    hinge[3 * nh + h] = d;
}

// c_h = 3 |e|^2 / (A1 + A2) and the rest angle.
__global__ void k_rest_hinge(int nh, const int *hinge, const double *X, double *coef, double *tbar) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= nh) return;
    d3 x[4];
    for (int k = 0; k < 4; ++k) x[k] = ld3(X, hinge[k * nh + h]);
    const d3 e = x[1] - x[0];
    const d3 N1 = cross(e, x[2] - x[0]), N2 = cross(x[3] - x[0], e);
    const double A1 = 0.5 * sqrt(dot(N1, N1)), A2 = 0.5 * sqrt(dot(N2, N2));
    coef[h] = 3.0 * dot(e, e) / (A1 + A2);
    double th = 0.0;
    d3 g[4];
    if (!hinge_eval(x, th, g)) th = 0.0;
    tbar[h] = th;
}

pc_status topo_build(Ctx *ctx, const pc_mesh *mesh, hipStream_t s) {
    const int nv = ctx->nv, nt = ctx->nt;
    const int TB = 256;
    hipLaunchKernelGGL(k_rest_tri, dim3((nt + TB - 1) / TB), dim3(TB), 0, s, nt, nv, ctx->tri, ctx->tmp,
                       ctx->Bm, ctx->A0, ctx->status);
    // hinges: bucket directed edges by lower vertex
    int *ecnt = ctx->inc_cnt;  // zero on entry, zero again after the fill
    int *eptr = ctx->inc_ptr;
    int *elist = nullptr, *hcnt = nullptr, *hptr = nullptr;
    pc_status st;
    if ((st = dev_alloc(ctx, (void **)&elist, sizeof(int) * 3 * (size_t)nt))) return st;
    if ((st = dev_alloc(ctx, (void **)&hcnt, sizeof(int) * (size_t)nv))) return st;
    if ((st = dev_alloc(ctx, (void **)&hptr, sizeof(int) * (size_t)(nv + 1)))) return st;
    const int64_t ne = 3 * (int64_t)nt;
    hipLaunchKernelGGL(k_edge_count, dim3((ne + TB - 1) / TB), dim3(TB), 0, s, nt, ctx->tri, ecnt);
    if ((st = scan_excl(ctx, ecnt, eptr, nv, s))) return st;
    hipLaunchKernelGGL(k_edge_fill, dim3((ne + TB - 1) / TB), dim3(TB), 0, s, nt, ctx->tri, ecnt, eptr, elist);
    const int nb = ((nv + 7) / 8) * 8;
    hipLaunchKernelGGL(k_hinge_rows<false>, dim3(nb), dim3(64), 0, s, nv, nt, ctx->tri, eptr, elist, hcnt,
                       (const int *)nullptr, (int *)nullptr, 0, ctx->status);
    if ((st = scan_excl(ctx, hcnt, hptr, nv, s))) return st;
    int nh = 0, bits = 0;
    PC_HIP(hipMemcpyAsync(&nh, hptr + nv, sizeof(int), hipMemcpyDeviceToHost, s));
    PC_HIP(hipMemcpyAsync(&bits, ctx->status, sizeof(int), hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
    if (bits) {
        dev_free(ctx, elist); dev_free(ctx, hcnt); dev_free(ctx, hptr);
        if (bits & ST_BUCKET_OVERFLOW) {
            ctx->err = "a vertex is the lower end of more than 64 directed triangle edges";
            return PC_ERR_CAPACITY;
        }
        ctx->err = "mesh rejected (device check bits " + std::to_string(bits) + ")";
        return PC_ERR_MESH;
    }
    ctx->nh = nh;
    if ((st = dev_alloc(ctx, (void **)&ctx->hinge, sizeof(int) * 4 * (size_t)(nh > 0 ? nh : 1)))) return st;
    if ((st = dev_alloc(ctx, (void **)&ctx->hcoef, sizeof(double) * (size_t)(nh > 0 ? nh : 1)))) return st;
    if ((st = dev_alloc(ctx, (void **)&ctx->htbar, sizeof(double) * (size_t)(nh > 0 ? nh : 1)))) return st;
    hipLaunchKernelGGL(k_hinge_rows<true>, dim3(nb), dim3(64), 0, s, nv, nt, ctx->tri, eptr, elist, hcnt,
                       hptr, ctx->hinge, nh, ctx->status);
    if (nh > 0)
        hipLaunchKernelGGL(k_rest_hinge, dim3((nh + TB - 1) / TB), dim3(TB), 0, s, nh, ctx->hinge, ctx->tmp,
                           ctx->hcoef, ctx->htbar);
    PC_HIP(hipGetLastError());
    PC_HIP(hipMemcpyAsync(&bits, ctx->status, sizeof(int), hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
    dev_free(ctx, elist);
    dev_free(ctx, hcnt);
    dev_free(ctx, hptr);
    if (bits) {
        ctx->err = "mesh rejected (device check bits " + std::to_string(bits) + ")";
        return PC_ERR_MESH;
    }
    return PC_OK;
}

// ---------------------------------------------------------------- incidences
// Bucket every corner of every element (3 per triangle, 4 per hinge, 4 per
// contact) at its vertex; codes as in pc_common.h.
__global__ void k_inc_count(int nt, int nh, int nc, const int *tri, const int *hinge, const int *cverts,
                            int *cnt) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntc = 3 * (int64_t)nt, nhc = 4 * (int64_t)nh;
    if (idx < ntc) {
        atomicAdd(&cnt[tri[idx]], 1);
    } else if (idx < ntc + nhc) {
        atomicAdd(&cnt[hinge[idx - ntc]], 1);
    } else if (idx < ntc + nhc + 4 * (int64_t)nc) {
        atomicAdd(&cnt[cverts[idx - ntc - nhc]], 1);
    }
}

__global__ void k_inc_fill(int nt, int nh, int nc, const int *tri, const int *hinge, const int *cverts, int *cnt,
                           const int *ptr, int *inc) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntc = 3 * (int64_t)nt, nhc = 4 * (int64_t)nh;
    int v;
    unsigned code;
    if (idx < ntc) {
        const int k = (int)(idx / nt), t = (int)(idx % nt);
        v = tri[idx];
        code = inc_code(INC_TRI, (unsigned)t, (unsigned)k);
    } else if (idx < ntc + nhc) {
        const int64_t j = idx - ntc;
        const int k = (int)(j / nh), h = (int)(j % nh);
        v = hinge[j];
        code = inc_code(INC_HINGE, (unsigned)h, (unsigned)k);
    } else if (idx < ntc + nhc + 4 * (int64_t)nc) {
        const int64_t j = idx - ntc - nhc;   // contacts are vertex-major: (contact, corner)
        const int e = (int)(j >> 2), k = (int)(j & 3);
        v = cverts[j];
        code = inc_code(INC_CONTACT, (unsigned)e, (unsigned)k);
    } else {
        return;
    }
    const int slot = atomicSub(&cnt[v], 1) - 1;
    inc[ptr[v] + slot] = (int)code;
}

// Validation of a contact set: indices in range, four distinct vertices,
// weights summing to zero, unit normals.
__global__ void k_check_contacts(int nc, int nv, const int *cv, const double *w, const double *n, int *bad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nc) return;
    bool ok = true;
    for (int k = 0; k < 4; ++k) {
        const int a = cv[4 * e + k];
        ok = ok && a >= 0 && a < nv;
        for (int l = 0; l < k; ++l) ok = ok && cv[4 * e + l] != a;
    }
    double s = 0.0, sa = 0.0;
    for (int k = 0; k < 4; ++k) {
        s += w[4 * e + k];
        sa += fabs(w[4 * e + k]);
    }
    ok = ok && isfinite(s) && fabs(s) <= 1e-9 * sa && sa > 0.0;
    const double nn = n[3 * e] * n[3 * e] + n[3 * e + 1] * n[3 * e + 1] + n[3 * e + 2] * n[3 * e + 2];
    ok = ok && fabs(nn - 1.0) <= 1e-6;
    if (!ok) atomicOr(bad, 1);
}

// ---------------------------------------------------------------- element records
// Every element is evaluated once per assembly, one thread per element, into
// SoA planes of FP64 (plane q of element e at rec[q * n + e]):
//   triangle  the three off-diagonal stiffness blocks K_01, K_02, K_12 at x
//             (planes 9 p .. 9 p + 8 for pair p = (0,1), (0,2), (1,2), 3x3
//             row-major; K_lk = K_kl^T), then the forces on corners 0, 1, 2
//             at the force state (planes 27 + 3 k .. 29 + 3 k);
//   hinge     0..11 G = sqrt(2 k_b c_h) grad theta at x (corner-major xyz),
//             12 phi = -sqrt(2 k_b c_h) (theta - theta_bar) at the force
//             state, and with the lookahead force 13..24 G at the force
//             state; the force on corner k is phi G_k (of the force state),
//             the stiffness block (k, l) is G_k G_l^T;
//   contact   0 k_c while the gap at x is below the thickness (else 0),
//             1 k_c (eta - g) at the force state while below it (else 0).
// The force state is x + h v with the lookahead force (rhs_mode 0), else x.
constexpr int TREC = 36;
constexpr int HREC = 13, HREC_LOOK = 25;
constexpr int CREC = 2;

// Membrane stiffness block K_kl (Sec. 2.5, solver Jacobian of Eq. 3):
//   A0 [mu (b_k.b_l) F F^T + mu u_l u_k^T + lam u_k u_l^T + (b_k^T S+ b_l) I],  u_k = F b_k.
__device__ __forceinline__ void tri_block(const double F[3][2], const double Sp[3], const double bk[2],
                                          const double bl[2], double a0, double mu, double lam, double K[9]) {
    double uk[3], ul[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        uk[a] = F[a][0] * bk[0] + F[a][1] * bk[1];
        ul[a] = F[a][0] * bl[0] + F[a][1] * bl[1];
    }
    const double bb = bk[0] * bl[0] + bk[1] * bl[1];
    const double bSb = bk[0] * (Sp[0] * bl[0] + Sp[1] * bl[1]) + bk[1] * (Sp[1] * bl[0] + Sp[2] * bl[1]);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double fft = F[a][0] * F[b][0] + F[a][1] * F[b][1];
            double val = mu * bb * fft + mu * ul[a] * uk[b] + lam * uk[a] * ul[b];
            if (a == b) val += bSb;
            K[3 * a + b] = a0 * val;
        }
}

__global__ void __launch_bounds__(256) k_tri_eval(int nt, const int *tri, const double *Bm, const double *A0,
                                                  const double *x, const double *v, DevParams P, double *rec) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nt) return;
    TriShape sh;
    const double B0 = Bm[e], B1 = Bm[nt + e], B2 = Bm[2 * nt + e], B3 = Bm[3 * nt + e];
    sh.b[1][0] = B0; sh.b[1][1] = B1;
    sh.b[2][0] = B2; sh.b[2][1] = B3;
    sh.b[0][0] = -B0 - B2; sh.b[0][1] = -B1 - B3;
    const double a0 = A0[e];
    d3 xs[3];
    int vid[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        vid[q] = tri[q * nt + e];
        xs[q] = ld3(x, vid[q]);
    }
    double F[3][2], S[3], Sp[3];
    tri_F(xs, sh, F);
    tri_stress(F, P.mu, P.lam, S);
    psd_part(S, Sp);
    const int64_t n = nt;
    const int pk[3] = {0, 0, 1}, pl[3] = {1, 2, 2};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        double K[9];
        tri_block(F, Sp, sh.b[pk[p]], sh.b[pl[p]], a0, P.mu, P.lam, K);
#pragma unroll
        for (int q = 0; q < 9; ++q) rec[(9 * p + q) * n + e] = K[q];
    }
    // forces f_k = -A0 F S beta_k at the force state
    if (P.s_look != 0.0) {
        d3 ys[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) ys[q] = xs[q] + (P.s_look * P.h) * ld3(v, vid[q]);
        tri_F(ys, sh, F);
        tri_stress(F, P.mu, P.lam, S);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double sb0 = S[0] * sh.b[k][0] + S[1] * sh.b[k][1];
        const double sb1 = S[1] * sh.b[k][0] + S[2] * sh.b[k][1];
#pragma unroll
        for (int a = 0; a < 3; ++a) rec[(27 + 3 * k + a) * n + e] = -a0 * (F[a][0] * sb0 + F[a][1] * sb1);
    }
}

__global__ void __launch_bounds__(256) k_hinge_eval(int nh, const int *hinge, const double *hcoef,
                                                    const double *htbar, const double *x, const double *v,
                                                    DevParams P, double *rec) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nh) return;
    const double sc = sqrt(2.0 * P.kb * hcoef[e]), tb = htbar[e];
    d3 xs[4], g[4];
    int vid[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        vid[q] = hinge[q * nh + e];
        xs[q] = ld3(x, vid[q]);
    }
    const int64_t n = nh;
    double th = 0.0;
    const bool ok = hinge_eval(xs, th, g);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        rec[(3 * q) * n + e] = ok ? sc * g[q].x : 0.0;
        rec[(3 * q + 1) * n + e] = ok ? sc * g[q].y : 0.0;
        rec[(3 * q + 2) * n + e] = ok ? sc * g[q].z : 0.0;
    }
    if (P.s_look != 0.0) {
        d3 ys[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) ys[q] = xs[q] + (P.s_look * P.h) * ld3(v, vid[q]);
        double thf = 0.0;
        const bool okf = hinge_eval(ys, thf, g);
        rec[12 * n + e] = okf ? -sc * (thf - tb) : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            rec[(13 + 3 * q) * n + e] = okf ? sc * g[q].x : 0.0;
            rec[(14 + 3 * q) * n + e] = okf ? sc * g[q].y : 0.0;
            rec[(15 + 3 * q) * n + e] = okf ? sc * g[q].z : 0.0;
        }
    } else {
        rec[12 * n + e] = ok ? -sc * (th - tb) : 0.0;
    }
}

__global__ void __launch_bounds__(256) k_contact_eval(int nc, const int *cverts, const double *cw, const double *cn,
                                                      double eta, double kc, const double *x, const double *v,
                                                      DevParams P, double *rec) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nc) return;
    const d3 nrm = mk(cn[3 * e], cn[3 * e + 1], cn[3 * e + 2]);
    double gx = 0.0, gy = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double c = cw[4 * e + q];
        const int vq = cverts[4 * e + q];
        const d3 xq = ld3(x, vq);
        const d3 yq = xq + (P.s_look * P.h) * ld3(v, vq);
        gx += c * dot(nrm, xq);
        gy += c * dot(nrm, yq);
    }
    rec[e] = gx < eta ? kc : 0.0;
    rec[(int64_t)nc + e] = gy < eta ? kc * (eta - gy) : 0.0;
}

struct AsmArgs {
    int nv, nt, nh;
    const int *tri, *hinge, *inc_ptr;
    int *inc;                    // per-row incidence codes; the pattern pass sorts each row in place
    int nc;                      // contacts: vertices (nc x 4), weights (nc x 4), normals (nc x 3)
    const int *cverts;
    const double *cw, *cn;
    const double *Bm, *A0, *mass;
    const double *trec, *hrec, *crec;   // element records of this assembly
    const uint8_t *pinned;
    const double *v;
    DevParams prm;
    int *rowlen, *rowptr, *colidx, *jcol;
    // blocks of each row in the solver layout: rowlen, less the diagonal
    // block when it is zero (D_i = 0 unless the row is free and has a pinned
    // column; the SpMV applies the mass term apart)
    int *rowlen_s;
    int16_t *jdel;
    const int *row_lane, *lane_row, *row_slice, *slice_row0, *slice_vbase, *slot_off;
    const uint8_t *slot_cnt;
    uint8_t *row_state;          // ROW_GROUP, ROW_WIDE, ROW_OVERFLOW or ROW_WIDE_OVERFLOW
    int *wide_rows, *wide_count; // rows of the wide-row pass (list and its length)
    int nslices;
    // per row of the row group pass, from the pattern pass to the value pass:
    // its columns at cols_tmp[3 p0 + i ..] (p0 = inc_ptr[i]; at most 3 n + 1),
    // its (incidence, corner) pairs sorted by column slot then incidence at
    // pairs_tmp[3 p0 ..] (key slot << 7 | m << 2 | l), and their number
    int *cols_tmp;
    int *pairs_tmp;
    int *row_npairs;
    void *jval;
    double *jval_hi;   // FP64 copy (nullptr when the solver copy is FP64)
    double *b, *diag;
    float *dinv;
    float *binv;   // inverse diagonal blocks, 6 per row (xx, xy, xz, yy, yz, zz)
    int *status;
};

// ---------------------------------------------------------------- row groups
// A row is handled by a group of G lanes: G = 16 in the main passes (four
// rows per 64-lane workgroup), G = 64 in the wide-row passes (one row per
// workgroup, larger capacities), for rows with more than RG_NI incidences.
// The group's LDS holds the row's incidence codes (sorted: triangles, hinges,
// contacts, each by index), the vertices of each incidence's element, the
// column candidates (the element neighbours of the row's vertex) and the
// row's distinct columns.
constexpr int RG = 16, RG_ROWS = 4, RG_NI = 32;
constexpr int WIDE_NI = 512;
// Which pass assembles a row: the row group pass, the wide-row pass, or
// neither because the row exceeds the capacities (found by the row group
// pass: more than MAX_COLS columns; by the wide-row pass: more than WIDE_NI
// incidences or MAX_COLS columns).  Such a row gets a zero diagonal block
// and the status word makes every solve refuse the matrix.
enum : uint8_t { ROW_GROUP = 0, ROW_WIDE = 1, ROW_OVERFLOW = 2, ROW_WIDE_OVERFLOW = 3 };

template <int NI>
struct RowGroupLDS {
    unsigned code[NI];
    int4 ev[NI];             // element vertices (w = -1 for triangles)
    int cand[3 * NI];        // column candidates, in no particular order
    uint8_t first[3 * NI];   // candidate p is the first of its value
    int cols[3 * NI + 1];    // distinct columns ascending, diagonal included; the
                             // pattern pass also stages the unsorted codes here
    int ncand;
};

__device__ __forceinline__ int4 element_vertices(const AsmArgs &A, unsigned code) {
    const int e = inc_elem(code);
    const unsigned type = inc_type(code);
    if (type == INC_HINGE)
        return make_int4(A.hinge[e], A.hinge[A.nh + e], A.hinge[2 * A.nh + e], A.hinge[3 * A.nh + e]);
    if (type == INC_CONTACT)
        return make_int4(A.cverts[4 * e], A.cverts[4 * e + 1], A.cverts[4 * e + 2], A.cverts[4 * e + 3]);
    return make_int4(A.tri[e], A.tri[A.nt + e], A.tri[2 * A.nt + e], -1);
}

// Column candidates of one incidence: the other corners of a triangle, the
// opposite wing of a hinge in which the row's vertex is a wing (the edge's
// endpoints already share a triangle with both wings), the other three
// vertices of a contact, appended to the group's list.
template <int NI>
__device__ __forceinline__ void push_candidates(RowGroupLDS<NI> &L, unsigned code, int4 ev) {
    const int k = inc_corner(code);
    const unsigned type = inc_type(code);
    if (type == INC_TRI) {
        const int pos = atomicAdd(&L.ncand, 2);
        L.cand[pos] = k == 0 ? ev.y : (k == 1 ? ev.z : ev.x);
        L.cand[pos + 1] = k == 0 ? ev.z : (k == 1 ? ev.x : ev.y);
    } else if (type == INC_HINGE) {
        if (k >= 2) L.cand[atomicAdd(&L.ncand, 1)] = k == 2 ? ev.w : ev.z;
    } else {
        const int pos = atomicAdd(&L.ncand, 3);
        L.cand[pos] = k == 0 ? ev.y : ev.x;
        L.cand[pos + 1] = k <= 1 ? ev.z : ev.y;
        L.cand[pos + 2] = k <= 2 ? ev.w : ev.z;
    }
}

// Sum over the G lanes of a group (fixed butterfly order; G divides 64).
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
    return v;
}
template <int G>
__device__ __forceinline__ int group_sum_int(int v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
    return v;
}

// Steps shared by both passes, called by every lane of the workgroup (they
// contain its barriers).  `act`: the group works on row i with n incidences
// (n <= NI), whose sorted codes are in L.code.
// 1. element vertices and column candidates of each incidence;
// 2. first occurrence of each candidate value;
// 3. distinct columns ascending with the diagonal, returns their number.
template <int G, int NI>
__device__ __forceinline__ int row_columns_g(RowGroupLDS<NI> &L, const AsmArgs &A, int i, int n, bool act, int t) {
    if (act) {
        if (t == 0) L.ncand = 0;
    }
    __syncthreads();
    if (act) {
        for (int m = t; m < n; m += G) {
            const unsigned code = L.code[m];
            const int4 ev = element_vertices(A, code);
            L.ev[m] = ev;
            push_candidates(L, code, ev);
        }
    }
    __syncthreads();
    const int nc = act ? L.ncand : 0;
    for (int p = t; p < nc; p += G) {
        const int c = L.cand[p];
        bool f = true;
#pragma unroll 4
        for (int q = 0; q < p; ++q) f = f && L.cand[q] != c;
        L.first[p] = f ? 1 : 0;
    }
    __syncthreads();
    int nd = 0, below = 0;
#pragma unroll 4
    for (int p = 0; p < nc; ++p) {
        const int f = L.first[p];
        nd += f;
        below += f && L.cand[p] < i;
    }
    for (int p = t; p < nc; p += G) {
        if (!L.first[p]) continue;
        const int c = L.cand[p];
        int r = 0;
#pragma unroll 4
        for (int q = 0; q < nc; ++q) r += L.first[q] && L.cand[q] < c;
        L.cols[r + (c > i ? 1 : 0)] = c;
    }
    if (act && t == 0) L.cols[below] = i;
    __syncthreads();
    return nd + 1;
}

// Pattern pass of one row: sort its incidence codes (rank sort; codes of a
// row are distinct) and write them back in place, then count its distinct
// columns.  Returns the row length, 0 when n > NI (not handled here).
template <int G, int NI>
__device__ __forceinline__ int row_pattern_g(RowGroupLDS<NI> &L, const AsmArgs &A, int i, bool act, int t,
                                             bool &keep) {
    int p0 = 0, n = 0;
    if (act) {
        p0 = A.inc_ptr[i];
        n = A.inc_ptr[i + 1] - p0;
    }
    const bool fits = act && n <= NI;
    if (fits)
        for (int m = t; m < n; m += G) L.cols[m] = A.inc[p0 + m];
    __syncthreads();
    if (fits)
        for (int m = t; m < n; m += G) {
            const unsigned key = (unsigned)L.cols[m];
            int r = 0;
#pragma unroll 4
            for (int q = 0; q < n; ++q) r += (unsigned)L.cols[q] < key;
            L.code[r] = key;
        }
    __syncthreads();
    if (fits)
        for (int m = t; m < n; m += G) A.inc[p0 + m] = (int)L.code[m];
    const int len = row_columns_g<G, NI>(L, A, i, n, fits, t);
    // does the row keep its diagonal block: free, with a pinned column
    int anyp = 0;
    if (fits)
        for (int q = t; q < len; q += G) {
            const int c = L.cols[q];
            anyp |= (c != i && A.pinned[c]) ? 1 : 0;
        }
    anyp = group_sum_int<G>(anyp);
    keep = fits && anyp > 0 && !A.pinned[i];
    return fits ? len : 0;
}

// Lane-level: rows a group passes on to the wide-row pass, and rows beyond
// every capacity (length 1, reported through the status word).
__device__ __forceinline__ void row_record(const AsmArgs &A, int i, int len, bool keep, bool wide_pass) {
    if (len > MAX_COLS || (len == 0 && wide_pass)) {
        atomicOr(A.status, len > MAX_COLS ? ST_COL_OVERFLOW : ST_INC_OVERFLOW);
        A.rowlen[i] = 1;
        A.rowlen_s[i] = 1;
        A.row_state[i] = wide_pass ? ROW_WIDE_OVERFLOW : ROW_OVERFLOW;
    } else if (len == 0) {
        A.row_state[i] = ROW_WIDE;
        A.wide_rows[atomicAdd(A.wide_count, 1)] = i;
    } else {
        A.rowlen[i] = len;
        A.rowlen_s[i] = keep ? len : len - 1;
        A.row_state[i] = wide_pass ? ROW_WIDE : ROW_GROUP;
    }
}

// For the value pass of a row group row: its columns, and every (incidence
// m, corner l != k) pair grouped by the column slot of corner l's vertex,
// slots ascending and each slot's pairs in incidence order.  Lane t takes
// the slots s = t, t + 16, ...: it counts the pairs of each slot by scanning
// the row's incidences, the counts give each slot's first position, and a
// second scan writes the pairs.  Called by every lane.
__device__ __forceinline__ int slot_pairs(const RowGroupLDS<RG_NI> &L, int n, int c, int q0, int *out, int s) {
    int cnt = 0;
#pragma unroll 4
    for (int m = 0; m < n; ++m) {
        const int4 ev = L.ev[m];
        const int k = inc_corner(L.code[m]);
        const int l = ev.x == c ? 0 : (ev.y == c ? 1 : (ev.z == c ? 2 : (ev.w == c ? 3 : -1)));
        if (l >= 0 && l != k) {
            if (out) out[q0 + cnt] = (s << 7) | (m << 2) | l;
            ++cnt;
        }
    }
    return cnt;
}

__device__ __forceinline__ void row_pairs_g(RowGroupLDS<RG_NI> &L, const AsmArgs &A, int i, int len, bool act,
                                            int t) {
    int p0 = 0, n = 0;
    if (act) {
        p0 = A.inc_ptr[i];
        n = A.inc_ptr[i + 1] - p0;
        for (int s = t; s < len; s += RG) {
            const int c = L.cols[s];
            A.cols_tmp[3 * p0 + i + s] = c;
            L.cand[s] = c == i ? 0 : slot_pairs(L, n, c, 0, nullptr, s);   // pairs per slot
        }
    }
    __syncthreads();
    if (act) {
        for (int s = t; s < len; s += RG) {
            int q0 = 0;
            for (int r = 0; r < s; ++r) q0 += L.cand[r];
            const int c = L.cols[s];
            if (c != i) slot_pairs(L, n, c, q0, A.pairs_tmp + 3 * (int64_t)p0, s);
        }
        if (t == 0) {
            int np = 0;
            for (int r = 0; r < len; ++r) np += L.cand[r];
            A.row_npairs[i] = np;
        }
    }
}

__global__ void __launch_bounds__(64) k_row_pattern(AsmArgs A) {
    __shared__ RowGroupLDS<RG_NI> Ls[RG_ROWS];
    const int g = threadIdx.x / RG, t = threadIdx.x % RG;
    const int i = xcd_remap(blockIdx.x, gridDim.x) * RG_ROWS + g;
    const bool act = i < A.nv;
    bool keep = false;
    const int len = row_pattern_g<RG, RG_NI>(Ls[g], A, i, act, t, keep);
    if (act && t == 0) row_record(A, i, len, keep, false);
    row_pairs_g(Ls[g], A, i, len, act && len > 0 && len <= MAX_COLS, t);
}

// Wide rows: one workgroup per row, a grid-stride loop over the list the
// row group pass made (every workgroup leaves the loop once the list ends).
__global__ void __launch_bounds__(64) k_row_pattern_wide(AsmArgs A) {
    __shared__ RowGroupLDS<WIDE_NI> L;
    const int nw = *A.wide_count;
    for (int idx = blockIdx.x; idx < nw; idx += gridDim.x) {
        const int i = A.wide_rows[idx];
        bool keep = false;
        const int len = row_pattern_g<WAVE, WIDE_NI>(L, A, i, true, threadIdx.x, keep);
        if (threadIdx.x == 0) row_record(A, i, len, keep, true);
        __syncthreads();
    }
}


// Solver layout of one slice (up to 64 consecutive rows of one instance):
// rows ordered by decreasing length (ties by row), lane_row / row_lane give
// the order, slot_cnt[k] = rows with more than k blocks.  Block k of the row
// in lane l of slice s then sits at slice_vbase[s] +
// sum_{k' < k} slot_width(slot_cnt[k']) + l (slice_vbase: exclusive scan of
// slice_psize, the padded block count of each slice).
__global__ void __launch_bounds__(64) k_slice_layout(int nslices, const int *slice_row0, const int *rowlen,
                                                     int *lane_row, int *row_lane, uint8_t *slot_cnt,
                                                     int *slot_off, int *slice_psize) {
    const int s = blockIdx.x;
    if (s >= nslices) return;
    const int t = threadIdx.x;
    const int r0 = slice_row0[s], r1 = slice_row0[s + 1];
    const int row = r0 + t;
    const bool in = row < r1;
    const int len = in ? rowlen[row] : 0;
    const int key = ((WAVE - len) << 8) | t;   // len <= 64
    int rank = 0;
    for (int m = 0; m < WAVE; ++m) rank += (__shfl(key, m, WAVE) < key) ? 1 : 0;
    lane_row[s * WAVE + rank] = in ? row : -1;
    if (in) row_lane[row] = rank;
    int c = 0;
    for (int k = 0; k < MAX_COLS; ++k) {
        unsigned long long bal = __ballot(len > k);
        if (t == k) c = __popcll(bal);
    }
    slot_cnt[s * WAVE + t] = (uint8_t)c;
    slot_off[s * WAVE + t] = wave_excl_scan(slot_width(c));
    const int padded = wave_sum_int(slot_width(c));
    if (t == 0) slice_psize[s] = padded;
}

// A row that overflowed the per-row limits has length 1 (set by the pattern
// pass): store a zero diagonal block so the layout stays consistent.  The
// status word makes every solve refuse the matrix.
template <typename TB>
__device__ void write_overflow_row(const AsmArgs &A, int i) {
    const int s = A.row_slice[i];
    const int64_t seg = A.slice_vbase[s];
    const int w = slot_width((int)A.slot_cnt[s * WAVE]);
    const int lane = A.row_lane[i];
    A.colidx[A.rowptr[i]] = i;
    A.jcol[seg + lane] = i;
    A.jdel[seg + lane] = (int16_t)(i - A.slice_row0[s]);
    const double zero[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    BlockIO<TB>::store((TB *)A.jval + 9 * seg, w, lane, zero);
    if (A.jval_hi) BlockIO<double>::store(A.jval_hi + 9 * seg, w, lane, zero);
    const double mi = A.mass[i];
    for (int a = 0; a < 3; ++a) {
        A.b[3 * i + a] = 0.0;
        A.diag[3 * i + a] = mi;
        A.dinv[3 * i + a] = (float)(1.0 / mi);
    }
    const float im = (float)(1.0 / mi);
    float *bi = A.binv + 6 * (int64_t)i;
    bi[0] = im; bi[1] = 0.0f; bi[2] = 0.0f; bi[3] = im; bi[4] = 0.0f; bi[5] = im;
}

// Inverse of the symmetric 3x3 block [[a, b, c], [b, d, e], [c, e, f]] by its
// adjugate, written as (xx, xy, xz, yy, yz, zz).  A block that is not
// positive definite (impossible for M + c K with K PSD, but guarded) falls
// back to the inverse of its diagonal.
__device__ __forceinline__ void store_block_inverse(float *out, double a, double b, double c, double d, double e,
                                                    double f) {
    const double c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
    const double c11 = a * f - c * c, c12 = b * c - a * e, c22 = a * d - b * b;
    const double det = a * c00 + b * c01 + c * c02;
    if (det > 0.0 && a > 0.0 && c22 > 0.0 && isfinite(det)) {   // leading minors positive
        const double id = 1.0 / det;
        out[0] = (float)(c00 * id); out[1] = (float)(c01 * id); out[2] = (float)(c02 * id);
        out[3] = (float)(c11 * id); out[4] = (float)(c12 * id); out[5] = (float)(c22 * id);
    } else {
        out[0] = (float)(1.0 / a); out[1] = 0.0f; out[2] = 0.0f;
        out[3] = (float)(1.0 / d); out[4] = 0.0f; out[5] = (float)(1.0 / f);
    }
}

// ---------------------------------------------------------------- values
// Stiffness block K_kl of one incidence (the row's vertex is corner k, the
// column's vertex corner l) from the element records, added to acc:
//   triangle  A0 [mu (b_k.b_l) F F^T + mu u_l u_k^T + lam u_k u_l^T + (b_k^T S+ b_l) I],  u = F b
//   hinge     G_k G_l^T
//   contact   kc_act c_k c_l n n^T
__device__ __forceinline__ void add_stiffness(const AsmArgs &A, unsigned code, int l, double acc[9]) {
    const int e = inc_elem(code), k = inc_corner(code);
    const unsigned type = inc_type(code);
    if (type == INC_TRI) {
        // the record holds K_kl for k < l; K_lk = K_kl^T
        const int lo = k < l ? k : l, hi = k < l ? l : k;
        const int p = lo + hi - 1;   // (0,1) -> 0, (0,2) -> 1, (1,2) -> 2
        const int n = A.nt;          // 36 n < 2^31 (checked at pc_create)
        const double *R = A.trec + 9 * p * n + e;
        double K[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) K[q] = R[q * n];
        if (k < l) {
#pragma unroll
            for (int q = 0; q < 9; ++q) acc[q] += K[q];
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) acc[3 * a + b] += K[3 * b + a];
        }
    } else if (type == INC_HINGE) {
        const int n = A.nh;          // 25 n < 2^31 (checked at pc_create)
        const double *Rk = A.hrec + 3 * k * n + e, *Rl = A.hrec + 3 * l * n + e;
        const double gk[3] = {Rk[0], Rk[n], Rk[2 * n]};
        const double gl[3] = {Rl[0], Rl[n], Rl[2 * n]};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) acc[3 * a + b] += gk[a] * gl[b];
    } else {
        // written so that the (l, k) block is the exact transpose of (k, l)
        const double nr[3] = {A.cn[3 * e], A.cn[3 * e + 1], A.cn[3 * e + 2]};
        const double sc = A.crec[e] * (A.cw[4 * e + k] * A.cw[4 * e + l]);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) acc[3 * a + b] += sc * (nr[a] * nr[b]);
    }
}

// Force of one incidence on the row's vertex (corner k) at the force state.
__device__ __forceinline__ void add_force(const AsmArgs &A, unsigned code, double f[3]) {
    const int e = inc_elem(code), k = inc_corner(code);
    const unsigned type = inc_type(code);
    const bool look = A.prm.s_look != 0.0;
    if (type == INC_TRI) {
        const int n = A.nt;
        const double *R = A.trec + (27 + 3 * k) * n + e;
#pragma unroll
        for (int a = 0; a < 3; ++a) f[a] += R[a * n];
    } else if (type == INC_HINGE) {
        const int n = A.nh;
        const double phi = A.hrec[12 * n + e];
        const double *R = A.hrec + (look ? 13 + 3 * k : 3 * k) * n + e;
#pragma unroll
        for (int a = 0; a < 3; ++a) f[a] += phi * R[a * n];
    } else {
        const double m = A.crec[(int64_t)A.nc + e] * A.cw[4 * e + k];
#pragma unroll
        for (int a = 0; a < 3; ++a) f[a] += m * A.cn[3 * e + a];
    }
}

// Block s of row i (column col) into the block-CSR column list and the
// solver layout, in the solver's type and, when kept, in FP64.
// The solver slot of the row's s-th column (dpos: the diagonal's position;
// -1 for a diagonal block the solver layout leaves out).
__device__ __forceinline__ int solver_slot(const AsmArgs &A, int i, int s, int dpos) {
    const bool keep = A.rowlen_s[i] == A.rowlen[i];
    return keep || s < dpos ? s : (s == dpos ? -1 : s - 1);
}

template <typename TB>
__device__ __forceinline__ void store_row_block(const AsmArgs &A, int i, int s, int dpos, int col,
                                                const double blk[9]) {
    A.colidx[A.rowptr[i] + s] = col;
    s = solver_slot(A, i, s, dpos);
    if (s < 0) return;
    const int si = A.row_slice[i];
    const int w = slot_width((int)A.slot_cnt[si * WAVE + s]);
    const int64_t seg = (int64_t)A.slice_vbase[si] + A.slot_off[si * WAVE + s];
    const int lane = A.row_lane[i];
    A.jcol[seg + lane] = col;
    // offset from the slice's first row; meaningful only when it fits (the
    // solver checks every slice before using it)
    A.jdel[seg + lane] = (int16_t)(col - A.slice_row0[si]);
    BlockIO<TB>::store((TB *)A.jval + 9 * seg, w, lane, blk);
    if (A.jval_hi) BlockIO<double>::store(A.jval_hi + 9 * seg, w, lane, blk);
}

// The row's own outputs: the diagonal slot's block D_i = -c sum_{j pinned}
// K_ij (0 for a pinned row), b_i = h (f_i + m_i g - kv K v), diag(A)_i,
// 1 / diag(A)_i and the inverse of the diagonal block A_ii = m_i I - c sum_j
// K_ij (every element's block rows sum to zero).  red: K v, the diagonal of
// sum_{j != i} K_ij, its symmetrised off-diagonal entries; pin: sum_{j
// pinned} K_ij; f: the element forces.
template <typename TB>
__device__ __forceinline__ void write_row_diagonal(const AsmArgs &A, int i, int dslot, bool rowpin,
                                                   const double red[9], const double pin[9], const double f[3]) {
    const DevParams &P = A.prm;
    const double mi = A.mass[i];
    double blk[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) blk[q] = rowpin ? 0.0 : -P.c * pin[q];
    // force: gravity plus the element forces
    const double f0 = mi * P.g[0] + f[0], f1 = mi * P.g[1] + f[1], f2 = mi * P.g[2] + f[2];
    double bi0 = P.h * (f0 - P.kv_coef * red[0]);
    double bi1 = P.h * (f1 - P.kv_coef * red[1]);
    double bi2 = P.h * (f2 - P.kv_coef * red[2]);
    double d0 = mi - P.c * red[3], d1 = mi - P.c * red[4], d2 = mi - P.c * red[5];
    if (rowpin) {
        bi0 = bi1 = bi2 = 0.0;
        d0 = d1 = d2 = mi;
    }
    if (!isfinite(bi0) || !isfinite(bi1) || !isfinite(bi2)) atomicOr(A.status, ST_NONFINITE);
    A.b[3 * i] = bi0; A.b[3 * i + 1] = bi1; A.b[3 * i + 2] = bi2;
    A.diag[3 * i] = d0; A.diag[3 * i + 1] = d1; A.diag[3 * i + 2] = d2;
    A.dinv[3 * i] = (float)(1.0 / d0);
    A.dinv[3 * i + 1] = (float)(1.0 / d1);
    A.dinv[3 * i + 2] = (float)(1.0 / d2);
    const double o01 = rowpin ? 0.0 : -P.c * red[6];
    const double o02 = rowpin ? 0.0 : -P.c * red[7];
    const double o12 = rowpin ? 0.0 : -P.c * red[8];
    store_block_inverse(A.binv + 6 * (int64_t)i, d0, o01, o02, d1, o12, d2);
    store_row_block<TB>(A, i, dslot, dslot, i, blk);
}

// Values of one row.  Lane t of the group owns the column slots s = t, t + G,
// ...; for each it sums, in the row's incidence order, the stiffness blocks
// of every incident element containing the column's vertex (a deterministic
// segmented reduce, no floating-point atomics), and writes c K_ij (zero when
// row or column is pinned).  Row totals (K v, the diagonal of sum_j K_ij, the
// pinned-column sums for D_i, the off-diagonal sums of the diagonal block)
// and the element forces are summed per lane in slot / incidence order and
// then over the group in a fixed butterfly order; the lane holding the
// diagonal slot writes D_i, b_i, diag(A)_i and both preconditioners.
template <typename TB, int G, int NI>
__device__ __forceinline__ void row_values_g(RowGroupLDS<NI> &L, const AsmArgs &A, int i, bool act, int t) {
    int p0 = 0, n = 0;
    if (act) {
        p0 = A.inc_ptr[i];
        n = A.inc_ptr[i + 1] - p0;
        for (int m = t; m < n; m += G) L.code[m] = (unsigned)A.inc[p0 + m];
    }
    __syncthreads();
    const int len = row_columns_g<G, NI>(L, A, i, n, act, t);
    const DevParams &P = A.prm;
    double red[9];   // K v (3), diagonal of sum_j K_ij (3), its symmetrised off-diagonal entries (3)
#pragma unroll
    for (int q = 0; q < 9; ++q) red[q] = 0.0;
    double f[3] = {0.0, 0.0, 0.0};
    int dslot = -1, npin = 0;
    bool rowpin = false;
    if (act) {
        rowpin = A.pinned[i] != 0;
        const d3 vi = ld3(A.v, i);
        int dpos = 0;
        for (int q = 0; q < len; ++q) dpos += L.cols[q] < i ? 1 : 0;
        for (int s = t; s < len; s += G) {
            const int col = L.cols[s];
            if (col == i) {
                dslot = s;
                continue;
            }
            double acc[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) acc[q] = 0.0;
            for (int m = 0; m < n; ++m) {
                const int4 ev = L.ev[m];
                const int l = ev.x == col ? 0 : (ev.y == col ? 1 : (ev.z == col ? 2 : (ev.w == col ? 3 : -1)));
                if (l >= 0) add_stiffness(A, L.code[m], l, acc);
            }
            const bool colpin = A.pinned[col] != 0;
            npin += colpin ? 1 : 0;
            const d3 dvv = ld3(A.v, col) - vi;
            red[0] += acc[0] * dvv.x + acc[1] * dvv.y + acc[2] * dvv.z;
            red[1] += acc[3] * dvv.x + acc[4] * dvv.y + acc[5] * dvv.z;
            red[2] += acc[6] * dvv.x + acc[7] * dvv.y + acc[8] * dvv.z;
            red[3] += acc[0];
            red[4] += acc[4];
            red[5] += acc[8];
            // off-diagonal entries of sum_j K_ij (symmetrised): the diagonal block is
            // A_ii = m_i I - c sum_{j != i} K_ij since every element's block rows sum to zero
            red[6] += 0.5 * (acc[1] + acc[3]);
            red[7] += 0.5 * (acc[2] + acc[6]);
            red[8] += 0.5 * (acc[5] + acc[7]);
            double blk[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) blk[q] = (rowpin || colpin) ? 0.0 : P.c * acc[q];
            store_row_block<TB>(A, i, s, dpos, col, blk);
        }
        for (int m = t; m < n; m += G) add_force(A, L.code[m], f);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) red[q] = group_sum<G>(red[q]);
    npin = group_sum_int<G>(npin);
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] = group_sum<G>(f[a]);
    if (dslot < 0) return;
    // D_i = -c sum_{j pinned} K_ij for a free row, 0 for a pinned row: the
    // blocks of pinned columns, summed in incidence order (rows next to a pin only)
    double pin[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) pin[q] = 0.0;
    if (!rowpin && npin > 0)
        for (int m = 0; m < n; ++m) {
            const unsigned code = L.code[m];
            const int4 ev = L.ev[m];
            const int k = inc_corner(code);
            const int nq = inc_type(code) == INC_TRI ? 3 : 4;
            for (int l = 0; l < nq; ++l) {
                const int vl = l == 0 ? ev.x : (l == 1 ? ev.y : (l == 2 ? ev.z : ev.w));
                if (l != k && A.pinned[vl]) add_stiffness(A, code, l, pin);
            }
        }
    write_row_diagonal<TB>(A, i, dslot, rowpin, red, pin, f);
}

// Value pass of the row group rows, four rows per 64-lane workgroup, 16
// lanes per row (the pattern pass has left each row's columns and its
// (incidence, corner) pairs sorted by column slot).  Lane t of a row owns
// the column slots s = t, t + 16, ...; for each it sums, in incidence order,
// the stiffness blocks of the pairs of that slot (a contiguous range of the
// sorted pairs) from the element records: a deterministic segmented reduce
// with no floating-point atomics.  Row totals and the forces are summed per
// lane, then over the 16 lanes in a fixed butterfly order; the lane holding
// the diagonal slot writes the row's own outputs.
struct RowPairsLDS {
    unsigned code[RG_NI];
    int pair[3 * RG_NI];
    int cols[MAX_COLS];
};

template <typename TB>
__global__ void __launch_bounds__(64) k_row_values(AsmArgs A) {
    __shared__ RowPairsLDS Ls[RG_ROWS];
    const int g = threadIdx.x / RG, t = threadIdx.x % RG;
    const int i = xcd_remap(blockIdx.x, gridDim.x) * RG_ROWS + g;
    const int st = i < A.nv ? (int)A.row_state[i] : -1;
    if (st == ROW_OVERFLOW && t == 0) write_overflow_row<TB>(A, i);
    const bool act = st == ROW_GROUP;
    RowPairsLDS &L = Ls[g];
    int p0 = 0, n = 0, np = 0, len = 0;
    if (act) {
        p0 = A.inc_ptr[i];
        n = A.inc_ptr[i + 1] - p0;
        np = A.row_npairs[i];
        len = A.rowlen[i];
        for (int m = t; m < n; m += RG) L.code[m] = (unsigned)A.inc[p0 + m];
        for (int q = t; q < np; q += RG) L.pair[q] = A.pairs_tmp[3 * p0 + q];
        for (int q = t; q < len; q += RG) L.cols[q] = A.cols_tmp[3 * p0 + i + q];
    }
    __syncthreads();
    const DevParams &P = A.prm;
    double red[9];   // K v (3), diagonal of sum_j K_ij (3), its symmetrised off-diagonal entries (3)
#pragma unroll
    for (int q = 0; q < 9; ++q) red[q] = 0.0;
    double f[3] = {0.0, 0.0, 0.0};
    int dslot = -1, npin = 0;
    bool rowpin = false;
    if (act) {
        rowpin = A.pinned[i] != 0;
        const d3 vi = ld3(A.v, i);
        int dpos = 0;
        for (int q = 0; q < len; ++q) dpos += L.cols[q] < i ? 1 : 0;
        for (int s = t; s < len; s += RG) {
            const int col = L.cols[s];
            if (col == i) {
                dslot = s;
                continue;
            }
            // first pair of slot s (pairs are sorted by slot)
            int lo = 0, hi = np;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((L.pair[mid] >> 7) < s) lo = mid + 1; else hi = mid;
            }
            double acc[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) acc[q] = 0.0;
            for (int q = lo; q < np; ++q) {
                const int key = L.pair[q];
                if ((key >> 7) != s) break;
                add_stiffness(A, L.code[(key >> 2) & 31], key & 3, acc);
            }
            const bool colpin = A.pinned[col] != 0;
            npin += colpin ? 1 : 0;
            const d3 dvv = ld3(A.v, col) - vi;
            red[0] += acc[0] * dvv.x + acc[1] * dvv.y + acc[2] * dvv.z;
            red[1] += acc[3] * dvv.x + acc[4] * dvv.y + acc[5] * dvv.z;
            red[2] += acc[6] * dvv.x + acc[7] * dvv.y + acc[8] * dvv.z;
            red[3] += acc[0];
            red[4] += acc[4];
            red[5] += acc[8];
            red[6] += 0.5 * (acc[1] + acc[3]);
            red[7] += 0.5 * (acc[2] + acc[6]);
            red[8] += 0.5 * (acc[5] + acc[7]);
            double blk[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) blk[q] = (rowpin || colpin) ? 0.0 : P.c * acc[q];
            store_row_block<TB>(A, i, s, dpos, col, blk);
        }
        for (int m = t; m < n; m += RG) add_force(A, L.code[m], f);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) red[q] = group_sum<RG>(red[q]);
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] = group_sum<RG>(f[a]);
    npin = group_sum_int<RG>(npin);
    if (dslot < 0) return;
    // pinned-column sums for D_i, pair by pair in (slot, incidence) order
    // (rows next to a pin only)
    double pin[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) pin[q] = 0.0;
    if (!rowpin && npin > 0)
        for (int q = 0; q < np; ++q) {
            const int key = L.pair[q];
            if (A.pinned[L.cols[key >> 7]]) add_stiffness(A, L.code[(key >> 2) & 31], key & 3, pin);
        }
    write_row_diagonal<TB>(A, i, dslot, rowpin, red, pin, f);
}

template <typename TB>
__global__ void __launch_bounds__(64) k_row_values_wide(AsmArgs A) {
    __shared__ RowGroupLDS<WIDE_NI> L;
    const int nw = *A.wide_count;
    for (int idx = blockIdx.x; idx < nw; idx += gridDim.x) {
        const int i = A.wide_rows[idx];
        const int st = (int)A.row_state[i];
        if (st == ROW_WIDE_OVERFLOW && threadIdx.x == 0) write_overflow_row<TB>(A, i);
        row_values_g<TB, WAVE, WIDE_NI>(L, A, i, st == ROW_WIDE, threadIdx.x);
        __syncthreads();
    }
}

// Export: solver layout -> block-CSR FP64 with the true diagonal block
// A_ii = m_i I + D_i - sum_{j != i} A_ij; optionally D_i.
template <typename TB>
__global__ void __launch_bounds__(64) k_export(int nv, const int *rowptr, const int *colidx, const int *rowlen_s,
                                               const int *row_lane, const int *row_slice, const int *slice_vbase,
                                               const uint8_t *slot_cnt, const void *jval, const double *mass,
                                               const double *vscale, double *out, double *Dout) {
    const int i = blockIdx.x;
    if (i >= nv) return;
    const int t = threadIdx.x;
    const int s = row_slice[i];
    // solver slot t of the slice: width and offset
    const int w = slot_width((int)slot_cnt[s * WAVE + t]);
    const int off = wave_excl_scan(w);
    const int len = rowptr[i + 1] - rowptr[i];
    const bool active = t < len;
    const int col = active ? colidx[rowptr[i] + t] : -1;
    // CSR position t -> solver slot (the diagonal may be left out when zero)
    const unsigned long long dmask = __ballot(col == i);
    const int dpos = dmask ? __ffsll((long long)dmask) - 1 : len;
    const bool keep = rowlen_s[i] == len;
    const int ss = keep || t < dpos ? t : (t == dpos ? -1 : t - 1);
    const int w_ss = __shfl(w, ss < 0 ? 0 : ss, WAVE);
    const int off_ss = __shfl(off, ss < 0 ? 0 : ss, WAVE);
    double blk[9];
    if (active && ss >= 0) {
        // element-wise reads through val_index (the solver reads whole blocks
        // through BlockIO; the two must agree)
        const int64_t seg = (int64_t)slice_vbase[s] + off_ss;
        const int lane = row_lane[i];
        const TB *val = (const TB *)jval + 9 * seg;
#pragma unroll
        for (int q = 0; q < 9; ++q) blk[q] = to_f64(val[val_index<TB>(q, w_ss, lane)]);
        if constexpr (BlockIO<TB>::SCALED) {
#pragma unroll
            for (int q = 0; q < 9; ++q) blk[q] *= vscale[2 * s + 1];
        }
    } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) blk[q] = 0.0;
    }
    const bool isdiag = active && col == i;
    double red[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) red[q] = wave_sum((active && !isdiag) ? blk[q] : 0.0);
    if (!active) return;
    double *o = out + 9 * (int64_t)(rowptr[i] + t);
    if (isdiag) {
        const double mi = mass[i];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            double v = blk[q] - red[q];
            if (q == 0 || q == 4 || q == 8) v += mi;
            o[q] = v;
            if (Dout) Dout[9 * (int64_t)i + q] = blk[q];
        }
    } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) o[q] = blk[q];
    }
}

// ---------------------------------------------------------------- FP16 blocks
// With FP16 storage the value pass writes the FP64 copy only.  The largest
// magnitude over every stored block then fixes a power-of-two scale S with
// max |S a| in [2^13, 2^14) (FP16's largest finite value is 65504, its
// smallest normal 2^-14), and the FP16 copy holds S a rounded to nearest.
// One wavefront per slice walks the slice's slots; lanes past a slot's row
// count hold padding and are skipped.
__global__ void __launch_bounds__(64) k_f16_absmax(int nslices, const int *slice_vbase, const uint8_t *slot_cnt,
                                                   const int *slot_off, const double *hi, double *part) {
    const int si = blockIdx.x;
    if (si >= nslices) return;
    const int lane = threadIdx.x;
    const int my_cnt = (int)slot_cnt[si * WAVE + lane];
    const int nslots = __popcll(__ballot(my_cnt > 0));
    double m = 0.0;
    for (int k = 0; k < nslots; ++k) {
        const int c = __shfl(my_cnt, k, WAVE);
        if (lane < c) {
            const int64_t off = (int64_t)slice_vbase[si] + slot_off[si * WAVE + k];
            double v[9];
            BlockIO<double>::load(hi + 9 * off, slot_width(c), lane, v);
#pragma unroll
            for (int q = 0; q < 9; ++q) m = fmax(m, fabs(v[q]));
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = fmax(m, __shfl_xor(m, d, WAVE));
    if (lane == 0) part[si] = m;
}

// One workgroup per instance: S of the instance's slices [inst_slice0[i],
// inst_slice0[i + 1]) from their maxima (S = 1 for all-zero or non-finite
// blocks; the solver's own checks report the latter), written to each of
// those slices as (S, 1 / S).  Instances are scaled apart, so an instance
// solved in a batch gives the same bits as solved alone.
__global__ void __launch_bounds__(1024) k_f16_scale(const int *inst_slice0, const double *part, double *scale) {
    __shared__ double sh[16];
    const int s0 = inst_slice0[blockIdx.x], s1 = inst_slice0[blockIdx.x + 1];
    double m = 0.0;
    for (int i = s0 + (int)threadIdx.x; i < s1; i += blockDim.x) m = fmax(m, part[i]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = fmax(m, __shfl_xor(m, d, WAVE));
    if (lane_id() == 0) sh[threadIdx.x / WAVE] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / WAVE); ++w) m = fmax(m, sh[w]);
        sh[0] = m;
    }
    __syncthreads();
    m = sh[0];
    double S = 1.0;
    if (m > 0.0 && isfinite(m)) {
        int e = 0;
        (void)frexp(m, &e);                 // m < 2^e
        e = max(-960, min(960, e));
        S = ldexp(1.0, 14 - e);
    }
    for (int i = s0 + (int)threadIdx.x; i < s1; i += blockDim.x) {
        scale[2 * i] = S;
        scale[2 * i + 1] = 1.0 / S;
    }
}

__global__ void __launch_bounds__(64) k_f16_store(int nslices, const int *slice_vbase, const uint8_t *slot_cnt,
                                                  const int *slot_off, const double *hi, const double *scale,
                                                  f16_t *out) {
    const int si = blockIdx.x;
    if (si >= nslices) return;
    const int lane = threadIdx.x;
    const int my_cnt = (int)slot_cnt[si * WAVE + lane];
    const int nslots = __popcll(__ballot(my_cnt > 0));
    const double S = scale[2 * si];
    for (int k = 0; k < nslots; ++k) {
        const int c = __shfl(my_cnt, k, WAVE);
        if (lane < c) {
            const int64_t off = (int64_t)slice_vbase[si] + slot_off[si * WAVE + k];
            double v[9];
            BlockIO<double>::load(hi + 9 * off, slot_width(c), lane, v);
#pragma unroll
            for (int q = 0; q < 9; ++q) v[q] *= S;
            BlockIO<f16_t>::store(out + 9 * off, slot_width(c), lane, v);
        }
    }
}

static size_t dtype_size(pc_dtype d) { return d == PC_F64 ? 8 : (d == PC_F32 ? 4 : 2); }

__global__ void k_clear_bits(int *status, int mask) {
    if (threadIdx.x == 0 && blockIdx.x == 0) status[0] &= ~mask;
}

pc_status check_contacts(Ctx *ctx, int nc, int *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, (int *)ctx->counter, 0, (int64_t)1);
    hipLaunchKernelGGL(k_check_contacts, dim3((nc + 255) / 256), dim3(256), 0, s, nc, ctx->nv, ctx->cverts, ctx->cw,
                       ctx->cn, (int *)ctx->counter);
    PC_HIP(hipGetLastError());
    PC_HIP(hipMemcpyAsync(ctx->status_host, ctx->counter, sizeof(int), hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
    *bad = *ctx->status_host;
    return PC_OK;
}

pc_status assemble_run(Ctx *ctx, const double *x, const double *v, pc_dtype dtype, double *b,
                       double *diag_out, hipStream_t s) {
    const int nv = ctx->nv, nt = ctx->nt, nh = ctx->nh;
    const int TB = 256;
    pc_status st;
    const size_t need = (size_t)ctx->vcap * 9 * dtype_size(dtype);
    if (need > ctx->jval_bytes) {
        if (ctx->jval) dev_free(ctx, ctx->jval);
        ctx->jval = nullptr;
        ctx->jval_bytes = 0;
        if ((st = dev_alloc(ctx, &ctx->jval, need))) return st;
        ctx->jval_bytes = need;
    }
    ctx->dtype = dtype;
    ctx->win_valid = false;
    ctx->last_x = x;
    ctx->last_v = v;
    if (dtype != PC_F64 && ctx->hi_blocks < ctx->vcap) {
        if (ctx->jval_hi) dev_free(ctx, ctx->jval_hi);
        ctx->jval_hi = nullptr;
        ctx->hi_blocks = 0;
        if ((st = dev_alloc(ctx, (void **)&ctx->jval_hi, (size_t)ctx->vcap * 9 * sizeof(double)))) return st;
        ctx->hi_blocks = ctx->vcap;
    }
    ctx->hi_valid = dtype != PC_F64;
    // element records of this assembly (their size depends on the force state and the contact set)
    const bool look = ctx->prm.s_look != 0.0;
    const int nc = ctx->nc;
    struct Need { double **p; size_t *have; size_t n; } recs[3] = {
        {&ctx->trec, &ctx->trec_elems, (size_t)TREC * nt},
        {&ctx->hrec, &ctx->hrec_elems, (size_t)(look ? HREC_LOOK : HREC) * nh},
        {&ctx->crec, &ctx->crec_elems, (size_t)CREC * nc}};
    for (auto &r : recs)
        if (r.n > *r.have) {
            dev_free(ctx, *r.p);
            *r.p = nullptr;
            *r.have = 0;
            if ((st = dev_alloc(ctx, (void **)r.p, sizeof(double) * r.n))) return st;
            *r.have = r.n;
        }
    if (dtype == PC_F16 && ctx->f16_cap < ctx->nslices) {
        dev_free(ctx, ctx->f16_part);
        dev_free(ctx, ctx->f16_scale);
        ctx->f16_part = ctx->f16_scale = nullptr;
        ctx->f16_cap = 0;
        if ((st = dev_alloc(ctx, (void **)&ctx->f16_part, sizeof(double) * (size_t)ctx->nslices))) return st;
        if ((st = dev_alloc(ctx, (void **)&ctx->f16_scale, sizeof(double) * 2 * (size_t)ctx->nslices))) return st;
        ctx->f16_cap = ctx->nslices;
    }
    if (!ctx->row_state) {
        if ((st = dev_alloc(ctx, (void **)&ctx->rowlen_s, sizeof(int) * (size_t)nv))) return st;
        if ((st = dev_alloc(ctx, (void **)&ctx->row_state, (size_t)nv))) return st;
        if ((st = dev_alloc(ctx, (void **)&ctx->wide_rows, sizeof(int) * (size_t)nv))) return st;
        if ((st = dev_alloc(ctx, (void **)&ctx->row_npairs, sizeof(int) * (size_t)nv))) return st;
    }
    // per-row columns and pair lists between the two passes: 3 per incidence (+1 column per row)
    if (ctx->pair_incs < ctx->ninc) {
        dev_free(ctx, ctx->cols_tmp);
        dev_free(ctx, ctx->pairs_tmp);
        ctx->cols_tmp = nullptr;
        ctx->pairs_tmp = nullptr;
        ctx->pair_incs = 0;
        if ((st = dev_alloc(ctx, (void **)&ctx->cols_tmp, sizeof(int) * (3 * (size_t)ctx->ninc + nv)))) return st;
        if ((st = dev_alloc(ctx, (void **)&ctx->pairs_tmp, sizeof(int) * 3 * (size_t)ctx->ninc))) return st;
        ctx->pair_incs = ctx->ninc;
    }
    const int slot_all = ctx->prof.begin(PK_ASM_ALL, s);
    // 1. elements, each evaluated once
    int slot = ctx->prof.begin(PK_ELEMENTS, s);
    hipLaunchKernelGGL(k_tri_eval, dim3((nt + TB - 1) / TB), dim3(TB), 0, s, nt, ctx->tri, ctx->Bm, ctx->A0, x, v,
                       ctx->prm, ctx->trec);
    if (nh > 0)
        hipLaunchKernelGGL(k_hinge_eval, dim3((nh + TB - 1) / TB), dim3(TB), 0, s, nh, ctx->hinge, ctx->hcoef,
                           ctx->htbar, x, v, ctx->prm, ctx->hrec);
    if (nc > 0)
        hipLaunchKernelGGL(k_contact_eval, dim3((nc + TB - 1) / TB), dim3(TB), 0, s, nc, ctx->cverts, ctx->cw,
                           ctx->cn, ctx->ceta, ctx->ckc, x, v, ctx->prm, ctx->crec);
    ctx->prof.end(slot, s);
    // 2. incidence buckets (the row-limit bits describe this assembly only)
    hipLaunchKernelGGL(k_clear_bits, dim3(1), dim3(64), 0, s, ctx->status, ST_INC_OVERFLOW | ST_COL_OVERFLOW);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, (int *)ctx->counter + 1, 0, (int64_t)1);
    const int64_t ni = 3 * (int64_t)nt + 4 * (int64_t)nh + 4 * (int64_t)nc;
    hipLaunchKernelGGL(k_inc_count, dim3((ni + TB - 1) / TB), dim3(TB), 0, s, nt, nh, nc, ctx->tri, ctx->hinge,
                       ctx->cverts, ctx->inc_cnt);
    if ((st = scan_excl(ctx, ctx->inc_cnt, ctx->inc_ptr, nv, s))) return st;
    hipLaunchKernelGGL(k_inc_fill, dim3((ni + TB - 1) / TB), dim3(TB), 0, s, nt, nh, nc, ctx->tri, ctx->hinge,
                       ctx->cverts, ctx->inc_cnt, ctx->inc_ptr, ctx->inc);
    // 3. row patterns: sorted incidences, row lengths, pointers
    AsmArgs a;
    a.nv = nv; a.nt = nt; a.nh = nh;
    a.tri = ctx->tri; a.hinge = ctx->hinge; a.inc_ptr = ctx->inc_ptr; a.inc = ctx->inc;
    a.nc = nc; a.cverts = ctx->cverts; a.cw = ctx->cw; a.cn = ctx->cn;
    a.Bm = ctx->Bm; a.A0 = ctx->A0; a.mass = ctx->mass;
    a.trec = ctx->trec; a.hrec = ctx->hrec; a.crec = ctx->crec;
    a.pinned = ctx->pinned; a.v = v; a.prm = ctx->prm;
    a.rowlen = ctx->rowlen; a.rowlen_s = ctx->rowlen_s; a.rowptr = ctx->rowptr; a.colidx = ctx->colidx; a.jcol = ctx->jcol; a.jdel = ctx->jdel;
    a.row_lane = ctx->row_lane; a.lane_row = ctx->lane_row; a.slot_cnt = ctx->slot_cnt; a.slot_off = ctx->slot_off; a.jval = ctx->jval;
    a.row_slice = ctx->row_slice; a.slice_row0 = ctx->slice_row0; a.slice_vbase = ctx->slice_vbase;
    a.row_state = ctx->row_state; a.wide_rows = ctx->wide_rows; a.wide_count = (int *)ctx->counter + 1;
    a.nslices = ctx->nslices;
    a.cols_tmp = ctx->cols_tmp; a.pairs_tmp = ctx->pairs_tmp; a.row_npairs = ctx->row_npairs;
    a.jval_hi = dtype != PC_F64 ? ctx->jval_hi : nullptr;
    if (dtype == PC_F16) {
        // the value pass writes the FP64 copy; the FP16 copy is converted from it
        a.jval = ctx->jval_hi;
        a.jval_hi = nullptr;
    }
    a.b = b; a.diag = diag_out ? diag_out : ctx->diag; a.dinv = ctx->dinv; a.binv = ctx->binv; a.status = ctx->status;
    // four rows per workgroup; a multiple of 8 workgroups for the XCD mapping
    const int ng = (((nv + RG_ROWS - 1) / RG_ROWS + 7) / 8) * 8;
    const int nwide = 256;   // workgroups of the wide-row passes (grid-stride over the list)
    slot = ctx->prof.begin(PK_ROW_PAT, s);
    hipLaunchKernelGGL(k_row_pattern, dim3(ng), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_row_pattern_wide, dim3(nwide), dim3(64), 0, s, a);
    ctx->prof.end(slot, s);
    if ((st = scan_excl(ctx, ctx->rowlen, ctx->rowptr, nv, s))) return st;
    // 4. solver layout
    hipLaunchKernelGGL(k_slice_layout, dim3(ctx->nslices), dim3(64), 0, s, ctx->nslices, ctx->slice_row0,
                       ctx->rowlen_s, ctx->lane_row, ctx->row_lane, ctx->slot_cnt, ctx->slot_off, ctx->slice_psize);
    if ((st = scan_excl(ctx, ctx->slice_psize, ctx->slice_vbase, ctx->nslices, s))) return st;
    // 5. values
    slot = ctx->prof.begin(PK_ROW_ASM, s);
    switch (dtype) {
        case PC_F64:
            hipLaunchKernelGGL(k_row_values<double>, dim3(ng), dim3(64), 0, s, a);
            hipLaunchKernelGGL(k_row_values_wide<double>, dim3(nwide), dim3(64), 0, s, a);
            break;
        case PC_F32:
            hipLaunchKernelGGL(k_row_values<float>, dim3(ng), dim3(64), 0, s, a);
            hipLaunchKernelGGL(k_row_values_wide<float>, dim3(nwide), dim3(64), 0, s, a);
            break;
        case PC_BF16:
            hipLaunchKernelGGL(k_row_values<bf16_t>, dim3(ng), dim3(64), 0, s, a);
            hipLaunchKernelGGL(k_row_values_wide<bf16_t>, dim3(nwide), dim3(64), 0, s, a);
            break;
        case PC_F16:
            hipLaunchKernelGGL(k_row_values<double>, dim3(ng), dim3(64), 0, s, a);
            hipLaunchKernelGGL(k_row_values_wide<double>, dim3(nwide), dim3(64), 0, s, a);
            hipLaunchKernelGGL(k_f16_absmax, dim3(ctx->nslices), dim3(64), 0, s, ctx->nslices, ctx->slice_vbase,
                               ctx->slot_cnt, ctx->slot_off, ctx->jval_hi, ctx->f16_part);
            hipLaunchKernelGGL(k_f16_scale, dim3(ctx->ninst), dim3(1024), 0, s, ctx->inst_slice0, ctx->f16_part,
                               ctx->f16_scale);
            hipLaunchKernelGGL(k_f16_store, dim3(ctx->nslices), dim3(64), 0, s, ctx->nslices, ctx->slice_vbase,
                               ctx->slot_cnt, ctx->slot_off, ctx->jval_hi, ctx->f16_scale, (f16_t *)ctx->jval);
            break;
    }
    ctx->prof.end(slot, s);
    ctx->prof.end(slot_all, s);
    if (diag_out && diag_out != ctx->diag)
        PC_HIP(hipMemcpyAsync(ctx->diag, diag_out, sizeof(double) * 3 * (size_t)nv, hipMemcpyDeviceToDevice, s));
    PC_HIP(hipGetLastError());
    ctx->assembled = true;
    return PC_OK;
}

pc_status export_blocks(Ctx *ctx, double *vals, double *D, bool solver, hipStream_t s) {
    if (!ctx->assembled) {
        ctx->err = "cloth_export_blocks: nothing assembled";
        return PC_ERR_ARG;
    }
    const pc_dtype dt = solver ? ctx->dtype : PC_F64;
    const void *src = (solver || !ctx->hi_valid) ? ctx->jval : (const void *)ctx->jval_hi;
    switch (dt) {
        case PC_F64:
            hipLaunchKernelGGL(k_export<double>, dim3(ctx->nv), dim3(64), 0, s, ctx->nv, ctx->rowptr, ctx->colidx,
                               ctx->rowlen_s, ctx->row_lane, ctx->row_slice, ctx->slice_vbase, ctx->slot_cnt, src,
                               ctx->mass, ctx->f16_scale, vals, D);
            break;
        case PC_F32:
            hipLaunchKernelGGL(k_export<float>, dim3(ctx->nv), dim3(64), 0, s, ctx->nv, ctx->rowptr, ctx->colidx,
                               ctx->rowlen_s, ctx->row_lane, ctx->row_slice, ctx->slice_vbase, ctx->slot_cnt, src,
                               ctx->mass, ctx->f16_scale, vals, D);
            break;
        case PC_BF16:
            hipLaunchKernelGGL(k_export<bf16_t>, dim3(ctx->nv), dim3(64), 0, s, ctx->nv, ctx->rowptr, ctx->colidx,
                               ctx->rowlen_s, ctx->row_lane, ctx->row_slice, ctx->slice_vbase, ctx->slot_cnt, src,
                               ctx->mass, ctx->f16_scale, vals, D);
            break;
        case PC_F16:
            hipLaunchKernelGGL(k_export<f16_t>, dim3(ctx->nv), dim3(64), 0, s, ctx->nv, ctx->rowptr, ctx->colidx,
                               ctx->rowlen_s, ctx->row_lane, ctx->row_slice, ctx->slice_vbase, ctx->slot_cnt, src,
                               ctx->mass, ctx->f16_scale, vals, D);
            break;
    }
    PC_HIP(hipGetLastError());
    return PC_OK;
}

}  // namespace pc
