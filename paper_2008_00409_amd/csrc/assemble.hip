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

// LDS of the pattern pass (incidences, their vertices, column candidates,
// columns) and of the assembly pass, which adds the element data.  The
// pattern kernel declares only the first, so more of its rows fit per CU.
struct RowPatLDS {
    unsigned inc[64];
    int ev[64][4];
    unsigned cand[256];
    int cols[64];
};
struct RowLDS : RowPatLDS {
    double ed[64][14];   // element data of each incidence
    double fk[64][3];    // force on this row's corner of each incidence
};

struct AsmArgs {
    int nv, nt, nh;
    const int *tri, *hinge, *inc_ptr, *inc;
    int nc;                      // contacts: vertices (nc x 4), weights (nc x 4), normals (nc x 3)
    const int *cverts;
    const double *cw, *cn;
    double ceta, ckc;            // thickness, stiffness
    const double *Bm, *A0, *hcoef, *htbar, *mass;
    const uint8_t *pinned;
    const double *x, *v;
    DevParams prm;
    int *rowlen, *rowptr, *colidx, *jcol;
    int16_t *jdel;
    const int *row_lane, *row_slice, *slice_row0, *slice_vbase;
    const uint8_t *slot_cnt;
    void *jval;
    double *jval_hi;   // FP64 copy (nullptr when the solver copy is FP64)
    double *b, *diag;
    float *dinv;
    float *binv;   // inverse diagonal blocks, 6 per row (xx, xy, xz, yy, yz, zz)
    int *status;
};

// Load the row's incidences (sorted) and the vertices of each element.
__device__ __forceinline__ int row_load(RowPatLDS &L, const AsmArgs &A, int i) {
    const int t = threadIdx.x;
    const int p0 = A.inc_ptr[i];
    const int n = A.inc_ptr[i + 1] - p0;
    if (n > MAX_INC) return -1;
    L.inc[t] = t < n ? (unsigned)A.inc[p0 + t] : NONE;
    __syncthreads();
    bitonic_lds<64>(L.inc);
    if (t < n) {
        const unsigned code = L.inc[t];
        const int e = inc_elem(code);
        const unsigned type = inc_type(code);
        if (type == INC_HINGE) {
#pragma unroll
            for (int q = 0; q < 4; ++q) L.ev[t][q] = A.hinge[q * A.nh + e];
        } else if (type == INC_CONTACT) {
#pragma unroll
            for (int q = 0; q < 4; ++q) L.ev[t][q] = A.cverts[4 * e + q];
        } else {
#pragma unroll
            for (int q = 0; q < 3; ++q) L.ev[t][q] = A.tri[q * A.nt + e];
            L.ev[t][3] = -1;
        }
    }
    __syncthreads();
    return n;
}

// Distinct block columns of row i, ascending, diagonal included.  The column
// set is {i} together with the other corners of every incident triangle, the
// opposite wing of every hinge in which i is a wing (edge endpoints of a
// hinge already share a triangle with its wings) and the other three
// vertices of every incident contact.  Each incidence offers up to 3
// candidates (4 slots per lane, 256 in all), sorted and de-duplicated.
// Returns the row length or -1 when it exceeds MAX_COLS; L.cols holds the
// columns.
__device__ __forceinline__ int row_columns(RowPatLDS &L, int i, int n) {
    const int t = threadIdx.x;
    unsigned c[4] = {NONE, NONE, NONE, NONE};
    if (t < n) {
        const unsigned code = L.inc[t];
        const int k = inc_corner(code);
        const unsigned type = inc_type(code);
        if (type == INC_TRI) {
            c[0] = (unsigned)L.ev[t][(k + 1) % 3];
            c[1] = (unsigned)L.ev[t][(k + 2) % 3];
        } else if (type == INC_HINGE) {
            if (k == 2) c[0] = (unsigned)L.ev[t][3];
            if (k == 3) c[0] = (unsigned)L.ev[t][2];
        } else {   // the three corners other than k, in order
            c[0] = (unsigned)L.ev[t][k == 0 ? 1 : 0];
            c[1] = (unsigned)L.ev[t][k <= 1 ? 2 : 1];
            c[2] = (unsigned)L.ev[t][k <= 2 ? 3 : 2];
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) L.cand[4 * t + q] = c[q];
    __syncthreads();
    bitonic_lds<256>(L.cand);
    int u[4], cnt = 0, below = 0;
    const unsigned ui = (unsigned)i;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int idx = 4 * t + q;
        c[q] = L.cand[idx];
        const unsigned prev = idx > 0 ? L.cand[idx - 1] : NONE;
        u[q] = (c[q] != NONE) && (idx == 0 || c[q] != prev);
        cnt += u[q];
        below += (u[q] && c[q] < ui);
    }
    const int pre = wave_excl_scan(cnt);
    const int total = __shfl(pre + cnt, WAVE - 1, WAVE);
    const int dpos = wave_sum_int(below);
    if (total + 1 > MAX_COLS) return -1;
    int o = pre;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (u[q]) {
            L.cols[o + (c[q] > ui ? 1 : 0)] = (int)c[q];
            ++o;
        }
    if (t == 0) L.cols[dpos] = i;
    __syncthreads();
    return total + 1;
}

__global__ void __launch_bounds__(64) k_row_pattern(AsmArgs A) {
    __shared__ RowPatLDS L;
    const int i = xcd_remap(blockIdx.x, gridDim.x);
    if (i >= A.nv) return;
    const int n = row_load(L, A, i);
    if (n < 0) {
        if (threadIdx.x == 0) {
            atomicOr(A.status, ST_INC_OVERFLOW);
            A.rowlen[i] = 1;
        }
        return;
    }
    const int len = row_columns(L, i, n);
    if (threadIdx.x == 0) {
        if (len < 0) atomicOr(A.status, ST_COL_OVERFLOW);
        A.rowlen[i] = len < 0 ? 1 : len;
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
                                                     int *slice_psize) {
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

template <typename TB>
__global__ void __launch_bounds__(64) k_row_assemble(AsmArgs A) {
    __shared__ RowLDS L;
    const int i = xcd_remap(blockIdx.x, gridDim.x);
    if (i >= A.nv) return;
    const int t = threadIdx.x;
    const int n = row_load(L, A, i);
    if (n < 0) {  // reported by the pattern pass; keep the layout valid
        if (t == 0) write_overflow_row<TB>(A, i);
        return;
    }
    const DevParams &P = A.prm;

    // ---- phase A: lane t evaluates incidence t's element
    if (t < n) {
        const unsigned code = L.inc[t];
        const int e = inc_elem(code);
        const int k = inc_corner(code);
        const unsigned type = inc_type(code);
        if (type == INC_CONTACT) {
            // repulsion element: gap g = n . sum_q c_q x_q, energy kc/2 (eta - g)^2
            // while g < eta; K_kl = kc c_k c_l n n^T (active at x), force on
            // corner k kc (eta - g) c_k n (active at the force state)
            const d3 nrm = mk(A.cn[3 * e], A.cn[3 * e + 1], A.cn[3 * e + 2]);
            double cw[4];
            double gx = 0.0, gy = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                cw[q] = A.cw[4 * e + q];
                const int vq = L.ev[t][q];
                const d3 xq = ld3(A.x, vq);
                const d3 yq = xq + (P.s_look * P.h) * ld3(A.v, vq);
                gx += cw[q] * dot(nrm, xq);
                gy += cw[q] * dot(nrm, yq);
            }
            double *ed = L.ed[t];
            ed[0] = nrm.x; ed[1] = nrm.y; ed[2] = nrm.z;
            ed[3] = cw[0]; ed[4] = cw[1]; ed[5] = cw[2]; ed[6] = cw[3];
            ed[7] = gx < A.ceta ? A.ckc : 0.0;
            const double ck = k == 0 ? cw[0] : (k == 1 ? cw[1] : (k == 2 ? cw[2] : cw[3]));
            const double m = gy < A.ceta ? A.ckc * (A.ceta - gy) * ck : 0.0;
            L.fk[t][0] = m * nrm.x; L.fk[t][1] = m * nrm.y; L.fk[t][2] = m * nrm.z;
        } else if (type == INC_TRI) {
            TriShape sh;
            const double B0 = A.Bm[e], B1 = A.Bm[A.nt + e], B2 = A.Bm[2 * A.nt + e], B3 = A.Bm[3 * A.nt + e];
            sh.b[1][0] = B0; sh.b[1][1] = B1;
            sh.b[2][0] = B2; sh.b[2][1] = B3;
            sh.b[0][0] = -B0 - B2; sh.b[0][1] = -B1 - B3;
            const double a0 = A.A0[e];
            d3 xs[3], ys[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int vq = L.ev[t][q];
                xs[q] = ld3(A.x, vq);
                ys[q] = xs[q] + (P.s_look * P.h) * ld3(A.v, vq);
            }
            double F[3][2], S[3], Sp[3];
            tri_F(xs, sh, F);
            tri_stress(F, P.mu, P.lam, S);
            psd_part(S, Sp);
            double *ed = L.ed[t];
            ed[0] = F[0][0]; ed[1] = F[0][1]; ed[2] = F[1][0]; ed[3] = F[1][1]; ed[4] = F[2][0]; ed[5] = F[2][1];
            ed[6] = Sp[0]; ed[7] = Sp[1]; ed[8] = Sp[2];
            ed[9] = B0; ed[10] = B1; ed[11] = B2; ed[12] = B3; ed[13] = a0;
            // force on corner k at the lookahead state: f_k = -A0 F S beta_k
            double Fy[3][2], Sy[3];
            tri_F(ys, sh, Fy);
            tri_stress(Fy, P.mu, P.lam, Sy);
            // corner k's shape gradient, selected without indexing a private array
            const double bk0 = k == 0 ? sh.b[0][0] : (k == 1 ? sh.b[1][0] : sh.b[2][0]);
            const double bk1 = k == 0 ? sh.b[0][1] : (k == 1 ? sh.b[1][1] : sh.b[2][1]);
            const double sb0 = Sy[0] * bk0 + Sy[1] * bk1;
            const double sb1 = Sy[1] * bk0 + Sy[2] * bk1;
#pragma unroll
            for (int a = 0; a < 3; ++a) L.fk[t][a] = -a0 * (Fy[a][0] * sb0 + Fy[a][1] * sb1);
        } else {
            const double ch = A.hcoef[e], tb = A.htbar[e];
            d3 xs[4], ys[4], g[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int vq = L.ev[t][q];
                xs[q] = ld3(A.x, vq);
                ys[q] = xs[q] + (P.s_look * P.h) * ld3(A.v, vq);
            }
            double th;
            double *ed = L.ed[t];
            if (hinge_eval(xs, th, g)) {
                const double sc = sqrt(2.0 * P.kb * ch);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    ed[3 * q] = sc * g[q].x; ed[3 * q + 1] = sc * g[q].y; ed[3 * q + 2] = sc * g[q].z;
                }
            } else {
#pragma unroll
                for (int q = 0; q < 12; ++q) ed[q] = 0.0;
            }
            if (hinge_eval(ys, th, g)) {
                const double s = -2.0 * P.kb * ch * (th - tb);
                d3 gk = g[0];
#pragma unroll
                for (int q = 1; q < 4; ++q)
                    if (q == k) gk = g[q];
                L.fk[t][0] = s * gk.x; L.fk[t][1] = s * gk.y; L.fk[t][2] = s * gk.z;
            } else {
                L.fk[t][0] = L.fk[t][1] = L.fk[t][2] = 0.0;
            }
        }
    }
    __syncthreads();
    const int len = row_columns(L, i, n);
    if (len < 0) {
        if (t == 0) write_overflow_row<TB>(A, i);
        return;
    }

    // ---- phase B: lane t owns column cols[t]; sum the contributions of all
    // incidences in their sorted order.
    const bool active = t < len;
    const int col = active ? L.cols[t] : i;
    const bool isdiag = active && col == i;
    double acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.0;
    if (active && !isdiag) {
        for (int m = 0; m < n; ++m) {
            const unsigned code = L.inc[m];
            const int k = inc_corner(code);
            const unsigned type = inc_type(code);
            int l = -1;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (L.ev[m][q] == col) l = q;
            if (l < 0) continue;
            const double *ed = L.ed[m];
            if (type == INC_CONTACT) {
                const double ck = ed[3 + k], cl = ed[3 + l];
                const double sc = ed[7] * ck * cl;
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) acc[3 * a + b] += sc * ed[a] * ed[b];
            } else if (type == INC_TRI) {
                // K_kl = A0 [mu (b_k.b_l) F F^T + mu u_l u_k^T + lam u_k u_l^T + (b_k^T S+ b_l) I]
                double bk0, bk1, bl0, bl1;
                const double B0 = ed[9], B1 = ed[10], B2 = ed[11], B3 = ed[12];
                if (k == 0) { bk0 = -B0 - B2; bk1 = -B1 - B3; }
                else if (k == 1) { bk0 = B0; bk1 = B1; }
                else { bk0 = B2; bk1 = B3; }
                if (l == 0) { bl0 = -B0 - B2; bl1 = -B1 - B3; }
                else if (l == 1) { bl0 = B0; bl1 = B1; }
                else { bl0 = B2; bl1 = B3; }
                const double a0 = ed[13];
                const double F00 = ed[0], F01 = ed[1], F10 = ed[2], F11 = ed[3], F20 = ed[4], F21 = ed[5];
                const double uk[3] = {F00 * bk0 + F01 * bk1, F10 * bk0 + F11 * bk1, F20 * bk0 + F21 * bk1};
                const double ul[3] = {F00 * bl0 + F01 * bl1, F10 * bl0 + F11 * bl1, F20 * bl0 + F21 * bl1};
                const double Fr[3][2] = {{F00, F01}, {F10, F11}, {F20, F21}};
                const double bb = bk0 * bl0 + bk1 * bl1;
                const double bSb = bk0 * (ed[6] * bl0 + ed[7] * bl1) + bk1 * (ed[7] * bl0 + ed[8] * bl1);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const double fft = Fr[a][0] * Fr[b][0] + Fr[a][1] * Fr[b][1];
                        double val = P.mu * bb * fft + P.mu * ul[a] * uk[b] + P.lam * uk[a] * ul[b];
                        if (a == b) val += bSb;
                        acc[3 * a + b] += a0 * val;
                    }
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) acc[3 * a + b] += ed[3 * k + a] * ed[3 * l + b];
            }
        }
    }

    // ---- phase C: row totals (fixed butterfly order) and outputs
    const bool rowpin = A.pinned[i] != 0;
    const bool colpin = active && !isdiag && A.pinned[col] != 0;
    const d3 vi = ld3(A.v, i);
    d3 dvv = mk(0.0, 0.0, 0.0);
    if (active && !isdiag) dvv = ld3(A.v, col) - vi;
    double red[18];
    red[0] = acc[0] * dvv.x + acc[1] * dvv.y + acc[2] * dvv.z;
    red[1] = acc[3] * dvv.x + acc[4] * dvv.y + acc[5] * dvv.z;
    red[2] = acc[6] * dvv.x + acc[7] * dvv.y + acc[8] * dvv.z;
    red[3] = acc[0];
    red[4] = acc[4];
    red[5] = acc[8];
#pragma unroll
    for (int q = 0; q < 9; ++q) red[6 + q] = colpin ? acc[q] : 0.0;
    // off-diagonal entries of sum_j K_ij (symmetrised): the diagonal block is
    // A_ii = m_i I - c sum_{j != i} K_ij since every element's block rows sum to zero
    red[15] = 0.5 * (acc[1] + acc[3]);
    red[16] = 0.5 * (acc[2] + acc[6]);
    red[17] = 0.5 * (acc[5] + acc[7]);
#pragma unroll
    for (int q = 0; q < 18; ++q) red[q] = wave_sum(red[q]);

    const double mi = A.mass[i];
    double blk[9];
    if (isdiag) {
        // D_i = -c sum_{j pinned} K_ij for a free row, 0 for a pinned row
#pragma unroll
        for (int q = 0; q < 9; ++q) blk[q] = rowpin ? 0.0 : -P.c * red[6 + q];
        // force: gravity plus element forces in incidence order
        double f0 = mi * P.g[0], f1 = mi * P.g[1], f2 = mi * P.g[2];
        for (int m = 0; m < n; ++m) {
            f0 += L.fk[m][0];
            f1 += L.fk[m][1];
            f2 += L.fk[m][2];
        }
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
        const double o01 = rowpin ? 0.0 : -P.c * red[15];
        const double o02 = rowpin ? 0.0 : -P.c * red[16];
        const double o12 = rowpin ? 0.0 : -P.c * red[17];
        store_block_inverse(A.binv + 6 * (int64_t)i, d0, o01, o02, d1, o12, d2);
    } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) blk[q] = (rowpin || colpin) ? 0.0 : P.c * acc[q];
    }

    // block-CSR pattern and solver layout
    const int s = A.row_slice[i];
    const int w = slot_width((int)A.slot_cnt[s * WAVE + t]);
    const int off = wave_excl_scan(w);
    if (active) {
        A.colidx[A.rowptr[i] + t] = col;
        const int64_t seg = (int64_t)A.slice_vbase[s] + off;
        const int lane = A.row_lane[i];
        A.jcol[seg + lane] = col;
        // offset from the slice's first row; meaningful only when it fits
        // (the solver checks every slice before using it)
        A.jdel[seg + lane] = (int16_t)(col - A.slice_row0[s]);
        BlockIO<TB>::store((TB *)A.jval + 9 * seg, w, lane, blk);
        if (A.jval_hi) BlockIO<double>::store(A.jval_hi + 9 * seg, w, lane, blk);
    }
}

// Export: solver layout -> block-CSR FP64 with the true diagonal block
// A_ii = m_i I + D_i - sum_{j != i} A_ij; optionally D_i.
template <typename TB>
__global__ void __launch_bounds__(64) k_export(int nv, const int *rowptr, const int *row_lane, const int *row_slice,
                                               const int *slice_vbase, const uint8_t *slot_cnt, const int *jcol,
                                               const void *jval, const double *mass, double *out, double *Dout) {
    const int i = blockIdx.x;
    if (i >= nv) return;
    const int t = threadIdx.x;
    const int s = row_slice[i];
    const int w = slot_width((int)slot_cnt[s * WAVE + t]);
    const int off = wave_excl_scan(w);
    const int len = rowptr[i + 1] - rowptr[i];
    const bool active = t < len;
    double blk[9];
    int col = -1;
    if (active) {
        // element-wise reads through val_index (the solver reads whole blocks
        // through BlockIO; the two must agree)
        const int64_t seg = (int64_t)slice_vbase[s] + off;
        const int lane = row_lane[i];
        col = jcol[seg + lane];
        const TB *val = (const TB *)jval + 9 * seg;
#pragma unroll
        for (int q = 0; q < 9; ++q) blk[q] = to_f64(val[val_index<TB>(q, w, lane)]);
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
    // 1. incidence buckets (the row-limit bits describe this assembly only)
    const int slot_all = ctx->prof.begin(PK_ASM_ALL, s);
    hipLaunchKernelGGL(k_clear_bits, dim3(1), dim3(64), 0, s, ctx->status, ST_INC_OVERFLOW | ST_COL_OVERFLOW);
    const int nc = ctx->nc;
    const int64_t ni = 3 * (int64_t)nt + 4 * (int64_t)nh + 4 * (int64_t)nc;
    hipLaunchKernelGGL(k_inc_count, dim3((ni + TB - 1) / TB), dim3(TB), 0, s, nt, nh, nc, ctx->tri, ctx->hinge,
                       ctx->cverts, ctx->inc_cnt);
    if ((st = scan_excl(ctx, ctx->inc_cnt, ctx->inc_ptr, nv, s))) return st;
    hipLaunchKernelGGL(k_inc_fill, dim3((ni + TB - 1) / TB), dim3(TB), 0, s, nt, nh, nc, ctx->tri, ctx->hinge,
                       ctx->cverts, ctx->inc_cnt, ctx->inc_ptr, ctx->inc);
    // 2. row lengths and pointers
    AsmArgs a;
    a.nv = nv; a.nt = nt; a.nh = nh;
    a.tri = ctx->tri; a.hinge = ctx->hinge; a.inc_ptr = ctx->inc_ptr; a.inc = ctx->inc;
    a.nc = nc; a.cverts = ctx->cverts; a.cw = ctx->cw; a.cn = ctx->cn; a.ceta = ctx->ceta; a.ckc = ctx->ckc;
    a.Bm = ctx->Bm; a.A0 = ctx->A0; a.hcoef = ctx->hcoef; a.htbar = ctx->htbar; a.mass = ctx->mass;
    a.pinned = ctx->pinned; a.x = x; a.v = v; a.prm = ctx->prm;
    a.rowlen = ctx->rowlen; a.rowptr = ctx->rowptr; a.colidx = ctx->colidx; a.jcol = ctx->jcol; a.jdel = ctx->jdel;
    a.row_lane = ctx->row_lane; a.slot_cnt = ctx->slot_cnt; a.jval = ctx->jval;
    a.row_slice = ctx->row_slice; a.slice_row0 = ctx->slice_row0; a.slice_vbase = ctx->slice_vbase;
    a.jval_hi = dtype != PC_F64 ? ctx->jval_hi : nullptr;
    a.b = b; a.diag = diag_out ? diag_out : ctx->diag; a.dinv = ctx->dinv; a.binv = ctx->binv; a.status = ctx->status;
    const int nb = ((nv + 7) / 8) * 8;
    int slot = ctx->prof.begin(PK_ROW_PAT, s);
    hipLaunchKernelGGL(k_row_pattern, dim3(nb), dim3(64), 0, s, a);
    ctx->prof.end(slot, s);
    if ((st = scan_excl(ctx, ctx->rowlen, ctx->rowptr, nv, s))) return st;
    // 3. solver layout
    hipLaunchKernelGGL(k_slice_layout, dim3(ctx->nslices), dim3(64), 0, s, ctx->nslices, ctx->slice_row0,
                       ctx->rowlen, ctx->lane_row, ctx->row_lane, ctx->slot_cnt, ctx->slice_psize);
    if ((st = scan_excl(ctx, ctx->slice_psize, ctx->slice_vbase, ctx->nslices, s))) return st;
    // 4. values
    slot = ctx->prof.begin(PK_ROW_ASM, s);
    switch (dtype) {
        case PC_F64: hipLaunchKernelGGL(k_row_assemble<double>, dim3(nb), dim3(64), 0, s, a); break;
        case PC_F32: hipLaunchKernelGGL(k_row_assemble<float>, dim3(nb), dim3(64), 0, s, a); break;
        case PC_BF16: hipLaunchKernelGGL(k_row_assemble<bf16_t>, dim3(nb), dim3(64), 0, s, a); break;
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
            hipLaunchKernelGGL(k_export<double>, dim3(ctx->nv), dim3(64), 0, s, ctx->nv, ctx->rowptr, ctx->row_lane,
                               ctx->row_slice, ctx->slice_vbase, ctx->slot_cnt, ctx->jcol, src, ctx->mass, vals, D);
            break;
        case PC_F32:
            hipLaunchKernelGGL(k_export<float>, dim3(ctx->nv), dim3(64), 0, s, ctx->nv, ctx->rowptr, ctx->row_lane,
                               ctx->row_slice, ctx->slice_vbase, ctx->slot_cnt, ctx->jcol, src, ctx->mass, vals, D);
            break;
        case PC_BF16:
            hipLaunchKernelGGL(k_export<bf16_t>, dim3(ctx->nv), dim3(64), 0, s, ctx->nv, ctx->rowptr, ctx->row_lane,
                               ctx->row_slice, ctx->slice_vbase, ctx->slot_cnt, ctx->jcol, src, ctx->mass, vals, D);
            break;
    }
    PC_HIP(hipGetLastError());
    return PC_OK;
}

}  // namespace pc
