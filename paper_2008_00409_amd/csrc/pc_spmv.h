// The CG's block SpMV: the solver layout's row loop, the work schedule it
// runs on, the per-item partial sums, and the kernel q = A p with partials
// of p.q (difference form, see pcg.hip).  Kept apart from the rest of the
// solver so that hardware-counter figures of this kernel can be tied to
// exactly this code.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "pc_ctx.h"

namespace pc {

struct SpmvArgs {
    int nv, nslices;
    const int *rowptr;
    const int *slice_vbase;
    const int *slice_row0;
    const uint8_t *slot_cnt;
    const int *lane_row;
    const int *jcol;
    const int16_t *jdel;   // block columns as offsets from the slice's first row
    const void *jval;
    const double *mass;
    // f16 blocks: per slice, the storage scale S of its instance and 1 / S
    // (vscale[2 s], vscale[2 s + 1]); unused for the other types
    const double *vscale;
};

// Tuning knobs of the SpMV row loop (compile time):
//   PC_SPMV_UNROLL  slots whose loads are issued together
//   PC_SPMV_PIPE    1: the loads of the next group of slots are issued
//                   before the arithmetic of the current group
#ifndef PC_SPMV_UNROLL
#define PC_SPMV_UNROLL 2
#endif
#ifndef PC_SPMV_PIPE
#define PC_SPMV_PIPE 1
#endif

// the FP32 search direction, packed (ld3)
struct VecF3 {
    const float *p;
    template <typename T>
    __device__ __forceinline__ void load(int i, T &a, T &b, T &c) const {
        const float4 v = ld3(p, i);
        a = v.x; b = v.y; c = v.z;
    }
};
// p staged in LDS: the window [lo, lo + n) of rows that the work item's
// columns span (see k_item_windows).
struct VecLds {
    const float4 *w;
    int lo;
    template <typename T>
    __device__ __forceinline__ void load(int i, T &a, T &b, T &c) const {
        const float4 v = w[i - lo];
        a = v.x; b = v.y; c = v.z;
    }
};
struct VecD3 {
    const double *p;
    template <typename T>
    __device__ __forceinline__ void load(int i, T &a, T &b, T &c) const {
        a = p[3 * i]; b = p[3 * i + 1]; c = p[3 * i + 2];
    }
};

// Arithmetic type of the row sums: FP64, except for BF16 and FP16 blocks
// applied to the FP32 search direction, whose products and differences are
// taken in FP32 (the stored values carry 8 or 11 significant bits; FP32
// rounding adds about 6e-8 of the row's terms, the blocks' own rounding 4e-3
// or 5e-4; differences of two FP32 values within a factor 2 of each other are
// exact).  The mass term is always FP64.
template <typename TB> struct SpmvAcc { typedef double T; };
template <> struct SpmvAcc<bf16_t> { typedef float T; };
template <> struct SpmvAcc<f16_t> { typedef float T; };

// One row of the difference-form product for the lane's row of `slice`.
// Lane k of the wavefront holds slot k's row count and start offset, so the
// per-slot values are read with readlane instead of memory loads; slots are
// processed UNROLL at a time with all column-index and value loads of the
// group issued before the gathers of x, to keep several loads in flight.
// The loop body is branch-free so that the compiler can keep every load of
// a group in flight: lanes past a slot's row count (and slots past the
// row's last) load a valid neighbouring element and their contribution is
// masked afterwards; the diagonal slot gathers x_i itself.  Each block is
// read with 16-byte loads (BlockIO).
// NARROW: columns come from the 16-bit offsets jdel (added to the slice's
// first row r0) instead of the 32-bit jcol.
template <typename TB, int UNROLL, bool NARROW>
struct SlotGroup {
    typedef typename BlockIO<TB>::R R;
    int jc[UNROLL];
    R v[UNROLL][9];
    bool act[UNROLL];

    __device__ __forceinline__ void load(const SpmvArgs &M, int k, int nslots, int lane, int my_cnt, int my_off,
                                         int r0) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int kk = min(k + u, nslots - 1);
            const int c = __builtin_amdgcn_readlane(my_cnt, kk);   // >= 1 since kk < nslots
            const int off = __builtin_amdgcn_readlane(my_off, kk);
            act[u] = (k + u < nslots) && lane < c;
            const int l = min(lane, c - 1);
            if (NARROW)
                jc[u] = r0 + (int)M.jdel[off + l];
            else
                jc[u] = M.jcol[off + l];
            BlockIO<TB>::load((const TB *)M.jval + 9 * (int64_t)off, slot_width(c), l, v[u]);
        }
    }
    template <typename V, typename A>
    __device__ __forceinline__ void apply(const V &x, int row, A x0, A x1, A x2, A &a0, A &a1, A &a2) const {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            A d0, d1, d2;
            x.load(jc[u], d0, d1, d2);
            const bool off_diag = jc[u] != row;
            d0 -= off_diag ? x0 : A(0);
            d1 -= off_diag ? x1 : A(0);
            d2 -= off_diag ? x2 : A(0);
            d0 = act[u] ? d0 : A(0);
            d1 = act[u] ? d1 : A(0);
            d2 = act[u] ? d2 : A(0);
            a0 += (A)v[u][0] * d0 + (A)v[u][1] * d1 + (A)v[u][2] * d2;
            a1 += (A)v[u][3] * d0 + (A)v[u][4] * d1 + (A)v[u][5] * d2;
            a2 += (A)v[u][6] * d0 + (A)v[u][7] * d1 + (A)v[u][8] * d2;
        }
    }
};

template <typename TB, typename V, bool NARROW = false, int UNROLL = PC_SPMV_UNROLL>
__device__ __forceinline__ int spmv_row(const SpmvArgs &M, int slice, int lane, const V &x, double y[3],
                                        double xi[3]) {
    const int row = M.lane_row[slice * WAVE + lane];
    const int my_cnt = (int)M.slot_cnt[slice * WAVE + lane];
    const int my_off = M.slice_vbase[slice] + wave_excl_scan(slot_width(my_cnt));
    const int r0 = NARROW ? M.slice_row0[slice] : 0;
    const int nslots = __popcll(__ballot(my_cnt > 0));  // counts are non-increasing in the slot
    // FP64 input vectors (residuals, the API's product) keep FP64 sums
    typedef typename std::conditional<std::is_same<V, VecD3>::value, double, typename SpmvAcc<TB>::T>::type A;
    A x0 = 0, x1 = 0, x2 = 0;
    if (row >= 0) x.load(row, x0, x1, x2);
    A a0 = 0, a1 = 0, a2 = 0;
#if PC_SPMV_PIPE
    // a slice may store no block at all (rows whose only block, a zero
    // diagonal, is left out): then there is nothing to prefetch
    if (nslots > 0) {
        SlotGroup<TB, UNROLL, NARROW> cur;
        cur.load(M, 0, nslots, lane, my_cnt, my_off, r0);
        for (int k = 0; k < nslots; k += UNROLL) {
            SlotGroup<TB, UNROLL, NARROW> nxt;
            nxt.load(M, k + UNROLL, nslots, lane, my_cnt, my_off, r0);
            cur.apply(x, row, x0, x1, x2, a0, a1, a2);
            cur = nxt;
        }
    }
#else
    for (int k = 0; k < nslots; k += UNROLL) {
        SlotGroup<TB, UNROLL, NARROW> g;
        g.load(M, k, nslots, lane, my_cnt, my_off, r0);
        g.apply(x, row, x0, x1, x2, a0, a1, a2);
    }
#endif
    if (row >= 0) {
        const double m = M.mass[row];
        double s0 = (double)a0, s1 = (double)a1, s2 = (double)a2;
        if constexpr (BlockIO<TB>::SCALED) {
            const double vi = M.vscale[2 * slice + 1];   // a power of two: exact
            s0 *= vi; s1 *= vi; s2 *= vi;
        }
        y[0] = s0 + m * (double)x0;
        y[1] = s1 + m * (double)x1;
        y[2] = s2 + m * (double)x2;
    } else {
        y[0] = y[1] = y[2] = 0.0;
    }
    xi[0] = x0; xi[1] = x1; xi[2] = x2;
    return row;
}


// Work schedules (built by build_schedule): SpMV items of up to `spb`
// slices, vector items of up to `rpb` rows; items of one instance are
// contiguous (inst_sitem0 / inst_vitem0 give the ranges).
struct Sched {
    int n_sitems, n_vitems, ninst;
    const int4 *sitem;   // inst, first slice, number of slices, -
    const int4 *vitem;   // inst, first row, end row, -
    const int *inst_sitem0, *inst_vitem0;
};

__device__ __forceinline__ int item_of_block(int n) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    return b < n ? b : -1;
}

// ---------------------------------------------------------------- reductions
// Deterministic two-stage sums without device-scope fences: every block of a
// producing kernel writes its NV partial sums for its work item (plain
// stores), and a finalize kernel launched next adds the items of each
// instance in item order; the kernel boundary makes the partials visible.
// partials layout: [q][item].
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double *partials, int item, int nitems) {
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
        partials[(size_t)q * nitems + item] = s;
    }
}

// q = A p (stored as TQ) and per-item partials of p.q.  When the item's column window fits
// in win_cap rows, p[window] is first copied to LDS with coalesced loads and
// the rows gather from there; otherwise they gather from global memory.
template <typename TB, bool NARROW, typename TQ>
__global__ void __launch_bounds__(1024) k_pcg_spmv(SpmvArgs M, Sched S, const float *p, TQ *q,
                                                  const PcgState *st, double *partials, const int2 *win,
                                                  int win_cap) {
    extern __shared__ float4 pwin[];
    const int it = item_of_block(S.n_sitems);
    if (it < 0) return;
    const int4 I = S.sitem[it];
    if (st[I.x].done) return;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const int lane = lane_id();
    int2 W = make_int2(0, -1);
    if (win_cap > 0) W = win[it];
    const int wn = W.y - W.x + 1;
    const bool use_lds = win_cap > 0 && wn > 0 && wn <= win_cap;   // uniform per block
    if (use_lds) {
        for (int k = threadIdx.x; k < wn; k += blockDim.x) pwin[k] = ld3(p, W.x + k);
        __syncthreads();
    }
    double pq = 0.0;
    if (w < I.z) {
        double y[3], xi[3];
        const int row = use_lds ? spmv_row<TB, VecLds, NARROW>(M, I.y + w, lane, VecLds{pwin, W.x}, y, xi)
                                : spmv_row<TB, VecF3, NARROW>(M, I.y + w, lane, VecF3{p}, y, xi);
        if (row >= 0) {
            // q as stored (FP64, or FP32 for the inner vectors of a refinement
            // sweep); p.q with the stored values, which the update uses
            const TQ q0 = (TQ)y[0], q1 = (TQ)y[1], q2 = (TQ)y[2];
            q[3 * row] = q0;
            q[3 * row + 1] = q1;
            q[3 * row + 2] = q2;
            pq = xi[0] * (double)q0 + xi[1] * (double)q1 + xi[2] * (double)q2;
        }
    }
    double v[1] = {pq};
    block_partials<1>(v, partials, it, S.n_sitems);
}

}  // namespace pc
