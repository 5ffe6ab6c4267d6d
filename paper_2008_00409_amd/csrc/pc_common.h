// Shared device helpers of the HIP library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pc {

constexpr int WAVE = 64;
constexpr int MAX_INC = 64;    // incident element corners per vertex
constexpr int MAX_COLS = 64;   // distinct block columns per row
constexpr unsigned NONE = 0xFFFFFFFFu;

// Device-side error bits (atomicOr into the context's status word).
enum : int {
    ST_INC_OVERFLOW = 1,
    ST_COL_OVERFLOW = 2,
    ST_NONMANIFOLD = 4,
    ST_ORIENT = 8,
    ST_DEGENERATE = 16,
    ST_NONFINITE = 32,
    ST_BADINDEX = 64,
    ST_BUCKET_OVERFLOW = 128,
};

struct DevParams {
    double h, mu, lam, kb, beta;
    double g[3];
    double c;        // h (h + beta): scale of K in A
    double s_look;   // 1: force at x + h v (Eq. 3), 0: force at x
    double kv_coef;  // coefficient of K v in b / h
};

// Workgroups are dispatched round-robin over the 8 XCDs; map workgroup b to
// a logical index so that each XCD works on one contiguous range (neighbouring
// rows share gathers through that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    const int per = (nblocks + 7) >> 3;
    const int logical = (b & 7) * per + (b >> 3);
    return logical;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
    return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
    return v;
}

__device__ __forceinline__ int wave_excl_scan(int v) {
    const int lane = lane_id();
    int x = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int y = __shfl_up(x, d, WAVE);
        if (lane >= d) x += y;
    }
    return x - v;
}

// Bitonic sort of N keys held in LDS by one 64-lane workgroup (ascending).
// The caller must have synchronised after writing `keys`.
template <int N, typename K>
__device__ __forceinline__ void bitonic_lds(K *keys) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int p = t; p < N / 2; p += WAVE) {
                const int i = (p / j) * 2 * j + (p % j);
                const int q = i + j;
                K a = keys[i], b = keys[q];
                const bool up = (i & k) == 0;
                if ((a > b) == up) {
                    keys[i] = b;
                    keys[q] = a;
                }
            }
            __syncthreads();
        }
    }
}

// Block value storage types.  bf16 is stored as the upper half of an fp32
// (round to nearest even on the way in).
struct bf16_t {
    uint16_t bits;
};

__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(float v) { return (double)v; }
__device__ __forceinline__ double to_f64(bf16_t v) {
    return (double)__uint_as_float(((unsigned)v.bits) << 16);
}

template <typename T> __device__ __forceinline__ T from_f64(double v);
template <> __device__ __forceinline__ double from_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_f64<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ bf16_t from_f64<bf16_t>(double v) {
    float f = (float)v;
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) {  // inf / nan pass through
        bf16_t r{(uint16_t)(u >> 16)};
        if (u & 0x007fffffu) r.bits |= 0x40;
        return r;
    }
    unsigned rounding = 0x7fffu + ((u >> 16) & 1u);
    return bf16_t{(uint16_t)((u + rounding) >> 16)};
}

}  // namespace pc
