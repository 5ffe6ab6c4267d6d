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

// Incidence codes of the per-vertex buckets: element type in bits 30..31
// (triangle, hinge, contact), element index in bits 2..29, corner in 0..1.
// Sorting the codes orders a row's incidences triangles first, then hinges,
// then contacts, each by index.
enum : unsigned { INC_TRI = 0u, INC_HINGE = 1u, INC_CONTACT = 2u };
__host__ __device__ __forceinline__ unsigned inc_code(unsigned type, unsigned e, unsigned k) {
    return (type << 30) | (e << 2) | k;
}
__host__ __device__ __forceinline__ unsigned inc_type(unsigned code) { return code >> 30; }
__host__ __device__ __forceinline__ int inc_elem(unsigned code) { return (int)((code & 0x3fffffffu) >> 2); }
__host__ __device__ __forceinline__ int inc_corner(unsigned code) { return (int)(code & 3u); }
constexpr int MAX_ELEMS = 1 << 28;   // elements of one type the codes can index

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

// Vectors of three FP32 per row stored packed, 12 B per row (the CG search
// direction and the stored preconditioned residual): row i at 3 i.  The
// three loads or stores of a row merge into one 12-byte access.
__device__ __forceinline__ float4 ld3(const float *v, int64_t i) {
    return make_float4(v[3 * i], v[3 * i + 1], v[3 * i + 2], 0.0f);
}
__device__ __forceinline__ void st3(float *v, int64_t i, float a, float b, float c) {
    v[3 * i] = a;
    v[3 * i + 1] = b;
    v[3 * i + 2] = c;
}

// Block value storage types.  bf16 is stored as the upper half of an fp32
// (round to nearest even on the way in).  f16 is IEEE binary16; f16 blocks
// are stored multiplied by a power-of-two scale chosen at each assembly
// (BlockIO<f16_t>::SCALED), which the SpMV divides out of its row sums.
struct bf16_t {
    uint16_t bits;
};
struct f16_t {
    uint16_t bits;
};

__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(float v) { return (double)v; }
__device__ __forceinline__ double to_f64(bf16_t v) {
    return (double)__uint_as_float(((unsigned)v.bits) << 16);
}
__device__ __forceinline__ float f16_to_f32(unsigned bits) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)bits);
}
__device__ __forceinline__ double to_f64(f16_t v) { return (double)f16_to_f32(v.bits); }

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
// FP64 -> FP32 -> FP16, each step rounding to nearest even (values beyond
// the FP16 range become infinities, which the scale choice rules out)
template <> __device__ __forceinline__ f16_t from_f64<f16_t>(double v) {
    return f16_t{__builtin_bit_cast(uint16_t, (_Float16)(float)v)};
}

// ---------------------------------------------------------------- solver block storage
// Slot k of a 64-row slice (the k-th block of every row with more than k
// blocks, c rows) is stored for w = slot_width(c) lanes, a multiple of 8, so
// that every slot starts 16-byte aligned (its first block has index voff, a
// multiple of 8, and its values start at element 9 voff).  Inside the slot
// the first 8 values of each block are 16-byte chunks (CE = 16 / sizeof(TB)
// values per chunk; chunk plane q holds values CE q .. CE q + CE - 1 of every
// lane) and value 8 has a plane of its own:
//   value e < 8 of lane l at  q w CE + l CE + e % CE   (q = e / CE),
//   value 8       of lane l at  8 w + l.
__host__ __device__ __forceinline__ int slot_width(int c) { return (c + 7) & ~7; }

template <typename TB>
__device__ __forceinline__ int64_t val_index(int e, int w, int l) {
    constexpr int CE = 16 / (int)sizeof(TB);
    return e < 8 ? (int64_t)(e / CE) * w * CE + (int64_t)l * CE + (e % CE) : 8 * (int64_t)w + l;
}

// Whole-block load / store of lane l in a slot of width w whose values start
// at seg (16-byte aligned): vector accesses of the chunks, one scalar access
// for value 8.  R is the register type the loads convert to.
template <typename TB> struct BlockIO;

template <> struct BlockIO<float> {
    typedef float R;
    static constexpr bool SCALED = false;
    __device__ __forceinline__ static void load(const float *seg, int w, int l, float v[9]) {
        const float4 a = reinterpret_cast<const float4 *>(seg)[l];
        const float4 b = reinterpret_cast<const float4 *>(seg + 4 * (int64_t)w)[l];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        v[8] = seg[8 * (int64_t)w + l];
    }
    __device__ __forceinline__ static void store(float *seg, int w, int l, const double b[9]) {
        reinterpret_cast<float4 *>(seg)[l] = make_float4((float)b[0], (float)b[1], (float)b[2], (float)b[3]);
        reinterpret_cast<float4 *>(seg + 4 * (int64_t)w)[l] =
            make_float4((float)b[4], (float)b[5], (float)b[6], (float)b[7]);
        seg[8 * (int64_t)w + l] = (float)b[8];
    }
};

template <> struct BlockIO<bf16_t> {
    typedef float R;
    static constexpr bool SCALED = false;
    __device__ __forceinline__ static void load(const bf16_t *seg, int w, int l, float v[9]) {
        const uint4 a = reinterpret_cast<const uint4 *>(seg)[l];
        v[0] = __uint_as_float(a.x << 16); v[1] = __uint_as_float(a.x & 0xffff0000u);
        v[2] = __uint_as_float(a.y << 16); v[3] = __uint_as_float(a.y & 0xffff0000u);
        v[4] = __uint_as_float(a.z << 16); v[5] = __uint_as_float(a.z & 0xffff0000u);
        v[6] = __uint_as_float(a.w << 16); v[7] = __uint_as_float(a.w & 0xffff0000u);
        v[8] = __uint_as_float(((unsigned)seg[8 * (int64_t)w + l].bits) << 16);
    }
    __device__ __forceinline__ static void store(bf16_t *seg, int w, int l, const double b[9]) {
        unsigned u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            u[q] = (unsigned)from_f64<bf16_t>(b[2 * q]).bits | ((unsigned)from_f64<bf16_t>(b[2 * q + 1]).bits << 16);
        reinterpret_cast<uint4 *>(seg)[l] = make_uint4(u[0], u[1], u[2], u[3]);
        seg[8 * (int64_t)w + l] = from_f64<bf16_t>(b[8]);
    }
};

template <> struct BlockIO<f16_t> {
    typedef float R;
    static constexpr bool SCALED = true;
    __device__ __forceinline__ static void load(const f16_t *seg, int w, int l, float v[9]) {
        const uint4 a = reinterpret_cast<const uint4 *>(seg)[l];
        v[0] = f16_to_f32(a.x & 0xffffu); v[1] = f16_to_f32(a.x >> 16);
        v[2] = f16_to_f32(a.y & 0xffffu); v[3] = f16_to_f32(a.y >> 16);
        v[4] = f16_to_f32(a.z & 0xffffu); v[5] = f16_to_f32(a.z >> 16);
        v[6] = f16_to_f32(a.w & 0xffffu); v[7] = f16_to_f32(a.w >> 16);
        v[8] = f16_to_f32(seg[8 * (int64_t)w + l].bits);
    }
    // b: values already multiplied by the scale
    __device__ __forceinline__ static void store(f16_t *seg, int w, int l, const double b[9]) {
        unsigned u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            u[q] = (unsigned)from_f64<f16_t>(b[2 * q]).bits | ((unsigned)from_f64<f16_t>(b[2 * q + 1]).bits << 16);
        reinterpret_cast<uint4 *>(seg)[l] = make_uint4(u[0], u[1], u[2], u[3]);
        seg[8 * (int64_t)w + l] = from_f64<f16_t>(b[8]);
    }
};

template <> struct BlockIO<double> {
    typedef double R;
    static constexpr bool SCALED = false;
    __device__ __forceinline__ static void load(const double *seg, int w, int l, double v[9]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 a = reinterpret_cast<const double2 *>(seg + 2 * (int64_t)q * w)[l];
            v[2 * q] = a.x;
            v[2 * q + 1] = a.y;
        }
        v[8] = seg[8 * (int64_t)w + l];
    }
    __device__ __forceinline__ static void store(double *seg, int w, int l, const double b[9]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            reinterpret_cast<double2 *>(seg + 2 * (int64_t)q * w)[l] = make_double2(b[2 * q], b[2 * q + 1]);
        seg[8 * (int64_t)w + l] = b[8];
    }
};

}  // namespace pc
