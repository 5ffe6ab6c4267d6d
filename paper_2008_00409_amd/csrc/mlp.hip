// Learned CG warm start: per-vertex features, a 27-64-64-64-3 ReLU MLP on
// BF16 matrix cores (gfx950's v_mfma_f32_16x16x32_bf16, FP32 accumulation), its
// backward pass, split-K weight gradients and Adam.  The prediction is a
// correction to the previous step's velocity increment and starts the CG
// solve of Eq. 3 (paper Sec. 2.5).
//
// Products are arranged as (weights^T) x (activations): a wavefront handles
// 16 vertices, the vertex index is the MFMA's N dimension, so the FP32
// accumulator tile of one layer (lane l: vertex l % 16, features 4 (l / 16) +
// i) is, after bias, ReLU and rounding to BF16, exactly the B operand of the
// next layer.  Padded sizes: input 32 (27 features, 5 zeros), hidden 64,
// output 16 (3 used).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "pc_mlp.h"

namespace pc {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// gfx950's 16 x 16 x 32 product on two K tiles at once: lane l holds rows /
// columns l % 16 and K values 8 (l / 16) .. + 7 of A and B, so two 16 x 16 x 16
// operand pairs (K 4 (l / 16) .. + 3 of tiles 0 and 1) concatenated in the
// same order on both sides give the sum of both tile products (the order of
// the K terms does not change the product).  D has the 16 x 16 x 16 layout.
__device__ __forceinline__ f32x4 mfma32(bf16x4 a0, bf16x4 a1, bf16x4 b0, bf16x4 b1, f32x4 c) {
    const s16x8 a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
    const s16x8 b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

__device__ __forceinline__ short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (short)((u >> 16) | ((u & 0x7fffffu) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf2f(short s) { return __uint_as_float(((unsigned)(unsigned short)s) << 16); }

// Offsets of the padded parameter layout (floats).
constexpr int OFF_W1 = 0;                       // [32][64]
constexpr int OFF_B1 = OFF_W1 + 32 * 64;        // [64]
constexpr int OFF_W2 = OFF_B1 + 64;             // [64][64]
constexpr int OFF_B2 = OFF_W2 + 64 * 64;
constexpr int OFF_W3 = OFF_B2 + 64;             // [64][64]
constexpr int OFF_B3 = OFF_W3 + 64 * 64;
constexpr int OFF_W4 = OFF_B3 + 64;             // [64][16]
constexpr int OFF_B4 = OFF_W4 + 64 * 16;        // [16]
static_assert(OFF_B4 + 16 == MLP_PADDED, "padded parameter count");

// ---------------------------------------------------------------- layout probe
// D = A * B with A[i][k] = i * 16 + k and B = I (then D must equal A), and
// with A = I and B[k][j] = k * 16 + j (then D must equal B): checks the lane
// layout the kernels assume for A, B and D of the 16 x 16 x 16 product.  Then
// the 16 x 16 x 32 product through mfma32 on the tile pairs (A0, A1), (B0,
// B1) with A0[i][k] = 16 i + k, A1[i][k] = 256 - 16 i - k: with B0 = I, B1 =
// 0 it must return A0, with B0 = 0, B1 = I it must return A1 (all values are
// integers of at most 256, exact in BF16).
__global__ void __launch_bounds__(64) k_mfma_probe(float *out) {
    const int l = threadIdx.x;
    for (int t = 0; t < 2; ++t) {
        bf16x4 a, b;
        for (int i = 0; i < 4; ++i) {
            const int row = l % 16, k = 4 * (l / 16) + i;   // A[row][k]
            const int col = l % 16;                          // B[k][col]
            const float av = t == 0 ? (float)(row * 16 + k) : (row == k ? 1.0f : 0.0f);
            const float bv = t == 0 ? (k == col ? 1.0f : 0.0f) : (float)(k * 16 + col);
            a[i] = f2bf(av);
            b[i] = f2bf(bv);
        }
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        c = mfma16(a, b, c);
        for (int i = 0; i < 4; ++i) out[t * 256 + (4 * (l / 16) + i) * 16 + (l % 16)] = c[i];
    }
    for (int t = 0; t < 2; ++t) {
        bf16x4 a0, a1, b0, b1;
        for (int i = 0; i < 4; ++i) {
            const int row = l % 16, k = 4 * (l / 16) + i, col = l % 16;
            a0[i] = f2bf((float)(16 * row + k));
            a1[i] = f2bf((float)(256 - 16 * row - k));
            const float id = k == col ? 1.0f : 0.0f;
            b0[i] = f2bf(t == 0 ? id : 0.0f);
            b1[i] = f2bf(t == 0 ? 0.0f : id);
        }
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        c = mfma32(a0, a1, b0, b1, c);
        for (int i = 0; i < 4; ++i) out[(2 + t) * 256 + (4 * (l / 16) + i) * 16 + (l % 16)] = c[i];
    }
}

// ---------------------------------------------------------------- features
// The 27 features of vertex i (see the oracle's definition), rounded to
// BF16, in a row of 32 (features 27..31 = 0).  Rows nv..nv_pad-1 are zero.
__global__ void k_ws_features(int nv, int nv_pad, const int *rowptr, const int *colidx, const double *x,
                              const double *v, const double *b, const double *diag, const double *mass,
                              const uint8_t *pinned, const double *dvp, double ell, double h, short *X) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv_pad) return;
    float f[32];
    for (int q = 0; q < 32; ++q) f[q] = 0.0f;
    if (i < nv) {
        const double sv = ell / h;
        const double mi = mass[i];
        double sdv[3] = {0, 0, 0}, sbm[3] = {0, 0, 0}, svv[3] = {0, 0, 0}, sx[3] = {0, 0, 0};
        int cnt = 0;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const int j = colidx[p];
            if (j == i) continue;
            ++cnt;
            const double mj = mass[j];
            for (int a = 0; a < 3; ++a) {
                sdv[a] += dvp[3 * j + a];
                sbm[a] += b[3 * j + a] / mj;
                svv[a] += v[3 * j + a];
                sx[a] += x[3 * j + a];
            }
        }
        const double inv = 1.0 / (double)(cnt > 0 ? cnt : 1);
        double dsum = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double bi = b[3 * i + a], bmi = bi / mi;
            f[0 + a] = (float)(v[3 * i + a] / sv);
            f[3 + a] = (float)(bmi / sv);
            f[6 + a] = (float)(dvp[3 * i + a] / sv);
            f[9 + a] = (float)(sdv[a] * inv / sv);
            f[12 + a] = (float)(bi / diag[3 * i + a] / sv);
            f[15 + a] = (float)((sbm[a] * inv - bmi) / sv);
            f[18 + a] = (float)((svv[a] * inv - v[3 * i + a]) / sv);
            f[21 + a] = (float)((sx[a] * inv - x[3 * i + a]) / ell);
            dsum += diag[3 * i + a];
        }
        f[24] = pinned[i] ? 1.0f : 0.0f;
        f[25] = (float)log10(dsum / 3.0 / mi);
        f[26] = (float)(cnt / 12.0);
    }
    for (int q = 0; q < 32; ++q) X[(int64_t)i * 32 + q] = f2bf(f[q]);
}

// ---------------------------------------------------------------- forward
// A-operand tile of W^T (rows: output features m0.., K: input features k0..)
// from the row-major [in][out] BF16 weights.
__device__ __forceinline__ bf16x4 load_wt(const short *W, int out, int m0, int k0) {
    const int l = threadIdx.x & 63;
    bf16x4 a;
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = W[(k0 + 4 * (l / 16) + i) * out + m0 + l % 16];
    return a;
}
// A-operand tile of W (rows: input features m0.., K: output features k0..).
__device__ __forceinline__ bf16x4 load_w(const short *W, int out, int m0, int k0) {
    const int l = threadIdx.x & 63;
    bf16x4 a;
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = W[(m0 + l % 16) * out + k0 + 4 * (l / 16) + i];
    return a;
}
// B-operand / accumulator-layout tile of a vertex-major [v][width] BF16 array.
__device__ __forceinline__ bf16x4 load_act(const short *H, int width, int v0, int f0) {
    const int l = threadIdx.x & 63;
    const short *p = H + (int64_t)(v0 + l % 16) * width + f0 + 4 * (l / 16);
    bf16x4 r;
    r[0] = p[0]; r[1] = p[1]; r[2] = p[2]; r[3] = p[3];
    return r;
}
__device__ __forceinline__ void store_act(short *H, int width, int v0, int f0, bf16x4 r) {
    const int l = threadIdx.x & 63;
    short *p = H + (int64_t)(v0 + l % 16) * width + f0 + 4 * (l / 16);
    p[0] = r[0]; p[1] = r[1]; p[2] = r[2]; p[3] = r[3];
}

// Bias + ReLU + BF16 of an accumulator tile whose rows are features f0..f0+15.
__device__ __forceinline__ bf16x4 act_relu(f32x4 c, const float *bias, int f0) {
    const int l = threadIdx.x & 63;
    bf16x4 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = f2bf(fmaxf(c[i] + bias[f0 + 4 * (l / 16) + i], 0.0f));
    return r;
}

struct FwdArgs {
    int nv, ntiles;
    const short *X;
    const short *Wb;      // BF16 weights, padded layout
    const float *Wf;      // FP32 parameters (biases read from here)
    short *H1, *H2, *H3;  // stored when training (nullptr otherwise)
    const double *dvp;
    const uint8_t *pinned;
    double sv;
    double *dv0;          // start: dv_prev + s_v y (free), 0 (pinned); dvp == nullptr: s_v y
};

// One wavefront per 16-vertex tile, grid-stride over tiles; weights stay in
// registers for all tiles of the wavefront.
__global__ void __launch_bounds__(256) k_mlp_fwd(FwdArgs F) {
    const int l = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int nwaves = gridDim.x * (blockDim.x / 64);
    const short *W1 = F.Wb + OFF_W1, *W2 = F.Wb + OFF_W2, *W3 = F.Wb + OFF_W3, *W4 = F.Wb + OFF_W4;
    bf16x4 A1[4][2], A2[4][4], A3[4][4], A4[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int k = 0; k < 2; ++k) A1[m][k] = load_wt(W1, 64, 16 * m, 16 * k);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            A2[m][k] = load_wt(W2, 64, 16 * m, 16 * k);
            A3[m][k] = load_wt(W3, 64, 16 * m, 16 * k);
        }
        A4[m] = load_wt(W4, 16, 0, 16 * m);
    }
    const float *b1 = F.Wf + OFF_B1, *b2 = F.Wf + OFF_B2, *b3 = F.Wf + OFF_B3, *b4 = F.Wf + OFF_B4;
    for (int t = wave; t < F.ntiles; t += nwaves) {
        const int v0 = 16 * t;
        bf16x4 X0 = load_act(F.X, 32, v0, 0), X1 = load_act(F.X, 32, v0, 16);
        bf16x4 H1[4], H2[4], H3[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            c = mfma32(A1[m][0], A1[m][1], X0, X1, c);
            H1[m] = act_relu(c, b1, 16 * m);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            c = mfma32(A2[m][0], A2[m][1], H1[0], H1[1], c);
            c = mfma32(A2[m][2], A2[m][3], H1[2], H1[3], c);
            H2[m] = act_relu(c, b2, 16 * m);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            c = mfma32(A3[m][0], A3[m][1], H2[0], H2[1], c);
            c = mfma32(A3[m][2], A3[m][3], H2[2], H2[3], c);
            H3[m] = act_relu(c, b3, 16 * m);
        }
        f32x4 y = {0.f, 0.f, 0.f, 0.f};
        y = mfma32(A4[0], A4[1], H3[0], H3[1], y);
        y = mfma32(A4[2], A4[3], H3[2], H3[3], y);
        if (F.H1) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                store_act(F.H1, 64, v0, 16 * m, H1[m]);
                store_act(F.H2, 64, v0, 16 * m, H2[m]);
                store_act(F.H3, 64, v0, 16 * m, H3[m]);
            }
        }
        // lanes 0..15 hold output rows 0..3 of vertex v0 + l
        const int vtx = v0 + l;
        if (l < 16 && vtx < F.nv) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double ya = (double)(y[a] + b4[a]);
                const double base = F.dvp ? F.dvp[3 * vtx + a] : 0.0;
                F.dv0[3 * vtx + a] = F.pinned[vtx] ? 0.0 : base + F.sv * ya;
            }
        }
    }
}

// ---------------------------------------------------------------- backward
// Output gradient g4 = s_v (A dv0 - b) / E0 on free vertices as BF16 rows of
// 16 (components 3..15 and pad rows zero).  Ad = A dv0 (FP64 blocks).
__global__ void k_ws_out_grad(int nv, int nv_pad, const double *Ad, const double *b, const uint8_t *pinned,
                              double sv, const double *E0, short *G4) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv_pad) return;
    float g[3] = {0.f, 0.f, 0.f};
    if (i < nv && !pinned[i]) {
        const double s = sv / E0[0];
        for (int a = 0; a < 3; ++a) g[a] = (float)(s * (Ad[3 * i + a] - b[3 * i + a]));
    }
    for (int q = 0; q < 16; ++q) G4[(int64_t)i * 16 + q] = f2bf(q < 3 ? g[q] : 0.0f);
}

struct BwdArgs {
    int ntiles;
    const short *Wb;
    const short *H1, *H2, *H3, *G4;
    short *G1, *G2, *G3;
};

// G3 = (W4 G4) . [H3 > 0], G2 = (W3 G3) . [H2 > 0], G1 = (W2 G2) . [H1 > 0],
// each rounded to BF16 and stored for the weight gradients.
__global__ void __launch_bounds__(256) k_mlp_bwd(BwdArgs B) {
    const int l = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int nwaves = gridDim.x * (blockDim.x / 64);
    const short *W2 = B.Wb + OFF_W2, *W3 = B.Wb + OFF_W3, *W4 = B.Wb + OFF_W4;
    bf16x4 A4[4], A3[4][4], A2[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        A4[m] = load_w(W4, 16, 16 * m, 0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            A3[m][k] = load_w(W3, 64, 16 * m, 16 * k);
            A2[m][k] = load_w(W2, 64, 16 * m, 16 * k);
        }
    }
    (void)l;
    for (int t = wave; t < B.ntiles; t += nwaves) {
        const int v0 = 16 * t;
        const bf16x4 g4 = load_act(B.G4, 16, v0, 0);
        bf16x4 G3[4], G2[4], G1[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            c = mfma16(A4[m], g4, c);
            const bf16x4 h = load_act(B.H3, 64, v0, 16 * m);
            bf16x4 r;
#pragma unroll
            for (int i = 0; i < 4; ++i) r[i] = f2bf(bf2f(h[i]) > 0.0f ? c[i] : 0.0f);
            G3[m] = r;
            store_act(B.G3, 64, v0, 16 * m, r);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            c = mfma32(A3[m][0], A3[m][1], G3[0], G3[1], c);
            c = mfma32(A3[m][2], A3[m][3], G3[2], G3[3], c);
            const bf16x4 h = load_act(B.H2, 64, v0, 16 * m);
            bf16x4 r;
#pragma unroll
            for (int i = 0; i < 4; ++i) r[i] = f2bf(bf2f(h[i]) > 0.0f ? c[i] : 0.0f);
            G2[m] = r;
            store_act(B.G2, 64, v0, 16 * m, r);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
            c = mfma32(A2[m][0], A2[m][1], G2[0], G2[1], c);
            c = mfma32(A2[m][2], A2[m][3], G2[2], G2[3], c);
            const bf16x4 h = load_act(B.H1, 64, v0, 16 * m);
            bf16x4 r;
#pragma unroll
            for (int i = 0; i < 4; ++i) r[i] = f2bf(bf2f(h[i]) > 0.0f ? c[i] : 0.0f);
            G1[m] = r;
            store_act(B.G1, 64, v0, 16 * m, r);
        }
    }
}

// ---------------------------------------------------------------- weight gradients
// Output tiles of 16 x 16: weight tiles (layer, input block, output block)
// and bias tiles (layer, output block; A operand = a row of ones).
struct GradTile {
    int layer, mb, nb, bias;
};
__constant__ GradTile c_tiles[MLP_GRAD_TILES];

// Split-K over vertex tiles: block b handles tiles [t0, t1) of the vertex
// dimension, 32 vertices (two tiles, the K of one 16 x 16 x 32 product) at a
// time; its 4 wavefronts share the output tiles round-robin.  Registers are
// capped for 3 waves per SIMD (the accumulators then live in VGPRs), and the
// grid is three blocks per CU.  Partial tiles
// go to part[block][tile][16 x 16] (row-major).
//
// A lane's K values are 8 vertices of one feature, 128 bytes apart in the
// vertex-major activations, so each 32-vertex chunk of all eight arrays
// (X, H1..H3, G1..G4: 27 KiB) is first copied to LDS with 16-byte loads, in
// the same vertex-major order.  Every array gets rows of WG_P = 68 values
// (64 + 4 padding, whatever its width): the 2-byte operand reads of the four
// lane groups (rows 4 apart) then fall on distinct banks, and a read's offset
// from its tile's base is a constant.  Vertices past the block's range are
// staged as zeros.
// Arrays k = 0..7: X (32 features), H1, H2, H3, G1, G2, G3 (64), G4 (16).
constexpr int WG_V = 32, WG_P = 68;
__host__ __device__ constexpr int wg_width(int k) { return k == 0 ? 32 : (k == 7 ? 16 : 64); }
__host__ __device__ constexpr int wg_off(int k) { return k * WG_V * WG_P; }
// first 16-byte unit of array k in a chunk
__host__ __device__ constexpr int wg_units(int k) {
    return k == 0 ? 0 : (k <= 7 ? WG_V * 32 / 8 + (k - 1) * WG_V * 64 / 8 : WG_V * (32 + 6 * 64 + 16) / 8);
}
constexpr int WG_LDS = wg_off(8);       // 17,408 values
constexpr int WG_UNITS = wg_units(8);   // 1,728 16-byte units per chunk
static_assert(wg_units(7) + WG_V * wg_width(7) / 8 == WG_UNITS, "unit count");
static_assert(WG_P % 4 == 0, "LDS rows must stay 8-byte aligned");

__global__ void __launch_bounds__(256, 3) k_mlp_wgrad(int ntiles, const short *X, const short *H1, const short *H2,
                                                   const short *H3, const short *G1, const short *G2,
                                                   const short *G3, const short *G4, float *part) {
    __shared__ __align__(16) short L[WG_LDS];
    const int l = threadIdx.x & 63;
    const int w = threadIdx.x / 64;
    const int per = (ntiles + gridDim.x - 1) / gridDim.x;
    const int t0 = blockIdx.x * per, t1 = min(ntiles, t0 + per);
    const short *const src[8] = {X, H1, H2, H3, G1, G2, G3, G4};
    constexpr int MAXT = (MLP_GRAD_TILES + 3) / 4;
    f32x4 acc[MAXT];
#pragma unroll
    for (int q = 0; q < MAXT; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    // this thread's 16-byte units of a chunk: unit u = threadIdx.x + 256 j
    // lies in array j (threads 0..127) or j + 1 (threads 128..255) for
    // j < 6; for j = 6 in G3 (0..127) or G4 (128..191).  The next chunk's
    // units are loaded into registers while the current chunk's products run.
    constexpr int UPT = (WG_UNITS + 255) / 256;
    static_assert(UPT == 7 && WG_UNITS == 6 * 256 + 192, "unit split");
    const bool hi = threadIdx.x >= 128;
    const int uidx = hi ? (int)threadIdx.x - 128 : (int)threadIdx.x + 128;   // unit within its array (k >= 1)
    uint4 pre[UPT];
    auto load_chunk = [&](int t) {
        const int v0 = 16 * t;
        const int nvalid = min(WG_V, 16 * (t1 - t));
#pragma unroll
        for (int j = 0; j < UPT; ++j) {
            const int k = hi ? j + 1 : j;
            const int W = wg_width(k);
            const int e = 8 * (k == 0 ? (int)threadIdx.x : uidx);
            const short *p = hi ? src[j + 1] : src[j];
            pre[j] = make_uint4(0u, 0u, 0u, 0u);
            if ((j < 6 || threadIdx.x < 192) && e / W < nvalid)
                pre[j] = *reinterpret_cast<const uint4 *>(p + (int64_t)v0 * W + e);
        }
    };
    auto store_chunk = [&]() {
#pragma unroll
        for (int j = 0; j < UPT; ++j) {
            if (j == 6 && threadIdx.x >= 192) continue;
            const int k = hi ? j + 1 : j;
            const int W = wg_width(k);
            const int e = 8 * (k == 0 ? (int)threadIdx.x : uidx);
            uint2 *dst = reinterpret_cast<uint2 *>(L + wg_off(k) + (e / W) * WG_P + e % W);
            dst[0] = make_uint2(pre[j].x, pre[j].y);
            dst[1] = make_uint2(pre[j].z, pre[j].w);
        }
    };
    if (t0 < t1) load_chunk(t0);
    for (int t = t0; t < t1; t += 2) {
        store_chunk();
        __syncthreads();
        if (t + 2 < t1) load_chunk(t + 2);
#pragma unroll
        for (int q = 0; q < MAXT; ++q) {
            const int tile = w + 4 * q;
            if (tile >= MLP_GRAD_TILES) continue;       // uniform per wavefront
            const GradTile T = c_tiles[tile];
            const int kin = T.layer, kout = 4 + T.layer;
            const short *Lin = L + wg_off(kin) + 4 * (l / 16) * WG_P + 16 * T.mb + l % 16;
            const short *Lout = L + wg_off(kout) + 4 * (l / 16) * WG_P + 16 * T.nb + l % 16;
            bf16x4 a[2], bb[2];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    // vertex 16 h + 4 (l / 16) + i of the chunk
                    a[h][i] = T.bias ? (short)((l % 16) == 0 ? 0x3F80 : 0) : Lin[(16 * h + i) * WG_P];
                    bb[h][i] = Lout[(16 * h + i) * WG_P];
                }
            acc[q] = mfma32(a[0], a[1], bb[0], bb[1], acc[q]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < MAXT; ++q) {
        const int tile = w + 4 * q;
        if (tile >= MLP_GRAD_TILES) continue;
        float *o = part + ((int64_t)blockIdx.x * MLP_GRAD_TILES + tile) * 256;
#pragma unroll
        for (int i = 0; i < 4; ++i) o[(4 * (l / 16) + i) * 16 + l % 16] = acc[q][i];
    }
}

// Sum the per-block partial tiles and scatter them to the padded parameter
// layout.  Workgroup (tile, quarter) owns 64 of the tile's 256 entries: lane
// group g (16 lanes, one float4 each) adds the partials of blocks g, g + 16,
// g + 32, ... and the 16 group sums are then added in group order through
// LDS, so the result is the same on every run.
__global__ void __launch_bounds__(256) k_mlp_grad_reduce(int nblocks, const float *part, float *grad) {
    __shared__ float4 red[16][16];
    const int tile = blockIdx.x, quarter = blockIdx.y;
    const int j = threadIdx.x % 16, g = threadIdx.x / 16;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int b = g; b < nblocks; b += 16) {
        const float4 p =
            *reinterpret_cast<const float4 *>(part + ((int64_t)b * MLP_GRAD_TILES + tile) * 256 + 64 * quarter + 4 * j);
        acc.x += p.x; acc.y += p.y; acc.z += p.z; acc.w += p.w;
    }
    red[g][j] = acc;
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const int e = threadIdx.x;
    float s = 0.0f;
    for (int q = 0; q < 16; ++q) {
        const float4 v = red[q][e / 4];
        s += (e % 4) == 0 ? v.x : ((e % 4) == 1 ? v.y : ((e % 4) == 2 ? v.z : v.w));
    }
    const int rc = 64 * quarter + e, r = rc / 16, c = rc % 16;
    const GradTile T = c_tiles[tile];
    const int offW[4] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4}, offB[4] = {OFF_B1, OFF_B2, OFF_B3, OFF_B4};
    const int wout = T.layer == 3 ? 16 : 64;
    if (T.bias) {
        if (r == 0) grad[offB[T.layer] + 16 * T.nb + c] = s;
    } else {
        grad[offW[T.layer] + (16 * T.mb + r) * wout + 16 * T.nb + c] = s;
    }
}

// Adam on the FP32 parameters (pads stay zero: their gradients are zero),
// refreshing the BF16 copy.
__global__ void k_adam(int n, float *w, float *m, float *v, const float *g, short *wb, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
}

__global__ void k_to_bf16(int n, const float *w, short *wb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = f2bf(w[i]);
}

// ---------------------------------------------------------------- reductions
// Partial sums of NV products over vertices (3 components each) for the
// loss and the start's safeguard factor: out[q][block].
__global__ void __launch_bounds__(256) k_ws_dots(int n3, const double *a0, const double *b0, const double *a1,
                                                 const double *b1, const double *a2, const double *b2,
                                                 const float *wdiag, double *part) {
    __shared__ double sh[3][4];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    if (k < n3) {
        s[0] = a0[k] * b0[k];
        s[1] = a1[k] * b1[k];
        s[2] = wdiag ? a2[k] * b2[k] * (double)wdiag[k] : a2[k] * b2[k];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    for (int q = 0; q < 3; ++q) {
        double r = s[q];
        for (int m = 32; m >= 1; m >>= 1) r += __shfl_xor(r, m, 64);
        if (lane == 0) sh[q][w] = r;
    }
    __syncthreads();
    if (threadIdx.x < 3) part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] =
        sh[threadIdx.x][0] + sh[threadIdx.x][1] + sh[threadIdx.x][2] + sh[threadIdx.x][3];
}

__global__ void k_ws_dots_final(int nb, const double *part, double *out) {
    __shared__ double sh[3][16];
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        for (int q = 0; q < 3; ++q) s[q] += part[(int64_t)q * nb + b];
    for (int q = 0; q < 3; ++q) {
        double r = s[q];
        for (int m = 32; m >= 1; m >>= 1) r += __shfl_xor(r, m, 64);
        if (lane == 0) sh[q][w] = r;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double r = 0.0;
        for (int k = 0; k < (int)blockDim.x / 64; ++k) r += sh[threadIdx.x][k];
        out[threadIdx.x] = r;
    }
}

// Line search along the network's correction u from the previous increment:
// x = dv_prev + g u with g = (u.b - w.dv_prev) / u.w, w = A u (A symmetric,
// so w.dv_prev = u.A dv_prev); g = 0 when u.w is not positive.
__device__ __forceinline__ double line_step(const double *d) {
    const double g = (d[0] - d[2]) / d[1];
    return (d[1] > 0.0 && isfinite(g)) ? g : 0.0;
}

__global__ void k_line_start(int64_t n, const double *dvp, const double *u, const double *dots, double *x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = dvp[i] + line_step(dots) * u[i];
}

// ---------------------------------------------------------------- host side
static std::vector<GradTile> grad_tiles() {
    std::vector<GradTile> t;
    const int nin[4] = {2, 4, 4, 4}, nout[4] = {4, 4, 4, 1};
    for (int L = 0; L < 4; ++L) {
        for (int mb = 0; mb < nin[L]; ++mb)
            for (int nb = 0; nb < nout[L]; ++nb) t.push_back(GradTile{L, mb, nb, 0});
        for (int nb = 0; nb < nout[L]; ++nb) t.push_back(GradTile{L, 0, nb, 1});
    }
    return t;
}

pc_status mlp_init(Ctx *ctx, MlpState *M) {
    if (M->ready) return PC_OK;
    const std::vector<GradTile> tiles = grad_tiles();
    if ((int)tiles.size() != MLP_GRAD_TILES) {
        ctx->err = "internal: gradient tile count";
        return PC_ERR_ARG;
    }
    PC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tiles), tiles.data(), sizeof(GradTile) * tiles.size()));
    M->nv_pad = ((ctx->nv + 15) / 16) * 16;
    const size_t nvp = (size_t)M->nv_pad;
    pc_status st;
    void **bufs[] = {(void **)&M->w, (void **)&M->m, (void **)&M->v, (void **)&M->g, (void **)&M->wb};
    const size_t sizes[] = {sizeof(float) * MLP_PADDED, sizeof(float) * MLP_PADDED, sizeof(float) * MLP_PADDED,
                            sizeof(float) * MLP_PADDED, sizeof(short) * MLP_PADDED};
    for (int k = 0; k < 5; ++k)
        if ((st = dev_alloc(ctx, bufs[k], sizes[k]))) return st;
    if ((st = dev_alloc(ctx, (void **)&M->X, sizeof(short) * 32 * nvp))) return st;
    if ((st = dev_alloc(ctx, (void **)&M->dots, sizeof(double) * 8))) return st;
    if ((st = dev_alloc(ctx, (void **)&M->dpart, sizeof(double) * 3 * (size_t)(3 * ctx->nv / 256 + 16)))) return st;
    PC_HIP(hipMemset(M->w, 0, sizeof(float) * MLP_PADDED));
    PC_HIP(hipMemset(M->m, 0, sizeof(float) * MLP_PADDED));
    PC_HIP(hipMemset(M->v, 0, sizeof(float) * MLP_PADDED));
    PC_HIP(hipMemset(M->g, 0, sizeof(float) * MLP_PADDED));
    PC_HIP(hipMemset(M->wb, 0, sizeof(short) * MLP_PADDED));
    M->ready = true;
    return PC_OK;
}

static pc_status mlp_train_buffers(Ctx *ctx, MlpState *M) {
    if (M->H1) return PC_OK;
    const size_t nvp = (size_t)M->nv_pad;
    pc_status st;
    short **bufs[] = {&M->H1, &M->H2, &M->H3, &M->G1, &M->G2, &M->G3};
    for (short **b : bufs)
        if ((st = dev_alloc(ctx, (void **)b, sizeof(short) * 64 * nvp))) return st;
    if ((st = dev_alloc(ctx, (void **)&M->G4, sizeof(short) * 16 * nvp))) return st;
    if ((st = dev_alloc(ctx, (void **)&M->Ad, sizeof(double) * 3 * (size_t)ctx->nv))) return st;
    if ((st = dev_alloc(ctx, (void **)&M->part, sizeof(float) * 256 * MLP_GRAD_TILES * (size_t)MLP_WGRAD_BLOCKS)))
        return st;
    PC_HIP(hipMemset(M->G4, 0, sizeof(short) * 16 * nvp));
    return PC_OK;
}

// Oracle flat layout (per layer: W [in][out] row-major, then bias) <-> padded.
static void flat_to_padded(const float *flat, std::vector<float> &pad) {
    pad.assign(MLP_PADDED, 0.0f);
    const int in[4] = {27, 64, 64, 64}, out[4] = {64, 64, 64, 3}, wout[4] = {64, 64, 64, 16};
    const int offW[4] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4}, offB[4] = {OFF_B1, OFF_B2, OFF_B3, OFF_B4};
    int o = 0;
    for (int L = 0; L < 4; ++L) {
        for (int i = 0; i < in[L]; ++i)
            for (int j = 0; j < out[L]; ++j) pad[offW[L] + i * wout[L] + j] = flat[o++];
        for (int j = 0; j < out[L]; ++j) pad[offB[L] + j] = flat[o++];
    }
}
static void padded_to_flat(const std::vector<float> &pad, float *flat) {
    const int in[4] = {27, 64, 64, 64}, out[4] = {64, 64, 64, 3}, wout[4] = {64, 64, 64, 16};
    const int offW[4] = {OFF_W1, OFF_W2, OFF_W3, OFF_W4}, offB[4] = {OFF_B1, OFF_B2, OFF_B3, OFF_B4};
    int o = 0;
    for (int L = 0; L < 4; ++L) {
        for (int i = 0; i < in[L]; ++i)
            for (int j = 0; j < out[L]; ++j) flat[o++] = pad[offW[L] + i * wout[L] + j];
        for (int j = 0; j < out[L]; ++j) flat[o++] = pad[offB[L] + j];
    }
}

pc_status mlp_set_params(Ctx *ctx, MlpState *M, const float *flat) {
    pc_status st = mlp_init(ctx, M);
    if (st) return st;
    std::vector<float> pad;
    flat_to_padded(flat, pad);
    PC_HIP(hipMemcpy(M->w, pad.data(), sizeof(float) * MLP_PADDED, hipMemcpyHostToDevice));
    PC_HIP(hipMemset(M->m, 0, sizeof(float) * MLP_PADDED));
    PC_HIP(hipMemset(M->v, 0, sizeof(float) * MLP_PADDED));
    hipLaunchKernelGGL(k_to_bf16, dim3((MLP_PADDED + 255) / 256), dim3(256), 0, 0, MLP_PADDED, M->w, M->wb);
    PC_HIP(hipGetLastError());
    PC_HIP(hipDeviceSynchronize());
    M->step = 0;
    M->has_params = true;
    return PC_OK;
}

pc_status mlp_get_params(Ctx *ctx, MlpState *M, float *flat) {
    if (!M->has_params) {
        ctx->err = "no warm-start parameters set";
        return PC_ERR_ARG;
    }
    std::vector<float> pad(MLP_PADDED);
    PC_HIP(hipMemcpy(pad.data(), M->w, sizeof(float) * MLP_PADDED, hipMemcpyDeviceToHost));
    padded_to_flat(pad, flat);
    return PC_OK;
}

pc_status mlp_get_grads(Ctx *ctx, MlpState *M, float *flat) {
    std::vector<float> pad(MLP_PADDED);
    PC_HIP(hipMemcpy(pad.data(), M->g, sizeof(float) * MLP_PADDED, hipMemcpyDeviceToHost));
    padded_to_flat(pad, flat);
    return PC_OK;
}

pc_status mlp_features(Ctx *ctx, MlpState *M, const double *x, const double *v, const double *b, const double *dvp,
                       hipStream_t s) {
    pc_status st = mlp_init(ctx, M);
    if (st) return st;
    if (!ctx->assembled) {
        ctx->err = "warm start: nothing assembled";
        return PC_ERR_ARG;
    }
    hipLaunchKernelGGL(k_ws_features, dim3((M->nv_pad + 255) / 256), dim3(256), 0, s, ctx->nv, M->nv_pad,
                       ctx->rowptr, ctx->colidx, x, v, b, ctx->diag, ctx->mass, ctx->pinned, dvp, ctx->ell,
                       ctx->prm.h, M->X);
    PC_HIP(hipGetLastError());
    return PC_OK;
}

pc_status mlp_forward(Ctx *ctx, MlpState *M, const double *dvp, double *dv0, bool train, hipStream_t s) {
    pc_status st;
    if (train && (st = mlp_train_buffers(ctx, M))) return st;
    FwdArgs F;
    F.nv = ctx->nv;
    F.ntiles = M->nv_pad / 16;
    F.X = M->X;
    F.Wb = M->wb;
    F.Wf = M->w;
    F.H1 = train ? M->H1 : nullptr;
    F.H2 = train ? M->H2 : nullptr;
    F.H3 = train ? M->H3 : nullptr;
    F.dvp = dvp;
    F.pinned = ctx->pinned;
    F.sv = ctx->ell / ctx->prm.h;
    F.dv0 = dv0;
    const int blocks = std::min(1024, (F.ntiles + 3) / 4);
    hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, F);
    PC_HIP(hipGetLastError());
    return PC_OK;
}

// dots[0..2] = (a0.b0, a1.b1, a2.b2 [* wdiag]) over the 3 nv components.
static pc_status dots3(Ctx *ctx, MlpState *M, const double *a0, const double *b0, const double *a1,
                       const double *b1, const double *a2, const double *b2, const float *wdiag, double *out,
                       hipStream_t s) {
    const int n3 = 3 * ctx->nv;
    const int nb = (n3 + 255) / 256;
    hipLaunchKernelGGL(k_ws_dots, dim3(nb), dim3(256), 0, s, n3, a0, b0, a1, b1, a2, b2, wdiag, M->dpart);
    hipLaunchKernelGGL(k_ws_dots_final, dim3(1), dim3(1024), 0, s, nb, M->dpart, out);
    PC_HIP(hipGetLastError());
    return PC_OK;
}

pc_status mlp_gradient(Ctx *ctx, MlpState *M, const double *x, const double *v, const double *b, const double *dvp,
                       double *loss, hipStream_t s) {
    pc_status st;
    if (!M->has_params) {
        ctx->err = "no warm-start parameters set";
        return PC_ERR_ARG;
    }
    if ((st = mlp_features(ctx, M, x, v, b, dvp, s))) return st;
    if ((st = mlp_train_buffers(ctx, M))) return st;
    double *dv0 = ctx->q;  // scratch of the solver (not in use between solves)
    if ((st = mlp_forward(ctx, M, dvp, dv0, true, s))) return st;
    if ((st = spmv_run(ctx, dv0, M->Ad, false, s))) return st;
    // dots: [dv0.A dv0, b.dv0, b.D^-1 b]
    if ((st = dots3(ctx, M, dv0, M->Ad, b, dv0, b, b, ctx->dinv, M->dots, s))) return st;
    hipLaunchKernelGGL(k_ws_out_grad, dim3((M->nv_pad + 255) / 256), dim3(256), 0, s, ctx->nv, M->nv_pad, M->Ad, b,
                       ctx->pinned, ctx->ell / ctx->prm.h, M->dots + 2, M->G4);
    BwdArgs Bw;
    Bw.ntiles = M->nv_pad / 16;
    Bw.Wb = M->wb;
    Bw.H1 = M->H1; Bw.H2 = M->H2; Bw.H3 = M->H3; Bw.G4 = M->G4;
    Bw.G1 = M->G1; Bw.G2 = M->G2; Bw.G3 = M->G3;
    const int blocks = std::min(1024, (Bw.ntiles + 3) / 4);
    hipLaunchKernelGGL(k_mlp_bwd, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, Bw);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(MLP_WGRAD_BLOCKS), dim3(256), 0, s, M->nv_pad / 16, M->X, M->H1, M->H2,
                       M->H3, M->G1, M->G2, M->G3, M->G4, M->part);
    hipLaunchKernelGGL(k_mlp_grad_reduce, dim3(MLP_GRAD_TILES, 4), dim3(256), 0, s, MLP_WGRAD_BLOCKS, M->part,
                       M->g);
    PC_HIP(hipGetLastError());
    if (loss) {
        double d[3];
        PC_HIP(hipMemcpyAsync(d, M->dots, sizeof(d), hipMemcpyDeviceToHost, s));
        PC_HIP(hipStreamSynchronize(s));
        *loss = (0.5 * d[0] - d[1]) / d[2];
    }
    return PC_OK;
}

pc_status mlp_adam(Ctx *ctx, MlpState *M, double lr, hipStream_t s) {
    M->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)M->step), c2 = 1.0f - powf(b2, (float)M->step);
    hipLaunchKernelGGL(k_adam, dim3((MLP_PADDED + 255) / 256), dim3(256), 0, s, MLP_PADDED, M->w, M->m, M->v, M->g,
                       M->wb, (float)lr, b1, b2, 1e-8f, c1, c2);
    PC_HIP(hipGetLastError());
    return PC_OK;
}

// Learned start: the network's correction u = s_v MLP(features) is added to
// the previous increment with the step g that minimises the A-norm error of
// dv_prev + g u (one SpMV with the FP64 blocks), so the start is never worse
// in the A-norm than the previous increment itself.  u goes through u_buf
// (nv * 3 doubles of scratch).  *used = 2 when g != 0, 1 otherwise.
pc_status mlp_start(Ctx *ctx, MlpState *M, const double *x, const double *v, const double *b, const double *dvp,
                    double *dv0, double *u_buf, int *used, hipStream_t s) {
    pc_status st;
    *used = 1;
    if (!M->has_params) {
        ctx->err = "no warm-start parameters set";
        return PC_ERR_ARG;
    }
    if ((st = mlp_features(ctx, M, x, v, b, dvp, s))) return st;
    if ((st = mlp_forward(ctx, M, nullptr, u_buf, false, s))) return st;
    if (!M->Ad && (st = dev_alloc(ctx, (void **)&M->Ad, sizeof(double) * 3 * (size_t)ctx->nv))) return st;
    if ((st = spmv_run(ctx, u_buf, M->Ad, false, s))) return st;
    // dots: [u.b, u.w, w.dv_prev]
    if ((st = dots3(ctx, M, u_buf, b, u_buf, M->Ad, M->Ad, dvp, nullptr, M->dots, s))) return st;
    const int64_t n3 = 3 * (int64_t)ctx->nv;
    hipLaunchKernelGGL(k_line_start, dim3((n3 + 255) / 256), dim3(256), 0, s, n3, dvp, u_buf, M->dots, dv0);
    PC_HIP(hipGetLastError());
    double d[3];
    PC_HIP(hipMemcpyAsync(d, M->dots, sizeof(d), hipMemcpyDeviceToHost, s));
    PC_HIP(hipStreamSynchronize(s));
    const double g = (d[0] - d[2]) / d[1];
    M->last_scale = (d[1] > 0.0 && std::isfinite(g)) ? g : 0.0;
    *used = M->last_scale != 0.0 ? 2 : 1;
    return PC_OK;
}

// ---------------------------------------------------------------- prediction without allocation
// pc_ws_predict_noalloc keeps the network's input rows (BF16 features) in
// this file-scope array instead of the context's feature buffer: 64 MiB, the
// rows of up to WS_NOALLOC_MAX_ROWS vertices.  Every GPU the library runs on
// holds its own copy from the module's load until the process ends; all
// contexts on a GPU share it, and each call overwrites it.
constexpr int WS_NOALLOC_MAX_ROWS = 1 << 20;
static __device__ __align__(256) short scratch[(size_t)WS_NOALLOC_MAX_ROWS * 32];

// Device address of `scratch` on each GPU, looked up once per device with
// that device current.  Host code passes this address to kernels, never the
// array's own name (a host-side stand-in, not a device address).
constexpr int WS_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[WS_MAX_DEVICES] = {};

pc_status mlp_scratch_init(Ctx *ctx) {
    int dev = 0;
    PC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= WS_MAX_DEVICES) {
        ctx->err = "device index " + std::to_string(dev) + " beyond the library's " +
                   std::to_string(WS_MAX_DEVICES);
        return PC_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            ctx->err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return PC_ERR_HIP;
        }
        g_scratch_dev[dev] = p;
    }
    ctx->ws_scratch = g_scratch_dev[dev];
    return PC_OK;
}

// The same two launches as pc_ws_predict (features, then the forward pass),
// with the features in the per-GPU scratch.  Allocates nothing: the network's
// state must exist already (pc_ws_set_params).  The features kernel writes
// every row below nv_pad (zeros past nv), so nothing of the previous call's
// contents is read.
pc_status mlp_predict_noalloc(Ctx *ctx, const double *x, const double *v, const double *b, const double *dvp,
                              double *dv0, hipStream_t s) {
    const int nv_pad = ((ctx->nv + 15) / 16) * 16;
    if (nv_pad > WS_NOALLOC_MAX_ROWS) {
        ctx->err = "pc_ws_predict_noalloc: " + std::to_string(ctx->nv) + " vertices exceed its scratch of " +
                   std::to_string(WS_NOALLOC_MAX_ROWS) + " rows; use pc_ws_predict";
        return PC_ERR_CAPACITY;
    }
    if (!ctx->ws_scratch) {
        ctx->err = "pc_ws_predict_noalloc: scratch not set up";
        return PC_ERR_HIP;
    }
    MlpState *M = ctx->mlp;
    if (!M || !M->ready || !M->has_params) {
        ctx->err = "pc_ws_predict_noalloc: no warm-start parameters set";
        return PC_ERR_ARG;
    }
    if (!ctx->assembled) {
        ctx->err = "pc_ws_predict_noalloc: nothing assembled";
        return PC_ERR_ARG;
    }
    short *X = (short *)ctx->ws_scratch;
    hipLaunchKernelGGL(k_ws_features, dim3((nv_pad + 255) / 256), dim3(256), 0, s, ctx->nv, nv_pad, ctx->rowptr,
                       ctx->colidx, x, v, b, ctx->diag, ctx->mass, ctx->pinned, dvp, ctx->ell, ctx->prm.h, X);
    PC_HIP(hipGetLastError());
    FwdArgs F;
    F.nv = ctx->nv;
    F.ntiles = nv_pad / 16;
    F.X = X;
    F.Wb = M->wb;
    F.Wf = M->w;
    F.H1 = F.H2 = F.H3 = nullptr;
    F.dvp = dvp;
    F.pinned = ctx->pinned;
    F.sv = ctx->ell / ctx->prm.h;
    F.dv0 = dv0;
    const int blocks = std::min(1024, (F.ntiles + 3) / 4);
    hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, F);
    PC_HIP(hipGetLastError());
    return PC_OK;
}

pc_status mlp_probe(Ctx *ctx, float *host_out) {
    float *d = nullptr;
    pc_status st = dev_alloc(ctx, (void **)&d, sizeof(float) * 1024);
    if (st) return st;
    hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, 0, d);
    PC_HIP(hipGetLastError());
    PC_HIP(hipMemcpy(host_out, d, sizeof(float) * 1024, hipMemcpyDeviceToHost));
    dev_free(ctx, d);
    return PC_OK;
}

void mlp_free(Ctx *ctx, MlpState *M) {
    void *ptrs[] = {M->w, M->m, M->v, M->g, M->wb, M->X, M->H1, M->H2, M->H3, M->G1, M->G2, M->G3,
                    M->G4, M->Ad, M->part, M->dots, M->dpart};
    for (void *p : ptrs)
        if (p) dev_free(ctx, p);
    *M = MlpState{};
}

}  // namespace pc
