// Learned warm start: device state and entry points (see mlp.hip).
#pragma once
#include "pc_ctx.h"

namespace pc {

constexpr int MLP_PARAMS = 27 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3;  // 10,307
constexpr int MLP_PADDED = 32 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 * 16 + 16;  // 11,472
constexpr int MLP_GRAD_TILES = 57;
constexpr int MLP_WGRAD_BLOCKS = 768;   // three per CU, all resident at once at 3 waves per SIMD

struct MlpState {
    bool ready = false, has_params = false;
    int nv_pad = 0;
    int step = 0;
    double last_scale = 0.0;
    float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // padded FP32 parameters, Adam moments, gradient
    short *wb = nullptr;                                             // BF16 copy of w
    short *X = nullptr;                                              // features [nv_pad][32]
    short *H1 = nullptr, *H2 = nullptr, *H3 = nullptr;               // activations [nv_pad][64]
    short *G1 = nullptr, *G2 = nullptr, *G3 = nullptr;               // gradients [nv_pad][64]
    short *G4 = nullptr;                                             // output gradient [nv_pad][16]
    double *Ad = nullptr;                                            // A dv0
    float *part = nullptr;                                           // split-K partial gradient tiles
    double *dots = nullptr, *dpart = nullptr;
};

pc_status mlp_init(Ctx *ctx, MlpState *M);
pc_status mlp_set_params(Ctx *ctx, MlpState *M, const float *flat);
pc_status mlp_get_params(Ctx *ctx, MlpState *M, float *flat);
pc_status mlp_get_grads(Ctx *ctx, MlpState *M, float *flat);
pc_status mlp_features(Ctx *ctx, MlpState *M, const double *x, const double *v, const double *b, const double *dvp,
                       hipStream_t s);
pc_status mlp_forward(Ctx *ctx, MlpState *M, const double *dvp, double *dv0, bool train, hipStream_t s);
pc_status mlp_gradient(Ctx *ctx, MlpState *M, const double *x, const double *v, const double *b, const double *dvp,
                       double *loss, hipStream_t s);
pc_status mlp_adam(Ctx *ctx, MlpState *M, double lr, hipStream_t s);
pc_status mlp_start(Ctx *ctx, MlpState *M, const double *x, const double *v, const double *b, const double *dvp,
                    double *dv0, double *u_buf, int *used, hipStream_t s);
pc_status mlp_probe(Ctx *ctx, float *host_out);
void mlp_free(Ctx *ctx, MlpState *M);
pc_status mlp_scratch_init(Ctx *ctx);
pc_status mlp_predict_noalloc(Ctx *ctx, const double *x, const double *v, const double *b, const double *dvp,
                              double *dv0, hipStream_t s);

}  // namespace pc
