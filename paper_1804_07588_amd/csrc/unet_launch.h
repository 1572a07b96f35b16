// Host launchers of the U-Net kernels (tensors channels-last, cube edge R,
// N samples; positions S = N R^3).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace unet {
// out = act(conv3x3x3(X) + bias); mode 0 bf16 store, 1 f32 store, 2 f32 add
hipError_t conv(const __bf16 *X, int Ci, const __bf16 *W, const float *bias, int Co, int R, int N, int mode,
                int relu, void *out, hipStream_t st);
// Reductions over positions go through per-block partials (part, device
// scratch of the sizes below) added in a fixed order: results are bitwise
// reproducible.
constexpr int LOSS_BLOCKS = 2048;
// chunks of the weight gradient (part holds chunks x Co x 27 x Ci floats)
int wgrad_chunks(int R, int N);
// GW[co][tap][ci] = sum_s GY[s][co] X[s + off(tap)][ci]
hipError_t wgrad(const __bf16 *GY, int Co, const __bf16 *X, int Ci, int R, int N, float *GW, float *part,
                 hipStream_t st);
// blocks of act_bwd over n values of C channels (part holds blocks x C floats)
int act_bwd_blocks(size_t n, int C);
// gb = g * (y > 0) (no mask if y is null) as bf16; gbias[c] = sum_s gb
hipError_t act_bwd(const float *g, const __bf16 *y, size_t n, int C, __bf16 *gb, float *gbias, float *part,
                   hipStream_t st);
hipError_t pool(const __bf16 *X, int R, int C, int N, __bf16 *Y, hipStream_t st);
hipError_t pool_bwd(const float *GO, int R, int C, int N, float *GI, hipStream_t st);
hipError_t up(const __bf16 *X, int r, int C, int N, __bf16 *Y, int Ct, int off, hipStream_t st);
hipError_t up_bwd(const float *GO, int r, int C, int Ct, int off, int N, float *GI, hipStream_t st);
hipError_t copy_ch(const __bf16 *X, int C, __bf16 *Y, int Ct, int off, size_t npos, hipStream_t st);
hipError_t copy_ch_bwd(const float *GY, int C, int Ct, int off, size_t npos, float *GX, hipStream_t st);
hipError_t input(const float *in, int cin, int Cp, size_t npos, __bf16 *X, hipStream_t st);
// part: LOSS_BLOCKS doubles
hipError_t loss(const float *P, int Cp, const float *T, const float *Wt, int nt, size_t npos, double inv_wsum,
                float *G, double *l, double *part, hipStream_t st);
hipError_t adam(float *p, float *m, float *v, const float *g, size_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t st);
hipError_t wcast(const float *w, int Co, int Ci, __bf16 *W, __bf16 *WT, hipStream_t st);
}  // namespace unet
