// Kernels of the learned warm start: a 3-D U-Net over a cubic lattice of
// edge R (channels-last tensors [n][z][y][x][c], bf16 activations, FP32
// accumulation), trained on the GPU.  Convolutions (3x3x3, stride 1, zero
// padding 1) are implicit GEMMs on the bf16 MFMA of gfx950
// (v_mfma_f32_16x16x32_bf16); the rest are elementwise kernels and
// reductions.
//
// MFMA 16x16x32 bf16 operand layout (lane l of the wavefront):
//   A (16 x 32, M x K): row l % 16, columns 8 (l / 16) .. 8 (l / 16) + 7
//   B (32 x 16, K x N): rows 8 (l / 16) .. + 7, column l % 16
//   D (16 x 16):        rows 4 (l / 16) .. + 3, column l % 16
#include <hip/hip_runtime.h>

#include "unet_launch.h"

namespace unet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TPB = 256;

__device__ inline bf16x8 zero8() {
  bf16x8 z;
#pragma unroll
  for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
  return z;
}

// ---------------------------------------------------------------------------
// convolution as implicit GEMM: out[s][co] = act(sum_{tap,ci} W[co][tap][ci]
// X[s + off(tap)][ci] + bias[co]).  One workgroup: 64 consecutive positions
// (M) x BN output channels; wave w owns positions 16w .. 16w + 15.
// mode: 0 store bf16, 1 store f32, 2 add into f32.  Ci % 32 == 0,
// Co % BN == 0, S % 64 == 0 (host-checked).
// ---------------------------------------------------------------------------
template <int BN>
__global__ void __launch_bounds__(TPB) k_conv(const __bf16 *__restrict__ X, int Ci, const __bf16 *__restrict__ W,
                                              const float *__restrict__ bias, int Co, int R, int mode, int relu,
                                              void *__restrict__ out) {
  constexpr int NT = BN / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int s0 = blockIdx.x * 64 + wave * 16;
  const int co0 = blockIdx.y * BN;
  const int R3 = R * R * R;
  const int s = s0 + m;  // this lane's A row
  const int x = s % R, y = (s / R) % R, z = (s / (R * R)) % R, base = s - (s % R3);
  f32x4 acc[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int tap = 0; tap < 27; ++tap) {
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int zz = z + dz, yy = y + dy, xx = x + dx;
    const bool ok = (unsigned)zz < (unsigned)R && (unsigned)yy < (unsigned)R && (unsigned)xx < (unsigned)R;
    const __bf16 *xp = X + (size_t)(ok ? base + (zz * R + yy) * R + xx : 0) * Ci + kq * 8;
    const __bf16 *wp = W + ((size_t)(co0 + m) * 27 + tap) * Ci + kq * 8;
    for (int c0 = 0; c0 < Ci; c0 += 32) {
      const bf16x8 a = ok ? *reinterpret_cast<const bf16x8 *>(xp + c0) : zero8();
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(wp + (size_t)j * 16 * 27 * Ci + c0);
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int co = co0 + j * 16 + m;
    const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const size_t o = (size_t)(s0 + 4 * kq + i) * Co + co;
      float v = acc[j][i] + bv;
      if (relu) v = fmaxf(v, 0.0f);
      if (mode == 0) static_cast<__bf16 *>(out)[o] = (__bf16)v;
      else if (mode == 1) static_cast<float *>(out)[o] = v;
      else static_cast<float *>(out)[o] += v;
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: gW[co][tap][ci] += sum_s gY[s][co] X[s + off(tap)][ci].
// Grid (27 taps, chunks of WG_CH positions, groups of 16 output tiles of
// 16 x 16).  Per step of 32 positions the workgroup stages gY and the shifted
// X rows in LDS; wave w of group g owns tiles 16 g + w + 4 t, t < 4.
// ---------------------------------------------------------------------------
constexpr int WG_CH = 2048;  // positions per workgroup
constexpr int WG_MAXT = 4;   // tiles per wave
constexpr int WG_MAXC = 224; // largest channel count staged

__global__ void __launch_bounds__(TPB) k_wgrad(const __bf16 *__restrict__ GY, int Co,
                                               const __bf16 *__restrict__ X, int Ci, int R, int S,
                                               float *__restrict__ GW) {
  __shared__ __bf16 sg[32 * WG_MAXC];
  __shared__ __bf16 sx[32 * WG_MAXC];
  const int tap = blockIdx.x;
  const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int nci = Ci / 16, ntile = (Co / 16) * nci, tile0 = blockIdx.z * 16;
  const int R3 = R * R * R;
  f32x4 acc[WG_MAXT];
#pragma unroll
  for (int t = 0; t < WG_MAXT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int p0 = blockIdx.y * WG_CH, p1 = min(S, p0 + WG_CH);
  for (int sb = p0; sb < p1; sb += 32) {
    __syncthreads();
    // stage 32 rows of gY (Co wide) and of shifted X (Ci wide)
    for (int e = threadIdx.x; e < 32 * Co; e += TPB) {
      const int r = e / Co, c = e % Co;
      sg[r * Co + c] = GY[(size_t)(sb + r) * Co + c];
    }
    for (int e = threadIdx.x; e < 32 * Ci; e += TPB) {
      const int r = e / Ci, c = e % Ci;
      const int s = sb + r;
      const int x = s % R + dx, y = (s / R) % R + dy, z = (s / (R * R)) % R + dz;
      __bf16 v = (__bf16)0.0f;
      if ((unsigned)x < (unsigned)R && (unsigned)y < (unsigned)R && (unsigned)z < (unsigned)R)
        v = X[(size_t)(s - (s % R3) + (z * R + y) * R + x) * Ci + c];
      sx[r * Ci + c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < WG_MAXT; ++t) {
      const int tile = tile0 + wave + 4 * t;
      if (tile < ntile) {
        const int ct = tile / nci, it = tile % nci;
        bf16x8 a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          a[i] = sg[(8 * kq + i) * Co + ct * 16 + m];  // A[m = co][k = position]
          b[i] = sx[(8 * kq + i) * Ci + it * 16 + m];  // B[k = position][n = ci]
        }
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < WG_MAXT; ++t) {
    const int tile = tile0 + wave + 4 * t;
    if (tile < ntile) {
      const int ct = tile / nci, it = tile % nci;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = ct * 16 + 4 * kq + i, ci = it * 16 + m;
        atomicAdd(&GW[((size_t)co * 27 + tap) * Ci + ci], acc[t][i]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// elementwise and reductions
// ---------------------------------------------------------------------------
// bf16 gradient of a pre-activation from the f32 gradient of the layer
// output (ReLU mask from the stored output y when y is given) and the bias
// gradient (sum over positions, one atomic per channel and block)
__global__ void __launch_bounds__(TPB) k_act_bwd(const float *__restrict__ g, const __bf16 *__restrict__ y,
                                                 size_t n, int C, __bf16 *__restrict__ gb,
                                                 float *__restrict__ gbias) {
  __shared__ float sb[WG_MAXC];
  for (int c = threadIdx.x; c < C; c += TPB) sb[c] = 0.0f;
  __syncthreads();
  const size_t per = (size_t)TPB * 16;
  const size_t e0 = (size_t)blockIdx.x * per;
  for (size_t e = e0 + threadIdx.x; e < e0 + per && e < n; e += TPB) {
    float v = g[e];
    if (y && !((float)y[e] > 0.0f)) v = 0.0f;
    gb[e] = (__bf16)v;
    atomicAdd(&sb[e % C], v);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += TPB)
    if (sb[c] != 0.0f) atomicAdd(&gbias[c], sb[c]);
}

// 2x2x2 average pooling, edge R -> R/2
__global__ void k_pool(const __bf16 *__restrict__ X, int R, int C, size_t n_out, __bf16 *__restrict__ Y) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n_out) return;
  const int r = R / 2;
  const int c = (int)(e % C);
  const size_t p = e / C;
  const int x = (int)(p % r), y = (int)((p / r) % r), z = (int)((p / ((size_t)r * r)) % r);
  const size_t b = p / ((size_t)r * r * r);
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int zz = 2 * z + (k >> 2), yy = 2 * y + ((k >> 1) & 1), xx = 2 * x + (k & 1);
    s += (float)X[((b * R + zz) * R + yy) * (size_t)R * C + (size_t)xx * C + c];
  }
  Y[e] = (__bf16)(0.125f * s);
}
// its adjoint: G_in += G_out / 8 (f32)
__global__ void k_pool_bwd(const float *__restrict__ GO, int R, int C, size_t n_in, float *__restrict__ GI) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n_in) return;
  const int r = R / 2;
  const int c = (int)(e % C);
  const size_t p = e / C;
  const int x = (int)(p % R), y = (int)((p / R) % R), z = (int)((p / ((size_t)R * R)) % R);
  const size_t b = p / ((size_t)R * R * R);
  GI[e] += 0.125f * GO[(((b * r + z / 2) * r + y / 2) * r + x / 2) * (size_t)C + c];
}

// nearest 2x upsampling of X (edge r, C channels) into channels [off, off+C)
// of Y (edge 2r, Ct channels)
__global__ void k_up(const __bf16 *__restrict__ X, int r, int C, __bf16 *__restrict__ Y, int Ct, int off,
                     size_t n_out) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n_out) return;
  const int R = 2 * r;
  const int c = (int)(e % C);
  const size_t p = e / C;
  const int x = (int)(p % R), y = (int)((p / R) % R), z = (int)((p / ((size_t)R * R)) % R);
  const size_t b = p / ((size_t)R * R * R);
  Y[p * Ct + off + c] = X[(((b * r + z / 2) * r + y / 2) * r + x / 2) * (size_t)C + c];
}
// its adjoint: G_in (edge r, C) = sum of the 8 children's G_out[.., off + c]
__global__ void k_up_bwd(const float *__restrict__ GO, int r, int C, int Ct, int off, size_t n_in,
                         float *__restrict__ GI) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n_in) return;
  const int R = 2 * r;
  const int c = (int)(e % C);
  const size_t p = e / C;
  const int x = (int)(p % r), y = (int)((p / r) % r), z = (int)((p / ((size_t)r * r)) % r);
  const size_t b = p / ((size_t)r * r * r);
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int zz = 2 * z + (k >> 2), yy = 2 * y + ((k >> 1) & 1), xx = 2 * x + (k & 1);
    s += GO[(((b * R + zz) * R + yy) * (size_t)R + xx) * Ct + off + c];
  }
  GI[e] = s;
}

// channel copy X (C) -> Y[.., off + c] (Ct channels), and its adjoint (+=)
__global__ void k_copy_ch(const __bf16 *__restrict__ X, int C, __bf16 *__restrict__ Y, int Ct, int off, size_t n) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n) return;
  Y[(e / C) * Ct + off + e % C] = X[e];
}
__global__ void k_copy_ch_bwd(const float *__restrict__ GY, int C, int Ct, int off, size_t n, float *__restrict__ GX) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n) return;
  GX[e] += GY[(e / C) * Ct + off + e % C];
}

// network input: f32 [s][cin] -> bf16 [s][Cp] zero-padded
__global__ void k_input(const float *__restrict__ in, int cin, int Cp, size_t n, __bf16 *__restrict__ X) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e % Cp);
  X[e] = (__bf16)(c < cin ? in[(e / Cp) * cin + c] : 0.0f);
}

// weighted squared error: out f32 [s][Cp] (first nt used), target and weight
// f32 [s][nt]; loss = sum w (p - t)^2 / wsum, gradient into G [s][Cp]
__global__ void __launch_bounds__(TPB) k_loss(const float *__restrict__ P, int Cp, const float *__restrict__ T,
                                              const float *__restrict__ Wt, int nt, size_t npos, double inv_wsum,
                                              float *__restrict__ G, double *__restrict__ loss) {
  __shared__ double sh[TPB];
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  double l = 0.0;
  if (e < npos * Cp) {
    const size_t s = e / Cp;
    const int c = (int)(e % Cp);
    float g = 0.0f;
    if (c < nt) {
      const float d = P[e] - T[s * nt + c], w = Wt[s * nt + c];
      l = (double)w * d * d;
      g = (float)(2.0 * inv_wsum * w * d);
    }
    G[e] = g;
  }
  sh[threadIdx.x] = l;
  __syncthreads();
  for (int k = TPB / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0 && sh[0] != 0.0) atomicAdd(loss, sh[0] * inv_wsum);
}

// Adam on the FP32 master parameters, then the bf16 copies the convolutions
// read: W [co][tap][ci] and the flipped transpose WT [ci][26 - tap][co]
__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.0f - b1) * gi;
  const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}
__global__ void k_wcast(const float *__restrict__ w, int Co, int Ci, __bf16 *__restrict__ W,
                        __bf16 *__restrict__ WT) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  const size_t n = (size_t)Co * 27 * Ci;
  if (e >= n) return;
  const int ci = (int)(e % Ci), tap = (int)((e / Ci) % 27), co = (int)(e / ((size_t)Ci * 27));
  const __bf16 b = (__bf16)w[e];
  W[e] = b;
  if (WT) WT[((size_t)ci * 27 + (26 - tap)) * Co + co] = b;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static unsigned nblk(size_t n) { return (unsigned)((n + TPB - 1) / TPB); }

hipError_t conv(const __bf16 *X, int Ci, const __bf16 *W, const float *bias, int Co, int R, int N, int mode,
                int relu, void *out, hipStream_t st) {
  const int S = N * R * R * R;
  if (Ci % 32 || Co % 32 || S % 64) return hipErrorInvalidValue;
  if (Co % 64 == 0)
    hipLaunchKernelGGL(k_conv<64>, dim3(S / 64, Co / 64), dim3(TPB), 0, st, X, Ci, W, bias, Co, R, mode, relu, out);
  else
    hipLaunchKernelGGL(k_conv<32>, dim3(S / 64, Co / 32), dim3(TPB), 0, st, X, Ci, W, bias, Co, R, mode, relu, out);
  return hipGetLastError();
}

hipError_t wgrad(const __bf16 *GY, int Co, const __bf16 *X, int Ci, int R, int N, float *GW, hipStream_t st) {
  const int S = N * R * R * R;
  if (Ci % 16 || Co % 16 || Ci > WG_MAXC || Co > WG_MAXC || S % 32) return hipErrorInvalidValue;
  const int groups = ((Co / 16) * (Ci / 16) + 15) / 16;
  hipLaunchKernelGGL(k_wgrad, dim3(27, (S + WG_CH - 1) / WG_CH, groups), dim3(TPB), 0, st, GY, Co, X, Ci, R, S,
                     GW);
  return hipGetLastError();
}

hipError_t act_bwd(const float *g, const __bf16 *y, size_t n, int C, __bf16 *gb, float *gbias, hipStream_t st) {
  if (C > WG_MAXC) return hipErrorInvalidValue;
  const size_t per = (size_t)TPB * 16;
  hipLaunchKernelGGL(k_act_bwd, dim3((unsigned)((n + per - 1) / per)), dim3(TPB), 0, st, g, y, n, C, gb, gbias);
  return hipGetLastError();
}

hipError_t pool(const __bf16 *X, int R, int C, int N, __bf16 *Y, hipStream_t st) {
  const size_t n = (size_t)N * (R / 2) * (R / 2) * (R / 2) * C;
  hipLaunchKernelGGL(k_pool, dim3(nblk(n)), dim3(TPB), 0, st, X, R, C, n, Y);
  return hipGetLastError();
}
hipError_t pool_bwd(const float *GO, int R, int C, int N, float *GI, hipStream_t st) {
  const size_t n = (size_t)N * R * R * R * C;
  hipLaunchKernelGGL(k_pool_bwd, dim3(nblk(n)), dim3(TPB), 0, st, GO, R, C, n, GI);
  return hipGetLastError();
}
hipError_t up(const __bf16 *X, int r, int C, int N, __bf16 *Y, int Ct, int off, hipStream_t st) {
  const size_t n = (size_t)N * 8 * r * r * r * C;
  hipLaunchKernelGGL(k_up, dim3(nblk(n)), dim3(TPB), 0, st, X, r, C, Y, Ct, off, n);
  return hipGetLastError();
}
hipError_t up_bwd(const float *GO, int r, int C, int Ct, int off, int N, float *GI, hipStream_t st) {
  const size_t n = (size_t)N * r * r * r * C;
  hipLaunchKernelGGL(k_up_bwd, dim3(nblk(n)), dim3(TPB), 0, st, GO, r, C, Ct, off, n, GI);
  return hipGetLastError();
}
hipError_t copy_ch(const __bf16 *X, int C, __bf16 *Y, int Ct, int off, size_t npos, hipStream_t st) {
  const size_t n = npos * C;
  hipLaunchKernelGGL(k_copy_ch, dim3(nblk(n)), dim3(TPB), 0, st, X, C, Y, Ct, off, n);
  return hipGetLastError();
}
hipError_t copy_ch_bwd(const float *GY, int C, int Ct, int off, size_t npos, float *GX, hipStream_t st) {
  const size_t n = npos * C;
  hipLaunchKernelGGL(k_copy_ch_bwd, dim3(nblk(n)), dim3(TPB), 0, st, GY, C, Ct, off, n, GX);
  return hipGetLastError();
}
hipError_t input(const float *in, int cin, int Cp, size_t npos, __bf16 *X, hipStream_t st) {
  const size_t n = npos * Cp;
  hipLaunchKernelGGL(k_input, dim3(nblk(n)), dim3(TPB), 0, st, in, cin, Cp, n, X);
  return hipGetLastError();
}
hipError_t loss(const float *P, int Cp, const float *T, const float *Wt, int nt, size_t npos, double inv_wsum,
                float *G, double *l, hipStream_t st) {
  hipLaunchKernelGGL(k_loss, dim3(nblk(npos * Cp)), dim3(TPB), 0, st, P, Cp, T, Wt, nt, npos, inv_wsum, G, l);
  return hipGetLastError();
}
hipError_t adam(float *p, float *m, float *v, const float *g, size_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(TPB), 0, st, p, m, v, g, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t wcast(const float *w, int Co, int Ci, __bf16 *W, __bf16 *WT, hipStream_t st) {
  const size_t n = (size_t)Co * 27 * Ci;
  hipLaunchKernelGGL(k_wcast, dim3(nblk(n)), dim3(TPB), 0, st, w, Co, Ci, W, WT);
  return hipGetLastError();
}

}  // namespace unet
