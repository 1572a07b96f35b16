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

#include <algorithm>

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
// X[s + off(tap)][ci] + bias[co]).  One workgroup: 128 consecutive positions
// (M) x BN output channels.  Per K step (one tap, 32 input channels) the
// workgroup stages the 128 shifted input rows (zero outside the cube) and the
// BN weight rows in LDS; wave w then multiplies positions 32w .. 32w + 31
// (two 16-row tiles) by all BN channels (BN/16 tiles) from LDS.
// mode: 0 store bf16, 1 store f32, 2 add into f32.  Ci % 32 == 0,
// Co % BN == 0, S % 128 == 0 (host-checked).
// ---------------------------------------------------------------------------
constexpr int CV_M = 128;

template <int BN>
__global__ void __launch_bounds__(TPB) k_conv(const __bf16 *__restrict__ X, int Ci, const __bf16 *__restrict__ W,
                                              const float *__restrict__ bias, int Co, int R, int mode, int relu,
                                              void *__restrict__ out) {
  constexpr int NT = BN / 16, MT = 2;
  __shared__ bf16x8 sa[CV_M * 4];  // [position][4 chunks of 8 channels]
  __shared__ bf16x8 sb[BN * 4];    // [output channel][4 chunks]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int s_blk = blockIdx.x * CV_M;
  const int co0 = blockIdx.y * BN;
  const int R3 = R * R * R;
  // staging assignment: A chunks q = tid, tid + 256 (position q / 4, chunk q % 4)
  int a_x[2], a_y[2], a_z[2], a_base[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int s = s_blk + ((int)threadIdx.x + h * TPB) / 4;

    a_x[h] = s % R;
    a_y[h] = (s / R) % R;
    a_z[h] = (s / (R * R)) % R;
    a_base[h] = s - (s % R3);
  }
  const int a_ch = ((int)threadIdx.x % 4) * 8;
  f32x4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int tap = 0; tap < 27; ++tap) {
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const __bf16 *src[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int zz = a_z[h] + dz, yy = a_y[h] + dy, xx = a_x[h] + dx;
      const bool ok = (unsigned)zz < (unsigned)R && (unsigned)yy < (unsigned)R && (unsigned)xx < (unsigned)R;
      src[h] = ok ? X + (size_t)(a_base[h] + (zz * R + yy) * R + xx) * Ci + a_ch : nullptr;
    }
    for (int c0 = 0; c0 < Ci; c0 += 32) {
      __syncthreads();  // the previous step's tiles are consumed
#pragma unroll
      for (int h = 0; h < 2; ++h)
        sa[threadIdx.x + h * TPB] = src[h] ? *reinterpret_cast<const bf16x8 *>(src[h] + c0) : zero8();
      for (int q = threadIdx.x; q < BN * 4; q += TPB)
        sb[q] = *reinterpret_cast<const bf16x8 *>(W + ((size_t)(co0 + q / 4) * 27 + tap) * Ci + c0 + (q % 4) * 8);
      __syncthreads();
      bf16x8 a[MT], b[NT];
#pragma unroll
      for (int i = 0; i < MT; ++i) a[i] = sa[(wave * 32 + i * 16 + m) * 4 + kq];
#pragma unroll
      for (int j = 0; j < NT; ++j) b[j] = sb[(j * 16 + m) * 4 + kq];
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int co = co0 + j * 16 + m;
    const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t o = (size_t)(s_blk + wave * 32 + i * 16 + 4 * kq + r) * Co + co;
        float v = acc[i][j][r] + bv;
        if (relu) v = fmaxf(v, 0.0f);
        if (mode == 0) static_cast<__bf16 *>(out)[o] = (__bf16)v;
        else if (mode == 1) static_cast<float *>(out)[o] = v;
        else static_cast<float *>(out)[o] += v;
      }
  }
}

// ---------------------------------------------------------------------------
// the same convolution for cubes of side R = 16, 32 or 64 and at least 96
// input channels (used there only: with one or two 32-channel chunks the
// per-tap staging of k_conv, with its weights in LDS, is faster), where a block's
// 128 positions are 128 / R whole x rows of one z plane: per 32 input
// channels the workgroup stages the block's halo once (3 planes x (128/R + 2)
// rows x (R + 2) positions, zero outside the cube) and every tap reads its
// shifted rows from it; the weight fragments come straight from global
// memory (the layer's weights stay in L2).  The K steps run chunk-major,
// taps inside, which for Ci = 32 is the order k_conv takes.
// ---------------------------------------------------------------------------
constexpr int CH_ROWS = 3 * (128 / 64 + 2) * (64 + 2);  // largest halo (R = 64)

template <int BN>
__global__ void __launch_bounds__(TPB) k_conv_halo(const __bf16 *__restrict__ X, int Ci,
                                                   const __bf16 *__restrict__ W, const float *__restrict__ bias,
                                                   int Co, int R, int mode, int relu, void *__restrict__ out) {
  constexpr int NT = BN / 16, MT = 2;
  __shared__ bf16x8 sh[CH_ROWS * 4];  // [halo row][4 chunks of 8 channels]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int s_blk = blockIdx.x * CV_M;
  const int co0 = blockIdx.y * BN;
  const int R2 = R * R, R3 = R2 * R;
  const int YH = CV_M / R + 2, XH = R + 2, nrow = 3 * YH * XH;
  const int base = s_blk - s_blk % R3;  // first position of this sample
  const int z0 = (s_blk % R3) / R2, y0 = (s_blk % R2) / R;
  // halo row of each MFMA row at tap (0, 0, 0), less the tap's offset
  int hrow[MT];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    const int p = wave * 32 + i * 16 + m;
    hrow[i] = (p / R) * XH + p % R;
  }
  f32x4 acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int c0 = 0; c0 < Ci; c0 += 32) {
    __syncthreads();  // the previous chunk's halo is consumed
    for (int u = threadIdx.x; u < nrow * 4; u += TPB) {
      const int row = u / 4, a = row / (YH * XH), b = (row / XH) % YH, c = row % XH;
      const int z = z0 + a - 1, y = y0 + b - 1, x = c - 1;
      const bool ok = (unsigned)z < (unsigned)R && (unsigned)y < (unsigned)R && (unsigned)x < (unsigned)R;
      sh[u] = ok ? *reinterpret_cast<const bf16x8 *>(X + (size_t)(base + (z * R + y) * R + x) * Ci + c0 + (u % 4) * 8)
                 : zero8();
    }
    __syncthreads();
    for (int tap = 0; tap < 27; ++tap) {
      const int hz = tap / 9, hy = (tap / 3) % 3, hx = tap % 3;  // offsets + 1
      const int off = (hz * YH + hy) * XH + hx;
      bf16x8 a[MT], b[NT];
#pragma unroll
      for (int j = 0; j < NT; ++j)
        b[j] = *reinterpret_cast<const bf16x8 *>(W + ((size_t)(co0 + j * 16 + m) * 27 + tap) * Ci + c0 + kq * 8);
#pragma unroll
      for (int i = 0; i < MT; ++i) a[i] = sh[(hrow[i] + off) * 4 + kq];
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    const int co = co0 + j * 16 + m;
    const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t o = (size_t)(s_blk + wave * 32 + i * 16 + 4 * kq + r) * Co + co;
        float v = acc[i][j][r] + bv;
        if (relu) v = fmaxf(v, 0.0f);
        if (mode == 0) static_cast<__bf16 *>(out)[o] = (__bf16)v;
        else if (mode == 1) static_cast<float *>(out)[o] = v;
        else static_cast<float *>(out)[o] += v;
      }
  }
}

// ---------------------------------------------------------------------------
// weight gradient, one partial per chunk of positions:
// gWp[chunk][co][tap][ci] = sum over the chunk's s of gY[s][co] X[s + off(tap)][ci]
// (k_colsum then adds the chunks in a fixed order, so the result does not
// depend on the order in which workgroups run).
// Work items (27 taps, chunks of L positions, groups of 16 output tiles of
// 16 x 16) on a 1-D grid, XCD-aware: workgroups are dispatched round-robin
// over the 8 XCDs, and every item of chunk c runs on XCD c % 8, so the 27
// taps and all groups of a chunk, which read the same gY rows and
// overlapping X rows, share that XCD's L2.  Per step of K positions the
// workgroup stages gY and, of the shifted X rows, the input channels of its
// group in LDS: group g takes input-channel tiles g itg .. g itg + itg - 1
// with every output-channel tile (at most 16 tiles), and wave w owns the
// group's tiles w + 4 t, t < 4.
// ---------------------------------------------------------------------------
constexpr int WG_XCD = 8;
constexpr int WG_CH = 2048;  // positions per workgroup, at least
constexpr int WG_NC = 256;   // chunks per launch, at most
constexpr int WG_MAXT = 4;   // tiles per wave
constexpr int WG_MAXC = 224; // largest channel count staged

constexpr int WG_K = 64;  // positions staged per step (128 for narrow layers)

// LDS row stride (bf16) of a staged [position][channel] tile: 16 x an odd
// number, so that eight consecutive rows start in eight different 32-byte
// bank groups and the transposing fragment reads below are conflict-free
__host__ __device__ constexpr int wg_stride(int C) { return (C / 16) % 2 ? C : C + 16; }

typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

// 16 x 16 x 32 MFMA operand fragment from a [position][channel] LDS tile:
// lane (m, kq) receives channel c0 + m at 8 positions, those of rows
// row0 + 4 kq + e and row0 + 16 + 4 kq + e (e < 4).  Each transposing read
// (ds_read_b64_tr_b16) serves 16 lanes: lane j of the group points at row
// j / 4, channels 4 (j % 4) .. +3, and lane n of the group gets channel n of
// those 4 rows.  A and B are read with the same rows, so every slot of the
// contraction pairs the same position.
__device__ inline bf16x8 wg_frag(const __bf16 *t, int stride, int row0, int c0, int lane) {
  const int m = lane & 15, kq = lane >> 4;
  const __bf16 *p = t + (size_t)(row0 + 4 * kq + (m >> 2)) * stride + c0 + 4 * (m & 3);
  typedef __attribute__((address_space(3))) i16x4 lds_i16x4;
  const i16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4 *)(p));
  const i16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4 *)(p + (size_t)16 * stride));
  return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

template <int K>
__global__ void __launch_bounds__(TPB) k_wgrad(const __bf16 *__restrict__ GY, int Co,
                                               const __bf16 *__restrict__ X, int Ci, int R, int S, int L,
                                               int ncl, int groups, int itg, float *__restrict__ GWp) {
  // tiles [K positions][channel] as they lie in memory, staged with one
  // 16-byte global load and one 16-byte LDS write per 8 channels of a
  // position; the MFMA fragments are read transposed (wg_frag)
  extern __shared__ __attribute__((aligned(16))) __bf16 wg_lds[];  // K rows of SG, then of SX
  const int SG = wg_stride(Co), SX = wg_stride(min(Ci, 16 * itg));
  __bf16 *sg = wg_lds, *sx = wg_lds + (size_t)K * SG;
  // work item of this workgroup: XCD blockIdx.x % 8 takes chunks of that
  // residue, taps fastest, then groups
  const int xcd = (int)blockIdx.x % WG_XCD, k = (int)blockIdx.x / WG_XCD;
  const int chunk = (k / (27 * groups)) * WG_XCD + xcd;
  if (chunk >= ncl) return;  // whole workgroup: no barrier reached
  const int group = (k / 27) % groups, tap = k % 27;
  const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  // group g: input-channel tiles it0 .. it0 + itn - 1 with every output-channel
  // tile (at most 16 tiles), so it stages only those itn * 16 input channels
  const int it0 = group * itg, itn = min(itg, Ci / 16 - it0), ntile = (Co / 16) * itn;
  const int R3 = R * R * R;
  f32x4 acc[WG_MAXT];
#pragma unroll
  for (int t = 0; t < WG_MAXT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int p0 = chunk * L, p1 = min(S, p0 + L);
  const int r = (int)threadIdx.x % K;  // this thread's staged position
  for (int sb = p0; sb < p1; sb += K) {
    __syncthreads();
    const int s = sb + r;
    for (int q = (int)threadIdx.x / K; q < Co / 8; q += TPB / K)
      *reinterpret_cast<bf16x8 *>(sg + r * SG + 8 * q) =
          *reinterpret_cast<const bf16x8 *>(GY + (size_t)s * Co + 8 * q);
    const int x = s % R + dx, y = (s / R) % R + dy, z = (s / (R * R)) % R + dz;
    const bool ok = (unsigned)x < (unsigned)R && (unsigned)y < (unsigned)R && (unsigned)z < (unsigned)R;
    const __bf16 *xs = X + (size_t)(ok ? s - (s % R3) + (z * R + y) * R + x : 0) * Ci + 16 * it0;
    for (int q = (int)threadIdx.x / K; q < 2 * itn; q += TPB / K)
      *reinterpret_cast<bf16x8 *>(sx + r * SX + 8 * q) =
          ok ? *reinterpret_cast<const bf16x8 *>(xs + 8 * q) : zero8();
    __syncthreads();
#pragma unroll
    for (int t = 0; t < WG_MAXT; ++t) {
      const int tile = wave + 4 * t;
      if (tile < ntile) {
        const int ct = tile / itn, it = tile % itn;
#pragma unroll
        for (int ks = 0; ks < K / 32; ++ks) {
          // A[m = co][k = position], B[k = position][n = ci]
          const bf16x8 a = wg_frag(sg, SG, 32 * ks, ct * 16, lane);
          const bf16x8 b = wg_frag(sx, SX, 32 * ks, it * 16, lane);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < WG_MAXT; ++t) {
    const int tile = wave + 4 * t;
    if (tile < ntile) {
      const int ct = tile / itn, it = tile % itn;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = ct * 16 + 4 * kq + i, ci = (it0 + it) * 16 + m;
        GWp[(size_t)chunk * Co * 27 * Ci + ((size_t)co * 27 + tap) * Ci + ci] = acc[t][i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// elementwise and reductions
// ---------------------------------------------------------------------------
// bf16 gradient of a pre-activation from the f32 gradient of the layer
// output (ReLU mask from the stored output y when y is given) and this
// block's share of the bias gradient (sum over positions).  C % 8 == 0
// (host-checked); thread t < (TPB / C8) C8 always moves channel group
// t % C8 (8 channels) of positions t / C8 + k TPB / C8 of the block's range,
// adds them in position order, and the block adds its threads' sums in
// thread order into part[block][C]; k_colsum adds the blocks in order.
__global__ void __launch_bounds__(TPB) k_act_bwd(const float *__restrict__ g, const __bf16 *__restrict__ y,
                                                 size_t npos, int C, int pos_per_block, __bf16 *__restrict__ gb,
                                                 float *__restrict__ part) {
  __shared__ float sb[TPB][8];
  const int C8 = C / 8, per_round = TPB / C8;
  const int cg = (int)threadIdx.x % C8, q = (int)threadIdx.x / C8;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (q < per_round) {
    const size_t s0 = (size_t)blockIdx.x * pos_per_block;
    const size_t s1 = min(npos, s0 + (size_t)pos_per_block);
    for (size_t s = s0 + q; s < s1; s += per_round) {
      const size_t e = s * C8 + cg;
      const f32x4 v0 = *reinterpret_cast<const f32x4 *>(g + 8 * e);
      const f32x4 v1 = *reinterpret_cast<const f32x4 *>(g + 8 * e + 4);
      float v[8] = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
      if (y) {
        const bf16x8 yy = *reinterpret_cast<const bf16x8 *>(y + 8 * e);
#pragma unroll
        for (int i = 0; i < 8; ++i)
          if (!((float)yy[i] > 0.0f)) v[i] = 0.0f;
      }
      bf16x8 o;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        o[i] = (__bf16)v[i];
        acc[i] += v[i];
      }
      *reinterpret_cast<bf16x8 *>(gb + 8 * e) = o;
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) sb[threadIdx.x][i] = acc[i];
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += TPB) {
    float sum = 0.0f;
    for (int k = 0; k < per_round; ++k) sum += sb[k * C8 + c / 8][c % 8];
    part[(size_t)blockIdx.x * C + c] = sum;
  }
}

// out[col] = sum over rows r of P[r][col] in a fixed association: CW
// columns per workgroup, TPB / CW row classes per column (class k adds rows
// k, k + TPB/CW, ... in order), the classes then added in class order.  CW =
// 64 for wide matrices (few rows: weight-gradient chunks), CW = 8 for narrow
// ones (many rows: the bias partials of many blocks).
template <int CW>
__global__ void __launch_bounds__(TPB) k_colsum(const float *__restrict__ P, int nrow, size_t ncol,
                                                float *__restrict__ out) {
  constexpr int NCLS = TPB / CW;
  __shared__ float sh[NCLS][CW];
  const int lc = (int)threadIdx.x % CW, cls = (int)threadIdx.x / CW;
  const size_t col = (size_t)blockIdx.x * CW + lc;
  float sum = 0.0f;
  if (col < ncol)
    for (int r = cls; r < nrow; r += NCLS) sum += P[(size_t)r * ncol + col];
  sh[cls][lc] = sum;
  __syncthreads();
  if (cls == 0 && col < ncol) {
    float t = sh[0][lc];
    for (int k = 1; k < NCLS; ++k) t += sh[k][lc];
    out[col] = t;
  }
}

static void colsum(const float *P, int nrow, size_t ncol, float *out, hipStream_t st) {
  if (ncol >= 64 * 256)
    hipLaunchKernelGGL(k_colsum<64>, dim3((unsigned)((ncol + 63) / 64)), dim3(TPB), 0, st, P, nrow, ncol, out);
  else
    hipLaunchKernelGGL(k_colsum<8>, dim3((unsigned)((ncol + 7) / 8)), dim3(TPB), 0, st, P, nrow, ncol, out);
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
__global__ void k_pool_bwd(const float *__restrict__ GO, int R, int C, size_t n_in8, float *__restrict__ GI) {
  // one thread per (input position, 8 channels); C % 8 == 0 (host-checked)
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n_in8) return;
  const int r = R / 2, C8 = C / 8;
  const int c = 8 * (int)(e % C8);
  const size_t p = e / C8;
  const int x = (int)(p % R), y = (int)((p / R) % R), z = (int)((p / ((size_t)R * R)) % R);
  const size_t b = p / ((size_t)R * R * R);
  const float *q = GO + (((b * r + z / 2) * r + y / 2) * r + x / 2) * (size_t)C + c;
  f32x4 *o = reinterpret_cast<f32x4 *>(GI + p * C + c);
  o[0] += 0.125f * *reinterpret_cast<const f32x4 *>(q);
  o[1] += 0.125f * *reinterpret_cast<const f32x4 *>(q + 4);
}

// nearest 2x upsampling, edge r -> R = 2r, into channels off .. off + C - 1
// of a Ct-channel tensor; one thread per (output position, 8 channels)
// (C, Ct and off multiples of 8, host-checked: 16-byte moves)
__global__ void k_up(const __bf16 *__restrict__ X, int r, int C, __bf16 *__restrict__ Y, int Ct, int off,
                     size_t n_out8) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n_out8) return;
  const int R = 2 * r, C8 = C / 8;
  const int c = 8 * (int)(e % C8);
  const size_t p = e / C8;
  const int x = (int)(p % R), y = (int)((p / R) % R), z = (int)((p / ((size_t)R * R)) % R);
  const size_t b = p / ((size_t)R * R * R);
  const bf16x8 v = *reinterpret_cast<const bf16x8 *>(X + (((b * r + z / 2) * r + y / 2) * r + x / 2) * (size_t)C + c);
  *reinterpret_cast<bf16x8 *>(Y + p * Ct + off + c) = v;
}
// its adjoint: G_in (edge r, C) = sum of the 8 children's G_out[.., off + c],
// one thread per (input position, 8 channels)
__global__ void k_up_bwd(const float *__restrict__ GO, int r, int C, int Ct, int off, size_t n_in8,
                         float *__restrict__ GI) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n_in8) return;
  const int R = 2 * r, C8 = C / 8;
  const int c = 8 * (int)(e % C8);
  const size_t p = e / C8;
  const int x = (int)(p % r), y = (int)((p / r) % r), z = (int)((p / ((size_t)r * r)) % r);
  const size_t b = p / ((size_t)r * r * r);
  f32x4 s0 = {0.0f, 0.0f, 0.0f, 0.0f}, s1 = s0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int zz = 2 * z + (k >> 2), yy = 2 * y + ((k >> 1) & 1), xx = 2 * x + (k & 1);
    const float *q = GO + (((b * R + zz) * R + yy) * (size_t)R + xx) * Ct + off + c;
    s0 += *reinterpret_cast<const f32x4 *>(q);
    s1 += *reinterpret_cast<const f32x4 *>(q + 4);
  }
  float *o = GI + p * C + c;
  *reinterpret_cast<f32x4 *>(o) = s0;
  *reinterpret_cast<f32x4 *>(o + 4) = s1;
}

// channel copy X (C) -> Y[.., off + c] (Ct channels), and its adjoint (+=);
// one thread per (position, 8 channels), C, Ct and off multiples of 8
// (host-checked)
__global__ void k_copy_ch(const __bf16 *__restrict__ X, int C, __bf16 *__restrict__ Y, int Ct, int off, size_t n8) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n8) return;
  const int C8 = C / 8;
  const size_t p = e / C8;
  const int c = 8 * (int)(e % C8);
  *reinterpret_cast<bf16x8 *>(Y + p * Ct + off + c) = *reinterpret_cast<const bf16x8 *>(X + p * C + c);
}
__global__ void k_copy_ch_bwd(const float *__restrict__ GY, int C, int Ct, int off, size_t n8,
                              float *__restrict__ GX) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n8) return;
  const int C8 = C / 8;
  const size_t p = e / C8;
  const int c = 8 * (int)(e % C8);
  const float *q = GY + p * Ct + off + c;
  f32x4 *o = reinterpret_cast<f32x4 *>(GX + p * C + c);
  o[0] += *reinterpret_cast<const f32x4 *>(q);
  o[1] += *reinterpret_cast<const f32x4 *>(q + 4);
}

// network input: f32 [s][cin] -> bf16 [s][Cp] zero-padded
__global__ void k_input(const float *__restrict__ in, int cin, int Cp, size_t n, __bf16 *__restrict__ X) {
  const size_t e = (size_t)blockIdx.x * TPB + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e % Cp);
  X[e] = (__bf16)(c < cin ? in[(e / Cp) * cin + c] : 0.0f);
}

// weighted squared error: out f32 [s][Cp] (first nt used), target and weight
// f32 [s][nt]; loss = sum w (p - t)^2 / wsum, gradient into G [s][Cp]; each
// block's share of the sum into part[block] (k_loss_sum adds them in order)
__global__ void __launch_bounds__(TPB) k_loss(const float *__restrict__ P, int Cp, const float *__restrict__ T,
                                              const float *__restrict__ Wt, int nt, size_t npos, double inv_wsum,
                                              float *__restrict__ G, double *__restrict__ part) {
  __shared__ double sh[TPB];
  double l = 0.0;
  const size_t n = npos * Cp;
  for (size_t e = (size_t)blockIdx.x * TPB + threadIdx.x; e < n; e += (size_t)gridDim.x * TPB) {
    const size_t s = e / Cp;
    const int c = (int)(e % Cp);
    float g = 0.0f;
    if (c < nt) {
      const float d = P[e] - T[s * nt + c], w = Wt[s * nt + c];
      l += (double)w * d * d;
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
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
// loss = inv_wsum * (sum of the blocks' partials): thread t adds partials
// t, t + TPB, ... in order, then the threads' sums are added pairwise in a
// fixed tree
__global__ void __launch_bounds__(TPB) k_loss_sum(const double *__restrict__ part, int nb, double inv_wsum,
                                                  double *__restrict__ loss) {
  __shared__ double sh[TPB];
  double l = 0.0;
  for (int b = (int)threadIdx.x; b < nb; b += TPB) l += part[b];
  sh[threadIdx.x] = l;
  __syncthreads();
  for (int k = TPB / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sh[0] * inv_wsum;
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
  if (Ci % 32 || Co % 32 || S % CV_M) return hipErrorInvalidValue;
  if (Co % 64 && Ci >= 96 && (R == 16 || R == 32 || R == 64))  // three or more 32-channel chunks
    hipLaunchKernelGGL(k_conv_halo<32>, dim3(S / CV_M, Co / 32), dim3(TPB), 0, st, X, Ci, W, bias, Co, R, mode,
                       relu, out);
  else if (Co % 64 == 0)
    hipLaunchKernelGGL(k_conv<64>, dim3(S / CV_M, Co / 64), dim3(TPB), 0, st, X, Ci, W, bias, Co, R, mode, relu,
                       out);
  else
    hipLaunchKernelGGL(k_conv<32>, dim3(S / CV_M, Co / 32), dim3(TPB), 0, st, X, Ci, W, bias, Co, R, mode, relu,
                       out);
  return hipGetLastError();
}

int wgrad_chunks(int R, int N) {
  const int S = N * R * R * R;
  return std::min(WG_NC, (S + WG_CH - 1) / WG_CH);
}

template <int K>
static void wgrad_launch(const __bf16 *GY, int Co, const __bf16 *X, int Ci, int R, int S, int nc, int groups,
                         int itg, float *part, int *ncl_out, hipStream_t st) {
  const size_t lds = (size_t)K * (wg_stride(Co) + wg_stride(std::min(Ci, 16 * itg))) * sizeof(__bf16);
  const int L = ((S + nc - 1) / nc + K - 1) / K * K;  // chunk length, whole staging steps
  const int ncl = (S + L - 1) / L;
  const int per_xcd = (ncl + WG_XCD - 1) / WG_XCD;  // chunks per XCD, at most
  hipLaunchKernelGGL(k_wgrad<K>, dim3(WG_XCD * per_xcd * 27 * groups), dim3(TPB), lds, st, GY, Co, X, Ci, R, S, L,
                     ncl, groups, itg, part);
  *ncl_out = ncl;
}

hipError_t wgrad(const __bf16 *GY, int Co, const __bf16 *X, int Ci, int R, int N, float *GW, float *part,
                 hipStream_t st) {
  const int S = N * R * R * R;
  if (Ci % 16 || Co % 16 || Ci > WG_MAXC || Co > WG_MAXC || S % WG_K) return hipErrorInvalidValue;
  // tile groups: itg input-channel tiles with every output-channel tile each
  const int itg = std::max(1, 16 / (Co / 16)), groups = (Ci / 16 + itg - 1) / itg;
  const int nc = wgrad_chunks(R, N);
  int ncl;
  if (Co + Ci <= 64 && S % (2 * WG_K) == 0)
    wgrad_launch<2 * WG_K>(GY, Co, X, Ci, R, S, nc, groups, itg, part, &ncl, st);
  else
    wgrad_launch<WG_K>(GY, Co, X, Ci, R, S, nc, groups, itg, part, &ncl, st);
  const size_t nw = (size_t)Co * 27 * Ci;
  colsum(part, ncl, nw, GW, st);
  return hipGetLastError();
}

int act_bwd_blocks(size_t n, int C) {
  const int C8 = C / 8, pos_per_block = TPB / C8 * 16;
  return (int)((n / C + pos_per_block - 1) / pos_per_block);
}

hipError_t act_bwd(const float *g, const __bf16 *y, size_t n, int C, __bf16 *gb, float *gbias, float *part,
                   hipStream_t st) {
  if (C > WG_MAXC || C % 8 || n % C) return hipErrorInvalidValue;
  const int C8 = C / 8, pos_per_block = TPB / C8 * 16;  // 16 positions per active thread
  const int nb = act_bwd_blocks(n, C);
  hipLaunchKernelGGL(k_act_bwd, dim3(nb), dim3(TPB), 0, st, g, y, n / C, C, pos_per_block, gb, part);
  colsum(part, nb, (size_t)C, gbias, st);
  return hipGetLastError();
}

hipError_t pool(const __bf16 *X, int R, int C, int N, __bf16 *Y, hipStream_t st) {
  const size_t n = (size_t)N * (R / 2) * (R / 2) * (R / 2) * C;
  hipLaunchKernelGGL(k_pool, dim3(nblk(n)), dim3(TPB), 0, st, X, R, C, n, Y);
  return hipGetLastError();
}
hipError_t pool_bwd(const float *GO, int R, int C, int N, float *GI, hipStream_t st) {
  if (C % 8) return hipErrorInvalidValue;
  const size_t n8 = (size_t)N * R * R * R * (C / 8);
  hipLaunchKernelGGL(k_pool_bwd, dim3(nblk(n8)), dim3(TPB), 0, st, GO, R, C, n8, GI);
  return hipGetLastError();
}
hipError_t up(const __bf16 *X, int r, int C, int N, __bf16 *Y, int Ct, int off, hipStream_t st) {
  if (C % 8 || Ct % 8 || off % 8) return hipErrorInvalidValue;
  const size_t n8 = (size_t)N * 8 * r * r * r * (C / 8);
  hipLaunchKernelGGL(k_up, dim3(nblk(n8)), dim3(TPB), 0, st, X, r, C, Y, Ct, off, n8);
  return hipGetLastError();
}
hipError_t up_bwd(const float *GO, int r, int C, int Ct, int off, int N, float *GI, hipStream_t st) {
  if (C % 8 || Ct % 8 || off % 8) return hipErrorInvalidValue;
  const size_t n8 = (size_t)N * r * r * r * (C / 8);
  hipLaunchKernelGGL(k_up_bwd, dim3(nblk(n8)), dim3(TPB), 0, st, GO, r, C, Ct, off, n8, GI);
  return hipGetLastError();
}
hipError_t copy_ch(const __bf16 *X, int C, __bf16 *Y, int Ct, int off, size_t npos, hipStream_t st) {
  if (C % 8 || Ct % 8 || off % 8) return hipErrorInvalidValue;
  const size_t n8 = npos * (C / 8);
  hipLaunchKernelGGL(k_copy_ch, dim3(nblk(n8)), dim3(TPB), 0, st, X, C, Y, Ct, off, n8);
  return hipGetLastError();
}
hipError_t copy_ch_bwd(const float *GY, int C, int Ct, int off, size_t npos, float *GX, hipStream_t st) {
  if (C % 8 || Ct % 8 || off % 8) return hipErrorInvalidValue;
  const size_t n8 = npos * (C / 8);
  hipLaunchKernelGGL(k_copy_ch_bwd, dim3(nblk(n8)), dim3(TPB), 0, st, GY, C, Ct, off, n8, GX);
  return hipGetLastError();
}
hipError_t input(const float *in, int cin, int Cp, size_t npos, __bf16 *X, hipStream_t st) {
  const size_t n = npos * Cp;
  hipLaunchKernelGGL(k_input, dim3(nblk(n)), dim3(TPB), 0, st, in, cin, Cp, n, X);
  return hipGetLastError();
}
hipError_t loss(const float *P, int Cp, const float *T, const float *Wt, int nt, size_t npos, double inv_wsum,
                float *G, double *l, double *part, hipStream_t st) {
  const unsigned g = std::min(nblk(npos * Cp), (unsigned)LOSS_BLOCKS);  // grid-stride
  hipLaunchKernelGGL(k_loss, dim3(g), dim3(TPB), 0, st, P, Cp, T, Wt, nt, npos, inv_wsum, G, part);
  hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(TPB), 0, st, part, (int)g, inv_wsum, l);
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
