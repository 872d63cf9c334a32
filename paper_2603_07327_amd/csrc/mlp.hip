// mlp.hip -- the surrogate network on gfx950 matrix cores: a ReLU MLP with
// BF16 weights and activations, FP32 accumulation (v_mfma_f32_16x16x32_bf16),
// softmax cross-entropy, backpropagation and Adam on FP32 master weights.
//
// All matrix products go through one LDS-tiled kernel: a 256-lane block
// computes a 64 x 64 tile of C = A B with 4 waves of 32 x 32 (2 x 2 MFMA tiles
// of 16 x 16), stepping K by 32.  Operands are staged in LDS K-contiguous, so
// each lane feeds an MFMA with one 16-byte LDS read per operand; operands that
// are K-strided in memory (the transposes of the backward pass) are transposed
// on their way into LDS.  Rows are padded to multiples of 256, layer widths
// to 128 and the input width to 64; padded weights and biases are zero and
// padded rows carry zero gradient.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gpet_internal.hpp"

namespace gpet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;     // input width padding
constexpr int kRowPad = 256;   // padding of rows (256-row product tiles)
constexpr int kWidthPad = 128; // padding of layer widths (128-column product tiles)
constexpr int kTk = 32;
// bf16 per LDS row: with 16 of padding the products' LDS bank-conflict
// cycles are half those with 8 or 24
constexpr int kLdsRow = kTk + 16;
constexpr int kTableSlices = 16; // row slices of the offset-table gradient

// float -> bfloat16 bits, round to nearest even
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

enum : int { EPI_BIAS_RELU_BF16 = 0, EPI_BIAS_F32 = 1, EPI_F32 = 2, EPI_MASK_HILO = 3, EPI_BIAS_F32_STATS = 4 };

// C[m][n] = sum_k A(m, k) B(k, n) over a padded problem (M a multiple of BM,
// N of BN, K of 32).  A(m, k) = a[m lda + k] (AT: a[k lda + m]);
// B(k, n) = b[n ldb + k] (BT: b[k ldb + n]).  Four waves in a 2 x 2 grid,
// each computing a (BM / 2) x (BN / 2) block of 16 x 16 MFMA tiles; the
// next K step's operands are loaded into registers while the current one is
// multiplied.  Epilogue per EPI.
//
// Two-term operands (k_half > 0): the backward pass keeps each gradient as
// hi + lo, two BF16 planes a_lo elements apart (hi = bf16(g), lo =
// bf16(g - hi)), so its products keep FP32-like precision on the BF16
// matrix cores.  Then K = 2 k_half: steps k >= k_half read the lo plane at
// k - k_half and B again at k - k_half, so C = (hi + lo) B in one pass.
template <int BM, int BN, bool AT, bool BT, int EPI>
__global__ void __launch_bounds__(256) k_gemm(const uint16_t *__restrict__ a, int lda, const uint16_t *__restrict__ b,
                                              int ldb, int K, const float *__restrict__ bias,
                                              const uint16_t *__restrict__ mask, void *__restrict__ out, int ldc,
                                              size_t split_stride, size_t a_lo, int k_half) {
  // split K: slice z covers [z K, (z + 1) K) and writes its partial product
  // split_stride elements further on (EPI_F32); EPI_MASK_HILO writes the lo
  // plane of its result split_stride elements after the hi plane
  const int kz = blockIdx.z * K;
  if constexpr (EPI == EPI_F32) out = (float *)out + blockIdx.z * split_stride;
  constexpr int TM = BM / 32, TN = BN / 32; // MFMA tiles per wave and axis
  constexpr int PA = BM / 64, PB = BN / 64; // 16-byte loads per thread and operand
  __shared__ __attribute__((aligned(16))) uint16_t sa[BM * kLdsRow];
  __shared__ __attribute__((aligned(16))) uint16_t sb[BN * kLdsRow];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  floatx4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  uint4 ra[PA], rb[PB];
  // global -> registers for the K step at k0 of this slice
  auto load = [&](int k0) {
    const int kg = kz + k0;
    const bool lo = k_half > 0 && kg >= k_half; // a step never straddles k_half (a multiple of 32)
    const int kk = lo ? kg - k_half : kg;
    const uint16_t *ap = lo ? a + a_lo : a;
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      const int t = tid + 256 * p;
      if constexpr (!AT) ra[p] = *(const uint4 *)&ap[(size_t)(m0 + (t >> 2)) * lda + kk + (t & 3) * 8];
      else ra[p] = *(const uint4 *)&ap[(size_t)(kk + t / (BM / 8)) * lda + m0 + (t % (BM / 8)) * 8];
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      const int t = tid + 256 * p;
      if constexpr (!BT) rb[p] = *(const uint4 *)&b[(size_t)(n0 + (t >> 2)) * ldb + kk + (t & 3) * 8];
      else rb[p] = *(const uint4 *)&b[(size_t)(kk + t / (BN / 8)) * ldb + n0 + (t % (BN / 8)) * 8];
    }
  };
  // registers -> LDS, K-contiguous rows
  auto store = [&]() {
#pragma unroll
    for (int p = 0; p < PA; ++p) {
      const int t = tid + 256 * p;
      if constexpr (!AT) {
        *(uint4 *)&sa[(t >> 2) * kLdsRow + (t & 3) * 8] = ra[p];
      } else {
        const int kk = t / (BM / 8), c = (t % (BM / 8)) * 8;
        const uint16_t *e = (const uint16_t *)&ra[p];
#pragma unroll
        for (int j = 0; j < 8; ++j) sa[(c + j) * kLdsRow + kk] = e[j];
      }
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      const int t = tid + 256 * p;
      if constexpr (!BT) {
        *(uint4 *)&sb[(t >> 2) * kLdsRow + (t & 3) * 8] = rb[p];
      } else {
        const int kk = t / (BN / 8), c = (t % (BN / 8)) * 8;
        const uint16_t *e = (const uint16_t *)&rb[p];
#pragma unroll
        for (int j = 0; j < 8; ++j) sb[(c + j) * kLdsRow + kk] = e[j];
      }
    }
  };
  load(0);
  store();
  __syncthreads();
  const int lr = lane & 15, lk = (lane >> 4) * 8; // lane l: row/column l % 16, k = 8 (l / 16) .. + 8
  for (int k0 = 0; k0 < K; k0 += kTk) {
    const bool more = k0 + kTk < K;
    if (more) load(k0 + kTk);
    bf16x8 fa[TM], fb[TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
      fa[i] = __builtin_bit_cast(bf16x8, *(const uint4 *)&sa[(wm + 16 * i + lr) * kLdsRow + lk]);
#pragma unroll
    for (int j = 0; j < TN; ++j)
      fb[j] = __builtin_bit_cast(bf16x8, *(const uint4 *)&sb[(wn + 16 * j + lr) * kLdsRow + lk]);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    __syncthreads();
    if (more) {
      store();
      __syncthreads();
    }
  }
  // ---- epilogue: lane l holds column l % 16, rows 4 (l / 16) .. + 4 of each tile
  const int cn = lane & 15, rb4 = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm + 16 * i + rb4 + q, n = n0 + wn + 16 * j + cn;
        const float v = acc[i][j][q];
        const size_t o = (size_t)m * ldc + n;
        if constexpr (EPI == EPI_BIAS_RELU_BF16) {
          ((uint16_t *)out)[o] = f2bf(fmaxf(v + bias[n], 0.0f));
        } else if constexpr (EPI == EPI_BIAS_F32) {
          ((float *)out)[o] = v + bias[n];
        } else if constexpr (EPI == EPI_F32) {
          ((float *)out)[o] = v;
        } else { // masked by the ReLU of the layer input, kept as hi + lo
          const float g = bf2f(mask[o]) > 0.0f ? v : 0.0f;
          const uint16_t hi = f2bf(g);
          ((uint16_t *)out)[o] = hi;
          ((uint16_t *)out)[o + split_stride] = f2bf(g - bf2f(hi));
        }
      }
}

// The forward products (both operands K-contiguous, K <= 256): a 256 x 128
// block of 8 waves (64 x 64 each) keeps its whole 128-column slab of the
// weights in LDS for the full K and streams the activations through a
// double-buffered 256 x 32 LDS stage (one barrier per K step), the next
// stage's rows loaded into registers while the current one is multiplied.
constexpr int kNtKmax = 256;
constexpr int kNtRowB = kNtKmax + 16; // bf16 per weight-slab row in LDS
constexpr size_t kNtLds = (size_t)(128 * kNtRowB + 2 * 256 * kLdsRow) * sizeof(uint16_t);

// EPI_BIAS_F32_STATS also writes, per row and 128-column block, the maximum
// of the logits of the columns below n_valid and the sum of their exponentials
// relative to it: stats[row * gridDim.x + block column] = (max, sum).
// Blocks go to the 8 XCDs in turn (block L to XCD L mod 8), and each XCD has
// its own L2: the 1-D grid is mapped so that the column blocks of one 256-row
// block run on one XCD, one after the other, and its activation rows are
// fetched from HBM once per XCD instead of once per column block.
__device__ __forceinline__ void xcd_tile(uint32_t L, uint32_t total, uint32_t nbx, uint32_t &bx, uint32_t &by) {
  const uint32_t x = L % 8u, slot = L / 8u;
  uint32_t base = 0; // blocks of the XCDs before x: XCD y has (total + 7 - y) / 8
  for (uint32_t y = 0; y < x; ++y) base += (total + 7u - y) / 8u;
  const uint32_t v = base + slot;
  by = v / nbx;
  bx = v - by * nbx;
}

template <int EPI>
__global__ void __launch_bounds__(512) k_gemm_nt(const uint16_t *__restrict__ a, int lda,
                                                 const uint16_t *__restrict__ b, int ldb, int K,
                                                 const float *__restrict__ bias, void *__restrict__ out, int ldc,
                                                 float2 *__restrict__ stats, int n_valid, int nbx) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds_nt[];
  uint16_t *sbw = lds_nt;                   // 128 x kNtRowB weight slab
  uint16_t *sac = lds_nt + 128 * kNtRowB;   // 2 x 256 x kLdsRow activation stages
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t bx, by;
  xcd_tile(blockIdx.x, gridDim.x, (uint32_t)nbx, bx, by);
  const int m0 = (int)by * 256, n0 = (int)bx * 128;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int kc = K / 8; // 16-byte chunks per row
  for (int t = tid; t < 128 * kc; t += 512) {
    const int r = t / kc, c = (t - r * kc) * 8;
    *(uint4 *)&sbw[r * kNtRowB + c] = *(const uint4 *)&b[(size_t)(n0 + r) * ldb + c];
  }
  floatx4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  // thread t moves rows (t >> 2) and (t >> 2) + 128, chunk t & 3, of each
  // activation stage
  const int ar = tid >> 2, ac = (tid & 3) * 8;
  const uint16_t *pa = a + (size_t)(m0 + ar) * lda + ac;
  const size_t half = (size_t)128 * lda;
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  // one K step on LDS stage q: fragments and the 16 products of this wave
  auto step = [&](int q, int k0) {
    const uint16_t *sa = sac + q * 256 * kLdsRow;
    bf16x8 fa[4], fb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) fa[i] = __builtin_bit_cast(bf16x8, *(const uint4 *)&sa[(wm + 16 * i + fr) * kLdsRow + fk]);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      fb[j] = __builtin_bit_cast(bf16x8, *(const uint4 *)&sbw[(wn + 16 * j + fr) * kNtRowB + k0 + fk]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
  };
  auto stage = [&](int q, uint4 x0, uint4 x1) {
    uint16_t *sn = sac + q * 256 * kLdsRow;
    *(uint4 *)&sn[ar * kLdsRow + ac] = x0;
    *(uint4 *)&sn[(ar + 128) * kLdsRow + ac] = x1;
  };
  if (K == kNtKmax) {
    // all eight chunks into registers at once (8 x 2 x 16 B per thread): the
    // block waits on memory once instead of once per K step
    constexpr int kSteps = kNtKmax / kTk;
    uint4 r0[kSteps], r1[kSteps];
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
      r0[s] = *(const uint4 *)(pa + s * kTk);
      r1[s] = *(const uint4 *)(pa + half + s * kTk);
    }
    stage(0, r0[0], r1[0]);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
      step(s & 1, s * kTk);
      if (s + 1 < kSteps) stage((s + 1) & 1, r0[s + 1 < kSteps ? s + 1 : s], r1[s + 1 < kSteps ? s + 1 : s]);
      __syncthreads();
    }
  } else {
    // the next stage's rows loaded into registers while the current one is multiplied
    uint4 r0 = *(const uint4 *)pa, r1 = *(const uint4 *)(pa + half);
    stage(0, r0, r1);
    __syncthreads();
    int q = 0;
    for (int k0 = 0; k0 < K; k0 += kTk) {
      const bool more = k0 + kTk < K;
      if (more) {
        r0 = *(const uint4 *)(pa + k0 + kTk);
        r1 = *(const uint4 *)(pa + half + k0 + kTk);
      }
      step(q, k0);
      if (more) stage(q ^ 1, r0, r1);
      __syncthreads();
      q ^= 1;
    }
  }
  const int cn = lane & 15, rb4 = (lane >> 4) * 4;
  if constexpr (EPI == EPI_BIAS_F32_STATS) {
    // a row's 64 columns of this wave sit in the 16 lanes of its lane group
    // (4 each): max and exponential sum over them, then the two waves of a
    // row block (wn = 0, 64) merge through LDS (free after the last K step)
    float *sred = (float *)lds_nt;
    float rm[16], rs[16];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int m = m0 + wm + 16 * i + rb4 + qq;
        float v[4], vm = -INFINITY;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int n = n0 + wn + 16 * j + cn;
          const float x = acc[i][j][qq] + bias[n];
          ((float *)out)[(size_t)m * ldc + n] = x;
          v[j] = n < n_valid ? x : -INFINITY;
          vm = fmaxf(vm, v[j]);
        }
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) vm = fmaxf(vm, __shfl_xor(vm, o));
        float sum = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) sum += v[j] > -INFINITY ? __expf(v[j] - vm) : 0.0f;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) sum += __shfl_xor(sum, o);
        rm[4 * i + qq] = vm;
        rs[4 * i + qq] = sum;
        if (wn == 64 && cn == 0) {
          const int rl = wm + 16 * i + rb4 + qq;
          sred[2 * rl] = vm;
          sred[2 * rl + 1] = sum;
        }
      }
    __syncthreads();
    if (wn == 0 && cn == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int rl = wm + 16 * i + rb4 + qq;
          const float m1 = rm[4 * i + qq], s1 = rs[4 * i + qq], m2 = sred[2 * rl], s2 = sred[2 * rl + 1];
          const float M = fmaxf(m1, m2);
          const float S = (m1 > -INFINITY ? s1 * __expf(m1 - M) : 0.0f) + (m2 > -INFINITY ? s2 * __expf(m2 - M) : 0.0f);
          stats[(size_t)(m0 + rl) * nbx + bx] = make_float2(M, S);
        }
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int m = m0 + wm + 16 * i + rb4 + qq, n = n0 + wn + 16 * j + cn;
          const float v = acc[i][j][qq] + bias[n];
          const size_t o = (size_t)m * ldc + n;
          if constexpr (EPI == EPI_BIAS_RELU_BF16) ((uint16_t *)out)[o] = f2bf(fmaxf(v, 0.0f));
          else ((float *)out)[o] = v;
        }
  }
}

// The forward products with K = 256 on a persistent grid: a block keeps the
// weight slab of one 128-column block in LDS and walks a sequence of 256-row
// tiles, so the slab is loaded once per block instead of once per tile, and
// the next tile's activation chunks are loaded into registers as the current
// tile's are staged (each chunk register is refilled right after its stage
// store), so the loads overlap the products and the epilogue.  Per XCD (the
// blocks b = x mod 8) the first nbx * groups blocks form `groups` groups of
// the nbx column blocks; group g of XCD x takes row tiles x groups + g,
// stepping by 8 groups: the column blocks of a row tile run on one XCD at
// about the same time, so its activation rows come from HBM once per XCD.
// Same operand fragments, K order and epilogue as k_gemm_nt: same output.
template <int EPI>
__global__ void __launch_bounds__(512) k_gemm_nt_rows(const uint16_t *__restrict__ a, int lda,
                                                      const uint16_t *__restrict__ b, int ldb,
                                                      const float *__restrict__ bias, void *__restrict__ out,
                                                      int ldc, int nbx, int groups, int row_tiles) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds_nt[];
  uint16_t *sbw = lds_nt;                   // 128 x kNtRowB weight slab
  uint16_t *sac = lds_nt + 128 * kNtRowB;   // 2 x 256 x kLdsRow activation stages
  const int x = (int)(blockIdx.x & 7u), kk = (int)(blockIdx.x >> 3);
  if (kk >= nbx * groups) return; // (a whole block: no barrier is left waiting)
  const int g = kk / nbx, bx = kk - g * nbx;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n0 = bx * 128;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  constexpr int K = kNtKmax, kc = K / 8;
  for (int t = tid; t < 128 * kc; t += 512) {
    const int r = t / kc, c = (t - r * kc) * 8;
    *(uint4 *)&sbw[r * kNtRowB + c] = *(const uint4 *)&b[(size_t)(n0 + r) * ldb + c];
  }
  const int ar = tid >> 2, ac = (tid & 3) * 8;
  const size_t half = (size_t)128 * lda;
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  const int cn = lane & 15, rb4 = (lane >> 4) * 4;
  const int stride = 8 * groups;
  int by = x * groups + g;
  if (by >= row_tiles) return; // (uniform per block; the slab loads above need no barrier)
  constexpr int kSteps = K / kTk;
  uint4 r0[kSteps], r1[kSteps];
  {
    const uint16_t *pa = a + (size_t)(by * 256 + ar) * lda + ac;
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
      r0[s] = *(const uint4 *)(pa + s * kTk);
      r1[s] = *(const uint4 *)(pa + half + s * kTk);
    }
  }
  for (; by < row_tiles; by += stride) {
    const int nby = by + stride;
    const bool next = nby < row_tiles;
    const uint16_t *pn = a + (size_t)((next ? nby : by) * 256 + ar) * lda + ac;
    auto stage = [&](int q, uint4 x0, uint4 x1) {
      uint16_t *sn = sac + q * 256 * kLdsRow;
      *(uint4 *)&sn[ar * kLdsRow + ac] = x0;
      *(uint4 *)&sn[(ar + 128) * kLdsRow + ac] = x1;
    };
    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // each chunk register is refilled with the next tile's chunk right after its stage store
    stage(0, r0[0], r1[0]);
    if (next) {
      r0[0] = *(const uint4 *)pn;
      r1[0] = *(const uint4 *)(pn + half);
    }
    __syncthreads(); // (the first time: also the weight slab)
#pragma unroll
    for (int s = 0; s < kSteps; ++s) {
      const uint16_t *sa = sac + (s & 1) * 256 * kLdsRow;
      bf16x8 fa[4], fb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        fa[i] = __builtin_bit_cast(bf16x8, *(const uint4 *)&sa[(wm + 16 * i + fr) * kLdsRow + fk]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        fb[j] = __builtin_bit_cast(bf16x8, *(const uint4 *)&sbw[(wn + 16 * j + fr) * kNtRowB + s * kTk + fk]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
      if (s + 1 < kSteps) {
        const int sn = s + 1 < kSteps ? s + 1 : s;
        stage(sn & 1, r0[sn], r1[sn]);
        if (next) {
          r0[sn] = *(const uint4 *)(pn + sn * kTk);
          r1[sn] = *(const uint4 *)(pn + half + sn * kTk);
        }
      }
      __syncthreads();
    }
    const size_t m0 = (size_t)by * 256;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const size_t m = m0 + wm + 16 * i + rb4 + qq;
          const int n = n0 + wn + 16 * j + cn;
          const float v = acc[i][j][qq] + bias[n];
          const size_t o = m * ldc + n;
          if constexpr (EPI == EPI_BIAS_RELU_BF16) ((uint16_t *)out)[o] = f2bf(fmaxf(v, 0.0f));
          else ((float *)out)[o] = v;
        }
  }
}

// The hidden layers of an inference pass in one kernel, for networks whose
// hidden widths are all 256 (input width <= 256): a block of 128 rows keeps
// its activations in LDS from the network input to the last hidden layer and
// streams each layer's weights through a double-buffered 256 x 32 stage.  A
// wave computes a 32 x 128 tile.  Every layer's products, bias, ReLU and BF16
// rounding are those of the layer-by-layer products (same operand fragments,
// same K order), so the result is bit-identical to them; only the last hidden
// layer's activations go back to HBM.
constexpr int kStackRows = 128;
constexpr int kStackWidth = 256;
constexpr int kStackRowA = kStackWidth + 16; // bf16 per activation row in LDS
constexpr int kStackMax = 8;                // hidden layers
constexpr size_t kStackLds = (size_t)(kStackRows * kStackRowA + 2 * kStackWidth * kLdsRow) * sizeof(uint16_t);

struct StackArgs {
  const uint16_t *w[kStackMax]; // layer l's weights [256][k[l]] (K-contiguous)
  const float *bias[kStackMax];
  int k[kStackMax];             // layer l's input width: a multiple of 32, at most 256
  int n;                        // hidden layers
};

__global__ void __launch_bounds__(512) k_mlp_stack(const uint16_t *__restrict__ in, StackArgs P,
                                                   uint16_t *__restrict__ out) {
  extern __shared__ __attribute__((aligned(16))) uint16_t lds_stack[];
  uint16_t *sa = lds_stack;                            // kStackRows x kStackRowA activations
  uint16_t *sw = lds_stack + kStackRows * kStackRowA;  // 2 x 256 x kLdsRow weight stages
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const size_t m0 = (size_t)blockIdx.x * kStackRows;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 128;
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  const int cn = lane & 15, rb4 = (lane >> 4) * 4;
  {
    const int kc = P.k[0] / 8; // 16-byte chunks per input row
    for (int t = tid; t < kStackRows * kc; t += 512) {
      const int r = t / kc, c = (t - r * kc) * 8;
      *(uint4 *)&sa[r * kStackRowA + c] = *(const uint4 *)&in[(m0 + r) * P.k[0] + c];
    }
  }
  // thread t moves column t >> 1, half t & 1 (16 bf16) of each 32-wide weight chunk
  const int wc = tid >> 1, wh = (tid & 1) * 16;
  for (int l = 0; l < P.n; ++l) {
    const int K = P.k[l];
    const uint16_t *wrow = P.w[l] + (size_t)wc * K + wh;
    uint4 w0 = *(const uint4 *)wrow, w1 = *(const uint4 *)(wrow + 8);
    *(uint4 *)&sw[wc * kLdsRow + wh] = w0;
    *(uint4 *)&sw[wc * kLdsRow + wh + 8] = w1;
    __syncthreads(); // (also: the previous layer's activations are all in sa)
    floatx4 acc[2][8];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    int q = 0;
    for (int k0 = 0; k0 < K; k0 += kTk) {
      const bool more = k0 + kTk < K;
      if (more) {
        w0 = *(const uint4 *)(wrow + k0 + kTk);
        w1 = *(const uint4 *)(wrow + k0 + kTk + 8);
      }
      const uint16_t *s = sw + q * kStackWidth * kLdsRow;
      bf16x8 fa[2], fb[8];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        fa[i] = __builtin_bit_cast(bf16x8, *(const uint4 *)&sa[(wm + 16 * i + fr) * kStackRowA + k0 + fk]);
#pragma unroll
      for (int j = 0; j < 8; ++j) fb[j] = __builtin_bit_cast(bf16x8, *(const uint4 *)&s[(wn + 16 * j + fr) * kLdsRow + fk]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
      if (more) {
        uint16_t *sn = sw + (q ^ 1) * kStackWidth * kLdsRow;
        *(uint4 *)&sn[wc * kLdsRow + wh] = w0;
        *(uint4 *)&sn[wc * kLdsRow + wh + 8] = w1;
      }
      __syncthreads(); // (after the last step: every wave has read sa for this layer)
      q ^= 1;
    }
    const float *bias = P.bias[l];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int n = wn + 16 * j + cn;
      const float b = bias[n];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) sa[(wm + 16 * i + rb4 + qq) * kStackRowA + n] = f2bf(fmaxf(acc[i][j][qq] + b, 0.0f));
    }
  }
  __syncthreads();
  for (int t = tid; t < kStackRows * (kStackWidth / 8); t += 512) {
    const int r = t / (kStackWidth / 8), c = (t - r * (kStackWidth / 8)) * 8;
    *(uint4 *)&out[(m0 + r) * kStackWidth + c] = *(const uint4 *)&sa[r * kStackRowA + c];
  }
}

// 128 x 128 tiles where both sizes allow them (the wide layers), else 64 x 64;
// `splits` K slices (K / splits a multiple of 32), partial products
// split_stride elements apart
template <bool AT, bool BT, int EPI>
static void gemm(const uint16_t *a, int lda, const uint16_t *b, int ldb, int M, int N, int K, const float *bias,
                 const uint16_t *mask, void *out, int ldc, hipStream_t st, int splits = 1, size_t split_stride = 0,
                 size_t a_lo = 0, int k_half = 0) {
  if constexpr (!AT && !BT && (EPI == EPI_BIAS_RELU_BF16 || EPI == EPI_BIAS_F32)) {
    if (M % 256 == 0 && N % 128 == 0 && K % kTk == 0 && K <= kNtKmax) {
      // many row tiles per column block and K = 256: the persistent grid
      const int nbx = N / 128, row_tiles = M / 256, groups = nbx <= 32 ? 32 / nbx : 0;
      if (K == kNtKmax && groups > 0 && row_tiles >= 4 * 8 * groups) {
        hipLaunchKernelGGL(k_gemm_nt_rows<EPI>, dim3(256), dim3(512), kNtLds, st, a, lda, b, ldb, bias, out, ldc, nbx,
                           groups, row_tiles);
        return;
      }
      hipLaunchKernelGGL(k_gemm_nt<EPI>, dim3((N / 128) * (M / 256)), dim3(512), kNtLds, st, a, lda, b, ldb, K, bias,
                         out, ldc, (float2 *)nullptr, 0, N / 128);
      return;
    }
  }
  const int Ks = K / splits;
  if (M % 128 == 0 && N % 128 == 0)
    hipLaunchKernelGGL((k_gemm<128, 128, AT, BT, EPI>), dim3(N / 128, M / 128, splits), dim3(256), 0, st, a, lda, b,
                       ldb, Ks, bias, mask, out, ldc, split_stride, a_lo, k_half);
  else
    hipLaunchKernelGGL((k_gemm<64, 64, AT, BT, EPI>), dim3(N / 64, M / 64, splits), dim3(256), 0, st, a, lda, b, ldb,
                       Ks, bias, mask, out, ldc, split_stride, a_lo, k_half);
}

// number of K slices for an M x N product over K rows: enough blocks for
// the whole chip, each slice at least 128 deep and K / slices a multiple of 32
static int split_want(int M, int N) {
  const int tiles = (M % 128 == 0 && N % 128 == 0) ? (M / 128) * (N / 128) : (M / 64) * (N / 64);
  return (1024 + tiles - 1) / tiles;
}
static int split_count(int M, int N, int K) {
  const int want = split_want(M, N);
  int best = 1;
  for (int s = 1; s <= want && s * 128 <= K; ++s)
    if (K % (32 * s) == 0) best = s;
  return best;
}
// upper bound of split_count over every K <= K_max
static int split_bound(int M, int N, int K_max) { return std::max(1, std::min(split_want(M, N), K_max / 128)); }

// ---------------------------------------------------------------------------
// elementwise and reduction kernels
// ---------------------------------------------------------------------------
// rows of fp32 inputs [n][n_in] -> bf16 [n_pad][in_pad] (zero padded); with
// idx, row r takes input row idx[r] (and label y[idx[r]])
__global__ void k_pack_input(const float *x, const int32_t *y, const uint32_t *idx, uint32_t n, int n_in, int in_pad,
                             uint32_t n_pad, uint16_t *xb, int32_t *yb) {
  const uint32_t r = blockIdx.x * blockDim.y + threadIdx.y;
  if (r >= n_pad) return;
  const int c = threadIdx.x;
  const bool live = r < n;
  const uint32_t src = live ? (idx ? idx[r] : r) : 0u;
  for (int k = c; k < in_pad; k += blockDim.x)
    xb[(size_t)r * in_pad + k] = (live && k < n_in) ? f2bf(x[(size_t)src * n_in + k]) : (uint16_t)0;
  if (yb && c == 0) yb[r] = live ? y[src] : -1;
}

// Row statistics of a logit row by one wave: running maximum m and sum of
// exp(z - m) over the first C entries, 4 consecutive entries per lane per
// 256-entry tile (16-byte loads; ld a multiple of 4), combined across lanes.
__device__ __forceinline__ void row_max_sum(const float *zr, int C, int lane, float &m, float &s) {
  m = -INFINITY;
  s = 0.f;
  for (int c0 = 4 * lane; c0 < C; c0 += 256) {
    const float4 v = *(const float4 *)(zr + c0);
    const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (c0 + j >= C) break;
      if (e[j] > m) {
        s *= __expf(m - e[j]);
        m = e[j];
      }
      s += __expf(e[j] - m);
    }
  }
  float M = m;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) M = fmaxf(M, __shfl_xor(M, o));
  s = m == -INFINITY ? 0.f : s * __expf(m - M);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  m = M;
}

// one wave per row: loss = logsumexp(z) - z[y]; dz = (softmax(z) - onehot(y)) / n
// as hi + lo bf16 planes, the lo plane dz_lo elements after the hi plane (zero
// in padded columns and rows); a label outside [0, C) sets *bad and is read
// as class 0
__global__ void __launch_bounds__(256) k_softmax_ce(const float *z, int ldz, int C, const int32_t *y, uint32_t n,
                                                    uint32_t n_pad, float inv_n, uint16_t *dz, size_t dz_lo,
                                                    double *row_loss, uint32_t *bad) {
  const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= n_pad) return;
  const float *zr = z + (size_t)r * ldz;
  uint16_t *dr = dz + (size_t)r * ldz;
  if (r >= n) {
    for (int c = lane; c < ldz; c += 64) dr[c] = dr[c + dz_lo] = 0;
    if (lane == 0) row_loss[r] = 0.0;
    return;
  }
  float mx, s;
  row_max_sum(zr, C, lane, mx, s);
  const float inv_s = 1.0f / s;
  int yy = y[r];
  if (yy < 0 || yy >= C) {
    if (lane == 0) atomicOr(bad, 1u);
    yy = 0;
  }
  for (int c0 = 4 * lane; c0 < ldz; c0 += 256) {
    const float4 v = *(const float4 *)(zr + c0);
    const float e[4] = {v.x, v.y, v.z, v.w};
    uint16_t o[4], ol[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + j;
      const float p = c < C ? __expf(e[j] - mx) * inv_s : 0.0f;
      const float g = (c == yy ? p - 1.0f : p) * inv_n;
      o[j] = f2bf(g);
      ol[j] = f2bf(g - bf2f(o[j]));
    }
    *(uint2 *)(dr + c0) = make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16), (uint32_t)o[2] | ((uint32_t)o[3] << 16));
    *(uint2 *)(dr + dz_lo + c0) =
        make_uint2((uint32_t)ol[0] | ((uint32_t)ol[1] << 16), (uint32_t)ol[2] | ((uint32_t)ol[3] << 16));
  }
  if (lane == 0) row_loss[r] = (double)mx + log((double)s) - (double)zr[yy];
}

// Factored output (energy head, then the position given the energy): the
// first n1 logits are the energy classes (0 = none), then G blocks of n2
// position logits; energy class e > 0 uses block g(e) = (e - 1) G / (n1 - 1)
// (contiguous groups of energy classes), shifted by the row T[e - 1] of the
// offset table.  A joint label y is 0 (e = 0) or 1 + k (n1 - 1) + (e - 1).
__device__ __forceinline__ void factored_label(int y, int n1, int &e, int &k) {
  e = y > 0 ? 1 + (y - 1) % (n1 - 1) : 0;
  k = y > 0 ? (y - 1) / (n1 - 1) : 0;
}
__device__ __forceinline__ int position_block(int e, int n1, int n2, int G) {
  return n1 + ((e - 1) * G) / (n1 - 1) * n2;
}

// wave-wide maximum and sum of exp(v - max) of z2[c] + t[c], c < n2 (strided by lane)
__device__ __forceinline__ void offset_row_max_sum(const float *z2, const float *t, int n2, int lane, float &m,
                                                   float &s) {
  m = -INFINITY;
  for (int c = lane; c < n2; c += 64) m = fmaxf(m, z2[c] + t[c]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  s = 0.f;
  for (int c = lane; c < n2; c += 64) s += __expf(z2[c] + t[c] - m);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
}

// one wave per row: loss = -log P(e) - [e > 0] log P(k | e) and its gradient
// with respect to the logits, as hi + lo bf16 planes (zero in padded columns
// and rows); erow[r] = e (0 for padded rows); a label outside the classes sets
// *bad and is read as 0.  n1 <= 64.
__global__ void __launch_bounds__(256) k_factored_ce(const float *z, int ldz, int n1, int n2, int G, const float *T,
                                                     const int32_t *y, uint32_t n, uint32_t n_pad, float inv_n,
                                                     uint16_t *dz, size_t dz_lo, double *row_loss, int32_t *erow,
                                                     uint32_t *bad) {
  const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= n_pad) return;
  const float *zr = z + (size_t)r * ldz;
  uint16_t *dr = dz + (size_t)r * ldz;
  if (r >= n) {
    for (int c = lane; c < ldz; c += 64) dr[c] = dr[c + dz_lo] = 0;
    if (lane == 0) {
      row_loss[r] = 0.0;
      erow[r] = 0;
    }
    return;
  }
  int yy = y[r];
  if (yy < 0 || yy > n2 * (n1 - 1)) {
    if (lane == 0) atomicOr(bad, 1u);
    yy = 0;
  }
  int e, k;
  factored_label(yy, n1, e, k);
  // energy head: one class per lane
  const float v1 = lane < n1 ? zr[lane] : -INFINITY;
  float m1 = v1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m1 = fmaxf(m1, __shfl_xor(m1, o));
  float s1 = lane < n1 ? __expf(v1 - m1) : 0.f;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s1 += __shfl_xor(s1, o);
  // position head given e (its block of position logits)
  const int pb = e > 0 ? position_block(e, n1, n2, G) : n1;
  const float *z2 = zr + pb;
  const float *t = T + (size_t)(e > 0 ? e - 1 : 0) * n2;
  float m2 = 0.f, s2 = 1.f;
  if (e > 0) offset_row_max_sum(z2, t, n2, lane, m2, s2);
  const float inv_s1 = 1.0f / s1, inv_s2 = 1.0f / s2;
  for (int c = lane; c < ldz; c += 64) {
    float g = 0.f;
    if (c < n1) {
      g = (__expf(zr[c] - m1) * inv_s1 - (c == e ? 1.0f : 0.0f)) * inv_n;
    } else if (e > 0 && c >= pb && c < pb + n2) {
      const int j = c - pb;
      g = (__expf(z2[j] + t[j] - m2) * inv_s2 - (j == k ? 1.0f : 0.0f)) * inv_n;
    }
    const uint16_t hi = f2bf(g);
    dr[c] = hi;
    dr[c + dz_lo] = f2bf(g - bf2f(hi));
  }
  if (lane == 0) {
    double l = (double)m1 + log((double)s1) - (double)zr[e];
    if (e > 0) l += (double)m2 + log((double)s2) - ((double)z2[k] + (double)t[k]);
    row_loss[r] = l;
    erow[r] = e;
  }
}

// partial offset-table gradients: slice blockIdx.z of `slices` sums, over its
// rows r with energy class e = blockIdx.y + 1, the position-head gradient
// (hi + lo) into part[slice][(e - 1) n2 + j]
__global__ void k_table_grad_part(const uint16_t *dz, size_t dz_lo, int ldz, int n1, int n2, int G,
                                  const int32_t *erow, uint32_t rows, int slices, float *part) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int e = (int)blockIdx.y + 1;
  if (j >= n2) return;
  const uint32_t per = (rows + slices - 1) / slices;
  const uint32_t r0 = blockIdx.z * per, r1 = min(rows, r0 + per);
  const int pb = position_block(e, n1, n2, G);
  float a = 0.f;
  for (uint32_t r = r0; r < r1; ++r)
    if (erow[r] == e) {
      const size_t o = (size_t)r * ldz + pb + j;
      a += bf2f(dz[o]) + bf2f(dz[o + dz_lo]);
    }
  part[(size_t)blockIdx.z * (n1 - 1) * n2 + (size_t)(e - 1) * n2 + j] = a;
}

// Factored sampling, one wave per queue entry: the energy class e = first
// class whose cumulative softmax mass reaches u0 * total (u0: word 0 of
// Philox (0, event, inst_rng, 4 + photon)); for e > 0 the position k = first
// position whose cumulative mass under softmax(z2 + T[e - 1]) over the
// positions that exist (inside their layer's array around the entry's
// anchors) reaches u2 * total (word 2).  cls = the joint label.
//
// The positions of layer l (W^2 of them, W = 2H + 1) sit in C = ceil(W^2 / 64)
// chunks of 64 of their own, so a chunk never straddles two layers: chunk
// l C + q holds positions l W^2 + 64 q + lane (none past W^2).  A chunk's
// layer, anchors and first crystal offset are then the same for the whole
// wave (scalar registers), and a lane's offset (dt, da) is that first offset
// plus the lane's own, with one carry.  Chunk q of layer l goes to register
// l C + q of every lane; the chunk totals are reduced over the lanes by
// halving exchanges (each level keeps half of the chunks per lane and adds the
// partner's copy of that half), so lane t ends with the total of chunk
// t >> (6 - log2 P) (P = B rounded up to a power of two); a wave scan of the
// totals in chunk order picks the chunk, one wave prefix sum inside it the
// position: the draw is the natural-order inverse CDF.
// base[i] through a 32-bit byte offset (i < 2^30), so that the load takes the
// wave-uniform base from scalar registers and the offset alone per lane
__device__ __forceinline__ float load_at(const float *base, uint32_t i) {
  return *(const float *)((const char *)base + (i << 2));
}

// lo for the lanes whose bit s is clear, hi for the others, plus the partner
// lane's (lane ^ s) copy of the same element.  For s = 32 (16) the swap of the
// upper half-wave (odd rows) of lo with the lower half-wave (even rows) of hi
// leaves each lane one register with its own kept value and one with its
// partner's, so their sum is the result.
__device__ __forceinline__ float halve_pair(float lo, float hi, int s) {
  if (s == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  if (s == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const bool up = (__lane_id() & (uint32_t)s) != 0u;
  return (up ? hi : lo) + lane_xor_f(up ? lo : hi, s);
}

template <int B>
__global__ void __launch_bounds__(256) k_sample_factored(const float *z, int ldz, int n1, int n2, int G,
                                                         const float *T, uint32_t n, const uint32_t *ev,
                                                         const uint32_t *meta, const uint32_t *anchor,
                                                         const DevScene *S, int H, uint32_t k0, uint32_t k1,
                                                         uint32_t inst_rng, uint32_t *cls, uint32_t *nonzero) {
  constexpr int P = B <= 8 ? 8 : B <= 16 ? 16 : 32; // chunks rounded up to a power of two
  constexpr int KP = P == 8 ? 3 : P == 16 ? 4 : 5;  // its log2
  const uint32_t r = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  // the loads that do not wait for the energy class go out first (a wave is
  // latency-bound here): entry words, energy logits, anchors, and with one
  // position block (G = 1, the block is the same for every energy class) the
  // position logits too
  const float *zr = z + (size_t)r * ldz;
  const uint32_t mt = meta[r], evr = ev[r];
  const float v1 = lane < n1 ? zr[lane] : -INFINITY;
  const int nl = S->n_layers;
  int nt[kMaxLayers], na[kMaxLayers], at[kMaxLayers], aa[kMaxLayers];
#pragma unroll
  for (int q = 0; q < kMaxLayers; ++q) {
    const bool on = q < nl;
    const uint32_t aw = on ? anchor[(size_t)kMaxLayers * r + q] : 0u;
    nt[q] = on ? S->layer[q].n_t : 0;
    na[q] = on ? S->layer[q].n_a : 0;
    at[q] = (int)(aw & 0xFFFFu) - H;
    aa[q] = (int)(aw >> 16) - H;
  }
  const int W = 2 * H + 1, WW = W * W, C = (WW + 63) / 64;
  // offset (dt, da) of in-layer position p: dt = floor((p + 1/2) / W) in
  // FP32, exact for p < 2^11 and W <= 64 (the rounding error stays below 1/(2W))
  const float inv_w = 1.0f / (float)W;
  const bool early = G == 1;
  // chunk c: its positions' indices j[c] and whether each exists (ok[c])
  uint32_t j[B];
  bool ok[B];
  float zp[B]; // with one position block: the position logits
  {
    // chunk c: layer L (its anchors and sizes in atL, aaL, ntL, naL; the
    // layers after it queued behind), chunk q of it
    int L = 0, q = 0;
    int atL = at[0], aaL = aa[0], ntL = nt[0], naL = na[0];
    int at1 = at[1], aa1 = aa[1], nt1 = nt[1], na1 = na[1];
    int at2 = at[2], aa2 = aa[2], nt2 = nt[2], na2 = na[2];
    int at3 = at[3], aa3 = aa[3], nt3 = nt[3], na3 = na[3];
    static_assert(kMaxLayers == 4, "the layer queue holds four layers");
#pragma unroll
    for (int c = 0; c < B; ++c) {
      const uint32_t p = (uint32_t)(q * 64 + lane);
      const int dt = (int)(((float)p + 0.5f) * inv_w);
      const int da = (int)p - __mul24(dt, W);
      const bool in = L < nl && p < (uint32_t)WW;
      ok[c] = in & ((uint32_t)(atL + dt) < (uint32_t)ntL) & ((uint32_t)(aaL + da) < (uint32_t)naL);
      j[c] = ok[c] ? (uint32_t)(L * WW) + p : 0u; // (position 0 stands in for none: every load is in the row)
      zp[c] = early ? load_at(zr, (uint32_t)n1 + j[c]) : 0.f;
      if (++q == C) {
        q = 0;
        ++L;
        atL = at1, aaL = aa1, ntL = nt1, naL = na1;
        at1 = at2, aa1 = aa2, nt1 = nt2, na1 = na2;
        at2 = at3, aa2 = aa3, nt2 = nt3, na2 = na3;
      }
    }
  }
  if (mt == kQueueHole) { // an empty queue slot
    if (lane == 0) {
      cls[r] = 0u;
      nonzero[r] = 0u;
    }
    return;
  }
  const uint4 w = philox(k0, k1, make_uint4(0u, evr, inst_rng, 4u + (mt & 1u)));
  // energy class: one class per lane
  float m1 = v1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m1 = fmaxf(m1, __shfl_xor(m1, o));
  const float p1 = lane < n1 ? __expf(v1 - m1) : 0.f;
  float incl = p1;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const float tt = __shfl_up(incl, o);
    if (lane >= o) incl += tt;
  }
  const float target1 = to_unit(w.x) * __shfl(incl, 63);
  const uint64_t c1 = __ballot(incl >= target1 && lane < n1);
  const int e = c1 ? __ffsll((unsigned long long)c1) - 1 : n1 - 1;
  if (e == 0) {
    if (lane == 0) {
      cls[r] = 0u;
      nonzero[r] = 0u;
    }
    return;
  }
  const float *z2 = zr + position_block(e, n1, n2, G);
  const float *t = T + (size_t)(e - 1) * n2;
  // (two loops: a select between the registers and a load would move the
  // registers to memory)
  float v[B];
  if (early) {
#pragma unroll
    for (int c = 0; c < B; ++c) v[c] = zp[c] + load_at(t, j[c]);
  } else {
#pragma unroll
    for (int c = 0; c < B; ++c) v[c] = load_at(z2, j[c]) + load_at(t, j[c]);
  }
  float m = -INFINITY;
#pragma unroll
  for (int c = 0; c < B; ++c) {
    v[c] = ok[c] ? v[c] : -INFINITY;
    m = fmaxf(m, v[c]);
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) m = fmaxf(m, lane_xor_f(m, o));
  float x[P];
#pragma unroll
  for (int c = 0; c < P; ++c) {
    if (c < B) v[c] = ok[c] ? __expf(v[c] - m) : 0.f;
    x[c] = c < B ? v[c] : 0.f;
  }
  // chunk totals: halving exchanges over the top KP lane bits, then plain
  // butterflies over the rest; lane t holds the total of chunk t >> (6 - KP)
#pragma unroll
  for (int h = P / 2, s = 32; h >= 1; h >>= 1, s >>= 1)
#pragma unroll
    for (int i = 0; i < h; ++i) x[i] = halve_pair(x[i], x[i + h], s);
#pragma unroll
  for (int s = 32 >> KP; s >= 1; s >>= 1) x[0] += lane_xor_f(x[0], s);
  constexpr int kGroup = 64 >> KP; // lanes per chunk total
  const int chunk = lane / kGroup;
  // running sum of the totals in chunk order (one lane per chunk counts)
  float run = (lane % kGroup) == 0 && chunk < B ? x[0] : 0.f;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const float tt = __shfl_up(run, o);
    if (lane >= o) run += tt;
  }
  const float sl = __shfl(run, 63);
  const float target2 = to_unit(w.z) * sl;
  // (a chunk without mass cannot hold the draw, even when the target is 0)
  const uint64_t reach = __ballot((lane % kGroup) == 0 && chunk < B && x[0] > 0.f && run >= target2);
  int k;
  if (!reach) { // rounding left the target beyond the total: the last position that exists
    int last = -1;
#pragma unroll
    for (int c = 0; c < B; ++c)
      if (v[c] > 0.f) last = (int)j[c];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) last = max(last, (int)lane_xor((uint32_t)last, o));
    k = last;
  } else {
    const int cs = (__ffsll((unsigned long long)reach) - 1) / kGroup; // the chunk
    const float carry = cs > 0 ? __shfl(run, cs * kGroup - 1) : 0.f; // the running sum before it
    // its values: the first chunk whose bit is set in `reach` (a test of the
    // mask itself, not of an index, which keeps the chunks in registers)
    float vc = 0.f;
    uint32_t jc = 0;
    bool found = false;
#pragma unroll
    for (int c = 0; c < B; ++c) {
      const bool here = !found && ((reach >> (c * kGroup)) & 1u);
      vc = here ? v[c] : vc;
      jc = here ? j[c] : jc;
      found = found || here;
    }
    float in2 = vc;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const float tt = __shfl_up(in2, o);
      if (lane >= o) in2 += tt;
    }
    const uint64_t cr = __ballot(carry + in2 >= target2 && vc > 0.f);
    const uint64_t ex = __ballot(vc > 0.f);
    // (rounding inside the chunk: its last position that exists)
    const int kl = cr ? __ffsll((unsigned long long)cr) - 1 : 63 - __clzll((long long)ex);
    k = (int)__shfl(jc, kl);
  }
  if (lane == 0) {
    cls[r] = 1u + (uint32_t)k * (uint32_t)(n1 - 1) + (uint32_t)(e - 1);
    nonzero[r] = 1u;
  }
}

__global__ void __launch_bounds__(1024) k_sum_f64(const double *v, uint32_t n, double *out) {
  __shared__ double s[1024];
  double a = 0.0;
  for (uint32_t i = threadIdx.x; i < n; i += 1024) a += v[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

// partial column sums: slice blockIdx.y of `slices` sums its rows of dz
// (hi + lo planes, dz_lo elements apart) into part[slice][c]
__global__ void k_col_sum_part(const uint16_t *dz, size_t dz_lo, int ld, uint32_t rows, int cols, int slices,
                               float *part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  const uint32_t per = (rows + slices - 1) / slices;
  const uint32_t r0 = blockIdx.y * per, r1 = min(rows, r0 + per);
  float a = 0.f;
  for (uint32_t r = r0; r < r1; ++r) a += bf2f(dz[(size_t)r * ld + c]) + bf2f(dz[(size_t)r * ld + c + dz_lo]);
  part[(size_t)blockIdx.y * cols + c] = a;
}

// out[i] = sum over s of part[s n + i] (slices summed in order)
__global__ void k_reduce_slices(const float *part, int slices, size_t n, float *out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float a = 0.f;
  for (int s = 0; s < slices; ++s) a += part[(size_t)s * n + i];
  out[i] = a;
}

// Adam on one tensor: master [rows][cols] against gradients with row stride
// ldg; refreshes the bf16 copy wb [rows][ldb] and/or the fp32 copy fc [cols]
// (biases, rows = 1)
__global__ void k_adam(float *w, float *m, float *v, const float *g, int rows, int cols, int ldg, float lr, float b1,
                       float b2, float eps, float c1, float c2, uint16_t *wb, int ldb, float *fc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int r = i / cols, c = i - r * cols;
  const float gg = g[(size_t)r * ldg + c];
  const float mm = b1 * m[i] + (1.0f - b1) * gg;
  const float vv = b2 * v[i] + (1.0f - b2) * gg * gg;
  m[i] = mm;
  v[i] = vv;
  const float nw = w[i] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
  w[i] = nw;
  if (wb) wb[(size_t)r * ldb + c] = f2bf(nw);
  if (fc) fc[i] = nw;
}

// bf16 copy of a master weight matrix into its padded buffer
__global__ void k_to_bf16(const float *w, int rows, int cols, uint16_t *wb, int ldb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int r = i / cols, c = i - r * cols;
  wb[(size_t)r * ldb + c] = f2bf(w[i]);
}

// training batch indices: uniform with replacement from Philox (key seed,
// counter (step, r / 4, 0, 9))
__global__ void k_batch_indices(uint32_t k0, uint32_t k1, uint32_t step, uint32_t n, uint64_t n_pairs, uint32_t *idx) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const uint4 w = philox(k0, k1, make_uint4(step, r >> 2, 0u, 9u));
  const uint32_t word = (r & 3) == 0 ? w.x : (r & 3) == 1 ? w.y : (r & 3) == 2 ? w.z : w.w;
  idx[r] = (uint32_t)(((unsigned long long)word * n_pairs) >> 32);
}

// ---------------------------------------------------------------------------
// surrogate sampling: one wave per queue entry
// ---------------------------------------------------------------------------
// class = first c whose cumulative softmax mass reaches u * total: the row's
// maximum and total in one pass, then 256-class tiles in class order (4
// consecutive classes per lane, a wave prefix sum per tile) until the tile
// that crosses, where the crossing lane walks its 4 classes
__global__ void __launch_bounds__(256) k_sample_classes(const float *z, int ldz, int C, uint32_t n, const uint32_t *ev,
                                                        const uint32_t *meta, uint32_t k0, uint32_t k1,
                                                        uint32_t inst_rng, uint32_t *cls, uint32_t *nonzero) {
  const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  if (meta[r] == kQueueHole) { // an empty queue slot
    if (lane == 0) {
      cls[r] = 0u;
      nonzero[r] = 0u;
    }
    return;
  }
  const float *zr = z + (size_t)r * ldz;
  float mx, total;
  row_max_sum(zr, C, lane, mx, total);
  const uint4 w = philox(k0, k1, make_uint4(0u, ev[r], inst_rng, 4u + (meta[r] & 1u)));
  const float target = to_unit(w.x) * total;
  int c_out = C - 1;
  float acc = 0.f; // mass of the tiles before this one
  for (int t0 = 0; t0 < C; t0 += 256) {
    const int c0 = t0 + 4 * lane;
    float p[4] = {0.f, 0.f, 0.f, 0.f};
    if (c0 < C) {
      const float4 v = *(const float4 *)(zr + c0);
      const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) p[j] = c0 + j < C ? __expf(e[j] - mx) : 0.f;
    }
    const float part = (p[0] + p[1]) + (p[2] + p[3]);
    float incl = part;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const float tt = __shfl_up(incl, o);
      if (lane >= o) incl += tt;
    }
    const uint64_t crossed = __ballot(acc + incl >= target && c0 < C);
    if (crossed) {
      const int L = __ffsll((unsigned long long)crossed) - 1;
      int found = min(c0 + 3, C - 1);
      float a = acc + incl - part;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a += p[j];
        if (a >= target && c0 + j < C) {
          found = c0 + j;
          break;
        }
      }
      c_out = __shfl(found, L);
      break;
    }
    acc += __shfl(incl, 63);
  }
  if (lane == 0) {
    cls[r] = (uint32_t)c_out;
    nonzero[r] = c_out != 0 ? 1u : 0u;
  }
}

// The same draw from the per-tile statistics of the last product: the row's
// maximum and total from its (max, sum) pairs (one per 128-class tile, at
// most 64), the tile whose cumulative mass reaches u * total, then the class
// inside that tile from its 128 logits (two per lane) -- 1 KB read per row
// instead of the whole row twice.  Sums run in another order than in
// k_sample_classes, so a draw within rounding of a class boundary may land
// on the neighbouring class.
__global__ void __launch_bounds__(256) k_sample_tiles(const float2 *stats, int n_tiles, const float *z, int ldz, int C,
                                                      uint32_t n, const uint32_t *ev, const uint32_t *meta,
                                                      uint32_t k0, uint32_t k1, uint32_t inst_rng, uint32_t *cls,
                                                      uint32_t *nonzero) {
  const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= n) return;
  if (meta[r] == kQueueHole) { // an empty queue slot
    if (lane == 0) {
      cls[r] = 0u;
      nonzero[r] = 0u;
    }
    return;
  }
  const float2 t = lane < n_tiles ? stats[(size_t)r * n_tiles + lane] : make_float2(-INFINITY, 0.0f);
  float mx = t.x;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  const float w = t.x > -INFINITY ? t.y * __expf(t.x - mx) : 0.0f;
  float incl = w;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const float tt = __shfl_up(incl, o);
    if (lane >= o) incl += tt;
  }
  const float total = __shfl(incl, 63);
  const uint4 wr = philox(k0, k1, make_uint4(0u, ev[r], inst_rng, 4u + (meta[r] & 1u)));
  const float target = to_unit(wr.x) * total;
  const uint64_t crossed = __ballot(incl >= target && lane < n_tiles);
  const int T = crossed ? __ffsll((unsigned long long)crossed) - 1 : n_tiles - 1;
  const float before = __shfl(incl - w, T);
  const float *zr = z + (size_t)r * ldz;
  const int c0 = T * 128 + 2 * lane;
  const float p0 = c0 < C ? __expf(zr[c0] - mx) : 0.0f;
  const float p1 = c0 + 1 < C ? __expf(zr[c0 + 1] - mx) : 0.0f;
  const float part = p0 + p1;
  float in2 = part;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const float tt = __shfl_up(in2, o);
    if (lane >= o) in2 += tt;
  }
  const uint64_t cr2 = __ballot(before + in2 >= target && c0 < C);
  int c_out = min(T * 128 + 127, C - 1); // rounding left the target beyond the tile
  if (cr2) {
    const int L = __ffsll((unsigned long long)cr2) - 1;
    const int mine = (before + in2 - part + p0 >= target || c0 + 1 >= C) ? c0 : c0 + 1;
    c_out = __shfl(mine, L);
  }
  if (lane == 0) {
    cls[r] = (uint32_t)c_out;
    nonzero[r] = c_out != 0 ? 1u : 0u;
  }
}

// one synthetic hit per entry with a class other than 0, at *hit_count + pos
__global__ void k_emit_hits(uint32_t n, const uint32_t *cls, const uint32_t *pos, const uint32_t *ev,
                            const uint32_t *meta, const uint32_t *anchor, const float *e_in,
                            const unsigned long long *time, const DevScene *Sp, SurSpecD P, uint32_t k0, uint32_t k1,
                            uint32_t inst_rng, RunArgs H) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n || cls[r] == 0) return;
  const DevScene &S = *Sp;
  const int c = (int)cls[r] - 1;
  const int nb = P.n_ebins + 1, W = 2 * P.chalf + 1;
  const int b = c % nb, k = c / nb;
  const int l = k / (W * W), rr = k - l * W * W;
  const int dt = rr / W, da = rr - dt * W;
  const uint32_t aw = anchor[(size_t)kMaxLayers * r + l];
  const int it = (int)(aw & 0xFFFFu) + dt - P.chalf, ia = (int)(aw >> 16) + da - P.chalf;
  const uint32_t m = meta[r];
  const int panel = (int)((m >> 1) & 127u), module = (int)(m >> 8);
  const int gid = panel * S.crystals_per_panel + module * S.crystals_per_module + S.layer[l].base +
                  ia * S.layer[l].n_t + it;
  const uint4 w = philox(k0, k1, make_uint4(0u, ev[r], inst_rng, 4u + (m & 1u)));
  const float edep = b == P.n_ebins ? e_in[r] : P.e_min + P.ebin * ((float)b + to_unit(w.y));
  const unsigned long long i = *H.hit_count + pos[r];
  if (i >= H.capacity) return;
  H.h_event[i] = ev[r];
  H.h_gid[i] = (uint32_t)gid;
  H.h_edep[i] = edep;
  H.h_depth[i] = 0.5f * (S.layer[l].d0 + S.layer[l].d1);
  H.h_time[i] = time[r];
  H.h_aux[i] = (m & 1u) | (3u << 1);
  if (H.h_inst) H.h_inst[i] = 0u;
}

__global__ void k_add_u64(unsigned long long *p, unsigned long long v) { *p += v; }

static inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }
static inline int pad_to(int x, int m) { return (x + m - 1) / m * m; }

} // namespace gpet

using namespace gpet;

namespace {

gpet_status mlp_fail(gpet_mlp *q, gpet_status code, const std::string &msg) {
  if (q && q->ctx) q->ctx->err = msg;
  return code;
}

void free_workspace(gpet_mlp *q) {
  for (uint16_t *p : q->act)
    if (p) (void)hipFree(p);
  q->act.clear();
  for (void *p : {(void *)q->logits, (void *)q->dz[0], (void *)q->dz[1], (void *)q->yb, (void *)q->idx,
                  (void *)q->row_loss, (void *)q->loss_sum, (void *)q->flag, (void *)q->part, (void *)q->part_b,
                  (void *)q->tstats, (void *)q->erow})
    if (p) (void)hipFree(p);
  q->flag = nullptr;
  q->tstats = nullptr;
  q->part = q->part_b = nullptr;
  q->logits = nullptr;
  q->dz[0] = q->dz[1] = nullptr;
  q->yb = nullptr;
  q->idx = nullptr;
  q->row_loss = q->loss_sum = nullptr;
  q->erow = nullptr;
  q->cap = 0;
}

// workspace for at least n rows (rounded up to a tile)
gpet_status ensure_workspace(gpet_mlp *q, uint32_t n) {
  const uint32_t need = (uint32_t)pad_to((int)std::max<uint32_t>(n, 1), kRowPad);
  if (need <= q->cap) return GPET_OK;
  free_workspace(q);
  bool ok = true;
  q->act.assign(q->n_layers, nullptr);
  int widest = 0;
  for (int l = 0; l < q->n_layers; ++l) {
    ok = ok && hipMalloc((void **)&q->act[l], (size_t)need * q->psize[l] * 2) == hipSuccess;
    widest = std::max(widest, q->psize[l + 1]);
  }
  ok = ok && hipMalloc((void **)&q->logits, (size_t)need * q->psize[q->n_layers] * 4) == hipSuccess;
  ok = ok && hipMalloc((void **)&q->tstats, (size_t)need * (q->psize[q->n_layers] / 128) * sizeof(float2)) == hipSuccess;
  // gradients as hi + lo bf16 planes
  ok = ok && hipMalloc((void **)&q->dz[0], (size_t)need * widest * 4) == hipSuccess;
  ok = ok && hipMalloc((void **)&q->dz[1], (size_t)need * widest * 4) == hipSuccess;
  ok = ok && hipMalloc((void **)&q->yb, (size_t)need * 4) == hipSuccess;
  ok = ok && hipMalloc((void **)&q->idx, (size_t)need * 4) == hipSuccess;
  ok = ok && hipMalloc((void **)&q->row_loss, (size_t)need * 8) == hipSuccess;
  ok = ok && hipMalloc((void **)&q->erow, (size_t)need * 4) == hipSuccess;
  ok = ok && hipMalloc((void **)&q->loss_sum, 8) == hipSuccess;
  ok = ok && hipMalloc((void **)&q->flag, 8) == hipSuccess;
  // split-K partial products of the weight gradients and partial bias sums
  size_t part = 0;
  for (int l = 0; l < q->n_layers; ++l) {
    const int M = q->psize[l + 1], N = q->psize[l];
    part = std::max(part, (size_t)split_bound(M, N, 2 * (int)need) * M * N);
  }
  if (q->n_first) part = std::max(part, (size_t)kTableSlices * (q->n_first - 1) * q->n_second);
  ok = ok && hipMalloc((void **)&q->part, part * 4) == hipSuccess;
  ok = ok && hipMalloc((void **)&q->part_b, (size_t)64 * widest * 4) == hipSuccess;
  if (!ok) {
    free_workspace(q);
    return mlp_fail(q, GPET_ERR_HIP, "mlp: workspace allocation failed");
  }
  q->cap = need;
  return GPET_OK;
}

// forward pass of the rows packed in act[0]; logits (fp32, padded) at q->logits
void forward(gpet_mlp *q, uint32_t n_pad, hipStream_t st) {
  for (int l = 0; l < q->n_layers; ++l) {
    const int K = q->psize[l], N = q->psize[l + 1];
    const float *bias = q->bp + l * q->bp_stride;
    if (l + 1 < q->n_layers)
      gemm<false, false, EPI_BIAS_RELU_BF16>(q->act[l], K, q->wb[l], K, (int)n_pad, N, K, bias, nullptr, q->act[l + 1],
                                             N, st);
    else
      gemm<false, false, EPI_BIAS_F32>(q->act[l], K, q->wb[l], K, (int)n_pad, N, K, bias, nullptr, q->logits, N, st);
  }
}

// forward pass for inference (no activations kept for a backward pass): the
// hidden layers in one kernel where the widths allow it, else layer by layer
void forward_infer(gpet_mlp *q, uint32_t n_pad, hipStream_t st) {
  const int L = q->n_layers;
  bool stack = L >= 2 && L - 1 <= kStackMax && n_pad % kStackRows == 0 && q->psize[0] % kTk == 0 &&
               q->psize[0] <= kStackWidth;
  for (int l = 1; l < L; ++l) stack = stack && q->psize[l] == kStackWidth;
  if (!stack) {
    forward(q, n_pad, st);
    return;
  }
  StackArgs P{};
  for (int l = 0; l + 1 < L; ++l) {
    P.w[l] = q->wb[l];
    P.bias[l] = q->bp + l * q->bp_stride;
    P.k[l] = q->psize[l];
  }
  P.n = L - 1;
  hipLaunchKernelGGL(k_mlp_stack, dim3(n_pad / kStackRows), dim3(512), kStackLds, st, q->act[0], P, q->act[L - 1]);
  const int K = q->psize[L - 1], N = q->psize[L];
  gemm<false, false, EPI_BIAS_F32>(q->act[L - 1], K, q->wb[L - 1], K, (int)n_pad, N, K, q->bp + (L - 1) * q->bp_stride,
                                   nullptr, q->logits, N, st);
}

// forward pass for sampling: the last product also leaves per-tile row
// statistics in q->tstats (the forward product kernel always applies: rows
// padded to 256, widths to 128, K <= 256 for the hidden layers)
void forward_sample(gpet_mlp *q, uint32_t n_pad, hipStream_t st) {
  const int L = q->n_layers;
  for (int l = 0; l + 1 < L; ++l) {
    const int K = q->psize[l], N = q->psize[l + 1];
    gemm<false, false, EPI_BIAS_RELU_BF16>(q->act[l], K, q->wb[l], K, (int)n_pad, N, K, q->bp + l * q->bp_stride,
                                           nullptr, q->act[l + 1], N, st);
  }
  const int K = q->psize[L - 1], N = q->psize[L];
  hipLaunchKernelGGL(k_gemm_nt<EPI_BIAS_F32_STATS>, dim3((N / 128) * (n_pad / 256)), dim3(512), kNtLds, st,
                     q->act[L - 1], K, q->wb[L - 1], K, K, q->bp + (L - 1) * q->bp_stride, (void *)q->logits, N,
                     (float2 *)q->tstats, q->size[L], N / 128);
}

// loss of the rows in act[0] / yb and the gradient of the mean loss into gw / gb.
// Each gradient with respect to a pre-activation is kept as hi + lo BF16
// planes (the lo plane n_pad x N elements after the hi plane), and every
// product with it runs over both planes, so the backward pass rounds like
// FP32 storage while the matrix cores take BF16 operands.
void backward(gpet_mlp *q, uint32_t n, uint32_t n_pad, hipStream_t st) {
  const int L = q->n_layers;
  const int C = q->size[L], Cp = q->psize[L];
  if (q->n_first) {
    const int n1 = q->n_first, n2 = q->n_second, G = q->n_groups;
    const float *T = q->master + q->tab_off;
    hipLaunchKernelGGL(k_factored_ce, dim3(cdiv(n_pad, 4)), dim3(256), 0, st, q->logits, Cp, n1, n2, G, T, q->yb, n,
                       n_pad, 1.0f / (float)n, q->dz[0], (size_t)n_pad * Cp, q->row_loss, q->erow, q->flag);
    const size_t nt = (size_t)(n1 - 1) * n2;
    hipLaunchKernelGGL(k_table_grad_part, dim3(cdiv(n2, 256), n1 - 1, kTableSlices), dim3(256), 0, st, q->dz[0],
                       (size_t)n_pad * Cp, Cp, n1, n2, G, q->erow, n_pad, kTableSlices, q->part);
    hipLaunchKernelGGL(k_reduce_slices, dim3(cdiv(nt, 256)), dim3(256), 0, st, q->part, kTableSlices, nt,
                       q->gb + q->tab_off);
  } else {
    hipLaunchKernelGGL(k_softmax_ce, dim3(cdiv(n_pad, 4)), dim3(256), 0, st, q->logits, Cp, C, q->yb, n, n_pad,
                       1.0f / (float)n, q->dz[0], (size_t)n_pad * Cp, q->row_loss, q->flag);
  }
  hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(1024), 0, st, q->row_loss, n_pad, q->loss_sum);
  int cur = 0;
  for (int l = L - 1; l >= 0; --l) {
    const int K = q->psize[l], N = q->psize[l + 1];
    const size_t lo = (size_t)n_pad * N; // the lo plane of dz
    // dW[o][i] = sum_r dz[r][o] act[r][i]: A = dz^T (M = N, K = rows, twice:
    // hi then lo), B(k = r, n = i) = act[r][i]; split over rows into partial
    // products, then summed in slice order
    const int K2 = 2 * (int)n_pad;
    const int sp = split_count(N, K, K2);
    const size_t ne = (size_t)N * K;
    if (sp > 1) {
      gemm<true, true, EPI_F32>(q->dz[cur], N, q->act[l], K, N, K, K2, nullptr, nullptr, q->part, K, st, sp, ne, lo,
                                (int)n_pad);
      hipLaunchKernelGGL(k_reduce_slices, dim3(cdiv(ne, 256)), dim3(256), 0, st, q->part, sp, ne, q->gw[l]);
    } else {
      gemm<true, true, EPI_F32>(q->dz[cur], N, q->act[l], K, N, K, K2, nullptr, nullptr, q->gw[l], K, st, 1, 0, lo,
                                (int)n_pad);
    }
    const int cols = q->size[l + 1], slices = (int)std::min<uint32_t>(64u, std::max<uint32_t>(1u, n_pad / 128));
    hipLaunchKernelGGL(k_col_sum_part, dim3(cdiv(cols, 256), slices), dim3(256), 0, st, q->dz[cur], lo, N, n_pad,
                       cols, slices, q->part_b);
    hipLaunchKernelGGL(k_reduce_slices, dim3(cdiv(cols, 256)), dim3(256), 0, st, q->part_b, slices, (size_t)cols,
                       q->gb + q->b_off[l]);
    if (l) {
      // dh[r][i] = sum_o dz[r][o] W[o][i] over both planes of dz (K = 2N),
      // masked by the ReLU of layer l's input and split into the next hi + lo
      gemm<false, true, EPI_MASK_HILO>(q->dz[cur], N, q->wb[l], K, (int)n_pad, K, 2 * N, nullptr, q->act[l],
                                       q->dz[cur ^ 1], K, st, 1, (size_t)n_pad * K, lo, N);
      cur ^= 1;
    }
  }
}

} // namespace

int gpet::surrogate_hits(gpet_mlp *q, const DevScene *d_scene, const SurSpecD &P, const SurQueue &Q, uint32_t nq,
                         uint32_t k0, uint32_t k1, uint32_t inst_rng, const RunArgs &H, hipStream_t st,
                         std::string &err, uint64_t *n_none) {
  if (nq == 0) return GPET_OK;
  constexpr uint32_t kChunk = 1u << 18;
  if (ensure_workspace(q, std::min(nq, kChunk)) != GPET_OK) {
    err = q->ctx->err;
    return GPET_ERR_HIP;
  }
  const int C = q->size[q->n_layers], Cp = q->psize[q->n_layers];
  // the tile statistics need the forward product kernel for the last layer
  // (input width <= 256) and at most 64 tiles of 128 classes
  const int Kl = q->psize[q->n_layers - 1];
  const bool tiles = Kl <= kNtKmax && Kl % kTk == 0 && Cp / 128 <= 64;
  for (uint32_t off = 0; off < nq; off += kChunk) {
    const uint32_t n = std::min(kChunk, nq - off);
    const uint32_t n_pad = (uint32_t)pad_to((int)n, kRowPad);
    hipLaunchKernelGGL(k_pack_input, dim3(cdiv(n_pad, 8)), dim3(32, 8), 0, st, Q.x + (size_t)6 * off,
                       (const int32_t *)nullptr, (const uint32_t *)nullptr, n, q->size[0], q->psize[0], n_pad,
                       q->act[0], (int32_t *)nullptr);
    if (q->n_first) {
      forward_infer(q, n_pad, st);
      const float *T = q->master + q->tab_off;
      const uint32_t *an = Q.anchor + (size_t)kMaxLayers * off;
      const int n2 = q->n_second;
      // the positions in registers: each layer's W^2 in chunks of 64 of their
      // own, B the smallest of 8, 20, 32 that holds them all
      const int WW = (2 * P.chalf + 1) * (2 * P.chalf + 1);
      const int chunks = n2 / WW * ((WW + 63) / 64);
      if (chunks <= 8)
        hipLaunchKernelGGL(k_sample_factored<8>, dim3(cdiv(n, 4)), dim3(256), 0, st, q->logits, Cp, q->n_first, n2,
                           q->n_groups, T, n, Q.ev + off, Q.meta + off, an, d_scene, P.chalf, k0, k1, inst_rng,
                           Q.cls + off, Q.pos + off);
      else if (chunks <= 20)
        hipLaunchKernelGGL(k_sample_factored<20>, dim3(cdiv(n, 4)), dim3(256), 0, st, q->logits, Cp, q->n_first, n2,
                           q->n_groups, T, n, Q.ev + off, Q.meta + off, an, d_scene, P.chalf, k0, k1, inst_rng,
                           Q.cls + off, Q.pos + off);
      else // at most 32 chunks (checked by the caller)
        hipLaunchKernelGGL(k_sample_factored<32>, dim3(cdiv(n, 4)), dim3(256), 0, st, q->logits, Cp, q->n_first, n2,
                           q->n_groups, T, n, Q.ev + off, Q.meta + off, an, d_scene, P.chalf, k0, k1, inst_rng,
                           Q.cls + off, Q.pos + off);
    } else if (tiles) {
      forward_sample(q, n_pad, st);
      hipLaunchKernelGGL(k_sample_tiles, dim3(cdiv(n, 4)), dim3(256), 0, st, (const float2 *)q->tstats, Cp / 128,
                         q->logits, Cp, C, n, Q.ev + off, Q.meta + off, k0, k1, inst_rng, Q.cls + off, Q.pos + off);
    } else {
      forward_infer(q, n_pad, st);
      hipLaunchKernelGGL(k_sample_classes, dim3(cdiv(n, 4)), dim3(256), 0, st, q->logits, Cp, C, n, Q.ev + off,
                         Q.meta + off, k0, k1, inst_rng, Q.cls + off, Q.pos + off);
    }
  }
  // nonzero flags -> positions; the class-0 count comes from the same scan
  unsigned long long *cnt = H.hit_count;
  uint32_t last[2] = {0u, 0u};
  (void)hipMemcpyAsync(&last[0], Q.pos + nq - 1, 4, hipMemcpyDeviceToHost, st);
  scan_exclusive_u32(Q.pos, nq, Q.scan_tmp, st);
  (void)hipMemcpyAsync(&last[1], Q.pos + nq - 1, 4, hipMemcpyDeviceToHost, st);
  hipLaunchKernelGGL(k_emit_hits, dim3(cdiv(nq, 256)), dim3(256), 0, st, nq, Q.cls, Q.pos, Q.ev, Q.meta, Q.anchor, Q.e,
                     Q.time, d_scene, P, k0, k1, inst_rng, H);
  if (wait_stream(st) != hipSuccess) {
    err = "surrogate: kernel error";
    return GPET_ERR_HIP;
  }
  const uint64_t kept = (uint64_t)last[1] + last[0];
  *n_none += nq - kept;
  // hit count += kept (device-side, after the emit kernel read the old value)
  hipLaunchKernelGGL(k_add_u64, dim3(1), dim3(1), 0, st, cnt, (unsigned long long)kept);
  return hipGetLastError() == hipSuccess ? GPET_OK : GPET_ERR_HIP;
}

extern "C" {

static gpet_status mlp_create(gpet_ctx *c, int32_t n_sizes, const int32_t *sizes, int32_t n_first,
                              int32_t n_groups, const float *weights, gpet_mlp **out) {
  if (!c || !out || !sizes) return GPET_ERR_ARG;
  *out = nullptr;
  if (n_sizes < 2 || n_sizes > 16) {
    c->err = "mlp: 2..16 layer widths";
    return GPET_ERR_ARG;
  }
  if (sizes[0] < 1 || sizes[0] > 256) {
    c->err = "mlp: input width in 1..256";
    return GPET_ERR_ARG;
  }
  for (int i = 1; i < n_sizes; ++i)
    if (sizes[i] < 1 || sizes[i] > 8192) {
      c->err = "mlp: layer widths in 1..8192";
      return GPET_ERR_ARG;
    }
  if (n_first && (n_first < 2 || n_first > 64 || n_first >= sizes[n_sizes - 1] || n_groups < 1 ||
                  n_groups > n_first - 1 || (sizes[n_sizes - 1] - n_first) % n_groups != 0)) {
    c->err = "mlp: the energy head takes 2..64 of the outputs, the rest splits into 1..n_first - 1 equal "
             "position blocks";
    return GPET_ERR_ARG;
  }
  gpet_mlp *q = new (std::nothrow) gpet_mlp();
  if (!q) return GPET_ERR_ARG;
  q->ctx = c;
  q->device = c->device;
  q->size.assign(sizes, sizes + n_sizes);
  q->n_layers = n_sizes - 1;
  q->psize.resize(n_sizes);
  q->psize[0] = pad_to(sizes[0], kTile);
  for (int i = 1; i < n_sizes; ++i) q->psize[i] = pad_to(sizes[i], kWidthPad);
  size_t o = 0;
  for (int l = 0; l < q->n_layers; ++l) {
    q->w_off.push_back(o);
    o += (size_t)sizes[l] * sizes[l + 1];
    q->b_off.push_back(o);
    o += (size_t)sizes[l + 1];
  }
  q->n_first = n_first;
  q->n_groups = n_first ? n_groups : 0;
  q->n_second = n_first ? (sizes[n_sizes - 1] - n_first) / n_groups : 0;
  q->tab_off = o; // the offset table of a factored output follows the layers
  if (n_first) o += (size_t)(n_first - 1) * q->n_second;
  q->n_params = o;
  (void)hipSetDevice(c->device);
  int widest = 0;
  for (int i = 1; i < n_sizes; ++i) widest = std::max(widest, q->psize[i]);
  q->bp_stride = widest;
  bool ok = hipMalloc((void **)&q->master, o * 4) == hipSuccess && hipMalloc((void **)&q->m, o * 4) == hipSuccess &&
            hipMalloc((void **)&q->v, o * 4) == hipSuccess && hipMalloc((void **)&q->gb, o * 4) == hipSuccess &&
            hipMalloc((void **)&q->bp, (size_t)q->n_layers * widest * 4) == hipSuccess &&
            hipMemset(q->bp, 0, (size_t)q->n_layers * widest * 4) == hipSuccess;
  q->wb.assign(q->n_layers, nullptr);
  q->gw.assign(q->n_layers, nullptr);
  for (int l = 0; ok && l < q->n_layers; ++l) {
    const size_t e = (size_t)q->psize[l] * q->psize[l + 1];
    ok = hipMalloc((void **)&q->wb[l], e * 2) == hipSuccess && hipMalloc((void **)&q->gw[l], e * 4) == hipSuccess &&
         hipMemset(q->wb[l], 0, e * 2) == hipSuccess;
  }
  if (!ok) {
    gpet_mlp_destroy(q);
    c->err = "mlp: device allocation failed";
    return GPET_ERR_HIP;
  }
  *out = q;
  if (weights) return gpet_mlp_set_weights(q, weights);
  std::vector<float> zero(o, 0.f);
  return gpet_mlp_set_weights(q, zero.data());
}

gpet_status gpet_mlp_create(gpet_ctx *c, int32_t n_sizes, const int32_t *sizes, const float *weights, gpet_mlp **out) {
  return mlp_create(c, n_sizes, sizes, 0, 0, weights, out);
}

gpet_status gpet_mlp_create_factored(gpet_ctx *c, int32_t n_sizes, const int32_t *sizes, int32_t n_first,
                                     int32_t n_groups, const float *weights, gpet_mlp **out) {
  if (n_first < 2) {
    if (c) c->err = "mlp: the energy head needs at least 2 classes";
    return GPET_ERR_ARG;
  }
  return mlp_create(c, n_sizes, sizes, n_first, n_groups, weights, out);
}

void gpet_mlp_destroy(gpet_mlp *q) {
  if (!q) return;
  (void)hipSetDevice(q->device);
  (void)hipDeviceSynchronize();
  free_workspace(q);
  for (uint16_t *p : q->wb)
    if (p) (void)hipFree(p);
  for (float *p : q->gw)
    if (p) (void)hipFree(p);
  for (void *p : {(void *)q->master, (void *)q->m, (void *)q->v, (void *)q->gb, (void *)q->bp})
    if (p) (void)hipFree(p);
  delete q;
}

gpet_status gpet_mlp_set_weights(gpet_mlp *q, const float *w) {
  if (!q || !w) return GPET_ERR_ARG;
  gpet_ctx *c = q->ctx;
  (void)hipSetDevice(q->device);
  for (size_t i = 0; i < q->n_params; ++i)
    if (!std::isfinite(w[i])) return mlp_fail(q, GPET_ERR_ARG, "mlp: weights must be finite");
  if (hipMemcpy(q->master, w, q->n_params * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(q->m, 0, q->n_params * 4) != hipSuccess || hipMemset(q->v, 0, q->n_params * 4) != hipSuccess)
    return mlp_fail(q, GPET_ERR_HIP, "mlp: upload failed");
  q->adam_t = 0;
  for (int l = 0; l < q->n_layers; ++l) {
    const int rows = q->size[l + 1], cols = q->size[l];
    hipLaunchKernelGGL(k_to_bf16, dim3(cdiv((size_t)rows * cols, 256)), dim3(256), 0, c->stream,
                       q->master + q->w_off[l], rows, cols, q->wb[l], q->psize[l]);
    (void)hipMemcpyAsync(q->bp + l * q->bp_stride, q->master + q->b_off[l], (size_t)rows * 4,
                         hipMemcpyDeviceToDevice, c->stream);
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return mlp_fail(q, GPET_ERR_HIP, "mlp: weight conversion");
  return GPET_OK;
}

gpet_status gpet_mlp_get_weights(gpet_mlp *q, float *w) {
  if (!q || !w) return GPET_ERR_ARG;
  (void)hipSetDevice(q->device);
  if (hipStreamSynchronize(q->ctx->stream) != hipSuccess ||
      hipMemcpy(w, q->master, q->n_params * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return mlp_fail(q, GPET_ERR_HIP, "mlp: download failed");
  return GPET_OK;
}

gpet_status gpet_mlp_get_state(gpet_mlp *q, float *w, float *m, float *v, uint64_t *step) {
  if (!q || !w || !m || !v || !step) return GPET_ERR_ARG;
  (void)hipSetDevice(q->device);
  if (hipStreamSynchronize(q->ctx->stream) != hipSuccess ||
      hipMemcpy(w, q->master, q->n_params * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(m, q->m, q->n_params * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(v, q->v, q->n_params * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return mlp_fail(q, GPET_ERR_HIP, "mlp: state download failed");
  *step = q->adam_t;
  return GPET_OK;
}

gpet_status gpet_mlp_set_state(gpet_mlp *q, const float *w, const float *m, const float *v, uint64_t step) {
  if (!q || !w || !m || !v) return GPET_ERR_ARG;
  for (size_t i = 0; i < q->n_params; ++i)
    if (!std::isfinite(m[i]) || !std::isfinite(v[i]) || v[i] < 0.0f)
      return mlp_fail(q, GPET_ERR_ARG, "mlp: Adam moments must be finite (second moments >= 0)");
  // the weights (and the BF16 copies and biases the kernels read), then the moments and the step
  gpet_status s = gpet_mlp_set_weights(q, w);
  if (s) return s;
  (void)hipSetDevice(q->device);
  if (hipMemcpy(q->m, m, q->n_params * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(q->v, v, q->n_params * 4, hipMemcpyHostToDevice) != hipSuccess)
    return mlp_fail(q, GPET_ERR_HIP, "mlp: state upload failed");
  q->adam_t = step;
  return GPET_OK;
}

gpet_status gpet_mlp_forward(gpet_mlp *q, uint32_t n, const float *x, float *logits) {
  if (!q) return GPET_ERR_ARG;
  if (n && (!x || !logits)) return mlp_fail(q, GPET_ERR_ARG, "mlp forward: null buffers");
  if (n == 0) return GPET_OK;
  (void)hipSetDevice(q->device);
  gpet_status s = ensure_workspace(q, n);
  if (s) return s;
  hipStream_t st = q->ctx->stream;
  const uint32_t n_pad = (uint32_t)pad_to((int)n, kRowPad);
  hipLaunchKernelGGL(k_pack_input, dim3(cdiv(n_pad, 8)), dim3(32, 8), 0, st, x, (const int32_t *)nullptr,
                     (const uint32_t *)nullptr, n, q->size[0], q->psize[0], n_pad, q->act[0], (int32_t *)nullptr);
  forward_infer(q, n_pad, st);
  const int C = q->size[q->n_layers], Cp = q->psize[q->n_layers];
  if (hipMemcpy2DAsync(logits, (size_t)C * 4, q->logits, (size_t)Cp * 4, (size_t)C * 4, n, hipMemcpyDeviceToDevice,
                       st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return mlp_fail(q, GPET_ERR_HIP, "mlp forward");
  return GPET_OK;
}

gpet_status gpet_mlp_loss_grad(gpet_mlp *q, uint32_t n, const float *x, const int32_t *y, double *loss, float *grad) {
  if (!q) return GPET_ERR_ARG;
  if (!n || !x || !y || !loss || !grad) return mlp_fail(q, GPET_ERR_ARG, "mlp loss_grad: arguments");
  (void)hipSetDevice(q->device);
  gpet_status s = ensure_workspace(q, n);
  if (s) return s;
  hipStream_t st = q->ctx->stream;
  const uint32_t n_pad = (uint32_t)pad_to((int)n, kRowPad);
  launch_fill_u32(q->flag, 0u, 1, st);
  hipLaunchKernelGGL(k_pack_input, dim3(cdiv(n_pad, 8)), dim3(32, 8), 0, st, x, y, (const uint32_t *)nullptr, n,
                     q->size[0], q->psize[0], n_pad, q->act[0], q->yb);
  forward(q, n_pad, st);
  backward(q, n, n_pad, st);
  double ls = 0.0;
  uint32_t bad = 0;
  std::vector<float> gpad;
  if (hipMemcpyAsync(&ls, q->loss_sum, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&bad, q->flag, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(grad, q->gb, q->n_params * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return mlp_fail(q, GPET_ERR_HIP, "mlp loss_grad");
  if (bad) return mlp_fail(q, GPET_ERR_ARG, "mlp loss_grad: a label lies outside [0, classes)");
  // weight gradients from their padded buffers (biases were read with gb)
  for (int l = 0; l < q->n_layers; ++l) {
    const int rows = q->size[l + 1], cols = q->size[l], ld = q->psize[l];
    gpad.resize((size_t)q->psize[l + 1] * ld);
    if (hipMemcpy(gpad.data(), q->gw[l], gpad.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return mlp_fail(q, GPET_ERR_HIP, "mlp loss_grad");
    for (int r = 0; r < rows; ++r) std::memcpy(grad + q->w_off[l] + (size_t)r * cols, &gpad[(size_t)r * ld], cols * 4);
  }
  *loss = ls / (double)n;
  return GPET_OK;
}

gpet_status gpet_mlp_train(gpet_mlp *q, uint64_t n_pairs, const float *x, const int32_t *y,
                           const gpet_train_params *hp, float *loss_per_step) {
  if (!q) return GPET_ERR_ARG;
  if (!hp || !x || !y || n_pairs == 0) return mlp_fail(q, GPET_ERR_ARG, "mlp train: arguments");
  if (hp->batch < 1 || hp->batch > (1u << 20) || !(hp->lr > 0) || !(hp->beta1 >= 0 && hp->beta1 < 1) ||
      !(hp->beta2 >= 0 && hp->beta2 < 1) || !(hp->eps > 0))
    return mlp_fail(q, GPET_ERR_ARG, "mlp train: hyperparameters");
  (void)hipSetDevice(q->device);
  gpet_status s = ensure_workspace(q, hp->batch);
  if (s) return s;
  hipStream_t st = q->ctx->stream;
  const uint32_t n = hp->batch, n_pad = (uint32_t)pad_to((int)n, kRowPad);
  std::vector<double> losses(hp->steps, 0.0);
  double *d_losses = nullptr;
  if (hp->steps && hipMalloc((void **)&d_losses, (size_t)hp->steps * 8) != hipSuccess)
    return mlp_fail(q, GPET_ERR_HIP, "mlp train: allocation failed");
  launch_fill_u32(q->flag, 0u, 1, st);
  for (uint32_t t = 0; t < hp->steps; ++t) {
    hipLaunchKernelGGL(k_batch_indices, dim3(cdiv(n, 256)), dim3(256), 0, st, (uint32_t)hp->seed,
                       (uint32_t)(hp->seed >> 32), (uint32_t)(q->adam_t + 1), n, n_pairs, q->idx);
    hipLaunchKernelGGL(k_pack_input, dim3(cdiv(n_pad, 8)), dim3(32, 8), 0, st, x, y, (const uint32_t *)q->idx, n,
                       q->size[0], q->psize[0], n_pad, q->act[0], q->yb);
    forward(q, n_pad, st);
    backward(q, n, n_pad, st);
    (void)hipMemcpyAsync(d_losses + t, q->loss_sum, 8, hipMemcpyDeviceToDevice, st);
    ++q->adam_t;
    const float c1 = (float)(1.0 / (1.0 - std::pow(hp->beta1, (double)q->adam_t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(hp->beta2, (double)q->adam_t)));
    for (int l = 0; l < q->n_layers; ++l) {
      const int rows = q->size[l + 1], cols = q->size[l];
      hipLaunchKernelGGL(k_adam, dim3(cdiv((size_t)rows * cols, 256)), dim3(256), 0, st, q->master + q->w_off[l],
                         q->m + q->w_off[l], q->v + q->w_off[l], q->gw[l], rows, cols, q->psize[l], (float)hp->lr,
                         (float)hp->beta1, (float)hp->beta2, (float)hp->eps, c1, c2, q->wb[l], q->psize[l],
                         (float *)nullptr);
      hipLaunchKernelGGL(k_adam, dim3(cdiv(rows, 256)), dim3(256), 0, st, q->master + q->b_off[l],
                         q->m + q->b_off[l], q->v + q->b_off[l], q->gb + q->b_off[l], 1, rows, rows, (float)hp->lr,
                         (float)hp->beta1, (float)hp->beta2, (float)hp->eps, c1, c2, (uint16_t *)nullptr, 0,
                         q->bp + l * q->bp_stride);
    }
    if (q->n_first) { // the offset table: fp32 master only (the kernels read it there)
      const int rows = q->n_first - 1, cols = q->n_second;
      hipLaunchKernelGGL(k_adam, dim3(cdiv((size_t)rows * cols, 256)), dim3(256), 0, st, q->master + q->tab_off,
                         q->m + q->tab_off, q->v + q->tab_off, q->gb + q->tab_off, rows, cols, cols, (float)hp->lr,
                         (float)hp->beta1, (float)hp->beta2, (float)hp->eps, c1, c2, (uint16_t *)nullptr, 0,
                         (float *)nullptr);
    }
  }
  bool ok = hipGetLastError() == hipSuccess;
  if (hp->steps)
    ok = ok && hipMemcpyAsync(losses.data(), d_losses, (size_t)hp->steps * 8, hipMemcpyDeviceToHost, st) == hipSuccess;
  uint32_t bad = 0;
  ok = ok && hipMemcpyAsync(&bad, q->flag, 4, hipMemcpyDeviceToHost, st) == hipSuccess;
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (d_losses) (void)hipFree(d_losses);
  if (!ok) return mlp_fail(q, GPET_ERR_HIP, "mlp train: kernel error");
  if (bad) return mlp_fail(q, GPET_ERR_ARG, "mlp train: a label lies outside [0, classes)");
  if (loss_per_step)
    for (uint32_t t = 0; t < hp->steps; ++t) loss_per_step[t] = (float)(losses[t] / (double)n);
  return GPET_OK;
}

} // extern "C"
