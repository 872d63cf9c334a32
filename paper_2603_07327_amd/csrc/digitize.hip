// digitize.hip -- crystal-level digitizer for gfx950.
//
// Pipeline (all on the device, stream ordered):
//   1. hits -> 64-bit keys (instance, event, crystal, photon, hit index),
//      grouped by event bucket (counters with one atomic per group of equal
//      buckets in a wave) and sorted inside each bucket by one wave;
//   2. adder: one single per run of equal (instance, event, crystal); energy
//      and energy-weighted depth are summed as exact 2^-32 fixed-point
//      integers, so the result does not depend on the order of the hits;
//   3. Gaussian blur from the digitizer Philox stream and the energy window;
//   4. windowed singles sorted by (instance, time, single index): stable radix
//      passes over the time bucket, then one wave per bucket; split into
//      clusters at gaps larger than the coincidence window; inside a cluster,
//      non-retriggering windows are resolved sequentially by the cluster's
//      first lane; counts are scanned so that the coincidence list comes out
//      in a fixed order.
// A bucket too large for the in-LDS sort sends the step to a plain LSD radix
// sort over every key bit.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "gpet_internal.hpp"

namespace gpet {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanBlock * kScanItems;

// exclusive prefix sum of one value per thread over a 256-thread block
// (wave_tot: 4 words of LDS; ends with the block synchronized once)
__device__ __forceinline__ uint32_t block_exclusive_256(uint32_t x, uint32_t *wave_tot) {
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wave_tot[w] = inc;
  __syncthreads();
  uint32_t before = 0;
  for (int k = 0; k < w; ++k) before += wave_tot[k];
  return before + inc - x;
}

// ---------------------------------------------------------------------------
// exclusive scan of u32 in place: tile sums, their scan (recursively), then
// each tile scanned with its offset.  The grand total can go straight to a
// (pinned host) word, so no copy is needed to read it back.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(const uint32_t *a, size_t n, uint32_t *tile_sums) {
  __shared__ uint32_t ws[kScanBlock / 64];
  const size_t base = (size_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
#pragma unroll
  for (int r = 0; r < kScanItems; ++r) {
    const size_t i = base + (size_t)r * kScanBlock + threadIdx.x;
    if (i < n) s += a[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (__lane_id() == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

// thread t scans the 16 consecutive items [t 16, t 16 + 16) of its tile.
// tile_offs: the tiles' offsets, or (raw) their sums, of which the block adds
// up those before its own tile.
__global__ void __launch_bounds__(kScanBlock) k_scan_apply(uint32_t *a, size_t n, const uint32_t *tile_offs,
                                                           uint32_t *total, int raw) {
  __shared__ uint32_t ws[kScanBlock / 64];
  __shared__ uint32_t s_off;
  if (raw) {
    uint32_t t = 0;
    for (uint32_t k = threadIdx.x; k < blockIdx.x; k += kScanBlock) t += tile_offs[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if (__lane_id() == 0) ws[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) s_off = ws[0] + ws[1] + ws[2] + ws[3];
    __syncthreads();
  }
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  const bool full = base + kScanItems <= n && (((uintptr_t)a) & 15u) == 0;
  if (full) {
    const uint4 *q = (const uint4 *)(a + base);
#pragma unroll
    for (int k = 0; k < kScanItems / 4; ++k) {
      const uint4 u = q[k];
      v[4 * k] = u.x;
      v[4 * k + 1] = u.y;
      v[4 * k + 2] = u.z;
      v[4 * k + 3] = u.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = base + k < n ? a[base + k] : 0u;
  }
  uint32_t run = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t t = v[k];
    v[k] = run;
    run += t;
  }
  const uint32_t off = block_exclusive_256(run, ws) + (raw ? s_off : tile_offs ? tile_offs[blockIdx.x] : 0u);
  if (full) {
    uint4 *q = (uint4 *)(a + base);
#pragma unroll
    for (int k = 0; k < kScanItems / 4; ++k)
      q[k] = make_uint4(v[4 * k] + off, v[4 * k + 1] + off, v[4 * k + 2] + off, v[4 * k + 3] + off);
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
      if (base + k < n) a[base + k] = v[k] + off;
  }
  // the thread holding the last item knows the grand total
  if (total && base < n && base + kScanItems >= n) *total = off + run;
}

static size_t scan_scratch_words(size_t n) {
  size_t w = 0;
  while (n > (size_t)kScanTile) {
    n = (n + kScanTile - 1) / kScanTile;
    w += n;
  }
  return w + 1;
}

// Tiles up to which each apply block adds up the sums of the tiles before its
// own (at most 4096 words read per block, 16.7 M items) instead of a scan of
// its own.
constexpr size_t kScanRawTiles = 4096;

// `total` (may be null) receives the sum
static void exclusive_scan(uint32_t *a, size_t n, uint32_t *tmp, hipStream_t st, uint32_t *total = nullptr) {
  if (n == 0) return;
  const size_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanBlock), 0, st, a, n, (const uint32_t *)nullptr, total, 0);
    return;
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(kScanBlock), 0, st, (const uint32_t *)a, n, tmp);
  const int raw = tiles <= kScanRawTiles ? 1 : 0;
  if (!raw) exclusive_scan(tmp, tiles, tmp + tiles, st);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)tiles), dim3(kScanBlock), 0, st, a, n, (const uint32_t *)tmp,
                     total, raw);
}

// ---------------------------------------------------------------------------
// Bucket map: a monotone map of (u64) keys spread evenly over their range
// (event ids, event times) to buckets of a few dozen keys.
// ---------------------------------------------------------------------------
// Bucket of a key: instance i = key >> inst_shift owns buckets
// [base[i], base[i] + count[i]); inside them the bucket grows linearly with the
// key's local value v = (key >> local_shift) & local_mask (event index or time),
// so every instance gets buckets in proportion to its item count.  A key whose
// instance lies outside the map gets bucket nb.
// With one instance its map travels in the kernel arguments (base0, count0,
// scale0) and the arrays are not read.
struct BucketMap {
  int inst_shift, local_shift;
  unsigned long long local_mask;
  const uint32_t *base, *count;
  const float *scale; // buckets per unit of v
  uint32_t n_inst, nb;
  uint32_t base0, count0;
  float scale0;
};

__device__ __forceinline__ uint32_t bucket_of(const BucketMap &M, unsigned long long key) {
  const uint32_t i = M.inst_shift < 64 ? (uint32_t)(key >> M.inst_shift) : 0u;
  if (i >= M.n_inst) return M.nb;
  const unsigned long long v = (key >> M.local_shift) & M.local_mask;
  const bool one = M.n_inst == 1;
  const float sc = one ? M.scale0 : M.scale[i];
  const uint32_t cnt = one ? M.count0 : M.count[i], base = one ? M.base0 : M.base[i];
  // The map only has to be non-decreasing in the key (each bucket is then
  // sorted by key and value, so any such map gives the same order).  A value
  // of 32 bits or more is taken as hi 2^32 + lo in one FMA of its two halves
  // converted to FP32: below 2^56 the high half converts exactly, above it the
  // low half is under half an ULP, and rounding is monotone either way.
  const float fv = M.local_mask >> 32
                       ? fmaf((float)(uint32_t)(v >> 32), 4294967296.0f, (float)(uint32_t)v)
                       : (float)(uint32_t)v;
  const uint32_t b = min((uint32_t)(fv * sc), cnt - 1u);
  return base + b;
}

// ---------------------------------------------------------------------------
// Stable LSD radix passes over (u64 key, u32 value) with up to 8-bit digits.
// A digit is either a byte of the key or a digit of its bucket.  Tiles of 4096
// items: a histogram pass, a scan of the (digit, tile) counts, then a scatter
// that ranks the tile in LDS (wave ballots keep equal digits in input order)
// and writes it out digit by digit, so stores come in runs.
// ---------------------------------------------------------------------------
constexpr int kTileBlock = 256;
constexpr int kTileItems = 16;
constexpr int kTile = kTileBlock * kTileItems;
constexpr int kTileWaveItems = kTile / (kTileBlock / 64);

struct KeyDigit {
  int shift;
  __device__ __forceinline__ uint32_t operator()(unsigned long long k) const { return (uint32_t)(k >> shift) & 255u; }
};

struct BucketDigit {
  BucketMap M;
  int shift;
  uint32_t mask;
  __device__ __forceinline__ uint32_t operator()(unsigned long long k) const {
    return (bucket_of(M, k) >> shift) & mask;
  }
};

// lanes of the wave holding the same digit (among `valid` lanes)
__device__ __forceinline__ uint64_t digit_peers(uint32_t digit, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (digit >> b) & 1u;
    const uint64_t v = __ballot(bit);
    m &= bit ? v : ~v;
  }
  return m;
}

template <class Digit>
__global__ void __launch_bounds__(kTileBlock) k_tile_hist(const unsigned long long *keys, size_t n, Digit dg,
                                                          uint32_t *hist, uint32_t n_tiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * kTile;
#pragma unroll 4
  for (int r = 0; r < kTileItems; ++r) {
    const size_t i = base + (size_t)r * kTileBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[dg(keys[i])], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// `offs` = exclusive scan of the histogram (digit-major), i.e. where the
// tile's first item of each digit goes
template <class Digit>
__global__ void __launch_bounds__(kTileBlock) k_tile_scatter(const unsigned long long *kin, const uint32_t *vin,
                                                             unsigned long long *kout, uint32_t *vout, size_t n,
                                                             Digit dg, const uint32_t *offs, uint32_t n_tiles) {
  constexpr int kWaves = kTileBlock / 64;
  __shared__ unsigned long long sk[kTile];
  __shared__ uint32_t sv[kTile];
  __shared__ uint8_t sd[kTile];
  __shared__ uint32_t wcnt[kWaves][256]; // per-wave running counts, then per-wave starts
  __shared__ uint32_t lstart[256], gstart[256], wave_tot[kWaves];
  const int t = threadIdx.x, w = t >> 6, lane = __lane_id();
#pragma unroll
  for (int k = 0; k < kWaves; ++k) wcnt[k][t] = 0;
  gstart[t] = offs[(size_t)t * n_tiles + blockIdx.x];
  __syncthreads();
  // wave w ranks items [w 1024, w 1024 + 1024) of the tile, 64 per round, in order
  const size_t base = (size_t)blockIdx.x * kTile + (size_t)w * kTileWaveItems;
  const uint64_t below = __lanemask_lt();
  unsigned long long k[kTileItems];
  uint32_t v[kTileItems], d[kTileItems], rk[kTileItems];
#pragma unroll
  for (int r = 0; r < kTileItems; ++r) {
    const size_t i = base + (size_t)r * 64 + lane;
    const bool valid = i < n;
    k[r] = valid ? kin[i] : 0ull;
    v[r] = valid ? vin[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kTileItems; ++r) {
    const bool valid = base + (size_t)r * 64 + lane < n;
    d[r] = valid ? dg(k[r]) : 0u;
    const uint64_t peers = digit_peers(d[r], valid);
    const uint32_t before = (uint32_t)__popcll(peers & below);
    const uint32_t run = wcnt[w][d[r]];
    rk[r] = run + before;
    // LDS operations of a wave complete in order, so every lane has read the
    // count before its group's first lane replaces it
    if (valid && before == 0) wcnt[w][d[r]] = run + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  uint32_t c[kWaves], tot = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) {
    c[q] = wcnt[q][t];
    tot += c[q];
  }
  const uint32_t ls = block_exclusive_256(tot, wave_tot);
  lstart[t] = ls;
  uint32_t acc = ls;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) {
    wcnt[q][t] = acc;
    acc += c[q];
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kTileItems; ++r) {
    if (base + (size_t)r * 64 + lane < n) {
      const uint32_t p = wcnt[w][d[r]] + rk[r];
      sk[p] = k[r];
      sv[p] = v[r];
      sd[p] = (uint8_t)d[r];
    }
  }
  __syncthreads();
  const size_t t0 = (size_t)blockIdx.x * kTile;
  const uint32_t cnt = (uint32_t)min((size_t)kTile, n - t0);
  for (uint32_t idx = t; idx < cnt; idx += kTileBlock) {
    const uint32_t dd = sd[idx];
    const uint32_t pos = gstart[dd] + (idx - lstart[dd]);
    if (pos < n) {
      kout[pos] = sk[idx];
      vout[pos] = sv[idx];
    }
  }
}

struct SortBufs {
  unsigned long long *k0, *k1;
  uint32_t *v0, *v1;
  uint32_t *hist;    // 256 * tiles
  uint32_t *scan_tmp;
};

static inline uint32_t tile_count(size_t n) { return (uint32_t)((n + kTile - 1) / kTile); }

// one stable pass (ki, vi) -> (ko, vo) by the digit dg
template <class Digit>
static void radix_pass(SortBufs &b, const unsigned long long *ki, const uint32_t *vi, unsigned long long *ko,
                       uint32_t *vo, size_t n, Digit dg, hipStream_t st) {
  const uint32_t tiles = tile_count(n);
  hipLaunchKernelGGL(k_tile_hist<Digit>, dim3(tiles), dim3(kTileBlock), 0, st, ki, n, dg, b.hist, tiles);
  exclusive_scan(b.hist, (size_t)256 * tiles, b.scan_tmp, st);
  hipLaunchKernelGGL(k_tile_scatter<Digit>, dim3(tiles), dim3(kTileBlock), 0, st, ki, vi, ko, vo, n, dg, b.hist,
                     tiles);
}

// sorts (k0, v0) over the low `bits` bits; returns true if the result sits in (k1, v1)
static bool radix_sort(SortBufs &b, size_t n, int bits, hipStream_t st) {
  if (n <= 1 || bits <= 0) return false;
  bool flip = false;
  for (int shift = 0; shift < bits; shift += 8) {
    unsigned long long *ki = flip ? b.k1 : b.k0, *ko = flip ? b.k0 : b.k1;
    uint32_t *vi = flip ? b.v1 : b.v0, *vo = flip ? b.v0 : b.v1;
    radix_pass(b, ki, vi, ko, vo, n, KeyDigit{shift}, st);
    flip = !flip;
  }
  return flip;
}

// Per-instance constants of the digitizer (device arrays of n_inst entries).
struct InstTab {
  const uint32_t *first, *n_events, *cpp, *rng;
  const uint32_t *ncr; // crystals of the instance's scanner
  uint32_t n_inst;
};

// The hits a sort key is built from.
struct HitSrc {
  const uint32_t *ev, *gid, *aux, *inst; // inst may be null (one instance)
  InstTab T;
  int gid_bits, inst_shift;
  uint32_t *err; // set to 2 for a hit whose ids lie outside its instance
  // one: a single instance, whose first event, event count and crystal count
  // come here, so that the checks take no per-lane table loads
  bool one;
  uint32_t first0, n_events0, ncr0;
};

// key = instance | (event - first) | gid | photon | index of the hit within its
// photon (7 bits, saturated): unique per hit, so the sorted order is fixed.
// Hits outside their instance's event range or with a crystal id outside the
// instance's scanner are flagged (*H.err = 2).
__device__ __forceinline__ unsigned long long hit_key(const HitSrc &H, size_t i) {
  if (H.one) { // the same checks and key with the table values in scalars
    const uint32_t a = H.aux[i], g = H.gid[i], in = H.inst ? H.inst[i] : 0u;
    const uint32_t low = ((a & 1u) << 7) | min(a >> 8, 127u);
    uint32_t e = H.ev[i] - H.first0;
    if (in != 0u || e >= H.n_events0 || g >= H.ncr0 || (H.gid_bits < 32 && (g >> H.gid_bits) != 0)) {
      *H.err = 2u;
      e = 0;
    }
    return ((((unsigned long long)e << H.gid_bits) | (g & ((1ull << H.gid_bits) - 1))) << 8) | low;
  }
  const InstTab &T = H.T;
  const uint32_t in = H.inst ? H.inst[i] : 0u;
  const uint32_t a = H.aux[i];
  const uint32_t low = ((a & 1u) << 7) | min(a >> 8, 127u);
  uint32_t e = 0;
  const uint32_t g = H.gid[i];
  if (in >= T.n_inst || H.ev[i] - T.first[in] >= T.n_events[in] || g >= T.ncr[in] ||
      (H.gid_bits < 32 && (g >> H.gid_bits) != 0)) {
    *H.err = 2u;
  } else {
    e = H.ev[i] - T.first[in];
  }
  const unsigned long long inst_bits =
      H.inst_shift < 64 ? (unsigned long long)(in < T.n_inst ? in : 0u) << H.inst_shift : 0ull;
  return inst_bits | ((((unsigned long long)e << H.gid_bits) | (g & ((1ull << H.gid_bits) - 1))) << 8) | low;
}

__global__ void k_hit_keys(size_t n, HitSrc H, unsigned long long *key, uint32_t *val) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = hit_key(H, i);
  val[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// Bucket sort of (u64 key, u32 value) by (key, value): order the items by
// bucket, then sort each bucket: a wave per few buckets with a register
// bitonic network, the rare larger bucket in LDS.  Two ways to group by bucket:
//   * clustered keys (hits: an event's hits share a bucket) -- per-bucket
//     counters with one atomic per group of equal buckets in a wave, scan,
//     scatter; the order inside a bucket depends on the atomics;
//   * spread keys (times) -- stable radix passes over the bucket number, no
//     global atomics, then bucket starts from the sorted buckets.
// The final sort by (key, value) makes the result deterministic either way.
// ---------------------------------------------------------------------------
constexpr int kLocalSort = 1024; // largest bucket sorted in LDS
constexpr int kBucketMean = 48;  // target items per bucket: most fit one per lane

// lanes of the wave whose value equals this lane's (one ballot per distinct
// value; the leader's value is read as a wave-uniform lane read)
__device__ __forceinline__ uint64_t equal_peers(uint32_t v, bool valid) {
  uint64_t left = __ballot(valid), mine = 0;
  while (left) {
    const int leader = __ffsll((unsigned long long)left) - 1;
    const uint32_t lv = __builtin_amdgcn_readlane(v, leader);
    const bool eq = valid && v == lv;
    const uint64_t m = __ballot(eq); // (every lane of this value is still left)
    if (eq) mine = m;
    left &= ~m;
  }
  return mine;
}

// keys whose bucket falls outside the map are skipped and flagged (*flag = 2).
// FROM_HITS: the keys are built from the hits here (and in the scatter), not
// read from a key array, and the values are the hit indices.
template <bool FROM_HITS>
__global__ void k_bucket_count(const unsigned long long *key, HitSrc H, size_t n, BucketMap M, uint32_t *count,
                               uint32_t *flag) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t kb = i < n ? bucket_of(M, FROM_HITS ? hit_key(H, i) : key[i]) : 0u;
  if (i < n && kb >= M.nb) *flag = 2u;
  const bool valid = i < n && kb < M.nb;
  const uint32_t b = valid ? kb : 0u;
  const uint64_t peers = equal_peers(b, valid);
  if (valid && (peers & __lanemask_lt()) == 0) atomicAdd(&count[b], (uint32_t)__popcll(peers));
}

// cursor holds bucket starts on entry and bucket ends on exit
template <bool FROM_HITS>
__global__ void k_bucket_scatter(const unsigned long long *kin, const uint32_t *vin, HitSrc H, size_t n, BucketMap M,
                                 uint32_t *cursor, unsigned long long *kout, uint32_t *vout) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long k = i < n ? (FROM_HITS ? hit_key(H, i) : kin[i]) : 0ull;
  const uint32_t kb = i < n ? bucket_of(M, k) : 0u;
  const bool valid = i < n && kb < M.nb;
  const uint32_t b = valid ? kb : 0u;
  const uint64_t below = __lanemask_lt();
  const uint64_t peers = equal_peers(b, valid);
  const int leader = valid ? __ffsll((unsigned long long)peers) - 1 : 0;
  uint32_t base = 0;
  if (valid && (peers & below) == 0) base = atomicAdd(&cursor[b], (uint32_t)__popcll(peers));
  base = __shfl(base, leader);
  const uint32_t pos = base + (uint32_t)__popcll(peers & below);
  if (valid && pos < n) {
    kout[pos] = k;
    vout[pos] = FROM_HITS ? (uint32_t)i : vin[i];
  }
}

// start[b] = first position of bucket b in keys sorted by bucket, b in [0, nb];
// keys outside the map (bucket nb) sit at the end and are flagged (*flag = 2)
__global__ void k_bucket_bounds(const unsigned long long *key, size_t n, BucketMap M, uint32_t *start,
                                uint32_t *flag) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t b = min(bucket_of(M, key[i]), M.nb);
  if (b == M.nb && (i == 0 || min(bucket_of(M, key[i - 1]), M.nb) != M.nb)) *flag = 2u;
  const int64_t prev = i ? (int64_t)min(bucket_of(M, key[i - 1]), M.nb) : -1;
  for (int64_t q = prev + 1; q <= (int64_t)b; ++q) start[q] = (uint32_t)i;
  if (i == n - 1)
    for (uint32_t q = b + 1; q <= M.nb; ++q) start[q] = (uint32_t)n;
}

// Items per instance: a block counts kInstItems items in an LDS histogram
// (for up to kInstLds instances) and adds its nonzero bins to the global
// counts; with more instances every item adds to the global count directly.
constexpr int kInstLds = 4096;
constexpr int kInstItems = 16;

template <class Inst, class Weight>
__device__ __forceinline__ void inst_histogram(size_t n, uint32_t n_inst, uint32_t *count, Inst inst_of,
                                               Weight weight_of) {
  __shared__ uint32_t h[kInstLds];
  const bool lds = n_inst <= (uint32_t)kInstLds;
  if (lds)
    for (uint32_t b = threadIdx.x; b < n_inst; b += blockDim.x) h[b] = 0u;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * blockDim.x * kInstItems;
  for (int r = 0; r < kInstItems; ++r) {
    const size_t i = base + (size_t)r * blockDim.x + threadIdx.x;
    if (i >= n) break;
    const uint32_t wgt = weight_of(i);
    if (wgt == 0u) continue;
    const uint32_t v = inst_of(i);
    if (v < n_inst) {
      if (lds) atomicAdd(&h[v], wgt);
      else atomicAdd(&count[v], wgt);
    }
  }
  __syncthreads();
  if (lds)
    for (uint32_t b = threadIdx.x; b < n_inst; b += blockDim.x)
      if (h[b]) atomicAdd(&count[b], h[b]);
}

// items per instance (instance = key >> shift)
__global__ void __launch_bounds__(256) k_inst_count(const unsigned long long *key, size_t n, int shift,
                                                    uint32_t n_inst, uint32_t *count) {
  inst_histogram(
      n, n_inst, count, [&](size_t i) { return shift < 64 ? (uint32_t)(key[i] >> shift) : 0u; },
      [](size_t) { return 1u; });
}

static inline unsigned inst_grid(size_t n) { return (unsigned)((n + 256 * kInstItems - 1) / (256 * kInstItems)); }

__device__ __forceinline__ bool pair_less(unsigned long long ka, uint32_t va, unsigned long long kb, uint32_t vb) {
  return ka < kb || (ka == kb && va < vb);
}

// lane_xor for the sorting networks: the DPP forms as plain DPP moves (every
// lane reads a lane that exists, so no old value has to be set up first)
__device__ __forceinline__ uint32_t lane_xor_mov(uint32_t x, int lx) {
  switch (lx) {
  case 1:
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false); // quad_perm [1,0,3,2]
  case 2:
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false); // quad_perm [2,3,0,1]
  case 8:
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, false); // row_ror:8
  default:
    return lane_xor(x, lx);
  }
}

__device__ __forceinline__ unsigned long long lane_xor_u64(unsigned long long x, int lx) {
  const uint32_t lo = lane_xor_mov((uint32_t)x, lx), hi = lane_xor_mov((uint32_t)(x >> 32), lx);
  return ((unsigned long long)hi << 32) | lo;
}

// Bitonic sort of P = 64 E packed u64 items held E per lane, ascending.
// Element l E + r sits in register r of lane l, so partners closer than E stay
// in the lane and the others are one lane exchange away.
template <int E>
__device__ __forceinline__ void wave_bitonic_u64(unsigned long long (&p)[E]) {
  const int lane = __lane_id();
  constexpr int P = 64 * E;
#pragma unroll
  for (int kk = 2; kk <= P; kk <<= 1) {
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1) {
      if (j < E) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int u = r ^ j;
          if (u > r) {
            const bool asc = ((lane * E + r) & kk) == 0;
            const unsigned long long lo = p[r] < p[u] ? p[r] : p[u], hi = p[r] < p[u] ? p[u] : p[r];
            p[r] = asc ? lo : hi;
            p[u] = asc ? hi : lo;
          }
        }
      } else {
        const int lx = j / E; // partner lane distance
        const bool lower = (lane & lx) == 0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const bool asc = ((lane * E + r) & kk) == 0;
          const unsigned long long q = lane_xor_u64(p[r], lx);
          const bool q_less = q < p[r];
          // the lower element of an ascending pair keeps the smaller one
          if (lower == asc ? q_less : !q_less) p[r] = q;
        }
      }
    }
  }
}

// Sorts the first 64 E (key, value) items of k/v (lane-major, `size` >= 1
// real items, the rest ~0) with one wave.  Each key is taken relative to the
// first item's key b: u = key - b + 2^(63 - vbits), and u << vbits | value is
// one u64 whose order is the (key, value) order when every value is below
// 2^vbits and every u fits 64 - vbits bits short of all ones.  Returns false,
// leaving k/v as they were, when some key lies too far from b.
template <int E>
__device__ __forceinline__ bool wave_sort_packed(unsigned long long (&k)[2], uint32_t (&v)[2], uint32_t size,
                                                 int vbits) {
  const uint32_t lane = __lane_id();
  const unsigned long long b =
      ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(k[0] >> 32)) << 32) |
      (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)k[0]);
  const long long bias = 1ll << (63 - vbits);
  bool far = false;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const long long d = (long long)(k[r] - b);
    if (lane * E + r < size && (d < -bias || d > bias - 2)) far = true;
  }
  if (__ballot(far)) return false;
  unsigned long long p[E];
#pragma unroll
  for (int r = 0; r < E; ++r)
    p[r] = lane * E + r < size ? ((k[r] - b + (unsigned long long)bias) << vbits) | v[r] : ~0ull;
  wave_bitonic_u64<E>(p);
  const unsigned long long vmask = (1ull << vbits) - 1ull;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    k[r] = (p[r] >> vbits) + b - (unsigned long long)bias;
    v[r] = (uint32_t)(p[r] & vmask);
  }
  return true;
}

constexpr int kWaveSort = 128;   // largest bucket sorted by one wave
// consecutive buckets per wave: with one, the network's constant lane masks
// are made where they are used (a loop over several buckets kept them live
// across it and spilled them to vector lanes)
constexpr int kWaveBuckets = 1;

// a bucket of up to 64 items goes one per lane, up to 128 two per lane
__device__ __forceinline__ void wave_load_bucket(const unsigned long long *key, const uint32_t *val, uint32_t lo,
                                                 uint32_t size, unsigned long long (&k)[2], uint32_t (&v)[2]) {
  const uint32_t lane = __lane_id();
  const uint32_t e = size <= 64 ? 1u : 2u;
  const uint32_t n_ld = size <= (uint32_t)kWaveSort ? size : 0u;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const uint32_t t = lane * e + r;
    const bool ld = r < (int)e && t < n_ld;
    k[r] = ld ? key[lo + t] : ~0ull;
    v[r] = ld ? val[lo + t] : ~0u;
  }
}

// kWaveBuckets consecutive buckets per wave (with more than one, the next one
// loading while the current one sorts); bucket b spans [start[b], start[b + 1]).  Buckets a wave
// cannot take (over 128 items, keys spanning 2^32 or more) are listed in big[]
// (count in *n_big) for the block sort.  Values are below 2^vbits (1..32).
// heads (may be null): for keys whose runs of equal key >> head_shift never
// cross a bucket, heads[i] = 1 where such a run starts (the run heads of the
// adder), written here for the buckets sorted here.
__global__ void __launch_bounds__(256) k_bucket_wave_sort(unsigned long long *key, uint32_t *val,
                                                          const uint32_t *start, uint32_t nb, int vbits,
                                                          uint32_t *big, uint32_t *n_big, uint32_t *heads,
                                                          int head_shift) {
  const uint32_t b0 = (blockIdx.x * 4u + (threadIdx.x >> 6)) * kWaveBuckets;
  if (b0 >= nb) return;
  const uint32_t lane = __lane_id();
  const uint32_t nq = min((uint32_t)kWaveBuckets, nb - b0);
  // the wave's bucket bounds, start[b0 + j] in lane j <= nq, all loaded at once
  const uint32_t bound = lane <= nq ? start[b0 + lane] : 0u;
  uint32_t lo = __shfl(bound, 0), hi = __shfl(bound, 1);
  unsigned long long k[2];
  uint32_t v[2];
  wave_load_bucket(key, val, lo, hi - lo, k, v);
#pragma unroll 1
  for (uint32_t q = 0; q < nq; ++q) {
    uint32_t nhi = hi;
    unsigned long long kn[2] = {~0ull, ~0ull};
    uint32_t vn[2] = {~0u, ~0u};
    if (q + 1 < nq) {
      nhi = __shfl(bound, (int)q + 2);
      wave_load_bucket(key, val, hi, nhi - hi, kn, vn);
    }
    const uint32_t size = hi - lo;
    bool listed = size > (uint32_t)kWaveSort;
    if (size == 1 && heads && lane == 0) heads[lo] = 1u;
    if (size > 1 && !listed) {
      const uint32_t e = size <= 64 ? 1u : 2u;
      if (e == 1 ? wave_sort_packed<1>(k, v, size, vbits) : wave_sort_packed<2>(k, v, size, vbits)) {
        // the item before element r of this lane: element r - 1 of the lane, or
        // the last element of the lane before
        const unsigned long long last = e == 1 ? k[0] : k[1];
        const unsigned long long up = ((unsigned long long)__shfl_up((uint32_t)(last >> 32), 1) << 32) |
                                      __shfl_up((uint32_t)last, 1);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const uint32_t t = lane * e + r;
          if (r < (int)e && t < size) {
            key[lo + t] = k[r];
            val[lo + t] = v[r];
            if (heads) {
              const unsigned long long prev = r == 0 ? up : k[0];
              heads[lo + t] = (t == 0 || (k[r] >> head_shift) != (prev >> head_shift)) ? 1u : 0u;
            }
          }
        }
      } else {
        listed = true;
      }
    }
    if (listed && lane == 0) big[atomicAdd(n_big, 1u)] = b0 + q;
    lo = hi;
    hi = nhi;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      k[r] = kn[r];
      v[r] = vn[r];
    }
  }
}

// one block per listed bucket (grid-stride over the list), bitonic network in LDS
__global__ void __launch_bounds__(256) k_bucket_block_sort(unsigned long long *key, uint32_t *val,
                                                           const uint32_t *start, const uint32_t *big,
                                                           const uint32_t *n_big, uint32_t *overflow,
                                                           uint32_t *heads, int head_shift) {
  __shared__ unsigned long long sk[kLocalSort];
  __shared__ uint32_t sv[kLocalSort];
  const uint32_t listed = *n_big;
  for (uint32_t it = blockIdx.x; it < listed; it += gridDim.x) {
    const uint32_t b = big[it];
    const uint32_t lo = start[b], hi = start[b + 1];
    const uint32_t size = hi - lo;
    if (size > (uint32_t)kLocalSort) {
      if (threadIdx.x == 0) *overflow = 1u;
      // (its heads are cleared, so every head flag stays 0 or 1 until the
      // caller's fallback sort redoes them)
      if (heads)
        for (uint32_t t = threadIdx.x; t < size; t += blockDim.x) heads[lo + t] = 0u;
      continue;
    }
    uint32_t P = 2;
    while (P < size) P <<= 1;
    for (uint32_t t = threadIdx.x; t < P; t += blockDim.x) {
      sk[t] = t < size ? key[lo + t] : ~0ull;
      sv[t] = t < size ? val[lo + t] : ~0u;
    }
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t t = threadIdx.x; t < P; t += blockDim.x) {
          const uint32_t u = t ^ j;
          if (u > t) {
            const bool up = (t & k) == 0;
            const bool swap = up ? pair_less(sk[u], sv[u], sk[t], sv[t]) : pair_less(sk[t], sv[t], sk[u], sv[u]);
            if (swap) {
              const unsigned long long tk = sk[t];
              sk[t] = sk[u];
              sk[u] = tk;
              const uint32_t tv = sv[t];
              sv[t] = sv[u];
              sv[u] = tv;
            }
          }
        }
        __syncthreads();
      }
    }
    for (uint32_t t = threadIdx.x; t < size; t += blockDim.x) {
      key[lo + t] = sk[t];
      val[lo + t] = sv[t];
      if (heads) heads[lo + t] = (t == 0 || (sk[t] >> head_shift) != (sk[t - 1] >> head_shift)) ? 1u : 0u;
    }
    __syncthreads();
  }
}

static int log2_ceil(uint64_t x) {
  int b = 0;
  while ((1ull << b) < x && b < 63) ++b;
  return b;
}

struct BucketBufs {
  uint32_t *count;       // nb + 1 bucket starts (>= max_buckets + 1 words)
  size_t max_buckets;
  uint32_t *n_big;       // device word: listed big buckets
  uint32_t *big;         // big-bucket list (>= max_buckets words)
  uint32_t *map;         // per-instance bucket map (3 words per instance)
  uint32_t *pinned_flag; // pinned host word the kernels set when the bucket sort fails
  uint32_t *pinned_map;
};

// Sorts the items (b.k0, b.v0), whose values are below value_bound (at most
// 2^32), by (key, value) into (out_k, out_v), which is
// (b.k1, b.v1) or, after an even number of radix passes, (b.k0, b.v0).
// CLUSTERED picks the grouping by bucket counters, which leaves (k0, v0)
// intact; the radix passes over the bucket number use both pairs.  `items[i]`
// is the number of keys of instance i and `range[i]` the extent of their local
// value.  Returns 1 when the map needs more buckets than the scratch holds
// (nothing launched).  Otherwise the work is enqueued; the caller zeroes
// *bb.pinned_flag beforehand and finds it nonzero after the stream has run the
// work when a bucket was too large for LDS (1) or a key fell outside the map
// (2): then the output is not sorted.  The kernels store to the pinned word
// directly, so no copy is needed to read it.
template <bool CLUSTERED>
static uint32_t bucket_sort(SortBufs &b, BucketBufs &bb, size_t n, uint64_t value_bound, int inst_shift, int local_shift,
                            unsigned long long local_mask, const std::vector<uint64_t> &items,
                            const std::vector<double> &range, hipStream_t st, uint32_t *scan_tmp,
                            const unsigned long long *&out_k, const uint32_t *&out_v, const HitSrc *hits = nullptr,
                            uint32_t *zero_extra = nullptr, size_t n_extra = 0, uint32_t *heads = nullptr,
                            int head_shift = 0) {
  const size_t ni = items.size();
  std::vector<uint32_t> base(ni), cnt(ni);
  std::vector<float> scale(ni);
  size_t nb = 0;
  for (size_t i = 0; i < ni; ++i) {
    const uint64_t c = std::max<uint64_t>(1, (items[i] + kBucketMean - 1) / kBucketMean);
    base[i] = (uint32_t)nb;
    cnt[i] = (uint32_t)c;
    scale[i] = (float)((double)c / std::max(range[i], 1.0));
    nb += c;
  }
  if (nb > bb.max_buckets) return 1u; // let the caller fall back
  // per-instance map arrays live behind the bucket counters
  uint32_t *d_base = bb.map, *d_cnt = bb.map + ni;
  float *d_scale = (float *)(bb.map + 2 * ni);
  if (ni > 1) {
    std::memcpy(bb.pinned_map, base.data(), ni * 4);
    std::memcpy(bb.pinned_map + ni, cnt.data(), ni * 4);
    std::memcpy(bb.pinned_map + 2 * ni, scale.data(), ni * 4);
    (void)hipMemcpyAsync(bb.map, bb.pinned_map, 3 * ni * 4, hipMemcpyHostToDevice, st);
  }
  BucketMap M{inst_shift, local_shift, local_mask, d_base, d_cnt, d_scale, (uint32_t)ni, (uint32_t)nb,
              base[0], cnt[0], scale[0]};
  // one launch zeroes the big-bucket count, the bucket counters (clustered) and
  // the caller's extra words (flags the kernels below may set)
  launch_zero3(bb.n_big, 1, CLUSTERED ? bb.count : nullptr, nb + 1, zero_extra, n_extra, st);
  const unsigned g = (unsigned)((n + 255) / 256);
  unsigned long long *ko = b.k1;
  uint32_t *vo = b.v1;
  if constexpr (CLUSTERED) {
    // count[0] = 0 and count[1 + b] counts bucket b: after the scan and the
    // scatter, count[b] is the start of bucket b and count[b + 1] its end
    // (with a hit source the keys come from the hits, and (k0, v0) are not read)
    const HitSrc H = hits ? *hits : HitSrc{};
    if (hits)
      hipLaunchKernelGGL(k_bucket_count<true>, dim3(g), dim3(256), 0, st, (const unsigned long long *)nullptr, H, n,
                         M, bb.count + 1, bb.pinned_flag);
    else
      hipLaunchKernelGGL(k_bucket_count<false>, dim3(g), dim3(256), 0, st, b.k0, H, n, M, bb.count + 1,
                         bb.pinned_flag);
    exclusive_scan(bb.count + 1, nb, scan_tmp, st);
    if (hits)
      hipLaunchKernelGGL(k_bucket_scatter<true>, dim3(g), dim3(256), 0, st, (const unsigned long long *)nullptr,
                         (const uint32_t *)nullptr, H, n, M, bb.count + 1, b.k1, b.v1);
    else
      hipLaunchKernelGGL(k_bucket_scatter<false>, dim3(g), dim3(256), 0, st, b.k0, b.v0, H, n, M, bb.count + 1,
                         b.k1, b.v1);
  } else {
    // stable passes over the bucket number, low digit first, (k0, v0) -> (k1, v1) -> ...
    const int bits = std::max(1, log2_ceil(nb + 1));
    const int passes = (bits + 7) / 8;
    const int width = (bits + passes - 1) / passes;
    for (int p = 0; p < passes; ++p) {
      const bool odd = (p & 1) != 0;
      radix_pass(b, odd ? b.k1 : b.k0, odd ? b.v1 : b.v0, odd ? b.k0 : b.k1, odd ? b.v0 : b.v1, n,
                 BucketDigit{M, p * width, (1u << width) - 1u}, st);
    }
    ko = (passes & 1) ? b.k1 : b.k0;
    vo = (passes & 1) ? b.v1 : b.v0;
    hipLaunchKernelGGL(k_bucket_bounds, dim3(g), dim3(256), 0, st, ko, n, M, bb.count, bb.pinned_flag);
  }
  const size_t sort_waves = (nb + kWaveBuckets - 1) / kWaveBuckets;
  hipLaunchKernelGGL(k_bucket_wave_sort, dim3((unsigned)((sort_waves + 3) / 4)), dim3(256), 0, st, ko, vo, bb.count,
                     (uint32_t)nb, std::max(1, log2_ceil(value_bound)), bb.big, bb.n_big, heads, head_shift);
  hipLaunchKernelGGL(k_bucket_block_sort, dim3(256), dim3(256), 0, st, ko, vo, bb.count, bb.big, bb.n_big,
                     bb.pinned_flag, heads, head_shift);
  out_k = ko;
  out_v = vo;
  return 0u;
}

// ---------------------------------------------------------------------------
// digitizer stages
// ---------------------------------------------------------------------------
// first hit of each (instance, event, crystal) run
__global__ void k_heads(size_t n, const unsigned long long *key, uint32_t *flag) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || (key[i] >> 8) != (key[i - 1] >> 8)) ? 1u : 0u;
}

// light sharing: the crystal read instead of `gid` (one of its existing edge
// neighbours in the same layer and module, in the order t-1, t+1, a-1, a+1,
// picked by the high half of pick * count); geo holds per instance the
// crystals per module and the layer words, row-major over instances
__device__ __forceinline__ uint32_t shared_crystal(uint32_t gid, const uint32_t *geo, uint32_t ni, uint32_t in,
                                                   uint32_t pick) {
  const uint32_t cpm = geo[in];
  const uint32_t *lw = geo + ni; // [word][instance]
  const uint32_t local = gid % cpm;
  const int nl = (int)lw[in];
  int l = 0;
  for (int k = 1; k < nl; ++k)
    if (local >= lw[(1 + k) * ni + in]) l = k;
  const uint32_t base = lw[(1 + l) * ni + in];
  const uint32_t nt = lw[(1 + kMaxLayers + l) * ni + in], na = lw[(1 + 2 * kMaxLayers + l) * ni + in];
  const uint32_t it = (local - base) % nt, ia = (local - base) / nt;
  uint32_t nb[4];
  uint32_t cnt = 0;
  if (it > 0) nb[cnt++] = gid - 1;
  if (it + 1 < nt) nb[cnt++] = gid + 1;
  if (ia > 0) nb[cnt++] = gid - nt;
  if (ia + 1 < na) nb[cnt++] = gid + nt;
  return cnt ? nb[((unsigned long long)pick * cnt) >> 32] : gid;
}

// parameters of the blur stage (energy and optional time / DOI resolution,
// light sharing, window, tallies) and its outputs per single
struct BlurArgs {
  uint32_t k0, k1;
  float fwhm, e_lo, e_hi;
  uint32_t *spp, *spec; // tallies (null when not kept here)
  uint32_t n_spp;
  float time_sigma, doi_sigma;
  unsigned long long ls_thresh;
  const uint32_t *geo;
  float *s_energy;
  uint32_t *s_win, *wflag;
  unsigned long long *block_max;
};

// Blur of single i (event ev, instance in_i, crystal gid hit, energy E): the
// blurred energy and window flags are written here; the crystal read (light
// sharing), the time and the depth are updated in place for the caller.
// Normal deviates by Box-Muller from the digitizer stream of (gid, event,
// instance): words 0, 1 for the energy, 2, 3 for the time.
__device__ __forceinline__ void blur_single(const BlurArgs &B, const InstTab &T, size_t i, uint32_t in_i,
                                            uint32_t ev, uint32_t &gid, float E, unsigned long long &tm,
                                            float &depth) {
  const uint32_t rng = T.rng[in_i];
  const uint32_t w_gid = gid; // the counters take the crystal that was hit
  const uint4 w = philox(B.k0, B.k1, make_uint4(gid, ev, rng, 3u));
  const float u0 = to_unit(w.x), u1 = to_unit(w.y);
  const float g = sqrtf(-2.0f * logf(u0)) * cos_rev(u1);
  const float sig = B.fwhm * sqrtf(511.0f * E) * (1.0f / 2.354820045f);
  const float Eb = E + sig * g;
  const uint32_t in = (Eb >= B.e_lo && Eb <= B.e_hi) ? 1u : 0u;
  B.s_energy[i] = Eb;
  B.s_win[i] = in;
  B.wflag[i] = in;
  if (B.ls_thresh) { // light sharing: stream 8 of (gid, event, instance)
    const uint4 v = philox(B.k0, B.k1, make_uint4(gid, ev, rng, 8u));
    if ((unsigned long long)v.x < B.ls_thresh) gid = shared_crystal(gid, B.geo, T.n_inst, in_i, v.y);
  }
  if (B.spp && in && gid < B.n_spp) atomicAdd(&B.spp[gid], 1u);
  if (B.spec && Eb >= 0.0f && Eb < 700.0f) atomicAdd(&B.spec[(int)Eb], 1u);
  if (B.time_sigma > 0.0f) { // timing resolution: rounded to the ps, not below 0
    const float gt = sqrtf(-2.0f * logf(to_unit(w.z))) * cos_rev(to_unit(w.w));
    const long long tb = (long long)tm + (long long)rintf(B.time_sigma * gt);
    tm = tb > 0 ? (unsigned long long)tb : 0ull;
  }
  if (B.doi_sigma > 0.0f) { // DOI resolution: stream 6 of (gid, event, instance)
    const uint4 v = philox(B.k0, B.k1, make_uint4(w_gid, ev, rng, 6u));
    depth += B.doi_sigma * (sqrtf(-2.0f * logf(to_unit(v.x))) * cos_rev(to_unit(v.y)));
  }
}

// the block's largest time stamp into B.block_max[blockIdx.x] (every window's
// keys must fit its width)
__device__ __forceinline__ void block_max_time(const BlurArgs &B, unsigned long long tm) {
  __shared__ unsigned long long s_max[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = __shfl_xor(tm, o);
    tm = t > tm ? t : tm;
  }
  if (__lane_id() == 0) s_max[threadIdx.x >> 6] = tm;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long b = s_max[0];
    for (int k = 1; k < 4; ++k) b = s_max[k] > b ? s_max[k] : b;
    B.block_max[blockIdx.x] = b;
  }
}

// the blur over singles already in the output arrays (after a module or panel
// readout merged them)
__global__ void __launch_bounds__(256) k_blur(size_t n, const uint32_t *s_ev, uint32_t *s_gid,
                                              const uint32_t *s_inst, InstTab T, const float *s_edep,
                                              unsigned long long *s_time, float *s_depth, BlurArgs B) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long tm = 0;
  if (i < n) {
    const uint32_t g0 = s_gid[i];
    uint32_t gid = g0;
    tm = s_time[i];
    float depth = B.doi_sigma > 0.0f ? s_depth[i] : 0.0f;
    blur_single(B, T, i, s_inst[i], s_ev[i], gid, s_edep[i], tm, depth);
    if (gid != g0) s_gid[i] = gid;
    if (B.time_sigma > 0.0f) s_time[i] = tm;
    if (B.doi_sigma > 0.0f) s_depth[i] = depth;
  }
  block_max_time(B, tm);
}

// One single per run of equal (instance, event, crystal) in key order; the
// event and crystal come out of the key.  e/d/t are the hits' energy, depth
// and time, indexed by perm.  BLUR: the blur stage of each single runs here
// too (crystal readout), so the singles are read back by no separate pass.
// Thread t of block g takes positions g 256 kAdderR + r 256 + t, r <
// kAdderR.  Every position's key, run index, hit index and that hit's
// payload are loaded before any run is summed (two dependent loads deep), so
// a single of one hit -- most of them -- needs nothing more; a run's further
// hits are loaded by its head.
constexpr int kAdderR = 4;

static inline unsigned adder_grid(size_t n) { return (unsigned)((n + 256 * kAdderR - 1) / (256 * kAdderR)); }

template <bool BLUR>
__global__ void __launch_bounds__(256) k_adder(size_t n, const unsigned long long *key, const uint32_t *perm,
                                               const uint32_t *seg, const float *edep, const float *depth,
                                               const unsigned long long *time, InstTab T, int gid_bits,
                                               unsigned long long ev_mask, int inst_shift, uint32_t *s_ev,
                                               uint32_t *s_gid, float *s_edep, float *s_depth,
                                               unsigned long long *s_time, uint32_t *s_inst_int,
                                               uint32_t *s_inst_out, uint64_t cap, BlurArgs B) {
  constexpr int R = kAdderR;
  const uint32_t lane = __lane_id();
  const size_t base = (size_t)blockIdx.x * blockDim.x * R + threadIdx.x;
  size_t i[R];
  unsigned long long k[R];
  uint32_t sg[R], h[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    i[r] = base + (size_t)r * blockDim.x;
    const bool in = i[r] < n;
    k[r] = in ? key[i[r]] : ~0ull;
    sg[r] = in ? seg[i[r]] : 0u;
    h[r] = in ? perm[i[r]] : 0u;
  }
  float e[R], d[R];
  unsigned long long t[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool in = i[r] < n;
    e[r] = in ? edep[h[r]] : 0.0f;
    d[r] = in ? depth[h[r]] : 0.0f;
    t[r] = in ? time[h[r]] : 0ull;
  }
  unsigned long long tmax = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    // the keys before and after this position: the neighbouring lanes', or
    // loaded at the wave's edges
    unsigned long long kprev = ((unsigned long long)__shfl_up((uint32_t)(k[r] >> 32), 1) << 32) |
                               __shfl_up((uint32_t)k[r], 1);
    unsigned long long knext = ((unsigned long long)__shfl_down((uint32_t)(k[r] >> 32), 1) << 32) |
                               __shfl_down((uint32_t)k[r], 1);
    const size_t ir = i[r];
    if (ir >= n) continue;
    if (lane == 0 && ir > 0) kprev = key[ir - 1];
    if (lane == 63 || ir + 1 >= n) knext = ir + 1 < n ? key[ir + 1] : ~0ull;
    const unsigned long long run = k[r] >> 8;
    const bool head = ir == 0 || (kprev >> 8) != run;
    if constexpr (BLUR) {
      // the window flags past the singles are zero: the k-th non-head hit
      // (k = i - seg[i]) clears position n - 1 - k, so [singles, n) is covered
      if (!head) {
        const size_t z = n - 1 - (ir - (size_t)sg[r]); // seg[i] <= i: head flags are 0 or 1
        if (z < n) B.wflag[z] = 0u;
      }
    }
    if (!head) continue;
    unsigned long long se = (unsigned long long)(e[r] * 4294967296.0f);
    unsigned long long sd = (unsigned long long)((e[r] * d[r]) * 4294967296.0f);
    unsigned long long tm = t[r];
    if (ir + 1 < n && (knext >> 8) == run) { // further hits of the run
      size_t j = ir + 1;
      do {
        const uint32_t hj = perm[j];
        const float ej = edep[hj];
        se += (unsigned long long)(ej * 4294967296.0f);
        sd += (unsigned long long)((ej * depth[hj]) * 4294967296.0f);
        tm = min(tm, time[hj]);
        ++j;
      } while (j < n && (key[j] >> 8) == run);
    }
    const uint32_t s = sg[r];
    if (s < cap) {
      const double E = (double)se * 0x1p-32;
      const uint32_t inst = inst_shift < 64 ? (uint32_t)(k[r] >> inst_shift) : 0u;
      const uint32_t ev = T.first[inst] + (uint32_t)((run >> gid_bits) & ev_mask);
      uint32_t gid = (uint32_t)(run & ((1ull << gid_bits) - 1));
      const float e_sum = (float)E;
      float dep = se ? (float)((double)sd / (double)se) : 0.0f;
      s_ev[s] = ev;
      s_edep[s] = e_sum;
      s_inst_int[s] = inst;
      if (s_inst_out) s_inst_out[s] = inst;
      if constexpr (BLUR) {
        blur_single(B, T, s, inst, ev, gid, e_sum, tm, dep);
        tmax = tm > tmax ? tm : tmax;
      }
      s_gid[s] = gid;
      s_depth[s] = dep;
      s_time[s] = tm;
    }
  }
  if constexpr (BLUR) block_max_time(B, tmax);
}

__global__ void __launch_bounds__(1024) k_max_u64(const unsigned long long *v, size_t n, unsigned long long *out) {
  __shared__ unsigned long long s[1024];
  unsigned long long m = 0;
#pragma unroll 8
  for (size_t i = threadIdx.x; i < n; i += 1024) m = v[i] > m ? v[i] : m;
  s[threadIdx.x] = m;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = s[threadIdx.x + o] > s[threadIdx.x] ? s[threadIdx.x + o] : s[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

// windowed singles: key = instance | time, value = single index
// ---------------------------------------------------------------------------
// readout levels: crystal singles (in instance, event, gid order) of one
// event in one readout unit (gid / unit[instance] crystals) form a run
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool same_unit(size_t i, size_t j, const uint32_t *ev, const uint32_t *gid,
                                          const uint32_t *inst, const uint32_t *unit) {
  const uint32_t a = inst[i];
  return a == inst[j] && ev[i] == ev[j] && gid[i] / unit[a] == gid[j] / unit[a];
}

__global__ void k_readout_heads(size_t n, const uint32_t *ev, const uint32_t *gid, const uint32_t *inst,
                                const uint32_t *unit, uint32_t *flag) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || !same_unit(i, i - 1, ev, gid, inst, unit)) ? 1u : 0u;
}

// one readout single per run: energies summed, earliest time, crystal and depth
// of the largest deposit (the first, i.e. lowest gid, on a tie); written at
// the run's scanned index into the o_* arrays
__global__ void k_readout_merge(size_t n, const uint32_t *seg, const uint32_t *ev, const uint32_t *gid,
                                const uint32_t *inst, const uint32_t *unit, const float *edep, const float *depth,
                                const unsigned long long *time, uint32_t *o_ev, uint32_t *o_gid, float *o_edep,
                                float *o_depth, unsigned long long *o_time, uint32_t *o_inst) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || (i > 0 && same_unit(i, i - 1, ev, gid, inst, unit))) return;
  double e = 0.0;
  unsigned long long tm = ~0ull;
  size_t best = i, j = i;
  do {
    e += (double)edep[j];
    tm = time[j] < tm ? time[j] : tm;
    if (edep[j] > edep[best]) best = j;
    ++j;
  } while (j < n && same_unit(j, i, ev, gid, inst, unit));
  const uint32_t g = seg[i];
  o_ev[g] = ev[best];
  o_gid[g] = gid[best];
  o_edep[g] = (float)e;
  o_depth[g] = depth[best];
  o_time[g] = tm;
  o_inst[g] = inst[best];
}

__global__ void k_readout_copy(size_t n, const uint32_t *a_ev, const uint32_t *a_gid, const float *a_edep,
                               const float *a_depth, const unsigned long long *a_time, const uint32_t *a_inst,
                               uint32_t *ev, uint32_t *gid, float *edep, float *depth, unsigned long long *time,
                               uint32_t *inst, uint32_t *inst_out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ev[i] = a_ev[i];
  gid[i] = a_gid[i];
  edep[i] = a_edep[i];
  depth[i] = a_depth[i];
  time[i] = a_time[i];
  inst[i] = a_inst[i];
  if (inst_out) inst_out[i] = a_inst[i];
}

// energy window of a sweep on the blurred energies: flag and a copy to scan
__global__ void k_window_flags(size_t n, const float *energy, const uint32_t *s_win, float e_lo, float e_hi,
                               uint32_t *flag, uint32_t *pos) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t in = (energy[i] >= e_lo && energy[i] <= e_hi && !(s_win[i] & 2u)) ? 1u : 0u;
  flag[i] = in;
  pos[i] = in;
}

// pos: the exclusive scan of the 0/1 window flags (in the window and not
// lost) over the n singles, `total` their sum; single i is flagged exactly
// when the scan steps by one after it, so the flags themselves are not read
__global__ void k_time_keys(size_t n, const uint32_t *pos, uint32_t total, const unsigned long long *s_time,
                            const uint32_t *s_inst, int time_bits, unsigned long long *key, uint32_t *val) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t p = pos[i], q = i + 1 < n ? pos[i + 1] : total;
  if (q - p != 1u || p >= total) return;
  key[p] = time_bits < 64 ? ((unsigned long long)s_inst[i] << time_bits) | s_time[i] : s_time[i];
  val[p] = (uint32_t)i;
}

// coincidences of the cluster starting at sorted position k (k must be a head)
template <bool WRITE>
__device__ __forceinline__ uint32_t resolve_cluster(size_t k, size_t n, const unsigned long long *t,
                                                    const uint32_t *idx, const uint32_t *s_gid,
                                                    const uint32_t *s_inst, const uint32_t *cpp_of,
                                                    unsigned long long W, uint32_t *first, uint32_t *second,
                                                    uint32_t out, uint64_t cap) {
  size_t end = k + 1;
  while (end < n && t[end] - t[end - 1] <= W) ++end;
  uint32_t c = 0;
  size_t i = k;
  while (i < end) {
    size_t j = i + 1;
    while (j < end && t[j] - t[i] <= W) ++j;
    if (j - i == 2) {
      const uint32_t a = idx[i], b = idx[i + 1];
      // a window never spans two instances (s_inst null: one instance)
      const uint32_t cpp = cpp_of[s_inst ? s_inst[a] : 0u];
      if (s_gid[a] / cpp != s_gid[b] / cpp) {
        if (WRITE && out + c < cap) {
          first[out + c] = a;
          second[out + c] = b;
        }
        ++c;
      }
    }
    i = j;
  }
  return c;
}

__global__ void k_coinc_count(size_t n, const unsigned long long *t, const uint32_t *idx, const uint32_t *s_gid,
                              const uint32_t *s_inst, const uint32_t *cpp_of, unsigned long long W, uint32_t *cnt) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const bool head = k == 0 || t[k] - t[k - 1] > W;
  cnt[k] = head ? resolve_cluster<false>(k, n, t, idx, s_gid, s_inst, cpp_of, W, nullptr, nullptr, 0, 0) : 0u;
}

__global__ void k_coinc_write(size_t n, const unsigned long long *t, const uint32_t *idx, const uint32_t *s_gid,
                              const uint32_t *s_inst, const uint32_t *cpp_of, unsigned long long W,
                              const uint32_t *off, uint32_t *first, uint32_t *second, uint64_t cap) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const bool head = k == 0 || t[k] - t[k - 1] > W;
  if (head) resolve_cluster<true>(k, n, t, idx, s_gid, s_inst, cpp_of, W, first, second, off[k], cap);
}

// coincidences per instance (instance of the first single)
__global__ void __launch_bounds__(256) k_coinc_inst(size_t n, const uint32_t *first, const uint32_t *s_inst,
                                                    uint32_t n_inst, uint32_t *count) {
  inst_histogram(n, n_inst, count, [&](size_t k) { return s_inst[first[k]]; }, [](size_t) { return 1u; });
}

// coincidences per instance from the per-cluster counts of time-sorted keys
// (instance = key >> shift)
__global__ void __launch_bounds__(256) k_coinc_inst_counts(size_t n, const uint32_t *cnt,
                                                           const unsigned long long *key, int shift,
                                                           uint32_t n_inst, uint32_t *count) {
  inst_histogram(
      n, n_inst, count, [&](size_t k) { return shift < 64 ? (uint32_t)(key[k] >> shift) : 0u; },
      [&](size_t k) { return cnt[k]; });
}

// runs after the hit keys have validated every crystal id; the bound on the
// per-crystal histogram is kept anyway, so no id can write past it
__global__ void k_hit_tallies(size_t n, const uint32_t *gid, const float *depth, uint32_t *hpc, uint32_t n_cr,
                              uint32_t *doi, int doi_bins, float panel_depth) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t g = gid[i];
  if (hpc && g < n_cr) atomicAdd(&hpc[g], 1u);
  if (doi) {
    int b = (int)floorf(depth[i] / panel_depth * (float)doi_bins);
    b = b < 0 ? 0 : (b >= doi_bins ? doi_bins - 1 : b);
    atomicAdd(&doi[b], 1u);
  }
}

// ---------------------------------------------------------------------------
// Dead time: the blurred singles in (instance, unit, time, index) order -- a
// stable radix sort by time, then a stable one by (instance, unit) -- and
// each unit's run scanned for losses.
// ---------------------------------------------------------------------------
__global__ void k_dead_time_keys(size_t n, const unsigned long long *s_time, unsigned long long *key,
                                 uint32_t *val) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = s_time[i];
  val[i] = (uint32_t)i;
}

// key of the single at sorted position p: (instance, unit); vin may alias vout
__global__ void k_dead_unit_keys(size_t n, const uint32_t *vin, const uint32_t *s_gid, const uint32_t *s_inst,
                                 const uint32_t *unit_size, int unit_bits, unsigned long long *kout,
                                 uint32_t *vout) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t i = vin[p];
  const uint32_t in = s_inst ? s_inst[i] : 0u;
  kout[p] = ((unsigned long long)in << unit_bits) | (s_gid[i] / unit_size[in]);
  vout[p] = i;
}

// paralyzable: lost when the previous single of the unit came less than tau earlier
__global__ void k_dead_paralyzable(size_t n, const unsigned long long *key, const uint32_t *val,
                                   const unsigned long long *s_time, unsigned long long tau, uint32_t *lost) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t i = val[p];
  uint32_t l = 0u;
  if (p > 0 && key[p] == key[p - 1]) l = s_time[i] - s_time[val[p - 1]] < tau ? 1u : 0u;
  lost[i] = l;
}

__global__ void k_dead_heads(size_t n, const unsigned long long *key, uint32_t *head) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  head[p] = (p == 0 || key[p] != key[p - 1]) ? 1u : 0u;
}

// start of each unit's run (pos: exclusive scan of the head flags)
__global__ void k_dead_starts(size_t n, const unsigned long long *key, const uint32_t *pos, uint32_t *start) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (p == 0 || key[p] != key[p - 1]) start[pos[p]] = (uint32_t)p;
}

// times in unit order, so the scan below reads them contiguously
__global__ void k_dead_gather(size_t n, const uint32_t *val, const unsigned long long *s_time,
                              unsigned long long *t_sorted) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  t_sorted[p] = s_time[val[p]];
}

// non-paralyzable: one wave per unit walks its run 1024 singles at a time,
// lane c taking the chunk of kDeadChunk consecutive singles c.  A chunk's
// kept set follows from the state entering it (whether a single was kept
// before, and the time of the last one): each lane runs the rule over its
// chunk from a guessed entry, takes the exit of the lane before as its next
// entry, and runs again until no entry changes.  Lane c is exact after c + 1
// rounds; as chains from different entries merge within a few singles, two
// or three rounds settle most windows.
constexpr int kDeadChunk = 16;
__global__ void __launch_bounds__(256) k_dead_nonparalyzable(uint32_t n_runs, const uint32_t *start, size_t n,
                                                             const uint32_t *val,
                                                             const unsigned long long *t_sorted,
                                                             unsigned long long tau, uint32_t *lost) {
  const uint32_t run = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (run >= n_runs) return; // whole waves leave together
  const int lane = (int)__lane_id();
  const size_t b = start[run], e = run + 1 < n_runs ? start[run + 1] : n;
  bool have_prev = false; // state entering the window (wave-uniform)
  unsigned long long last_prev = 0;
  for (size_t base = b; base < e; base += (size_t)64 * kDeadChunk) {
    const size_t c0 = base + (size_t)lane * kDeadChunk;
    const int nk = c0 >= e ? 0 : (e - c0 < (size_t)kDeadChunk ? (int)(e - c0) : kDeadChunk);
    unsigned long long t[kDeadChunk];
#pragma unroll
    for (int k = 0; k < kDeadChunk; ++k) t[k] = k < nk ? t_sorted[c0 + k] : 0ull;
    bool in_have = lane == 0 ? have_prev : false;
    unsigned long long in_last = lane == 0 ? last_prev : 0ull;
    uint32_t mask = 0;
    bool out_have = false;
    unsigned long long out_last = 0;
    for (int round = 0; round <= 64; ++round) {
      bool h = in_have;
      unsigned long long L = in_last;
      uint32_t m = 0;
#pragma unroll
      for (int k = 0; k < kDeadChunk; ++k) {
        if (k < nk && (!h || t[k] - L >= tau)) {
          m |= 1u << k;
          L = t[k];
          h = true;
        }
      }
      mask = m;
      out_have = h;
      out_last = L;
      // the entry of lane c is the exit of lane c - 1
      bool nh = __shfl_up((int)h, 1) != 0;
      unsigned long long nl = ((unsigned long long)(uint32_t)__shfl_up((int)(uint32_t)(L >> 32), 1) << 32) |
                              (uint32_t)__shfl_up((int)(uint32_t)L, 1);
      if (lane == 0) {
        nh = have_prev;
        nl = last_prev;
      }
      const bool changed = nh != in_have || (nh && nl != in_last);
      in_have = nh;
      in_last = nl;
      if (__ballot(changed) == 0) break;
    }
#pragma unroll
    for (int k = 0; k < kDeadChunk; ++k)
      if (k < nk) lost[val[c0 + k]] = ((mask >> k) & 1u) ? 0u : 1u;
    // empty chunks pass their entry through, so the last lane holds the window's exit
    have_prev = __builtin_amdgcn_readlane((int)out_have, 63) != 0;
    last_prev = ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(out_last >> 32), 63) << 32) |
                (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)out_last, 63);
  }
}

// lost singles leave the window (bit 1 of in_window); the in-window tallies
// and the spectrum count what survives
__global__ void k_dead_apply(size_t n, const uint32_t *lost, uint32_t *s_win, uint32_t *wflag, const uint32_t *s_gid,
                             const float *s_energy, uint32_t *spp, uint32_t n_spp, uint32_t *spec) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t l = lost[i], in = s_win[i] & 1u;
  s_win[i] = in | (l << 1);
  wflag[i] = (in && !l) ? 1u : 0u;
  if (l) return;
  if (spp && in && s_gid[i] < n_spp) atomicAdd(&spp[s_gid[i]], 1u);
  const float Eb = s_energy[i];
  if (spec && Eb >= 0.0f && Eb < 700.0f) atomicAdd(&spec[(int)Eb], 1u);
}

static inline unsigned grid_for(size_t n) { return (unsigned)((n + 255) / 256); }
// rows of the per-instance table: first event, event count, crystals per
// panel, RNG id, readout unit, dead-time unit, crystals per module, layer
// words, crystals of the scanner
constexpr int kTabRows = 8 + kLayerWords;

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int run_digitize(DigitizeArgs &D, DigitizeScratch &scr, hipStream_t st, std::string &err) {
  const size_t n = D.n_hits;
  const size_t ni = D.first.size();
  gpet_singles *S = D.singles;
  gpet_coincidences *C = D.coinc;
  const gpet_tallies *T = D.tallies;
  S->count = 0;
  S->windowed = 0;
  C->count = 0;
  if (D.sweep_out) std::fill(D.sweep_out, D.sweep_out + D.sweep_lo.size() * ni, (uint64_t)0);
  if (D.coinc_per_inst) std::fill(D.coinc_per_inst, D.coinc_per_inst + ni, 0ull);
  if (n == 0) return wait_stream(st) == hipSuccess ? GPET_OK : GPET_ERR_HIP;

  // scratch: 2 key + 2 value arrays, flags, positions, single instances, radix
  // histogram, scan temp, bucket counters and maps, instance table
  const size_t tiles = tile_count(n);
  const size_t max_buckets = n / kBucketMean + 1024 + 2 * ni;
  const size_t scan_words = scan_scratch_words(std::max<size_t>(std::max<size_t>(256 * tiles, n), max_buckets));
  // (each term one take() below, in the same order)
  const size_t need = align_up(n * 8) * 2 + align_up(n * 4) * 5 + align_up(256 * tiles * 4) +
                      align_up(scan_words * 4) + align_up((max_buckets + 1) * 4) + align_up(max_buckets * 4) +
                      align_up(8) + align_up(ni * 4 * 3) + align_up(ni * 4 * kTabRows) + align_up(ni * 4);
  // readback words: [0, 16) scalars that kernels write (scan totals, maximum
  // time, failure flags), [16, 16 + ni) per-instance counts, then the staging
  // of uploads: 3 ni words of bucket map, kTabRows ni words of instance table
  const size_t rb_words = 16 + (4 + kTabRows) * ni;
  if (scr.fixed) {
    // fixed scratch: nothing is allocated; the readback words sit behind the
    // sort buffers in device memory and are copied to a host array at each
    // synchronization
    if (ni != 1 || rb_words > kFixedHostWords) {
      err = "digitize: the fixed scratch serves one instance";
      return GPET_ERR_ARG;
    }
    if (need + align_up(rb_words * 4) > scr.bytes) {
      err = "digitize: " + std::to_string(n) + " hits need " + std::to_string(need + align_up(rb_words * 4)) +
            " bytes of scratch, more than the " + std::to_string(scr.bytes) + " bytes of the fixed scratch";
      return GPET_ERR_ARG;
    }
  } else {
    if (scr.bytes < need) {
      // a quarter of headroom: hit counts drift from call to call, and a
      // free + allocate pair costs about as much as the whole digitizer
      if (scr.buf) (void)hipFree(scr.buf);
      scr.buf = nullptr;
      scr.bytes = 0;
      scr.tab_at = nullptr; // the table went with the old buffer
      const size_t grow = need + need / 4;
      if (hipMalloc(&scr.buf, grow) != hipSuccess) {
        err = "digitize: device scratch allocation failed";
        return GPET_ERR_HIP;
      }
      scr.bytes = grow;
    }
    if (scr.pinned_bytes < rb_words * 4) {
      if (scr.pinned) (void)hipHostFree(scr.pinned);
      scr.pinned = nullptr;
      scr.pinned_bytes = 0;
      if (hipHostMalloc((void **)&scr.pinned, rb_words * 4, hipHostMallocDefault) != hipSuccess) {
        err = "digitize: pinned readback allocation failed";
        return GPET_ERR_HIP;
      }
      scr.pinned_bytes = rb_words * 4;
    }
  }
  char *p = (char *)scr.buf;
  auto take = [&](size_t bytes) {
    char *r = p;
    p += align_up(bytes);
    return (void *)r;
  };
  SortBufs sb;
  sb.k0 = (unsigned long long *)take(n * 8);
  sb.k1 = (unsigned long long *)take(n * 8);
  sb.v0 = (uint32_t *)take(n * 4);
  sb.v1 = (uint32_t *)take(n * 4);
  uint32_t *flag = (uint32_t *)take(n * 4);
  uint32_t *wpos = (uint32_t *)take(n * 4);
  uint32_t *s_inst = (uint32_t *)take(n * 4);
  sb.hist = (uint32_t *)take(256 * tiles * 4);
  sb.scan_tmp = (uint32_t *)take(scan_words * 4);
  BucketBufs bb;
  bb.count = (uint32_t *)take((max_buckets + 1) * 4);
  bb.max_buckets = max_buckets;
  bb.big = (uint32_t *)take(max_buckets * 4);
  bb.n_big = (uint32_t *)take(8);
  bb.map = (uint32_t *)take(ni * 4 * 3);
  // first, n_events, cpp, rng, readout unit, dead-time unit, crystals per module, layer words
  uint32_t *d_tab = (uint32_t *)take(ni * 4 * kTabRows);
  uint32_t *d_icount = (uint32_t *)take(ni * 4);
  // rb: the words kernels write (pinned host memory, or device memory behind
  // the fixed scratch); rbh: where the host reads them after a synchronization
  // and stages its uploads (the same pinned words, or a host array)
  uint32_t host_words[kFixedHostWords];
  uint32_t *rb = scr.fixed ? (uint32_t *)take(rb_words * 4) : (uint32_t *)scr.pinned;
  uint32_t *rbh = scr.fixed ? host_words : rb;
  if ((size_t)(p - (char *)scr.buf) > scr.bytes) {
    err = "digitize: scratch accounting does not cover its allocations";
    return GPET_ERR_HIP;
  }
  uint32_t *rb_count = rb + 16;         // device-visible per-instance counts
  const uint32_t *rbh_count = rbh + 16; // their host view
  bb.pinned_flag = rb + 12;
  bb.pinned_map = rbh + 16 + ni;
  uint32_t *tab = rbh + 16 + 4 * ni;
  auto sync = [&](const char *what) {
    if (wait_stream(st) != hipSuccess) {
      err = std::string("digitize: stream error ") + what;
      return false;
    }
    if (rbh != rb && hipMemcpy(rbh, rb, (16 + ni) * 4, hipMemcpyDeviceToHost) != hipSuccess) {
      err = std::string("digitize: readback failed ") + what;
      return false;
    }
    return true;
  };

  // instance table on the device (its pinned staging is not reused before the call ends)
  for (size_t i = 0; i < ni; ++i) {
    tab[i] = D.first[i];
    tab[ni + i] = D.n_events[i];
    tab[2 * ni + i] = D.cpp[i];
    tab[3 * ni + i] = D.rng[i];
    // crystals per readout unit (a crystal is its own unit at crystal level)
    tab[4 * ni + i] = D.readout == GPET_READOUT_MODULE ? std::max(1u, D.cpm[i])
                      : D.readout == GPET_READOUT_PANEL ? std::max(1u, D.cpp[i])
                                                        : 1u;
    tab[5 * ni + i] = D.dead_level == GPET_READOUT_MODULE ? std::max(1u, D.cpm[i])
                      : D.dead_level == GPET_READOUT_PANEL ? std::max(1u, D.cpp[i])
                                                           : 1u;
    tab[6 * ni + i] = std::max(1u, D.cpm[i]);
    const bool have_layers = D.layers.size() >= (i + 1) * kLayerWords;
    for (int k = 0; k < kLayerWords; ++k) // without a layout: one layer of 1 x 1 (no neighbours)
      tab[(7 + k) * ni + i] = have_layers ? D.layers[i * kLayerWords + k] : (k == 0 || k > kMaxLayers ? 1u : 0u);
    tab[(7 + kLayerWords) * ni + i] = D.ncr[i];
  }
  // (the upload is skipped when this scratch already holds the same table)
  const size_t tab_words = ni * kTabRows;
  const bool same_tab = !scr.fixed && scr.tab_at == (const void *)d_tab && scr.tab_last.size() == tab_words &&
                        std::equal(tab, tab + tab_words, scr.tab_last.begin());
  if (!same_tab) {
    (void)hipMemcpyAsync(d_tab, tab, tab_words * 4, hipMemcpyHostToDevice, st);
    if (!scr.fixed) {
      scr.tab_at = d_tab;
      scr.tab_last.assign(tab, tab + tab_words);
    }
  }
  const InstTab IT{d_tab, d_tab + ni, d_tab + 2 * ni, d_tab + 3 * ni, d_tab + (7 + kLayerWords) * ni, (uint32_t)ni};
  // per-crystal tallies are kept for one scanner (the plain entry point)
  const uint32_t n_tally = D.ncr[0];
  uint32_t max_events = 1;
  for (size_t i = 0; i < ni; ++i) max_events = std::max(max_events, D.n_events[i]);
  int event_bits = 1;
  while (event_bits < 32 && ((uint64_t)(max_events - 1) >> event_bits) != 0) ++event_bits;
  const int hit_shift = D.gid_bits + 8; // local value of a hit key: the event index
  const int inst_bits = ni > 1 ? log2_ceil(ni) : 0;
  const int inst_shift = ni > 1 ? event_bits + hit_shift : 64;
  if (event_bits + hit_shift + inst_bits > 64) {
    err = "digitize: instance, event and crystal ids do not fit a 64-bit sort key";
    return GPET_ERR_ARG;
  }

  // 1. sort hits by (instance, event, gid, photon, index).  With one instance
  //    the bucket count and scatter build the keys from the hits themselves;
  //    the key array (k0, v0) is written only when a full radix sort needs it.
  uint32_t *err_flag = rb + 13; // checked at the next synchronization
  const HitSrc HS{D.h_event, D.h_gid, D.h_aux, D.h_inst, IT, D.gid_bits, inst_shift, err_flag,
                  ni == 1, ni == 1 ? D.first[0] : 0u, ni == 1 ? D.n_events[0] : 0u, ni == 1 ? D.ncr[0] : 0u};
  bool keys_built = false;
  auto build_keys = [&]() {
    if (!keys_built)
      hipLaunchKernelGGL(k_hit_keys, dim3(grid_for(n)), dim3(256), 0, st, n, HS, sb.k0, sb.v0);
    keys_built = true;
  };
  // the bucket overflow and id-range flags (rb[12], rb[13]) start at zero: with
  // one instance the bucket sort's first launch clears them, else this one
  if (ni > 1) {
    launch_fill_u32(rb + 12, 0u, 2, st);
    build_keys();
  }
  std::vector<uint64_t> items(ni, n);
  if (ni > 1) { // per-instance counts size the bucket map
    launch_fill_u32(d_icount, 0u, ni, st);
    hipLaunchKernelGGL(k_inst_count, dim3(inst_grid(n)), dim3(256), 0, st, sb.k0, n, inst_shift, (uint32_t)ni,
                       d_icount);
    (void)hipMemcpyAsync(rb_count, d_icount, ni * 4, hipMemcpyDefault, st);
    if (!sync("building hit keys")) return GPET_ERR_HIP;
  }
  std::vector<double> range(ni);
  for (size_t i = 0; i < ni; ++i) {
    if (ni > 1) items[i] = rbh_count[i];
    range[i] = (double)D.n_events[i];
  }
  const unsigned long long ev_mask = (1ull << event_bits) - 1;
  const int hit_bits = hit_shift + event_bits + inst_bits;
  const unsigned long long *hk = sb.k1;
  const uint32_t *hp = sb.v1;
  const unsigned long long *bk = nullptr;
  const uint32_t *bv = nullptr;
  // 2. adder: single index of each run = exclusive scan of run heads (the
  //    bucket sort marks them as it writes each bucket: an event's hits share a
  //    bucket, so no run crosses one)
  bool heads_done = false;
  auto run_heads = [&]() {
    if (!heads_done) hipLaunchKernelGGL(k_heads, dim3(grid_for(n)), dim3(256), 0, st, n, hk, flag);
    heads_done = false;
    exclusive_scan(flag, n, sb.scan_tmp, st, rb + 1);
  };
  const bool mapped = bucket_sort<true>(sb, bb, n, n, inst_shift, hit_shift, ev_mask, items, range, st,
                                        sb.scan_tmp, bk, bv, keys_built ? nullptr : &HS,
                                        keys_built ? nullptr : rb + 12, 2, flag, 8) == 0;
  heads_done = mapped;
  if (mapped) {
    hk = bk;
    hp = bv;
  } else { // too many buckets for the scratch: sort every key bit instead
    if (!keys_built) launch_fill_u32(rb + 12, 0u, 2, st);
    build_keys();
    const bool f1 = radix_sort(sb, n, hit_bits, st);
    hk = f1 ? sb.k1 : sb.k0;
    hp = f1 ? sb.v1 : sb.v0;
  }
  run_heads();
  // Without tallies, dead time or a module / panel readout nothing before the
  // energy window needs the singles count on the host: the adder (with the
  // blur) runs over every hit position, the window flags are scanned over n
  // positions (the adder zeroes those beyond the singles), and the checks of
  // the hit sort wait for the synchronization after the window.
  const bool any_tally = T && (T->hits_per_crystal || T->doi || T->singles_per_crystal || T->energy_spectrum);
  const bool defer = !any_tally && D.readout == GPET_READOUT_CRYSTAL && D.dead_mode == GPET_DEAD_NONE;
  const char *range_msg = "digitize: a hit's instance, event or crystal id lies outside its declared range";
  const char *cap_msg = "digitize: singles capacity too small (it must hold the crystal-level singles)";
  uint64_t ns = 0;
  if (!defer) {
    if (!sync("after the hit sort")) return GPET_ERR_HIP;
    if (rbh[13] & 2u) {
      err = range_msg;
      return GPET_ERR_ARG;
    }
    // hit tallies once every id is known to be in range
    if (T && (T->hits_per_crystal || T->doi))
      hipLaunchKernelGGL(k_hit_tallies, dim3(grid_for(n)), dim3(256), 0, st, n, D.h_gid, D.h_depth,
                         T->hits_per_crystal, n_tally, T->doi, T->doi_bins, D.panel_depth);
    if (mapped && rbh[12]) { // a bucket overflowed LDS: sort every key bit and redo the heads
      build_keys();
      const bool f1 = radix_sort(sb, n, hit_bits, st);
      hk = f1 ? sb.k1 : sb.k0;
      hp = f1 ? sb.v1 : sb.v0;
      run_heads();
      if (!sync("after the hit sort")) return GPET_ERR_HIP;
    }
    ns = rbh[1];
    S->count = ns;
    S->windowed = 0;
    if (ns > S->capacity) { // the crystal singles pass through the output arrays
      err = cap_msg;
      return GPET_ERR_CAPACITY;
    }
  }
  // 3. blur + window (fused into the adder at crystal readout); per-block
  //    maxima of the time stamps go to the radix histogram (n / 4 bytes, free
  //    here; the keys must stay intact for a fallback sort), and one block
  //    reduces them.  With dead time the tallies wait until the
  //    losses are known.
  const bool dead = D.dead_mode != GPET_DEAD_NONE && ns > 0;
  const bool fuse_blur = D.readout == GPET_READOUT_CRYSTAL;
  unsigned long long *s_time = (unsigned long long *)S->time_ps;
  BlurArgs BA{D.k0, D.k1, D.fwhm_511, D.e_lo, D.e_hi,
              (T && !dead) ? T->singles_per_crystal : nullptr, (T && !dead) ? T->energy_spectrum : nullptr,
              n_tally, D.time_sigma, D.doi_sigma, D.ls_thresh, d_tab + 6 * ni, S->energy_kev, S->in_window,
              wpos, (unsigned long long *)sb.hist}; // the radix histogram is free until the time sort
  auto launch_adder = [&]() {
    if (fuse_blur)
      hipLaunchKernelGGL(k_adder<true>, dim3(adder_grid(n)), dim3(256), 0, st, n, hk, hp, flag, D.h_edep, D.h_depth,
                         D.h_time, IT, D.gid_bits, ev_mask, inst_shift, S->event, S->gid, S->edep_kev, S->depth_mm,
                         s_time, s_inst, S->instance, S->capacity, BA);
    else
      hipLaunchKernelGGL(k_adder<false>, dim3(adder_grid(n)), dim3(256), 0, st, n, hk, hp, flag, D.h_edep, D.h_depth,
                         D.h_time, IT, D.gid_bits, ev_mask, inst_shift, S->event, S->gid, S->edep_kev, S->depth_mm,
                         s_time, s_inst, S->instance, S->capacity, BA);
  };
  launch_adder();
  // 2b. module / panel readout: runs of (instance, event, unit) merge into the
  //     free sort buffers, then back into the output arrays
  if (D.readout != GPET_READOUT_CRYSTAL) {
    const uint32_t *unit = d_tab + 4 * ni;
    uint32_t *o_ev = sb.v0, *o_gid = sb.v1, *o_inst = wpos;
    float *o_edep = (float *)sb.k1, *o_depth = (float *)sb.k1 + n;
    unsigned long long *o_time = sb.k0;
    hipLaunchKernelGGL(k_readout_heads, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, S->event, S->gid, s_inst,
                       unit, flag);
    exclusive_scan(flag, ns, sb.scan_tmp, st, rb + 1);
    hipLaunchKernelGGL(k_readout_merge, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, flag, S->event, S->gid,
                       s_inst, unit, S->edep_kev, S->depth_mm, (const unsigned long long *)S->time_ps, o_ev, o_gid,
                       o_edep, o_depth, o_time, o_inst);
    if (!sync("in the readout")) return GPET_ERR_HIP;
    ns = rbh[1];
    S->count = ns;
    hipLaunchKernelGGL(k_readout_copy, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, o_ev, o_gid, o_edep,
                       o_depth, o_time, o_inst, S->event, S->gid, S->edep_kev, S->depth_mm,
                       (unsigned long long *)S->time_ps, s_inst, S->instance);
  }
  if (!fuse_blur)
    hipLaunchKernelGGL(k_blur, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, S->event, S->gid, s_inst, IT,
                       S->edep_kev, s_time, S->depth_mm, BA);
  auto reduce_max = [&]() {
    hipLaunchKernelGGL(k_max_u64, dim3(1), dim3(1024), 0, st, (const unsigned long long *)BA.block_max,
                       (size_t)(fuse_blur ? adder_grid(n) : grid_for(ns)), (unsigned long long *)(rb + 4));
  };
  reduce_max();
  if (dead) {
    // 3b. dead time per unit (free here: the key/value pairs, flag, wpos)
    if (!sync("after the blur")) return GPET_ERR_HIP;
    const unsigned long long tm = (unsigned long long)rbh[4] | ((unsigned long long)rbh[5] << 32);
    int tbits = 1;
    while (tbits < 64 && (tm >> tbits) != 0) ++tbits;
    hipLaunchKernelGGL(k_dead_time_keys, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns,
                       (const unsigned long long *)s_time, sb.k0, sb.v0);
    const bool f1 = radix_sort(sb, ns, tbits, st);
    const int unit_bits = D.gid_bits;
    hipLaunchKernelGGL(k_dead_unit_keys, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, f1 ? sb.v1 : sb.v0,
                       S->gid, ni > 1 ? s_inst : nullptr, d_tab + 5 * ni, unit_bits, sb.k0, sb.v0);
    const bool f2 = radix_sort(sb, ns, unit_bits + inst_bits, st);
    const unsigned long long *uk = f2 ? sb.k1 : sb.k0;
    const uint32_t *uv = f2 ? sb.v1 : sb.v0;
    uint32_t *lost = flag;
    if (D.dead_mode == GPET_DEAD_PARALYZABLE) {
      hipLaunchKernelGGL(k_dead_paralyzable, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, uk, uv,
                         (const unsigned long long *)s_time, D.dead_ps, lost);
    } else {
      uint32_t *start = f2 ? sb.v0 : sb.v1;               // the free value array
      unsigned long long *t_sorted = f2 ? sb.k0 : sb.k1;  // and the free key array
      hipLaunchKernelGGL(k_dead_heads, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, uk, wpos);
      exclusive_scan(wpos, ns, sb.scan_tmp, st, rb + 6);
      hipLaunchKernelGGL(k_dead_starts, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, uk, wpos, start);
      hipLaunchKernelGGL(k_dead_gather, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, uv,
                         (const unsigned long long *)s_time, t_sorted);
      if (!sync("in the dead time")) return GPET_ERR_HIP;
      const uint32_t n_runs = rbh[6];
      hipLaunchKernelGGL(k_dead_nonparalyzable, dim3((n_runs + 3) / 4), dim3(256), 0, st, n_runs, start,
                         (size_t)ns, uv, (const unsigned long long *)t_sorted, D.dead_ps, lost);
    }
    hipLaunchKernelGGL(k_dead_apply, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, lost, S->in_window, wpos,
                       S->gid, S->energy_kev, T ? T->singles_per_crystal : nullptr, n_tally,
                       T ? T->energy_spectrum : nullptr);
  }
  exclusive_scan(wpos, defer ? n : ns, sb.scan_tmp, st, rb + 3);
  if (!sync("after the energy window")) return GPET_ERR_HIP;
  if (defer) { // the checks of the hit sort
    if (rbh[13] & 2u) {
      err = range_msg;
      return GPET_ERR_ARG;
    }
    if (mapped && rbh[12]) { // a bucket overflowed LDS: sort every key bit and redo the adder
      build_keys();
      const bool f1 = radix_sort(sb, n, hit_bits, st);
      hk = f1 ? sb.k1 : sb.k0;
      hp = f1 ? sb.v1 : sb.v0;
      run_heads();
      launch_adder();
      reduce_max();
      exclusive_scan(wpos, n, sb.scan_tmp, st, rb + 3);
      if (!sync("after the energy window")) return GPET_ERR_HIP;
    }
    ns = rbh[1];
    S->count = ns;
    S->windowed = 0;
    if (ns > S->capacity) {
      err = cap_msg;
      return GPET_ERR_CAPACITY;
    }
  }
  const size_t nw = rbh[3];
  S->windowed = nw;
  const unsigned long long tmax = (unsigned long long)rbh[4] | ((unsigned long long)rbh[5] << 32);
  // time bits leave room for the window, so keys of two instances differ by more than it
  int time_bits = 0;
  while (time_bits < 63 && ((tmax + D.window_ps + 1) >> time_bits) != 0) ++time_bits;
  const size_t n_sweep = D.sweep_lo.size();
  if (D.coinc_per_inst) std::fill(D.coinc_per_inst, D.coinc_per_inst + ni, 0ull);
  if (D.sweep_out) std::fill(D.sweep_out, D.sweep_out + n_sweep * ni, (uint64_t)0);
  if (nw == 0 && n_sweep == 0) return GPET_OK;
  if (time_bits + inst_bits > 64) {
    err = "digitize: instance and time stamp do not fit a 64-bit sort key";
    return GPET_ERR_ARG;
  }
  std::vector<double> trange(ni, (double)tmax + 1.0);
  for (size_t i = 0; i < ni; ++i)
    if (D.duration.size() == ni && D.duration[i]) trange[i] = (double)D.duration[i] + 1048576.0;
  const int tb = ni > 1 ? time_bits : 64;
  const unsigned long long t_mask = time_bits < 64 ? (1ull << time_bits) - 1 : ~0ull;

  // 4-5. The singles of a window (wpos: the exclusive scan of its flags,
  // nwin of them) in (instance, time, index) order, split into clusters and
  // paired.  list: write the coincidence list (count in rb[7]); otherwise
  // count the coincidences per instance into rb_count.  make_flags() rebuilds
  // wpos if the pairing overwrote it (flag doubles as the window's flags and
  // the pair counts).
  auto pair_window = [&](size_t nwin, bool list, auto &&make_flags) -> int {
    hipLaunchKernelGGL(k_time_keys, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, (const uint32_t *)wpos,
                       (uint32_t)nwin, (const unsigned long long *)S->time_ps, s_inst, tb, sb.k0, sb.v0);
    std::vector<uint64_t> witems(ni, nwin);
    if (ni > 1) {
      launch_fill_u32(d_icount, 0u, ni, st);
      hipLaunchKernelGGL(k_inst_count, dim3(inst_grid(nwin)), dim3(256), 0, st, sb.k0, nwin, time_bits,
                         (uint32_t)ni, d_icount);
      (void)hipMemcpyAsync(rb_count, d_icount, ni * 4, hipMemcpyDefault, st);
      if (!sync("counting windowed singles")) return GPET_ERR_HIP;
      for (size_t i = 0; i < ni; ++i) witems[i] = rbh_count[i];
    }
    const unsigned long long *tk = sb.k1;
    const uint32_t *ti = sb.v1;
    auto count_pairs = [&]() {
      const uint32_t *c_inst = ni > 1 ? s_inst : nullptr;
      hipLaunchKernelGGL(k_coinc_count, dim3(grid_for(nwin)), dim3(256), 0, st, nwin, tk, ti, S->gid, c_inst, IT.cpp,
                         D.window_ps, flag);
      if (list) {
        exclusive_scan(flag, nwin, sb.scan_tmp, st, rb + 7);
        hipLaunchKernelGGL(k_coinc_write, dim3(grid_for(nwin)), dim3(256), 0, st, nwin, tk, ti, S->gid, c_inst,
                           IT.cpp, D.window_ps, flag, C->first, C->second, C->capacity);
      } else {
        launch_fill_u32(d_icount, 0u, ni, st);
        hipLaunchKernelGGL(k_coinc_inst_counts, dim3(inst_grid(nwin)), dim3(256), 0, st, nwin, flag, tk, tb,
                           (uint32_t)ni, d_icount);
        (void)hipMemcpyAsync(rb_count, d_icount, ni * 4, hipMemcpyDefault, st);
      }
    };
    bool mapped_t = false; // (the bucket sort clears the overflow flag rb[12] it may set)
    if (nwin == 1) {
      tk = sb.k0;
      ti = sb.v0;
    } else if (bucket_sort<false>(sb, bb, nwin, ns, tb, 0, t_mask, witems, trange, st, sb.scan_tmp, bk, bv, nullptr,
                                  rb + 12, 1) == 0) {
      mapped_t = true;
      tk = bk;
      ti = bv;
    } else {
      const bool f2 = radix_sort(sb, nwin, time_bits + inst_bits, st);
      tk = f2 ? sb.k1 : sb.k0;
      ti = f2 ? sb.v1 : sb.v0;
    }
    count_pairs();
    if (!sync("in coincidence sorting")) return GPET_ERR_HIP;
    if (mapped_t && rbh[12]) { // a bucket overflowed LDS: rebuild the keys, sort every bit, redo the pairing
      make_flags();
      hipLaunchKernelGGL(k_time_keys, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, (const uint32_t *)wpos,
                         (uint32_t)nwin, (const unsigned long long *)S->time_ps, s_inst, tb, sb.k0, sb.v0);
      const bool f2 = radix_sort(sb, nwin, time_bits + inst_bits, st);
      tk = f2 ? sb.k1 : sb.k0;
      ti = f2 ? sb.v1 : sb.v0;
      count_pairs();
      if (!sync("in coincidence sorting")) return GPET_ERR_HIP;
    }
    return GPET_OK;
  };

  // the main window: the coincidence list
  if (nw > 0) {
    const int r = pair_window(nw, true, [] {});
    if (r != GPET_OK) return r;
    C->count = rbh[7];
    if (C->count > C->capacity) {
      err = "digitize: coincidence capacity too small";
      return GPET_ERR_CAPACITY;
    }
    if (D.coinc_per_inst) {
      if (ni == 1) {
        D.coinc_per_inst[0] = C->count;
      } else {
        launch_fill_u32(d_icount, 0u, ni, st);
        if (C->count)
          hipLaunchKernelGGL(k_coinc_inst, dim3(inst_grid(C->count)), dim3(256), 0, st, (size_t)C->count,
                             C->first, s_inst, (uint32_t)ni, d_icount);
        (void)hipMemcpyAsync(rb_count, d_icount, ni * 4, hipMemcpyDefault, st);
        if (!sync("counting coincidences per instance")) return GPET_ERR_HIP;
        for (size_t i = 0; i < ni; ++i) D.coinc_per_inst[i] = rbh_count[i];
      }
    }
  }
  // the sweep windows on the same blurred energies: counts only
  for (size_t w = 0; w < n_sweep; ++w) {
    auto make_flags = [&]() {
      hipLaunchKernelGGL(k_window_flags, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, S->energy_kev,
                         S->in_window, D.sweep_lo[w], D.sweep_hi[w], flag, wpos);
      exclusive_scan(wpos, ns, sb.scan_tmp, st, rb + 3);
    };
    make_flags();
    if (!sync("in the window sweep")) return GPET_ERR_HIP;
    const size_t nsw = rbh[3];
    if (nsw == 0) continue;
    const int r = pair_window(nsw, false, make_flags);
    if (r != GPET_OK) return r;
    for (size_t i = 0; i < ni; ++i) D.sweep_out[w * ni + i] = rbh_count[i];
  }
  return GPET_OK;
}

hipError_t wait_stream(hipStream_t st) {
  for (;;) {
    const hipError_t e = hipStreamQuery(st);
    if (e != hipErrorNotReady) return e;
    __builtin_ia32_pause();
  }
}

size_t scan_tmp_words(size_t n) { return scan_scratch_words(n); }
void scan_exclusive_u32(uint32_t *a, size_t n, uint32_t *tmp, hipStream_t st, uint32_t *total) {
  exclusive_scan(a, n, tmp, st, total);
}

// The scratch of gpet_digitize_noalloc: one copy per GPU, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host the name is a stand-in, not a device address); it passes the address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

void *fixed_scratch(int device, std::string &err) {
  static std::mutex mu;
  static std::vector<void *> addr; // per device
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) {
    err = "fixed scratch: bad device";
    return nullptr;
  }
  if ((size_t)device >= addr.size()) addr.resize(device + 1, nullptr);
  if (!addr[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      err = std::string("fixed scratch: hipGetSymbolAddress failed: ") + hipGetErrorString(e);
      return nullptr;
    }
    addr[device] = ptr;
  }
  return addr[device];
}

void free_scratch(DigitizeScratch &scr) {
  if (scr.pinned) (void)hipHostFree(scr.pinned);
  scr.pinned = nullptr;
  scr.pinned_bytes = 0;
  if (scr.buf) (void)hipFree(scr.buf);
  scr.buf = nullptr;
  scr.bytes = 0;
  scr.tab_at = nullptr;
  scr.tab_last.clear();
}

} // namespace gpet
