// digitize.hip -- crystal-level digitizer for gfx950.
//
// Pipeline (all on the device, stream ordered):
//   1. hits -> 64-bit keys (event - first) << gid_bits | gid, stable LSD radix
//      sort (8-bit digits, ranks from wave ballots so equal digits keep their
//      order);
//   2. adder: one single per run of equal keys; energy and energy-weighted
//      depth are summed as exact 2^-32 fixed-point integers, so the result does
//      not depend on the (atomic) order the hits were appended in;
//   3. Gaussian blur from the digitizer Philox stream and the energy window;
//   4. windowed singles sorted by time (stable, so ties stay in (event, gid)
//      order), split into clusters at gaps larger than the coincidence window;
//      inside a cluster, non-retriggering windows are resolved sequentially by
//      the cluster's first lane; counts are scanned so that the coincidence
//      list comes out in a fixed order.
#include <algorithm>

#include "gpet_internal.hpp"

namespace gpet {

constexpr int kSortBlock = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

// ---------------------------------------------------------------------------
// exclusive scan of u32 (in place); block totals scanned recursively
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kScanBlock) k_scan_tiles(uint32_t *a, size_t n, uint32_t *tile_sums) {
  __shared__ uint32_t s[kScanBlock];
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems], run = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? a[base + k] : 0u;
    const uint32_t t = v[k];
    v[k] = run;
    run += t;
  }
  s[threadIdx.x] = run;
  __syncthreads();
  for (int o = 1; o < kScanBlock; o <<= 1) {
    const uint32_t t = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  const uint32_t excl = s[threadIdx.x] - run;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) a[base + k] = v[k] + excl;
  if (threadIdx.x == kScanBlock - 1 && tile_sums) tile_sums[blockIdx.x] = s[kScanBlock - 1];
}

__global__ void k_scan_add(uint32_t *a, size_t n, const uint32_t *tile_offs) {
  const size_t i = (size_t)blockIdx.x * kScanTile + threadIdx.x;
  const uint32_t off = tile_offs[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (i + (size_t)k * kScanBlock < n) a[i + (size_t)k * kScanBlock] += off;
}

static size_t scan_scratch_words(size_t n) {
  size_t w = 0;
  while (n > (size_t)kScanTile) {
    n = (n + kScanTile - 1) / kScanTile;
    w += n;
  }
  return w + 1;
}

static void exclusive_scan(uint32_t *a, size_t n, uint32_t *tmp, hipStream_t st) {
  if (n == 0) return;
  const size_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanBlock), 0, st, a, n, (uint32_t *)nullptr);
    return;
  }
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kScanBlock), 0, st, a, n, tmp);
  exclusive_scan(tmp, tiles, tmp + tiles, st);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kScanBlock), 0, st, a, n, tmp);
}

// ---------------------------------------------------------------------------
// LSD radix sort of (u64 key, u32 value), 8-bit digits
// ---------------------------------------------------------------------------
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

__global__ void __launch_bounds__(kSortBlock) k_radix_hist(const unsigned long long *keys, size_t n, int shift,
                                                           uint32_t *hist, uint32_t n_tiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t below = __lanemask_lt();
  const size_t base = (size_t)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    const size_t i = base + (size_t)it * kSortBlock + threadIdx.x;
    const bool valid = i < n;
    const uint32_t dg = valid ? (uint32_t)(keys[i] >> shift) & 255u : 0u;
    const uint64_t peers = digit_peers(dg, valid);
    if (valid && (peers & below) == 0) atomicAdd(&h[dg], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kSortBlock) k_radix_scatter(const unsigned long long *kin, const uint32_t *vin,
                                                              unsigned long long *kout, uint32_t *vout, size_t n,
                                                              int shift, const uint32_t *offs, uint32_t n_tiles) {
  constexpr int kWaves = kSortBlock / 64;
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_cnt[kWaves][256];
  const int wave = threadIdx.x >> 6;
  const uint64_t below = __lanemask_lt();
  s_base[threadIdx.x] = offs[(size_t)threadIdx.x * n_tiles + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s_cnt[w][threadIdx.x] = 0;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * kSortTile;
  for (int it = 0; it < kSortItems; ++it) {
    const size_t i = base + (size_t)it * kSortBlock + threadIdx.x;
    const bool valid = i < n;
    const unsigned long long key = valid ? kin[i] : 0ull;
    const uint32_t val = valid ? vin[i] : 0u;
    const uint32_t dg = (uint32_t)(key >> shift) & 255u;
    const uint64_t peers = digit_peers(dg, valid);
    const uint32_t rank = (uint32_t)__popcll(peers & below);
    if (valid && rank == 0) s_cnt[wave][dg] = (uint32_t)__popcll(peers);
    __syncthreads();
    uint32_t pos = 0;
    if (valid) {
      pos = s_base[dg] + rank;
      for (int w = 0; w < wave; ++w) pos += s_cnt[w][dg];
    }
    __syncthreads();
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      tot += s_cnt[w][threadIdx.x];
      s_cnt[w][threadIdx.x] = 0;
    }
    s_base[threadIdx.x] += tot;
    __syncthreads();
    if (valid && pos < n) {
      kout[pos] = key;
      vout[pos] = val;
    }
  }
}

struct SortBufs {
  unsigned long long *k0, *k1;
  uint32_t *v0, *v1;
  uint32_t *hist;    // 256 * tiles
  uint32_t *scan_tmp;
};

// sorts (k0, v0) over the low `bits` bits; returns true if the result sits in (k1, v1)
static bool radix_sort(SortBufs &b, size_t n, int bits, hipStream_t st) {
  if (n <= 1 || bits <= 0) return false;
  const uint32_t tiles = (uint32_t)((n + kSortTile - 1) / kSortTile);
  bool flip = false;
  for (int shift = 0; shift < bits; shift += 8) {
    unsigned long long *ki = flip ? b.k1 : b.k0, *ko = flip ? b.k0 : b.k1;
    uint32_t *vi = flip ? b.v1 : b.v0, *vo = flip ? b.v0 : b.v1;
    hipLaunchKernelGGL(k_radix_hist, dim3(tiles), dim3(kSortBlock), 0, st, ki, n, shift, b.hist, tiles);
    exclusive_scan(b.hist, (size_t)256 * tiles, b.scan_tmp, st);
    hipLaunchKernelGGL(k_radix_scatter, dim3(tiles), dim3(kSortBlock), 0, st, ki, vi, ko, vo, n, shift, b.hist,
                       tiles);
    flip = !flip;
  }
  return flip;
}

// ---------------------------------------------------------------------------
// Bucket sort of (u64 key, u32 value) for keys spread evenly over their range
// (event ids, event times): count per bucket (key >> shift), scan, scatter by
// bucket, then sort each bucket (about 256 items) in LDS with a bitonic network
// ordered by (key, value).  The scatter order inside a bucket depends on
// atomics; the local sort by (key, value) makes the result deterministic.
// ---------------------------------------------------------------------------
constexpr int kLocalSort = 1024; // largest bucket sorted in LDS

// lanes of the wave whose value equals this lane's (one ballot per distinct value)
__device__ __forceinline__ uint64_t equal_peers(uint32_t v, bool valid) {
  uint64_t left = __ballot(valid), mine = 0;
  while (left) {
    const int leader = __ffsll((unsigned long long)left) - 1;
    const uint32_t lv = __shfl(v, leader);
    const uint64_t m = __ballot(valid && v == lv) & left;
    if (valid && v == lv) mine = m;
    left &= ~m;
  }
  return mine;
}

// keys whose bucket lies at or past nb are skipped and flagged (bit 1 of *flag)
template <bool AGG>
__global__ void k_bucket_count(const unsigned long long *key, size_t n, int shift, size_t nb, uint32_t *count,
                               uint32_t *flag) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long kb = i < n ? key[i] >> shift : 0ull;
  if (i < n && kb >= nb) atomicOr(flag, 2u);
  const bool valid = i < n && kb < nb;
  const uint32_t b = valid ? (uint32_t)kb : 0u;
  if constexpr (AGG) {
    const uint64_t peers = equal_peers(b, valid);
    if (valid && (peers & __lanemask_lt()) == 0) atomicAdd(&count[b], (uint32_t)__popcll(peers));
  } else {
    if (valid) atomicAdd(&count[b], 1u);
  }
}

// cursor holds bucket starts on entry and bucket ends on exit
template <bool AGG>
__global__ void k_bucket_scatter(const unsigned long long *kin, const uint32_t *vin, size_t n, int shift, size_t nb,
                                 uint32_t *cursor, unsigned long long *kout, uint32_t *vout) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned long long k = i < n ? kin[i] : 0ull;
  const bool valid = i < n && (k >> shift) < nb;
  const uint32_t b = valid ? (uint32_t)(k >> shift) : 0u;
  uint32_t pos = 0;
  if constexpr (AGG) {
    const uint64_t below = __lanemask_lt();
    const uint64_t peers = equal_peers(b, valid);
    const int leader = valid ? __ffsll((unsigned long long)peers) - 1 : 0;
    uint32_t base = 0;
    if (valid && (peers & below) == 0) base = atomicAdd(&cursor[b], (uint32_t)__popcll(peers));
    base = __shfl(base, leader);
    pos = base + (uint32_t)__popcll(peers & below);
  } else {
    if (valid) pos = atomicAdd(&cursor[b], 1u);
  }
  if (valid && pos < n) {
    kout[pos] = k;
    vout[pos] = vin[i];
  }
}

__device__ __forceinline__ bool pair_less(unsigned long long ka, uint32_t va, unsigned long long kb, uint32_t vb) {
  return ka < kb || (ka == kb && va < vb);
}

// one block per bucket; `end` holds bucket ends (the scattered cursor)
__global__ void __launch_bounds__(256) k_bucket_local_sort(unsigned long long *key, uint32_t *val,
                                                           const uint32_t *end, uint32_t *overflow) {
  __shared__ unsigned long long sk[kLocalSort];
  __shared__ uint32_t sv[kLocalSort];
  const uint32_t b = blockIdx.x;
  const uint32_t lo = b ? end[b - 1] : 0u, hi = end[b];
  const uint32_t size = hi - lo;
  if (size <= 1) return;
  if (size > (uint32_t)kLocalSort) {
    if (threadIdx.x == 0) atomicOr(overflow, 1u);
    return;
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
  }
}

static int log2_ceil(uint64_t x) {
  int b = 0;
  while ((1ull << b) < x && b < 63) ++b;
  return b;
}

struct BucketBufs {
  uint32_t *count;        // bucket counters (>= max_buckets words)
  size_t max_buckets;
  uint32_t *overflow;     // device flag
  uint32_t *pinned_flag;  // host mirror
};

// Sorts (b.k0, b.v0) into (b.k1, b.v1) by (key, value) for keys <= key_max.
// Returns 0 when sorted, bit 0 when a bucket was too large for LDS, bit 1 when
// a key exceeded key_max (then (k1, v1) are not sorted).
template <bool AGG>
static uint32_t bucket_sort(SortBufs &b, BucketBufs &bb, size_t n, unsigned long long key_max, hipStream_t st,
                            uint32_t *scan_tmp) {
  const int key_bits = key_max ? 64 - __builtin_clzll(key_max) : 1;
  const int want = log2_ceil(n / 256 + 1);
  int shift = key_bits > want ? key_bits - want : 0;
  size_t nb = (size_t)(key_max >> shift) + 1;
  while (nb > bb.max_buckets) {
    ++shift;
    nb = (size_t)(key_max >> shift) + 1;
  }
  launch_fill_u32(bb.count, 0u, nb, st);
  launch_fill_u32(bb.overflow, 0u, 1, st);
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_bucket_count<AGG>, dim3(g), dim3(256), 0, st, b.k0, n, shift, nb, bb.count, bb.overflow);
  exclusive_scan(bb.count, nb, scan_tmp, st);
  hipLaunchKernelGGL(k_bucket_scatter<AGG>, dim3(g), dim3(256), 0, st, b.k0, b.v0, n, shift, nb, bb.count, b.k1,
                     b.v1);
  hipLaunchKernelGGL(k_bucket_local_sort, dim3((unsigned)nb), dim3(256), 0, st, b.k1, b.v1, bb.count, bb.overflow);
  (void)hipMemcpyAsync(bb.pinned_flag, bb.overflow, 4, hipMemcpyDeviceToHost, st);
  (void)hipStreamSynchronize(st);
  return *bb.pinned_flag;
}

// ---------------------------------------------------------------------------
// digitizer stages
// ---------------------------------------------------------------------------
// key = (event - first) | gid | photon | index of the hit within its photon
// (7 bits, saturated): unique per hit, so the sorted order is fixed
__global__ void k_hit_keys(size_t n, const uint32_t *ev, const uint32_t *gid, const uint32_t *aux, uint32_t first,
                           int gid_bits, unsigned long long *key, uint32_t *val) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t a = aux[i];
  const uint32_t low = ((a & 1u) << 7) | min(a >> 8, 127u);
  key[i] = ((((unsigned long long)(ev[i] - first) << gid_bits) | gid[i]) << 8) | low;
  val[i] = (uint32_t)i;
}

// first hit of each (event, crystal) run
__global__ void k_heads(size_t n, const unsigned long long *key, uint32_t *flag) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  flag[i] = (i == 0 || (key[i] >> 8) != (key[i - 1] >> 8)) ? 1u : 0u;
}

__global__ void k_adder(size_t n, const unsigned long long *key, const uint32_t *perm, const uint32_t *seg,
                        const uint32_t *ev, const uint32_t *gid, const float *edep, const float *depth,
                        const unsigned long long *time, uint32_t *s_ev, uint32_t *s_gid, float *s_edep,
                        float *s_depth, unsigned long long *s_time, uint64_t cap) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long run = key[i] >> 8;
  if (i > 0 && (key[i - 1] >> 8) == run) return;
  unsigned long long se = 0, sd = 0, tm = ~0ull;
  size_t j = i;
  do {
    const uint32_t h = perm[j];
    const float e = edep[h];
    se += (unsigned long long)(e * 4294967296.0f);
    sd += (unsigned long long)((e * depth[h]) * 4294967296.0f);
    tm = min(tm, time[h]);
    ++j;
  } while (j < n && (key[j] >> 8) == run);
  const uint32_t s = seg[i];
  if (s >= cap) return;
  const uint32_t h = perm[i];
  const double E = (double)se * 0x1p-32;
  s_ev[s] = ev[h];
  s_gid[s] = gid[h];
  s_edep[s] = (float)E;
  s_depth[s] = se ? (float)((double)sd / (double)se) : 0.0f;
  s_time[s] = tm;
}

__global__ void __launch_bounds__(256) k_blur(size_t n, const uint32_t *s_ev, const uint32_t *s_gid,
                                              const float *s_edep, float *s_energy, uint32_t *s_win, uint32_t *wflag,
                                              uint32_t k0, uint32_t k1, uint32_t inst, float fwhm, float e_lo,
                                              float e_hi, uint32_t *spp, uint32_t *spec,
                                              const unsigned long long *s_time, unsigned long long *block_max) {
  __shared__ unsigned long long s_max[4];
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long tm = 0; // largest time stamp among windowed singles
  if (i < n) {
    // normal deviate by Box-Muller from the digitizer stream of (gid, event)
    const uint4 w = philox(k0, k1, make_uint4(s_gid[i], s_ev[i], inst, 3u));
    const float u0 = to_unit(w.x), u1 = to_unit(w.y);
    const float g = sqrtf(-2.0f * logf(u0)) * cos_rev(u1);
    const float E = s_edep[i];
    const float sig = fwhm * sqrtf(511.0f * E) * (1.0f / 2.354820045f);
    const float Eb = E + sig * g;
    const uint32_t in = (Eb >= e_lo && Eb <= e_hi) ? 1u : 0u;
    s_energy[i] = Eb;
    s_win[i] = in;
    wflag[i] = in;
    if (spp && in) atomicAdd(&spp[s_gid[i]], 1u);
    if (spec && Eb >= 0.0f && Eb < 700.0f) atomicAdd(&spec[(int)Eb], 1u);
    if (in) tm = s_time[i];
  }
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
    block_max[blockIdx.x] = b;
  }
}

__global__ void __launch_bounds__(1024) k_max_u64(const unsigned long long *v, size_t n, unsigned long long *out) {
  __shared__ unsigned long long s[1024];
  unsigned long long m = 0;
  for (size_t i = threadIdx.x; i < n; i += 1024) m = v[i] > m ? v[i] : m;
  s[threadIdx.x] = m;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = s[threadIdx.x + o] > s[threadIdx.x] ? s[threadIdx.x + o] : s[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

__global__ void k_time_keys(size_t n, const uint32_t *win, const uint32_t *pos, const unsigned long long *s_time,
                            unsigned long long *key, uint32_t *val) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !win[i] || pos[i] >= n) return;
  key[pos[i]] = s_time[i];
  val[pos[i]] = (uint32_t)i;
}

// coincidences of the cluster starting at sorted position k (k must be a head)
template <bool WRITE>
__device__ __forceinline__ uint32_t resolve_cluster(size_t k, size_t n, const unsigned long long *t,
                                                    const uint32_t *idx, const uint32_t *s_gid, uint32_t cpp,
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
                              uint32_t cpp, unsigned long long W, uint32_t *cnt) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const bool head = k == 0 || t[k] - t[k - 1] > W;
  cnt[k] = head ? resolve_cluster<false>(k, n, t, idx, s_gid, cpp, W, nullptr, nullptr, 0, 0) : 0u;
}

__global__ void k_coinc_write(size_t n, const unsigned long long *t, const uint32_t *idx, const uint32_t *s_gid,
                              uint32_t cpp, unsigned long long W, const uint32_t *off, uint32_t *first,
                              uint32_t *second, uint64_t cap) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const bool head = k == 0 || t[k] - t[k - 1] > W;
  if (head) resolve_cluster<true>(k, n, t, idx, s_gid, cpp, W, first, second, off[k], cap);
}

__global__ void k_hit_tallies(size_t n, const uint32_t *gid, const float *depth, uint32_t *hpc, uint32_t *doi,
                              int doi_bins, float panel_depth) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (hpc) atomicAdd(&hpc[gid[i]], 1u);
  if (doi) {
    int b = (int)floorf(depth[i] / panel_depth * (float)doi_bins);
    b = b < 0 ? 0 : (b >= doi_bins ? doi_bins - 1 : b);
    atomicAdd(&doi[b], 1u);
  }
}

static inline unsigned grid_for(size_t n) { return (unsigned)((n + 255) / 256); }

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int run_digitize(DigitizeArgs &D, DigitizeScratch &scr, hipStream_t st, std::string &err) {
  const size_t n = D.n_hits;
  gpet_singles *S = D.singles;
  gpet_coincidences *C = D.coinc;
  const gpet_tallies *T = D.tallies;
  S->count = 0;
  C->count = 0;
  if (T && (T->hits_per_crystal || T->doi) && n)
    hipLaunchKernelGGL(k_hit_tallies, dim3(grid_for(n)), dim3(256), 0, st, n, D.h_gid, D.h_depth,
                       T->hits_per_crystal, T->doi, T->doi_bins, D.panel_depth);
  if (n == 0) return hipStreamSynchronize(st) == hipSuccess ? GPET_OK : GPET_ERR_HIP;

  // scratch: 2 key + 2 value arrays, 2 flag arrays, radix histogram, scan temp, time maximum
  const size_t tiles = (n + kSortTile - 1) / kSortTile;
  const size_t max_buckets = n / 128 + 1024;
  const size_t scan_words = scan_scratch_words(std::max<size_t>(std::max<size_t>(256 * tiles, n), max_buckets));
  const size_t need = align_up(n * 8) * 2 + align_up(n * 4) * 4 + align_up(256 * tiles * 4) +
                      align_up(scan_words * 4) + align_up(max_buckets * 4) + 512;
  if (scr.bytes < need) {
    if (scr.buf) (void)hipFree(scr.buf);
    scr.buf = nullptr;
    scr.bytes = 0;
    if (hipMalloc(&scr.buf, need) != hipSuccess) {
      err = "digitize: device scratch allocation failed";
      return GPET_ERR_HIP;
    }
    scr.bytes = need;
  }
  if (!scr.pinned && hipHostMalloc((void **)&scr.pinned, 64, hipHostMallocDefault) != hipSuccess) {
    err = "digitize: pinned readback allocation failed";
    return GPET_ERR_HIP;
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
  sb.hist = (uint32_t *)take(256 * tiles * 4);
  sb.scan_tmp = (uint32_t *)take(scan_words * 4);
  unsigned long long *tmax_dev = (unsigned long long *)take(8);
  BucketBufs bb;
  bb.count = (uint32_t *)take(max_buckets * 4);
  bb.max_buckets = max_buckets;
  bb.overflow = (uint32_t *)take(8);
  uint32_t *rb = (uint32_t *)scr.pinned; // pinned readback words
  bb.pinned_flag = rb + 12;
  auto sync = [&](const char *what) {
    if (hipStreamSynchronize(st) != hipSuccess) {
      err = std::string("digitize: stream error ") + what;
      return false;
    }
    return true;
  };

  // 1. sort hits by (event, gid)
  hipLaunchKernelGGL(k_hit_keys, dim3(grid_for(n)), dim3(256), 0, st, n, D.h_event, D.h_gid, D.h_aux,
                     D.first_event, D.gid_bits, sb.k0, sb.v0);
  const int hit_bits = D.event_bits + D.gid_bits + 8;
  const unsigned long long hit_max =
      ((unsigned long long)(D.n_events - 1) << (D.gid_bits + 8)) | ((1ull << (D.gid_bits + 8)) - 1);
  const unsigned long long *hk = sb.k1;
  const uint32_t *hp = sb.v1;
  const uint32_t hflag = bucket_sort<true>(sb, bb, n, hit_max, st, sb.scan_tmp);
  if (hflag & 2u) {
    err = "digitize: a hit's event id lies outside [first_event, first_event + n_events)";
    return GPET_ERR_ARG;
  }
  if (hflag) { // a bucket overflowed LDS
    const bool f1 = radix_sort(sb, n, hit_bits, st);
    hk = f1 ? sb.k1 : sb.k0;
    hp = f1 ? sb.v1 : sb.v0;
  }
  // 2. adder: single index of each run = exclusive scan of run heads
  hipLaunchKernelGGL(k_heads, dim3(grid_for(n)), dim3(256), 0, st, n, hk, flag);
  (void)hipMemcpyAsync(rb + 0, flag + n - 1, 4, hipMemcpyDeviceToHost, st);
  exclusive_scan(flag, n, sb.scan_tmp, st);
  (void)hipMemcpyAsync(rb + 1, flag + n - 1, 4, hipMemcpyDeviceToHost, st);
  if (!sync("after the hit sort")) return GPET_ERR_HIP;
  const uint64_t ns = (uint64_t)rb[1] + rb[0];
  S->count = ns;
  if (ns > S->capacity) {
    err = "digitize: singles capacity too small";
    return GPET_ERR_CAPACITY;
  }
  hipLaunchKernelGGL(k_adder, dim3(grid_for(n)), dim3(256), 0, st, n, hk, hp, flag, D.h_event, D.h_gid, D.h_edep,
                     D.h_depth, D.h_time, S->event, S->gid, S->edep_kev, S->depth_mm, (unsigned long long *)S->time_ps, S->capacity);
  // 3. blur + window; per-block maxima of the windowed time stamps go to the
  //    (now free) second key array, then one block reduces them
  hipLaunchKernelGGL(k_blur, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, S->event, S->gid, S->edep_kev,
                     S->energy_kev, S->in_window, wpos, D.k0, D.k1, D.instance, D.fwhm_511, D.e_lo, D.e_hi,
                     T ? T->singles_per_crystal : nullptr, T ? T->energy_spectrum : nullptr,
                     (const unsigned long long *)S->time_ps, sb.k1);
  hipLaunchKernelGGL(k_max_u64, dim3(1), dim3(1024), 0, st, (const unsigned long long *)sb.k1,
                     (size_t)grid_for(ns), tmax_dev);
  (void)hipMemcpyAsync(rb + 2, wpos + ns - 1, 4, hipMemcpyDeviceToHost, st);
  exclusive_scan(wpos, ns, sb.scan_tmp, st);
  (void)hipMemcpyAsync(rb + 3, wpos + ns - 1, 4, hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(rb + 4, tmax_dev, 8, hipMemcpyDeviceToHost, st);
  // 4. windowed singles in time order (stable: ties keep (event, gid) order)
  hipLaunchKernelGGL(k_time_keys, dim3(grid_for(ns)), dim3(256), 0, st, (size_t)ns, S->in_window, wpos,
                     (const unsigned long long *)S->time_ps, sb.k0, sb.v0);
  if (!sync("after the energy window")) return GPET_ERR_HIP;
  const size_t nw = (size_t)rb[3] + rb[2];
  const unsigned long long tmax = (unsigned long long)rb[4] | ((unsigned long long)rb[5] << 32);
  int time_bits = 0;
  while (time_bits < 64 && (tmax >> time_bits) != 0) ++time_bits;
  if (nw == 0) return GPET_OK;
  const unsigned long long *tk = sb.k1;
  const uint32_t *ti = sb.v1;
  if (nw > 1 && bucket_sort<false>(sb, bb, nw, tmax, st, sb.scan_tmp) != 0u) {
    const bool f2 = radix_sort(sb, nw, time_bits, st);
    tk = f2 ? sb.k1 : sb.k0;
    ti = f2 ? sb.v1 : sb.v0;
  } else if (nw == 1) {
    tk = sb.k0;
    ti = sb.v0;
  }
  // 5. coincidences: count per cluster, scan, write
  hipLaunchKernelGGL(k_coinc_count, dim3(grid_for(nw)), dim3(256), 0, st, nw, tk, ti, S->gid,
                     (uint32_t)D.crystals_per_panel, D.window_ps, flag);
  (void)hipMemcpyAsync(rb + 6, flag + nw - 1, 4, hipMemcpyDeviceToHost, st);
  exclusive_scan(flag, nw, sb.scan_tmp, st);
  (void)hipMemcpyAsync(rb + 7, flag + nw - 1, 4, hipMemcpyDeviceToHost, st);
  hipLaunchKernelGGL(k_coinc_write, dim3(grid_for(nw)), dim3(256), 0, st, nw, tk, ti, S->gid,
                     (uint32_t)D.crystals_per_panel, D.window_ps, flag, C->first, C->second, C->capacity);
  if (!sync("in coincidence sorting")) return GPET_ERR_HIP;
  C->count = (uint64_t)rb[7] + rb[6];
  if (C->count > C->capacity) {
    err = "digitize: coincidence capacity too small";
    return GPET_ERR_CAPACITY;
  }
  return GPET_OK;
}

void free_scratch(DigitizeScratch &scr) {
  if (scr.pinned) (void)hipHostFree(scr.pinned);
  scr.pinned = nullptr;
  if (scr.buf) (void)hipFree(scr.buf);
  scr.buf = nullptr;
  scr.bytes = 0;
}

} // namespace gpet
