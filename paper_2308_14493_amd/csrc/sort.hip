// Device primitives: LSD radix sort of u64 keys, exclusive scans, fills.
//
// Radix sort: 8-bit digits, tiles of 4096 keys per 256-thread block.
//   hist    : per-tile digit histogram -> hist[digit * nblk + blk]
//   scan    : digit-major exclusive scan of hist (per-digit row scan, then
//             a scan of the 256 row totals)
//   scatter : stable rank inside the tile (16 rounds of 256 consecutive keys;
//             rank within a wave by 8 ballots, across waves through LDS)
// Counts may live on the device so that the whole sort is capturable with a
// size known only to earlier kernels; tiles beyond the count exit at once,
// and the histogram scans read only the tiles that hold keys.
// Sorts whose capacity fits one workgroup's LDS run as one kernel
// (k_rs_small).
#include "gc_internal.h"

namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
constexpr int RS_WAVES = RS_THREADS / 64;

__device__ __forceinline__ int64_t rs_count(int64_t max_count, const unsigned long long* d_count) {
  if (!d_count) return max_count;
  int64_t c = (int64_t)*d_count;
  return c < max_count ? c : max_count;
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const unsigned long long* __restrict__ keys,
                                                       int64_t max_count, const unsigned long long* d_count,
                                                       int shift, uint32_t* __restrict__ hist, int64_t nblk) {
  __shared__ uint32_t h[256];
  const int64_t count = rs_count(max_count, d_count);
  const int64_t blk = blockIdx.x;
  const int64_t base = blk * RS_TILE;
  if (base >= count) return;  // tiles past the count are not scanned (uniform per block)
  h[threadIdx.x] = 0;
  __syncthreads();
  for (int r = 0; r < RS_ROUNDS; ++r) {
    int64_t i = base + r * RS_THREADS + threadIdx.x;
    if (i < count) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blk] = h[threadIdx.x];
}

// tiles holding keys: the histogram rows are read only that far
__device__ __forceinline__ int64_t rs_tiles(int64_t max_count, const unsigned long long* d_count) {
  return (rs_count(max_count, d_count) + RS_TILE - 1) / RS_TILE;
}

// One block per digit: exclusive scan of that digit's row; row total out.
__global__ __launch_bounds__(1024) void k_rs_rowscan(uint32_t* __restrict__ hist, int64_t nblk,
                                                     uint32_t* __restrict__ totals, int64_t max_count,
                                                     const unsigned long long* d_count) {
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t carry;
  uint32_t* row = hist + (int64_t)blockIdx.x * nblk;
  const int64_t nt = rs_tiles(max_count, d_count);
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nt; base += 1024) {
    int64_t i = base + threadIdx.x;
    uint32_t v = i < nt ? row[i] : 0u;
    int32_t inc = wave_incl_scan32((int32_t)v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) wsum[w] = (uint32_t)inc;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before += wsum[k];
    uint32_t c = carry;
    if (i < nt) row[i] = c + before + (uint32_t)inc - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = c + before + (uint32_t)inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(256) void k_rs_addtotals(uint32_t* __restrict__ hist, int64_t nblk,
                                                      const uint32_t* __restrict__ totals, int64_t max_count,
                                                      const unsigned long long* d_count) {
  __shared__ uint32_t pre[256];
  const int64_t nt = rs_tiles(max_count, d_count);
  if (nt == 0) return;  // uniform
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int d = 0; d < 256; ++d) { pre[d] = s; s += totals[d]; }
  }
  __syncthreads();
  const int64_t total = nt * 256;  // digit d, tile b < nt: hist[d * nblk + b]
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = i / nt;
    hist[d * nblk + (i - d * nt)] += pre[d];
  }
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const unsigned long long* __restrict__ keys,
                                                          unsigned long long* __restrict__ out,
                                                          int64_t max_count, const unsigned long long* d_count,
                                                          int shift, const uint32_t* __restrict__ hist,
                                                          int64_t nblk) {
  __shared__ uint32_t base_off[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[RS_WAVES][256];
  const int64_t count = rs_count(max_count, d_count);
  const int64_t blk = blockIdx.x;
  const int64_t tbase = blk * RS_TILE;
  if (tbase >= count) return;  // uniform per block
  const int tid = threadIdx.x, w = tid >> 6;
  base_off[tid] = hist[(int64_t)tid * nblk + blk];
  run[tid] = 0;
  for (int k = 0; k < RS_WAVES; ++k) wcnt[k][tid] = 0;
  __syncthreads();
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t i = tbase + r * RS_THREADS + tid;
    const bool valid = i < count;
    unsigned long long key = valid ? keys[i] : 0ull;
    const uint32_t d = (uint32_t)(key >> shift) & 255u;
    uint64_t same = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      uint64_t bb = __ballot((d >> b) & 1u);
      same &= ((d >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t wrank = (uint32_t)__popcll(same & lanemask_lt());
    const bool leader = valid && (same & lanemask_lt()) == 0;
    if (leader) wcnt[w][d] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t before = run[d];
      for (int k = 0; k < w; ++k) before += wcnt[k][d];
      out[base_off[d] + before + wrank] = key;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int k = 0; k < RS_WAVES; ++k) { add += wcnt[k][tid]; wcnt[k][tid] = 0; }
    run[tid] += add;
    __syncthreads();
  }
}

// Sorts of at most RSS_MAX keys (the ingest of batches of up to a few
// thousand updates) in one workgroup: the keys stay in LDS through every
// digit, each digit a stable counting sort (digit histogram by LDS atomics,
// its exclusive scan by one wave, then the tile's ranking of k_rs_scatter in
// rounds of RSS_T consecutive keys), so a sort is one launch instead of four
// per digit.  Same digits, same stable order: the result equals the
// multi-block sort's, and lands in the same buffer.
constexpr int RSS_T = 1024;
constexpr int RSS_MAX = 4096;
constexpr int RSS_WAVES = RSS_T / 64;

__global__ __launch_bounds__(RSS_T) void k_rs_small(const unsigned long long* keys,
                                                    unsigned long long* out, int64_t max_count,
                                                    const unsigned long long* d_count, int bits) {
  __shared__ unsigned long long buf[2][RSS_MAX];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[RSS_WAVES][256];
  const int32_t count = (int32_t)rs_count(max_count, d_count);  // <= max_count <= RSS_MAX
  const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
  for (int32_t i = tid; i < count; i += RSS_T) buf[0][i] = keys[i];
  for (int k = tid; k < RSS_WAVES * 256; k += RSS_T) (&wcnt[0][0])[k] = 0u;
  int cur = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    const unsigned long long* src = buf[cur];
    unsigned long long* dst = buf[cur ^ 1];
    if (tid < 256) { hist[tid] = 0u; run[tid] = 0u; }
    __syncthreads();
    for (int32_t i = tid; i < count; i += RSS_T) atomicAdd(&hist[(uint32_t)(src[i] >> shift) & 255u], 1u);
    __syncthreads();
    if (w == 0) {  // exclusive scan of the 256 digit counts, four per lane
      uint32_t c[4], t = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) { c[k] = hist[4 * l + k]; t += c[k]; }
      uint32_t before = (uint32_t)wave_incl_scan32((int32_t)t) - t;
#pragma unroll
      for (int k = 0; k < 4; ++k) { hist[4 * l + k] = before; before += c[k]; }
    }
    __syncthreads();
    for (int32_t r0 = 0; r0 < count; r0 += RSS_T) {
      const int32_t i = r0 + tid;
      const bool valid = i < count;
      const unsigned long long key = valid ? src[i] : 0ull;
      const uint32_t d = (uint32_t)(key >> shift) & 255u;
      uint64_t same = __ballot(valid);
      for (int b = 0; b < 8; ++b) {
        const uint64_t bb = __ballot((d >> b) & 1u);
        same &= ((d >> b) & 1u) ? bb : ~bb;
      }
      const uint32_t wrank = (uint32_t)__popcll(same & lanemask_lt());
      if (valid && (same & lanemask_lt()) == 0) wcnt[w][d] = (uint32_t)__popcll(same);
      __syncthreads();
      if (valid) {
        uint32_t before = hist[d] + run[d];
        for (int k = 0; k < w; ++k) before += wcnt[k][d];
        dst[before + wrank] = key;
      }
      __syncthreads();
      if (tid < 256) {
        uint32_t add = 0;
        for (int k = 0; k < RSS_WAVES; ++k) { add += wcnt[k][tid]; wcnt[k][tid] = 0u; }
        run[tid] += add;
      }
      __syncthreads();
    }
    cur ^= 1;
  }
  for (int32_t i = tid; i < count; i += RSS_T) out[i] = buf[cur][i];
}

// ------------------------------------------------------------- scans
constexpr int SC_THREADS = 1024;
constexpr int SC_ITEMS = 4;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

// Scans may take their element count from the device (d_n, at most the
// capacity n the grid is sized for): entries from the count on are neither
// read nor written, and the total goes to out[count] and out[n].
__device__ __forceinline__ int64_t scan_count(int64_t n, const int64_t* d_n) {
  if (!d_n) return n;
  const int64_t c = *d_n;
  return c < 0 ? 0 : (c < n ? c : n);
}

template <class TIn>
__global__ __launch_bounds__(SC_THREADS) void k_scan_reduce(const TIn* __restrict__ in, int64_t n,
                                                            const int64_t* d_n, int64_t* __restrict__ bsum) {
  __shared__ int64_t ws[SC_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SC_TILE;
  const int64_t nn = scan_count(n, d_n);
  int64_t s = 0;
  for (int k = 0; k < SC_ITEMS; ++k) {
    int64_t i = base + (int64_t)k * SC_THREADS + threadIdx.x;
    if (i < nn) s += (int64_t)in[i];
  }
  s = wave_sum64(s);
  if (lane_id() == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int k = 0; k < SC_THREADS / 64; ++k) t += ws[k];
    bsum[blockIdx.x] = t;
  }
}

// single block: exclusive scan of nb block sums in place
__global__ __launch_bounds__(SC_THREADS) void k_scan_top(int64_t* __restrict__ bsum, int64_t nb) {
  __shared__ int64_t ws[SC_THREADS / 64];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += SC_THREADS) {
    int64_t i = base + threadIdx.x;
    int64_t v = i < nb ? bsum[i] : 0;
    int64_t inc = wave_incl_scan64(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) ws[w] = inc;
    __syncthreads();
    int64_t before = carry;
    for (int k = 0; k < w; ++k) before += ws[k];
    if (i < nb) bsum[i] = before + inc - v;
    __syncthreads();
    if (threadIdx.x == SC_THREADS - 1) carry = before + inc;
    __syncthreads();
  }
}

template <class TIn>
__global__ __launch_bounds__(SC_THREADS) void k_scan_down(const TIn* __restrict__ in, int64_t n,
                                                          const int64_t* d_n, const int64_t* __restrict__ bsum,
                                                          int64_t* __restrict__ out) {
  __shared__ int64_t ws[SC_THREADS / 64];
  // each thread owns SC_ITEMS consecutive elements
  const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
  const int64_t nn = scan_count(n, d_n);
  int64_t v[SC_ITEMS];
  int64_t s = 0;
  for (int k = 0; k < SC_ITEMS; ++k) {
    int64_t i = base + k;
    v[k] = i < nn ? (int64_t)in[i] : 0;
    s += v[k];
  }
  int64_t inc = wave_incl_scan64(s);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) ws[w] = inc;
  __syncthreads();
  int64_t before = bsum[blockIdx.x];
  for (int k = 0; k < w; ++k) before += ws[k];
  int64_t run = before + inc - s;
  for (int k = 0; k < SC_ITEMS; ++k) {
    int64_t i = base + k;
    if (i < nn) out[i] = run;
    run += v[k];
  }
  // total at out[n] (and at out[count])
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SC_THREADS - 1) {
    out[n] = run;
    if (nn < n) out[nn] = run;
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// p[i] = v for i < min(mult * (*count), max_n): a fill whose size is known
// only to earlier kernels
__global__ void k_fill_u64_count(unsigned long long* p, unsigned long long v, const unsigned long long* count,
                                 int64_t mult, int64_t max_n) {
  int64_t n = (int64_t)*count * mult;
  if (n > max_n) n = max_n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

inline int64_t rs_nblk(int64_t max_count) { return (max_count + RS_TILE - 1) / RS_TILE; }

template <class TIn>
void scan_impl(const TIn* in, int64_t* out, int64_t n, void* tmp, hipStream_t s, const int64_t* d_n = nullptr) {
  int64_t nb = (n + SC_TILE - 1) / SC_TILE;
  if (nb == 0) nb = 1;
  int64_t* bsum = (int64_t*)tmp;
  hipLaunchKernelGGL(k_scan_reduce<TIn>, dim3((unsigned)nb), dim3(SC_THREADS), 0, s, in, n, d_n, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SC_THREADS), 0, s, bsum, nb);
  hipLaunchKernelGGL(k_scan_down<TIn>, dim3((unsigned)nb), dim3(SC_THREADS), 0, s, in, n, d_n, bsum, out);
}

}  // namespace

size_t radix_sort_tmp_bytes(int64_t max_count) {
  int64_t nblk = rs_nblk(max_count);
  if (nblk < 1) nblk = 1;
  return (size_t)(nblk * 256 + 256) * sizeof(uint32_t);
}

unsigned long long* radix_sort_u64(unsigned long long* keys, unsigned long long* alt, void* tmp,
                                   int64_t max_count, const unsigned long long* d_count, int bits,
                                   hipStream_t s) {
  if (max_count <= 0 || bits <= 0) return keys;
  if (max_count <= RSS_MAX) {
    unsigned long long* out = radix_sort_result(keys, alt, max_count, bits);
    hipLaunchKernelGGL(k_rs_small, dim3(1), dim3(RSS_T), 0, s, keys, out, max_count, d_count, bits);
    return out;
  }
  int64_t nblk = rs_nblk(max_count);
  uint32_t* hist = (uint32_t*)tmp;
  uint32_t* totals = hist + nblk * 256;
  unsigned long long* src = keys;
  unsigned long long* dst = alt;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nblk), dim3(RS_THREADS), 0, s, src, max_count, d_count,
                       shift, hist, nblk);
    hipLaunchKernelGGL(k_rs_rowscan, dim3(256), dim3(1024), 0, s, hist, nblk, totals, max_count, d_count);
    unsigned g = (unsigned)((nblk * 256 + 255) / 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_rs_addtotals, dim3(g), dim3(256), 0, s, hist, nblk, totals, max_count, d_count);
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nblk), dim3(RS_THREADS), 0, s, src, dst, max_count,
                       d_count, shift, hist, nblk);
    unsigned long long* t = src; src = dst; dst = t;
  }
  return src;
}

unsigned long long* radix_sort_result(unsigned long long* keys, unsigned long long* alt, int64_t max_count, int bits) {
  if (max_count <= 0 || bits <= 0) return keys;
  const int passes = (bits + 7) / 8;
  return passes % 2 == 0 ? keys : alt;
}

size_t scan_tmp_bytes(int64_t n) { return (size_t)((n + SC_TILE - 1) / SC_TILE + 2) * sizeof(int64_t); }

void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t s) {
  scan_impl<int32_t>(in, out, n, tmp, s);
}
void exclusive_scan_i32_to_i64_count(const int32_t* in, int64_t* out, int64_t n, const int64_t* d_n, void* tmp,
                                     hipStream_t s) {
  scan_impl<int32_t>(in, out, n, tmp, s, d_n);
}
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t s) {
  scan_impl<int64_t>(in, out, n, tmp, s);
}

void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
}
void fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
}
void fill_u64_count(unsigned long long* p, unsigned long long v, const unsigned long long* count, int64_t mult,
                    int64_t max_n, hipStream_t s) {
  if (max_n <= 0) return;
  int64_t g = (max_n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_fill_u64_count, dim3((unsigned)g), dim3(256), 0, s, p, v, count, mult, max_n);
}
