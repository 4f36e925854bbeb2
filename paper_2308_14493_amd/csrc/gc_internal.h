// Internal declarations of the graphlet-4 library (not part of the C ABI).
//
// Data model.  A pool holds one or more graphs in one vertex id space.  Graph
// g owns internal ids [base_g, base_g + n_g); inside a graph, internal ids are
// the vertices sorted by (degree at build time, external id), so "id order"
// is a degree order and every row of the adjacency is sorted ascending by id.
// Any fixed total order makes the oriented enumerations below exact; the
// degree order only bounds their cost.
//
// Rows live in an arena of uint32 entries with per-row slack:
//   off[v] (int64), len[v] (int32), cap[v] (int32);  entry = id | flags
// During a counting pass the arena holds the union view of the versions it
// compares: G_0 (before) and G_1 (after) for one batch, or G_0 .. G_k for k
// queued batches of one graph counted together.  Bit 28 + x of an entry is
// set when its edge is absent from version x; between passes no bit is set.
// A structure (edge, wedge, triangle, 4-clique) exists in version x iff none
// of its entries carries bit 28 + x, so the OR of its entries' flags decides
// every version at once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GC_VSHIFT 28
#define GC_F_NEW 0x10000000u   // absent from version 0 (inserted by the pass)
#define GC_F_DEL 0x20000000u   // absent from version 1 (deleted, one-batch pass)
#define GC_FLAGS 0xF0000000u
#define GC_ID    0x0FFFFFFFu
#define GC_MAX_VERTICES (1 << 28)
#define GC_NV_MAX 4            // versions per pass
#define GC_SEQ_MAX 3           // batches of one graph per pass (GC_NV_MAX - 1)

// versions (bit x = version x) in which a structure whose entries' flags OR
// to f exists
template <int NV> __host__ __device__ __forceinline__ constexpr uint32_t vfull() { return (1u << NV) - 1u; }
template <int NV> __host__ __device__ __forceinline__ uint32_t vpresent(uint32_t f) {
  return ~(f >> GC_VSHIFT) & vfull<NV>();
}

// Sigma terms accumulated per graph and version (u64, two's complement):
enum {
  SG_S1 = 0,   // sum_v C(d,3)                      -> non-induced 3-stars
  SG_S2 = 1,   // sum_e (d_u - 1)(d_v - 1)          -> 3-paths + 3 T
  SG_T = 2,    // sum_e t_e (three times the triangles)
  SG_DIA = 3,  // sum_e C(t_e, 2)                   -> non-induced diamonds
  SG_PAW = 4,  // sum_e t_e (d_u + d_v - 4)         -> twice the non-induced paws
  SG_K4 = 5,   // 4-cliques
  SG_C4 = 6,   // 4-cycles
  SG_W = 7,    // sum_v C(d,2)
  SG_D1 = 8,   // sum_v d  (twice the edge count)
  SG_N = 9
};
// per graph: sig[g][version][term]
#define SIG_IDX(g, x, k) (((int64_t)(g) * GC_NV_MAX + (x)) * SG_N + (k))

// Device state per graph (int64): F_conn[6], T, W, m, n, error count
enum { ST_F0 = 0, ST_T = 6, ST_W = 7, ST_M = 8, ST_N = 9, ST_ERR = 10, ST_STRIDE = 16 };

// Statistics written by kernels (u64 counters on the device): first a block
// per batch of the pass (ingest), then the pass-wide counters.
enum { PB_LOOPS = 0, PB_DUPS, PB_CANCEL, PB_INS_EXIST, PB_DEL_MISS, PB_EFF_INS, PB_EFF_DEL, PB_ERR, PB_N };
#define PB_IDX(j, k) ((j) * PB_N + (k))
// Counting-stage counters run from BS_COUNT_STAGE to BS_COUNT.  BS_RETRY: a
// kernel met a vertex larger than its scratch; combine and purge then change
// nothing and the host runs the counting stage again with more scratch.
enum {
  BS_TOUCHED = GC_SEQ_MAX * PB_N, BS_ERR, BS_ARENA_OVF,
  BS_COUNT_STAGE, BS_C4_S = BS_COUNT_STAGE, BS_C4_M, BS_C4_L, BS_WEDGES, BS_TRIPROBE, BS_RETRY,
  BS_C4_WINDOWS,  // dense LDS windows of the large 4-cycle tier
  BS_C4_SEARCH,   // cursor searches of that tier (lower neighbours x window passes)
  BS_TRI_GLOBAL,  // vertices counted by the global-scratch triangle tier
  BS_TRI_REBUILD, // vertices whose version-specific edges overflowed the exception list
  BS_TRI_E,       // adjacency entries the triangle tiers read: N+(u) and the lists N+(v) probed
  BS_K4_SPLIT,    // changed edges whose edge-local 4-cliques were split into chunks
  BS_COUNT
};

struct PoolDev {
  int64_t N;           // vertices in the pool
  int64_t* off;        // [N]
  int32_t* len;        // [N]
  int32_t* cap;        // [N]
  uint32_t* col;       // [arena_cap]
  int64_t arena_cap;
  unsigned long long* arena_top;  // bump pointer (device scalar)
  int32_t* gid;        // [N] graph of each internal vertex
  int32_t* ext2int;    // [N] pool-global external id -> internal id
};

// Region-restricted union view in compact CSR form.
struct RegionDev {
  int64_t* roff;       // [N + 1]
  uint32_t* rcol;      // [E_R]
  int32_t* rlow;       // [N] entries with id < v (N-(v) is the row prefix)
  int32_t* rrow;       // [E_R] row (vertex) of every entry
  int32_t* d;          // [N][NV] degree of v in version x inside the region: d[v * NV + x]
  // triangles through the edge of each entry, per version.  Two versions:
  // t[p] = t_0 | t_1 << 32.  Four versions: t_x = t[p] + field x of the
  // 32-bit pairs tp[2p] (x = 0, 1) and tp[2p + 1] (x = 2, 3) (t[p] holds the
  // triangles present in every version, tp the others)
  unsigned long long* t;   // [E_R]
  unsigned long long* tp;  // [2 E_R] (four versions only)
  int32_t* vpos;       // [E_R] per lower entry v -> w: position of v in row w
};

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int32_t wave_sum32(int32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int32_t wave_incl_scan32(int32_t v) {
  const int l = lane_id();
  for (int o = 1; o < 64; o <<= 1) {
    int32_t t = __shfl_up(v, o);
    if (l >= o) v += t;
  }
  return v;
}
__device__ __forceinline__ int64_t wave_incl_scan64(int64_t v) {
  const int l = lane_id();
  for (int o = 1; o < 64; o <<= 1) {
    int64_t t = __shfl_up(v, o);
    if (l >= o) v += t;
  }
  return v;
}
__device__ __forceinline__ int32_t wave_max32(int32_t v) {
  for (int o = 32; o > 0; o >>= 1) { int32_t t = __shfl_xor(v, o); v = t > v ? t : v; }
  return v;
}

__host__ __device__ __forceinline__ int64_t c2(int64_t x) { return x * (x - 1) / 2; }
__host__ __device__ __forceinline__ int64_t c3(int64_t x) { return x * (x - 1) * (x - 2) / 6; }

// First index in sorted row[0..n) whose id is >= key (flags ignored).
__device__ __forceinline__ int32_t lower_bound_id(const uint32_t* row, int32_t n, uint32_t key) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if ((row[mid] & GC_ID) < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Largest i in [0, n) with pre[i] <= x (pre ascending, pre[0] <= x).
__device__ __forceinline__ int64_t upper_bound_i64(const int64_t* pre, int64_t n, int64_t x) {
  int64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (pre[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// Flush per-lane partial sums for graph g into sig (one atomic per wave).
__device__ __forceinline__ void flush_sig(unsigned long long* sig, int g, int x, int k, int64_t v) {
  v = wave_sum64(v);
  if (lane_id() == 0 && v != 0) atomicAdd(&sig[SIG_IDX(g, x, k)], (unsigned long long)v);
}

// ------------------------------------------------------------ launchers
// sort.hip / scan utilities
size_t radix_sort_tmp_bytes(int64_t max_count);
// Sorts keys[0..count) ascending on bits [0, bits); count may live on the
// device (d_count != nullptr, max_count is then an upper bound).  Returns the
// buffer that holds the result (keys or alt).
unsigned long long* radix_sort_u64(unsigned long long* keys, unsigned long long* alt,
                                   void* tmp, int64_t max_count, const unsigned long long* d_count,
                                   int bits, hipStream_t s);
// The buffer radix_sort_u64 leaves its result in (known before it runs).
unsigned long long* radix_sort_result(unsigned long long* keys, unsigned long long* alt, int64_t max_count, int bits);
size_t scan_tmp_bytes(int64_t n);
// out[i] = sum_{j<i} in[j] for i in [0, n]; out has n + 1 entries.
void exclusive_scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t s);
// the same over the first min(*d_n, n) entries (a count known only on the
// device); out[*d_n] and out[n] get the total, entries in between are left
void exclusive_scan_i32_to_i64_count(const int32_t* in, int64_t* out, int64_t n, const int64_t* d_n, void* tmp,
                                     hipStream_t s);
void exclusive_scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t s);

// fill helpers (kernels, capturable)
void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s);
// p[i] = v for i < min(mult * (*count), max_n), count on the device
void fill_u64_count(unsigned long long* p, unsigned long long v, const unsigned long long* count, int64_t mult,
                    int64_t max_n, hipStream_t s);
