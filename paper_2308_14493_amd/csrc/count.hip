// Counting kernels: the local static counter applied to the region, fused
// over the two versions (G_b before, G_a after the batch; Alg. 2 counts both
// and adds C_a - C_b).  Every structure is enumerated once in the union view
// and its presence in each version is read off the flags of its entries.
//
// Per-edge counting (the PGD approach of Sec. 3: iterate over edges, count
// triangles, 4-cliques and 4-cycles, derive the rest by combinatorics):
//   triangles  oriented by id: u < v < w found at u, with v in N+(u) and
//              w in N+(u) & N+(v).  Each triangle adds 1 to t of its three
//              edges (t_e = common neighbours of the endpoints of e).
//   4-cliques  u < v < w < x, x in N+(u) & N+(v) & N+(w).
//   4-cycles   counted once, at the largest vertex v, through the opposite
//              vertex w < v: c(v,w) = #{u < v adjacent to both}, and
//              sum_w C(c(v,w), 2).
//   the non-induced counts follow:
//     N_K13 = sum_v C(d,3)        N_P4 = sum_e (d_u-1)(d_v-1) - 3T
//     N_paw = sum_tri (d_u + d_v + d_w - 6)   N_dia = sum_e C(t_e, 2)
//     N_K4, N_C4 as enumerated.
//
// Tiers (work lists built by the per-vertex pass):
//   tri  S: out-degree <= 64, one wave per vertex, bit matrices in LDS
//   tri  L: larger out-degree, one workgroup per vertex, LDS hash
//   c4   S / M: wedge bound <= 256 / <= 4096, LDS hash per wave / workgroup
//   c4   L: one workgroup per vertex, dense counters in global memory
#include "gc_kernels.h"

namespace {

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

__device__ __forceinline__ uint32_t hash32(uint32_t x) { return x * 2654435761u; }

__device__ __forceinline__ int32_t ld_relaxed(int32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }

// find key in an open-addressing table of size mask+1 (keys -1 = empty)
__device__ __forceinline__ int lookup_slot(const int32_t* keys, const int16_t* vals, uint32_t mask, int shift,
                                           uint32_t key) {
  uint32_t h = hash32(key) >> shift;
  while (true) {
    int32_t k = keys[h];
    if (k == (int32_t)key) return vals[h];
    if (k == -1) return -1;
    h = (h + 1) & mask;
  }
}

// add `add` to the counter of key (insert on first use)
template <class V>
__device__ __forceinline__ void hash_add(int32_t* keys, V* vals, uint32_t mask, int shift, uint32_t key, V add) {
  uint32_t h = hash32(key) >> shift;
  while (true) {
    int32_t k = ld_relaxed(&keys[h]);
    if (k == (int32_t)key) { atomicAdd(&vals[h], add); return; }
    if (k == -1) {
      int32_t old = atomicCAS(&keys[h], -1, (int32_t)key);
      if (old == -1 || old == (int32_t)key) { atomicAdd(&vals[h], add); return; }
    }
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ int log2i(uint32_t x) { return 31 - __clz(x); }

// Segment search for wave-flattened loops: every lane holds one segment
// with exclusive prefix `excl`; returns the lane whose segment holds idx
// (largest lane with excl <= idx).  All 64 lanes must call it.
__device__ __forceinline__ int seg_of(int32_t excl, int32_t idx) {
  int lo = 0, hi = 64;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    int mid = (lo + hi) >> 1;
    int32_t e = __shfl(excl, mid);
    if (e <= idx) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ unsigned long long pack2(uint32_t b, uint32_t a) {
  return (unsigned long long)b | ((unsigned long long)a << 32);
}

// flush lane-private sums of a wave whose lanes all work for graph g
__device__ __forceinline__ void flush2(unsigned long long* sig, int g, int k, int64_t& b, int64_t& a) {
  flush_sig(sig, g, 0, k, b);
  flush_sig(sig, g, 1, k, a);
  b = 0; a = 0;
}

// ------------------------------------------------------ triangles, tier S
constexpr int TS_WAVES = 4;

__global__ __launch_bounds__(256) void k_tri_small(CountArgs A) {
  __shared__ int32_t hkey[TS_WAVES][128];
  __shared__ int16_t hval[TS_WAVES][128];
  __shared__ uint32_t fsl[TS_WAVES][64];
  __shared__ unsigned long long EB[TS_WAVES][64], EA[TS_WAVES][64], TB[TS_WAVES][64], TA[TS_WAVES][64];
  const int w = threadIdx.x >> 6, l = lane_id();
  const RegionDev& R = A.R;
  const int64_t n = (int64_t)A.c[C_LIST0 + L_TRI_S];
  const int32_t* list = A.lists + L_TRI_S * A.list_stride;
  int cur_g = -1;
  int64_t kb_ = 0, ka_ = 0;
  for (int64_t it = (int64_t)blockIdx.x * TS_WAVES + w; it < n; it += (int64_t)gridDim.x * TS_WAVES) {
    const int32_t u = list[it];
    const int g = A.gid[u];
    if (g != cur_g) {
      if (cur_g >= 0) flush2(A.sig, cur_g, SG_K4, kb_, ka_);
      cur_g = g;
    }
    const int64_t ub = R.roff[u] + R.rlow[u];
    const int32_t dp = (int32_t)(R.roff[u + 1] - ub);
    uint32_t vi = 0, fi = 0;
    if (l < dp) { const uint32_t x = R.rcol[ub + l]; vi = x & GC_ID; fi = x & GC_FLAGS; }
    hkey[w][l] = -1; hkey[w][l + 64] = -1;
    EB[w][l] = 0; EA[w][l] = 0; TB[w][l] = 0; TA[w][l] = 0;
    fsl[w][l] = fi;
    wave_sync();
    if (l < dp) {
      uint32_t h = hash32(vi) >> 25;
      while (atomicCAS(&hkey[w][h], -1, (int32_t)vi) != -1) h = (h + 1) & 127u;
      hval[w][h] = (int16_t)l;
    }
    wave_sync();
    int64_t sb = 0;
    int32_t sl = 0;
    if (l < dp) { sb = R.roff[vi] + R.rlow[vi]; sl = (int32_t)(R.roff[vi + 1] - sb); }
    const int32_t incl = wave_incl_scan32(sl);
    const int32_t total = __shfl(incl, 63);
    const int32_t excl = incl - sl;
    for (int32_t base = 0; base < total; base += 64) {
      const int32_t idx = base + l;
      const int i = seg_of(excl, idx);
      const int64_t sbi = __shfl(sb, i);
      const int32_t exi = __shfl(excl, i);
      if (idx < total) {
        const int64_t pos = sbi + (idx - exi);
        const uint32_t y = R.rcol[pos];
        const int j = lookup_slot(hkey[w], hval[w], 127u, 25, y & GC_ID);
        if (j >= 0) {
          const uint32_t fy = y & GC_FLAGS;
          const unsigned long long bj = 1ull << j, bi = 1ull << i;
          if (!(fy & GC_F_NEW)) { atomicOr(&EB[w][i], bj); atomicOr(&TB[w][j], bi); }
          if (!(fy & GC_F_DEL)) { atomicOr(&EA[w][i], bj); atomicOr(&TA[w][j], bi); }
          const uint32_t ab = fsl[w][i] | fsl[w][j] | fy;
          const uint32_t xb = !(ab & GC_F_NEW), xa = !(ab & GC_F_DEL);
          if (xb | xa) atomicAdd(&R.t[pos], pack2(xb, xa));
        }
      }
    }
    wave_sync();
    const uint64_t Pb = __ballot(l < dp && !(fi & GC_F_NEW));
    const uint64_t Pa = __ballot(l < dp && !(fi & GC_F_DEL));
    if (l < dp) {
      const bool pb = (Pb >> l) & 1ull, pa = (Pa >> l) & 1ull;
      const uint64_t rb = EB[w][l] & Pb, ra = EA[w][l] & Pa;
      const uint64_t cb = TB[w][l] & Pb, ca = TA[w][l] & Pa;
      const int32_t tub = pb ? __popcll(rb | cb) : 0, tua = pa ? __popcll(ra | ca) : 0;
      int64_t k4b = 0, k4a = 0;
      if (pb) for (uint64_t m = rb; m; m &= m - 1) k4b += __popcll(rb & EB[w][__builtin_ctzll(m)] & Pb);
      if (pa) for (uint64_t m = ra; m; m &= m - 1) k4a += __popcll(ra & EA[w][__builtin_ctzll(m)] & Pa);
      kb_ += k4b; ka_ += k4a;
      if (tub | tua) atomicAdd(&R.t[ub + l], pack2(tub, tua));
    }
    wave_sync();
  }
  if (cur_g >= 0) flush2(A.sig, cur_g, SG_K4, kb_, ka_);
}

// ------------------------------------------------------ triangles, tier L
// One workgroup per vertex u with out-degree above 64.  N+(u) goes into a
// hash (slot = position in the sorted suffix, i.e. id order).  The waves
// walk the lists N+(v_i) of 64 slots i at a time, flattened over lanes: a
// hit j is a triangle (u, v_i, w_j); it updates t of the three edges and
// records the edge v_i -> w_j as bit j of row i of the bit matrix E (the
// graph induced on N+(u), union view).  4-cliques u < v_i < v_j < v_k then
// follow from AND-popcounts of rows:
//   K4_x(u) = sum_{i in P_x} sum_{j in E[i] & P_x} |E[i] & E[j] & P_x|
// with P_x the slots whose edge from u exists in version x.  Edges among
// N+(u) that exist in one version only are few; the triangles of E that
// contain such an edge absent from version x are removed from K4_x one by
// one (each once, at its first such edge in list order).  If the list
// overflows, the matrix is rebuilt per version instead.
constexpr int TL_EXC = 256;    // version-specific edges tracked per vertex

struct TriL {
  unsigned long long* E;   // [dp][W] row bitsets
  unsigned long long* P;   // [2][W] slot masks of versions b, a
  uint32_t* ids;           // [dp]
  int32_t* hkey;           // [H]
  int16_t* hval;           // [H]
  uint32_t* tuc;           // [dp] packed 16-bit halves (b low, a high)
  uint32_t* exc;           // [TL_EXC] i << 17 | j << 2 | flags >> 30
  int32_t* nexc;           // [1]
  int32_t W;               // words per row
};

__device__ __forceinline__ bool Ebit(const TriL& S, int32_t p, int32_t q) {  // edge between slots p != q
  if (p > q) { int32_t t = p; p = q; q = t; }
  return (S.E[(int64_t)p * S.W + (q >> 6)] >> (q & 63)) & 1ull;
}

// One wave: slots [g0, g0 + 64) of N+(u), their out-lists flattened over
// lanes.  only = 0: union matrix plus all triangle bookkeeping; only = 1/2:
// matrix of version b / a alone.
__device__ __forceinline__ void tri_large_probe(const CountArgs& A, const TriL& S, uint32_t hmask, int shift,
                                                int32_t g0, int32_t dp, int only) {
  const RegionDev& R = A.R;
  const int l = lane_id();
  const int32_t i0 = g0 + l;
  int64_t sb = 0;
  int32_t sl = 0;
  uint32_t fi = 0;
  if (i0 < dp) {
    const uint32_t xi = S.ids[i0];
    const uint32_t v = xi & GC_ID;
    fi = xi & GC_FLAGS;
    sb = R.roff[v] + R.rlow[v];
    sl = (int32_t)(R.roff[v + 1] - sb);
  }
  const int32_t incl = wave_incl_scan32(sl);
  const int32_t tot = __shfl(incl, 63);
  const int32_t excl = incl - sl;
  for (int32_t base = 0; base < tot; base += 64) {
    const int32_t idx = base + l;
    const int s = seg_of(excl, idx);
    const int64_t sbs = __shfl(sb, s);
    const int32_t exs = __shfl(excl, s);
    const uint32_t fs = __shfl(fi, s);
    if (idx >= tot) continue;
    const int32_t i = g0 + s;
    const int64_t pos = sbs + (idx - exs);
    const uint32_t y = R.rcol[pos];
    const int j = lookup_slot(S.hkey, S.hval, hmask, shift, y & GC_ID);
    if (j < 0) continue;
    unsigned long long* Ei = S.E + (int64_t)i * S.W;
    const uint32_t fy = y & GC_FLAGS;
    if (only) {
      if (!(fy & (only == 1 ? GC_F_NEW : GC_F_DEL))) atomicOr(&Ei[j >> 6], 1ull << (j & 63));
      continue;
    }
    atomicOr(&Ei[j >> 6], 1ull << (j & 63));
    if (fy) {
      const int32_t p = atomicAdd(S.nexc, 1);
      if (p < TL_EXC) S.exc[p] = ((uint32_t)i << 17) | ((uint32_t)j << 2) | (fy >> 30);
    }
    const uint32_t ab = fs | (S.ids[j] & GC_FLAGS) | fy;
    const uint32_t xb = !(ab & GC_F_NEW), xa = !(ab & GC_F_DEL);
    if (xb | xa) {
      atomicAdd(&R.t[pos], pack2(xb, xa));
      atomicAdd(&S.tuc[j], xb | (xa << 16));
      atomicAdd(&S.tuc[i], xb | (xa << 16));
    }
  }
}

// sum over i in mask, j in E[i] & mask of |E[i] & E[j] & mask|  (one wave's rows)
__device__ __forceinline__ int64_t k4_rows(const TriL& S, const unsigned long long* mask, int32_t dp, int nwaves) {
  const int w = threadIdx.x >> 6, l = lane_id();
  int64_t cnt = 0;
  for (int32_t i = w; i < dp; i += nwaves) {
    if (!((mask[i >> 6] >> (i & 63)) & 1ull)) continue;
    const unsigned long long* Ei = S.E + (int64_t)i * S.W;
    for (int32_t w0 = i >> 6; w0 < S.W; ++w0) {
      const unsigned long long m = Ei[w0] & mask[w0];
      if (!m) continue;
      if ((m >> l) & 1ull) {
        const int32_t j = w0 * 64 + l;
        const unsigned long long* Ej = S.E + (int64_t)j * S.W;
        for (int32_t q = j >> 6; q < S.W; ++q) cnt += __popcll(Ei[q] & Ej[q] & mask[q]);
      }
    }
  }
  return cnt;
}

__device__ void tri_large_vertex(const CountArgs& A, const TriL& S, int32_t u, int64_t ub, int32_t dp,
                                 int64_t& kb_, int64_t& ka_) {
  const RegionDev& R = A.R;
  const int w = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int32_t W = S.W;
  int H = 1;
  while (H < 2 * dp) H <<= 1;
  const uint32_t hmask = (uint32_t)H - 1u;
  const int shift = 32 - log2i((uint32_t)H);
  for (int32_t k = threadIdx.x; k < dp; k += blockDim.x) { S.ids[k] = R.rcol[ub + k]; S.tuc[k] = 0; }
  for (int32_t k = threadIdx.x; k < H; k += blockDim.x) S.hkey[k] = -1;
  for (int64_t k = threadIdx.x; k < (int64_t)dp * W; k += blockDim.x) S.E[k] = 0ull;
  for (int32_t k = threadIdx.x; k < 2 * W; k += blockDim.x) S.P[k] = 0ull;
  if (threadIdx.x == 0) *S.nexc = 0;
  __syncthreads();
  for (int32_t k = threadIdx.x; k < dp; k += blockDim.x) {
    const uint32_t x = S.ids[k];
    const uint32_t id = x & GC_ID;
    uint32_t h = hash32(id) >> shift;
    while (atomicCAS(&S.hkey[h], -1, (int32_t)id) != -1) h = (h + 1) & hmask;
    S.hval[h] = (int16_t)k;
    if (!(x & GC_F_NEW)) atomicOr(&S.P[k >> 6], 1ull << (k & 63));
    if (!(x & GC_F_DEL)) atomicOr(&S.P[W + (k >> 6)], 1ull << (k & 63));
  }
  __syncthreads();
  for (int32_t g0 = w * 64; g0 < dp; g0 += nwaves * 64) tri_large_probe(A, S, hmask, shift, g0, dp, 0);
  __syncthreads();
  const int32_t ne = *S.nexc;
  const unsigned long long* Pb = S.P;
  const unsigned long long* Pa = S.P + W;
  if (ne <= TL_EXC) {
    bool same = true;
    for (int32_t q = 0; q < W; ++q) same &= Pb[q] == Pa[q];
    const int64_t cb = k4_rows(S, Pb, dp, nwaves);
    const int64_t ca = same ? cb : k4_rows(S, Pa, dp, nwaves);
    kb_ += cb;
    ka_ += ca;
    // triangles of E (inside P_x) holding an edge absent from version x
    const int l = lane_id();
    for (int32_t e = w; e < ne; e += nwaves) {
      const uint32_t ex = S.exc[e];
      const int32_t i = (int32_t)(ex >> 17), j = (int32_t)((ex >> 2) & 0x7FFF);
      const uint32_t fl = (ex & 3u) << 30;
      for (int x = 0; x < 2; ++x) {
        const uint32_t absent = x == 0 ? GC_F_NEW : GC_F_DEL;
        if (!(fl & absent)) continue;
        const unsigned long long* Px = x == 0 ? Pb : Pa;
        if (!((Px[i >> 6] >> (i & 63)) & 1ull) || !((Px[j >> 6] >> (j & 63)) & 1ull)) continue;
        int64_t sub = 0;
        for (int32_t k = l; k < dp; k += 64) {
          if (k == i || k == j || !((Px[k >> 6] >> (k & 63)) & 1ull)) continue;
          if (!Ebit(S, i, k) || !Ebit(S, j, k)) continue;
          // count once: skip if an earlier listed edge of this triangle is absent from x
          bool first = true;
          for (int32_t f = 0; f < e && first; ++f) {
            const uint32_t ef = S.exc[f];
            if (!(((ef & 3u) << 30) & absent)) continue;
            const int32_t fi = (int32_t)(ef >> 17), fj = (int32_t)((ef >> 2) & 0x7FFF);
            if ((fi == i && fj == k) || (fi == k && fj == i) || (fi == j && fj == k) || (fi == k && fj == j))
              first = false;
          }
          sub += first;
        }
        if (x == 0) kb_ -= sub; else ka_ -= sub;
      }
    }
  } else {
    // too many version-specific edges: rebuild E per version and count
    for (int x = 0; x < 2; ++x) {
      __syncthreads();
      for (int64_t k = threadIdx.x; k < (int64_t)dp * W; k += blockDim.x) S.E[k] = 0ull;
      __syncthreads();
      for (int32_t g0 = w * 64; g0 < dp; g0 += nwaves * 64) tri_large_probe(A, S, hmask, shift, g0, dp, x + 1);
      __syncthreads();
      const int64_t c = k4_rows(S, x == 0 ? Pb : Pa, dp, nwaves);
      if (x == 0) kb_ += c; else ka_ += c;
    }
  }
  __syncthreads();
  for (int32_t k = threadIdx.x; k < dp; k += blockDim.x) {
    const uint32_t c = S.tuc[k];
    if (c) atomicAdd(&R.t[ub + k], pack2(c & 0xFFFFu, c >> 16));
  }
  __syncthreads();
}

// global-scratch slot layout (u64 words): E [cap*W] | P [2W] | then u32 words:
// ids [cap] | tuc [cap] | hkey [4 cap] | hval [2 cap] | exc [TL_EXC] | nexc [2]
__host__ __device__ inline int64_t tri_slot_words64(int64_t cap) {
  const int64_t W = ((cap + 63) / 64) | 1;
  return cap * W + 2 * W + (cap + cap + 4 * cap + 2 * cap + TL_EXC + 2 + 1) / 2 + 8;
}

// Vertices with out-degree in (LO, CAP]; CAP = 0 selects the global-memory
// scratch for everything above LO.
template <int CAP, int THREADS>
__global__ __launch_bounds__(THREADS) void k_tri_large(CountArgs A, int32_t lo_dp) {
  const RegionDev& R = A.R;
  const int64_t n = (int64_t)A.c[C_LIST0 + L_TRI_L];
  const int32_t* list = A.lists + L_TRI_L * A.list_stride;
  int cur_g = -1;
  int64_t kb_ = 0, ka_ = 0;
  TriL S;
  if constexpr (CAP == 0) {
    const int64_t cap = A.tri_cap;
    const int64_t W = ((cap + 63) / 64) | 1;
    unsigned long long* base = (unsigned long long*)A.tri_scratch + (int64_t)blockIdx.x * tri_slot_words64(cap);
    S.W = (int32_t)W;
    S.E = base;
    S.P = base + cap * W;
    uint32_t* u32 = (uint32_t*)(S.P + 2 * W);
    S.ids = u32;
    S.tuc = u32 + cap;
    S.hkey = (int32_t*)(u32 + 2 * cap);
    S.hval = (int16_t*)(u32 + 6 * cap);
    S.exc = u32 + 8 * cap;
    S.nexc = (int32_t*)(u32 + 8 * cap + TL_EXC);
  } else {
    constexpr int CW = CAP / 64;
    constexpr int CWS = CW | 1;  // largest odd row stride used
    __shared__ unsigned long long E[CAP * CWS];
    __shared__ unsigned long long P[2 * CWS];
    __shared__ uint32_t ids[CAP];
    __shared__ uint32_t tuc[CAP];
    __shared__ int32_t hkey[2 * CAP];
    __shared__ int16_t hval[2 * CAP];
    __shared__ uint32_t exc[TL_EXC];
    __shared__ int32_t nexc;
    S.E = E; S.P = P; S.ids = ids; S.tuc = tuc; S.hkey = hkey; S.hval = hval; S.exc = exc; S.nexc = &nexc;
    S.W = CWS;
  }
  for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
    const int32_t u = list[it];
    const int64_t ub = R.roff[u] + R.rlow[u];
    const int32_t dp = (int32_t)(R.roff[u + 1] - ub);
    if (dp <= lo_dp || (CAP != 0 && dp > CAP)) continue;
    const int g = A.gid[u];
    if (g != cur_g) {
      if (cur_g >= 0) flush2(A.sig, cur_g, SG_K4, kb_, ka_);
      cur_g = g;
    }
    if constexpr (CAP != 0) S.W = ((dp + 63) / 64) | 1;  // odd row stride: rows spread over LDS banks
    tri_large_vertex(A, S, u, ub, dp, kb_, ka_);
  }
  if (cur_g >= 0) flush2(A.sig, cur_g, SG_K4, kb_, ka_);
}

constexpr int TL_MID = 256;
constexpr int TL_MAX = 1024;

// ------------------------------------------------------------ edge pass
// After all triangles, per upper entry u -> w present in version x, with
// t = t_x(u, w) and d = d_x:
//   S2  += (d_u - 1)(d_w - 1)      DIA += C(t, 2)
//   T3  += t                        (= 3 T)
//   PAW2 += t (d_u + d_w - 4)       (= 2 N_paw: a triangle on the edge plus a
//                                    pendant edge at one of its ends)
constexpr int EP_RUN = 128;

__global__ __launch_bounds__(256) void k_edge_pass(CountArgs A) {
  const RegionDev& R = A.R;
  const int64_t E = (int64_t)A.c[C_ER];
  int cur_g = -1;
  int64_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // s2 b/a, dia b/a, t3 b/a, paw2 b/a
  const int keys[4] = {SG_S2, SG_DIA, SG_T, SG_PAW};
  for (int64_t run = gtid(); run * EP_RUN < E; run += gstride()) {
    const int64_t p0 = run * EP_RUN;
    const int64_t p1 = p0 + EP_RUN < E ? p0 + EP_RUN : E;
    int64_t u = upper_bound_i64(R.roff, A.N, p0);
    int64_t nxt = R.roff[u + 1];
    int32_t dBu = R.dB[u], dAu = R.dA[u];
    for (int64_t p = p0; p < p1; ++p) {
      while (nxt <= p) { ++u; nxt = R.roff[u + 1]; dBu = R.dB[u]; dAu = R.dA[u]; }
      const uint32_t x = R.rcol[p];
      const uint32_t wv = x & GC_ID;
      if (wv <= (uint32_t)u) continue;
      const int g = A.gid[u];
      if (g != cur_g) {
        if (cur_g >= 0)
          for (int k = 0; k < 8; ++k) {
            if (acc[k]) atomicAdd(&A.sig[SIG_IDX(cur_g, k & 1, keys[k >> 1])], (unsigned long long)acc[k]);
            acc[k] = 0;
          }
        cur_g = g;
      }
      const unsigned long long tt = R.t[p];
      if (!(x & GC_F_NEW)) {
        const int64_t t = (int64_t)(tt & 0xFFFFFFFFull);
        const int32_t dw = R.dB[wv];
        acc[0] += (int64_t)(dBu - 1) * (dw - 1);
        acc[2] += c2(t);
        acc[4] += t;
        acc[6] += t * (dBu + dw - 4);
      }
      if (!(x & GC_F_DEL)) {
        const int64_t t = (int64_t)(tt >> 32);
        const int32_t dw = R.dA[wv];
        acc[1] += (int64_t)(dAu - 1) * (dw - 1);
        acc[3] += c2(t);
        acc[5] += t;
        acc[7] += t * (dAu + dw - 4);
      }
    }
  }
  // wave-uniform graph: one atomic per wave, else per lane
  const int g0 = __shfl(cur_g, 0);
  const bool uniform = __ballot(cur_g == g0 || cur_g < 0) == ~0ull && g0 >= 0;
  for (int k = 0; k < 8; ++k) {
    if (uniform) flush_sig(A.sig, g0, k & 1, keys[k >> 1], acc[k]);
    else if (cur_g >= 0 && acc[k]) atomicAdd(&A.sig[SIG_IDX(cur_g, k & 1, keys[k >> 1])], (unsigned long long)acc[k]);
  }
}

// ------------------------------------------------------------ 4-cycles
// Segment of the wedges through u for apex v: entries of row u below v.
__device__ __forceinline__ void c4_segment(const RegionDev& R, uint32_t v, uint32_t u, int64_t& sb, int32_t& sl) {
  sb = R.roff[u];
  const int32_t L = (int32_t)(R.roff[u + 1] - sb);
  sl = lower_bound_id(R.rcol + sb, L, v);
}

// Wave-flattened walk over the wedges (v, u, w) for the lower neighbours
// u in positions [g0, g0 + 64) of row v; calls f(w, add_b, add_a).
template <class F>
__device__ __forceinline__ void c4_group(const RegionDev& R, uint32_t v, int64_t rb, int32_t nlow, int32_t g0, F f) {
  const int l = lane_id();
  const int32_t q = g0 + l;
  int64_t sb = 0;
  int32_t sl = 0;
  uint32_t fvu = 0;
  if (q < nlow) {
    const uint32_t x = R.rcol[rb + q];
    fvu = x & GC_FLAGS;
    c4_segment(R, v, x & GC_ID, sb, sl);
  }
  const int32_t incl = wave_incl_scan32(sl);
  const int32_t tot = __shfl(incl, 63);
  const int32_t excl = incl - sl;
  for (int32_t base = 0; base < tot; base += 64) {
    const int32_t idx = base + l;
    const int s = seg_of(excl, idx);
    const int64_t sbs = __shfl(sb, s);
    const int32_t exs = __shfl(excl, s);
    const uint32_t fs = __shfl(fvu, s);
    if (idx < tot) {
      const uint32_t y = R.rcol[sbs + (idx - exs)];
      const uint32_t ab = fs | (y & GC_FLAGS);
      const uint32_t xb = !(ab & GC_F_NEW), xa = !(ab & GC_F_DEL);
      if (xb | xa) f(y & GC_ID, xb, xa);
    }
  }
}

constexpr int C4S_SLOTS = 512;
constexpr int C4S_WAVES = 4;

__global__ __launch_bounds__(256) void k_c4_small(CountArgs A) {
  __shared__ int32_t hkey[C4S_WAVES][C4S_SLOTS];
  __shared__ uint32_t hcnt[C4S_WAVES][C4S_SLOTS];
  const int w = threadIdx.x >> 6, l = lane_id();
  const RegionDev& R = A.R;
  const int64_t n = (int64_t)A.c[C_LIST0 + L_C4_S];
  const int32_t* list = A.lists + L_C4_S * A.list_stride;
  int cur_g = -1;
  int64_t cb_ = 0, ca_ = 0;
  for (int s = l; s < C4S_SLOTS; s += 64) { hkey[w][s] = -1; hcnt[w][s] = 0; }
  wave_sync();
  for (int64_t it = (int64_t)blockIdx.x * C4S_WAVES + w; it < n; it += (int64_t)gridDim.x * C4S_WAVES) {
    const int32_t v = list[it];
    const int g = A.gid[v];
    if (g != cur_g) { if (cur_g >= 0) flush2(A.sig, cur_g, SG_C4, cb_, ca_); cur_g = g; }
    const int64_t rb = R.roff[v];
    const int32_t nlow = R.rlow[v];
    int32_t* hk = hkey[w];
    uint32_t* hc = hcnt[w];
    for (int32_t g0 = 0; g0 < nlow; g0 += 64)
      c4_group(R, (uint32_t)v, rb, nlow, g0, [&](uint32_t wid, uint32_t xb, uint32_t xa) {
        hash_add<uint32_t>(hk, hc, C4S_SLOTS - 1, 23, wid, xb | (xa << 16));
      });
    wave_sync();
    for (int s = l; s < C4S_SLOTS; s += 64) {
      if (hk[s] != -1) {
        const uint32_t c = hc[s];
        cb_ += c2(c & 0xFFFFu);
        ca_ += c2(c >> 16);
        hk[s] = -1; hc[s] = 0;
      }
    }
    wave_sync();
  }
  if (cur_g >= 0) flush2(A.sig, cur_g, SG_C4, cb_, ca_);
}

constexpr int C4M_SLOTS = 8192;

__global__ __launch_bounds__(256) void k_c4_mid(CountArgs A) {
  __shared__ int32_t hkey[C4M_SLOTS];
  __shared__ uint32_t hcnt[C4M_SLOTS];
  const int w = threadIdx.x >> 6;
  const RegionDev& R = A.R;
  const int64_t n = (int64_t)A.c[C_LIST0 + L_C4_M];
  const int32_t* list = A.lists + L_C4_M * A.list_stride;
  int cur_g = -1;
  int64_t cb_ = 0, ca_ = 0;
  for (int s = threadIdx.x; s < C4M_SLOTS; s += blockDim.x) { hkey[s] = -1; hcnt[s] = 0; }
  __syncthreads();
  for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
    const int32_t v = list[it];
    const int g = A.gid[v];
    if (g != cur_g) { if (cur_g >= 0) flush2(A.sig, cur_g, SG_C4, cb_, ca_); cur_g = g; }
    const int64_t rb = R.roff[v];
    const int32_t nlow = R.rlow[v];
    for (int32_t g0 = w * 64; g0 < nlow; g0 += 64 * 4)
      c4_group(R, (uint32_t)v, rb, nlow, g0, [&](uint32_t wid, uint32_t xb, uint32_t xa) {
        hash_add<uint32_t>(hkey, hcnt, C4M_SLOTS - 1, 19, wid, xb | (xa << 16));
      });
    __syncthreads();
    for (int s = threadIdx.x; s < C4M_SLOTS; s += blockDim.x) {
      if (hkey[s] != -1) {
        const uint32_t c = hcnt[s];
        cb_ += c2(c & 0xFFFFu);
        ca_ += c2(c >> 16);
        hkey[s] = -1; hcnt[s] = 0;
      }
    }
    __syncthreads();
  }
  if (cur_g >= 0) flush2(A.sig, cur_g, SG_C4, cb_, ca_);
}

// Large tier: one workgroup per hub v at a time, hubs in decreasing order of
// wedge work.  The opposite vertices w < v are taken in windows of ids from
// v downwards; a window with enough hits gets dense LDS counters (16-bit
// halves while c(v, w) <= 65535 can be guaranteed, which doubles the window).
// Hits concentrate just below v because ids are a degree order and a wedge
// reaches w with odds growing with deg w.  Once a window is sparse, all
// wedges below it go to dense counters in global memory (one array per
// resident workgroup, with a touched list).  Each lower neighbour u keeps a
// cursor in its row: one binary search for v, then a short backward gallop
// per window, so rows are read about once.
constexpr int C4W_WIN = 16384;
constexpr int C4W_T = 1024;

struct C4Chunk {
  int64_t sb[C4W_T];
  int32_t pre[C4W_T + 1];
  uint32_t fl[C4W_T];
  int32_t wsum[C4W_T / 64];
  long long red[C4W_T / 64][2];
};

// first p in [0, c) with id(row[p]) >= lo, rows sorted, id(row[c-1]) < v
__device__ __forceinline__ int32_t gallop_down(const uint32_t* row, int32_t c, uint32_t lo) {
  if (c == 0 || (row[c - 1] & GC_ID) < lo) return c;
  int32_t k = 1;
  while (c - 1 - k >= 0 && (row[c - 1 - k] & GC_ID) >= lo) k <<= 1;
  const int32_t a = c - 1 - k > 0 ? c - 1 - k : 0;   // row[a] < lo or a == 0
  const int32_t z = c - 1 - (k >> 1);                 // row[z] >= lo
  return a + lower_bound_id(row + a, z - a + 1, lo);
}

// block sum of two values (all threads call; result valid in every thread)
__device__ __forceinline__ void block_sum2(C4Chunk& C, long long& x, long long& y) {
  const int t = threadIdx.x, wv = t >> 6;
  x = wave_sum64(x); y = wave_sum64(y);
  if (lane_id() == 0) { C.red[wv][0] = x; C.red[wv][1] = y; }
  __syncthreads();
  x = 0; y = 0;
  for (int k = 0; k < C4W_T / 64; ++k) { x += C.red[k][0]; y += C.red[k][1]; }
  __syncthreads();
}

// Walk the wedges (v, u_q, w) for q in [0, nlow) with w in row u_q at
// positions [urow[q] + p0(q), urow[q] + p1(q)); f(w, add_b, add_a).
// Short slices (the common case: u_q has few entries in the id range) are
// walked by their own thread; long ones are spread over the whole block
// with a scan of their lengths and a binary search per element.
constexpr int32_t C4W_SHORT = 8;

template <class P0, class P1, class F>
__device__ __forceinline__ void c4_block_walk(const RegionDev& R, int64_t rb, int32_t nlow, const int64_t* urow,
                                              P0 p0f, P1 p1f, C4Chunk& C, F f) {
  const int t = threadIdx.x, l = lane_id(), wv = t >> 6;
  for (int32_t c0 = 0; c0 < nlow; c0 += C4W_T) {
    const int32_t q = c0 + t;
    int32_t sl = 0;
    if (q < nlow) {
      const int32_t p0 = p0f(q), p1 = p1f(q);
      const int64_t sb = urow[q] + p0;
      const uint32_t fl = R.rcol[rb + q] & GC_FLAGS;
      if (p1 - p0 <= C4W_SHORT) {
        for (int64_t p = sb; p < sb + (p1 - p0); ++p) {
          const uint32_t y = R.rcol[p];
          const uint32_t ab = fl | (y & GC_FLAGS);
          const uint32_t xb = !(ab & GC_F_NEW), xa = !(ab & GC_F_DEL);
          if (xb | xa) f(y & GC_ID, xb, xa);
        }
      } else {
        C.sb[t] = sb;
        C.fl[t] = fl;
        sl = p1 - p0;
      }
    }
    // long slices: block-wide flattened walk (skipped when there are none)
    const int32_t inc = wave_incl_scan32(sl);
    if (l == 63) C.wsum[wv] = inc;
    __syncthreads();
    int32_t before = 0, tot = 0;
    for (int k = 0; k < C4W_T / 64; ++k) { if (k < wv) before += C.wsum[k]; tot += C.wsum[k]; }
    if (tot > 0) {
      C.pre[t] = before + inc - sl;
      if (t == C4W_T - 1) C.pre[C4W_T] = before + inc;
      __syncthreads();
      for (int32_t base = 0; base < tot; base += C4W_T) {
        const int32_t idx = base + t;
        if (idx < tot) {
          int32_t a = 0, z = C4W_T;  // largest a with pre[a] <= idx
          while (z - a > 1) { const int32_t m = (a + z) >> 1; if (C.pre[m] <= idx) a = m; else z = m; }
          const uint32_t y = R.rcol[C.sb[a] + (idx - C.pre[a])];
          const uint32_t ab = C.fl[a] | (y & GC_FLAGS);
          const uint32_t xb = !(ab & GC_F_NEW), xa = !(ab & GC_F_DEL);
          if (xb | xa) f(y & GC_ID, xb, xa);
        }
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(C4W_T) void k_c4_large(CountArgs A, unsigned long long* qhead) {
  __shared__ unsigned long long win[C4W_WIN];
  __shared__ C4Chunk C;
  __shared__ int64_t s_item;
  __shared__ int32_t s_nt;
  const RegionDev& R = A.R;
  const int64_t n = (int64_t)A.c[C_LIST0 + L_C4_L];
  const int32_t* list = A.lists + L_C4_L * A.list_stride;
  unsigned long long* cnt = A.c4_dense + (int64_t)blockIdx.x * A.N;
  int32_t* touch = A.c4_touch + (int64_t)blockIdx.x * A.N;
  int64_t* urow = A.c4_cur + (int64_t)blockIdx.x * 2 * A.c4_maxlow;
  int32_t* ucur = (int32_t*)(urow + A.c4_maxlow);
  int32_t* unext = ucur + A.c4_maxlow;
  const int t = threadIdx.x;
  int cur_g = -1;
  int64_t cb_ = 0, ca_ = 0, tail_ = 0;
  while (true) {
    __syncthreads();  // every thread has read the previous item before it is replaced
    if (t == 0) { s_item = (int64_t)atomicAdd(qhead, 1ull); s_nt = 0; }
    __syncthreads();
    const int64_t item = s_item;
    if (item >= n) break;
    const int32_t v = list[item];
    const int g = A.gid[v];
    if (g != cur_g) { if (cur_g >= 0) flush2(A.sig, cur_g, SG_C4, cb_, ca_); cur_g = g; }
    const int64_t rb = R.roff[v];
    const int32_t nlow = R.rlow[v];
    // c(v, w) <= nlow: 16-bit halves suffice up to 65535 lower neighbours
    const bool narrow = nlow <= A.c4_narrow_max;
    const int64_t ws = narrow ? 2 * (int64_t)A.c4_win : (int64_t)A.c4_win;
    for (int32_t q = t; q < nlow; q += C4W_T) {
      urow[q] = R.roff[R.rcol[rb + q] & GC_ID];
      ucur[q] = R.vpos[rb + q];
    }
    __syncthreads();
    int64_t hi = v;
    while (hi > 0) {
      const uint32_t lo = (uint32_t)(hi - ws > 0 ? hi - ws : 0);
      long long wtot = 0, rest = 0;
      for (int32_t q = t; q < nlow; q += C4W_T) {
        const int32_t c = ucur[q];
        const int32_t p0 = gallop_down(R.rcol + urow[q], c, lo);
        unext[q] = p0;
        wtot += c - p0;
        rest += p0;
      }
      block_sum2(C, wtot, rest);
      if (wtot >= A.c4_dense_min) {
        for (int s = t; s < A.c4_win; s += C4W_T) win[s] = 0ull;
        __syncthreads();
        if (narrow) {
          uint32_t* w32 = (uint32_t*)win;
          c4_block_walk(R, rb, nlow, urow, [&](int32_t q) { return unext[q]; }, [&](int32_t q) { return ucur[q]; }, C,
                        [&](uint32_t wid, uint32_t xb, uint32_t xa) { atomicAdd(&w32[wid - lo], xb | (xa << 16)); });
          for (int s = t; s < 2 * A.c4_win; s += C4W_T) {
            const uint32_t c = w32[s];
            if (c) { cb_ += c2((int64_t)(c & 0xFFFFu)); ca_ += c2((int64_t)(c >> 16)); }
          }
        } else {
          c4_block_walk(R, rb, nlow, urow, [&](int32_t q) { return unext[q]; }, [&](int32_t q) { return ucur[q]; }, C,
                        [&](uint32_t wid, uint32_t xb, uint32_t xa) { atomicAdd(&win[wid - lo], pack2(xb, xa)); });
          for (int s = t; s < A.c4_win; s += C4W_T) {
            const unsigned long long c = win[s];
            if (c) { cb_ += c2((int64_t)(c & 0xFFFFFFFFull)); ca_ += c2((int64_t)(c >> 32)); }
          }
        }
        for (int32_t q = t; q < nlow; q += C4W_T) ucur[q] = unext[q];
        __syncthreads();
        hi = lo;
        if (rest == 0) break;
      } else {
        // sparse from here down: every remaining wedge in global memory
        c4_block_walk(R, rb, nlow, urow, [&](int32_t) { return 0; }, [&](int32_t q) { return ucur[q]; }, C,
                      [&](uint32_t wid, uint32_t xb, uint32_t xa) {
                        ++tail_;
                        const unsigned long long old = atomicAdd(&cnt[wid], pack2(xb, xa));
                        if (old == 0ull) touch[atomicAdd(&s_nt, 1)] = (int32_t)wid;
                      });
        const int32_t nt = s_nt;
        for (int32_t q = t; q < nt; q += C4W_T) {
          const int32_t wid = touch[q];
          const unsigned long long c = cnt[wid];
          cnt[wid] = 0ull;
          cb_ += c2((int64_t)(c & 0xFFFFFFFFull));
          ca_ += c2((int64_t)(c >> 32));
        }
        __syncthreads();
        break;
      }
    }
  }
  if (cur_g >= 0) flush2(A.sig, cur_g, SG_C4, cb_, ca_);
  tail_ = wave_sum64(tail_);
  if (lane_id() == 0 && tail_) atomicAdd(&A.bstats[BS_TRIPROBE], (unsigned long long)tail_);
}

// hubs of the large tier in decreasing order of wedge work
__global__ void k_c4_order(const unsigned long long* sorted, const unsigned long long* c, int32_t* list) {
  const int64_t n = (int64_t)c[C_LIST0 + L_C4_L];
  for (int64_t i = gtid(); i < n; i += gstride()) list[i] = (int32_t)(sorted[i] & 0xFFFFFFFFull);
}

// --------------------------------------------------------------- combine
// C' = C_a - C_b on the six connected classes (Alg. 2), through the
// non-induced counts of each version and the triangular relation between
// non-induced and induced counts (copies of pattern X inside class Y).
__global__ void k_combine(const unsigned long long* sig, long long* state, int32_t k) {
  const int64_t g = gtid();
  if (g >= k) return;
  int64_t N[2][6], T[2], W[2], D1[2];
  int bad = 0;
  for (int x = 0; x < 2; ++x) {
    const unsigned long long* s = sig + SIG_IDX(g, x, 0);
    const int64_t t3 = (int64_t)s[SG_T], paw2 = (int64_t)s[SG_PAW];
    bad |= (t3 % 3 != 0) | (paw2 % 2 != 0);
    const int64_t t = t3 / 3;
    N[x][0] = (int64_t)s[SG_S2] - 3 * t;      // 3-paths
    N[x][1] = (int64_t)s[SG_S1];              // 3-stars
    N[x][2] = (int64_t)s[SG_C4];              // 4-cycles
    N[x][3] = paw2 / 2;                       // paws
    N[x][4] = (int64_t)s[SG_DIA];             // diamonds
    N[x][5] = (int64_t)s[SG_K4];              // 4-cliques
    T[x] = t; W[x] = (int64_t)s[SG_W]; D1[x] = (int64_t)s[SG_D1];
    bad |= (D1[x] % 2 != 0);
  }
  int64_t d[6];
  for (int c = 0; c < 6; ++c) d[c] = N[1][c] - N[0][c];
  int64_t I[6];
  I[5] = d[5];
  I[4] = d[4] - 6 * I[5];
  I[3] = d[3] - 4 * I[4] - 12 * I[5];
  I[2] = d[2] - I[4] - 3 * I[5];
  I[0] = d[0] - 2 * I[3] - 4 * I[2] - 6 * I[4] - 12 * I[5];
  I[1] = d[1] - I[3] - 2 * I[4] - 4 * I[5];
  long long* st = state + g * ST_STRIDE;
  for (int c = 0; c < 6; ++c) st[ST_F0 + c] += I[c];
  st[ST_T] += T[1] - T[0];
  st[ST_W] += W[1] - W[0];
  st[ST_M] += (D1[1] - D1[0]) / 2;
  if (bad) st[ST_ERR] += 1;
}

inline unsigned cap_grid(int64_t want, unsigned cap) {
  if (want < 1) want = 1;
  return (unsigned)(want > cap ? cap : want);
}

}  // namespace

int32_t c4_window_max() { return C4W_WIN; }
int64_t tri_scratch_words64(int64_t cap) { return tri_slot_words64(cap); }
int32_t tri_lds_max() { return TL_MAX; }

void launch_count(const CountArgs& A, const unsigned long long* hc, hipStream_t s, hipEvent_t* ev) {
  const int64_t E = (int64_t)hc[C_ER];
  if (ev) (void)hipEventRecord(ev[0], s);
  fill_u64(A.R.t, 0ull, E, s);
  const int64_t nts = (int64_t)hc[C_LIST0 + L_TRI_S], ntl = (int64_t)hc[C_LIST0 + L_TRI_L];
  if (nts) hipLaunchKernelGGL(k_tri_small, dim3(cap_grid((nts + 3) / 4, 8192)), dim3(256), 0, s, A);
  if (ntl) {
    hipLaunchKernelGGL((k_tri_large<TL_MID, 256>), dim3(cap_grid(ntl, 4096)), dim3(256), 0, s, A, 64);
    if ((int64_t)hc[C_MAXDP] > TL_MID)
      hipLaunchKernelGGL((k_tri_large<TL_MAX, 512>), dim3(cap_grid(ntl, 1024)), dim3(512), 0, s, A, TL_MID);
    if ((int64_t)hc[C_MAXDP] > TL_MAX)
      hipLaunchKernelGGL((k_tri_large<0, 256>), dim3(cap_grid(ntl, (unsigned)A.tri_slots)), dim3(256), 0, s, A, TL_MAX);
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  if (E) hipLaunchKernelGGL(k_edge_pass, dim3(cap_grid((E / EP_RUN + 255) / 256, 8192)), dim3(256), 0, s, A);
  if (ev) (void)hipEventRecord(ev[2], s);
  const int64_t ncs = (int64_t)hc[C_LIST0 + L_C4_S], ncm = (int64_t)hc[C_LIST0 + L_C4_M],
                ncl = (int64_t)hc[C_LIST0 + L_C4_L];
  if (ncs) hipLaunchKernelGGL(k_c4_small, dim3(cap_grid((ncs + 3) / 4, 8192)), dim3(256), 0, s, A);
  if (ev) (void)hipEventRecord(ev[3], s);
  if (ncm) hipLaunchKernelGGL(k_c4_mid, dim3(cap_grid(ncm, 4096)), dim3(256), 0, s, A);
  if (ev) (void)hipEventRecord(ev[4], s);
  if (ncl) {
    // order the hubs by decreasing wedge work (keys written by the per-vertex pass)
    unsigned long long* sk = radix_sort_u64(A.c4_keys, A.c4_keys_alt, A.sort_tmp, ncl, A.c + C_LIST0 + L_C4_L, 64, s);
    hipLaunchKernelGGL(k_c4_order, dim3(cap_grid((ncl + 255) / 256, 1024)), dim3(256), 0, s, sk, A.c,
                       (int32_t*)(A.lists + L_C4_L * A.list_stride));
    hipLaunchKernelGGL(k_c4_large, dim3(cap_grid(ncl, (unsigned)A.slots)), dim3(C4W_T), 0, s, A,
                       (unsigned long long*)(A.c + C_QHEAD));
  }
  if (ev) (void)hipEventRecord(ev[5], s);
}

void launch_combine(const unsigned long long* sig, long long* state, int32_t k, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3((k + 63) / 64), dim3(64), 0, s, sig, state, k);
}
