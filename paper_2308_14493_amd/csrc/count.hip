// Counting kernels: the local static counter applied to the region, fused
// over the versions of the pass (Alg. 2 counts G_b and G_a and adds
// C_a - C_b; a pass over several queued batches counts every intermediate
// graph as well).  Every structure is enumerated once in the union view and
// the versions it exists in are read off the flags of its entries.  Kernels
// are instantiated for NV = 2 versions (one batch) and NV = 4 (up to three
// batches of one graph).
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
//   tri  L: larger out-degree, one workgroup per vertex, LDS hash; tiers of
//           out-degree <= 128, 256, 512, 1024, 1280, and global-memory
//           scratch above
//   c4   S / M: wedge bound <= 256 / <= 4096, LDS hash per wave / workgroup
//   c4   L: one workgroup per vertex, windows of dense counters in LDS,
//           then dense counters in global memory
#include "gc_kernels.h"

#include <type_traits>

namespace {

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

__device__ __forceinline__ uint32_t hash32(uint32_t x) { return x * 2654435761u; }

__device__ __forceinline__ int32_t ld_relaxed(int32_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }

// Lookups in two steps so that the lookups of several entries overlap:
// read() loads the first two slots of the key's run (no branch between the
// loads and their use), pos() picks the key's position from them, going on
// in a loop only for longer runs (rare at load factor <= 1/2), and val()
// reads the 32-bit value of a position.
struct HashLook {
  const int32_t* keys;
  const uint32_t* vals;
  uint32_t mask;
  int shift;
  struct Two { uint32_t h; int32_t k0, k1; };
  __device__ __forceinline__ Two read(uint32_t key) const {
    const uint32_t h = hash32(key) >> shift;
    return Two{h, keys[h], keys[(h + 1) & mask]};
  }
  __device__ __forceinline__ int pos(const Two& t, uint32_t key) const {
    const int32_t k = (int32_t)key;
    int r = t.k0 == k ? (int)t.h : (t.k1 == k ? (int)((t.h + 1) & mask) : -1);
    if (r < 0 && t.k0 != -1 && t.k1 != -1) {
      for (uint32_t q = (t.h + 2) & mask;; q = (q + 1) & mask) {
        const int32_t kq = keys[q];
        if (kq == k) { r = (int)q; break; }
        if (kq == -1) break;
      }
    }
    return r;
  }
  __device__ __forceinline__ uint32_t val(int p) const { return vals[p]; }
  __device__ __forceinline__ int find(uint32_t key) const { return pos(read(key), key); }  // position or -1
};

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

__device__ __forceinline__ int32_t rdl32(int32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

// Vertices of a per-wave tier in chunks of up to QV_CHUNK (as many as the
// list holds per wave of the grid, so that a short list still uses every
// wave): a wave's first chunk is its own index (no atomic: waves without one
// leave at once), later ones come from a shared counter counting on from the
// grid's wave count, so that the waves that drew light vertices take more
// than a fixed stride would give them.  Returns the same chunk on every lane.
constexpr int64_t QV_CHUNK = 16;
__device__ __forceinline__ int64_t qv_chunk(int64_t n, int64_t nwaves) {
  return max((int64_t)1, min(QV_CHUNK, n / max(nwaves, (int64_t)1)));
}
__device__ __forceinline__ int64_t wave_next_chunk(const unsigned long long* ctr_, int64_t nwaves) {
  unsigned long long c = 0;
  if ((__lane_id()) == 0) c = atomicAdd((unsigned long long*)ctr_, 1ull);
  return nwaves + (int64_t)__shfl(c, 0);
}
__device__ __forceinline__ int64_t rdl64(int64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Walk the lists of a wave's lanes (lane l: positions [sb, sb + sl) of the
// entry array col, with a 32-bit payload pl) calling f(list lane, position,
// payload of that lane, entry).  Lists of at least WALK_LONG entries go one
// at a time through the whole wave (consecutive lanes read consecutive
// entries, D loads in flight per lane; the list's lane is read with scalar
// reads); the others are flattened over the lanes with a segment search per
// step.  Most entries sit in long lists, which then cost no cross-lane
// traffic.  All lanes must call it.
constexpr int32_t WALK_LONG = 32;

template <int D = 4, class F>
__device__ __forceinline__ void wave_walk(const uint32_t* col, int64_t sb, int32_t sl, uint32_t pl, F f) {
  const int l = lane_id();
  const bool lng = sl >= WALK_LONG;
  uint64_t lm = __ballot(lng);
  while (lm) {
    const int s = __builtin_ctzll(lm);
    lm &= lm - 1;
    const int64_t b = rdl64(sb, s);
    const int32_t n = rdl32(sl, s);
    const uint32_t ps = (uint32_t)rdl32((int32_t)pl, s);
    for (int32_t k = l; k < n; k += 64 * D) {
      uint32_t y[D];
#pragma unroll
      for (int u = 0; u < D; ++u) y[u] = k + 64 * u < n ? col[b + k + 64 * u] : 0u;
#pragma unroll
      for (int u = 0; u < D; ++u)
        if (k + 64 * u < n) f(s, b + k + 64 * u, ps, y[u]);
    }
  }
  const int32_t ss = lng ? 0 : sl;
  const int32_t incl = wave_incl_scan32(ss);
  const int32_t tot = __shfl(incl, 63);
  const int32_t excl = incl - ss;
  for (int32_t base = 0; base < tot; base += 64) {
    const int32_t idx = base + l;
    const int s = seg_of(excl, idx);
    const int64_t sbs = __shfl(sb, s);
    const int32_t exs = __shfl(excl, s);
    const uint32_t ps = (uint32_t)__shfl((int32_t)pl, s);
    if (idx < tot) {
      const int64_t pos = sbs + (idx - exs);
      f(s, pos, ps, col[pos]);
    }
  }
}

__device__ __forceinline__ unsigned long long wave_or64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) v |= (unsigned long long)__shfl_xor((long long)v, o);
  return v;
}
template <class T>
__device__ __forceinline__ T wave_add(T v) {
  for (int o = 32; o > 0; o >>= 1) {
    if constexpr (sizeof(T) == 8) v += (T)__shfl_xor((long long)v, o);
    else v += (T)__shfl_xor((int)v, o);
  }
  return v;
}

// The long lists of a wave's lanes (at least WALK_LONG entries), one at a
// time through the whole wave: begin(s) -> per-list state; every entry y is
// looked up (hl, key y & GC_ID) and f(state, s, pos, y, value) is called for
// the keys found; end(state, s).  Each lane loads WALK_DEPTH entries (indexes
// clamped to the list, so the loads need no branch), reads the hash slots of
// all of them before picking any and their values before handling any, so
// their memory and LDS accesses overlap.  The list's lane s is uniform, so
// per-list work can be hoisted into begin/end.
constexpr int WALK_DEPTH = 3;  // entries per lane loaded and looked up together (more waves fit than with 4)

template <class B, class F, class E>
__device__ __forceinline__ void wave_walk_long(const uint32_t* col, int64_t sb, int32_t sl, B begin,
                                               const HashLook& hl, F f, E end) {
  const int l = lane_id();
  uint64_t lm = __ballot(sl >= WALK_LONG);
  while (lm) {
    const int s = __builtin_ctzll(lm);
    lm &= lm - 1;
    const int64_t b = rdl64(sb, s);
    const int32_t n = rdl32(sl, s);
    auto st = begin(s);
    for (int32_t k = l; k < n; k += 64 * WALK_DEPTH) {
      uint32_t y[WALK_DEPTH], jv[WALK_DEPTH];
      HashLook::Two tw[WALK_DEPTH];
      int hp[WALK_DEPTH];
#pragma unroll
      for (int u = 0; u < WALK_DEPTH; ++u) y[u] = col[b + min(k + 64 * u, n - 1)];
#pragma unroll
      for (int u = 0; u < WALK_DEPTH; ++u) tw[u] = hl.read(y[u] & GC_ID);
#pragma unroll
      for (int u = 0; u < WALK_DEPTH; ++u) {
        const int p = hl.pos(tw[u], y[u] & GC_ID);
        hp[u] = k + 64 * u < n ? p : -1;
      }
#pragma unroll
      for (int u = 0; u < WALK_DEPTH; ++u) jv[u] = hl.val(max(hp[u], 0));
#pragma unroll
      for (int u = 0; u < WALK_DEPTH; ++u)
        if (hp[u] >= 0) f(st, s, b + k + 64 * u, y[u], jv[u]);
    }
    end(st, s);
  }
}

__device__ __forceinline__ unsigned long long pack2(uint32_t b, uint32_t a) {
  return (unsigned long long)b | ((unsigned long long)a << 32);
}

// Per-version counters packed in one word: NF fields of FB bits each.
template <int NF, int FB>
struct Fields {
  using T = typename std::conditional<(NF * FB <= 32), uint32_t, unsigned long long>::type;
  // 1 in field x for every bit x of pm
  __device__ static __forceinline__ T spread(uint32_t pm) {
    T r = 0;
#pragma unroll
    for (int x = 0; x < NF; ++x) r |= (T)((pm >> x) & 1u) << (FB * x);
    return r;
  }
  __device__ static __forceinline__ int64_t get(T c, int x) {
    return (int64_t)((c >> (FB * x)) & (T)((1ull << FB) - 1ull));
  }
};

// flush lane-private per-version sums of a wave whose lanes all work for graph g
template <int NV>
__device__ __forceinline__ void flushv(unsigned long long* sig, int g, int k, int64_t (&a)[NV]) {
#pragma unroll
  for (int x = 0; x < NV; ++x) {
    flush_sig(sig, g, x, k, a[x]);
    a[x] = 0;
  }
}

template <int NV>
__device__ __forceinline__ void zerov(int64_t (&a)[NV]) {
#pragma unroll
  for (int x = 0; x < NV; ++x) a[x] = 0;
}

// t of entry pos: one triangle (or c of them) present in the versions of pm
template <int NV>
__device__ __forceinline__ void t_add(const RegionDev& R, int64_t pos, uint32_t pm, uint32_t c = 1u) {
  if constexpr (NV == 2) {
    atomicAdd(&R.t[pos], pack2((pm & 1u) * c, ((pm >> 1) & 1u) * c));
  } else {
    if (pm == 0xFu) { atomicAdd(&R.t[pos], (unsigned long long)c); return; }
    if (pm & 3u) atomicAdd(&R.tp[2 * pos], pack2((pm & 1u) * c, ((pm >> 1) & 1u) * c));
    if (pm & 12u) atomicAdd(&R.tp[2 * pos + 1], pack2(((pm >> 2) & 1u) * c, ((pm >> 3) & 1u) * c));
  }
}

// t of entry pos: c[x] triangles in version x
template <int NV>
__device__ __forceinline__ void t_addv(const RegionDev& R, int64_t pos, const uint32_t (&c)[NV]) {
  if constexpr (NV == 2) {
    if (c[0] | c[1]) atomicAdd(&R.t[pos], pack2(c[0], c[1]));
  } else {
    const uint32_t m = min(min(c[0], c[1]), min(c[2], c[3]));
    if (m) atomicAdd(&R.t[pos], (unsigned long long)m);
    if ((c[0] - m) | (c[1] - m)) atomicAdd(&R.tp[2 * pos], pack2(c[0] - m, c[1] - m));
    if ((c[2] - m) | (c[3] - m)) atomicAdd(&R.tp[2 * pos + 1], pack2(c[2] - m, c[3] - m));
  }
}

template <int NV>
__device__ __forceinline__ void t_read(const RegionDev& R, int64_t pos, int64_t (&t)[NV]) {
  const unsigned long long a = R.t[pos];
  if constexpr (NV == 2) {
    t[0] = (int64_t)(a & 0xFFFFFFFFull);
    t[1] = (int64_t)(a >> 32);
  } else {
    const ulonglong2 p = *(const ulonglong2*)(R.tp + 2 * pos);
    t[0] = (int64_t)(a + (p.x & 0xFFFFFFFFull));
    t[1] = (int64_t)(a + (p.x >> 32));
    t[2] = (int64_t)(a + (p.y & 0xFFFFFFFFull));
    t[3] = (int64_t)(a + (p.y >> 32));
  }
}

template <int NV>
__device__ __forceinline__ void d_read(const RegionDev& R, int64_t v, int32_t (&d)[NV]) {
  if constexpr (NV == 2) {
    const int2 q = *(const int2*)(R.d + v * 2);
    d[0] = q.x; d[1] = q.y;
  } else {
    const int4 q = *(const int4*)(R.d + v * 4);
    d[0] = q.x; d[1] = q.y; d[2] = q.z; d[3] = q.w;
  }
}

__device__ __forceinline__ bool absent_in(uint32_t flags, int x) { return (flags >> (GC_VSHIFT + x)) & 1u; }

// ------------------------------------------------------ triangles, tier S
// One wave per vertex u with out-degree <= 64.  Bit matrices over the slots
// of N+(u): EU[i] has bit j (j > i) when v_i -> v_j is an edge of the union
// view, TU its transpose, and EX[x] / TX[x] the same for the edges absent
// from version x (only edges with flags land there).  A wave that met no
// flag at all counts version 0 once and copies it to the others.
constexpr int TS_WAVES = 4;

template <int NV>
__global__ __launch_bounds__(256) void k_tri_small(CountArgs A) {
  __shared__ int32_t hkey[TS_WAVES][256];  // load factor <= 1/4
  __shared__ uint32_t hval[TS_WAVES][256];  // slot | its flags
  __shared__ unsigned long long EU[TS_WAVES][64], TU[TS_WAVES][64];
  __shared__ unsigned long long EX[TS_WAVES][NV][64], TX[TS_WAVES][NV][64];
  __shared__ uint32_t dirty[TS_WAVES];
  const int w = threadIdx.x >> 6, l = lane_id();
  const RegionDev& R = A.R;
  const int64_t n = (int64_t)A.c[C_LIST0 + L_TRI_S];
  const int32_t* list = A.lists + L_TRI_S * A.list_stride;
  int cur_g = -1;
  int64_t kacc[NV];
  zerov<NV>(kacc);
  int64_t ent = 0;  // entries of N+(u) and of the lists probed (algorithmic reads)
  const int64_t nwv = (int64_t)gridDim.x * TS_WAVES, cq = qv_chunk(n, nwv);
  for (int64_t ch = (int64_t)blockIdx.x * TS_WAVES + w; ch * cq < n; ch = wave_next_chunk(A.c + C_QTS, nwv))
  for (int64_t it = ch * cq; it < min(n, (ch + 1) * cq); ++it) {
    const int32_t u = list[it];
    const int g = A.gid[u];
    if (g != cur_g) {
      if (cur_g >= 0) flushv<NV>(A.sig, cur_g, SG_K4, kacc);
      cur_g = g;
    }
    const int64_t ub = R.roff[u] + R.rlow[u];
    const int32_t dp = (int32_t)(R.roff[u + 1] - ub);
    uint32_t vi = 0, fi = 0;
    if (l < dp) { const uint32_t x = R.rcol[ub + l]; vi = x & GC_ID; fi = x & GC_FLAGS; }
#pragma unroll
    for (int q = 0; q < 4; ++q) hkey[w][l + 64 * q] = -1;
    EU[w][l] = 0; TU[w][l] = 0;
#pragma unroll
    for (int x = 0; x < NV; ++x) { EX[w][x][l] = 0; TX[w][x][l] = 0; }
    if (l == 0) dirty[w] = 0;
    wave_sync();
    if (l < dp) {
      uint32_t h = hash32(vi) >> 24;
      while (atomicCAS(&hkey[w][h], -1, (int32_t)vi) != -1) h = (h + 1) & 255u;
      hval[w][h] = (uint32_t)l | fi;
    }
    wave_sync();
    int64_t sb = 0;
    int32_t sl = 0;
    if (l < dp) { sb = R.roff[vi] + R.rlow[vi]; sl = (int32_t)(R.roff[vi + 1] - sb); ent += 1 + sl; }
    // one probe of list i: a hit (slot j with flags, jv) is the triangle
    // (u, v_i, v_j); row i's bits collect in ei (the caller writes them)
    const HashLook hl{hkey[w], hval[w], 255u, 24};
    auto hit = [&](int i, int64_t pos, uint32_t fs, uint32_t y, uint32_t jv, unsigned long long& ei) {
      const int j = (int)(jv & GC_ID);
      const uint32_t fy = y & GC_FLAGS;
      const unsigned long long bj = 1ull << j, bi = 1ull << i;
      ei |= bj;
      atomicOr(&TU[w][j], bi);
      if (fy) {
        dirty[w] = 1u;
#pragma unroll
        for (int x = 0; x < NV; ++x)
          if (absent_in(fy, x)) { atomicOr(&EX[w][x][i], bj); atomicOr(&TX[w][x][j], bi); }
      }
      const uint32_t pm = vpresent<NV>(fs | (jv & GC_FLAGS) | fy);
      if (pm) t_add<NV>(R, pos, pm);
    };
    struct LongState { int i; uint32_t fs; unsigned long long ei; };
    wave_walk_long(
        R.rcol, sb, sl,
        [&](int s) { return LongState{s, (uint32_t)rdl32((int32_t)fi, s), 0ull}; }, hl,
        [&](LongState& st, int, int64_t pos, uint32_t y, uint32_t jv) { hit(st.i, pos, st.fs, y, jv, st.ei); },
        [&](LongState& st, int) {
          const unsigned long long e = wave_or64(st.ei);
          if (lane_id() == 0 && e) atomicOr(&EU[w][st.i], e);
        });
    wave_walk(R.rcol, sb, sl >= WALK_LONG ? 0 : sl, fi, [&](int i, int64_t pos, uint32_t fs, uint32_t y) {
      const int p = hl.find(y & GC_ID);
      if (p < 0) return;
      unsigned long long ei = 0;
      hit(i, pos, fs, y, hl.val(p), ei);
      atomicOr(&EU[w][i], ei);
    });
    wave_sync();
    const bool clean = __ballot(l < dp && fi != 0) == 0ull && dirty[w] == 0u;
    uint64_t Px[NV];
#pragma unroll
    for (int x = 0; x < NV; ++x) Px[x] = __ballot(l < dp && !absent_in(fi, x));
    if (l < dp) {
      uint32_t tu[NV];
      int64_t kv[NV];
#pragma unroll
      for (int x = 0; x < NV; ++x) {
        tu[x] = 0;
        kv[x] = 0;
        if (x > 0 && clean) { tu[x] = tu[0]; kv[x] = kv[0]; continue; }
        if (!((Px[x] >> l) & 1ull)) continue;
        const unsigned long long e = EU[w][l] & ~EX[w][x][l] & Px[x];
        const unsigned long long tt = TU[w][l] & ~TX[w][x][l] & Px[x];
        tu[x] = (uint32_t)__popcll(e | tt);
        int64_t k4 = 0;
        for (unsigned long long m = e; m; m &= m - 1) {
          const int j = __builtin_ctzll(m);
          k4 += __popcll(e & EU[w][j] & ~EX[w][x][j] & Px[x]);
        }
        kv[x] = k4;
      }
#pragma unroll
      for (int x = 0; x < NV; ++x) kacc[x] += kv[x];
      t_addv<NV>(R, ub + l, tu);
    }
    wave_sync();
  }
  if (cur_g >= 0) flushv<NV>(A.sig, cur_g, SG_K4, kacc);
  ent = wave_sum64(ent);
  if (l == 0 && ent) atomicAdd(&A.bstats[BS_TRI_E], (unsigned long long)ent);
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
// with P_x the slots whose edge from u exists in version x (versions with
// equal P_x share one count).  Edges among N+(u) that are absent from some
// version are few; the triangles of E that contain such an edge absent from
// version x are removed from K4_x one by one (each once, at its first such
// edge in list order).  If the list overflows, the matrix is rebuilt per
// version instead.
constexpr int TL_EXC = 256;  // edges with flags tracked per vertex

// Words of the triangular bit matrix of n slots with W words per full row:
// row i keeps only words (i >> 6) .. W - 1 (its bits j > i).
__host__ __device__ __forceinline__ int64_t tri_words(int64_t n, int64_t W) {
  const int64_t b = n >> 6;
  return n * W - (32 * b * (b - 1) + (n - 64 * b) * b);
}

template <int NV>
struct TriL {
  using TU = typename Fields<NV, 16>::T;  // per-slot triangle counts, 16-bit field per version
  unsigned long long* E;    // triangular row bitsets, tri_words(dp, W) words
  // word w >= (i >> 6) of row i is erow(i)[w]
  __device__ __forceinline__ unsigned long long* erow(int32_t i) const {
    return E + tri_words(i, W) - (i >> 6);
  }
  unsigned long long* P;    // [NV][W] slot masks per version
  uint32_t* ids;            // [dp]
  int32_t* hkey;            // [H]
  uint32_t* hval;           // [H] slot | its flags
  int32_t hcap;             // slots of hkey / hval (a power of two)
  TU* tuc;                  // [dp]
  unsigned long long* exc;  // [TL_EXC] i << 32 | j << 4 | absence mask
  int32_t* nexc;            // [1]
  int32_t W;                // words per row
};

template <int NV>
__device__ __forceinline__ bool Ebit(const TriL<NV>& S, int32_t p, int32_t q) {  // edge between slots p != q
  if (p > q) { int32_t t = p; p = q; q = t; }
  return (S.erow(p)[q >> 6] >> (q & 63)) & 1ull;
}

__device__ __forceinline__ bool bit_of(const unsigned long long* m, int32_t k) { return (m[k >> 6] >> (k & 63)) & 1ull; }

// One wave: slots g0 + gs * l (lane l) of N+(u), their out-lists walked
// together.  The slots of a vertex are dealt to the waves of the block in
// turn, so every wave gets a share whatever the out-degree.  only = 0: union
// matrix plus all triangle bookkeeping; only = x+1: matrix of version x alone.
template <int NV>
__device__ __forceinline__ void tri_large_probe(const CountArgs& A, const TriL<NV>& S, uint32_t hmask, int shift,
                                                int32_t g0, int32_t gs, int32_t dp, int only, int64_t& ent) {
  const RegionDev& R = A.R;
  const int l = lane_id();
  const int32_t i0 = g0 + gs * l;
  int64_t sb = 0;
  int32_t sl = 0;
  uint32_t fi = 0;
  if (i0 < dp) {
    const uint32_t xi = S.ids[i0];
    const uint32_t v = xi & GC_ID;
    fi = xi & GC_FLAGS;
    sb = R.roff[v] + R.rlow[v];
    sl = (int32_t)(R.roff[v + 1] - sb);
    if (only == 0) ent += sl;
  }
  using TU = typename TriL<NV>::TU;
  // one probe of list i: a hit (slot j with flags, jv) is the triangle
  // (u, v_i, w_j); returns the increment of t(u, v_i), which the caller adds
  // to tuc[i]
  const HashLook hl{S.hkey, S.hval, hmask, shift};
  auto hit = [&](int32_t i, unsigned long long* Ei, uint32_t fs, int64_t pos, uint32_t y, uint32_t jv) -> TU {
    const int j = (int)(jv & GC_ID);
    const uint32_t fy = y & GC_FLAGS;
    if (only) {
      if (!absent_in(fy, only - 1)) atomicOr(&Ei[j >> 6], 1ull << (j & 63));
      return (TU)0;
    }
    atomicOr(&Ei[j >> 6], 1ull << (j & 63));
    if (fy) {
      const int32_t p = atomicAdd(S.nexc, 1);
      if (p < TL_EXC)
        S.exc[p] = ((unsigned long long)i << 32) | ((unsigned long long)j << 4) | (unsigned long long)(fy >> GC_VSHIFT);
    }
    const uint32_t pm = vpresent<NV>(fs | (jv & GC_FLAGS) | fy);
    if (!pm) return (TU)0;
    t_add<NV>(R, pos, pm);
    const TU add = Fields<NV, 16>::spread(pm);
    atomicAdd(&S.tuc[j], add);
    return add;
  };
  struct LongState { int32_t i; unsigned long long* Ei; uint32_t fs; TU acc; };
  wave_walk_long(
      R.rcol, sb, sl,
      [&](int s) { return LongState{g0 + gs * s, S.erow(g0 + gs * s), (uint32_t)rdl32((int32_t)fi, s), (TU)0}; }, hl,
      [&](LongState& st, int, int64_t pos, uint32_t y, uint32_t jv) { st.acc += hit(st.i, st.Ei, st.fs, pos, y, jv); },
      [&](LongState& st, int) {
        const TU tot = wave_add<TU>(st.acc);
        if (lane_id() == 0 && tot) atomicAdd(&S.tuc[st.i], tot);
      });
  wave_walk(R.rcol, sb, sl >= WALK_LONG ? 0 : sl, fi, [&](int s, int64_t pos, uint32_t fs, uint32_t y) {
    const int p = hl.find(y & GC_ID);
    if (p < 0) return;
    const int32_t i = g0 + gs * s;
    const TU add = hit(i, S.erow(i), fs, pos, y, hl.val(p));
    if (add) atomicAdd(&S.tuc[i], add);
  });
}

// sum over i in mask, j in E[i] & mask of |E[i] & E[j] & mask|  (one wave's rows)
template <int NV>
__device__ __forceinline__ int64_t k4_rows(const TriL<NV>& S, const unsigned long long* mask, int32_t dp, int nwaves) {
  const int w = threadIdx.x >> 6, l = lane_id();
  int64_t cnt = 0;
  for (int32_t i = w; i < dp; i += nwaves) {
    if (!bit_of(mask, i)) continue;
    const unsigned long long* Ei = S.erow(i);
    for (int32_t w0 = i >> 6; w0 < S.W; ++w0) {
      const unsigned long long m = Ei[w0] & mask[w0];
      if (!m) continue;
      if ((m >> l) & 1ull) {
        const int32_t j = w0 * 64 + l;
        const unsigned long long* Ej = S.erow(j);
        for (int32_t q = j >> 6; q < S.W; ++q) cnt += __popcll(Ei[q] & Ej[q] & mask[q]);
      }
    }
  }
  return cnt;
}

template <int NV>
__device__ void tri_large_vertex(const CountArgs& A, const TriL<NV>& S, int64_t ub, int32_t dp,
                                 int64_t (&kacc)[NV], int64_t& ent) {
  const RegionDev& R = A.R;
  const int w = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  const int32_t W = S.W;
  // load factor <= 1/8 where the table has room, else as low as it allows
  int H = 1;
  while (H < 8 * dp) H <<= 1;
  while (H > S.hcap) H >>= 1;
  const uint32_t hmask = (uint32_t)H - 1u;
  const int shift = 32 - log2i((uint32_t)H);
  for (int32_t k = threadIdx.x; k < dp; k += blockDim.x) { S.ids[k] = R.rcol[ub + k]; S.tuc[k] = 0; }
  for (int32_t k = threadIdx.x; k < H; k += blockDim.x) S.hkey[k] = -1;
  const int64_t ew = tri_words(dp, W);
  for (int64_t k = threadIdx.x; k < ew; k += blockDim.x) S.E[k] = 0ull;
  for (int32_t k = threadIdx.x; k < NV * W; k += blockDim.x) S.P[k] = 0ull;
  if (threadIdx.x == 0) *S.nexc = 0;
  __syncthreads();
  for (int32_t k = threadIdx.x; k < dp; k += blockDim.x) {
    const uint32_t x = S.ids[k];
    const uint32_t id = x & GC_ID;
    uint32_t h = hash32(id) >> shift;
    while (atomicCAS(&S.hkey[h], -1, (int32_t)id) != -1) h = (h + 1) & hmask;
    S.hval[h] = (uint32_t)k | (x & GC_FLAGS);
#pragma unroll
    for (int q = 0; q < NV; ++q)
      if (!absent_in(x, q)) atomicOr(&S.P[q * W + (k >> 6)], 1ull << (k & 63));
  }
  __syncthreads();
  if (threadIdx.x == 0) ent += dp;
  for (int32_t g0 = w; g0 < dp; g0 += nwaves * 64) tri_large_probe<NV>(A, S, hmask, shift, g0, nwaves, dp, 0, ent);
  __syncthreads();
  const int32_t ne = *S.nexc;
  if (ne <= TL_EXC) {
    // versions with the same slot mask share one count
    int64_t kv[NV];
#pragma unroll
    for (int x = 0; x < NV; ++x) {
      int same = -1;
      for (int y = 0; y < x && same < 0; ++y) {
        bool eq = true;
        for (int32_t q = 0; q < W && eq; ++q) eq = S.P[x * W + q] == S.P[y * W + q];
        if (eq) same = y;
      }
      if (same >= 0) {
#pragma unroll
        for (int y = 0; y < NV; ++y)
          if (y == same) kv[x] = kv[y];
      } else {
        kv[x] = k4_rows<NV>(S, S.P + x * W, dp, nwaves);
      }
    }
    // The exceptions by slot pair, in the probe hash table (not read again
    // for this vertex): key min << 16 | max, value the exception's index.
    // Pairs are unique (each found from its lower slot's list only).
    const bool keyed = dp <= 65536;
    if (keyed) {
      for (int32_t k = threadIdx.x; k < H; k += blockDim.x) S.hkey[k] = -1;
      __syncthreads();
      for (int32_t e = threadIdx.x; e < ne; e += blockDim.x) {
        const unsigned long long ex = S.exc[e];
        const uint32_t a = (uint32_t)(ex >> 32), b = (uint32_t)((ex >> 4) & 0xFFFFFFFull);
        const uint32_t key = (min(a, b) << 16) | max(a, b);
        uint32_t h = hash32(key) >> shift;
        while (atomicCAS(&S.hkey[h], -1, (int32_t)key) != -1) h = (h + 1) & hmask;
        S.hval[h] = (uint32_t)e;
      }
      __syncthreads();
    }
    // index of the exception on slot pair (a, b), or -1
    auto exc_of = [&](int32_t a, int32_t b) -> int32_t {
      const uint32_t key = ((uint32_t)min(a, b) << 16) | (uint32_t)max(a, b);
      uint32_t h = hash32(key) >> shift;
      for (;;) {
        const int32_t q = S.hkey[h];
        if (q == -1) return -1;
        if ((uint32_t)q == key) return (int32_t)S.hval[h];
        h = (h + 1) & hmask;
      }
    };
    // triangles of E (inside P_x) holding an edge absent from version x
    const int l = lane_id();
    for (int32_t e = w; e < ne; e += nwaves) {
      const unsigned long long ex = S.exc[e];
      const int32_t i = (int32_t)(ex >> 32), j = (int32_t)((ex >> 4) & 0xFFFFFFFull);
      const uint32_t am = (uint32_t)(ex & 0xFull);
#pragma unroll
      for (int x = 0; x < NV; ++x) {
        if (!((am >> x) & 1u)) continue;
        const unsigned long long* Px = S.P + x * W;
        if (!bit_of(Px, i) || !bit_of(Px, j)) continue;
        int64_t sub = 0;
        for (int32_t k = l; k < dp; k += 64) {
          if (k == i || k == j || !bit_of(Px, k)) continue;
          if (!Ebit<NV>(S, i, k) || !Ebit<NV>(S, j, k)) continue;
          // count once: skip if an earlier listed edge of this triangle is absent from x
          bool first = true;
          if (keyed) {
            const int32_t f1 = exc_of(i, k), f2 = exc_of(j, k);
            if (f1 >= 0 && f1 < e && ((S.exc[f1] >> x) & 1ull)) first = false;
            if (f2 >= 0 && f2 < e && ((S.exc[f2] >> x) & 1ull)) first = false;
          } else {
            for (int32_t f = 0; f < e && first; ++f) {
              const unsigned long long ef = S.exc[f];
              if (!((ef >> x) & 1ull)) continue;
              const int32_t fi = (int32_t)(ef >> 32), fj = (int32_t)((ef >> 4) & 0xFFFFFFFull);
              if ((fi == i && fj == k) || (fi == k && fj == i) || (fi == j && fj == k) || (fi == k && fj == j))
                first = false;
            }
          }
          sub += first;
        }
        kv[x] -= sub;
      }
    }
#pragma unroll
    for (int x = 0; x < NV; ++x) kacc[x] += kv[x];
  } else {
    // too many version-specific edges: rebuild E per version and count
    if (threadIdx.x == 0) atomicAdd(&A.bstats[BS_TRI_REBUILD], 1ull);
    for (int x = 0; x < NV; ++x) {
      __syncthreads();
      for (int64_t k = threadIdx.x; k < ew; k += blockDim.x) S.E[k] = 0ull;
      __syncthreads();
      for (int32_t g0 = w; g0 < dp; g0 += nwaves * 64) tri_large_probe<NV>(A, S, hmask, shift, g0, nwaves, dp, x + 1, ent);
      __syncthreads();
      const int64_t c = k4_rows<NV>(S, S.P + x * W, dp, nwaves);
#pragma unroll
      for (int y = 0; y < NV; ++y)
        if (y == x) kacc[y] += c;
    }
  }
  __syncthreads();
  for (int32_t k = threadIdx.x; k < dp; k += blockDim.x) {
    const typename TriL<NV>::TU c = S.tuc[k];
    if (c) {
      uint32_t cv[NV];
#pragma unroll
      for (int x = 0; x < NV; ++x) cv[x] = (uint32_t)Fields<NV, 16>::get(c, x);
      t_addv<NV>(R, ub + k, cv);
    }
  }
  __syncthreads();
}

// global-scratch slot layout (u64 words): E [tri_words(cap, W)] | P [NV*W] |
// tuc [cap] | exc [TL_EXC] | then u32 words: ids [cap] | hkey [4 cap] |
// hval [4 cap] | nexc [2]
template <int NV>
__host__ __device__ inline int64_t tri_slot_words64(int64_t cap) {
  const int64_t W = (cap + 63) / 64;
  return tri_words(cap, W) + NV * W + cap + TL_EXC + (cap + 4 * cap + 4 * cap + 2 + 1) / 2 + 8;
}

constexpr int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// The vertices of work list L (out-degree at most CAP; CAP = 0 selects the
// global-memory scratch), taken one at a time from the queue whose head is
// qhead.
template <int CAP, int THREADS, int NV>
__global__ __launch_bounds__(THREADS) void k_tri_large(CountArgs A, int L, unsigned long long* qhead) {
  const RegionDev& R = A.R;
  const int64_t n = (int64_t)A.c[C_LIST0 + L];
  const int32_t* list = A.lists + L * A.list_stride;
  __shared__ int64_t item_s;
  int cur_g = -1;
  int64_t kacc[NV];
  zerov<NV>(kacc);
  int64_t ent = 0;  // entries of N+(u) and of the lists probed (algorithmic reads)
  TriL<NV> S;
  using TU = typename TriL<NV>::TU;
  if constexpr (CAP == 0) {
    // slot layout for capacity tri_cap (no slot is touched while tri_cap == 0)
    const int64_t cap = A.tri_cap > 0 ? A.tri_cap : 1;
    const int64_t W = (cap + 63) / 64;
    unsigned long long* base = A.tri_scratch + (int64_t)blockIdx.x * tri_slot_words64<NV>(cap);
    S.W = (int32_t)W;
    S.E = base;
    S.P = base + tri_words(cap, W);
    S.tuc = (TU*)(S.P + NV * W);
    S.exc = S.P + NV * W + cap;
    uint32_t* u32 = (uint32_t*)(S.exc + TL_EXC);
    S.ids = u32;
    S.hkey = (int32_t*)(u32 + cap);
    S.hval = u32 + 5 * cap;
    S.nexc = (int32_t*)(u32 + 9 * cap);
    int32_t hc = 1;
    while (2 * hc <= 4 * cap) hc <<= 1;
    S.hcap = hc;
  } else {
    constexpr int CW = CAP / 64;
    constexpr int HC = CAP <= 1024 ? pow2_at_least(8 * CAP) : pow2_at_least(2 * CAP);
    __shared__ unsigned long long E[32 * CW * CW + 32 * CW];  // tri_words(CAP, CW)
    __shared__ unsigned long long P[NV * CW];
    __shared__ uint32_t ids[CAP];
    __shared__ TU tuc[CAP];
    __shared__ int32_t hkey[HC];
    __shared__ uint32_t hval[HC];
    __shared__ unsigned long long exc[TL_EXC];
    __shared__ int32_t nexc;
    S.E = E; S.P = P; S.ids = ids; S.tuc = tuc; S.hkey = hkey; S.hval = hval; S.exc = exc; S.nexc = &nexc;
    S.W = CW;
    S.hcap = HC;
  }
  while (true) {
    __syncthreads();  // every thread has read the previous item before it is replaced
    if (threadIdx.x == 0) item_s = (int64_t)atomicAdd(qhead, 1ull);
    __syncthreads();
    const int64_t it = item_s;
    if (it >= n) break;
    const int32_t u = list[it];
    const int64_t ub = R.roff[u] + R.rlow[u];
    const int32_t dp = (int32_t)(R.roff[u + 1] - ub);
    if (CAP != 0 && dp > CAP) {  // cannot happen: the lists are cut at the tier capacities
      if (threadIdx.x == 0) atomicAdd(&A.bstats[BS_ERR], 1ull);
      continue;
    }
    if (CAP == 0 && dp > A.tri_cap) {  // scratch too small: the host counts again with more
      if (threadIdx.x == 0) atomicAdd(&A.bstats[BS_RETRY], 1ull);
      continue;
    }
    if (CAP == 0 && threadIdx.x == 0) atomicAdd(&A.bstats[BS_TRI_GLOBAL], 1ull);
    const int g = A.gid[u];
    if (g != cur_g) {
      if (cur_g >= 0) flushv<NV>(A.sig, cur_g, SG_K4, kacc);
      cur_g = g;
    }
    if constexpr (CAP != 0) S.W = (dp + 63) / 64;
    tri_large_vertex<NV>(A, S, ub, dp, kacc, ent);
  }
  if (cur_g >= 0) flushv<NV>(A.sig, cur_g, SG_K4, kacc);
  ent = wave_sum64(ent);
  if (lane_id() == 0 && ent) atomicAdd(&A.bstats[BS_TRI_E], (unsigned long long)ent);
}

template <int NV> constexpr int tl_max() { return TRI_LDS_MAX; }

// ------------------------------------------------------------ edge pass
// After all triangles, per upper entry u -> w present in version x, with
// t = t_x(u, w) and d = d_x:
//   S2  += (d_u - 1)(d_w - 1)      DIA += C(t, 2)
//   T3  += t                        (= 3 T)
//   PAW2 += t (d_u + d_w - 4)       (= 2 N_paw: a triangle on the edge plus a
//                                    pendant edge at one of its ends)
// One thread per entry: each workgroup takes one contiguous range of the
// entries, consecutive lanes read consecutive entries (row ids come from the
// region build), and a lane meets a new graph of a pool only at a graph
// boundary of its range, so its per-graph sums are flushed rarely.
template <int NV>
__device__ __forceinline__ void edge_flush_lane(unsigned long long* sig, int g, int64_t (&acc)[4][NV]) {
  const int keys[4] = {SG_S2, SG_DIA, SG_T, SG_PAW};
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int x = 0; x < NV; ++x) {
      if (acc[k][x]) atomicAdd(&sig[SIG_IDX(g, x, keys[k])], (unsigned long long)acc[k][x]);
      acc[k][x] = 0;
    }
}

template <int NV>
__global__ __launch_bounds__(256) void k_edge_pass(CountArgs A) {
  const RegionDev& R = A.R;
  const int64_t E = (int64_t)A.c[C_ER];
  int cur_g = -1;
  int64_t acc[4][NV];  // s2, dia, t3, paw2 per version
#pragma unroll
  for (int k = 0; k < 4; ++k) zerov<NV>(acc[k]);
  const int64_t per = ((E + gridDim.x - 1) / gridDim.x + 255) / 256 * 256;
  const int64_t end = min(E, per * (blockIdx.x + 1));
  for (int64_t p = per * blockIdx.x + threadIdx.x; p < end; p += 256) {
    const uint32_t x = R.rcol[p];
    const uint32_t wv = x & GC_ID;
    const int32_t u = R.rrow[p];
    if (wv <= (uint32_t)u) continue;
    const int g = A.gid[u];
    if (g != cur_g) {
      if (cur_g >= 0) edge_flush_lane<NV>(A.sig, cur_g, acc);
      cur_g = g;
    }
    const uint32_t pm = vpresent<NV>(x);
    int64_t t[NV];
    int32_t du[NV], dw[NV];
    t_read<NV>(R, p, t);
    d_read<NV>(R, u, du);
    d_read<NV>(R, wv, dw);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      if (!((pm >> q) & 1u)) continue;
      acc[0][q] += (int64_t)(du[q] - 1) * (dw[q] - 1);
      acc[1][q] += c2(t[q]);
      acc[2][q] += t[q];
      acc[3][q] += t[q] * (du[q] + dw[q] - 4);
    }
  }
  // Sums of a wave that worked for one graph (or none) go through a block
  // reduction: one atomic per value and block when every wave of the block
  // has the same graph (many atomics on the few words of one graph would
  // queue at one L2 channel), else one per value and wave.  Lanes that saw
  // several graphs flush on their own.
  __shared__ int64_t red[4][4 * NV];
  __shared__ int wg[4];
  const int wv_ = threadIdx.x >> 6;
  int g0 = __shfl(cur_g, 0);
  for (int l = 1; l < 64 && g0 < 0; ++l) g0 = __shfl(cur_g, l);
  const bool wuni = __ballot(cur_g == g0 || cur_g < 0) == ~0ull;
  if (!wuni && cur_g >= 0) edge_flush_lane<NV>(A.sig, cur_g, acc);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int64_t v = wave_sum64(wuni ? acc[k][q] : 0);
      if (lane_id() == 0) red[wv_][k * NV + q] = v;
    }
  if (lane_id() == 0) wg[wv_] = wuni ? g0 : -1;
  __syncthreads();
  if (threadIdx.x < 4 * NV) {
    const int keys[4] = {SG_S2, SG_DIA, SG_T, SG_PAW};
    const int k = threadIdx.x / NV, q = threadIdx.x % NV;
    int gb = -1;
    bool same = true;
    for (int w = 0; w < 4; ++w) {
      if (wg[w] < 0) continue;
      if (gb < 0) gb = wg[w];
      else if (wg[w] != gb) same = false;
    }
    if (same) {
      int64_t v = 0;
      for (int w = 0; w < 4; ++w) v += red[w][threadIdx.x];
      if (gb >= 0 && v) atomicAdd(&A.sig[SIG_IDX(gb, q, keys[k])], (unsigned long long)v);
    } else {
      for (int w = 0; w < 4; ++w)
        if (wg[w] >= 0 && red[w][threadIdx.x])
          atomicAdd(&A.sig[SIG_IDX(wg[w], q, keys[k])], (unsigned long long)red[w][threadIdx.x]);
    }
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
// u in positions [g0, g0 + 64) of row v; calls f(w, flags of both entries).
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
  wave_walk(R.rcol, sb, sl, fvu, [&](int, int64_t, uint32_t fs, uint32_t y) { f(y & GC_ID, fs | (y & GC_FLAGS)); });
}

constexpr int C4S_SLOTS = 512;
constexpr int C4S_WAVES = 4;

// c(v, w) <= wedges of v <= 4096 in the small and mid tiers: 16-bit fields
template <int NV>
__global__ __launch_bounds__(256) void k_c4_small(CountArgs A) {
  using F = Fields<NV, 16>;
  using T = typename F::T;
  __shared__ int32_t hkey[C4S_WAVES][C4S_SLOTS];
  __shared__ T hcnt[C4S_WAVES][C4S_SLOTS];
  const int w = threadIdx.x >> 6, l = lane_id();
  const RegionDev& R = A.R;
  const int64_t n = (int64_t)A.c[C_LIST0 + L_C4_S];
  const int32_t* list = A.lists + L_C4_S * A.list_stride;
  int cur_g = -1;
  int64_t acc[NV];
  zerov<NV>(acc);
  for (int s = l; s < C4S_SLOTS; s += 64) { hkey[w][s] = -1; hcnt[w][s] = 0; }
  wave_sync();
  // a fixed stride: the vertices of this tier are uniformly light (a shared
  // counter costs more than it balances)
  for (int64_t it = (int64_t)blockIdx.x * C4S_WAVES + w; it < n; it += (int64_t)gridDim.x * C4S_WAVES) {
    const int32_t v = list[it];
    const int g = A.gid[v];
    if (g != cur_g) { if (cur_g >= 0) flushv<NV>(A.sig, cur_g, SG_C4, acc); cur_g = g; }
    const int64_t rb = R.roff[v];
    const int32_t nlow = R.rlow[v];
    int32_t* hk = hkey[w];
    T* hc = hcnt[w];
    for (int32_t g0 = 0; g0 < nlow; g0 += 64)
      c4_group(R, (uint32_t)v, rb, nlow, g0, [&](uint32_t wid, uint32_t fl) {
        const uint32_t pm = vpresent<NV>(fl);
        if (pm) hash_add<T>(hk, hc, C4S_SLOTS - 1, 23, wid, F::spread(pm));
      });
    wave_sync();
    for (int s = l; s < C4S_SLOTS; s += 64) {
      if (hk[s] != -1) {
        const T c = hc[s];
#pragma unroll
        for (int x = 0; x < NV; ++x) acc[x] += c2(F::get(c, x));
        hk[s] = -1; hc[s] = 0;
      }
    }
    wave_sync();
  }
  if (cur_g >= 0) flushv<NV>(A.sig, cur_g, SG_C4, acc);
}

constexpr int C4M_SLOTS = 8192;

template <int NV>
__global__ __launch_bounds__(256) void k_c4_mid(CountArgs A) {
  using F = Fields<NV, 16>;
  using T = typename F::T;
  __shared__ int32_t hkey[C4M_SLOTS];
  __shared__ T hcnt[C4M_SLOTS];
  const int w = threadIdx.x >> 6;
  const RegionDev& R = A.R;
  const int64_t n = (int64_t)A.c[C_LIST0 + L_C4_M];
  const int32_t* list = A.lists + L_C4_M * A.list_stride;
  int cur_g = -1;
  int64_t acc[NV];
  zerov<NV>(acc);
  for (int s = threadIdx.x; s < C4M_SLOTS; s += blockDim.x) { hkey[s] = -1; hcnt[s] = 0; }
  __syncthreads();
  // first vertex by block index (no atomic: blocks without one leave at
  // once), later ones from the shared counter counting on from the grid size
  __shared__ int64_t item_s;
  for (int64_t it = blockIdx.x; it < n; it = item_s) {
    const int32_t v = list[it];
    const int g = A.gid[v];
    if (g != cur_g) { if (cur_g >= 0) flushv<NV>(A.sig, cur_g, SG_C4, acc); cur_g = g; }
    const int64_t rb = R.roff[v];
    const int32_t nlow = R.rlow[v];
    for (int32_t g0 = w * 64; g0 < nlow; g0 += 64 * 4)
      c4_group(R, (uint32_t)v, rb, nlow, g0, [&](uint32_t wid, uint32_t fl) {
        const uint32_t pm = vpresent<NV>(fl);
        if (pm) hash_add<T>(hkey, hcnt, C4M_SLOTS - 1, 19, wid, F::spread(pm));
      });
    __syncthreads();
    for (int s = threadIdx.x; s < C4M_SLOTS; s += blockDim.x) {
      if (hkey[s] != -1) {
        const T c = hcnt[s];
#pragma unroll
        for (int x = 0; x < NV; ++x) acc[x] += c2(F::get(c, x));
        hkey[s] = -1; hcnt[s] = 0;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) item_s = (int64_t)gridDim.x + (int64_t)atomicAdd((unsigned long long*)(A.c + C_QC4M), 1ull);
    __syncthreads();
  }
  if (cur_g >= 0) flushv<NV>(A.sig, cur_g, SG_C4, acc);
}

// Large tier: one workgroup per hub v at a time, hubs in decreasing order of
// wedge work.  The opposite vertices w < v are taken in windows of ids from
// v downwards, each with dense LDS counters: one field per w for the wedges
// present in every version (8 bits where no row of the window exceeds 255
// entries, else 16 bits while c(v, w) <= 65535 can be guaranteed, else 32),
// the other wedges in per-version global counters.  Hits concentrate just
// below v because ids are a degree order and a wedge reaches w with odds
// growing with deg w.  Once a window is sparse, all wedges below it go to
// the global counters (one array per resident workgroup, with a touched
// list).  Each lower neighbour u keeps a cursor in its row, starting at v's
// position, and walks it backwards window by window, so rows are read about
// once.  Four versions with 32-bit fields would not fit a 64-bit counter:
// such hubs are walked twice, for versions 0-1 and 2-3.
constexpr int C4W_WIN = 18432;  // 144 KB of 64-bit words
constexpr int C4W_T = 1024;
constexpr int C4_BLK_LOG = 10;  // ids per entry of the row-length maxima: 1024
constexpr int C4_BLK = 1 << C4_BLK_LOG;

struct C4Chunk {
  long long red[C4W_T / 64][2];
};

struct C4Smem {
  unsigned long long win[C4W_WIN];
  C4Chunk C;
  int64_t item;
  int32_t nt;
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

// block maximum (all threads call; result valid in every thread)
__device__ __forceinline__ int32_t block_max32(C4Chunk& C, int32_t x) {
  const int wv = threadIdx.x >> 6;
  x = wave_max32(x);
  if (lane_id() == 0) C.red[wv][0] = x;
  __syncthreads();
  x = 0;
  for (int k = 0; k < C4W_T / 64; ++k) x = max(x, (int32_t)C.red[k][0]);
  __syncthreads();
  return x;
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
// positions [urow[q] + p0(q), urow[q] + p1(q)); f(w, flags of both entries).
// Thread q takes u_q: short slices (the common case: u_q has few entries in
// the id range) are walked by their own thread, long ones by their whole
// wave, one at a time (wave_walk).
constexpr int32_t C4W_SHORT = 128;  // entries a thread walks itself before the gallop

template <class P0, class P1, class F>
__device__ __forceinline__ void c4_block_walk(const RegionDev& R, int64_t rb, int32_t nlow, const int64_t* urow,
                                              P0 p0f, P1 p1f, F f) {
  const int t = threadIdx.x;
  for (int32_t c0 = 0; c0 < nlow; c0 += C4W_T) {
    const int32_t q = c0 + t;
    int64_t sb = 0;
    int32_t sl = 0;
    uint32_t fl = 0;
    int32_t p0 = 0, p1 = 0;
    if (q < nlow) { p0 = p0f(q); p1 = p1f(q); }
    if (p1 > p0) {
      sb = urow[q] + p0;
      fl = R.rcol[rb + q] & GC_FLAGS;
      if (p1 - p0 <= C4W_SHORT) {
        const int32_t len = p1 - p0;
        for (int32_t k = 0; k < len; k += 4) {  // four loads in flight
          uint32_t y[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) y[u] = k + u < len ? R.rcol[sb + k + u] : 0u;
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (k + u < len) f(y[u] & GC_ID, fl | (y[u] & GC_FLAGS));
        }
      } else {
        sl = p1 - p0;
      }
    }
    if (__ballot(sl > 0))
      wave_walk(R.rcol, sb, sl, fl, [&](int, int64_t, uint32_t fs, uint32_t y) { f(y & GC_ID, fs | (y & GC_FLAGS)); });
  }
  __syncthreads();
}

// One window of ids [lo, ...) of hub v: every lower neighbour u_q walks its
// row backwards from its cursor while the ids stay >= lo and leaves the
// cursor at the first position below the window, so the slice is read once
// and no search precedes it.  The thread reads up to C4W_SHORT entries itself,
// four at a time; the rest of a longer slice is delimited by a gallop and
// walked by the whole wave.  wtot += entries walked, rest += entries left
// below the window (per thread).
template <class F>
__device__ __forceinline__ void c4_window_walk(const RegionDev& R, int64_t rb, int32_t nlow, const int64_t* urow,
                                               int32_t* ucur, uint32_t lo, F f, long long& wtot, long long& rest) {
  const int t = threadIdx.x;
  for (int32_t c0 = 0; c0 < nlow; c0 += C4W_T) {
    const int32_t q = c0 + t;
    int64_t sb = 0;
    int32_t sl = 0;
    uint32_t fl = 0;
    if (q < nlow) {
      const int32_t c = ucur[q];
      int32_t k = c;  // positions [k, c) are walked
      if (c > 0) {
        const int64_t base = urow[q];
        const uint32_t* row = R.rcol + base;
        fl = R.rcol[rb + q] & GC_FLAGS;
        const int32_t a0 = (int32_t)(base & 3);  // row start within its 16-byte group
        bool open = true;
        while (open && c - k < C4W_SHORT) {
          // one 16-byte load: the aligned group of four entries holding
          // position k - 1.  Its positions in [0, k) with ids >= lo are a
          // run ending at k - 1 (rows are sorted), so each entry is tested
          // on its own; the walk goes on while the whole group was taken.
          const int32_t top = k - 1;
          const int32_t g = ((top + a0) & ~3) - a0;  // position of the group's first entry (>= -3)
          const uint4 g4 = *(const uint4*)(row + g);
          const uint32_t y[4] = {g4.x, g4.y, g4.z, g4.w};
          int32_t took = 0;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t id = y[u] & GC_ID;
            const bool ok = g + u >= 0 && g + u <= top && id >= lo;
            took += ok ? 1 : 0;
            if (ok) f(id, fl | (y[u] & GC_FLAGS));
          }
          open = g > 0 && took == top + 1 - g;
          k -= took;
        }
        if (open) {  // more than C4W_SHORT entries in the window
          const int32_t p0 = gallop_down(row, k, lo);
          sb = base + p0;
          sl = k - p0;
          k = p0;
        }
        ucur[q] = k;
      }
      wtot += c - k;
      rest += k;
    }
    if (__ballot(sl > 0))  // slices this long run to hundreds of entries: eight loads in flight per lane
      wave_walk<8>(R.rcol, sb, sl, fl, [&](int, int64_t, uint32_t fs, uint32_t y) { f(y & GC_ID, fs | (y & GC_FLAGS)); });
  }
}

// Pair sums of one 16-byte piece of single-field window counters of FB bits:
// s += c(c - 1) for every counter c, with no branch on zero counters.
template <int FB>
__device__ __forceinline__ void window_pairs(const uint4 q, uint64_t& s) {
  const uint32_t wv[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if constexpr (FB == 8) {
      uint32_t p = 0;  // four products < 2^16 each
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t a = (wv[k] >> (8 * b)) & 0xFFu;
        p += a * (a - 1u);
      }
      s += p;
    } else if constexpr (FB == 16) {
      const uint32_t a = wv[k] & 0xFFFFu, b = wv[k] >> 16;
      s += (uint64_t)(a * (a - 1u));  // < 2^32 for a < 2^16, and 0 for a = 0
      s += (uint64_t)(b * (b - 1u));
    } else {
      s += (uint64_t)wv[k] * (uint64_t)(wv[k] - 1u);
    }
  }
}

// One hub v, versions [vsh, vsh + NF) of an NV-version pass.  The window
// counts, per opposite vertex w, the wedges present in exactly the reference
// versions (c_A(w), one field of FBW bits, or of 8 bits over twice the ids
// where every row of the window's blocks has at most 255 entries, which
// bounds c_A; the reference set M is every
// version, or every version but 0 when version 0 is the empty graph); the
// other wedges (few: they hold a flagged entry) go to the block's global
// counters (e_x(w) per version x, one u64 of NF fields of 64 / NF bits, by
// atomics whose result nobody waits for, with w listed once per wedge, or
// the whole id range read back when the list would outgrow it).  With
// c_x = [x in M] c_A + e_x,
//   sum_w C(c_x(w), 2) = [x in M] sum_w C(c_A(w), 2)
//                        + sum_{w with exceptions} ([x in M] c_A e_x + C(e_x, 2)),
// so one scan of the window serves every version of M and the exceptions add
// the rest.  The tail uses the same global counters.  The window and the
// global counters are clear on entry and on return (each pass clears what it
// read).
template <int NV, int NF, int FBW>
__device__ void c4_hub(const CountArgs& A, C4Smem& S, int32_t v, int vsh, int64_t (&acc)[NV], int64_t& tail_) {
  using TFd = Fields<NF, 64 / NF>;
  constexpr int IPW = 32 / FBW;  // ids per 32-bit window word
  const RegionDev& R = A.R;
  const int t = threadIdx.x;
  unsigned long long* cnt = A.c4_dense + (int64_t)blockIdx.x * A.N;
  int32_t* touch = A.c4_touch + (int64_t)blockIdx.x * A.N;
  int64_t* urow = A.c4_cur + (int64_t)blockIdx.x * 2 * A.c4_maxlow;
  int32_t* ucur = (int32_t*)(urow + A.c4_maxlow);
  const int64_t rb = R.roff[v];
  const int32_t nlow = R.rlow[v];
  const uint32_t fmask = (1u << NF) - 1u;
  const uint32_t ref = (A.c4_ref >> vsh) & fmask;
  const int64_t ws = (int64_t)A.c4_win * 2 * IPW;  // ids per window
  uint32_t* wc = (uint32_t*)S.win;
  // field layout of the current window: 2^sh ids of fw bits per 32-bit word
  int sh = FBW == 16 ? 1 : 0, fw = FBW;
  auto count_of = [&](uint32_t o) -> uint32_t {  // c_A of the id at offset o in the window
    const uint32_t im = (1u << sh) - 1u;
    return (uint32_t)(((uint64_t)wc[o >> sh] >> (fw * (o & im))) & ((1ull << fw) - 1ull));
  };
  if (t == 0) S.nt = 0;
  for (int32_t q = t; q < nlow; q += C4W_T) {
    urow[q] = R.roff[R.rcol[rb + q] & GC_ID];
    ucur[q] = R.vpos[rb + q];
  }
  __syncthreads();
  int64_t hi = v;
  while (hi > 0) {
    int64_t wsz = ws;
    sh = FBW == 16 ? 1 : 0;
    fw = FBW;
    if constexpr (FBW == 16) {
      // 8-bit fields over twice the ids when no row there is longer than 255
      const int64_t lo8 = hi - 2 * ws > 0 ? hi - 2 * ws : 0;
      const int64_t b0 = lo8 >> C4_BLK_LOG, b1 = (hi - 1) >> C4_BLK_LOG;
      int32_t m = 0;
      for (int64_t b = b0 + t; b <= b1; b += C4W_T) m = max(m, A.c4_blk[b]);
      if (block_max32(S.C, m) <= 255) { sh = 2; fw = 8; wsz = 2 * ws; }
    }
    const uint32_t lo = (uint32_t)(hi - wsz > 0 ? hi - wsz : 0);
    const int32_t wcap = (int32_t)(hi - lo);  // list capacity: ids of the window (<= N)
    if (t == 0) {
      atomicAdd(&A.bstats[BS_C4_SEARCH], (unsigned long long)nlow);
      atomicAdd(&A.bstats[BS_C4_WINDOWS], 1ull);
    }
    long long wtot = 0, rest = 0;
    // the window walk with the field layout as constants (8-bit fields, or FBW)
    auto walk = [&](auto fwc) {
      constexpr int FW = decltype(fwc)::value;
      constexpr int SH = FW == 8 ? 2 : (FW == 16 ? 1 : 0);
      constexpr uint32_t IM = (1u << SH) - 1u;
      c4_window_walk(R, rb, nlow, urow, ucur, lo,
                     [&](uint32_t wid, uint32_t fl) {
                       const uint32_t sub = (vpresent<NV>(fl) >> vsh) & fmask;
                       const uint32_t o = wid - lo;
                       if (sub == ref) {
                         atomicAdd(&wc[o >> SH], 1u << (FW * (o & IM)));
                       } else if (sub) {  // present in some versions only
                         // no wait for the global atomic: the id is listed once per
                         // exception wedge (while the list is shorter than the window)
                         atomicAdd(&cnt[wid], (unsigned long long)TFd::spread(sub));
                         const int32_t p = atomicAdd(&S.nt, 1);
                         if (p < wcap) touch[p] = (int32_t)wid;
                       }
                     },
                     wtot, rest);
    };
    if (fw == 8) walk(std::integral_constant<int, 8>{});
    else walk(std::integral_constant<int, FBW>{});
    block_sum2(S.C, wtot, rest);  // also orders the window's counter updates before the passes below
    if (const int32_t nt = S.nt) {  // the window's exceptions
      auto one = [&](int32_t k, unsigned long long e) {
        const int64_t c = (int64_t)count_of((uint32_t)k - lo);
#pragma unroll
        for (int x = 0; x < NF; ++x) {
          const int64_t ex = TFd::get(e, x);
          acc[vsh + x] += ((ref >> x) & 1u ? c * ex : 0) + c2(ex);
        }
      };
      if (nt <= wcap) {
        // an id listed several times: the first exchange takes its counter
        for (int32_t q = t; q < nt; q += C4W_T) {
          const int32_t k = touch[q];
          const unsigned long long e = atomicExch(&cnt[k], 0ull);
          if (e) one(k, e);
        }
      } else {
        // more exception wedges than ids in the window: every counter of it
        for (int64_t k = lo + t; k < hi; k += C4W_T) {
          const unsigned long long e = __hip_atomic_load(&cnt[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (e) {
            cnt[k] = 0ull;
            one((int32_t)k, e);
          }
        }
      }
      __syncthreads();
      if (t == 0) S.nt = 0;
    }
    {
      uint4* w4 = (uint4*)S.win;
      uint64_t s2 = 0;
      for (int qi = t; qi < A.c4_win / 2; qi += C4W_T) {
        const uint4 q = w4[qi];
        w4[qi] = make_uint4(0u, 0u, 0u, 0u);
        if (fw == 8) window_pairs<8>(q, s2);
        else window_pairs<FBW>(q, s2);
      }
#pragma unroll
      for (int x = 0; x < NF; ++x)
        if ((ref >> x) & 1u) acc[vsh + x] += (int64_t)(s2 >> 1);  // sum of c(c - 1), all even
    }
    __syncthreads();
    hi = lo;
    if (rest == 0) break;
    if (wtot < A.c4_dense_min) {
      // sparse from here down: every remaining wedge in global memory
      const int32_t tcap = (int32_t)lo;  // list capacity: the ids below the windows (<= N)
      c4_block_walk(R, rb, nlow, urow, [&](int32_t) { return 0; }, [&](int32_t q) { return ucur[q]; },
                    [&](uint32_t wid, uint32_t fl) {
                      const uint32_t sub = (vpresent<NV>(fl) >> vsh) & fmask;
                      if (!sub) return;
                      ++tail_;
                      // as in the windows: no wait for the global atomic, the id
                      // listed once per wedge while the list is shorter than [0, lo)
                      atomicAdd(&cnt[wid], (unsigned long long)TFd::spread(sub));
                      const int32_t p = atomicAdd(&S.nt, 1);
                      if (p < tcap) touch[p] = (int32_t)wid;
                    });
      const int32_t nt = S.nt;
      if (nt <= tcap) {
        for (int32_t q = t; q < nt; q += C4W_T) {
          const unsigned long long c = atomicExch(&cnt[touch[q]], 0ull);
#pragma unroll
          for (int x = 0; x < NF; ++x) acc[vsh + x] += c2(TFd::get(c, x));
        }
      } else {
        for (int64_t k = t; k < (int64_t)lo; k += C4W_T) {
          const unsigned long long c = __hip_atomic_load(&cnt[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (c) {
            cnt[k] = 0ull;
#pragma unroll
            for (int x = 0; x < NF; ++x) acc[vsh + x] += c2(TFd::get(c, x));
          }
        }
      }
      __syncthreads();
      if (t == 0) S.nt = 0;
      break;
    }
  }
  __syncthreads();
}

template <int NV>
__global__ __launch_bounds__(C4W_T) void k_c4_large(CountArgs A, unsigned long long* qhead) {
  __shared__ C4Smem S;
  const RegionDev& R = A.R;
  const int64_t n = (int64_t)A.c[C_LIST0 + L_C4_L];
  const int32_t* list = A.lists + L_C4_L * A.list_stride;
  const int t = threadIdx.x;
  int cur_g = -1;
  int64_t acc[NV];
  zerov<NV>(acc);
  int64_t tail_ = 0;
  for (int s = t; s < A.c4_win; s += C4W_T) S.win[s] = 0ull;  // kept clear between windows
  while (true) {
    __syncthreads();  // every thread has read the previous item before it is replaced
    if (t == 0) S.item = (int64_t)atomicAdd(qhead, 1ull);
    __syncthreads();
    const int64_t item = S.item;
    if (item >= n) break;
    const int32_t v = list[item];
    const int g = A.gid[v];
    if (g != cur_g) { if (cur_g >= 0) flushv<NV>(A.sig, cur_g, SG_C4, acc); cur_g = g; }
    if (R.rlow[v] > A.c4_maxlow) {  // cursor scratch too small: the host counts again with more
      if (t == 0) atomicAdd(&A.bstats[BS_RETRY], 1ull);
      continue;
    }
    // c(v, w) <= nlow: 16-bit fields suffice up to 65535 lower neighbours
    const bool narrow = R.rlow[v] <= A.c4_narrow_max;
    if constexpr (NV == 2) {
      if (narrow) c4_hub<2, 2, 16>(A, S, v, 0, acc, tail_);
      else c4_hub<2, 2, 32>(A, S, v, 0, acc, tail_);
    } else {
      if (narrow) {
        c4_hub<4, 4, 16>(A, S, v, 0, acc, tail_);
      } else {
        c4_hub<4, 2, 32>(A, S, v, 0, acc, tail_);
        c4_hub<4, 2, 32>(A, S, v, 2, acc, tail_);
      }
    }
  }
  if (cur_g >= 0) flushv<NV>(A.sig, cur_g, SG_C4, acc);
  tail_ = wave_sum64(tail_);
  if (lane_id() == 0 && tail_) atomicAdd(&A.bstats[BS_TRIPROBE], (unsigned long long)tail_);
}

// Largest union row length in each block of C4_BLK ids: bounds c(v, w) for
// every w of the block, so a hub window over blocks whose rows are all at
// most 255 long can count in 8-bit fields.  blk must be zero on entry.
__global__ void k_c4_blkmax(const int64_t* __restrict__ roff, int64_t N, int32_t* __restrict__ blk) {
  for (int64_t v0 = (int64_t)blockIdx.x * 256 * 4; v0 < N; v0 += (int64_t)gridDim.x * 256 * 4) {
    int32_t m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t v = v0 + threadIdx.x + 256 * k;
      if (v < N) m = max(m, (int32_t)(roff[v + 1] - roff[v]));
    }
    // the 1024 ids of one iteration form one block (v0 is block aligned)
    m = wave_max32(m);
    if (lane_id() == 0 && m) atomicMax(&blk[v0 >> C4_BLK_LOG], m);
  }
}

// hubs of the large tier in decreasing order of wedge work
__global__ void k_c4_order(const unsigned long long* sorted, const unsigned long long* c, int32_t* list) {
  const int64_t n = (int64_t)c[C_LIST0 + L_C4_L];
  for (int64_t i = gtid(); i < n; i += gstride()) list[i] = (int32_t)(sorted[i] & 0xFFFFFFFFull);
}

// --------------------------------------------------------------- combine
// C' = C_x - C_0 on the six connected classes for every later version x
// (Alg. 2), through the non-induced counts of each version and the
// triangular relation between non-induced and induced counts (copies of
// pattern X inside class Y).
template <int NV>
__global__ void k_combine(const unsigned long long* sig, long long* state, long long* vout, int32_t k,
                          const unsigned long long* bstats) {
  const int64_t g = gtid();
  if (g >= k || bstats[BS_RETRY]) return;
  int64_t N[NV][6], T[NV], W[NV], D1[NV];
  int bad = 0;
  for (int x = 0; x < NV; ++x) {
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
  long long* st = state + g * ST_STRIDE;
  long long base[ST_STRIDE];
  for (int c = 0; c < ST_STRIDE; ++c) base[c] = st[c];
  for (int x = 1; x < NV; ++x) {
    int64_t d[6];
    for (int c = 0; c < 6; ++c) d[c] = N[x][c] - N[0][c];
    int64_t I[6];
    I[5] = d[5];
    I[4] = d[4] - 6 * I[5];
    I[3] = d[3] - 4 * I[4] - 12 * I[5];
    I[2] = d[2] - I[4] - 3 * I[5];
    I[0] = d[0] - 2 * I[3] - 4 * I[2] - 6 * I[4] - 12 * I[5];
    I[1] = d[1] - I[3] - 2 * I[4] - 4 * I[5];
    long long* o = vout + ((int64_t)(x - 1) * k + g) * ST_STRIDE;
    for (int c = 0; c < ST_STRIDE; ++c) o[c] = base[c];
    for (int c = 0; c < 6; ++c) o[ST_F0 + c] += I[c];
    o[ST_T] += T[x] - T[0];
    o[ST_W] += W[x] - W[0];
    o[ST_M] += (D1[x] - D1[0]) / 2;
    if (bad) o[ST_ERR] += 1;
    if (x == NV - 1)
      for (int c = 0; c < ST_STRIDE; ++c) st[c] = o[c];
  }
}

inline unsigned cap_grid(int64_t want, unsigned cap) {
  if (want < 1) want = 1;
  return (unsigned)(want > cap ? cap : want);
}

template <int NV>
void launch_count_t(const CountArgs& A, hipStream_t s, hipEvent_t* ev) {
  constexpr int TLM = tl_max<NV>();
  const int64_t N = A.N;
  const unsigned long long* cnt_er = A.c + C_ER;
  if (ev) (void)hipEventRecord(ev[0], s);
  fill_u64_count(A.R.t, 0ull, cnt_er, 1, A.e_max, s);
  if (NV == 4) fill_u64_count(A.R.tp, 0ull, cnt_er, 2, 2 * A.e_max, s);
  hipLaunchKernelGGL(k_tri_small<NV>, dim3(cap_grid((N + 3) / 4, 8192)), dim3(256), 0, s, A);
  // out-degree tiers (64,128] (256] (512] (1024] (TLM] and above, one list each
  unsigned long long* qt = (unsigned long long*)(A.c + C_QTRI) - L_TRI_1;
  hipLaunchKernelGGL((k_tri_large<128, 128, NV>), dim3(cap_grid(N, 8192)), dim3(128), 0, s, A, (int)L_TRI_1,
                     qt + L_TRI_1);
  hipLaunchKernelGGL((k_tri_large<256, 256, NV>), dim3(cap_grid(N, 4096)), dim3(256), 0, s, A, (int)L_TRI_2,
                     qt + L_TRI_2);
  hipLaunchKernelGGL((k_tri_large<512, 512, NV>), dim3(cap_grid(N, 2048)), dim3(512), 0, s, A, (int)L_TRI_3,
                     qt + L_TRI_3);
  hipLaunchKernelGGL((k_tri_large<1024, 1024, NV>), dim3(cap_grid(N, 1024)), dim3(1024), 0, s, A, (int)L_TRI_4,
                     qt + L_TRI_4);
  hipLaunchKernelGGL((k_tri_large<TLM, 1024, NV>), dim3(cap_grid(N, 1024)), dim3(1024), 0, s, A, (int)L_TRI_5,
                     qt + L_TRI_5);
  hipLaunchKernelGGL((k_tri_large<0, 256, NV>), dim3(cap_grid(N, (unsigned)A.tri_slots)), dim3(256), 0, s, A,
                     (int)L_TRI_G, qt + L_TRI_G);
  if (ev) (void)hipEventRecord(ev[1], s);
  // at least 4096 entries per workgroup: few flushes of per-graph sums
  hipLaunchKernelGGL(k_edge_pass<NV>, dim3(cap_grid((A.e_max + 4095) / 4096, 2048)), dim3(256), 0, s, A);
  if (ev) (void)hipEventRecord(ev[2], s);
  hipLaunchKernelGGL(k_c4_small<NV>, dim3(cap_grid((N + 3) / 4, 8192)), dim3(256), 0, s, A);
  if (ev) (void)hipEventRecord(ev[3], s);
  hipLaunchKernelGGL(k_c4_mid<NV>, dim3(cap_grid(N, 4096)), dim3(256), 0, s, A);
  if (ev) (void)hipEventRecord(ev[4], s);
  // order the hubs by decreasing wedge work (keys written by the per-vertex pass)
  unsigned long long* sk = radix_sort_u64(A.c4_keys, A.c4_keys_alt, A.sort_tmp, N, A.c + C_LIST0 + L_C4_L, 64, s);
  hipLaunchKernelGGL(k_c4_order, dim3(cap_grid((N + 255) / 256, 1024)), dim3(256), 0, s, sk, A.c,
                     (int32_t*)(A.lists + L_C4_L * A.list_stride));
  fill_u32((uint32_t*)A.c4_blk, 0u, N / C4_BLK + 2, s);
  hipLaunchKernelGGL(k_c4_blkmax, dim3(cap_grid((N + 1023) / 1024, 4096)), dim3(256), 0, s, A.R.roff, N, A.c4_blk);
  hipLaunchKernelGGL(k_c4_large<NV>, dim3(cap_grid(N, (unsigned)A.slots)), dim3(C4W_T), 0, s, A,
                     (unsigned long long*)(A.c + C_QHEAD));
  if (ev) (void)hipEventRecord(ev[5], s);
}

}  // namespace

int32_t c4_window_max() { return C4W_WIN; }
int32_t c4_block_ids() { return C4_BLK; }
int64_t tri_scratch_words64(int nv, int64_t cap) {
  return nv == 2 ? tri_slot_words64<2>(cap) : tri_slot_words64<4>(cap);
}
int32_t tri_lds_max(int nv) { return nv == 2 ? tl_max<2>() : tl_max<4>(); }

void launch_count(int nv, const CountArgs& A, hipStream_t s, hipEvent_t* ev) {
  if (nv == 2) launch_count_t<2>(A, s, ev);
  else launch_count_t<4>(A, s, ev);
}

void launch_combine(int nv, const unsigned long long* sig, long long* state, long long* vout, int32_t k,
                    const unsigned long long* bstats, hipStream_t s) {
  if (nv == 2) hipLaunchKernelGGL(k_combine<2>, dim3((k + 63) / 64), dim3(64), 0, s, sig, state, vout, k, bstats);
  else hipLaunchKernelGGL(k_combine<4>, dim3((k + 63) / 64), dim3(64), 0, s, sig, state, vout, k, bstats);
}
