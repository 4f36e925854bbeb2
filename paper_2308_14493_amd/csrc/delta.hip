// Edge-local update of the Sigma terms of a one-batch pass: instead of
// counting the region of change in both versions, only the structures that
// contain a changed pair are enumerated (the idea of updating the count from
// where the change is located, Sec. 4.1), giving C(G_a) - C(G_b) exactly.
//
// Input: the union view left by the tombstone merge (rows sorted by id; an
// entry carries GC_F_NEW when it is absent before the batch, GC_F_DEL when
// absent after it), the sorted directed change lists dirA / dirD and the
// touched rows.  Output: the per-graph sums of version 1 of the pass hold
// the deltas of every Sigma term (version 0 stays zero), so the combine
// kernel applies them unchanged; the per-vertex triangle counts Tv move to
// the graph after the batch.
//
// A structure (triangle, 4-clique, 4-cycle) that holds several changed pairs
// is counted once, from the changed pair with the smallest key (min << bits |
// max); it adds [present after] - [present before], decided by the OR of its
// entries' flags.  Per term:
//   S1, W, D1   touched vertices (their degrees before and after);
//   S2          edges at touched vertices, each once;
//   T, DIA      the affected edges -- changed edges and the other two edges
//               of every triangle on a changed edge (deduplicated): t before
//               and after by row intersection, sum of [p] t and [p] C(t, 2);
//   PAW         sum_e t_e (d_u + d_v - 4): affected edges directly; for the
//               other edges at a vertex x whose degree changed, their t sum
//               is 2 T(x) minus the affected ones (T(x) kept per vertex);
//   K4          per changed edge e = (u, v): pairs {w, x} of common
//               neighbours S(e) joined by an edge;
//   C4          per changed edge: paths s - a - b - o closing the cycle with
//               e = (s, o), from the common ids of N(a) and N(o) for each
//               pair (s, a): rows of similar length merged by a wave, a
//               shorter N(a) walked against an LDS hash table of a small
//               enough N(o), the others by walking the shorter row and
//               searching the other.
#include "gc_kernels.h"

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ int64_t ctr(const unsigned long long* c, int k) { return (int64_t)c[k]; }

// flags of an entry as a 2-bit nibble: bit 0 = absent before, bit 1 = absent after
__device__ __forceinline__ uint32_t nib(uint32_t entry) { return (entry >> GC_VSHIFT) & 3u; }
// [present after] - [present before] of a structure whose entries' nibbles OR to f
__device__ __forceinline__ int64_t delta_of(uint32_t f) { return (int64_t)((f & 2u) == 0) - (int64_t)((f & 1u) == 0); }

__device__ __forceinline__ unsigned long long pkey(uint32_t a, uint32_t b, int bits) {
  const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
  return ((unsigned long long)lo << bits) | hi;
}

// Position of id in row r (sorted, flags ignored) or -1.
__device__ __forceinline__ int64_t find_in_row(const PoolDev& P, uint32_t r, uint32_t id) {
  const uint32_t* row = P.col + P.off[r];
  const int32_t n = P.len[r];
  const int32_t p = lower_bound_id(row, n, id);
  return (p < n && (row[p] & GC_ID) == id) ? P.off[r] + p : -1;
}

// The common ids of two id-sorted rows, the wave together: each step loads
// the next 64 entries of both rows (one per lane), finds each a entry in the
// b window by a search over the lanes, and consumes the window with the
// smaller last id together with the entries of the other window up to that
// id.  No common id is ever consumed on one side only, so each is met once,
// in the step that consumes it, with both of its entries in the windows.
// f(entry of a, entry of b) per common id, on the lane holding the a entry.
// The step bookkeeping is wave-uniform (scalar registers and branches): lanes
// past a row's end load its last entry again instead of branching, the
// windows' last ids are read from lane 63, and the lane exchanges address
// ds_bpermute by byte (lane * 4) directly.
__device__ __forceinline__ uint32_t bperm4(uint32_t byte_lane, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((int)byte_lane, (int)v);
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
  return (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32)) << 32) |
                   __builtin_amdgcn_readfirstlane((uint32_t)x));
}

// Rows a = col + oa (na entries) and b = col + ob (nb entries), the same on
// every lane of the wave.
template <class F>
__device__ __forceinline__ void wave_window_common(const uint32_t* __restrict__ col, int64_t oa_, int32_t na_,
                                                   int64_t ob_, int32_t nb_, F f) {
  const int64_t oa = uniform64(oa_), ob = uniform64(ob_);
  const int32_t na = __builtin_amdgcn_readfirstlane(na_), nb = __builtin_amdgcn_readfirstlane(nb_);
  const int32_t l = lane_id();
  int32_t i0 = 0, j0 = 0;
  while (i0 < na && j0 < nb) {
    const int32_t ra = na - i0, rb = nb - j0;  // > 0
    const bool va = l < ra, vb = l < rb;
    const uint32_t* aw = col + (oa + i0);
    const uint32_t* bw = col + (ob + j0);
    const uint32_t ea = aw[(uint32_t)min(l, ra - 1)], eb = bw[(uint32_t)min(l, rb - 1)];
    const uint32_t ida = ea & GC_ID, idb = eb & GC_ID;
    // last ids of the windows (lane 63 holds the last entry of a short one)
    const uint32_t amax = __builtin_amdgcn_readlane(ida, 63), bmax = __builtin_amdgcn_readlane(idb, 63);
    const uint32_t ia = va ? ida : 0xFFFFFFFFu, ib = vb ? idb : 0xFFFFFFFFu;
    // 4 x (number of window ids of b below ia): the window ascends and is
    // padded above; a count of 64 reads lane 0 (ds_bpermute wraps), whose
    // id is below ia, so it never matches
    uint32_t lo4 = 0;
#pragma unroll
    for (uint32_t sp = 32; sp >= 1; sp >>= 1) lo4 = bperm4(lo4 + 4 * (sp - 1), ib) < ia ? lo4 + 4 * sp : lo4;
    const uint32_t ibp = bperm4(lo4, ib), ebp = bperm4(lo4, eb);
    if (va && ibp == ia) f(ea, ebp);
    if (amax <= bmax) {
      j0 += (int32_t)__popcll(__ballot(ib <= amax));
      i0 += 64;
    } else {
      i0 += (int32_t)__popcll(__ballot(ia <= bmax));
      j0 += 64;
    }
  }
}

// Work items for the waves of a grid: each wave's first item is its own
// index (no atomic, so a small input costs no contention: waves without an
// item leave at once), and a wave that finished one takes the next from a
// shared counter counting on from the grid's wave count, so that waves which
// met light items take more (a fixed share per wave leaves the kernel
// waiting for the wave that drew the heaviest ones).  One item at a time:
// the items in flight stay a moving window of consecutive ones, whose rows
// (one changed edge's opposite row, one vertex's row) the waves share in L2
// (chunks of 16 spread the waves over the item space: both kernels slower by
// half and more).  Returns the same item on every lane.
__device__ __forceinline__ int64_t wave_next(unsigned long long* ctr_, int64_t nwaves) {
  unsigned long long c = 0;
  if (lane_id() == 0) c = atomicAdd(ctr_, 1ull);
  return nwaves + (int64_t)__shfl(c, 0);
}

// degree of v in version x (0 before, 1 after): touched rows carry flags and
// have their two degrees in dd; the others have none
__device__ __forceinline__ int64_t deg_of(const DeltaArgs& D, uint32_t v, int x) {
  return D.mark[v] ? (int64_t)D.dd[2 * (int64_t)v + x] : (int64_t)D.P.len[v];
}

__device__ __forceinline__ void add_sig(const DeltaArgs& D, int g, int k, int64_t v) {
  v = wave_sum64(v);
  if (lane_id() == 0 && v != 0) atomicAdd(&D.sig[SIG_IDX(g, 1, k)], (unsigned long long)v);
}

}  // namespace

// --------------------------------------------------------------- changed
// The changed pairs (u < v) of the pass from the directed lists, with the
// pair's nibble in bits 60..61.
__global__ void k_delta_edges(DeltaArgs D) {
  const int64_t na = ctr(D.c, C_DIRA), nd = ctr(D.c, C_DIRD);
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  for (int64_t i = gtid(); i < na + nd; i += gstride()) {
    const unsigned long long k = i < na ? D.dirA[i] : D.dirD[i - na];
    const unsigned long long key = k & DIR_KEY_MASK;
    const uint32_t r = (uint32_t)(key >> D.bits), c = (uint32_t)(key & idmask);
    if (r >= c) continue;
    const unsigned long long p = atomicAdd(&D.dc[DC_EDGES], 1ull);
    if ((int64_t)p < D.ce_cap) D.ce[p] = key | ((unsigned long long)(i < na ? 1u : 2u) << DIR_MASK_SHIFT);
  }
}

// ------------------------------------------------------- touched vertices
// The touched rows are cut in pieces of at most TV_CHUNK entries (a hub row
// in many), numbered by a scan, and each wave takes one piece at a time: no
// wave walks a whole hub row alone.

// pieces per touched row (0 past the touched count, for the scan)
__global__ void k_delta_titems(DeltaArgs D) {
  const int64_t nt = ctr(D.c, C_TOUCH);
  for (int64_t t = gtid(); t < D.tcap; t += gstride()) {
    int32_t n = 0;
    if (t < nt) {
      const int32_t x = D.touched[t];
      n = max(1, (D.P.len[x] + TV_CHUNK - 1) / TV_CHUNK);
      D.dd[2 * (int64_t)x] = 0;
      D.dd[2 * (int64_t)x + 1] = 0;
    }
    D.tv_items[t] = n;
  }
}

// touched row and entry range of piece k (wave-uniform)
__device__ __forceinline__ void touched_piece(const DeltaArgs& D, int64_t nt, int64_t k, uint32_t& x, int32_t& k0,
                                              int32_t& k1) {
  int64_t lo = 0, hi = nt;  // largest t with tv_ioff[t] <= k
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (D.tv_ioff[mid] <= k) lo = mid; else hi = mid;
  }
  x = (uint32_t)D.touched[lo];
  k0 = (int32_t)((k - D.tv_ioff[lo]) * TV_CHUNK);
  k1 = min(D.P.len[x], k0 + TV_CHUNK);
}

// degrees of the touched rows before and after the batch, by pieces
__global__ void k_delta_vertex(DeltaArgs D) {
  const int64_t nt = ctr(D.c, C_TOUCH);
  if (nt == 0) return;
  const int64_t np = D.tv_ioff[nt];
  const int l = lane_id();
  const int64_t w0 = gtid() >> 6, ws = gstride() >> 6;
  for (int64_t k = w0; k < np; k += ws) {
    uint32_t x;
    int32_t k0, k1;
    touched_piece(D, nt, k, x, k0, k1);
    const uint32_t* row = D.P.col + D.P.off[x];
    int32_t db = 0, da = 0;
    for (int32_t q = k0 + l; q < k1; q += 64) {
      const uint32_t f = nib(row[q]);
      db += (f & 1u) == 0;
      da += (f & 2u) == 0;
    }
    db = wave_sum32(db);
    da = wave_sum32(da);
    if (l == 0) {
      if (db) atomicAdd(&D.dd[2 * (int64_t)x], db);
      if (da) atomicAdd(&D.dd[2 * (int64_t)x + 1], da);
    }
  }
}

// the 3-star, wedge and degree-sum terms of each touched vertex
__global__ void k_delta_vertex_fin(DeltaArgs D) {
  const int64_t nt = ctr(D.c, C_TOUCH);
  for (int64_t t = gtid(); t < nt; t += gstride()) {
    const uint32_t x = (uint32_t)D.touched[t];
    const int64_t db = D.dd[2 * (int64_t)x], da = D.dd[2 * (int64_t)x + 1];
    const int g = D.gid[x];
    const int64_t s1 = c3(da) - c3(db), w2 = c2(da) - c2(db), d1 = da - db;
    if (s1) atomicAdd(&D.sig[SIG_IDX(g, 1, SG_S1)], (unsigned long long)s1);
    if (w2) atomicAdd(&D.sig[SIG_IDX(g, 1, SG_W)], (unsigned long long)w2);
    if (d1) atomicAdd(&D.sig[SIG_IDX(g, 1, SG_D1)], (unsigned long long)d1);
  }
}

// S2 = sum_e (d_u - 1)(d_v - 1) changes only on edges at a touched vertex;
// an edge between two touched vertices is taken at the smaller id.
__global__ void k_delta_s2(DeltaArgs D) {
  const int64_t nt = ctr(D.c, C_TOUCH);
  if (nt == 0) return;
  const int64_t np = D.tv_ioff[nt];
  const int l = lane_id();
  const int64_t w0 = gtid() >> 6, ws = gstride() >> 6;
  for (int64_t k = w0; k < np; k += ws) {
    uint32_t x;
    int32_t k0, k1;
    touched_piece(D, nt, k, x, k0, k1);
    const uint32_t* row = D.P.col + D.P.off[x];
    const int64_t dbx = D.dd[2 * (int64_t)x] - 1, dax = D.dd[2 * (int64_t)x + 1] - 1;
    int64_t acc = 0;
    for (int32_t q = k0 + l; q < k1; q += 64) {
      const uint32_t e = row[q], y = e & GC_ID, f = nib(e);
      if (D.mark[y] && y < x) continue;
      if ((f & 2u) == 0) acc += dax * (deg_of(D, y, 1) - 1);
      if ((f & 1u) == 0) acc -= dbx * (deg_of(D, y, 0) - 1);
    }
    add_sig(D, D.gid[x], SG_S2, acc);
  }
}

// ---------------------------------------------- triangles and 4-cliques
// One workgroup per changed edge e = (u, v) at a time (a queue over the
// changed edges).  S(e) = N(u) & N(v) in the union view: the shorter row's
// entries are searched in the longer row.  Each w in S(e) gives the affected
// edges (u, w), (v, w) and is marked in the workgroup's dense slot with the
// nibbles of (u, w) and (v, w).  Then every pair {w, x} of S(e) joined by an
// edge closes a 4-clique {u, v, w, x}: for each w, the shorter of its row
// above w and S(e) is tested against the other.
// 4-cliques {u, v, w, x} through the changed edge (u, v) (key K, nibble fe)
// for the common neighbours w = S[i], i in [i0, i1) (one wave per w, the
// workgroup's waves in turn): x runs over S(e) above w, joined to w by an
// edge; S(e) is marked in `mark` (a byte per vertex: bit 7, the nibble of
// (u, x) in bits 0-1 and of (v, x) in bits 2-3) and listed in S (ids, flag
// bits above them ignored).  Returns this lane's share of the sum.
__device__ int64_t k4_through(const DeltaArgs& D, const uint8_t* mark, const uint32_t* S, int32_t ns, int32_t i0,
                              int32_t i1, uint32_t u, uint32_t v, unsigned long long K, uint32_t fe) {
  int64_t k4 = 0;
  for (int32_t i = i0 + (int32_t)(threadIdx.x >> 6); i < i1; i += (int32_t)(blockDim.x >> 6)) {
    const uint32_t w = S[i] & GC_ID;
    const uint32_t mw = mark[w];
    const uint32_t* wrow = D.P.col + D.P.off[w];
    const int32_t wl = D.P.len[w];
    const int32_t above = lower_bound_id(wrow, wl, w + 1);
    const int32_t nab = wl - above;
    int64_t acc = 0;
    auto clique = [&](uint32_t x, uint32_t fwx, uint32_t mx) {
      const uint32_t fuw = mw & 3u, fvw = (mw >> 2) & 3u;
      const uint32_t fux = mx & 3u, fvx = (mx >> 2) & 3u;
      // counted from the changed edge of smallest key only
      if ((fuw && pkey(u, w, D.bits) < K) || (fvw && pkey(v, w, D.bits) < K) || (fux && pkey(u, x, D.bits) < K) ||
          (fvx && pkey(v, x, D.bits) < K) || (fwx && pkey(w, x, D.bits) < K))
        return;
      acc += delta_of(fe | fuw | fvw | fux | fvx | fwx);
    };
    if (nab <= ns) {
      for (int32_t k = above + lane_id(); k < wl; k += 64) {
        const uint32_t ex = wrow[k], x = ex & GC_ID;
        const uint32_t mx = mark[x];
        if (mx) clique(x, nib(ex), mx);
      }
    } else {
      for (int32_t j = lane_id(); j < ns; j += 64) {
        const uint32_t x = S[j] & GC_ID;
        if (x <= w) continue;
        const int32_t p = lower_bound_id(wrow, wl, x);
        if (p < wl && (wrow[p] & GC_ID) == x) clique(x, nib(wrow[p]), mark[x]);
      }
    }
    k4 += acc;
  }
  return k4;
}

__global__ __launch_bounds__(TPB) void k_delta_tri(DeltaArgs D) {
  __shared__ int64_t item_s, split_s;
  __shared__ int32_t ns_s;
  const int64_t ne = min(ctr(D.dc, DC_EDGES), D.ce_cap);
  // marks of S(e), one byte per vertex (bit 7 set, the nibbles of (u, w) and
  // (v, w) in bits 0-1 and 2-3) in the first N bytes of the workgroup's
  // slot (denser than a word per vertex for the random reads of the
  // 4-clique step); all zero again when the kernel ends
  uint8_t* mark = (uint8_t*)(D.slot_mark + (int64_t)blockIdx.x * D.N);
  uint32_t* S = D.slot_list + (int64_t)blockIdx.x * D.slot_cap;
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  int64_t k4acc = 0;
  int cur_g = -1;
  while (true) {
    __syncthreads();
    if (threadIdx.x == 0) { item_s = (int64_t)atomicAdd(&D.dc[DC_QTRI], 1ull); ns_s = 0; }
    __syncthreads();
    const int64_t it = item_s;
    if (it >= ne) break;
    const unsigned long long ek = D.ce[it];
    const unsigned long long K = ek & DIR_KEY_MASK;
    const uint32_t fe = (uint32_t)(ek >> DIR_MASK_SHIFT) & 3u;
    const uint32_t u = (uint32_t)(K >> D.bits), v = (uint32_t)(K & idmask);
    const int g = D.gid[u];
    if (g != cur_g) {
      if (cur_g >= 0) add_sig(D, cur_g, SG_K4, k4acc);
      k4acc = 0;
      cur_g = g;
    }
    const uint32_t s = D.P.len[u] <= D.P.len[v] ? u : v, o = s == u ? v : u;
    const uint32_t* srow = D.P.col + D.P.off[s];
    const int32_t sl = D.P.len[s];
    if (sl > D.slot_cap) {  // more common neighbours possible than the slot holds: count again with more
      if (threadIdx.x == 0) { atomicAdd(&D.bstats[BS_RETRY], 1ull); atomicMax(&D.dc[DC_SLOT_NEED], (unsigned long long)sl); }
      continue;
    }
    for (int32_t k = threadIdx.x; k < sl; k += blockDim.x) {
      const uint32_t es = srow[k], w = es & GC_ID;
      if (w == o) continue;
      const int64_t p = find_in_row(D.P, o, w);
      if (p < 0) continue;
      const uint32_t eo = D.P.col[p];
      const uint32_t fu = nib(s == u ? es : eo), fv = nib(s == u ? eo : es);
      mark[w] = (uint8_t)(0x80u | fu | (fv << 2));
      S[atomicAdd(&ns_s, 1)] = w;
      // affected edges (u, w), (v, w)
      const unsigned long long q = atomicAdd(&D.dc[DC_AFF], 2ull);
      if ((int64_t)q + 1 < D.ae_cap) { D.ae[q] = pkey(u, w, D.bits); D.ae[q + 1] = pkey(v, w, D.bits); }
    }
    __syncthreads();
    const int32_t ns = ns_s;
    // an edge with many common neighbours hands its 4-cliques to
    // k_delta_k4_split in chunks (when the fixed buffers hold it)
    if (ns >= K4_HEAVY_MIN) {
      if (threadIdx.x == 0) {
        const int32_t nch = (ns + K4_CHUNK - 1) / K4_CHUNK;
        int64_t off = (int64_t)atomicAdd(&D.dc[DC_HS], (unsigned long long)ns);
        bool ok = off + ns <= K4_HS_CAP;
        int64_t first = -1;
        if (ok) {
          first = (int64_t)atomicAdd(&D.dc[DC_HITEMS], (unsigned long long)nch);
          if (first + nch > K4_IT_CAP) {
            for (int64_t t = first; t < min(first + nch, K4_IT_CAP); ++t) D.k4_item[2 * t] = -1;
            ok = false;
          }
        }
        if (ok) {
          const int64_t h = (int64_t)atomicAdd(&D.dc[DC_HEAVY], 1ull);
          if (h >= K4_HE_CAP) {
            for (int64_t t = first; t < first + nch; ++t) D.k4_item[2 * t] = -1;
            ok = false;
          } else {
            D.k4_edge[3 * h] = it;
            D.k4_edge[3 * h + 1] = off;
            D.k4_edge[3 * h + 2] = ns;
            for (int32_t c = 0; c < nch; ++c) {
              D.k4_item[2 * (first + c)] = (int32_t)h;
              D.k4_item[2 * (first + c) + 1] = c;
            }
            atomicAdd(&D.bstats[BS_K4_SPLIT], 1ull);
          }
        }
        split_s = ok ? off : -1;
      }
      __syncthreads();
    } else if (threadIdx.x == 0) {
      split_s = -1;
    }
    __syncthreads();
    const int64_t off = split_s;
    if (off >= 0) {
      for (int32_t i = threadIdx.x; i < ns; i += blockDim.x) {
        const uint32_t w = S[i], m = mark[w];
        D.k4_s[off + i] = w | ((m & 3u) << 28) | (((m >> 2) & 3u) << 30);
      }
    } else {
      k4acc += k4_through(D, mark, S, ns, 0, ns, u, v, K, fe);
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < ns; i += blockDim.x) mark[S[i]] = 0;
  }
  if (cur_g >= 0) add_sig(D, cur_g, SG_K4, k4acc);
}

// The 4-cliques of the edges k_delta_tri split: each workgroup takes chunks
// of K4_CHUNK common neighbours from a queue, marks the edge's common
// neighbours in its own slot (kept while the next chunk is of the same
// edge) and counts the chunk's 4-cliques; the slot is clear on return.
__global__ __launch_bounds__(TPB) void k_delta_k4_split(DeltaArgs D) {
  if (D.bstats[BS_RETRY]) return;
  __shared__ int64_t item_s;
  const int64_t nit = min((int64_t)ctr(D.dc, DC_HITEMS), K4_IT_CAP);
  uint8_t* mark = (uint8_t*)(D.slot_mark + (int64_t)blockIdx.x * D.N);
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  int64_t k4acc = 0;
  int cur_g = -1;
  int32_t cur_h = -1, cur_ns = 0;
  const uint32_t* cur_S = nullptr;
  while (true) {
    __syncthreads();
    if (threadIdx.x == 0) item_s = (int64_t)atomicAdd(&D.dc[DC_QK4], 1ull);
    __syncthreads();
    const int64_t t = item_s;
    if (t >= nit) break;
    const int32_t h = D.k4_item[2 * t], c = D.k4_item[2 * t + 1];
    if (h < 0) continue;
    const int64_t i = D.k4_edge[3 * h], off = D.k4_edge[3 * h + 1];
    const int32_t ns = (int32_t)D.k4_edge[3 * h + 2];
    const uint32_t* Sh = D.k4_s + off;
    if (h != cur_h) {
      for (int32_t j = threadIdx.x; j < cur_ns; j += blockDim.x) mark[cur_S[j] & GC_ID] = 0;
      __syncthreads();
      for (int32_t j = threadIdx.x; j < ns; j += blockDim.x) {
        const uint32_t e = Sh[j];
        mark[e & GC_ID] = (uint8_t)(0x80u | ((e >> 28) & 3u) | (((e >> 30) & 3u) << 2));
      }
      __syncthreads();
      cur_h = h;
      cur_ns = ns;
      cur_S = Sh;
    }
    const unsigned long long ek = D.ce[i];
    const unsigned long long K = ek & DIR_KEY_MASK;
    const uint32_t fe = (uint32_t)(ek >> DIR_MASK_SHIFT) & 3u;
    const uint32_t u = (uint32_t)(K >> D.bits), v = (uint32_t)(K & idmask);
    const int g = D.gid[u];
    if (g != cur_g) {
      if (cur_g >= 0) add_sig(D, cur_g, SG_K4, k4acc);
      k4acc = 0;
      cur_g = g;
    }
    k4acc += k4_through(D, mark, Sh, ns, c * K4_CHUNK, min(ns, (c + 1) * K4_CHUNK), u, v, K, fe);
  }
  __syncthreads();
  for (int32_t j = threadIdx.x; j < cur_ns; j += blockDim.x) mark[cur_S[j] & GC_ID] = 0;
  if (cur_g >= 0) add_sig(D, cur_g, SG_K4, k4acc);
}

// ------------------------------------------------------- affected edges
// The changed edges join the affected list (after the triangle kernel, so
// its count is final), then the list is sorted and each distinct edge
// (x, y) is taken by one wave: t before / after from the intersection of
// its rows, presence from its own entry.
__global__ void k_delta_aff_changed(DeltaArgs D) {
  if (D.bstats[BS_RETRY]) return;
  const int64_t ne = min(ctr(D.dc, DC_EDGES), D.ce_cap);
  const int64_t base = (int64_t)D.dc[DC_AFF];
  for (int64_t i = gtid(); i < ne; i += gstride()) {
    const int64_t q = base + i;
    if (q < D.ae_cap) D.ae[q] = D.ce[i] & DIR_KEY_MASK;
  }
  if (gtid() == 0) {
    const int64_t tot = base + ne;
    D.dc[DC_AFF_TOTAL] = (unsigned long long)(tot < D.ae_cap ? tot : D.ae_cap);
    if (tot > D.ae_cap) {
      atomicAdd(&D.bstats[BS_RETRY], 1ull);
      atomicMax(&D.dc[DC_AFF_NEED], (unsigned long long)tot);
    }
  }
}

__global__ void k_delta_aff(DeltaArgs D, const unsigned long long* __restrict__ keys) {
  if (D.bstats[BS_RETRY]) return;
  const int64_t na = ctr(D.dc, DC_AFF_TOTAL);
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  const int l = lane_id();
  int64_t s3 = 0, s4 = 0, s5 = 0;
  int cur_g = -1;
  const int64_t nwv = gstride() >> 6;
  for (int64_t i = gtid() >> 6; i < na; i = wave_next(&D.dc[DC_QAFF], nwv)) {
    const unsigned long long key = keys[i];
    if (i > 0 && keys[i - 1] == key) continue;
    const uint32_t x = (uint32_t)(key >> D.bits), y = (uint32_t)(key & idmask);
    const int g = D.gid[x];
    if (g != cur_g) {
      if (cur_g >= 0) { add_sig(D, cur_g, SG_T, s3); add_sig(D, cur_g, SG_DIA, s4); add_sig(D, cur_g, SG_PAW, s5); }
      s3 = s4 = s5 = 0;
      cur_g = g;
    }
    const uint32_t a = D.P.len[x] <= D.P.len[y] ? x : y, b = a == x ? y : x;
    const uint32_t* arow = D.P.col + D.P.off[a];
    const int32_t al = D.P.len[a], bl = D.P.len[b];
    int32_t tb = 0, ta = 0;
    if (al > 0 && (int64_t)bl <= (int64_t)al * ((30 - __clz(max(bl, 1))) / 2)) {
      // rows of similar length (as for the 4-cycle pairs): both walked
      // together, 64 entries of each a step, instead of a search of the
      // longer row per entry of the shorter
      wave_window_common(D.P.col, D.P.off[a], al, D.P.off[b], bl, [&](uint32_t ea, uint32_t eb) {
        const uint32_t f = nib(ea) | nib(eb);
        tb += (f & 1u) == 0;
        ta += (f & 2u) == 0;
      });
    } else {
      // the shorter row's entries searched in the longer
      for (int32_t k = l; k < al; k += 64) {
        const uint32_t ea = arow[k], w = ea & GC_ID;
        if (w == b) continue;
        const int64_t p = find_in_row(D.P, b, w);
        if (p < 0) continue;
        const uint32_t f = nib(ea) | nib(D.P.col[p]);
        tb += (f & 1u) == 0;
        ta += (f & 2u) == 0;
      }
    }
    tb = wave_sum32(tb);
    ta = wave_sum32(ta);
    if (l == 0) {
      const int64_t p = find_in_row(D.P, x, y);
      const uint32_t f = p >= 0 ? nib(D.P.col[p]) : 3u;
      const int64_t pb = (f & 1u) == 0, pa = (f & 2u) == 0;
      const int64_t tbp = pb * tb, tap = pa * ta;
      s3 += tap - tbp;
      s4 += pa * c2(ta) - pb * c2(tb);
      s5 += tap * (deg_of(D, x, 1) + deg_of(D, y, 1) - 4) - tbp * (deg_of(D, x, 0) + deg_of(D, y, 0) - 4);
      // twice the change of T at both ends; t before on the affected edges at a touched end
      if (tap != tbp) { atomicAdd(&D.dT[x], (unsigned long long)(tap - tbp)); atomicAdd(&D.dT[y], (unsigned long long)(tap - tbp)); }
      if (tbp) {
        if (D.mark[x]) atomicAdd(&D.sbt[x], (unsigned long long)tbp);
        if (D.mark[y]) atomicAdd(&D.sbt[y], (unsigned long long)tbp);
      }
    }
  }
  if (cur_g >= 0) {
    // sums are held by lane 0 only: the wave sums add zeros from the others
    add_sig(D, cur_g, SG_T, s3); add_sig(D, cur_g, SG_DIA, s4); add_sig(D, cur_g, SG_PAW, s5);
  }
}

// At a touched vertex x whose degree changed, the edges that are not
// affected keep their t and present in both versions; their share of the
// paw term changes by t (d_a(x) - d_b(x)), and their t sum is 2 T(x) minus
// the t before of the affected edges at x.
__global__ void k_delta_vertex2(DeltaArgs D) {
  if (D.bstats[BS_RETRY]) return;
  const int64_t nt = ctr(D.c, C_TOUCH);
  for (int64_t t = gtid(); t < nt; t += gstride()) {
    const uint32_t x = (uint32_t)D.touched[t];
    const int64_t dd = (int64_t)D.dd[2 * (int64_t)x + 1] - D.dd[2 * (int64_t)x];
    const int64_t sb = (int64_t)D.sbt[x];
    D.sbt[x] = 0ull;
    if (dd) {
      const int64_t v = dd * (2 * D.Tv[x] - sb);
      atomicAdd(&D.sig[SIG_IDX(D.gid[x], 1, SG_PAW)], (unsigned long long)v);
    }
  }
}

// T(v) after the batch: every affected edge's ends take their share once.
__global__ void k_delta_tv(DeltaArgs D, const unsigned long long* __restrict__ keys) {
  if (D.bstats[BS_RETRY]) return;
  const int64_t na = ctr(D.dc, DC_AFF_TOTAL);
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  for (int64_t i = gtid(); i < na; i += gstride()) {
    const unsigned long long key = keys[i];
    const uint32_t ends[2] = {(uint32_t)(key >> D.bits), (uint32_t)(key & idmask)};
    for (uint32_t x : ends) {
      const long long d2 = (long long)atomicExch(&D.dT[x], 0ull);
      if (d2) {
        if (d2 & 1) atomicAdd(&D.bstats[BS_ERR], 1ull);
        atomicAdd((unsigned long long*)&D.Tv[x], (unsigned long long)(d2 / 2));
      }
    }
  }
}

// ------------------------------------------------------------- 4-cycles
// Through a changed edge e = (s, o) run the 4-cycles s - a - b - o with
// a in N(s) - {o}, b in N(a) & N(o) - {s}.  Per pair (s, a) the shorter of
// N(a) and N(o) is walked and each entry searched in the other row, so a hub
// on either side costs at most the other side's degree; s is the end with
// the smaller sum over its neighbours a of min(d_a, d_o).  The work is
// balanced over the whole chip: every pair (e, a) gets its walk length, a
// scan places the walked entries of all pairs in one index space, and each
// lane takes entries of that space (a hub pair is spread over many waves).

// per changed edge: the end to walk from and its number of pairs.  The
// walk of an end u costs sum_{a in N(u)} min(d_a, d_v); both rows of every
// changed edge are cut in pieces of at most TV_CHUNK entries (the touched
// rows' arrays hold the numbering; they are free again after the degree
// passes), each wave sums one piece at a time into the edge's two totals
// (kept in pair_off, free until the pair scan), and a last pass picks the
// cheaper end.
__global__ void k_delta_plan_items(DeltaArgs D) {
  const int64_t ne = min(ctr(D.dc, DC_EDGES), D.ce_cap);
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  for (int64_t i = gtid(); i < D.tcap; i += gstride()) {
    int32_t n = 0;
    if (i < ne) {
      const unsigned long long K = D.ce[i] & DIR_KEY_MASK;
      const uint32_t u = (uint32_t)(K >> D.bits), v = (uint32_t)(K & idmask);
      n = max(1, (D.P.len[u] + TV_CHUNK - 1) / TV_CHUNK) + max(1, (D.P.len[v] + TV_CHUNK - 1) / TV_CHUNK);
      D.pair_off[2 * i] = 0;
      D.pair_off[2 * i + 1] = 0;
    }
    D.tv_items[i] = n;
  }
}

__global__ void k_delta_c4_plan(DeltaArgs D) {
  const int64_t ne = min(ctr(D.dc, DC_EDGES), D.ce_cap);
  if (ne == 0) return;
  const int64_t np = D.tv_ioff[ne];
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  const int l = lane_id();
  const int64_t w0 = gtid() >> 6, ws = gstride() >> 6;
  for (int64_t k = w0; k < np; k += ws) {
    int64_t lo = 0, hi = ne;  // the edge holding piece k
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (D.tv_ioff[mid] <= k) lo = mid; else hi = mid;
    }
    const int64_t i = lo;
    const unsigned long long K = D.ce[i] & DIR_KEY_MASK;
    const uint32_t u = (uint32_t)(K >> D.bits), v = (uint32_t)(K & idmask);
    const int32_t du = D.P.len[u], dv = D.P.len[v];
    const int64_t nu = max(1, (du + TV_CHUNK - 1) / TV_CHUNK);
    const int64_t pk = k - D.tv_ioff[i];
    const bool side_v = pk >= nu;  // pieces of u first, then of v
    const uint32_t x = side_v ? v : u;
    const int32_t dx = side_v ? dv : du, other = side_v ? du : dv;
    const int32_t k0 = (int32_t)((side_v ? pk - nu : pk) * TV_CHUNK), k1 = min(dx, k0 + TV_CHUNK);
    const uint32_t* rx = D.P.col + D.P.off[x];
    int64_t c = 0;
    for (int32_t q = k0 + l; q < k1; q += 64) c += min((int64_t)D.P.len[rx[q] & GC_ID], (int64_t)other);
    c = wave_sum64(c);
    if (l == 0 && c) atomicAdd((unsigned long long*)&D.pair_off[2 * i + (side_v ? 1 : 0)], (unsigned long long)c);
  }
}

__global__ void k_delta_plan_fin(DeltaArgs D) {
  const int64_t ne = min(ctr(D.dc, DC_EDGES), D.ce_cap);
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  for (int64_t i = gtid(); i < D.ce_cap; i += gstride()) {
    if (i >= ne) {
      D.c4_nch[i] = 0;
      D.c4_side[i] = 0;
      continue;
    }
    const unsigned long long K = D.ce[i] & DIR_KEY_MASK;
    const uint32_t u = (uint32_t)(K >> D.bits), v = (uint32_t)(K & idmask);
    const bool from_u = D.pair_off[2 * i] <= D.pair_off[2 * i + 1];
    D.c4_side[i] = from_u ? 0 : 1;
    D.c4_nch[i] = from_u ? D.P.len[u] : D.P.len[v];
  }
}

// per pair (e, a): its position and its walk length min(d_a, d_o)
__global__ void k_delta_c4_pairs(DeltaArgs D) {
  const int64_t ne = min(ctr(D.dc, DC_EDGES), D.ce_cap);
  const int64_t npairs = D.c4_off[D.ce_cap];
  if (gtid() == 0 && npairs > D.pair_cap) {
    atomicAdd(&D.bstats[BS_RETRY], 1ull);
    atomicMax(&D.dc[DC_PAIR_NEED], (unsigned long long)npairs);
  }
  if (npairs > D.pair_cap) return;
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  const int l = lane_id();
  const int64_t w0 = gtid() >> 6, ws = gstride() >> 6;
  for (int64_t i = w0; i < ne; i += ws) {
    const unsigned long long K = D.ce[i] & DIR_KEY_MASK;
    const uint32_t u = (uint32_t)(K >> D.bits), v = (uint32_t)(K & idmask);
    const uint32_t s = D.c4_side[i] ? v : u, o = s == u ? v : u;
    const uint32_t* srow = D.P.col + D.P.off[s];
    const int32_t sl = D.P.len[s], ol = D.P.len[o];
    const int64_t base = D.c4_off[i];
    for (int32_t k = l; k < sl; k += 64) {
      const uint32_t a = srow[k] & GC_ID;
      const int32_t al = D.P.len[a];
      const int32_t mn = min(al, ol), mx = max(al, ol);
      D.pair_edge[base + k] = (int32_t)i;
      // rows of similar length (the longer at most (log2 of it - 1) / 2
      // times the shorter, the best split measured) are merged by a wave;
      // of the others, a shorter N(a) against an N(o) small enough for an
      // LDS hash table is walked against the table (k_delta_c4_hash), and
      // the rest walk the shorter row and search the longer, lane by lane
      const bool merge = a != o && mn > 0 && (int64_t)mx <= (int64_t)mn * ((30 - __clz(max(mx, 1))) / 2);
      const bool hashed = !merge && a != o && al > 0 && al < ol && ol <= C4H_MAX;
      D.pair_len[base + k] = a == o || merge || hashed ? 0 : mn;
      D.pair_hlen[base + k] = hashed ? al : 0;
      if (merge) D.pair_merge[atomicAdd(&D.dc[DC_MERGE], 1ull)] = (int32_t)(base + k);
    }
  }
}

__global__ __launch_bounds__(TPB) void k_delta_c4(DeltaArgs D) {
  if (D.bstats[BS_RETRY]) return;
  const int64_t npairs = D.c4_off[D.ce_cap];
  const int64_t total = D.pair_off[npairs];
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  const int l = lane_id();
  // each wave takes one contiguous range of whole 64-entry chunks of the
  // index space (equal ranges: balanced by construction); its lanes walk
  // entries f = chunk * 64 + lane, so a lane's pair only moves forward and
  // is found by stepping, and the pair's row data is loaded once per pair
  const int64_t nchunk = (total + 63) >> 6, nw = gstride() >> 6;
  const int64_t per = (nchunk + nw - 1) / nw;
  const int64_t c0 = (gtid() >> 6) * per, c1 = min(nchunk, c0 + per);
  int64_t acc = 0;
  int cur_g = -1;
  if (c0 < c1) {
    // the pair holding the range's first entry: largest p with
    // pair_off[p] <= f (empty pairs share their offset with the next)
    const int64_t fs = c0 << 6;
    int64_t p = 0;
    {
      int64_t lo = 0, hi = npairs;
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (D.pair_off[mid] <= fs) lo = mid; else hi = mid;
      }
      p = lo;
    }
    int64_t pend = D.pair_off[p + 1], pbeg = D.pair_off[p];
    bool fresh = true;
    // the current pair's data
    unsigned long long K = 0;
    uint32_t fe = 0, s = 0, o = 0, eaj = 0, a = 0, fsa = 0;
    const uint32_t* orow = nullptr;
    const uint32_t* arow = nullptr;
    int32_t ol = 0, al = 0;
    int g = 0;
    for (int64_t c = c0; c < c1; ++c) {
      const int64_t f = (c << 6) + l;
      if (f >= total) break;
      while (pend <= f) {
        ++p;
        pbeg = pend;
        pend = D.pair_off[p + 1];
        fresh = true;
      }
      if (fresh) {
        fresh = false;
        const int32_t i = D.pair_edge[p];
        const unsigned long long ek = D.ce[i];
        K = ek & DIR_KEY_MASK;
        fe = (uint32_t)(ek >> DIR_MASK_SHIFT) & 3u;
        const uint32_t u = (uint32_t)(K >> D.bits), v = (uint32_t)(K & idmask);
        s = D.c4_side[i] ? v : u;
        o = s == u ? v : u;
        eaj = D.P.col[D.P.off[s] + (p - D.c4_off[i])];
        a = eaj & GC_ID;
        fsa = nib(eaj);
        orow = D.P.col + D.P.off[o];
        arow = D.P.col + D.P.off[a];
        ol = D.P.len[o];
        al = D.P.len[a];
        g = D.gid[u];
      }
      const int32_t q = (int32_t)(f - pbeg);
      uint32_t b, fab = 0, fob = 0;
      bool hit;
      if (al <= ol) {  // walk N(a), search N(o)
        const uint32_t eab = arow[q];
        b = eab & GC_ID;
        fab = nib(eab);
        const int32_t x = lower_bound_id(orow, ol, b);
        hit = x < ol && (orow[x] & GC_ID) == b;
        if (hit) fob = nib(orow[x]);
      } else {         // walk N(o), search N(a)
        const uint32_t eob = orow[q];
        b = eob & GC_ID;
        fob = nib(eob);
        const int32_t x = lower_bound_id(arow, al, b);
        hit = x < al && (arow[x] & GC_ID) == b;
        if (hit) fab = nib(arow[x]);
      }
      if (hit && b != s) {
        const bool skip = (fsa && pkey(s, a, D.bits) < K) || (fab && pkey(a, b, D.bits) < K) ||
                          (fob && pkey(o, b, D.bits) < K);
        if (!skip) {
          if (g != cur_g) {
            if (cur_g >= 0 && acc) atomicAdd(&D.sig[SIG_IDX(cur_g, 1, SG_C4)], (unsigned long long)acc);
            acc = 0;
            cur_g = g;
          }
          acc += delta_of(fe | fsa | fab | fob);
        }
      }
    }
  }
  // one atomic per wave when its lanes hold sums of one graph
  const uint64_t has = __ballot(cur_g >= 0 && acc != 0);
  if (has) {
    const int gl = __shfl(cur_g, __builtin_ctzll(has));
    if (__ballot(acc != 0 && cur_g != gl) == 0) {
      const int64_t t = wave_sum64(acc);
      if (lane_id() == 0 && t) atomicAdd(&D.sig[SIG_IDX(gl, 1, SG_C4)], (unsigned long long)t);
    } else if (acc) {
      atomicAdd(&D.sig[SIG_IDX(cur_g, 1, SG_C4)], (unsigned long long)acc);
    }
  }
}

// The pairs (e, a) whose rows N(a) and N(o) have similar lengths: one wave
// per pair merges both rows (wave_window_common); each common b != s closes
// the path s - a - b - o.
__global__ __launch_bounds__(TPB) void k_delta_c4_merge(DeltaArgs D) {
  if (D.bstats[BS_RETRY]) return;
  const int64_t nm = ctr(D.dc, DC_MERGE);
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  int64_t acc = 0;
  int cur_g = -1;
  const int64_t nwv = gstride() >> 6;
  for (int64_t m = gtid() >> 6; m < nm; m = wave_next(&D.dc[DC_QMERGE], nwv)) {
    const int64_t p = D.pair_merge[m];
    const int32_t i = D.pair_edge[p];
    const unsigned long long ek = D.ce[i];
    const unsigned long long K = ek & DIR_KEY_MASK;
    const uint32_t fe = (uint32_t)(ek >> DIR_MASK_SHIFT) & 3u;
    const uint32_t u = (uint32_t)(K >> D.bits), v = (uint32_t)(K & idmask);
    const uint32_t s = D.c4_side[i] ? v : u, o = s == u ? v : u;
    const uint32_t eaj = D.P.col[D.P.off[s] + (p - D.c4_off[i])], a = eaj & GC_ID;
    const uint32_t fsa = nib(eaj);
    const int g = D.gid[u];
    if (g != cur_g) {
      // the wave's graph changes: flush per lane (wave-uniform branch)
      if (cur_g >= 0 && acc) atomicAdd(&D.sig[SIG_IDX(cur_g, 1, SG_C4)], (unsigned long long)acc);
      acc = 0;
      cur_g = g;
    }
    wave_window_common(D.P.col, D.P.off[a], D.P.len[a], D.P.off[o], D.P.len[o],
                       [&](uint32_t eab, uint32_t eob) {
                         const uint32_t b = eab & GC_ID;
                         if (b == s) return;
                         const uint32_t fab = nib(eab), fob = nib(eob);
                         const bool skip = (fsa && pkey(s, a, D.bits) < K) || (fab && pkey(a, b, D.bits) < K) ||
                                           (fob && pkey(o, b, D.bits) < K);
                         if (!skip) acc += delta_of(fe | fsa | fab | fob);
                       });
  }
  if (cur_g >= 0) {
    const int64_t t = wave_sum64(acc);
    if (lane_id() == 0 && t) atomicAdd(&D.sig[SIG_IDX(cur_g, 1, SG_C4)], (unsigned long long)t);
  }
}

// Entries of the walked rows per chunk of hashed pairs: at least
// C4H_CHUNK_MIN and four times |N(o)|, so that building the table of N(o)
// costs at most a quarter of a chunk.
__device__ __forceinline__ int64_t c4h_chunk(int32_t ol) { return max(C4H_CHUNK_MIN, 4 * (int64_t)ol); }

// Chunks of the hashed pairs per changed edge (0 past the edge count, for
// the scan).
__global__ void k_delta_hitems(DeltaArgs D) {
  const int64_t ne = min(ctr(D.dc, DC_EDGES), D.ce_cap);
  const bool fits = D.c4_off[D.ce_cap] <= D.pair_cap;  // else the pairs were not listed (count again)
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  for (int64_t i = gtid(); i < D.tcap; i += gstride()) {
    int32_t n = 0;
    if (i < ne && fits) {
      const int64_t h = D.pair_hoff[D.c4_off[i + 1]] - D.pair_hoff[D.c4_off[i]];
      if (h > 0) {
        const unsigned long long K = D.ce[i] & DIR_KEY_MASK;
        const uint32_t u = (uint32_t)(K >> D.bits), v = (uint32_t)(K & idmask);
        const uint32_t o = D.c4_side[i] ? u : v;
        const int64_t T = c4h_chunk(D.P.len[o]);
        n = (int32_t)((h + T - 1) / T);
      }
    }
    D.tv_items[i] = n;
  }
}

// The hashed pairs (e, a): each workgroup takes chunks from a queue, builds
// an LDS hash table of N(o) for the chunk's edge (kept while the next chunk
// is of the same edge): id, the nibble of (o, b), and whether (o, b) is a
// changed pair of smaller key than e (such paths are counted from that
// pair).  Its waves split the chunk's entries in contiguous pieces; a lane
// steps through the pairs of its piece and probes the table with each entry
// b of N(a): a hit with b != s closes the path s - a - b - o.
__global__ __launch_bounds__(C4H_T) void k_delta_c4_hash(DeltaArgs D) {
  __shared__ uint32_t tab[C4H_SLOTS];
  __shared__ int64_t item_s;
  if (D.bstats[BS_RETRY]) return;
  const int64_t ne = min(ctr(D.dc, DC_EDGES), D.ce_cap);
  if (ne == 0) return;
  const int64_t nitems = D.tv_ioff[ne];
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  const int32_t l = lane_id(), wv = (int32_t)(threadIdx.x >> 6), nwv = (int32_t)(blockDim.x >> 6);
  constexpr uint32_t EMPTY = 0xFFFFFFFFu;
  int64_t acc = 0;
  int cur_g = -1;
  int64_t cur_i = -1;
  while (true) {
    __syncthreads();
    if (threadIdx.x == 0) item_s = (int64_t)atomicAdd(&D.dc[DC_QH], 1ull);
    __syncthreads();
    const int64_t it = item_s;
    if (it >= nitems) break;
    int64_t lo = 0, hi = ne;  // the item's edge: largest i with tv_ioff[i] <= it
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (D.tv_ioff[mid] <= it) lo = mid; else hi = mid;
    }
    const int64_t i = lo;
    const unsigned long long ek = D.ce[i];
    const unsigned long long K = ek & DIR_KEY_MASK;
    const uint32_t fe = (uint32_t)(ek >> DIR_MASK_SHIFT) & 3u;
    const uint32_t u = (uint32_t)(K >> D.bits), v = (uint32_t)(K & idmask);
    const uint32_t s = D.c4_side[i] ? v : u, o = s == u ? v : u;
    const int32_t ol = D.P.len[o];  // <= C4H_MAX: the edge has hashed pairs
    int tb = 8;  // table of 2^tb slots: at least 4 |N(o)| where LDS allows
    while ((1 << tb) < 4 * ol && (1 << tb) < C4H_SLOTS) ++tb;
    const uint32_t tmask = (1u << tb) - 1u;
    if (i != cur_i) {
      for (int32_t k = (int32_t)threadIdx.x; k <= (int32_t)tmask; k += (int32_t)blockDim.x) tab[k] = EMPTY;
      __syncthreads();
      const uint32_t* orow = D.P.col + D.P.off[o];
      for (int32_t k = (int32_t)threadIdx.x; k < ol; k += (int32_t)blockDim.x) {
        const uint32_t e = orow[k], b = e & GC_ID, f = nib(e);
        const uint32_t val = b | (f << 28) | ((f && pkey(o, b, D.bits) < K) ? (1u << 30) : 0u);
        uint32_t h = (b * 2654435761u) >> (32 - tb);
        while (atomicCAS(&tab[h], EMPTY, val) != EMPTY) h = (h + 1) & tmask;
      }
      __syncthreads();
      cur_i = i;
    }
    const int g = D.gid[u];
    if (g != cur_g) {
      if (cur_g >= 0) add_sig(D, cur_g, SG_C4, acc);
      acc = 0;
      cur_g = g;
    }
    // the chunk: entries [r0, r1) of the hashed walk index space
    const int64_t p0 = D.c4_off[i], p1 = D.c4_off[i + 1];
    const int64_t T = c4h_chunk(ol);
    const int64_t r0 = D.pair_hoff[p0] + (it - D.tv_ioff[i]) * T, r1 = min(D.pair_hoff[p1], r0 + T);
    const int64_t nst = (r1 - r0 + 63) >> 6, per = (nst + nwv - 1) / nwv;
    const int64_t st0 = wv * per, st1 = min(nst, st0 + per);
    if (st0 >= st1) continue;
    // this lane's first pair: largest p with pair_hoff[p] <= f (pairs
    // walked elsewhere share their offset with the next)
    int64_t f = r0 + (st0 << 6) + l;
    int64_t p = p0;
    {
      int64_t a0 = p0, a1 = p1;
      while (a1 - a0 > 1) {
        const int64_t mid = (a0 + a1) >> 1;
        if (D.pair_hoff[mid] <= f) a0 = mid; else a1 = mid;
      }
      p = a0;
    }
    int64_t pbeg = D.pair_hoff[p], pend = D.pair_hoff[p + 1];
    bool fresh = true;
    const uint32_t* srow = D.P.col + D.P.off[s];
    const uint32_t* arow = nullptr;
    uint32_t a = 0, fsa = 0;
    bool skip_sa = false;
    for (int64_t st = st0; st < st1; ++st) {
      f = r0 + (st << 6) + l;
      if (f >= r1) break;
      while (pend <= f) {
        ++p;
        pbeg = pend;
        pend = D.pair_hoff[p + 1];
        fresh = true;
      }
      if (fresh) {
        fresh = false;
        const uint32_t eaj = srow[p - p0];
        a = eaj & GC_ID;
        fsa = nib(eaj);
        skip_sa = fsa && pkey(s, a, D.bits) < K;
        arow = D.P.col + D.P.off[a];
      }
      const uint32_t eab = arow[f - pbeg], b = eab & GC_ID;
      uint32_t h = (b * 2654435761u) >> (32 - tb), sv;
      while (true) {
        sv = tab[h];
        if (sv == EMPTY || (sv & GC_ID) == b) break;
        h = (h + 1) & tmask;
      }
      if (sv != EMPTY && b != s) {
        const uint32_t fab = nib(eab);
        if (!(skip_sa || (fab && pkey(a, b, D.bits) < K) || ((sv >> 30) & 1u)))
          acc += delta_of(fe | fsa | fab | ((sv >> 28) & 3u));
      }
    }
  }
  if (cur_g >= 0) add_sig(D, cur_g, SG_C4, acc);
}

// ------------------------------------------------ T(v) in the region path
// After the triangle kernels of a region (or whole-graph) pass, t holds the
// triangles of every upper entry (id order) of the region per version.  A
// changed triangle at v lies inside the region and sits on two edges at v,
// so T(v) moves by half the change of t summed over the edges at v: each
// upper entry hands its change to both ends, then each region vertex takes
// its half once.
template <int NV>
__global__ void k_tv_entries(RegionDev R, const unsigned long long* c, unsigned long long* __restrict__ dT,
                             const unsigned long long* bstats) {
  if (bstats[BS_RETRY]) return;
  const int64_t ne = ctr(c, C_ER);
  for (int64_t p = gtid(); p < ne; p += gstride()) {
    const uint32_t w = R.rcol[p] & GC_ID;
    const int32_t v = R.rrow[p];
    if ((int64_t)w <= (int64_t)v) continue;
    int64_t d;
    if constexpr (NV == 2) {
      const unsigned long long x = R.t[p];
      d = (int64_t)(x >> 32) - (int64_t)(x & 0xFFFFFFFFull);
    } else {
      // t_x = t[p] + field x of tp[2p] (x = 0, 1) and tp[2p + 1] (x = 2, 3)
      d = (int64_t)(R.tp[2 * p + 1] >> 32) - (int64_t)(R.tp[2 * p] & 0xFFFFFFFFull);
    }
    if (d) {
      atomicAdd(&dT[v], (unsigned long long)d);
      atomicAdd(&dT[w], (unsigned long long)d);
    }
  }
}

__global__ void k_tv_apply(const int32_t* __restrict__ rlist, const unsigned long long* c,
                           unsigned long long* __restrict__ dT, long long* __restrict__ Tv,
                           unsigned long long* bstats) {
  if (bstats[BS_RETRY]) return;
  const int64_t nr = ctr(c, C_RLIST);
  for (int64_t i = gtid(); i < nr; i += gstride()) {
    const int32_t v = rlist[i];
    const long long d2 = (long long)atomicExch(&dT[v], 0ull);
    if (d2) {
      if (d2 & 1) atomicAdd(&bstats[BS_ERR], 1ull);
      Tv[v] += d2 / 2;
    }
  }
}

// ---------------------------------------------------------- launchers
void launch_delta(const DeltaArgs& D, int slots, hipStream_t s) {
  fill_u64(D.dc, 0ull, DC_COUNT, s);
  hipLaunchKernelGGL(k_delta_edges, dim3(1024), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_titems, dim3(1024), dim3(TPB), 0, s, D);
  exclusive_scan_i32_to_i64(D.tv_items, D.tv_ioff, D.tcap, D.scan_tmp, s);
  hipLaunchKernelGGL(k_delta_vertex, dim3(2048), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_vertex_fin, dim3(256), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_s2, dim3(2048), dim3(TPB), 0, s, D);
  // every kernel that can find a buffer too small (and raise BS_RETRY)
  // runs before the first one that moves T(v) or clears scratch
  hipLaunchKernelGGL(k_delta_tri, dim3(slots), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_k4_split, dim3(slots), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_aff_changed, dim3(1024), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_plan_items, dim3(1024), dim3(TPB), 0, s, D);
  exclusive_scan_i32_to_i64(D.tv_items, D.tv_ioff, D.tcap, D.scan_tmp, s);
  hipLaunchKernelGGL(k_delta_c4_plan, dim3(2048), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_plan_fin, dim3(256), dim3(TPB), 0, s, D);
  exclusive_scan_i32_to_i64(D.c4_nch, D.c4_off, D.ce_cap, D.scan_tmp, s);
  // every pair below the count c4_off[ce_cap] gets both lengths, and only
  // offsets up to that count are read: no clearing, scans up to the count
  hipLaunchKernelGGL(k_delta_c4_pairs, dim3(1024), dim3(TPB), 0, s, D);
  exclusive_scan_i32_to_i64_count(D.pair_len, D.pair_off, D.pair_cap, D.c4_off + D.ce_cap, D.scan_tmp, s);
  exclusive_scan_i32_to_i64_count(D.pair_hlen, D.pair_hoff, D.pair_cap, D.c4_off + D.ce_cap, D.scan_tmp, s);
  hipLaunchKernelGGL(k_delta_hitems, dim3(256), dim3(TPB), 0, s, D);
  exclusive_scan_i32_to_i64(D.tv_items, D.tv_ioff, D.tcap, D.scan_tmp, s);
  unsigned long long* sorted =
      radix_sort_u64(D.ae, D.ae_alt, D.sort_tmp, D.ae_cap, D.dc + DC_AFF_TOTAL, 2 * D.bits, s);
  hipLaunchKernelGGL(k_delta_aff, dim3(4096), dim3(TPB), 0, s, D, (const unsigned long long*)sorted);
  hipLaunchKernelGGL(k_delta_vertex2, dim3(1024), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_tv, dim3(1024), dim3(TPB), 0, s, D, (const unsigned long long*)sorted);
  hipLaunchKernelGGL(k_delta_c4, dim3(4096), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_c4_merge, dim3(4096), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_c4_hash, dim3(256), dim3(C4H_T), 0, s, D);
}

void launch_tv_region(int nv, const RegionDev& R, const int32_t* rlist, const unsigned long long* c,
                      unsigned long long* dT, long long* Tv, unsigned long long* bstats, hipStream_t s) {
  if (nv == 2)
    hipLaunchKernelGGL(k_tv_entries<2>, dim3(4096), dim3(TPB), 0, s, R, c, dT, (const unsigned long long*)bstats);
  else
    hipLaunchKernelGGL(k_tv_entries<4>, dim3(4096), dim3(TPB), 0, s, R, c, dT, (const unsigned long long*)bstats);
  hipLaunchKernelGGL(k_tv_apply, dim3(2048), dim3(TPB), 0, s, rlist, c, dT, Tv, bstats);
}
