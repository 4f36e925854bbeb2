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
//               e = (s, o), walked from the side with fewer wedges.
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
// One wave per touched row: its degree before and after; the 3-star, wedge
// and degree-sum terms.
__global__ void k_delta_vertex(DeltaArgs D) {
  const int64_t nt = ctr(D.c, C_TOUCH);
  const int l = lane_id();
  const int64_t w0 = gtid() >> 6, ws = gstride() >> 6;
  for (int64_t t = w0; t < nt; t += ws) {
    const uint32_t x = (uint32_t)D.touched[t];
    const uint32_t* row = D.P.col + D.P.off[x];
    const int32_t L = D.P.len[x];
    int32_t db = 0, da = 0;
    for (int32_t k = l; k < L; k += 64) {
      const uint32_t f = nib(row[k]);
      db += (f & 1u) == 0;
      da += (f & 2u) == 0;
    }
    db = wave_sum32(db);
    da = wave_sum32(da);
    if (l == 0) { D.dd[2 * (int64_t)x] = db; D.dd[2 * (int64_t)x + 1] = da; }
    const int g = D.gid[x];
    if (l == 0) {
      const int64_t s1 = c3(da) - c3(db), w2 = c2(da) - c2(db), d1 = (int64_t)da - db;
      if (s1) atomicAdd(&D.sig[SIG_IDX(g, 1, SG_S1)], (unsigned long long)s1);
      if (w2) atomicAdd(&D.sig[SIG_IDX(g, 1, SG_W)], (unsigned long long)w2);
      if (d1) atomicAdd(&D.sig[SIG_IDX(g, 1, SG_D1)], (unsigned long long)d1);
    }
  }
}

// S2 = sum_e (d_u - 1)(d_v - 1) changes only on edges at a touched vertex;
// an edge between two touched vertices is taken at the smaller id.
__global__ void k_delta_s2(DeltaArgs D) {
  const int64_t nt = ctr(D.c, C_TOUCH);
  const int l = lane_id();
  const int64_t w0 = gtid() >> 6, ws = gstride() >> 6;
  for (int64_t t = w0; t < nt; t += ws) {
    const uint32_t x = (uint32_t)D.touched[t];
    const uint32_t* row = D.P.col + D.P.off[x];
    const int32_t L = D.P.len[x];
    const int64_t dbx = D.dd[2 * (int64_t)x] - 1, dax = D.dd[2 * (int64_t)x + 1] - 1;
    int64_t acc = 0;
    for (int32_t k = l; k < L; k += 64) {
      const uint32_t e = row[k], y = e & GC_ID, f = nib(e);
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
__global__ __launch_bounds__(TPB) void k_delta_tri(DeltaArgs D) {
  __shared__ int64_t item_s;
  __shared__ int32_t ns_s;
  const int64_t ne = min(ctr(D.dc, DC_EDGES), D.ce_cap);
  unsigned long long* mark = D.slot_mark + (int64_t)blockIdx.x * D.N;
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
      mark[w] = 0x100ull | fu | (fv << 4);
      S[atomicAdd(&ns_s, 1)] = w;
      // affected edges (u, w), (v, w)
      const unsigned long long q = atomicAdd(&D.dc[DC_AFF], 2ull);
      if ((int64_t)q + 1 < D.ae_cap) { D.ae[q] = pkey(u, w, D.bits); D.ae[q + 1] = pkey(v, w, D.bits); }
    }
    __syncthreads();
    const int32_t ns = ns_s;
    // 4-cliques: pairs w < x in S(e) with an edge (w, x)
    for (int32_t i = threadIdx.x >> 6; i < ns; i += blockDim.x >> 6) {
      const uint32_t w = S[i];
      const unsigned long long mw = mark[w];
      const uint32_t* wrow = D.P.col + D.P.off[w];
      const int32_t wl = D.P.len[w];
      const int32_t above = lower_bound_id(wrow, wl, w + 1);
      const int32_t nab = wl - above;
      int64_t acc = 0;
      auto clique = [&](uint32_t x, uint32_t fwx, unsigned long long mx) {
        const uint32_t fuw = (uint32_t)mw & 15u, fvw = (uint32_t)(mw >> 4) & 15u;
        const uint32_t fux = (uint32_t)mx & 15u, fvx = (uint32_t)(mx >> 4) & 15u;
        // counted from the changed edge of smallest key only
        if ((fuw && pkey(u, w, D.bits) < K) || (fvw && pkey(v, w, D.bits) < K) || (fux && pkey(u, x, D.bits) < K) ||
            (fvx && pkey(v, x, D.bits) < K) || (fwx && pkey(w, x, D.bits) < K))
          return;
        acc += delta_of(fe | fuw | fvw | fux | fvx | fwx);
      };
      if (nab <= ns) {
        for (int32_t k = above + lane_id(); k < wl; k += 64) {
          const uint32_t ex = wrow[k], x = ex & GC_ID;
          const unsigned long long mx = mark[x];
          if (mx) clique(x, nib(ex), mx);
        }
      } else {
        for (int32_t j = lane_id(); j < ns; j += 64) {
          const uint32_t x = S[j];
          if (x <= w) continue;
          const int32_t p = lower_bound_id(wrow, wl, x);
          if (p < wl && (wrow[p] & GC_ID) == x) clique(x, nib(wrow[p]), mark[x]);
        }
      }
      k4acc += acc;
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < ns; i += blockDim.x) mark[S[i]] = 0ull;
  }
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
  const int64_t w0 = gtid() >> 6, ws = gstride() >> 6;
  int64_t s3 = 0, s4 = 0, s5 = 0;
  int cur_g = -1;
  for (int64_t i = w0; i < na; i += ws) {
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
    const int32_t al = D.P.len[a];
    int32_t tb = 0, ta = 0;
    for (int32_t k = l; k < al; k += 64) {
      const uint32_t ea = arow[k], w = ea & GC_ID;
      if (w == b) continue;
      const int64_t p = find_in_row(D.P, b, w);
      if (p < 0) continue;
      const uint32_t f = nib(ea) | nib(D.P.col[p]);
      tb += (f & 1u) == 0;
      ta += (f & 2u) == 0;
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
// One workgroup per changed edge e = (s, o) at a time: the neighbours of o
// are marked (with the nibble of (o, b)) in the workgroup's dense slot; the
// wedges s - a - b with a != o, b != s closing on a marked b are the
// 4-cycles s - a - b - o through e.  s is the end whose neighbours have the
// smaller degree sum.  The rows of a in N(s) are walked by the waves 64
// entries of N(s) at a time, their rows concatenated over the lanes.
__global__ __launch_bounds__(TPB) void k_delta_c4(DeltaArgs D) {
  if (D.bstats[BS_RETRY]) return;
  constexpr int NW = TPB / 64;
  __shared__ int64_t item_s;
  __shared__ int64_t side_s[2];
  __shared__ int32_t pre_s[NW][65];
  __shared__ uint32_t aid_s[NW][64];
  const int64_t ne = min(ctr(D.dc, DC_EDGES), D.ce_cap);
  unsigned long long* mark = D.slot_mark + (int64_t)blockIdx.x * D.N;
  const unsigned long long idmask = (1ull << D.bits) - 1ull;
  const int wv = threadIdx.x >> 6, l = lane_id();
  int64_t acc = 0;
  int cur_g = -1;
  while (true) {
    __syncthreads();
    if (threadIdx.x == 0) { item_s = (int64_t)atomicAdd(&D.dc[DC_QC4], 1ull); side_s[0] = 0; side_s[1] = 0; }
    __syncthreads();
    const int64_t it = item_s;
    if (it >= ne) break;
    const unsigned long long ek = D.ce[it];
    const unsigned long long K = ek & DIR_KEY_MASK;
    const uint32_t fe = (uint32_t)(ek >> DIR_MASK_SHIFT) & 3u;
    const uint32_t u = (uint32_t)(K >> D.bits), v = (uint32_t)(K & idmask);
    const int g = D.gid[u];
    if (g != cur_g) {
      if (cur_g >= 0) add_sig(D, cur_g, SG_C4, acc);
      acc = 0;
      cur_g = g;
    }
    // wedge counts from each end
    for (int q = 0; q < 2; ++q) {
      const uint32_t r = q ? v : u;
      const uint32_t* row = D.P.col + D.P.off[r];
      const int32_t L = D.P.len[r];
      int64_t sum = 0;
      for (int32_t k = threadIdx.x; k < L; k += blockDim.x) sum += D.P.len[row[k] & GC_ID];
      sum = wave_sum64(sum);
      if (l == 0) atomicAdd((unsigned long long*)&side_s[q], (unsigned long long)sum);
    }
    __syncthreads();
    const uint32_t s = side_s[0] <= side_s[1] ? u : v, o = s == u ? v : u;
    const uint32_t* orow = D.P.col + D.P.off[o];
    const int32_t ol = D.P.len[o];
    for (int32_t k = threadIdx.x; k < ol; k += blockDim.x) {
      const uint32_t eb = orow[k];
      mark[eb & GC_ID] = 0x100ull | nib(eb);
    }
    __syncthreads();
    const uint32_t* srow = D.P.col + D.P.off[s];
    const int32_t sl = D.P.len[s];
    for (int32_t c0 = wv * 64; c0 < sl; c0 += NW * 64) {
      // 64 entries a of N(s) per wave, their rows dealt over the lanes
      const int32_t k = c0 + l;
      uint32_t ea = 0, a = 0;
      int32_t len = 0;
      if (k < sl) {
        ea = srow[k];
        a = ea & GC_ID;
        if (a != o) len = D.P.len[a];
      }
      int32_t incl = wave_incl_scan32(len);
      pre_s[wv][l + 1] = incl;
      if (l == 0) pre_s[wv][0] = 0;
      aid_s[wv][l] = ea;
      wave_sync();
      const int32_t total = __shfl(incl, 63);
      for (int32_t f0 = 0; f0 < total; f0 += 64) {
        const int32_t f = f0 + l;
        if (f < total) {
          // segment j with pre[j] <= f < pre[j + 1]
          int32_t lo = 0, hi = 64;
          while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (pre_s[wv][mid] <= f) lo = mid; else hi = mid;
          }
          const uint32_t eaj = aid_s[wv][lo], aj = eaj & GC_ID;
          const uint32_t eab = D.P.col[D.P.off[aj] + (f - pre_s[wv][lo])];
          const uint32_t b = eab & GC_ID;
          if (b != s) {
            const unsigned long long mb = mark[b];
            if (mb) {
              const uint32_t fsa = nib(eaj), fab = nib(eab), fob = (uint32_t)mb & 15u;
              const bool skip = (fsa && pkey(s, aj, D.bits) < K) || (fab && pkey(aj, b, D.bits) < K) ||
                                (fob && pkey(o, b, D.bits) < K);
              if (!skip) acc += delta_of(fe | fsa | fab | fob);
            }
          }
        }
      }
      wave_sync();
    }
    __syncthreads();
    for (int32_t k = threadIdx.x; k < ol; k += blockDim.x) mark[orow[k] & GC_ID] = 0ull;
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
  hipLaunchKernelGGL(k_delta_vertex, dim3(2048), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_s2, dim3(2048), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_tri, dim3(slots), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_aff_changed, dim3(1024), dim3(TPB), 0, s, D);
  unsigned long long* sorted =
      radix_sort_u64(D.ae, D.ae_alt, D.sort_tmp, D.ae_cap, D.dc + DC_AFF_TOTAL, 2 * D.bits, s);
  hipLaunchKernelGGL(k_delta_aff, dim3(4096), dim3(TPB), 0, s, D, (const unsigned long long*)sorted);
  hipLaunchKernelGGL(k_delta_vertex2, dim3(1024), dim3(TPB), 0, s, D);
  hipLaunchKernelGGL(k_delta_tv, dim3(1024), dim3(TPB), 0, s, D, (const unsigned long long*)sorted);
  hipLaunchKernelGGL(k_delta_c4, dim3(slots), dim3(TPB), 0, s, D);
}

void launch_tv_region(int nv, const RegionDev& R, const int32_t* rlist, const unsigned long long* c,
                      unsigned long long* dT, long long* Tv, unsigned long long* bstats, hipStream_t s) {
  if (nv == 2)
    hipLaunchKernelGGL(k_tv_entries<2>, dim3(4096), dim3(TPB), 0, s, R, c, dT, (const unsigned long long*)bstats);
  else
    hipLaunchKernelGGL(k_tv_entries<4>, dim3(4096), dim3(TPB), 0, s, R, c, dT, (const unsigned long long*)bstats);
  hipLaunchKernelGGL(k_tv_apply, dim3(2048), dim3(TPB), 0, s, rlist, c, dT, Tv, bstats);
}
