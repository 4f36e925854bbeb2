// Graph-side kernels: batch ingest, merge of a batch into the slack CSR
// (tombstone phase before counting, purge phase after), region-of-change
// marking, the region CSR and its per-vertex pass, and the initial build.
//
// Batch semantics (the stream model of Sec. 3 and the batch protocol of
// Sec. 6): pairs are unordered, self loops are not edges, repeats collapse,
// a pair both inserted and deleted by one batch is dropped, and only the
// effective part A' = A - E, D' = D & E changes the graph.  Several batches
// of one graph may share a pass: they act in order, each on the graph left by
// the previous one, and every version in between is kept (entry flags).
#include "gc_kernels.h"

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ int64_t gwave() { return gtid() >> 6; }
__device__ __forceinline__ int64_t gwaves() { return gstride() >> 6; }

__device__ __forceinline__ int64_t ctr(const unsigned long long* c, int k) { return (int64_t)c[k]; }

// Is (a, b) an edge of the pre-batch graph?  Binary search in the shorter row.
__device__ __forceinline__ bool edge_exists(const PoolDev& P, uint32_t a, uint32_t b) {
  if (P.len[b] < P.len[a]) { uint32_t t = a; a = b; b = t; }
  const uint32_t* row = P.col + P.off[a];
  int32_t n = P.len[a];
  int32_t p = lower_bound_id(row, n, b);
  return p < n && (row[p] & GC_ID) == b;
}

// ------------------------------------------------------------- ingest
__global__ void k_ingest_keys(PoolDev P, BatchIn B, int bits, unsigned long long* __restrict__ keys,
                              unsigned long long* __restrict__ cc, unsigned long long* __restrict__ bstats) {
  const int64_t n_ins = B.ins_seg[B.k], n_del = B.del_seg[B.k];
  const int64_t total = n_ins + n_del;
  if (gtid() == 0) cc[C_NKEYS] = (unsigned long long)total;
  const uint64_t idmask = (1ull << bits) - 1ull;
  for (int64_t i = gtid(); i < total; i += gstride()) {
    const bool del = i >= n_ins;
    const int64_t j = del ? i - n_ins : i;
    int32_t u = del ? B.du[j] : B.iu[j];
    int32_t v = del ? B.dv[j] : B.iv[j];
    // segment of this entry: a graph of the pool, or a batch of graph 0
    const int64_t* seg = del ? B.del_seg : B.ins_seg;
    int lo = 0, hi = B.k;
    while (hi - lo > 1) { int mid = (lo + hi) >> 1; if (seg[mid] <= j) lo = mid; else hi = mid; }
    const int g = B.seq ? 0 : lo, bj = B.seq ? lo : 0;
    const int64_t base = B.gbase[g], n = B.gn[g];
    if (u < 0 || v < 0 || u >= n || v >= n || (B.dead && (B.dead[base + u] | B.dead[base + v]))) {
      atomicAdd(&bstats[PB_IDX(bj, PB_ERR)], 1ull);
      keys[i] = ~0ull;
      continue;
    }
    if (u == v) {
      atomicAdd(&bstats[PB_IDX(bj, PB_LOOPS)], 1ull);
      keys[i] = ~0ull;
      continue;
    }
    uint64_t a = (uint64_t)(uint32_t)P.ext2int[base + u];
    uint64_t b = (uint64_t)(uint32_t)P.ext2int[base + v];
    uint64_t mn = a < b ? a : b, mx = a < b ? b : a;
    keys[i] = (((mn << bits) | (mx & idmask)) << 3) | ((uint64_t)bj << 1) | (del ? 1ull : 0ull);
  }
}

// After sorting: one decision per distinct pair, at its first key.  The
// batches of the pass act on the pair in order, each by the rules above on
// the graph the previous one left.  Bit x of the absence mask says that the
// pair is not an edge of version x (x = 0 before the pass, x = j + 1 after
// batch j; versions past the last batch repeat the last one).  Pairs whose
// mask is neither empty nor full change: existing edges go to dirD (flags),
// the others to dirA (new entries), and those absent from the last version
// also to dirR (removed by the purge).
__global__ void k_ingest_classify(PoolDev P, const unsigned long long* __restrict__ keys, int bits, int nb, int nv,
                                  unsigned long long* __restrict__ dirA, unsigned long long* __restrict__ dirD,
                                  unsigned long long* __restrict__ dirR, unsigned long long* __restrict__ c,
                                  unsigned long long* __restrict__ bstats) {
  const int64_t total = ctr(c, C_NKEYS);
  const uint64_t idmask = (1ull << bits) - 1ull;
  for (int64_t i = gtid(); i < total; i += gstride()) {
    const unsigned long long key = keys[i];
    if (key == ~0ull) continue;
    const unsigned long long pair = key >> 3;
    if (i > 0 && (keys[i - 1] >> 3) == pair) continue;
    uint32_t ins = 0, del = 0;  // bit j: batch j inserts / deletes the pair
    for (int64_t q = i; q < total && (keys[q] >> 3) == pair; ++q) {
      const int j = (int)((keys[q] >> 1) & 3ull);
      if (q > i && keys[q] == keys[q - 1]) { atomicAdd(&bstats[PB_IDX(j, PB_DUPS)], 1ull); continue; }
      if (keys[q] & 1ull) del |= 1u << j; else ins |= 1u << j;
    }
    const uint32_t a = (uint32_t)(pair >> bits), b = (uint32_t)(pair & idmask);
    const bool p0 = edge_exists(P, a, b);
    bool p = p0;
    uint32_t am = p ? 0u : 1u;
    for (int j = 0; j < nb; ++j) {
      const bool in = (ins >> j) & 1u, de = (del >> j) & 1u;
      if (in && de) {
        atomicAdd(&bstats[PB_IDX(j, PB_CANCEL)], 1ull);
      } else if (in) {
        if (p) atomicAdd(&bstats[PB_IDX(j, PB_INS_EXIST)], 1ull);
        else { p = true; atomicAdd(&bstats[PB_IDX(j, PB_EFF_INS)], 1ull); }
      } else if (de) {
        if (!p) atomicAdd(&bstats[PB_IDX(j, PB_DEL_MISS)], 1ull);
        else { p = false; atomicAdd(&bstats[PB_IDX(j, PB_EFF_DEL)], 1ull); }
      }
      if (!p) am |= 1u << (j + 1);
    }
    if (!p)
      for (int x = nb + 1; x < nv; ++x) am |= 1u << x;
    if (am == 0u || am == (1u << nv) - 1u) continue;
    const unsigned long long ab = ((unsigned long long)a << bits) | b, ba = ((unsigned long long)b << bits) | a;
    const unsigned long long mk = (unsigned long long)am << DIR_MASK_SHIFT;
    unsigned long long* out = p0 ? dirD : dirA;
    const unsigned long long q = atomicAdd(&c[p0 ? C_DIRD : C_DIRA], 2ull);
    out[q] = ab | mk;
    out[q + 1] = ba | mk;
    if (!p) {
      const unsigned long long r = atomicAdd(&c[C_DIRR], 2ull);
      dirR[r] = ab;
      dirR[r + 1] = ba;
    }
  }
}

// Row segments of a sorted directed list; touched-row list (each row once).
__global__ void k_mark_rows(const unsigned long long* __restrict__ dir, const unsigned long long* c, int which,
                            int bits, int32_t* __restrict__ beg, int32_t* __restrict__ cnt,
                            int32_t* __restrict__ mark, int32_t* __restrict__ touched,
                            int32_t* __restrict__ tix, unsigned long long* __restrict__ cc) {
  const int64_t n = ctr(c, which);
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const uint32_t row = (uint32_t)((dir[i] & DIR_KEY_MASK) >> bits);
    if (i > 0 && (uint32_t)((dir[i - 1] & DIR_KEY_MASK) >> bits) == row) continue;
    if (beg) {
      const unsigned long long nxt = (unsigned long long)(row + 1) << bits;
      int64_t lo = i + 1, hi = n;
      while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((dir[mid] & DIR_KEY_MASK) < nxt) lo = mid + 1; else hi = mid;
      }
      beg[row] = (int32_t)i;
      cnt[row] = (int32_t)(lo - i);
    }
    if (atomicOr(&mark[row], 1) == 0) {
      unsigned long long p = atomicAdd(&cc[C_TOUCH], 1ull);
      touched[p] = (int32_t)row;
      tix[row] = (int32_t)p;
    }
  }
}

// --------------------------------------------------- tombstone merge
// Plan: rows that receive insertions get a destination (in place when the
// slack suffices, else a fresh bump-allocated segment).
__global__ void k_plan_rows(PoolDev P, const int32_t* __restrict__ touched, const unsigned long long* c,
                            int64_t max_touched, const int32_t* __restrict__ na, float slack,
                            int64_t* __restrict__ dest, int32_t* __restrict__ newcap, int32_t* __restrict__ tlen,
                            unsigned long long* __restrict__ bstats) {
  const int64_t nt = ctr(c, C_TOUCH);
  for (int64_t i = gtid(); i < max_touched; i += gstride()) {
    if (i >= nt) { tlen[i] = 0; continue; }
    const int32_t r = touched[i];
    const int32_t add = na[r];
    const int32_t L = P.len[r];
    tlen[i] = L;  // copied to scratch for the merge and again for the purge
    if (add == 0) { dest[i] = P.off[r]; newcap[i] = P.cap[r]; continue; }
    const int32_t nl = L + add;
    if (nl <= P.cap[r]) { dest[i] = P.off[r]; newcap[i] = P.cap[r]; continue; }
    int64_t nc = (int64_t)nl + (int64_t)((float)nl * slack) + 4;
    unsigned long long pos = atomicAdd(P.arena_top, (unsigned long long)nc);
    if ((int64_t)pos + nc > P.arena_cap) {
      atomicAdd(&bstats[BS_ARENA_OVF], 1ull);
      dest[i] = -1;
      newcap[i] = P.cap[r];
      continue;
    }
    dest[i] = (int64_t)pos;
    newcap[i] = (int32_t)nc;
  }
}

// Flat copy of the touched rows into scratch (positions from tpre); skipped
// while *skip != 0 (skip may be null).
__global__ void k_copy_rows(PoolDev P, const int32_t* __restrict__ touched, const unsigned long long* c,
                            const int64_t* __restrict__ tpre, uint32_t* __restrict__ scratch,
                            const unsigned long long* skip) {
  if (skip && *skip) return;
  const int64_t nt = ctr(c, C_TOUCH);
  if (nt == 0) return;
  const int64_t total = tpre[nt];
  for (int64_t i = gtid(); i < total; i += gstride()) {
    const int64_t t = upper_bound_i64(tpre, nt, i);
    const int32_t r = touched[t];
    scratch[i] = P.col[P.off[r] + (i - tpre[t])];
  }
}

// Merge: old entries shift right by the insertions before them; insertions
// land after the old entries before them.  Inserted entries carry their
// absence mask (at least F_NEW: absent before the pass).
__global__ void k_merge_old(PoolDev P, const int32_t* __restrict__ touched, const unsigned long long* c,
                            const int64_t* __restrict__ tpre, const uint32_t* __restrict__ scratch,
                            const unsigned long long* __restrict__ dirA, int bits,
                            const int32_t* __restrict__ a_beg, const int32_t* __restrict__ na,
                            const int64_t* __restrict__ dest) {
  const int64_t nt = ctr(c, C_TOUCH);
  if (nt == 0) return;
  const int64_t total = tpre[nt];
  const uint64_t idmask = (1ull << bits) - 1ull;
  for (int64_t i = gtid(); i < total; i += gstride()) {
    const int64_t t = upper_bound_i64(tpre, nt, i);
    const int32_t r = touched[t];
    const int32_t cntA = na[r];
    if (cntA == 0 || dest[t] < 0) continue;
    const int64_t k = i - tpre[t];
    const uint32_t x = scratch[i];
    const uint32_t id = x & GC_ID;
    const unsigned long long* A = dirA + a_beg[r];
    int32_t lo = 0, hi = cntA;
    while (lo < hi) { int32_t mid = (lo + hi) >> 1; if ((uint32_t)(A[mid] & idmask) < id) lo = mid + 1; else hi = mid; }
    P.col[dest[t] + k + lo] = x;
  }
}

__global__ void k_merge_new(PoolDev P, const unsigned long long* c, const unsigned long long* __restrict__ dirA,
                            int bits, const int32_t* __restrict__ a_beg, const int32_t* __restrict__ tix,
                            const int64_t* __restrict__ tpre, const uint32_t* __restrict__ scratch,
                            const int64_t* __restrict__ dest) {
  const int64_t n = ctr(c, C_DIRA);
  const uint64_t idmask = (1ull << bits) - 1ull;
  for (int64_t j = gtid(); j < n; j += gstride()) {
    const uint32_t r = (uint32_t)((dirA[j] & DIR_KEY_MASK) >> bits);
    const uint32_t id = (uint32_t)(dirA[j] & idmask);
    const uint32_t fl = (uint32_t)(dirA[j] >> DIR_MASK_SHIFT) << GC_VSHIFT;
    const int32_t t = tix[r];
    if (dest[t] < 0) continue;
    const int32_t q = (int32_t)(j - a_beg[r]);
    const uint32_t* old = scratch + tpre[t];
    const int32_t L = (int32_t)(tpre[t + 1] - tpre[t]);
    int32_t p = lower_bound_id(old, L, id);
    P.col[dest[t] + q + p] = id | fl;
  }
}

__global__ void k_commit_rows(PoolDev P, const int32_t* __restrict__ touched, const unsigned long long* c,
                              const int32_t* __restrict__ na, const int64_t* __restrict__ dest,
                              const int32_t* __restrict__ newcap) {
  const int64_t nt = ctr(c, C_TOUCH);
  for (int64_t i = gtid(); i < nt; i += gstride()) {
    const int32_t r = touched[i];
    if (na[r] == 0 || dest[i] < 0) continue;
    P.off[r] = dest[i];
    P.cap[r] = newcap[i];
    P.len[r] += na[r];
  }
}

// existing edges that change: their entries take the absence mask
__global__ void k_flag_rows(PoolDev P, const unsigned long long* c, const unsigned long long* __restrict__ dirD,
                            int bits, unsigned long long* __restrict__ bstats) {
  const int64_t n = ctr(c, C_DIRD);
  const uint64_t idmask = (1ull << bits) - 1ull;
  for (int64_t j = gtid(); j < n; j += gstride()) {
    const uint32_t r = (uint32_t)((dirD[j] & DIR_KEY_MASK) >> bits);
    const uint32_t id = (uint32_t)(dirD[j] & idmask);
    const uint32_t fl = (uint32_t)(dirD[j] >> DIR_MASK_SHIFT) << GC_VSHIFT;
    uint32_t* row = P.col + P.off[r];
    int32_t p = lower_bound_id(row, P.len[r], id);
    if (p < P.len[r] && (row[p] & GC_ID) == id) row[p] |= fl;
    else atomicAdd(&bstats[BS_ERR], 1ull);
  }
}

// ------------------------------------------------------------- purge
// Remove the entries absent from the last version and clear every flag in
// the touched rows (from a scratch copy of the union rows); reset the per-row
// batch arrays.
__global__ void k_touched_len(PoolDev P, const int32_t* __restrict__ touched, const unsigned long long* c,
                              int64_t max_touched, int32_t* __restrict__ tlen, const unsigned long long* skip) {
  if (*skip) return;
  const int64_t nt = ctr(c, C_TOUCH);
  for (int64_t i = gtid(); i < max_touched; i += gstride()) tlen[i] = i < nt ? P.len[touched[i]] : 0;
}

__global__ void k_purge_rows(PoolDev P, const int32_t* __restrict__ touched, const unsigned long long* c,
                             const int64_t* __restrict__ tpre, const uint32_t* __restrict__ scratch,
                             const unsigned long long* __restrict__ dirR, int bits, uint32_t fin,
                             const int32_t* __restrict__ r_beg, const int32_t* __restrict__ nr,
                             const unsigned long long* skip) {
  if (*skip) return;
  const int64_t nt = ctr(c, C_TOUCH);
  if (nt == 0) return;
  const int64_t total = tpre[nt];
  const uint64_t idmask = (1ull << bits) - 1ull;
  for (int64_t i = gtid(); i < total; i += gstride()) {
    const int64_t t = upper_bound_i64(tpre, nt, i);
    const int32_t r = touched[t];
    const uint32_t x = scratch[i];
    if (x & fin) continue;
    const int64_t k = i - tpre[t];
    const int32_t cntD = nr[r];
    int32_t lo = 0;
    if (cntD) {
      const unsigned long long* D = dirR + r_beg[r];
      const uint32_t id = x & GC_ID;
      int32_t hi = cntD;
      while (lo < hi) { int32_t mid = (lo + hi) >> 1; if ((uint32_t)(D[mid] & idmask) < id) lo = mid + 1; else hi = mid; }
    }
    P.col[P.off[r] + k - lo] = x & GC_ID;
  }
}

// nrem: the per-row counts of the removal list k_purge_rows used (nr, or na
// when the pass is undone)
__global__ void k_purge_commit(PoolDev P, const int32_t* __restrict__ touched, const unsigned long long* c,
                               int32_t* a_beg, int32_t* na, int32_t* r_beg, int32_t* nr, int32_t* __restrict__ mark,
                               int32_t* __restrict__ tix, const int32_t* nrem, const unsigned long long* skip) {
  if (*skip) return;
  const int64_t nt = ctr(c, C_TOUCH);
  for (int64_t i = gtid(); i < nt; i += gstride()) {
    const int32_t r = touched[i];
    P.len[r] -= nrem[r];
    a_beg[r] = 0; na[r] = 0; r_beg[r] = 0; nr[r] = 0; mark[r] = 0; tix[r] = 0;
  }
}

// ------------------------------------------------------------ region
// Levels: 0 = endpoint of a changed pair, k = first reached after k hops,
// LV_OUT = outside.  The region is every vertex with level <= radius; the
// counting runs on the subgraph induced on it (an induced superset of the
// changed 4-sets, see region_mark in the host code for the radius).
constexpr int32_t LV_OUT = 0x7fffffff;

__global__ void k_level0(const int32_t* __restrict__ touched, const unsigned long long* c,
                         int32_t* __restrict__ level, int32_t* __restrict__ rlist, unsigned long long* __restrict__ cc) {
  const int64_t nt = ctr(c, C_TOUCH);
  for (int64_t i = gtid(); i < nt; i += gstride()) {
    const int32_t r = touched[i];
    level[r] = 0;
    rlist[i] = r;
  }
  if (gtid() == 0) { cc[C_RLIST] = (unsigned long long)nt; cc[C_LVL0 + 1] = (unsigned long long)nt; cc[C_LVL0] = 0; }
}

// Append the lanes with `take` to the region list (one atomic per wave).
__device__ __forceinline__ void wave_append(bool take, int32_t v, int32_t* __restrict__ rlist,
                                            unsigned long long* __restrict__ cc) {
  const uint64_t m = __ballot(take);
  if (!m) return;
  unsigned long long base = 0;
  if (lane_id() == 0) base = atomicAdd(&cc[C_RLIST], (unsigned long long)__popcll(m));
  base = (unsigned long long)__shfl((long long)base, 0);
  if (take) rlist[base + __popcll(m & lanemask_lt())] = v;
}

// Expand the vertices of list range [lvl_beg, lvl_end) by one hop.
__global__ void k_expand(PoolDev P, int lvl, int32_t* __restrict__ level, int32_t* __restrict__ rlist,
                         unsigned long long* __restrict__ cc) {
  const int64_t b = ctr(cc, C_LVL0 + lvl), e = ctr(cc, C_LVL0 + lvl + 1);
  for (int64_t i = b + gwave(); i < e; i += gwaves()) {
    const int32_t v = rlist[i];
    const uint32_t* row = P.col + P.off[v];
    const int32_t L = P.len[v];
    for (int32_t k0 = 0; k0 < L; k0 += 64) {
      const int32_t k = k0 + lane_id();
      uint32_t w = 0;
      bool take = false;
      if (k < L) {
        w = row[k] & GC_ID;
        take = level[w] == LV_OUT && atomicCAS(&level[w], LV_OUT, lvl + 1) == LV_OUT;
      }
      wave_append(take, (int32_t)w, rlist, cc);
    }
  }
}

__global__ void k_level_end(unsigned long long* cc, int lvl) {
  if (gtid() == 0) cc[C_LVL0 + lvl + 1] = cc[C_RLIST];
}

// Whole-graph region: every vertex with a non-empty row.
__global__ void k_all_rows(PoolDev P, int32_t* __restrict__ rlist, unsigned long long* __restrict__ cc) {
  const int64_t lim = (P.N + 63) / 64 * 64;  // whole waves take part in the appends
  for (int64_t v = gtid(); v < lim; v += gstride()) {
    const bool take = v < P.N && P.len[v] > 0;
    wave_append(take, (int32_t)v, rlist, cc);
  }
}

// Region row lengths (entries whose other end is in the region).
__global__ void k_region_len(PoolDev P, const int32_t* __restrict__ rlist, const unsigned long long* cc,
                             const int32_t* __restrict__ level, int32_t radius, int32_t* __restrict__ rlen) {
  const int64_t n = ctr(cc, C_RLIST);
  for (int64_t i = gwave(); i < n; i += gwaves()) {
    const int32_t v = rlist[i];
    const int32_t L = P.len[v];
    if (radius < 0 || level[v] < radius) { if (lane_id() == 0) rlen[v] = L; continue; }
    const uint32_t* row = P.col + P.off[v];
    int32_t cnt = 0;
    for (int32_t k = lane_id(); k < L; k += 64) cnt += level[row[k] & GC_ID] <= radius;
    cnt = wave_sum32(cnt);
    if (lane_id() == 0) rlen[v] = cnt;
  }
}

__global__ void k_region_fill(PoolDev P, RegionDev R, const int32_t* __restrict__ rlist, const unsigned long long* cc,
                              const int32_t* __restrict__ level, int32_t radius) {
  const int64_t n = ctr(cc, C_RLIST);
  for (int64_t i = gwave(); i < n; i += gwaves()) {
    const int32_t v = rlist[i];
    const int32_t L = P.len[v];
    const uint32_t* row = P.col + P.off[v];
    uint32_t* out = R.rcol + R.roff[v];
    int32_t* orow = R.rrow + R.roff[v];
    if (radius < 0 || level[v] < radius) {
      for (int32_t k = lane_id(); k < L; k += 64) { out[k] = row[k]; orow[k] = v; }
      continue;
    }
    int32_t base = 0;
    for (int32_t k0 = 0; k0 < L; k0 += 64) {
      const int32_t k = k0 + lane_id();
      uint32_t x = 0;
      bool keep = false;
      if (k < L) { x = row[k]; keep = level[x & GC_ID] <= radius; }
      const uint64_t m = __ballot(keep);
      if (keep) {
        const int32_t o = base + __popcll(m & lanemask_lt());
        out[o] = x;
        orow[o] = v;
      }
      base += __popcll(m);
    }
  }
}

// First index in sorted row[0..n) whose id is >= key, by an exponential
// search from the end: ids are a degree order, so for w < v the position of
// v in row w is usually among the last few entries.
__device__ __forceinline__ int32_t lower_bound_from_end(const uint32_t* row, int32_t n, uint32_t key) {
  int32_t hi = n, step = 1;  // row[hi..n) >= key
  while (hi > 0) {
    const int32_t p = hi - step > 0 ? hi - step : 0;
    if ((row[p] & GC_ID) < key) return p + 1 + lower_bound_id(row + p + 1, hi - p - 1, key);
    hi = p;
    step <<= 1;
  }
  return 0;
}

// Per-vertex pass over the region: degrees per version, N- split, the
// 3-star and wedge terms, and the work lists of the counting kernels.
template <int NV>
__device__ __forceinline__ void flush_vertex_terms(unsigned long long* sig, int g, int64_t (&s1)[NV],
                                                   int64_t (&w2)[NV], int64_t (&d1)[NV]) {
#pragma unroll
  for (int x = 0; x < NV; ++x) {
    if (s1[x]) atomicAdd(&sig[SIG_IDX(g, x, SG_S1)], (unsigned long long)s1[x]);
    if (w2[x]) atomicAdd(&sig[SIG_IDX(g, x, SG_W)], (unsigned long long)w2[x]);
    if (d1[x]) atomicAdd(&sig[SIG_IDX(g, x, SG_D1)], (unsigned long long)d1[x]);
    s1[x] = 0; w2[x] = 0; d1[x] = 0;
  }
}

// List appends of the per-vertex pass, batched per wave: lane k keeps the
// decisions of the wave's k-th vertex of the current group of 64, and one
// atomic per list reserves room for the whole group.
struct DegDecision {
  int32_t v = -1;
  int32_t tri = -1;  // L_TRI_S .. L_TRI_G or -1
  int32_t c4 = -1;   // L_C4_S / L_C4_M / L_C4_L or -1
  unsigned long long key = 0;  // sort key of the large 4-cycle tier
};

__device__ __forceinline__ void flush_decisions(DegDecision& d, unsigned long long* cc, int32_t* lists,
                                                int64_t list_stride, unsigned long long* c4_keys) {
  const int l = lane_id();
  for (int L = 0; L < L_NUM; ++L) {
    const bool mine = (L <= L_TRI_G ? d.tri : d.c4) == L && d.v >= 0;
    const uint64_t m = __ballot(mine);
    if (!m) continue;
    unsigned long long base = 0;
    if (l == 0) base = atomicAdd(&cc[C_LIST0 + L], (unsigned long long)__popcll(m));
    base = (unsigned long long)__shfl((long long)base, 0);
    if (mine) {
      const unsigned long long p = base + __popcll(m & lanemask_lt());
      lists[L * list_stride + p] = d.v;
      if (L == L_C4_L) c4_keys[p] = d.key;
    }
  }
  d = DegDecision();
}

// Segment of entry idx of a wave's concatenated lists: the last lane s whose
// exclusive prefix excl(s) is <= idx (excl nondecreasing over the lanes,
// excl(0) = 0, idx below the total).  All lanes must call it.
__device__ __forceinline__ int wave_segment(int32_t excl, int32_t idx) {
  int lo = 0, hi = 64;
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    const int mid = (lo + hi) >> 1;
    if (__shfl(excl, mid) <= idx) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int64_t wave_max64(int64_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t t = __shfl_xor(v, o);
    v = t > v ? t : v;
  }
  return v;
}

// a value equal in every lane, read from the first one (scalar registers)
__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A wave takes a group of 64 region vertices at a time, one per lane: the
// rows of the shorter ones are concatenated and dealt over the lanes (a
// segment search per step), so the lanes' searches for v in the rows of its
// lower neighbours overlap instead of one vertex's chain of loads at a time;
// the per-vertex sums meet in LDS, one slot per lane.  Rows of at least
// wave_row (<= 65536) entries are walked by the whole wave, one at a time.
template <int NV>
__global__ __launch_bounds__(TPB) void k_degrees(RegionDev R, const int32_t* __restrict__ gid, const int32_t* __restrict__ rlist,
                          unsigned long long* __restrict__ cc, unsigned long long* __restrict__ sig,
                          int32_t* __restrict__ lists, int64_t list_stride, int32_t tri_small, int32_t c4_small,
                          int32_t c4_mid, int32_t wave_row, unsigned long long* __restrict__ bstats,
                          unsigned long long* __restrict__ c4_keys) {
  __shared__ uint32_t sdv[TPB / 64][NV][64];          // degree per version
  __shared__ uint32_t slow[TPB / 64][64];             // lower entries
  __shared__ unsigned long long sws[TPB / 64][64];    // wedge bound
  const int l = lane_id(), wv = threadIdx.x >> 6;
#pragma unroll
  for (int x = 0; x < NV; ++x) sdv[wv][x][l] = 0u;
  slow[wv][l] = 0u;
  sws[wv][l] = 0ull;
  wave_sync();
  const int64_t n = ctr(cc, C_RLIST);
  int cur_g = -1;  // graph of the running sums s1, w2, d1 (lane 0)
  int64_t s1[NV], w2[NV], d1[NV];
#pragma unroll
  for (int x = 0; x < NV; ++x) { s1[x] = 0; w2[x] = 0; d1[x] = 0; }
  // per lane until the end
  int64_t wedges = 0, c4e[3] = {0, 0, 0};
  int32_t maxdp = 0, maxlow = 0;
  int64_t maxw = 0;
  DegDecision dec;
  // group c holds the region vertices c, c + C, c + 2C, ... (C groups): one
  // from each 64th of the list, so the high-degree vertices (ids follow the
  // degree order) are spread over the groups
  const int64_t C = (n + 63) / 64;
  for (int64_t c = gwave(); c < C; c += gwaves()) {
    const int64_t i = c + (int64_t)l * C;
    int32_t v = -1, L = 0;
    int64_t b = 0;
    if (i < n) {
      v = rlist[i];
      b = R.roff[v];
      L = (int32_t)(R.roff[v + 1] - b);
    }
    // entry at region position p of the row of lane s (vertex vs)
    auto entry = [&](int s, int32_t vs, int64_t p) {
      const uint32_t x = R.rcol[p];
      const uint32_t pm = vpresent<NV>(x);
#pragma unroll
      for (int q = 0; q < NV; ++q)
        if ((pm >> q) & 1u) atomicAdd(&sdv[wv][q][s], 1u);
      const uint32_t w = x & GC_ID;
      if (w < (uint32_t)vs) {
        // wedges (vs, w, .) below vs: entries of row w smaller than vs (kept
        // for the 4-cycle kernels as the starting cursor in row w)
        atomicAdd(&slow[wv][s], 1u);
        const int64_t wb = R.roff[w];
        const int32_t pos = lower_bound_from_end(R.rcol + wb, (int32_t)(R.roff[w + 1] - wb), (uint32_t)vs);
        R.vpos[p] = pos;
        if (pos) atomicAdd(&sws[wv][s], (unsigned long long)pos);
      }
    };
    {
      const int32_t ss = L < wave_row ? L : 0;  // total < 64 * 65536
      const int32_t incl = wave_incl_scan32(ss);
      const int32_t tot = __shfl(incl, 63);
      const int32_t excl = incl - ss;
      for (int32_t base = 0; base < tot; base += 64) {
        const int32_t idx = base + l;
        const int s = wave_segment(excl, idx);
        const int32_t vs = __shfl(v, s);
        const int64_t bs = __shfl(b, s);
        const int32_t es = __shfl(excl, s);
        if (idx < tot) entry(s, vs, bs + (idx - es));
      }
    }
    for (uint64_t lm = __ballot(L >= wave_row); lm; lm &= lm - 1) {
      const int s = __builtin_ctzll(lm);
      const int32_t vs = __shfl(v, s), Ls = __shfl(L, s);
      const int64_t bs = __shfl(b, s);
      for (int32_t k = l; k < Ls; k += 64) entry(s, vs, bs + k);
    }
    wave_sync();
    int32_t dv[NV];
#pragma unroll
    for (int x = 0; x < NV; ++x) {
      dv[x] = (int32_t)sdv[wv][x][l];
      sdv[wv][x][l] = 0u;
    }
    const int32_t low = (int32_t)slow[wv][l];
    const int64_t wsum = (int64_t)sws[wv][l];
    slow[wv][l] = 0u;
    sws[wv][l] = 0ull;
    wave_sync();
    const bool has = v >= 0;
    if (has) {
      if constexpr (NV == 2) {
        *(int2*)(R.d + (int64_t)v * 2) = make_int2(dv[0], dv[1]);
      } else {
        *(int4*)(R.d + (int64_t)v * 4) = make_int4(dv[0], dv[1], dv[2], dv[3]);
      }
      R.rlow[v] = low;
    }
    // the 3-star and wedge terms, summed over the lanes of each graph in the
    // group into running sums of one graph (the same in every lane), flushed
    // by lane 0 when the graph changes
    {
      const int g = has ? gid[v] : -1;
      for (uint64_t left = __ballot(has); left;) {
        const int gs = __builtin_amdgcn_readfirstlane(__shfl(g, __builtin_ctzll(left)));
        const bool in = has && g == gs;
        left &= ~__ballot(in);
        if (gs != cur_g) {
          if (cur_g >= 0 && l == 0) flush_vertex_terms<NV>(sig, cur_g, s1, w2, d1);
#pragma unroll
          for (int x = 0; x < NV; ++x) { s1[x] = 0; w2[x] = 0; d1[x] = 0; }
          cur_g = gs;
        }
#pragma unroll
        for (int x = 0; x < NV; ++x) {
          s1[x] += uniform64(wave_sum64(in ? c3(dv[x]) : 0));
          w2[x] += uniform64(wave_sum64(in ? c2(dv[x]) : 0));
          d1[x] += uniform64(wave_sum64(in ? (int64_t)dv[x] : 0));
        }
      }
    }
    const int32_t dplus = L - low;
    const bool tri = has && dplus >= 2, c4 = has && low >= 2 && wsum >= 2;
    dec.v = has ? v : -1;
    dec.tri = tri ? tri_list_of(dplus, tri_small) : -1;
    dec.c4 = c4 ? (wsum <= c4_small ? L_C4_S : (wsum <= c4_mid ? L_C4_M : L_C4_L)) : -1;
    if (dec.c4 == L_C4_L) {
      const uint64_t wk = wsum < 0xFFFFFFFFll ? (uint64_t)wsum : 0xFFFFFFFFull;
      dec.key = ((0xFFFFFFFFull - wk) << 32) | (uint32_t)v;
    }
    if (tri) maxdp = dplus > maxdp ? dplus : maxdp;
    if (c4) {
      const int which = wsum <= c4_small ? 0 : (wsum <= c4_mid ? 1 : 2);
      maxw = wsum > maxw ? wsum : maxw;
      wedges += wsum;
      c4e[which] += wsum + low;
      if (which == 2) maxlow = low > maxlow ? low : maxlow;
    }
    flush_decisions(dec, cc, lists, list_stride, c4_keys);
  }
  maxdp = wave_max32(maxdp);
  maxlow = wave_max32(maxlow);
  maxw = wave_max64(maxw);
  wedges = wave_sum64(wedges);
#pragma unroll
  for (int q = 0; q < 3; ++q) c4e[q] = wave_sum64(c4e[q]);
  // The waves' totals (held by lane 0) meet in LDS: one set of atomics per
  // workgroup instead of per wave (the few words of one graph's sums and the
  // shared maxima would otherwise queue at one L2 channel).
  constexpr int NW = TPB / 64, NR = 3 * NV + 7;
  __shared__ int64_t red[NW][NR];
  __shared__ int wg[NW];
  if (lane_id() == 0) {
    wg[wv] = cur_g;
#pragma unroll
    for (int x = 0; x < NV; ++x) { red[wv][x] = s1[x]; red[wv][NV + x] = w2[x]; red[wv][2 * NV + x] = d1[x]; }
    red[wv][3 * NV] = maxdp;
    red[wv][3 * NV + 1] = maxw;
    red[wv][3 * NV + 2] = maxlow;
    red[wv][3 * NV + 3] = wedges;
    for (int q = 0; q < 3; ++q) red[wv][3 * NV + 4 + q] = c4e[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int gb = -1;
    bool same = true;
    for (int w = 0; w < NW; ++w) {
      if (wg[w] < 0) continue;
      if (gb < 0) gb = wg[w];
      else if (wg[w] != gb) same = false;
    }
    int64_t t1[NV], t2[NV], t3[NV];
    if (same) {  // one graph (or none): sum the waves, one flush
#pragma unroll
      for (int x = 0; x < NV; ++x) { t1[x] = 0; t2[x] = 0; t3[x] = 0; }
      for (int w = 0; w < NW; ++w) {
        if (wg[w] < 0) continue;
#pragma unroll
        for (int x = 0; x < NV; ++x) { t1[x] += red[w][x]; t2[x] += red[w][NV + x]; t3[x] += red[w][2 * NV + x]; }
      }
      if (gb >= 0) flush_vertex_terms<NV>(sig, gb, t1, t2, t3);
    } else {  // waves of different graphs of a pool: one flush each
      for (int w = 0; w < NW; ++w) {
        if (wg[w] < 0) continue;
#pragma unroll
        for (int x = 0; x < NV; ++x) { t1[x] = red[w][x]; t2[x] = red[w][NV + x]; t3[x] = red[w][2 * NV + x]; }
        flush_vertex_terms<NV>(sig, wg[w], t1, t2, t3);
      }
    }
    int64_t mdp = 0, mw = 0, ml = 0, wd = 0, ce[3] = {0, 0, 0};
    for (int w = 0; w < NW; ++w) {
      mdp = max(mdp, red[w][3 * NV]);
      mw = max(mw, red[w][3 * NV + 1]);
      ml = max(ml, red[w][3 * NV + 2]);
      wd += red[w][3 * NV + 3];
      for (int q = 0; q < 3; ++q) ce[q] += red[w][3 * NV + 4 + q];
    }
    if (mdp) atomicMax(&cc[C_MAXDP], (unsigned long long)mdp);
    if (mw) atomicMax(&cc[C_MAXW], (unsigned long long)mw);
    if (ml) atomicMax(&cc[C_MAXLOW], (unsigned long long)ml);
    if (wd) atomicAdd(&bstats[BS_WEDGES], (unsigned long long)wd);
    for (int q = 0; q < 3; ++q)
      if (ce[q]) atomicAdd(&bstats[BS_C4_S + q], (unsigned long long)ce[q]);
  }
}

__global__ void k_region_total(const int64_t* roff, int64_t N, unsigned long long* cc) {
  if (gtid() == 0) cc[C_ER] = (unsigned long long)roff[N];
}

// ------------------------------------------------------------ init build
__global__ void k_init_keys(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, int64_t m,
                            const int64_t* __restrict__ seg, const int64_t* __restrict__ gbase, int32_t k,
                            int bits, unsigned long long* __restrict__ keys) {
  const uint64_t idmask = (1ull << bits) - 1ull;
  for (int64_t i = gtid(); i < m; i += gstride()) {
    int lo = 0, hi = k;
    while (hi - lo > 1) { int mid = (lo + hi) >> 1; if (seg[mid] <= i) lo = mid; else hi = mid; }
    const uint64_t u = (uint64_t)(gbase[lo] + src[i]), v = (uint64_t)(gbase[lo] + dst[i]);
    if (u == v) { keys[i] = ~0ull; continue; }
    const uint64_t a = u < v ? u : v, b = u < v ? v : u;
    keys[i] = (a << bits) | (b & idmask);
  }
}

// unique edges -> degree count (external ids)
__global__ void k_init_unique(const unsigned long long* __restrict__ keys, int64_t m, int bits,
                              unsigned long long* __restrict__ uniq, unsigned long long* __restrict__ cc,
                              int32_t* __restrict__ deg) {
  const uint64_t idmask = (1ull << bits) - 1ull;
  for (int64_t i = gtid(); i < m; i += gstride()) {
    const unsigned long long k = keys[i];
    if (k == ~0ull || (i > 0 && keys[i - 1] == k)) continue;
    unsigned long long p = atomicAdd(&cc[C_DIRA], 1ull);
    uniq[p] = k;
    atomicAdd(&deg[k >> bits], 1);
    atomicAdd(&deg[k & idmask], 1);
  }
}

// rank keys: (graph, degree, local id)
__global__ void k_rank_keys(const int32_t* __restrict__ deg, const int32_t* __restrict__ gid,
                            const int64_t* __restrict__ gbase, int64_t N, int lbits,
                            unsigned long long* __restrict__ keys) {
  for (int64_t v = gtid(); v < N; v += gstride()) {
    const int g = gid[v];
    const uint64_t local = (uint64_t)(v - gbase[g]);
    keys[v] = ((uint64_t)g << (2 * lbits)) | ((uint64_t)deg[v] << lbits) | local;
  }
}

__global__ void k_rank_assign(const unsigned long long* __restrict__ sorted, const int64_t* __restrict__ gbase,
                              int64_t N, int lbits, int32_t* __restrict__ ext2int) {
  const uint64_t lmask = (1ull << lbits) - 1ull;
  for (int64_t p = gtid(); p < N; p += gstride()) {
    const unsigned long long k = sorted[p];
    const int g = (int)(k >> (2 * lbits));
    const int64_t ext = gbase[g] + (int64_t)(k & lmask);
    ext2int[ext] = (int32_t)p;
  }
}

__global__ void k_init_dir(const unsigned long long* __restrict__ uniq, const unsigned long long* cc, int bits,
                           const int32_t* __restrict__ ext2int, unsigned long long* __restrict__ dir,
                           int32_t* __restrict__ len) {
  const int64_t m = ctr(cc, C_DIRA);
  const uint64_t idmask = (1ull << bits) - 1ull;
  for (int64_t i = gtid(); i < m; i += gstride()) {
    const uint64_t a = (uint64_t)(uint32_t)ext2int[uniq[i] >> bits];
    const uint64_t b = (uint64_t)(uint32_t)ext2int[uniq[i] & idmask];
    dir[2 * i] = (a << bits) | b;
    dir[2 * i + 1] = (b << bits) | a;
    atomicAdd(&len[a], 1);
    atomicAdd(&len[b], 1);
  }
}

__global__ void k_init_caps(PoolDev P, float slack) {
  for (int64_t v = gtid(); v < P.N; v += gstride()) {
    const int32_t L = P.len[v];
    P.cap[v] = L + (int32_t)((float)L * slack) + (L > 0 ? 2 : 0);
  }
}

// entries carry F_NEW: at build time the graph before is empty
__global__ void k_init_fill(PoolDev P, const unsigned long long* __restrict__ dir, const unsigned long long* cc,
                            int bits, const int64_t* __restrict__ rstart, uint32_t flag) {
  const int64_t n = 2 * ctr(cc, C_DIRA);
  const uint64_t idmask = (1ull << bits) - 1ull;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const uint32_t r = (uint32_t)(dir[i] >> bits);
    P.col[P.off[r] + (i - rstart[r])] = (uint32_t)(dir[i] & idmask) | flag;
  }
}

__global__ void k_set_top(PoolDev P, const int64_t* off_end) {
  if (gtid() == 0) *P.arena_top = (unsigned long long)*off_end;
}

// set or clear flag bits on every entry of every row
__global__ void k_all_flags(PoolDev P, uint32_t set, uint32_t keep) {
  for (int64_t v = gwave(); v < P.N; v += gwaves()) {
    uint32_t* row = P.col + P.off[v];
    const int32_t L = P.len[v];
    for (int32_t k = lane_id(); k < L; k += 64) row[k] = (row[k] & keep) | set;
  }
}

// compaction: copy rows into a fresh arena with new offsets
__global__ void k_compact_copy(PoolDev P, const int64_t* __restrict__ noff, uint32_t* __restrict__ ncol) {
  for (int64_t v = gwave(); v < P.N; v += gwaves()) {
    const uint32_t* row = P.col + P.off[v];
    uint32_t* out = ncol + noff[v];
    const int32_t L = P.len[v];
    for (int32_t k = lane_id(); k < L; k += 64) out[k] = row[k];
  }
}

// edge list export (internal -> external ids, each edge once)
__global__ void k_export_edges(PoolDev P, const int32_t* __restrict__ int2ext, const int64_t* __restrict__ gbase,
                               const int64_t* __restrict__ pre, int32_t* __restrict__ src, int32_t* __restrict__ dst) {
  for (int64_t v = gwave(); v < P.N; v += gwaves()) {
    const uint32_t* row = P.col + P.off[v];
    const int32_t L = P.len[v];
    const int g = P.gid[v];
    int64_t base = pre[v];
    for (int32_t k0 = 0; k0 < L; k0 += 64) {
      const int32_t k = k0 + lane_id();
      bool up = false;
      uint32_t w = 0;
      if (k < L) { w = row[k] & GC_ID; up = w > (uint32_t)v; }
      const uint64_t m = __ballot(up);
      if (up) {
        const int64_t p = base + __popcll(m & lanemask_lt());
        src[p] = (int32_t)(int2ext[v] - gbase[g]);
        dst[p] = (int32_t)(int2ext[w] - gbase[g]);
      }
      base += __popcll(m);
    }
  }
}

// rows of given vertices of a single graph (external ids): their lengths,
// then their edges (x, neighbour) in external ids, x's at pre[i]
__global__ void k_row_len(PoolDev P, const int32_t* __restrict__ ids, int64_t k, int32_t* __restrict__ out) {
  for (int64_t i = gtid(); i < k; i += gstride()) out[i] = P.len[P.ext2int[ids[i]]];
}

__global__ void k_row_gather(PoolDev P, const int32_t* __restrict__ int2ext, const int32_t* __restrict__ ids,
                             int64_t k, const int64_t* __restrict__ pre, int32_t* __restrict__ u,
                             int32_t* __restrict__ v) {
  for (int64_t i = gwave(); i < k; i += gwaves()) {
    const int32_t x = ids[i], r = P.ext2int[x];
    const uint32_t* row = P.col + P.off[r];
    const int32_t L = P.len[r];
    const int64_t b = pre[i];
    for (int32_t j = lane_id(); j < L; j += 64) {
      u[b + j] = x;
      v[b + j] = int2ext[row[j] & GC_ID];
    }
  }
}

__global__ void k_set_bytes(uint8_t* __restrict__ a, const int32_t* __restrict__ ids, int64_t k, uint8_t val) {
  for (int64_t i = gtid(); i < k; i += gstride()) a[ids[i]] = val;
}

__global__ void k_upper_count(PoolDev P, int32_t* __restrict__ cnt) {
  for (int64_t v = gwave(); v < P.N; v += gwaves()) {
    const uint32_t* row = P.col + P.off[v];
    const int32_t L = P.len[v];
    int32_t c = 0;
    for (int32_t k = lane_id(); k < L; k += 64) c += (row[k] & GC_ID) > (uint32_t)v;
    c = wave_sum32(c);
    if (lane_id() == 0) cnt[v] = c;
  }
}

__global__ void k_invert_perm(const int32_t* __restrict__ ext2int, int64_t N, int32_t* __restrict__ int2ext) {
  for (int64_t e = gtid(); e < N; e += gstride()) int2ext[ext2int[e]] = (int32_t)e;
}

inline unsigned grid_for(int64_t n, int per = TPB, unsigned cap = 65535u * 4) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

// ================================================================ launchers
void launch_ingest_keys(const PoolDev& P, const BatchIn& B, int bits, unsigned long long* keys, unsigned long long* c,
                        unsigned long long* bstats, int64_t cap_total, hipStream_t s) {
  hipLaunchKernelGGL(k_ingest_keys, dim3(grid_for(cap_total)), dim3(TPB), 0, s, P, B, bits, keys, c, bstats);
}

void launch_ingest_classify(const PoolDev& P, const unsigned long long* keys, int64_t cap_total, int bits, int nb,
                            int nv, unsigned long long* dirA, unsigned long long* dirD, unsigned long long* dirR,
                            unsigned long long* c, unsigned long long* bstats, hipStream_t s) {
  if (cap_total == 0) return;
  hipLaunchKernelGGL(k_ingest_classify, dim3(grid_for(cap_total)), dim3(TPB), 0, s, P, keys, bits, nb, nv, dirA,
                     dirD, dirR, c, bstats);
}

void launch_mark_rows(const unsigned long long* dir, int64_t max_n, unsigned long long* c, int which, int bits,
                      int32_t* beg, int32_t* cnt, int32_t* mark, int32_t* touched, int32_t* tix, hipStream_t s) {
  if (max_n == 0) return;
  hipLaunchKernelGGL(k_mark_rows, dim3(grid_for(max_n)), dim3(TPB), 0, s, dir, c, which, bits, beg, cnt, mark,
                     touched, tix, c);
}

void launch_merge(const PoolDev& P, const BatchWork& W, int64_t max_touched, int64_t max_dirA, int bits, float slack,
                  unsigned long long* bstats, void* scan_tmp, hipStream_t s) {
  if (max_touched == 0) return;
  hipLaunchKernelGGL(k_plan_rows, dim3(grid_for(max_touched)), dim3(TPB), 0, s, P, W.touched, W.c, max_touched,
                     W.na, slack, W.dest, W.newcap, W.tlen, bstats);
  exclusive_scan_i32_to_i64(W.tlen, W.tpre, max_touched, scan_tmp, s);
  const unsigned g = 4096;
  hipLaunchKernelGGL(k_copy_rows, dim3(g), dim3(TPB), 0, s, P, W.touched, W.c, W.tpre, W.scratch,
                     (const unsigned long long*)nullptr);
  hipLaunchKernelGGL(k_merge_old, dim3(g), dim3(TPB), 0, s, P, W.touched, W.c, W.tpre, W.scratch, W.dirA, bits,
                     W.a_beg, W.na, W.dest);
  if (max_dirA)
    hipLaunchKernelGGL(k_merge_new, dim3(grid_for(max_dirA)), dim3(TPB), 0, s, P, W.c, W.dirA, bits, W.a_beg, W.tix,
                       W.tpre, W.scratch, W.dest);
  hipLaunchKernelGGL(k_commit_rows, dim3(grid_for(max_touched)), dim3(TPB), 0, s, P, W.touched, W.c, W.na, W.dest,
                     W.newcap);
}

void launch_flag_rows(const PoolDev& P, const BatchWork& W, int64_t max_dirD, int bits, unsigned long long* bstats,
                      hipStream_t s) {
  if (max_dirD == 0) return;
  hipLaunchKernelGGL(k_flag_rows, dim3(grid_for(max_dirD)), dim3(TPB), 0, s, P, W.c, W.dirD, bits, bstats);
}

void launch_purge(const PoolDev& P, const BatchWork& W, int64_t max_touched, int bits, uint32_t fin,
                  const unsigned long long* skip, void* scan_tmp, hipStream_t s, bool undo) {
  if (max_touched == 0) return;
  // undo: keep version 0 instead of the last version (remove the new
  // entries, listed in dirA, and clear the flags of the others)
  const unsigned long long* rm = undo ? W.dirA : W.dirR;
  const int32_t* rm_beg = undo ? W.a_beg : W.r_beg;
  const int32_t* rm_n = undo ? W.na : W.nr;
  if (undo) fin = GC_F_NEW;
  // lengths of the union rows, then a copy, then the compaction (the scan of
  // stale lengths under skip is harmless: nothing reads it)
  hipLaunchKernelGGL(k_touched_len, dim3(grid_for(max_touched)), dim3(TPB), 0, s, P, W.touched, W.c, max_touched,
                     W.tlen, skip);
  exclusive_scan_i32_to_i64(W.tlen, W.tpre, max_touched, scan_tmp, s);
  hipLaunchKernelGGL(k_copy_rows, dim3(4096), dim3(TPB), 0, s, P, W.touched, W.c, W.tpre, W.scratch, skip);
  hipLaunchKernelGGL(k_purge_rows, dim3(4096), dim3(TPB), 0, s, P, W.touched, W.c, W.tpre, W.scratch, rm, bits,
                     fin, rm_beg, rm_n, skip);
  hipLaunchKernelGGL(k_purge_commit, dim3(grid_for(max_touched)), dim3(TPB), 0, s, P, W.touched, W.c, W.a_beg, W.na,
                     W.r_beg, W.nr, W.mark, W.tix, rm_n, skip);
}

// Purge of a pass without deletions (Alg. 1's insert-only batches): nothing
// leaves the rows, so the new entries (listed in dirA) only lose their flags
// in place; no row is copied or compacted.
__global__ void k_clear_new(PoolDev P, const unsigned long long* __restrict__ dirA, const unsigned long long* c,
                            int bits, const unsigned long long* skip) {
  if (*skip) return;
  const int64_t n = ctr(c, C_DIRA);
  const uint64_t idmask = (1ull << bits) - 1ull;
  for (int64_t i = gtid(); i < n; i += gstride()) {
    const unsigned long long key = dirA[i] & DIR_KEY_MASK;
    const uint32_t r = (uint32_t)(key >> bits), id = (uint32_t)(key & idmask);
    uint32_t* row = P.col + P.off[r];
    const int32_t p = lower_bound_id(row, P.len[r], id);
    if (p < P.len[r] && (row[p] & GC_ID) == id) row[p] = id;
  }
}

void launch_purge_insert_only(const PoolDev& P, const BatchWork& W, int64_t max_touched, int64_t max_dirA, int bits,
                              const unsigned long long* skip, hipStream_t s) {
  if (max_touched == 0) return;
  if (max_dirA > 0)
    hipLaunchKernelGGL(k_clear_new, dim3(grid_for(max_dirA)), dim3(TPB), 0, s, P, W.dirA, W.c, bits, skip);
  hipLaunchKernelGGL(k_purge_commit, dim3(grid_for(max_touched)), dim3(TPB), 0, s, P, W.touched, W.c, W.a_beg, W.na,
                     W.r_beg, W.nr, W.mark, W.tix, (const int32_t*)W.nr, skip);
}

void launch_region(const PoolDev& P, const BatchWork& W, int radius, int32_t* level, int32_t* rlist, int32_t* rlen,
                   hipStream_t s) {
  const int64_t N = P.N;
  fill_u32((uint32_t*)rlen, 0u, N, s);
  if (radius < 0) {
    hipLaunchKernelGGL(k_all_rows, dim3(grid_for(N)), dim3(TPB), 0, s, P, rlist, W.c);
    hipLaunchKernelGGL(k_region_len, dim3(4096), dim3(TPB), 0, s, P, rlist, W.c, level, -1, rlen);
    return;
  }
  fill_u32((uint32_t*)level, (uint32_t)LV_OUT, N, s);
  hipLaunchKernelGGL(k_level0, dim3(grid_for(N)), dim3(TPB), 0, s, W.touched, W.c, level, rlist, W.c);
  for (int l = 0; l < radius; ++l) {
    hipLaunchKernelGGL(k_expand, dim3(4096), dim3(TPB), 0, s, P, l, level, rlist, W.c);
    hipLaunchKernelGGL(k_level_end, dim3(1), dim3(64), 0, s, W.c, l + 1);
  }
  hipLaunchKernelGGL(k_region_len, dim3(4096), dim3(TPB), 0, s, P, rlist, W.c, level, radius, rlen);
}

void launch_region_fill(const PoolDev& P, const RegionDev& R, const BatchWork& W, int radius, const int32_t* level,
                        const int32_t* rlist, const int32_t* rlen, void* scan_tmp, hipStream_t s) {
  exclusive_scan_i32_to_i64(rlen, R.roff, P.N, scan_tmp, s);
  hipLaunchKernelGGL(k_region_total, dim3(1), dim3(64), 0, s, R.roff, P.N, W.c);
  hipLaunchKernelGGL(k_region_fill, dim3(4096), dim3(TPB), 0, s, P, R, rlist, W.c, level, radius);
}

void launch_degrees(int nv, const RegionDev& R, const int32_t* gid, const int32_t* rlist, unsigned long long* c,
                    unsigned long long* sig, int32_t* lists, int64_t list_stride, int32_t tri_small, int32_t c4_small,
                    int32_t c4_mid, int32_t wave_row, unsigned long long* bstats, unsigned long long* c4_keys,
                    hipStream_t s) {
  // at least 1024 vertices (list_stride = N bounds the region) per workgroup
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (list_stride + 1023) / 1024));
  if (nv == 2)
    hipLaunchKernelGGL(k_degrees<2>, dim3(grid), dim3(TPB), 0, s, R, gid, rlist, c, sig, lists, list_stride,
                       tri_small, c4_small, c4_mid, wave_row, bstats, c4_keys);
  else
    hipLaunchKernelGGL(k_degrees<4>, dim3(grid), dim3(TPB), 0, s, R, gid, rlist, c, sig, lists, list_stride,
                       tri_small, c4_small, c4_mid, wave_row, bstats, c4_keys);
}

// ---------------------------------------------------------------- build
void launch_init_keys(const int32_t* src, const int32_t* dst, int64_t m, const int64_t* seg, const int64_t* gbase,
                      int32_t k, int bits, unsigned long long* keys, hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_init_keys, dim3(grid_for(m)), dim3(TPB), 0, s, src, dst, m, seg, gbase, k, bits, keys);
}
void launch_init_unique(const unsigned long long* keys, int64_t m, int bits, unsigned long long* uniq,
                        unsigned long long* c, int32_t* deg, hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_init_unique, dim3(grid_for(m)), dim3(TPB), 0, s, keys, m, bits, uniq, c, deg);
}
void launch_rank(const int32_t* deg, const int32_t* gid, const int64_t* gbase, int64_t N, int lbits, int total_bits,
                 unsigned long long* keys, unsigned long long* alt, void* sort_tmp, int32_t* ext2int, int32_t* int2ext,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_rank_keys, dim3(grid_for(N)), dim3(TPB), 0, s, deg, gid, gbase, N, lbits, keys);
  unsigned long long* sorted = radix_sort_u64(keys, alt, sort_tmp, N, nullptr, total_bits, s);
  hipLaunchKernelGGL(k_rank_assign, dim3(grid_for(N)), dim3(TPB), 0, s, sorted, gbase, N, lbits, ext2int);
  hipLaunchKernelGGL(k_invert_perm, dim3(grid_for(N)), dim3(TPB), 0, s, ext2int, N, int2ext);
}
void launch_init_dir(const unsigned long long* uniq, int64_t max_m, unsigned long long* c, int bits,
                     const int32_t* ext2int, unsigned long long* dir, int32_t* len, hipStream_t s) {
  if (max_m == 0) return;
  hipLaunchKernelGGL(k_init_dir, dim3(grid_for(max_m)), dim3(TPB), 0, s, uniq, c, bits, ext2int, dir, len);
}
void launch_init_csr(const PoolDev& P, const unsigned long long* dir, int64_t max_dir, unsigned long long* c, int bits,
                     int64_t* rstart, float slack, void* scan_tmp, uint32_t flag, hipStream_t s) {
  hipLaunchKernelGGL(k_init_caps, dim3(grid_for(P.N)), dim3(TPB), 0, s, P, slack);
  exclusive_scan_i32_to_i64(P.len, rstart, P.N, scan_tmp, s);
  exclusive_scan_i32_to_i64(P.cap, P.off, P.N, scan_tmp, s);
  hipLaunchKernelGGL(k_set_top, dim3(1), dim3(64), 0, s, P, P.off + P.N);
  if (max_dir)
    hipLaunchKernelGGL(k_init_fill, dim3(grid_for(max_dir)), dim3(TPB), 0, s, P, dir, c, bits, rstart, flag);
}
void launch_caps(const PoolDev& P, float slack, hipStream_t s) {
  hipLaunchKernelGGL(k_init_caps, dim3(grid_for(P.N)), dim3(TPB), 0, s, P, slack);
}
void launch_all_flags(const PoolDev& P, uint32_t set, uint32_t keep, hipStream_t s) {
  hipLaunchKernelGGL(k_all_flags, dim3(4096), dim3(TPB), 0, s, P, set, keep);
}
void launch_compact(const PoolDev& P, int64_t* noff, uint32_t* ncol, hipStream_t s) {
  hipLaunchKernelGGL(k_compact_copy, dim3(4096), dim3(TPB), 0, s, P, noff, ncol);
}
void launch_upper_count(const PoolDev& P, int32_t* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_upper_count, dim3(4096), dim3(TPB), 0, s, P, cnt);
}
void launch_row_len(const PoolDev& P, const int32_t* ids, int64_t k, int32_t* out, hipStream_t s) {
  if (k > 0) hipLaunchKernelGGL(k_row_len, dim3(grid_for(k)), dim3(TPB), 0, s, P, ids, k, out);
}
void launch_row_gather(const PoolDev& P, const int32_t* int2ext, const int32_t* ids, int64_t k, const int64_t* pre,
                       int32_t* u, int32_t* v, hipStream_t s) {
  if (k > 0)
    hipLaunchKernelGGL(k_row_gather, dim3((unsigned)std::min<int64_t>(4096, (k + 3) / 4)), dim3(TPB), 0, s, P,
                       int2ext, ids, k, pre, u, v);
}
void launch_set_bytes(uint8_t* a, const int32_t* ids, int64_t k, uint8_t val, hipStream_t s) {
  if (k > 0) hipLaunchKernelGGL(k_set_bytes, dim3(grid_for(k)), dim3(TPB), 0, s, a, ids, k, val);
}
void launch_export(const PoolDev& P, const int32_t* int2ext, const int64_t* gbase, const int64_t* pre, int32_t* src,
                   int32_t* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_export_edges, dim3(4096), dim3(TPB), 0, s, P, int2ext, gbase, pre, src, dst);
}
