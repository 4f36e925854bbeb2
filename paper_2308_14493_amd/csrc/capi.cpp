// C ABI of the graphlet-4 library: handle management, the per-batch
// pipeline (ingest -> merge -> region -> count -> combine -> purge) on one
// HIP stream, and the exact 128-bit finalisation of the eleven counts.
#include "../../include/graphlet4.h"
#include "gc_kernels.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

// Batch staging of gc_apply_batch_dev_noalloc: one fixed array per device
// that the library runs on, held until the process ends.  Host code reaches
// it only through the address hipGetSymbolAddress returns for the current
// device (noalloc_scratch_ptr); the array's name itself is not a device
// address on the host.
static constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

thread_local std::string g_err;

struct GcError {
  int code;
};

[[noreturn]] void raise(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  throw GcError{code};
}

#define HIPCHK(x)                                                                           \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess) raise(GC_EDEVICE, "%s failed: %s", #x, hipGetErrorString(e_));     \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  // grow-only; contents are not preserved
  void ensure(size_t bytes) {
    bytes = std::max<size_t>(bytes, 16);  // as the no-allocation checks assume
    if (bytes <= cap) return;
    release();
    size_t nb = std::max(bytes, cap + cap / 2);
    hipError_t e = hipMalloc(&p, nb);
    if (e != hipSuccess) {
      p = nullptr;
      raise(GC_ENOMEM, "hipMalloc(%zu bytes) failed: %s", nb, hipGetErrorString(e));
    }
    cap = nb;
  }
  template <class T> T* as() const { return (T*)p; }
  void swap(DevBuf& o) { std::swap(p, o.p); std::swap(cap, o.cap); }
};

int bits_for(int64_t x) {  // smallest b >= 1 with x <= 2^b
  int b = 1;
  while (b < 62 && (1ll << b) < x) ++b;
  return b;
}

typedef __int128 i128;

i128 c2w(i128 x) { return x * (x - 1) / 2; }
i128 c4w(i128 x) { return x * (x - 1) * (x - 2) * (x - 3) / 24; }

// The five disconnected classes from the connected counts and global totals
// (sums over all 4-subsets of: triangles, 2-paths, disjoint edge pairs,
// edges, subsets), in exact 128-bit arithmetic.
void finalize(const long long* st, int64_t n, i128 I[11]) {
  for (int c = 0; c < 6; ++c) I[c] = st[ST_F0 + c];
  const i128 T = st[ST_T], W = st[ST_W], m = st[ST_M], nn = n;
  I[6] = T * (nn - 3) - I[3] - 2 * I[4] - 4 * I[5];
  I[7] = W * (nn - 3) - 3 * I[6] - 3 * I[1] - 2 * I[0] - 4 * I[2] - 5 * I[3] - 8 * I[4] - 12 * I[5];
  I[8] = (c2w(m) - W) - I[0] - 2 * I[2] - I[3] - 2 * I[4] - 3 * I[5];
  I[9] = m * c2w(nn - 2) - 2 * I[8] - 2 * I[7] - 3 * I[6] - 3 * I[1] - 3 * I[0] - 4 * I[2] - 4 * I[3] -
         5 * I[4] - 6 * I[5];
  i128 s = 0;
  for (int c = 0; c < 10; ++c) s += I[c];
  I[10] = c4w(nn) - s;
}

// The four induced 3-vertex classes (triangle, 2-path, edge + isolated
// vertex, empty) from T, W = sum C(d,2) and m: a triangle holds three
// 2-paths, and every triple is counted by its edges in m (n - 2).
void finalize3(const long long* st, int64_t n, i128 I[4]) {
  const i128 T = st[ST_T], W = st[ST_W], m = st[ST_M], nn = n;
  I[0] = T;
  I[1] = W - 3 * T;
  I[2] = m * (nn - 2) - 2 * I[1] - 3 * I[0];
  I[3] = nn * (nn - 1) * (nn - 2) / 6 - I[0] - I[1] - I[2];
}

void to_int64(const i128 I[11], int64_t out[11], uint32_t* mask) {
  uint32_t mk = 0;
  for (int c = 0; c < 11; ++c) {
    out[c] = (int64_t)(uint64_t)I[c];
    if (I[c] > (i128)INT64_MAX || I[c] < (i128)INT64_MIN) mk |= 1u << c;
  }
  if (mask) *mask = mk;
}

// Tier thresholds: largest out-degree of the one-wave triangle tier (its bit
// matrices hold 64 slots), largest wedge bound of the one-wave and of the
// one-workgroup 4-cycle tiers (their hash tables hold twice as many).  Lower
// values are valid too; they move vertices to the next tier up.
constexpr int TRI_SMALL_MAX = 64;
constexpr int C4_SMALL_MAX = 256;
constexpr int C4_MID_MAX = 4096;

}  // namespace

void gc_set_error(const char* msg) { g_err = msg ? msg : ""; }

// Device bytes a single-graph handle reaches, from the sizing rules of
// build(), alloc_vertex_arrays() and size_count_scratch() (multi-version
// passes included), for a graph of n vertices and m edges whose largest
// degree is max_deg and whose largest out-degree under the build order is
// max_out.  Batch staging is not included.
int64_t gc_footprint_estimate(int64_t n, int64_t m, double slack, int64_t max_deg, int64_t max_out) {
  const int64_t N = std::max<int64_t>(n, 1), E = 2 * m;
  int64_t b = 0;
  // resident rows (off, len, cap, gid, ext2int, int2ext) and the arena
  b += 28 * N;
  const int64_t used = (int64_t)((1.0 + slack) * (double)E) + 2 * N;
  b += 4 * std::max<int64_t>(4 * used, used + (1 << 20));
  // per-vertex pass arrays and work lists
  b += (10 + L_NUM) * 4 * N;
  // region view of the union (entries grow by a quarter when exceeded) and
  // the merge scratch: rcol, rrow, t, vpos (20 B) + tp (16 B) per entry
  const int64_t e_alloc = E + E / 2 + (1 << 20);
  b += 36 * e_alloc + 4 * e_alloc;
  b += 8 * (N + 1) + 16 * N + 4 * GC_NV_MAX * N;  // roff, c4 keys, degrees per version
  b += (int64_t)radix_sort_tmp_bytes(std::max<int64_t>(2 * m, N)) + (int64_t)scan_tmp_bytes(N + 1);
  // hub counters of the large 4-cycle tier and their cursors
  const int64_t per = 12 * N;
  int64_t slots = std::max<int64_t>(1, std::min<int64_t>(256, ((int64_t)16 << 30) / per));
  slots = std::min<int64_t>(slots, N);
  b += slots * per;
  b += slots * 2 * (max_deg + max_deg / 4 + 64) * 8;
  // triangles above the LDS tiers
  if (max_out > tri_lds_max(4)) {
    const int64_t cap = std::min<int64_t>(32767, max_out + max_out / 8 + 16);
    b += 256 * tri_scratch_words64(4, cap) * 8;
  }
  // triangles per vertex and the edge-local passes' scratch (affected edges
  // of a batch of 2^18 updates; common neighbours per hub-counter slot)
  b += 24 * N;
  b += 2 * 8 * (8 * ((int64_t)1 << 18) + 4096);
  b += slots * (max_deg + max_deg / 4 + 4096) * 4;
  // transient arrays of the build (edge keys, directed entries, ranks)
  b += 64 * m + 24 * N;
  return b + ((int64_t)64 << 20);
}

struct gc_graph {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  gc_options opt{};
  bool broken = false;

  int32_t k = 1;
  // per graph: first internal id, id capacity (the internal id space), ids
  // issued so far, live vertices (the n of the counts)
  std::vector<int64_t> gbase, gn, gi, gl;
  // vertices taken out of V (single-graph handles): their ids stay invalid
  std::vector<uint8_t> dead_h;
  DevBuf dead_d;
  bool any_dead = false;
  int64_t N = 0;
  int bits = 1;

  // resident graph
  DevBuf off, len, cap, col, top, gid, ext2int, int2ext;
  int64_t arena_cap = 0, arena_top = 0, entries = 0;

  // small device state; vout: state after each later version of a pass
  DevBuf state, state_tmp, vout, sig, ctr, bstats, tables;
  std::vector<long long> hstate;

  // batch scratch
  DevBuf bin, keys, keys_alt, dirA, dirA_alt, dirD, dirD_alt, dirR, dirR_alt;
  DevBuf a_beg, na, r_beg, nr, mark, tix;
  DevBuf touched, dest, newcap, tlen, tpre, scratch, sort_tmp, scan_tmp;

  // region and counting
  DevBuf roff, rcol, rrow, rlow, dver, t, tp, vpos, level, rlist, rlen, lists;
  DevBuf c4_dense, c4_touch, c4_cur, c4_blk, c4_keys, c4_keys_alt, tri_scratch;
  // triangles at each vertex (kept for the edge-local passes) and the
  // scratch of those passes
  DevBuf Tv, dTs, sbt, ce, ae, ae_alt, slot_list, dctr, c4_nch, c4_side, c4_off, pair_edge, pair_len, pair_off,
      pair_merge, pair_hlen, pair_hoff, k4_s, k4_edge, k4_item, tv_items, tv_ioff;
  int64_t ae_cap = 0, slot_cap = 0, pair_cap = 0;
  // largest affected-edge and 4-cycle-pair demand per update seen in an
  // edge-local pass: later passes size their lists for their batch capacity
  // at that rate instead of finding them short and counting again
  double ae_per_update = 0, pair_per_update = 0;
  // cost model of the two kinds of one-batch pass (autotune): per
  // half-decade of batch size and kind (0 region, 1 edge-local), the mean
  // wall ms, mean batch size and passes seen; the mean of all region passes
  double mode_ms[16][2] = {};
  double mode_sz[16][2] = {};
  int64_t mode_n[16][2] = {};
  double region_ms_all = 0;
  int64_t region_n_all = 0;
  // least wall ms of an edge-local one-batch pass (< 0: none yet), taken as
  // the fixed cost of that kind (launches, ingest, purge, result copy)
  double delta_ms_min = -1;
  // mean wall ms of multi-version passes by their number of batches
  double multi_ms[GC_NV_MAX] = {};
  int64_t multi_n[GC_NV_MAX] = {};
  int64_t c4_cur_low = 0;
  int32_t c4_slots = 0, tri_slots = 0;
  int64_t c4_dense_n = 0;            // vertex count the hub counters are sized for
  int64_t tri_cap = 0;
  int64_t e_alloc = 0;               // entries of the region arrays
  int64_t seen_maxdp = 0, seen_maxlow = 0;  // largest out-degree / lower degree counted so far

  // captured passes: everything an enqueued pass depends on -> executable graph
  std::map<std::vector<uint64_t>, hipGraphExec_t> graphs;
  int64_t graph_launches = 0, graph_captures = 0;

  // tier thresholds (tri_small, c4_small, c4_mid): the best so far, those of
  // the pass being enqueued, and the trials of the autotuner (each measured
  // on a pass that counts a region anyway: time per triangle entry read for
  // the first, per wedge for the other two)
  int32_t tiers_best[3] = {TRI_SMALL_MAX, C4_SMALL_MAX, C4_MID_MAX};
  int32_t tiers_now[3] = {TRI_SMALL_MAX, C4_SMALL_MAX, C4_MID_MAX};
  bool tiers_forced = false;
  std::vector<std::array<int32_t, 3>> tier_cands{
      {TRI_SMALL_MAX, C4_SMALL_MAX, C4_MID_MAX}, {32, C4_SMALL_MAX, C4_MID_MAX}, {TRI_SMALL_MAX, 128, C4_MID_MAX},
      {TRI_SMALL_MAX, C4_SMALL_MAX, 2048}, {TRI_SMALL_MAX, C4_SMALL_MAX, 1024}};
  std::vector<double> tier_tri_cost, tier_c4_cost;
  int tier_next = 0;

  // online autotuner (speed knobs only)
  std::vector<int64_t> tune_cands{96, 192, 384, 768, 1536};
  std::vector<double> tune_ms, tune_wedges;
  int tune_next = 0;
  int64_t dense_min_best = 256;
  // rows at least this long go through a whole wave in the per-vertex pass
  // (GC_DEG_WAVE_ROW overrides it: tests lower it to reach that path)
  int32_t deg_wave_row = 1 << 16;
  double region_frac[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
  // counting attempts after the first when scratch proves too small
  // (GC_RETRY_LIMIT overrides it: tests set 0 to reach the failure path)
  int retry_limit = 2;
  // set while the resident graph holds a pass's union view (from the merge
  // until the purge has been read back): a failure then leaves it unusable
  bool in_pass = false;
  // the pass being settled has no deletions (its purge only clears flags)
  bool pass_insert_only = false;
  int64_t pass_max_dirA = 0;

  void* pin = nullptr;
  size_t pin_cap = 0;
  // pinned results of a pass: ctr [C_COUNT] | bstats [BS_COUNT] | state [k ST] |
  // vout [(GC_NV_MAX - 1) k ST] | arena top
  void* pout = nullptr;
  hipEvent_t ev[10] = {};

  ~gc_graph() {
    if (stream) (void)hipStreamSynchronize(stream);
    drop_graphs();
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (pin) (void)hipHostFree(pin);
    if (pout) (void)hipHostFree(pout);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  unsigned long long* out_ctr() const { return (unsigned long long*)pout; }
  unsigned long long* out_bst() const { return out_ctr() + C_COUNT; }
  long long* out_state() const { return (long long*)(out_bst() + BS_COUNT); }
  long long* out_vout() const { return out_state() + (size_t)k * ST_STRIDE; }
  unsigned long long* out_top() const {
    return (unsigned long long*)(out_vout() + (size_t)(GC_NV_MAX - 1) * k * ST_STRIDE);
  }
  size_t out_bytes() const {
    return (size_t)(C_COUNT + BS_COUNT + 1) * 8 + (size_t)GC_NV_MAX * k * ST_STRIDE * 8;
  }

  PoolDev pd() const {
    PoolDev P;
    P.N = N;
    P.off = off.as<int64_t>();
    P.len = len.as<int32_t>();
    P.cap = cap.as<int32_t>();
    P.col = col.as<uint32_t>();
    P.arena_cap = arena_cap;
    P.arena_top = top.as<unsigned long long>();
    P.gid = gid.as<int32_t>();
    P.ext2int = ext2int.as<int32_t>();
    return P;
  }
  RegionDev rd() const {
    RegionDev R;
    R.roff = roff.as<int64_t>();
    R.rcol = rcol.as<uint32_t>();
    R.rlow = rlow.as<int32_t>();
    R.rrow = rrow.as<int32_t>();
    R.d = dver.as<int32_t>();
    R.t = t.as<unsigned long long>();
    R.tp = tp.as<unsigned long long>();
    R.vpos = vpos.as<int32_t>();
    return R;
  }
  void* pinned(size_t bytes) {
    if (bytes > pin_cap) {
      if (pin) (void)hipHostFree(pin);
      pin = nullptr;
      size_t nb = std::max(bytes, pin_cap * 2);
      HIPCHK(hipHostMalloc(&pin, nb, hipHostMallocDefault));
      pin_cap = nb;
    }
    return pin;
  }
  void sync() { HIPCHK(hipStreamSynchronize(stream)); }
  int64_t m_total() const {
    int64_t s = 0;
    for (int g = 0; g < k; ++g) s += hstate[g * ST_STRIDE + ST_M];
    return s;
  }
};

namespace {

void zero_small(gc_graph* G) {
  fill_u64(G->ctr.as<unsigned long long>(), 0ull, C_COUNT, G->stream);
  fill_u64(G->bstats.as<unsigned long long>(), 0ull, BS_COUNT, G->stream);
  fill_u64(G->sig.as<unsigned long long>(), 0ull, (int64_t)G->k * GC_NV_MAX * SG_N, G->stream);
}

// Before a second attempt of the counting stage: its counters, statistics
// and sums (the ingest and merge counters stay).
void reset_count_stage(gc_graph* G) {
  fill_u64(G->ctr.as<unsigned long long>() + C_RLIST, 0ull, C_COUNT - C_RLIST, G->stream);
  fill_u64(G->bstats.as<unsigned long long>() + BS_COUNT_STAGE, 0ull, BS_COUNT - BS_COUNT_STAGE, G->stream);
  fill_u64(G->sig.as<unsigned long long>(), 0ull, (int64_t)G->k * GC_NV_MAX * SG_N, G->stream);
}

// Scratch of the counting stage for a union view of up to `entries` entries.
// Hub and triangle scratch follow the largest degrees counted so far; a
// kernel that meets a larger vertex asks for a second attempt (BS_RETRY).
// Allocates: never called during stream capture.
void size_count_scratch(gc_graph* G, int nv, int64_t entries) {
  const int64_t N = G->N;
  G->roff.ensure((N + 1) * sizeof(int64_t));
  G->c4_keys.ensure(N * sizeof(unsigned long long));
  G->c4_keys_alt.ensure(N * sizeof(unsigned long long));
  G->sort_tmp.ensure(radix_sort_tmp_bytes(N) + 64);
  G->scan_tmp.ensure(scan_tmp_bytes(N + 1) + 64);
  if (entries > G->e_alloc) G->e_alloc = entries + entries / 4 + 1024;
  const int64_t E = G->e_alloc;
  G->rcol.ensure(E * sizeof(uint32_t));
  G->rrow.ensure(E * sizeof(int32_t));
  G->t.ensure(E * sizeof(unsigned long long));
  G->vpos.ensure(E * sizeof(int32_t));
  if (nv > 2) G->tp.ensure(2 * E * sizeof(unsigned long long));
  G->dver.ensure((size_t)N * GC_NV_MAX * sizeof(int32_t));
  // large 4-cycle tier: dense counters per resident workgroup (one
  // 1024-thread block per CU fills the chip)
  const int64_t per = N * (int64_t)(sizeof(unsigned long long) + sizeof(int32_t));
  int64_t slots = std::max<int64_t>(1, std::min<int64_t>(256, ((int64_t)16 << 30) / std::max<int64_t>(per, 1)));
  slots = std::min<int64_t>(slots, std::max<int64_t>(1, N));
  // (re)sized when more slots fit or the id space changed: slot j of vertex
  // v is word j * N + v
  if (slots > G->c4_slots || N != G->c4_dense_n) {
    G->c4_dense.release();
    G->c4_touch.release();
    G->c4_dense.ensure((size_t)(slots * N) * sizeof(unsigned long long));
    G->c4_touch.ensure((size_t)(slots * N) * sizeof(int32_t));
    fill_u64(G->c4_dense.as<unsigned long long>(), 0ull, slots * N, G->stream);
    G->c4_slots = (int32_t)slots;
    G->c4_dense_n = N;
  }
  if (G->seen_maxlow > G->c4_cur_low) G->c4_cur_low = G->seen_maxlow + G->seen_maxlow / 4 + 64;
  G->c4_cur_low = std::max<int64_t>(G->c4_cur_low, 64);
  G->c4_cur.ensure((size_t)(G->c4_slots * 2 * G->c4_cur_low) * sizeof(int64_t));
  G->c4_blk.ensure((size_t)(N / c4_block_ids() + 2) * sizeof(int32_t));
  // triangles above the LDS tiers: scratch slots in global memory
  if (G->seen_maxdp > tri_lds_max(nv)) {
    if (G->seen_maxdp > 32767)
      raise(GC_EINVAL, "oriented out-degree %lld exceeds the supported 32767", (long long)G->seen_maxdp);
    const int64_t cap = std::max<int64_t>(G->tri_cap, std::min<int64_t>(32767, G->seen_maxdp + G->seen_maxdp / 8 + 16));
    const size_t need = (size_t)(tri_scratch_words64(nv, cap) * 256) * sizeof(unsigned long long);
    if (need > G->tri_scratch.cap) {
      G->tri_scratch.release();
      G->tri_scratch.ensure(need);
    }
    G->tri_cap = cap;
    G->tri_slots = 256;
  }
}

// nullptr when size_count_scratch(G, nv, entries) would neither allocate nor
// change a size; else the part that would.
const char* count_scratch_short(const gc_graph* G, int nv, int64_t entries) {
  const int64_t N = G->N;
  auto has = [](const DevBuf& b, size_t bytes) { return b.p != nullptr && std::max<size_t>(bytes, 16) <= b.cap; };
  if (!has(G->roff, (N + 1) * sizeof(int64_t)) || !has(G->c4_keys, N * sizeof(unsigned long long)) ||
      !has(G->c4_keys_alt, N * sizeof(unsigned long long)))
    return "per-vertex region arrays";
  if (!has(G->sort_tmp, radix_sort_tmp_bytes(N) + 64) || !has(G->scan_tmp, scan_tmp_bytes(N + 1) + 64))
    return "sort and scan temporaries";
  if (entries > G->e_alloc) return "region view (entries)";
  const int64_t E = G->e_alloc;
  if (!has(G->rcol, E * sizeof(uint32_t)) || !has(G->rrow, E * sizeof(int32_t)) ||
      !has(G->t, E * sizeof(unsigned long long)) || !has(G->vpos, E * sizeof(int32_t)))
    return "region view (arrays)";
  if (nv > 2 && !has(G->tp, 2 * E * sizeof(unsigned long long))) return "multi-version triangle counts";
  if (!has(G->dver, (size_t)N * GC_NV_MAX * sizeof(int32_t))) return "per-version degrees";
  const int64_t per = N * (int64_t)(sizeof(unsigned long long) + sizeof(int32_t));
  int64_t slots = std::max<int64_t>(1, std::min<int64_t>(256, ((int64_t)16 << 30) / std::max<int64_t>(per, 1)));
  slots = std::min<int64_t>(slots, std::max<int64_t>(1, N));
  if (slots > G->c4_slots || N != G->c4_dense_n) return "hub counters";
  if (G->seen_maxlow > G->c4_cur_low || G->c4_cur_low < 64) return "hub cursors (lower degree)";
  if (!has(G->c4_cur, (size_t)(G->c4_slots * 2 * G->c4_cur_low) * sizeof(int64_t))) return "hub cursors";
  if (!has(G->c4_blk, (size_t)(N / c4_block_ids() + 2) * sizeof(int32_t))) return "4-cycle blocks";
  if (G->seen_maxdp > tri_lds_max(nv)) {
    if (G->seen_maxdp > 32767) return "triangle scratch (out-degree above 32767)";
    const int64_t cap = std::max<int64_t>(G->tri_cap, std::min<int64_t>(32767, G->seen_maxdp + G->seen_maxdp / 8 + 16));
    if (cap != G->tri_cap) return "triangle scratch (out-degree)";
    if ((size_t)(tri_scratch_words64(nv, cap) * 256) * sizeof(unsigned long long) > G->tri_scratch.cap)
      return "triangle scratch";
  }
  return nullptr;
}

CountArgs make_count_args(gc_graph* G, int nv, int64_t dense_min, bool fresh) {
  (void)nv;
  CountArgs A;
  A.R = G->rd();
  A.gid = G->gid.as<int32_t>();
  A.lists = G->lists.as<int32_t>();
  A.list_stride = G->N;
  A.c = G->ctr.as<unsigned long long>();
  A.sig = G->sig.as<unsigned long long>();
  A.bstats = G->bstats.as<unsigned long long>();
  A.N = G->N;
  // window of the large 4-cycle tier; GC_C4_WINDOW / GC_C4_NARROW_MAX /
  // GC_C4_DENSE_MIN override the defaults (tests shrink them to reach every
  // path on small graphs)
  A.c4_win = c4_window_max();
  A.c4_narrow_max = 65535;
  if (const char* e = std::getenv("GC_C4_WINDOW")) A.c4_win = std::max(64, std::min(c4_window_max(), std::atoi(e)));
  A.c4_win &= ~1;  // the window is scanned 16 bytes at a time
  if (const char* e = std::getenv("GC_C4_NARROW_MAX")) A.c4_narrow_max = std::max(0, std::min(65535, std::atoi(e)));
  A.c4_dense_min = dense_min;
  // the hub windows count the wedges present in every version; in a count of
  // a whole graph inserted into the empty one, version 0 has none
  A.c4_ref = (1u << nv) - 1u;
  if (fresh) A.c4_ref &= ~1u;
  if (const char* e = std::getenv("GC_C4_DENSE_MIN")) A.c4_dense_min = std::max<int64_t>(0, std::atoll(e));
  A.c4_cur = G->c4_cur.as<int64_t>();
  A.c4_blk = G->c4_blk.as<int32_t>();
  A.c4_maxlow = G->c4_cur_low;
  A.c4_keys = G->c4_keys.as<unsigned long long>();
  A.c4_keys_alt = G->c4_keys_alt.as<unsigned long long>();
  A.sort_tmp = G->sort_tmp.p;
  A.c4_dense = G->c4_dense.as<unsigned long long>();
  A.c4_touch = G->c4_touch.as<int32_t>();
  A.slots = std::max(1, G->c4_slots);
  A.tri_scratch = G->tri_scratch.as<unsigned long long>();
  A.tri_cap = G->tri_cap;
  A.tri_slots = 256;  // blocks of the global-scratch tier (no slot is used while tri_cap == 0)
  A.e_max = G->e_alloc;
  return A;
}

// Region + per-vertex pass + counting over nv versions + combine into
// `state_d` (and G->vout for every later version).  `radius` < 0 counts
// every vertex.  Enqueue only: no allocation, no synchronisation.
void enqueue_count(gc_graph* G, int nv, int radius, long long* state_d, BatchWork& W, const CountArgs& A, bool timed,
                   bool tv) {
  hipStream_t s = G->stream;
  PoolDev P = G->pd();
  launch_region(P, W, radius, G->level.as<int32_t>(), G->rlist.as<int32_t>(), G->rlen.as<int32_t>(), s);
  launch_region_fill(P, A.R, W, radius, G->level.as<int32_t>(), G->rlist.as<int32_t>(), G->rlen.as<int32_t>(),
                     G->scan_tmp.p, s);
  launch_degrees(nv, A.R, G->gid.as<int32_t>(), G->rlist.as<int32_t>(), G->ctr.as<unsigned long long>(),
                 G->sig.as<unsigned long long>(), G->lists.as<int32_t>(), G->N, G->tiers_now[0], G->tiers_now[1], G->tiers_now[2],
                 G->deg_wave_row, G->bstats.as<unsigned long long>(), G->c4_keys.as<unsigned long long>(), s);
  if (timed) HIPCHK(hipEventRecord(G->ev[1], s));
  launch_count(nv, A, s, timed ? &G->ev[2] : nullptr);
  if (tv)
    launch_tv_region(nv, A.R, G->rlist.as<int32_t>(), G->ctr.as<unsigned long long>(), G->dTs.as<unsigned long long>(),
                     G->Tv.as<long long>(), G->bstats.as<unsigned long long>(), s);
  launch_combine(nv, G->sig.as<unsigned long long>(), state_d, G->vout.as<long long>(), G->k,
                 G->bstats.as<unsigned long long>(), s);
}

// Results of a pass into the pinned buffer (enqueue only).
void enqueue_readback(gc_graph* G, const long long* state_d) {
  hipStream_t s = G->stream;
  const size_t st = (size_t)G->k * ST_STRIDE * 8;
  HIPCHK(hipMemcpyAsync(G->out_ctr(), G->ctr.p, C_COUNT * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(G->out_bst(), G->bstats.p, BS_COUNT * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(G->out_state(), state_d, st, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(G->out_vout(), G->vout.p, (GC_NV_MAX - 1) * st, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(G->out_top(), G->top.p, 8, hipMemcpyDeviceToHost, s));
}

void note_maxima(gc_graph* G) {
  G->seen_maxdp = std::max<int64_t>(G->seen_maxdp, (int64_t)G->out_ctr()[C_MAXDP]);
  G->seen_maxlow = std::max<int64_t>(G->seen_maxlow, (int64_t)G->out_ctr()[C_MAXLOW]);
}

// The purge of the current pass: rows drop the entries absent from the last
// version and lose every flag (a pass without deletions only clears flags).
void enqueue_purge(gc_graph* G, BatchWork& W, int64_t max_touched, int nv) {
  const unsigned long long* skip = G->bstats.as<unsigned long long>() + BS_RETRY;
  if (G->pass_insert_only)
    launch_purge_insert_only(G->pd(), W, max_touched, G->pass_max_dirA, G->bits, skip, G->stream);
  else
    launch_purge(G->pd(), W, max_touched, G->bits, 1u << (GC_VSHIFT + nv - 1), skip, G->scan_tmp.p, G->stream);
}

// After a pass whose results are in the pinned buffer: while a kernel asked
// for more scratch (the combine and the purge then changed nothing), grow it
// from the observed degrees and count again.  Returns the attempts made.
int settle_retries(gc_graph* G, int nv, int radius, long long* state_d, BatchWork& W, int64_t dense_min,
                   int64_t entries, bool purge, int64_t max_touched, bool fresh, bool tv) {
  int attempts = 0;
  while (G->out_bst()[BS_RETRY]) {
    if (++attempts > G->retry_limit)
      raise(GC_EDEVICE, "counting scratch still too small after %d more attempts", G->retry_limit);
    note_maxima(G);
    size_count_scratch(G, nv, entries);
    reset_count_stage(G);
    CountArgs A = make_count_args(G, nv, dense_min, fresh);
    enqueue_count(G, nv, radius, state_d, W, A, false, tv);
    if (purge)
      enqueue_purge(G, W, max_touched, nv);
    enqueue_readback(G, state_d);
    G->sync();
  }
  note_maxima(G);
  return attempts;
}

// Per-batch staging of a pass: the input table and the batch's keys, the
// directed merge lists and the per-touched-row arrays.  The handle's own
// buffers, or (gc_apply_batch_dev_noalloc) pieces of the static scratch.
struct Staging {
  void* bin = nullptr;
  unsigned long long *keys = nullptr, *keys_alt = nullptr, *dirA = nullptr, *dirA_alt = nullptr;
  unsigned long long *dirD = nullptr, *dirD_alt = nullptr, *dirR = nullptr, *dirR_alt = nullptr;
  int32_t* touched = nullptr;
  int64_t* dest = nullptr;
  int32_t* newcap = nullptr;
  int32_t* tlen = nullptr;
  int64_t* tpre = nullptr;
};

Staging handle_staging(gc_graph* G) {
  Staging S;
  S.bin = G->bin.p;
  S.keys = G->keys.as<unsigned long long>();
  S.keys_alt = G->keys_alt.as<unsigned long long>();
  S.dirA = G->dirA.as<unsigned long long>();
  S.dirA_alt = G->dirA_alt.as<unsigned long long>();
  S.dirD = G->dirD.as<unsigned long long>();
  S.dirD_alt = G->dirD_alt.as<unsigned long long>();
  S.dirR = G->dirR.as<unsigned long long>();
  S.dirR_alt = G->dirR_alt.as<unsigned long long>();
  S.touched = G->touched.as<int32_t>();
  S.dest = G->dest.as<int64_t>();
  S.newcap = G->newcap.as<int32_t>();
  S.tlen = G->tlen.as<int32_t>();
  S.tpre = G->tpre.as<int64_t>();
  return S;
}

BatchWork make_work(gc_graph* G, const Staging& S) {
  BatchWork W;
  W.c = G->ctr.as<unsigned long long>();
  W.dirA = S.dirA;
  W.dirD = S.dirD;
  W.dirR = S.dirR;
  W.a_beg = G->a_beg.as<int32_t>();
  W.na = G->na.as<int32_t>();
  W.r_beg = G->r_beg.as<int32_t>();
  W.nr = G->nr.as<int32_t>();
  W.mark = G->mark.as<int32_t>();
  W.tix = G->tix.as<int32_t>();
  W.touched = S.touched;
  W.dest = S.dest;
  W.newcap = S.newcap;
  W.tlen = S.tlen;
  W.tpre = S.tpre;
  W.scratch = G->scratch.as<uint32_t>();
  return W;
}

BatchWork make_work(gc_graph* G) { return make_work(G, handle_staging(G)); }

void alloc_vertex_arrays(gc_graph* G) {
  const int64_t N = G->N;
  hipStream_t s = G->stream;
  for (DevBuf* b : {&G->a_beg, &G->na, &G->r_beg, &G->nr, &G->mark, &G->tix}) {
    b->ensure(N * sizeof(int32_t));
    fill_u32(b->as<uint32_t>(), 0u, N, s);
  }
  for (DevBuf* b : {&G->rlow, &G->level, &G->rlist, &G->rlen}) b->ensure(N * sizeof(int32_t));
  G->lists.ensure((size_t)L_NUM * N * sizeof(int32_t));
  G->state.ensure((size_t)G->k * ST_STRIDE * sizeof(long long));
  G->state_tmp.ensure((size_t)G->k * ST_STRIDE * sizeof(long long));
  G->vout.ensure((size_t)(GC_NV_MAX - 1) * G->k * ST_STRIDE * sizeof(long long));
  G->sig.ensure((size_t)G->k * GC_NV_MAX * SG_N * sizeof(unsigned long long));
  G->ctr.ensure(C_COUNT * sizeof(unsigned long long));
  G->bstats.ensure(BS_COUNT * sizeof(unsigned long long));
  G->top.ensure(sizeof(unsigned long long));
  for (DevBuf* b : {&G->Tv, &G->dTs, &G->sbt}) {
    b->ensure(N * sizeof(long long));
    fill_u64(b->as<unsigned long long>(), 0ull, N, s);
  }
  G->dctr.ensure(DC_COUNT * sizeof(unsigned long long));
  if (!G->pout) HIPCHK(hipHostMalloc(&G->pout, G->out_bytes(), hipHostMallocDefault));
}

// fresh arena with new slack; keeps ids
void compact(gc_graph* G, int64_t extra) {
  hipStream_t s = G->stream;
  const int64_t N = G->N;
  DevBuf ncap, noff, ncol;
  ncap.ensure(N * sizeof(int32_t));
  noff.ensure((N + 1) * sizeof(int64_t));
  PoolDev P = G->pd();
  P.cap = ncap.as<int32_t>();
  launch_caps(P, G->opt.slack, s);
  G->scan_tmp.ensure(scan_tmp_bytes(N + 1) + 64);
  exclusive_scan_i32_to_i64(ncap.as<int32_t>(), noff.as<int64_t>(), N, G->scan_tmp.p, s);
  int64_t used = 0;
  HIPCHK(hipMemcpyAsync(&used, noff.as<int64_t>() + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  G->sync();
  int64_t capn = std::max<int64_t>(4 * used, used + extra + (1 << 20));
  ncol.ensure((size_t)capn * sizeof(uint32_t));
  launch_compact(G->pd(), noff.as<int64_t>(), ncol.as<uint32_t>(), s);
  G->sync();
  G->col.swap(ncol);
  G->off.swap(noff);
  G->cap.swap(ncap);
  G->arena_cap = capn;
  G->arena_top = used;
  HIPCHK(hipMemcpyAsync(G->top.p, &G->arena_top, sizeof(int64_t), hipMemcpyHostToDevice, s));
  G->sync();
}

void read_state(gc_graph* G) {
  G->hstate.resize((size_t)G->k * ST_STRIDE);
  HIPCHK(hipMemcpyAsync(G->hstate.data(), G->state.p, G->hstate.size() * sizeof(long long), hipMemcpyDeviceToHost,
                        G->stream));
  G->sync();
}

// Address of the static staging array on each device, looked up once per
// device with that device current (at the first handle built on it).
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

void noalloc_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) raise(GC_EDEVICE, "device %d beyond the supported %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) raise(GC_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  g_noalloc_ptr[device] = ptr;
}

void* noalloc_scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  return (device >= 0 && device < kMaxDevices) ? g_noalloc_ptr[device] : nullptr;
}

void setup_handle(gc_graph* G, const gc_options* opt) {
  if (opt) G->opt = *opt; else gc_options_default(&G->opt);
  if (const char* e = std::getenv("GC_DEG_WAVE_ROW")) G->deg_wave_row = std::max(1, std::min(1 << 16, std::atoi(e)));
  if (const char* e = std::getenv("GC_RETRY_LIMIT")) G->retry_limit = std::max(0, std::min(8, std::atoi(e)));
  if (G->opt.radius < 0 || G->opt.radius > 4) raise(GC_EINVAL, "radius must be in [0, 4]");
  if (!(G->opt.slack >= 0.0f && G->opt.slack <= 16.0f)) raise(GC_EINVAL, "slack must be in [0, 16]");
  {
    const int32_t ts = G->opt.tri_small_max, cs = G->opt.c4_small_max, cm = G->opt.c4_mid_max;
    if (ts || cs || cm) {
      const int32_t t0 = ts ? ts : TRI_SMALL_MAX, c0 = cs ? cs : C4_SMALL_MAX, m0 = cm ? cm : C4_MID_MAX;
      if (t0 < 1 || t0 > TRI_SMALL_MAX) raise(GC_EINVAL, "tri_small_max must be in [1, %d]", TRI_SMALL_MAX);
      if (c0 < 1 || c0 > C4_SMALL_MAX) raise(GC_EINVAL, "c4_small_max must be in [1, %d]", C4_SMALL_MAX);
      if (m0 < c0 || m0 > C4_MID_MAX) raise(GC_EINVAL, "c4_mid_max must be in [c4_small_max, %d]", C4_MID_MAX);
      G->tiers_best[0] = G->tiers_now[0] = t0;
      G->tiers_best[1] = G->tiers_now[1] = c0;
      G->tiers_best[2] = G->tiers_now[2] = m0;
      G->tiers_forced = true;
    }
  }
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (G->opt.device < 0 || G->opt.device >= ndev) raise(GC_EDEVICE, "device %d not present", G->opt.device);
  G->device = G->opt.device;
  HIPCHK(hipSetDevice(G->device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, G->device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    raise(GC_EDEVICE, "device %d is %s; this library is built for gfx950", G->device, prop.gcnArchName);
  noalloc_scratch_setup(G->device);
  if (G->opt.stream) {
    G->stream = (hipStream_t)G->opt.stream;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&G->stream, hipStreamNonBlocking));
    G->own_stream = true;
  }
  for (auto& e : G->ev) HIPCHK(hipEventCreate(&e));
}

// Build k graphs from host edge lists and count them (one insertion batch
// into the empty graph: version b is empty, every entry carries F_NEW).
void build(gc_graph* G, int32_t k, const int64_t* n, const int32_t* const* src, const int32_t* const* dst,
           const int64_t* m) {
  hipStream_t s = G->stream;
  G->k = k;
  G->gbase.assign(k, 0);
  G->gn.assign(n, n + k);
  G->gi.assign(n, n + k);
  G->gl.assign(n, n + k);
  int64_t N = 0, M = 0, maxn = 1;
  for (int g = 0; g < k; ++g) {
    if (n[g] < 1) raise(GC_EINVAL, "graph %d: n must be >= 1", g);
    if (m[g] < 0) raise(GC_EINVAL, "graph %d: negative edge count", g);
    if (m[g] > 0 && (!src || !src[g] || !dst || !dst[g])) raise(GC_EINVAL, "graph %d: null edge arrays", g);
    G->gbase[g] = N;
    N += n[g];
    M += m[g];
    maxn = std::max(maxn, n[g]);
    for (int64_t i = 0; i < m[g]; ++i)
      if (src[g][i] < 0 || src[g][i] >= n[g] || dst[g][i] < 0 || dst[g][i] >= n[g])
        raise(GC_EINVAL, "graph %d: edge %lld has a vertex id outside [0, %lld)", g, (long long)i, (long long)n[g]);
  }
  if (N >= GC_MAX_VERTICES) raise(GC_EINVAL, "total vertex count must be below 2^28");
  G->N = N;
  G->bits = bits_for(N);
  const int lbits = bits_for(maxn + 1);
  const int gbits = k > 1 ? bits_for(k) : 0;
  if (gbits + 2 * lbits > 64) raise(GC_EINVAL, "graphs too large for one pool");

  alloc_vertex_arrays(G);
  // per-vertex graph ids
  {
    std::vector<int32_t> gid(N);
    for (int g = 0; g < k; ++g) std::fill(gid.begin() + G->gbase[g], gid.begin() + G->gbase[g] + n[g], g);
    G->gid.ensure(N * sizeof(int32_t));
    HIPCHK(hipMemcpyAsync(G->gid.p, gid.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, s));
    G->sync();
  }
  // upload the edge lists and the segment tables
  DevBuf esrc, edst, seg, gb;
  esrc.ensure(std::max<int64_t>(M, 1) * sizeof(int32_t));
  edst.ensure(std::max<int64_t>(M, 1) * sizeof(int32_t));
  std::vector<int64_t> hseg(k + 1, 0);
  for (int g = 0; g < k; ++g) {
    hseg[g + 1] = hseg[g] + m[g];
    if (m[g]) {
      HIPCHK(hipMemcpyAsync(esrc.as<int32_t>() + hseg[g], src[g], m[g] * sizeof(int32_t), hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(edst.as<int32_t>() + hseg[g], dst[g], m[g] * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
  }
  seg.ensure((k + 1) * sizeof(int64_t));
  gb.ensure(k * sizeof(int64_t));
  HIPCHK(hipMemcpyAsync(seg.p, hseg.data(), (k + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(gb.p, G->gbase.data(), k * sizeof(int64_t), hipMemcpyHostToDevice, s));

  zero_small(G);
  DevBuf ek, ek2, uniq, deg;
  ek.ensure(std::max<int64_t>(M, 1) * 8);
  ek2.ensure(std::max<int64_t>(M, 1) * 8);
  uniq.ensure(std::max<int64_t>(M, 1) * 8);
  deg.ensure(N * sizeof(int32_t));
  fill_u32(deg.as<uint32_t>(), 0u, N, s);
  G->sort_tmp.ensure(radix_sort_tmp_bytes(std::max<int64_t>(2 * M, N)) + 64);
  launch_init_keys(esrc.as<int32_t>(), edst.as<int32_t>(), M, seg.as<int64_t>(), gb.as<int64_t>(), k, G->bits,
                   ek.as<unsigned long long>(), s);
  unsigned long long* sk =
      radix_sort_u64(ek.as<unsigned long long>(), ek2.as<unsigned long long>(), G->sort_tmp.p, M, nullptr,
                     2 * G->bits, s);
  launch_init_unique(sk, M, G->bits, uniq.as<unsigned long long>(), G->ctr.as<unsigned long long>(),
                     deg.as<int32_t>(), s);
  // rank: (graph, degree, local id)
  G->ext2int.ensure(N * sizeof(int32_t));
  G->int2ext.ensure(N * sizeof(int32_t));
  DevBuf rk, rk2;
  rk.ensure(N * 8);
  rk2.ensure(N * 8);
  launch_rank(deg.as<int32_t>(), G->gid.as<int32_t>(), gb.as<int64_t>(), N, lbits, gbits + 2 * lbits,
              rk.as<unsigned long long>(), rk2.as<unsigned long long>(), G->sort_tmp.p, G->ext2int.as<int32_t>(),
              G->int2ext.as<int32_t>(), s);
  // directed entries in internal ids
  DevBuf dir, dir2;
  dir.ensure(std::max<int64_t>(2 * M, 1) * 8);
  dir2.ensure(std::max<int64_t>(2 * M, 1) * 8);
  G->len.ensure(N * sizeof(int32_t));
  fill_u32(G->len.as<uint32_t>(), 0u, N, s);
  launch_init_dir(uniq.as<unsigned long long>(), M, G->ctr.as<unsigned long long>(), G->bits, G->ext2int.as<int32_t>(),
                  dir.as<unsigned long long>(), G->len.as<int32_t>(), s);
  unsigned long long mu = 0;
  HIPCHK(hipMemcpyAsync(&mu, G->ctr.as<unsigned long long>() + C_DIRA, 8, hipMemcpyDeviceToHost, s));
  G->sync();
  const int64_t nd = 2 * (int64_t)mu;
  unsigned long long* sd = radix_sort_u64(dir.as<unsigned long long>(), dir2.as<unsigned long long>(), G->sort_tmp.p,
                                          nd, nullptr, 2 * G->bits, s);
  // rows with slack
  G->cap.ensure(N * sizeof(int32_t));
  G->off.ensure((N + 1) * sizeof(int64_t));
  DevBuf rstart;
  rstart.ensure((N + 1) * sizeof(int64_t));
  G->scan_tmp.ensure(scan_tmp_bytes(N + 1) + 64);
  PoolDev P = G->pd();
  launch_caps(P, G->opt.slack, s);
  exclusive_scan_i32_to_i64(P.len, rstart.as<int64_t>(), N, G->scan_tmp.p, s);
  exclusive_scan_i32_to_i64(P.cap, P.off, N, G->scan_tmp.p, s);
  int64_t used = 0;
  HIPCHK(hipMemcpyAsync(&used, P.off + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  G->sync();
  G->arena_cap = std::max<int64_t>(4 * used, used + (1 << 20));
  G->col.ensure((size_t)G->arena_cap * sizeof(uint32_t));
  G->arena_top = used;
  HIPCHK(hipMemcpyAsync(G->top.p, &G->arena_top, sizeof(int64_t), hipMemcpyHostToDevice, s));
  P = G->pd();
  launch_init_csr(P, sd, nd, G->ctr.as<unsigned long long>(), G->bits, rstart.as<int64_t>(), G->opt.slack,
                  G->scan_tmp.p, GC_F_NEW, s);
  // the fill kernel reads the number of edges from ctr[C_DIRA]
  // count: whole graph, version b empty
  fill_u64((unsigned long long*)G->state.p, 0ull, (int64_t)k * ST_STRIDE, s);
  zero_small(G);
  BatchWork W = make_work(G);
  size_count_scratch(G, 2, nd);
  // the merge's copy of the touched rows, as large as the region view, so
  // that a batch can be applied without growing it
  G->scratch.ensure(std::max<int64_t>(G->e_alloc, 1) * 4);
  // sort and scan temporaries for batches up to the allocation-free limit
  // (2^18 insertions and 2^18 deletions: 2^20 touched rows at most)
  G->sort_tmp.ensure(radix_sort_tmp_bytes(std::max<int64_t>(std::max<int64_t>(2 * M, N), 1 << 20)) + 64);
  G->scan_tmp.ensure(scan_tmp_bytes(std::max<int64_t>(N, 1 << 20) + 1) + 64);
  enqueue_count(G, 2, -1, G->state.as<long long>(), W, make_count_args(G, 2, G->dense_min_best, true), false, true);
  enqueue_readback(G, G->state.as<long long>());
  G->sync();
  settle_retries(G, 2, -1, G->state.as<long long>(), W, G->dense_min_best, nd, false, 0, true, true);
  launch_all_flags(P, 0u, GC_ID, s);
  G->sync();
  G->entries = nd;
  read_state(G);
  for (int g = 0; g < k; ++g)
    if (G->hstate[g * ST_STRIDE + ST_ERR]) raise(GC_EDEVICE, "graph %d: inexact totals in the initial count", g);
  for (int g = 0; g < k; ++g) G->hstate[g * ST_STRIDE + ST_N] = n[g];
}

void fill_stats(gc_graph* G, gc_batch_stats* st, const unsigned long long* hb, const unsigned long long* hc, int j,
                int nb, int64_t n_ins, int64_t n_del, bool timed, double ms_total, uint32_t ovf) {
  if (!st) return;
  std::memset(st, 0, sizeof(*st));
  st->offered_ins = n_ins;
  st->offered_del = n_del;
  st->eff_ins = (int64_t)hb[PB_IDX(j, PB_EFF_INS)];
  st->eff_del = (int64_t)hb[PB_IDX(j, PB_EFF_DEL)];
  st->loops = (int64_t)hb[PB_IDX(j, PB_LOOPS)];
  st->dups = (int64_t)hb[PB_IDX(j, PB_DUPS)];
  st->cancelled = (int64_t)hb[PB_IDX(j, PB_CANCEL)];
  st->ins_existing = (int64_t)hb[PB_IDX(j, PB_INS_EXIST)];
  st->del_missing = (int64_t)hb[PB_IDX(j, PB_DEL_MISS)];
  st->touched_vertices = (int64_t)hc[C_TOUCH];
  st->region_vertices = (int64_t)hc[C_RLIST];
  st->region_entries = (int64_t)hc[C_ER];
  st->wedges = (int64_t)hb[BS_WEDGES];
  st->c4_entries_small = (int64_t)hb[BS_C4_S];
  st->c4_entries_mid = (int64_t)hb[BS_C4_M];
  st->c4_entries_large = (int64_t)hb[BS_C4_L];
  st->c4_tail_wedges = (int64_t)hb[BS_TRIPROBE];
  st->max_out_degree = (int64_t)hc[C_MAXDP];
  st->tier_tri_small = (int64_t)hc[C_LIST0 + L_TRI_S];
  st->tier_tri_large = 0;
  for (int L = L_TRI_1; L <= L_TRI_G; ++L) st->tier_tri_large += (int64_t)hc[C_LIST0 + L];
  st->tier_c4_small = (int64_t)hc[C_LIST0 + L_C4_S];
  st->tier_c4_mid = (int64_t)hc[C_LIST0 + L_C4_M];
  st->tier_c4_large = (int64_t)hc[C_LIST0 + L_C4_L];
  st->overflow_mask = ovf;
  st->pass_batches = nb;
  st->c4_windows = (int64_t)hb[BS_C4_WINDOWS];
  st->c4_searches = (int64_t)hb[BS_C4_SEARCH];
  st->tri_global_vertices = (int64_t)hb[BS_TRI_GLOBAL];
  st->tri_exc_rebuilds = (int64_t)hb[BS_TRI_REBUILD];
  st->tri_entries = (int64_t)hb[BS_TRI_E];
  st->k4_split_edges = (int64_t)hb[BS_K4_SPLIT];
  st->delta = 0;
  st->ms_total = (float)ms_total;
  if (timed) {
    float a = 0;
    (void)hipEventElapsedTime(&a, G->ev[0], G->ev[1]); st->ms_prepare = a;
    (void)hipEventElapsedTime(&a, G->ev[2], G->ev[3]); st->ms_tri = a;
    (void)hipEventElapsedTime(&a, G->ev[3], G->ev[4]); st->ms_edge = a;
    (void)hipEventElapsedTime(&a, G->ev[4], G->ev[5]); st->ms_c4_small = a;
    (void)hipEventElapsedTime(&a, G->ev[5], G->ev[6]); st->ms_c4_mid = a;
    (void)hipEventElapsedTime(&a, G->ev[6], G->ev[7]); st->ms_c4_large = a;
    (void)hipEventElapsedTime(&a, G->ev[7], G->ev[8]); st->ms_finish = a;
  }
}

// Host-side check of one batch's arrays (sizes, pointers, ids in [0, n)).
void check_batch(const gc_batch_desc& b, int64_t n, int which, const uint8_t* dead = nullptr) {
  if (b.n_ins < 0 || b.n_del < 0) raise(GC_EINVAL, "batch %d: negative size", which);
  if ((b.n_ins && (!b.ins_src || !b.ins_dst)) || (b.n_del && (!b.del_src || !b.del_dst)))
    raise(GC_EINVAL, "batch %d: null array", which);
  auto bad = [&](int32_t x) { return x < 0 || x >= n || (dead && dead[x]); };
  for (int64_t i = 0; i < b.n_ins; ++i)
    if (bad(b.ins_src[i]) || bad(b.ins_dst[i]))
      raise(GC_EINVAL, "batch %d: insertion %lld has a vertex id outside [0, %lld) or of a removed vertex", which,
            (long long)i, (long long)n);
  for (int64_t i = 0; i < b.n_del; ++i)
    if (bad(b.del_src[i]) || bad(b.del_dst[i]))
      raise(GC_EINVAL, "batch %d: deletion %lld has a vertex id outside [0, %lld) or of a removed vertex", which,
            (long long)i, (long long)n);
}

int64_t pow2_at_least(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Host-side sizes of one pass.  Array layouts and grids use the capacities
// (powers of two), so passes whose batches fall in the same capacity class
// enqueue the same work and can replay one captured graph.
struct PassPlan {
  int nseg = 1, npass = 1, nv = 2;
  bool seq = false, dev = false;
  int64_t ni = 0, ndl = 0, total = 0;
  int64_t cap_i = 1, cap_d = 1, cap_t = 2, max_touched = 2, union_bound = 0;
  size_t tab_words = 0, in_bytes = 0;
  int radius = 2;
  int64_t dense_min = 256;
  bool delta = false;  // edge-local pass (one batch per graph) instead of the region count
};

DeltaArgs make_delta_args(gc_graph* G, const BatchWork& W) {
  DeltaArgs D;
  D.P = G->pd();
  D.N = G->N;
  D.bits = G->bits;
  D.dirA = W.dirA;
  D.dirD = W.dirD;
  D.c = G->ctr.as<unsigned long long>();
  D.touched = W.touched;
  D.mark = W.mark;
  D.gid = G->gid.as<int32_t>();
  D.sig = G->sig.as<unsigned long long>();
  D.bstats = G->bstats.as<unsigned long long>();
  D.dd = G->dver.as<int32_t>();
  D.Tv = G->Tv.as<long long>();
  D.dT = G->dTs.as<unsigned long long>();
  D.sbt = G->sbt.as<unsigned long long>();
  D.ce = G->ce.as<unsigned long long>();
  D.ce_cap = (int64_t)(G->ce.cap / 8);
  D.ae = G->ae.as<unsigned long long>();
  D.ae_alt = G->ae_alt.as<unsigned long long>();
  D.ae_cap = G->ae_cap;
  D.sort_tmp = G->sort_tmp.p;
  D.slot_mark = G->c4_dense.as<unsigned long long>();
  D.slot_list = G->slot_list.as<uint32_t>();
  D.slot_cap = G->slot_cap;
  D.dc = G->dctr.as<unsigned long long>();
  D.c4_nch = G->c4_nch.as<int32_t>();
  D.c4_side = G->c4_side.as<int32_t>();
  D.c4_off = G->c4_off.as<int64_t>();
  D.pair_edge = G->pair_edge.as<int32_t>();
  D.pair_len = G->pair_len.as<int32_t>();
  D.pair_merge = G->pair_merge.as<int32_t>();
  D.k4_s = G->k4_s.as<uint32_t>();
  D.k4_edge = G->k4_edge.as<int64_t>();
  D.k4_item = G->k4_item.as<int32_t>();
  D.tv_items = G->tv_items.as<int32_t>();
  D.tv_ioff = G->tv_ioff.as<int64_t>();
  D.tcap = 2 * (int64_t)(G->ce.cap / 8);
  D.pair_off = G->pair_off.as<int64_t>();
  D.pair_hlen = G->pair_hlen.as<int32_t>();
  D.pair_hoff = G->pair_hoff.as<int64_t>();
  D.pair_cap = G->pair_cap;
  D.scan_tmp = G->scan_tmp.p;
  return D;
}

// Buffers of an edge-local pass for batches of capacity cap_t (allocates:
// never called during stream capture).
void size_delta(gc_graph* G, int64_t cap_t, int64_t ae_need, int64_t slot_need, int64_t pair_need = 0) {
  const int64_t ce_cap = std::max<int64_t>(cap_t, 64);
  G->ce.ensure(ce_cap * 8);
  G->c4_nch.ensure(G->ce.cap / 8 * 4);
  G->c4_side.ensure(G->ce.cap / 8 * 4);
  G->c4_off.ensure((G->ce.cap / 8 + 1) * 8);
  G->pair_cap = std::max<int64_t>(G->pair_cap, std::max<int64_t>(pair_need, 64 * cap_t + 4096));
  G->pair_edge.ensure(G->pair_cap * 4);
  G->pair_len.ensure(G->pair_cap * 4);
  G->pair_merge.ensure(G->pair_cap * 4);
  G->pair_hlen.ensure(G->pair_cap * 4);
  G->pair_hoff.ensure((G->pair_cap + 1) * 8);
  G->k4_s.ensure(K4_HS_CAP * 4);
  G->k4_edge.ensure(K4_HE_CAP * 3 * 8);
  G->k4_item.ensure(K4_IT_CAP * 2 * 4);
  // touched rows: at most both ends of every change
  G->tv_items.ensure(2 * (G->ce.cap / 8) * 4);
  G->tv_ioff.ensure((2 * (G->ce.cap / 8) + 1) * 8);
  G->pair_off.ensure((G->pair_cap + 1) * 8);
  G->scan_tmp.ensure(scan_tmp_bytes(std::max<int64_t>(2 * (G->ce.cap / 8), G->pair_cap) + 1) + 64);
  G->ae_cap = std::max<int64_t>(G->ae_cap, std::max<int64_t>(ae_need, 8 * cap_t + 4096));
  G->ae.ensure(G->ae_cap * 8);
  G->ae_alt.ensure(G->ae_cap * 8);
  G->sort_tmp.ensure(radix_sort_tmp_bytes(G->ae_cap) + 64);
  G->slot_cap = std::max<int64_t>(G->slot_cap, std::max<int64_t>(slot_need, 4096));
  G->slot_list.ensure((size_t)std::max(1, G->c4_slots) * G->slot_cap * 4);
}

// After an edge-local pass whose affected-edge list or common-neighbour slot
// was too small (the combine and the purge then changed nothing): grow them
// from the sizes the kernels asked for and run the stage again.
int settle_delta(gc_graph* G, const PassPlan& L, BatchWork& W);

// Expected wall ms of the two kinds of one-batch pass (< 0: no estimate):
// region, this bucket's mean, else the mean of all region passes (its cost
// hardly depends on the batch); edge-local, affine in the batch size: the
// fixed cost F (the fastest edge-local pass seen) plus a per-update cost
// fitted to this bucket's mean, else the nearest measured bucket's,
// (ms - F) / size.  A half-decade spans sizes 3.2x apart and the edge-local
// work grows with the changed pairs, so even the own bucket's mean is scaled
// to the batch; and scaling a small bucket's time in proportion would
// charge the large batch its fixed cost many times over.
void pass_estimates(const gc_graph* G, int b, int64_t total, double& est_r, double& est_d) {
  const int64_t* n = G->mode_n[b];
  est_r = n[0] > 0 ? G->mode_ms[b][0] : (G->region_n_all > 0 ? G->region_ms_all : -1.0);
  est_d = -1;
  int nb = n[1] > 0 ? b : -1;
  for (int k = 1; k < 16 && nb < 0; ++k)
    for (int bb : {b - k, b + k})
      if (bb >= 0 && bb < 16 && G->mode_n[bb][1] > 0 && nb < 0) nb = bb;
  if (nb < 0) return;
  const double ms = G->mode_ms[nb][1];
  const double F = G->delta_ms_min >= 0 ? std::min(G->delta_ms_min, ms) : ms;
  est_d = F + (ms - F) * (double)std::max<int64_t>(total, 1) / std::max(1.0, G->mode_sz[nb][1]);
}

int size_bucket(int64_t total) {
  return (int)std::min(15.0, std::floor(2.0 * std::log10((double)total + 1.0)));
}

// Edge-local or region pass for a batch of `total` updates in half-decade
// `b`: the kind with the smaller expected wall time (pass_estimates), else
// a first try edge-local for batches of at most 1000 updates (also while no
// region pass has been measured).  Both kinds measured in a bucket: every
// 32nd pass there tries the other.  A bucket with no edge-local pass yet
// tries one while the carried-over estimate is within 1.25x of the region's
// (a per-update cost taken from other sizes is rough).
bool choose_delta(gc_graph* G, int b, int64_t total) {
  const int64_t* n = G->mode_n[b];
  // nothing measured for the region kind yet: small batches start edge-local
  if (G->region_n_all == 0) return total <= 1000;
  double est_r, est_d;
  pass_estimates(G, b, total, est_r, est_d);
  if (est_d < 0) return total <= 1000;
  if (n[0] > 0 && n[1] > 0) {
    const bool d = est_d < est_r;
    return (n[0] + n[1]) % 32 == 31 ? !d : d;
  }
  if (n[1] == 0) return est_d < 1.25 * est_r;
  return est_d < est_r;
}

// Whether q queued batches of one graph (gc_apply_batch_seq, the server)
// should share one multi-version pass rather than run one by one (each then
// edge-local where that is faster): by the cost model, when autotuning with
// automatic pass kinds; always with edge-local passes off (or no autotune),
// never with them forced.
bool fold_batches(const gc_graph* G, const gc_batch_desc* b, int q) {
  if (q < 2) return false;
  if (G->opt.delta < 0 || !G->opt.autotune) return true;
  if (G->opt.delta > 0) return false;
  bool all_small = true;
  double one_by_one = 0;
  for (int j = 0; j < q; ++j) {
    const int64_t t = b[j].n_ins + b[j].n_del;
    all_small = all_small && t <= 1000;
    double er, ed;
    pass_estimates(G, size_bucket(t), t, er, ed);
    const double e = er >= 0 && ed >= 0 ? std::min(er, ed) : (er >= 0 ? er : ed);
    if (e < 0) return !all_small;  // nothing measured: small batches start edge-local
    one_by_one += e;
  }
  double multi = G->multi_n[q] > 0 ? G->multi_ms[q] : -1.0;
  if (multi < 0 && G->region_n_all > 0) multi = G->region_ms_all * (1.0 + 0.25 * (q - 1));
  if (multi < 0) return !all_small;
  return multi < one_by_one;
}

// Every device step of a pass, in stream order: upload, ingest, merge,
// counting, purge, results to the pinned buffer.  No allocation and no
// synchronisation (except the device-array id check, which is never
// captured), so the same sequence runs directly or under stream capture.
void enqueue_pass(gc_graph* G, const PassPlan& L, BatchIn& B, BatchWork& W, const Staging& S, bool timed,
                  bool upload) {
  hipStream_t s = G->stream;
  PoolDev P = G->pd();
  unsigned long long* bst = G->bstats.as<unsigned long long>();
  unsigned long long* ctr = G->ctr.as<unsigned long long>();
  zero_small(G);
  if (upload) HIPCHK(hipMemcpyAsync(S.bin, G->pin, L.in_bytes, hipMemcpyHostToDevice, s));
  if (timed) HIPCHK(hipEventRecord(G->ev[0], s));
  launch_ingest_keys(P, B, G->bits, S.keys, ctr, bst, L.cap_t, s);
  unsigned long long* sk = radix_sort_u64(S.keys, S.keys_alt, G->sort_tmp.p, L.cap_t, ctr + C_NKEYS, 2 * G->bits + 3, s);
  launch_ingest_classify(P, sk, L.cap_t, G->bits, L.npass, L.nv, S.dirA, S.dirD, S.dirR, ctr, bst, s);
  if (L.dev) {
    unsigned long long err = 0;
    HIPCHK(hipMemcpyAsync(&err, bst + PB_IDX(0, PB_ERR), 8, hipMemcpyDeviceToHost, s));
    G->sync();
    if (err) raise(GC_EINVAL, "batch has %llu vertex ids outside the graph", err);
  }
  unsigned long long* sA = radix_sort_u64(S.dirA, S.dirA_alt, G->sort_tmp.p, 2 * L.cap_i, ctr + C_DIRA, 2 * G->bits, s);
  // a pass without deletions (insert-only batches, Alg. 1) has empty flag and
  // removal lists: their sorts, marks and flag kernels are skipped
  const bool ins_only = L.ndl == 0;
  unsigned long long* sD = ins_only ? W.dirD
                                    : radix_sort_u64(S.dirD, S.dirD_alt, G->sort_tmp.p, 2 * L.cap_d, ctr + C_DIRD,
                                                     2 * G->bits, s);
  unsigned long long* sR = ins_only ? W.dirR
                                    : radix_sort_u64(S.dirR, S.dirR_alt, G->sort_tmp.p, 2 * L.cap_d, ctr + C_DIRR,
                                                     2 * G->bits, s);
  if (sA != W.dirA || sD != W.dirD || sR != W.dirR) raise(GC_EDEVICE, "sorted merge lists not where expected");
  G->in_pass = true;  // from here on the resident graph holds the union view until the purge
  launch_mark_rows(sA, 2 * L.cap_i, ctr, C_DIRA, G->bits, W.a_beg, W.na, W.mark, W.touched, W.tix, s);
  if (!ins_only) {
    launch_mark_rows(sD, 2 * L.cap_d, ctr, C_DIRD, G->bits, nullptr, nullptr, W.mark, W.touched, W.tix, s);
    launch_mark_rows(sR, 2 * L.cap_d, ctr, C_DIRR, G->bits, W.r_beg, W.nr, W.mark, W.touched, W.tix, s);
  }
  launch_merge(P, W, L.max_touched, 2 * L.cap_i, G->bits, G->opt.slack, bst, G->scan_tmp.p, s);
  if (!ins_only) launch_flag_rows(P, W, 2 * L.cap_d, G->bits, bst, s);
  if (L.delta) {
    if (timed) HIPCHK(hipEventRecord(G->ev[1], s));
    launch_delta(make_delta_args(G, W), G->c4_slots, s);
    if (timed)
      for (int e = 2; e <= 7; ++e) HIPCHK(hipEventRecord(G->ev[e], s));
    launch_combine(2, G->sig.as<unsigned long long>(), G->state.as<long long>(), G->vout.as<long long>(), G->k, bst, s);
  } else {
    enqueue_count(G, L.nv, L.radius, G->state.as<long long>(), W, make_count_args(G, L.nv, L.dense_min, false), timed,
                  true);
  }
  enqueue_purge(G, W, L.max_touched, L.nv);
  if (timed) HIPCHK(hipEventRecord(G->ev[8], s));
  enqueue_readback(G, G->state.as<long long>());
}

int settle_delta(gc_graph* G, const PassPlan& L, BatchWork& W) {
  int attempts = 0;
  hipStream_t s = G->stream;
  while (G->out_bst()[BS_RETRY]) {
    if (++attempts > G->retry_limit)
      raise(GC_EDEVICE, "edge-local scratch still too small after %d more attempts", G->retry_limit);
    unsigned long long dc[DC_COUNT];
    HIPCHK(hipMemcpyAsync(dc, G->dctr.p, sizeof(dc), hipMemcpyDeviceToHost, s));
    G->sync();
    const double tot = (double)std::max<int64_t>(L.total, 1);
    G->ae_per_update = std::max(G->ae_per_update, (double)dc[DC_AFF_NEED] / tot);
    G->pair_per_update = std::max(G->pair_per_update, (double)dc[DC_PAIR_NEED] / tot);
    size_delta(G, L.cap_t, (int64_t)dc[DC_AFF_NEED] + (int64_t)dc[DC_AFF_NEED] / 4,
               (int64_t)dc[DC_SLOT_NEED] + (int64_t)dc[DC_SLOT_NEED] / 4,
               (int64_t)dc[DC_PAIR_NEED] + (int64_t)dc[DC_PAIR_NEED] / 4);
    reset_count_stage(G);
    launch_delta(make_delta_args(G, W), G->c4_slots, s);
    launch_combine(2, G->sig.as<unsigned long long>(), G->state.as<long long>(), G->vout.as<long long>(), G->k,
                   G->bstats.as<unsigned long long>(), s);
    enqueue_purge(G, W, L.max_touched, 2);
    enqueue_readback(G, G->state.as<long long>());
    G->sync();
  }
  return attempts;
}

// What an enqueued pass depends on: its sizes and knobs and every buffer
// address it reads or writes.  Equal signatures enqueue identical work.
std::vector<uint64_t> pass_signature(gc_graph* G, const PassPlan& L, const CountArgs& A) {
  std::vector<uint64_t> v = {(uint64_t)L.nseg, (uint64_t)L.seq, (uint64_t)L.npass, (uint64_t)L.nv,
                             (uint64_t)L.cap_i, (uint64_t)L.cap_d, (uint64_t)(int64_t)L.radius,
                             (uint64_t)A.c4_dense_min, (uint64_t)A.c4_win, (uint64_t)A.c4_narrow_max, (uint64_t)A.c4_ref,
                             (uint64_t)A.c4_maxlow, (uint64_t)A.slots, (uint64_t)A.tri_cap, (uint64_t)A.e_max,
                             (uint64_t)G->arena_cap, (uint64_t)L.in_bytes, (uint64_t)G->k, (uint64_t)G->N,
                             (uint64_t)G->bits, (uint64_t)L.delta, (uint64_t)G->ae_cap, (uint64_t)G->slot_cap,
                             (uint64_t)G->ce.cap, (uint64_t)G->pair_cap, (uint64_t)(L.ndl == 0),
                             (uint64_t)G->tiers_now[0], (uint64_t)G->tiers_now[1], (uint64_t)G->tiers_now[2]};
  const DevBuf* bufs[] = {&G->off, &G->len, &G->cap, &G->col, &G->top, &G->gid, &G->ext2int, &G->state, &G->vout,
                          &G->sig, &G->ctr, &G->bstats, &G->bin, &G->keys, &G->keys_alt, &G->dirA, &G->dirA_alt,
                          &G->dirD, &G->dirD_alt, &G->dirR, &G->dirR_alt, &G->a_beg, &G->na, &G->r_beg, &G->nr,
                          &G->mark, &G->tix, &G->touched, &G->dest, &G->newcap, &G->tlen, &G->tpre, &G->scratch,
                          &G->sort_tmp, &G->scan_tmp, &G->roff, &G->rcol, &G->rrow, &G->rlow, &G->dver, &G->t,
                          &G->tp, &G->vpos, &G->level, &G->rlist, &G->rlen, &G->lists, &G->c4_dense, &G->c4_touch,
                          &G->c4_cur, &G->c4_blk, &G->c4_keys, &G->c4_keys_alt, &G->tri_scratch, &G->Tv, &G->dTs,
                          &G->sbt, &G->ce, &G->ae, &G->ae_alt, &G->slot_list, &G->dctr, &G->c4_nch, &G->c4_side,
                          &G->c4_off, &G->pair_edge, &G->pair_len, &G->pair_off, &G->dead_d, &G->pair_merge, &G->pair_hlen, &G->pair_hoff, &G->k4_s, &G->k4_edge, &G->k4_item, &G->tv_items,
                          &G->tv_ioff};
  for (const DevBuf* b : bufs) v.push_back((uint64_t)(uintptr_t)b->p);
  v.push_back((uint64_t)(uintptr_t)G->pin);
  v.push_back((uint64_t)(uintptr_t)G->pout);
  return v;
}

// One counting pass.  seq == false: b[g] is the batch of graph g of the pool
// (G->k of them; host arrays unless dev, which needs k == 1).  seq == true:
// b[0..nb) are successive batches of graph 0 of a single-graph handle (host
// arrays, nb <= GC_SEQ_MAX); counts[j] and stats[j] are those after batch j.
// The pass compares nv versions: 2 for one batch per graph, 4 for several
// batches (versions past the last batch repeat it).  Untimed host-array
// passes replay a captured graph of the whole pass when one with the same
// signature exists (captured on first use).
void apply(gc_graph* G, const gc_batch_desc* b, int nb, bool dev, bool seq, int64_t (*counts)[11],
           gc_batch_stats* stats) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  if (G->broken) raise(GC_ESTATE, "handle unusable after an earlier device failure");
  HIPCHK(hipSetDevice(G->device));
  hipStream_t s = G->stream;
  const int k = G->k;
  PassPlan L;
  L.seq = seq;
  L.dev = dev;
  L.nseg = seq ? nb : k;         // segments of the update arrays
  L.npass = seq ? nb : 1;        // batches acting in sequence
  L.nv = L.npass > 1 ? 4 : 2;
  std::vector<int64_t> ins_seg(L.nseg + 1, 0), del_seg(L.nseg + 1, 0);
  for (int q = 0; q < L.nseg; ++q) {
    const int64_t n = G->gi[seq ? 0 : q];
    if (!dev) check_batch(b[q], n, q, G->any_dead ? G->dead_h.data() : nullptr);
    else if (b[q].n_ins < 0 || b[q].n_del < 0) raise(GC_EINVAL, "negative batch size");
    ins_seg[q + 1] = ins_seg[q] + b[q].n_ins;
    del_seg[q + 1] = del_seg[q] + b[q].n_del;
  }
  L.ni = ins_seg[L.nseg];
  L.ndl = del_seg[L.nseg];
  L.total = L.ni + L.ndl;
  L.cap_i = pow2_at_least(std::max<int64_t>(L.ni, 64));
  L.cap_d = pow2_at_least(std::max<int64_t>(L.ndl, 64));
  L.cap_t = L.cap_i + L.cap_d;
  L.max_touched = 2 * L.cap_t;
  L.union_bound = G->entries + 2 * L.ni;
  const bool timed = stats != nullptr;

  // speed knobs (results never depend on them)
  L.radius = G->opt.radius == 0 ? -1 : G->opt.radius;
  int tune_idx = -1, tier_idx = -1;
  const int decade = (int)std::min<double>(7.0, std::floor(std::log10((double)L.total + 1.0)));
  L.dense_min = G->dense_min_best;
  if (G->opt.autotune) {
    // whole-graph mode once a batch no larger than this one saw a region of
    // >= 90% of the entries (a larger batch's region covers at least as much
    // in expectation); exact radii only
    bool wide = false;
    for (int d = 0; d <= decade; ++d) wide = wide || G->region_frac[d] >= 0.9;
    if (L.radius >= 2 && wide) L.radius = -1;
  }
  // edge-local pass: one batch per graph and an exact radius; forced by the
  // option, or (autotune) the kind with the smaller expected time
  const int bucket = size_bucket(L.total);
  if (L.nv == 2 && G->opt.radius != 1) {
    if (G->opt.delta > 0) L.delta = true;
    else if (G->opt.delta == 0 && G->opt.autotune) L.delta = choose_delta(G, bucket, L.total);
  }
  // trials of the region count's knobs, each on a pass that counts a region
  // anyway: first the hub-window density thresholds, then the tier thresholds
  std::copy(G->tiers_best, G->tiers_best + 3, G->tiers_now);
  if (G->opt.autotune && !L.delta) {
    if (G->tune_next < (int)G->tune_cands.size()) {
      tune_idx = G->tune_next;
      L.dense_min = G->tune_cands[tune_idx];
    } else if (!G->tiers_forced && G->tier_next < (int)G->tier_cands.size()) {
      tier_idx = G->tier_next;
      std::copy(G->tier_cands[tier_idx].begin(), G->tier_cands[tier_idx].end(), G->tiers_now);
    }
  }
  const bool timed_run = timed || (G->opt.autotune && (tune_idx >= 0 || tier_idx >= 0));

  // buffers (all allocation happens here, before anything is enqueued)
  G->keys.ensure(L.cap_t * 8);
  G->keys_alt.ensure(L.cap_t * 8);
  for (DevBuf* d : {&G->dirA, &G->dirA_alt}) d->ensure(2 * L.cap_i * 8);
  for (DevBuf* d : {&G->dirD, &G->dirD_alt, &G->dirR, &G->dirR_alt}) d->ensure(2 * L.cap_d * 8);
  G->touched.ensure(L.max_touched * 4);
  G->dest.ensure(L.max_touched * 8);
  G->newcap.ensure(L.max_touched * 4);
  G->tlen.ensure(L.max_touched * 4);
  G->tpre.ensure((L.max_touched + 1) * 8);
  G->scratch.ensure(std::max<int64_t>(L.union_bound, 1) * 4);
  G->sort_tmp.ensure(radix_sort_tmp_bytes(std::max<int64_t>(std::max(L.cap_t, 2 * std::max(L.cap_i, L.cap_d)), G->N)) +
                     64);
  G->scan_tmp.ensure(scan_tmp_bytes(std::max<int64_t>(L.max_touched, G->N) + 1) + 64);
  size_count_scratch(G, L.nv, L.union_bound);
  if (L.delta) {
    // at the demand per update seen so far (within 2^26 entries a list: a
    // larger demand is met by the retry, which sizes for the batch at hand);
    // a common-neighbour slot holds the shorter row of a changed edge, at
    // most about the largest lower degree counted (ids follow the degree
    // order, so a hub's neighbours are nearly all below it)
    const double lim = (double)(1ll << 26);
    size_delta(G, L.cap_t, (int64_t)std::min(lim, 1.25 * G->ae_per_update * (double)L.cap_t),
               std::min<int64_t>(1ll << 26, G->seen_maxlow + G->seen_maxlow / 4 + 64),
               (int64_t)std::min(lim, 1.25 * G->pair_per_update * (double)L.cap_t));
  }
  // arena reserve: enough for every touched row to move
  const int64_t need = (int64_t)((1.0 + G->opt.slack) * (double)L.union_bound) + 8 * L.max_touched + 1024;
  if (G->arena_cap - G->arena_top < need) compact(G, need);

  // pinned input: [ins_seg | del_seg | gbase | gn] int64, then the id arrays
  // at capacity offsets (insertions u, v, deletions u, v)
  L.tab_words = (size_t)(2 * (L.nseg + 1) + 2 * k);
  L.in_bytes = L.tab_words * 8 + (dev ? 0 : (size_t)(2 * L.cap_t) * sizeof(int32_t));
  char* pin = (char*)G->pinned(L.in_bytes + 64);
  int64_t* tab = (int64_t*)pin;
  std::memcpy(tab, ins_seg.data(), (L.nseg + 1) * 8);
  std::memcpy(tab + L.nseg + 1, del_seg.data(), (L.nseg + 1) * 8);
  std::memcpy(tab + 2 * (L.nseg + 1), G->gbase.data(), k * 8);
  std::memcpy(tab + 2 * (L.nseg + 1) + k, G->gi.data(), k * 8);
  G->bin.ensure(L.in_bytes + 64);
  BatchIn B;
  B.n_ins = L.ni;
  B.n_del = L.ndl;
  B.k = L.nseg;
  B.seq = seq ? 1 : 0;
  char* dbase = (char*)G->bin.p;
  B.ins_seg = (const int64_t*)dbase;
  B.del_seg = B.ins_seg + L.nseg + 1;
  B.gbase = B.ins_seg + 2 * (L.nseg + 1);
  B.gn = B.gbase + k;
  B.dead = G->any_dead ? G->dead_d.as<uint8_t>() : nullptr;
  if (dev) {
    B.iu = b[0].ins_src; B.iv = b[0].ins_dst; B.du = b[0].del_src; B.dv = b[0].del_dst;
  } else {
    int32_t* ids = (int32_t*)(pin + L.tab_words * 8);
    int32_t* d_ids = (int32_t*)(dbase + L.tab_words * 8);
    int32_t *iu = ids, *iv = ids + L.cap_i, *du = ids + 2 * L.cap_i, *dv = ids + 2 * L.cap_i + L.cap_d;
    for (int q = 0; q < L.nseg; ++q) {
      if (b[q].n_ins) {
        std::memcpy(iu + ins_seg[q], b[q].ins_src, b[q].n_ins * 4);
        std::memcpy(iv + ins_seg[q], b[q].ins_dst, b[q].n_ins * 4);
      }
      if (b[q].n_del) {
        std::memcpy(du + del_seg[q], b[q].del_src, b[q].n_del * 4);
        std::memcpy(dv + del_seg[q], b[q].del_dst, b[q].n_del * 4);
      }
    }
    B.iu = d_ids; B.iv = d_ids + L.cap_i; B.du = d_ids + 2 * L.cap_i; B.dv = d_ids + 2 * L.cap_i + L.cap_d;
  }
  int retries = 0;
  G->pass_insert_only = L.ndl == 0;
  G->pass_max_dirA = 2 * L.cap_i;
  const Staging S = handle_staging(G);
  BatchWork W = make_work(G, S);
  W.dirA = radix_sort_result(S.dirA, S.dirA_alt, 2 * L.cap_i, 2 * G->bits);
  W.dirD = radix_sort_result(S.dirD, S.dirD_alt, 2 * L.cap_d, 2 * G->bits);
  W.dirR = radix_sort_result(S.dirR, S.dirR_alt, 2 * L.cap_d, 2 * G->bits);

  const bool use_graph = G->opt.graphs && !dev && !timed_run;
  // A failure once the merge may have run leaves the union view in the
  // resident graph: the handle is then marked unusable (GC_ESTATE).
  try {
  if (use_graph) {
    const std::vector<uint64_t> sig = pass_signature(G, L, make_count_args(G, L.nv, L.dense_min, false));
    auto it = G->graphs.find(sig);
    if (it == G->graphs.end()) {
      if (G->graphs.size() >= 32) G->drop_graphs();
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      hipGraph_t gr = nullptr;
      try {
        enqueue_pass(G, L, B, W, S, false, true);
      } catch (...) {
        (void)hipStreamEndCapture(s, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
      }
      HIPCHK(hipStreamEndCapture(s, &gr));
      hipGraphExec_t ex = nullptr;
      const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (e != hipSuccess) raise(GC_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
      it = G->graphs.emplace(sig, ex).first;
      ++G->graph_captures;
    }
    G->in_pass = true;
    HIPCHK(hipGraphLaunch(it->second, s));
    ++G->graph_launches;
  } else {
    enqueue_pass(G, L, B, W, S, timed_run, true);
  }
  G->sync();
  if (L.delta) retries += settle_delta(G, L, W);
  retries += settle_retries(G, L.nv, L.radius, G->state.as<long long>(), W, L.dense_min, L.union_bound, true,
                            L.max_touched, false, true);
  } catch (...) {
    if (G->in_pass) G->broken = true;
    G->in_pass = false;
    throw;
  }
  G->in_pass = false;

  const unsigned long long* hbp = G->out_bst();
  const std::vector<unsigned long long> hb(hbp, hbp + BS_COUNT);
  const std::vector<unsigned long long> hc(G->out_ctr(), G->out_ctr() + C_COUNT);
  G->arena_top = (int64_t)*G->out_top();
  std::vector<long long> st(G->out_state(), G->out_state() + (size_t)k * ST_STRIDE);
  std::vector<long long> vo(G->out_vout(), G->out_vout() + (size_t)(L.nv - 1) * k * ST_STRIDE);
  long long cerr = 0;
  for (int g = 0; g < k; ++g) cerr += st[g * ST_STRIDE + ST_ERR];
  if (hb[BS_ARENA_OVF] || hb[BS_ERR] || cerr) {
    G->broken = true;
    raise(GC_EDEVICE, "device-side inconsistency (arena overflow %llu, errors %llu, inexact totals %lld)",
          hb[BS_ARENA_OVF], hb[BS_ERR], cerr);
  }
  for (int g = 0; g < k; ++g) st[g * ST_STRIDE + ST_N] = G->gl[g];
  G->hstate = st;
  for (int j = 0; j < L.npass; ++j)
    G->entries += 2 * ((int64_t)hb[PB_IDX(j, PB_EFF_INS)] - (int64_t)hb[PB_IDX(j, PB_EFF_DEL)]);
  // results: per graph of the pool, or per batch of the sequence
  const int nout = seq ? nb : k;
  std::vector<uint32_t> ovf(nout, 0);
  for (int o = 0; o < nout; ++o) {
    long long* so = seq ? &vo[(size_t)o * ST_STRIDE] : &G->hstate[(size_t)o * ST_STRIDE];
    so[ST_N] = G->gl[seq ? 0 : o];
    i128 I[11];
    finalize(so, G->gl[seq ? 0 : o], I);
    int64_t tmp[11];
    to_int64(I, counts ? counts[o] : tmp, &ovf[o]);
  }
  if (G->opt.autotune) {
    if (L.radius > 0 && L.union_bound > 0)
      G->region_frac[decade] = (double)hc[C_ER] / (double)std::max<int64_t>(1, G->entries);
    if (tune_idx >= 0 && retries == 0) {
      float c4ms = 0;
      (void)hipEventElapsedTime(&c4ms, G->ev[6], G->ev[7]);
      G->tune_ms.push_back(c4ms);
      G->tune_wedges.push_back((double)hb[BS_WEDGES] + 1.0);
      ++G->tune_next;
      if (G->tune_next == (int)G->tune_cands.size()) {
        int best = 0;
        for (int i = 1; i < (int)G->tune_ms.size(); ++i)
          if (G->tune_ms[i] / G->tune_wedges[i] < G->tune_ms[best] / G->tune_wedges[best]) best = i;
        G->dense_min_best = G->tune_cands[best];
      }
    }
    if (tier_idx >= 0 && retries == 0) {
      float tri_ms = 0, c4_ms = 0;
      (void)hipEventElapsedTime(&tri_ms, G->ev[2], G->ev[3]);
      (void)hipEventElapsedTime(&c4_ms, G->ev[4], G->ev[7]);
      G->tier_tri_cost.push_back(tri_ms / ((double)hb[BS_TRI_E] + 1.0));
      G->tier_c4_cost.push_back(c4_ms / ((double)hb[BS_WEDGES] + 1.0));
      ++G->tier_next;
      if (G->tier_next == (int)G->tier_cands.size()) {
        // the triangle threshold from the trials that differ in it only,
        // the 4-cycle pair from the others
        int bt = 0, bc = 0;
        for (int i = 1; i < (int)G->tier_cands.size(); ++i) {
          const auto& c = G->tier_cands[i];
          const bool tri_only = c[1] == G->tier_cands[0][1] && c[2] == G->tier_cands[0][2];
          if (tri_only && G->tier_tri_cost[i] < G->tier_tri_cost[bt]) bt = i;
          if (!tri_only && G->tier_c4_cost[i] < G->tier_c4_cost[bc]) bc = i;
        }
        G->tiers_best[0] = G->tier_cands[bt][0];
        G->tiers_best[1] = G->tier_cands[bc][1];
        G->tiers_best[2] = G->tier_cands[bc][2];
      }
    }
  }
  const int32_t tiers_used[3] = {G->tiers_now[0], G->tiers_now[1], G->tiers_now[2]};
  std::copy(G->tiers_best, G->tiers_best + 3, G->tiers_now);
  const double ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  if (L.nv == 4 && retries == 0 && L.npass < GC_NV_MAX) {
    double& avg = G->multi_ms[L.npass];
    avg = G->multi_n[L.npass] == 0 ? ms : 0.75 * avg + 0.25 * ms;
    ++G->multi_n[L.npass];
  }
  if (L.nv == 2 && retries == 0) {
    const int m = L.delta ? 1 : 0;
    int64_t& cnt = G->mode_n[bucket][m];
    double& avg = G->mode_ms[bucket][m];
    double& sz = G->mode_sz[bucket][m];
    avg = cnt == 0 ? ms : 0.75 * avg + 0.25 * ms;
    sz = cnt == 0 ? (double)L.total : 0.75 * sz + 0.25 * (double)L.total;
    ++cnt;
    if (L.delta) G->delta_ms_min = G->delta_ms_min < 0 ? ms : std::min(G->delta_ms_min, ms);
    if (!L.delta) {
      G->region_ms_all = G->region_n_all == 0 ? ms : 0.75 * G->region_ms_all + 0.25 * ms;
      ++G->region_n_all;
    }
  }
  if (stats) {
    const int nst = seq ? nb : 1;
    for (int q = 0; q < nst; ++q) {
      uint32_t mk = 0;
      if (seq) mk = ovf[q];
      else for (uint32_t m : ovf) mk |= m;
      fill_stats(G, &stats[q], hb.data(), hc.data(), seq ? q : 0, L.npass, seq ? b[q].n_ins : L.ni, seq ? b[q].n_del : L.ndl,
                 timed && retries == 0, ms, mk);
      stats[q].c4_dense_min = L.dense_min;
      stats[q].whole_graph = L.radius < 0 && !L.delta;
      stats[q].retries = retries;
      stats[q].delta = L.delta;
      stats[q].tri_small_max = tiers_used[0];
      stats[q].c4_small_max = tiers_used[1];
      stats[q].c4_mid_max = tiers_used[2];
    }
  }
}

// Carves the batch staging of a one-batch device-array pass with batch
// capacities cap_i, cap_d out of `base` (nullptr: sizes only); returns the
// bytes used.
size_t carve_staging(char* base, int64_t cap_i, int64_t cap_d, size_t table_bytes, Staging* S) {
  const int64_t cap_t = cap_i + cap_d, mt = 2 * cap_t;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return (void*)p;
  };
  S->bin = take(table_bytes);
  S->keys = (unsigned long long*)take(cap_t * 8);
  S->keys_alt = (unsigned long long*)take(cap_t * 8);
  S->dirA = (unsigned long long*)take(2 * cap_i * 8);
  S->dirA_alt = (unsigned long long*)take(2 * cap_i * 8);
  S->dirD = (unsigned long long*)take(2 * cap_d * 8);
  S->dirD_alt = (unsigned long long*)take(2 * cap_d * 8);
  S->dirR = (unsigned long long*)take(2 * cap_d * 8);
  S->dirR_alt = (unsigned long long*)take(2 * cap_d * 8);
  S->touched = (int32_t*)take(mt * 4);
  S->dest = (int64_t*)take(mt * 8);
  S->newcap = (int32_t*)take(mt * 4);
  S->tlen = (int32_t*)take(mt * 4);
  S->tpre = (int64_t*)take((mt + 1) * 8);
  return off;
}

struct Table6 {
  int64_t v[6];
};
__global__ void k_put_table(int64_t* dst, Table6 t) {
  if (threadIdx.x < 6) dst[threadIdx.x] = t.v[threadIdx.x];
}

// One batch given as device arrays, applied with no allocation: the batch
// staging comes from the static array, every other buffer is the handle's
// and must already be large enough (checked before anything is enqueued).
// A pass whose counting asks for more scratch is undone (the purge removes
// the new entries and clears the flags) and the call fails with the graph
// unchanged.  Host side: no heap allocation either (fixed-size arrays only).
void apply_noalloc(gc_graph* G, const int32_t* iu, const int32_t* iv, int64_t n_ins, const int32_t* du,
                   const int32_t* dv, int64_t n_del, int64_t counts[11], gc_batch_stats* stats) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  if (G->broken) raise(GC_ESTATE, "handle unusable after an earlier device failure");
  if (G->k != 1) raise(GC_EINVAL, "handle holds %d graphs", G->k);
  if (n_ins < 0 || n_del < 0) raise(GC_EINVAL, "negative batch size");
  if ((n_ins && (!iu || !iv)) || (n_del && (!du || !dv))) raise(GC_EINVAL, "null batch array");
  HIPCHK(hipSetDevice(G->device));
  char* base = (char*)noalloc_scratch_ptr(G->device);
  if (!base) raise(GC_EDEVICE, "static staging of device %d not set up", G->device);
  hipStream_t s = G->stream;
  PassPlan L;
  L.dev = true;
  L.ni = n_ins;
  L.ndl = n_del;
  L.total = n_ins + n_del;
  L.cap_i = pow2_at_least(std::max<int64_t>(L.ni, 64));
  L.cap_d = pow2_at_least(std::max<int64_t>(L.ndl, 64));
  L.cap_t = L.cap_i + L.cap_d;
  L.max_touched = 2 * L.cap_t;
  L.union_bound = G->entries + 2 * L.ni;
  L.tab_words = 6;
  L.in_bytes = L.tab_words * 8;
  Staging S;
  const size_t need_bytes = carve_staging(nullptr, L.cap_i, L.cap_d, L.in_bytes, &S);
  if (need_bytes > kNoAllocBytes)
    raise(GC_EINVAL,
          "batch of %lld insertions and %lld deletions needs %zu bytes of staging; the allocation-free entry point "
          "has %zu (every batch of at most 262144 insertions and 262144 deletions fits)",
          (long long)n_ins, (long long)n_del, need_bytes, kNoAllocBytes);
  // speed knobs as apply() chooses them, without autotuning trials
  L.radius = G->opt.radius == 0 ? -1 : G->opt.radius;
  const int decade = (int)std::min<double>(7.0, std::floor(std::log10((double)L.total + 1.0)));
  L.dense_min = G->dense_min_best;
  if (G->opt.autotune) {
    bool wide = false;
    for (int d = 0; d <= decade; ++d) wide = wide || G->region_frac[d] >= 0.9;
    if (L.radius >= 2 && wide) L.radius = -1;
  }
  // every buffer the pass uses besides the staging must already fit
  const size_t sort_need = radix_sort_tmp_bytes(std::max<int64_t>(std::max(L.cap_t, 2 * std::max(L.cap_i, L.cap_d)), G->N)) + 64;
  const size_t scan_need = scan_tmp_bytes(std::max<int64_t>(L.max_touched, G->N) + 1) + 64;
  const int64_t arena_need = (int64_t)((1.0 + G->opt.slack) * (double)L.union_bound) + 8 * L.max_touched + 1024;
  const char* short_of = G->sort_tmp.cap < sort_need                                          ? "sort temporaries"
                         : G->scan_tmp.cap < scan_need                                        ? "scan temporaries"
                         : G->scratch.cap < (size_t)std::max<int64_t>(L.union_bound, 4) * 4 ? "merge scratch"
                         : count_scratch_short(G, 2, L.union_bound)                           ? count_scratch_short(G, 2, L.union_bound)
                         : G->arena_cap - G->arena_top < arena_need                           ? "resident rows"
                                                                                              : nullptr;
  if (short_of)
    raise(GC_ENOMEM,
          "the handle's buffers (%s) are not sized for this batch (graph of %lld entries plus %lld insertions); "
          "one gc_apply_batch_dev call of this size grows them",
          short_of, (long long)G->entries, (long long)n_ins);

  // the input table (segment bounds, graph base and size) by a kernel: no host staging
  carve_staging(base, L.cap_i, L.cap_d, L.in_bytes, &S);
  Table6 tb = {{0, n_ins, 0, n_del, G->gbase[0], G->gi[0]}};
  hipLaunchKernelGGL(k_put_table, dim3(1), dim3(64), 0, s, (int64_t*)S.bin, tb);
  BatchIn B;
  B.n_ins = n_ins;
  B.n_del = n_del;
  B.k = 1;
  B.seq = 0;
  B.ins_seg = (const int64_t*)S.bin;
  B.del_seg = B.ins_seg + 2;
  B.gbase = B.ins_seg + 4;
  B.gn = B.ins_seg + 5;
  B.dead = G->any_dead ? G->dead_d.as<uint8_t>() : nullptr;
  B.iu = iu; B.iv = iv; B.du = du; B.dv = dv;
  BatchWork W = make_work(G, S);
  W.dirA = radix_sort_result(S.dirA, S.dirA_alt, 2 * L.cap_i, 2 * G->bits);
  W.dirD = radix_sort_result(S.dirD, S.dirD_alt, 2 * L.cap_d, 2 * G->bits);
  W.dirR = radix_sort_result(S.dirR, S.dirR_alt, 2 * L.cap_d, 2 * G->bits);
  G->pass_insert_only = L.ndl == 0;
  G->pass_max_dirA = 2 * L.cap_i;
  const bool timed = stats != nullptr;
  try {
    enqueue_pass(G, L, B, W, S, timed, false);
    G->sync();
    if (G->out_bst()[BS_RETRY]) {
      // counting needs more scratch: undo the merge, keep the graph as it was
      unsigned long long* bst = G->bstats.as<unsigned long long>();
      fill_u64(bst + BS_RETRY, 0ull, 1, s);
      launch_purge(G->pd(), W, L.max_touched, G->bits, 0u, bst + BS_RETRY, G->scan_tmp.p, s, true);
      G->sync();
      G->arena_top = (int64_t)*G->out_top();
      G->in_pass = false;
      note_maxima(G);
      raise(GC_ENOMEM,
            "a vertex outgrew the counting scratch; the batch was undone and the graph is unchanged "
            "(one gc_apply_batch_dev call grows the scratch)");
    }
  } catch (...) {
    if (G->in_pass) G->broken = true;
    G->in_pass = false;
    throw;
  }
  G->in_pass = false;
  note_maxima(G);
  const unsigned long long* hb = G->out_bst();
  const unsigned long long* hc = G->out_ctr();
  G->arena_top = (int64_t)*G->out_top();
  const long long* st = G->out_state();
  if (hb[BS_ARENA_OVF] || hb[BS_ERR] || st[ST_ERR]) {
    G->broken = true;
    raise(GC_EDEVICE, "device-side inconsistency (arena overflow %llu, errors %llu, inexact totals %lld)",
          hb[BS_ARENA_OVF], hb[BS_ERR], st[ST_ERR]);
  }
  std::memcpy(G->hstate.data(), st, ST_STRIDE * sizeof(long long));
  G->hstate[ST_N] = G->gl[0];
  G->entries += 2 * ((int64_t)hb[PB_IDX(0, PB_EFF_INS)] - (int64_t)hb[PB_IDX(0, PB_EFF_DEL)]);
  i128 I[11];
  finalize(G->hstate.data(), G->gl[0], I);
  int64_t tmp[11];
  uint32_t ovf = 0;
  to_int64(I, counts ? counts : tmp, &ovf);
  if (G->opt.autotune && L.radius > 0 && L.union_bound > 0)
    G->region_frac[decade] = (double)hc[C_ER] / (double)std::max<int64_t>(1, G->entries);
  if (stats) {
    const double ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
    fill_stats(G, stats, hb, hc, 0, 1, n_ins, n_del, true, ms, ovf);
    stats->c4_dense_min = L.dense_min;
    stats->whole_graph = L.radius < 0;
    stats->retries = 0;
  }
}

// Edges of graph `graph`, each once, external ids, into host arrays of
// capacity capn; returns the edge count.
int64_t export_edges(gc_graph* g, int32_t graph, int32_t* src, int32_t* dst, int64_t capn) {
  HIPCHK(hipSetDevice(g->device));
  const int64_t m = g->hstate[graph * ST_STRIDE + ST_M];
  if (capn < m) raise(GC_EINVAL, "capacity %lld below the edge count %lld", (long long)capn, (long long)m);
  if (m > 0 && (!src || !dst)) raise(GC_EINVAL, "NULL output arrays");
  hipStream_t s = g->stream;
  const int64_t N = g->N;
  DevBuf cnt, pre, es, ed, gb;
  cnt.ensure(N * 4);
  pre.ensure((N + 1) * 8);
  const int64_t total = g->entries / 2;
  es.ensure(std::max<int64_t>(total, 1) * 4);
  ed.ensure(std::max<int64_t>(total, 1) * 4);
  gb.ensure(g->k * 8);
  HIPCHK(hipMemcpyAsync(gb.p, g->gbase.data(), g->k * 8, hipMemcpyHostToDevice, s));
  PoolDev P = g->pd();
  launch_upper_count(P, cnt.as<int32_t>(), s);
  g->scan_tmp.ensure(scan_tmp_bytes(N + 1) + 64);
  exclusive_scan_i32_to_i64(cnt.as<int32_t>(), pre.as<int64_t>(), N, g->scan_tmp.p, s);
  launch_export(P, g->int2ext.as<int32_t>(), gb.as<int64_t>(), pre.as<int64_t>(), es.as<int32_t>(),
                ed.as<int32_t>(), s);
  int64_t range[2];
  HIPCHK(hipMemcpyAsync(&range[0], pre.as<int64_t>() + g->gbase[graph], 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&range[1], pre.as<int64_t>() + g->gbase[graph] + g->gn[graph], 8, hipMemcpyDeviceToHost, s));
  g->sync();
  if (range[1] - range[0] != m) raise(GC_EDEVICE, "edge count mismatch (%lld vs %lld)",
                                      (long long)(range[1] - range[0]), (long long)m);
  if (m) {
    HIPCHK(hipMemcpyAsync(src, es.as<int32_t>() + range[0], m * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(dst, ed.as<int32_t>() + range[0], m * 4, hipMemcpyDeviceToHost, s));
  }
  g->sync();
  return m;
}

// Removed vertices on the device: a byte per id of the internal id space,
// allocated and cleared on the first removal.
void mark_dead(gc_graph* G, const int32_t* ids_dev, const std::vector<int32_t>& ids) {
  hipStream_t s = G->stream;
  if (!G->any_dead) {
    G->dead_h.assign(G->N, 0);
    G->dead_d.ensure(G->N);
    HIPCHK(hipMemsetAsync(G->dead_d.p, 0, G->N, s));
  }
  for (int32_t x : ids) G->dead_h[x] = 1;
  launch_set_bytes(G->dead_d.as<uint8_t>(), ids_dev, (int64_t)ids.size(), 1, s);
  G->sync();
  G->any_dead = true;
}

// A larger id space for a single graph: its edges are read back and the
// graph is built again over cap ids.  External ids, counts and removed
// vertices are kept; captured passes are dropped (their buffers change).
void regrow_ids(gc_graph* G, int64_t cap) {
  if (cap >= GC_MAX_VERTICES) raise(GC_EINVAL, "vertex ids must stay below 2^28");
  const int64_t m = G->hstate[ST_M];
  std::vector<int32_t> src(std::max<int64_t>(m, 1)), dst(std::max<int64_t>(m, 1));
  export_edges(G, 0, src.data(), dst.data(), m);
  const int64_t gi = G->gi[0], gl = G->gl[0];
  G->sync();
  G->drop_graphs();
  try {
    const int32_t* ps = src.data();
    const int32_t* pd = dst.data();
    build(G, 1, &cap, &ps, &pd, &m);
    G->gi[0] = gi;
    G->gl[0] = gl;
    G->hstate[ST_N] = gl;
    if (G->any_dead) {
      G->dead_h.resize(cap, 0);
      G->dead_d.ensure(cap);
      HIPCHK(hipMemcpyAsync(G->dead_d.p, G->dead_h.data(), cap, hipMemcpyHostToDevice, G->stream));
      G->sync();
    }
  } catch (...) {
    G->broken = true;
    throw;
  }
}

void counts_now(gc_graph* G, int64_t counts[11]) {
  if (!counts) return;
  i128 I[11];
  finalize(G->hstate.data(), G->gl[0], I);
  to_int64(I, counts, nullptr);
}

void add_vertices(gc_graph* G, int64_t count, int64_t* first_id) {
  if (G->broken) raise(GC_ESTATE, "handle unusable after an earlier device failure");
  if (G->k != 1) raise(GC_EINVAL, "handle holds %d graphs: vertices are added to single-graph handles", G->k);
  if (count < 0) raise(GC_EINVAL, "negative vertex count");
  HIPCHK(hipSetDevice(G->device));
  const int64_t need = G->gi[0] + count;
  if (need >= GC_MAX_VERTICES) raise(GC_EINVAL, "vertex ids must stay below 2^28");
  if (need > G->gn[0]) regrow_ids(G, std::min<int64_t>(GC_MAX_VERTICES - 1, std::max(need, 2 * G->gn[0])));
  if (first_id) *first_id = G->gi[0];
  G->gi[0] = need;
  G->gl[0] += count;
  G->hstate[ST_N] = G->gl[0];
}

// Deletes every edge at the given vertices in one batch (through the
// ordinary batch path: counts, statistics and failure rules of a batch),
// then takes them out of V.
void remove_vertices(gc_graph* G, const int32_t* ids, int64_t count, int64_t counts[11], gc_batch_stats* stats) {
  if (G->broken) raise(GC_ESTATE, "handle unusable after an earlier device failure");
  if (G->k != 1) raise(GC_EINVAL, "handle holds %d graphs: vertices are removed from single-graph handles", G->k);
  if (count < 0 || (count > 0 && !ids)) raise(GC_EINVAL, "bad vertex list");
  std::vector<int32_t> v(ids, ids + count);
  std::sort(v.begin(), v.end());
  for (int64_t i = 0; i < count; ++i) {
    if (v[i] < 0 || v[i] >= G->gi[0]) raise(GC_EINVAL, "vertex id %d outside [0, %lld)", v[i], (long long)G->gi[0]);
    if (G->any_dead && G->dead_h[v[i]]) raise(GC_EINVAL, "vertex %d was removed already", v[i]);
    if (i && v[i] == v[i - 1]) raise(GC_EINVAL, "vertex %d listed twice", v[i]);
  }
  HIPCHK(hipSetDevice(G->device));
  hipStream_t s = G->stream;
  // the incident edges, read from the resident rows
  DevBuf did, dlen, dpre, du, dv;
  std::vector<int32_t> len(std::max<int64_t>(count, 1));
  std::vector<int64_t> pre(count + 1, 0);
  did.ensure(std::max<int64_t>(count, 1) * 4);
  dlen.ensure(std::max<int64_t>(count, 1) * 4);
  if (count) HIPCHK(hipMemcpyAsync(did.p, v.data(), count * 4, hipMemcpyHostToDevice, s));
  launch_row_len(G->pd(), did.as<int32_t>(), count, dlen.as<int32_t>(), s);
  if (count) HIPCHK(hipMemcpyAsync(len.data(), dlen.p, count * 4, hipMemcpyDeviceToHost, s));
  G->sync();
  for (int64_t i = 0; i < count; ++i) pre[i + 1] = pre[i] + len[i];
  const int64_t e = pre[count];
  std::vector<int32_t> eu(std::max<int64_t>(e, 1)), ev(std::max<int64_t>(e, 1));
  if (e) {
    dpre.ensure((count + 1) * 8);
    du.ensure(e * 4);
    dv.ensure(e * 4);
    HIPCHK(hipMemcpyAsync(dpre.p, pre.data(), (count + 1) * 8, hipMemcpyHostToDevice, s));
    launch_row_gather(G->pd(), G->int2ext.as<int32_t>(), did.as<int32_t>(), count, dpre.as<int64_t>(),
                      du.as<int32_t>(), dv.as<int32_t>(), s);
    HIPCHK(hipMemcpyAsync(eu.data(), du.p, e * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(ev.data(), dv.p, e * 4, hipMemcpyDeviceToHost, s));
    G->sync();
  }
  // an edge between two removed vertices is listed from both ends: the
  // batch rules drop the repeat
  gc_batch_desc b{nullptr, nullptr, 0, eu.data(), ev.data(), e};
  apply(G, &b, 1, false, false, nullptr, stats);
  if (count) mark_dead(G, did.as<int32_t>(), v);
  G->gl[0] -= count;
  G->hstate[ST_N] = G->gl[0];
  counts_now(G, counts);
  if (stats) {
    // the batch's int64 overflow flags, now for the smaller vertex set
    i128 I[11];
    finalize(G->hstate.data(), G->gl[0], I);
    int64_t tmp[11];
    to_int64(I, tmp, &stats->overflow_mask);
  }
}

template <class F>
int guard(F f) {
  try {
    f();
    return GC_OK;
  } catch (const GcError& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return GC_ENOMEM;
  } catch (...) {
    g_err = "unexpected exception";
    return GC_EDEVICE;
  }
}

}  // namespace

extern "C" {

int gc_options_default(gc_options* opt) {
  if (!opt) return GC_EINVAL;
  opt->radius = 2;
  opt->slack = 0.25f;
  opt->device = 0;
  opt->stream = nullptr;
  opt->autotune = 1;
  opt->graphs = 1;
  opt->delta = 0;
  opt->vertex_capacity = 0;
  opt->tri_small_max = 0;
  opt->c4_small_max = 0;
  opt->c4_mid_max = 0;
  return GC_OK;
}

int gc_pool_init(int32_t k, const int64_t* n, const int32_t* const* src, const int32_t* const* dst, const int64_t* m,
                 const gc_options* opt, gc_graph** out, int64_t (*counts)[11]) {
  return guard([&] {
    if (!out) raise(GC_EINVAL, "out is NULL");
    *out = nullptr;
    if (k < 1 || !n || !m) raise(GC_EINVAL, "need k >= 1 graphs with sizes");
    gc_graph* G = new gc_graph();
    try {
      setup_handle(G, opt);
      // a single graph may reserve ids for vertices added later
      std::vector<int64_t> ncap(n, n + k);
      if (k == 1 && G->opt.vertex_capacity > n[0]) {
        for (int64_t i = 0; i < m[0]; ++i)
          if (src[0][i] < 0 || src[0][i] >= n[0] || dst[0][i] < 0 || dst[0][i] >= n[0])
            raise(GC_EINVAL, "edge %lld has a vertex id outside [0, %lld)", (long long)i, (long long)n[0]);
        ncap[0] = G->opt.vertex_capacity;
      }
      build(G, k, ncap.data(), src, dst, m);
      for (int g = 0; g < k; ++g) {
        G->gi[g] = G->gl[g] = n[g];
        G->hstate[g * ST_STRIDE + ST_N] = n[g];
      }
    } catch (...) {
      delete G;
      throw;
    }
    if (counts)
      for (int g = 0; g < k; ++g) {
        i128 I[11];
        finalize(&G->hstate[g * ST_STRIDE], G->gl[g], I);
        to_int64(I, counts[g], nullptr);
      }
    *out = G;
  });
}

int gc_graph_init(int64_t n, const int32_t* src, const int32_t* dst, int64_t m, const gc_options* opt, gc_graph** out,
                  int64_t counts[11]) {
  const int32_t* s[1] = {src};
  const int32_t* d[1] = {dst};
  return gc_pool_init(1, &n, s, d, &m, opt, out, counts ? (int64_t(*)[11])counts : nullptr);
}

int gc_apply_batch(gc_graph* g, const int32_t* ins_src, const int32_t* ins_dst, int64_t n_ins, const int32_t* del_src,
                   const int32_t* del_dst, int64_t n_del, int64_t counts[11], gc_batch_stats* stats) {
  return guard([&] {
    if (!g) raise(GC_EINVAL, "graph is NULL");
    if (g->k != 1) raise(GC_EINVAL, "handle holds %d graphs: use gc_apply_batches", g->k);
    gc_batch_desc b{ins_src, ins_dst, n_ins, del_src, del_dst, n_del};
    apply(g, &b, 1, false, false, counts ? (int64_t(*)[11])counts : nullptr, stats);
  });
}

int gc_apply_batch_dev(gc_graph* g, const int32_t* ins_src, const int32_t* ins_dst, int64_t n_ins,
                       const int32_t* del_src, const int32_t* del_dst, int64_t n_del, int64_t counts[11],
                       gc_batch_stats* stats) {
  return guard([&] {
    if (!g) raise(GC_EINVAL, "graph is NULL");
    if (g->k != 1) raise(GC_EINVAL, "handle holds %d graphs: use gc_apply_batches", g->k);
    gc_batch_desc b{ins_src, ins_dst, n_ins, del_src, del_dst, n_del};
    apply(g, &b, 1, true, false, counts ? (int64_t(*)[11])counts : nullptr, stats);
  });
}

int gc_apply_batch_dev_noalloc(gc_graph* g, const int32_t* ins_src, const int32_t* ins_dst, int64_t n_ins,
                               const int32_t* del_src, const int32_t* del_dst, int64_t n_del, int64_t counts[11],
                               gc_batch_stats* stats) {
  return guard([&] {
    if (!g) raise(GC_EINVAL, "graph is NULL");
    apply_noalloc(g, ins_src, ins_dst, n_ins, del_src, del_dst, n_del, counts, stats);
  });
}

int gc_apply_batches(gc_graph* pool, const gc_batch_desc* batch, int64_t (*counts)[11], gc_batch_stats* stats) {
  return guard([&] {
    if (!pool || !batch) raise(GC_EINVAL, "NULL argument");
    apply(pool, batch, pool->k, false, false, counts, stats);
  });
}

int gc_apply_batch_seq(gc_graph* g, const gc_batch_desc* batches, int32_t nb, int64_t (*counts)[11],
                       gc_batch_stats* stats) {
  return guard([&] {
    if (!g || (nb > 0 && !batches)) raise(GC_EINVAL, "NULL argument");
    if (g->k != 1) raise(GC_EINVAL, "handle holds %d graphs: gc_apply_batch_seq needs a single graph", g->k);
    if (nb < 0) raise(GC_EINVAL, "negative batch count");
    for (int j = 0; j < nb; ++j)
      check_batch(batches[j], g->gi[0], j, g->any_dead ? g->dead_h.data() : nullptr);  // all-or-nothing
    for (int j0 = 0; j0 < nb;) {
      int q = std::min(GC_SEQ_MAX, nb - j0);
      if (!fold_batches(g, batches + j0, q)) q = 1;
      apply(g, batches + j0, q, false, q > 1, counts ? counts + j0 : nullptr, stats ? stats + j0 : nullptr);
      j0 += q;
    }
  });
}

int gc_get_counts(const gc_graph* g, int32_t graph, int64_t counts[11], uint32_t* overflow_mask) {
  return guard([&] {
    if (!g || !counts) raise(GC_EINVAL, "NULL argument");
    if (graph < 0 || graph >= g->k) raise(GC_EINVAL, "graph index out of range");
    i128 I[11];
    finalize(&g->hstate[graph * ST_STRIDE], g->gl[graph], I);
    to_int64(I, counts, overflow_mask);
  });
}

int gc_get_counts_exact(const gc_graph* g, int32_t graph, int64_t hi[11], uint64_t lo[11]) {
  return guard([&] {
    if (!g || !hi || !lo) raise(GC_EINVAL, "NULL argument");
    if (graph < 0 || graph >= g->k) raise(GC_EINVAL, "graph index out of range");
    i128 I[11];
    finalize(&g->hstate[graph * ST_STRIDE], g->gl[graph], I);
    for (int c = 0; c < 11; ++c) { lo[c] = (uint64_t)I[c]; hi[c] = (int64_t)(I[c] >> 64); }
  });
}

int gc_get_counts3(const gc_graph* g, int32_t graph, int64_t hi[4], uint64_t lo[4]) {
  return guard([&] {
    if (!g || !hi || !lo) raise(GC_EINVAL, "NULL argument");
    if (graph < 0 || graph >= g->k) raise(GC_EINVAL, "graph index out of range");
    i128 I[4];
    finalize3(&g->hstate[graph * ST_STRIDE], g->gl[graph], I);
    for (int c = 0; c < 4; ++c) { lo[c] = (uint64_t)I[c]; hi[c] = (int64_t)(I[c] >> 64); }
  });
}

int gc_recount_exact(gc_graph* g, int32_t graph, int64_t hi[11], uint64_t lo[11]) {
  return guard([&] {
    if (!g || !hi || !lo) raise(GC_EINVAL, "NULL argument");
    if (graph < 0 || graph >= g->k) raise(GC_EINVAL, "graph index out of range");
    if (g->broken) raise(GC_ESTATE, "handle unusable after an earlier device failure");
    HIPCHK(hipSetDevice(g->device));
    hipStream_t s = g->stream;
    PoolDev P = g->pd();
    BatchWork W = make_work(g);
    size_count_scratch(g, 2, g->entries);
    std::vector<long long> st;
    // every entry carries the insertion flag until the last line: a failure
    // in between leaves the handle unusable
    try {
      launch_all_flags(P, GC_F_NEW, GC_ID, s);
      fill_u64((unsigned long long*)g->state_tmp.p, 0ull, (int64_t)g->k * ST_STRIDE, s);
      zero_small(g);
      enqueue_count(g, 2, -1, g->state_tmp.as<long long>(), W, make_count_args(g, 2, g->dense_min_best, true),
                    false, false);
      enqueue_readback(g, g->state_tmp.as<long long>());
      g->sync();
      settle_retries(g, 2, -1, g->state_tmp.as<long long>(), W, g->dense_min_best, g->entries, false, 0, true, false);
      launch_all_flags(P, 0u, GC_ID, s);
      st.assign(g->out_state(), g->out_state() + (size_t)g->k * ST_STRIDE);
      g->sync();
    } catch (...) {
      g->broken = true;
      throw;
    }
    if (st[graph * ST_STRIDE + ST_ERR]) raise(GC_EDEVICE, "inexact totals in the recount");
    i128 I[11];
    finalize(&st[graph * ST_STRIDE], g->gl[graph], I);
    for (int c = 0; c < 11; ++c) { lo[c] = (uint64_t)I[c]; hi[c] = (int64_t)(I[c] >> 64); }
  });
}

int gc_graph_info(const gc_graph* g, int32_t* num_graphs, int32_t graph, int64_t* n, int64_t* m) {
  return guard([&] {
    if (!g) raise(GC_EINVAL, "NULL argument");
    if (num_graphs) *num_graphs = g->k;
    if (graph < 0 || graph >= g->k) raise(GC_EINVAL, "graph index out of range");
    if (n) *n = g->gl[graph];
    if (m) *m = g->hstate[graph * ST_STRIDE + ST_M];
  });
}

int gc_export_edges(gc_graph* g, int32_t graph, int32_t* src, int32_t* dst, int64_t capn, int64_t* m_out) {
  return guard([&] {
    if (!g || !m_out) raise(GC_EINVAL, "NULL argument");
    if (graph < 0 || graph >= g->k) raise(GC_EINVAL, "graph index out of range");
    *m_out = export_edges(g, graph, src, dst, capn);
  });
}

int gc_add_vertices(gc_graph* g, int64_t count, int64_t* first_id, int64_t counts[11]) {
  return guard([&] {
    if (!g) raise(GC_EINVAL, "graph is NULL");
    add_vertices(g, count, first_id);
    counts_now(g, counts);
  });
}

int gc_remove_vertices(gc_graph* g, const int32_t* ids, int64_t count, int64_t counts[11], gc_batch_stats* stats) {
  return guard([&] {
    if (!g) raise(GC_EINVAL, "graph is NULL");
    remove_vertices(g, ids, count, counts, stats);
  });
}

int gc_graph_footprint(int64_t n, const int32_t* src, const int32_t* dst, int64_t m, const gc_options* opt,
                       int64_t* bytes) {
  return guard([&] {
    if (!bytes) raise(GC_EINVAL, "bytes is NULL");
    if (n < 1 || m < 0 || (m > 0 && (!src || !dst))) raise(GC_EINVAL, "bad graph size or edge arrays");
    gc_options o;
    if (opt) o = *opt; else gc_options_default(&o);
    // the largest degree and the largest out-degree under the build order
    // (degree, then id) of the edge list as given; repeats counted, which
    // can only raise the estimate
    std::vector<int32_t> deg((size_t)n, 0), out((size_t)n, 0);
    for (int64_t i = 0; i < m; ++i) {
      const int32_t u = src[i], v = dst[i];
      if (u < 0 || u >= n || v < 0 || v >= n) raise(GC_EINVAL, "edge %lld has a vertex id outside [0, n)", (long long)i);
      if (u != v) { ++deg[u]; ++deg[v]; }
    }
    for (int64_t i = 0; i < m; ++i) {
      const int32_t u = src[i], v = dst[i];
      if (u == v) continue;
      const bool u_first = deg[u] < deg[v] || (deg[u] == deg[v] && u < v);
      ++out[u_first ? u : v];
    }
    int64_t max_deg = 0, max_out = 0;
    for (int64_t v = 0; v < n; ++v) {
      max_deg = std::max<int64_t>(max_deg, deg[v]);
      max_out = std::max<int64_t>(max_out, out[v]);
    }
    *bytes = gc_footprint_estimate(std::max<int64_t>(n, o.vertex_capacity), m, o.slack, max_deg, max_out);
  });
}

int gc_graph_replays(const gc_graph* g, int64_t* captures, int64_t* launches) {
  return guard([&] {
    if (!g) raise(GC_EINVAL, "NULL argument");
    if (captures) *captures = g->graph_captures;
    if (launches) *launches = g->graph_launches;
  });
}

int gc_copy_tuning(gc_graph* dst, const gc_graph* src) {
  return guard([&] {
    if (!dst || !src) raise(GC_EINVAL, "NULL argument");
    if (dst == src) return;
    // hub-window threshold and its trials
    dst->tune_cands = src->tune_cands;
    dst->tune_ms = src->tune_ms;
    dst->tune_wedges = src->tune_wedges;
    dst->tune_next = src->tune_next;
    dst->dense_min_best = src->dense_min_best;
    // tier thresholds and their trials (unless the destination's are forced)
    if (!dst->tiers_forced) {
      dst->tier_cands = src->tier_cands;
      dst->tier_tri_cost = src->tier_tri_cost;
      dst->tier_c4_cost = src->tier_c4_cost;
      dst->tier_next = src->tier_next;
      std::copy(src->tiers_best, src->tiers_best + 3, dst->tiers_best);
      std::copy(src->tiers_best, src->tiers_best + 3, dst->tiers_now);
    }
    // whole-graph switch, pass-kind and multi-version cost models, and the
    // edge-local list demand per update
    std::copy(src->region_frac, src->region_frac + 8, dst->region_frac);
    std::copy(&src->mode_ms[0][0], &src->mode_ms[0][0] + 32, &dst->mode_ms[0][0]);
    std::copy(&src->mode_sz[0][0], &src->mode_sz[0][0] + 32, &dst->mode_sz[0][0]);
    std::copy(&src->mode_n[0][0], &src->mode_n[0][0] + 32, &dst->mode_n[0][0]);
    dst->region_ms_all = src->region_ms_all;
    dst->region_n_all = src->region_n_all;
    dst->delta_ms_min = src->delta_ms_min;
    std::copy(src->multi_ms, src->multi_ms + GC_NV_MAX, dst->multi_ms);
    std::copy(src->multi_n, src->multi_n + GC_NV_MAX, dst->multi_n);
    dst->ae_per_update = src->ae_per_update;
    dst->pair_per_update = src->pair_per_update;
  });
}

int gc_graph_free(gc_graph* g) {
  if (!g) return GC_OK;
  (void)hipSetDevice(g->device);
  delete g;
  return GC_OK;
}

const char* gc_strerror(int code) {
  switch (code) {
    case GC_OK: return "ok";
    case GC_EINVAL: return "invalid argument";
    case GC_ENOMEM: return "out of memory";
    case GC_EDEVICE: return "device error";
    case GC_EBUSY: return "busy";
    case GC_ESTATE: return "handle unusable";
  }
  return "unknown error";
}

const char* gc_last_error(void) { return g_err.c_str(); }

}  // extern "C"
