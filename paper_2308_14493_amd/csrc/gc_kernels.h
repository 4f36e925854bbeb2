// Launcher declarations shared by the kernel files and the host code.
#pragma once
#include "gc_internal.h"

// device counters (u64) of one batch
enum {
  C_DIRA = 0,     // directed entries of pairs absent before the pass and present in a later version
  C_DIRD,         // directed entries of existing edges absent from a later version
  C_DIRR,         // directed entries absent from the last version (removed by the purge)
  C_TOUCH,        // rows touched by the pass
  C_NKEYS,        // update entries of the pass (set by the ingest kernel)
  C_RLIST,        // region vertices (first counter of the counting stage)
  C_LVL0,         // C_LVL0 + k: end of level-k vertices in the region list (k = 0..4)
  C_ER = C_LVL0 + 6,  // region entries
  C_MAXDP,        // max oriented out-degree
  C_MAXW,         // max wedge bound
  C_MAXLOW,       // max lower degree in the large 4-cycle tier
  C_LIST0,        // C_LIST0 + L_*: work list sizes
  C_QHEAD = C_LIST0 + 12,  // dynamic queue head of the large 4-cycle tier
  C_QTRI,                  // C_QTRI + k: queue head of list L_TRI_1 + k (k < 6)
  C_QTS = C_QTRI + 6,      // queue heads of the small triangle tier and of the mid 4-cycle tier
  C_QC4M,
  C_COUNT
};
// Work lists: triangles by out-degree (<= 64 one wave per vertex, then the
// workgroup tiers (64,128] (128,256] (256,512] (512,1024] (1024,TRI_LDS_MAX]
// in LDS and the global-scratch tier above), 4-cycles by wedge bound.
enum { L_TRI_S = 0, L_TRI_1, L_TRI_2, L_TRI_3, L_TRI_4, L_TRI_5, L_TRI_G, L_C4_S, L_C4_M, L_C4_L, L_NUM };
constexpr int TRI_LDS_MAX = 1280;
static_assert(L_NUM <= 12, "list counters");

__host__ __device__ inline int tri_list_of(int32_t dplus, int32_t small) {
  if (dplus <= small) return L_TRI_S;
  if (dplus <= 128) return L_TRI_1;
  if (dplus <= 256) return L_TRI_2;
  if (dplus <= 512) return L_TRI_3;
  if (dplus <= 1024) return L_TRI_4;
  if (dplus <= TRI_LDS_MAX) return L_TRI_5;
  return L_TRI_G;
}

// Directed entry keys of the merge lists: row << bits | col, with the
// absence mask of the edge (bit x = absent from version x) in bits 60..63.
#define DIR_MASK_SHIFT 60
#define DIR_KEY_MASK ((1ull << DIR_MASK_SHIFT) - 1ull)

// Segments of the update arrays: one per graph of a pool (seq = 0), or one
// per successive batch of graph 0 (seq = 1).
struct BatchIn {
  const int32_t* iu; const int32_t* iv; const int32_t* du; const int32_t* dv;
  int64_t n_ins, n_del;
  const int64_t* ins_seg;  // [k+1] insertion segment bounds
  const int64_t* del_seg;  // [k+1]
  const int64_t* gbase;    // [graphs] first vertex of each graph
  const int64_t* gn;       // [graphs] vertex count of each graph
  int32_t k;               // segments
  int32_t seq;
  const uint8_t* dead;     // [N] 1 for a vertex taken out of its graph (nullptr: none)
};

struct BatchWork {
  unsigned long long* c;       // counters
  unsigned long long* dirA;    // sorted directed entry keys (see DIR_MASK_SHIFT)
  unsigned long long* dirD;
  unsigned long long* dirR;
  // per row: segment of dirA (a_beg, na) and of dirR (r_beg, nr)
  int32_t* a_beg; int32_t* na; int32_t* r_beg; int32_t* nr; int32_t* mark; int32_t* tix;  // [N]
  int32_t* touched;            // [max_touched]
  int64_t* dest; int32_t* newcap; int32_t* tlen; int64_t* tpre;  // [max_touched (+1)]
  uint32_t* scratch;           // copy of the touched rows
};

// graph.hip
// The update counts live on the device (ins_seg[k], del_seg[k]); cap_total
// bounds their sum and sizes the grid.  Sets c[C_NKEYS].
void launch_ingest_keys(const PoolDev& P, const BatchIn& B, int bits, unsigned long long* keys, unsigned long long* c,
                        unsigned long long* bstats, int64_t cap_total, hipStream_t s);
// keys: pair << 3 | batch << 1 | op (c[C_NKEYS] of them); nb batches in the
// pass, nv versions
void launch_ingest_classify(const PoolDev& P, const unsigned long long* keys, int64_t cap_total, int bits, int nb,
                            int nv, unsigned long long* dirA, unsigned long long* dirD, unsigned long long* dirR,
                            unsigned long long* c, unsigned long long* bstats, hipStream_t s);
// beg/cnt may be null (rows are then only marked as touched)
void launch_mark_rows(const unsigned long long* dir, int64_t max_n, unsigned long long* c, int which, int bits,
                      int32_t* beg, int32_t* cnt, int32_t* mark, int32_t* touched, int32_t* tix, hipStream_t s);
void launch_merge(const PoolDev& P, const BatchWork& W, int64_t max_touched, int64_t max_dirA, int bits, float slack,
                  unsigned long long* bstats, void* scan_tmp, hipStream_t s);
void launch_flag_rows(const PoolDev& P, const BatchWork& W, int64_t max_dirD, int bits, unsigned long long* bstats,
                      hipStream_t s);
// removes the entries carrying `fin` (absent from the last version), clears
// all flags; does nothing while *skip != 0.  undo: removes the entries new
// in the pass instead (GC_F_NEW, listed in W.dirA), which restores the graph
// as it was before a one-batch pass whose counting did not complete
void launch_purge(const PoolDev& P, const BatchWork& W, int64_t max_touched, int bits, uint32_t fin,
                  const unsigned long long* skip, void* scan_tmp, hipStream_t s, bool undo = false);
// the purge of a pass without deletions: the flags of the new entries are
// cleared in place (max_dirA bounds their count)
void launch_purge_insert_only(const PoolDev& P, const BatchWork& W, int64_t max_touched, int64_t max_dirA, int bits,
                              const unsigned long long* skip, hipStream_t s);
void launch_region(const PoolDev& P, const BatchWork& W, int radius, int32_t* level, int32_t* rlist, int32_t* rlen,
                   hipStream_t s);
void launch_region_fill(const PoolDev& P, const RegionDev& R, const BatchWork& W, int radius, const int32_t* level,
                        const int32_t* rlist, const int32_t* rlen, void* scan_tmp, hipStream_t s);
// wave_row in [1, 65536]: rows at least this long are walked by a whole wave
void launch_degrees(int nv, const RegionDev& R, const int32_t* gid, const int32_t* rlist, unsigned long long* c,
                    unsigned long long* sig, int32_t* lists, int64_t list_stride, int32_t tri_small, int32_t c4_small,
                    int32_t c4_mid, int32_t wave_row, unsigned long long* bstats, unsigned long long* c4_keys,
                    hipStream_t s);
void launch_init_keys(const int32_t* src, const int32_t* dst, int64_t m, const int64_t* seg, const int64_t* gbase,
                      int32_t k, int bits, unsigned long long* keys, hipStream_t s);
void launch_init_unique(const unsigned long long* keys, int64_t m, int bits, unsigned long long* uniq,
                        unsigned long long* c, int32_t* deg, hipStream_t s);
void launch_rank(const int32_t* deg, const int32_t* gid, const int64_t* gbase, int64_t N, int lbits, int total_bits,
                 unsigned long long* keys, unsigned long long* alt, void* sort_tmp, int32_t* ext2int, int32_t* int2ext,
                 hipStream_t s);
void launch_init_dir(const unsigned long long* uniq, int64_t max_m, unsigned long long* c, int bits,
                     const int32_t* ext2int, unsigned long long* dir, int32_t* len, hipStream_t s);
void launch_init_csr(const PoolDev& P, const unsigned long long* dir, int64_t max_dir, unsigned long long* c, int bits,
                     int64_t* rstart, float slack, void* scan_tmp, uint32_t flag, hipStream_t s);
void launch_caps(const PoolDev& P, float slack, hipStream_t s);  // P.cap <- len + slack
void launch_all_flags(const PoolDev& P, uint32_t set, uint32_t keep, hipStream_t s);
void launch_compact(const PoolDev& P, int64_t* noff, uint32_t* ncol, hipStream_t s);
void launch_upper_count(const PoolDev& P, int32_t* cnt, hipStream_t s);
// rows of k vertices of a single graph (external ids): lengths, then the
// edges (x, neighbour) in external ids at the exclusive prefix pre
void launch_row_len(const PoolDev& P, const int32_t* ids, int64_t k, int32_t* out, hipStream_t s);
void launch_row_gather(const PoolDev& P, const int32_t* int2ext, const int32_t* ids, int64_t k, const int64_t* pre,
                       int32_t* u, int32_t* v, hipStream_t s);
// a[ids[i]] = val
void launch_set_bytes(uint8_t* a, const int32_t* ids, int64_t k, uint8_t val, hipStream_t s);
void launch_export(const PoolDev& P, const int32_t* int2ext, const int64_t* gbase, const int64_t* pre, int32_t* src,
                   int32_t* dst, hipStream_t s);

// count.hip
struct CountArgs {
  RegionDev R;
  const int32_t* gid;
  const int32_t* lists;     // L_NUM lists of list_stride entries
  int64_t list_stride;
  const unsigned long long* c;
  unsigned long long* sig;
  unsigned long long* bstats;
  // per-slot scratch of the large tiers
  unsigned long long* c4_dense;   // [slots][N] (two versions, or four with 16-bit fields)
  int32_t* c4_touch;              // [slots][N]
  int64_t N;
  int32_t slots;                  // workgroups of the large 4-cycle tier
  int32_t c4_win;                 // 64-bit words of the LDS window of the large tier (<= c4_window_max())
  int32_t c4_narrow_max;          // up to this many lower neighbours, 16-bit counters (2x window)
  int64_t c4_dense_min;           // hits that earn a window dense LDS counters
  uint32_t c4_ref;                // versions whose common wedges the hub windows count (the rest are exceptions)
  int64_t* c4_cur;                // [slots][2 * c4_maxlow]: row starts, cursors
  int32_t* c4_blk;                // [N / C4_BLK + 1] largest union row length per block of C4_BLK ids
  int64_t c4_maxlow;              // largest lower degree of a large-tier vertex
  unsigned long long* c4_keys;    // [N] sort keys of the large tier (written by the per-vertex pass)
  unsigned long long* c4_keys_alt;
  void* sort_tmp;
  int32_t tri_slots;              // workgroups of the global-scratch triangle tier
  unsigned long long* tri_scratch;  // [tri_slots][tri_scratch_words64(tri_cap)] above the LDS tier
  int64_t tri_cap;                  // out-degree capacity of a scratch slot (0: no scratch)
  int64_t e_max;                    // capacity of the region arrays (entries)
};
// nv = 2 or 4 versions.  Grids come from host bounds (A.N, A.e_max, the
// scratch sizes); work sizes from the device counters.
void launch_count(int nv, const CountArgs& A, hipStream_t s,
                  hipEvent_t* ev /* nullable: 6 events between the kernel phases */);
int64_t tri_scratch_words64(int nv, int64_t cap);  // u64 words of one triangle scratch slot
int32_t tri_lds_max(int nv);                        // largest out-degree of the LDS triangle tiers
int32_t c4_window_max();                            // u64 words of the LDS window of the large 4-cycle tier
int32_t c4_block_ids();                             // ids per entry of CountArgs::c4_blk
// Per graph g: the state after version x (x = 1 .. nv-1) goes to
// vout[((x - 1) * k + g) * ST_STRIDE ...]; state becomes the one of version nv-1.
// nothing is written while bstats[BS_RETRY] != 0
void launch_combine(int nv, const unsigned long long* sig, long long* state, long long* vout, int32_t k,
                    const unsigned long long* bstats, hipStream_t s);

// capi.cpp: thread-local error text read by gc_last_error()
// delta.hip: edge-local update of the Sigma terms of a one-batch pass
enum { DC_EDGES = 0, DC_AFF, DC_AFF_TOTAL, DC_AFF_NEED, DC_SLOT_NEED, DC_QTRI, DC_QC4, DC_PAIR_NEED, DC_MERGE,
       DC_HS, DC_HITEMS, DC_HEAVY, DC_QK4, DC_QH, DC_QAFF, DC_QMERGE, DC_COUNT };
// 4-cliques of changed edges with many common neighbours, spread over the
// workgroups in chunks: the common neighbours of such edges (with their
// flags), the edges, and the chunks (fixed capacities; an edge that does not
// fit is counted in place)
constexpr int K4_HEAVY_MIN = 256;       // common neighbours from which an edge is split
constexpr int K4_CHUNK = 64;            // common neighbours per chunk
constexpr int64_t K4_HS_CAP = 1 << 22;  // stored common neighbours
constexpr int64_t K4_HE_CAP = 1 << 14;  // split edges
constexpr int64_t K4_IT_CAP = 1 << 18;  // chunks
constexpr int32_t TV_CHUNK = 4096;      // entries of a touched row per piece in the edge-local degree passes
// 4-cycle pairs (e, a) with a shorter N(a) that is not merged, counted
// against an LDS hash table of N(o): rows N(o) of at most C4H_MAX entries
// (table of C4H_SLOTS, load <= 1/2); work in chunks of at least
// C4H_CHUNK_MIN entries of the walked rows and four times |N(o)| (the
// table build)
constexpr int C4H_SLOTS = 32768;
constexpr int32_t C4H_MAX = 16384;
constexpr int64_t C4H_CHUNK_MIN = 16384;
constexpr int C4H_T = 1024;
struct DeltaArgs {
  PoolDev P;                          // union view left by the tombstone merge
  int64_t N;
  int bits;
  const unsigned long long* dirA;     // sorted directed change lists (counts in c)
  const unsigned long long* dirD;
  const unsigned long long* c;        // batch counters (C_DIRA, C_DIRD, C_TOUCH)
  const int32_t* touched;             // touched rows
  const int32_t* mark;                // [N] 1 on touched rows
  const int32_t* gid;                 // [N] graph of each vertex
  unsigned long long* sig;            // per-graph sums; version 1 receives the deltas
  unsigned long long* bstats;         // BS_RETRY when a buffer below is too small
  int32_t* dd;                        // [N][2] degrees before / after of the touched rows
  long long* Tv;                      // [N] triangles at each vertex (moved to the graph after the batch)
  unsigned long long* dT;             // [N] scratch, zero between passes: twice the change of T(v)
  unsigned long long* sbt;            // [N] scratch, zero between passes: t before of affected edges at v
  unsigned long long* ce;             // changed pairs (u < v) | nibble << 60
  int64_t ce_cap;
  unsigned long long* ae;             // affected edge keys and their sort buffer
  unsigned long long* ae_alt;
  int64_t ae_cap;
  void* sort_tmp;                     // radix sort scratch for ae_cap keys
  unsigned long long* slot_mark;      // [slots][N] dense marks, zero between uses
  uint32_t* slot_list;                // [slots][slot_cap] common neighbours of a changed edge
  int64_t slot_cap;
  unsigned long long* dc;             // [DC_COUNT] counters of the stage
  int32_t* c4_nch;                    // [ce_cap] pairs (e, a) per changed edge: degree of the end walked from
  int32_t* c4_side;                   // [ce_cap] 0: walk from u, 1: from v
  int64_t* c4_off;                    // [ce_cap + 1] exclusive scan of c4_nch
  int32_t* pair_edge;                 // [pair_cap] changed edge of each pair
  int32_t* pair_len;                  // [pair_cap] walk length of each pair (0: merged instead)
  int32_t* pair_merge;                // [pair_cap] pairs whose rows are merged by a wave (DC_MERGE of them)
  uint32_t* k4_s;                     // [K4_HS_CAP] common neighbours of split edges: id | nibble(u, w) << 28 | nibble(v, w) << 30
  int64_t* k4_edge;                   // [K4_HE_CAP][3] split edges: changed edge index, offset in k4_s, count
  int32_t* k4_item;                   // [K4_IT_CAP][2] chunks: split edge (-1: none), chunk index
  int32_t* tv_items;                  // [tcap] pieces of each touched row (rows split in TV_CHUNK entries)
  int64_t* tv_ioff;                   // [tcap + 1] exclusive scan of tv_items
  int64_t tcap;                       // touched rows the two arrays cover (>= the touched count)
  int64_t* pair_off;                  // [pair_cap + 1] exclusive scan of pair_len
  int32_t* pair_hlen;                 // [pair_cap] entries of N(a) walked against the hash of N(o) (0: other ways)
  int64_t* pair_hoff;                 // [pair_cap + 1] exclusive scan of pair_hlen
  int64_t pair_cap;
  void* scan_tmp;                     // scan scratch for max(ce_cap, pair_cap) + 1 entries
};
// launches the delta stage with `slots` workgroups for the per-edge kernels
void launch_delta(const DeltaArgs& D, int slots, hipStream_t s);
// T(v) of the region vertices after a region pass (t of the last version
// minus t of version 0); dT zero before and after
void launch_tv_region(int nv, const RegionDev& R, const int32_t* rlist, const unsigned long long* c,
                      unsigned long long* dT, long long* Tv, unsigned long long* bstats, hipStream_t s);

void gc_set_error(const char* msg);
// device bytes a single-graph handle reaches (capi.cpp); used by the server's admission
int64_t gc_footprint_estimate(int64_t n, int64_t m, double slack, int64_t max_deg, int64_t max_out);
