// Host-side launchers and device records shared between the libslim
// translation units.
//
// Every compute call works on a *graph set*: one or more graphs laid out
// back to back in a union CSR (graph g owns vertices [vb, vb+nv) and CSR
// entries [eb, eb+ne) of the union, with union vertex ids in the columns).
// A single-graph call is a set of one whose union is the caller's CSR; a
// batch gathers its graphs into a union first.  Work tiles never straddle
// two graphs, so the graph of a tile -- its random key, threshold, output
// arrays and counters -- is a per-tile constant.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/slim.h"
#include "slim_device.h"

namespace slim {

// One graph of a set.
struct GDesc {
  uint64_t vb, nv;         // union vertices [vb, vb + nv)
  uint64_t eb, ne;         // union CSR entries [eb, eb + ne)
  uint64_t thr;            // triangle selected / edge deleted iff Philox word 0 < thr
  double ups;              // spectral sparsification parameter upsilon
  uint32_t k0, k1;         // Philox key (seed)
  uint32_t op;             // SLIM_OP_* code of the graph's job
  uint32_t pad;
  uint64_t cap;            // capacity of out_col in entries
  const int64_t* in_row;   // the graph's own CSR (gather source of a batch)
  const uint32_t* in_col;
  void* out_row;           // row starts, nv + 1 (int64; uint32 for the DAG)
  uint32_t* out_col;       // columns, local ids
  float* out_w;            // spectral sparsification: weight per output entry (optional)
  slim_stats_t* stats;     // optional
};

// One work tile: union entries [j0, j0 + span) of graph g.  It owns the row
// starts of union rows [lo, hi); the last tile of a graph owns the rows up
// to the graph's end and also writes the graph's end offset.
struct TileRec {
  int64_t j0;
  uint32_t span;
  uint32_t g;
  uint32_t lo, hi;
  uint32_t last;
  uint32_t pad;
};

void fill_u32(uint32_t* p, uint64_t len, uint32_t v, hipStream_t s);
void fill_i64(int64_t* p, uint64_t len, int64_t v, hipStream_t s);

uint64_t scan_tmp_elems(uint64_t len);
template <typename TI>
void scan_excl(const TI* in, uint64_t len, uint64_t* out, uint64_t* tmp, hipStream_t s);

uint64_t sort_hist_elems(uint64_t n);
void degree_rank(const int64_t* row_off, uint64_t n, int passes, uint32_t* ka, uint32_t* va,
                 uint32_t* kb, uint32_t* vb, uint32_t* hist, uint64_t* hist_scan,
                 uint64_t* scan_tmp, uint32_t** order_out, uint32_t* rank, hipStream_t s);

// Copies up to 512 bytes of host data (descriptors) to device memory by a
// kernel launch: no host-to-device copy, so it can sit in a captured graph.
void put_bytes(void* dst, const void* src, uint32_t bytes, hipStream_t s);
// Tile records of a set with `tile` entries per tile; tile0[g] is the first
// tile of graph g (tile0[count] = ntiles; every graph has at least one tile).
void tile_recs(const int64_t* row_off, const GDesc* gd, const uint64_t* tile0, uint32_t count,
               uint64_t ntiles, uint64_t tile, TileRec* recs, hipStream_t s);
// Gathers the graphs of a set into the union CSR (union ids in ucol).
// vtile0 / etile0: per-graph prefixes of kTile-sized vertex / entry chunks.
void gather(const GDesc* gd, uint32_t count, const uint64_t* vtile0, const uint64_t* etile0,
            uint64_t nvt, uint64_t net, uint64_t N, uint64_t NNZ, int64_t* urow, uint32_t* ucol,
            hipStream_t s);

// DAG: dag_col = rank ids of the forward entries, fstart = row starts;
// rcol[j] = rank of col[j] for every entry.
void orient(const int64_t* row_off, const uint32_t* col, const uint32_t* rank, uint32_t* rcol,
            const GDesc* gd_union, const uint64_t* tile0, const TileRec* recs, uint64_t ntiles,
            uint32_t* tile_cnt, uint64_t* masks, uint64_t* tile_base, uint64_t* scan_tmp,
            hipStream_t s);
void dag_ranges(const uint32_t* order, const uint32_t* fstart, uint64_t n, uint2* dag_rng,
                hipStream_t s);
// Output CSRs of every graph of the set: TR graphs keep the entries whose
// edge is unmarked, ES graphs the entries whose edge is not sampled out.
// eid/del may be NULL when the set has no TR graph.  masks: kChunks words per
// tile (the count pass's ballots, read back by the scatter pass).
// Packs the per-edge deletion bytes into the bitmap the compaction reads
// (32 bytes -> one word).
void pack_marks(const uint8_t* marks, uint32_t* del, uint64_t m, hipStream_t s);
void compact_out(const int64_t* row_off, const uint32_t* col, const uint32_t* eid,
                 const uint32_t* del, uint64_t m, const GDesc* gd, const uint64_t* tile0,
                 const TileRec* recs, uint64_t ntiles, uint32_t* tile_cnt, uint64_t* masks,
                 uint64_t* tile_base, uint64_t* scan_tmp, hipStream_t s);
// Per-graph stats from the triangle counters (2 per graph, may be NULL) and
// the compaction's tile scan.
void write_stats(const GDesc* gd, uint32_t count, const uint64_t* tile0,
                 const uint64_t* counters, const uint64_t* tile_base, hipStream_t s);
void validate_offsets(const int64_t* row_off, uint64_t n, uint64_t nnz, uint32_t* err,
                      hipStream_t s);
void validate_entries(const int64_t* row_off, const uint32_t* col, uint64_t n,
                      const TileRec* recs, uint64_t ntiles, uint32_t* err, hipStream_t s);

// Every DAG row is sorted by rank id (slim_sort.hip); rows of length up to
// kSortMin by one thread each.
constexpr uint32_t kSortMin = 32;
void sort_rows(const uint2* dag_rng, uint64_t n, uint32_t* dag_col, uint32_t* lists,
               uint32_t* counts, int num_cu, hipStream_t s);
// fence[q] = dag_col[kFenceStep * q]: the first rank id of every 128-byte
// line of the sorted DAG columns, so that a search for a rank id in a DAG
// row reads the row's samples and then a single line of dag_col.
constexpr uint32_t kFenceStep = 32;
void fence_samples(const uint32_t* dag_col, uint64_t m, uint32_t* fence, hipStream_t s);

// Triangle listing + selection + deletion marks (slim_tri.hip).
struct TriArgs {
  const int64_t* row_off;
  const uint32_t* col;
  const uint32_t* rank;
  const uint32_t* rcol;    // rank id of every CSR column
  const uint32_t* order;
  const uint2* dag_rng;    // DAG row of each rank id
  const uint32_t* fstart;  // DAG row start of each union id (N+1)
  const uint32_t* dag_col;
  const uint32_t* fence;   // dag_col[kFenceStep * q] for every q
  uint32_t* eid;           // backward CSR entries get their DAG position here
  uint8_t* marks;          // deletion marks over DAG positions, one byte per edge
  uint64_t* counters;      // per graph: [2g] triangles, [2g+1] selected
  const GDesc* gd;
  const TileRec* recs;     // graph-aligned tiles of at most tri_tile_max() entries
  uint64_t ntiles;
  uint32_t* tcount;        // Min-Count: triangles per DAG edge (NULL if unused)
  uint64_t* minkey;        // Edge-Once: smallest bid per DAG edge in the current round
  uint32_t* closed;        // Edge-Once: bitmap of closed DAG edges
  uint64_t* eo_und;        // Edge-Once: undecided selected triangles of round r at [r]
  uint32_t* eo_live;       // Edge-Once: last round in which each tile bid
  uint4* eo_list;          // Edge-Once: two lists of undecided triangles (two
                           //   uint4 each), eo_cap triangles apart
  uint64_t* eo_list_cnt;   // Edge-Once: triangles written to list 0 and list 1
  uint32_t* eo_state;      // Edge-Once: [0] = round that listed the triangles (0: none)
  uint64_t eo_cap;         // Edge-Once: capacity of each list in triangles
  uint32_t gcount;         // graphs of the set (gd[0 .. gcount))
  uint32_t pass;           // 0: Min-Count counting, 1: selection and marks,
                           // 2: Edge-Once bids
  uint32_t round;          // Edge-Once round (1, 2, ...)
  uint32_t eo_list_try;    // Edge-Once: Tuning::eo_list_try
};
uint64_t tri_tile_max();
// Instantiations of the triangle kernel: plain (p-1 only), general (also
// p-2 and the Min-Count selection pass), Edge-Once (its bidding passes), and
// counting (the Min-Count counting pass: per-edge triangle counts only, no
// selection, so hits are counted where they are found).
constexpr int kModePlain = 0, kModeGeneral = 1, kModeEO = 2, kModeCount = 3;
void triangles(const TriArgs& a, int mode, uint32_t* tile_ctr, int num_cu,
               int blocks_per_cu, int chunk, hipStream_t s);

// Op codes that list triangles.
__host__ __device__ inline bool op_lists_triangles(uint32_t op) {
  return op == SLIM_OP_TR || op == SLIM_OP_TR2 || op == SLIM_OP_MCTR || op == SLIM_OP_EOTR;
}
__host__ __device__ inline bool op_valid(int op) {
  return op >= SLIM_OP_TR && op <= SLIM_OP_EOTR;
}

// Edge-Once rounds: each round clears the bids (closing, from the second
// round on, every edge that got none) and runs the bidding and acceptance
// passes; every launch returns at once after the round that found no
// undecided triangle.  Rounds are enqueued Tuning::eo_rounds at a time, the
// host checks the last round's counter in between; kEoMaxRounds bounds the
// counter array (the rounds of greedy parallel maximal independent set with
// random priorities grow as log of the triangle count).
constexpr uint32_t kEoMaxRounds = 1024;
// Capacity of each Edge-Once list in triangles per DAG edge.  A bidding
// pass tries to start the list once the previous round's undecided count is
// at most Tuning::eo_list_try percent of the capacity (R-MAT graphs keep
// about a third to two fifths of them per round); if its own bidders
// overflow the list, the round accepts by the edge-parallel kernel and the
// next round may list again.
// Later rounds copy the survivors from one list into the other, so their
// cost falls with the undecided count.  The two lists take
// 2 * 32 * kEoListPerEdge bytes of workspace per edge.
constexpr uint64_t kEoListPerEdge = 3;
// A list round clears the previous round's bids through that round's list
// records when there are at most this many (three random stores each),
// instead of sweeping every edge.
constexpr uint64_t kEoListClearMax = 1ull << 23;
void eo_clear_bids(uint64_t* minkey, uint32_t* closed, uint64_t m, const uint64_t* eo_und,
                   const uint32_t* eo_state, const uint64_t* eo_list_cnt, uint32_t round,
                   hipStream_t s);
// Acceptance of round a.round by an edge-parallel kernel over the n union
// vertices (returns at once once the triangles are listed).
void eo_accept_edges(const TriArgs& a, uint64_t n, int num_cu, hipStream_t s);
// Start of round a.round: a list that the previous round started but
// overflowed is dropped (the round accepted by the edge-parallel kernel).
void eo_round_start(const TriArgs& a, hipStream_t s);
// Clears the bids of the previous round through its list records, when the
// round runs on the lists and they are few (k_eo_clear_bids sweeps otherwise).
void eo_list_clear(const TriArgs& a, int num_cu, hipStream_t s);
// Bids and acceptance of round a.round on the triangle lists (both return
// at once unless the list was started in an earlier round; acceptance also
// in the listing round).  Round r after the listing round L bids from list
// (r - L - 1) mod 2 and copies the triangles that bid into the other list,
// which its acceptance then reads; the listing round's acceptance reads
// list 0.
void eo_list_round(const TriArgs& a, int num_cu, hipStream_t s);

// Scheduling knobs; never change results.
struct Tuning {
  int tri_chunk = 2048;       // out-list entries hashed per pass
  int tri_blocks_per_cu = 2;  // resident blocks of the triangle kernel per CU
  int tri_tile = 1024;        // CSR entries per triangle tile (a power of two, 256..1024)
  int eo_rounds = 16;         // Edge-Once rounds enqueued before the host checks (1..64)
  int eo_list_try = 250;      // Edge-Once: list from a round whose previous undecided count is
                              //   at most this percent of the list capacity (0..100000)
};
Tuning& tuning();
// Checks a knob value; returns false if `key` is unknown or out of range.
bool tune_apply(Tuning& t, const char* key, int64_t value);
bool tune_read(const Tuning& t, const char* key, int64_t* value);

}  // namespace slim
