// The shape, workspace layout and launch sequence of a graph set, shared by
// the single-graph calls, batches and the server.
#pragma once

#include <mutex>
#include <vector>

#include "slim_internal.h"

struct slim_graph {
  const int64_t* row_off;
  const uint32_t* col;
  uint64_t n;
  uint64_t nnz;
  int device;
  int num_cu;
};

namespace slim {

constexpr uint64_t kTriTileMin = 256;  // smallest triangle tile (workspace is sized for it)

struct SetShape {
  uint32_t count = 0;
  uint64_t N = 0, NNZ = 0;  // union vertices and CSR entries
  bool gathered = false;    // union built in the workspace (batches)
  bool has_tr = false;      // some graph lists triangles (TR, TR2, MCTR, EOTR)
  bool has_list = false;    // some graph runs TR, TR2 or MCTR (the selection pass)
  bool general = false;     // some graph runs TR2 or MCTR (general kernel for the selection pass)
  bool has_mc = false;      // some graph runs MCTR (counting pass)
  bool has_eo = false;      // some graph runs EOTR (rounds of bids and acceptance)
  uint64_t n_c = 0;         // graph-aligned tiles of kTile entries (compaction)
  uint64_t n_u = 0;         // union tiles of kTile entries (orientation)
  uint64_t n_tri[3] = {0, 0, 0};  // graph-aligned triangle tiles of 256, 512, 1024 entries
  uint64_t nvt = 0, net = 0;      // gather chunks: vertex and entry
  int passes = 1;                 // radix passes of the degree sort
  uint64_t n_t(int tile) const { return n_tri[tile <= 256 ? 0 : tile <= 512 ? 1 : 2]; }
};

// Byte offsets into the workspace.
struct SetLayout {
  uint64_t gd, t0c, t0t, t0u, vt0, et0, hdr_bytes;
  uint64_t urow, ucol;
  uint64_t recs_c, recs_u, recs_t;
  uint64_t tile_cnt, tile_base, scan_tmp, masks;
  uint64_t ka, va, kb, vb, rank, rcol, hist, hist_scan;
  uint64_t fstart, dag_rng, dag_col, fence, eid, del, marks, counters;
  uint64_t sort_lists, sort_counts, tri_ctr, tcount;
  uint64_t minkey, closed, eo_und, eo_live, eo_list, eo_misc;
  uint64_t total;
};

int fail(int code, const char* fmt, ...);
int ok();
int hip_check(const char* what);
const char* last_error();
uint64_t threshold(double p);
int check_p(double p);
// p of an operation: a probability in [0,1], or upsilon >= 0 for spectral
// sparsification.
int check_param(int op, double p);
int radix_passes(uint64_t maxdeg);
uint64_t tiles_of(uint64_t ne, uint64_t tile);
SetLayout set_layout(const SetShape& S);
GDesc union_desc(const SetShape& S, const SetLayout& L, void* ws);
void run_set(const SetShape& S, const SetLayout& L, const Tuning& knobs, int num_cu, void* ws,
             const int64_t* row_off, const uint32_t* col, hipStream_t s, bool profile);
// Sets with Edge-Once graphs: after run_set (or the replay of its capture)
// on stream s, waits for s, runs further rounds while the last one still
// found undecided triangles and then compacts again.  SLIM_OK at once for
// other sets.
int eo_finish(const SetShape& S, const SetLayout& L, const Tuning& knobs, int num_cu, void* ws,
              const int64_t* row_off, const uint32_t* col, hipStream_t s);
void prof_reset();
std::mutex& tuning_mutex();

// A set of graphs as planned on the host: per-graph descriptors with union
// bases, tile and gather-chunk prefixes, and the set's shape.
struct SetPlan {
  SetShape shape;
  std::vector<GDesc> gd;  // count (+1 slot for the union, filled per run)
  std::vector<uint64_t> t0c, vt0, et0, ne;
};
// Fills bases, prefixes and shape from descriptors whose vb/eb are unset
// (nv, ne, op, thr, key, inputs given).  Returns SLIM_EINVAL if the union
// exceeds the id limits.
int plan_set(const std::vector<GDesc>& graphs, SetPlan& P);
// Host image of the set header for workspace `ws` (per-graph outputs come
// from P.gd).
void fill_header(const SetPlan& P, const SetLayout& L, const Tuning& knobs, void* ws,
                 std::vector<char>& hdr);

}  // namespace slim
