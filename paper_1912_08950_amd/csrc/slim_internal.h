// Host-side launchers shared between the libslim translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/slim.h"
#include "slim_device.h"

namespace slim {

void fill_u32(uint32_t* p, uint64_t len, uint32_t v, hipStream_t s);
void fill_i64(int64_t* p, uint64_t len, int64_t v, hipStream_t s);

uint64_t scan_tmp_elems(uint64_t len);
template <typename TI>
void scan_excl(const TI* in, uint64_t len, uint64_t* out, uint64_t* tmp, hipStream_t s);

uint64_t sort_hist_elems(uint64_t n);
void degree_rank(const int64_t* row_off, uint64_t n, int passes, uint32_t* ka, uint32_t* va,
                 uint32_t* kb, uint32_t* vb, uint32_t* hist, uint64_t* hist_scan,
                 uint64_t* scan_tmp, uint32_t** order_out, uint32_t* rank, hipStream_t s);

void tile_lo_build(const int64_t* row_off, uint64_t n, uint64_t nnz, uint64_t ntiles,
                   uint32_t* tile_lo, hipStream_t s, uint64_t tile = kTile);
void orient(const int64_t* row_off, const uint32_t* col, const uint32_t* rank, uint64_t n,
            uint64_t nnz, uint64_t ntiles, const uint32_t* tile_lo, uint32_t* tile_cnt,
            uint64_t* tile_base, uint64_t* scan_tmp, uint32_t* dag_col, uint32_t* eid,
            uint32_t* fstart, hipStream_t s);
void dag_ranges(const uint32_t* order, const uint32_t* fstart, uint64_t n, uint2* dag_rng,
                hipStream_t s);
void compact_tr(const int64_t* row_off, const uint32_t* col, const uint32_t* eid,
                const uint32_t* del, uint64_t n, uint64_t nnz, uint64_t ntiles,
                const uint32_t* tile_lo, uint32_t* tile_cnt, uint64_t* tile_base,
                uint64_t* scan_tmp, uint32_t* out_col, int64_t* out_row_off, hipStream_t s);
void compact_es(const int64_t* row_off, const uint32_t* col, uint64_t thr, uint64_t seed,
                uint64_t n, uint64_t nnz, uint64_t ntiles, const uint32_t* tile_lo,
                uint32_t* tile_cnt, uint64_t* tile_base, uint64_t* scan_tmp, uint32_t* out_col,
                int64_t* out_row_off, hipStream_t s);
void write_stats(uint64_t n, uint64_t nnz, const uint64_t* counters, const uint64_t* kept,
                 slim_stats_t* st, hipStream_t s);
void validate_offsets(const int64_t* row_off, uint64_t n, uint64_t nnz, uint32_t* err,
                      hipStream_t s);
void validate_entries(const int64_t* row_off, const uint32_t* col, uint64_t n, uint64_t nnz,
                      uint64_t ntiles, const uint32_t* tile_lo, uint32_t* err, hipStream_t s);

// Every DAG row is sorted by rank id (slim_sort.hip); rows of length up to
// kSortMin by one thread each.
constexpr uint32_t kSortMin = 32;
void sort_rows(const uint2* dag_rng, uint64_t n, uint32_t* dag_col, uint32_t* lists,
               uint32_t* counts, int num_cu, hipStream_t s);

// Triangle listing + selection + deletion marks (slim_tri.hip).
struct TriArgs {
  const int64_t* row_off;
  const uint32_t* col;
  const uint32_t* rank;
  const uint32_t* order;
  const uint2* dag_rng;    // DAG row of each rank id
  const uint32_t* fstart;  // DAG row start of each original id (n+1)
  const uint32_t* dag_col;
  uint32_t* eid;       // backward CSR entries get their DAG position here
  uint32_t* del;       // deletion bitmap over DAG positions
  uint64_t* counters;  // [0] triangles, [1] selected
  uint64_t n;
  uint64_t nnz;
  uint64_t thr;
  uint32_t k0, k1;
};
uint64_t tri_tiles(uint64_t nnz);
uint64_t tri_tile_entries();
void triangles(const TriArgs& a, const uint32_t* tlo, uint32_t* tile_ctr, int num_cu,
               hipStream_t s);

// Scheduling knobs (slim_tune_set); never change results.
struct Tuning {
  int tri_chunk = 2048;
  int tri_blocks_per_cu = 2;
};
Tuning& tuning();

}  // namespace slim
