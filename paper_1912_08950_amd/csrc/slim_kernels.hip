// HIP kernels of libslim (gfx950): graph-set tiles and gather, degree-rank
// relabelling, DAG orientation, CSR compaction and per-graph stats.
//
// Data layout (all in HBM, caller-provided workspace), over the union CSR of
// the set (n vertices, nnz entries, m = nnz/2 edges):
//   rank[n], order[n]   union id -> rank id and back; rank order = (degree, id)
//   rcol[nnz]           rank id of every CSR column (streamed by the orientation)
//   dag_col[m]          rank ids of the higher-ranked neighbours, rows laid
//                       out in union-id row order (a stream compaction of CSR)
//   dag_rng[n]          (begin, end) of row x of the DAG, indexed by rank id
//   eid[nnz]            for every CSR entry of a TR graph, the DAG position of its edge
//   marks[m]            deletion marks over DAG positions, one byte per edge
//                       (set by the triangle kernels with byte stores)
//   del[m/32]           the same marks packed into a bitmap for the compaction
//   minkey[m], closed[m/32]  Edge-Once bids and closed edges over DAG positions
#include "slim_internal.h"

namespace slim {

// ------------------------------------------------------------------ fills
__global__ void k_fill_u32(uint32_t* p, uint64_t len, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < len;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_i64(int64_t* p, uint64_t len, int64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < len;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

static unsigned grid_for(uint64_t len, unsigned cap = 65536) {
  uint64_t b = (len + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (unsigned)(b < cap ? b : cap);
}

void fill_u32(uint32_t* p, uint64_t len, uint32_t v, hipStream_t s) {
  if (len) hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(len)), dim3(kBlock), 0, s, p, len, v);
}

void fill_i64(int64_t* p, uint64_t len, int64_t v, hipStream_t s) {
  if (len) hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(len)), dim3(kBlock), 0, s, p, len, v);
}

// ---------------------------------------------------- Edge-Once bids
// Start of Edge-Once round `round`: from the second round on, an edge that
// no undecided triangle bid on in the previous round is closed (every
// selected triangle on it is decided); then every bid is reset.  A wave
// takes 64 edges, so the two bitmap words of its chunk are its own.
__global__ void k_eo_clear_bids(uint64_t* minkey, uint32_t* closed, uint64_t m,
                                const uint64_t* eo_und, const uint32_t* eo_state,
                                const uint64_t* eo_list_cnt, uint32_t round) {
  if (round > 1 && eo_und[round - 1] == 0) return;  // the rounds have ended
  // a round on the lists whose previous bidders are few clears their bids
  // through their list records (k_eo_list_clear); every edge of an
  // undecided triangle got a bid then, so closing unbid edges is moot
  const uint32_t listed = eo_state[0];
  if (listed != 0 && listed < round &&
      eo_list_cnt[(round - listed - 1) & 1u] <= kEoListClearMax)
    return;
  const uint32_t lane = lane_id();
  const uint64_t waves = (uint64_t)gridDim.x * kWavesPerBlock;
  for (uint64_t c = blockIdx.x * (uint64_t)kWavesPerBlock + threadIdx.x / kWave;
       c * kWave < m; c += waves) {
    const uint64_t i = c * kWave + lane;
    bool dead = false;
    if (i < m) {
      dead = round > 1 && minkey[i] == ~0ull;
      minkey[i] = ~0ull;
    }
    const uint64_t bal = __ballot(dead);
    if (lane == 0 && bal) {
      closed[2 * c] |= (uint32_t)bal;
      closed[2 * c + 1] |= (uint32_t)(bal >> 32);
    }
  }
}

void eo_clear_bids(uint64_t* minkey, uint32_t* closed, uint64_t m, const uint64_t* eo_und,
                   const uint32_t* eo_state, const uint64_t* eo_list_cnt, uint32_t round,
                   hipStream_t s) {
  if (!m) return;
  const uint64_t chunks = (m + kWave - 1) / kWave;
  hipLaunchKernelGGL(k_eo_clear_bids, dim3(grid_for(chunks * kWave)), dim3(kBlock), 0, s, minkey,
                     closed, m, eo_und, eo_state, eo_list_cnt, round);
}

// --------------------------------------------------------- deletion marks
// Word i of the bitmap gets bit b set iff byte 32i + b of the marks is set;
// each thread reads its 32 bytes as two uint4.
__global__ __launch_bounds__(kBlock) void k_pack_marks(const uint8_t* marks, uint32_t* del,
                                                       uint64_t m) {
  const uint64_t words = (m + 31) / 32;
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * kBlock) {
    uint32_t v = 0;
    if (32 * i + 32 <= m) {
      const uint4* q = reinterpret_cast<const uint4*>(marks + 32 * i);
      const uint4 a = q[0], b = q[1];
      const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if ((w[k] >> (8 * t)) & 0xffu) v |= 1u << (4 * k + t);
    } else {
      for (uint64_t e = 32 * i; e < m; ++e)
        if (marks[e]) v |= 1u << (e - 32 * i);
    }
    del[i] = v;
  }
}

void pack_marks(const uint8_t* marks, uint32_t* del, uint64_t m, hipStream_t s) {
  if (m) hipLaunchKernelGGL(k_pack_marks, dim3(grid_for((m + 31) / 32)), dim3(kBlock), 0, s, marks,
                            del, m);
}

// ------------------------------------------------------------------- scan
// Exclusive prefix sum of TI[len] into uint64[len+1] (out[len] = total):
// per-block reduce, recursive scan of the block sums, per-block apply.
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ uint64_t block_excl_sum64(uint64_t v, uint64_t* total,
                                                     uint64_t* lds /*[kWavesPerBlock]*/) {
  const int w = threadIdx.x / kWave;
  uint64_t incl = wave_incl_sum64(v);
  if (lane_id() == kWave - 1) lds[w] = incl;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kWavesPerBlock; ++i) {
    if (i < w) before += lds[i];
    all += lds[i];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

template <typename TI>
__global__ void k_scan_reduce(const TI* in, uint64_t len, uint64_t* bsum) {
  __shared__ uint64_t lds[kWavesPerBlock];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    uint64_t i = base + (uint64_t)k * kBlock + threadIdx.x;
    if (i < len) s += (uint64_t)in[i];
  }
  uint64_t total;
  block_excl_sum64(s, &total, lds);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

template <typename TI>
__global__ void k_scan_apply(const TI* in, uint64_t len, const uint64_t* bbase, uint64_t* out) {
  __shared__ uint64_t lds[kWavesPerBlock];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    uint64_t i = base + k;
    v[k] = i < len ? (uint64_t)in[i] : 0;
    s += v[k];
  }
  uint64_t total;
  uint64_t run = block_excl_sum64(s, &total, lds) + (bbase ? bbase[blockIdx.x] : 0);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    uint64_t i = base + k;
    if (i < len) out[i] = run;
    run += v[k];
    if (i + 1 == len) out[len] = run;
  }
}

static uint64_t scan_blocks(uint64_t len) { return (len + kScanTile - 1) / kScanTile; }

uint64_t scan_tmp_elems(uint64_t len) {
  uint64_t nb = scan_blocks(len);
  if (nb <= 1) return 0;
  return 2 * nb + 2 + scan_tmp_elems(nb);
}

template <typename TI>
void scan_excl(const TI* in, uint64_t len, uint64_t* out, uint64_t* tmp, hipStream_t s) {
  if (len == 0) {
    fill_i64(reinterpret_cast<int64_t*>(out), 1, 0, s);
    return;
  }
  uint64_t nb = scan_blocks(len);
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_apply<TI>, dim3(1), dim3(kBlock), 0, s, in, len,
                       (const uint64_t*)nullptr, out);
    return;
  }
  uint64_t* bsum = tmp;
  uint64_t* bbase = tmp + nb + 1;
  hipLaunchKernelGGL(k_scan_reduce<TI>, dim3((unsigned)nb), dim3(kBlock), 0, s, in, len, bsum);
  scan_excl<uint64_t>(bsum, nb, bbase, tmp + 2 * nb + 2, s);
  hipLaunchKernelGGL(k_scan_apply<TI>, dim3((unsigned)nb), dim3(kBlock), 0, s, in, len,
                     (const uint64_t*)bbase, out);
}

template void scan_excl<uint32_t>(const uint32_t*, uint64_t, uint64_t*, uint64_t*, hipStream_t);
template void scan_excl<uint64_t>(const uint64_t*, uint64_t, uint64_t*, uint64_t*, hipStream_t);

// ------------------------------------------------------ stable radix sort
// LSD radix sort of (uint32 key, uint32 value) pairs, 8-bit digits.  The
// scatter ranks equal digits inside a wave with ballots, so the order of
// equal keys is kept (stable).
constexpr int kSortTile = kTile;

__global__ void k_radix_hist(const uint32_t* keys, uint64_t n, int shift, uint32_t nb,
                             uint32_t* hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kItems; ++k) {
    uint64_t i = base + (uint64_t)k * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_radix_scatter(const uint32_t* kin, const uint32_t* vin, uint32_t* kout,
                                uint32_t* vout, uint64_t n, int shift, uint32_t nb,
                                const uint64_t* off) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kWavesPerBlock][256];
  const int t = threadIdx.x, w = t / kWave;
  base[t] = (uint32_t)off[(uint64_t)t * nb + blockIdx.x];
#pragma unroll
  for (int i = 0; i < kWavesPerBlock; ++i) wcnt[i][t] = 0;
  __syncthreads();
  const uint64_t tile0 = (uint64_t)blockIdx.x * kSortTile;
  const uint64_t lt = lanemask_lt();
  for (int k = 0; k < kItems; ++k) {
    const uint64_t i = tile0 + (uint64_t)k * kBlock + t;
    const bool valid = i < n;
    uint32_t key = 0, val = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
    }
    const uint32_t d = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(valid && bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rnk = __popcll(peers & lt);
    if (valid && rnk == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + rnk;
      for (int i2 = 0; i2 < w; ++i2) pos += wcnt[i2][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int i2 = 0; i2 < kWavesPerBlock; ++i2) {
      add += wcnt[i2][t];
      wcnt[i2][t] = 0;
    }
    base[t] += add;
    __syncthreads();
  }
}

uint64_t sort_hist_elems(uint64_t n) {
  uint64_t nb = (n + kSortTile - 1) / kSortTile;
  return 256 * nb;
}

// Sorts (keys,vals) in buffers A by key with `passes` 8-bit passes, using B
// as the ping-pong buffer.  Returns true if the result ended in B.
bool radix_sort_pairs(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, uint64_t n,
                      int passes, uint32_t* hist, uint64_t* hist_scan, uint64_t* scan_tmp,
                      hipStream_t s) {
  const uint32_t nb = (uint32_t)((n + kSortTile - 1) / kSortTile);
  bool in_b = false;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    uint32_t* ki = in_b ? kb : ka;
    uint32_t* vi = in_b ? vb : va;
    uint32_t* ko = in_b ? ka : kb;
    uint32_t* vo = in_b ? va : vb;
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kBlock), 0, s, ki, n, shift, nb, hist);
    scan_excl<uint32_t>(hist, (uint64_t)256 * nb, hist_scan, scan_tmp, s);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kBlock), 0, s, ki, vi, ko, vo, n, shift,
                       nb, hist_scan);
    in_b = !in_b;
  }
  return in_b;
}

// ------------------------------------------------------- degree ranking
__global__ void k_deg_keys(const int64_t* row_off, uint64_t n, uint32_t* key, uint32_t* val) {
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n;
       v += (uint64_t)gridDim.x * blockDim.x) {
    key[v] = (uint32_t)(row_off[v + 1] - row_off[v]);
    val[v] = (uint32_t)v;
  }
}

__global__ void k_invert(const uint32_t* order, uint64_t n, uint32_t* rank) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n;
       x += (uint64_t)gridDim.x * blockDim.x)
    rank[order[x]] = (uint32_t)x;
}

void degree_rank(const int64_t* row_off, uint64_t n, int passes, uint32_t* ka, uint32_t* va,
                 uint32_t* kb, uint32_t* vb, uint32_t* hist, uint64_t* hist_scan,
                 uint64_t* scan_tmp, uint32_t** order_out, uint32_t* rank, hipStream_t s) {
  hipLaunchKernelGGL(k_deg_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, row_off, n, ka, va);
  bool in_b = radix_sort_pairs(ka, va, kb, vb, n, passes, hist, hist_scan, scan_tmp, s);
  uint32_t* order = in_b ? vb : va;
  hipLaunchKernelGGL(k_invert, dim3(grid_for(n)), dim3(kBlock), 0, s, order, n, rank);
  *order_out = order;
}

// --------------------------------------------------------- small writes
// Copies up to 512 bytes of host data to device memory as a kernel argument,
// so that a call can set up its descriptors without a host-to-device copy
// (and stays capturable in a HIP graph).
struct Blob {
  uint32_t w[128];
};

__global__ void k_put(uint32_t* dst, Blob b, uint32_t words) {
  if (threadIdx.x < words) dst[threadIdx.x] = b.w[threadIdx.x];
}

void put_bytes(void* dst, const void* src, uint32_t bytes, hipStream_t s) {
  Blob b{};
  __builtin_memcpy(b.w, src, bytes);
  hipLaunchKernelGGL(k_put, dim3(1), dim3(128), 0, s, static_cast<uint32_t*>(dst), b,
                     (bytes + 3) / 4);
}

// ------------------------------------------------------ CSR tile machinery
// Last graph g with tile0[g] <= t (tile0 is non-decreasing; graphs without
// tiles are skipped over).
__device__ __forceinline__ uint32_t graph_of_tile(const uint64_t* tile0, uint32_t count,
                                                  uint64_t t) {
  uint32_t lo = 0, hi = count;
  while (hi - lo > 1) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (tile0[mid] <= t)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// First union row r in [vb, ve] with row_off[r] >= j.
__device__ __forceinline__ uint32_t first_row_at(const int64_t* row_off, uint64_t vb,
                                                 uint64_t ve, int64_t j) {
  uint64_t lo = vb, hi = ve;
  while (lo < hi) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (row_off[mid] < j)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (uint32_t)lo;
}

__global__ void k_tile_recs(const int64_t* row_off, const GDesc* gd, const uint64_t* tile0,
                            uint32_t count, uint64_t ntiles, uint64_t tile, TileRec* recs) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ntiles;
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t g = graph_of_tile(tile0, count, t);
    const GDesc& G = gd[g];
    const uint64_t end = G.eb + G.ne, ve = G.vb + G.nv;
    const int64_t j0 = (int64_t)(G.eb + (t - tile0[g]) * tile);
    const uint64_t left = end > (uint64_t)j0 ? end - (uint64_t)j0 : 0;
    const uint32_t span = (uint32_t)(left < tile ? left : tile);
    const bool last = t + 1 == tile0[g + 1];
    TileRec R;
    R.j0 = j0;
    R.span = span;
    R.g = g;
    R.lo = first_row_at(row_off, G.vb, ve, j0);
    R.hi = last ? (uint32_t)ve : first_row_at(row_off, G.vb, ve, j0 + span);
    R.last = last ? 1u : 0u;
    R.pad = 0;
    recs[t] = R;
  }
}

void tile_recs(const int64_t* row_off, const GDesc* gd, const uint64_t* tile0, uint32_t count,
               uint64_t ntiles, uint64_t tile, TileRec* recs, hipStream_t s) {
  if (ntiles)
    hipLaunchKernelGGL(k_tile_recs, dim3(grid_for(ntiles)), dim3(kBlock), 0, s, row_off, gd,
                       tile0, count, ntiles, tile, recs);
}

// Union CSR of a set: block-sized chunks of each graph's row offsets
// (shifted by the graph's first entry) and columns (shifted by its first
// vertex).
__global__ __launch_bounds__(kBlock) void k_gather(const GDesc* gd, uint32_t count,
                                                   const uint64_t* vtile0,
                                                   const uint64_t* etile0, uint64_t nvt,
                                                   uint64_t net, uint64_t N, uint64_t NNZ,
                                                   int64_t* urow, uint32_t* ucol) {
  if (blockIdx.x == 0 && threadIdx.x == 0) urow[N] = (int64_t)NNZ;
  for (uint64_t t = blockIdx.x; t < nvt + net; t += gridDim.x) {
    const bool vert = t < nvt;
    const uint64_t tt = vert ? t : t - nvt;
    const uint64_t* pre = vert ? vtile0 : etile0;
    const uint32_t g = graph_of_tile(pre, count, tt);
    const GDesc& G = gd[g];
    const uint64_t i0 = (tt - pre[g]) * kTile;
    if (vert) {
      const uint64_t i1 = i0 + kTile < G.nv ? i0 + kTile : G.nv;
      for (uint64_t i = i0 + threadIdx.x; i < i1; i += kBlock)
        urow[G.vb + i] = G.in_row[i] + (int64_t)G.eb;
    } else {
      const uint64_t i1 = i0 + kTile < G.ne ? i0 + kTile : G.ne;
      const uint32_t vb = (uint32_t)G.vb;
      for (uint64_t i = i0 + threadIdx.x; i < i1; i += kBlock) ucol[G.eb + i] = G.in_col[i] + vb;
    }
  }
}

void gather(const GDesc* gd, uint32_t count, const uint64_t* vtile0, const uint64_t* etile0,
            uint64_t nvt, uint64_t net, uint64_t N, uint64_t NNZ, int64_t* urow, uint32_t* ucol,
            hipStream_t s) {
  uint64_t blocks = nvt + net;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks), dim3(kBlock), 0, s, gd, count, vtile0,
                     etile0, nvt, net, N, NNZ, urow, ucol);
}

struct TileRows {
  uint32_t srow[kTile];
  uint32_t cmax[kChunks];
};

// Fills L.srow so that the row of tile entry i is max(srow[i], cmax[i/64]).
__device__ void tile_rows(const int64_t* row_off, int64_t j0, uint32_t lo, uint32_t hi,
                          TileRows& L) {
  const int t = threadIdx.x, w = t / kWave, lane = lane_id();
  for (int i = t; i < kTile; i += kBlock) L.srow[i] = 0;
  __syncthreads();
  if (t == 0) L.srow[0] = lo > 0 ? lo - 1 : 0;
  __syncthreads();
  for (uint64_t r = lo + (uint64_t)t; r < hi; r += kBlock) {
    const int64_t b = row_off[r], e = row_off[r + 1];
    const int64_t s = b - j0;
    if (e > b && s >= 0 && s < kTile) L.srow[s] = r;
  }
  __syncthreads();
  for (int c = w; c < kChunks; c += kWavesPerBlock) {
    uint32_t v = wave_incl_max(L.srow[c * kWave + lane]);
    L.srow[c * kWave + lane] = v;
    if (lane == kWave - 1) L.cmax[c] = v;
  }
  __syncthreads();
  if (w == 0) {
    const uint32_t v = L.cmax[lane];
    const uint32_t incl = wave_incl_max(v);
    uint32_t excl = __shfl_up(incl, 1, kWave);
    if (lane == 0) excl = 0;
    L.cmax[lane] = excl;
  }
  __syncthreads();
}

__device__ __forceinline__ uint32_t tile_row_of(const TileRows& L, int i) {
  const uint32_t a = L.srow[i], b = L.cmax[i >> 6];
  return a > b ? a : b;
}

// ------------------------------------------------ flag stream compaction
// Policies decide per CSR entry j (union row r) whether it is kept and what
// is written; kept entries keep their CSR order, so rows stay sorted.  A
// policy's Ctx holds what it needs of the tile's graph.
// Orientation: keep (r,c) iff rank(c) > rank(r) and write rank(c).  The
// counting pass gathers rank(c) once per entry and streams it to rcol; the
// scatter pass and the triangle kernel read rcol instead of gathering.
struct OrientCountPolicy {
  static constexpr bool kWeights = false;
  const uint32_t* col;
  const uint32_t* rank;
  uint32_t* rcol;
  struct Ctx {};
  __device__ Ctx ctx(const GDesc&) const { return {}; }
  __device__ bool needs_rows(const GDesc&) const { return true; }
  __device__ bool flag(const Ctx&, uint64_t j, uint32_t r) const {
    const uint32_t rc = rank[col[j]];
    rcol[j] = rc;
    return rc > rank[r];
  }
  __device__ uint32_t value(const Ctx&, uint64_t j) const { return rank[col[j]]; }
};

struct OrientScatterPolicy {
  static constexpr bool kWeights = false;
  const uint32_t* rcol;
  const uint32_t* rank;
  struct Ctx {};
  __device__ Ctx ctx(const GDesc&) const { return {}; }
  __device__ bool needs_rows(const GDesc&) const { return true; }
  __device__ bool flag(const Ctx&, uint64_t j, uint32_t r) const { return rcol[j] > rank[r]; }
  __device__ uint32_t value(const Ctx&, uint64_t j) const { return rcol[j]; }
};

// Output of a compression job, per graph: a graph of a triangle operation
// keeps (r,c) iff its edge is not marked deleted; an ES graph keeps {a<b}
// (local ids) iff Philox(a,b,0,1) word 0 >= thr; a spectral sparsification
// graph keeps {a<b} iff Philox(a,b,0,2) word 0 < floor(p_ab 2^32) with
// p_ab = min(1, upsilon / min(d_a, d_b)) in double precision (section 4.2.1)
// and weighs it 1/p_ab.  Written values are local ids.
struct OutPolicy {
  static constexpr bool kWeights = true;
  const uint32_t* col;
  const uint32_t* eid;
  const uint32_t* del;
  const int64_t* row_off;
  uint64_t m;
  struct Ctx {
    uint64_t thr;
    double ups;
    uint32_t vb, k0, k1, mode;  // mode: 0 triangle ops, 1 ES, 2 spectral
  };
  __device__ Ctx ctx(const GDesc& G) const {
    return Ctx{G.thr, G.ups, (uint32_t)G.vb, G.k0, G.k1,
               G.op == SLIM_OP_ES ? 1u : (G.op == SLIM_OP_SPECTRAL ? 2u : 0u)};
  }
  __device__ bool needs_rows(const GDesc& G) const {
    return G.op == SLIM_OP_ES || G.op == SLIM_OP_SPECTRAL;
  }
  // keep probability of the spectral scheme for entry (r, col[j])
  __device__ double spectral_p(const Ctx& x, uint64_t j, uint32_t r) const {
    const uint32_t c = col[j];
    const int64_t dr = row_off[r + 1] - row_off[r], dc = row_off[c + 1] - row_off[c];
    const double pe = x.ups / (double)(dr < dc ? dr : dc);
    return pe > 1.0 ? 1.0 : pe;
  }
  __device__ bool flag(const Ctx& x, uint64_t j, uint32_t r) const {
    if (x.mode != 0) {
      const uint32_t c = col[j] - x.vb, rl = r - x.vb;
      const uint32_t a = c < rl ? c : rl, b = c < rl ? rl : c;
      uint32_t w0, w1;
      if (x.mode == 1) {
        philox_w01(a, b, 0u, 1u, x.k0, x.k1, w0, w1);
        return !((uint64_t)w0 < x.thr);
      }
      const double pe = spectral_p(x, j, r);
      const uint64_t thr = pe >= 1.0 ? (uint64_t(1) << 32) : (uint64_t)floor(pe * 4294967296.0);
      philox_w01(a, b, 0u, 2u, x.k0, x.k1, w0, w1);
      return (uint64_t)w0 < thr;
    }
    const uint32_t e = eid[j];
    return e >= m || !bit_get(del, e);  // e >= m only for inputs breaking the contract
  }
  __device__ uint32_t value(const Ctx& x, uint64_t j) const { return col[j] - x.vb; }
  __device__ float weight(const Ctx& x, uint64_t j, uint32_t r) const {
    return (float)(1.0 / spectral_p(x, j, r));
  }
};

// The count pass keeps the ballot of every 64-entry chunk (masks, 512 B per
// tile), so the scatter pass neither recomputes the flags (Philox draws,
// bitmap gathers) nor needs the rows of its entries.
template <class P>
__global__ __launch_bounds__(kBlock) void k_compact_count(P p, const int64_t* row_off,
                                                          const GDesc* gd, const TileRec* recs,
                                                          uint32_t* tile_cnt, uint64_t* masks) {
  __shared__ TileRows L;
  __shared__ uint32_t wsum[kWavesPerBlock];
  const TileRec R = recs[blockIdx.x];
  const GDesc& G = gd[R.g];
  const typename P::Ctx x = p.ctx(G);
  const bool rows = p.needs_rows(G);
  const int w = threadIdx.x / kWave, lane = lane_id();
  if (rows) tile_rows(row_off, R.j0, R.lo, R.hi, L);
  uint32_t cnt = 0;
  for (int c = w; c < kChunks; c += kWavesPerBlock) {
    const int i = c * kWave + lane;
    bool f = false;
    if ((uint32_t)i < R.span) f = p.flag(x, (uint64_t)R.j0 + i, rows ? tile_row_of(L, i) : 0u);
    const uint64_t m = __ballot(f);
    if (lane == 0) masks[(uint64_t)blockIdx.x * kChunks + c] = m;
    cnt += __popcll(m);
  }
  if (lane == 0) wsum[w] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) s += wsum[i];
    tile_cnt[blockIdx.x] = s;
  }
}

// Kept entries go to the tile's graph's output at (scan of the set) minus
// (scan at the graph's first tile); the tile also writes the row starts it
// owns and, if it is the graph's last tile, the end offset.
template <class P, typename OffT>
__global__ __launch_bounds__(kBlock) void k_compact_scatter(P p, const int64_t* row_off,
                                                            const GDesc* gd,
                                                            const uint64_t* tile0,
                                                            const TileRec* recs,
                                                            const uint64_t* tile_base,
                                                            const uint64_t* masks) {
  __shared__ TileRows L;
  __shared__ uint64_t cmask[kChunks];
  __shared__ uint32_t cbase[kChunks + 1];
  const TileRec R = recs[blockIdx.x];
  const GDesc& G = gd[R.g];
  const typename P::Ctx x = p.ctx(G);
  // rows only for the weights of spectral sparsification
  const bool rows = P::kWeights && G.out_w && G.op == SLIM_OP_SPECTRAL;
  const int w = threadIdx.x / kWave, lane = lane_id();
  if (rows) tile_rows(row_off, R.j0, R.lo, R.hi, L);
  uint32_t fbits = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    const int c = w + k * kWavesPerBlock;
    const uint64_t m = masks[(uint64_t)blockIdx.x * kChunks + c];  // the count pass's ballot
    if (lane == 0) cmask[c] = m;
    if ((m >> lane) & 1u) fbits |= 1u << k;
  }
  __syncthreads();
  if (w == 0) {
    const uint32_t v = __popcll(cmask[lane]);
    const uint64_t incl = wave_incl_sum64(v);
    cbase[lane] = (uint32_t)(incl - v);
    if (lane == kWave - 1) cbase[kChunks] = (uint32_t)incl;
  }
  __syncthreads();
  const uint64_t cap = G.cap;
  uint32_t* out = G.out_col;
  OffT* rstart = static_cast<OffT*>(G.out_row);
  const uint64_t base = tile_base[blockIdx.x] - tile_base[tile0[R.g]];
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int k = 0; k < kItems; ++k) {
    if (fbits & (1u << k)) {
      const int c = w + k * kWavesPerBlock;
      const uint64_t j = (uint64_t)R.j0 + c * kWave + lane;
      const uint64_t pos = base + cbase[c] + __popcll(cmask[c] & lt);
      if (pos < cap) {  // always true for inputs that meet the contract
        out[pos] = p.value(x, j);
        if constexpr (P::kWeights)
          if (rows) G.out_w[pos] = p.weight(x, j, tile_row_of(L, c * kWave + lane));
      }
    }
  }
  const uint32_t total = cbase[kChunks];
  for (uint64_t r = R.lo + (uint64_t)threadIdx.x; r < R.hi; r += kBlock) {
    const int64_t s = row_off[r] - R.j0;
    uint64_t v = base + total;
    if (s >= 0 && s < (int64_t)R.span) {
      const int c = (int)(s >> 6);
      v = base + cbase[c] + __popcll(cmask[c] & ((uint64_t(1) << (s & 63)) - 1));
    }
    rstart[r - G.vb] = (OffT)(v < cap ? v : cap);
  }
  if (R.last && threadIdx.x == 0) {
    const uint64_t v = base + total;
    rstart[G.nv] = (OffT)(v < cap ? v : cap);
  }
}

// Count (policy Pc), scan, scatter (policy Ps): both policies flag the same
// entries.
template <class Pc, class Ps, typename OffT>
void compact(const Pc& pc, const Ps& ps, const int64_t* row_off, const GDesc* gd,
             const uint64_t* tile0, const TileRec* recs, uint64_t ntiles, uint32_t* tile_cnt,
             uint64_t* masks, uint64_t* tile_base, uint64_t* scan_tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_compact_count<Pc>, dim3((unsigned)ntiles), dim3(kBlock), 0, s, pc,
                     row_off, gd, recs, tile_cnt, masks);
  scan_excl<uint32_t>(tile_cnt, ntiles, tile_base, scan_tmp, s);
  hipLaunchKernelGGL((k_compact_scatter<Ps, OffT>), dim3((unsigned)ntiles), dim3(kBlock), 0, s,
                     ps, row_off, gd, tile0, recs, (const uint64_t*)tile_base,
                     (const uint64_t*)masks);
}

void orient(const int64_t* row_off, const uint32_t* col, const uint32_t* rank, uint32_t* rcol,
            const GDesc* gd_union, const uint64_t* tile0, const TileRec* recs, uint64_t ntiles,
            uint32_t* tile_cnt, uint64_t* masks, uint64_t* tile_base, uint64_t* scan_tmp,
            hipStream_t s) {
  OrientCountPolicy pc{col, rank, rcol};
  OrientScatterPolicy ps{rcol, rank};
  compact<OrientCountPolicy, OrientScatterPolicy, uint32_t>(pc, ps, row_off, gd_union, tile0, recs,
                                                            ntiles, tile_cnt, masks, tile_base,
                                                            scan_tmp, s);
}

__global__ void k_dag_rng(const uint32_t* order, const uint32_t* fstart, uint64_t n,
                          uint2* dag_rng) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n;
       x += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t u = order[x];
    dag_rng[x] = make_uint2(fstart[u], fstart[u + 1]);
  }
}

void dag_ranges(const uint32_t* order, const uint32_t* fstart, uint64_t n, uint2* dag_rng,
                hipStream_t s) {
  hipLaunchKernelGGL(k_dag_rng, dim3(grid_for(n)), dim3(kBlock), 0, s, order, fstart, n,
                     dag_rng);
}

void compact_out(const int64_t* row_off, const uint32_t* col, const uint32_t* eid,
                 const uint32_t* del, uint64_t m, const GDesc* gd, const uint64_t* tile0,
                 const TileRec* recs, uint64_t ntiles, uint32_t* tile_cnt, uint64_t* masks,
                 uint64_t* tile_base, uint64_t* scan_tmp, hipStream_t s) {
  OutPolicy p{col, eid, del, row_off, m};
  compact<OutPolicy, OutPolicy, int64_t>(p, p, row_off, gd, tile0, recs, ntiles, tile_cnt, masks,
                                         tile_base, scan_tmp, s);
}

// --------------------------------------------------------------- stats
__global__ void k_stats(const GDesc* gd, uint32_t count, const uint64_t* tile0,
                        const uint64_t* counters, const uint64_t* tile_base) {
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < count;
       g += gridDim.x * blockDim.x) {
    const GDesc& G = gd[g];
    // gd[count] describes the union: its stats pointer, if set, is an array
    // of one record per graph (the per-graph copy a batch keeps)
    slim_stats_t* all = gd[count].stats;
    if (!G.stats && !all) continue;
    const uint64_t m = G.ne / 2;
    const uint64_t m_out = (tile_base[tile0[g + 1]] - tile_base[tile0[g]]) / 2;
    const bool tr = op_lists_triangles(G.op) && counters;
    slim_stats_t st;
    st.n = G.nv;
    st.m_in = m;
    st.triangles = tr ? counters[2 * g] : 0;
    st.selected = tr ? counters[2 * g + 1] : 0;
    st.deleted = m - m_out;
    st.m_out = m_out;
    if (G.stats) *G.stats = st;
    if (all) all[g] = st;
  }
}

void write_stats(const GDesc* gd, uint32_t count, const uint64_t* tile0,
                 const uint64_t* counters, const uint64_t* tile_base, hipStream_t s) {
  if (count)
    hipLaunchKernelGGL(k_stats, dim3(grid_for(count)), dim3(kBlock), 0, s, gd, count, tile0,
                       counters, tile_base);
}

// ------------------------------------------------------------ validation
// err bits: 1 offsets, 2 id >= n, 4 self-loop, 8 unsorted/duplicate, 16 asymmetric
__global__ void k_validate_offsets(const int64_t* row_off, uint64_t n, uint64_t nnz,
                                   uint32_t* err) {
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r <= n;
       r += (uint64_t)gridDim.x * blockDim.x) {
    bool bad = false;
    if (r == 0 && row_off[0] != 0) bad = true;
    if (r == n && row_off[n] != (int64_t)nnz) bad = true;
    if (r < n && row_off[r + 1] < row_off[r]) bad = true;
    if (bad) atomicOr(err, 1u);
  }
}

__global__ __launch_bounds__(kBlock) void k_validate_entries(const int64_t* row_off,
                                                             const uint32_t* col, uint64_t n,
                                                             const TileRec* recs,
                                                             uint32_t* err) {
  __shared__ TileRows L;
  const TileRec R = recs[blockIdx.x];
  tile_rows(row_off, R.j0, R.lo, R.hi, L);
  uint32_t e = 0;
  for (int i = threadIdx.x; (uint32_t)i < R.span; i += kBlock) {
    const uint64_t j = (uint64_t)R.j0 + i;
    const uint32_t r = tile_row_of(L, i);
    const uint32_t c = col[j];
    if ((uint64_t)c >= n) {
      e |= 2u;
      continue;
    }
    if (c == r) e |= 4u;
    if ((int64_t)j > row_off[r] && col[j - 1] >= c) e |= 8u;
    int64_t lo = row_off[c], hi = row_off[c + 1];
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (col[mid] < r)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (!(lo < row_off[c + 1] && col[lo] == r)) e |= 16u;
  }
  if (e) atomicOr(err, e);
}

void validate_offsets(const int64_t* row_off, uint64_t n, uint64_t nnz, uint32_t* err,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_validate_offsets, dim3(grid_for(n + 1)), dim3(kBlock), 0, s, row_off, n,
                     nnz, err);
}

void validate_entries(const int64_t* row_off, const uint32_t* col, uint64_t n,
                      const TileRec* recs, uint64_t ntiles, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_validate_entries, dim3((unsigned)ntiles), dim3(kBlock), 0, s, row_off,
                     col, n, recs, err);
}

}  // namespace slim
