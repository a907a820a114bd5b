// Triangle listing with selection and deletion marks (Triangle p-1-Reduction,
// section 4.3: every triangle of the input graph runs kernel `p-1-reduction`
// once; a selected triangle deletes one uniformly chosen edge).
//
// Each triangle {y,x,w} with rank(y) < rank(x) < rank(w) is found exactly
// once, from its middle vertex x: w lies in out(x) (kept in an LDS hash
// table) and in out(y) for an in-neighbour y of x (scanned from the DAG).
// The DAG position of every edge of the triangle is known at that point, so
// the deletion is an idempotent atomic OR into a bitmap over DAG positions.
// Selection uses only the id-sorted triple, so the result does not depend
// on the order in which triangles are found.
#include "slim_internal.h"

namespace slim {

constexpr int kHashSlots = 4096;  // LDS hash table capacity; out(x) is hashed in
                                  // passes of at most `chunk` <= kHashSlots/2 entries
constexpr uint32_t kEmpty = 0xffffffffu;

__device__ __forceinline__ uint32_t hslot(uint32_t w, int lg) {
  return (w * 0x9E3779B1u) >> (32 - lg);
}

__global__ __launch_bounds__(kBlock) void k_triangles_v1(TriArgs a, uint32_t kChunkMax) {
  __shared__ uint32_t hkey[kHashSlots];
  __shared__ uint32_t hpos[kHashSlots];
  __shared__ uint32_t hold[kHashSlots];
  __shared__ uint64_t red[2][kWavesPerBlock];
  const int tid = threadIdx.x;
  uint64_t n_tri = 0, n_sel = 0;
  for (uint64_t x = blockIdx.x; x < a.n; x += gridDim.x) {
    const uint32_t u0 = a.order[x];
    const int64_t rb = a.row_off[u0], re = a.row_off[u0 + 1];
    if (re == rb) continue;  // isolated vertex (block-uniform)
    const uint2 xr = a.dag_rng[x];
    const uint32_t ox = xr.y - xr.x;
    for (uint32_t c0 = 0; c0 == 0 || c0 < ox; c0 += kChunkMax) {
      const uint32_t clen = ox - c0 < kChunkMax ? ox - c0 : kChunkMax;
      int lg = 6;
      while ((1u << lg) < 2 * clen) ++lg;
      const uint32_t mask = (1u << lg) - 1;
      for (uint32_t i = tid; i <= mask; i += kBlock) hkey[i] = kEmpty;
      __syncthreads();
      for (uint32_t k = tid; k < clen; k += kBlock) {
        const uint32_t w = a.dag_col[xr.x + c0 + k];
        uint32_t slot = hslot(w, lg);
        while (atomicCAS(&hkey[slot], kEmpty, w) != kEmpty) slot = (slot + 1) & mask;
        hpos[slot] = c0 + k;
        hold[slot] = a.order[w];
      }
      __syncthreads();
      for (int64_t j = rb + tid; j < re; j += kBlock) {
        const uint32_t c = a.col[j];
        const uint32_t y = a.rank[c];
        if (y >= x) continue;  // forward entry: not an in-edge of x
        const uint2 yr = a.dag_rng[y];
        uint32_t e_yx = kEmpty;
        bool del_yx = false;
        for (uint32_t i = yr.x; i < yr.y; ++i) {
          const uint32_t w = a.dag_col[i];
          if (w == x) {
            e_yx = i;
            continue;
          }
          if (w < x || clen == 0) continue;
          uint32_t slot = hslot(w, lg), hk;
          for (;;) {
            hk = hkey[slot];
            if (hk == w || hk == kEmpty) break;
            slot = (slot + 1) & mask;
          }
          if (hk != w) continue;
          // triangle {c, u0, ow} in original ids
          const uint32_t ow = hold[slot];
          const uint32_t kpos = hpos[slot];
          ++n_tri;
          uint32_t t0 = c, t1 = u0, t2 = ow;
          sort3(t0, t1, t2);
          uint32_t w0, w1;
          philox_w01(t0, t1, t2, 0u, a.k0, a.k1, w0, w1);
          if ((uint64_t)w0 < a.thr) {
            ++n_sel;
            const uint32_t kk = __umulhi(w1, 3u);  // 0:{t0,t1} 1:{t0,t2} 2:{t1,t2}
            const uint32_t excl = kk == 0 ? t2 : (kk == 1 ? t1 : t0);
            if (excl == ow)
              del_yx = true;  // edge {c,u0} = (y,x)
            else if (excl == u0)
              bit_set(a.del, i);  // edge {c,ow} = (y,w)
            else
              bit_set(a.del, xr.x + kpos);  // edge {u0,ow} = (x,w)
          }
        }
        if (c0 == 0) a.eid[j] = e_yx;
        if (del_yx && e_yx != kEmpty) bit_set(a.del, e_yx);
      }
      __syncthreads();
    }
  }
  const int w = tid / kWave;
  n_tri = wave_sum64(n_tri);
  n_sel = wave_sum64(n_sel);
  if (lane_id() == 0) {
    red[0][w] = n_tri;
    red[1][w] = n_sel;
  }
  __syncthreads();
  if (tid == 0) {
    uint64_t s0 = 0, s1 = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
      s0 += red[0][i];
      s1 += red[1][i];
    }
    if (s0) atomicAdd((unsigned long long*)&a.counters[0], (unsigned long long)s0);
    if (s1) atomicAdd((unsigned long long*)&a.counters[1], (unsigned long long)s1);
  }
}

void triangles(const TriArgs& a, int num_cu, hipStream_t s) {
  const Tuning& t = tuning();
  uint64_t blocks = (uint64_t)num_cu * t.tri_blocks_per_cu;
  if (blocks > a.n) blocks = a.n;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_triangles_v1, dim3((unsigned)blocks), dim3(kBlock), 0, s, a,
                     (uint32_t)t.tri_chunk);
}

}  // namespace slim
