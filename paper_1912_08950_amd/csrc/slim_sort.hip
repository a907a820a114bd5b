// Sorting DAG rows by rank id.
//
// The triangle kernel finds the in-neighbour edge (y,x) inside out(y) by
// binary search and scans only the part of out(y) ranked above x, which is
// the suffix of a sorted row.  Rows of length 2..kSortMin are sorted by one
// thread each (insertion sort in a private LDS slice), up to 2048 by one
// wave in registers (a bitonic network over 64 lanes x E values: pairs
// within a lane are exchanged in registers, pairs across lanes by a lane
// shuffle, so no LDS traffic and no barrier), up to 4096 by one block in
// LDS, longer rows by one block in global memory.
#include "slim_internal.h"

namespace slim {

constexpr uint32_t kWaveSortMax = 2048;
constexpr uint32_t kBlockSortMax = 4096;
constexpr uint32_t kPad = 0xffffffffu;  // larger than every rank id (n <= 2^32-1)

__device__ __forceinline__ uint32_t pow2_ceil(uint32_t v) {
  uint32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sort short rows in place (one thread each) and classify the others:
// wave_list gets rows for the wave sort, block_list for the block sort,
// huge_list for the global sort; counts[0..2] their lengths.
__global__ __launch_bounds__(kBlock) void k_sort_classify(const uint2* dag_rng, uint64_t n,
                                                          uint32_t* dag_col, uint32_t* wave_list,
                                                          uint32_t* block_list,
                                                          uint32_t* huge_list, uint32_t* counts) {
  __shared__ uint32_t slice[kBlock * (kSortMin + 1)];  // stride kSortMin+1: no bank conflicts
  uint32_t* my = slice + threadIdx.x * (kSortMin + 1);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    const uint64_t x = base + threadIdx.x;
    uint32_t len = 0, beg = 0;
    if (x < n) {
      const uint2 r = dag_rng[x];
      len = r.y - r.x;
      beg = r.x;
    }
    if (len >= 2 && len <= kSortMin) {
      for (uint32_t i = 0; i < len; ++i) {
        const uint32_t v = dag_col[beg + i];
        uint32_t k = i;
        while (k > 0 && my[k - 1] > v) {
          my[k] = my[k - 1];
          --k;
        }
        my[k] = v;
      }
      for (uint32_t i = 0; i < len; ++i) dag_col[beg + i] = my[i];
    }
    const bool cls[3] = {len > kSortMin && len <= kWaveSortMax,
                         len > kWaveSortMax && len <= kBlockSortMax, len > kBlockSortMax};
    uint32_t* lists[3] = {wave_list, block_list, huge_list};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const uint64_t bal = __ballot(cls[c]);
      if (bal == 0) continue;
      const uint32_t cnt = __popcll(bal);
      uint32_t base_idx = 0;
      const int leader = __ffsll((unsigned long long)bal) - 1;
      if ((int)lane_id() == leader) base_idx = atomicAdd(&counts[c], cnt);
      base_idx = __shfl(base_idx, leader, kWave);
      if (cls[c]) lists[c][base_idx + __popcll(bal & lanemask_lt())] = (uint32_t)x;
    }
  }
}

// Bitonic sort of one row of len <= 64 * E entries in the registers of one
// wave: element i = lane * E + r sits in register r of its lane, padded with
// kPad past len.  Step (k, j) pairs i with i ^ j; the lower index of the pair
// keeps the minimum where (i & k) == 0, the maximum elsewhere.
template <int E>
__device__ __forceinline__ void wave_sort_regs(uint32_t* row, uint32_t len) {
  const uint32_t lane = lane_id();
  uint32_t v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const uint32_t i = lane * E + r;
    v[r] = i < len ? row[i] : kPad;
  }
#pragma unroll
  for (uint32_t k = 2; k <= 64u * E; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      if (j < (uint32_t)E) {  // the pair is in this lane: registers r and r | j
#pragma unroll
        for (int r = 0; r < E; ++r) {
          if ((r & j) != 0) continue;
          const bool up = ((lane * E + r) & k) == 0;
          const uint32_t a = v[r], b = v[r | j];
          const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
          v[r] = up ? lo : hi;
          v[r | j] = up ? hi : lo;
        }
      } else {  // the partner is register r of lane ^ (j / E)
        const uint32_t lj = j / E;
        const bool lower = (lane & lj) == 0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const bool up = ((lane * E + r) & k) == 0;
          const uint32_t o = __shfl_xor(v[r], (int)lj, kWave);
          const uint32_t lo = v[r] < o ? v[r] : o, hi = v[r] < o ? o : v[r];
          v[r] = lower == up ? lo : hi;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const uint32_t i = lane * E + r;
    if (i < len) row[i] = v[r];
  }
}

// One wave per row (kSortMin < len <= 2048): the register sort with the
// fewest values per lane that holds the row.
__global__ __launch_bounds__(kBlock) void k_sort_wave(const uint2* dag_rng, uint32_t* dag_col,
                                                      const uint32_t* list,
                                                      const uint32_t* count) {
  const int w = threadIdx.x / kWave;
  const uint32_t total = *count;
  for (uint32_t i = blockIdx.x * kWavesPerBlock + w; i < total;
       i += gridDim.x * kWavesPerBlock) {
    const uint2 r = dag_rng[list[i]];
    const uint32_t len = r.y - r.x;
    uint32_t* row = dag_col + r.x;
    if (len <= 64)
      wave_sort_regs<1>(row, len);
    else if (len <= 128)
      wave_sort_regs<2>(row, len);
    else if (len <= 256)
      wave_sort_regs<4>(row, len);
    else if (len <= 512)
      wave_sort_regs<8>(row, len);
    else if (len <= 1024)
      wave_sort_regs<16>(row, len);
    else
      wave_sort_regs<32>(row, len);
  }
}

// One block per row (2048 < len <= 4096): bitonic sort in LDS.
__global__ __launch_bounds__(kBlock) void k_sort_block(const uint2* dag_rng, uint32_t* dag_col,
                                                       const uint32_t* list,
                                                       const uint32_t* count) {
  __shared__ uint32_t s[kBlockSortMax];
  const uint32_t total = *count;
  for (uint32_t i = blockIdx.x; i < total; i += gridDim.x) {
    const uint2 r = dag_rng[list[i]];
    const uint32_t len = r.y - r.x, P = pow2_ceil(len);
    for (uint32_t k = threadIdx.x; k < P; k += kBlock) s[k] = k < len ? dag_col[r.x + k] : kPad;
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t t = threadIdx.x; t < P / 2; t += kBlock) {
          const uint32_t a = ((t & ~(j - 1)) << 1) | (t & (j - 1));
          const uint32_t b = a | j;
          const bool up = (a & k) == 0;
          const uint32_t va = s[a], vb = s[b];
          if ((va > vb) == up) {
            s[a] = vb;
            s[b] = va;
          }
        }
        __syncthreads();
      }
    }
    for (uint32_t k = threadIdx.x; k < len; k += kBlock) dag_col[r.x + k] = s[k];
    __syncthreads();
  }
}

// One block per row (len > 4096): bitonic sort in place in global memory.
// Every merge is ascending (the first step of a merge pairs i with its mirror
// i ^ (k-1)), so the virtual +inf padding past `len` never moves and pairs
// that reach past the end are skipped.
__global__ __launch_bounds__(1024) void k_sort_huge(const uint2* dag_rng, uint32_t* dag_col,
                                                    const uint32_t* list,
                                                    const uint32_t* count) {
  const uint32_t total = *count;
  for (uint32_t i = blockIdx.x; i < total; i += gridDim.x) {
    const uint2 r = dag_rng[list[i]];
    uint32_t* a = dag_col + r.x;
    const uint32_t len = r.y - r.x, P = pow2_ceil(len);
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
          const uint32_t lo = ((t & ~(j - 1)) << 1) | (t & (j - 1));
          const uint32_t hi = (j == (k >> 1)) ? (lo ^ (k - 1)) : (lo | j);
          if (hi < len) {
            const uint32_t va = a[lo], vb = a[hi];
            if (va > vb) {
              a[lo] = vb;
              a[hi] = va;
            }
          }
        }
        __threadfence_block();
        __syncthreads();
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_fence(const uint32_t* dag_col, uint64_t m,
                                                  uint32_t* fence) {
  const uint64_t nq = (m + kFenceStep - 1) / kFenceStep;
  for (uint64_t q = blockIdx.x * (uint64_t)kBlock + threadIdx.x; q < nq;
       q += (uint64_t)gridDim.x * kBlock)
    fence[q] = dag_col[q * kFenceStep];
}

void fence_samples(const uint32_t* dag_col, uint64_t m, uint32_t* fence, hipStream_t s) {
  const uint64_t nq = (m + kFenceStep - 1) / kFenceStep;
  if (nq == 0) return;
  uint64_t g = (nq + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_fence, dim3((unsigned)g), dim3(kBlock), 0, s, dag_col, m, fence);
}

void sort_rows(const uint2* dag_rng, uint64_t n, uint32_t* dag_col, uint32_t* lists,
               uint32_t* counts, int num_cu, hipStream_t s) {
  fill_u32(counts, 4, 0, s);
  uint32_t* wave_list = lists;
  uint32_t* block_list = lists + n;
  uint32_t* huge_list = lists + 2 * n;
  unsigned g = (unsigned)((n + kBlock - 1) / kBlock);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_sort_classify, dim3(g), dim3(kBlock), 0, s, dag_rng, n, dag_col,
                     wave_list, block_list, huge_list, counts);
  hipLaunchKernelGGL(k_sort_wave, dim3(num_cu * 8), dim3(kBlock), 0, s, dag_rng, dag_col,
                     wave_list, counts + 0);
  hipLaunchKernelGGL(k_sort_block, dim3(num_cu * 4), dim3(kBlock), 0, s, dag_rng, dag_col,
                     block_list, counts + 1);
  hipLaunchKernelGGL(k_sort_huge, dim3(num_cu), dim3(1024), 0, s, dag_rng, dag_col, huge_list,
                     counts + 2);
}

}  // namespace slim
