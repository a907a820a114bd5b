// Accuracy metric of a compression (section 5): the Kullback-Leibler
// divergence D_KL(P||Q) = sum_k P(k) log2(P(k)/Q(k)) of the degree
// distribution Q of the compressed graph from the distribution P of its
// input, P(k) and Q(k) being the fractions of vertices of degree k.
//
// Two degree histograms (bins 0..n; LDS counters for the small degrees,
// where almost all vertices of a power-law graph fall, global atomics for
// the rest), then the sum of the terms over the bins: per block in a fixed
// tree, then the block partials in order, so the result is reproducible.
// Both phases are bound by HBM: 16 bytes of offsets per vertex, 16 bytes of
// counts per bin.
#include <math.h>

#include "slim_batch.h"

namespace slim {

constexpr int kHistLds = 4096;   // degrees below this are counted in LDS
constexpr int kKlBlocks = 1024;  // most blocks of the partial sums

__global__ __launch_bounds__(kBlock) void k_deg_hist(const int64_t* row_off, uint64_t n,
                                                     uint64_t* hist) {
  __shared__ uint32_t h[kHistLds];
  for (int i = threadIdx.x; i < kHistLds; i += kBlock) h[i] = 0;
  __syncthreads();
  for (uint64_t v = blockIdx.x * (uint64_t)kBlock + threadIdx.x; v < n;
       v += (uint64_t)gridDim.x * kBlock) {
    const int64_t d = row_off[v + 1] - row_off[v];
    uint64_t k = d > 0 ? (uint64_t)d : 0u;
    if (k > n) k = n;
    if (k < (uint64_t)kHistLds)
      atomicAdd(&h[k], 1u);
    else
      atomicAdd((unsigned long long*)&hist[k], 1ull);
  }
  __syncthreads();
  for (uint64_t i = threadIdx.x; i < (uint64_t)kHistLds && i <= n; i += kBlock)
    if (h[i]) atomicAdd((unsigned long long*)&hist[i], (unsigned long long)h[i]);
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kWavesPerBlock; ++i) t += red[i];
  __syncthreads();
  return t;
}

// Block b adds the terms of bins b*kBlock + i*stride + t; a bin present in
// P and absent from Q makes the term (and the sum) +infinity.
__global__ __launch_bounds__(kBlock) void k_kl_partial(const uint64_t* hp, const uint64_t* hq,
                                                       uint64_t bins, double inv_n,
                                                       double* part) {
  __shared__ double red[kWavesPerBlock];
  double acc = 0;
  for (uint64_t k = blockIdx.x * (uint64_t)kBlock + threadIdx.x; k < bins;
       k += (uint64_t)gridDim.x * kBlock) {
    const uint64_t cp = hp[k], cq = hq[k];
    if (cp) acc += cq ? (double)cp * inv_n * log2((double)cp / (double)cq) : __builtin_inf();
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_kl_final(const double* part, uint32_t nb,
                                                     double* out) {
  __shared__ double red[kWavesPerBlock];
  double acc = 0;
  for (uint32_t i = threadIdx.x; i < nb; i += kBlock) acc += part[i];
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) *out = t;
}

namespace {

struct KlLayout {
  uint64_t hp, hq, part, total;
};

KlLayout kl_layout(uint64_t n) {
  KlLayout L{};
  auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
  L.hp = 0;
  L.hq = al(L.hp + 8 * (n + 1));
  L.part = al(L.hq + 8 * (n + 1));
  L.total = al(L.part + 8 * (uint64_t)kKlBlocks);
  return L;
}

}  // namespace
}  // namespace slim

using namespace slim;

extern "C" {

int slim_degree_kl_workspace(uint64_t n, uint64_t* bytes) {
  if (!bytes) return fail(SLIM_EINVAL, "bytes is NULL");
  if (n > 0xffffffffull) return fail(SLIM_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
  *bytes = kl_layout(n).total;
  return ok();
}

int slim_degree_kl(const int64_t* d_row_off_p, const int64_t* d_row_off_q, uint64_t n,
                   void* d_ws, uint64_t ws_bytes, double* d_out, void* stream) {
  if (!d_out) return fail(SLIM_EINVAL, "d_out is NULL");
  if (!d_row_off_p || !d_row_off_q) return fail(SLIM_EINVAL, "row offsets are NULL");
  if (n > 0xffffffffull) return fail(SLIM_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
  const KlLayout L = kl_layout(n);
  if (ws_bytes < L.total)
    return fail(SLIM_ENOMEM, "workspace has %llu bytes, %llu needed", (unsigned long long)ws_bytes,
                (unsigned long long)L.total);
  if (!d_ws) return fail(SLIM_EINVAL, "d_ws is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(SLIM_EINVAL, "d_ws must be 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  char* ws = static_cast<char*>(d_ws);
  uint64_t* hp = reinterpret_cast<uint64_t*>(ws + L.hp);
  uint64_t* hq = reinterpret_cast<uint64_t*>(ws + L.hq);
  double* part = reinterpret_cast<double*>(ws + L.part);
  const uint64_t bins = n + 1;
  fill_u32(reinterpret_cast<uint32_t*>(hp), 2 * bins, 0, s);
  fill_u32(reinterpret_cast<uint32_t*>(hq), 2 * bins, 0, s);
  uint32_t nb = 0;
  if (n > 0) {
    uint64_t g = (n + kBlock - 1) / kBlock;
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_deg_hist, dim3((unsigned)g), dim3(kBlock), 0, s, d_row_off_p, n, hp);
    hipLaunchKernelGGL(k_deg_hist, dim3((unsigned)g), dim3(kBlock), 0, s, d_row_off_q, n, hq);
    uint64_t b = (bins + kBlock - 1) / kBlock;
    if (b > (uint64_t)kKlBlocks) b = kKlBlocks;
    nb = (uint32_t)b;
    hipLaunchKernelGGL(k_kl_partial, dim3(nb), dim3(kBlock), 0, s, hp, hq, bins,
                       1.0 / (double)n, part);
  }
  hipLaunchKernelGGL(k_kl_final, dim3(1), dim3(kBlock), 0, s, part, nb, d_out);
  return hip_check("slim_degree_kl");
}

}  // extern "C"
