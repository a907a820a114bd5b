// Accuracy metrics of a compression (section 5): the Kullback-Leibler
// divergence D_KL(P||Q) = sum_k P(k) log2(P(k)/Q(k)) of the degree
// distribution Q of the compressed graph from the distribution P of its
// input, P(k) and Q(k) being the fractions of vertices of degree k; and
// PageRank with the divergence of two score vectors (Table `tab:pr-KL`
// compares the PageRank distributions of original and compressed graphs).
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

// ---------------------------------------------------------------- PageRank
// Jacobi iteration x' = (1-d)/n + d * sum over neighbours u of x(u)/deg(u)
// from x = 1/n; a vertex without edges passes nothing on.  A wave takes 64
// consecutive vertices: each lane sums the neighbours of its own vertex if
// it has at most kPrLight of them, and the wave sums every longer row
// together (lane l takes entries l, l+64, ..., then a fixed-order tree), so
// hubs do not serialise one lane and every sum has a fixed order.  The
// kernel writes x' and the next contributions x'(v)/deg(v).
constexpr uint32_t kPrLight = 64;

__global__ __launch_bounds__(kBlock) void k_pr_init(const int64_t* row_off, uint64_t n,
                                                    double* x, double* contrib) {
  for (uint64_t v = blockIdx.x * (uint64_t)kBlock + threadIdx.x; v < n;
       v += (uint64_t)gridDim.x * kBlock) {
    const int64_t d = row_off[v + 1] - row_off[v];
    const double xv = 1.0 / (double)n;
    x[v] = xv;
    contrib[v] = d > 0 ? xv / (double)d : 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_pr_step(const int64_t* row_off, const uint32_t* col,
                                                    uint64_t n, double base, double damp,
                                                    const double* contrib, double* x_out,
                                                    double* contrib_out) {
  const uint32_t lane = lane_id();
  const uint64_t waves = (uint64_t)gridDim.x * kWavesPerBlock;
  for (uint64_t g = blockIdx.x * (uint64_t)kWavesPerBlock + threadIdx.x / kWave; g * kWave < n;
       g += waves) {
    const uint64_t v = g * kWave + lane;
    int64_t b = 0, e = 0;
    if (v < n) {
      b = row_off[v];
      e = row_off[v + 1];
    }
    const bool heavy = e - b > (int64_t)kPrLight;
    double acc = 0.0;
    if (!heavy)
      for (int64_t j = b; j < e; ++j) acc += contrib[col[j]];
    uint64_t hm = __ballot(heavy);
    while (hm) {  // rows longer than kPrLight, one at a time by the whole wave
      const int src = __builtin_ctzll(hm);
      hm &= hm - 1;
      const int64_t hb = __shfl(b, src, kWave), he = __shfl(e, src, kWave);
      double part = 0.0;
      for (int64_t j = hb + lane; j < he; j += kWave) part += contrib[col[j]];
      for (int d = kWave / 2; d > 0; d >>= 1) part += __shfl_xor(part, d, kWave);
      if ((int)lane == src) acc = part;
    }
    if (v < n) {
      const double xv = base + damp * acc;
      x_out[v] = xv;
      contrib_out[v] = e > b ? xv / (double)(e - b) : 0.0;
    }
  }
}

// sum_i P(i) log2(P(i)/Q(i)) with P = p / sum p, Q = q / sum q: block
// partials of the two sums, then of the terms, each in a fixed order.
__global__ __launch_bounds__(kBlock) void k_sum_partial(const double* a, const double* b,
                                                        uint64_t n, double* part) {
  __shared__ double red[kWavesPerBlock];
  double sa = 0, sb = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock) {
    sa += a[i];
    sb += b[i];
  }
  const double ta = block_sum(sa, red);
  const double tb = block_sum(sb, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ta;
    part[2 * blockIdx.x + 1] = tb;
  }
}

__global__ __launch_bounds__(kBlock) void k_sum_final(const double* part, uint32_t nb,
                                                      double* sums) {
  __shared__ double red[kWavesPerBlock];
  double sa = 0, sb = 0;
  for (uint32_t i = threadIdx.x; i < nb; i += kBlock) {
    sa += part[2 * i];
    sb += part[2 * i + 1];
  }
  const double ta = block_sum(sa, red);
  const double tb = block_sum(sb, red);
  if (threadIdx.x == 0) {
    sums[0] = ta;
    sums[1] = tb;
  }
}

__global__ __launch_bounds__(kBlock) void k_vec_kl_partial(const double* p, const double* q,
                                                           uint64_t n, const double* sums,
                                                           double* part) {
  __shared__ double red[kWavesPerBlock];
  const double ip = 1.0 / sums[0], iq = 1.0 / sums[1];
  double acc = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock) {
    const double pi = p[i] * ip, qi = q[i] * iq;
    if (pi > 0) acc += qi > 0 ? pi * log2(pi / qi) : __builtin_inf();
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
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

struct PrLayout {
  uint64_t x1, c0, c1, total;
};

PrLayout pr_layout(uint64_t n) {
  PrLayout L{};
  auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
  L.x1 = 0;
  L.c0 = al(L.x1 + 8 * n);
  L.c1 = al(L.c0 + 8 * n);
  L.total = al(L.c1 + 8 * n);
  return L;
}

uint64_t vec_kl_bytes() { return (uint64_t)(3 * kKlBlocks + 2) * 8; }

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

int slim_pagerank_workspace(uint64_t n, uint64_t* bytes) {
  if (!bytes) return fail(SLIM_EINVAL, "bytes is NULL");
  if (n > 0xffffffffull) return fail(SLIM_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
  *bytes = pr_layout(n).total;
  return ok();
}

int slim_pagerank(const int64_t* d_row_off, const uint32_t* d_col, uint64_t n, double damping,
                  uint32_t iters, void* d_ws, uint64_t ws_bytes, double* d_pr, void* stream) {
  if (!d_pr && n) return fail(SLIM_EINVAL, "d_pr is NULL");
  if (!d_row_off && n) return fail(SLIM_EINVAL, "d_row_off is NULL");
  if (n > 0xffffffffull) return fail(SLIM_EINVAL, "n = %llu exceeds 2^32-1", (unsigned long long)n);
  if (!(damping >= 0.0 && damping <= 1.0))
    return fail(SLIM_EINVAL, "damping must lie in [0, 1]");
  const PrLayout L = pr_layout(n);
  if (ws_bytes < L.total)
    return fail(SLIM_ENOMEM, "workspace has %llu bytes, %llu needed", (unsigned long long)ws_bytes,
                (unsigned long long)L.total);
  if (n == 0) return ok();
  if (!d_ws) return fail(SLIM_EINVAL, "d_ws is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(SLIM_EINVAL, "d_ws must be 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  char* ws = static_cast<char*>(d_ws);
  double* xb[2] = {d_pr, reinterpret_cast<double*>(ws + L.x1)};
  double* cb[2] = {reinterpret_cast<double*>(ws + L.c0), reinterpret_cast<double*>(ws + L.c1)};
  // the last step writes d_pr: start from the buffer that makes it so
  int cur = iters % 2 == 0 ? 0 : 1;
  uint64_t g = (n + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_pr_init, dim3((unsigned)g), dim3(kBlock), 0, s, d_row_off, n, xb[cur],
                     cb[cur]);
  uint64_t gw = (n + kBlock - 1) / kBlock;
  if (gw > 16384) gw = 16384;
  const double base = (1.0 - damping) / (double)n;
  for (uint32_t it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(k_pr_step, dim3((unsigned)gw), dim3(kBlock), 0, s, d_row_off, d_col, n,
                       base, damping, cb[cur], xb[1 - cur], cb[1 - cur]);
    cur = 1 - cur;
  }
  return hip_check("slim_pagerank");
}

int slim_kl_divergence_workspace(uint64_t n, uint64_t* bytes) {
  if (!bytes) return fail(SLIM_EINVAL, "bytes is NULL");
  (void)n;
  *bytes = vec_kl_bytes();
  return ok();
}

int slim_kl_divergence(const double* d_p, const double* d_q, uint64_t n, void* d_ws,
                       uint64_t ws_bytes, double* d_out, void* stream) {
  if (!d_out) return fail(SLIM_EINVAL, "d_out is NULL");
  if (n && (!d_p || !d_q)) return fail(SLIM_EINVAL, "d_p or d_q is NULL");
  if (ws_bytes < vec_kl_bytes())
    return fail(SLIM_ENOMEM, "workspace has %llu bytes, %llu needed", (unsigned long long)ws_bytes,
                (unsigned long long)vec_kl_bytes());
  if (!d_ws) return fail(SLIM_EINVAL, "d_ws is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(SLIM_EINVAL, "d_ws must be 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  double* part = static_cast<double*>(d_ws);        // 2 * kKlBlocks sums, then kKlBlocks terms
  double* terms = part + 2 * kKlBlocks;
  double* sums = terms + kKlBlocks;
  uint32_t nb = 0;
  if (n) {
    uint64_t b = (n + kBlock - 1) / kBlock;
    if (b > (uint64_t)kKlBlocks) b = kKlBlocks;
    nb = (uint32_t)b;
    hipLaunchKernelGGL(k_sum_partial, dim3(nb), dim3(kBlock), 0, s, d_p, d_q, n, part);
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, part, nb, sums);
    hipLaunchKernelGGL(k_vec_kl_partial, dim3(nb), dim3(kBlock), 0, s, d_p, d_q, n, sums, terms);
  }
  hipLaunchKernelGGL(k_kl_final, dim3(1), dim3(kBlock), 0, s, terms, nb, d_out);
  return hip_check("slim_kl_divergence");
}

}  // extern "C"
