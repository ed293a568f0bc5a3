// Pruning of the configuration space on the GPU (sections 3.4, 4.1 and 4.2 of
// the paper): normalize the benchmark table, cluster its rows with k-means
// and turn each centroid into one deployed configuration.
//
// Everything is integer so that any correct implementation reaches the same
// bits: Q16 normalized values, exact int64 squared distances and sums,
// rounded-mean centroids floor((2*sum + n_j) / (2*n_j)), lowest index on every
// tie.  k-means++ initialisation draws from a SplitMix64 stream seeded with
// seed + restart.  One work-group runs one restart; restarts run in parallel.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "kt_internal.hpp"

namespace kt {

static constexpr int Q16 = 65535;
static constexpr int STD_LO = 58982;   // ceil(0.9 * 65535)

// ----------------------------------------------------------- normalization

// One work-group per row: t_best = smallest positive time of the row, then
// q = floor((2*65535*t_best + t) / (2*t)) and the chosen variant.
__global__ void __launch_bounds__(256)
normalize_kernel(const int64_t* __restrict__ T, int32_t n_cfg, int32_t norm,
                 const uint16_t* __restrict__ lut, uint16_t* __restrict__ out) {
  const int64_t row = blockIdx.x;
  const int64_t* t = T + row * n_cfg;
  __shared__ int64_t red[256];
  int64_t best = INT64_MAX;
  for (int c = threadIdx.x; c < n_cfg; c += blockDim.x) {
    const int64_t v = t[c];
    if (v > 0 && v < best) best = v;
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && red[threadIdx.x + s] < red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  best = red[0];
  for (int c = threadIdx.x; c < n_cfg; c += blockDim.x) {
    const int64_t v = t[c];
    int64_t q = 0;
    if (v > 0 && best != INT64_MAX) q = (2 * (int64_t)Q16 * best + v) / (2 * v);
    if (norm == KT_NORM_RAWCUT) {
      if (10 * q < 9 * (int64_t)Q16) q = 0;
    } else if (norm == KT_NORM_STDCUT) {
      if (10 * q < 9 * (int64_t)Q16) q = 0;
      else {
        const int64_t num = (q - STD_LO) * Q16, den = Q16 - STD_LO;
        q = (2 * num + den) / (2 * den);
      }
    } else if (norm == KT_NORM_SIGMOID) {
      q = lut[q];
    }
    out[row * n_cfg + c] = (uint16_t)q;
  }
}

const std::vector<uint16_t>& sigmoid_table(Ctx* h) {
  if (h->sigmoid_lut.empty()) {
    h->sigmoid_lut.resize(Q16 + 1);
    for (int v = 0; v <= Q16; ++v) {
      const double f = (double)Q16 / (1.0 + exp(50.0 * (0.85 - (double)v / Q16)));
      h->sigmoid_lut[v] = (uint16_t)floor(f + 0.5);
    }
  }
  return h->sigmoid_lut;
}

// ------------------------------------------------------------------ k-means

static constexpr int KM_THREADS = 1024;
static constexpr int KM_MAX_ROWS = 4096;
static constexpr int KM_MAX_KD = 8192;      // k * d int64 centroids in LDS

struct KmeansOut {      // per restart, in the workspace
  int64_t inertia;
  int32_t iterations;
  int32_t pad;
};

__device__ __forceinline__ uint64_t sm64_next(uint64_t& state) {
  uint64_t z = state + 0x9E3779B97F4A7C15ull;
  state = z;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Block-wide argmax of val[i] over i < n, lowest index on ties.
__device__ void block_argmax(const int64_t* val, int n, int64_t* s_val, int32_t* s_idx,
                             int64_t& out_val, int32_t& out_idx) {
  const int tid = threadIdx.x;
  int64_t bv = INT64_MIN;
  int32_t bi = INT32_MAX;
  for (int i = tid; i < n; i += KM_THREADS) {
    if (val[i] > bv) { bv = val[i]; bi = i; }   // ascending i: first max kept
  }
  s_val[tid] = bv;
  s_idx[tid] = bi;
  __syncthreads();
  for (int s = KM_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s) {
      const int64_t ov = s_val[tid + s];
      const int32_t oi = s_idx[tid + s];
      if (ov > s_val[tid] || (ov == s_val[tid] && oi < s_idx[tid])) { s_val[tid] = ov; s_idx[tid] = oi; }
    }
    __syncthreads();
  }
  out_val = s_val[0];
  out_idx = s_idx[0];
  __syncthreads();
}

__device__ int64_t block_sum(int64_t v, int64_t* s_val) {
  const int tid = threadIdx.x;
  s_val[tid] = v;
  __syncthreads();
  for (int s = KM_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s) s_val[tid] += s_val[tid + s];
    __syncthreads();
  }
  const int64_t r = s_val[0];
  __syncthreads();
  return r;
}

// Squared distance between row i of X and centroid c (int64 values).
__device__ __forceinline__ int64_t sqdist_row(const uint16_t* __restrict__ X, int d, int i,
                                              const int64_t* c) {
  const uint16_t* x = X + (int64_t)i * d;
  int64_t s = 0;
  for (int f = 0; f < d; ++f) {
    const int64_t df = (int64_t)x[f] - c[f];
    s += df * df;
  }
  return s;
}

// One restart per work-group.  Outputs in global memory: centroids
// [restart][k][d], labels [restart][n], KmeansOut [restart].
__global__ void __launch_bounds__(KM_THREADS)
kmeans_kernel(const uint16_t* __restrict__ X, int n, int d, int k, uint64_t seed, int max_iter,
              int64_t* __restrict__ g_cent, int32_t* __restrict__ g_labels,
              KmeansOut* __restrict__ g_out) {
  extern __shared__ int64_t smem[];
  int64_t* C = smem;                                  // [k][d]
  int64_t* dist = C + (int64_t)k * d;                 // [n]
  int64_t* s_val = dist + n;                          // [KM_THREADS]
  int32_t* labels = (int32_t*)(s_val + KM_THREADS);   // [n]
  int32_t* counts = labels + n;                       // [k]
  int32_t* s_idx = counts + k;                        // [KM_THREADS]
  __shared__ int32_t s_flag;
  __shared__ int32_t s_pick;
  __shared__ int32_t s_centres[64];

  const int tid = threadIdx.x;
  const int r = blockIdx.x;
  uint64_t state = seed + (uint64_t)r;   // thread 0 owns the stream

  // ---- k-means++ initialisation
  if (tid == 0) {
    const uint64_t draw = sm64_next(state);
    s_pick = (int)(draw % (uint64_t)n);
    s_centres[0] = s_pick;
  }
  __syncthreads();
  for (int f = tid; f < d; f += KM_THREADS) C[f] = X[(int64_t)s_pick * d + f];
  __syncthreads();
  for (int i = tid; i < n; i += KM_THREADS) dist[i] = sqdist_row(X, d, i, C);
  __syncthreads();
  for (int c = 1; c < k; ++c) {
    // Prefix search: each thread owns a contiguous chunk of rows.
    const int chunk = (n + KM_THREADS - 1) / KM_THREADS;
    const int lo = tid * chunk, hi = min(n, lo + chunk);
    int64_t part = 0;
    for (int i = lo; i < hi; ++i) part += dist[i];
    s_val[tid] = part;
    __syncthreads();
    if (tid == 0) {
      int64_t S = 0;
      for (int t = 0; t < KM_THREADS; ++t) S += s_val[t];
      const uint64_t draw = sm64_next(state);
      int pick = -1;
      if (S == 0) {
        for (int i = 0; i < n && pick < 0; ++i) {
          bool used = false;
          for (int j = 0; j < c; ++j) used = used || (s_centres[j] == i);
          if (!used) pick = i;
        }
      } else {
        const int64_t rr = (int64_t)(draw % (uint64_t)S);
        int64_t run = 0;
        int t = 0;
        while (t < KM_THREADS && run + s_val[t] <= rr) { run += s_val[t]; ++t; }
        for (int i = t * chunk; i < n; ++i) {
          run += dist[i];
          if (run > rr) { pick = i; break; }
        }
      }
      if (pick < 0) pick = 0;   // unreachable for 1 <= k <= n; keeps the index in range
      s_pick = pick;
      s_centres[c] = pick;
    }
    __syncthreads();
    int64_t* Cc = C + (int64_t)c * d;
    for (int f = tid; f < d; f += KM_THREADS) Cc[f] = X[(int64_t)s_pick * d + f];
    __syncthreads();
    for (int i = tid; i < n; i += KM_THREADS) {
      const int64_t v = sqdist_row(X, d, i, Cc);
      if (v < dist[i]) dist[i] = v;
    }
    __syncthreads();
  }

  // ---- Lloyd iterations
  for (int i = tid; i < n; i += KM_THREADS) labels[i] = -1;
  __syncthreads();
  int it = 0;
  bool converged = false;
  for (;;) {
    // assignment: nearest centroid, lowest index on ties
    if (tid == 0) s_flag = 0;
    __syncthreads();
    int changed = 0;
    for (int i = tid; i < n; i += KM_THREADS) {
      int64_t bd = INT64_MAX;
      int bj = 0;
      for (int j = 0; j < k; ++j) {
        const int64_t v = sqdist_row(X, d, i, C + (int64_t)j * d);
        if (v < bd) { bd = v; bj = j; }
      }
      dist[i] = bd;
      if (labels[i] != bj) changed = 1;
      labels[i] = bj;
    }
    if (changed) atomicOr(&s_flag, 1);
    __syncthreads();
    if (s_flag == 0 && it > 0) { converged = true; break; }
    if (it >= max_iter) break;   // labels/dist already reflect the final centroids
    // update: per-dimension sums into C (C is not needed after the assignment)
    for (int j = tid; j < k; j += KM_THREADS) counts[j] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += KM_THREADS) atomicAdd(&counts[labels[i]], 1);
    for (int64_t e = tid; e < (int64_t)k * d; e += KM_THREADS) C[e] = 0;
    __syncthreads();
    for (int f = tid; f < d; f += KM_THREADS) {
      for (int i = 0; i < n; ++i) C[(int64_t)labels[i] * d + f] += X[(int64_t)i * d + f];
    }
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)k * d; e += KM_THREADS) {
      const int64_t nj = counts[e / d];
      if (nj > 0) C[e] = (2 * C[e] + nj) / (2 * nj);
    }
    __syncthreads();
    // empty clusters take the farthest row (lowest index on ties); its distance is zeroed
    for (int j = 0; j < k; ++j) {
      if (counts[j] != 0) continue;
      int64_t fv;
      int32_t fi;
      block_argmax(dist, n, s_val, s_idx, fv, fi);
      for (int f = tid; f < d; f += KM_THREADS) C[(int64_t)j * d + f] = X[(int64_t)fi * d + f];
      __syncthreads();
      if (tid == 0) dist[fi] = 0;
      __syncthreads();
    }
    ++it;
  }
  (void)converged;
  int64_t part = 0;
  for (int i = tid; i < n; i += KM_THREADS) part += dist[i];
  const int64_t inertia = block_sum(part, s_val);
  for (int64_t e = tid; e < (int64_t)k * d; e += KM_THREADS) g_cent[(int64_t)r * k * d + e] = C[e];
  for (int i = tid; i < n; i += KM_THREADS) g_labels[(int64_t)r * n + i] = labels[i];
  if (tid == 0) {
    g_out[r].inertia = inertia;
    g_out[r].iterations = it;
  }
}

// Pick the winning restart (lowest inertia, lowest restart on ties) and map
// its centroids to k distinct configurations: centroid j takes its largest
// coordinate (lowest configuration on ties) among those not yet chosen.
__global__ void choose_kernel(const int64_t* __restrict__ g_cent, const KmeansOut* __restrict__ g_out,
                              int n_init, int k, int d, int32_t* __restrict__ chosen,
                              int32_t* __restrict__ best_restart) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int br = 0;
  for (int r = 1; r < n_init; ++r)
    if (g_out[r].inertia < g_out[br].inertia) br = r;
  *best_restart = br;
  const int64_t* C = g_cent + (int64_t)br * k * d;
  for (int j = 0; j < k; ++j) {
    int best = -1;
    for (int f = 0; f < d; ++f) {
      bool used = false;
      for (int q = 0; q < j; ++q) used = used || (chosen[q] == f);
      if (used) continue;
      if (best < 0 || C[(int64_t)j * d + f] > C[(int64_t)j * d + best]) best = f;
    }
    chosen[j] = best;
  }
}

static size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

struct PrunePlan {
  size_t off_T, off_X, off_cent, off_lab, off_out, off_chosen, total;
};

static PrunePlan prune_plan(int32_t n, int32_t d, int32_t k, int32_t n_init) {
  PrunePlan p;
  p.off_T = 0;
  p.off_X = a256(p.off_T + (size_t)n * d * 8);
  p.off_cent = a256(p.off_X + (size_t)n * d * 2);
  p.off_lab = a256(p.off_cent + (size_t)n_init * k * d * 8);
  p.off_out = a256(p.off_lab + (size_t)n_init * n * 4);
  p.off_chosen = a256(p.off_out + (size_t)n_init * sizeof(KmeansOut));
  p.total = a256(p.off_chosen + (size_t)(k + 1) * 4);
  return p;
}

static size_t kmeans_lds_bytes(int n, int d, int k) {
  return (size_t)k * d * 8 + (size_t)n * 8 + KM_THREADS * 8 + (size_t)n * 4 + (size_t)k * 4 +
         KM_THREADS * 4;
}

static kt_status check_table(Ctx* h, int32_t n, int32_t d) {
  if (n < 1 || d < 1) return fail(h, KT_EINVAL, "empty time table");
  return KT_OK;
}

// Upload a host table and normalize it into the workspace (shared by prune and Top-N).
static kt_status ensure_lut(Ctx* h, hipStream_t st);

static kt_status upload_normalize(Ctx* h, const int64_t* time_ns, int32_t n, int32_t d, kt_norm norm,
                                  char* ws, const PrunePlan& p, hipStream_t st) {
  kt_status s = ensure_lut(h, st);
  if (s != KT_OK) return s;
  hipError_t e = hipMemcpyAsync(ws + p.off_T, time_ns, (size_t)n * d * 8, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(h, e, "upload time table");
  hipLaunchKernelGGL(normalize_kernel, dim3(n), dim3(256), 0, st, (const int64_t*)(ws + p.off_T), d,
                     (int32_t)norm, (const uint16_t*)h->d_lut, (uint16_t*)(ws + p.off_X));
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "normalize launch");
  return KT_OK;
}

// Device copy of the sigmoid table, owned by the handle (128 KiB, made once).
static kt_status ensure_lut(Ctx* h, hipStream_t st) {
  if (h->d_lut) return KT_OK;
  const std::vector<uint16_t>& lut = sigmoid_table(h);
  hipError_t e = hipMalloc(&h->d_lut, lut.size() * 2);
  if (e != hipSuccess) { h->d_lut = nullptr; return hip_fail(h, e, "hipMalloc sigmoid table"); }
  e = hipMemcpyAsync(h->d_lut, lut.data(), lut.size() * 2, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(h, e, "upload sigmoid table");
  return KT_OK;
}

kt_status normalize_table_host(Ctx* h, const int64_t* time_ns, int32_t n, int32_t d, kt_norm norm,
                               void* workspace, size_t ws_bytes, hipStream_t st, uint16_t* out) {
  if (!need_device(h)) return KT_EINVAL;
  kt_status s = check_table(h, n, d);
  if (s != KT_OK) return s;
  if ((int)norm < 0 || (int)norm > 3) return fail(h, KT_EINVAL, "bad normalization");
  const PrunePlan p = prune_plan(n, d, 1, 1);
  if (!workspace || ws_bytes < p.total) return fail(h, KT_EWORKSPACE, "normalization workspace too small");
  s = upload_normalize(h, time_ns, n, d, norm, (char*)workspace, p, st);
  if (s != KT_OK) return s;
  hipError_t e = hipMemcpyAsync(out, (char*)workspace + p.off_X, (size_t)n * d * 2,
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(h, e, "read normalized table");
  return KT_OK;
}

}  // namespace kt

using namespace kt;

extern "C" {

kt_status kt_normalize(kt_handle hh, const int64_t* d_time, int32_t n_rows, int32_t n_configs,
                       kt_norm norm, uint16_t* d_out, void* stream) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (n_rows < 0 || n_configs < 0) return fail(h, KT_EINVAL, "negative size");
  if ((int)norm < 0 || (int)norm > 3) return fail(h, KT_EINVAL, "bad normalization");
  if (n_rows == 0 || n_configs == 0) return KT_OK;
  if (!d_time || !d_out) return fail(h, KT_EINVAL, "NULL table");
  hipStream_t st = (hipStream_t)stream;
  kt_status s = ensure_lut(h, st);
  if (s != KT_OK) return s;
  hipLaunchKernelGGL(normalize_kernel, dim3(n_rows), dim3(256), 0, st, d_time, n_configs, (int32_t)norm,
                     (const uint16_t*)h->d_lut, d_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "normalize launch");
  return KT_OK;
}

kt_status kt_prune_workspace_bytes(int32_t n_rows, int32_t n_configs, int32_t k, int32_t n_init,
                                   size_t* bytes) {
  if (!bytes || n_rows < 1 || n_configs < 1 || k < 1 || n_init < 1) return KT_EINVAL;
  *bytes = prune_plan(n_rows, n_configs, k, n_init).total;
  return KT_OK;
}

kt_status kt_prune(kt_handle hh, const int64_t* time_ns, int32_t n, int32_t d, int32_t k,
                   kt_norm norm, uint64_t seed, int32_t n_init, int32_t max_iter, void* workspace,
                   size_t ws_bytes, void* stream, int32_t* chosen, int64_t* inertia_out,
                   int32_t* labels, int64_t* centroids) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  kt_status s = check_table(h, n, d);
  if (s != KT_OK) return s;
  if (!time_ns || !chosen || !inertia_out) return fail(h, KT_EINVAL, "NULL argument");
  if ((int)norm < 0 || (int)norm > 3) return fail(h, KT_EINVAL, "bad normalization");
  if (k < 1 || k > n || k > d || k > 64) return fail(h, KT_EINVAL, "need 1 <= k <= min(n_rows, n_configs, 64)");
  if (n_init < 1 || max_iter < 0) return fail(h, KT_EINVAL, "need n_init >= 1 and max_iter >= 0");
  if (n > KM_MAX_ROWS || (int64_t)k * d > KM_MAX_KD)
    return fail(h, KT_EUNSUPPORTED, "k-means limits: n_rows <= 4096 and k * n_configs <= 8192");
  const PrunePlan p = prune_plan(n, d, k, n_init);
  if (!workspace || ws_bytes < p.total) return fail(h, KT_EWORKSPACE, "prune workspace too small");
  char* ws = (char*)workspace;
  hipStream_t st = (hipStream_t)stream;
  s = upload_normalize(h, time_ns, n, d, norm, ws, p, st);
  if (s != KT_OK) return s;
  const size_t lds = kmeans_lds_bytes(n, d, k);
  hipError_t e = hipFuncSetAttribute((const void*)kmeans_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return hip_fail(h, e, "kmeans LDS attribute");
  hipLaunchKernelGGL(kmeans_kernel, dim3(n_init), dim3(KM_THREADS), lds, st,
                     (const uint16_t*)(ws + p.off_X), n, d, k, seed, max_iter,
                     (int64_t*)(ws + p.off_cent), (int32_t*)(ws + p.off_lab),
                     (KmeansOut*)(ws + p.off_out));
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "kmeans launch");
  int32_t* d_chosen = (int32_t*)(ws + p.off_chosen);
  hipLaunchKernelGGL(choose_kernel, dim3(1), dim3(64), 0, st, (const int64_t*)(ws + p.off_cent),
                     (const KmeansOut*)(ws + p.off_out), n_init, k, d, d_chosen, d_chosen + k);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "choose launch");
  std::vector<int32_t> hc(k + 1);
  e = hipMemcpyAsync(hc.data(), d_chosen, (size_t)(k + 1) * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(h, e, "read chosen");
  const int br = hc[k];
  KmeansOut o;
  e = hipMemcpy(&o, ws + p.off_out + br * sizeof(KmeansOut), sizeof o, hipMemcpyDeviceToHost);
  if (e == hipSuccess && labels)
    e = hipMemcpy(labels, ws + p.off_lab + (size_t)br * n * 4, (size_t)n * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && centroids)
    e = hipMemcpy(centroids, ws + p.off_cent + (size_t)br * k * d * 8, (size_t)k * d * 8,
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "read k-means result");
  memcpy(chosen, hc.data(), (size_t)k * 4);
  *inertia_out = o.inertia;
  return KT_OK;
}

kt_status kt_kmeans_u16(kt_handle hh, const uint16_t* X, int32_t n, int32_t d, int32_t k,
                        uint64_t seed, int32_t n_init, int32_t max_iter, void* workspace,
                        size_t ws_bytes, void* stream, int32_t* labels, int64_t* centroids,
                        int64_t* inertia_out) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  if (n < 1 || d < 1) return fail(h, KT_EINVAL, "need n >= 1 and d >= 1");
  if (!X || !labels || !inertia_out) return fail(h, KT_EINVAL, "NULL argument");
  if (k < 1 || k > n || k > 64) return fail(h, KT_EINVAL, "need 1 <= k <= min(n, 64)");
  if (n_init < 1 || max_iter < 0) return fail(h, KT_EINVAL, "need n_init >= 1 and max_iter >= 0");
  if (n > KM_MAX_ROWS || (int64_t)k * d > KM_MAX_KD)
    return fail(h, KT_EUNSUPPORTED, "k-means limits: n <= 4096 and k * d <= 8192");
  const PrunePlan p = prune_plan(n, d, k, n_init);
  if (!workspace || ws_bytes < p.total) return fail(h, KT_EWORKSPACE, "k-means workspace too small");
  char* ws = (char*)workspace;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(ws + p.off_X, X, (size_t)n * d * 2, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(h, e, "upload vectors");
  const size_t lds = kmeans_lds_bytes(n, d, k);
  e = hipFuncSetAttribute((const void*)kmeans_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds);
  if (e != hipSuccess) return hip_fail(h, e, "kmeans LDS attribute");
  hipLaunchKernelGGL(kmeans_kernel, dim3(n_init), dim3(KM_THREADS), lds, st,
                     (const uint16_t*)(ws + p.off_X), n, d, k, seed, max_iter,
                     (int64_t*)(ws + p.off_cent), (int32_t*)(ws + p.off_lab),
                     (KmeansOut*)(ws + p.off_out));
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "kmeans launch");
  // the restart with the lowest inertia (its per-coordinate picks are unused)
  int32_t* d_chosen = (int32_t*)(ws + p.off_chosen);
  hipLaunchKernelGGL(choose_kernel, dim3(1), dim3(64), 0, st, (const int64_t*)(ws + p.off_cent),
                     (const KmeansOut*)(ws + p.off_out), n_init, k, d, d_chosen, d_chosen + k);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "choose launch");
  int32_t br = 0;
  e = hipMemcpyAsync(&br, d_chosen + k, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(h, e, "read best restart");
  KmeansOut o;
  e = hipMemcpy(&o, ws + p.off_out + br * sizeof(KmeansOut), sizeof o, hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(labels, ws + p.off_lab + (size_t)br * n * 4, (size_t)n * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && centroids)
    e = hipMemcpy(centroids, ws + p.off_cent + (size_t)br * k * d * 8, (size_t)k * d * 8,
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(h, e, "read k-means result");
  *inertia_out = o.inertia;
  return KT_OK;
}

kt_status kt_prune_topn(kt_handle hh, const int64_t* time_ns, int32_t n, int32_t d, int32_t k,
                        void* workspace, size_t ws_bytes, void* stream, int32_t* chosen) {
  Ctx* h = reinterpret_cast<Ctx*>(hh);
  if (!h) return fail(nullptr, KT_EINVAL, "NULL handle");
  if (!need_device(h)) return KT_EINVAL;
  kt_status s = check_table(h, n, d);
  if (s != KT_OK) return s;
  if (!time_ns || !chosen || k < 1 || k > d) return fail(h, KT_EINVAL, "bad arguments");
  const PrunePlan p = prune_plan(n, d, 1, 1);
  if (!workspace || ws_bytes < p.total) return fail(h, KT_EWORKSPACE, "Top-N workspace too small");
  hipStream_t st = (hipStream_t)stream;
  s = upload_normalize(h, time_ns, n, d, KT_NORM_RELATIVE, (char*)workspace, p, st);
  if (s != KT_OK) return s;
  std::vector<uint16_t> X((size_t)n * d);
  hipError_t e = hipMemcpyAsync(X.data(), (char*)workspace + p.off_X, X.size() * 2,
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(h, e, "read normalized table");
  std::vector<int64_t> count(d, 0);
  for (int32_t i = 0; i < n; ++i) {
    const uint16_t* x = &X[(size_t)i * d];
    int best = 0;
    for (int f = 1; f < d; ++f) if (x[f] > x[best]) best = f;
    count[best]++;
  }
  std::vector<int32_t> order(d);
  for (int f = 0; f < d; ++f) order[f] = f;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return count[a] > count[b]; });
  for (int j = 0; j < k; ++j) chosen[j] = order[j];
  return KT_OK;
}

}  // extern "C"
