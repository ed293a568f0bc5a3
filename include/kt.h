/*
 * kt -- ML-pruned, per-shape-selected GEMM kernels for AMD MI355X (gfx950).
 *
 * C ABI of libkt.so.  Implements the method of J. Lawson, "Performance
 * portability through machine learning guided kernel selection in SYCL
 * libraries" (arXiv 2008.13145): a parameterized tiled matrix multiply
 * (section 3), an exhaustive benchmark of its configuration space
 * (sections 3 and 3.1), normalization of the timings (section 3.4), k-means
 * pruning to k deployable kernels (sections 4.1-4.2), a decision-tree
 * selector trained on the benchmark labels (section 5.1) and its evaluation
 * against exhaustive search (section 4.3).
 *
 * Conventions (all entry points)
 * ------------------------------
 * - Matrices are row-major.  op(A) is M x K: stored M x K (lda >= K) when
 *   transA == 0, stored K x M (lda >= M) when transA == 1.  op(B) is K x N:
 *   stored K x N (ldb >= N) when transB == 0, N x K (ldb >= K) when 1.
 *   C is M x N (ldc >= N).  Batch item b starts at ptr + b * stride.
 * - Device pointers are owned by the caller and must stay valid until the
 *   work queued on `stream` completes.  Host pointers are read or written
 *   before the call returns.  The library allocates device memory only
 *   where an entry point says so.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * - Every function returns a kt_status and never throws or aborts.  On
 *   failure kt_last_error(handle) holds a message.  Asynchronous kernel
 *   faults surface at the next synchronizing call.
 * - A handle is not thread-safe; use one per thread.
 */
#ifndef KT_H
#define KT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KT_OK = 0,
  KT_EINVAL = -1,        /* bad argument (negative size, short leading dimension, ...) */
  KT_EUNSUPPORTED = -2,  /* dtype / configuration / layout not compiled into this build */
  KT_EHIP = -3,          /* a HIP runtime call failed; message has hipGetErrorString text */
  KT_ENOTFITTED = -4,    /* selection requested before a selector was fitted or loaded */
  KT_EWORKSPACE = -5,    /* workspace missing or smaller than the size query returned */
  KT_EIO = -6            /* file could not be read / written, or is malformed */
} kt_status;

typedef enum { KT_F32 = 0, KT_BF16 = 1, KT_FP8E4M3 = 2 } kt_dtype;

/* Normalizations of section 3.4 (integer Q16 reading, 65535 = 1.0). */
typedef enum {
  KT_NORM_RELATIVE = 0,  /* t_best / t */
  KT_NORM_RAWCUT = 1,    /* relative, values below 0.9 set to 0 */
  KT_NORM_STDCUT = 2,    /* raw cutoff, then [0.9, 1] rescaled onto [0, 1] */
  KT_NORM_SIGMOID = 3    /* 1 / (1 + exp(50 (0.85 - x))) of the relative value */
} kt_norm;

/* Selectors: decision trees A/B/C of section 5.1, the MLP cost model, or
 * exhaustive timing of every compiled configuration (cached per shape). */
typedef enum {
  KT_SEL_DT_A = 0,       /* no depth limit, min 1 sample per leaf */
  KT_SEL_DT_B = 1,       /* depth <= 6, min 3 samples per leaf */
  KT_SEL_DT_C = 2,       /* depth <= 3, min 4 samples per leaf */
  KT_SEL_MLP = 3,
  KT_SEL_EXHAUSTIVE = 4
} kt_selector;

typedef struct {
  int64_t M, N, K, batch;
  int32_t transA, transB;
} kt_shape;

/* One tile configuration (the layout comes from the shape).
 * bm x bn: work-group output tile; t: per-lane thread tile, so each wave
 * owns an (8t) x (8t) block and each lane t*t accumulators; bk: K depth of
 * one LDS stage. */
typedef struct {
  int32_t bm, bn, t, bk;
  int32_t dtype; /* kt_dtype */
} kt_config;

typedef struct kt_ctx* kt_handle;

/* ---------------------------------------------------------------- handle */

/* Create a handle.  device >= 0 binds the handle to that HIP device (it
 * becomes current on the calling thread).  device == -1 gives a host-only
 * handle: configuration tables, selector fitting for decision trees,
 * selection, save and load work; every entry point that launches GPU work
 * returns KT_EINVAL. */
kt_status kt_create(kt_handle* out, int device);
kt_status kt_destroy(kt_handle h);
/* Message of the last failed call on this handle ("" if none). Valid until the
 * next call on the handle.  Also works with h == NULL (errors of kt_create). */
const char* kt_last_error(kt_handle h);
/* Semantic version of the ABI, e.g. 100 for 0.1.0. */
int32_t kt_abi_version(void);

/* ------------------------------------------------------ configuration space */

/* Number of tile configurations of a dtype (per layout; a deploy build may
 * compile only some of them, see kt_config_compiled).
 * KT_F32: the space of section 3's kernel re-designed for MFMA: bm, bn in
 * {8,16,32,64,128}, t in {1,2,4,8}, bk in {8,16,32,64}, with bm and bn
 * multiples of 8t and 1..16 waves per work-group: 164 configurations.
 * KT_BF16 / KT_FP8E4M3: bm, bn in {32,64,128,256}, t in {4,8,16} (wave
 * blocks of 32x32, 64x64 or 128x128 outputs on the 32x32 MFMAs), bk in
 * {32,64,128} (BF16) or {64,128,256} (FP8: multiples of its 64-deep MFMA),
 * 1..16 waves, double-buffered LDS stages within 160 KiB: 68 configurations
 * each (ids 0..67); then t = 2 (16x16 wave blocks on the 16x16 MFMAs) with
 * bm, bn in {16,...,256}, 1..16 waves, bk in {32,64} (BF16) or {128} (FP8):
 * 98 BF16 and 83 FP8 configurations in all. */
kt_status kt_num_configs(kt_handle h, kt_dtype dtype, int32_t* n);
/* Configuration `id` (0 <= id < n) of a dtype.  KT_EINVAL if out of range. */
kt_status kt_get_config(kt_handle h, kt_dtype dtype, int32_t id, kt_config* out);
/* 1 if kernel `id` (a configuration, or a split-K variant through its base
 * configuration) is compiled for the (transA, transB) layout. */
kt_status kt_config_compiled(kt_handle h, kt_dtype dtype, int32_t id, int32_t transA,
                             int32_t transB, int32_t* compiled);

/* ----------------------------------------------------------------- kernels */

/* The kernels of a dtype, the columns of its sweep table and the ids that
 * pruning and selection return: its configurations (kernel id = configuration
 * id, 0 <= id < kt_num_configs) followed by split-K variants, the separate
 * kernel type section 3 names for deep products with few output tiles (K
 * divided among work-groups, partial results reduced afterwards).  A variant
 * runs a base configuration over `slices` slices of K exactly as
 * kt_gemm_splitk(splits = slices, config_id = base) does, when its partial
 * planes (S * batch * M * N floats with S the slices really used, at most
 * 256 MiB) fit the workspace it is given; otherwise it runs as the base
 * configuration unsplit.  Variants: for each work-group tile 16x16, 32x32,
 * 64x64, 128x128, 16x128 and 128x16 (in this order), the configuration with
 * the deepest K tile and then the most waves, over 2, 4, 8 and 16 slices (24
 * variants per dtype).  A variant
 * needs no code of its own: it is compiled wherever its base is. */
kt_status kt_num_kernels(kt_handle h, kt_dtype dtype, int32_t* n);
/* Kernel `id`: its configuration (the base's for a variant), the base
 * configuration id (id itself for a configuration) and the slice count
 * (1 for a configuration).  All outputs host pointers.  KT_EINVAL if out of
 * range. */
kt_status kt_get_kernel(kt_handle h, kt_dtype dtype, int32_t id, kt_config* cfg,
                        int32_t* base_id, int32_t* slices);
/* Partial-plane bytes kernel `id` needs on shape s to run split (0 when it
 * runs unsplit: a configuration, one slice, or planes beyond 256 MiB).
 * Host only. */
kt_status kt_kernel_workspace_bytes(kt_handle h, kt_dtype dtype, const kt_shape* s, int32_t id,
                                    size_t* bytes);
/* Device workspace (caller-owned, may be NULL with bytes 0) that kt_gemm
 * gives a split-K kernel for its partial planes, whether selected or forced.
 * The handle keeps the pointer, not the memory: it must stay allocated and
 * untouched by the caller while kt_gemm work queued on any stream may use
 * it, and kt_gemm calls of one handle that run split-K kernels on different
 * streams at once race on it.  Without it (or when it is too small for a
 * product) split-K kernels run as their base configuration unsplit. */
kt_status kt_set_workspace(kt_handle h, void* workspace, size_t bytes);

/* ------------------------------------------------------------------- GEMM */

/* C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b]   (section 3).
 * in_dtype selects the element type of A and B (FP32, BF16 stored as uint16
 * bit patterns, or FP8 e4m3 codes); C is always FP32.  FP8 multiplies the
 * product by alpha / (scaleA[0] * scaleB[0]) where scaleA/scaleB are device
 * pointers to the per-tensor quantization scales (NULL for other dtypes).
 * config_id >= 0 forces that kernel (a configuration or a split-K variant,
 * see kt_num_kernels; a variant takes its partial planes from the workspace
 * set with kt_set_workspace); -1 asks the fitted selector, whose pick may be
 * a split-K variant.
 * With beta == 0, C is never read (NaN in C does not propagate).  M, N or
 * batch == 0 is a no-op; K == 0 gives C = beta * C.  Unaligned pointers or
 * leading dimensions are never an error (FP32 rows load as dword-aligned
 * 16-byte vectors whatever the leading dimension). */
kt_status kt_gemm(kt_handle h, kt_dtype in_dtype, const kt_shape* s, float alpha,
                  const void* A, int64_t lda, int64_t strideA,
                  const void* B, int64_t ldb, int64_t strideB,
                  float beta, float* C, int64_t ldc, int64_t strideC,
                  const float* scaleA, const float* scaleB,
                  int32_t config_id, void* stream);

/* Which pipeline the GEMM kernels take for these operands (host only,
 * nothing launched): *dma = 1 when every row of A and B starts on a 16-byte
 * boundary (base, leading dimension and, for batch > 1, batch stride) and no
 * 16-byte chunk read leaves an operand: its contiguous extent (K for an
 * operand stored K-contiguous, M or N otherwise) is a whole number of 16-byte
 * chunks or, after kt_set_full_rows(h, 1), at least one chunk with the
 * leading dimension reaching the next 16-byte boundary -- tiles then move
 * from HBM to LDS by LDS DMA with several stages in flight; otherwise 0
 * (register-staged loads).  BF16 / FP8: every configuration has both
 * pipelines and they give the same bits.  FP32: configurations with t >= 2
 * whose A and B tiles are whole KiB (bm * bk, bn * bk multiples of 256) have
 * the DMA pipeline; it sums K in another order than the register-staged one
 * (results within the same bound, not bit-identical); the others always run
 * register-staged. */
kt_status kt_dma_pipeline(kt_handle h, kt_dtype dtype, const kt_shape* s, const void* A,
                         int64_t lda, int64_t strideA, const void* B, int64_t ldb, int64_t strideB,
                         int32_t* dma);
/* Promise (enabled = 1) that every BF16 / FP8 operand later passed to this
 * handle's GEMM calls is allocated to whole rows of its leading dimension,
 * the last row included, so that the DMA pipeline may read a row up to its
 * next 16-byte boundary beyond the logical extent (values there only reach
 * outputs that are not stored, or are zeroed in LDS).  Default 0. */
kt_status kt_set_full_rows(kt_handle h, int32_t enabled);

/* Split-K form of kt_gemm for deep products with few output tiles, the
 * tall-skinny / very deep K case that section 3 names as its kernel's worst
 * (fix: divide the K range among work-groups).  The K range is cut into
 * S = ceil(K / kc) slices of depth kc = ceil(K / splits) rounded up to a
 * multiple of 64 (so S <= splits; the last slice may be shallower); slice q
 * is computed with configuration config_id (-1: the configuration of the
 * kernel the selector picks for the shape M, N, kc with batch * S items)
 * into FP32 partial planes in the
 * workspace (device, dense, [S][batch][M][N]), and one reduction pass writes
 * C = alpha * (sum of the planes in slice order) + beta * C (C not read when
 * beta == 0).  Arguments and layouts as kt_gemm; 0 <= splits <= 64.
 * splits == 0 chooses S: the configuration is config_id, or the
 * configuration of the selector's pick for the whole product, and S doubles from 1 while that configuration
 * fills fewer than 2048 work-groups (tiles x batch x S), each slice stays at
 * least 256 deep and S < 64.  When S == 1 (also splits == 1 or K <= 64)
 * this is exactly kt_gemm and needs no workspace.  *used_splits (host, may
 * be NULL) receives S.  The workspace
 * must stay untouched until the work on `stream` has finished.
 * KT_EWORKSPACE if it is smaller than kt_gemm_splitk_workspace_bytes. */
kt_status kt_gemm_splitk(kt_handle h, kt_dtype in_dtype, const kt_shape* s, int32_t splits,
                         float alpha, const void* A, int64_t lda, int64_t strideA,
                         const void* B, int64_t ldb, int64_t strideB, float beta, float* C,
                         int64_t ldc, int64_t strideC, const float* scaleA, const float* scaleB,
                         int32_t config_id, void* workspace, size_t ws_bytes, void* stream,
                         int32_t* used_splits);
/* Workspace bytes of kt_gemm_splitk: splits * batch * M * N floats, rounded
 * up to 256 bytes (0 for splits == 1); for splits == 0 a bound that covers
 * every automatic choice, min(64 * batch * M * N, 2^28) floats.  Host only. */
kt_status kt_gemm_splitk_workspace_bytes(const kt_shape* s, int32_t splits, size_t* bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): kt_gemm_splitk
 * with the partial planes in a static device array the library owns instead
 * of a caller workspace.  Same arguments, kernels, results (bit for bit) and
 * slice choice as kt_gemm_splitk.  The array holds
 * kt_gemm_splitk_noalloc_max_bytes() bytes (32 MiB) on every GPU the
 * library runs on, from kt_create on that device until the process ends; a
 * product that needs more (slices * batch * M * N * 4 bytes) returns
 * KT_EWORKSPACE before anything is launched.  Nothing is allocated: no
 * hipMalloc, hipFree or allocating library call, so config_id = -1 with an
 * exhaustive selector works only for shapes it has already timed
 * (KT_EUNSUPPORTED otherwise).  Nothing in the array needs clearing: every
 * partial plane is fully written before the reduction reads it.  All calls
 * on one GPU share the one array and keep the last call's contents, so
 * calls that overlap on one GPU (other streams, other threads, other
 * handles) race; serialize them, e.g. on one stream. */
kt_status kt_gemm_splitk_noalloc(kt_handle h, kt_dtype in_dtype, const kt_shape* s,
                                 int32_t splits, float alpha, const void* A, int64_t lda,
                                 int64_t strideA, const void* B, int64_t ldb, int64_t strideB,
                                 float beta, float* C, int64_t ldc, int64_t strideC,
                                 const float* scaleA, const float* scaleB, int32_t config_id,
                                 void* stream, int32_t* used_splits);
/* Size of the static scratch of kt_gemm_splitk_noalloc in bytes.  Host only. */
kt_status kt_gemm_splitk_noalloc_max_bytes(size_t* bytes);

/* ------------------------------------------------------------ convolution */

/* Convolution layers through the selected GEMMs (section 6 runs VGG16, whose
 * convolutions and fully connected layers are matrix multiplications).
 * Activations are NHWC FP32 (n, H, W, C), filters (R, S, Cin, Cout) FP32,
 * zero padding `pad` on every side, output (n, Ho, Wo, Cout) with
 * Ho = (H + 2 pad - R) / stride + 1 (Wo likewise):
 *   y[b,i,j,o] = act(bias[o] + sum_{r,s,c} x[b, i*stride-pad+r, j*stride-pad+s, c] * w[r,s,c,o]).
 * KT_CONV_IM2COL: any R, S, stride; the rows of the (n Ho Wo) x (R S Cin)
 * patch matrix are built in the workspace and multiplied by the filter.
 * KT_CONV_WINOGRAD: F(2x2, 3x3) (Lavin and Gray): R = S = 3, stride 1
 * (KT_EUNSUPPORTED otherwise); input and filter transforms in the workspace,
 * 16 GEMMs of T x Cin by Cin x Cout in one batched launch (T = n ceil(Ho/2)
 * ceil(Wo/2) tiles), output transform with bias and activation fused. */
typedef enum {
  KT_CONV_IM2COL = 0,
  KT_CONV_WINOGRAD = 1,
  /* Winograd with w holding the 16 x Cin x Cout transformed filter written
   * by kt_winograd_filter (weights transformed once, when they are loaded) */
  KT_CONV_WINOGRAD_PRETRANSFORMED = 2
} kt_conv_algo;

typedef struct {
  int64_t n, H, W, Cin, Cout;
  int32_t R, S, stride, pad;
} kt_conv_shape;

/* The GEMM a convolution runs (what the selector is asked about):
 * im2col {n Ho Wo, Cout, R S Cin, batch 1}, Winograd {T, Cout, Cin, batch 16},
 * both non-transposed.  Host only. */
kt_status kt_conv2d_gemm_shape(const kt_conv_shape* c, kt_conv_algo algo, kt_shape* out);
/* Device workspace of kt_conv2d for a `splits` value (im2col: the patch
 * matrix, none for a 1x1 filter with stride 1 and no padding, whose patch
 * matrix is x itself, followed by the split-K partial planes of
 * kt_gemm_splitk_workspace_bytes when splits != 1; Winograd: the
 * transformed input, filter and the 16 products, each 256-byte aligned). */
kt_status kt_conv2d_workspace_bytes(const kt_conv_shape* c, kt_conv_algo algo, int32_t splits,
                                    size_t* bytes);
/* y = conv(x, w) + bias, then ReLU when relu != 0.  x, w, bias (NULL = no
 * bias; Cout floats), y and workspace are device pointers; y must not alias
 * x or the workspace.  config_id: FP32 configuration of the GEMM, -1 = the
 * kernel the fitted selector picks for kt_conv2d_gemm_shape (with splits = 1
 * and im2col, a selected split-K kernel runs split with the partial planes in
 * the kt_set_workspace buffer when they fit; otherwise its configuration
 * runs with the layer's `splits`).  splits (im2col only; Winograd
 * takes 0 or 1 and never splits): 1 = the plain GEMM, otherwise the GEMM
 * runs as kt_gemm_splitk with this splits value (0 = automatic), which suits
 * the fully connected layers of a single image (M = 1, deep K).  Empty n, Ho
 * or Wo is a no-op.  Asynchronous on `stream`. */
kt_status kt_conv2d(kt_handle h, kt_conv_algo algo, const kt_conv_shape* c, const float* x,
                    const float* w, const float* bias, int32_t relu, float* y, int32_t config_id,
                    int32_t splits, void* workspace, size_t ws_bytes, void* stream);
/* The Winograd F(2x2, 3x3) filter transform U[k][c][o] = (G g Gt)[k] of the
 * 3x3 filters g = w[:, :, c, o] (device arrays: w is (3, 3, Cin, Cout), U is
 * 16 x Cin x Cout floats), for KT_CONV_WINOGRAD_PRETRANSFORMED.
 * Asynchronous on `stream`. */
kt_status kt_winograd_filter(kt_handle h, const float* w, int64_t Cin, int64_t Cout, float* U,
                             void* stream);
/* 2x2 max pooling with stride 2 on NHWC FP32 (device): y is
 * (n, H/2, W/2, C); an odd trailing row or column is dropped. */
kt_status kt_maxpool2x2(kt_handle h, const float* x, int64_t n, int64_t H, int64_t W, int64_t C,
                        float* y, void* stream);

/* Fill dst[i] (device, n floats) with the seeded operand stream
 * x(seed, offset + i) = (splitmix64(seed XOR (offset + i)) >> 40) * 2^-23 - 1,
 * values in [-1, 1) exact in FP32. */
kt_status kt_fill_uniform(kt_handle h, float* dst, int64_t n, uint64_t seed, int64_t offset,
                          void* stream);

/* Convert n FP32 values (device) to BF16 bit patterns (device uint16),
 * round to nearest even, NaN kept quiet.  Asynchronous on `stream`. */
kt_status kt_convert_bf16(kt_handle h, const float* x, int64_t n, uint16_t* y, void* stream);

/* Per-tensor FP8-e4m3 quantization of n FP32 values (device): s = 448 / amax
 * (FP32, s = 1 when every value is 0) is written to d_scale[0] (device) and
 * y[i] = e4m3(x[i] * s) (OCP e4m3fn codes, round to nearest even, saturating
 * at +-448, NaN -> 0x7F).  Dequantized value = decode(y) / s.  The workspace
 * (device, >= 4 bytes) holds the running amax.  Asynchronous on `stream`. */
kt_status kt_quantize_fp8(kt_handle h, const float* x, int64_t n, uint8_t* y, float* d_scale,
                          void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------ sweep */

typedef struct {
  int32_t warmup;       /* untimed launches before timing (>= 0), default 1 */
  float target_ms;      /* timed reps = clamp(ceil(target_ms / t_first), min_reps, max_reps) */
  int32_t min_reps, max_reps;
  float cut_factor;     /* if the first launch is slower than cut_factor x the row's best so
                           far, record it and skip the timed reps (0 disables) */
  float pause_ms;       /* host sleep between rows, to limit heating */
  uint64_t seed;        /* operand seed base: A, B (and C if beta != 0) are filled per row */
  float alpha, beta;
  int32_t pad_rows;     /* 1: rows of A and B padded to a multiple of 16 elements (leading
                           dimension rounded up, rows allocated in full: 16-byte rows in
                           every dtype); 0: dense rows */
} kt_sweep_opts;

/* Device workspace needed to sweep these shapes with any kernels: operands
 * of the largest shape (rows padded to 16 elements, which also covers dense
 * rows), 256-byte aligned, plus the largest partial planes any split-K
 * variant of the dtype takes on it. */
kt_status kt_sweep_workspace_bytes(const kt_shape* shapes, int32_t n_shapes, kt_dtype dtype,
                                   size_t* bytes);
/* Time every (shape, kernel) pair (sections 3 and 3.1): for each shape the
 * operands are filled in the workspace, then each kernel is launched
 * `warmup` times and timed with HIP events over its reps (a split-K variant
 * as its slice launches plus reduction, its partial planes after the
 * operands in the workspace); the mean nanoseconds per launch go to
 * time_ns[shape * n_configs + c] (host, int64).  config_ids (host) selects
 * kernels (NULL = all kernels of the dtype, configurations and split-K
 * variants, in id order).  Entries already >= 0 in time_ns are kept
 * (resume).  KT_EWORKSPACE if the workspace is smaller than a shape's
 * operands plus the partial planes of the listed kernels.  The call
 * synchronizes `stream`. */
kt_status kt_sweep(kt_handle h, kt_dtype dtype, const kt_shape* shapes, int32_t n_shapes,
                   const int32_t* config_ids, int32_t n_configs, const kt_sweep_opts* opts,
                   void* workspace, size_t ws_bytes, void* stream, int64_t* time_ns);

/* ---------------------------------------------------------- normalization */

/* Normalize a device int64 time table [n_rows][n_configs] into device uint16
 * Q16 values (section 3.4): q = round_half_up(65535 * t_best / t) with t_best
 * the row's smallest positive time (t <= 0 gives 0), then the chosen variant.
 * Runs on `stream`, asynchronously.  The first call on a handle uploads the
 * 128 KiB sigmoid table into device memory the handle owns. */
kt_status kt_normalize(kt_handle h, const int64_t* d_time, int32_t n_rows, int32_t n_configs,
                       kt_norm norm, uint16_t* d_out, void* stream);

/* ---------------------------------------------------------------- pruning */

/* Workspace bytes for kt_prune. */
kt_status kt_prune_workspace_bytes(int32_t n_rows, int32_t n_configs, int32_t k, int32_t n_init,
                                   size_t* bytes);
/* Choose k configurations by k-means over the normalized rows (sections 4.1
 * and 4.2), on the GPU.  time_ns is a host table [n_rows][n_configs].
 * k-means++ initialisation from a SplitMix64 stream seeded with seed + r for
 * restart r, integer Lloyd iterations (exact int64 distances and sums,
 * rounded-mean centroids), n_init restarts (lowest inertia wins, lowest r on
 * ties), at most max_iter updates each.  Limits: n_rows <= 4096,
 * k <= 64, k * n_configs <= 8192.  Centroid j yields its best
 * configuration not already chosen.  Outputs (host): chosen[k] column
 * indices in cluster order, *inertia_out, and optionally labels[n_rows] and
 * centroids[k * n_configs] (NULL to skip).  Synchronizes `stream`. */
kt_status kt_prune(kt_handle h, const int64_t* time_ns, int32_t n_rows, int32_t n_configs,
                   int32_t k, kt_norm norm, uint64_t seed, int32_t n_init, int32_t max_iter,
                   void* workspace, size_t ws_bytes, void* stream,
                   int32_t* chosen, int64_t* inertia_out, int32_t* labels, int64_t* centroids);

/* The same integer k-means as kt_prune (k-means++ from the SplitMix64
 * stream seeded seed + restart, Lloyd, n_init restarts, lowest inertia wins)
 * on arbitrary 16-bit vectors X (host array, n x d row-major), for pruning
 * in a reduced space (section 4.1 clusters after a dimensionality
 * reduction).  Writes labels[n] and, if centroids is not NULL,
 * centroids[k * d] (rounded means) of the winning restart, and its inertia.
 * Workspace sized by kt_prune_workspace_bytes(n, d, k, n_init).  Limits as
 * kt_prune: n <= 4096, k <= 64, k * d <= 8192 (KT_EUNSUPPORTED beyond).
 * Synchronizes `stream`. */
kt_status kt_kmeans_u16(kt_handle h, const uint16_t* X, int32_t n, int32_t d, int32_t k,
                        uint64_t seed, int32_t n_init, int32_t max_iter, void* workspace,
                        size_t ws_bytes, void* stream, int32_t* labels, int64_t* centroids,
                        int64_t* inertia_out);

/* Decision-tree pruning (section 4.1: a regression tree from the matrix
 * sizes to the performance vector, limited to k leaves, each leaf's vector
 * standing for the problems that reach it).  shapes[n] and Xq (n x d
 * normalized Q16 rows, as written by kt_normalize) are host arrays; the
 * features are (M, N, K, batch, transA, transB).  A split of a node's rows
 * into L and R is scored by A / n_L + B / n_R (A, B: squared norms of the
 * children's column sums; the maximum minimises the squared error to the
 * children's means), thresholds floor(sqrt(a*b)) between consecutive
 * distinct values, x <= t goes left, features scanned 0..5 and thresholds
 * ascending with the first maximum kept.  Growth is best first: while there
 * are fewer than k leaves, the leaf whose best split gains most over
 * P / n (lowest node id on ties) is split if that gain is positive.  Leaves
 * in pre-order pick the configuration with the largest rounded mean
 * floor((2 s + n) / (2 n)) not already chosen (lowest index on ties); with
 * fewer than k leaves the rest are the unchosen columns with the largest
 * sums.  chosen[k] (host) receives the picks.  Host only (works on a handle
 * without a device); n <= 4096, k <= d <= 256 (KT_EUNSUPPORTED beyond). */
kt_status kt_prune_tree(kt_handle h, const kt_shape* shapes, const uint16_t* Xq, int32_t n,
                        int32_t d, int32_t k, int32_t* chosen);

/* The same decision-tree pruning as kt_prune_tree, returning the leaves
 * instead of the picks: labels[i] (host, n) = pre-order position of the leaf
 * row i reaches, *n_leaves = number of leaves (<= k).  Feeding the labels to
 * kt_representatives(KT_REP_MEAN) gives kt_prune_tree's picks;
 * KT_REP_GEOMEAN gives the paper's rule for label-only clusters.  Host only,
 * limits as kt_prune_tree. */
kt_status kt_prune_tree_leaves(kt_handle h, const kt_shape* shapes, const uint16_t* Xq, int32_t n,
                               int32_t d, int32_t k, int32_t* labels, int32_t* n_leaves);

/* ------------------------------------------- clusters -> kernels (4.2) */

/* How a cluster becomes the kernel to deploy (section 4.2).  A clustering
 * that yields a representative deploys the configuration best for it; one
 * that yields only labels deploys the configuration best for the geometric
 * mean of the members. */
typedef enum {
  KT_REP_MEAN = 0,      /* rounded member mean floor((2 s + n) / (2 n)): the k-means centroid */
  KT_REP_GEOMEAN = 1,   /* geometric mean of the members' Q16 values, 0 counted as 1 / 65535 */
  KT_REP_CENTROID = 2   /* PCA pruning only: the k-means centroid read back through the
                           components as Q16 values of every configuration */
} kt_rep;

/* One configuration per cluster from labels (host arrays: Xq n x d Q16
 * rows, labels[n] in 0..n_clusters-1).  Clusters in label order each take
 * their best configuration not already taken (lowest index on ties); empty
 * clusters take nothing; a short list is completed with the unpicked
 * configurations of largest column sum over all rows (of the values for
 * KT_REP_MEAN, of their logarithms for KT_REP_GEOMEAN).  KT_REP_GEOMEAN
 * compares products through the fixed-point logarithm of
 * kt_log2_q16_table, summed exactly in int64.  chosen[k] (host) receives the
 * picks.  Host only (works on a handle without a device); n <= 2^26. */
kt_status kt_representatives(kt_handle h, const uint16_t* Xq, int32_t n, int32_t d,
                             const int32_t* labels, int32_t n_clusters, int32_t k, kt_rep rep,
                             int32_t* chosen);
/* table[q] = round(2^32 * log2(max(q, 1) / 65535)) for q = 0..65535 (host,
 * 65536 int64): the logarithm KT_REP_GEOMEAN sums. */
kt_status kt_log2_q16_table(int64_t* table);

/* Principal components of the rows x = q / 65535 of a Q16 table (section
 * 4.1, PCA before k-means; host, FP64): centred at the column means,
 * covariance Xc^T Xc / (n - 1), unit eigenvectors by decreasing eigenvalue
 * (cyclic Jacobi), each signed so that its first entry within a factor
 * 1 - 1e-9 of its largest magnitude is positive.  Optional host outputs:
 * mean[d], components[m][d] (the first m), variances[d] (every eigenvalue,
 * decreasing), U[n][m] = rint((Z - lo) / span * 65535) with Z = Xc V_m and
 * one offset lo = min Z and scale span = max Z - lo for every coordinate
 * (U = 0 when span = 0), lo_span[2] = {lo, span}, *explained = the first m
 * eigenvalues' share of the trace.  Needs n >= 2, 1 <= m <= d <= 1024. */
kt_status kt_pca(kt_handle h, const uint16_t* Xq, int32_t n, int32_t d, int32_t m, double* mean,
                 double* components, double* variances, uint16_t* U, double* lo_span,
                 double* explained);

/* PCA + k-means pruning (section 4.1): normalize the host time table on the
 * GPU (kt_normalize), project the rows on their first m principal
 * components and quantize them (kt_pca), cluster with the integer k-means of
 * kt_kmeans_u16 (same seed, restarts and limits), and take one kernel per
 * cluster: KT_REP_CENTROID reads each centroid c back as the point
 * mean + V_m (lo + c span / 65535) and takes its largest Q16 value
 * rint(65535 x); KT_REP_GEOMEAN applies kt_representatives to the labels on
 * the normalized table.  Picks are distinct, in cluster order.  Workspace:
 * kt_prune_workspace_bytes(n_rows, n_configs, k, n_init).  Outputs (host):
 * chosen[k], *inertia_out (of the quantized k-means), optionally
 * labels[n_rows] and *explained.  Synchronizes `stream`. */
kt_status kt_prune_pca(kt_handle h, const int64_t* time_ns, int32_t n_rows, int32_t n_configs,
                       int32_t k, kt_norm norm, int32_t m, kt_rep rep, uint64_t seed,
                       int32_t n_init, int32_t max_iter, void* workspace, size_t ws_bytes,
                       void* stream, int32_t* chosen, int64_t* inertia_out, int32_t* labels,
                       double* explained);

/* k-means pruning (kt_prune) under each normalization of section 3.4,
 * keeping the one whose chosen set scores best on the same rows by the
 * paper's measure (kt_evaluate's geometric-mean ceiling; ties keep the
 * earlier normalization).  chosen[k], *norm_out and, if not NULL,
 * scores[4] (the ceiling of each normalization) are host outputs.
 * Workspace as kt_prune.  Synchronizes `stream`. */
kt_status kt_prune_auto(kt_handle h, const int64_t* time_ns, int32_t n_rows, int32_t n_configs,
                        int32_t k, uint64_t seed, int32_t n_init, int32_t max_iter,
                        void* workspace, size_t ws_bytes, void* stream, int32_t* chosen,
                        int32_t* norm_out, double* scores);

/* ------------------------------------------------------ evaluation (4.3) */

typedef struct {
  double geomean;       /* geometric mean of r = t_best / t_used: the paper's figure */
  double mean, min;
  double frac_ge_0_9;   /* share of rows with r >= 0.9 */
  double time_weighted; /* sum t_best / sum t_used */
  int32_t n;
} kt_eval;

/* Fraction of the optimal performance a selection keeps (section 4.3), on
 * a host time table [n_rows][n_configs] (t <= 0: unmeasured).  Evaluated rows:
 * rows[n_eval] (host), or every row when rows is NULL.  t_best is the row's
 * smallest measured time over all configurations; t_used is the time of
 * picks[e] for the e-th evaluated row when picks (host) is not NULL (a
 * selector's choice), else the smallest measured time among chosen[k] (the
 * ceiling of a pruned set).  KT_EINVAL when a row has no measured t_best or
 * t_used.  Host only. */
kt_status kt_evaluate(kt_handle h, const int64_t* time_ns, int32_t n_rows, int32_t n_configs,
                      const int32_t* rows, int32_t n_eval, const int32_t* picks,
                      const int32_t* chosen, int32_t k, kt_eval* out);

/* Top-N baseline of section 4.2: the k configurations that are best (largest
 * relative value, lowest index on ties) for the most rows, ties in the count
 * to the lower index.  time_ns and chosen are host arrays; the workspace is
 * sized by kt_prune_workspace_bytes(n_rows, n_configs, 1, 1).  Synchronizes
 * `stream`. */
kt_status kt_prune_topn(kt_handle h, const int64_t* time_ns, int32_t n_rows, int32_t n_configs,
                        int32_t k, void* workspace, size_t ws_bytes, void* stream,
                        int32_t* chosen);

/* ------------------------------------------------------------- selection */

typedef struct {
  int32_t steps;          /* full-batch Adam steps (default 3000) */
  float lr;               /* default 1e-3 */
  const float* init;      /* host, optional: W1 (64x6), b1, W2 (64x64), b2, W3 (k x 64), b3
                             packed in that order, row-major [out][in]; NULL = He-uniform
                             U(+-sqrt(6/fan_in)) from SplitMix64(seed), zero biases */
  uint64_t seed;
  int32_t graph_steps;    /* > 1: capture this many steps in a hipGraph and replay it;
                             0 or 1: launch every step directly */
} kt_mlp_opts;

/* Fit the runtime selector of one dtype on n_rows problems (section 5.1);
 * each dtype (its own configuration space and sweep table) has its own
 * selector, and kt_gemm(config_id = -1) asks the one of its input dtype.
 * shapes and
 * time_ns are host arrays; chosen[k] are the deployed configuration ids.
 * Each row is labelled with the fastest chosen configuration (lowest
 * position on equal times).  Decision trees are fitted on the host (integer
 * Gini CART on the raw features M, N, K, batch, transA, transB; split
 * thresholds floor(sqrt(a*b)) between consecutive values; x <= t goes left).
 * KT_SEL_MLP trains the cost model on the GPU (needs a device handle and a
 * workspace of kt_mlp_workspace_bytes).  KT_SEL_EXHAUSTIVE needs no data. */
kt_status kt_fit_selector(kt_handle h, kt_dtype dtype, kt_selector sel, const kt_shape* shapes,
                          const int64_t* time_ns, int32_t n_rows, int32_t n_configs,
                          const int32_t* chosen, int32_t k, const kt_mlp_opts* mlp,
                          void* workspace, size_t ws_bytes, void* stream);

/* Fit the selector of section 5.1 that generalizes best: decision trees A,
 * B, C and the MLP cost model are each fitted on the rows with
 * is_validation[i] == 0 (host array, n_rows) and scored on the others by the
 * geometric mean of t_best / t_picked (section 4.3; t_best over all
 * configurations of the row, the model's own pick without the fallback
 * below); the best (earliest kind on ties) is then refitted on all rows and
 * kept.  *kind_out receives it, scores[4] (optional, host) every kind's
 * validation score (0 for the MLP on a handle without a device, which
 * cannot train it).  Other arguments as kt_fit_selector. */
kt_status kt_fit_selector_validated(kt_handle h, kt_dtype dtype, const kt_shape* shapes,
                                    const int64_t* time_ns, int32_t n_rows, int32_t n_configs,
                                    const int32_t* chosen, int32_t k, const uint8_t* is_validation,
                                    const kt_mlp_opts* mlp, void* workspace, size_t ws_bytes,
                                    void* stream, int32_t* kind_out, double* scores);

/* Configuration id for a shape (host).  KT_ENOTFITTED before a fit or load,
 * except for KT_SEL_EXHAUSTIVE, which times every compiled configuration for
 * an unseen shape once (on scratch buffers the handle allocates) and caches
 * the winner.  Fallback (decision trees and MLP, on by default): a shape
 * whose M, N, K or batch lies outside the range the selector was fitted on
 * is not given to the model; the chosen configurations are timed on it once
 * (scratch as above, synchronizing) and the fastest is cached for the
 * shape.  Entry points that must not allocate keep the model's pick. */
kt_status kt_select(kt_handle h, kt_dtype dtype, const kt_shape* s, int32_t* config_id);

/* The out-of-range fallback of kt_select for the selector of a dtype (kept
 * across refits; saved by kt_save): 0 off (the model's pick stands), 1 (the
 * default) the chosen kernels and the split-K variants of their
 * configurations -- the code a deployed library holds --, 2 exhaustive:
 * every kernel this library holds (kt_num_kernels), timed once per shape and
 * cached like the exhaustive selector.  KT_EINVAL for another value. */
kt_status kt_set_fallback(kt_handle h, kt_dtype dtype, int32_t enabled);

/* The fitted selector of a dtype (host outputs, each optional): *kind
 * (kt_selector, -1 = none), *k and chosen[k] (pass NULL to query k first),
 * box[8] = the smallest then the largest M, N, K, batch it was fitted on
 * (0 ... -1 when unknown), *fallback. */
kt_status kt_selector_info(kt_handle h, kt_dtype dtype, int32_t* kind, int32_t* k,
                           int32_t* chosen, int64_t* box, int32_t* fallback);

/* Same for n shapes on the device: d_shapes and d_ids are device arrays.
 * Always the fitted model's pick (the out-of-range fallback of kt_select
 * times kernels on the host side and does not apply here). */
kt_status kt_select_batch(kt_handle h, kt_dtype dtype, const kt_shape* d_shapes, int32_t n,
                          int32_t* d_ids, void* stream);

/* Inspect the fitted tree: node arrays in pre-order (left child first);
 * feature = -1 marks a leaf, whose class indexes `chosen`.  Pass NULL arrays
 * to query *n_nodes only. */
kt_status kt_get_tree(kt_handle h, kt_dtype dtype, int32_t* n_nodes, int32_t* feature,
                      int64_t* threshold, int32_t* left, int32_t* right, int32_t* cls);

/* Save / load the selectors of every dtype that has one (kind, chosen ids,
 * tree or MLP weights) as a versioned text file.  kt_load returns KT_EIO for a missing or malformed
 * file and leaves the handle unchanged in that case. */
kt_status kt_save(kt_handle h, const char* path);
kt_status kt_load(kt_handle h, const char* path);

/* ------------------------------------------------- grouped GEMM (BF16) */

/* A batch of uneven GEMMs C_i = alpha * A_i * B_i + beta * C_i (BF16 A_i row-
 * major M x K, BF16 B_i row-major K x N, FP32 C_i row-major M x N; members
 * must have batch 1 and no transposes) run by one persistent kernel: the
 * members' output tiles form one work list that resident work-groups walk.
 * Members with M * N <= small_max_area take the smaller of the plan's two
 * tiles.  The kernel is captured with its setup in a hipGraph; one plan = one
 * graph launch per run.  Member leading dimensions: `ld` is a host array of
 * 3n values (lda_i >= K, ldb_i >= N, ldc_i >= N), or NULL for dense rows.  A
 * member whose A and B rows start on 16-byte boundaries (16-byte aligned
 * pointer, leading dimension a multiple of 8) and whose last 16-byte chunk of
 * a row ends within the leading dimension moves tiles by LDS DMA; its rows
 * are then read up to the next 16-byte boundary, so every row (the last one
 * included) must be allocated to its full leading dimension. */
typedef struct {
  int32_t config_id;        /* BF16 tile of the members (kt_get_config(KT_BF16, id)) */
  int32_t small_config_id;  /* BF16 tile of members with M * N <= small_max_area; -1 = none */
  int64_t small_max_area;
  int32_t schedule;         /* 0: static round robin over work-groups; 1: atomic work counter */
  int32_t order;            /* bit 0: members largest K first (else as given); bit 1: each
                               member's tiles in XCD blocks (its tile grid cut into 8
                               rectangles, interleaved so round-robin dispatch gives each XCD
                               one rectangle), else row by row */
  int32_t wgs_per_cu;       /* persistent work-groups per compute unit (1..4) */
  int32_t pipeline;         /* 0: members that allow it take the LDS-DMA pipeline (the kernel
                               then reserves its LDS); 1: every member register-staged (the
                               smaller LDS footprint keeps more work-groups resident) */
  uint32_t* visits;         /* optional device counters [n_work]: each work item adds 1 (tests) */
} kt_grouped_opts;

typedef struct kt_grouped_plan_s* kt_grouped_plan;

/* Device workspace for a group (descriptors, work list, counter). */
kt_status kt_grouped_workspace_bytes(const kt_shape* shapes, int32_t n, size_t* bytes);
/* Number of tile pairs (large, small) the grouped kernel is compiled for. */
kt_status kt_grouped_num_candidates(int32_t* n);
/* Build a plan: uploads descriptors and the work list into the workspace
 * (which must stay untouched while the plan lives) and captures the graph.
 * A, B, C are host arrays of n device pointers.  opts NULL = the options the
 * autotuner found on this handle, else a default.  KT_EUNSUPPORTED for a
 * tile pair that is not compiled.  Synchronizes `stream`. */
kt_status kt_grouped_plan_create(kt_handle h, kt_dtype dtype, const kt_shape* shapes, int32_t n,
                                 const void* const* A, const void* const* B, float* const* C,
                                 const int64_t* ld, float alpha, float beta,
                                 const kt_grouped_opts* opts, void* workspace, size_t ws_bytes,
                                 void* stream, kt_grouped_plan* out);
/* One graph launch of the plan on `stream` (asynchronous). */
kt_status kt_grouped_plan_launch(kt_handle h, kt_grouped_plan plan, void* stream);
/* Work-list length and options of a plan. */
kt_status kt_grouped_plan_info(kt_grouped_plan plan, int32_t* n_work, kt_grouped_opts* opts);
kt_status kt_grouped_plan_destroy(kt_grouped_plan plan);
/* Plan, launch once, synchronize, destroy. */
kt_status kt_grouped_gemm(kt_handle h, kt_dtype dtype, const kt_shape* shapes, int32_t n,
                          const void* const* A, const void* const* B, float* const* C,
                          const int64_t* ld, float alpha, float beta, const kt_grouped_opts* opts,
                          void* workspace, size_t ws_bytes, void* stream);
/* The library's autotuner: successive halving over (tile pair, small-member
 * area in {0, 128^2, 256^2, 512^2}, schedule, order (all four values), work-groups per CU,
 * pipeline -- DMA only when some member allows it),
 * timing whole graph launches of the real group (C is overwritten with
 * alpha = 1, beta = 0).  The winner is returned and kept on the handle as the
 * default for later plans. */
kt_status kt_autotune_grouped(kt_handle h, kt_dtype dtype, const kt_shape* shapes, int32_t n,
                              const void* const* A, const void* const* B, float* const* C,
                              const int64_t* ld, void* workspace, size_t ws_bytes, void* stream,
                              kt_grouped_opts* best, float* best_ms, int32_t* evaluations);

/* ------------------------------------------------------- MLP cost model */

/* The learned selector: 6 -> 64 -> 64 -> k network (ReLU, linear output) on
 * features [log2 M/12, log2 N/12, log2 K/12, log2 batch/6, transA, transB]
 * regressing the relative performance of the k chosen kernels (MSE); the
 * selection is the argmax.  Parameters are packed W1 b1 W2 b2 W3 b3 (FP32). */

/* Workspace bytes for kt_fit_selector(KT_SEL_MLP). */
kt_status kt_mlp_workspace_bytes(int32_t n_rows, int32_t n_configs, int32_t k, size_t* bytes);
/* Number of packed parameters for k outputs (5128 for k = 8). */
kt_status kt_mlp_num_params(int32_t k, int32_t* n_params);
/* Features of n device shapes into d_X[n][6] (device, FP32). */
kt_status kt_mlp_features(kt_handle h, const kt_shape* d_shapes, int32_t n, float* d_X, void* stream);
/* One full-batch forward (and backward) pass with the training kernels, at
 * the given device parameters: predictions d_pred[n][k] (optional), the
 * gradient of the mean squared error w.r.t. every parameter d_grad (optional,
 * packed like the parameters) and the sum of squared errors d_loss[0]
 * (optional; the loss is that over n*k).  Gradients need d_Y[n][k] and a
 * workspace of nblocks*(n_params*4) + nblocks*4 bytes (256-aligned parts),
 * nblocks = ceil(n / 32); kt_mlp_workspace_bytes is always enough. */
kt_status kt_mlp_forward_backward(kt_handle h, const float* d_params, const float* d_X,
                                  const float* d_Y, int32_t n, int32_t k, float* d_pred,
                                  float* d_grad, float* d_loss, void* workspace, size_t ws_bytes,
                                  void* stream);
/* Copy the fitted MLP parameters (host).  NULL params queries *n_params. */
kt_status kt_get_mlp(kt_handle h, kt_dtype dtype, int32_t* n_params, float* params);

#ifdef __cplusplus
}
#endif

#endif /* KT_H */
