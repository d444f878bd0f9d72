/*
 * libbitrev -- the bit-reversed permutation of n = 2^k elements on AMD
 * Instinct MI355X (gfx950).  C ABI.
 *
 * The operation (arXiv:1708.01873, Introduction): for an array of n = 2^k
 * elements, the element at index i moves to index rev_k(i), where rev_k
 * reverses exactly the low k bits of i (n = 8: 0 1 2 3 4 5 6 7 becomes
 * 0 4 2 6 1 5 3 7).  rev_k(rev_k(i)) = i, so the permutation is its own
 * inverse and its own adjoint, and it can be done in place by swapping each
 * pair i < rev_k(i) once.
 *
 * Elements are opaque blocks of elem_size bytes (1, 2, 4, 8 or 16); their
 * bits are moved, never interpreted, so results are byte-exact for any type
 * (integers, floats including NaN payloads and signed zeros, complex pairs).
 *
 * Conventions for every entry point:
 *   - Data pointers are DEVICE pointers (memory from hipMalloc or an
 *     allocator built on it) on the current HIP device.  The caller owns all
 *     memory: data, workspace and stream.  The library never allocates, frees
 *     or synchronises on these paths, so they may be captured into a HIP graph.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Work is enqueued asynchronously on it, in stream order.
 *   - Argument errors are detected on the host and returned before any HIP
 *     call is made; nothing is enqueued then.  A failed launch returns
 *     BITREV_ERROR_HIP and bitrev_last_hip_error() holds the hipError_t of the
 *     calling thread.
 *   - No C++ exception crosses this interface.  Calls are thread-safe.
 */
#ifndef BITREV_H
#define BITREV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BITREV_ABI_VERSION 2
#define BITREV_MAX_LOG2N 40

typedef enum bitrev_status {
  BITREV_SUCCESS = 0,
  /* a null pointer, log2n outside [0, BITREV_MAX_LOG2N], elem_size not in
   * {1,2,4,8,16}, a pointer not aligned to elem_size, a negative count, or a
   * config field out of range */
  BITREV_ERROR_INVALID_VALUE = 1,
  /* source and destination ranges overlap: use the in-place entry point */
  BITREV_ERROR_ALIAS = 2,
  /* batched workspace missing, misaligned or smaller than
   * bitrev_batched_workspace_size(); or more arrays than the built-in
   * scratch of bitrev_batched_noalloc holds */
  BITREV_ERROR_WORKSPACE = 3,
  /* a HIP runtime call or kernel launch failed; see bitrev_last_hip_error() */
  BITREV_ERROR_HIP = 4,
  /* valid arguments that this build cannot run: a forced tile width that is
   * not compiled or whose LDS does not fit the device, or more than 2^32
   * middle-bit tiles */
  BITREV_ERROR_NOT_SUPPORTED = 5
} bitrev_status_t;

/* Optional launch configuration for the *_ex entry points.  A zero field
 * means "library choice" (tuning table, else built-in default). */
typedef struct bitrev_config {
  int tile_bits;   /* b: tiles of 2^b x 2^b elements, 0..7 (0 = choose); the
                    * method splits the index bits as [high b | middle | low b] */
  int grid_blocks; /* workgroups launched; >0 makes the kernel loop over its
                    * work items with a grid stride (persistent); 0 = choose */
  int order;       /* work-item order: 0 = choose, 1 = natural, 2 = balanced
                    * bit dealing (spreads tile rows over HBM channels),
                    * 3 = grouped (the tile index y = [t | c | s] with t and
                    * s of 3 bits: in place, the pairs of the 64 tiles that
                    * share their middle bits c run together; out of place,
                    * (t, s) vary fastest and c is dealt as in the balanced
                    * order; either way both sides of the permutation touch
                    * runs of neighbouring tiles) */
  int variant;     /* tile kernel: 0 = choose, 1 = one work item per
                    * workgroup, 2 = persistent and software-pipelined (each
                    * workgroup loads its next tiles while storing the
                    * current ones; grid = resident workgroups unless
                    * grid_blocks is set), 3 = register-staged (in place:
                    * half the threads hold the pair in registers and
                    * transpose its tiles in turn through one LDS tile, so
                    * twice the pairs are in flight per compute unit; out of
                    * place it is variant 1) */
  int xcd_remap;   /* 0 = choose, 1 = give each XCD a contiguous range of work
                    * items (the dispatcher deals workgroups to the XCDs round
                    * robin), 2 = leave the dispatch order as is */
  int cache_hints; /* tile kernels' global accesses: 0 = choose, 1 = plain,
                    * 2 = streaming (non-temporal) loads, 3 = streaming
                    * stores, 4 = streaming loads and write-through stores
                    * (device scope: each written line goes through the
                    * XCD's L2 to the memory side instead of staying dirty
                    * there); applies to the one-item and register-staged
                    * tile kernels with 16-byte accesses, otherwise plain.
                    * The choice: plain below 32 MiB out of place and 64 MiB
                    * in place; streaming loads for 1- and 2-byte elements
                    * beyond 256 MiB and for 4-byte elements out of place
                    * at 128-256 MiB; 4 otherwise */
} bitrev_config_t;

/* Which code path and geometry a call uses (bitrev_plan_query). */
typedef enum bitrev_path {
  BITREV_PATH_NONE = 0,  /* nothing to do (in place with n <= 2, or no rows) */
  BITREV_PATH_WAVE = 1,  /* n <= 64: one wavefront per array, lane shuffles */
  BITREV_PATH_TILE = 2,  /* tiles of 2^b x 2^b staged through LDS */
  BITREV_PATH_BATCHED = 3 /* persistent batched kernel (tiles + whole-array LDS) */
} bitrev_path_t;

typedef struct bitrev_plan {
  int path;             /* bitrev_path_t */
  int tile_bits;        /* b */
  int mid_bits;         /* m = log2n - 2b */
  int block_threads;    /* threads per workgroup */
  int grid_blocks;      /* workgroups launched */
  int order;            /* 1 natural, 2 balanced, 3 grouped */
  int vector_access;    /* 1: 16-byte global accesses; 0: one element per access */
  int variant;          /* 1 one item per workgroup, 2 persistent pipelined, 3 register-staged */
  int xcd_remap;        /* 1 contiguous ranges per XCD, 2 dispatch order */
  int cache_hints;      /* 1 plain, 2 streaming loads, 3 streaming stores,
                         * 4 streaming loads and write-through stores */
  uint64_t work_items;  /* tile pairs (in place) or tiles (out of place), all rows */
  uint64_t lds_bytes;   /* LDS per workgroup */
} bitrev_plan_t;

/* ------------------------------------------------------------------------ */
/* Plain permutations                                                        */
/* ------------------------------------------------------------------------ */

/* In place: data[0 .. 2^log2n) is replaced by its bit-reversed permutation
 * (Introduction: swap i and rev(i) once per pair).  data is a device
 * pointer to 2^log2n contiguous elements of elem_size bytes, aligned to
 * elem_size. */
bitrev_status_t bitrev_inplace(void* data, int log2n, size_t elem_size, void* stream);

/* Out of place: dst[rev(i)] = src[i] for every i < 2^log2n (Introduction,
 * the buffered method's out-of-place statement).  src and dst are device
 * pointers to non-overlapping arrays of 2^log2n elements; overlapping ranges
 * return BITREV_ERROR_ALIAS. */
bitrev_status_t bitrev_outofplace(const void* src, void* dst, int log2n, size_t elem_size,
                                  void* stream);

/* `rows` independent arrays of 2^log2n elements stored back to back
 * (row-major [rows][2^log2n]); each row is permuted on its own.
 * src == dst means in place; otherwise the two ranges must not overlap.
 * rows == 0 is a no-op.  This is the forward and the backward of the
 * differentiable form: the permutation's adjoint is itself. */
bitrev_status_t bitrev_rows(const void* src, void* dst, int log2n, int64_t rows,
                            size_t elem_size, void* stream);

/* Strided rows: `rows` arrays of 2^log2n elements, array r starting at
 * element r * src_stride of src and r * dst_stride of dst (strides in
 * elements, >= 2^log2n).  src == dst (equal strides) is in place; otherwise
 * the spans [src, src + ((rows-1) src_stride + 2^log2n) elem_size) and the
 * same for dst must not overlap (BITREV_ERROR_ALIAS, a conservative check). */
bitrev_status_t bitrev_rows_strided(const void* src, void* dst, int log2n, int64_t rows,
                                    int64_t src_stride, int64_t dst_stride, size_t elem_size,
                                    void* stream);

/* One even-odd split per row, out of place (Introduction: the Stockham
 * auto-sort's step, the n/2 x 2 matrix transposition): dst[j] = src[2j] and
 * dst[n/2 + j] = src[2j + 1] for j < n/2, each of `rows` contiguous rows of
 * n = 2^log2n >= 2 elements.  Applied to nested halves log2n times it gives
 * the bit-reversed order.  src and dst must not overlap. */
bitrev_status_t bitrev_evenodd(const void* src, void* dst, int log2n, int64_t rows,
                               size_t elem_size, void* stream);

/* ------------------------------------------------------------------------ */
/* Batched: many arrays of different lengths in one persistent launch        */
/* ------------------------------------------------------------------------ */

/* Bytes of device workspace bitrev_batched needs for num_arrays arrays
 * ((num_arrays + 3) * 8, rounded up to 256).  Returns 0 for num_arrays < 0. */
size_t bitrev_batched_workspace_size(int64_t num_arrays);

/* In place, every array a in [0, num_arrays): the elements
 * data[offsets[a] .. offsets[a+1]) (counted in elements of elem_size bytes)
 * are replaced by their bit-reversed permutation of length 2^log2n[a].
 *   data       device pointer, data_elems elements, aligned to elem_size
 *   offsets    device pointer, num_arrays + 1 int64 (CSR style)
 *   log2n      device pointer, num_arrays int32
 *   workspace  device pointer, >= bitrev_batched_workspace_size(num_arrays)
 *              bytes, 8-byte aligned; owned by the caller, overwritten, and
 *              holds after the call: [0] the number of arrays rejected,
 *              [1] the first rejected array (or -1) -- see
 *              bitrev_batched_errors()
 * Two kernels are enqueued: a one-workgroup prep kernel that checks every
 * array (offsets[a+1] - offsets[a] == 2^log2n[a], 0 <= offsets[a],
 * offsets[a+1] <= data_elems, 0 <= log2n[a] <= BITREV_MAX_LOG2N) and scans
 * the per-array work counts into the workspace, then the persistent kernel.
 * A rejected array is left untouched; the others are still permuted.
 * Arrays must not overlap (the length check makes valid ones disjoint). */
bitrev_status_t bitrev_batched(void* data, int64_t data_elems, const int64_t* offsets,
                               const int32_t* log2n, int64_t num_arrays, size_t elem_size,
                               void* workspace, size_t workspace_bytes, void* stream);

/* Out of place: dst[offsets[a] + rev(i)] = src[offsets[a] + i] for every
 * array, src and dst sharing one packed layout of data_elems elements (the
 * two ranges must not overlap: BITREV_ERROR_ALIAS).  Arrays with n <= 2 are
 * copied.  Otherwise as bitrev_batched (workspace, checks, rejection). */
bitrev_status_t bitrev_batched_outofplace(const void* src, void* dst, int64_t data_elems,
                                          const int64_t* offsets, const int32_t* log2n,
                                          int64_t num_arrays, size_t elem_size, void* workspace,
                                          size_t workspace_bytes, void* stream);

/* Synchronous debug helper: waits for `stream`, then reads the rejection
 * count and first rejected array that the last bitrev_batched on this
 * workspace wrote.  Either output pointer may be NULL. */
bitrev_status_t bitrev_batched_errors(const void* workspace, int64_t* num_rejected,
                                      int64_t* first_rejected, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * in-place batched permutation as bitrev_batched with the built-in plan, with
 * its workspace taken from a fixed array inside the library instead of from
 * the caller.  No allocating call of any kind is made.
 *   data, data_elems, offsets, log2n, num_arrays, elem_size, stream: as
 *   bitrev_batched; the caller still owns data, offsets and log2n.
 *   num_arrays <= BITREV_NOALLOC_MAX_ARRAYS (65536), else
 *   BITREV_ERROR_WORKSPACE before any HIP call.
 * The array (bitrev_batched_workspace_size(BITREV_NOALLOC_MAX_ARRAYS) =
 * 524,544 bytes, 512 KiB and 256 bytes) exists once
 * per GPU the library runs on and is held until the process ends.  Every call
 * on one GPU uses that GPU's array and leaves its contents behind; each call
 * rewrites all of it that it reads, so nothing has to be cleared between
 * calls.  Calls that overlap in time on one GPU (other streams, other
 * threads) race on the array: serialise them.  Rejected arrays are left
 * untouched as in bitrev_batched, but the rejection count is not readable
 * (bitrev_batched_errors needs a caller-owned workspace). */
#define BITREV_NOALLOC_MAX_ARRAYS 65536
bitrev_status_t bitrev_batched_noalloc(void* data, int64_t data_elems, const int64_t* offsets,
                                       const int32_t* log2n, int64_t num_arrays, size_t elem_size,
                                       void* stream);

/* ------------------------------------------------------------------------ */
/* Explicit configuration (autotuner, tile-width sweeps)                     */
/* ------------------------------------------------------------------------ */

/* As the plain calls, with a launch configuration (NULL = library choice).
 * A tile width that is not compiled for elem_size, or whose LDS does not fit
 * the device, returns BITREV_ERROR_NOT_SUPPORTED. */
bitrev_status_t bitrev_inplace_ex(void* data, int log2n, size_t elem_size,
                                  const bitrev_config_t* cfg, void* stream);
bitrev_status_t bitrev_outofplace_ex(const void* src, void* dst, int log2n, size_t elem_size,
                                     const bitrev_config_t* cfg, void* stream);
/* Kernel timing for measurement: as bitrev_inplace_ex / bitrev_outofplace_ex,
 * and the launch of the call's one kernel records start_event as the kernel
 * starts and stop_event as it ends (hipExtLaunchKernel), so that
 * hipEventElapsedTime between them is the kernel's own duration, without the
 * dispatch latency that events recorded on the stream around the call also
 * include.  Both events are the caller's (hipEvent_t created with timing
 * enabled); both must be given (else BITREV_ERROR_INVALID_VALUE).  Where the
 * call runs no kernel the events are recorded back to back.  This launch path
 * adds dispatch latency on the stream (about 9 us measured on MI355X), so it
 * times the kernel, not the throughput of a sequence of calls.  Events from
 * bitrev_timing_event_create bracket the kernel alone; events created with
 * default flags also include the writeback of the L2 that their system-scope
 * fence performs (2-3 us after a 128 MiB in-place call on MI355X). */
bitrev_status_t bitrev_inplace_timed(void* data, int log2n, size_t elem_size,
                                     const bitrev_config_t* cfg, void* start_event,
                                     void* stop_event, void* stream);
bitrev_status_t bitrev_outofplace_timed(const void* src, void* dst, int log2n, size_t elem_size,
                                        const bitrev_config_t* cfg, void* start_event,
                                        void* stop_event, void* stream);
/* Events for the *_timed entries.  bitrev_timing_event_create makes a HIP
 * event with timing enabled and the system-scope fence disabled
 * (hipEventDisableSystemFence): reaching it does not write back the L2, so
 * it timestamps the kernel's end rather than the end of that writeback.  It
 * is for timing only: it does not make the kernel's results visible to the
 * host or to other devices.  The caller owns the event and frees it with
 * bitrev_timing_event_destroy (NULL is a no-op).  bitrev_timing_elapsed_ms
 * waits for stop_event and writes the milliseconds between the two events to
 * *ms.  NULL arguments return BITREV_ERROR_INVALID_VALUE (create: event;
 * elapsed: any); HIP failures return BITREV_ERROR_HIP. */
bitrev_status_t bitrev_timing_event_create(void** event);
bitrev_status_t bitrev_timing_event_destroy(void* event);
bitrev_status_t bitrev_timing_elapsed_ms(void* start_event, void* stop_event, float* ms);
bitrev_status_t bitrev_rows_ex(const void* src, void* dst, int log2n, int64_t rows,
                               size_t elem_size, const bitrev_config_t* cfg, void* stream);
bitrev_status_t bitrev_batched_ex(void* data, int64_t data_elems, const int64_t* offsets,
                                  const int32_t* log2n, int64_t num_arrays, size_t elem_size,
                                  void* workspace, size_t workspace_bytes,
                                  const bitrev_config_t* cfg, void* stream);

/* The plan a call would use, without launching anything.  mode: 0 in place,
 * 1 out of place, 2 batched (log2n ignored).  Uses the current device's
 * properties when a device is present, else MI355X figures (gfx950, 256
 * compute units, 160 KiB LDS). */
bitrev_status_t bitrev_plan_query(int log2n, size_t elem_size, int64_t rows, int mode,
                                  const bitrev_config_t* cfg, bitrev_plan_t* plan);

/* Load a tuning table (text; see bitrev_tuning_format()).  NULL restores the
 * built-in defaults.  Its plan rows have the built-in table's form: each is
 * keyed by device (gcnArchName, compute units), kind of launch, element size
 * and size class, so rows tuned on one device or partition mode do not apply
 * on another; they are consulted before the built-in rows.  Exact entries
 * keyed by (mode, element size, log2n) override both.  A file that cannot be
 * read or has a malformed line is rejected with BITREV_ERROR_INVALID_VALUE
 * and the table in use is kept.  If the environment variable
 * BITREV_TUNING_FILE names a file, it is loaded at the first call that needs
 * a plan. */
bitrev_status_t bitrev_load_tuning(const char* path);

/* One line describing the tuning file's format. */
const char* bitrev_tuning_format(void);

/* ------------------------------------------------------------------------ */
/* Digit reversal for radix-4 and radix-8 FFTs                               */
/* ------------------------------------------------------------------------ */

/* The permutation a radix-2^d decimation-in-time FFT needs: the order of the
 * d-bit digits of each index is reversed (each digit keeps its bits); the
 * paper's bit reversal is d = 1 (Introduction: the reversal performs the
 * FFT's recursive index splits up front -- a radix-2^d FFT splits by 2^d
 * residues per level).  It is an involution too, so in place it swaps pairs.
 * digit_bits in {1, 2, 3}; log2n must be a multiple of digit_bits, else
 * BITREV_ERROR_INVALID_VALUE.  Other arguments as bitrev_inplace and
 * bitrev_outofplace; same tile method with tile widths and the middle width
 * whole numbers of digits. */
bitrev_status_t bitrev_digitrev_inplace(void* data, int log2n, int digit_bits, size_t elem_size,
                                        void* stream);
bitrev_status_t bitrev_digitrev_outofplace(const void* src, void* dst, int log2n, int digit_bits,
                                           size_t elem_size, void* stream);
/* With a launch configuration (NULL = library choice): tile_bits must be a
 * multiple of digit_bits (else BITREV_ERROR_NOT_SUPPORTED, as for a width
 * that is not compiled or does not fit); order sets the source-tile order out
 * of place (in place the pairs follow the grouped digit order); grid_blocks,
 * xcd_remap and cache_hints as in bitrev_config_t; variant is ignored.  A
 * config field out of range returns BITREV_ERROR_INVALID_VALUE. */
bitrev_status_t bitrev_digitrev_inplace_ex(void* data, int log2n, int digit_bits,
                                           size_t elem_size, const bitrev_config_t* cfg,
                                           void* stream);
bitrev_status_t bitrev_digitrev_outofplace_ex(const void* src, void* dst, int log2n,
                                              int digit_bits, size_t elem_size,
                                              const bitrev_config_t* cfg, void* stream);

/* ------------------------------------------------------------------------ */
/* Bit reversal fused with the first FFT levels                              */
/* ------------------------------------------------------------------------ */

/* `rows` arrays of 2^log2n complex elements (dtype 0: complex64, two float32;
 * 1: complex128, two float64; interleaved real, imaginary), each replaced by
 * its bit-reversed permutation followed by the first `stages` levels of a
 * radix-2 decimation-in-time FFT (the paper's motivation, Introduction: the
 * reversal performs all even-odd splits up front, after which each FFT level
 * works on contiguous blocks).  Afterwards every block of 2^stages
 * consecutive outputs J holds the length-2^stages DFT of the subsequence
 * x[rev(J) + 2^(log2n - stages) u], u = 0 .. 2^stages - 1, with twiddles
 * exp(-2 pi i / 2^s) (inverse = 1: exp(+2 pi i / 2^s), unscaled).  The first
 * levels (up to three, where a thread's loads hold whole blocks of them) run
 * in registers between the loads and the LDS stage, the others on the tile
 * rows staged in LDS, so the HBM traffic is that of the plain permutation.  src == dst is in place; otherwise the ranges must not overlap.
 * 0 <= stages <= min(floor(log2n / 2), 6), else BITREV_ERROR_NOT_SUPPORTED;
 * stages = 0 is bitrev_rows.  Arithmetic in the element's precision with
 * twiddles rounded once from double precision. */
bitrev_status_t bitrev_dit_stages(const void* src, void* dst, int log2n, int64_t rows, int stages,
                                  int inverse, int dtype, void* stream);
/* The same with a launch configuration: tile_bits (>= stages; the default
 * is the plain kernel's width, at least stages), order, grid_blocks,
 * xcd_remap and cache_hints as in bitrev_config_t.  variant: 0 = choose,
 * 1 = square tiles of 2^b x 2^b, 2 and 3 = out of place only, rectangular
 * tiles: the index split as [high b | middle | low b - 1] (variant 2) or
 * [high b | middle | low b - 2] (variant 3), so a tile is 2^b source rows
 * of 2^(b-1) or 2^(b-2) elements landing as destination rows of 2^b
 * outputs, the levels' blocks, with a half or a quarter of the square
 * tile's LDS and threads; b = 5 or 6 and 16-byte aligned arrays, else
 * BITREV_ERROR_NOT_SUPPORTED.  In place (square tiles only: a rectangular
 * tile's image is not a tile of the same shape) variant 3 keeps the tile
 * pair in registers and stages its tiles through one LDS tile in turn, with
 * half the threads (2b <= log2n, else BITREV_ERROR_NOT_SUPPORTED);
 * variant 2 in place returns BITREV_ERROR_NOT_SUPPORTED.  stages = 0 runs bitrev_rows_ex with this
 * config, its variant ignored (and a tile width too wide for square tiles
 * left to the plan). */
bitrev_status_t bitrev_dit_stages_ex(const void* src, void* dst, int log2n, int64_t rows,
                                     int stages, int inverse, int dtype,
                                     const bitrev_config_t* cfg, void* stream);

/* ------------------------------------------------------------------------ */
/* The paper's recursive scheme, as an A/B baseline for the one-pass kernels */
/* ------------------------------------------------------------------------ */

/* In place, by the paper's cache-oblivious recursive method (Methods,
 * "cache-oblivious recursive bit-reversed permutation"; Results, where its
 * GPU variant recurses twice and needs k divisible by 4): with k = log2n
 * even and h = k/2, (1) reverse the low h bits within each of the 2^h
 * contiguous blocks, (2) transpose the 2^h x 2^h matrix in place, (3)
 * reverse within each block again.  levels = 2: the block reversals of (1)
 * and (3) recurse once more -- each block is staged in LDS and reversed
 * there by the same three steps on h/2 bits -- which needs h even and a
 * block of at most 64 KiB (2^h * elem_size), else BITREV_ERROR_NOT_SUPPORTED.
 * levels = 1: the block reversals are the one-pass tile kernels.  levels = 0:
 * two where they apply, else one.  Three passes over the array (3 * 2 n s
 * bytes) either way, where bitrev_inplace makes one; the result is
 * identical.  Odd log2n returns BITREV_ERROR_NOT_SUPPORTED (the paper's
 * odd-k pre-step needs an n/2 buffer).  Other arguments as bitrev_inplace;
 * levels outside 0..2 returns BITREV_ERROR_INVALID_VALUE. */
bitrev_status_t bitrev_inplace_recursive_ex(void* data, int log2n, size_t elem_size, int levels,
                                            void* stream);
/* bitrev_inplace_recursive_ex with levels = 0. */
bitrev_status_t bitrev_inplace_recursive(void* data, int log2n, size_t elem_size, void* stream);

/* In-place transpose of a square 2^log2side x 2^log2side row-major matrix of
 * elem_size-byte elements (the middle step above): element (r, c) moves to
 * (c, r).  2 * log2side <= BITREV_MAX_LOG2N. */
bitrev_status_t bitrev_transpose_inplace(void* data, int log2side, size_t elem_size, void* stream);

/* ------------------------------------------------------------------------ */
/* Reference copy (the HBM roofline denominator), status, version            */
/* ------------------------------------------------------------------------ */

/* dst[0 .. bytes) = src[0 .. bytes): a plain streaming copy with the same
 * byte count as an out-of-place permutation, used to measure attainable HBM
 * bandwidth.  Ranges must not overlap.  bitrev_copy takes the cache hint
 * measured fastest (streaming loads and write-through stores, at 128 MiB and
 * at 4 GiB); bitrev_copy_ex takes it from cache_hints as in bitrev_config_t
 * (0 = that choice). */
bitrev_status_t bitrev_copy(const void* src, void* dst, size_t bytes, void* stream);
bitrev_status_t bitrev_copy_ex(const void* src, void* dst, size_t bytes, int cache_hints,
                               void* stream);

/* The reference copy in the tile kernels' order: dst = src for 2^log2n
 * elements of elem_size bytes, visiting the tiles of the out-of-place plan
 * (tile width b, tile order, XCD mapping, cache hints and grid from cfg or
 * the plan's own choice; variant is ignored) and copying each tile's 2^b
 * rows of 2^b elements to the same place of dst.  It reads exactly what the
 * out-of-place permutation reads, in the same order and row shape, and
 * writes rows of the same shape, without the LDS stage: a copy that walks
 * memory the way the tile kernels do, used with the linear copy to bound the
 * permutation (on MI355X a linear sweep over multi-GiB arrays is slower than
 * the tile order).  src and dst must not overlap (BITREV_ERROR_ALIAS) and
 * must be aligned to elem_size; a base that is not 16-byte aligned (or, for
 * rows shorter than 16 bytes, aligned to the row) returns
 * BITREV_ERROR_NOT_SUPPORTED.  Arrays of at most 64 elements are copied
 * linearly. */
bitrev_status_t bitrev_copy_tiled(const void* src, void* dst, int log2n, size_t elem_size,
                                  const bitrev_config_t* cfg, void* stream);

const char* bitrev_status_string(bitrev_status_t status);
int bitrev_last_hip_error(void);
int bitrev_abi_version(void);

/* ------------------------------------------------------------------------ */
/* Host mirrors of the kernels' index arithmetic (the same source, compiled */
/* for the host), so that tests can check it on a machine without a GPU.     */
/* ------------------------------------------------------------------------ */

/* rev_j(v): the low j bits of v reversed, 0 <= j <= 32. */
uint32_t bitrev_debug_rev(uint32_t v, int j);
/* Number of tile pairs {y, rev_m(y)} with y <= rev_m(y), 0 <= m <= 32. */
uint64_t bitrev_debug_pair_count(int m);
/* The w-th such y in the kernels' enumeration order (balanced: 0 or 1). */
uint32_t bitrev_debug_pair_at(int m, uint64_t w, int balanced);
/* The w-th tile of the in-place kernels' order (the other tile of its pair
 * is its reversal): order 1 natural, 2 balanced, 3 grouped -- see
 * bitrev_config_t.order.  0xFFFFFFFF when m, w or order is out of range. */
uint32_t bitrev_debug_inplace_pair_at(int m, uint64_t w, int order);
/* The w-th source tile of the out-of-place kernels' order (1 natural,
 * 2 balanced, 3 grouped); 0xFFFFFFFF when m, w or order is out of range. */
uint32_t bitrev_debug_oop_tile_at(int m, uint32_t w, int order);
/* The balanced bit dealing of a width-bit value. */
uint32_t bitrev_debug_spread(uint32_t w, int width);
/* The w-th tile pair (r <= c) of the square transpose, column by column. */
void bitrev_debug_tri_pair(uint64_t w, uint32_t* r, uint32_t* c);
/* Digit reversal of the low j bits of v in d-bit digits (j a multiple of d). */
uint32_t bitrev_debug_digit_rev(uint32_t v, int j, int d);
/* Number of y in [0, 2^m) with y <= drev(y), and the w-th such y. */
uint64_t bitrev_debug_digit_pair_count(int m, int d);
uint32_t bitrev_debug_digit_pair_at(int m, uint64_t w, int d);
/* The w-th tile of the in-place digit kernels' order (grouped; the other
 * tile of its pair is its digit reversal). */
uint32_t bitrev_debug_digit_inplace_pair_at(int m, uint64_t w, int d);

#ifdef __cplusplus
}
#endif

#endif /* BITREV_H */
