/*
 * curvealign.h -- C ABI of the MI355X (gfx950) closed-curve alignment library.
 *
 * The library computes, for pairs of closed planar curves given as n uniform
 * arc-length nodes each, the optimal starting point and rotation of
 * Dogan, Bernal and Hagwood, "FFT-based alignment of 2d closed curves with
 * application to elastic shape analysis", section 2 (Algorithm 2), and the
 * mismatch energy of Eq. (disc-energy) at that optimum.  It also provides the
 * uniform arc-length resampling of section 2 (Eq. arc-length-param followed
 * by cubic-spline interpolation) that turns raw vertex lists into such nodes.
 *
 * Curves are complex signals z[k] = x_k + i y_k.  For a pair (z1, z2) with n
 * nodes the library evaluates the circular cross-correlation
 *     C(s) = sum_k z1[k] conj(z2[(k - s) mod n]),   s = 0..n-1,
 * (the FFT route: C = IFFT(FFT(z1) . conj(FFT(z2)))) and returns
 *     shift  = argmax_s |C(s)|            (smallest s among exact ties)
 *     theta  = arg C(shift)               (counter-clockwise rotation applied to z2)
 *     e0     = n1 + n2 - 2 |C(shift)| / n,  n_i = (1/n) sum_k |z_i[k]|^2.
 * In the paper's notation (start index m, t0 = m/n, clockwise R(theta)) the
 * same optimum reads m = (n - shift) mod n and theta_paper = -theta; e0 is
 * E^h(t0, R) of Eq. (disc-energy) with h = 1/n.  |C(s)| is the value of
 * tr(R A^T) maximised over R for A = A(t_m) of Eq. (A-mtx).
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers (hipMalloc'ed or torch CUDA
 *     tensors) owned by the caller, unless stated otherwise.  The library
 *     never frees or retains them.
 *   - Complex arrays are interleaved: float pairs (complex64) for the FP32 and
 *     split-BF16 precisions, double pairs (complex128) for FP64.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Every call is stream-ordered and asynchronous: it validates arguments on
 *     the host, enqueues kernels and returns.  Results are ready when the
 *     stream is synchronised.
 *   - Errors: a negative status means nothing was enqueued (argument errors are
 *     detected synchronously on the host) or, for CA_ERR_HIP, that a HIP call
 *     failed (ca_last_error() has the text).  Data conditions never fail a
 *     call: they set per-result flags (CA_FLAG_*).
 *   - A context is not thread-safe; use one per host thread.  Calls that
 *     share a context must be issued to the same stream or be serialised
 *     by the caller (they share the context's workspace).
 */
#ifndef CURVEALIGN_H
#define CURVEALIGN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ca_status_t;
enum {
    CA_OK = 0,
    CA_ERR_INVALID_ARG = -1,   /* null pointer, negative count, bad option value  */
    CA_ERR_UNSUPPORTED_N = -2, /* n outside the supported set (see align_batch)   */
    CA_ERR_HIP = -3,           /* a HIP runtime call failed; see ca_last_error()  */
    CA_ERR_OOM = -4,           /* workspace allocation failed                    */
    CA_ERR_NO_DEVICE = -5,     /* no gfx950 device at the requested index        */
    CA_ERR_INTERNAL = -6,
    CA_ERR_TOO_LARGE = -7      /* input exceeds the static scratch of an
                                  allocation-free entry point                  */
};

/* Per-pair result: 32 bytes, 8-byte aligned. */
typedef struct {
    int32_t shift;    /* optimal correlation shift s* in [0, n)                      */
    uint32_t flags;   /* CA_FLAG_* bits                                              */
    double theta;     /* arg C(s*), radians in (-pi, pi]: the arc tangent of the
                         FP64 re-scored C(s*), taken in FP32 on the FP32 and
                         split-BF16 paths and in FP64 on the FP64 path or when
                         theta_fp64 is set                                             */
    double e0;        /* n1 + n2 - 2|C(s*)|/n with |C(s*)| and n_i in FP64           */
    float err_est;    /* relative half-width of the path's |C| error bound at s*     */
    float gap;        /* (|C|best - |C|runner-up) / |C|best, FP64 values when more
                         than one shift was re-scored, else the path's own values     */
} ca_result_t;

enum {
    CA_FLAG_NEAR_TIE = 1u << 0,     /* best and runner-up |C| within 1e-6 relative   */
    CA_FLAG_RESCORED = 1u << 1,     /* more than one shift was re-scored in FP64     */
    CA_FLAG_CAND_CAPPED = 1u << 2,  /* candidate window held more than 32 shifts (split-
                                       BF16 n = 1024: more peaks than its FP64 searches) */
    CA_FLAG_DEGENERATE = 1u << 3,   /* a curve has zero norm; shift 0, theta 0,
                                       e0 = n1 + n2                                  */
    CA_FLAG_NONFINITE = 1u << 4,    /* NaN/Inf in the input; shift 0, theta 0, e0 NaN */
    CA_FLAG_THETA_FP64 = 1u << 5,   /* theta taken from the FP64 C(s*)               */
    CA_FLAG_UNSUPPORTED_N = 1u << 6, /* ragged pair with an unsupported n; not aligned */
    CA_FLAG_CLOCKWISE = 1u << 7      /* resample_arclength: the polygon's signed area is
                                        negative (vertices run clockwise)             */
};

enum { CA_PREC_FP32 = 0, CA_PREC_SPLIT_BF16 = 1, CA_PREC_FP64 = 2 };

/* Which shifts are re-scored with an FP64 dot product.  The FP64 value of
 * C at the chosen shift is always computed (it enters e0).
 *   TOP2   (default): the FP32 best and runner-up, when their |C| gap is below
 *          twice the FP32 error bound.
 *   WINDOW: every shift whose FP32 |C| lies within twice the error bound of
 *          the maximum; beyond 32 such shifts (CA_FLAG_CAND_CAPPED) the 32
 *          largest are kept (power-of-two n up to 1024 and the split-BF16
 *          path, by bisection on |C|^2) or the TOP2 pair (other n).          */
enum { CA_RESCORE_TOP2 = 0, CA_RESCORE_WINDOW = 1 };

enum { CA_RESAMPLE_SPLINE = 0, CA_RESAMPLE_LINEAR = 1 };
#define CA_RESAMPLE_MAX_RAW 32768   /* raw vertices per curve, resample_arclength */

typedef struct {
    int32_t precision;   /* CA_PREC_*                                         */
    int32_t rescore;     /* CA_RESCORE_*                                      */
    int32_t theta_fp64;  /* nonzero: theta from the FP64 C(s*)                */
    int32_t reserved;    /* must be 0                                         */
} ca_options_t;          /* NULL options pointer = {FP32, TOP2, 0, 0}         */

typedef struct ca_context* ca_context_t;

/* Create a context on HIP device `device` (must be gfx950).  The context owns
 * twiddle tables, DFT matrices and workspace, all released by ca_destroy.
 * tune_cache_path (host string, may be NULL): a launch-tuning file written by
 * ca_tune_save (format under ca_tune_save below), loaded as by ca_tune_load;
 * NULL leaves the default launch choices.  A file that cannot be read or
 * parsed fails the call with CA_ERR_INVALID_ARG (no context is created); a
 * file written for another architecture or CU count installs nothing.
 * Workspace that a call needs beyond what the context holds is allocated in
 * that call (never under stream capture: size it with an eager call of the
 * largest batch first); a buffer the context outgrows is kept until
 * ca_destroy, so a HIP graph captured earlier stays valid. */
ca_status_t ca_create(ca_context_t* ctx, int device, const char* tune_cache_path);
ca_status_t ca_destroy(ca_context_t ctx);
const char* ca_status_string(ca_status_t status);
/* Text of the last error raised on this thread (empty if none). */
const char* ca_last_error(void);

/* Largest n accepted by align_pair / align_batch (uniform and ragged), and
 * how a single n is handled:
 *   1 -- 2 <= n <= CA_MAX_N with no prime factor above 7: transforms of size n;
 *   2 -- any other n in [2, CA_MAX_N]: the correlation is evaluated exactly
 *        through zero-padded transforms of the smallest size M >= 2n with no
 *        prime factor above 7 (curve 1 followed by zeros, curve 2 repeated
 *        twice; no wrap-around at the lags that hold C(s)).  FP32 takes every
 *        such n, FP64 those with M <= 4096 (n <= 2048);
 *   0 -- n outside [2, CA_MAX_N]. */
#define CA_MAX_N 4096
int32_t ca_n_supported(int32_t n);

/*
 * align_pair -- Algorithm 2 for one pair (section 2).
 *   z1, z2 : n nodes each (complex64, or complex128 when precision = FP64)
 *   out    : one ca_result_t in device memory
 * Same semantics as align_batch with num_pairs = 1.
 */
ca_status_t align_pair(ca_context_t ctx, const void* z1, const void* z2, int32_t n,
                       ca_result_t* out, const ca_options_t* opt, void* stream);

/*
 * align_batch -- Algorithm 2 for many independent pairs.
 *   Uniform batch (offsets == NULL): pair p uses z1 + p*n and z2 + p*n
 *     (n nodes each); ca_n_supported(n) must be nonzero (and, for FP64 with
 *     ca_n_supported(n) == 2, n <= 2048), else CA_ERR_UNSUPPORTED_N.
 *   Ragged batch (offsets != NULL): offsets is a device array of num_pairs+1
 *     int64 node offsets, nondecreasing, offsets[0] = 0; pair p uses nodes
 *     [offsets[p], offsets[p+1]) of both z1 and z2; `n` is ignored.  A pair
 *     whose size is not supported gets CA_FLAG_UNSUPPORTED_N and is skipped.
 *   out: num_pairs results in device memory (pair order).
 *   precision SPLIT_BF16 requires a uniform batch with n == 128 or n == 1024
 *   (DFT-matrix products on the matrix cores with BF16 hi/lo operand splits
 *   and FP32 accumulation); its |C| error (~1e-5 relative) is above the
 *   near-tie threshold, so the shift is always settled by FP64 correlations
 *   and options.rescore is ignored: n = 128 re-scores every shift within
 *   twice the split-BF16 error bound of the largest |C|; n = 1024 computes the
 *   FP64 C at the vertex of a least-squares parabola through the split-BF16
 *   |C|^2 near its peak and at its two neighbours, climbs to a local FP64
 *   maximum, and climbs again from every separate peak whose split-BF16 |C|
 *   could exceed that maximum (CA_FLAG_CAND_CAPPED when more than 8, or 16
 *   for nearly circular shapes, were needed).
 * num_pairs == 0 is a no-op.
 */
ca_status_t align_batch(ca_context_t ctx, const void* z1, const void* z2,
                        const int64_t* offsets, int32_t n, int64_t num_pairs,
                        ca_result_t* out, const ca_options_t* opt, void* stream);

/*
 * align_all_pairs -- Algorithm 2 of section 2 for every unordered pair (i, j),
 * i < j, of a gallery of m curves with n nodes each (complex64,
 * curve-contiguous [m][n]): the distance-matrix use of the rigid alignment
 * that section 3 builds on (a matrix of pairwise shape distances).  The
 * correlation of each pair is the inverse transform of the product of the two
 * curves' spectra (the convolution-theorem argument of section 2), so
 * per-curve spectra and norms are computed once and only the product, one
 * transform and the epilogue run per pair.  Results are packed in row-major
 * upper-triangle order: pair (i, j) is at k = i*m - i*(i+1)/2 + (j - i - 1),
 * m*(m-1)/2 results in total.  FP32 precision only; n must be a power of
 * two in [64, 1024], else CA_ERR_UNSUPPORTED_N.
 */
ca_status_t align_all_pairs(ca_context_t ctx, const void* curves, int32_t m, int32_t n,
                            ca_result_t* out_upper, const ca_options_t* opt, void* stream);

/*
 * align_all_pairs_noalloc -- align_all_pairs for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  Same arguments, validation, kernels and
 * results (bit for bit) as align_all_pairs; the per-curve spectra and norms
 * live in a static device array of CA_NOALLOC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends, instead of
 * context workspace.  The call allocates and frees nothing (the context's
 * tables are built by ca_create).
 *   Scratch needed: round_up(m * n * 8, 256) + m * 8 bytes (spectra, then
 *   FP64 norms); a larger gallery (e.g. 4096 x 512 and 2048 x 1024 fit,
 *   16384 x 128 does not) returns CA_ERR_TOO_LARGE and enqueues nothing.
 *   Every call on one device shares that device's array and leaves the last
 *   call's spectra in it: calls that overlap on one device (other streams,
 *   other contexts or host threads) race and must be serialised by the caller.
 */
#define CA_NOALLOC_SCRATCH_BYTES (16 * 1024 * 1024 + 64 * 1024)
ca_status_t align_all_pairs_noalloc(ca_context_t ctx, const void* curves, int32_t m, int32_t n,
                                    ca_result_t* out_upper, const ca_options_t* opt, void* stream);

/*
 * resample_arclength -- uniform arc-length resampling (section 2, Eq.
 * arc-length-param and the cubic-spline step after it).
 *   raw         : raw vertices, complex64, all curves back to back
 *   raw_offsets : int64 [num_curves+1] vertex offsets (device)
 *   out_offsets : int64 [num_curves+1] node offsets (device); curve c gets
 *                 out_offsets[c+1] - out_offsets[c] nodes (>= 2)
 *   out         : complex64 nodes, centred on their mean and scaled by the
 *                 reciprocal of the raw perimeter (unit length)
 *   norms_out   : optional FP64 (1/n) sum |z|^2 per curve (NULL to skip)
 *   flags_out   : optional uint32 per curve; CA_FLAG_DEGENERATE when fewer than
 *                 3 distinct vertices remain or the perimeter is zero (nodes
 *                 are then 0); CA_FLAG_NONFINITE for NaN/Inf vertices;
 *                 otherwise CA_FLAG_CLOCKWISE when the cleaned polygon's
 *                 signed (shoelace) area is negative.  Section 1 takes both
 *                 curves counter-clockwise; the nodes keep the given order, and
 *                 a pair whose curves differ in this flag is aligned as given
 *   mode        : CA_RESAMPLE_SPLINE (periodic C2 cubic spline through the
 *                 arc-length knots) or CA_RESAMPLE_LINEAR
 * Input rules: vertices are counter-clockwise and not closed; trailing copies
 * of the first vertex and runs of consecutive duplicates are dropped.
 * Raw curves may have at most CA_RESAMPLE_MAX_RAW = 32768 vertices before
 * cleaning (the offsets live on the device, so this cannot be checked on the
 * host: a longer curve gets CA_FLAG_UNSUPPORTED_N and zero nodes).
 */
ca_status_t resample_arclength(ca_context_t ctx, const void* raw, const int64_t* raw_offsets,
                               int64_t num_curves, const int64_t* out_offsets, void* out,
                               double* norms_out, uint32_t* flags_out, int32_t mode,
                               void* stream);

/*
 * to_initializer -- hand-off to an elastic shape-distance solver (section 3:
 * the iterative solver is started from the rigid optimum (t0*, R*) with
 * gamma(t) = t).  Converts alignment records into the paper's notation.
 *   results : count records written by align_pair / align_batch /
 *             align_all_pairs (device)
 *   n       : node count of every pair, or 0 when offsets is given
 *   offsets : int64 [count+1] node offsets of a ragged batch (device, the
 *             same array passed to align_batch), or NULL
 *   t0_out  : FP64 [count] (device): t0* = ((n - shift) mod n) / n in [0, 1),
 *             the start parameter at which curve 2 is read, beta2(t + t0*)
 *   rot_out : FP64 [count][4] (device), row-major R* = R(theta_p) of section 2,
 *             [[cos theta_p, sin theta_p], [-sin theta_p, cos theta_p]] with
 *             theta_p = -theta, so that R* beta2(t + t0*) is aligned to beta1(t)
 * Records flagged DEGENERATE, NONFINITE or UNSUPPORTED_N carry shift 0 and
 * theta 0 and convert to t0* = 0, R* = identity.  count = 0 is a no-op.
 */
ca_status_t to_initializer(ca_context_t ctx, const ca_result_t* results, int32_t n,
                           const int64_t* offsets, int64_t count, double* t0_out, double* rot_out,
                           void* stream);

/*
 * srv_transform -- square-root-velocity function of section 3,
 * q = beta' / |beta'|^(1/2), for curves given as n nodes at the uniform
 * parameters t_k = k / n.  The curve is read as the closed polygon through
 * its nodes, so q is piecewise constant on the segments:
 *     q_k = d_k / |d_k|^(1/2),  d_k = n (z[k+1 mod n] - z[k]),
 * and q_k = 0 on a segment of zero length.  (1/n) sum |q_k|^2 is the
 * polygon's length.  FP32 (complex64) in and out.
 *   curves  : nodes, complex64 (device); uniform [count][n] or ragged flat
 *   offsets : int64 [count+1] node offsets of a ragged set (device), or NULL
 *   n       : nodes per curve (>= 2) when offsets is NULL, else 0
 *   q_out   : complex64, same layout and size as curves (device)
 * With the SRV functions of two curves on the same grid, the (t0, R) step of
 * Eq. (dist2-energy), the integral of |R q1(t + t0) - q2*(t)|^2, is
 * align_batch on (z1 = q2*, z2 = q1) followed by to_initializer.
 * count = 0 is a no-op.
 */
ca_status_t srv_transform(ca_context_t ctx, const void* curves, const int64_t* offsets, int32_t n,
                          int64_t count, void* q_out, void* stream);

/*
 * Library-owned HIP graphs: a whole step of the method (for example the
 * resampling of a ragged batch's raw polygons followed by its alignment, or
 * an all-pairs matrix) recorded once and replayed as one graph launch
 * (section 2's pipeline: Eq. arc-length-param, then Algorithm 2).
 *   ca_graph_begin -- opens a capture on a stream the context owns (default
 *     priority) and returns it in *capture_stream (host handle, a
 *     hipStream_t).  Issue the calls to record with that stream, with the
 *     device buffers the replays will use; nothing they enqueue runs before a
 *     launch.  The capture is in relaxed mode: workspace a call needs is
 *     allocated at capture time and kept by the context, as for eager calls.
 *   ca_graph_end -- closes the capture and instantiates it into *graph.  A
 *     call that failed during the capture fails ca_graph_end with
 *     CA_ERR_INVALID_ARG (the capture is discarded).
 *   ca_graph_launch -- replays the graph on `stream` (NULL = default stream),
 *     stream-ordered like any call; the recorded pointers and sizes are fixed,
 *     the buffers' contents are read at replay time.
 *   ca_graph_destroy -- releases the graph (NULL is a no-op).
 * One capture per context at a time; the context must outlive its graphs.
 */
typedef struct ca_graph* ca_graph_t;
ca_status_t ca_graph_begin(ca_context_t ctx, void** capture_stream);
ca_status_t ca_graph_end(ca_context_t ctx, ca_graph_t* graph);
ca_status_t ca_graph_launch(ca_graph_t graph, void* stream);
ca_status_t ca_graph_destroy(ca_graph_t graph);

/*
 * Launch tuning.  The kernels above take a few launch choices at run time;
 * each context holds one value per (knob, key), starting from defaults that
 * need no tuning.  A choice changes how work is scheduled, never what is
 * computed: grid and tile knobs give bit-identical results; a radix
 * schedule changes the rounding order of the FFT and a thread count that of
 * the FP64 norm and re-scoring sums (results stay within the error bound
 * every record reports).
 *
 *   knob                    key                          values (count)
 *   CA_TUNE_TEAM_GRID       n in {64,...,1024}           1: persistent blocks per CU of
 *                           (uniform FP32 batches)          the team kernel, in multiples of
 *                                                           its occupancy limit, 1..8, or 0
 *                                                           for one block per group of pairs
 *                                                           (default 1)
 *   CA_TUNE_ALLPAIRS_COLS   n in {64,...,1024}           1: columns per all-pairs tile,
 *                                                           1..256 (default 64)
 *   CA_TUNE_BLOCK_PLAN      M, a transform size with no  1..16: radix schedule of the block
 *                           prime factor above 7,           engine's FFT of size M, radices
 *                           2 <= M <= 2 * CA_MAX_N          2, 3, 4, 5, 7, 8 (and 16 when
 *                                                           M > 2048) whose product is M
 *                                                           (default: eights, then a four
 *                                                           or two, then 3, 5, 7)
 *   CA_TUNE_BLOCK_GRID      size class 0..4 of the block 1: persistent blocks per CU,
 *                           engine (M <= 512, 1024, 2048,   multiples of the occupancy limit,
 *                           4096, 8192)                     1..8, or 0 for one block per pair
 *                                                           (default 1)
 *   CA_TUNE_BLOCK_THREADS   size class 3 or 4            1: threads per block of the FP32
 *                                                           class kernel, 256 or 512, or for
 *                                                           class 4 also 1024 (defaults 256
 *                                                           for class 3, 1024 for class 4;
 *                                                           FP64 keeps 256)
 *
 * ca_tune_set and ca_tune_load change the tables the kernels read: they
 * synchronise the device first and must not be called while work of this
 * context is in flight on another stream or during stream capture.
 */
enum {
    CA_TUNE_TEAM_GRID = 0,
    CA_TUNE_ALLPAIRS_COLS = 1,
    CA_TUNE_BLOCK_PLAN = 2,
    CA_TUNE_BLOCK_GRID = 3,
    CA_TUNE_BLOCK_THREADS = 4
};

/*
 * ca_autotune -- measure every candidate of one (knob, key) on a synthetic
 * batch that the library generates on the device (smooth star-shaped curves
 * with rotated, shifted templates; up to 2^25 nodes per side; the size-class
 * knobs block_grid and block_threads use a ragged batch of 2^24 nodes whose
 * curve sizes are spread over every n whose transform falls in the class),
 * install the fastest and report its time per launch in *best_ms (optional).
 * Candidates:
 * grid knobs 1, 2, 4 and 0; all-pairs columns 2, 4, 8, 16, 32, 64; threads
 * 256 and 512 (and 1024 for class 4); radix
 * schedules: the orderings of the power-of-two part as eights, fours,
 * mixed or (M > 2048) sixteens, each with the odd radices first or last.  The first candidate runs
 * for about 20 ms first so that the clock settles; then every candidate is
 * timed with HIP events on `stream` in each of three rounds (three launches
 * after one warm-up launch per round) and keeps its best round.
 * Allocates and frees its own device buffers and synchronises the stream.
 * CA_ERR_UNSUPPORTED_N: the key names no size the knob serves (a transform
 * size that no n in [2, CA_MAX_N] uses).
 */
ca_status_t ca_autotune(ca_context_t ctx, int32_t knob, int32_t key, float* best_ms, void* stream);

/*
 * ca_tune_get -- current values of (knob, key) into values[0..*count) (host
 * memory); on entry *count is the capacity of values (16 is always enough),
 * on return the number of values.  ca_tune_set -- install values[0..count)
 * (host memory), validated as in the table above.
 */
ca_status_t ca_tune_get(ca_context_t ctx, int32_t knob, int32_t key, int32_t* values, int32_t* count);
ca_status_t ca_tune_set(ca_context_t ctx, int32_t knob, int32_t key, const int32_t* values,
                        int32_t count);

/*
 * ca_tune_save -- write every non-default choice of the context to a JSON
 * file (host path):
 *   {"format": "curvealign-tune/1", "arch": "gfx950", "num_cus": 256,
 *    "entries": [{"knob": "team_grid", "key": 1024, "values": [2], "ms": 0.41}, ...]}
 * knob names: team_grid, allpairs_cols, block_plan, block_grid, block_threads;
 * "ms" is the
 * time ca_autotune measured (-1 for values set by hand).
 * ca_tune_load -- read such a file and install its entries.  The whole file
 * is validated before anything is installed: a file that cannot be read or
 * parsed, or holds an invalid entry, returns CA_ERR_INVALID_ARG and leaves the
 * context's choices unchanged.  A file written for another architecture or
 * CU count installs nothing and returns CA_OK.  *applied (optional) receives
 * the number of entries installed.
 */
ca_status_t ca_tune_save(ca_context_t ctx, const char* path);
ca_status_t ca_tune_load(ca_context_t ctx, const char* path, int32_t* applied);

#ifdef __cplusplus
}
#endif

#endif /* CURVEALIGN_H */
