/*
 * libmmlttb -- MinMaxLTTB time-series downsampling on AMD Instinct MI355X (gfx950).
 *
 * MinMaxLTTB (Van Der Donckt et al., 2023) selects n_out points of a series
 * (x, y) of n points for line-chart display in two steps (section 3):
 *   (i)  MinMax preselection: in each of nb = floor(n_out * r_ps / 2) equal-index
 *        bins over the interior points 1..n-2, keep the index of the minimum and
 *        of the maximum of y (section 2.2.1, MinMax; r_ps/2 sub-buckets per LTTB
 *        bucket, section 3), plus the first and the last point;
 *   (ii) LTTB on the preselected points only: per bucket keep the point spanning
 *        the largest triangle with the point kept in the previous bucket and the
 *        mean (x, y) of the next bucket (section 2.2.1, LTTB; Fig. 3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Buffers named x, y, out_idx, out_count, ws, MX, MY are DEVICE pointers
 *   owned by the caller; segs_host (and the ms array of mmlttb_profile_samples)
 *   is a HOST pointer. The library never allocates or frees
 *   device memory inside these calls: scratch lives in the caller's workspace
 *   `ws` of `ws_bytes` bytes, sized by the matching *_workspace_size call.
 * - `stream` is a hipStream_t (NULL = the default stream). Work is enqueued on
 *   it in order; calls return before the device finishes. ws must not be
 *   reused by another call until the stream has passed this call.
 * - y: float32[n], finite (precondition, not checked on the device). With NaN
 *   or infinite values the output is unspecified, but every index the float32
 *   paths produce or read still lies inside its bin and the series (decoded
 *   key offsets are clamped to their bin; a bucket whose areas are all NaN
 *   keeps its first point).
 * - x: with MMLTTB_X_IMPLICIT, x must be NULL and x_i = i; with MMLTTB_X_INT64,
 *   x is int64[n], strictly increasing (precondition, not checked). x never
 *   affects binning (bins are equal-index); it enters only the LTTB means and
 *   areas, as binary64 values rounded from the integers.
 * - Output indices are int64, ascending, into the series (segment-local in
 *   batched mode). The selected values are y[idx] and x[idx]: exact copies.
 * - Determinism: every output is a pure function of the inputs (no dependence
 *   on launch geometry, tuning or timing); the CPU oracle gives the same
 *   indices bit for bit.
 * - Errors: arguments are checked on the host before anything is enqueued;
 *   on error nothing is enqueued and the return is negative. A failed HIP
 *   launch returns MMLTTB_EDEVICE. The message of the last error of the calling
 *   thread is in mmlttb_last_error(). No C++ exception crosses this boundary.
 * - Limits: 1 <= n <= 2^62; 3 <= n_out <= 2^31-1; 2 <= r_ps (1 <= r_ps for
 *   mmlttb_minmax alone); floor(n_out*r_ps/2) <= 2^31-1; each MinMax bin
 *   holds < 2^32 points. M4 and EveryNth state their own limits.
 */
#ifndef LIBMMLTTB_H
#define LIBMMLTTB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MMLTTB_OK = 0,
    MMLTTB_EINVAL = -1,  /* bad argument; nothing enqueued */
    MMLTTB_ENOMEM = -2,  /* ws_bytes below the required workspace size */
    MMLTTB_EDEVICE = -3, /* a HIP call or kernel launch failed */
    MMLTTB_ENOTSUP = -4  /* valid request the library does not handle */
} mmlttb_status_t;

typedef enum {
    MMLTTB_X_IMPLICIT = 0, /* x_i = i, x == NULL */
    MMLTTB_X_INT64 = 1,    /* x is int64[n] */
    MMLTTB_X_F64 = 2       /* x is binary64[n] (the *_typed calls only) */
} mmlttb_xkind_t;

typedef enum {
    MMLTTB_Y_F32 = 0, /* y is float32[n] */
    MMLTTB_Y_F64 = 1, /* y is binary64[n] */
    MMLTTB_Y_I32 = 2  /* y is int32[n] */
} mmlttb_ykind_t;

/* One series of a batch (segment). offset: first element of the series in
 * x_base/y_base; n, n_out, r_ps: as for mmlttb_minmaxlttb; out_offset: first
 * slot of its min(n, n_out) output indices in out_idx_base. */
typedef struct mmlttb_segment {
    int64_t offset;
    int64_t n;
    int64_t n_out;
    int32_t r_ps;
    int32_t reserved; /* must be 0 */
    int64_t out_offset;
} mmlttb_segment_t;

/* Library version string, static storage. */
const char *mmlttb_version(void);

/* Message of the last failed call on the calling thread ("" if none). */
const char *mmlttb_last_error(void);

/* Workspace bytes for mmlttb_minmax and mmlttb_minmaxlttb. The size depends
 * on n_out and r_ps only, never on n: the method keeps O(n_out) state
 * (Table 1, memory column; section 3.2). r_ps = 1 is accepted (the size for
 * mmlttb_minmax). Returns 0 on invalid arguments. */
size_t mmlttb_workspace_size(int64_t n, int64_t n_out, int32_t r_ps);

/* Workspace bytes for mmlttb_lttb (next-bucket means and chain scratch:
 * about 2.9 KB per bucket for n_out - 2 <= 2^24 buckets, which includes the
 * per-slab highs and lows, candidate lists and transition tables of wide
 * buckets); independent of n. Returns 0 on invalid arguments. */
size_t mmlttb_lttb_workspace_size(int64_t n, int64_t n_out);

/* MinMax preselection alone (section 2.2.1 MinMax; section 3 step (i)).
 * Writes the sorted distinct preselected indices P = {0, n-1} plus, for each
 * non-empty bin, the lowest index of its minimum and of its maximum of y
 * (values compared as numbers, so -0.0 == +0.0) to out_idx[0..m-1] and m to
 * the device scalar *out_count. out_idx capacity: 2*floor(n_out*r_ps/2) + 2
 * (or n if smaller). x is validated but not read (bins are equal-index).
 * r_ps = 1 gives the MinMax downsampler of Table 1 itself: floor(n_out/2)
 * bins, at most n_out points plus the first and last (section 3 footnote:
 * MinMaxLTTB with r_ps = 1 is MinMax aggregation). */
int mmlttb_minmax(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps,
                  int64_t *out_idx, int64_t *out_count, void *ws, size_t ws_bytes, void *stream);

/* Plain LTTB over all n points (section 2.2.1 LTTB; Fig. 3): the comparator
 * MinMaxLTTB is measured against. out_idx receives exactly min(n, n_out)
 * indices: 0, one index per interior bucket, n-1. Interior buckets are the
 * n_out-2 equal-index ranges 1 + floor(k*(n-2)/(n_out-2)); the next-bucket
 * mean is the exact sum of x and of y, each rounded once to binary64, divided
 * by the count (last bucket: the last point); the area is
 * |(Xa-MX)*(Yj-Ya) - (Xa-Xj)*(MY-Ya)| in binary64, one rounding per operation,
 * and ties go to the lowest index. n <= n_out returns 0..n-1. Buckets wider
 * than 64 points are run by transition tables (each candidate predecessor's
 * pick computed in parallel with the same arithmetic, exact scans where a
 * pick is not a candidate) unless the sequential pass is chosen with
 * mmlttb_set_tuning; both give the same indices. */
int mmlttb_lttb(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int64_t *out_idx, void *ws,
                size_t ws_bytes, void *stream);

/* The next-bucket means of LTTB over m given points (section 2.2.1 LTTB:
 * each bucket's third vertex is the average point of the bucket after it),
 * the step MinMaxLTTB runs on the preselected points. With B = n_out-2
 * interior buckets 1 + floor(k*(m-2)/B), MX[k] and MY[k] (k < B) are the
 * mean x and y of bucket k+1 (k = B-1: the last point alone): the exact sum
 * of the x (int64, or the position when xk is MMLTTB_X_IMPLICIT and x is NULL)
 * and of the float32 y, each rounded once to binary64, divided by the count in
 * binary64. MX and MY are device arrays of n_out-2 doubles owned by the
 * caller; nothing else is written and no workspace is needed.
 * MMLTTB_EINVAL unless m > n_out >= 3 (LTTB keeps every point otherwise) and
 * the pointers are valid as for mmlttb_lttb. */
int mmlttb_lttb_means(int xk, const int64_t *x, const float *y, int64_t m, int64_t n_out, double *MX, double *MY,
                      void *stream);

/* MinMaxLTTB (section 3): MinMax preselection (as mmlttb_minmax), then LTTB
 * (as mmlttb_lttb) on the preselected points only, with buckets, means and
 * areas taken over the preselected set. out_idx receives exactly
 * min(n, n_out) indices into the original series. n <= n_out returns 0..n-1. */
int mmlttb_minmaxlttb(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps,
                      int64_t *out_idx, void *ws, size_t ws_bytes, void *stream);

/* Bytes of the fixed device array that mmlttb_minmaxlttb_noalloc uses as its
 * workspace (4 MiB: enough for n_out * r_ps up to about 87000, e.g.
 * n_out = 16384 at r_ps = 4). */
#define MMLTTB_NOALLOC_SCRATCH_BYTES (4u << 20)

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): mmlttb_minmaxlttb
 * with the same arguments, meaning and result, minus ws and ws_bytes. Its
 * workspace is a fixed array of MMLTTB_NOALLOC_SCRATCH_BYTES bytes inside the
 * library, one per device, held from the first call on that device until the
 * process ends; its address is looked up on that first call, with the device
 * current, and kept. The call never allocates or frees memory. x, y and
 * out_idx are caller-owned device buffers on the current device, and stream
 * must belong to the current device. Errors: those of mmlttb_minmaxlttb, plus
 * MMLTTB_EINVAL (nothing enqueued) when mmlttb_workspace_size(n, n_out, r_ps)
 * exceeds MMLTTB_NOALLOC_SCRATCH_BYTES, and MMLTTB_EDEVICE if the array's
 * address cannot be looked up. Every call on one device shares that device's
 * array and leaves its contents behind (no part of the path needs it zeroed):
 * calls that overlap on one device -- on two streams, or from two threads
 * without ordering -- race on it and give undefined results. */
int mmlttb_minmaxlttb_noalloc(int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps,
                              int64_t *out_idx, void *stream);

/* Workspace bytes for mmlttb_minmaxlttb_batched over these segments (host
 * array). Independent of the segment lengths. Returns 0 on invalid input. */
size_t mmlttb_batched_workspace_size(const mmlttb_segment_t *segs_host, int64_t n_segs);

/* MinMaxLTTB over many series in one call: segment s reads
 * x_base[offset_s .. offset_s+n_s) (or implicit local x = 0..n_s-1) and
 * y_base[offset_s ..], and writes min(n_s, n_out_s) SEGMENT-LOCAL indices to
 * out_idx_base[out_offset_s ..]. Each segment's result equals
 * mmlttb_minmaxlttb on that series alone. segs_host is copied into ws before
 * the call returns. All segments are checked before anything is enqueued. */
int mmlttb_minmaxlttb_batched(int xk, const int64_t *x_base, const float *y_base, const mmlttb_segment_t *segs_host,
                              int64_t n_segs, int64_t *out_idx_base, void *ws, size_t ws_bytes, void *stream);

/* Line simplifiers that can follow the MinMax preselection in place of LTTB
 * (section 4 names them as future work, without definitions). */
typedef enum {
    MMLTTB_SIMPLIFY_VW = 1, /* Visvalingam-Whyatt */
    MMLTTB_SIMPLIFY_DP = 2, /* Douglas-Peucker with a point budget */
    MMLTTB_SIMPLIFY_LLB = 3 /* Longest-Line-Bucket */
} mmlttb_simplify_t;

/* Workspace bytes for mmlttb_minmax_simplify; independent of n. Returns 0 on
 * invalid arguments. */
size_t mmlttb_simplify_workspace_size(int64_t n, int64_t n_out, int32_t r_ps);

/* MinMax preselection (as mmlttb_minmaxlttb, r_ps >= 2), then, in place of
 * LTTB, another simplifier on the m preselected points with X = x (or the
 * index) rounded to binary64 and Y = y widened to binary64:
 *  VW:  while more than n_out points remain, remove the interior point whose
 *       doubled triangle area with its current neighbours a < j < b,
 *       |(Xa-Xb)*(Yj-Ya) - (Xa-Xj)*(Yb-Ya)|, is smallest (lowest index on
 *       ties), then recompute its neighbours' areas.
 *  DP:  start from the first and last point; a segment's farthest point
 *       maximises c = |(Xb-Xa)*(Yj-Ya) - (Xj-Xa)*(Yb-Ya)| (lowest index on
 *       ties) and its key is c*c / ((Xb-Xa)^2 + (Yb-Ya)^2), one rounding per
 *       operation (NaN, from a zero-length chord, counts as -1); while fewer
 *       than n_out points are kept, keep the farthest point of the segment
 *       with the largest key (lowest point on ties).
 *  LLB: LTTB's buckets; one point per bucket, first and last fixed,
 *       maximising the polyline's total length, sum of
 *       sqrt((Xj-Xi)^2 + (Yj-Yi)^2) accumulated bucket by bucket; each point
 *       keeps the lowest-index predecessor giving the largest total.
 * out_idx receives exactly min(n, n_out) ascending series indices; n <= n_out
 * returns 0..n-1. Extra limit: 2*floor(n_out*r_ps/2) + 2 <= 2^31-1. VW and
 * LLB run in one wave (32 bytes of state per point). DP builds the tree of
 * splits a level at a time in one workgroup (40 bytes per point) and keeps
 * the points a step-by-step greedy loop would keep; trees deeper than 512
 * levels, and series whose last-ranked group of nodes needs more than 256
 * step-by-step picks or holds more than 512 nodes, go to that greedy loop
 * itself (one wave). State lives in LDS when it fits, else in the workspace. */
int mmlttb_minmax_simplify(int alg, int xk, const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps,
                           int64_t *out_idx, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for mmlttb_minmax_typed and mmlttb_minmaxlttb_typed;
 * independent of n. Returns 0 on invalid arguments. */
size_t mmlttb_typed_workspace_size(int64_t n, int64_t n_out, int32_t r_ps);

/* MinMax preselection (as mmlttb_minmax, section 2.2.1 MinMax and section 3
 * step (i)) for y of kind yk: float32, binary64 or int32, aligned to its value
 * size. Values compare as numbers (-0.0 == +0.0 for the floating types); y
 * finite (precondition). Same bins, ties, output and capacity as
 * mmlttb_minmax; r_ps >= 1. */
int mmlttb_minmax_typed(int yk, const void *y, int64_t n, int64_t n_out, int32_t r_ps, int64_t *out_idx,
                        int64_t *out_count, void *ws, size_t ws_bytes, void *stream);

/* MinMaxLTTB (section 3) for y of kind yk (float32, binary64, int32) and x of
 * kind xk (implicit, int64 or binary64; binary64 x finite and strictly
 * increasing, preconditions). Preselection as mmlttb_minmax_typed; LTTB over
 * P on Y = y as binary64 (exact) and X = x (binary64 x) or x rounded to
 * binary64 (int64 x); next-bucket means are the exact sums of the stored x
 * and of Y, each rounded once to binary64, divided by the count (a sum beyond
 * the binary64 range rounds to an infinity); areas and ties as mmlttb_lttb.
 * out_idx receives exactly min(n, n_out) indices. float32 y with implicit or
 * int64 x gives the indices of mmlttb_minmaxlttb (which is faster). */
int mmlttb_minmaxlttb_typed(int xk, const void *x, int yk, const void *y, int64_t n, int64_t n_out, int32_t r_ps,
                            int64_t *out_idx, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for mmlttb_minmax_xbins and mmlttb_minmaxlttb_xbins;
 * independent of n. Returns 0 on invalid arguments. */
size_t mmlttb_xbins_workspace_size(int64_t n, int64_t n_out, int32_t r_ps);

/* MinMax preselection with bins of equal x WIDTH, for irregular timestamps
 * (a bin has edges in x, Fig. 3; section 2.2.1 MinMax). x: int64[n], strictly
 * increasing (precondition: unsorted x gives meaningless indices, never an
 * access out of bounds). The interior points 1..n-2 fall into
 * nb = floor(n_out*r_ps/2) bins with edges e_b = x_1 + floor(b*(x_{n-1}-x_1)/nb):
 * point i is in bin b when e_b <= x_i < e_{b+1}. With x_i = i this is the
 * equal-index binning of mmlttb_minmax. Empty bins (gaps) are skipped. Output
 * as mmlttb_minmax: sorted distinct P in out_idx[0..m-1] (capacity
 * 2*nb + 2, or n if smaller), m in the device scalar *out_count. Limits:
 * 1 <= n <= 2^32+1, 3 <= n_out <= 2^31-1, r_ps >= 1, nb <= 2^31-1. */
int mmlttb_minmax_xbins(const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps, int64_t *out_idx,
                        int64_t *out_count, void *ws, size_t ws_bytes, void *stream);

/* MinMaxLTTB (section 3) with the preselection of mmlttb_minmax_xbins. LTTB
 * then runs over P as in mmlttb_minmaxlttb; when gaps leave P with n_out
 * points or fewer, every point of P is kept. out_idx (capacity n_out)
 * receives min(n, n_out, m) ascending indices and *out_count (device scalar)
 * their number. r_ps >= 2; other limits as mmlttb_minmax_xbins. */
int mmlttb_minmaxlttb_xbins(const int64_t *x, const float *y, int64_t n, int64_t n_out, int32_t r_ps,
                            int64_t *out_idx, int64_t *out_count, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for mmlttb_m4 (one key pair per bin); independent of n.
 * Returns 0 on invalid arguments. */
size_t mmlttb_m4_workspace_size(int64_t n, int64_t n_out);

/* M4 (section 2.2.1, M4; Table 1): nb = floor(n_out/4) equal-index bins over
 * all points, bin b = [floor(b*n/nb), floor((b+1)*n/nb)); per bin the first
 * and the last index and the lowest index of the minimum and of the maximum of
 * y (compared as numbers, -0.0 == +0.0). Writes the sorted distinct indices
 * to out_idx[0..m-1] (capacity n_out suffices) and m to the device scalar
 * *out_count. n <= n_out keeps 0..n-1. y: float32[n], finite, 4-byte
 * aligned; x is not an argument (bins are equal-index). Limits:
 * 1 <= n <= 2^62; 4 <= n_out <= 2^31-1; each bin holds < 2^32 points;
 * otherwise MMLTTB_EINVAL. ws: mmlttb_m4_workspace_size bytes (may be NULL
 * when n <= n_out). */
int mmlttb_m4(const float *y, int64_t n, int64_t n_out, int64_t *out_idx, int64_t *out_count, void *ws,
              size_t ws_bytes, void *stream);

/* EveryNth (section 2.2.1, EveryNth; Table 1): out_idx[k] = floor(k*n/n_out)
 * for k = 0..n_out-1, the n_out evenly spaced indices; n <= n_out writes
 * 0..n-1. out_idx receives min(n, n_out) indices; no data is read and no
 * workspace is used. Limits: 1 <= n <= 2^62; 1 <= n_out <= 2^31-1;
 * otherwise MMLTTB_EINVAL. */
int mmlttb_everynth(int64_t n, int64_t n_out, int64_t *out_idx, void *stream);

/* Graph replay of batched calls. With max_graphs > 0, a batched call on a
 * non-default stream is captured into a HIP graph (every kernel, reading the
 * header and segment table from a device copy that the cache allocates and
 * fills once at capture) the first time its exact arguments are seen
 * (pointers, stream, x kind, tuning, segment table), and replayed by later
 * calls with the same arguments; at most max_graphs graphs are kept (least
 * recently used evicted, after its last replay completes). The cache holds
 * one device table copy (about 12 KB plus 184 bytes per segment) per graph.
 * 0 (the default) disables it and releases every graph. Process-wide; not
 * thread-safe with concurrent calls.
 * mmlttb_graph_cache_stats reports entries held, replays and captures since
 * the cache was last disabled. */
int mmlttb_set_graph_cache(int max_graphs);
int mmlttb_graph_cache_stats(int64_t *entries, int64_t *hits, int64_t *captures);

/* Execution tuning (never changes results): unroll = 16-byte loads in flight
 * per lane of the single-series MinMax streams (1, 2, 4 or 8); chunk = points
 * per single-series MinMax work item (rounded up to a multiple of
 * 256*unroll); chain = LTTB pass form: 1 sequential (one wave walks every
 * bucket in order), 2 segmented (segments walked from every start point in
 * parallel, then linked; used when buckets hold at most 64 points), 3
 * automatic (segmented when possible); tile = points a workgroup stages in
 * LDS for small bins, of batched series and of single float32 series long
 * enough for the chunked short-bin stream (2048, 4096 or 8192; bins of at
 * most tile/4 points take that path); batch_unroll and batch_chunk = unroll and
 * chunk of the batched large-bin stream. The compiled defaults are the best
 * settings measured on MI355X: unroll 4, chunk 2^20, chain 3, tile 4096,
 * batch_unroll 4, batch_chunk 65536 (environment variables MMLTTB_UNROLL,
 * MMLTTB_CHUNK, MMLTTB_CHAIN, MMLTTB_TILE, MMLTTB_BATCH_UNROLL and
 * MMLTTB_BATCH_CHUNK override them when the library loads). A value of 0
 * keeps the current setting; mmlttb_get_tuning reports every field as a
 * settable value, so passing its results back restores a saved setting.
 * Returns MMLTTB_EINVAL for other values. Process-wide; not thread-safe with
 * concurrent calls. */
int mmlttb_set_tuning(int unroll, int64_t chunk, int chain, int tile, int batch_unroll, int64_t batch_chunk);
int mmlttb_get_tuning(int *unroll, int64_t *chunk, int *chain, int *tile, int *batch_unroll, int64_t *batch_chunk);

/* Kernel timing for measurement. When enabled, timing-only HIP events (no
 * system-scope fence) are recorded on the caller's stream around every launch
 * of the named kernels; mmlttb_profile_read
 * synchronises those events and returns the summed milliseconds and the
 * launch count of `kernel` since the last reset. Launches on a stream that is
 * being captured into a graph are not timed. Not thread-safe; off by default. */
int mmlttb_profile_enable(int on);
int mmlttb_profile_reset(void);
int mmlttb_profile_read(const char *kernel, double *total_ms, int64_t *launches);
/* The individual durations behind mmlttb_profile_read, in launch order: copies
 * the first min(cap, available) of them (milliseconds) into the HOST array `ms`
 * and sets *count to the number available (at most 65536 per name are kept
 * since the last reset). Besides the kernel names, "call_minmaxlttb" holds one
 * span per successful mmlttb_minmaxlttb call: from an event recorded on its
 * stream before its first launch to one recorded after its last, so back-to-back
 * calls give the device time per call. MMLTTB_EINVAL for a NULL name or count,
 * a negative cap, or ms == NULL with cap > 0. Not thread-safe. */
int mmlttb_profile_samples(const char *name, float *ms, int64_t cap, int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* LIBMMLTTB_H */
