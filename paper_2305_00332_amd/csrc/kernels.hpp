// Launch interface of the libmmlttb kernels (host side of the library only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace mmlttb {

// Work decomposition of minmax_bin_reduce: bins.parts bins over the interior
// (bins.len = n - 2 points), each cut into chunks_per_bin items of at most
// `chunk` points (a multiple of 4 * 64 * unroll). One wave per item.
struct MinMaxGeom {
    Split bins;
    int64_t chunk;
    int64_t chunks_per_bin;
    int64_t n_items;
};

// Workgroups of a MinMax / M4 stream launch (4 waves each). Waves loop over
// work items, so the grid may be smaller than the item count: with items of
// at least kLongItem points, 2048 waves (8 per CU) streaming several items each
// beat one wave per item (n = 1e9 with 8000 bins: 0.577 vs 0.596 ms); with
// shorter items the restart of each wave's load pipeline costs more than it
// saves, and every item gets its own wave.
constexpr int64_t kStreamWaves = 2048;
constexpr int64_t kLongItem = 32768;
inline int64_t stream_blocks(const MinMaxGeom &g)
{
    const int64_t blocks = (g.n_items + 3) / 4;
    return (g.chunk >= kLongItem && blocks > kStreamWaves / 4) ? kStreamWaves / 4 : blocks;
}

// Bins shorter than kShortBin points, in series long enough for 2048 chunks,
// are streamed by fixed chunks of kShortBinChunk points across bin ends
// instead of one work item per bin
// (n = 1e9: 477-point bins 1.64 -> 1.03 ms, 3815-point bins 0.644 -> 0.622
// ms; at 7629 points one item per bin is still ahead, 0.601 vs 0.608 ms).
constexpr int64_t kShortBin = 4096;
constexpr int64_t kShortBinChunk = 65536;
hipError_t launch_minmax_stream_chunks(const float *y, const Split &bins, int unroll, unsigned long long *keys,
                                      hipStream_t s);
// Bins per small-bin tile for one series' bins of at most maxbin points (0:
// the bins are too long for `tile`-point tiles, or too many for the tile
// planner's binary64 bin starts), and the single-series small-bin launch.
int small_tile_bins(int64_t maxbin, int64_t nb, int tile);
hipError_t launch_minmax_small_tiles(const float *y, const Split &bins, int tile, unsigned long long *keys,
                                     hipStream_t s);

// LDS window of the sequential chain, in points.
constexpr int kChainStage = 1024;

// Segmented chain: buckets per segment, start points per segment (one lane
// each, so buckets may hold at most this many points), segments per LDS
// window while the segments are linked.
constexpr int kSegLen = 32;
constexpr int kSegStarts = 64;
constexpr int kChaseWindow = 512;

static_assert(kSegLen == 32 && kSegStarts <= 256, "segment paths are written as 32-byte rows of byte offsets");

// LDS of one segment walk: x, y of up to stage_cap points and the kSegLen
// means (binary64), kSegLen + 1 bucket starts, a byte per point (its pick in
// the next bucket).
inline size_t seg_walk_lds_bytes(int stage_cap)
{
    return (size_t)(2 * stage_cap + 2 * kSegLen) * sizeof(double) + (kSegLen + 1) * sizeof(int32_t) +
           (size_t)stage_cap;
}

template <class XT, class YT>
struct SegChainArgsT {
    const XT *XP;          // x of the points (NULL: x = position)
    const YT *YP;          // y of the points
    const int64_t *m_ptr;  // device point count (NULL: m_const)
    int64_t m_const;
    int64_t B;             // interior buckets
    const double *MX, *MY; // next-bucket means
    uint8_t *path;         // [S][kSegStarts][kSegLen]: pick offset inside its bucket
    uint8_t *finals;       // [S][kSegStarts]: pick offset in the segment's last bucket
    uint8_t *start;        // [S]: start lane of segment s on the chain from point 0
    int64_t S;             // segments
    int stage_cap;         // LDS points per segment (kSegLen * bucket-size bound)
};
// Points as stored by the float32 path (raw int64 x, float32 y) and by the
// typed path (binary64 coordinates).
using SegChainArgs = SegChainArgsT<int64_t, float>;
using SegChainArgsD = SegChainArgsT<double, double>;

// ---------------------------------------------------------------- batched

enum SegMode : int32_t { kSegIdentity = 0, kSegAll = 1, kSegMinMax = 2 };

// Small-bin tiles: a workgroup of kTileThreads stages up to `tile` consecutive
// points (whole bins; tile in {2048, 4096, 8192}, a tuning choice) in LDS; a
// power-of-two group of lanes reduces each bin. Bins of at most tile / 4
// points take this path.
constexpr int kTileThreads = 256;

// One series of a batch as planned on the host (copied to the workspace).
struct BatchSeg {
    int64_t offset;     // first element in x_base / y_base
    int64_t n, n_out, out_offset;
    int32_t r_ps, mode; // SegMode
    Split bins;         // interior split into nb bins (kSegMinMax)
    int64_t chunk;      // large bins: points per work item (one wave streams a chunk across bin ends)
    int32_t small;      // 1: bins reduced by LDS tiles
    int32_t tile_bins;  // small: bins per tile (power of two, 4..256)
    int64_t li0, ln;    // large-bin items: start and count in the flat item space
    int64_t ti0, tn;    // small-bin tiles: start and count in the flat tile space
    int64_t key0;       // pooled key pairs
    int64_t p0;         // pooled P / XP / YP slots
    int64_t B;          // interior LTTB buckets (n_out - 2)
    int64_t b0;         // pooled MX / MY slots
    int64_t c0;         // pooled chain-segment slots (path / finals / start)
    int64_t cw0, cwn;   // chain walk units in the flat chain space (cwn = 0: sequential chain)
    int32_t stage_cap;  // LDS points per chain segment
    int32_t seq;        // 1: sequential chain
};

// Longest stream of one wave (positions relative to its start fit in int32).
constexpr int64_t kMaxStreamChunk = (int64_t)1 << 30;

// Coarse owner tables: entry q (0..kOwnerTable) holds the series owning unit
// min(total - 1, floor(q * total / kOwnerTable)) of a flat work space; unit i
// with q = floor(i * kOwnerTable / total) is owned by a series between
// entries q and q + 1.
constexpr int kOwnerTable = 1024;

struct BatchHeader {
    int64_t n_segs;
    int64_t n_keys;
    int64_t n_large_items, n_small_tiles, n_chain_units;
    int64_t max_stage_cap;
    int64_t max_B; // most interior LTTB buckets of any series
    int64_t off_segs, off_keys, off_P, off_XP, off_YP, off_m, off_MX, off_MY, off_path, off_finals, off_start;
    int32_t own_large[kOwnerTable + 1], own_small[kOwnerTable + 1], own_chain[kOwnerTable + 1];
};

struct BatchPtrs {
    const BatchHeader *hdr; // device copy of the header (owner tables)
    const BatchSeg *segs;
    int64_t n_segs;
    int xk;
    const int64_t *x_base;
    const float *y_base;
    int64_t *out_base;
    unsigned long long *keys;
    int64_t *P, *XP;
    float *YP;
    int64_t *m;
    double *MX, *MY;
    uint8_t *path, *finals, *start;
    int64_t n_keys, n_large_items, n_small_tiles, n_chain_units;
    int64_t max_B;
    int stage_cap_max;
};

hipError_t launch_batch_init(const BatchPtrs &b, hipStream_t s);
hipError_t launch_batch_large(const BatchPtrs &b, int unroll, hipStream_t s);
hipError_t launch_batch_small(const BatchPtrs &b, int tile, hipStream_t s);
hipError_t launch_batch_compact(const BatchPtrs &b, hipStream_t s);
hipError_t launch_batch_means(const BatchPtrs &b, hipStream_t s);
hipError_t launch_batch_chain(const BatchPtrs &b, hipStream_t s);
hipError_t launch_batch_link_emit(const BatchPtrs &b, hipStream_t s);
hipError_t launch_batch_chain_seq(const BatchPtrs &b, hipStream_t s);

inline int64_t seg_count(int64_t B) { return (B + kSegLen - 1) / kSegLen; }
// Two-level link for long chains (more than kTwoLevelLink segments): the S-1
// segment-to-segment transitions are cut into chunks of kLinkChunk; each
// chunk's composed start->exit map is formed in parallel, one chain over the
// chunk maps gives every chunk's start, and each chunk then fills its own
// segments' starts. In the workspace region of the S start lanes they are
// followed, from the next multiple of 64 bytes, by the chunk maps (64 bytes
// each) and the chunk starts (one byte per chunk, plus one).
constexpr int kLinkChunk = 64;
constexpr int64_t kTwoLevelLink = 2 * kChaseWindow;
inline int64_t seg_chunks(int64_t B) { return (seg_count(B) - 1 + kLinkChunk - 1) / kLinkChunk; }
inline int64_t seg_maps_offset(int64_t S) { return (S + 63) / 64 * 64; }
inline size_t seg_start_bytes(int64_t B)
{
    return (size_t)seg_maps_offset(seg_count(B)) + (size_t)seg_chunks(B) * kSegStarts + (size_t)seg_chunks(B) + 1;
}
inline size_t seg_path_bytes(int64_t B) { return (size_t)seg_count(B) * kSegStarts * kSegLen; }
inline size_t seg_finals_bytes(int64_t B) { return (size_t)seg_count(B) * kSegStarts; }

// `ticket` (optional): cleared for a k_preselect_tail launch that follows.
hipError_t launch_init_keys(unsigned long long *keys, int64_t nb, hipStream_t s, unsigned int *ticket = nullptr);
hipError_t launch_minmax_bin_reduce(const float *y, const MinMaxGeom &g, int unroll, unsigned long long *keys,
                                    hipStream_t s, unsigned int *ticket = nullptr);
// Bins per workgroup of the tiled compaction (1024 threads, 4 slabs), and the
// bin count above which it replaces the one-workgroup compaction: that one
// walks every bin in rounds of 4096 (nb = 32768: 105 us with the means).
constexpr int64_t kCompactTileBins = 4096;
constexpr int64_t kFusedCompactBins = 16384;
inline int64_t compact_tiles(int64_t nb) { return (nb + kCompactTileBins - 1) / kCompactTileBins; }
hipError_t launch_compact_tiled(const unsigned long long *keys, const Split &bins, int64_t n, const int64_t *x,
                                const float *y, int64_t *P, int64_t *XP, float *YP, int64_t *m_out, int64_t *tile_slot,
                                hipStream_t s);
hipError_t launch_preselect_compact(const unsigned long long *keys, const Split &bins, int64_t n, const int64_t *x,
                                    const float *y, int64_t *P, int64_t *XP, float *YP, int64_t *m_out, hipStream_t s);
// The fused tail (compaction, means, segmented chain, output): one
// workgroup of kTailThreads per chain segment, for at most kTailBins bins and
// segments whose points (with the bucket before and after) fit kTailPts.
constexpr int kTailThreads = 256;
constexpr int kTailBins = 3840; // keys staged in at most 64 KiB of dynamic LDS
constexpr int kTailPts = 640;
bool preselect_tail_fits(int64_t nb, int64_t maxb_bound);
hipError_t launch_preselect_tail(const unsigned long long *keys, const Split &bins, int64_t n, const int64_t *x,
                                 const float *y, int64_t B, int stage_cap, int64_t *P, uint8_t *path, uint8_t *finals,
                                 uint8_t *start, unsigned int *ticket, int64_t *out, hipStream_t s);
hipError_t launch_preselect_compact_means(const unsigned long long *keys, const Split &bins, int64_t n,
                                          const int64_t *x, const float *y, int64_t *P, int64_t *XP, float *YP,
                                          int64_t *m_out, int64_t B, double *MX, double *MY, hipStream_t s);
hipError_t launch_preselect_all(int64_t n, const int64_t *x, const float *y, int64_t *P, int64_t *XP, float *YP,
                                int64_t *m_out, hipStream_t s);
hipError_t launch_iota(int64_t *out, int64_t n, int64_t *count_out, hipStream_t s);
hipError_t launch_m4_bin_reduce(const float *y, const MinMaxGeom &g, int unroll, unsigned long long *keys,
                                hipStream_t s);
hipError_t launch_m4_compact(const unsigned long long *keys, const Split &bins, int64_t *out, int64_t *count,
                             hipStream_t s);
hipError_t launch_everynth(int64_t n, int64_t n_out, int64_t *out, hipStream_t s);
// Other simplifiers on the preselected points (1 VW, 2 DP, 3 LLB). Per-point
// state lives in LDS (in_lds) or at `scratch` in the workspace; DP's split
// tree keeps its most used arrays in LDS when tree_in_lds is set.
struct SimplifyArgs {
    const int64_t *XP;    // raw x (or the index) of the m points
    const float *YP;      // y of the points
    const int64_t *m_ptr; // device point count
    const int64_t *Pmap;  // series index of each point
    int64_t *out;         // n_out series indices
    int64_t n_out;
    int64_t cap;          // bound on m the state is sized for
    int64_t cap_bucket;   // bound on the points of one LTTB bucket (LLB)
    unsigned char *scratch;
    int in_lds;
    int tree_in_lds;
};
int64_t simplify_scratch_bytes(int64_t cap);
int64_t simplify_state_lds_bytes(int64_t cap); // the greedy loops' state
int64_t simplify_tree_lds_bytes(int64_t cap);  // DP's split tree (dynamic LDS)
int64_t simplify_tree_static_lds();            // bound on its static LDS
hipError_t launch_simplify(int alg, const SimplifyArgs &a, hipStream_t s);
// Let the LDS forms of the kernels take state_bytes (greedy loops) and
// tree_bytes (DP's split tree) of dynamic LDS; 0 leaves a limit as it is.
hipError_t simplify_allow_lds(size_t state_bytes, size_t tree_bytes);

// Value types of the typed path (y) and the per-work-item MinMax partial.
enum { kYF32 = 0, kYF64 = 1, kYI32 = 2 };
struct TypedPartial {
    uint64_t kmin;
    int64_t imin;
    uint64_t kmax;
    int64_t imax;
};
hipError_t launch_typed_bin_reduce(int yk, const void *y, const MinMaxGeom &g, int unroll, TypedPartial *part,
                                   hipStream_t s);
hipError_t launch_typed_bin_merge(const TypedPartial *part, int64_t nb, int64_t cpb, int64_t *pairs, hipStream_t s);
hipError_t launch_typed_compact(int xk, int yk, const int64_t *pairs, const Split &bins, int64_t n, const void *x,
                                const void *y, int64_t *P, double *XD, double *YD, int64_t *m_out, bool all,
                                hipStream_t s);
hipError_t launch_typed_bucket_means(int xk, const int64_t *P, const void *x, const double *YD, const int64_t *m_ptr,
                                     int64_t B, double *MX, double *MY, hipStream_t s);
hipError_t launch_xbin_bounds(const int64_t *x, int64_t n, int64_t nb, int64_t *bounds, hipStream_t s);
hipError_t launch_xbin_reduce(const float *y, const int64_t *bounds, int64_t n, int64_t nb, int64_t chunk,
                              int unroll, unsigned long long *keys, hipStream_t s);
hipError_t launch_xbin_compact(const unsigned long long *keys, const int64_t *bounds, int64_t nb, int64_t n,
                               const int64_t *x, const float *y, int64_t *P, int64_t *XP, float *YP, int64_t *m_true,
                               int64_t *m_eff, int64_t pad_to, int64_t B, double *MX, double *MY, hipStream_t s);
hipError_t launch_xbin_finish(const int64_t *P, const int64_t *m_true, int64_t n_out, int64_t *out, int64_t *count,
                              hipStream_t s);

hipError_t launch_bucket_mean_small(const int64_t *XP, const float *YP, const int64_t *m_ptr, int64_t m_const,
                                    int64_t B, double *MX, double *MY, hipStream_t s);
// YR (may be NULL): the y range of every bucket, for the table form.
hipError_t launch_bucket_mean_wide(const int64_t *X, const float *Y, int64_t m, int64_t B, double *MX, double *MY,
                                   float2 *YR, hipStream_t s);
hipError_t launch_lttb_chain(const int64_t *XP, const float *YP, const int64_t *m_ptr, int64_t m_const, int64_t B,
                             const double *MX, const double *MY, const int64_t *Pmap, int64_t *out, hipStream_t s);
hipError_t launch_lttb_chain_seg(const SegChainArgs &a, const int64_t *Pmap, int64_t *out, hipStream_t s);
hipError_t launch_lttb_chain_seg(const SegChainArgsD &a, const int64_t *Pmap, int64_t *out, hipStream_t s);
hipError_t launch_lttb_chain(const double *XP, const double *YP, const int64_t *m_ptr, int64_t m_const, int64_t B,
                             const double *MX, const double *MY, const int64_t *Pmap, int64_t *out, hipStream_t s);
// Whole-series LTTB by transition tables: a first pass (next-bucket means, y
// ranges, the highest and lowest point of each of kSlabsHost slabs), candidate
// picks per bucket (hull points of the arc the predecessors' slopes can touch,
// at most kCandMax, count -1 when more), the pick in each bucket for every
// candidate of the bucket before (over the candidates where a rounding
// certificate holds, else over the whole bucket), and a walk that scans a
// bucket in full where its predecessor is not a candidate.
constexpr int kCandMax = 64;
constexpr int kSlabsHost = 128; // slabs per bucket (pass 1)
// Largest bucket count the table form runs (its grids and tables grow with B),
// and largest bucket (offsets in 32-bit keys).
constexpr int64_t kTableMaxBuckets = (int64_t)1 << 24;
constexpr int64_t kTableMaxBucket = (int64_t)1 << 31;
hipError_t launch_lttb_scan(const int64_t *X, const float *Y, int64_t n, int64_t B, double *MX, double *MY, float2 *YR,
                            unsigned long long *slab_hi, unsigned long long *slab_lo, hipStream_t s);
hipError_t launch_lttb_hull(const int64_t *X, const float *Y, int64_t n, int64_t B, const double *MX, const double *MY,
                            const float2 *YR, const unsigned long long *slab_hi, const unsigned long long *slab_lo,
                            int32_t *cand_cnt, int32_t *cand, double *delta, double2 *brk, hipStream_t s);
hipError_t launch_lttb_tables(const int64_t *X, const float *Y, int64_t n, int64_t B, const double *MX,
                              const double *MY, const float2 *YR, const int32_t *cand_cnt, const int32_t *cand,
                              const double *delta, const double2 *brk, int2 *tab, hipStream_t s);
hipError_t launch_lttb_table_walk(const int64_t *X, const float *Y, int64_t n, int64_t B, const double *MX,
                                  const double *MY, const int32_t *cand_cnt, const int32_t *cand, const int2 *tab,
                                  int64_t *out, hipStream_t s);
hipError_t launch_lttb_chain_wide(const int64_t *X, const float *Y, int64_t m, int64_t B, const double *MX,
                                  const double *MY, int64_t *out, hipStream_t s);

} // namespace mmlttb
