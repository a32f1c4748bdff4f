// Library-internal declarations shared by the runtime and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace latch {

// Window geometry.
constexpr int kWin = 48;                 // upright window side
constexpr int kHalf = 24;                // pixel (i, j) sits at offset (j - 24, i - 24)
constexpr int kPatchR = 3;               // 7 x 7 patches
constexpr int kTriplets = 512;
constexpr int kWords = 16;
constexpr int kBins = 4096;
// Window gather order: per angle class (32 bins), chains of four window
// positions (u, v), (u + 1, v) and their mirrors (-u, -v), (-u - 1, -v),
// covering [-24, 24]^2 (613 chains; the first members of a row's chains
// overlap by one position at its end), sorted by the band of a quarter image
// row at unit scale of the first member, then by its image column
// (host-built); for each of the 128 extraction threads its 5 chains (chains
// 128 m + thread; the last slots repeat the centre's chain) as 16-bit entries
// u & 0xff | (v & 0xff) << 8.  A class's table holds, for thread t, chains
// 0..3 at entries 4 t .. 4 t + 3 and chain 4 at entry 512 + t, so that a
// thread reads its chains with one 8-byte and one 2-byte load and every load
// of a wavefront is contiguous.
constexpr int kGatherClasses = kBins / 32;
constexpr int kGatherChains = 5;
constexpr int kGatherHeadChains = 4;
constexpr int kGatherClassEntries = 128 * kGatherChains;

// Extraction LDS layout, per workgroup.
//  * Copies s = 0..7: copy s holds, for every window row y and quadword
//    q = 0..4, the 7 window bytes (y, 8 q + s .. 8 q + s + 6) followed by a
//    zero byte, at byte s * kCopyBytes + y * kCopyRowBytes + 8 q.  A 7-byte
//    patch row starting at column x <= 39 is then one 8-byte-aligned
//    quadword whose last byte is zero.
//  * Edge copies for x = 40 and 41 (patch centres in columns 43, 44): the
//    quadword of row y sits at kEdgeBase + y * kCopyRowBytes + 32 + 8 (x - 40).
//    The two interleave without overlap, so all patch rows share the row
//    stride kCopyRowBytes.
//  * The plain window, 48 rows of kRawStride bytes (13 dwords per row, so
//    the lanes of a column-wise byte write fall in distinct banks), and a
//    49th row and column that the gather fills and nothing reads (it samples
//    positions in pairs (u, v), (-u, -v) over [-24, 24]^2).
constexpr int kCopies = 8;
constexpr int kCopyQwords = 5;
constexpr int kCopyRowBytes = 8 * kCopyQwords;                     // 40
constexpr int kCopyBytes = kWin * kCopyRowBytes;                   // 1920
constexpr int kEdgeBase = kCopies * kCopyBytes;                    // 15360
constexpr int kEdgeBytes = kCopyBytes + 8;                         // 1928
constexpr int kRawBase = (kEdgeBase + kEdgeBytes + 15) / 16 * 16;  // 17296
constexpr int kRawStride = 52;
constexpr int kBallotBase = kRawBase + (kWin + 1) * kRawStride;    // 19844: 8 ballot words per wavefront
constexpr int kWinLdsBytes = kBallotBase + 2 * 8 * 4;              // 19908 per workgroup
constexpr int kExtractWaves = 2;                           // wavefronts per workgroup
constexpr int kLdsPerCu = 160 * 1024;                      // gfx950

// Matching.
constexpr int kTileRows = 32;                    // train rows per MFMA tile
constexpr int kTileBytes = kTileRows * 512;      // expanded tile: 16 steps x 64 lanes x 16 B
constexpr int kMaxSplitRows = (1 << 21) - 32;    // split-local train index < 2^21 - 1
constexpr int64_t kMaxSplits = 65535;            // train splits of a single-pair call (grid y)
constexpr uint64_t kNoNeighbour = ~0ull;         // partial-result sentinel

// Sticky error-word bits (same values as the LATCH_FLAG_* of the C ABI).
constexpr uint32_t kFlagBadKeypoint = 1u;
constexpr uint32_t kFlagBadImage = 2u;
constexpr uint32_t kFlagBadPair = 4u;
constexpr int64_t kMaxRows = 2147483647LL;

// Layout-compatible with latch_image of the C ABI.
struct ImageEntry {
    const uint8_t *img;
    int32_t height, width, pitch, reserved;
};
static_assert(sizeof(ImageEntry) == 24, "latch_image layout");

// Per-pixel patch weights of the weighted kernel: row r, pixel pair i of an
// 8 x 8 patch as two 16-bit lanes (w[r][2i] | w[r][2i + 1] << 16).
struct WeightRows {
    uint32_t pair[32];
};

struct ExtractArgs {
    const uint8_t *img;            // single image (table == nullptr)
    int height, width, pitch;
    const ImageEntry *table;       // batch: image table and per-keypoint image ids
    const int32_t *image_id;
    int n_images;
    const float4 *kps;
    int64_t n;                     // keypoints (upper bound when n_dev is set)
    const int64_t *n_dev;          // optional device-side keypoint count
    const int2 *rot;          // [4096] {cos_q14, sin_q14}
    const uint2 *trip_off;    // [512] by slot: {offA | off1 << 16, off2} LDS byte offsets
    const uint32_t *unperm;   // [128] per (wavefront, lane): slots of its four output bits
    const uint16_t *gather;   // [kGatherClasses][kGatherClassEntries] gather order
    uint32_t *desc;
    uint32_t *flags;
    int num_cus;
    // Weighted geometry (window 0: the default 48 x 48, 7 x 7, unit weights).
    int window = 0;
    const uint2 *wtrip_off = nullptr;   // [512] by slot: LDS byte offsets of the patches
    const uint32_t *wunperm = nullptr;  // [256] per (wavefront, lane): slots of its two output bits
    WeightRows weights = {};
    // Batches: keypoint index at each position of a spatial order (default
    // kernel only), or nullptr to take the keypoints as given.
    const int32_t *order = nullptr;
};

hipError_t launch_extract(const ExtractArgs &a, hipStream_t stream);

// Spatial order of a batch's keypoints: (image, band of rows) buckets, a
// counting sort in the handle's or plan's workspace.  Batches of at least
// kOrderMinKeypoints keypoints (max_kps) are ordered before extraction.
constexpr int kOrderBandRows = 32;
constexpr int kOrderMaxBands = 64;
constexpr int64_t kOrderMinKeypoints = 1 << 18;

struct OrderLayout {
    int64_t max_buckets;                          // kOrderMaxBands * n_images + 1
    size_t band_base, counts, bucket, rank, order, total;   // byte offsets, total bytes
};
OrderLayout order_layout(int n_images, int64_t max_kps);
// Enqueues the order's five kernels; the order lands at ws + order_layout().order.
hipError_t launch_order(const ExtractArgs &a, uint8_t *ws, hipStream_t stream);
hipError_t launch_extract_weighted(const ExtractArgs &a, hipStream_t stream);
// LDS byte offset of the top-left pixel (top, left) of a patch in the
// weighted kernel's window of side `window` (48 or 64).
uint32_t weighted_patch_offset(int window, int top, int left);

// Dense extraction (every pixel of a region, upright, scale 1) and dense
// matching within a search window.
struct DenseArgs {
    const uint8_t *img;
    int height, width, pitch;
    int x0, y0, gw, gh;
    const uint2 *toff;        // [512] triplet order: texture offsets of A | C1 << 16, C2
    uint32_t *desc;
};

struct DenseMatchArgs {
    const uint32_t *query, *train;
    int gw, gh, radius, k;
    float ratio;
    int32_t *idx, *dist;
    uint8_t *accept;
};

constexpr int kDenseMaxRadius = 8;

hipError_t launch_dense_extract(const DenseArgs &a, hipStream_t stream);
hipError_t launch_dense_match(const DenseMatchArgs &a, hipStream_t stream);
// Texture offset of a patch centre (r, c) in the dense kernel's tile.
uint32_t dense_patch_offset(int r, int c);

// Keypoint detection (FAST-9, suppression, intensity-centroid orientation).
constexpr int kDetectBorder = 16;
constexpr int kOrientRadius = 15;

struct DetectArgs {
    const uint8_t *img;
    int height, width, pitch, threshold;
    uint64_t *masks;          // workspace: survivor mask per (row, 64-column tile)
    uint8_t *counts;          // workspace: survivors per (row, tile), rows of count_stride bytes
    int count_stride;         // bytes per counts row: tiles rounded up to a multiple of 16
    int64_t *row_first;       // workspace: height (absolute output slot of each row)
    int64_t *base;            // workspace: the count on entry
    float4 *kps;
    int64_t max_kps;
    int64_t *n_kps;           // device, in/out: keypoints already in kps, then the new total
    int32_t *image_id;        // optional
    int32_t image_index;
};

hipError_t launch_detect(const DetectArgs &a, hipStream_t stream);

struct KnnPlan {
    int64_t nq, nt;
    int64_t split_rows;       // multiple of kTileRows, <= kMaxSplitRows
    int nsplit;
};

// Single-pair matching over train splits.  With one split the results are
// written directly; otherwise each (split, query) writes its two best as
// partials and launch_knn_merge reduces them.
// Which matcher kernel runs.
enum class SplitKernel { kMfmaI8, kMfmaFp4, kPopcount };

// Tile shapes and selection variants of the MFMA matchers (from the tuning
// table; none changes results).
struct KnnShape {
    int fp4_query_blocks = 3;       // 32-query blocks per wavefront of the MXFP4 kernels: 2 or 3
    int batch_groups_per_cu = 2;    // persistent workgroups per CU of the batched MFMA matchers
};

struct KnnSplitArgs {
    const uint32_t *query, *train;
    KnnShape shape;
    KnnPlan plan;
    uint64_t *partial;
    int k;
    float ratio;
    int32_t *idx, *dist;
    uint8_t *accept;
};

constexpr int64_t kFp4MaxSplitRows = 1 << 14;    // MXFP4 keys hold a 14-bit split-local index
constexpr int kMfmaWaves = 4;                    // wavefronts per MFMA matcher workgroup

hipError_t launch_knn_split(const KnnSplitArgs &a, SplitKernel which, hipStream_t stream);
// Queries per workgroup of a matcher kernel (the unit of query groups and batch items).
int queries_per_group(SplitKernel which, const KnnShape &shape);
hipError_t launch_knn_merge(const KnnSplitArgs &a, hipStream_t stream);

// Layout-compatible with latch_pair of the C ABI.
struct PairEntry {
    int64_t query_first, nq, train_first, nt, out_first;
};
static_assert(sizeof(PairEntry) == 40, "latch_pair layout");

struct PairInfo {            // per pair, computed on the device
    int64_t item_first;
    int32_t qgroups;
    int32_t valid;
};

struct BatchState {          // batch header in the workspace
    int64_t items;
    uint32_t next_item;      // atomic work counter, reset by the setup kernel
    uint32_t pad;
};


struct BatchArgs {
    const uint32_t *query, *train;
    int64_t query_rows, train_rows, out_rows;
    const PairEntry *pairs;
    int n_pairs;
    int64_t item_capacity;
    PairInfo *info;
    BatchState *state;
    int32_t *item_pair;
    int k;
    float ratio;
    int32_t *idx, *dist;
    uint8_t *accept;
    uint32_t *flags;
    int num_cus;
    SplitKernel kind;
    KnnShape shape;
};

hipError_t launch_knn_batch(const BatchArgs &a, hipStream_t stream);

}  // namespace latch
