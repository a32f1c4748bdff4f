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

// Extraction LDS layout, per wavefront: eight byte-shifted copies of the
// 48 x 48 u8 window.  Copy s holds, at byte (r * kRowBytes + x), window byte
// (r, x + s).  Any 7-byte patch row starting at column c0 is then the first
// 7 bytes of the 8-byte-aligned quadword at copy (c0 & 7), column c0 - (c0 & 7).
constexpr int kShiftCopies = 8;
constexpr int kRowBytes = 48;
constexpr int kCopyBytes = kWin * kRowBytes;               // 2304
constexpr int kWinLdsBytes = kShiftCopies * kCopyBytes;    // 18432 per workgroup
constexpr int kExtractWaves = 2;                           // wavefronts per workgroup
constexpr int kLdsPerCu = 160 * 1024;                      // gfx950

// Matching.
constexpr int kTileRows = 32;                    // train rows per MFMA tile
constexpr int kTileBytes = kTileRows * 512;      // expanded tile: 16 steps x 64 lanes x 16 B
constexpr int kMaxSplitRows = (1 << 21) - 32;    // split-local train index < 2^21 - 1
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
    const uint2 *trip_off;    // [512] {offA | off1 << 16, off2} LDS byte offsets
    uint32_t *desc;
    uint32_t *flags;
    int num_cus;
};

hipError_t launch_extract(const ExtractArgs &a, hipStream_t stream);

struct KnnPlan {
    int64_t nq, nt;
    int64_t split_rows;       // multiple of kTileRows, <= kMaxSplitRows
    int nsplit;
};

hipError_t launch_knn_mfma(const uint32_t *query, const uint32_t *train, const KnnPlan &plan,
                           uint64_t *partial, hipStream_t stream);
hipError_t launch_knn_popcount(const uint32_t *query, const uint32_t *train, const KnnPlan &plan,
                               uint64_t *partial, hipStream_t stream);
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
    bool mfma;
};

hipError_t launch_knn_batch(const BatchArgs &a, hipStream_t stream);

hipError_t launch_knn_merge(const uint64_t *partial, const KnnPlan &plan, int k, float ratio,
                            int32_t *idx, int32_t *dist, uint8_t *accept, hipStream_t stream);

}  // namespace latch
