// Keypoint detection for gfx950: FAST-9 corners with suppression and an
// intensity-centroid orientation (the paper detects FAST keypoints and
// extracts LATCH at their orientation, Sec. 3.2; the score, suppression and
// orientation method are not stated there and are fixed as follows).
//
//   * Score: for the 16 pixels of the radius-3 circle and c the centre, the
//     largest over the 16 arcs of 9 consecutive circle pixels and over both
//     polarities of the smallest difference on the arc (q - c brighter,
//     c - q darker).  A corner for threshold t has score > t.
//   * Pixels at least kDetectBorder from every edge are tested; others score
//     0.  Suppression keeps p iff S(p) > 0 and S(p) > S(q) for its 8
//     neighbours.
//   * Output in raster order, appended after the keypoints already counted
//     in *n_kps.
//   * Orientation: moments m10 = sum dx I, m01 = sum dy I over the disc of
//     radius kOrientRadius, bin = rne(atan2(m01, m10) * 4096 / 2 pi) mod 4096
//     in double (integer moments keep the angle far enough from a bin
//     boundary that the bin does not depend on the last bits of atan2), and
//     the keypoint angle bin * 360 / 4096 degrees, exact in float.
//
// Three launches:
//   1. detect_tile_kernel: a 64 x 16 tile per workgroup.  The image tile with
//      a 4-pixel halo is staged in LDS, scores of the tile and a 1-pixel halo
//      go to LDS, and each wavefront's ballot over one tile row is that row's
//      64-bit survivor mask; the mask and its popcount (one byte per row and
//      tile, rows of the count array padded to 16 bytes) go to the workspace.
//   2. detect_scan_kernel: one workgroup sums each row's count bytes (two
//      rows per thread) and scans them into each row's first output slot and
//      the new total.
//   3. detect_emit_kernel: per tile, the image window of every disc staged in
//      LDS; per tile row, the slot of each survivor from the row's first slot,
//      the count bytes of the tiles to its left and the mask, its orientation
//      with one disc row per lane (two keypoints per wavefront), then the
//      keypoint written once, complete.
#include "internal.h"

namespace latch {
namespace {

constexpr int kTileW = 64, kTileH = 16;
constexpr int kHaloImg = 4;                            // circle radius 3 + suppression 1
constexpr int kImgW = kTileW + 2 * kHaloImg;           // 72
constexpr int kImgH = kTileH + 2 * kHaloImg;           // 24
constexpr int kScoreW = kTileW + 2, kScoreH = kTileH + 2;   // 66 x 18
constexpr int kThreads = 256;
constexpr int kScanThreads = 1024;
constexpr int kDiscRows = 2 * kOrientRadius + 1;       // 31

// Circle offsets, clockwise from the top (y downwards).
__constant__ int2 kCircle[16] = {{0, -3}, {1, -3},  {2, -2},  {3, -1}, {3, 0},   {3, 1},
                                 {2, 2},  {1, 3},   {0, 3},   {-1, 3}, {-2, 2},  {-3, 1},
                                 {-3, 0}, {-3, -1}, {-2, -2}, {-1, -3}};

// FAST-9 score of the pixel at p (an LDS image tile of row stride kImgW).
__device__ __forceinline__ int fast_score(const uint8_t *p)
{
    const int c = p[0];
    int d[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) d[i] = (int)p[kCircle[i].y * kImgW + kCircle[i].x] - c;
    // Smallest (brighter) and largest (darker) difference on each arc of 9,
    // by doubling: arcs of 2, 4, 8, then 9.
    int lo2[16], hi2[16], lo4[16], hi4[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        lo2[i] = min(d[i], d[(i + 1) & 15]);
        hi2[i] = max(d[i], d[(i + 1) & 15]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        lo4[i] = min(lo2[i], lo2[(i + 2) & 15]);
        hi4[i] = max(hi2[i], hi2[(i + 2) & 15]);
    }
    int best = -256;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int lo9 = min(min(lo4[i], lo4[(i + 4) & 15]), d[(i + 8) & 15]);
        const int hi9 = max(max(hi4[i], hi4[(i + 4) & 15]), d[(i + 8) & 15]);
        best = max(best, max(lo9, -hi9));
    }
    return best;
}

// Copies rows ry0 .. ry0 + kRows - 1 and columns cx0 .. cx0 + kCols - 1 of
// the image into LDS (row stride kStride), coordinates clamped to the image
// (callers never use the clamped values).  kDword: 4-byte loads, for a
// 4-byte-aligned image whose pitch and width are multiples of 4 (cx0 and
// kCols are); otherwise byte loads.  Every load is issued before the first
// LDS write; lds must hold kStageRows<kDword, kRows, kCols> rows.
template <bool kDword, int kRows, int kCols>
struct Stage {
    static constexpr int kUnit = kDword ? 4 : 1;
    static constexpr int kPerRow = kCols / kUnit;
    static constexpr int kLoads = (kRows * kPerRow + kThreads - 1) / kThreads;
    static constexpr int kLdsRows = (kLoads * kThreads + kPerRow - 1) / kPerRow;
};

template <bool kDword, int kRows, int kCols, int kStride>
__device__ __forceinline__ void stage_window(const uint8_t *__restrict__ img, int height, int width,
                                             int pitch, int ry0, int cx0, uint8_t *lds)
{
    using S = Stage<kDword, kRows, kCols>;
    const int t = threadIdx.x;
    uint32_t v[S::kLoads];
#pragma unroll
    for (int k = 0; k < S::kLoads; ++k) {
        const int i = t + k * kThreads;
        const int yy = min(max(ry0 + i / S::kPerRow, 0), height - 1);
        const int xx = min(max(cx0 + S::kUnit * (i % S::kPerRow), 0), width - S::kUnit);
        const uint8_t *p = img + (size_t)yy * pitch + xx;
        if constexpr (kDword)
            v[k] = *reinterpret_cast<const uint32_t *>(p);
        else
            v[k] = *p;
    }
#pragma unroll
    for (int k = 0; k < S::kLoads; ++k) {
        const int i = t + k * kThreads;
        uint8_t *q = lds + (i / S::kPerRow) * kStride + S::kUnit * (i % S::kPerRow);
        if constexpr (kDword)
            *reinterpret_cast<uint32_t *>(q) = v[k];
        else
            *q = (uint8_t)v[k];
    }
}

template <int kRows, int kCols>
constexpr int stage_lds_rows()
{
    return Stage<true, kRows, kCols>::kLdsRows > Stage<false, kRows, kCols>::kLdsRows
               ? Stage<true, kRows, kCols>::kLdsRows
               : Stage<false, kRows, kCols>::kLdsRows;
}

template <bool kDword>
__global__ __launch_bounds__(kThreads) void detect_tile_kernel(
    const uint8_t *__restrict__ img, int height, int width, int pitch, int threshold, int tiles_x,
    uint64_t *__restrict__ masks, uint8_t *__restrict__ counts, int count_stride)
{
    __shared__ __align__(16) uint8_t timg[stage_lds_rows<kImgH, kImgW>() * kImgW];
    __shared__ uint8_t tscore[kScoreH * kScoreW];
    const int tx = (int)(blockIdx.x % (unsigned)tiles_x), ty = (int)(blockIdx.x / (unsigned)tiles_x);
    const int x0 = tx * kTileW, y0 = ty * kTileH;
    const int t = threadIdx.x;

    // Image tile with halo.  Clamped pixels only reach scores outside the
    // tested region, which are 0 regardless.
    stage_window<kDword, kImgH, kImgW, kImgW>(img, height, width, pitch, y0 - kHaloImg, x0 - kHaloImg,
                                              timg);
    __syncthreads();

    // Scores of the tile and a 1-pixel halo.
    for (int i = t; i < kScoreH * kScoreW; i += kThreads) {
        const int sy = i / kScoreW, sx = i % kScoreW;
        const int yy = y0 - 1 + sy, xx = x0 - 1 + sx;
        int s = 0;
        if (yy >= kDetectBorder && yy < height - kDetectBorder && xx >= kDetectBorder &&
            xx < width - kDetectBorder) {
            s = fast_score(&timg[(sy + kHaloImg - 1) * kImgW + sx + kHaloImg - 1]);
            s = s > threshold ? s : 0;
        }
        tscore[i] = (uint8_t)s;
    }
    __syncthreads();

    // Suppression: wavefront w takes tile rows w, w + 4, ...; lane = column.
    const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    for (int r = wave; r < kTileH; r += kThreads / 64) {
        const int y = y0 + r;
        if (y >= height) break;                         // uniform across the wavefront
        const uint8_t *p = &tscore[(r + 1) * kScoreW + lane + 1];
        const int s = p[0];
        const bool keep = s > 0 && s > p[-kScoreW - 1] && s > p[-kScoreW] && s > p[-kScoreW + 1] &&
                          s > p[-1] && s > p[1] && s > p[kScoreW - 1] && s > p[kScoreW] &&
                          s > p[kScoreW + 1];
        const uint64_t m = __ballot(keep);
        if (lane == 0) {
            masks[(size_t)tx * height + y] = m;
            counts[(size_t)y * count_stride + tx] = (uint8_t)__popcll(m);
        }
    }
}

// Inclusive scan over the 1024 threads of the workgroup (wavefront shuffles,
// then the 16 wavefront totals).
__device__ __forceinline__ int64_t block_inclusive_scan(int64_t v, int64_t *wave_tot)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(v, o);
        if (lane >= o) v += u;
    }
    if (lane == 63) wave_tot[wave] = v;
    __syncthreads();
    int64_t before = 0;
    for (int i = 0; i < wave; ++i) before += wave_tot[i];
    __syncthreads();                                    // wave_tot is reused by the next call
    return v + before;
}

__global__ __launch_bounds__(kScanThreads) void detect_scan_kernel(
    const uint8_t *__restrict__ counts, int count_stride, int height, int tiles_x,
    int64_t *__restrict__ row_first, int64_t *__restrict__ base_out, int64_t *__restrict__ n_kps)
{
    __shared__ int64_t wave_tot[kScanThreads / 64];
    __shared__ int64_t base, chunk_total;
    if (threadIdx.x == 0) {
        const int64_t n0 = *n_kps;
        base = n0 > 0 ? n0 : 0;                          // a negative count is taken as 0
        *base_out = base;
    }
    __syncthreads();
    const int chunks = count_stride / 16;                 // 16 tile counts per chunk
    // Survivors of row r: its counts, one byte per tile, four 16-byte chunks
    // in flight; bytes past tiles_x (never written) are masked off.
    auto row_count = [&](const uint4 (&v)[4], int i) {
        int64_t c = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int valid = min(max(tiles_x - 16 * (i + k), 0), 16);
            const uint32_t w[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const int nb = min(max(valid - 4 * d, 0), 4);
                const uint32_t keep = nb == 4 ? 0xffffffffu : (1u << (8 * nb)) - 1u;
                c += __builtin_amdgcn_sad_u8(w[d] & keep, 0u, 0u);
            }
        }
        return c;
    };
    int64_t carry = base;
    // Two rows per thread, so one pass covers 2048 rows.
    for (int r0 = 0; r0 < height; r0 += 2 * kScanThreads) {
        const int r = r0 + 2 * (int)threadIdx.x;
        int64_t c0 = 0, c1 = 0;
        if (r < height) {
            const uint4 *row0 = reinterpret_cast<const uint4 *>(counts + (size_t)r * count_stride);
            const uint4 *row1 =
                reinterpret_cast<const uint4 *>(counts + (size_t)min(r + 1, height - 1) * count_stride);
            for (int i = 0; i < chunks; i += 4) {
                uint4 v0[4], v1[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    v0[k] = row0[min(i + k, chunks - 1)];
                    v1[k] = row1[min(i + k, chunks - 1)];
                }
                c0 += row_count(v0, i);
                c1 += row_count(v1, i);
            }
            if (r + 1 >= height) c1 = 0;
        }
        const int64_t c = c0 + c1;
        const int64_t incl = block_inclusive_scan(c, wave_tot);
        if (r < height) row_first[r] = carry + incl - c;
        if (r + 1 < height) row_first[r + 1] = carry + incl - c1;
        if (threadIdx.x == kScanThreads - 1) chunk_total = incl;
        __syncthreads();
        carry += chunk_total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_kps = carry;
}

// Image window of one tile for the orientation: rows y0 - 15 .. y0 + 30 and
// columns x0 - 16 .. x0 + 79 (every disc of a pixel of the tile), row stride
// kOriStride bytes (25 dwords: the lanes of a disc, one row each, fall in
// distinct banks).
constexpr int kOriRows = kTileH + 2 * kOrientRadius;          // 46
constexpr int kOriCols = kTileW + 32;                          // 96
constexpr int kOriStride = 100;

// Byte masks of disc row dy (lane = dy + 15): of the 32 bytes starting at
// dx = -15, bytes k = 15 - r .. 15 + r with r = floor(sqrt(15^2 - dy^2)).
__device__ __forceinline__ void disc_masks(int dy, uint32_t (&bm)[8])
{
    const int r2 = kOrientRadius * kOrientRadius - dy * dy;
    // floor(sqrt(r2)) for r2 in [0, 225]: sqrt(k^2 + 1/2) and sqrt(k^2 - 1/2)
    // lie 1/(4k) from k, far beyond the rounding of sqrtf.
    const int r = (int)__builtin_sqrtf((float)r2 + 0.5f);
    const uint32_t keep = (uint32_t)(((1ull << (kOrientRadius + r + 1)) - 1ull) &
                                     ~((1ull << (kOrientRadius - r)) - 1ull));
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t nib = (keep >> (4 * i)) & 15u;
        bm[i] = ((nib * 0x00204081u) & 0x01010101u) * 0xffu;
    }
}

// Disc row dy of the keypoint at tile column j and tile row r_tile:
// S = sum I and W = sum k I with k = dx + 15, from 9 aligned dwords of the
// window.
__device__ __forceinline__ void disc_row(const uint8_t *win, int j, int r_tile, int dy,
                                         const uint32_t (&bm)[8], uint32_t &S, uint32_t &W)
{
    const int c = j + 1;                                   // window column of dx = -15
    const uint32_t *w =
        reinterpret_cast<const uint32_t *>(win + (r_tile + kOrientRadius + dy) * kOriStride) + (c >> 2);
    const uint32_t sh = (uint32_t)(c & 3);
    uint32_t d[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) d[i] = w[i];
    S = 0;
    W = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t v = __builtin_amdgcn_alignbyte(d[i + 1], d[i], sh) & bm[i];
        S = __builtin_amdgcn_udot4(v, 0x01010101u, S, false);
        W = __builtin_amdgcn_udot4(v, (uint32_t)(4 * i) * 0x01010101u + 0x03020100u, W, false);
    }
}

// Sum over each row of 16 lanes (DPP: swap neighbours, swap pairs, mirror
// halves, mirror the row); every lane of the row gets the row's sum.
__device__ __forceinline__ int row16_sum(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false);  // row_mirror
    return v;
}

// A value equal on every lane, in scalar registers.
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Angle bin of moments (m10, m01), in double as the definition states.
__device__ __forceinline__ int orientation_bin(int m10, int m01)
{
    const double a = atan2((double)m01, (double)m10);
    return (int)((int64_t)rint(a * (4096.0 / (2.0 * 3.14159265358979323846))) & 4095);
}

// One workgroup per tile: the tile's image window goes to LDS, then
// wavefront w takes the survivors of tile rows w, w + 4, ...  Moments are
// summed two keypoints per pass (one per half-wavefront, a disc row per
// lane); each keypoint's moments and slot are parked in the registers of
// lane n (its index in the wavefront's queue), and when 63 or more are
// queued, or at the end, every queued lane computes its angle and writes its
// keypoint.
template <bool kDword>
__global__ __launch_bounds__(kThreads) void detect_emit_kernel(
    const uint8_t *__restrict__ img, int height, int width, int pitch, int tiles_x,
    const uint64_t *__restrict__ masks, const uint8_t *__restrict__ counts, int count_stride,
    const int64_t *__restrict__ row_first, float4 *__restrict__ kps, int64_t max_kps,
    int32_t *__restrict__ image_id, int32_t image_index)
{
    // Rows past kOriRows take the rounding of the load count (never read).
    __shared__ __align__(16) uint8_t win[stage_lds_rows<kOriRows, kOriCols>() * kOriStride];
    const int tx = (int)(blockIdx.x % (unsigned)tiles_x), ty = (int)(blockIdx.x / (unsigned)tiles_x);
    const int x0 = tx * kTileW, y0 = ty * kTileH;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int half = lane >> 5, hl = lane & 31;
    const int dy = hl - kOrientRadius;

    // Coordinates clamped to the image: discs of survivors never leave it.
    stage_window<kDword, kOriRows, kOriCols, kOriStride>(img, height, width, pitch, y0 - kOrientRadius,
                                                         x0 - 16, win);
    uint32_t bm[8];
    disc_masks(dy, bm);
    __syncthreads();

    // The queue: lane n holds the n-th queued keypoint.
    int q_m10 = 0, q_m01 = 0, q_x = 0, q_y = 0;
    int64_t q_slot = 0;
    int queued = 0;                                       // uniform
    auto flush = [&]() {
        if (lane < queued && q_slot < max_kps) {
            const int bin = orientation_bin(q_m10, q_m01);
            kps[q_slot] = make_float4((float)q_x, (float)q_y, (float)bin * (360.0f / 4096.0f), 1.0f);
            if (image_id) image_id[q_slot] = image_index;
        }
        queued = 0;
    };

    for (int rt = wave; rt < kTileH; rt += kThreads / 64) {
        const int y = y0 + rt;
        if (y >= height) break;                           // uniform across the wavefront
        uint64_t m = masks[(size_t)tx * height + y];
        const int64_t rf = row_first[y];
        // Survivors of the tiles to the left in this row: their count bytes,
        // one tile per lane (one coalesced load for up to 64 tiles).
        int left = 0;
        for (int i = lane; i < tx; i += 64) left += counts[(size_t)y * count_stride + i];
        if (m == 0) continue;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) left += __shfl_xor(left, o);
        const int64_t first = uniform64(rf + left);
        if (first >= max_kps) continue;
        int rank = 0;                                     // survivors already queued from this row
        while (m) {
            const int j0 = __builtin_ctzll(m);
            const uint64_t m1 = m & (m - 1);
            const int j1 = m1 ? __builtin_ctzll(m1) : -1;
            m = m1 ? (m1 & (m1 - 1)) : 0;
            const int j = half ? j1 : j0;
            uint32_t S = 0, W = 0;
            if (j >= 0 && hl < kDiscRows) disc_row(win, j, rt, dy, bm, S, W);
            const int s10 = row16_sum((int)W - kOrientRadius * (int)S);
            const int s01 = row16_sum(dy * (int)S);
            // Half-wavefront sums from rows of 16 lanes.
            const int a10 = __builtin_amdgcn_readlane(s10, 0) + __builtin_amdgcn_readlane(s10, 16);
            const int a01 = __builtin_amdgcn_readlane(s01, 0) + __builtin_amdgcn_readlane(s01, 16);
            if (lane == queued) {
                q_m10 = a10;
                q_m01 = a01;
                q_x = x0 + j0;
                q_y = y;
                q_slot = first + rank;
            }
            if (j1 >= 0) {
                const int b10 = __builtin_amdgcn_readlane(s10, 32) + __builtin_amdgcn_readlane(s10, 48);
                const int b01 = __builtin_amdgcn_readlane(s01, 32) + __builtin_amdgcn_readlane(s01, 48);
                if (lane == queued + 1) {
                    q_m10 = b10;
                    q_m01 = b01;
                    q_x = x0 + j1;
                    q_y = y;
                    q_slot = first + rank + 1;
                }
                queued += 2;
                rank += 2;
            } else {
                queued += 1;
                rank += 1;
            }
            if (queued >= 63) flush();
        }
    }
    flush();
}

}  // namespace

hipError_t launch_detect(const DetectArgs &a, hipStream_t stream)
{
    const int tiles_x = (a.width + kTileW - 1) / kTileW;
    const int64_t tiles = (int64_t)tiles_x * ((a.height + kTileH - 1) / kTileH);
    const bool dword = (reinterpret_cast<uintptr_t>(a.img) & 3) == 0 && (a.pitch & 3) == 0 &&
                       (a.width & 3) == 0;
    hipLaunchKernelGGL(dword ? detect_tile_kernel<true> : detect_tile_kernel<false>,
                       dim3((unsigned)tiles), dim3(kThreads), 0, stream, a.img, a.height, a.width,
                       a.pitch, a.threshold, tiles_x, a.masks, a.counts, a.count_stride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(detect_scan_kernel, dim3(1), dim3(kScanThreads), 0, stream, a.counts,
                       a.count_stride, a.height, tiles_x, a.row_first, a.base, a.n_kps);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(dword ? detect_emit_kernel<true> : detect_emit_kernel<false>,
                       dim3((unsigned)tiles), dim3(kThreads), 0, stream, a.img, a.height, a.width,
                       a.pitch, tiles_x, a.masks, a.counts, a.count_stride, a.row_first, a.kps,
                       a.max_kps, a.image_id, a.image_index);
    return hipGetLastError();
}

}  // namespace latch
