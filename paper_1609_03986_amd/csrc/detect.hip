// Keypoint detection for gfx950: FAST-9 corners with suppression and an
// intensity-centroid orientation (the paper detects FAST keypoints and
// extracts LATCH at their orientation, Sec. 3.2; the score, suppression and
// orientation method are not stated there and are fixed as follows).
//
//   * Score: for the 16 pixels of the radius-3 circle and c the centre, the
//     largest over the 16 arcs of 9 consecutive circle pixels and over both
//     polarities of the smallest difference on the arc (q - c brighter,
//     c - q darker).  A corner for threshold t has score > t.
//   * Pixels at least kDetectBorder from every edge are tested; the score
//     map holds the score of corners there and 0 elsewhere.  Suppression
//     keeps p iff S(p) > 0 and S(p) > S(q) for its 8 neighbours.
//   * Output in raster order: per-row counts, a scan, then per-row writes.
//   * Orientation: moments m10 = sum dx I, m01 = sum dy I over the disc of
//     radius kOrientRadius, bin = rne(atan2(m01, m10) * 4096 / 2 pi) mod 4096
//     in double (integer moments keep the angle far enough from a bin
//     boundary that the bin does not depend on the last bits of atan2), and
//     the keypoint angle bin * 360 / 4096 degrees, exact in float.
#include "internal.h"

namespace latch {
namespace {

constexpr int kScoreBlockX = 64, kScoreBlockY = 4;
constexpr int kRowThreads = 256;

// Circle offsets, clockwise from the top (y downwards).
__constant__ int2 kCircle[16] = {{0, -3}, {1, -3},  {2, -2},  {3, -1}, {3, 0},   {3, 1},
                                 {2, 2},  {1, 3},   {0, 3},   {-1, 3}, {-2, 2},  {-3, 1},
                                 {-3, 0}, {-3, -1}, {-2, -2}, {-1, -3}};

__global__ __launch_bounds__(kScoreBlockX *kScoreBlockY) void fast_score_kernel(
    const uint8_t *__restrict__ img, int height, int width, int pitch, int threshold,
    uint8_t *__restrict__ score, int x_blocks)
{
    // One-dimensional grid (the y extent of a tall image exceeds grid.y).
    const int x = (int)(blockIdx.x % (unsigned)x_blocks) * kScoreBlockX + threadIdx.x;
    const int y = (int)(blockIdx.x / (unsigned)x_blocks) * kScoreBlockY + threadIdx.y;
    if (x >= width || y >= height) return;
    int s = 0;
    if (x >= kDetectBorder && x < width - kDetectBorder && y >= kDetectBorder &&
        y < height - kDetectBorder) {
        const uint8_t *p = img + (size_t)y * pitch + x;
        const int c = p[0];
        int d[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) d[i] = (int)p[kCircle[i].y * pitch + kCircle[i].x] - c;
        // Smallest (brighter) and largest (darker) difference on each arc of
        // 9, by doubling: arcs of 2, 4, 8, then 9.
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
        s = best > threshold ? best : 0;
    }
    score[(size_t)y * width + x] = (uint8_t)s;
}

__device__ __forceinline__ bool keep_at(const uint8_t *__restrict__ score, int width, int x, int y)
{
    const uint8_t *p = score + (size_t)y * width + x;
    const int s = p[0];
    if (s == 0) return false;      // also every pixel outside the tested region
    return s > p[-width - 1] && s > p[-width] && s > p[-width + 1] && s > p[-1] && s > p[1] &&
           s > p[width - 1] && s > p[width] && s > p[width + 1];
}

// Suppression survivors per row.
__global__ __launch_bounds__(kRowThreads) void nms_count_kernel(const uint8_t *__restrict__ score,
                                                                int height, int width,
                                                                int32_t *__restrict__ row_count)
{
    __shared__ int part[kRowThreads / 64];
    const int y = blockIdx.x;
    int c = 0;
    if (y >= kDetectBorder && y < height - kDetectBorder)
        for (int x = threadIdx.x; x < width; x += kRowThreads) c += keep_at(score, width, x, y);
    // Wavefront sums, then the block's.
    for (int m = 32; m > 0; m >>= 1) c += __shfl_xor(c, m);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < kRowThreads / 64; ++i) t += part[i];
        row_count[y] = t;
    }
}

// Exclusive scan of the row counts (one block), and the total.
__global__ __launch_bounds__(1024) void row_scan_kernel(const int32_t *__restrict__ row_count,
                                                        int height, int64_t *__restrict__ row_first,
                                                        int64_t *__restrict__ total)
{
    __shared__ int64_t buf[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < height; base += 1024) {
        const int i = base + threadIdx.x;
        const int64_t v = i < height ? row_count[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t add = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < height) row_first[i] = carry + buf[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// Keypoints of one row, in order of x.
__global__ __launch_bounds__(kRowThreads) void nms_write_kernel(
    const uint8_t *__restrict__ score, int height, int width, const int64_t *__restrict__ row_first,
    float4 *__restrict__ kps, int64_t max_kps, int32_t *__restrict__ image_id, int32_t image_index)
{
    __shared__ int part[kRowThreads / 64];
    const int y = blockIdx.x;
    if (y < kDetectBorder || y >= height - kDetectBorder) return;
    int64_t next = row_first[y];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int x0 = 0; x0 < width; x0 += kRowThreads) {
        if (next >= max_kps) break;                      // uniform across the block
        const int x = x0 + threadIdx.x;
        const bool k = x < width && keep_at(score, width, x, y);
        const uint64_t mask = __ballot(k);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) part[wave] = __popcll(mask);
        __syncthreads();
        int offset = 0, total = 0;
        for (int i = 0; i < kRowThreads / 64; ++i) {
            offset += i < wave ? part[i] : 0;
            total += part[i];
        }
        const int64_t slot = next + offset + before;
        if (k && slot < max_kps) {
            kps[slot] = make_float4((float)x, (float)y, 0.f, 1.f);
            if (image_id) image_id[slot] = image_index;
        }
        next += total;
        __syncthreads();                                 // part[] is reused
    }
}

// Orientation of each keypoint: one wavefront per keypoint; lanes 0..30
// and 32..62 take dx = -15..15 of two disc rows per pass.
__global__ __launch_bounds__(256) void orient_kernel(const uint8_t *__restrict__ img, int pitch,
                                                     float4 *__restrict__ kps,
                                                     const int64_t *__restrict__ n_dev,
                                                     int64_t max_kps)
{
    const int lane = threadIdx.x & 63;
    const int64_t n = min(*n_dev, max_kps);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int dx = (lane & 31) - kOrientRadius;
    const int row_in_pass = lane >> 5;
    for (int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); k < n; k += waves) {
        const float4 kp = kps[k];
        const int x = (int)kp.x, y = (int)kp.y;
        int m10 = 0, m01 = 0;
        if ((lane & 31) <= 2 * kOrientRadius) {
            for (int dy0 = -kOrientRadius; dy0 <= kOrientRadius; dy0 += 2) {
                const int dy = dy0 + row_in_pass;
                if (dy <= kOrientRadius && dx * dx + dy * dy <= kOrientRadius * kOrientRadius) {
                    const int v = img[(size_t)(y + dy) * pitch + (x + dx)];
                    m10 += dx * v;
                    m01 += dy * v;
                }
            }
        }
        for (int m = 32; m > 0; m >>= 1) {
            m10 += __shfl_xor(m10, m);
            m01 += __shfl_xor(m01, m);
        }
        if (lane == 0) {
            const double a = atan2((double)m01, (double)m10);
            const int bin = (int)((int64_t)rint(a * (4096.0 / (2.0 * 3.14159265358979323846))) & 4095);
            kps[k].z = (float)bin * (360.0f / 4096.0f);
        }
    }
}

}  // namespace

hipError_t launch_detect(const DetectArgs &a, hipStream_t stream)
{
    const int x_blocks = (a.width + kScoreBlockX - 1) / kScoreBlockX;
    const int64_t y_blocks = (a.height + kScoreBlockY - 1) / kScoreBlockY;
    hipLaunchKernelGGL(fast_score_kernel, dim3((unsigned)(x_blocks * y_blocks)),
                       dim3(kScoreBlockX, kScoreBlockY), 0, stream, a.img, a.height, a.width,
                       a.pitch, a.threshold, a.score, x_blocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(nms_count_kernel, dim3((unsigned)a.height), dim3(kRowThreads), 0, stream,
                       a.score, a.height, a.width, a.row_count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(row_scan_kernel, dim3(1), dim3(1024), 0, stream, a.row_count, a.height,
                       a.row_first, a.n_kps);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(nms_write_kernel, dim3((unsigned)a.height), dim3(kRowThreads), 0, stream,
                       a.score, a.height, a.width, a.row_first, a.kps, a.max_kps, a.image_id,
                       a.image_index);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.max_kps > 0) {
        const int64_t want = (a.max_kps + 3) / 4;
        const int64_t cap = (int64_t)a.num_cus * 16;
        const int blocks = (int)(want < cap ? want : cap);
        hipLaunchKernelGGL(orient_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a.img,
                           a.pitch, a.kps, a.n_kps, a.max_kps);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace latch
