// Spatial order of a batch's keypoints for extraction.
//
// A batched extraction reads each keypoint's window from its image.  With
// keypoints in arbitrary order, the workgroups in flight on one XCD touch
// the whole of an image that is larger than that XCD's L2, and the gather
// re-fetches most of its lines (on 64 images of 3000 x 2000, about 18 KB per
// keypoint from beyond L2).  Ordering the keypoints by (image, band of image
// rows) before extraction makes the keypoints an XCD works on at any time a
// few bands of one image.  The order is a counting sort into buckets
// (image i, band b), with band b of an image of height H holding the rows
// y with floor(y * bands / H) = b, bands = min(ceil(H / 32), 64):
//   1. per image, the first bucket (one workgroup, an exclusive scan);
//   2. the bucket counts are cleared;
//   3. each keypoint takes its bucket and a rank in it (counted per chunk of
//      keypoints in LDS, one global atomic add per chunk and bucket);
//   4. the counts become first positions (one workgroup, an exclusive scan);
//   5. each keypoint's index is written at its bucket's first position plus
//      its rank.
// Keypoints of a malformed image entry, or with a non-finite y, go to a last
// bucket of their own (extraction then flags them as before).  The order
// within a bucket depends on the atomics' timing, which changes nothing:
// every descriptor depends on its own keypoint only.
#include "internal.h"

namespace latch {
namespace {

constexpr int kOrderThreads = 256;

__device__ __forceinline__ bool image_ok(const ImageEntry &e)
{
    return e.img != nullptr && e.height >= 1 && e.width >= 1 && e.pitch >= e.width &&
           e.height < (1 << 23) && e.pitch < (1 << 23) &&
           (int64_t)e.height * e.pitch <= (int64_t)0x7fffffff;
}

__device__ __forceinline__ int bands_of(const ImageEntry &e)
{
    return image_ok(e) ? min((e.height + kOrderBandRows - 1) / kOrderBandRows, kOrderMaxBands) : 1;
}

// Exclusive scan of v over one workgroup (256 threads), in place over n
// entries (chunks of 256 with a running carry); returns the total.
__device__ int64_t block_scan(int32_t *v, int64_t n, int32_t *part)
{
    const int t = threadIdx.x;
    int64_t carry = 0;
    for (int64_t base = 0; base < n; base += kOrderThreads) {
        const int64_t i = base + t;
        const int32_t x = i < n ? v[i] : 0;
        part[t] = x;
        __syncthreads();
        for (int off = 1; off < kOrderThreads; off <<= 1) {
            const int32_t y = t >= off ? part[t - off] : 0;
            __syncthreads();
            part[t] += y;
            __syncthreads();
        }
        if (i < n) v[i] = (int32_t)(carry + part[t] - x);
        carry += part[kOrderThreads - 1];
        __syncthreads();
    }
    return carry;
}

// Step 1: first bucket of every image; band_base[n_images] is the bucket of
// the malformed keypoints (the last one).
__global__ __launch_bounds__(kOrderThreads) void order_bands_kernel(
    const ImageEntry *__restrict__ table, int n_images, int32_t *__restrict__ band_base)
{
    __shared__ int32_t part[kOrderThreads];
    for (int i = threadIdx.x; i < n_images; i += kOrderThreads) band_base[i] = bands_of(table[i]);
    __syncthreads();
    const int64_t total = block_scan(band_base, n_images, part);
    if (threadIdx.x == 0) band_base[n_images] = (int32_t)total;
}

// Step 2: clear the bucket counts.
__global__ __launch_bounds__(kOrderThreads) void order_clear_kernel(int32_t *__restrict__ counts,
                                                                   int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kOrderThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kOrderThreads)
        counts[i] = 0;
}

__device__ __forceinline__ int64_t keypoint_count(int64_t n_host, const int64_t *n_dev)
{
    int64_t n = n_host;
    if (n_dev) n = min(n, max(*n_dev, (int64_t)0));
    return n;
}

// Step 3: bucket and rank of every keypoint.  A workgroup takes a chunk of
// kOrderChunk consecutive keypoints.  When the chunk's buckets span fewer
// than kOrderChunk values (keypoints of one or two images, as a batch built
// image by image has them) it counts them in LDS, ranking each keypoint
// within the chunk, then takes one global atomic per bucket it touched for
// the chunk's first rank there; otherwise every keypoint takes its rank with
// a global atomic.
constexpr int kOrderChunk = 4096;
constexpr int kOrderPerThread = kOrderChunk / kOrderThreads;

__device__ __forceinline__ int bucket_of(const float4 *__restrict__ kps,
                                         const int32_t *__restrict__ image_id,
                                         const ImageEntry *__restrict__ table, int n_images,
                                         const int32_t *__restrict__ band_base, int64_t p)
{
    const int id = image_id[p];
    int b = band_base[n_images];
    if (id >= 0 && id < n_images) {
        const ImageEntry e = table[id];
        const float y = kps[p].y;
        if (image_ok(e) && __builtin_isfinite(y)) {
            const int bands = bands_of(e);
            const int row = (int)fminf(fmaxf(floorf(y), 0.0f), (float)(e.height - 1));
            b = band_base[id] + (int)((int64_t)row * bands / e.height);
        }
    }
    return b;
}

__global__ __launch_bounds__(kOrderThreads) void order_count_kernel(
    const float4 *__restrict__ kps, const int32_t *__restrict__ image_id,
    const ImageEntry *__restrict__ table, int n_images, int64_t n_host,
    const int64_t *__restrict__ n_dev, const int32_t *__restrict__ band_base,
    int32_t *__restrict__ counts, int32_t *__restrict__ bucket, int32_t *__restrict__ rank)
{
    __shared__ int32_t hist[kOrderChunk];
    __shared__ int32_t lo_s, hi_s;
    const int64_t n = keypoint_count(n_host, n_dev);
    const int64_t first = (int64_t)blockIdx.x * kOrderChunk;
    if (first >= n) return;                       // uniform over the workgroup
    const int t = threadIdx.x;
    int b[kOrderPerThread];
    int lo = 0x7fffffff, hi = -1;
#pragma unroll
    for (int i = 0; i < kOrderPerThread; ++i) {
        const int64_t p = first + i * kOrderThreads + t;
        b[i] = p < n ? bucket_of(kps, image_id, table, n_images, band_base, p) : -1;
        if (b[i] >= 0) {
            lo = min(lo, b[i]);
            hi = max(hi, b[i]);
        }
    }
    if (t == 0) {
        lo_s = 0x7fffffff;
        hi_s = -1;
    }
    __syncthreads();
    atomicMin(&lo_s, lo);
    atomicMax(&hi_s, hi);
    __syncthreads();
    const int base = lo_s, span = hi_s - lo_s + 1;    // the chunk has a keypoint: span >= 1
    if (span > kOrderChunk) {
#pragma unroll
        for (int i = 0; i < kOrderPerThread; ++i) {
            const int64_t p = first + i * kOrderThreads + t;
            if (b[i] >= 0) {
                bucket[p] = b[i];
                rank[p] = atomicAdd(&counts[b[i]], 1);
            }
        }
        return;
    }
    for (int i = t; i < span; i += kOrderThreads) hist[i] = 0;
    __syncthreads();
    int r[kOrderPerThread];
#pragma unroll
    for (int i = 0; i < kOrderPerThread; ++i)
        r[i] = b[i] >= 0 ? atomicAdd(&hist[b[i] - base], 1) : 0;
    __syncthreads();
    for (int i = t; i < span; i += kOrderThreads) {
        const int c = hist[i];
        if (c > 0) hist[i] = atomicAdd(&counts[base + i], c);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kOrderPerThread; ++i) {
        const int64_t p = first + i * kOrderThreads + t;
        if (b[i] >= 0) {
            bucket[p] = b[i];
            rank[p] = hist[b[i] - base] + r[i];
        }
    }
}

// Step 4: counts -> first positions.
__global__ __launch_bounds__(kOrderThreads) void order_scan_kernel(
    const int32_t *__restrict__ band_base, int n_images, int32_t *__restrict__ counts)
{
    __shared__ int32_t part[kOrderThreads];
    block_scan(counts, (int64_t)band_base[n_images] + 1, part);
}

// Step 5: the order.
__global__ __launch_bounds__(kOrderThreads) void order_scatter_kernel(
    int64_t n_host, const int64_t *__restrict__ n_dev, const int32_t *__restrict__ first,
    const int32_t *__restrict__ bucket, const int32_t *__restrict__ rank,
    int32_t *__restrict__ order)
{
    const int64_t n = keypoint_count(n_host, n_dev);
    for (int64_t p = (int64_t)blockIdx.x * kOrderThreads + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * kOrderThreads)
        order[first[bucket[p]] + rank[p]] = (int32_t)p;
}

}  // namespace

OrderLayout order_layout(int n_images, int64_t max_kps)
{
    auto up = [](size_t v) { return (v + 255) / 256 * 256; };
    OrderLayout l;
    l.max_buckets = (int64_t)kOrderMaxBands * n_images + 1;
    l.band_base = 0;
    l.counts = up(((size_t)n_images + 1) * sizeof(int32_t));
    l.bucket = l.counts + up((size_t)l.max_buckets * sizeof(int32_t));
    l.rank = l.bucket + up((size_t)max_kps * sizeof(int32_t));
    l.order = l.rank + up((size_t)max_kps * sizeof(int32_t));
    l.total = l.order + up((size_t)max_kps * sizeof(int32_t));
    return l;
}

hipError_t launch_order(const ExtractArgs &a, uint8_t *ws, hipStream_t stream)
{
    const OrderLayout l = order_layout(a.n_images, a.n);
    int32_t *band_base = reinterpret_cast<int32_t *>(ws + l.band_base);
    int32_t *counts = reinterpret_cast<int32_t *>(ws + l.counts);
    int32_t *bucket = reinterpret_cast<int32_t *>(ws + l.bucket);
    int32_t *rank = reinterpret_cast<int32_t *>(ws + l.rank);
    int32_t *order = reinterpret_cast<int32_t *>(ws + l.order);
    const int64_t per_pass = (int64_t)a.num_cus * 8 * kOrderThreads;
    const unsigned grid_kps = (unsigned)min((a.n + kOrderThreads - 1) / kOrderThreads,
                                            per_pass / kOrderThreads);
    const unsigned grid_chunks = (unsigned)((a.n + kOrderChunk - 1) / kOrderChunk);
    const unsigned grid_clear = (unsigned)min((l.max_buckets + kOrderThreads - 1) / kOrderThreads,
                                              per_pass / kOrderThreads);
    hipLaunchKernelGGL(order_bands_kernel, dim3(1), dim3(kOrderThreads), 0, stream, a.table,
                       a.n_images, band_base);
    hipLaunchKernelGGL(order_clear_kernel, dim3(grid_clear), dim3(kOrderThreads), 0, stream, counts,
                       l.max_buckets);
    hipLaunchKernelGGL(order_count_kernel, dim3(grid_chunks), dim3(kOrderThreads), 0, stream, a.kps,
                       a.image_id, a.table, a.n_images, a.n, a.n_dev, band_base, counts, bucket,
                       rank);
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(kOrderThreads), 0, stream, band_base,
                       a.n_images, counts);
    hipLaunchKernelGGL(order_scatter_kernel, dim3(grid_kps), dim3(kOrderThreads), 0, stream, a.n,
                       a.n_dev, counts, bucket, rank, order);
    return hipGetLastError();
}

}  // namespace latch
