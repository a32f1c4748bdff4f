// LATCH descriptor extraction for gfx950.
//
// A workgroup of two wavefronts computes one descriptor at a time
// (grid-stride over keypoints):
//   1. resampling rule steps 1-3 on the keypoint (uniform across the group);
//   2. gather of the 48 x 48 upright window (steps 4-5): thread t owns window
//      dwords d = t + 128 m, i.e. 20 or 16 samples, issued as independent
//      byte loads one keypoint ahead so that their latency overlaps the
//      previous descriptor's arithmetic;
//   3. eight byte-shifted copies of the window in LDS, so that every 7-byte
//      patch row is the head of one 8-byte-aligned ds_read_b64;
//   4. Eq. 1 (Sec. 3.1) for 512 triplets: each wavefront takes 4 rounds of 64
//      lanes, one triplet per lane per round, in exact integer arithmetic;
//   5. a 64-bit ballot per round packs the bits; 8 lanes per wavefront store
//      its 8 words.
//
// Patch distances.  With A, C the 7 x 7 patches of the anchor and one
// companion, ||A - C||^2 = sum A^2 + sum C^2 - 2 sum A C.  sum A^2 is shared by
// both sides of Eq. 1, so bit = [sum C1^2 - 2 sum A C1 > sum C2^2 - 2 sum A C2].
// Each 7-pixel row is 8 packed u8 (the 8th byte masked to zero in the
// companion operands) and each sum is a chain of v_dot4_u32_u8.  All sums are
// < 49 * 255^2 < 2^22, so the int32 result equals the exact integer one.
//
// The paper's CUDA kernel (Sec. 3.2) spreads one descriptor over 32 warps of
// a 1024-thread block with float32 patches in shared memory; here two 64-lane
// wavefronts share an 18 KB byte window (eight LDS windows per CU, four
// wavefronts per SIMD) and synchronise three times per descriptor.
#include "internal.h"

namespace latch {
namespace {

constexpr int kThreads = kExtractWaves * 64;             // 128: two wavefronts per window
constexpr int kGatherDwords = kWin * kWin / 4;            // 576
constexpr int kRowDwords = kRowBytes / 4;                 // 12
constexpr int kGatherPerThread = (kGatherDwords + kThreads - 1) / kThreads;   // 5
constexpr int kSamples = 4 * kGatherPerThread;            // 20
constexpr int kRoundsPerWave = 8 / kExtractWaves;         // 4
static_assert(kGatherDwords == kThreads * (kGatherPerThread - 1) + 64,
              "the last gather dword row belongs to wavefront 0 exactly");

// n / 2^22 rounded half away from zero, for |n| < 2^31 - 2^21.
// n >= 0: floor((n + 2^21) / 2^22).  n < 0: floor((n + 2^21 - 1) / 2^22),
// which equals ceil((n - 2^21) / 2^22) = -floor((-n + 2^21) / 2^22).
__device__ __forceinline__ int round_q22(int n)
{
    return (n + (1 << 21) + (n >> 31)) >> 22;
}

__device__ __forceinline__ int clamp_med3(int x, int lo, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

// 24-bit signed multiplies, kept as such (the compiler would otherwise fold
// them into quarter-rate 32-bit multiplies by the precomputed sq * C).
__device__ __forceinline__ int mul_i24(int a, int b)
{
    int r;
    asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ int mad_i24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ uint32_t dot4(uint32_t a, uint32_t b, uint32_t acc)
{
    return __builtin_amdgcn_udot4(a, b, acc, false);
}

// Rule steps 1-3 for one keypoint (uniform across the workgroup), with the
// image it samples.
struct Keypoint {
    bool ok;        // inside the rule's domain (and a real keypoint)
    bool interior;  // every sample lies inside the image: no clamping needed
    int cx, cy;
    int c, s, sq;   // C[b], S[b] (Q14) and the Q8 scale
    int ca, sb;     // sq * C[b], sq * S[b]
    const uint8_t *img;
    int height, width, pitch;
};

// Where keypoints find their image: one image given by value, or a device
// table of images indexed by a per-keypoint image id.
struct ImageSource {
    const uint8_t *img;          // single image
    int height, width, pitch;
    const ImageEntry *table;     // batch: table[image_id[k]]
    const int32_t *image_id;
    int n_images;
};

// Rule steps 1-3 for 64 keypoints at once: lane j takes keypoint
// first + j * stride.  The result stays in registers; each keypoint's
// parameters are then read out with readlane, so the two dependent loads
// (record, table entry) are paid once per 64 keypoints.
struct KeypointBatch {
    int cx, cy;
    int cs;          // C[b] & 0xffff | S[b] << 16
    int sq_flags;    // sq | ok << 16 | interior << 17 | bad image << 18
    int img_lo, img_hi;
    int height, width, pitch;
};

template <bool kTable>
__device__ __forceinline__ KeypointBatch prepare_batch(const float4 *__restrict__ kps, int64_t n,
                                                       int64_t first, int64_t stride, int lane,
                                                       const int2 *__restrict__ rot,
                                                       const ImageSource &src)
{
    KeypointBatch kb;
    const int64_t idx = first + stride * lane;
    const bool real = idx < n;
    const uint8_t *img = src.img;
    int height = src.height, width = src.width, pitch = src.pitch;
    bool image_ok = true;
    if (kTable) {
        const int id = real ? src.image_id[idx] : 0;
        image_ok = id >= 0 && id < src.n_images;
        const ImageEntry e = image_ok ? src.table[id] : ImageEntry{nullptr, 1, 1, 1, 0};
        img = e.img;
        height = e.height;
        width = e.width;
        pitch = e.pitch;
        image_ok = image_ok && img != nullptr && height >= 1 && width >= 1 && pitch >= width &&
                   height < (1 << 23) && pitch < (1 << 23) &&
                   (int64_t)height * pitch <= (int64_t)0x7fffffff;
        if (!image_ok) {
            height = width = pitch = 1;
        }
    }
    const float4 kp = real ? kps[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
    bool ok = real && image_ok && __builtin_isfinite(kp.x) && __builtin_isfinite(kp.y) &&
              __builtin_isfinite(kp.z) && __builtin_isfinite(kp.w);
    ok = ok && fabsf(kp.x) <= 16777216.0f && fabsf(kp.y) <= 16777216.0f && fabsf(kp.z) <= 1.0e6f;
    const double sqd = ok ? rint((double)kp.w * 256.0) : 0.0;
    ok = ok && sqd >= 1.0 && sqd <= 1024.0;
    int cx = 0, cy = 0, bin = 0, sq = 0;
    if (ok) {
        cx = (int)floor((double)kp.x + 0.5);
        cy = (int)floor((double)kp.y + 0.5);
        bin = (int)rint((double)kp.z * (4096.0 / 360.0)) & (kBins - 1);
        sq = (int)sqd;
    }
    const int2 cs = rot[bin];
    // |offset| <= (24 sq (|C| + |S|) + 2^21) / 2^22 < reach.
    const int reach = ((24 * sq * (abs(cs.x) + abs(cs.y))) >> 22) + 1;
    const bool interior = ok && cx - reach >= 0 && cx + reach <= width - 1 && cy - reach >= 0 &&
                          cy + reach <= height - 1;
    kb.cx = cx;
    kb.cy = cy;
    kb.cs = (cs.x & 0xffff) | (cs.y << 16);
    kb.sq_flags = sq | ((int)ok << 16) | ((int)interior << 17) | ((int)(real && !image_ok) << 18);
    kb.img_lo = (int)(uint32_t)reinterpret_cast<uintptr_t>(img);
    kb.img_hi = (int)(uint32_t)(reinterpret_cast<uintptr_t>(img) >> 32);
    kb.height = height;
    kb.width = width;
    kb.pitch = pitch;
    return kb;
}

__device__ __forceinline__ Keypoint batch_get(const KeypointBatch &kb, int j, bool *bad_image)
{
    Keypoint k;
    k.cx = __builtin_amdgcn_readlane(kb.cx, j);
    k.cy = __builtin_amdgcn_readlane(kb.cy, j);
    const int cs = __builtin_amdgcn_readlane(kb.cs, j);
    const int f = __builtin_amdgcn_readlane(kb.sq_flags, j);
    k.c = (int)(short)(cs & 0xffff);
    k.s = cs >> 16;
    k.sq = f & 0xffff;
    k.ok = (f >> 16) & 1;
    k.interior = (f >> 17) & 1;
    *bad_image = (f >> 18) & 1;
    k.ca = k.sq * k.c;     // |ca|, |sb| <= 2^24
    k.sb = k.sq * k.s;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane(kb.img_lo, j);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane(kb.img_hi, j);
    k.img = reinterpret_cast<const uint8_t *>(lo | (hi << 32));
    k.height = __builtin_amdgcn_readlane(kb.height, j);
    k.width = __builtin_amdgcn_readlane(kb.width, j);
    k.pitch = __builtin_amdgcn_readlane(kb.pitch, j);
    return k;
}

// Window coordinates (u, v) = (4 (d % 12) - 24, d / 12 - 24) of this
// thread's window dwords d = tid + 128 m, packed as (u & 0xffff) | (v << 16).
__device__ __forceinline__ void thread_coords(int tid, int (&uv)[kGatherPerThread])
{
#pragma unroll
    for (int m = 0; m < kGatherPerThread; ++m) {
        const int d = min(tid + kThreads * m, kGatherDwords - 1);
        const int i = d / kRowDwords;
        uv[m] = ((4 * (d - kRowDwords * i) - kHalf) & 0xffff) | ((i - kHalf) << 16);
    }
}

// Rule steps 4-5: issue the byte loads of this thread (window dwords
// d = tid + 128 m, bytes b = 0..3, i.e. row d / 12, column 4 (d % 12) + b);
// dword m exists for m < 4, and for m = 4 in the first wavefront only.
// sq (C u - S v) is formed from 24-bit products: |C u - S v| < 2^20 and
// sq <= 2^10, so every product is exact and full rate.
__device__ __forceinline__ void issue_gather(const Keypoint &k, bool has_last,
                                             const int (&uv)[kGatherPerThread],
                                             uint32_t (&g)[kSamples])
{
    const uint8_t *__restrict__ img = k.img;
    const int height = k.height, width = k.width, pitch = k.pitch;
#pragma unroll
    for (int m = 0; m < kGatherPerThread; ++m) {
        if (m == kGatherPerThread - 1 && !has_last) break;
        const int u = (int)(short)(uv[m] & 0xffff);
        const int v = uv[m] >> 16;
        int dx = mul_i24(mad_i24(k.c, u, -mul_i24(k.s, v)), k.sq);   // |dx|, |dy| < 2^30
        int dy = mul_i24(mad_i24(k.s, u, mul_i24(k.c, v)), k.sq);
        if (k.interior) {
            const int base = k.cy * pitch + k.cx;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int off = __mul24(round_q22(dy), pitch) + round_q22(dx) + base;
                g[4 * m + b] = img[(uint32_t)off];
                dx += k.ca;
                dy += k.sb;
            }
        } else {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int X = clamp_med3(k.cx + round_q22(dx), 0, width - 1);
                const int Y = clamp_med3(k.cy + round_q22(dy), 0, height - 1);
                g[4 * m + b] = img[(uint32_t)__mul24(Y, pitch) + (uint32_t)X];
                dx += k.ca;
                dy += k.sb;
            }
        }
    }
}

// Patch rows of one triplet: anchor, companion 1, companion 2, 7 rows each.
struct Rows {
    uint2 a[7], c[7], e[7];
};

__device__ __forceinline__ void load_rows(const uint8_t *winb, uint32_t oa, uint32_t o1, uint32_t o2,
                                          Rows &r)
{
#pragma unroll
    for (int k = 0; k < 2 * kPatchR + 1; ++k) {
        r.a[k] = *reinterpret_cast<const uint2 *>(winb + oa + kRowBytes * k);
        r.c[k] = *reinterpret_cast<const uint2 *>(winb + o1 + kRowBytes * k);
        r.e[k] = *reinterpret_cast<const uint2 *>(winb + o2 + kRowBytes * k);
    }
}

// Eq. 1 on one triplet: [||A - C1||^2 > ||A - C2||^2], via
// ||A - Ck||^2 - sum A^2 = sum Ck^2 - 2 sum A Ck.
__device__ __forceinline__ bool triplet_bit(const Rows &r)
{
    uint32_t ac1 = 0, ac2 = 0, q1 = 0, q2 = 0;
#pragma unroll
    for (int k = 0; k < 2 * kPatchR + 1; ++k) {
        const uint32_t c1 = r.c[k].y & 0x00ffffffu, e1 = r.e[k].y & 0x00ffffffu;
        ac1 = dot4(r.a[k].x, r.c[k].x, ac1);
        ac1 = dot4(r.a[k].y, c1, ac1);
        ac2 = dot4(r.a[k].x, r.e[k].x, ac2);
        ac2 = dot4(r.a[k].y, e1, ac2);
        q1 = dot4(r.c[k].x, r.c[k].x, q1);
        q1 = dot4(c1, c1, q1);
        q2 = dot4(r.e[k].x, r.e[k].x, q2);
        q2 = dot4(e1, e1, q2);
    }
    return (int)(q1 - 2u * ac1) > (int)(q2 - 2u * ac2);
}

template <bool kTable>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void extract_kernel(
    ImageSource src, const float4 *__restrict__ kps, int64_t n_host, const int64_t *__restrict__ n_dev,
    const int2 *__restrict__ rot, const uint2 *__restrict__ trip_off, uint32_t *__restrict__ desc,
    uint32_t *__restrict__ flags)
{
    __shared__ __attribute__((aligned(16))) uint32_t win[kWinLdsBytes / 4];
    const uint8_t *winb = reinterpret_cast<const uint8_t *>(win);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool has_last = wave == 0;          // window dwords 512..575 belong to wavefront 0

    // Wavefront w evaluates rounds 4 w .. 4 w + 3: triplet t = 64 r + lane in round r.
    uint32_t off_a1[kRoundsPerWave], off_2[kRoundsPerWave];
#pragma unroll
    for (int r = 0; r < kRoundsPerWave; ++r) {
        const uint2 o = trip_off[64 * (kRoundsPerWave * wave + r) + lane];
        off_a1[r] = o.x;
        off_2[r] = o.y;
    }

    // Keypoint count: a host value, or (batches) a device value capped by it.
    int64_t n = n_host;
    if (n_dev) n = min(n, *n_dev);
    int64_t p = blockIdx.x;
    if (p >= n) return;
    const int64_t stride = gridDim.x;
    int uv[kGatherPerThread];
    thread_coords(tid, uv);
    uint32_t g[kSamples];
    KeypointBatch batch = prepare_batch<kTable>(kps, n, p, stride, lane, rot, src);
    bool bad_image = false;
    Keypoint cur = batch_get(batch, 0, &bad_image);
    if (cur.ok) issue_gather(cur, has_last, uv, g);

    for (int i = 0; p < n; ++i, p += stride) {
        const bool compute = cur.ok;
        if (!compute) {
            if (tid < kWords) desc[p * kWords + tid] = 0u;
            if (tid == 0) atomicOr(flags, bad_image ? kFlagBadImage : kFlagBadKeypoint);
        } else {
            // Copy 0: the window itself, row pitch 48 bytes.
            uint32_t w[kGatherPerThread];
#pragma unroll
            for (int m = 0; m < kGatherPerThread; ++m)
                w[m] = g[4 * m] | (g[4 * m + 1] << 8) | (g[4 * m + 2] << 16) | (g[4 * m + 3] << 24);
            __syncthreads();   // the previous descriptor's reads of `win` are done
#pragma unroll
            for (int m = 0; m < kGatherPerThread; ++m) {
                if (m == kGatherPerThread - 1 && !has_last) break;
                win[tid + kThreads * m] = w[m];
            }
            __syncthreads();
            // Copies 1..7: copy s holds at (row r, byte x) the window byte
            // (r, x + s).  Bytes past column 47 of a row are only ever read
            // masked; past the last row they are zero.
#pragma unroll
            for (int m = 0; m < kGatherPerThread; ++m) {
                if (m == kGatherPerThread - 1 && !has_last) break;
                const int d = tid + kThreads * m;
                const uint32_t n1 = d + 1 < kGatherDwords ? win[d + 1] : 0u;
                const uint32_t n2 = d + 2 < kGatherDwords ? win[d + 2] : 0u;
                win[1 * (kCopyBytes / 4) + d] = __builtin_amdgcn_alignbyte(n1, w[m], 1);
                win[2 * (kCopyBytes / 4) + d] = __builtin_amdgcn_alignbyte(n1, w[m], 2);
                win[3 * (kCopyBytes / 4) + d] = __builtin_amdgcn_alignbyte(n1, w[m], 3);
                win[4 * (kCopyBytes / 4) + d] = n1;
                win[5 * (kCopyBytes / 4) + d] = __builtin_amdgcn_alignbyte(n2, n1, 1);
                win[6 * (kCopyBytes / 4) + d] = __builtin_amdgcn_alignbyte(n2, n1, 2);
                win[7 * (kCopyBytes / 4) + d] = __builtin_amdgcn_alignbyte(n2, n1, 3);
            }
            __syncthreads();
        }

        // Start the next keypoint's gather; it completes during the arithmetic below.
        const int j = (i + 1) & 63;
        if (j == 0) batch = prepare_batch<kTable>(kps, n, p + stride, stride, lane, rot, src);
        cur = batch_get(batch, j, &bad_image);
        if (cur.ok) issue_gather(cur, has_last, uv, g);
        if (!compute) continue;

        // Eq. 1 for this wavefront's 256 triplets.
        uint32_t out_word = 0;
#pragma unroll
        for (int r = 0; r < kRoundsPerWave; ++r) {
            Rows rows;
            load_rows(winb, off_a1[r] & 0xffffu, off_a1[r] >> 16, off_2[r], rows);
            const uint64_t bits = __ballot(triplet_bit(rows));
            if (lane == 2 * r) out_word = (uint32_t)bits;
            if (lane == 2 * r + 1) out_word = (uint32_t)(bits >> 32);
        }
        if (lane < 2 * kRoundsPerWave)
            desc[p * kWords + 2 * kRoundsPerWave * wave + lane] = out_word;
    }
}

}  // namespace

hipError_t launch_extract(const ExtractArgs &a, hipStream_t stream)
{
    if (a.n <= 0) return hipSuccess;
    int64_t blocks = a.n;
    const int64_t resident = (int64_t)a.num_cus * (kLdsPerCu / kWinLdsBytes);
    if (blocks > resident) blocks = resident;
    ImageSource src{a.img, a.height, a.width, a.pitch, a.table, a.image_id, a.n_images};
    if (a.table)
        hipLaunchKernelGGL(extract_kernel<true>, dim3((unsigned)blocks), dim3(kThreads), 0, stream,
                           src, a.kps, a.n, a.n_dev, a.rot, a.trip_off, a.desc, a.flags);
    else
        hipLaunchKernelGGL(extract_kernel<false>, dim3((unsigned)blocks), dim3(kThreads), 0, stream,
                           src, a.kps, a.n, a.n_dev, a.rot, a.trip_off, a.desc, a.flags);
    return hipGetLastError();
}

}  // namespace latch
