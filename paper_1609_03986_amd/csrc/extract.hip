// LATCH descriptor extraction for gfx950.
//
// One wavefront computes one descriptor at a time (grid-stride over keypoints):
//   1. resampling rule steps 1-3 on the keypoint (uniform across the wave);
//   2. gather of the 48 x 48 upright window (steps 4-5) from the image into
//      LDS, 36 samples per lane, packed four to a dword;
//   3. three byte-shifted copies of the window so that any 7-byte patch row
//      is the head of two dword-aligned LDS words;
//   4. Eq. 1 (Sec. 3.1) for 512 triplets, 8 rounds of 64 lanes, one triplet
//      per lane per round, in exact integer arithmetic;
//   5. a 64-bit ballot per round packs the bits; lanes 0..15 store the
//      16 words.
//
// Patch distances.  With A, C the 7 x 7 patches of the anchor and one
// companion, ||A - C||^2 = sum A^2 + sum C^2 - 2 sum A C.  sum A^2 is shared by
// both sides of Eq. 1, so bit = [sum C1^2 - 2 sum A C1 > sum C2^2 - 2 sum A C2].
// Each 7-pixel row is two dwords of packed u8 (the 8th byte masked to zero in
// the companion operands) and each sum is a chain of v_dot4_u32_u8.  All sums
// are < 49 * 255^2 < 2^22, so the int32 result equals the exact integer one.
//
// The paper's CUDA kernel (Sec. 3.2) spreads one descriptor over 32 warps of
// a 1024-thread block with float32 patches in shared memory; here a single
// 64-lane wavefront owns a descriptor, needs no workgroup barrier, and works
// on bytes.
#include "internal.h"

namespace latch {
namespace {

constexpr int kThreads = kExtractWaves * 64;
constexpr int kGatherDwords = kWin * kWin / 4;          // 576
constexpr int kRowDwords = kRowBytes / 4;               // 12
constexpr int kGatherPerLane = kGatherDwords / 64;      // 9
static_assert(kGatherDwords % 64 == 0, "gather must tile the wavefront");

// LDS ordering among the lanes of one wavefront: LDS instructions of a
// wavefront execute in order, so only the compiler needs to be fenced.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// n / 2^22 rounded half away from zero, for |n| < 2^31 - 2^21.
// n >= 0: floor((n + 2^21) / 2^22).  n < 0: floor((n + 2^21 - 1) / 2^22),
// which equals ceil((n - 2^21) / 2^22) = -floor((-n + 2^21) / 2^22).
__device__ __forceinline__ int round_q22(int n)
{
    return (n + (1 << 21) + (n >> 31)) >> 22;
}

__device__ __forceinline__ uint32_t dot4(uint32_t a, uint32_t b, uint32_t acc)
{
    return __builtin_amdgcn_udot4(a, b, acc, false);
}

__global__ __launch_bounds__(kThreads) void extract_kernel(
    const uint8_t *__restrict__ img, int height, int width, int pitch,
    const float4 *__restrict__ kps, int64_t n, const int2 *__restrict__ rot,
    const uint2 *__restrict__ trip_off, uint32_t *__restrict__ desc,
    uint32_t *__restrict__ flags)
{
    __shared__ uint32_t lds[kExtractWaves][kWaveLdsBytes / 4];

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t *win = lds[wave];
    const uint8_t *winb = reinterpret_cast<const uint8_t *>(win);

    // Triplet t = 64 r + lane is evaluated by this lane in round r.
    uint32_t off_a1[8], off_2[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const uint2 o = trip_off[64 * r + lane];
        off_a1[r] = o.x;
        off_2[r] = o.y;
    }

    const int64_t stride = (int64_t)gridDim.x * kExtractWaves;
    for (int64_t p = (int64_t)blockIdx.x * kExtractWaves + wave; p < n; p += stride) {
        const float4 kp = kps[p];

        // Rule steps 1-3 and the domain check.
        bool ok = __builtin_isfinite(kp.x) && __builtin_isfinite(kp.y) &&
                  __builtin_isfinite(kp.z) && __builtin_isfinite(kp.w);
        ok = ok && fabsf(kp.x) <= 16777216.0f && fabsf(kp.y) <= 16777216.0f &&
             fabsf(kp.z) <= 1.0e6f;
        const double sqd = rint((double)kp.w * 256.0);
        ok = ok && sqd >= 1.0 && sqd <= 1024.0;
        if (!ok) {
            if (lane < kWords) desc[p * kWords + lane] = 0u;
            if (lane == 0) atomicOr(flags, 1u);
            continue;
        }
        const int cx = (int)floor((double)kp.x + 0.5);
        const int cy = (int)floor((double)kp.y + 0.5);
        const int bin = (int)rint((double)kp.z * (4096.0 / 360.0)) & (kBins - 1);
        const int sq = (int)sqd;
        const int2 cs = rot[bin];
        const int ca = sq * cs.x;      // |ca|, |sb| <= 2^24
        const int sb = sq * cs.y;

        wave_lds_sync();   // the previous descriptor's reads of `win` are done

        // Rule steps 4-5: lane gathers dwords d = lane + 64 m, i.e. window row
        // d / 12, columns 4 (d % 12) .. 4 (d % 12) + 3.
#pragma unroll
        for (int m = 0; m < kGatherPerLane; ++m) {
            const int d = lane + 64 * m;
            const int i = d / kRowDwords;
            const int w = d - kRowDwords * i;
            const int v = i - kHalf;
            const int u = 4 * w - kHalf;
            int dx = ca * u - sb * v;        // |dx|, |dy| < 2^30
            int dy = sb * u + ca * v;
            uint32_t word = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int X = min(max(cx + round_q22(dx), 0), width - 1);
                const int Y = min(max(cy + round_q22(dy), 0), height - 1);
                word |= (uint32_t)img[(uint32_t)(Y * pitch + X)] << (8 * b);
                dx += ca;
                dy += sb;
            }
            win[d] = word;
        }
        wave_lds_sync();

        // Byte-shifted copies 1..3 (the tail of each row beyond column 47 is
        // zero; it only ever lands in masked bytes).
#pragma unroll
        for (int m = 0; m < kGatherPerLane; ++m) {
            const int d = lane + 64 * m;
            const int w = d % kRowDwords;
            const uint32_t cur = win[d];
            const uint32_t nxt = (w != kRowDwords - 1) ? win[d + 1] : 0u;
            win[1 * (kCopyBytes / 4) + d] = __builtin_amdgcn_alignbyte(nxt, cur, 1);
            win[2 * (kCopyBytes / 4) + d] = __builtin_amdgcn_alignbyte(nxt, cur, 2);
            win[3 * (kCopyBytes / 4) + d] = __builtin_amdgcn_alignbyte(nxt, cur, 3);
        }
        wave_lds_sync();

        // Eq. 1 for the 512 triplets.
        uint32_t out_word = 0;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const uint32_t oa = off_a1[r] & 0xffffu;
            const uint32_t o1 = off_a1[r] >> 16;
            const uint32_t o2 = off_2[r];
            uint32_t ac1 = 0, ac2 = 0, q1 = 0, q2 = 0;
#pragma unroll
            for (int k = 0; k < 2 * kPatchR + 1; ++k) {
                const uint32_t *pa = reinterpret_cast<const uint32_t *>(winb + oa + kRowBytes * k);
                const uint32_t *p1 = reinterpret_cast<const uint32_t *>(winb + o1 + kRowBytes * k);
                const uint32_t *p2 = reinterpret_cast<const uint32_t *>(winb + o2 + kRowBytes * k);
                const uint32_t a0 = pa[0], a1 = pa[1];
                const uint32_t c0 = p1[0], c1 = p1[1] & 0x00ffffffu;
                const uint32_t e0 = p2[0], e1 = p2[1] & 0x00ffffffu;
                ac1 = dot4(a0, c0, ac1);
                ac1 = dot4(a1, c1, ac1);
                ac2 = dot4(a0, e0, ac2);
                ac2 = dot4(a1, e1, ac2);
                q1 = dot4(c0, c0, q1);
                q1 = dot4(c1, c1, q1);
                q2 = dot4(e0, e0, q2);
                q2 = dot4(e1, e1, q2);
            }
            // ||A - Ck||^2 - sum A^2 = qk - 2 ack
            const int s1 = (int)(q1 - 2u * ac1);
            const int s2 = (int)(q2 - 2u * ac2);
            const uint64_t bits = __ballot(s1 > s2);
            if (lane == 2 * r) out_word = (uint32_t)bits;
            if (lane == 2 * r + 1) out_word = (uint32_t)(bits >> 32);
        }
        if (lane < kWords) desc[p * kWords + lane] = out_word;
    }
}

}  // namespace

hipError_t launch_extract(const ExtractArgs &a, hipStream_t stream)
{
    if (a.n <= 0) return hipSuccess;
    const int64_t waves = a.n;
    int64_t blocks = (waves + kExtractWaves - 1) / kExtractWaves;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(extract_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, stream, a.img,
                       a.height, a.width, a.pitch, a.kps, a.n, a.rot, a.trip_off, a.desc,
                       a.flags);
    return hipGetLastError();
}

}  // namespace latch
