// LATCH descriptor extraction for gfx950.
//
// A workgroup of two wavefronts computes one descriptor at a time
// (grid-stride over keypoints):
//   1. resampling rule steps 1-3 on the keypoint (uniform across the group);
//   2. gather of the 48 x 48 upright window (steps 4-5), one byte load per
//      window position.  Rounding half away from zero is odd, so positions
//      (u, v) and (-u, -v) sample at offsets (ox, oy) and (-ox, -oy), and the
//      unrounded offsets of (u + 1, v) are those of (u, v) plus a per-keypoint
//      constant: a thread takes 5 chains (u, v), (u + 1, v), (-u, -v),
//      (-u - 1, -v) with two roundings per coordinate each (over
//      [-24, 24]^2; the extra row and column are gathered and not read).
//      The chains are taken in an order that keeps each load's samples on
//      nearby image bytes: for the keypoint's angle class (32 bins), sorted
//      by the band of image rows their first member samples at the class's
//      middle angle, then by column (a host-built table).  The loads are
//      issued one keypoint ahead so that their latency overlaps the previous
//      descriptor's arithmetic;
//   3. the samples are written to a plain window in LDS, and a copy pass
//      builds eight byte-shifted copies of it in which every 7-byte patch
//      row is one 8-byte-aligned quadword with a zero last byte;
//   4. Eq. 1 (Sec. 3.1) for 512 triplets: each wavefront takes 4 rounds of 64
//      lanes, one triplet per lane per round, in exact integer arithmetic;
//   5. a 64-bit ballot per round packs the bits.  Triplets sit in (round,
//      lane) slots chosen on the host so that the 32-lane halves of a
//      ds_read_b64 hit few bank conflicts; four table lookups and ballots
//      put the bits back in triplet order, and 8 lanes per wavefront store
//      its 8 words.
//
// Patch distances.  With A, C the 7 x 7 patches of the anchor and one
// companion, ||A - C||^2 = sum A^2 + sum C^2 - 2 sum A C.  sum A^2 is shared by
// both sides of Eq. 1, so bit = [sum C1^2 - 2 sum A C1 > sum C2^2 - 2 sum A C2].
// Each patch row is a quadword of 7 u8 and a zero byte, and each sum is a
// chain of v_dot4_u32_u8.  All sums are < 49 * 255^2 < 2^22, so the int32
// result equals the exact integer one.
//
// The paper's CUDA kernel (Sec. 3.2) spreads one descriptor over 32 warps of
// a 1024-thread block with float32 patches in shared memory; here two 64-lane
// wavefronts share a 19.4 KB byte window (eight per CU, four wavefronts per
// SIMD) and synchronise twice per descriptor.
#include "internal.h"

namespace latch {
namespace {

constexpr int kThreads = kExtractWaves * 64;             // 128: two wavefronts per window
constexpr int kRoundsPerWave = 8 / kExtractWaves;         // 4

// Gather slots per thread: chains 128 m + tid of the gather order, four
// samples each.
constexpr int kGatherSlots = kGatherChains;               // 5
constexpr int kRawCentre = kRawBase + kHalf * kRawStride + kHalf;
static_assert(kGatherHeadChains == 4 && kGatherSlots == 5, "one uint2 and one uint16 of entries");
static_assert(kRawStride >= kWin + 1, "raw rows hold u = -24 .. 24");

// Copy pass: units (row y, quadword q), 240 per window, unit e = 5 y + q.
constexpr int kCopyUnits = kWin * kCopyQwords;
static_assert(kCopyUnits > kThreads && kCopyUnits <= 2 * kThreads, "two copy units per thread");
static_assert(kWinLdsBytes * 8 <= kLdsPerCu, "eight windows per CU");

#include "keypoint.h"

// Raw-window byte of the first member (u, v) of the chain in half `h` of
// packed entry pair `d`; (u + 1, v) is the next byte, (-u, -v) sits at
// 2 kRawCentre minus it and (-u - 1, -v) one byte before that.
__device__ __forceinline__ uint32_t raw_of(uint32_t d, int h)
{
    const int u = __builtin_amdgcn_sbfe((int)d, 16 * h, 8);
    const int v = __builtin_amdgcn_sbfe((int)d, 16 * h + 8, 8);
    return (uint32_t)(kRawCentre + mad_i24(v, kRawStride, u));
}

// Rule steps 4-5 for this thread's 5 chains of keypoint k: its entries of
// the keypoint's angle class (an 8-byte and a 2-byte load; kept in e, two per
// dword, for write_raw) and the byte loads of chain m's members (u, v),
// (u + 1, v), (-u, -v), (-u - 1, -v) into g[4 m .. 4 m + 3].  The unrounded
// offsets of (u, v) are sq (C u - S v) and sq (S u + C v), formed from
// 24-bit products (|C u - S v| < 2^20 and sq <= 2^10, so every product is
// exact and full rate); those of (u + 1, v) add sq C and sq S (|sq C| <= 2^24,
// a scalar product), and rounding half away from zero is odd, so the mirrors
// sample at the negated offsets.  Two roundings per coordinate serve the
// chain's four samples.
__device__ __forceinline__ void issue_gather(const Keypoint &k, const uint16_t *__restrict__ order,
                                             int tid, uint32_t (&e)[(kGatherSlots + 1) / 2],
                                             uint32_t (&g)[4 * kGatherSlots])
{
    const uint16_t *cls = order + (size_t)k.cls * kGatherClassEntries;
    const uint2 t0 = reinterpret_cast<const uint2 *>(cls)[tid];
    e[0] = t0.x, e[1] = t0.y;
    e[2] = cls[kGatherHeadChains * kThreads + tid];
    GlobalByte *img = (GlobalByte *)k.img;
    const int xm = k.width - 1, ym = k.height - 1;
    const int sqc = k.sq * k.c, sqs = k.sq * k.s;
#pragma unroll
    for (int m = 0; m < kGatherSlots; ++m) {
        const int u = __builtin_amdgcn_sbfe((int)e[m >> 1], 16 * (m & 1), 8);
        const int v = __builtin_amdgcn_sbfe((int)e[m >> 1], 16 * (m & 1) + 8, 8);
        const int nx = mul_i24_s(k.sq, mad_i24_s(k.c, u, mul_i24_s(-k.s, v)));
        const int ny = mul_i24_s(k.sq, mad_i24_s(k.s, u, mul_i24_s(k.c, v)));
        const int ox0 = round_q22(nx), oy0 = round_q22(ny);
        const int ox1 = round_q22(nx + sqc), oy1 = round_q22(ny + sqs);
        uint32_t a[4];
        if (k.interior) {
            // Every sample is inside the image, so |offset| * pitch < 2^31 and the
            // 24-bit multiply-adds are exact.
            const int d0 = mad_i24_s(k.pitch, oy0, ox0);
            const int d1 = mad_i24_s(k.pitch, oy1, ox1);
            a[0] = (uint32_t)(k.centre + d0);
            a[1] = (uint32_t)(k.centre + d1);
            a[2] = (uint32_t)(k.centre - d0);
            a[3] = (uint32_t)(k.centre - d1);
        } else {
            a[0] = (uint32_t)mad_i24(clamp_med3(k.cy + oy0, 0, ym), k.pitch, clamp_med3(k.cx + ox0, 0, xm));
            a[1] = (uint32_t)mad_i24(clamp_med3(k.cy + oy1, 0, ym), k.pitch, clamp_med3(k.cx + ox1, 0, xm));
            a[2] = (uint32_t)mad_i24(clamp_med3(k.cy - oy0, 0, ym), k.pitch, clamp_med3(k.cx - ox0, 0, xm));
            a[3] = (uint32_t)mad_i24(clamp_med3(k.cy - oy1, 0, ym), k.pitch, clamp_med3(k.cx - ox1, 0, xm));
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) g[4 * m + i] = img[a[i]];
    }
}

// The gathered samples into the raw window.  Chains overlap at the end of a
// row and the padding slots repeat the centre's chain: such bytes are written
// more than once, always with the same sample.
__device__ __forceinline__ void write_raw(uint8_t *lds, const uint32_t (&e)[(kGatherSlots + 1) / 2],
                                          const uint32_t (&g)[4 * kGatherSlots])
{
#pragma unroll
    for (int m = 0; m < kGatherSlots; ++m) {
        const uint32_t r = raw_of(e[m >> 1], m & 1);
        const uint32_t rm = 2 * kRawCentre - 1 - r;          // (-u - 1, -v)
        lds[r] = (uint8_t)g[4 * m];
        lds[r + 1] = (uint8_t)g[4 * m + 1];
        lds[rm + 1] = (uint8_t)g[4 * m + 2];
        lds[rm] = (uint8_t)g[4 * m + 3];
    }
}

// Copy unit e = 5 y + q: from raw bytes (y, 8 q .. 8 q + 15) build the
// quadword q of row y of every copy (and of the edge copies when q = 4).
__device__ __forceinline__ void copy_unit(uint8_t *lds, int e)
{
    const int y = e / kCopyQwords, q = e - kCopyQwords * y;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(lds + kRawBase + y * kRawStride + 8 * q);
    const uint32_t d0 = src[0], d1 = src[1], d2 = src[2], d3 = src[3];
    constexpr uint32_t m = 0x00ffffffu;
    uint32_t lo[kCopies], hi[kCopies];
    lo[0] = d0;
    lo[1] = __builtin_amdgcn_alignbyte(d1, d0, 1);
    lo[2] = __builtin_amdgcn_alignbyte(d1, d0, 2);
    lo[3] = __builtin_amdgcn_alignbyte(d1, d0, 3);
    lo[4] = d1;
    lo[5] = __builtin_amdgcn_alignbyte(d2, d1, 1);
    lo[6] = __builtin_amdgcn_alignbyte(d2, d1, 2);
    lo[7] = __builtin_amdgcn_alignbyte(d2, d1, 3);
#pragma unroll
    for (int s = 0; s < 4; ++s) hi[s] = lo[s + 4] & m;
    hi[4] = d2 & m;
    hi[5] = __builtin_amdgcn_alignbyte(d3, d2, 1) & m;
    hi[6] = __builtin_amdgcn_alignbyte(d3, d2, 2) & m;
    hi[7] = __builtin_amdgcn_alignbyte(d3, d2, 3) & m;
#pragma unroll
    for (int s = 0; s < kCopies; ++s)
        *reinterpret_cast<uint2 *>(lds + s * kCopyBytes + 8 * e) = make_uint2(lo[s], hi[s]);
    if (q == kCopyQwords - 1) {
        // Columns 40..46 and 41..47.
        *reinterpret_cast<uint2 *>(lds + kEdgeBase + 8 * e) = make_uint2(d2, d3 & m);
        *reinterpret_cast<uint2 *>(lds + kEdgeBase + 8 + 8 * e) =
            make_uint2(__builtin_amdgcn_alignbyte(d3, d2, 1), d3 >> 8);
    }
}

// Patch rows of one triplet: anchor, companion 1, companion 2, 7 rows each.
struct Rows {
    uint2 a[7], c[7], e[7];
};

// The 21 patch rows of a triplet, each one ds_read_b64, then a wait for all
// of them.  Written out because the compiler would pair rows k and k + 1 of
// a patch into a ds_read2_b64, which gfx950 serves 16 lanes and one address
// at a time (at best half the rate of two ds_read_b64, and bank-conflicted
// unless the 16-lane quarters, rather than the 32-lane halves, of a wavefront
// are spread over the banks).  Every address is a host-checked patch offset
// plus a row offset inside the copies.
__device__ __forceinline__ void load_rows(const uint8_t *lds, uint32_t oa, uint32_t o1, uint32_t o2,
                                          Rows &r)
{
    static_assert(kCopyRowBytes == 40, "row offsets below");
    const uint32_t base = (uint32_t)(uintptr_t)lds;
    uint64_t a0, a1, a2, a3, a4, a5, a6, c0, c1, c2, c3, c4, c5, c6, e0, e1, e2, e3, e4, e5, e6;
    asm volatile(
        "ds_read_b64 %0, %21\n"
        "ds_read_b64 %7, %22\n"
        "ds_read_b64 %14, %23\n"
        "ds_read_b64 %1, %21 offset:40\n"
        "ds_read_b64 %8, %22 offset:40\n"
        "ds_read_b64 %15, %23 offset:40\n"
        "ds_read_b64 %2, %21 offset:80\n"
        "ds_read_b64 %9, %22 offset:80\n"
        "ds_read_b64 %16, %23 offset:80\n"
        "ds_read_b64 %3, %21 offset:120\n"
        "ds_read_b64 %10, %22 offset:120\n"
        "ds_read_b64 %17, %23 offset:120\n"
        "ds_read_b64 %4, %21 offset:160\n"
        "ds_read_b64 %11, %22 offset:160\n"
        "ds_read_b64 %18, %23 offset:160\n"
        "ds_read_b64 %5, %21 offset:200\n"
        "ds_read_b64 %12, %22 offset:200\n"
        "ds_read_b64 %19, %23 offset:200\n"
        "ds_read_b64 %6, %21 offset:240\n"
        "ds_read_b64 %13, %22 offset:240\n"
        "ds_read_b64 %20, %23 offset:240\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(a0), "=&v"(a1), "=&v"(a2), "=&v"(a3), "=&v"(a4), "=&v"(a5), "=&v"(a6),
          "=&v"(c0), "=&v"(c1), "=&v"(c2), "=&v"(c3), "=&v"(c4), "=&v"(c5), "=&v"(c6),
          "=&v"(e0), "=&v"(e1), "=&v"(e2), "=&v"(e3), "=&v"(e4), "=&v"(e5), "=&v"(e6)
        : "v"(base + oa), "v"(base + o1), "v"(base + o2)
        : "memory");
    const uint64_t a[7] = {a0, a1, a2, a3, a4, a5, a6};
    const uint64_t c[7] = {c0, c1, c2, c3, c4, c5, c6};
    const uint64_t e[7] = {e0, e1, e2, e3, e4, e5, e6};
#pragma unroll
    for (int k = 0; k < 2 * kPatchR + 1; ++k) {
        r.a[k] = make_uint2((uint32_t)a[k], (uint32_t)(a[k] >> 32));
        r.c[k] = make_uint2((uint32_t)c[k], (uint32_t)(c[k] >> 32));
        r.e[k] = make_uint2((uint32_t)e[k], (uint32_t)(e[k] >> 32));
    }
}

// Eq. 1 on one triplet: [||A - C1||^2 > ||A - C2||^2], via
// ||A - Ck||^2 - sum A^2 = sum Ck^2 - 2 sum A Ck.  The zero last byte of
// every row quadword keeps the sums to the 7 x 7 patch.
__device__ __forceinline__ bool triplet_bit(const Rows &r)
{
    uint32_t ac1 = 0, ac2 = 0, q1 = 0, q2 = 0;
#pragma unroll
    for (int k = 0; k < 2 * kPatchR + 1; ++k) {
        ac1 = dot4(r.a[k].x, r.c[k].x, ac1);
        ac1 = dot4(r.a[k].y, r.c[k].y, ac1);
        ac2 = dot4(r.a[k].x, r.e[k].x, ac2);
        ac2 = dot4(r.a[k].y, r.e[k].y, ac2);
        q1 = dot4(r.c[k].x, r.c[k].x, q1);
        q1 = dot4(r.c[k].y, r.c[k].y, q1);
        q2 = dot4(r.e[k].x, r.e[k].x, q2);
        q2 = dot4(r.e[k].y, r.e[k].y, q2);
    }
    return (int)(q1 - 2u * ac1) > (int)(q2 - 2u * ac2);
}

template <bool kTable>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void extract_kernel(
    ImageSource src, const float4 *__restrict__ kps, int64_t n_host, const int64_t *__restrict__ n_dev,
    const int2 *__restrict__ rot, const uint2 *__restrict__ trip_off,
    const uint32_t *__restrict__ unperm, const uint16_t *__restrict__ gather_order,
    uint32_t *__restrict__ desc, uint32_t *__restrict__ flags)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[kWinLdsBytes];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // Wavefront w evaluates triplets 256 w .. 256 w + 255 in 4 rounds; slot
    // 64 r + lane holds the triplet the bank-aware assignment put there, and
    // `slots` names, for output bits 256 w + 64 k + lane, k = 0..3, the slots
    // that computed them.
    // Offsets: anchor | companion 1 << 16 per round, and the companion-2
    // offsets of rounds 2 q and 2 q + 1 packed in off_2[q] (all < 2^16).
    uint32_t off_a1[kRoundsPerWave], off_2[kRoundsPerWave / 2];
#pragma unroll
    for (int r = 0; r < kRoundsPerWave; ++r) {
        const uint2 o = trip_off[64 * (kRoundsPerWave * wave + r) + lane];
        off_a1[r] = o.x;
        if (r & 1)
            off_2[r >> 1] |= o.y << 16;
        else
            off_2[r >> 1] = o.y;
    }
    uint32_t *ballots = reinterpret_cast<uint32_t *>(lds + kBallotBase) + 8 * wave;

    // Keypoint count: a host value, or (batches) a device value capped by it.
    int64_t n_all = n_host;
    if (n_dev) n_all = min(n_all, *n_dev);
    const KeypointRange range = xcd_range(n_all);
    const int64_t n = range.end;
    int64_t p = range.first;
    if (p >= n) return;
    // This lane's output bits 256 w + 64 k + lane come from slots
    // (slots >> 8 k) & 0xff of its wavefront (constant over keypoints).
    const uint32_t slots = unperm[64 * wave + lane];
    const int64_t stride = range.stride;
    uint32_t e[(kGatherSlots + 1) / 2], g[4 * kGatherSlots];
    KeypointBatch batch = prepare_batch<kTable, kHalf>(kps, n, p, stride, lane, rot, src);
    bool bad_image = false;
    Keypoint cur = batch_get<kTable>(batch, 0, src, &bad_image);
    if (cur.ok) issue_gather(cur, gather_order, tid, e, g);

    for (int i = 0; p < n; ++i, p += stride) {
        const bool compute = cur.ok;
        // Descriptor row of this position's keypoint (the position itself
        // unless a batch order permutes the keypoints).
        const int64_t q = kTable && src.order ? (int64_t)cur.key : p;
        if (!compute) {
            if (tid < kWords) uniform_words(desc + q * kWords)[(uint32_t)tid] = 0u;
            if (tid == 0) atomicOr(flags, bad_image ? kFlagBadImage : kFlagBadKeypoint);
        } else {
            // The raw window was last read by the previous descriptor's copy
            // pass, which ended before that descriptor's second barrier.
            write_raw(lds, e, g);
            __syncthreads();   // raw window complete; the previous triplet reads are done
            copy_unit(lds, tid);
            if (tid < kCopyUnits - kThreads) copy_unit(lds, tid + kThreads);
            __syncthreads();   // copies complete
        }

        // Start the next keypoint's gather; it completes during the arithmetic below.
        const int j = (i + 1) & 63;
        if (j == 0) batch = prepare_batch<kTable, kHalf>(kps, n, p + stride, stride, lane, rot, src);
        cur = batch_get<kTable>(batch, j, src, &bad_image);
        if (cur.ok) issue_gather(cur, gather_order, tid, e, g);
        if (!compute) continue;

        // Eq. 1 for this wavefront's 256 triplets, in slot order.
        uint32_t slot_word = 0;
#pragma unroll
        for (int r = 0; r < kRoundsPerWave; ++r) {
            Rows rows;
            load_rows(lds, off_a1[r] & 0xffffu, off_a1[r] >> 16, (off_2[r >> 1] >> (16 * (r & 1))) & 0xffffu,
                      rows);
            const uint64_t bits = __ballot(triplet_bit(rows));
            if (lane == 2 * r) slot_word = (uint32_t)bits;
            if (lane == 2 * r + 1) slot_word = (uint32_t)(bits >> 32);
        }
        // Back to triplet order through this wavefront's 8 ballot words in
        // LDS (written and read by the same wavefront, so in order).
        if (lane < 2 * kRoundsPerWave) ballots[lane] = slot_word;
        uint32_t out_word = 0;
#pragma unroll
        for (int k = 0; k < kRoundsPerWave; ++k) {
            const uint32_t s = (slots >> (8 * k)) & 0xffu;
            const uint64_t bits = __ballot((ballots[s >> 5] >> (s & 31u)) & 1u);
            if (lane == 2 * k) out_word = (uint32_t)bits;
            if (lane == 2 * k + 1) out_word = (uint32_t)(bits >> 32);
        }
        if (lane < 2 * kRoundsPerWave)
            uniform_words(desc + (q * kWords + 2 * kRoundsPerWave * wave))[(uint32_t)lane] = out_word;
    }
}

}  // namespace

hipError_t launch_extract(const ExtractArgs &a, hipStream_t stream)
{
    if (a.n <= 0) return hipSuccess;
    int64_t blocks = a.n;
    const int64_t resident = (int64_t)a.num_cus * (kLdsPerCu / kWinLdsBytes);
    if (blocks > resident) blocks = resident;
    ImageSource src{a.img, a.height, a.width, a.pitch, a.table, a.image_id, a.n_images, a.order};
    if (a.table)
        hipLaunchKernelGGL(extract_kernel<true>, dim3((unsigned)blocks), dim3(kThreads), 0, stream,
                           src, a.kps, a.n, a.n_dev, a.rot, a.trip_off, a.unperm, a.gather, a.desc,
                           a.flags);
    else
        hipLaunchKernelGGL(extract_kernel<false>, dim3((unsigned)blocks), dim3(kThreads), 0, stream,
                           src, a.kps, a.n, a.n_dev, a.rot, a.trip_off, a.unperm, a.gather, a.desc,
                           a.flags);
    return hipGetLastError();
}

}  // namespace latch
