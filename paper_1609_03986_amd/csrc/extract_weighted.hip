// LATCH extraction with the paper's CLATCH geometry and per-pixel patch
// weights (Sec. 3.2: 64 x 64 windows, 8 x 8 patches, an integer weight per
// patch pixel; zero weights on one row and one column give the 7 x 7 patch).
//
// For each triplet, S_j = sum w[a][b] (A[a][b] - P_j[a][b])^2 over the patch
// pixels and bit = [S_1 > S_2].  Per pixel,
//     w (A - P_1)^2 - w (A - P_2)^2 = w d s,  d = P_1 - P_2,  s = P_1 + P_2 - 2 A,
// so bit = [sum w d s > 0].  Weights lie in [0, 128], d in [-255, 255] and s in
// [-510, 510], so d, s and w d fit signed 16-bit lanes: per patch row of 8
// pixels (4 pairs) the kernel forms d, P_1 + P_2 and s with packed 16-bit
// subtract, add and multiply-add, w d with a packed 16-bit multiply, and
// accumulates (w d) s with v_dot2_i32_i16.  |sum| <= 64 * 128 * 255 * 510
// < 2^31: exact.  7 x 7 patches run as 8 x 8 ones whose last row and column
// weigh 0.
//
// A workgroup of four wavefronts computes one descriptor at a time
// (grid-stride over keypoints):
//   1. resampling rule steps 1-3 on the keypoint (uniform);
//   2. the W x W window gathered with the rule (W * W / 256 samples per
//      thread, issued one keypoint ahead), written to LDS as 16-bit pixels
//      in four copies shifted by 0..3 columns, so that the 8 pixels of any
//      patch row start on a quadword of one copy (two ds_read_b64);
//   3. two triplets per thread: wavefront w evaluates triplets 64 w + l and
//      256 + 64 w + l (l = 0..63) in two rounds, in (round, lane) slots the
//      host chose so that the 32-lane halves of a ds_read_b64 hit few bank
//      conflicts; a ballot per round gives 64 bits, and four ballot words per
//      wavefront in LDS put them back in triplet order.
#include "internal.h"

namespace latch {
namespace {

#include "keypoint.h"

typedef short short2v __attribute__((ext_vector_type(2)));

constexpr int kWThreads = 256;

template <int kW>
struct WGeom {
    static constexpr int kHalfW = kW / 2;
    static constexpr int kRowBytes = 2 * (kW + 8);               // 16-bit pixels, 8 spare
    static constexpr int kCopyBytes = (kW + 1) * kRowBytes;      // one spare (zero) row
    static constexpr int kLds = 4 * kCopyBytes;
    static constexpr int kSamples = kW * kW / kWThreads;         // per thread
    static_assert(kW * kW % kWThreads == 0, "whole samples per thread");
};

// Rule steps 4-5 for the sample of unrounded offsets (nx, ny) = (sq (C u - S v),
// sq (S u + C v)) of a window position (u, v).
__device__ __forceinline__ uint32_t sample_at(const Keypoint &k, GlobalByte *img, int nx, int ny)
{
    const int ox = round_q22(nx), oy = round_q22(ny);
    if (k.interior) return img[(uint32_t)(k.centre + mad_i24_s(k.pitch, oy, ox))];
    const int x = clamp_med3(k.cx + ox, 0, k.width - 1);
    const int y = clamp_med3(k.cy + oy, 0, k.height - 1);
    return img[(uint32_t)mad_i24(y, k.pitch, x)];
}

// This thread's samples: window positions q = tid + 256 m (u = q mod W - W/2,
// v = q div W - W/2).  |C u - S v| < 2^20 and sq <= 2^10, so the 24-bit
// products are exact.  When W divides 256 every sample of a thread has the
// same u and v grows by 256 / W per sample, so the unrounded offsets step by
// the keypoint's -(256 / W) sq S and (256 / W) sq C (|step| <= 2^26, exact).
template <int kW>
__device__ __forceinline__ void issue_samples(const Keypoint &k, int tid,
                                              uint32_t (&g)[WGeom<kW>::kSamples])
{
    using G = WGeom<kW>;
    GlobalByte *img = (GlobalByte *)k.img;
    if constexpr (kWThreads % kW == 0) {
        constexpr int kDv = kWThreads / kW;
        const int u = tid % kW - G::kHalfW, v = tid / kW - G::kHalfW;
        int nx = mul_i24_s(k.sq, mad_i24_s(k.c, u, mul_i24_s(-k.s, v)));
        int ny = mul_i24_s(k.sq, mad_i24_s(k.s, u, mul_i24_s(k.c, v)));
        const int dx = -kDv * k.sq * k.s, dy = kDv * k.sq * k.c;
#pragma unroll
        for (int m = 0; m < G::kSamples; ++m, nx += dx, ny += dy) g[m] = sample_at(k, img, nx, ny);
    } else {
#pragma unroll
        for (int m = 0; m < G::kSamples; ++m) {
            const int q = tid + kWThreads * m;
            const int u = q % kW - G::kHalfW, v = q / kW - G::kHalfW;
            g[m] = sample_at(k, img, mul_i24_s(k.sq, mad_i24_s(k.c, u, mul_i24_s(-k.s, v))),
                             mul_i24_s(k.sq, mad_i24_s(k.s, u, mul_i24_s(k.c, v))));
        }
    }
}

// Pixel (i, j) goes to element j - s of row i of copy s, s = 0..3.  For
// j < s that is element W + 8 + j - s of the row before (or, for i = 0, of
// the previous copy's spare row): one of the last three spare elements of a
// row, which no patch read reaches (a patch row reads elements up to W), so
// the writes need no condition.
template <int kW>
__device__ __forceinline__ void write_window(uint8_t *lds, int tid, const uint32_t (&g)[WGeom<kW>::kSamples])
{
    using G = WGeom<kW>;
#pragma unroll
    for (int m = 0; m < G::kSamples; ++m) {
        const int q = tid + kWThreads * m;
        const int i = q / kW, j = q % kW;
        uint8_t *row = lds + i * G::kRowBytes + 2 * j;
        const uint16_t v = (uint16_t)g[m];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            *reinterpret_cast<uint16_t *>(row + s * G::kCopyBytes - 2 * s) = v;
    }
}

// Rows r and r + 1 of the three patches (two quadwords each) as twelve single
// ds_read_b64, then a wait for all of them: v[6 k + 2 p + h] is quadword h
// of row r + k of patch p (anchor, companion 1, companion 2).  Written out
// because the compiler would pair the quadwords into ds_read2_b64, which
// gfx950 serves 16 lanes and one address at a time (at best half the rate of
// two ds_read_b64).  Every address is a host-checked patch offset plus a row
// offset inside the copies.
template <int kOff, int kRowBytes>
__device__ __forceinline__ void load_row_pair(uint32_t pa, uint32_t pc, uint32_t pe, uint64_t (&v)[12])
{
    asm volatile(
        "ds_read_b64 %0, %12 offset:%15\n"
        "ds_read_b64 %1, %12 offset:%16\n"
        "ds_read_b64 %2, %13 offset:%15\n"
        "ds_read_b64 %3, %13 offset:%16\n"
        "ds_read_b64 %4, %14 offset:%15\n"
        "ds_read_b64 %5, %14 offset:%16\n"
        "ds_read_b64 %6, %12 offset:%17\n"
        "ds_read_b64 %7, %12 offset:%18\n"
        "ds_read_b64 %8, %13 offset:%17\n"
        "ds_read_b64 %9, %13 offset:%18\n"
        "ds_read_b64 %10, %14 offset:%17\n"
        "ds_read_b64 %11, %14 offset:%18\n"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(v[0]), "=&v"(v[1]), "=&v"(v[2]), "=&v"(v[3]), "=&v"(v[4]), "=&v"(v[5]),
          "=&v"(v[6]), "=&v"(v[7]), "=&v"(v[8]), "=&v"(v[9]), "=&v"(v[10]), "=&v"(v[11])
        : "v"(pa), "v"(pc), "v"(pe), "i"(kOff), "i"(kOff + 8), "i"(kOff + kRowBytes),
          "i"(kOff + kRowBytes + 8)
        : "memory");
}

// c + a b per 16-bit half (v_pk_mad_i16; the compiler splits the multiply-add
// of 16-bit vectors into a shift, an add and a subtract).  b is uniform.
__device__ __forceinline__ short2v pk_mad_i16(short2v a, uint32_t b, short2v c)
{
    uint32_t r;
    asm("v_pk_mad_i16 %0, %1, %2, %3"
        : "=v"(r)
        : "v"(__builtin_bit_cast(uint32_t, a)), "s"(b), "v"(__builtin_bit_cast(uint32_t, c)));
    return __builtin_bit_cast(short2v, r);
}

// One patch row (4 pixel pairs) of sum w d s.
__device__ __forceinline__ void weighted_row(const uint32_t *wrow, uint64_t a0, uint64_t a1, uint64_t c0,
                                             uint64_t c1, uint64_t e0, uint64_t e1, int &acc)
{
    const uint32_t av[4] = {(uint32_t)a0, (uint32_t)(a0 >> 32), (uint32_t)a1, (uint32_t)(a1 >> 32)};
    const uint32_t cv[4] = {(uint32_t)c0, (uint32_t)(c0 >> 32), (uint32_t)c1, (uint32_t)(c1 >> 32)};
    const uint32_t ev[4] = {(uint32_t)e0, (uint32_t)(e0 >> 32), (uint32_t)e1, (uint32_t)(e1 >> 32)};
    constexpr uint32_t kMinus2 = 0xfffefffeu;       // -2 in both 16-bit halves
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const short2v wv = __builtin_bit_cast(short2v, wrow[i]);
        const short2v A = __builtin_bit_cast(short2v, av[i]);
        const short2v P1 = __builtin_bit_cast(short2v, cv[i]);
        const short2v P2 = __builtin_bit_cast(short2v, ev[i]);
        const short2v d = P1 - P2;
        const short2v s = pk_mad_i16(A, kMinus2, P1 + P2);
        acc = __builtin_amdgcn_sdot2(wv * d, s, acc, false);
    }
}

template <int kR, int kRowBytes>
__device__ __forceinline__ void weighted_rows(uint32_t base, uint32_t oa, uint32_t o1, uint32_t o2,
                                              const WeightRows &w, int &acc)
{
    uint64_t v[12];
    load_row_pair<kR * kRowBytes, kRowBytes>(base + oa, base + o1, base + o2, v);
    weighted_row(w.pair + 4 * kR, v[0], v[1], v[2], v[3], v[4], v[5], acc);
    weighted_row(w.pair + 4 * (kR + 1), v[6], v[7], v[8], v[9], v[10], v[11], acc);
}

// S_j of one triplet: patch rows at byte offsets off + r kRowBytes.
template <int kW>
__device__ __forceinline__ bool weighted_bit(const uint8_t *lds, uint32_t oa, uint32_t o1, uint32_t o2,
                                             const WeightRows &w)
{
    constexpr int kRB = WGeom<kW>::kRowBytes;
    const uint32_t base = (uint32_t)(uintptr_t)lds;
    int acc = 0;                   // S_1 - S_2
    weighted_rows<0, kRB>(base, oa, o1, o2, w, acc);
    weighted_rows<2, kRB>(base, oa, o1, o2, w, acc);
    weighted_rows<4, kRB>(base, oa, o1, o2, w, acc);
    weighted_rows<6, kRB>(base, oa, o1, o2, w, acc);
    return acc > 0;
}

template <bool kTable, int kW>
__global__ __launch_bounds__(kWThreads) void extract_weighted_kernel(
    ImageSource src, const float4 *__restrict__ kps, int64_t n_host, const int64_t *__restrict__ n_dev,
    const int2 *__restrict__ rot, const uint2 *__restrict__ trip_off,
    const uint32_t *__restrict__ unperm, WeightRows w, uint32_t *__restrict__ desc,
    uint32_t *__restrict__ flags)
{
    using G = WGeom<kW>;
    __shared__ __attribute__((aligned(16))) uint8_t lds[G::kLds];
    __shared__ uint32_t ballot_words[4 * (kWThreads / 64)];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // The spare columns and row that patch reads reach stay zero (they meet
    // zero weights only).
    for (int i = tid; i < G::kLds / 4; i += kWThreads) reinterpret_cast<uint32_t *>(lds)[i] = 0u;

    // This lane's slots in rounds 0 and 1, and the slots of its output bits
    // (triplets 64 wave + lane and 256 + 64 wave + lane).
    const uint2 t0 = trip_off[128 * wave + lane], t1 = trip_off[128 * wave + 64 + lane];
    const uint32_t un = unperm[64 * wave + lane];
    uint32_t *bw = ballot_words + 4 * wave;

    int64_t n_all = n_host;
    if (n_dev) n_all = min(n_all, *n_dev);
    const KeypointRange range = xcd_range(n_all);
    const int64_t n = range.end;
    int64_t p = range.first;
    if (p >= n) return;
    const int64_t stride = range.stride;
    uint32_t g[G::kSamples];
    KeypointBatch batch = prepare_batch<kTable, G::kHalfW>(kps, n, p, stride, lane, rot, src);
    bool bad_image = false;
    Keypoint cur = batch_get<kTable>(batch, 0, src, &bad_image);
    if (cur.ok) issue_samples<kW>(cur, tid, g);

    for (int i = 0; p < n; ++i, p += stride) {
        const bool compute = cur.ok;
        __syncthreads();   // the previous descriptor's patch reads are done
        if (!compute) {
            if (tid < kWords) uniform_words(desc + p * kWords)[(uint32_t)tid] = 0u;
            if (tid == 0) atomicOr(flags, bad_image ? kFlagBadImage : kFlagBadKeypoint);
        } else {
            write_window<kW>(lds, tid, g);
        }
        __syncthreads();   // window complete

        // Next keypoint's gather, in flight during the arithmetic below.
        const int j = (i + 1) & 63;
        if (j == 0) batch = prepare_batch<kTable, G::kHalfW>(kps, n, p + stride, stride, lane, rot, src);
        cur = batch_get<kTable>(batch, j, src, &bad_image);
        if (cur.ok) issue_samples<kW>(cur, tid, g);
        if (!compute) continue;

        const uint64_t b0 = __ballot(weighted_bit<kW>(lds, t0.x & 0xffffu, t0.x >> 16, t0.y, w));
        const uint64_t b1 = __ballot(weighted_bit<kW>(lds, t1.x & 0xffffu, t1.x >> 16, t1.y, w));
        // Slot order -> triplet order through this wavefront's ballot words
        // (written and read by the same wavefront, so in order).
        if (lane < 4) {
            const uint64_t b = lane < 2 ? b0 : b1;
            bw[lane] = (uint32_t)(lane & 1 ? b >> 32 : b);
        }
        const uint32_t s0 = un & 0xffu, s1 = (un >> 8) & 0xffu;
        const uint64_t o0 = __ballot((bw[s0 >> 5] >> (s0 & 31u)) & 1u);
        const uint64_t o1 = __ballot((bw[s1 >> 5] >> (s1 & 31u)) & 1u);
        if (lane < 4) {
            const uint64_t o = lane < 2 ? o0 : o1;
            const uint32_t word = (uint32_t)(lane & 1 ? o >> 32 : o);
            desc[p * kWords + 8 * (lane >> 1) + 2 * wave + (lane & 1)] = word;
        }
    }
}

template <int kW>
hipError_t launch_weighted_w(const ExtractArgs &a, hipStream_t stream)
{
    int64_t blocks = a.n;
    const int64_t resident = (int64_t)a.num_cus * (kLdsPerCu / WGeom<kW>::kLds);
    if (blocks > resident) blocks = resident;
    ImageSource src{a.img, a.height, a.width, a.pitch, a.table, a.image_id, a.n_images, nullptr};
    if (a.table)
        hipLaunchKernelGGL((extract_weighted_kernel<true, kW>), dim3((unsigned)blocks), dim3(kWThreads),
                           0, stream, src, a.kps, a.n, a.n_dev, a.rot, a.wtrip_off, a.wunperm, a.weights,
                           a.desc, a.flags);
    else
        hipLaunchKernelGGL((extract_weighted_kernel<false, kW>), dim3((unsigned)blocks),
                           dim3(kWThreads), 0, stream, src, a.kps, a.n, a.n_dev, a.rot, a.wtrip_off,
                           a.wunperm, a.weights, a.desc, a.flags);
    return hipGetLastError();
}

}  // namespace

uint32_t weighted_patch_offset(int window, int top, int left)
{
    const int s = left & 3, e = left - s;
    if (window == 64)
        return (uint32_t)(s * WGeom<64>::kCopyBytes + top * WGeom<64>::kRowBytes + 2 * e);
    return (uint32_t)(s * WGeom<48>::kCopyBytes + top * WGeom<48>::kRowBytes + 2 * e);
}

hipError_t launch_extract_weighted(const ExtractArgs &a, hipStream_t stream)
{
    if (a.n <= 0) return hipSuccess;
    return a.window == 64 ? launch_weighted_w<64>(a, stream) : launch_weighted_w<48>(a, stream);
}

}  // namespace latch
