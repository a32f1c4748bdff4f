// Dense CLATCH and dense matching for gfx950 (Sec. 6 proposes CLATCH for
// dense pixel matching).
//
// Dense extraction: the descriptor of every pixel p of a region, upright and
// at scale 1 (the resampling rule then samples I(p + (u, v)) with clamping,
// so the window is the edge-padded image around p).  For a triplet with
// patch centres A, C1, C2 (window coordinates), Eq. 1 compares
//     S1 - S2 = sum over the 7 x 7 box of G(q),
//     G(q) = (I(q + c1) - I(q + c2)) (I(q + c1) + I(q + c2) - 2 I(q + a)),
// with a, c1, c2 the centres minus (24, 24): bit = [box7x7(G)(p) > 0].  So a
// workgroup that owns a tile of pixels evaluates G once per position and
// triplet, sums it over 7 rows with a running sum held in registers (lane =
// column, walking down the rows) and over 7 columns across lanes: about 10
// operations per pixel and triplet instead of 3 x 49 products.  |G| <= 130,050
// and the box sum < 2^23, so int32 is exact, and the result is bit-identical
// to extracting at every pixel.
//
// Dense matching: per query pixel, the two nearest train pixels by Hamming
// distance within +/- R rows and columns (R <= 8), ties to the lower raster
// index, ratio test as in hamming_knn.  A workgroup owns 16 x 16 queries and
// stages the (16 + 2R)^2 train descriptors around them in LDS.
#include "internal.h"

namespace latch {
namespace {

constexpr int kDThreads = 256;
constexpr int kDTileW = 58;                         // output columns: lanes 0..57 (+6 halo lanes)
constexpr int kDTileH = 32;                         // output rows per workgroup
constexpr int kDRegionRows = kDTileH + 6;           // rows of G per tile
constexpr int kDTexRows = kDRegionRows + 41;        // image rows: 79
constexpr int kDTexCols = 64 + 41;                  // image columns: 105
constexpr int kDTexStride = 108;
constexpr int kDTexLoads = (kDTexRows * kDTexCols + kDThreads - 1) / kDThreads;   // 33

__device__ __forceinline__ int mul24(int a, int b)
{
    int r;
    asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// a b + c with 24-bit signed a, b (b an inline constant here).
__device__ __forceinline__ int mad24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "i"(b), "v"(c));
    return r;
}

// 1 if h > 0, else 0, in one instruction (median of h, 0 and 1).
__device__ __forceinline__ uint32_t bit_of(int h)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, 1" : "=v"(r) : "v"(h));
    return (uint32_t)r;
}

// Lane l receives lane l + 1's value (DPP wave_shl:1; lane 63 receives 0
// through bound_ctrl, so no old value has to be set up).
__device__ __forceinline__ int lane_next(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true);
}

// Sum of v over lanes l .. l + 6 (only lanes 0 .. 57 are used), in Horner
// form t = v + (t of the next lane), six times: each step is one add whose
// shifted operand comes through DPP (whole-wavefront shift), with no LDS
// traffic.
__device__ __forceinline__ int sum7_down(int v)
{
    int t = v;
#pragma unroll
    for (int k = 0; k < 6; ++k) t = v + lane_next(t);
    return t;
}

__global__ __launch_bounds__(kDThreads) void dense_extract_kernel(
    const uint8_t *__restrict__ img, int height, int width, int pitch, int x0, int y0, int gw, int gh,
    int tiles_x, const uint2 *__restrict__ toff, uint32_t *__restrict__ desc)
{
    __shared__ uint8_t tex[(kDTexLoads * kDThreads + kDTexCols - 1) / kDTexCols * kDTexStride];
    const int tx = (int)(blockIdx.x % (unsigned)tiles_x), ty = (int)(blockIdx.x / (unsigned)tiles_x);
    const int X0 = x0 + tx * kDTileW, Y0 = y0 + ty * kDTileH;
    const int t = threadIdx.x;
    const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);

    // Image rows Y0 - 24 .. Y0 + 54 and columns X0 - 24 .. X0 + 80, clamped
    // to the image (the rule's clamp-to-edge); three batches of 11 loads in
    // flight, so that the staging does not set the kernel's register count.
    static_assert(kDTexLoads == 33, "three batches of 11");
#pragma unroll
    for (int batch = 0; batch < 3; ++batch) {
        uint32_t v[11];
#pragma unroll
        for (int k = 0; k < 11; ++k) {
            const int i = t + (11 * batch + k) * kDThreads;
            const int yy = min(max(Y0 - 24 + i / kDTexCols, 0), height - 1);
            const int xx = min(max(X0 - 24 + i % kDTexCols, 0), width - 1);
            v[k] = img[(size_t)yy * pitch + xx];
        }
#pragma unroll
        for (int k = 0; k < 11; ++k) {
            const int i = t + (11 * batch + k) * kDThreads;
            tex[(i / kDTexCols) * kDTexStride + i % kDTexCols] = (uint8_t)v[k];
        }
    }
    __syncthreads();

    // Wavefront w computes output words w, w + 4, w + 8, w + 12.
    for (int word = wave; word < kWords; word += 4) {
        uint32_t bits[kDTileH];
#pragma unroll
        for (int o = 0; o < kDTileH; ++o) bits[o] = 0u;
        for (int b = 0; b < 32; ++b) {
            const uint2 off = toff[32 * word + b];           // uniform: scalar loads
            const uint8_t *pa = tex + lane + (off.x & 0xffffu);
            const uint8_t *p1 = tex + lane + (off.x >> 16);
            const uint8_t *p2 = tex + lane + off.y;
            int ring[7];
            int s = 0;
#pragma unroll
            for (int rr = 0; rr < kDRegionRows; ++rr) {
                const int a = pa[rr * kDTexStride], c1 = p1[rr * kDTexStride], c2 = p2[rr * kDTexStride];
                const int g = mul24(c1 - c2, mad24(a, -2, c1 + c2));
                ring[rr % 7] = g;
                s += g;
                if (rr >= 6) {
                    const int h = sum7_down(s);                // box over rows rr-6..rr, columns l..l+6
                    // Shift in from the right: triplet b ends at bit 31 - b.
                    bits[rr - 6] = (bits[rr - 6] << 1) | bit_of(h);
                    s -= ring[(rr - 6) % 7];
                }
            }
        }
#pragma unroll
        for (int o = 0; o < kDTileH; ++o) bits[o] = __builtin_bitreverse32(bits[o]);
        const int px = X0 + lane;
        if (lane < kDTileW && px < x0 + gw) {
#pragma unroll
            for (int o = 0; o < kDTileH; ++o) {
                const int py = Y0 + o;
                if (py < y0 + gh)
                    desc[((size_t)(py - y0) * gw + (px - x0)) * kWords + word] = bits[o];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Dense matching.

constexpr int kMTile = 16;                               // queries per side
constexpr int kMaxRadius = 8;
static_assert((kMTile + 2 * kMaxRadius) * (kMTile + 2 * kMaxRadius) * 64 <= 65536,
              "the largest region fits the default dynamic LDS limit");

__global__ __launch_bounds__(kDThreads) void dense_match_kernel(
    const uint32_t *__restrict__ query, const uint32_t *__restrict__ train, int gw, int gh, int radius,
    int tiles_x, int k, float ratio, int32_t *__restrict__ idx, int32_t *__restrict__ dist,
    uint8_t *__restrict__ accept)
{
    // Train descriptors of the (16 + 2 radius)^2 region, 64 B each, stored
    // chunk-major: the 16-byte chunk c of position p is region[c plane + p].
    // The 16 lanes of a query row read chunk c of 16 consecutive positions,
    // 256 contiguous bytes, which LDS serves without bank conflicts.  The
    // launch sizes the region for the radius (36 KB at radius 4).
    extern __shared__ uint4 region[];
    const int tx = (int)(blockIdx.x % (unsigned)tiles_x), ty = (int)(blockIdx.x / (unsigned)tiles_x);
    const int t = threadIdx.x;
    const int side = kMTile + 2 * radius;
    const int plane = side * side;
    const int rx0 = tx * kMTile - radius, ry0 = ty * kMTile - radius;
    for (int i = t; i < side * side * 4; i += kDThreads) {
        const int p = i >> 2, c = i & 3;
        const int gy = ry0 + p / side, gx = rx0 + p % side;
        uint4 val = make_uint4(0u, 0u, 0u, 0u);
        if (gy >= 0 && gy < gh && gx >= 0 && gx < gw)
            val = reinterpret_cast<const uint4 *>(train + ((size_t)gy * gw + gx) * kWords)[c];
        region[c * plane + p] = val;
    }
    const int qx = tx * kMTile + (t & 15), qy = ty * kMTile + (t >> 4);
    const bool real = qx < gw && qy < gh;
    uint32_t qd[kWords];
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(query + ((size_t)(real ? qy : 0) * gw + (real ? qx : 0)) * kWords);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const uint4 w = src[c];
            qd[4 * c] = w.x;
            qd[4 * c + 1] = w.y;
            qd[4 * c + 2] = w.z;
            qd[4 * c + 3] = w.w;
        }
    }
    __syncthreads();

    // Keys d << 9 | window index: smaller is better; the window index grows
    // with the raster index of the candidate, so ties go to the lower one.
    uint32_t best1 = 0xffffffffu, best2 = 0xffffffffu;
    const int wside = 2 * radius + 1;
    for (int dy = -radius; dy <= radius; ++dy) {
        const bool row_ok = qy + dy >= 0 && qy + dy < gh;
        for (int dx = -radius; dx <= radius; ++dx) {
            const int p = ((t >> 4) + radius + dy) * side + (t & 15) + radius + dx;
            uint32_t d = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const uint4 w = region[c * plane + p];
                d += __builtin_popcount(w.x ^ qd[4 * c]) + __builtin_popcount(w.y ^ qd[4 * c + 1]) +
                     __builtin_popcount(w.z ^ qd[4 * c + 2]) + __builtin_popcount(w.w ^ qd[4 * c + 3]);
            }
            const bool ok = row_ok && qx + dx >= 0 && qx + dx < gw;
            const uint32_t key = ok ? (d << 9) | (uint32_t)((dy + radius) * wside + dx + radius) : 0xffffffffu;
            const uint32_t lo = min(best1, key);
            best2 = min(best2, max(best1, key));
            best1 = lo;
        }
    }
    if (!real) return;
    const int ny = min(gh - 1, qy + radius) - max(0, qy - radius) + 1;
    const int nx = min(gw - 1, qx + radius) - max(0, qx - radius) + 1;
    const int n = ny * nx;
    auto decode = [&](uint32_t key, int32_t &i_out, int32_t &d_out) {
        if (key == 0xffffffffu) {
            i_out = -1;
            d_out = 513;
            return;
        }
        const int w = (int)(key & 511u);
        const int dy = w / wside - radius, dx = w % wside - radius;
        i_out = (qy + dy) * gw + qx + dx;
        d_out = (int)(key >> 9);
    };
    const size_t q = (size_t)qy * gw + qx;
    int32_t i1, d1, i2, d2;
    decode(best1, i1, d1);
    decode(best2, i2, d2);
    idx[k * q] = i1;
    dist[k * q] = d1;
    if (k == 2) {
        idx[k * q + 1] = i2;
        dist[k * q + 1] = d2;
    }
    if (accept) accept[q] = (uint8_t)(n >= 2 && (double)d1 < (double)ratio * (double)d2);
}

}  // namespace

uint32_t dense_patch_offset(int r, int c)
{
    return (uint32_t)((r - 3) * kDTexStride + (c - 3));
}

hipError_t launch_dense_extract(const DenseArgs &a, hipStream_t stream)
{
    const int tiles_x = (a.gw + kDTileW - 1) / kDTileW;
    const int64_t tiles = (int64_t)tiles_x * ((a.gh + kDTileH - 1) / kDTileH);
    hipLaunchKernelGGL(dense_extract_kernel, dim3((unsigned)tiles), dim3(kDThreads), 0, stream, a.img,
                       a.height, a.width, a.pitch, a.x0, a.y0, a.gw, a.gh, tiles_x, a.toff, a.desc);
    return hipGetLastError();
}

hipError_t launch_dense_match(const DenseMatchArgs &a, hipStream_t stream)
{
    const int tiles_x = (a.gw + kMTile - 1) / kMTile;
    const int64_t tiles = (int64_t)tiles_x * ((a.gh + kMTile - 1) / kMTile);
    if (a.radius < 0 || a.radius > kMaxRadius) return hipErrorInvalidValue;
    const int side = kMTile + 2 * a.radius;
    const size_t lds = (size_t)side * side * 4 * sizeof(uint4);   // <= 64 KB
    hipLaunchKernelGGL(dense_match_kernel, dim3((unsigned)tiles), dim3(kDThreads), lds, stream, a.query,
                       a.train, a.gw, a.gh, a.radius, tiles_x, a.k, a.ratio, a.idx, a.dist, a.accept);
    return hipGetLastError();
}

}  // namespace latch
