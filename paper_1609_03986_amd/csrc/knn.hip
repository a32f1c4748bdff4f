// Brute-force 2-NN Hamming matching for gfx950 (Sec. 4, "Descriptor matching
// on the GPU": exhaustive distances between all query/train pairs).
//
// Two interchangeable paths produce identical partial results:
//
//   MFMA.  With a, b in {0,1}^512, Hamming(a, b) = |a| + |b| - 2 a.b, and a.b
//   over all pairs is an int8 x int8 -> int32 matrix product with K = 512.
//   Packed train tiles (32 rows, 2 KB) are expanded to 0/1 bytes in the exact
//   fragment order of v_mfma_i32_32x32x32_i8 while being staged in LDS, so
//   HBM carries packed bits only and the MFMA operands come from contiguous,
//   conflict-free ds_read_b128.  Queries stay resident in VGPRs (64 queries,
//   128 VGPRs per wavefront).  The sum is exact in int32 (<= 512).
//
//   POPCOUNT.  Each lane owns one query (16 VGPRs); train rows are uniform
//   across the wavefront and arrive through scalar loads; 16 x (v_xor,
//   v_bcnt) per pair.
//
// Top-2 selection packs (distance, split-local index) into one 32-bit key so
// that one min/max and one med3 keep the two best per lane; ties resolve to
// the lowest index because the index is part of the key.  Each (query,
// train split) writes its best two as 64-bit (distance << 32 | index) values;
// a merge kernel reduces over splits and applies the ratio test.
#include "internal.h"

namespace latch {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr uint32_t kLocalBits = 21;
constexpr uint32_t kLocalMask = (1u << kLocalBits) - 1;

__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c)
{
    return max(min(a, b), min(max(a, b), c));
}

// Four bits -> four bytes of value 0/1 (bit e of nib -> byte e).  The four
// shifted copies of nib occupy disjoint bit ranges, so the product has no carries.
__device__ __forceinline__ uint32_t spread_nibble(uint32_t nib)
{
    return (nib * 0x00204081u) & 0x01010101u;
}

// 16 bits -> 16 bytes of value 0/1, byte m = bit m.
__device__ __forceinline__ v4i expand16(uint32_t x)
{
    v4i r;
    r[0] = (int)spread_nibble(x & 0xfu);
    r[1] = (int)spread_nibble((x >> 4) & 0xfu);
    r[2] = (int)spread_nibble((x >> 8) & 0xfu);
    r[3] = (int)spread_nibble((x >> 12) & 0xfu);
    return r;
}

// ---------------------------------------------------------------------------
// MFMA matcher.  Workgroup = 4 wavefronts x 64 queries; grid (query groups,
// train splits).
//
// Operands.  Train bits enter as bytes b_k in {0, 1} (operand A), query bits
// as signed bytes 2 a_k - 1 in {-1, +1} (operand B, resident in VGPRs), so the
// int8 MFMA sum over K = 512 is directly
//   s = sum_k (2 a_k - 1) b_k = 2 a.b - |b| = |a| - Hamming(a, b),
// exact in int32, and no train-side popcount is needed.
//
// Fragment order.  For a 32-row train tile, step s (0..15) and lane l
// (0..63), the A fragment is 16 bytes: bits 32 s + 16 (l / 32) + m, m = 0..15,
// of tile row l % 32.  Query fragments use the same bit -> (step, lane, byte)
// map, so the MFMA k-sum covers every bit exactly once whatever its internal k
// order.  Each tile is expanded from its packed 2 KB into this order while
// being staged in LDS (16 KB) and read back with contiguous, conflict-free
// ds_read_b128.
//
// Keys.  For train row j with split-local index jl,
//   key = ((s + 512) << 21) + (2^21 - 1 - jl),   s + 512 in [0, 1024],
// so for a fixed query the largest key is the smallest (distance, index).
// Split-local indices stay below 2^21 - 1, so a real key is never 0; rows
// past nt (only in the last tile) are forced to key 0 = "no neighbour".
//
// Accumulator layout of v_mfma_i32_32x32x32_i8 (output 32 x 32, 16 values
// per lane): lane l holds column l % 32 and rows 8 (r / 4) + 4 (l / 32) + r % 4
// for r = 0..15.  Train rows are the MFMA rows and queries the columns, so
// each lane keeps a running top-2 for one query; lanes l and l ^ 32 merge at
// the end.
// ---------------------------------------------------------------------------
constexpr int kMfmaWaves = 4;
constexpr int kMfmaThreads = kMfmaWaves * 64;
constexpr int kQueryBlocks = 2;                        // 32-query blocks per wavefront
constexpr int kQueriesPerWave = 32 * kQueryBlocks;
constexpr int kQueriesPerGroup = kMfmaWaves * kQueriesPerWave;
constexpr int kTileVec = kTileBytes / 16;              // 16-byte fragments per tile (1024)
static_assert(kMfmaThreads == 8 * kTileRows, "staging: 8 threads per tile row");

// 16 bits -> 16 signed bytes, +1 for a set bit and -1 for a clear one: byte
// b in {0, 1} becomes 0xff ^ 0xfe b, and 0xfe b = (b << 8) - (b << 1) stays
// inside its own byte, so the whole dword is ~((x << 8) - (x << 1)) mod 2^32.
__device__ __forceinline__ v4i expand16_pm1(uint32_t x)
{
    v4i r = expand16(x);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t b = (uint32_t)r[i];
        r[i] = (int)~((b << 8) - (b << 1));
    }
    return r;
}

// Staging role of a thread: tile row tid % 32, packed words 2 (tid / 32) and
// 2 (tid / 32) + 1, i.e. steps 2 (tid / 32) + {0, 1}, both halves.
__device__ __forceinline__ uint2 load_tile(const uint32_t *__restrict__ train, int nt, int tile,
                                           int tid)
{
    const int row = tile * kTileRows + (tid & 31);
    return row < nt ? reinterpret_cast<const uint2 *>(train + (size_t)row * kWords)[tid >> 5]
                    : make_uint2(0, 0);
}

__device__ __forceinline__ void stage_tile(uint2 w, int tid, v4i *__restrict__ buf)
{
    const int r = tid & 31;
    const int c = tid >> 5;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const uint32_t word = e == 0 ? w.x : w.y;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            buf[(2 * c + e) * 64 + 32 * h + r] = expand16((word >> (16 * h)) & 0xffffu);
    }
}

__global__ __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void
knn_mfma_kernel(const uint32_t *__restrict__ query, int nq, const uint32_t *__restrict__ train,
                int nt, int split_rows, uint64_t *__restrict__ partial)
{
    __shared__ v4i tbuf[2][kTileVec];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int half = lane >> 5;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int split = blockIdx.y;
    const int qbase = blockIdx.x * kQueriesPerGroup + wave * kQueriesPerWave;

    const int ntiles_all = (nt + kTileRows - 1) / kTileRows;
    const int tiles_per_split = split_rows / kTileRows;
    const int t_begin = split * tiles_per_split;
    const int t_end = min(ntiles_all, t_begin + tiles_per_split);

    uint2 ld = make_uint2(0, 0);
    if (t_begin < t_end) ld = load_tile(train, nt, t_begin, tid);

    // Resident query fragments and query popcounts.
    v4i bq[kQueryBlocks][16];
    int na[kQueryBlocks];
#pragma unroll
    for (int qb = 0; qb < kQueryBlocks; ++qb) {
        const int qn = qbase + 32 * qb + (lane & 31);
        int pc = 0;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const uint32_t w = qn < nq ? query[(size_t)qn * kWords + s] : 0u;
            pc += __popc(w);
            bq[qb][s] = expand16_pm1((w >> (16 * half)) & 0xffffu);
        }
        na[qb] = pc;
    }

    uint32_t k1[kQueryBlocks], k2[kQueryBlocks];
#pragma unroll
    for (int qb = 0; qb < kQueryBlocks; ++qb) k1[qb] = k2[qb] = 0u;

    if (t_begin < t_end) stage_tile(ld, tid, tbuf[0]);
    __syncthreads();

    for (int tile = t_begin; tile < t_end; ++tile) {
        const int buf = (tile - t_begin) & 1;
        const bool more = tile + 1 < t_end;
        if (more) ld = load_tile(train, nt, tile + 1, tid);     // lands during the MFMAs below

        v16i acc[kQueryBlocks];
#pragma unroll
        for (int qb = 0; qb < kQueryBlocks; ++qb) acc[qb] = (v16i){};
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const v4i a = tbuf[buf][s * 64 + lane];
#pragma unroll
            for (int qb = 0; qb < kQueryBlocks; ++qb)
                acc[qb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, bq[qb][s], acc[qb], 0, 0, 0);
        }

        // Epilogue.  Register r = 4 g + e holds tile row m = 8 g + 4 half + e,
        // split-local index tile * 32 - split * split_rows + m.  Padding rows
        // (past nt, last tile only) have all-zero bytes, so s = 0 there and a
        // zero key base makes their key 0.
        const uint32_t kt = (512u << kLocalBits) + kLocalMask -
                            (uint32_t)(tile * kTileRows - split * split_rows) - 4u * half;
        const int valid_rows = nt - tile * kTileRows;        // < 32 only in the last tile
        uint32_t cb[16];
        if (valid_rows >= kTileRows) {
#pragma unroll
            for (int r = 0; r < 16; ++r) cb[r] = kt - (uint32_t)(8 * (r >> 2) + (r & 3));
        } else {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = 8 * (r >> 2) + 4 * half + (r & 3);
                cb[r] = m < valid_rows ? kt - (uint32_t)(8 * (r >> 2) + (r & 3)) : 0u;
            }
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
#pragma unroll
            for (int qb = 0; qb < kQueryBlocks; ++qb) {
                const uint32_t key = ((uint32_t)acc[qb][r] << kLocalBits) + cb[r];
                k2[qb] = umed3(k1[qb], k2[qb], key);
                k1[qb] = max(k1[qb], key);
            }
        }

        if (more) stage_tile(ld, tid, tbuf[buf ^ 1]);
        __syncthreads();
    }

    // Merge the two row halves, decode (d = |a| + 512 - (key >> 21)), store.
#pragma unroll
    for (int qb = 0; qb < kQueryBlocks; ++qb) {
        const uint32_t o1 = __shfl_xor(k1[qb], 32);
        const uint32_t o2 = __shfl_xor(k2[qb], 32);
        const uint32_t b1 = max(k1[qb], o1);
        const uint32_t b2 = max(min(k1[qb], o1), max(k2[qb], o2));
        const int qn = qbase + 32 * qb + (lane & 31);
        if (half == 0 && qn < nq) {
            uint64_t r[2];
            const uint32_t kk[2] = {b1, b2};
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                if (kk[e] == 0u) {
                    r[e] = kNoNeighbour;
                } else {
                    const uint32_t score = kk[e] >> kLocalBits;
                    const uint32_t d = (uint32_t)na[qb] + 512u - score;
                    const uint32_t j = (uint32_t)split * (uint32_t)split_rows +
                                       (kLocalMask - (kk[e] & kLocalMask));
                    r[e] = ((uint64_t)d << 32) | j;
                }
            }
            uint64_t *dst = partial + ((size_t)split * nq + qn) * 2;
            dst[0] = r[0];
            dst[1] = r[1];
        }
    }
}

// ---------------------------------------------------------------------------
// Popcount matcher.  One query per lane; grid (query blocks of 256, splits).
// key = (d << 21) | jl with d <= 512, jl < 2^21 - 1, so ~0u means "none".
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void knn_popcount_kernel(
    const uint32_t *__restrict__ query, int nq, const uint32_t *__restrict__ train, int nt,
    int split_rows, uint64_t *__restrict__ partial)
{
    const int qn = blockIdx.x * 256 + threadIdx.x;
    const int split = blockIdx.y;
    const int j0 = split * split_rows;
    const int j1 = min(nt, j0 + split_rows);

    uint32_t q[kWords];
#pragma unroll
    for (int w = 0; w < kWords; ++w) q[w] = qn < nq ? query[(size_t)qn * kWords + w] : 0u;

    uint32_t k1 = ~0u, k2 = ~0u;
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
        const uint32_t *t = train + (size_t)j * kWords;
        uint32_t d = 0;
#pragma unroll
        for (int w = 0; w < kWords; ++w) d = __popc(q[w] ^ t[w]) + d;
        const uint32_t key = (d << kLocalBits) | (uint32_t)(j - j0);
        k2 = umed3(k1, k2, key);
        k1 = min(k1, key);
    }

    if (qn < nq) {
        const uint32_t kk[2] = {k1, k2};
        uint64_t *dst = partial + ((size_t)split * nq + qn) * 2;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            dst[e] = kk[e] == ~0u ? kNoNeighbour
                                  : (((uint64_t)(kk[e] >> kLocalBits) << 32) |
                                     (uint32_t)(j0 + (int)(kk[e] & kLocalMask)));
        }
    }
}

// ---------------------------------------------------------------------------
// Merge per-split partials (64-bit keys: distance << 32 | global index, so the
// integer order is the lexicographic one) and apply the ratio test exactly:
// a float32 ratio times an integer <= 512 is exact in double.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void knn_merge_kernel(
    const uint64_t *__restrict__ partial, int nq, int nsplit, int nt, int k, float ratio,
    int32_t *__restrict__ idx, int32_t *__restrict__ dist, uint8_t *__restrict__ accept)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= nq) return;
    uint64_t b1 = kNoNeighbour, b2 = kNoNeighbour;
    // Eight splits' loads in flight at a time, then a branch-free top-2 update.
    for (int s0 = 0; s0 < nsplit; s0 += 8) {
        uint64_t v[16];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const bool in = s0 + i < nsplit;
            const uint64_t *src = partial + ((size_t)(in ? s0 + i : 0) * nq + q) * 2;
            v[2 * i] = in ? src[0] : kNoNeighbour;
            v[2 * i + 1] = in ? src[1] : kNoNeighbour;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            b2 = min(b2, max(b1, v[i]));
            b1 = min(b1, v[i]);
        }
    }
    const int d1 = b1 == kNoNeighbour ? 513 : (int)(b1 >> 32);
    const int d2 = b2 == kNoNeighbour ? 513 : (int)(b2 >> 32);
    const int j1 = b1 == kNoNeighbour ? -1 : (int)(uint32_t)b1;
    const int j2 = b2 == kNoNeighbour ? -1 : (int)(uint32_t)b2;
    idx[(size_t)q * k] = j1;
    dist[(size_t)q * k] = d1;
    if (k == 2) {
        idx[(size_t)q * k + 1] = j2;
        dist[(size_t)q * k + 1] = d2;
    }
    if (accept) accept[q] = (uint8_t)(nt >= 2 && (double)d1 < (double)ratio * (double)d2);
}

}  // namespace

hipError_t launch_knn_mfma(const uint32_t *query, const uint32_t *train, const KnnPlan &plan,
                           uint64_t *partial, hipStream_t stream)
{
    const int64_t qblocks = (plan.nq + kQueriesPerGroup - 1) / kQueriesPerGroup;
    hipLaunchKernelGGL(knn_mfma_kernel, dim3((unsigned)qblocks, (unsigned)plan.nsplit),
                       dim3(kMfmaThreads), 0, stream, query, (int)plan.nq, train, (int)plan.nt,
                       (int)plan.split_rows, partial);
    return hipGetLastError();
}

hipError_t launch_knn_popcount(const uint32_t *query, const uint32_t *train, const KnnPlan &plan,
                               uint64_t *partial, hipStream_t stream)
{
    const int64_t qblocks = (plan.nq + 255) / 256;
    hipLaunchKernelGGL(knn_popcount_kernel, dim3((unsigned)qblocks, (unsigned)plan.nsplit),
                       dim3(256), 0, stream, query, (int)plan.nq, train, (int)plan.nt,
                       (int)plan.split_rows, partial);
    return hipGetLastError();
}

hipError_t launch_knn_merge(const uint64_t *partial, const KnnPlan &plan, int k, float ratio,
                            int32_t *idx, int32_t *dist, uint8_t *accept, hipStream_t stream)
{
    const int64_t blocks = (plan.nq + 255) / 256;
    hipLaunchKernelGGL(knn_merge_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, partial,
                       (int)plan.nq, plan.nsplit, (int)plan.nt, k, ratio, idx, dist, accept);
    return hipGetLastError();
}

}  // namespace latch
