// Brute-force 2-NN Hamming matching for gfx950 (Sec. 4, "Descriptor matching
// on the GPU": exhaustive distances between all query/train pairs).
//
// Two interchangeable paths produce identical partial results:
//
//   MFMA.  With a, b in {0,1}^512, Hamming(a, b) = |a| + |b| - 2 a.b, and a.b
//   over all pairs is an int8 x int8 -> int32 matrix product with K = 512.
//   A prep kernel expands train bits to 0/1 bytes in the exact fragment
//   order of v_mfma_i32_32x32x32_i8 (one 16 KB tile per 32 train rows), so
//   the main kernel streams tiles HBM -> LDS -> MFMA with contiguous,
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
// MFMA operand prep.
//
// Fragment order: for tile tau (train rows 32 tau .. 32 tau + 31), step s
// (0..15) and lane l (0..63), the 16 bytes at tau * 16384 + s * 1024 + l * 16
// are bits 32 s + 16 (l / 32) + m, m = 0..15, of train row 32 tau + (l % 32),
// as 0/1 bytes.  Query fragments use the same bit -> (step, lane, byte) map,
// so the MFMA's k-summation covers every bit exactly once whatever its
// internal k order.  Rows beyond nt are zero.
//
// rowbase[j] = ((512 - |t_j|) << 21) + (2^21 - 1 - (j mod split_rows)) for
// j < nt, 0 beyond: the constant part of the match key (see knn_mfma_kernel).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void knn_prep_kernel(const uint32_t *__restrict__ train,
                                                        int nt, int split_rows,
                                                        uint4 *__restrict__ expanded,
                                                        uint32_t *__restrict__ rowbase)
{
    const int tile = blockIdx.x;
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int f = t + 256 * i;          // fragment index within the tile
        const int s = f >> 6;
        const int l = f & 63;
        const int row = tile * kTileRows + (l & 31);
        uint32_t x = 0;
        if (row < nt) x = (train[(size_t)row * kWords + s] >> (16 * (l >> 5))) & 0xffffu;
        const v4i e = expand16(x);
        expanded[(size_t)tile * (kTileBytes / 16) + f] = make_uint4(e[0], e[1], e[2], e[3]);
    }
    if (t < kTileRows) {
        const int row = tile * kTileRows + t;
        uint32_t base = 0;
        if (row < nt) {
            uint32_t pc = 0;
#pragma unroll
            for (int w = 0; w < kWords; ++w) pc += __popc(train[(size_t)row * kWords + w]);
            const uint32_t local = (uint32_t)(row % split_rows);
            base = ((512u - pc) << kLocalBits) + (kLocalMask - local);
        }
        rowbase[row] = base;
    }
}

// ---------------------------------------------------------------------------
// MFMA matcher.  Workgroup = 4 wavefronts x 64 queries; grid (query blocks,
// splits).  For train row j (split-local index jl) and a query,
//   key = (a.b << 22) + rowbase[j] = ((2 a.b + 512 - |b|) << 21) + (2^21 - 1 - jl),
// and 2 a.b - |b| = |a| - Hamming(a, b), so for a fixed query the largest key
// is the smallest (distance, index).  Key 0 only arises for padding rows
// (split-local indices stay below 2^21 - 1), so 0 means "no neighbour".
//
// Accumulator layout of v_mfma_i32_32x32x32_i8 (output 32 x 32, 16 values
// per lane): lane l holds column l % 32 and rows 8 (r / 4) + 4 (l / 32) + r % 4
// for r = 0..15.  Train rows are the MFMA rows (operand A, streamed from LDS)
// and queries the columns (operand B, resident), so each lane keeps a
// running top-2 for one query; lanes l and l ^ 32 merge at the end.
// ---------------------------------------------------------------------------
constexpr int kMfmaWaves = 4;
constexpr int kQueryBlocks = 2;                        // 32-query blocks per wavefront
constexpr int kQueriesPerWave = 32 * kQueryBlocks;
constexpr int kQueriesPerGroup = kMfmaWaves * kQueriesPerWave;
constexpr int kTileVec = kTileBytes / 16;              // uint4 per tile (1024)

__global__ __launch_bounds__(kMfmaWaves * 64) __attribute__((amdgpu_waves_per_eu(2, 2))) void knn_mfma_kernel(
    const uint32_t *__restrict__ query, int nq, const uint4 *__restrict__ expanded,
    const uint32_t *__restrict__ rowbase, int nt, int split_rows, uint64_t *__restrict__ partial)
{
    __shared__ v4i tbuf[2][kTileVec];
    __shared__ uint4 bbuf[2][kTileRows / 4];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int half = lane >> 5;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int split = blockIdx.y;
    const int qbase = blockIdx.x * kQueriesPerGroup + wave * kQueriesPerWave;

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
            bq[qb][s] = expand16((w >> (16 * half)) & 0xffffu);
        }
        na[qb] = pc;
    }

    const int ntiles_all = (nt + kTileRows - 1) / kTileRows;
    const int tiles_per_split = split_rows / kTileRows;
    const int t_begin = split * tiles_per_split;
    const int t_end = min(ntiles_all, t_begin + tiles_per_split);

    uint32_t k1[kQueryBlocks], k2[kQueryBlocks];
#pragma unroll
    for (int qb = 0; qb < kQueryBlocks; ++qb) k1[qb] = k2[qb] = 0u;

    // Stage the first tile.
    if (t_begin < t_end) {
        const v4i *src = reinterpret_cast<const v4i *>(expanded) + (size_t)t_begin * kTileVec;
#pragma unroll
        for (int i = 0; i < 4; ++i) tbuf[0][tid + 256 * i] = src[tid + 256 * i];
        if (tid < kTileRows / 4)
            bbuf[0][tid] = reinterpret_cast<const uint4 *>(rowbase + (size_t)t_begin * kTileRows)[tid];
    }
    __syncthreads();

    for (int tile = t_begin; tile < t_end; ++tile) {
        const int buf = (tile - t_begin) & 1;
        const bool more = tile + 1 < t_end;

        // Prefetch the next tile into registers.
        v4i nx[4];
        uint4 nb = make_uint4(0, 0, 0, 0);
        if (more) {
            const v4i *src = reinterpret_cast<const v4i *>(expanded) + (size_t)(tile + 1) * kTileVec;
#pragma unroll
            for (int i = 0; i < 4; ++i) nx[i] = src[tid + 256 * i];
            if (tid < kTileRows / 4)
                nb = reinterpret_cast<const uint4 *>(rowbase + (size_t)(tile + 1) * kTileRows)[tid];
        }

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

        // Epilogue: rows 8 g + 4 half + e, g = 0..3, e = 0..3.
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const uint4 bb = bbuf[buf][2 * g + half];
            const uint32_t base[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
#pragma unroll
                for (int qb = 0; qb < kQueryBlocks; ++qb) {
                    const uint32_t key = ((uint32_t)acc[qb][4 * g + e] << 22) + base[e];
                    k2[qb] = umed3(k1[qb], k2[qb], key);
                    k1[qb] = max(k1[qb], key);
                }
            }
        }

        if (more) {
#pragma unroll
            for (int i = 0; i < 4; ++i) tbuf[buf ^ 1][tid + 256 * i] = nx[i];
            if (tid < kTileRows / 4) bbuf[buf ^ 1][tid] = nb;
        }
        __syncthreads();
    }

    // Merge the two row halves, decode, store.
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
    for (int s = 0; s < nsplit; ++s) {
        const uint64_t *src = partial + ((size_t)s * nq + q) * 2;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint64_t v = src[e];
            if (v < b1) {
                b2 = b1;
                b1 = v;
            } else if (v < b2) {
                b2 = v;
            }
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

hipError_t launch_knn_prep(const uint32_t *train, int64_t nt, const KnnPlan &plan,
                           uint8_t *expanded, uint32_t *rowbase, hipStream_t stream)
{
    const int64_t tiles = (nt + kTileRows - 1) / kTileRows;
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(knn_prep_kernel, dim3((unsigned)tiles), dim3(256), 0, stream, train,
                       (int)nt, (int)plan.split_rows, reinterpret_cast<uint4 *>(expanded), rowbase);
    return hipGetLastError();
}

hipError_t launch_knn_mfma(const uint32_t *query, const uint8_t *expanded,
                           const uint32_t *rowbase, const KnnPlan &plan, uint64_t *partial,
                           hipStream_t stream)
{
    const int64_t qblocks = (plan.nq + kQueriesPerGroup - 1) / kQueriesPerGroup;
    hipLaunchKernelGGL(knn_mfma_kernel, dim3((unsigned)qblocks, (unsigned)plan.nsplit),
                       dim3(kMfmaWaves * 64), 0, stream, query, (int)plan.nq,
                       reinterpret_cast<const uint4 *>(expanded), rowbase, (int)plan.nt,
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

int knn_queries_per_group_mfma() { return kQueriesPerGroup; }

}  // namespace latch
