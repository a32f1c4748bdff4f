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
// that a max3, a med3 and a max fold two keys into the two best per lane;
// ties resolve to the lowest index because the index is part of the key.  Each (query,
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

// Two keys x, y into a running top two (k1 >= k2, as a multiset): the new
// largest is max(k1, x, y); the new second is max(k2, med3(k1, x, y)), since
// if k1 stays largest the second is max(k2, x, y) = max(k2, med3), and if x
// (or y) is largest the second is max(k1, y) (or max(k1, x)), which is the
// median of k1, x, y and is >= k2.  Three operations per two keys, against
// two per key inserted one at a time.
__device__ __forceinline__ void insert_pair_u32(uint32_t &k1, uint32_t &k2, uint32_t x, uint32_t y)
{
    k2 = max(k2, umed3(k1, x, y));
    k1 = max(max(k1, x), y);
}


// Four bits -> four bytes of value 0/1 (bit e of nib -> byte e).  The four
// shifted copies of nib occupy disjoint bit ranges, so the product has no
// carries; nib < 16 and the constant < 2^24 make it a full-rate 24-bit multiply.
__device__ __forceinline__ uint32_t spread_nibble(uint32_t nib)
{
    return __umul24(nib, 0x00204081u) & 0x01010101u;
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
constexpr int kMfmaThreads = kMfmaWaves * 64;
constexpr int kQueryBlocks = 2;                        // 32-query blocks per wavefront
constexpr int kQueriesPerWave = 32 * kQueryBlocks;
constexpr int kQueriesPerGroup = kMfmaWaves * kQueriesPerWave;
static_assert(kQueriesPerGroup == 256, "query groups of 256 in every matcher");
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
    // Rows past nt load row nt - 1 (or row 0 of an empty set, which is never
    // staged) and are zeroed, without a branch.
    const int row = tile * kTileRows + (tid & 31);
    const int src = max(min(row, nt - 1), 0);
    const uint2 w = reinterpret_cast<const uint2 *>(train + (size_t)src * kWords)[tid >> 5];
    return row < nt ? w : make_uint2(0, 0);
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

// Where a work item's results go: per-(split, query) partials for a later
// merge, or (one split only) the final idx / dist / accept rows directly.
struct ItemOut {
    uint64_t *partial;      // partial + (split * nq + q) * 2, or nullptr for direct
    int32_t *idx;           // direct: rows q of this item's query range
    int32_t *dist;
    uint8_t *accept;
    int k;
    float ratio;
};

// Final results of one query from its two best packed (distance << 32 | index).
__device__ __forceinline__ void store_final(uint64_t b1, uint64_t b2, int nt, const ItemOut &o,
                                            int q)
{
    const int d1 = b1 == kNoNeighbour ? 513 : (int)(b1 >> 32);
    const int d2 = b2 == kNoNeighbour ? 513 : (int)(b2 >> 32);
    const int j1 = b1 == kNoNeighbour ? -1 : (int)(uint32_t)b1;
    const int j2 = b2 == kNoNeighbour ? -1 : (int)(uint32_t)b2;
    o.idx[(size_t)q * o.k] = j1;
    o.dist[(size_t)q * o.k] = d1;
    if (o.k == 2) {
        o.idx[(size_t)q * o.k + 1] = j2;
        o.dist[(size_t)q * o.k + 1] = d2;
    }
    if (o.accept) o.accept[q] = (uint8_t)(nt >= 2 && (double)d1 < (double)o.ratio * (double)d2);
}

__device__ __forceinline__ void store_pair(uint64_t b1, uint64_t b2, int nq, int nt, int split,
                                           const ItemOut &o, int q)
{
    if (o.partial) {
        uint64_t *dst = o.partial + ((size_t)split * nq + q) * 2;
        dst[0] = b1;
        dst[1] = b2;
    } else {
        store_final(b1, b2, nt, o, q);
    }
}

// The 16 words of query row qn, zeros past nq, with every load issued
// before any is used: one memory round trip per row.  (Loads guarded word by
// word compile to a branch and a wait per word.)
__device__ __forceinline__ void load_query_row(const uint32_t *__restrict__ query, int nq, int qn,
                                               uint32_t (&w)[kWords])
{
    const bool real = qn < nq;
#pragma unroll
    for (int i = 0; i < kWords; ++i) w[i] = 0u;
    if (nq > 0) {
        const uint32_t *src = query + (size_t)(real ? qn : 0) * kWords;
#pragma unroll
        for (int i = 0; i < kWords; ++i) w[i] = src[i];
    }
#pragma unroll
    for (int i = 0; i < kWords; ++i) w[i] = real ? w[i] : 0u;
}

// One work item of the MFMA matcher: queries qgroup * 256 .. + 255 of
// `query` (nq rows) against train rows split * split_rows .. + split_rows - 1
// of `train` (nt rows).  All 256 threads of the workgroup take part; tbuf is
// the workgroup's 2 x 16 KB LDS staging buffer.
__device__ __forceinline__ void mfma_item(const uint32_t *__restrict__ query, int nq,
                                          const uint32_t *__restrict__ train, int nt, int qgroup,
                                          int split, int split_rows, const ItemOut &out,
                                          v4i (*tbuf)[kTileVec])
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int half = lane >> 5;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int qbase = qgroup * kQueriesPerGroup + wave * kQueriesPerWave;

    const int ntiles_all = (nt + kTileRows - 1) / kTileRows;
    const int tiles_per_split = split_rows / kTileRows;
    const int t_begin = split * tiles_per_split;
    const int t_end = min(ntiles_all, t_begin + tiles_per_split);

    // The next tile's load is issued at the start of a tile and staged at
    // its end (the query fragments leave no registers for a deeper queue).
    uint2 ld0 = make_uint2(0, 0);
    if (t_begin < t_end) ld0 = load_tile(train, nt, t_begin, tid);

    // Resident query fragments and query popcounts.
    v4i bq[kQueryBlocks][16];
    int na[kQueryBlocks];
    uint32_t qw[kQueryBlocks][kWords];
#pragma unroll
    for (int qb = 0; qb < kQueryBlocks; ++qb) load_query_row(query, nq, qbase + 32 * qb + (lane & 31), qw[qb]);
#pragma unroll
    for (int qb = 0; qb < kQueryBlocks; ++qb) {
        int pc = 0;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const uint32_t w = qw[qb][s];
            pc += __popc(w);
            bq[qb][s] = expand16_pm1((w >> (16 * half)) & 0xffffu);
        }
        na[qb] = pc;
    }

    uint32_t k1[kQueryBlocks], k2[kQueryBlocks];
#pragma unroll
    for (int qb = 0; qb < kQueryBlocks; ++qb) k1[qb] = k2[qb] = 0u;

    __syncthreads();       // the staging buffer may still be read by a previous item
    if (t_begin < t_end) stage_tile(ld0, tid, tbuf[0]);
    __syncthreads();

    // One tile: MFMAs over LDS buffer `buf`, then the top-2 update.
    auto tile_step = [&](int tile, int buf) {
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
        for (int r = 0; r < 16; r += 2) {
#pragma unroll
            for (int qb = 0; qb < kQueryBlocks; ++qb)
                insert_pair_u32(k1[qb], k2[qb], ((uint32_t)acc[qb][r] << kLocalBits) + cb[r],
                                ((uint32_t)acc[qb][r + 1] << kLocalBits) + cb[r + 1]);
        }
    };

    // Straight-line body: the load past the split reads train rows of the
    // next split or none (rows past nt load nothing and give zeros), and
    // staging into the idle buffer is harmless.
    for (int tile = t_begin; tile < t_end; ++tile) {
        const int buf = (tile - t_begin) & 1;
        const uint2 ld = load_tile(train, nt, tile + 1, tid);
        tile_step(tile, buf);
        stage_tile(ld, tid, tbuf[buf ^ 1]);
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
            store_pair(r[0], r[1], nq, nt, split, out, qn);
        }
    }
}

// The two smallest of the pairs (a1 <= a2) and (c1 <= c2).
__device__ __forceinline__ void top2_pair(uint64_t &a1, uint64_t &a2, uint64_t c1, uint64_t c2)
{
    const uint64_t lo = min(a1, c1);
    a2 = min(max(a1, c1), min(a2, c2));
    a1 = lo;
}

// ---------------------------------------------------------------------------
// MXFP4 matcher.  Same tiling as the int8 path, on the block-scaled FP4
// matrix instruction v_mfma_scale_f32_32x32x64_f8f6f4 (K = 64 per
// instruction, twice the int8 rate on gfx950).
//
// Operands.  FP4 (e2m1) holds 0 (0x0), +-0.5 (0x1 / 0x9), +-1 (0x2 / 0xa)
// and +-2 (0x4 / 0xc) exactly.  A train bit enters as 0 or c (c = 0.5, 1 or
// 2 by its place in the fragment, below) with block scale 2^0, and the query
// bit it meets as +1 / c or -1 / c (set / clear) with block scale 2^14, so
// each product is 0 or +-2^14 and the f32 sum over K = 512 is 2^14 s with
// s = |a| - Hamming(a, b) as in the int8 path, exact (|2^14 s| <= 2^23).
//
// Keys.  For tile row m the accumulator starts at c_m = 2^14 - 1 - m, so it
// ends at 2^14 s + c_m; the running top-2 of a lane is kept in the frame of
// the current tile and moved up by 32 when the next tile starts, so a key
// from split-local row jl = 32 t + m ends as 2^14 s + 2^14 - 1 - jl + 32 T
// after T tiles (T < 512): integers below 2^24 in magnitude, exact in f32.
// For a fixed query the largest key is the smallest (distance, index).  Rows
// past nt (last tile only) start at -2^25 instead, below every real key,
// which also marks "no neighbour".  Top-2 selection takes the keys two at a
// time: v_med3_f32, v_max3_f32 and v_max_f32 per two pairs.
//
// Fragment order.  Step s (0..7), lane l: the 32 elements of row l % 32 at
// K = 64 s + 32 (l / 32) + 0..31 are the bits of packed word 2 s + l / 32 of
// that row, bit 4 i + j in nibble i of dword j (16 bytes); queries use the
// same map, so the K sum covers every bit once.  In this order a train word
// becomes FP4 with four AND masks and one shift, no table: dword j keeps its
// bits where they are, as nibble bit 0, 1, 2 (values 0.5, 1, 2) for
// j = 0, 1, 2, and bit 3 (the sign) is moved down to bit 2 for j = 3, so
// c = 0.5, 1, 2, 2 by dword.
//
// Tile shape.  A wavefront holds QB blocks of 32 queries (QB = 2 or 3, from
// the tuning table), so each train fragment read from LDS feeds QB MFMAs and
// each staged tile serves 128 QB queries of the workgroup.  Measured on 63
// pairs of 20k x 20k random descriptors: 4.98 ms per batched launch with
// the table-based expansion and one-key insertion, 4.70 ms with the masks
// and two-key insertion (QB = 3, whose 256 VGPRs hold 96 of query
// fragments; QB = 2 is about 5% slower).
// ---------------------------------------------------------------------------
typedef float v16f __attribute__((ext_vector_type(16)));
typedef int v8i __attribute__((ext_vector_type(8)));

constexpr int kFp4Steps = 8;                          // K = 512 = 8 x 64
constexpr int kFp4TileVec = kFp4Steps * 64;           // 16-byte fragments per tile (512)
constexpr int kFp4ScaleTrain = 127;                   // E8M0 2^0
constexpr int kFp4ScaleQuery = 127 + 14;              // E8M0 2^14
constexpr float kFp4None = -33554432.0f;              // -2^25

// Train word -> its four FP4 dwords (0 or c per bit, c = 0.5, 1, 2, 2).
__device__ __forceinline__ uint4 fp4_train(uint32_t w)
{
    return make_uint4(w & 0x11111111u, w & 0x22222222u, w & 0x44444444u, (w >> 1) & 0x44444444u);
}

// Per nibble: `one` where m has its bit 0 set, `minus` elsewhere (m holds
// bit 0 of each nibble only, so m * 15 is a nibble mask without carries).
__device__ __forceinline__ uint32_t fp4_select(uint32_t m, uint32_t one, uint32_t minus)
{
    const uint32_t mask = m * 0xfu;
    return (one & mask) | (minus & ~mask);
}

// Query word -> its four FP4 dwords (+-1 / c per bit: +-2, +-1, +-0.5, +-0.5).
__device__ __forceinline__ uint4 fp4_query(uint32_t w)
{
    return make_uint4(fp4_select(w & 0x11111111u, 0x44444444u, 0xccccccccu),
                      fp4_select((w >> 1) & 0x11111111u, 0x22222222u, 0xaaaaaaaau),
                      fp4_select((w >> 2) & 0x11111111u, 0x11111111u, 0x99999999u),
                      fp4_select((w >> 3) & 0x11111111u, 0x11111111u, 0x99999999u));
}

// Two keys into a running top two (k1 >= k2), as insert_pair_u32 does for
// integer keys: t = med3(k1, x, y), k1 = max3(k1, x, y), k2 = max(k2, t), as
// one unit (the independent chains of the query blocks interleave; the
// instructions are written out, since the IEEE-mode fmaxf adds NaN quieting
// per operand; keys are never NaN).
__device__ __forceinline__ void insert_pair(float &k1, float &k2, float x, float y)
{
    float t;
    asm("v_med3_f32 %2, %0, %3, %4\n\t"
        "v_max3_f32 %0, %0, %3, %4\n\t"
        "v_max_f32 %1, %1, %2"
        : "+v"(k1), "+v"(k2), "=&v"(t)
        : "v"(x), "v"(y));
}

__device__ __forceinline__ v8i fp4_operand(uint4 f)
{
    v8i r = {};
    r[0] = (int)f.x;
    r[1] = (int)f.y;
    r[2] = (int)f.z;
    r[3] = (int)f.w;
    return r;
}

// Staging role of a thread: tile row tid % 32, packed words 2 (tid / 32) and
// 2 (tid / 32) + 1, i.e. step tid / 32, both lane halves.
__device__ __forceinline__ void stage_tile_fp4(uint2 w, int tid, uint4 *__restrict__ buf)
{
    const int r = tid & 31;
    const int s = tid >> 5;
    buf[s * 64 + r] = fp4_train(w.x);
    buf[s * 64 + 32 + r] = fp4_train(w.y);
}

// One (query group, train range) of the MXFP4 matcher.  Train rows
// split * split_rows .. + split_rows - 1 (split_rows <= 2^14); each lane's
// queries' best two (distance << 32 | index) are merged into best[qb].
template <int QB>
__device__ __forceinline__ void fp4_item(const uint32_t *__restrict__ query, int nq,
                                         const uint32_t *__restrict__ train, int nt, int qgroup,
                                         int split, int split_rows, uint64_t (&best)[QB][2],
                                         uint4 (*tbuf)[kFp4TileVec])
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int half = lane >> 5;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int qbase = qgroup * (kMfmaWaves * 32 * QB) + wave * (32 * QB);

    const int ntiles_all = (nt + kTileRows - 1) / kTileRows;
    const int tiles_per_split = split_rows / kTileRows;
    const int t_begin = split * tiles_per_split;
    const int t_end = min(ntiles_all, t_begin + tiles_per_split);

    // Tile loads two tiles ahead of staging, as in the int8 path.
    uint2 ld0 = make_uint2(0, 0), ra = ld0, rb = ld0;
    if (t_begin < t_end) ld0 = load_tile(train, nt, t_begin, tid);
    if (t_begin + 1 < t_end) ra = load_tile(train, nt, t_begin + 1, tid);
    if (t_begin + 2 < t_end) rb = load_tile(train, nt, t_begin + 2, tid);

    // Resident query fragments (+-1) and query popcounts.
    uint4 bq[QB][kFp4Steps];
    int na[QB];
    uint32_t qw[QB][kWords];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) load_query_row(query, nq, qbase + 32 * qb + (lane & 31), qw[qb]);
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        int pc = 0;
#pragma unroll
        for (int s = 0; s < kFp4Steps; ++s) {
            const uint32_t w0 = qw[qb][2 * s], w1 = qw[qb][2 * s + 1];
            pc += __popc(w0) + __popc(w1);
            bq[qb][s] = fp4_query(half ? w1 : w0);
        }
        na[qb] = pc;
    }

    float k1[QB], k2[QB];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) k1[qb] = k2[qb] = kFp4None;

    // Accumulator start values c_m; register r = 4 g + e holds tile row
    // m = 8 g + 4 half + e.
    v16f c0;
#pragma unroll
    for (int r = 0; r < 16; ++r) c0[r] = (float)((1 << 14) - 1 - (8 * (r >> 2) + 4 * half + (r & 3)));

    __syncthreads();       // the staging buffers may still be read for a previous range
    if (t_begin < t_end) stage_tile_fp4(ld0, tid, tbuf[0]);
    __syncthreads();

    // The MFMAs of one tile over LDS buffer `buf`.
    auto tile_mfma = [&](int buf, v16f (&acc)[QB]) {
#pragma unroll
        for (int s = 0; s < kFp4Steps; ++s) {
            const v8i a = fp4_operand(tbuf[buf][s * 64 + lane]);
#pragma unroll
            for (int qb = 0; qb < QB; ++qb)
                acc[qb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                    a, fp4_operand(bq[qb][s]), s == 0 ? c0 : acc[qb], 4, 4, 0, kFp4ScaleTrain, 0,
                    kFp4ScaleQuery);
        }
    };
    // The top-2 update with one tile's keys: the running top two move into
    // this tile's frame, then take the tile's 16 keys per query block, two
    // at a time.
    auto tile_top2 = [&](const v16f (&acc)[QB]) {
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            k1[qb] += 32.0f;
            k2[qb] += 32.0f;
        }
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) insert_pair(k1[qb], k2[qb], acc[qb][r], acc[qb][r + 1]);
        }
    };
    // Rows past nt (in the last tile only) take a key below every real one.
    auto mask_tail = [&](int tile, v16f (&acc)[QB]) {
        const int valid_rows = nt - tile * kTileRows;
        if (valid_rows < kTileRows) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (8 * (r >> 2) + 4 * half + (r & 3) >= valid_rows)
#pragma unroll
                    for (int qb = 0; qb < QB; ++qb) acc[qb][r] = kFp4None;
        }
    };
    auto tile_step = [&](int tile, int buf) {
        v16f acc[QB];
        tile_mfma(buf, acc);
        mask_tail(tile, acc);
        tile_top2(acc);
    };

    // Straight-line body, as in the int8 path.  (The first update moves the
    // empty keys up by 32 too, which keeps them below -2^24.)
    for (int tile = t_begin; tile < t_end; tile += 2) {
        tile_step(tile, 0);
        stage_tile_fp4(ra, tid, tbuf[1]);
        ra = load_tile(train, nt, tile + 3, tid);
        __syncthreads();
        if (tile + 1 >= t_end) break;
        tile_step(tile + 1, 1);
        stage_tile_fp4(rb, tid, tbuf[0]);
        rb = load_tile(train, nt, tile + 4, tid);
        __syncthreads();
    }

    // Merge the two row halves and decode
    // key = 2^14 (|a| - d) + 2^14 - 1 - jl + 32 (tiles - 1).
    const int shift = 32 * max(t_end - t_begin - 1, 0);
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        const float o1 = __shfl_xor(k1[qb], 32);
        const float o2 = __shfl_xor(k2[qb], 32);
        const float b1 = fmaxf(k1[qb], o1);
        const float b2 = fmaxf(fminf(k1[qb], o1), fmaxf(k2[qb], o2));
        uint64_t r[2];
        const float kk[2] = {b1, b2};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (kk[e] < -16777216.0f) {                  // a row past nt, or none
                r[e] = kNoNeighbour;
            } else {
                const int key = (int)kk[e] - shift;
                const uint32_t d = (uint32_t)(na[qb] - (key >> 14));
                const uint32_t j = (uint32_t)split * (uint32_t)split_rows +
                                   (uint32_t)((1 << 14) - 1 - (key & 0x3fff));
                r[e] = ((uint64_t)d << 32) | j;
            }
        }
        top2_pair(best[qb][0], best[qb][1], r[0], r[1]);
    }
}

template <int QB>
__device__ __forceinline__ void fp4_init_best(uint64_t (&best)[QB][2])
{
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) best[qb][0] = best[qb][1] = kNoNeighbour;
}

// Lanes 0..31 of each wavefront store their queries' results.
template <int QB>
__device__ __forceinline__ void fp4_store(const uint64_t (&best)[QB][2], int nq, int nt, int qgroup,
                                          int split, const ItemOut &out)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        const int qn = qgroup * (kMfmaWaves * 32 * QB) + wave * (32 * QB) + 32 * qb + (lane & 31);
        if (lane < 32 && qn < nq) store_pair(best[qb][0], best[qb][1], nq, nt, split, out, qn);
    }
}

// ---------------------------------------------------------------------------
// Popcount matcher.  One query per lane; grid (query blocks of 256, splits).
// key = (d << 21) | jl with d <= 512, jl < 2^21 - 1, so ~0u means "none".
// ---------------------------------------------------------------------------
__device__ __forceinline__ void popcount_item(const uint32_t *__restrict__ query, int nq,
                                              const uint32_t *__restrict__ train, int nt,
                                              int qgroup, int split, int split_rows,
                                              const ItemOut &out)
{
    const int qn = qgroup * 256 + threadIdx.x;
    const int j0 = split * split_rows;
    const int j1 = min(nt, j0 + split_rows);

    uint32_t q[kWords];
    load_query_row(query, nq, qn, q);

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
        uint64_t r[2];
#pragma unroll
        for (int e = 0; e < 2; ++e)
            r[e] = kk[e] == ~0u ? kNoNeighbour
                                : (((uint64_t)(kk[e] >> kLocalBits) << 32) |
                                   (uint32_t)(j0 + (int)(kk[e] & kLocalMask)));
        store_pair(r[0], r[1], nq, nt, split, out, qn);
    }
}

// ---------------------------------------------------------------------------
// Merge per-split partials (64-bit keys: distance << 32 | global index, so the
// integer order is the lexicographic one) and apply the ratio test exactly:
// a float32 ratio times an integer <= 512 is exact in double.
// ---------------------------------------------------------------------------
// Arguments of the split matchers.  nsplit == 1: results go straight to
// idx / dist / accept; otherwise per-(split, query) partials for the merge
// kernel.
struct SplitArgs {
    const uint32_t *query;
    const uint32_t *train;
    int nq, nt, split_rows, nsplit;
    uint64_t *partial;
    int k;
    float ratio;
    int32_t *idx, *dist;
    uint8_t *accept;
};

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m)
{
    const uint32_t lo = __shfl_xor((uint32_t)v, m), hi = __shfl_xor((uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// Four lanes per query: lane g of a query reads splits g, g + 4, ... (all
// loads in flight), then two shuffle rounds combine the four top-2 pairs.
constexpr int kMergeLanes = 4;

__global__ __launch_bounds__(256) void knn_merge_kernel(const uint64_t *__restrict__ partial, int nq,
                                                        int nsplit, int nt, int k, float ratio,
                                                        int32_t *__restrict__ idx,
                                                        int32_t *__restrict__ dist,
                                                        uint8_t *__restrict__ accept)
{
    const int g = threadIdx.x & (kMergeLanes - 1);
    const int q = blockIdx.x * (256 / kMergeLanes) + threadIdx.x / kMergeLanes;
    const bool real = q < nq;
    uint64_t b1 = kNoNeighbour, b2 = kNoNeighbour;
    for (int s0 = g; s0 < nsplit; s0 += 4 * kMergeLanes) {
        ulonglong2 v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int sp = s0 + kMergeLanes * i;
            v[i] = real && sp < nsplit
                       ? reinterpret_cast<const ulonglong2 *>(partial)[(size_t)sp * nq + q]
                       : make_ulonglong2(kNoNeighbour, kNoNeighbour);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) top2_pair(b1, b2, v[i].x, v[i].y);
    }
#pragma unroll
    for (int m = 1; m < kMergeLanes; m <<= 1) top2_pair(b1, b2, shfl_xor_u64(b1, m), shfl_xor_u64(b2, m));
    if (real && g == 0) store_final(b1, b2, nt, ItemOut{nullptr, idx, dist, accept, k, ratio}, q);
}

__global__ __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void
knn_mfma_kernel(SplitArgs a)
{
    __shared__ v4i tbuf[2][kTileVec];
    const ItemOut direct{nullptr, a.idx, a.dist, a.accept, a.k, a.ratio};
    const ItemOut part{a.partial, nullptr, nullptr, nullptr, 2, 0.f};
    mfma_item(a.query, a.nq, a.train, a.nt, blockIdx.x, blockIdx.y, a.split_rows,
              a.nsplit == 1 ? direct : part, tbuf);
}

template <int QB>
__global__ __launch_bounds__(kMfmaThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void
knn_fp4_kernel(SplitArgs a)
{
    __shared__ uint4 tbuf[2][kFp4TileVec];
    const ItemOut direct{nullptr, a.idx, a.dist, a.accept, a.k, a.ratio};
    const ItemOut part{a.partial, nullptr, nullptr, nullptr, 2, 0.f};
    uint64_t best[QB][2];
    fp4_init_best(best);
    fp4_item<QB>(a.query, a.nq, a.train, a.nt, blockIdx.x, blockIdx.y, a.split_rows, best, tbuf);
    fp4_store(best, a.nq, a.nt, blockIdx.x, blockIdx.y, a.nsplit == 1 ? direct : part);
}

__global__ __launch_bounds__(256) void knn_popcount_kernel(SplitArgs a)
{
    const ItemOut direct{nullptr, a.idx, a.dist, a.accept, a.k, a.ratio};
    const ItemOut part{a.partial, nullptr, nullptr, nullptr, 2, 0.f};
    popcount_item(a.query, a.nq, a.train, a.nt, blockIdx.x, blockIdx.y, a.split_rows,
                  a.nsplit == 1 ? direct : part);
}

// ---------------------------------------------------------------------------
// Batched matching: many (query range, train range, output range) pairs in
// one persistent launch.  Work item = (pair, query group) over the pair's
// whole train range, so results are final and go straight to the outputs.
// A one-block setup kernel validates the pairs, lays their items out and
// resets the atomic work counter (so the sequence is replayable from a HIP
// graph without memset nodes); a fill kernel writes the item -> pair map;
// persistent workgroups then claim items through the counter.
//
// Items are laid out longest first (an item's time grows with its pair's
// train rows): pairs go to 256 cost classes, 8 per doubling of the train
// tile count, and the classes are laid out in decreasing order, so that the
// last items claimed are the shortest and the workgroups finish together.
// The order within a class follows the atomics and does not matter: every
// item writes its own outputs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool pair_ok(const PairEntry &e, int64_t query_rows, int64_t train_rows,
                                        int64_t out_rows)
{
    return e.nq >= 0 && e.nt >= 0 && e.nq <= kMaxRows && e.nt <= kMaxSplitRows &&
           e.query_first >= 0 && e.query_first + e.nq <= query_rows &&
           (e.nt == 0 || (e.train_first >= 0 && e.train_first + e.nt <= train_rows)) &&
           e.out_first >= 0 && e.out_first + e.nq <= out_rows;
}

// Cost class of a pair, 0 for the longest items: 255 - floor(8 log2(tiles + 1))
// with the fraction taken from the three bits after the leading one.
__device__ __forceinline__ int cost_class(int64_t nt)
{
    nt = max((int64_t)0, min(nt, (int64_t)kMaxSplitRows));          // invalid pairs: any class
    const uint32_t x = (uint32_t)((nt + kTileRows - 1) / kTileRows) + 1u;   // <= 2^16
    const int lz = __clz((int)x);
    const uint32_t frac = ((x << lz) >> 28) & 7u;
    return 255 - min(255, 8 * (31 - lz) + (int)frac);
}

__global__ __launch_bounds__(256) void knn_batch_setup_kernel(
    const PairEntry *__restrict__ pairs, int n_pairs, int64_t query_rows, int64_t train_rows,
    int64_t out_rows, int64_t item_capacity, int group, PairInfo *__restrict__ info,
    BatchState *__restrict__ st, uint32_t *__restrict__ flags)
{
    __shared__ unsigned long long classes[256];
    __shared__ int bad_s;
    const int tid = threadIdx.x;
    classes[tid] = 0;
    if (tid == 0) bad_s = 0;
    __syncthreads();
    // Items per class; each pair's rank in its class goes to info[p].item_first.
    bool bad = false;
    for (int p = tid; p < n_pairs; p += 256) {
        const PairEntry e = pairs[p];
        const bool ok = pair_ok(e, query_rows, train_rows, out_rows);
        bad |= !ok;
        const unsigned long long groups = ok ? (unsigned long long)((e.nq + group - 1) / group) : 0ull;
        info[p].item_first = (int64_t)atomicAdd(&classes[cost_class(e.nt)], groups);
    }
    if (bad) atomicOr(&bad_s, 1);
    __syncthreads();
    // Inclusive scan of the 256 class totals (Hillis-Steele); class c's
    // items start at the exclusive prefix.
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned long long v = tid >= off ? classes[tid - off] : 0ull;
        __syncthreads();
        classes[tid] += v;
        __syncthreads();
    }
    const int64_t total = (int64_t)classes[255];
    // The item map holds item_capacity entries, enough for every batch whose
    // pairs' output ranges do not overlap; a batch that needs more is not run.
    const bool overflow = total > item_capacity;
    for (int p = tid; p < n_pairs; p += 256) {
        const PairEntry e = pairs[p];
        const bool ok = pair_ok(e, query_rows, train_rows, out_rows);
        const int c = cost_class(e.nt);
        const int64_t groups = ok && !overflow ? (e.nq + group - 1) / group : 0;
        info[p].item_first += (int64_t)(c > 0 ? classes[c - 1] : 0ull);
        info[p].qgroups = (int32_t)groups;
        info[p].valid = ok && !overflow;
    }
    if ((bad_s || overflow) && tid == 0) atomicOr(flags, kFlagBadPair);
    if (tid == 255) {
        st->items = overflow ? 0 : total;
        st->next_item = 0;
    }
}

__global__ __launch_bounds__(256) void knn_batch_fill_kernel(const PairInfo *__restrict__ info,
                                                             int n_pairs,
                                                             int32_t *__restrict__ item_pair)
{
    for (int p = blockIdx.x; p < n_pairs; p += gridDim.x) {
        const PairInfo pi = info[p];
        for (int i = threadIdx.x; i < pi.qgroups; i += 256) item_pair[pi.item_first + i] = p;
    }
}

// Claims the next work item for the whole workgroup; -1 when none is left.
__device__ __forceinline__ int64_t claim_item(BatchState *__restrict__ st, int *slot)
{
    if (threadIdx.x == 0) {
        const uint32_t it = atomicAdd(&st->next_item, 1u);
        *slot = (int64_t)it < st->items ? (int)it : -1;
    }
    __syncthreads();
    const int it = *slot;
    __syncthreads();
    return it;
}

enum class BatchKind { kPopcount, kMfmaI8, kMfmaFp4 };

template <BatchKind kKind, int QB>
__device__ __forceinline__ void batch_loop(const uint32_t *__restrict__ query,
                                           const uint32_t *__restrict__ train,
                                           const PairEntry *__restrict__ pairs,
                                           const PairInfo *__restrict__ info,
                                           const int32_t *__restrict__ item_pair,
                                           BatchState *__restrict__ st, int k, float ratio,
                                           int32_t *__restrict__ idx, int32_t *__restrict__ dist,
                                           uint8_t *__restrict__ accept, void *tbuf,
                                           int *slot, int n_pairs)
{
    for (;;) {
        const int item = claim_item(st, slot);
        if (item < 0) break;
        const int p = item_pair[item];
        if (p < 0 || p >= n_pairs) continue;     // cannot happen for a map written by the fill kernel
        const PairEntry e = pairs[p];
        const int qgroup = (int)(item - info[p].item_first);
        const int nt = (int)e.nt;
        const ItemOut out{nullptr, idx + e.out_first * k, dist + e.out_first * k,
                          accept ? accept + e.out_first : nullptr, k, ratio};
        const uint32_t *q = query + (size_t)e.query_first * kWords;
        const uint32_t *t = train + (size_t)(nt ? e.train_first : 0) * kWords;
        if constexpr (kKind == BatchKind::kMfmaFp4) {
            // The pair's whole train range in ranges of at most 2^14 rows
            // (the MXFP4 keys' index field), merged in registers.
            uint64_t best[QB][2];
            fp4_init_best(best);
            const int ranges = max(1, (nt + (int)kFp4MaxSplitRows - 1) / (int)kFp4MaxSplitRows);
            for (int r = 0; r < ranges; ++r)
                fp4_item<QB>(q, (int)e.nq, t, nt, qgroup, r, (int)kFp4MaxSplitRows, best,
                             reinterpret_cast<uint4 (*)[kFp4TileVec]>(tbuf));
            fp4_store(best, (int)e.nq, nt, qgroup, 0, out);
        } else {
            const int split_rows = max(kTileRows, (nt + kTileRows - 1) / kTileRows * kTileRows);
            if constexpr (kKind == BatchKind::kMfmaI8)
                mfma_item(q, (int)e.nq, t, nt, qgroup, 0, split_rows, out,
                          reinterpret_cast<v4i (*)[kTileVec]>(tbuf));
            else
                popcount_item(q, (int)e.nq, t, nt, qgroup, 0, split_rows, out);
        }
    }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void
knn_batch_mfma_kernel(const uint32_t *__restrict__ query, const uint32_t *__restrict__ train,
                      const PairEntry *__restrict__ pairs, int n_pairs,
                      const PairInfo *__restrict__ info,
                      const int32_t *__restrict__ item_pair, BatchState *__restrict__ st, int k,
                      float ratio, int32_t *__restrict__ idx, int32_t *__restrict__ dist,
                      uint8_t *__restrict__ accept)
{
    __shared__ v4i tbuf[2][kTileVec];
    __shared__ int slot;
    batch_loop<BatchKind::kMfmaI8, kQueryBlocks>(query, train, pairs, info, item_pair, st, k, ratio,
                                                 idx, dist, accept, tbuf, &slot, n_pairs);
}

template <int QB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void
knn_batch_fp4_kernel(const uint32_t *__restrict__ query, const uint32_t *__restrict__ train,
                     const PairEntry *__restrict__ pairs, int n_pairs,
                     const PairInfo *__restrict__ info, const int32_t *__restrict__ item_pair,
                     BatchState *__restrict__ st, int k, float ratio, int32_t *__restrict__ idx,
                     int32_t *__restrict__ dist, uint8_t *__restrict__ accept)
{
    __shared__ uint4 tbuf[2][kFp4TileVec];
    __shared__ int slot;
    batch_loop<BatchKind::kMfmaFp4, QB>(query, train, pairs, info, item_pair, st, k, ratio, idx,
                                        dist, accept, tbuf, &slot, n_pairs);
}

__global__ __launch_bounds__(256) void knn_batch_popcount_kernel(
    const uint32_t *__restrict__ query, const uint32_t *__restrict__ train,
    const PairEntry *__restrict__ pairs, int n_pairs, const PairInfo *__restrict__ info,
    const int32_t *__restrict__ item_pair, BatchState *__restrict__ st, int k, float ratio,
    int32_t *__restrict__ idx, int32_t *__restrict__ dist, uint8_t *__restrict__ accept)
{
    __shared__ int slot;
    batch_loop<BatchKind::kPopcount, 1>(query, train, pairs, info, item_pair, st, k, ratio, idx,
                                        dist, accept, nullptr, &slot, n_pairs);
}

}  // namespace

int queries_per_group(SplitKernel which, const KnnShape &shape)
{
    return which == SplitKernel::kMfmaFp4 ? kMfmaWaves * 32 * shape.fp4_query_blocks : 256;
}

hipError_t launch_knn_split(const KnnSplitArgs &a, SplitKernel which, hipStream_t stream)
{
    const SplitArgs k{a.query, a.train, (int)a.plan.nq, (int)a.plan.nt, (int)a.plan.split_rows,
                      a.plan.nsplit, a.partial, a.k, a.ratio, a.idx, a.dist, a.accept};
    const int64_t group = queries_per_group(which, a.shape);
    const int64_t qgroups = (a.plan.nq + group - 1) / group;
    const dim3 grid((unsigned)qgroups, (unsigned)a.plan.nsplit);
    if (which == SplitKernel::kMfmaI8)
        hipLaunchKernelGGL(knn_mfma_kernel, grid, dim3(kMfmaThreads), 0, stream, k);
    else if (which == SplitKernel::kMfmaFp4 && a.shape.fp4_query_blocks == 3)
        hipLaunchKernelGGL(knn_fp4_kernel<3>, grid, dim3(kMfmaThreads), 0, stream, k);
    else if (which == SplitKernel::kMfmaFp4)
        hipLaunchKernelGGL(knn_fp4_kernel<2>, grid, dim3(kMfmaThreads), 0, stream, k);
    else
        hipLaunchKernelGGL(knn_popcount_kernel, grid, dim3(256), 0, stream, k);
    return hipGetLastError();
}

hipError_t launch_knn_merge(const KnnSplitArgs &a, hipStream_t stream)
{
    const int64_t per_block = 256 / kMergeLanes;
    const int64_t blocks = (a.plan.nq + per_block - 1) / per_block;
    hipLaunchKernelGGL(knn_merge_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a.partial,
                       (int)a.plan.nq, a.plan.nsplit, (int)a.plan.nt, a.k, a.ratio, a.idx, a.dist,
                       a.accept);
    return hipGetLastError();
}

hipError_t launch_knn_batch(const BatchArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(knn_batch_setup_kernel, dim3(1), dim3(256), 0, stream, a.pairs, a.n_pairs,
                       a.query_rows, a.train_rows, a.out_rows, a.item_capacity,
                       queries_per_group(a.kind, a.shape), a.info, a.state, a.flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int fill_blocks = a.n_pairs < 4096 ? a.n_pairs : 4096;
    hipLaunchKernelGGL(knn_batch_fill_kernel, dim3(fill_blocks), dim3(256), 0, stream, a.info,
                       a.n_pairs, a.item_pair);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int blocks =
        a.num_cus * (a.kind == SplitKernel::kPopcount ? 8 : a.shape.batch_groups_per_cu);
    if (a.kind == SplitKernel::kMfmaI8)
        hipLaunchKernelGGL(knn_batch_mfma_kernel, dim3(blocks), dim3(256), 0, stream, a.query,
                           a.train, a.pairs, a.n_pairs, a.info, a.item_pair, a.state, a.k, a.ratio,
                           a.idx, a.dist, a.accept);
    else if (a.kind == SplitKernel::kMfmaFp4 && a.shape.fp4_query_blocks == 3)
        hipLaunchKernelGGL(knn_batch_fp4_kernel<3>, dim3(blocks), dim3(256), 0, stream, a.query,
                           a.train, a.pairs, a.n_pairs, a.info, a.item_pair, a.state, a.k, a.ratio,
                           a.idx, a.dist, a.accept);
    else if (a.kind == SplitKernel::kMfmaFp4)
        hipLaunchKernelGGL(knn_batch_fp4_kernel<2>, dim3(blocks), dim3(256), 0, stream, a.query,
                           a.train, a.pairs, a.n_pairs, a.info, a.item_pair, a.state, a.k, a.ratio,
                           a.idx, a.dist, a.accept);
    else
        hipLaunchKernelGGL(knn_batch_popcount_kernel, dim3(blocks), dim3(256), 0, stream, a.query,
                           a.train, a.pairs, a.n_pairs, a.info, a.item_pair, a.state, a.k, a.ratio,
                           a.idx, a.dist, a.accept);
    return hipGetLastError();
}

}  // namespace latch
