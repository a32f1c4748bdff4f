// C ABI of the LATCH library: handle, argument checks, tables, workspace and
// launches.  Every call only enqueues on the caller's stream (see latch.h).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/latch.h"
#include "internal.h"

using namespace latch;

struct latch_ctx {
    int device = 0;
    int num_cus = 0;
    int2 *rot_dev = nullptr;           // [4096] {cos_q14, sin_q14}
    uint2 *trip_off_dev = nullptr;     // [512] by slot: LDS byte offsets of the three patches
    uint32_t *unperm_dev = nullptr;    // [128] output-bit slots per (wavefront, lane)
    uint16_t *gather_dev = nullptr;    // [kGatherClasses][kGatherClassEntries] window gather order
    uint32_t *flags_dev = nullptr;     // sticky error word
    // Weighted geometry (latch_create_geometry); window 0 runs the default kernel.
    int window = 0;
    uint2 *wtrip_dev = nullptr;        // [512] by slot: weighted-kernel patch offsets
    uint32_t *wunperm_dev = nullptr;   // [256] per (wavefront, lane): slots of its two output bits
    uint2 *dense_off_dev = nullptr;    // [512] in triplet order: dense-kernel texture offsets
    WeightRows weights = {};
    uint8_t *ws = nullptr;             // grow-only workspace
    size_t ws_bytes = 0;
    uint8_t *scratch = nullptr;        // this device's copy of the static scratch array
    latch_tuning tuning;               // LATCH_PATH_AUTO table and split targets
    std::string last_error;
    // Event timing (latch_timing_enable).
    bool timing = false;
    struct Timed {
        const char *name;
        hipEvent_t start, stop;
    };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> event_pool;
};

namespace {

int fail(latch_handle h, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));

int fail(latch_handle h, int code, const char *fmt, ...)
{
    if (h) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        h->last_error = buf;
    }
    return code;
}

int hip_fail(latch_handle h, hipError_t e, const char *what)
{
    return fail(h, e == hipErrorOutOfMemory ? LATCH_ENOMEM : LATCH_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

// Rule step 2: the first octant from libm, the rest from the exact
// symmetries cos(90 - a) = sin(a) and (C, S)(a + 90) = (-S, C)(a).
void rotation_table(int16_t *c, int16_t *s)
{
    const double step = M_PI / 2048.0;
    for (int a = 0; a <= 512; ++a) {
        c[a] = (int16_t)std::lrint(16384.0 * std::cos(step * a));
        s[a] = (int16_t)std::lrint(16384.0 * std::sin(step * a));
    }
    for (int a = 513; a < 1024; ++a) {
        c[a] = s[1024 - a];
        s[a] = c[1024 - a];
    }
    for (int a = 1024; a < kBins; ++a) {
        c[a] = (int16_t)(-s[a - 1024]);
        s[a] = c[a - 1024];
    }
}

// Gather order of the extraction kernel.  Rounding half away from zero is
// odd, so positions (u, v) and (-u, -v) sample at offsets (ox, oy) and
// (-ox, -oy), and the unrounded offsets of (u + 1, v) are those of (u, v)
// plus s C and s S: the kernel takes positions in chains (u, v), (u + 1, v),
// (-u, -v), (-u - 1, -v), with two rounded offset pairs per chain.  Over
// [-24, 24]^2 (the window and one more row and column, which nothing reads)
// the first members run over rows v = 1..24 with u = -24, -22, .., 22 and 23
// (the last chain overlaps the one before it at (23, v)), and over row 0
// with u = 0, 2, .., 22 and 23: 613 chains, whose mirrors cover the other
// half.  For angle class c (bins 32 c .. 32 c + 31), with (C, S) the cosine
// and sine of the class's middle angle, position (u, v) samples image row
// offset about s (S u + C v) and column offset s (C u - S v) at scale s.
// Chains are sorted by the band floor(4 (S u + C v)) of their first member
// (a quarter row at unit scale), then by its column offset (ties by
// position), so that the lanes of a load sample nearby image bytes and the
// mirrored members form the mirrored band.  Sorted chain k goes to thread
// k % 128, slot k / 128; the 27 slots left over repeat the centre's chain
// (0, 0), (1, 0).  Entry: u & 0xff | (v & 0xff) << 8; slots 0..3 of thread t
// at 4 t + slot, slot 4 at 512 + t (one 8-byte and one 2-byte load per
// thread).
std::vector<uint16_t> gather_order()
{
    constexpr int kThreads = 2 * 64;
    std::vector<uint16_t> table((size_t)kGatherClasses * kGatherClassEntries, 0);
    std::vector<std::pair<int, int>> units;                      // first members
    for (int v = 0; v <= kHalf; ++v) {
        for (int u = v > 0 ? -kHalf : 0; u < kHalf - 1; u += 2) units.emplace_back(u, v);
        units.emplace_back(kHalf - 1, v);                        // (23, v), (24, v)
    }
    const int n = (int)units.size();                             // 24 * 25 + 13 = 613
    std::vector<int> idx(n);
    std::vector<double> row(n), col(n);
    for (int c = 0; c < kGatherClasses; ++c) {
        const double a = 2.0 * M_PI * (32.0 * c + 16.0) / kBins;
        const double cs = std::cos(a), sn = std::sin(a);
        for (int p = 0; p < n; ++p) {
            const int u = units[p].first, v = units[p].second;
            idx[p] = p;
            row[p] = std::floor(4.0 * (sn * u + cs * v));
            col[p] = cs * u - sn * v;
        }
        std::sort(idx.begin(), idx.end(), [&](int x, int y) {
            if (row[x] != row[y]) return row[x] < row[y];
            if (col[x] != col[y]) return col[x] < col[y];
            return x < y;
        });
        for (int k = 0; k < kThreads * kGatherChains; ++k) {
            const int p = k < n ? idx[k] : 0;                    // units[0]: the centre's chain
            const int u = units[p].first, v = units[p].second;
            const int t = k % kThreads, m = k / kThreads;
            const int at = m < kGatherHeadChains ? kGatherHeadChains * t + m
                                                 : kGatherHeadChains * kThreads + t;
            table[(size_t)c * kGatherClassEntries + at] = (uint16_t)((u & 0xff) | ((v & 0xff) << 8));
        }
    }
    static_assert(24 * 25 + 13 <= kThreads * kGatherChains, "chains per thread");
    static_assert(kGatherChains == kGatherHeadChains + 1, "one chain after the head");
    return table;
}

// LDS byte offset of the top-left byte of the 7 x 7 patch centred on (r, c):
// the quadword of the copy that holds its first row (see internal.h).
uint32_t patch_offset(int r, int c)
{
    const int x = c - kPatchR, y = r - kPatchR;
    if (x < 8 * kCopyQwords)
        return (uint32_t)((x & 7) * kCopyBytes + y * kCopyRowBytes + 8 * (x >> 3));
    return (uint32_t)(kEdgeBase + 8 * (x - 8 * kCopyQwords) + y * kCopyRowBytes + 8 * (kCopyQwords - 1));
}

// Slot assignment of the extraction kernels.  Wavefront w evaluates
// `per_wave` triplets (members 0 .. per_wave - 1 of toff[per_wave w ..]) in
// rounds of 64 lanes; slot 64 r + l is lane l of round r.  On gfx950 (measured
// with a probe over random and structured address patterns):
//  * a ds_read_b64 is served 32 lanes at a time over 64 dword banks, so its
//    32-lane halves read without conflicts when their quadword addresses
//    differ mod 32;
//  * a ds_read2_b64 is served 16 lanes and one address at a time over 32
//    banks, so its 16-lane quarters read without conflicts when their
//    quadword addresses differ mod 16.
// `group` (lanes served together) and `cols` (quadword banks) name the
// model of the kernel's row reads.  Every patch row read of a lane is its
// patch offset plus a uniform row offset, so the bank of all rows follows
// from the patch offset.  A deterministic annealing search over swaps puts
// triplets into the lane groups of a wavefront so that, per group and per
// patch (anchor, companion 1, companion 2), the largest number of lanes
// sharing a bank is as small as it gets.  slot_of[per_wave w + i] is the
// slot (within its wavefront) of member i; results never depend on it, only
// speed does.
void search_slots(const uint2 *toff, int waves, int per_wave, int group, int cols, uint8_t *slot_of)
{
    constexpr int kIters = 3000000;
    for (int w = 0; w < waves; ++w) {
        std::vector<std::array<int, 3>> col(per_wave);
        for (int i = 0; i < per_wave; ++i) {
            const uint2 o = toff[per_wave * w + i];
            const uint32_t off[3] = {o.x & 0xffffu, o.x >> 16, o.y};
            for (int k = 0; k < 3; ++k) col[i][k] = (int)((off[k] >> 3) & (uint32_t)(cols - 1));
        }
        std::vector<int> group_of(per_wave);
        int cnt[16][3][32];
        std::memset(cnt, 0, sizeof cnt);
        for (int i = 0; i < per_wave; ++i) {
            group_of[i] = i / group;
            for (int k = 0; k < 3; ++k) ++cnt[group_of[i]][k][col[i][k]];
        }
        auto gmax = [&](int g, int k) {
            int m = 0;
            for (int c = 0; c < cols; ++c) m = cnt[g][k][c] > m ? cnt[g][k][c] : m;
            return m;
        };
        uint32_t rs = 0x9e3779b9u + (uint32_t)w;
        auto rnd = [&]() {
            rs ^= rs << 13;
            rs ^= rs >> 17;
            rs ^= rs << 5;
            return rs;
        };
        for (int it = 0; it < kIters; ++it) {
            const int i = (int)(rnd() % (uint32_t)per_wave), j = (int)(rnd() % (uint32_t)per_wave);
            const int G = group_of[i], H = group_of[j];
            if (G == H) continue;
            int before = 0, after = 0, sq = 0;
            for (int k = 0; k < 3; ++k) before += gmax(G, k) + gmax(H, k);
            for (int k = 0; k < 3; ++k) {
                const int a = col[i][k], b = col[j][k];
                if (a == b) continue;
                sq += 2 * (cnt[G][k][b] - cnt[G][k][a] + 1) + 2 * (cnt[H][k][a] - cnt[H][k][b] + 1);
                --cnt[G][k][a];
                ++cnt[G][k][b];
                --cnt[H][k][b];
                ++cnt[H][k][a];
            }
            for (int k = 0; k < 3; ++k) after += gmax(G, k) + gmax(H, k);
            // Objective: the summed largest bank multiplicity, then the sum of
            // squared counts; worse moves pass with a probability that
            // shrinks to zero over the search.
            const int d = 64 * (after - before) + sq;
            const double temp = 40.0 * (1.0 - (double)it / kIters);
            const bool accept =
                d <= 0 || (temp > 0.5 && (double)(rnd() & 0xffffu) < 65536.0 * std::exp(-d / temp));
            if (accept) {
                group_of[i] = H;
                group_of[j] = G;
            } else {
                for (int k = 0; k < 3; ++k) {
                    const int a = col[i][k], b = col[j][k];
                    if (a == b) continue;
                    ++cnt[G][k][a];
                    --cnt[G][k][b];
                    ++cnt[H][k][b];
                    --cnt[H][k][a];
                }
            }
        }
        // Group g = (64 / group) r + h is lanes group h .. group (h + 1) - 1
        // of round r.
        const int per_round = 64 / group;
        int fill[16] = {0};
        for (int i = 0; i < per_wave; ++i) {
            const int g = group_of[i];
            slot_of[per_wave * w + i] = (uint8_t)(64 * (g / per_round) + group * (g % per_round) + fill[g]++);
        }
    }
}

// search_slots takes a few hundred milliseconds; its result depends only on
// the offsets, so it is kept per process for each offset table.
void assign_slots(const uint2 *toff, int waves, int per_wave, int group, int cols, uint8_t *slot_of)
{
    static std::mutex mu;
    static std::map<std::vector<uint32_t>, std::vector<uint8_t>> cache;
    const int n = waves * per_wave;
    std::vector<uint32_t> key;
    key.reserve(2 * n + 4);
    key.push_back((uint32_t)waves);
    key.push_back((uint32_t)per_wave);
    key.push_back((uint32_t)group);
    key.push_back((uint32_t)cols);
    for (int i = 0; i < n; ++i) {
        key.push_back(toff[i].x);
        key.push_back(toff[i].y);
    }
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            std::memcpy(slot_of, it->second.data(), (size_t)n);
            return;
        }
    }
    search_slots(toff, waves, per_wave, group, cols, slot_of);
    std::lock_guard<std::mutex> lock(mu);
    cache.emplace(std::move(key), std::vector<uint8_t>(slot_of, slot_of + n));
}

// Work calls never allocate or wait: a call whose need exceeds the handle's
// workspace fails before it enqueues anything (latch_reserve sizes it).
int check_workspace(latch_handle h, size_t need, const char *call)
{
    if (need <= h->ws_bytes) return LATCH_OK;
    return fail(h, LATCH_EWORKSPACE,
                "%s needs %zu workspace bytes and the handle holds %zu: call latch_reserve first",
                call, need, h->ws_bytes);
}

// Table uploads of handle creation: host arrays copied (or, with a null
// source, zero-filled) on a private stream, waiting for that stream only.
struct Upload {
    void *dst;
    const void *src;
    size_t bytes;
};

hipError_t upload(const Upload *u, int n)
{
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    for (int i = 0; i < n && e == hipSuccess; ++i)
        e = u[i].src ? hipMemcpyAsync(u[i].dst, u[i].src, u[i].bytes, hipMemcpyHostToDevice, s)
                     : hipMemsetAsync(u[i].dst, 0, u[i].bytes, s);
    if (s) {
        const hipError_t e2 = hipStreamSynchronize(s);
        if (e == hipSuccess) e = e2;
        (void)hipStreamDestroy(s);
    }
    return e;
}

hipEvent_t pool_event(latch_handle h)
{
    if (!h->event_pool.empty()) {
        hipEvent_t e = h->event_pool.back();
        h->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs one launch, bracketed by events when timing is on.
template <typename F>
hipError_t timed_launch(latch_handle h, const char *name, hipStream_t stream, F &&launch)
{
    if (!h->timing) return launch();
    latch_ctx::Timed t{name, pool_event(h), pool_event(h)};
    if (!t.start || !t.stop) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(t.start, stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(t.stop, stream);
    if (e != hipSuccess) return e;
    h->timed.push_back(t);
    return hipSuccess;
}

void release_timed(latch_handle h)
{
    for (auto &t : h->timed) {
        h->event_pool.push_back(t.start);
        h->event_pool.push_back(t.stop);
    }
    h->timed.clear();
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Train splits: enough (query group, split) workgroups to fill every CU
// once (by default two MFMA or eight popcount workgroups per CU),
// at least 8 tiles (256 rows) per split, split-local indices below 2^21 - 1.
int size_bucket(int64_t n)
{
    int b = 0;
    while (b < 7 && (n >> (2 * (b + 1))) > 0) ++b;
    return b;
}

void default_tuning(latch_tuning *t)
{
    std::memset(t, 0, sizeof *t);
    std::memset(t->path, LATCH_PATH_MFMA_FP4, sizeof t->path);
    t->batch_path = LATCH_PATH_MFMA_FP4;
    t->fp4_query_blocks = 3;
    t->mfma_groups_per_cu = 2;
    t->popcount_groups_per_cu = 8;
    t->batch_groups_per_cu = 2;
}

KnnShape knn_shape(const latch_tuning &t)
{
    KnnShape s;
    s.fp4_query_blocks = t.fp4_query_blocks;
    s.batch_groups_per_cu = t.batch_groups_per_cu;
    return s;
}

SplitKernel split_kernel(int path)
{
    return path == LATCH_PATH_MFMA       ? SplitKernel::kMfmaI8
           : path == LATCH_PATH_MFMA_FP4 ? SplitKernel::kMfmaFp4
                                         : SplitKernel::kPopcount;
}

// Split plan of a single-pair call.  The base choice fills the GPU's
// workgroup slots once (slots / query groups splits), raised to what the
// split-local index needs and capped at 8 tiles per split.  Work items
// (query group, split) then run in rounds of `slots`, each costing about its
// split's tiles; when the base count leaves the last round partly empty (the
// index raised it, or the query groups alone exceed the slots), a larger
// count can spread the same tiles over fuller rounds.  Over counts up to 4x
// the base (at most 512 more), within `partial_cap` bytes of partials, the
// smallest count whose rounds x tiles per split is within 2% of the least is
// taken (more splits also mean more merge work and partials), unless the
// base itself is.
KnnPlan plan_knn(int64_t nq, int64_t nt, int path, int num_cus, const latch_tuning &tune,
                 size_t partial_cap)
{
    KnnPlan p;
    p.nq = nq;
    p.nt = nt;
    const int64_t tiles = (nt + kTileRows - 1) / kTileRows;
    if (tiles == 0) {
        p.nsplit = 1;
        p.split_rows = kTileRows;
        return p;
    }
    const int64_t group = queries_per_group(split_kernel(path), knn_shape(tune));
    const int64_t qgroups = (nq + group - 1) / group;
    const int64_t slots = (int64_t)num_cus * (path == LATCH_PATH_POPCOUNT ? tune.popcount_groups_per_cu
                                                                        : tune.mfma_groups_per_cu);
    int64_t nsplit = qgroups >= slots ? 1 : slots / qgroups;
    const int64_t max_by_size = (tiles + 7) / 8;
    if (nsplit > max_by_size) nsplit = max_by_size;
    if (nsplit < 1) nsplit = 1;
    const int64_t max_rows = path == LATCH_PATH_MFMA_FP4 ? kFp4MaxSplitRows : kMaxSplitRows;
    const int64_t min_by_index = (nt + max_rows - 1) / max_rows;
    if (nsplit < min_by_index) nsplit = min_by_index;
    if (nsplit > kMaxSplits) nsplit = kMaxSplits;
    auto tiles_per = [&](int64_t n) { return (tiles + n - 1) / n; };
    auto cost = [&](int64_t n) {                       // rounds x tiles per split
        const int64_t tps = tiles_per(n), used = (tiles + tps - 1) / tps;
        return (qgroups * used + slots - 1) / slots * tps;
    };
    const int64_t n_hi = std::min({(int64_t)kMaxSplits, std::max(nsplit, max_by_size), 4 * nsplit + 8,
                                   nsplit + 512});
    const int64_t base_cost = cost(nsplit);
    int64_t least = base_cost, top = nsplit;
    for (int64_t n = nsplit + 1; n <= n_hi; ++n) {
        if ((size_t)n * (size_t)nq * 2 * sizeof(uint64_t) > partial_cap) break;
        least = std::min(least, cost(n));
        top = n;
    }
    if (base_cost * 50 > least * 51)
        for (int64_t n = nsplit + 1; n <= top; ++n)
            if (cost(n) * 50 <= least * 51) {
                nsplit = n;
                break;
            }
    const int64_t tiles_per_split = tiles_per(nsplit);
    p.split_rows = tiles_per_split * kTileRows;
    p.nsplit = (int)((tiles + tiles_per_split - 1) / tiles_per_split);
    return p;
}

// The split kernel a single-pair call runs: LATCH_PATH_AUTO resolved by the
// tuning table, and the MXFP4 path, whose keys hold a 14-bit split-local
// index, replaced by the int8 one (identical results) when the train rows
// would need more than the 65,535 splits a grid dimension allows.
int resolve_path(latch_handle h, int path, int64_t nq, int64_t nt)
{
    if (path == LATCH_PATH_AUTO) path = h->tuning.path[size_bucket(nq)][size_bucket(nt)];
    if (path == LATCH_PATH_MFMA_FP4 && nt > kMaxSplits * kFp4MaxSplitRows) path = LATCH_PATH_MFMA;
    return path;
}

// Partial top-2 keys of a split plan: 16 bytes per (split, query).
size_t knn_workspace_bytes(const KnnPlan &p)
{
    return p.nsplit > 1 ? align_up((size_t)p.nsplit * p.nq * 2 * sizeof(uint64_t), 256) : 0;
}

// Detection: survivor masks (one u64 per row and 64-column tile), the first
// output slot of every row, the per-(row, tile) survivor counts (rows padded
// to 16 bytes) and the count on entry.
struct DetectLayout {
    size_t mask_bytes, first_bytes, count_bytes, total;
    int count_stride;
};

DetectLayout detect_layout(int height, int width)
{
    DetectLayout l;
    l.mask_bytes = align_up((size_t)height * ((width + 63) / 64) * sizeof(uint64_t), 256);
    l.first_bytes = align_up((size_t)height * sizeof(int64_t), 256);
    l.count_stride = (int)align_up((size_t)(width + 63) / 64, 16);
    l.count_bytes = align_up((size_t)height * l.count_stride, 256);
    l.total = l.mask_bytes + l.first_bytes + l.count_bytes + sizeof(int64_t);
    return l;
}

size_t batch_workspace_bytes(int n_pairs, int64_t out_rows)
{
    const int64_t item_capacity = out_rows / 256 + n_pairs + 1;
    return align_up((size_t)n_pairs * sizeof(PairInfo), 256) + 256 +
           align_up((size_t)item_capacity * sizeof(int32_t), 256);
}

// Arguments of the batched matcher with its workspace at `ws`
// (batch_workspace_bytes bytes).
BatchArgs batch_args(latch_handle h, uint8_t *ws, const uint32_t *query_dev, int64_t query_rows,
                     const uint32_t *train_dev, int64_t train_rows, const latch_pair *pairs_dev,
                     int n_pairs, int k, float ratio, int32_t *idx_dev, int32_t *dist_dev,
                     uint8_t *accept_dev, int64_t out_rows, int path)
{
    const size_t info_bytes = align_up((size_t)n_pairs * sizeof(PairInfo), 256);
    BatchArgs a;
    a.query = query_dev;
    a.train = train_dev;
    a.query_rows = query_rows;
    a.train_rows = train_rows;
    a.out_rows = out_rows;
    a.pairs = reinterpret_cast<const PairEntry *>(pairs_dev);
    a.n_pairs = n_pairs;
    a.item_capacity = out_rows / 256 + n_pairs + 1;
    a.info = reinterpret_cast<PairInfo *>(ws);
    a.state = reinterpret_cast<BatchState *>(ws + info_bytes);
    a.item_pair = reinterpret_cast<int32_t *>(ws + info_bytes + 256);
    a.k = k;
    a.ratio = ratio;
    a.idx = idx_dev;
    a.dist = dist_dev;
    a.accept = accept_dev;
    a.flags = h->flags_dev;
    a.num_cus = h->num_cus;
    a.kind = split_kernel(path);
    a.shape = knn_shape(h->tuning);
    return a;
}

ExtractArgs batch_extract_args(latch_handle h, const latch_image *images_dev, int n_images,
                               const int32_t *image_id_dev, const latch_keypoint *kps_dev,
                               int64_t max_kps, const int64_t *n_kps_dev, uint32_t *desc_dev)
{
    ExtractArgs a;
    a.img = nullptr;
    a.height = a.width = a.pitch = 0;
    a.table = reinterpret_cast<const ImageEntry *>(images_dev);
    a.image_id = image_id_dev;
    a.n_images = n_images;
    a.kps = reinterpret_cast<const float4 *>(kps_dev);
    a.n = max_kps;
    a.n_dev = n_kps_dev;
    a.rot = h->rot_dev;
    a.trip_off = h->trip_off_dev;
    a.unperm = h->unperm_dev;
    a.gather = h->gather_dev;
    a.desc = desc_dev;
    a.flags = h->flags_dev;
    a.num_cus = h->num_cus;
    a.window = h->window;
    a.wtrip_off = h->wtrip_dev;
    a.wunperm = h->wunperm_dev;
    a.weights = h->weights;
    return a;
}

// The handle's extraction kernel: the weighted one for a geometry handle.
hipError_t run_extract(const ExtractArgs &a, hipStream_t stream)
{
    return a.window ? launch_extract_weighted(a, stream) : launch_extract(a, stream);
}

// Workspace of a batched extraction's spatial order (0: extracted as given).
constexpr int kOrderMaxImages = 1 << 16;

size_t extract_batch_workspace(latch_handle h, int n_images, int64_t max_kps)
{
    if (h->window || max_kps < kOrderMinKeypoints || n_images < 1 || n_images > kOrderMaxImages)
        return 0;
    return order_layout(n_images, max_kps).total;
}

// A batched extraction: the order's kernels (when the batch has one, in
// workspace `ws`), then the extraction kernel.  A plan's capture records no
// timing events (timed = false).
hipError_t run_extract_batch(latch_handle h, ExtractArgs a, uint8_t *ws, hipStream_t stream,
                             bool timed)
{
    auto launch = [&](const char *name, auto &&f) {
        return timed ? timed_launch(h, name, stream, f) : f();
    };
    if (extract_batch_workspace(h, a.n_images, a.n) > 0) {
        const hipError_t e = launch("extract_order", [&] { return launch_order(a, ws, stream); });
        if (e != hipSuccess) return e;
        a.order = reinterpret_cast<const int32_t *>(ws + order_layout(a.n_images, a.n).order);
    }
    return launch("extract", [&] { return run_extract(a, stream); });
}

// Scratch of hamming_knn_noalloc: a static device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never names
// it directly (on the host `scratch` is only a stand-in symbol): it uses the
// device address hipGetSymbolAddress gives, looked up once per device.
static __device__ __align__(256) uint8_t scratch[LATCH_NOALLOC_SCRATCH_BYTES];

std::mutex scratch_mutex;
std::map<int, uint8_t *> scratch_by_device;

// Address of `device`'s copy of the scratch array; `device` must be current.
hipError_t scratch_address(int device, uint8_t **out)
{
    std::lock_guard<std::mutex> lock(scratch_mutex);
    auto it = scratch_by_device.find(device);
    if (it == scratch_by_device.end()) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        it = scratch_by_device.emplace(device, static_cast<uint8_t *>(ptr)).first;
    }
    *out = it->second;
    return hipSuccess;
}

// A handle with the rotation table and the error word (no triplet data).
int create_base(latch_ctx **out)
{
    latch_ctx *h = new latch_ctx();
    default_tuning(&h->tuning);
    hipError_t e = hipGetDevice(&h->device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&h->num_cus, hipDeviceAttributeMultiprocessorCount, h->device);
    if (e == hipSuccess && h->num_cus >= 1) e = scratch_address(h->device, &h->scratch);
    if (e != hipSuccess || h->num_cus < 1) {
        delete h;
        return LATCH_EDEVICE;
    }
    int16_t c[kBins], s[kBins];
    rotation_table(c, s);
    int2 rot[kBins];
    for (int a = 0; a < kBins; ++a) rot[a] = make_int2(c[a], s[a]);
    if ((e = hipMalloc((void **)&h->rot_dev, sizeof rot)) == hipSuccess &&
        (e = hipMalloc((void **)&h->flags_dev, sizeof(uint32_t))) == hipSuccess) {
        const Upload u[2] = {{h->rot_dev, rot, sizeof rot}, {h->flags_dev, nullptr, sizeof(uint32_t)}};
        e = upload(u, 2);
    }
    if (e != hipSuccess) {
        const int rc = e == hipErrorOutOfMemory ? LATCH_ENOMEM : LATCH_EDEVICE;
        latch_destroy(h);
        return rc;
    }
    *out = h;
    return LATCH_OK;
}

// hamming_knn and hamming_knn_noalloc: the same checks and launches; the
// split partials go to the handle's workspace or to the static scratch.
int knn_call(latch_handle h, const uint32_t *query_dev, int64_t nq, const uint32_t *train_dev,
             int64_t nt, int k, float ratio, int32_t *idx_dev, int32_t *dist_dev,
             uint8_t *accept_dev, int path, hipStream_t stream, bool noalloc)
{
    if (!h) return LATCH_EINVAL;
    h->last_error.clear();
    if (nq < 0 || nq > LATCH_MAX_ROWS || nt < 0 || nt > LATCH_MAX_ROWS)
        return fail(h, LATCH_EINVAL, "sizes nq = %lld, nt = %lld out of [0, 2^31)", (long long)nq,
                    (long long)nt);
    if (k != 1 && k != 2) return fail(h, LATCH_ERANGE, "k = %d (must be 1 or 2)", k);
    if (!(ratio > 0.0f && ratio <= 1.0f))
        return fail(h, LATCH_ERANGE, "ratio = %g (must be in (0, 1])", (double)ratio);
    if (path < LATCH_PATH_AUTO || path > LATCH_PATH_MFMA_FP4)
        return fail(h, LATCH_EINVAL, "unknown path %d", path);
    if (nq == 0) return LATCH_OK;
    if (!query_dev || !idx_dev || !dist_dev || (nt > 0 && !train_dev))
        return fail(h, LATCH_EINVAL, "null buffer");
    path = resolve_path(h, path, nq, nt);

    KnnSplitArgs a;
    a.query = query_dev;
    a.train = train_dev;
    a.shape = knn_shape(h->tuning);
    a.plan = plan_knn(nq, nt, path, h->num_cus, h->tuning,
                      noalloc ? (size_t)LATCH_NOALLOC_SCRATCH_BYTES : SIZE_MAX);
    a.partial = nullptr;
    a.k = k;
    a.ratio = ratio;
    a.idx = idx_dev;
    a.dist = dist_dev;
    a.accept = accept_dev;
    if (a.plan.nsplit > 1) {
        const size_t need = knn_workspace_bytes(a.plan);
        if (noalloc) {
            // Every (split, query) partial is written by the split kernel
            // before the merge reads it, so nothing needs clearing.
            if (need > LATCH_NOALLOC_SCRATCH_BYTES)
                return fail(h, LATCH_ERANGE,
                            "hamming_knn_noalloc needs %zu scratch bytes (%d train splits x %lld "
                            "queries) and its static scratch holds %zu",
                            need, a.plan.nsplit, (long long)nq, (size_t)LATCH_NOALLOC_SCRATCH_BYTES);
            a.partial = reinterpret_cast<uint64_t *>(h->scratch);
        } else {
            const int rc = check_workspace(h, need, "hamming_knn");
            if (rc != LATCH_OK) return rc;
            a.partial = reinterpret_cast<uint64_t *>(h->ws);
        }
    }
    const SplitKernel which = split_kernel(path);
    const char *name = which == SplitKernel::kMfmaI8    ? "knn_mfma"
                       : which == SplitKernel::kMfmaFp4 ? "knn_fp4"
                                                        : "knn_popcount";
    // The allocation-free call records no timing events (creating one may allocate).
    auto launch = [&](const char *what, auto &&f) {
        return noalloc ? f() : timed_launch(h, what, stream, f);
    };
    hipError_t e = launch(name, [&] { return launch_knn_split(a, which, stream); });
    if (e != hipSuccess) return hip_fail(h, e, name);
    if (a.plan.nsplit > 1) {
        e = launch("knn_merge", [&] { return launch_knn_merge(a, stream); });
        if (e != hipSuccess) return hip_fail(h, e, "merge launch");
    }
    return LATCH_OK;
}

}  // namespace

struct latch_plan_ctx {
    latch_handle h = nullptr;
    uint8_t *ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

const char *latch_version(void) { return "latch-gfx950 0.2"; }

int latch_rotation_table(int16_t *cos_q14, int16_t *sin_q14)
{
    if (!cos_q14 || !sin_q14) return LATCH_EINVAL;
    rotation_table(cos_q14, sin_q14);
    return LATCH_OK;
}

int latch_create(latch_handle *out, const uint8_t *triplets_host)
{
    if (!out || !triplets_host) return LATCH_EINVAL;
    *out = nullptr;
    for (int i = 0; i < kTriplets * 6; ++i)
        if (triplets_host[i] < kPatchR || triplets_host[i] > kWin - 1 - kPatchR) return LATCH_ERANGE;

    latch_ctx *h = nullptr;
    int rc = create_base(&h);
    if (rc != LATCH_OK) return rc;
    uint2 toff[kTriplets];
    for (int t = 0; t < kTriplets; ++t) {
        const uint8_t *tr = triplets_host + 6 * t;
        toff[t].x = patch_offset(tr[0], tr[1]) | (patch_offset(tr[2], tr[3]) << 16);
        toff[t].y = patch_offset(tr[4], tr[5]);
    }
    // Triplets by slot, and per (wavefront w, lane l) the slots of output
    // bits 256 w + 64 k + l, k = 0..3, one byte each.
    uint8_t slot_of[kTriplets];
    assign_slots(toff, 2, 256, 32, 32, slot_of);   // row reads: ds_read_b64
    uint2 toff_slot[kTriplets];
    uint32_t unperm[2 * 64] = {};
    for (int t = 0; t < kTriplets; ++t) {
        const int w = t >> 8;
        toff_slot[256 * w + slot_of[t]] = toff[t];
        const int k = (t >> 6) & 3, l = t & 63;
        unperm[64 * w + l] |= (uint32_t)slot_of[t] << (8 * k);
    }
    uint2 doff[kTriplets];
    for (int t = 0; t < kTriplets; ++t) {
        const uint8_t *tr = triplets_host + 6 * t;
        doff[t] = make_uint2(dense_patch_offset(tr[0], tr[1]) | (dense_patch_offset(tr[2], tr[3]) << 16),
                             dense_patch_offset(tr[4], tr[5]));
    }
    const std::vector<uint16_t> order = gather_order();
    const size_t order_bytes = order.size() * sizeof(uint16_t);
    hipError_t e;
    if ((e = hipMalloc((void **)&h->trip_off_dev, sizeof toff_slot)) == hipSuccess &&
        (e = hipMalloc((void **)&h->unperm_dev, sizeof unperm)) == hipSuccess &&
        (e = hipMalloc((void **)&h->dense_off_dev, sizeof doff)) == hipSuccess &&
        (e = hipMalloc((void **)&h->gather_dev, order_bytes)) == hipSuccess) {
        const Upload u[4] = {{h->dense_off_dev, doff, sizeof doff},
                             {h->trip_off_dev, toff_slot, sizeof toff_slot},
                             {h->unperm_dev, unperm, sizeof unperm},
                             {h->gather_dev, order.data(), order_bytes}};
        e = upload(u, 4);
    }
    if (e != hipSuccess) {
        rc = e == hipErrorOutOfMemory ? LATCH_ENOMEM : LATCH_EDEVICE;
        latch_destroy(h);
        return rc;
    }
    *out = h;
    return LATCH_OK;
}

int latch_create_geometry(latch_handle *out, const uint8_t *triplets_host, int window, int patch,
                          const uint8_t *weights_host)
{
    if (!out || !triplets_host) return LATCH_EINVAL;
    *out = nullptr;
    if ((window != 48 && window != 64) || (patch != 7 && patch != 8)) return LATCH_ERANGE;
    uint8_t w[64];
    bool unit = true;
    for (int i = 0; i < patch * patch; ++i) {
        w[i] = weights_host ? weights_host[i] : 1;
        if (w[i] > 128) return LATCH_ERANGE;
        unit = unit && w[i] == 1;
    }
    for (int i = 0; i < kTriplets * 6; ++i) {
        const int first = triplets_host[i] - patch / 2;
        if (first < 0 || first + patch > window) return LATCH_ERANGE;
    }
    if (window == kWin && patch == 2 * kPatchR + 1 && unit) return latch_create(out, triplets_host);

    latch_ctx *h = nullptr;
    int rc = create_base(&h);
    if (rc != LATCH_OK) return rc;
    h->window = window;
    // 7 x 7 patches run as 8 x 8 ones whose last row and column weigh 0.
    for (int r = 0; r < 8; ++r)
        for (int i = 0; i < 4; ++i) {
            const int c0 = 2 * i, c1 = 2 * i + 1;
            const uint32_t lo = (r < patch && c0 < patch) ? w[r * patch + c0] : 0u;
            const uint32_t hi = (r < patch && c1 < patch) ? w[r * patch + c1] : 0u;
            h->weights.pair[4 * r + i] = lo | (hi << 16);
        }
    uint2 toff[kTriplets];
    for (int t = 0; t < kTriplets; ++t) {
        const uint8_t *tr = triplets_host + 6 * t;
        uint32_t o[3];
        for (int k = 0; k < 3; ++k)
            o[k] = weighted_patch_offset(window, tr[2 * k] - patch / 2, tr[2 * k + 1] - patch / 2);
        toff[t] = make_uint2(o[0] | (o[1] << 16), o[2]);
    }
    // Wavefront w evaluates triplets 64 w + l and 256 + 64 w + l (members l
    // and 64 + l) in two rounds; bank-aware slots, and per lane the slots of
    // its two output bits.
    const int kWWaves = 4, kWPerWave = kTriplets / kWWaves;
    auto member = [](int w, int i) { return i < 64 ? 64 * w + i : 256 + 64 * w + (i - 64); };
    uint2 mem[kTriplets];
    for (int w = 0; w < kWWaves; ++w)
        for (int i = 0; i < kWPerWave; ++i) mem[kWPerWave * w + i] = toff[member(w, i)];
    uint8_t slot_of[kTriplets];
    assign_slots(mem, kWWaves, kWPerWave, 32, 32, slot_of);   // row reads: ds_read_b64
    uint2 toff_slot[kTriplets];
    uint32_t unperm[kWWaves * 64] = {};
    for (int w = 0; w < kWWaves; ++w)
        for (int i = 0; i < kWPerWave; ++i) {
            toff_slot[kWPerWave * w + slot_of[kWPerWave * w + i]] = mem[kWPerWave * w + i];
            unperm[64 * w + (i & 63)] |= (uint32_t)slot_of[kWPerWave * w + i] << (8 * (i >> 6));
        }
    hipError_t e;
    if ((e = hipMalloc((void **)&h->wtrip_dev, sizeof toff_slot)) == hipSuccess &&
        (e = hipMalloc((void **)&h->wunperm_dev, sizeof unperm)) == hipSuccess) {
        const Upload u[2] = {{h->wtrip_dev, toff_slot, sizeof toff_slot},
                             {h->wunperm_dev, unperm, sizeof unperm}};
        e = upload(u, 2);
    }
    if (e != hipSuccess) {
        rc = e == hipErrorOutOfMemory ? LATCH_ENOMEM : LATCH_EDEVICE;
        latch_destroy(h);
        return rc;
    }
    *out = h;
    return LATCH_OK;
}

void latch_destroy(latch_handle h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();
    if (h->rot_dev) (void)hipFree(h->rot_dev);
    if (h->trip_off_dev) (void)hipFree(h->trip_off_dev);
    if (h->unperm_dev) (void)hipFree(h->unperm_dev);
    if (h->gather_dev) (void)hipFree(h->gather_dev);
    if (h->flags_dev) (void)hipFree(h->flags_dev);
    if (h->wtrip_dev) (void)hipFree(h->wtrip_dev);
    if (h->wunperm_dev) (void)hipFree(h->wunperm_dev);
    if (h->dense_off_dev) (void)hipFree(h->dense_off_dev);
    if (h->ws) (void)hipFree(h->ws);
    release_timed(h);
    for (hipEvent_t e : h->event_pool) (void)hipEventDestroy(e);
    delete h;
}

const char *latch_last_error(latch_handle h) { return h ? h->last_error.c_str() : "null handle"; }

int latch_extract(latch_handle h, const uint8_t *img_dev, int height, int width, int pitch,
                  const latch_keypoint *kps_dev, int64_t n_kps, uint32_t *desc_dev,
                  hipStream_t stream)
{
    if (!h) return LATCH_EINVAL;
    h->last_error.clear();
    if (n_kps < 0 || n_kps > LATCH_MAX_ROWS)
        return fail(h, LATCH_EINVAL, "n_kps = %lld out of [0, 2^31)", (long long)n_kps);
    if (height < 1 || width < 1 || pitch < width)
        return fail(h, LATCH_EINVAL, "bad image shape %d x %d, pitch %d", height, width, pitch);
    if ((int64_t)height * pitch > (int64_t)INT32_MAX || height >= (1 << 23) || pitch >= (1 << 23))
        return fail(h, LATCH_EINVAL, "image of %d rows x %d pitch: need rows, pitch < 2^23 and "
                    "rows * pitch < 2^31", height, pitch);
    if (n_kps == 0) return LATCH_OK;
    if (!img_dev || !kps_dev || !desc_dev) return fail(h, LATCH_EINVAL, "null buffer");
    ExtractArgs a;
    a.img = img_dev;
    a.height = height;
    a.width = width;
    a.pitch = pitch;
    a.table = nullptr;
    a.image_id = nullptr;
    a.n_images = 0;
    a.kps = reinterpret_cast<const float4 *>(kps_dev);
    a.n = n_kps;
    a.n_dev = nullptr;
    a.rot = h->rot_dev;
    a.trip_off = h->trip_off_dev;
    a.unperm = h->unperm_dev;
    a.gather = h->gather_dev;
    a.desc = desc_dev;
    a.flags = h->flags_dev;
    a.num_cus = h->num_cus;
    a.window = h->window;
    a.wtrip_off = h->wtrip_dev;
    a.wunperm = h->wunperm_dev;
    a.weights = h->weights;
    hipError_t e = timed_launch(h, "extract", stream, [&] { return run_extract(a, stream); });
    return e == hipSuccess ? LATCH_OK : hip_fail(h, e, "extract launch");
}

int latch_extract_batch(latch_handle h, const latch_image *images_dev, int n_images,
                        const int32_t *image_id_dev, const latch_keypoint *kps_dev, int64_t max_kps,
                        const int64_t *n_kps_dev, uint32_t *desc_dev, hipStream_t stream)
{
    if (!h) return LATCH_EINVAL;
    h->last_error.clear();
    if (max_kps < 0 || max_kps > LATCH_MAX_ROWS)
        return fail(h, LATCH_EINVAL, "max_kps = %lld out of [0, 2^31)", (long long)max_kps);
    if (n_images < 0) return fail(h, LATCH_EINVAL, "n_images = %d < 0", n_images);
    if (max_kps == 0) return LATCH_OK;
    if (!images_dev || !image_id_dev || !kps_dev || !desc_dev || n_images == 0)
        return fail(h, LATCH_EINVAL, "null buffer or empty image table");
    const int rc = check_workspace(h, extract_batch_workspace(h, n_images, max_kps),
                                   "latch_extract_batch");
    if (rc != LATCH_OK) return rc;
    const ExtractArgs a = batch_extract_args(h, images_dev, n_images, image_id_dev, kps_dev,
                                             max_kps, n_kps_dev, desc_dev);
    const hipError_t e = run_extract_batch(h, a, h->ws, stream, true);
    return e == hipSuccess ? LATCH_OK : hip_fail(h, e, "batched extract launch");
}

int latch_extract_dense(latch_handle h, const uint8_t *img_dev, int height, int width, int pitch,
                        int x0, int y0, int gw, int gh, uint32_t *desc_dev, hipStream_t stream)
{
    if (!h) return LATCH_EINVAL;
    h->last_error.clear();
    if (!h->dense_off_dev)
        return fail(h, LATCH_EINVAL, "dense extraction needs a handle of the default geometry");
    if (height < 1 || width < 1 || pitch < width || height >= (1 << 23) || pitch >= (1 << 23) ||
        (int64_t)height * pitch > (int64_t)INT32_MAX)
        return fail(h, LATCH_EINVAL, "image %d x %d, pitch %d outside the limits", height, width, pitch);
    if (gw < 0 || gh < 0 || (int64_t)gw * gh > LATCH_MAX_ROWS || x0 < -(1 << 24) || y0 < -(1 << 24) ||
        (int64_t)x0 + gw > (1 << 24) || (int64_t)y0 + gh > (1 << 24))
        return fail(h, LATCH_ERANGE, "region (%d, %d) + %d x %d outside the limits", x0, y0, gw, gh);
    if (gw == 0 || gh == 0) return LATCH_OK;
    if (!img_dev || !desc_dev) return fail(h, LATCH_EINVAL, "null buffer");
    DenseArgs a;
    a.img = img_dev;
    a.height = height;
    a.width = width;
    a.pitch = pitch;
    a.x0 = x0;
    a.y0 = y0;
    a.gw = gw;
    a.gh = gh;
    a.toff = h->dense_off_dev;
    a.desc = desc_dev;
    const hipError_t e =
        timed_launch(h, "dense_extract", stream, [&] { return launch_dense_extract(a, stream); });
    return e == hipSuccess ? LATCH_OK : hip_fail(h, e, "dense extract launch");
}

int hamming_knn_window(latch_handle h, const uint32_t *query_dev, const uint32_t *train_dev, int gw,
                       int gh, int radius, int k, float ratio, int32_t *idx_dev, int32_t *dist_dev,
                       uint8_t *accept_dev, hipStream_t stream)
{
    if (!h) return LATCH_EINVAL;
    h->last_error.clear();
    if (gw < 0 || gh < 0 || (int64_t)gw * gh > LATCH_MAX_ROWS)
        return fail(h, LATCH_EINVAL, "grid %d x %d", gw, gh);
    if (radius < 0 || radius > kDenseMaxRadius)
        return fail(h, LATCH_ERANGE, "radius %d (must be in [0, %d])", radius, kDenseMaxRadius);
    if (k != 1 && k != 2) return fail(h, LATCH_ERANGE, "k = %d (must be 1 or 2)", k);
    if (!(ratio > 0.0f && ratio <= 1.0f))
        return fail(h, LATCH_ERANGE, "ratio = %g (must be in (0, 1])", (double)ratio);
    if (gw == 0 || gh == 0) return LATCH_OK;
    if (!query_dev || !train_dev || !idx_dev || !dist_dev) return fail(h, LATCH_EINVAL, "null buffer");
    DenseMatchArgs a;
    a.query = query_dev;
    a.train = train_dev;
    a.gw = gw;
    a.gh = gh;
    a.radius = radius;
    a.k = k;
    a.ratio = ratio;
    a.idx = idx_dev;
    a.dist = dist_dev;
    a.accept = accept_dev;
    const hipError_t e =
        timed_launch(h, "knn_window", stream, [&] { return launch_dense_match(a, stream); });
    return e == hipSuccess ? LATCH_OK : hip_fail(h, e, "dense match launch");
}

int latch_detect(latch_handle h, const uint8_t *img_dev, int height, int width, int pitch,
                 int threshold, latch_keypoint *kps_dev, int64_t max_kps, int64_t *n_kps_dev,
                 int32_t *image_id_dev, int32_t image_index, hipStream_t stream)
{
    if (!h) return LATCH_EINVAL;
    h->last_error.clear();
    if (!img_dev || !n_kps_dev || (max_kps > 0 && !kps_dev))
        return fail(h, LATCH_EINVAL, "null buffer");
    if (height < 1 || width < 1 || pitch < width || height >= (1 << 23) || pitch >= (1 << 23) ||
        (int64_t)height * pitch > (int64_t)0x7fffffff)
        return fail(h, LATCH_EINVAL, "image %d x %d, pitch %d outside the limits", height, width,
                    pitch);
    if (threshold < 0 || threshold > 255)
        return fail(h, LATCH_ERANGE, "threshold %d (must be in [0, 255])", threshold);
    if (max_kps < 0 || max_kps > LATCH_MAX_ROWS)
        return fail(h, LATCH_EINVAL, "max_kps = %lld", (long long)max_kps);
    const DetectLayout l = detect_layout(height, width);
    const int rc = check_workspace(h, l.total, "latch_detect");
    if (rc != LATCH_OK) return rc;
    DetectArgs a;
    a.img = img_dev;
    a.height = height;
    a.width = width;
    a.pitch = pitch;
    a.threshold = threshold;
    a.masks = reinterpret_cast<uint64_t *>(h->ws);
    a.row_first = reinterpret_cast<int64_t *>(h->ws + l.mask_bytes);
    a.counts = h->ws + l.mask_bytes + l.first_bytes;
    a.count_stride = l.count_stride;
    a.base = reinterpret_cast<int64_t *>(h->ws + l.mask_bytes + l.first_bytes + l.count_bytes);
    a.kps = reinterpret_cast<float4 *>(kps_dev);
    a.max_kps = max_kps;
    a.n_kps = n_kps_dev;
    a.image_id = image_id_dev;
    a.image_index = image_index;
    const hipError_t e = timed_launch(h, "detect", stream, [&] { return launch_detect(a, stream); });
    return e == hipSuccess ? LATCH_OK : hip_fail(h, e, "detect launch");
}

int hamming_knn(latch_handle h, const uint32_t *query_dev, int64_t nq, const uint32_t *train_dev,
                int64_t nt, int k, float ratio, int32_t *idx_dev, int32_t *dist_dev,
                uint8_t *accept_dev, int path, hipStream_t stream)
{
    return knn_call(h, query_dev, nq, train_dev, nt, k, ratio, idx_dev, dist_dev, accept_dev, path,
                    stream, false);
}

int hamming_knn_noalloc(latch_handle h, const uint32_t *query_dev, int64_t nq,
                        const uint32_t *train_dev, int64_t nt, int k, float ratio,
                        int32_t *idx_dev, int32_t *dist_dev, uint8_t *accept_dev, int path,
                        hipStream_t stream)
{
    return knn_call(h, query_dev, nq, train_dev, nt, k, ratio, idx_dev, dist_dev, accept_dev, path,
                    stream, true);
}

int hamming_knn_workspace_size(latch_handle h, int64_t nq, int64_t nt, int path, size_t *bytes)
{
    if (!h || !bytes) return LATCH_EINVAL;
    if (nq < 0 || nq > LATCH_MAX_ROWS || nt < 0 || nt > LATCH_MAX_ROWS)
        return fail(h, LATCH_EINVAL, "sizes nq = %lld, nt = %lld out of [0, 2^31)", (long long)nq,
                    (long long)nt);
    if (path < LATCH_PATH_AUTO || path > LATCH_PATH_MFMA_FP4)
        return fail(h, LATCH_EINVAL, "unknown path %d", path);
    path = resolve_path(h, path, nq, nt);
    *bytes = nq == 0 ? 0 : knn_workspace_bytes(plan_knn(nq, nt, path, h->num_cus, h->tuning, SIZE_MAX));
    return LATCH_OK;
}

int hamming_knn_batch_workspace_size(latch_handle h, int n_pairs, int64_t out_rows, size_t *bytes)
{
    if (!h || !bytes) return LATCH_EINVAL;
    if (n_pairs < 0 || out_rows < 0 || out_rows > LATCH_MAX_ROWS)
        return fail(h, LATCH_EINVAL, "negative or too large batch size");
    *bytes = n_pairs == 0 ? 0 : batch_workspace_bytes(n_pairs, out_rows);
    return LATCH_OK;
}

int latch_detect_workspace_size(latch_handle h, int height, int width, size_t *bytes)
{
    if (!h || !bytes) return LATCH_EINVAL;
    if (height < 1 || width < 1 || height >= (1 << 23))
        return fail(h, LATCH_EINVAL, "image %d x %d outside the limits", height, width);
    *bytes = detect_layout(height, width).total;
    return LATCH_OK;
}

int latch_extract_batch_workspace_size(latch_handle h, int n_images, int64_t max_kps,
                                       size_t *bytes)
{
    if (!h || !bytes) return LATCH_EINVAL;
    if (n_images < 0 || max_kps < 0 || max_kps > LATCH_MAX_ROWS)
        return fail(h, LATCH_EINVAL, "n_images = %d, max_kps = %lld out of range", n_images,
                    (long long)max_kps);
    *bytes = extract_batch_workspace(h, n_images, max_kps);
    return LATCH_OK;
}

int latch_reserve(latch_handle h, size_t bytes, size_t *held_out)
{
    if (!h) return LATCH_EINVAL;
    h->last_error.clear();
    if (bytes > h->ws_bytes) {
        const size_t want = align_up(bytes, 256);
        if (h->ws) {
            // Work enqueued on any stream may still use the old buffer.
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(h, e, "hipDeviceSynchronize");
            (void)hipFree(h->ws);
            h->ws = nullptr;
            h->ws_bytes = 0;
        }
        const hipError_t e = hipMalloc((void **)&h->ws, want);
        if (e != hipSuccess) {
            h->ws = nullptr;
            if (held_out) *held_out = 0;
            return hip_fail(h, e, "hipMalloc(workspace)");
        }
        h->ws_bytes = want;
    }
    if (held_out) *held_out = h->ws_bytes;
    return LATCH_OK;
}

int latch_get_tuning(latch_handle h, latch_tuning *out)
{
    if (!h || !out) return LATCH_EINVAL;
    *out = h->tuning;
    return LATCH_OK;
}

int latch_set_tuning(latch_handle h, const latch_tuning *t)
{
    if (!h || !t) return LATCH_EINVAL;
    auto ok_path = [](int p) {
        return p == LATCH_PATH_MFMA || p == LATCH_PATH_POPCOUNT || p == LATCH_PATH_MFMA_FP4;
    };
    for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j)
            if (!ok_path(t->path[i][j])) return fail(h, LATCH_ERANGE, "tuning path[%d][%d]", i, j);
    if (!ok_path(t->batch_path)) return fail(h, LATCH_ERANGE, "tuning batch_path");
    if (t->mfma_groups_per_cu < 1 || t->popcount_groups_per_cu < 1)
        return fail(h, LATCH_ERANGE, "tuning workgroup targets must be >= 1");
    if (t->fp4_query_blocks != 2 && t->fp4_query_blocks != 3)
        return fail(h, LATCH_ERANGE, "tuning fp4_query_blocks = %d (must be 2 or 3)",
                    t->fp4_query_blocks);
    if (t->batch_groups_per_cu < 1 || t->batch_groups_per_cu > 8)
        return fail(h, LATCH_ERANGE, "tuning batch_groups_per_cu = %d (must be in [1, 8])",
                    t->batch_groups_per_cu);
    h->tuning = *t;
    return LATCH_OK;
}

int latch_timing_enable(latch_handle h, int enable)
{
    if (!h) return LATCH_EINVAL;
    if (enable) {
        // Earlier records must be complete before their events are reused.
        for (auto &t : h->timed) (void)hipEventSynchronize(t.stop);
        release_timed(h);
    }
    h->timing = enable != 0;
    return LATCH_OK;
}

int latch_timing_read(latch_handle h, const char *kernel, int *launches, double *total_ms)
{
    if (!h || !kernel || !launches || !total_ms) return LATCH_EINVAL;
    int n = 0;
    double ms = 0.0;
    for (auto &t : h->timed) {
        if (std::strcmp(t.name, kernel) != 0) continue;
        hipError_t e = hipEventSynchronize(t.stop);
        float v = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&v, t.start, t.stop);
        if (e != hipSuccess) return hip_fail(h, e, "reading timing events");
        ++n;
        ms += v;
    }
    *launches = n;
    *total_ms = ms;
    return LATCH_OK;
}

int hamming_knn_batch(latch_handle h, const uint32_t *query_dev, int64_t query_rows,
                      const uint32_t *train_dev, int64_t train_rows, const latch_pair *pairs_dev,
                      int n_pairs, int k, float ratio, int32_t *idx_dev, int32_t *dist_dev,
                      uint8_t *accept_dev, int64_t out_rows, int path, hipStream_t stream)
{
    if (!h) return LATCH_EINVAL;
    h->last_error.clear();
    if (n_pairs < 0 || query_rows < 0 || train_rows < 0 || out_rows < 0 ||
        query_rows > LATCH_MAX_ROWS || train_rows > LATCH_MAX_ROWS || out_rows > LATCH_MAX_ROWS)
        return fail(h, LATCH_EINVAL, "negative or too large batch size");
    if (k != 1 && k != 2) return fail(h, LATCH_ERANGE, "k = %d (must be 1 or 2)", k);
    if (!(ratio > 0.0f && ratio <= 1.0f))
        return fail(h, LATCH_ERANGE, "ratio = %g (must be in (0, 1])", (double)ratio);
    if (path < LATCH_PATH_AUTO || path > LATCH_PATH_MFMA_FP4)
        return fail(h, LATCH_EINVAL, "unknown path %d", path);
    if (n_pairs == 0) return LATCH_OK;
    if (!pairs_dev || !idx_dev || !dist_dev || (query_rows > 0 && !query_dev) ||
        (train_rows > 0 && !train_dev))
        return fail(h, LATCH_EINVAL, "null buffer");
    if (path == LATCH_PATH_AUTO) path = h->tuning.batch_path;

    const int rc = check_workspace(h, batch_workspace_bytes(n_pairs, out_rows), "hamming_knn_batch");
    if (rc != LATCH_OK) return rc;
    const BatchArgs a = batch_args(h, h->ws, query_dev, query_rows, train_dev, train_rows,
                                   pairs_dev, n_pairs, k, ratio, idx_dev, dist_dev, accept_dev,
                                   out_rows, path);
    const char *name = a.kind == SplitKernel::kPopcount  ? "knn_batch_popcount"
                       : a.kind == SplitKernel::kMfmaFp4 ? "knn_batch_fp4"
                                                         : "knn_batch_mfma";
    hipError_t e = timed_launch(h, name, stream,
                                [&] { return launch_knn_batch(a, stream); });
    return e == hipSuccess ? LATCH_OK : hip_fail(h, e, "batched knn launch");
}

int latch_plan_create(latch_handle h, const latch_plan_desc *d, latch_plan *out)
{
    if (!h || !d || !out) return LATCH_EINVAL;
    *out = nullptr;
    h->last_error.clear();
    if (d->max_kps < 0 || d->max_kps > LATCH_MAX_ROWS || d->n_images < 1 || d->n_pairs < 0 ||
        d->out_rows < 0 || d->out_rows > LATCH_MAX_ROWS)
        return fail(h, LATCH_EINVAL, "bad plan sizes");
    if (d->k != 1 && d->k != 2) return fail(h, LATCH_ERANGE, "k = %d (must be 1 or 2)", d->k);
    if (!(d->ratio > 0.0f && d->ratio <= 1.0f))
        return fail(h, LATCH_ERANGE, "ratio = %g (must be in (0, 1])", (double)d->ratio);
    if (d->path < LATCH_PATH_AUTO || d->path > LATCH_PATH_MFMA_FP4)
        return fail(h, LATCH_EINVAL, "unknown path %d", d->path);
    if (!d->images || !d->image_id || !d->kps || !d->desc ||
        (d->n_pairs > 0 && (!d->pairs || !d->idx || !d->dist)))
        return fail(h, LATCH_EINVAL, "null buffer");

    latch_plan_ctx *p = new latch_plan_ctx();
    p->h = h;
    // Plan workspace: the matcher's state, then the extraction's order.
    const size_t knn_bytes = align_up(batch_workspace_bytes(d->n_pairs, d->out_rows), 256);
    const size_t order_bytes = extract_batch_workspace(h, d->n_images, d->max_kps);
    hipError_t e = hipMalloc((void **)&p->ws, knn_bytes + order_bytes);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(h, e, "hipMalloc(plan workspace)");
    }
    const ExtractArgs ea = batch_extract_args(h, d->images, d->n_images, d->image_id, d->kps,
                                              d->max_kps, d->n_kps, d->desc);
    const BatchArgs ba = batch_args(h, p->ws, d->desc, d->max_kps, d->desc, d->max_kps, d->pairs,
                                    d->n_pairs, d->k, d->ratio, d->idx, d->dist, d->accept,
                                    d->out_rows,
                                    d->path == LATCH_PATH_AUTO ? h->tuning.batch_path : d->path);
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess && d->max_kps > 0) e = run_extract_batch(h, ea, p->ws + knn_bytes, s, false);
    if (e == hipSuccess && d->n_pairs > 0) e = launch_knn_batch(ba, s);
    hipGraph_t graph = nullptr;
    if (s) {
        const hipError_t e2 = hipStreamEndCapture(s, &graph);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    p->graph = graph;
    if (s) (void)hipStreamDestroy(s);
    if (e != hipSuccess) {
        latch_plan_destroy(p);
        return hip_fail(h, e, "plan capture");
    }
    *out = p;
    return LATCH_OK;
}

int latch_plan_run(latch_plan p, hipStream_t stream)
{
    if (!p) return LATCH_EINVAL;
    const hipError_t e = hipGraphLaunch(p->exec, stream);
    return e == hipSuccess ? LATCH_OK : hip_fail(p->h, e, "graph launch");
}

void latch_plan_destroy(latch_plan p)
{
    if (!p) return;
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->ws) (void)hipFree(p->ws);
    delete p;
}

int latch_check_errors(latch_handle h, hipStream_t stream, uint32_t *flags_out, int clear)
{
    if (!h || !flags_out) return LATCH_EINVAL;
    uint32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, h->flags_dev, sizeof v, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(h, e, "reading error word");
    *flags_out = v;
    if (clear) {
        e = hipMemsetAsync(h->flags_dev, 0, sizeof v, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(h, e, "clearing error word");
    }
    return LATCH_OK;
}

}  // extern "C"
