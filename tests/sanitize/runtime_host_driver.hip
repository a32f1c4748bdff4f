// The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Built together with the other library sources, the host pass sanitized and
// the device code as usual, with this file including the runtime's source so
// that its internal host functions are reachable.  It launches no kernel and
// needs no GPU.  It runs the host logic that every
// handle and call goes through: the rotation table, the gather order tables,
// the triplet slot search, the split planner and the workspace sizes, and the
// C ABI's argument checks with null and out-of-range arguments (which return
// before any HIP call).  Prints a digest of the results; exits non-zero on a
// failed check.
#include "../../paper_1609_03986_amd/csrc/runtime.hip"

#include <cstdio>
#include <cstdlib>

namespace {

uint64_t digest = 1469598103934665603ull;

void mix(const void *p, size_t n)
{
    const uint8_t *b = static_cast<const uint8_t *>(p);
    for (size_t i = 0; i < n; ++i) {
        digest ^= b[i];
        digest *= 1099511628211ull;
    }
}

int failures = 0;

void check(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "check failed: %s\n", what);
        ++failures;
    }
}

uint64_t rng = 88172645463325252ull;

uint32_t next()
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (uint32_t)(rng >> 32);
}

}  // namespace

int main()
{
    // Rotation table through the C ABI, and its quarter-turn symmetry.
    std::vector<int16_t> c(kBins), s(kBins);
    check(latch_rotation_table(c.data(), s.data()) == LATCH_OK, "rotation table");
    check(latch_rotation_table(nullptr, s.data()) == LATCH_EINVAL, "rotation table null");
    for (int a = 0; a + 1024 < kBins; ++a)
        check(c[a + 1024] == -s[a] && s[a + 1024] == c[a], "quarter turn");
    mix(c.data(), c.size() * 2);
    mix(s.data(), s.size() * 2);

    // Gather order: in every class the chains (u, v), (u + 1, v), (-u, -v),
    // (-u - 1, -v) cover every position of [-24, 24]^2, stay inside it, and
    // the 27 padding slots repeat the centre's chain.
    const std::vector<uint16_t> order = gather_order();
    check(order.size() == (size_t)kGatherClasses * kGatherClassEntries, "gather order size");
    constexpr int kSide = kWin + 1;
    for (int cl = 0; cl < kGatherClasses; ++cl) {
        std::vector<int> seen(kSide * kSide, 0);
        int centre_chains = 0;
        for (int t = 0; t < 128; ++t)
            for (int m = 0; m < kGatherChains; ++m) {
                const size_t at = m < kGatherHeadChains ? (size_t)kGatherHeadChains * t + m
                                                        : (size_t)kGatherHeadChains * 128 + t;
                const uint16_t e = order[(size_t)cl * kGatherClassEntries + at];
                const int u = (int8_t)(e & 0xff), v = (int8_t)(e >> 8);
                check(u >= -kHalf && u + 1 <= kHalf && v >= 0 && v <= kHalf && (v > 0 || u >= 0),
                      "gather chain range");
                centre_chains += u == 0 && v == 0;
                for (int d = 0; d < 2; ++d) {
                    ++seen[(v + kHalf) * kSide + (u + d + kHalf)];
                    ++seen[(-v + kHalf) * kSide + (-u - d + kHalf)];
                }
            }
        for (int p = 0; p < kSide * kSide; ++p) check(seen[p] >= 1, "gather chains cover each position");
        check(centre_chains == 128 * kGatherChains - (24 * 25 + 13) + 1, "centre chain pads the slots");
    }
    mix(order.data(), order.size() * 2);

    // Triplet slots for a random table, both kernels' groupings.
    uint2 toff[kTriplets];
    for (int t = 0; t < kTriplets; ++t) {
        int v[6];
        for (int i = 0; i < 6; ++i) v[i] = 3 + (int)(next() % 42);
        toff[t].x = patch_offset(v[0], v[1]) | (patch_offset(v[2], v[3]) << 16);
        toff[t].y = patch_offset(v[4], v[5]);
    }
    uint8_t slot_of[kTriplets];
    assign_slots(toff, 2, 256, 32, 32, slot_of);
    for (int w = 0; w < 2; ++w) {
        std::vector<int> used(256, 0);
        for (int t = 0; t < 256; ++t) ++used[slot_of[256 * w + t]];
        for (int i = 0; i < 256; ++i) check(used[i] == 1, "slots are a permutation");
    }
    mix(slot_of, sizeof slot_of);

    // Split plans and workspace sizes over a grid of sizes, paths and tunings.
    latch_tuning tune;
    default_tuning(&tune);
    latch_ctx probe;                      // host fields only: the tuning table
    default_tuning(&probe.tuning);
    const int64_t sizes[] = {1, 31, 32, 255, 256, 10000, 16384, 16385, 20000, 1000000, 2147483647LL};
    for (int qb : {2, 3})
        for (int path : {LATCH_PATH_MFMA, LATCH_PATH_POPCOUNT, LATCH_PATH_MFMA_FP4})
            for (int64_t nq : sizes)
                for (int64_t nt : sizes) {
                    tune.fp4_query_blocks = (int8_t)qb;
                    const int run = resolve_path(&probe, path, nq, nt);
                    check(run == path || (path == LATCH_PATH_MFMA_FP4 && run == LATCH_PATH_MFMA),
                          "resolved path");
                    const KnnPlan p = plan_knn(nq, nt, run, 256, tune, SIZE_MAX);
                    check(p.nsplit <= kMaxSplits && p.split_rows <= kMaxSplitRows, "plan limits");
                    check(p.nsplit >= 1 && p.split_rows >= kTileRows && p.split_rows % kTileRows == 0,
                          "plan shape");
                    check((int64_t)p.nsplit * p.split_rows >= nt, "plan covers the train rows");
                    if (run == LATCH_PATH_MFMA_FP4) check(p.split_rows <= kFp4MaxSplitRows, "fp4 split");
                    const size_t ws = knn_workspace_bytes(p);
                    mix(&p.nsplit, sizeof p.nsplit);
                    mix(&p.split_rows, sizeof p.split_rows);
                    mix(&ws, sizeof ws);
                }
    for (int n_pairs : {1, 63, 255, 100000})
        for (int64_t rows : {1LL, 1280000LL, 2147483647LL}) {
            const size_t b = batch_workspace_bytes(n_pairs, rows);
            mix(&b, sizeof b);
        }
    for (int h : {1, 33, 1080, 4000})
        for (int w : {1, 63, 64, 65, 1920, 3000}) {
            const DetectLayout l = detect_layout(h, w);
            check(l.total >= l.mask_bytes + l.first_bytes + l.count_bytes, "detect layout");
            mix(&l.total, sizeof l.total);
        }
    for (int n_images : {1, 64, 65536})
        for (int64_t kps : {262144LL, 1280000LL, 2147483647LL}) {
            const OrderLayout l = order_layout(n_images, kps);
            check(l.order + (size_t)kps * 4 <= l.total, "order layout");
            mix(&l.total, sizeof l.total);
        }

    // The C ABI's argument checks (all return before any HIP call).
    size_t bytes = 0;
    latch_handle none = nullptr;
    check(latch_create(nullptr, nullptr) == LATCH_EINVAL, "create null");
    check(latch_create_geometry(nullptr, nullptr, 64, 8, nullptr) == LATCH_EINVAL, "geometry null");
    check(latch_extract(none, nullptr, 1, 1, 1, nullptr, 0, nullptr, nullptr) == LATCH_EINVAL, "extract");
    check(latch_extract_batch(none, nullptr, 1, nullptr, nullptr, 1, nullptr, nullptr, nullptr) ==
              LATCH_EINVAL, "extract batch");
    check(hamming_knn(none, nullptr, 1, nullptr, 1, 2, 0.8f, nullptr, nullptr, nullptr, 0, nullptr) ==
              LATCH_EINVAL, "knn");
    check(hamming_knn_noalloc(none, nullptr, 1, nullptr, 1, 2, 0.8f, nullptr, nullptr, nullptr, 0,
                              nullptr) == LATCH_EINVAL, "knn noalloc");
    check(hamming_knn_workspace_size(none, 1, 1, 0, &bytes) == LATCH_EINVAL, "knn ws");
    check(hamming_knn_batch_workspace_size(none, 1, 1, &bytes) == LATCH_EINVAL, "batch ws");
    check(latch_detect_workspace_size(none, 1, 1, &bytes) == LATCH_EINVAL, "detect ws");
    check(latch_extract_batch_workspace_size(none, 1, 1, &bytes) == LATCH_EINVAL, "extract ws");
    check(latch_reserve(none, 100, &bytes) == LATCH_EINVAL, "reserve");
    check(latch_set_tuning(none, &tune) == LATCH_EINVAL, "set tuning");
    check(latch_plan_run(nullptr, nullptr) == LATCH_EINVAL, "plan run");
    latch_destroy(nullptr);
    latch_plan_destroy(nullptr);
    check(std::strlen(latch_last_error(nullptr)) > 0, "last error of no handle");
    check(std::strlen(latch_version()) > 0, "version");

    std::printf("%016llx\n", (unsigned long long)digest);
    return failures ? 1 : 0;
}
