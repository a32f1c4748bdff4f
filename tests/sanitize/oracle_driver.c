/*
 * Runs every entry point of the oracle (oracle/latch_oracle.c) on small seeded
 * inputs, edge cases included: 1 x 1 images and images with pitch > width,
 * windows far past the borders, keypoints outside the resampling rule's
 * domain (non-finite fields, huge coordinates and angles, scales whose Q8
 * value is 0 or above 1024), the 64 x 64 / 8 x 8 weighted geometry, empty and
 * one-row matching, dense matching at radius 0 and past the grid, and
 * detection at and below its minimum image size.  Prints an FNV-1a digest of
 * every output.  The CPU test builds it twice, plainly and with
 * AddressSanitizer and UndefinedBehaviorSanitizer: both builds must exit 0
 * with the same digest and no sanitizer report.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_rotation_table(int16_t *cos_q14, int16_t *sin_q14);
unsigned oracle_sample_window(const uint8_t *img, int height, int width, int pitch, float x,
                              float y, float angle_deg, float scale, const int16_t *cos_q14,
                              const int16_t *sin_q14, uint8_t *tile);
void oracle_describe_tile(const uint8_t *tile, const uint8_t *triplets, uint32_t *desc);
int oracle_triplets_valid(const uint8_t *triplets);
unsigned oracle_extract(const uint8_t *img, int height, int width, int pitch, const float *kps,
                        int64_t n, const uint8_t *triplets, uint32_t *desc);
int oracle_triplets_valid_geom(const uint8_t *triplets, int win, int k);
unsigned oracle_extract_geom(const uint8_t *img, int height, int width, int pitch,
                             const float *kps, int64_t n, const uint8_t *triplets, int win, int k,
                             const uint8_t *weights, uint32_t *desc);
void oracle_knn_window(const uint32_t *query, const uint32_t *train, int gw, int gh, int radius,
                       int k, float ratio, int32_t *idx, int32_t *dist, uint8_t *accept);
int oracle_hamming(const uint32_t *a, const uint32_t *b);
void oracle_knn(const uint32_t *query, int64_t nq, const uint32_t *train, int64_t nt, int k,
                float ratio, int32_t *idx, int32_t *dist, uint8_t *accept);
int oracle_fast_score(const uint8_t *img, int pitch, int x, int y);
int oracle_orientation_bin(const uint8_t *img, int pitch, int x, int y, int64_t *m10_out,
                           int64_t *m01_out);
int64_t oracle_detect(const uint8_t *img, int height, int width, int pitch, int threshold,
                      float *kps, int64_t max_kps);
void oracle_set_threads(int n);

static uint64_t digest = 1469598103934665603ull;

static void mix(const void *p, size_t n)
{
    const uint8_t *b = (const uint8_t *)p;
    for (size_t i = 0; i < n; ++i) {
        digest ^= b[i];
        digest *= 1099511628211ull;
    }
}

static uint64_t rng = 88172645463325252ull;

static uint32_t next(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (uint32_t)(rng >> 32);
}

/* An image in a buffer of exactly height * pitch bytes (the sanitizer sees
 * any read past it), random bytes smoothed a little so FAST finds corners. */
static uint8_t *image(int height, int width, int pitch)
{
    uint8_t *img = (uint8_t *)malloc((size_t)height * pitch);
    for (int i = 0; i < height * pitch; ++i) img[i] = (uint8_t)next();
    for (int y = 0; y < height; ++y)
        for (int x = 1; x < width; ++x)
            img[y * pitch + x] = (uint8_t)((img[y * pitch + x] + img[y * pitch + x - 1]) / 2);
    return img;
}

static void keypoints(float *kps, int n, int height, int width)
{
    const float special[][4] = {
        {0.0f, 0.0f, 0.0f, 1.0f},           {-300.0f, 5.0f, 45.0f, 2.0f},
        {1e7f, 1e7f, 10.0f, 1.0f},          {17000000.0f, 0.0f, 0.0f, 1.0f},
        {NAN, 3.0f, 0.0f, 1.0f},            {3.0f, INFINITY, 0.0f, 1.0f},
        {3.0f, 3.0f, 2e6f, 1.0f},           {3.0f, 3.0f, -1e6f, 1.0f},
        {3.0f, 3.0f, 0.0f, 0.001f},         {3.0f, 3.0f, 0.0f, 4.0f},
        {3.0f, 3.0f, 0.0f, 4.01f},          {(float)width - 0.5f, (float)height - 0.5f, 359.99f, 3.5f},
        {-0.5f, -0.5f, -90.0f, 1.0f},       {2.5f, 1.5f, 22.5f, 1.44f},
    };
    const int ns = (int)(sizeof special / sizeof special[0]);
    for (int i = 0; i < n; ++i) {
        if (i < ns) {
            memcpy(kps + 4 * i, special[i], sizeof special[i]);
            continue;
        }
        kps[4 * i + 0] = (float)(next() % (unsigned)(width + 60)) - 30.0f + (float)(next() % 4) * 0.25f;
        kps[4 * i + 1] = (float)(next() % (unsigned)(height + 60)) - 30.0f;
        kps[4 * i + 2] = (float)(next() % 7200) * 0.05f - 180.0f;
        kps[4 * i + 3] = 1.0f + (float)(next() % 300) * 0.01f;
    }
}

static void extraction(const uint8_t *triplets)
{
    const int sizes[][3] = {{1, 1, 1}, {1, 7, 9}, {5, 3, 3}, {48, 48, 48}, {64, 80, 96}};
    for (int s = 0; s < 5; ++s) {
        const int h = sizes[s][0], w = sizes[s][1], pitch = sizes[s][2];
        uint8_t *img = image(h, w, pitch);
        const int n = 40;
        float *kps = (float *)malloc(sizeof(float) * 4 * n);
        uint32_t *desc = (uint32_t *)malloc(sizeof(uint32_t) * 16 * n);
        keypoints(kps, n, h, w);
        unsigned f = oracle_extract(img, h, w, pitch, kps, n, triplets, desc);
        mix(&f, sizeof f);
        mix(desc, sizeof(uint32_t) * 16 * n);
        f = oracle_extract(img, h, w, pitch, kps, 0, triplets, desc);   /* empty */
        mix(&f, sizeof f);
        uint8_t weights[64];
        for (int i = 0; i < 64; ++i) weights[i] = (uint8_t)(next() % 129);
        f = oracle_extract_geom(img, h, w, pitch, kps, n, triplets, 64, 8, weights, desc);
        mix(&f, sizeof f);
        mix(desc, sizeof(uint32_t) * 16 * n);
        f = oracle_extract_geom(img, h, w, pitch, kps, n, triplets, 48, 7, weights, desc);
        mix(&f, sizeof f);
        mix(desc, sizeof(uint32_t) * 16 * n);
        int16_t c[4096], sn[4096];
        uint8_t tile[48 * 48];
        oracle_rotation_table(c, sn);
        mix(c, sizeof c);
        mix(sn, sizeof sn);
        f = oracle_sample_window(img, h, w, pitch, kps[4 * 20], kps[4 * 20 + 1], kps[4 * 20 + 2],
                                 kps[4 * 20 + 3], c, sn, tile);
        mix(&f, sizeof f);
        if (!f) {
            oracle_describe_tile(tile, triplets, desc);
            mix(desc, sizeof(uint32_t) * 16);
        }
        free(desc);
        free(kps);
        free(img);
    }
}

static void matching(void)
{
    const int64_t shapes[][2] = {{0, 5}, {3, 0}, {3, 1}, {4, 2}, {17, 33}, {1, 64}};
    for (int s = 0; s < 6; ++s) {
        const int64_t nq = shapes[s][0], nt = shapes[s][1];
        uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * 16 * (size_t)(nq + 1));
        uint32_t *t = (uint32_t *)malloc(sizeof(uint32_t) * 16 * (size_t)(nt + 1));
        for (int64_t i = 0; i < 16 * nq; ++i) q[i] = next() & next();
        for (int64_t i = 0; i < 16 * nt; ++i) t[i] = next() & next();
        if (nt > 1) memcpy(t + 16, t, 64);            /* a duplicate row: a tie */
        int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(nq + 1));
        int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(nq + 1));
        uint8_t *acc = (uint8_t *)malloc((size_t)nq + 1);
        for (int k = 1; k <= 2; ++k) {
            oracle_knn(q, nq, t, nt, k, 0.8f, idx, dist, acc);
            mix(idx, sizeof(int32_t) * k * (size_t)nq);
            mix(dist, sizeof(int32_t) * k * (size_t)nq);
            mix(acc, (size_t)nq);
            oracle_knn(q, nq, t, nt, k, 1.0f, idx, dist, NULL);
            mix(idx, sizeof(int32_t) * k * (size_t)nq);
        }
        if (nq && nt) {
            const int d = oracle_hamming(q, t);
            mix(&d, sizeof d);
        }
        free(acc);
        free(dist);
        free(idx);
        free(t);
        free(q);
    }
    const int grids[][3] = {{1, 1, 0}, {5, 3, 1}, {7, 6, 2}, {2, 9, 12}};
    for (int s = 0; s < 4; ++s) {
        const int gw = grids[s][0], gh = grids[s][1], radius = grids[s][2];
        const int n = gw * gh;
        uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * 16 * (size_t)n);
        uint32_t *t = (uint32_t *)malloc(sizeof(uint32_t) * 16 * (size_t)n);
        for (int i = 0; i < 16 * n; ++i) {
            q[i] = next();
            t[i] = next() | next();
        }
        int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)n);
        int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)n);
        uint8_t *acc = (uint8_t *)malloc((size_t)n);
        for (int k = 1; k <= 2; ++k) {
            oracle_knn_window(q, t, gw, gh, radius, k, 0.75f, idx, dist, acc);
            mix(idx, sizeof(int32_t) * k * (size_t)n);
            mix(dist, sizeof(int32_t) * k * (size_t)n);
            mix(acc, (size_t)n);
        }
        free(acc);
        free(dist);
        free(idx);
        free(t);
        free(q);
    }
}

static void detection(void)
{
    const int sizes[][3] = {{32, 32, 32}, {33, 33, 40}, {33, 60, 64}, {70, 45, 45}, {10, 200, 200}};
    for (int s = 0; s < 5; ++s) {
        const int h = sizes[s][0], w = sizes[s][1], pitch = sizes[s][2];
        uint8_t *img = image(h, w, pitch);
        float kps[4 * 8];
        for (int threshold = 0; threshold <= 40; threshold += 20) {
            const int64_t n = oracle_detect(img, h, w, pitch, threshold, kps, 8);
            mix(&n, sizeof n);
            mix(kps, sizeof(float) * 4 * (size_t)(n < 8 ? n : 8));
        }
        if (h >= 33 && w >= 33) {
            const int sc = oracle_fast_score(img, pitch, 16, 16);
            int64_t m10, m01;
            const int b = oracle_orientation_bin(img, pitch, 16, 16, &m10, &m01);
            mix(&sc, sizeof sc);
            mix(&b, sizeof b);
            mix(&m10, sizeof m10);
            mix(&m01, sizeof m01);
        }
        free(img);
    }
}

int main(void)
{
    oracle_set_threads(2);
    uint8_t triplets[512 * 6];
    for (int i = 0; i < 512 * 6; ++i) triplets[i] = (uint8_t)(4 + next() % 41);   /* [4, 44] */
    if (!oracle_triplets_valid(triplets) || !oracle_triplets_valid_geom(triplets, 64, 8) ||
        !oracle_triplets_valid_geom(triplets, 48, 7)) {
        fprintf(stderr, "triplet table rejected\n");
        return 2;
    }
    extraction(triplets);
    matching();
    detection();
    printf("%016llx\n", (unsigned long long)digest);
    return 0;
}
