/*
 * LATCH oracle: plain, slow CPU implementation of the hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * What it computes (paper: "The CUDA LATCH Binary Descriptor", arXiv 1609.03986):
 *
 *   - Eq. 1 (Sec. 3.1): bit t of the descriptor of keypoint p is 1 iff the
 *     squared Frobenius distance between the anchor patch P_{t,A} and the
 *     first companion P_{t,1} is strictly larger than the distance between
 *     P_{t,A} and the second companion P_{t,2}; k x k patches with k = 7 and
 *     T = 512 triplets (Sec. 3.1, closing paragraph of "The LATCH feature
 *     descriptor").
 *   - Sec. 3.2 "Memory optimization": the rotated window around the oriented
 *     keypoint (x, y, theta) is resampled into an upright square before the
 *     patches are compared.  The paper does not state the resampling, the
 *     window size used here (48), the scale handling or the rounding; this
 *     file fixes them as "rule R" (see oracle_sample_window below), written
 *     out step by step.
 *   - Sec. 3.2 "Weighing pixels in LATCH patches": the CLATCH geometry (64 x 64
 *     windows, 8 x 8 patches) with an integer weight per patch pixel
 *     (oracle_extract_geom).
 *   - Sec. 6: dense per-pixel CLATCH and matching within a search window
 *     (oracle_knn_window; dense extraction is extraction at every pixel).
 *   - Sec. 4 "Descriptor matching on the GPU": exhaustive (brute-force)
 *     Hamming matching.  k = 2 nearest neighbours, ties to the lowest train
 *     index, ratio test d1 < ratio * d2 evaluated exactly.
 *
 * All arithmetic is integer except the three conversions of rule R steps 1-3,
 * which are done in IEEE double.  Integer intermediates are kept in int64 so
 * that no overflow argument is needed here.
 *
 * Parity pins: every function is pinned by the CPU tests against closed
 * forms, invariants and brute force (hand-built tiles, numpy crops, textbook
 * rotation, full sorts); see the test files named test_oracle_*.py.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_WIN 48          /* upright window side, pixels */
#define OR_HALF 24         /* window offset: pixel (i, j) sits at (j - 24, i - 24) */
#define OR_R 3             /* patch radius: 7 x 7 patches */
#define OR_T 512           /* triplets = bits per descriptor */
#define OR_WORDS 16        /* 512 bits as 16 little-endian uint32 words */
#define OR_BINS 4096       /* angle bins of the Q14 rotation table */
#define OR_Q14 16384.0
#define OR_NO_NEIGHBOUR_DIST 513
#define OR_FLAG_BAD_KEYPOINT 1u

/* ------------------------------------------------------------------------ */
/* Rule R, step 2: the Q14 rotation table.                                   */
/* ------------------------------------------------------------------------ */
/*
 * First octant from libm in double, rounded to nearest-even; the other seven
 * octants by the exact symmetries cos(90-a) = sin(a) and a rotation by a
 * quarter turn (C, S) -> (-S, C).  This makes the table exactly symmetric
 * under 90-degree rotations, which is what makes the descriptor of a
 * quarter-turned image bit-identical.
 */
void oracle_rotation_table(int16_t *cos_q14, int16_t *sin_q14)
{
    int16_t c_oct[513], s_oct[513];
    for (int a = 0; a <= 512; ++a) {
        double theta = 2.0 * M_PI * (double)a / (double)OR_BINS;
        c_oct[a] = (int16_t)rint(OR_Q14 * cos(theta));
        s_oct[a] = (int16_t)rint(OR_Q14 * sin(theta));
    }
    for (int a = 0; a < 1024; ++a) {
        if (a <= 512) {
            cos_q14[a] = c_oct[a];
            sin_q14[a] = s_oct[a];
        } else {
            cos_q14[a] = s_oct[1024 - a];
            sin_q14[a] = c_oct[1024 - a];
        }
    }
    for (int a = 1024; a < OR_BINS; ++a) {
        cos_q14[a] = (int16_t)(-sin_q14[a - 1024]);
        sin_q14[a] = cos_q14[a - 1024];
    }
}

/* Round half away from zero of n / 2^22, for any integer n. */
static int64_t round_q22(int64_t n)
{
    int64_t mag = n < 0 ? -n : n;
    int64_t r = (mag + ((int64_t)1 << 21)) >> 22;
    return n < 0 ? -r : r;
}

static int64_t clamp64(int64_t v, int64_t lo, int64_t hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/*
 * Rule R, steps 1-5: resample the 48 x 48 upright window of one keypoint.
 *
 *   1. centre  cx = floor(x + 1/2), cy = floor(y + 1/2), in double;
 *   2. angle   b = rne(angle_deg * (4096/360)) mod 4096, in double;
 *   3. scale   sq = rne(scale * 256), must lie in [1, 1024];
 *   4. offsets for window pixel (i, j), u = j - 24, v = i - 24:
 *        dx = sq * (C[b] u - S[b] v),  dy = sq * (S[b] u + C[b] v)
 *      and ox, oy = dx, dy / 2^22 rounded half away from zero;
 *   5. sample  tile[i][j] = img[clamp(cy + oy, 0, H-1) * pitch
 *                               + clamp(cx + ox, 0, W-1)].
 *
 * Returns 0, or OR_FLAG_BAD_KEYPOINT (tile untouched) when the keypoint is
 * outside the domain of the rule: a non-finite field, |x| or |y| > 2^24,
 * |angle| > 1e6 degrees, or sq outside [1, 1024].
 */
unsigned oracle_sample_window(const uint8_t *img, int height, int width, int pitch,
                              float x, float y, float angle_deg, float scale,
                              const int16_t *cos_q14, const int16_t *sin_q14,
                              uint8_t *tile)
{
    if (!isfinite(x) || !isfinite(y) || !isfinite(angle_deg) || !isfinite(scale))
        return OR_FLAG_BAD_KEYPOINT;
    if (fabs((double)x) > 16777216.0 || fabs((double)y) > 16777216.0)
        return OR_FLAG_BAD_KEYPOINT;
    if (fabs((double)angle_deg) > 1.0e6)
        return OR_FLAG_BAD_KEYPOINT;

    int64_t cx = (int64_t)floor((double)x + 0.5);
    int64_t cy = (int64_t)floor((double)y + 0.5);

    int64_t braw = (int64_t)rint((double)angle_deg * (4096.0 / 360.0));
    int64_t b = ((braw % OR_BINS) + OR_BINS) % OR_BINS;

    int64_t sq = (int64_t)rint((double)scale * 256.0);
    if (sq < 1 || sq > 1024)
        return OR_FLAG_BAD_KEYPOINT;

    int64_t c = cos_q14[b], s = sin_q14[b];
    for (int i = 0; i < OR_WIN; ++i) {
        for (int j = 0; j < OR_WIN; ++j) {
            int64_t u = j - OR_HALF, v = i - OR_HALF;
            int64_t dx = sq * (c * u - s * v);
            int64_t dy = sq * (s * u + c * v);
            int64_t X = clamp64(cx + round_q22(dx), 0, width - 1);
            int64_t Y = clamp64(cy + round_q22(dy), 0, height - 1);
            tile[i * OR_WIN + j] = img[Y * (int64_t)pitch + X];
        }
    }
    return 0;
}

/*
 * Eq. 1 for one triplet on one tile: the two squared Frobenius distances,
 * summed over the 7 x 7 patches centred on the anchor (rA, cA) and on the
 * companions (r1, c1), (r2, c2).  trip = {rA, cA, r1, c1, r2, c2}, each in
 * [3, 44] so that every patch lies inside the 48 x 48 tile.
 */
void oracle_triplet_distances(const uint8_t *tile, const uint8_t *trip,
                              int64_t *dist1, int64_t *dist2)
{
    int rA = trip[0], cA = trip[1];
    int r1 = trip[2], c1 = trip[3];
    int r2 = trip[4], c2 = trip[5];
    int64_t s1 = 0, s2 = 0;
    for (int dr = -OR_R; dr <= OR_R; ++dr) {
        for (int dc = -OR_R; dc <= OR_R; ++dc) {
            int64_t a = tile[(rA + dr) * OR_WIN + (cA + dc)];
            int64_t p = tile[(r1 + dr) * OR_WIN + (c1 + dc)];
            int64_t q = tile[(r2 + dr) * OR_WIN + (c2 + dc)];
            s1 += (a - p) * (a - p);
            s2 += (a - q) * (a - q);
        }
    }
    *dist1 = s1;
    *dist2 = s2;
}

/* Eq. 1 applied to all 512 triplets; bit t goes to word t/32, bit t%32. */
void oracle_describe_tile(const uint8_t *tile, const uint8_t *triplets, uint32_t *desc)
{
    memset(desc, 0, OR_WORDS * sizeof(uint32_t));
    for (int t = 0; t < OR_T; ++t) {
        int64_t s1, s2;
        oracle_triplet_distances(tile, triplets + 6 * t, &s1, &s2);
        if (s1 > s2)
            desc[t / 32] |= (uint32_t)1 << (t % 32);
    }
}

/* Returns 1 if every triplet centre lies in [3, 44], else 0. */
int oracle_triplets_valid(const uint8_t *triplets)
{
    for (int i = 0; i < OR_T * 6; ++i)
        if (triplets[i] < OR_R || triplets[i] > OR_WIN - 1 - OR_R)
            return 0;
    return 1;
}

/*
 * Extraction for n keypoints: kps holds n records {x, y, angle_deg, scale}
 * (float32).  A keypoint outside the domain of rule R gets an all-zero
 * descriptor and sets bit 0 of the returned flag word.
 */
unsigned oracle_extract(const uint8_t *img, int height, int width, int pitch,
                        const float *kps, int64_t n, const uint8_t *triplets,
                        uint32_t *desc)
{
    int16_t cos_q14[OR_BINS], sin_q14[OR_BINS];
    oracle_rotation_table(cos_q14, sin_q14);
    unsigned flags = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : flags)
    for (int64_t p = 0; p < n; ++p) {
        uint8_t tile[OR_WIN * OR_WIN];
        const float *kp = kps + 4 * p;
        unsigned f = oracle_sample_window(img, height, width, pitch, kp[0], kp[1], kp[2],
                                          kp[3], cos_q14, sin_q14, tile);
        if (f) {
            memset(desc + OR_WORDS * p, 0, OR_WORDS * sizeof(uint32_t));
            flags |= f;
        } else {
            oracle_describe_tile(tile, triplets, desc + OR_WORDS * p);
        }
    }
    return flags;
}

/* ------------------------------------------------------------------------ */
/* The paper's CLATCH geometry and per-pixel patch weights (Sec. 3.2).       */
/* ------------------------------------------------------------------------ */
/*
 * Sec. 3.2 extracts CLATCH from 64 x 64 windows with 8 x 8 patches, and lets
 * each patch pixel carry an integer weight ("Weighing pixels in LATCH
 * patches"): zero weights on one row and one column of the 8 x 8 patch give
 * the original 7 x 7 LATCH, and Gaussian weights are suggested.  The
 * functions below generalise the window side (win, even) and the patch side
 * (k), and replace Eq. 1's plain sums by weighted ones:
 *
 *   S_j = sum over (a, b) in [0, k)^2 of w[a][b] * (A[a][b] - P_j[a][b])^2,
 *   bit = [S_1 > S_2],
 *
 * where the patch of a triplet centre (r, c) has its top-left pixel at
 * (r - k/2, c - k/2) (for k = 7 that is the 7 x 7 patch centred on (r, c);
 * for k = 8 the centre is the pixel right and below the middle).  Rule R is
 * unchanged except that window pixel (i, j) sits at (j - win/2, i - win/2).
 */
unsigned oracle_sample_window_geom(const uint8_t *img, int height, int width, int pitch,
                                   float x, float y, float angle_deg, float scale,
                                   const int16_t *cos_q14, const int16_t *sin_q14, int win,
                                   uint8_t *tile)
{
    if (!isfinite(x) || !isfinite(y) || !isfinite(angle_deg) || !isfinite(scale))
        return OR_FLAG_BAD_KEYPOINT;
    if (fabs((double)x) > 16777216.0 || fabs((double)y) > 16777216.0)
        return OR_FLAG_BAD_KEYPOINT;
    if (fabs((double)angle_deg) > 1.0e6)
        return OR_FLAG_BAD_KEYPOINT;
    int64_t sq = (int64_t)rint((double)scale * 256.0);
    if (sq < 1 || sq > 1024)
        return OR_FLAG_BAD_KEYPOINT;
    int64_t cx = (int64_t)floor((double)x + 0.5);
    int64_t cy = (int64_t)floor((double)y + 0.5);
    int64_t braw = (int64_t)rint((double)angle_deg * (4096.0 / 360.0));
    int64_t b = ((braw % OR_BINS) + OR_BINS) % OR_BINS;
    int64_t c = cos_q14[b], s = sin_q14[b];
    int half = win / 2;
    for (int i = 0; i < win; ++i)
        for (int j = 0; j < win; ++j) {
            int64_t u = j - half, v = i - half;
            int64_t X = clamp64(cx + round_q22(sq * (c * u - s * v)), 0, width - 1);
            int64_t Y = clamp64(cy + round_q22(sq * (s * u + c * v)), 0, height - 1);
            tile[i * win + j] = img[Y * (int64_t)pitch + X];
        }
    return 0;
}

/* Weighted patch distances of one triplet on a win x win tile. */
void oracle_triplet_distances_weighted(const uint8_t *tile, int win, int k, const uint8_t *weights,
                                       const uint8_t *trip, int64_t *dist1, int64_t *dist2)
{
    int top[3], left[3];
    for (int p = 0; p < 3; ++p) {
        top[p] = trip[2 * p] - k / 2;
        left[p] = trip[2 * p + 1] - k / 2;
    }
    int64_t s1 = 0, s2 = 0;
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            int64_t w = weights[a * k + b];
            int64_t A = tile[(top[0] + a) * win + left[0] + b];
            int64_t P = tile[(top[1] + a) * win + left[1] + b];
            int64_t Q = tile[(top[2] + a) * win + left[2] + b];
            s1 += w * (A - P) * (A - P);
            s2 += w * (A - Q) * (A - Q);
        }
    *dist1 = s1;
    *dist2 = s2;
}

/* 1 if every patch of every triplet lies inside the win x win tile. */
int oracle_triplets_valid_geom(const uint8_t *triplets, int win, int k)
{
    for (int i = 0; i < OR_T * 6; ++i) {
        int first = triplets[i] - k / 2;
        if (first < 0 || first + k > win)
            return 0;
    }
    return 1;
}

/* Extraction with window side win, patch side k and weights[k][k]. */
unsigned oracle_extract_geom(const uint8_t *img, int height, int width, int pitch,
                             const float *kps, int64_t n, const uint8_t *triplets, int win, int k,
                             const uint8_t *weights, uint32_t *desc)
{
    int16_t cos_q14[OR_BINS], sin_q14[OR_BINS];
    oracle_rotation_table(cos_q14, sin_q14);
    unsigned flags = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : flags)
    for (int64_t p = 0; p < n; ++p) {
        uint8_t *tile = (uint8_t *)malloc((size_t)win * win);
        const float *kp = kps + 4 * p;
        uint32_t *d = desc + OR_WORDS * p;
        memset(d, 0, OR_WORDS * sizeof(uint32_t));
        unsigned f = oracle_sample_window_geom(img, height, width, pitch, kp[0], kp[1], kp[2],
                                               kp[3], cos_q14, sin_q14, win, tile);
        if (f) {
            flags |= f;
        } else {
            for (int t = 0; t < OR_T; ++t) {
                int64_t s1, s2;
                oracle_triplet_distances_weighted(tile, win, k, weights, triplets + 6 * t, &s1, &s2);
                if (s1 > s2)
                    d[t / 32] |= (uint32_t)1 << (t % 32);
            }
        }
        free(tile);
    }
    return flags;
}

int oracle_hamming(const uint32_t *a, const uint32_t *b);

/* ------------------------------------------------------------------------ */
/* Dense matching (Sec. 6: CLATCH for dense pixel matching).                 */
/* ------------------------------------------------------------------------ */
/*
 * query and train are descriptor grids of gh rows and gw columns (row-major,
 * 16 words per pixel).  For query pixel (y, x) the candidates are the train
 * pixels (y', x') with |y' - y| <= radius and |x' - x| <= radius inside the
 * grid, scanned in raster order; the k = 1 or 2 nearest by Hamming distance,
 * ties to the lower raster index y' gw + x', and the ratio test as in
 * oracle_knn.  idx holds raster indices (-1 and distance 513 when missing).
 */
void oracle_knn_window(const uint32_t *query, const uint32_t *train, int gw, int gh, int radius,
                       int k, float ratio, int32_t *idx, int32_t *dist, uint8_t *accept)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < (int64_t)gw * gh; ++q) {
        int y = (int)(q / gw), x = (int)(q % gw);
        int b1 = -1, b2 = -1, d1 = OR_NO_NEIGHBOUR_DIST, d2 = OR_NO_NEIGHBOUR_DIST;
        int n = 0;
        for (int yy = y - radius; yy <= y + radius; ++yy) {
            if (yy < 0 || yy >= gh) continue;
            for (int xx = x - radius; xx <= x + radius; ++xx) {
                if (xx < 0 || xx >= gw) continue;
                int j = yy * gw + xx;
                int d = oracle_hamming(query + OR_WORDS * q, train + OR_WORDS * (int64_t)j);
                ++n;
                if (d < d1) {
                    b2 = b1; d2 = d1;
                    b1 = j; d1 = d;
                } else if (d < d2) {
                    b2 = j; d2 = d;
                }
            }
        }
        idx[k * q] = b1;
        dist[k * q] = d1;
        if (k == 2) {
            idx[k * q + 1] = b2;
            dist[k * q + 1] = d2;
        }
        if (accept)
            accept[q] = (uint8_t)(n >= 2 && (double)d1 < (double)ratio * (double)d2);
    }
}

/* Hamming distance between two 512-bit descriptors. */
int oracle_hamming(const uint32_t *a, const uint32_t *b)
{
    int d = 0;
    for (int w = 0; w < OR_WORDS; ++w)
        d += __builtin_popcount(a[w] ^ b[w]);
    return d;
}

/*
 * Brute-force k-NN (k = 1 or 2) under Hamming distance.  For each query the
 * two lexicographically smallest (distance, train index) pairs are found by
 * a plain scan in index order.  Missing neighbours (nt < k) get index -1 and
 * distance 513.  accept[q] = (nt >= 2) && d1 < ratio * d2, exactly (float32
 * ratio times an integer <= 512 is exact in double).  accept may be NULL.
 */
void oracle_knn(const uint32_t *query, int64_t nq, const uint32_t *train, int64_t nt,
                int k, float ratio, int32_t *idx, int32_t *dist, uint8_t *accept)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nq; ++q) {
        int64_t j1 = -1, j2 = -1;
        int d1 = OR_NO_NEIGHBOUR_DIST, d2 = OR_NO_NEIGHBOUR_DIST;
        for (int64_t j = 0; j < nt; ++j) {
            int d = oracle_hamming(query + OR_WORDS * q, train + OR_WORDS * j);
            if (d < d1) {
                d2 = d1;
                j2 = j1;
                d1 = d;
                j1 = j;
            } else if (d < d2) {
                d2 = d;
                j2 = j;
            }
        }
        idx[q * k] = (int32_t)j1;
        dist[q * k] = d1;
        if (k == 2) {
            idx[q * k + 1] = (int32_t)j2;
            dist[q * k + 1] = d2;
        }
        if (accept)
            accept[q] = (uint8_t)(nt >= 2 && (double)d1 < (double)ratio * (double)d2);
    }
}

/*
 * Keypoint detection (Sec. 3.2: the paper detects FAST keypoints and uses
 * their orientation; neither the FAST score, the suppression nor the
 * orientation method is stated, so this file fixes them):
 *
 *   - FAST-9 segment test (Rosten and Drummond): the 16 pixels of the
 *     radius-3 circle around p, clockwise from the top.  With c = I(p), the
 *     score is the largest, over the 16 arcs of 9 consecutive circle pixels
 *     and over both polarities, of the smallest difference on the arc
 *     (I(q) - c for "brighter", c - I(q) for "darker").  p is a corner for
 *     threshold t iff its score is > t, i.e. iff some arc of 9 is entirely
 *     brighter than c + t or entirely darker than c - t.
 *   - Only pixels at least DETECT_BORDER from every image edge are tested.
 *     S(p) = score(p) for a corner there, 0 otherwise.  Suppression keeps p
 *     iff S(p) > 0 and S(p) > S(q) for its 8 neighbours.
 *   - Orientation: intensity-centroid moments m10 = sum dx I, m01 = sum dy I
 *     over the disc dx^2 + dy^2 <= ORIENT_RADIUS^2 (y downwards, so angles
 *     turn clockwise on screen, as in the resampling rule), angle bin
 *     b = rne(atan2(m01, m10) * 4096 / 2 pi) mod 4096 in double, and the
 *     keypoint angle b * 360 / 4096 degrees (exact in float), scale 1.
 *   - Keypoints in raster order (y, then x).
 */
#define DETECT_BORDER 16
#define ORIENT_RADIUS 15

static const int fast_circle[16][2] = {
    {0, -3}, {1, -3}, {2, -2}, {3, -1}, {3, 0}, {3, 1}, {2, 2}, {1, 3},
    {0, 3}, {-1, 3}, {-2, 2}, {-3, 1}, {-3, 0}, {-3, -1}, {-2, -2}, {-1, -3}};

/* FAST-9 score of pixel (x, y); the caller keeps the circle inside the image. */
int oracle_fast_score(const uint8_t *img, int pitch, int x, int y)
{
    const int c = img[(int64_t)y * pitch + x];
    int best = -256;
    for (int polarity = 0; polarity < 2; ++polarity) {
        int d[16];
        for (int i = 0; i < 16; ++i) {
            const int q = img[(int64_t)(y + fast_circle[i][1]) * pitch + x + fast_circle[i][0]];
            d[i] = polarity == 0 ? q - c : c - q;
        }
        for (int k = 0; k < 16; ++k) {
            int m = 256;
            for (int j = 0; j < 9; ++j) {
                const int v = d[(k + j) % 16];
                if (v < m) m = v;
            }
            if (m > best) best = m;
        }
    }
    return best;
}

/* Orientation bin of pixel (x, y) from its intensity centroid. */
int oracle_orientation_bin(const uint8_t *img, int pitch, int x, int y, int64_t *m10_out,
                           int64_t *m01_out)
{
    int64_t m10 = 0, m01 = 0;
    for (int dy = -ORIENT_RADIUS; dy <= ORIENT_RADIUS; ++dy)
        for (int dx = -ORIENT_RADIUS; dx <= ORIENT_RADIUS; ++dx) {
            if (dx * dx + dy * dy > ORIENT_RADIUS * ORIENT_RADIUS) continue;
            const int v = img[(int64_t)(y + dy) * pitch + x + dx];
            m10 += (int64_t)dx * v;
            m01 += (int64_t)dy * v;
        }
    if (m10_out) *m10_out = m10;
    if (m01_out) *m01_out = m01;
    const double a = atan2((double)m01, (double)m10);
    return (int)((int64_t)rint(a * (4096.0 / (2.0 * 3.14159265358979323846))) & 4095);
}

/* Detect: writes up to max_kps keypoints (x, y, angle_deg, 1) in raster
 * order to kps (float[max_kps][4]) and returns the number of corners found,
 * which may exceed max_kps. */
int64_t oracle_detect(const uint8_t *img, int height, int width, int pitch, int threshold,
                      float *kps, int64_t max_kps)
{
    if (height < 2 * DETECT_BORDER + 1 || width < 2 * DETECT_BORDER + 1) return 0;
    int *S = (int *)calloc((size_t)height * width, sizeof(int));
    if (!S) return -1;
#pragma omp parallel for schedule(dynamic, 8)
    for (int y = DETECT_BORDER; y < height - DETECT_BORDER; ++y)
        for (int x = DETECT_BORDER; x < width - DETECT_BORDER; ++x) {
            const int sc = oracle_fast_score(img, pitch, x, y);
            S[(int64_t)y * width + x] = sc > threshold ? sc : 0;
        }
    int64_t n = 0;
    for (int y = DETECT_BORDER; y < height - DETECT_BORDER; ++y)
        for (int x = DETECT_BORDER; x < width - DETECT_BORDER; ++x) {
            const int s0 = S[(int64_t)y * width + x];
            if (s0 <= 0) continue;
            int keep = 1;
            for (int dy = -1; dy <= 1 && keep; ++dy)
                for (int dx = -1; dx <= 1; ++dx)
                    if ((dx || dy) && S[(int64_t)(y + dy) * width + x + dx] >= s0) {
                        keep = 0;
                        break;
                    }
            if (!keep) continue;
            if (n < max_kps) {
                const int b = oracle_orientation_bin(img, pitch, x, y, 0, 0);
                kps[4 * n + 0] = (float)x;
                kps[4 * n + 1] = (float)y;
                kps[4 * n + 2] = (float)b * (360.0f / 4096.0f);
                kps[4 * n + 3] = 1.0f;
            }
            ++n;
        }
    free(S);
    return n;
}

/* Number of OpenMP threads the parallel loops above use. */
int oracle_num_threads(void)
{
    return omp_get_max_threads();
}

/* Sets that number (n >= 1); used to time the oracle on one core. */
void oracle_set_threads(int n)
{
    omp_set_num_threads(n < 1 ? 1 : n);
}
