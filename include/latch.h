/*
 * latch.h - C ABI of the gfx950 LATCH extraction + Hamming matching library.
 *
 * The library computes, on one MI355X (gfx950) GPU:
 *   - LATCH binary descriptors (paper: "The CUDA LATCH Binary Descriptor",
 *     arXiv 1609.03986, Sec. 3.1 Eq. 1 and Sec. 3.2): for each oriented,
 *     scaled keypoint, 512 bits, bit t = [ ||P_A - P_1||^2 > ||P_A - P_2||^2 ]
 *     over 7 x 7 patches of triplet t inside a 48 x 48 window resampled
 *     upright around the keypoint;
 *   - brute-force 2-NN Hamming matching of such descriptors with a ratio
 *     test (Sec. 4, "Descriptor matching on the GPU").
 *
 * Conventions shared by every call:
 *   - All buffers named *_dev are device pointers owned by the caller; the
 *     library never frees or retains them past the call's stream work.
 *   - Every call that takes a stream only enqueues work on that stream and
 *     returns; results are ready when the stream reaches that point.  The
 *     work calls (extraction, detection, matching, plan runs) never allocate,
 *     free or synchronise.  The calls that wait, and for what:
 *       latch_create, latch_create_geometry: their own table uploads, on a
 *         private stream (nothing the caller enqueued);
 *       latch_reserve: the whole device, only when it replaces a smaller
 *         workspace (work on any stream may still use the old one);
 *       latch_plan_create: its own capture stream (no device work runs);
 *       latch_check_errors: the given stream;
 *       latch_timing_enable, latch_timing_read: the recorded events;
 *       latch_destroy, latch_plan_destroy: the whole device.
 *   - A handle owns device copies of the rotation table and triplet table,
 *     a sticky error word and a workspace that only latch_reserve sizes.
 *     hamming_knn (with more than one train split), hamming_knn_batch,
 *     latch_detect and large batched extractions need workspace; the
 *     *_workspace_size calls give the bytes
 *     for given sizes, and a call whose need exceeds what the handle holds
 *     returns LATCH_EWORKSPACE and enqueues nothing.  A handle is not
 *     thread-safe, and work enqueued through one handle on different streams
 *     shares its workspace: order such calls yourself or use one handle per
 *     stream.
 *   - Return values: LATCH_OK (0) or a negative latch_status.  Host-checkable
 *     argument errors are reported synchronously and enqueue nothing.
 *
 * Resampling rule (the paper states that the rotated window is loaded as an
 * upright square but not how; this library fixes the rule below, exactly):
 *   1. cx = floor(x + 1/2), cy = floor(y + 1/2), evaluated in double;
 *   2. b = rne(angle_deg * (4096/360)) mod 4096 (double multiply, round to
 *      nearest even), an index into a Q14 table of cos/sin whose first octant
 *      is rne(16384 cos), rne(16384 sin) of 2 pi a / 4096 and whose other
 *      octants follow from the exact symmetries (see latch_rotation_table);
 *   3. sq = rne(scale * 256), which must lie in [1, 1024];
 *   4. window pixel (i, j), i, j in [0, 47], with u = j - 24, v = i - 24,
 *      samples offsets ox, oy = sq (C u - S v), sq (S u + C v) divided by 2^22
 *      and rounded half away from zero;
 *   5. the sample is img[clamp(cy + oy, 0, H-1) * pitch + clamp(cx + ox, 0, W-1)]
 *      (clamp-to-edge borders, nearest sampling).
 * Angles are in degrees and rotate (u right, v down) clockwise on screen.
 */
#ifndef LATCH_H
#define LATCH_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LATCH_WINDOW 48          /* side of the upright window, pixels */
#define LATCH_PATCH 7            /* patch side k (Sec. 3.1) */
#define LATCH_TRIPLETS 512       /* bits per descriptor (Sec. 3.1) */
#define LATCH_DESC_WORDS 16      /* 512 bits as uint32[16]; bit t in word t/32, bit t%32 */
#define LATCH_ANGLE_BINS 4096
#define LATCH_NO_NEIGHBOUR_DIST 513
#define LATCH_MAX_ROWS 2147483647LL

/* Keypoint record, 16 bytes.  Pixel centres are at integer coordinates. */
typedef struct {
    float x, y;        /* position in pixels */
    float angle_deg;   /* orientation, degrees, |angle| <= 1e6 */
    float scale;       /* window scale; rne(scale * 256) in [1, 1024] */
} latch_keypoint;

typedef struct latch_ctx *latch_handle;

typedef enum {
    LATCH_OK = 0,
    LATCH_EINVAL = -1,   /* bad argument (null pointer, negative or too large size, ...) */
    LATCH_ENOMEM = -2,   /* device allocation failed */
    LATCH_EDEVICE = -3,  /* a HIP runtime call failed */
    LATCH_ERANGE = -4,   /* a value outside its documented range (triplet centre, k, ratio) */
    LATCH_EWORKSPACE = -5  /* the handle's workspace is smaller than the call needs: reserve
                              the size the matching *_workspace_size call gives, then retry */
} latch_status;

typedef enum {
    LATCH_PATH_AUTO = 0,      /* the library chooses */
    LATCH_PATH_MFMA = 1,      /* int8 MFMA: sum of (2a - 1) b over 0/1 bits = |a| - Hamming */
    LATCH_PATH_POPCOUNT = 2,  /* XOR + popcount */
    LATCH_PATH_MFMA_FP4 = 3   /* block-scaled FP4 MFMA (values 0, +-1 are exact in e2m1; sums
                                 accumulate exactly in f32): twice the int8 MFMA rate */
} latch_path;

/* Bits of the sticky device error word. */
#define LATCH_FLAG_BAD_KEYPOINT 1u  /* a keypoint outside the resampling rule's domain; its descriptor is all zero */
#define LATCH_FLAG_BAD_IMAGE 2u     /* batched extraction: image id out of range or malformed image entry */
#define LATCH_FLAG_BAD_PAIR 4u      /* batched matching: a pair outside its arrays (skipped, outputs untouched) */

/* One image of a batched extraction (device memory), 24 bytes. */
typedef struct {
    const uint8_t *img;   /* device pointer: row-major u8 image */
    int32_t height;       /* rows, in [1, 2^23) */
    int32_t width;        /* columns, >= 1 */
    int32_t pitch;        /* bytes per row, in [width, 2^23); height * pitch < 2^31 */
    int32_t reserved;     /* set to 0 */
} latch_image;

/*
 * Create a handle on the current HIP device.
 *   triplets_host: host array uint8[512][3][2]: for triplet t, the (row, col)
 *     window coordinates of the anchor, companion 1 and companion 2 (the order
 *     of Eq. 1).  Every value must lie in [3, 44] so that each 7 x 7 patch lies
 *     inside the 48 x 48 window (LATCH_ERANGE otherwise).  Copied; the caller
 *     keeps ownership.
 * On success *h receives the handle.  Allocates device memory (LATCH_ENOMEM).
 */
int latch_create(latch_handle *h, const uint8_t *triplets_host);

/*
 * Create a handle whose extraction uses another window and patch geometry and
 * per-pixel integer patch weights (Sec. 3.2: the paper's CLATCH extracts from
 * 64 x 64 windows with 8 x 8 patches, each patch pixel optionally weighted;
 * zero weights on one row and column reproduce the 7 x 7 patch, and Gaussian
 * weights are suggested).  Bit t is [S_1 > S_2] with
 *     S_j = sum_{a,b < patch} w[a][b] (A[a][b] - P_j[a][b])^2,
 * where the patch of centre (r, c) has its top-left pixel at
 * (r - patch/2, c - patch/2), and window pixel (i, j) is sampled at offset
 * (j - window/2, i - window/2) by the same resampling rule.
 *   window:       48 or 64; patch: 7 or 8 (LATCH_ERANGE otherwise).
 *   triplets_host: uint8[512][3][2] centres as for latch_create, each with its
 *                 patch inside the window: r - patch/2 >= 0 and
 *                 r - patch/2 + patch <= window (LATCH_ERANGE otherwise).
 *   weights_host: uint8[patch][patch] row-major, each in [0, 128]
 *                 (LATCH_ERANGE otherwise), or NULL for all ones.  Copied.
 * 48 / 7 / all ones is the latch_create handle.  Any other geometry runs a
 * second extraction kernel (16-bit packed arithmetic, exact), for
 * latch_extract, latch_extract_batch and plans alike; matching is unchanged.
 */
int latch_create_geometry(latch_handle *h, const uint8_t *triplets_host, int window, int patch,
                          const uint8_t *weights_host);

/* Release a handle and its device memory (synchronises the device first).  NULL is a no-op. */
void latch_destroy(latch_handle h);

/*
 * Workspace sizes (host arithmetic only: no GPU work, no synchronisation).
 * *bytes receives the device workspace the call with these arguments needs
 * on this handle, 0 when it needs none.
 *   hamming_knn_workspace_size: the train rows are split over workgroups
 *     (Sec. 4 streams the gallery through the matcher in parts); with more
 *     than one split, 16 bytes per (query, split) of partial top-2 keys.
 *     The split count depends on nq, nt, the path (LATCH_PATH_AUTO resolved
 *     by the handle's current tuning table) and the tuning's workgroup
 *     targets, so query after latch_set_tuning.
 *   hamming_knn_batch_workspace_size: the pair table's per-pair state and
 *     the work-item list of the persistent matcher.
 *   latch_detect_workspace_size: survivor masks, counts and row offsets of
 *     an image of height x width.
 *   latch_extract_batch_workspace_size: a latch_create handle orders a batch
 *     of at least 2^18 keypoints (max_kps) over at most 65536 images by
 *     (image, band of rows) before extracting it, so that each XCD's L2
 *     holds the image rows its workgroups read; 12 bytes per keypoint plus
 *     about 256 bytes per image for the counting sort.  0 for smaller
 *     batches and for geometry handles (extracted in the given order).
 * LATCH_EINVAL for a NULL pointer or sizes outside the limits of the call.
 */
int hamming_knn_workspace_size(latch_handle h, int64_t nq, int64_t nt, int path, size_t *bytes);
int hamming_knn_batch_workspace_size(latch_handle h, int n_pairs, int64_t out_rows, size_t *bytes);
int latch_detect_workspace_size(latch_handle h, int height, int width, size_t *bytes);
int latch_extract_batch_workspace_size(latch_handle h, int n_images, int64_t max_kps,
                                       size_t *bytes);

/*
 * Make the handle's workspace at least `bytes` (a set-up call, made before
 * the work calls that need it, e.g. once per serving slot for its largest
 * request, or before capturing a graph).  A handle that holds at least
 * `bytes` is left as it is.  Otherwise a new buffer of `bytes` (rounded up
 * to 256) is allocated with hipMalloc; when a smaller one exists, the call
 * first waits for the whole device and frees it.  *held_out (may be NULL)
 * receives the size now held, so latch_reserve(h, 0, &held) only reports.
 * LATCH_ENOMEM if the allocation fails (the handle then holds no workspace).
 * A HIP graph captured from calls that use the workspace holds its address:
 * reserve enough before capturing, since a later reservation that replaces
 * the buffer invalidates such graphs.
 */
int latch_reserve(latch_handle h, size_t bytes, size_t *held_out);

/*
 * Extract LATCH descriptors (Sec. 3.1 Eq. 1; window resampling per rule 1-5 above).
 *   img_dev:  uint8 image, row-major, height rows of `pitch` bytes (pitch >= width);
 *             height and pitch must be < 2^23 and height * pitch < 2^31
 *             (LATCH_EINVAL otherwise).
 *   kps_dev:  latch_keypoint[n_kps].
 *   desc_dev: uint32[n_kps][16] output.
 * n_kps == 0 is a no-op.  A keypoint outside the rule's domain (non-finite
 * field, |x| or |y| > 2^24, |angle| > 1e6, rne(scale*256) outside [1, 1024])
 * gets an all-zero descriptor and sets LATCH_FLAG_BAD_KEYPOINT in the sticky
 * error word (read it with latch_check_errors).
 */
int latch_extract(latch_handle h, const uint8_t *img_dev, int height, int width, int pitch,
                  const latch_keypoint *kps_dev, int64_t n_kps, uint32_t *desc_dev,
                  hipStream_t stream);

/*
 * Batched extraction: keypoints of many images of uneven size and count in
 * one launch (Sec. 4 "CUDA Integration" runs several images concurrently on
 * streams; here they share one persistent grid).  Same rule and result per
 * keypoint as latch_extract on its own image.
 *   images_dev:   latch_image[n_images], device memory (the caller's work list).
 *   image_id_dev: int32[max_kps], device memory: image of each keypoint.
 *   kps_dev:      latch_keypoint[max_kps]; desc_dev: uint32[max_kps][16].
 *   n_kps_dev:    NULL (process max_kps keypoints) or a device int64 holding
 *                 the count to process this time, capped at max_kps.  With it,
 *                 a captured HIP graph can be replayed over new batch contents.
 * A keypoint whose image id is outside [0, n_images), or whose image entry
 * violates the limits above or has a NULL pointer, gets an all-zero
 * descriptor and sets LATCH_FLAG_BAD_IMAGE.  Host-checked: max_kps in
 * [0, 2^31), n_images >= 1 when max_kps > 0, non-NULL buffers (LATCH_EINVAL).
 * Large batches use the handle's workspace for their spatial order
 * (latch_extract_batch_workspace_size; LATCH_EWORKSPACE if it holds less);
 * the descriptors do not depend on it.
 */
int latch_extract_batch(latch_handle h, const latch_image *images_dev, int n_images,
                        const int32_t *image_id_dev, const latch_keypoint *kps_dev,
                        int64_t max_kps, const int64_t *n_kps_dev, uint32_t *desc_dev,
                        hipStream_t stream);

/*
 * Dense CLATCH (Sec. 6 proposes CLATCH for dense pixel matching): the
 * descriptor of every pixel (x, y) of the region [x0, x0 + gw) x [y0, y0 + gh),
 * upright and at scale 1 -- exactly latch_extract at the keypoints
 * (x, y, 0, 1) -- computed with box filters over the region instead of per
 * keypoint.  Needs a latch_create handle (LATCH_EINVAL for a geometry handle).
 *   img_dev: as latch_extract.  The region may extend past the image (samples
 *            clamp to the edge); |x0|, |y0|, x0 + gw, y0 + gh <= 2^24 and
 *            gw * gh < 2^31 (LATCH_ERANGE otherwise).
 *   desc_dev: uint32[gh][gw][16], raster order.
 */
int latch_extract_dense(latch_handle h, const uint8_t *img_dev, int height, int width, int pitch,
                        int x0, int y0, int gw, int gh, uint32_t *desc_dev, hipStream_t stream);

/*
 * Dense matching of two descriptor grids of gh rows and gw columns (Sec. 6):
 * for query pixel (y, x), the k = 1 or 2 nearest train pixels by Hamming
 * distance among (y', x') with |y' - y| <= radius, |x' - x| <= radius inside
 * the grid; ties to the lower raster index; accept = at least two candidates
 * and d1 < ratio * d2 (exact).  idx holds raster indices y' gw + x' (-1 and
 * distance 513 when missing).
 *   query_dev, train_dev: uint32[gh][gw][16]; radius in [0, 8] (LATCH_ERANGE).
 *   idx_dev, dist_dev: int32[gh * gw][k]; accept_dev: uint8[gh * gw] or NULL.
 */
int hamming_knn_window(latch_handle h, const uint32_t *query_dev, const uint32_t *train_dev, int gw,
                       int gh, int radius, int k, float ratio, int32_t *idx_dev, int32_t *dist_dev,
                       uint8_t *accept_dev, hipStream_t stream);

/*
 * Keypoint detection (Sec. 3.2: the paper extracts LATCH at FAST keypoints
 * and their orientation; score, suppression and orientation method are
 * not stated there and are fixed as follows).
 *   - FAST-9: for the 16 pixels of the radius-3 circle around p and c the
 *     value at p, score = the largest, over the 16 arcs of 9 consecutive
 *     circle pixels and both polarities, of the smallest difference on the
 *     arc (q - c brighter, c - q darker); p is a corner iff score > threshold.
 *   - Only pixels at least 16 from every edge are tested.  Suppression keeps
 *     a corner whose score exceeds that of every corner among its 8
 *     neighbours (strictly).
 *   - Orientation: m10 = sum dx I, m01 = sum dy I over the disc of radius 15
 *     (y downwards); angle bin b = rne(atan2(m01, m10) * 4096 / 2 pi) mod
 *     4096 in double; angle_deg = b * 360 / 4096 (exact, so extraction uses
 *     bin b); scale 1.
 *   img_dev:    u8, height x width, row stride pitch (limits as latch_extract).
 *   threshold:  in [0, 255] (LATCH_ERANGE otherwise).
 *   kps_dev:    latch_keypoint[max_kps].  The image's keypoints are appended
 *               in raster order (y, then x) after the n0 already there, as far
 *               as max_kps allows.
 *   n_kps_dev:  one int64 (device), in/out: n0 on entry (zero for a fresh
 *               array; a negative value is taken as zero), n0 plus the number of keypoints found on exit, which
 *               may exceed max_kps.  Detecting several images in turn into
 *               one array, then latch_extract_batch with this count, runs
 *               detection and extraction with no host round trip.
 *   image_id_dev: int32[max_kps] or NULL: if given, image_index is written
 *               for every keypoint written.
 * Uses the handle's workspace (latch_detect_workspace_size: about
 * 8 * height * ceil(width / 64) + 8 * height + 16 * height * ceil(ceil(width / 64) / 16)
 * bytes; LATCH_EWORKSPACE if the handle holds less); images below 33 x 33
 * have no keypoints.  Calls that share a handle or a count must be ordered
 * (one stream).
 */
int latch_detect(latch_handle h, const uint8_t *img_dev, int height, int width, int pitch,
                 int threshold, latch_keypoint *kps_dev, int64_t max_kps, int64_t *n_kps_dev,
                 int32_t *image_id_dev, int32_t image_index, hipStream_t stream);

/*
 * Brute-force k-NN under Hamming distance (Sec. 4, "Descriptor matching on the GPU").
 *   query_dev: uint32[nq][16], train_dev: uint32[nt][16] descriptors.
 *   k:         1 or 2 (LATCH_ERANGE otherwise).
 *   ratio:     in (0, 1] (LATCH_ERANGE otherwise).
 *   idx_dev, dist_dev: int32[nq][k] outputs: for each query the k
 *              lexicographically smallest (distance, train index) pairs; ties
 *              go to the lowest train index.  Missing neighbours (nt < k) get
 *              index -1 and distance 513.
 *   accept_dev: uint8[nq] or NULL: 1 iff nt >= 2 and d1 < ratio * d2, evaluated
 *              exactly (the second neighbour is always searched, also for k = 1).
 *   path:      a latch_path value; every path returns identical results.  With more
 *              than 65,535 x 16,384 train rows the MXFP4 path (whose keys hold a
 *              14-bit split-local index) runs the int8 MFMA kernel instead.
 * nq == 0 is a no-op.  nq and nt must be < 2^31.  The train rows are split
 * over workgroups; with more than one split a merge kernel follows and the
 * partials live in the handle's workspace (hamming_knn_workspace_size;
 * LATCH_EWORKSPACE if the handle holds less).  Calls on one handle must not
 * overlap in time on different streams.
 */
int hamming_knn(latch_handle h, const uint32_t *query_dev, int64_t nq,
                const uint32_t *train_dev, int64_t nt, int k, float ratio,
                int32_t *idx_dev, int32_t *dist_dev, uint8_t *accept_dev, int path,
                hipStream_t stream);

/*
 * Allocation-free hamming_knn, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, checks and results as hamming_knn, but the
 * split partials live in a static device array of LATCH_NOALLOC_SCRATCH_BYTES
 * that the library holds on every GPU it runs on until the process ends, not
 * in the handle's workspace: the call never allocates, frees or reserves, and
 * records no timing events.  The split plan is hamming_knn's (the one
 * hamming_knn_workspace_size prices), except that the extra splits the
 * planner may add to fill the last round of workgroups are taken only while
 * the partials fit the scratch; a call whose partials exceed the scratch even
 * without them (16 bytes per (query, train split) when the train rows are
 * split) returns LATCH_ERANGE and enqueues nothing.  Every call on one GPU shares that GPU's scratch:
 * calls that overlap in time on one GPU (any handle, any stream) race, so
 * order them on one stream.  The scratch keeps the last call's contents;
 * nothing in it needs to start at zero.
 */
#define LATCH_NOALLOC_SCRATCH_BYTES (16u << 20)
int hamming_knn_noalloc(latch_handle h, const uint32_t *query_dev, int64_t nq,
                        const uint32_t *train_dev, int64_t nt, int k, float ratio,
                        int32_t *idx_dev, int32_t *dist_dev, uint8_t *accept_dev, int path,
                        hipStream_t stream);

/* One pair of a batched matching (device memory), 40 bytes. */
typedef struct {
    int64_t query_first;  /* first row of this pair's queries in query_dev */
    int64_t nq;           /* query rows, >= 0 */
    int64_t train_first;  /* first row of its train descriptors in train_dev */
    int64_t nt;           /* train rows, in [0, 2^21 - 32] */
    int64_t out_first;    /* first output row in idx/dist (rows of k) and accept */
} latch_pair;

/*
 * Batched brute-force 2-NN: many (query range, train range) pairs in one
 * persistent launch, e.g. the consecutive image pairs of an SfM batch
 * (Sec. 4-5: matching dominates the pipeline's run time).  Each pair gives
 * exactly what hamming_knn gives for its ranges, with train indices relative
 * to train_first, written to output rows out_first .. out_first + nq - 1.
 *   query_dev: uint32[query_rows][16]; train_dev: uint32[train_rows][16]
 *              (the same array may serve as both).
 *   pairs_dev: latch_pair[n_pairs], device memory (the caller's work list;
 *              contents may change between replays of a captured graph).
 *   idx_dev, dist_dev: int32[out_rows][k]; accept_dev: uint8[out_rows] or NULL.
 * A pair whose ranges fall outside query_rows / train_rows / out_rows, or
 * with nt > 2^21 - 32, is skipped and sets LATCH_FLAG_BAD_PAIR.  Pairs'
 * output ranges should not overlap (they are written concurrently).  k,
 * ratio and path as for hamming_knn.  Uses the handle's workspace
 * (hamming_knn_batch_workspace_size; LATCH_EWORKSPACE if the handle holds
 * less).
 */
int hamming_knn_batch(latch_handle h, const uint32_t *query_dev, int64_t query_rows,
                      const uint32_t *train_dev, int64_t train_rows, const latch_pair *pairs_dev,
                      int n_pairs, int k, float ratio, int32_t *idx_dev, int32_t *dist_dev,
                      uint8_t *accept_dev, int64_t out_rows, int path, hipStream_t stream);

/*
 * Plans: one batched extract + match sequence captured once as a HIP graph
 * and replayed with a single graph launch.  The paper describes and then
 * matches many images of a scene for structure from motion, where matching
 * dominates the run time (Sec. 5, Table 2), and overlaps the images' work on
 * streams (Sec. 4, "CUDA Integration"); a plan runs a whole batch of uneven
 * images and image pairs as two persistent launches instead.  The plan fixes
 * the device buffers below (pointers), not their contents: between runs the
 * caller may rewrite the image table, keypoints, image ids, keypoint count
 * and pairs.  Each run extracts descriptors for the batch's keypoints into
 * `desc` (as latch_extract_batch) and then matches the pairs, whose query and
 * train rows both index `desc` (as hamming_knn_batch).  The plan owns its
 * matching workspace, so the handle's is not used.
 */
typedef struct latch_plan_ctx *latch_plan;

typedef struct {
    const latch_image *images;     /* [n_images] */
    int32_t n_images;
    const int32_t *image_id;       /* [max_kps] */
    const latch_keypoint *kps;     /* [max_kps] */
    const int64_t *n_kps;          /* device count to process (<= max_kps), or NULL for max_kps */
    int64_t max_kps;
    uint32_t *desc;                /* [max_kps][16] */
    const latch_pair *pairs;       /* [n_pairs]; ranges index desc rows */
    int32_t n_pairs;
    int32_t k;                     /* 1 or 2 */
    float ratio;                   /* (0, 1] */
    int32_t path;                  /* latch_path */
    int32_t *idx, *dist;           /* [out_rows][k] */
    uint8_t *accept;               /* [out_rows] or NULL */
    int64_t out_rows;
} latch_plan_desc;

/*
 * Capture a plan.  Validates the host-checkable fields as the two batched
 * calls do, allocates the plan's own workspace (device memory it owns until
 * latch_plan_destroy) and captures the graph on a private stream.  The plan
 * uses the handle's tables and error word: destroy plans before their handle.
 */
int latch_plan_create(latch_handle h, const latch_plan_desc *desc, latch_plan *out);

/* One replay of the plan's graph on `stream` (asynchronous, like every call). */
int latch_plan_run(latch_plan p, hipStream_t stream);

/* Release a plan (synchronises the device first).  NULL is a no-op. */
void latch_plan_destroy(latch_plan p);

/*
 * Read the sticky device error word (LATCH_FLAG_* bits) after all work
 * enqueued on `stream` so far; synchronises that stream.  If clear != 0 the
 * word is reset to zero afterwards.
 */
int latch_check_errors(latch_handle h, hipStream_t stream, uint32_t *flags_out, int clear);

/* Text of the last error reported through this handle ("" if none).  Valid until the next call. */
const char *latch_last_error(latch_handle h);

/*
 * Host-only (no GPU needed): the rotation table of rule step 2, as used by
 * the kernels.  cos_q14 and sin_q14 receive int16[4096].  For a in [0, 512]:
 * rne(16384 cos(2 pi a / 4096)) and rne(16384 sin(2 pi a / 4096)); for a in
 * (512, 1024): (sin, cos) of 1024 - a; every a >= 1024: (C, S)[a] =
 * (-S, C)[a - 1024].  Returns LATCH_OK or LATCH_EINVAL for NULL pointers.
 */
int latch_rotation_table(int16_t *cos_q14, int16_t *sin_q14);

/*
 * Tuning.  LATCH_PATH_AUTO picks the matcher path from a per-handle table
 * indexed by size buckets, bucket(n) = min(7, floor(log2(max(n, 1)) / 2)),
 * and the split planner of hamming_knn aims at the given number of
 * workgroups per CU.  The MXFP4 matchers hold 2 or 3 blocks of 32 queries
 * per wavefront (a workgroup of 4 wavefronts takes 256 or 384 queries
 * against each staged train tile); the
 * batched MFMA matchers run the given number of persistent workgroups per
 * CU.  Defaults: MFMA_FP4 everywhere (batches too), 2 (both MFMA paths) and
 * 8 (popcount) workgroups per CU, 3 query blocks, 2 batched
 * workgroups per CU.  Tuning never changes results, only speed.
 */
typedef struct {
    int8_t path[8][8];               /* [bucket(nq)][bucket(nt)]: LATCH_PATH_MFMA, _POPCOUNT or _MFMA_FP4 */
    int8_t batch_path;               /* path of batched matching under LATCH_PATH_AUTO */
    int8_t fp4_query_blocks;         /* 2 or 3 */
    int8_t reserved[2];              /* 0 */
    int32_t mfma_groups_per_cu;      /* >= 1 */
    int32_t popcount_groups_per_cu;  /* >= 1 */
    int32_t batch_groups_per_cu;     /* in [1, 8] */
} latch_tuning;

int latch_get_tuning(latch_handle h, latch_tuning *out);
/* LATCH_ERANGE if a path entry is not MFMA, POPCOUNT or MFMA_FP4, a target is < 1,
 * fp4_query_blocks is not 2 or 3, or batch_groups_per_cu outside [1, 8]. */
int latch_set_tuning(latch_handle h, const latch_tuning *t);

/*
 * Per-kernel timing with HIP events, for measurement.  While enabled, every
 * kernel the handle launches is bracketed by two hipEventRecord calls on the
 * launch stream.  latch_timing_enable(h, 1) starts a fresh record (0 stops
 * recording).  latch_timing_read waits for the recorded events and returns,
 * for one kernel name ("extract", "dense_extract", "knn_window", "detect", "knn_mfma", "knn_fp4", "knn_popcount", "knn_merge",
 * "knn_batch_mfma", "knn_batch_fp4", "knn_batch_popcount"; the batch names cover the whole
 * batched sequence), the number of launches recorded and their summed
 * duration in milliseconds.  Not for use under stream capture.
 */
int latch_timing_enable(latch_handle h, int enable);
int latch_timing_read(latch_handle h, const char *kernel, int *launches, double *total_ms);

/* Library version string. */
const char *latch_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LATCH_H */
