// Device helpers shared by the extraction kernels: resampling rule steps 1-3
// for batches of keypoints (with the image each keypoint samples), and the
// exact small-integer arithmetic of rule step 4.  Included inside
// namespace latch { namespace { ... } } of each kernel file.
#pragma once

typedef const __attribute__((address_space(1))) uint8_t GlobalByte;
typedef __attribute__((address_space(1))) uint32_t GlobalWord;

// A wavefront-uniform global pointer, kept in scalar registers.
__device__ __forceinline__ GlobalWord *uniform_words(uint32_t *ptr)
{
    const uint64_t v = reinterpret_cast<uintptr_t>(ptr);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (GlobalWord *)(lo | (hi << 32));
}

// n / 2^22 rounded half away from zero, for |n| < 2^31 - 2^21.
// n >= 0: floor((n + 2^21) / 2^22).  n < 0: floor((n + 2^21 - 1) / 2^22),
// which equals ceil((n - 2^21) / 2^22) = -floor((-n + 2^21) / 2^22).
__device__ __forceinline__ int round_q22(int n)
{
    return (n + (1 << 21) + (n >> 31)) >> 22;
}

__device__ __forceinline__ int clamp_med3(int x, int lo, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

// 24-bit signed multiplies, kept as such (the compiler would otherwise fold
// them into quarter-rate 32-bit multiplies by the precomputed sq * C).
__device__ __forceinline__ int mul_i24(int a, int b)
{
    int r;
    asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ int mad_i24(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// The same with a wavefront-uniform first factor `a` read from a scalar
// register (no copy into a vector register first).
__device__ __forceinline__ int mul_i24_s(int a, int b)
{
    int r;
    asm("v_mul_i32_i24 %0, %1, %2" : "=v"(r) : "s"(a), "v"(b));
    return r;
}

__device__ __forceinline__ int mad_i24_s(int a, int b, int c)
{
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "s"(a), "v"(b), "v"(c));
    return r;
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t dot4(uint32_t a, uint32_t b, uint32_t acc)
{
    return __builtin_amdgcn_udot4(a, b, acc, false);
}

// The keypoints one workgroup of a grid-stride extraction takes.  The chip's
// 8 XCDs (workgroups go to them round-robin by index) take contiguous eighths
// of [0, n), so that one XCD's L2 holds the images (or, for keypoints in
// raster order, the image rows) its own workgroups read, rather than every
// XCD fetching every image; within its eighth an XCD's workgroups stride
// over the keypoints.  Keypoint p of the range is first + m * stride.
struct KeypointRange {
    int64_t first, end, stride;
};

__device__ __forceinline__ KeypointRange xcd_range(int64_t n)
{
    constexpr int kXcds = 8;
    const int g = gridDim.x, b = blockIdx.x;
    KeypointRange r;
    if (g < kXcds) {
        r.first = b;
        r.end = n;
        r.stride = g;
        return r;
    }
    const int xcd = b % kXcds;
    const int64_t per = (n + kXcds - 1) / kXcds;
    r.first = (int64_t)xcd * per + b / kXcds;
    r.end = min(n, (int64_t)(xcd + 1) * per);
    r.stride = (g - xcd + kXcds - 1) / kXcds;     // workgroups on this XCD
    return r;
}

// Rule steps 1-3 for one keypoint (uniform across the workgroup), with the
// image it samples.
struct Keypoint {
    bool ok;        // inside the rule's domain (and a real keypoint)
    bool interior;  // every sample lies inside the image: no clamping needed
    int cx, cy;
    int c, s, sq;   // C[b], S[b] (Q14) and the Q8 scale
    int cls;        // angle class b >> 5 (0..127), which orders the window gather
    const uint8_t *img;
    int height, width, pitch;
    int centre;     // cy * pitch + cx (meaningful when interior)
    int key;        // the keypoint's index in the keypoint and descriptor arrays
};

// Where keypoints find their image: one image given by value, or a device
// table of images indexed by a per-keypoint image id.
struct ImageSource {
    const uint8_t *img;          // single image
    int height, width, pitch;
    const ImageEntry *table;     // batch: table[image_id[k]]
    const int32_t *image_id;
    int n_images;
    const int32_t *order;        // batch: keypoint index at each position, or nullptr (identity)
};

// Rule steps 1-3 for 64 keypoints at once: lane j takes keypoint
// first + j * stride.  The result stays in registers; each keypoint's
// parameters are then read out with readlane, so the two dependent loads
// (record, table entry) are paid once per 64 keypoints.
struct KeypointBatch {
    int cx, cy;
    int cs;          // C[b] & 0xffff | S[b] << 16
    int sq_flags;    // sq | ok << 16 | interior << 17 | bad image << 18 | (b >> 5) << 19
    int id;          // image table: the keypoint's image (0 when out of range)
    int key;         // keypoint index (the position itself without an order)
};

// kHalfSide: the largest |u|, |v| of a window position (half the window side).
template <bool kTable, int kHalfSide>
__device__ __forceinline__ KeypointBatch prepare_batch(const float4 *__restrict__ kps, int64_t n,
                                                       int64_t first, int64_t stride, int lane,
                                                       const int2 *__restrict__ rot,
                                                       const ImageSource &src)
{
    KeypointBatch kb;
    int64_t idx = first + stride * lane;
    const bool real = idx < n;
    if (kTable && src.order && real) idx = src.order[idx];
    const uint8_t *img = src.img;
    int height = src.height, width = src.width, pitch = src.pitch;
    bool image_ok = true;
    int image_id = 0;
    if (kTable) {
        const int id = real ? src.image_id[idx] : 0;
        image_ok = id >= 0 && id < src.n_images;
        image_id = image_ok ? id : 0;
        const ImageEntry e = image_ok ? src.table[id] : ImageEntry{nullptr, 1, 1, 1, 0};
        img = e.img;
        height = e.height;
        width = e.width;
        pitch = e.pitch;
        image_ok = image_ok && img != nullptr && height >= 1 && width >= 1 && pitch >= width &&
                   height < (1 << 23) && pitch < (1 << 23) &&
                   (int64_t)height * pitch <= (int64_t)0x7fffffff;
        if (!image_ok) {
            height = width = pitch = 1;
        }
    }
    const float4 kp = real ? kps[idx] : make_float4(0.f, 0.f, 0.f, 0.f);
    bool ok = real && image_ok && __builtin_isfinite(kp.x) && __builtin_isfinite(kp.y) &&
              __builtin_isfinite(kp.z) && __builtin_isfinite(kp.w);
    ok = ok && fabsf(kp.x) <= 16777216.0f && fabsf(kp.y) <= 16777216.0f && fabsf(kp.z) <= 1.0e6f;
    const double sqd = ok ? rint((double)kp.w * 256.0) : 0.0;
    ok = ok && sqd >= 1.0 && sqd <= 1024.0;
    int cx = 0, cy = 0, bin = 0, sq = 0;
    if (ok) {
        cx = (int)floor((double)kp.x + 0.5);
        cy = (int)floor((double)kp.y + 0.5);
        bin = (int)rint((double)kp.z * (4096.0 / 360.0)) & (kBins - 1);
        sq = (int)sqd;
    }
    const int2 cs = rot[bin];
    // |offset| <= (kHalfSide sq (|C| + |S|) + 2^21) / 2^22 < reach.
    const int reach = ((kHalfSide * sq * (abs(cs.x) + abs(cs.y))) >> 22) + 1;
    const bool interior = ok && cx - reach >= 0 && cx + reach <= width - 1 && cy - reach >= 0 &&
                          cy + reach <= height - 1;
    kb.cx = cx;
    kb.cy = cy;
    kb.cs = (cs.x & 0xffff) | (cs.y << 16);
    kb.sq_flags = sq | ((int)ok << 16) | ((int)interior << 17) | ((int)(real && !image_ok) << 18) |
                  ((bin >> 5) << 19);
    kb.id = image_id;
    kb.key = (int)idx;
    return kb;
}

template <bool kTable>
__device__ __forceinline__ Keypoint batch_get(const KeypointBatch &kb, int j, const ImageSource &src,
                                              bool *bad_image)
{
    Keypoint k;
    k.key = __builtin_amdgcn_readlane(kb.key, j);
    k.cx = __builtin_amdgcn_readlane(kb.cx, j);
    k.cy = __builtin_amdgcn_readlane(kb.cy, j);
    const int cs = __builtin_amdgcn_readlane(kb.cs, j);
    const int f = __builtin_amdgcn_readlane(kb.sq_flags, j);
    k.c = (int)(short)(cs & 0xffff);
    k.s = cs >> 16;
    k.sq = f & 0xffff;
    k.ok = (f >> 16) & 1;
    k.interior = (f >> 17) & 1;
    *bad_image = (f >> 18) & 1;
    k.cls = f >> 19;
    if (kTable) {
        // The keypoint's image entry, a uniform (scalar) load; the entry was
        // validated per lane in prepare_batch, and ok is false otherwise.
        // The fields go to scalar registers: every use below is uniform.
        const ImageEntry e = src.table[__builtin_amdgcn_readlane(kb.id, j)];
        const uint64_t ip = reinterpret_cast<uintptr_t>(e.img);
        k.img = reinterpret_cast<const uint8_t *>(
            (uint64_t)(uint32_t)uniform_int((int)(uint32_t)ip) |
            ((uint64_t)(uint32_t)uniform_int((int)(uint32_t)(ip >> 32)) << 32));
        k.height = uniform_int(e.height);
        k.width = uniform_int(e.width);
        k.pitch = uniform_int(e.pitch);
    } else {
        k.img = src.img;
        k.height = src.height;
        k.width = src.width;
        k.pitch = src.pitch;
    }
    // Only an interior keypoint uses it, and then cy * pitch + cx < 2^31.
    k.centre = k.interior ? k.cy * k.pitch + k.cx : 0;
    return k;
}
