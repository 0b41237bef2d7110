/*
 * Seeded synthetic grayscale images with the structure of face-sized frames.
 *
 * This file holds input generation only (noise, blur, rectangles, impulse
 * noise, flat patches); none of the LDP arithmetic.  It is deterministic on
 * every machine: all arithmetic is integer and the random numbers come from a
 * counter-based generator (SplitMix64, the finaliser published by Steele, Lea
 * and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014,
 * with the constants of Vigna's reference implementation), keyed by
 * (seed, image index), so one image of a large batch can be regenerated alone.
 *
 * Recipes (kind):
 *   0  iid uniform bytes 0..255.
 *   1  iid uniform bytes, blurred by a separable integer Gaussian of sigma 1.5
 *      (9 taps, weights 2 9 28 55 68 55 28 9 2 / 256, mirrored borders,
 *      rounded), then 8 filled rectangles of random size and intensity
 *      (height in [ceil(H/16), ceil(H/2)], width in [ceil(W/16), ceil(W/2)]).
 *   2  kind-1 blur, then 5% salt-and-pepper (each pixel independently, with
 *      probability 1/20, set to 0 or 255 with equal odds), then 32 square
 *      patches of one constant intensity (side in [64, 1024], clipped to the
 *      image), painted last so they are exactly flat.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* sequential stream for the few per-image draws */
typedef struct { uint64_t key, ctr; } stream_t;
static inline uint64_t next64(stream_t *s) { return mix64(s->key ^ mix64(s->ctr++)); }
static inline int64_t uniform_int(stream_t *s, int64_t lo, int64_t hi)
{
    uint64_t span = (uint64_t)(hi - lo + 1);
    return lo + (int64_t)(next64(s) % span);
}

static uint64_t image_key(uint64_t seed, uint64_t index)
{
    return mix64(mix64(seed) ^ (index * 0xd1b54a32d192ed03ULL));
}

static const int GW[9] = {2, 9, 28, 55, 68, 55, 28, 9, 2}; /* sum 256 */

static inline int64_t mirror(int64_t i, int64_t n)
{
    /* half-sample symmetric reflection: -1 -> 0, n -> n-1 */
    while (i < 0 || i >= n) {
        if (i < 0) i = -i - 1;
        if (i >= n) i = 2 * n - i - 1;
    }
    return i;
}

static void noise(uint8_t *dst, int64_t H, int64_t W, int64_t stride, uint64_t key)
{
    for (int64_t r = 0; r < H; ++r)
        for (int64_t c = 0; c < W; ++c) {
            uint64_t p = (uint64_t)(r * W + c);
            uint64_t w = mix64(key ^ mix64(0x5eed0000ULL + (p >> 3)));
            dst[r * stride + c] = (uint8_t)(w >> (8 * (p & 7)));
        }
}

static void blur(uint8_t *img, int64_t H, int64_t W, int64_t stride)
{
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(H * W));
    if (!tmp) abort();
    for (int64_t r = 0; r < H; ++r)
        for (int64_t c = 0; c < W; ++c) {
            uint32_t acc = 0;
            for (int t = -4; t <= 4; ++t)
                acc += (uint32_t)GW[t + 4] * img[r * stride + mirror(c + t, W)];
            tmp[r * W + c] = acc;
        }
    for (int64_t r = 0; r < H; ++r)
        for (int64_t c = 0; c < W; ++c) {
            uint32_t acc = 0;
            for (int t = -4; t <= 4; ++t)
                acc += (uint32_t)GW[t + 4] * tmp[mirror(r + t, H) * W + c];
            uint32_t v = (acc + 32768u) >> 16;
            img[r * stride + c] = (uint8_t)(v > 255 ? 255 : v);
        }
    free(tmp);
}

static void fill_rect(uint8_t *img, int64_t stride, int64_t r0, int64_t c0, int64_t h,
                      int64_t w, uint8_t v)
{
    for (int64_t r = r0; r < r0 + h; ++r)
        memset(img + r * stride + c0, v, (size_t)w);
}

static void make_one(uint8_t *dst, int64_t H, int64_t W, int64_t stride, int kind,
                     uint64_t seed, uint64_t index)
{
    uint64_t key = image_key(seed, index);
    stream_t s = {key, 1};
    noise(dst, H, W, stride, key);
    if (kind == 0)
        return;
    blur(dst, H, W, stride);
    if (kind == 1) {
        int64_t hmin = (H + 15) / 16, hmax = (H + 1) / 2;
        int64_t wmin = (W + 15) / 16, wmax = (W + 1) / 2;
        for (int n = 0; n < 8; ++n) {
            int64_t h = uniform_int(&s, hmin, hmax), w = uniform_int(&s, wmin, wmax);
            int64_t r0 = uniform_int(&s, 0, H - h), c0 = uniform_int(&s, 0, W - w);
            fill_rect(dst, stride, r0, c0, h, w, (uint8_t)uniform_int(&s, 0, 255));
        }
        return;
    }
    /* kind 2: salt and pepper, then flat square patches */
    for (int64_t r = 0; r < H; ++r)
        for (int64_t c = 0; c < W; ++c) {
            uint64_t u = mix64(key ^ mix64(0x5a1700000000ULL + (uint64_t)(r * W + c)));
            if (u % 20 == 0)
                dst[r * stride + c] = ((u >> 32) & 1) ? 255 : 0;
        }
    for (int n = 0; n < 32; ++n) {
        int64_t side = uniform_int(&s, 64, 1024);
        int64_t h = side < H ? side : H, w = side < W ? side : W;
        int64_t r0 = uniform_int(&s, 0, H - h), c0 = uniform_int(&s, 0, W - w);
        fill_rect(dst, stride, r0, c0, h, w, (uint8_t)uniform_int(&s, 0, 255));
    }
}

/* Fill n images.  Image j has H[j] rows, W[j] columns and row pitch stride[j]
 * bytes and starts at base + offset[j]; it is image number first_index + j of
 * the stream keyed by seed.  Returns 0, or -1 on invalid sizes. */
int synth_images(uint8_t *base, const int64_t *offset, const int32_t *H, const int32_t *W,
                 const int64_t *stride, int32_t n, int32_t kind, uint64_t seed,
                 uint64_t first_index)
{
    for (int32_t j = 0; j < n; ++j)
        if (H[j] < 1 || W[j] < 1 || stride[j] < W[j] || kind < 0 || kind > 2)
            return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t j = 0; j < n; ++j)
        make_one(base + offset[j], H[j], W[j], stride[j], kind, seed, first_index + (uint64_t)j);
    return 0;
}

/* n uniform integers in [lo, hi] from the stream keyed by seed (for sizes). */
void synth_uniform_ints(int32_t *out, int32_t n, int32_t lo, int32_t hi, uint64_t seed)
{
    stream_t s = {mix64(seed ^ 0x51e5ULL), 0};
    for (int32_t j = 0; j < n; ++j)
        out[j] = (int32_t)uniform_int(&s, lo, hi);
}

/* n raw 64-bit words from the stream keyed by seed (for arrival times). */
void synth_u64(uint64_t *out, int32_t n, uint64_t seed)
{
    stream_t s = {mix64(seed ^ 0xa77ULL), 0};
    for (int32_t j = 0; j < n; ++j)
        out[j] = next64(&s);
}
