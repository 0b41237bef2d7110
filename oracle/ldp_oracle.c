/*
 * Plain scalar C oracle for Local Directional Pattern codes and histograms.
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it (through oracle/native.py).
 *
 * It computes the definition with nothing shared between masks or pixels:
 *   - Eq. 1 (Section 2.2.1): eight Kirsch responses per interior pixel by
 *     direct 3x3 correlation (no kernel flip);
 *   - Eqs. 2-3 (Section 2.2.2): m_k is the k-th element of the eight
 *     responses sorted in descending order with duplicates kept, and bit i of
 *     the code is set when m_i - m_k >= 0 (optionally on |m_i|);
 *   - Eqs. 4-5 (Section 2.2.3): 256-bin histograms of the codes per cell of a
 *     floor-partitioned cells_y x cells_x grid over the interior code map.
 * Conventions: x is the row, y the column; masks M0..M7 are the Kirsch
 * compass masks East, North-East, North, North-West, West, South-West, South,
 * South-East; only interior pixels get codes, stored densely as
 * codes[(x-1)*(W-2) + (y-1)].
 *
 * ldp_oracle_extract_batch runs the two per-image functions over many images,
 * one image per OpenMP task: the arithmetic of every image is exactly that of
 * the single-image calls, only several images are computed at once.
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared -o liboracle_ldp.so ldp_oracle.c
 */
#include <stdint.h>
#include <string.h>

/* Kirsch masks, [mask][row a][column b]; row a = 0,1,2 is x-1, x, x+1 and
 * column b = 0,1,2 is y-1, y, y+1. */
static const int KIRSCH[8][3][3] = {
    {{-3, -3, 5}, {-3, 0, 5}, {-3, -3, 5}},     /* M0 East */
    {{-3, 5, 5}, {-3, 0, 5}, {-3, -3, -3}},     /* M1 North-East */
    {{5, 5, 5}, {-3, 0, -3}, {-3, -3, -3}},     /* M2 North */
    {{5, 5, -3}, {5, 0, -3}, {-3, -3, -3}},     /* M3 North-West */
    {{5, -3, -3}, {5, 0, -3}, {5, -3, -3}},     /* M4 West */
    {{-3, -3, -3}, {5, 0, -3}, {5, 5, -3}},     /* M5 South-West */
    {{-3, -3, -3}, {-3, 0, -3}, {5, 5, 5}},     /* M6 South */
    {{-3, -3, -3}, {-3, 0, 5}, {-3, 5, 5}},     /* M7 South-East */
};

/* flags: bit 0 set ranks the responses by absolute value (Eqs. 2-3 applied
 * to |m_i|).  Returns 0 on success, -1 on invalid arguments. */
int ldp_oracle_codes_ex(const uint8_t *img, int32_t H, int32_t W, int64_t stride,
                        int32_t k, int32_t flags, uint8_t *codes)
{
    if (!img || !codes || H < 3 || W < 3 || stride < W || k < 1 || k > 8 || (flags & ~1))
        return -1;
    for (int32_t x = 1; x <= H - 2; ++x) {
        for (int32_t y = 1; y <= W - 2; ++y) {
            int m[8];
            for (int i = 0; i < 8; ++i) {
                int acc = 0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        acc += KIRSCH[i][a][b] *
                               (int)img[(int64_t)(x + a - 1) * stride + (y + b - 1)];
                m[i] = (flags & 1) && acc < 0 ? -acc : acc;
            }
            /* descending insertion sort of a copy, duplicates kept */
            int s[8];
            memcpy(s, m, sizeof s);
            for (int i = 1; i < 8; ++i) {
                int v = s[i];
                int j = i - 1;
                while (j >= 0 && s[j] < v) {
                    s[j + 1] = s[j];
                    --j;
                }
                s[j + 1] = v;
            }
            int mk = s[k - 1];
            int code = 0;
            for (int i = 0; i < 8; ++i)
                if (m[i] - mk >= 0)
                    code |= 1 << i;
            codes[(int64_t)(x - 1) * (W - 2) + (y - 1)] = (uint8_t)code;
        }
    }
    return 0;
}

int ldp_oracle_codes(const uint8_t *img, int32_t H, int32_t W, int64_t stride,
                     int32_t k, uint8_t *codes)
{
    return ldp_oracle_codes_ex(img, H, W, stride, k, 0, codes);
}

/* hist has cells_y * cells_x * 256 entries, [(cy * cells_x + cx) * 256 + v];
 * it is overwritten.  H and W are the image dimensions; the code map is
 * (H-2) x (W-2).  Returns 0 on success, -1 on invalid arguments. */
int ldp_oracle_histograms(const uint8_t *codes, int32_t H, int32_t W,
                          int32_t cells_y, int32_t cells_x, uint32_t *hist)
{
    if (!codes || !hist || H < 3 || W < 3)
        return -1;
    int64_t hc = H - 2, wc = W - 2;
    if (cells_y < 1 || cells_x < 1 || cells_y > hc || cells_x > wc)
        return -1;
    memset(hist, 0, sizeof(uint32_t) * (size_t)cells_y * (size_t)cells_x * 256u);
    for (int64_t r = 0; r < hc; ++r) {
        int64_t cy = r * cells_y / hc;
        for (int64_t c = 0; c < wc; ++c) {
            int64_t cx = c * cells_x / wc;
            hist[(cy * cells_x + cx) * 256 + codes[r * wc + c]] += 1u;
        }
    }
    return 0;
}

/* Codes and histograms of n images (each as ldp_oracle_codes_ex followed by
 * ldp_oracle_histograms), images distributed over `threads` OpenMP threads
 * (threads < 1: one).  Image j has Hs[j] rows of Ws[j] bytes with pitch
 * strides[j], starting at base + img_off[j]; its codes go to
 * codes + code_off[j] ((H-2)*(W-2) bytes) and its histograms to
 * hist + j*cells_y*cells_x*256.  Returns 0, or -1 if any image's arguments are
 * invalid (checked before any image is computed). */
int ldp_oracle_extract_batch(const uint8_t *base, const int64_t *img_off, const int32_t *Hs,
                             const int32_t *Ws, const int64_t *strides, int32_t n, int32_t k,
                             int32_t flags, int32_t cells_y, int32_t cells_x, uint8_t *codes,
                             const int64_t *code_off, uint32_t *hist, int32_t threads)
{
    if (n < 0 || (n > 0 && (!base || !img_off || !Hs || !Ws || !strides || !codes ||
                            !code_off || !hist)))
        return -1;
    if (k < 1 || k > 8 || (flags & ~1) || cells_y < 1 || cells_x < 1)
        return -1;
    for (int32_t j = 0; j < n; ++j)
        if (Hs[j] < 3 || Ws[j] < 3 || strides[j] < Ws[j] || cells_y > Hs[j] - 2 ||
            cells_x > Ws[j] - 2)
            return -1;
    const int64_t per = (int64_t)cells_y * cells_x * 256;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads < 1 ? 1 : threads) \
    reduction(| : bad)
    for (int32_t j = 0; j < n; ++j) {
        bad |= ldp_oracle_codes_ex(base + img_off[j], Hs[j], Ws[j], strides[j], k, flags,
                                   codes + code_off[j]) != 0;
        bad |= ldp_oracle_histograms(codes + code_off[j], Hs[j], Ws[j], cells_y, cells_x,
                                     hist + (int64_t)j * per) != 0;
    }
    return bad ? -1 : 0;
}
