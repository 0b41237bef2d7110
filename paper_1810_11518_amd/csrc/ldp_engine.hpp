// ldp_engine.hpp -- the per-lane row walk shared by every LDP kernel.
//
// A task is one column group (8 code columns) of one image over a range of
// code rows.  The lane keeps the three image rows around the current code
// row in registers, loads each new row once (prefetched one row ahead) with
// hardware bounds-checked buffer loads, computes the 8 codes, and hands them
// to the store and/or the LDS histogram.
#pragma once
#include "ldp_device.hpp"

namespace ldp {

// An image as the kernels see it.  `off0` is the image start relative to the
// 4-aligned base address in the buffer descriptor.
struct ImgView {
    __amdgpu_buffer_rsrc_t rsrc;
    uint32_t off0;
    int64_t stride;
    int32_t H, W;      // image
    int32_t Hc, Wc;    // code map
    uint8_t *codes;    // may be null
};

__device__ __forceinline__ ImgView make_view(const uint8_t *img, int64_t stride, int32_t H,
                                             int32_t W, uint8_t *codes)
{
    ImgView v;
    uintptr_t p = (uintptr_t)img;
    uintptr_t base = p & ~(uintptr_t)3;
    v.off0 = (uint32_t)(p - base);
    int64_t extent = (int64_t)v.off0 + (int64_t)(H - 1) * stride + W;
    uint32_t nrec = (uint32_t)((extent + 3) & ~(int64_t)3);
    v.rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)nrec, 0x00020000);
    v.stride = stride;
    v.H = H;
    v.W = W;
    v.Hc = H - 2;
    v.Wc = W - 2;
    v.codes = codes;
    return v;
}

// Rows start on 4-byte boundaries: the lane's dwords need no realignment.
__device__ __forceinline__ bool image_aligned_dev(const uint8_t *img, int64_t stride)
{
    return ((uintptr_t)img & 3u) == 0 && (stride & 3) == 0;
}

// First code row (column) of cell `c` in a floor partition of n rows into
// `cells` cells: the smallest r with r*cells/n == c.
__host__ __device__ __forceinline__ int32_t cell_start(int32_t c, int32_t n, int32_t cells)
{
    return (int32_t)(((int64_t)c * n + cells - 1) / cells);
}

__device__ __forceinline__ void store8(uint8_t *p, uint32_t lo, uint32_t hi, int nvalid)
{
    if (nvalid >= 8) {
        uint32_t a = (uint32_t)(uintptr_t)p & 3u;
        if (a == 0) {
            reinterpret_cast<uint32_t *>(p)[0] = lo;
            reinterpret_cast<uint32_t *>(p)[1] = hi;
        } else if (a == 2) {
            reinterpret_cast<uint16_t *>(p)[0] = (uint16_t)lo;
            reinterpret_cast<uint16_t *>(p)[1] = (uint16_t)(lo >> 16);
            reinterpret_cast<uint16_t *>(p)[2] = (uint16_t)hi;
            reinterpret_cast<uint16_t *>(p)[3] = (uint16_t)(hi >> 16);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                p[q] = (uint8_t)(lo >> (8 * q));
                p[4 + q] = (uint8_t)(hi >> (8 * q));
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (q < nvalid)
                p[q] = (uint8_t)((q < 4 ? lo : hi) >> (8 * (q & 3)));
        }
    }
}

// LDS histogram window of a task: cell rows [cy0, cy0 + ncy) x all cells_x
// cell columns, 256 uint32 bins each, at lds[((cy - cy0)*cells_x + cx)*256].
struct HistWin {
    uint32_t *lds;
    int32_t cells_y, cells_x;
    int32_t cy0;
};

template <int K, bool ALIGNED, bool HIST>
__device__ __forceinline__ void run_task(const ImgView &im, const HistWin &hw, int32_t g,
                                         int32_t r0, int32_t r1)
{
    const int32_t j0 = 8 * g;              // first code column of the lane
    const int nvalid = min(8, im.Wc - j0); // pixels of the lane inside the map
    uint32_t off = im.off0 + (uint32_t)((int64_t)r0 * im.stride) + (uint32_t)j0;
    const uint32_t ostride = (uint32_t)im.stride;

    // histogram addressing: byte offset of each pixel's cell in the window
    uint32_t colb[8];
    int32_t cyr = 0, next_cy_row = 0;
    uint32_t rowb = 0;
    if constexpr (HIST) {
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            int32_t j = min(j0 + p, im.Wc - 1);
            colb[p] = (uint32_t)(((int64_t)j * hw.cells_x) / im.Wc) * 1024u;
        }
        cyr = (int32_t)(((int64_t)r0 * hw.cells_y) / im.Hc);
        next_cy_row = cell_start(cyr + 1, im.Hc, hw.cells_y);
        rowb = (uint32_t)((cyr - hw.cy0) * hw.cells_x) * 1024u;
    }
    const bool one_cell = HIST && nvalid >= 8 && colb[0] == colb[7];

    RawRow raw;
    Row t, m, b;
    load_row<ALIGNED>(raw, im.rsrc, off);
    unpack_row<ALIGNED>(t, raw);
    load_row<ALIGNED>(raw, im.rsrc, off + ostride);
    unpack_row<ALIGNED>(m, raw);
    load_row<ALIGNED>(raw, im.rsrc, off + 2 * ostride);
    uint32_t Vt[6];
#pragma unroll
    for (int a = 0; a < 6; ++a)
        Vt[a] = t.X[a] + m.X[a];

    uint8_t *cp = im.codes ? im.codes + (int64_t)r0 * im.Wc + j0 : nullptr;
    for (int32_t r = r0; r < r1; ++r) {
        unpack_row<ALIGNED>(b, raw);
        // prefetch the next image row (clamped to the last row)
        uint32_t noff = off + (uint32_t)(min(r + 3, im.H - 1) - r0) * ostride;
        load_row<ALIGNED>(raw, im.rsrc, noff);

        uint32_t Vb[6];
#pragma unroll
        for (int a = 0; a < 6; ++a)
            Vb[a] = m.X[a] + b.X[a];
        uint32_t lo, hi;
        code_row<K>(t, b, Vt, Vb, lo, hi);

        if (cp) {
            store8(cp, lo, hi, nvalid);
            cp += im.Wc;
        }
        if constexpr (HIST) {
            if (r == next_cy_row) {
                ++cyr;
                next_cy_row = cell_start(cyr + 1, im.Hc, hw.cells_y);
                rowb = (uint32_t)((cyr - hw.cy0) * hw.cells_x) * 1024u;
            }
            // byte address of bin `code` of pixel p's cell: cell offsets are
            // multiples of 1024, so (code << 2) is OR-ed in (v_bitop3_b32)
            char *lds = reinterpret_cast<char *>(hw.lds);
            if (one_cell && lo == hi && lo == __builtin_amdgcn_alignbyte(lo, lo, 1)) {
                // eight equal codes in one cell (flat regions): one update
                const uint32_t addr = (rowb + colb[0]) | ((lo & 0xFFu) << 2);
                atomicAdd(reinterpret_cast<uint32_t *>(lds + addr), 8u);
            } else {
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    const uint32_t w = p < 4 ? lo : hi;
                    const int q = p & 3;
                    const uint32_t sh = q == 0 ? (w << 2) : (w >> (8 * q - 2));
                    const uint32_t addr = __builtin_amdgcn_bitop3_b32(sh, 0x3FCu, rowb + colb[p], 0xEA);
                    if (nvalid >= 8 || p < nvalid)
                        atomicAdd(reinterpret_cast<uint32_t *>(lds + addr), 1u);
                }
            }
        }
        t = m;
        m = b;
#pragma unroll
        for (int a = 0; a < 6; ++a)
            Vt[a] = Vb[a];
    }
}

// ---------------------------------------------------------------- work items
// One workgroup per work item of one image: the code rows [r0, r1) of cell
// rows [cy0, cy1) (r0/r1 may cut a cell row when `split` > 1, and the
// histogram flush then adds atomically into a zeroed array).
template <int K, bool ALIGNED>
__device__ __forceinline__ void fused_item(const ImgView &im, uint32_t *lds, int32_t cells_y,
                                           int32_t cells_x, int32_t cy0, int32_t cy1, int32_t r0,
                                           int32_t r1, uint32_t *hist, bool atomic_flush,
                                           int32_t min_task_rows)
{
    const int tid = threadIdx.x, nthreads = blockDim.x;
    const int32_t nbins = (cy1 - cy0) * cells_x * 256;
    for (int32_t i = tid; i < nbins; i += nthreads)
        lds[i] = 0;
    __syncthreads();
    const int32_t ngroups = (im.Wc + 7) / 8;
    const int32_t nr = r1 - r0;
    // row sub-bands per column group: as many as the threads allow, but no
    // shorter than min_task_rows code rows
    int32_t nsub = max(1, min(nthreads / ngroups, (nr + min_task_rows - 1) / min_task_rows));
    const int32_t ntasks = ngroups * nsub;
    HistWin hw{lds, cells_y, cells_x, cy0};
    for (int32_t task = tid; task < ntasks; task += nthreads) {
        int32_t g = task % ngroups, sb = task / ngroups;
        int32_t a0 = r0 + (int32_t)((int64_t)nr * sb / nsub);
        int32_t a1 = r0 + (int32_t)((int64_t)nr * (sb + 1) / nsub);
        if (a1 > a0)
            run_task<K, ALIGNED, true>(im, hw, g, a0, a1);
    }
    __syncthreads();
    uint32_t *dst = hist + (int64_t)cy0 * cells_x * 256;
    for (int32_t i = tid; i < nbins; i += nthreads) {
        uint32_t v = lds[i];
        if (!atomic_flush)
            dst[i] = v;
        else if (v)
            atomicAdd(dst + i, v);
    }
}

}  // namespace ldp
