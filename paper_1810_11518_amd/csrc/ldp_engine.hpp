// ldp_engine.hpp -- the per-lane row walk shared by every LDP kernel.
//
// A task is one column group (8 adjacent code columns) of one image over a
// range of code rows that lies inside one cell row.  The lane keeps the three
// image rows around the current code row in registers, loads each new row
// once (two rows ahead) with hardware bounds-checked buffer loads,
// computes the 8 codes, stores them and counts them in the LDS histogram.
//
// Every lane owns 8 code columns: the last group of a row is moved left so
// that it ends at the last column (it recomputes, and stores again with the
// same values, the columns it shares with the previous group; its first
// 8 - n columns go to a discard bin of the histogram so every pixel is
// counted once).  Only code maps narrower than 8 columns take a masked path.
//
// A work item (one workgroup at a time) is a range of code rows covering
// whole cell rows (or part of one); its histogram cells live in LDS.  Every
// lane keeps one column group and one row band of each cell row for the whole
// item, so the per-pixel cell lookup is done once per item.
#pragma once
#include "ldp_device.hpp"

namespace ldp {

// An image as the kernels see it.  `off0` is the image start relative to the
// 4-aligned base address in the image's buffer descriptor.
struct ImgView {
    __amdgpu_buffer_rsrc_t rsrc;   // image bytes
    __amdgpu_buffer_rsrc_t crsrc;  // code map bytes
    uint32_t off0;
    uint32_t stride;
    int32_t H, W;    // image
    int32_t Hc, Wc;  // code map
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
    v.stride = (uint32_t)stride;
    v.H = H;
    v.W = W;
    v.Hc = H - 2;
    v.Wc = W - 2;
    // the range check of the descriptor keeps every store inside the map
    int64_t csize = codes ? (int64_t)v.Hc * v.Wc : 0;
    v.crsrc = __builtin_amdgcn_make_buffer_rsrc((void *)codes, (short)0, (int)csize, 0x00020000);
    return v;
}

// First code row (column) of cell `c` in a floor partition of n rows into
// `cells` cells: the smallest r with r*cells/n == c.  c <= cells <= n <= 65534,
// so c*n + cells - 1 < 2^32 and unsigned 32-bit arithmetic is exact.
__host__ __device__ __forceinline__ int32_t cell_start(int32_t c, int32_t n, int32_t cells)
{
    return (int32_t)(((uint32_t)c * (uint32_t)n + (uint32_t)cells - 1u) / (uint32_t)cells);
}

// floor(x / d) for x < 2^20 and 1 <= d < 2^20, without the 32-bit division
// sequence: q = trunc(x * rcp(d)) in f32.  v_rcp_f32 is within 1 ulp, so
// x * rcp(d) is within x/d * 2^-22 < 1/(4d) of x/d; writing x/d = m + f/d
// (0 <= f < d), q is m when f > 0 and m or m - 1 when f = 0, and the
// remainder test adds the missing one.
__device__ __forceinline__ uint32_t udiv_small(uint32_t x, uint32_t d)
{
    const uint32_t q = (uint32_t)((float)x * __builtin_amdgcn_rcpf((float)d));
    return q + (x - __umul24(q, d) >= d ? 1u : 0u);
}

// floor(x / d) for any x and 1 <= d < 2^20: udiv_small when x < 2^20 (the
// usual case), the full 32-bit division otherwise
__device__ __forceinline__ uint32_t udiv_u32(uint32_t x, uint32_t d)
{
    if (x < (1u << 20))
        return udiv_small(x, d);
    return x / d;
}

// Histogram cells of a code map: code row r lies in cell row r*ay/by, code
// column j in cell column j*ax/bx; ny x nx cells.
//   cells (Eqs. 4-5 over a grid): ay = cells_y, by = Hc, ax = cells_x, bx = Wc;
//   windows of wy x wx code pixels: ay = ax = 1, by = wy, bx = wx,
//   ny = ceil(Hc / wy), nx = ceil(Wc / wx) (the last ones cut at the edge).
// All operands are below 2^16 (window sides are clamped to the map), so the
// products below are exact in 32 bits.
struct Geom {
    uint32_t ay, by, ax, bx;
    int32_t ny, nx;
};

__host__ __device__ __forceinline__ Geom make_geom(int32_t Hc, int32_t Wc, int32_t gy, int32_t gx,
                                                   bool windows)
{
    Geom g;
    if (windows) {
        const int32_t wy = gy < Hc ? gy : Hc, wx = gx < Wc ? gx : Wc;
        g.ay = g.ax = 1;
        g.by = (uint32_t)wy;
        g.bx = (uint32_t)wx;
        g.ny = (Hc + wy - 1) / wy;
        g.nx = (Wc + wx - 1) / wx;
    } else {
        g.ay = (uint32_t)gy;
        g.by = (uint32_t)Hc;
        g.ax = (uint32_t)gx;
        g.bx = (uint32_t)Wc;
        g.ny = gy;
        g.nx = gx;
    }
    return g;
}

// First code row of cell row c (c = ny gives Hc), and first code column of
// cell column c.
__host__ __device__ __forceinline__ int32_t geom_row_start(const Geom &g, int32_t c, int32_t Hc)
{
    const int32_t r = (int32_t)(((uint32_t)c * g.by + g.ay - 1u) / g.ay);
    return r < Hc ? r : Hc;
}
__host__ __device__ __forceinline__ int32_t geom_col_start(const Geom &g, int32_t c, int32_t Wc)
{
    const int32_t j = (int32_t)(((uint32_t)c * g.bx + g.ax - 1u) / g.ax);
    return j < Wc ? j : Wc;
}

// Cell columns of a row cut into runs for workgroups whose LDS holds at
// most 63 cells of a cell row: cell_runs(nx) runs of near-equal length (at
// least 32 cells each when nx > 63), run i starting at cell_run_start.
__host__ __device__ __forceinline__ int32_t cell_runs(int32_t nx) { return (nx + 62) / 63; }
__host__ __device__ __forceinline__ int32_t cell_run_start(int32_t nx, int32_t runs, int32_t i)
{
    return (int32_t)((int64_t)nx * i / runs);
}

// LDS histograms of a work item: per cell row, its nx cells (of the item's
// column range) of 256 uint32 bins followed by one discard cell (pixels that
// another lane or item counts).
__host__ __device__ __forceinline__ uint32_t hist_row_bytes(int32_t nx)
{
    return (uint32_t)(nx + 1) * 1024u;
}

// Loads one image row for the lane: 16 bytes from the 4-aligned offset at or
// below the lane's first byte (aligned dwords never leave the image's last
// page), then realigns them.  ALIGNED: the lane's first byte is 4-aligned
// (a wave-wide fact, decided per task), so 12 bytes cover its 10 and no
// realignment is needed.
template <bool ALIGNED>
__device__ __forceinline__ void load_raw(RawRow &rr, __amdgpu_buffer_rsrc_t rsrc, uint32_t off)
{
    if constexpr (ALIGNED) {
        rr.s = 0;
        rr.w[0] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)off, 0, 0);
        rr.w[1] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)(off + 4), 0, 0);
        rr.w[2] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)(off + 8), 0, 0);
        rr.w[3] = 0;
    } else {
        rr.s = off & 3u;
        const uint32_t a = off & ~3u;
        rr.w[0] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)a, 0, 0);
        rr.w[1] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)(a + 4), 0, 0);
        rr.w[2] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)(a + 8), 0, 0);
        rr.w[3] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)(a + 12), 0, 0);
    }
}

template <int MODE, bool ALIGNED>
__device__ __forceinline__ void unpack_raw(Row &r, const RawRow &rr)
{
    if constexpr (ALIGNED) {
        make_row<MODE>(r, rr.w[0], rr.w[1], rr.w[2]);
    } else {
        uint32_t u0 = __builtin_amdgcn_alignbyte(rr.w[1], rr.w[0], rr.s);
        uint32_t u1 = __builtin_amdgcn_alignbyte(rr.w[2], rr.w[1], rr.s);
        uint32_t u2 = __builtin_amdgcn_alignbyte(rr.w[3], rr.w[2], rr.s);
        make_row<MODE>(r, u0, u1, u2);
    }
}

// Column group of a lane inside the item's column range [c_lo, c_hi): its
// first code column (groups of 8 from c_lo, the last one moved left to end at
// c_hi - 1) and the LDS cell of each pixel, one byte per pixel, laid out like
// the code words of code_row (bytes of d0: pixels 0, 1, 4, 5; of d1: pixels
// 2, 3, 6, 7): the cell column minus cx0, or the discard cell (ncell) for the
// leading columns that the previous group counts.  A range is at least 8
// columns wide.
struct Cols {
    int32_t j0;
    uint32_t d0, d1;
    bool uniform_cell;  // all 8 pixels counted in one cell
};

template <bool HIST>
__device__ __forceinline__ Cols group_cols(const Geom &geo, int32_t g, int32_t c_lo, int32_t c_hi,
                                           int32_t cx0, int32_t ncell, int32_t Wc)
{
    Cols c;
    c.j0 = min(c_lo + 8 * g, c_hi - 8);
    c.d0 = c.d1 = 0;
    c.uniform_cell = false;
    if constexpr (HIST) {
        const int32_t skip = c_lo + 8 * g - c.j0;
        // Cells at least 8 columns wide (the usual case, decided per image):
        // the 8 columns meet at most one cell boundary, so two divisions (the
        // first column's cell and the next cell's first column) place them
        // all.  Narrower cells: one division per column.
        // (all products below 2^32: columns and cell counts are below 2^16)
        const bool wide = geo.bx >= 8u * geo.ax;
        const uint32_t cxa = udiv_u32((uint32_t)c.j0 * geo.ax, geo.bx);
        const uint32_t next =
            wide ? min(udiv_u32((cxa + 1u) * geo.bx + geo.ax - 1u, geo.ax), (uint32_t)Wc) : 0u;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const uint32_t j = (uint32_t)(c.j0 + p);
            const uint32_t cx = wide ? cxa + (j >= next ? 1u : 0u) : udiv_u32(j * geo.ax, geo.bx);
            const uint32_t d = (p < skip ? (uint32_t)ncell : cx - (uint32_t)cx0)
                               << (8 * ((p & 1) | ((p >> 1) & 2)));
            if (p & 2)
                c.d1 |= d;
            else
                c.d0 |= d;
        }
        c.uniform_cell = c.d0 == c.d1 && c.d0 == __builtin_amdgcn_alignbyte(c.d0, c.d0, 1);
    }
    return c;
}

// Per-task state of the row walk.
struct Walk {
    uint32_t off, last_off;  // image byte offset of the prefetched / last row
    uint32_t coff;           // code byte offset of the current code row
    uint32_t d0, d1;         // per-pixel LDS cell index: cell row * (nx + 1) + cell column
    bool uniform_cell;
};

// LDS bins: the bin of code v in LDS cell c is the word at byte
// base + ((c << 8) | v) * 4.  An item's LDS holds at most 64 cells (64 KB),
// so c < 64 and the byte offset fits 16 bits.  One v_perm_b32 gathers two
// pixels' (code, cell) byte pairs from a code word x and its cell word d into
// the 16-bit halves of `pr`: [code a, cell a, code b, cell b] (sel picks
// bytes qa and qb); one v_mad_u32_u16 per pixel (half * 4 + base) makes its
// address.
typedef __attribute__((address_space(3))) uint32_t lds_u32;

__device__ __forceinline__ uint32_t lds_base(uint32_t *p)
{
    return (uint32_t)(uintptr_t)(lds_u32 *)p;
}
__device__ __forceinline__ uint32_t bin_pair(uint32_t x, uint32_t d, int qa, int qb)
{
    const uint32_t sel = (uint32_t)qa | ((uint32_t)(4 + qa) << 8) | ((uint32_t)qb << 16) |
                         ((uint32_t)(4 + qb) << 24);
    return __builtin_amdgcn_perm(d, x, sel);
}
// Written as instructions: the compiler would otherwise mask, shift and add
// the base in separate steps.
__device__ __forceinline__ uint32_t bin_lo(uint32_t pr, uint32_t base)
{
    uint32_t r;
    asm("v_mad_u32_u16 %0, %1, 4, %2" : "=v"(r) : "v"(pr), "s"(base));
    return r;
}
__device__ __forceinline__ uint32_t bin_hi(uint32_t pr, uint32_t base)
{
    uint32_t r;
    asm("v_mad_u32_u16 %0, %1, 4, %2 op_sel:[1,0,0,0]" : "=v"(r) : "v"(pr), "s"(base));
    return r;
}
__device__ __forceinline__ void lds_count(uint32_t addr, uint32_t n)
{
    __hip_atomic_fetch_add((lds_u32 *)(uintptr_t)addr, n, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Cache policy of a buffer store: non-temporal (streamed past the caches).
constexpr int kStoreNT = 2;

// One code row: the next image row arrives in `raw` and becomes `b` (t and m
// are the two rows above); the row after it moves from `raw2` to `raw`, and
// the row after that is loaded into `raw2` (clamped to the image's last row).
// Loading two rows ahead measured 1.2% faster on the batched kernel than one
// row ahead, whose next step waited for the previous row's code store too,
// and faster than giving each row slot its own buffer (no copies, but more
// live registers: setup values spilled to scratch).
template <int K, int MODE, bool HIST, bool CODES, bool ALIGNED, bool NT = false>
__device__ __forceinline__ void step(const ImgView &im, uint32_t *lds_bins, Walk &w, RawRow &raw,
                                     const Row &t, const Row &m, Row &b, RawRow &raw2)
{
    unpack_raw<MODE, ALIGNED>(b, raw);
    raw = raw2;
    w.off = min(w.off + im.stride, w.last_off);
    load_raw<ALIGNED>(raw2, im.rsrc, w.off);
    uint32_t q0, q1;
    code_row<K, MODE>(t, m, b, q0, q1);
    if constexpr (CODES) {
        // pixels 0-3 and 4-7 in column order; dword stores at any byte offset
        // (the target allows unaligned access)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_amdgcn_perm(q1, q0, 0x05040100u), im.crsrc,
                                              (int)w.coff, 0, NT ? kStoreNT : 0);
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_amdgcn_perm(q1, q0, 0x07060302u), im.crsrc,
                                              (int)(w.coff + 4), 0, NT ? kStoreNT : 0);
        w.coff += (uint32_t)im.Wc;
    }
    if constexpr (HIST) {
        const uint32_t base = lds_base(lds_bins);
        if (w.uniform_cell && q0 == q1 && q0 == __builtin_amdgcn_alignbyte(q0, q0, 1)) {
            // eight equal codes in one cell (flat regions): one update
            lds_count(bin_lo(bin_pair(q0, w.d0, 0, 1), base), 8u);
        } else {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const uint32_t pr = bin_pair(h & 1 ? q1 : q0, h & 1 ? w.d1 : w.d0, h & 2, (h & 2) + 1);
                lds_count(bin_lo(pr, base), 1u);
                lds_count(bin_hi(pr, base), 1u);
            }
        }
    }
}

// The row walk of a task from its first code row: n >= 1 rows, as a loop of
// three steps and a tail of one to `tail` steps (2 or 3, the same in every
// lane of the wave).  A wave runs the loop as long as any of its lanes does
// and the tail steps any lane needs, so it takes max(n) steps over its lanes
// when they all run the loop equally often: n / 3 times with a tail of up to
// 2, (n - 1) / 3 times with a tail of up to 3.
template <int K, int MODE, bool HIST, bool CODES, bool ALIGNED, bool NT = false>
__device__ __forceinline__ void walk_rows(const ImgView &im, uint32_t *lds_bins, Walk &w, int32_t n,
                                          int32_t tail)
{
    RawRow raw;
    Row A, B, C;
    load_raw<ALIGNED>(raw, im.rsrc, w.off);
    unpack_raw<MODE, ALIGNED>(A, raw);
    w.off += im.stride;
    load_raw<ALIGNED>(raw, im.rsrc, w.off);
    unpack_raw<MODE, ALIGNED>(B, raw);
    w.off += im.stride;
    load_raw<ALIGNED>(raw, im.rsrc, w.off);  // rows r0 .. r0 + 2 are in the image
    RawRow raw2;
    w.off = min(w.off + im.stride, w.last_off);
    load_raw<ALIGNED>(raw2, im.rsrc, w.off);
    // the three rows rotate through A, B, C so no registers are copied
    // between rows
    for (; n > tail; n -= 3) {
        step<K, MODE, HIST, CODES, ALIGNED, NT>(im, lds_bins, w, raw, A, B, C, raw2);
        step<K, MODE, HIST, CODES, ALIGNED, NT>(im, lds_bins, w, raw, B, C, A, raw2);
        step<K, MODE, HIST, CODES, ALIGNED, NT>(im, lds_bins, w, raw, C, A, B, raw2);
    }
    if (n >= 1)
        step<K, MODE, HIST, CODES, ALIGNED, NT>(im, lds_bins, w, raw, A, B, C, raw2);
    if (n >= 2)
        step<K, MODE, HIST, CODES, ALIGNED, NT>(im, lds_bins, w, raw, B, C, A, raw2);
    if (n >= 3)
        step<K, MODE, HIST, CODES, ALIGNED, NT>(im, lds_bins, w, raw, C, A, B, raw2);
}

// Run code rows [r0, r1) of the column group `c`; with HIST they all lie in
// the cell row whose histograms start at LDS byte `rowb`.
template <int K, int MODE, bool HIST, bool CODES, bool NT = false>
__device__ __forceinline__ void run_task(const ImgView &im, uint32_t *lds_bins, uint32_t rowb,
                                         const Cols &c, int32_t r0, int32_t r1)
{
    Walk w;
    w.off = im.off0 + (uint32_t)r0 * im.stride + (uint32_t)c.j0;
    w.last_off = im.off0 + (uint32_t)(im.H - 1) * im.stride + (uint32_t)c.j0;
    w.coff = __umul24((uint32_t)r0, (uint32_t)im.Wc) + (uint32_t)c.j0;  // both below 2^16
    // the cell row's first LDS cell, added to every pixel's byte
    const uint32_t row_cells = (rowb >> 10) * 0x01010101u;
    w.d0 = c.d0 + row_cells;
    w.d1 = c.d1 + row_cells;
    w.uniform_cell = c.uniform_cell;
    // tail of 3 when the wave's lanes agree on (n - 1) / 3 (row bands of
    // lengths 3j+1..3j+3, e.g. 17 and 18), else of 2 (lengths 3j..3j+2).
    // (n - 1) / 3 as a multiply and shift, exact for n - 1 < 2^16.
    const int32_t n = r1 - r0;
    const uint32_t q = ((uint32_t)(n - 1) * 0xAAABu) >> 17;
    const int32_t tail = __all(q == (uint32_t)__builtin_amdgcn_readfirstlane(q)) ? 3 : 2;
    // every row of every lane of the wave starts 4-aligned: the walk without
    // realignment (typical: all column groups but an image's last one)
    if (__all(((w.off | im.stride) & 3u) == 0))
        walk_rows<K, MODE, HIST, CODES, true, NT>(im, lds_bins, w, n, tail);
    else
        walk_rows<K, MODE, HIST, CODES, false, NT>(im, lds_bins, w, n, tail);
}

// Code rows [r0, r1) of a code map narrower than 8 columns: one lane, the
// pixels past the map masked (counted in the discard cell).
template <int K, int MODE, bool HIST, bool CODES>
__device__ void run_task_narrow(const ImgView &im, uint32_t *lds_bins, uint32_t rowb,
                                const Geom &geo, int32_t r0, int32_t r1)
{
    const int nvalid = im.Wc;
    const uint32_t off = im.off0 + (uint32_t)r0 * im.stride;
    RawRow raw;
    Row t, m, b;
    load_raw<false>(raw, im.rsrc, off);
    unpack_raw<MODE, false>(t, raw);
    load_raw<false>(raw, im.rsrc, off + im.stride);
    unpack_raw<MODE, false>(m, raw);
    uint32_t cb[8];
    if constexpr (HIST) {
        for (int p = 0; p < 8; ++p) {
            const uint32_t cx =
                p < nvalid ? ((uint32_t)p * geo.ax) / geo.bx : (uint32_t)geo.nx;
            cb[p] = rowb + cx * 1024u;
        }
    }
    for (int32_t r = r0; r < r1; ++r) {
        load_raw<false>(raw, im.rsrc, off + (uint32_t)(r + 2 - r0) * im.stride);
        unpack_raw<MODE, false>(b, raw);
        uint32_t q0, q1;
        code_row<K, MODE>(t, m, b, q0, q1);
        if constexpr (CODES) {
            const uint32_t coff = (uint32_t)r * (uint32_t)im.Wc;
            for (int p = 0; p < nvalid; ++p)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)code_of(q0, q1, p), im.crsrc,
                                                     (int)(coff + p), 0, 0);
        }
        if constexpr (HIST) {
            char *lds = reinterpret_cast<char *>(lds_bins);
            for (int p = 0; p < 8; ++p)
                atomicAdd(reinterpret_cast<uint32_t *>(lds + (cb[p] | (code_of(q0, q1, p) << 2))),
                          1u);
        }
        t = m;
        m = b;
    }
}

// ---------------------------------------------------------------- work items
// One workgroup per work item: code rows [r0, r1) of cell rows [cy0, cy1) and
// the cells [cx0, cx1) of those rows (all of them, or a run of at most 63
// when a cell row has more cells than one workgroup's LDS holds; the ranges
// of an image's items tile its cell columns).  When r0/r1 cut a cell row (an
// image split across workgroups) the flush adds atomically into a zeroed
// histogram; otherwise it stores.  Columns just outside the range that a
// group shifted to the range's end computes are stored again with the same
// codes and counted in the discard cell.
//
// Work split: a task is (row band, column group) of one cell row, and a lane
// keeps the same task in every cell row of the item.  With q = threads /
// ngroups >= 1, every column group gets q row bands (fewer if that would make
// bands shorter than min_task_rows); the threads left over, threads - q *
// ngroups, give as many groups one band more, so that no lane idles.  Lanes
// [0, base) take the q-band groups, column group fastest (neighbouring lanes
// read neighbouring columns), lanes [base, threads) the (q+1)-band groups.
// Wider maps (more column groups than threads) take whole cell rows per task.
//
// With COPIES = 2 the LDS holds two copies of the item's histograms,
// copy_words apart, and even and odd lanes count into different copies:
// neighbouring lanes (eight columns apart) often give a pixel the same code,
// and two lanes adding into one LDS word are serialised.  The flush adds the
// copies.  (A compile-time count: with one copy the code is that of a single
// set of histograms, whose per-item work small items feel.)
//
// NT: code and histogram stores are non-temporal, for work whose output is
// mostly histograms (small windows): they stream past the caches instead of
// displacing the image rows that neighbouring lanes still read.
template <int K, int MODE, bool CODES, int COPIES = 1, bool NT = false>
__device__ __forceinline__ void fused_item(const ImgView &im, uint32_t *lds, const Geom &geo,
                                           int32_t cy0, int32_t cy1, int32_t cx0, int32_t cx1,
                                           int32_t r0, int32_t r1, uint32_t *hist,
                                           bool atomic_flush, int32_t min_task_rows,
                                           int32_t copy_words = 0)
{
    static_assert(COPIES == 1 || COPIES == 2, "one or two copies");
    const int tid = threadIdx.x, nthreads = blockDim.x;
    const int32_t ncell = cx1 - cx0;
    const uint32_t row_bytes = hist_row_bytes(ncell);
    const int32_t row_words = (ncell + 1) * 256;
    const int32_t c_lo = geom_col_start(geo, cx0, im.Wc), c_hi = geom_col_start(geo, cx1, im.Wc);
    // 16-byte LDS writes (the histograms start 16-byte aligned and every
    // cell row is a multiple of 1 KB)
#pragma unroll
    for (int32_t c = 0; c < COPIES; ++c) {
        uint4 *lds4 = reinterpret_cast<uint4 *>(lds + c * copy_words);
        for (int32_t i = tid; i < (cy1 - cy0) * (row_words / 4); i += nthreads)
            lds4[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    // this lane's copy
    uint32_t *const bins = COPIES > 1 ? lds + (tid & 1) * copy_words : lds;
    __syncthreads();
    // code rows [a, b) of the current cell row inside [r0, r1)
    int32_t a = max(r0, geom_row_start(geo, cy0, im.Hc));
    int32_t b = min(r1, geom_row_start(geo, cy0 + 1, im.Hc));
    if (im.Wc < 8) {
        for (int32_t cy = cy0; cy < cy1; ++cy) {
            if (cy > cy0) {
                a = b;
                b = min(r1, geom_row_start(geo, cy + 1, im.Hc));
            }
            const int32_t nr = b - a, nsub = min(nthreads, nr);
            if (tid < nsub) {
                const int32_t a0 = a + (int32_t)(((uint32_t)nr * tid) / (uint32_t)nsub);
                const int32_t a1 = a + (int32_t)(((uint32_t)nr * (tid + 1)) / (uint32_t)nsub);
                if (a1 > a0)
                    run_task_narrow<K, MODE, true, CODES>(im, bins, (cy - cy0) * row_bytes, geo,
                                                    a0, a1);
            }
        }
    } else {
        const int32_t ngroups = (c_hi - c_lo + 7) / 8;
        // operands below 2^16 (threads <= 1024, rows <= 65534): udiv_small
        const int32_t q = (int32_t)udiv_small((uint32_t)nthreads, (uint32_t)ngroups);
        if (q >= 1) {
            const int32_t cap = (int32_t)udiv_small((uint32_t)(b - a + min_task_rows - 1),
                                                    (uint32_t)min_task_rows);
            const int32_t nsub = max(1, min(q, cap));
            // groups with one band more (only when bands stay long enough)
            const int32_t nx = (nsub == q && cap > q) ? nthreads - q * ngroups : 0;
            const int32_t base = nsub * (ngroups - nx);
            if (tid < base + (nsub + 1) * nx) {
                uint32_t g, sb, nb;
                if (tid < base) {
                    const uint32_t m = (uint32_t)(ngroups - nx);
                    sb = udiv_small((uint32_t)tid, m);
                    g = (uint32_t)tid - __umul24(sb, m);
                    nb = (uint32_t)nsub;
                } else {
                    sb = udiv_small((uint32_t)(tid - base), (uint32_t)nx);
                    g = (uint32_t)(ngroups - nx) + (uint32_t)(tid - base) - __umul24(sb, (uint32_t)nx);
                    nb = (uint32_t)nsub + 1;
                }
                const Cols c = group_cols<true>(geo, (int32_t)g, c_lo, c_hi, cx0, ncell, im.Wc);
                for (int32_t cy = cy0; cy < cy1; ++cy) {
                    if (cy > cy0) {
                        a = b;
                        b = min(r1, geom_row_start(geo, cy + 1, im.Hc));
                    }
                    // band sb of nb over nr rows: [nr*sb/nb, nr*(sb+1)/nb).  With
                    // nr = qn*nb + rn, nr*s/nb = qn*s + rn*s/nb, and rn*s < nb^2
                    // <= 2^20 (nb <= 1024 threads); every product has factors
                    // below 2^24 and a result below 2^32 (24-bit multiplies)
                    const uint32_t nr = (uint32_t)max(b - a, 0);
                    const uint32_t qn = udiv_small(nr, nb), rn = nr - __umul24(qn, nb);
                    const uint32_t rs = __umul24(rn, sb), qs = __umul24(qn, sb);
                    const int32_t a0 = a + (int32_t)(qs + udiv_small(rs, nb));
                    const int32_t a1 = a + (int32_t)(qs + qn + udiv_small(rs + rn, nb));
                    if (a1 > a0)
                        run_task<K, MODE, true, CODES, NT>(im, bins, (cy - cy0) * row_bytes, c, a0,
                                                           a1);
                }
            }
        } else {
            for (int32_t cy = cy0; cy < cy1; ++cy) {
                if (cy > cy0) {
                    a = b;
                    b = min(r1, geom_row_start(geo, cy + 1, im.Hc));
                }
                for (int32_t g = tid; g < ngroups; g += nthreads)
                    run_task<K, MODE, true, CODES, NT>(
                        im, bins, (cy - cy0) * row_bytes,
                        group_cols<true>(geo, g, c_lo, c_hi, cx0, ncell, im.Wc), a, b);
            }
        }
    }
    __syncthreads();
    // the histograms are device memory: global (not flat) stores and atomics
    typedef __attribute__((address_space(1))) uint32_t global_u32;
    if (!atomic_flush && ((uintptr_t)hist & 15u) == 0) {
        // 16 bytes per access: every cell row is nx * 1 KB in both places
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        typedef __attribute__((address_space(1))) u32x4 global_u32x4;
        for (int32_t r = 0; r < cy1 - cy0; ++r) {
            const u32x4 *src = reinterpret_cast<const u32x4 *>(lds + r * row_words);
            const u32x4 *src1 = reinterpret_cast<const u32x4 *>(lds + copy_words + r * row_words);
            global_u32x4 *dst =
                (global_u32x4 *)(hist + ((int64_t)(cy0 + r) * geo.nx + cx0) * 256);
            for (int32_t i = tid; i < ncell * 64; i += nthreads) {
                const u32x4 v = COPIES > 1 ? src[i] + src1[i] : src[i];
                if constexpr (NT)
                    __builtin_nontemporal_store(v, &dst[i]);
                else
                    dst[i] = v;
            }
        }
        return;
    }
    for (int32_t r = 0; r < cy1 - cy0; ++r) {
        const uint32_t *src = lds + r * row_words;
        global_u32 *dst = (global_u32 *)(hist + ((int64_t)(cy0 + r) * geo.nx + cx0) * 256);
        for (int32_t i = tid; i < ncell * 256; i += nthreads) {
            const uint32_t v = COPIES > 1 ? src[i] + src[copy_words + i] : src[i];
            if (!atomic_flush)
                dst[i] = v;
            else if (v)
                __hip_atomic_fetch_add(dst + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace ldp
