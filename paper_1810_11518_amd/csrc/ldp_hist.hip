// ldp_hist.hip -- per-cell 256-bin histograms of a code map (Eqs. 4-5): the
// second call of the two-call path (ldp_codes, then ldp_histograms), also
// used by the window histograms and by ldp_extract when a cell row has too
// many cells for one workgroup's LDS.
//
// A workgroup takes one work item: the code rows [r0, r1) of one cell row
// and the cells [cx0, cx1) of that row (at most kItemCells of them, so their
// bins fit in LDS with one discard cell).  A lane owns a chunk of 16
// adjacent code columns and a band of the item's rows.  It finds the LDS cell
// of each of its 16 columns once, then walks its rows: 16 codes per row
// (five dword loads from the 4-aligned offset at or below them, realigned;
// four when every row of the wave starts 4-aligned), one LDS add per code,
// or a single add of 16 when all 16 codes are equal and in one cell (flat
// regions, where many lanes would otherwise add to one bin).
//
// The last chunk of a column range is moved left to end at the range's last
// column; the columns it shares with the previous chunk (counted there) go to
// the discard cell, as do the columns past a range narrower than 16.
//
// Every bin is held kCopies times in neighbouring LDS words, lane l adding to
// copy l % kCopies: codes repeat across nearby columns, and lanes adding to
// the same LDS word are serialised, so the copies cut that contention
// kCopies-fold; the flush sums them.
#include "ldp_engine.hpp"
#include "ldp_host.hpp"

namespace ldp {

namespace {

constexpr int kChunk = 16;    // code columns per lane
constexpr int kCopies = 4;    // LDS copies of every bin
constexpr int kItemCells = 7; // cells of a cell row per item: (7 + 1) x 4 KiB of LDS

// LDS byte address of the bin of the (code, cell) pair in one 16-bit half of
// `pr`: half * 4 * kCopies + the lane's base (its copy), one v_mad_u32_u16.
__device__ __forceinline__ uint32_t cbin_lo(uint32_t pr, uint32_t base)
{
    uint32_t r;
    asm("v_mad_u32_u16 %0, %1, 16, %2" : "=v"(r) : "v"(pr), "v"(base));
    return r;
}
__device__ __forceinline__ uint32_t cbin_hi(uint32_t pr, uint32_t base)
{
    uint32_t r;
    asm("v_mad_u32_u16 %0, %1, 16, %2 op_sel:[1,0,0,0]" : "=v"(r) : "v"(pr), "v"(base));
    return r;
}
static_assert(kCopies == 4, "cbin_lo/cbin_hi multiply by 4 * kCopies = 16");

__global__ void hist_zero_kernel(uint32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// One row of a lane's chunk: 16 codes in four words, byte p of q[p / 4] the
// code of column c0 + p.  ALIGNED: the row starts 4-aligned.
template <bool ALIGNED>
__device__ __forceinline__ void load_codes(uint32_t (&q)[4], __amdgpu_buffer_rsrc_t rsrc,
                                           uint32_t off)
{
    if constexpr (ALIGNED) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            q[i] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)(off + 4 * i), 0, 0);
    } else {
        const uint32_t a = off & ~3u, s = off & 3u;
        uint32_t w[5];
#pragma unroll
        for (int i = 0; i < 5; ++i)
            w[i] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)(a + 4 * i), 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            q[i] = __builtin_amdgcn_alignbyte(w[i + 1], w[i], s);
    }
}

// Count one row of 16 codes: q holds the codes, d the LDS cell of each
// column in the same byte positions; `base` is the LDS address of the lane's
// bin copy.
__device__ __forceinline__ void count_row(const uint32_t (&q)[4], const uint32_t (&d)[4],
                                          bool uniform_cell, uint32_t base)
{
    if (uniform_cell && q[0] == q[1] && q[0] == q[2] && q[0] == q[3] &&
        q[0] == __builtin_amdgcn_alignbyte(q[0], q[0], 1)) {
        lds_count(cbin_lo(bin_pair(q[0], d[0], 0, 1), base), 16u);
        return;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t pr = bin_pair(q[i], d[i], 2 * h, 2 * h + 1);
            lds_count(cbin_lo(pr, base), 1u);
            lds_count(cbin_hi(pr, base), 1u);
        }
    }
}

template <bool ALIGNED>
__device__ __forceinline__ void walk_chunk(__amdgpu_buffer_rsrc_t rsrc, uint32_t off,
                                           uint32_t pitch, int32_t n, const uint32_t (&d)[4],
                                           bool uniform_cell, uint32_t base)
{
    uint32_t q[4], nq[4];
    load_codes<ALIGNED>(q, rsrc, off);
    for (int32_t r = 0; r < n; ++r) {
        // prefetch the next row (the last row loads itself again: in bounds)
        off += r + 1 < n ? pitch : 0u;
        load_codes<ALIGNED>(nq, rsrc, off);
        count_row(q, d, uniform_cell, base);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            q[i] = nq[i];
    }
}

// Work item `blockIdx.x` = (cell row cy, cell-column range xi, row part sp).
__global__ void __launch_bounds__(1024) hist_kernel(const uint8_t *__restrict__ codes,
                                                    int32_t Hc, int32_t Wc, Geom geo,
                                                    int32_t cells_per_item, int32_t split,
                                                    int32_t min_band, uint32_t *__restrict__ hist)
{
    extern __shared__ uint32_t lds[];
    const int tid = threadIdx.x, nthreads = blockDim.x;
    const int32_t nxi = (geo.nx + cells_per_item - 1) / cells_per_item;
    const int32_t sp = blockIdx.x % split, t = blockIdx.x / split;
    const int32_t xi = t % nxi, cy = t / nxi;
    const int32_t cx0 = xi * cells_per_item, cx1 = min(cx0 + cells_per_item, geo.nx);
    const int32_t ncell = cx1 - cx0;
    const int32_t ry0 = geom_row_start(geo, cy, Hc), ry1 = geom_row_start(geo, cy + 1, Hc);
    const int32_t r0 = ry0 + (int32_t)((int64_t)(ry1 - ry0) * sp / split);
    const int32_t r1 = ry0 + (int32_t)((int64_t)(ry1 - ry0) * (sp + 1) / split);
    const int32_t c_lo = geom_col_start(geo, cx0, Wc), c_hi = geom_col_start(geo, cx1, Wc);

    uint4 *lds4 = reinterpret_cast<uint4 *>(lds);
    for (int32_t i = tid; i < (ncell + 1) * 64 * kCopies; i += nthreads)
        lds4[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();

    // the item's rows through a bounds-checked buffer descriptor based at the
    // 4-aligned address at or below their start (item offsets stay below
    // 2^30: the host splits cell rows so)
    const uintptr_t p = (uintptr_t)(codes + (int64_t)r0 * Wc), pbase = p & ~(uintptr_t)3;
    const uint32_t off0 = (uint32_t)(p - pbase);
    const int64_t extent = (int64_t)off0 + (int64_t)(r1 - r0) * Wc;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)pbase, (short)0, (int)((extent + 3) & ~(int64_t)3), 0x00020000);
    const uint32_t base = lds_base(lds) + 4u * (uint32_t)(tid % kCopies);

    const int32_t width = c_hi - c_lo, rows = r1 - r0;
    const int32_t nchunks = (width + kChunk - 1) / kChunk;
    // row bands per chunk: enough lanes for every thread, bands of at least
    // min_band rows
    const int32_t q = max(1, min(nthreads / max(nchunks, 1), (rows + min_band - 1) / min_band));
    const bool wide = geo.bx >= (uint32_t)kChunk * geo.ax;  // cells at least 16 columns wide
    for (int32_t task = tid; task < nchunks * q; task += nthreads) {
        const int32_t chunk = task % nchunks, band = task / nchunks;
        const int32_t cs = c_lo + kChunk * chunk;
        const int32_t c0 = cs + kChunk <= c_hi ? cs : max(c_lo, c_hi - kChunk);
        // LDS cell of each column (ncell: discard)
        uint32_t d[4] = {0u, 0u, 0u, 0u};
        const uint32_t cxa = ((uint32_t)c0 * geo.ax) / geo.bx;
        const uint32_t nxt = wide ? (uint32_t)geom_col_start(geo, (int32_t)cxa + 1, Wc) : 0u;
#pragma unroll
        for (int pp = 0; pp < kChunk; ++pp) {
            const uint32_t c = (uint32_t)(c0 + pp);
            const uint32_t cx = wide ? cxa + (c >= nxt ? 1u : 0u) : (c * geo.ax) / geo.bx;
            const bool mine = c0 + pp >= cs && c0 + pp < c_hi;
            d[pp / 4] |= (mine ? cx - (uint32_t)cx0 : (uint32_t)ncell) << (8 * (pp % 4));
        }
        const bool uniform_cell = d[0] == d[1] && d[0] == d[2] && d[0] == d[3] &&
                                  d[0] == __builtin_amdgcn_alignbyte(d[0], d[0], 1);
        const int32_t a0 = r0 + (int32_t)((int64_t)rows * band / q);
        const int32_t a1 = r0 + (int32_t)((int64_t)rows * (band + 1) / q);
        if (a1 <= a0)
            continue;
        const uint32_t off = off0 + (uint32_t)(a0 - r0) * (uint32_t)Wc + (uint32_t)c0;
        if (__all(((off | (uint32_t)Wc) & 3u) == 0))
            walk_chunk<true>(rsrc, off, (uint32_t)Wc, a1 - a0, d, uniform_cell, base);
        else
            walk_chunk<false>(rsrc, off, (uint32_t)Wc, a1 - a0, d, uniform_cell, base);
    }
    __syncthreads();
    // flush: plain stores when the item holds whole cells, else atomic adds
    // into the zeroed histograms
    typedef __attribute__((address_space(1))) uint32_t global_u32;
    global_u32 *dst = (global_u32 *)(hist + ((int64_t)cy * geo.nx + cx0) * 256);
    for (int32_t i = tid; i < ncell * 256; i += nthreads) {
        const uint4 c = lds4[i];  // the kCopies copies of bin i
        const uint32_t v = c.x + c.y + c.z + c.w;
        if (split == 1)
            dst[i] = v;
        else if (v)
            __hip_atomic_fetch_add(dst + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace

int launch_histograms(const uint8_t *codes, int32_t H, int32_t W, int32_t gy, int32_t gx,
                      bool windows, uint32_t *hist, hipStream_t s)
{
    const int32_t Hc = H - 2, Wc = W - 2;
    const Geom geo = make_geom(Hc, Wc, gy, gx, windows);
    const int32_t cpi = std::min<int32_t>(geo.nx, kItemCells);
    const int32_t nxi = (geo.nx + cpi - 1) / cpi;
    const int64_t items = (int64_t)geo.ny * nxi;
    // columns of the widest item: threads for one 16-column chunk each
    const int32_t item_cols = geom_col_start(geo, cpi, Wc);
    const int32_t nchunks = (item_cols + kChunk - 1) / kChunk;
    const int threads = nchunks > 512 ? 1024 : nchunks > 256 ? 512 : 256;
    // split cell rows until there are ~2048 work items, keeping parts of at
    // least 16 rows, and so that no item spans 2^30 bytes of the map
    const int32_t min_band = 8;
    const int64_t max_rows = windows ? (int64_t)geo.by : ((int64_t)Hc + geo.ny - 1) / geo.ny;
    int64_t split = std::max<int64_t>(
        1, std::min<int64_t>(2048 / std::max<int64_t>(items, 1), max_rows / 16));
    split = std::max<int64_t>(split, (max_rows * Wc + (1 << 30) - 1) >> 30);
    split = std::min<int64_t>(split, max_rows);
    if (split > 1) {
        const int64_t n = (int64_t)geo.ny * geo.nx * 256;
        hipLaunchKernelGGL(hist_zero_kernel,
                           dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0,
                           s, hist, n);
    }
    const size_t lds = (size_t)(cpi + 1) * 1024 * kCopies;
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)(items * split)), dim3(threads), lds, s, codes,
                       Hc, Wc, geo, cpi, (int32_t)split, min_band, hist);
    return hipGetLastError() == hipSuccess ? LDP_OK : LDP_ERR_HIP;
}

}  // namespace ldp
