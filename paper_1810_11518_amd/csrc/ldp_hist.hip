// ldp_hist.hip -- per-cell 256-bin histograms of a code map (Eqs. 4-5): the
// second call of the two-call path (ldp_codes, then ldp_histograms), also
// used by the window histograms.
//
// A workgroup takes one work item: the code rows [r0, r1) of one cell.  A
// lane owns a chunk of 16 adjacent code columns of the cell and a band of the
// item's rows; per row it loads the 16 codes (five dword loads from the
// 4-aligned offset at or below them, realigned; four when every row of the
// wave starts 4-aligned) and adds one to each code's bin in LDS, or 16 at
// once when all 16 codes are equal (flat regions).
//
// Every bin is held in 32 copies, lane l adding to copy l % 32, and copy c of
// bin b is LDS word b * 32 + c: the 32 lanes of a half-wave always add into
// 32 different LDS banks, whatever their codes, so the adds never wait on
// each other; the flush sums the copies.  The columns of a chunk that lie
// outside the cell (the last chunk of a cell is moved left to end at the
// cell's last column, and a cell narrower than 16 columns leaves some over)
// go to a 257th, discard bin.
#include "ldp_engine.hpp"
#include "ldp_host.hpp"

namespace ldp {

namespace {

constexpr int kChunk = 16;         // code columns per lane
constexpr int kCopies = 32;        // LDS copies of every bin
constexpr int kBins = 257;         // 256 codes and the discard bin
constexpr int kLdsBytes = kBins * kCopies * 4;

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

// LDS byte address of the bin in one 16-bit half of `pr` (the code, plus 256
// for the discard bin): half * 4 * kCopies + the lane's copy base, one
// v_mad_u32_u16 (the multiplier, 128, in a scalar register).
__device__ __forceinline__ uint32_t xbin_lo(uint32_t pr, uint32_t mul, uint32_t base)
{
    uint32_t r;
    asm("v_mad_u32_u16 %0, %1, %2, %3" : "=v"(r) : "v"(pr), "s"(mul), "v"(base));
    return r;
}
__device__ __forceinline__ uint32_t xbin_hi(uint32_t pr, uint32_t mul, uint32_t base)
{
    uint32_t r;
    asm("v_mad_u32_u16 %0, %1, %2, %3 op_sel:[1,0,0,0]" : "=v"(r) : "v"(pr), "s"(mul), "v"(base));
    return r;
}

// The per-lane view of a chunk: `keep` has 0xFF in the bytes of the columns
// the lane counts and 0 elsewhere; `disc` has 1 in the other bytes (their
// code, masked to 0, then addresses bin 256).
struct Chunk {
    uint32_t keep[4], disc[4];
    bool all_mine;
};

__device__ __forceinline__ void count_row(const uint32_t (&q)[4], const Chunk &ch, uint32_t mul,
                                          uint32_t base)
{
    if (ch.all_mine && q[0] == q[1] && q[0] == q[2] && q[0] == q[3] &&
        q[0] == __builtin_amdgcn_alignbyte(q[0], q[0], 1)) {
        lds_count(xbin_lo(bin_pair(q[0], 0u, 0, 1), mul, base), 16u);
        return;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t x = q[i] & ch.keep[i];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t pr = bin_pair(x, ch.disc[i], 2 * h, 2 * h + 1);
            lds_count(xbin_lo(pr, mul, base), 1u);
            lds_count(xbin_hi(pr, mul, base), 1u);
        }
    }
}

template <bool ALIGNED>
__device__ __forceinline__ void walk_chunk(__amdgpu_buffer_rsrc_t rsrc, uint32_t off,
                                           uint32_t pitch, int32_t n, const Chunk &ch,
                                           uint32_t mul, uint32_t base)
{
    uint32_t q[4], nq[4];
    load_codes<ALIGNED>(q, rsrc, off);
    for (int32_t r = 0; r < n; ++r) {
        // prefetch the next row (the last row loads itself again: in bounds)
        off += r + 1 < n ? pitch : 0u;
        load_codes<ALIGNED>(nq, rsrc, off);
        count_row(q, ch, mul, base);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            q[i] = nq[i];
    }
}

// Work item `blockIdx.x` = (cell (cy, cx), row part sp of split).
__global__ void __launch_bounds__(1024) hist_kernel(const uint8_t *__restrict__ codes,
                                                   int32_t Hc, int32_t Wc, Geom geo, int32_t split,
                                                   int32_t min_band, uint32_t *__restrict__ hist)
{
    extern __shared__ uint32_t lds[];
    const int tid = threadIdx.x, nthreads = blockDim.x;
    const int32_t sp = blockIdx.x % split, t = blockIdx.x / split;
    const int32_t cx = t % geo.nx, cy = t / geo.nx;
    const int32_t ry0 = geom_row_start(geo, cy, Hc), ry1 = geom_row_start(geo, cy + 1, Hc);
    const int32_t r0 = ry0 + (int32_t)((int64_t)(ry1 - ry0) * sp / split);
    const int32_t r1 = ry0 + (int32_t)((int64_t)(ry1 - ry0) * (sp + 1) / split);
    const int32_t c_lo = geom_col_start(geo, cx, Wc), c_hi = geom_col_start(geo, cx + 1, Wc);

    uint4 *lds4 = reinterpret_cast<uint4 *>(lds);
    for (int32_t i = tid; i < kLdsBytes / 16; i += nthreads)
        lds4[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();

    // the item's rows through a bounds-checked buffer descriptor based at the
    // 4-aligned address at or below their start (item offsets stay below
    // 2^30: the host splits cells so)
    const uintptr_t p = (uintptr_t)(codes + (int64_t)r0 * Wc), pbase = p & ~(uintptr_t)3;
    const uint32_t off0 = (uint32_t)(p - pbase);
    const int64_t extent = (int64_t)off0 + (int64_t)(r1 - r0) * Wc;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)pbase, (short)0, (int)((extent + 3) & ~(int64_t)3), 0x00020000);
    const uint32_t base = lds_base(lds) + 4u * (uint32_t)(tid % kCopies);
    const uint32_t mul = 4u * kCopies;

    const int32_t width = c_hi - c_lo, rows = r1 - r0;
    const int32_t nchunks = (width + kChunk - 1) / kChunk;
    // row bands per chunk: enough lanes for every thread, bands of at least
    // min_band rows
    const int32_t q = max(1, min(nthreads / max(nchunks, 1), (rows + min_band - 1) / min_band));
    for (int32_t task = tid; task < nchunks * q; task += nthreads) {
        const int32_t chunk = task % nchunks, band = task / nchunks;
        const int32_t cs = c_lo + kChunk * chunk;
        const int32_t c0 = cs + kChunk <= c_hi ? cs : max(c_lo, c_hi - kChunk);
        Chunk ch;
        ch.all_mine = true;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ch.keep[i] = 0u;
            ch.disc[i] = 0u;
        }
#pragma unroll
        for (int pp = 0; pp < kChunk; ++pp) {
            const bool mine = c0 + pp >= cs && c0 + pp < c_hi;
            ch.keep[pp / 4] |= (mine ? 0xFFu : 0u) << (8 * (pp % 4));
            ch.disc[pp / 4] |= (mine ? 0u : 1u) << (8 * (pp % 4));
            ch.all_mine = ch.all_mine && mine;
        }
        const int32_t a0 = r0 + (int32_t)((int64_t)rows * band / q);
        const int32_t a1 = r0 + (int32_t)((int64_t)rows * (band + 1) / q);
        if (a1 <= a0)
            continue;
        const uint32_t off = off0 + (uint32_t)(a0 - r0) * (uint32_t)Wc + (uint32_t)c0;
        if (__all(((off | (uint32_t)Wc) & 3u) == 0))
            walk_chunk<true>(rsrc, off, (uint32_t)Wc, a1 - a0, ch, mul, base);
        else
            walk_chunk<false>(rsrc, off, (uint32_t)Wc, a1 - a0, ch, mul, base);
    }
    __syncthreads();
    // flush: each bin is the sum of its 32 copies; plain stores when the item
    // holds the whole cell, else atomic adds into the zeroed histograms
    typedef __attribute__((address_space(1))) uint32_t global_u32;
    global_u32 *dst = (global_u32 *)(hist + ((int64_t)cy * geo.nx + cx) * 256);
    for (int32_t b = tid; b < 256; b += nthreads) {
        uint32_t v = 0;
#pragma unroll
        for (int i = 0; i < kCopies / 4; ++i) {
            const uint4 c = lds4[b * (kCopies / 4) + i];
            v += c.x + c.y + c.z + c.w;
        }
        if (split == 1)
            dst[b] = v;
        else if (v)
            __hip_atomic_fetch_add(dst + b, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace

int launch_histograms(const uint8_t *codes, int32_t H, int32_t W, int32_t gy, int32_t gx,
                      bool windows, uint32_t *hist, hipStream_t s)
{
    const int32_t Hc = H - 2, Wc = W - 2;
    const Geom geo = make_geom(Hc, Wc, gy, gx, windows);
    const int64_t cells = (int64_t)geo.ny * geo.nx;
    // split cells into row parts until there are ~2048 work items, keeping
    // parts of at least 32 rows, and so that no item spans 2^30 bytes
    const int32_t min_band = 4;
    const int64_t max_rows = windows ? (int64_t)geo.by : ((int64_t)Hc + geo.ny - 1) / geo.ny;
    int64_t split = std::max<int64_t>(
        1, std::min<int64_t>(2048 / std::max<int64_t>(cells, 1), max_rows / 32));
    split = std::max<int64_t>(split, (max_rows * Wc + (1 << 30) - 1) >> 30);
    split = std::min<int64_t>(split, max_rows);
    if (cells * split > INT32_MAX)
        return LDP_ERR_UNSUPPORTED;
    // workgroup size: the one of 256, 512, 1024 threads whose lanes the
    // 16-column chunks of the widest cell (times whole row bands) fill best
    const int32_t cell_cols = geom_col_start(geo, 1, Wc);
    const int32_t nchunks = std::max<int32_t>(1, (cell_cols + kChunk - 1) / kChunk);
    int threads = 256;
    double best = -1.0;
    for (int t : {256, 512, 1024}) {
        const double used = nchunks <= t ? (double)(nchunks * (t / nchunks)) / t
                                         : (double)nchunks / ((double)t * ((nchunks + t - 1) / t));
        if (used > best + 0.02) {
            best = used;
            threads = t;
        }
    }
    if (split > 1) {
        const int64_t n = cells * 256;
        hipLaunchKernelGGL(hist_zero_kernel,
                           dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0,
                           s, hist, n);
    }
    hipLaunchKernelGGL(hist_kernel, dim3((unsigned)(cells * split)), dim3(threads), kLdsBytes, s,
                       codes, Hc, Wc, geo, (int32_t)split, min_band, hist);
    return hipGetLastError() == hipSuccess ? LDP_OK : LDP_ERR_HIP;
}

}  // namespace ldp
