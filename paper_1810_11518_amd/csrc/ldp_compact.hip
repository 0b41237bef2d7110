// ldp_compact.hip -- Eq. 6's compact feature vector from 256-bin histograms.
//
// For k, the pattern values C_1 < C_2 < ... (Eq. 4) are the C(8, k) codes with
// exactly k bits set, in ascending order; a cell's compact vector is
// (H_1, ..., H_C(8,k)) followed by one bin counting every other code (codes
// with more than k bits come from ties with m_k).  One wave per cell: lane l
// reads bins l, l+64, l+128, l+192 (coalesced), stores the pattern bins to
// their places and sums the rest across the wave.
#include <stdint.h>

#include "ldp_host.hpp"

namespace ldp {

struct CompactTables {
    uint8_t bin[9][256];  // [k][code]: position among the k-bit codes, or C(8, k)
};

constexpr int bit_count(int v)
{
    int n = 0;
    for (; v; v >>= 1)
        n += v & 1;
    return n;
}

constexpr CompactTables make_compact_tables()
{
    CompactTables t{};
    for (int k = 0; k <= 8; ++k) {
        int n = 0;
        for (int c = 0; c < 256; ++c)
            if (bit_count(c) == k)
                t.bin[k][c] = (uint8_t)n++;
        for (int c = 0; c < 256; ++c)
            if (bit_count(c) != k)
                t.bin[k][c] = (uint8_t)n;
    }
    return t;
}

__constant__ CompactTables kCompact = make_compact_tables();

constexpr int32_t compact_patterns(int k)
{
    int n = 0;
    for (int c = 0; c < 256; ++c)
        n += bit_count(c) == k;
    return n;
}

#ifndef LDP_COMPACT_CELLS_PER_WAVE
#define LDP_COMPACT_CELLS_PER_WAVE 4
#endif
#ifndef LDP_COMPACT_MAX_BLOCKS
#define LDP_COMPACT_MAX_BLOCKS 8192
#endif

// Each wave takes LDP_COMPACT_CELLS_PER_WAVE consecutive cells per round and
// issues all their loads before using them (more loads in flight).
__global__ void __launch_bounds__(256) compact_kernel(const uint32_t *__restrict__ hist,
                                                      int64_t n_cells, int32_t k, int32_t npat,
                                                      uint32_t *__restrict__ out)
{
    constexpr int C = LDP_COMPACT_CELLS_PER_WAVE;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    int b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        b[q] = kCompact.bin[k][lane + 64 * q];
    for (int64_t c0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * C;
         c0 < n_cells; c0 += waves * C) {
        uint32_t v[C][4];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                v[c][q] = c0 + c < n_cells ? hist[(c0 + c) * 256 + lane + 64 * q] : 0u;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (c0 + c >= n_cells)
                break;
            uint32_t *o = out + (c0 + c) * (npat + 1);
            uint32_t rest = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (b[q] < npat)
                    o[b[q]] = v[c][q];
                else
                    rest += v[c][q];
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1)
                rest += __shfl_xor(rest, off);
            if (lane == 0)
                o[npat] = rest;
        }
    }
}

}  // namespace ldp

extern "C" {

int32_t ldp_compact_bins(int32_t k)
{
    if (k < 1 || k > 8)
        return LDP_ERR_INVALID_ARG;
    return ldp::compact_patterns(k) + 1;
}

int ldp_compact_histograms(const uint32_t *hist, int64_t n_cells, int32_t k, uint32_t *out,
                           ldp_stream_t stream)
{
    if (k < 1 || k > 8 || n_cells < 0 || (n_cells > 0 && (!hist || !out)))
        return LDP_ERR_INVALID_ARG;
    if (n_cells == 0)
        return LDP_OK;
    const int32_t npat = ldp::compact_patterns(k);
    const int64_t cells_per_block = 4 * LDP_COMPACT_CELLS_PER_WAVE;
    const int64_t blocks =
        std::min<int64_t>((n_cells + cells_per_block - 1) / cells_per_block, LDP_COMPACT_MAX_BLOCKS);
    hipLaunchKernelGGL(ldp::compact_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, hist, n_cells, k, npat, out);
    return hipGetLastError() == hipSuccess ? LDP_OK : LDP_ERR_HIP;
}

}  // extern "C"
