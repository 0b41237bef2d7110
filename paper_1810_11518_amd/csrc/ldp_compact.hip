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

__global__ void __launch_bounds__(256) compact_kernel(const uint32_t *__restrict__ hist,
                                                      int64_t n_cells, int32_t k, int32_t npat,
                                                      uint32_t *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t cell = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
         cell < n_cells; cell += waves) {
        const uint32_t *h = hist + cell * 256;
        uint32_t *o = out + cell * (npat + 1);
        uint32_t rest = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int code = lane + 64 * q;
            const uint32_t v = h[code];
            const int b = kCompact.bin[k][code];
            if (b < npat)
                o[b] = v;
            else
                rest += v;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            rest += __shfl_xor(rest, off);
        if (lane == 0)
            o[npat] = rest;
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
    // one cell per wave (a loop only beyond 2^20 workgroups): many loads in flight
    const int64_t blocks = std::min<int64_t>((n_cells + 3) / 4, int64_t(1) << 20);
    hipLaunchKernelGGL(ldp::compact_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, hist, n_cells, k, npat, out);
    return hipGetLastError() == hipSuccess ? LDP_OK : LDP_ERR_HIP;
}

}  // extern "C"
