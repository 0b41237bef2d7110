// ldp_kernels.hip -- single-image LDP kernels and their C ABI entry points.
//
//   ldp_codes       codes of every interior pixel (Eqs. 1-3)
//   ldp_histograms  per-cell 256-bin histograms of a code map (Eqs. 4-5;
//                   the kernel is in ldp_hist.hip)
//   ldp_extract     both in one launch, without reading the codes back
#include "ldp_engine.hpp"
#include "ldp_host.hpp"

#ifndef LDP_CODES_LANES
#define LDP_CODES_LANES 524288
#endif
#ifndef LDP_CODES_MIN_BAND
#define LDP_CODES_MIN_BAND 8
#endif

namespace ldp {

// ---------------------------------------------------------------- codes
// One thread per task: task = (row band, column group).
#ifndef LDP_CODES_ATTR
#define LDP_CODES_ATTR
#endif

template <int K, int MODE>
__global__ void __launch_bounds__(256) LDP_CODES_ATTR codes_kernel(const uint8_t *__restrict__ img,
                                                    int64_t stride, int32_t H, int32_t W,
                                                    uint8_t *__restrict__ codes, int32_t band_rows,
                                                    int32_t ngroups, int32_t ntasks)
{
    int32_t task = blockIdx.x * blockDim.x + threadIdx.x;
    if (task >= ntasks)
        return;
    const ImgView im = make_view(img, stride, H, W, codes);
    const int32_t g = task % ngroups;
    const int32_t band = task / ngroups;
    const int32_t r0 = band * band_rows;
    const int32_t r1 = min(r0 + band_rows, im.Hc);
    const Geom none{1, 1, 1, 1, 1, 1};  // no histograms here
    if (im.Wc < 8)
        run_task_narrow<K, MODE, false, true>(im, nullptr, 0, none, r0, r1);
    else
        run_task<K, MODE, false, true>(im, nullptr, 0,
                                       group_cols<false>(none, g, 0, im.Wc, 0, 0, im.Wc), r0, r1);
}

__global__ void zero_kernel(uint32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---------------------------------------------------------------- fused
// Workgroup = (cell row cy, cell-column run xi of nxi, row part sp of split).
template <int K, int MODE, bool CODES>
__global__ void __launch_bounds__(1024) fused_kernel(const uint8_t *__restrict__ img,
                                                     int64_t stride, int32_t H, int32_t W,
                                                     uint8_t *codes, uint32_t *hist, Geom geo,
                                                     int32_t nxi, int32_t split)
{
    extern __shared__ uint32_t lds[];
    const ImgView im = make_view(img, stride, H, W, codes);
    const int32_t sp = blockIdx.x % split, t = blockIdx.x / split;
    const int32_t xi = t % nxi, cy = t / nxi;
    const int32_t cx0 = cell_run_start(geo.nx, nxi, xi), cx1 = cell_run_start(geo.nx, nxi, xi + 1);
    const int32_t ry0 = geom_row_start(geo, cy, im.Hc), ry1 = geom_row_start(geo, cy + 1, im.Hc);
    const int32_t r0 = ry0 + (int32_t)((int64_t)(ry1 - ry0) * sp / split);
    const int32_t r1 = ry0 + (int32_t)((int64_t)(ry1 - ry0) * (sp + 1) / split);
    fused_item<K, MODE, CODES>(im, lds, geo, cy, cy + 1, cx0, cx1, r0, r1, hist, split > 1, 4);
}

// ---------------------------------------------------------------- dispatch
// F<K, MODE, FLAG>::launch(args...) for k in 1..8, the kernel mode and a flag
// (LBP codes do not depend on k: one instantiation).
template <template <int, int, bool> class F, typename... Args>
static hipError_t dispatch(int k, int mode, bool flag, Args &&...args)
{
    if (mode == CODE_LBP)
        return flag ? F<1, CODE_LBP, true>::launch(args...) : F<1, CODE_LBP, false>::launch(args...);
#define LDP_MODE(KK, MM)                                                                    \
    case MM:                                                                                \
        return flag ? F<KK, MM, true>::launch(args...) : F<KK, MM, false>::launch(args...);
#define LDP_CASE(KK)                                                                        \
    case KK:                                                                                \
        switch (mode) {                                                                     \
            LDP_MODE(KK, RANK_SIGNED) LDP_MODE(KK, RANK_MAGNITUDE) LDP_MODE(KK, DIRECT_MASKS) \
        }                                                                                   \
        break;
    switch (k) {
        LDP_CASE(1) LDP_CASE(2) LDP_CASE(3) LDP_CASE(4)
        LDP_CASE(5) LDP_CASE(6) LDP_CASE(7) LDP_CASE(8)
    }
#undef LDP_CASE
#undef LDP_MODE
    return hipErrorInvalidValue;
}

template <int K, int MODE, bool UNUSED>
struct CodesLaunch {
    static hipError_t launch(dim3 grid, dim3 block, hipStream_t s, const uint8_t *img,
                             int64_t stride, int32_t H, int32_t W, uint8_t *codes, int32_t band,
                             int32_t ngroups, int32_t ntasks)
    {
        if constexpr (UNUSED)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL((codes_kernel<K, MODE>), grid, block, 0, s, img, stride, H, W, codes,
                           band, ngroups, ntasks);
        return hipGetLastError();
    }
};

template <int K, int MODE, bool CODES>
struct FusedLaunch {
    static hipError_t launch(dim3 grid, dim3 block, size_t lds, hipStream_t s, const uint8_t *img,
                             int64_t stride, int32_t H, int32_t W, uint8_t *codes,
                             uint32_t *hist, Geom geo, int32_t nxi, int32_t split)
    {
        hipLaunchKernelGGL((fused_kernel<K, MODE, CODES>), grid, block, lds, s, img, stride, H, W,
                           codes, hist, geo, nxi, split);
        return hipGetLastError();
    }
};

int launch_codes(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                 int32_t flags, uint8_t *codes, hipStream_t s)
{
    const int32_t Hc = H - 2, Wc = W - 2;
    const int32_t ngroups = (Wc + 7) / 8;
    // band height: enough lanes to keep every SIMD several waves deep
    int64_t lanes_rows = (int64_t)ngroups * Hc;
    int32_t band = (int32_t)std::min<int64_t>(64, std::max<int64_t>(LDP_CODES_MIN_BAND, lanes_rows / LDP_CODES_LANES + 1));
    int32_t nbands = (Hc + band - 1) / band;
    int32_t ntasks = ngroups * nbands;
    dim3 block(256), grid((ntasks + 255) / 256);
    hipError_t e = dispatch<CodesLaunch>(k, rank_mode(flags), false, grid, block, s, img,
                                         stride, H, W, codes, band, ngroups, ntasks);
    return e == hipSuccess ? LDP_OK : LDP_ERR_HIP;
}

int launch_extract(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                   int32_t flags, int32_t gy, int32_t gx, bool windows, uint8_t *codes,
                   uint32_t *hist, hipStream_t s)
{
    const int32_t Hc = H - 2, Wc = W - 2;
    const Geom geo = make_geom(Hc, Wc, gy, gx, windows);
    // cell rows with more cells than one workgroup's LDS holds are cut into
    // runs of at most kMaxFusedCellsX cells
    const int32_t nxi = cell_runs(geo.nx);
    const int32_t run_cells = (geo.nx + nxi - 1) / nxi;
    const int32_t ngroups = (geom_col_start(geo, run_cells, Wc) + 7) / 8;
    int threads = ngroups >= 768 ? 1024 : ngroups >= 384 ? 512 : 256;
    // enough workgroups to fill the device: split cell rows
    int32_t split = 1;
    const int32_t rows_per_cell = Hc / geo.ny;
    while ((int64_t)geo.ny * nxi * split < 512 && rows_per_cell / (split * 2) >= 8 && split < 64)
        split *= 2;
    if (split > 1) {
        int64_t n = (int64_t)geo.ny * geo.nx * 256;
        hipLaunchKernelGGL(zero_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)),
                           dim3(256), 0, s, hist, n);
    }
    const size_t lds = hist_row_bytes(run_cells);
    hipError_t e = dispatch<FusedLaunch>(k, rank_mode(flags), codes != nullptr,
                                         dim3((unsigned)((int64_t)geo.ny * nxi * split)),
                                         dim3(threads), lds, s, img, stride, H, W, codes, hist,
                                         geo, nxi, split);
    return e == hipSuccess ? LDP_OK : LDP_ERR_HIP;
}

}  // namespace ldp

// ---------------------------------------------------------------- C ABI
extern "C" {

int ldp_codes_ex(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                 int32_t flags, uint8_t *codes, ldp_stream_t stream)
{
    int st = ldp::check_image(img, H, W, stride);
    if (st != LDP_OK)
        return st;
    if (!codes || k < 1 || k > 8 || !ldp::flags_ok(flags))
        return LDP_ERR_INVALID_ARG;
    return ldp::launch_codes(img, H, W, stride, k, flags, codes, (hipStream_t)stream);
}

int ldp_codes(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
              uint8_t *codes, ldp_stream_t stream)
{
    return ldp_codes_ex(img, H, W, stride, k, 0, codes, stream);
}

int ldp_histograms(const uint8_t *codes, int32_t H, int32_t W, int32_t cells_y,
                   int32_t cells_x, uint32_t *hist, ldp_stream_t stream)
{
    if (!codes || !hist || H < 3 || W < 3 || H > LDP_MAX_SIDE || W > LDP_MAX_SIDE)
        return LDP_ERR_INVALID_ARG;
    int st = ldp::check_cells(H, W, cells_y, cells_x);
    if (st != LDP_OK)
        return st;
    return ldp::launch_histograms(codes, H, W, cells_y, cells_x, false, hist, (hipStream_t)stream);
}

int ldp_extract_ex(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                   int32_t flags, int32_t cells_y, int32_t cells_x, uint8_t *codes,
                   uint32_t *hist, ldp_stream_t stream)
{
    int st = ldp::check_image(img, H, W, stride);
    if (st != LDP_OK)
        return st;
    if (!hist || k < 1 || k > 8 || !ldp::flags_ok(flags))
        return LDP_ERR_INVALID_ARG;
    st = ldp::check_cells(H, W, cells_y, cells_x);
    if (st != LDP_OK)
        return st;
    return ldp::launch_extract(img, H, W, stride, k, flags, cells_y, cells_x, false, codes, hist,
                               (hipStream_t)stream);
}

int ldp_extract(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                int32_t cells_y, int32_t cells_x, uint8_t *codes, uint32_t *hist,
                ldp_stream_t stream)
{
    return ldp_extract_ex(img, H, W, stride, k, 0, cells_y, cells_x, codes, hist, stream);
}

int ldp_window_grid(int32_t H, int32_t W, int32_t win_y, int32_t win_x, int32_t *ny,
                    int32_t *nx)
{
    if (H < 3 || W < 3 || H > LDP_MAX_SIDE || W > LDP_MAX_SIDE || win_y < 1 || win_x < 1)
        return LDP_ERR_INVALID_ARG;
    const ldp::Geom geo = ldp::make_geom(H - 2, W - 2, win_y, win_x, true);
    if (ny)
        *ny = geo.ny;
    if (nx)
        *nx = geo.nx;
    return LDP_OK;
}

int ldp_histograms_windows(const uint8_t *codes, int32_t H, int32_t W, int32_t win_y,
                           int32_t win_x, uint32_t *hist, ldp_stream_t stream)
{
    if (!codes || !hist || H < 3 || W < 3 || H > LDP_MAX_SIDE || W > LDP_MAX_SIDE || win_y < 1 ||
        win_x < 1)
        return LDP_ERR_INVALID_ARG;
    return ldp::launch_histograms(codes, H, W, win_y, win_x, true, hist, (hipStream_t)stream);
}

int ldp_extract_windows(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                        int32_t flags, int32_t win_y, int32_t win_x, uint8_t *codes,
                        uint32_t *hist, ldp_stream_t stream)
{
    int st = ldp::check_image(img, H, W, stride);
    if (st != LDP_OK)
        return st;
    if (!hist || k < 1 || k > 8 || !ldp::flags_ok(flags) || win_y < 1 || win_x < 1)
        return LDP_ERR_INVALID_ARG;
    return ldp::launch_extract(img, H, W, stride, k, flags, win_y, win_x, true, codes, hist,
                               (hipStream_t)stream);
}

}  // extern "C"
