// ldp_host.hpp -- host-side argument checks and launch helpers shared by the
// single-image entry points, the batch plan and the server.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/ldp.h"

namespace ldp {

// Largest byte extent of one image that the 32-bit buffer offsets address.
constexpr int64_t kMaxExtent = (int64_t(1) << 31) - 64;

inline int check_image(const uint8_t *img, int32_t H, int32_t W, int64_t stride)
{
    if (!img || H < 3 || W < 3 || H > LDP_MAX_SIDE || W > LDP_MAX_SIDE || stride < W)
        return LDP_ERR_INVALID_ARG;
    if ((int64_t)(H - 1) * stride + W + 8 > kMaxExtent)
        return LDP_ERR_UNSUPPORTED;
    return LDP_OK;
}

inline int check_cells(int32_t H, int32_t W, int32_t cells_y, int32_t cells_x)
{
    if (cells_y < 1 || cells_x < 1 || cells_y > H - 2 || cells_x > W - 2)
        return LDP_ERR_INVALID_ARG;
    return LDP_OK;
}

// At most one flag: the variants exclude each other.
inline bool flags_ok(int32_t flags)
{
    return flags == 0 || flags == LDP_RANK_MAGNITUDE || flags == LDP_DIRECT_MASKS ||
           flags == LDP_CODE_LBP;
}

// Kernel mode (ldp_device.hpp: RANK_SIGNED 0, RANK_MAGNITUDE 1, DIRECT_MASKS 2,
// CODE_LBP 3) for valid public flags.
inline int rank_mode(int32_t flags)
{
    return flags == LDP_RANK_MAGNITUDE ? 1 : flags == LDP_DIRECT_MASKS ? 2 : flags == LDP_CODE_LBP ? 3 : 0;
}

// Largest cells_x the fused kernels keep in LDS (one cell row, 1 KiB per
// cell, plus a discard cell).
constexpr int32_t kMaxFusedCellsX = 63;

int launch_codes(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                 int32_t flags, uint8_t *codes, hipStream_t s);
// (gy, gx) are the cell counts (cells_y, cells_x), or with `windows` the
// window sides in code pixels.
int launch_histograms(const uint8_t *codes, int32_t H, int32_t W, int32_t gy, int32_t gx,
                      bool windows, uint32_t *hist, hipStream_t s);
int launch_extract(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                   int32_t flags, int32_t gy, int32_t gx, bool windows, uint8_t *codes,
                   uint32_t *hist, hipStream_t s);

// Sets an empty batch on plan `p` and launches its graph on `s` anyway (its
// workgroups find no work items and exit), and likewise the kernel that
// takes a batch in its arguments: the first launch of a kernel on a stream
// pays one-time runtime set-up, which a server takes at creation instead of
// on its first requests.
int warm_plan(ldp_batch_plan *p, hipStream_t s);

// ldp_batch_launch: runs batch `descs[0..n)` on plan `p` on stream `s`,
// checked as ldp_batch_plan_set checks it.  A signed-ranking cell-grid batch
// of at most LDP_ARG_BATCH_IMAGES images and LDP_ARG_BATCH_ITEMS work items
// is launched with its tables in the kernel's arguments (no table upload, no
// graph; the plan's loaded batch is left as it was); any other batch is
// loaded with ldp_batch_plan_set and run.
int run_batch(ldp_batch_plan *p, const ldp_image_desc *descs, int32_t n, hipStream_t s);

}  // namespace ldp
