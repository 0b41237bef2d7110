// ldp_batch.hip -- many images of any sizes in one persistent launch.
//
// The host cuts every image into work items of whole cell rows, so each
// item's histogram cells belong to exactly one workgroup and are written with
// plain stores (no atomics, no zeroing pass).  Items are sorted largest
// first and pulled by the resident workgroups from a device queue counter,
// which the last workgroup to find the queue empty resets for the next
// launch.  The persistent kernel is captured once in a HIP graph when the
// plan is made; it reads the item count and tables from device memory, so
// loading a new batch never re-captures the graph.  A batch small enough to
// travel in the kernel's arguments can instead be launched directly with its
// tables as arguments (no upload: `run_batch`).
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "ldp_engine.hpp"
#include "ldp_host.hpp"

namespace ldp {

// A work item: cell rows [cy0, cy1) and cell columns [cx0, cx1) of one image
// (at most 65534 of either).  The image's size class (whose target code rows
// per lane task the kernel takes from its MinRows argument) sits in the top
// two bits of `img`, the descriptor index in the rest.
struct Item {
    uint32_t img;
    uint16_t cy0, cy1;
    uint16_t cx0, cx1;
};
constexpr uint32_t kImgBits = 30;
constexpr int32_t kMaxPlanImages = (int32_t)(1u << kImgBits);

struct MinRows {
    int32_t v[LDP_MAX_SIZE_CLASSES];
};

// The queue of a launch: item count, next item number, workgroups that found
// the queue empty, item table.  The last workgroup to find it empty resets
// `next` and `exited` to 0, so a replay of the same batch starts a fresh queue
// (a new batch uploads zeros with its tables).  The item table's address is
// read from here because a window plan's table can grow when a new batch is
// loaded, without re-capturing the graph.
struct Meta {
    uint32_t n_items, next, exited, unused;
    const Item *items;
};

// At least 5 waves per SIMD: at most 96 VGPRs (allocated in steps of 8), the
// occupancy the batch kernel is tuned for (4 waves measure ~17% slower).
#ifndef LDP_BATCH_ATTR
#define LDP_BATCH_ATTR __attribute__((amdgpu_waves_per_eu(5)))
#endif

typedef __attribute__((address_space(4))) const Item ConstItem;  // read-only while a kernel runs

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}

// Tables of a launch read from device memory (the graph launch).  The item
// table does not change while a kernel runs: it is read through the constant
// address space, so an item (and the descriptor it indexes) arrives in scalar
// registers.
struct DeviceTables {
    const ConstItem *items;
    const ldp_image_desc *descs;
    __device__ __forceinline__ Item item(uint32_t i) const
    {
        const ConstItem &ci = items[i];
        Item w;
        w.img = ci.img;
        w.cy0 = ci.cy0;
        w.cy1 = ci.cy1;
        w.cx0 = ci.cx0;
        w.cx1 = ci.cx1;
        return w;
    }
    __device__ __forceinline__ ldp_image_desc desc(int32_t j) const { return descs[j]; }
};

// A batch carried in the kernel's arguments: at most kArgImages images and
// kArgItems work items (3,480 bytes of arguments).
constexpr int32_t kArgImages = LDP_ARG_BATCH_IMAGES, kArgItems = LDP_ARG_BATCH_ITEMS;
struct ArgBatch {
    uint32_t n_items, unused;
    ldp_image_desc descs[kArgImages];
    Item items[kArgItems];
};

struct ArgTables {
    const ArgBatch *b;  // the kernel's argument segment
    __device__ __forceinline__ Item item(uint32_t i) const { return b->items[i]; }
    __device__ __forceinline__ ldp_image_desc desc(int32_t j) const { return b->descs[j]; }
};

// The work of one workgroup: pull item numbers from the queue counter until
// all n_items are taken, each item a fused pass over its cell rows.
// (gy, gx): cells_y x cells_x cells, or with `windows` window sides in code
// pixels (every image's cell grid follows from its own size).  The item
// number is broadcast through the LDS word after the histograms (`item_slot`,
// in words): the kernels have no static LDS, and the histograms start at the
// beginning of the dynamic LDS, in COPIES (1 or 2) copies item_slot /
// COPIES words apart.
template <int K, int MODE, int COPIES, bool NT, class Tables>
__device__ __forceinline__ void run_queue(const Tables &tab, uint32_t n_items, Meta *meta,
                                          int32_t gy, int32_t gx, int32_t windows,
                                          int32_t item_slot, const MinRows &min_rows)
{
    extern __shared__ uint32_t lds[];
    uint32_t &s_item = lds[item_slot];
    for (;;) {
        if (threadIdx.x == 0)
            s_item = atomicAdd(&meta->next, 1u);
        __syncthreads();
        const uint32_t it = uniform(s_item);
        __syncthreads();
        if (it >= n_items)
            break;
        const Item w = tab.item(it);
        const ldp_image_desc d = tab.desc((int32_t)(w.img & ((1u << kImgBits) - 1u)));
        const int32_t task_rows = min_rows.v[w.img >> kImgBits];
        uint32_t *hist = d.hist;
        ImgView im = make_view(d.img, d.stride, d.H, d.W, d.codes);
        const Geom geo = make_geom(im.Hc, im.Wc, gy, gx, windows != 0);
        const int32_t r0 = geom_row_start(geo, w.cy0, im.Hc);
        const int32_t r1 = geom_row_start(geo, w.cy1, im.Hc);
        // a null code pointer gives an empty store range: stores are dropped
        fused_item<K, MODE, true, COPIES, NT>(im, lds, geo, w.cy0, w.cy1, w.cx0, w.cx1, r0, r1,
                                              hist, false, task_rows, item_slot / COPIES);
    }
    // Every workgroup has taken its last number once all have counted
    // themselves here: the last one resets the queue for the next launch
    // (atomics: device-scope, through L2).
    if (threadIdx.x == 0 && atomicAdd(&meta->exited, 1u) == gridDim.x - 1) {
        atomicExch(&meta->next, 0u);
        atomicExch(&meta->exited, 0u);
    }
}

template <int K, int MODE, int COPIES>
__global__ void __launch_bounds__(1024) LDP_BATCH_ATTR batch_kernel(const ldp_image_desc *__restrict__ descs,
                                                     Meta *meta, int32_t gy, int32_t gx,
                                                     int32_t windows, int32_t item_slot,
                                                     MinRows min_rows)
{
    // the item count and table address are the same for every lane:
    // readfirstlane keeps them (and what is read through them) in scalar
    // registers, which the buffer descriptors built from them must be in
    const uint32_t n_items = uniform(meta->n_items);
    const DeviceTables tab{
        (const ConstItem *)(uintptr_t)uniform64(reinterpret_cast<uint64_t>(meta->items)), descs};
    run_queue<K, MODE, COPIES, false>(tab, n_items, meta, gy, gx, windows, item_slot, min_rows);
}

// The same kernel with one copy of the histograms and non-temporal code and
// histogram stores (window plans whose windows are small: their output is
// mostly histograms).
template <int K, int MODE>
__global__ void __launch_bounds__(1024) LDP_BATCH_ATTR batch_kernel_nt(const ldp_image_desc *__restrict__ descs,
                                                        Meta *meta, int32_t gy, int32_t gx,
                                                        int32_t windows, int32_t item_slot,
                                                        MinRows min_rows)
{
    const uint32_t n_items = uniform(meta->n_items);
    const DeviceTables tab{
        (const ConstItem *)(uintptr_t)uniform64(reinterpret_cast<uint64_t>(meta->items)), descs};
    run_queue<K, MODE, 1, true>(tab, n_items, meta, gy, gx, windows, item_slot, min_rows);
}

// The same pass over a batch given in the arguments; only the queue counter
// is read from device memory.
template <int K, int MODE, int COPIES>
__global__ void __launch_bounds__(1024) LDP_BATCH_ATTR batch_arg_kernel(const ArgBatch b, Meta *meta,
                                                         int32_t gy, int32_t gx,
                                                         int32_t windows, int32_t item_slot,
                                                         MinRows min_rows)
{
    run_queue<K, MODE, COPIES, false>(ArgTables{&b}, b.n_items, meta, gy, gx, windows, item_slot,
                                      min_rows);
}

typedef void (*batch_arg_fn)(const ArgBatch, Meta *, int32_t, int32_t, int32_t, int32_t, MinRows);

template <int COPIES>
static batch_arg_fn batch_arg_kernel_for_copies(int k)
{
    switch (k) {
    case 1: return batch_arg_kernel<1, RANK_SIGNED, COPIES>;
    case 2: return batch_arg_kernel<2, RANK_SIGNED, COPIES>;
    case 3: return batch_arg_kernel<3, RANK_SIGNED, COPIES>;
    case 4: return batch_arg_kernel<4, RANK_SIGNED, COPIES>;
    case 5: return batch_arg_kernel<5, RANK_SIGNED, COPIES>;
    case 6: return batch_arg_kernel<6, RANK_SIGNED, COPIES>;
    case 7: return batch_arg_kernel<7, RANK_SIGNED, COPIES>;
    case 8: return batch_arg_kernel<8, RANK_SIGNED, COPIES>;
    }
    return nullptr;
}

static batch_arg_fn batch_arg_kernel_for(int k, int copies = 1)
{
    return copies == 2 ? batch_arg_kernel_for_copies<2>(k) : batch_arg_kernel_for_copies<1>(k);
}

typedef void (*batch_fn)(const ldp_image_desc *, Meta *, int32_t, int32_t, int32_t, int32_t,
                         MinRows);

template <int MODE, int COPIES>
static batch_fn batch_kernel_for_mode(int k)
{
    switch (k) {
    case 1: return batch_kernel<1, MODE, COPIES>;
    case 2: return batch_kernel<2, MODE, COPIES>;
    case 3: return batch_kernel<3, MODE, COPIES>;
    case 4: return batch_kernel<4, MODE, COPIES>;
    case 5: return batch_kernel<5, MODE, COPIES>;
    case 6: return batch_kernel<6, MODE, COPIES>;
    case 7: return batch_kernel<7, MODE, COPIES>;
    case 8: return batch_kernel<8, MODE, COPIES>;
    }
    return nullptr;
}

template <int COPIES>
static batch_fn batch_kernel_for_copies(int k, int mode)
{
    switch (mode) {
    case RANK_MAGNITUDE: return batch_kernel_for_mode<RANK_MAGNITUDE, COPIES>(k);
    case DIRECT_MASKS: return batch_kernel_for_mode<DIRECT_MASKS, COPIES>(k);
    case CODE_LBP: return batch_kernel<1, CODE_LBP, COPIES>;  // LBP codes do not depend on k
    }
    return batch_kernel_for_mode<RANK_SIGNED, COPIES>(k);
}

// The batch kernel for k, the ranking mode and one or two LDS copies of the
// histograms (a template argument: each kernel holds one form, whose
// registers and schedule are not shared with the other).
static batch_fn batch_kernel_for(int k, int mode, int copies = 1)
{
    return copies == 2 ? batch_kernel_for_copies<2>(k, mode) : batch_kernel_for_copies<1>(k, mode);
}

template <int MODE>
static batch_fn batch_kernel_nt_for_mode(int k)
{
    switch (k) {
    case 1: return batch_kernel_nt<1, MODE>;
    case 2: return batch_kernel_nt<2, MODE>;
    case 3: return batch_kernel_nt<3, MODE>;
    case 4: return batch_kernel_nt<4, MODE>;
    case 5: return batch_kernel_nt<5, MODE>;
    case 6: return batch_kernel_nt<6, MODE>;
    case 7: return batch_kernel_nt<7, MODE>;
    case 8: return batch_kernel_nt<8, MODE>;
    }
    return nullptr;
}

// The non-temporal-store batch kernel for k and the ranking mode.
static batch_fn batch_kernel_nt_for(int k, int mode)
{
    switch (mode) {
    case RANK_MAGNITUDE: return batch_kernel_nt_for_mode<RANK_MAGNITUDE>(k);
    case DIRECT_MASKS: return batch_kernel_nt_for_mode<DIRECT_MASKS>(k);
    case CODE_LBP: return batch_kernel_nt<1, CODE_LBP>;
    }
    return batch_kernel_nt_for_mode<RANK_SIGNED>(k);
}

}  // namespace ldp

struct ldp_batch_plan {
    int32_t k = 3, flags = 0, max_images = 0;
    int32_t gy = 1, gx = 1;  // cells_y, cells_x, or window sides when `windows`
    int32_t max_width = LDP_MAX_SIDE;  // widest image a window plan takes
    bool windows = false;
    int32_t nx_max = 1;      // most cells of a cell row in one work item (LDS sizing), <= 63
    int64_t max_pixels = 0, max_items = 0;
    int32_t threads = 256, grid = 0;
    int32_t n_classes = 1;
    ldp_size_class classes[LDP_MAX_SIZE_CLASSES] = {{INT64_MAX, 1, 8}};
    ldp::MinRows min_rows{};   // classes[c].rows_per_task, as the kernels take them
    size_t lds_bytes = 0;
    int32_t copies = 1;     // copies of the histograms in LDS (fused_item)
    bool store_nt = false;  // non-temporal code and histogram stores
    int device = 0;
    // One device block and its pinned staging mirror, laid out as
    // [meta | descriptors | work items], so that a batch uploads in one copy.
    // A window plan whose batch needs more items than the block holds moves
    // its item table to allocations of its own (the kernel reads the table's
    // address from the meta words).
    char *d_block = nullptr, *h_block = nullptr;
    size_t descs_off = 0, items_off = 0;
    bool items_in_block = true;
    ldp_image_desc *d_descs = nullptr;
    ldp::Item *d_items = nullptr;
    ldp::Meta *d_meta = nullptr;
    ldp_image_desc *h_descs = nullptr;  // pinned staging
    ldp::Item *h_items = nullptr;       // pinned staging
    ldp::Meta *h_meta = nullptr;        // pinned staging
    std::vector<ldp_image_desc> descs;  // the loaded batch
    int64_t n_items = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t uploaded = nullptr;
    // recorded after every launch of the plan (launches on one plan are
    // ordered: they share its queue), so that a table the plan replaces or
    // frees is released only once the last launch that can read it has ended
    hipEvent_t ran = nullptr;
};

namespace {

void release(ldp_batch_plan *p)
{
    if (!p)
        return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->uploaded) (void)hipEventDestroy(p->uploaded);
    if (p->ran) (void)hipEventDestroy(p->ran);
    if (!p->items_in_block) {
        if (p->d_items) (void)hipFree(p->d_items);
        if (p->h_items) (void)hipHostFree(p->h_items);
    }
    if (p->d_block) (void)hipFree(p->d_block);
    if (p->h_block) (void)hipHostFree(p->h_block);
    delete p;
}

}  // namespace

namespace {

// Shared by the cell-grid and window plans; nx_max bounds an image's cell
// columns.  Cell rows wider than 63 cells are cut into runs of near-equal
// length (cell_runs); the plan keeps that run length as nx_max, cuts every
// image's cell rows into runs no longer than it, and sizes an item's LDS for
// nx_max + 1 cells per cell row.
int create_plan(ldp_batch_plan **out, int32_t max_images, int64_t max_pixels, int32_t k,
                int32_t flags, bool windows, int32_t gy, int32_t gx, int32_t nx_max,
                const ldp_tune *tune)
{
    const int32_t runs_max = ldp::cell_runs(nx_max);
    nx_max = (nx_max + runs_max - 1) / runs_max;
    *out = nullptr;
    ldp_batch_plan *p = new (std::nothrow) ldp_batch_plan();
    if (!p)
        return LDP_ERR_NO_MEMORY;
    p->k = k;
    p->flags = flags;
    p->gy = gy;
    p->gx = gx;
    p->windows = windows;
    p->nx_max = nx_max;
    p->max_images = max_images;
    p->max_pixels = max_pixels;
    if (tune) {
        if (tune->block_threads)
            p->threads = tune->block_threads;
        if (tune->grid_blocks)
            p->grid = tune->grid_blocks;
        if (tune->n_classes < 0 || tune->n_classes > LDP_MAX_SIZE_CLASSES) {
            delete p;
            return LDP_ERR_INVALID_ARG;
        }
        if (tune->n_classes > 0) {
            p->n_classes = tune->n_classes;
            for (int c = 0; c < p->n_classes; ++c) {
                ldp_size_class sc = tune->classes[c];
                if (sc.cell_rows_per_item == 0)
                    sc.cell_rows_per_item = 1;
                if (sc.rows_per_task == 0)
                    sc.rows_per_task = 8;
                p->classes[c] = sc;
            }
        }
    }
    // any whole number of waves: the lane tasks of a cell row are spread over
    // the workgroup's threads, whatever their count
    if (p->threads < 64 || p->threads > 1024 || p->threads % 64 != 0 || p->grid < 0) {
        delete p;
        return LDP_ERR_INVALID_ARG;
    }
    // an item's cell rows of histograms must fit in 64 KB of LDS (nx_max <= 63
    // leaves room for at least one), and take at most 32 KB when one row
    // allows it: five 256-thread workgroups per CU (160 KB of LDS), the
    // occupancy the kernel is built for
    const int32_t lds_cpi = std::max<int32_t>(1, (int32_t)(32768u / ldp::hist_row_bytes(nx_max)));
    int32_t max_cpi = 1, min_cpi = windows ? 65535 : gy;
    for (int c = 0; c < p->n_classes; ++c) {
        ldp_size_class &sc = p->classes[c];
        if (sc.cell_rows_per_item < 1 || sc.rows_per_task < 1 || sc.max_pixels < 1) {
            delete p;
            return LDP_ERR_INVALID_ARG;
        }
        sc.cell_rows_per_item = std::min(sc.cell_rows_per_item, lds_cpi);
        if (!windows)
            sc.cell_rows_per_item = std::min(sc.cell_rows_per_item, gy);
        max_cpi = std::max(max_cpi, sc.cell_rows_per_item);
        min_cpi = std::min(min_cpi, sc.cell_rows_per_item);
    }
    p->classes[p->n_classes - 1].max_pixels = INT64_MAX;
    for (int c = 0; c < LDP_MAX_SIZE_CLASSES; ++c)
        p->min_rows.v[c] = p->classes[std::min(c, p->n_classes - 1)].rows_per_task;
    // item table: enough for max_images images of a cell grid; window plans
    // start at 8 items per image and grow when a batch needs more
    p->max_items = (int64_t)max_images *
                   (windows ? 8 : (int64_t)((gy + min_cpi - 1) / min_cpi) * runs_max);
    // LDS: the largest item's cell rows, each with its discard cell, then the
    // item broadcast word (16 bytes keep the allocation aligned)
    const size_t hist_bytes = (size_t)max_cpi * ldp::hist_row_bytes(nx_max);
    p->lds_bytes = hist_bytes + 16;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return LDP_ERR_HIP;
    }
    // Cell-grid plans: two copies of the histograms (even and odd lanes)
    // when that kernel, with the LDS they take, keeps as many workgroups on a
    // CU as the one-copy kernel (registers usually decide that number, and
    // the copies use LDS left over).  Window plans keep one copy (their
    // rows of windows fill the LDS).  The second copy starts 16 words (16
    // banks) past the end of the first: the histograms are a multiple of 64
    // words long, so without the gap an even and an odd lane adding into the
    // same bin would still address one bank.
    ldp::batch_fn fn = ldp::batch_kernel_for(k, ldp::rank_mode(flags), 1);
    if (!windows) {
        ldp::batch_fn fn2 = ldp::batch_kernel_for(k, ldp::rank_mode(flags), 2);
        int occ1 = 0, occ2 = 0;
        const size_t lds2 = 2 * (hist_bytes + 64) + 16;
        if (lds2 <= 65536u &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ1, reinterpret_cast<const void *>(fn),
                                                         p->threads, p->lds_bytes) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ2, reinterpret_cast<const void *>(fn2),
                                                         p->threads, lds2) == hipSuccess &&
            occ2 > 0 && occ2 >= occ1) {
            p->copies = 2;
            p->lds_bytes = lds2;
            fn = fn2;
        }
        (void)hipGetLastError();
    }
    // Window plans of small windows (at most 1024 pixels: a 1 KB histogram
    // for every 1024 code bytes or fewer) store non-temporally: measured on
    // 490x640 frames, 20-px windows 6% and 25-px windows 3% faster, while
    // 50- and 100-px windows, like the cell grid, are not faster that way.
    if (windows && (int64_t)gy * gx <= 1024) {
        fn = ldp::batch_kernel_nt_for(k, ldp::rank_mode(flags));
        p->store_nt = true;
    }
    auto fail = [&](int st) {
        release(p);
        return st;
    };
    auto round256 = [](size_t n) { return (n + 255) & ~(size_t)255; };
    p->descs_off = round256(sizeof(ldp::Meta));
    p->items_off = p->descs_off + round256(sizeof(ldp_image_desc) * (size_t)max_images);
    const size_t block = p->items_off + sizeof(ldp::Item) * (size_t)p->max_items;
    if (hipMalloc(&p->d_block, block) != hipSuccess ||
        hipHostMalloc(&p->h_block, block) != hipSuccess)
        return fail(LDP_ERR_NO_MEMORY);
    p->d_meta = reinterpret_cast<ldp::Meta *>(p->d_block);
    p->d_descs = reinterpret_cast<ldp_image_desc *>(p->d_block + p->descs_off);
    p->d_items = reinterpret_cast<ldp::Item *>(p->d_block + p->items_off);
    p->h_meta = reinterpret_cast<ldp::Meta *>(p->h_block);
    p->h_descs = reinterpret_cast<ldp_image_desc *>(p->h_block + p->descs_off);
    p->h_items = reinterpret_cast<ldp::Item *>(p->h_block + p->items_off);
    if (hipMemset(p->d_meta, 0, sizeof(ldp::Meta)) != hipSuccess)
        return fail(LDP_ERR_HIP);

    if (!p->grid) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn),
                                                         p->threads, p->lds_bytes) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) !=
                hipSuccess)
            return fail(LDP_ERR_HIP);
        p->grid = std::max(1, per_cu) * std::max(1, cus);
    }
    if (hipStreamCreate(&p->cap_stream) != hipSuccess ||
        hipEventCreateWithFlags(&p->uploaded, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ran, hipEventDisableTiming) != hipSuccess)
        return fail(LDP_ERR_HIP);
    // capture: the persistent kernel (it leaves its queue reset for the next
    // launch)
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(LDP_ERR_HIP);
    hipLaunchKernelGGL(fn, dim3(p->grid), dim3(p->threads), p->lds_bytes, p->cap_stream,
                       (const ldp_image_desc *)p->d_descs, p->d_meta, gy, gx, windows ? 1 : 0,
                       (int32_t)((p->lds_bytes - 16) / 4), p->min_rows);
    hipError_t ce = hipStreamEndCapture(p->cap_stream, &p->graph);
    if (ce != hipSuccess || hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) !=
                                hipSuccess)
        return fail(LDP_ERR_HIP);
    *out = p;
    return LDP_OK;
}

bool common_args_ok(ldp_batch_plan **out, int32_t max_images, int64_t max_pixels, int32_t k,
                    int32_t flags)
{
    return out && max_images >= 1 && max_images < ldp::kMaxPlanImages && max_pixels >= 9 &&
           k >= 1 && k <= 8 && ldp::flags_ok(flags);
}

}  // namespace

namespace {

// Checks a batch against the plan and cuts it into work items (per image,
// groups of its size class's cell rows), largest first.  Changes nothing.
int cut_items(const ldp_batch_plan *p, const ldp_image_desc *descs, int32_t n,
              std::vector<ldp::Item> &out)
{
    if (n > p->max_images)
        return LDP_ERR_NO_MEMORY;
    int64_t pixels = 0;
    for (int32_t j = 0; j < n; ++j) {
        const ldp_image_desc &d = descs[j];
        int st = ldp::check_image(d.img, d.H, d.W, d.stride);
        if (st != LDP_OK)
            return st;
        if (!d.hist)
            return LDP_ERR_INVALID_ARG;
        if (!p->windows && (d.H - 2 < p->gy || d.W - 2 < p->gx))
            return LDP_ERR_INVALID_ARG;
        if (p->windows && d.W > p->max_width)
            return LDP_ERR_INVALID_ARG;  // wider than the plan's max_width
        pixels += (int64_t)d.H * d.W;
    }
    if (pixels > p->max_pixels)
        return LDP_ERR_NO_MEMORY;
    std::vector<ldp::Item> items;
    std::vector<int64_t> size;
    for (int32_t j = 0; j < n; ++j) {
        const int64_t px = (int64_t)descs[j].H * descs[j].W;
        int c = 0;
        while (c < p->n_classes - 1 && px > p->classes[c].max_pixels)
            ++c;
        const int32_t cpi = p->classes[c].cell_rows_per_item;
        const int32_t Hc = descs[j].H - 2, Wc = descs[j].W - 2;
        const ldp::Geom geo = ldp::make_geom(Hc, Wc, p->gy, p->gx, p->windows);
        // runs of at most the plan's nx_max cells (the LDS of an item)
        const int32_t runs = (geo.nx + p->nx_max - 1) / p->nx_max;
        for (int32_t cy = 0; cy < geo.ny; cy += cpi) {
            const int32_t cy1 = std::min(cy + cpi, geo.ny);
            const int64_t rows =
                ldp::geom_row_start(geo, cy1, Hc) - ldp::geom_row_start(geo, cy, Hc);
            for (int32_t xi = 0; xi < runs; ++xi) {
                const int32_t cx0 = ldp::cell_run_start(geo.nx, runs, xi);
                const int32_t cx1 = ldp::cell_run_start(geo.nx, runs, xi + 1);
                items.push_back({(uint32_t)j | ((uint32_t)c << ldp::kImgBits), (uint16_t)cy,
                                 (uint16_t)cy1, (uint16_t)cx0, (uint16_t)cx1});
                size.push_back(rows * (ldp::geom_col_start(geo, cx1, Wc) -
                                       ldp::geom_col_start(geo, cx0, Wc)));
            }
        }
    }
    if ((int64_t)items.size() > p->max_items && !p->windows)
        return LDP_ERR_NO_MEMORY;
    std::vector<int64_t> order(items.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return size[a] > size[b]; });
    out.resize(items.size());
    for (size_t i = 0; i < order.size(); ++i)
        out[i] = items[order[i]];
    return LDP_OK;
}

}  // namespace

extern "C" {

int ldp_batch_plan_create_ex(ldp_batch_plan **out, int32_t max_images, int64_t max_pixels,
                             int32_t k, int32_t flags, int32_t cells_y, int32_t cells_x,
                             const ldp_tune *tune)
{
    if (!common_args_ok(out, max_images, max_pixels, k, flags) || cells_y < 1 || cells_x < 1 ||
        cells_y > LDP_MAX_SIDE - 2 || cells_x > LDP_MAX_SIDE - 2)
        return LDP_ERR_INVALID_ARG;
    return create_plan(out, max_images, max_pixels, k, flags, false, cells_y, cells_x, cells_x,
                       tune);
}

int ldp_batch_plan_create_windows(ldp_batch_plan **out, int32_t max_images, int64_t max_pixels,
                                  int32_t max_width, int32_t k, int32_t flags, int32_t win_y,
                                  int32_t win_x, const ldp_tune *tune)
{
    if (!common_args_ok(out, max_images, max_pixels, k, flags) || max_width < 3 ||
        max_width > LDP_MAX_SIDE || win_y < 1 || win_x < 1)
        return LDP_ERR_INVALID_ARG;
    const int32_t wc = max_width - 2, wx = std::min(win_x, wc);
    const int32_t nx_max = (wc + wx - 1) / wx;
    ldp_batch_plan *p = nullptr;
    const int st = create_plan(&p, max_images, max_pixels, k, flags, true, win_y, win_x, nx_max,
                               tune);
    if (st == LDP_OK)
        p->max_width = max_width;
    *out = p;
    return st;
}

int ldp_batch_plan_create(ldp_batch_plan **out, int32_t max_images, int64_t max_pixels, int32_t k,
                          int32_t cells_y, int32_t cells_x, const ldp_tune *tune)
{
    return ldp_batch_plan_create_ex(out, max_images, max_pixels, k, 0, cells_y, cells_x, tune);
}

int ldp_batch_plan_set(ldp_batch_plan *p, const ldp_image_desc *descs, int32_t n,
                       ldp_stream_t stream)
{
    if (!p || n < 0 || (n > 0 && !descs))
        return LDP_ERR_INVALID_ARG;
    std::vector<ldp::Item> items;
    int rc = cut_items(p, descs, n, items);
    if (rc != LDP_OK)
        return rc;
    // the staging buffers may still feed the previous upload
    if (hipEventSynchronize(p->uploaded) != hipSuccess)
        return LDP_ERR_HIP;
    p->descs.assign(descs, descs + n);
    if ((int64_t)items.size() > p->max_items) {
        // window plans grow their item table (the graph reads its address
        // from the meta words, so nothing is re-captured)
        const int64_t cap = std::max<int64_t>((int64_t)items.size(), p->max_items * 3 / 2);
        ldp::Item *d = nullptr, *h = nullptr;
        if (hipMalloc(&d, sizeof(ldp::Item) * cap) != hipSuccess)
            return LDP_ERR_NO_MEMORY;
        if (hipHostMalloc(&h, sizeof(ldp::Item) * cap) != hipSuccess) {
            (void)hipFree(d);
            return LDP_ERR_NO_MEMORY;
        }
        // the old table may still feed a launch in flight: wait for the
        // plan's last launch (not the whole device)
        if (hipEventSynchronize(p->ran) != hipSuccess) {
            (void)hipFree(d);
            (void)hipHostFree(h);
            return LDP_ERR_HIP;
        }
        if (!p->items_in_block) {
            (void)hipFree(p->d_items);
            (void)hipHostFree(p->h_items);
        }
        p->items_in_block = false;
        p->d_items = d;
        p->h_items = h;
        p->max_items = cap;
    }
    std::copy(items.begin(), items.end(), p->h_items);
    std::copy(descs, descs + n, p->h_descs);
    p->n_items = (int64_t)items.size();
    p->h_meta->n_items = (uint32_t)p->n_items;
    p->h_meta->next = 0;
    p->h_meta->exited = 0;
    p->h_meta->items = p->d_items;
    hipStream_t s = (hipStream_t)stream;
    // meta and descriptors (and the items while they are in the block) in
    // one copy
    const size_t head = p->items_in_block
                            ? p->items_off + sizeof(ldp::Item) * (size_t)p->n_items
                            : p->descs_off + sizeof(ldp_image_desc) * (size_t)n;
    if (hipMemcpyAsync(p->d_block, p->h_block, head, hipMemcpyHostToDevice, s) != hipSuccess ||
        (!p->items_in_block && p->n_items > 0 &&
         hipMemcpyAsync(p->d_items, p->h_items, sizeof(ldp::Item) * p->n_items,
                        hipMemcpyHostToDevice, s) != hipSuccess) ||
        hipEventRecord(p->uploaded, s) != hipSuccess)
        return LDP_ERR_HIP;
    return LDP_OK;
}

int ldp_batch_launch(ldp_batch_plan *p, const ldp_image_desc *descs, int32_t n,
                     ldp_stream_t stream)
{
    return ldp::run_batch(p, descs, n, (hipStream_t)stream);
}

int ldp_batch_run(ldp_batch_plan *p, ldp_stream_t stream)
{
    if (!p)
        return LDP_ERR_INVALID_ARG;
    if (p->n_items == 0)
        return LDP_OK;
    return hipGraphLaunch(p->exec, (hipStream_t)stream) == hipSuccess &&
                   hipEventRecord(p->ran, (hipStream_t)stream) == hipSuccess
               ? LDP_OK
               : LDP_ERR_HIP;
}

int ldp_batch_run_per_image(ldp_batch_plan *p, ldp_stream_t stream)
{
    if (!p)
        return LDP_ERR_INVALID_ARG;
    for (const ldp_image_desc &d : p->descs) {
        int st = ldp::launch_extract(d.img, d.H, d.W, d.stride, p->k, p->flags, p->gy, p->gx,
                                     p->windows, d.codes, d.hist, (hipStream_t)stream);
        if (st != LDP_OK)
            return st;
    }
    return hipEventRecord(p->ran, (hipStream_t)stream) == hipSuccess ? LDP_OK : LDP_ERR_HIP;
}

int ldp_batch_plan_info(const ldp_batch_plan *p, int64_t *work_items, int32_t *grid_blocks)
{
    if (!p)
        return LDP_ERR_INVALID_ARG;
    if (work_items)
        *work_items = p->n_items;
    if (grid_blocks)
        *grid_blocks = p->grid;
    return LDP_OK;
}

int ldp_batch_plan_layout(const ldp_batch_plan *p, int32_t *threads, int32_t *lds_bytes,
                          int32_t *hist_copies, int32_t *nt_stores)
{
    if (!p)
        return LDP_ERR_INVALID_ARG;
    if (threads)
        *threads = p->threads;
    if (lds_bytes)
        *lds_bytes = (int32_t)p->lds_bytes;
    if (hist_copies)
        *hist_copies = p->copies;
    if (nt_stores)
        *nt_stores = p->store_nt ? 1 : 0;
    return LDP_OK;
}

int ldp_batch_plan_destroy(ldp_batch_plan *p)
{
    if (!p)
        return LDP_ERR_INVALID_ARG;
    // the plan's last launch and last upload (other streams run on)
    if (p->ran)
        (void)hipEventSynchronize(p->ran);
    if (p->uploaded)
        (void)hipEventSynchronize(p->uploaded);
    release(p);
    return LDP_OK;
}

}  // extern "C"

namespace ldp {
namespace {

// The plan's kernel for batches in the launch arguments (nullptr when its
// batches always go through the loaded tables: windows, or flags).
batch_arg_fn arg_kernel(const ldp_batch_plan *p)
{
    return !p->windows && rank_mode(p->flags) == RANK_SIGNED ? batch_arg_kernel_for(p->k, p->copies)
                                                             : nullptr;
}

int launch_args(const ldp_batch_plan *p, batch_arg_fn fn, ArgBatch &b, hipStream_t s)
{
    // no more workgroups than items (at least one); the queue counter is zero
    // between launches on this plan (each launch resets it)
    const int32_t grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>(p->grid, b.n_items));
    Meta *meta = p->d_meta;
    int32_t gy = p->gy, gx = p->gx, windows = 0;
    int32_t item_slot = (int32_t)((p->lds_bytes - 16) / 4);
    MinRows min_rows = p->min_rows;
    void *args[] = {&b, &meta, &gy, &gx, &windows, &item_slot, &min_rows};
    return hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3(grid), dim3(p->threads), args,
                           p->lds_bytes, s) == hipSuccess &&
                   hipEventRecord(p->ran, s) == hipSuccess
               ? LDP_OK
               : LDP_ERR_HIP;
}

}  // namespace

int warm_plan(ldp_batch_plan *p, hipStream_t s)
{
    int rc = ldp_batch_plan_set(p, nullptr, 0, (ldp_stream_t)s);
    if (rc != LDP_OK)
        return rc;
    if (hipGraphLaunch(p->exec, s) != hipSuccess)
        return LDP_ERR_HIP;
    // the argument-table kernel too: one workgroup that finds no work item
    const batch_arg_fn fn = arg_kernel(p);
    if (!fn)
        return LDP_OK;
    ArgBatch b{};
    return launch_args(p, fn, b, s);
}

int run_batch(ldp_batch_plan *p, const ldp_image_desc *descs, int32_t n, hipStream_t s)
{
    if (!p || n < 0 || (n > 0 && !descs))
        return LDP_ERR_INVALID_ARG;
    const batch_arg_fn fn = n <= kArgImages ? arg_kernel(p) : nullptr;
    if (fn) {
        std::vector<Item> items;
        int rc = cut_items(p, descs, n, items);
        if (rc != LDP_OK)
            return rc;
        if (items.empty())
            return LDP_OK;
        if ((int64_t)items.size() <= kArgItems) {
            ArgBatch b{};
            b.n_items = (uint32_t)items.size();
            std::copy(descs, descs + n, b.descs);
            std::copy(items.begin(), items.end(), b.items);
            return launch_args(p, fn, b, s);
        }
    }
    int rc = ldp_batch_plan_set(p, descs, n, (ldp_stream_t)s);
    return rc == LDP_OK ? ldp_batch_run(p, (ldp_stream_t)s) : rc;
}
}  // namespace ldp

// ---------------------------------------------------------------- no allocation
// ldp_batch_launch_noalloc: the argument-table launch of ldp_batch_launch with
// its work-queue words in a file-scope device array instead of a plan's
// allocation.  Each device holds its own copy of the array until the process
// ends; the host reaches it through the address hipGetSymbolAddress returns
// with that device current (the array's name is not a device address in host
// code), taken once per device and kept.
namespace ldp {
namespace {

constexpr int kScratchBytes = 256;  // the queue words (Meta), padded
static_assert(sizeof(Meta) <= kScratchBytes, "queue words fit the scratch array");
constexpr int kMaxDevices = 64;
// Launch shape for these small batches (as the server's): one cell row per
// work item, lane tasks of >= 4 rows, 1024-thread workgroups.
constexpr int kNoallocThreads = 1024;
constexpr int32_t kNoallocTaskRows = 4;

__global__ void clear_words_kernel(uint32_t *p, int32_t n)
{
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x)
        p[i] = 0u;
}

std::mutex g_scratch_mu;
Meta *g_scratch[kMaxDevices] = {};

}  // namespace
}  // namespace ldp

static __device__ __align__(256) unsigned char scratch[ldp::kScratchBytes];

namespace ldp {
namespace {

// The device address of this device's scratch array; on the first call for a
// device its words are cleared by a kernel on `s` (ahead of any launch the
// caller then makes on `s`).
int scratch_for(int dev, hipStream_t s, Meta **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return LDP_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return LDP_ERR_HIP;
        hipLaunchKernelGGL(clear_words_kernel, dim3(1), dim3(64), 0, s,
                           reinterpret_cast<uint32_t *>(ptr), kScratchBytes / 4);
        if (hipGetLastError() != hipSuccess)
            return LDP_ERR_HIP;
        g_scratch[dev] = reinterpret_cast<Meta *>(ptr);
    }
    *out = g_scratch[dev];
    return LDP_OK;
}

// Work items of a batch for the argument table, in fixed-size storage (no
// heap): one cell row per item, each cell row cut into runs of at most 63
// cells, largest first.  Errors as ldp_batch_launch, and LDP_ERR_UNSUPPORTED
// past LDP_ARG_BATCH_IMAGES images or LDP_ARG_BATCH_ITEMS items.
int cut_items_fixed(const ldp_image_desc *descs, int32_t n, int32_t gy, int32_t gx, ArgBatch &b,
                    int32_t &run_cells)
{
    if (n > kArgImages)
        return LDP_ERR_UNSUPPORTED;
    const int32_t runs = cell_runs(gx);
    run_cells = (gx + runs - 1) / runs;
    int64_t size[kArgItems];
    int32_t m = 0;
    for (int32_t j = 0; j < n; ++j) {
        const ldp_image_desc &d = descs[j];
        const int st = check_image(d.img, d.H, d.W, d.stride);
        if (st != LDP_OK)
            return st;
        if (!d.hist || d.H - 2 < gy || d.W - 2 < gx)
            return LDP_ERR_INVALID_ARG;
    }
    for (int32_t j = 0; j < n; ++j) {
        const ldp_image_desc &d = descs[j];
        const int32_t Hc = d.H - 2, Wc = d.W - 2;
        const Geom geo = make_geom(Hc, Wc, gy, gx, false);
        for (int32_t cy = 0; cy < geo.ny; ++cy) {
            const int64_t rows = geom_row_start(geo, cy + 1, Hc) - geom_row_start(geo, cy, Hc);
            for (int32_t xi = 0; xi < runs; ++xi) {
                if (m == kArgItems)
                    return LDP_ERR_UNSUPPORTED;
                const int32_t cx0 = cell_run_start(geo.nx, runs, xi);
                const int32_t cx1 = cell_run_start(geo.nx, runs, xi + 1);
                const Item it{(uint32_t)j, (uint16_t)cy, (uint16_t)(cy + 1), (uint16_t)cx0,
                              (uint16_t)cx1};
                const int64_t sz = rows * (geom_col_start(geo, cx1, Wc) -
                                           geom_col_start(geo, cx0, Wc));
                // insertion, largest first (stable)
                int32_t at = m;
                while (at > 0 && size[at - 1] < sz) {
                    b.items[at] = b.items[at - 1];
                    size[at] = size[at - 1];
                    --at;
                }
                b.items[at] = it;
                size[at] = sz;
                ++m;
            }
        }
    }
    b.n_items = (uint32_t)m;
    for (int32_t j = 0; j < n; ++j)
        b.descs[j] = descs[j];
    return LDP_OK;
}

}  // namespace
}  // namespace ldp

extern "C" int ldp_batch_launch_noalloc(const ldp_image_desc *descs, int32_t n, int32_t k,
                                        int32_t cells_y, int32_t cells_x, ldp_stream_t stream)
{
    using namespace ldp;
    if (n < 0 || (n > 0 && !descs) || k < 1 || k > 8 || cells_y < 1 || cells_x < 1 ||
        cells_y > LDP_MAX_SIDE - 2 || cells_x > LDP_MAX_SIDE - 2)
        return LDP_ERR_INVALID_ARG;
    ArgBatch b{};
    int32_t run_cells = 1;
    int rc = cut_items_fixed(descs, n, cells_y, cells_x, b, run_cells);
    if (rc != LDP_OK)
        return rc;
    if (b.n_items == 0)
        return LDP_OK;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return LDP_ERR_HIP;
    Meta *meta = nullptr;
    rc = scratch_for(dev, s, &meta);
    if (rc != LDP_OK)
        return rc;
    // one cell row of histograms per item, then the item broadcast word
    const size_t hist_bytes = hist_row_bytes(run_cells);
    const size_t lds_bytes = hist_bytes + 16;
    int32_t gy = cells_y, gx = cells_x, windows = 0;
    int32_t item_slot = (int32_t)(hist_bytes / 4);
    MinRows min_rows{{kNoallocTaskRows, kNoallocTaskRows, kNoallocTaskRows, kNoallocTaskRows}};
    void *args[] = {&b, &meta, &gy, &gx, &windows, &item_slot, &min_rows};
    // no more workgroups than items: each takes items until the queue is
    // empty, and the last one out leaves the queue words at zero
    const batch_arg_fn fn = batch_arg_kernel_for(k);
    return hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3(b.n_items),
                           dim3(kNoallocThreads), args, lds_bytes, s) == hipSuccess
               ? LDP_OK
               : LDP_ERR_HIP;
}
