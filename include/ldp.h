/*
 * ldp.h -- C ABI of the MI355X (gfx950) Local Directional Pattern library.
 *
 * Method: "An Acceleration Scheme to The Local Directional Pattern"
 * (Ayami and Shabat, arXiv 1810.11518).  For every interior pixel of an
 * 8-bit grayscale image the library computes the eight Kirsch directional
 * responses (Section 2.2.1, Eq. 1) through shared neighbour sums (the
 * redundancy-omitting scheme of Section 2.3, Eqs. 7-29), selects the k-th
 * largest response and forms the 8-bit LDP code (Section 2.2.2, Eqs. 2-3),
 * and counts codes in per-cell histograms (Section 2.2.3, Eqs. 4-5).
 *
 * Conventions (fixed by the library; see the design notes):
 *   - x is the row, y the column; M0..M7 are the Kirsch compass masks
 *     East, North-East, North, North-West, West, South-West, South,
 *     South-East, applied as a correlation (Eq. 1);
 *   - responses are signed; m_k is the k-th element of the eight responses
 *     in descending order with duplicates kept; bit i of the code is set when
 *     m_i >= m_k (Eq. 3), so ties can set more than k bits;
 *   - only interior pixels (1 <= x <= H-2, 1 <= y <= W-2) get a code; the
 *     code map is dense, (H-2) rows of (W-2) bytes:
 *         codes[(x-1)*(W-2) + (y-1)];
 *   - histograms have 256 uint32 bins per cell, indexed by the raw code, for a
 *     cells_y x cells_x grid laid over the code map with a floor partition
 *     (code row r is in cell row r*cells_y/(H-2), code column c in cell column
 *     c*cells_x/(W-2)); layout hist[(cy*cells_x + cx)*256 + code]; every call
 *     overwrites the whole histogram array.
 *
 * Memory: every pointer argument except the descriptor arrays of the batch
 * calls is DEVICE memory owned by the caller; the library never frees it.
 * Images may have any alignment and any row pitch ("stride", bytes, >= W).
 *
 * Streams and errors: calls enqueue work on `stream` (0 = the null stream)
 * and return at once.  Argument errors are detected on the host before
 * anything is launched and return LDP_ERR_INVALID_ARG; a failed launch
 * returns LDP_ERR_HIP.  Faults during execution surface at the caller's next
 * synchronisation of the stream.  Nothing is thrown across this boundary.
 * Calls on different streams may run concurrently; the kernels keep no state.
 */
#ifndef LDP_H
#define LDP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *ldp_stream_t; /* the same type as hipStream_t */

enum {
    LDP_OK = 0,
    LDP_ERR_INVALID_ARG = -1,
    LDP_ERR_HIP = -2,
    LDP_ERR_NO_MEMORY = -3,
    LDP_ERR_UNSUPPORTED = -4,
    LDP_ERR_BUSY = -5
};

/* Largest image side the kernels accept (rows and columns). */
#define LDP_MAX_SIDE 65536

/* Human-readable text for a status code (static storage). */
const char *ldp_status_string(int status);

/* Library ABI version, currently 1. */
int ldp_version(void);

/*
 * ldp_codes -- LDP code of every interior pixel (Eqs. 1-3).
 *   img     device, H rows of W bytes, row pitch `stride` bytes (>= W).
 *   H, W    image rows and columns, 3 <= H, W <= LDP_MAX_SIDE.
 *   k       number of most outstanding responses, 1..8 (the paper uses 3).
 *   codes   device, (H-2)*(W-2) bytes, written densely as described above.
 * Errors: LDP_ERR_INVALID_ARG for a null pointer, H or W out of range,
 * stride < W or k outside 1..8.
 */
int ldp_codes(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
              uint8_t *codes, ldp_stream_t stream);

/*
 * ldp_histograms -- per-cell 256-bin histograms of a code map (Eqs. 4-5).
 *   codes   device, the dense (H-2)x(W-2) code map of an H x W image.
 *   H, W    the IMAGE dimensions (3..LDP_MAX_SIDE).
 *   cells_y, cells_x  grid, 1 <= cells_y <= H-2, 1 <= cells_x <= W-2.
 *   hist    device, cells_y*cells_x*256 uint32, overwritten.
 * Errors: LDP_ERR_INVALID_ARG for a null pointer or sizes out of range.
 */
int ldp_histograms(const uint8_t *codes, int32_t H, int32_t W, int32_t cells_y,
                   int32_t cells_x, uint32_t *hist, ldp_stream_t stream);

/*
 * ldp_extract -- codes and histograms of one image in a single launch
 * (Eqs. 1-5): the same results as ldp_codes followed by ldp_histograms,
 * without reading the code map back.  Arguments as above; `codes` may be
 * NULL when only the histograms are wanted.
 */
int ldp_extract(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                int32_t cells_y, int32_t cells_x, uint8_t *codes, uint32_t *hist,
                ldp_stream_t stream);

/* ---------------------------------------------------------------- variants
 *
 * The _ex calls take `flags`: 0 or exactly one of
 *   LDP_RANK_MAGNITUDE  rank the responses by absolute value: Eqs. 2-3
 *                       applied to |m_0|, ..., |m_7| (the convention of the
 *                       original LDP descriptor that Section 2.2 builds on;
 *                       the paper's Eq. 2 ranks signed responses, flags 0).
 *   LDP_DIRECT_MASKS    the codes of flags 0, with every response computed
 *                       as Eq. 1's 8-tap mask correlation (multiply-adds, no
 *                       shared sums): the unaccelerated LDP computation that
 *                       Section 2.3's scheme is measured against.
 *   LDP_CODE_LBP        Local Binary Pattern labels (Section 2.1) instead of
 *                       LDP codes: bit i is set when the neighbour in compass
 *                       direction i (E, NE, N, NW, W, SW, S, SE) is >= the
 *                       centre pixel; same code map and histogram layout; k
 *                       must be valid (1..8) and is ignored.
 * Anything else: LDP_ERR_INVALID_ARG.  Flags 0 is exactly the call without
 * _ex.
 */
#define LDP_RANK_MAGNITUDE 1
#define LDP_DIRECT_MASKS 2
#define LDP_CODE_LBP 4
#define LDP_FLAGS_ALL 7

/* ldp_codes with flags. */
int ldp_codes_ex(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                 int32_t flags, uint8_t *codes, ldp_stream_t stream);

/* ldp_extract with flags. */
int ldp_extract_ex(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                   int32_t flags, int32_t cells_y, int32_t cells_x, uint8_t *codes,
                   uint32_t *hist, ldp_stream_t stream);

/*
 * Eq. 6's compact feature vector.  Eq. 4 counts the pixels whose code equals
 * the i-th pattern value C_i; the pattern values are the C(8, k) codes with
 * exactly k bits set (56 for k = 3), taken in ascending order.  A compact
 * histogram is (H_1, ..., H_C(8,k)) followed by one bin that counts every
 * other code (a tie with m_k sets more than k bits), so its bins sum to the
 * cell's pixel count.
 *
 * ldp_compact_bins -- C(8, k) + 1 for k in 1..8, else LDP_ERR_INVALID_ARG.
 *
 * ldp_compact_histograms -- compact vectors of n_cells cells.
 *   hist    device, n_cells * 256 uint32 (raw-code histograms, e.g. from
 *           ldp_extract: cell c at hist[c*256]).
 *   n_cells >= 0 (0: nothing is launched).
 *   k       1..8, the k the codes were made with.
 *   out     device, n_cells * ldp_compact_bins(k) uint32, cell c at
 *           out[c * ldp_compact_bins(k)], overwritten; must not overlap hist.
 * Errors: LDP_ERR_INVALID_ARG for k outside 1..8, n_cells < 0 or a null
 * pointer with n_cells > 0.
 */
int32_t ldp_compact_bins(int32_t k);
int ldp_compact_histograms(const uint32_t *hist, int64_t n_cells, int32_t k, uint32_t *out,
                           ldp_stream_t stream);

/* ---------------------------------------------------------------- windows
 *
 * Histograms per window instead of per grid cell (Section 3.2 extracts
 * features over windows of 10x10 .. 100x100 pixels): non-overlapping windows
 * of win_y x win_x code pixels tile the code map from its first row and
 * column; the last row and column of windows are cut at the map's edge
 * (ny = ceil((H-2)/win_y), nx = ceil((W-2)/win_x) windows; a 280x280 image
 * with 10x10 windows has 28 x 28 = 784, as Table 3 lists).  Window (wy, wx)
 * is at hist[(wy*nx + wx)*256 + code]; win_y, win_x >= 1 (sides larger than
 * the map count as the map).
 */

/* ldp_window_grid -- ny and nx for an H x W image (either pointer may be
 * NULL).  Errors: LDP_ERR_INVALID_ARG for sizes out of range. */
int ldp_window_grid(int32_t H, int32_t W, int32_t win_y, int32_t win_x, int32_t *ny, int32_t *nx);

/* ldp_histograms_windows -- ldp_histograms with windows; hist has
 * ny*nx*256 uint32, overwritten. */
int ldp_histograms_windows(const uint8_t *codes, int32_t H, int32_t W, int32_t win_y,
                           int32_t win_x, uint32_t *hist, ldp_stream_t stream);

/* ldp_extract_windows -- ldp_extract_ex with windows (one launch; `codes` may
 * be NULL for any window grid). */
int ldp_extract_windows(const uint8_t *img, int32_t H, int32_t W, int64_t stride, int32_t k,
                        int32_t flags, int32_t win_y, int32_t win_x, uint8_t *codes,
                        uint32_t *hist, ldp_stream_t stream);

/* ---------------------------------------------------------------- batches
 *
 * Many images of any sizes in ONE persistent launch: the work (row bands of
 * every image, split so that histogram cells are owned by one workgroup) is
 * laid out in a device table, workgroups pull work items from a device queue,
 * and the launch is captured once in a HIP graph and replayed.  Each image's
 * codes and histograms are exactly those of ldp_extract on that image.
 */
typedef struct ldp_image_desc {
    const uint8_t *img; /* device, H x W, pitch `stride` */
    uint8_t *codes;     /* device, (H-2)*(W-2) bytes, or NULL for histograms only */
    uint32_t *hist;     /* device, cells_y*cells_x*256 uint32 */
    int64_t stride;     /* bytes between rows, >= W */
    int32_t H, W;       /* 3..LDP_MAX_SIDE */
} ldp_image_desc;

/* Launch shape and work split of the batched kernel, chosen by the autotuner
 * (paper_1810_11518_amd/autotune.py); zero fields take defaults.  Images are
 * put in the first size class whose max_pixels >= H*W (the last class takes
 * the rest); a class fixes how many cell rows of an image one work item
 * covers and how many code rows one lane task covers at least. */
#define LDP_MAX_SIZE_CLASSES 4
typedef struct ldp_size_class {
    int64_t max_pixels;         /* upper bound of H*W for the class */
    int32_t cell_rows_per_item; /* cell rows of one image per work item, >= 1; lowered so
                                   that an item's histograms ((c + 1) KiB per cell row in LDS,
                                   c = the cells of a row one item covers: all of them, or a
                                   run of at most 63 when a row has more) take at most 32 KiB,
                                   or one cell row */
    int32_t rows_per_task;      /* target code rows per lane task, >= 1 */
} ldp_size_class;

typedef struct ldp_tune {
    int32_t block_threads; /* threads per workgroup: a multiple of 64, 64..1024 (default 256) */
    int32_t grid_blocks;   /* persistent workgroups; 0 = fill the device */
    int32_t n_classes;     /* 0 (one default class) .. LDP_MAX_SIZE_CLASSES */
    int32_t reserved;
    ldp_size_class classes[LDP_MAX_SIZE_CLASSES];
} ldp_tune;

typedef struct ldp_batch_plan ldp_batch_plan;

/*
 * ldp_batch_plan_create -- a plan for up to max_images images and up to
 * max_pixels total pixels, for fixed k and cell grid.  Allocates the plan's
 * device work table and queue (owned by the plan, released by destroy).
 * `tune` may be NULL.  Errors: LDP_ERR_INVALID_ARG, LDP_ERR_NO_MEMORY.
 */
int ldp_batch_plan_create(ldp_batch_plan **plan, int32_t max_images, int64_t max_pixels,
                          int32_t k, int32_t cells_y, int32_t cells_x, const ldp_tune *tune);

/* ldp_batch_plan_create with flags (as for ldp_extract_ex); the plan's runs
 * give each image ldp_extract_ex's results with these flags. */
int ldp_batch_plan_create_ex(ldp_batch_plan **plan, int32_t max_images, int64_t max_pixels,
                             int32_t k, int32_t flags, int32_t cells_y, int32_t cells_x,
                             const ldp_tune *tune);

/* A plan whose runs give each image ldp_extract_windows' results (every
 * image's hist holds its own ny*nx*256 bins).  Images may be at most
 * max_width columns wide (wider ones: LDP_ERR_INVALID_ARG from set).  A row
 * of more than 63 windows is split over several work items.  The plan's
 * device work table grows when a batch needs more work items. */
int ldp_batch_plan_create_windows(ldp_batch_plan **plan, int32_t max_images, int64_t max_pixels,
                                  int32_t max_width, int32_t k, int32_t flags, int32_t win_y,
                                  int32_t win_x, const ldp_tune *tune);

/*
 * ldp_batch_plan_set -- (re)load the batch: `descs` is a HOST array of n
 * descriptors (copied; the caller may reuse it on return).  Builds the work
 * table on the host and uploads it on `stream`.  The captured graph is
 * reused when only the descriptors change.  Every image must satisfy the
 * ldp_extract argument rules and have at least cells_y+2 rows and cells_x+2
 * columns.  Errors: LDP_ERR_INVALID_ARG (the offending image is not
 * launched; nothing is), LDP_ERR_NO_MEMORY if n or the pixel total exceed
 * the plan's capacity.
 */
int ldp_batch_plan_set(ldp_batch_plan *plan, const ldp_image_desc *descs, int32_t n,
                       ldp_stream_t stream);

/* ldp_batch_run -- run the loaded batch on `stream` (one graph launch). */
int ldp_batch_run(ldp_batch_plan *plan, ldp_stream_t stream);

/*
 * ldp_batch_launch -- load and run a batch in one call: the results of
 * ldp_batch_plan_set followed by ldp_batch_run, with the same checks and
 * errors.  On a plan with cells (not windows) and flags 0, a batch of at most
 * LDP_ARG_BATCH_IMAGES images and LDP_ARG_BATCH_ITEMS work items (see
 * ldp_batch_plan_info) travels in the kernel launch's own arguments: no table
 * upload and no graph launch, and the plan's loaded batch (what
 * ldp_batch_run runs) stays as it was.  Any other batch is loaded with
 * ldp_batch_plan_set (it becomes the loaded batch) and run.  Launches on one
 * plan share its work queue: order them (one stream, or events across
 * streams), as for ldp_batch_run.
 */
#define LDP_ARG_BATCH_IMAGES 28
#define LDP_ARG_BATCH_ITEMS 196
int ldp_batch_launch(ldp_batch_plan *plan, const ldp_image_desc *descs, int32_t n,
                     ldp_stream_t stream);

/*
 * ldp_batch_launch_noalloc -- for callers that cannot allocate memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Runs a small batch like ldp_batch_launch on a plan for cells
 * (flags 0): each image gets ldp_extract's codes (when `codes` is not NULL)
 * and cells_y x cells_x histograms for k.  No plan: the batch travels in the
 * kernel's arguments and the work-queue words live in a fixed 256-byte device
 * array of the library, one per GPU, kept until the process ends.  The call
 * allocates nothing, host or device (the first call on a GPU also clears that
 * GPU's array with a small kernel on `stream`).  Limits: at most
 * LDP_ARG_BATCH_IMAGES images and LDP_ARG_BATCH_ITEMS work items (one item
 * per cell row, per run of at most 63 cells of it); larger batches return
 * LDP_ERR_UNSUPPORTED and launch nothing.  Every call on one GPU shares its
 * queue words: calls that overlap on one GPU (different streams without
 * ordering) race and give wrong results; order them.  Other errors as
 * ldp_batch_launch (LDP_ERR_INVALID_ARG for a bad image, k or grid).
 */
int ldp_batch_launch_noalloc(const ldp_image_desc *descs, int32_t n, int32_t k, int32_t cells_y,
                             int32_t cells_x, ldp_stream_t stream);

/* ldp_batch_run_per_image -- the same batch as one ldp_extract launch per
 * image, for comparison with the persistent launch. */
int ldp_batch_run_per_image(ldp_batch_plan *plan, ldp_stream_t stream);

/* ldp_batch_plan_info -- work items and persistent workgroups of the loaded
 * batch (either pointer may be NULL). */
int ldp_batch_plan_info(const ldp_batch_plan *plan, int64_t *work_items, int32_t *grid_blocks);

/* ldp_batch_plan_layout -- the plan's launch shape, chosen at creation:
 * threads per workgroup, LDS bytes per workgroup, the copies (1 or 2) of an
 * item's histograms in that LDS (two when the kernel keeps as many workgroups
 * per CU with them), and 1 when its code and histogram stores are
 * non-temporal (window plans of windows of at most 1024 pixels), else 0.
 * Any pointer may be NULL. */
int ldp_batch_plan_layout(const ldp_batch_plan *plan, int32_t *threads, int32_t *lds_bytes,
                          int32_t *hist_copies, int32_t *nt_stores);

/* ldp_batch_plan_destroy -- release the plan (waits for the plan's last
 * launch and last upload, not for other work on the device). */
int ldp_batch_plan_destroy(ldp_batch_plan *plan);

/* ---------------------------------------------------------------- serving
 *
 * Continuous batching of single-image requests.  A request (a HOST image and
 * HOST result buffers) is admitted when the server's memory pool has room for
 * its image, codes and histograms (the buffers the GPU cannot address in
 * place) and a request slot is free; otherwise it waits, in arrival order.
 * The pool has a page-locked host mirror of the same size (made at creation
 * for pools up to 256 MiB, at the first request that needs it above): a
 * dispatcher thread packs each admitted pageable image into the request's
 * mirror region and launches the admitted requests as one persistent batch
 * (ldp_batch_launch: a small batch's tables travel in the launch arguments,
 * a larger one's are uploaded; the work queue lives on the device) on one
 * of `depth` streams; the kernel reads the images there and writes codes
 * and histograms there, over the bus, and the dispatcher copies them to the
 * caller's buffers once the batch has finished.  Requests that arrive while
 * earlier batches run are admitted as memory frees up and their work
 * overlaps on the device.  When a batch's results are on the host its
 * memory and slots are released.  Without the mirror (its allocation
 * failed) the device pool holds the requests and images and results are
 * copied in and out on the batch's stream.  Results are exactly those of
 * ldp_extract on the image alone.
 */
typedef struct ldp_server ldp_server;

typedef struct ldp_server_config {
    int64_t pool_bytes;    /* pool for images + codes + histograms (device
                            * memory and a page-locked host mirror of it) */
    int32_t max_inflight;  /* requests admitted at once (slots) */
    int32_t max_batch;     /* requests per launch */
    int32_t depth;         /* launches in flight at once (streams), 1..8 */
    int32_t k;             /* 1..8 */
    int32_t cells_y, cells_x;
    int32_t dry_run;       /* 1: no device work at all (policy tests on a CPU):
                            * admission and batching run, batches "complete"
                            * dry_run_us microseconds after launch, outputs are
                            * not written */
    int32_t dry_run_us;
    int32_t flags;         /* 0, or LDP_SERVER_NO_MIRROR: no page-locked mirror;
                            * buffers the GPU cannot address in place go
                            * through the device pool with copies in and out
                            * (the path taken when the mirror cannot be
                            * allocated) */
} ldp_server_config;

#define LDP_SERVER_NO_MIRROR 1

/* Completion record of a request; times are ldp_now() seconds. */
typedef struct ldp_completion {
    int64_t id;
    double t_submit;  /* when ldp_server_submit accepted it */
    double t_admit;   /* when it got device memory and a slot */
    double t_done;    /* when its results were in the caller's buffers */
    int32_t status;   /* LDP_OK or the error of its batch */
    int32_t batch_size;
} ldp_completion;

typedef struct ldp_server_stats {
    int64_t submitted, completed, rejected, launches;
    int64_t memory_waits;     /* requests that reached the head of the queue and
                               * waited there for pool memory */
    int64_t peak_pool_bytes;  /* most pool bytes in use at once */
    int32_t peak_inflight;    /* most requests admitted at once */
    int32_t peak_batches;     /* most launches in flight at once */
    int32_t max_batch_seen;
    int32_t waiting;          /* requests waiting for admission now */
} ldp_server_stats;

/* Monotonic clock (seconds) used for every server timestamp. */
double ldp_now(void);

/* Create a server (allocates the pool and, up to 256 MiB, its page-locked
 * mirror, streams and batch plans; starts the dispatcher thread).  Without dry_run it also launches every slot's batch
 * kernels (graph and argument-table forms) once on an empty batch and runs
 * one small copy of each kind on the slot's stream, synchronously, so that
 * one-time runtime set-up does not fall on the first requests (a few
 * milliseconds at creation).  Errors:
 * LDP_ERR_INVALID_ARG, LDP_ERR_NO_MEMORY, LDP_ERR_HIP. */
int ldp_server_create(ldp_server **server, const ldp_server_config *config);

/* Queue one request.  img is HOST memory, H x W with pitch `stride`; codes
 * ((H-2)*(W-2) bytes, may be NULL) and hist (cells_y*cells_x*256 uint32) are
 * HOST outputs written before the request completes.  All three buffers must
 * stay valid until completion; page-locked img and hist buffers that the GPU
 * addresses at their host addresses are read and written by the kernel in
 * place (no pool space, no host copy), other buffers go through the pool's
 * mirror (one host copy each way).  Returns the
 * request id in *id.  Errors: LDP_ERR_INVALID_ARG (bad sizes),
 * LDP_ERR_NO_MEMORY (the request can never fit the pool: rejected). */
int ldp_server_submit(ldp_server *server, const uint8_t *img, int32_t H, int32_t W,
                      int64_t stride, uint8_t *codes, uint32_t *hist, int64_t *id);

/* Completed requests since the last poll (up to max), waiting up to
 * wait_us microseconds for at least one.  *n receives the count. */
int ldp_server_poll(ldp_server *server, ldp_completion *out, int32_t max, int32_t *n,
                    int32_t wait_us);

int ldp_server_stats_get(ldp_server *server, ldp_server_stats *stats);

/* Stop the dispatcher after the queued requests complete, release all. */
int ldp_server_destroy(ldp_server *server);

/* ---------------------------------------------------------------- measurement
 *
 * ldp_stream_copy -- copies `bytes` bytes from src to dst (device memory,
 * both 16-byte aligned, not overlapping) with a plain streaming kernel that
 * reads and writes every byte once.  Not part of the method: it is the
 * measuring stick for the LDP kernels (the device-memory rate a kernel that
 * touches each byte once reaches, and a kernel of known traffic for scaling
 * hardware byte counters).  Errors: LDP_ERR_INVALID_ARG for bytes < 0, a null
 * or misaligned pointer with bytes > 0; LDP_ERR_HIP for a failed launch.
 */
int ldp_stream_copy(const void *src, void *dst, int64_t bytes, ldp_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LDP_H */
