/*
 * ccl.h -- C ABI of the gfx950 (MI355X) two-pass connected component
 * labeling library, after Gupta et al., "A New Parallel Algorithm for
 * Two-Pass Connected Component Labeling" (arXiv 1606.05973).
 *
 * Problem (Section III): a binary image of H x W pixels; every object
 * (foreground) pixel receives a label so that connected object pixels share a
 * label.  Foreground here means a nonzero byte.  Connectivity is 8 (the only
 * one the paper uses) or 4.
 *
 * Output numbering: 0 for background; the components are numbered 1..K in
 * the order of their smallest raster index r*W + c (the first pixel of each
 * component met in a row-major scan).  This is the numbering the paper's
 * sequential CCLRemSP (Algorithm 1) produces; it does not depend on tiling
 * or on scheduling, so results are bit-exact and reproducible.
 *
 * The work runs on a caller-provided HIP stream and is asynchronous: a call
 * returns after launching; results are valid once the stream (or an event
 * recorded after the call) has completed.  All pointers named "device" must
 * be device memory of the current HIP device.
 *
 * Errors: argument errors are detected on the host before anything is
 * launched and returned as a negative ccl_status; nothing is written then.
 * CCL_ERR_HIP reports a failed HIP runtime call or launch.
 */
#ifndef CCL_H_
#define CCL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *hipStream_t;

typedef enum {
    CCL_OK = 0,
    CCL_ERR_NULL = -1,      /* a required pointer is NULL                      */
    CCL_ERR_SHAPE = -2,     /* H <= 0 or W <= 0                                 */
    CCL_ERR_STRIDE = -3,    /* stride < W                                       */
    CCL_ERR_CONN = -4,      /* conn is neither 4 nor 8                          */
    CCL_ERR_TOO_LARGE = -5, /* H*W >= 2^31 - 1 or a side >= 2^31 - 256 (int32 labels and keys), or an
                               image so elongated that tiles x boundary slots per tile reaches 2^31
                               (32-bit union-find ids; e.g. one row of 2^30 pixels) */
    CCL_ERR_NOMEM = -6,     /* the workspace could not be allocated             */
    CCL_ERR_HIP = -7,       /* a HIP runtime call or kernel launch failed       */
    CCL_ERR_TILE = -8,      /* unknown tile configuration id                    */
    CCL_ERR_CAPTURE = -9,   /* workspace must grow while the stream is captured */
    CCL_ERR_BATCH = -10,    /* n < 0, or descs NULL with n > 0                  */
    CCL_ERR_LEVEL = -11,    /* threshold level outside 0..255                   */
    CCL_ERR_SCAN = -12,     /* unknown scan strategy                            */
    CCL_ERR_BUDGET = -13,   /* request needs more workspace than a server slot  */
    CCL_ERR_TICKET = -14,   /* unknown server ticket                            */
    CCL_ERR_GRAY = -15,     /* gray flag other than 0 or 1                      */
    CCL_ERR_ORDER = -16,    /* unknown output order                             */
    CCL_ERR_SCRATCH = -17   /* image needs more than ccl_label_noalloc's static scratch */
} ccl_status;

/*
 * Tile-local scan strategy (the comparison of Table II, redone inside a
 * tile).  Nodes of the tile-local union-find are runs of foreground pixels:
 *   CCL_SCAN_PAIR  runs of the OR of two image rows (8-connectivity only):
 *                  the two-row scan mask of ARemSP (Fig. 1b, Algorithm 6),
 *                  which visits two rows per step; under 8-connectivity any
 *                  two horizontally adjacent columns of a row pair that both
 *                  hold foreground are connected, so such a run is one piece.
 *                  The default; under 4-connectivity it means CCL_SCAN_ROW.
 *   CCL_SCAN_ROW   runs of single rows, the one-row scan of CCLRemSP
 *                  (Algorithm 4's mask); diagonal contacts are unions.
 * Both give the same labels.
 */
typedef enum { CCL_SCAN_PAIR = 0, CCL_SCAN_ROW = 1 } ccl_scan;

/*
 * Output numbering.
 *   CCL_ORDER_CANONICAL    components numbered 1..K by their smallest raster
 *                          index (the default; independent of tiling).
 *   CCL_ORDER_PROVISIONAL  the flatten's numbering (Algorithm 3, Section III):
 *                          1..K in the order of each set's smallest
 *                          provisional label, the provisional labels being
 *                          the tile-local components in (tile in raster
 *                          order, component in the tile's node order) order,
 *                          as PARemSP (Algorithm 7) numbers each thread's
 *                          labels after those of the threads before it.  The
 *                          partition into components is the same; only the
 *                          numbers differ, and they depend on the tile shape.
 *                          Skips the tile-local canonical keys and the
 *                          per-row rank scan.
 */
typedef enum { CCL_ORDER_CANONICAL = 0, CCL_ORDER_PROVISIONAL = 1 } ccl_order;

/*
 * ccl_label -- label one image (the whole two-pass method of Section III/IV:
 * tile-local scan with RemSP unions, parallel RemSP merge across tile
 * boundaries, flatten, canonical ranking, labeling pass).
 *
 *   img     device, H rows of W bytes, row pitch `stride` bytes (>= W);
 *           nonzero = foreground.  Read only.  Any alignment is accepted;
 *           16-byte aligned rows take the fast load path.
 *   H, W    image size in pixels, H*W < 2^31 - 1 and H, W < 2^31 - 256.
 *   stride  row pitch of img in bytes.
 *   conn    4 or 8.
 *   labels  device, dense H x W int32, row pitch W elements.  Written
 *           completely and only after every read of img, so it must not
 *           overlap img.  16-byte alignment and W % 4 == 0 take the fast
 *           store path.
 *   stream  HIP stream (NULL = default stream).
 *
 * Ownership: the caller owns img and labels.  The library owns a cached
 * workspace per (device, stream), grown on demand (see ccl_reserve).
 * Calls on different streams use different workspaces and may overlap;
 * calls on one stream are serialised by the stream.
 */
int ccl_label(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn,
              int32_t *labels, hipStream_t stream);

/* One image of ccl_label_batch; fields as for ccl_label. */
typedef struct {
    const uint8_t *img;      /* device */
    int64_t H, W, stride;
    int conn;                /* 4 or 8, may differ between images */
    int32_t *labels;         /* device, dense H x W */
    int32_t *num_components; /* device int32 receiving K, or NULL */
} ccl_image_desc;

/*
 * ccl_label_batch -- label n independent images of any sizes with one
 * launch per phase for the whole batch (tiles of all images share each
 * grid; images that take different tile-local scans, 8- and 4-connectivity,
 * form separate launch groups).
 *   descs   host array of n descriptors (read during the call only).
 *   n       number of images (0 is a no-op returning CCL_OK).
 * Every descriptor is validated first; the first invalid one makes the call
 * return its error with nothing launched (CCL_ERR_BATCH for n < 0 or descs
 * NULL with n > 0).  No host synchronisation.  The call may be captured
 * into a HIP graph in any capture mode (after ccl_reserve of
 * ccl_workspace_bytes / ccl_batch_workspace_bytes on that stream): with
 * n > 1 the image table then travels in the arguments of small store kernels
 * that the graph records, so every replay writes it again before the
 * labeling kernels.  A graph captured from any call of this library uses the
 * stream's workspace: it must not be replayed after that workspace was grown
 * by a later, larger call on the same stream or freed by ccl_release, nor
 * while other work on that workspace (eager calls on the same stream excepted,
 * which the stream orders) is in flight.
 */
int ccl_label_batch(const ccl_image_desc *descs, int n, hipStream_t stream);

/* Workspace bytes one ccl_label call needs for an H x W image (0 for
 * invalid arguments).  Used for admission by HBM footprint: footprint =
 * image + labels + workspace. */
size_t ccl_workspace_bytes(int64_t H, int64_t W, int conn);

/*
 * ccl_reserve -- grow the workspace of (current device, stream) to at least
 * `bytes` now, synchronising the stream if it has to reallocate.  Call it
 * before capturing a stream into a HIP graph: inside capture the workspace
 * cannot grow and a call that needs more returns CCL_ERR_CAPTURE.
 */
int ccl_reserve(size_t bytes, hipStream_t stream);

/* Static description of a status code. */
const char *ccl_strerror(int status);

/* ------------------------------------------------------------------------
 * Extended calls: the calls above with the options of the extensions (fused
 * threshold, gray-level labeling, tile-local scan strategy, tile shape).
 * ------------------------------------------------------------------------ */

/*
 * ccl_label_ex -- as ccl_label, plus
 *   num_components  device int32 receiving K, or NULL.
 *   tile            tile configuration id from ccl_tile_config (0 = the default
 *                   for the image's kind, ccl_tile_default).
 */
int ccl_label_ex(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn,
                 int32_t *labels, int32_t *num_components, int tile, hipStream_t stream);

/*
 * ccl_label_level -- as ccl_label_ex, on a grayscale image binarized inside
 * the labeling: a pixel is foreground iff its byte is greater than `level`
 * (0..255).  This is the binarization step that precedes labeling in the
 * paper's experiments (Section V: each image is converted to binary with a
 * luminance threshold of 0.5); fused into the image read, it costs no extra
 * memory traffic.  A fractional threshold f of the full range (a pixel v is
 * foreground iff v > f * 255) is level = floor(f * 255), so f = 0.5 is
 * level 127.  level 0 is the nonzero test of ccl_label; level 255 makes
 * every pixel background.  Returns CCL_ERR_LEVEL for a level outside 0..255.
 */
int ccl_label_level(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int level, int conn,
                    int32_t *labels, int32_t *num_components, int tile, hipStream_t stream);

/*
 * ccl_label_gray -- gray-level labeling, the extension Section V mentions
 * (the abstract: adjacent pixels sharing the same features get the same
 * label): object pixels are the bytes greater than `level` (0 = nonzero), and
 * two neighbouring object pixels (4- or 8-neighbours) are connected when
 * their bytes are equal.  On a 0/1 image this is ccl_label.  Numbering as
 * for ccl_label (components ranked by smallest raster index).  The tile-local
 * nodes are single-row runs of equal bytes.  Arguments and errors as for
 * ccl_label_level.
 */
int ccl_label_gray(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int level, int conn,
                   int32_t *labels, int32_t *num_components, int tile, hipStream_t stream);

/*
 * ccl_label_provisional -- as ccl_label_ex, numbering the components in
 * provisional order (CCL_ORDER_PROVISIONAL): consecutive labels 1..K, as the
 * paper's flatten hands them out.  K is the same as with ccl_label, and
 * renumbering the output by smallest raster index gives ccl_label's output.
 */
int ccl_label_provisional(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn,
                          int32_t *labels, int32_t *num_components, int tile, hipStream_t stream);

/*
 * ccl_label_noalloc -- ccl_label_ex (default tile) for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It calls no hipMalloc, hipFree or other
 * allocating routine and records no profiling events.  Its workspace is a
 * static device array of CCL_NOALLOC_SCRATCH_BYTES that every device the
 * library runs on holds until the process ends (looked up on the call's
 * first use of a device).
 *   img, H, W, stride, conn, labels, num_components, stream
 *           as for ccl_label_ex (caller-owned device memory; num_components
 *           may be NULL).
 * Limit: images whose ccl_workspace_bytes(H, W, conn) exceeds
 * CCL_NOALLOC_SCRATCH_BYTES return CCL_ERR_SCRATCH with nothing launched
 * (4096 x 4096 fits at both connectivities).  Other argument errors as for
 * ccl_label.  All calls on one device share the one array and it keeps the
 * last call's contents: calls that overlap on one device (different streams
 * without ordering between them) race and give undefined labels; calls on
 * one stream are ordered by the stream.  The output is the same as
 * ccl_label's.
 */
#define CCL_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
int ccl_label_noalloc(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn,
                      int32_t *labels, int32_t *num_components, hipStream_t stream);

/* One image of an extended batch.  The first seven fields are those of
 * ccl_image_desc; the options are as in ccl_label_level / ccl_label_gray /
 * ccl_label_provisional.  All-zero options give ccl_label's labeling. */
typedef struct {
    const uint8_t *img;      /* device */
    int64_t H, W, stride;
    int conn;                /* 4 or 8, may differ between images */
    int32_t *labels;         /* device, dense H x W */
    int32_t *num_components; /* device or NULL */
    int level;               /* foreground iff byte > level; 0 = nonzero */
    int scan;                /* ccl_scan; 0 = CCL_SCAN_PAIR */
    int gray;                /* 1: gray-level labeling (see ccl_label_gray; scan is ignored) */
    int order;               /* ccl_order; 0 = CCL_ORDER_CANONICAL */
    int tile;                /* tile configuration id for this image; 0 = the call's tile */
} ccl_image_desc_ex;

/*
 * ccl_label_batch_ex -- ccl_label_batch over extended descriptors, with
 *   tile    tile configuration id for the images whose descriptor names
 *           none (0 = each image's kind takes its default, ccl_tile_default).
 * Images are launched in groups of the same kind (row pairs, single rows,
 * gray levels), output order and tile configuration: one launch per phase
 * per group.  Errors, capture and workspace as for ccl_label_batch, plus
 * CCL_ERR_TILE / CCL_ERR_ORDER for a descriptor's tile or order.
 */
int ccl_label_batch_ex(const ccl_image_desc_ex *descs, int n, int tile, hipStream_t stream);

/*
 * Captured batches.  ccl_batch_graph_create labels nothing: it gives the
 * batch its own workspace and device descriptor table (uploaded before
 * capture), captures every launch of ccl_label_batch_ex for these
 * descriptors into a HIP graph and instantiates it.  ccl_graph_launch
 * replays the whole batch on `stream` with one graph launch; the image and
 * label buffers named in the descriptors are the ones used on every replay
 * (refill the images between replays to label new content of the same
 * shapes).  The graph holds kernel nodes only.  ccl_graph_destroy
 * synchronises the device and frees the graph and its workspace.  Errors as
 * for ccl_label_batch_ex, plus CCL_ERR_NOMEM if the graph's workspace cannot
 * be allocated.
 */
typedef struct ccl_graph ccl_graph;
int ccl_batch_graph_create(const ccl_image_desc_ex *descs, int n, int tile, ccl_graph **graph);
int ccl_graph_launch(ccl_graph *graph, hipStream_t stream);
int ccl_graph_destroy(ccl_graph *graph);

/* Workspace bytes for a ccl_label_batch_ex call (0 for invalid arguments);
 * with tile 0 and default options it is what ccl_label_batch needs. */
size_t ccl_batch_workspace_bytes(const ccl_image_desc_ex *descs, int n, int tile);

/* Free every cached workspace of the current device (synchronises the
 * device first). */
int ccl_release(void);

/* Tile configuration `id` (1-based) -> block rows and tile width in
 * pixels.  A tile is `block rows` x 2 image rows under 8-connectivity with
 * the row-pair scan (two rows at a time), `block rows` x 1 with single rows
 * (4-connectivity, CCL_SCAN_ROW), and `block rows` / 2 x 1 for gray levels
 * (where every pixel may be its own run).  Returns CCL_OK, or CCL_ERR_TILE
 * when id is out of range; id 0 reports configuration 1.  ccl_tile_count()
 * gives the number of configurations. */
int ccl_tile_config(int id, int *block_rows, int *tile_w);
int ccl_tile_count(void);

/* The configuration id that tile id 0 selects for an image of this kind
 * (each kind of a batch takes its own): row pairs (conn 8, CCL_SCAN_PAIR),
 * single rows (conn 4 or CCL_SCAN_ROW) and gray levels (gray = 1; the scan
 * is then ignored) have separate defaults.  0 for invalid arguments. */
int ccl_tile_default(int conn, int scan, int gray);

/*
 * Phase timing.  ccl_profile(1) makes every later call record a HIP event on
 * its stream before each of its CCL_NUM_PHASES kernels and after the last;
 * ccl_profile_read waits for the recorded events and writes the summed
 * milliseconds of each phase over all calls since the previous read into
 * ms[0..nphase) (phases: tile scan, boundary merge, flatten, scan blocks,
 * scan totals, component labels, labeling pass), and the number of calls into
 * *ncalls (may be NULL).  Used by the benchmark to time single kernels on
 * the stream they run on.
 */
#define CCL_NUM_PHASES 7
int ccl_profile(int enable);
int ccl_profile_read(double *ms, int nphase, int *ncalls);

/*
 * Continuous-batching server.  Labeling requests (one image each, described
 * as for ccl_label_batch_ex) arrive at any time from any thread.  A scheduler
 * thread inside the library keeps up to n_streams batches in flight, each on
 * its own HIP stream with its own workspace of hbm_budget / n_streams bytes:
 * whenever a stream's batch has completed, the requests waiting at that
 * moment (in arrival order, up to max_batch images, max_batch_pixels pixels
 * and the slot's workspace) are launched together as one batch, so requests
 * that arrive while others are on the GPU join the next batch and batches on
 * different streams overlap on the device.  Admission is by HBM footprint:
 * a request is admitted into a batch only if its workspace region fits the
 * free slot's workspace; one that could never fit is refused at submission
 * with CCL_ERR_BUDGET.  Each result equals that of ccl_label_batch on the
 * image alone (labels do not depend on batching).
 *
 * The workspaces are allocated once, at creation, on the current device;
 * the images and label buffers belong to the caller and must stay valid
 * until their request has completed.
 */
typedef struct ccl_server ccl_server;

typedef struct {
    int n_streams;              /* batches in flight at once, >= 1 */
    int max_batch;              /* images per batch, >= 1 */
    int64_t max_batch_pixels;   /* pixels per batch (a larger single image still runs alone) */
    size_t hbm_budget;          /* device bytes of all slot workspaces together */
    int tile;                   /* tile configuration id (0 = per-kind default) */
} ccl_server_config;

typedef struct {
    int64_t submitted, completed, rejected, batches, in_flight_max;
    double pixels_completed;
    double p50_ms, p99_ms, mean_ms;  /* submission-to-completion latency of completed requests */
} ccl_server_stats;

/* Create a server on the current device (CCL_ERR_BATCH for a config value
 * out of range, CCL_ERR_NOMEM if the workspaces cannot be allocated). */
int ccl_server_create(const ccl_server_config *cfg, ccl_server **out);

/* Queue one request.  `ready`: a stream whose work so far must finish before
 * the image is read and the labels written (e.g. the stream that produced
 * the image), or NULL if the buffers are ready now.  *ticket identifies the
 * request (> 0).  Argument errors as for ccl_label_batch_ex; CCL_ERR_BUDGET if
 * the image can never fit a slot. */
int ccl_server_submit(ccl_server *s, const ccl_image_desc_ex *d, hipStream_t ready, uint64_t *ticket);

/* 1 if the request has completed (*latency_ms, if not NULL, gets its
 * submission-to-completion time), 0 if not yet, CCL_ERR_TICKET if unknown. */
int ccl_server_poll(ccl_server *s, uint64_t ticket, double *latency_ms);

/* Block until the request has completed; returns CCL_OK or the first
 * failure the scheduler met. */
int ccl_server_wait(ccl_server *s, uint64_t ticket, double *latency_ms);

/* Block until every submitted request has completed. */
int ccl_server_drain(ccl_server *s);

/* Counters and latency percentiles since creation. */
int ccl_server_stats_get(ccl_server *s, ccl_server_stats *out);

/* Finish all queued requests, stop the scheduler and free the server. */
int ccl_server_destroy(ccl_server *s);

#ifdef __cplusplus
}
#endif

#endif /* CCL_H_ */
