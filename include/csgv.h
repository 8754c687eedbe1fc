/*
 * csgv.h -- C ABI of the MI355X (gfx950) CSGV brick decoder.
 *
 * The paper's decode stage decompresses every newly requested brick of a
 * compressed segmentation volume, in parallel, into the brick-cache slots the
 * assign stage handed out, at the level of detail (LOD) each brick was
 * requested at (Methods > "GPU rendering pipeline": request, provision,
 * assign, decode; Methods > "Memory management": a brick shrinks 8x per LOD).
 * The compressed volume -- brick records plus the "Brick Starts" offset table
 * -- stays resident in GPU memory (Methods > "Memory management", encoding
 * buffer optimizations).  This library is that decode stage, plus the host-side
 * CPU encoder that produces the compressed volume (Methods > "Compressed
 * segmentation volumes": compression runs on the CPU, parallel over bricks).
 *
 * Conventions
 *  - Pointers named d_* are device memory, h_* host memory.  The caller owns
 *    every buffer; the library never frees or retains caller memory.
 *  - Entry points taking a hipStream_t enqueue work and return; the work runs
 *    in stream order.  Inputs must stay alive until that work completes.
 *  - Argument errors are reported synchronously as CSGV_EINVAL before anything
 *    is enqueued; HIP failures as CSGV_EHIP.  csgv_last_error() describes the
 *    most recent failure of the calling thread.  No C++ exception crosses the ABI.
 *  - Per-task failures are reported in d_status (see the CSGV_TASK_* words),
 *    never as a return code: a damaged record cannot fault or hang the decoder.
 *
 * Volume container (little-endian; the byte-level format is this library's
 * own -- the paper describes the encoding only in outline):
 *   header (128 B): magic 'CSGV', version 1, dims[3], default log2(brick side),
 *   label_bytes (4 or 8), encoder op mask, n_bricks, brick grid[3], rANS
 *   frequency table u16[16] (sum 4096), offsets position, directory position,
 *   total bytes, neighbour mode.
 *   offsets: n_bricks + 1 u64 byte offsets of the brick records from the
 *   container start ("Brick Starts"; 64-bit, so no 16 GiB limit and no split
 *   buffers are needed); the last entry is the end of the final record.
 *   directory (optional): per brick u32 origin x, y, z and log2(brick side).
 *   brick records, each 8-byte aligned:
 *     u8 coder (0 plain 4-bit, 1 rANS), u8 log2(side), u8 label_bytes,
 *     u8 log2(rANS lanes); u32 palette count; u32 sym_end[log2(side) + 1]
 *     (symbols consumed after each level); rANS only: u32 word count of each
 *     64-lane group, u32 state of each lane; the palette; the payload (plain:
 *     two 4-bit symbols per byte, low nibble first; rANS: u16 words, group by
 *     group).  A symbol is op | stop << 3 with op 0 PARENT, 1..3 NEIGHBOR_X/Y/Z,
 *     4 PALETTE_ADV, 5 PALETTE_LAST, 6 PALETTE_DELTA (followed by its 4-bit
 *     delta entries), 7 invalid.
 */
#ifndef CSGV_H
#define CSGV_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CSGV_OK = 0,
    CSGV_EINVAL = -1,   /* bad argument; nothing was enqueued */
    CSGV_ECORRUPT = -2, /* csgv_check_status: at least one task failed */
    CSGV_ENOMEM = -3,   /* device or host allocation failed */
    CSGV_EHIP = -4      /* a HIP runtime call failed */
} csgv_status;

/* Per-task status words written to d_status. */
enum {
    CSGV_TASK_OK = 0,
    /* brick id >= n_bricks, LOD > log2(brick side), or the task's output range
       does not fit the output buffer: the output is left untouched */
    CSGV_TASK_INVALID = 1,
    /* the brick record or its operation stream is malformed: PARENT on the
       root, a neighbour outside the brick, PALETTE_ADV past the palette,
       PALETTE_LAST with no palette entry read yet, a delta of 0 or beyond the
       entries read, operation 7, a level whose operations do not end exactly
       at its sym_end, rANS words exhausted, or (at full resolution) a palette
       count different from the PALETTE_ADV count; also a record whose offsets,
       side, label width, coder or sizes do not fit.  The task's output range
       is zero-filled when it is valid, otherwise left untouched */
    CSGV_TASK_CORRUPT = 2
};

/* Decoder forms. */
enum {
    CSGV_MODE_PLAIN = 0,      /* one kernel launch per task (a single work-group each) */
    CSGV_MODE_PERSISTENT = 2  /* one launch of resident work-groups popping tasks from a device queue */
};

/* Host-side view of a container header (csgv_volume_parse). */
typedef struct {
    uint32_t dims[3];
    uint32_t log2b;        /* default brick side (bricks may override per record) */
    uint32_t label_bytes;  /* 4 or 8 */
    uint32_t op_mask;      /* operations the encoder could use (the decoder accepts all) */
    uint32_t n_bricks;
    uint32_t grid[3];      /* brick grid; 0 when irregular */
    uint16_t rans_freq[16];
    uint64_t offsets_pos;  /* byte position of the offset table */
    uint64_t dir_pos;      /* byte position of the brick directory, 0 if none */
    uint64_t total_bytes;  /* container size */
    uint32_t neighbor_mode;
    uint32_t max_log2b;    /* largest log2(brick side) any record claims (sizes decoder scratch) */
    uint32_t max_palette;  /* largest palette count of any record (|P|max of cache paletting) */
} csgv_volume_info;

/* Launch shape.  Zero (or -1 for sort_tasks) selects the default. */
typedef struct {
    int mode;            /* CSGV_MODE_* (plans are always PERSISTENT)                      */
    int wg_size;         /* work-group size 128, 256, 512 or 1024; default 256              */
    int wgs_per_cu;      /* persistent form: work-groups per compute unit; default = as many
                            as LDS and wave slots allow                                     */
    int sort_tasks;      /* persistent form: pop tasks in decreasing estimated cost
                            (record bytes + output bytes, by powers of two); default 1      */
    int bricks_per_wave; /* tasks a wavefront takes at a time; only 1 is implemented        */
    int lds_slots;       /* LDS split: 16-bit slots per work-group for the explicit nodes of
                            level 5 (bricks needing more use global scratch); the area also
                            holds the rANS table, so 8192..32760; default 10240             */
    int palette_bits;    /* 0: labels (default).  I in 1..31: cache-paletted output, see
                            CSGV_PALETTED_WORDS                                             */
} csgv_decode_opts;

/*
 * Cache-paletted output (Methods > Memory management > Cache paletting):
 * with palette_bits = I a task writes, instead of its S^3 labels, their
 * indices into the brick's palette (the index the operation stream assigns:
 * the label's position in the palette), I bits each, floor(32 / I) per 32-bit
 * word: voxel k of the cube (x fastest) sits in word k / e at bit
 * (k mod e) * I, e = floor(32 / I), unused high bits zero.  d_out is then
 * 32-bit words and d_out_offsets / out_capacity count words; a task occupies
 * CSGV_PALETTED_WORDS(S^3, I) words.  I = max(1, ceil(log2(max_palette)))
 * fits every brick of a volume.  A task whose record has more than 2^I
 * palette entries, or that asks for a 64^3 cube, is CSGV_TASK_INVALID
 * (output untouched).
 */
#define CSGV_PALETTED_WORDS(voxels, bits) (((voxels) + 32u / (bits) - 1u) / (32u / (bits)))

/*
 * Parse and validate a container held in host memory (the "Brick Starts"
 * table and records of Methods > "Memory management").  `bytes` is the size
 * of h_container and must cover the whole container (total_bytes): the
 * offset table must lie inside it, and max_log2b is read from the records.
 * Returns CSGV_OK or CSGV_EINVAL.  The device copy handed to the decode calls
 * must hold the same total_bytes bytes.
 */
csgv_status csgv_volume_parse(const void* h_container, uint64_t bytes, csgv_volume_info* out);

/*
 * Decode a batch of bricks: the decode stage of Methods > "GPU rendering
 * pipeline" (bricks decoded in parallel into cache slots) at per-task LOD
 * (Methods > "Memory management").
 *   vol            header of the container, from csgv_volume_parse.
 *   d_container    the whole container in device memory (vol->total_bytes).
 *   d_brick_ids    n tasks: brick id of each task.
 *   d_lods         n tasks: LOD, 0 = full resolution; LOD k yields a cube of
 *                  side (brick side >> k) whose voxels are the mode-of-8
 *                  multi-resolution labels of that level.
 *   d_out_offsets  n tasks: element offset of each task's output in d_out, or
 *                  NULL: tasks are packed back to back in task order (a task
 *                  whose brick id, record or LOD is unusable occupies nothing).
 *   n              number of tasks (0 is allowed and enqueues nothing).
 *   d_out          labels of vol->label_bytes each; task j writes its cube,
 *                  linear with x fastest, at d_out + offset of task j.
 *   out_capacity   number of label elements available in d_out.
 *   d_status       n task status words (CSGV_TASK_*), or NULL.
 *   opts           NULL for defaults (plain form).
 * Output ranges of different tasks must not overlap.  Device scratch is
 * allocated and freed stream-ordered inside the call.  Returns CSGV_OK,
 * CSGV_EINVAL, CSGV_ENOMEM or CSGV_EHIP.
 */
csgv_status csgv_decode_bricks(hipStream_t stream, const csgv_volume_info* vol, const void* d_container,
                               const uint32_t* d_brick_ids, const uint8_t* d_lods, const uint64_t* d_out_offsets,
                               uint32_t n, void* d_out, uint64_t out_capacity, uint32_t* d_status,
                               const csgv_decode_opts* opts);

/*
 * csgv_decode_bricks without allocating anything, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, outputs and errors, and
 * nothing is allocated or freed: the scratch is a fixed device array of
 * CSGV_NOALLOC_SCRATCH_BYTES inside the library, one per GPU it runs on, held
 * until the process ends (its device address is looked up on the first call
 * on each device).  Limits: at most CSGV_NOALLOC_MAX_TASKS tasks per call
 * (else CSGV_EINVAL), and the persistent grid holds only as many work-groups
 * as the array's scratch share fits (about 250 for 32^3 bricks, 75 for 64^3),
 * so large batches run slower than with csgv_decode_bricks.  Every call on a
 * GPU uses that GPU's one array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.  The array keeps
 * the last call's contents; each call resets what it needs with kernels.
 */
#define CSGV_NOALLOC_SCRATCH_BYTES (128ull << 20)
#define CSGV_NOALLOC_MAX_TASKS 262144u
csgv_status csgv_decode_bricks_noalloc(hipStream_t stream, const csgv_volume_info* vol, const void* d_container,
                                       const uint32_t* d_brick_ids, const uint8_t* d_lods,
                                       const uint64_t* d_out_offsets, uint32_t n, void* d_out, uint64_t out_capacity,
                                       uint32_t* d_status, const csgv_decode_opts* opts);

/*
 * Synchronise `stream` and report whether any of the n status words is
 * nonzero: CSGV_OK when all tasks succeeded, CSGV_ECORRUPT otherwise.
 */
csgv_status csgv_check_status(const uint32_t* d_status, uint32_t n, hipStream_t stream);

/*
 * Batched plans: the decode stage of Methods > "GPU rendering pipeline" as
 * one persistent launch -- resident work-groups popping tasks from a device
 * queue, optionally in decreasing estimated cost -- plus the rANS table and
 * dense-offset kernels, all captured into one HIP graph.  The plan owns its
 * device scratch (sized by vol->max_log2b and the grid).  A plan serves one
 * stream at a time; distinct plans may be used from different threads.
 * max_tasks bounds n of every launch.
 */
typedef struct csgv_plan csgv_plan;

csgv_status csgv_plan_create(const csgv_volume_info* vol, uint32_t max_tasks, const csgv_decode_opts* opts,
                             csgv_plan** out);

/* Same task arguments as csgv_decode_bricks (including NULL d_out_offsets);
   enqueued on `stream`. */
csgv_status csgv_plan_launch(csgv_plan* plan, hipStream_t stream, const void* d_container, const uint32_t* d_brick_ids,
                             const uint8_t* d_lods, const uint64_t* d_out_offsets, uint32_t n, void* d_out,
                             uint64_t out_capacity, uint32_t* d_status);

/* Launch through a captured HIP graph of the whole sequence (default 1), or
   enqueue the kernels directly (0).  A graph is re-captured whenever the task
   arguments or the shape differ from the previous launch. */
csgv_status csgv_plan_set_graph(csgv_plan* plan, int enable);

/* When enabled, launches bypass the graph and bracket the decode kernel with
   HIP events on the launch stream (read with csgv_plan_last_kernel_ms). */
csgv_status csgv_plan_set_timing(csgv_plan* plan, int enable);

/* Change the launch shape (fields left 0, or -1 for sort_tasks and
   wgs_per_cu, keep their value); scratch is re-sized when needed, which
   synchronises the device. */
csgv_status csgv_plan_set_opts(csgv_plan* plan, const csgv_decode_opts* opts);

/* The shape the plan launches with (wgs_per_cu resolved to the grid / CUs). */
csgv_status csgv_plan_get_opts(const csgv_plan* plan, csgv_decode_opts* out);

/* Duration of the most recent decode kernel launched by the plan, in milliseconds
   (measured with HIP events on the plan's launch stream; synchronises on them). */
csgv_status csgv_plan_last_kernel_ms(csgv_plan* plan, float* ms);

void csgv_plan_destroy(csgv_plan* plan);

/*
 * Autotuner for the batched decode (the paper specialises its decoder per
 * volume, Methods > "GPU rendering pipeline"; here the shape is searched at
 * run time): times the plan on this task list under every candidate shape --
 * work-group size {128, 256, 512} x LDS split {8192, 10240, 16384, 24576}
 * slots, as many resident groups per CU as fit -- with HIP events on
 * `stream` (first launch of each shape discarded, best of three kept), and
 * leaves the plan on the fastest.  cache_path (or NULL): a text file of
 * "key<TAB>wg lds wgs_per_cu" lines; the key is the GPU architecture, CU
 * count, volume (label width, brick side, bricks, bytes) and task list (count,
 * LOD histogram).  A key already in the file is applied without timing.
 * Writes d_out/d_status like a launch; synchronises `stream`.
 */
typedef struct {
    int from_cache;            /* 1: shape taken from cache_path */
    int tried;                 /* shapes timed */
    float best_ms;             /* decode-kernel time of the chosen shape */
    float default_ms;          /* decode-kernel time of the default shape (256 threads, 10240 slots) */
    csgv_decode_opts chosen;   /* the plan's shape afterwards */
} csgv_tune_report;

csgv_status csgv_plan_autotune(csgv_plan* plan, hipStream_t stream, const void* d_container,
                               const uint32_t* d_brick_ids, const uint8_t* d_lods, const uint64_t* d_out_offsets,
                               uint32_t n, void* d_out, uint64_t out_capacity, uint32_t* d_status,
                               const char* cache_path, csgv_tune_report* report);

/*
 * Served decode: the request / provision / assign stages of Methods > "GPU
 * rendering pipeline" on the host in front of batched decode plans, with the
 * brick cache of Methods > "Memory management" in caller device memory.
 *  - A request is a set of (brick id, LOD) pairs that must all be resident in
 *    the cache; it completes when the last missing pair has been decoded.
 *  - The cache (d_cache, cache_elements labels of vol->label_bytes) is carved
 *    into slots of one cube each (side = brick side >> LOD; a slot keeps its
 *    size once carved).  Residency is keyed by (id, LOD); pairs of pending
 *    requests are pinned, unpinned resident pairs are evicted least recently
 *    used first within their size class, and a full cache with nothing pinned
 *    is reset (defragmentation).
 *  - Admission is in arrival order and waits for cache space.  Admitted misses
 *    are decoded in batches of up to max_batch tasks on n_streams HIP streams:
 *    whenever a stream is free, the queued tasks go out on it, so requests
 *    admitted while earlier batches run overlap with them on the device.
 *  - Times are seconds on the server's steady clock (csgv_server_clock).
 *  - A completed request's pairs stay pinned (their cache contents cannot
 *    change) until the next csgv_server_step, or with keep_pinned until
 *    csgv_server_release.
 *  - Shards (n_shards > 1): brick b belongs to shard b mod n_shards, which
 *    owns an equal, contiguous range of the cache, its own n_streams streams
 *    and its own LRU lists; every request is split into one part per shard.
 *    A request completes when its last part does (admission and completion
 *    times are the latest over its parts, pair counts the sums, status -1 if
 *    a part is rejected).  Admission is in arrival order within a shard.
 *    csgv_server_run serves the shards from one host thread each.
 * h_brick_log2b: side exponent per brick (n_bricks entries), or NULL for
 * vol->log2b everywhere.  Calls on one server come from one host thread at a
 * time.
 */
typedef struct csgv_server csgv_server;

typedef struct {
    int n_streams;            /* HIP streams (batches in flight), default 2, at most 16 */
    uint32_t max_batch;       /* tasks per batch, default 4096 */
    int keep_pinned;          /* completed requests stay pinned until csgv_server_release */
    csgv_decode_opts shape;   /* launch shape of every batch (fields 0 / -1 = defaults) */
    int n_shards;             /* cache shards (host threads in csgv_server_run), default 1, at most 16;
                                 each holds floor(cache_elements / n_shards) rounded down to 64 elements */
} csgv_server_config;

typedef struct {
    uint64_t req;             /* id returned by csgv_server_submit (or run order) */
    double t_arrival, t_admit, t_done;  /* seconds; latency = t_done - t_arrival */
    uint32_t n_pairs;         /* distinct pairs of the request */
    uint32_t n_decoded;       /* pairs this request caused to be decoded (cache misses) */
    int32_t status;           /* 0 ok, -1 rejected: the request does not fit the whole cache */
} csgv_request_done;

typedef struct {
    /* pairs_requested = hits (resident) + joined (already queued or in flight) + decoded */
    uint64_t requests_done, pairs_requested, hits, joined, decoded, evictions, resets, batches;
    uint64_t decoded_elements, requested_elements, cache_top, resident, pinned, failed_tasks;
    uint64_t splits;          /* slots of a larger class split to provide slots of a smaller one */
    uint64_t record_bytes;    /* compressed record bytes of every decoded pair (algorithmic reads) */
    double kernel_ms;         /* decode-kernel time of every batch, HIP events on the batch's stream */
    uint32_t max_batch_seen;
} csgv_server_stats;

csgv_status csgv_server_create(const csgv_volume_info* vol, const void* d_container, const uint8_t* h_brick_log2b,
                               void* d_cache, uint64_t cache_elements, const csgv_server_config* cfg,
                               csgv_server** out);
/* Seconds since the server was created (the time base of every request). */
double csgv_server_clock(const csgv_server* server);
/* Queue a request arriving at t_arrival (it is not admitted before then).
   EINVAL when a pair names no brick or a LOD beyond its brick side. */
csgv_status csgv_server_submit(csgv_server* server, const uint32_t* h_ids, const uint8_t* h_lods, uint32_t n,
                               double t_arrival, uint64_t* req);
/* One scheduling step now: retire finished batches, admit, launch.
   *busy = 1 while requests are waiting or batches are queued or in flight. */
csgv_status csgv_server_step(csgv_server* server, int* busy);
/* Completed requests (up to cap) since the last drain. */
csgv_status csgv_server_drain(csgv_server* server, csgv_request_done* out, uint32_t cap, uint32_t* n_out);
csgv_status csgv_server_release(csgv_server* server, uint64_t req);
/* Element offset in d_cache of a resident pair (EINVAL if not resident). */
csgv_status csgv_server_where(csgv_server* server, uint32_t id, uint8_t lod, uint64_t* elem_offset);
/* Serve a whole trace: request r is pairs [h_req_start[r], h_req_start[r+1])
   arriving h_arrival[r] seconds after the call starts; steps until every
   request has completed; out[r] is request r's record (times relative to
   the call's start). */
csgv_status csgv_server_run(csgv_server* server, const uint32_t* h_ids, const uint8_t* h_lods,
                            const uint64_t* h_req_start, uint32_t n_req, const double* h_arrival,
                            csgv_request_done* out);
csgv_status csgv_server_get_stats(csgv_server* server, csgv_server_stats* out);
const char* csgv_server_last_error(void);
void csgv_server_destroy(csgv_server* server);

/*
 * Device-resident cache stages (Methods > "GPU rendering pipeline": the
 * request, provision and assign stages that run before decompression;
 * Methods > "Memory management": per-LOD free stacks of released slots and an
 * atomic cache top).  A batch of (brick, LOD) requests becomes decode tasks on
 * the device, with no host round trip:
 *
 *   csgv_dcache_request(c, s, d_ids, d_lods, n, d_task_ids, d_slot, d_state);
 *   csgv_plan_launch(plan, s, d_container, d_task_ids, d_lods, d_slot, n,
 *                    d_cache, cache_elements, d_status);
 *
 * The cache is a flat array of cache_elements labels owned by the caller; a
 * pair of side exponent t = log2(brick side) - lod occupies 8^t elements at
 * its slot (element offset).  The library owns a device slot table (8 bytes
 * per brick and LOD), free stacks of stack_cap entries per size class t
 * (0 = 2^20; with one brick side a class is one LOD, as in the paper) and the
 * cache top, about 8 * (8 * n_bricks + 7 * stack_cap) bytes of device memory.
 * The brick side of a pair is read from its record in d_container, which must
 * stay valid for the cache's lifetime.
 *
 * csgv_dcache_request, one thread per request (device arrays of n entries):
 *   d_state[i]    CSGV_DC_NEW: the pair was absent and got a slot; request i
 *                 is its decode task (d_task_ids[i] = its brick id).
 *                 CSGV_DC_HIT: resident already (possibly placed by another
 *                 request of the same call).  CSGV_DC_JOINED: another request
 *                 of the same call provisions it.  CSGV_DC_FULL: absent, and
 *                 neither the free stack of its class nor the cache top had
 *                 room (then every request of the pair is FULL).
 *                 CSGV_DC_INVALID: no such brick, a LOD beyond its
 *                 side, or an unusable record.
 *   d_slot[i]     element offset of the pair's slot (NEW, HIT, JOINED), else
 *                 0xFFFFFFFFFFFFFFFF.
 *   d_task_ids[i] the brick id for NEW, else 0xFFFFFFFF, which every decode
 *                 entry point rejects (CSGV_TASK_INVALID) before it touches
 *                 the output; so d_task_ids / d_lods / d_slot are the decode's
 *                 task arrays as they stand.
 *   Exactly one request per absent pair is NEW unless the cache is full; which
 *   one, and which slot it gets, depends on the order the device runs them.
 * csgv_dcache_free releases pairs (duplicates and absent pairs are ignored):
 *   their slots go onto the free stack of their class for reuse by later
 *   requests of the same class (a full stack drops the slot until a reset).
 * csgv_dcache_reset empties the cache (all pairs absent, top 0, stacks empty).
 * csgv_dcache_query copies the top (elements) and the 7 stack counts to the
 *   host and synchronizes the stream.  The top only grows; a request that
 *   does not fit leaves it past cache_elements, and from then on until a reset
 *   only the free stacks provide slots (the paper resets a full cache).
 * Calls are stream-ordered: a request, decode and free issued on one stream
 * run in that order; calls on one cache from several streams at once race.
 * Errors: CSGV_EINVAL for null arguments (nothing enqueued), CSGV_EHIP when a
 * launch fails, CSGV_ENOMEM when the state does not fit; the message is in
 * csgv_dcache_last_error.
 */
enum {
    CSGV_DC_NEW = 0,
    CSGV_DC_HIT = 1,
    CSGV_DC_JOINED = 2,
    CSGV_DC_FULL = 3,
    CSGV_DC_INVALID = 4
};
typedef struct csgv_dcache csgv_dcache;
csgv_status csgv_dcache_create(const csgv_volume_info* vol, const void* d_container, uint64_t cache_elements,
                               uint32_t stack_cap, hipStream_t stream, csgv_dcache** out);
csgv_status csgv_dcache_request(csgv_dcache* cache, hipStream_t stream, const uint32_t* d_ids, const uint8_t* d_lods,
                                uint32_t n, uint32_t* d_task_ids, uint64_t* d_slot, uint32_t* d_state);
csgv_status csgv_dcache_free(csgv_dcache* cache, hipStream_t stream, const uint32_t* d_ids, const uint8_t* d_lods,
                             uint32_t n);
csgv_status csgv_dcache_reset(csgv_dcache* cache, hipStream_t stream);
csgv_status csgv_dcache_query(csgv_dcache* cache, hipStream_t stream, uint64_t* h_top, int32_t* h_counts);
const char* csgv_dcache_last_error(void);
void csgv_dcache_destroy(csgv_dcache* cache);

/*
 * CPU encoder (host only, multi-threaded over bricks; Methods > "Compressed
 * segmentation volumes": one operation per explicit node, coarse to fine,
 * copy from parent or neighbour when possible, else from the palette).
 *   h_voxels       all bricks concatenated; brick k holds (1 << h_log2b[k])^3
 *                  labels of label_bytes each, x fastest.
 *   h_log2b        per brick log2(side), 1..6.
 *   dims, grid     informational volume size and brick grid (may be NULL).
 *   h_origins      n_bricks x 3 voxel origins for the directory, or NULL.
 *   op_mask        bit0 PARENT, bit1 NEIGHBOR_X, bit2 NEIGHBOR_Y, bit3 NEIGHBOR_Z,
 *                  bit4 PALETTE_LAST, bit5 PALETTE_DELTA (PALETTE_ADV is always on);
 *                  bit6 limits PALETTE_DELTA to back references of at most 16 entries
 *                  (the original format's limit; labels further back are appended again,
 *                  which duplicates palette entries -- Methods > "Memory management" >
 *                  "Cache paletting").
 *   neighbor_mode  0: neighbour copies at any position; 1: only across sibling groups.
 *   coder_policy   0: per brick the smaller of plain 4-bit and rANS; 1: plain; 2: rANS.
 *   lane_syms      target symbols per rANS lane (sets the lane count W <= 256).
 *   n_threads      worker threads (0 = all hardware threads).
 * On success *h_out is a malloc'd container of *out_bytes bytes; free it with
 * csgv_free_host.
 */
csgv_status csgv_encode_bricks(const void* h_voxels, const uint8_t* h_log2b, uint32_t n_bricks, uint32_t label_bytes,
                               const uint32_t dims[3], uint32_t default_log2b, const uint32_t grid[3],
                               const uint32_t* h_origins, uint32_t op_mask, uint32_t neighbor_mode,
                               uint32_t coder_policy, uint32_t lane_syms, int n_threads, void** h_out,
                               uint64_t* out_bytes);

/*
 * Streaming form of the same encoder, for volumes produced piece by piece
 * (e.g. in z-slabs): bricks are symbolised as they are added -- their voxels
 * may be released right after csgv_encoder_add returns -- and the volume's
 * rANS frequency table and records are built by csgv_encoder_finish, whose
 * container is byte-identical to csgv_encode_bricks over all bricks in the
 * order added.  with_directory: each csgv_encoder_add passes h_origins.
 */
typedef struct csgv_encoder csgv_encoder;

csgv_status csgv_encoder_create(uint32_t label_bytes, const uint32_t dims[3], uint32_t default_log2b,
                                const uint32_t grid[3], int with_directory, uint32_t op_mask, uint32_t neighbor_mode,
                                uint32_t coder_policy, uint32_t lane_syms, int n_threads, csgv_encoder** out);
csgv_status csgv_encoder_add(csgv_encoder* enc, const void* h_voxels, const uint8_t* h_log2b, uint32_t n_bricks,
                             const uint32_t* h_origins);
csgv_status csgv_encoder_finish(csgv_encoder* enc, void** h_out, uint64_t* out_bytes);
void csgv_encoder_destroy(csgv_encoder* enc);

void csgv_free_host(void* p);

/* Thread-local description of the last failure ("" if none). */
const char* csgv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CSGV_H */
