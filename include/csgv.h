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
 *  - Per-task failures are reported in d_status (see csgv_task_status), never
 *    as a return code: a damaged record cannot fault or hang the decoder.
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
 *   brick records, each 8-byte aligned (layout in the design notes).
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
    /* the brick record or its operation stream is malformed (any rule the
       decoder checks, see the design notes): the task's output range is
       zero-filled when it is valid, otherwise untouched */
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
} csgv_volume_info;

typedef struct {
    int mode;            /* CSGV_MODE_* (default PERSISTENT for plans, PLAIN for csgv_decode_bricks) */
    int wg_size;         /* work-group size 256/512/1024; 0 = library default */
    int wgs_per_cu;      /* persistent form: resident work-groups per compute unit; 0 = default */
    int sort_tasks;      /* persistent form: pop tasks in decreasing estimated cost; -1 = default */
} csgv_decode_opts;

/*
 * Parse and validate a container header in host memory.
 * h_container: at least 128 bytes (bytes = available size).  Checks magic,
 * version, label width and that the offset table lies inside `bytes`.
 * Returns CSGV_OK or CSGV_EINVAL.
 */
csgv_status csgv_volume_parse(const void* h_container, uint64_t bytes, csgv_volume_info* out);

/*
 * Decode a batch of bricks (the decode stage).
 *   vol            header of the container, from csgv_volume_parse.
 *   d_container    the whole container in device memory (vol->total_bytes).
 *   d_brick_ids    n tasks: brick id of each task.
 *   d_lods         n tasks: LOD, 0 = full resolution; LOD k yields a cube of
 *                  side (brick side >> k) whose voxels are the mode-of-8
 *                  multi-resolution labels of that level.
 *   d_out_offsets  n tasks: element offset of each task's output in d_out.
 *   n              number of tasks (0 is allowed and enqueues nothing).
 *   d_out          labels of vol->label_bytes each; task j writes its cube,
 *                  linear with x fastest, at d_out + d_out_offsets[j].
 *   out_capacity   number of label elements available in d_out.
 *   d_status       n task status words (CSGV_TASK_*), or NULL.
 *   opts           NULL for defaults (plain form).
 * Output ranges of different tasks must not overlap.  Returns CSGV_OK,
 * CSGV_EINVAL, CSGV_ENOMEM or CSGV_EHIP.
 */
csgv_status csgv_decode_bricks(hipStream_t stream, const csgv_volume_info* vol, const void* d_container,
                               const uint32_t* d_brick_ids, const uint8_t* d_lods, const uint64_t* d_out_offsets,
                               uint32_t n, void* d_out, uint64_t out_capacity, uint32_t* d_status,
                               const csgv_decode_opts* opts);

/*
 * Synchronise `stream` and report whether any of the n status words is
 * nonzero: CSGV_OK when all tasks succeeded, CSGV_ECORRUPT otherwise.
 */
csgv_status csgv_check_status(const uint32_t* d_status, uint32_t n, hipStream_t stream);

/*
 * Batched plans: the persistent work-queue decoder with its scratch, an
 * optional cost-sorted task order and a captured HIP graph of the whole
 * launch sequence.  A plan serves one stream at a time; distinct plans may be
 * used from different threads.  max_tasks bounds n of every launch.
 */
typedef struct csgv_plan csgv_plan;

csgv_status csgv_plan_create(const csgv_volume_info* vol, uint32_t max_tasks, const csgv_decode_opts* opts,
                             csgv_plan** out);

/* Same task arguments as csgv_decode_bricks; enqueued on `stream`. */
csgv_status csgv_plan_launch(csgv_plan* plan, hipStream_t stream, const void* d_container, const uint32_t* d_brick_ids,
                             const uint8_t* d_lods, const uint64_t* d_out_offsets, uint32_t n, void* d_out,
                             uint64_t out_capacity, uint32_t* d_status);

/* Launch through a captured HIP graph of the whole sequence (default 1), or
   enqueue the kernels directly (0).  A graph is re-captured whenever the task
   arguments differ from the previous launch. */
csgv_status csgv_plan_set_graph(csgv_plan* plan, int enable);

/* When enabled, launches bypass the graph and bracket the decode kernel with
   HIP events on the launch stream (read with csgv_plan_last_kernel_ms). */
csgv_status csgv_plan_set_timing(csgv_plan* plan, int enable);

/* Work-group size (256, 512 or 1024) and whether tasks are popped in
   decreasing estimated cost (record bytes + output bytes, by powers of two). */
csgv_status csgv_plan_set_shape(csgv_plan* plan, int wg_size, int sort_tasks);

/* Options a plan resolved to (after autotuning or defaults). */
csgv_status csgv_plan_get_opts(const csgv_plan* plan, csgv_decode_opts* out);

/* Duration of the most recent decode kernel launched by the plan, in milliseconds
   (measured with HIP events on the plan's launch stream; synchronises on them). */
csgv_status csgv_plan_last_kernel_ms(csgv_plan* plan, float* ms);

void csgv_plan_destroy(csgv_plan* plan);

/*
 * CPU encoder (host only, multi-threaded over bricks).
 *   h_voxels       all bricks concatenated; brick k holds (1 << h_log2b[k])^3
 *                  labels of label_bytes each, x fastest.
 *   h_log2b        per brick log2(side), 1..6.
 *   dims, grid     informational volume size and brick grid (may be NULL).
 *   h_origins      n_bricks x 3 voxel origins for the directory, or NULL.
 *   op_mask        bit0 PARENT, bit1 NEIGHBOR_X, bit2 NEIGHBOR_Y, bit3 NEIGHBOR_Z,
 *                  bit4 PALETTE_LAST, bit5 PALETTE_DELTA (PALETTE_ADV is always on).
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

void csgv_free_host(void* p);

/* Thread-local description of the last failure ("" if none). */
const char* csgv_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CSGV_H */
