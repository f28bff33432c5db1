/*
 * ldpc.h -- C ABI of the MI355X (gfx950) layered normalised min-sum decoder
 * for 5G-NR-shaped quasi-cyclic LDPC codes.
 *
 * Method: Ling & Cautereels, "Fast LDPC GPU Decoder for Cloud RAN".
 *   - code: quasi-cyclic, base graph lifted by Z, K = K_b*Z information bits,
 *     the first two information columns punctured, rate set by the number of
 *     base rows kept (§II);
 *   - decoding: horizontal layered belief propagation with the normalised
 *     min-sum check rule, posterior and extrinsic updates, iterate until the
 *     hard decisions satisfy every check or the iteration limit (§III);
 *   - per-row intermediates min, second min and sign product (§IV);
 *   - 8-bit fixed point and packed binary16 number formats (§I, §IV).
 *
 * Conventions shared by every entry point
 *   - All array arguments of decode calls are DEVICE pointers owned by the
 *     caller; graph registration takes HOST pointers and copies them.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Decode calls are asynchronous: outputs are valid once the stream has
 *     reached the point of the call.
 *   - A call that returns an error code has launched nothing and written no
 *     output.
 *   - Variables are ordered column-block-major: bit j = c*Z + z.
 *     Circulant convention: block (r, c) with shift s joins check row z of
 *     block row r to variable (z + s) mod Z of block column c.
 *   - The library is reentrant; graph registration and plan look-ups are
 *     serialised by a mutex. Calls on different streams may overlap.
 */
#ifndef LDPC_MI355X_H
#define LDPC_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define LDPC_OK 0
#define LDPC_EINVAL (-1)   /* an argument is out of range or a pointer is NULL */
#define LDPC_ENOMEM (-2)   /* device or host allocation failed */
#define LDPC_EHIP (-3)     /* a HIP runtime call failed (see ldpc_last_hip_error) */
#define LDPC_ENOGRAPH (-4) /* no graph registered for (bg, Z) */

/* Number formats (ldpc_args.precision). */
#define LDPC_I8 0  /* 8-bit saturating fixed point, symmetric +-127 */
#define LDPC_F16 1 /* IEEE binary16, round to nearest even after every op */

/* Supported lifts: Z a multiple of 8 with 8 <= Z <= 384, which covers the
 * lifts {16, 32, 64, 96, 128, 192, 256, 384}. Base graphs: 4 to 46 rows, up
 * to 68 columns, row weight 2..32. */
#define LDPC_MAX_Z 384
#define LDPC_MAX_ROWS 46
#define LDPC_MAX_COLS 68
#define LDPC_MAX_ROW_WEIGHT 32
#define LDPC_MAX_ITER 64

/*
 * Graph tables are data. The library holds no base-graph generator and so
 * exports no seeded initialiser: the caller registers each lifted base graph
 * with ldpc_set_graph (the same call would load the standard's tables), can
 * read back what is registered with ldpc_get_graph, and can check it by its
 * digest (ldpc_graph_digest). A checker that must decode the same graph as
 * the library takes the table from ldpc_get_graph.
 *
 * ldpc_set_graph -- register the full base graph `bg` (an identifier >= 1)
 * lifted by Z (§II). The graph has m_rows block rows and n_cols = kb + m_rows
 * block columns, the first 2 columns punctured. Block e of row r
 * (row_ptr[r] <= e < row_ptr[r+1], strictly ascending col) has column col[e]
 * and shift shift[e] in [0, Z). Keeping the first `rows` block rows and the
 * first kb + rows columns must give a valid sub-code for every rows in
 * [4, m_rows], so every block of row r must lie in a column
 * < kb + max(r + 1, 4) (as in the 5G base graphs); m_rows >= 4, row
 * weights 2..32. Host pointers; the library copies
 * them to device memory. Re-registering (bg, Z) replaces the graph; the
 * caller must not do so while a decode of (bg, Z) is in flight.
 * Errors: LDPC_EINVAL (shape, ordering, shift or weight out of range),
 * LDPC_ENOMEM, LDPC_EHIP.
 */
int ldpc_set_graph(int bg, int Z, int m_rows, int kb, const int32_t *row_ptr,
                   const int16_t *col, const int16_t *shift);

/* Sizes of the sub-code keeping `rows` block rows of graph (bg, Z):
 * K information bits, T transmitted LLRs per codeword ((kb+rows-2)*Z),
 * Nc = (kb+rows)*Z code bits, E nonzero blocks. Any output may be NULL. */
int ldpc_query(int bg, int Z, int rows, int *K, int *T, int *Nc, int *E);

/*
 * ldpc_get_graph -- the registered base graph (bg, Z) as a list of nonzero
 * blocks, row-major with columns ascending within a row (§II: block (r, c)
 * with shift s is a Z x Z cyclic permutation). Host pointers owned by the
 * caller. *nnz is in/out: on entry the capacity of row/col/shift, on return
 * the number of blocks E. With row, col and shift all NULL only the sizes
 * are returned (m_rows, kb, nnz may each be NULL).
 * Errors: LDPC_ENOGRAPH; LDPC_EINVAL (some but not all of row/col/shift
 * NULL, nnz NULL, or capacity below E; nothing is written).
 */
int ldpc_get_graph(int bg, int Z, int *m_rows, int *kb, int *nnz, int16_t *row, int16_t *col,
                   int16_t *shift);

/*
 * ldpc_graph_digest -- 64-bit FNV-1a digest of the registered graph
 * (bg, Z): the bytes hashed are little-endian int32 words bg, Z, m_rows,
 * kb, row_ptr[0..m_rows], col[0..E), shift[0..E) (col and shift
 * sign-extended). Host-side only; no device call.
 * Errors: LDPC_EINVAL (out NULL), LDPC_ENOGRAPH.
 */
int ldpc_graph_digest(int bg, int Z, uint64_t *out);

/*
 * ldpc_decode -- layered normalised min-sum (beta = 3/4), int8 path, early
 * exit on a zero syndrome (§III).
 *   bg, Z, rows : registered graph and number of block rows kept, 4..m_rows
 *   n_cw        : number of codewords (>= 1)
 *   llr_in      : int8 [n_cw][T], channel LLRs of the transmitted bits in
 *                 variable order (punctured columns absent), LLR units of
 *                 1/4 (any value is legal; -128 is read as -127); 4-byte
 *                 aligned (the kernels read it as 32-bit words), else
 *                 LDPC_EINVAL
 *   max_iter    : 1..64 iterations
 *   out_bits    : uint8 [n_cw][K/8] hard decisions of the K information
 *                 bits (including the punctured ones), packed LSB first
 *   out_iters   : int32 [n_cw] iterations run (the first iteration after
 *                 which every check held, else max_iter)
 * Errors: LDPC_EINVAL, LDPC_ENOGRAPH, LDPC_EHIP, LDPC_ENOMEM.
 */
int ldpc_decode(int bg, int Z, int rows, int n_cw, const int8_t *llr_in, int max_iter,
                uint8_t *out_bits, int32_t *out_iters, void *stream);

/* Extended decode arguments. Fields not used by a precision are ignored. */
typedef struct ldpc_args {
    int bg, Z, rows, n_cw;
    int precision;          /* LDPC_I8 or LDPC_F16 */
    int max_iter;           /* 1..64 */
    int early_exit;         /* 1: stop a codeword once all its checks hold;
                               0: run max_iter iterations (out_ok still set) */
    const int8_t *llr_in;   /* int8 [n_cw][T] (both precisions), 4-byte aligned */
    /* Normalisation of the min-sum magnitude (§III correction factor):
     *   i8  : a = min((w*max(m - offset_q, 0) + 64) >> 7, 127), w = beta_q
     *         or wq[min(t, wq_iters) - 1][r] (Q1.7, 0..255) when wq != NULL
     *   f16 : a = w * max(m - offset_h, 0) in binary16, w = beta_h or
     *         wh[min(t, wh_iters) - 1][r] (binary16 bit patterns)        */
    int beta_q;             /* Q1.7 multiplier, default 96 (= 3/4) */
    int offset_q;           /* 0..127, default 0 */
    const uint8_t *wq;      /* device uint8 [wq_iters][rows] or NULL */
    int wq_iters;
    uint16_t beta_h;        /* binary16, default 0x3A00 (= 0.75) */
    uint16_t offset_h;      /* binary16, default 0 */
    const uint16_t *wh;     /* device binary16 [wh_iters][rows] or NULL */
    int wh_iters;
    uint8_t *out_bits;      /* uint8 [n_cw][K/8] */
    int32_t *out_iters;     /* int32 [n_cw] */
    uint8_t *out_ok;        /* uint8 [n_cw] or NULL: 1 if every check holds */
    void *out_llr;          /* NULL, or final posteriors [n_cw][Nc] in
                               variable order: int8 (I8) or binary16 (F16) */
    int cw_per_block;       /* 0 = library default; else codewords per
                               workgroup (tuning knob; the int8 path decodes
                               codewords in pairs and rounds it up to even;
                               by default codeword pairs fill about 768
                               lanes per workgroup, or fewer when the
                               batch has fewer pairs than that per CU, so
                               that a small batch spreads over the CUs) */
    int msg_placement;      /* where the int8 path keeps its check-to-
                               variable messages: LDPC_MSG_AUTO,
                               LDPC_MSG_LDS (next to the posteriors in LDS;
                               LDPC_EINVAL if one codeword pair's posteriors
                               and messages, 2*(Nc/Z + E)*Z bytes, exceed a
                               workgroup's LDS -- with row pairs, one
                               codeword's, (Nc/Z + E)*Z bytes: 147 kB for
                               BG1 at Z = 384) or LDPC_MSG_DEVICE (device
                               memory, allocated
                               by the library per call, stream-ordered; more
                               codewords then share a CU). AUTO: codeword
                               pairs as described under pairing's default;
                               row pairs in LDS for at most one codeword per
                               CU when no row is heavier than 10 blocks and
                               the state fits, else in device memory.
                               binary16 always uses device memory. */
    int lanes_per_row;      /* int8: lanes cooperating on one check row
                               (the paper's alpha): 0 or 1 = one lane per row
                               (the throughput mapping); 2 or 4 = the
                               low-latency mapping (§IV): each block row is
                               cut into alpha chunks of consecutive blocks,
                               one per lane, and the chunks' minima, second
                               minima and sign parities are merged through
                               LDS. Needs device-placed messages, row weights
                               up to min(20, 10*alpha), alpha*P*Z <= 1024 and
                               P*Z a multiple of 64 for P = cw_per_block/2
                               pairs per workgroup (default: the fewest pairs
                               that give whole waves); else LDPC_EINVAL.
                               Results are identical for every alpha. */
    int schedule;           /* LDPC_SCHED_STATIC (0, the default) = one
                               fixed block of codewords per workgroup;
                               LDPC_SCHED_PERSISTENT (1) = as many
                               workgroups as run at once, whose codeword
                               pairs take the next codeword as soon as one
                               of theirs finishes (int8 with early exit, one
                               lane per row, device-placed messages, plain
                               normalisation and cw_per_block = 0, else
                               LDPC_EINVAL; message memory for the resident
                               workgroups only). Results are identical under
                               both. */
    int max_workgroups;     /* persistent schedule: at most this many
                               workgroups (0 = as many as fit the device) */
    int pairing;            /* int8: what shares a lane's two 16-bit halves.
                               LDPC_PAIR_CODEWORDS (1): two codewords (the
                               same check row of each; Z lanes per pair).
                               LDPC_PAIR_ROWS (2): check rows u and u + Z/2
                               of one codeword (Z/2 lanes per codeword,
                               cw_per_block codewords per workgroup, default
                               up to Z = 128 the most that fit one wave, at
                               most 4; 2 to Z = 256; 1 above); the static
                               schedule and one lane per row, else
                               LDPC_EINVAL; messages placed as msg_placement
                               says): for
                               small batches of large lifts, where a pair's
                               2Z lanes would put two waves on some of a
                               CU's SIMDs, and for early exit (one codeword
                               per workgroup leaves its CU as soon as it
                               converges). LDPC_PAIR_AUTO (0, the default):
                               with one lane per row, the static schedule,
                               cw_per_block 0 and message placement AUTO,
                               row pairs at Z > 256 for n_cw at most the
                               device's CU count and with early exit (if no
                               row weighs more than 10 blocks, not for n_cw
                               of four to eight times the CU count, four
                               excluded), and at
                               Z = 16 .. 256 with early exit for n_cw above
                               four times the CU count; else codeword
                               pairs.
                               Results are identical under both. */
    void *stream;
} ldpc_args;

#define LDPC_MSG_AUTO 0
#define LDPC_MSG_LDS 1
#define LDPC_MSG_DEVICE 2
#define LDPC_SCHED_STATIC 0
#define LDPC_SCHED_PERSISTENT 1
#define LDPC_PAIR_AUTO 0
#define LDPC_PAIR_CODEWORDS 1
#define LDPC_PAIR_ROWS 2

/* Fill `a` with the defaults above (beta 3/4, no offset, early exit on,
 * int8, 10 iterations, no optional outputs). */
void ldpc_args_init(ldpc_args *a);

/* ldpc_decode_ex -- decode with the options of ldpc_args. Messages kept in
 * device memory take 2*ceil(n_cw/2)*E_pad*Z bytes (int8; E_pad = E with
 * every row's weight rounded up to even; n_cw*E_pad*Z + 16 with row pairs;
 * under the persistent schedule
 * 2*G*P*E_pad*Z bytes plus at most 528 for G workgroups of P pairs, G at
 * most the workgroups that run at once) or 2*n_cw*Rd*Z bytes (binary16,
 * where every row's messages are stored exactly as a record of a1, a2 and
 * per-block sign and argmin flags: Rd = the sum over rows of 3 dwords for
 * rows of up to 8 blocks, 4 up to 16, 6 up to 32), allocated per call with
 * hipMallocAsync on `stream` and released the same way.
 * Errors: as ldpc_decode. */
int ldpc_decode_ex(const ldpc_args *a);

/*
 * ldpc_decode_noalloc -- ldpc_decode_ex for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments, checks, kernels and results, but the
 * check-to-variable messages live in a static per-device scratch array of
 * LDPC_NOALLOC_SCRATCH_BYTES (64 MiB, part of the library's code object,
 * held on every device the library runs on until the process ends) instead
 * of a per-call allocation. No device or host memory is allocated or freed.
 *   - Always the static schedule (one fixed block of codewords per
 *     workgroup).
 *   - Limit: the message bytes of ldpc_decode_ex (int8:
 *     2*ceil(n_cw/2)*E_pad*Z + 16 unless the messages are placed in LDS,
 *     more with lanes_per_row > 1; binary16: 2*n_cw*Rd*Z) must not exceed
 *     the scratch, else LDPC_EINVAL and ldpc_last_error_message() names both
 *     sizes. At BG1 Z = 384 with 46 rows that is up to 514 int8 or 578
 *     binary16 codewords per call.
 *   - The graph's device tables must already be resident on the current
 *     device (any ldpc_decode / ldpc_decode_ex call of (bg, Z) there uploads
 *     them), else LDPC_ENOGRAPH with a message saying so.
 *   - Every call on one device shares that device's scratch: calls that
 *     overlap on one device (different streams, or other threads) race and
 *     give wrong results. Serialise them, e.g. on one stream. The decoders
 *     write every message before reading it, so nothing needs clearing
 *     between calls.
 * Errors: as ldpc_decode_ex (LDPC_ENOMEM never occurs).
 */
#define LDPC_NOALLOC_SCRATCH_BYTES (64u << 20)
int ldpc_decode_noalloc(const ldpc_args *a);

/*
 * ldpc_tune -- autotuning of the int8 launch configuration. Times the
 * candidate configurations of ldpc_decode_ex on the arguments in `a` (their
 * launch knobs lanes_per_row, cw_per_block, msg_placement and pairing must
 * be at their defaults 0, 0, AUTO, AUTO, and schedule static): the
 * library's default launch (if it is fastest nothing is recorded and
 * out->cw_per_block is 0), the persistent schedule where it applies, one
 * lane per check row with 1, 2, 3, 4, 6, 8, 12, 16, 24 or 48 codeword
 * pairs per workgroup (those that fit) and the messages in LDS or in
 * device memory, 2 or 4 lanes per check row with the fewest pairs that
 * give whole waves and twice that, and row pairs with 1, 2 or 4 codewords
 * per workgroup. Every candidate decodes a's input into a's outputs (all give
 * the same results), four times, and the fastest after the first is
 * recorded for (bg, Z, rows, n_cw rounded up to a power of two,
 * early_exit): later int8 ldpc_decode_ex / ldpc_decode_noalloc calls whose
 * launch knobs are at their defaults use it. Synchronises a->stream.
 * out (may be NULL): the chosen knobs, its time and the number of
 * candidates timed. Errors: LDPC_EINVAL (not int8, knobs not at their
 * defaults, or no candidate applies), as ldpc_decode_ex otherwise.
 */
typedef struct ldpc_tuning {
    int lanes_per_row, cw_per_block, msg_placement;
    int schedule; /* LDPC_SCHED_PERSISTENT: the persistent schedule won */
    int pairing;  /* LDPC_PAIR_ROWS: row pairs won (cw_per_block codewords
                     per workgroup); LDPC_PAIR_CODEWORDS: codeword pairs;
                     AUTO: the default launch won */
    float ms;
    int candidates;
} ldpc_tuning;
int ldpc_tune(const ldpc_args *a, ldpc_tuning *out);

/*
 * Mixed-shape batches. A job is a set of codewords of one shape (bg, Z,
 * rows) with its own device buffers: llr int8 [n_cw][T] (4-byte aligned,
 * else LDPC_EINVAL), out_bits
 * [n_cw][K/8], out_iters int32 [n_cw], out_ok uint8 [n_cw] or NULL, and
 * optional per-(iteration, row) Q1.7 weights wq [wq_iters][rows] (NULL:
 * beta = 3/4). All of a batch's jobs are decoded by ONE persistent launch of
 * the int8 kernel (messages in device memory): each 384-lane workgroup takes
 * tasks from a device counter until none are left. A task is up to
 * 2*floor(384/Z) codewords of one job, or, for lifts up to 64, a bundle of
 * six wave tasks (one per 64-lane wave, each up to 2*floor(64/Z) codewords
 * of its own job), so small shapes with few codewords do not leave most of
 * a workgroup idle. A job with `split` set is cut finer, for latency when
 * the launch has the device to itself: one codeword pair per task (the
 * workgroup's other pair slots idle), and for lifts above 256 one codeword
 * per task as check rows u and u + Z/2 per lane. Results are identical to decoding each job alone
 * (ldpc_decode_ex with the same options). Lifts up to 384, row weights up
 * to 20.
 */
typedef struct ldpc_job {
    int bg, Z, rows, n_cw;
    const int8_t *llr;
    uint8_t *out_bits;
    int32_t *out_iters;
    uint8_t *out_ok;
    const uint8_t *wq;
    int wq_iters;
    int split;              /* 1: small tasks (see above); 0: full tasks */
} ldpc_job;

/* One-shot batch decode: builds a transient plan, launches it on `stream`,
 * waits for the stream, and releases the plan. */
int ldpc_decode_batch(const ldpc_job *jobs, int n_jobs, int max_iter, int early_exit,
                      void *stream);

/* Asynchronous one-shot batch: the job tables, task queue and message
 * regions are allocated, used and released in stream order on `stream`;
 * the call returns without waiting. *bytes_in_flight (may be NULL) receives
 * the device memory the launch holds until it completes. Launches needing
 * at most 32 MiB take it from a buffer the library keeps per (device,
 * stream), reused by the next such launch on that stream in stream order
 * (it grows to the largest of them, a power of two, and is kept until the
 * process ends); larger ones allocate and free in stream order. */
int ldpc_decode_batch_async(const ldpc_job *jobs, int n_jobs, int max_iter, int early_exit,
                            void *stream, size_t *bytes_in_flight);

/* Device bytes that ldpc_decode_batch_async would hold in flight for these
 * jobs (tables, task queue and per-workgroup message regions), computed on
 * the host without allocating or launching: what a caller admitting work
 * against a memory budget must reserve. Same argument checks as the batch
 * calls. Errors: LDPC_EINVAL, LDPC_ENOGRAPH. */
int ldpc_decode_batch_bytes(const ldpc_job *jobs, int n_jobs, size_t *bytes);

/* A reusable plan bound to the jobs' buffers (refill the inputs and launch
 * again). Flags: LDPC_PLAN_GRAPH captures the launch (a counter-reset
 * kernel, then the decode) as a HIP graph that ldpc_plan_launch replays;
 * LDPC_PLAN_AUTOTUNE times 1..k workgroups per CU on the plan's own work
 * (running it, so the outputs are written) and keeps the fastest. Creation
 * synchronises `stream`. Plans launched on different streams must not
 * overlap (they share the plan's counter and message regions). */
typedef struct ldpc_plan ldpc_plan;
#define LDPC_PLAN_GRAPH 1
#define LDPC_PLAN_AUTOTUNE 2
int ldpc_plan_create(const ldpc_job *jobs, int n_jobs, int max_iter, int early_exit, int flags,
                     void *stream, ldpc_plan **out);
int ldpc_plan_launch(ldpc_plan *plan, void *stream);
/* grid: persistent workgroups; n_tasks: tasks in the queue (a bundle of
 * small-lift wave tasks counts once); tuned_ms: time
 * of the chosen grid when autotuned (else 0). Any output may be NULL. */
int ldpc_plan_info(const ldpc_plan *plan, int *grid, int *n_tasks, float *tuned_ms);
void ldpc_plan_destroy(ldpc_plan *plan);

/*
 * Serving queue -- SWITCHED OFF: ldpc_server_create returns LDPC_EINVAL and
 * creates nothing (on MI355X the persistent kernel did not finish in
 * testing and the cause is not known), so no other ldpc_server_* call has a
 * server to act on. The design it implements:
 * Serving queue (continuous batching on the device). A persistent decode
 * kernel takes tasks from a ring of descriptors that the host keeps
 * appending while it runs: workgroup 0 polls the count of published tasks
 * in pinned host memory, the others claim published tasks one at a time,
 * decode them (one task = up to 2*floor(384/Z) codewords of one job, int8,
 * one lane per check row, beta = 3/4 or the job's Q1.7 weights) and publish
 * each task's completion in pinned host memory, so the host polls it
 * without a device call. The job's outputs may live in pinned host memory
 * (written directly by the kernel and visible once the task is done) or in
 * device memory; its LLRs must be on the device before submission. The
 * kernel leaves by itself after about idle_polls empty polls (0: 4000, a
 * few milliseconds); ldpc_server_submit and ldpc_server_pump relaunch it
 * whenever tasks are pending and no launch is running. Device memory: a
 * message region of 384*46*20 pair words per decode workgroup.
 *   ldpc_server_create : capacity = tasks in flight at most (ring slots);
 *                        grid = decode workgroups (0: one per CU)
 *   ldpc_server_submit : appends the job's tasks; *first_ticket and *n_tasks
 *                        name them (tickets first .. first + n - 1).
 *                        LDPC_ENOMEM if the ring has no room (nothing is
 *                        appended); row weights above 20: LDPC_EINVAL.
 *   ldpc_server_done   : 1 once the task has completed, else 0.
 *   ldpc_server_pump   : relaunches the kernel if needed; optional
 *                        *outstanding (tasks not yet completed) and
 *                        *launches (kernel launches so far).
 *   ldpc_server_destroy: asks the kernel to stop, waits for it, frees.
 * One host thread at a time per server (calls are serialised by a mutex).
 */
typedef struct ldpc_server ldpc_server;
int ldpc_server_create(int capacity, int grid, int max_iter, int early_exit, int idle_polls,
                       ldpc_server **out);
int ldpc_server_submit(ldpc_server *s, const ldpc_job *job, unsigned *first_ticket,
                       int *n_tasks);
int ldpc_server_done(ldpc_server *s, unsigned ticket);
int ldpc_server_pump(ldpc_server *s, int *outstanding, int *launches);
int ldpc_server_destroy(ldpc_server *s);

/*
 * ldpc_nwms_loss_grad -- learned weighted min-sum (the min-sum correction
 * factor of §III replaced by one trainable multiplier w[t][r] per iteration
 * t and block row r): fp32 unrolled forward pass over n_iter iterations
 * (no early exit), loss, and the exact gradient from a hand-written
 * backward pass through the layered schedule.
 *   llr   : float [n_cw][T] channel LLRs (device), in units where the
 *           natural-log LLR is llr / scale
 *   cbits : uint8 [n_cw][Nc] the transmitted codewords, 0/1 (device)
 *   w     : float [n_iter][rows] multipliers (device)
 *   iter_w: float [n_iter] loss weight of each iteration (device), or NULL
 *           for 1/n_iter each
 *   loss  : float [n_cw] out: sum over iterations t of iter_w[t] times the
 *           mean over code bits j of BCE(sigmoid(-L_tj / scale), c_j), L_t
 *           the posteriors after t
 *   grad  : float [n_iter][rows] out: d(sum of loss)/dw, summed over the
 *           codewords in index order
 *   out_llr : float [n_cw][Nc] final posteriors or NULL
 * Signs and argmins are held fixed in the backward pass (min-sum is
 * piecewise linear); argmin ties resolve to the first block in the row.
 * Workspace (about (n_iter+1)*(E+Nc)*Z*4 bytes per codeword) is allocated
 * per call on `stream`. Row weights up to LDPC_NWMS_MAX_ROW_WEIGHT and
 * Nc*4 bytes of LDS per codeword.
 * Errors: LDPC_EINVAL, LDPC_ENOGRAPH, LDPC_ENOMEM, LDPC_EHIP.
 */
#define LDPC_NWMS_MAX_ROW_WEIGHT 20
int ldpc_nwms_loss_grad(int bg, int Z, int rows, int n_cw, const float *llr,
                        const uint8_t *cbits, int n_iter, const float *w, const float *iter_w,
                        float scale, float *loss, float *grad, float *out_llr, void *stream);

/* Error text for a return code; the last HIP error code seen by the
 * library (hipError_t as int, 0 if none). */
const char *ldpc_strerror(int code);
int ldpc_last_hip_error(void);

/* Text naming the last failed HIP call on this thread and its error
 * ("" if none). */
const char *ldpc_last_error_message(void);

/* Release every device table the library holds (graphs). */
void ldpc_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* LDPC_MI355X_H */
