// Internal interface between the C-ABI front end (ldpc_api.hip) and the
// decode kernels (decode_i8.hip, decode_f16.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include <vector>

namespace ldpc {

// Packed per-block metadata for the binary16 kernel's row-pair layout.
// With Zh = Z/2, lane u of a codeword owns check rows u and u + Zh of the
// current block row; block column c of the posteriors is stored as Zh
// "pair words", word p holding the variables p and p + Zh of that column.
// A block with shift s = s_lo + Zh*s_hi (s_lo < Zh) sends both rows of lane
// u to pair word c*Zh + (u + s_lo) mod Zh; the two halves arrive swapped
// when [u + s_lo >= Zh] xor s_hi. With T = Zh - s_lo the wrap test is
// simply u >= T, so a gather is: word = c*Zh + s_lo + u - (u >= T ? Zh : 0).
//   bits [0, 16)  c * Zh + s_lo   (pair word before the wrap)
//   bits [16, 24) T = Zh - s_lo   (1..Zh)
//   bit  24       s_hi
// The device copy of every table carries kMetaPad zero entries after the
// last block so that a kernel may read a fixed-size window from any row
// start.
constexpr int kMetaPad = 64;

__host__ __device__ inline uint32_t pack_meta(int c, int s, int Zh) {
    const int s_lo = s % Zh;
    return (uint32_t)(c * Zh + s_lo) | ((uint32_t)(Zh - s_lo) << 16) | ((uint32_t)(s / Zh) << 24);
}

// Graph tables as seen by the kernels: constant address space, so uniform
// reads are scalar loads even when the pointer itself was loaded from a
// device table (a generic pointer would give per-lane flat loads).
typedef const __attribute__((address_space(4))) uint32_t *cmeta_t;
typedef const __attribute__((address_space(4))) int32_t *crow_t;

struct DecodeLaunch {
    const int8_t *llr;        // [n_cw][T]
    uint8_t *out_bits;        // [n_cw][K/8]
    int32_t *out_iters;       // [n_cw]
    uint8_t *out_ok;          // [n_cw] or null
    void *out_llr;            // [n_cw][Nc] or null
    const int32_t *row_ptr;   // device [rows + 1]
    const int32_t *row_pad;   // device [rows + 1] even-padded row starts (int8)
    const uint32_t *meta;     // device [E]: int8 pack_meta_i8, binary16 pack_meta
    const uint8_t *wq;        // int8 path per-(iteration,row) weights or null
    const uint16_t *wh;       // binary16 path weights or null
    uint32_t *msg;            // check-to-variable messages in device memory
                              // (binary16: always, [n_cw][E_pad][Zh] record
                              // dwords; int8:
                              // when not kept in LDS, [ceil(n_cw/2)][E_pad*Z]
                              // pair words, see BlockWork; else null)
    int w_iters;
    int n_cw, rows, n_cols, kb, Z, E, E_pad;
    int max_iter, early_exit;
    int beta, offset;         // int8: Q1.7 beta and offset; f16: bit patterns
    size_t msg_bytes;         // bytes allocated at msg (int8 device placement;
                              // kMsgTail bytes past the last pair's region)
    int cpw;                  // codewords per workgroup (int8: even, two per pair)
    int alpha;                // int8: lanes per check row (1, 2 or 4; 2 and 4:
                              // the low-latency mapping, E_pad = its message
                              // pair words per check row, device placement)
    int wmax;                 // max row weight over the kept rows
    uint64_t groups;          // int8: bit r set = row r starts a new layer
                              // group (see layer_groups)
    int refill;               // int8: persistent schedule (see
                              // decode_i8_refill_kernel): `grid` workgroups,
                              // each with a msg region of cpw / 2 pairs,
                              // taking codewords from *counter
    int grid;
    int rowpair;              // int8: the row-pair kernel (decode_i8_rp_kernel:
                              // cpw codewords of Z/2 lanes per workgroup,
                              // meta = pack_meta_i8rp, msg = [n_cw][E_pad*Z/2]
                              // pair words)
    unsigned *counter;        // refill: codewords handed out (reset per launch)
};

// A workgroup's share of an int8 decode: n codewords of one shape held as
// `slots` codeword pairs (Z lanes per pair), each pair with its own
// (device placement) message region.
struct BlockWork {
    const int8_t *llr;        // first codeword's LLRs, [n][T]
    uint8_t *out_bits;        // [n][K/8]
    int32_t *out_iters;       // [n]
    uint8_t *out_ok;          // [n] or null
    int8_t *out_llr;          // [n][Nc] or null
    uint16_t *msg;            // device placement: [slots][E_pad*Z] pair words;
                              // row r of a pair occupies pair words
                              // [row_pad[r]*Z, row_pad[r+1]*Z), lane u's Wp
                              // (the row weight rounded up to even) messages
                              // contiguous at u*Wp
    uint32_t msg_records;     // device placement: bytes of the message region
                              // this workgroup may touch (its allocated pairs
                              // plus the allocation's tail), the raw buffer's
                              // range: a read beyond it returns zero
    const int32_t *row_pad;   // even-padded row starts
    uint64_t groups;          // bit r: row r needs a barrier before it
    const uint8_t *wq;        // per-(iteration, row) weights or null
    int w_iters, w_stride;    // weight rows and row stride
    int n, slots;             // codewords here; codeword pairs of the block
    int rows, n_cols, kb, Z, E, E_pad;
    int max_iter, early_exit, beta, offset;
};

// Mixed-shape batch: one job per (shape, buffers), tasks of up to `slots`
// codewords (an even number: slots/2 pairs of Z lanes within kBatchLanes)
// of one job.
constexpr int kBatchLanes = 384;
struct BatchJob {
    const int8_t *llr;
    uint8_t *out_bits;
    int32_t *out_iters;
    uint8_t *out_ok;
    const int32_t *row_ptr;
    const int32_t *row_pad;
    const uint32_t *meta;
    const uint32_t *meta_rp;  // row-pair metadata (pack_meta_i8rp)
    const uint8_t *wq;
    uint64_t groups;
    int w_iters, w_stride;
    int rows, n_cols, kb, Z, E, E_pad, slots;
    int split;                // small tasks: one pair, or one codeword as row
                              // pairs above kBatchRowPairZ
};
// Lifts above this decode in the batch kernel's small tasks as row pairs,
// one codeword per task (see decode_rp): a codeword pair's 2Z lanes would
// put two waves on some SIMDs of a CU, and a single codeword leaves its
// workgroup as soon as it converges.
constexpr int kBatchRowPairZ = 256;
// A task is either codewords [first, first + n) of job `job` for the whole
// workgroup (nwave = 0), codeword `first` of job `job` as row pairs on the
// workgroup's first Z/2 lanes (nwave = -1, n = 1), or a bundle of nwave
// wave tasks waves[first ..
// first + nwave), one per wave of the workgroup (small lifts: a codeword
// pair of Z <= 64 fits one wave, so each wave decodes its own shape).
struct BatchTask {
    int job, first, n, nwave;
};
struct WaveTask {
    int job, first, n, pad;
};
constexpr int kWaveLanes = 64;
constexpr int kWavesPerBlock = kBatchLanes / kWaveLanes;
struct BatchLaunch {
    const BatchTask *tasks;
    const BatchJob *jobs;
    const WaveTask *waves;    // wave tasks of the bundles
    int wave_lds;             // LDS bytes per wave of a bundle
    int wave_msg;             // message pair words per wave of a bundle
    int n_tasks;
    unsigned *counter;
    uint16_t *msg;            // grid * msg_per_block pair words
    int msg_per_block;
    int max_iter, early_exit, beta, offset;
    int grid, lanes, lds, wmax;
    int counter_zeroed;       // 1: *counter is already zero on the stream (no
                              // reset kernel before the decode)
    int row_pairs;            // 1: the tasks include row-pair tasks (the
                              // kernel variant that decodes them)
};
hipError_t launch_decode_batch(const BatchLaunch &b, hipStream_t stream);

// Serving queue: tasks (codewords [first, first + n) of one job) that the
// host writes into a ring in pinned host memory while a persistent kernel
// runs. Completion of a task is published as done[ticket % capacity] =
// ticket + 1 (pinned host memory, so the host polls it without a device
// call; the value tells reuses of a slot apart).
struct ServeTask {
    BatchJob job;
    int first, n;
    unsigned ticket;
    int pad;
};
struct ServeLaunch {
    const ServeTask *ring;      // pinned host memory [capacity]
    int capacity;
    const unsigned *host_ctl;   // pinned: [0] tasks published, [1] stop request
    unsigned *done;             // pinned [capacity]
    unsigned *dev_ctl;          // device: [0] tasks claimed, [1] published (mirror), [2] stop
    uint16_t *msg;              // (grid - 1) * msg_per_block pair words (+ tail)
    int msg_per_block;
    int max_iter, early_exit;
    int grid, lds;
    int idle_polls;             // a decode workgroup leaves after this many empty polls
};
// LDS bytes and message pair words of a serving workgroup (kBatchLanes
// lanes): enough for floor(kBatchLanes / Z) codeword pairs of any shape with
// up to 68 columns, 46 rows and row weights up to 20.
constexpr int kServeLds = 53248;
constexpr int kServeMsgPerBlock = kBatchLanes * 46 * 20;
hipError_t launch_serve(const ServeLaunch &s, hipStream_t stream);

// Tasks of a mixed batch (see BatchTask), longest first, with the LDS and
// message sizes a workgroup needs. Returns LDPC_OK or LDPC_EINVAL.
struct TaskSet {
    std::vector<BatchTask> tasks;
    std::vector<WaveTask> waves;
    int lds = 0, msg_per_block = 0, wave_lds = 0, wave_msg = 0;
    bool row_pairs = false;  // some tasks are row-pair tasks (nwave = -1)
};
int build_tasks(const std::vector<BatchJob> &jobs, const std::vector<int> &job_cw, int lds_cap,
                TaskSet &ts);

struct Plan;
int plan_build(Plan *p, const std::vector<BatchJob> &jobs, const std::vector<int> &job_cw,
               int lanes, int max_iter, int early_exit, int beta, int offset, int wmax,
               int lds_cap, hipStream_t stream);
int plan_autotune(Plan *p, hipStream_t stream);
int plan_capture(Plan *p);
int plan_launch(Plan *p, hipStream_t stream);
void plan_destroy(Plan *p);
Plan *plan_new();
void plan_info(const Plan *p, int *grid, int *n_tasks, float *tuned_ms);
int batch_async_bytes(const std::vector<BatchJob> &jobs, const std::vector<int> &job_cw,
                      int lds_cap, size_t *bytes);
int batch_async(const std::vector<BatchJob> &jobs, const std::vector<int> &job_cw, int lanes,
                int max_iter, int early_exit, int wmax, int lds_cap, hipStream_t stream,
                size_t *bytes_in_flight);

// Bytes allocated past the last int8 message region: a lane's message loads
// move whole dwordx4 chunks, which for the last lane of the last pair can
// reach up to 12 bytes past its row (the dwords beyond the row are unused).
constexpr size_t kMsgTail = 16;

// Bytes of LDS one int8 codeword pair needs (posteriors and messages, or
// posteriors only) and one binary16 codeword.
__host__ __device__ inline int lds_bytes_i8_pair(int n_cols, int E, int Z) {
    return 2 * (n_cols + E) * Z;
}
__host__ __device__ inline int lds_bytes_i8_pair_post(int n_cols, int Z) { return 2 * n_cols * Z; }
// The int8 workgroup's flag words after its pairs: one syndrome flag per
// codeword and one workgroup-wide "all finished" word (plus padding).
// LDS words after the pairs' posteriors: per codeword a failing-check flag,
// one workgroup flag, one spare word, and (refill schedule) per codeword the
// index of the codeword it holds.
__host__ __device__ inline int lds_flags_bytes_i8(int pairs) { return 4 * (4 * pairs + 2); }
__host__ __device__ inline int lds_bytes_f16(int n_cols, int Z) { return n_cols * Z * 2; }

// Layer groups: consecutive block rows that share no block column read and
// write disjoint posteriors, so they may follow each other without a
// workgroup barrier and the result is the one of the strictly sequential
// layered schedule. Greedy from row 0: bit r is set when row r shares a
// column with a row of the current group (row 0 always starts one).
inline uint64_t layer_groups(const int32_t *row_ptr, const int16_t *col, int rows) {
    uint64_t bits = 1, used[2] = {0, 0};  // columns < 128 as a bit set
    for (int r = 0; r < rows; ++r) {
        uint64_t cur[2] = {0, 0};
        for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) cur[col[e] >> 6] |= 1ull << (col[e] & 63);
        if (r > 0 && ((cur[0] & used[0]) | (cur[1] & used[1]))) {
            bits |= 1ull << r;
            used[0] = used[1] = 0;
        }
        used[0] |= cur[0];
        used[1] |= cur[1];
    }
    return bits;
}

// Per-block metadata for the int8 pair kernel: bits [0, 16) the byte offset
// 2(c*Z + s) of variable s of column c in a pair's posteriors, bits
// [16, 25) the wrap threshold Z - s (lane u reads variable (u + s) mod Z,
// which wraps for u >= Z - s).
__host__ __device__ inline uint32_t pack_meta_i8(int c, int s, int Z) {
    return (uint32_t)(2 * (c * Z + s)) | ((uint32_t)(Z - s) << 16);
}

// Per-block metadata for the int8 row-pair kernel (one codeword; lane u of
// its Zh = Z/2 lanes owns check rows u and u + Zh; pair word p of column c
// holds variables p and p + Zh): for the shift s = s_lo + Zh*s_hi (s_lo <
// Zh), bits [0, 15) the byte offset 2(c*Zh + s_lo) of the pair word before
// the wrap, bit 15 s_hi, bits [16, 25) the wrap threshold Zh - s_lo (lane u
// reads pair word c*Zh + (u + s_lo) mod Zh, which wraps for u >= Zh - s_lo).
__host__ __device__ inline uint32_t pack_meta_i8rp(int c, int s, int Zh) {
    const int s_lo = s % Zh;
    return (uint32_t)(2 * (c * Zh + s_lo)) | ((uint32_t)(s / Zh) << 15) |
           ((uint32_t)(Zh - s_lo) << 16);
}

// Per-block metadata for the one-check-row-per-lane learned min-sum:
// bits [0, 16) c * Z, bits [16, 25) shift.
__host__ __device__ inline uint32_t pack_meta_row(int c, int s, int Z) {
    return (uint32_t)(c * Z) | ((uint32_t)s << 16);
}

// Low-latency int8 mapping (alpha lanes per check row): chunks of at most
// kLLChunkMax blocks per lane; LDS of `pairs` pairs' posteriors, their flags
// and the two alternating exchange buffers [alpha][3][pairs * Z] dwords;
// message pair words per check row of the first `rows` rows.
constexpr int kLLChunkMax = 10;
__host__ __device__ inline int ll_lds_bytes(int n_cols, int Z, int pairs, int alpha) {
    return pairs * lds_bytes_i8_pair_post(n_cols, Z) + lds_flags_bytes_i8(pairs) +
           2 * alpha * 3 * pairs * Z * 4;
}
int ll_message_pair_words(const int32_t *row_ptr, int rows, int alpha);

// binary16 message record of a row of w blocks (a1, a2 and the sign and
// argmin flag words), in dwords per lane.
__host__ __device__ inline int f16_record_dwords(int w) {
    return 2 + (w <= 8 ? 1 : (w <= 16 ? 2 : 4));
}

// Host launchers; return hipSuccess or the launch error.
hipError_t launch_decode_i8(const DecodeLaunch &p, hipStream_t stream);
hipError_t launch_decode_f16(const DecodeLaunch &p, hipStream_t stream);

// Learned weighted min-sum: forward, backward and gradient reduction.
size_t nwms_workspace_floats(int n_cw, int rows, int n_cols, int Z, int E, int n_iter);
hipError_t launch_nwms(const float *llr, const uint8_t *cbits, const float *w,
                       const float *iter_w, float *loss,
                       float *grad, float *out_llr, float *ws, int n_cw, int rows, int n_cols,
                       int Z, int E, int n_iter, float scale, const int32_t *row_ptr,
                       const uint32_t *meta_row, int wmax, hipStream_t stream);

// Largest dynamic LDS a workgroup may use on the device (bytes).
int max_lds_bytes();

// Remember a failed HIP call for ldpc_last_error_message().
void note_hip_error(const char *where, hipError_t e);

}  // namespace ldpc
