// Mixed-shape batch plans: one persistent launch decodes many jobs (each a
// set of codewords of one (bg, Z, rows) shape with its own buffers). A plan
// owns the device task and job tables, the per-workgroup message regions and
// the work counter; it can be captured once as a HIP graph (a counter-reset
// kernel, then the decode) and replayed, and it can pick its grid size by
// timing the candidates on its own work (autotuning).
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/ldpc.h"
#include "ldpc_internal.h"

namespace ldpc {

struct Plan {
    BatchLaunch launch{};
    BatchTask *d_tasks = nullptr;
    BatchJob *d_jobs = nullptr;
    WaveTask *d_waves = nullptr;
    unsigned *d_counter = nullptr;
    uint16_t *d_msg = nullptr;
    size_t msg_capacity = 0;  // pair words allocated
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int cus = 0, max_per_cu = 1;
    float tuned_ms = 0.0f;
};

namespace {

void free_plan(Plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_tasks) (void)hipFree(p->d_tasks);
    if (p->d_jobs) (void)hipFree(p->d_jobs);
    if (p->d_waves) (void)hipFree(p->d_waves);
    if (p->d_counter) (void)hipFree(p->d_counter);
    if (p->d_msg) (void)hipFree(p->d_msg);
    delete p;
}

// Grow the message workspace to `grid` workgroups.
hipError_t size_messages(Plan *p, int grid) {
    const size_t need = (size_t)grid * p->launch.msg_per_block;
    if (need > p->msg_capacity) {
        if (p->d_msg) (void)hipFree(p->d_msg);
        p->d_msg = nullptr;
        p->msg_capacity = 0;
        hipError_t e = hipMalloc(&p->d_msg, need * sizeof(uint16_t) + kMsgTail);
        if (e != hipSuccess) return e;
        p->msg_capacity = need;
    }
    p->launch.msg = p->d_msg;
    p->launch.grid = grid;
    return hipSuccess;
}

}  // namespace

int build_tasks(const std::vector<BatchJob> &jobs, const std::vector<int> &job_cw, int lds_cap,
                TaskSet &ts) {
    auto cost = [&](int j) { return (long)jobs[j].E * jobs[j].Z; };
    std::vector<WaveTask> waves;
    for (size_t j = 0; j < jobs.size(); ++j) {
        const BatchJob &jb = jobs[j];
        if (jb.Z <= kWaveLanes) {
            const int pairs = kWaveLanes / jb.Z, slots = 2 * pairs;
            int need = pairs * lds_bytes_i8_pair_post(jb.n_cols, jb.Z) + lds_flags_bytes_i8(pairs);
            need = (need + 15) & ~15;
            ts.wave_lds = std::max(ts.wave_lds, need);
            ts.wave_msg = std::max(ts.wave_msg, pairs * jb.E_pad * jb.Z);
            for (int f = 0; f < job_cw[j]; f += slots)
                waves.push_back(WaveTask{(int)j, f, std::min(slots, job_cw[j] - f), 0});
        } else if (jb.split && jb.Z > kBatchRowPairZ) {
            // one codeword per task on Z/2 lanes (row pairs)
            const int Zh = jb.Z / 2;
            ts.lds = std::max(ts.lds, lds_bytes_i8_pair_post(jb.n_cols, Zh) + lds_flags_bytes_i8(1));
            ts.msg_per_block = std::max(ts.msg_per_block, jb.E_pad * Zh);
            for (int f = 0; f < job_cw[j]; ++f) ts.tasks.push_back(BatchTask{(int)j, f, 1, -1});
            ts.row_pairs = true;
        } else {
            // jb.slots codewords per task, or one pair per task when split
            // (the workgroup's other pair slots stay idle)
            const int pairs = jb.slots / 2, per = jb.split ? 2 : jb.slots;
            ts.lds = std::max(ts.lds, pairs * lds_bytes_i8_pair_post(jb.n_cols, jb.Z) +
                                          lds_flags_bytes_i8(pairs));
            ts.msg_per_block = std::max(ts.msg_per_block, pairs * jb.E_pad * jb.Z);
            for (int f = 0; f < job_cw[j]; f += per)
                ts.tasks.push_back(BatchTask{(int)j, f, std::min(per, job_cw[j] - f), 0});
        }
    }
    // Longest first (larger lifts and more rows), so that the tail of the
    // persistent loop holds the short ones; wave tasks of similar length
    // share a bundle.
    std::stable_sort(waves.begin(), waves.end(),
                     [&](const WaveTask &a, const WaveTask &b) { return cost(a.job) > cost(b.job); });
    std::vector<long> task_cost;
    for (const BatchTask &t : ts.tasks) task_cost.push_back(cost(t.job));
    for (size_t i = 0; i < waves.size(); i += kWavesPerBlock) {
        const int nw = (int)std::min<size_t>(kWavesPerBlock, waves.size() - i);
        ts.tasks.push_back(BatchTask{-1, (int)i, 0, nw});
        task_cost.push_back(cost(waves[i].job));
    }
    ts.waves = std::move(waves);
    if (!ts.waves.empty()) {
        ts.lds = std::max(ts.lds, kWavesPerBlock * ts.wave_lds);
        ts.msg_per_block = std::max(ts.msg_per_block, kWavesPerBlock * ts.wave_msg);
    }
    std::vector<int> order(ts.tasks.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return task_cost[a] > task_cost[b]; });
    std::vector<BatchTask> sorted;
    for (int i : order) sorted.push_back(ts.tasks[i]);
    ts.tasks = std::move(sorted);
    if (ts.lds > lds_cap || ts.tasks.empty()) return LDPC_EINVAL;
    return LDPC_OK;
}

// Fills the job table from the registered graphs; called under the graph
// registry lock by ldpc_plan_create.
int plan_build(Plan *p, const std::vector<BatchJob> &jobs, const std::vector<int> &job_cw,
               int lanes, int max_iter, int early_exit, int beta, int offset, int wmax,
               int lds_cap, hipStream_t stream) {
    TaskSet ts;
    const int rc = build_tasks(jobs, job_cw, lds_cap, ts);
    if (rc != LDPC_OK) return rc;
    const std::vector<BatchTask> &tasks = ts.tasks;
    const int lds = ts.lds, msg_per_block = ts.msg_per_block;
    hipError_t e;
    if ((e = hipMalloc(&p->d_tasks, sizeof(BatchTask) * std::max<size_t>(tasks.size(), 1))) !=
            hipSuccess ||
        (e = hipMalloc(&p->d_jobs, sizeof(BatchJob) * jobs.size())) != hipSuccess ||
        (e = hipMalloc(&p->d_waves, sizeof(WaveTask) * std::max<size_t>(ts.waves.size(), 1))) !=
            hipSuccess ||
        (e = hipMalloc(&p->d_counter, sizeof(unsigned))) != hipSuccess ||
        (!ts.waves.empty() &&
         (e = hipMemcpyAsync(p->d_waves, ts.waves.data(), sizeof(WaveTask) * ts.waves.size(),
                             hipMemcpyHostToDevice, stream)) != hipSuccess) ||
        (e = hipMemcpyAsync(p->d_tasks, tasks.data(), sizeof(BatchTask) * tasks.size(),
                            hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (e = hipMemcpyAsync(p->d_jobs, jobs.data(), sizeof(BatchJob) * jobs.size(),
                            hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess) {
        note_hip_error("plan tables", e);
        return e == hipErrorOutOfMemory ? LDPC_ENOMEM : LDPC_EHIP;
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (p->cus < 1) p->cus = 1;
    p->max_per_cu = std::max(1, std::min(8, lds_cap / std::max(lds, 1)));
    BatchLaunch &b = p->launch;
    b.row_pairs = ts.row_pairs ? 1 : 0;
    b.tasks = p->d_tasks;
    b.jobs = p->d_jobs;
    b.waves = p->d_waves;
    b.wave_lds = ts.wave_lds;
    b.wave_msg = ts.wave_msg;
    b.n_tasks = (int)tasks.size();
    b.counter = p->d_counter;
    b.msg_per_block = msg_per_block;
    b.max_iter = max_iter;
    b.early_exit = early_exit;
    b.beta = beta;
    b.offset = offset;
    b.lanes = lanes;
    b.lds = lds;
    b.wmax = wmax;
    // default grid: as many workgroups as LDS allows on every CU, but no
    // more than there are tasks
    const int grid = std::max(1, std::min(b.n_tasks, p->cus * p->max_per_cu));
    e = size_messages(p, grid);
    if (e != hipSuccess) {
        note_hip_error("plan message workspace", e);
        return e == hipErrorOutOfMemory ? LDPC_ENOMEM : LDPC_EHIP;
    }
    return LDPC_OK;
}

// Times each candidate grid (1..max_per_cu workgroups per CU) on the
// plan's own work and keeps the fastest.
int plan_autotune(Plan *p, hipStream_t stream) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LDPC_EHIP;
    float best = 1e30f;
    int best_grid = p->launch.grid;
    for (int per = 1; per <= p->max_per_cu; ++per) {
        const int grid = std::max(1, std::min(p->launch.n_tasks, p->cus * per));
        if (size_messages(p, grid) != hipSuccess) break;
        float t = 0.0f;
        for (int rep = 0; rep < 3; ++rep) {
            (void)hipEventRecord(e0, stream);
            if (launch_decode_batch(p->launch, stream) != hipSuccess) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return LDPC_EHIP;
            }
            (void)hipEventRecord(e1, stream);
            (void)hipEventSynchronize(e1);
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) t += ms;  // first run warms up
        }
        t /= 2.0f;
        if (t < best) {
            best = t;
            best_grid = grid;
        }
        if (grid >= p->launch.n_tasks) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (size_messages(p, best_grid) != hipSuccess) return LDPC_ENOMEM;
    p->tuned_ms = best;
    return LDPC_OK;
}

int plan_capture(Plan *p) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return LDPC_EHIP;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t el = launch_decode_batch(p->launch, s);
        e = hipStreamEndCapture(s, &p->graph);
        if (el != hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(s);
    if (e != hipSuccess) {
        note_hip_error("plan graph capture", e);
        return LDPC_EHIP;
    }
    return LDPC_OK;
}

int plan_launch(Plan *p, hipStream_t stream) {
    const hipError_t e = p->exec ? hipGraphLaunch(p->exec, stream)
                                 : launch_decode_batch(p->launch, stream);
    if (e != hipSuccess) {
        note_hip_error("plan launch", e);
        return LDPC_EHIP;
    }
    return LDPC_OK;
}

void plan_destroy(Plan *p) { free_plan(p); }

namespace {
// Device memory layout of a one-shot asynchronous batch launch:
// tasks | jobs | wave tasks | counter | messages (256-aligned).
struct AsyncLayout {
    int grid = 1;
    size_t tb = 0, jbytes = 0, wbytes = 0, o_waves = 0, o_counter = 0, o_msg = 0, total = 0;
};

AsyncLayout async_layout(const TaskSet &ts, size_t n_jobs, int lds_cap) {
    AsyncLayout L;
    int dev = 0, cus = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int per_cu = std::max(1, std::min(8, lds_cap / std::max(ts.lds, 1)));
    L.grid = std::max(1, std::min((int)ts.tasks.size(), std::max(cus, 1) * per_cu));
    L.tb = sizeof(BatchTask) * ts.tasks.size();
    L.jbytes = sizeof(BatchJob) * n_jobs;
    L.wbytes = sizeof(WaveTask) * ts.waves.size();
    L.o_waves = L.tb + L.jbytes;
    L.o_counter = (L.o_waves + L.wbytes + 255) & ~(size_t)255;
    L.o_msg = L.o_counter + 256;
    L.total = L.o_msg + (size_t)L.grid * ts.msg_per_block * sizeof(uint16_t) + kMsgTail;
    return L;
}
}  // namespace

int batch_async_bytes(const std::vector<BatchJob> &jobs, const std::vector<int> &job_cw,
                      int lds_cap, size_t *bytes) {
    TaskSet ts;
    const int rc = build_tasks(jobs, job_cw, lds_cap, ts);
    if (rc != LDPC_OK) return rc;
    *bytes = async_layout(ts, jobs.size(), lds_cap).total;
    return LDPC_OK;
}

namespace {

// Device buffers of asynchronous launches of at most kArenaMax bytes, one
// per (device, stream), reused from launch to launch: a stream-ordered free
// costs about 25 us of host time per launch, a third of a small launch's
// host path. Launches on one stream are ordered by the stream; the event
// recorded after each use also orders a later use from another stream that
// was given the same handle. A buffer grows to the largest such launch on
// its stream and is kept until the process ends.
constexpr size_t kArenaMax = size_t(32) << 20;
struct Arena {
    uint8_t *buf = nullptr;
    size_t bytes = 0;
    hipEvent_t used = nullptr;  // recorded after the last launch that used buf
};
std::mutex g_arena_mu;
std::map<std::pair<int, hipStream_t>, Arena> g_arenas;

// Makes A hold at least `need` bytes for a launch enqueued next on `stream`
// (caller holds g_arena_mu).
hipError_t arena_acquire(Arena &A, size_t need, hipStream_t stream) {
    hipError_t e = hipSuccess;
    if (!A.used) e = hipEventCreateWithFlags(&A.used, hipEventDisableTiming);
    else e = hipStreamWaitEvent(stream, A.used, 0);
    if (e != hipSuccess || A.bytes >= need) return e;
    if (A.buf) {
        e = hipFreeAsync(A.buf, stream);
        A.buf = nullptr;
        A.bytes = 0;
        if (e != hipSuccess) return e;
    }
    size_t cap = size_t(1) << 16;
    while (cap < need) cap <<= 1;
    e = hipMallocAsync(reinterpret_cast<void **>(&A.buf), cap, stream);
    if (e == hipSuccess) A.bytes = cap;
    return e;
}

}  // namespace

// One launch over `jobs` with every buffer stream-ordered on `stream`: the
// tables and message regions come from the stream's reused buffer (launches
// of at most kArenaMax bytes) or from hipMallocAsync and hipFreeAsync, and
// are filled and used by the persistent kernel, all without blocking the
// host. Returns the device bytes the launch holds while in flight.
int batch_async(const std::vector<BatchJob> &jobs, const std::vector<int> &job_cw, int lanes,
                int max_iter, int early_exit, int wmax, int lds_cap, hipStream_t stream,
                size_t *bytes_in_flight) {
    TaskSet ts;
    const int rc = build_tasks(jobs, job_cw, lds_cap, ts);
    if (rc != LDPC_OK) return rc;
    const std::vector<BatchTask> &tasks = ts.tasks;
    const int lds = ts.lds, msg_per_block = ts.msg_per_block;
    const AsyncLayout lay = async_layout(ts, jobs.size(), lds_cap);
    const int grid = lay.grid;
    const size_t tb = lay.tb, jbytes = lay.jbytes;
    const size_t o_waves = lay.o_waves, o_counter = lay.o_counter, o_msg = lay.o_msg;
    const size_t total = lay.total;
    uint8_t *buf = nullptr;
    const bool pooled = total <= kArenaMax;
    std::unique_lock<std::mutex> lk(g_arena_mu, std::defer_lock);
    Arena *A = nullptr;
    hipError_t e = hipSuccess;
    if (pooled) {
        int dev = 0;
        e = hipGetDevice(&dev);
        lk.lock();
        A = &g_arenas[{dev, stream}];
        if (e == hipSuccess) e = arena_acquire(*A, total, stream);
        buf = A->buf;
    } else {
        e = hipMallocAsync(reinterpret_cast<void **>(&buf), total, stream);
    }
    if (e != hipSuccess) {
        note_hip_error(pooled ? "batch buffer" : "hipMallocAsync(batch)", e);
        return e == hipErrorOutOfMemory ? LDPC_ENOMEM : LDPC_EHIP;
    }
    BatchLaunch b{};
    b.tasks = reinterpret_cast<BatchTask *>(buf);
    b.jobs = reinterpret_cast<BatchJob *>(buf + tb);
    b.waves = reinterpret_cast<WaveTask *>(buf + o_waves);
    b.wave_lds = ts.wave_lds;
    b.wave_msg = ts.wave_msg;
    b.counter = reinterpret_cast<unsigned *>(buf + o_counter);
    b.msg = reinterpret_cast<uint16_t *>(buf + o_msg);
    b.n_tasks = (int)tasks.size();
    b.msg_per_block = msg_per_block;
    b.max_iter = max_iter;
    b.early_exit = early_exit;
    b.beta = 96;
    b.offset = 0;
    b.grid = grid;
    b.lanes = lanes;
    b.lds = lds;
    b.wmax = wmax;
    // The task, job and wave-task tables and the zeroed task counter as one
    // host image, moved by one copy (the counter needs no reset kernel).
    // Pageable source: the runtime has staged it when the call returns.
    std::vector<uint8_t> img(o_counter + sizeof(unsigned), 0);
    std::memcpy(img.data(), tasks.data(), tb);
    std::memcpy(img.data() + tb, jobs.data(), jbytes);
    if (!ts.waves.empty())
        std::memcpy(img.data() + o_waves, ts.waves.data(), sizeof(WaveTask) * ts.waves.size());
    e = hipMemcpyAsync(buf, img.data(), img.size(), hipMemcpyHostToDevice, stream);
    b.counter_zeroed = 1;
    b.row_pairs = ts.row_pairs ? 1 : 0;
    if (e == hipSuccess) e = launch_decode_batch(b, stream);
    const hipError_t ef = pooled ? hipEventRecord(A->used, stream) : hipFreeAsync(buf, stream);
    if (e != hipSuccess) {
        note_hip_error("batch_async", e);
        return LDPC_EHIP;
    }
    if (ef != hipSuccess) {
        note_hip_error(pooled ? "hipEventRecord(batch buffer)" : "hipFreeAsync(batch)", ef);
        return LDPC_EHIP;
    }
    if (bytes_in_flight) *bytes_in_flight = total;
    return LDPC_OK;
}

Plan *plan_new() { return new Plan(); }

void plan_info(const Plan *p, int *grid, int *n_tasks, float *tuned_ms) {
    if (grid) *grid = p->launch.grid;
    if (n_tasks) *n_tasks = p->launch.n_tasks;
    if (tuned_ms) *tuned_ms = p->tuned_ms;
}

}  // namespace ldpc
