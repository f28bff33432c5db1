// Serving queue (host side): a ring of task descriptors, a published count,
// a stop request and per-task completion flags in pinned host memory, read
// and written by a persistent decode kernel (serve_kernel) while the host
// keeps appending. The host relaunches the kernel whenever tasks are pending
// and the previous launch has ended (the kernel leaves by itself once idle).
#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/ldpc.h"
#include "ldpc_internal.h"

namespace ldpc {
int serve_job(const ldpc_job &job, BatchJob &bj, int &wmax);  // ldpc_api.hip
}

using namespace ldpc;

struct ldpc_server {
    int dev = 0;
    int capacity = 0;
    ServeLaunch launch{};
    ServeTask *ring = nullptr;   // pinned
    unsigned *ctl = nullptr;     // pinned: [0] published, [1] stop
    unsigned *done = nullptr;    // pinned [capacity]
    unsigned *dev_ctl = nullptr; // device: [0] claimed, [1] published mirror, [2] stop mirror
    uint16_t *msg = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ended = nullptr;
    bool launched = false;
    unsigned published = 0;      // tasks written to the ring
    unsigned oldest = 0;         // every ticket below it has completed
    int launches = 0;
    std::mutex mu;
};

namespace {

constexpr bool kServerEnabled = false;

void server_free(ldpc_server *s) {
    if (s->ended) (void)hipEventDestroy(s->ended);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->msg) (void)hipFree(s->msg);
    if (s->dev_ctl) (void)hipFree(s->dev_ctl);
    if (s->done) (void)hipHostFree(s->done);
    if (s->ctl) (void)hipHostFree(s->ctl);
    if (s->ring) (void)hipHostFree(s->ring);
    delete s;
}

inline unsigned host_load(const unsigned *p) {
    return __atomic_load_n(p, __ATOMIC_ACQUIRE);
}

// Advances s->oldest past completed tickets (caller holds s->mu).
void retire(ldpc_server *s) {
    while (s->oldest != s->published &&
           host_load(s->done + s->oldest % (unsigned)s->capacity) == s->oldest + 1u)
        ++s->oldest;
}

// Launches the persistent kernel if tasks are outstanding and no launch is
// running (caller holds s->mu).
int ensure_running(ldpc_server *s) {
    retire(s);
    if (s->oldest == s->published) return LDPC_OK;
    if (s->launched) {
        const hipError_t q = hipEventQuery(s->ended);
        if (q == hipErrorNotReady) return LDPC_OK;
        if (q != hipSuccess) {
            note_hip_error("serve_kernel", q);
            return LDPC_EHIP;
        }
    }
    (void)hipSetDevice(s->dev);
    // clear the device stop mirror left by an earlier stop (a one-lane store
    // kernel is not needed: nothing is captured here)
    hipError_t e = hipMemsetAsync(s->dev_ctl + 2, 0, sizeof(unsigned), s->stream);
    if (e == hipSuccess) e = launch_serve(s->launch, s->stream);
    if (e == hipSuccess) e = hipEventRecord(s->ended, s->stream);
    if (e != hipSuccess) {
        note_hip_error("serve relaunch", e);
        return LDPC_EHIP;
    }
    s->launched = true;
    ++s->launches;
    return LDPC_OK;
}

}  // namespace

extern "C" {

int ldpc_server_create(int capacity, int grid, int max_iter, int early_exit, int idle_polls,
                       ldpc_server **out) {
    // Switched off: on MI355X the persistent queue kernel did not finish
    // (no task completed, and it did not leave on the stop request) and the
    // cause has not been found. The rest of this file is kept, unreachable,
    // for that investigation; nothing is allocated or launched here.
    if (!kServerEnabled) return LDPC_EINVAL;
    if (!out || capacity < 1 || capacity > (1 << 20) || grid < 0 || max_iter < 1 ||
        max_iter > LDPC_MAX_ITER || idle_polls < 0)
        return LDPC_EINVAL;
    ldpc_server *s = new ldpc_server();
    hipError_t e = hipGetDevice(&s->dev);
    int cus = 0;
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->dev);
    const int decode_wgs = grid > 0 ? grid : std::max(1, cus);
    // message region of a workgroup: any shape the queue takes (at most
    // floor(kBatchLanes / Z) pairs of E_pad * Z pair words, row weights up
    // to 20, so E_pad <= LDPC_MAX_ROWS * 20)
    const int msg_per_block = kServeMsgPerBlock;
    s->capacity = capacity;
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&s->ring), sizeof(ServeTask) * capacity,
                          hipHostMallocCoherent);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&s->ctl), 64, hipHostMallocCoherent);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&s->done), sizeof(unsigned) * capacity,
                          hipHostMallocCoherent);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&s->dev_ctl), 256);
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void **>(&s->msg),
                      (size_t)decode_wgs * msg_per_block * sizeof(uint16_t) + kMsgTail);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ended, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemset(s->dev_ctl, 0, 256);
    if (e != hipSuccess) {
        note_hip_error("ldpc_server_create", e);
        server_free(s);
        return e == hipErrorOutOfMemory ? LDPC_ENOMEM : LDPC_EHIP;
    }
    s->ctl[0] = 0;
    s->ctl[1] = 0;
    for (int i = 0; i < capacity; ++i) s->done[i] = 0;
    ServeLaunch &L = s->launch;
    L.ring = s->ring;
    L.capacity = capacity;
    L.host_ctl = s->ctl;
    L.done = s->done;
    L.dev_ctl = s->dev_ctl;
    L.msg = s->msg;
    L.msg_per_block = msg_per_block;
    L.max_iter = max_iter;
    L.early_exit = early_exit ? 1 : 0;
    L.grid = decode_wgs + 1;
    L.lds = kServeLds;
    L.idle_polls = idle_polls > 0 ? idle_polls : 4000;
    if (L.lds > max_lds_bytes()) {
        server_free(s);
        return LDPC_EINVAL;
    }
    *out = s;
    return LDPC_OK;
}

int ldpc_server_submit(ldpc_server *s, const ldpc_job *job, unsigned *first_ticket,
                       int *n_tasks) {
    if (!s || !job) return LDPC_EINVAL;
    BatchJob bj{};
    int wmax = 0;
    const int rc = serve_job(*job, bj, wmax);
    if (rc != LDPC_OK) return rc;
    const int per = bj.slots;  // codewords per task: the workgroup's pairs
    const int nt = (job->n_cw + per - 1) / per;
    std::lock_guard<std::mutex> lk(s->mu);
    retire(s);
    if ((long)(s->published - s->oldest) + nt > s->capacity) return LDPC_ENOMEM;
    const unsigned first = s->published;
    for (int i = 0; i < nt; ++i) {
        ServeTask &t = s->ring[(first + i) % (unsigned)s->capacity];
        t.job = bj;
        t.first = i * per;
        t.n = std::min(per, job->n_cw - i * per);
        t.ticket = first + i;
        t.pad = 0;
    }
    s->published = first + nt;
    // descriptors before the count that publishes them
    std::atomic_thread_fence(std::memory_order_release);
    __atomic_store_n(s->ctl, s->published, __ATOMIC_RELEASE);
    if (first_ticket) *first_ticket = first;
    if (n_tasks) *n_tasks = nt;
    return ensure_running(s);
}

int ldpc_server_done(ldpc_server *s, unsigned ticket) {
    if (!s) return LDPC_EINVAL;
    return host_load(s->done + ticket % (unsigned)s->capacity) == ticket + 1u ? 1 : 0;
}

int ldpc_server_pump(ldpc_server *s, int *outstanding, int *launches) {
    if (!s) return LDPC_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    const int rc = ensure_running(s);
    if (outstanding) *outstanding = (int)(s->published - s->oldest);
    if (launches) *launches = s->launches;
    return rc;
}

int ldpc_server_destroy(ldpc_server *s) {
    if (!s) return LDPC_EINVAL;
    int rc = LDPC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        __atomic_store_n(s->ctl + 1, 1u, __ATOMIC_RELEASE);
        if (s->launched) {
            const hipError_t e = hipEventSynchronize(s->ended);
            if (e != hipSuccess) {
                note_hip_error("ldpc_server_destroy", e);
                rc = LDPC_EHIP;
            }
        }
    }
    server_free(s);
    return rc;
}

}  // extern "C"
