// C-ABI front end of the decoder library: argument checks, the graph
// registry (host copies plus lazily uploaded per-device tables), launch
// configuration and error reporting. Declarations and contracts:
// include/ldpc.h.
#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/ldpc.h"
#include "ldpc_internal.h"

namespace ldpc {
namespace {

struct HostGraph {
    int bg = 0, Z = 0, m_rows = 0, kb = 0;
    std::vector<int32_t> row_ptr;
    std::vector<int16_t> col, shift;
};

struct DevTables {
    int32_t *row_ptr = nullptr;   // [m_rows + 1]
    uint32_t *meta = nullptr;     // [E_full + kMetaPad] row-pair layout
    uint32_t *meta_row = nullptr; // [E_full + kMetaPad] one row per lane
    uint32_t *meta_i8 = nullptr;  // [E_full + kMetaPad] int8 codeword pairs
    uint32_t *meta_i8rp = nullptr;  // [E_full + kMetaPad] int8 row pairs
    int32_t *row_pad = nullptr;   // [m_rows + 1] prefix of even-padded row weights
};

std::mutex g_mu;
std::map<std::pair<int, int>, HostGraph> g_graphs;                 // (bg, Z)
std::map<std::tuple<int, int, int>, DevTables> g_dev;             // (device, bg, Z)
std::map<int, int> g_lds;                                          // device -> bytes
std::mutex g_lds_mu;
int g_last_hip = 0;
thread_local char g_msg[256] = "";

int hip_fail(hipError_t e, const char *where = "HIP call") {
    note_hip_error(where, e);
    return e == hipErrorOutOfMemory ? LDPC_ENOMEM : LDPC_EHIP;
}

bool valid_lift(int Z) { return Z >= 8 && Z <= LDPC_MAX_Z && Z % 8 == 0; }

void free_tables(DevTables &t) {
    if (t.row_ptr) (void)hipFree(t.row_ptr);
    if (t.meta) (void)hipFree(t.meta);
    if (t.meta_row) (void)hipFree(t.meta_row);
    if (t.meta_i8) (void)hipFree(t.meta_i8);
    if (t.meta_i8rp) (void)hipFree(t.meta_i8rp);
    if (t.row_pad) (void)hipFree(t.row_pad);
    t.row_ptr = nullptr;
    t.meta = nullptr;
    t.meta_row = nullptr;
    t.meta_i8 = nullptr;
    t.meta_i8rp = nullptr;
    t.row_pad = nullptr;
}

// Row starts of the int8 device message layout: each row's weight rounded
// up to even, so that a lane's messages of a row fill whole dwords.
std::vector<int32_t> padded_row_ptr(const HostGraph &g) {
    std::vector<int32_t> rp(g.row_ptr.size(), 0);
    for (size_t r = 0; r + 1 < g.row_ptr.size(); ++r) {
        const int w = g.row_ptr[r + 1] - g.row_ptr[r];
        rp[r + 1] = rp[r] + w + (w & 1);
    }
    return rp;
}

// Device tables of graph (bg, Z) on the current device, uploaded on first
// use unless `upload` is false (then LDPC_ENOGRAPH when they are not yet
// resident); caller holds g_mu.
int tables_for(const HostGraph &g, DevTables **out, bool upload = true) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    auto key = std::make_tuple(dev, g.bg, g.Z);
    auto it = g_dev.find(key);
    if (it != g_dev.end()) {
        *out = &it->second;
        return LDPC_OK;
    }
    if (!upload) return LDPC_ENOGRAPH;
    const int Zh = g.Z / 2;
    const int E = g.row_ptr.back();
    std::vector<uint32_t> meta(E + kMetaPad, 0u), meta_row(E + kMetaPad, 0u),
        meta_i8(E + kMetaPad, 0u), meta_i8rp(E + kMetaPad, 0u);
    for (int e2 = 0; e2 < E; ++e2) {
        meta[e2] = pack_meta(g.col[e2], g.shift[e2], Zh);
        meta_row[e2] = pack_meta_row(g.col[e2], g.shift[e2], g.Z);
        meta_i8[e2] = pack_meta_i8(g.col[e2], g.shift[e2], g.Z);
        meta_i8rp[e2] = pack_meta_i8rp(g.col[e2], g.shift[e2], Zh);
    }
    const std::vector<int32_t> row_pad = padded_row_ptr(g);
    DevTables t;
    if ((e = hipMalloc(&t.row_ptr, sizeof(int32_t) * g.row_ptr.size())) != hipSuccess ||
        (e = hipMalloc(&t.row_pad, sizeof(int32_t) * row_pad.size())) != hipSuccess ||
        (e = hipMemcpy(t.row_pad, row_pad.data(), sizeof(int32_t) * row_pad.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMalloc(&t.meta, sizeof(uint32_t) * meta.size())) != hipSuccess ||
        (e = hipMalloc(&t.meta_row, sizeof(uint32_t) * meta_row.size())) != hipSuccess ||
        (e = hipMalloc(&t.meta_i8, sizeof(uint32_t) * meta_i8.size())) != hipSuccess ||
        (e = hipMalloc(&t.meta_i8rp, sizeof(uint32_t) * meta_i8rp.size())) != hipSuccess ||
        (e = hipMemcpy(t.row_ptr, g.row_ptr.data(), sizeof(int32_t) * g.row_ptr.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(t.meta, meta.data(), sizeof(uint32_t) * meta.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(t.meta_row, meta_row.data(), sizeof(uint32_t) * meta_row.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(t.meta_i8, meta_i8.data(), sizeof(uint32_t) * meta_i8.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(t.meta_i8rp, meta_i8rp.data(), sizeof(uint32_t) * meta_i8rp.size(),
                       hipMemcpyHostToDevice)) != hipSuccess) {
        free_tables(t);
        return hip_fail(e);
    }
    *out = &(g_dev[key] = t);
    return LDPC_OK;
}

int sub_sizes(const HostGraph &g, int rows, int *K, int *T, int *Nc, int *E) {
    if (rows < 4 || rows > g.m_rows) return LDPC_EINVAL;
    const int n = g.kb + rows;
    if (K) *K = g.kb * g.Z;
    if (T) *T = (n - 2) * g.Z;
    if (Nc) *Nc = n * g.Z;
    if (E) *E = g.row_ptr[rows];
    return LDPC_OK;
}

// Argument checks, graph look-up and launch shape of one decode call, shared
// by ldpc_decode_ex and ldpc_decode_noalloc (upload = false: the graph's
// device tables must already be resident; nothing is allocated on the device
// or the host heap). msg_bytes: the device message buffer the launch needs
// unless msg_in_lds.
// Launch configurations chosen by ldpc_tune, per (bg, Z, rows, n_cw rounded
// up to a power of two, early exit).
struct Tuned {
    int lanes_per_row, cw_per_block, msg_placement, schedule, pairing;
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int>, Tuned> g_tuned;

int pow2_bucket(int n) {
    int b = 1;
    while (b < n && b < (1 << 30)) b <<= 1;
    return b;
}

// Compute units of the current device, 0 if the runtime cannot say.
int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return cus;
}

// Whether an int8 call decodes with the row-pair kernel: on request
// (LDPC_PAIR_ROWS; the static schedule and one lane per row, else the
// caller gets LDPC_EINVAL), or by default (one lane per row, the static
// schedule, the default packing and message placement):
// * at lifts above 256 with early exit (but for rows of weight at most 10
//   not for five to eight codewords per CU), and for at most one codeword per
//   CU (a codeword pair's 2Z lanes would put two waves on some SIMDs of a
//   CU, where one codeword's Z/2 lanes leave every wave a SIMD of its own);
// * at lifts 16 to 256 with early exit for more than four codewords per CU:
//   codeword pairs then need more than one round of workgroups per CU, and
//   a workgroup of codeword pairs runs until the slowest of its codewords
//   has converged, where row-pair workgroups of one to four codewords leave
//   as soon as theirs have (4,096 codewords: 30 to 45 % less time at lifts
//   32 to 128). Up to 1,024 codewords, codeword pairs spread over the CUs
//   were as fast or faster (row pairs spend two more instructions per edge).
// Sets g_msg when a request cannot be met.
// Default codewords per row-pair workgroup: up to Z = 128 the most whose
// Z/2 lanes fit in one wave, at most four (no barrier then couples waves;
// four at Z = 16 to 32, two to 64, one to 128), two to Z = 256 and one above.
// Measured on 4,096-codeword early-exit batches: fuller waves or larger
// workgroups were not faster (at Z = 16 four codewords per wave beat eight;
// at Z = 208 three per workgroup were a third slower than two).
int row_pair_default_cpw(int Z) {
    const int Zh = Z / 2;
    if (Z > 256) return 1;
    if (Z > 128) return 2;
    return std::max(1, std::min(4, 64 / Zh));
}

bool use_row_pairs(const ldpc_args *a, int Z, int wmax) {
    const bool can = a->schedule == LDPC_SCHED_STATIC && a->lanes_per_row <= 1;
    if (a->pairing == LDPC_PAIR_ROWS) {
        if (!can)
            snprintf(g_msg, sizeof(g_msg),
                     "row pairs need the static schedule and one lane per row");
        return can;
    }
    if (a->pairing != LDPC_PAIR_AUTO || !can || a->cw_per_block != 0 ||
        a->msg_placement != LDPC_MSG_AUTO || Z < 16)
        return false;
    const int cus = device_cus();
    if (Z > 256) {
        if (a->n_cw <= cus) return true;
        if (!a->early_exit) return false;
        // Rows of weight 10 or less (BG2-shaped), five to eight codewords per
        // CU: codeword pairs measured faster (2,048 codewords at Z = 288 and
        // 384: 15 to 25 % less time at 0.5 to 1.5 dB), where at four per CU
        // (1,024) row pairs were up to 10 % faster and at 16 the two were
        // within 13 % either way depending on the Eb/N0.
        return !(wmax <= 10 && a->n_cw > 4 * cus && a->n_cw <= 8 * cus);
    }
    return a->early_exit && a->n_cw > 4 * cus;
}

int prepare_decode(const ldpc_args *a0, bool upload, DecodeLaunch &p, bool &msg_in_lds,
                   size_t &msg_bytes, bool allow_refill = false) {
    if (!a0) return LDPC_EINVAL;
    // an int8 call with every launch knob at its default takes the tuned
    // configuration of its shape and batch size, if ldpc_tune recorded one
    ldpc_args ar = *a0;
    if (ar.precision == LDPC_I8 && ar.lanes_per_row == 0 && ar.cw_per_block == 0 &&
        ar.msg_placement == LDPC_MSG_AUTO && ar.schedule == LDPC_SCHED_STATIC &&
        ar.max_workgroups == 0 && ar.pairing == LDPC_PAIR_AUTO) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(std::make_tuple(ar.bg, ar.Z, ar.rows, pow2_bucket(ar.n_cw),
                                               ar.early_exit ? 1 : 0));
        if (it != g_tuned.end()) {
            ar.lanes_per_row = it->second.lanes_per_row;
            ar.cw_per_block = it->second.cw_per_block;
            ar.msg_placement = it->second.msg_placement;
            ar.schedule = it->second.schedule;
            ar.pairing = it->second.pairing;
        }
    }
    const ldpc_args *a = &ar;
    if ( a->n_cw < 1 || a->max_iter < 1 || a->max_iter > LDPC_MAX_ITER || !a->llr_in ||
        (reinterpret_cast<uintptr_t>(a->llr_in) & 3u) != 0 ||
        !a->out_bits || !a->out_iters || (a->precision != LDPC_I8 && a->precision != LDPC_F16) ||
        a->beta_q < 0 || a->beta_q > 255 || a->offset_q < 0 || a->offset_q > 127 ||
        (a->wq && a->wq_iters < 1) || (a->wh && a->wh_iters < 1) || a->cw_per_block < 0 ||
        a->msg_placement < LDPC_MSG_AUTO || a->msg_placement > LDPC_MSG_DEVICE ||
        (a->lanes_per_row != 0 && a->lanes_per_row != 1 && a->lanes_per_row != 2 &&
         a->lanes_per_row != 4) ||
        (a->schedule != LDPC_SCHED_STATIC && a->schedule != LDPC_SCHED_PERSISTENT) ||
        a->max_workgroups < 0 || a->pairing < LDPC_PAIR_AUTO || a->pairing > LDPC_PAIR_ROWS ||
        (a->pairing == LDPC_PAIR_ROWS && a->precision != LDPC_I8))
        return LDPC_EINVAL;
    g_msg[0] = '\0';
    int lds_cap = 0;
    const uint32_t *meta_rp = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_graphs.find({a->bg, a->Z});
        if (it == g_graphs.end()) return LDPC_ENOGRAPH;
        const HostGraph &g = it->second;
        int E = 0;
        if (sub_sizes(g, a->rows, nullptr, nullptr, nullptr, &E) != LDPC_OK) return LDPC_EINVAL;
        DevTables *t = nullptr;
        const int rc = tables_for(g, &t, upload);
        if (rc == LDPC_ENOGRAPH)
            snprintf(g_msg, sizeof(g_msg),
                     "graph (%d, %d) has no device tables on this device yet: decode it once "
                     "with ldpc_decode or ldpc_decode_ex first", a->bg, a->Z);
        if (rc != LDPC_OK) return rc;
        int wmax = 0, e_pad = 0;
        for (int r = 0; r < a->rows; ++r) {
            const int w = g.row_ptr[r + 1] - g.row_ptr[r];
            if (w > wmax) wmax = w;
            e_pad += w + (w & 1);
        }
        p.row_ptr = t->row_ptr;
        p.row_pad = t->row_pad;
        p.E_pad = e_pad;
        p.meta = a->precision == LDPC_I8 ? t->meta_i8 : t->meta;
        meta_rp = t->meta_i8rp;
        p.rows = a->rows;
        p.n_cols = g.kb + a->rows;
        p.kb = g.kb;
        p.Z = g.Z;
        p.E = E;
        p.wmax = wmax;
        p.groups = layer_groups(g.row_ptr.data(), g.col.data(), a->rows);
        p.alpha = a->lanes_per_row > 1 ? a->lanes_per_row : 1;
        if (p.alpha > 1) p.E_pad = ll_message_pair_words(g.row_ptr.data(), a->rows, p.alpha);
        if (a->precision == LDPC_F16) {
            // binary16: E_pad counts message record dwords per lane
            int rec = 0;
            for (int r = 0; r < a->rows; ++r) rec += f16_record_dwords(g.row_ptr[r + 1] - g.row_ptr[r]);
            p.E_pad = rec;
        }
        lds_cap = max_lds_bytes();
    }
    p.llr = a->llr_in;
    p.out_bits = a->out_bits;
    p.out_iters = a->out_iters;
    p.out_ok = a->out_ok;
    p.out_llr = a->out_llr;
    p.n_cw = a->n_cw;
    p.max_iter = a->max_iter;
    p.early_exit = a->early_exit ? 1 : 0;
    const int Zh = p.Z / 2;
    const bool i8 = a->precision == LDPC_I8;
    int cpw = 0;
    msg_in_lds = false;
    const bool rowpair = i8 && use_row_pairs(a, p.Z, p.wmax);
    if (a->pairing == LDPC_PAIR_ROWS && !rowpair) return LDPC_EINVAL;
    if (p.alpha > 1) {
        // Low-latency mapping: alpha lanes per check row, device-placed
        // messages, whole waves per chunk group (pairs * Z a multiple of 64).
        if (!i8 || a->msg_placement == LDPC_MSG_LDS || p.wmax > 20 ||
            p.wmax > kLLChunkMax * p.alpha)
            return LDPC_EINVAL;
        int pairs = (a->cw_per_block + 1) / 2;
        if (pairs == 0) {
            pairs = 1;
            while ((pairs * p.Z) % 64 != 0) ++pairs;
        }
        if ((pairs * p.Z) % 64 != 0 || p.alpha * pairs * p.Z > 1024 ||
            ll_lds_bytes(p.n_cols, p.Z, pairs, p.alpha) > lds_cap)
            return LDPC_EINVAL;
        cpw = 2 * pairs;
    } else if (rowpair) {
        // One codeword per Z/2 lanes (row pairs); messages in device memory,
        // or in LDS after each codeword's posteriors on request.
        p.rowpair = 1;
        p.meta = meta_rp;
        // By default the messages go to LDS for at most one codeword per CU
        // when every row has weight 10 or less and one codeword's state fits
        // (BG2-shaped at Z = 384: 28.8 against 32.3 us per iteration; with
        // weight-19 rows the separate 16-bit message accesses cancel it).
        msg_in_lds = a->msg_placement == LDPC_MSG_LDS ||
                     (a->msg_placement == LDPC_MSG_AUTO && a->cw_per_block == 0 &&
                      p.wmax <= 10 && a->n_cw <= device_cus() &&
                      lds_bytes_i8_pair(p.n_cols, p.E, Zh) + 16 <= lds_cap - 8);
        const int per_cw = (msg_in_lds ? lds_bytes_i8_pair(p.n_cols, p.E, Zh)
                                       : lds_bytes_i8_pair_post(p.n_cols, Zh)) + 16;
        cpw = a->cw_per_block > 0 ? a->cw_per_block : row_pair_default_cpw(p.Z);
        cpw = std::min(cpw, (lds_cap - 8) / per_cw);
        cpw = std::min(cpw, 768 / Zh);
        cpw = std::min(cpw, a->n_cw);
        if (cpw < 1) {
            snprintf(g_msg, sizeof(g_msg), "one codeword's row-pair state does not fit in LDS");
            return LDPC_EINVAL;
        }
    } else if (i8) {
        // Codewords go in pairs of Z lanes. Message placement: LDS when two
        // pairs' full state fits a CU, else device memory so that several
        // pairs share a CU.
        // per pair: its LDS state plus its four flag / index words
        const int full = lds_bytes_i8_pair(p.n_cols, p.E, p.Z) + 16;
        if (a->msg_placement == LDPC_MSG_LDS)
            msg_in_lds = true;
        else if (a->msg_placement == LDPC_MSG_DEVICE)
            msg_in_lds = false;
        else  // the persistent schedule places messages in device memory
            msg_in_lds = a->schedule != LDPC_SCHED_PERSISTENT && 2 * full + 8 <= lds_cap;
        const int per_pair = msg_in_lds ? full : lds_bytes_i8_pair_post(p.n_cols, p.Z) + 16;
        int pairs = (a->cw_per_block + 1) / 2;
        // Default: about 256 lanes per workgroup with the whole state in LDS,
        // else about 768 (two pairs per workgroup at the largest lift, one
        // workgroup per CU: measured as fast as three pairs per CU in steady
        // state, and with a finer tail for batches of a few thousand).
        // A batch of fewer pairs than that fills the device spreads them
        // over the CUs instead (eight codewords at Z = 256 in one
        // workgroup: 62 us per iteration against 41 on separate CUs).
        if (pairs == 0) {
            pairs = std::max(1, (msg_in_lds ? 256 : 768) / p.Z);
            const int cus = device_cus();
            if (cus > 0) {
                const int n_pairs = (a->n_cw + 1) / 2;
                pairs = std::min(pairs, std::max(1, (n_pairs + cus - 1) / cus));
            }
        }
        pairs = std::min(pairs, (lds_cap - 8) / per_pair);
        pairs = std::min(pairs, 768 / p.Z);
        pairs = std::min(pairs, (a->n_cw + 1) / 2);
        if (pairs < 1) return LDPC_EINVAL;  // a single pair does not fit
        cpw = 2 * pairs;
    } else {
        const int per_cw = lds_bytes_f16(p.n_cols, p.Z) + 4;
        cpw = a->cw_per_block;
        // Default: about 128 lanes (Z/2 per codeword) per workgroup.
        if (cpw == 0) cpw = std::max(1, 128 / Zh);
        cpw = std::min(cpw, lds_cap / per_cw);
        cpw = std::min(cpw, 512 / Zh);
        cpw = std::min(cpw, a->n_cw);
        if (cpw < 1) return LDPC_EINVAL;  // a single codeword does not fit
    }
    p.cpw = cpw;
    if (i8) {
        p.wq = a->wq;
        p.w_iters = a->wq_iters;
        p.beta = a->beta_q;
        p.offset = a->offset_q;
    } else {
        p.wh = a->wh;
        p.w_iters = a->wh_iters;
        p.beta = a->beta_h;
        p.offset = a->offset_h;
    }
    msg_bytes = msg_in_lds ? 0
                : p.rowpair ? (size_t)a->n_cw * p.E_pad * Zh * 2 + kMsgTail
                : i8 ? (((size_t)a->n_cw + 1) / 2) * p.E_pad * p.Z * 2 + kMsgTail
                     : (size_t)a->n_cw * p.E_pad * Zh * 4;
    // Persistent schedule: as many workgroups as run at once (LDS-bound:
    // one 768-lane workgroup per CU at the largest lifts), each with a
    // message region for its own pairs, then the codeword counter.
    p.refill = 0;
    p.grid = 0;
    p.counter = nullptr;
    if (a->schedule == LDPC_SCHED_PERSISTENT) {
        if (!allow_refill || !i8 || p.alpha != 1 || msg_in_lds || !a->early_exit || a->wq ||
            a->cw_per_block != 0) {
            snprintf(g_msg, sizeof(g_msg),
                     "the persistent schedule needs int8 with early exit, one lane per row, "
                     "device-placed messages, plain normalisation and the default packing "
                     "(and is not available to ldpc_decode_noalloc)");
            return LDPC_EINVAL;
        }
        const int pairs = cpw / 2;
        const int lds = pairs * lds_bytes_i8_pair_post(p.n_cols, p.Z) + lds_flags_bytes_i8(pairs);
        const int waves = (pairs * p.Z + 63) / 64;
        int dev = 0, cus = 1;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        // four waves per SIMD at most (the kernel's register budget)
        const int per_cu = std::max(1, std::min(lds_cap / std::max(lds, 1), 16 / waves));
        long grid = std::min<long>(((long)a->n_cw + cpw - 1) / cpw, (long)std::max(cus, 1) * per_cu);
        if (a->max_workgroups > 0) grid = std::min<long>(grid, a->max_workgroups);
        const size_t region = (size_t)pairs * p.E_pad * p.Z * 2;  // bytes
        p.refill = 1;
        p.grid = (int)grid;
        msg_bytes = (((size_t)grid * region + kMsgTail + 255) & ~(size_t)255) + 256;
    }
    return LDPC_OK;
}

// Static message scratch of ldpc_decode_noalloc: one copy per device,
// held until the process ends. In host code `scratch` names a host-side
// stand-in, not device memory: its device address is resolved per device
// with hipGetSymbolAddress and only that address is handed to kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_dev[64] = {};  // device ordinal -> address of its `scratch`

// Address of the current device's scratch (resolved once per device).
int scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return LDPC_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return LDPC_OK;
}

}  // namespace

void note_hip_error(const char *where, hipError_t e) {
    g_last_hip = (int)e;
    snprintf(g_msg, sizeof(g_msg), "%s: %s (%d)", where, hipGetErrorName(e), (int)e);
}

int max_lds_bytes() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    std::lock_guard<std::mutex> lk(g_lds_mu);
    auto it = g_lds.find(dev);
    if (it != g_lds.end()) return it->second;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess ||
        v <= 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
                hipSuccess ||
            v <= 0)
            v = 65536;
    }
    if (v > 163840) v = 163840;
    g_lds[dev] = v;
    return v;
}

}  // namespace ldpc

using namespace ldpc;

extern "C" {

int ldpc_set_graph(int bg, int Z, int m_rows, int kb, const int32_t *row_ptr, const int16_t *col,
                   const int16_t *shift) {
    if (bg < 1 || !valid_lift(Z) || m_rows < 4 || m_rows > LDPC_MAX_ROWS || kb < 2 ||
        kb + m_rows > LDPC_MAX_COLS || !row_ptr || !col || !shift || row_ptr[0] != 0)
        return LDPC_EINVAL;
    for (int r = 0; r < m_rows; ++r) {
        const int w = row_ptr[r + 1] - row_ptr[r];
        if (w < 2 || w > LDPC_MAX_ROW_WEIGHT) return LDPC_EINVAL;
        const int col_limit = kb + (r + 1 > 4 ? r + 1 : 4);
        for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
            if (col[e] < 0 || col[e] >= col_limit || shift[e] < 0 || shift[e] >= Z)
                return LDPC_EINVAL;
            if (e > row_ptr[r] && col[e] <= col[e - 1]) return LDPC_EINVAL;
        }
    }
    HostGraph g;
    g.bg = bg;
    g.Z = Z;
    g.m_rows = m_rows;
    g.kb = kb;
    const int E = row_ptr[m_rows];
    g.row_ptr.assign(row_ptr, row_ptr + m_rows + 1);
    g.col.assign(col, col + E);
    g.shift.assign(shift, shift + E);
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto it = g_dev.begin(); it != g_dev.end();) {
        if (std::get<1>(it->first) == bg && std::get<2>(it->first) == Z) {
            free_tables(it->second);
            it = g_dev.erase(it);
        } else {
            ++it;
        }
    }
    g_graphs[{bg, Z}] = std::move(g);
    return LDPC_OK;
}

// FNV-1a (64-bit) over the registered table serialised as little-endian
// int32 words: bg, Z, m_rows, kb, row_ptr[0..m_rows], col[0..E), shift[0..E).
int ldpc_graph_digest(int bg, int Z, uint64_t *out) {
    if (!out) return LDPC_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_graphs.find({bg, Z});
    if (it == g_graphs.end()) return LDPC_ENOGRAPH;
    const HostGraph &g = it->second;
    uint64_t h = 0xcbf29ce484222325ull;
    auto word = [&h](int32_t v) {
        const uint32_t u = (uint32_t)v;
        for (int b = 0; b < 4; ++b) {
            h ^= (u >> (8 * b)) & 0xFFu;
            h *= 0x100000001b3ull;
        }
    };
    word(g.bg);
    word(g.Z);
    word(g.m_rows);
    word(g.kb);
    for (int32_t v : g.row_ptr) word(v);
    for (int16_t v : g.col) word(v);
    for (int16_t v : g.shift) word(v);
    *out = h;
    return LDPC_OK;
}

int ldpc_get_graph(int bg, int Z, int *m_rows, int *kb, int *nnz, int16_t *row, int16_t *col,
                   int16_t *shift) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_graphs.find({bg, Z});
    if (it == g_graphs.end()) return LDPC_ENOGRAPH;
    const HostGraph &g = it->second;
    const int E = g.row_ptr.back();
    if ((row || col || shift) && (!row || !col || !shift || !nnz || *nnz < E))
        return LDPC_EINVAL;
    if (m_rows) *m_rows = g.m_rows;
    if (kb) *kb = g.kb;
    if (row) {
        for (int r = 0; r < g.m_rows; ++r)
            for (int e = g.row_ptr[r]; e < g.row_ptr[r + 1]; ++e) {
                row[e] = (int16_t)r;
                col[e] = g.col[e];
                shift[e] = g.shift[e];
            }
    }
    if (nnz) *nnz = E;
    return LDPC_OK;
}

int ldpc_query(int bg, int Z, int rows, int *K, int *T, int *Nc, int *E) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_graphs.find({bg, Z});
    if (it == g_graphs.end()) return LDPC_ENOGRAPH;
    return sub_sizes(it->second, rows, K, T, Nc, E);
}

void ldpc_args_init(ldpc_args *a) {
    if (!a) return;
    *a = ldpc_args{};
    a->precision = LDPC_I8;
    a->max_iter = 10;
    a->early_exit = 1;
    a->beta_q = 96;
    a->offset_q = 0;
    a->beta_h = 0x3A00;
    a->offset_h = 0;
}

int ldpc_decode_ex(const ldpc_args *a) {
    DecodeLaunch p{};
    bool msg_in_lds = false;
    size_t msg_bytes = 0;
    int rc = prepare_decode(a, true, p, msg_in_lds, msg_bytes, true);
    if (rc != LDPC_OK) return rc;
    hipStream_t stream = static_cast<hipStream_t>(a->stream);
    const bool i8 = a->precision == LDPC_I8;
    void *msg = nullptr;
    hipError_t e;
    if (!msg_in_lds) {
        p.msg_bytes = msg_bytes;
        e = hipMallocAsync(&msg, msg_bytes, stream);
        if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(messages)");
        // the persistent schedule's codeword counter: the last 256 bytes
        if (p.refill)
            p.counter = reinterpret_cast<unsigned *>(static_cast<uint8_t *>(msg) + msg_bytes - 256);
    }
    p.msg = static_cast<uint32_t *>(msg);
    e = i8 ? launch_decode_i8(p, stream) : launch_decode_f16(p, stream);
    const hipError_t ef = msg ? hipFreeAsync(msg, stream) : hipSuccess;
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? LDPC_ENOMEM : LDPC_EHIP;
    if (ef != hipSuccess) return hip_fail(ef, "hipFreeAsync(messages)");
    return LDPC_OK;
}

int ldpc_decode_noalloc(const ldpc_args *a) {
    DecodeLaunch p{};
    bool msg_in_lds = false;
    size_t msg_bytes = 0;
    int rc = prepare_decode(a, false, p, msg_in_lds, msg_bytes);
    if (rc != LDPC_OK) return rc;
    void *msg = nullptr;
    if (!msg_in_lds) {
        if (msg_bytes > kScratchBytes) {
            snprintf(g_msg, sizeof(g_msg),
                     "ldpc_decode_noalloc: messages need %zu bytes, the static scratch holds %zu",
                     msg_bytes, kScratchBytes);
            return LDPC_EINVAL;
        }
        rc = scratch_ptr(&msg);
        if (rc != LDPC_OK) return rc;
        p.msg_bytes = msg_bytes;
    }
    p.msg = static_cast<uint32_t *>(msg);
    hipStream_t stream = static_cast<hipStream_t>(a->stream);
    const hipError_t e = a->precision == LDPC_I8 ? launch_decode_i8(p, stream)
                                                 : launch_decode_f16(p, stream);
    if (e != hipSuccess) return LDPC_EHIP;
    return LDPC_OK;
}

int ldpc_tune(const ldpc_args *a, ldpc_tuning *out) {
    if (!a || a->precision != LDPC_I8 || a->lanes_per_row != 0 || a->cw_per_block != 0 ||
        a->msg_placement != LDPC_MSG_AUTO || a->schedule != LDPC_SCHED_STATIC ||
        a->max_workgroups != 0 || a->pairing != LDPC_PAIR_AUTO)
        return LDPC_EINVAL;
    {
        // forget an earlier choice for this key, so the candidates below
        // are not redirected to it
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned.erase(std::make_tuple(a->bg, a->Z, a->rows, pow2_bucket(a->n_cw),
                                      a->early_exit ? 1 : 0));
    }
    // first the library's default launch: if it wins, nothing is recorded
    std::vector<Tuned> cand{
        Tuned{0, 0, LDPC_MSG_AUTO, LDPC_SCHED_STATIC, LDPC_PAIR_AUTO},
        Tuned{1, 0, LDPC_MSG_AUTO, LDPC_SCHED_PERSISTENT, LDPC_PAIR_CODEWORDS}};
    for (int pairs : {1, 2, 3, 4, 6, 8, 12, 16, 24, 48}) {
        cand.push_back(Tuned{1, 2 * pairs, LDPC_MSG_LDS, LDPC_SCHED_STATIC, LDPC_PAIR_CODEWORDS});
        cand.push_back(
            Tuned{1, 2 * pairs, LDPC_MSG_DEVICE, LDPC_SCHED_STATIC, LDPC_PAIR_CODEWORDS});
    }
    for (int alpha : {2, 4}) {
        int base = 1;
        while ((base * a->Z) % 64 != 0) ++base;
        for (int k : {1, 2})
            cand.push_back(Tuned{alpha, 2 * base * k, LDPC_MSG_DEVICE, LDPC_SCHED_STATIC,
                                 LDPC_PAIR_CODEWORDS});
    }
    for (int cws : {1, 2, 4})
        cand.push_back(Tuned{1, cws, LDPC_MSG_DEVICE, LDPC_SCHED_STATIC, LDPC_PAIR_ROWS});
    hipStream_t stream = static_cast<hipStream_t>(a->stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return LDPC_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LDPC_EHIP;
    }
    float best = 1e30f;
    Tuned pick{0, 0, LDPC_MSG_AUTO, LDPC_SCHED_STATIC, LDPC_PAIR_AUTO};
    int tried = 0, rc = LDPC_OK;
    for (const Tuned &c : cand) {
        ldpc_args t = *a;
        t.lanes_per_row = c.lanes_per_row;
        t.cw_per_block = c.cw_per_block;
        t.msg_placement = c.msg_placement;
        t.schedule = c.schedule;
        t.pairing = c.pairing;
        DecodeLaunch probe{};
        bool in_lds = false;
        size_t mb = 0;
        if (prepare_decode(&t, true, probe, in_lds, mb, true) != LDPC_OK) continue;  // does not apply
        // the library rounds the packing to what fits: skip duplicates
        if (c.cw_per_block != 0 && probe.cpw != c.cw_per_block) continue;
        float ms = 1e30f;
        for (int rep = 0; rep < 4 && rc == LDPC_OK; ++rep) {
            (void)hipEventRecord(e0, stream);
            rc = ldpc_decode_ex(&t);
            (void)hipEventRecord(e1, stream);
            (void)hipEventSynchronize(e1);
            float m = 0.0f;
            (void)hipEventElapsedTime(&m, e0, e1);
            if (rep > 0) ms = std::min(ms, m);  // the first run warms up
        }
        if (rc != LDPC_OK) break;
        ++tried;
        if (ms < best) {
            best = ms;
            pick = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LDPC_OK) return rc;
    if (tried == 0) return LDPC_EINVAL;
    const bool is_default = pick.lanes_per_row == 0;
    if (!is_default) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[std::make_tuple(a->bg, a->Z, a->rows, pow2_bucket(a->n_cw),
                                a->early_exit ? 1 : 0)] = pick;
    }
    if (out) {
        out->lanes_per_row = pick.lanes_per_row > 0 ? pick.lanes_per_row : 1;
        out->cw_per_block = pick.cw_per_block;
        out->msg_placement = pick.msg_placement;
        out->schedule = pick.schedule;
        out->pairing = pick.pairing;
        out->ms = best;
        out->candidates = tried;
    }
    return LDPC_OK;
}

int ldpc_decode(int bg, int Z, int rows, int n_cw, const int8_t *llr_in, int max_iter,
                uint8_t *out_bits, int32_t *out_iters, void *stream) {
    ldpc_args a;
    ldpc_args_init(&a);
    a.bg = bg;
    a.Z = Z;
    a.rows = rows;
    a.n_cw = n_cw;
    a.llr_in = llr_in;
    a.max_iter = max_iter;
    a.out_bits = out_bits;
    a.out_iters = out_iters;
    a.stream = stream;
    return ldpc_decode_ex(&a);
}

int ldpc_nwms_loss_grad(int bg, int Z, int rows, int n_cw, const float *llr,
                        const uint8_t *cbits, int n_iter, const float *w, const float *iter_w,
                        float scale, float *loss, float *grad, float *out_llr, void *stream) {
    if (n_cw < 1 || n_iter < 1 || n_iter > LDPC_MAX_ITER || !llr || !cbits || !w || !loss ||
        !grad || !(scale > 0.0f))
        return LDPC_EINVAL;
    const int32_t *row_ptr = nullptr;
    const uint32_t *meta_row = nullptr;
    int E = 0, n_cols = 0, wmax = 0, lds_cap = 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_graphs.find({bg, Z});
        if (it == g_graphs.end()) return LDPC_ENOGRAPH;
        const HostGraph &g = it->second;
        if (sub_sizes(g, rows, nullptr, nullptr, nullptr, &E) != LDPC_OK) return LDPC_EINVAL;
        for (int r = 0; r < rows; ++r)
            if (g.row_ptr[r + 1] - g.row_ptr[r] > wmax) wmax = g.row_ptr[r + 1] - g.row_ptr[r];
        DevTables *t = nullptr;
        const int rc = tables_for(g, &t);
        if (rc != LDPC_OK) return rc;
        row_ptr = t->row_ptr;
        meta_row = t->meta_row;
        n_cols = g.kb + rows;
        lds_cap = max_lds_bytes();
    }
    if (wmax > LDPC_NWMS_MAX_ROW_WEIGHT || n_cols * Z * (int)sizeof(float) > lds_cap)
        return LDPC_EINVAL;
    hipStream_t stream_h = static_cast<hipStream_t>(stream);
    void *ws = nullptr;
    const size_t bytes = sizeof(float) * nwms_workspace_floats(n_cw, rows, n_cols, Z, E, n_iter);
    hipError_t e = hipMallocAsync(&ws, bytes, stream_h);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(nwms workspace)");
    e = launch_nwms(llr, cbits, w, iter_w, loss, grad, out_llr, static_cast<float *>(ws), n_cw,
                    rows,
                    n_cols, Z, E, n_iter, scale, row_ptr, meta_row, wmax, stream_h);
    const hipError_t ef = hipFreeAsync(ws, stream_h);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? LDPC_ENOMEM : LDPC_EHIP;
    if (ef != hipSuccess) return hip_fail(ef, "hipFreeAsync(nwms workspace)");
    return LDPC_OK;
}

struct ldpc_plan {
    ldpc::Plan *p;
};

namespace {
// Device job table entries for `jobs` (registered graphs, kept rows).
int batch_jobs(const ldpc_job *jobs, int n_jobs, std::vector<BatchJob> &bj,
               std::vector<int> &job_cw, int &wmax, int &lds_cap) {
    wmax = 0;
    std::lock_guard<std::mutex> lk(g_mu);
    for (int j = 0; j < n_jobs; ++j) {
        const ldpc_job &jb = jobs[j];
        auto it = g_graphs.find({jb.bg, jb.Z});
        if (it == g_graphs.end()) return LDPC_ENOGRAPH;
        const HostGraph &g = it->second;
        int E = 0;
        if (jb.n_cw < 1 || !jb.llr || (reinterpret_cast<uintptr_t>(jb.llr) & 3u) != 0 ||
            !jb.out_bits || !jb.out_iters || g.Z > kBatchLanes ||
            (jb.wq && jb.wq_iters < 1) ||
            sub_sizes(g, jb.rows, nullptr, nullptr, nullptr, &E) != LDPC_OK)
            return LDPC_EINVAL;
        for (int r = 0; r < jb.rows; ++r)
            wmax = std::max(wmax, (int)(g.row_ptr[r + 1] - g.row_ptr[r]));
        DevTables *t = nullptr;
        const int rc = tables_for(g, &t);
        if (rc != LDPC_OK) return rc;
        BatchJob b{};
        b.llr = jb.llr;
        b.out_bits = jb.out_bits;
        b.out_iters = jb.out_iters;
        b.out_ok = jb.out_ok;
        b.row_ptr = t->row_ptr;
        b.row_pad = t->row_pad;
        b.E_pad = padded_row_ptr(g)[jb.rows];
        b.groups = layer_groups(g.row_ptr.data(), g.col.data(), jb.rows);
        b.meta = t->meta_i8;
        b.meta_rp = t->meta_i8rp;
        b.wq = jb.wq;
        b.w_iters = jb.wq ? jb.wq_iters : 0;
        b.w_stride = jb.rows;
        b.rows = jb.rows;
        b.n_cols = g.kb + jb.rows;
        b.kb = g.kb;
        b.Z = g.Z;
        b.E = E;
        b.slots = 2 * (kBatchLanes / g.Z);
        b.split = jb.split ? 1 : 0;
        bj.push_back(b);
        job_cw.push_back(jb.n_cw);
    }
    lds_cap = max_lds_bytes();
    return wmax > 20 ? LDPC_EINVAL : LDPC_OK;
}
}  // namespace


int ldpc_plan_create(const ldpc_job *jobs, int n_jobs, int max_iter, int early_exit, int flags,
                     void *stream, ldpc_plan **out) {
    if (!jobs || n_jobs < 1 || !out || max_iter < 1 || max_iter > LDPC_MAX_ITER) return LDPC_EINVAL;
    constexpr int kLanes = kBatchLanes;
    std::vector<BatchJob> bj;
    std::vector<int> job_cw;
    int wmax = 0, lds_cap = 0;
    const int rcj = batch_jobs(jobs, n_jobs, bj, job_cw, wmax, lds_cap);
    if (rcj != LDPC_OK) return rcj;
    if (wmax > 20) return LDPC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    ldpc::Plan *p = plan_new();
    int rc = plan_build(p, bj, job_cw, kLanes, max_iter, early_exit ? 1 : 0, 96, 0, wmax,
                        lds_cap, s);
    if (rc == LDPC_OK && (flags & LDPC_PLAN_AUTOTUNE)) rc = plan_autotune(p, s);
    if (rc == LDPC_OK && (flags & LDPC_PLAN_GRAPH)) rc = plan_capture(p);
    if (rc != LDPC_OK) {
        plan_destroy(p);
        return rc;
    }
    *out = new ldpc_plan{p};
    return LDPC_OK;
}

int ldpc_plan_launch(ldpc_plan *plan, void *stream) {
    if (!plan || !plan->p) return LDPC_EINVAL;
    return plan_launch(plan->p, static_cast<hipStream_t>(stream));
}

int ldpc_plan_info(const ldpc_plan *plan, int *grid, int *n_tasks, float *tuned_ms) {
    if (!plan || !plan->p) return LDPC_EINVAL;
    plan_info(plan->p, grid, n_tasks, tuned_ms);
    return LDPC_OK;
}

void ldpc_plan_destroy(ldpc_plan *plan) {
    if (!plan) return;
    plan_destroy(plan->p);
    delete plan;
}

int ldpc_decode_batch_async(const ldpc_job *jobs, int n_jobs, int max_iter, int early_exit,
                            void *stream, size_t *bytes_in_flight) {
    if (!jobs || n_jobs < 1 || max_iter < 1 || max_iter > LDPC_MAX_ITER) return LDPC_EINVAL;
    std::vector<BatchJob> bj;
    std::vector<int> job_cw;
    int wmax = 0, lds_cap = 0;
    const int rc = batch_jobs(jobs, n_jobs, bj, job_cw, wmax, lds_cap);
    if (rc != LDPC_OK) return rc;
    return batch_async(bj, job_cw, kBatchLanes, max_iter, early_exit ? 1 : 0, wmax, lds_cap,
                       static_cast<hipStream_t>(stream), bytes_in_flight);
}

int ldpc_decode_batch_bytes(const ldpc_job *jobs, int n_jobs, size_t *bytes) {
    if (!jobs || n_jobs < 1 || !bytes) return LDPC_EINVAL;
    std::vector<BatchJob> bj;
    std::vector<int> job_cw;
    int wmax = 0, lds_cap = 0;
    const int rc = batch_jobs(jobs, n_jobs, bj, job_cw, wmax, lds_cap);
    if (rc != LDPC_OK) return rc;
    return batch_async_bytes(bj, job_cw, lds_cap, bytes);
}

int ldpc_decode_batch(const ldpc_job *jobs, int n_jobs, int max_iter, int early_exit,
                      void *stream) {
    ldpc_plan *plan = nullptr;
    int rc = ldpc_plan_create(jobs, n_jobs, max_iter, early_exit, 0, stream, &plan);
    if (rc != LDPC_OK) return rc;
    rc = ldpc_plan_launch(plan, stream);
    const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    ldpc_plan_destroy(plan);
    if (rc != LDPC_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(batch)");
    return LDPC_OK;
}

const char *ldpc_strerror(int code) {
    switch (code) {
        case LDPC_OK: return "ok";
        case LDPC_EINVAL: return "invalid argument";
        case LDPC_ENOMEM: return "out of memory";
        case LDPC_EHIP: return "HIP runtime error";
        case LDPC_ENOGRAPH: return "no graph registered for (bg, Z)";
        default: return "unknown error";
    }
}

int ldpc_last_hip_error(void) { return g_last_hip; }

const char *ldpc_last_error_message(void) { return g_msg; }

void ldpc_shutdown(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_dev) free_tables(kv.second);
    g_dev.clear();
}

}  // extern "C"

namespace ldpc {
// The batch-kernel job record of one serving job (registered graph, tables
// uploaded to the current device); row weights up to 20.
int serve_job(const ldpc_job &job, BatchJob &bj, int &wmax) {
    std::vector<BatchJob> v;
    std::vector<int> cw;
    int lds_cap = 0;
    const int rc = batch_jobs(&job, 1, v, cw, wmax, lds_cap);
    if (rc != LDPC_OK) return rc;
    bj = v[0];
    if ((bj.slots / 2) * bj.E_pad * bj.Z > kServeMsgPerBlock || bj.n_cols > LDPC_MAX_COLS)
        return LDPC_EINVAL;
    return LDPC_OK;
}
}  // namespace ldpc
