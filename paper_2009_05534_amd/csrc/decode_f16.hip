// Layered normalised min-sum decoding in IEEE binary16 for gfx950
// (Ling & Cautereels, §III decoding rules, §IV min/second-min/sign
// intermediates and the packed half-precision number format).
//
// Same row-pair organisation as the int8 kernel: lane u owns check rows u
// and u + Z/2 and holds them as one packed half2 register, so every update
// is a single v_pk_*_f16 (rounded to nearest even, no contraction). The
// posteriors live in LDS as half2 pair words (BG1-shaped at Z = 384:
// 52,224 bytes, so three codewords fit one CU); the check-to-variable
// messages do not fit and stream through device memory -- the paper's
// half-precision decoder met the same wall (§V). Every message of a row is
// +-a1 or +-a2 (§IV's min / second min), so a lane stores a row's messages
// exactly as one record: a1 and a2 (half2: rows u and u + Z/2), the sign
// bit of each block's message and a one-hot argmin flag per block, 3 dwords
// for rows of up to 8 blocks, 4 up to 16, 6 up to 32 (BG1-shaped: 151
// dwords per lane and iteration instead of 316). Magnitudes are compared as
// integers on the bit patterns (monotone for non-negative halves).
#include "ldpc_internal.h"

namespace ldpc {
namespace {

typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ inline h16x2 as_h(uint32_t v) { return __builtin_bit_cast(h16x2, v); }
__device__ inline u16x2 as_u(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ inline uint32_t bits_of(h16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ inline uint32_t bits_of(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// Message of block e for a lane: 32 bits at byte offset 4*(e*Zh + ro) from
// the workgroup's uniform base; unsigned 32-bit offsets let the access use
// the scalar-base + vector-offset form.
__device__ inline uint32_t msg_ld(const uint32_t *Rb, int e, int Zh, int ro) {
    const uint32_t off = 4u * (uint32_t)(e * Zh + ro);
    return *reinterpret_cast<const uint32_t *>(reinterpret_cast<const uint8_t *>(Rb) + off);
}
__device__ inline void msg_st(uint32_t *Rb, int e, int Zh, int ro, uint32_t v) {
    const uint32_t off = 4u * (uint32_t)(e * Zh + ro);
    *reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(Rb) + off) = v;
}

// Rotate a pair word right by `rot` bits: 16 when the halves arrive
// swapped, else 0 (a per-lane amount, so it lives in a VGPR, not a mask).
__device__ inline uint32_t swap_halves(uint32_t v, uint32_t rot) {
    return __builtin_amdgcn_alignbit(v, v, rot);
}

struct Gather {
    int addr;
    uint32_t rot;
};

// Pair word of lane u's two rows for block `md` (format in ldpc_internal.h)
// and the rotation that puts row u in the low half.
__device__ inline Gather gather(uint32_t md, int u, int Zh) {
    const int word = (int)(md & 0xFFFFu);
    const int thr = (int)((md >> 16) & 0xFFu);
    const bool shi = (md >> 24) & 1u;
    const bool wrap = u >= thr;
    return Gather{word + u + (wrap ? -Zh : 0), (wrap != shi) ? 16u : 0u};
}

// a = w * max(m - off, 0), each step rounded to binary16.
__device__ inline uint32_t normalise(uint32_t m, uint32_t off, h16x2 w) {
    h16x2 v = as_h(m);
    if (off) {
        v = v - as_h(off);
        v = __builtin_elementwise_max(v, (h16x2){(_Float16)0, (_Float16)0});
    }
    return bits_of(w * v);
}

// Message record of a row of W blocks: dwords 0 and 1 hold a1 and a2, then
// F(W) flag dwords with, per block k and half (bit b of the low half for
// row u, of the high half for row u + Z/2), the message's sign bit and a
// one-hot argmin flag:
//   W <= 8 : one dword, sign at bit k, argmin at bit 8 + k;
//   W <= 16: sign dword (bit k), argmin dword (bit k);
//   W <= 32: the same pair for blocks 0..15, then for blocks 16..31.
template <int W>
struct Rec {
    static constexpr int F = W <= 8 ? 1 : (W <= 16 ? 2 : 4);
    static constexpr int N = 2 + F;
    // dword and bit of block k's sign and argmin flag
    static constexpr int sw(int k) { return 2 + (F == 4 ? 2 * (k >> 4) : 0); }
    static constexpr int sb(int k) { return F == 4 ? (k & 15) : k; }
    static constexpr int ow(int k) { return F == 1 ? 2 : (F == 2 ? 3 : 3 + 2 * (k >> 4)); }
    static constexpr int ob(int k) { return F == 1 ? 8 + k : (F == 4 ? (k & 15) : k); }
};

// Per-half shifts of a pair word (both halves by the same amount; a
// constant once the callers' loops are unrolled).
__device__ inline uint32_t shl16(uint32_t v, int sh) {
    return bits_of(as_u(v) << (u16x2){(unsigned short)sh, (unsigned short)sh});
}
__device__ inline uint32_t shr16(uint32_t v, int sh) {
    return bits_of(as_u(v) >> (u16x2){(unsigned short)sh, (unsigned short)sh});
}

// Message of block k from the row's record: |R| = a2 on the argmin block,
// else a1, with the stored sign bit.
template <int W>
__device__ inline uint32_t rec_message(const uint32_t *rec, int k) {
    using RF = Rec<W>;
    const uint32_t sgn = shl16(rec[RF::sw(k)], 15 - RF::sb(k)) & 0x80008000u;
    // the argmin flag moved to bit 15 of each half, then spread over the half
    typedef short s16x2 __attribute__((ext_vector_type(2)));
    const s16x2 oh = __builtin_bit_cast(s16x2, shl16(rec[RF::ow(k)], 15 - RF::ob(k)));
    const uint32_t arg = __builtin_bit_cast(uint32_t, oh >> (s16x2){15, 15});
    return ((rec[1] & arg) | (rec[0] & ~arg)) | sgn;
}

// Adds block k's sign bit (bit 15 of each half of sgn) and argmin mask
// (0xFFFF halves of arg) to the record being built.
template <int W>
__device__ inline void rec_put(uint32_t *rec, int k, uint32_t sgn, uint32_t arg) {
    using RF = Rec<W>;
    rec[RF::sw(k)] |= shr16(sgn, 15 - RF::sb(k));
    rec[RF::ow(k)] |= arg & ((1u << RF::ob(k)) * 0x00010001u);
}

// Variable-to-check messages of blocks K0..K1-1: the check-to-variable
// messages rebuilt from the row's record (all zero in the first
// iteration), the posteriors read from LDS, then x = L - R rounded to
// binary16, folded into m1 / m2 / S.
template <int W, int K0, int K1, bool KEEP_GATHER>
__device__ __forceinline__ void row_phase1(const uint32_t *__restrict__ Lw, const uint32_t *rec,
                                           const uint32_t *md, int u, int Zh, bool first_iter,
                                           uint32_t *xv, int *la, uint32_t *sw, u16x2 &m1,
                                           u16x2 &m2, uint32_t &S) {
    constexpr int n = K1 - K0;
    uint32_t lraw[n], rraw[n], swl[n];
#pragma unroll
    for (int i = 0; i < n; ++i) {
        const Gather g = gather(md[K0 + i], u, Zh);
        swl[i] = g.rot;
        if (KEEP_GATHER) {
            la[K0 + i] = g.addr;
            sw[K0 + i] = g.rot;
        }
        lraw[i] = Lw[g.addr];
    }
    if (!first_iter) {
#pragma unroll
        for (int i = 0; i < n; ++i) rraw[i] = rec_message<W>(rec, K0 + i);
    } else {
#pragma unroll
        for (int i = 0; i < n; ++i) rraw[i] = 0;
    }
    if constexpr (KEEP_GATHER) {
        // Narrow rows (K0 = 0, every edge): each step over all edges at
        // once and the two smallest magnitudes by a pairwise tree, so
        // dependent packed operations are rarely adjacent (gfx950 inserts a
        // wait state between them). Magnitudes compare as integers.
#pragma unroll
        for (int i = 0; i < n; ++i)
            xv[i] = bits_of(as_h(swap_halves(lraw[i], swl[i])) - as_h(rraw[i]));
#pragma unroll
        for (int i = 0; i < n; ++i) S ^= xv[i];
        constexpr int NP = (n + 1) / 2;
        u16x2 lo[NP], hi[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const u16x2 a = as_u(xv[2 * q] & 0x7FFF7FFFu);
            const u16x2 b =
                2 * q + 1 < n ? as_u(xv[2 * q + 1] & 0x7FFF7FFFu) : (u16x2){0x7C00, 0x7C00};
            lo[q] = __builtin_elementwise_min(a, b);
            hi[q] = __builtin_elementwise_max(a, b);
        }
#pragma unroll
        for (int w = 1; w < NP; w *= 2) {
#pragma unroll
            for (int q = 0; q + w < NP; q += 2 * w) {
                const u16x2 l = __builtin_elementwise_min(lo[q], lo[q + w]);
                const u16x2 h = __builtin_elementwise_min(__builtin_elementwise_max(lo[q], lo[q + w]),
                                                          __builtin_elementwise_min(hi[q], hi[q + w]));
                lo[q] = l;
                hi[q] = h;
            }
        }
        m1 = lo[0];
        m2 = hi[0];
        return;
    }
#pragma unroll
    for (int i = 0; i < n; ++i) {
        const h16x2 L = as_h(swap_halves(lraw[i], swl[i]));
        const h16x2 x = L - as_h(rraw[i]);
        const uint32_t xb = bits_of(x);
        const u16x2 ax = as_u(xb & 0x7FFF7FFFu);
        m2 = __builtin_elementwise_min(m2, __builtin_elementwise_max(m1, ax));
        m1 = __builtin_elementwise_min(m1, ax);
        S ^= xb;
        xv[K0 + i] = xb;
    }
}

// One block row of exactly W blocks for lane u (rows u and u + Zh). As in
// the int8 kernel the row is branch-free: metadata in one batch of scalar
// loads, then the reads before any arithmetic; rows wider than 10 blocks
// read in two halves and recompute their gathers for the write-back.
// Row record dword j of this lane: Rb[(P + j) * Zh + ro] (uniform base,
// 32-bit lane offset); keep: store the new record (not in the last
// iteration, where nothing reads it).
template <int W>
__device__ __forceinline__ void row_update_w(uint32_t *__restrict__ Lw, uint32_t *__restrict__ Rb,
                                             int ro, const uint32_t *__restrict__ meta, int e0,
                                             int P, int u, int Zh, bool first_iter, bool keep,
                                             h16x2 wgt, uint32_t off) {
    using RF = Rec<W>;
    constexpr bool kWide = W > 10;
    uint32_t md[W], rec[RF::N];
#pragma unroll
    for (int k = 0; k < W; ++k) md[k] = meta[e0 + k];
    if (!first_iter) {
#pragma unroll
        for (int j = 0; j < RF::N; ++j) rec[j] = msg_ld(Rb, P + j, Zh, ro);
    }
    uint32_t xv[W], sw[W];
    int la[W];
    u16x2 m1 = {0x7C00, 0x7C00}, m2 = {0x7C00, 0x7C00};
    uint32_t S = 0;
    if constexpr (kWide) {
        constexpr int H = (W + 1) / 2;
        row_phase1<W, 0, H, false>(Lw, rec, md, u, Zh, first_iter, xv, la, sw, m1, m2, S);
        row_phase1<W, H, W, false>(Lw, rec, md, u, Zh, first_iter, xv, la, sw, m1, m2, S);
    } else {
        row_phase1<W, 0, W, true>(Lw, rec, md, u, Zh, first_iter, xv, la, sw, m1, m2, S);
    }
    const uint32_t a1 = normalise(bits_of(m1), off, wgt);
    const uint32_t a2 = normalise(bits_of(m2), off, wgt);
    const u16x2 m1p = m1 + (u16x2){1, 1};
    uint32_t nrec[RF::N];
    nrec[0] = a1;
    nrec[1] = a2;
#pragma unroll
    for (int j = 2; j < RF::N; ++j) nrec[j] = 0;
    // The write-back one step at a time over groups of edges (all of a
    // narrow row, four of a wide one), for the same reason.
    constexpr int G = kWide ? 4 : W;
#pragma unroll
    for (int g0 = 0; g0 < W; g0 += G) {
        uint32_t Rg[G], Lg[G], Sg[G], Ag[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int k = g0 + i;
            if (k >= W) continue;
            // mask = 0xFFFF on the argmin edge (|x| == m1), else 0.
            const u16x2 t = __builtin_elementwise_sub_sat(m1p, as_u(xv[k] & 0x7FFF7FFFu));
            Ag[i] = bits_of((u16x2){0, 0} - t);
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int k = g0 + i;
            if (k >= W) continue;
            const uint32_t mag = (a2 & Ag[i]) | (a1 & ~Ag[i]);
            Sg[i] = (S ^ xv[k]) & 0x80008000u;
            Rg[i] = mag | Sg[i];
            Lg[i] = bits_of(as_h(xv[k]) + as_h(Rg[i]));
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int k = g0 + i;
            if (k >= W) continue;
            if (kWide) {
                const Gather g = gather(md[k], u, Zh);
                Lw[g.addr] = swap_halves(Lg[i], g.rot);
            } else {
                Lw[la[k]] = swap_halves(Lg[i], sw[k]);
            }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int k = g0 + i;
            if (k >= W) continue;
            rec_put<W>(nrec, k, Sg[i], Ag[i]);
        }
    }
    if (keep) {
#pragma unroll
        for (int j = 0; j < RF::N; ++j) msg_st(Rb, P + j, Zh, ro, nrec[j]);
    }
}

// Parity of lane u's rows over a row of exactly W blocks (bits 15 and 31);
// hard decision [L_v < 0], negative zero decides 0.
template <int W>
__device__ __forceinline__ uint32_t row_parity_w(const uint32_t *__restrict__ Lw,
                                                 const uint32_t *__restrict__ meta, int e0, int u,
                                                 int Zh) {
    uint32_t md[W], raw[W], sw[W];
#pragma unroll
    for (int k = 0; k < W; ++k) md[k] = meta[e0 + k];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const Gather g = gather(md[k], u, Zh);
        sw[k] = g.rot;
        raw[k] = Lw[g.addr];
    }
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const uint32_t v = swap_halves(raw[k], sw[k]);
        const uint32_t lo = (v & 0xFFFFu) > 0x8000u ? 0x8000u : 0u;
        const uint32_t hi = (v >> 16) > 0x8000u ? 0x80000000u : 0u;
        acc ^= lo | hi;
    }
    return acc;
}

template <int W, int WMAX>
__device__ __forceinline__ void row_update(int w, uint32_t *Lw, uint32_t *Rb, int ro,
                                           const uint32_t *meta, int e0, int P, int u, int Zh,
                                           bool first_iter, bool keep, h16x2 wgt, uint32_t off) {
    if constexpr (W <= WMAX) {
        if (w == W) {
            row_update_w<W>(Lw, Rb, ro, meta, e0, P, u, Zh, first_iter, keep, wgt, off);
            return;
        }
        row_update<W + 1, WMAX>(w, Lw, Rb, ro, meta, e0, P, u, Zh, first_iter, keep, wgt, off);
    }
}

template <int W, int WMAX>
__device__ __forceinline__ uint32_t row_parity(int w, const uint32_t *Lw, const uint32_t *meta,
                                               int e0, int u, int Zh) {
    if constexpr (W <= WMAX) {
        if (w == W) return row_parity_w<W>(Lw, meta, e0, u, Zh);
        return row_parity<W + 1, WMAX>(w, Lw, meta, e0, u, Zh);
    }
    return 0;
}

// Syndrome check of an unfinished codeword: a failing check of lane u's rows
// marks the codeword in *fl (its LDS flag, zero on entry; every marking lane
// stores the same 1). One failing check decides the codeword, so a wave stops
// sweeping the rows once every codeword its lanes serve is marked; only a
// codeword whose checks all hold needs the full sweep.
template <int WMAX>
__device__ inline void syndrome_mark(const uint32_t *__restrict__ Lw,
                                     const int32_t *__restrict__ row_ptr,
                                     const uint32_t *__restrict__ meta, int rows, int u, int Zh,
                                     volatile int *fl) {
    for (int r = 0; r < rows; ++r) {
        const int e0 = row_ptr[r], w = row_ptr[r + 1] - e0;
        if (row_parity<2, WMAX>(w, Lw, meta, e0, u, Zh)) *fl = 1;
        if (__ballot(*fl == 0) == 0) break;
    }
}

// A codeword's channel LLRs into its posterior words (punctured columns 0
// and 1 carry none). The lanes read consecutive dwords (lane u: dwords
// u, u + Zh, u + 2Zh, ...), KB loads in flight per lane, so the whole
// codeword costs a couple of memory round trips. Dword k*Zh + u starts at
// byte 2k*Z + 4u: column 2 + 2k (+1 once 4u >= Z), variable 4u mod Z, and
// its four bytes (Z is a multiple of 8) share one column and one half of
// the pair words. Each byte, clamped to -127, becomes a binary16 half.
template <int KB>
__device__ inline void load_llrs_f16(uint32_t *Lw, const int8_t *q, int N, int Z, int u) {
    const int Zh = Z >> 1;
    Lw[u] = 0;
    Lw[Zh + u] = 0;
    const int nd = (N - 2) * Z / 4;
    const int kmax = (N - 1) / 2;  // ceil((N - 2) / 2) dwords per lane at most
    const int cu = 4 * u >= Z ? 1 : 0, v = 4 * u - cu * Z, hi = v >= Zh ? 1 : 0;
    // binary16 slot of this lane's first byte; +2 per byte, +4*Zh per k
    uint16_t *dst0 = reinterpret_cast<uint16_t *>(Lw) + 2 * ((2 + cu) * Zh + v - hi * Zh) + hi;
    const uint32_t *q32 = reinterpret_cast<const uint32_t *>(q);
#pragma unroll 1
    for (int k0 = 0; k0 < kmax; k0 += KB) {
        uint32_t d[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int idx = (k0 + k) * Zh + u;
            d[k] = q32[idx < nd ? idx : nd - 1];
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            if ((k0 + k) * Zh + u < nd) {
                uint16_t *dst = dst0 + 4 * Zh * (k0 + k);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    int x = (int)(int8_t)(d[k] >> (8 * b));
                    x = x < -127 ? -127 : x;
                    dst[2 * b] = __builtin_bit_cast(uint16_t, (_Float16)x);
                }
            }
        }
    }
}

template <int WMAX>
__global__ __launch_bounds__(512) void decode_f16_kernel(DecodeLaunch p,
                                                         const int32_t *__restrict__ row_ptr,
                                                         const uint32_t *__restrict__ meta) {
    static_assert(WMAX <= kMetaPad, "row metadata window exceeds the table padding");
    extern __shared__ __align__(16) uint8_t smem[];
    const int Z = p.Z, Zh = Z >> 1;
    const int N = p.n_cols, E = p.E, T = (N - 2) * Z;
    const int slot_bytes = lds_bytes_f16(N, Z);
    const int slot = threadIdx.x / Zh;
    const int u = threadIdx.x - slot * Zh;
    const int cw = blockIdx.x * p.cpw + slot;
    const bool valid = cw < p.n_cw;
    uint32_t *Lw = reinterpret_cast<uint32_t *>(smem + slot * slot_bytes);
    int *flags = reinterpret_cast<int *>(smem + p.cpw * slot_bytes);
    // Message records: uniform base for the workgroup plus a 32-bit lane
    // offset; p.E_pad = record dwords per lane and iteration.
    uint32_t *Rb = p.msg + (size_t)blockIdx.x * p.cpw * p.E_pad * Zh;
    const int ro = slot * p.E_pad * Zh + u;
    (void)E;

    if (valid) load_llrs_f16<17>(Lw, p.llr + (size_t)cw * T, N, Z, u);
    __syncthreads();

    const uint32_t off = (uint32_t)(p.offset & 0xFFFF) * 0x00010001u;
    bool done = !valid;
    int iters = p.max_iter, ok = 0;
    for (int t = 1; t <= p.max_iter; ++t) {
        uint32_t wt = (uint32_t)(p.beta & 0xFFFF);
        const uint16_t *wrow = nullptr;
        if (p.wh) wrow = p.wh + (size_t)((t < p.w_iters ? t : p.w_iters) - 1) * p.rows;
        // a barrier only where the next row shares a column with the rows
        // since the last one (layer groups), and after the last row
        const uint64_t bar = (p.groups >> 1) | (1ull << (p.rows - 1));
        const bool keep = t < p.max_iter;  // the last iteration's records are never read
        int P = 0;
        for (int r = 0; r < p.rows; ++r) {
            const int e0 = row_ptr[r], w = row_ptr[r + 1] - e0;
            if (wrow) wt = wrow[r];
            const h16x2 wgt = as_h(wt * 0x00010001u);
            if (!done)
                row_update<2, WMAX>(w, Lw, Rb, ro, meta, e0, P, u, Zh, t == 1, keep, wgt, off);
            P += f16_record_dwords(w);
            if ((bar >> r) & 1) __syncthreads();
        }
        if (p.early_exit || t == p.max_iter) {
            if ((int)threadIdx.x < p.cpw) flags[threadIdx.x] = 0;
            __syncthreads();
            if (!done) syndrome_mark<WMAX>(Lw, row_ptr, meta, p.rows, u, Zh, flags + slot);
            __syncthreads();
            const bool holds = flags[slot] == 0;
            if (!done) {
                if (p.early_exit && holds) {
                    done = true;
                    iters = t;
                    ok = 1;
                } else if (t == p.max_iter) {
                    ok = holds;
                }
            }
            if (p.early_exit && __syncthreads_and(done)) break;
            __syncthreads();
        }
    }
    if (!valid) return;

    // Outputs (see the int8 kernel): byte j of a column packs bits 8j..8j+7.
    const uint16_t *Lh = reinterpret_cast<const uint16_t *>(Lw);
    const int bytes_per_col = Z / 8;
    uint8_t *ob = p.out_bits + (size_t)cw * (p.kb * bytes_per_col);
#pragma unroll 1
    for (int c = 0; c < p.kb; ++c) {
#pragma unroll 1
        for (int j = u; j < bytes_per_col; j += Zh) {
            uint32_t byte = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int z = 8 * j + i;
                const int hi = z >= Zh;
                const uint16_t h = Lh[2 * (c * Zh + z - hi * Zh) + hi];
                byte |= (uint32_t)(h > 0x8000u) << i;
            }
            ob[c * bytes_per_col + j] = (uint8_t)byte;
        }
    }
    if (u == 0) {
        p.out_iters[cw] = iters;
        if (p.out_ok) p.out_ok[cw] = (uint8_t)ok;
    }
    if (p.out_llr) {
        uint16_t *o = static_cast<uint16_t *>(p.out_llr) + (size_t)cw * N * Z;
#pragma unroll 1
        for (int c = 0; c < N; ++c) {
            const uint32_t w = Lw[c * Zh + u];
            o[c * Z + u] = (uint16_t)(w & 0xFFFFu);
            o[c * Z + u + Zh] = (uint16_t)(w >> 16);
        }
    }
}

template <int WMAX>
hipError_t launch_w(const DecodeLaunch &p, hipStream_t stream) {
    const int Zh = p.Z / 2;
    const int lds = p.cpw * lds_bytes_f16(p.n_cols, p.Z) + p.cpw * (int)sizeof(int);
    static std::once_flag attr_once;  // once per process, also under concurrent calls
    std::call_once(attr_once, [] {
        // Opt in to more than the default 64 KiB of dynamic LDS.
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&decode_f16_kernel<WMAX>),
            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
        if (e != hipSuccess) note_hip_error("hipFuncSetAttribute(decode_f16_kernel)", e);
    });
    const int blocks = (p.n_cw + p.cpw - 1) / p.cpw;
    // hipGetLastError reports the last error of ANY earlier runtime call on
    // this thread; clear it so the check below sees this launch only.
    (void)hipGetLastError();
    hipLaunchKernelGGL(decode_f16_kernel<WMAX>, dim3(blocks), dim3(p.cpw * Zh), lds, stream, p,
                       p.row_ptr, p.meta);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) note_hip_error("launch decode_f16_kernel", e);
    return e;
}

}  // namespace

hipError_t launch_decode_f16(const DecodeLaunch &p, hipStream_t stream) {
    if (p.wmax <= 10) return launch_w<10>(p, stream);
    if (p.wmax <= 20) return launch_w<20>(p, stream);
    return launch_w<32>(p, stream);
}

}  // namespace ldpc
