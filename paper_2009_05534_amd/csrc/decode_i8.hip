// Layered normalised min-sum decoding in 8-bit saturating fixed point for
// gfx950 (Ling & Cautereels, §III decoding rules, §IV min/second-min/sign
// intermediates and the 8-bit number format).
//
// Codeword pairs. A workgroup holds `slots` pairs; pair p is codewords 2p
// and 2p+1 of the workgroup's range and occupies lanes [p*Z, (p+1)*Z). Lane
// u of a pair owns check row u of every block row for BOTH codewords: a
// 32-bit register carries two 16-bit lanes, the low one for codeword 2p and
// the high one for 2p+1, so every packed VALU instruction advances the same
// check of two codewords. Both codewords share the graph, so the circulant
// gather of block (c, s) reads the same variable (u + s) mod Z for both
// halves: the posterior of variable v of column c is one 16-bit pair word
// in LDS (low byte codeword 2p, high byte 2p+1) and a gather is an address
// plus one fixed byte shuffle, with no per-lane half swapping.
//
// The Z independent rows of a layer (§II) run in parallel, layers strictly
// in order, with a workgroup barrier wherever the next layer shares a block
// column with the layers since the last barrier; after every iteration the
// syndrome of the hard decisions is checked per codeword (a sweep that stops
// at the first failing check), and a codeword whose checks all hold has its
// outputs written at once (its half of the pair is still computed, but
// nothing reads it again).
//
// Register format: each int8 value sits in the HIGH byte of its 16-bit lane
// ("x * 256"), so the int16 saturating subtract clamps at +127 (plus a low
// byte of 0xFF) and one max clamps at -127; the low byte is cleared before a
// value is negated or stored.
#include "ldpc_internal.h"

namespace ldpc {
namespace {

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ inline s16x2 as_s(uint32_t v) { return __builtin_bit_cast(s16x2, v); }
__device__ inline u16x2 as_u(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ inline uint32_t bits_of(s16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ inline uint32_t bits_of(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// v_perm selectors (source bytes 0..3 = the word, 0x0c = zero byte).
constexpr uint32_t kUnpack = 0x010c000cu;  // pair word -> (b0 << 8, b1 << 24)
constexpr uint32_t kPack = 0x0c0c0301u;    // inverse of kUnpack
constexpr uint32_t kUnpackSw = 0x000c010cu;  // pair word -> (b1 << 8, b0 << 24)
constexpr uint32_t kPackSw = 0x0c0c0103u;    // inverse of kUnpackSw

__device__ inline uint32_t perm(uint32_t word, uint32_t sel) {
    return __builtin_amdgcn_perm(0u, word, sel);
}

// Normalised magnitude on the high bytes: a = min((w*max(m - off, 0) + 64)
// >> 7, 127), returned as a * 256 (low byte zero).
__device__ inline u16x2 normalise(u16x2 m, u16x2 off16, u16x2 w) {
    const u16x2 mo = __builtin_elementwise_sub_sat(m, off16);
    u16x2 v = (mo >> (u16x2){8, 8}) * w + (u16x2){64, 64};
    v = __builtin_elementwise_min(v >> (u16x2){7, 7}, (u16x2){127, 127});
    return v << (u16x2){8, 8};
}

// Block metadata md = 2(c*Z + s) | (Z - s) << 16 (column c, shift s) and
// its low half off = 2(c*Z + s). Lane u reads variable (u + s) mod Z of
// column c: LDS byte address lb + off, minus 2Z when u + s wraps
// (u >= Z - s); lb = pair posteriors + 2u. With the lane key
// U = u << 16 | 0xFFFF, U >= md exactly when u >= Z - s, so the compare
// takes md as loaded (no scalar shift); the lane work is one compare, one
// select, one add.
__device__ inline uint32_t lane_key(uint32_t u) { return u << 16 | 0xFFFFu; }

__device__ inline uint32_t gather(uint32_t md, uint32_t off, uint32_t lb, uint32_t U,
                                  uint32_t Z) {
    const uint32_t wrap = U >= md ? 2u * Z : 0u;
    return lb + off - wrap;
}

// Row-pair layout (one codeword; lane u of its Zh = Z/2 lanes owns check
// rows u and u + Zh, the low and high halves of its packed registers; pair
// word p of column c holds variables p (low byte) and p + Zh (high byte)).
// Block metadata md = 2(c*Zh + s_lo) | s_hi << 15 | (Zh - s_lo) << 16 for
// the shift s = s_lo + Zh*s_hi: the address is the pair kernel's gather
// with Zh for Z and the offset in bits [0, 15), and the word's halves
// arrive swapped (row u's variable in the high byte) when
// [u + s_lo >= Zh] xor s_hi.
__device__ inline bool rp_swapped(uint32_t md, uint32_t U) {
    return (U >= md) != ((md & 0x8000u) != 0u);
}
template <bool RP>
constexpr uint32_t off_mask() {
    return RP ? 0x7FFFu : 0xFFFFu;
}

__device__ inline uint32_t lds_ld16(const uint8_t *smem, uint32_t a) {
    return *reinterpret_cast<const uint16_t *>(smem + a);
}
__device__ inline void lds_st16(uint8_t *smem, uint32_t a, uint32_t v) {
    *reinterpret_cast<uint16_t *>(smem + a) = (uint16_t)v;
}

// Check-to-variable messages of one block row, moved as dwords of two pair
// words (messages 2j and 2j+1 of the lane in dword j).
// Device placement: row r of the pair's region holds Wp (the row weight
// rounded up to even) messages per lane, lane u's contiguous, so a lane
// moves its whole row in one to three dwordx4 / x2 / x1 raw-buffer
// accesses: the vector offset is the lane's (pair base + u * 2Wp), the
// scalar offset the row's.
// LDS placement: [e][Z] pair words (lane-contiguous per edge, conflict
// free); the two halves of a dword move as separate 16-bit accesses.
template <bool IN_LDS>
struct MsgRow {
    __amdgpu_buffer_rsrc_t rsrc;  // device placement
    uint8_t *lds;                 // LDS placement: the LDS array
    uint32_t ro;                  // device: pair base; LDS: lane's edge-0 byte address
    uint32_t row;                 // device: byte offset of the row in the pair region
    bool keep;                    // false in the last iteration: nothing reads them again
    bool rmask_on;                // device: AND the loaded message dwords with rmask
    uint32_t rmask;               //   (clears the bytes of halves that start afresh)

    // Loads the row's message dwords d[C0 .. (W + 1) / 2) (device placement;
    // LDS placement loads them all).
    template <int W, int C0 = 0>
    __device__ inline void load(uint32_t *d, uint32_t u, int Z, int wr = W) const {
        constexpr int ND = (W + 1) / 2;
        if constexpr (IN_LDS) {
            // wr (<= W): the row's weight; messages from wr on are not read
#pragma unroll
            for (int j = 0; j < ND; ++j) {
                const uint32_t a = ro + 4u * (uint32_t)(j * Z);
                const uint32_t lo =
                    2 * j < wr ? *reinterpret_cast<const uint16_t *>(lds + a) : 0u;
                const uint32_t hi =
                    2 * j + 1 < wr ? *reinterpret_cast<const uint16_t *>(lds + a + 2u * Z) : 0u;
                d[j] = lo | hi << 16;
            }
        } else {
            const uint32_t v = ro + u * (4u * ND);
#pragma unroll
            for (int c = C0; c < ND; c += 4) {
                const uint32_t so = row + 4u * c;
                if (ND - c >= 4) {
                    const auto q = __builtin_amdgcn_raw_buffer_load_b128(rsrc, v, so, 0);
                    d[c] = q[0], d[c + 1] = q[1], d[c + 2] = q[2], d[c + 3] = q[3];
                } else if (ND - c == 3) {
                    const auto q = __builtin_amdgcn_raw_buffer_load_b96(rsrc, v, so, 0);
                    d[c] = q[0], d[c + 1] = q[1], d[c + 2] = q[2];
                } else if (ND - c == 2) {
                    const auto q = __builtin_amdgcn_raw_buffer_load_b64(rsrc, v, so, 0);
                    d[c] = q[0], d[c + 1] = q[1];
                } else {
                    d[c] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, v, so, 0);
                }
            }
        }
    }
    // Device placement, rows of nd (runtime) dwords: loads the chunks of four
    // dwords [C0, MAXD) that start below nd (a chunk may run past the row;
    // those dwords are not used).
    template <int MAXD, int C0>
    __device__ inline void load_rt(uint32_t *d, uint32_t u, int nd) const {
        const uint32_t v = ro + u * (4u * (uint32_t)nd);
#pragma unroll
        for (int c = C0; c < MAXD; c += 4) {
            if (c >= nd) continue;
            const uint32_t so = row + 4u * c;
            if (MAXD - c >= 4) {
                const auto q = __builtin_amdgcn_raw_buffer_load_b128(rsrc, v, so, 0);
                d[c] = q[0], d[c + 1] = q[1], d[c + 2] = q[2], d[c + 3] = q[3];
            } else if (MAXD - c == 3) {
                const auto q = __builtin_amdgcn_raw_buffer_load_b96(rsrc, v, so, 0);
                d[c] = q[0], d[c + 1] = q[1], d[c + 2] = q[2];
            } else if (MAXD - c == 2) {
                const auto q = __builtin_amdgcn_raw_buffer_load_b64(rsrc, v, so, 0);
                d[c] = q[0], d[c + 1] = q[1];
            } else {
                d[c] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, v, so, 0);
            }
        }
    }
    // Device placement, rows of nd (runtime) dwords: stores dwords
    // [c, c + n) with n in 1..4 decided at run time.
    __device__ inline void store_rt(const uint32_t *d, uint32_t u, int nd, int c, int n) const {
        if (!keep) return;
        typedef uint32_t v4u __attribute__((ext_vector_type(4)));
        typedef uint32_t v3u __attribute__((ext_vector_type(3)));
        typedef uint32_t v2u __attribute__((ext_vector_type(2)));
        const uint32_t v = ro + u * (4u * (uint32_t)nd), so = row + 4u * c;
        if (n >= 4) {
            const v4u q = {d[c], d[c + 1], d[c + 2], d[c + 3]};
            __builtin_amdgcn_raw_buffer_store_b128(q, rsrc, v, so, 0);
        } else if (n == 3) {
            const v3u q = {d[c], d[c + 1], d[c + 2]};
            __builtin_amdgcn_raw_buffer_store_b96(q, rsrc, v, so, 0);
        } else if (n == 2) {
            const v2u q = {d[c], d[c + 1]};
            __builtin_amdgcn_raw_buffer_store_b64(q, rsrc, v, so, 0);
        } else {
            __builtin_amdgcn_raw_buffer_store_b32(d[c], rsrc, v, so, 0);
        }
    }
    // Device placement: the first four message dwords of a row of nd dwords
    // (whatever follows the row fills the rest; a read past the region's end
    // returns zero).
    __device__ inline void load4(uint32_t *d, uint32_t u, int nd) const {
        const auto q =
            __builtin_amdgcn_raw_buffer_load_b128(rsrc, ro + u * (4u * (uint32_t)nd), row, 0);
        d[0] = q[0], d[1] = q[1], d[2] = q[2], d[3] = q[3];
    }
    // Stores the n (1..4) message dwords d[c .. c+n) of the row (c and n are
    // constants once the caller's loop is unrolled).
    template <int W>
    __device__ inline void store(const uint32_t *d, uint32_t u, int Z, int c, int n,
                                 int wr = W) const {
        constexpr int ND = (W + 1) / 2;
        if (!keep) return;
        if constexpr (IN_LDS) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = c + i;
                if (i < n && j < ND) {
                    const uint32_t a = ro + 4u * (uint32_t)(j * Z);
                    *reinterpret_cast<uint16_t *>(lds + a) = (uint16_t)d[j];
                    if (2 * j + 1 < wr)
                        *reinterpret_cast<uint16_t *>(lds + a + 2u * Z) = (uint16_t)(d[j] >> 16);
                }
            }
        } else {
            typedef uint32_t v4u __attribute__((ext_vector_type(4)));
            typedef uint32_t v3u __attribute__((ext_vector_type(3)));
            typedef uint32_t v2u __attribute__((ext_vector_type(2)));
            const uint32_t v = ro + u * (4u * ND), so = row + 4u * c;
            if (n == 4) {
                const v4u q = {d[c], d[c + 1], d[c + 2], d[c + 3]};
                __builtin_amdgcn_raw_buffer_store_b128(q, rsrc, v, so, 0);
            } else if (n == 3) {
                const v3u q = {d[c], d[c + 1], d[c + 2]};
                __builtin_amdgcn_raw_buffer_store_b96(q, rsrc, v, so, 0);
            } else if (n == 2) {
                const v2u q = {d[c], d[c + 1]};
                __builtin_amdgcn_raw_buffer_store_b64(q, rsrc, v, so, 0);
            } else {
                __builtin_amdgcn_raw_buffer_store_b32(d[c], rsrc, v, so, 0);
            }
        }
    }
};

// Device placement prefetches the first four message dwords (eight
// messages) of the next row right after the current row: their memory
// latency then overlaps the layer barrier and the next row's metadata and
// posterior reads.
constexpr int kPreDwords = 4;

// v_perm selectors for the second pair word of a dword (bytes 2, 3) and for
// packing two messages into one dword.
constexpr uint32_t kUnpackHi = 0x030c020cu;  // dword -> (b2 << 8, b3 << 24)
constexpr uint32_t kPack2 = 0x07050301u;     // (R_k, R_k+1) -> pair words k, k+1

// Variable-to-check messages of blocks K0..K1-1 of the row from the
// check-to-variable message dwords rd (already loaded), the posterior reads
// issued first, then x = sat(L - R), folded into m1 / m2 / S.
// RP: the row-pair layout; each edge's unpack selector follows its swap,
// and (KEEP_GATHER) ps keeps the matching pack selector for the write-back.
template <int K0, int K1, bool KEEP_GATHER, bool RP = false>
__device__ __forceinline__ void row_phase1(const uint8_t *__restrict__ smem, uint32_t lb,
                                           const uint32_t *rd, const uint32_t *md,
                                           const uint32_t *mo, uint32_t u,
                                           int Z, int wr, uint32_t *xv, uint32_t *axv,
                                           uint32_t *la, uint32_t *ps, u16x2 &m1, u16x2 &m2,
                                           uint32_t &S) {
    constexpr int n = K1 - K0;
    uint32_t lraw[n], us[n];
#pragma unroll
    for (int i = 0; i < n; ++i) {
        if (K0 + i < wr) {  // wr: the row's weight (below K1 in the generic path)
            const uint32_t a = gather(md[K0 + i], mo[K0 + i], lb, lane_key(u), (uint32_t)Z);
            if (KEEP_GATHER) la[K0 + i] = a;
            if constexpr (RP) {
                const bool sw = rp_swapped(md[K0 + i], lane_key(u));
                us[i] = sw ? kUnpackSw : kUnpack;
                if (KEEP_GATHER) ps[K0 + i] = sw ? kPackSw : kPack;
            } else {
                us[i] = kUnpack;
            }
            lraw[i] = lds_ld16(smem, a);
        }
    }
    if constexpr (KEEP_GATHER) {
        // Narrow rows (every edge present, K0 = 0): each step over all
        // edges at once, and the two smallest magnitudes by a pairwise tree,
        // so dependent packed operations are rarely adjacent.
        s16x2 x[n];
#pragma unroll
        for (int k = 0; k < n; ++k)
            x[k] = __builtin_elementwise_sub_sat(as_s(perm(lraw[k], RP ? us[k] : kUnpack)),
                                                 as_s(perm(rd[k >> 1], (k & 1) ? kUnpackHi : kUnpack)));
#pragma unroll
        for (int k = 0; k < n; ++k)
            x[k] = __builtin_elementwise_max(x[k], (s16x2){-127 * 256, -127 * 256});
#pragma unroll
        for (int k = 0; k < n; ++k) {
            axv[k] = bits_of(__builtin_elementwise_max(x[k], (s16x2){0, 0} - x[k]));
            xv[k] = bits_of(x[k]);
        }
#pragma unroll
        for (int k = 0; k < n; ++k) S ^= xv[k];
        // (lo, hi) of edge pairs, then merged: the smallest of a merge is
        // min(lo1, lo2), the second min(max(lo1, lo2), min(hi1, hi2)).
        constexpr int NP = (n + 1) / 2;
        u16x2 lo[NP], hi[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const u16x2 a = as_u(axv[2 * q]);
            const u16x2 b = 2 * q + 1 < n ? as_u(axv[2 * q + 1]) : (u16x2){0x7FFF, 0x7FFF};
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
        const int k = K0 + i;
        if (k < wr) {
            const s16x2 L = as_s(perm(lraw[i], RP ? us[i] : kUnpack));
            const s16x2 Rm = as_s(perm(rd[k >> 1], (k & 1) ? kUnpackHi : kUnpack));
            s16x2 x = __builtin_elementwise_sub_sat(L, Rm);
            x = __builtin_elementwise_max(x, (s16x2){-127 * 256, -127 * 256});
            const s16x2 ax = __builtin_elementwise_max(x, (s16x2){0, 0} - x);
            const u16x2 axu = as_u(bits_of(ax));
            m2 = __builtin_elementwise_min(m2, __builtin_elementwise_max(m1, axu));
            m1 = __builtin_elementwise_min(m1, axu);
            S ^= bits_of(x);
            xv[k] = bits_of(x);
            if (KEEP_GATHER) axv[k] = bits_of(ax);
        }
    }
}

// One block row of W blocks for lane u: variable-to-check messages,
// min / second min / sign product, normalisation, check-to-variable
// messages and posterior write-back, for both codewords of the pair.
// Specialising on W keeps the row free of branches: the row's metadata
// arrives in one batch of scalar loads and the LDS reads are issued before
// any arithmetic. Rows wider than 10 blocks read in two halves and
// recompute |x| and their gathers for the write-back, which keeps the
// register count low enough for several pairs per CU.
// GEN: W is only an upper bound and wr the row's weight; blocks k >= wr are
// skipped by scalar branches.
// RP: the row-pair layout (rows u and u + Zh of one codeword; Z is Zh).
template <int W, bool IN_LDS, bool FIRST, bool GEN = false, bool RP = false>
__device__ __forceinline__ void row_update_w(uint8_t *__restrict__ smem, uint32_t lb,
                                             const MsgRow<IN_LDS> &R, cmeta_t meta, int e0,
                                             uint32_t u, int Z, u16x2 wgt, u16x2 off16,
                                             const uint32_t *pre, int wr = W) {
    constexpr bool kWide = W > 10;
    const int wrow = GEN ? wr : W;
    uint32_t md[W], mo[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        md[k] = meta[e0 + k];  // the table is padded
        mo[k] = md[k] & off_mask<RP>();
    }
    // This row's check-to-variable messages (none in the first iteration).
    constexpr int ND = (W + 1) / 2;
    const int nd = GEN ? (wr + 1) / 2 : ND;
    uint32_t rd[ND];
    if (FIRST) {
#pragma unroll
        for (int j = 0; j < ND; ++j) rd[j] = 0;
    } else if (IN_LDS) {
        R.template load<W>(rd, u, Z, wrow);
    } else {
#pragma unroll
        for (int j = 0; j < ND && j < kPreDwords; ++j) rd[j] = pre[j];
        if (GEN)
            R.template load_rt<ND, kPreDwords>(rd, u, nd);
        else if (ND > kPreDwords)
            R.template load<W, kPreDwords>(rd, u, Z);
        if (R.rmask_on) {
#pragma unroll
            for (int j = 0; j < ND; ++j) rd[j] &= R.rmask;
        }
    }
    uint32_t xv[W], axv[W], la[W], ps[RP ? W : 1];
    u16x2 m1 = {0x7FFF, 0x7FFF}, m2 = {0x7FFF, 0x7FFF};
    uint32_t S = 0;
    if constexpr (kWide) {
        constexpr int H = (W + 1) / 2;
        row_phase1<0, H, false, RP>(smem, lb, rd, md, mo, u, Z, wrow, xv, axv, la, ps, m1, m2, S);
        // keep the halves apart: the scheduler would otherwise issue every
        // read of the row up front and hold both halves' registers at once
        __builtin_amdgcn_sched_barrier(0);
        row_phase1<H, W, false, RP>(smem, lb, rd, md, mo, u, Z, wrow, xv, axv, la, ps, m1, m2, S);
    } else {
        row_phase1<0, W, true, RP>(smem, lb, rd, md, mo, u, Z, wrow, xv, axv, la, ps, m1, m2, S);
    }
    const u16x2 a1 = normalise(m1, off16, wgt);
    const u16x2 a2 = normalise(m2, off16, wgt);
    // b = (-1)^S * a: the message with the row's sign product applied; each
    // edge then takes sgn(x_k) * b_k, which removes its own sign from S.
    const s16x2 Sm = as_s(S) >> (s16x2){15, 15};
    const s16x2 b1 = (as_s(bits_of(a1)) ^ Sm) - Sm;
    const s16x2 b2 = (as_s(bits_of(a2)) ^ Sm) - Sm;
    const u16x2 d21 = as_u(bits_of(b2 - b1));
    const u16x2 m1p = m1 + (u16x2){1, 1};
    uint32_t sd[ND];
    uint32_t rprev = 0;
    if constexpr (!kWide && !GEN) {
        // Narrow rows: each step over all edges at once (the edges are
        // independent), so dependent packed operations are not adjacent.
        s16x2 Rv[W], Lv[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const u16x2 t = __builtin_elementwise_sub_sat(m1p, as_u(axv[k]));
            Rv[k] = as_s(bits_of(t * d21 + as_u(bits_of(b1))));
        }
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const s16x2 sx = as_s(xv[k]) >> (s16x2){15, 15};
            Rv[k] = (Rv[k] ^ sx) - sx;
        }
#pragma unroll
        for (int k = 0; k < W; ++k)
            Lv[k] = __builtin_elementwise_max(__builtin_elementwise_add_sat(as_s(xv[k]), Rv[k]),
                                              (s16x2){-127 * 256, -127 * 256});
#pragma unroll
        for (int k = 0; k < W; ++k) lds_st16(smem, la[k], perm(bits_of(Lv[k]), RP ? ps[k] : kPack));
#pragma unroll
        for (int j = 0; j < ND; ++j)
            sd[j] = 2 * j + 1 < W ? __builtin_amdgcn_perm(bits_of(Rv[2 * j + 1]), bits_of(Rv[2 * j]), kPack2)
                                  : perm(bits_of(Rv[2 * j]), kPack);
#pragma unroll
        for (int c = 0; c < ND; c += 4) R.template store<W>(sd, u, Z, c, ND - c < 4 ? ND - c : 4);
        return;
    }
    // Wide rows: the same steps over groups of four edges (a group's values
    // stay in registers; the whole row's would not).
#pragma unroll
    for (int g = 0; g < W; g += 4) {
        s16x2 Rg[4], Lg[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = g + i;
            if (k >= W || k >= wrow) continue;
            const s16x2 x = as_s(xv[k]);
            const s16x2 ax = kWide ? __builtin_elementwise_max(x, (s16x2){0, 0} - x) : as_s(axv[k]);
            // t = 1 on the argmin edge (|x| == m1), else 0.
            const u16x2 t = __builtin_elementwise_sub_sat(m1p, as_u(bits_of(ax)));
            Rg[i] = as_s(bits_of(t * d21 + as_u(bits_of(b1))));
        }
        // R' = sgn(x) * b; L' = sat(x + R'). The low byte of x is 0 or 0xFF
        // and that of R' is 0, so no carry reaches the high byte.
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = g + i;
            if (k >= W || k >= wrow) continue;
            const s16x2 sx = as_s(xv[k]) >> (s16x2){15, 15};
            Rg[i] = (Rg[i] ^ sx) - sx;
            Lg[i] = __builtin_elementwise_max(__builtin_elementwise_add_sat(as_s(xv[k]), Rg[i]),
                                              (s16x2){-127 * 256, -127 * 256});
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = g + i;
            if (k >= W || k >= wrow) continue;
            const uint32_t a =
                kWide ? gather(md[k], mo[k], lb, lane_key(u), (uint32_t)Z) : la[k];
            uint32_t psel = kPack;
            if constexpr (RP)
                psel = kWide ? (rp_swapped(md[k], lane_key(u)) ? kPackSw : kPack) : ps[k];
            lds_st16(smem, a, perm(bits_of(Lg[i]), psel));
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = g + i;
            if (k >= W || k >= wrow) continue;
            const s16x2 Rn = Rg[i];
            // messages k-1 and k share a dword (an odd row's last dword pads
            // with a zero pair word); store each group of 4 dwords once complete
            const int j = k >> 1;
            if (k & 1) {
                sd[j] = __builtin_amdgcn_perm(bits_of(Rn), rprev, kPack2);
            } else {
                rprev = bits_of(Rn);
                if (k == wrow - 1) sd[j] = perm(bits_of(Rn), kPack);
            }
            if (GEN && IN_LDS) {
                if ((k & 1) || k == wrow - 1) R.template store<W>(sd, u, Z, j, 1, wrow);
            } else if (GEN) {
                if ((k & 1) || k == wrow - 1) {
                    if ((j & 3) == 3) R.store_rt(sd, u, nd, j & ~3, 4);
                    else if (j == nd - 1) R.store_rt(sd, u, nd, j & ~3, nd - (j & ~3));
                }
            } else if ((k & 1) || k == W - 1) {
                if ((j & 3) == 3) R.template store<W>(sd, u, Z, j & ~3, 4);
                else if (j == ND - 1) R.template store<W>(sd, u, Z, j & ~3, ND - (j & ~3));
            }
        }
    }
}

// Parity of check row u over a row of exactly W blocks for both codewords:
// the XOR of the raw pair words, whose bits 7 and 15 are the hard decisions
// [L_v < 0] of the two codewords.
// RP (row-pair layout): each word is unpacked in its lane's row order
// first, so the hard decisions of rows u and u + Zh land in bits 15 and 31.
template <int W, bool RP = false>
__device__ __forceinline__ uint32_t row_parity_w(const uint8_t *__restrict__ smem, uint32_t lb,
                                                 cmeta_t meta, int e0, uint32_t u, int Z) {
    uint32_t md[W], mo[W], raw[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        md[k] = meta[e0 + k];
        mo[k] = md[k] & off_mask<RP>();
    }
#pragma unroll
    for (int k = 0; k < W; ++k)
        raw[k] = lds_ld16(smem, gather(md[k], mo[k], lb, lane_key(u), (uint32_t)Z));
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        if constexpr (RP)
            acc ^= perm(raw[k], rp_swapped(md[k], lane_key(u)) ? kUnpackSw : kUnpack);
        else
            acc ^= raw[k];
    }
    return acc;
}

// Scalar dispatch on the row weight w in [W, WMAX].
template <int W, int WMAX, bool IN_LDS, bool FIRST, bool RP = false>
__device__ __forceinline__ void row_update(int w, uint8_t *smem, uint32_t lb,
                                           const MsgRow<IN_LDS> &R, cmeta_t meta, int e0,
                                           uint32_t u, int Z, u16x2 wgt, u16x2 off16,
                                           const uint32_t *pre) {
    if constexpr (W <= WMAX) {
        if (w == W) {
            row_update_w<W, IN_LDS, FIRST, false, RP>(smem, lb, R, meta, e0, u, Z, wgt, off16,
                                                      pre);
            return;
        }
        row_update<W + 1, WMAX, IN_LDS, FIRST, RP>(w, smem, lb, R, meta, e0, u, Z, wgt, off16,
                                                   pre);
    }
}

// Row update for any weight up to WMAX: exact code for weights up to 10
// (and 19, the core rows of BG1-shaped graphs); other wide rows run through
// one bound-WMAX body with scalar guards, which keeps the kernel's register
// allocation to a few row shapes.
template <int WMAX, bool IN_LDS, bool FIRST, bool RP = false>
__device__ __forceinline__ void row_update_any(int w, uint8_t *smem, uint32_t lb,
                                               const MsgRow<IN_LDS> &R, cmeta_t meta, int e0,
                                               uint32_t u, int Z, u16x2 wgt, u16x2 off16,
                                               const uint32_t *pre) {
    if constexpr (WMAX <= 10) {
        row_update<2, WMAX, IN_LDS, FIRST, RP>(w, smem, lb, R, meta, e0, u, Z, wgt, off16, pre);
    } else {
        constexpr int kCore = WMAX >= 19 ? 19 : WMAX;
        if (w <= 10)
            row_update<2, 10, IN_LDS, FIRST, RP>(w, smem, lb, R, meta, e0, u, Z, wgt, off16, pre);
        else if (w == kCore)
            row_update_w<kCore, IN_LDS, FIRST, false, RP>(smem, lb, R, meta, e0, u, Z, wgt, off16,
                                                          pre);
        else
            row_update_w<WMAX, IN_LDS, FIRST, true, RP>(smem, lb, R, meta, e0, u, Z, wgt, off16,
                                                        pre, w);
    }
}

template <int W, int WMAX, bool RP = false>
__device__ __forceinline__ uint32_t row_parity(int w, const uint8_t *smem, uint32_t lb,
                                               cmeta_t meta, int e0, uint32_t u, int Z) {
    if constexpr (W <= WMAX) {
        if (w == W) return row_parity_w<W, RP>(smem, lb, meta, e0, u, Z);
        return row_parity<W + 1, WMAX, RP>(w, smem, lb, meta, e0, u, Z);
    }
    return 0;
}

// Syndrome check of the pair's unfinished codewords (needA: codeword 2p,
// needB: 2p+1): a failing check of row u marks its codeword in fl[0] /
// fl[1] (the pair's LDS flags, zero on entry; every marking lane stores the
// same 1). One failing check decides a codeword, so a wave stops sweeping
// the rows as soon as every codeword its lanes serve is decided (marked by
// any wave) -- only codewords whose checks all hold need the full sweep,
// which keeps the check cheap in the iterations before convergence.
// RP: rows u and u + Zh of one codeword (needA), either failing marks fl[0].
template <int WMAX, bool RP = false>
__device__ __forceinline__ void syndrome_mark(const uint8_t *__restrict__ smem, uint32_t lb,
                                     crow_t row_ptr, cmeta_t meta, int rows, uint32_t u, int Z,
                                     volatile int *fl, bool needA, bool needB) {
    for (int r = 0; r < rows; ++r) {
        const int e0 = row_ptr[r], w = row_ptr[r + 1] - e0;
        const uint32_t par = row_parity<2, WMAX, RP>(w, smem, lb, meta, e0, u, Z);
        if (needA && (par & (RP ? 0x80008000u : 0x80u))) fl[0] = 1;
        if (needB && (par & 0x8000u)) fl[1] = 1;
        const bool open = (needA && fl[0] == 0) || (needB && fl[1] == 0);
        if (__ballot(open) == 0) break;
    }
}

// Outputs of the pair's codewords selected by `which` (bit 0: codeword 2p,
// bit 1: 2p+1) from the current posteriors: hard decisions of the K
// information bits packed LSB first (byte j of a column covers variables
// 8j..8j+7, one 16-byte LDS read of pair words), iteration count, syndrome
// flag and optionally the posteriors. Lanes of the pair share the work.
__device__ inline void write_outputs(const BlockWork &bw, const uint8_t *Lp, int pair,
                                     uint32_t u, int which, int iters, int okA, int okB) {
    // An opaque copy of the pair index: keeps the compiler from hoisting
    // this (rarely run) output addressing out of the iteration loop, where
    // it would hold registers through every layer.
    int Z = bw.Z;
    __asm__ volatile("" : "+v"(pair), "+v"(u), "+s"(Z));
    const int bpc = Z / 8, nbytes = bw.kb * bpc;
    const int kbytes = bw.kb * Z / 8;
    const int cw0 = 2 * pair;
#pragma unroll 1
    for (int i = (int)u; i < nbytes; i += Z) {
        const int c = i / bpc, j = i - c * bpc;
        const uint2 *w2 = reinterpret_cast<const uint2 *>(Lp + 2 * (c * Z + 8 * j));
        uint32_t ba = 0, bb = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint2 w = w2[h];
            const uint32_t d0 = w.x, d1 = w.y;
            ba |= (((d0 >> 7) & 1u) | ((d0 >> 22) & 2u) | ((d1 << 2) >> 7 & 4u) |
                   ((d1 >> 20) & 8u)) << (4 * h);
            bb |= (((d0 >> 15) & 1u) | ((d0 >> 30) & 2u) | ((d1 >> 13) & 4u) |
                   ((d1 >> 28) & 8u)) << (4 * h);
        }
        if (which & 1) bw.out_bits[(size_t)cw0 * kbytes + i] = (uint8_t)ba;
        if (which & 2) bw.out_bits[(size_t)(cw0 + 1) * kbytes + i] = (uint8_t)bb;
    }
    if (u == 0) {
        if (which & 1) {
            bw.out_iters[cw0] = iters;
            if (bw.out_ok) bw.out_ok[cw0] = (uint8_t)okA;
        }
        if (which & 2) {
            bw.out_iters[cw0 + 1] = iters;
            if (bw.out_ok) bw.out_ok[cw0 + 1] = (uint8_t)okB;
        }
    }
    if (bw.out_llr) {
        const int Nc = bw.n_cols * Z;
        const uint16_t *Lw = reinterpret_cast<const uint16_t *>(Lp);
#pragma unroll 1
        for (int c = 0; c < bw.n_cols; ++c) {
            const uint16_t v = Lw[c * Z + u];
            if (which & 1) bw.out_llr[(size_t)cw0 * Nc + c * Z + u] = (int8_t)(v & 0xFF);
            if (which & 2) bw.out_llr[(size_t)(cw0 + 1) * Nc + c * Z + u] = (int8_t)(v >> 8);
        }
    }
}

// Outputs of the pair's halves that hold codewords cwA / cwB (absolute
// indices from bw's output bases; -1 = nothing to write for that half),
// each with its own iteration count and syndrome flag. Same packing as
// write_outputs.
__device__ inline void write_outputs_ids(const BlockWork &bw, const uint8_t *Lp, uint32_t u,
                                         int cwA, int cwB, int itA, int itB, int okA, int okB) {
    int Z = bw.Z;
    __asm__ volatile("" : "+v"(cwA), "+v"(cwB), "+v"(u), "+s"(Z));
    const int bpc = Z / 8, nbytes = bw.kb * bpc;
    const int kbytes = bw.kb * Z / 8;
#pragma unroll 1
    for (int i = (int)u; i < nbytes; i += Z) {
        const int c = i / bpc, j = i - c * bpc;
        const uint2 *w2 = reinterpret_cast<const uint2 *>(Lp + 2 * (c * Z + 8 * j));
        uint32_t ba = 0, bb = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint2 w = w2[h];
            const uint32_t d0 = w.x, d1 = w.y;
            ba |= (((d0 >> 7) & 1u) | ((d0 >> 22) & 2u) | ((d1 << 2) >> 7 & 4u) |
                   ((d1 >> 20) & 8u)) << (4 * h);
            bb |= (((d0 >> 15) & 1u) | ((d0 >> 30) & 2u) | ((d1 >> 13) & 4u) |
                   ((d1 >> 28) & 8u)) << (4 * h);
        }
        if (cwA >= 0) bw.out_bits[(size_t)cwA * kbytes + i] = (uint8_t)ba;
        if (cwB >= 0) bw.out_bits[(size_t)cwB * kbytes + i] = (uint8_t)bb;
    }
    if (u == 0) {
        if (cwA >= 0) {
            bw.out_iters[cwA] = itA;
            if (bw.out_ok) bw.out_ok[cwA] = (uint8_t)okA;
        }
        if (cwB >= 0) {
            bw.out_iters[cwB] = itB;
            if (bw.out_ok) bw.out_ok[cwB] = (uint8_t)okB;
        }
    }
    if (bw.out_llr) {
        const int Nc = bw.n_cols * Z;
        const uint16_t *Lw = reinterpret_cast<const uint16_t *>(Lp);
#pragma unroll 1
        for (int c = 0; c < bw.n_cols; ++c) {
            const uint16_t v = Lw[c * Z + u];
            if (cwA >= 0) bw.out_llr[(size_t)cwA * Nc + c * Z + u] = (int8_t)(v & 0xFF);
            if (cwB >= 0) bw.out_llr[(size_t)cwB * Nc + c * Z + u] = (int8_t)(v >> 8);
        }
    }
}

// Row-pair layout: one codeword's channel LLRs into its pair words (word p
// of column c: variable p in the low byte, p + Zh in the high byte; the
// punctured columns 0 and 1 at zero), clamped at -127. The codeword's Zh
// lanes read its (N - 2) Z bytes as consecutive dwords, lane u taking
// dwords u, u + Zh, ...: dword k*Zh + u starts at byte 2k*Z + 4u, i.e.
// column 2 + 2k (+1 once 4u >= Z), variable 4u mod Z, and its four bytes
// (Z a multiple of 8) share one column and one half of the pair words, so
// each lane's destinations are a fixed LDS byte plus 4*Zh per k and 2 per
// byte.
template <int KB>
__device__ inline void load_rp_llrs(uint8_t *Lc, const int8_t *q, int N, int Z, uint32_t u) {
    const int Zh = Z >> 1;
    uint16_t *Lw = reinterpret_cast<uint16_t *>(Lc);
    Lw[u] = 0;
    Lw[Zh + (int)u] = 0;
    const int nd = (N - 2) * Z / 4;
    const int kmax = (N - 1) / 2;  // ceil((N - 2) / 2) dwords per lane at most
    const int cu = 4 * (int)u >= Z ? 1 : 0, v = 4 * (int)u - cu * Z, hi = v >= Zh ? 1 : 0;
    uint8_t *dst0 = Lc + 2 * ((2 + cu) * Zh + v - hi * Zh) + hi;
    const uint32_t *q32 = reinterpret_cast<const uint32_t *>(q);
#pragma unroll 1
    for (int k0 = 0; k0 < kmax; k0 += KB) {
        uint32_t d[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int idx = (k0 + k) * Zh + (int)u;
            d[k] = q32[idx < nd ? idx : nd - 1];
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            if ((k0 + k) * Zh + (int)u < nd) {
                uint8_t *dst = dst0 + 4 * Zh * (k0 + k);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int x = (int)(int8_t)(d[k] >> (8 * b));
                    dst[2 * b] = (uint8_t)(x < -127 ? -127 : x);
                }
            }
        }
    }
}

// Row-pair layout: outputs of codeword cw (index from bw's output bases)
// from its pair words Lc; bw.Z is Zh. Same output formats as write_outputs.
__device__ inline void write_outputs_rp(const BlockWork &bw, const uint8_t *Lc, int cw,
                                        uint32_t u, int iters, int ok) {
    int Zh = bw.Z;
    __asm__ volatile("" : "+v"(cw), "+v"(u), "+s"(Zh));
    const int Z = 2 * Zh, bpc = Z / 8, nbytes = bw.kb * bpc;
#pragma unroll 1
    for (int i = (int)u; i < nbytes; i += Zh) {
        const int c = i / bpc, j = i - c * bpc;
        uint32_t byte = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int v = 8 * j + b, hi = v >= Zh ? 1 : 0;
            byte |= (uint32_t)(Lc[2 * (c * Zh + v - hi * Zh) + hi] >> 7) << b;
        }
        bw.out_bits[(size_t)cw * nbytes + i] = (uint8_t)byte;
    }
    if (u == 0) {
        bw.out_iters[cw] = iters;
        if (bw.out_ok) bw.out_ok[cw] = (uint8_t)ok;
    }
    if (bw.out_llr) {
        const int Nc = bw.n_cols * Z;
        const uint16_t *Lw = reinterpret_cast<const uint16_t *>(Lc);
#pragma unroll 1
        for (int c = 0; c < bw.n_cols; ++c) {
            const uint16_t w = Lw[c * Zh + (int)u];
            bw.out_llr[(size_t)cw * Nc + c * Z + u] = (int8_t)(w & 0xFF);
            bw.out_llr[(size_t)cw * Nc + c * Z + u + Zh] = (int8_t)(w >> 8);
        }
    }
}

typedef const __attribute__((address_space(4))) uint32_t *cw32_t;

// Synchronisation of the lanes that decode one block of work: the whole
// workgroup, or (WAVE) a single wave that owns its block alone -- a wave's
// LDS accesses are performed in order, so a wave-scope fence that the
// compiler may not move accesses across is enough.
template <bool WAVE>
__device__ inline void block_sync() {
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// Q1.7 weight of row r from a per-row byte table in the constant address
// space, read as the aligned dword that holds it (a scalar load; the dword
// never crosses the page of the byte it holds).
__device__ inline int row_weight(const uint8_t *wrow, int r) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(wrow + r);
    const uint32_t word = *reinterpret_cast<cw32_t>(a & ~(uintptr_t)3);
    return (int)((word >> (8u * (uint32_t)(a & 3u))) & 0xFFu);
}

// Message row of block row r: LDS placement from the row's first edge e0,
// device placement from its padded start p0.
template <bool IN_LDS>
__device__ inline MsgRow<IN_LDS> msg_row(uint8_t *smem, uint32_t ro,
                                         __amdgpu_buffer_rsrc_t rsrc, int e0, int p0, int Z) {
    MsgRow<IN_LDS> R{rsrc, nullptr, 0u, 0u, true, false, 0xFFFFFFFFu};
    if (IN_LDS) {
        R.lds = smem;
        R.ro = ro + 2u * (uint32_t)(e0 * Z);
    } else {
        R.ro = ro;
        R.row = 2u * (uint32_t)(p0 * Z);
    }
    return R;
}

// One iteration's sweep over the block rows (layers) in order, a workgroup
// barrier between layers that share a block column. wrow: this iteration's
// per-row Q1.7 weights or null (bw.beta for every row). keep: whether the
// check-to-variable messages are stored (not in the last iteration).
template <int WMAX, bool IN_LDS, bool FIRST, bool WAVE, bool RP = false>
__device__ __forceinline__ void layer_pass(const BlockWork &bw, uint8_t *smem, uint32_t lb,
                                           uint32_t ro, __amdgpu_buffer_rsrc_t rsrc,
                                           crow_t row_ptr, cmeta_t meta, const uint8_t *wrow,
                                           uint32_t u, bool busy, u16x2 off16, uint32_t *pre,
                                           bool keep, bool rmask_on = false,
                                           uint32_t rmask = 0xFFFFFFFFu) {
    const int Z = bw.Z;
    crow_t row_pad = (crow_t)bw.row_pad;
    // a barrier only where the next row shares a column with the rows since
    // the last one (layer groups), and after the last row
    const uint64_t bar = (bw.groups >> 1) | (1ull << (bw.rows - 1));
    // Row bounds travel one row ahead in scalar registers, so a row's block
    // metadata loads need not wait for its bounds after the barrier.
    int e0 = row_ptr[0], e1 = row_ptr[1], p0 = IN_LDS ? 0 : row_pad[0];
    int p1 = IN_LDS ? 0 : row_pad[1];
    for (int r = 0; r < bw.rows; ++r) {
        // the next row: r + 1, or row 0 of the next iteration; its messages
        // exist once this is not the first iteration, or for row 0
        const bool last = r + 1 == bw.rows;
        const int rn = last ? 0 : r + 1;
        const int e2 = last ? row_ptr[1] : row_ptr[r + 2];
        const int p2 = IN_LDS ? 0 : (last ? row_pad[1] : row_pad[r + 2]);
        const int en = last ? row_ptr[0] : e1, pn = IN_LDS ? 0 : (last ? row_pad[0] : p1);
        const int w = e1 - e0;
        const int wt = wrow ? row_weight(wrow, r) : bw.beta;
        const u16x2 wgt = {(unsigned short)wt, (unsigned short)wt};
        MsgRow<IN_LDS> R = msg_row<IN_LDS>(smem, ro, rsrc, e0, p0, Z);
        R.keep = keep;
        R.rmask_on = rmask_on;
        R.rmask = rmask;
        if (busy) {
            row_update_any<WMAX, IN_LDS, FIRST, RP>(w, smem, lb, R, meta, e0, u, Z, wgt, off16,
                                                    pre);
            // the next row's messages exist unless this is the first
            // iteration; after the last row, only if another iteration runs
            if (!IN_LDS && (last ? keep : !FIRST))
                msg_row<IN_LDS>(smem, ro, rsrc, 0, pn, Z).load4(pre, u, (p2 - pn) / 2);
        }
        if ((bar >> r) & 1) block_sync<WAVE>();
        e0 = en;
        e1 = e2;
        p0 = pn;
        p1 = p2;
        (void)rn;
    }
}

// One codeword's channel LLRs into one half of a pair's words (half 0: the
// low bytes, codeword 2p; half 1: the high bytes), clamped at -127, with
// the punctured columns 0 and 1 at zero; q == nullptr (no codeword) writes
// zeros. The pair's Z lanes read the codeword's (N - 2) Z bytes as
// consecutive dwords (lane u takes dwords u, u + Z, u + 2Z, ...: every load
// coalesced, KB of a lane's loads in flight together) and scatter the
// bytes to their pair words: LLR byte j is variable 2Z + j, LDS byte
// 2 (2Z + j) + half. KB trades registers for round trips: a whole codeword
// (up to 17 dwords per lane) is one round trip.
template <int KB>
__device__ inline void load_half_llrs(uint8_t *Lpair, int half, const int8_t *q, int N, int Z,
                                      uint32_t u) {
    constexpr int kMaxK = (68 - 2 + 3) / 4 + 1;  // dwords per lane for up to 68 columns
    uint8_t *Lh = Lpair + half;
    Lh[2 * u] = 0;
    Lh[2 * (Z + (int)u)] = 0;
    const int nd = (N - 2) * Z / 4;  // Z is a multiple of 8
    const uint32_t *q32 = reinterpret_cast<const uint32_t *>(q);
#pragma unroll 1
    for (int k0 = 0; k0 < kMaxK; k0 += KB) {
        if (k0 * Z >= nd) break;
        uint32_t v[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int idx = (k0 + k) * Z + (int)u;
            v[k] = q ? q32[idx < nd ? idx : nd - 1] : 0u;
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int idx = (k0 + k) * Z + (int)u;
            if (idx < nd) {
                uint8_t *dst = Lh + 2 * (2 * Z + 4 * idx);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int x = (int)(int8_t)(v[k] >> (8 * b));
                    dst[2 * b] = (uint8_t)(x < -127 ? -127 : x);
                }
            }
        }
    }
}

// Decodes `bw.n` codewords of one shape in this workgroup as bw.slots pairs
// (lanes beyond the last valid pair only join the barriers; the partner of
// an odd last codeword decodes all-zero inputs and writes nothing). Every
// thread of the workgroup must call it.
// IN_LDS: the check-to-variable messages live next to the posteriors in
// LDS; otherwise they stream through device memory (bw.msg, [pair][E][Z]
// pair words) and only the posteriors occupy LDS, so several pairs share a
// CU (§IV's placement of L_v in shared and L_{c->v} in main memory).
// WAVE: one wave decodes the block by itself (lanes = threadIdx.x mod 64,
// Z <= 64) and synchronises only itself, so the other waves of the
// workgroup may decode other blocks of other shapes at the same time.
template <int WMAX, bool IN_LDS, bool WAVE = false>
__device__ __forceinline__ void decode_block(const BlockWork &bw, uint8_t *smem, crow_t row_ptr,
                                             cmeta_t meta) {
    static_assert(WMAX <= kMetaPad, "row metadata window exceeds the table padding");
    const int Z = bw.Z;
    const int N = bw.n_cols, E = bw.E, T = (N - 2) * Z;
    const int pair_bytes = IN_LDS ? lds_bytes_i8_pair(N, E, Z) : lds_bytes_i8_pair_post(N, Z);
    const int tid = WAVE ? (int)(threadIdx.x & 63u) : (int)threadIdx.x;
    const int p = tid / Z;
    const uint32_t u = tid - p * Z;
    const bool validA = 2 * p < bw.n, validB = 2 * p + 1 < bw.n;
    const int ps = validA ? p : 0;  // keeps idle lanes' addresses in range
    uint8_t *Lp = smem + ps * pair_bytes;
    uint16_t *Lw = reinterpret_cast<uint16_t *>(Lp);
    const uint32_t lb = (uint32_t)(ps * pair_bytes) + 2u * u;
    uint32_t ro;
    if (IN_LDS)
        ro = (uint32_t)(ps * pair_bytes + 2 * N * Z) + 2u * u;
    else
        ro = 2u * (uint32_t)(ps * bw.E_pad * Z);
    int *flags = reinterpret_cast<int *>(smem + bw.slots * pair_bytes);
    // The workgroup's message region as a raw buffer (dword 3 = 0x00020000:
    // untyped 32-bit data format for gfx9 raw buffer access).
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(bw.msg, 0, IN_LDS ? 0 : bw.msg_records, 0x00020000);

    // Initialisation: the pair's channel LLRs (punctured columns 0 and 1
    // carry none).
    if (validA) {
        load_half_llrs<17>(Lp, 0, bw.llr + (size_t)(2 * p) * T, N, Z, u);
        load_half_llrs<17>(Lp, 1, validB ? bw.llr + (size_t)(2 * p + 1) * T : nullptr, N, Z, u);
    }
    block_sync<WAVE>();

    const u16x2 off16 = {(unsigned short)(bw.offset << 8), (unsigned short)(bw.offset << 8)};
    bool doneA = !validA, doneB = !validB;
    uint32_t pre[kPreDwords] = {0u, 0u, 0u, 0u};
    for (int t = 1; t <= bw.max_iter; ++t) {
        const uint8_t *wrow = nullptr;
        if (bw.wq) wrow = bw.wq + (size_t)((t < bw.w_iters ? t : bw.w_iters) - 1) * bw.w_stride;
        const bool busy = !(doneA && doneB);
        // the first iteration has no check-to-variable messages yet
        if (t == 1)
            layer_pass<WMAX, IN_LDS, true, WAVE>(bw, smem, lb, ro, rsrc, row_ptr, meta, wrow, u, busy,
                                           off16, pre, t < bw.max_iter);
        else
            layer_pass<WMAX, IN_LDS, false, WAVE>(bw, smem, lb, ro, rsrc, row_ptr, meta, wrow, u, busy,
                                            off16, pre, t < bw.max_iter);
        if (bw.early_exit || t == bw.max_iter) {
            // flags[0, 2*slots): a failing check per codeword; flags[2*slots]:
            // stays 1 while every codeword of the workgroup is finished
            if (tid <= 2 * bw.slots) flags[tid] = tid == 2 * bw.slots;
            block_sync<WAVE>();
            if (busy)
                syndrome_mark<WMAX>(smem, lb, row_ptr, meta, bw.rows, u, Z, flags + 2 * p, !doneA,
                                    !doneB);
            block_sync<WAVE>();
            const bool holdsA = flags[2 * ps] == 0, holdsB = flags[2 * ps + 1] == 0;
            bool finA = false, finB = false;
            if (t == bw.max_iter) {
                finA = !doneA;
                finB = !doneB;
            } else {
                finA = !doneA && holdsA;
                finB = !doneB && holdsB;
            }
            if (finA || finB)
                write_outputs(bw, Lp, p, u, (finA ? 1 : 0) | (finB ? 2 : 0), t, holdsA, holdsB);
            doneA = doneA || finA;
            doneB = doneB || finB;
            if (!(doneA && doneB)) flags[2 * bw.slots] = 0;
            block_sync<WAVE>();
            if (flags[2 * bw.slots]) break;
        }
    }
}

// Row-pair decoding (§II: the Z check rows of a block row are independent):
// codeword i of the workgroup's bw.n occupies lanes [i*Zh, (i+1)*Zh), Zh =
// Z/2 = bw.Z, and lane u updates its check rows u and u + Zh as the two
// halves of its packed registers, the same arithmetic as the pair kernel
// (the pair kernel with Zh lanes, the row-pair metadata and per-edge
// unpack / pack selectors). For small batches of large lifts: a pair's 2Z
// lanes would put two waves on some SIMDs of a CU, where one codeword's Zh
// lanes leave every wave a SIMD of its own. Device-placed messages,
// [codeword][E_pad * Zh] pair words. Every thread of the workgroup must
// call it; lanes past the last codeword only join the barriers.
template <int WMAX, bool IN_LDS = false>
__device__ __forceinline__ void decode_rp(const BlockWork &bw, uint8_t *smem, crow_t row_ptr,
                                          cmeta_t meta) {
    static_assert(WMAX <= kMetaPad, "row metadata window exceeds the table padding");
    const int Zh = bw.Z, Z = 2 * Zh;
    const int N = bw.n_cols, T = (N - 2) * Z;
    // a codeword's LDS: its posteriors, then (IN_LDS) its messages as
    // [edge][Zh] pair words
    const int cw_bytes = IN_LDS ? lds_bytes_i8_pair(N, bw.E, Zh) : lds_bytes_i8_pair_post(N, Zh);
    const int tid = (int)threadIdx.x;
    const int i = tid / Zh;
    const uint32_t u = tid - i * Zh;
    const bool valid = i < bw.n;
    const int is = valid ? i : 0;  // keeps idle lanes' addresses in range
    uint8_t *Lc = smem + is * cw_bytes;
    const uint32_t lb = (uint32_t)(is * cw_bytes) + 2u * u;
    const uint32_t ro = IN_LDS ? (uint32_t)(is * cw_bytes + 2 * N * Zh) + 2u * u
                               : 2u * (uint32_t)(is * bw.E_pad * Zh);
    int *flags = reinterpret_cast<int *>(smem + bw.slots * cw_bytes);
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(bw.msg, 0, IN_LDS ? 0 : bw.msg_records, 0x00020000);
    if (valid) load_rp_llrs<17>(Lc, bw.llr + (size_t)i * T, N, Z, u);
    __syncthreads();

    const u16x2 off16 = {(unsigned short)(bw.offset << 8), (unsigned short)(bw.offset << 8)};
    bool done = !valid;
    uint32_t pre[kPreDwords] = {0u, 0u, 0u, 0u};
    for (int t = 1; t <= bw.max_iter; ++t) {
        const uint8_t *wrow = nullptr;
        if (bw.wq) wrow = bw.wq + (size_t)((t < bw.w_iters ? t : bw.w_iters) - 1) * bw.w_stride;
        const bool busy = !done;
        if (t == 1)
            layer_pass<WMAX, IN_LDS, true, false, true>(bw, smem, lb, ro, rsrc, row_ptr, meta,
                                                        wrow, u, busy, off16, pre,
                                                        t < bw.max_iter);
        else
            layer_pass<WMAX, IN_LDS, false, false, true>(bw, smem, lb, ro, rsrc, row_ptr, meta,
                                                         wrow, u, busy, off16, pre,
                                                         t < bw.max_iter);
        if (bw.early_exit || t == bw.max_iter) {
            // flags[0, slots): a failing check per codeword; flags[slots]:
            // stays 1 while every codeword of the workgroup is finished
            if (tid <= bw.slots) flags[tid] = tid == bw.slots;
            __syncthreads();
            if (busy)
                syndrome_mark<WMAX, true>(smem, lb, row_ptr, meta, bw.rows, u, Zh, flags + i, true,
                                          false);
            __syncthreads();
            const bool holds = flags[is] == 0;
            const bool fin = !done && (t == bw.max_iter || holds);
            if (fin) write_outputs_rp(bw, Lc, i, u, t, holds);
            done = done || fin;
            if (!done) flags[bw.slots] = 0;
            __syncthreads();
            if (flags[bw.slots]) break;
        }
    }
}

// Persistent schedule for int8 decodes with early exit and device-placed
// messages: the grid holds only as many workgroups as run at once, and each
// half of each codeword pair takes the next codeword from a device counter
// as soon as its own finishes (all checks hold, or max_iter), so no lane
// waits for a slower partner or for the slowest codeword of its block, and
// no workgroup waits for the launch's last wave of blocks. A fresh half
// starts at its iteration 1 while its partner continues: its posteriors
// are loaded over its bytes of the pair words, and in its first round its
// bytes of every message dword this lane loads (those of the codeword
// before) are masked to zero, so it reads zero messages exactly as a
// codeword that starts with its pair. Every half's arithmetic depends only on its own codeword,
// so the results are those of any other schedule. Plain normalisation only
// (per-iteration weights would differ between the halves). The loop ends
// once no half holds a codeword; each round advances every held codeword
// by one iteration and the counter only grows, so it ends after at most
// max_iter rounds per codeword handed to the workgroup.
template <int WMAX>
__device__ __forceinline__ void decode_refill(const BlockWork &bw, uint8_t *smem, crow_t row_ptr,
                                              cmeta_t meta, unsigned *counter, int n_total) {
    static_assert(WMAX <= kMetaPad, "row metadata window exceeds the table padding");
    const int Z = bw.Z;
    const int N = bw.n_cols, T = (N - 2) * Z;
    const int pair_bytes = lds_bytes_i8_pair_post(N, Z);
    const int tid = (int)threadIdx.x;
    const int p = tid / Z;
    const uint32_t u = tid - p * Z;
    uint8_t *Lp = smem + p * pair_bytes;
    uint16_t *Lw = reinterpret_cast<uint16_t *>(Lp);
    const uint32_t lb = (uint32_t)(p * pair_bytes) + 2u * u;
    const uint32_t ro = 2u * (uint32_t)(p * bw.E_pad * Z);
    int *flags = reinterpret_cast<int *>(smem + bw.slots * pair_bytes);
    int *held = flags + 2 * bw.slots + 2;  // codeword index per half, -1 = none
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(bw.msg, 0, bw.msg_records, 0x00020000);
    crow_t row_pad = (crow_t)bw.row_pad;

    if (tid == 0) {
        const int want = 2 * bw.slots;
        const unsigned base = atomicAdd(counter, (unsigned)want);
        for (int h = 0; h < want; ++h)
            held[h] = (long)base + h < (long)n_total ? (int)(base + (unsigned)h) : -1;
    }
    __syncthreads();
    int idA = held[2 * p], idB = held[2 * p + 1];
    load_half_llrs<4>(Lp, 0, idA >= 0 ? bw.llr + (size_t)idA * T : nullptr, N, Z, u);
    load_half_llrs<4>(Lp, 1, idB >= 0 ? bw.llr + (size_t)idB * T : nullptr, N, Z, u);
    __syncthreads();

    const u16x2 off16 = {(unsigned short)(bw.offset << 8), (unsigned short)(bw.offset << 8)};
    uint32_t pre[kPreDwords] = {0u, 0u, 0u, 0u};
    int tA = 1, tB = 1;  // the iteration each half runs next
    uint32_t rkeep = 0xFFFFFFFFu;  // message bytes kept this round (fresh halves: none)
    for (bool first = true;; first = false) {
        const bool actA = idA >= 0, actB = idB >= 0;
        const bool busy = actA || actB;
        // a wave-uniform switch: some lane of this wave holds a fresh half
        const bool masked = __ballot(rkeep != 0xFFFFFFFFu) != 0;
        // messages are always stored: a half may go on after this round
        if (first)
            layer_pass<WMAX, false, true, false>(bw, smem, lb, ro, rsrc, row_ptr, meta, nullptr, u,
                                                 busy, off16, pre, true);
        else
            layer_pass<WMAX, false, false, false>(bw, smem, lb, ro, rsrc, row_ptr, meta, nullptr,
                                                  u, busy, off16, pre, true, masked, rkeep);
        rkeep = 0xFFFFFFFFu;
        if (tid < 2 * bw.slots) flags[tid] = 0;
        __syncthreads();
        if (busy)
            syndrome_mark<WMAX>(smem, lb, row_ptr, meta, bw.rows, u, Z, flags + 2 * p, actA, actB);
        __syncthreads();
        const bool holdsA = flags[2 * p] == 0, holdsB = flags[2 * p + 1] == 0;
        const bool finA = actA && (holdsA || tA >= bw.max_iter);
        const bool finB = actB && (holdsB || tB >= bw.max_iter);
        if (finA || finB)
            write_outputs_ids(bw, Lp, u, finA ? idA : -1, finB ? idB : -1, tA, tB, holdsA ? 1 : 0,
                              holdsB ? 1 : 0);
        // the next codewords for the halves that finished (one lane per pair)
        if (u == 0 && (finA || finB)) {
            const unsigned need = (finA ? 1u : 0u) + (finB ? 1u : 0u);
            unsigned base = atomicAdd(counter, need);
            if (finA) {
                held[2 * p] = (long)base < (long)n_total ? (int)base : -1;
                ++base;
            }
            if (finB) held[2 * p + 1] = (long)base < (long)n_total ? (int)base : -1;
        }
        __syncthreads();
        const int nA = finA ? held[2 * p] : idA, nB = finB ? held[2 * p + 1] : idB;
        const bool freshA = finA && nA >= 0, freshB = finB && nB >= 0;
        if (freshA || freshB) {
            // the new codewords' channel LLRs over their bytes of the pair words
            // (four dwords at a time: the round's state is still live)
            if (freshA) load_half_llrs<4>(Lp, 0, bw.llr + (size_t)nA * T, N, Z, u);
            if (freshB) load_half_llrs<4>(Lp, 1, bw.llr + (size_t)nB * T, N, Z, u);
            // the fresh halves' bytes of the messages this lane loads in
            // the next round (those of the codewords before) read as zero
            rkeep = (freshA ? 0xFF00FF00u : 0xFFFFFFFFu) & (freshB ? 0x00FF00FFu : 0xFFFFFFFFu);
#pragma unroll
            for (int j = 0; j < kPreDwords; ++j) pre[j] &= rkeep;
        }
        if (finA) {
            idA = nA;
            tA = 1;
        } else if (actA) {
            ++tA;
        }
        if (finB) {
            idB = nB;
            tB = 1;
        } else if (actB) {
            ++tB;
        }
        if (!__syncthreads_or(idA >= 0 || idB >= 0)) break;
    }
}

template <int WMAX>
__global__ __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(4))) void decode_i8_refill_kernel(
    DecodeLaunch p, const int32_t *__restrict__ row_ptr, const uint32_t *__restrict__ meta) {
    extern __shared__ __align__(16) uint8_t smem[];
    BlockWork bw;
    bw.n = p.cpw;
    bw.slots = p.cpw / 2;
    bw.llr = p.llr;
    bw.out_bits = p.out_bits;
    bw.out_iters = p.out_iters;
    bw.out_ok = p.out_ok;
    bw.out_llr = static_cast<int8_t *>(p.out_llr);
    // this workgroup's message region: cpw / 2 pairs
    const size_t region = (size_t)(p.cpw / 2) * p.E_pad * p.Z;  // pair words
    bw.msg = reinterpret_cast<uint16_t *>(p.msg) + (size_t)blockIdx.x * region;
    bw.msg_records = (uint32_t)(2 * region);
    bw.row_pad = p.row_pad;
    bw.E_pad = p.E_pad;
    bw.groups = p.groups;
    bw.wq = nullptr;
    bw.w_iters = 0;
    bw.w_stride = p.rows;
    bw.rows = p.rows;
    bw.n_cols = p.n_cols;
    bw.kb = p.kb;
    bw.Z = p.Z;
    bw.E = p.E;
    bw.max_iter = p.max_iter;
    bw.early_exit = 1;
    bw.beta = p.beta;
    bw.offset = p.offset;
    decode_refill<WMAX>(bw, smem, (crow_t)row_ptr, (cmeta_t)meta, p.counter, p.n_cw);
}

// Four waves per SIMD: a 768-lane workgroup whose pairs fill the LDS runs
// one per CU (three waves per SIMD) whatever the register count, and the
// register budget this leaves (up to 128) keeps every path free of scratch
// spills.
template <int WMAX, bool IN_LDS>
__global__ __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(4))) void decode_i8_kernel(DecodeLaunch p,
                                                         const int32_t *__restrict__ row_ptr,
                                                         const uint32_t *__restrict__ meta) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int T = (p.n_cols - 2) * p.Z, first = blockIdx.x * p.cpw;
    BlockWork bw;
    bw.n = p.n_cw - first < p.cpw ? p.n_cw - first : p.cpw;
    bw.slots = p.cpw / 2;
    bw.llr = p.llr + (size_t)first * T;
    bw.out_bits = p.out_bits + (size_t)first * (p.kb * p.Z / 8);
    bw.out_iters = p.out_iters + first;
    bw.out_ok = p.out_ok ? p.out_ok + first : nullptr;
    bw.out_llr = p.out_llr ? static_cast<int8_t *>(p.out_llr) + (size_t)first * p.n_cols * p.Z
                           : nullptr;
    bw.msg = IN_LDS ? nullptr
                    : reinterpret_cast<uint16_t *>(p.msg) + (size_t)(first / 2) * p.E_pad * p.Z;
    if (!IN_LDS) {
        // this workgroup's pairs up to the end of the allocation (the last
        // workgroup may hold fewer than cpw / 2 pairs)
        const size_t base = (size_t)(first / 2) * p.E_pad * p.Z * 2;
        const size_t full = (size_t)(p.cpw / 2) * p.E_pad * p.Z * 2;
        const size_t left = p.msg_bytes - base;
        bw.msg_records = (uint32_t)(left < full ? left : full);
    }
    bw.row_pad = p.row_pad;
    bw.E_pad = p.E_pad;
    bw.groups = p.groups;
    bw.wq = p.wq;
    bw.w_iters = p.w_iters;
    bw.w_stride = p.rows;
    bw.rows = p.rows;
    bw.n_cols = p.n_cols;
    bw.kb = p.kb;
    bw.Z = p.Z;
    bw.E = p.E;
    bw.max_iter = p.max_iter;
    bw.early_exit = p.early_exit;
    bw.beta = p.beta;
    bw.offset = p.offset;
    decode_block<WMAX, IN_LDS>(bw, smem, (crow_t)row_ptr, (cmeta_t)meta);
}

template <int WMAX, bool IN_LDS>
hipError_t launch_w(const DecodeLaunch &p, hipStream_t stream) {
    const int per_pair = IN_LDS ? lds_bytes_i8_pair(p.n_cols, p.E, p.Z)
                                : lds_bytes_i8_pair_post(p.n_cols, p.Z);
    const int pairs = p.cpw / 2;
    const int lds = pairs * per_pair + lds_flags_bytes_i8(pairs);
    static std::once_flag attr_once;  // once per process, also under concurrent calls
    std::call_once(attr_once, [] {
        // Opt in to more than the default 64 KiB of dynamic LDS.
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&decode_i8_kernel<WMAX, IN_LDS>),
            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
        if (e != hipSuccess) note_hip_error("hipFuncSetAttribute(decode_i8_kernel)", e);
    });
    if (p.cpw < 2 || (p.cpw & 1) || pairs * p.Z > 768) {
        note_hip_error("decode_i8_kernel: bad workgroup shape", hipErrorInvalidValue);
        return hipErrorInvalidValue;
    }
    const int blocks = (p.n_cw + p.cpw - 1) / p.cpw;
    // hipGetLastError reports the last error of ANY earlier runtime call on
    // this thread; clear it so the check below sees this launch only.
    (void)hipGetLastError();
    hipLaunchKernelGGL((decode_i8_kernel<WMAX, IN_LDS>), dim3(blocks), dim3(pairs * p.Z), lds,
                       stream, p, p.row_ptr, p.meta);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) note_hip_error("launch decode_i8_kernel", e);
    return e;
}

template <bool IN_LDS>
hipError_t launch_placed(const DecodeLaunch &p, hipStream_t stream) {
    if (p.wmax <= 10) return launch_w<10, IN_LDS>(p, stream);
    if (p.wmax <= 20) return launch_w<20, IN_LDS>(p, stream);
    return launch_w<32, IN_LDS>(p, stream);
}

// Row-pair kernel: p.cpw codewords of Z/2 lanes per workgroup (see
// decode_rp); p.meta is the row-pair metadata table. Five waves per SIMD:
// at Z = 384 six one-codeword workgroups (18 waves, 157 kB of LDS) share a
// CU; the register budget this leaves (up to 102) spills six values, none
// inside a row update (the four-wave budget fits five workgroups and was
// 1.5 % slower).
template <int WMAX, bool IN_LDS>
__global__ __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(5))) void decode_i8_rp_kernel(
    DecodeLaunch p, const int32_t *__restrict__ row_ptr, const uint32_t *__restrict__ meta) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int Zh = p.Z / 2, T = (p.n_cols - 2) * p.Z, first = blockIdx.x * p.cpw;
    BlockWork bw;
    bw.n = p.n_cw - first < p.cpw ? p.n_cw - first : p.cpw;
    bw.slots = p.cpw;
    bw.llr = p.llr + (size_t)first * T;
    bw.out_bits = p.out_bits + (size_t)first * (p.kb * p.Z / 8);
    bw.out_iters = p.out_iters + first;
    bw.out_ok = p.out_ok ? p.out_ok + first : nullptr;
    bw.out_llr = p.out_llr ? static_cast<int8_t *>(p.out_llr) + (size_t)first * p.n_cols * p.Z
                           : nullptr;
    bw.msg = nullptr;
    bw.msg_records = 0;
    if (!IN_LDS) {
        bw.msg = reinterpret_cast<uint16_t *>(p.msg) + (size_t)first * p.E_pad * Zh;
        // this workgroup's codewords up to the end of the allocation
        const size_t base = (size_t)first * p.E_pad * Zh * 2;
        const size_t full = (size_t)p.cpw * p.E_pad * Zh * 2;
        const size_t left = p.msg_bytes - base;
        bw.msg_records = (uint32_t)(left < full ? left : full);
    }
    bw.row_pad = p.row_pad;
    bw.E_pad = p.E_pad;
    bw.groups = p.groups;
    bw.wq = p.wq;
    bw.w_iters = p.w_iters;
    bw.w_stride = p.rows;
    bw.rows = p.rows;
    bw.n_cols = p.n_cols;
    bw.kb = p.kb;
    bw.Z = Zh;
    bw.E = p.E;
    bw.max_iter = p.max_iter;
    bw.early_exit = p.early_exit;
    bw.beta = p.beta;
    bw.offset = p.offset;
    decode_rp<WMAX, IN_LDS>(bw, smem, (crow_t)row_ptr, (cmeta_t)meta);
}

// Row-pair launch: messages in device memory (p.msg) or, without p.msg,
// in LDS after each codeword's posteriors.
template <int WMAX, bool IN_LDS>
hipError_t launch_rp_w(const DecodeLaunch &p, hipStream_t stream) {
    const int Zh = p.Z / 2;
    const int per_cw =
        IN_LDS ? lds_bytes_i8_pair(p.n_cols, p.E, Zh) : lds_bytes_i8_pair_post(p.n_cols, Zh);
    const int lds = p.cpw * per_cw + lds_flags_bytes_i8(p.cpw);
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&decode_i8_rp_kernel<WMAX, IN_LDS>),
            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
        if (e != hipSuccess) note_hip_error("hipFuncSetAttribute(decode_i8_rp_kernel)", e);
    });
    if (p.cpw < 1 || p.cpw * Zh > 768 || Zh % 4 != 0 || (!IN_LDS && !p.msg) ||
        lds > max_lds_bytes()) {
        note_hip_error("decode_i8_rp_kernel: bad workgroup shape", hipErrorInvalidValue);
        return hipErrorInvalidValue;
    }
    const int blocks = (p.n_cw + p.cpw - 1) / p.cpw;
    (void)hipGetLastError();
    hipLaunchKernelGGL((decode_i8_rp_kernel<WMAX, IN_LDS>), dim3(blocks), dim3(p.cpw * Zh), lds,
                       stream, p, p.row_ptr, p.meta);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) note_hip_error("launch decode_i8_rp_kernel", e);
    return e;
}

__global__ void reset_counter_kernel(unsigned *counter);

template <int WMAX>
hipError_t launch_refill_w(const DecodeLaunch &p, hipStream_t stream) {
    const int pairs = p.cpw / 2;
    const int lds = pairs * lds_bytes_i8_pair_post(p.n_cols, p.Z) + lds_flags_bytes_i8(pairs);
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&decode_i8_refill_kernel<WMAX>),
            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
        if (e != hipSuccess) note_hip_error("hipFuncSetAttribute(decode_i8_refill_kernel)", e);
    });
    if (p.cpw < 2 || (p.cpw & 1) || pairs * p.Z > 768 || p.grid < 1 || !p.counter || !p.msg) {
        note_hip_error("decode_i8_refill_kernel: bad launch shape", hipErrorInvalidValue);
        return hipErrorInvalidValue;
    }
    (void)hipGetLastError();
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, p.counter);
    hipLaunchKernelGGL((decode_i8_refill_kernel<WMAX>), dim3(p.grid), dim3(pairs * p.Z), lds,
                       stream, p, p.row_ptr, p.meta);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) note_hip_error("launch decode_i8_refill_kernel", e);
    return e;
}

// Persistent mixed-shape decode: each workgroup takes tasks (up to a
// workgroup's worth of codeword pairs of one shape) from a device counter
// until none are left, so every wave reaches the exit once the counter
// passes n_tasks. Messages use the device placement with one region per
// workgroup, reused from task to task. Five waves per SIMD keeps three
// 384-lane workgroups of BG1 Z = 384 on a CU; at that register budget (96)
// the bound-20 body spills three per-task values, which are reloaded once
// per task or iteration, never inside a row update.
// RPT: the variant that also decodes row-pair tasks (nwave = -1), launched
// only for launches that hold some: its extra path changes the register
// allocation of the whole kernel (spills inside row updates), which the
// variant without it keeps clear of.
template <int WMAX, bool RPT = false>
__global__ __launch_bounds__(kBatchLanes) __attribute__((amdgpu_waves_per_eu(5))) void decode_batch_kernel(
    const BatchTask *__restrict__ tasks, const BatchJob *__restrict__ jobs,
    const WaveTask *__restrict__ waves, int n_tasks, unsigned *counter, uint16_t *msg_ws,
    int msg_per_block, int wave_lds, int wave_msg, int max_iter, int early_exit, int beta,
    int offset) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ int task_id;
    for (;;) {
        if (threadIdx.x == 0) task_id = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int ti = task_id;
        __syncthreads();
        if (ti >= n_tasks) break;
        const BatchTask tk = tasks[ti];
        // a whole-workgroup task, a row-pair task or this wave's task of a
        // bundle (uniform within a wave; readfirstlane lets the compiler know)
        const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWaveLanes));
        const bool wave_task = tk.nwave > 0;
        if (RPT && tk.nwave < 0) {
            const BatchJob &jb = jobs[tk.job];
            const int Zh = jb.Z / 2, T = (jb.n_cols - 2) * jb.Z;
            BlockWork bw;
            bw.n = 1;
            bw.slots = 1;
            bw.llr = jb.llr + (size_t)tk.first * T;
            bw.out_bits = jb.out_bits + (size_t)tk.first * (jb.kb * jb.Z / 8);
            bw.out_iters = jb.out_iters + tk.first;
            bw.out_ok = jb.out_ok ? jb.out_ok + tk.first : nullptr;
            bw.out_llr = nullptr;
            bw.msg = msg_ws + (size_t)blockIdx.x * msg_per_block;
            bw.msg_records = 2u * (uint32_t)(jb.E_pad * Zh) + (uint32_t)kMsgTail;
            bw.row_pad = jb.row_pad;
            bw.E_pad = jb.E_pad;
            bw.groups = jb.groups;
            bw.wq = jb.wq;
            bw.w_iters = jb.w_iters;
            bw.w_stride = jb.w_stride;
            bw.rows = jb.rows;
            bw.n_cols = jb.n_cols;
            bw.kb = jb.kb;
            bw.Z = Zh;
            bw.E = jb.E;
            bw.max_iter = max_iter;
            bw.early_exit = early_exit;
            bw.beta = beta;
            bw.offset = offset;
            decode_rp<WMAX>(bw, smem, (crow_t)jb.row_ptr, (cmeta_t)jb.meta_rp);
        } else if (!wave_task || wv < tk.nwave) {
            int job = tk.job, first = tk.first, n = tk.n;
            if (wave_task) {
                const WaveTask wt = waves[tk.first + wv];
                job = wt.job;
                first = wt.first;
                n = wt.n;
            }
            const BatchJob &jb = jobs[job];
            const int T = (jb.n_cols - 2) * jb.Z;
            BlockWork bw;
            bw.n = n;
            bw.slots = wave_task ? kWaveLanes / jb.Z : jb.slots / 2;
            bw.llr = jb.llr + (size_t)first * T;
            bw.out_bits = jb.out_bits + (size_t)first * (jb.kb * jb.Z / 8);
            bw.out_iters = jb.out_iters + first;
            bw.out_ok = jb.out_ok ? jb.out_ok + first : nullptr;
            bw.out_llr = nullptr;
            bw.msg = msg_ws + (size_t)blockIdx.x * msg_per_block +
                     (wave_task ? (size_t)wv * wave_msg : 0);
            // the task's pairs lie inside the workgroup's region; the region
            // of the last workgroup is followed by the allocation's tail
            bw.msg_records = 2u * (uint32_t)(bw.slots * jb.E_pad * jb.Z) + (uint32_t)kMsgTail;
            bw.row_pad = jb.row_pad;
            bw.E_pad = jb.E_pad;
            bw.groups = jb.groups;
            bw.wq = jb.wq;
            bw.w_iters = jb.w_iters;
            bw.w_stride = jb.w_stride;
            bw.rows = jb.rows;
            bw.n_cols = jb.n_cols;
            bw.kb = jb.kb;
            bw.Z = jb.Z;
            bw.E = jb.E;
            bw.max_iter = max_iter;
            bw.early_exit = early_exit;
            bw.beta = beta;
            bw.offset = offset;
            if (wave_task)
                decode_block<WMAX, false, true>(bw, smem + wv * wave_lds, (crow_t)jb.row_ptr,
                                                (cmeta_t)jb.meta);
            else
                decode_block<WMAX, false>(bw, smem, (crow_t)jb.row_ptr, (cmeta_t)jb.meta);
        }
        __syncthreads();
    }
}

__global__ void reset_counter_kernel(unsigned *counter) { *counter = 0u; }

// ---------------------------------------------------------------------
// Serving queue: a persistent decode kernel fed while it runs.
// ---------------------------------------------------------------------
// Workgroup 0 is the dispatcher: one lane polls the count of tasks the host
// has published (pinned host memory, system scope) and mirrors it into
// device memory, where the decode workgroups claim tasks one at a time with
// a compare-and-swap on the claimed count (a task is claimed only once it is
// published, so no claim is ever lost). A decode workgroup reads the task's
// descriptor from the host ring, decodes it with the one-lane-per-row
// mapping (one task = one workgroup's worth of codewords of one shape),
// writes the outputs (which may live in pinned host memory), fences them to
// system scope and publishes done[ticket % capacity] = ticket + 1. Every
// loop is bounded: the dispatcher leaves after twice idle_polls polls
// without news or on the stop request, a decode workgroup after idle_polls
// empty polls or once the dispatcher has seen the stop request; the host
// relaunches the kernel when tasks are pending and the last launch has
// ended.
// Polls are relaxed atomic loads. An acquire load at agent or system scope
// is followed by an invalidation of the whole L2 of the XCD (and a release
// store by a write-back), so acquire polling by hundreds of idle workgroups
// would keep every L2 invalidating while other workgroups decode; ordering
// is instead taken once, by one fence after a successful claim (and one
// release store per change of the published count).
__device__ inline unsigned sys_peek(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ inline unsigned dev_peek(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kBatchLanes) __attribute__((amdgpu_waves_per_eu(5))) void serve_kernel(
    ServeLaunch s) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ int task_id;
    __shared__ unsigned desc[sizeof(ServeTask) / 4];
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            unsigned last = dev_peek(s.dev_ctl + 1);
            for (int idle = 0; idle < 2 * s.idle_polls;) {
                if (sys_peek(s.host_ctl + 1)) {
                    __hip_atomic_store(s.dev_ctl + 2, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                const unsigned t = sys_peek(s.host_ctl);
                if (t != last) {
                    // the host wrote the descriptors before the count: pass
                    // that order on (acquire, then a release store; a
                    // claimer's fence after reading the mirror completes it)
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                    __hip_atomic_store(s.dev_ctl + 1, t, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    last = t;
                    idle = 0;
                } else {
                    ++idle;
                    __builtin_amdgcn_s_sleep(8);
                }
            }
        }
        return;
    }
    const uint16_t *msg_base = s.msg + (size_t)(blockIdx.x - 1) * s.msg_per_block;
    for (;;) {
        if (threadIdx.x == 0) {
            int id = -1;
            for (int idle = 0; idle < s.idle_polls;) {
                if (dev_peek(s.dev_ctl + 2)) break;
                const unsigned t = dev_peek(s.dev_ctl + 1);
                unsigned h = dev_peek(s.dev_ctl);
                if (h < t) {
                    if (__hip_atomic_compare_exchange_strong(s.dev_ctl, &h, h + 1, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) {
                        id = (int)h;
                        // the task's descriptor and LLRs were written after
                        // this kernel started (LLRs possibly into memory an
                        // earlier task read): drop cached lines before the
                        // workgroup reads them
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                        break;
                    }
                    continue;  // another workgroup claimed it first
                }
                ++idle;
                __builtin_amdgcn_s_sleep(32);
            }
            task_id = id;
        }
        __syncthreads();
        const int id = task_id;
        if (id < 0) break;
        // the descriptor, one word per lane, at system scope (host memory)
        constexpr int kWords = (int)(sizeof(ServeTask) / 4);
        if ((int)threadIdx.x < kWords)
            desc[threadIdx.x] = __hip_atomic_load(
                reinterpret_cast<const unsigned *>(s.ring + (unsigned)id % (unsigned)s.capacity) +
                    threadIdx.x,
                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __syncthreads();
        // uniform copy (scalar registers: the tables are read with scalar loads)
        unsigned words[kWords];
#pragma unroll
        for (int i = 0; i < kWords; ++i) words[i] = __builtin_amdgcn_readfirstlane(desc[i]);
        ServeTask tk;
        __builtin_memcpy(&tk, words, sizeof(ServeTask));
        const BatchJob &jb = tk.job;
        const int T = (jb.n_cols - 2) * jb.Z;
        BlockWork bw;
        bw.n = tk.n;
        bw.slots = jb.slots / 2;
        bw.llr = jb.llr + (size_t)tk.first * T;
        bw.out_bits = jb.out_bits + (size_t)tk.first * (jb.kb * jb.Z / 8);
        bw.out_iters = jb.out_iters + tk.first;
        bw.out_ok = jb.out_ok ? jb.out_ok + tk.first : nullptr;
        bw.out_llr = nullptr;
        bw.msg = const_cast<uint16_t *>(msg_base);
        bw.msg_records = 2u * (uint32_t)(bw.slots * jb.E_pad * jb.Z) + (uint32_t)kMsgTail;
        bw.row_pad = jb.row_pad;
        bw.E_pad = jb.E_pad;
        bw.groups = jb.groups;
        bw.wq = jb.wq;
        bw.w_iters = jb.w_iters;
        bw.w_stride = jb.w_stride;
        bw.rows = jb.rows;
        bw.n_cols = jb.n_cols;
        bw.kb = jb.kb;
        bw.Z = jb.Z;
        bw.E = jb.E;
        bw.max_iter = s.max_iter;
        bw.early_exit = s.early_exit;
        bw.beta = 96;
        bw.offset = 0;
        decode_block<20, false>(bw, smem, (crow_t)jb.row_ptr, (cmeta_t)jb.meta);
        // every lane's output stores done and visible to the host, then the flag
        __threadfence_system();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(s.done + tk.ticket % (unsigned)s.capacity, tk.ticket + 1u,
                               __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}


// ---------------------------------------------------------------------
// Low-latency mapping: ALPHA cooperating lanes per check row (§IV).
// ---------------------------------------------------------------------
// Block row r of weight w is cut into ALPHA chunks of c = ceil(w / ALPHA)
// consecutive blocks (the last ones shorter, possibly empty). Chunk a of
// every check row of the workgroup's pairs is handled by the a-th group of
// L = slots * Z lanes (whole waves, so the chunk's block metadata stays
// wave-uniform and lives in scalar registers). Each lane reduces its chunk
// to (min, second min, sign parity), the ALPHA partials of a check row meet
// in LDS, every lane merges all of them with the same min / second-min rule
// (associative, so all lanes of a row agree) and writes back its chunk. One
// exchange barrier per row buys a dependent chain of c instead of w edges
// per lane. Messages stream through device memory: row r's region holds the
// ALPHA chunk regions one after the other, chunk a as [Z][(wc_a + 1) / 2]
// dwords of two pair words (wc_a the chunk's width).

// Message dwords per check row of a row of weight w cut into ALPHA chunks.
template <int ALPHA>
__host__ __device__ inline int ll_row_dwords(int w) {
    const int c = (w + ALPHA - 1) / ALPHA;
    const int nfull = w / c, rem = w - nfull * c;
    return nfull * ((c + 1) / 2) + (rem + 1) / 2;
}

// Chunk a of a row of weight w: first block k0, width wc (0 if empty),
// dword offset of the chunk's region per check row (times Z * 4 bytes).
template <int ALPHA>
__device__ inline void ll_chunk(int w, int a, int &k0, int &wc, int &dw_off) {
    const int c = (w + ALPHA - 1) / ALPHA;
    k0 = a * c;
    const int left = w - k0;
    wc = left < 0 ? 0 : (left < c ? left : c);
    dw_off = a * ((c + 1) / 2);
}

// One row of the low-latency mapping for a lane whose chunk has exactly W
// blocks (W = 0: an empty chunk, which only takes part in the exchange).
// xb: this row's exchange buffer [ALPHA][3][L] dwords (min, second min,
// sign word of each chunk); a, l: the lane's chunk and lane within the
// chunk group.
template <int W, bool FIRST, int ALPHA>
__device__ __forceinline__ void ll_row_w(uint8_t *__restrict__ smem, uint32_t lb,
                                         const MsgRow<false> &R, cmeta_t meta, int e0,
                                         uint32_t u, int Z, u16x2 wgt, u16x2 off16,
                                         const uint32_t *pre, bool busy, uint32_t *xb, int a,
                                         int L, int l) {
    constexpr int NW = W > 0 ? W : 1;
    constexpr int ND = (NW + 1) / 2;
    uint32_t md[NW], mo[NW], rd[ND], xv[NW], axv[NW], la[NW];
    u16x2 m1 = {0x7FFF, 0x7FFF}, m2 = {0x7FFF, 0x7FFF};
    uint32_t S = 0;
    if constexpr (W > 0) {
        if (busy) {
#pragma unroll
            for (int k = 0; k < W; ++k) {
                md[k] = meta[e0 + k];
                mo[k] = md[k] & 0xFFFFu;
            }
            if (FIRST) {
#pragma unroll
                for (int j = 0; j < ND; ++j) rd[j] = 0;
            } else {
#pragma unroll
                for (int j = 0; j < ND && j < kPreDwords; ++j) rd[j] = pre[j];
                if (ND > kPreDwords) R.template load<W, kPreDwords>(rd, u, Z);
            }
            uint32_t ps_unused[1];
            row_phase1<0, W, true>(smem, lb, rd, md, mo, u, Z, W, xv, axv, la, ps_unused, m1, m2,
                                   S);
        }
    }
    // exchange of the chunk partials
    xb[(a * 3 + 0) * L + l] = bits_of(m1);
    xb[(a * 3 + 1) * L + l] = bits_of(m2);
    xb[(a * 3 + 2) * L + l] = S;
    __syncthreads();
    if constexpr (W > 0) {
        if (!busy) return;
        u16x2 M1 = {0x7FFF, 0x7FFF}, M2 = {0x7FFF, 0x7FFF};
        uint32_t SS = 0;
#pragma unroll
        for (int b = 0; b < ALPHA; ++b) {
            const u16x2 p1 = as_u(xb[(b * 3 + 0) * L + l]);
            const u16x2 p2 = as_u(xb[(b * 3 + 1) * L + l]);
            M2 = __builtin_elementwise_min(__builtin_elementwise_max(M1, p1),
                                           __builtin_elementwise_min(M2, p2));
            M1 = __builtin_elementwise_min(M1, p1);
            SS ^= xb[(b * 3 + 2) * L + l];
        }
        const u16x2 a1 = normalise(M1, off16, wgt);
        const u16x2 a2 = normalise(M2, off16, wgt);
        const s16x2 Sm = as_s(SS) >> (s16x2){15, 15};
        const s16x2 b1 = (as_s(bits_of(a1)) ^ Sm) - Sm;
        const s16x2 b2 = (as_s(bits_of(a2)) ^ Sm) - Sm;
        const u16x2 d21 = as_u(bits_of(b2 - b1));
        const u16x2 m1p = M1 + (u16x2){1, 1};
        s16x2 Rv[W], Lv[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            // t = 1 where |x| equals the row's minimum (argmin, or a tie,
            // where both magnitudes are equal anyway)
            const u16x2 t = __builtin_elementwise_sub_sat(m1p, as_u(axv[k]));
            Rv[k] = as_s(bits_of(t * d21 + as_u(bits_of(b1))));
        }
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const s16x2 sx = as_s(xv[k]) >> (s16x2){15, 15};
            Rv[k] = (Rv[k] ^ sx) - sx;
        }
#pragma unroll
        for (int k = 0; k < W; ++k)
            Lv[k] = __builtin_elementwise_max(__builtin_elementwise_add_sat(as_s(xv[k]), Rv[k]),
                                              (s16x2){-127 * 256, -127 * 256});
#pragma unroll
        for (int k = 0; k < W; ++k) lds_st16(smem, la[k], perm(bits_of(Lv[k]), kPack));
        uint32_t sd[ND];
#pragma unroll
        for (int j = 0; j < ND; ++j)
            sd[j] = 2 * j + 1 < W ? __builtin_amdgcn_perm(bits_of(Rv[2 * j + 1]), bits_of(Rv[2 * j]),
                                                          kPack2)
                                  : perm(bits_of(Rv[2 * j]), kPack);
#pragma unroll
        for (int c = 0; c < ND; c += 4) R.template store<W>(sd, u, Z, c, ND - c < 4 ? ND - c : 4);
    }
}

template <int W, bool FIRST, int ALPHA>
__device__ __forceinline__ void ll_row(int wc, uint8_t *smem, uint32_t lb, const MsgRow<false> &R,
                                       cmeta_t meta, int e0, uint32_t u, int Z, u16x2 wgt,
                                       u16x2 off16, const uint32_t *pre, bool busy, uint32_t *xb,
                                       int a, int L, int l) {
    if constexpr (W <= kLLChunkMax) {
        if (wc == W) {
            ll_row_w<W, FIRST, ALPHA>(smem, lb, R, meta, e0, u, Z, wgt, off16, pre, busy, xb, a,
                                      L, l);
            return;
        }
        ll_row<W + 1, FIRST, ALPHA>(wc, smem, lb, R, meta, e0, u, Z, wgt, off16, pre, busy, xb,
                                    a, L, l);
    }
}

// One iteration of the low-latency mapping: rows in order, the exchange
// barrier inside every row, the layer-group barrier after rows that share
// a column with the next. Exchange buffers alternate between rows.
template <bool FIRST, int ALPHA>
__device__ __forceinline__ void ll_layer_pass(const BlockWork &bw, uint8_t *smem, uint32_t lb,
                                              uint32_t ro, __amdgpu_buffer_rsrc_t rsrc,
                                              crow_t row_ptr, cmeta_t meta, const uint8_t *wrow,
                                              uint32_t u, bool busy, u16x2 off16, uint32_t *pre,
                                              bool keep, uint32_t *xbuf, int a, int L, int l) {
    const int Z = bw.Z;
    const uint64_t bar = (bw.groups >> 1) | (1ull << (bw.rows - 1));
    int e0 = row_ptr[0], e1 = row_ptr[1];
    int roff = 0;  // dword offset (per check row) of the row's message region
    for (int r = 0; r < bw.rows; ++r) {
        const bool last = r + 1 == bw.rows;
        const int e2 = last ? row_ptr[1] : row_ptr[r + 2];
        const int en = last ? row_ptr[0] : e1;
        const int w = e1 - e0;
        int k0, wc, doff;
        ll_chunk<ALPHA>(w, a, k0, wc, doff);
        const int wt = wrow ? row_weight(wrow, r) : bw.beta;
        const u16x2 wgt = {(unsigned short)wt, (unsigned short)wt};
        MsgRow<false> R{rsrc, nullptr, ro, 4u * (uint32_t)((roff + doff) * Z), keep};
        ll_row<0, FIRST, ALPHA>(wc, smem, lb, R, meta, e0 + k0, u, Z, wgt, off16, pre, busy,
                                xbuf + (r & 1) * (ALPHA * 3 * L), a, L, l);
        const int rnext = last ? 0 : roff + ll_row_dwords<ALPHA>(w);
        // prefetch of the next row's (first) message dwords of this chunk
        if (busy && (last ? keep : !FIRST)) {
            int k0n, wcn, doffn;
            ll_chunk<ALPHA>(e2 - en, a, k0n, wcn, doffn);
            if (wcn > 0) {
                const MsgRow<false> Rn{rsrc, nullptr, ro, 4u * (uint32_t)((rnext + doffn) * Z),
                                       true};
                Rn.load4(pre, u, (wcn + 1) / 2);
            }
        }
        if ((bar >> r) & 1) __syncthreads();
        e0 = en;
        e1 = e2;
        roff = rnext;
    }
}

// Decodes bw.n codewords as bw.slots pairs with ALPHA lanes per check row:
// lane tid belongs to chunk group a = tid / L (L = slots * Z) and serves
// check row u of pair p within it. Initialisation, the syndrome check and
// the outputs are done by chunk group 0 alone (whole rows, as in the
// one-lane-per-row mapping). Every thread must call it.
template <int WMAX, int ALPHA>
__device__ __forceinline__ void decode_block_ll(const BlockWork &bw, uint8_t *smem,
                                                crow_t row_ptr, cmeta_t meta) {
    static_assert(WMAX <= kMetaPad, "row metadata window exceeds the table padding");
    const int Z = bw.Z, L = bw.slots * Z;
    const int N = bw.n_cols, T = (N - 2) * Z;
    const int pair_bytes = lds_bytes_i8_pair_post(N, Z);
    const int tid = (int)threadIdx.x;
    const int a = __builtin_amdgcn_readfirstlane(tid / L);  // whole waves (L % 64 == 0)
    const int l = tid - a * L;
    const int p = l / Z;
    const uint32_t u = l - p * Z;
    const bool validA = 2 * p < bw.n, validB = 2 * p + 1 < bw.n;
    const int ps = validA ? p : 0;
    uint8_t *Lp = smem + ps * pair_bytes;
    uint16_t *Lw = reinterpret_cast<uint16_t *>(Lp);
    const uint32_t lb = (uint32_t)(ps * pair_bytes) + 2u * u;
    const uint32_t ro = 2u * (uint32_t)(ps * bw.E_pad * Z);
    int *flags = reinterpret_cast<int *>(smem + bw.slots * pair_bytes);
    uint32_t *xbuf = reinterpret_cast<uint32_t *>(smem + bw.slots * pair_bytes +
                                                  lds_flags_bytes_i8(bw.slots));
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(bw.msg, 0, bw.msg_records, 0x00020000);

    if (a == 0 && validA) {
        load_half_llrs<17>(Lp, 0, bw.llr + (size_t)(2 * p) * T, N, Z, u);
        load_half_llrs<17>(Lp, 1, validB ? bw.llr + (size_t)(2 * p + 1) * T : nullptr, N, Z, u);
    }
    __syncthreads();

    const u16x2 off16 = {(unsigned short)(bw.offset << 8), (unsigned short)(bw.offset << 8)};
    bool doneA = !validA, doneB = !validB;
    uint32_t pre[kPreDwords] = {0u, 0u, 0u, 0u};
    for (int t = 1; t <= bw.max_iter; ++t) {
        const uint8_t *wrow = nullptr;
        if (bw.wq) wrow = bw.wq + (size_t)((t < bw.w_iters ? t : bw.w_iters) - 1) * bw.w_stride;
        const bool busy = !(doneA && doneB);
        if (t == 1)
            ll_layer_pass<true, ALPHA>(bw, smem, lb, ro, rsrc, row_ptr, meta, wrow, u, busy, off16,
                                       pre, t < bw.max_iter, xbuf, a, L, l);
        else
            ll_layer_pass<false, ALPHA>(bw, smem, lb, ro, rsrc, row_ptr, meta, wrow, u, busy,
                                        off16, pre, t < bw.max_iter, xbuf, a, L, l);
        if (bw.early_exit || t == bw.max_iter) {
            if (tid <= 2 * bw.slots) flags[tid] = tid == 2 * bw.slots;
            __syncthreads();
            if (a == 0 && busy)
                syndrome_mark<WMAX>(smem, lb, row_ptr, meta, bw.rows, u, Z, flags + 2 * p, !doneA,
                                    !doneB);
            __syncthreads();
            const bool holdsA = flags[2 * ps] == 0, holdsB = flags[2 * ps + 1] == 0;
            bool finA = false, finB = false;
            if (t == bw.max_iter) {
                finA = !doneA;
                finB = !doneB;
            } else {
                finA = !doneA && holdsA;
                finB = !doneB && holdsB;
            }
            if (a == 0 && (finA || finB))
                write_outputs(bw, Lp, p, u, (finA ? 1 : 0) | (finB ? 2 : 0), t, holdsA, holdsB);
            doneA = doneA || finA;
            doneB = doneB || finB;
            if (!(doneA && doneB)) flags[2 * bw.slots] = 0;
            __syncthreads();
            if (flags[2 * bw.slots]) break;
        }
    }
}

template <int WMAX, int ALPHA>
__global__ __launch_bounds__(1024) void decode_i8_ll_kernel(DecodeLaunch p,
                                                            const int32_t *__restrict__ row_ptr,
                                                            const uint32_t *__restrict__ meta) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int T = (p.n_cols - 2) * p.Z, first = blockIdx.x * p.cpw;
    BlockWork bw;
    bw.n = p.n_cw - first < p.cpw ? p.n_cw - first : p.cpw;
    bw.slots = p.cpw / 2;
    bw.llr = p.llr + (size_t)first * T;
    bw.out_bits = p.out_bits + (size_t)first * (p.kb * p.Z / 8);
    bw.out_iters = p.out_iters + first;
    bw.out_ok = p.out_ok ? p.out_ok + first : nullptr;
    bw.out_llr = p.out_llr ? static_cast<int8_t *>(p.out_llr) + (size_t)first * p.n_cols * p.Z
                           : nullptr;
    bw.msg = reinterpret_cast<uint16_t *>(p.msg) + (size_t)(first / 2) * p.E_pad * p.Z;
    {
        const size_t base = (size_t)(first / 2) * p.E_pad * p.Z * 2;
        const size_t full = (size_t)(p.cpw / 2) * p.E_pad * p.Z * 2;
        const size_t left = p.msg_bytes - base;
        bw.msg_records = (uint32_t)(left < full ? left : full);
    }
    bw.row_pad = p.row_pad;
    bw.E_pad = p.E_pad;
    bw.groups = p.groups;
    bw.wq = p.wq;
    bw.w_iters = p.w_iters;
    bw.w_stride = p.rows;
    bw.rows = p.rows;
    bw.n_cols = p.n_cols;
    bw.kb = p.kb;
    bw.Z = p.Z;
    bw.E = p.E;
    bw.max_iter = p.max_iter;
    bw.early_exit = p.early_exit;
    bw.beta = p.beta;
    bw.offset = p.offset;
    decode_block_ll<WMAX, ALPHA>(bw, smem, (crow_t)row_ptr, (cmeta_t)meta);
}

template <int WMAX, int ALPHA>
hipError_t launch_ll(const DecodeLaunch &p, hipStream_t stream) {
    const int pairs = p.cpw / 2, L = pairs * p.Z;
    const int lds = ll_lds_bytes(p.n_cols, p.Z, pairs, ALPHA);
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&decode_i8_ll_kernel<WMAX, ALPHA>),
            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
        if (e != hipSuccess) note_hip_error("hipFuncSetAttribute(decode_i8_ll_kernel)", e);
    });
    if (p.cpw < 2 || (p.cpw & 1) || L % 64 != 0 || ALPHA * L > 1024 || !p.msg ||
        p.wmax > WMAX || p.wmax > kLLChunkMax * ALPHA || lds > max_lds_bytes()) {
        note_hip_error("decode_i8_ll_kernel: bad workgroup shape", hipErrorInvalidValue);
        return hipErrorInvalidValue;
    }
    const int blocks = (p.n_cw + p.cpw - 1) / p.cpw;
    (void)hipGetLastError();
    hipLaunchKernelGGL((decode_i8_ll_kernel<WMAX, ALPHA>), dim3(blocks), dim3(ALPHA * L), lds,
                       stream, p, p.row_ptr, p.meta);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) note_hip_error("launch decode_i8_ll_kernel", e);
    return e;
}


}  // namespace

hipError_t launch_decode_i8(const DecodeLaunch &p, hipStream_t stream) {
    if (p.alpha == 2) return p.wmax <= 10 ? launch_ll<10, 2>(p, stream) : launch_ll<20, 2>(p, stream);
    if (p.alpha == 4) return p.wmax <= 10 ? launch_ll<10, 4>(p, stream) : launch_ll<20, 4>(p, stream);
    if (p.rowpair && p.msg) {
        if (p.wmax <= 10) return launch_rp_w<10, false>(p, stream);
        if (p.wmax <= 20) return launch_rp_w<20, false>(p, stream);
        return launch_rp_w<32, false>(p, stream);
    }
    if (p.rowpair) {
        if (p.wmax <= 10) return launch_rp_w<10, true>(p, stream);
        if (p.wmax <= 20) return launch_rp_w<20, true>(p, stream);
        return launch_rp_w<32, true>(p, stream);
    }
    if (p.refill) {
        if (p.wmax <= 10) return launch_refill_w<10>(p, stream);
        if (p.wmax <= 20) return launch_refill_w<20>(p, stream);
        return launch_refill_w<32>(p, stream);
    }
    return p.msg ? launch_placed<false>(p, stream) : launch_placed<true>(p, stream);
}

hipError_t launch_serve(const ServeLaunch &s, hipStream_t stream) {
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
        const hipError_t e =
            hipFuncSetAttribute(reinterpret_cast<const void *>(&serve_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
        if (e != hipSuccess) note_hip_error("hipFuncSetAttribute(serve_kernel)", e);
    });
    (void)hipGetLastError();
    hipLaunchKernelGGL(serve_kernel, dim3(s.grid), dim3(kBatchLanes), s.lds, stream, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) note_hip_error("launch serve_kernel", e);
    return e;
}

int ll_message_pair_words(const int32_t *row_ptr, int rows, int alpha) {
    int e = 0;
    for (int r = 0; r < rows; ++r) {
        const int w = row_ptr[r + 1] - row_ptr[r];
        e += 2 * (alpha == 2 ? ll_row_dwords<2>(w) : alpha == 4 ? ll_row_dwords<4>(w) : (w + 1) / 2);
    }
    return e;
}

hipError_t launch_decode_batch(const BatchLaunch &b, hipStream_t stream) {
    if (b.lanes != kBatchLanes) {
        note_hip_error("decode_batch_kernel: bad workgroup size", hipErrorInvalidValue);
        return hipErrorInvalidValue;
    }
    (void)hipGetLastError();
    hipError_t e = hipSuccess;
    if (!b.counter_zeroed) {
        hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, b.counter);
        e = hipGetLastError();
        if (e != hipSuccess) {
            note_hip_error("launch reset_counter_kernel", e);
            return e;
        }
    }
    static std::once_flag attr_once[4];  // once per process, also under concurrent calls
    const int vi = (b.wmax <= 10 ? 0 : 1) + (b.row_pairs ? 2 : 0);
    const void *fns[4] = {reinterpret_cast<const void *>(&decode_batch_kernel<10, false>),
                          reinterpret_cast<const void *>(&decode_batch_kernel<20, false>),
                          reinterpret_cast<const void *>(&decode_batch_kernel<10, true>),
                          reinterpret_cast<const void *>(&decode_batch_kernel<20, true>)};
    const void *fn = fns[vi];
    std::call_once(attr_once[vi], [fn] {
        const hipError_t ea =
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
        if (ea != hipSuccess) note_hip_error("hipFuncSetAttribute(decode_batch_kernel)", ea);
    });
    (void)hipGetLastError();
#define LDPC_BATCH_ARGS                                                                          \
    b.tasks, b.jobs, b.waves, b.n_tasks, b.counter, b.msg, b.msg_per_block, b.wave_lds,         \
        b.wave_msg, b.max_iter, b.early_exit, b.beta, b.offset
    const dim3 grid(b.grid), block(b.lanes);
    switch (vi) {
        case 0: hipLaunchKernelGGL((decode_batch_kernel<10, false>), grid, block, b.lds, stream, LDPC_BATCH_ARGS); break;
        case 1: hipLaunchKernelGGL((decode_batch_kernel<20, false>), grid, block, b.lds, stream, LDPC_BATCH_ARGS); break;
        case 2: hipLaunchKernelGGL((decode_batch_kernel<10, true>), grid, block, b.lds, stream, LDPC_BATCH_ARGS); break;
        default: hipLaunchKernelGGL((decode_batch_kernel<20, true>), grid, block, b.lds, stream, LDPC_BATCH_ARGS); break;
    }
#undef LDPC_BATCH_ARGS
    e = hipGetLastError();
    if (e != hipSuccess) note_hip_error("launch decode_batch_kernel", e);
    return e;
}

}  // namespace ldpc
