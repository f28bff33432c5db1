// Layered normalised min-sum decoding in 8-bit saturating fixed point for
// gfx950 (Ling & Cautereels, §III decoding rules, §IV min/second-min/sign
// intermediates and the 8-bit number format).
//
// One workgroup decodes `cpw` codewords; each codeword's posteriors L_v and
// check-to-variable messages L_{c->v} live in LDS for the whole decode
// (BG1-shaped at Z = 384: 26,112 + 121,344 bytes). Lane u of a codeword
// owns the check rows u and u + Z/2 of every block row, so the Z independent
// rows of a layer (§II) run as Z/2 lanes with two rows each in packed 16-bit
// VALU arithmetic. Layers run strictly in order with one workgroup barrier
// each; after every iteration the full syndrome of the hard decisions is
// checked and a codeword whose checks all hold stops changing.
//
// Storage: pair words (16 bit) -- the low byte is the value for row/variable
// p, the high byte for p + Z/2. In registers each int8 value sits in the
// HIGH byte of a 16-bit lane ("x * 256"), so the int16 saturating subtract
// clamps at +127 (plus a low byte of 0xFF) and one max clamps at -127; the
// low byte is cleared before a value is negated or stored.
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
constexpr uint32_t kUnpack = 0x010c000cu;      // word -> (b0 << 8, b1 << 24)
constexpr uint32_t kUnpackSwap = 0x000c010cu;  // word -> (b1 << 8, b0 << 24)
constexpr uint32_t kPack = 0x0c0c0301u;        // inverse of kUnpack
constexpr uint32_t kPackSwap = 0x0c0c0103u;    // inverse of kUnpackSwap

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

// Where lane u's two rows meet block `md`: byte offset of the pair word
// from the lane's base (lb = codeword posteriors + 2u) and the unpack/pack
// selectors. The offset is one compare, one select and one three-way add.
struct Gather {
    int off;
    uint32_t sel_unpack, sel_pack;
};

__device__ inline Gather gather(uint32_t md, int u, int Zh2) {
    const int word = (int)(md & 0xFFFFu);
    const int thr = (int)((md >> 16) & 0xFFu);
    const bool shi = (md >> 24) & 1u;
    const bool wrap = u >= thr;
    Gather g;
    g.off = 2 * word + (wrap ? -Zh2 : 0);
    const bool swap = wrap != shi;
    g.sel_unpack = swap ? kUnpackSwap : kUnpack;
    g.sel_pack = swap ? kPackSwap : kPack;
    return g;
}

// Message of block e for a lane: 16 bits at byte offset 2*(e*Zh + ro) from
// the workgroup's uniform base (LDS or device memory). Unsigned 32-bit
// offsets let a device access use the scalar-base + vector-offset form.
__device__ inline uint32_t msg_ld(const uint16_t *Rb, int e, int Zh, int ro) {
    const uint32_t off = 2u * (uint32_t)(e * Zh + ro);
    return *reinterpret_cast<const uint16_t *>(reinterpret_cast<const uint8_t *>(Rb) + off);
}
__device__ inline void msg_st(uint16_t *Rb, int e, int Zh, int ro, uint32_t v) {
    const uint32_t off = 2u * (uint32_t)(e * Zh + ro);
    *reinterpret_cast<uint16_t *>(reinterpret_cast<uint8_t *>(Rb) + off) = (uint16_t)v;
}

// 16-bit LDS load/store at a byte offset from lb. The load's upper half is
// left unspecified: every consumer goes through v_perm, which reads only
// bytes 0 and 1.
__device__ inline uint32_t lds_ld16(const uint8_t *lb, int off) {
    return *reinterpret_cast<const uint16_t *>(lb + off);
}
__device__ inline void lds_st16(uint8_t *lb, int off, uint32_t v) {
    *reinterpret_cast<uint16_t *>(lb + off) = (uint16_t)v;
}

// Variable-to-check messages of blocks K0..K1-1 of the row: reads first
// (messages, then posteriors), then x = sat(L - R), folded into m1 / m2 / S.
template <int K0, int K1, bool KEEP_GATHER>
__device__ __forceinline__ void row_phase1(const uint8_t *__restrict__ lb,
                                           const uint16_t *__restrict__ Rb, int ro,
                                           const uint32_t *md, int e0, int u, int Zh,
                                           bool first_iter, uint32_t *xv, uint32_t *axv, int *la,
                                           uint32_t *sp, u16x2 &m1, u16x2 &m2, uint32_t &S) {
    constexpr int n = K1 - K0;
    uint32_t lraw[n], rraw[n], su[n];
    if (!first_iter) {
#pragma unroll
        for (int i = 0; i < n; ++i) rraw[i] = msg_ld(Rb, e0 + K0 + i, Zh, ro);
    } else {
#pragma unroll
        for (int i = 0; i < n; ++i) rraw[i] = 0;
    }
#pragma unroll
    for (int i = 0; i < n; ++i) {
        const Gather g = gather(md[K0 + i], u, 2 * Zh);
        su[i] = g.sel_unpack;
        if (KEEP_GATHER) {
            la[K0 + i] = g.off;
            sp[K0 + i] = g.sel_pack;
        }
        lraw[i] = lds_ld16(lb, g.off);
    }
#pragma unroll
    for (int i = 0; i < n; ++i) {
        const s16x2 L = as_s(perm(lraw[i], su[i]));
        const s16x2 R = as_s(perm(rraw[i], kUnpack));
        s16x2 x = __builtin_elementwise_sub_sat(L, R);
        x = __builtin_elementwise_max(x, (s16x2){-127 * 256, -127 * 256});
        const s16x2 ax = __builtin_elementwise_max(x, (s16x2){0, 0} - x);
        const u16x2 axu = as_u(bits_of(ax));
        m2 = __builtin_elementwise_min(m2, __builtin_elementwise_max(m1, axu));
        m1 = __builtin_elementwise_min(m1, axu);
        S ^= bits_of(x);
        xv[K0 + i] = bits_of(x);
        if (KEEP_GATHER) axv[K0 + i] = bits_of(ax);
    }
}

// One block row of exactly W blocks for lane u (rows u and u + Zh):
// variable-to-check messages, min / second min / sign product,
// normalisation, check-to-variable messages and posterior write-back.
// Specialising on W keeps the row free of branches, so the row's metadata
// arrives in one batch of scalar loads and the LDS reads are issued before
// any arithmetic (scalar and LDS loads share one completion counter; a
// scalar result consumed between LDS reads would serialise them).
// Message of block e for this lane: Rb[e * Zh + ro], with Rb uniform across
// the workgroup (LDS or device memory, carried by the pointer's address
// space) and ro a 32-bit lane offset, so a device access is a scalar base
// plus one vector offset. Rows wider than 10 blocks read in two halves and
// recompute |x| and their gathers for the write-back, which keeps the
// kernel under the register budget of six codewords per CU.
template <int W>
__device__ __forceinline__ void row_update_w(uint8_t *__restrict__ lb,
                                             uint16_t *__restrict__ Rb, int ro,
                                             cmeta_t meta, int e0, int u,
                                             int Zh, bool first_iter, u16x2 wgt, u16x2 off16) {
    constexpr bool kWide = W > 10;
    uint32_t md[W];
#pragma unroll
    for (int k = 0; k < W; ++k) md[k] = meta[e0 + k];
    uint32_t xv[W], axv[W], sp[W];
    int la[W];
    u16x2 m1 = {0x7FFF, 0x7FFF}, m2 = {0x7FFF, 0x7FFF};
    uint32_t S = 0;
    if constexpr (kWide) {
        constexpr int H = (W + 1) / 2;
        row_phase1<0, H, false>(lb, Rb, ro, md, e0, u, Zh, first_iter, xv, axv, la, sp, m1, m2,
                                S);
        row_phase1<H, W, false>(lb, Rb, ro, md, e0, u, Zh, first_iter, xv, axv, la, sp, m1, m2,
                                S);
    } else {
        row_phase1<0, W, true>(lb, Rb, ro, md, e0, u, Zh, first_iter, xv, axv, la, sp, m1, m2, S);
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
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const s16x2 x = as_s(xv[k]);
        const s16x2 ax = kWide ? __builtin_elementwise_max(x, (s16x2){0, 0} - x) : as_s(axv[k]);
        // t = 1 on the argmin edge (|x| == m1), else 0.
        const u16x2 t = __builtin_elementwise_sub_sat(m1p, as_u(bits_of(ax)));
        const s16x2 b = as_s(bits_of(t * d21 + as_u(bits_of(b1))));
        // R' = sgn(x) * b; L' = sat(x + R'). The low byte of x is 0 or 0xFF
        // and that of R' is 0, so no carry reaches the high byte.
        const s16x2 sx = x >> (s16x2){15, 15};
        const s16x2 Rn = (b ^ sx) - sx;
        const s16x2 Ln = __builtin_elementwise_max(__builtin_elementwise_add_sat(x, Rn),
                                                   (s16x2){-127 * 256, -127 * 256});
        if (kWide) {
            const Gather g = gather(md[k], u, 2 * Zh);
            lds_st16(lb, g.off, perm(bits_of(Ln), g.sel_pack));
        } else {
            lds_st16(lb, la[k], perm(bits_of(Ln), sp[k]));
        }
        msg_st(Rb, e0 + k, Zh, ro, perm(bits_of(Rn), kPack));
    }
}

// Parity of lane u's two rows over a row of exactly W blocks, as sign bits
// 15 and 31 (hard decision [L_v < 0]).
template <int W>
__device__ __forceinline__ uint32_t row_parity_w(const uint8_t *__restrict__ lb,
                                                 cmeta_t meta, int e0, int u,
                                                 int Zh) {
    uint32_t md[W], raw[W], su[W];
#pragma unroll
    for (int k = 0; k < W; ++k) md[k] = meta[e0 + k];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const Gather g = gather(md[k], u, 2 * Zh);
        su[k] = g.sel_unpack;
        raw[k] = lds_ld16(lb, g.off);
    }
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) acc ^= perm(raw[k], su[k]);
    return acc;
}

// Scalar dispatch on the row weight w in [W, WMAX].
template <int W, int WMAX>
__device__ __forceinline__ void row_update(int w, uint8_t *lb, uint16_t *Rb, int ro,
                                           cmeta_t meta, int e0, int u, int Zh,
                                           bool first_iter, u16x2 wgt, u16x2 off16) {
    if constexpr (W <= WMAX) {
        if (w == W) {
            row_update_w<W>(lb, Rb, ro, meta, e0, u, Zh, first_iter, wgt, off16);
            return;
        }
        row_update<W + 1, WMAX>(w, lb, Rb, ro, meta, e0, u, Zh, first_iter, wgt, off16);
    }
}

template <int W, int WMAX>
__device__ __forceinline__ uint32_t row_parity(int w, const uint8_t *lb, cmeta_t meta,
                                               int e0, int u, int Zh) {
    if constexpr (W <= WMAX) {
        if (w == W) return row_parity_w<W>(lb, meta, e0, u, Zh);
        return row_parity<W + 1, WMAX>(w, lb, meta, e0, u, Zh);
    }
    return 0;
}

// Nonzero if some check of lane u's two rows fails on the current hard
// decisions.
template <int WMAX>
__device__ inline uint32_t syndrome_fails(const uint8_t *__restrict__ lb,
                                          crow_t row_ptr, cmeta_t meta, int rows, int u,
                                          int Zh) {
    uint32_t bad = 0;
    for (int r = 0; r < rows; ++r) {
        const int e0 = row_ptr[r], w = row_ptr[r + 1] - e0;
        bad |= row_parity<2, WMAX>(w, lb, meta, e0, u, Zh);
    }
    return bad & 0x80008000u;
}

// Decodes `bw.n` codewords of one shape in this workgroup: codeword `slot`
// is held by lanes [slot*Z/2, (slot+1)*Z/2); lanes beyond n*Z/2 only join
// the barriers. Every thread of the workgroup must call it.
// MSG_IN_LDS: the check-to-variable messages live next to the posteriors in
// LDS (one BG1-shaped Z = 384 codeword fills a CU); otherwise they stream
// through device memory (bw.msg, [n][E][Z/2] pair words) and only the
// posteriors occupy LDS, so several codewords share a CU (§IV's placement
// of L_v in shared memory and L_{c->v} in main memory).
template <int WMAX, bool MSG_IN_LDS>
__device__ __forceinline__ void decode_block(const BlockWork &bw, uint8_t *smem, crow_t row_ptr,
                                             cmeta_t meta) {
    static_assert(WMAX <= kMetaPad, "row metadata window exceeds the table padding");
    const int Z = bw.Z, Zh = Z >> 1;
    const int N = bw.n_cols, E = bw.E, T = (N - 2) * Z;
    const int slot_bytes = MSG_IN_LDS ? lds_bytes_i8(N, E, Z) : lds_bytes_i8_post(N, Z);
    const int slot = threadIdx.x / Zh;
    const int u = threadIdx.x - slot * Zh;
    const bool valid = slot < bw.n;
    const int sl = valid ? slot : 0;  // keeps idle lanes' pointers in range
    uint16_t *Lw = reinterpret_cast<uint16_t *>(smem + sl * slot_bytes);
    // Lane base for gathers: the codeword's posteriors plus 2u bytes.
    uint8_t *lb = reinterpret_cast<uint8_t *>(Lw) + 2 * u;
    // Messages: uniform base plus a 32-bit lane offset (see row_update_w).
    uint16_t *Rb;
    int ro;
    if (MSG_IN_LDS) {
        Rb = reinterpret_cast<uint16_t *>(smem) + N * Zh;
        ro = sl * (slot_bytes / 2) + u;
    } else {
        Rb = bw.msg;
        ro = sl * E * Zh + u;
    }
    int *flags = reinterpret_cast<int *>(smem + bw.slots * slot_bytes);

    // Initialisation: punctured columns 0 and 1 carry no channel LLR.
    if (valid) {
        Lw[u] = 0;
        Lw[Zh + u] = 0;
        const int8_t *q = bw.llr + (size_t)slot * T;
#pragma unroll 1
        for (int c = 2; c < N; ++c) {
            int lo = q[(c - 2) * Z + u], hi = q[(c - 2) * Z + u + Zh];
            lo = lo < -127 ? -127 : lo;
            hi = hi < -127 ? -127 : hi;
            Lw[c * Zh + u] = (uint16_t)((lo & 0xFF) | ((hi & 0xFF) << 8));
        }
    }
    __syncthreads();

    const u16x2 off16 = {(unsigned short)(bw.offset << 8), (unsigned short)(bw.offset << 8)};
    bool done = !valid;
    int iters = bw.max_iter, ok = 0;
    for (int t = 1; t <= bw.max_iter; ++t) {
        int wt = bw.beta;
        // weights through the constant address space: a scalar load per row
        typedef const __attribute__((address_space(4))) uint8_t *cw8_t;
        cw8_t wrow = nullptr;
        if (bw.wq)
            wrow = (cw8_t)(bw.wq + (size_t)((t < bw.w_iters ? t : bw.w_iters) - 1) * bw.w_stride);
        for (int r = 0; r < bw.rows; ++r) {
            const int e0 = row_ptr[r], w = row_ptr[r + 1] - e0;
            if (wrow) wt = wrow[r];
            const u16x2 wgt = {(unsigned short)wt, (unsigned short)wt};
            if (!done) row_update<2, WMAX>(w, lb, Rb, ro, meta, e0, u, Zh, t == 1, wgt, off16);
            __syncthreads();
        }
        if (bw.early_exit || t == bw.max_iter) {
            if ((int)threadIdx.x < bw.slots) flags[threadIdx.x] = 0;
            __syncthreads();
            if (!done && syndrome_fails<WMAX>(lb, row_ptr, meta, bw.rows, u, Zh))
                atomicOr(&flags[slot], 1);
            __syncthreads();
            const bool holds = flags[sl] == 0;
            if (!done) {
                if (bw.early_exit && holds) {
                    done = true;
                    iters = t;
                    ok = 1;
                } else if (t == bw.max_iter) {
                    ok = holds;
                }
            }
            if (bw.early_exit && __syncthreads_and(done)) break;
            __syncthreads();
        }
    }
    if (valid) {
        // Outputs: hard decisions of the K information bits packed LSB
        // first. Byte j of a codeword covers bits 8j..8j+7, all in one block
        // column since Z is a multiple of 8; lane u packs byte u of each
        // column.
        const uint8_t *Lb = reinterpret_cast<const uint8_t *>(Lw);
        const int bytes_per_col = Z / 8;
        uint8_t *ob = bw.out_bits + (size_t)slot * (bw.kb * bytes_per_col);
#pragma unroll 1
        for (int c = 0; c < bw.kb; ++c) {
#pragma unroll 1
            for (int j = u; j < bytes_per_col; j += Zh) {
                uint32_t byte = 0;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int z = 8 * j + i;
                    const int hi = z >= Zh;
                    const int8_t L = (int8_t)Lb[2 * (c * Zh + z - hi * Zh) + hi];
                    byte |= (uint32_t)(L < 0) << i;
                }
                ob[c * bytes_per_col + j] = (uint8_t)byte;
            }
        }
        if (u == 0) {
            bw.out_iters[slot] = iters;
            if (bw.out_ok) bw.out_ok[slot] = (uint8_t)ok;
        }
        if (bw.out_llr) {
            int8_t *o = bw.out_llr + (size_t)slot * N * Z;
#pragma unroll 1
            for (int c = 0; c < N; ++c) {
                const uint16_t w = Lw[c * Zh + u];
                o[c * Z + u] = (int8_t)(w & 0xFF);
                o[c * Z + u + Zh] = (int8_t)(w >> 8);
            }
        }
    }
}

template <int WMAX, bool MSG_IN_LDS>
__global__ __launch_bounds__(512) void decode_i8_kernel(DecodeLaunch p,
                                                         const int32_t *__restrict__ row_ptr,
                                                         const uint32_t *__restrict__ meta) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int Zh = p.Z >> 1, T = (p.n_cols - 2) * p.Z, first = blockIdx.x * p.cpw;
    BlockWork bw;
    bw.n = p.n_cw - first < p.cpw ? p.n_cw - first : p.cpw;
    bw.slots = p.cpw;
    bw.llr = p.llr + (size_t)first * T;
    bw.out_bits = p.out_bits + (size_t)first * (p.kb * p.Z / 8);
    bw.out_iters = p.out_iters + first;
    bw.out_ok = p.out_ok ? p.out_ok + first : nullptr;
    bw.out_llr = p.out_llr ? static_cast<int8_t *>(p.out_llr) + (size_t)first * p.n_cols * p.Z
                           : nullptr;
    bw.msg = MSG_IN_LDS ? nullptr
                        : reinterpret_cast<uint16_t *>(p.msg) + (size_t)first * p.E * Zh;
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
    decode_block<WMAX, MSG_IN_LDS>(bw, smem, (crow_t)row_ptr, (cmeta_t)meta);
}

template <int WMAX, bool MSG_IN_LDS>
hipError_t launch_w(const DecodeLaunch &p, hipStream_t stream) {
    const int Zh = p.Z / 2;
    const int per_cw = MSG_IN_LDS ? lds_bytes_i8(p.n_cols, p.E, p.Z)
                                  : lds_bytes_i8_post(p.n_cols, p.Z);
    const int lds = p.cpw * per_cw + p.cpw * (int)sizeof(int);
    static bool attr_set = false;
    if (!attr_set) {
        // Opt in to more than the default 64 KiB of dynamic LDS.
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&decode_i8_kernel<WMAX, MSG_IN_LDS>),
            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
        if (e != hipSuccess) note_hip_error("hipFuncSetAttribute(decode_i8_kernel)", e);
        attr_set = true;
    }
    const int blocks = (p.n_cw + p.cpw - 1) / p.cpw;
    // hipGetLastError reports the last error of ANY earlier runtime call on
    // this thread; clear it so the check below sees this launch only.
    (void)hipGetLastError();
    hipLaunchKernelGGL((decode_i8_kernel<WMAX, MSG_IN_LDS>), dim3(blocks), dim3(p.cpw * Zh), lds,
                       stream, p, p.row_ptr, p.meta);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) note_hip_error("launch decode_i8_kernel", e);
    return e;
}

template <bool MSG_IN_LDS>
hipError_t launch_placed(const DecodeLaunch &p, hipStream_t stream) {
    if (p.wmax <= 10) return launch_w<10, MSG_IN_LDS>(p, stream);
    if (p.wmax <= 20) return launch_w<20, MSG_IN_LDS>(p, stream);
    return launch_w<32, MSG_IN_LDS>(p, stream);
}


// Persistent mixed-shape decode: each workgroup takes tasks (up to a
// workgroup's worth of codewords of one shape) from a device counter until
// none are left, so every wave reaches the exit once the counter passes
// n_tasks. Messages use the device placement with one region per
// workgroup, reused from task to task.
template <int WMAX>
__global__ __launch_bounds__(256) void decode_batch_kernel(const BatchTask *__restrict__ tasks,
                                                            const BatchJob *__restrict__ jobs,
                                                            int n_tasks, unsigned *counter,
                                                            uint16_t *msg_ws, int msg_per_block,
                                                            int max_iter, int early_exit,
                                                            int beta, int offset) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ int task_id;
    for (;;) {
        if (threadIdx.x == 0) task_id = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int ti = task_id;
        __syncthreads();
        if (ti >= n_tasks) break;
        const BatchTask tk = tasks[ti];
        const BatchJob &jb = jobs[tk.job];
        const int T = (jb.n_cols - 2) * jb.Z;
        BlockWork bw;
        bw.n = tk.n;
        bw.slots = jb.slots;
        bw.llr = jb.llr + (size_t)tk.first * T;
        bw.out_bits = jb.out_bits + (size_t)tk.first * (jb.kb * jb.Z / 8);
        bw.out_iters = jb.out_iters + tk.first;
        bw.out_ok = jb.out_ok ? jb.out_ok + tk.first : nullptr;
        bw.out_llr = nullptr;
        bw.msg = msg_ws + (size_t)blockIdx.x * msg_per_block;
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
        decode_block<WMAX, false>(bw, smem, (crow_t)jb.row_ptr, (cmeta_t)jb.meta);
        __syncthreads();
    }
}

__global__ void reset_counter_kernel(unsigned *counter) { *counter = 0u; }

}  // namespace

hipError_t launch_decode_i8(const DecodeLaunch &p, hipStream_t stream) {
    return p.msg ? launch_placed<false>(p, stream) : launch_placed<true>(p, stream);
}

hipError_t launch_decode_batch(const BatchLaunch &b, hipStream_t stream) {
    (void)hipGetLastError();
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, b.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        note_hip_error("launch reset_counter_kernel", e);
        return e;
    }
    static bool attr_set[2] = {false, false};
    const void *fn = b.wmax <= 10 ? reinterpret_cast<const void *>(&decode_batch_kernel<10>)
                                  : reinterpret_cast<const void *>(&decode_batch_kernel<20>);
    bool &set = attr_set[b.wmax <= 10 ? 0 : 1];
    if (!set) {
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
        if (e != hipSuccess) note_hip_error("hipFuncSetAttribute(decode_batch_kernel)", e);
        set = true;
    }
    (void)hipGetLastError();
    if (b.wmax <= 10)
        hipLaunchKernelGGL(decode_batch_kernel<10>, dim3(b.grid), dim3(b.lanes), b.lds, stream,
                           b.tasks, b.jobs, b.n_tasks, b.counter, b.msg, b.msg_per_block,
                           b.max_iter, b.early_exit, b.beta, b.offset);
    else
        hipLaunchKernelGGL(decode_batch_kernel<20>, dim3(b.grid), dim3(b.lanes), b.lds, stream,
                           b.tasks, b.jobs, b.n_tasks, b.counter, b.msg, b.msg_per_block,
                           b.max_iter, b.early_exit, b.beta, b.offset);
    e = hipGetLastError();
    if (e != hipSuccess) note_hip_error("launch decode_batch_kernel", e);
    return e;
}

}  // namespace ldpc
