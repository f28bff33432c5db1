// Learned (neural) weighted min-sum in fp32: unrolled forward pass and its
// hand-written backward pass (Ling & Cautereels §III layered min-sum, with
// the correction factor replaced by one trainable multiplier per
// (iteration, block row)).
//
// Forward (one workgroup per codeword, one check row z per lane): the
// layered schedule with L_v in LDS, check-to-variable messages R in device
// memory; every variable-to-check message x is recorded on a device tape,
// and after each iteration t the loss gradient of the posteriors,
//     dLoss/dL_tj = lambda_t * (c_j - sigmoid(-L_tj/scale)) / (N*Z * scale),
// is stored (loss = sum over t of lambda_t times the mean over j of
// BCE(sigmoid(-L_tj/scale), c_j); lambda_t = iter_w[t], or 1/n_iter).
// Backward: the same schedule in reverse with dLoss/dL in LDS and dLoss/dR
// in device memory; per check row, with signs and argmins fixed,
//     g_k  = (gL'_k + gR'_k) * s_k,  dw += sum_k g_k * (k == k1 ? m2 : m1),
//     gx_k = gL'_k + [k == k1] sgn(x_k1) w sum_{j != k1} g_j
//                  + [k == k2] sgn(x_k2) w g_k1,
//     gL_k = gx_k, gR_k = -gx_k   (k1 first argmin, k2 first argmin of the
//                                   rest; sgn from the sign bit).
// The per-codeword weight gradients are summed in a fixed order.
#include "ldpc_internal.h"

namespace ldpc {
namespace {

constexpr int kNwmsWmax = 20;

__device__ inline float sgn_bit(float v) { return __builtin_signbit(v) ? -1.0f : 1.0f; }

// Variable index of check row z through a block with metadata md (c*Z in
// bits [0, 16), shift in bits [16, 25)).
__device__ inline int var_index(uint32_t md, int z, int Z) {
    const int cz = (int)(md & 0xFFFFu);
    const int s = (int)((md >> 16) & 0x1FFu);
    const int t = z + s;
    return cz + (t >= Z ? t - Z : t);
}

__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline float softplusf(float v) {
    return v > 0.0f ? v + log1pf(expf(-v)) : log1pf(expf(v));
}

template <int W>
__device__ __forceinline__ void fwd_row(float *__restrict__ L, float *__restrict__ R,
                                        float *__restrict__ tape, const uint32_t *__restrict__ meta,
                                        int e0, int z, int Z, bool first, float wt) {
    uint32_t md[W];
#pragma unroll
    for (int k = 0; k < W; ++k) md[k] = meta[e0 + k];
    float x[W];
    int vi[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        vi[k] = var_index(md[k], z, Z);
        const float r = first ? 0.0f : R[(size_t)(e0 + k) * Z + z];
        x[k] = L[vi[k]] - r;
    }
    float m1 = __builtin_inff(), m2 = __builtin_inff();
    int k1 = -1;
    uint32_t S = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        tape[(size_t)(e0 + k) * Z + z] = x[k];
        const float a = __builtin_fabsf(x[k]);
        if (a < m1) {
            m2 = m1;
            m1 = a;
            k1 = k;
        } else if (a < m2) {
            m2 = a;
        }
        S ^= __float_as_uint(x[k]);
    }
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const float mag = wt * (k == k1 ? m2 : m1);
        const float rn = ((S ^ __float_as_uint(x[k])) & 0x80000000u) ? -mag : mag;
        R[(size_t)(e0 + k) * Z + z] = rn;
        L[vi[k]] = x[k] + rn;
    }
}

template <int W>
__device__ __forceinline__ float bwd_row(float *__restrict__ gL, float *__restrict__ gR,
                                         const float *__restrict__ tape,
                                         const uint32_t *__restrict__ meta, int e0, int z, int Z,
                                         bool last, float wt) {
    uint32_t md[W];
#pragma unroll
    for (int k = 0; k < W; ++k) md[k] = meta[e0 + k];
    float x[W], g[W];
    int vi[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        vi[k] = var_index(md[k], z, Z);
        x[k] = tape[(size_t)(e0 + k) * Z + z];
    }
    float m1 = __builtin_inff(), m2 = __builtin_inff();
    int k1 = -1, k2 = -1;
    uint32_t S = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const float a = __builtin_fabsf(x[k]);
        if (a < m1) {
            m2 = m1;
            k2 = k1;
            m1 = a;
            k1 = k;
        } else if (a < m2) {
            m2 = a;
            k2 = k;
        }
        S ^= __float_as_uint(x[k]);
    }
    float gw = 0.0f, gsum = 0.0f, gk1 = 0.0f;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const float gr = last ? 0.0f : gR[(size_t)(e0 + k) * Z + z];
        const float sk = ((S ^ __float_as_uint(x[k])) & 0x80000000u) ? -1.0f : 1.0f;
        g[k] = (gL[vi[k]] + gr) * sk;
        gw += g[k] * (k == k1 ? m2 : m1);
        if (k != k1) gsum += g[k];
        if (k == k1) gk1 = g[k];
    }
#pragma unroll
    for (int k = 0; k < W; ++k) {
        float gx = gL[vi[k]];
        if (k == k1) gx += sgn_bit(x[k]) * wt * gsum;
        if (k == k2) gx += sgn_bit(x[k]) * wt * gk1;
        gL[vi[k]] = gx;
        gR[(size_t)(e0 + k) * Z + z] = -gx;
    }
    return gw;
}

template <int W>
__device__ __forceinline__ void fwd_dispatch(int w, float *L, float *R, float *tape,
                                             const uint32_t *meta, int e0, int z, int Z, bool first,
                                             float wt) {
    if constexpr (W <= kNwmsWmax) {
        if (w == W) {
            fwd_row<W>(L, R, tape, meta, e0, z, Z, first, wt);
            return;
        }
        fwd_dispatch<W + 1>(w, L, R, tape, meta, e0, z, Z, first, wt);
    }
}

template <int W>
__device__ __forceinline__ float bwd_dispatch(int w, float *gL, float *gR, const float *tape,
                                              const uint32_t *meta, int e0, int z, int Z,
                                              bool last, float wt) {
    if constexpr (W <= kNwmsWmax) {
        if (w == W) return bwd_row<W>(gL, gR, tape, meta, e0, z, Z, last, wt);
        return bwd_dispatch<W + 1>(w, gL, gR, tape, meta, e0, z, Z, last, wt);
    }
    return 0.0f;
}

// Workspace layout per codeword (floats): tape [n_iter][E][Z], dloss
// [n_iter][Nc], R [E][Z], gR [E][Z]; plus gw partials [n_cw][n_iter][rows].
struct NwmsLaunch {
    const float *llr;        // [n_cw][T]
    const uint8_t *cbits;    // [n_cw][Nc]
    const float *w;          // [n_iter][rows]
    const float *iter_w;     // [n_iter] loss weight per iteration, or null (1/n_iter)
    float *loss;             // [n_cw]
    float *out_llr;          // [n_cw][Nc] final posteriors or null
    float *ws;               // per-codeword workspace
    float *gw_part;          // [n_cw][n_iter][rows]
    size_t ws_per_cw;        // floats
    int n_cw, rows, n_cols, Z, E, n_iter;
    float scale;
};

__global__ __launch_bounds__(512) void nwms_forward_kernel(NwmsLaunch p,
                                                           const int32_t *__restrict__ row_ptr,
                                                           const uint32_t *__restrict__ meta) {
    extern __shared__ __align__(16) uint8_t smem[];
    float *L = reinterpret_cast<float *>(smem);
    __shared__ float wpart[8];
    const int Z = p.Z, N = p.n_cols, E = p.E, Nc = N * Z, T = (N - 2) * Z;
    const int cw = blockIdx.x;
    const int z = threadIdx.x;
    const bool lane = z < Z;
    float *ws = p.ws + (size_t)cw * p.ws_per_cw;
    float *tape = ws;
    float *dloss = tape + (size_t)p.n_iter * E * Z;
    float *R = dloss + (size_t)p.n_iter * Nc;
    const uint8_t *c = p.cbits + (size_t)cw * Nc;
    if (lane) {
        L[z] = 0.0f;
        L[Z + z] = 0.0f;
        for (int col = 2; col < N; ++col) L[col * Z + z] = p.llr[(size_t)cw * T + (col - 2) * Z + z];
    }
    __syncthreads();
    float lsum = 0.0f;
    for (int t = 0; t < p.n_iter; ++t) {
        const float lam = p.iter_w ? p.iter_w[t] : 1.0f / (float)p.n_iter;
        const float coef = lam / ((float)Nc * p.scale);
        float *tp = tape + (size_t)t * E * Z;
        for (int r = 0; r < p.rows; ++r) {
            const int e0 = row_ptr[r], w = row_ptr[r + 1] - e0;
            const float wt = p.w[t * p.rows + r];
            if (lane) fwd_dispatch<2>(w, L, R, tp, meta, e0, z, Z, t == 0, wt);
            __syncthreads();
        }
        if (lane) {
            float *dl = dloss + (size_t)t * Nc;
            for (int col = 0; col < N; ++col) {
                const int j = col * Z + z;
                const float y = L[j] / p.scale;
                const float pr = 1.0f / (1.0f + expf(y));  // sigmoid(-y)
                dl[j] = ((float)c[j] - pr) * coef;
                lsum += lam * (c[j] ? softplusf(y) : softplusf(-y));
            }
        }
    }
    if (p.out_llr && lane)
        for (int col = 0; col < N; ++col) p.out_llr[(size_t)cw * Nc + col * Z + z] = L[col * Z + z];
    // loss of the codeword: weighted over iterations, mean over bits
    const float ws_sum = wave_sum(lane ? lsum : 0.0f);
    if ((threadIdx.x & 63) == 0) wpart[threadIdx.x >> 6] = ws_sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += wpart[i];
        p.loss[cw] = s / (float)Nc;
    }
}

__global__ __launch_bounds__(512) void nwms_backward_kernel(NwmsLaunch p,
                                                            const int32_t *__restrict__ row_ptr,
                                                            const uint32_t *__restrict__ meta) {
    extern __shared__ __align__(16) uint8_t smem[];
    float *gL = reinterpret_cast<float *>(smem);
    __shared__ float wpart[2][8];
    const int Z = p.Z, N = p.n_cols, E = p.E, Nc = N * Z;
    const int cw = blockIdx.x;
    const int z = threadIdx.x;
    const bool lane = z < Z;
    const int nw = blockDim.x >> 6;
    float *ws = p.ws + (size_t)cw * p.ws_per_cw;
    const float *tape = ws;
    const float *dloss = tape + (size_t)p.n_iter * E * Z;
    float *gR = const_cast<float *>(dloss) + (size_t)p.n_iter * Nc + (size_t)E * Z;
    float *gwp = p.gw_part + (size_t)cw * p.n_iter * p.rows;
    if (lane)
        for (int col = 0; col < N; ++col) gL[col * Z + z] = 0.0f;
    __syncthreads();
    int step = 0;
    for (int t = p.n_iter - 1; t >= 0; --t) {
        if (lane) {
            const float *dl = dloss + (size_t)t * Nc;
            for (int col = 0; col < N; ++col) gL[col * Z + z] += dl[col * Z + z];
        }
        __syncthreads();
        const float *tp = tape + (size_t)t * E * Z;
        for (int r = p.rows - 1; r >= 0; --r, ++step) {
            const int e0 = row_ptr[r], w = row_ptr[r + 1] - e0;
            const float wt = p.w[t * p.rows + r];
            float gw = 0.0f;
            if (lane) gw = bwd_dispatch<2>(w, gL, gR, tp, meta, e0, z, Z, t == p.n_iter - 1, wt);
            gw = wave_sum(gw);
            // double-buffered wave partials; summed in a fixed order by
            // thread 0 after the row's barrier
            if ((threadIdx.x & 63) == 0) wpart[step & 1][threadIdx.x >> 6] = gw;
            __syncthreads();
            if (threadIdx.x == 0) {
                float s = 0.0f;
                for (int i = 0; i < nw; ++i) s += wpart[step & 1][i];
                gwp[t * p.rows + r] = s;
            }
        }
    }
}

// grad[i] = sum over codewords of gw_part[cw][i], in codeword order.
__global__ void nwms_reduce_kernel(const float *__restrict__ part, int n_cw, int n, float *grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int c = 0; c < n_cw; ++c) s += part[(size_t)c * n + i];
    grad[i] = s;
}

}  // namespace

size_t nwms_workspace_floats(int n_cw, int rows, int n_cols, int Z, int E, int n_iter) {
    const size_t per = (size_t)n_iter * E * Z + (size_t)n_iter * n_cols * Z + 2 * (size_t)E * Z;
    return per * n_cw + (size_t)n_cw * n_iter * rows;
}

hipError_t launch_nwms(const float *llr, const uint8_t *cbits, const float *w,
                       const float *iter_w, float *loss, float *grad, float *out_llr, float *ws, int n_cw, int rows, int n_cols,
                       int Z, int E, int n_iter, float scale, const int32_t *row_ptr,
                       const uint32_t *meta_row, int wmax, hipStream_t stream) {
    if (wmax > kNwmsWmax) return hipErrorInvalidValue;
    NwmsLaunch p{};
    p.llr = llr;
    p.cbits = cbits;
    p.w = w;
    p.iter_w = iter_w;
    p.loss = loss;
    p.out_llr = out_llr;
    p.ws = ws;
    p.ws_per_cw = (size_t)n_iter * E * Z + (size_t)n_iter * n_cols * Z + 2 * (size_t)E * Z;
    p.gw_part = ws + p.ws_per_cw * n_cw;
    p.n_cw = n_cw;
    p.rows = rows;
    p.n_cols = n_cols;
    p.Z = Z;
    p.E = E;
    p.n_iter = n_iter;
    p.scale = scale;
    const int threads = (Z + 63) / 64 * 64;
    const int lds = n_cols * Z * (int)sizeof(float);
    static std::once_flag attr_once;  // once per process, also under concurrent calls
    std::call_once(attr_once, [] {
        hipError_t e1 = hipFuncSetAttribute(reinterpret_cast<const void *>(&nwms_forward_kernel),
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            max_lds_bytes());
        hipError_t e2 = hipFuncSetAttribute(reinterpret_cast<const void *>(&nwms_backward_kernel),
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            max_lds_bytes());
        if (e1 != hipSuccess) note_hip_error("hipFuncSetAttribute(nwms_forward_kernel)", e1);
        if (e2 != hipSuccess) note_hip_error("hipFuncSetAttribute(nwms_backward_kernel)", e2);
    });
    (void)hipGetLastError();
    hipLaunchKernelGGL(nwms_forward_kernel, dim3(n_cw), dim3(threads), lds, stream, p, row_ptr,
                       meta_row);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        note_hip_error("launch nwms_forward_kernel", e);
        return e;
    }
    hipLaunchKernelGGL(nwms_backward_kernel, dim3(n_cw), dim3(threads), lds, stream, p, row_ptr,
                       meta_row);
    e = hipGetLastError();
    if (e != hipSuccess) {
        note_hip_error("launch nwms_backward_kernel", e);
        return e;
    }
    const int n = n_iter * rows;
    hipLaunchKernelGGL(nwms_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, stream,
                       p.gw_part, n_cw, n, grad);
    e = hipGetLastError();
    if (e != hipSuccess) note_hip_error("launch nwms_reduce_kernel", e);
    return e;
}

}  // namespace ldpc
