// Kernels of the learned reserve surrogate (gfx950).
//
// Matrix work runs on the bfloat16 MFMA (v_mfma_f32_16x16x32_bf16, FP32
// accumulation).  In one such instruction lane l holds, of a 16x32 A tile,
// row l%16 and columns 8(l/16) .. 8(l/16)+7; of a 32x16 B tile, rows
// 8(l/16) .. +7 of column l%16; and of the 16x16 result, rows 4(l/16) .. +3
// of column l%16.
//
// Training uses a plain GEMM kernel C = A B^T over operands stored with the
// contraction index contiguous, with fused epilogues.  Inference uses a fused
// kernel that computes the transposed layers Z^T = W^T X^T for 64 rows per
// wavefront: the result of one layer is, lane for lane, already the B operand
// of the next (up to a fixed permutation of the hidden units, which is folded
// into the order of the next layer's weights), so activations never leave
// registers and the weights sit in LDS.
#include "rr_mlp.h"

#include <algorithm>

namespace rr {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 load8(const bf16_t *p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(p));
}

// Round to nearest even: two FP32 values -> packed bfloat16 (a in the low half).
__device__ __forceinline__ unsigned int pack2(float a, float b)
{
    const f32x2 v = {a, b};
    return __builtin_bit_cast(unsigned int, __builtin_convertvector(v, bf16x2));
}

__device__ __forceinline__ float from_bf16(bf16_t h) { return __uint_as_float((unsigned int)h << 16); }

__device__ __forceinline__ bf16x8 pack8(f32x4 a, f32x4 b)
{
    const u32x4 u = {pack2(a[0], a[1]), pack2(a[2], a[3]), pack2(b[0], b[1]), pack2(b[2], b[3])};
    return __builtin_bit_cast(bf16x8, u);
}

// GELU, tanh form (Hendrycks and Gimpel, 2016): 0.5 x (1 + tanh(u)),
// u = sqrt(2/pi) (x + 0.044715 x^3), evaluated as x * sigmoid(2u) with the
// hardware base-2 exponential and reciprocal.
constexpr float GELU_W0 = 1.5957691216057308f;                     // 2 sqrt(2/pi)
constexpr float GELU_K0 = -1.5957691216057308f * 1.4426950408889634f;  // -2 sqrt(2/pi) log2(e)
constexpr float GELU_K1 = GELU_K0 * 0.044715f;

__device__ __forceinline__ float sig2u(float x)
{
    const float t = x * x;
    const float e = __builtin_amdgcn_exp2f(x * fmaf(t, GELU_K1, GELU_K0));
    return __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ __forceinline__ float gelu_f(float x) { return x * sig2u(x); }

__device__ __forceinline__ float gelu_grad_f(float x)
{
    const float s = sig2u(x);
    const float w1 = fmaf(x * x, 3.0f * 0.044715f * GELU_W0, GELU_W0);   // d(2u)/dx
    return fmaf(x * s * (1.0f - s), w1, s);
}

__device__ __forceinline__ f32x4 gelu4(f32x4 z)
{
    return f32x4{gelu_f(z[0]), gelu_f(z[1]), gelu_f(z[2]), gelu_f(z[3])};
}

// Sum over a wavefront by an XOR butterfly: every lane ends with the same bits.
__device__ __forceinline__ float wave_sum_f(float x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// ---------------------------------------------------------------------------
// Training GEMM: C[m][n] = sum_k A[m][k] B[n][k]
// A workgroup computes a 64 x 64 tile, each wavefront a 32 x 32 quarter of
// it as 2 x 2 MFMA tiles, reading 16-byte fragments straight from memory.
// ---------------------------------------------------------------------------
template <int EPI>
__device__ __forceinline__ void gemm_store(const Gemm &g, f32x4 c, int mb, int nb, int lane)
{
    const int n = nb + (lane & 15);
    const int m = mb + (lane >> 4) * 4;
    if constexpr (EPI == EPI_PARTIAL) {
        float *C = g.C + (long long)blockIdx.z * g.M * g.N;
#pragma unroll
        for (int i = 0; i < 4; ++i) C[(long long)(m + i) * g.N + n] = c[i];
    } else if constexpr (EPI == EPI_FWD) {
        const float b = g.bias[n];
        f32x4 z, a;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            z[i] = c[i] + b;
            a[i] = gelu_f(z[i]);
        }
        if (g.Z) {
#pragma unroll
            for (int i = 0; i < 4; ++i) g.Z[(long long)(m + i) * g.N + n] = z[i];
        }
        const unsigned int lo = pack2(a[0], a[1]), hi = pack2(a[2], a[3]);
        if (g.Aq) {
            g.Aq[(long long)(m + 0) * g.N + n] = (bf16_t)(lo & 0xffffu);
            g.Aq[(long long)(m + 1) * g.N + n] = (bf16_t)(lo >> 16);
            g.Aq[(long long)(m + 2) * g.N + n] = (bf16_t)(hi & 0xffffu);
            g.Aq[(long long)(m + 3) * g.N + n] = (bf16_t)(hi >> 16);
        }
        if (g.AqT) *reinterpret_cast<u32x2 *>(g.AqT + (long long)n * g.ldt + m) = u32x2{lo, hi};
    } else {
        f32x4 d;
#pragma unroll
        for (int i = 0; i < 4; ++i) d[i] = c[i] * gelu_grad_f(g.Zin[(long long)(m + i) * g.N + n]);
        *reinterpret_cast<u32x2 *>(g.AqT + (long long)n * g.ldt + m) =
            u32x2{pack2(d[0], d[1]), pack2(d[2], d[3])};
    }
}

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(Gemm g)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
    if (m0 >= g.M || n0 >= g.N) return;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const long long kbeg = (long long)blockIdx.z * g.K + kq;
    const bf16_t *a0 = g.A + (long long)(m0 + r) * g.lda + kbeg;
    const bf16_t *a1 = a0 + 16 * g.lda;
    const bf16_t *b0 = g.B + (long long)(n0 + r) * g.ldb + kbeg;
    const bf16_t *b1 = b0 + 16 * g.ldb;
    f32x4 c00 = {0.f, 0.f, 0.f, 0.f}, c01 = c00, c10 = c00, c11 = c00;
#pragma unroll 2
    for (int k = 0; k < g.K; k += 32) {
        const bf16x8 A0 = load8(a0 + k), A1 = load8(a1 + k);
        const bf16x8 B0 = load8(b0 + k), B1 = load8(b1 + k);
        c00 = mfma(A0, B0, c00);
        c01 = mfma(A0, B1, c01);
        c10 = mfma(A1, B0, c10);
        c11 = mfma(A1, B1, c11);
    }
    gemm_store<EPI>(g, c00, m0, n0, lane);
    gemm_store<EPI>(g, c01, m0, n0 + 16, lane);
    gemm_store<EPI>(g, c10, m0 + 16, n0, lane);
    gemm_store<EPI>(g, c11, m0 + 16, n0 + 16, lane);
}

hipError_t launch_gemm(const Gemm &g, int epi, hipStream_t s)
{
    if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.M % 32 || g.N % 32 || g.K % 32 || g.splits < 1)
        return hipErrorInvalidValue;
    const dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, g.splits);
    switch (epi) {
    case EPI_FWD: hipLaunchKernelGGL(k_gemm<EPI_FWD>, grid, dim3(256), 0, s, g); break;
    case EPI_DGELU: hipLaunchKernelGGL(k_gemm<EPI_DGELU>, grid, dim3(256), 0, s, g); break;
    case EPI_PARTIAL: hipLaunchKernelGGL(k_gemm<EPI_PARTIAL>, grid, dim3(256), 0, s, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inputs and small reductions
// ---------------------------------------------------------------------------
__global__ void k_prep_input(const float *__restrict__ z, int n, int n_pad, bf16_t *__restrict__ xq)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;   // pair of inputs
    if (i >= (long long)n_pad * K_IN / 2) return;
    const long long row = (2 * i) / K_IN;
    float a = 0.f, b = 0.f;
    if (row < n) {
        a = z[2 * i];
        b = z[2 * i + 1];
    }
    reinterpret_cast<unsigned int *>(xq)[i] = pack2(a, b);
}

hipError_t launch_prep_input(const float *z, int n, int n_pad, bf16_t *xq, hipStream_t s)
{
    const long long pairs = (long long)n_pad * K_IN / 2;
    hipLaunchKernelGGL(k_prep_input, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, z, n,
                       n_pad, xq);
    return hipGetLastError();
}

// 64 rows x 32 inputs per block through LDS.
__global__ void __launch_bounds__(256) k_transpose_x(const bf16_t *__restrict__ xq, int n,
                                                     bf16_t *__restrict__ xqt, long long ld)
{
    __shared__ bf16_t t[K_IN][ROWS + 2];
    const int r0 = blockIdx.x * ROWS;
    for (int e = threadIdx.x; e < ROWS * K_IN; e += 256) {
        const int r = e / K_IN, k = e % K_IN;
        t[k][r] = r0 + r < n ? xq[(long long)(r0 + r) * K_IN + k] : (bf16_t)0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ROWS * K_IN; e += 256) {
        const int k = e / ROWS, r = e % ROWS;
        if (r0 + r < n) xqt[(long long)k * ld + r0 + r] = t[k][r];
    }
}

hipError_t launch_transpose_x(const bf16_t *xq, int n, bf16_t *xqt, long long ld, hipStream_t s)
{
    hipLaunchKernelGGL(k_transpose_x, dim3((n + ROWS - 1) / ROWS), dim3(256), 0, s, xq, n, xqt, ld);
    return hipGetLastError();
}

// Head and output gradient: 16 rows per block, thread = hidden unit.
struct HeadArgs {
    const bf16_t *a2q;
    const float *z2;
    const float *w3e;
    const float *b3;
    const float *t;
    int n_valid;
    float inv_n;
    int grads;
    float *y, *dy, *loss_part;
    bf16_t *dz2q, *dz2qt;
    long long ldt;
};

__global__ void __launch_bounds__(256) k_head(HeadArgs h)
{
    __shared__ float part[4][16];
    __shared__ float dys[16];
    __shared__ float sq[16];
    const int o = threadIdx.x, lane = o & 63, wave = o >> 6;
    const int r0 = blockIdx.x * 16;
    const float w3 = h.w3e[o];
    for (int r = 0; r < 16; ++r) {
        const float p = wave_sum_f(from_bf16(h.a2q[(long long)(r0 + r) * HID + o]) * w3);
        if (lane == 0) part[wave][r] = p;
    }
    __syncthreads();
    if (o < 16) {
        const int r = r0 + o;
        const float y = ((part[0][o] + part[1][o]) + (part[2][o] + part[3][o])) + h.b3[0];
        h.y[r] = y;
        float d = 0.f, e2 = 0.f;
        if (h.t && r < h.n_valid) {
            const float e = y - h.t[r];
            d = 2.0f * e * h.inv_n;
            e2 = e * e;
        }
        dys[o] = d;
        sq[o] = e2;
        if (h.dy) h.dy[r] = d;
    }
    __syncthreads();
    if (o == 0 && h.loss_part) {
        float s = 0.f;
        for (int r = 0; r < 16; ++r) s += sq[r];
        h.loss_part[blockIdx.x] = s;
    }
    if (h.grads) {
        unsigned int pk[8];
#pragma unroll
        for (int r = 0; r < 16; r += 2) {
            const float g0 = dys[r] * w3 * gelu_grad_f(h.z2[(long long)(r0 + r) * HID + o]);
            const float g1 = dys[r + 1] * w3 * gelu_grad_f(h.z2[(long long)(r0 + r + 1) * HID + o]);
            pk[r / 2] = pack2(g0, g1);
            h.dz2q[(long long)(r0 + r) * HID + o] = (bf16_t)(pk[r / 2] & 0xffffu);
            h.dz2q[(long long)(r0 + r + 1) * HID + o] = (bf16_t)(pk[r / 2] >> 16);
        }
        u32x4 *dst = reinterpret_cast<u32x4 *>(h.dz2qt + (long long)o * h.ldt + r0);
        dst[0] = u32x4{pk[0], pk[1], pk[2], pk[3]};
        dst[1] = u32x4{pk[4], pk[5], pk[6], pk[7]};
    }
}

hipError_t launch_head(const bf16_t *a2q, const float *z2, const Weights &w, const float *t,
                       int n_pad, int n_valid, float inv_n, bool grads, float *y, float *dy,
                       float *loss_part, bf16_t *dz2q, bf16_t *dz2qt, long long ldt, hipStream_t s)
{
    if (n_pad % 16) return hipErrorInvalidValue;
    HeadArgs h{a2q, z2, w.w3e, w.master + OFF_B3, t, n_valid, inv_n, grads ? 1 : 0, y, dy,
               loss_part, dz2q, dz2qt, ldt};
    hipLaunchKernelGGL(k_head, dim3(n_pad / 16), dim3(256), 0, s, h);
    return hipGetLastError();
}

__device__ float block_sum_256(float x, float *red)
{
    red[threadIdx.x] = x;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

__global__ void __launch_bounds__(256) k_vec_grads(const bf16_t *__restrict__ dz1qt,
                                                   const bf16_t *__restrict__ dz2qt,
                                                   const bf16_t *__restrict__ a2qt,
                                                   const float *__restrict__ dy, long long ldt,
                                                   int n_pad, float *__restrict__ grad)
{
    __shared__ float red[256];
    const int b = blockIdx.x, tid = threadIdx.x;
    float acc = 0.f;
    int out;
    if (b < HID) {
        const bf16_t *row = dz1qt + (long long)b * ldt;
        for (int i = tid; i < n_pad; i += 256) acc += from_bf16(row[i]);
        out = OFF_B1 + b;
    } else if (b < 2 * HID) {
        const bf16_t *row = dz2qt + (long long)(b - HID) * ldt;
        for (int i = tid; i < n_pad; i += 256) acc += from_bf16(row[i]);
        out = OFF_B2 + b - HID;
    } else if (b < 3 * HID) {
        const bf16_t *row = a2qt + (long long)(b - 2 * HID) * ldt;
        for (int i = tid; i < n_pad; i += 256) acc += from_bf16(row[i]) * dy[i];
        out = OFF_W3 + b - 2 * HID;
    } else {
        for (int i = tid; i < n_pad; i += 256) acc += dy[i];
        out = OFF_B3;
    }
    const float s = block_sum_256(acc, red);
    if (tid == 0) grad[out] = s;
}

hipError_t launch_vec_grads(const bf16_t *dz1qt, const bf16_t *dz2qt, const bf16_t *a2qt,
                            const float *dy, long long ldt, int n_pad, float *grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_vec_grads, dim3(3 * HID + 1), dim3(256), 0, s, dz1qt, dz2qt, a2qt, dy,
                       ldt, n_pad, grad);
    return hipGetLastError();
}

__global__ void k_reduce_grads(const float *__restrict__ p1, int s1, const float *__restrict__ p2,
                               int s2, float *__restrict__ grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < K_IN * HID) {
        float a = 0.f;
        for (int z = 0; z < s1; ++z) a += p1[(long long)z * K_IN * HID + i];
        grad[OFF_W1 + i] = a;
    } else if (i < K_IN * HID + HID * HID) {
        const int j = i - K_IN * HID;
        float a = 0.f;
        for (int z = 0; z < s2; ++z) a += p2[(long long)z * HID * HID + j];
        grad[OFF_W2 + j] = a;
    }
}

hipError_t launch_reduce_grads(const float *p1, int s1, const float *p2, int s2, float *grad,
                               hipStream_t s)
{
    const int n = K_IN * HID + HID * HID;
    hipLaunchKernelGGL(k_reduce_grads, dim3((n + 255) / 256), dim3(256), 0, s, p1, s1, p2, s2, grad);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_sum(const float *__restrict__ x, int n, float scale,
                                             float *out)
{
    __shared__ float red[256];
    float a = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) a += x[i];
    const float s = block_sum_256(a, red);
    if (threadIdx.x == 0) *out = s * scale;
}

hipError_t launch_sum(const float *x, int n, float scale, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, x, n, scale, out);
    return hipGetLastError();
}

// Adam (0.9, 0.999, 1e-8) on the FP32 master; c1, c2 = bias corrections.
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N_PARAMS) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    w[i] = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

hipError_t launch_adam(float *w, float *m, float *v, const float *g, float lr, float c1, float c2,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3((N_PARAMS + 255) / 256), dim3(256), 0, s, w, m, v, g, lr, c1, c2);
    return hipGetLastError();
}

// Hidden unit of slot s (0..31) of contraction chunk c in the fused kernel:
// the layer-1 (and layer-2) result tiles 2c and 2c+1 hold, in lane group q,
// units 32c + 4q + (0..3) and 32c + 16 + 4q + (0..3).
__device__ __forceinline__ int slot_unit(int c, int s)
{
    const int q = s >> 3, e = s & 7;
    return 32 * c + (e >> 2) * 16 + q * 4 + (e & 3);
}

__device__ __forceinline__ bf16_t to_bf16(float a) { return (bf16_t)(pack2(a, 0.f) & 0xffffu); }

__global__ void k_export(const float *__restrict__ P, bf16_t *__restrict__ w1t,
                         bf16_t *__restrict__ w2t, bf16_t *__restrict__ w2n,
                         float *__restrict__ w3e, bf16_t *__restrict__ w1_inf,
                         bf16_t *__restrict__ w2_inf, bf16_t *__restrict__ w3_inf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= HID * HID) return;
    const float *W1 = P + OFF_W1, *W2 = P + OFF_W2, *W3 = P + OFF_W3;
    {   // W2 copies; i = o * HID + h for the transposed one
        const int o = i / HID, h = i % HID;
        w2t[i] = to_bf16(W2[h * HID + o]);
        w2n[i] = to_bf16(W2[i]);
        // fused layout: row o, 32 chunks of 8 slots, chunk j = 4c + q stored at j ^ (o & 15)
        const int pch = (i % HID) / 8, e = i % 8;
        const int j = pch ^ (o & 15);
        const int hh = slot_unit(j >> 2, (j & 3) * 8 + e);
        w2_inf[i] = to_bf16(W2[hh * HID + o]);
    }
    if (i < HID * K_IN) {
        const int h = i / K_IN, k = i % K_IN;
        w1t[i] = to_bf16(W1[k * HID + h]);
        // fused layout: row h, 4 chunks of 8 inputs, chunk q stored at q ^ ((h >> 2) & 3)
        const int pch = k / 8, e = k % 8;
        const int q = pch ^ ((h >> 2) & 3);
        w1_inf[i] = to_bf16(W1[(8 * q + e) * HID + h]);
    }
    if (i < 8 * 16 * 32) {   // head tiles: chunk c, row (only row 0 non-zero), slot
        const int c = i / 512, row = (i % 512) / 32, sl = i % 32;
        w3_inf[i] = row == 0 ? to_bf16(W3[slot_unit(c, sl)]) : (bf16_t)0;
    }
    if (i < HID) w3e[i] = from_bf16(to_bf16(W3[i]));
}

hipError_t launch_export(const Weights &w, hipStream_t s)
{
    hipLaunchKernelGGL(k_export, dim3(HID * HID / 256), dim3(256), 0, s, w.master, w.w1t, w.w2t,
                       w.w2n, w.w3e, w.w1_inf, w.w2_inf, w.w3_inf);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Features
// ---------------------------------------------------------------------------
// Sum of log v over the 12 months of tenor segment blockIdx.y for 64 scenarios.
__global__ void k_zero_seg(const double *__restrict__ v, int n_steps, int scen_pad, int node_begin,
                           int scen_begin, int scen_count, double *__restrict__ seg)
{
    const int s = blockIdx.x * 64 + threadIdx.x;
    const int T = blockIdx.y, k = blockIdx.z;
    if (s >= scen_count) return;
    const double *vc = v + (long long)(node_begin + k) * n_steps * scen_pad + scen_begin + s;
    double acc = 0.0;
    const int t1 = min(12 * T + 12, n_steps);
    for (int t = 12 * T; t < t1; ++t) acc += log(vc[(long long)t * scen_pad]);
    seg[((long long)k * N_TENORS + T) * scen_count + s] = acc;
}

hipError_t launch_zero_rates(const double *v, int n_steps, int scen_pad, int node_begin,
                             int node_count, int scen_begin, int scen_count, double *seg,
                             hipStream_t s)
{
    if (node_count <= 0 || scen_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_seg, dim3((scen_count + 63) / 64, N_TENORS, node_count), dim3(64), 0,
                       s, v, n_steps, scen_pad, node_begin, scen_begin, scen_count, seg);
    return hipGetLastError();
}

__device__ __forceinline__ bf16_t std_bf16(double x, double mu, double sd)
{
    return to_bf16((float)((x - mu) / sd));
}

__device__ __forceinline__ bool in_box(double x, const Norm &nm, int f)
{
    return x >= nm.lo[f] && x <= nm.hi[f];
}

// One thread per (node, scenario): zero rates from the segment sums, short
// rate, curve factors, shock; raw (optional), standardised features 8..15
// for state 0 and the in-box flag (when a model is given).
__global__ void k_scen_features(const double *__restrict__ v, int n_steps, int scen_pad,
                                const double *__restrict__ shock,
                                const double *__restrict__ seg, int node_begin, int node_count,
                                int scen_begin, int scen_count, Norm nm, double *__restrict__ raw,
                                double *__restrict__ zout, bf16_t *__restrict__ feat,
                                int *__restrict__ ok)
{
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)node_count * scen_count) return;
    const int k = (int)(id / scen_count), s = (int)(id % scen_count);
    double z[N_TENORS];
    double cum = 0.0;
    for (int T = 0; T < N_TENORS; ++T) {
        cum += seg[((long long)k * N_TENORS + T) * scen_count + s];
        const int m = min(12 * (T + 1), n_steps);
        z[T] = -12.0 * cum / (double)m;
    }
    if (zout) {
        for (int T = 0; T < N_TENORS; ++T) zout[id * N_TENORS + T] = z[T];
    }
    double x[5];
    x[0] = -12.0 * log(v[(long long)(node_begin + k) * n_steps * scen_pad + scen_begin + s]);
    for (int j = 0; j < N_FACTORS; ++j) {
        double f = 0.0;
        if (nm.evec) {
            for (int T = 0; T < N_TENORS; ++T) f += nm.evec[j * N_TENORS + T] * (z[T] - nm.zbar[T]);
        }
        x[1 + j] = f;
    }
    x[4] = shock ? shock[node_begin + k] : 1.0;
    if (raw) {
        for (int j = 0; j < 5; ++j) raw[id * 5 + j] = x[j];
    }
    if (!nm.mu) return;
    bool good = true;
    bf16_t out[8];
    for (int j = 0; j < 5; ++j) {
        const int f = 8 + j;
        good = good && in_box(x[j], nm, f);
        out[j] = std_bf16(x[j], nm.mu[f], nm.sd[f]);
    }
    for (int j = 0; j < 3; ++j) {   // state one-hot of state 0
        const int f = 13 + j;
        const double sv = j == 0 ? 1.0 : 0.0;
        good = good && in_box(sv, nm, f);
        out[5 + j] = std_bf16(sv, nm.mu[f], nm.sd[f]);
    }
    u32x4 pk;
    for (int j = 0; j < 4; ++j) pk[j] = (unsigned int)out[2 * j] | ((unsigned int)out[2 * j + 1] << 16);
    *reinterpret_cast<u32x4 *>(feat + id * 8) = pk;
    ok[id] = good ? 1 : 0;
}

hipError_t launch_scen_features(const double *v, int n_steps, int scen_pad, const double *shock,
                                const double *seg, int node_begin, int node_count, int scen_begin,
                                int scen_count, const Norm &nm, double *raw, bf16_t *feat,
                                int *ok, hipStream_t s)
{
    const long long n = (long long)node_count * scen_count;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scen_features, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, v, n_steps,
                       scen_pad, shock, seg, node_begin, node_count, scen_begin, scen_count, nm, raw,
                       (double *)nullptr, feat, ok);
    return hipGetLastError();
}

hipError_t launch_curves_out(const double *v, int n_steps, int scen_pad, const double *seg,
                             int node_begin, int node_count, int scen_begin, int scen_count,
                             double *zout, hipStream_t s)
{
    const long long n = (long long)node_count * scen_count;
    if (n <= 0) return hipSuccess;
    Norm nm{};
    hipLaunchKernelGGL(k_scen_features, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, v, n_steps,
                       scen_pad, (const double *)nullptr, seg, node_begin, node_count, scen_begin,
                       scen_count, nm, (double *)nullptr, zout, (bf16_t *)nullptr, (int *)nullptr);
    return hipGetLastError();
}

// Product codes of the one-hot (single-life annuity, joint-life annuity,
// term assurance, pure endowment).
__constant__ int kSurrogateProducts[4] = {0, 1, 4, 5};

__global__ void k_policy_features(Policies p, int node_begin, int node_count, int node_step, Norm nm,
                                  double *__restrict__ raw, bf16_t *__restrict__ feat,
                                  bf16_t *__restrict__ feat2, int *__restrict__ flag,
                                  double *__restrict__ oscale, double *__restrict__ ooffset)
{
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)node_count * p.n) return;
    const int k = (int)(id / p.n), i = (int)(id % p.n);
    const int shift = (node_begin + k) * node_step;
    const int prod = p.product[i];
    int slot = -1;
    for (int j = 0; j < 4; ++j)
        if (prod == kSurrogateProducts[j]) slot = j;
    double x[9];
    x[0] = (double)(p.age1[i] + shift) / 12.0;
    x[1] = (double)(p.term[i] - shift) / 12.0;
    for (int j = 0; j < 4; ++j) x[2 + j] = slot == j ? 1.0 : 0.0;
    x[6] = log(p.amount[i]);
    x[7] = 12.0 * p.premium[i] / p.amount[i];
    x[8] = slot == 1 ? (double)(p.age2[i] + shift) / 12.0 : 0.0;
    if (raw) {
        for (int j = 0; j < 9; ++j) raw[id * 9 + j] = x[j];
    }
    bool supported = slot >= 0 && !(p.patterned && p.patterned[i]);
    if (supported && nm.signature) {
        const int *sg = nm.signature + 3 * slot;
        supported = sg[0] >= 0 && p.table1[i] == sg[0] && (sg[1] < 0 || p.table2[i] == sg[1]) &&
                    (sg[2] < 0 || p.timing[i] == sg[2]);
    }
    const bool expired = p.term[i] - shift <= 0;
    if (!nm.mu) {
        if (flag) flag[id] = expired ? 2 : (supported ? 1 : 0);
        return;
    }
    bool good = supported;
    bf16_t out[8];
    for (int j = 0; j < 8; ++j) {
        good = good && in_box(x[j], nm, j);
        out[j] = std_bf16(x[j], nm.mu[j], nm.sd[j]);
    }
    good = good && in_box(x[8], nm, 16);
    u32x4 pk;
    for (int j = 0; j < 4; ++j) pk[j] = (unsigned int)out[2 * j] | ((unsigned int)out[2 * j + 1] << 16);
    *reinterpret_cast<u32x4 *>(feat + id * 8) = pk;
    feat2[id] = std_bf16(x[8], nm.mu[16], nm.sd[16]);
    flag[id] = expired ? 2 : (good ? 1 : 0);
    const int j = slot >= 0 ? slot : 0;
    oscale[id] = p.amount[i] * nm.tsd[j];
    ooffset[id] = p.amount[i] * nm.tmu[j];
}

hipError_t launch_policy_features(const Policies &p, int node_begin, int node_count,
                                  int node_step, const Norm &nm, double *raw, bf16_t *feat,
                                  bf16_t *feat2, int *flag, double *scale, double *offset,
                                  hipStream_t s)
{
    const long long n = (long long)node_count * p.n;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_policy_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p,
                       node_begin, node_count, node_step, nm, raw, feat, feat2, flag, scale, offset);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused inference: a wavefront takes a unit (node, chunk of policies, 64
// scenarios) and, per policy, runs the network on the 64 (policy, scenario)
// rows as four 16-row groups.  LDS holds the weights in fragment order:
// layer 2 as 256 rows (output unit) of 32 16-byte chunks, chunk 4c + q
// holding the inputs of slots 8q..8q+7 of contraction chunk c, XOR-swizzled
// by the row; layer 1 as 256 rows of 4 chunks; the head as 8 16x32 tiles
// whose row 0 is W3.
// ---------------------------------------------------------------------------
constexpr int LDS_W2 = 0;
constexpr int LDS_W1 = LDS_W2 + HID * HID * 2;
constexpr int LDS_W3 = LDS_W1 + HID * K_IN * 2;
constexpr int LDS_B1 = LDS_W3 + 8 * 16 * 32 * 2;
constexpr int LDS_B2 = LDS_B1 + HID * 4;
constexpr int LDS_BYTES = LDS_B2 + HID * 4;   // 157,696
constexpr int INFER_THREADS = 512;

__device__ __forceinline__ bf16x8 lds8(const unsigned char *base, int byte_off)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(base + byte_off));
}

__device__ __forceinline__ f32x4 lds_f4(const unsigned char *base, int byte_off)
{
    return *reinterpret_cast<const f32x4 *>(base + byte_off);
}

// Pre-activations of layer-2 output chunk c2 (units 32 c2 .. 32 c2 + 31) for
// NG row groups: bias plus the eight contraction chunks of a1.
template <int NG>
__device__ __forceinline__ void layer2_chunk(const unsigned char *lds, int w2lane, int q, int r16,
                                             int c2, const bf16x8 (&a1)[NG][8], f32x4 (&za)[NG],
                                             f32x4 (&zb)[NG])
{
    const f32x4 ba = lds_f4(lds, LDS_B2 + (32 * c2 + 4 * q) * 4);
    const f32x4 bb = lds_f4(lds, LDS_B2 + (32 * c2 + 16 + 4 * q) * 4);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        za[g] = ba;
        zb[g] = bb;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int sw = ((4 * c + q) ^ r16) * 16;
        const bf16x8 wa = lds8(lds, w2lane + c2 * (32 * 512) + sw);
        const bf16x8 wb = lds8(lds, w2lane + c2 * (32 * 512) + 16 * 512 + sw);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            za[g] = mfma(wa, a1[g][c], za[g]);
            zb[g] = mfma(wb, a1[g][c], zb[g]);
        }
    }
}

// NG groups of 16 rows (scenarios) per unit.
template <int NG>
__global__ void __launch_bounds__(INFER_THREADS, 1) k_infer(Infer f, Weights w)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds[LDS_BYTES];
    {
        const u32x4 *src2 = reinterpret_cast<const u32x4 *>(w.w2_inf);
        const u32x4 *src1 = reinterpret_cast<const u32x4 *>(w.w1_inf);
        const u32x4 *src3 = reinterpret_cast<const u32x4 *>(w.w3_inf);
        const u32x4 *srcb1 = reinterpret_cast<const u32x4 *>(w.master + OFF_B1);
        const u32x4 *srcb2 = reinterpret_cast<const u32x4 *>(w.master + OFF_B2);
        u32x4 *dst = reinterpret_cast<u32x4 *>(lds);
        for (int i = threadIdx.x; i < LDS_BYTES / 16; i += INFER_THREADS) {
            u32x4 x;
            if (i < LDS_W1 / 16) x = src2[i];
            else if (i < LDS_W3 / 16) x = src1[i - LDS_W1 / 16];
            else if (i < LDS_B1 / 16) x = src3[i - LDS_W3 / 16];
            else if (i < LDS_B2 / 16) x = srcb1[i - LDS_B1 / 16];
            else x = srcb2[i - LDS_B2 / 16];
            dst[i] = x;
        }
    }
    __syncthreads();

    constexpr int SB = 16 * NG;   // scenarios per unit
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4, r16 = lane & 15;
    const int waves = gridDim.x * (INFER_THREADS / 64);
    const int n_chunks = (f.n + f.chunk - 1) / f.chunk;
    const int n_sblk = (f.scen_count + SB - 1) / SB;
    const long long units = (long long)f.node_count * n_chunks * n_sblk;
    const float b3 = w.master[OFF_B3];
    // Lane part of the layer-1 fragment address (row 16 hb + r16, swizzle q ^ (r16 >> 2)).
    const int w1lane = LDS_W1 + r16 * 64 + ((q ^ (r16 >> 2)) * 16);
    // Lane part of the layer-2 fragment address (row 32 c2 + r16, or + 16).
    const int w2lane = LDS_W2 + r16 * 512;

    for (long long u = (long long)blockIdx.x * (INFER_THREADS / 64) + (threadIdx.x >> 6); u < units;
         u += waves) {
        const int node = (int)(u / ((long long)n_chunks * n_sblk));
        const int rem = (int)(u % ((long long)n_chunks * n_sblk));
        const int chunk = rem / n_sblk, sblk = rem % n_sblk;
        const int s0 = sblk * SB;
        const long long srow = (long long)node * f.scen_count + s0 + r16;   // + 16 g

        int sok[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) sok[g] = s0 + 16 * g + r16 < f.scen_count ? 1 + f.sok[srow + 16 * g] : 0;
        // sok: 0 = no such scenario, 1 = outside the box, 2 = inside
        double tot[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) tot[g] = 0.0;
        const int p_end = min(f.n, (chunk + 1) * f.chunk);
        for (int p = chunk * f.chunk; p < p_end; ++p) {
            const long long pi = (long long)node * f.n + p;
            const int flag = __builtin_amdgcn_readfirstlane(f.pflag[pi]);
            const long long orow = pi * f.scen_count + s0 + r16;   // + 16 g
            if (flag == 2) {   // expired: reserve 0, not in totals
                if (f.r0 && lane < 16) {
#pragma unroll
                    for (int g = 0; g < NG; ++g)
                        if (sok[g]) f.r0[orow + 16 * g] = 0.0;
                }
                continue;
            }
            if (flag == 0) {   // outside the box: the exact values are already in place
                if (lane < 16) {
#pragma unroll
                    for (int g = 0; g < NG; ++g)
                        if (sok[g]) tot[g] += f.exact[orow + 16 * g];
                }
                continue;
            }
            // Inputs: lane group 0 policy features 0-7, group 1 scenario
            // features 8-15, group 2 feature 16, group 3 zero padding.
            bf16x8 xf[NG];
            {
                const u32x4 pf = *reinterpret_cast<const u32x4 *>(f.pfeat + pi * 8);
                const unsigned int p2 = (unsigned int)f.pfeat2[pi];
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    u32x4 x = {0u, 0u, 0u, 0u};
                    if (q == 1 && sok[g]) x = *reinterpret_cast<const u32x4 *>(f.sfeat + (srow + 16 * g) * 8);
                    if (q == 0) x = pf;
                    if (q == 2) x = u32x4{p2, 0u, 0u, 0u};
                    xf[g] = __builtin_bit_cast(bf16x8, x);
                }
            }
            // Layer 1 + GELU: a1[g][c] is the B operand of layer 2 for chunk c.
            bf16x8 a1[NG][8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const bf16x8 wa = lds8(lds, w1lane + (2 * c) * 1024);
                const bf16x8 wb = lds8(lds, w1lane + (2 * c + 1) * 1024);
                const f32x4 ba = lds_f4(lds, LDS_B1 + (32 * c + 4 * q) * 4);
                const f32x4 bb = lds_f4(lds, LDS_B1 + (32 * c + 16 + 4 * q) * 4);
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const f32x4 za = mfma(wa, xf[g], ba);
                    const f32x4 zb = mfma(wb, xf[g], bb);
                    a1[g][c] = pack8(gelu4(za), gelu4(zb));
                }
            }
            // Layer 2 + GELU + head, two output tiles (one head chunk) at a
            // time, as a two-stage pipeline: while the MFMAs of chunk c2 run,
            // the VALU evaluates the GELU of chunk c2 - 1, NG values per
            // contraction step (scheduling fences keep them interleaved), so
            // the matrix and vector units of the SIMD work at once.  Every
            // accumulator sees the same operations in the same order as in a
            // plain loop.
            f32x4 yacc[NG];
#pragma unroll
            for (int g = 0; g < NG; ++g) yacc[g] = f32x4{0.f, 0.f, 0.f, 0.f};
            f32x4 za[NG], zb[NG];
            layer2_chunk<NG>(lds, w2lane, q, r16, 0, a1, za, zb);
#pragma unroll 1
            for (int c2 = 1; c2 < 8; ++c2) {
                float h[NG][8];   // GELU of chunk c2 - 1: [g][0..3] from za, [g][4..7] from zb
#pragma unroll
                for (int g = 0; g < NG; ++g) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        h[g][i] = za[g][i];
                        h[g][4 + i] = zb[g][i];
                    }
                }
                const f32x4 ba = lds_f4(lds, LDS_B2 + (32 * c2 + 4 * q) * 4);
                const f32x4 bb = lds_f4(lds, LDS_B2 + (32 * c2 + 16 + 4 * q) * 4);
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    za[g] = ba;
                    zb[g] = bb;
                }
                constexpr int PER = NG * 8 / 8;   // GELU values per contraction step
                // Weight fragments one contraction step ahead of their MFMAs.
                const int wrow = w2lane + c2 * (32 * 512);
                bf16x8 wa = lds8(lds, wrow + ((q ^ r16) * 16));
                bf16x8 wb = lds8(lds, wrow + 16 * 512 + ((q ^ r16) * 16));
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    bf16x8 na = wa, nb = wb;
                    if (c < 7) {
                        const int sw = ((4 * (c + 1) + q) ^ r16) * 16;
                        na = lds8(lds, wrow + sw);
                        nb = lds8(lds, wrow + 16 * 512 + sw);
                    }
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        za[g] = mfma(wa, a1[g][c], za[g]);
                        zb[g] = mfma(wb, a1[g][c], zb[g]);
                    }
                    wa = na;
                    wb = nb;
#pragma unroll
                    for (int j = 0; j < PER; ++j) {
                        const int e = c * PER + j;
                        h[e / 8][e % 8] = gelu_f(h[e / 8][e % 8]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                const bf16x8 w3 = lds8(lds, LDS_W3 + (c2 - 1) * 1024 + r16 * 64 + q * 16);
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const f32x4 lo = {h[g][0], h[g][1], h[g][2], h[g][3]};
                    const f32x4 hi = {h[g][4], h[g][5], h[g][6], h[g][7]};
                    yacc[g] = mfma(w3, pack8(lo, hi), yacc[g]);
                }
            }
            {
                const bf16x8 w3 = lds8(lds, LDS_W3 + 7 * 1024 + r16 * 64 + q * 16);
#pragma unroll
                for (int g = 0; g < NG; ++g) yacc[g] = mfma(w3, pack8(gelu4(za[g]), gelu4(zb[g])), yacc[g]);
            }
            if (lane < 16) {
                const double sc = f.scale[pi], of = f.offset[pi];
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const long long o = orow + 16 * g;
                    if (sok[g] == 2) {
                        const double y = (double)(yacc[g][0] + b3);
                        const double r = y * sc + of;
                        if (f.r0) f.r0[o] = r;
                        tot[g] += r;
                    } else if (sok[g] == 1) {
                        tot[g] += f.exact[o];
                    }
                }
            }
        }
        if (lane < 16) {
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                if (sok[g])
                    f.partial[((long long)node * n_chunks + chunk) * f.scen_count + s0 + 16 * g + r16] = tot[g];
            }
        }
    }
}

constexpr int INFER_NG = 2;

int infer_rows_per_unit() { return 16 * INFER_NG; }

hipError_t launch_infer(const Infer &f, const Weights &w, hipStream_t s)
{
    if (f.node_count <= 0 || f.scen_count <= 0 || f.n <= 0) return hipSuccess;
    if (f.chunk <= 0) return hipErrorInvalidValue;
    int dev = 0, n_cu = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    const long long units = (long long)f.node_count * ((f.n + f.chunk - 1) / f.chunk) *
                            ((f.scen_count + 16 * INFER_NG - 1) / (16 * INFER_NG));
    const long long per_wg = INFER_THREADS / 64;
    const int grid = (int)std::min<long long>(n_cu, (units + per_wg - 1) / per_wg);
    hipLaunchKernelGGL(k_infer<INFER_NG>, dim3(grid), dim3(INFER_THREADS), 0, s, f, w);
    return hipGetLastError();
}

// Totals over the policy chunks of the fused kernel, in a fixed order: the
// chunks are split into CT_GROUPS contiguous groups (one workgroup column
// each, four interleaved lanes per scenario), then the groups are summed.
constexpr int CT_GROUPS = 16;

__global__ void __launch_bounds__(256) k_chunk_partial(const double *__restrict__ partial,
                                                       int n_chunks, int scen_count,
                                                       double *__restrict__ work)
{
    __shared__ double red[4][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int s = blockIdx.x * 64 + tx, g = blockIdx.y, k = blockIdx.z;
    const int per = (n_chunks + CT_GROUPS - 1) / CT_GROUPS;
    const int c0 = g * per, c1 = min(n_chunks, c0 + per);
    double a = 0.0;
    if (s < scen_count) {
        for (int c = c0 + ty; c < c1; c += 4) a += partial[((long long)k * n_chunks + c) * scen_count + s];
    }
    red[ty][tx] = a;
    __syncthreads();
    if (ty == 0 && s < scen_count)
        work[((long long)k * CT_GROUPS + g) * scen_count + s] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

__global__ void k_chunk_final(const double *__restrict__ work, int node_count, int scen_count,
                              double *__restrict__ totals)
{
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long long)node_count * scen_count) return;
    const int k = (int)(id / scen_count), s = (int)(id % scen_count);
    double a = 0.0;
    for (int g = 0; g < CT_GROUPS; ++g) a += work[((long long)k * CT_GROUPS + g) * scen_count + s];
    totals[id] = a;
}

long long chunk_totals_work(int node_count, int scen_count)
{
    return (long long)node_count * CT_GROUPS * scen_count;
}

hipError_t launch_chunk_totals(const double *partial, int node_count, int n_chunks, int scen_count,
                               double *work, double *totals, hipStream_t s)
{
    const long long n = (long long)node_count * scen_count;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_partial, dim3((scen_count + 63) / 64, CT_GROUPS, node_count), dim3(256),
                       0, s, partial, n_chunks, scen_count, work);
    hipLaunchKernelGGL(k_chunk_final, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, work,
                       node_count, scen_count, totals);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Training data
// ---------------------------------------------------------------------------
__global__ void k_samples(const double *__restrict__ praw, const double *__restrict__ sraw,
                          const double *__restrict__ r_all, const double *__restrict__ amount,
                          const int2 *__restrict__ pairs, const long long *__restrict__ pair_off,
                          const long long *__restrict__ row_off, int node_count, int n,
                          int scen_count, long long n_rows, double *__restrict__ X,
                          double *__restrict__ T)
{
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    int k = 0;
    while (k + 1 < node_count && row_off[k + 1] <= r) ++k;
    const long long np = pair_off[k + 1] - pair_off[k];
    const long long local = r - row_off[k];
    const int s = (int)(local / np);
    const int2 pr = pairs[pair_off[k] + local % np];
    const int i = pr.x, st = pr.y;
    const double *pv = praw + ((long long)k * n + i) * 9;
    const double *sv = sraw + ((long long)k * scen_count + s) * 5;
    double *x = X + r * N_FEAT;
    for (int j = 0; j < 8; ++j) x[j] = pv[j];
    for (int j = 0; j < 5; ++j) x[8 + j] = sv[j];
    for (int j = 0; j < 3; ++j) x[13 + j] = st == j ? 1.0 : 0.0;
    x[16] = pv[8];
    T[r] = r_all[(((long long)k * n + i) * scen_count + s) * 4 + st] / amount[i];
}

hipError_t launch_samples(const double *praw, const double *sraw, const double *r_all,
                          const double *amount, const int2 *pairs, const long long *pair_off,
                          const long long *row_off, int node_count, int n, int scen_count,
                          long long n_rows, double *X, double *T, hipStream_t s)
{
    if (n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_samples, dim3((unsigned)((n_rows + 255) / 256)), dim3(256), 0, s, praw,
                       sraw, r_all, amount, pairs, pair_off, row_off, node_count, n, scen_count,
                       n_rows, X, T);
    return hipGetLastError();
}

// Value and weight of row r in statistics column c.
__device__ __forceinline__ void col_value(const double *X, const double *T, long long r, int c,
                                          double &x, double &w)
{
    if (c < N_FEAT) {
        x = X[r * N_FEAT + c];
        w = 1.0;
    } else {
        x = T[r];
        w = c == N_FEAT ? 1.0 : X[r * N_FEAT + 2 + (c - N_FEAT - 1)];
    }
}

// mode 0: per block, weighted sum, weight, min and max of each column;
// mode 1: weighted sum of squared deviations from the column mean.
// work[block][STAT_COLS][4].
__global__ void __launch_bounds__(256) k_colstats(const double *__restrict__ X,
                                                  const double *__restrict__ T, long long n,
                                                  int mode, const double *__restrict__ stats,
                                                  double *__restrict__ work)
{
    __shared__ double red[256];
    for (int c = 0; c < STAT_COLS; ++c) {
        double a = 0.0, cnt = 0.0, lo = 1.0e300, hi = -1.0e300;
        const double mu = mode ? stats[4 * c] : 0.0;
        for (long long r = (long long)blockIdx.x * 256 + threadIdx.x; r < n; r += 256LL * STAT_BLOCKS) {
            double x, w;
            col_value(X, T, r, c, x, w);
            if (w == 0.0) continue;
            if (mode) {
                a += (x - mu) * (x - mu);
            } else {
                a += x;
                cnt += 1.0;
                lo = fmin(lo, x);
                hi = fmax(hi, x);
            }
        }
        for (int st = 0; st < (mode ? 1 : 4); ++st) {
            red[threadIdx.x] = st == 0 ? a : (st == 1 ? cnt : (st == 2 ? lo : hi));
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if ((int)threadIdx.x < w) {
                    const double o = red[threadIdx.x + w];
                    const double m = red[threadIdx.x];
                    red[threadIdx.x] = st < 2 ? m + o : (st == 2 ? fmin(m, o) : fmax(m, o));
                }
                __syncthreads();
            }
            if (threadIdx.x == 0) work[((long long)blockIdx.x * STAT_COLS + c) * 4 + st] = red[0];
            __syncthreads();
        }
    }
}

// out[c][0..3] = mean, population sd, min, max (mode 0: mean, min, max;
// mode 1: sd).  Weight sums are kept in out[c][1] between the passes.
__global__ void k_colstats_final(const double *__restrict__ work, int mode, double *__restrict__ out)
{
    const int c = threadIdx.x;
    if (c >= STAT_COLS) return;
    if (mode == 0) {
        double a = 0.0, cnt = 0.0, lo = 1.0e300, hi = -1.0e300;
        for (int b = 0; b < STAT_BLOCKS; ++b) {
            const double *w = work + ((long long)b * STAT_COLS + c) * 4;
            a += w[0];
            cnt += w[1];
            lo = fmin(lo, w[2]);
            hi = fmax(hi, w[3]);
        }
        out[c * 4 + 0] = cnt > 0.0 ? a / cnt : 0.0;
        out[c * 4 + 1] = cnt;
        out[c * 4 + 2] = cnt > 0.0 ? lo : 0.0;
        out[c * 4 + 3] = cnt > 0.0 ? hi : 0.0;
    } else {
        double a = 0.0;
        for (int b = 0; b < STAT_BLOCKS; ++b) a += work[((long long)b * STAT_COLS + c) * 4 + 0];
        const double cnt = out[c * 4 + 1];
        out[c * 4 + 1] = cnt > 0.0 ? sqrt(a / cnt) : 0.0;
    }
}

hipError_t launch_colstats(const double *X, const double *T, long long n, double *work,
                           double *out, hipStream_t s)
{
    if (n <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_colstats, dim3(STAT_BLOCKS), dim3(256), 0, s, X, T, n, 0,
                       (const double *)nullptr, work);
    hipLaunchKernelGGL(k_colstats_final, dim3(1), dim3(64), 0, s, work, 0, out);
    hipLaunchKernelGGL(k_colstats, dim3(STAT_BLOCKS), dim3(256), 0, s, X, T, n, 1, out, work);
    hipLaunchKernelGGL(k_colstats_final, dim3(1), dim3(64), 0, s, work, 1, out);
    return hipGetLastError();
}

__global__ void k_build(const double *__restrict__ X, const double *__restrict__ T, long long n,
                        const int *__restrict__ perm, const double *__restrict__ mu,
                        const double *__restrict__ sd, const double *__restrict__ tmu,
                        const double *__restrict__ tsd, bf16_t *__restrict__ xq,
                        float *__restrict__ tq, unsigned char *__restrict__ prod)
{
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const long long d = perm[r];
    unsigned int pk[16];
    for (int j = 0; j < 16; ++j) {
        const int f0 = 2 * j, f1 = 2 * j + 1;
        const float a = f0 < N_FEAT ? (float)((X[r * N_FEAT + f0] - mu[f0]) / sd[f0]) : 0.f;
        const float b = f1 < N_FEAT ? (float)((X[r * N_FEAT + f1] - mu[f1]) / sd[f1]) : 0.f;
        pk[j] = pack2(a, b);
    }
    u32x4 *dst = reinterpret_cast<u32x4 *>(xq + d * K_IN);
    for (int j = 0; j < 4; ++j) dst[j] = u32x4{pk[4 * j], pk[4 * j + 1], pk[4 * j + 2], pk[4 * j + 3]};
    int j = 0;
    for (int k = 1; k < 4; ++k)
        if (X[r * N_FEAT + 2 + k] > X[r * N_FEAT + 2 + j]) j = k;
    tq[d] = (float)((T[r] - tmu[j]) / tsd[j]);
    prod[d] = (unsigned char)j;
}

hipError_t launch_build(const double *X, const double *T, long long n, const int *perm,
                        const double *mu, const double *sd, const double *tmu, const double *tsd,
                        bf16_t *xq, float *tq, unsigned char *prod, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_build, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, T, n, perm,
                       mu, sd, tmu, tsd, xq, tq, prod);
    return hipGetLastError();
}

// Residual t - y per one-hot product, per block of 1024 rows in a fixed
// order: out[block][0..3] sums, out[block][4..7] counts.
__global__ void __launch_bounds__(256) k_residuals(const float *__restrict__ y,
                                                   const float *__restrict__ t,
                                                   const unsigned char *__restrict__ prod, int n,
                                                   double *__restrict__ out)
{
    __shared__ double red[256];
    const int r0 = blockIdx.x * 1024;
    const int r1 = min(n, r0 + 1024);
    for (int j = 0; j < 4; ++j) {
        double a = 0.0, c = 0.0;
        for (int i = r0 + threadIdx.x; i < r1; i += 256) {
            if (prod[i] == j) {
                a += (double)t[i] - (double)y[i];
                c += 1.0;
            }
        }
        for (int st = 0; st < 2; ++st) {
            red[threadIdx.x] = st ? c : a;
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
                __syncthreads();
            }
            if (threadIdx.x == 0) out[(long long)blockIdx.x * 8 + st * 4 + j] = red[0];
            __syncthreads();
        }
    }
}

int residual_blocks(int n) { return (n + 1023) / 1024; }

hipError_t launch_residuals(const float *y, const float *t, const unsigned char *prod, int n,
                            double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_residuals, dim3(residual_blocks(n)), dim3(256), 0, s, y, t, prod, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Node-level model helpers
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mean_inner(const double *__restrict__ x, long long rows,
                                                    int n_inner, int width,
                                                    double *__restrict__ out, int out_stride)
{
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= rows * width) return;
    const long long r = id / width;
    const int j = (int)(id % width);
    const double *p = x + (size_t)r * n_inner * width + j;
    double acc = 0.0;
    for (int i = 0; i < n_inner; ++i) acc += p[(size_t)i * width];
    out[(size_t)r * out_stride + j] = acc / (double)n_inner;
}

hipError_t launch_mean_inner(const double *x, long long rows, int n_inner, int width, double *out,
                             int out_stride, hipStream_t s)
{
    const long long n = rows * width;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mean_inner, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, rows,
                       n_inner, width, out, out_stride);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_node_scatter(const float *__restrict__ y,
                                                      const int2 *__restrict__ rowmap,
                                                      long long rows, int n,
                                                      const double *__restrict__ scale,
                                                      const double *__restrict__ offset,
                                                      double *__restrict__ out)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= rows) return;
    const int2 ki = rowmap[j];
    const size_t o = (size_t)ki.x * n + ki.y;
    out[o] = (double)y[j] * scale[o] + offset[o];
}

hipError_t launch_node_scatter(const float *y, const int2 *rowmap, long long rows, int n,
                               const double *scale, const double *offset, double *out,
                               hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_node_scatter, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, y,
                       rowmap, rows, n, scale, offset, out);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_select(const double *__restrict__ src,
                                                const unsigned char *__restrict__ mask,
                                                long long count, double *__restrict__ out)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count && mask[j]) out[j] = src[j];
}

hipError_t launch_select(const double *src, const unsigned char *mask, long long count, double *out,
                         hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, src, mask,
                       count, out);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_row_sums(const double *__restrict__ x, int n,
                                                  double *__restrict__ out)
{
    __shared__ double sh[256];
    const double *p = x + (size_t)blockIdx.x * n;
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += p[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

hipError_t launch_row_sums(const double *x, int rows, int n, double *out, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_sums, dim3(rows), dim3(256), 0, s, x, n, out);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace rr
