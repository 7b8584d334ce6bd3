// Device kernels of the reserve recurrence (gfx950, FP64 vector ALU).
//
// One lane per policy, K scenarios per lane: lane i of a wavefront walks its
// policy's steps backward (Sec. 3.8.2) carrying K reserve chains in
// registers.  The per-policy work of a step (gather of the monthly q from the
// LDS copy of the mortality table, W entries, W c) is shared by the K
// chains; the scenario's one-step discount factor v_t is wavefront-uniform
// and read with scalar loads from the month-major curve array.  Work items
// (node, tile of 64 policies, block of K scenarios) are taken from per-XCD
// queues, longest first, by a persistent grid.
#include "rr_internal.h"

namespace rr {

__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Sum over the 64 lanes (butterfly: every lane ends with the same value, and
// the order of additions is fixed, so the result is deterministic).
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <bool LDSQ>
__device__ __forceinline__ double qload(const double *__restrict__ lds, const double *__restrict__ glob,
                                        int idx)
{
    if constexpr (LDSQ) return lds[idx];
    else return glob[idx];
}

// Store the item's results: per-lane r0 slots and per-scenario wave totals.
template <int K>
__device__ __forceinline__ void store_results(const RecParams &P, int node_rel, int tile, int sb,
                                              int lane, int uid, bool live, const double (&r0)[K],
                                              const double (&r1)[K], const double (&r2)[K],
                                              bool has1, bool has2)
{
    if (P.r0 != nullptr && uid >= 0) {
        double *o = P.r0 + (((size_t)node_rel * P.n_user + uid) * P.scen_count + sb) * P.r0_states;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (sb + k < P.scen_count) {
                if (P.r0_states == 1) {
                    o[k] = live ? r0[k] : 0.0;
                } else {
                    o[4 * k + 0] = live ? r0[k] : 0.0;
                    o[4 * k + 1] = (live && has1) ? r1[k] : 0.0;
                    o[4 * k + 2] = (live && has2) ? r2[k] : 0.0;
                    o[4 * k + 3] = 0.0;
                }
            }
        }
    }
    if (P.partial != nullptr) {
        double *pt = P.partial + ((size_t)node_rel * P.n_tiles + tile) * P.scen_count + sb;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double s = wave_sum(live ? r0[k] : 0.0);
            if (lane == 0 && sb + k < P.scen_count) pt[k] = s;
        }
    }
}

// Steps per block of the all-lanes-active phase: every load of a block (q
// from LDS, v with scalar loads) is issued before its arithmetic, so memory
// latency is paid once per block.  U*K <= 32 keeps the curve values of a
// block within the scalar register file.
template <int K>
struct StepBlock {
    static constexpr int U = K >= 32 ? 1 : (K >= 16 ? 2 : 4);
};

template <bool LDSQ, bool SHOCK>
__device__ __forceinline__ double q_eff(const double *__restrict__ lq, const double *__restrict__ gq,
                                        int idx, double m)
{
    double q = qload<LDSQ>(lq, gq, idx);
    if constexpr (SHOCK) q = fmin(1.0, m * q);
    return q;
}

// Scalar-reserve models: one life (annuity, term assurance, endowment,
// endowment assurance; Sec. 4.1 with the zero-reserve states removed) and the
// joint-life annuity (Sec. 4.2.1 b: only state 00 carries a reserve, and its
// one-step survival probability is px * py).  Per step and scenario:
//   r <- a0 + v * (p * r + c),  c = p * a1 + q * b1 = b1 + p * (a1 - b1).
template <int K, bool LDSQ, bool TWO, bool SHOCK>
__device__ __forceinline__ void scalar_steps(const double *__restrict__ lq,
                                             const double *__restrict__ gq,
                                             const double *__restrict__ vb, int stride, int qa,
                                             int qb, double m, double a0, double a1, double b1,
                                             int S, int smax, int smin, double (&r)[K],
                                             double *path)
{
    const double a1mb1 = a1 - b1;
    auto coeffs = [&](double q1, double q2, double &p, double &c) {
        if constexpr (TWO) {
            p = (1.0 - q1) * (1.0 - q2);
            c = p * a1;
        } else {
            p = 1.0 - q1;
            c = fma(p, a1mb1, b1);
        }
    };
    auto apply = [&](const double (&vk)[K], double p, double c, int t) {
#pragma unroll
        for (int k = 0; k < K; ++k) r[k] = fma(vk[k], fma(p, r[k], c), a0);
        if constexpr (K == 1) {
            if (path != nullptr) path[t] = r[0];
        }
    };
    int t = smax - 1;
    const double *vt = vb + (ptrdiff_t)t * stride;
    for (; t >= smin; --t, vt -= stride) {   // ragged head: lanes join when t < S
        double vk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vk[k] = vt[k];
        if (t < S) {
            double p, c;
            coeffs(q_eff<LDSQ, SHOCK>(lq, gq, qa + t, m),
                   TWO ? q_eff<LDSQ, SHOCK>(lq, gq, qb + t, m) : 0.0, p, c);
            apply(vk, p, c, t);
        }
    }
    constexpr int U = StepBlock<K>::U;
    for (; t >= U - 1; t -= U, vt -= U * stride) {   // every valid lane active
        double vk[U][K], q1[U], q2[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) vk[u][k] = vt[k - u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            q1[u] = q_eff<LDSQ, SHOCK>(lq, gq, qa + t - u, m);
            q2[u] = TWO ? q_eff<LDSQ, SHOCK>(lq, gq, qb + t - u, m) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double p, c;
            coeffs(q1[u], q2[u], p, c);
            apply(vk[u], p, c, t - u);
        }
    }
    for (; t >= 0; --t, vt -= stride) {
        double vk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vk[k] = vt[k];
        double p, c;
        coeffs(q_eff<LDSQ, SHOCK>(lq, gq, qa + t, m),
               TWO ? q_eff<LDSQ, SHOCK>(lq, gq, qb + t, m) : 0.0, p, c);
        apply(vk, p, c, t);
    }
}

template <int K, bool LDSQ, bool TWO>
__device__ __forceinline__ void run_scalar(const RecParams &P, const double *__restrict__ lq,
                                           const double *__restrict__ vcurves, int node_rel,
                                           int tile, const Tile &T, int sb, int lane)
{
    const int node = P.node_begin + node_rel;
    const int shift = node * P.node_step;
    const int slot = T.first + lane;
    const int S = P.term[slot] - shift;
    const int uid = P.uidx[slot];
    const bool live = (uid >= 0) && (S > 0);
    const int smax = T.smax - shift;
    const int smin = max(T.smin - shift, 0);
    const double m = P.shock[node];
    const double a0 = P.coef[0 * P.n_pad + slot];
    const double a1 = P.coef[1 * P.n_pad + slot];
    const double b1 = P.coef[2 * P.n_pad + slot];
    const double rS = P.coef[3 * P.n_pad + slot];
    const int qa = P.qoff1[slot] + P.age1[slot] + shift;
    const int qb = TWO ? P.qoff2[slot] + P.age2[slot] + shift : 0;
    const double *vb = vcurves + (size_t)node * P.n_steps * P.scen_pad + (P.scen_begin + sb);

    double r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = rS;

    double *path = nullptr;
    if constexpr (K == 1) {
        if (P.path != nullptr && live) {
            path = P.path + P.path_off[uid];
            path[S] = rS;
        }
    }
    if (m == 1.0)
        scalar_steps<K, LDSQ, TWO, false>(lq, P.q, vb, P.scen_pad, qa, qb, m, a0, a1, b1, S, smax,
                                          smin, r, path);
    else
        scalar_steps<K, LDSQ, TWO, true>(lq, P.q, vb, P.scen_pad, qa, qb, m, a0, a1, b1, S, smax,
                                         smin, r, path);
    store_results<K>(P, node_rel, tile, sb, lane, uid, live, r, r, r, false, false);
}

// Two-life annuities with a vector reserve (Sec. 4.2.1 a, c).  States 00, 01,
// 10 of the 4-state model (state 11 is a zero-reserve state); REV keeps 00
// and 10 only (01 is a zero-reserve state for a reversion to life 2).  With
// y = c_arrears + r' (per state) and W row 00 = (px py, px qy, qx py, .),
// row 01 = (., px, ., qx), row 10 = (., ., py, qy):
//   r00 <- c00_adv + v (px py y00 + px qy y01 + qx py y10)
//   r01 <- c01_adv + v px y01
//   r10 <- c10_adv + v py y10
template <int K, bool LDSQ, bool LAST, bool SHOCK>
__device__ __forceinline__ void vector_steps(const double *__restrict__ lq,
                                             const double *__restrict__ gq,
                                             const double *__restrict__ vb, int stride, int qa,
                                             int qb, double m, const double (&cf)[6], int S,
                                             int smax, int smin, double (&r0)[K], double (&r1)[K],
                                             double (&r2)[K], double *path)
{
    const double c00a = cf[0], c00r = cf[1], c01a = cf[2], c01r = cf[3], c10a = cf[4], c10r = cf[5];
    auto apply = [&](const double (&vk)[K], double qx, double qy, int t) {
        const double px = 1.0 - qx, py = 1.0 - qy;
        const double w00 = px * py, w10 = qx * py;
        const double w01 = px * qy;
        double cw0 = fma(w10, c10r, w00 * c00r);
        if constexpr (LAST) cw0 = fma(w01, c01r, cw0);
        const double cw1 = px * c01r;
        const double cw2 = py * c10r;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double a = fma(w00, r0[k], cw0);
            a = fma(w10, r2[k], a);
            if constexpr (LAST) a = fma(w01, r1[k], a);
            const double c = fma(py, r2[k], cw2);
            if constexpr (LAST) {
                const double b = fma(px, r1[k], cw1);
                r1[k] = fma(vk[k], b, c01a);
            }
            r0[k] = fma(vk[k], a, c00a);
            r2[k] = fma(vk[k], c, c10a);
        }
        if constexpr (K == 1) {
            if (path != nullptr) path[t] = r0[0];
        }
    };
    int t = smax - 1;
    const double *vt = vb + (ptrdiff_t)t * stride;
    for (; t >= smin; --t, vt -= stride) {
        double vk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vk[k] = vt[k];
        if (t < S)
            apply(vk, q_eff<LDSQ, SHOCK>(lq, gq, qa + t, m), q_eff<LDSQ, SHOCK>(lq, gq, qb + t, m), t);
    }
    constexpr int U = StepBlock<K>::U;
    for (; t >= U - 1; t -= U, vt -= U * stride) {
        double vk[U][K], qx[U], qy[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) vk[u][k] = vt[k - u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            qx[u] = q_eff<LDSQ, SHOCK>(lq, gq, qa + t - u, m);
            qy[u] = q_eff<LDSQ, SHOCK>(lq, gq, qb + t - u, m);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) apply(vk[u], qx[u], qy[u], t - u);
    }
    for (; t >= 0; --t, vt -= stride) {
        double vk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vk[k] = vt[k];
        apply(vk, q_eff<LDSQ, SHOCK>(lq, gq, qa + t, m), q_eff<LDSQ, SHOCK>(lq, gq, qb + t, m), t);
    }
}

template <int K, bool LDSQ, bool LAST>
__device__ __forceinline__ void run_vector(const RecParams &P, const double *__restrict__ lq,
                                           const double *__restrict__ vcurves, int node_rel,
                                           int tile, const Tile &T, int sb, int lane)
{
    const int node = P.node_begin + node_rel;
    const int shift = node * P.node_step;
    const int slot = T.first + lane;
    const int S = P.term[slot] - shift;
    const int uid = P.uidx[slot];
    const bool live = (uid >= 0) && (S > 0);
    const int smax = T.smax - shift;
    const int smin = max(T.smin - shift, 0);
    const double m = P.shock[node];
    double cf[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) cf[j] = P.coef[j * P.n_pad + slot];
    const int qa = P.qoff1[slot] + P.age1[slot] + shift;
    const int qb = P.qoff2[slot] + P.age2[slot] + shift;
    const double *vb = vcurves + (size_t)node * P.n_steps * P.scen_pad + (P.scen_begin + sb);

    double r0[K], r1[K], r2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { r0[k] = 0.0; r1[k] = 0.0; r2[k] = 0.0; }

    double *path = nullptr;
    if constexpr (K == 1) {
        if (P.path != nullptr && live) {
            path = P.path + P.path_off[uid];
            path[S] = 0.0;
        }
    }
    if (m == 1.0)
        vector_steps<K, LDSQ, LAST, false>(lq, P.q, vb, P.scen_pad, qa, qb, m, cf, S, smax, smin,
                                           r0, r1, r2, path);
    else
        vector_steps<K, LDSQ, LAST, true>(lq, P.q, vb, P.scen_pad, qa, qb, m, cf, S, smax, smin,
                                          r0, r1, r2, path);
    store_results<K>(P, node_rel, tile, sb, lane, uid, live, r0, r1, r2, LAST, true);
}

// Persistent grid: each wavefront takes items from its XCD's queue (the
// hardware places workgroup b on XCD b mod 8), then steals from the others.
// The read-only inputs are separate __restrict__ arguments so that the
// compiler may read the wavefront-uniform curve values with scalar loads.
template <int K, bool LDSQ, bool VEC>
__global__ void __launch_bounds__(WG_THREADS)
k_recurrence(RecParams P, const double *__restrict__ vcurves, const Item *__restrict__ items,
             const Tile *__restrict__ tiles, const int *__restrict__ qbeg)
{
    extern __shared__ double s_q[];
    if constexpr (LDSQ) {
        for (int i = threadIdx.x; i < P.n_q; i += blockDim.x) s_q[i] = P.q[i];
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    int qcur = blockIdx.x % P.n_queues;
    int tried = 0;
    while (tried < P.n_queues) {
        int idx = 0;
        if (lane == 0) idx = atomicAdd(&P.counters[qcur], 1);
        idx = wave_uniform(__shfl(idx, 0, 64));
        const int beg = wave_uniform(qbeg[qcur]);
        const int end = wave_uniform(qbeg[qcur + 1]);
        if (beg + idx >= end) {
            qcur = (qcur + 1 == P.n_queues) ? 0 : qcur + 1;
            ++tried;
            continue;
        }
        const Item it = items[beg + idx];
        const int node_rel = wave_uniform(it.node_rel);
        const int tile = wave_uniform(it.tile);
        const int sb = wave_uniform(it.sblock);
        Tile T = tiles[tile];
        T.kind = wave_uniform(T.kind);
        T.first = wave_uniform(T.first);
        T.smax = wave_uniform(T.smax);
        T.smin = wave_uniform(T.smin);
        if (T.kind == KIND_SINGLE) {
            run_scalar<K, LDSQ, false>(P, s_q, vcurves, node_rel, tile, T, sb, lane);
        } else if (T.kind == KIND_JOINT) {
            run_scalar<K, LDSQ, true>(P, s_q, vcurves, node_rel, tile, T, sb, lane);
        } else if constexpr (VEC) {
            if (T.kind == KIND_REV)
                run_vector<K, LDSQ, false>(P, s_q, vcurves, node_rel, tile, T, sb, lane);
            else
                run_vector<K, LDSQ, true>(P, s_q, vcurves, node_rel, tile, T, sb, lane);
        }
    }
    // The last wavefront to finish re-arms the queues for the next launch.
    if (lane == 0) {
        const int total = (int)(gridDim.x * (blockDim.x / 64));
        if (atomicAdd(&P.counters[MAX_QUEUES], 1) == total - 1) {
            for (int i = 0; i <= MAX_QUEUES; ++i) atomicExch(&P.counters[i], 0);
        }
    }
}

bool supported_k(int K)
{
    return K == 1 || K == 2 || K == 4 || K == 8 || K == 16 || K == 32;
}

int max_lds_tables_doubles() { return 8192; }   // 64 KiB of tables per workgroup

template <int K>
static hipError_t launch_k(const RecParams &p, int grid, size_t lds, hipStream_t s)
{
    const dim3 g(grid), b(WG_THREADS);
    if (p.q_in_lds) {
        if (p.has_vector)
            hipLaunchKernelGGL((k_recurrence<K, true, true>), g, b, lds, s, p, p.v, p.items, p.tiles, p.qbeg);
        else
            hipLaunchKernelGGL((k_recurrence<K, true, false>), g, b, lds, s, p, p.v, p.items, p.tiles, p.qbeg);
    } else {
        if (p.has_vector)
            hipLaunchKernelGGL((k_recurrence<K, false, true>), g, b, 0, s, p, p.v, p.items, p.tiles, p.qbeg);
        else
            hipLaunchKernelGGL((k_recurrence<K, false, false>), g, b, 0, s, p, p.v, p.items, p.tiles, p.qbeg);
    }
    return hipGetLastError();
}

hipError_t launch_recurrence(int K, const RecParams &p, int grid, size_t lds_bytes,
                             hipStream_t stream)
{
    switch (K) {
    case 1: return launch_k<1>(p, grid, lds_bytes, stream);
    case 2: return launch_k<2>(p, grid, lds_bytes, stream);
    case 4: return launch_k<4>(p, grid, lds_bytes, stream);
    case 8: return launch_k<8>(p, grid, lds_bytes, stream);
    case 16: return launch_k<16>(p, grid, lds_bytes, stream);
    case 32: return launch_k<32>(p, grid, lds_bytes, stream);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Portfolio totals: sum of the per-tile partials of each (node, scenario) in
// tile order (fixed order, no atomics).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_totals_wide(const double *__restrict__ partial,
                                                     int n_tiles, int scen_count,
                                                     double *__restrict__ totals)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const int node = blockIdx.y;
    if (s >= scen_count) return;
    const double *p = partial + (size_t)node * n_tiles * scen_count + s;
    double acc = 0.0;
    for (int t = 0; t < n_tiles; ++t) acc += p[(size_t)t * scen_count];
    totals[(size_t)node * scen_count + s] = acc;
}

// Few scenarios, many tiles: one workgroup per (node, scenario); strided
// partial sums then a fixed tree.
__global__ void __launch_bounds__(256) k_totals_narrow(const double *__restrict__ partial,
                                                       int n_tiles, int scen_count,
                                                       double *__restrict__ totals)
{
    __shared__ double sh[256];
    const int s = blockIdx.x;
    const int node = blockIdx.y;
    const double *p = partial + (size_t)node * n_tiles * scen_count + s;
    double acc = 0.0;
    for (int t = threadIdx.x; t < n_tiles; t += 256) acc += p[(size_t)t * scen_count];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[(size_t)node * scen_count + s] = sh[0];
}

hipError_t launch_totals(const double *partial, int node_count, int n_tiles, int scen_count,
                         double *totals, hipStream_t stream)
{
    if (node_count <= 0 || scen_count <= 0) return hipSuccess;
    if (scen_count >= 64) {
        dim3 grid((scen_count + 255) / 256, node_count);
        hipLaunchKernelGGL(k_totals_wide, grid, dim3(256), 0, stream, partial, n_tiles,
                           scen_count, totals);
    } else {
        dim3 grid(scen_count, node_count);
        hipLaunchKernelGGL(k_totals_narrow, grid, dim3(256), 0, stream, partial, n_tiles,
                           scen_count, totals);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-node statistics of the scenario totals: mean (fixed-order tree) and the
// rank-th largest total (the paper's 1-in-200 liability: the 5th largest of
// 1,000 scenarios, Sec. 2.1).  Ties are broken by scenario index, so exactly
// one scenario has each rank.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_stats(const double *__restrict__ totals, int scen_count,
                                               int rank, double *__restrict__ stats)
{
    __shared__ double sh[256];
    const int node = blockIdx.x;
    const double *x = totals + (size_t)node * scen_count;
    double acc = 0.0;
    for (int i = threadIdx.x; i < scen_count; i += 256) acc += x[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) stats[2 * node] = sh[0] / (double)scen_count;
    for (int i = threadIdx.x; i < scen_count; i += 256) {
        const double xi = x[i];
        int above = 0;
        for (int j = 0; j < scen_count; ++j) {
            const double xj = x[j];
            above += (xj > xi) || (xj == xi && j < i);
        }
        if (above == rank - 1) stats[2 * node + 1] = xi;
    }
}

hipError_t launch_stats(const double *totals, int node_count, int scen_count, int rank,
                        double *stats, hipStream_t stream)
{
    if (node_count <= 0 || scen_count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stats, dim3(node_count), dim3(256), 0, stream, totals, scen_count, rank,
                       stats);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small utilities
// ---------------------------------------------------------------------------
__global__ void k_fill(double *dst, long long n, double value)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = value;
}

__global__ void k_fill_int(int *dst, int n, int value)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = value;
}

hipError_t launch_fill(double *dst, long long n, double value, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const long long blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, stream, dst, n, value);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *dst, int n, int value, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, stream, dst, n, value);
    return hipGetLastError();
}

// Curves [node][scen][step] -> [node][step][scen_pad]; padding scenarios get
// v = 1 (they are never written out).
__global__ void __launch_bounds__(256) k_transpose_curves(const double *__restrict__ src,
                                                          double *__restrict__ dst, int n_scen,
                                                          int n_steps, int scen_pad)
{
    __shared__ double tile[32][33];
    const int node = blockIdx.z;
    const int t0 = blockIdx.x * 32, s0 = blockIdx.y * 32;
    const double *sn = src + (size_t)node * n_scen * n_steps;
    double *dn = dst + (size_t)node * n_steps * scen_pad;
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int s = s0 + j, t = t0 + threadIdx.x;
        tile[j][threadIdx.x] = (s < n_scen && t < n_steps) ? sn[(size_t)s * n_steps + t] : 1.0;
    }
    __syncthreads();
    for (int j = threadIdx.y; j < 32; j += 8) {
        const int t = t0 + j, s = s0 + threadIdx.x;
        if (t < n_steps && s < scen_pad) dn[(size_t)t * scen_pad + s] = tile[threadIdx.x][j];
    }
}

hipError_t launch_transpose_curves(const double *src, double *dst, int n_nodes, int n_scen,
                                   int n_steps, int scen_pad, hipStream_t stream)
{
    dim3 grid((n_steps + 31) / 32, (scen_pad + 31) / 32, n_nodes);
    hipLaunchKernelGGL(k_transpose_curves, grid, dim3(32, 8), 0, stream, src, dst, n_scen,
                       n_steps, scen_pad);
    return hipGetLastError();
}

}  // namespace rr
