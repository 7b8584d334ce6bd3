// Launch code of the reserve recurrence and the reduction kernels (portfolio
// totals, per-node statistics, fills, curve transpose).
#include "rr_recurrence.h"

namespace rr {

bool supported_k(int K)
{
    return K == 1 || K == 2 || K == 4 || K == 8 || K == 16 || K == 32;
}

bool supported_kj(int K, int J)
{
    if (J == 1) return supported_k(K);
    if (J == 2) return K == 4 || K == 8 || K == 16;
    if (J == 4) return K == 2 || K == 4 || K == 8 || K == 16;
    return false;
}

int max_lds_tables_doubles() { return 8192; }   // 64 KiB of tables per workgroup

hipError_t launch_recurrence(int K, int J, const RecParams &p, int grid, size_t lds_bytes,
                             hipStream_t stream, bool ring)
{
    if (ring) {
        if (p.has_vector || p.pat_g != nullptr || !supported_ring(K, J)) return hipErrorInvalidValue;
        return launch_recurrence_ring(K, J, p, grid, lds_bytes, stream);
    }
    if (p.pat_g != nullptr && p.pat_code != nullptr)
        return launch_recurrence_pat(K, J, p, grid, lds_bytes, stream);
    return launch_switch<false>(K, J, p, grid, lds_bytes, stream);
}

// ---------------------------------------------------------------------------
// Portfolio totals: sum of the per-tile partials of each (node, scenario) in
// a fixed order (no atomics), so totals are bitwise reproducible.
// ---------------------------------------------------------------------------
constexpr int TOT_SCEN = 64;     // scenarios per workgroup (one wavefront wide)
constexpr int TOT_GROUPS = 16;   // tile groups summed in parallel, then in order
constexpr int TOT_CHUNK = 256;   // tiles per workgroup when the tiles are split

// Number of tile chunks the wide pass splits a node's tiles into (1: one
// pass straight into the totals).  Many tiles and few scenario blocks would
// otherwise leave the chip idle (e.g. 7,813 tiles x 1,000 scenarios: 16
// workgroups).
static int totals_chunks(int n_tiles, int scen_count)
{
    if (scen_count < 32 || n_tiles <= 2 * TOT_CHUNK) return 1;
    return (n_tiles + TOT_CHUNK - 1) / TOT_CHUNK;
}

long long totals_scratch_doubles(int node_count, int n_tiles, int scen_count)
{
    const int nc = totals_chunks(n_tiles, scen_count);
    return nc > 1 ? (long long)node_count * nc * scen_count : 0;
}

// Workgroup (scenario block, node, chunk): the sum over the chunk's tiles,
// TOT_GROUPS strided partial sums then those in order.  Output
// out[node][chunk][scen] (n_chunks = 1: the totals).
__global__ void __launch_bounds__(TOT_SCEN * TOT_GROUPS)
k_totals_wide(const double *__restrict__ partial, int n_tiles, int scen_count, int chunk_tiles,
              int n_chunks, double *__restrict__ out)
{
    __shared__ double sh[TOT_GROUPS][TOT_SCEN];
    const int sx = threadIdx.x, g = threadIdx.y;
    const int s = blockIdx.x * TOT_SCEN + sx;
    const int node = blockIdx.y;
    const int chunk = blockIdx.z;
    const int t0 = chunk * chunk_tiles;
    const int t1 = min(t0 + chunk_tiles, n_tiles);
    double acc = 0.0;
    if (s < scen_count) {
        const double *p = partial + (size_t)node * n_tiles * scen_count + s;
        for (int t = t0 + g; t < t1; t += TOT_GROUPS) acc += p[(size_t)t * scen_count];
    }
    sh[g][sx] = acc;
    __syncthreads();
    if (g == 0 && s < scen_count) {
        double tot = 0.0;
#pragma unroll
        for (int j = 0; j < TOT_GROUPS; ++j) tot += sh[j][sx];
        out[((size_t)node * n_chunks + chunk) * scen_count + s] = tot;
    }
}

// Chunk sums of each (node, scenario) added in chunk order.
__global__ void __launch_bounds__(256) k_totals_merge(const double *__restrict__ chunks, int n_chunks,
                                                      int scen_count, double *__restrict__ totals)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int node = blockIdx.y;
    if (s >= scen_count) return;
    const double *p = chunks + (size_t)node * n_chunks * scen_count + s;
    double tot = 0.0;
    for (int c = 0; c < n_chunks; ++c) tot += p[(size_t)c * scen_count];
    totals[(size_t)node * scen_count + s] = tot;
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
                         double *totals, double *scratch, hipStream_t stream)
{
    if (node_count <= 0 || scen_count <= 0) return hipSuccess;
    if (scen_count >= 32) {
        const int nc = totals_chunks(n_tiles, scen_count);
        if (nc > 1 && scratch == nullptr) return hipErrorInvalidValue;
        dim3 grid((scen_count + TOT_SCEN - 1) / TOT_SCEN, node_count, nc);
        hipLaunchKernelGGL(k_totals_wide, grid, dim3(TOT_SCEN, TOT_GROUPS), 0, stream, partial,
                           n_tiles, scen_count, nc > 1 ? TOT_CHUNK : n_tiles, nc,
                           nc > 1 ? scratch : totals);
        if (nc > 1) {
            dim3 mgrid((scen_count + 255) / 256, node_count);
            hipLaunchKernelGGL(k_totals_merge, mgrid, dim3(256), 0, stream, scratch, nc, scen_count,
                               totals);
        }
    } else {
        dim3 grid(scen_count, node_count);
        hipLaunchKernelGGL(k_totals_narrow, grid, dim3(256), 0, stream, partial, n_tiles,
                           scen_count, totals);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-node statistics of the scenario totals: mean (fixed-order tree over
// the scenarios) and the rank-th largest total (the paper's 1-in-200
// liability: the 5th largest of 1,000 scenarios, Sec. 2.1).
//
// The rank-th largest is found by a most-significant-digit radix select on
// an order-preserving 64-bit key of each total: eight passes of 8-bit digits,
// each a 256-bin LDS histogram of the keys that match the digits chosen so
// far, a suffix scan of the bins and the choice of the bin holding the rank.
// The answer is the unique rank-th largest value, whatever the order of ties.
// ---------------------------------------------------------------------------
__device__ double block_sum_fixed(double x, double *sh)
{
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ inline unsigned long long order_key(double x)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ inline double key_value(unsigned long long k)
{
    const unsigned long long u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)u);
}

__global__ void __launch_bounds__(256) k_stats_select(const double *__restrict__ totals,
                                                      int scen_count, int rank,
                                                      double *__restrict__ stats)
{
    __shared__ double red[256];
    __shared__ unsigned int hist[256];
    __shared__ unsigned int scan[256];
    __shared__ unsigned long long sel_prefix;
    __shared__ unsigned int sel_rank;
    const int node = blockIdx.x;
    const int tid = threadIdx.x;
    const double *x = totals + (size_t)node * scen_count;

    double acc = 0.0;
    for (int i = tid; i < scen_count; i += 256) acc += x[i];
    const double total = block_sum_fixed(acc, red);
    if (tid == 0) {
        stats[2 * node] = total / (double)scen_count;
        sel_prefix = 0ull;
        sel_rank = (unsigned int)rank;
    }

    for (int shift = 56; shift >= 0; shift -= 8) {
        hist[tid] = 0u;
        __syncthreads();
        const unsigned long long prefix = sel_prefix;
        // Keys agree with the prefix on every bit above `shift + 8`.
        const unsigned long long hi_mask = shift == 56 ? 0ull : (~0ull << (shift + 8));
        for (int i = tid; i < scen_count; i += 256) {
            const unsigned long long k = order_key(x[i]);
            if ((k & hi_mask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1u);
        }
        __syncthreads();
        // Suffix sums: scan[b] = number of matching keys with digit >= b.
        scan[tid] = hist[tid];
        __syncthreads();
        for (int w = 1; w < 256; w <<= 1) {
            const unsigned int add = tid + w < 256 ? scan[tid + w] : 0u;
            __syncthreads();
            scan[tid] += add;
            __syncthreads();
        }
        const unsigned int r = sel_rank;
        const unsigned int above = tid < 255 ? scan[tid + 1] : 0u;
        const unsigned int here = scan[tid];
        __syncthreads();
        if (above < r && r <= here) {
            sel_prefix = prefix | ((unsigned long long)tid << shift);
            sel_rank = r - above;
        }
        __syncthreads();
    }
    if (tid == 0) stats[2 * node + 1] = key_value(sel_prefix);
}

// Small ranks (the 1-in-200 statistic): the rank largest totals are taken
// one per round, the largest remaining one each time (ties: the lowest
// scenario index), so the last one taken is the rank-th largest.  Each
// thread keeps its TOP_PER_THREAD totals in registers; a round is a local
// maximum, a wavefront arg-max by XOR butterfly and a pick among the four
// wavefronts.
constexpr int TOP_MAX_RANK = 32;
constexpr int TOP_PER_THREAD = 16;

__device__ __forceinline__ bool top_better(double a, int ia, double b, int ib)
{
    return a > b || (a == b && ia < ib);
}

__global__ void __launch_bounds__(256) k_stats_top(const double *__restrict__ totals,
                                                   int scen_count, int rank,
                                                   double *__restrict__ stats)
{
    __shared__ double red[256];
    __shared__ double wv[4];
    __shared__ int wi[4];
    const int node = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double *x = totals + (size_t)node * scen_count;
    double v[TOP_PER_THREAD];
    unsigned int live = 0u;
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < TOP_PER_THREAD; ++j) {
        const int i = tid + 256 * j;
        v[j] = i < scen_count ? x[i] : 0.0;
        if (i < scen_count) {
            acc += v[j];
            live |= 1u << j;
        }
    }
    const double total = block_sum_fixed(acc, red);
    if (tid == 0) stats[2 * node] = total / (double)scen_count;
    double g = 0.0;
    for (int round = 0; round < rank; ++round) {
        double bv = -__builtin_huge_val();
        int bi = 0x7fffffff;
#pragma unroll
        for (int j = 0; j < TOP_PER_THREAD; ++j) {
            const int i = tid + 256 * j;
            if (((live >> j) & 1u) && top_better(v[j], i, bv, bi)) {
                bv = v[j];
                bi = i;
            }
        }
        // a thread with no live entry holds (-inf, INT_MAX), which every live
        // (finite) total beats
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off);
            const int oi = __shfl_xor(bi, off);
            if (top_better(ov, oi, bv, bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            wv[wave] = bv;
            wi[wave] = bi;
        }
        __syncthreads();
        double gv = wv[0];
        int gi = wi[0];
        for (int w = 1; w < 4; ++w)
            if (top_better(wv[w], wi[w], gv, gi)) {
                gv = wv[w];
                gi = wi[w];
            }
        __syncthreads();
        if ((gi & 255) == tid) live &= ~(1u << (gi >> 8));
        g = gv;
    }
    if (tid == 0) stats[2 * node + 1] = g;
}

hipError_t launch_stats(const double *totals, int node_count, int scen_count, int rank,
                        double *stats, hipStream_t stream)
{
    if (node_count <= 0 || scen_count <= 0) return hipSuccess;
    if (rank < 1 || rank > scen_count) return hipErrorInvalidValue;
    if (rank <= TOP_MAX_RANK && scen_count <= 256 * TOP_PER_THREAD)
        hipLaunchKernelGGL(k_stats_top, dim3(node_count), dim3(256), 0, stream, totals, scen_count,
                           rank, stats);
    else
        hipLaunchKernelGGL(k_stats_select, dim3(node_count), dim3(256), 0, stream, totals,
                           scen_count, rank, stats);
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

// ---------------------------------------------------------------------------
// Mean discount curve of a node's scenarios: the reserve is linear in the
// discount products D_t = v_0 ... v_{t-1} (Eq. (3.5) with mortality independent
// of the interest path), so the scenario-averaged reserve is the reserve on
// the curve whose products are the scenario means of D_t.
// ---------------------------------------------------------------------------
constexpr int DISC_CHUNK = 32;

// D[(kr * n_steps + t) * sc + s] = product of v over steps 0..t of scenario
// scen_begin + s of node node_begin + kr (the one-step factors are loaded a
// chunk ahead: they do not depend on the product).
__global__ void __launch_bounds__(64) k_disc_products(const double *__restrict__ v, int n_steps,
                                                     int scen_pad, int node_begin, int node_count,
                                                     int scen_begin, int sc, double *__restrict__ D)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= node_count * sc) return;
    const int kr = id / sc, s = id % sc;
    const double *vk = v + (size_t)(node_begin + kr) * n_steps * scen_pad + scen_begin + s;
    double *dk = D + (size_t)kr * n_steps * sc + s;
    double prod = 1.0;
    double cur[DISC_CHUNK];
#pragma unroll
    for (int i = 0; i < DISC_CHUNK; ++i) cur[i] = i < n_steps ? vk[(size_t)i * scen_pad] : 1.0;
    for (int t0 = 0; t0 < n_steps; t0 += DISC_CHUNK) {
        double nxt[DISC_CHUNK];
#pragma unroll
        for (int i = 0; i < DISC_CHUNK; ++i) {
            const int t = t0 + DISC_CHUNK + i;
            nxt[i] = t < n_steps ? vk[(size_t)t * scen_pad] : 1.0;
        }
#pragma unroll
        for (int i = 0; i < DISC_CHUNK; ++i) {
            const int t = t0 + i;
            if (t < n_steps) {
                prod *= cur[i];
                dk[(size_t)t * sc] = prod;
            }
        }
#pragma unroll
        for (int i = 0; i < DISC_CHUNK; ++i) cur[i] = nxt[i];
    }
}

// Mean over scenarios (in order) of D, then the one-step factors of the mean
// curve, written at scenario 0 of vbar[node][t][64] (other lanes 1).
__global__ void __launch_bounds__(256) k_mean_curve(const double *__restrict__ D, int n_steps,
                                                    int node_begin, int node_count, int sc,
                                                    double *__restrict__ vbar)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= node_count * n_steps) return;
    const int kr = id / n_steps, t = id % n_steps;
    const double *row = D + ((size_t)kr * n_steps + t) * sc;
    double acc = 0.0;
    for (int s = 0; s < sc; ++s) acc += row[s];
    double prev = 1.0;
    if (t > 0) {
        const double *pr = D + ((size_t)kr * n_steps + t - 1) * sc;
        double a = 0.0;
        for (int s = 0; s < sc; ++s) a += pr[s];
        prev = a / sc;
    }
    double *o = vbar + ((size_t)(node_begin + kr) * n_steps + t) * 64;
    o[0] = (acc / sc) / prev;
    for (int j = 1; j < 64; ++j) o[j] = 1.0;
}

hipError_t launch_mean_curve(const double *v, int n_steps, int scen_pad, int node_begin,
                             int node_count, int scen_begin, int scen_count, double *D,
                             double *vbar, hipStream_t stream)
{
    if (node_count <= 0 || scen_count <= 0 || n_steps <= 0) return hipSuccess;
    const int nt = node_count * scen_count;
    hipLaunchKernelGGL(k_disc_products, dim3((nt + 63) / 64), dim3(64), 0, stream, v, n_steps,
                       scen_pad, node_begin, node_count, scen_begin, scen_count, D);
    const int nm = node_count * n_steps;
    hipLaunchKernelGGL(k_mean_curve, dim3((nm + 255) / 256), dim3(256), 0, stream, D, n_steps,
                       node_begin, node_count, scen_count, vbar);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_pow_curves(const double *__restrict__ src,
                                                    double *__restrict__ dst, long long n, double f)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = pow(src[i], f);
}

hipError_t launch_pow_curves(const double *src, double *dst, long long n, double f,
                             hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pow_curves, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, src,
                       dst, n, f);
    return hipGetLastError();
}

}  // namespace rr
