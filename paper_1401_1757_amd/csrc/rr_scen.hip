// Interest scenarios generated on the device (the interest model of Sec. 3.4
// and 3.7.2, here the Vasicek short rate): a counter-based generator, normals
// by the Box-Muller transform, and the exact joint-Gaussian step of the short
// rate and its integral over a step.
//
// The random numbers of (node k, scenario s, step t) are the Philox4x64-10
// block of the counter (t, s, k, 0) under the caller's key, so every value
// is computed independently: the normals of all steps in parallel, then the
// short-rate chain per scenario (a first-order linear recurrence in t), then
// the discount factors in parallel again.
#include "rr_internal.h"

namespace rr {

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011): per round the words 0
// and 2 are multiplied by the round multipliers; the high halves are xored
// with the other two words and the key, the low halves become words 1 and 3;
// the key is bumped by the Weyl increments between rounds.
__device__ __forceinline__ void philox4x64_10(unsigned long long &c0, unsigned long long &c1,
                                              unsigned long long &c2, unsigned long long &c3,
                                              unsigned long long k0, unsigned long long k1)
{
    constexpr unsigned long long M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    constexpr unsigned long long W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const unsigned long long hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const unsigned long long hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const unsigned long long n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
}

__device__ __forceinline__ double u01(unsigned long long x)
{
    return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// Normals of every (node, step, scenario), stored month-major like the
// curves: z[(k * n_steps + t) * scen_pad + s].
__global__ void __launch_bounds__(256) k_vas_normals(VasParams P, double *__restrict__ z0,
                                                     double *__restrict__ z1)
{
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)P.n_nodes * P.n_steps * P.n_scen;
    if (id >= total) return;
    const int s = (int)(id % P.n_scen);
    const long long kt = id / P.n_scen;
    const int t = (int)(kt % P.n_steps);
    const int k = (int)(kt / P.n_steps);
    unsigned long long c0 = (unsigned long long)t, c1 = (unsigned long long)s,
                       c2 = (unsigned long long)k, c3 = 0;
    philox4x64_10(c0, c1, c2, c3, P.key0, P.key1);
    const double rad = sqrt(-2.0 * log(u01(c0)));
    double sn, cs;
    sincos(6.283185307179586476925286766559 * u01(c1), &sn, &cs);
    const size_t o = (size_t)kt * P.scen_pad + s;
    z0[o] = rad * cs;
    z1[o] = rad * sn;
}

// Short-rate chain of each (node, scenario): r[(k * (n_steps + 1) + t) *
// scen_pad + s] for t = 0..n_steps.  Consecutive threads take consecutive
// scenarios, so every load and store of a step is coalesced.  The chain is
// sequential in t but its normals are not: they are loaded RATES_CHUNK steps
// ahead into registers, so a step waits on arithmetic, not on memory.
constexpr int RATES_CHUNK = 32;
constexpr int RATES_THREADS = 64;

__global__ void __launch_bounds__(RATES_THREADS) k_vas_rates(VasParams P,
                                                             const double *__restrict__ r0,
                                                             const double *__restrict__ z0,
                                                             double *__restrict__ r)
{
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= P.n_nodes * P.n_scen) return;
    const int k = id / P.n_scen, s = id % P.n_scen;
    const double *zk = z0 + (size_t)k * P.n_steps * P.scen_pad + s;
    double *rk = r + (size_t)k * (P.n_steps + 1) * P.scen_pad + s;
    double rt = r0[k];
    rk[0] = rt;
    double zc[RATES_CHUNK];
#pragma unroll
    for (int i = 0; i < RATES_CHUNK; ++i)
        zc[i] = i < P.n_steps ? zk[(size_t)i * P.scen_pad] : 0.0;
    for (int t0 = 0; t0 < P.n_steps; t0 += RATES_CHUNK) {
        double zn[RATES_CHUNK];
#pragma unroll
        for (int i = 0; i < RATES_CHUNK; ++i) {
            const int t = t0 + RATES_CHUNK + i;
            zn[i] = t < P.n_steps ? zk[(size_t)t * P.scen_pad] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < RATES_CHUNK; ++i) {
            const int t = t0 + i;
            if (t < P.n_steps) {
                rt = P.b + (rt - P.b) * P.e + P.sd_r * zc[i];
                rk[(size_t)(t + 1) * P.scen_pad] = rt;
            }
        }
#pragma unroll
        for (int i = 0; i < RATES_CHUNK; ++i) zc[i] = zn[i];
    }
}

// Discount factor of each (node, step, scenario): v = exp(-Y), Y the
// integral of the short rate over the step given r_t and the two normals.
// month_major: v[(k * n_steps + t) * ld + s] (the library's curve layout,
// padding scenarios set to 1), else v[(k * n_scen + s) * n_steps + t].
__global__ void __launch_bounds__(256) k_vas_discount(VasParams P, const double *__restrict__ z0,
                                                      const double *__restrict__ z1,
                                                      const double *__restrict__ r,
                                                      double *__restrict__ v, int month_major)
{
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)P.n_nodes * P.n_steps * P.scen_pad;
    if (id >= total) return;
    const int s = (int)(id % P.scen_pad);
    const long long kt = id / P.scen_pad;
    const int t = (int)(kt % P.n_steps);
    const int k = (int)(kt / P.n_steps);
    if (s >= P.n_scen) {
        if (month_major) v[id] = 1.0;
        return;
    }
    const double rt = r[((size_t)k * (P.n_steps + 1) + t) * P.scen_pad + s];
    const double y = P.b * P.dt + (rt - P.b) * P.om + P.rho_sd_y * z0[id] + P.sd_y_perp * z1[id];
    const double x = exp(-y);
    if (month_major) v[id] = x;
    else v[((size_t)k * P.n_scen + s) * P.n_steps + t] = x;
}

// Short rates in the caller's layout r_out[(k * n_scen + s) * (n_steps + 1) + t].
__global__ void __launch_bounds__(256) k_vas_rates_out(VasParams P, const double *__restrict__ r,
                                                       double *__restrict__ r_out)
{
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)P.n_nodes * (P.n_steps + 1) * P.n_scen;
    if (id >= total) return;
    const int s = (int)(id % P.n_scen);
    const long long kt = id / P.n_scen;
    const int t = (int)(kt % (P.n_steps + 1));
    const int k = (int)(kt / (P.n_steps + 1));
    r_out[((size_t)k * P.n_scen + s) * (P.n_steps + 1) + t] = r[(size_t)kt * P.scen_pad + s];
}

static unsigned blocks_of(long long n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_vasicek(const VasParams &P, const double *r0, double *work, double *v,
                          int month_major, double *r_out, hipStream_t stream)
{
    if (P.n_nodes <= 0 || P.n_scen <= 0 || P.n_steps <= 0) return hipSuccess;
    const size_t zn = (size_t)P.n_nodes * P.n_steps * P.scen_pad;
    double *z0 = work, *z1 = work + zn, *r = work + 2 * zn;
    hipLaunchKernelGGL(k_vas_normals, dim3(blocks_of((long long)P.n_nodes * P.n_steps * P.n_scen)),
                       dim3(256), 0, stream, P, z0, z1);
    hipLaunchKernelGGL(k_vas_rates,
                       dim3((unsigned)(((long long)P.n_nodes * P.n_scen + RATES_THREADS - 1) / RATES_THREADS)),
                       dim3(RATES_THREADS), 0, stream, P, r0, z0, r);
    hipLaunchKernelGGL(k_vas_discount, dim3(blocks_of((long long)zn)), dim3(256), 0, stream, P, z0,
                       z1, r, v, month_major);
    if (r_out)
        hipLaunchKernelGGL(k_vas_rates_out,
                           dim3(blocks_of((long long)P.n_nodes * (P.n_steps + 1) * P.n_scen)),
                           dim3(256), 0, stream, P, r, r_out);
    return hipGetLastError();
}

size_t vasicek_work_doubles(int n_nodes, int n_scen, int n_steps, int scen_pad)
{
    (void)n_scen;
    return (size_t)n_nodes * scen_pad * (3 * (size_t)n_steps + 1);
}

}  // namespace rr
