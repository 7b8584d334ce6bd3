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

// DPP lane permutation of a double (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes with a fixed association, as VALU work only: within
// each row of 16 lanes, pairs, quads, half-rows and rows are added through
// DPP permutations (every lane of a row ends with the same row sum, bit for
// bit, since each addition sees the same two operands); the four row sums are
// then added in lane order.  The result is wavefront-uniform and identical on
// every call with the same inputs.
__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp_f64<0xb1>(x);    // quad_perm [1,0,3,2]
    x += dpp_f64<0x4e>(x);    // quad_perm [2,3,0,1]
    x += dpp_f64<0x141>(x);   // row_half_mirror
    x += dpp_f64<0x140>(x);   // row_mirror
    const int lo0 = __builtin_amdgcn_readlane(__double2loint(x), 0);
    const int hi0 = __builtin_amdgcn_readlane(__double2hiint(x), 0);
    const int lo1 = __builtin_amdgcn_readlane(__double2loint(x), 16);
    const int hi1 = __builtin_amdgcn_readlane(__double2hiint(x), 16);
    const int lo2 = __builtin_amdgcn_readlane(__double2loint(x), 32);
    const int hi2 = __builtin_amdgcn_readlane(__double2hiint(x), 32);
    const int lo3 = __builtin_amdgcn_readlane(__double2loint(x), 48);
    const int hi3 = __builtin_amdgcn_readlane(__double2hiint(x), 48);
    return (__hiloint2double(hi0, lo0) + __hiloint2double(hi1, lo1)) +
           (__hiloint2double(hi2, lo2) + __hiloint2double(hi3, lo3));
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

// The all-lanes-active phase runs in blocks of U steps.  Every load of a block
// (q from LDS, v with scalar loads) is issued one block ahead, right after the
// wait for the current block, so its latency overlaps the current block's
// arithmetic: scalar loads complete out of order, so each wait is a wait for
// all of them, and the issue point has to come after that wait.  U*K <= 16
// curve values per block (double-buffered: 64 scalar registers); K = 32 uses
// single blocks of one step.  With J policies per lane a block carries
// U*K*J*2 <= 128 FMAs, so one scalar load feeds J times more arithmetic and a
// block outlasts a scalar-cache miss.
template <int K, int J = 1>
struct StepBlock {
    static constexpr int U0 = K >= 16 ? 1 : (16 / K > 8 ? 8 : 16 / K);
    static constexpr int U1 = (64 / (K * J)) < 1 ? 1 : 64 / (K * J);
    static constexpr int U2 = (8 / J) < 1 ? 1 : 8 / J;   // <= 8 policy-steps of table values per block
    static constexpr int U01 = U0 < U1 ? U0 : U1;
    static constexpr int U = U01 < U2 ? U01 : U2;
    static constexpr bool PIPE = K <= 16;
};

// Make the arithmetic that follows wait here for the loads of the block in
// flight (the wait is inserted before this point because it reads them).
__device__ __forceinline__ void wait_for(double q, double v)
{
    asm volatile("" ::"v"(q), "s"(v));
}

// Survival probability over one step with the node's mortality shock m
// applied to the death probability (capped at 1).
template <bool LDSQ, bool SHOCK>
__device__ __forceinline__ double p_eff(const double *__restrict__ lq, const double *__restrict__ gq,
                                        int idx, double m)
{
    double p = qload<LDSQ>(lq, gq, idx);
    if constexpr (SHOCK) p = 1.0 - fmin(1.0, m * (1.0 - p));
    return p;
}

// Per-lane state of one policy in a scalar-reserve item.
struct ScalarLane {
    int S;        // remaining term at the node (<= 0: expired or padding)
    int qa, qb;   // LDS indices of the q of life 1 / life 2 at t = 0
    double a0, a1mb1, b1, a1;
    double rS;    // boundary reserve (state 0)
};

// Scalar-reserve models: one life (annuity, term assurance, endowment,
// endowment assurance; Sec. 4.1 with the zero-reserve states removed) and the
// joint-life annuity (Sec. 4.2.1 b: only state 00 carries a reserve, and its
// one-step survival probability is px * py).  Per step and scenario:
//   r <- a0 + v * (p * r + c),  c = p * a1 + q * b1 = b1 + p * (a1 - b1).
// Each lane carries J policies (one per tile of the item) x K scenarios.
template <int K, int J, bool LDSQ, bool TWO, bool SHOCK>
__device__ __forceinline__ void scalar_steps(const double *__restrict__ lq,
                                             const double *__restrict__ gq,
                                             const double *__restrict__ vb, int stride,
                                             const ScalarLane (&L)[J], double m, int smax,
                                             int smin, double (&r)[J][K], double *path)
{
    // x1, x2: one-step survival probabilities from the staged table.
    auto coeffs = [&](const ScalarLane &l, double x1, double x2, double &p, double &c) {
        if constexpr (SHOCK) {
            x1 = 1.0 - fmin(1.0, m * (1.0 - x1));
            if constexpr (TWO) x2 = 1.0 - fmin(1.0, m * (1.0 - x2));
        }
        if constexpr (TWO) {
            p = x1 * x2;
            c = p * l.a1;
        } else {
            p = x1;
            c = fma(p, l.a1mb1, l.b1);
        }
    };
    auto apply = [&](double (&rj)[K], const double (&vk)[K], double p, double c, double a0) {
#pragma unroll
        for (int k = 0; k < K; ++k) rj[k] = fma(vk[k], fma(p, rj[k], c), a0);
    };
    constexpr int U = StepBlock<K, J>::U;
    auto load_block = [&](int tb, const double *vtb, double (&vk)[U][K], double (&q1)[U][J],
                          double (&q2)[U][J]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) vk[u][k] = vtb[k - u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < J; ++j) {
                q1[u][j] = qload<LDSQ>(lq, gq, L[j].qa + tb - u);
                q2[u][j] = TWO ? qload<LDSQ>(lq, gq, L[j].qb + tb - u) : 0.0;
            }
    };
    // One block of U steps, every policy of the block active (t < smin).
    auto run_block = [&](int tb, const double (&vk)[U][K], const double (&q1)[U][J],
                         const double (&q2)[U][J]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                double p, c;
                coeffs(L[j], q1[u][j], q2[u][j], p, c);
                apply(r[j], vk[u], p, c, L[j].a0);
            }
            if constexpr (K == 1 && J == 1) {
                if (path != nullptr) path[tb - u] = r[0][0];
            }
        }
    };
    // Ragged head of the item (t >= smin): a policy that has not started
    // (t >= S) takes the step with p = 0, c = 0, a0 = r_S, which leaves its
    // reserve at the boundary value exactly (v * 0 + r_S = r_S), so the loop
    // needs no branches.  Its table reads land in the staged table's padding.
    int t = smax - 1;
    for (; t >= smin; --t) {
        const double *vt = vb + (ptrdiff_t)t * stride;
        double vk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vk[k] = vt[k];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            double p, c;
            coeffs(L[j], qload<LDSQ>(lq, gq, L[j].qa + t),
                   TWO ? qload<LDSQ>(lq, gq, L[j].qb + t) : 0.0, p, c);
            const bool on = t < L[j].S;
            p = on ? p : 0.0;
            c = on ? c : 0.0;
            apply(r[j], vk, p, c, on ? L[j].a0 : L[j].rS);
        }
        if constexpr (K == 1 && J == 1) {
            if (path != nullptr && t < L[0].S) path[t] = r[0][0];
        }
    }
    if constexpr (StepBlock<K, J>::PIPE) {
        // Pairs of blocks through two named buffers (ping-pong): no register
        // copy of a block in flight and no branch between a prefetch and its
        // use, so the compiler keeps every load at its issue point.  The
        // prefetch after the last pair is clamped in bounds and unused.
        const int npair = ((t + 1) / U) / 2;
        if (npair > 0) {
            double av[U][K], aq1[U][J], aq2[U][J], bv[U][K], bq1[U][J], bq2[U][J];
            load_block(t, vb + (ptrdiff_t)t * stride, av, aq1, aq2);
            for (int i = 0; i < npair; ++i) {
                wait_for(aq1[0][0], av[0][0]);
                __builtin_amdgcn_sched_barrier(0);
                load_block(t - U, vb + (ptrdiff_t)(t - U) * stride, bv, bq1, bq2);
                __builtin_amdgcn_sched_barrier(0);
                run_block(t, av, aq1, aq2);
                wait_for(bq1[0][0], bv[0][0]);
                const int tl = max(t - 2 * U, U - 1);
                __builtin_amdgcn_sched_barrier(0);
                load_block(tl, vb + (ptrdiff_t)tl * stride, av, aq1, aq2);
                __builtin_amdgcn_sched_barrier(0);
                run_block(t - U, bv, bq1, bq2);
                t -= 2 * U;
            }
        }
    }
    for (; t >= U - 1; t -= U) {
        double vk[U][K], q1[U][J], q2[U][J];
        load_block(t, vb + (ptrdiff_t)t * stride, vk, q1, q2);
        run_block(t, vk, q1, q2);
    }
    for (; t >= 0; --t) {   // fewer than U steps left
        const double *vt = vb + (ptrdiff_t)t * stride;
        double vk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vk[k] = vt[k];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            double p, c;
            coeffs(L[j], qload<LDSQ>(lq, gq, L[j].qa + t),
                   TWO ? qload<LDSQ>(lq, gq, L[j].qb + t) : 0.0, p, c);
            apply(r[j], vk, p, c, L[j].a0);
        }
        if constexpr (K == 1 && J == 1) {
            if (path != nullptr) path[t] = r[0][0];
        }
    }
}

// An item of `count` (<= J) consecutive tiles of one scalar model and a block
// of K scenarios: lane l carries slot first + 64 j + l of every tile j.
template <int K, int J, bool LDSQ, bool TWO>
__device__ __forceinline__ void run_scalar(const RecParams &P, const double *__restrict__ lq,
                                           const double *__restrict__ vcurves, int node_rel,
                                           int tile, int count, const Tile &T0, int item_smax,
                                           int item_smin, int sb, int lane)
{
    const int node = P.node_begin + node_rel;
    const int shift = node * P.node_step;
    const int smax = item_smax - shift;
    const int smin = max(item_smin - shift, 0);
    const double m = P.shock[node];
    ScalarLane L[J];
    int uid[J];
    double r[J][K];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int slot = T0.first + j * TILE + lane;   // tiles of an item are consecutive
        if (j < count) {
            L[j].S = P.term[slot] - shift;
            uid[j] = P.uidx[slot];
            L[j].a0 = P.coef[0 * P.n_pad + slot];
            L[j].a1 = P.coef[1 * P.n_pad + slot];
            L[j].b1 = P.coef[2 * P.n_pad + slot];
            L[j].a1mb1 = L[j].a1 - L[j].b1;
            L[j].qa = P.qoff1[slot] + P.age1[slot] + shift;
            L[j].qb = TWO ? P.qoff2[slot] + P.age2[slot] + shift : 0;
            L[j].rS = P.coef[3 * P.n_pad + slot];
#pragma unroll
            for (int k = 0; k < K; ++k) r[j][k] = L[j].rS;
        } else {   // missing tile of a short item: an always-inactive lane
            L[j].S = -1;
            uid[j] = -1;
            L[j].a0 = L[j].a1 = L[j].b1 = L[j].a1mb1 = L[j].rS = 0.0;
            L[j].qa = shift;
            L[j].qb = shift;
#pragma unroll
            for (int k = 0; k < K; ++k) r[j][k] = 0.0;
        }
    }
    const double *vb = vcurves + (size_t)node * P.n_steps * P.scen_pad + (P.scen_begin + sb);
    double *path = nullptr;
    if constexpr (K == 1 && J == 1) {
        if (P.path != nullptr && uid[0] >= 0 && L[0].S > 0) {
            path = P.path + P.path_off[uid[0]];
            path[L[0].S] = r[0][0];
        }
    }
    if (m == 1.0)
        scalar_steps<K, J, LDSQ, TWO, false>(lq, P.q, vb, P.scen_pad, L, m, smax, smin, r, path);
    else
        scalar_steps<K, J, LDSQ, TWO, true>(lq, P.q, vb, P.scen_pad, L, m, smax, smin, r, path);
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (j < count) {
            const bool live = uid[j] >= 0 && L[j].S > 0;
            store_results<K>(P, node_rel, tile + j, sb, lane, uid[j], live, r[j], r[j], r[j], false,
                             false);
        }
    }
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
    auto apply = [&](const double (&vk)[K], double px, double py, int t) {
        const double qx = 1.0 - px, qy = 1.0 - py;
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
            apply(vk, p_eff<LDSQ, SHOCK>(lq, gq, qa + t, m), p_eff<LDSQ, SHOCK>(lq, gq, qb + t, m), t);
    }
    constexpr int U = StepBlock<K>::U;
    auto load_block = [&](int tb, const double *vtb, double (&vk)[U][K], double (&qx)[U],
                          double (&qy)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) vk[u][k] = vtb[k - u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            qx[u] = qload<LDSQ>(lq, gq, qa + tb - u);
            qy[u] = qload<LDSQ>(lq, gq, qb + tb - u);
        }
    };
    auto run_block = [&](int tb, const double (&vk)[U][K], const double (&qx)[U],
                         const double (&qy)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double x = qx[u], y = qy[u];
            if constexpr (SHOCK) {
                x = 1.0 - fmin(1.0, m * (1.0 - x));
                y = 1.0 - fmin(1.0, m * (1.0 - y));
            }
            apply(vk[u], x, y, tb - u);
        }
    };
    if constexpr (StepBlock<K>::PIPE) {
        {
            const int npair = ((t + 1) / U) / 2;
            if (npair > 0) {
                double av[U][K], aqx[U], aqy[U], bv[U][K], bqx[U], bqy[U];
                load_block(t, vt, av, aqx, aqy);
                for (int i = 0; i < npair; ++i) {
                    wait_for(aqx[0], av[0][0]);
                    __builtin_amdgcn_sched_barrier(0);
                    load_block(t - U, vb + (ptrdiff_t)(t - U) * stride, bv, bqx, bqy);
                    __builtin_amdgcn_sched_barrier(0);
                    run_block(t, av, aqx, aqy);
                    wait_for(bqx[0], bv[0][0]);
                    const int tl = max(t - 2 * U, U - 1);
                    __builtin_amdgcn_sched_barrier(0);
                    load_block(tl, vb + (ptrdiff_t)tl * stride, av, aqx, aqy);
                    __builtin_amdgcn_sched_barrier(0);
                    run_block(t - U, bv, bqx, bqy);
                    t -= 2 * U;
                }
            }
            vt = vb + (ptrdiff_t)t * stride;
        }
    }
    {
        for (; t >= U - 1; t -= U, vt -= U * stride) {
            double vk[U][K], qx[U], qy[U];
            load_block(t, vt, vk, qx, qy);
            run_block(t, vk, qx, qy);
        }
    }
    for (; t >= 0; --t, vt -= stride) {
        double vk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vk[k] = vt[k];
        apply(vk, p_eff<LDSQ, SHOCK>(lq, gq, qa + t, m), p_eff<LDSQ, SHOCK>(lq, gq, qb + t, m), t);
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
template <int K, int J, bool LDSQ, bool VEC>
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
        idx = wave_uniform(idx);   // every lane is active here: lane 0's value
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
        const int count = wave_uniform(it.count);
        Tile T = tiles[tile];
        T.kind = wave_uniform(T.kind);
        T.first = wave_uniform(T.first);
        T.smax = wave_uniform(T.smax);
        T.smin = wave_uniform(T.smin);
        // Terms are bucketed, not strictly sorted: take the extremes over the
        // item's tiles.
        int smax = T.smax, smin = T.smin;
        for (int j = 1; j < count; ++j) {
            smax = max(smax, wave_uniform(tiles[tile + j].smax));
            smin = min(smin, wave_uniform(tiles[tile + j].smin));
        }
        if (T.kind == KIND_SINGLE) {
            run_scalar<K, J, LDSQ, false>(P, s_q, vcurves, node_rel, tile, count, T, smax, smin, sb,
                                          lane);
        } else if (T.kind == KIND_JOINT) {
            run_scalar<K, J, LDSQ, true>(P, s_q, vcurves, node_rel, tile, count, T, smax, smin, sb,
                                         lane);
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

bool supported_kj(int K, int J)
{
    if (J == 1) return supported_k(K);
    if (J == 2) return K == 4 || K == 8 || K == 16;
    if (J == 4) return K == 2 || K == 4 || K == 8 || K == 16;
    return false;
}

int max_lds_tables_doubles() { return 8192; }   // 64 KiB of tables per workgroup

template <int K, int J>
static hipError_t launch_kj(const RecParams &p, int grid, size_t lds, hipStream_t s)
{
    const dim3 g(grid), b(WG_THREADS);
    if (p.q_in_lds) {
        if (p.has_vector)
            hipLaunchKernelGGL((k_recurrence<K, J, true, true>), g, b, lds, s, p, p.v, p.items, p.tiles, p.qbeg);
        else
            hipLaunchKernelGGL((k_recurrence<K, J, true, false>), g, b, lds, s, p, p.v, p.items, p.tiles, p.qbeg);
    } else {
        if (p.has_vector)
            hipLaunchKernelGGL((k_recurrence<K, J, false, true>), g, b, 0, s, p, p.v, p.items, p.tiles, p.qbeg);
        else
            hipLaunchKernelGGL((k_recurrence<K, J, false, false>), g, b, 0, s, p, p.v, p.items, p.tiles, p.qbeg);
    }
    return hipGetLastError();
}

hipError_t launch_recurrence(int K, int J, const RecParams &p, int grid, size_t lds_bytes,
                             hipStream_t stream)
{
    switch (J * 64 + K) {
    case 64 + 1: return launch_kj<1, 1>(p, grid, lds_bytes, stream);
    case 64 + 2: return launch_kj<2, 1>(p, grid, lds_bytes, stream);
    case 64 + 4: return launch_kj<4, 1>(p, grid, lds_bytes, stream);
    case 64 + 8: return launch_kj<8, 1>(p, grid, lds_bytes, stream);
    case 64 + 16: return launch_kj<16, 1>(p, grid, lds_bytes, stream);
    case 64 + 32: return launch_kj<32, 1>(p, grid, lds_bytes, stream);
    case 128 + 4: return launch_kj<4, 2>(p, grid, lds_bytes, stream);
    case 128 + 8: return launch_kj<8, 2>(p, grid, lds_bytes, stream);
    case 128 + 16: return launch_kj<16, 2>(p, grid, lds_bytes, stream);
    case 256 + 2: return launch_kj<2, 4>(p, grid, lds_bytes, stream);
    case 256 + 4: return launch_kj<4, 4>(p, grid, lds_bytes, stream);
    case 256 + 8: return launch_kj<8, 4>(p, grid, lds_bytes, stream);
    case 256 + 16: return launch_kj<16, 4>(p, grid, lds_bytes, stream);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Portfolio totals: sum of the per-tile partials of each (node, scenario) in
// a fixed order (no atomics), so totals are bitwise reproducible.
// ---------------------------------------------------------------------------
constexpr int TOT_SCEN = 64;     // scenarios per workgroup (one wavefront wide)
constexpr int TOT_GROUPS = 16;   // tile groups summed in parallel, then in order

__global__ void __launch_bounds__(TOT_SCEN * TOT_GROUPS)
k_totals_wide(const double *__restrict__ partial, int n_tiles, int scen_count,
              double *__restrict__ totals)
{
    __shared__ double sh[TOT_GROUPS][TOT_SCEN];
    const int sx = threadIdx.x, g = threadIdx.y;
    const int s = blockIdx.x * TOT_SCEN + sx;
    const int node = blockIdx.y;
    double acc = 0.0;
    if (s < scen_count) {
        const double *p = partial + (size_t)node * n_tiles * scen_count + s;
        for (int t = g; t < n_tiles; t += TOT_GROUPS) acc += p[(size_t)t * scen_count];
    }
    sh[g][sx] = acc;
    __syncthreads();
    if (g == 0 && s < scen_count) {
        double tot = 0.0;
#pragma unroll
        for (int j = 0; j < TOT_GROUPS; ++j) tot += sh[j][sx];
        totals[(size_t)node * scen_count + s] = tot;
    }
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
    if (scen_count >= 32) {
        dim3 grid((scen_count + TOT_SCEN - 1) / TOT_SCEN, node_count);
        hipLaunchKernelGGL(k_totals_wide, grid, dim3(TOT_SCEN, TOT_GROUPS), 0, stream, partial,
                           n_tiles, scen_count, totals);
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

}  // namespace rr
