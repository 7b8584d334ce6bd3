// Device templates of the reserve recurrence kernel, instantiated by
// rr_kernels.hip (level portfolios) and rr_kernels_pat.hip (portfolios
// with annuity payment patterns).
//
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
#pragma once

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

// Path output (one scenario and one policy per lane): the state-0 reserve at
// every step, stored per policy as consecutive doubles.  Written directly, a
// step's store touches 64 cache lines (one per lane).  Instead the wavefront
// keeps the last PATH_T steps of its 64 lanes in LDS and, when a block of
// PATH_T aligned steps is complete, writes it out per policy: lane l takes
// step t0 + l % PATH_T of policy (64 / PATH_T) j + l / PATH_T in round j, so a
// store instruction covers four runs of PATH_T consecutive doubles.  The
// stage's rows are PATH_ROW doubles apart, which spreads a round's reads over
// the LDS banks; each lane's round targets (address and S of the policy it
// writes for) are fetched once per item.
struct PathStage {
    double *base;    // this lane's path (entry t at base[t]); null: the lane writes none
    int S;           // entries t < S come from the steps (entry S is written first)
    double *buf;     // the wavefront's PATH_STAGE_DOUBLES of LDS; null: no path output
    unsigned long long rdst[PATH_T];   // flush round j: the path this lane writes into
    int rS[PATH_T];                    // and that policy's S (0: no path)
};

// The flush targets of the lane's rounds, once per item (every lane, after
// base and S are set): round j writes for policy (64 / PATH_T) j + l / PATH_T.
__device__ __forceinline__ void path_prepare(PathStage &ps, int lane)
{
    constexpr int PER = 64 / PATH_T;
    const int Sm = ps.base != nullptr ? ps.S : 0;
#pragma unroll
    for (int j = 0; j < PATH_T; ++j) {
        const int src = PER * j + lane / PATH_T;
        ps.rdst[j] = __shfl((unsigned long long)ps.base, src);
        ps.rS[j] = __shfl(Sm, src);
    }
}

// Every lane of the wavefront calls path_put for each step t, from its top
// step down to t = 0 (the values of a lane with t >= S are not written out).
__device__ __forceinline__ void path_put(const PathStage &ps, int t, double r, int lane)
{
    ps.buf[(t & (PATH_T - 1)) * PATH_ROW + lane] = r;
    if ((t & (PATH_T - 1)) == 0) {
        __builtin_amdgcn_wave_barrier();
        const int u = lane & (PATH_T - 1);
        constexpr int PER = 64 / PATH_T;   // policies per round
        constexpr int B = 4;               // rounds whose LDS operations are issued together
        // A global store: a flat one would also count against the LDS
        // counter and make the next rounds' LDS operations wait for it.
        typedef __attribute__((address_space(1))) double global_double;
#pragma unroll
        for (int j0 = 0; j0 < 64 / PER; j0 += B) {
            double x[B];
#pragma unroll
            for (int i = 0; i < B; ++i) x[i] = ps.buf[u * PATH_ROW + PER * (j0 + i) + lane / PATH_T];
#pragma unroll
            for (int i = 0; i < B; ++i)
                if (t + u < ps.rS[j0 + i]) ((global_double *)ps.rdst[j0 + i])[t + u] = x[i];
        }
        __builtin_amdgcn_wave_barrier();
    }
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
                                              bool has1, bool has2, const double *r3 = nullptr)
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
                    o[4 * k + 3] = (live && r3 != nullptr) ? r3[k] : 0.0;
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

__device__ __forceinline__ void wait_for_v(double q, double v)
{
    asm volatile("" ::"v"(q), "v"(v));
}

// Curve ring of one wavefront (level scalar-reserve items): the discount
// factors of the item's K scenarios pass through LDS in chunks of RING_C
// steps, two chunk slots per wavefront.  A chunk is read from the curves with
// vector loads one chunk ahead (vector loads complete in order, so the wait
// for a chunk never waits for a later one) and written to its slot when the
// wavefront enters the chunk before it; every step then reads its K values
// with wavefront-uniform LDS reads (broadcast, no bank conflicts) one block
// ahead.  Ring row d (d = steps below the first step of the ring phase) is at
// (d mod 2 RING_C) * K: the chunk of row d is slot (d / RING_C) mod 2.
template <int K>
struct Ring {
    static constexpr int PL = RING_C * K / 64;   // doubles per lane per chunk
    static_assert(PL >= 1 && K % PL == 0, "a lane's share of a chunk lies in one step row");
};

// Lane's share of the chunk whose first row is step tt (rows tt, tt - 1, ...,
// clamped at step 0): row (lane PL) / K, scenarios (lane PL) mod K onwards.
template <int K>
__device__ __forceinline__ void ring_fetch(const double *__restrict__ vb, int stride, int tt,
                                           int lane, double (&g)[Ring<K>::PL])
{
    constexpr int PL = Ring<K>::PL;
    const int e = lane * PL;
    const double *src = vb + (ptrdiff_t)max(tt - e / K, 0) * stride + e % K;
#pragma unroll
    for (int i = 0; i < PL; ++i) g[i] = src[i];
}

template <int K>
__device__ __forceinline__ void ring_store(double *ring, int slot, int lane,
                                           const double (&g)[Ring<K>::PL])
{
    constexpr int PL = Ring<K>::PL;
    double *dst = ring + slot * RING_C * K + lane * PL;
#pragma unroll
    for (int i = 0; i < PL; ++i) dst[i] = g[i];
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
    int tmax;     // largest remaining term of the lane's tile (wavefront-uniform)
    int qa, qb;   // LDS indices of the q of life 1 / life 2 at t = 0
    double a0, a1mb1, b1, a1;
    double rS;    // boundary reserve (state 0)
    const double *cfb;   // table tiles: cash flow of step t at cfb[t * cf_cols]
};

// Payment pattern of one lane (escalating or annually paid annuity in
// payment, Sec. 5.3): every cash flow of such a policy is its level value
// times F(T), T = base + t the payment time in months after node 0, with
// F(T) = (1+e)^n(T), n(T) = number of anniversaries in (0, T] (anniversaries
// at a, a + 12, ...), and for annual payment 12 F(T) at an anniversary and 0
// elsewhere.  Steps are taken in decreasing t, one at a time, so n falls by
// at most one per step and the level follows by one multiplication by
// 1/(1+e) at each anniversary crossed.
struct PatLane {
    int base;      // node shift + payment offset (1 for arrears)
    int a;         // months from node 0 to the first anniversary, 1..12
    int annual;
    double ginv;   // 1 / (1 + e)
    double lev;    // (1 + e)^n at the last step taken
    int n;         // n(T) at the last step taken
};

// n(T) for T >= 0: floor((T + 12 - a) / 12).
__device__ __forceinline__ unsigned pat_count(int T, int a) { return (unsigned)(T + 12 - a) / 12u; }

// Lane state for a walk that starts at step t0 (its first call is for t0).
__device__ __forceinline__ PatLane pat_init(const RecParams &P, int slot, int shift, int t0)
{
    PatLane pl;
    const int code = P.pat_code[slot];
    const double g = P.pat_g[slot];
    pl.a = code & 255;
    pl.annual = code & PAT_ANNUAL;
    pl.base = shift + ((code & PAT_ARREARS) ? 1 : 0);
    pl.ginv = 1.0 / g;
    const int n0 = (int)pat_count(max(pl.base + t0, 0), pl.a);
    double lev = 1.0, x = g;   // g^n0 by repeated squaring
    for (int k = n0; k > 0; k >>= 1) {
        if (k & 1) lev *= x;
        x *= x;
    }
    pl.lev = lev;
    pl.n = n0;
    return pl;
}

// F(base + t), advancing the lane's state to step t.
__device__ __forceinline__ double pat_factor(PatLane &pl, int t)
{
    const int T = pl.base + t;
    const unsigned w = (unsigned)(T + 12 - pl.a);
    const int n = (int)(w / 12u);
    pl.lev = n < pl.n ? pl.lev * pl.ginv : pl.lev;
    pl.n = n;
    const bool at = n > 0 && w == 12u * (unsigned)n;
    return pl.annual ? (at ? 12.0 * pl.lev : 0.0) : pl.lev;
}

// Scalar-reserve models: one life (annuity, term assurance, endowment,
// endowment assurance; Sec. 4.1 with the zero-reserve states removed) and the
// two-life models whose only reserve is state 00 (joint-life annuity, Sec.
// 4.2.1 b; two-life endowment, Sec. 4.2.2; first-death assurance, Sec. 4.2.3),
// with one-step survival probability p = px * py.  Per step and scenario:
//   r <- a0 + v * (p * r + c),  c = p * a1 + (1 - p) * b1 = b1 + p * (a1 - b1).
// Each lane carries J policies (one per tile of the item) x K scenarios.
// FLOW_PATTERN: annuities with a payment pattern (J = 1; no death benefit),
// whose a0 and a1 at step t are the level amounts times F of the payment
// time.  FLOW_TABLE: one life (J = 1), c at step t = p x the table's cash
// flow of the step (loaded with the mortality values of the block).
//
// VR: the all-active phase reads the curves through the wavefront's ring
// (level flows; `ring` is the wavefront's 2 RING_C K doubles of LDS).
template <int K, int J, bool LDSQ, bool TWO, bool SHOCK, int FLOW, bool VR = false>
__device__ __forceinline__ void scalar_steps(const double *__restrict__ lq,
                                             const double *__restrict__ gq,
                                             const double *__restrict__ vb, int stride,
                                             const ScalarLane (&L)[J], PatLane (&PL)[J], int cfs,
                                             double m, int smax, int smin, double (&r)[J][K],
                                             const PathStage &ps, double *ring = nullptr)
{
    const int plane = threadIdx.x & 63;
    // Cash flow of step t from the table (table tiles only).
    auto cfload = [&](int j, int t) -> double {
        if constexpr (FLOW == FLOW_TABLE) return L[j].cfb[(ptrdiff_t)t * cfs];
        else return 0.0;
    };
    // x1, x2: one-step survival probabilities from the staged table.
    auto coeffs = [&](int j, int t, double x1, double x2, double cv, double &p, double &c,
                      double &a0) {
        const ScalarLane &l = L[j];
        if constexpr (SHOCK) {
            x1 = 1.0 - fmin(1.0, m * (1.0 - x1));
            if constexpr (TWO) x2 = 1.0 - fmin(1.0, m * (1.0 - x2));
        }
        p = TWO ? x1 * x2 : x1;
        if constexpr (FLOW == FLOW_PATTERN) {
            const double f = pat_factor(PL[j], t);
            c = p * (f * l.a1);
            a0 = f * l.a0;
        } else if constexpr (FLOW == FLOW_TABLE) {
            c = p * cv;
            a0 = l.a0;
        } else {
            c = fma(p, l.a1mb1, l.b1);   // p a1 + (1 - p) b1: arrears amount, death benefit
            a0 = l.a0;
        }
    };
    auto apply = [&](double (&rj)[K], const double (&vk)[K], double p, double c, double a0) {
#pragma unroll
        for (int k = 0; k < K; ++k) rj[k] = fma(vk[k], fma(p, rj[k], c), a0);
    };
    constexpr int U = StepBlock<K, J>::U;
    auto load_block = [&](int tb, const double *vtb, double (&vk)[U][K], double (&q1)[U][J],
                          double (&q2)[U][J], double (&cv)[U][J]) {
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
                cv[u][j] = cfload(j, tb - u);
            }
    };
    // One block of U steps, every policy of the block active (t < smin).
    // Path output goes out after the block, so that the block's steps stay
    // one branch-free stretch of code (the coefficients of later steps
    // overlap the chain of earlier ones).
    auto run_block = [&](int tb, const double (&vk)[U][K], const double (&q1)[U][J],
                         const double (&q2)[U][J], const double (&cv)[U][J]) {
        [[maybe_unused]] double hist[U];   // path output (one scenario and policy per lane)
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                double p, c, a0;
                coeffs(j, tb - u, q1[u][j], q2[u][j], cv[u][j], p, c, a0);
                apply(r[j], vk[u], p, c, a0);
            }
            if constexpr (K == 1 && J == 1) hist[u] = r[0][0];
        }
        if constexpr (K == 1 && J == 1) {
            if (ps.buf != nullptr) {
#pragma unroll
                for (int u = 0; u < U; ++u) path_put(ps, tb - u, hist[u], plane);
            }
        }
    };
    // Ragged head of the item (t >= smin): a policy that has not started
    // (t >= S) takes the step with p = 0, c = 0, a0 = r_S, which leaves its
    // reserve at the boundary value exactly (v * 0 + r_S = r_S), so the loop
    // needs no branches.  Its table reads land in the staged table's padding.
    // A tile none of whose policies has started yet (t >= its largest term)
    // skips the step as a whole (a wavefront-uniform branch).
    int t = smax - 1;
    for (; t >= smin; --t) {
        const double *vt = vb + (ptrdiff_t)t * stride;
        double vk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vk[k] = vt[k];
        double x1[J], x2[J], cv[J];   // every table read issued before the first branch
#pragma unroll
        for (int j = 0; j < J; ++j) {
            x1[j] = qload<LDSQ>(lq, gq, L[j].qa + t);
            x2[j] = TWO ? qload<LDSQ>(lq, gq, L[j].qb + t) : 0.0;
            cv[j] = cfload(j, t);
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (J > 1 && t >= L[j].tmax) continue;
            double p, c, a0;
            coeffs(j, t, x1[j], x2[j], cv[j], p, c, a0);
            const bool on = t < L[j].S;
            p = on ? p : 0.0;
            c = on ? c : 0.0;
            apply(r[j], vk, p, c, on ? a0 : L[j].rS);
        }
        if constexpr (K == 1 && J == 1) {
            if (ps.buf != nullptr) path_put(ps, t, r[0][0], plane);
        }
    }
    if constexpr (VR) {
        // Whole chunks of the all-active phase through the ring; the steps
        // after the last whole chunk take the loops below.
        constexpr int C = RING_C;
        static_assert(C % (2 * U) == 0, "a chunk holds whole pairs of blocks");
        const int lane = threadIdx.x & 63;
        const int nfull = (t + 1) / C;
        if (nfull > 0) {
            const int top0 = t;
            double g[Ring<K>::PL];
            ring_fetch<K>(vb, stride, top0, lane, g);
            ring_store<K>(ring, 0, lane, g);
            if (nfull > 1) ring_fetch<K>(vb, stride, top0 - C, lane, g);
            auto load_ring = [&](int tb, double (&vk)[U][K], double (&q1)[U][J], double (&q2)[U][J],
                                 double (&cv)[U][J]) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double *row = ring + ((top0 - tb + u) & (2 * C - 1)) * K;
#pragma unroll
                    for (int k = 0; k < K; ++k) vk[u][k] = row[k];
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int j = 0; j < J; ++j) {
                        q1[u][j] = qload<LDSQ>(lq, gq, L[j].qa + tb - u);
                        q2[u][j] = TWO ? qload<LDSQ>(lq, gq, L[j].qb + tb - u) : 0.0;
                        cv[u][j] = 0.0;
                    }
            };
            double av[U][K], aq1[U][J], aq2[U][J], acv[U][J];
            double bv[U][K], bq1[U][J], bq2[U][J], bcv[U][J];
            load_ring(t, av, aq1, aq2, acv);
            for (int ci = 0; ci < nfull; ++ci) {
                // Entering chunk ci: its successor goes to the slot chunk
                // ci - 1 used (whose reads are all done), and the chunk after
                // that is fetched.
                if (ci + 1 < nfull) {
                    __builtin_amdgcn_sched_barrier(0);
                    ring_store<K>(ring, (ci + 1) & 1, lane, g);
                    if (ci + 2 < nfull) ring_fetch<K>(vb, stride, top0 - (ci + 2) * C, lane, g);
                    __builtin_amdgcn_sched_barrier(0);
                }
                for (int i = 0; i < C / (2 * U); ++i) {
                    wait_for_v(aq1[0][0], av[0][0]);
                    __builtin_amdgcn_sched_barrier(0);
                    load_ring(t - U, bv, bq1, bq2, bcv);
                    __builtin_amdgcn_sched_barrier(0);
                    run_block(t, av, aq1, aq2, acv);
                    wait_for_v(bq1[0][0], bv[0][0]);
                    const int tl = max(t - 2 * U, U - 1);
                    __builtin_amdgcn_sched_barrier(0);
                    load_ring(tl, av, aq1, aq2, acv);
                    __builtin_amdgcn_sched_barrier(0);
                    run_block(t - U, bv, bq1, bq2, bcv);
                    t -= 2 * U;
                }
            }
        }
    } else if constexpr (StepBlock<K, J>::PIPE) {
        // Pairs of blocks through two named buffers (ping-pong): no register
        // copy of a block in flight and no branch between a prefetch and its
        // use, so the compiler keeps every load at its issue point.  The
        // prefetch after the last pair is clamped in bounds and unused.
        const int npair = ((t + 1) / U) / 2;
        if (npair > 0) {
            double av[U][K], aq1[U][J], aq2[U][J], acv[U][J];
            double bv[U][K], bq1[U][J], bq2[U][J], bcv[U][J];
            load_block(t, vb + (ptrdiff_t)t * stride, av, aq1, aq2, acv);
            for (int i = 0; i < npair; ++i) {
                wait_for(aq1[0][0], av[0][0]);
                __builtin_amdgcn_sched_barrier(0);
                load_block(t - U, vb + (ptrdiff_t)(t - U) * stride, bv, bq1, bq2, bcv);
                __builtin_amdgcn_sched_barrier(0);
                run_block(t, av, aq1, aq2, acv);
                wait_for(bq1[0][0], bv[0][0]);
                const int tl = max(t - 2 * U, U - 1);
                __builtin_amdgcn_sched_barrier(0);
                load_block(tl, vb + (ptrdiff_t)tl * stride, av, aq1, aq2, acv);
                __builtin_amdgcn_sched_barrier(0);
                run_block(t - U, bv, bq1, bq2, bcv);
                t -= 2 * U;
            }
        }
    }
    for (; t >= U - 1; t -= U) {
        double vk[U][K], q1[U][J], q2[U][J], cv[U][J];
        load_block(t, vb + (ptrdiff_t)t * stride, vk, q1, q2, cv);
        run_block(t, vk, q1, q2, cv);
    }
    for (; t >= 0; --t) {   // fewer than U steps left
        const double *vt = vb + (ptrdiff_t)t * stride;
        double vk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vk[k] = vt[k];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            double p, c, a0;
            coeffs(j, t, qload<LDSQ>(lq, gq, L[j].qa + t),
                   TWO ? qload<LDSQ>(lq, gq, L[j].qb + t) : 0.0, cfload(j, t), p, c, a0);
            apply(r[j], vk, p, c, a0);
        }
        if constexpr (K == 1 && J == 1) {
            if (ps.buf != nullptr) path_put(ps, t, r[0][0], plane);
        }
    }
}

// An item of `count` (<= J) consecutive tiles of one scalar model and a block
// of K scenarios: lane l carries slot first + 64 j + l of every tile j.
template <int K, int J, bool LDSQ, bool TWO, int FLOW, bool VR = false>
__device__ __forceinline__ void run_scalar(const RecParams &P, const double *__restrict__ lq,
                                           const double *__restrict__ vcurves, int node_rel,
                                           int tile, int count, const Tile &T0, int item_smax,
                                           int item_smin, int sb, int lane, double *ring = nullptr,
                                           double *pstage = nullptr)
{
    const int node = P.node_begin + node_rel;
    const int shift = node * P.node_step;
    const int smax = item_smax - shift;
    const int smin = max(item_smin - shift, 0);
    const double m = P.shock[node];
    ScalarLane L[J];
    PatLane PL[J];
    int uid[J];
    double r[J][K];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int slot = T0.first + j * TILE + lane;   // tiles of an item are consecutive
        if (j < count) {
            L[j].tmax = wave_uniform(P.tiles[tile + j].smax) - shift;
            L[j].S = P.term[slot] - shift;
            uid[j] = P.uidx[slot];
            L[j].a0 = P.coef[0 * P.n_pad + slot];
            L[j].a1 = P.coef[1 * P.n_pad + slot];
            L[j].b1 = P.coef[2 * P.n_pad + slot];
            L[j].a1mb1 = L[j].a1 - L[j].b1;
            L[j].qa = P.qoff1[slot] + P.age1[slot] + shift;
            L[j].qb = TWO ? P.qoff2[slot] + P.age2[slot] + shift : 0;
            L[j].rS = P.coef[3 * P.n_pad + slot];
            L[j].cfb = nullptr;
            if constexpr (FLOW == FLOW_PATTERN) PL[j] = pat_init(P, slot, shift, smax - 1);
            if constexpr (FLOW == FLOW_TABLE)
                L[j].cfb = P.cf_t + P.pat_code[slot] + (ptrdiff_t)shift * P.cf_cols;
#pragma unroll
            for (int k = 0; k < K; ++k) r[j][k] = L[j].rS;
        } else {   // missing tile of a short item: an always-inactive lane
            L[j].tmax = -1;
            L[j].S = -1;
            uid[j] = -1;
            L[j].a0 = L[j].a1 = L[j].b1 = L[j].a1mb1 = L[j].rS = 0.0;
            L[j].qa = shift;
            L[j].qb = shift;
            L[j].cfb = FLOW == FLOW_TABLE ? P.cf_t + (ptrdiff_t)shift * P.cf_cols : nullptr;
            if constexpr (FLOW == FLOW_PATTERN) PL[j] = PatLane{0, 12, 0, 1.0, 1.0, 0};
#pragma unroll
            for (int k = 0; k < K; ++k) r[j][k] = 0.0;
        }
    }
    const double *vb = vcurves + (size_t)node * P.n_steps * P.scen_pad + (P.scen_begin + sb);
    PathStage ps{nullptr, 0, nullptr};
    if constexpr (K == 1 && J == 1) {
        ps.buf = pstage;
        ps.S = L[0].S;
        if (P.path != nullptr && uid[0] >= 0) {
            if (L[0].S > 0) {
                ps.base = P.path + P.path_off[uid[0]];
                ps.base[L[0].S] = r[0][0];
            } else {
                P.path[P.path_off[uid[0]]] = 0.0;   // expired: its one entry is 0
            }
        }
        if (ps.buf != nullptr) path_prepare(ps, lane);
    }
    if (m == 1.0)
        scalar_steps<K, J, LDSQ, TWO, false, FLOW, VR>(lq, P.q, vb, P.scen_pad, L, PL, P.cf_cols, m,
                                                       smax, smin, r, ps, ring);
    else
        scalar_steps<K, J, LDSQ, TWO, true, FLOW, VR>(lq, P.q, vb, P.scen_pad, L, PL, P.cf_cols, m,
                                                      smax, smin, r, ps, ring);
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
//
// ESC: an annuity with a payment pattern (premium 0): every coefficient at
// step t is its level value times F of the payment time.
template <int K, bool LDSQ, bool LAST, bool SHOCK, bool ESC>
__device__ __forceinline__ void vector_steps(const double *__restrict__ lq,
                                             const double *__restrict__ gq,
                                             const double *__restrict__ vb, int stride, int qa,
                                             int qb, double m, const double (&cf)[7], PatLane &pl,
                                             int S, int smax, int smin, double (&r0)[K],
                                             double (&r1)[K], double (&r2)[K], const PathStage &ps)
{
    const int plane = threadIdx.x & 63;
    // Path output: every lane at every step (uniform control flow).
    auto put = [&](int t) {
        if constexpr (K == 1) {
            if (ps.buf != nullptr) path_put(ps, t, r0[0], plane);
        }
    };
    auto apply = [&](const double (&vk)[K], double px, double py, int t) {
        double f = 1.0;
        if constexpr (ESC) f = pat_factor(pl, t);
        const double c00a = ESC ? f * cf[0] : cf[0], c00r = ESC ? f * cf[1] : cf[1];
        const double c01a = ESC ? f * cf[2] : cf[2], c01r = ESC ? f * cf[3] : cf[3];
        const double c10a = ESC ? f * cf[4] : cf[4], c10r = ESC ? f * cf[5] : cf[5];
        const double qx = 1.0 - px, qy = 1.0 - py;
        const double w00 = px * py, w10 = qx * py;
        const double w01 = px * qy;
        // y-independent terms: arrears amounts and, for LAST, the benefit d
        // paid on the second death (from 00 both die: qx qy; from 01 x dies:
        // qx; from 10 y dies: qy); d = 0 leaves every value unchanged.
        const double d = cf[6];
        double cw0 = fma(w10, c10r, w00 * c00r);
        if constexpr (LAST) cw0 = fma(qx * qy, d, fma(w01, c01r, cw0));
        const double cw1 = LAST ? fma(qx, d, px * c01r) : px * c01r;
        const double cw2 = LAST ? fma(qy, d, py * c10r) : py * c10r;
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
    };
    int t = smax - 1;
    const double *vt = vb + (ptrdiff_t)t * stride;
    for (; t >= smin; --t, vt -= stride) {
        double vk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) vk[k] = vt[k];
        if (t < S)
            apply(vk, p_eff<LDSQ, SHOCK>(lq, gq, qa + t, m), p_eff<LDSQ, SHOCK>(lq, gq, qb + t, m), t);
        put(t);
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
    // Path output after the block (the block's steps stay branch-free).
    auto run_block = [&](int tb, const double (&vk)[U][K], const double (&qx)[U],
                         const double (&qy)[U]) {
        [[maybe_unused]] double hist[U];   // path output (one scenario per lane)
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double x = qx[u], y = qy[u];
            if constexpr (SHOCK) {
                x = 1.0 - fmin(1.0, m * (1.0 - x));
                y = 1.0 - fmin(1.0, m * (1.0 - y));
            }
            apply(vk[u], x, y, tb - u);
            if constexpr (K == 1) hist[u] = r0[0];
        }
        if constexpr (K == 1) {
            if (ps.buf != nullptr) {
#pragma unroll
                for (int u = 0; u < U; ++u) path_put(ps, tb - u, hist[u], plane);
            }
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
        put(t);
    }
}

template <int K, bool LDSQ, bool LAST, bool ESC>
__device__ __forceinline__ void run_vector(const RecParams &P, const double *__restrict__ lq,
                                           const double *__restrict__ vcurves, int node_rel,
                                           int tile, const Tile &T, int sb, int lane,
                                           double *pstage)
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
    double cf[7];
#pragma unroll
    for (int j = 0; j < 6; ++j) cf[j] = P.coef[j * P.n_pad + slot];
    cf[6] = LAST ? P.coef[6 * P.n_pad + slot] : 0.0;
    const int qa = P.qoff1[slot] + P.age1[slot] + shift;
    const int qb = P.qoff2[slot] + P.age2[slot] + shift;
    const double *vb = vcurves + (size_t)node * P.n_steps * P.scen_pad + (P.scen_begin + sb);

    double r0[K], r1[K], r2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { r0[k] = 0.0; r1[k] = 0.0; r2[k] = 0.0; }

    PathStage ps{nullptr, S, nullptr};
    if constexpr (K == 1) {
        ps.buf = pstage;
        if (P.path != nullptr && live) {
            ps.base = P.path + P.path_off[uid];
            ps.base[S] = 0.0;
        } else if (P.path != nullptr && uid >= 0) {
            P.path[P.path_off[uid]] = 0.0;         // expired: its one entry is 0
        }
        if (ps.buf != nullptr) path_prepare(ps, lane);
    }
    // A lane takes its first step at t = S - 1 (the head skips t >= S).
    PatLane pl{0, 12, 0, 1.0, 1.0, 0};
    if constexpr (ESC) pl = pat_init(P, slot, shift, S - 1);
    if (m == 1.0)
        vector_steps<K, LDSQ, LAST, false, ESC>(lq, P.q, vb, P.scen_pad, qa, qb, m, cf, pl, S, smax,
                                                smin, r0, r1, r2, ps);
    else
        vector_steps<K, LDSQ, LAST, true, ESC>(lq, P.q, vb, P.scen_pad, qa, qb, m, cf, pl, S, smax,
                                               smin, r0, r1, r2, ps);
    store_results<K>(P, node_rel, tile, sb, lane, uid, live, r0, r1, r2, LAST, true);
}

// Single- and joint-life annuities paid at the fraction f of each month
// (Sec. 3.1's f; survival to t + f by f x the month's death probability):
//   r <- -P + v^f * pf * pay + v * p * r',  pf = prod over lives of (1 - f + f p_l).
// A lane idles (r stays 0) until its first step; one policy per lane.
template <int K, bool LDSQ, bool TWO, bool SHOCK>
__device__ __forceinline__ void run_frac(const RecParams &P, const double *__restrict__ lq,
                                         const double *__restrict__ vcurves, int node_rel, int tile,
                                         const Tile &T, int sb, int lane, double *pstage)
{
    const int node = P.node_begin + node_rel;
    const int shift = node * P.node_step;
    const int slot = T.first + lane;
    const int S = P.term[slot] - shift;
    const int uid = P.uidx[slot];
    const bool live = (uid >= 0) && (S > 0);
    const int smax = T.smax - shift;
    const double m = P.shock[node];
    const double a0 = P.coef[slot];
    const double pay = P.coef[P.n_pad + slot];
    const double f = P.frac, g = 1.0 - P.frac;
    const int qa = P.qoff1[slot] + P.age1[slot] + shift;
    const int qb = TWO ? P.qoff2[slot] + P.age2[slot] + shift : 0;
    const size_t off = (size_t)node * P.n_steps * P.scen_pad + (P.scen_begin + sb);
    const double *vb = vcurves + off;
    const double *vfb = P.vf + off;
    double r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = 0.0;
    PathStage ps{nullptr, S, nullptr};
    if constexpr (K == 1) {
        ps.buf = pstage;
        if (P.path != nullptr && uid >= 0) {
            if (live) {
                ps.base = P.path + P.path_off[uid];
                ps.base[S] = 0.0;
            } else {
                P.path[P.path_off[uid]] = 0.0;   // expired: its one entry is 0
            }
        }
        if (ps.buf != nullptr) path_prepare(ps, lane);
    }
    for (int t = smax - 1; t >= 0; --t) {
        const double x1 = p_eff<LDSQ, SHOCK>(lq, P.q, qa + t, m);
        const double x2 = TWO ? p_eff<LDSQ, SHOCK>(lq, P.q, qb + t, m) : 1.0;
        const double p = TWO ? x1 * x2 : x1;
        const double pf = TWO ? fma(f, x1, g) * fma(f, x2, g) : fma(f, x1, g);
        const double c = pf * pay;
        const bool on = t < S;
        const double *vt = vb + (ptrdiff_t)t * P.scen_pad;
        const double *vft = vfb + (ptrdiff_t)t * P.scen_pad;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double nr = fma(vt[k], p * r[k], fma(vft[k], c, a0));
            r[k] = on ? nr : r[k];
        }
        if constexpr (K == 1) {
            if (ps.buf != nullptr) path_put(ps, t, r[0], lane);
        }
    }
    store_results<K>(P, node_rel, tile, sb, lane, uid, live, r, r, r, false, false);
}

// One life on an uploaded Markov model (Sec. 4.5; the matrix need not be
// upper triangular): up to four states, zero padded to four.  With y = c +
// r' per state (c: the benefits paid at the end of a month ending in the
// state) and W_t the model's matrix at the attained age:
//   r_i <- a_i + v * sum_j W_t[i][j] * y_j,  a_0 = - premium, a_i = 0 else.
// The lane's matrix of the next step is loaded while the current one is
// used.  The scenarios go through in chunks of KM <= 4 chains (the matrix is
// read again per chunk, from L2), so this path needs few registers and the
// kernel's register budget stays that of the level paths.
template <int KM>
__device__ __forceinline__ void markov_chunk(const RecParams &P, const double2 *__restrict__ wb,
                                             const double *__restrict__ vb, int S, int smax,
                                             double a0, const double (&c)[4], double *path,
                                             double (&r)[4][KM])
{
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < KM; ++k) r[i][k] = 0.0;
    // The lane starts at its own last step (t < S); padding and expired
    // lanes take no step (S <= 0).
    int t = min(S, smax) - 1;
    double2 wn[8];
    if (t >= 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) wn[e] = wb[(size_t)t * 8 + e];
    }
    for (; t >= 0; --t) {
        double w[16];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            w[2 * e] = wn[e].x;
            w[2 * e + 1] = wn[e].y;
        }
        if (t > 0) {
#pragma unroll
            for (int e = 0; e < 8; ++e) wn[e] = wb[(size_t)(t - 1) * 8 + e];
        }
        const double *vt = vb + (ptrdiff_t)t * P.scen_pad;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const double v = vt[k];
            double y[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) y[j] = c[j] + r[j][k];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                double acc = w[4 * i] * y[0];
                acc = fma(w[4 * i + 1], y[1], acc);
                acc = fma(w[4 * i + 2], y[2], acc);
                acc = fma(w[4 * i + 3], y[3], acc);
                r[i][k] = fma(v, acc, i == 0 ? a0 : 0.0);
            }
        }
        if (path != nullptr) path[t] = r[0][0];
    }
}

// Models of 5 to 9 states: the lane's matrix (rows of 9, zero padded) is
// read row by row from memory at each step, one scenario chain at a time
// (these tiles are rare; the point is a small register footprint), and the
// benefits are the model's times the policy's amount:
//   r_i <- a_i + v * sum_j W_t[i][j] * (amount c_j + r'_j).
__device__ __forceinline__ void markov9_chain(const RecParams &P, const double *__restrict__ wb,
                                              const double *__restrict__ vb, int S, int smax, double a0,
                                              const double (&c)[MAX_MK_STATES], double *path,
                                              double (&r)[MAX_MK_STATES])
{
    constexpr int M = MAX_MK_STATES;
#pragma unroll
    for (int i = 0; i < M; ++i) r[i] = 0.0;
    for (int t = min(S, smax) - 1; t >= 0; --t) {
        const double v = vb[(ptrdiff_t)t * P.scen_pad];
        const double *w = wb + (size_t)t * M * M;
        double y[M];
#pragma unroll
        for (int j = 0; j < M; ++j) y[j] = c[j] + r[j];
#pragma unroll
        for (int i = 0; i < M; ++i) {
            double acc = w[i * M] * y[0];
#pragma unroll
            for (int j = 1; j < M; ++j) acc = fma(w[i * M + j], y[j], acc);
            r[i] = fma(v, acc, i == 0 ? a0 : 0.0);
        }
        if (path != nullptr) path[t] = r[0];
    }
}

template <int K>
__device__ __forceinline__ void run_markov9(const RecParams &P, const double *__restrict__ vcurves,
                                            int node_rel, int tile, const Tile &T, int sb, int lane)
{
    constexpr int M = MAX_MK_STATES;
    const int node = P.node_begin + node_rel;
    const int shift = node * P.node_step;
    const int slot = T.first + lane;
    const int S = P.term[slot] - shift;
    const int uid = P.uidx[slot];
    const bool live = (uid >= 0) && (S > 0);
    const int smax = T.smax - shift;
    const double a0 = P.coef[slot];
    const double amount = P.coef[P.n_pad + slot];
    const int model = uid >= 0 ? P.pat_code[slot] : 0;
    double c[M];
#pragma unroll
    for (int j = 0; j < M; ++j) c[j] = amount * P.mk_c[model * M + j];
    const int age0 = uid >= 0 ? P.age1[slot] + shift : 0;
    const double *wb = P.mk_w + ((size_t)model * P.mk_ages + age0) * (M * M);
    const double *vb = vcurves + (size_t)node * P.n_steps * P.scen_pad + (P.scen_begin + sb);
    double *path = nullptr;
    if constexpr (K == 1) {
        if (P.path != nullptr && uid >= 0) {
            if (live) {
                path = P.path + P.path_off[uid];
                path[S] = 0.0;
            } else {
                P.path[P.path_off[uid]] = 0.0;   // expired: its one entry is 0
            }
        }
    }
    for (int k = 0; k < K; ++k) {
        double r[M];
        markov9_chain(P, wb, vb + k, S, smax, a0, c, path, r);
        double x0[1] = {r[0]}, x1[1] = {r[1]}, x2[1] = {r[2]}, x3[1] = {r[3]};
        store_results<1>(P, node_rel, tile, sb + k, lane, uid, live, x0, x1, x2, true, true, x3);
    }
}

// Three lives (Sec. 4.3, two-state model each): a state with some life
// alive is the set A of living lives (bit l - 1 for life l); the state with
// none alive has reserve 0 (Sec. 3.6.4).  Per step, with the survival p_l and
// death probability q_l = 1 - p_l of each life shared by the chains,
// arrears amount a1, advance amounts a0 (and, all alive, minus the premium)
// and y_B = a1 + r'_B:
//   r_A = a0 + v sum_{B subset of A, B nonempty} prod_{l in B} p_l prod_{l in A\B} q_l y_B.
// The last-survivor annuity pays in every such state; the joint-life annuity
// only in A = {1,2,3}, whose reserve then needs only its own chain (the
// other states never pay again).  One scenario chain at a time: rare tiles,
// small register footprint.  Output slots: state j of the binary labels (life
// 1 the high digit, 1 = dead): A = {1,2,3}, {1,2}, {1,3}, {1}.
template <int K, bool LDSQ, bool SHOCK>
__device__ __forceinline__ void run_three(const RecParams &P, const double *__restrict__ lq,
                                          const double *__restrict__ vcurves, int node_rel, int tile,
                                          const Tile &T, int sb, int lane)
{
    const int node = P.node_begin + node_rel;
    const int shift = node * P.node_step;
    const int slot = T.first + lane;
    const int S = P.term[slot] - shift;
    const int uid = P.uidx[slot];
    const bool live = (uid >= 0) && (S > 0);
    const int smax = T.smax - shift;
    const double m = P.shock[node];
    const bool last = T.kind == KIND_LAST;
    const double a0all = P.coef[slot];              // advance amount - premium (all alive)
    const double a1 = P.coef[P.n_pad + slot];       // arrears amount
    const double a0 = P.coef[2 * P.n_pad + slot];   // advance amount (other states)
    const int qa = P.qoff1[slot] + P.age1[slot] + shift;
    const int qb = P.qoff2[slot] + P.age2[slot] + shift;
    const int qc = P.qoff3[slot] + P.age3[slot] + shift;
    const double *vb = vcurves + (size_t)node * P.n_steps * P.scen_pad + (P.scen_begin + sb);
    double *path = nullptr;
    if constexpr (K == 1) {
        if (P.path != nullptr && uid >= 0) {
            if (live) {
                path = P.path + P.path_off[uid];
                path[S] = 0.0;
            } else {
                P.path[P.path_off[uid]] = 0.0;   // expired: its one entry is 0
            }
        }
    }
    for (int k = 0; k < K; ++k) {
        double r1 = 0.0, r2 = 0.0, r3 = 0.0, r4 = 0.0, r5 = 0.0, r6 = 0.0, r7 = 0.0;   // r_A, A = mask
        for (int t = min(S, smax) - 1; t >= 0; --t) {
            const double p1 = p_eff<LDSQ, SHOCK>(lq, P.q, qa + t, m);
            const double p2 = p_eff<LDSQ, SHOCK>(lq, P.q, qb + t, m);
            const double p3 = p_eff<LDSQ, SHOCK>(lq, P.q, qc + t, m);
            const double q1 = 1.0 - p1, q2 = 1.0 - p2, q3 = 1.0 - p3;
            const double v = vb[(ptrdiff_t)t * P.scen_pad + k];
            const double y7 = a1 + r7;
            if (!last) {
                r7 = fma(v, p1 * p2 * p3 * y7, a0all);
            } else {
                const double y1 = a1 + r1, y2 = a1 + r2, y3 = a1 + r3, y4 = a1 + r4, y5 = a1 + r5,
                             y6 = a1 + r6;
                double n7 = p1 * p2 * p3 * y7;
                n7 = fma(p1 * p2 * q3, y3, n7);
                n7 = fma(p1 * q2 * p3, y5, n7);
                n7 = fma(q1 * p2 * p3, y6, n7);
                n7 = fma(p1 * q2 * q3, y1, n7);
                n7 = fma(q1 * p2 * q3, y2, n7);
                n7 = fma(q1 * q2 * p3, y4, n7);
                const double n3 = fma(p1 * p2, y3, fma(p1 * q2, y1, q1 * p2 * y2));   // {1,2}
                const double n5 = fma(p1 * p3, y5, fma(p1 * q3, y1, q1 * p3 * y4));   // {1,3}
                const double n6 = fma(p2 * p3, y6, fma(p2 * q3, y2, q2 * p3 * y4));   // {2,3}
                r7 = fma(v, n7, a0all);
                r3 = fma(v, n3, a0);
                r5 = fma(v, n5, a0);
                r6 = fma(v, n6, a0);
                r1 = fma(v, p1 * y1, a0);
                r2 = fma(v, p2 * y2, a0);
                r4 = fma(v, p3 * y4, a0);
            }
            if (path != nullptr) path[t] = r7;
        }
        double x0[1] = {r7}, x1[1] = {r3}, x2[1] = {r5}, x3[1] = {r1};
        store_results<1>(P, node_rel, tile, sb + k, lane, uid, live, x0, x1, x2, last, last,
                         last ? x3 : nullptr);
    }
}

template <int K>
__device__ __forceinline__ void run_markov(const RecParams &P, const double *__restrict__ vcurves,
                                           int node_rel, int tile, const Tile &T, int sb, int lane)
{
    if (P.mk_states > 4) {
        run_markov9<K>(P, vcurves, node_rel, tile, T, sb, lane);
        return;
    }
    constexpr int KM = K < 4 ? K : 4;
    const int node = P.node_begin + node_rel;
    const int shift = node * P.node_step;
    const int slot = T.first + lane;
    const int S = P.term[slot] - shift;
    const int uid = P.uidx[slot];
    const bool live = (uid >= 0) && (S > 0);
    const int smax = T.smax - shift;
    const double a0 = P.coef[slot];
    double c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = P.coef[(1 + j) * P.n_pad + slot];
    // rows of the model at the policy's attained age at t = 0 (padding lanes: model 0, age 0)
    const int age0 = uid >= 0 ? P.age1[slot] + shift : 0;
    const double2 *wb = reinterpret_cast<const double2 *>(
        P.mk_w + ((size_t)P.pat_code[slot] * P.mk_ages + age0) * 16);
    const double *vb = vcurves + (size_t)node * P.n_steps * P.scen_pad + (P.scen_begin + sb);
    double *path = nullptr;
    if constexpr (K == 1) {
        if (P.path != nullptr && uid >= 0) {
            if (live) {
                path = P.path + P.path_off[uid];
                path[S] = 0.0;
            } else {
                P.path[P.path_off[uid]] = 0.0;   // expired: its one entry is 0
            }
        }
    }
    for (int kc = 0; kc < K; kc += KM) {
        double r[4][KM];
        markov_chunk<KM>(P, wb, vb + kc, S, smax, a0, c, path, r);
        store_results<KM>(P, node_rel, tile, sb + kc, lane, uid, live, r[0], r[1], r[2], true, true,
                          r[3]);
    }
}

// Persistent grid: each wavefront takes items from its XCD's queue (the
// hardware places workgroup b on XCD b mod 8), then steals from the others.
// The read-only inputs are separate __restrict__ arguments so that the
// compiler may read the wavefront-uniform curve values with scalar loads.
// PAT: the portfolio has tiles whose cash flows vary in time (payment
// patterns or cash-flow tables), run with one policy per lane whatever J.
// VR: level scalar-reserve portfolios with the curve ring (no vector or
// pattern tiles); the wavefront's ring follows the tables in LDS.
template <int K, int J, bool LDSQ, bool VEC, bool PAT, bool VR = false>
__global__ void __launch_bounds__(WG_THREADS)
k_recurrence(RecParams P, const double *__restrict__ vcurves, const Item *__restrict__ items,
             const Tile *__restrict__ tiles, const int *__restrict__ qbeg)
{
    extern __shared__ double s_q[];
    if constexpr (LDSQ) {
        // Stage the tables with 16-byte loads, eight in flight per thread
        // before their LDS writes (one round trip per batch, not per value).
        constexpr int B = 8;
        const int n2 = P.n_q >> 1;
        const double2 *src = reinterpret_cast<const double2 *>(P.q);
        double2 *dst = reinterpret_cast<double2 *>(s_q);
        for (int base = 0; base < n2; base += B * WG_THREADS) {
            double2 a[B];
#pragma unroll
            for (int u = 0; u < B; ++u)   // clamped: every load in bounds, none predicated
                a[u] = src[min(base + u * WG_THREADS + (int)threadIdx.x, n2 - 1)];
#pragma unroll
            for (int u = 0; u < B; ++u)   // all B loads issued before the first write
                asm volatile("" ::"v"(a[u].x), "v"(a[u].y));
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int i = base + u * WG_THREADS + (int)threadIdx.x;
                if (i < n2) dst[i] = a[u];
            }
        }
        if ((P.n_q & 1) && threadIdx.x == 0) s_q[P.n_q - 1] = P.q[P.n_q - 1];
        __syncthreads();
    }
    double *ring = nullptr;
    if constexpr (VR) ring = s_q + P.ring_off + (threadIdx.x >> 6) * ring_doubles_per_wave(K);
    double *pstage = nullptr;   // path output (one scenario per lane): the wavefront's stage
    if constexpr (K == 1) {
        if (P.path != nullptr) pstage = s_q + P.path_lds + (threadIdx.x >> 6) * PATH_STAGE_DOUBLES;
    }
    const int lane = threadIdx.x & 63;
    int qcur = blockIdx.x % P.n_queues;
    __shared__ int s_win[2];   // window mode: first item of the window, its queue (-1: none left)
    while (true) {
        int idx = 0;
        if (P.win) {
            // The workgroup takes a window of WG_THREADS/64 consecutive items
            // with one atomic, one item per wavefront, and starts them
            // together; the next window waits for all of them.  Thread 0
            // moves the workgroup to another queue when this one is empty.
            constexpr int NW = WG_THREADS / 64;
            __syncthreads();
            if (threadIdx.x == 0) {
                int q = qcur, base = -1;
                for (int scan = 0; scan <= P.n_queues && base < 0; ++scan) {
                    const int b = atomicAdd(&P.counters[q], NW);
                    if (qbeg[q] + b < qbeg[q + 1]) {
                        base = b;
                        break;
                    }
                    int nq = -1;   // next queue with items left (heads may be stale: rescan)
                    for (int i = 1; i <= P.n_queues && nq < 0; ++i) {
                        const int c = (q + i) % P.n_queues;
                        const int h = __hip_atomic_load(&P.counters[c], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
                        if (qbeg[c] + h < qbeg[c + 1]) nq = c;
                    }
                    if (nq < 0) break;
                    q = nq;
                }
                s_win[0] = base;
                s_win[1] = base < 0 ? -1 : q;
            }
            __syncthreads();
            if (s_win[1] < 0) break;
            qcur = s_win[1];
            idx = s_win[0] + (int)(threadIdx.x >> 6);
            if (wave_uniform(qbeg[qcur]) + idx >= wave_uniform(qbeg[qcur + 1])) continue;   // partial window
        } else {
            if (lane == 0) idx = atomicAdd(&P.counters[qcur], 1);
            idx = wave_uniform(idx);   // every lane is active here: lane 0's value
        }
        const int beg = wave_uniform(qbeg[qcur]);
        const int end = wave_uniform(qbeg[qcur + 1]);
        if (beg + idx >= end) {
            // This queue is empty: read every queue's head at once (lane i:
            // queue i) and move to the next one, in queue order after this
            // one, that still has items; none left: done.  A head read here
            // may be stale, so a queue can turn out empty at its atomic, and
            // the scan repeats.
            bool more = false;
            if (lane < P.n_queues) {
                const int h = __hip_atomic_load(&P.counters[lane], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
                more = qbeg[lane] + h < qbeg[lane + 1];
            }
            const unsigned long long m = __ballot(more);
            if (m == 0ull) break;
            const unsigned long long after = m & ~((2ull << qcur) - 1ull);   // queues > qcur
            qcur = after ? __builtin_ctzll(after) : __builtin_ctzll(m);
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
        T.flow = wave_uniform(T.flow);
        // Terms are bucketed, not strictly sorted: take the extremes over the
        // item's tiles.
        int smax = T.smax, smin = T.smin;
        for (int j = 1; j < count; ++j) {
            smax = max(smax, wave_uniform(tiles[tile + j].smax));
            smin = min(smin, wave_uniform(tiles[tile + j].smin));
        }
        if (PAT && T.flow != FLOW_LEVEL) {
            if constexpr (PAT) {
                if (T.flow == FLOW_FRAC) {
                    const bool shock = P.shock[P.node_begin + node_rel] != 1.0;
                    if (T.kind == KIND_JOINT) {
                        if (shock) run_frac<K, LDSQ, true, true>(P, s_q, vcurves, node_rel, tile, T, sb, lane, pstage);
                        else run_frac<K, LDSQ, true, false>(P, s_q, vcurves, node_rel, tile, T, sb, lane, pstage);
                    } else {
                        if (shock) run_frac<K, LDSQ, false, true>(P, s_q, vcurves, node_rel, tile, T, sb, lane, pstage);
                        else run_frac<K, LDSQ, false, false>(P, s_q, vcurves, node_rel, tile, T, sb, lane, pstage);
                    }
                } else if (T.flow == FLOW_MARKOV) {
                    run_markov<K>(P, vcurves, node_rel, tile, T, sb, lane);
                } else if (T.flow == FLOW_THREE) {
                    if (P.shock[P.node_begin + node_rel] != 1.0)
                        run_three<K, LDSQ, true>(P, s_q, vcurves, node_rel, tile, T, sb, lane);
                    else
                        run_three<K, LDSQ, false>(P, s_q, vcurves, node_rel, tile, T, sb, lane);
                } else if (T.flow == FLOW_TABLE)
                    run_scalar<K, 1, LDSQ, false, FLOW_TABLE>(P, s_q, vcurves, node_rel, tile, 1, T,
                                                              T.smax, T.smin, sb, lane, nullptr,
                                                              pstage);
                else if (T.kind == KIND_SINGLE)
                    run_scalar<K, 1, LDSQ, false, FLOW_PATTERN>(P, s_q, vcurves, node_rel, tile, 1, T,
                                                                T.smax, T.smin, sb, lane, nullptr,
                                                                pstage);
                else if (T.kind == KIND_JOINT)
                    run_scalar<K, 1, LDSQ, true, FLOW_PATTERN>(P, s_q, vcurves, node_rel, tile, 1, T,
                                                               T.smax, T.smin, sb, lane, nullptr,
                                                               pstage);
                else if (T.kind == KIND_REV)
                    run_vector<K, LDSQ, false, true>(P, s_q, vcurves, node_rel, tile, T, sb, lane,
                                                 pstage);
                else
                    run_vector<K, LDSQ, true, true>(P, s_q, vcurves, node_rel, tile, T, sb, lane,
                                                 pstage);
            }
        } else if (T.kind == KIND_SINGLE) {
            run_scalar<K, J, LDSQ, false, FLOW_LEVEL, VR>(P, s_q, vcurves, node_rel, tile, count, T,
                                                          smax, smin, sb, lane, ring, pstage);
        } else if (T.kind == KIND_JOINT) {
            run_scalar<K, J, LDSQ, true, FLOW_LEVEL, VR>(P, s_q, vcurves, node_rel, tile, count, T,
                                                         smax, smin, sb, lane, ring, pstage);
        } else if constexpr (VEC) {
            if (T.kind == KIND_REV)
                run_vector<K, LDSQ, false, false>(P, s_q, vcurves, node_rel, tile, T, sb, lane,
                                                 pstage);
            else
                run_vector<K, LDSQ, true, false>(P, s_q, vcurves, node_rel, tile, T, sb, lane,
                                                 pstage);
        }
    }
    // The last workgroup to finish re-arms the queues for the next launch.
    // One atomic per workgroup, not per wavefront: every completion atomic
    // goes to the same address and they serialise there, which at the end
    // of a launch whose wavefronts finish together cost tens of microseconds.
    __syncthreads();
    if (threadIdx.x == 0) {
        if (atomicAdd(&P.counters[MAX_QUEUES], 1) == (int)gridDim.x - 1) {
            for (int i = 0; i <= MAX_QUEUES; ++i) atomicExch(&P.counters[i], 0);
        }
    }
}

template <int K, int J, bool PAT>
static void launch_kjp(const RecParams &p, int grid, size_t lds, hipStream_t s)
{
    const dim3 g(grid), b(WG_THREADS);
    if (p.q_in_lds) {
        if (p.has_vector)
            hipLaunchKernelGGL((k_recurrence<K, J, true, true, PAT>), g, b, lds, s, p, p.v, p.items, p.tiles, p.qbeg);
        else
            hipLaunchKernelGGL((k_recurrence<K, J, true, false, PAT>), g, b, lds, s, p, p.v, p.items, p.tiles, p.qbeg);
    } else {
        // lds: the path stages when the run writes a path, else 0
        if (p.has_vector)
            hipLaunchKernelGGL((k_recurrence<K, J, false, true, PAT>), g, b, lds, s, p, p.v, p.items, p.tiles, p.qbeg);
        else
            hipLaunchKernelGGL((k_recurrence<K, J, false, false, PAT>), g, b, lds, s, p, p.v, p.items, p.tiles, p.qbeg);
    }
}


// Launch of the (K, J) instance for the supported pairs (supported_kj).
template <bool PAT>
static hipError_t launch_switch(int K, int J, const RecParams &p, int grid, size_t lds,
                                hipStream_t s)
{
    switch (J * 64 + K) {
    case 64 + 1: launch_kjp<1, 1, PAT>(p, grid, lds, s); break;
    case 64 + 2: launch_kjp<2, 1, PAT>(p, grid, lds, s); break;
    case 64 + 4: launch_kjp<4, 1, PAT>(p, grid, lds, s); break;
    case 64 + 8: launch_kjp<8, 1, PAT>(p, grid, lds, s); break;
    case 64 + 16: launch_kjp<16, 1, PAT>(p, grid, lds, s); break;
    case 64 + 32: launch_kjp<32, 1, PAT>(p, grid, lds, s); break;
    case 128 + 4: launch_kjp<4, 2, PAT>(p, grid, lds, s); break;
    case 128 + 8: launch_kjp<8, 2, PAT>(p, grid, lds, s); break;
    case 128 + 16: launch_kjp<16, 2, PAT>(p, grid, lds, s); break;
    case 256 + 2: launch_kjp<2, 4, PAT>(p, grid, lds, s); break;
    case 256 + 4: launch_kjp<4, 4, PAT>(p, grid, lds, s); break;
    case 256 + 8: launch_kjp<8, 4, PAT>(p, grid, lds, s); break;
    case 256 + 16: launch_kjp<16, 4, PAT>(p, grid, lds, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Curve-ring instance of (K, J) for level scalar-reserve portfolios.
template <int K, int J>
static void launch_kj_ring(const RecParams &p, int grid, size_t lds, hipStream_t s)
{
    const dim3 g(grid), b(WG_THREADS);
    if (p.q_in_lds)
        hipLaunchKernelGGL((k_recurrence<K, J, true, false, false, true>), g, b, lds, s, p, p.v, p.items, p.tiles, p.qbeg);
    else
        hipLaunchKernelGGL((k_recurrence<K, J, false, false, false, true>), g, b, lds, s, p, p.v, p.items, p.tiles, p.qbeg);
}

// Curve-ring instances (rr_kernels_ring.hip).
hipError_t launch_recurrence_ring(int K, int J, const RecParams &p, int grid, size_t lds_bytes,
                                  hipStream_t stream);

// Launch of the kernels with the payment-pattern paths (rr_kernels_pat.hip).
hipError_t launch_recurrence_pat(int K, int J, const RecParams &p, int grid, size_t lds_bytes,
                                 hipStream_t stream);

}  // namespace rr
