/*
 * rr.h -- C ABI of the MI355X reserve-recurrence library.
 *
 * Computes prospective reserves of non-unit-linked life policies with the
 * general backward vector recurrence of Tucker & Bull, "An efficient
 * algorithm for the calculation of reserves for non-unit linked life
 * policies" (arXiv 1401.1757), Eq. (3.1):
 *
 *     r_t = v_t^f W_{t,f} c_t + v_t W_{t,1} r_{t+1},
 *
 * run backward from a boundary condition (Sec. 3.8.2), for every policy x
 * scenario (x outer node), in FP64 on one gfx950 GPU.  W is built on the
 * device from the per-life monthly death probabilities (Sec. 3.5, Sec. 4),
 * v from the uploaded scenario discount curves (Sec. 3.4), c from each
 * policy's product, amounts and timing (Sec. 3.3, Sec. 4).  Zero-reserve
 * states are dropped as in Sec. 3.6.4; their outputs are exactly 0.
 *
 * Conventions used by every call:
 *   - monthly steps; step t covers [t, t+1) months after the valuation node;
 *     the reserve r_t is held at time t, before the premium due at t;
 *   - premiums are paid in advance (f = 0) while every life is alive;
 *     annuity payments at f = 0 (RR_ADVANCE) or f = 1 (RR_ARREARS); death
 *     benefits at the end of the month of death (f = 1);
 *   - transition matrices are row = state at the start of the step; states
 *     use the binary (two-state lives) or ternary (assurances) labels of
 *     Sec. 2.4.2 and Sec. 4.1.3, life 1 being the most significant digit;
 *   - at outer node k (0-based) every life is 12*k months older (node_step_m
 *     months per node), the remaining term is term_m - k*node_step_m and the
 *     node's curves and mortality shock apply; policies whose remaining term
 *     is <= 0 at a node have expired: their outputs are 0 and they are left
 *     out of totals.
 *
 * Ownership: uploads copy what they are given (host or device memory) into
 * library-owned device memory; the caller may free its buffers on return.
 * Output buffers of rr_reserve_recurrence / rr_surrogate_infer are
 * caller-owned device memory (e.g. torch tensors), written asynchronously
 * on the context's stream.
 *
 * Errors: every call returns an rr_status; no exception crosses the ABI.  On
 * error, rr_last_error(ctx) gives a message naming the first bad argument or
 * policy index, valid until the next call on the context.  A context must
 * not be used from two host threads at once; calls on one context that
 * overlap on the GPU (different streams) race.
 */
#ifndef RR_H
#define RR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rr_ctx rr_ctx;

/* Status codes. */
#define RR_OK       0
#define RR_EINVAL  (-1)   /* invalid argument or input data */
#define RR_ENOMEM  (-2)   /* device or host allocation failed */
#define RR_EDEVICE (-3)   /* HIP runtime error */
#define RR_ERANGE  (-4)   /* output buffer too small / size limit exceeded */
#define RR_ESTATE  (-5)   /* call out of order (no basis, portfolio or model) */

/* Products (Sec. 4).  Amount = annual annuity (paid amount/12 each month)
 * for the annuities, sum assured otherwise. */
#define RR_SL_ANN       0  /* single-life annuity, 2-state model (Sec. 4.1.1) */
#define RR_JL_ANN       1  /* joint-life annuity, 4-state model, c = (1,0,0,0) (Sec. 4.2.1 b) */
#define RR_REV_ANN      2  /* reversionary annuity to life 2 after life 1 dies, c = (0,0,1,0) (Sec. 4.2.1 a) */
#define RR_LS_ANN       3  /* last-survivor annuity, c = (1,1,1,0) (Sec. 4.2.1 c) */
#define RR_TERM         4  /* term assurance, 3-state model, c = (0,1,0), r_S = 0 (Sec. 4.1.3) */
#define RR_ENDOW        5  /* pure endowment, boundary r_S = (SA, 0) (Sec. 4.1.2) */
#define RR_ENDOW_ASSUR  6  /* endowment assurance: term assurance with r_S = (SA, 0, 0) */
#define RR_CF_TABLE     7  /* one life, 2-state model; pays amount x cf[cf_row][T] at the end of
                              month T (months since node 0) if alive, level premium in advance,
                              r_S = 0 (Sec. 4.6: c_t holds the nominal amounts) */
#define RR_JL_ENDOW     8  /* two-life pure endowment: SA at the end of the term if both lives are
                              alive, r_S = (SA, 0, 0, 0) (Sec. 4.2.2) */
#define RR_JL_ASSUR1    9  /* two-life term assurance, SA at the end of the month of the first
                              death, 9-state model, c = (0,1,0,1,1,0,0,0,0) SA (Sec. 4.2.3) */
#define RR_JL_ASSUR2   10  /* two-life term assurance, SA at the end of the month of the second
                              death, c = (0,0,0,0,1,1,0,1,0) SA (Sec. 4.2.3).  Premiums of the
                              two-life products are paid while both lives are alive.  With
                              RR_OUT_ALL_STATES the 9-state reserves are reported as (both alive,
                              life 1 only, life 2 only, none). */

#define RR_MARKOV      11  /* one life on an uploaded Markov model (rr_markov_upload; table1 =
                              model, age1_m indexes its tables): starts in state 0, pays
                              amount x benefit[state] at the end of each month that ends in
                              that state, premium in advance while in state 0, r_S = 0
                              (Sec. 4.5: reversible models, W not upper triangular).  The
                              node shock does not apply to uploaded models.  With
                              RR_OUT_ALL_STATES slot j is the reserve of state j. */

#define RR_JL3_ANN     12  /* joint-life annuity on three lives, paid while all three are alive:
                              the 2^3 = 8-state Kronecker model of Sec. 4.3, c = e_0 (binary labels,
                              life 1 the high digit, 1 = dead); needs age3_m and table3 */
#define RR_LS3_ANN     13  /* last-survivor annuity on three lives, paid while any is alive,
                              c = (1,1,1,1,1,1,1,0) (Sec. 4.3).  Three-life annuities are level
                              (no payment pattern) and paid in advance or in arrears; with
                              RR_OUT_ALL_STATES slot j is the reserve of state j (0: all alive,
                              1: life 3 dead, 2: life 2 dead, 3: lives 2 and 3 dead). */

#define RR_ADVANCE 0       /* annuity paid at the start of each month (f = 0) */
#define RR_ARREARS 1       /* annuity paid at the end of each month (f = 1) */
#define RR_FRACTIONAL 2    /* annuity paid at the basis's fraction frac of each month
                              (0 < frac < 1): survival to t + frac by frac x the month's death
                              probability (uniform deaths), discount v^frac (Sec. 3.1's f).
                              RR_SL_ANN and RR_JL_ANN without payment patterns only. */

#define RR_HOST   0        /* input arrays are in host memory */
#define RR_DEVICE 1        /* input arrays are in device memory */

/* Output selection for rr_run.out_mask. */
#define RR_OUT_R0          1u   /* reserve at t = 0 per (node, policy, scenario) */
#define RR_OUT_TOTALS      2u   /* portfolio total per (node, scenario) */
#define RR_OUT_PATH        4u   /* state-0 reserve at every t (one node, one scenario) */
#define RR_OUT_ALL_STATES  8u   /* with RR_OUT_R0: all 4 state slots, not just state 0 */
#define RR_OUT_STATS      16u   /* per-node mean and tail quantile of the totals */

/*
 * Valuation basis: mortality tables and scenario discount curves.
 *   q[n_tables][n_ages]      monthly death probability by attained age in whole
 *                            months, 0 <= q <= 1 (Sec. 3.5, 3.7.3).
 *   v[n_nodes][n_scen][n_steps]  one-step discount factor of month t for the
 *                            scenario's interest path, 0 < v, finite
 *                            (Sec. 3.4, 3.7.2: any interest model).
 *   shock[n_nodes] or NULL   per-node multiplier m >= 0 on every q (capped at 1).
 */
typedef struct {
    int32_t n_tables;
    int32_t n_ages;
    const double *q;
    int32_t n_nodes;
    int32_t n_scen;
    int32_t n_steps;
    const double *v;
    const double *shock;
    int32_t mem_kind;        /* RR_HOST or RR_DEVICE, for all three arrays */
    double frac;             /* payment point of RR_FRACTIONAL annuities, in (0, 1); 0 = none.
                                The library keeps v^frac beside v (8 bytes per curve value). */
} rr_basis;

/*
 * Portfolio, structure of arrays of length n (n >= 0).  age2_m/table2 are read
 * for two-life products only.  timing may be NULL (all RR_ARREARS); premium
 * may be NULL (all 0).  Requirements: 1 <= term_m <= n_steps of the basis,
 * age + term_m <= n_ages - 1 for every life used, valid table indices, finite
 * amount and premium >= 0.
 *
 * Annuity payment patterns (the representative annuity portfolio, Sec. 5.3),
 * three optional arrays, each NULL for "none":
 *   escalation[i]  yearly escalation rate e >= 0 (finite, at most 1);
 *   anniv_m[i]     months from node 0 to the next policy anniversary, 1..12
 *                  (NULL: 12); further anniversaries follow every 12 months;
 *   annual[i]      1 = the amount is paid once a year, at each anniversary;
 *                  0 = amount / 12 every month.
 * A payment at time T (months after node 0; T = t for RR_ADVANCE and t + 1 for
 * RR_ARREARS in step t) is the level payment times (1+e)^n(T), n(T) the number
 * of anniversaries in (0, T]; an annual payer pays 12 level monthly payments
 * times that factor at an anniversary and nothing in other months.  A policy
 * with e > 0 or annual = 1 is "patterned": it must be an annuity (RR_SL_ANN,
 * RR_JL_ANN, RR_REV_ANN, RR_LS_ANN) in payment, i.e. with premium 0; anything
 * else is RR_EINVAL.  Level policies ignore anniv_m (values must still be in
 * range).  Patterned policies are outside the surrogate's domain and take its
 * exact fallback.
 */
typedef struct {
    int32_t n;
    const int32_t *product;
    const int32_t *age1_m;   /* attained age of life 1 at node 0, months */
    const int32_t *age2_m;   /* attained age of life 2 at node 0, months */
    const int32_t *term_m;   /* remaining term at node 0, months */
    const int32_t *table1;
    const int32_t *table2;
    const int32_t *timing;   /* RR_ADVANCE / RR_ARREARS */
    const double *amount;
    const double *premium;   /* level monthly premium, paid in advance */
    int32_t mem_kind;        /* RR_HOST or RR_DEVICE, for all arrays */
    const double *escalation;   /* or NULL: payment patterns, see above */
    const int32_t *anniv_m;     /* or NULL */
    const int32_t *annual;      /* or NULL */
    /* Cash-flow tables of RR_CF_TABLE policies (NULL/0 when there are none):
     * cf[cf_n_rows][cf_len] cash flows per unit amount, finite; policy i uses
     * row cf_row[i] (0 <= row < cf_n_rows) and needs term_m[i] <= cf_len.  The
     * library keeps amount x row values per policy and month in device memory
     * (8 bytes x policies x longest term). */
    const int32_t *cf_row;
    const double *cf;
    int32_t cf_n_rows;
    int32_t cf_len;
    /* Life 3 of RR_JL3_ANN / RR_LS3_ANN policies (NULL when there are none):
     * attained age at node 0 in months and mortality table. */
    const int32_t *age3_m;
    const int32_t *table3;
} rr_portfolio;

/* One valuation run over nodes [node_begin, node_begin + node_count) and
 * scenarios [scen_begin, scen_begin + scen_count) of the uploaded basis. */
typedef struct {
    int32_t node_begin;
    int32_t node_count;
    int32_t scen_begin;
    int32_t scen_count;
    int32_t node_step_m;     /* months between consecutive nodes (12 for annual) */
    uint32_t out_mask;       /* RR_OUT_* */
    double tail;             /* RR_OUT_STATS: quantile tail, e.g. 0.005 -> ceil(0.005 K)-th largest */
} rr_run;

/*
 * Caller-owned device outputs (NULL = not wanted; must be non-NULL when the
 * matching out_mask bit is set).
 *   r0[node_count][n][scen_count][S]  S = 4 with RR_OUT_ALL_STATES else 1;
 *                                     policies in upload order.
 *   totals[node_count][scen_count]    sum of state-0 reserves of live policies.
 *   path[sum_i (max(S_i,0) + 1)]      RR_OUT_PATH (node_count = scen_count = 1):
 *                                     policy i, step t at offset
 *                                     off_i + t, off_i = sum_{j<i}(max(S_j,0)+1),
 *                                     S_i = term_i - node*node_step_m (a policy
 *                                     expired at the node has one entry, 0);
 *                                     path_cap is its length in doubles.
 *   stats[node_count][2]              RR_OUT_STATS: mean over scenarios and the
 *                                     ceil(tail*scen_count)-th largest total.
 */
typedef struct {
    double *r0;
    double *totals;
    double *path;
    int64_t path_cap;
    double *stats;
} rr_outputs;

/* Context bound to one device and one HIP stream (0 = the null stream).  The
 * stream may be torch.cuda.current_stream().cuda_stream.  rr_create returns
 * RR_EDEVICE when no GPU is present. */
int rr_create(rr_ctx **out, int device, uint64_t stream);
int rr_destroy(rr_ctx *ctx);
const char *rr_last_error(const rr_ctx *ctx);
int rr_set_stream(rr_ctx *ctx, uint64_t stream);
int rr_sync(rr_ctx *ctx);   /* waits for the context's stream */

/* Host-only validation (no device work); msg receives the reason. */
int rr_check_basis(const rr_basis *b, char *msg, size_t msg_len);
int rr_check_portfolio(const rr_portfolio *p, int32_t n_steps, int32_t n_ages,
                       int32_t n_tables, char *msg, size_t msg_len);

/* Copy the basis into device memory (curves re-laid out month-major so a
 * wavefront reads consecutive scenarios of one month).  Replaces any
 * previous basis.  A loaded portfolio that the new basis does not cover
 * (terms, ages or table indices) is dropped: rr_reserve_recurrence then
 * returns RR_ESTATE until a portfolio is uploaded again. */
int rr_basis_upload(rr_ctx *ctx, const rr_basis *b);

/* Copy, check, sort (by state model, payment pattern, remaining term
 * descending, age) and tile the portfolio (Sec. 3.8.2's per-policy inputs; the
 * paper balances uneven terms with a dynamic schedule, Sec. 5.1.1). */
int rr_portfolio_upload(rr_ctx *ctx, const rr_portfolio *p);

/*
 * Interest scenarios generated on the device (Sec. 3.4 and 3.7.2 leave the
 * interest model open; this is the Vasicek short rate dr = a (b - r) dt +
 * sigma dW).  Scenario s of node k starts from r0[k]; over each step of dt
 * years the short rate r and its integral Y are drawn from their exact joint
 * Gaussian law given r at the start of the step, and the step's discount
 * factor is v = exp(-Y).  The two normals of (node k, scenario s, step t) are
 * the Box-Muller transform of the uniforms ((x >> 11) + 0.5) 2^-53 of the
 * first two words x of the Philox4x64-10 block with counter (t, s, k, 0) under
 * `key`, so a scenario's numbers do not depend on how many are drawn.
 */
typedef struct {
    double a;            /* mean-reversion speed, > 0 */
    double b;            /* long-run mean, finite */
    double sigma;        /* volatility, >= 0 */
    double dt;           /* years per step, > 0 (1/12: monthly) */
    const double *r0;    /* host [n_nodes] short rate at the start of each node */
    uint64_t key[2];     /* Philox4x64-10 key */
} rr_vasicek;

/* Install a basis whose curves are generated on the device: q, shock and
 * the sizes come from b (b->v must be NULL), the curves from vs.  Otherwise
 * as rr_basis_upload (synchronous; drops a portfolio the basis does not
 * cover). */
int rr_basis_generate_vasicek(rr_ctx *ctx, const rr_basis *b, const rr_vasicek *vs);

/* Regenerate the installed basis's curves in place (same sizes), e.g. for the
 * next outer node of a nested valuation: asynchronous on the context's stream;
 * portfolio, plans and captured graphs stay valid.  Waits for the stream only
 * when vs->r0 differs from the values of the previous generation. */
int rr_curves_generate_vasicek(rr_ctx *ctx, const rr_vasicek *vs);

/* The curves of a generator in caller-owned device memory (asynchronous):
 * v[n_nodes][n_scen][n_steps] and, if r is not NULL, the short rates
 * r[n_nodes][n_scen][n_steps + 1] (r[..][0] = r0). */
int rr_vasicek_curves(rr_ctx *ctx, const rr_vasicek *vs, int32_t n_nodes, int32_t n_scen,
                      int32_t n_steps, double *v, double *r);

/*
 * Markov models for RR_MARKOV policies (Sec. 4.5), copied to the device:
 *   w[n_models][n_ages][n_states][n_states]  one-month transition probabilities
 *       by attained age in months; row i = state at the start of the month;
 *       entries in [0, 1], each row summing to 1 within 1e-12;
 *   benefit[n_models][n_states]  paid per unit amount at the end of a month
 *       that ends in the state (finite).
 * 2 <= n_states <= 9 (e.g. the 9-state two-life model of Sec. 4.2.3 by the
 * attained age of life 1), n_ages >= 2, n_models >= 1.  Replaces earlier models;
 * a loaded portfolio that the new models do not cover is dropped.
 */
typedef struct {
    int32_t n_models;
    int32_t n_states;
    int32_t n_ages;
    const double *w;
    const double *benefit;
    int32_t mem_kind;
} rr_markov;
int rr_markov_upload(rr_ctx *ctx, const rr_markov *m);

/* Length in doubles of the RR_OUT_PATH buffer for a node. */
int rr_path_size(rr_ctx *ctx, int32_t node, int32_t node_step_m, int64_t *n_out);

/*
 * The hot call: the backward recurrence, Eq. (3.1), for every policy x
 * scenario x node of the run, from the boundary condition at the end of each
 * term (Sec. 4.1.1-4.2.1) down to t = 0 (Sec. 3.8.2), plus the requested
 * reductions.  Asynchronous on the context's stream.  RR_ESTATE without a
 * basis and a portfolio; RR_ERANGE if path_cap is too small.
 */
int rr_reserve_recurrence(rr_ctx *ctx, const rr_run *run, const rr_outputs *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * it): rr_reserve_recurrence with the same run, outputs and results, except
 * that it allocates nothing.  Its work lists, queue counters and partial
 * totals live in one static device array of 64 MiB per GPU, which every call
 * on that GPU shares (from any context) and which is held until the process
 * ends.  Consequences:
 *   - a run whose scratch exceeds 64 MiB is RR_ERANGE (the partial totals take
 *     8 bytes x nodes x tiles of 64 policies x scenarios when totals or
 *     statistics are requested: e.g. 10,000 policies x 60 nodes x 500
 *     scenarios fits, 500,000 policies x 1,000 scenarios does not);
 *   - calls that overlap on one GPU (two streams, or two host threads) race on
 *     the array: the caller serialises them;
 *   - RR_OUT_PATH is RR_EINVAL (its offsets need an upload);
 *   - no autotuning (it builds and uploads candidate plans): the launch shape
 *     is the pinned options, else the shape an earlier rr_reserve_recurrence
 *     call chose for this run shape, else K = 16, J = 2, one workgroup per CU;
 *   - no graph replay and no kernel timing; the work lists are copied from
 *     host memory the context keeps on every call (a few tens of KB).
 * The basis and portfolio uploads still allocate: call them beforehand.
 */
int rr_reserve_recurrence_noalloc(rr_ctx *ctx, const rr_run *run, const rr_outputs *out);

/* Options (rr_set_option). */
#define RR_OPT_BLOCK_K      1   /* scenarios per lane: 0 = autotune, or 1,2,4,8,16,32 */
#define RR_OPT_WG_PER_CU    2   /* persistent workgroups per CU: 0 = autotune, 1..8 */
#define RR_OPT_USE_GRAPH    3   /* 1 = replay captured hipGraphs (default), 0 = direct launches */
#define RR_OPT_KERNEL_TIMING 4  /* 1 = record HIP events around each recurrence kernel
                                   (and each fused surrogate inference kernel) */
#define RR_OPT_XCD_QUEUES   5   /* 1 = per-XCD work queues with stealing (default), 0 = one queue */
#define RR_OPT_LAST_K       6   /* read-only: scenarios per lane of the last launch */
#define RR_OPT_LAST_WG      7   /* read-only: workgroups per CU of the last launch */
#define RR_OPT_BLOCK_J      8   /* policies per lane (scalar-reserve models): 0 = autotune, 1, 2, 4 */
#define RR_OPT_LAST_J       9   /* read-only: policies per lane of the last launch */
#define RR_OPT_TERM_BUCKET 10   /* months per remaining-term bucket when tiling (default 4);
                                   applies from the next rr_portfolio_upload */
#define RR_OPT_CURVE_RING  11   /* level single-/joint-life portfolios: stage each wavefront's
                                   scenario curves in an LDS ring (-1 = autotune, 0 = off
                                   (default), 1 = on for the shapes that have it: K = 16 with
                                   J = 1, 2 and K = 8 with J = 2) */
#define RR_OPT_LAST_RING   12   /* read-only: 1 if the last launch used the curve ring */
#define RR_OPT_LANE_SPREAD 13   /* 1 = order the lanes of each tile so that their mortality-table
                                   reads spread over the LDS banks (default), 0 = sorted order;
                                   applies from the next rr_portfolio_upload */
#define RR_OPT_CURVE_SHARE 14   /* 2 = order each work queue in windows of one item per
                                   wavefront of a workgroup, of one scenario block and about the
                                   same length, each workgroup taking a window with one atomic and
                                   running its items together, so that its wavefronts read the same
                                   curve lines; 1 = the same order, items taken one by one; 0 =
                                   plain longest-first order; -1 = 2 or 1, whichever the autotuner
                                   finds faster (default) */
#define RR_OPT_LAST_WINDOWS 15  /* read-only: 1 if the last launch took windows per workgroup */
#define RR_OPT_LAST_TABLES_LDS 16  /* read-only: 1 if the last launch staged the survival tables in
                                   LDS, 0 if it read them from device memory (bases whose tables
                                   exceed 64 KiB) */
int rr_set_option(rr_ctx *ctx, int32_t option, int64_t value);
int rr_get_option(rr_ctx *ctx, int32_t option, int64_t *value);

/* Durations (ms) of the recurrence kernels launched since the previous call,
 * recorded when RR_OPT_KERNEL_TIMING is on; waits for them to finish. */
int rr_kernel_times(rr_ctx *ctx, double *ms, int32_t cap, int32_t *count);

/* ------------------------------------------------------------------------
 * Learned reserve surrogate.  Not part of the paper's method: a multilayer
 * perceptron fitted on the GPU to reserves that rr_reserve_recurrence
 * computes, inferred with the exact FP64 recurrence as fallback for inputs
 * outside its training box.
 *
 * Features of a row (node k, scenario s, policy i, reserve-vector state j),
 * raw values in FP64:
 *    0 age of life 1 in years at the node, (age1_m + k node_step_m) / 12
 *    1 remaining term in years, (term_m - k node_step_m) / 12
 *    2..5 one-hot of the product: single-life annuity, joint-life annuity,
 *         term assurance, pure endowment (other products are outside the
 *         model's domain)
 *    6 log amount;  7 annual premium per unit amount, 12 premium / amount
 *    8 short rate -12 log v[k][s][0]
 *    9..11 scores of the scenario's zero-rate curve on the model's three
 *         principal components; zero rates at tenors T = 1..50 years are
 *         z_T = -(12 / m_T) sum_{t < m_T} log v[k][s][t], m_T = min(12 T, n_steps)
 *   12 mortality shock of the node (1 without shocks)
 *   13..15 one-hot of the state j (0, 1, 2)
 *   16 age of life 2 in years at the node (joint-life annuity; else 0)
 * Target: reserve of state j / amount.  Features are standardised with the
 * training mean and population standard deviation, the target with those of
 * the training rows of the same product.
 * A row is inside the box when every raw feature lies within the training
 * [min, max] and the policy's tables and annuity timing are those the
 * training policies of its product had.
 *
 * Network: 32 inputs (features, zero-padded) -> 256 -> GELU -> 256 -> GELU
 * -> 1, GELU in the tanh form (Hendrycks and Gimpel, 2016); weights and
 * activations bfloat16 (round to nearest even), sums FP32 (MFMA); FP32
 * master weights updated by Adam (beta 0.9, 0.999, eps 1e-8); loss = mean
 * squared error of the standardised target.
 * ------------------------------------------------------------------------ */

#define RR_SG_FEATURES 17
#define RR_SG_INPUTS   32
#define RR_SG_HIDDEN   256
#define RR_SG_TENORS   50
#define RR_SG_FACTORS  3
/* FP32 parameter vector: W1[32][256] (input, unit), b1[256], W2[256][256]
 * (unit in, unit out), b2[256], W3[256], b3. */
#define RR_SG_PARAMS   74497

typedef struct {
    rr_run run;              /* the samples: every live (node, scenario, policy,
                                state) of this run of the loaded basis and
                                portfolio, states 0-2 for joint-life annuities
                                and 0 otherwise; out_mask and tail are ignored */
    int32_t epochs;          /* >= 1 */
    int32_t batch;           /* rows per Adam step, multiple of 64 */
    float lr;                /* Adam step size at the first step (> 0) */
    float lr_final;          /* cosine decay to this at the last step (>= 0) */
    float holdout;           /* fraction of samples held out, in [0, 0.5] */
    int32_t init;            /* 1: new weights from seed and new standardisation,
                                curve factors and box from these samples;
                                0: continue training the loaded model on them */
    uint64_t seed;           /* weight initialisation and sample order */
} rr_train_cfg;

typedef struct {
    int64_t n_samples;
    int64_t n_train;         /* a multiple of batch; the rest is the holdout */
    int64_t n_holdout;
    int32_t steps;
    float first_loss;        /* mean loss over the first epoch */
    float final_loss;        /* mean loss over the last epoch */
    float holdout_loss;      /* loss on the holdout after the epochs */
    float calibration[4];    /* per one-hot product: mean residual of the trained
                                network over the training rows (standardised
                                units), added to the product's target mean */
    double data_ms;          /* exact reserves, features, statistics, dataset */
    double train_ms;         /* epochs */
} rr_train_report;

typedef struct {
    int64_t n_in_range;      /* (node, scenario, policy) rows from the network */
    int64_t n_fallback;      /* live rows from the exact recurrence */
} rr_infer_report;

/*
 * Train on the GPU (synchronous).  Samples come from the exact recurrence
 * (rr_reserve_recurrence's kernels) on cfg->run; features, the principal
 * components of the curves (fitted on the host from the device-computed
 * zero rates), standardisation, the bfloat16 MFMA forward and backward
 * kernels and Adam run on the device.  After the epochs each product's
 * target mean is shifted by the network's mean residual over that product's
 * training rows (an output calibration; see rr_train_report.calibration).  RR_ESTATE without a basis and a
 * portfolio (or, with init = 0, without a model); RR_EINVAL for bad
 * settings, for fewer samples than one batch, or when the training policies
 * of one product use several (table, timing) combinations.
 */
int rr_surrogate_train(rr_ctx *ctx, const rr_train_cfg *cfg, rr_train_report *rep);

/*
 * Model blob, little-endian: a 96-byte header (char magic[8] = "RRSURR01";
 * int32 version = 1, features = 17, inputs = 32, hidden = 256, tenors = 50,
 * factors = 3, params = 74497, adam_step, signature[4][3] = per one-hot
 * product (table1, table2 or -1, timing or -1; table1 = -1: product not
 * trained), 2 reserved), then FP64 mean[17], sd[17], lo[17], hi[17],
 * target_mean[4], target_sd[4] (per one-hot product), curve_mean[50],
 * components[3][50], then FP32
 * params[74497], adam_m[74497], adam_v[74497].  get_weights writes the
 * blob to host memory (bytes >= *needed, else RR_ERANGE with *needed set;
 * host may be NULL to query); set_weights loads one (RR_EINVAL if malformed).
 */
int rr_surrogate_get_weights(rr_ctx *ctx, void *host, size_t bytes, size_t *needed);
int rr_surrogate_set_weights(rr_ctx *ctx, const void *host, size_t bytes);

/*
 * Same outputs as rr_reserve_recurrence for RR_OUT_R0 (state 0),
 * RR_OUT_TOTALS and RR_OUT_STATS: rows inside the box from the network
 * (FP32 prediction, scaled back in FP64), the others from the exact FP64
 * recurrence; expired policies 0.  Waits for the range flags on the first
 * call of a run shape.  RR_ESTATE without a model, basis or portfolio.
 * rep may be NULL.
 */
int rr_surrogate_infer(rr_ctx *ctx, const rr_run *run, const rr_outputs *out,
                       rr_infer_report *rep);

/*
 * Node-level surrogate (not in the paper): the reserve of each policy
 * averaged over a node's scenarios, predicted by the same network from the
 * policy features and the node's scenario features averaged over its
 * scenarios (short rate, curve scores, shock; state 0) -- a regression of
 * inner-scenario averages on the node's risk factors, for nested valuations
 * where one expected reserve per node replaces its inner recurrences.
 *   train:  as rr_surrogate_train, on one row per live (node, policy) of
 *           cfg->run: the state-0 reserve averaged over the run's scenarios
 *           (exact recurrence) per unit amount.  Own model slot; blob as for
 *           rr_surrogate_get_weights with magic "RRSURN01".
 *   infer:  for the run's nodes, node_r0[node_count][n] (upload order) and
 *           node_totals[node_count] (sum over policies, fixed order), device
 *           memory, either may be NULL.  Rows of policies and nodes inside
 *           the training box come from the network, the others are exact
 *           (rr_node_expected_reserves); expired policies 0.  rep counts
 *           (node, policy) rows (may be NULL).
 */
int rr_node_surrogate_train(rr_ctx *ctx, const rr_train_cfg *cfg, rr_train_report *rep);

/*
 * The exact scenario average of every reserve at the run's nodes, by the
 * linearity of Eq. (3.5) in the discount products D_t = v_0 ... v_{t-1}
 * (mortality does not depend on the interest path and the cash flows are
 * fixed in advance): the reserve on the curve whose products are the means of
 * D_t over the run's scenarios.  One recurrence per (node, policy) instead of
 * scen_count.  node_r0[node_count][n] and node_totals[node_count] (device,
 * either may be NULL), asynchronous on the context's stream; run->out_mask
 * and run->tail are ignored.  The node-level surrogate below predicts the same
 * quantity.
 */
int rr_node_expected_reserves(rr_ctx *ctx, const rr_run *run, double *node_r0, double *node_totals);
int rr_node_surrogate_infer(rr_ctx *ctx, const rr_run *run, double *node_r0, double *node_totals,
                            rr_infer_report *rep);
int rr_node_surrogate_get_weights(rr_ctx *ctx, void *host, size_t bytes, size_t *needed);
int rr_node_surrogate_set_weights(rr_ctx *ctx, const void *host, size_t bytes);

/*
 * Layer-level calls on the loaded model (device pointers, asynchronous on
 * the context's stream):
 *   forward:   y[n] = network(z[n][32]) for standardised inputs z (FP32,
 *              rounded to bfloat16 inside);
 *   gradients: grad[RR_SG_PARAMS] of the mean squared error over the n rows
 *              against targets t[n]; loss[1] (may be NULL) = that error;
 *   adam_step: one Adam step of the FP32 master weights with gradient grad;
 *   features:  raw policy features pol[node_count][n][9] (features 0-7 and
 *              16), raw scenario features scen[node_count][scen_count][5]
 *              (features 8-12), policy flags pflag[node_count][n] (1 inside
 *              the box, 0 outside, 2 expired) and scenario flags
 *              sflag[node_count][scen_count] (1 inside); any may be NULL.
 */
int rr_surrogate_forward(rr_ctx *ctx, const float *z, int64_t n, float *y);
int rr_surrogate_gradients(rr_ctx *ctx, const float *z, const float *t, int64_t n,
                           float *grad, float *loss);
int rr_surrogate_adam_step(rr_ctx *ctx, const float *grad, float lr);
int rr_surrogate_features(rr_ctx *ctx, const rr_run *run, double *pol, double *scen,
                          int32_t *pflag, int32_t *sflag);

#ifdef __cplusplus
}
#endif

#endif /* RR_H */
