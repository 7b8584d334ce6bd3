// Internal declarations shared by the host side of the library (rr_host.cpp)
// and its device kernels (rr_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rr {

// State models a tile of 64 policies runs (Sec. 3.6.4: zero-reserve states
// removed).  Every policy in a tile shares its model.
enum Kind : int {
    KIND_SINGLE = 0,   // one life, scalar reserve (annuity, assurance, endowment)
    KIND_JOINT = 1,    // two lives, scalar reserve in state 00, p = px * py (joint-life
                       // annuity, two-life endowment, first-death assurance)
    KIND_REV = 2,      // two lives, states {00, 10} of the 4-state model
    KIND_LAST = 3,     // two lives, states {00, 01, 10} (last-survivor annuity,
                       // second-death assurance)
    N_KINDS = 4
};

constexpr int TILE = 64;          // policies per tile = lanes per wavefront
constexpr int N_COEF = 7;         // per-policy cash-flow coefficients
constexpr int MAX_QUEUES = 8;     // one work queue per XCD
#ifndef RR_WG_THREADS
#define RR_WG_THREADS 512   // eight wavefronts: two per SIMD, one work window per CU
#endif
constexpr int WG_THREADS = RR_WG_THREADS;   // wavefronts per workgroup x 64

// Per-policy coefficients (rows of coef[N_COEF][n_pad]):
//  KIND_SINGLE / KIND_JOINT:  0: a0 advance amount in state 0 (annuity due - premium;
//                                table policies: - premium)
//                             1: a1 arrears amount paid if alive at the end of the step
//                             2: b1 death benefit paid at the end of the step of death
//                             3: boundary reserve r_S of state 0
//  KIND_REV / KIND_LAST:      0/1: advance/arrears amount in state 00
//                             2/3: advance/arrears amount in state 01
//                             4/5: advance/arrears amount in state 10
//                             6: KIND_LAST: benefit on the second death (end of its step)
//  Markov tiles:              0: a0 = - premium (state 0), 1..4: amount x benefit of states 0..3
//                             (models of 5-9 states: 1: amount; benefits per model in mk_c)
//  three-life tiles:          0: advance amount - premium (all alive), 1: arrears amount,
//                             2: advance amount in the other states (last survivor)

// How a tile's cash flows vary in time.  Tiles other than level ones run
// one tile per item.
enum Flow : int {
    FLOW_LEVEL = 0,     // level amounts (coef rows)
    FLOW_PATTERN = 1,   // annuities in payment with escalation or annual payment
    FLOW_TABLE = 2,     // single life, cash flow of step t from a per-policy table
    FLOW_MARKOV = 3,    // one life on an uploaded Markov model (up to 9 states)
    FLOW_FRAC = 4,      // single- or joint-life annuity paid at a fraction of the month
    FLOW_THREE = 5      // annuity on three lives (KIND_JOINT: joint life, KIND_LAST: last survivor)
};
constexpr int N_FLOWS = 6;
constexpr int MAX_MK_STATES = 9;   // largest uploaded Markov model

struct Tile {
    int kind;
    int first;    // first sorted slot (multiple of TILE)
    int smax;     // largest remaining term at node 0 among valid lanes
    int smin;     // smallest remaining term at node 0 among valid lanes
    int flow;     // Flow
};

// Payment pattern of a slot in a pattern tile: the code packs the months to
// the first anniversary after node 0 (bits 0-7, 1..12), annual payment (bit 8)
// and the payment offset f (bit 9: 1 for arrears, payment at t + 1).  For a
// slot of a table tile the code is its column in the table array.
constexpr int PAT_ANNUAL = 1 << 8;
constexpr int PAT_ARREARS = 1 << 9;

struct Item {
    int node_rel;  // node - node_begin
    int tile;      // first tile of the item
    int sblock;    // first scenario of the block, relative to scen_begin
    int count;     // consecutive tiles of one model in the item (1..J)
};

struct RecParams {
    // basis
    const double *q;          // [n_tables][n_ages_stage] one-step survival p = 1 - q
    int n_ages_stage;
    int n_q;                  // n_tables * n_ages_stage
    int q_in_lds;
    int has_vector;           // some tile is KIND_REV or KIND_LAST
    const double *v;          // [n_nodes][n_steps][scen_pad] month-major
    int n_steps;
    int scen_pad;
    const double *shock;      // [n_nodes]: multiplier on q (1.0 when none)
    // portfolio, sorted and padded to whole tiles
    const int *age1;          // attained age at node 0 (padding: 0)
    const int *age2;
    const int *term;          // remaining term at node 0 (padding: 0)
    const int *qoff1;         // table1 * n_ages_stage
    const int *qoff2;
    const int *uidx;          // upload index, -1 for padding
    const double *coef;       // [N_COEF][n_pad]
    const double *pat_g;      // [n_pad] 1 + escalation rate (pattern tiles), or null
    const int *pat_code;      // [n_pad] anniversary / annual / timing code or table column, or null
    const double *cf_t;       // [cf_steps][cf_cols] amount x table value of the step, or null
    int cf_cols;
    const double *mk_w;       // [model][mk_ages][4][4] uploaded Markov matrices (zero padded),
                              // [model][mk_ages][9][9] for models of 5-9 states
    int mk_ages;
    int mk_states;
    const double *mk_c;       // [model][9] benefits per unit amount (models of 5-9 states)
    const int *age3;          // life 3 of three-life tiles (other slots: 0)
    const int *qoff3;
    const double *vf;         // v^frac, laid out as v (fractional tiles), or null
    double frac;
    int n_pad;
    int n_user;
    int ring_off;             // curve-ring launches: first double of the rings in LDS
    int path_lds;             // path output: first double of the wavefronts' stages in LDS
    const Tile *tiles;
    int n_tiles;
    // work
    const Item *items;
    const int *qbeg;          // [n_queues + 1]
    int *counters;            // [MAX_QUEUES + 1]: queue heads, then finished-workgroup count
    int n_queues;
    int win;                  // 1: workgroups take windows of WG_THREADS/64 items together
    // run
    int node_begin;
    int scen_begin;
    int scen_count;
    int node_step;
    // outputs
    double *r0;               // [node_count][n_user][scen_count][r0_states] or null
    int r0_states;
    double *partial;          // [node_count][n_tiles][scen_count] or null
    double *path;             // or null
    const long long *path_off;  // [n_user + 1] (path mode)
};

// Curve ring (level scalar-reserve portfolios): each wavefront stages the
// discount factors of its K scenarios in LDS, two chunks of RING_C steps.
constexpr int RING_C = 16;
constexpr int ring_doubles_per_wave(int K) { return 2 * RING_C * K; }

// Path output stage (one policy per lane): each wavefront keeps PATH_T steps
// of its 64 lanes in LDS, rows PATH_ROW doubles apart (PATH_ROW = 2 mod 32
// puts the 32 lanes of a half-wave read on distinct banks).
constexpr int PATH_T = 16;
constexpr int PATH_ROW = 66;
constexpr int PATH_STAGE_DOUBLES = PATH_T * PATH_ROW;

// Launchers (rr_kernels.hip).  All are asynchronous on `stream`.  ring: the
// curve-ring instances (supported_ring(K, J); no vector or pattern tiles;
// lds_bytes then includes the rings after the tables, at p.ring_off).
hipError_t launch_recurrence(int K, int J, const RecParams &p, int grid, size_t lds_bytes,
                             hipStream_t stream, bool ring = false);
bool supported_ring(int K, int J);
// scratch: totals_scratch_doubles(node_count, n_tiles, scen_count) doubles
// (may be null when that is 0).
hipError_t launch_totals(const double *partial, int node_count, int n_tiles, int scen_count,
                         double *totals, double *scratch, hipStream_t stream);
long long totals_scratch_doubles(int node_count, int n_tiles, int scen_count);
hipError_t launch_stats(const double *totals, int node_count, int scen_count, int rank,
                        double *stats, hipStream_t stream);
hipError_t launch_fill(double *dst, long long n, double value, hipStream_t stream);
hipError_t launch_fill_int(int *dst, int n, int value, hipStream_t stream);
hipError_t launch_transpose_curves(const double *src, double *dst, int n_nodes, int n_scen,
                                   int n_steps, int scen_pad, hipStream_t stream);
// dst[i] = src[i]^f for i < n.
hipError_t launch_pow_curves(const double *src, double *dst, long long n, double f,
                             hipStream_t stream);
// Vasicek scenario generation (rr_scen.hip).  Constants of the exact step
// (e = exp(-a dt), om = (1 - e)/a, the standard deviations and the
// correlation part) are computed on the host.
struct VasParams {
    double b, dt, e, om, sd_r, rho_sd_y, sd_y_perp;
    unsigned long long key0, key1;
    int n_nodes, n_scen, n_steps, scen_pad;
};
// work: vasicek_work_doubles(...) doubles (normals and short rates, month-
// major with stride scen_pad); r0: device [n_nodes]; v: month-major with
// stride scen_pad (the library's curves) or [node][scen][step]; r_out:
// [node][scen][step + 1] or null.
hipError_t launch_vasicek(const VasParams &P, const double *r0, double *work, double *v,
                          int month_major, double *r_out, hipStream_t stream);
size_t vasicek_work_doubles(int n_nodes, int n_scen, int n_steps, int scen_pad);
// Mean discount curve of the run's scenarios per node (rr_kernels.hip): D
// holds node_count * n_steps * scen_count doubles; vbar is [n_nodes][n_steps][64]
// with the curve at lane 0 of the run's nodes.
hipError_t launch_mean_curve(const double *v, int n_steps, int scen_pad, int node_begin,
                             int node_count, int scen_begin, int scen_count, double *D,
                             double *vbar, hipStream_t stream);
int max_lds_tables_doubles();
// Static device scratch of rr_reserve_recurrence_noalloc (rr_noalloc.hip):
// its device address on `device`, the current device (looked up once per
// device); NOALLOC_SCRATCH_BYTES is its size.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
hipError_t noalloc_scratch(int device, void **ptr);
bool supported_k(int K);
bool supported_kj(int K, int J);   // (scenarios, policies) per lane

}  // namespace rr
