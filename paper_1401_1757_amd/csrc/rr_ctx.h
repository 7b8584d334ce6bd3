// Host-side context of the library, shared by the C ABI implementation
// (rr_host.cpp) and the surrogate runtime (rr_surrogate.cpp).
#pragma once

#include "rr.h"
#include "rr_internal.h"
#include "rr_surrogate.h"

#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

namespace rr {
namespace host {

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t count)
    {
        if (count <= n && p) return hipSuccess;
        release();
        if (count == 0) count = 1;
        hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
        if (e == hipSuccess) n = count;
        else p = nullptr;
        return e;
    }
};

struct Plan {
    int K = 1;
    int J = 1;
    int wg_per_cu = 2;
    int ring = 0;       // launch with the curve-ring instances
    int win = 0;        // workgroups take their windows of items together
    int grid = 1;
    int n_items = 0;
    int n_queues = 1;
    DevBuf<Item> items;
    DevBuf<int> qbeg;
    // Work lists and queue counters in memory the plan does not own (the
    // static scratch of the allocation-free entry point); used instead of
    // items/qbeg and the context's counters when set.
    const Item *items_ext = nullptr;
    const int *qbeg_ext = nullptr;
    int *counters_ext = nullptr;
};

// A plan's work lists on the host (the allocation-free entry point copies
// them into its static scratch on every call).
struct HostPlan {
    std::vector<Item> items;
    std::vector<int> qbeg;
};

struct PlanKey {
    int node_begin, node_count, scen_begin, scen_count, node_step, K, J, queues, gen, wg;
    bool operator<(const PlanKey &o) const
    {
        return std::tie(node_begin, node_count, scen_begin, scen_count, node_step, K, J, queues, gen,
                        wg) < std::tie(o.node_begin, o.node_count, o.scen_begin, o.scen_count,
                                       o.node_step, o.K, o.J, o.queues, o.gen, o.wg);
    }
};

struct LaunchCfg {
    int K = 1, J = 1, wg = 2;
    int ring = 0;       // curve-ring instances (level scalar-reserve portfolios)
    int win = 0;        // workgroups take windows of items together (one atomic per window)
};

struct TuneKey {
    int node_count, scen_count, r0_states, has_path, gen;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(node_count, scen_count, r0_states, has_path, gen) <
               std::tie(o.node_count, o.scen_count, o.r0_states, o.has_path, o.gen);
    }
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> key;
};

}  // namespace host
}  // namespace rr

// The context is a global-namespace type (the C ABI declares it opaque).
using rr::host::DevBuf;
using rr::host::GraphEntry;
using rr::host::LaunchCfg;
using rr::host::Plan;
using rr::host::PlanKey;
using rr::host::TuneKey;
using rr::Item;
using rr::Tile;

struct rr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::string err;
    int n_cu = 256;
    size_t lds_per_block = 65536;
    size_t lds_per_cu = 65536;           // LDS of one CU (resident workgroups x their LDS)

    // basis
    bool has_basis = false;
    int n_tables = 0, n_ages = 0, n_nodes = 0, n_scen = 0, n_steps = 0, scen_pad = 0;
    std::vector<double> q_host;          // [n_tables][n_ages]
    DevBuf<double> v;                    // [n_nodes][n_steps][scen_pad]
    DevBuf<double> shock;                // [n_nodes]
    double frac = 0.0;                   // payment point of fractional annuities (0: none)
    DevBuf<double> vf;                   // v^frac, laid out as v
    DevBuf<double> q_stage;              // [n_tables][n_ages_stage]
    DevBuf<double> vas_work;             // normals and short rates of the generator
    DevBuf<double> mean_D, mean_v;       // scenario-mean discount products and curve
    const double *v_override = nullptr;  // curves read instead of v (stride pad_override)
    int pad_override = 0;
    DevBuf<double> vas_r0;               // [n_nodes] start rates on the device
    std::vector<double> vas_r0_host;     // their values (the last generation's)
    int n_ages_stage = 0;
    std::vector<double> shock_host;

    // portfolio
    bool has_pf = false;
    int n_user = 0, n_pad = 0, n_tiles = 0;
    int max_age_needed = 0;
    int head_pad = 0;                     // largest ragged head of an item (steps)
    std::vector<int32_t> h_product, h_age1, h_age2, h_term, h_table1, h_table2, h_timing;
    std::vector<int32_t> h_age3, h_table3;   // life 3 (0 for other products)
    std::vector<double> h_amount, h_premium;
    std::vector<int32_t> h_patterned;     // 1: escalating or annual annuity
    std::vector<Tile> tiles_host;
    std::vector<int> slot_of_user;       // user index -> sorted slot
    DevBuf<int> age1, age2, term, qoff1, qoff2, uidx;
    DevBuf<int> age3, qoff3;              // life 3 of three-life tiles (0 elsewhere)
    DevBuf<double> coef;
    DevBuf<double> pat_g;                 // [n_pad] (with pattern or table tiles)
    DevBuf<int> pat_code;
    DevBuf<double> cf_t;                  // [cf_steps][cf_cols] (table tiles)
    int cf_cols = 0;
    bool has_flow = false;                // some tile is not FLOW_LEVEL

    // uploaded Markov models
    bool has_markov = false;
    int mk_models = 0, mk_states = 0, mk_ages = 0;
    std::vector<double> mk_c_host;        // [model][mk_states] benefits
    DevBuf<double> mk_w;                  // [model][mk_ages][4][4] ([9][9] above 4 states)
    DevBuf<double> mk_c;                  // [model][9] benefits per unit amount
    DevBuf<Tile> tiles;
    int gen = 0;                          // bumps on every upload
    long long curve_gen = 0;              // bumps whenever the curve values change (uploads
                                          // and in-place regeneration)

    // run resources
    double *scratch = nullptr;            // static device scratch of rr_reserve_recurrence_noalloc
                                          // on this device (shared by every context on it)
    std::map<rr::host::PlanKey, rr::host::HostPlan> host_plans;
    DevBuf<int> counters;
    DevBuf<double> partial;
    DevBuf<double> totals_tmp;
    DevBuf<long long> path_off;
    int path_off_node = -1, path_off_step = -1, path_off_gen = -1;
    std::map<PlanKey, std::unique_ptr<Plan>> plans;
    std::map<TuneKey, LaunchCfg> tuned;

    // options
    int opt_k = 0, opt_j = 0, opt_wg = 0, opt_graph = 1, opt_timing = 0, opt_xcd = 1;
    int opt_term_bucket = 4;              // months per remaining-term bucket in the sort
    int opt_ring = 0;                     // -1: autotune, 0: off (default), 1: on where supported
    int opt_lane_spread = 1;              // deal tile lanes over LDS banks (next upload)
    int opt_curve_share = -1;             // 0: plain queues, 1: dealt windows, 2: windows per
                                          // workgroup, -1: 1 or 2, whichever the autotuner finds faster
    int last_k = 0, last_j = 0, last_wg = 0, last_ring = 0, last_win = 0, last_qlds = 0;   // configuration of the last recurrence launch

    // timing
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;

    // graphs
    std::vector<GraphEntry> graphs;

    // work lists of the surrogate's exact fallback
    Plan item_plan[2];

    // surrogate
    rr::Surrogate *sur = nullptr;
    rr::Surrogate *nsur = nullptr;       // node-level model (scenario-averaged reserves)
};

namespace rr {
namespace host {

int fail(rr_ctx *c, int code, const char *fmt, ...);

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e__ = (expr);                                                              \
        if (e__ != hipSuccess)                                                                \
            return rr::host::fail(ctx, e__ == hipErrorOutOfMemory ? RR_ENOMEM : RR_EDEVICE,   \
                                  "%s: %s", #expr, hipGetErrorString(e__));                   \
    } while (0)

template <typename T>
int upload_vec(rr_ctx *c, DevBuf<T> &d, const std::vector<T> &h)
{
    HIPCHK(c, d.alloc(h.size()));
    if (!h.empty()) HIPCHK(c, hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return RR_OK;
}

// Run the recurrence kernel (K scenarios per lane, one tile per item) on a
// given list of work items of run `run`, writing state-0 reserves r_0
// [node][policy][scen] only; asynchronous on the context's stream.  slot
// (0 or 1) selects the device copy of the list, so two lists can be in
// flight; fresh = false reuses the copy uploaded by the previous call on
// that slot (the caller guarantees the same list).
int run_items(rr_ctx *c, const rr_run *run, const std::vector<Item> &items, int K, double *r0,
              int slot, bool fresh);

}  // namespace host
}  // namespace rr
