// Host side of the reserve-recurrence library: the C ABI of include/rr.h,
// input checks, the planner (sort, tiles, work queues), the autotuner, HIP
// graph replay and kernel timing.
#include "rr_ctx.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

using namespace rr;
using namespace rr::host;


// ---------------------------------------------------------------------------
// Error helpers
// ---------------------------------------------------------------------------
int rr::host::fail(rr_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}



static void set_msg(char *msg, size_t len, const std::string &s)
{
    if (msg && len) {
        size_t n = std::min(len - 1, s.size());
        memcpy(msg, s.data(), n);
        msg[n] = 0;
    }
}

static bool is_three_life(int product) { return product == RR_JL3_ANN || product == RR_LS3_ANN; }

// Products with a second life (the three-life annuities included).
static bool is_two_life(int product)
{
    return product == RR_JL_ANN || product == RR_REV_ANN || product == RR_LS_ANN ||
           product == RR_JL_ENDOW || product == RR_JL_ASSUR1 || product == RR_JL_ASSUR2 ||
           is_three_life(product);
}

// State model after the zero-reserve states are removed (Sec. 3.6.4): the
// first-death assurance and the two-life endowment keep only state 00, the
// second-death assurance keeps 00 and the two one-life-dead states.
static int kind_of(int product)
{
    switch (product) {
    case RR_JL_ANN:
    case RR_JL_ENDOW:
    case RR_JL3_ANN:
    case RR_JL_ASSUR1: return KIND_JOINT;
    case RR_REV_ANN: return KIND_REV;
    case RR_LS_ANN:
    case RR_LS3_ANN:
    case RR_JL_ASSUR2: return KIND_LAST;
    default: return KIND_SINGLE;
    }
}

// VALU operations per scenario-step of each model (for cost estimates).
static int ops_of_kind(int kind)
{
    switch (kind) {
    case KIND_SINGLE: return 2;
    case KIND_JOINT: return 2;
    case KIND_REV: return 5;
    default: return 8;
    }
}
static int overhead_of_kind(int kind) { return kind == KIND_SINGLE ? 6 : 12; }

// Copy n elements of T from host or device memory to a host vector.
template <typename T>
static int fetch(rr_ctx *c, const T *src, size_t n, int mem_kind, std::vector<T> &dst)
{
    dst.resize(n);
    if (n == 0) return RR_OK;
    if (mem_kind == RR_DEVICE) {
        HIPCHK(c, hipMemcpy(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost));
    } else {
        memcpy(dst.data(), src, n * sizeof(T));
    }
    return RR_OK;
}

// ---------------------------------------------------------------------------
// Validation (host only)
// ---------------------------------------------------------------------------
// v == nullptr with generated = true: the curves come from a generator.
static std::string check_basis_arrays(int n_tables, int n_ages, const double *q, int n_nodes,
                                      int n_scen, int n_steps, const double *v,
                                      const double *shock, bool generated = false)
{
    char b[256];
    if (n_tables < 1 || n_ages < 2) return "basis: need n_tables >= 1 and n_ages >= 2";
    if (n_nodes < 1 || n_scen < 1 || n_steps < 1) return "basis: need n_nodes, n_scen, n_steps >= 1";
    if ((long long)n_nodes * n_steps * (((long long)n_scen + 31) / 32 * 32 + 32) > (1LL << 31))
        return "basis: curve array exceeds 2^31 values";
    if (!q || (!v && !generated)) return "basis: q and v must not be NULL";
    if (v && generated) return "basis: v must be NULL when the curves are generated";
    for (long long i = 0; i < (long long)n_tables * n_ages; ++i) {
        double x = q[i];
        if (!(x >= 0.0 && x <= 1.0)) {
            snprintf(b, sizeof b, "basis: q[%lld] = %g is not a probability in [0, 1]", i, x);
            return b;
        }
    }
    for (long long i = 0; v && i < (long long)n_nodes * n_scen * n_steps; ++i) {
        double x = v[i];
        if (!(x > 0.0) || !std::isfinite(x)) {
            snprintf(b, sizeof b, "basis: v[%lld] = %g is not a positive finite discount factor", i, x);
            return b;
        }
    }
    if (shock)
        for (int i = 0; i < n_nodes; ++i)
            if (!(shock[i] >= 0.0) || !std::isfinite(shock[i])) {
                snprintf(b, sizeof b, "basis: shock[%d] = %g must be finite and >= 0", i, shock[i]);
                return b;
            }
    return "";
}

static std::string check_portfolio_arrays(int n, const int32_t *product, const int32_t *age1,
                                          const int32_t *age2, const int32_t *term,
                                          const int32_t *table1, const int32_t *table2,
                                          const int32_t *timing, const double *amount,
                                          const double *premium, const double *escalation,
                                          const int32_t *anniv, const int32_t *annual,
                                          const int32_t *cf_row, const double *cf, int cf_n_rows,
                                          int cf_len, int n_steps, int n_ages, int n_tables,
                                          int mk_models = -1, int mk_ages = -1, double frac = -1.0,
                                          const int32_t *age3 = nullptr, const int32_t *table3 = nullptr)
{
    char b[256];
    if (n < 0) return "portfolio: n must be >= 0";
    if (cf_n_rows < 0 || cf_len < 0) return "portfolio: cf_n_rows and cf_len must be >= 0";
    if (cf) {
        const long long m = (long long)cf_n_rows * cf_len;
        for (long long k = 0; k < m; ++k)
            if (!std::isfinite(cf[k])) {
                snprintf(b, sizeof b, "portfolio: cf[%lld] = %g is not finite", k, cf[k]);
                return b;
            }
    }
    if (n > (1 << 28)) return "portfolio: n too large";
    if (n > 0 && (!product || !age1 || !term || !table1 || !amount))
        return "portfolio: product, age1_m, term_m, table1 and amount must not be NULL";
    for (int i = 0; i < n; ++i) {
        int pr = product[i];
        if (pr < RR_SL_ANN || pr > RR_LS3_ANN) {
            snprintf(b, sizeof b, "portfolio: policy %d has unknown product %d", i, pr);
            return b;
        }
        if (term[i] < 1 || term[i] > n_steps) {
            snprintf(b, sizeof b, "portfolio: policy %d term %d outside [1, n_steps=%d]", i, term[i], n_steps);
            return b;
        }
        if (pr == RR_MARKOV) {   // table1 is the model; ages index its tables (-1: not known here)
            if (mk_models == 0) return "portfolio: RR_MARKOV policies need rr_markov_upload first";
            if (table1[i] < 0 || (mk_models > 0 && table1[i] >= mk_models)) {
                snprintf(b, sizeof b, "portfolio: policy %d model %d outside [0, %d)", i, table1[i], mk_models);
                return b;
            }
            if (age1[i] < 0 || (mk_ages > 0 && (long long)age1[i] + term[i] > mk_ages - 1)) {
                snprintf(b, sizeof b, "portfolio: policy %d age %d + term %d exceeds the Markov tables (%d ages)",
                         i, age1[i], term[i], mk_ages);
                return b;
            }
        } else {
            if (age1[i] < 0 || (long long)age1[i] + term[i] > n_ages - 1) {
                snprintf(b, sizeof b, "portfolio: policy %d age %d + term %d exceeds the tables (n_ages=%d)",
                         i, age1[i], term[i], n_ages);
                return b;
            }
            if (table1[i] < 0 || table1[i] >= n_tables) {
                snprintf(b, sizeof b, "portfolio: policy %d table1 %d outside [0, %d)", i, table1[i], n_tables);
                return b;
            }
        }
        if (is_two_life(pr)) {
            if (!age2 || !table2) return "portfolio: two-life products need age2_m and table2";
            if (age2[i] < 0 || (long long)age2[i] + term[i] > n_ages - 1) {
                snprintf(b, sizeof b, "portfolio: policy %d second age %d + term %d exceeds the tables",
                         i, age2[i], term[i]);
                return b;
            }
            if (table2[i] < 0 || table2[i] >= n_tables) {
                snprintf(b, sizeof b, "portfolio: policy %d table2 %d outside [0, %d)", i, table2[i], n_tables);
                return b;
            }
        }
        if (is_three_life(pr)) {
            if (!age3 || !table3) return "portfolio: three-life products need age3_m and table3";
            if (age3[i] < 0 || (long long)age3[i] + term[i] > n_ages - 1) {
                snprintf(b, sizeof b, "portfolio: policy %d third age %d + term %d exceeds the tables",
                         i, age3[i], term[i]);
                return b;
            }
            if (table3[i] < 0 || table3[i] >= n_tables) {
                snprintf(b, sizeof b, "portfolio: policy %d table3 %d outside [0, %d)", i, table3[i], n_tables);
                return b;
            }
        }
        if (pr == RR_CF_TABLE) {
            if (!cf_row || !cf) return "portfolio: RR_CF_TABLE policies need cf_row and cf";
            if (cf_row[i] < 0 || cf_row[i] >= cf_n_rows) {
                snprintf(b, sizeof b, "portfolio: policy %d cf_row %d outside [0, %d)", i, cf_row[i],
                         cf_n_rows);
                return b;
            }
            if (term[i] > cf_len) {
                snprintf(b, sizeof b, "portfolio: policy %d term %d exceeds cf_len %d", i, term[i], cf_len);
                return b;
            }
        }
        if (timing && timing[i] != RR_ADVANCE && timing[i] != RR_ARREARS && timing[i] != RR_FRACTIONAL) {
            snprintf(b, sizeof b, "portfolio: policy %d timing %d is not 0, 1 or 2", i, timing[i]);
            return b;
        }
        if (timing && timing[i] == RR_FRACTIONAL) {   // -1: the basis is not known here
            if (pr != RR_SL_ANN && pr != RR_JL_ANN) {
                snprintf(b, sizeof b, "portfolio: policy %d: fractional timing needs RR_SL_ANN or RR_JL_ANN", i);
                return b;
            }
            if (frac == 0.0) {
                snprintf(b, sizeof b, "portfolio: policy %d: fractional timing needs a basis with frac > 0", i);
                return b;
            }
            if ((escalation && escalation[i] > 0.0) || (annual && annual[i] == 1)) {
                snprintf(b, sizeof b, "portfolio: policy %d: fractional timing with a payment pattern", i);
                return b;
            }
        }
        if (!std::isfinite(amount[i]) || amount[i] < 0.0) {
            snprintf(b, sizeof b, "portfolio: policy %d amount %g must be finite and >= 0", i, amount[i]);
            return b;
        }
        if (premium && (!std::isfinite(premium[i]) || premium[i] < 0.0)) {
            snprintf(b, sizeof b, "portfolio: policy %d premium %g must be finite and >= 0", i, premium[i]);
            return b;
        }
        const double e = escalation ? escalation[i] : 0.0;
        if (!(e >= 0.0 && e <= 1.0)) {
            snprintf(b, sizeof b, "portfolio: policy %d escalation %g outside [0, 1]", i, e);
            return b;
        }
        if (anniv && (anniv[i] < 1 || anniv[i] > 12)) {
            snprintf(b, sizeof b, "portfolio: policy %d anniv_m %d outside [1, 12]", i, anniv[i]);
            return b;
        }
        if (annual && annual[i] != 0 && annual[i] != 1) {
            snprintf(b, sizeof b, "portfolio: policy %d annual %d is not 0 or 1", i, annual[i]);
            return b;
        }
        if (e > 0.0 || (annual && annual[i] == 1)) {
            if (pr != RR_SL_ANN && pr != RR_JL_ANN && pr != RR_REV_ANN && pr != RR_LS_ANN) {
                snprintf(b, sizeof b, "portfolio: policy %d has a payment pattern but product %d is not an annuity",
                         i, pr);
                return b;
            }
            if (premium && premium[i] != 0.0) {
                snprintf(b, sizeof b, "portfolio: policy %d has a payment pattern and premium %g (must be 0)",
                         i, premium[i]);
                return b;
            }
        }
    }
    return "";
}

extern "C" int rr_check_basis(const rr_basis *b, char *msg, size_t msg_len)
{
    if (!b) { set_msg(msg, msg_len, "basis is NULL"); return RR_EINVAL; }
    if (b->mem_kind != RR_HOST) { set_msg(msg, msg_len, "rr_check_basis needs host arrays"); return RR_EINVAL; }
    std::string s = check_basis_arrays(b->n_tables, b->n_ages, b->q, b->n_nodes, b->n_scen,
                                       b->n_steps, b->v, b->shock);
    set_msg(msg, msg_len, s);
    return s.empty() ? RR_OK : RR_EINVAL;
}

extern "C" int rr_check_portfolio(const rr_portfolio *p, int32_t n_steps, int32_t n_ages,
                                  int32_t n_tables, char *msg, size_t msg_len)
{
    if (!p) { set_msg(msg, msg_len, "portfolio is NULL"); return RR_EINVAL; }
    if (p->mem_kind != RR_HOST) { set_msg(msg, msg_len, "rr_check_portfolio needs host arrays"); return RR_EINVAL; }
    std::string s = check_portfolio_arrays(p->n, p->product, p->age1_m, p->age2_m, p->term_m,
                                           p->table1, p->table2, p->timing, p->amount,
                                           p->premium, p->escalation, p->anniv_m, p->annual,
                                           p->cf_row, p->cf, p->cf_n_rows, p->cf_len,
                                           n_steps, n_ages, n_tables, -1, -1, -1.0, p->age3_m,
                                           p->table3);
    set_msg(msg, msg_len, s);
    return s.empty() ? RR_OK : RR_EINVAL;
}

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
extern "C" int rr_create(rr_ctx **out, int device, uint64_t stream)
{
    if (!out) return RR_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return RR_EDEVICE;
    if (device < 0 || device >= ndev) return RR_EINVAL;
    std::unique_ptr<rr_ctx> c(new rr_ctx());
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) return RR_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return RR_EDEVICE;
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->lds_per_block = prop.sharedMemPerBlock;
    c->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor > 0 ? prop.maxSharedMemoryPerMultiProcessor
                                                              : prop.sharedMemPerBlock;
    c->stream = (hipStream_t)(uintptr_t)stream;   // 0 = the null stream
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) return RR_EDEVICE;
    void *scratch = nullptr;   // static scratch of rr_reserve_recurrence_noalloc on this device
    if (noalloc_scratch(device, &scratch) != hipSuccess) return RR_EDEVICE;
    c->scratch = static_cast<double *>(scratch);
    if (c->counters.alloc(MAX_QUEUES + 1) != hipSuccess) return RR_ENOMEM;
    if (hipMemset(c->counters.p, 0, sizeof(int) * (MAX_QUEUES + 1)) != hipSuccess) return RR_EDEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return RR_EDEVICE;
    *out = c.release();
    return RR_OK;
}

static void drop_graphs(rr_ctx *c)
{
    for (auto &g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

extern "C" int rr_destroy(rr_ctx *c)
{
    if (!c) return RR_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    for (auto &e : c->ev_pending) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto &e : c->ev_free) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    rr::surrogate_destroy(c->sur);
    c->sur = nullptr;
    rr::surrogate_destroy(c->nsur);
    c->nsur = nullptr;
    c->plans.clear();
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return RR_OK;
}

extern "C" const char *rr_last_error(const rr_ctx *c) { return c ? c->err.c_str() : "null context"; }

extern "C" int rr_set_stream(rr_ctx *c, uint64_t stream)
{
    if (!c) return RR_EINVAL;
    drop_graphs(c);
    c->stream = (hipStream_t)(uintptr_t)stream;
    return RR_OK;
}

extern "C" int rr_sync(rr_ctx *c)
{
    if (!c) return RR_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RR_OK;
}

extern "C" int rr_set_option(rr_ctx *c, int32_t option, int64_t value)
{
    if (!c) return RR_EINVAL;
    switch (option) {
    case RR_OPT_BLOCK_K:
        if (value != 0 && !supported_k((int)value)) return fail(c, RR_EINVAL, "K must be 0 (auto) or 1,2,4,8,16,32");
        c->opt_k = (int)value;
        return RR_OK;
    case RR_OPT_WG_PER_CU:
        if (value < 0 || value > 8) return fail(c, RR_EINVAL, "workgroups per CU must be 0..8");
        c->opt_wg = (int)value;
        return RR_OK;
    case RR_OPT_TERM_BUCKET:
        if (value < 1 || value > 1200) return fail(c, RR_EINVAL, "term bucket must be 1..1200 months");
        c->opt_term_bucket = (int)value;   // applies from the next portfolio upload
        return RR_OK;
    case RR_OPT_BLOCK_J:
        if (value != 0 && value != 1 && value != 2 && value != 4)
            return fail(c, RR_EINVAL, "J must be 0 (auto) or 1, 2, 4");
        c->opt_j = (int)value;
        return RR_OK;
    case RR_OPT_CURVE_RING:
        if (value < -1 || value > 1) return fail(c, RR_EINVAL, "curve ring must be -1 (auto), 0 or 1");
        c->opt_ring = (int)value;
        return RR_OK;
    case RR_OPT_LANE_SPREAD: c->opt_lane_spread = value ? 1 : 0; return RR_OK;   // next upload
    case RR_OPT_CURVE_SHARE:
        if (value < -1 || value > 2) return fail(c, RR_EINVAL, "curve share must be -1, 0, 1 or 2");
        if (c->opt_curve_share != value) {
            HIPCHK(c, hipStreamSynchronize(c->stream));   // launches in flight read the old queues
            drop_graphs(c);                                 // captured kernels carry the mode
            if ((c->opt_curve_share != 0) != (value != 0)) c->plans.clear();   // queue order changes
            c->tuned.clear();
        }
        c->opt_curve_share = (int)value;
        return RR_OK;
    case RR_OPT_USE_GRAPH: c->opt_graph = value ? 1 : 0; return RR_OK;
    case RR_OPT_KERNEL_TIMING: c->opt_timing = value ? 1 : 0; return RR_OK;
    case RR_OPT_XCD_QUEUES:
        c->opt_xcd = value ? 1 : 0;
        return RR_OK;
    default: return fail(c, RR_EINVAL, "unknown option %d", option);
    }
}

extern "C" int rr_get_option(rr_ctx *c, int32_t option, int64_t *value)
{
    if (!c || !value) return RR_EINVAL;
    switch (option) {
    case RR_OPT_BLOCK_K: *value = c->opt_k; return RR_OK;
    case RR_OPT_WG_PER_CU: *value = c->opt_wg; return RR_OK;
    case RR_OPT_USE_GRAPH: *value = c->opt_graph; return RR_OK;
    case RR_OPT_KERNEL_TIMING: *value = c->opt_timing; return RR_OK;
    case RR_OPT_XCD_QUEUES: *value = c->opt_xcd; return RR_OK;
    case RR_OPT_BLOCK_J: *value = c->opt_j; return RR_OK;
    case RR_OPT_TERM_BUCKET: *value = c->opt_term_bucket; return RR_OK;
    case RR_OPT_LAST_K: *value = c->last_k; return RR_OK;
    case RR_OPT_LAST_J: *value = c->last_j; return RR_OK;
    case RR_OPT_LAST_WG: *value = c->last_wg; return RR_OK;
    case RR_OPT_CURVE_RING: *value = c->opt_ring; return RR_OK;
    case RR_OPT_LAST_RING: *value = c->last_ring; return RR_OK;
    case RR_OPT_LANE_SPREAD: *value = c->opt_lane_spread; return RR_OK;
    case RR_OPT_CURVE_SHARE: *value = c->opt_curve_share; return RR_OK;
    case RR_OPT_LAST_WINDOWS: *value = c->last_win; return RR_OK;
    case RR_OPT_LAST_TABLES_LDS: *value = c->last_qlds; return RR_OK;
    default: return fail(c, RR_EINVAL, "unknown option %d", option);
    }
}

// ---------------------------------------------------------------------------
// Uploads
// ---------------------------------------------------------------------------
static int stage_tables(rr_ctx *c)
{
    // Keep only the ages the portfolio can reach, so the tables fit in LDS,
    // plus head_pad entries: a policy that has not started yet (ragged head of
    // an item) reads up to head_pad ages past its last one; those values are
    // never used.
    int used = c->has_pf ? c->max_age_needed + 1 : c->n_ages;
    used = std::max(2, std::min(used, c->n_ages));
    const int need = used + (c->has_pf ? c->head_pad : 0);
    c->n_ages_stage = need;
    // The kernels read one-step survival probabilities p = 1 - q.
    std::vector<double> st((size_t)c->n_tables * need, 0.0);
    for (int t = 0; t < c->n_tables; ++t)
        for (int a = 0; a < used; ++a)
            st[(size_t)t * need + a] = 1.0 - c->q_host[(size_t)t * c->n_ages + a];
    HIPCHK(c, c->q_stage.alloc(st.size()));
    HIPCHK(c, hipMemcpy(c->q_stage.p, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice));
    return RR_OK;
}

// Constants of the exact Vasicek step (see rr_vasicek in rr.h) after
// checking the parameters; r0 gets the n_nodes start rates.
static int vasicek_params(rr_ctx *c, const rr_vasicek *vs, int n_nodes, int n_scen, int n_steps,
                          int scen_pad, VasParams *P, std::vector<double> *r0)
{
    if (!vs) return fail(c, RR_EINVAL, "vasicek: parameters are NULL");
    if (!vs->r0) return fail(c, RR_EINVAL, "vasicek: r0 must not be NULL");
    if (!(vs->a > 0.0) || !std::isfinite(vs->a)) return fail(c, RR_EINVAL, "vasicek: a must be finite and > 0");
    if (!std::isfinite(vs->b)) return fail(c, RR_EINVAL, "vasicek: b must be finite");
    if (!(vs->sigma >= 0.0) || !std::isfinite(vs->sigma))
        return fail(c, RR_EINVAL, "vasicek: sigma must be finite and >= 0");
    if (!(vs->dt > 0.0) || !std::isfinite(vs->dt)) return fail(c, RR_EINVAL, "vasicek: dt must be finite and > 0");
    if (n_nodes < 1 || n_scen < 1 || n_steps < 1)
        return fail(c, RR_EINVAL, "vasicek: n_nodes, n_scen and n_steps must be >= 1");
    if ((long long)n_nodes * scen_pad * (3LL * n_steps + 1) > (1LL << 31))
        return fail(c, RR_EINVAL, "vasicek: more than 2^31 generated values");
    r0->assign(vs->r0, vs->r0 + n_nodes);
    for (int k = 0; k < n_nodes; ++k)
        if (!std::isfinite((*r0)[k])) return fail(c, RR_EINVAL, "vasicek: r0[%d] is not finite", k);
    const double a = vs->a, sg = vs->sigma, dt = vs->dt;
    const double e = std::exp(-a * dt);
    const double var_r = sg * sg * (1.0 - e * e) / (2.0 * a);
    const double var_y =
        std::max(0.0, sg * sg / (a * a) * (dt - 2.0 * (1.0 - e) / a + (1.0 - e * e) / (2.0 * a)));
    const double cov = sg * sg / (2.0 * a * a) * (1.0 - e) * (1.0 - e);
    const double sd_r = std::sqrt(var_r), sd_y = std::sqrt(var_y);
    const double rho = (sd_r > 0.0 && sd_y > 0.0) ? cov / (sd_r * sd_y) : 0.0;
    P->b = vs->b;
    P->dt = dt;
    P->e = e;
    P->om = (1.0 - e) / a;
    P->sd_r = sd_r;
    P->rho_sd_y = rho * sd_y;
    P->sd_y_perp = sd_y * std::sqrt(std::max(0.0, 1.0 - rho * rho));
    P->key0 = vs->key[0];
    P->key1 = vs->key[1];
    P->n_nodes = n_nodes;
    P->n_scen = n_scen;
    P->n_steps = n_steps;
    P->scen_pad = scen_pad;
    return RR_OK;
}

// Enqueue a generation: start rates to the device (waiting for the stream
// first if they change while earlier work may still read them), the work
// buffer sized, then the kernels.
static int enqueue_vasicek(rr_ctx *c, const VasParams &P, const std::vector<double> &r0, double *v,
                           int month_major, double *r_out)
{
    const size_t need = vasicek_work_doubles(P.n_nodes, P.n_scen, P.n_steps, P.scen_pad);
    const bool new_r0 = r0 != c->vas_r0_host;
    if (need > c->vas_work.n || new_r0 || r0.size() > c->vas_r0.n)
        HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, c->vas_work.alloc(need));
    if (new_r0 || r0.size() > c->vas_r0.n) {
        HIPCHK(c, c->vas_r0.alloc(r0.size()));
        HIPCHK(c, hipMemcpy(c->vas_r0.p, r0.data(), r0.size() * sizeof(double), hipMemcpyHostToDevice));
        c->vas_r0_host = r0;
    }
    HIPCHK(c, launch_vasicek(P, c->vas_r0.p, c->vas_work.p, v, month_major, r_out, c->stream));
    // Regenerating an installed basis in place: v^frac follows (install_basis
    // sizes and fills it itself after the first generation).
    if (c->has_basis && v == c->v.p && c->frac > 0.0 && c->vf.p)
        HIPCHK(c, launch_pow_curves(c->v.p, c->vf.p, (long long)c->n_nodes * c->n_steps * c->scen_pad,
                                    c->frac, c->stream));
    return RR_OK;
}

// Shared tail of rr_basis_upload and rr_basis_generate_vasicek: install the
// checked mortality part and the sizes, then the curves from the host copy
// `v` (scenario-major) or from the generator.
static int install_basis(rr_ctx *c, const rr_basis *b, std::vector<double> &q,
                         const std::vector<double> &sh, const std::vector<double> *v,
                         const VasParams *gen, const std::vector<double> *gen_r0)
{
    // A loaded portfolio that the new basis does not cover is dropped.
    bool keep_pf = c->has_pf;
    if (keep_pf) {
        for (int i = 0; i < c->n_user && keep_pf; ++i) {
            if (c->h_product[i] == RR_MARKOV) {   // uploaded model: only the term matters here
                if (c->h_term[i] > b->n_steps) keep_pf = false;
                continue;
            }
            int two = is_two_life(c->h_product[i]), three = is_three_life(c->h_product[i]);
            int amax = std::max({c->h_age1[i], two ? c->h_age2[i] : 0, three ? c->h_age3[i] : 0}) +
                       c->h_term[i];
            int tmax = std::max({c->h_table1[i], two ? c->h_table2[i] : 0, three ? c->h_table3[i] : 0});
            if (c->h_term[i] > b->n_steps || amax > b->n_ages - 1 || tmax >= b->n_tables) keep_pf = false;
            if (c->h_timing[i] == RR_FRACTIONAL && !(b->frac > 0.0)) keep_pf = false;
        }
    }
    c->has_pf = keep_pf;
    drop_graphs(c);
    c->plans.clear();
    c->tuned.clear();
    c->has_basis = false;
    c->frac = b->frac;
    c->n_tables = b->n_tables;
    c->n_ages = b->n_ages;
    c->n_nodes = b->n_nodes;
    c->n_scen = b->n_scen;
    c->n_steps = b->n_steps;
    c->scen_pad = (b->n_scen + 31) / 32 * 32 + 32;   // a block of up to 32 may overrun the last scenario
    c->q_host.swap(q);
    c->shock_host.assign((size_t)b->n_nodes, 1.0);
    if (b->shock) c->shock_host = sh;
    HIPCHK(c, c->v.alloc((size_t)b->n_nodes * b->n_steps * c->scen_pad));
    int rc;
    if (v) {   // curves as given, transposed to month-major on the device
        const size_t nv = v->size();
        DevBuf<double> tmp;
        HIPCHK(c, tmp.alloc(nv));
        HIPCHK(c, hipMemcpy(tmp.p, v->data(), nv * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(c, launch_transpose_curves(tmp.p, c->v.p, b->n_nodes, b->n_scen, b->n_steps,
                                          c->scen_pad, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        VasParams P = *gen;
        P.scen_pad = c->scen_pad;
        if ((rc = enqueue_vasicek(c, P, *gen_r0, c->v.p, 1, nullptr))) return rc;
    }
    if (c->frac > 0.0) {   // v^frac beside v for fractional annuities
        const long long nvv = (long long)b->n_nodes * b->n_steps * c->scen_pad;
        HIPCHK(c, c->vf.alloc((size_t)nvv));
        HIPCHK(c, launch_pow_curves(c->v.p, c->vf.p, nvv, c->frac, c->stream));
    }
    HIPCHK(c, c->shock.alloc((size_t)b->n_nodes));
    HIPCHK(c, hipMemcpy(c->shock.p, c->shock_host.data(), sizeof(double) * b->n_nodes,
                        hipMemcpyHostToDevice));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if ((rc = stage_tables(c))) return rc;
    c->has_basis = true;
    ++c->gen;
    ++c->curve_gen;
    return RR_OK;
}

extern "C" int rr_basis_upload(rr_ctx *c, const rr_basis *b)
{
    if (!c) return RR_EINVAL;
    if (!b) return fail(c, RR_EINVAL, "basis is NULL");
    if (b->mem_kind != RR_HOST && b->mem_kind != RR_DEVICE) return fail(c, RR_EINVAL, "bad mem_kind");
    HIPCHK(c, hipSetDevice(c->device));
    if (b->n_tables < 1 || b->n_ages < 2 || b->n_nodes < 1 || b->n_scen < 1 || b->n_steps < 1)
        return fail(c, RR_EINVAL, "basis: sizes must be positive (n_ages >= 2)");
    if (!b->q || !b->v) return fail(c, RR_EINVAL, "basis: q and v must not be NULL");
    if (!(b->frac >= 0.0 && b->frac < 1.0)) return fail(c, RR_EINVAL, "basis: frac must be in [0, 1)");
    std::vector<double> q, v, sh;
    int rc;
    size_t nv = (size_t)b->n_nodes * b->n_scen * b->n_steps;
    if ((rc = fetch(c, b->q, (size_t)b->n_tables * b->n_ages, b->mem_kind, q))) return rc;
    if ((rc = fetch(c, b->v, nv, b->mem_kind, v))) return rc;
    if (b->shock && (rc = fetch(c, b->shock, (size_t)b->n_nodes, b->mem_kind, sh))) return rc;
    std::string s = check_basis_arrays(b->n_tables, b->n_ages, q.data(), b->n_nodes, b->n_scen,
                                       b->n_steps, v.data(), b->shock ? sh.data() : nullptr);
    if (!s.empty()) return fail(c, RR_EINVAL, "%s", s.c_str());
    return install_basis(c, b, q, sh, &v, nullptr, nullptr);
}

extern "C" int rr_basis_generate_vasicek(rr_ctx *c, const rr_basis *b, const rr_vasicek *vs)
{
    if (!c) return RR_EINVAL;
    if (!b) return fail(c, RR_EINVAL, "basis is NULL");
    if (b->mem_kind != RR_HOST && b->mem_kind != RR_DEVICE) return fail(c, RR_EINVAL, "bad mem_kind");
    HIPCHK(c, hipSetDevice(c->device));
    if (b->n_tables < 1 || b->n_ages < 2 || b->n_nodes < 1 || b->n_scen < 1 || b->n_steps < 1)
        return fail(c, RR_EINVAL, "basis: sizes must be positive (n_ages >= 2)");
    if (!b->q) return fail(c, RR_EINVAL, "basis: q must not be NULL");
    if (b->v) return fail(c, RR_EINVAL, "basis: v must be NULL when the curves are generated");
    if (!(b->frac >= 0.0 && b->frac < 1.0)) return fail(c, RR_EINVAL, "basis: frac must be in [0, 1)");
    std::vector<double> q, sh, r0;
    int rc;
    if ((rc = fetch(c, b->q, (size_t)b->n_tables * b->n_ages, b->mem_kind, q))) return rc;
    if (b->shock && (rc = fetch(c, b->shock, (size_t)b->n_nodes, b->mem_kind, sh))) return rc;
    std::string s = check_basis_arrays(b->n_tables, b->n_ages, q.data(), b->n_nodes, b->n_scen,
                                       b->n_steps, nullptr, b->shock ? sh.data() : nullptr, true);
    if (!s.empty()) return fail(c, RR_EINVAL, "%s", s.c_str());
    VasParams P;
    const int scen_pad = (b->n_scen + 31) / 32 * 32 + 32;
    if ((rc = vasicek_params(c, vs, b->n_nodes, b->n_scen, b->n_steps, scen_pad, &P, &r0))) return rc;
    return install_basis(c, b, q, sh, nullptr, &P, &r0);
}

extern "C" int rr_curves_generate_vasicek(rr_ctx *c, const rr_vasicek *vs)
{
    if (!c) return RR_EINVAL;
    if (!c->has_basis) return fail(c, RR_ESTATE, "no basis installed");
    HIPCHK(c, hipSetDevice(c->device));
    VasParams P;
    std::vector<double> r0;
    int rc;
    if ((rc = vasicek_params(c, vs, c->n_nodes, c->n_scen, c->n_steps, c->scen_pad, &P, &r0))) return rc;
    ++c->curve_gen;   // cached per-scenario decisions (the surrogate's range flags) are stale
    return enqueue_vasicek(c, P, r0, c->v.p, 1, nullptr);
}

extern "C" int rr_vasicek_curves(rr_ctx *c, const rr_vasicek *vs, int32_t n_nodes, int32_t n_scen,
                                 int32_t n_steps, double *v, double *r)
{
    if (!c) return RR_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    VasParams P;
    std::vector<double> r0;
    int rc;
    const int scen_pad = (n_scen + 63) / 64 * 64;
    if ((rc = vasicek_params(c, vs, n_nodes, n_scen, n_steps, scen_pad, &P, &r0))) return rc;
    if (!v) return fail(c, RR_EINVAL, "vasicek: v must not be NULL");
    return enqueue_vasicek(c, P, r0, v, 0, r);
}

extern "C" int rr_portfolio_upload(rr_ctx *c, const rr_portfolio *p)
{
    if (!c) return RR_EINVAL;
    if (!p) return fail(c, RR_EINVAL, "portfolio is NULL");
    if (!c->has_basis) return fail(c, RR_ESTATE, "upload a basis before the portfolio");
    if (p->mem_kind != RR_HOST && p->mem_kind != RR_DEVICE) return fail(c, RR_EINVAL, "bad mem_kind");
    if (p->n < 0) return fail(c, RR_EINVAL, "portfolio: n must be >= 0");
    HIPCHK(c, hipSetDevice(c->device));
    const size_t n = (size_t)p->n;
    std::vector<int32_t> product, age1, age2, term, table1, table2, timing;
    std::vector<double> amount, premium, escalation, cf;
    std::vector<int32_t> anniv, annual, cf_row, age3, table3;
    int rc;
    if (n > 0 && (!p->product || !p->age1_m || !p->term_m || !p->table1 || !p->amount))
        return fail(c, RR_EINVAL, "portfolio: product, age1_m, term_m, table1 and amount must not be NULL");
    if ((rc = fetch(c, p->product, n, p->mem_kind, product))) return rc;
    if ((rc = fetch(c, p->age1_m, n, p->mem_kind, age1))) return rc;
    if ((rc = fetch(c, p->term_m, n, p->mem_kind, term))) return rc;
    if ((rc = fetch(c, p->table1, n, p->mem_kind, table1))) return rc;
    if ((rc = fetch(c, p->amount, n, p->mem_kind, amount))) return rc;
    if (p->age2_m) { if ((rc = fetch(c, p->age2_m, n, p->mem_kind, age2))) return rc; }
    else age2.assign(n, 0);
    if (p->table2) { if ((rc = fetch(c, p->table2, n, p->mem_kind, table2))) return rc; }
    else table2.assign(n, 0);
    if (p->timing) { if ((rc = fetch(c, p->timing, n, p->mem_kind, timing))) return rc; }
    else timing.assign(n, RR_ARREARS);
    if (p->premium) { if ((rc = fetch(c, p->premium, n, p->mem_kind, premium))) return rc; }
    else premium.assign(n, 0.0);
    if (p->escalation) { if ((rc = fetch(c, p->escalation, n, p->mem_kind, escalation))) return rc; }
    else escalation.assign(n, 0.0);
    if (p->anniv_m) { if ((rc = fetch(c, p->anniv_m, n, p->mem_kind, anniv))) return rc; }
    else anniv.assign(n, 12);
    if (p->annual) { if ((rc = fetch(c, p->annual, n, p->mem_kind, annual))) return rc; }
    else annual.assign(n, 0);
    if (p->cf_n_rows < 0 || p->cf_len < 0) return fail(c, RR_EINVAL, "portfolio: cf_n_rows and cf_len must be >= 0");
    if (p->cf_row) { if ((rc = fetch(c, p->cf_row, n, p->mem_kind, cf_row))) return rc; }
    if (p->age3_m) { if ((rc = fetch(c, p->age3_m, n, p->mem_kind, age3))) return rc; }
    if (p->table3) { if ((rc = fetch(c, p->table3, n, p->mem_kind, table3))) return rc; }
    if (p->cf) {
        if ((rc = fetch(c, p->cf, (size_t)p->cf_n_rows * p->cf_len, p->mem_kind, cf))) return rc;
    }
    bool any_two = false;
    for (size_t i = 0; i < n; ++i) any_two |= is_two_life(product[i]);
    std::string s = check_portfolio_arrays(p->n, product.data(), age1.data(),
                                           (p->age2_m || !any_two) ? age2.data() : nullptr,
                                           term.data(), table1.data(),
                                           (p->table2 || !any_two) ? table2.data() : nullptr,
                                           timing.data(), amount.data(), premium.data(),
                                           escalation.data(), anniv.data(), annual.data(),
                                           p->cf_row ? cf_row.data() : nullptr,
                                           p->cf ? cf.data() : nullptr, p->cf_n_rows, p->cf_len,
                                           c->n_steps, c->n_ages, c->n_tables,
                                           c->has_markov ? c->mk_models : 0,
                                           c->has_markov ? c->mk_ages : 0, c->frac,
                                           p->age3_m ? age3.data() : nullptr,
                                           p->table3 ? table3.data() : nullptr);
    if (!s.empty()) return fail(c, RR_EINVAL, "%s", s.c_str());
    if (!p->age3_m) age3.assign(n, 0);
    if (!p->table3) table3.assign(n, 0);

    drop_graphs(c);
    c->plans.clear();
    c->tuned.clear();
    c->has_pf = false;

    // Sort: state model, cash-flow kind (level, payment pattern, table),
    // remaining term descending, age (stable on index).
    std::vector<int32_t> patterned(n, 0), flow(n, FLOW_LEVEL);
    for (size_t i = 0; i < n; ++i) {
        patterned[i] = (escalation[i] > 0.0 || annual[i] == 1) ? 1 : 0;
        flow[i] = product[i] == RR_CF_TABLE      ? FLOW_TABLE
                  : product[i] == RR_MARKOV      ? FLOW_MARKOV
                  : is_three_life(product[i])    ? FLOW_THREE
                  : timing[i] == RR_FRACTIONAL   ? FLOW_FRAC
                  : patterned[i]                 ? FLOW_PATTERN
                                                 : FLOW_LEVEL;
    }
    auto group_of = [&](int u) { return N_FLOWS * kind_of(product[u]) + flow[u]; };
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    // Within a model, remaining terms are bucketed (width term_bucket months,
    // default 4, longest first) and each bucket is ordered by table and age:
    // tiles of neighbouring table entries at the price of at most term_bucket
    // ragged steps (the lanes are then dealt over the LDS banks below).
    const int tb = std::max(1, c->opt_term_bucket);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        int ka = group_of(a), kb = group_of(b);
        if (ka != kb) return ka < kb;
        const int ba = (term[a] - 1) / tb, bb = (term[b] - 1) / tb;
        if (ba != bb) return ba > bb;
        if (table1[a] != table1[b]) return table1[a] < table1[b];
        if (age1[a] != age1[b]) return age1[a] < age1[b];
        return term[a] > term[b];
    });
    // Slots: each model's run padded to whole tiles.
    std::vector<int> s_age1, s_age2, s_age3, s_term, s_qoff1, s_qoff2, s_qoff3, s_uidx;
    std::vector<Tile> tiles;
    std::vector<int> slot_user;
    size_t i0 = 0;
    int max_age = 1;
    while (i0 < n) {
        const int group = group_of(order[i0]);
        size_t i1 = i0;
        while (i1 < n && group_of(order[i1]) == group) ++i1;
        for (size_t a = i0; a < i1; a += TILE) {
            Tile T;
            T.kind = group / N_FLOWS;
            T.flow = group % N_FLOWS;
            T.first = (int)s_uidx.size();
            T.smax = 0;
            T.smin = 1 << 30;
            for (int l = 0; l < TILE; ++l) {
                size_t j = a + l;
                if (j < i1) {
                    int u = order[j];
                    s_uidx.push_back(u);
                    s_age1.push_back(age1[u]);
                    bool two = is_two_life(product[u]);
                    s_age2.push_back(two ? age2[u] : 0);
                    s_term.push_back(term[u]);
                    const bool mk = product[u] == RR_MARKOV;   // no mortality table
                    s_qoff1.push_back(mk ? 0 : table1[u]);   // scaled below
                    s_qoff2.push_back(two ? table2[u] : 0);
                    const bool three = is_three_life(product[u]);
                    s_age3.push_back(three ? age3[u] : 0);
                    s_qoff3.push_back(three ? table3[u] : 0);
                    T.smax = std::max(T.smax, term[u]);
                    T.smin = std::min(T.smin, term[u]);
                    if (!mk) max_age = std::max(max_age, age1[u] + term[u]);
                    if (two) max_age = std::max(max_age, age2[u] + term[u]);
                    if (three) max_age = std::max(max_age, age3[u] + term[u]);
                } else {
                    s_uidx.push_back(-1);
                    s_age1.push_back(0);
                    s_age2.push_back(0);
                    s_term.push_back(0);
                    s_qoff1.push_back(0);
                    s_qoff2.push_back(0);
                    s_age3.push_back(0);
                    s_qoff3.push_back(0);
                }
            }
            tiles.push_back(T);
        }
        i0 = i1;
    }
    const int n_pad = (int)s_uidx.size();
    c->max_age_needed = max_age;
    // Ragged head of the widest item: up to 4 consecutive tiles of one model.
    int head_pad = 0;
    for (size_t t0 = 0; t0 < tiles.size(); ++t0) {
        int smax = 0, smin = 1 << 30;
        const size_t span = tiles[t0].flow != FLOW_LEVEL ? 1 : 4;
        for (size_t t1 = t0; t1 < tiles.size() && t1 < t0 + span && tiles[t1].kind == tiles[t0].kind &&
                             tiles[t1].flow == tiles[t0].flow;
             ++t1) {
            smax = std::max(smax, tiles[t1].smax);
            smin = std::min(smin, tiles[t1].smin);
            head_pad = std::max(head_pad, smax - smin);
        }
    }
    c->head_pad = head_pad;
    c->has_pf = true;          // stage_tables reads max_age_needed
    if ((rc = stage_tables(c))) { c->has_pf = false; return rc; }
    for (int j = 0; j < n_pad; ++j) {
        s_qoff1[j] *= c->n_ages_stage;
        s_qoff2[j] *= c->n_ages_stage;
        s_qoff3[j] *= c->n_ages_stage;
    }
    // Lane order within each tile.  All lanes of a tile take the same step t
    // together, so lane l reads the staged table at (qoff + age)_l + shift + t
    // in one LDS instruction per life: the bank of that read is fixed by
    // (qoff + age)_l modulo the bank count for the whole recurrence.  Ages
    // sorted a few months apart put many lanes on few banks; instead the
    // lanes are dealt so that every group of 16 lanes holds distinct residues
    // modulo 16 and every half-wavefront distinct residues modulo 32 as far
    // as the tile's residues allow (each life counted, two-life tiles too).
    if (c->opt_lane_spread) {
        std::vector<int> perm(TILE);
        for (const Tile &T : tiles) {
            const bool two = T.kind != KIND_SINGLE;
            int c16[4][16] = {}, c32[2][32] = {}, used[4] = {};
            int d16[4][16] = {}, d32[2][32] = {};
            // residues of life 1 and (two lives) life 2 per slot
            std::vector<int> order(TILE);
            std::iota(order.begin(), order.end(), 0);
            int freq[16] = {};
            for (int l = 0; l < TILE; ++l) ++freq[(s_qoff1[T.first + l] + s_age1[T.first + l]) & 15];
            std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
                const int fa = freq[(s_qoff1[T.first + a] + s_age1[T.first + a]) & 15];
                const int fb = freq[(s_qoff1[T.first + b] + s_age1[T.first + b]) & 15];
                return fa > fb;   // most crowded residues first
            });
            for (int l : order) {
                const int j = T.first + l;
                const int a = (s_qoff1[j] + s_age1[j]) & 31;
                const int b = two ? (s_qoff2[j] + s_age2[j]) & 31 : 0;
                int best = -1;
                long cost_best = 0;
                for (int g = 0; g < 4; ++g) {
                    if (used[g] == 16) continue;
                    long cost = 4L * c16[g][a & 15] + c32[g / 2][a];
                    if (two) cost += 4L * d16[g][b & 15] + d32[g / 2][b];
                    if (best < 0 || cost < cost_best) { best = g; cost_best = cost; }
                }
                ++c16[best][a & 15];
                ++c32[best / 2][a];
                if (two) { ++d16[best][b & 15]; ++d32[best / 2][b]; }
                perm[best * 16 + used[best]++] = j;
            }
            auto apply = [&](std::vector<int> &v) {
                int tmp[TILE];
                for (int l = 0; l < TILE; ++l) tmp[l] = v[perm[l]];
                for (int l = 0; l < TILE; ++l) v[T.first + l] = tmp[l];
            };
            apply(s_uidx);
            apply(s_age1);
            apply(s_age2);
            apply(s_term);
            apply(s_qoff1);
            apply(s_qoff2);
            apply(s_age3);
            apply(s_qoff3);
        }
    }
    // Coefficients.
    std::vector<double> coef((size_t)N_COEF * std::max(n_pad, 1), 0.0);
    auto C = [&](int row, int slot) -> double & { return coef[(size_t)row * n_pad + slot]; };
    for (int j = 0; j < n_pad; ++j) {
        int u = s_uidx[j];
        if (u < 0) continue;
        const int pr = product[u];
        const double pay = amount[u] / 12.0;
        const bool adv = timing[u] == RR_ADVANCE;
        const double P = premium[u];
        switch (pr) {
        case RR_SL_ANN:
        case RR_JL_ANN:
            C(0, j) = (adv ? pay : 0.0) - P;
            C(1, j) = adv ? 0.0 : pay;
            break;
        case RR_TERM:
            C(0, j) = -P;
            C(2, j) = amount[u];
            break;
        case RR_ENDOW:
            C(0, j) = -P;
            C(3, j) = amount[u];
            break;
        case RR_ENDOW_ASSUR:
            C(0, j) = -P;
            C(2, j) = amount[u];
            C(3, j) = amount[u];
            break;
        case RR_CF_TABLE:      // the survival cash flows come from the table
            C(0, j) = -P;
            break;
        case RR_JL_ENDOW:
            C(0, j) = -P;
            C(3, j) = amount[u];
            break;
        case RR_JL_ASSUR1:     // c = p a1 + (1 - p) b1 with p = px py
            C(0, j) = -P;
            C(2, j) = amount[u];
            break;
        case RR_JL_ASSUR2:
            C(0, j) = -P;
            C(6, j) = amount[u];
            break;
        case RR_MARKOV:        // premium in state 0, benefits per state
            C(0, j) = -P;
            if (c->mk_states <= 4) {
                for (int st = 0; st < c->mk_states; ++st)
                    C(1 + st, j) = amount[u] * c->mk_c_host[(size_t)table1[u] * c->mk_states + st];
            } else {
                C(1, j) = amount[u];   // the kernel scales the model's benefits
            }
            break;
        case RR_JL3_ANN:
            C(0, j) = (adv ? pay : 0.0) - P;
            C(1, j) = adv ? 0.0 : pay;
            break;
        case RR_LS3_ANN:       // premium while all three are alive
            C(0, j) = (adv ? pay : 0.0) - P;
            C(1, j) = adv ? 0.0 : pay;
            C(2, j) = adv ? pay : 0.0;
            break;
        case RR_REV_ANN:
            C(0, j) = -P;
            C(4, j) = adv ? pay : 0.0;
            C(5, j) = adv ? 0.0 : pay;
            break;
        case RR_LS_ANN:
            C(0, j) = (adv ? pay : 0.0) - P;
            C(1, j) = adv ? 0.0 : pay;
            C(2, j) = adv ? pay : 0.0;
            C(3, j) = adv ? 0.0 : pay;
            C(4, j) = adv ? pay : 0.0;
            C(5, j) = adv ? 0.0 : pay;
            break;
        }
    }
    if ((rc = upload_vec(c, c->age1, s_age1))) return rc;
    if ((rc = upload_vec(c, c->age2, s_age2))) return rc;
    if ((rc = upload_vec(c, c->term, s_term))) return rc;
    if ((rc = upload_vec(c, c->qoff1, s_qoff1))) return rc;
    if ((rc = upload_vec(c, c->qoff2, s_qoff2))) return rc;
    if ((rc = upload_vec(c, c->age3, s_age3))) return rc;
    if ((rc = upload_vec(c, c->qoff3, s_qoff3))) return rc;
    if ((rc = upload_vec(c, c->uidx, s_uidx))) return rc;
    if ((rc = upload_vec(c, c->coef, coef))) return rc;
    if ((rc = upload_vec(c, c->tiles, tiles))) return rc;
    // Payment patterns of the slots (level slots: g = 1, anniversary 12) and
    // the cash flows of table slots, amount x table value, month-major over
    // the table tiles' slots (padding slots: 0).
    c->has_flow = false;
    for (const Tile &T : tiles) c->has_flow |= T.flow != FLOW_LEVEL;
    c->cf_cols = 0;
    if (c->has_flow) {
        std::vector<double> pg(n_pad, 1.0);
        std::vector<int> pc(n_pad, 12);
        int first_tab = -1, cf_steps = 0;
        for (const Tile &T : tiles)
            if (T.flow == FLOW_TABLE) {
                if (first_tab < 0) first_tab = T.first;
                c->cf_cols += TILE;
                cf_steps = std::max(cf_steps, T.smax);
            }
        for (const Tile &T : tiles) {
            for (int l = 0; l < TILE; ++l) {
                const int j = T.first + l;
                const int u = s_uidx[j];
                if (T.flow == FLOW_TABLE) {
                    pc[j] = j - first_tab;   // table tiles are consecutive
                } else if (T.flow == FLOW_MARKOV) {
                    pc[j] = u >= 0 ? table1[u] : 0;   // the model
                } else if (T.flow == FLOW_PATTERN && u >= 0) {
                    pg[j] = 1.0 + escalation[u];
                    pc[j] = anniv[u] | (annual[u] ? PAT_ANNUAL : 0) |
                            (timing[u] == RR_ARREARS ? PAT_ARREARS : 0);
                }
            }
        }
        if ((rc = upload_vec(c, c->pat_g, pg))) return rc;
        if ((rc = upload_vec(c, c->pat_code, pc))) return rc;
        if (c->cf_cols > 0) {
            std::vector<double> ct((size_t)std::max(cf_steps, 1) * c->cf_cols, 0.0);
            for (const Tile &T : tiles) {
                if (T.flow != FLOW_TABLE) continue;
                for (int l = 0; l < TILE; ++l) {
                    const int j = T.first + l, u = s_uidx[j];
                    if (u < 0) continue;
                    const double *row = cf.data() + (size_t)cf_row[u] * p->cf_len;
                    for (int t = 0; t < term[u]; ++t)
                        ct[(size_t)t * c->cf_cols + (j - first_tab)] = amount[u] * row[t];
                }
            }
            if ((rc = upload_vec(c, c->cf_t, ct))) return rc;
        }
    }
    c->n_user = (int)n;
    c->n_pad = n_pad;
    c->n_tiles = (int)tiles.size();
    c->tiles_host = tiles;
    c->h_product.swap(product);
    c->h_age1.swap(age1);
    c->h_age2.swap(age2);
    c->h_term.swap(term);
    c->h_table1.swap(table1);
    c->h_table2.swap(table2);
    c->h_age3.swap(age3);
    c->h_table3.swap(table3);
    c->h_timing.swap(timing);
    c->h_amount.swap(amount);
    c->h_premium.swap(premium);
    c->h_patterned.swap(patterned);
    c->slot_of_user.assign(n, -1);
    for (int j = 0; j < n_pad; ++j)
        if (s_uidx[j] >= 0) c->slot_of_user[s_uidx[j]] = j;
    ++c->gen;
    return RR_OK;
}

extern "C" int rr_node_expected_reserves(rr_ctx *c, const rr_run *run, double *node_r0,
                                         double *node_totals)
{
    if (!c) return RR_EINVAL;
    if (!c->has_basis || !c->has_pf) return fail(c, RR_ESTATE, "upload a basis and a portfolio first");
    if (!run) return fail(c, RR_EINVAL, "run must not be NULL");
    if (run->node_count < 0 || run->scen_count < 1) return fail(c, RR_EINVAL, "need node_count >= 0 and scen_count >= 1");
    if (run->node_begin < 0 || run->node_begin + run->node_count > c->n_nodes)
        return fail(c, RR_EINVAL, "node range outside the basis");
    if (run->scen_begin < 0 || run->scen_begin + run->scen_count > c->n_scen)
        return fail(c, RR_EINVAL, "scenario range outside the basis");
    for (int i = 0; i < c->n_user; ++i)
        if (c->h_timing[i] == RR_FRACTIONAL)
            return fail(c, RR_EINVAL, "fractional timing: the scenario mean is not the mean-curve reserve "
                                      "(policy %d)", i);
    if (run->node_count == 0 || (!node_r0 && !node_totals)) return RR_OK;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, c->mean_D.alloc((size_t)run->node_count * c->n_steps * run->scen_count));
    HIPCHK(c, c->mean_v.alloc((size_t)c->n_nodes * c->n_steps * 64));
    HIPCHK(c, launch_mean_curve(c->v.p, c->n_steps, c->scen_pad, run->node_begin, run->node_count,
                                run->scen_begin, run->scen_count, c->mean_D.p, c->mean_v.p,
                                c->stream));
    // One scenario per node on the mean curve, through the ordinary path
    // (direct launches: a captured graph would hold the curve pointer).
    rr_run r = *run;
    r.scen_begin = 0;
    r.scen_count = 1;
    r.out_mask = (node_r0 ? RR_OUT_R0 : 0u) | (node_totals ? RR_OUT_TOTALS : 0u);
    rr_outputs o;
    memset(&o, 0, sizeof o);
    o.r0 = node_r0;
    o.totals = node_totals;
    const int graph = c->opt_graph;
    c->opt_graph = 0;
    c->v_override = c->mean_v.p;
    c->pad_override = 64;
    const int rc = rr_reserve_recurrence(c, &r, &o);
    c->v_override = nullptr;
    c->pad_override = 0;
    c->opt_graph = graph;
    return rc;
}

extern "C" int rr_markov_upload(rr_ctx *c, const rr_markov *m)
{
    if (!c) return RR_EINVAL;
    if (!m) return fail(c, RR_EINVAL, "markov: models are NULL");
    if (m->mem_kind != RR_HOST && m->mem_kind != RR_DEVICE) return fail(c, RR_EINVAL, "bad mem_kind");
    if (m->n_models < 1 || m->n_states < 2 || m->n_states > MAX_MK_STATES || m->n_ages < 2)
        return fail(c, RR_EINVAL, "markov: need n_models >= 1, 2 <= n_states <= 9, n_ages >= 2");
    if (!m->w || !m->benefit) return fail(c, RR_EINVAL, "markov: w and benefit must not be NULL");
    const int M = m->n_states;
    // Device layout: rows padded to 4 states ([4][4], 16-byte row pairs) up
    // to 4 states, to 9 ([9][9]) above.
    const int MP = M <= 4 ? 4 : MAX_MK_STATES;
    if ((long long)m->n_models * m->n_ages * MP * MP > (1LL << 31))
        return fail(c, RR_EINVAL, "markov: tables too large");
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<double> w, ben;
    int rc;
    if ((rc = fetch(c, m->w, (size_t)m->n_models * m->n_ages * M * M, m->mem_kind, w))) return rc;
    if ((rc = fetch(c, m->benefit, (size_t)m->n_models * M, m->mem_kind, ben))) return rc;
    for (size_t k = 0; k < ben.size(); ++k)
        if (!std::isfinite(ben[k])) return fail(c, RR_EINVAL, "markov: benefit[%zu] is not finite", k);
    std::vector<double> wp((size_t)m->n_models * m->n_ages * MP * MP, 0.0);
    for (int md = 0; md < m->n_models; ++md)
        for (int a = 0; a < m->n_ages; ++a)
            for (int i = 0; i < M; ++i) {
                double sum = 0.0;
                for (int j = 0; j < M; ++j) {
                    const double x = w[(((size_t)md * m->n_ages + a) * M + i) * M + j];
                    if (!(x >= 0.0 && x <= 1.0))
                        return fail(c, RR_EINVAL, "markov: model %d age %d w[%d][%d] = %g is not a probability",
                                    md, a, i, j, x);
                    sum += x;
                    wp[(((size_t)md * m->n_ages + a) * MP + i) * MP + j] = x;
                }
                if (std::fabs(sum - 1.0) > 1e-12)
                    return fail(c, RR_EINVAL, "markov: model %d age %d row %d sums to %.17g", md, a, i, sum);
            }
    HIPCHK(c, c->mk_w.alloc(wp.size()));
    HIPCHK(c, hipMemcpy(c->mk_w.p, wp.data(), wp.size() * sizeof(double), hipMemcpyHostToDevice));
    std::vector<double> cpad((size_t)m->n_models * MAX_MK_STATES, 0.0);
    for (int md = 0; md < m->n_models; ++md)
        for (int j = 0; j < M; ++j) cpad[(size_t)md * MAX_MK_STATES + j] = ben[(size_t)md * M + j];
    if ((rc = upload_vec(c, c->mk_c, cpad))) return rc;
    c->mk_c_host.swap(ben);
    c->mk_models = m->n_models;
    c->mk_states = M;
    c->mk_ages = m->n_ages;
    c->has_markov = true;
    // A portfolio with RR_MARKOV policies holds the old benefits: drop it.
    bool has_mk = false;
    for (int i = 0; i < c->n_user; ++i) has_mk |= c->h_product[i] == RR_MARKOV;
    if (c->has_pf && has_mk) c->has_pf = false;
    drop_graphs(c);
    c->plans.clear();
    c->tuned.clear();
    ++c->gen;
    return RR_OK;
}

extern "C" int rr_path_size(rr_ctx *c, int32_t node, int32_t node_step_m, int64_t *n_out)
{
    if (!c || !n_out) return RR_EINVAL;
    if (!c->has_pf) return fail(c, RR_ESTATE, "no portfolio loaded");
    int64_t s = 0;
    for (int i = 0; i < c->n_user; ++i) s += std::max(c->h_term[i] - node * node_step_m, 0) + 1;
    *n_out = s;
    return RR_OK;
}

// ---------------------------------------------------------------------------
// Planner: work items and per-XCD queues, longest first
// ---------------------------------------------------------------------------
// Work items of a run (the host side of a plan): up to J consecutive tiles
// of one scalar model (one tile for the vector models) x a block of K
// scenarios x a node, dealt to the work queues, longest first.
static void plan_lists(rr_ctx *c, const rr_run *run, const LaunchCfg &cfg, int queues,
                       std::vector<Item> &items, std::vector<int> &qbeg)
{
    const int K = cfg.K, J = cfg.J;
    const int nsb = (run->scen_count + K - 1) / K;
    struct W { long long cost; Item item; };
    std::vector<std::vector<W>> qs(queues);
    // Items: up to J consecutive tiles of one scalar model (one tile for the
    // vector models) x a block of K scenarios x a node.
    std::vector<std::pair<int, int>> groups;   // (first tile, count)
    for (int t = 0; t < c->n_tiles;) {
        const int kind = c->tiles_host[t].kind;
        const int flow = c->tiles_host[t].flow;
        const int jmax = ((kind == KIND_SINGLE || kind == KIND_JOINT) && flow == FLOW_LEVEL) ? J : 1;
        int count = 1;
        while (count < jmax && t + count < c->n_tiles && c->tiles_host[t + count].kind == kind &&
               c->tiles_host[t + count].flow == flow)
            ++count;
        groups.push_back({t, count});
        t += count;
    }
    auto item_cost = [&](int first, int count, int shift) -> long long {
        const Tile &T = c->tiles_host[first];
        int smax = T.smax;
        for (int j = 1; j < count; ++j) smax = std::max(smax, c->tiles_host[first + j].smax);
        const long long steps = std::max(smax - shift, 0);
        return steps * count * (ops_of_kind(T.kind) * K + overhead_of_kind(T.kind) + (T.flow ? 16 : 0)) +
               64;
    };
    for (int nr = 0; nr < run->node_count; ++nr) {
        const int shift = (run->node_begin + nr) * run->node_step_m;
        for (const auto &g : groups) {
            const long long cost = item_cost(g.first, g.second, shift);
            for (int b = 0; b < nsb; ++b) {
                const int qid = queues > 1 ? (int)(((long long)nr * nsb + b) % queues) : 0;
                qs[qid].push_back({cost, Item{nr, g.first, b * K, g.second}});
            }
        }
    }
    items.clear();
    qbeg.assign(queues + 1, 0);
    const int share = c->opt_curve_share != 0 ? WG_THREADS / 64 : 1;
    for (int qi = 0; qi < queues; ++qi) {
        // Longest first.  An item's curves are read with scalar loads
        // through the scalar cache that neighbouring CUs share, so the
        // queue is then dealt in windows of `share` tile groups of about
        // the same length (one per wavefront of a workgroup, taken at
        // about the same time): within a window the items are ordered by
        // scenario block, so wavefronts that start together walk the same
        // curve lines and one cache miss serves them all.
        std::stable_sort(qs[qi].begin(), qs[qi].end(), [](const W &a, const W &b) {
            if (a.cost != b.cost) return a.cost > b.cost;
            return a.item.tile < b.item.tile;
        });
        qbeg[qi] = (int)items.size();
        size_t u0 = 0;
        while (u0 < qs[qi].size()) {
            // a window: the items of `share` consecutive (node, tile group) units
            size_t u1 = u0;
            int units = 0;
            while (u1 < qs[qi].size() && units < share) {
                const Item &h = qs[qi][u1].item;
                while (u1 < qs[qi].size() && qs[qi][u1].item.tile == h.tile &&
                       qs[qi][u1].item.node_rel == h.node_rel)
                    ++u1;
                ++units;
            }
            std::stable_sort(qs[qi].begin() + u0, qs[qi].begin() + u1, [](const W &a, const W &b) {
                if (a.item.node_rel != b.item.node_rel) return a.item.node_rel < b.item.node_rel;
                return a.item.sblock < b.item.sblock;
            });
            u0 = u1;
        }
        for (auto &w : qs[qi]) items.push_back(w.item);
    }
    qbeg[queues] = (int)items.size();
}

static int build_plan(rr_ctx *c, const rr_run *run, const LaunchCfg &cfg, Plan **out)
{
    const int queues = c->opt_xcd ? MAX_QUEUES : 1;
    const int K = cfg.K, J = cfg.J;
    PlanKey key{run->node_begin, run->node_count, run->scen_begin, run->scen_count,
                run->node_step_m, K, J, queues, c->gen, cfg.wg};
    auto it = c->plans.find(key);
    Plan *pl;
    if (it == c->plans.end()) {
        std::unique_ptr<Plan> np(new Plan());
        std::vector<Item> items;
        std::vector<int> qbeg;
        plan_lists(c, run, cfg, queues, items, qbeg);
        np->K = K;
        np->J = J;
        np->n_items = (int)items.size();
        np->n_queues = queues;
        int rc;
        if ((rc = upload_vec(c, np->items, items))) return rc;
        if ((rc = upload_vec(c, np->qbeg, qbeg))) return rc;
        pl = np.get();
        c->plans[key] = std::move(np);
    } else {
        pl = it->second.get();
    }
    const int waves_per_wg = WG_THREADS / 64;
    pl->wg_per_cu = cfg.wg;
    pl->ring = cfg.ring;
    pl->win = cfg.win;
    pl->grid = std::max(1, std::min(c->n_cu * cfg.wg, (pl->n_items + waves_per_wg - 1) / waves_per_wg));
    *out = pl;
    return RR_OK;
}

// Whether a workgroup stages the survival tables in LDS (else it reads them
// from device memory).
static bool tables_in_lds(const rr_ctx *c)
{
    const size_t nq = (size_t)c->n_tables * c->n_ages_stage;
    return nq <= (size_t)max_lds_tables_doubles() && nq * 8 <= c->lds_per_block;
}

static RecParams make_params(rr_ctx *c, const rr_run *run, const rr_outputs *out, const Plan *pl,
                             double *partial)
{
    RecParams P;
    memset(&P, 0, sizeof P);
    P.q = c->q_stage.p;
    P.n_ages_stage = c->n_ages_stage;
    P.n_q = c->n_tables * c->n_ages_stage;
    P.q_in_lds = tables_in_lds(c) ? 1 : 0;
    P.ring_off = P.q_in_lds ? (P.n_q + 1) / 2 * 2 : 0;   // 16-byte aligned rings after the tables
    P.win = pl->win;
    P.v = c->v_override ? c->v_override : c->v.p;
    P.n_steps = c->n_steps;
    P.scen_pad = c->v_override ? c->pad_override : c->scen_pad;
    P.shock = c->shock.p;
    P.age1 = c->age1.p;
    P.age2 = c->age2.p;
    P.term = c->term.p;
    P.qoff1 = c->qoff1.p;
    P.qoff2 = c->qoff2.p;
    P.uidx = c->uidx.p;
    P.coef = c->coef.p;
    P.pat_g = c->has_flow ? c->pat_g.p : nullptr;
    P.pat_code = c->has_flow ? c->pat_code.p : nullptr;
    P.cf_t = (c->has_flow && c->cf_cols > 0) ? c->cf_t.p : nullptr;
    P.cf_cols = c->cf_cols;
    P.mk_w = c->has_markov ? c->mk_w.p : nullptr;
    P.mk_ages = c->mk_ages;
    P.mk_states = c->mk_states;
    P.mk_c = c->has_markov ? c->mk_c.p : nullptr;
    P.age3 = c->age3.p;
    P.qoff3 = c->qoff3.p;
    P.vf = c->frac > 0.0 ? c->vf.p : nullptr;
    P.frac = c->frac;
    P.n_pad = c->n_pad;
    P.n_user = c->n_user;
    P.tiles = c->tiles.p;
    P.n_tiles = c->n_tiles;
    P.has_vector = 0;
    for (const Tile &T : c->tiles_host) P.has_vector |= (T.kind == KIND_REV || T.kind == KIND_LAST);
    P.items = pl->items_ext ? pl->items_ext : pl->items.p;
    P.qbeg = pl->qbeg_ext ? pl->qbeg_ext : pl->qbeg.p;
    P.counters = pl->counters_ext ? pl->counters_ext : c->counters.p;
    P.n_queues = pl->n_queues;
    P.node_begin = run->node_begin;
    P.scen_begin = run->scen_begin;
    P.scen_count = run->scen_count;
    P.node_step = run->node_step_m;
    const bool want_r0 = (run->out_mask & RR_OUT_R0) != 0;
    P.r0 = want_r0 ? out->r0 : nullptr;
    P.r0_states = (run->out_mask & RR_OUT_ALL_STATES) ? 4 : 1;
    P.partial = partial;
    P.path = (run->out_mask & RR_OUT_PATH) ? out->path : nullptr;
    P.path_off = (run->out_mask & RR_OUT_PATH) ? c->path_off.p : nullptr;
    P.path_lds = P.q_in_lds ? (P.n_q + 1) / 2 * 2 : 0;   // path stages after the tables
    return P;
}

// Dynamic LDS of a recurrence launch: the staged tables, then (curve ring)
// one ring per wavefront of the workgroup, or (path output, one scenario per
// lane) one path stage per wavefront.
static size_t recurrence_lds_bytes(const RecParams &P, int K, int ring)
{
    size_t d = P.q_in_lds ? (size_t)P.n_q : 0;
    if (ring) d = (size_t)P.ring_off + (size_t)(WG_THREADS / 64) * ring_doubles_per_wave(K);
    if (P.path) d = (size_t)P.path_lds + (size_t)(WG_THREADS / 64) * PATH_STAGE_DOUBLES;
    return d * sizeof(double);
}

// Whether the curve-ring instances can run this portfolio (level single- and
// joint-life tiles only) with (K, J) and fit their LDS.
static bool ring_ok(const rr_ctx *c, int K, int J)
{
    if (!supported_ring(K, J) || c->has_flow) return false;
    for (const Tile &T : c->tiles_host)
        if (T.kind == KIND_REV || T.kind == KIND_LAST) return false;
    const size_t nq = (size_t)c->n_tables * c->n_ages_stage;
    const size_t d = (tables_in_lds(c) ? (nq + 1) / 2 * 2 : 0) + (size_t)(WG_THREADS / 64) * ring_doubles_per_wave(K);
    return d * sizeof(double) <= c->lds_per_block;
}

static int enqueue_run(rr_ctx *c, const rr_run *run, const rr_outputs *out, Plan *pl,
                       double *partial, double *totals, hipStream_t s, bool timed)
{
    RecParams P = make_params(c, run, out, pl, partial);
    const size_t lds = recurrence_lds_bytes(P, pl->K, pl->ring);
    if (lds > c->lds_per_block)   // tables (<= 64 KB) and path stages (68 KB) fit 160 KB
        return fail(c, RR_ERANGE, "recurrence launch needs more LDS than a workgroup has");
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (timed) {
        if (!c->ev_free.empty()) {
            ev = c->ev_free.back();
            c->ev_free.pop_back();
        } else {
            HIPCHK(c, hipEventCreate(&ev.first));
            HIPCHK(c, hipEventCreate(&ev.second));
        }
        HIPCHK(c, hipEventRecord(ev.first, s));
    }
    // Persistent workgroups beyond what the CUs' LDS holds at once would only
    // start once the queues are drained: leave them out.
    int grid = pl->grid;
    if (lds > 0) grid = std::min(grid, c->n_cu * std::max(1, (int)(c->lds_per_cu / lds)));
    HIPCHK(c, launch_recurrence(pl->K, pl->J, P, grid, lds, s, pl->ring != 0));
    if (timed) {
        HIPCHK(c, hipEventRecord(ev.second, s));
        c->ev_pending.push_back(ev);
    }
    if (totals) {
        HIPCHK(c, launch_totals(partial, run->node_count, c->n_tiles, run->scen_count, totals,
                                partial + (size_t)run->node_count * c->n_tiles * run->scen_count, s));
    }
    if ((run->out_mask & RR_OUT_STATS) && out->stats) {
        double tail = run->tail > 0.0 ? run->tail : 0.005;
        int rank = (int)std::ceil(tail * run->scen_count - 1e-9);
        rank = std::max(1, std::min(rank, run->scen_count));
        HIPCHK(c, launch_stats(totals, run->node_count, run->scen_count, rank, out->stats, s));
    }
    return RR_OK;
}

int rr::host::run_items(rr_ctx *c, const rr_run *run, const std::vector<Item> &items, int K,
                        double *r0, int slot, bool fresh)
{
    if (items.empty()) return RR_OK;
    if (!supported_kj(K, 1) || slot < 0 || slot > 1) return fail(c, RR_EINVAL, "bad item launch");
    HIPCHK(c, hipSetDevice(c->device));
    Plan &pl = c->item_plan[slot];
    int rc;
    if (fresh || pl.n_items != (int)items.size()) {
        HIPCHK(c, hipStreamSynchronize(c->stream));   // the item buffers may be in use
        // Longest first, dealt round-robin to the per-XCD queues, taken in
        // windows of WG_THREADS/64 items: one queue taken item by item put
        // every wavefront's atomic on the same counter.
        std::vector<Item> sorted(items);
        auto steps = [&](const Item &it) {
            return c->tiles_host[it.tile].smax - (run->node_begin + it.node_rel) * run->node_step_m;
        };
        std::stable_sort(sorted.begin(), sorted.end(),
                         [&](const Item &a, const Item &b) { return steps(a) > steps(b); });
        const int nq = c->opt_xcd ? MAX_QUEUES : 1;
        std::vector<Item> dealt;
        dealt.reserve(sorted.size());
        std::vector<int> qbeg(nq + 1, 0);
        for (int q = 0; q < nq; ++q) {
            qbeg[q] = (int)dealt.size();
            for (size_t i = q; i < sorted.size(); i += nq) dealt.push_back(sorted[i]);
        }
        qbeg[nq] = (int)dealt.size();
        if ((rc = upload_vec(c, pl.items, dealt))) return rc;
        if ((rc = upload_vec(c, pl.qbeg, qbeg))) return rc;
        pl.n_queues = nq;
    }
    pl.K = K;
    pl.J = 1;
    pl.n_items = (int)items.size();
    pl.win = 1;
    pl.wg_per_cu = 2;
    pl.grid = std::max(1, std::min(c->n_cu * 2, (pl.n_items + WG_THREADS / 64 - 1) / (WG_THREADS / 64)));
    rr_run r = *run;
    r.out_mask = RR_OUT_R0;
    rr_outputs o;
    memset(&o, 0, sizeof o);
    o.r0 = r0;
    RecParams P = make_params(c, &r, &o, &pl, nullptr);
    const size_t lds = P.q_in_lds ? (size_t)P.n_q * sizeof(double) : 0;
    HIPCHK(c, launch_recurrence(K, 1, P, pl.grid, lds, c->stream));
    return RR_OK;
}

// Time one configuration for the autotuner: the minimum over `reps`
// measurements of `burst` back-to-back launches (per launch).
static int time_config(rr_ctx *c, const rr_run *run, const rr_outputs *out, const LaunchCfg &cfg,
                       double *partial, double *totals, float *ms, int reps = 3, int burst = 1)
{
    Plan *pl;
    int rc;
    if ((rc = build_plan(c, run, cfg, &pl))) return rc;
    hipEvent_t a, b;
    HIPCHK(c, hipEventCreate(&a));
    HIPCHK(c, hipEventCreate(&b));
    float best = 1e30f;
    for (int rep = 0; rep < reps; ++rep) {
        HIPCHK(c, hipEventRecord(a, c->stream));
        for (int i = 0; i < burst; ++i)
            if ((rc = enqueue_run(c, run, out, pl, partial, totals, c->stream, false))) return rc;
        HIPCHK(c, hipEventRecord(b, c->stream));
        HIPCHK(c, hipEventSynchronize(b));
        float t = 0;
        HIPCHK(c, hipEventElapsedTime(&t, a, b));
        best = std::min(best, t / (float)burst);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = best;
    return RR_OK;
}

// Launch shape: pinned options, else the autotuner's choice for this run shape
// (every candidate produces bitwise-identical results, so tuning runs write
// the real outputs).
static int choose_config(rr_ctx *c, const rr_run *run, const rr_outputs *out, double *partial,
                         double *totals, LaunchCfg *cfg_out)
{
    const bool path = (run->out_mask & RR_OUT_PATH) != 0;
    int Kfix = c->opt_k, Jfix = c->opt_j, wgfix = c->opt_wg;
    if (path || run->scen_count == 1) { Kfix = 1; Jfix = 1; }
    if (Kfix && Jfix && !supported_kj(Kfix, Jfix)) Jfix = 1;
    const int win0 = (c->opt_curve_share == 2 || c->opt_curve_share == -1) ? 1 : 0;
    if (Kfix && Jfix && wgfix && c->opt_ring >= 0 && c->opt_curve_share >= 0) {
        *cfg_out = LaunchCfg{Kfix, Jfix, wgfix, (c->opt_ring == 1 && ring_ok(c, Kfix, Jfix)) ? 1 : 0, win0};
        return RR_OK;
    }
    TuneKey key{run->node_count, run->scen_count, (run->out_mask & RR_OUT_ALL_STATES) ? 4 : 1,
                path ? 1 : 0, c->gen};
    auto it = c->tuned.find(key);
    if (it != c->tuned.end() && (!Kfix || it->second.K == Kfix) && (!Jfix || it->second.J == Jfix) &&
        (!wgfix || it->second.wg == wgfix) && (c->opt_ring < 0 || it->second.ring == c->opt_ring)) {
        *cfg_out = it->second;
        return RR_OK;
    }
    static const int kj_list[][2] = {{8, 4}, {16, 4}, {16, 2}, {8, 2}, {4, 4}, {32, 1}, {16, 1}, {8, 1}};
    std::vector<LaunchCfg> cands;
    for (auto &kj : kj_list) {
        if (Kfix && kj[0] != Kfix) continue;
        if (Jfix && kj[1] != Jfix) continue;
        if (kj[0] > std::max(4, run->scen_count)) continue;
        // scalar-load instances, then (where it runs) the curve-ring instance
        if (c->opt_ring != 1 || !ring_ok(c, kj[0], kj[1]))
            cands.push_back(LaunchCfg{kj[0], kj[1], wgfix ? wgfix : 2, 0, win0});
        if (c->opt_ring != 0 && ring_ok(c, kj[0], kj[1]))
            cands.push_back(LaunchCfg{kj[0], kj[1], wgfix ? wgfix : 2, 1, win0});
    }
    if (cands.empty())
        cands.push_back(LaunchCfg{Kfix ? Kfix : 8, Jfix ? Jfix : 1, wgfix ? wgfix : 2, 0, win0});
    LaunchCfg best = cands[0];
    float best_ms = 1e30f;
    int rc;
    std::vector<std::pair<float, LaunchCfg>> timed;
    auto try_cfg = [&](const LaunchCfg &cf) -> int {
        float ms;
        int r = time_config(c, run, out, cf, partial, totals, &ms);
        if (r) return r;
        timed.push_back({ms, cf});
        if (ms < best_ms) { best_ms = ms; best = cf; }
        return RR_OK;
    };
    // Every (K, J) shape at one and two workgroups per CU (registers decide
    // which fits better), then more workgroups for the best.
    for (const LaunchCfg &c0 : cands) {
        if (!supported_kj(c0.K, c0.J)) continue;
        for (int w : {1, 2}) {
            if (wgfix && w != wgfix) continue;
            LaunchCfg cf = c0;
            cf.wg = wgfix ? wgfix : w;
            if ((rc = try_cfg(cf))) return rc;
        }
    }
    if (!wgfix) {
        const LaunchCfg b0 = best;
        for (int w : {3, 4}) {
            LaunchCfg cf = b0;
            cf.wg = w;
            if ((rc = try_cfg(cf))) return rc;
        }
    }
    if (c->opt_curve_share == -1) {   // windows taken item by item instead
        LaunchCfg cf = best;
        cf.win = 0;
        if ((rc = try_cfg(cf))) return rc;
    }
    // The three fastest again, in turn, five times each, as bursts of eight
    // back-to-back launches (the steady state a graph replay sees): a clock
    // that was still rising during the first pass, or idle gaps between
    // single launches, must not decide between shapes a few per cent apart.
    if (timed.size() > 1) {
        std::stable_sort(timed.begin(), timed.end(),
                         [](const std::pair<float, LaunchCfg> &x, const std::pair<float, LaunchCfg> &y) {
                             return x.first < y.first;
                         });
        const size_t nf = std::min<size_t>(3, timed.size());
        std::vector<float> fin(nf, 1e30f);
        for (int rep = 0; rep < 5; ++rep) {
            for (size_t i = 0; i < nf; ++i) {
                float ms;
                if ((rc = time_config(c, run, out, timed[i].second, partial, totals, &ms, 1, 8))) return rc;
                fin[i] = std::min(fin[i], ms);
            }
        }
        size_t bi = 0;
        for (size_t i = 1; i < nf; ++i)
            if (fin[i] < fin[bi]) bi = i;
        best = timed[bi].second;
    }
    c->tuned[key] = best;
    *cfg_out = best;
    return RR_OK;
}

// Checks shared by the recurrence entry points: state, ranges, output mask
// and buffers (path capacity included).
static int check_run_outputs(rr_ctx *c, const rr_run *run, const rr_outputs *out)
{
    if (!run || !out) return fail(c, RR_EINVAL, "run and outputs must not be NULL");
    if (!c->has_basis || !c->has_pf) return fail(c, RR_ESTATE, "upload a basis and a portfolio first");
    HIPCHK(c, hipSetDevice(c->device));
    const uint32_t mask = run->out_mask;
    if (mask & ~(RR_OUT_R0 | RR_OUT_TOTALS | RR_OUT_PATH | RR_OUT_ALL_STATES | RR_OUT_STATS))
        return fail(c, RR_EINVAL, "unknown bits in out_mask");
    if (run->node_count < 0 || run->scen_count < 0) return fail(c, RR_EINVAL, "negative counts");
    if (run->node_begin < 0 || run->node_begin + run->node_count > c->n_nodes)
        return fail(c, RR_EINVAL, "node range [%d, %d) outside the basis (%d nodes)", run->node_begin,
                    run->node_begin + run->node_count, c->n_nodes);
    if (run->scen_begin < 0 || run->scen_begin + run->scen_count > c->n_scen)
        return fail(c, RR_EINVAL, "scenario range [%d, %d) outside the basis (%d scenarios)",
                    run->scen_begin, run->scen_begin + run->scen_count, c->n_scen);
    if (run->node_step_m < 0) return fail(c, RR_EINVAL, "node_step_m must be >= 0");
    if ((long long)(run->node_begin + run->node_count) * run->node_step_m > (1 << 24))
        return fail(c, RR_EINVAL, "node_step_m too large");
    if ((mask & RR_OUT_R0) && !out->r0 && c->n_user > 0)   // an empty portfolio has nothing to write
        return fail(c, RR_EINVAL, "RR_OUT_R0 needs outputs.r0");
    if ((mask & RR_OUT_TOTALS) && !out->totals) return fail(c, RR_EINVAL, "RR_OUT_TOTALS needs outputs.totals");
    if ((mask & RR_OUT_STATS) && !out->stats) return fail(c, RR_EINVAL, "RR_OUT_STATS needs outputs.stats");
    if ((mask & RR_OUT_ALL_STATES) && !(mask & RR_OUT_R0))
        return fail(c, RR_EINVAL, "RR_OUT_ALL_STATES needs RR_OUT_R0");
    if (mask & RR_OUT_STATS && !(run->tail >= 0.0 && run->tail < 1.0))
        return fail(c, RR_EINVAL, "tail must be in [0, 1)");
    if (mask & RR_OUT_PATH) {
        if (run->node_count != 1 || run->scen_count != 1)
            return fail(c, RR_EINVAL, "RR_OUT_PATH needs node_count == 1 and scen_count == 1");
        if (!out->path) return fail(c, RR_EINVAL, "RR_OUT_PATH needs outputs.path");
        int64_t need;
        rr_path_size(c, run->node_begin, run->node_step_m, &need);
        if (out->path_cap < need)
            return fail(c, RR_ERANGE, "path_cap %lld < %lld doubles needed", (long long)out->path_cap,
                        (long long)need);
    }
    return RR_OK;
}

extern "C" int rr_reserve_recurrence(rr_ctx *c, const rr_run *run, const rr_outputs *out)
{
    if (!c) return RR_EINVAL;
    int rc0 = check_run_outputs(c, run, out);
    if (rc0) return rc0;
    const uint32_t mask = run->out_mask;
    if (mask & RR_OUT_PATH) {
        if (c->path_off_node != run->node_begin || c->path_off_step != run->node_step_m ||
            c->path_off_gen != c->gen) {
            std::vector<long long> off((size_t)c->n_user + 1, 0);
            for (int i = 0; i < c->n_user; ++i)
                off[i + 1] = off[i] + std::max(c->h_term[i] - run->node_begin * run->node_step_m, 0) + 1;
            int rc = upload_vec(c, c->path_off, off);
            if (rc) return rc;
            c->path_off_node = run->node_begin;
            c->path_off_step = run->node_step_m;
            c->path_off_gen = c->gen;
            drop_graphs(c);
        }
    }
    if (run->node_count == 0 || run->scen_count == 0) return RR_OK;
    const bool need_tot = (mask & (RR_OUT_TOTALS | RR_OUT_STATS)) != 0;
    double *totals = nullptr;
    if (need_tot) {
        if (mask & RR_OUT_TOTALS) totals = out->totals;
        else {
            HIPCHK(c, c->totals_tmp.alloc((size_t)run->node_count * run->scen_count));
            totals = c->totals_tmp.p;
        }
    }
    if (c->n_user == 0) {   // nothing to value: zero totals and statistics
        if (totals) HIPCHK(c, launch_fill(totals, (long long)run->node_count * run->scen_count, 0.0, c->stream));
        if ((mask & RR_OUT_STATS)) HIPCHK(c, launch_fill(out->stats, 2LL * run->node_count, 0.0, c->stream));
        return RR_OK;
    }
    double *partial = nullptr;
    if (need_tot) {
        // per-tile partials, then the scratch of the chunked totals pass
        size_t np = (size_t)run->node_count * c->n_tiles * run->scen_count +
                    (size_t)totals_scratch_doubles(run->node_count, c->n_tiles, run->scen_count);
        if (np > c->partial.n) drop_graphs(c);
        HIPCHK(c, c->partial.alloc(np));
        partial = c->partial.p;
    }
    LaunchCfg cfg;
    int rc;
    if ((rc = choose_config(c, run, out, partial, totals, &cfg))) return rc;
    Plan *pl;
    if ((rc = build_plan(c, run, cfg, &pl))) return rc;
    c->last_k = cfg.K;
    c->last_j = cfg.J;
    c->last_wg = cfg.wg;
    c->last_ring = cfg.ring;
    c->last_win = cfg.win;
    c->last_qlds = tables_in_lds(c) ? 1 : 0;

    if (c->opt_graph && !c->opt_timing) {
        std::vector<uint64_t> key = {
            (uint64_t)(uintptr_t)pl, (uint64_t)pl->grid, (uint64_t)pl->ring, (uint64_t)pl->win,
            (uint64_t)run->node_begin,
            (uint64_t)run->node_count, (uint64_t)run->scen_begin, (uint64_t)run->scen_count,
            (uint64_t)run->node_step_m, (uint64_t)mask, (uint64_t)(uintptr_t)out->r0,
            (uint64_t)(uintptr_t)out->totals, (uint64_t)(uintptr_t)out->path,
            (uint64_t)(uintptr_t)out->stats, (uint64_t)(uintptr_t)partial,
            (uint64_t)(uintptr_t)totals, (uint64_t)c->gen};
        uint64_t tail_bits;
        memcpy(&tail_bits, &run->tail, 8);
        key.push_back(tail_bits);
        GraphEntry *ge = nullptr;
        for (auto &g : c->graphs)
            if (g.key == key) { ge = &g; break; }
        if (!ge) {
            if (c->graphs.size() >= 8) drop_graphs(c);
            GraphEntry g;
            g.key = key;
            HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            rc = enqueue_run(c, run, out, pl, partial, totals, c->cap_stream, false);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
            if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
            HIPCHK(c, e);
            g.graph = graph;
            HIPCHK(c, hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
            c->graphs.push_back(g);
            ge = &c->graphs.back();
        }
        HIPCHK(c, hipGraphLaunch(ge->exec, c->stream));
        return RR_OK;
    }
    return enqueue_run(c, run, out, pl, partial, totals, c->stream, c->opt_timing != 0);
}

// Launch shape of the allocation-free entry point, which cannot autotune
// (the autotuner builds and uploads candidate plans): pinned options, else
// the shape the autotuner chose for this run shape on an earlier
// rr_reserve_recurrence call, else 16 scenarios x 2 tiles per wavefront at
// one workgroup per CU (fewer scenarios: the largest K that fits).
static LaunchCfg noalloc_config(rr_ctx *c, const rr_run *run)
{
    const int win = (c->opt_curve_share == 2 || c->opt_curve_share == -1) ? 1 : 0;
    int K = c->opt_k, J = c->opt_j, wg = c->opt_wg;
    if (run->scen_count == 1) { K = 1; J = 1; }
    if (K && J && !supported_kj(K, J)) J = 1;
    if (K && J && wg)
        return LaunchCfg{K, J, wg, (c->opt_ring == 1 && ring_ok(c, K, J)) ? 1 : 0, win};
    TuneKey key{run->node_count, run->scen_count, (run->out_mask & RR_OUT_ALL_STATES) ? 4 : 1, 0, c->gen};
    auto it = c->tuned.find(key);
    if (it != c->tuned.end() && (!K || it->second.K == K) && (!J || it->second.J == J) &&
        (!wg || it->second.wg == wg))
        return it->second;
    if (!K) {
        K = 16;
        while (K > 1 && K > run->scen_count) K /= 2;
    }
    if (!J) J = supported_kj(K, 2) ? 2 : 1;
    return LaunchCfg{K, J, wg ? wg : 1, 0, win};
}

extern "C" int rr_reserve_recurrence_noalloc(rr_ctx *c, const rr_run *run, const rr_outputs *out)
{
    if (!c) return RR_EINVAL;
    if (run && (run->out_mask & RR_OUT_PATH))
        return fail(c, RR_EINVAL, "rr_reserve_recurrence_noalloc does not write paths (RR_OUT_PATH)");
    int rc = check_run_outputs(c, run, out);
    if (rc) return rc;
    if (!c->scratch) return fail(c, RR_EDEVICE, "no static scratch on device %d", c->device);
    if (run->node_count == 0 || run->scen_count == 0) return RR_OK;
    const uint32_t mask = run->out_mask;
    const long long ns = (long long)run->node_count * run->scen_count;
    const bool need_tot = (mask & (RR_OUT_TOTALS | RR_OUT_STATS)) != 0;
    const LaunchCfg cfg = noalloc_config(c, run);
    const int queues = c->opt_xcd ? MAX_QUEUES : 1;
    PlanKey key{run->node_begin, run->node_count, run->scen_begin, run->scen_count,
                run->node_step_m, cfg.K, cfg.J, queues, c->gen, cfg.wg};
    auto it = c->host_plans.find(key);
    if (it == c->host_plans.end()) {
        HostPlan hp;
        plan_lists(c, run, cfg, queues, hp.items, hp.qbeg);
        it = c->host_plans.emplace(key, std::move(hp)).first;
    }
    const HostPlan &hp = it->second;
    // Layout of the scratch, in doubles, each part 256-byte aligned:
    // counters, queue offsets, work items, totals (statistics without
    // RR_OUT_TOTALS), per-tile partial totals and the chunked-totals scratch.
    long long off = 0;
    auto take = [&](long long doubles) {
        const long long o = off;
        off += (doubles + 31) / 32 * 32;
        return o;
    };
    const long long o_cnt = take((MAX_QUEUES + 2) / 2);
    const long long o_qbeg = take(((long long)hp.qbeg.size() + 1) / 2);
    static_assert(sizeof(Item) % sizeof(double) == 0, "work items are whole doubles");
    const long long o_items = take((long long)hp.items.size() * (long long)(sizeof(Item) / sizeof(double)));
    const bool own_tot = need_tot && !(mask & RR_OUT_TOTALS);
    const long long o_tot = own_tot ? take(ns) : -1;
    const long long np = need_tot ? ns * c->n_tiles + totals_scratch_doubles(run->node_count, c->n_tiles,
                                                                               run->scen_count)
                                  : 0;
    const long long o_part = need_tot ? take(np) : -1;
    const long long cap = (long long)(NOALLOC_SCRATCH_BYTES / sizeof(double));
    if (off > cap)
        return fail(c, RR_ERANGE,
                    "this run needs %.1f MiB of scratch; rr_reserve_recurrence_noalloc has %lld MiB "
                    "(split the run into fewer nodes or scenarios, or use rr_reserve_recurrence)",
                    off * 8.0 / (1 << 20), (long long)(NOALLOC_SCRATCH_BYTES >> 20));
    double *S = c->scratch;
    double *totals = need_tot ? ((mask & RR_OUT_TOTALS) ? out->totals : S + o_tot) : nullptr;
    const hipStream_t st = c->stream;
    if (c->n_user == 0) {
        if (totals) HIPCHK(c, launch_fill(totals, ns, 0.0, st));
        if (mask & RR_OUT_STATS) HIPCHK(c, launch_fill(out->stats, 2LL * run->node_count, 0.0, st));
        return RR_OK;
    }
    // The array keeps the contents of the last call on this device: the queue
    // counters must start at zero (a kernel, not a memset node).
    int *counters = reinterpret_cast<int *>(S + o_cnt);
    HIPCHK(c, launch_fill_int(counters, MAX_QUEUES + 1, 0, st));
    HIPCHK(c, hipMemcpyAsync(S + o_qbeg, hp.qbeg.data(), hp.qbeg.size() * sizeof(int),
                             hipMemcpyHostToDevice, st));
    if (!hp.items.empty())
        HIPCHK(c, hipMemcpyAsync(S + o_items, hp.items.data(), hp.items.size() * sizeof(Item),
                                 hipMemcpyHostToDevice, st));
    Plan pl;
    pl.K = cfg.K;
    pl.J = cfg.J;
    pl.n_items = (int)hp.items.size();
    pl.n_queues = queues;
    pl.items_ext = reinterpret_cast<const Item *>(S + o_items);
    pl.qbeg_ext = reinterpret_cast<const int *>(S + o_qbeg);
    pl.counters_ext = counters;
    pl.wg_per_cu = cfg.wg;
    pl.ring = cfg.ring;
    pl.win = cfg.win;
    const int waves_per_wg = WG_THREADS / 64;
    pl.grid = std::max(1, std::min(c->n_cu * cfg.wg, (pl.n_items + waves_per_wg - 1) / waves_per_wg));
    c->last_k = cfg.K;
    c->last_j = cfg.J;
    c->last_wg = cfg.wg;
    c->last_ring = cfg.ring;
    c->last_win = cfg.win;
    c->last_qlds = tables_in_lds(c) ? 1 : 0;
    return enqueue_run(c, run, out, &pl, need_tot ? S + o_part : nullptr, totals, st, false);
}

extern "C" int rr_kernel_times(rr_ctx *c, double *ms, int32_t cap, int32_t *count)
{
    if (!c || !count) return RR_EINVAL;
    int n = 0;
    for (auto &e : c->ev_pending) {
        HIPCHK(c, hipEventSynchronize(e.second));
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, e.first, e.second));
        if (ms && n < cap) ms[n] = t;
        ++n;
        c->ev_free.push_back(e);
    }
    c->ev_pending.clear();
    *count = n;
    return RR_OK;
}

// Accessors used by the surrogate module (same library).
namespace rr {
}  // namespace rr
