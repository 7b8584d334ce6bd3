// Surrogate runtime: the rr_surrogate_* calls of include/rr.h.  Training data
// come from the exact recurrence on the loaded basis and portfolio; every
// per-row step (features, standardisation, forward, backward, Adam,
// inference, totals) runs in the kernels of rr_mlp.hip and rr_kernels.hip.
// The host fits the three curve components (Jacobi eigen-decomposition of a
// 50 x 50 covariance), keeps the model's small arrays, orders samples and
// plans the exact fallback.
#include "rr_ctx.h"
#include "rr_mlp.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

using namespace rr;
using namespace rr::host;
namespace M = rr::mlp;

namespace {

constexpr char kMagic[8] = {'R', 'R', 'S', 'U', 'R', 'R', '0', '1'};
constexpr char kMagicNode[8] = {'R', 'R', 'S', 'U', 'R', 'N', '0', '1'};   // node-level model
constexpr int kVersion = 1;
constexpr int kProducts[4] = {RR_SL_ANN, RR_JL_ANN, RR_TERM, RR_ENDOW};
constexpr int kChunk = 16;   // policies per work unit of the fused inference kernel
constexpr int kFbK = 8;      // scenarios per lane of the exact fallback items

struct BlobHeader {
    char magic[8];
    int32_t version, n_feat, k_in, hidden, n_tenors, n_factors, n_params, adam_step;
    int32_t signature[12];
    int32_t reserved[2];
};
static_assert(sizeof(BlobHeader) == 96, "blob header layout");
constexpr size_t kBlobDoubles = 4 * M::N_FEAT + 8 + M::N_TENORS + M::N_FACTORS * M::N_TENORS;
constexpr size_t kBlobBytes = sizeof(BlobHeader) + kBlobDoubles * 8 + 3 * (size_t)M::N_PARAMS * 4;

// splitmix64 (Steele, Lea and Flood, 2014).
struct SplitMix {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }   // (0, 1)
    double normal()   // Box-Muller
    {
        const double u = uniform(), v = uniform();
        return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
    }
    uint64_t below(uint64_t n) { return next() % n; }
};

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Eigen-decomposition of a symmetric matrix by cyclic Jacobi rotations
// (Golub and Van Loan, Sec. 8.5): a is overwritten, eigenvalues on its
// diagonal, eigenvectors in the columns of v.
void jacobi_eigen(std::vector<double> &a, std::vector<double> &v, int n)
{
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double x = a[(size_t)i * n + j] * a[(size_t)i * n + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {   // columns p, q
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - s * akq;
                    a[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {   // rows p, q
                    const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - s * aqk;
                    a[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = c * vkp - s * vkq;
                    v[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
}

}  // namespace

struct rr::Surrogate {
    // model, host copies
    bool has_model = false;
    int version = 0;                      // bumps on every model change
    std::vector<double> mu, sd, lo, hi;   // [N_FEAT]
    std::vector<double> tmu, tsd;         // [4] target statistics per one-hot product
    std::vector<double> zbar, evec;       // [N_TENORS], [N_FACTORS][N_TENORS]
    int32_t sig[12];
    int32_t adam_step = 0;

    // model, device
    DevBuf<float> master, adam_m, adam_v;
    DevBuf<uint16_t> w1t, w2t, w2n, w1_inf, w2_inf, w3_inf;
    DevBuf<float> w3e;
    DevBuf<double> d_mu, d_sd, d_lo, d_hi, d_zbar, d_evec, d_tmu, d_tsd;
    DevBuf<int> d_sig;

    // portfolio copies in upload order
    int pol_gen = -1;
    DevBuf<int> product, age1, age2, term, table1, table2, timing, patterned;
    DevBuf<double> amount, premium;

    // feature and inference workspaces
    DevBuf<double> seg, zcurves, sraw, praw;
    DevBuf<uint16_t> sfeat, pfeat, pfeat2;
    DevBuf<int> sok, pflag;
    DevBuf<double> partial, exact, totals_tmp, oscale, ooffset, ct_work;
    // node-level inference workspaces
    DevBuf<double> nraw, node_vals, node_dummy, node_X, node_T, node_means;
    DevBuf<float> node_y, node_t;
    DevBuf<uint16_t> node_xq;
    DevBuf<unsigned char> node_prod, node_fbmask;
    DevBuf<int> node_perm;
    DevBuf<int2> node_rowmap, node_pairs;
    DevBuf<long long> node_poff, node_roff;

    // fallback plan cache
    std::vector<uint64_t> plan_key;
    std::vector<Item> fb_items;     // exact fallback: tiles with a policy outside the box x every
                                    // block of kFbK scenarios, other tiles x the blocks holding a
                                    // scenario outside the box
    int64_t fb_rows = 0, in_rows = 0;

    // network workspaces (rows padded to 64)
    long long ws_rows = 0;
    DevBuf<uint16_t> xq, xqt, a1q, a1qt, a2q, a2qt, dz2q, dz2qt, dz1qt;
    DevBuf<float> z1, z2, y, dy, t, loss_part, p1, p2, grad, scal;

    M::Weights weights()
    {
        return M::Weights{master.p, w1t.p, w2t.p, w2n.p, w3e.p, w1_inf.p, w2_inf.p, w3_inf.p};
    }
    M::Norm norm()
    {
        return M::Norm{d_mu.p, d_sd.p, d_lo.p, d_hi.p, d_zbar.p, d_evec.p, d_sig.p, d_tmu.p, d_tsd.p};
    }
};

void rr::surrogate_destroy(Surrogate *s) { delete s; }

namespace {

Surrogate *sur_of(rr_ctx *c)
{
    if (!c->sur) c->sur = new Surrogate();
    return c->sur;
}

Surrogate *nsur_of(rr_ctx *c)
{
    if (!c->nsur) c->nsur = new Surrogate();
    return c->nsur;
}

int alloc_model(rr_ctx *c, Surrogate *S)
{
    HIPCHK(c, S->master.alloc(M::N_PARAMS));
    HIPCHK(c, S->adam_m.alloc(M::N_PARAMS));
    HIPCHK(c, S->adam_v.alloc(M::N_PARAMS));
    HIPCHK(c, S->w1t.alloc(M::HID * M::K_IN));
    HIPCHK(c, S->w2t.alloc(M::HID * M::HID));
    HIPCHK(c, S->w2n.alloc(M::HID * M::HID));
    HIPCHK(c, S->w1_inf.alloc(M::HID * M::K_IN));
    HIPCHK(c, S->w2_inf.alloc(M::HID * M::HID));
    HIPCHK(c, S->w3_inf.alloc(8 * 16 * 32));
    HIPCHK(c, S->w3e.alloc(M::HID));
    HIPCHK(c, S->d_sig.alloc(12));
    return RR_OK;
}

// Host model arrays -> device (standardisation, box, components, signature).
int upload_norm(rr_ctx *c, Surrogate *S)
{
    int rc;
    if ((rc = upload_vec(c, S->d_mu, S->mu))) return rc;
    if ((rc = upload_vec(c, S->d_sd, S->sd))) return rc;
    if ((rc = upload_vec(c, S->d_lo, S->lo))) return rc;
    if ((rc = upload_vec(c, S->d_hi, S->hi))) return rc;
    if ((rc = upload_vec(c, S->d_zbar, S->zbar))) return rc;
    if ((rc = upload_vec(c, S->d_evec, S->evec))) return rc;
    if ((rc = upload_vec(c, S->d_tmu, S->tmu))) return rc;
    if ((rc = upload_vec(c, S->d_tsd, S->tsd))) return rc;
    std::vector<int> sg(S->sig, S->sig + 12);
    if ((rc = upload_vec(c, S->d_sig, sg))) return rc;
    return RR_OK;
}

int sync_policies(rr_ctx *c, Surrogate *S)
{
    if (S->pol_gen == c->gen) return RR_OK;
    int rc;
    if ((rc = upload_vec(c, S->product, c->h_product))) return rc;
    if ((rc = upload_vec(c, S->age1, c->h_age1))) return rc;
    if ((rc = upload_vec(c, S->age2, c->h_age2))) return rc;
    if ((rc = upload_vec(c, S->term, c->h_term))) return rc;
    if ((rc = upload_vec(c, S->table1, c->h_table1))) return rc;
    if ((rc = upload_vec(c, S->table2, c->h_table2))) return rc;
    if ((rc = upload_vec(c, S->timing, c->h_timing))) return rc;
    if ((rc = upload_vec(c, S->amount, c->h_amount))) return rc;
    if ((rc = upload_vec(c, S->premium, c->h_premium))) return rc;
    if ((rc = upload_vec(c, S->patterned, c->h_patterned))) return rc;
    S->pol_gen = c->gen;
    return RR_OK;
}

M::Policies policies_of(Surrogate *S, int n)
{
    return M::Policies{n, S->product.p, S->age1.p, S->age2.p, S->term.p, S->table1.p,
                       S->table2.p, S->timing.p, S->amount.p, S->premium.p, S->patterned.p};
}

int check_run(rr_ctx *c, const rr_run *run)
{
    if (!run) return fail(c, RR_EINVAL, "run must not be NULL");
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
    return RR_OK;
}

// Features of every (node, scenario) and (node, policy) of a run.  With
// with_model, standardised features and flags; without, raw values only
// (curve scores 0) and policy flags 2 expired / 1 supported / 0 not.
int compute_features(rr_ctx *c, Surrogate *S, const rr_run *run, bool with_model, bool want_raw,
                     bool want_curves)
{
    const hipStream_t st = c->stream;
    const long long ns = (long long)run->node_count * run->scen_count;
    const long long np = (long long)run->node_count * c->n_user;
    int rc;
    if ((rc = sync_policies(c, S))) return rc;
    HIPCHK(c, S->seg.alloc((size_t)std::max(1LL, ns * M::N_TENORS)));
    HIPCHK(c, M::launch_zero_rates(c->v.p, c->n_steps, c->scen_pad, run->node_begin,
                                   run->node_count, run->scen_begin, run->scen_count, S->seg.p, st));
    if (want_curves) {
        HIPCHK(c, S->zcurves.alloc((size_t)std::max(1LL, ns * M::N_TENORS)));
        HIPCHK(c, M::launch_curves_out(c->v.p, c->n_steps, c->scen_pad, S->seg.p, run->node_begin,
                                       run->node_count, run->scen_begin, run->scen_count,
                                       S->zcurves.p, st));
    }
    M::Norm nm{};
    if (with_model) nm = S->norm();
    else {
        nm.zbar = S->d_zbar.p;     // components, when already fitted
        nm.evec = S->d_evec.p;
        nm.signature = S->d_sig.p;
    }
    if (want_raw) {
        HIPCHK(c, S->sraw.alloc((size_t)std::max(1LL, ns * 5)));
        HIPCHK(c, S->praw.alloc((size_t)std::max(1LL, np * 9)));
    }
    HIPCHK(c, S->sfeat.alloc((size_t)std::max(1LL, ns * 8)));
    HIPCHK(c, S->sok.alloc((size_t)std::max(1LL, ns)));
    HIPCHK(c, S->pfeat.alloc((size_t)std::max(1LL, np * 8)));
    HIPCHK(c, S->pfeat2.alloc((size_t)std::max(1LL, np)));
    HIPCHK(c, S->pflag.alloc((size_t)std::max(1LL, np)));
    HIPCHK(c, S->oscale.alloc((size_t)std::max(1LL, np)));
    HIPCHK(c, S->ooffset.alloc((size_t)std::max(1LL, np)));
    HIPCHK(c, M::launch_scen_features(c->v.p, c->n_steps, c->scen_pad, c->shock.p, S->seg.p,
                                      run->node_begin, run->node_count, run->scen_begin,
                                      run->scen_count, nm, want_raw ? S->sraw.p : nullptr,
                                      S->sfeat.p, S->sok.p, st));
    HIPCHK(c, M::launch_policy_features(policies_of(S, c->n_user), run->node_begin, run->node_count,
                                        run->node_step_m, nm, want_raw ? S->praw.p : nullptr,
                                        S->pfeat.p, S->pfeat2.p, S->pflag.p, S->oscale.p,
                                        S->ooffset.p, st));
    return RR_OK;
}

int ensure_ws(rr_ctx *c, Surrogate *S, long long rows)
{
    if (rows <= S->ws_rows) return RR_OK;
    const size_t r = (size_t)rows;
    HIPCHK(c, S->xq.alloc(r * M::K_IN));
    HIPCHK(c, S->xqt.alloc(r * M::K_IN));
    HIPCHK(c, S->a1q.alloc(r * M::HID));
    HIPCHK(c, S->a1qt.alloc(r * M::HID));
    HIPCHK(c, S->a2q.alloc(r * M::HID));
    HIPCHK(c, S->a2qt.alloc(r * M::HID));
    HIPCHK(c, S->dz2q.alloc(r * M::HID));
    HIPCHK(c, S->dz2qt.alloc(r * M::HID));
    HIPCHK(c, S->dz1qt.alloc(r * M::HID));
    HIPCHK(c, S->z1.alloc(r * M::HID));
    HIPCHK(c, S->z2.alloc(r * M::HID));
    HIPCHK(c, S->y.alloc(r));
    HIPCHK(c, S->dy.alloc(r));
    HIPCHK(c, S->t.alloc(r));
    HIPCHK(c, S->loss_part.alloc(r / 16 + 1));
    HIPCHK(c, S->p1.alloc((size_t)32 * M::K_IN * M::HID));
    HIPCHK(c, S->p2.alloc((size_t)32 * M::HID * M::HID));
    HIPCHK(c, S->grad.alloc(M::N_PARAMS));
    HIPCHK(c, S->scal.alloc(4));
    S->ws_rows = rows;
    return RR_OK;
}

long long pad64(long long n) { return (n + 63) / 64 * 64; }

// Forward over rows xq[n_pad][32]; with t, the loss (scaled by 1/n) goes to
// *loss_out and, with grads, the gradient to grad.
int network_pass(rr_ctx *c, Surrogate *S, const uint16_t *xq, long long n, long long n_pad,
                 const float *t, bool grads, float *grad, float *loss_out, float *y_out)
{
    const hipStream_t st = c->stream;
    const M::Weights w = S->weights();
    M::Gemm g{};
    g.A = xq;
    g.lda = M::K_IN;
    g.B = S->w1t.p;
    g.ldb = M::K_IN;
    g.M = (int)n_pad;
    g.N = M::HID;
    g.K = M::K_IN;
    g.splits = 1;
    g.bias = S->master.p + M::OFF_B1;
    g.Z = S->z1.p;
    g.Aq = S->a1q.p;
    g.AqT = grads ? S->a1qt.p : nullptr;
    g.ldt = n_pad;
    HIPCHK(c, M::launch_gemm(g, M::EPI_FWD, st));
    g.A = S->a1q.p;
    g.lda = M::HID;
    g.B = S->w2t.p;
    g.ldb = M::HID;
    g.K = M::HID;
    g.bias = S->master.p + M::OFF_B2;
    g.Z = S->z2.p;
    g.Aq = S->a2q.p;
    g.AqT = grads ? S->a2qt.p : nullptr;
    HIPCHK(c, M::launch_gemm(g, M::EPI_FWD, st));
    HIPCHK(c, M::launch_head(S->a2q.p, S->z2.p, w, t, (int)n_pad, (int)n, 1.0f / (float)n, grads,
                             y_out ? y_out : S->y.p, S->dy.p, t ? S->loss_part.p : nullptr,
                             S->dz2q.p, S->dz2qt.p, n_pad, st));
    if (t && loss_out)
        HIPCHK(c, M::launch_sum(S->loss_part.p, (int)(n_pad / 16), 1.0f / (float)n, loss_out, st));
    if (!grads) return RR_OK;
    // dZ1 = (dZ2 W2^T) * gelu'(Z1), stored transposed
    M::Gemm d{};
    d.A = S->dz2q.p;
    d.lda = M::HID;
    d.B = S->w2n.p;
    d.ldb = M::HID;
    d.M = (int)n_pad;
    d.N = M::HID;
    d.K = M::HID;
    d.splits = 1;
    d.Zin = S->z1.p;
    d.AqT = S->dz1qt.p;
    d.ldt = n_pad;
    HIPCHK(c, M::launch_gemm(d, M::EPI_DGELU, st));
    HIPCHK(c, M::launch_transpose_x(xq, (int)n_pad, S->xqt.p, n_pad, st));
    HIPCHK(c, M::launch_vec_grads(S->dz1qt.p, S->dz2qt.p, S->a2qt.p, S->dy.p, n_pad, (int)n_pad,
                                  grad, st));
    // weight gradients, split over the rows
    int splits = (int)std::max(1LL, std::min(32LL, n_pad / 256));
    while ((n_pad / 32) % splits) --splits;
    const int kspl = (int)(n_pad / splits);
    M::Gemm w2{};
    w2.A = S->a1qt.p;
    w2.lda = n_pad;
    w2.B = S->dz2qt.p;
    w2.ldb = n_pad;
    w2.M = M::HID;
    w2.N = M::HID;
    w2.K = kspl;
    w2.splits = splits;
    w2.C = S->p2.p;
    HIPCHK(c, M::launch_gemm(w2, M::EPI_PARTIAL, st));
    M::Gemm w1 = w2;
    w1.A = S->xqt.p;
    w1.B = S->dz1qt.p;
    w1.M = M::K_IN;
    w1.C = S->p1.p;
    HIPCHK(c, M::launch_gemm(w1, M::EPI_PARTIAL, st));
    HIPCHK(c, M::launch_reduce_grads(S->p1.p, splits, S->p2.p, splits, grad, st));
    return RR_OK;
}

int adam_step(rr_ctx *c, Surrogate *S, const float *grad, float lr)
{
    S->adam_step += 1;
    const double c1 = 1.0 / (1.0 - std::pow(0.9, S->adam_step));
    const double c2 = 1.0 / (1.0 - std::pow(0.999, S->adam_step));
    HIPCHK(c, M::launch_adam(S->master.p, S->adam_m.p, S->adam_v.p, grad, lr, (float)c1, (float)c2,
                             c->stream));
    HIPCHK(c, M::launch_export(S->weights(), c->stream));
    S->version += 1;
    return RR_OK;
}

int check_model(rr_ctx *c, Surrogate *S)
{
    if (!S || !S->has_model) return fail(c, RR_ESTATE, "no surrogate model loaded");
    return RR_OK;
}

// Fresh weights: W ~ N(0, 1/fan_in) over the real inputs, zero biases.
std::vector<float> init_params(uint64_t seed)
{
    SplitMix rng{seed ^ 0x5eed5eed12345678ull};
    std::vector<float> p(M::N_PARAMS, 0.f);
    for (int k = 0; k < M::N_FEAT; ++k)
        for (int h = 0; h < M::HID; ++h)
            p[M::OFF_W1 + k * M::HID + h] = (float)(rng.normal() / std::sqrt((double)M::N_FEAT));
    for (int i = 0; i < M::HID * M::HID; ++i)
        p[M::OFF_W2 + i] = (float)(rng.normal() / std::sqrt((double)M::HID));
    for (int i = 0; i < M::HID; ++i) p[M::OFF_W3 + i] = (float)(rng.normal() / std::sqrt((double)M::HID));
    return p;
}

// Per one-hot product, the (table1, table2, timing) of the training policies
// (level payments only: patterned annuities are outside the domain).
int product_signature(rr_ctx *c, int32_t sig[12])
{
    for (int j = 0; j < 4; ++j) {
        sig[3 * j] = -1;
        sig[3 * j + 1] = -1;
        sig[3 * j + 2] = -1;
        bool seen = false;
        for (int i = 0; i < c->n_user; ++i) {
            if (c->h_product[i] != kProducts[j] || c->h_patterned[i]) continue;
            const int t1 = c->h_table1[i];
            const int t2 = kProducts[j] == RR_JL_ANN ? c->h_table2[i] : -1;
            const int tm = (kProducts[j] == RR_SL_ANN || kProducts[j] == RR_JL_ANN) ? c->h_timing[i] : -1;
            if (!seen) {
                sig[3 * j] = t1;
                sig[3 * j + 1] = t2;
                sig[3 * j + 2] = tm;
                seen = true;
            } else if (sig[3 * j] != t1 || sig[3 * j + 1] != t2 || sig[3 * j + 2] != tm) {
                return fail(c, RR_EINVAL,
                            "training policies of product %d use several (table, timing) "
                            "combinations (policy %d)", kProducts[j], i);
            }
        }
    }
    return RR_OK;
}

// Curve components from the zero-rate curves of every (node, scenario).
int fit_components(rr_ctx *c, Surrogate *S, long long ns)
{
    std::vector<double> z((size_t)ns * M::N_TENORS);
    HIPCHK(c, hipMemcpyAsync(z.data(), S->zcurves.p, z.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int T = M::N_TENORS;
    S->zbar.assign(T, 0.0);
    for (long long r = 0; r < ns; ++r)
        for (int j = 0; j < T; ++j) S->zbar[j] += z[(size_t)r * T + j];
    for (int j = 0; j < T; ++j) S->zbar[j] /= (double)ns;
    std::vector<double> cov((size_t)T * T, 0.0);
    std::vector<double> d(T);
    for (long long r = 0; r < ns; ++r) {
        for (int j = 0; j < T; ++j) d[j] = z[(size_t)r * T + j] - S->zbar[j];
        for (int i = 0; i < T; ++i)
            for (int j = 0; j < T; ++j) cov[(size_t)i * T + j] += d[i] * d[j];
    }
    for (auto &x : cov) x /= (double)ns;
    std::vector<double> vec;
    jacobi_eigen(cov, vec, T);
    std::vector<int> order(T);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return cov[(size_t)a * T + a] > cov[(size_t)b * T + b];
    });
    S->evec.assign((size_t)M::N_FACTORS * T, 0.0);
    for (int f = 0; f < M::N_FACTORS; ++f) {
        const int col = order[f];
        int arg = 0;
        for (int j = 1; j < T; ++j)
            if (std::fabs(vec[(size_t)j * T + col]) > std::fabs(vec[(size_t)arg * T + col])) arg = j;
        const double sgn = vec[(size_t)arg * T + col] < 0 ? -1.0 : 1.0;
        for (int j = 0; j < T; ++j) S->evec[(size_t)f * T + j] = sgn * vec[(size_t)j * T + col];
    }
    int rc;
    if ((rc = upload_vec(c, S->d_zbar, S->zbar))) return rc;
    if ((rc = upload_vec(c, S->d_evec, S->evec))) return rc;
    return RR_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Model blob
// ---------------------------------------------------------------------------
static int get_weights(rr_ctx *c, Surrogate *S, const char *magic, void *host, size_t bytes,
                       size_t *needed)
{
    if (!c) return RR_EINVAL;
    if (needed) *needed = kBlobBytes;
    int rc;
    if ((rc = check_model(c, S))) return rc;
    if (!host) return RR_OK;
    if (bytes < kBlobBytes) return fail(c, RR_ERANGE, "blob needs %zu bytes", kBlobBytes);
    HIPCHK(c, hipSetDevice(c->device));
    BlobHeader h;
    memset(&h, 0, sizeof h);
    memcpy(h.magic, magic, 8);
    h.version = kVersion;
    h.n_feat = M::N_FEAT;
    h.k_in = M::K_IN;
    h.hidden = M::HID;
    h.n_tenors = M::N_TENORS;
    h.n_factors = M::N_FACTORS;
    h.n_params = M::N_PARAMS;
    h.adam_step = S->adam_step;
    memcpy(h.signature, S->sig, sizeof h.signature);
    unsigned char *o = (unsigned char *)host;
    memcpy(o, &h, sizeof h);
    double *dd = (double *)(o + sizeof h);
    size_t k = 0;
    for (int j = 0; j < M::N_FEAT; ++j) dd[k++] = S->mu[j];
    for (int j = 0; j < M::N_FEAT; ++j) dd[k++] = S->sd[j];
    for (int j = 0; j < M::N_FEAT; ++j) dd[k++] = S->lo[j];
    for (int j = 0; j < M::N_FEAT; ++j) dd[k++] = S->hi[j];
    for (int j = 0; j < 4; ++j) dd[k++] = S->tmu[j];
    for (int j = 0; j < 4; ++j) dd[k++] = S->tsd[j];
    for (int j = 0; j < M::N_TENORS; ++j) dd[k++] = S->zbar[j];
    for (int j = 0; j < M::N_FACTORS * M::N_TENORS; ++j) dd[k++] = S->evec[j];
    float *ff = (float *)(dd + kBlobDoubles);
    HIPCHK(c, hipMemcpyAsync(ff, S->master.p, M::N_PARAMS * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ff + M::N_PARAMS, S->adam_m.p, M::N_PARAMS * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ff + 2 * M::N_PARAMS, S->adam_v.p, M::N_PARAMS * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return RR_OK;
}

static int set_weights(rr_ctx *c, bool node, const void *host, size_t bytes)
{
    if (!c) return RR_EINVAL;
    if (!host || bytes < kBlobBytes) return fail(c, RR_EINVAL, "blob must hold %zu bytes", kBlobBytes);
    BlobHeader h;
    memcpy(&h, host, sizeof h);
    if (memcmp(h.magic, node ? kMagicNode : kMagic, 8) != 0 || h.version != kVersion)
        return fail(c, RR_EINVAL, node ? "not a node-level surrogate blob" : "not a surrogate blob");
    if (h.n_feat != M::N_FEAT || h.k_in != M::K_IN || h.hidden != M::HID || h.n_tenors != M::N_TENORS ||
        h.n_factors != M::N_FACTORS || h.n_params != M::N_PARAMS || h.adam_step < 0)
        return fail(c, RR_EINVAL, "blob dimensions do not match this library");
    const unsigned char *o = (const unsigned char *)host;
    const double *dd = (const double *)(o + sizeof h);
    for (size_t k = 0; k < kBlobDoubles; ++k)
        if (!std::isfinite(dd[k])) return fail(c, RR_EINVAL, "non-finite value in the blob's statistics");
    for (int j = 0; j < M::N_FEAT; ++j) {
        if (!(dd[M::N_FEAT + j] > 0.0)) return fail(c, RR_EINVAL, "feature %d: standard deviation must be > 0", j);
        if (dd[2 * M::N_FEAT + j] > dd[3 * M::N_FEAT + j]) return fail(c, RR_EINVAL, "feature %d: box lo > hi", j);
    }
    for (int j = 0; j < 4; ++j)
        if (!(dd[4 * M::N_FEAT + 4 + j] > 0.0))
            return fail(c, RR_EINVAL, "target standard deviation %d must be > 0", j);
    const float *ff = (const float *)(dd + kBlobDoubles);
    for (size_t k = 0; k < 3 * (size_t)M::N_PARAMS; ++k)
        if (!std::isfinite(ff[k])) return fail(c, RR_EINVAL, "non-finite parameter at %zu", k);
    for (int j = 0; j < 4; ++j)
        if (h.signature[3 * j] < -1 || h.signature[3 * j + 1] < -1 || h.signature[3 * j + 2] < -1)
            return fail(c, RR_EINVAL, "bad product signature");
    HIPCHK(c, hipSetDevice(c->device));
    Surrogate *S = node ? nsur_of(c) : sur_of(c);
    int rc;
    if ((rc = alloc_model(c, S))) return rc;
    size_t k = 0;
    S->mu.assign(dd + k, dd + k + M::N_FEAT); k += M::N_FEAT;
    S->sd.assign(dd + k, dd + k + M::N_FEAT); k += M::N_FEAT;
    S->lo.assign(dd + k, dd + k + M::N_FEAT); k += M::N_FEAT;
    S->hi.assign(dd + k, dd + k + M::N_FEAT); k += M::N_FEAT;
    S->tmu.assign(dd + k, dd + k + 4); k += 4;
    S->tsd.assign(dd + k, dd + k + 4); k += 4;
    S->zbar.assign(dd + k, dd + k + M::N_TENORS); k += M::N_TENORS;
    S->evec.assign(dd + k, dd + k + M::N_FACTORS * M::N_TENORS);
    memcpy(S->sig, h.signature, sizeof S->sig);
    S->adam_step = h.adam_step;
    if ((rc = upload_norm(c, S))) return rc;
    HIPCHK(c, hipMemcpy(S->master.p, ff, M::N_PARAMS * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(S->adam_m.p, ff + M::N_PARAMS, M::N_PARAMS * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(S->adam_v.p, ff + 2 * M::N_PARAMS, M::N_PARAMS * 4, hipMemcpyHostToDevice));
    HIPCHK(c, M::launch_export(S->weights(), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    S->has_model = true;
    S->version += 1;
    return RR_OK;
}

extern "C" int rr_surrogate_get_weights(rr_ctx *c, void *host, size_t bytes, size_t *needed)
{
    return c ? get_weights(c, c->sur, kMagic, host, bytes, needed) : RR_EINVAL;
}

extern "C" int rr_surrogate_set_weights(rr_ctx *c, const void *host, size_t bytes)
{
    return set_weights(c, false, host, bytes);
}

extern "C" int rr_node_surrogate_get_weights(rr_ctx *c, void *host, size_t bytes, size_t *needed)
{
    return c ? get_weights(c, c->nsur, kMagicNode, host, bytes, needed) : RR_EINVAL;
}

extern "C" int rr_node_surrogate_set_weights(rr_ctx *c, const void *host, size_t bytes)
{
    return set_weights(c, true, host, bytes);
}

// ---------------------------------------------------------------------------
// Layer-level calls
// ---------------------------------------------------------------------------
extern "C" int rr_surrogate_forward(rr_ctx *c, const float *z, int64_t n, float *y)
{
    if (!c) return RR_EINVAL;
    int rc;
    if ((rc = check_model(c, c->sur))) return rc;
    if (n < 0 || n > (1LL << 26)) return fail(c, RR_EINVAL, "n out of range");
    if (n == 0) return RR_OK;
    if (!z || !y) return fail(c, RR_EINVAL, "z and y must not be NULL");
    HIPCHK(c, hipSetDevice(c->device));
    Surrogate *S = c->sur;
    const long long n_pad = pad64(n);
    if ((rc = ensure_ws(c, S, n_pad))) return rc;
    HIPCHK(c, M::launch_prep_input(z, (int)n, (int)n_pad, S->xq.p, c->stream));
    if ((rc = network_pass(c, S, S->xq.p, n, n_pad, nullptr, false, nullptr, nullptr, S->y.p))) return rc;
    HIPCHK(c, hipMemcpyAsync(y, S->y.p, (size_t)n * 4, hipMemcpyDeviceToDevice, c->stream));
    return RR_OK;
}

extern "C" int rr_surrogate_gradients(rr_ctx *c, const float *z, const float *t, int64_t n,
                                      float *grad, float *loss)
{
    if (!c) return RR_EINVAL;
    int rc;
    if ((rc = check_model(c, c->sur))) return rc;
    if (n < 1 || n > (1LL << 26)) return fail(c, RR_EINVAL, "n out of range");
    if (!z || !t || !grad) return fail(c, RR_EINVAL, "z, t and grad must not be NULL");
    HIPCHK(c, hipSetDevice(c->device));
    Surrogate *S = c->sur;
    const long long n_pad = pad64(n);
    if ((rc = ensure_ws(c, S, n_pad))) return rc;
    HIPCHK(c, M::launch_prep_input(z, (int)n, (int)n_pad, S->xq.p, c->stream));
    HIPCHK(c, hipMemcpyAsync(S->t.p, t, (size_t)n * 4, hipMemcpyDeviceToDevice, c->stream));
    return network_pass(c, S, S->xq.p, n, n_pad, S->t.p, true, grad, loss ? loss : S->scal.p, nullptr);
}

extern "C" int rr_surrogate_adam_step(rr_ctx *c, const float *grad, float lr)
{
    if (!c) return RR_EINVAL;
    int rc;
    if ((rc = check_model(c, c->sur))) return rc;
    if (!grad) return fail(c, RR_EINVAL, "grad must not be NULL");
    if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(c, RR_EINVAL, "lr must be finite and >= 0");
    HIPCHK(c, hipSetDevice(c->device));
    return adam_step(c, c->sur, grad, lr);
}

extern "C" int rr_surrogate_features(rr_ctx *c, const rr_run *run, double *pol, double *scen,
                                     int32_t *pflag, int32_t *sflag)
{
    if (!c) return RR_EINVAL;
    int rc;
    if ((rc = check_model(c, c->sur))) return rc;
    if (!c->has_basis || !c->has_pf) return fail(c, RR_ESTATE, "upload a basis and a portfolio first");
    if ((rc = check_run(c, run))) return rc;
    if (run->node_count == 0 || run->scen_count == 0) return RR_OK;
    HIPCHK(c, hipSetDevice(c->device));
    Surrogate *S = c->sur;
    if ((rc = compute_features(c, S, run, true, true, false))) return rc;
    const size_t ns = (size_t)run->node_count * run->scen_count;
    const size_t np = (size_t)run->node_count * c->n_user;
    const hipStream_t st = c->stream;
    if (pol && np) HIPCHK(c, hipMemcpyAsync(pol, S->praw.p, np * 9 * 8, hipMemcpyDeviceToDevice, st));
    if (scen) HIPCHK(c, hipMemcpyAsync(scen, S->sraw.p, ns * 5 * 8, hipMemcpyDeviceToDevice, st));
    if (pflag && np) HIPCHK(c, hipMemcpyAsync(pflag, S->pflag.p, np * 4, hipMemcpyDeviceToDevice, st));
    if (sflag) HIPCHK(c, hipMemcpyAsync(sflag, S->sok.p, ns * 4, hipMemcpyDeviceToDevice, st));
    return RR_OK;
}

// ---------------------------------------------------------------------------
// Training
// ---------------------------------------------------------------------------
// Training of the per-scenario model (rows: node, scenario, policy, state)
// or, with node_level, of the node-level model (rows: node, policy; features
// of the node's scenarios and the state-0 reserves averaged over them).
static int train_impl(rr_ctx *c, const rr_train_cfg *cfg, rr_train_report *rep, bool node_level)
{
    if (!c) return RR_EINVAL;
    if (!cfg) return fail(c, RR_EINVAL, "cfg must not be NULL");
    if (!c->has_basis || !c->has_pf) return fail(c, RR_ESTATE, "upload a basis and a portfolio first");
    int rc;
    const rr_run *run = &cfg->run;
    if ((rc = check_run(c, run))) return rc;
    if (cfg->epochs < 1) return fail(c, RR_EINVAL, "epochs must be >= 1");
    if (cfg->batch < 64 || cfg->batch % 64 || cfg->batch > (1 << 20))
        return fail(c, RR_EINVAL, "batch must be a positive multiple of 64 (<= 2^20)");
    if (!(cfg->lr > 0.f) || !std::isfinite(cfg->lr) || !(cfg->lr_final >= 0.f) || !std::isfinite(cfg->lr_final))
        return fail(c, RR_EINVAL, "lr must be > 0 and lr_final >= 0");
    if (!(cfg->holdout >= 0.f && cfg->holdout <= 0.5f)) return fail(c, RR_EINVAL, "holdout must be in [0, 0.5]");
    if (cfg->init != 0 && cfg->init != 1) return fail(c, RR_EINVAL, "init must be 0 or 1");
    Surrogate *S = node_level ? nsur_of(c) : sur_of(c);
    if (!cfg->init && !S->has_model) return fail(c, RR_ESTATE, "init = 0 needs a loaded model");
    if (run->node_count == 0 || run->scen_count == 0 || c->n_user == 0)
        return fail(c, RR_EINVAL, "the run has no samples");
    HIPCHK(c, hipSetDevice(c->device));
    const hipStream_t st = c->stream;
    const double t0 = now_ms();
    if ((rc = alloc_model(c, S))) return rc;

    int32_t sig[12];
    if (cfg->init) {
        if ((rc = product_signature(c, sig))) return rc;
        memcpy(S->sig, sig, sizeof sig);
        std::vector<int> sg(sig, sig + 12);
        if ((rc = upload_vec(c, S->d_sig, sg))) return rc;
    }

    // Exact reserves of every state (the node-level model: state 0).
    const int n = c->n_user;
    const long long ns = (long long)run->node_count * run->scen_count;
    DevBuf<double> r_all;
    HIPCHK(c, r_all.alloc((size_t)ns * n * (node_level ? 1 : 4)));
    {
        rr_run er = *run;
        er.out_mask = node_level ? RR_OUT_R0 : (RR_OUT_R0 | RR_OUT_ALL_STATES);
        rr_outputs eo;
        memset(&eo, 0, sizeof eo);
        eo.r0 = r_all.p;
        if ((rc = rr_reserve_recurrence(c, &er, &eo))) return rc;
    }
    // Curve components (fitted on these scenarios for a new model).
    if (cfg->init) {
        if ((rc = compute_features(c, S, run, false, false, true))) return rc;
        if ((rc = fit_components(c, S, ns))) return rc;
    }
    if ((rc = compute_features(c, S, run, false, true, false))) return rc;

    // Sample rows: (node, scenario, policy, state), policies with flag 1.
    std::vector<int> flags((size_t)run->node_count * n);
    HIPCHK(c, hipMemcpyAsync(flags.data(), S->pflag.p, flags.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    std::vector<int2> pairs;
    std::vector<long long> pair_off(run->node_count + 1, 0), row_off(run->node_count + 1, 0);
    for (int k = 0; k < run->node_count; ++k) {
        for (int i = 0; i < n; ++i) {
            if (flags[(size_t)k * n + i] != 1) continue;
            const int states = (c->h_product[i] == RR_JL_ANN && !node_level) ? 3 : 1;
            for (int j = 0; j < states; ++j) pairs.push_back(make_int2(i, j));
        }
        pair_off[k + 1] = (long long)pairs.size();
        row_off[k + 1] = row_off[k] + (pair_off[k + 1] - pair_off[k]) * (node_level ? 1 : run->scen_count);
    }
    const long long N = row_off[run->node_count];
    const long long n_hold_min = (long long)std::ceil((double)cfg->holdout * (double)N);
    const long long n_train = (N - n_hold_min) / cfg->batch * cfg->batch;
    if (n_train < cfg->batch)
        return fail(c, RR_EINVAL, "%lld samples: fewer than one batch for training", N);
    const long long n_hold = N - n_train;
    DevBuf<int2> d_pairs;
    DevBuf<long long> d_poff, d_roff;
    if ((rc = upload_vec(c, d_pairs, pairs))) return rc;
    if ((rc = upload_vec(c, d_poff, pair_off))) return rc;
    if ((rc = upload_vec(c, d_roff, row_off))) return rc;
    DevBuf<double> X, T;
    HIPCHK(c, X.alloc((size_t)N * M::N_FEAT));
    HIPCHK(c, T.alloc((size_t)N));
    if (node_level) {
        // One row per (node, policy): the node's scenario features and the
        // state-0 reserves averaged over its scenarios, laid out as a run of
        // one scenario per node with four state slots.
        DevBuf<double> nraw, rmean;
        HIPCHK(c, nraw.alloc((size_t)run->node_count * 5));
        HIPCHK(c, rmean.alloc((size_t)run->node_count * n * 4));
        HIPCHK(c, launch_fill(rmean.p, (long long)run->node_count * n * 4, 0.0, st));
        HIPCHK(c, M::launch_mean_inner(S->sraw.p, run->node_count, run->scen_count, 5, nraw.p, 5, st));
        HIPCHK(c, M::launch_mean_inner(r_all.p, (long long)run->node_count * n, run->scen_count, 1,
                                       rmean.p, 4, st));
        HIPCHK(c, M::launch_samples(S->praw.p, nraw.p, rmean.p, S->amount.p, d_pairs.p, d_poff.p,
                                    d_roff.p, run->node_count, n, 1, N, X.p, T.p, st));
        HIPCHK(c, hipStreamSynchronize(st));
    } else {
        HIPCHK(c, M::launch_samples(S->praw.p, S->sraw.p, r_all.p, S->amount.p, d_pairs.p, d_poff.p,
                                    d_roff.p, run->node_count, n, run->scen_count, N, X.p, T.p, st));
    }
    r_all.release();

    // Standardisation and box (new model).
    if (cfg->init) {
        DevBuf<double> work, stats;
        HIPCHK(c, work.alloc((size_t)M::STAT_BLOCKS * M::STAT_COLS * 4));
        HIPCHK(c, stats.alloc((size_t)M::STAT_COLS * 4));
        HIPCHK(c, M::launch_colstats(X.p, T.p, N, work.p, stats.p, st));
        std::vector<double> hs(M::STAT_COLS * 4);
        HIPCHK(c, hipMemcpyAsync(hs.data(), stats.p, hs.size() * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        S->mu.resize(M::N_FEAT);
        S->sd.resize(M::N_FEAT);
        S->lo.resize(M::N_FEAT);
        S->hi.resize(M::N_FEAT);
        for (int j = 0; j < M::N_FEAT; ++j) {
            S->mu[j] = hs[j * 4 + 0];
            S->sd[j] = hs[j * 4 + 1] > 0.0 ? hs[j * 4 + 1] : 1.0;
            S->lo[j] = hs[j * 4 + 2];
            S->hi[j] = hs[j * 4 + 3];
        }
        S->tmu.assign(4, 0.0);
        S->tsd.assign(4, 1.0);
        for (int j = 0; j < 4; ++j) {
            const double *cs = &hs[(M::N_FEAT + 1 + j) * 4];
            S->tmu[j] = cs[0];
            S->tsd[j] = cs[1] > 0.0 ? cs[1] : 1.0;
        }
        if ((rc = upload_norm(c, S))) return rc;
    }

    // Dataset in a seeded random order; the holdout is its tail.
    SplitMix rng{cfg->seed};
    std::vector<int> perm((size_t)N);
    std::iota(perm.begin(), perm.end(), 0);
    for (long long i = N - 1; i > 0; --i) std::swap(perm[i], perm[rng.below((uint64_t)i + 1)]);
    DevBuf<int> d_perm;
    if ((rc = upload_vec(c, d_perm, perm))) return rc;
    const long long N_pad = pad64(N);
    DevBuf<uint16_t> xq;
    DevBuf<float> tq;
    DevBuf<unsigned char> prod;
    HIPCHK(c, xq.alloc((size_t)N_pad * M::K_IN));
    HIPCHK(c, tq.alloc((size_t)N_pad));
    HIPCHK(c, prod.alloc((size_t)N_pad));
    HIPCHK(c, hipMemsetAsync(xq.p, 0, (size_t)N_pad * M::K_IN * 2, st));
    HIPCHK(c, hipMemsetAsync(tq.p, 0, (size_t)N_pad * 4, st));
    HIPCHK(c, M::launch_build(X.p, T.p, N, d_perm.p, S->d_mu.p, S->d_sd.p, S->d_tmu.p,
                              S->d_tsd.p, xq.p, tq.p, prod.p, st));
    HIPCHK(c, hipStreamSynchronize(st));
    X.release();
    T.release();

    if (cfg->init) {
        std::vector<float> p0 = init_params(cfg->seed);
        HIPCHK(c, hipMemcpy(S->master.p, p0.data(), p0.size() * 4, hipMemcpyHostToDevice));
        HIPCHK(c, hipMemset(S->adam_m.p, 0, M::N_PARAMS * 4));
        HIPCHK(c, hipMemset(S->adam_v.p, 0, M::N_PARAMS * 4));
        S->adam_step = 0;
    }
    HIPCHK(c, M::launch_export(S->weights(), st));
    S->has_model = true;
    S->version += 1;
    const double t1 = now_ms();

    // Epochs: batches in a new random order each epoch, cosine step size.
    const long long B = cfg->batch;
    const long long n_batches = n_train / B;
    const long long total = n_batches * cfg->epochs;
    if ((rc = ensure_ws(c, S, std::max(B, pad64(std::max(n_hold, 1LL)))))) return rc;
    DevBuf<float> hist;
    HIPCHK(c, hist.alloc((size_t)total));
    std::vector<long long> order((size_t)n_batches);
    std::iota(order.begin(), order.end(), 0);
    long long step = 0;
    for (int e = 0; e < cfg->epochs; ++e) {
        for (long long i = n_batches - 1; i > 0; --i) std::swap(order[i], order[rng.below((uint64_t)i + 1)]);
        for (long long b = 0; b < n_batches; ++b, ++step) {
            const long long r0 = order[b] * B;
            const double frac = total > 1 ? (double)step / (double)(total - 1) : 1.0;
            const float lr = (float)(cfg->lr_final + 0.5 * (cfg->lr - cfg->lr_final) * (1.0 + std::cos(3.141592653589793 * frac)));
            if ((rc = network_pass(c, S, xq.p + r0 * M::K_IN, B, B, tq.p + r0, true, S->grad.p,
                                   hist.p + step, nullptr)))
                return rc;
            if ((rc = adam_step(c, S, S->grad.p, lr))) return rc;
        }
    }
    std::vector<float> h((size_t)total);
    HIPCHK(c, hipMemcpyAsync(h.data(), hist.p, h.size() * 4, hipMemcpyDeviceToHost, st));
    // Holdout loss.
    float hold = 0.f;
    if (n_hold > 0) {
        const long long hp = pad64(n_hold);
        if ((rc = network_pass(c, S, xq.p + n_train * M::K_IN, n_hold, hp, tq.p + n_train, false,
                               nullptr, S->scal.p, nullptr)))
            return rc;
        HIPCHK(c, hipMemcpyAsync(&hold, S->scal.p, 4, hipMemcpyDeviceToHost, st));
    }
    // Output calibration: per product, shift the target mean by the mean
    // residual of the trained network over the training rows (the least-
    // squares offset given the network).
    double calib[4] = {0.0, 0.0, 0.0, 0.0};
    {
        const long long rb = M::residual_blocks((int)B);
        DevBuf<double> part;
        HIPCHK(c, part.alloc((size_t)(n_batches * rb * 8)));
        for (long long b = 0; b < n_batches; ++b) {
            if ((rc = network_pass(c, S, xq.p + b * B * M::K_IN, B, B, nullptr, false, nullptr,
                                   nullptr, S->y.p)))
                return rc;
            HIPCHK(c, M::launch_residuals(S->y.p, tq.p + b * B, prod.p + b * B, (int)B,
                                          part.p + b * rb * 8, st));
        }
        std::vector<double> hp((size_t)(n_batches * rb * 8));
        HIPCHK(c, hipMemcpyAsync(hp.data(), part.p, hp.size() * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        for (int j = 0; j < 4; ++j) {
            double a = 0.0, cnt = 0.0;
            for (long long b = 0; b < n_batches * rb; ++b) {
                a += hp[(size_t)b * 8 + j];
                cnt += hp[(size_t)b * 8 + 4 + j];
            }
            if (cnt > 0.0) calib[j] = a / cnt;
            S->tmu[j] += S->tsd[j] * calib[j];
        }
        if ((rc = upload_norm(c, S))) return rc;
        S->version += 1;
    }
    HIPCHK(c, hipStreamSynchronize(st));
    const double t2 = now_ms();
    if (rep) {
        memset(rep, 0, sizeof *rep);
        rep->n_samples = N;
        rep->n_train = n_train;
        rep->n_holdout = n_hold;
        rep->steps = (int32_t)total;
        double f = 0.0, l = 0.0;
        for (long long i = 0; i < n_batches; ++i) {
            f += h[(size_t)i];
            l += h[(size_t)(total - n_batches + i)];
        }
        rep->first_loss = (float)(f / (double)n_batches);
        rep->final_loss = (float)(l / (double)n_batches);
        rep->holdout_loss = hold;
        for (int j = 0; j < 4; ++j) rep->calibration[j] = (float)calib[j];
        rep->data_ms = t1 - t0;
        rep->train_ms = t2 - t1;
    }
    return RR_OK;
}

extern "C" int rr_surrogate_train(rr_ctx *c, const rr_train_cfg *cfg, rr_train_report *rep)
{
    return train_impl(c, cfg, rep, false);
}

extern "C" int rr_node_surrogate_train(rr_ctx *c, const rr_train_cfg *cfg, rr_train_report *rep)
{
    return train_impl(c, cfg, rep, true);
}

// ---------------------------------------------------------------------------
// Inference
// ---------------------------------------------------------------------------
extern "C" int rr_surrogate_infer(rr_ctx *c, const rr_run *run, const rr_outputs *out,
                                  rr_infer_report *rep)
{
    if (!c) return RR_EINVAL;
    int rc;
    if ((rc = check_model(c, c->sur))) return rc;
    if (!c->has_basis || !c->has_pf) return fail(c, RR_ESTATE, "upload a basis and a portfolio first");
    if ((rc = check_run(c, run))) return rc;
    if (!out) return fail(c, RR_EINVAL, "outputs must not be NULL");
    const uint32_t mask = run->out_mask;
    if (mask & ~(RR_OUT_R0 | RR_OUT_TOTALS | RR_OUT_STATS))
        return fail(c, RR_EINVAL, "the surrogate produces RR_OUT_R0, RR_OUT_TOTALS and RR_OUT_STATS only");
    if ((mask & RR_OUT_R0) && !out->r0 && c->n_user > 0) return fail(c, RR_EINVAL, "RR_OUT_R0 needs outputs.r0");
    if ((mask & RR_OUT_TOTALS) && !out->totals) return fail(c, RR_EINVAL, "RR_OUT_TOTALS needs outputs.totals");
    if ((mask & RR_OUT_STATS) && !out->stats) return fail(c, RR_EINVAL, "RR_OUT_STATS needs outputs.stats");
    if ((mask & RR_OUT_STATS) && !(run->tail >= 0.0 && run->tail < 1.0))
        return fail(c, RR_EINVAL, "tail must be in [0, 1)");
    if (rep) memset(rep, 0, sizeof *rep);
    if (run->node_count == 0 || run->scen_count == 0) return RR_OK;
    HIPCHK(c, hipSetDevice(c->device));
    Surrogate *S = c->sur;
    const hipStream_t st = c->stream;
    const int n = c->n_user;
    const long long ns = (long long)run->node_count * run->scen_count;
    double *totals = nullptr;
    if (mask & (RR_OUT_TOTALS | RR_OUT_STATS)) {
        if (mask & RR_OUT_TOTALS) totals = out->totals;
        else {
            HIPCHK(c, S->totals_tmp.alloc((size_t)ns));
            totals = S->totals_tmp.p;
        }
    }
    if (n == 0) {
        if (totals) HIPCHK(c, launch_fill(totals, ns, 0.0, st));
        if (mask & RR_OUT_STATS) HIPCHK(c, launch_fill(out->stats, 2LL * run->node_count, 0.0, st));
        return RR_OK;
    }
    if ((rc = compute_features(c, S, run, true, false, false))) return rc;

    // Fallback plan: work items of the exact kernel covering every row outside the box.
    // The scenario flags depend on the curve values, so a regeneration of the
    // curves in place (same sizes, same gen) invalidates the plan too.
    const std::vector<uint64_t> key = {(uint64_t)c->gen, (uint64_t)c->curve_gen, (uint64_t)S->version,
                                       (uint64_t)run->node_begin, (uint64_t)run->node_count,
                                       (uint64_t)run->scen_begin, (uint64_t)run->scen_count,
                                       (uint64_t)run->node_step_m};
    const bool fresh = key != S->plan_key;
    if (fresh) {
        std::vector<int> pf((size_t)run->node_count * n), so((size_t)ns);
        HIPCHK(c, hipMemcpyAsync(pf.data(), S->pflag.p, pf.size() * 4, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(so.data(), S->sok.p, so.size() * 4, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        std::vector<Item> fb_items;
        int64_t fb = 0, in = 0;
        for (int k = 0; k < run->node_count; ++k) {
            std::vector<char> bad_tile(c->n_tiles, 0), bad_scen(run->scen_count, 0);
            int64_t live = 0, live_ok = 0, nbad_scen = 0;
            for (int i = 0; i < n; ++i) {
                const int f = pf[(size_t)k * n + i];
                if (f == 2) continue;
                ++live;
                if (f == 1) ++live_ok;
                else bad_tile[c->slot_of_user[i] / TILE] = 1;
            }
            for (int s = 0; s < run->scen_count; ++s)
                if (!so[(size_t)k * run->scen_count + s]) { bad_scen[s] = 1; ++nbad_scen; }
            in += live_ok * (run->scen_count - nbad_scen);
            fb += live * run->scen_count - live_ok * (run->scen_count - nbad_scen);
            // Blocks of kFbK scenarios holding one outside the box: the
            // block's other rows are computed too and later overwritten by
            // the network (one launch for both kinds of fallback rows).
            std::vector<char> bad_block((run->scen_count + kFbK - 1) / kFbK, 0);
            for (int s = 0; s < run->scen_count; ++s)
                if (bad_scen[s]) bad_block[s / kFbK] = 1;
            for (int tl = 0; tl < c->n_tiles; ++tl)
                for (int b = 0; b < (int)bad_block.size(); ++b)
                    if (bad_tile[tl] || bad_block[b]) fb_items.push_back(Item{k, tl, b * kFbK, 1});
        }
        S->fb_items.swap(fb_items);
        S->fb_rows = fb;
        S->in_rows = in;
        S->plan_key = key;
    }
    double *exact = nullptr;
    if (!S->fb_items.empty()) {
        if (mask & RR_OUT_R0) exact = out->r0;
        else {
            HIPCHK(c, S->exact.alloc((size_t)ns * n));
            exact = S->exact.p;
        }
        if ((rc = run_items(c, run, S->fb_items, kFbK, exact, 0, fresh))) return rc;
    }
    if (S->fb_rows > 0 && !exact)   // k_infer would read exact rows nobody computed
        return fail(c, RR_EDEVICE, "surrogate fallback plan has %lld rows but no work items",
                    (long long)S->fb_rows);
    const int n_chunks = (n + kChunk - 1) / kChunk;
    HIPCHK(c, S->partial.alloc((size_t)run->node_count * n_chunks * run->scen_count));
    M::Infer f{};
    f.node_count = run->node_count;
    f.scen_count = run->scen_count;
    f.n = n;
    f.chunk = kChunk;
    f.pfeat = S->pfeat.p;
    f.pfeat2 = S->pfeat2.p;
    f.pflag = S->pflag.p;
    f.sfeat = S->sfeat.p;
    f.sok = S->sok.p;
    f.scale = S->oscale.p;
    f.offset = S->ooffset.p;
    f.r0 = (mask & RR_OUT_R0) ? out->r0 : nullptr;
    f.exact = exact;
    f.partial = S->partial.p;
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (c->opt_timing) {   // events around the fused kernel, read by rr_kernel_times
        if (!c->ev_free.empty()) {
            ev = c->ev_free.back();
            c->ev_free.pop_back();
        } else {
            HIPCHK(c, hipEventCreate(&ev.first));
            HIPCHK(c, hipEventCreate(&ev.second));
        }
        HIPCHK(c, hipEventRecord(ev.first, st));
    }
    HIPCHK(c, M::launch_infer(f, S->weights(), st));
    if (c->opt_timing) {
        HIPCHK(c, hipEventRecord(ev.second, st));
        c->ev_pending.push_back(ev);
    }
    if (totals) {
        HIPCHK(c, S->ct_work.alloc((size_t)M::chunk_totals_work(run->node_count, run->scen_count)));
        HIPCHK(c, M::launch_chunk_totals(S->partial.p, run->node_count, n_chunks, run->scen_count,
                                         S->ct_work.p, totals, st));
    }
    if (mask & RR_OUT_STATS) {
        const double tail = run->tail > 0.0 ? run->tail : 0.005;
        int rank = (int)std::ceil(tail * run->scen_count - 1e-9);
        rank = std::max(1, std::min(rank, run->scen_count));
        HIPCHK(c, launch_stats(totals, run->node_count, run->scen_count, rank, out->stats, st));
    }
    if (rep) {
        rep->n_in_range = S->in_rows;
        rep->n_fallback = S->fb_rows;
    }
    return RR_OK;
}

// ---------------------------------------------------------------------------
// Node-level model: scenario-averaged reserves per (node, policy)
// ---------------------------------------------------------------------------
extern "C" int rr_node_surrogate_infer(rr_ctx *c, const rr_run *run, double *node_r0,
                                       double *node_totals, rr_infer_report *rep)
{
    if (!c) return RR_EINVAL;
    int rc;
    if ((rc = check_model(c, c->nsur))) return rc;
    if (!c->has_basis || !c->has_pf) return fail(c, RR_ESTATE, "upload a basis and a portfolio first");
    if ((rc = check_run(c, run))) return rc;
    if (rep) memset(rep, 0, sizeof *rep);
    if (run->node_count == 0) return RR_OK;
    if (run->scen_count == 0) return fail(c, RR_EINVAL, "node features need at least one scenario");
    HIPCHK(c, hipSetDevice(c->device));
    Surrogate *S = c->nsur;
    const hipStream_t st = c->stream;
    const int n = c->n_user;
    const int K = run->node_count;
    const long long nk = (long long)K * n;
    double *vals = node_r0;
    if (!vals) {
        HIPCHK(c, S->node_vals.alloc((size_t)std::max(1LL, nk)));
        vals = S->node_vals.p;
    }
    if (nk > 0) HIPCHK(c, launch_fill(vals, nk, 0.0, st));   // expired policies: 0
    if (n == 0) {
        if (node_totals) HIPCHK(c, launch_fill(node_totals, K, 0.0, st));
        return RR_OK;
    }
    if ((rc = compute_features(c, S, run, true, true, false))) return rc;
    HIPCHK(c, S->nraw.alloc((size_t)K * 5));
    HIPCHK(c, M::launch_mean_inner(S->sraw.p, K, run->scen_count, 5, S->nraw.p, 5, st));
    std::vector<double> hn((size_t)K * 5);
    std::vector<int> pf((size_t)nk);
    HIPCHK(c, hipMemcpyAsync(hn.data(), S->nraw.p, hn.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(pf.data(), S->pflag.p, pf.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    // A node is in the model's domain when its mean scenario features (8..12)
    // and the state-0 one-hot (13..15) lie in the training box.
    const double st0[3] = {1.0, 0.0, 0.0};
    std::vector<int2> rowmap, pairs;
    std::vector<long long> poff(K + 1, 0), roff(K + 1, 0);
    std::vector<unsigned char> fbmask((size_t)nk, 0);
    int64_t n_fb = 0;
    for (int k = 0; k < K; ++k) {
        bool ok = true;
        for (int j = 0; j < 5; ++j) {
            const double x = hn[(size_t)k * 5 + j];
            ok = ok && x >= S->lo[8 + j] && x <= S->hi[8 + j];
        }
        for (int j = 0; j < 3; ++j) ok = ok && st0[j] >= S->lo[13 + j] && st0[j] <= S->hi[13 + j];
        for (int i = 0; i < n; ++i) {
            const int f = pf[(size_t)k * n + i];
            if (f == 1 && ok) {
                rowmap.push_back(make_int2(k, i));
                pairs.push_back(make_int2(i, 0));
            } else if (f != 2) {
                fbmask[(size_t)k * n + i] = 1;
                ++n_fb;
            }
        }
        poff[k + 1] = (long long)pairs.size();
        roff[k + 1] = poff[k + 1];
    }
    const long long N = (long long)rowmap.size();
    if (N > 0) {
        const long long N_pad = pad64(N);
        if ((rc = upload_vec(c, S->node_rowmap, rowmap))) return rc;
        if ((rc = upload_vec(c, S->node_pairs, pairs))) return rc;
        if ((rc = upload_vec(c, S->node_poff, poff))) return rc;
        if ((rc = upload_vec(c, S->node_roff, roff))) return rc;
        std::vector<int> perm((size_t)N);
        std::iota(perm.begin(), perm.end(), 0);
        if ((rc = upload_vec(c, S->node_perm, perm))) return rc;
        HIPCHK(c, S->node_dummy.alloc((size_t)nk * 4));
        HIPCHK(c, launch_fill(S->node_dummy.p, nk * 4, 0.0, st));
        HIPCHK(c, S->node_X.alloc((size_t)N * M::N_FEAT));
        HIPCHK(c, S->node_T.alloc((size_t)N));
        HIPCHK(c, S->node_xq.alloc((size_t)N_pad * M::K_IN));
        HIPCHK(c, S->node_t.alloc((size_t)N_pad));
        HIPCHK(c, S->node_prod.alloc((size_t)N_pad));
        HIPCHK(c, S->node_y.alloc((size_t)N_pad));
        HIPCHK(c, hipMemsetAsync(S->node_xq.p, 0, (size_t)N_pad * M::K_IN * 2, st));
        HIPCHK(c, M::launch_samples(S->praw.p, S->nraw.p, S->node_dummy.p, S->amount.p,
                                    S->node_pairs.p, S->node_poff.p, S->node_roff.p, K, n, 1, N,
                                    S->node_X.p, S->node_T.p, st));
        HIPCHK(c, M::launch_build(S->node_X.p, S->node_T.p, N, S->node_perm.p, S->d_mu.p, S->d_sd.p,
                                  S->d_tmu.p, S->d_tsd.p, S->node_xq.p, S->node_t.p,
                                  S->node_prod.p, st));
        const long long B = 65536;   // rows per network pass
        if ((rc = ensure_ws(c, S, B))) return rc;
        for (long long r0 = 0; r0 < N; r0 += B) {
            const long long nb = std::min(B, N - r0);
            if ((rc = network_pass(c, S, S->node_xq.p + r0 * M::K_IN, nb, pad64(nb), nullptr, false,
                                   nullptr, nullptr, S->node_y.p + r0)))
                return rc;
        }
        HIPCHK(c, M::launch_node_scatter(S->node_y.p, S->node_rowmap.p, N, n, S->oscale.p,
                                         S->ooffset.p, vals, st));
    }
    if (n_fb > 0) {
        // Exact scenario averages of the fallback rows: the reserves on the
        // node's mean discount curve (linearity in the discount products).
        HIPCHK(c, S->node_means.alloc((size_t)nk));
        if ((rc = rr_node_expected_reserves(c, run, S->node_means.p, nullptr))) return rc;
        if ((rc = upload_vec(c, S->node_fbmask, fbmask))) return rc;
        HIPCHK(c, M::launch_select(S->node_means.p, S->node_fbmask.p, nk, vals, st));
    }
    if (node_totals) HIPCHK(c, M::launch_row_sums(vals, K, n, node_totals, st));
    if (rep) {
        rep->n_in_range = N;
        rep->n_fallback = n_fb;
    }
    return RR_OK;
}
