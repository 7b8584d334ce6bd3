/*
 * Reserve oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU evaluation of prospective reserves of
 * non-unit-linked life policies, written from Tucker & Bull, "An efficient
 * algorithm for the calculation of reserves for non-unit linked life
 * policies" (arXiv 1401.1757).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code with the
 * GPU library.
 *
 * Two evaluations are provided:
 *   - orc_reserves: the general vector recurrence, Eq. (3.1), applied densely
 *     (full n x n transition matrices, every state kept, no zero-reserve-state
 *     reduction) and backward from the boundary condition (Sec. 3.8.2);
 *   - orc_reserve_path_summation: the reserve summation, Eq. (3.5), evaluated
 *     directly at every time step, O(S^2) per policy (Sec. 3.8.1), used only
 *     to check the recurrence on tiny inputs.
 *
 * Readings of the paper (where it is silent or ambiguous):
 *   - W row index = state at the start of the step (the explicit matrices of
 *     Sec. 2.4.2 and 4 and the per-state relation, Eq. (3.7)); the entry
 *     (j, i) is the probability of moving from j to i.
 *   - Each cash-flow type is its own stream with its own timing f; the
 *     streams are summed (Eq. (3.5) is linear in c).  Premiums are paid at
 *     f = 0 in state 0, annuity payments at f = 0 or 1 (policy timing), death
 *     benefits at f = 1 in the died-in-step state.
 *   - For f in (0, 1) the fractional death probability is f*q (uniform
 *     distribution of deaths) and the discount is v^f; annuities with timing
 *     2 pay at the basis's fraction f of each month.
 *   - Time t counts months since the node; life l has attained age
 *     age_l + node*node_step + t (equivalent to the paper's age-shift form by
 *     the cash-flow shift identity, Eq. (3.2)).
 *   - Node shock m multiplies every monthly q, capped at 1.
 *   - Annuity payment patterns (the representative portfolio of Sec. 5.3):
 *     a policy anniversary falls a months after node 0 (1 <= a <= 12) and
 *     every 12 months after; with escalation rate e every payment at a time
 *     T (months after node 0) carries the factor (1+e)^n(T), n(T) the number
 *     of anniversaries in (0, T]; monthly policies pay amount/12 each month,
 *     annual ones pay amount at each anniversary only.  The time-varying
 *     annuity stream c_t of Eq. (3.1) is the level stream times this factor
 *     at the payment time (t for f = 0, t + 1 for f = 1).
 *   - A cash-flow-table policy (one life) pays amount x cf[row][T] at the
 *     end of step T (months since node 0) if alive then, plus the level
 *     premium in advance; its boundary reserve is 0.
 *   - A policy whose remaining term at the node is <= 0 has expired: all its
 *     outputs are 0 and it is left out of totals.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Product codes (input format). */
enum {
    O_SL_ANN = 0, O_JL_ANN = 1, O_REV_ANN = 2, O_LS_ANN = 3,
    O_TERM = 4, O_ENDOW = 5, O_ENDOW_ASSUR = 6, O_CF_TABLE = 7,
    O_JL_ENDOW = 8, O_JL_ASSUR1 = 9, O_JL_ASSUR2 = 10, O_MARKOV = 11,
    O_JL3_ANN = 12, O_LS3_ANN = 13, O_N_PRODUCTS = 14
};

#define ORC_MAX_STATES 9
#define ORC_OUT_STATES 4

typedef struct {
    int n_ages;
    int n_tables;
    const double *q;        /* [n_tables][n_ages] monthly death probability */
    int n_nodes;
    int n_scen;
    int n_steps;
    const double *v;        /* [n_nodes][n_scen][n_steps] one-step discount */
    const double *shock;    /* [n_nodes] multiplier on q, or NULL */
    double frac;            /* payment point of timing-2 annuities within the month, in (0, 1) */
} orc_basis;

typedef struct {
    int n;
    const int32_t *product;
    const int32_t *age1;
    const int32_t *age2;
    const int32_t *term;
    const int32_t *table1;
    const int32_t *table2;
    const int32_t *timing;   /* 0: annuity at f = 0, 1: at f = 1 */
    const double *amount;    /* annual annuity amount, or sum assured */
    const double *premium;   /* level monthly premium, paid in advance */
    const double *escalation;/* annuity escalation rate per anniversary, or NULL */
    const int32_t *anniv;    /* months from node 0 to the first anniversary, or NULL */
    const int32_t *annual;   /* 1: one payment a year, at anniversaries; or NULL */
    const int32_t *cf_row;   /* O_CF_TABLE: row of the cash-flow table, or NULL */
    const double *cf;        /* [n_cf_rows][cf_len] cash flow per unit amount, or NULL */
    int n_cf_rows;
    int cf_len;
    /* Uploaded Markov models (O_MARKOV; table1 = model): one-step matrices
     * mk_w[model][age][m][m] by attained age in months (row = state at the
     * start of the month) and benefits mk_c[model][m] per unit amount, paid
     * at the end of a month that ends in the state. */
    int mk_models;
    int mk_states;
    int mk_ages;
    const double *mk_w;
    const double *mk_c;
    /* Life 3 of the three-life products (NULL when there are none). */
    const int32_t *age3;
    const int32_t *table3;
} orc_portfolio;

/* A contract in the paper's state-space form (Sec. 3.1, Sec. 4). */
typedef struct {
    int n_lives;
    int life_model;                     /* 2: alive/dead; 3: alive/died-in-step/dead */
    int n_states;
    double f_ann;                       /* timing of the annuity stream */
    double c_ann[ORC_MAX_STATES];       /* annuity stream, at f_ann */
    double c_ben[ORC_MAX_STATES];       /* death benefit stream, at f = 1 */
    double c_prem[ORC_MAX_STATES];      /* premium stream, at f = 0 */
    double boundary[ORC_MAX_STATES];    /* reserve vector at the end of the term */
    int gross;                          /* absolute values of every cash flow */
} orc_contract;

/* ------------------------------------------------------------------------ */
/* Transition matrices (Sec. 4.1, 4.1.3, 4.2, 4.3).                          */
/* ------------------------------------------------------------------------ */

/* One life over a fraction g of a step, death probability q over the whole
 * step.  2-state model (Sec. 4.1): [[gp, gq], [0, 1]].  3-state model
 * (Sec. 4.1.3): [[gp, gq, 0], [0, 0, 1], [0, 0, 1]]. */
static int life_matrix(int model, double q, double g, double *W)
{
    double gq = g * q;
    double gp = 1.0 - gq;
    if (model == 2) {
        W[0] = gp;  W[1] = gq;
        W[2] = 0.0; W[3] = 1.0;
        return 2;
    }
    W[0] = gp;  W[1] = gq;  W[2] = 0.0;
    W[3] = 0.0; W[4] = 0.0; W[5] = 1.0;
    W[6] = 0.0; W[7] = 0.0; W[8] = 1.0;
    return 3;
}

/* Kronecker product C = A (na x na) (x) B (nb x nb). */
static void kron(const double *A, int na, const double *B, int nb, double *C)
{
    int n = na * nb;
    for (int i1 = 0; i1 < na; ++i1)
        for (int j1 = 0; j1 < na; ++j1)
            for (int i2 = 0; i2 < nb; ++i2)
                for (int j2 = 0; j2 < nb; ++j2)
                    C[(i1 * nb + i2) * n + (j1 * nb + j2)] = A[i1 * na + j1] * B[i2 * nb + j2];
}

/* W for m independent lives by the Kronecker recursion of Sec. 4.3,
 * starting from the 1 x 1 matrix (1).  Life 1 is the most significant digit
 * of the state label (binary labels of Sec. 2.4.2, ternary of Sec. 4.2.3).
 * Returns the number of states. */
int orc_build_w(int n_lives, int model, const double *q, double g, double *W)
{
    double acc[ORC_MAX_STATES * ORC_MAX_STATES];
    double tmp[ORC_MAX_STATES * ORC_MAX_STATES];
    double L[9];
    int n = 1;
    acc[0] = 1.0;
    for (int l = 0; l < n_lives; ++l) {
        int nl = life_matrix(model, q[l], g, L);
        if (n * nl > ORC_MAX_STATES) return -1;
        kron(acc, n, L, nl, tmp);
        n *= nl;
        memcpy(acc, tmp, sizeof(double) * n * n);
    }
    memcpy(W, acc, sizeof(double) * n * n);
    return n;
}

/* y = A x for an n x n matrix. */
static void matvec(const double *A, const double *x, int n, double *y)
{
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += A[j * n + i] * x[i];
        y[j] = s;
    }
}

/* C = A B for n x n matrices. */
static void matmul(const double *A, const double *B, int n, double *C)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
            C[i * n + j] = s;
        }
}

/* ------------------------------------------------------------------------ */
/* Contracts (Sec. 4).                                                       */
/* ------------------------------------------------------------------------ */

/* Fill the state model, cash-flow vectors and boundary condition of one
 * policy.  With gross != 0 every amount is taken positive, so the result is
 * PV(benefits) + PV(premiums). */
int orc_contract_of(int product, int timing, double amount, double premium,
                    int gross, orc_contract *k)
{
    memset(k, 0, sizeof(*k));
    double prem = gross ? fabs(premium) : -premium;
    double pay = (gross ? fabs(amount) : amount) / 12.0;    /* monthly annuity */
    double sa = gross ? fabs(amount) : amount;
    if (timing < 0 || timing > 2) return -1;
    k->f_ann = timing == 2 ? 0.5 : (double)timing;   /* 2: the basis's fraction, set by contract_for */
    switch (product) {
    case O_SL_ANN:       /* Sec. 4.1.1: c = (theta, 0) */
        k->n_lives = 1; k->life_model = 2; k->n_states = 2;
        k->c_ann[0] = pay;
        break;
    case O_ENDOW:        /* Sec. 4.1.2: boundary (1, 0) times SA */
        k->n_lives = 1; k->life_model = 2; k->n_states = 2;
        k->boundary[0] = sa;
        break;
    case O_TERM:         /* Sec. 4.1.3: c = (0, 1, 0) times SA, boundary 0 */
        k->n_lives = 1; k->life_model = 3; k->n_states = 3;
        k->c_ben[1] = sa;
        break;
    case O_ENDOW_ASSUR:  /* term assurance with the pure-endowment boundary */
        k->n_lives = 1; k->life_model = 3; k->n_states = 3;
        k->c_ben[1] = sa;
        k->boundary[0] = sa;
        break;
    case O_JL_ANN:       /* Sec. 4.2.1 b: c = (1, 0, 0, 0) */
        k->n_lives = 2; k->life_model = 2; k->n_states = 4;
        k->c_ann[0] = pay;
        break;
    case O_REV_ANN:      /* Sec. 4.2.1 a: c = (0, 0, 1, 0) */
        k->n_lives = 2; k->life_model = 2; k->n_states = 4;
        k->c_ann[2] = pay;
        break;
    case O_LS_ANN:       /* Sec. 4.2.1 c: c = (1, 1, 1, 0) */
        k->n_lives = 2; k->life_model = 2; k->n_states = 4;
        k->c_ann[0] = pay; k->c_ann[1] = pay; k->c_ann[2] = pay;
        break;
    case O_JL_ENDOW:     /* Sec. 4.2.2: two-life pure endowment, boundary (1, 0, 0, 0) x SA */
        k->n_lives = 2; k->life_model = 2; k->n_states = 4;
        k->boundary[0] = sa;
        break;
    case O_JL_ASSUR1:    /* Sec. 4.2.3, 9-state model: benefit on the first death,
                            c = (0, 1, 0, 1, 1, 0, 0, 0, 0) x SA */
        k->n_lives = 2; k->life_model = 3; k->n_states = 9;
        k->c_ben[1] = sa; k->c_ben[3] = sa; k->c_ben[4] = sa;
        break;
    case O_JL_ASSUR2:    /* Sec. 4.2.3: benefit on the second death,
                            c = (0, 0, 0, 0, 1, 1, 0, 1, 0) x SA */
        k->n_lives = 2; k->life_model = 3; k->n_states = 9;
        k->c_ben[4] = sa; k->c_ben[5] = sa; k->c_ben[7] = sa;
        break;
    case O_JL3_ANN:      /* Sec. 4.3: three lives, 2^3 = 8 states (binary labels, life 1
                            the high digit); joint life: paid while all three are alive */
        k->n_lives = 3; k->life_model = 2; k->n_states = 8;
        k->c_ann[0] = pay;
        break;
    case O_LS3_ANN:      /* Sec. 4.3: last survivor of three: paid in every state with a
                            living life, c = (1, 1, 1, 1, 1, 1, 1, 0) */
        k->n_lives = 3; k->life_model = 2; k->n_states = 8;
        for (int j = 0; j < 7; ++j) k->c_ann[j] = pay;
        break;
    case O_MARKOV:       /* Sec. 4.5: an uploaded state model; the benefit vector
                            and the size are set by contract_for */
        k->n_lives = 1; k->life_model = 2; k->n_states = 2;
        k->f_ann = 1.0;
        break;
    case O_CF_TABLE:     /* single life, c_t = amount x table value, at f = 1
                            (Sec. 4.6: c_t holds the nominal amounts) */
        k->n_lives = 1; k->life_model = 2; k->n_states = 2;
        k->f_ann = 1.0;
        k->c_ann[0] = gross ? fabs(amount) : amount;
        break;
    default:
        return -1;
    }
    k->c_prem[0] = prem;   /* premiums while every life is alive */
    k->gross = gross;
    return 0;
}

static double q_at(const orc_basis *b, int table, int age, double m)
{
    double q = b->q[(size_t)table * b->n_ages + age];
    double s = m * q;
    return s < 1.0 ? s : 1.0;
}

/* Per-life death probabilities over step t (q[3]: lives 1-3). */
static void step_q(const orc_basis *b, const orc_portfolio *p, int i,
                   int age_shift, double m, int t, double *q)
{
    q[0] = q[1] = q[2] = 0.0;
    if (p->product[i] == O_MARKOV) return;   /* an uploaded model carries its own transitions */
    q[0] = q_at(b, p->table1[i], p->age1[i] + age_shift + t, m);
    q[1] = q_at(b, p->table2[i], p->age2[i] + age_shift + t, m);
    if (p->product[i] == O_JL3_ANN || p->product[i] == O_LS3_ANN)
        q[2] = q_at(b, p->table3[i], p->age3[i] + age_shift + t, m);
}

/* The contract of policy i (an uploaded model: its size and benefits; a
 * fractional timing: the basis's payment point). */
static void contract_for(const orc_basis *b, const orc_portfolio *p, int i, int gross,
                         orc_contract *k)
{
    orc_contract_of(p->product[i], p->timing[i], p->amount[i], p->premium[i], gross, k);
    /* the annuities' payment point; cash-flow tables and uploaded models pay
     * at the end of the month whatever their timing field says */
    const int annuity = p->product[i] == O_SL_ANN || p->product[i] == O_JL_ANN ||
                        p->product[i] == O_REV_ANN || p->product[i] == O_LS_ANN ||
                        p->product[i] == O_JL3_ANN || p->product[i] == O_LS3_ANN;
    if (p->timing[i] == 2 && annuity) k->f_ann = b->frac;
    if (p->product[i] == O_MARKOV) {
        int m = p->mk_states;
        const double *c = p->mk_c + (size_t)p->table1[i] * m;
        k->n_states = m;
        for (int j = 0; j < m; ++j) {
            double x = p->amount[i] * c[j];
            k->c_ann[j] = gross ? fabs(x) : x;
        }
    }
}

/* One-step matrix over a fraction g of step t: the Kronecker product of the
 * lives' models (Sec. 4.3), or an uploaded model's table at the attained age
 * (g = 1; g = 0 is the identity). */
static void step_w(const orc_portfolio *p, int i, const orc_contract *k, const double *q,
                   int age_shift, int t, double g, double *W)
{
    if (p->product[i] != O_MARKOV) {
        orc_build_w(k->n_lives, k->life_model, q, g, W);
        return;
    }
    int m = p->mk_states;
    if (g == 0.0) {
        for (int a = 0; a < m * m; ++a) W[a] = 0.0;
        for (int a = 0; a < m; ++a) W[a * m + a] = 1.0;
        return;
    }
    int age = p->age1[i] + age_shift + t;
    memcpy(W, p->mk_w + (((size_t)p->table1[i] * p->mk_ages + age) * m) * m, sizeof(double) * m * m);
}

/* Add v^g W_g c to acc, one cash-flow stream of Eq. (3.1). */
static void add_stream(const orc_contract *k, const double *W, double v, double g,
                       const double *c, double *acc)
{
    int n = k->n_states, any = 0;
    for (int j = 0; j < n; ++j) any |= (c[j] != 0.0);
    if (!any) return;
    double y[ORC_MAX_STATES];
    matvec(W, c, n, y);
    double vg = pow(v, g);
    for (int j = 0; j < n; ++j) acc[j] += vg * y[j];
}

/* Factor of the level annuity stream for a payment at time T (months after
 * node 0): (1+e)^n(T) with n(T) the anniversaries in (0, T], times 12 at an
 * anniversary and 0 elsewhere for annual payment.  For a cash-flow table the
 * factor is the table's value for the step ending at T. */
static double payment_factor(const orc_portfolio *p, int i, int T, const orc_contract *k)
{
    if (p->product[i] == O_CF_TABLE) {
        double c = p->cf[(size_t)p->cf_row[i] * p->cf_len + (T - 1)];
        return k->gross ? fabs(c) : c;
    }
    double e = p->escalation ? p->escalation[i] : 0.0;
    int a = p->anniv ? p->anniv[i] : 12;
    int annual = p->annual ? p->annual[i] : 0;
    int n = T < a ? 0 : 1 + (T - a) / 12;
    int at_anniv = T >= a && (T - a) % 12 == 0;
    double lev = pow(1.0 + e, (double)n);
    if (annual) return at_anniv ? 12.0 * lev : 0.0;
    return lev;
}

/* Backward recurrence, Eq. (3.1), for one policy / node / scenario.  Writes
 * the reserve vector at t = 0 into r0 (n_states entries) and, if path is not
 * NULL, the state-0 reserve at t = 0..S into path[0..S]. */
static void recurrence_one(const orc_basis *b, const orc_portfolio *p, int i,
                           const orc_contract *k, int node, int age_shift, int S,
                           const double *vcurve, double *r0, double *path)
{
    int n = k->n_states;
    double m = b->shock ? b->shock[node] : 1.0;
    double r[ORC_MAX_STATES], rn[ORC_MAX_STATES], q[3];
    double W1[ORC_MAX_STATES * ORC_MAX_STATES], y[ORC_MAX_STATES];
    for (int j = 0; j < n; ++j) r[j] = k->boundary[j];
    if (path) path[S] = r[0];
    for (int t = S - 1; t >= 0; --t) {
        double v = vcurve[t];
        step_q(b, p, i, age_shift, m, t, q);
        for (int j = 0; j < n; ++j) rn[j] = 0.0;
        double Wg[ORC_MAX_STATES * ORC_MAX_STATES];
        step_w(p, i, k, q, age_shift, t, 0.0, Wg);
        add_stream(k, Wg, v, 0.0, k->c_prem, rn);
        double c_pay[ORC_MAX_STATES];
        double fac = payment_factor(p, i, age_shift + t + (k->f_ann == 1.0 ? 1 : 0), k);
        for (int j = 0; j < n; ++j) c_pay[j] = fac * k->c_ann[j];
        step_w(p, i, k, q, age_shift, t, k->f_ann, Wg);
        add_stream(k, Wg, v, k->f_ann, c_pay, rn);
        step_w(p, i, k, q, age_shift, t, 1.0, Wg);
        add_stream(k, Wg, v, 1.0, k->c_ben, rn);
        step_w(p, i, k, q, age_shift, t, 1.0, W1);
        matvec(W1, r, n, y);
        for (int j = 0; j < n; ++j) rn[j] += v * y[j];
        for (int j = 0; j < n; ++j) r[j] = rn[j];
        if (path) path[t] = r[0];
    }
    for (int j = 0; j < n; ++j) r0[j] = r[j];
}

/* Neumaier-compensated sum. */
typedef struct { double s, c; } neumaier;
static void nm_add(neumaier *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static int validate(const orc_basis *b, const orc_portfolio *p)
{
    for (int i = 0; i < p->n; ++i) {
        if (p->product[i] < 0 || p->product[i] >= O_N_PRODUCTS) return -1;
        if (p->term[i] < 1 || p->term[i] > b->n_steps) return -1;
        if (p->anniv && (p->anniv[i] < 1 || p->anniv[i] > 12)) return -1;
        if (p->timing[i] < 0 || p->timing[i] > 2) return -1;
        if (p->timing[i] == 2 && !(b->frac > 0.0 && b->frac < 1.0)) return -1;
        if (p->escalation && !(p->escalation[i] >= 0.0)) return -1;
        if (p->product[i] == O_MARKOV) {   /* table1 is the model, ages index its tables */
            if (!p->mk_w || !p->mk_c || p->mk_states < 2 || p->mk_states > ORC_MAX_STATES) return -1;
            if (p->table1[i] < 0 || p->table1[i] >= p->mk_models) return -1;
            if (p->age1[i] < 0 || p->age1[i] + p->term[i] > p->mk_ages - 1) return -1;
            continue;
        }
        if (p->age1[i] < 0 || p->age1[i] + p->term[i] > b->n_ages - 1) return -1;
        if (p->table1[i] < 0 || p->table1[i] >= b->n_tables) return -1;
        if (p->product[i] == O_CF_TABLE) {
            if (!p->cf_row || !p->cf) return -1;
            if (p->cf_row[i] < 0 || p->cf_row[i] >= p->n_cf_rows) return -1;
            if (p->term[i] > p->cf_len) return -1;
        }
        int two = p->product[i] == O_JL_ANN || p->product[i] == O_REV_ANN ||
                  p->product[i] == O_LS_ANN || p->product[i] == O_JL_ENDOW ||
                  p->product[i] == O_JL_ASSUR1 || p->product[i] == O_JL_ASSUR2;
        int three = p->product[i] == O_JL3_ANN || p->product[i] == O_LS3_ANN;
        if (two || three) {
            if (p->age2[i] < 0 || p->age2[i] + p->term[i] > b->n_ages - 1) return -1;
            if (p->table2[i] < 0 || p->table2[i] >= b->n_tables) return -1;
        }
        if (three) {
            if (!p->age3 || !p->table3) return -1;
            if (p->age3[i] < 0 || p->age3[i] + p->term[i] > b->n_ages - 1) return -1;
            if (p->table3[i] < 0 || p->table3[i] >= b->n_tables) return -1;
        }
    }
    return 0;
}

/*
 * Reserves of every policy at nodes [node0, node0+nnode) and scenarios
 * [scen0, scen0+nscen).
 *   r_all  [nnode][n][nscen][4]  reserve vector at t = 0 (states >= n_states: 0;
 *                                two-life 9-state models: states 0, 2, 6, 8)
 *   gross  [nnode][n][nscen]     PV(benefits) + PV(premiums), state 0 (or NULL)
 *   totals [nnode][nscen]        sum over live policies of state-0 reserves
 *   gross_totals [nnode][nscen]  same for gross (or NULL)
 * Any output pointer may be NULL.  Returns 0, or -1 on invalid input.
 */
int orc_reserves(const orc_basis *b, const orc_portfolio *p, int node0, int nnode,
                 int scen0, int nscen, int node_step, double *r_all, double *gross,
                 double *totals, double *gross_totals, int n_threads)
{
    if (validate(b, p)) return -1;
    if (node0 < 0 || nnode < 0 || node0 + nnode > b->n_nodes) return -1;
    if (scen0 < 0 || nscen < 0 || scen0 + nscen > b->n_scen) return -1;
    int n = p->n;
    double *r0s = (double *)calloc((size_t)nnode * n * nscen, sizeof(double));
    double *g0s = (double *)calloc((size_t)nnode * n * nscen, sizeof(double));
    if (!r0s || !g0s) { free(r0s); free(g0s); return -2; }
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
    for (int i = 0; i < n; ++i) {
        orc_contract k, kg;
        contract_for(b, p, i, 0, &k);
        contract_for(b, p, i, 1, &kg);
        double r0[ORC_MAX_STATES], g0[ORC_MAX_STATES];
        for (int a = 0; a < nnode; ++a) {
            int node = node0 + a;
            int shift = node * node_step;
            int S = p->term[i] - shift;
            for (int s = 0; s < nscen; ++s) {
                size_t o = ((size_t)a * n + i) * nscen + s;
                double *ro = r_all ? r_all + o * ORC_OUT_STATES : NULL;
                if (ro) for (int j = 0; j < ORC_OUT_STATES; ++j) ro[j] = 0.0;
                if (S <= 0) { r0s[o] = 0.0; g0s[o] = 0.0; if (gross) gross[o] = 0.0; continue; }
                const double *vc = b->v + ((size_t)node * b->n_scen + (scen0 + s)) * b->n_steps;
                recurrence_one(b, p, i, &k, node, shift, S, vc, r0, NULL);
                if (ro && k.n_lives == 2 && k.life_model == 3) {
                    /* two-life 3-state models in the 4-state labelling (both
                     * alive, x only, y only, none): the dead states 2, 6, 8
                     * (the died-in-step states carry the same reserves) */
                    ro[0] = r0[0]; ro[1] = r0[2]; ro[2] = r0[6]; ro[3] = r0[8];
                } else if (ro) {
                    for (int j = 0; j < k.n_states && j < ORC_OUT_STATES; ++j) ro[j] = r0[j];
                }
                r0s[o] = r0[0];
                if (gross || gross_totals) {
                    recurrence_one(b, p, i, &kg, node, shift, S, vc, g0, NULL);
                    g0s[o] = g0[0];
                    if (gross) gross[o] = g0[0];
                }
            }
        }
    }
    for (int a = 0; a < nnode; ++a)
        for (int s = 0; s < nscen; ++s) {
            neumaier tr = {0, 0}, tg = {0, 0};
            for (int i = 0; i < n; ++i) {
                size_t o = ((size_t)a * n + i) * nscen + s;
                nm_add(&tr, r0s[o]);
                nm_add(&tg, g0s[o]);
            }
            if (totals) totals[(size_t)a * nscen + s] = tr.s + tr.c;
            if (gross_totals) gross_totals[(size_t)a * nscen + s] = tg.s + tg.c;
        }
    free(r0s);
    free(g0s);
    return 0;
}

/*
 * State-0 reserve path of every policy at one node and one scenario:
 * path[off_i + t] for t = 0..S_i, with S_i = term_i - node*node_step and
 * off_i = sum over j < i of (max(S_j, 0) + 1) ... for expired policies
 * (S_i <= 0) the single entry path[off_i] is 0.
 */
int orc_reserve_paths(const orc_basis *b, const orc_portfolio *p, int node, int scen,
                      int node_step, double *path, int n_threads)
{
    if (validate(b, p)) return -1;
    if (node < 0 || node >= b->n_nodes || scen < 0 || scen >= b->n_scen) return -1;
    int n = p->n;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!off) return -2;
    off[0] = 0;
    for (int i = 0; i < n; ++i) {
        int S = p->term[i] - node * node_step;
        off[i + 1] = off[i] + (S > 0 ? S : 0) + 1;
    }
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads)
    for (int i = 0; i < n; ++i) {
        int S = p->term[i] - node * node_step;
        if (S <= 0) { path[off[i]] = 0.0; continue; }
        orc_contract k;
        double r0[ORC_MAX_STATES];
        contract_for(b, p, i, 0, &k);
        const double *vc = b->v + ((size_t)node * b->n_scen + scen) * b->n_steps;
        recurrence_one(b, p, i, &k, node, node * node_step, S, vc, r0, path + off[i]);
    }
    free(off);
    return 0;
}

/*
 * Reserve summation, Eq. (3.5), for one policy at one node and scenario,
 * evaluated independently at every t = 0..S (two nested forward loops,
 * O(S^2) matrix products; Sec. 3.8.1).  The probability of moving from
 * state j at t to state i at t+s+g is the (j, i) entry of the product of the
 * one-step matrices over [t, t+s) times W_g of step t+s (Eq. (3.4)); the
 * discount is the product of the one-step factors (Eq. (3.3)) times v^g.
 * The boundary vector enters as a cash flow at the end of the term.
 * Writes the full vector r_t into out[t*n_states ..] for t = 0..S.
 */
int orc_reserve_path_summation(const orc_basis *b, const orc_portfolio *p, int i,
                               int node, int scen, int node_step, double *out)
{
    if (validate(b, p)) return -1;
    int shift = node * node_step;
    int S = p->term[i] - shift;
    if (S <= 0) return -1;
    orc_contract k;
    contract_for(b, p, i, 0, &k);
    int n = k.n_states;
    double m = b->shock ? b->shock[node] : 1.0;
    const double *vc = b->v + ((size_t)node * b->n_scen + scen) * b->n_steps;
    double P[ORC_MAX_STATES * ORC_MAX_STATES], T[ORC_MAX_STATES * ORC_MAX_STATES];
    double Wg[ORC_MAX_STATES * ORC_MAX_STATES], PW[ORC_MAX_STATES * ORC_MAX_STATES];
    double y[ORC_MAX_STATES], q[3];
    const double *streams[3] = {k.c_prem, k.c_ann, k.c_ben};
    double gs[3] = {0.0, k.f_ann, 1.0};
    for (int t = 0; t <= S; ++t) {
        double r[ORC_MAX_STATES] = {0};
        /* P = identity (probabilities from t to t), D = 1 */
        for (int a = 0; a < n * n; ++a) P[a] = 0.0;
        for (int a = 0; a < n; ++a) P[a * n + a] = 1.0;
        double D = 1.0;
        for (int u = t; u < S; ++u) {
            step_q(b, p, i, shift, m, u, q);
            double v = vc[u];
            for (int st = 0; st < 3; ++st) {
                step_w(p, i, &k, q, shift, u, gs[st], Wg);
                matmul(P, Wg, n, PW);
                matvec(PW, streams[st], n, y);
                double d = D * pow(v, gs[st]);
                if (st == 1) d *= payment_factor(p, i, shift + u + (k.f_ann == 1.0 ? 1 : 0), &k);
                for (int j = 0; j < n; ++j) r[j] += d * y[j];
            }
            step_w(p, i, &k, q, shift, u, 1.0, Wg);
            matmul(P, Wg, n, T);
            memcpy(P, T, sizeof(double) * n * n);
            D *= v;
        }
        matvec(P, k.boundary, n, y);
        for (int j = 0; j < n; ++j) r[j] += D * y[j];
        for (int j = 0; j < n; ++j) out[(size_t)t * n + j] = r[j];
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Reduced mode: the recurrence with the zero-reserve states removed         */
/* (Sec. 3.6.4), written per product from Eq. (3.7).                         */
/* ------------------------------------------------------------------------ */
/*
 * The same reserves as orc_reserves without forming any W: a state whose
 * reserve stays 0 for the whole term (no cash flow can be reached from it)
 * is dropped, and each remaining state's row of Eq. (3.7) is written out
 * with the per-life survival p_l = 1 - q_l of the step.  With s_l = 1 - f q_l
 * and d_l = f q_l the survival and death over the fraction f of a step
 * (uniform deaths; s = 1, d = 0 at f = 0 and s = p, d = q at f = 1), and
 * a = payment x pattern factor, P the premium (paid at f = 0 in the first
 * state), B the sum assured and primes the values at t + 1:
 *   one life, 2 states (annuity, pure endowment, cash-flow table):
 *       r0 = -P + v^f s a + v p r0'                     (boundary SA or 0)
 *   one life, 3 states (term / endowment assurance):
 *       r0 = -P + v (q B + p r0')
 *   two lives, 4 states (binary labels, life 1 the high digit):
 *       joint life, two-life endowment: r0 = -P + v^f s1 s2 a + v p1 p2 r0'
 *       reversionary (paid in state 2):  r2 = v^f s2 a + v p2 r2',
 *                     r0 = -P + v^f d1 s2 a + v (p1 p2 r0' + q1 p2 r2')
 *       last survivor (states 0, 1, 2): r1 = v^f s1 a + v p1 r1',
 *                     r2 = v^f s2 a + v p2 r2',
 *                     r0 = -P + v^f (s1 s2 + s1 d2 + d1 s2) a
 *                          + v (p1 p2 r0' + p1 q2 r1' + q1 p2 r2')
 *   two lives, 9 states (ternary labels: alive, died in the step, dead):
 *       first death:  r0 = -P + v ((1 - p1 p2) B + p1 p2 r0')
 *       second death: the died-in-step states of one life carry the
 *                     reserve of its dead state, so with r2 = (alive, dead)
 *                     and r6 = (dead, alive):
 *                     r2 = v (q1 B + p1 r2'),  r6 = v (q2 B + p2 r6'),
 *                     r0 = -P + v (q1 q2 B + p1 p2 r0' + p1 q2 r2' + q1 p2 r6')
 *   uploaded Markov models: the full m x m step (nothing to drop).
 * The boundary is the product's (SA in state 0 for the endowments).
 * Reported state slots follow orc_reserves.  Only accessors (q lookup,
 * payment factor, contract amounts, validation) are shared with the dense
 * mode; no transition matrix is formed for the life models.
 */
static void reduced_one(const orc_portfolio *p, int i, const orc_contract *k, int S,
                        const double *vc, const double *q1s, const double *q2s, const double *as,
                        double *out4)
{
    const int prod = p->product[i];
    const double P = -k->c_prem[0];             /* premium, positive when paid */
    const double f = k->f_ann;
    double r0 = k->boundary[0], r1 = 0.0, r2 = 0.0;
    double B = 0.0;
    for (int j = 0; j < k->n_states; ++j)
        if (k->c_ben[j] != 0.0) B = k->c_ben[j];
    for (int t = S - 1; t >= 0; --t) {
        const double v = vc[t];
        const double q1 = q1s[t], q2 = q2s[t];
        const double p1 = 1.0 - q1, p2 = 1.0 - q2;
        const double a = as[t];
        const double vf = (f == 1.0) ? v : (f == 0.0 ? 1.0 : pow(v, f));
        const double s1 = 1.0 - f * q1, s2 = 1.0 - f * q2, d1 = f * q1, d2 = f * q2;
        switch (prod) {
        case O_SL_ANN:
        case O_CF_TABLE:
            r0 = -P + vf * s1 * a + v * p1 * r0;
            break;
        case O_ENDOW:
            r0 = -P + v * p1 * r0;
            break;
        case O_TERM:
        case O_ENDOW_ASSUR:
            r0 = -P + v * (q1 * B + p1 * r0);
            break;
        case O_JL_ANN:
            r0 = -P + vf * s1 * s2 * a + v * p1 * p2 * r0;
            break;
        case O_JL_ENDOW:
            r0 = -P + v * p1 * p2 * r0;
            break;
        case O_REV_ANN: {
            const double n2 = vf * s2 * a + v * p2 * r2;
            r0 = -P + vf * d1 * s2 * a + v * (p1 * p2 * r0 + q1 * p2 * r2);
            r2 = n2;
            break;
        }
        case O_LS_ANN: {
            const double n1 = vf * s1 * a + v * p1 * r1;
            const double n2 = vf * s2 * a + v * p2 * r2;
            r0 = -P + vf * (s1 * s2 + s1 * d2 + d1 * s2) * a + v * (p1 * p2 * r0 + p1 * q2 * r1 + q1 * p2 * r2);
            r1 = n1;
            r2 = n2;
            break;
        }
        case O_JL_ASSUR1:
            r0 = -P + v * ((1.0 - p1 * p2) * B + p1 * p2 * r0);
            break;
        case O_JL_ASSUR2: {
            const double n1 = v * (q1 * B + p1 * r1);   /* (alive, dead) */
            const double n2 = v * (q2 * B + p2 * r2);   /* (dead, alive) */
            r0 = -P + v * (q1 * q2 * B + p1 * p2 * r0 + p1 * q2 * r1 + q1 * p2 * r2);
            r1 = n1;
            r2 = n2;
            break;
        }
        default:
            break;
        }
    }
    out4[0] = r0;
    out4[1] = out4[2] = out4[3] = 0.0;
    if (prod == O_REV_ANN) out4[2] = r2;
    if (prod == O_LS_ANN) { out4[1] = r1; out4[2] = r2; }
    if (prod == O_JL_ASSUR2) { out4[1] = r1; out4[2] = r2; }
}

/* Three lives (Sec. 4.3), two-state model each.  A state with at least one
 * life alive is identified by the set A of living lives (bit l-1 of a mask
 * for life l); the state with none alive has reserve 0 and is dropped.
 * With d_l = f q_l the death probability of life l over the fraction f of
 * a step, the last-survivor annuity pays in state A if some life of A is
 * alive at t + f (probability 1 - prod_{l in A} d_l) and the joint-life
 * annuity only in A = {1,2,3}, if all are alive at t + f (probability
 * prod_l (1 - d_l)); its other states never pay again and are dropped too:
 *   r_A = -P [A = {1,2,3}] + v^f a (payment probability)
 *         + v sum_{B subset of A, B nonempty} prod_{l in B} p_l prod_{l in A\B} q_l r'_B.  Slots: state j of the binary labels (life 1 the high digit, 1 =
 * dead), j = 0..3: A = {1,2,3}, {1,2}, {1,3}, {1}. */
static void three_one(const orc_portfolio *p, int i, const orc_contract *k, int S, const double *vc,
                      const double *q1s, const double *q2s, const double *q3s, const double *as,
                      double *out4)
{
    const int joint = p->product[i] == O_JL3_ANN;
    const double P = -k->c_prem[0];
    const double f = k->f_ann;
    double r[8] = {0}, rn[8];
    for (int t = S - 1; t >= 0; --t) {
        const double v = vc[t];
        const double vf = (f == 1.0) ? v : (f == 0.0 ? 1.0 : pow(v, f));
        const double q[3] = {q1s[t], q2s[t], q3s[t]};
        for (int A = 1; A < 8; ++A) {
            if (joint && A != 7) { rn[A] = 0.0; continue; }
            /* the payment's probability: some life of A alive at t + f (last
             * survivor), every life alive at t + f (joint life) */
            double pay_prob = 1.0;
            for (int l = 0; l < 3; ++l)
                if (A >> l & 1) pay_prob *= joint ? 1.0 - f * q[l] : f * q[l];
            if (!joint) pay_prob = 1.0 - pay_prob;
            double acc = 0.0;
            for (int B = 1; B < 8; ++B) {
                if ((B & A) != B) continue;
                double pr = 1.0;
                for (int l = 0; l < 3; ++l)
                    if (A >> l & 1) pr *= (B >> l & 1) ? 1.0 - q[l] : q[l];
                acc += pr * r[B];
            }
            rn[A] = vf * as[t] * pay_prob + v * acc - (A == 7 ? P : 0.0);
        }
        for (int A = 1; A < 8; ++A) r[A] = rn[A];
    }
    out4[0] = r[7];
    out4[1] = r[3];   /* lives 1, 2 */
    out4[2] = r[5];   /* lives 1, 3 */
    out4[3] = r[1];   /* life 1 */
}

/* An uploaded Markov model: every state kept, r_j = -P [j = 0] +
 * v sum_i w_{j,i} (c_i + r_i'), benefits c at the end of the month. */
static void markov_one(const orc_portfolio *p, int i, const orc_contract *k, int shift, int S,
                       const double *vc, double *out4)
{
    const int m = p->mk_states;
    const double P = -k->c_prem[0];
    double r[ORC_MAX_STATES], rn[ORC_MAX_STATES];
    for (int j = 0; j < m; ++j) r[j] = 0.0;
    for (int t = S - 1; t >= 0; --t) {
        const double v = vc[t];
        const double *w = p->mk_w + (((size_t)p->table1[i] * p->mk_ages + p->age1[i] + shift + t) * m) * m;
        for (int j = 0; j < m; ++j) {
            double acc = 0.0;
            for (int x = 0; x < m; ++x) acc += w[j * m + x] * (k->c_ann[x] + r[x]);
            rn[j] = v * acc;
        }
        rn[0] -= P;
        for (int j = 0; j < m; ++j) r[j] = rn[j];
    }
    for (int j = 0; j < ORC_OUT_STATES; ++j) out4[j] = j < m ? r[j] : 0.0;
}

/*
 * orc_reserves in the reduced mode: r_all [nnode][n][nscen][4] (or NULL),
 * totals [nnode][nscen] (or NULL) and abs_totals [nnode][nscen] (or NULL),
 * the sums of |r_0| over the same policies (a scale for the rounding of a
 * total that needs no per-policy output), no gross values.  OpenMP over policies
 * (dynamic schedule); per policy the death probabilities of each step are
 * looked up once and shared by the scenarios.  Returns 0, -1 on invalid
 * input, -2 without memory.
 */
int orc_reserves_reduced(const orc_basis *b, const orc_portfolio *p, int node0, int nnode,
                         int scen0, int nscen, int node_step, double *r_all, double *totals,
                         double *abs_totals, int n_threads)
{
    if (validate(b, p)) return -1;
    if (node0 < 0 || nnode < 0 || node0 + nnode > b->n_nodes) return -1;
    if (scen0 < 0 || nscen < 0 || scen0 + nscen > b->n_scen) return -1;
    const int n = p->n;
    double *r0s = (double *)calloc((size_t)nnode * n * nscen + 1, sizeof(double));
    if (!r0s) return -2;
    int bad = 0;
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel num_threads(n_threads)
    {
        double *q1s = (double *)malloc(sizeof(double) * (size_t)(b->n_steps + 1));
        double *q2s = (double *)malloc(sizeof(double) * (size_t)(b->n_steps + 1));
        double *q3s = (double *)malloc(sizeof(double) * (size_t)(b->n_steps + 1));
        double *as = (double *)malloc(sizeof(double) * (size_t)(b->n_steps + 1));
        if (!q1s || !q2s || !q3s || !as) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < n; ++i) {
            if (!q1s || !q2s || !q3s || !as) continue;
            orc_contract k;
            contract_for(b, p, i, 0, &k);
            double pay = 0.0;   /* the annuity (or table) stream's amount, one state at a time */
            for (int j = 0; j < k.n_states; ++j)
                if (k.c_ann[j] != 0.0) pay = k.c_ann[j];
            for (int a = 0; a < nnode; ++a) {
                const int node = node0 + a;
                const int shift = node * node_step;
                const int S = p->term[i] - shift;
                const double m = b->shock ? b->shock[node] : 1.0;
                /* per policy and node, as the paper's forward loop obtains c_t
                 * and the transition probabilities before the backward loop */
                if (S > 0 && p->product[i] != O_MARKOV)
                    for (int t = 0; t < S; ++t) {
                        double q[3];
                        step_q(b, p, i, shift, m, t, q);
                        q1s[t] = q[0];
                        q2s[t] = q[1];
                        q3s[t] = q[2];
                        as[t] = pay != 0.0
                                    ? pay * payment_factor(p, i, shift + t + (k.f_ann == 1.0 ? 1 : 0), &k)
                                    : 0.0;
                    }
                for (int s = 0; s < nscen; ++s) {
                    const size_t o = ((size_t)a * n + i) * nscen + s;
                    double r4[ORC_OUT_STATES] = {0.0, 0.0, 0.0, 0.0};
                    if (S > 0) {
                        const double *vc = b->v + ((size_t)node * b->n_scen + (scen0 + s)) * b->n_steps;
                        if (p->product[i] == O_MARKOV) markov_one(p, i, &k, shift, S, vc, r4);
                        else if (p->product[i] == O_JL3_ANN || p->product[i] == O_LS3_ANN)
                            three_one(p, i, &k, S, vc, q1s, q2s, q3s, as, r4);
                        else reduced_one(p, i, &k, S, vc, q1s, q2s, as, r4);
                    }
                    r0s[o] = r4[0];
                    if (r_all)
                        for (int j = 0; j < ORC_OUT_STATES; ++j) r_all[o * ORC_OUT_STATES + j] = r4[j];
                }
            }
        }
        free(q1s);
        free(q2s);
        free(q3s);
        free(as);
    }
    if (bad) { free(r0s); return -2; }
    if (totals || abs_totals)
        for (int a = 0; a < nnode; ++a)
            for (int s = 0; s < nscen; ++s) {
                neumaier tr = {0, 0}, ta = {0, 0};
                for (int i = 0; i < n; ++i) {
                    const double x = r0s[((size_t)a * n + i) * nscen + s];
                    nm_add(&tr, x);
                    nm_add(&ta, fabs(x));
                }
                if (totals) totals[(size_t)a * nscen + s] = tr.s + tr.c;
                if (abs_totals) abs_totals[(size_t)a * nscen + s] = ta.s + ta.c;
            }
    free(r0s);
    return 0;
}

/* Number of states of a product's model (for callers sizing buffers). */
int orc_n_states(int product)
{
    orc_contract k;
    if (orc_contract_of(product, 1, 1.0, 0.0, 0, &k)) return -1;
    return k.n_states;
}

/* ------------------------------------------------------------------------ */
/* Scenario generation (the interest model of Sec. 3.4 / 3.7.2, here       */
/* Vasicek): a counter-based generator, normals, and the exact step.       */
/* ------------------------------------------------------------------------ */

/* Philox4x64-10: ten rounds of the Philox S-box on a 4 x 64-bit counter
 * under a 2 x 64-bit key, as defined by Salmon, Moraes, Dror and Shaw
 * ("Parallel random numbers: as easy as 1, 2, 3", SC 2011): per round the
 * words 0 and 2 are multiplied by the two round multipliers, the high
 * halves are xored with the other words and the key, and the key is bumped
 * by the two Weyl increments. */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0, 1) from the top 53 bits. */
static double orc_u01(uint64_t x) { return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

/* Two independent standard normals for (node, scenario, step) by the
 * Box-Muller transform of the first two uniforms of the Philox block with
 * counter (step, scenario, node, 0). */
void orc_normals(uint64_t key0, uint64_t key1, int node, int scen, int step, double z[2])
{
    const uint64_t ctr[4] = {(uint64_t)step, (uint64_t)scen, (uint64_t)node, 0};
    const uint64_t key[2] = {key0, key1};
    uint64_t x[4];
    orc_philox4x64_10(ctr, key, x);
    double u0 = orc_u01(x[0]), u1 = orc_u01(x[1]);
    double rad = sqrt(-2.0 * log(u0));
    double ang = 6.283185307179586476925286766559 * u1;   /* 2 pi u1 */
    z[0] = rad * cos(ang);
    z[1] = rad * sin(ang);
}

/*
 * Vasicek short rate dr = a (b - r) dt + sigma dW, stepped exactly over dt:
 * given r_t, (r_{t+dt}, Y_t = integral of r over the step) is Gaussian with
 *   E r_{t+dt} = b + (r_t - b) e,            e = exp(-a dt)
 *   E Y_t      = b dt + (r_t - b)(1 - e)/a
 *   Var r      = sigma^2 (1 - e^2) / (2a)
 *   Var Y      = sigma^2/a^2 (dt - 2(1 - e)/a + (1 - e^2)/(2a))
 *   Cov(r, Y)  = sigma^2/(2a^2) (1 - e)^2
 * sampled as r_{t+dt} = E r + sd_r z0 and Y = E Y + sd_y (rho z0 +
 * sqrt(1 - rho^2) z1).  The one-step discount factor is v_t = exp(-Y_t).
 * r0[node] starts node `node`.  Writes v[node][scen][step] and, if r is not
 * NULL, r[node][scen][0..n_steps].  Returns 0, or -1 on invalid input.
 */
int orc_vasicek_curves(double a, double b, double sigma, double dt, const double *r0, int n_nodes,
                       int n_scen, int n_steps, uint64_t key0, uint64_t key1, double *v, double *r)
{
    if (!(a > 0.0) || !(sigma >= 0.0) || !(dt > 0.0) || n_nodes < 0 || n_scen < 0 || n_steps < 0)
        return -1;
    double e = exp(-a * dt);
    double var_r = sigma * sigma * (1.0 - e * e) / (2.0 * a);
    double var_y = sigma * sigma / (a * a) * (dt - 2.0 * (1.0 - e) / a + (1.0 - e * e) / (2.0 * a));
    double cov = sigma * sigma / (2.0 * a * a) * (1.0 - e) * (1.0 - e);
    double sd_r = sqrt(var_r), sd_y = sqrt(var_y);
    double rho = (sd_r > 0.0 && sd_y > 0.0) ? cov / (sd_r * sd_y) : 0.0;
    double sd_y_perp = sd_y * sqrt(fmax(0.0, 1.0 - rho * rho));
    for (int k = 0; k < n_nodes; ++k)
        for (int s = 0; s < n_scen; ++s) {
            double rt = r0[k];
            double *vo = v + ((size_t)k * n_scen + s) * n_steps;
            double *ro = r ? r + ((size_t)k * n_scen + s) * (n_steps + 1) : NULL;
            if (ro) ro[0] = rt;
            for (int t = 0; t < n_steps; ++t) {
                double z[2];
                orc_normals(key0, key1, k, s, t, z);
                double y = b * dt + (rt - b) * (1.0 - e) / a + rho * sd_y * z[0] + sd_y_perp * z[1];
                rt = b + (rt - b) * e + sd_r * z[0];
                vo[t] = exp(-y);
                if (ro) ro[t + 1] = rt;
            }
        }
    return 0;
}
