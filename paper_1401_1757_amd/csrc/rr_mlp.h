// Internal declarations of the reserve-surrogate kernels (rr_mlp.hip) used by
// the surrogate runtime (rr_surrogate.cpp).  The network maps 17 standardised
// features (zero-padded to 32 inputs) through two 256-wide GELU layers to one
// output; weights and activations are bfloat16, sums FP32 (MFMA).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rr {
namespace mlp {

constexpr int N_FEAT = 17;
constexpr int K_IN = 32;
constexpr int HID = 256;
constexpr int N_TENORS = 50;
constexpr int N_FACTORS = 3;
constexpr int ROWS = 64;      // rows per wavefront tile in the GEMMs and the fused kernel

// Offsets of the parameters in the FP32 vector (and in gradient vectors).
constexpr int OFF_W1 = 0;                       // W1[K_IN][HID]   (input, hidden)
constexpr int OFF_B1 = OFF_W1 + K_IN * HID;     // b1[HID]
constexpr int OFF_W2 = OFF_B1 + HID;            // W2[HID][HID]    (hidden in, hidden out)
constexpr int OFF_B2 = OFF_W2 + HID * HID;      // b2[HID]
constexpr int OFF_W3 = OFF_B2 + HID;            // W3[HID]
constexpr int OFF_B3 = OFF_W3 + HID;            // b3
constexpr int N_PARAMS = OFF_B3 + 1;            // 74,497

typedef uint16_t bf16_t;   // bfloat16 bits

// bfloat16 copies of the weights, rebuilt from the FP32 master after every
// change.  Training GEMMs read operands with the contraction index
// contiguous; the fused inference kernel copies the *_inf arrays verbatim
// into LDS (their order is the MFMA fragment order, see rr_mlp.hip).
struct Weights {
    const float *master;     // [N_PARAMS]
    bf16_t *w1t;             // [HID][K_IN]   W1 transposed
    bf16_t *w2t;             // [HID][HID]    W2 transposed (out, in)
    bf16_t *w2n;             // [HID][HID]    W2 (in, out)
    float *w3e;              // [HID]         float(bf16(W3))
    bf16_t *w1_inf;          // [HID][K_IN]   swizzled fragments
    bf16_t *w2_inf;          // [HID][HID]    permuted + swizzled fragments
    bf16_t *w3_inf;          // [8][16][32]   head fragments (row 0 = W3)
};

enum Epilogue : int {
    EPI_FWD = 0,       // Z = acc + bias; A = bf16(gelu(Z)) (row-major and transposed)
    EPI_DGELU = 1,     // dZ = bf16(acc * gelu'(Zin)), transposed only
    EPI_PARTIAL = 2,   // C[split][M][N] = acc
};

// C[m][n] = sum_k A[m][k] B[n][k] over bfloat16 operands (both with k
// contiguous), FP32 accumulation; M, N multiples of 32, K of 32 per split.
struct Gemm {
    const bf16_t *A;
    long long lda;
    const bf16_t *B;
    long long ldb;
    int M, N, K, splits;
    const float *bias;       // EPI_FWD: [N]
    float *Z;                // EPI_FWD: [M][N] pre-activation, or null
    bf16_t *Aq;              // EPI_FWD: [M][N], or null
    bf16_t *AqT;             // EPI_FWD / EPI_DGELU: [N][ldt], or null
    long long ldt;
    const float *Zin;        // EPI_DGELU: [M][N]
    float *C;                // EPI_PARTIAL: [splits][M][N]
};

hipError_t launch_gemm(const Gemm &g, int epi, hipStream_t s);

// Standardised FP32 inputs z[n][K_IN] -> bfloat16 rows [n_pad][K_IN] (zero rows past n).
hipError_t launch_prep_input(const float *z, int n, int n_pad, bf16_t *xq, hipStream_t s);
// rows [n][K_IN] -> columns [K_IN][ld] for the rows of one batch.
hipError_t launch_transpose_x(const bf16_t *xq, int n, bf16_t *xqt, long long ld, hipStream_t s);

// Head, loss and output gradient for rows [0, n_pad) of a batch (n_pad a
// multiple of 16): y = A2q W3 + b3; for rows < n_valid with targets,
// dy = 2 (y - t) * inv_n and the squared error goes to loss_part[block];
// with grads, dZ2 = bf16(dy W3 gelu'(Z2)) row-major and transposed.
hipError_t launch_head(const bf16_t *a2q, const float *z2, const Weights &w, const float *t,
                       int n_pad, int n_valid, float inv_n, bool grads, float *y, float *dy,
                       float *loss_part, bf16_t *dz2q, bf16_t *dz2qt, long long ldt, hipStream_t s);
// db1, db2, dW3, db3 into grad (fixed-order sums over the batch).
hipError_t launch_vec_grads(const bf16_t *dz1qt, const bf16_t *dz2qt, const bf16_t *a2qt,
                            const float *dy, long long ldt, int n_pad, float *grad, hipStream_t s);
// dW1 and dW2 from split-K partials, fixed order.
hipError_t launch_reduce_grads(const float *p1, int s1, const float *p2, int s2, float *grad,
                               hipStream_t s);
// scale * (sum of n floats, fixed order) into *out (one block).
hipError_t launch_sum(const float *x, int n, float scale, float *out, hipStream_t s);
hipError_t launch_adam(float *w, float *m, float *v, const float *g, float lr, float c1, float c2,
                       hipStream_t s);
hipError_t launch_export(const Weights &w, hipStream_t s);

// ---- features ------------------------------------------------------------
// Standardisation and range box of the model (FP64, device).
struct Norm {
    const double *mu;        // [N_FEAT]
    const double *sd;
    const double *lo;
    const double *hi;
    const double *zbar;      // [N_TENORS]
    const double *evec;      // [N_FACTORS][N_TENORS]
    const int *signature;    // [4][3] table1, table2 (-1), timing (-1); table1 -1 = absent
    const double *tmu;       // [4] target mean per one-hot product
    const double *tsd;       // [4] target standard deviation per one-hot product
};

// Per (node, scenario): sums of log v over the 12 months of each tenor year,
// seg[node][N_TENORS][scen], from month-major curves v[node][t][scen_pad].
hipError_t launch_zero_rates(const double *v, int n_steps, int scen_pad, int node_begin,
                             int node_count, int scen_begin, int scen_count, double *seg,
                             hipStream_t s);
// Zero-rate curves z[node][scen][N_TENORS] from the segment sums.
hipError_t launch_curves_out(const double *v, int n_steps, int scen_pad, const double *seg,
                             int node_begin, int node_count, int scen_begin, int scen_count,
                             double *z, hipStream_t s);
// Per (node, scenario): raw scenario features [node][scen][5], standardised
// bfloat16 features 8..15 (state 0) [node][scen][8] and the in-box flag.
hipError_t launch_scen_features(const double *v, int n_steps, int scen_pad, const double *shock,
                                const double *seg, int node_begin, int node_count, int scen_begin,
                                int scen_count, const Norm &nm, double *raw, bf16_t *feat,
                                int *ok, hipStream_t s);
// Portfolio in upload order (device copies).
struct Policies {
    int n;
    const int *product, *age1, *age2, *term, *table1, *table2, *timing;
    const double *amount, *premium;
    const int *patterned;   // 1: annuity with a payment pattern (outside the domain), or null
};
// Per (node, policy): raw features [node][n][9] (features 0-7 and 16),
// standardised bfloat16 features 0-7 [node][n][8] and 16 [node][n],
// state flag [node][n] (1 in the box, 0 outside, 2 expired) and the output
// map r = y * scale + offset (amount x target sd / mean of the product).
hipError_t launch_policy_features(const Policies &p, int node_begin, int node_count,
                                  int node_step, const Norm &nm, double *raw, bf16_t *feat,
                                  bf16_t *feat2, int *flag, double *scale, double *offset,
                                  hipStream_t s);

// ---- fused inference -------------------------------------------------------
struct Infer {
    int node_count, scen_count, n;
    int chunk;               // policies per work unit
    const bf16_t *pfeat;     // [node][n][8]
    const bf16_t *pfeat2;    // [node][n]
    const int *pflag;        // [node][n]
    const bf16_t *sfeat;     // [node][scen][8]
    const int *sok;          // [node][scen]
    const double *scale;     // [node][n] reserve = y * scale + offset
    const double *offset;    // [node][n]
    double *r0;              // [node][n][scen] predictions written here, or null
    const double *exact;     // [node][n][scen] fallback values for rows outside the box
    double *partial;         // [node][n_chunks][scen]
};
hipError_t launch_infer(const Infer &f, const Weights &w, hipStream_t s);
int infer_rows_per_unit();   // scenarios per work unit of the fused kernel
// totals[node][scen] = sum over chunks of partial[node][chunk][scen], fixed
// order; work holds chunk_totals_work(node_count, scen_count) doubles.
long long chunk_totals_work(int node_count, int scen_count);
hipError_t launch_chunk_totals(const double *partial, int node_count, int n_chunks,
                               int scen_count, double *work, double *totals, hipStream_t s);

// ---- training data --------------------------------------------------------
// Raw sample rows X[N][N_FEAT] and targets from exact reserves
// r_all[node][n][scen][4]; rows enumerate (node, scen, pair) with pairs
// (policy, state) listed per node.
hipError_t launch_samples(const double *praw, const double *sraw, const double *r_all,
                          const double *amount, const int2 *pairs, const long long *pair_off,
                          const long long *row_off, int node_count, int n, int scen_count,
                          long long n_rows, double *X, double *T, hipStream_t s);
// Column statistics in a fixed order, out[STAT_COLS][4] = mean, population
// sd, min, max: columns 0-16 the features, 17 the target, 18-21 the target
// over the rows of each one-hot product (count 0: mean 0, sd 0).
constexpr int STAT_COLS = N_FEAT + 1 + 4;
constexpr int STAT_BLOCKS = 256;
hipError_t launch_colstats(const double *X, const double *T, long long n, double *work,
                           double *out, hipStream_t s);
// Standardised bfloat16 rows at permuted positions and FP32 targets
// (standardised with the statistics of the row's product).
hipError_t launch_build(const double *X, const double *T, long long n, const int *perm,
                        const double *mu, const double *sd, const double *tmu, const double *tsd,
                        bf16_t *xq, float *tq, unsigned char *prod, hipStream_t s);
// Sums of t - y and row counts per one-hot product for each block of 1024
// rows: out[block][0..3], out[block][4..7], residual_blocks(n) blocks.
int residual_blocks(int n);
hipError_t launch_residuals(const float *y, const float *t, const unsigned char *prod, int n,
                            double *out, hipStream_t s);

// ---- node-level model -------------------------------------------------------
// out[r * out_stride + j] = (sum over i < n_inner, in order, of
// x[(r * n_inner + i) * width + j]) / n_inner.
hipError_t launch_mean_inner(const double *x, long long rows, int n_inner, int width, double *out,
                             int out_stride, hipStream_t s);
// Predictions of rows (node k, policy i) = rowmap[j]: out[k * n + i] =
// y[j] * scale[k * n + i] + offset[k * n + i].
hipError_t launch_node_scatter(const float *y, const int2 *rowmap, long long rows, int n,
                               const double *scale, const double *offset, double *out,
                               hipStream_t s);
// out[j] = src[j] where mask[j] != 0, for j < count.
hipError_t launch_select(const double *src, const unsigned char *mask, long long count, double *out,
                         hipStream_t s);
// out[r] = sum over i < n of x[r * n + i] (fixed-order tree, one block per row).
hipError_t launch_row_sums(const double *x, int rows, int n, double *out, hipStream_t s);

}  // namespace mlp
}  // namespace rr
