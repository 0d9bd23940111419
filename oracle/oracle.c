/*
 * oracle.c -- CPU oracle for the masked-L2 patch search of exemplar-based
 * inpainting (Dahmen et al., "Space-Filling Curve Indices as Acceleration
 * Structure for Exemplar-Based Inpainting"), and its L1 variant
 * (Section III.K).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do. It shares no code with the GPU library.
 *
 * Plain, single-threaded C11, written to be read against the paper. Build with
 *   gcc -O2 -std=gnu11 -ffp-contract=off -fno-fast-math -shared -fPIC
 * so that every floating-point operation is the one written here (no fused
 * multiply-add unless fmaf() is called, no reassociation, denormals kept).
 *
 * Layout conventions (shared by the inputs only, not by code):
 *   volume  float32 [shape[0], ..., shape[nd-1], C], channel innermost
 *   mask    uint8   [shape...], 1 = known
 *   voxel id = row-major linear index over the spatial dims
 *   patch offset rho = row-major index over the K^nd box, offset rho_i - h,
 *   h = (K-1)/2; element e = rho*C + ch.
 *
 * Parity status per function is stated in each header comment.
 */
#define _GNU_SOURCE   /* qsort_r */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXD 3

/* ------------------------------------------------------------------ */
/* geometry helpers                                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    int nd;
    int64_t shape[ORC_MAXD];
    int64_t stride[ORC_MAXD];
    int64_t nvox;
} grid_t;

static grid_t make_grid(int nd, const int64_t *shape)
{
    grid_t g;
    g.nd = nd;
    g.nvox = 1;
    for (int i = nd - 1; i >= 0; i--) {
        g.shape[i] = shape[i];
        g.stride[i] = g.nvox;
        g.nvox *= shape[i];
    }
    return g;
}

static void coords_of(const grid_t *g, int64_t v, int64_t *c)
{
    for (int i = 0; i < g->nd; i++) {
        c[i] = v / g->stride[i];
        v = v % g->stride[i];
    }
}

static int64_t ipow(int64_t b, int e)
{
    int64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}

/* patch offset rho -> per-axis offsets in [-h, h] */
static void rho_offsets(int nd, int K, int64_t rho, int64_t *off)
{
    int h = (K - 1) / 2;
    for (int i = nd - 1; i >= 0; i--) {
        off[i] = (rho % K) - h;
        rho /= K;
    }
}

/* voxel at centre c (coords cc) + offset rho; returns -1 if out of bounds */
static int64_t voxel_at(const grid_t *g, const int64_t *cc, int K, int64_t rho)
{
    int64_t off[ORC_MAXD];
    rho_offsets(g->nd, K, rho, off);
    int64_t v = 0;
    for (int i = 0; i < g->nd; i++) {
        int64_t x = cc[i] + off[i];
        if (x < 0 || x >= g->shape[i]) return -1;
        v += x * g->stride[i];
    }
    return v;
}

/* ------------------------------------------------------------------ */
/* Fill front and target construction (Fig. 1a, Section II)            */
/* ------------------------------------------------------------------ */

/* The fill front: known voxels with at least one unknown face neighbour
 * (Fig. 1a defines it as known pixels adjacent to unknown ones; adjacency is
 * read as face adjacency). Writes ascending voxel ids; returns the count
 * (which may exceed cap: then only cap ids are written). */
int64_t orc_front(const uint8_t *mask, int nd, const int64_t *shape,
                  int64_t *out, int64_t cap)
{
    grid_t g = make_grid(nd, shape);
    int64_t cnt = 0, cc[ORC_MAXD];
    for (int64_t v = 0; v < g.nvox; v++) {
        if (!mask[v]) continue;
        coords_of(&g, v, cc);
        int front = 0;
        for (int i = 0; i < nd && !front; i++) {
            if (cc[i] > 0 && !mask[v - g.stride[i]]) front = 1;
            if (cc[i] + 1 < g.shape[i] && !mask[v + g.stride[i]]) front = 1;
        }
        if (front) {
            if (cnt < cap) out[cnt] = v;
            cnt++;
        }
    }
    return cnt;
}

/* Target patch and its pixel mask at each centre: t = volume value where the
 * pixel is in bounds and known, 0 otherwise; m = in bounds and known.
 * t is float32 [Q, K^nd, C], m is uint8 [Q, K^nd]. */
void orc_extract(const float *vol, const uint8_t *mask, int nd, const int64_t *shape,
                 int C, int K, const int64_t *centres, int64_t Q, float *t, uint8_t *m)
{
    grid_t g = make_grid(nd, shape);
    int64_t Kd = ipow(K, nd), cc[ORC_MAXD];
    for (int64_t q = 0; q < Q; q++) {
        coords_of(&g, centres[q], cc);
        for (int64_t rho = 0; rho < Kd; rho++) {
            int64_t v = voxel_at(&g, cc, K, rho);
            int known = (v >= 0) && mask[v];
            m[q * Kd + rho] = (uint8_t)known;
            for (int ch = 0; ch < C; ch++)
                t[(q * Kd + rho) * C + ch] = known ? vol[v * C + ch] : 0.0f;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Dictionary and cost (Sections I and II)                             */
/* ------------------------------------------------------------------ */

/* The dictionary: every centre whose K^nd box lies inside the volume and is
 * fully known, in ascending voxel id. Returns n (ids written up to cap). */
int64_t orc_dictionary(const uint8_t *mask, int nd, const int64_t *shape, int K,
                       int64_t *ids, int64_t cap)
{
    grid_t g = make_grid(nd, shape);
    int64_t Kd = ipow(K, nd), cc[ORC_MAXD], n = 0;
    int h = (K - 1) / 2;
    for (int64_t v = 0; v < g.nvox; v++) {
        coords_of(&g, v, cc);
        int ok = 1;
        for (int i = 0; i < nd; i++)
            if (cc[i] < h || cc[i] >= g.shape[i] - h) ok = 0;
        for (int64_t rho = 0; ok && rho < Kd; rho++)
            if (!mask[voxel_at(&g, cc, K, rho)]) ok = 0;
        if (ok) {
            if (n < cap) ids[n] = v;
            n++;
        }
    }
    return n;
}

/* Masked L2 cost (Section II: differences at unknown pixels count as zero).
 * Sum over known rho ascending, channel ascending, of d*d with d = t - V,
 * accumulated as a float32 fused multiply-add chain starting at +0. This
 * fixed-order float32 value is the cost that ranks candidates. */
float orc_cost(const float *vol, const grid_t *g, int C, int K, int64_t centre,
               const float *t, const uint8_t *m)
{
    int64_t Kd = ipow(K, g->nd), cc[ORC_MAXD];
    coords_of(g, centre, cc);
    float acc = 0.0f;
    for (int64_t rho = 0; rho < Kd; rho++) {
        if (!m[rho]) continue;
        int64_t v = voxel_at(g, cc, K, rho);
        for (int ch = 0; ch < C; ch++) {
            float d = t[rho * C + ch] - vol[v * C + ch];
            acc = fmaf(d, d, acc);
        }
    }
    return acc;
}

/* Masked L1 cost, the distance of Section III.K's variant: the same known
 * elements in the same order as the L2 cost, |d| with d = t - V added in
 * float32 (round to nearest) to an accumulator starting at +0. */
float orc_cost_l1(const float *vol, const grid_t *g, int C, int K, int64_t centre,
                  const float *t, const uint8_t *m)
{
    int64_t Kd = ipow(K, g->nd), cc[ORC_MAXD];
    coords_of(g, centre, cc);
    float acc = 0.0f;
    for (int64_t rho = 0; rho < Kd; rho++) {
        if (!m[rho]) continue;
        int64_t v = voxel_at(g, cc, K, rho);
        for (int ch = 0; ch < C; ch++) {
            float d = t[rho * C + ch] - vol[v * C + ch];
            acc = acc + fabsf(d);
        }
    }
    return acc;
}

/* The cost that ranks candidates under norm 0 (L2) or 1 (L1). */
static float cost_of(int norm, const float *vol, const grid_t *g, int C, int K, int64_t centre,
                     const float *t, const uint8_t *m)
{
    return norm ? orc_cost_l1(vol, g, C, K, centre, t, m) : orc_cost(vol, g, C, K, centre, t, m);
}

/* The same cost in float64 (no fused operations), for error checks. */
double orc_cost64_one(const float *vol, int nd, const int64_t *shape, int C, int K,
                      int64_t centre, const float *t, const uint8_t *m)
{
    grid_t g = make_grid(nd, shape);
    int64_t Kd = ipow(K, nd), cc[ORC_MAXD];
    coords_of(&g, centre, cc);
    double acc = 0.0;
    for (int64_t rho = 0; rho < Kd; rho++) {
        if (!m[rho]) continue;
        int64_t v = voxel_at(&g, cc, K, rho);
        for (int ch = 0; ch < C; ch++) {
            double d = (double)t[rho * C + ch] - (double)vol[v * C + ch];
            acc += d * d;
        }
    }
    return acc;
}

float orc_cost_one(const float *vol, int nd, const int64_t *shape, int C, int K,
                   int64_t centre, const float *t, const uint8_t *m)
{
    grid_t g = make_grid(nd, shape);
    return orc_cost(vol, &g, C, K, centre, t, m);
}

float orc_cost_l1_one(const float *vol, int nd, const int64_t *shape, int C, int K,
                      int64_t centre, const float *t, const uint8_t *m)
{
    grid_t g = make_grid(nd, shape);
    return orc_cost_l1(vol, &g, C, K, centre, t, m);
}

/* The L1 cost in float64, for error checks. */
double orc_cost64_l1_one(const float *vol, int nd, const int64_t *shape, int C, int K,
                         int64_t centre, const float *t, const uint8_t *m)
{
    grid_t g = make_grid(nd, shape);
    int64_t Kd = ipow(K, nd), cc[ORC_MAXD];
    coords_of(&g, centre, cc);
    double acc = 0.0;
    for (int64_t rho = 0; rho < Kd; rho++) {
        if (!m[rho]) continue;
        int64_t v = voxel_at(&g, cc, K, rho);
        for (int ch = 0; ch < C; ch++)
            acc += fabs((double)t[rho * C + ch] - (double)vol[v * C + ch]);
    }
    return acc;
}

/* Full scan (Section I: evaluate the cost for every dictionary patch and take
 * the global minimum), under norm 0 (L2) or 1 (L1). Ties go to the lowest id,
 * because dict is ascending and only a strictly smaller cost replaces the
 * current best. */
void orc_brute(const float *vol, int nd, const int64_t *shape, int C, int K,
               const int64_t *dict, int64_t n, const float *t, const uint8_t *m,
               int64_t Q, int64_t *best_id, float *best_cost, int norm)
{
    grid_t g = make_grid(nd, shape);
    int64_t Kd = ipow(K, nd);
    for (int64_t q = 0; q < Q; q++) {
        const float *tq = t + q * Kd * C;
        const uint8_t *mq = m + q * Kd;
        int64_t bi = -1;
        float bc = INFINITY;
        for (int64_t i = 0; i < n; i++) {
            float c = cost_of(norm, vol, &g, C, K, dict[i], tq, mq);
            if (bi < 0 || c < bc) {
                bc = c;
                bi = dict[i];
            }
        }
        best_id[q] = bi;
        best_cost[q] = bc;
    }
}

/* ------------------------------------------------------------------ */
/* Index build (Sections II, II.A-C)                                   */
/* ------------------------------------------------------------------ */

/* Quantise every value to a byte (the paper keeps principal coordinates as
 * bytes; the volume itself is quantised here so the projection is exact in
 * integers): vmin/vmax over known voxels of all channels,
 * s = 255/(vmax - vmin) in float32 (0 if vmax == vmin),
 * x = clamp(rint((v - vmin) * s), 0, 255). Returns 0, or -1 if nothing is
 * known. */
int orc_quantize(const float *vol, const uint8_t *mask, int64_t nvox, int C,
                 float *vmin_out, float *scale_out, uint8_t *xq)
{
    int any = 0;
    float lo = 0.0f, hi = 0.0f;
    for (int64_t v = 0; v < nvox; v++) {
        if (!mask[v]) continue;
        for (int ch = 0; ch < C; ch++) {
            float x = vol[v * C + ch];
            if (!any) { lo = hi = x; any = 1; }
            if (x < lo) lo = x;
            if (x > hi) hi = x;
        }
    }
    if (!any) return -1;
    float s = (hi > lo) ? 255.0f / (hi - lo) : 0.0f;
    for (int64_t i = 0; i < nvox * C; i++) {
        float r = rintf((vol[i] - lo) * s);
        if (!(r >= 0.0f)) r = 0.0f;
        if (r > 255.0f) r = 255.0f;
        xq[i] = (uint8_t)r;
    }
    *vmin_out = lo;
    *scale_out = s;
    return 0;
}

/* Byte code of one target value, the same rule as above. */
static int quant1(float x, float vmin, float s)
{
    float r = rintf((x - vmin) * s);
    if (!(r >= 0.0f)) r = 0.0f;
    if (r > 255.0f) r = 255.0f;
    return (int)r;
}

/* Pixel subsets (Section II, Fig. 2): one index per anchor, anchors at the
 * corners and edge midpoints of the patch, i.e. every a in {0,1,2}^nd except
 * the centre, at position a*(K-1)/2, in lexicographic order (axis 0 slowest).
 * Each subset holds the ceil(0.6*K^nd) pixels nearest its anchor by squared
 * distance, ties at the cut distance included. pix is [S][K^nd] (rho
 * ascending), npix[S]. Returns S = 3^nd - 1. */
int orc_subsets(int nd, int K, int32_t *npix, int32_t *pix)
{
    int64_t Kd = ipow(K, nd);
    int h = (K - 1) / 2;
    int64_t need = (6 * Kd + 9) / 10;
    int64_t *dist = malloc(sizeof(int64_t) * Kd);
    int64_t *sorted = malloc(sizeof(int64_t) * Kd);
    int S = 0;
    int n3 = (int)ipow(3, nd);
    for (int a = 0; a < n3; a++) {
        int digits[ORC_MAXD], centre = 1, rem = a;
        for (int i = nd - 1; i >= 0; i--) {
            digits[i] = rem % 3;
            rem /= 3;
            if (digits[i] != 1) centre = 0;
        }
        if (centre) continue;
        for (int64_t rho = 0; rho < Kd; rho++) {
            int64_t off[ORC_MAXD], d2 = 0;
            rho_offsets(nd, K, rho, off);
            for (int i = 0; i < nd; i++) {
                int64_t dd = (off[i] + h) - (int64_t)digits[i] * h;
                d2 += dd * dd;
            }
            dist[rho] = d2;
            sorted[rho] = d2;
        }
        /* insertion sort: plain and sufficient for K^nd <= 2197 */
        for (int64_t i = 1; i < Kd; i++) {
            int64_t x = sorted[i], j = i - 1;
            while (j >= 0 && sorted[j] > x) { sorted[j + 1] = sorted[j]; j--; }
            sorted[j + 1] = x;
        }
        int64_t r2 = sorted[need - 1];
        int cnt = 0;
        for (int64_t rho = 0; rho < Kd; rho++)
            if (dist[rho] <= r2) pix[S * Kd + cnt++] = (int32_t)rho;
        npix[S] = cnt;
        S++;
    }
    free(dist);
    free(sorted);
    return S;
}

/* Integer patch statistics for the PCA (Section II.A), over the strided
 * subsample of dictionary ranks r = 0, st, 2st, ... with st = ceil(n / 2^20):
 * sum[e] = sum of x_e, sumsq[e*P+f] = sum of x_e*x_f over all P elements.
 * Exact in int64 (n_sub <= 2^20, x <= 255). Returns n_sub. */
int64_t orc_cov_sums(const uint8_t *xq, int nd, const int64_t *shape, int C, int K,
                     const int64_t *dict, int64_t n, int64_t *sum, int64_t *sumsq)
{
    grid_t g = make_grid(nd, shape);
    int64_t Kd = ipow(K, nd), P = Kd * C, cc[ORC_MAXD];
    int64_t st = (n + (1 << 20) - 1) >> 20;
    if (st < 1) st = 1;
    int64_t *x = malloc(sizeof(int64_t) * P);
    memset(sum, 0, sizeof(int64_t) * P);
    memset(sumsq, 0, sizeof(int64_t) * P * P);
    int64_t nsub = 0;
    for (int64_t r = 0; r < n; r += st) {
        coords_of(&g, dict[r], cc);
        for (int64_t rho = 0; rho < Kd; rho++) {
            int64_t v = voxel_at(&g, cc, K, rho);
            for (int ch = 0; ch < C; ch++) x[rho * C + ch] = xq[v * C + ch];
        }
        for (int64_t e = 0; e < P; e++) {
            sum[e] += x[e];
            for (int64_t f = 0; f < P; f++) sumsq[e * P + f] += x[e] * x[f];
        }
        nsub++;
    }
    free(x);
    return nsub;
}

/* Scaled covariance of one subset's elements: A = n_sub*Sxx - Sx*Sx^T, exact
 * in int64, then converted to double (correctly rounded). elems[m] lists the
 * subset's element indices. */
void orc_cov_matrix(const int64_t *sum, const int64_t *sumsq, int64_t nsub, int64_t P,
                    const int32_t *elems, int m, double *A)
{
    for (int i = 0; i < m; i++)
        for (int j = 0; j < m; j++) {
            int64_t a = nsub * sumsq[(int64_t)elems[i] * P + elems[j]]
                      - sum[elems[i]] * sum[elems[j]];
            A[(int64_t)i * m + j] = (double)a;
        }
}

/* Symmetric eigendecomposition by Jacobi rotations in float64.
 *
 * Ordering: round-robin ("tournament") pairing, so each round's pairs are
 * disjoint: with M = m rounded up to even, round r pairs (r, M-1) and, for
 * k = 1..M/2-1, ((r+k) mod (M-1), (r-k) mod (M-1)); a pair touching the
 * padding index m (m odd) is idle. One sweep is M-1 rounds, so every pair
 * once. Per round, every pair (p<q) first decides from the matrix as it
 * stands at the start of the round:
 *   negligible: |a_pq| <= tiny, or both |a_pp| and |a_qq| absorb 100*|a_pq|
 *               -> a_pq = a_qp = 0, no rotation;
 *   otherwise   theta = (a_qq - a_pp) / (2 a_pq),
 *               t = sign(theta) / (|theta| + sqrt(1 + theta^2)) (sign(0)=+1),
 *               c = 1/sqrt(1+t^2), s = t*c.
 * Then the rotations are applied as A <- J^T A J in two passes (all rows of
 * the rotating pairs: B_p = c A_p - s A_q, B_q = s A_p + c A_q; then all their
 * columns the same way), the pair's a_pq and a_qp are set to exactly 0, and
 * V <- V J by columns. The two passes round the entries above and below the
 * diagonal differently, so each round ends by copying the upper triangle onto
 * the lower one: A stays exactly symmetric, and entry (i, j), i < j, is the
 * row rotation of i's pair followed by the column rotation of j's pair.
 * tiny = 2^-100 * max_i |a_ii| of the input.
 * Stops after a sweep with no rotation, or 60 sweeps. Returns the sweep count.
 * A (m*m, row-major) is overwritten; eigenvalues are its diagonal on return;
 * V (m*m, row-major) receives eigenvectors as columns. */
int orc_jacobi(double *A, int m, double *V)
{
    int M = m + (m & 1);
    int np = M / 2;
    double *B = malloc(sizeof(double) * (size_t)m * m);
    int *P = malloc(sizeof(int) * np), *Qi = malloc(sizeof(int) * np);
    int *act = malloc(sizeof(int) * np);
    double *cs = malloc(sizeof(double) * np), *sn = malloc(sizeof(double) * np);
    double tiny = 0.0;
    for (int i = 0; i < m; i++) {
        double a = fabs(A[(size_t)i * m + i]);
        if (a > tiny) tiny = a;
        for (int j = 0; j < m; j++) V[(size_t)i * m + j] = (i == j) ? 1.0 : 0.0;
    }
    tiny = ldexp(tiny, -100);
    int sweep = 0;
    while (sweep < 60) {
        int rotations = 0;
        for (int r = 0; r < M - 1; r++) {
            for (int k = 0; k < np; k++) {
                int a, b;
                if (k == 0) { a = r; b = M - 1; }
                else { a = (r + k) % (M - 1); b = (r - k + (M - 1)) % (M - 1); }
                P[k] = a < b ? a : b;
                Qi[k] = a < b ? b : a;
            }
            for (int k = 0; k < np; k++) {
                int p = P[k], q = Qi[k];
                act[k] = 0;
                if (q >= m) continue;
                double apq = A[(size_t)p * m + q];
                double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
                double g = 100.0 * fabs(apq);
                if (fabs(apq) <= tiny ||
                    (fabs(app) + g == fabs(app) && fabs(aqq) + g == fabs(aqq))) {
                    A[(size_t)p * m + q] = 0.0;
                    A[(size_t)q * m + p] = 0.0;
                    continue;
                }
                double theta = (aqq - app) / (2.0 * apq);
                double t = 1.0 / (fabs(theta) + sqrt(1.0 + theta * theta));
                if (theta < 0.0) t = -t;
                double c = 1.0 / sqrt(1.0 + t * t);
                act[k] = 1;
                cs[k] = c;
                sn[k] = t * c;
                rotations++;
            }
            /* rows */
            memcpy(B, A, sizeof(double) * (size_t)m * m);
            for (int k = 0; k < np; k++) {
                if (!act[k]) continue;
                int p = P[k], q = Qi[k];
                double c = cs[k], s = sn[k];
                for (int j = 0; j < m; j++) {
                    double x = A[(size_t)p * m + j], y = A[(size_t)q * m + j];
                    B[(size_t)p * m + j] = c * x - s * y;
                    B[(size_t)q * m + j] = s * x + c * y;
                }
            }
            /* columns */
            memcpy(A, B, sizeof(double) * (size_t)m * m);
            for (int k = 0; k < np; k++) {
                if (!act[k]) continue;
                int p = P[k], q = Qi[k];
                double c = cs[k], s = sn[k];
                for (int i = 0; i < m; i++) {
                    double x = B[(size_t)i * m + p], y = B[(size_t)i * m + q];
                    A[(size_t)i * m + p] = c * x - s * y;
                    A[(size_t)i * m + q] = s * x + c * y;
                }
            }
            for (int k = 0; k < np; k++) {
                if (!act[k]) continue;
                int p = P[k], q = Qi[k];
                A[(size_t)p * m + q] = 0.0;
                A[(size_t)q * m + p] = 0.0;
                double c = cs[k], s = sn[k];
                for (int i = 0; i < m; i++) {
                    double x = V[(size_t)i * m + p], y = V[(size_t)i * m + q];
                    V[(size_t)i * m + p] = c * x - s * y;
                    V[(size_t)i * m + q] = s * x + c * y;
                }
            }
            for (int i = 0; i < m; i++)
                for (int j = i + 1; j < m; j++) A[(size_t)j * m + i] = A[(size_t)i * m + j];
        }
        sweep++;
        if (rotations == 0) break;
    }
    free(B); free(P); free(Qi); free(act); free(cs); free(sn);
    return sweep;
}

/* Keep the first D principal components (Section II.A) as an int8 basis:
 * components ordered by eigenvalue descending (ties: lower column first);
 * each selected vector's largest-magnitude entry (first on ties) made
 * positive; one scale for the whole subset, g = max |v| over the selected
 * entries, w = rint(v * 127 / g). Writes w [m][D] row-major, the selected
 * columns to order[D], and returns 0 (or -1 if D > m). */
int orc_basis(const double *A, const double *V, int m, int D, int8_t *w, int32_t *order)
{
    if (D > m || D < 1) return -1;
    int *idx = malloc(sizeof(int) * m);
    for (int i = 0; i < m; i++) idx[i] = i;
    for (int i = 1; i < m; i++) { /* insertion sort: eigenvalue desc, index asc */
        int x = idx[i], j = i - 1;
        double lx = A[(size_t)x * m + x];
        while (j >= 0) {
            double lj = A[(size_t)idx[j] * m + idx[j]];
            if (lj < lx || (lj == lx && idx[j] > x)) { idx[j + 1] = idx[j]; j--; }
            else break;
        }
        idx[j + 1] = x;
    }
    double *sel = malloc(sizeof(double) * (size_t)m * D);
    double gmax = 0.0;
    for (int d = 0; d < D; d++) {
        int col = idx[d];
        order[d] = col;
        int best = 0;
        for (int i = 1; i < m; i++)
            if (fabs(V[(size_t)i * m + col]) > fabs(V[(size_t)best * m + col])) best = i;
        double sg = (V[(size_t)best * m + col] < 0.0) ? -1.0 : 1.0;
        for (int i = 0; i < m; i++) {
            double v = sg * V[(size_t)i * m + col];
            sel[(size_t)i * D + d] = v;
            if (fabs(v) > gmax) gmax = fabs(v);
        }
    }
    for (int i = 0; i < m; i++)
        for (int d = 0; d < D; d++)
            w[(size_t)i * D + d] = (int8_t)rint((sel[(size_t)i * D + d] * 127.0) / gmax);
    free(idx);
    free(sel);
    return 0;
}

/* Principal coordinates of every dictionary patch: y[c][d] = sum_i w[i][d] *
 * x[c][elems[i]], exact in int64. */
void orc_project(const uint8_t *xq, int nd, const int64_t *shape, int C, int K,
                 const int64_t *dict, int64_t n, const int32_t *elems, int m,
                 const int8_t *w, int D, int64_t *y)
{
    grid_t g = make_grid(nd, shape);
    int64_t cc[ORC_MAXD];
    for (int64_t c = 0; c < n; c++) {
        coords_of(&g, dict[c], cc);
        for (int d = 0; d < D; d++) y[c * D + d] = 0;
        for (int i = 0; i < m; i++) {
            int64_t rho = elems[i] / C;
            int ch = elems[i] % C;
            int64_t v = voxel_at(&g, cc, K, rho);
            int64_t x = xq[v * C + ch];
            for (int d = 0; d < D; d++) y[c * D + d] += (int64_t)w[(size_t)i * D + d] * x;
        }
    }
}

static int64_t floordiv(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0))) q--;
    return q;
}

/* Grid coordinates shared by all curves of a subset: lo_d / hi_d = min / max
 * of y_d over the dictionary, span = max(1, max_d(hi_d - lo_d)) (one span for
 * all dims keeps the grid isotropic). */
void orc_key_params(const int64_t *y, int64_t n, int D, int64_t *lo, int64_t *span)
{
    int64_t sp = 1;
    for (int d = 0; d < D; d++) {
        int64_t a = y[d], b = y[d];
        for (int64_t c = 1; c < n; c++) {
            if (y[c * D + d] < a) a = y[c * D + d];
            if (y[c * D + d] > b) b = y[c * D + d];
        }
        lo[d] = a;
        if (b - a > sp) sp = b - a;
    }
    *span = sp;
}

/* Interleave (Section II.C): for bit level l = b-1 .. 0, for dim d = 0 .. D-1,
 * shift bit l of v[d] in at the bottom; dim 0 (largest variance) is the most
 * significant at every level. The D*b-bit result is stored right-aligned in
 * W64 words, word 0 most significant. */
static void interleave(const uint32_t *v, int D, int b, int W64, uint64_t *key)
{
    for (int w = 0; w < W64; w++) key[w] = 0;
    for (int l = b - 1; l >= 0; l--)
        for (int d = 0; d < D; d++) {
            for (int w = 0; w < W64 - 1; w++) key[w] = (key[w] << 1) | (key[w + 1] >> 63);
            key[W64 - 1] = (key[W64 - 1] << 1) | ((v[d] >> l) & 1u);
        }
}

/* Hilbert order via J. Skilling's "Programming the Hilbert curve" (AIP Conf.
 * Proc. 707, 2004): convert axis coordinates to the transposed Hilbert index
 * in place, whose bit interleave is the Hilbert index. */
static void hilbert_transpose(uint32_t *X, int D, int b)
{
    uint32_t M = 1u << (b - 1);
    for (uint32_t Qb = M; Qb > 1; Qb >>= 1) {
        uint32_t P = Qb - 1;
        for (int i = 0; i < D; i++) {
            if (X[i] & Qb) {
                X[0] ^= P;
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < D; i++) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t Qb = M; Qb > 1; Qb >>= 1)
        if (X[D - 1] & Qb) t ^= Qb - 1;
    for (int i = 0; i < D; i++) X[i] ^= t;
}

/* Key of one coordinate vector v (already shifted), Morton (curve 0) or
 * Hilbert (curve 1). */
void orc_key_of(const uint32_t *v, int D, int b, int curve, uint64_t *key)
{
    int W64 = (D * b + 63) / 64;
    uint32_t X[64];
    for (int d = 0; d < D; d++) X[d] = v[d];
    if (curve == 1) hilbert_transpose(X, D, b);
    interleave(X, D, b, W64, key);
}

/* Shift of curve j: the same offset floor(j*R/(D+1)) on every dim, the
 * diagonal shifts of shifted-curve kNN search (Liao, Lopez and Leutenegger,
 * 2001). A divisor of D+1 rather than L keeps the offsets off the powers of two,
 * so that a shift changes the curve at every level. */
static int64_t shift_of(int j, int64_t R, int D)
{
    return ((int64_t)j * R) / (D + 1);
}

/* Grid cell of one principal vector: u_d = clamp(floor((y_d - lo_d)*(R-1) /
 * span), 0, R-1), plus the shift of curve j on every dim. */
static void cell_of(const int64_t *y, int D, const int64_t *lo, int64_t span, int64_t R,
                    int j, int L, uint32_t *v)
{
    int64_t sh = shift_of(j, R, D);
    (void)L;
    for (int d = 0; d < D; d++) {
        int64_t u = floordiv((y[d] - lo[d]) * (R - 1), span);
        if (u < 0) u = 0;
        if (u > R - 1) u = R - 1;
        v[d] = (uint32_t)(u + sh);
    }
}

/* Keys of all dictionary patches for curve j. R = 2^(b-1) when L > 1 (half
 * the range is headroom for the shifts), else 2^b. keys is [n][W64]. */
void orc_keys(const int64_t *y, int64_t n, int D, const int64_t *lo, int64_t span,
              int b, int j, int L, int curve, uint64_t *keys)
{
    int W64 = (D * b + 63) / 64;
    int64_t R = (L > 1) ? ((int64_t)1 << (b - 1)) : ((int64_t)1 << b);
    uint32_t v[64];
    for (int64_t c = 0; c < n; c++) {
        cell_of(y + c * D, D, lo, span, R, j, L, v);
        orc_key_of(v, D, b, curve, keys + c * W64);
    }
}

typedef struct {
    int w64;
    const uint64_t *keys;
    const int64_t *ids;
} sort_ctx;

static int cmp_entry(const void *pa, const void *pb, void *arg)
{
    const sort_ctx *cx = (const sort_ctx *)arg;
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    for (int w = 0; w < cx->w64; w++) {
        uint64_t ka = cx->keys[a * cx->w64 + w], kb = cx->keys[b * cx->w64 + w];
        if (ka != kb) return ka < kb ? -1 : 1;
    }
    if (cx->ids[a] != cx->ids[b]) return cx->ids[a] < cx->ids[b] ? -1 : 1;
    return 0;
}

/* Sort a curve's entries by (key, id) ascending (Section II.C sorts the
 * dictionary by curve position; ids are unique, so the order is total).
 * keys [n][W64] and ids [n] are permuted in place. Reentrant: independent
 * curves may be sorted from several threads at once. */
void orc_sort(uint64_t *keys, int64_t *ids, int64_t n, int W64)
{
    int64_t *perm = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) perm[i] = i;
    sort_ctx cx = { W64, keys, ids };
    qsort_r(perm, (size_t)n, sizeof(int64_t), cmp_entry, &cx);
    uint64_t *k2 = malloc(sizeof(uint64_t) * (n > 0 ? n : 1) * W64);
    int64_t *i2 = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        memcpy(k2 + i * W64, keys + perm[i] * W64, sizeof(uint64_t) * W64);
        i2[i] = ids[perm[i]];
    }
    memcpy(keys, k2, sizeof(uint64_t) * n * W64);
    memcpy(ids, i2, sizeof(int64_t) * n);
    free(perm); free(k2); free(i2);
}

/* ------------------------------------------------------------------ */
/* Index query (Fig. 1 b-d)                                            */
/* ------------------------------------------------------------------ */

/* Everything a query needs, as flat arrays filled by the caller. */
typedef struct {
    int nd;
    int64_t shape[ORC_MAXD];
    int C, K, S, D, L, b, curve, window;
    int64_t n;
    const int64_t *dict;          /* [n] */
    float vmin, qscale;
    const int32_t *npix;          /* [S] */
    const int32_t *pix;           /* [S][K^nd] */
    const int8_t *basis;          /* concatenated [m_s][D] */
    const int64_t *basis_off;     /* [S] */
    const int64_t *lo;            /* [S][D] */
    const int64_t *span;          /* [S] */
    const int64_t *sum;           /* [P] subsample sums (for the mean) */
    int64_t nsub;
    const uint64_t *const *keys;  /* [S*L] pointers, curve (s, j) at s*L + j: [n][W64] sorted */
    const int64_t *const *ids;    /* [S*L] pointers, curve (s, j): [n] ids in the same order */
    int norm;                     /* cost of the rescoring: 0 L2, 1 L1 */
} orc_index;

static int key_cmp(const uint64_t *a, const uint64_t *b, int W64)
{
    for (int w = 0; w < W64; w++)
        if (a[w] != b[w]) return a[w] < b[w] ? -1 : 1;
    return 0;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Principal coordinates of a partly known query (Fig. 1c-d: the query object
 * is the index's pixels, moved to principal space). Known elements enter
 * exactly, as for dictionary patches; the unknown ones are imputed with the
 * PCA model fitted to the known ones by least squares (the ad-hoc subspace of
 * Section II). With W the subset's int8 basis, k/u the known/unknown
 * elements, x the byte codes, S the subsample sums and ns their count:
 *   G = W_k^T W_k + I and r = W_k^T (ns x_k - S_k)   (exact integers),
 *   solve G z = r in float64 by Gaussian elimination without pivoting
 *   (G is symmetric positive definite), eliminating column by column and
 *   updating rows j = k+1..D-1, then back substitution;
 *   y_d = A_d + (B_d + sum_e H_de z_e) / ns, with A = W_k^T x_k,
 *   B = W_u^T S_u and H = W_u^T W_u (exact integers), the sum over e
 *   ascending starting from B_d.
 * A fully known query gives y = W^T x exactly, the dictionary's own value. */
static void query_coords(const orc_index *ix, const float *t, const uint8_t *m, int sb,
                         double *yq)
{
    int64_t Kd = ipow(ix->K, ix->nd);
    int D = ix->D;
    const int8_t *w = ix->basis + ix->basis_off[sb];
    int64_t A[64] = {0}, B[64] = {0}, G[64 * 64] = {0}, H[64 * 64] = {0}, r[64] = {0};
    int row = 0;
    for (int i = 0; i < ix->npix[sb]; i++) {
        int64_t rho = ix->pix[sb * Kd + i];
        for (int ch = 0; ch < ix->C; ch++, row++) {
            int64_t e = rho * ix->C + ch;
            const int8_t *wr = w + (int64_t)row * D;
            if (m[rho]) {
                int64_t x = quant1(t[e], ix->vmin, ix->qscale);
                int64_t c = ix->nsub * x - ix->sum[e];
                for (int d = 0; d < D; d++) {
                    A[d] += (int64_t)wr[d] * x;
                    r[d] += (int64_t)wr[d] * c;
                    for (int f = 0; f < D; f++) G[d * D + f] += (int64_t)wr[d] * wr[f];
                }
            } else {
                for (int d = 0; d < D; d++) {
                    B[d] += (int64_t)wr[d] * ix->sum[e];
                    for (int f = 0; f < D; f++) H[d * D + f] += (int64_t)wr[d] * wr[f];
                }
            }
        }
    }
    double a[64 * 64], z[64], rr[64];
    for (int d = 0; d < D; d++) {
        for (int f = 0; f < D; f++) a[d * D + f] = (double)(G[d * D + f] + (d == f));
        rr[d] = (double)r[d];
    }
    for (int k = 0; k < D; k++)
        for (int i = k + 1; i < D; i++) {
            double fct = a[i * D + k] / a[k * D + k];
            for (int j = k + 1; j < D; j++) a[i * D + j] = a[i * D + j] - fct * a[k * D + j];
            rr[i] = rr[i] - fct * rr[k];
        }
    for (int i = D - 1; i >= 0; i--) {
        double sacc = rr[i];
        for (int j = i + 1; j < D; j++) sacc = sacc - a[i * D + j] * z[j];
        z[i] = sacc / a[i * D + i];
    }
    for (int d = 0; d < D; d++) {
        double f = (double)B[d];
        for (int e = 0; e < D; e++) f = f + (double)H[d * D + e] * z[e];
        yq[d] = (double)A[d] + f / (double)ix->nsub;
    }
}

/* Grid cell of a real query vector: u_d = clamp(floor((y_d - lo_d)*(R-1) /
 * span), 0, R-1) in float64, plus the curve's shift. For integer y this is
 * the same cell as the exact integer rule. */
static void cell_of_real(const double *y, int D, const int64_t *lo, int64_t span, int64_t R,
                         int j, uint32_t *v)
{
    int64_t sh = shift_of(j, R, D);
    for (int d = 0; d < D; d++) {
        double u = floor(((y[d] - (double)lo[d]) * (double)(R - 1)) / (double)span);
        if (!(u >= 0.0)) u = 0.0;
        if (u > (double)(R - 1)) u = (double)(R - 1);
        v[d] = (uint32_t)((int64_t)u + sh);
    }
}

/* The query's subset (Fig. 1b: the index whose pixels best cover the search
 * area): the subset with the largest fraction k_s / n_s of its pixels known
 * in the target mask m, compared exactly as k_s * n_b > k_b * n_s; on equal
 * fractions the lower subset is kept. pix is [S][Kd], npix[S]. */
int orc_choose_subset(const int32_t *npix, const int32_t *pix, int S, int64_t Kd,
                      const uint8_t *m)
{
    int sb = 0;
    int64_t kb = -1, nb = 1;
    for (int s = 0; s < S; s++) {
        int64_t k = 0, ns = npix[s];
        for (int i = 0; i < ns; i++) k += m[pix[s * Kd + i]];
        if (kb < 0 || k * nb > kb * ns) { sb = s; kb = k; nb = ns; }
    }
    return sb;
}

/* The candidate window on one sorted curve: p = the first position whose key
 * is >= the query key qk (lower bound; n if none), then the W positions
 * starting at lo = p - floor(W/2), moved inside the array:
 * lo = clamp(lo, 0, max(n - W, 0)). Returns lo; the window is
 * [lo, min(lo + W, n)). keys is [n][W64], sorted; *p_out receives p. */
int64_t orc_window(const uint64_t *keys, int64_t n, int W64, const uint64_t *qk, int W,
                   int64_t *p_out)
{
    int64_t a = 0, z = n;
    while (a < z) {
        int64_t mid = a + (z - a) / 2;
        if (key_cmp(keys + mid * W64, qk, W64) < 0) a = mid + 1;
        else z = mid;
    }
    if (p_out) *p_out = a;
    int64_t lo = a - W / 2;
    int64_t lmax = n - W;
    if (lmax < 0) lmax = 0;
    if (lo > lmax) lo = lmax;
    if (lo < 0) lo = 0;
    return lo;
}

/* Exposed for tests: subset choice and real principal coordinates. */
int orc_query_point(const orc_index *ix, const float *t, const uint8_t *m, double *yq)
{
    int64_t Kd = ipow(ix->K, ix->nd);
    int sb = orc_choose_subset(ix->npix, ix->pix, ix->S, Kd, m);
    query_coords(ix, t, m, sb, yq);
    return sb;
}

/* One query against the multi-index:
 *  1. subset s* with the largest fraction of its pixels known (Fig. 1b),
 *     compared exactly by cross-multiplication, ties to the lower s;
 *  2-3. real principal coordinates of the subset's elements (query_coords),
 *     grid cell, one key per shifted curve;
 *  4. per curve, p = first position whose key is >= the query key, window
 *     [lo, lo+W) with lo = clamp(p - W/2, 0, max(n-W, 0));
 *  5. the union of the windows' ids, rescored with the masked cost (Fig. 1d:
 *     full scan in image space over the candidates); best = min (cost, id).
 * Writes the sorted unique candidate ids to cand (capacity L*W) and returns
 * their count. */
int64_t orc_query_one(const orc_index *ix, const float *vol, const float *t,
                      const uint8_t *m, int64_t *best_id, float *best_cost,
                      int64_t *cand, int32_t *subset_out)
{
    grid_t g = make_grid(ix->nd, ix->shape);
    int64_t Kd = ipow(ix->K, ix->nd);
    int64_t P = Kd * ix->C;
    int W64 = (ix->D * ix->b + 63) / 64;
    int64_t R = (ix->L > 1) ? ((int64_t)1 << (ix->b - 1)) : ((int64_t)1 << ix->b);
    /* 1 */
    int sb = orc_choose_subset(ix->npix, ix->pix, ix->S, Kd, m);
    if (subset_out) *subset_out = sb;
    /* 2, 3 */
    double yq[64];
    query_coords(ix, t, m, sb, yq);
    (void)P;
    /* 4 */
    int64_t nc = 0;
    uint64_t qk[4];
    uint32_t v[64];
    for (int j = 0; j < ix->L; j++) {
        cell_of_real(yq, ix->D, ix->lo + sb * ix->D, ix->span[sb], R, j, v);
        orc_key_of(v, ix->D, ix->b, ix->curve, qk);
        const uint64_t *keys = ix->keys[sb * ix->L + j];
        const int64_t *ids = ix->ids[sb * ix->L + j];
        int64_t lo = orc_window(keys, ix->n, W64, qk, ix->window, NULL);
        int64_t hi = lo + ix->window;
        if (hi > ix->n) hi = ix->n;
        for (int64_t i = lo; i < hi; i++) cand[nc++] = ids[i];
    }
    /* 5 */
    qsort(cand, (size_t)nc, sizeof(int64_t), cmp_i64);
    int64_t u = 0;
    for (int64_t i = 0; i < nc; i++)
        if (u == 0 || cand[i] != cand[u - 1]) cand[u++] = cand[i];
    int64_t bi = -1;
    float bc = INFINITY;
    for (int64_t i = 0; i < u; i++) {
        float c = cost_of(ix->norm, vol, &g, ix->C, ix->K, cand[i], t, m);
        if (bi < 0 || c < bc) { bc = c; bi = cand[i]; }
    }
    *best_id = bi;
    *best_cost = bc;
    return u;
}

/* Batch form: cand is [Q][L*W] padded with -1, ncand[Q]. */
void orc_query(const orc_index *ix, const float *vol, const float *t, const uint8_t *m,
               int64_t Q, int64_t *best_id, float *best_cost, int64_t *cand,
               int32_t *ncand, int32_t *subset)
{
    int64_t Kd = ipow(ix->K, ix->nd), cap = (int64_t)ix->L * ix->window;
    for (int64_t q = 0; q < Q; q++) {
        int64_t *cq = cand + q * cap;
        for (int64_t i = 0; i < cap; i++) cq[i] = -1;
        int64_t u = orc_query_one(ix, vol, t + q * Kd * ix->C, m + q * Kd,
                                  best_id + q, best_cost + q, cq, subset ? subset + q : 0);
        for (int64_t i = u; i < cap; i++) cq[i] = -1;
        ncand[q] = (int32_t)u;
    }
}

/* ------------------------------------------------------------------ */
/* Exact k-NN query (Sections II.D-E)                                   */
/* ------------------------------------------------------------------ */

/* Inverse of the Morton interleave: bit l*D + (D-1-d) of the key (word 0
 * most significant) is bit l of coordinate d. */
void orc_morton_decode(const uint64_t *key, int D, int b, uint32_t *v)
{
    int W64 = (D * b + 63) / 64;
    for (int d = 0; d < D; d++) v[d] = 0;
    for (int l = 0; l < b; l++)
        for (int d = 0; d < D; d++) {
            int pos = l * D + (D - 1 - d);
            uint64_t bit = (key[W64 - 1 - pos / 64] >> (pos % 64)) & 1u;
            v[d] |= (uint32_t)bit << l;
        }
}

typedef struct { int64_t dist, id; } dist_id;

static int cmp_dist_id(const void *a, const void *b)
{
    const dist_id *x = (const dist_id *)a, *y = (const dist_id *)b;
    if (x->dist != y->dist) return x->dist < y->dist ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* The k-NN query of Section II.D on the unshifted Morton curve, written as
 * what it computes: the query's subset and grid cell as in the windowed
 * query (steps 1-3 and the cell of curve 0), every dictionary patch's cell
 * on that curve (decoded from its key), the k patches of smallest squared
 * Euclidean cell distance (ties by lower id), then the cost of Section II
 * (or its L1 variant) over those k, lowest (cost, id). The recursive
 * outside-in traversal of the paper only avoids visiting the rest, so its
 * result is this set. cand receives the k ids ascending (fewer when
 * n < k); returns their count, or -1 for a Hilbert-ordered index. */
int64_t orc_knn_one(const orc_index *ix, const float *vol, const float *t, const uint8_t *m,
                    int k, int64_t *best_id, float *best_cost, int64_t *cand)
{
    if (ix->curve != 0 || k < 1) return -1;
    /* squared cell distances summed in int64: D * (2^b)^2 below 2^62 */
    int lg = 0;
    while ((1 << lg) < ix->D) lg++;
    if (2 * ix->b + lg > 62) return -1;
    grid_t g = make_grid(ix->nd, ix->shape);
    int64_t Kd = ipow(ix->K, ix->nd);
    int W64 = (ix->D * ix->b + 63) / 64;
    int64_t R = (ix->L > 1) ? ((int64_t)1 << (ix->b - 1)) : ((int64_t)1 << ix->b);
    int sb = orc_choose_subset(ix->npix, ix->pix, ix->S, Kd, m);
    double yq[64];
    query_coords(ix, t, m, sb, yq);
    uint32_t u[64], v[64];
    cell_of_real(yq, ix->D, ix->lo + sb * ix->D, ix->span[sb], R, 0, u);
    const uint64_t *keys = ix->keys[sb * ix->L];
    const int64_t *ids = ix->ids[sb * ix->L];
    dist_id *all = malloc(sizeof(dist_id) * (size_t)ix->n);
    for (int64_t i = 0; i < ix->n; i++) {
        orc_morton_decode(keys + i * W64, ix->D, ix->b, v);
        int64_t dsum = 0;
        for (int d = 0; d < ix->D; d++) {
            int64_t e = (int64_t)v[d] - (int64_t)u[d];
            dsum += e * e;
        }
        all[i].dist = dsum;
        all[i].id = ids[i];
    }
    qsort(all, (size_t)ix->n, sizeof(dist_id), cmp_dist_id);
    int64_t nk = ix->n < k ? ix->n : k;
    for (int64_t i = 0; i < nk; i++) cand[i] = all[i].id;
    free(all);
    qsort(cand, (size_t)nk, sizeof(int64_t), cmp_i64);
    int64_t bi = -1;
    float bc = INFINITY;
    for (int64_t i = 0; i < nk; i++) {
        float c = cost_of(ix->norm, vol, &g, ix->C, ix->K, cand[i], t, m);
        if (bi < 0 || c < bc) { bc = c; bi = cand[i]; }
    }
    *best_id = bi;
    *best_cost = bc;
    return nk;
}

/* Batch form: cand is [Q][k] padded with -1, ncand[Q]; returns -1 if the
 * index cannot answer k-NN queries (Hilbert order, k < 1). */
int orc_knn(const orc_index *ix, const float *vol, const float *t, const uint8_t *m, int64_t Q,
            int k, int64_t *best_id, float *best_cost, int64_t *cand, int32_t *ncand)
{
    int64_t Kd = ipow(ix->K, ix->nd);
    for (int64_t q = 0; q < Q; q++) {
        int64_t *cq = cand + q * k;
        for (int i = 0; i < k; i++) cq[i] = -1;
        int64_t nc = orc_knn_one(ix, vol, t + q * Kd * ix->C, m + q * Kd, k, best_id + q,
                                 best_cost + q, cq);
        if (nc < 0) return -1;
        ncand[q] = (int32_t)nc;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Inpainting loop (Section I; Criminisi order)                        */
/* ------------------------------------------------------------------ */

static double mean_intensity(const float *vol, int64_t v, int C)
{
    double s = 0.0;
    for (int ch = 0; ch < C; ch++) s += (double)vol[v * C + ch];
    return s / (double)C;
}

/* Criminisi-style priority of a front voxel p: P = Cp * Dp with
 *  Cp = (sum of confidence over the known in-bounds voxels of the box,
 *        rho ascending) / K^nd;
 *  Dp = |grad I^perp . n| (2D) or |grad I x n| (3D), where I is the channel
 *       mean, its gradient uses central differences where both neighbours are
 *       known, one-sided ones where one is, else 0; n is the difference of the
 *       known-indicator (out of bounds counts as known) across p, normalised
 *       (Dp = 0 if it vanishes).
 * The paper only cites Criminisi et al. for this heuristic; the formulas here
 * are a reading of it, pinned by closed forms on linear ramps (half-plane,
 * half-space and corner holes, borders, several channels, confidence below
 * one). */
static void priority_of(const float *vol, const uint8_t *mask, const double *conf,
                        const grid_t *g, int C, int K, int64_t p, double *Pout, double *Cout)
{
    int64_t Kd = ipow(K, g->nd), cc[ORC_MAXD];
    coords_of(g, p, cc);
    double cs = 0.0;
    for (int64_t rho = 0; rho < Kd; rho++) {
        int64_t v = voxel_at(g, cc, K, rho);
        if (v >= 0 && mask[v]) cs += conf[v];
    }
    double Cp = cs / (double)Kd;
    double gr[ORC_MAXD], nr[ORC_MAXD], nn = 0.0;
    double I0 = mean_intensity(vol, p, C);
    for (int i = 0; i < g->nd; i++) {
        int hasp = cc[i] + 1 < g->shape[i], hasm = cc[i] > 0;
        int64_t vp = p + g->stride[i], vm = p - g->stride[i];
        int kp = hasp && mask[vp], km = hasm && mask[vm];
        if (kp && km) gr[i] = (mean_intensity(vol, vp, C) - mean_intensity(vol, vm, C)) / 2.0;
        else if (kp) gr[i] = mean_intensity(vol, vp, C) - I0;
        else if (km) gr[i] = I0 - mean_intensity(vol, vm, C);
        else gr[i] = 0.0;
        int ip = hasp ? mask[vp] : 1, im = hasm ? mask[vm] : 1;
        nr[i] = (double)(ip - im);
        nn += nr[i] * nr[i];
    }
    double Dp = 0.0;
    if (nn > 0.0) {
        double len = sqrt(nn);
        for (int i = 0; i < g->nd; i++) nr[i] = nr[i] / len;
        if (g->nd == 2) {
            Dp = fabs(gr[0] * nr[1] - gr[1] * nr[0]);
        } else {
            double c0 = gr[1] * nr[2] - gr[2] * nr[1];
            double c1 = gr[2] * nr[0] - gr[0] * nr[2];
            double c2 = gr[0] * nr[1] - gr[1] * nr[0];
            Dp = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
        }
    }
    *Pout = Cp * Dp;
    *Cout = Cp;
}

/* The priority and confidence term of one front voxel p as the fill loop
 * computes them (the reading above), given the confidence map conf
 * (float64 per voxel). */
void orc_priority(const float *vol, const uint8_t *mask, const double *conf, int nd,
                  const int64_t *shape, int C, int K, int64_t p, double *P, double *Cp)
{
    grid_t g = make_grid(nd, shape);
    priority_of(vol, mask, conf, &g, C, K, p, P, Cp);
}

/* The fill loop: until no voxel is unknown, take the front voxel with the
 * highest (priority, confidence, -id) (order 0) or the lowest id (order 1),
 * query its target patch (mode 0 = full scan over dict, mode 3 = index), copy
 * the chosen patch's values into the unknown in-bounds voxels of the box,
 * mark them known and give them the chosen voxel's Cp. vol and mask are
 * updated in place; the dictionary is the one given (fixed for the run).
 * Logs (centre, source, cost) per iteration up to cap. Returns the number of
 * iterations, or -1 if unknown voxels remain but the front is empty, -2 if
 * the dictionary is empty. */
int64_t orc_inpaint(float *vol, uint8_t *mask, int nd, const int64_t *shape, int C, int K,
                    int order, int mode, const int64_t *dict, int64_t n,
                    const orc_index *ix, int64_t cap, int64_t *log_centre,
                    int64_t *log_source, float *log_cost)
{
    grid_t g = make_grid(nd, shape);
    int64_t Kd = ipow(K, nd), cc[ORC_MAXD], iters = 0;
    if (n <= 0) return -2;
    double *conf = malloc(sizeof(double) * g.nvox);
    for (int64_t v = 0; v < g.nvox; v++) conf[v] = mask[v] ? 1.0 : 0.0;
    float *t = malloc(sizeof(float) * Kd * C);
    uint8_t *m = malloc(Kd);
    int64_t *cand = malloc(sizeof(int64_t) * (ix ? (int64_t)ix->L * ix->window : 1));
    int64_t *front = malloc(sizeof(int64_t) * g.nvox);
    for (;;) {
        int64_t unknown = 0;
        for (int64_t v = 0; v < g.nvox; v++) unknown += !mask[v];
        if (!unknown) break;
        int64_t nf = orc_front(mask, nd, shape, front, g.nvox);
        if (nf == 0) { iters = -1; break; }
        int64_t best = front[0];
        double bp = 0.0, bcf = 0.0;
        if (order == 0) {
            for (int64_t i = 0; i < nf; i++) {
                double pp, cp;
                priority_of(vol, mask, conf, &g, C, K, front[i], &pp, &cp);
                if (i == 0 || pp > bp || (pp == bp && cp > bcf)) {
                    best = front[i]; bp = pp; bcf = cp;
                }
            }
        } else {
            priority_of(vol, mask, conf, &g, C, K, best, &bp, &bcf);
        }
        orc_extract(vol, mask, nd, shape, C, K, &best, 1, t, m);
        int64_t src;
        float cost;
        if (mode == 3 && ix) {
            orc_query_one(ix, vol, t, m, &src, &cost, cand, 0);
        } else {
            orc_brute(vol, nd, shape, C, K, dict, n, t, m, 1, &src, &cost, 0);
        }
        int64_t sc[ORC_MAXD];
        coords_of(&g, best, cc);
        coords_of(&g, src, sc);
        for (int64_t rho = 0; rho < Kd; rho++) {
            int64_t v = voxel_at(&g, cc, K, rho);
            if (v < 0 || mask[v]) continue;
            int64_t s = voxel_at(&g, sc, K, rho);
            for (int ch = 0; ch < C; ch++) vol[v * C + ch] = vol[s * C + ch];
            mask[v] = 1;
            conf[v] = bcf;
        }
        if (iters < cap) {
            log_centre[iters] = best;
            log_source[iters] = src;
            log_cost[iters] = cost;
        }
        iters++;
    }
    free(conf); free(t); free(m); free(cand); free(front);
    return iters;
}
