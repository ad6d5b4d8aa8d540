/*
 * ibmc_oracle.c -- plain, slow, obviously-correct CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke entry and the
 * CPU-baseline leg of the benchmark call into this file.  The product path
 * (the HIP library) never links it, and this file includes no header, table
 * or helper of that library.
 *
 * What it computes, and where the paper defines it:
 *   - neuron potential u = sum_j w_j * i_j + b              (Sec. II-A, Eq. (1))
 *   - sigmoid N(u) = 1 / (1 + e^-u)                          (Sec. II-A, Eq. (2))
 *   - the safety property "the classification of every image in the
 *     restricted set equals the clean classification"        (Sec. III-C, Eqs. (9)-(10))
 *     checked with an incrementally growing bound k           (Sec. II-B)
 *   - sign / value / distance change and the SS, DS, SV, DV
 *     neuron-pair covers with their coverage literal          (Sec. III-B, Eqs. (3)-(6))
 *   - Euclidean distance                                     (Sec. III-C, Eq. (7))
 *
 * Readings where the paper is silent (the same ones the library documents):
 *   - integer networks: int8 weights, int32 bias, hidden activation
 *     a = min(max(floor(u / 2^s), 0), 127)  (ReLU folded into the clamp);
 *     input activation a0 = pixel value 0..255; logits are the last
 *     layer's potentials; the label is the lowest index of the maximum.
 *   - the restricted set at bound k: all images that differ from the clean
 *     one in exactly k pixels p1 < ... < pk, pixel pj set to
 *     clamp(x[pj] + D[ij], 0, 255) for a delta index ij.  Points are counted
 *     as enumerated (duplicates from 0 in D or from clamping included).
 *   - the L2-ball restricted set (Eq. (9) with the distance of Eq. (7) on
 *     pixel values 0..255, b^2 given as an integer r2): every image x' in
 *     {0..255}^n with sum (x' - x)^2 <= r2, at bound k those that differ
 *     from the clean one in exactly k pixels (nothing is clamped: offsets
 *     that leave [0, 255] do not give an image); points are counted once.
 *   - rank of a point: (number of k-subsets lexicographically before S)
 *     * |D|^k + the delta indices read as a base-|D| number, i1 most
 *     significant.
 *   - sign(0) = 1; value change = no sign change and
 *     den * max(|a|,|b|) >= num * min(|a|,|b|) with max(|a|,|b|) > 0;
 *     distance change = no sign change in the whole layer and
 *     sum (a-b)^2 >= dist_sq_min; the SS first condition is read as a sign
 *     change of the condition neuron (as in SV); coverage counts neurons
 *     of the non-input layers.
 *   - float networks: a0 = x / 256, sigmoid on hidden layers, linear logits,
 *     evaluated in double.
 *
 * Arithmetic: integer potentials are accumulated in int64 and checked against
 * the int32 range the library promises; float work is done in double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_RANGE (-2)
#define ORC_E_OOM (-3)
#define ORC_TRAIN_MAX_LAYERS 16

/* ------------------------------------------------------------------------ */
/* network shapes (the oracle's own flat layout)                            */
/*   W: layers concatenated, layer l row-major [dims[l+1]][dims[l]]         */
/*   b: layers concatenated, [dims[l+1]]                                    */
/*   potentials: layers 1..L concatenated                                   */
/* ------------------------------------------------------------------------ */

static int64_t total_units(int L, const int32_t *dims) {
    int64_t t = 0;
    for (int l = 1; l <= L; ++l) t += dims[l];
    return t;
}

static int max_width(int L, const int32_t *dims) {
    int m = 0;
    for (int l = 0; l <= L; ++l) if (dims[l] > m) m = dims[l];
    return m;
}

/* Integer forward pass of one image (Eq. (1) per neuron, requantised ReLU
 * between layers).  pot receives every layer's potentials (may be NULL).
 * Returns ORC_E_RANGE if a potential leaves the int32 range. */
static int q8_forward(int L, const int32_t *dims, const int8_t *W, const int32_t *b,
                      const int32_t *shift, const uint8_t *x, int64_t *act_a, int64_t *act_b,
                      int64_t *pot, int32_t *label, int *top_tie) {
    int64_t *in = act_a, *out = act_b;
    for (int i = 0; i < dims[0]; ++i) in[i] = x[i];
    const int8_t *w = W;
    const int32_t *bb = b;
    int64_t po = 0;
    for (int l = 1; l <= L; ++l) {
        int nin = dims[l - 1], nout = dims[l];
        for (int j = 0; j < nout; ++j) {
            int64_t u = bb[j];
            const int8_t *row = w + (int64_t)j * nin;
            for (int i = 0; i < nin; ++i) u += (int64_t)row[i] * in[i];
            if (u > INT32_MAX || u < INT32_MIN) return ORC_E_RANGE;
            if (pot) pot[po + j] = u;
            if (l < L) {
                /* floor(u / 2^s), then clamp to [0, 127] */
                int64_t d = (int64_t)1 << shift[l - 1];
                int64_t q = u / d;
                if (u % d != 0 && u < 0) q -= 1;   /* C division truncates toward zero */
                if (q < 0) q = 0;
                if (q > 127) q = 127;
                out[j] = q;
            } else {
                out[j] = u;
            }
        }
        po += nout;
        w += (int64_t)nout * nin;
        bb += nout;
        int64_t *t = in; in = out; out = t;
    }
    /* label: lowest index attaining the maximum logit */
    int nc = dims[L];
    int best = 0;
    for (int j = 1; j < nc; ++j) if (in[j] > in[best]) best = j;
    if (label) *label = best;
    if (top_tie) {
        int cnt = 0;
        for (int j = 0; j < nc; ++j) cnt += (in[j] == in[best]);
        *top_tie = cnt > 1;
    }
    return ORC_OK;
}

int orc_q8_forward(int L, const int32_t *dims, const int8_t *W, const int32_t *b,
                   const int32_t *shift, const uint8_t *x, int64_t *pot, int32_t *label) {
    if (L < 1 || !dims || !W || !b || !x) return ORC_E_INVALID;
    int mw = max_width(L, dims);
    int64_t *a = malloc(sizeof(int64_t) * mw), *c = malloc(sizeof(int64_t) * mw);
    if (!a || !c) { free(a); free(c); return ORC_E_OOM; }
    int rc = q8_forward(L, dims, W, b, shift, x, a, c, pot, label, NULL);
    free(a); free(c);
    return rc;
}

/* Table sigmoid (the paper's CUDA code evaluated the sigmoid from a table,
 * Sec. IV-D): knots u_i = -8 + i/16, i = 0..256, values sigma(u_i) rounded to
 * FP32; between knots linear interpolation, outside [-8, 8] the end values. */
#define ORC_LUT_N 256
static double lut_value(int i) { return (double)(float)(1.0 / (1.0 + exp(-(-8.0 + i / 16.0)))); }

double orc_lut_sigmoid(double u) {
    double t = (u + 8.0) * 16.0;
    if (!(t > 0.0)) return lut_value(0);
    if (t >= ORC_LUT_N) return lut_value(ORC_LUT_N);
    int i = (int)floor(t);
    double f = t - i;
    double a = lut_value(i), c = lut_value(i + 1);
    return a + f * (c - a);
}

/* Double-precision forward of the float network (Eq. (2) on hidden layers;
 * lut: the table sigmoid instead).  logits (nullable) receives the last
 * layer. */
static void f64_forward_ex(int L, const int32_t *dims, const double *W, const double *b,
                           const uint8_t *x, double *act_a, double *act_b, double *pot,
                           int32_t *label, double *margin, double *top, int lut, double *logits);

static void f64_forward(int L, const int32_t *dims, const double *W, const double *b,
                        const uint8_t *x, double *act_a, double *act_b, double *pot,
                        int32_t *label, double *margin, double *top) {
    f64_forward_ex(L, dims, W, b, x, act_a, act_b, pot, label, margin, top, 0, NULL);
}

static void f64_forward_ex(int L, const int32_t *dims, const double *W, const double *b,
                           const uint8_t *x, double *act_a, double *act_b, double *pot,
                           int32_t *label, double *margin, double *top, int lut, double *logits) {
    double *in = act_a, *out = act_b;
    for (int i = 0; i < dims[0]; ++i) in[i] = (double)x[i] / 256.0;
    const double *w = W, *bb = b;
    int64_t po = 0;
    for (int l = 1; l <= L; ++l) {
        int nin = dims[l - 1], nout = dims[l];
        for (int j = 0; j < nout; ++j) {
            double u = bb[j];
            const double *row = w + (int64_t)j * nin;
            for (int i = 0; i < nin; ++i) u += row[i] * in[i];
            if (pot) pot[po + j] = u;
            out[j] = (l < L) ? (lut ? orc_lut_sigmoid(u) : 1.0 / (1.0 + exp(-u))) : u;
        }
        po += nout;
        w += (int64_t)nout * nin;
        bb += nout;
        double *t = in; in = out; out = t;
    }
    int nc = dims[L];
    int best = 0;
    for (int j = 1; j < nc; ++j) if (in[j] > in[best]) best = j;
    double second = -INFINITY;
    for (int j = 0; j < nc; ++j) if (j != best && in[j] > second) second = in[j];
    if (label) *label = best;
    if (margin) *margin = (nc > 1) ? in[best] - second : INFINITY;
    if (top) *top = in[best];
    if (logits) memcpy(logits, in, sizeof(double) * nc);
}

int orc_f64_forward(int L, const int32_t *dims, const double *W, const double *b,
                    const uint8_t *x, double *pot, int32_t *label, double *margin) {
    if (L < 1 || !dims || !W || !b || !x) return ORC_E_INVALID;
    int mw = max_width(L, dims);
    double *a = malloc(sizeof(double) * mw), *c = malloc(sizeof(double) * mw);
    if (!a || !c) { free(a); free(c); return ORC_E_OOM; }
    f64_forward(L, dims, W, b, x, a, c, pot, label, margin, NULL);
    free(a); free(c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* counting and decoding points                                              */
/* ------------------------------------------------------------------------ */

/* binomial coefficient by the multiplicative recurrence (exact while it fits) */
static int64_t binom(int64_t n, int64_t k) {
    if (k < 0 || n < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    __int128 r = 1;
    for (int64_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return (int64_t)r;
}

static int64_t ipow(int64_t a, int e) {
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= a;
    return r;
}

/* Number of points at bound k: the k-subsets of the n pixels times the
 * |D|^k delta choices. */
int64_t orc_points(int n, int m, int k) {
    if (k < 0 || k > n) return 0;
    return binom(n, k) * ipow(m, k);
}

/* Decode a rank at bound k into its pixels and delta indices.  The subset
 * part is found by walking the lexicographic order: the k-subsets whose
 * first element is q number C(n-1-q, k-1); skip whole blocks until the rank
 * falls inside one, then recurse on the remaining elements. */
int orc_decode(int n, int m, int k, int64_t rank, int32_t *pix, int32_t *didx) {
    if (k < 0 || k > n || m < 1) return ORC_E_INVALID;
    int64_t md = ipow(m, k);
    int64_t total = binom(n, k) * md;
    if (rank < 0 || rank >= total) return ORC_E_INVALID;
    int64_t srank = rank / md, drank = rank % md;
    for (int j = k - 1; j >= 0; --j) { didx[j] = (int32_t)(drank % m); drank /= m; }
    int q = 0;
    for (int j = 0; j < k; ++j) {
        for (;; ++q) {
            int64_t block = binom(n - 1 - q, k - 1 - j);
            if (srank < block) break;
            srank -= block;
        }
        pix[j] = q++;
    }
    return ORC_OK;
}

/* Apply a point to a copy of the clean image. */
static void apply_point(const uint8_t *x, int n, const int16_t *D, int k, const int32_t *pix,
                        const int32_t *didx, uint8_t *xp) {
    memcpy(xp, x, (size_t)n);
    for (int j = 0; j < k; ++j) {
        int v = (int)x[pix[j]] + (int)D[didx[j]];
        if (v < 0) v = 0;
        if (v > 255) v = 255;
        xp[pix[j]] = (uint8_t)v;
    }
}

/* ------------------------------------------------------------------------ */
/* exhaustive check (Sec. II-B bound loop around the Sec. III-C property)    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t *k; int64_t *rank; int32_t *label; double *margin;
    int64_t n, cap;
} rec_list;

static int rec_push(rec_list *r, int32_t k, int64_t rank, int32_t label, double margin) {
    if (r->n == r->cap) {
        int64_t nc = r->cap ? r->cap * 2 : 64;
        int32_t *a = realloc(r->k, sizeof(int32_t) * nc);
        if (!a) return ORC_E_OOM;
        r->k = a;
        int64_t *bq = realloc(r->rank, sizeof(int64_t) * nc);
        if (!bq) return ORC_E_OOM;
        r->rank = bq;
        int32_t *c = realloc(r->label, sizeof(int32_t) * nc);
        if (!c) return ORC_E_OOM;
        r->label = c;
        double *d = realloc(r->margin, sizeof(double) * nc);
        if (!d) return ORC_E_OOM;
        r->margin = d;
        r->cap = nc;
    }
    r->k[r->n] = k; r->rank[r->n] = rank; r->label[r->n] = label; r->margin[r->n] = margin;
    r->n++;
    return ORC_OK;
}

static void rec_free(rec_list *r) { free(r->k); free(r->rank); free(r->label); free(r->margin); }

/* Advance a k-subset (strictly increasing) to its lexicographic successor
 * whose first element stays `first`; returns 0 when exhausted. */
static int next_subset_tail(int32_t *pix, int k, int n) {
    for (int j = k - 1; j >= 1; --j) {
        if (pix[j] < n - (k - j)) {
            pix[j]++;
            for (int t = j + 1; t < k; ++t) pix[t] = pix[t - 1] + 1;
            return 1;
        }
    }
    return 0;
}

static int next_digits(int32_t *d, int k, int m) {
    for (int j = k - 1; j >= 0; --j) {
        if (++d[j] < m) return 1;
        d[j] = 0;
    }
    return 0;
}

typedef struct {
    int is_float;
    int L;
    const int32_t *dims;
    const int8_t *Wq; const int32_t *bq; const int32_t *shift;
    const double *Wf; const double *bf;
    double tie_rel;   /* float only: flag when margin <= tie_rel * max(1, |top|) */
    int lut;          /* float only: the table sigmoid */
    int literal;      /* 1: the threshold literal with reference value V (below) */
    double V;
} net_ref;

/* The paper's literal l_image_misclassified (Sec. III-C): the desired class
 * D falls below the reference value V while some other class exceeds it,
 * (z_D < V) and (max_{i != D} z_i > V).  *eq: how close the two compared
 * values come to V (0 when one equals it). */
static int literal_holds(const double *z, int nc, int D, double V, double *closest) {
    double other = -INFINITY;
    for (int i = 0; i < nc; ++i) if (i != D && z[i] > other) other = z[i];
    double a = fabs(z[D] - V), c = fabs(other - V);
    *closest = a < c ? a : c;
    return z[D] < V && other > V;
}

/* Evaluate one image against the clean label `clean` (-1: the clean image
 * itself).  Returns the label, *viol (the property's violation: the label
 * changes, or the literal holds), *tie (integer: exact top-2 tie, or with
 * the literal a compared value equal to V; float: the near-tie flag of the
 * decision taken) and the float margin. */
static int eval_image(const net_ref *nr, const uint8_t *xp, void *sa, void *sb, int32_t clean,
                      int32_t *label, int *viol, int *tie, double *margin) {
    int nc = nr->dims[nr->L];
    double z[1024];
    if (!nr->is_float) {
        *margin = 0.0;
        int64_t *in_last;
        int rc = q8_forward(nr->L, nr->dims, nr->Wq, nr->bq, nr->shift, xp, sa, sb, NULL, label, tie);
        if (rc) return rc;
        /* the logits sit in the buffer the last layer wrote */
        in_last = (nr->L % 2) ? (int64_t *)sb : (int64_t *)sa;
        if (nr->literal) {
            for (int i = 0; i < nc; ++i) z[i] = (double)in_last[i];
            double closest;
            *viol = clean >= 0 && literal_holds(z, nc, clean, nr->V, &closest);
            *tie = clean >= 0 ? closest == 0.0 : *tie;
        } else {
            *viol = clean >= 0 && *label != clean;
        }
        return ORC_OK;
    }
    double top;
    f64_forward_ex(nr->L, nr->dims, nr->Wf, nr->bf, xp, sa, sb, NULL, label, margin, &top, nr->lut, z);
    if (nr->literal && clean >= 0) {
        double closest;
        *viol = literal_holds(z, nc, clean, nr->V, &closest);
        double scale = fabs(nr->V) > 1.0 ? fabs(nr->V) : 1.0;
        *tie = closest <= nr->tie_rel * scale;
        return ORC_OK;
    }
    double scale = fabs(top) > 1.0 ? fabs(top) : 1.0;
    *tie = *margin <= nr->tie_rel * scale;
    *viol = clean >= 0 && *label != clean;
    return ORC_OK;
}

/* Enumerate bound k with first pixel `first`.  Ranks of these points form the
 * contiguous range starting at base_rank, visited in increasing order. */
static int enum_first(const net_ref *nr, const uint8_t *x, const int16_t *D, int m, int k,
                      int first, int64_t base_rank, int32_t clean, rec_list *cex, rec_list *ties,
                      int64_t *n_ties, uint8_t *xp, void *sa, void *sb) {
    int n = nr->dims[0];
    int32_t pix[64], dig[64];
    pix[0] = first;
    for (int j = 1; j < k; ++j) pix[j] = first + j;
    int64_t rank = base_rank;
    do {
        for (int j = 0; j < k; ++j) dig[j] = 0;
        do {
            apply_point(x, n, D, k, pix, dig, xp);
            int32_t lab; int tie, viol; double margin;
            int rc = eval_image(nr, xp, sa, sb, clean, &lab, &viol, &tie, &margin);
            if (rc) return rc;
            if (viol) {
                rc = rec_push(cex, k, rank, lab, margin);
                if (rc) return rc;
            }
            if (tie) {
                (*n_ties)++;
                if (ties) { rc = rec_push(ties, k, rank, lab, margin); if (rc) return rc; }
            }
            rank++;
        } while (next_digits(dig, k, m));
    } while (k > 1 && next_subset_tail(pix, k, n));
    return ORC_OK;
}

/* L2-ball domain (Sec. III-C, Eq. (9), the restriction R with the Euclidean
 * distance of Eq. (7)): the images x' in {0..255}^n with
 * sum_p (x'_p - x_p)^2 <= r2, grouped by support size k (the pixels where
 * x' differs from x).  For ranks a point of level k is written as its k
 * pixels and one digit per pixel: the offset e = x'_p - x_p (nonzero,
 * |e| <= rd = min(floor(sqrt(r2)), 255)) has digit e + rd when negative and
 * e + rd - 1 when positive, so m = 2 rd digits per pixel and the rank is
 * (subset rank) m^k + (digits read in base m), as in the box domain. */
int orc_ball_digits(int64_t r2) {
    if (r2 < 0) return 0;
    int64_t r = 0;
    while ((r + 1) * (r + 1) <= r2) ++r;
    return (int)(r < 255 ? r : 255);
}

static int ball_offset(int digit, int rd) { return digit < rd ? digit - rd : digit - rd + 1; }

/* Enumerate level k of the ball with first pixel `first` in rank order,
 * skipping digit vectors that leave [0, 255] or the ball.  *n_points counts
 * the points of the domain visited. */
static int enum_first_ball(const net_ref *nr, const uint8_t *x, int64_t r2, int rd, int k, int first,
                           int64_t base_rank, int32_t clean, rec_list *cex, int64_t *n_ties, int64_t *n_points,
                           uint8_t *xp, void *sa, void *sb) {
    int n = nr->dims[0], m = 2 * rd;
    int32_t pix[64], dig[64];
    pix[0] = first;
    for (int j = 1; j < k; ++j) pix[j] = first + j;
    int64_t rank = base_rank;
    do {
        for (int j = 0; j < k; ++j) dig[j] = 0;
        do {
            int64_t sq = 0;
            int inside = 1;
            memcpy(xp, x, (size_t)n);
            for (int j = 0; j < k; ++j) {
                int e = ball_offset(dig[j], rd);
                int v = (int)x[pix[j]] + e;
                if (v < 0 || v > 255) inside = 0;
                sq += (int64_t)e * e;
                xp[pix[j]] = (uint8_t)(v < 0 ? 0 : v > 255 ? 255 : v);
            }
            if (inside && sq <= r2) {
                int32_t lab; int tie, viol; double margin;
                int rc = eval_image(nr, xp, sa, sb, clean, &lab, &viol, &tie, &margin);
                if (rc) return rc;
                (*n_points)++;
                if (viol) {
                    rc = rec_push(cex, k, rank, lab, margin);
                    if (rc) return rc;
                }
                if (tie) (*n_ties)++;
            }
            rank++;
        } while (next_digits(dig, k, m));
    } while (k > 1 && next_subset_tail(pix, k, n));
    return ORC_OK;
}

/* Shared driver of the integer and the float check. */
static int check_impl(const net_ref *nr, const uint8_t *x, const int16_t *D, int m, int64_t ball_r2,
                      int k_min, int k_max, int k_step, int stop_at_first, int64_t cap,
                      int64_t *points, int64_t *cex_count, int64_t *tie_count,
                      int32_t *clean_label, int32_t *first_unsafe_k,
                      int32_t *out_k, int64_t *out_rank, int32_t *out_label,
                      int64_t *n_out, int64_t tie_cap, int32_t *tie_k, int64_t *tie_rank,
                      double *tie_margin, int64_t *n_tie_out, int nthreads) {
    int n = nr->dims[0];
    /* ball_r2 >= 0: the L2-ball domain (D unused, m = 2 rd); else the box D^k */
    const int ball = ball_r2 >= 0;
    const int rd = ball ? orc_ball_digits(ball_r2) : 0;
    if (ball) m = 2 * rd;
    if ((!ball && m < 1) || k_min < 0 || k_max < k_min || k_step < 1 || k_max > n || k_max > 64)
        return ORC_E_INVALID;
    int mw = max_width(nr->L, nr->dims);
    size_t elt = nr->is_float ? sizeof(double) : sizeof(int64_t);
    void *sa = malloc(elt * mw), *sb = malloc(elt * mw);
    if (!sa || !sb) { free(sa); free(sb); return ORC_E_OOM; }
    int32_t clean; int tie0, viol0; double mg0;
    int rc = eval_image(nr, x, sa, sb, -1, &clean, &viol0, &tie0, &mg0);
    if (!rc && nr->literal) rc = eval_image(nr, x, sa, sb, clean, &clean, &viol0, &tie0, &mg0);
    free(sa); free(sb);
    if (rc) return rc;
    *clean_label = clean;
    *first_unsafe_k = -1;
    int64_t written = 0, tie_written = 0;
    if (n_tie_out) *n_tie_out = 0;
    int level = 0;
    for (int k = k_min; k <= k_max; k += k_step, ++level) {
        points[level] = ball ? (k == 0) : orc_points(n, m, k);
        cex_count[level] = 0;
        tie_count[level] = 0;
        if (k == 0) {
            /* the empty perturbation is the clean image itself (no tie count
             * under the literal) */
            tie_count[level] = nr->literal ? 0 : tie0;
            continue;
        }
        if (ball && rd == 0) continue;   /* no nonzero offset fits: the level is empty */
        int64_t md = ipow(m, k);
        rec_list *lists = calloc((size_t)n, sizeof(rec_list));
        rec_list *tlists = calloc((size_t)n, sizeof(rec_list));
        int64_t *nties = calloc((size_t)n, sizeof(int64_t));
        int64_t *npts = calloc((size_t)n, sizeof(int64_t));
        int err = 0;
        if (!lists || !tlists || !nties || !npts) {
            free(lists); free(tlists); free(nties); free(npts);
            return ORC_E_OOM;
        }
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
        {
            uint8_t *xp = malloc((size_t)n);
            void *ta = malloc(elt * mw), *tb = malloc(elt * mw);
#pragma omp for schedule(dynamic, 1)
            for (int first = 0; first <= n - k; ++first) {
                if (!xp || !ta || !tb) { err = ORC_E_OOM; continue; }
                /* subsets starting below `first` come first in lexicographic order */
                int64_t before = 0;
                for (int q = 0; q < first; ++q) before += binom(n - 1 - q, k - 1);
                int r = ball ? enum_first_ball(nr, x, ball_r2, rd, k, first, before * md, clean, &lists[first],
                                               &nties[first], &npts[first], xp, ta, tb)
                             : enum_first(nr, x, D, m, k, first, before * md, clean, &lists[first],
                                          tie_k ? &tlists[first] : NULL, &nties[first], xp, ta, tb);
                if (r) err = r;
            }
            free(xp); free(ta); free(tb);
        }
        for (int first = 0; first < n && !err; ++first) {
            rec_list *r = &lists[first];
            for (int64_t i = 0; i < r->n; ++i) {
                if (written < cap) {
                    out_k[written] = r->k[i]; out_rank[written] = r->rank[i]; out_label[written] = r->label[i];
                }
                written++;
            }
            cex_count[level] += r->n;
            tie_count[level] += nties[first];
            if (ball) points[level] += npts[first];
            rec_list *t = &tlists[first];
            for (int64_t i = 0; i < t->n; ++i) {
                if (tie_written < tie_cap) {
                    tie_k[tie_written] = t->k[i]; tie_rank[tie_written] = t->rank[i];
                    if (tie_margin) tie_margin[tie_written] = t->margin[i];
                }
                tie_written++;
            }
        }
        for (int first = 0; first < n; ++first) { rec_free(&lists[first]); rec_free(&tlists[first]); }
        free(lists); free(tlists); free(nties); free(npts);
        if (err) return err;
        if (cex_count[level] > 0 && *first_unsafe_k < 0) *first_unsafe_k = k;
        if (stop_at_first && cex_count[level] > 0) { ++level; break; }
    }
    *n_out = written;
    if (n_tie_out) *n_tie_out = tie_written;
    return level;  /* number of levels evaluated (>= 0) */
}

/* Integer check.  Arrays indexed by level have room for the number of levels
 * k_min, k_min+k_step, ... <= k_max.  Counterexamples (k, rank, new label)
 * come out sorted by (k, rank); at most `cap` are written, n_out receives the
 * exact total.  Exact top-2 logit ties are counted per level.
 * Returns the number of levels evaluated, or a negative error. */
int orc_q8_check(int L, const int32_t *dims, const int8_t *W, const int32_t *b,
                 const int32_t *shift, const uint8_t *x, const int16_t *D, int m,
                 int k_min, int k_max, int k_step, int stop_at_first, int64_t cap,
                 int64_t *points, int64_t *cex_count, int64_t *tie_count,
                 int32_t *clean_label, int32_t *first_unsafe_k,
                 int32_t *out_k, int64_t *out_rank, int32_t *out_label, int64_t *n_out,
                 int nthreads) {
    if (L < 1 || !dims || !W || !b || !x || !D) return ORC_E_INVALID;
    net_ref nr = {0, L, dims, W, b, shift, NULL, NULL, 0.0, 0, 0, 0.0};
    return check_impl(&nr, x, D, m, -1, k_min, k_max, k_step, stop_at_first, cap, points, cex_count,
                      tie_count, clean_label, first_unsafe_k, out_k, out_rank, out_label, n_out,
                      0, NULL, NULL, NULL, NULL, nthreads);
}

/* Integer check over the L2-ball domain (see orc_ball_digits): the levels,
 * counts, ranks and records as in orc_q8_check, points[] the number of
 * images of each support size inside the ball. */
int orc_q8_ball_check(int L, const int32_t *dims, const int8_t *W, const int32_t *b,
                      const int32_t *shift, const uint8_t *x, int64_t r2,
                      int k_min, int k_max, int k_step, int stop_at_first, int64_t cap,
                      int64_t *points, int64_t *cex_count, int64_t *tie_count,
                      int32_t *clean_label, int32_t *first_unsafe_k,
                      int32_t *out_k, int64_t *out_rank, int32_t *out_label, int64_t *n_out,
                      int nthreads) {
    if (L < 1 || !dims || !W || !b || !x || r2 < 0) return ORC_E_INVALID;
    net_ref nr = {0, L, dims, W, b, shift, NULL, NULL, 0.0, 0, 0, 0.0};
    return check_impl(&nr, x, NULL, 0, r2, k_min, k_max, k_step, stop_at_first, cap, points, cex_count,
                      tie_count, clean_label, first_unsafe_k, out_k, out_rank, out_label, n_out,
                      0, NULL, NULL, NULL, NULL, nthreads);
}

/* Float (double-evaluated) check with near-tie flags: a point is flagged when
 * the gap between its two largest logits is <= tie_rel * max(1, |largest|). */
int orc_f64_check(int L, const int32_t *dims, const double *W, const double *b,
                  const uint8_t *x, const int16_t *D, int m,
                  int k_min, int k_max, int k_step, int stop_at_first, int64_t cap,
                  double tie_rel, int64_t *points, int64_t *cex_count, int64_t *tie_count,
                  int32_t *clean_label, int32_t *first_unsafe_k,
                  int32_t *out_k, int64_t *out_rank, int32_t *out_label, int64_t *n_out,
                  int64_t tie_cap, int32_t *tie_k, int64_t *tie_rank, double *tie_margin,
                  int64_t *n_tie_out, int nthreads) {
    if (L < 1 || !dims || !W || !b || !x || !D) return ORC_E_INVALID;
    net_ref nr = {1, L, dims, NULL, NULL, NULL, W, b, tie_rel, 0, 0, 0.0};
    return check_impl(&nr, x, D, m, -1, k_min, k_max, k_step, stop_at_first, cap, points, cex_count,
                      tie_count, clean_label, first_unsafe_k, out_k, out_rank, out_label, n_out,
                      tie_cap, tie_k, tie_rank, tie_margin, n_tie_out, nthreads);
}

/* The float check with the table sigmoid (lut != 0) and / or the threshold
 * literal (literal != 0, reference value V): with the literal a point is a
 * counterexample when (z_D < V) and (max_{i != D} z_i > V), D the clean
 * label, and it is flagged when z_D or the largest other logit lies within
 * tie_rel * max(1, |V|) of V.  Otherwise as orc_f64_check. */
int orc_f64_check_ex(int L, const int32_t *dims, const double *W, const double *b,
                     const uint8_t *x, const int16_t *D, int m,
                     int k_min, int k_max, int k_step, int stop_at_first, int64_t cap,
                     double tie_rel, int lut, int literal, double V,
                     int64_t *points, int64_t *cex_count, int64_t *tie_count,
                     int32_t *clean_label, int32_t *first_unsafe_k,
                     int32_t *out_k, int64_t *out_rank, int32_t *out_label, int64_t *n_out,
                     int64_t tie_cap, int32_t *tie_k, int64_t *tie_rank, double *tie_margin,
                     int64_t *n_tie_out, int nthreads) {
    if (L < 1 || !dims || !W || !b || !x || !D) return ORC_E_INVALID;
    net_ref nr = {1, L, dims, NULL, NULL, NULL, W, b, tie_rel, lut != 0, literal != 0, V};
    return check_impl(&nr, x, D, m, -1, k_min, k_max, k_step, stop_at_first, cap, points, cex_count,
                      tie_count, clean_label, first_unsafe_k, out_k, out_rank, out_label, n_out,
                      tie_cap, tie_k, tie_rank, tie_margin, n_tie_out, nthreads);
}

/* The integer check with the threshold literal, reference value V (an
 * integer logit value): a point is a counterexample when (z_D < V) and
 * (max_{i != D} z_i > V); ties count the points where one of the two equals
 * V.  Otherwise as orc_q8_check. */
int orc_q8_check_literal(int L, const int32_t *dims, const int8_t *W, const int32_t *b,
                         const int32_t *shift, const uint8_t *x, const int16_t *D, int m, int64_t V,
                         int k_min, int k_max, int k_step, int stop_at_first, int64_t cap,
                         int64_t *points, int64_t *cex_count, int64_t *tie_count,
                         int32_t *clean_label, int32_t *first_unsafe_k,
                         int32_t *out_k, int64_t *out_rank, int32_t *out_label, int64_t *n_out,
                         int nthreads) {
    if (L < 1 || !dims || !W || !b || !x || !D) return ORC_E_INVALID;
    net_ref nr = {0, L, dims, W, b, shift, NULL, NULL, 0.0, 0, 1, (double)V};
    return check_impl(&nr, x, D, m, -1, k_min, k_max, k_step, stop_at_first, cap, points, cex_count,
                      tie_count, clean_label, first_unsafe_k, out_k, out_rank, out_label, n_out,
                      0, NULL, NULL, NULL, NULL, nthreads);
}

/* Training loss of the float network (the networks are trained on labelled
 * examples by backpropagation, Sec. II-A): the mean over the n images of the
 * cross-entropy of the softmax of the logits against each image's label,
 * and its gradient with respect to theta = for each layer l in turn, W_l
 * row-major [dims[l]][dims[l-1]] then b_l [dims[l]].  Sigmoid hidden
 * layers, linear logits, a0 = x / 256, all in double.  Plain chain rule:
 * dL/du_L = (softmax - onehot) / n; dL/dW_l = dL/du_l a_{l-1}^T;
 * dL/db_l = dL/du_l; dL/du_{l-1} = (W_l^T dL/du_l) * a (1 - a). */
int orc_f64_loss_grad(int L, const int32_t *dims, const double *W, const double *b, const uint8_t *images,
                      const int32_t *labels, int64_t n_img, double *grad, double *loss) {
    if (L < 1 || L > ORC_TRAIN_MAX_LAYERS || !dims || !W || !b || !images || !labels || !grad || !loss || n_img < 1)
        return ORC_E_INVALID;
    /* per layer: offsets of its activations, its W and b, its theta block */
    int64_t a_off[ORC_TRAIN_MAX_LAYERS + 1], w_off[ORC_TRAIN_MAX_LAYERS + 1], b_off[ORC_TRAIN_MAX_LAYERS + 1];
    int64_t t_off[ORC_TRAIN_MAX_LAYERS + 1];
    int64_t U = dims[0], P = 0, nw = 0, nb = 0;
    a_off[0] = 0;
    for (int l = 1; l <= L; ++l) {
        a_off[l] = U; w_off[l] = nw; b_off[l] = nb; t_off[l] = P;
        U += dims[l]; nw += (int64_t)dims[l] * dims[l - 1]; nb += dims[l];
        P += (int64_t)dims[l] * dims[l - 1] + dims[l];
    }
    const int n = dims[0], nc = dims[L];
    double *act = malloc(sizeof(double) * U);   /* a0 | a1 | ... | aL (aL = logits) */
    double *del = malloc(sizeof(double) * U);   /* dL/du per unit, same layout */
    if (!act || !del) { free(act); free(del); return ORC_E_OOM; }
    for (int64_t t = 0; t < P; ++t) grad[t] = 0.0;
    double total = 0.0;
    int rc = ORC_OK;
    for (int64_t s = 0; s < n_img && rc == ORC_OK; ++s) {
        const int y = labels[s];
        if (y < 0 || y >= nc) { rc = ORC_E_INVALID; break; }
        for (int i = 0; i < n; ++i) act[i] = images[s * n + i] / 256.0;
        for (int l = 1; l <= L; ++l) {
            const int nin = dims[l - 1], nout = dims[l];
            for (int j = 0; j < nout; ++j) {
                double u = b[b_off[l] + j];
                for (int i = 0; i < nin; ++i) u += W[w_off[l] + (int64_t)j * nin + i] * act[a_off[l - 1] + i];
                act[a_off[l] + j] = (l < L) ? 1.0 / (1.0 + exp(-u)) : u;
            }
        }
        const double *z = act + a_off[L];
        double zmax = z[0];
        for (int c = 1; c < nc; ++c) if (z[c] > zmax) zmax = z[c];
        double sum = 0.0;
        for (int c = 0; c < nc; ++c) sum += exp(z[c] - zmax);
        total += log(sum) - (z[y] - zmax);
        for (int c = 0; c < nc; ++c) del[a_off[L] + c] = (exp(z[c] - zmax) / sum - (c == y ? 1.0 : 0.0)) / n_img;
        for (int l = L; l >= 1; --l) {
            const int nin = dims[l - 1], nout = dims[l];
            for (int j = 0; j < nout; ++j) {
                const double dj = del[a_off[l] + j];
                for (int i = 0; i < nin; ++i) grad[t_off[l] + (int64_t)j * nin + i] += dj * act[a_off[l - 1] + i];
                grad[t_off[l] + (int64_t)nout * nin + j] += dj;
            }
            if (l == 1) break;
            for (int i = 0; i < nin; ++i) {
                double da = 0.0;
                for (int j = 0; j < nout; ++j) da += W[w_off[l] + (int64_t)j * nin + i] * del[a_off[l] + j];
                const double a = act[a_off[l - 1] + i];
                del[a_off[l - 1] + i] = da * a * (1.0 - a);
            }
        }
    }
    if (rc == ORC_OK) *loss = total / n_img;
    free(act); free(del);
    return rc;
}

/* Replay / sample: decode each (k, rank), build the perturbed image and run
 * the integer forward.  logits (nullable) receives dims[L] values per point. */
int orc_q8_eval_points(int L, const int32_t *dims, const int8_t *W, const int32_t *b,
                       const int32_t *shift, const uint8_t *x, const int16_t *D, int m,
                       const int32_t *ks, const int64_t *ranks, int64_t npts,
                       int32_t *labels, int64_t *logits, int nthreads) {
    if (L < 1 || !dims || !W || !b || !x || !D || npts < 0) return ORC_E_INVALID;
    int n = dims[0], mw = max_width(L, dims);
    int64_t U = total_units(L, dims);
    int err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        uint8_t *xp = malloc((size_t)n);
        int64_t *sa = malloc(sizeof(int64_t) * mw), *sb = malloc(sizeof(int64_t) * mw);
        int64_t *pot = malloc(sizeof(int64_t) * U);
        int32_t pix[64], dig[64];
#pragma omp for schedule(static)
        for (int64_t t = 0; t < npts; ++t) {
            if (!xp || !sa || !sb || !pot) { err = ORC_E_OOM; continue; }
            if (ks[t] > 64 || orc_decode(n, m, ks[t], ranks[t], pix, dig)) { err = ORC_E_INVALID; continue; }
            apply_point(x, n, D, ks[t], pix, dig, xp);
            int r = q8_forward(L, dims, W, b, shift, xp, sa, sb, pot, &labels[t], NULL);
            if (r) { err = r; continue; }
            if (logits) memcpy(&logits[t * dims[L]], &pot[U - dims[L]], sizeof(int64_t) * dims[L]);
        }
        free(xp); free(sa); free(sb); free(pot);
    }
    return err;
}

int orc_f64_eval_points(int L, const int32_t *dims, const double *W, const double *b,
                        const uint8_t *x, const int16_t *D, int m,
                        const int32_t *ks, const int64_t *ranks, int64_t npts,
                        int32_t *labels, double *logits, double *margins, int nthreads) {
    if (L < 1 || !dims || !W || !b || !x || !D || npts < 0) return ORC_E_INVALID;
    int n = dims[0], mw = max_width(L, dims);
    int64_t U = total_units(L, dims);
    int err = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
    {
        uint8_t *xp = malloc((size_t)n);
        double *sa = malloc(sizeof(double) * mw), *sb = malloc(sizeof(double) * mw);
        double *pot = malloc(sizeof(double) * U);
        int32_t pix[64], dig[64];
#pragma omp for schedule(static)
        for (int64_t t = 0; t < npts; ++t) {
            if (!xp || !sa || !sb || !pot) { err = ORC_E_OOM; continue; }
            if (ks[t] > 64 || orc_decode(n, m, ks[t], ranks[t], pix, dig)) { err = ORC_E_INVALID; continue; }
            apply_point(x, n, D, ks[t], pix, dig, xp);
            double mg;
            f64_forward(L, dims, W, b, xp, sa, sb, pot, &labels[t], &mg, NULL);
            if (margins) margins[t] = mg;
            if (logits) memcpy(&logits[t * dims[L]], &pot[U - dims[L]], sizeof(double) * dims[L]);
        }
        free(xp); free(sa); free(sb); free(pot);
    }
    return err;
}

/* ------------------------------------------------------------------------ */
/* coverage (Sec. III-B)                                                     */
/* ------------------------------------------------------------------------ */

enum { ORC_SS = 0, ORC_DS = 1, ORC_SV = 2, ORC_DV = 3 };

static int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

/* Literal evaluation of one criterion over every adjacent-layer neuron pair
 * and every input pair.  widths[0..nl) are the widths of the non-input
 * layers; pot1/pot2 hold, per input pair, all their potentials
 * concatenated.  bits: pair (l, i, j) is bit off_l + i * widths[l+1] + j,
 * off_l = sum over earlier blocks of widths[q] * widths[q+1]; bit t lives in
 * word t / 64 at position t % 64.  counts = {covered pairs, total pairs,
 * covered neurons, total neurons}. */
int orc_coverage(int nl, const int32_t *widths, const int64_t *pot1, const int64_t *pot2,
                 int64_t n_pairs, int criterion, int64_t dist_sq_min, int32_t rnum, int32_t rden,
                 double P, uint64_t *bits, int64_t *counts, double *fraction, int32_t *literal) {
    if (nl < 1 || !widths || n_pairs < 0 || criterion < 0 || criterion > 3 || rnum < 1 || rden < 1)
        return ORC_E_INVALID;
    int64_t U = 0, total_pairs = 0;
    int64_t off[64], uoff[64];
    if (nl > 63) return ORC_E_INVALID;
    for (int l = 0; l < nl; ++l) {
        uoff[l] = U;
        U += widths[l];
        off[l] = total_pairs;
        if (l + 1 < nl) total_pairs += (int64_t)widths[l] * widths[l + 1];
    }
    int64_t nwords = (total_pairs + 63) / 64;
    memset(bits, 0, sizeof(uint64_t) * (size_t)(nwords ? nwords : 1));
    int mw = 0;
    for (int l = 0; l < nl; ++l) if (widths[l] > mw) mw = widths[l];
    unsigned char *sc = malloc((size_t)U), *vc = malloc((size_t)U);
    if (!sc || !vc) { free(sc); free(vc); return ORC_E_OOM; }
    for (int64_t t = 0; t < n_pairs; ++t) {
        const int64_t *a = pot1 + t * U, *c = pot2 + t * U;
        int nsc[64], dc[64];
        for (int l = 0; l < nl; ++l) {
            nsc[l] = 0;
            __int128 dist = 0;
            for (int i = 0; i < widths[l]; ++i) {
                int64_t x1 = a[uoff[l] + i], x2 = c[uoff[l] + i];
                int s1 = x1 >= 0, s2 = x2 >= 0;          /* sign(0) = 1 */
                sc[uoff[l] + i] = s1 != s2;
                nsc[l] += s1 != s2;
                int64_t hi = iabs64(x1) > iabs64(x2) ? iabs64(x1) : iabs64(x2);
                int64_t lo = iabs64(x1) > iabs64(x2) ? iabs64(x2) : iabs64(x1);
                vc[uoff[l] + i] = (s1 == s2) && hi > 0 && (int64_t)rden * hi >= (int64_t)rnum * lo;
                __int128 d = (__int128)x1 - x2;
                dist += d * d;
            }
            dc[l] = nsc[l] == 0 && dist >= (__int128)dist_sq_min;
        }
        for (int l = 0; l + 1 < nl; ++l) {
            for (int i = 0; i < widths[l]; ++i) {
                for (int j = 0; j < widths[l + 1]; ++j) {
                    int cond_sign = sc[uoff[l] + i] && nsc[l] == 1;
                    int hit;
                    switch (criterion) {
                        case ORC_SS: hit = cond_sign && sc[uoff[l + 1] + j]; break;
                        case ORC_DS: hit = dc[l] && sc[uoff[l + 1] + j]; break;
                        case ORC_SV: hit = cond_sign && vc[uoff[l + 1] + j]; break;
                        default:     hit = dc[l] && vc[uoff[l + 1] + j]; break;
                    }
                    if (hit) {
                        int64_t bit = off[l] + (int64_t)i * widths[l + 1] + j;
                        bits[bit / 64] |= (uint64_t)1 << (bit % 64);
                    }
                }
            }
        }
    }
    /* summary: a neuron is covered when it belongs to at least one covered pair */
    unsigned char *ncov = calloc((size_t)U, 1);
    if (!ncov) { free(sc); free(vc); return ORC_E_OOM; }
    int64_t covered_pairs = 0;
    for (int l = 0; l + 1 < nl; ++l)
        for (int i = 0; i < widths[l]; ++i)
            for (int j = 0; j < widths[l + 1]; ++j) {
                int64_t bit = off[l] + (int64_t)i * widths[l + 1] + j;
                if ((bits[bit / 64] >> (bit % 64)) & 1) {
                    covered_pairs++;
                    ncov[uoff[l] + i] = 1;
                    ncov[uoff[l + 1] + j] = 1;
                }
            }
    int64_t covered_neurons = 0;
    for (int64_t u = 0; u < U; ++u) covered_neurons += ncov[u];
    counts[0] = covered_pairs; counts[1] = total_pairs;
    counts[2] = covered_neurons; counts[3] = U;
    *fraction = U ? (double)covered_neurons / (double)U : 0.0;
    *literal = *fraction >= P;
    free(sc); free(vc); free(ncov);
    return ORC_OK;
}

/* Euclidean distance of two vectors (Eq. (7)). */
double orc_euclid(const double *p, const double *q, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (p[i] - q[i]) * (p[i] - q[i]);
    return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* proposal network: s = w2 . relu(W1 f + b1) + c, weighted logistic loss     */
/* ------------------------------------------------------------------------ */

static double softplus(double z) { return z > 0 ? z + log1p(exp(-z)) : log1p(exp(z)); }

/* Mean weighted binary cross-entropy over the batch and its gradients.
 * loss_b = -[pw * y log sigmoid(s) + (1 - y) log(1 - sigmoid(s))]
 *        =  pw * y * softplus(-s) + (1 - y) * softplus(s).
 * Shapes: f [B][F], W1 [H][F], b1 [H], w2 [H], c scalar.  Gradients
 * (nullable) have the parameter shapes; scores (nullable) gets s. */
int orc_prop_loss_grad(int B, int F, int H, const double *f, const double *y, double pw,
                       const double *W1, const double *b1, const double *w2, double c,
                       double *loss, double *gW1, double *gb1, double *gw2, double *gc,
                       double *scores) {
    if (B < 0 || F < 1 || H < 1) return ORC_E_INVALID;
    double *h = malloc(sizeof(double) * H), *hp = malloc(sizeof(double) * H);
    if (!h || !hp) { free(h); free(hp); return ORC_E_OOM; }
    if (gW1) memset(gW1, 0, sizeof(double) * H * F);
    if (gb1) memset(gb1, 0, sizeof(double) * H);
    if (gw2) memset(gw2, 0, sizeof(double) * H);
    double tot = 0.0, tc = 0.0;
    for (int t = 0; t < B; ++t) {
        const double *ft = f + (int64_t)t * F;
        double s = c;
        for (int j = 0; j < H; ++j) {
            double u = b1[j];
            for (int i = 0; i < F; ++i) u += W1[(int64_t)j * F + i] * ft[i];
            hp[j] = u;
            h[j] = u > 0 ? u : 0.0;
            s += w2[j] * h[j];
        }
        if (scores) scores[t] = s;
        tot += pw * y[t] * softplus(-s) + (1.0 - y[t]) * softplus(s);
        /* chain rule: d loss_b / d s = sigmoid(s) (pw y + 1 - y) - pw y */
        double sig = 1.0 / (1.0 + exp(-s));
        double g = (sig * (pw * y[t] + 1.0 - y[t]) - pw * y[t]) / (double)B;
        tc += g;
        for (int j = 0; j < H; ++j) {
            if (gw2) gw2[j] += g * h[j];
            double gh = hp[j] > 0 ? g * w2[j] : 0.0;
            if (gb1) gb1[j] += gh;
            if (gW1) for (int i = 0; i < F; ++i) gW1[(int64_t)j * F + i] += gh * ft[i];
        }
    }
    if (loss) *loss = B ? tot / B : 0.0;
    if (gc) *gc = tc;
    free(h); free(hp);
    return ORC_OK;
}

/* One Adam step (Kingma & Ba) on n parameters; t is the 1-based step count. */
void orc_adam_step(int64_t n, double *theta, const double *g, double *mom, double *vel, int t,
                   double lr, double beta1, double beta2, double eps) {
    double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int64_t i = 0; i < n; ++i) {
        mom[i] = beta1 * mom[i] + (1.0 - beta1) * g[i];
        vel[i] = beta2 * vel[i] + (1.0 - beta2) * g[i] * g[i];
        theta[i] -= lr * (mom[i] / c1) / (sqrt(vel[i] / c2) + eps);
    }
}

/* Features of every candidate (pixel p, delta index i) of an image for the
 * proposal network, in double: row/(rows-1), col/(cols-1), x/255, d/dmax,
 * e/dmax with e = clamp(x+d) - x, the L1 and L2 norms of the first-layer
 * weight column of p and its L1 norm over the first-layer units whose clean
 * potential lies in the requantiser's unsaturated window [0, 128 * 2^s),
 * each divided by its maximum over pixels (at least 1), then 1, then zeros
 * up to 32 entries. */
int orc_prop_features(int L, const int32_t *dims, const int8_t *W, const int32_t *b, const int32_t *shift,
                      const uint8_t *x, int rows, int cols, const int16_t *D, int m, double *feat) {
    if (L < 2 || !dims || !W || !b || !shift || !x || !D || m < 1 || rows * cols != dims[0]) return ORC_E_INVALID;
    int n = dims[0], h1 = dims[1];
    unsigned char *live = malloc((size_t)h1);
    double *n1 = malloc(sizeof(double) * n), *n2 = malloc(sizeof(double) * n), *nl = malloc(sizeof(double) * n);
    if (!live || !n1 || !n2 || !nl) { free(live); free(n1); free(n2); free(nl); return ORC_E_OOM; }
    int64_t top = (int64_t)128 << shift[0];
    for (int j = 0; j < h1; ++j) {
        int64_t u = b[j];
        for (int i = 0; i < n; ++i) u += (int64_t)W[(int64_t)j * n + i] * x[i];
        live[j] = u >= 0 && u < top;
    }
    double m1 = 1.0, m2 = 1.0;
    for (int p = 0; p < n; ++p) {
        double s1 = 0, s2 = 0, sl = 0;
        for (int j = 0; j < h1; ++j) {
            double w = W[(int64_t)j * n + p];
            s1 += fabs(w);
            s2 += w * w;
            if (live[j]) sl += fabs(w);
        }
        n1[p] = s1; n2[p] = sqrt(s2); nl[p] = sl;
        if (s1 > m1) m1 = s1;
        if (n2[p] > m2) m2 = n2[p];
    }
    double dmax = 1.0;
    for (int i = 0; i < m; ++i) if (fabs((double)D[i]) > dmax) dmax = fabs((double)D[i]);
    for (int p = 0; p < n; ++p) {
        int r = p / cols, c = p % cols;
        for (int i = 0; i < m; ++i) {
            double *f = feat + ((int64_t)p * m + i) * 32;
            int v = (int)x[p] + D[i];
            if (v < 0) v = 0;
            if (v > 255) v = 255;
            f[0] = rows > 1 ? (double)r / (rows - 1) : (double)r;
            f[1] = cols > 1 ? (double)c / (cols - 1) : (double)c;
            f[2] = x[p] / 255.0;
            f[3] = D[i] / dmax;
            f[4] = (v - (int)x[p]) / dmax;
            f[5] = n1[p] / m1;
            f[6] = n2[p] / m2;
            f[7] = nl[p] / m1;   /* live part of the column norm, on the full norm's scale */
            f[8] = 1.0;
            for (int z = 9; z < 32; ++z) f[z] = 0.0;
        }
    }
    free(live); free(n1); free(n2); free(nl);
    return ORC_OK;
}
