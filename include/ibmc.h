/*
 * ibmc.h -- C ABI of the MI355X (gfx950) library for exhaustive, incrementally
 * bounded checking of quantized multi-layer perceptrons and for their
 * neuron-pair coverage criteria.
 *
 * The method follows Sena et al., "Incremental Bounded Model Checking of
 * Artificial Neural Networks in CUDA" (arXiv 1907.12933):
 *   - network: neuron potential u = sum_j w_j i_j + b (Sec. II-A, Eq. (1));
 *     the sigmoid variant applies N(u) = 1 / (1 + e^-u) (Sec. II-A, Eq. (2));
 *   - safety property: every image of the restricted set keeps the clean
 *     image's classification; a violation is a counterexample
 *     (Sec. III-C, Eqs. (9)-(10));
 *   - incremental bound: the check is repeated for k = k_min, k_min+k_step,
 *     ... (Sec. II-B, including the increment granularity);
 *   - coverage: SS / DS / SV / DV neuron-pair covers and the covered-neuron
 *     literal (Sec. III-B, Eqs. (3)-(6)).
 *
 * The paper restricts images to a Euclidean ball around the clean image and
 * solves for a violating one symbolically.  Here the restricted set at bound k
 * is finite and enumerated: every image that differs from the clean image x in
 * exactly k pixels p1 < ... < pk, pixel pj becoming clamp(x[pj] + D[ij], 0, 255)
 * for a delta index ij into the caller's delta set D.  It holds
 * C(n, k) * |D|^k points, counted as enumerated (a zero delta or a clamp may
 * make two points the same image).  A point is named by (k, rank) with
 *   rank = (number of k-subsets of [0, n) lexicographically before
 *           {p1 < ... < pk}) * |D|^k + sum_j ij * |D|^(k-j),
 * i.e. subsets in lexicographic order, then the delta indices as a base-|D|
 * number with i1 most significant.
 *
 * Integer networks (IBMC_ACT_RELU_Q8): int8 weights, int32 biases, input
 * activation = pixel value 0..255; hidden activation
 * a = min(max(floor(u / 2^s), 0), 127) with a per-layer shift s (ReLU folded
 * into the clamp); the logits are the last layer's potentials; the label is
 * the lowest index attaining the largest logit.  Every accumulator must fit
 * int32: ibmc_load_mlp rejects (IBMC_E_RANGE) a network with a neuron whose
 * sum_i |W[j][i]| * M + |b[j]| + H reaches 2^31, with M = 256 for the first
 * layer and 128 for later ones and H = 64 * 2^s for a hidden layer of shift
 * s (the kernels accumulate offset forms of the potentials).  The integer
 * path is exact.
 *
 * Float networks (IBMC_ACT_SIGMOID_F32): float32 weights and biases, input
 * activation x / 256, sigmoid on hidden layers, linear logits, lowest-index
 * argmax.  Evaluated in float32; points whose two largest logits are within
 * near_tie_rel * max(1, |largest|) are reported as near ties.
 *
 * Conventions
 *   - Every call returns an ibmc_status: 0 = IBMC_OK, > 0 a warning, < 0 an
 *     error.  After an error, ibmc_last_error() returns a message for the
 *     calling thread.  No C++ exception crosses this boundary.
 *   - Host pointers are caller-owned and only read or written during the
 *     call.  Calls ending in _dev take device pointers (allocated by the
 *     caller on the context's device) for the bulk inputs; summaries and
 *     counterexample records are always written to host memory.
 *   - The library owns the objects behind ibmc_ctx, ibmc_mlp and
 *     ibmc_proposer.  ibmc_load_mlp copies the weights.
 *   - A context wraps one device and one HIP stream (the caller's or its
 *     own).  A context is not thread-safe; use one per thread.  Calls are
 *     synchronous with respect to the host: when a call returns, its results
 *     are in host memory.
 *   - Counterexamples and near ties come back sorted by (property, k, rank),
 *     whatever order the device found them in.
 */
#ifndef IBMC_H
#define IBMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ibmc_status;

#define IBMC_OK 0
#define IBMC_W_TRUNCATED 1      /* more records than capacity; totals stay exact */
#define IBMC_W_PARTIAL 2        /* stopped at chunk_budget: resume from next_cursor */
#define IBMC_E_INVALID (-1)     /* bad argument, size or null pointer */
#define IBMC_E_RANGE (-2)       /* a potential could leave int32 */
#define IBMC_E_HIP (-3)         /* a HIP runtime call failed */
#define IBMC_E_OOM (-4)         /* device or host allocation failed */
#define IBMC_E_ABORTED (-5)     /* stopped by ibmc_abort before completion */
#define IBMC_E_UNIMPL (-6)      /* shape outside what the kernels support */

#define IBMC_MAX_LEVELS 16
#define IBMC_MAX_LAYERS 4       /* weight layers (input layer not counted) */
#define IBMC_MAX_WIDTH 1024     /* widest layer the kernels accept */

typedef struct ibmc_ctx ibmc_ctx;
typedef struct ibmc_mlp ibmc_mlp;
typedef struct ibmc_proposer ibmc_proposer;

typedef enum { IBMC_ACT_RELU_Q8 = 0, IBMC_ACT_SIGMOID_F32 = 1 } ibmc_act;

/* The four covers of Sec. III-B.  IBMC_COV_VV names the fourth (the paper's
 * distance-value cover); it is not a separate criterion. */
typedef enum { IBMC_COV_SS = 0, IBMC_COV_DS = 1, IBMC_COV_SV = 2, IBMC_COV_DV = 3 } ibmc_criterion;
#define IBMC_COV_VV IBMC_COV_DV

/* Network description.  dims has n_layers + 1 entries: pixels, hidden
 * widths..., classes.  W[l] is row-major [dims[l+1]][dims[l]] (int8 for
 * IBMC_ACT_RELU_Q8, float for IBMC_ACT_SIGMOID_F32); b[l] has dims[l+1]
 * entries (int32 or float).  shift has n_layers - 1 entries (integer nets
 * only; each in 0..24).  2 <= n_layers <= IBMC_MAX_LAYERS; every width is
 * <= IBMC_MAX_WIDTH; the class count is <= 64. */
typedef struct {
    int32_t n_layers;
    const int32_t *dims;
    int32_t act;
    const void *const *W;
    const void *const *b;
    const int32_t *shift;
} ibmc_mlp_desc;

/* Options of a check.  k_min >= 0; k_max <= min(n_pixels, 8); k_step >= 1;
 * at most IBMC_MAX_LEVELS levels.  k = 0 is the clean image itself (one
 * point, never a counterexample).  stop_at_first: stop after the first level
 * that has a counterexample (Sec. II-B stops at the first violation).
 * cex_capacity / near_tie_capacity: room in the caller's record buffers.
 * near_tie_rel: float nets only; <= 0 selects 4e-5.
 * records_on_device: nonzero when cex_buf / near_tie_buf are device memory
 * of the context's device (the records then never cross to the host).
 * resume_cursor / chunk_budget (integer networks, one network per call, no
 * stop_at_first; else IBMC_E_UNIMPL when nonzero): the points of all levels
 * form one sequence of work chunks; a call checks the chunks from
 * resume_cursor on (0: from the start) and, with chunk_budget > 0, at most
 * that many.  A call that stops early (budget reached, or ibmc_abort)
 * reports in next_cursor the first chunk it did not check: every chunk
 * before it is checked, and its counts and records cover exactly the chunks
 * it checked.  Calling again with resume_cursor = next_cursor (same network,
 * image, deltas, k range and library build) continues the check; the union
 * of the calls' records and the sums of their counts equal one uninterrupted
 * call's.
 * property: IBMC_PROPERTY_LABEL (0) — a point violates the property when its
 * label differs from the clean label; IBMC_PROPERTY_LITERAL (1) — the
 * paper's literal l_image_misclassified (Sec. III-C): with D the clean
 * label and V = literal_v, a point violates it when z_D < V and some other
 * logit z_i > V (records still carry the point's label).  Integer networks:
 * V must be an integer in the int32 range, exact ties then count the points
 * where z_D or the largest other logit equals V; float networks: a point is
 * a near tie when one of the two lies within near_tie_rel * max(1, |V|) of
 * V.  Level 0 counts no ties under the literal.
 * sigmoid (float networks): IBMC_SIGMOID_EXP (0) — 1/(1 + e^-u);
 * IBMC_SIGMOID_TABLE (1) — the table sigmoid the paper's CUDA code used
 * (Sec. IV-D): knots -8 + i/16, i = 0..256, holding sigma in FP32, linear
 * between knots, the end values outside [-8, 8].
 * The literal and the table run on the lane-per-point kernels only: integer
 * networks with 1-2 hidden layers of at most 64 units and at most 16
 * classes, float networks with hidden widths up to 128 (else IBMC_E_UNIMPL);
 * neither combines with resume_cursor / chunk_budget or the ordered search
 * (IBMC_E_UNIMPL).  All-zero fields keep the label property and the
 * exponential. */
#define IBMC_PROPERTY_LABEL 0
#define IBMC_PROPERTY_LITERAL 1
#define IBMC_SIGMOID_EXP 0
#define IBMC_SIGMOID_TABLE 1
typedef struct {
    int32_t k_min, k_max, k_step, stop_at_first;
    int64_t cex_capacity;
    int64_t near_tie_capacity;
    float near_tie_rel;
    int32_t records_on_device;
    int64_t resume_cursor;
    int64_t chunk_budget;
    int32_t property;
    int32_t sigmoid;
    double literal_v;
} ibmc_check_opts;

/* One counterexample (or near tie): decode with ibmc_decode_point.  prop is
 * the property index in a batch (0 for single-property calls). */
typedef struct {
    int32_t prop;
    int32_t k;
    int64_t rank;
    int32_t new_label;
    int32_t reserved;
} ibmc_cex;

typedef struct {
    int32_t clean_label;
    int32_t first_unsafe_k;              /* -1: no counterexample at any checked level */
    int32_t n_levels;                    /* levels evaluated */
    int32_t safe_up_to_k;                /* largest checked k with no counterexample at or below it; -1 if none */
    int32_t level_k[IBMC_MAX_LEVELS];
    int64_t points[IBMC_MAX_LEVELS];     /* points enumerated per level */
    int64_t cex[IBMC_MAX_LEVELS];        /* counterexamples per level (exact) */
    int64_t ties[IBMC_MAX_LEVELS];       /* integer: exact top-2 logit ties; float: near ties */
    int64_t points_total;
    int64_t cex_total;
    int64_t near_ties_total;
    double seconds;                      /* device time of the call (HIP events) */
    double ttfc_seconds;                 /* ordered search: time to the first counterexample; -1 if none */
    int64_t points_before_first;         /* ordered search: points visited before the first counterexample; -1 if none */
    int64_t next_cursor;                 /* -1: checked to the end; else the chunk to resume from (see
                                            ibmc_check_opts); points[] still give the levels' sizes */
} ibmc_check_summary;

/* One property of a batch: a network, an image of dims[0] pixels, a delta
 * set (host memory) and its bounds. */
typedef struct {
    const ibmc_mlp *net;
    const uint8_t *image;                /* host (ibmc_check_batch) or device (ibmc_check_batch_dev) */
    const int16_t *deltas;               /* host */
    int32_t n_deltas;
    int32_t k_min, k_max, k_step;
} ibmc_property;

/* Coverage parameters (Sec. III-B): value change iff no sign change and
 * ratio_den * max(|a|,|b|) >= ratio_num * min(|a|,|b|) with max > 0;
 * distance change of a layer iff no sign change in it and
 * sum_i (a_i - b_i)^2 >= dist_sq_min; literal iff covered neurons / neurons
 * >= P.  Zero fields select the defaults 1, 3, 2 and 0.8. */
typedef struct {
    int64_t dist_sq_min;
    int32_t ratio_num, ratio_den;
    double P;
} ibmc_cov_params;

typedef struct {
    int64_t covered_pairs, total_pairs, covered_neurons, total_neurons;
    double fraction;
    int32_t literal;
    int32_t reserved;
    double seconds;
} ibmc_cov_summary;

/* ---- context ----------------------------------------------------------- */

/* Create a context on `device`.  hip_stream: a hipStream_t to run on, or NULL
 * for a stream the library creates (default priority). */
ibmc_status ibmc_ctx_create(int32_t device, void *hip_stream, ibmc_ctx **out);
void ibmc_ctx_destroy(ibmc_ctx *ctx);
/* Message of the last error on this thread ("" if none).  Valid until the
 * next call on this thread. */
const char *ibmc_last_error(void);
/* Number of multiprocessors of the context's device (for launch sizing). */
ibmc_status ibmc_device_info(ibmc_ctx *ctx, int32_t *n_cu, int32_t *arch_major, int32_t *arch_minor);

/* ---- networks ---------------------------------------------------------- */

/* Copy and validate a network; lay it out on the device for the kernels.
 * Errors: IBMC_E_INVALID (shape), IBMC_E_RANGE (int32 headroom),
 * IBMC_E_UNIMPL (wider than the kernels accept). */
ibmc_status ibmc_load_mlp(ibmc_ctx *ctx, const ibmc_mlp_desc *desc, ibmc_mlp **out);
/* Frees the network's device memory; allowed before or after its context
 * is destroyed (it is only used with that context). */
void ibmc_free_mlp(ibmc_mlp *net);

/* ---- the check (Sec. II-B bound loop around the Sec. III-C property) ---- */

/* Check one image.  image: n_pixels bytes (must equal dims[0]).  delta_set:
 * n_deltas int16 values (1..64).  cex_buf: room for opts->cex_capacity
 * records (may be NULL when the capacity is 0); near_tie_buf likewise
 * (float nets).  Returns IBMC_W_TRUNCATED when a buffer was too small; the
 * summary's totals stay exact.  IBMC_E_UNIMPL when dims[0] * n_deltas is
 * 2^24 or more (single-pixel candidates are indexed in 32-bit arithmetic). */
ibmc_status ibmc_check_property(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image,
                                int32_t n_pixels, const int16_t *delta_set, int32_t n_deltas,
                                const ibmc_check_opts *opts, ibmc_check_summary *out,
                                ibmc_cex *cex_buf, ibmc_cex *near_tie_buf);

/* Allocation-free ibmc_check_property, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * ibmc_check_property; the call itself allocates and frees nothing: every
 * device buffer it needs is carved from one fixed scratch array of
 * IBMC_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on
 * until the process ends (its address is looked up once per device, when a
 * context is created there).  A call whose worst-case need (record slots
 * for cex_capacity plus one block per wave, their sort space, near-tie
 * slots, tables) exceeds the array is rejected with IBMC_E_INVALID before
 * any device work.  Every call on a device shares that device's array and
 * clears what it uses, so two calls that overlap in time on one device (two
 * threads, or two contexts on different streams) race and must not be
 * made. */
#define IBMC_NOALLOC_SCRATCH_BYTES (64ll << 20)
ibmc_status ibmc_check_property_noalloc(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image,
                                        int32_t n_pixels, const int16_t *delta_set, int32_t n_deltas,
                                        const ibmc_check_opts *opts, ibmc_check_summary *out,
                                        ibmc_cex *cex_buf, ibmc_cex *near_tie_buf);

/* As ibmc_check_property with `image` a device pointer (n_pixels bytes on
 * the context's device); the delta set stays in host memory. */
ibmc_status ibmc_check_property_dev(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image,
                                    int32_t n_pixels, const int16_t *delta_set, int32_t n_deltas,
                                    const ibmc_check_opts *opts, ibmc_check_summary *out,
                                    ibmc_cex *cex_buf, ibmc_cex *near_tie_buf);

/* The L2-ball domain (Sec. III-C: the restriction R of Eq. (9) with the
 * Euclidean distance of Eq. (7), on pixel values): every image x' in
 * {0..255}^n with sum_p (x'_p - x_p)^2 <= radius_sq, checked level by level,
 * level k holding the images that differ from `image` in exactly k pixels.
 * Nothing is clamped: an offset that takes a pixel out of [0, 255] gives no
 * image.  Records use the point rank of the delta-set domain with the
 * implicit delta set -rd..-1, 1..rd, rd = ibmc_ball_digits(radius_sq) (so
 * ibmc_decode_point with n_deltas = 2 rd decodes them, digit i < rd being
 * offset i - rd and digit i >= rd offset i - rd + 1); summary.points[] count
 * the images of each level that lie in the ball.  opts as for
 * ibmc_check_property except: integer networks whose hidden layers (one or
 * two) have at most 64 units and at most 16 classes (else IBMC_E_UNIMPL);
 * near_tie_capacity must be 0; no resume_cursor / chunk_budget
 * (IBMC_E_UNIMPL); radius_sq in [0, 2^30] (else IBMC_E_INVALID).  A radius
 * below 1 leaves every level k >= 1 empty. */
int32_t ibmc_ball_digits(int64_t radius_sq);   /* min(floor(sqrt(radius_sq)), 255); 0 if negative */
ibmc_status ibmc_check_ball(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image, int32_t n_pixels,
                            int64_t radius_sq, const ibmc_check_opts *opts, ibmc_check_summary *out,
                            ibmc_cex *cex_buf);

/* One L2-ball property of a batch (image in host memory). */
typedef struct {
    const ibmc_mlp *net;
    const uint8_t *image;
    int64_t radius_sq;
    int32_t k_min, k_max, k_step;
    int32_t reserved;
} ibmc_ball_property;

/* ibmc_check_ball over many properties in one launch per network (records
 * tagged with their property index, as in ibmc_check_batch; opts k_min /
 * k_max / k_step are ignored in favour of the properties'). */
ibmc_status ibmc_check_ball_batch(ibmc_ctx *ctx, const ibmc_ball_property *props, int32_t n_props,
                                  const ibmc_check_opts *opts, ibmc_check_summary *outs, ibmc_cex *cex_buf);

/* Check many properties, possibly over different networks, as one
 * batch.  outs: one summary per property.  Records of all properties share
 * cex_buf / near_tie_buf (capacities in opts), tagged with ibmc_cex.prop.
 * With stop_at_first == 0 all levels of all properties run in one
 * persistent launch per network shape, captured and replayed as one HIP
 * graph; with stop_at_first != 0 each level is launched after the previous
 * level's verdicts are known. */
ibmc_status ibmc_check_batch(ibmc_ctx *ctx, const ibmc_property *props, int32_t n_props,
                             const ibmc_check_opts *opts, ibmc_check_summary *outs,
                             ibmc_cex *cex_buf, ibmc_cex *near_tie_buf);
/* As ibmc_check_batch, with every props[i].image a device pointer. */
ibmc_status ibmc_check_batch_dev(ibmc_ctx *ctx, const ibmc_property *props, int32_t n_props,
                                 const ibmc_check_opts *opts, ibmc_check_summary *outs,
                                 ibmc_cex *cex_buf, ibmc_cex *near_tie_buf);

/* Stop a running check from another host thread: the kernels poll a flag in
 * host-mapped memory before taking work and drain; the check returns
 * IBMC_E_ABORTED with the counts and records of the chunks it finished (and,
 * for a resumable call, next_cursor). */
ibmc_status ibmc_abort(ibmc_ctx *ctx);

/* Decode (k, rank) into ascending pixels[k] and delta indices[k] (host only,
 * no device work).  IBMC_E_INVALID if rank is outside [0, C(n,k) |D|^k). */
ibmc_status ibmc_decode_point(int32_t n_pixels, int32_t n_deltas, int32_t k, int64_t rank,
                              int32_t *pixels, int32_t *delta_idx);

/* Replay records on the device: rebuild each perturbed image, run the full
 * forward pass (no incremental update) and write its label.  Confirms a
 * counterexample the way the paper confirms them by re-running the network
 * outside the checker (Sec. IV-C). */
ibmc_status ibmc_replay(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image,
                        const int16_t *delta_set, int32_t n_deltas, const ibmc_cex *recs,
                        int64_t n, int32_t *labels_out);

/* Evaluate listed points (k[t], rank[t]) of one image of a float network
 * with the float enumeration's own FP32 arithmetic (incremental first
 * layer from the clean potentials, blocked sums, hardware-exponential
 * sigmoid), for checking that path against a double-precision reference
 * (Sec. II-A, Eqs. (1)-(2)).  Outputs, each nullable: logits [n][classes],
 * labels [n], top-2 margins [n], and the clean label (the same arithmetic on
 * the unperturbed image).  IBMC_E_INVALID for a k outside [0, min(pixels, 8)]
 * or a rank outside [0, C(n,k) |D|^k); IBMC_E_UNIMPL for integer networks
 * (their enumeration is exact: ibmc_replay confirms it). */
ibmc_status ibmc_eval_points_f32(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image,
                                 const int16_t *delta_set, int32_t n_deltas, const int32_t *ks,
                                 const int64_t *ranks, int64_t n, float *logits, int32_t *labels,
                                 float *margins, int32_t *clean_label);

/* Full forward pass of n_images images (host memory, dims[0] bytes each).
 * potentials (nullable): int32 [n_images][sum of dims[1..L]] for integer
 * nets, float for float nets; labels (nullable): [n_images]. */
ibmc_status ibmc_forward(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *images,
                         int64_t n_images, void *potentials, int32_t *labels);

/* ---- coverage (Sec. III-B) --------------------------------------------- */

/* Coverage of one criterion over n_pairs input pairs (x1[i], x2[i]) of an
 * integer network: potentials of every non-input layer, sign / value /
 * distance change, then the OR over pairs of the covered neuron pairs
 * (l, i, j) between adjacent non-input layers.  covered_bits (nullable):
 * ceil(total_pairs / 64) words; pair (l, i, j) is bit
 * off_l + i * h_{l+1} + j (off_l = sum of earlier h_q * h_{q+1}), bit t in
 * word t / 64 at position t % 64. */
ibmc_status ibmc_coverage(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *x1,
                          const uint8_t *x2, int64_t n_pairs, int32_t criterion,
                          const ibmc_cov_params *params, ibmc_cov_summary *out,
                          uint64_t *covered_bits);
/* As ibmc_coverage with x1 / x2 device pointers. */
ibmc_status ibmc_coverage_dev(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *x1,
                              const uint8_t *x2, int64_t n_pairs, int32_t criterion,
                              const ibmc_cov_params *params, ibmc_cov_summary *out,
                              uint64_t *covered_bits);
/* All four criteria from one forward pass: outs[4] and (nullable)
 * covered_bits[4 * words] in SS, DS, SV, DV order. */
ibmc_status ibmc_coverage_all_dev(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *x1,
                                  const uint8_t *x2, int64_t n_pairs,
                                  const ibmc_cov_params *params, ibmc_cov_summary *outs,
                                  uint64_t *covered_bits);
/* Coverage from given potentials (host int64 [n_pairs][sum widths]) of
 * n_layers layers of the given widths, e.g. the paper's worked tables. */
ibmc_status ibmc_coverage_from_potentials(ibmc_ctx *ctx, int32_t n_layers, const int32_t *widths,
                                          const int64_t *u1, const int64_t *u2, int64_t n_pairs,
                                          int32_t criterion, const ibmc_cov_params *params,
                                          ibmc_cov_summary *out, uint64_t *covered_bits);

/* Coverage-guided test generation (tests chosen by the covers of Sec. III-B,
 * which the paper leaves as future work in Sec. IV-C): every point of level
 * k of the delta-set domain of `image` is a candidate test x'; each pair
 * (image, x') covers a set of neuron pairs under `criterion` (as
 * ibmc_coverage computes for one pair).  Tests are taken greedily: each
 * time the candidate that covers the most pairs not covered by the tests
 * taken so far (the lowest rank among equals), until no candidate adds a
 * pair or max_tests are taken.  tests[i] (room for max_tests): the i-th
 * test as a point (k, rank, its label; prop 0), gains[i] (nullable) the
 * pairs it added; *n_tests the number taken; out: the coverage of all tests
 * together; covered_bits (nullable): their covered pairs in ibmc_coverage's
 * layout.  Integer networks whose non-input layers have at most 64 units,
 * at most 4,096 neuron pairs and at most 2^26 candidates (else
 * IBMC_E_UNIMPL). */
ibmc_status ibmc_coverage_search(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image, int32_t n_pixels,
                                 const int16_t *delta_set, int32_t n_deltas, int32_t k, int32_t criterion,
                                 const ibmc_cov_params *params, int32_t max_tests, ibmc_cex *tests,
                                 int64_t *gains, int32_t *n_tests, ibmc_cov_summary *out,
                                 uint64_t *covered_bits);

/* ---- training of the float networks ------------------------------------ */
/* The networks the checks run on are trained on labelled examples (Sec.
 * II-A); the verifier's counterexamples, each labelled with its clean
 * image's label, can be added to that training set (Sec. VI) and the
 * retrained network checked again.  Float (IBMC_ACT_SIGMOID_F32) networks
 * only (else IBMC_E_UNIMPL).  The loss of a labelled set is the mean over its
 * images of the cross-entropy of the softmax of the logits against the
 * label, with a_0 = x / 256, sigmoid hidden layers and linear logits as in
 * the checks.  theta, the flat parameter vector: for each layer l in turn,
 * W_l row-major [dims[l]][dims[l-1]] then b_l [dims[l]] (sum over layers of
 * dims[l] * (dims[l-1] + 1) floats).  images: host uint8 [n][dims[0]];
 * labels: host int32 [n], each in [0, classes) (else IBMC_E_INVALID). */

/* Loss (nullable, host double) and gradient (nullable, host float
 * [n_params] in theta's layout) of the net on n >= 1 labelled images. */
ibmc_status ibmc_mlp_loss_grad(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *images,
                               const int32_t *labels, int64_t n, float *grad, double *loss);

/* Mini-batch Adam (Kingma and Ba): each epoch visits the n images in an
 * order, in consecutive batches of `batch` (the last one smaller); each
 * batch takes one Adam step on its mean loss.  order (nullable, host int64
 * [epochs][n], each entry in [0, n)): the images of epoch e in order; NULL:
 * a Fisher-Yates shuffle per epoch from `seed` (splitmix64).  beta1, beta2,
 * eps of 0 take 0.9, 0.999, 1e-8. */
typedef struct {
    int32_t epochs;                       /* >= 1 */
    int32_t batch;                        /* >= 1 */
    float lr, beta1, beta2, eps;
    uint64_t seed;
    const int64_t *order;
} ibmc_fit_opts;

/* Train a copy of `net` from its parameters on n labelled images; *out
 * receives the trained network (a new handle, freed with ibmc_free_mlp;
 * `net` is left as it was), theta_out (nullable, host float [n_params]) its
 * parameters, epoch_loss (nullable, host double [epochs]) the mean loss of
 * each epoch's batches before their steps.  IBMC_E_RANGE if a parameter
 * becomes non-finite. */
ibmc_status ibmc_fit_mlp(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *images,
                         const int32_t *labels, int64_t n, const ibmc_fit_opts *opts,
                         ibmc_mlp **out, float *theta_out, double *epoch_loss);

/* ---- learned proposal network ------------------------------------------ */
/* A two-layer scorer s = w2 . relu(W1 f + b1) + c over 32 features of a
 * candidate (pixel, delta), trained with a positive-weighted logistic loss
 * and Adam by the library's own bf16 matrix-core kernels.  It only orders the
 * search: the ordered check still enumerates every point, so its verdicts
 * and records equal the plain check's. */

#define IBMC_PROP_FEATURES 32
#define IBMC_PROP_HIDDEN 128

typedef struct {
    int32_t epochs, batch;
    float lr, beta1, beta2, eps;
    float pos_weight;                     /* <= 0: n_negative / n_positive */
    uint64_t seed;                        /* initialisation and shuffles */
} ibmc_train_opts;

/* Create a proposer with seeded random weights (fp32 master copy). */
ibmc_status ibmc_proposer_create(ibmc_ctx *ctx, uint64_t seed, ibmc_proposer **out);
void ibmc_proposer_free(ibmc_proposer *p);
/* Read / write the fp32 parameters: W1 [128][32], b1 [128], w2 [128], c [1]
 * (host arrays, each nullable on get). */
ibmc_status ibmc_proposer_get(ibmc_proposer *p, float *W1, float *b1, float *w2, float *c);
ibmc_status ibmc_proposer_set(ibmc_proposer *p, const float *W1, const float *b1,
                              const float *w2, const float *c);
/* Candidate features of an image, n_pixels * n_deltas rows of 32 floats
 * (host), in candidate order (pixel-major, then delta index): row / (rows-1),
 * col / (cols-1), x / 255, d / dmax, e / dmax with e = clamp(x+d) - x,
 * L1 and L2 norms of the first-layer weight column normalised by their
 * maxima over pixels, the L1 norm restricted to first-layer units whose
 * clean potential is in the requantiser's linear window normalised the same
 * way, then 1, then zeros. */
ibmc_status ibmc_proposer_features(ibmc_ctx *ctx, const ibmc_mlp *net, const uint8_t *image,
                                   int32_t rows, int32_t cols, const int16_t *delta_set,
                                   int32_t n_deltas, float *features);
/* One forward/backward pass on a batch (host features [B][32], labels [B]
 * of 0/1): mean loss and gradients with the parameter shapes (host). */
ibmc_status ibmc_proposer_grad(ibmc_ctx *ctx, ibmc_proposer *p, const float *features,
                               const float *labels, int32_t B, float pos_weight, float *loss,
                               float *gW1, float *gb1, float *gw2, float *gc);
/* Train on N labelled candidates (host arrays); losses (nullable) receives
 * the mean loss of each epoch. */
ibmc_status ibmc_proposer_train(ibmc_ctx *ctx, ibmc_proposer *p, const float *features,
                                const float *labels, int64_t N, const ibmc_train_opts *opts,
                                float *losses);
/* Scores of an image's candidates (host float [n_pixels * n_deltas]). */
ibmc_status ibmc_proposer_score(ibmc_ctx *ctx, const ibmc_proposer *p, const ibmc_mlp *net,
                                const uint8_t *image, int32_t rows, int32_t cols,
                                const int16_t *delta_set, int32_t n_deltas, float *scores);

/* As ibmc_proposer_score with `image` (dims[0] bytes) and `scores`
 * (n_pixels * n_deltas floats) device pointers on the context's device. */
ibmc_status ibmc_proposer_score_dev(ibmc_ctx *ctx, const ibmc_proposer *p, const ibmc_mlp *net,
                                    const uint8_t *image, int32_t rows, int32_t cols,
                                    const int16_t *delta_set, int32_t n_deltas, float *scores);

/* Training labels from a property's counterexample records: labels_out
 * (host float [n_pixels * n_deltas], candidate p * n_deltas + i) is 1 for
 * every (pixel, delta index) that occurs in some record, else 0. */
ibmc_status ibmc_label_candidates(ibmc_ctx *ctx, int32_t n_pixels, int32_t n_deltas, const ibmc_cex *recs,
                                  int64_t n, float *labels_out);

/* As ibmc_label_candidates, with counts_out[c] the number of records in
 * which candidate c occurs (a graded training signal). */
ibmc_status ibmc_count_candidates(ibmc_ctx *ctx, int32_t n_pixels, int32_t n_deltas, const ibmc_cex *recs,
                                  int64_t n, float *counts_out);

/* Ordered check of levels k <= 2 (integer nets): level 1 visits candidates by
 * decreasing score; level 2 visits "shells": candidates sorted c0, c1, ...,
 * shell t holds the pairs (c_t, c_j), j < t, on distinct pixels, so every
 * level-2 point is visited once.  p == NULL visits the plain order (level 1
 * pixel-major, level 2 grouped by the first pixel and its delta).  Work is
 * handed out in visiting order; the summary's ttfc_seconds and
 * points_before_first report when the first counterexample was found (host
 * clock, from the call's start, including scoring and sorting).  The full
 * enumeration always completes unless opts->stop_at_first is set, in which
 * case the call returns once the first counterexample is confirmed. */
ibmc_status ibmc_check_property_ranked(ibmc_ctx *ctx, const ibmc_mlp *net,
                                       const ibmc_proposer *p, const uint8_t *image,
                                       int32_t n_pixels, int32_t rows, int32_t cols,
                                       const int16_t *delta_set, int32_t n_deltas,
                                       const ibmc_check_opts *opts, ibmc_check_summary *out,
                                       ibmc_cex *cex_buf);

/* ---- tuning ------------------------------------------------------------ */

/* Time the kernel variants of an integer network (matrix-core instances:
 * points per wave, weights staged in LDS or read through L2; the
 * lane-per-point kernel where the shape allows it) on a synthetic image,
 * delta set of n_deltas and level k, and remember the fastest for that
 * network shape in the context (every later check of the shape, single or
 * batched, launches it).  json_out (nullable, json_cap bytes) receives the
 * measurements as JSON. */
ibmc_status ibmc_autotune(ibmc_ctx *ctx, const ibmc_mlp *net, int32_t k, int32_t n_deltas,
                          char *json_out, int64_t json_cap);
/* The context's tuning table (shape key -> variant name, as a flat JSON
 * object): save it to a file, or merge a saved one into the context
 * (n_loaded: entries read).  IBMC_E_INVALID when the file cannot be
 * written / read or is malformed. */
ibmc_status ibmc_tune_save(ibmc_ctx *ctx, const char *path);
ibmc_status ibmc_tune_load(ibmc_ctx *ctx, const char *path, int32_t *n_loaded);
/* Name of the enumeration kernel a (non-resumable) check of the network
 * launches now: a forced variant, else the tuned one for its shape, else the
 * built-in choice ("f32" for float networks); written NUL-terminated into
 * out (cap bytes). */
ibmc_status ibmc_chosen_variant(ibmc_ctx *ctx, const ibmc_mlp *net, char *out, int64_t cap);
/* Batches over several networks run as one HIP graph; a batch whose
 * launches match the previous one's (same plans, buffers and counter
 * layout) replays its instantiated graph.  Graph launches and replays so
 * far in the context. */
ibmc_status ibmc_graph_stats(ibmc_ctx *ctx, int64_t *launches, int64_t *reuses);
/* Force a variant by its name (as listed by the tuner's JSON); NULL resets
 * to the built-in choice. */
ibmc_status ibmc_set_variant(ibmc_ctx *ctx, const ibmc_mlp *net, const char *variant);
/* Device time of the last enumeration kernel launches of this context, in
 * seconds, and the number of launches they span (for roofline reporting). */
ibmc_status ibmc_last_kernel_time(ibmc_ctx *ctx, double *seconds, int32_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* IBMC_H */
