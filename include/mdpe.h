/*
 * mdpe.h -- C ABI of libmdpe: evaluation and differentiation of a sparse
 * polynomial at power series truncated at degree d, in m-fold double
 * arithmetic, on an AMD Instinct MI355X (gfx950).
 *
 * Method: J. Verschelde, "Accelerated polynomial evaluation and
 * differentiation at power series in multiple double precision"
 * (arXiv 2101.10881).  The polynomial is eq. (3) of Section 4; products of
 * series are the truncated convolutions of eq. (1), Section 2; the gradient
 * comes from the forward / backward / cross products of Section 3, run as
 * layers of convolution jobs followed by levels of addition jobs on one
 * data array (Section 5, Fig. 1, eq. (6)).
 *
 * Conventions for every entry point:
 *   - Return 0 (MDPE_OK) on success or a negative mdpe_status; nothing
 *     throws.  last_error_string() gives a message for the calling thread.
 *   - A multiple double is m consecutive limbs of binary64, limb 0 the most
 *     significant; values are normalised expansions (|x_{j+1}| <= ulp(x_j)/2).
 *   - User series buffers are limb-planar and row-major (the m data arrays of
 *     Section 5): a batch of `count` series is double[m][count][d+1].
 *   - Device buffers are owned by the caller (e.g. torch tensors); the library
 *     allocates nothing during evaluation.  Work is enqueued on the caller's
 *     HIP stream (hipStream_t passed as void*; NULL = default stream) and is
 *     asynchronous: outputs are ready when that stream reaches them.
 */
#ifndef MDPE_H
#define MDPE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MDPE_OK = 0,
    MDPE_EINVAL = -1,       /* bad argument or polynomial description */
    MDPE_EUNSUPPORTED = -2, /* m not in {1,2,3,4,5,8,10}, or d too large for one workgroup's LDS */
    MDPE_ENOMEM = -3,       /* host or device allocation failed at plan time */
    MDPE_EDEVICE = -4       /* a HIP runtime call failed (its message is kept) */
} mdpe_status;

/* Opaque plan: job lists for one polynomial structure, immutable once built,
 * safe to share between threads. */
typedef struct mdpe_plan mdpe_plan;

/* Polynomial structure (Section 5, the input list: N, n, d, supports). */
typedef struct {
    int32_t n;              /* number of variables, n >= 1 */
    int32_t N;              /* number of monomials, a_0 not counted, N >= 0 */
    int32_t d;              /* truncation degree, d >= 0: every series has d+1 coefficients */
    int32_t m;              /* limbs per coefficient, one of 1, 2, 3, 4, 5, 8, 10 */
    const int32_t *nvars;   /* host [N]: n_k, 1 <= n_k <= n */
    const int32_t *vars;    /* host [sum n_k]: 0-based variable indices, strictly
                               increasing inside each monomial (Section 4) */
    uint32_t flags;         /* 0, or MDPE_KEEP_MONOMIAL_VALUES, MDPE_COMPLEX, MDPE_STREAM_OPERANDS,
                               MDPE_STAGE_OPERANDS, MDPE_ASAP_LAYERS, MDPE_FUSED_LAYERS,
                               MDPE_LAYER_LAUNCHES, MDPE_CHAIN_LAUNCH, MDPE_NO_CHAIN_LAUNCH,
                               MDPE_SINGLE_LAUNCH */
    const int32_t *exps;    /* host [sum n_k] exponents in 1..64 aligned with vars, or NULL
                               (every exponent one).  Monomial k is then
                               a_k prod_j z_{i_j}^{e_j}: Section 3 writes it as the
                               multilinear monomial with the common factor
                               a_k prod_j z_{i_j}^{e_j - 1}, taken from a table of
                               powers z_i^p := z_i^{p-1} * z_i; the partial derivative
                               for z_{i_j} is e_j times the multilinear one (an
                               m-double product with (e_j, 0, ..., 0), per part when
                               complex).  Not combinable with
                               MDPE_KEEP_MONOMIAL_VALUES when an exponent exceeds one
                               (MDPE_EUNSUPPORTED); plan_batch refuses such plans. */
} mdpe_poly_desc;

/* Plan flag: also compute and keep every monomial's product of variables
 * M_k = prod_{j in monomial k} z_j (one extra convolution per monomial with
 * n_k >= 2), so that eval_adjoint can run after eval_and_diff.  The value and
 * gradient are bit-identical with or without it. */
#define MDPE_KEEP_MONOMIAL_VALUES 1u

/* Plan flag: complex series (Sections 2 and 5 keep real and imaginary parts in
 * separate arrays).  Every coefficient, input and output buffer then holds
 * 2m limb planes, the m real limbs followed by the m imaginary limbs, e.g.
 * coeff double[2][m][N+1][d+1]; the workspace doubles.  A product of two
 * complex m-doubles is (xr yr - xi yi) + (xr yi + xi yr) i with each product
 * one m-double multiplication and each sum one m-double addition (the
 * difference adds the exactly negated product); a sum adds the parts.
 * Not combinable with MDPE_KEEP_MONOMIAL_VALUES (MDPE_EUNSUPPORTED), not
 * accepted by plan_batch (MDPE_EUNSUPPORTED). */
#define MDPE_COMPLEX 2u

/* Plan flag: read both convolution operands from global memory (L2) instead
 * of staging them in LDS.  Plans choose this by themselves when it is
 * estimated to be faster (few jobs per layer at a large degree), and when a
 * job's operands would not fit in one workgroup's LDS, i.e. beyond
 * (d+1)*w*8 > 131072 bytes (w = m doubles per coefficient, 2m complex; twice
 * that when w <= 2), which lifts the degree limit to d + 1 <= 65535.  Then
 * one job's coefficients may be spread over several wavefronts
 * (mdpe_plan_info.waves_per_job), and no convolution writes its own first
 * operand (the in-place multiplications get fresh output slots).  The
 * operation order, hence every output bit, is the same as with staged
 * operands.  plan_batch refuses streamed plans (MDPE_EUNSUPPORTED). */
#define MDPE_STREAM_OPERANDS 4u

/* Plan flag: stage the operands in LDS even where streaming them is
 * estimated to be faster (plans otherwise choose by a cost model: few jobs
 * per layer at a large degree stream, with several wavefronts per job).
 * MDPE_EUNSUPPORTED when they do not fit; excludes MDPE_STREAM_OPERANDS. */
#define MDPE_STAGE_OPERANDS 8u

/* Plan flag: keep every convolution at its earliest layer, the layering of
 * Section 5 (p1 at four variables per monomial: 3640, 5460, 5460 and 1820
 * jobs per layer).  Without it a plan moves jobs with slack to later layers
 * where that fills whole rounds of the GPU's SIMDs (p1: 3072, 4096, 6144 and
 * 3068 jobs; mdpe_plan_info.balanced_layers).  Any layering that keeps each
 * job after the jobs it depends on gives the same output bits. */
#define MDPE_ASAP_LAYERS 16u

/* Plan flag: run every convolution layer in one launch (plans do so by
 * themselves where it is estimated faster: at least four layers, one
 * wavefront per job, at most four jobs of a component per layer, and either
 * one double per coefficient, two up to d = 63, or layers under 512 jobs with
 * d <= 127 up to four doubles per coefficient, d <= 31 at five and ten, d <= 8
 * at other widths;
 * MDPE_LAYER_LAUNCHES keeps one launch per layer).  The jobs fall into
 * independent components -- no slot written by a job of one component is read
 * or written by a job of another (for multilinear polynomials, one component
 * per monomial) -- and one workgroup runs a component's layers in order, with
 * a workgroup barrier between layers, one job per wavefront at a time.  For
 * deep chains of small layers (many variables per monomial, few monomials)
 * this replaces one kernel boundary per layer, each costing a few
 * microseconds, by a barrier.  Each job's arithmetic, hence every output bit,
 * is that of the per-layer launches.  Ignored for streamed-operand plans
 * (mdpe_plan_info.fused_components is then 0); the batched executor keeps its
 * own schedule. */
#define MDPE_FUSED_LAYERS 32u

/* Plan flag: one launch per convolution layer, never fused or chained
 * (excludes MDPE_FUSED_LAYERS and MDPE_CHAIN_LAUNCH). */
#define MDPE_LAYER_LAUNCHES 64u

/* Plan flag: run the chains of products in one pipelined launch (plans do so
 * by themselves where it is estimated well under the layered or fused
 * launches: chains of at least 16 products holding a quarter of the
 * convolutions or more, such as p2's).  A chain is a sequence of
 * convolutions where each job's first operand is the previous job's output
 * and its second a staged input series: the forward products f_j = f_{j-1} *
 * z_{i_j} and the backward products b_j = b_{j-1} * z_{i_{n-j}} of Section 3.
 * Coefficient i of a product is final once its own i+1 terms are summed, and
 * the next product of its chain needs its first operand's coefficients in
 * increasing i, so one workgroup per chain overlaps the chain's products,
 * passing each coefficient on through LDS; the remaining convolutions (the
 * cross products) follow in layers after it.  Each coefficient is the same
 * sequential sum as in the per-layer launches, so every output bit is the
 * same.  Such plans give the in-place product b_{n-2} * a_k a fresh output
 * slot.  MDPE_EUNSUPPORTED when no chain qualifies or its first operands do
 * not fit in LDS; excludes MDPE_FUSED_LAYERS, MDPE_LAYER_LAUNCHES,
 * MDPE_STREAM_OPERANDS and MDPE_NO_CHAIN_LAUNCH. */
#define MDPE_CHAIN_LAUNCH 128u

/* Plan flag: never the chain launch; the plan chooses between layered and
 * fused launches as without it (excludes MDPE_CHAIN_LAUNCH). */
#define MDPE_NO_CHAIN_LAUNCH 256u

/* Plan flag: the whole evaluation in one launch of one workgroup (plans do so
 * by themselves where it is estimated under 0.7 of the per-launch time: plans
 * so small that the boundaries between their ~10 dependent launches, ~4.5 us
 * each on MI355X, dominate, such as 16 three-variable monomials at d = 8).
 * The workgroup's wavefronts run staging, every convolution layer (each
 * wavefront a group of jobs per round, as in a per-layer launch), the scale
 * stage, every addition level and the gather, with a workgroup barrier after
 * each.  Every output bit is that of the per-launch path.  Excludes
 * MDPE_FUSED_LAYERS, MDPE_LAYER_LAUNCHES, MDPE_STREAM_OPERANDS and
 * MDPE_CHAIN_LAUNCH. */
#define MDPE_SINGLE_LAUNCH 512u

/* Plan summary. */
typedef struct {
    int64_t n_series;       /* series slots in the data array A: e/(d+1) of eq. (6) */
    int64_t n_conv;         /* convolution jobs: sum over monomials of 3 n_k - 3 (1 if n_k = 1) */
    int64_t n_add;          /* addition jobs */
    int32_t n_layers;       /* convolution launches = largest n_k */
    int32_t n_levels;       /* addition launches */
    int64_t workspace_bytes;/* device workspace eval_and_diff needs: n_series*(d+1)*m*8, twice that
                               for MDPE_COMPLEX */
    int32_t jobs_per_group; /* convolution jobs per 64-lane workgroup */
    int32_t lane_steps;     /* multiply-add steps per lane per workgroup (lane schedule length) */
    int32_t n, N, d, m;
    int64_t n_reverse;      /* correlation jobs of the reverse pass (0 without the flag) */
    uint32_t flags;
    int64_t n_scale;        /* exponent scale jobs (0 for multilinear polynomials) */
    int32_t waves_per_job;  /* wavefronts sharing one convolution job (streamed operands) */
    int32_t streamed;       /* 1 if the convolution operands are read from global memory */
    int32_t simple_dealing; /* 1 if coefficients (of at most two doubles) are dealt to lanes in turn
                               instead of following the lane schedule */
    int32_t balanced_layers;/* 1 if convolutions with slack were moved to later layers (see
                               MDPE_ASAP_LAYERS) */
    int32_t fused_components;/* MDPE_FUSED_LAYERS: independent components, one workgroup each
                               (0 when the layers are launched one by one) */
    int32_t fused_waves;    /* MDPE_FUSED_LAYERS: wavefronts per component workgroup (at most 4;
                               fewer at launch where their LDS would not fit) */
    int32_t chain_layers;   /* MDPE_CHAIN_LAUNCH: layers 1..chain_layers run in the chain launch
                               (layer L: the L-th product of every chain); 0 without it */
    int32_t chain_count;    /* MDPE_CHAIN_LAUNCH: chains, one workgroup each */
    int32_t chain_waves;    /* MDPE_CHAIN_LAUNCH: wavefronts per chain workgroup (4, 8, 12 or 16) */
    int32_t chain_window;   /* MDPE_CHAIN_LAUNCH: steps between workgroup barriers */
    int32_t chain_ring;     /* MDPE_CHAIN_LAUNCH: LDS slots of first operands per chain */
    int32_t single_launch;  /* 1 if the whole evaluation runs in one workgroup (MDPE_SINGLE_LAUNCH) */
    int32_t single_waves;   /* MDPE_SINGLE_LAUNCH: wavefronts of that workgroup */
} mdpe_plan_info;

/*
 * Build a plan (Section 5, the data staging algorithm): series slots
 * a_0, a_1..a_N, z_1..z_n, then all forward, backward and cross products;
 * the convolution triplets of every layer; the addition pairs of every
 * level of the pairwise tree; the output slots; a hazard check (no job
 * writes a slot another job of its layer reads or writes).
 * device >= 0: the job arrays are uploaded to that HIP device once.
 * device == -1: a host-only plan for inspection (eval_and_diff refuses it).
 * desc and its arrays are only read during the call.
 */
int plan_polynomial(const mdpe_poly_desc *desc, int device, mdpe_plan **out);

int plan_info(const mdpe_plan *plan, mdpe_plan_info *out);

/* conv_sizes[n_layers], add_sizes[n_levels]: jobs per launch (either may be NULL). */
int plan_layer_sizes(const mdpe_plan *plan, int32_t *conv_sizes, int32_t *add_sizes);

/* Convolution jobs as rows {layer (1-based), t1, t2, t3} in slot units (a slot
 * is one series of d+1 coefficients; slot s starts at s*(d+1) in the paper's
 * array A); job meaning A[t3] := A[t1] * A[t2].  rows: int32[n_conv][4], in
 * launch order. */
int plan_conv_jobs(const mdpe_plan *plan, int32_t *rows);

/* MDPE_FUSED_LAYERS plans: the convolution jobs as rows {component, layer
 * (1-based), t1, t2, t3}, grouped by component, then layer, in the order the
 * fused launch runs them.  rows: int32[n_conv][5].  MDPE_EINVAL for a plan
 * without fused layers. */
int plan_fused_jobs(const mdpe_plan *plan, int32_t *rows);

/* MDPE_CHAIN_LAUNCH plans: the jobs of the chain launch as rows {chain,
 * position in the chain (0-based), t1, t2, t3}, chain after chain; position q
 * of every chain is convolution layer q+1.  rows: int32[n][5] with n the sum
 * of the chain lengths (the jobs of layers 1..chain_layers).  MDPE_EINVAL for
 * a plan without a chain launch. */
int plan_chain_jobs(const mdpe_plan *plan, int32_t *rows);

/*
 * The lane schedule of one chain (host only): L products of degree d on
 * `waves` wavefronts (4, 8, 12 or 16), a workgroup barrier every `window` steps, the
 * first operands in `ring` LDS slots (job j's in slot j mod ring).  codes:
 * int32[64 * waves][*stride], row r for thread r of the chain's workgroup:
 * (j << 16) | k computes coefficient k of the j-th product (k+1 steps, its
 * terms i = 0..k in increasing i), (0x7FFF << 16) | (g-1) idles g steps, -1
 * ends the row.  *steps: steps every thread runs (an even multiple of window).
 * codes NULL returns only *stride and *steps; else capacity is its length.
 */
int chain_schedule(int32_t L, int32_t d, int32_t waves, int32_t window, int32_t ring, int32_t *codes,
                   int64_t capacity, int32_t *stride, int32_t *steps);

/*
 * Check a chain schedule against the chain kernel's timing (host only):
 * step t's first operand coefficient is read from LDS in iteration t-1 (step
 * 0's before the loop), a coefficient is stored in the iteration of its last
 * step, and a workgroup barrier follows iteration s when (s+1) % window == 0.
 * Every coefficient of every product exactly once, within `steps`; each read
 * of a first-operand coefficient in a later window than its store by the
 * previous product, and its overwriting (by the product `ring` places later)
 * in a later window than the read.  MDPE_OK, or MDPE_EINVAL with the first
 * violation in last_error_string().
 */
int check_chain_schedule(int32_t L, int32_t d, int32_t waves, int32_t window, int32_t ring, int32_t steps,
                         const int32_t *codes, int32_t stride);

/* Addition jobs as rows {level (1-based), t1, t2}: A[t2] := A[t2] + A[t1].
 * rows: int32[n_add][3], in launch order. */
int plan_add_jobs(const mdpe_plan *plan, int32_t *rows);

/* out_slots[1+n]: slot holding the value, then for each variable the slot
 * holding its partial derivative, or -1 when the variable is absent. */
int plan_outputs(const mdpe_plan *plan, int32_t *out_slots);

/* Exponent scale jobs as rows {src, dst, e}: A[dst] := e * A[src], coefficient
 * by coefficient, after the last convolution layer and before the first
 * addition level.  rows: int32[n_scale][3]. */
int plan_scale_jobs(const mdpe_plan *plan, int32_t *rows);

/*
 * Check job lists against the rules a plan meets (Section 5: the jobs of one
 * layer are independent, so they may run in any order and at once).  Host
 * only: no device work, nothing is kept.  For callers that build or edit job
 * lists themselves, and for testing the checker that plan_polynomial runs on
 * every plan it builds.
 *   n, N          variables and monomials; slots 0 .. N+n hold the staged
 *                 inputs a_0..a_N, z_1..z_n
 *   n_series      slots in the data array A
 *   conv_rows     int32[n_conv][4] {layer, t1, t2, t3}, the format of
 *                 plan_conv_jobs: layers numbered from 1, nondecreasing
 *   add_rows      int32[n_add][3] {level, t1, t2}, the format of plan_add_jobs
 *   out_slots     int32[1+n] (value slot, then each partial derivative's, -1
 *                 when absent) or NULL: each must be written by some stage
 *   extra_staged  int32[n_extra] or NULL: further slots filled at staging
 *                 time (the derivative copies of one-variable monomials)
 *   waves_per_job wavefronts that share one convolution job (>= 1)
 *   streamed      nonzero when operands are read from global memory
 * Rules: a job reads only slots written before its stage (inputs, an earlier
 * layer, an earlier level; the convolutions all precede the additions); no two
 * jobs of a stage write one slot; no job reads a slot another job of its stage
 * writes; a convolution never writes its second operand, nor its first when
 * streamed or when waves_per_job > 1; every output slot is written.
 * Returns MDPE_OK, or MDPE_EINVAL with the first violated rule and its stage
 * in last_error_string().
 */
int check_plan_jobs(int32_t n, int32_t N, int64_t n_series, const int32_t *conv_rows, int64_t n_conv,
                    const int32_t *add_rows, int64_t n_add, const int32_t *out_slots, const int32_t *extra_staged,
                    int64_t n_extra, int32_t waves_per_job, int32_t streamed);

/*
 * Evaluate p and its gradient (Sections 4-5).
 *   coeff     device double[m][N+1][d+1], a_0 first (read only)
 *   z         device double[m][n][d+1] (read only)
 *   value     device double[m][d+1] (written)
 *   grad      device double[m][n][d+1] (written; absent variables get +0.0)
 *   (MDPE_COMPLEX plans: each of these has a leading [2], real then imaginary)
 *   workspace device buffer of plan_info().workspace_bytes, 256-byte aligned;
 *             its contents are scratch and may be reused between calls
 *             that are ordered on one stream
 *   stream    hipStream_t or NULL
 * Launches: one staging kernel; the convolutions as the plan chose them
 * (plan_info): one kernel per layer, one fused launch of every layer
 * (fused_components > 0), or the chain launch followed by one kernel per
 * remaining layer (chain_layers > 0); one scale kernel when an exponent exceeds
 * one; one addition kernel per level; one gather kernel.  A plan with
 * single_launch = 1 runs all of it in one kernel.  Calls on different streams
 * must not share a workspace.
 */
int eval_and_diff(const mdpe_plan *plan, const double *coeff, const double *z, double *value,
                  double *grad, void *workspace, void *stream);

/*
 * eval_and_diff without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a fixed array of
 * 64 MiB (67108864 bytes) that the library holds on each device from load to
 * process end; the call itself allocates nothing.  Plans whose
 * plan_info().workspace_bytes exceed it are refused with MDPE_EUNSUPPORTED
 * (use eval_and_diff).  Every call on one device shares that device's array:
 * calls that overlap on one device (other streams, other threads) race, and
 * the array keeps the last call's contents.  Arguments, launches and output
 * bits are those of eval_and_diff.
 */
int eval_and_diff_noalloc(const mdpe_plan *plan, const double *coeff, const double *z, double *value,
                          double *grad, void *stream);

/*
 * Reverse pass (needs MDPE_KEEP_MONOMIAL_VALUES).  For an upstream adjoint
 * ybar of the value series, L = sum_t ybar_t p_t, returns
 *   coeff_bar[k][s] = dL/da_k[s] = sum_{j=0..d-s} ybar[s+j] M_k[j]   (coeff_bar[0] = ybar)
 *   z_bar[i][s]     = dL/dz_i[s] = sum_{j=0..d-s} ybar[s+j] g_i[j]   (g_i = dp/dz_i)
 * since p is linear in every input series (Section 4, eq. (3)) and products
 * are the convolutions of eq. (1).  Each coefficient is md_mul(ybar_s, y_0)
 * followed by += md_mul(ybar_{s+j}, y_j) in increasing j: one layer of
 * N + (present variables) correlation jobs on the convolution kernel.
 *   ybar      device double[m][d+1] (read only)
 *   workspace the buffer of the preceding eval_and_diff with this plan, on
 *             the same stream, unmodified since: it holds the monomial
 *             products M_k (the pass writes its own slots of it)
 *   grad      device double[m][n][d+1] (read only): the gradient g that
 *             eval_and_diff returned, copied into the workspace first
 *   coeff_bar device double[m][N+1][d+1] (written)
 *   z_bar     device double[m][n][d+1] (written; absent variables get +0.0)
 * The adjoint of an m-double is returned as an m-double: limb 0 is the
 * double-precision value of the derivative and the lower limbs extend it.
 */
int eval_adjoint(const mdpe_plan *plan, const double *ybar, void *workspace, const double *grad, double *coeff_bar,
                 double *z_bar, void *stream);

/* Reverse-pass jobs as rows {t1 (ybar slot), t2 (M_k or gradient slot), t3}. */
int plan_reverse_jobs(const mdpe_plan *plan, int32_t *rows);

/* Per-kernel timing with HIP events recorded on the launch stream, in the
 * paper's four categories (Section 6.2: convolution, addition, their sum; the
 * caller measures wall time).  Times accumulate over calls until read. */
typedef struct mdpe_profiler mdpe_profiler;
typedef struct {
    double stage_ms, cnv_ms, add_ms, gather_ms;
    int64_t n_stage, n_cnv, n_add, n_gather; /* launches timed */
} mdpe_times;

int profiler_create(mdpe_profiler **out);
/* Same as eval_and_diff, with an event pair around every launch. */
int eval_and_diff_profiled(const mdpe_plan *plan, const double *coeff, const double *z, double *value,
                           double *grad, void *workspace, void *stream, mdpe_profiler *prof);
/* Same as eval_adjoint, timed (correlation launches count as convolution). */
int eval_adjoint_profiled(const mdpe_plan *plan, const double *ybar, void *workspace, const double *grad,
                          double *coeff_bar, double *z_bar, void *stream, mdpe_profiler *prof);
/* Which launches get an event pair: a mask of MDPE_TIME_STAGE, MDPE_TIME_CONV,
 * MDPE_TIME_ADD and MDPE_TIME_GATHER (all by default).  Each pair is two more
 * commands on the stream (~0.12 ms per p1 evaluation for all 17 launches), so
 * a caller that needs only the convolution launches' durations times just those.
 * MDPE_EINVAL for unknown bits, or while recorded events are unread. */
#define MDPE_TIME_STAGE 1u
#define MDPE_TIME_CONV 2u
#define MDPE_TIME_ADD 4u
#define MDPE_TIME_GATHER 8u
int profiler_set_classes(mdpe_profiler *prof, uint32_t classes);
/* Wait for the recorded events, add their durations into *out, reset. */
int profiler_read(mdpe_profiler *prof, mdpe_times *out);
void profiler_destroy(mdpe_profiler *prof);

/*
 * Elementwise m-double operation on device arrays (op 0: z = x + y,
 * op 1: z = x * y), planar double[m][count]; complex m-doubles (op 2: z = x + y,
 * op 3: z = x * y), planar double[2][m][count], real limbs then imaginary limbs.
 * Diagnostic entry point that exposes the device multiple-double library the
 * kernels use.
 */
int md_elementwise(int op, int m, int64_t count, const double *x, const double *y, double *z, void *stream);

/* ------------------------------------------------------- batched plans --
 * Many polynomials in one persistent launch.  The batch references its plans
 * (which must outlive it); each instance keeps its own buffers.  All stages
 * of all instances (staging, convolution layers, addition levels, gather)
 * become tasks; each instance goes whole to one of 8 queues, one per XCD,
 * balanced by estimated cost, so that producers and consumers of an instance
 * share one L2 -- except an instance whose estimated cost exceeds an eighth
 * of the batch (a batch of one), whose tasks, one group of jobs each, are
 * dealt over all queues in turn.  Every queue is ordered by pipeline depth.
 * One persistent kernel of one-wavefront workgroups claims the tasks of the
 * XCD it runs on, and a task waits (agent-scope acquire) on a per-instance
 * completion counter for the stages before its own.  Bits are identical to
 * eval_and_diff of each instance.
 * Precisions in one batch: all equal, or {2, 4}.
 */
typedef struct mdpe_batch mdpe_batch;

/* Tile choice for instances of precision m and degree d (from the autotuner);
 * zero fields take the defaults. */
typedef struct {
    int32_t m, d;
    int32_t jobs_per_group;     /* convolution jobs per wavefront pass (lane schedule) */
    int32_t groups_per_task;    /* passes per convolution task */
    int32_t add_items_per_task; /* coefficients per addition / staging / gather task */
    int32_t deal;               /* coefficients of at most two doubles: 0 the cost model's choice,
                                   1 the lane schedule, 2 dealt to the lanes in turn (either gives
                                   the same bits); ignored from three doubles on */
} mdpe_batch_tile;

typedef struct {
    int32_t count;
    int64_t n_tasks, n_conv_tasks, n_add_tasks;
    int64_t lds_bytes;
    int32_t grid;               /* persistent workgroups (known after the first launch) */
    int32_t m1, m2;
    int64_t workspace_bytes;    /* the one workspace eval_and_diff_batch needs: every
                                   instance's plan_info().workspace_bytes, each part
                                   rounded up to 256 bytes */
} mdpe_batch_info;

/* Plan the batch once (Section 5 builds the job lists once and evaluates them
 * per call; the batch does the same for all its instances).
 *   plans      [count] device plans on one device, which must outlive the batch
 *   tune_cache path of the autotuner's JSON cache, or NULL / "" for the
 *              default tiles.  The tiles listed under the device's
 *              architecture name ("gfx950") are used; a cache without that
 *              name gives the defaults.  MDPE_EINVAL when the file cannot be
 *              read or is not such a cache.  The file is read during the call
 *              only. */
int plan_batch(const mdpe_plan *const *plans, int count, const char *tune_cache, mdpe_batch **out);
/* The same with the tiles given directly: tiles may be NULL (ntiles = 0). */
int plan_batch_tiles(const mdpe_plan *const *plans, int count, const mdpe_batch_tile *tiles, int ntiles,
                     mdpe_batch **out);
/*
 * Evaluate every instance and its gradient in one persistent launch, replayed
 * from a hipGraph captured at the first call (the hot path of the batch).
 *   coeff, z, value, grad  host arrays [count] of device pointers, each with
 *             the meaning and layout of eval_and_diff for that instance
 *   workspace one device buffer of batch_info().workspace_bytes, 256-byte
 *             aligned; instance p uses its own part of it
 *   stream    hipStream_t or NULL
 * Stream-ordered and without host synchronisation: when a pointer differs
 * from the previous call's, the new pointer table is copied to the device on
 * `stream` (through one of four pinned host buffers; only a caller more than
 * four rebinds ahead of the device waits for the oldest copy), then the graph
 * is replayed on `stream`.  Bits are those of eval_and_diff per instance.
 * Calls (and batch_launch* calls) on different streams must not overlap: they
 * share the batch's pointer table and counters.
 */
int eval_and_diff_batch(mdpe_batch *batch, const double *const *coeff, const double *const *z,
                        double *const *value, double *const *grad, void *workspace, void *stream);
int batch_info(const mdpe_batch *batch, mdpe_batch_info *out);
/* rows int32[n_tasks][6]: {instance, kind (0 stage, 1 conv, 2 add, 3 gather),
 * counter threshold, count, first, queue (XCD)}, queues concatenated, each in
 * its claim order. */
int batch_tasks(const mdpe_batch *batch, int32_t *rows);
/* Host arrays [count] of device pointers, same meaning as in eval_and_diff;
 * copied to the device now (synchronously).  A captured graph reads them at
 * every replay, so they may change between launches. */
int batch_set_buffers(mdpe_batch *batch, const double *const *coeff, const double *const *z, double *const *value,
                      double *const *grad, void *const *workspace);
/* Enqueue [counter reset, persistent kernel] on stream. */
int batch_launch(mdpe_batch *batch, void *stream);
/* Same, as one hipGraph captured at the first call and replayed on stream. */
int batch_launch_graph(mdpe_batch *batch, void *stream);
/* Persistent workgroups to launch (0 = as many as are resident, the default);
 * for tuning and tests.  Must precede the first batch_launch_graph. */
int batch_set_grid(mdpe_batch *batch, int grid);
/* Wait for the device; report the persistent kernel's watchdog flag, or a
 * queue left undrained because no wavefront ran on its XCD. */
int batch_status(mdpe_batch *batch);
void batch_destroy(mdpe_batch *batch);

/* Release a plan (its device job arrays).  NULL is ignored. */
void plan_destroy(mdpe_plan *plan);

/* Message of the last failing call on this thread ("" if none). */
const char *last_error_string(void);

#ifdef __cplusplus
}
#endif
#endif /* MDPE_H */
