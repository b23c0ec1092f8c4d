/*
 * bound.h -- C ABI of the MI355X (gfx950) CROWN / alpha / beta bound-propagation library.
 *
 * The library computes the linear lower bound of Theorem 1 of the paper's Appendix B
 * (CROWN backward propagation through Linear / Conv2d layers and the ReLU relaxation
 * of Lemma 1), concretised over an input box by Theorem 2, for many instances
 * (inputs or branch-and-bound subdomains) at once.  It also evaluates the gradient of
 * that bound with respect to the free lower slopes alpha (Lemma 1) and the Lagrange
 * multipliers beta of ReLU split constraints, and performs the projected Adam step
 * that optimises them.
 *
 * Network: z_m = W_m h_{m-1} + b_m, h_m = ReLU(z_m) for m < L, h_0 = x (the
 * verification problem of Appendix B).  Neuron order inside a layer is C-major
 * (channel, row, column), as PyTorch flattens NCHW tensors.
 *
 * Conventions for every call:
 *  - All tensors are float32 (split indices int32, split signs int8), contiguous and
 *    row-major, and live in device memory unless a parameter says "host".
 *  - The caller owns every pointer it passes.  The library keeps none of them past the
 *    call, except the layer weights and biases handed to bound_init, which must stay
 *    valid until bound_destroy.
 *  - Work is enqueued asynchronously on the HIP stream passed in (NULL = the default
 *    stream).  Argument and shape errors are returned synchronously; a device-side
 *    failure is reported as BOUND_E_HIP by the call that observes it.
 *  - bound_last_error() returns a message for the last non-OK status of the calling
 *    thread.
 */
#ifndef BOUND_H
#define BOUND_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BOUND_OK = 0,
    BOUND_E_ARG = -1,    /* null / inconsistent argument */
    BOUND_E_SHAPE = -2,  /* layer chain or tensor shapes do not fit together */
    BOUND_E_NOMEM = -3,  /* request exceeds the workspace sized at bound_init */
    BOUND_E_HIP = -4,    /* a HIP runtime call failed */
    BOUND_E_STATE = -5,  /* call order violated (e.g. bound_grad with no saved pass) */
    BOUND_E_NUMERIC = -6 /* BOUND_OPT_CHECK found NaN / Inf in a product's output */
} bound_status;

enum { BOUND_LINEAR = 0, BOUND_CONV2D = 1 };

/* Pass flags. */
enum {
    BOUND_SAVE_FOR_GRAD = 1, /* keep the pre-relaxation coefficients for bound_grad */
    BOUND_NO_SLACK = 2,      /* report the raw bound without the FP32 rounding allowance */
    BOUND_BOTH_SIDES = 4,    /* also upper bounds: rows [spec; -spec], upper = -lower(-spec) */
    BOUND_RECOMPUTE = 8      /* with SAVE_FOR_GRAD: checkpointed layer recomputation (below) */
};

typedef struct bound_net bound_net; /* opaque, owned by the library */

/* One layer z = W h + b.  A ReLU follows every layer except the last.
 * Linear : weight [out_c, in_c] (in_c = in_c*in_h*in_w of a conv-shaped input,
 *          C-major), bias [out_c]; in_h = in_w = out_h = out_w = 1 unless the
 *          input is the flattened output of a conv layer (then in_c/in_h/in_w give
 *          that shape and the weight has in_c*in_h*in_w columns).
 * Conv2d : weight [out_c, in_c, kh, kw], bias [out_c]; square kernel (kh == kw),
 *          symmetric zero padding `pad`, stride 1 or 2,
 *          out_h = (in_h + 2 pad - kh) / stride + 1 (likewise out_w),
 *          kh * kw * in_c <= 1024 and kh * kw * out_c <= 1024. */
typedef struct {
    int32_t kind;
    int32_t in_c, in_h, in_w;
    int32_t out_c, out_h, out_w;
    int32_t kh, kw, stride, pad;
    const float *weight;
    const float *bias;
} bound_layer;

/* One bound pass: lower bounds of spec rows applied to z_target, for n_inst instances.
 * Let d_m = width of z_m, n_relu = d_1 + ... + d_{L-1}, relu_off(m) = d_1+...+d_{m-1}.
 *
 * spec      [n_inst, rows, d_target] coefficient rows (Theorem 1's A(L), generalised
 *           from I to a specification matrix), or NULL for the identity: rows must
 *           equal d_target and row r bounds neuron r of z_target (intermediate bounds).
 * lo, hi    [n_bounds, n_relu] pre-activation bounds (l, u of Lemma 1) of the ReLU
 *           layers; only layers 1 .. target-1 are read.
 * bound_of  [n_inst] row of lo/hi used by each instance (subdomains of one root share
 *           it), or NULL: instance i uses row i.  Rows outside [0, n_bounds) are
 *           clamped into it (the caller's arrays are never read out of range).
 * alpha     [n_inst, n_relu] lower relaxation slopes in [0, 1] (read at unstable
 *           neurons only), or NULL for the rule alpha = 1 if u >= -l else 0.
 * split_off [n_inst + 1], split_idx [nnz], split_sign [nnz]: CSR list of split
 *           constraints sign * z_j >= 0 (j a global ReLU index: relu_off(m) + neuron).
 *           A split clamps l (sign +1) or u (sign -1) to 0; an instance whose clamped
 *           box is empty gets lower = +inf (upper = -inf).  A neuron may appear in
 *           several entries of one instance: the clamps compose, every entry has its own
 *           multiplier, and their terms add.  Entries whose neuron lies outside layers
 *           1 .. target-1 are ignored.  All three NULL and nnz = 0 when there are no
 *           splits; nnz < 2^24.
 * beta      [nnz, rows] Lagrange multipliers (>= 0) of the splits, or NULL (= 0):
 *           entry q adds -beta[q, r] * sign[q] to row r's coefficient of its split
 *           neuron (after the relaxation of Lemma 1).
 * x_lo,x_hi [n_inst, d_0] the input box.  NULL: do not concretise; the pass then
 *           writes the coefficient form (bound_out.coeff / offset / offset_mag).
 * flags     BOUND_SAVE_FOR_GRAD (requires an explicit spec and n_inst * rows (x2 with
 *           BOTH_SIDES) <= max_save_rows), BOUND_NO_SLACK, BOUND_BOTH_SIDES (not with
 *           beta), BOUND_RECOMPUTE (with SAVE_FOR_GRAD, no early stop): instead of the
 *           pre-relaxation coefficients of every layer (kept at the unstable neurons),
 *           the pass keeps the coefficient rows Lambda_t entering every c-th product
 *           from the top (c = ceil(sqrt(target - 1))); bound_grad recomputes each
 *           segment's products from its checkpoint before the reverse pass crosses it
 *           (about one more backward pass of work; memory c dense rows + checkpoints
 *           instead of every layer's unstable coefficients -- the smaller footprint for
 *           deep chains).  The gradient is the same.
 * stop_layer, stop_mode  propagation early stop (Appendix B.2, the early-stop
 *           algorithm): 0 = propagate to the input and concretise over the input box.
 *           1 <= stop_layer < target: the backward search ends at the early-stop node
 *           of ReLU layer s = stop_layer and the bound is concretised over that node's
 *           box taken from lo / hi (after split clamping):
 *             BOUND_STOP_RELU   the node is the ReLU of layer s: its relaxation is not
 *                               applied; the box is [ReLU(l_s), ReLU(u_s)];
 *             BOUND_STOP_LINEAR the node is the linear layer producing z_s: the ReLU of
 *                               layer s is relaxed (alpha, beta) first; the box is
 *                               [l_s, u_s].
 *           x_lo / x_hi are still required (their values are not used). */
typedef struct {
    int32_t n_inst;
    int32_t rows;
    int32_t target;
    int32_t n_bounds;
    const float *spec;
    const float *lo;
    const float *hi;
    const int32_t *bound_of;
    const float *alpha;
    const int32_t *split_off;
    const int32_t *split_idx;
    const int8_t *split_sign;
    int32_t nnz;
    const float *beta;
    const float *x_lo;
    const float *x_hi;
    int32_t flags;
    int32_t stop_layer;
    int32_t stop_mode;
} bound_pass;

enum { BOUND_STOP_RELU = 1, BOUND_STOP_LINEAR = 2 };

/* Outputs of a pass.
 * lower  [n_inst, ld] lower bound of spec row r at lower[i*ld + r];
 * upper  same layout (BOTH_SIDES only, else may be NULL);
 * ld     row stride of lower/upper in elements (0 = rows);
 * coeff  [n_inst*rows(*2 with BOTH_SIDES), d_0] coefficients W~(1) on x (Theorem 1),
 * offset [n_inst*rows(*2)] the offsets b~(1), offset_mag [...] the sum of |terms| of
 *        b~(1) (for the rounding allowance) -- written only when x_lo == NULL;
 * best   [n_inst, ld] or NULL: updated to max(best, lower) (every alpha in [0, 1] and
 *        beta >= 0 gives a valid bound, so the best over optimisation steps is kept);
 * pass_id host pointer or NULL: a SAVE_FOR_GRAD pass writes its id (1, 2, ... per
 *        handle), which bound_grad can be asked to check;
 * best_upper [n_inst, ld] or NULL (BOTH_SIDES): updated to min(best_upper, upper). */
typedef struct {
    float *lower;
    float *upper;
    int64_t ld;
    float *coeff;
    float *offset;
    float *offset_mag;
    float *best;
    int64_t *pass_id;
    float *best_upper;
} bound_out;

/* Create a network handle for a chain of 1 <= n_layers <= 129 layers.  Validates the
 * layer chain, packs the weights for the gfx950 kernels and allocates the workspace:
 *  max_inst      most instances in one pass;
 *  max_rows      most coefficient rows (instances x rows, x2 with BOTH_SIDES) held at
 *                once; larger passes without SAVE_FOR_GRAD are processed in chunks;
 *  max_save_rows most rows of a SAVE_FOR_GRAD pass (0 = no gradient support).
 * stream is used for the packing kernels; the call returns after they finish. */
bound_status bound_init(const bound_layer *layers, int32_t n_layers, int32_t max_inst,
                        int64_t max_rows, int64_t max_save_rows, void *stream,
                        bound_net **out);

/* Widths d_0 .. d_L into d (host, n_layers + 1 entries; NULL to query n_layers first) and
 * n_relu into *n_relu. */
bound_status bound_dims(const bound_net *net, int32_t *n_layers, int32_t *d, int32_t *n_relu);

/* Backward bound pass (Theorem 1 with Lemma 1's relaxation, the split multipliers,
 * and Theorem 2's concretisation fused into the last layer).  With
 * BOUND_SAVE_FOR_GRAD the state needed by bound_grad is kept in the workspace until
 * the next bound_backward call on the same handle (any pass invalidates it). */
bound_status bound_backward(bound_net *net, const bound_pass *pass, const bound_out *out,
                            void *stream);

/* Search-integrated (empirical) pre-activation bounds (Section 3.2, approach 2): the
 * network is evaluated on per_sub sample inputs of each of n_sub subdomains and every
 * pre-activation z_1 .. z_{L-1} gets the minimum / maximum over its subdomain's samples.
 * x   [n_sub * per_sub, d_0] sample inputs (subdomain-major);
 * lo, hi [n_sub, n_relu] outputs in the lo/hi layout of bound_pass (both or neither);
 * out [n_sub * per_sub, d_L] network outputs z_L, or NULL.
 * These bounds hold for the samples, not for every point of the subdomain (the paper
 * accepts that for planning); they are meant as the early-stop node's box.
 * per_sub must not exceed max_rows; larger n_sub are processed in chunks.  Invalidates
 * the state kept for bound_grad. */
bound_status bound_sample_bounds(bound_net *net, int32_t n_sub, int32_t per_sub, const float *x,
                                 float *lo, float *hi, float *out, void *stream);

/* bound_sample_bounds over more samples of the same subdomains (the later rounds of a
 * search): lo and hi must hold bounds already and take lo = min(lo, samples' min),
 * hi = max(hi, samples' max).  Arguments and errors as bound_sample_bounds. */
bound_status bound_sample_bounds_merge(bound_net *net, int32_t n_sub, int32_t per_sub,
                                       const float *x, float *lo, float *hi, float *out,
                                       void *stream);

/* Standalone concretisation (Theorem 2 for a box) of coefficient rows:
 * lower[i*rows + r] = coeff[i,r,:] . c - |coeff[i,r,:]| . rad + offset[i,r]
 *                     - (unless BOUND_NO_SLACK) 64 * 2^-24 * (|coeff| . (|c| + rad)
 *                                                           + offset_mag[i,r])
 * with c = (x_lo + x_hi) / 2, rad = (x_hi - x_lo) / 2 per instance i.
 * coeff [n_inst, rows, d0]; offset, offset_mag [n_inst, rows] (offset_mag may be
 * NULL = 0); x_lo, x_hi [n_inst, d0]; lower [n_inst, rows]. */
bound_status bound_concretize(int32_t n_inst, int32_t rows, int32_t d0, const float *coeff,
                              const float *offset, const float *offset_mag,
                              const float *x_lo, const float *x_hi, int32_t flags,
                              float *lower, void *stream);

/* Gradient of sum_{i,r} grad_lower[i,r] * lower_raw[i,r] of the last SAVE_FOR_GRAD
 * pass (the raw bound, i.e. without the rounding allowance; intermediate bounds held
 * fixed) with respect to alpha and beta -- the reverse mode of Theorem 1's recursion and
 * Theorem 2's concretisation:
 * grad_lower [n_inst, rows] (rows = the pass's rows, twice them with BOTH_SIDES: the first
 * half weights the lower bounds, the second the lower bounds of -spec, i.e. -upper);
 * grad_alpha [n_inst, n_relu] (overwritten; zero outside unstable, unsplit neurons of
 * layers 1 .. target-1), grad_beta [nnz, rows] (overwritten; may be NULL): entry q of
 * row r gets -sign[q] * (the derivative with respect to its neuron's coefficient), so
 * repeated entries of one neuron get the same value up to their signs.
 * Infeasible instances get zero gradients.
 * pass_id: 0 = the last SAVE_FOR_GRAD pass, else the id that pass wrote to
 * bound_out.pass_id; BOUND_E_STATE when that pass is no longer the saved one (any later
 * bound_backward or bound_sample_bounds call invalidates it).  n_inst, rows and nnz state
 * the caller's buffer shapes; BOUND_E_SHAPE unless they are the saved pass's (nnz is
 * checked only when grad_beta is given). */
bound_status bound_grad(bound_net *net, int64_t pass_id, int32_t n_inst, int32_t rows,
                        int32_t nnz, const float *grad_lower, float *grad_alpha,
                        float *grad_beta, void *stream);

/* One projected Adam step on alpha (the form of bound_adam below) fused with
 * bound_grad's alpha-gradient (the alpha-CROWN optimisation of the relaxation slopes):
 * bound_grad's arguments and checks, grad_beta as there, but instead of writing a dense
 * gradient the library steps alpha itself at the entries the bound depends on -- the
 * unstable, unsplit neurons of layers 1 .. target-1 of each instance -- as soon as each
 * layer's gradient is formed, so the gradient never goes to memory and the other
 * entries are not touched.
 * alpha [n_inst, n_relu] (bound_pass.alpha's layout), updated in place.
 * m, v  [n_inst, n_relu] Adam moments in slot order: entry (i, off_l + s) belongs to the
 *       s-th unstable neuron (internal order: channel fastest, then pixel) of ReLU layer l
 *       under instance i's intermediate bounds, off_l the layer's offset in n_relu.  The
 *       order depends only on those bounds, so the moments stay valid across the steps of
 *       an optimisation with fixed intermediate bounds and splits; zero them when those
 *       change.
 * With the moments zero at the start, alpha after each step equals that of bound_grad
 * followed by bound_adam on the dense gradient, for alpha within [clip_lo, clip_hi]. */
typedef struct {
    float *alpha;
    float *m, *v;
    int32_t step;   /* 1-based */
    float lr, b1, b2, eps, grad_scale, clip_lo, clip_hi;
} bound_adam_step;
bound_status bound_grad_adam(bound_net *net, int64_t pass_id, int32_t n_inst, int32_t rows,
                             int32_t nnz, const float *grad_lower,
                             const bound_adam_step *alpha_step, float *grad_beta, void *stream);

/* One Adam step (PyTorch's bias-corrected form) on n parameters, minimising a loss
 * whose gradient is grad_scale * grad, then clipping to [clip_lo, clip_hi]:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps);  p = clip(p).
 * step is 1-based.  Used to maximise the bound (grad_scale = -1) over alpha in [0,1]
 * and beta in [0, inf). */
bound_status bound_adam(int64_t n, float *param, const float *grad, float *m, float *v,
                        int32_t step, float lr, float b1, float b2, float eps,
                        float grad_scale, float clip_lo, float clip_hi, void *stream);

/* Kernel selection: BOUND_OPT_GEMM_ONLY runs every product as an implicit GEMM (the
 * LDS-tiled direct-convolution kernels are otherwise used where the layer geometry fits
 * them).  BOUND_OPT_DIRECT_DMA makes the direct-convolution kernels of products that
 * bound_autotune has not planned stage their tiles by LDS DMA instead of through
 * registers.  All variants compute the same bound; the options exist to test and
 * compare them.  BOUND_OPT_CHECK (debugging): after every product of bound_backward and
 * bound_grad the library counts NaN and Inf values in the product's output (and in the
 * gradient it returns), waits for the count, and returns BOUND_E_NUMERIC naming the
 * product if there are any; the calls become synchronous.  Not applied while the stream
 * is being captured.  The environment variable BOUND_DEBUG=1 sets it at bound_init. */
/* BOUND_OPT_DETERMINISTIC: the row sums of the products (the bias and intercept terms
 * of Theorem 1, the concretised bound of Theorem 2 and the rounding-allowance
 * magnitudes) are formed without float atomics: every tile stores its partial sums in
 * a slot of its own and the slots are added in a fixed order, so bound_backward's
 * results are bitwise reproducible run to run (the gradient already is); slower.  The
 * slots take max_rows x (output pixels x ceil(channels / 16), at most over the layers)
 * x 8 bytes of device memory, allocated here on first use (BOUND_E_NOMEM if that
 * fails). */
enum { BOUND_OPT_GEMM_ONLY = 1, BOUND_OPT_DIRECT_DMA = 2, BOUND_OPT_CHECK = 4,
       BOUND_OPT_DETERMINISTIC = 8 };
bound_status bound_set_options(bound_net *net, int32_t options);

/* Kernel autotuning: runs the given pass (and, if grad_lower is not NULL and the pass
 * has SAVE_FOR_GRAD, its gradient) once in tuning mode -- every valid kernel variant of
 * every product (direct-convolution channel chunk, implicit-GEMM tile shape) is timed
 * on the live data and the fastest is kept for that product on this handle -- then runs
 * the pass again normally, so `out` and the saved state are those of a normal pass.
 * Synchronises the stream; must not be called while the stream is being captured.
 * bound_autotune_report copies the timing log (NUL-terminated, truncated to cap) and
 * returns its full length. */
bound_status bound_autotune(bound_net *net, const bound_pass *pass, const bound_out *out,
                            const float *grad_lower, void *stream);
int32_t bound_autotune_report(const bound_net *net, char *buf, int32_t cap);

/* Pins the kernel plan of one product, as bound_autotune would record it: product is
 * 'R' (backward relaxation step through layer `layer`), 'C' (the concretising step),
 * 'A' (adjoint step) or 'F' (forward step of sample rows); layer is 1-based; path 1 =
 * direct convolution (cfg: -1 staging through registers, 1 by LDS DMA, 2 / 3 the same
 * with 16x16 MFMA tiles for 32 output channels; cc: channel chunk, 0 = largest that
 * fits), path 2 = implicit GEMM (cfg: tile shape 0..10; 9 and 10 stage dense products by LDS DMA), path 0 = automatic.  A plan the layer cannot run falls back to the implicit GEMM at launch.
 * Lets a run reuse the plans of an earlier tuned run (the timing log's chosen lines). */
bound_status bound_set_plan(bound_net *net, char product, int32_t layer, int32_t path,
                            int32_t cfg, int32_t cc);

/* Per-launch timing: with enable != 0 every kernel the handle launches is bracketed by
 * HIP events recorded on its own stream (not while the stream is being captured).
 * bound_profile_read waits for the recorded events, adds their durations per kernel
 * label since the last read, and fills up to cap entries: names (cap x 48 chars,
 * NUL-terminated), total_ms and count; returns the number of labels (or < 0 on error). */
bound_status bound_profile(bound_net *net, int32_t enable);
int32_t bound_profile_read(bound_net *net, int32_t cap, char *names, double *total_ms,
                           int32_t *count);

void bound_destroy(bound_net *net);
const char *bound_last_error(void);

/* ------------------------------------------------------------------------------------
 * Branch and bound over input boxes (the planning loop of Algorithms 1-2 and the
 * branching heuristics of Section 3.1): the per-iteration steps around the bound pass.
 * A subdomain is a box [lo, hi] of dim coordinates with a lower bound f_lo of the
 * objective (bound_backward on the box) and an upper bound f_hi (the best objective its
 * search found).  Random numbers are inputs (uniforms in [0, 1)).  Ties are always
 * broken toward the lower index; -0.0 counts as +0.0 and NaN as +inf in comparisons.
 * ------------------------------------------------------------------------------------ */
typedef struct bound_bab bound_bab;

/* Workspace for up to max_dom subdomains of dim coordinates and up to max_samples
 * (<= 2048) search samples per subdomain.  Allocates device memory once. */
bound_status bound_bab_init(int32_t max_dom, int32_t dim, int32_t max_samples, bound_bab **out);
void bound_bab_destroy(bound_bab *bab);

/* batch_pick_out (Section 3.1, Eq. lf_pick): with n = min(n_pick, n_dom) and
 * n1 = floor(eta * n) (host double precision), picked[0 .. n1) are the n1 subdomains
 * with the smallest f_hi; picked[n1 .. n) are drawn without replacement from the
 * others with probability proportional to exp(-s_i / temperature), s_i = f_lo min-max
 * scaled over those others (0 if all equal), by the Gumbel-top-k rule on the supplied
 * standard Gumbel variates g_i (-log(-log U) of uniforms U): in ascending order of the
 * key s_i * fl(1 / temperature) - g_i, every operation rounded in FP32 (finite g;
 * ties toward the lower index); subdomains with non-finite f_lo come last.  rest
 * [n_dom - n] lists the others in ascending order.  f_lo, f_hi, g [n_dom];
 * temperature > 0; 0 <= eta <= 1; n_dom <= max_dom. */
bound_status bound_bab_pick_out(bound_bab *bab, int32_t n_dom, const float *f_lo,
                                const float *f_hi, const float *g, int32_t n_pick, float eta,
                                float temperature, int32_t *picked, int32_t *rest, void *stream);

/* batch_search, sampling: samples[i, m, :] = lo[i] + (hi[i] - lo[i]) * U[i, m, :], each
 * operation rounded separately in FP32.  lo, hi [n, dim]; U, samples [n, M, dim]. */
bound_status bound_bab_samples(bound_bab *bab, int32_t n, int32_t M, const float *lo,
                               const float *hi, const float *U, float *samples, void *stream);

/* batch_search, summary: per subdomain the smallest objective over its M samples
 * (f_hi [n]) and its k best samples in ascending order of objective (top [n, k, dim];
 * top[i, 0] is the best sample u~).  values [n, M] (the objective at the samples),
 * samples [n, M, dim]; 1 <= k <= M <= max_samples. */
bound_status bound_bab_search_summary(bound_bab *bab, int32_t n, int32_t M, const float *values,
                                      const float *samples, int32_t k, float *f_hi, float *top,
                                      void *stream);

/* batch_search by CEM (Section 3.3: the paper's search is CEM; it gives no details, so
 * this is the textbook cross-entropy method, one Gaussian per box with per-coordinate
 * mean mu and deviation sigma).  Each round: bound_bab_cem_samples, the objective at
 * the samples (bound_sample_bounds), bound_bab_cem_refit; the rounds' samples and
 * values gathered in archives go to bound_bab_search_summary.
 *
 * Start: mu[i] = u[i / u_div] when lo[i] <= that point <= hi[i] in every coordinate
 * (the best sample of a split box starts the search of the child that holds it), else
 * (lo[i] + hi[i]) * 0.5; sigma[i] = (hi[i] - lo[i]) * 0.5; FP32.  lo, hi, mu, sigma
 * [n, dim]; u [*, dim] or NULL (every mu the centre); u_div >= 1. */
bound_status bound_bab_cem_start(bound_bab *bab, int32_t n, const float *lo, const float *hi,
                                 const float *u, int32_t u_div, float *mu, float *sigma,
                                 void *stream);

/* Round samples: samples[i, m, :] = min(max(mu[i] + sigma[i] * Z[i, m, :], lo[i]), hi[i])
 * with the product and the sum each rounded in FP32 (finite inputs).  Z [n, M, dim]
 * standard normals supplied by the caller; samples [n, M, dim].  With archive != NULL
 * the samples are also written to archive[i, a0 + m, :] of an [n, ld, dim] buffer
 * (0 <= a0, a0 + M <= ld). */
bound_status bound_bab_cem_samples(bound_bab *bab, int32_t n, int32_t M, const float *lo,
                                   const float *hi, const float *mu, const float *sigma,
                                   const float *Z, float *samples, float *archive, int32_t ld,
                                   int32_t a0, void *stream);

/* Round refit: the n_elite samples of each box with the smallest values (ascending; ties
 * toward the lower index; NaN as +inf) give, per coordinate, mu[i] = their mean and
 * sigma[i] = sqrt(mean of (x - mu[i])^2) + jitter, the sums taken in that order in
 * FP32.  values [n, M]; samples [n, M, dim]; 1 <= n_elite <= M <= max_samples;
 * jitter >= 0.  With archive_values != NULL values[i, m] are also copied to
 * archive_values[i * ld + a0 + m] (0 <= a0, a0 + M <= ld). */
bound_status bound_bab_cem_refit(bound_bab *bab, int32_t n, int32_t M, const float *values,
                                 const float *samples, int32_t n_elite, float jitter, float *mu,
                                 float *sigma, float *archive_values, int32_t ld, int32_t a0,
                                 void *stream);

/* batch_split (Section 3.1): for each subdomain i the dimension j* maximising
 * (hi_j - lo_j) * |n_lo_j - n_up_j| over its k top samples (a sample is on the lower side
 * iff u_j <= mid_j, mid = (lo + hi) * 0.5 in FP32; if every score is 0, the widest
 * dimension), then the two halves: child 2i = [lo, hi with hi_j* = mid], child 2i + 1 =
 * [lo with lo_j* = mid, hi].  lo, hi [n, dim]; top [n, k, dim]; child_lo, child_hi
 * [2n, dim]; split_dim [n] (may be NULL). */
bound_status bound_bab_split(bound_bab *bab, int32_t n, const float *lo, const float *hi,
                             const float *top, int32_t k, float *child_lo, float *child_hi,
                             int32_t *split_dim, void *stream);

/* The best solution so far: if min_i f_hi[i] < *best (device scalar), *best takes that
 * value and u_best [dim] the sample top[i*, 0] of its subdomain i*.  f_hi [n];
 * top [n, k, dim]. */
bound_status bound_bab_update_best(bound_bab *bab, int32_t n, const float *f_hi,
                                   const float *top, int32_t k, float *best, float *u_best,
                                   void *stream);

/* Pruner: keep [*n_keep] = the indices i (ascending) with f_lo[i] <= *best, i.e. the
 * subdomains that may still hold a better solution (a subdomain is pruned iff
 * f_lo > best).  f_lo [n]; best and n_keep are device scalars; keep [n]. */
bound_status bound_bab_prune(bound_bab *bab, int32_t n, const float *f_lo, const float *best,
                             int32_t *keep, int32_t *n_keep, void *stream);

/* The pruner of bound_bab_prune (same arguments, same output, without a bound_bab
 * handle) for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  It allocates nothing; its
 * scratch (per-block counts of the stable compaction) is a fixed 16 KiB array in the
 * library that each GPU holds until the process ends.  0 <= n <= 4194304
 * (BOUND_E_ARG otherwise).  Every call on one GPU shares that GPU's scratch: calls that
 * overlap on one GPU (different streams or threads without ordering) race. */
bound_status bound_bab_prune_noalloc(int32_t n, const float *f_lo, const float *best,
                                     int32_t *keep, int32_t *n_keep, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* BOUND_H */
