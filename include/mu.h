/*
 * mu.h -- C ABI of the MI355X (gfx950) muSR chi^2 / Poisson-likelihood library.
 *
 * The library evaluates, on the GPU, the cost that the fit of a set of
 * positron histograms minimises (Locans et al., "Real-Time Computation of
 * Parameter Fitting and Image Reconstruction Using Graphical Processing
 * Units", Sec. 4):
 *
 *   N^j(t, P) = N0^j e^(-t/tau_mu) [1 + A^j(p^j, t)] + Nbkg^j        (Eq. 1)
 *   chi^2(P)  = sum_j sum_n (d_n^j - N^j(t_n, P))^2 / v_n^j           (Eq. 2)
 *   L(P)      = 2 sum_j sum_n [(N - d) + d ln(d / N)]                  (Eq. 3)
 *
 * with t_n = (n - t0_bin) dt (Eq. 1 text; t0_bin is 0 in the paper's
 * statement), v = d for d > 0 and v = 1 for an empty bin (Eq. 2 gives
 * d_err = sqrt(d); the empty-bin weight is this library's reading), and L
 * minimised (it is the Poisson likelihood-ratio statistic; Eq. 3's "maximised"
 * is read as a sign slip).  For d = 0 the likelihood term is 2N; for N <= 0 < d
 * it is +inf.
 *
 * A^j(t) is a theory program: a sum of up to MU_MAX_TERMS terms, each
 * coef * amp * prod of up to MU_MAX_FACTORS_PER_TERM primitives (Listing 2:
 * se, ge, sg, stg; Listing 3: tf).  Every scalar argument is a reference that
 * goes through the map row of the histogram: p[map[row][slot]], or the
 * function array f[map[row][slot]] with f = F p + f0, or a literal.  This is
 * the parameter / function / map indirection of Sec. 4.2.1 and Listing 3.
 * Units: t in us, rates in 1/us, frequencies in MHz, phases in radians.
 *
 * Histograms are copied to the device once (mu_data_create) and stay there
 * for the whole fit (Sec. 4.2: data sets do not change during the fit).
 *
 * Conventions of every entry point:
 *   - every function returns a mu_status; nothing throws or aborts;
 *   - on error no output is written and mu_ctx_last_error() names the cause;
 *   - the caller owns every input and output buffer; *_create deep-copies
 *     its inputs; a handle lives until its *_destroy;
 *   - mem == MU_MEM_HOST: params and outputs are host pointers and the call
 *     returns after the results are written (it synchronises the stream);
 *     mem == MU_MEM_DEVICE: they are device pointers on the context's device,
 *     the call only enqueues work on the context stream and returns;
 *   - one host thread at a time per context;
 *   - the same inputs give bitwise identical outputs (fixed-order reductions).
 */
#ifndef MU_H
#define MU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MU_ABI_VERSION 1
#define MU_MAX_TERMS 4
#define MU_MAX_FACTORS_PER_TERM 3
#define MU_MAX_PAR 1024

typedef struct mu_ctx mu_ctx;
typedef struct mu_data mu_data;
typedef struct mu_theory mu_theory;
typedef struct mu_seeder mu_seeder;

typedef enum {
  MU_OK = 0,
  MU_E_ARG = 1,          /* invalid argument: nothing was done */
  MU_E_NODEVICE = 2,     /* no usable GPU (or MU_FORCE_NODEVICE is set) */
  MU_E_NOMEM = 3,        /* device or host allocation failed */
  MU_E_DEVICE = 4,       /* a HIP call failed */
  MU_E_UNSUPPORTED = 5,  /* valid request outside the library's limits */
  MU_E_STATE = 6         /* handle in the wrong state (e.g. live children) */
} mu_status;

typedef enum { MU_COST_CHI2 = 0, MU_COST_POISSON = 1 } mu_cost;
enum { MU_MEM_HOST = 0, MU_MEM_DEVICE = 1 };

int mu_abi_version(void);
const char *mu_status_string(mu_status s);

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t on
 * that device that every call enqueues on (NULL: the context creates its own
 * default-priority stream).  flags: reserved, pass 0.  Returns MU_E_NODEVICE
 * when no device is visible or the environment variable MU_FORCE_NODEVICE is
 * set to a non-empty value other than "0". */
mu_status mu_ctx_create(int device, void *hip_stream, unsigned flags, mu_ctx **out);
/* MU_E_STATE (and nothing freed) while data, theories or seeders created on
 * this context are alive. */
mu_status mu_ctx_destroy(mu_ctx *ctx);
const char *mu_ctx_last_error(const mu_ctx *ctx);
mu_status mu_ctx_synchronize(mu_ctx *ctx);

/* -------------------------------------------------------------- histograms */

/* One positron histogram (Sec. 4.1): counts d_n for n = 0 .. n_bins-1, bin
 * width dt > 0 (us), time origin t0_bin (t_n = (n - t0_bin) dt), inclusive fit
 * range [first, last], and the map row that selects its parameters P^j.
 * Counts must be finite and >= 0.  They are stored as 32-bit unsigned
 * integers (8 d, exact) when every value in every fit range is an integer
 * below 2^29, else as FP64. */
typedef struct {
  const double *counts; /* host, n_bins values */
  int64_t n_bins;
  double dt;
  double t0_bin;
  int64_t first, last;
  int32_t map_row;
  int32_t reserved;
} mu_histo;

/* Check histogram descriptors without a device (same rules as
 * mu_data_create).  Writes a message into msg (may be NULL). */
mu_status mu_histo_check(const mu_histo *h, int32_t n_histo, char *msg, int32_t msg_len);
/* Upload n_histo histograms once; only the fit ranges are copied. */
mu_status mu_data_create(mu_ctx *ctx, const mu_histo *h, int32_t n_histo, mu_data **out);
mu_status mu_data_destroy(mu_data *data);
int64_t mu_data_bins(const mu_data *data);     /* total fit-range bins, -1 on NULL */
int32_t mu_data_histos(const mu_data *data);   /* number of histograms, -1 on NULL */
int32_t mu_data_is_f64(const mu_data *data);   /* 1 if counts are stored in FP64 */

/* ------------------------------------------------------------------ theory */

typedef enum { MU_SE = 0, MU_GE = 1, MU_SG = 2, MU_STG = 3, MU_TF = 4 } mu_prim;
/* Primitives and their argument lists (Listing 2, Listing 3):
 *   MU_SE  (lambda)        exp(-lambda t)
 *   MU_GE  (lambda, beta)  exp(-(lambda t)^beta)       (t >= 0; beta > 0)
 *   MU_SG  (sigma)         exp(-(sigma t)^2 / 2)
 *   MU_STG (sigma)         1/3 + 2/3 (1 - (sigma t)^2) exp(-(sigma t)^2 / 2)
 *   MU_TF  (phi, nu)       cos(2 pi nu t + phi)                               */
typedef enum { MU_REF_PAR = 0, MU_REF_FUN = 1, MU_REF_LIT = 2 } mu_ref_kind;
typedef struct {
  int32_t kind;    /* mu_ref_kind */
  int32_t slot;    /* map column for MU_REF_PAR / MU_REF_FUN */
  double literal;  /* value for MU_REF_LIT */
} mu_ref;
typedef struct {
  int32_t prim;    /* mu_prim */
  int32_t reserved;
  mu_ref arg[2];   /* only the first nargs(prim) are read */
} mu_factor;
typedef struct {
  double coef;                 /* literal coefficient */
  mu_ref amp;                  /* amplitude reference */
  int32_t first_factor;        /* index into the factor array */
  int32_t n_factors;           /* 0 .. MU_MAX_FACTORS_PER_TERM */
} mu_term;
typedef struct {
  double tau_mu;               /* muon lifetime in us, > 0 */
  mu_ref n0, nbkg;             /* N0^j and Nbkg^j */
  const mu_term *terms;
  int32_t n_terms;             /* 0 .. MU_MAX_TERMS */
  const mu_factor *factors;
  int32_t n_factors;
  const int32_t *map;          /* [n_rows][n_slots], row-major */
  int32_t n_rows, n_slots;
  const double *F;             /* [n_fun][n_par] or NULL when n_fun == 0 */
  const double *f0;            /* [n_fun] or NULL when n_fun == 0 */
  int32_t n_fun;
  int32_t n_par;               /* 1 .. MU_MAX_PAR */
} mu_theory_desc;

/* Validate a theory without a device.  MU_E_ARG for: n_par outside
 * [1, MU_MAX_PAR]; tau_mu <= 0 or non-finite; an unknown primitive or
 * reference kind; a slot outside [0, n_slots); a map entry outside [0, n_par)
 * for a parameter reference or outside [0, n_fun) for a function reference;
 * a literal beta <= 0; factor ranges that overlap or leave the array.
 * MU_E_UNSUPPORTED for more than MU_MAX_TERMS terms or
 * MU_MAX_FACTORS_PER_TERM factors in a term. */
mu_status mu_theory_check(const mu_theory_desc *d, char *msg, int32_t msg_len);
mu_status mu_theory_create(mu_ctx *ctx, const mu_theory_desc *d, mu_theory **out);
mu_status mu_theory_destroy(mu_theory *th);
int32_t mu_theory_npar(const mu_theory *th);

/* ------------------------------------------------- run-time compiled theory */

/* A theory whose asymmetry A(t) is written as an expression and compiled at
 * run time (the paper's user functions, Sec. 4.2.1 and Listing 3, there a C
 * function compiled when the fit starts; here hipRTC for gfx950).  The model
 * stays N = N0 e^(-t/tau_mu) (1 + A(t)) + Nbkg (Eq. 1) with N0 and Nbkg
 * references as for theory programs.  Grammar (whitespace ignored):
 *   expr    := term (("+" | "-") term)*
 *   term    := unary (("*" | "/") unary)*
 *   unary   := ("-" | "+") unary | power
 *   power   := primary ("^" unary)?
 *   primary := number | "t" | "pi" | "p[" slot "]" | "f[" slot "]"
 *            | name "(" expr ("," expr)* ")" | "(" expr ")"
 * p[i] is the parameter at slot i of the histogram's map row, f[i] the
 * function value at slot i (f = F p + f0); names: exp, log, sqrt, sin, cos,
 * pow(a, b), j0 (Bessel J0), the primitives se(lambda), ge(lambda, beta),
 * sg(sigma), stg(sigma), tf(phi, nu) (as MU_SE .. MU_TF), and
 *   sekt(a)        1/3 + 2/3 (1 - a t) e^(-a t)   (static Lorentzian Kubo-Toyabe)
 *   ab(sigma, g)   exp(-(sigma/g)^2 (e^(-g t) - 1 + g t))   (Abragam)
 *   b(phi, nu)     J0(2 pi nu t + phi)   (Bessel precession)
 *   ifld(alpha, phi, nu, lT, lL)   alpha cos(2 pi nu t + phi) e^(-lT t) + (1 - alpha) e^(-lL t)
 *   ibsl(alpha, phi, nu, lT, lL)   the same with J0 in place of cos
 * with t implicit in every primitive.  At most
 * 28 distinct references.  Each bin is evaluated directly (no recurrences),
 * with the derivatives in the references carried as dual numbers, so costs,
 * gradients, model values, batched launches, fits and mu_hesse all accept
 * such a theory (the allocation-free entry point too, since compilation
 * happens at creation).  Division by zero, log of a non-positive value and
 * the like give non-finite costs, as non-finite parameters do. */
typedef struct {
  double tau_mu;           /* muon lifetime in us, > 0 */
  mu_ref n0, nbkg;         /* N0^j and Nbkg^j */
  const char *asymmetry;   /* A(t), the grammar above */
  const int32_t *map;      /* [n_rows][n_slots] */
  int32_t n_rows, n_slots;
  const double *F;         /* [n_fun][n_par] or NULL when n_fun == 0 */
  const double *f0;        /* [n_fun] or NULL when n_fun == 0 */
  int32_t n_fun;
  int32_t n_par;           /* 1 .. MU_MAX_PAR */
} mu_expr_theory_desc;

/* Parse and validate without a device (the map rules of mu_theory_check for
 * N0, Nbkg and every reference of the expression).  MU_E_ARG for a syntax
 * error (the message gives the offset), an unknown name, a wrong argument
 * count or a bad reference; MU_E_UNSUPPORTED for more than 28 references. */
mu_status mu_theory_check_expr(const mu_expr_theory_desc *d, char *msg, int32_t msg_len);
/* The HIP source that would be compiled (*needed: its size with the final
 * zero; buf may be NULL). */
mu_status mu_theory_expr_source(const mu_expr_theory_desc *d, char *buf, int64_t buf_len, int64_t *needed);
/* Compile with hipRTC for gfx950 without a device (no context): MU_E_ARG
 * with the compiler's log in msg if the generated source does not build. */
mu_status mu_theory_compile_check(const mu_expr_theory_desc *d, char *msg, int32_t msg_len);
/* Create the theory: parse, compile (once per context and distinct source;
 * the module is kept until mu_ctx_destroy) and upload.  Destroy with
 * mu_theory_destroy. */
mu_status mu_theory_create_expr(mu_ctx *ctx, const mu_expr_theory_desc *d, mu_theory **out);

/* -------------------------------------------------------------- evaluation */

/* Cost of n_vec parameter vectors (params: [n_vec][n_par] row-major) over
 * every fit-range bin of every histogram of `data` (Eqs. 2-3), in one launch.
 * cost: [n_vec].  cost_per_histo: [n_vec][n_histo] or NULL.  Every map row a
 * histogram names must exist in the theory (else MU_E_ARG).  Non-finite
 * parameters give a NaN cost; the likelihood with N <= 0 < d gives +inf. */
mu_status mu_chi2_eval(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                       const double *params, int32_t n_vec, unsigned mem,
                       double *cost, double *cost_per_histo);

/* mu_chi2_eval for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * launches and results, bit for bit, as mu_chi2_eval with MU_MEM_DEVICE, but
 * no device or host allocation of any kind.  params, cost and cost_per_histo
 * are device pointers on the context's device; the call only enqueues work
 * on the context stream.  The partial slots live in a static array of the
 * library's code object on each device: 32768 slots of 256 B (8 MiB), held
 * until the process ends.  A launch needs one slot per work range plus
 * n_vec x n_histo; a call that needs more is refused with MU_E_UNSUPPORTED
 * before anything is enqueued (fewer vectors per call, or a larger
 * mu_ctx_set_tile, fits it).  Every call on one device shares that array:
 * calls that overlap on one GPU (other streams, other contexts, other host
 * threads) race and give wrong results; calls in order on one stream do not.
 * No kernel timing is recorded for this entry point.  Other errors as
 * mu_chi2_eval. */
mu_status mu_chi2_eval_static(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                              const double *params, int32_t n_vec, double *cost, double *cost_per_histo);

/* Cost and its analytic gradient d cost / d p (adjoint pass: per bin the
 * cost's derivative in N times dN/dp through Eq. 1, the product form of A and
 * the map / function array).  grad: [n_vec][n_par]. */
mu_status mu_chi2_grad(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                       const double *params, int32_t n_vec, unsigned mem,
                       double *cost, double *grad);

/* A minimiser's step over one dataset in one call: cost and gradient at the
 * n_grad vectors params_grad ([n_grad][n_par]) as mu_chi2_grad, and the cost
 * at the n_cost vectors params_cost ([n_cost][n_par]) as mu_chi2_eval (trial
 * or finite-difference points; Sec. 4 and Table 1 count such evaluations).
 * Both passes run on the context's stream as one evaluation launch (chi^2,
 * compiled theory shapes, 32-bit counts; otherwise two launches) and share
 * one merge launch.  The costs at params_cost are bitwise those of a separate
 * mu_chi2_eval call.  In one launch the gradient pass takes longer bin ranges
 * per wave than a mu_chi2_grad call of its own (unless mu_ctx_set_tile fixes
 * them), so its cost and gradient equal that call's to rounding; with two
 * launches, bitwise.  Outputs:
 * cost_grad [n_grad], grad [n_grad][n_par], cost [n_cost].  mem applies to
 * all parameter and output arrays.  Errors as mu_chi2_eval. */
mu_status mu_chi2_eval_grad(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                            const double *params_grad, int32_t n_grad, const double *params_cost,
                            int32_t n_cost, unsigned mem, double *cost_grad, double *grad, double *cost);

/* Batched evaluation of n_jobs independent (dataset, theory, parameter
 * vector) jobs of uneven sizes (Sec. 4: many cost evaluations per fit, here
 * across fits and datasets).  The fit ranges of all jobs whose theory matches
 * a compiled shape are concatenated and cut into equal ranges, one per
 * 64-lane wave, in ONE evaluation launch in which every segment runs its own
 * job's compiled shape; jobs of other theories (or FP64 counts) take one more
 * launch of the interpreted kernel; one merge launch follows.  params:
 * [n_jobs][ld] with ld >= every theory's n_par (each job reads its first
 * n_par entries).  cost: [n_jobs]; grad: [n_jobs][ld] or NULL (entries past a
 * job's n_par are left untouched).  Data and theories may repeat across jobs.
 * All datasets must share one count storage (MU_E_UNSUPPORTED otherwise). */
mu_status mu_chi2_batch(mu_ctx *ctx, int32_t n_jobs, const mu_data *const *data,
                        const mu_theory *const *th, mu_cost cost_kind, int32_t ld,
                        const double *params, unsigned mem, double *cost, double *grad);

/* Expected counts N(t_n) (Eq. 1) at every fit-range bin of every histogram,
 * concatenated in histogram order: out[mu_data_bins(data)]. */
mu_status mu_model_eval(mu_ctx *ctx, const mu_data *data, const mu_theory *th,
                        const double *params, unsigned mem, double *out);

/* Bins per work unit used by evaluation launches on this context; the unit
 * is one 64-lane wave (four share a workgroup).
 * Single-dataset launches (mu_chi2_eval, mu_chi2_grad, mu_model_eval) cut the
 * n_vec x bins work into equal ranges of this many bins, one per wave,
 * across histogram and vector boundaries; batched launches (mu_chi2_batch,
 * the fitter) cut the concatenated fit ranges of their jobs the same way,
 * across histogram and job boundaries.  0 (default): per launch, the choice
 * mu_autotune (single-dataset) or mu_autotune_batch (batched) measured for
 * the same kind of launch, theory shape, mode, cost and size (to a power of
 * two), else one range per resident wave (at least 64 bins).
 * Otherwise any value in [64, 2^26]; gradient passes cut their ranges at
 * 2^20 bins per wave (each lane then sums at most 2^14 terms plainly; cost
 * passes fold their per-lane sums by TwoSum at every anchor).  Results depend
 * on it only through the rounding order of the sums. */
mu_status mu_ctx_set_tile(mu_ctx *ctx, int32_t tile_bins);
int32_t mu_ctx_get_tile(const mu_ctx *ctx);

/* Lane steps between exact re-evaluations of the theory's factors (the rest
 * are advanced by exact recurrences of the uniform time grid); 0 restores the
 * default (64).  Range [1, 256], rounded up to a multiple of 4 lane steps
 * (the distance at which counts are read ahead of their use), so 1 .. 4 all
 * re-evaluate every fourth step.  The recurrence drift of a factor grows like
 * k eps (geometric, rotation) and k^2 eps / 2 (Gaussian): below 5e-13
 * relative at 64 and 8e-12 at 256. */
mu_status mu_ctx_set_anchor(mu_ctx *ctx, int32_t every);
int32_t mu_ctx_get_anchor(const mu_ctx *ctx);

/* 1 (default): theories whose shape matches a compiled specialisation
 * (A se tf; A sg tf; A stg; A1 se + A2 stg; A1 se tf + A2 stg) run that
 * kernel; 0: every theory runs the generic interpreted kernel.  Results agree
 * to rounding either way. */
mu_status mu_ctx_set_specialize(mu_ctx *ctx, int32_t on);

/* Kernel timing.  While enabled, the context records a pair of HIP events on
 * its stream around every evaluation-kernel and merge-kernel launch it makes
 * (mu_chi2_eval, mu_chi2_grad, mu_chi2_batch, mu_model_eval, the fitter).
 * enable != 0 discards earlier records and starts recording; enable == 0
 * stops (records are kept).  Events are reused across enables; they are the
 * only cost, and launches are not otherwise changed. */
typedef enum {
  MU_TIME_EVAL_COST = 0,  /* evaluation kernels, cost only */
  MU_TIME_EVAL_GRAD = 1,  /* evaluation kernels, cost and gradient */
  MU_TIME_EVAL_MODEL = 2, /* mu_model_eval kernels */
  MU_TIME_MERGE = 3,      /* merge kernels (both modes) */
  MU_TIME_EVAL_GRAD_COST = 4 /* mu_chi2_eval_grad's single evaluation launch */
} mu_time_kind;
mu_status mu_ctx_timing(mu_ctx *ctx, int32_t enable);
/* Waits for the recorded launches of `kind` to finish and writes how many
 * there were and their summed duration in milliseconds (start event to end
 * event on the stream).  MU_E_ARG for an unknown kind or NULL outputs. */
mu_status mu_ctx_timing_read(mu_ctx *ctx, int32_t kind, int32_t *n_launches, double *total_ms);

/* Measure the evaluation of n_vec vectors over `data` (cost, or cost and
 * gradient when grad != 0) for several bins-per-wave values (powers of
 * two from 1024 to 65536, and the values that give 1, 2, 3, 4, 6 or 8
 * waves per resident wave slot) and anchor intervals 32 .. 256, keep
 * candidates whose costs agree with the first to 1e-12 relative, time the
 * four fastest again (three interleaved rounds of ten launches; a candidate's
 * best round counts), and remember the fastest for later single-dataset
 * launches of the same theory
 * shape, mode, cost and size (to a power of two) while the tile size is 0.
 * Writes the choice and its time per launch in microseconds (any may be
 * NULL).  Leaves the explicit tile size and anchor interval unchanged. */
mu_status mu_autotune(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                      const double *params, int32_t n_vec, unsigned mem, int32_t grad,
                      int32_t *best_tile, int32_t *best_anchor, double *best_us);

/* Record (tile_bins, anchor_every) for later single-dataset launches of
 * n_vec vectors over `data` with this theory shape, cost and mode (gradient
 * when grad != 0), as if mu_autotune had chosen it: replays a choice measured
 * earlier (another process, a stored configuration) without measuring.
 * MU_E_ARG for tile_bins outside [64, 2^26], anchor_every outside [1, 256],
 * n_vec < 1 or an unknown cost kind. */
mu_status mu_autotune_set(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                          int32_t n_vec, int32_t grad, int32_t tile_bins, int32_t anchor_every);

/* The batched counterpart of mu_autotune (the paper plans auto-tuning of
 * its kernels, Secs. 3 and 6): runs the jobs of a mu_chi2_batch call (cost,
 * or cost and gradient when grad != 0) at several bins-per-wave values (1, 2,
 * 3, 4, 6 or 8 ranges per resident wave, powers of two from 1024 to 65536)
 * and anchor intervals 32 .. 256, keeps candidates whose costs agree with the
 * first to 1e-12 relative, times the four fastest again as mu_autotune does,
 * and remembers the fastest for later batched
 * launches of the same mode, cost and size (to a power of two) while the
 * tile size is 0.  Outputs as mu_autotune (any may be NULL). */
mu_status mu_autotune_batch(mu_ctx *ctx, int32_t n_jobs, const mu_data *const *data, const mu_theory *const *th,
                            mu_cost cost_kind, int32_t ld, const double *params, unsigned mem, int32_t grad,
                            int32_t *best_tile, int32_t *best_anchor, double *best_us);

/* Tuning cache file: the choices mu_autotune, mu_autotune_batch and
 * mu_autotune_set remembered on this context, as text:
 *   mu-autotune 1
 *   arch <device architecture, e.g. gfx950:sramecc+:xnack->
 *   <shape> <mode> <cost> <kind> <log2 size> <bins per wave> <anchor>   (one line each)
 * shape 0 interpreted, 1..5 compiled shapes, 6 batched launch of compiled
 * shapes; mode 0 cost, 1 gradient; cost 0 chi^2, 1 likelihood; kind 0
 * batched, 1 single-dataset; '#' starts a comment line.
 * mu_autotune_save writes the file (MU_E_ARG if it cannot).  mu_autotune_load
 * adds its choices to the context: MU_E_ARG, with nothing loaded, for a file
 * that is missing, malformed or holds an out-of-range entry;
 * MU_E_UNSUPPORTED, with nothing loaded, for a file written on another
 * architecture.  mu_autotune_check_file validates a file without a device
 * (same rules except the architecture) and writes a message into msg (may be
 * NULL). */
mu_status mu_autotune_save(mu_ctx *ctx, const char *path);
mu_status mu_autotune_load(mu_ctx *ctx, const char *path);
mu_status mu_autotune_check_file(const char *path, char *msg, int32_t msg_len);

/* ----------------------------------------------------------------- fitting */

/* Options of mu_fit_batch (zero-initialise, then set what you need). */
typedef struct {
  int32_t max_fcn;        /* cost evaluations per fit (0: 100000) */
  int32_t max_iter;       /* line-search iterations per fit (0: 1000) */
  double tol_edm;         /* stop the variable-metric stage when g^T V g / 2 < tol_edm (0: 1e-8) */
  double tol_step_rel;    /* ... or when every step is below tol * max(|p_k|, sigma_k) (0: 1e-7) */
  int32_t analytic_grad;  /* 1: gradients from the adjoint kernel; 0: central differences (2n costs) */
  int32_t batched;        /* 1: every round evaluates the requests of all active fits in one launch;
                             0: fits one after another, one launch per evaluated point */
  int32_t polish;         /* 1: finish with Newton steps on a Hessian from central differences of the
                             gradient until the relative step is below 1e-12 */
  int32_t reserved;
  const uint8_t *fixed;   /* [n_fits][ld]: non-zero entries are held at their start values; may be NULL */
} mu_fit_opts;

typedef struct {
  double cost;     /* cost at params_out */
  double edm;      /* estimated distance to the minimum, g^T V g / 2 */
  int32_t n_iter;  /* accepted variable-metric steps */
  int32_t n_fcn;   /* cost evaluations (gradient stencil points included) */
  int32_t n_grad;  /* gradient evaluations */
  int32_t status;  /* 0 converged: the final EDM (after a polish, from the differenced Hessian) is below
                      tol_edm, whatever stopped the iterations;
                      1 evaluation or iteration budget spent with the final EDM above tol_edm;
                      2 non-finite cost at the start;
                      3 line search failed with the final EDM above tol_edm (params_out is the best point found);
                      4 every step fell below tol_step_rel while the final EDM stayed above tol_edm (a nearly
                        flat valley: the point is not a certified minimum) */
} mu_fit_result;

/* Minimise the cost of n_fits independent fits (Sec. 4: the fit of P by
 * minimising Eq. 2 or Eq. 3; there with Minuit2's variable-metric method).
 * Fit f uses data[f], th[f] and start[f][0 .. n_par-1] (row stride ld >= every
 * theory's n_par).  Method: start Hessian by central differences of the
 * gradient, BFGS updates of the inverse Hessian V with a backtracking line
 * search along -V g, and optionally a final Newton polish.  Outputs:
 * params_out [n_fits][ld] (entries past n_par copied from start), cov_out
 * [n_fits][ld][ld] = 2 V (chi^2 and likelihood are -2 ln L up to a constant;
 * zero rows for fixed parameters; may be NULL), res [n_fits].  MU_E_ARG for a
 * non-finite start value.  A fit whose cost is not finite at its start ends
 * with status 2; this is not an error of the call. */
mu_status mu_fit_batch(mu_ctx *ctx, int32_t n_fits, const mu_data *const *data, const mu_theory *const *th,
                       mu_cost cost_kind, int32_t ld, const double *start, const mu_fit_opts *opts,
                       double *params_out, double *cov_out, mu_fit_result *res);

/* ------------------------------------------------------- parameter errors */

/* After the minimum (Sec. 4 fits with Minuit2's minimisation; the steps that
 * usually follow are its HESSE and MINOS): both costs are -2 ln L up to a
 * constant (Eqs. 2-3), so the covariance is 2 H^-1 and a rise of `up` = 1 in
 * the profiled cost marks one standard deviation. */
typedef enum {
  MU_HESSE_GAUSS_NEWTON = 0, /* H = sum_n c_n (dN_n/dp)(dN_n/dp)^T with c_n = d^2 term / dN^2 (2/v for chi^2,
                                2 d / N^2 for the likelihood): the bins' Jacobian rows from the evaluation kernel,
                                their Gram matrix per histogram on the FP64 matrix cores, the chain rule through
                                the map and function array on the host */
  MU_HESSE_DIFF = 1          /* central differences of the analytic gradient, the 2n points in one launch
                                (step 1e-5 max(|p_k|, 1e-3)) */
} mu_hesse_method;

/* Hessian of the cost at params (host, [n_par]) of one dataset and theory:
 * hess [n_par][n_par] (host; zero rows and columns for parameters with
 * fixed[k] != 0; fixed may be NULL).  cov [n_par][n_par] (host, may be NULL):
 * 2 H^-1 over the free block (zero rows / columns for fixed parameters), or
 * all NaN when the free block is not positive definite; *pos_def (may be
 * NULL) says which.  MU_E_ARG for a non-finite parameter or an unknown method
 * or cost kind.  Synchronous. */
mu_status mu_hesse(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind, int32_t method,
                   const double *params, const uint8_t *fixed, double *hess, double *cov, int32_t *pos_def);

/* Likelihood profile of parameter k: at each of the n_points values, the cost
 * minimised over every other parameter not fixed (all points as one batched
 * fit, mu_fit_batch with analytic gradients and polish, started at p_min
 * moved along k's correlations).  prof_cost [n_points]; prof_params
 * [n_points][n_par] and status [n_points] (the fits' status) may be NULL.
 * Host memory; synchronous. */
mu_status mu_profile(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind, const double *p_min,
                     const uint8_t *fixed, int32_t k, int32_t n_points, const double *values, double *prof_cost,
                     double *prof_params, int32_t *status);

/* MINOS-like errors of parameter k around the minimum p_min: the offsets
 * err_lo < 0 < err_hi where the profile of k reaches cost(p_min) + up.  Both
 * sides start one Hessian standard deviation out (doubled until bracketed)
 * and are refined together, one two-point mu_profile per round, by
 * interpolation in the squared offset (exact for a parabolic profile) until
 * the profile is within 1e-9 up of the target.  *n_rounds (may be NULL): the
 * rounds used.  MU_E_STATE (nothing written) if a side has not converged in 60
 * rounds.  Host memory; synchronous. */
mu_status mu_minos(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind, const double *p_min,
                   const uint8_t *fixed, int32_t k, double up, double *err_lo, double *err_hi, int32_t *n_rounds);

/* ------------------------------------------------------------------ seeder */

/* A learned seeder proposes start parameters for fits of the exp*cos family
 * (A(t) = A e^(-lambda t) cos(2 pi nu t + phi)) on histograms of 8192 bins of
 * 0.001 us from t = 0.  It is a 1024-512-256-128-8 perceptron with ReLU, run
 * with BF16 operands on the matrix cores and FP32 sums.  Input: the histogram
 * rebinned by 8 to 1024 bins c_b, as the asymmetry (c_b - 8 Nbkg) /
 * (8 N0 ebar_b) - 1 clipped to [-4, 4], where ebar_b is the lifetime decay
 * averaged over bin b and N0, Nbkg solve m = N0 e + Nbkg for the means m of
 * the first and last 256 bins (e: the decay averaged over each window).
 * Outputs 0..4: A / 0.3,
 * ln(lambda / 0.05) / ln 100, ln(nu / 0.1) / ln 500, cos phi, sin phi (outputs
 * 5..7 carry no loss).  The start's N0 and Nbkg are those window estimates
 * (the same rule as the default start).
 *
 * Parameter layout (FP32, mu_seeder_param_count() values): for each layer
 * l = 0..3 its weights [out][in] row-major, then its biases [out].
 *
 * Training data come from the method itself (mu_gen_histos): parameters
 * drawn from Philox4x32-10 with key `seed` and counters (sample, 0xFFFFFFFF,
 * 0 / 1): N0 log-uniform in [1e2, 1e5], Nbkg uniform in [1, 10], A uniform in
 * [0.05, 0.3], lambda log-uniform in [0.05, 5] /us, nu log-uniform in
 * [0.1, 50] MHz, phi uniform in [0, 2 pi); expected counts of the 1024
 * rebinned bins from Eq. 1; one Poisson draw per rebinned bin. */
typedef struct {
  uint64_t seed;          /* generator key */
  uint64_t first_sample;  /* index of the first training sample */
  int32_t batch;          /* samples per step */
  int32_t steps;          /* optimiser steps; step k uses samples first + k batch .. */
  float lr;               /* Adam learning rate at step 0 */
  float lr_final_frac;    /* cosine decay to lr * lr_final_frac at the last step */
} mu_seed_train_opts;

int64_t mu_seeder_param_count(void);
/* A seeder with the given initial parameters (host, FP32, finite). */
mu_status mu_seeder_create(mu_ctx *ctx, const float *init_params, mu_seeder **out);
mu_status mu_seeder_destroy(mu_seeder *s);
mu_status mu_seeder_get_params(const mu_seeder *s, float *out);  /* host, param_count values */
mu_status mu_seeder_get_grads(const mu_seeder *s, float *out);   /* gradient of the last step */
int64_t mu_seeder_steps(const mu_seeder *s);                     /* Adam steps taken */

/* Generate samples first .. first + n - 1 of the stream with key `seed`:
 * theta [n][6] = (N0, Nbkg, A, lambda, nu, phi); with fine == 0 the 1024
 * rebinned bins (expected count = sum of 8 fine bins, one Poisson draw each),
 * with fine != 0 the 8192 bins of 0.001 us (one Poisson draw per bin):
 * counts (FP32 integers) and mu (expected counts) of [n][1024] or [n][8192].
 * Any output may be NULL (not all).  Poisson draws: inversion below a mean of
 * 10, transformed rejection (Hoermann 1993) above; uniforms from Philox with
 * counters (sample, bin or 0x10000 + fine bin, iteration). */
mu_status mu_gen_histos(mu_ctx *ctx, uint64_t seed, uint64_t first, int32_t n, int32_t fine, unsigned mem,
                        float *counts, double *theta, double *mu);

/* Network output y [B][8] for BF16 inputs x [B][1024] (bit patterns). */
mu_status mu_seeder_forward(mu_ctx *ctx, mu_seeder *s, const uint16_t *x_bf16, int32_t B, unsigned mem, float *y);
/* One step on given inputs and targets [B][8]: loss (sum over the batch of
 * sum_o w_o (y - t)^2, divided by B; w = 1 for outputs 0..4), gradient, and an
 * Adam update (b1 0.9, b2 0.999, eps 1e-8) when update != 0.  loss may be NULL. */
mu_status mu_seeder_train_step(mu_ctx *ctx, mu_seeder *s, const uint16_t *x_bf16, const float *targets, int32_t B,
                               float lr, int32_t update, unsigned mem, float *loss);
/* The buffers of one layer (0 .. 3) as the last forward pass (mu_seeder_forward,
 * mu_seeder_train_step, mu_seed_infer) left them, for the first B samples of
 * that pass (host memory, any output may be NULL): x_in [B][K_l] the layer's
 * BF16 input (bit patterns; layer 0: the network input, else the BF16 ReLU of
 * the previous layer's pre-activation), z [B][N_l] its FP32 pre-activation
 * (layer 3: the output), and after a training step dz [B][N_l] the FP32
 * gradient of the loss in z and g [B][N_l] its BF16 copy used by the GEMMs.
 * MU_E_STATE when B exceeds the samples of the last pass. */
mu_status mu_seeder_layer(mu_ctx *ctx, const mu_seeder *s, int32_t layer, int32_t B, uint16_t *x_in, float *z,
                          float *dz, uint16_t *g);
/* Train on freshly generated samples; loss_curve [steps] (host) may be NULL. */
mu_status mu_seeder_train(mu_ctx *ctx, mu_seeder *s, const mu_seed_train_opts *opts, float *loss_curve);
/* Start vectors (N0, Nbkg, A, lambda, nu, phi) for n datasets, each one
 * histogram of 8192 integer counts in 0.001 us bins from t = 0 (else
 * MU_E_ARG).  ok_out[i] = 0 when the decoded values are not finite or leave
 * A in [0.01, 1], lambda in [0.005, 50], nu in [0.02, 250]; that row then
 * holds the default start (A 0.175, lambda 0.5, nu sqrt 5, phi 0). */
mu_status mu_seed_infer(mu_ctx *ctx, const mu_seeder *s, int32_t n, const mu_data *const *data, double *start_out,
                        uint8_t *ok_out);
/* Checkpoint (parameters, Adam moments, step count) and restore. */
mu_status mu_seeder_save(const mu_seeder *s, const char *path);
mu_status mu_seeder_load(mu_ctx *ctx, const char *path, mu_seeder **out);

#ifdef __cplusplus
}
#endif

#endif /* MU_H */
