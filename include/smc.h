/*
 * smc.h -- C ABI of libsmc: on-the-fly statistical model checking of
 * mass-action reaction networks on AMD Instinct MI355X (gfx950).
 *
 * Method: Ballarini, Forlin, Mazza, Prandi, "Efficient Parallel Statistical
 * Model Checking of Biochemical Networks" (PDMC 2009):
 *   - trajectories are drawn with Gillespie's direct method (Sec. 2.2,
 *     eqs. 1, 2a, 2b and the five-step SSA template);
 *   - each trajectory is checked against a BLTLc formula (Sec. 3.1) while it
 *     is generated and stops as soon as the formula is decided (Sec. 3.2);
 *   - the verdicts are Bernoulli samples; the estimate is their mean with the
 *     Wilson score interval (eq. 3), and the number of trajectories is chosen
 *     by the iterative Wilson procedure (eq. 4, Fig. 2) or fixed by the caller.
 *
 * Conventions (all entry points):
 *   - Return value: SMC_OK (0) or a negative SMC_E_* code.  No C++ exception
 *     crosses this interface.  The message of the last failure on a context
 *     is returned by smc_last_error().
 *   - Ownership: the caller owns every array it passes in or out; the library
 *     copies what it keeps.  The library owns the handles it creates; they are
 *     released with the matching *_destroy function.
 *   - Pointers are host pointers unless stated otherwise.
 *   - One context per host thread.  Work on a context is ordered on its HIP
 *     stream; every entry point returns after its results are on the host.
 *   - Randomness is a pure function of (seed, model_id, trajectory index,
 *     event index) through Philox4x32-10, so results do not depend on the
 *     launch configuration.
 */
#ifndef SMC_H
#define SMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SMC_OK 0
#define SMC_E_INVALID (-1)     /* bad argument, network or parameter          */
#define SMC_E_PARSE (-2)       /* formula text does not parse                 */
#define SMC_E_UNSUPPORTED (-3) /* formula outside the GPU monitor classes     */
#define SMC_E_HIP (-4)         /* HIP runtime error                           */
#define SMC_E_NOMEM (-5)       /* device or host allocation failed            */
#define SMC_E_CANCELLED (-6)   /* stopped by smc_cancel()                     */
#define SMC_E_TIMEOUT (-7)     /* exceeded the context's watchdog time        */

/* verdict_reason byte written per trajectory: verdict | reason << 1 */
#define SMC_REASON_STATE 0   /* decided by the state just entered             */
#define SMC_REASON_TIME 1    /* decided when a time bound passed              */
#define SMC_REASON_ABSORB 2  /* total propensity zero: no further event       */
#define SMC_REASON_CAP 3     /* undecided after max_events events: FALSE      */
#define SMC_REASON_TMAX 4    /* undecided past t_max: FALSE (Sec. 3.2 rule)   */

/* smc_params.flags */
#define SMC_CONSERVATIVE_START 1u /* first sample from eq. 4 at p = 0.5 (Sec. 3.3.2)  */
#define SMC_PAPER_ROUNDING 2u     /* Fig. 2 rounding exactly as printed: p +- eps may
                                     step across 0.5 (default: the step stops at 0.5) */
#define SMC_NO_SPECULATION 4u     /* iterative jobs: issue only the indices each batch
                                     needs.  Default: when every job of a launch is
                                     iterative and their capacities together fit in one
                                     pass over the device's lanes, every index up to each
                                     capacity runs at once and Fig. 2 is applied to the
                                     recorded outcomes in index order; results are
                                     identical, the extra trajectories are discarded.  */
#define SMC_DEVICE_PTRS 8u        /* the large arrays of the call are device pointers
                                     on the context's device (e.g. a torch tensor's
                                     data_ptr()): smc_trajectories' events and
                                     verdict_reason, smc_sample_state's counts.  The
                                     kernels write them in place, with no host copy;
                                     the call still returns once they are written.  For
                                     smc_surrogate_query the same bit goes in its own
                                     flags argument.                                 */

#define SMC_TREE_SUMS 16u         /* jobs that run in lane groups (smc_params.lanes,
                                     smc_set_lanes_per_trajectory) add their
                                     propensities in a tree over the group instead
                                     of in channel order: each lane sums its own
                                     block of channels and the group scans the block
                                     sums in log2(lanes) steps.  The direct method's
                                     distribution is unchanged (channel j with
                                     probability a_j/a0, tau ~ Exp(a0), Sec. 2.1),
                                     but a0 and the boundaries are rounded
                                     differently, so results equal the channel-order
                                     kernels' in distribution, not bit for bit:
                                     verdicts and event counts per trajectory agree
                                     except where a draw falls within a few ulps of
                                     a boundary, and event times differ in the last
                                     bits.  No effect on one lane per trajectory.
                                     The grouped jobs of one call must agree on it
                                     (else SMC_E_INVALID).                          */

typedef struct smc_ctx smc_ctx;
typedef struct smc_net smc_net;
typedef struct smc_formula smc_formula;

/* ---- context ----------------------------------------------------------- */
/* Create a context on HIP device `hip_device`.  `hip_stream` is a hipStream_t
 * to order work on (e.g. torch.cuda.current_stream().cuda_stream), or NULL for
 * a stream owned by the context.  Errors: SMC_E_INVALID (no such device),
 * SMC_E_HIP. */
int smc_ctx_create(int hip_device, void *hip_stream, smc_ctx **out);
void smc_ctx_destroy(smc_ctx *ctx);
/* Message of the last failure on ctx ("" if none); valid until the next call
 * on ctx.  With ctx == NULL: the last failure of smc_ctx_create on this
 * thread. */
const char *smc_last_error(const smc_ctx *ctx);
/* Watchdog: a call whose kernels run longer than `seconds` is stopped and
 * returns SMC_E_TIMEOUT (default 300 s; <= 0 disables). */
int smc_set_watchdog(smc_ctx *ctx, double seconds);
/* Launch shape of the SSA kernel: waves per compute unit (1..32, 0 = tuned
 * default).  Results do not depend on it. */
int smc_set_waves_per_cu(smc_ctx *ctx, int waves_per_cu);
/* Kernel specialisation.  For a launch whose jobs all share one network
 * structure (reactants and state changes, S <= 16 species, M <= 8 channels)
 * and one formula without arithmetic (RPN) predicates, the library can
 * compile, at run time, a kernel with that structure as constants (species
 * counts in registers, table indices as immediates) and cache it per device
 * and structure for the life of the process.  Rate constants, initial counts
 * and seeds stay inputs, so one kernel serves a whole rate sweep.  Results are
 * identical to the generic kernel's.  Modes: SMC_SPECIALIZE_AUTO (default:
 * specialise when supported; if run-time compilation fails, warn once on
 * stderr and use the generic kernel), SMC_SPECIALIZE_OFF (generic kernel
 * only), SMC_SPECIALIZE_REQUIRED (fail with SMC_E_UNSUPPORTED or SMC_E_HIP
 * instead of using the generic kernel).  Errors: SMC_E_INVALID. */
#define SMC_SPECIALIZE_AUTO 0
#define SMC_SPECIALIZE_OFF 1
#define SMC_SPECIALIZE_REQUIRED 2
int smc_set_specialization(smc_ctx *ctx, int mode);
/* Which SSA kernel the last estimation call on ctx launched: -1 none yet,
 * SMC_KERNEL_GENERIC_SMALL (table-driven, <= 4 channels), SMC_KERNEL_GENERIC
 * (table-driven, blocked prefix), SMC_KERNEL_SPECIALIZED,
 * SMC_KERNEL_GENERIC_GROUPED (table-driven, several lanes per trajectory),
 * SMC_KERNEL_GENERIC_TREE (the same with SMC_TREE_SUMS),
 * SMC_KERNEL_GENERIC_TRACE (table-driven, the launch holds trace programs). */
#define SMC_KERNEL_GENERIC_SMALL 0
#define SMC_KERNEL_GENERIC 1
#define SMC_KERNEL_SPECIALIZED 2
#define SMC_KERNEL_GENERIC_GROUPED 3
#define SMC_KERNEL_GENERIC_TREE 4
#define SMC_KERNEL_GENERIC_TRACE 5
int smc_last_kernel(const smc_ctx *ctx);
/* Register budget of specialised kernels: compile them so that
 * `waves_per_simd` waves fit on one SIMD (1..8; registers beyond the budget
 * go to scratch memory), or 0 for the compiler's own choice (default).
 * Results do not depend on it.  Errors: SMC_E_INVALID. */
int smc_set_kernel_occupancy(smc_ctx *ctx, int waves_per_simd);

/* Lanes per trajectory (1, 2, 4, 8 or 16; 0 = automatic) for networks of
 * more than four channels on the generic kernels.  A group of that many
 * consecutive lanes runs one trajectory: the channels' propensities are
 * shared out over the group and added in channel order lane after lane, so
 * every sum, selection and result is bit-identical to one lane per
 * trajectory; an event takes fewer instructions on each lane but the
 * device holds fewer trajectories at once.  It pays where trajectories are
 * few and long (a launch that leaves lanes idle).  A job's own
 * smc_params.lanes overrides the setting.  The group size is raised where
 * needed so that a group covers the channels in at most 8 rounds of 8 per
 * lane (e.g. at least 8 lanes for 512 channels); networks of more than 1024
 * channels and launches on specialised kernels use one lane.  Results do
 * not depend on it.  Errors: SMC_E_INVALID. */
int smc_set_lanes_per_trajectory(smc_ctx *ctx, int lanes);

/* Ask a running call on ctx (from another thread) to stop: it returns
 * SMC_E_CANCELLED. */
void smc_cancel(smc_ctx *ctx);
/* Number of compute units of the context's device. */
int smc_device_cus(const smc_ctx *ctx);

/* ---- reaction networks (Sec. 2.2) -------------------------------------- */
/* Mass-action network with S species and M reaction channels.  Reaction j has
 * rate constant c_j = rate[j] >= 0, reactants reactants[2j], reactants[2j+1]
 * (species index or -1; two equal indices form a homodimer), and a net state
 * change of change_val[4j+q] on species change_idx[4j+q] (q = 0..3, index -1
 * = unused entry).  Its propensity is c_j times the number of distinct
 * reactant combinations: 1, x_a, x_a x_b, or x_a (x_a - 1) / 2.
 * Errors (SMC_E_INVALID): S < 1, M < 1, a negative count or rate, a species
 * index out of range, or a change that consumes more of a species than the
 * reaction's reactants hold (counts could go negative), S > 16384.  names (S
 * strings, or NULL for X0, X1, ...) are the species names used by formulas.
 * Runs (estimates, trajectories, state samples) need S <= 255: a wave keeps
 * the counts of its 64 trajectories, plus one constant row, in 64 KiB of
 * LDS; larger networks give SMC_E_INVALID there. */
typedef struct {
    int32_t n_species;
    int32_t n_reactions;
    const int32_t *x0;         /* [S] initial counts                       */
    const double *rate;        /* [M] rate constants                       */
    const int32_t *reactants;  /* [M][2]                                   */
    const int32_t *change_idx; /* [M][4]                                   */
    const int32_t *change_val; /* [M][4]                                   */
    const char *const *names;  /* [S] or NULL                              */
} smc_net_desc;

int smc_net_create(smc_ctx *ctx, const smc_net_desc *desc, smc_net **out);
/* Replace the M rate constants (parameter sweeps). */
int smc_net_set_rates(smc_net *net, const double *rate);
void smc_net_destroy(smc_net *net);

/* ---- formulas (Sec. 3.1) ----------------------------------------------- */
/* Compile BLTLc text over the network's species names:
 *   phi ::= val op val | !phi | phi & phi | phi '|' phi | X I phi | phi U I phi
 *           | F I phi | G I phi | (phi) | true | false
 *   val ::= name | number | val (+ - * /) val | -val | sqrt(val) | pow(val, k) | (val)
 *   I   ::= [a,b] | <= b | (omitted: [0, inf))      op: < <= >= > = !=
 * Precedence: unary (!, X, F, G) > U (right associative) > & > |.
 * pow takes a constant integral exponent k in 0..64 and is evaluated by
 * binary powering (from 1, for the seven exponent bits from the most
 * significant: square, then multiply where the bit is set; one FP64 rounding
 * per multiplication); other exponents give SMC_E_UNSUPPORTED.
 * Compact GPU monitor classes (a few registers per trajectory): top-level boolean combinations of
 *   state predicates; F I p; G I p; p U I q; X I p; the nested until
 *   p U I (q U[0,c] r), also with F[0,c] r inside and as F I (q U[0,c] r);
 *   p U I (r & G[0,c] q), r optional;
 *   X I (p U J q), X I F J q and X I G J q;
 *   the response G I (p | F[0,d] q) and its dual
 *   F I (p & G[0,d] q) (either operand order, p optional), where p, q, r
 *   are boolean combinations of predicates.  At most two of the nested,
 *   next-until, until-G and response monitors per formula.
 * Any other formula (deeper nesting, temporal left operands of U, inner
 * windows that do not start at 0, ...) compiles to a trace program of at
 * most 32 nodes (F and G count as 2 and 4): each lane records the states of
 * its trajectory (entry time and predicate bits), the buffer of Sec. 3.2, and
 * decides the formula on that prefix, at checkpoints, finding the first
 * deciding state by bisection; the results are those of the compact monitors'
 * semantics (stop at the earliest decision).  Runs with a trace program need
 * max_events in 1..2^20 (states are recorded up to the cap), use one lane per
 * trajectory, record areas of about (13 + nodes) bytes per state and lane
 * within an 8 GiB budget (which bounds the lanes of the launch), and no
 * specialised kernel or allocation-free call.  More than 16 predicates, an
 * arithmetic predicate deeper than the GPU's stack, or a trace program of more
 * than 32 nodes give SMC_E_UNSUPPORTED; text that does not parse gives
 * SMC_E_PARSE. */
int smc_formula_compile(smc_ctx *ctx, const smc_net *net, const char *text, smc_formula **out);
/* Time span of the path the formula can depend on (+inf if unbounded). */
double smc_formula_horizon(const smc_formula *f);
/* The same compilation (Sec. 3.1 syntax, the GPU monitor classes above) on
 * the host only, with no context or device: for validating a formula over
 * species names n_names (names[0 .. n_names-1]) before a run.  Returns
 * SMC_OK, SMC_E_PARSE or SMC_E_UNSUPPORTED as smc_formula_compile would, or
 * SMC_E_INVALID for a null text or name.  When msg is not NULL, the reason
 * ("" on success) is copied into msg[0 .. cap-1], NUL-terminated and cut to
 * fit.  On success *horizon (if not NULL) receives the formula's horizon.
 * Nothing is allocated that outlives the call. */
int smc_formula_check(const char *text, const char *const *names, int n_names, double *horizon, char *msg,
                      size_t cap);
void smc_formula_destroy(smc_formula *f);

/* ---- estimation (Sec. 3.3) --------------------------------------------- */
typedef struct {
    double confidence;   /* 1 - alpha in (0,1)                                   */
    double half_width;   /* epsilon > 0: target interval [p - eps, p + eps]      */
    double z;            /* > 0: use this z_{1-alpha/2}; 0: derive from confidence */
    uint64_t fixed_n;    /* 0: iterative Wilson (Fig. 2); > 0: exactly this many  */
    uint64_t seed;       /* Philox key (words 0..1)                              */
    uint32_t model_id;   /* Philox counter word 2 (word 1: trajectory index)      */
    uint32_t max_events; /* 0: no cap; else undecided after this many events: FALSE */
    double t_max;        /* pessimistic horizon for unbounded formulas (+inf: none) */
    uint32_t flags;      /* SMC_CONSERVATIVE_START | SMC_PAPER_ROUNDING |
                            SMC_NO_SPECULATION | SMC_DEVICE_PTRS | SMC_TREE_SUMS */
    uint32_t lanes;      /* lanes per trajectory: 0 = the context's choice
                            (smc_set_lanes_per_trajectory), else 1, 2, 4, 8 or 16 */
} smc_params;

typedef struct {
    double p_hat;          /* successes / n                                      */
    double lo, hi;         /* Wilson interval (eq. 3) at confidence              */
    uint64_t n;            /* trajectories used                                  */
    uint64_t successes;    /* TRUE verdicts among them                           */
    uint64_t events;       /* SSA events (applied transitions) over them         */
    uint64_t truncated;    /* trajectories stopped by max_events                 */
    uint64_t batches;      /* sample-size iterations (1 with fixed_n)            */
    uint64_t wasted;       /* iterative jobs: trajectories issued past the final n
                              (run ahead of a batch decision, or every index up to
                              the capacity in a speculative launch) and discarded;
                              0 with fixed_n                                     */
    double z;              /* z_{1-alpha/2} used                                 */
    double device_seconds; /* kernel time on the device (HIP events)             */
    int32_t status;        /* SMC_OK or the failure of this job                  */
} smc_result;

/* One model: estimate P(formula) to the requested interval.  The trajectory
 * indices used are 0..n-1.  Errors: SMC_E_INVALID (eps <= 0, confidence
 * outside (0,1), unbounded formula with neither t_max nor max_events, sample
 * size above 2^32, more than 255 species), SMC_E_UNSUPPORTED, SMC_E_HIP, SMC_E_TIMEOUT,
 * SMC_E_CANCELLED. */
int smc_estimate(smc_ctx *ctx, const smc_net *net, const smc_formula *f, const smc_params *p,
                 smc_result *out);

/* Many models in one persistent launch; each stops at its own interval width.
 * Networks may differ in size.  out[k] receives job k's result; the return
 * value is the first failure (all jobs are attempted). */
typedef struct {
    const smc_net *net;
    const smc_formula *formula;
    smc_params params;
} smc_job;
int smc_estimate_batch(smc_ctx *ctx, const smc_job *jobs, size_t n_jobs, smc_result *out);

/* Autotuning of a batched launch (smc_estimate_batch), iterative and mixed
 * jobs included (replica parallelism, Sec. 4): lanes per trajectory for the
 * jobs whose lanes are automatic (smc_params.lanes = 0 and context setting
 * 0) and waves per compute unit.  Pilot runs estimate the same jobs with
 * each job's interval half-width widened by pilot_widen (1..64; iterative
 * jobs, about pilot_widen^2 times fewer trajectories by eq. 4) or its fixed
 * size divided by pilot_widen^2 (at least 64), on seeds derived from each
 * job's, so the estimate's own trajectories are not consumed.  A wider
 * interval makes the pilots cheaper but shifts the balance between the
 * throughput-bound bulk of a launch and its latency-bound tail (the longest
 * trajectories take as long either way), so pilot_widen = 1 (the batch as it
 * will run) is the faithful choice.  Candidates: 1, 2, 4, 8 and 16 lanes
 * (when the batch has automatic jobs of more than four channels; upwards until
 * a pilot takes 15 % longer than the best so far; a request that gives the
 * launch the same group size as the previous one, because the widest network
 * needs more lanes, is not timed again) at 16 waves per compute
 * unit, then 8 and 32 waves per compute unit at the best lanes; the shortest
 * device time wins.  The choice
 * is recorded on the context for the batch's signature (the structures of its
 * jobs, in order, and their count; rates, initial states and stopping
 * parameters do not enter): later smc_estimate_batch calls with that
 * signature use it in place of the context's settings, which are otherwise
 * left unchanged.  A second call with the same signature returns the recorded
 * choice without pilots.  Results are identical under every choice (with
 * SMC_TREE_SUMS: the same in distribution).  Errors: SMC_E_INVALID, and those
 * of smc_estimate_batch. */
typedef struct {
    int32_t lanes;           /* lanes per trajectory for the automatic wide jobs
                                (the launch's group size: 1, 2, 4, 8 or 16)    */
    int32_t waves_per_cu;    /* launch shape                                      */
    int32_t candidates;      /* configurations timed                              */
    int32_t pad_;
    double seconds;          /* pilot device time of the choice                   */
    double default_seconds;  /* pilot device time of one lane, 16 waves per CU    */
} smc_batch_tune_result;
int smc_autotune_batch(smc_ctx *ctx, const smc_job *jobs, size_t n_jobs, double pilot_widen,
                       smc_batch_tune_result *out);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * estimates as smc_estimate_batch (bit for bit) for at most
 * SMC_NOALLOC_MAX_JOBS jobs, with no device or pinned-host allocation and no
 * run-time kernel compilation.  The job descriptors, per-job counters and
 * results live in a fixed device array of the library (about 1.1 MB per GPU,
 * held until the process ends, its address looked up when a context is
 * created on that GPU); the kernels clear what must start at zero.  Every
 * call on one GPU shares that array, so calls that overlap on one GPU (from
 * any context or thread) race and must be serialised by the caller.
 * Differences from smc_estimate_batch: iterative jobs always use the batch
 * protocol (a speculative launch would need per-index records); a
 * specialised kernel is used only if one was already compiled on this
 * context for the jobs' structure (SMC_SPECIALIZE_REQUIRED without one gives
 * SMC_E_UNSUPPORTED).  Errors: SMC_E_INVALID (n_jobs above
 * SMC_NOALLOC_MAX_JOBS, or as smc_estimate_batch), and those of
 * smc_estimate_batch. */
#define SMC_NOALLOC_MAX_JOBS 64
int smc_estimate_batch_noalloc(smc_ctx *ctx, const smc_job *jobs, size_t n_jobs, smc_result *out);

/* Per-trajectory results for indices first .. first+count-1 (the same
 * trajectories smc_estimate would draw): events[k] = applied transitions,
 * verdict_reason[k] = verdict | reason << 1.  Either output may be NULL.
 * With SMC_DEVICE_PTRS in p->flags both are device pointers (events 4-byte
 * aligned) that the kernel writes directly; a NULL output is then skipped
 * too.  Errors: SMC_E_INVALID, and those of smc_estimate. */
int smc_trajectories(smc_ctx *ctx, const smc_net *net, const smc_formula *f, const smc_params *p,
                     uint64_t first, uint64_t count, uint32_t *events, uint8_t *verdict_reason);

/* SSA probe: the state sigma@T of trajectories first .. first+count-1,
 * counts[k*S + s] (no formula involved).  With SMC_DEVICE_PTRS in p->flags,
 * counts is a device pointer written in place. */
int smc_sample_state(smc_ctx *ctx, const smc_net *net, const smc_params *p, double T,
                     uint64_t first, uint64_t count, int32_t *counts);

/* Autotuning of the launch configuration (batching of many models into one
 * launch and its shape).  Runs short fixed-size pilot estimates of one model
 * (pilot_n trajectories, 1..2^26, with a seed derived from p->seed, so the
 * estimate's own trajectories are not consumed) for each candidate
 * configuration: generic or specialised kernel, the specialised kernel's
 * register budget (compiler default, 5, 6, 7 or 8 waves per SIMD) and waves
 * per compute unit (4, 8, 16, 24, 28, 32).  The fastest, in SSA events per second of
 * device time, is recorded on the context for the model's structure (network
 * tables and formula; rates, initial state and parameters do not enter): later
 * launches of fixed-size jobs that all share that structure use it in place
 * of the context's settings (smc_set_specialization, smc_set_kernel_occupancy,
 * smc_set_waves_per_cu), which are otherwise left unchanged.  A second call
 * for the same structure returns the recorded choice without pilots.
 * Estimates do not depend on the configuration.  Errors: SMC_E_INVALID, and
 * those of smc_estimate. */
typedef struct {
    int32_t waves_per_cu;         /* chosen launch shape                         */
    int32_t waves_per_simd;       /* chosen register budget (0: compiler's)      */
    int32_t specialization;       /* SMC_SPECIALIZE_AUTO or SMC_SPECIALIZE_OFF    */
    int32_t candidates;           /* configurations timed                        */
    double events_per_s;          /* pilot rate of the choice                    */
    double default_events_per_s;  /* pilot rate of the default configuration     */
} smc_tune_result;
int smc_autotune(smc_ctx *ctx, const smc_net *net, const smc_formula *f, const smc_params *p,
                 uint64_t pilot_n, smc_tune_result *out);

/* ---- Wilson formulas (host, no context) -------------------------------- */
/* z_{1-alpha/2} for confidence 1 - alpha. */
double smc_z_value(double confidence);
/* Eq. 4 before rounding; smc_wilson_sample rounds it up. */
double smc_wilson_sample_value(double p, double eps, double z);
uint64_t smc_wilson_sample(double p, double eps, double z);
/* Eq. 3 for k successes out of n, clipped to [0,1]. */
void smc_wilson_interval(uint64_t k, uint64_t n, double z, double *lo, double *hi);

/* The device's step of Fig. 2 for many (successes, n) pairs: out[k] =
 * ceil(eq. 4 at p = successes[k]/n[k] moved by eps towards 0.5), computed by
 * the same GPU code the persistent kernel uses to pick the next sample size
 * (flags: SMC_PAPER_ROUNDING).  For checking device and host arithmetic
 * against each other.  Errors: SMC_E_INVALID (n[k] == 0, eps outside
 * (0, 0.5)), SMC_E_HIP. */
int smc_wilson_next_device(smc_ctx *ctx, const uint64_t *successes, const uint64_t *n, size_t count,
                           double eps, double z, uint32_t flags, uint64_t *out);

/* ---- surrogate: learned p(rate constants) (MLP 3-256-256-1) -------------
 * A small network maps log10 rate constants (3 per point) to the estimated
 * satisfaction probability.  It is trained on estimates produced by
 * smc_estimate_batch over a parameter sweep, and answers a query only where it
 * is confident: inside the 3-D convex hull of the training points and at
 * least `margin` away from the query threshold; elsewhere the caller runs
 * plain SMC (the fallback that also measures the surrogate's error).
 * Arithmetic: BF16 weights and activations, FP32 accumulation on the GPU's
 * matrix cores (MFMA), FP32 master weights trained with Adam on the GPU.
 * Parameter vector (FP32): W1[256][3], b1[256], W2[256][256] (output-major),
 * b2[256], W3[256], b3, then mu[3], sigma[3] (input standardisation);
 * smc_surrogate_param_count() values in all. */
typedef struct smc_surrogate smc_surrogate;
typedef struct {
    uint32_t steps;   /* full-batch Adam steps                              */
    float lr;         /* learning rate (> 0)                                */
    float beta1;      /* Adam moments (0: 0.9 / 0.999); eps (0: 1e-8)       */
    float beta2;
    float adam_eps;
} smc_train_opts;
/* Seeded Glorot-uniform weights, zero biases, identity standardisation. */
int smc_surrogate_create(smc_ctx *ctx, uint64_t seed, smc_surrogate **out);
size_t smc_surrogate_param_count(void);
int smc_surrogate_set_params(smc_surrogate *s, const float *params, size_t count);
int smc_surrogate_get_params(const smc_surrogate *s, float *params, size_t count);
/* One forward and backward pass over n points: x[n][3] log10 rates, y[n]
 * target probabilities, w[n] weights (NULL: 1).  loss = sum_i w_i BCE(p_i,
 * y_i) / sum_i w_i; grads (optional) receives d loss / d params for the
 * first param_count - 6 values. */
int smc_surrogate_gradients(smc_surrogate *s, const float *x, const float *y, const float *w, size_t n,
                            float *loss, float *grads);
/* Set the standardisation and the training hull from x, then run
 * opts->steps Adam steps on the loss above; loss_out[steps] optional. */
int smc_surrogate_train(smc_surrogate *s, const float *x, const float *y, const float *w, size_t n,
                        const smc_train_opts *opts, float *loss_out);
/* p_out[k] = network output at x[k]; use_surrogate[k] (optional) = 1 when
 * x[k] lies in the training hull and |p_out[k] - threshold| >= margin.
 * flags: 0, or SMC_DEVICE_PTRS when x, p_out and use_surrogate are device
 * pointers on the surrogate's device (read and written in place, no host
 * copies). */
int smc_surrogate_query(smc_surrogate *s, const float *x, size_t n, float threshold, float margin,
                        uint32_t flags, float *p_out, uint8_t *use_surrogate);
/* Calibrate the gate on held-out plain-SMC estimates (points that were not
 * trained on): x[n][3] log10 rates and each point's Wilson interval
 * [lo[k], hi[k]] (eq. 3).  The gate answers a point only if the network's
 * output there, and at the six neighbours x +- delta e_k (delta in log10
 * units, 0 = the point alone), all lie on the same side of the threshold at
 * least m away from it: the point's stability is the least such distance.
 * For each delta in {0, 0.01, 0.02, 0.05, 0.1, 0.2}, m is the smallest value
 * >= min_margin above the stability of every held-out point in the training
 * hull whose output lies more than `bound` outside its interval; the delta
 * that answers the largest share of the held-out points is kept, with its m.
 * From then on smc_surrogate_query (at this threshold) applies that gate.
 * For points drawn like the held-out ones, an answer that lies more than
 * `bound` outside that point's interval has probability at most 1/(n+1)
 * for a fixed delta (exchangeability: it would have to be the largest of
 * n+1 stabilities), at most 6/(n+1) over the six choices.  If no delta
 * gives m <= 0.5, or no held-out point lies in the hull, the gate refuses
 * every query (use_surrogate = 0) until the network is retrained or
 * recalibrated; queries at another threshold are refused too.  Outputs
 * (optional): *margin_out = m (-1 when refused), *share_out = share of the
 * held-out points answered.  Training or setting parameters clears the
 * calibration.  Errors: SMC_E_INVALID. */
int smc_surrogate_calibrate(smc_surrogate *s, const float *x, const double *lo, const double *hi, size_t n,
                            float threshold, float bound, float min_margin, float *margin_out,
                            float *share_out);
/* Confirm answers with a few plain-SMC trajectories per answered point, which
 * the caller runs (e.g. smc_estimate_batch with fixed_n = trials[i], on a
 * seed of its own): p[i] is the surrogate's output and use_surrogate[i] its
 * gate from smc_surrogate_query, successes[i] of trials[i] trajectories
 * satisfied the formula.  An answer on the TRUE side (p >= threshold) stands
 * only if all trials succeeded, one on the FALSE side only if none did; the
 * others are withdrawn (use_surrogate[i] = 0, so the point goes to the SMC
 * fallback).  Entries with use_surrogate[i] = 0 are left alone.  Whatever the
 * network learned, a point whose true probability lies q or more on the other
 * side of its answer (p_true >= q for a FALSE answer, <= 1 - q for a TRUE one)
 * keeps its answer with probability at most (1 - q)^trials[i]: the trials are
 * independent Bernoulli draws of the property (Sec. 3.3).  flags: 0, or
 * SMC_DEVICE_PTRS when all four arrays are device pointers on the
 * surrogate's device (then an entry with more successes than trials
 * withdraws its answer).  Errors: SMC_E_INVALID (null array, unknown flag,
 * threshold outside [0, 1], on host arrays more successes than trials). */
int smc_surrogate_confirm(smc_surrogate *s, const float *p, const uint64_t *successes, const uint64_t *trials,
                          size_t n, float threshold, uint32_t flags, uint8_t *use_surrogate);
/* The calibrated neighbourhood size delta (0 if none or not calibrated). */
float smc_surrogate_neighbourhood(const smc_surrogate *s);
/* Facets of the training hull as planes (nx, ny, nz, d), inside: n.x <= d.
 * Writes up to cap planes; returns the number of facets. */
int smc_surrogate_hull(const smc_surrogate *s, float *planes, size_t cap);
void smc_surrogate_destroy(smc_surrogate *s);
/* The same hull construction without a context (host only): planes of the
 * convex hull of pts[n][3]; returns the number of facets (0 if the points
 * span less than three dimensions), writing up to cap planes. */
int smc_convex_hull(const float *pts, size_t n, float *planes, size_t cap);

#ifdef __cplusplus
}
#endif
#endif /* SMC_H */
