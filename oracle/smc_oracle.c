/*
 * smc_oracle.c -- CPU oracle for on-the-fly statistical model checking of
 * mass-action reaction networks (Ballarini, Forlin, Mazza, Prandi,
 * "Efficient Parallel Statistical Model Checking of Biochemical Networks",
 * PDMC 2009).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, CPU-side reference that
 * the tests, the smoke check and the benchmark's CPU-baseline leg compare the
 * GPU library against.  The product path never links, loads or calls it, and
 * it shares no source with the GPU library.
 *
 * What it computes, in the paper's order:
 *   - direct-method SSA (Sec. 2.2, template steps 1-5, eqs. 1, 2a, 2b):
 *     a_0 from the propensities, j drawn with probability a_j/a_0,
 *     tau drawn from Exp(a_0), x <- x + v_j, t <- t + tau;
 *   - BLTLc semantics (Sec. 3.1, the |= relation) evaluated in three-valued
 *     (Kleene) logic on a finite prefix of the timed path;
 *   - on-the-fly verification (Sec. 3.2): a trajectory stops at the first
 *     prefix on which the formula is decided, with the pessimistic rule for
 *     an undecided formula at t_max, and FALSE at the event cap.
 * The Wilson formulas (Sec. 3.3, eqs. 3-4, Fig. 2) live in oracle/wilson.py.
 *
 * Numeric contract shared (by specification, not by code) with the GPU path:
 *   - Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), key = (seed lo,
 *     seed hi), counter = (event index, trajectory index, model id, 0);
 *   - u1 = ((x0<<21 | x1>>11) + 1) * 2^-53 in (0,1], u2 = (x2<<21 | x3>>11) * 2^-53;
 *   - log built from IEEE +,-,*,/ only (atanh series, ln2 split hi/lo);
 *   - one rounding per propensity; sequential prefix sum in reaction order;
 *   - tau = (-log u1) / a0 (IEEE divide), r = u2 * a0, j = min{j : S_j > r};
 *   - relative time in nested operators = t_j - t_i (one subtraction);
 *   - built with -ffp-contract=off.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11).                                */
/* ------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { /* key schedule: Weyl increments between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------ */
/* Logarithm from IEEE basic operations only.                           */
/* x = m * 2^e with m in [sqrt(1/2), sqrt(2)), f = m - 1 (exact),       */
/* s = f / (2 + f), so that ln m = 2 atanh(s) = 2s + 2s R with           */
/* R = sum_k s^(2k) / (2k + 1).  Since 2s = f - s f and s f = hfsq (1-s) */
/* with hfsq = f^2 / 2,  ln m = f - (hfsq - s (hfsq + 2R)): the exact    */
/* leading term f keeps the rounding error below one ulp.                */
/* ------------------------------------------------------------------ */
double oracle_log(double x)
{
    /* Only positive finite normal inputs occur (u1 >= 2^-53). */
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    int e = (int)((bits >> 52) & 0x7FF) - 1023;
    uint64_t mbits = (bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
    double m;
    memcpy(&m, &mbits, sizeof m);                /* m in [1, 2) */
    const double sqrt2 = 1.4142135623730951;     /* nearest double to sqrt(2) */
    if (m > sqrt2) { m = m * 0.5; e = e + 1; }   /* exact */
    double f = m - 1.0;                          /* exact (Sterbenz) */
    double s = f / (2.0 + f);
    double z = s * s;
    /* R = sum_{k=1..10} z^k / (2k+1), Horner from the highest term. */
    /* Each Horner step and the final product-sum are single fused
     * multiply-adds (C99 fma, one rounding each). */
    double poly = 1.0 / 21.0;
    for (int k = 9; k >= 1; --k) {
        double ck = 1.0 / (double)(2 * k + 1);
        poly = fma(z, poly, ck);
    }
    double R = z * poly;
    double R2 = R + R;
    double hfsq = (0.5 * f) * f;
    const double ln2_hi = 6.93147180369123816490e-01; /* ln 2 with 20 trailing zero bits */
    const double ln2_lo = 1.90821492927058770002e-10; /* ln 2 - ln2_hi */
    double ed = (double)e;
    return ed * ln2_hi - ((hfsq - fma(s, hfsq + R2, ed * ln2_lo)) - f);
}

static inline double u53_open0_closed1(uint32_t a, uint32_t b)
{
    uint64_t v = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)(v + 1u) * 0x1p-53;
}

static inline double u53_closed0_open1(uint32_t a, uint32_t b)
{
    uint64_t v = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)v * 0x1p-53;
}

void oracle_uniforms(const uint32_t r[4], double out[2])
{
    out[0] = u53_open0_closed1(r[0], r[1]);
    out[1] = u53_closed0_open1(r[2], r[3]);
}

/* ------------------------------------------------------------------ */
/* Network (Sec. 2.2): S species, M reaction channels.                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t S, M;
    const int32_t *x0;         /* [S]            */
    const double *rate;        /* [M]   c_j      */
    const int32_t *reactants;  /* [M][2] species index or -1 */
    const int32_t *chg_idx;    /* [M][4] species index or -1 */
    const int32_t *chg_val;    /* [M][4] v_ji    */
} onet;

/* a_j(x): c_j times the number of distinct reactant combinations. */
static double propensity(const onet *n, int j, const int32_t *x)
{
    int ra = n->reactants[2 * j], rb = n->reactants[2 * j + 1];
    double c = n->rate[j];
    if (ra < 0 && rb < 0) return c;
    if (ra < 0) { ra = rb; rb = -1; }
    if (rb < 0) return c * (double)x[ra];
    if (ra == rb) {
        double xa = (double)x[ra];
        double pairs = (xa * (double)(x[ra] - 1)) * 0.5;
        return c * pairs;
    }
    return c * ((double)x[ra] * (double)x[rb]);
}

/* One SSA step from state x at time t using counter k of trajectory idx.
 * Writes the successor state into x (unless absorbing) and returns t'.
 * Also reports a0 (for tests). */
static double ssa_step(const onet *n, uint64_t idx, uint32_t model_id, uint64_t seed,
                       uint32_t k, int32_t *x, double t, double *S, double *a0_out)
{
    /* Step 1: a_0 = sum_j a_j(x), accumulated in reaction order. */
    double acc = 0.0;
    for (int j = 0; j < n->M; ++j) {
        acc = acc + propensity(n, j, x);
        S[j] = acc;
    }
    double a0 = acc;
    if (a0_out) *a0_out = a0;
    if (!(a0 > 0.0)) return INFINITY;            /* absorbing: tau = +inf */
    uint32_t ctr[4] = {k, (uint32_t)idx, model_id, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    double u1 = u53_open0_closed1(r[0], r[1]);
    double u2 = u53_closed0_open1(r[2], r[3]);
    /* Step 2 (eq. 2b): j with probability a_j / a_0. */
    double target = u2 * a0;
    int jsel = -1;
    for (int j = 0; j < n->M; ++j) {
        if (S[j] > target) { jsel = j; break; }
    }
    /* Step 3 (eq. 2a): tau ~ Exp(a_0). */
    double tau = (-oracle_log(u1)) / a0;
    /* Step 4: x <- x + v_j, t <- t + tau. */
    for (int q = 0; q < 4; ++q) {
        int s = n->chg_idx[4 * jsel + q];
        if (s >= 0) x[s] += n->chg_val[4 * jsel + q];
    }
    return t + tau;
}

/* ------------------------------------------------------------------ */
/* BLTLc formulas (Sec. 3.1).  F and G arrive already rewritten by the  */
/* parser as (tt U phi) and not(tt U not phi).                          */
/* ------------------------------------------------------------------ */
enum { N_TRUE = 0, N_FALSE = 1, N_PRED = 2, N_NOT = 3, N_AND = 4, N_OR = 5, N_NEXT = 6, N_UNTIL = 7 };
enum { V_F = 0, V_T = 1, V_U = 2 };                 /* three truth values */
enum { OP_LT = 0, OP_LE, OP_GE, OP_GT, OP_EQ, OP_NE };
/* value-expression stack program opcodes */
enum { E_VAR = 0, E_CONST, E_ADD, E_SUB, E_MUL, E_DIV, E_NEG, E_SQRT, E_POW };

typedef struct {
    int32_t n_nodes, root;
    const int32_t *type;     /* [n_nodes] */
    const int32_t *a, *b;    /* children (or -1) */
    const double *lo, *hi;   /* interval I = [lo, hi] for NEXT / UNTIL */
    const int32_t *pred;     /* predicate id for PRED nodes */
    int32_t n_preds;
    const int32_t *pred_op;  /* [n_preds] comparison */
    const int32_t *lhs_off, *lhs_len, *rhs_off, *rhs_len; /* ranges in the program */
    const int32_t *prog_op;  /* stack program */
    const double *prog_arg;  /* constant or species index */
} oformula;

/* pow(x, y) (Sec. 3.1, func).  The paper does not fix its rounding; read
 * here: for an integral y in 0..64 the product of y factors x formed by
 * binary powering, most significant of seven exponent bits first (square,
 * then multiply where the bit is set, from r = 1), each step one rounded
 * multiplication; any other y takes the C library's pow. */
static double pow_read(double x, double y)
{
    if (y >= 0.0 && y <= 64.0 && y == floor(y)) {
        const int k = (int)y;
        double r = 1.0;
        for (int b = 6; b >= 0; --b) {
            r = r * r;
            if ((k >> b) & 1) r = r * x;
        }
        return r;
    }
    return pow(x, y);
}

static double eval_val(const oformula *f, int off, int len, const int32_t *x)
{
    double st[64];
    int sp = 0;
    for (int p = off; p < off + len; ++p) {
        switch (f->prog_op[p]) {
        case E_VAR: st[sp++] = (double)x[(int)f->prog_arg[p]]; break;
        case E_CONST: st[sp++] = f->prog_arg[p]; break;
        case E_ADD: sp--; st[sp - 1] = st[sp - 1] + st[sp]; break;
        case E_SUB: sp--; st[sp - 1] = st[sp - 1] - st[sp]; break;
        case E_MUL: sp--; st[sp - 1] = st[sp - 1] * st[sp]; break;
        case E_DIV: sp--; st[sp - 1] = st[sp - 1] / st[sp]; break;
        case E_NEG: st[sp - 1] = -st[sp - 1]; break;
        case E_SQRT: st[sp - 1] = sqrt(st[sp - 1]); break;
        case E_POW: sp--; st[sp - 1] = pow_read(st[sp - 1], st[sp]); break;
        }
    }
    return st[0];
}

static int eval_pred(const oformula *f, int k, const int32_t *x)
{
    double l = eval_val(f, f->lhs_off[k], f->lhs_len[k], x);
    double r = eval_val(f, f->rhs_off[k], f->rhs_len[k], x);
    switch (f->pred_op[k]) {
    case OP_LT: return l < r;
    case OP_LE: return l <= r;
    case OP_GE: return l >= r;
    case OP_GT: return l > r;
    case OP_EQ: return l == r;
    default: return l != r;
    }
}

static int not3(int v) { return v == V_U ? V_U : (v == V_T ? V_F : V_T); }
static int and3(int p, int q)
{
    if (p == V_F || q == V_F) return V_F;
    if (p == V_T && q == V_T) return V_T;
    return V_U;
}
static int or3(int p, int q)
{
    if (p == V_T || q == V_T) return V_T;
    if (p == V_F && q == V_F) return V_F;
    return V_U;
}

/* A finite prefix of a timed path: states 0..n-1 with entry times
 * t[0..n-1]; when next_known, t[n] is the time the path leaves state n-1
 * (+inf if state n-1 is absorbing), while state n itself is not yet seen. */
typedef struct {
    int S;
    int64_t n;
    int next_known;
    const int32_t *states;  /* [n][S] */
    const double *t;        /* [n + 1] */
    uint8_t *memo;          /* [n_nodes][n], 0xFF = not computed */
    int64_t *skip;          /* [n_nodes][n + 1], see until_skip (NULL: plain scan) */
    uint8_t *skip_built;    /* [n_nodes] */
} oprefix;

/* 1: scan every position in until (the definition as written); 0: jump over
 * positions that cannot change the scan (until_skip).  Both give the same
 * values; the tests compare them on random paths. */
static int g_plain_scan = 0;
void oracle_set_plain_scan(int on) { g_plain_scan = on; }

static int eval3(const oformula *f, int node, int64_t i, const oprefix *P);

/* In the scan of eval_until, a position where the left operand is T and
 * the right one F changes nothing: or3(res, F) = res and and3(all1, T) =
 * all1.  Only the window test can end the scan there.  skip[k] is the first
 * position >= k that is not of this kind (n if there is none).  Without it a
 * nested until costs time quadratic in the prefix length, since the inner
 * until is scanned from every position of the outer one. */
static const int64_t *until_skip(const oformula *f, int node, const oprefix *P)
{
    int64_t *s = &P->skip[(int64_t)node * (P->n + 1)];
    if (!P->skip_built[node]) {
        s[P->n] = P->n;
        for (int64_t k = P->n - 1; k >= 0; --k) {
            int neutral = eval3(f, f->a[node], k, P) == V_T && eval3(f, f->b[node], k, P) == V_F;
            s[k] = neutral ? s[k + 1] : k;
        }
        P->skip_built[node] = 1;
    }
    return s;
}

static int eval_until(const oformula *f, int node, int64_t i, const oprefix *P)
{
    /* sigma^i |= p1 U^I p2 iff there is j >= i with t_j - t_i in I,
     * sigma^j |= p2 and sigma^l |= p1 for all i <= l < j. */
    double lo = f->lo[node], hi = f->hi[node];
    int res = V_F, all1 = V_T;
    const int64_t *skip = P->skip ? until_skip(f, node, P) : NULL;
    for (int64_t j = i;;) {
        if (j >= P->n) {
            /* State j is not in the prefix. */
            if (P->next_known) {
                double tj = P->t[P->n];
                if (isinf(tj)) break;            /* absorbing: no state j */
                if (tj - P->t[i] > hi) break;    /* window already closed */
            }
            if (all1 != V_F) res = or3(res, V_U);
            break;
        }
        double d = P->t[j] - P->t[i];
        if (d > hi) break;
        if (d >= lo) res = or3(res, and3(all1, eval3(f, f->b[node], j, P)));
        if (res == V_T) break;
        all1 = and3(all1, eval3(f, f->a[node], j, P));
        if (all1 == V_F) break;
        if (!skip) { ++j; continue; }
        /* Positions j+1 .. nj-1 change nothing.  Entry times do not
         * decrease, so the plain scan stops among them iff the last one
         * lies past the window. */
        int64_t nj = skip[j + 1];
        if (nj > j + 1 && P->t[nj - 1] - P->t[i] > hi) break;
        j = nj;
    }
    return res;
}

static int eval_next(const oformula *f, int node, int64_t i, const oprefix *P)
{
    /* sigma^i |= X^I p iff sigma^{i+1} |= p and delta(sigma, i) in I. */
    double lo = f->lo[node], hi = f->hi[node];
    if (i + 1 < P->n) {
        double d = P->t[i + 1] - P->t[i];
        if (!(d >= lo && d <= hi)) return V_F;
        return eval3(f, f->a[node], i + 1, P);
    }
    if (P->next_known) {
        double tn = P->t[P->n];
        if (isinf(tn)) return V_F;
        double d = tn - P->t[i];
        if (!(d >= lo && d <= hi)) return V_F;
    }
    return V_U;
}

static int eval3(const oformula *f, int node, int64_t i, const oprefix *P)
{
    uint8_t *m = P->memo ? &P->memo[(int64_t)node * P->n + i] : NULL;
    if (m && *m != 0xFF) return *m;
    int v;
    switch (f->type[node]) {
    case N_TRUE: v = V_T; break;
    case N_FALSE: v = V_F; break;
    case N_PRED: v = eval_pred(f, f->pred[node], &P->states[(int64_t)i * P->S]) ? V_T : V_F; break;
    case N_NOT: v = not3(eval3(f, f->a[node], i, P)); break;
    case N_AND: {
        int p = eval3(f, f->a[node], i, P);
        v = (p == V_F) ? V_F : and3(p, eval3(f, f->b[node], i, P));
        break;
    }
    case N_OR: {
        int p = eval3(f, f->a[node], i, P);
        v = (p == V_T) ? V_T : or3(p, eval3(f, f->b[node], i, P));
        break;
    }
    case N_NEXT: v = eval_next(f, node, i, P); break;
    default: v = eval_until(f, node, i, P); break;
    }
    if (m) *m = (uint8_t)v;
    return v;
}

/* Three-valued truth of the formula at position 0 of a caller-given prefix. */
int oracle_eval_prefix(const oformula *f, int S, int64_t n, int next_known,
                       const int32_t *states, const double *t)
{
    oprefix P = {S, n, next_known, states, t, NULL, NULL, NULL};
    size_t sz = (size_t)f->n_nodes * (size_t)n;
    P.memo = (uint8_t *)malloc(sz ? sz : 1);
    memset(P.memo, 0xFF, sz);
    if (!g_plain_scan) {
        P.skip = (int64_t *)malloc((size_t)f->n_nodes * (size_t)(n + 1) * sizeof(int64_t));
        P.skip_built = (uint8_t *)calloc((size_t)f->n_nodes, 1);
    }
    int v = eval3(f, f->root, 0, &P);
    free(P.memo); free(P.skip); free(P.skip_built);
    return v;
}

/* ------------------------------------------------------------------ */
/* On-the-fly verification of one trajectory (Sec. 3.2).               */
/* ------------------------------------------------------------------ */
enum { R_STATE = 0, R_TIME = 1, R_ABSORB = 2, R_CAP = 3, R_TMAX = 4 };

typedef struct {
    uint64_t seed;
    uint32_t model_id;
    uint32_t max_events;  /* 0 = no cap */
    double t_max;         /* +inf = none */
} oparams;

typedef struct {
    int32_t *states;   /* [cap_states][S] */
    double *t;         /* [cap_states + 1] */
    double *S;         /* [M] prefix scratch */
    uint8_t *memo;
    int64_t *skip;
    uint8_t *skip_built;
    int64_t cap_states;
    size_t memo_sz, skip_sz;
} oworkspace;

static void ws_reserve(oworkspace *w, int S, int64_t need)
{
    if (need <= w->cap_states) return;
    int64_t c = w->cap_states ? w->cap_states : 64;
    while (c < need) c *= 2;
    w->states = (int32_t *)realloc(w->states, (size_t)c * (size_t)S * sizeof(int32_t));
    w->t = (double *)realloc(w->t, (size_t)(c + 1) * sizeof(double));
    w->cap_states = c;
}

/* Decision test at evaluation point p = 2m + w: the prefix holds states
 * 0..m, and when w = 1 also the time at which state m is left. */
static int decided_at(const oformula *f, const onet *n, const oparams *pr, oworkspace *w,
                      int64_t gen, int absorbed, int64_t p, int *verdict, int *reason)
{
    int64_t m = p >> 1;
    int wnext = (int)(p & 1);
    int64_t len = m + 1;
    int next_known = wnext;
    (void)gen; (void)absorbed;
    size_t need = (size_t)f->n_nodes * (size_t)len;
    if (need > w->memo_sz) {
        w->memo = (uint8_t *)realloc(w->memo, need);
        w->memo_sz = need;
    }
    memset(w->memo, 0xFF, need);
    oprefix P = {n->S, len, next_known, w->states, w->t, w->memo, NULL, NULL};
    if (!g_plain_scan) {
        size_t need_skip = (size_t)f->n_nodes * (size_t)(len + 1);
        if (need_skip > w->skip_sz) {
            w->skip = (int64_t *)realloc(w->skip, need_skip * sizeof(int64_t));
            w->skip_sz = need_skip;
        }
        if (!w->skip_built) w->skip_built = (uint8_t *)malloc((size_t)f->n_nodes);
        memset(w->skip_built, 0, (size_t)f->n_nodes);
        P.skip = w->skip;
        P.skip_built = w->skip_built;
    }
    int v = eval3(f, f->root, 0, &P);
    if (v != V_U) {
        *verdict = (v == V_T);
        if (!wnext) *reason = R_STATE;
        else if (isinf(w->t[m + 1])) *reason = R_ABSORB;
        else *reason = R_TIME;
        return 1;
    }
    /* Pessimistic rule at t_max: once the latest known time exceeds t_max
     * the undecided formula is FALSE.  The first point where this fires is
     * always a w = 1 point; testing it at w = 0 points as well keeps the
     * decision predicate monotone along the points for the bisection. */
    if (w->t[m + (uint64_t)wnext] > pr->t_max) {
        *verdict = 0;
        *reason = R_TMAX;
        return 1;
    }
    if (!wnext && pr->max_events && (uint64_t)m == (uint64_t)pr->max_events) {
        *verdict = 0;
        *reason = R_CAP;
        return 1;
    }
    return 0;
}

int oracle_trajectory(const onet *n, const oformula *f, const oparams *pr, uint64_t idx,
                      oworkspace *w, uint32_t *events, uint8_t *verdict, uint8_t *reason)
{
    int S = n->S;
    ws_reserve(w, S, 64);
    memcpy(w->states, n->x0, (size_t)S * sizeof(int32_t));
    w->t[0] = 0.0;
    int64_t gen = 1;       /* states generated */
    int absorbed = 0;      /* t[gen] == +inf is known */
    int64_t cap = pr->max_events ? (int64_t)pr->max_events : INT64_MAX;
    int64_t target = 16;   /* states wanted before the next decision test */
    int64_t p_lo = 0;      /* every point below p_lo is known undecided */
    for (;;) {
        /* Extend the path (never past state index cap). */
        while (!absorbed && gen - 1 < cap && gen < target) {
            ws_reserve(w, S, gen + 1);
            int32_t *xn = &w->states[gen * S];
            memcpy(xn, &w->states[(gen - 1) * S], (size_t)S * sizeof(int32_t));
            double tn = ssa_step(n, idx, pr->model_id, pr->seed, (uint32_t)(gen - 1), xn,
                                 w->t[gen - 1], w->S, NULL);
            w->t[gen] = tn;
            if (isinf(tn)) absorbed = 1;
            else gen++;
        }
        /* Last evaluation point available with what has been generated. */
        int64_t p_hi;
        if (absorbed) p_hi = 2 * (gen - 1) + 1;
        else p_hi = 2 * (gen - 1);
        int vd, rs;
        int terminal = absorbed || (gen - 1 >= cap);
        if (terminal || decided_at(f, n, pr, w, gen, absorbed, p_hi, &vd, &rs)) {
            /* Binary search for the first decided point in [p_lo, p_hi]. */
            int64_t a = p_lo, b = p_hi;
            while (a < b) {
                int64_t mid = a + (b - a) / 2;
                int v2, r2;
                if (decided_at(f, n, pr, w, gen, absorbed, mid, &v2, &r2)) b = mid;
                else a = mid + 1;
            }
            if (!decided_at(f, n, pr, w, gen, absorbed, a, &vd, &rs)) {
                /* Only reachable at a terminal point that is undecided,
                 * which cannot happen: absorption decides every formula and
                 * the cap point decides by construction. */
                return -1;
            }
            *events = (uint32_t)(a >> 1);
            *verdict = (uint8_t)vd;
            *reason = (uint8_t)rs;
            return 0;
        }
        p_lo = p_hi + 1;
        target *= 2;
    }
}

/* ------------------------------------------------------------------ */
/* Many trajectories on a pthread pool (dynamic chunks of indices).     */
/* ------------------------------------------------------------------ */
typedef struct {
    const onet *n;
    const oformula *f;
    const oparams *pr;
    uint64_t first, count;
    uint32_t *events;
    uint8_t *verdict, *reason;
    volatile int64_t next;
    volatile int err;
    pthread_mutex_t mu;
} ojob;

static void *worker(void *arg)
{
    ojob *J = (ojob *)arg;
    oworkspace w;
    memset(&w, 0, sizeof w);
    w.S = (double *)malloc((size_t)(J->n->M > 0 ? J->n->M : 1) * sizeof(double));
    const int64_t chunk = 16;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        int64_t s = J->next;
        J->next += chunk;
        pthread_mutex_unlock(&J->mu);
        if (s >= (int64_t)J->count) break;
        int64_t e = s + chunk;
        if (e > (int64_t)J->count) e = (int64_t)J->count;
        for (int64_t q = s; q < e; ++q) {
            if (oracle_trajectory(J->n, J->f, J->pr, J->first + (uint64_t)q, &w, &J->events[q],
                                  &J->verdict[q], &J->reason[q]) != 0)
                J->err = 1;
        }
    }
    free(w.states); free(w.t); free(w.S); free(w.memo); free(w.skip); free(w.skip_built);
    return NULL;
}

int oracle_run(int32_t S, int32_t M, const int32_t *x0, const double *rate, const int32_t *reactants,
               const int32_t *chg_idx, const int32_t *chg_val,
               int32_t n_nodes, int32_t root, const int32_t *type, const int32_t *a, const int32_t *b,
               const double *lo, const double *hi, const int32_t *pred, int32_t n_preds,
               const int32_t *pred_op, const int32_t *lhs_off, const int32_t *lhs_len,
               const int32_t *rhs_off, const int32_t *rhs_len, const int32_t *prog_op,
               const double *prog_arg, uint64_t seed, uint32_t model_id, uint32_t max_events,
               double t_max, uint64_t first, uint64_t count, int32_t n_threads, uint32_t *events,
               uint8_t *verdict, uint8_t *reason)
{
    onet n = {S, M, x0, rate, reactants, chg_idx, chg_val};
    oformula f = {n_nodes, root, type, a, b, lo, hi, pred, n_preds, pred_op,
                  lhs_off, lhs_len, rhs_off, rhs_len, prog_op, prog_arg};
    oparams pr = {seed, model_id, max_events, t_max};
    ojob J;
    memset(&J, 0, sizeof J);
    J.n = &n; J.f = &f; J.pr = &pr; J.first = first; J.count = count;
    J.events = events; J.verdict = verdict; J.reason = reason;
    pthread_mutex_init(&J.mu, NULL);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    for (int q = 0; q < n_threads; ++q) pthread_create(&th[q], NULL, worker, &J);
    for (int q = 0; q < n_threads; ++q) pthread_join(th[q], NULL);
    pthread_mutex_destroy(&J.mu);
    return J.err ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Test probes.                                                         */
/* ------------------------------------------------------------------ */

/* Generate up to n_steps SSA steps of trajectory idx, recording states and
 * entry times.  Returns the number of states written (stops early at an
 * absorbing state, in which case times[ret] = +inf). */
int64_t oracle_path(int32_t S, int32_t M, const int32_t *x0, const double *rate,
                    const int32_t *reactants, const int32_t *chg_idx, const int32_t *chg_val,
                    uint64_t seed, uint32_t model_id, uint64_t idx, int64_t n_steps,
                    int32_t *states, double *times, double *a0s)
{
    onet n = {S, M, x0, rate, reactants, chg_idx, chg_val};
    double *Sbuf = (double *)malloc((size_t)(M > 0 ? M : 1) * sizeof(double));
    memcpy(states, x0, (size_t)S * sizeof(int32_t));
    times[0] = 0.0;
    int64_t q;
    for (q = 0; q < n_steps; ++q) {
        int32_t *xn = &states[(q + 1) * S];
        memcpy(xn, &states[q * S], (size_t)S * sizeof(int32_t));
        double a0;
        double tn = ssa_step(&n, idx, model_id, seed, (uint32_t)q, xn, times[q], Sbuf, &a0);
        if (a0s) a0s[q] = a0;
        times[q + 1] = tn;
        if (isinf(tn)) { free(Sbuf); return q + 1; }
    }
    free(Sbuf);
    return n_steps + 1;
}

/* State of trajectory idx at time T (sigma @ T), for SSA marginal tests. */
int oracle_sample_state(int32_t S, int32_t M, const int32_t *x0, const double *rate,
                        const int32_t *reactants, const int32_t *chg_idx, const int32_t *chg_val,
                        uint64_t seed, uint32_t model_id, double T, uint64_t first, uint64_t count,
                        int32_t *out)
{
    onet n = {S, M, x0, rate, reactants, chg_idx, chg_val};
    double *Sbuf = (double *)malloc((size_t)(M > 0 ? M : 1) * sizeof(double));
    int32_t *x = (int32_t *)malloc((size_t)S * sizeof(int32_t));
    int32_t *y = (int32_t *)malloc((size_t)S * sizeof(int32_t));
    for (uint64_t c = 0; c < count; ++c) {
        memcpy(x, x0, (size_t)S * sizeof(int32_t));
        double t = 0.0;
        for (uint32_t k = 0;; ++k) {
            memcpy(y, x, (size_t)S * sizeof(int32_t));
            double tn = ssa_step(&n, first + c, model_id, seed, k, y, t, Sbuf, NULL);
            if (tn > T) break;
            memcpy(x, y, (size_t)S * sizeof(int32_t));
            t = tn;
        }
        memcpy(&out[c * (uint64_t)S], x, (size_t)S * sizeof(int32_t));
    }
    free(Sbuf); free(x); free(y);
    return 0;
}

/* Three-valued evaluation of a formula on a caller-given prefix. */
int oracle_eval(int32_t S, int32_t n_nodes, int32_t root, const int32_t *type, const int32_t *a,
                const int32_t *b, const double *lo, const double *hi, const int32_t *pred,
                int32_t n_preds, const int32_t *pred_op, const int32_t *lhs_off,
                const int32_t *lhs_len, const int32_t *rhs_off, const int32_t *rhs_len,
                const int32_t *prog_op, const double *prog_arg, int64_t n, int32_t next_known,
                const int32_t *states, const double *t)
{
    oformula f = {n_nodes, root, type, a, b, lo, hi, pred, n_preds, pred_op,
                  lhs_off, lhs_len, rhs_off, rhs_len, prog_op, prog_arg};
    return oracle_eval_prefix(&f, S, n, next_known, states, t);
}
