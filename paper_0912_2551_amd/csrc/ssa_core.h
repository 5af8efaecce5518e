// ssa_core.h -- device code of the on-the-fly SSA + BLTLc monitor path for
// gfx950, shared by the generic kernels (ssa_kernel.hip, built ahead of time)
// and by kernels specialised to one network structure and formula (compiled
// at run time by the library, which passes this header to the runtime
// compiler).
//
// One trajectory per lane.  A wave works on one job (model) at a time; idle
// lanes are refilled with new trajectory indices of that job as soon as their
// trajectory is decided, so the wave stays full until the job runs out of
// issuable indices.  Per event and lane:
//   a_j and the running sum S_j in reaction order (Sec. 2.2, template step 1);
//   one Philox4x32-10 block per event, keyed by the job's seed, counter =
//   (event, trajectory, model);
//   tau = -log(u1) / a0 (eq. 2a); j = min{j : S_j > u2 a0} (eq. 2b);
//   x += v_j, t += tau (step 4); monitor update (Sec. 3.2).
// Time and propensity sums are FP64, with no contraction (built with
// -ffp-contract=off), so each lane reproduces the CPU reference bit for bit.
//
// Verdicts are reduced per wave (ballot/popcount) and added atomically to
// per-(job, batch) counters.  Iterative jobs run the Wilson stopping rule
// (eqs. 3-4, Fig. 2) on the device: the lane that completes a batch
// evaluates it and either publishes the next batch bound or finalises the
// job.  While a batch is pending, indices that every possible outcome of the
// batch would still require are issued ahead (no speculative waste).
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#endif

#include "smc_device.h"

namespace smc {

// ---------------------------------------------------------------------------
// Numeric primitives (independent implementation of the numeric contract)
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t a, b, c, d;
};

// a ^ b ^ c in one instruction (gfx950's three-input bit operation; 0x96 is
// the truth table of odd parity).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies, key bumped by the Weyl constants between rounds.
// philox_rounds<R> runs the last R rounds from a given state and round key.
template <int R>
__device__ __forceinline__ U4 philox_rounds(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t m0 = (uint64_t)c0 * 0xD2511F53ull;
        const uint64_t m1 = (uint64_t)c2 * 0xCD9E8D57ull;
        const uint32_t n0 = xor3((uint32_t)(m1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(m0 >> 32), c3, k1);
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}
__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
    return philox_rounds<10>(c0, c1, c2, c3, k0, k1);
}
__device__ __forceinline__ U4 philox9(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
    return philox_rounds<9>(c0, c1, c2, c3, k0, k1);
}

// 53-bit uniforms: (0,1] for the waiting time, [0,1) for the channel.
// v = hi 2^21 + (lo >> 11) is formed as vh 2^32 + vl from two 32-bit words;
// every step below is exact (all values are integers < 2^53, or such integers
// times a power of two), so the results equal (v + 1) 2^-53 and v 2^-53.
__device__ __forceinline__ double unif_oc(uint32_t hi, uint32_t lo)
{
    const double vh = (double)(hi >> 11);
    const double vl = (double)((hi << 21) | (lo >> 11));
    return fma(fma(vh, 0x1p32, vl), 0x1p-53, 0x1p-53);
}
__device__ __forceinline__ double unif_co(uint32_t hi, uint32_t lo)
{
    const double vh = (double)(hi >> 11);
    const double vl = (double)((hi << 21) | (lo >> 11));
    return fma(vh, 0x1p-21, vl * 0x1p-53);
}

// fma(a, b, c) for a constant c, read from scalar registers.  Left to
// itself the compiler keeps loop-invariant FP64 constants in vector registers
// and copies one before each accumulate-in-place multiply-add.
__device__ __forceinline__ double fma_sconst(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// Natural log of a positive normal double from IEEE operations only.
// Reduce x = m 2^e with m in [sqrt(1/2), sqrt(2)); with f = m - 1,
// s = f / (2 + f): ln m = f - (f^2/2 - s (f^2/2 + 2R)), R = sum_k s^2k/(2k+1).
__device__ __forceinline__ double ctr_log(double x)
{
    const uint64_t bits = __double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7FF) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double p = 1.0 / 21.0;
    p = fma_sconst(z, p, 1.0 / 19.0);
    p = fma_sconst(z, p, 1.0 / 17.0);
    p = fma_sconst(z, p, 1.0 / 15.0);
    p = fma_sconst(z, p, 1.0 / 13.0);
    p = fma_sconst(z, p, 1.0 / 11.0);
    p = fma_sconst(z, p, 1.0 / 9.0);
    p = fma_sconst(z, p, 1.0 / 7.0);
    p = fma_sconst(z, p, 1.0 / 5.0);
    p = fma_sconst(z, p, 1.0 / 3.0);
    const double R = z * p;
    const double R2 = R + R;
    const double h = (0.5 * f) * f;
    const double ed = (double)e;
    return ed * 6.93147180369123816490e-01 -
           ((h - fma(s, h + R2, ed * 1.90821492927058770002e-10)) - f);
}

// Eq. 4 (before rounding up), in the contract's operation order.
__device__ __forceinline__ double wilson_n(double p, double eps, double z)
{
    const double pq = p * (1.0 - p);
    const double e2 = eps * eps;
    const double d = p - 0.5;
    const double rad = pq * pq + (4.0 * e2) * (d * d);
    const double num = (pq - 2.0 * e2) + sqrt(rad);
    return (z * z) * num / (2.0 * e2);
}

// Fig. 2 rounding of the estimate towards 0.5 (optionally stopping at 0.5).
__device__ __forceinline__ double towards_half(double p, double eps, int literal)
{
    if (p <= 0.5) {
        const double q = p + eps;
        return literal ? q : fmin(q, 0.5);
    }
    const double q = p - eps;
    return literal ? q : fmax(q, 0.5);
}

__device__ __forceinline__ unsigned long long next_sample(double p_hat, double eps, double z,
                                                          int literal)
{
    return (unsigned long long)ceil(wilson_n(towards_half(p_hat, eps, literal), eps, z));
}

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T ld_relaxed(T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t read_lane_u32(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ unsigned long long read_lane_u64(unsigned long long v, int l)
{
    const uint32_t lo = read_lane_u32((uint32_t)v, l);
    const uint32_t hi = read_lane_u32((uint32_t)(v >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ int ffs64(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }

__device__ __forceinline__ int rank_in(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// ---------------------------------------------------------------------------
// Read-only tables are read through the constant address space: wave-uniform
// reads then compile to scalar loads even though the kernel also writes
// global memory (counters, records).
// ---------------------------------------------------------------------------
#define SMC_CONST __attribute__((address_space(4)))
template <typename T>
using cptr = const SMC_CONST T *;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T *p)
{
    return (cptr<T>)p;
}

// A pointer every lane holds identically, as a wave-uniform (scalar) value, so
// that reads at uniform indices through it become scalar loads.
template <typename T>
__device__ __forceinline__ cptr<T> uniform_ptr(cptr<T> p)
{
    const unsigned long long v = (unsigned long long)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (cptr<T>)(((unsigned long long)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// Per-wave view of a job: uniform values kept in scalar registers.
// ---------------------------------------------------------------------------
struct JobView {
    const Job *job;
    JobState *st;
    cptr<MonProg> mon;
    cptr<int32_t> x0;
    cptr<double> rate;
    cptr<int32_t> reac;
    cptr<uint32_t> chg;
    cptr<ChanDev> chan;
    int S, M, Mp;
    unsigned long long seed, first, capacity;
    uint32_t r1_hi, r1_lo;   // model id * 0xCD9E8D57: first Philox round's product (per job)
    uint32_t max_events;
    double t_max;
    int iterative, literal;
    double eps, z;
    int nb, bs;   // prefix blocks and reactions per block
    int lanes;    // lanes per trajectory
    int trace;    // the formula is a trace program
    uint32_t *rec_events;   // optional per-index outputs
    uint8_t *rec_vr;
    unsigned char *tr_base;   // trace programs: the waves' record areas
    unsigned long long tr_stride;
    uint32_t tr_cap;
    int tr_nskip;

    __device__ void load(const Job *jobs, int j)
    {
        j = __builtin_amdgcn_readfirstlane(j);   // the same job on every lane: scalar loads
        cptr<Job> J = as_const(jobs) + j;
        job = jobs + j;
        st = J->st;
        mon = as_const(J->mon);
        x0 = as_const(J->net.x0);
        rate = as_const(J->net.rate);
        reac = as_const(J->net.reac);
        chg = as_const(J->net.chg);
        chan = as_const(J->net.chan);
        S = J->net.S;
        M = J->net.M;
        Mp = J->net.Mp;
        seed = J->seed;
        first = J->first;
        capacity = J->capacity;
        const uint64_t m1 = (uint64_t)J->model_id * 0xCD9E8D57ull;
        r1_hi = (uint32_t)(m1 >> 32);
        r1_lo = (uint32_t)m1;
        max_events = J->max_events;
        t_max = J->t_max;
        iterative = J->iterative;
        literal = J->literal;
        eps = J->eps;
        z = J->z;
        // blocked prefix (networks of more than four channels): at most
        // kBlocks blocks, each a whole number of kSubBlock-channel steps
        const int nsub = Mp / kSubBlock;
        nb = nsub < kBlocks ? nsub : kBlocks;
        bs = (nsub + nb - 1) / nb * kSubBlock;
        lanes = J->lanes;
        trace = J->trace;
        rec_events = J->rec_events;
        rec_vr = J->rec_vr;
        tr_base = J->tr_base;
        tr_stride = J->tr_stride;
        tr_cap = J->tr_cap;
        tr_nskip = (int)J->tr_nskip;
    }
};

// ---------------------------------------------------------------------------
// Species counts of one lane's trajectory: species-major / lane-minor in the
// wave's LDS slice (consecutive lanes hit consecutive banks).
// ---------------------------------------------------------------------------
struct LdsCounts {
    int32_t *xs;
    int lane;
    __device__ __forceinline__ int32_t get(int s) const { return xs[s * kWave + lane]; }
    // counts of x0, and the constant-1 row S that missing reactants name
    __device__ __forceinline__ void init(cptr<int32_t> x0, int S)
    {
        for (int s = 0; s < S; ++s) xs[s * kWave + lane] = x0[s];
        xs[S * kWave + lane] = 1;
    }
    // the count in the row at byte offset off of the slice
    __device__ __forceinline__ int32_t at(int32_t off) const
    {
        return *reinterpret_cast<const int32_t *>(reinterpret_cast<const char *>(xs + lane) + off);
    }
    // four packed (species, delta) entries
    __device__ __forceinline__ void apply(uint32_t e0, uint32_t e1, uint32_t e2, uint32_t e3)
    {
        const uint32_t e[4] = {e0, e1, e2, e3};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t sp = e[q] >> 16;
            if (sp != 0xFFFFu) xs[sp * kWave + lane] += (int32_t)(int16_t)(e[q] & 0xFFFFu);
        }
    }
};

// ---------------------------------------------------------------------------
// Propensities (contract: one rounding per propensity, c * h(x)).
// ---------------------------------------------------------------------------
template <class C>
__device__ __forceinline__ double propensity(int ra, int rb, double c, const C &X)
{
    if (ra < 0) return c;
    const int32_t xa = X.get(ra);
    if (rb < 0) return c * (double)xa;
    if (ra == rb) return c * (((double)xa * (double)(xa - 1)) * 0.5);
    const int32_t xb = X.get(rb);
    return c * ((double)xa * (double)xb);
}

// The same propensity from counts already read (xa = x[ra], xb = x[rb]),
// without branches: the combinatorial factor h is selected, then c * h.  Each
// case performs the same operations as above (c * 1 = c exactly), so the
// result is identical; the generic kernels use this form because the kinds
// differ from channel to channel.
__device__ __forceinline__ double propensity_x(int ra, int rb, double c, int32_t xa, int32_t xb)
{
    const double da = (double)xa, db = (double)xb;
    const double hetero = da * db;
    const double homo = (da * (double)(xa - 1)) * 0.5;
    const double h = ra < 0 ? 1.0 : (rb < 0 ? da : (ra == rb ? homo : hetero));
    return c * h;
}

// field by field (the tables may sit in the constant address space)
__device__ __forceinline__ ChanDev load_chan(cptr<ChanDev> p)
{
    ChanDev e;
    e.a_off = p->a_off;
    e.b_code = p->b_code;
    return e;
}

// c h with h = (x_a (x_b - delta)) gamma (ChanDev): the same value as
// propensity_x for the channel's form, every factor being exact
__device__ __forceinline__ double chan_propensity(const ChanDev &e, double c, int32_t xa, int32_t xb)
{
    const bool homo = (e.b_code & 1) != 0;
    const double delta = homo ? 1.0 : 0.0, gamma = homo ? 0.5 : 1.0;
    const double h = ((double)xa * ((double)xb - delta)) * gamma;
    return c * h;
}

struct Change {
    uint32_t e0, e1, e2, e3;
};

// ---------------------------------------------------------------------------
// Monitor (compiled BLTLc program).  Per lane: masks of monitors known true
// (tm) and false (fm); nested untils keep "left operand held so far" bits
// (ok) and the latest admissible inner start time (ts, < 0: none).
// ---------------------------------------------------------------------------
struct MonState {
    uint32_t tm, fm, ok;
    double ts0, ts1;
};

// Monitor programs come either from device memory (generic kernels) or from
// a compile-time constant (kernels specialised to one formula).
template <class MP>
struct MonAccess {
    static constexpr bool kMemory = false;
};
template <>
struct MonAccess<cptr<MonProg>> {
    static constexpr bool kMemory = true;
};

// pow(x, k) for an integral k in 0..64 (Sec. 3.1, func), by binary powering:
// from r = 1, for the seven exponent bits from the most significant, square r
// and multiply by x where the bit is set; each step is one rounded FP64
// multiplication, so the value is fixed by k and x alone.
__device__ __forceinline__ double powi(double x, int k)
{
    double r = 1.0;
#pragma unroll
    for (int b = 6; b >= 0; --b) {
        r = r * r;
        r = ((k >> b) & 1) ? r * x : r;
    }
    return r;
}

template <class C>
__device__ __noinline__ double val_eval(cptr<MonProg> mp, int off, int len, const C &X)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int sp = 0;
    for (int o = off; o < off + len; ++o) {
        const int op = mp->vop[o];
        double v;
        if (op == VO_VAR || op == VO_CONST) {
            v = (op == VO_VAR) ? (double)X.get(mp->vvar[o]) : mp->vconst[o];
            if (sp == 0) s0 = v;
            else if (sp == 1) s1 = v;
            else if (sp == 2) s2 = v;
            else s3 = v;
            ++sp;
            continue;
        }
        if (op == VO_NEG || op == VO_SQRT || op == VO_POWI) {
            const double a = sp == 1 ? s0 : sp == 2 ? s1 : sp == 3 ? s2 : s3;
            v = (op == VO_NEG) ? -a : (op == VO_SQRT) ? sqrt(a) : powi(a, mp->vvar[o]);
            if (sp == 1) s0 = v;
            else if (sp == 2) s1 = v;
            else if (sp == 3) s2 = v;
            else s3 = v;
            continue;
        }
        const double b = sp == 2 ? s1 : sp == 3 ? s2 : s3;
        const double a = sp == 2 ? s0 : sp == 3 ? s1 : s2;
        if (op == VO_ADD) v = a + b;
        else if (op == VO_SUB) v = a - b;
        else if (op == VO_MUL) v = a * b;
        else v = a / b;
        --sp;
        if (sp == 1) s0 = v;
        else if (sp == 2) s1 = v;
        else s2 = v;
    }
    return s0;
}

template <typename T>
__device__ __forceinline__ bool compare(T l, T r, int op)
{
    switch (op) {
    case CMP_LT: return l < r;
    case CMP_LE: return l <= r;
    case CMP_GE: return l >= r;
    case CMP_GT: return l > r;
    case CMP_EQ: return l == r;
    default: return l != r;
    }
}

// lo <= x <= hi as one unsigned compare, then negated when asked
template <class PP>
__device__ __forceinline__ bool range_test(int32_t x, PP p)
{
    const uint32_t lo = (uint32_t)p->lo32;
    const bool in = ((uint32_t)x - lo) <= ((uint32_t)p->hi32 - lo);
    return in != (p->neg != 0);
}

// Bit q of the result = truth of predicate q in the current state.
template <class MP, class C>
__device__ __forceinline__ uint32_t eval_preds(MP mp, const C &X)
{
    uint32_t pm = 0;
    const int np = mp->n_preds;
    if (mp->all_var) {
#pragma unroll
        for (int q = 0; q < kMaxPreds; ++q) {
            if (q >= np) break;
            const auto p = &mp->preds[q];
            pm |= (range_test(X.get(p->var), p) ? 1u : 0u) << q;
        }
        return pm;
    }
    for (int q = 0; q < np; ++q) {
        const auto p = &mp->preds[q];
        const int kind = p->kind;
        bool r;
        if (kind == PK_VAR) {
            r = range_test(X.get(p->var), p);
        } else if (kind == PK_LINEAR) {
            long long v = p->c;
            const int nt = p->nterm;
            for (int k = 0; k < nt; ++k) v += p->w[k] * (long long)X.get(p->vars[k]);
            r = compare<long long>(v, 0ll, p->op);
        } else if constexpr (MonAccess<MP>::kMemory) {
            const double l = val_eval(mp, p->lhs_off, p->lhs_len, X);
            const double rr = val_eval(mp, p->rhs_off, p->rhs_len, X);
            r = compare<double>(l, rr, p->op);
        } else {
            r = false;   // arithmetic predicates are never compiled into constant programs
        }
        pm |= (r ? 1u : 0u) << q;
    }
    return pm;
}

// A state formula: lookup in its truth table.
template <class MP>
__device__ __forceinline__ bool prop_val(MP mp, int id, uint32_t pm)
{
    const auto P = &mp->props[id];
    const uint32_t idx = (pm >> P->off) & ((1u << P->cnt) - 1u);
    return (P->table >> idx) & 1u;
}

// Kleene value of the formula from the monitor masks: 0 open, 1 true, 2 false.
template <class MP>
__device__ __forceinline__ uint32_t top_value(MP mp, const MonState &ms)
{
    const int n = mp->n_atoms;
    const uint32_t idx = ms.tm | (ms.fm << n);
    uint64_t wt, wf;
    if (n <= 3) {
        wt = mp->topT[0];
        wf = mp->topF[0];
    } else {
        const uint32_t w = idx >> 6;
        wt = w == 0 ? mp->topT[0] : w == 1 ? mp->topT[1] : w == 2 ? mp->topT[2] : mp->topT[3];
        wf = w == 0 ? mp->topF[0] : w == 1 ? mp->topF[1] : w == 2 ? mp->topF[2] : mp->topF[3];
    }
    const uint32_t b = idx & 63u;
    return ((wt >> b) & 1ull) ? 1u : (((wf >> b) & 1ull) ? 2u : 0u);
}

__device__ __forceinline__ void mon_set(MonState &ms, int a, uint32_t v)
{
    ms.tm |= (v == 1u ? 1u : 0u) << a;
    ms.fm |= (v == 2u ? 1u : 0u) << a;
}

// The monitor updates below are written as selects: a monitor that is already
// decided (or a lane with nothing to inspect) keeps its registers, without a
// lane-divergent branch.

// The state just entered (index k, entry time t) is inspected.
template <class MP, class C>
__device__ __forceinline__ uint32_t mon_step(MP mp, MonState &ms, const C &X, uint32_t k, double t)
{
    const uint32_t pm = eval_preds(mp, X);
    const int na = mp->n_atoms;
#pragma unroll
    for (int a = 0; a < kMaxAtoms; ++a) {
        if (a >= na) break;
        const bool open = !(((ms.tm | ms.fm) >> a) & 1u);
        const auto A = &mp->atoms[a];
        const int kind = A->kind;
        uint32_t v = 0;
        if (kind == AK_PROP) {
            v = prop_val(mp, A->p1, pm) ? 1u : 2u;
        } else if (kind == AK_UNTIL) {
            const bool in_window = (t >= A->lo) && (t <= A->hi);
            const bool hit = in_window && prop_val(mp, A->p2, pm);
            const bool broken = !prop_val(mp, A->p1, pm);
            v = hit ? 1u : (broken ? 2u : 0u);
            if (A->neg) v = v ? 3u - v : 0u;
        } else if (kind == AK_NEXT) {
            v = (k == 1u) ? (prop_val(mp, A->p1, pm) ? 1u : 2u) : 0u;
        } else if (kind == AK_UNTILG) {
            // a p2-break ends the running start; an admissible state (p1 at
            // every earlier one, inside [lo, hi]) with p2 and p3 starts one
            // when none runs; false once none runs and no start can follow
            const bool s0 = A->slot == 0;
            double tc = s0 ? ms.ts0 : ms.ts1;
            const bool q = prop_val(mp, A->p2, pm);
            const uint32_t okb = (ms.ok >> a) & 1u;
            tc = q ? tc : -1.0;
            const bool start = tc < 0.0 && okb && (t >= A->lo) && (t <= A->hi) && q && prop_val(mp, A->p3, pm);
            tc = start ? t : tc;
            const uint32_t ok2 = okb & (prop_val(mp, A->p1, pm) ? 1u : 0u);
            v = (tc < 0.0 && (!ok2 || t > A->hi)) ? 2u : 0u;
            if (open) ms.ok = (ms.ok & ~(1u << a)) | (ok2 << a);
            if (s0) ms.ts0 = open ? tc : ms.ts0;
            else ms.ts1 = open ? tc : ms.ts1;
        } else if (kind == AK_NEXTU) {
            // from state 1 on: the until at position 1, its window measured
            // from state 1's entry time (the X window was checked when time
            // advanced to state 1)
            const bool s0 = A->slot == 0;
            double t1 = s0 ? ms.ts0 : ms.ts1;
            t1 = (k >= 1u && t1 < 0.0) ? t : t1;
            const double rel = t - t1;
            const bool hit = (rel >= A->lo2) && (rel <= A->hi2) && prop_val(mp, A->p2, pm);
            const bool broken = !prop_val(mp, A->p1, pm);
            v = hit ? 1u : (broken ? 2u : 0u);
            if (A->neg) v = v ? 3u - v : 0u;
            v = k >= 1u ? v : 0u;
            if (s0) ms.ts0 = open ? t1 : ms.ts0;
            else ms.ts1 = open ? t1 : ms.ts1;
        } else if (kind == AK_RESP) {
            // a p2-state meets every open obligation (each one's time limit was
            // checked when time advanced to this state); a position of the
            // window where p1 and p2 both fail opens one
            const bool s0 = A->slot == 0;
            double tp = s0 ? ms.ts0 : ms.ts1;
            const bool opens = (t >= A->lo) && (t <= A->hi) && !prop_val(mp, A->p1, pm);
            tp = (opens && tp < 0.0) ? t : tp;
            tp = prop_val(mp, A->p2, pm) ? -1.0 : tp;
            v = (tp < 0.0 && t > A->hi) ? 1u : 0u;
            if (A->neg) v = v ? 3u - v : 0u;
            if (s0) ms.ts0 = open ? tp : ms.ts0;
            else ms.ts1 = open ? tp : ms.ts1;
        } else {   // nested until
            const bool s0 = A->slot == 0;
            const uint32_t okb = (ms.ok >> a) & 1u;
            double tsv = s0 ? ms.ts0 : ms.ts1;
            tsv = (okb && t >= A->lo && t <= A->hi) ? t : tsv;     // new admissible start
            const bool hit = tsv >= 0.0 && prop_val(mp, A->p3, pm);
            tsv = (!hit && !prop_val(mp, A->p2, pm)) ? -1.0 : tsv; // inner left operand broken
            const uint32_t ok2 = okb & (prop_val(mp, A->p1, pm) ? 1u : 0u);
            // with no start pending, false once p has failed or the state
            // lies past the outer window (no later start is admissible)
            v = hit ? 1u : ((tsv < 0.0 && (!ok2 || t > A->hi)) ? 2u : 0u);
            if (open && !hit) ms.ok = (ms.ok & ~(1u << a)) | (ok2 << a);
            if (s0) ms.ts0 = open ? tsv : ms.ts0;
            else ms.ts1 = open ? tsv : ms.ts1;
        }
        mon_set(ms, a, open ? v : 0u);
    }
    return top_value(mp, ms);
}

// Time is about to advance to tn (absorbing: no further state).
template <class MP>
__device__ __forceinline__ uint32_t mon_advance(MP mp, MonState &ms, double tn, bool absorbing)
{
    const int na = mp->n_atoms;
#pragma unroll
    for (int a = 0; a < kMaxAtoms; ++a) {
        if (a >= na) break;
        const bool open = !(((ms.tm | ms.fm) >> a) & 1u);
        const auto A = &mp->atoms[a];
        const int kind = A->kind;
        uint32_t v = 0;
        if (kind == AK_UNTIL) {
            v = (absorbing || tn > A->hi) ? (A->neg ? 1u : 2u) : 0u;
        } else if (kind == AK_NEXT) {
            v = (absorbing || !(tn >= A->lo && tn <= A->hi)) ? 2u : 0u;
        } else if (kind == AK_UNTILG) {
            // the running start holds once its G window is over (or on
            // absorption); with none running, no start may be left
            const double tc = A->slot == 0 ? ms.ts0 : ms.ts1;
            const uint32_t okb = (ms.ok >> a) & 1u;
            v = tc >= 0.0 ? ((absorbing || tn - tc > A->hi2) ? 1u : 0u)
                          : ((!okb || absorbing || tn > A->hi) ? 2u : 0u);
        } else if (kind == AK_NEXTU) {
            // before state 1: the X window; after: the until's window
            const double t1 = A->slot == 0 ? ms.ts0 : ms.ts1;
            if (t1 < 0.0) {
                v = (absorbing || !(tn >= A->lo && tn <= A->hi)) ? 2u : 0u;
            } else {
                v = (absorbing || tn - t1 > A->hi2) ? 2u : 0u;
                if (A->neg) v = v ? 3u - v : 0u;
            }
        } else if (kind == AK_RESP) {
            // the oldest open obligation fails first; with none open, the
            // window's positions are all seen once time passes hi
            const double tp = A->slot == 0 ? ms.ts0 : ms.ts1;
            v = tp >= 0.0 ? ((absorbing || tn - tp > A->hi2) ? 2u : 0u)
                          : ((absorbing || tn > A->hi) ? 1u : 0u);
            if (A->neg) v = v ? 3u - v : 0u;
        } else if (kind == AK_NESTED) {
            const bool s0 = A->slot == 0;
            double tsv = s0 ? ms.ts0 : ms.ts1;
            tsv = (tsv >= 0.0 && (absorbing || tn - tsv > A->hi2)) ? -1.0 : tsv;
            const uint32_t okb = (ms.ok >> a) & 1u;
            v = (tsv < 0.0 && (!okb || absorbing || tn > A->hi)) ? 2u : 0u;
            if (s0) ms.ts0 = open ? tsv : ms.ts0;
            else ms.ts1 = open ? tsv : ms.ts1;
        }
        mon_set(ms, a, open ? v : 0u);
    }
    return top_value(mp, ms);
}

// ms = on ? src : ms, field by field (kept in registers)
__device__ __forceinline__ void ms_select(MonState &ms, const MonState &src, bool on)
{
    ms.tm = on ? src.tm : ms.tm;
    ms.fm = on ? src.fm : ms.fm;
    ms.ok = on ? src.ok : ms.ok;
    ms.ts0 = on ? src.ts0 : ms.ts0;
    ms.ts1 = on ? src.ts1 : ms.ts1;
}

__device__ __forceinline__ void mon_init(MonState &ms)
{
    ms.tm = 0;
    ms.fm = 0;
    ms.ok = 0xFFFFFFFFu;
    ms.ts0 = -1.0;
    ms.ts1 = -1.0;
}

// ---------------------------------------------------------------------------
// Trace programs: formulas outside the compact monitors (deeper nesting,
// temporal left operands of U, windows that do not start at 0 inside other
// operators).  The lane records each state it enters (entry time, predicate
// bits) in its record area, the buffer of Sec. 3.2, and decides the formula
// on that finite prefix in three-valued (Kleene) logic.  Points p = 2m + w:
// states 0..m are known, and with w = 1 also the time state m is left.  A
// point is decided when the formula's value at position 0 is known there, or
// by the t_max rule (the latest known time lies past t_max) or the event
// cap (m = max_events).  Decided stays decided as the prefix grows, so the
// lane tests points only at checkpoints (16 and 32 states, every 64th, 128th
// or 256th iteration of its wave, as the positions a test recomputes grow,
// for all lanes due together, the cap, absorption, t_max)
// and then finds the first decided point by bisection: the trajectory's
// result is the one it would have at that point.
//
// Evaluation is incremental.  After a test that leaves the formula open, each
// node keeps the count of its leading positions whose values no longer
// prefix can change (every state they depend on lies inside the tested
// prefix); later tests, and the bisection, which only looks at longer
// prefixes, recompute each node from that count on.  For a bounded window
// that is the tail of the prefix within the window's reach of its end.
// ---------------------------------------------------------------------------
enum : uint8_t { TV_F = 0, TV_T = 1, TV_U = 2 };

__device__ __forceinline__ uint8_t tv_not(uint8_t v) { return v == TV_U ? TV_U : (uint8_t)(TV_T - v); }
__device__ __forceinline__ uint8_t tv_and(uint8_t x, uint8_t y)
{
    return (x == TV_F || y == TV_F) ? TV_F : ((x == TV_T && y == TV_T) ? TV_T : TV_U);
}
__device__ __forceinline__ uint8_t tv_or(uint8_t x, uint8_t y)
{
    return (x == TV_T || y == TV_T) ? TV_T : ((x == TV_F && y == TV_F) ? TV_F : TV_U);
}

// One lane's view of its wave's record area: element e of an array sits at
// index 64 e of the lane's pointer (the lanes of a wave interleave).
struct TraceRec {
    double *t;
    uint32_t *bits;
    int32_t *need;
    int32_t *fin;
    int32_t *skip;
    uint8_t *val;
    uint32_t cap;
    __device__ __forceinline__ double T(int i) const { return t[(long)i << 6]; }
    __device__ __forceinline__ uint32_t B(int i) const { return bits[(long)i << 6]; }
    __device__ __forceinline__ int32_t &N(int q) const { return need[(long)q << 6]; }
    // final positions of node q: committed (F) and being formed (F2)
    __device__ __forceinline__ int32_t &F(int q) const { return fin[(long)q << 6]; }
    __device__ __forceinline__ int32_t &F2(int q) const { return fin[(long)(q + kMaxTrace) << 6]; }
    // until node q: positions [RS(q), k0) are all neutral (and final)
    __device__ __forceinline__ int32_t &RS(int q) const { return fin[(long)(q + 2 * kMaxTrace) << 6]; }
    __device__ __forceinline__ int32_t &K(int slot, int i) const
    {
        return skip[((long)slot * (cap + 1) + i) << 6];
    }
    __device__ __forceinline__ uint8_t &Vq(int q, int i) const { return val[((long)q * cap + i) << 6]; }
};

__device__ __forceinline__ TraceRec trace_rec(unsigned char *base, unsigned long long stride, uint32_t cap,
                                              int nskip, unsigned long long wave, int lane)
{
    unsigned char *a = base + wave * stride;
    TraceRec R;
    R.t = reinterpret_cast<double *>(a) + lane;
    R.bits = reinterpret_cast<uint32_t *>(a + TraceArea::bits_off(cap)) + lane;
    R.need = reinterpret_cast<int32_t *>(a + TraceArea::need_off(cap)) + lane;
    R.fin = reinterpret_cast<int32_t *>(a + TraceArea::fin_off(cap)) + lane;
    R.skip = reinterpret_cast<int32_t *>(a + TraceArea::skip_off(cap)) + lane;
    R.val = a + TraceArea::val_off(cap, nskip) + lane;
    R.cap = cap;
    return R;
}

// Value at position 0 of the prefix of `len` states (next_known: t[len] is
// the time the last one is left, +inf when it is absorbing).  Nodes are
// evaluated children first, each at the positions its parents read: from
// the root (position 0) down, a NOT, AND or OR reads its operands where it
// is read, a NEXT one position further, an UNTIL every position its scans
// reach (the scan from the last position reaches furthest).  An UNTIL's scan
// jumps over positions where its left operand holds and its right one fails:
// they change neither its result nor whether the left operand has held, so
// only the window can end the scan there, and it does so iff the last of
// them lies past the window.  Each node is recomputed from its committed
// final count on; below that its values, and its until scans' jumps, stand.
__device__ __noinline__ uint32_t trace_value(cptr<MonProg> mp, TraceRec R, int len, bool next_known)
{
    const int nn = mp->tr_n;
    for (int q = 0; q < nn; ++q) R.N(q) = 0;
    R.N(nn - 1) = 1;
    for (int q = nn - 1; q >= 0; --q) {
        const auto &N = mp->tnodes[q];
        const int nq = R.N(q);
        if (nq == 0) continue;
        int e = nq;
        if (N.kind == TN_NEXT) {
            e = nq + 1 < len ? nq + 1 : len;
        } else if (N.kind == TN_UNTIL) {
            // the last j with t_j - t_(nq-1) <= hi, by bisection (entry times
            // do not decrease, so the test holds on a prefix of positions)
            const double ti = R.T(nq - 1);
            int lo_j = nq - 1, hi_j = len;   // t_lo_j - ti <= hi holds; hi_j: first known to fail (or len)
            if (__builtin_isinf(N.hi)) lo_j = len - 1;
            while (hi_j - lo_j > 1) {
                const int mid = lo_j + (hi_j - lo_j) / 2;
                if (R.T(mid) - ti > N.hi) hi_j = mid;
                else lo_j = mid;
            }
            e = lo_j + 1;
        }
        if (N.kind >= TN_NOT) R.N(N.a) = R.N(N.a) > e ? R.N(N.a) : e;
        if (N.kind == TN_AND || N.kind == TN_OR || N.kind == TN_UNTIL) R.N(N.b) = R.N(N.b) > e ? R.N(N.b) : e;
    }
    for (int q = 0; q < nn; ++q) {
        const auto &N = mp->tnodes[q];
        const int kind = N.kind;
        const int nq = R.N(q);
        const int lo = R.F(q);
        // this node's values and its operands' (distinct arrays: the loops
        // below may keep several positions' loads in flight)
        uint8_t *__restrict__ out = R.val + (((long)q * R.cap) << 6);
        const uint8_t *__restrict__ va = N.a >= 0 ? R.val + (((long)N.a * R.cap) << 6) : nullptr;
        const uint8_t *__restrict__ vb = N.b >= 0 ? R.val + (((long)N.b * R.cap) << 6) : nullptr;
        const double *__restrict__ tt = R.t;
        if (kind == TN_TT || kind == TN_FF) {
            const uint8_t c = kind == TN_TT ? TV_T : TV_F;
#pragma unroll 8
            for (int i = lo; i < nq; ++i) out[(long)i << 6] = c;
        } else if (kind == TN_PRED) {
            const uint32_t *__restrict__ bb = R.bits;
            const int bit = N.pred;
#pragma unroll 8
            for (int i = lo; i < nq; ++i) out[(long)i << 6] = ((bb[(long)i << 6] >> bit) & 1u) ? TV_T : TV_F;
        } else if (kind == TN_NOT) {
#pragma unroll 8
            for (int i = lo; i < nq; ++i) out[(long)i << 6] = tv_not(va[(long)i << 6]);
        } else if (kind == TN_AND) {
#pragma unroll 8
            for (int i = lo; i < nq; ++i) out[(long)i << 6] = tv_and(va[(long)i << 6], vb[(long)i << 6]);
        } else if (kind == TN_OR) {
#pragma unroll 8
            for (int i = lo; i < nq; ++i) out[(long)i << 6] = tv_or(va[(long)i << 6], vb[(long)i << 6]);
        } else if (kind == TN_NEXT) {
            // X I a at i: the next state exists, is entered within I after
            // state i, and satisfies a
            for (int i = lo; i < nq; ++i) {
                uint8_t r;
                if (i + 1 < len) {
                    const double d = tt[(long)(i + 1) << 6] - tt[(long)i << 6];
                    r = (d >= N.lo && d <= N.hi) ? va[(long)(i + 1) << 6] : TV_F;
                } else if (next_known) {
                    const double tn = tt[(long)len << 6];
                    const double d = tn - tt[(long)i << 6];
                    r = (__builtin_isinf(tn) || !(d >= N.lo && d <= N.hi)) ? TV_F : TV_U;
                } else {
                    r = TV_U;
                }
                out[(long)i << 6] = r;
            }
        } else {
            // skip[k]: the first position >= k, below the operands' range e,
            // that is not neutral (e where there is none).  Below k0, where
            // both operands are final, the entries stand; each points no
            // further than the k0 of the commit that made it final, so a jump
            // never crosses a position whose operands could still change
            // (it may land on a neutral one, which the scan steps over).
            const int e = R.N(N.a);
            int32_t *__restrict__ sk = R.skip + (((long)N.pred * (R.cap + 1)) << 6);
            const int fa = R.F(N.a), fb = R.F(N.b);
            const int k0 = fa < fb ? fa : fb;
            const int rs = R.RS(q);
            sk[(long)e << 6] = e;
            int nxt = e;
            for (int k = e - 1; k >= k0; --k) {
                const bool neutral = va[(long)k << 6] == TV_T && vb[(long)k << 6] == TV_F;
                nxt = neutral ? nxt : k;
                sk[(long)k << 6] = nxt;
            }
            const double whi = N.hi, wlo = N.lo;
            // ws: the window's first position for i (the first j >= i with
            // t_j - t_i >= lo; it does not decrease with i), and bad: the
            // positions of [i, ws) where a is not known to hold.  With none,
            // the scan from i changes nothing before ws, so it starts there.
            int ws = lo, bad = 0;
            for (int i = lo; i < nq; ++i) {
                // a U I b at i: some j >= i entered within I after state i
                // satisfies b, and a holds at i .. j - 1
                const double ti = tt[(long)i << 6];
                if (i > lo) {
                    if (ws > i - 1) bad -= va[(long)(i - 1) << 6] != TV_T;
                    else ws = i;
                }
                while (ws < len && tt[(long)ws << 6] - ti < wlo) {
                    bad += va[(long)ws << 6] != TV_T;
                    ++ws;
                }
                uint8_t res = TV_F, all = TV_T;
                for (int j = bad == 0 ? ws : i;;) {
                    if (j >= len) {
                        // state j lies past the prefix: it exists unless the
                        // last state is absorbing, and may be in the window
                        // unless its entry time is known to lie past it
                        bool none = false;
                        if (next_known) {
                            const double tj = tt[(long)len << 6];
                            none = __builtin_isinf(tj) || tj - ti > whi;
                        }
                        if (!none && all != TV_F) res = tv_or(res, TV_U);
                        break;
                    }
                    const double d = tt[(long)j << 6] - ti;
                    if (d > whi) break;
                    if (d >= wlo) res = tv_or(res, tv_and(all, vb[(long)j << 6]));
                    if (res == TV_T) break;
                    all = tv_and(all, va[(long)j << 6]);
                    if (all == TV_F) break;
                    // positions j + 1 .. nj - 1 are neutral (nj = the range's
                    // end when they run to it); inside the final neutral run
                    // the jump goes to its end at once
                    int nj = j + 1 < e ? sk[(long)(j + 1) << 6] : j + 1;
                    nj = (j + 1 >= rs && j + 1 < k0 && nj < k0) ? k0 : nj;
                    if (nj > j + 1 && tt[(long)(nj - 1) << 6] - ti > whi) break;
                    j = nj;
                }
                out[(long)i << 6] = res;
            }
        }
    }
    return R.Vq(nn - 1, 0);
}

// After a test of the prefix of `len` states (the time the last one is left
// not yet known) that left the formula open: the new final counts, from the
// need counts of that test, children first.  Position i of a node is final
// when its value is the same on every longer prefix:
//  - a predicate, TT or FF: i < len;
//  - NOT, AND, OR: their operands are final at i;
//  - NEXT: state i + 1 is known and its operand final there;
//  - UNTIL over [lo, hi]: some position F' < len, below both operands' final
//    counts, is entered more than hi after state i; then the scan from i ends
//    at F' at the latest and reads only final values (an unbounded window
//    never qualifies).  Entry times do not decrease, so these positions form
//    a prefix, found by bisection.
// Then the jump entries of each until that become final are bounded by the
// new k0 (see trace_value), its final neutral run is extended over them or
// restarted after the last of them that is not neutral, and the counts are
// committed.  Returns the number of positions left open (over all nodes).
__device__ __noinline__ uint32_t trace_commit(cptr<MonProg> mp, TraceRec R, int len)
{
    const int nn = mp->tr_n;
    for (int q = 0; q < nn; ++q) {
        const auto &N = mp->tnodes[q];
        const int kind = N.kind;
        const int nq = R.N(q);
        int f = nq;
        if (kind == TN_NOT) {
            f = R.F2(N.a);
        } else if (kind == TN_AND || kind == TN_OR) {
            f = R.F2(N.a) < R.F2(N.b) ? R.F2(N.a) : R.F2(N.b);
        } else if (kind == TN_NEXT) {
            f = R.F2(N.a) - 1 < len - 1 ? R.F2(N.a) - 1 : len - 1;
        } else if (kind == TN_UNTIL) {
            int fp = R.F2(N.a) < R.F2(N.b) ? R.F2(N.a) : R.F2(N.b);
            fp = fp < len - 1 ? fp : len - 1;
            f = 0;
            if (!__builtin_isinf(N.hi) && fp > 0) {
                // the first i in [0, fp] with t_fp - t_i > hi false
                const double tf = R.T(fp);
                int a = 0, b = fp;
                while (a < b) {
                    const int mid = a + (b - a) / 2;
                    if (tf - R.T(mid) > N.hi) a = mid + 1;
                    else b = mid;
                }
                f = a;
            }
        }
        f = f < nq ? f : nq;
        R.F2(q) = f > 0 ? f : 0;
    }
    for (int q = 0; q < nn; ++q) {
        const auto &N = mp->tnodes[q];
        if (N.kind != TN_UNTIL) continue;
        const int k0o = R.F(N.a) < R.F(N.b) ? R.F(N.a) : R.F(N.b);
        const int k0n = R.F2(N.a) < R.F2(N.b) ? R.F2(N.a) : R.F2(N.b);
        int32_t *sk = R.skip + (((long)N.pred * (R.cap + 1)) << 6);
        const uint8_t *va = R.val + (((long)N.a * R.cap) << 6);
        const uint8_t *vb = R.val + (((long)N.b * R.cap) << 6);
        int rs = R.RS(q);
        for (int k = k0o; k < k0n; ++k) {
            const int v = sk[(long)k << 6];
            sk[(long)k << 6] = v < k0n ? v : k0n;
            const bool neutral = va[(long)k << 6] == TV_T && vb[(long)k << 6] == TV_F;
            rs = neutral ? rs : k + 1;
        }
        R.RS(q) = rs;
    }
    // the positions left open, which the next test recomputes at least
    uint32_t open = 0;
    for (int q = 0; q < nn; ++q) {
        open += (uint32_t)(R.N(q) - R.F2(q));
        R.F(q) = R.F2(q);
    }
    return open;
}

// Is point p decided?  Then its verdict and reason.
__device__ __noinline__ bool trace_decided(cptr<MonProg> mp, TraceRec R, uint32_t p, double t_max,
                                           uint32_t max_events, uint32_t *verdict, uint32_t *reason)
{
    const uint32_t m = p >> 1, w = p & 1u;
    const uint32_t v = trace_value(mp, R, (int)m + 1, w != 0u);
    if (v != TV_U) {
        *verdict = v == TV_T ? 1u : 0u;
        *reason = w == 0u ? (uint32_t)RS_STATE : (__builtin_isinf(R.T((int)m + 1)) ? (uint32_t)RS_ABSORB : (uint32_t)RS_TIME);
        return true;
    }
    if (R.T((int)(m + w)) > t_max) {   // the pessimistic rule (Sec. 3.2)
        *verdict = 0u;
        *reason = RS_TMAX;
        return true;
    }
    if (w == 0u && max_events != 0u && m == max_events) {
        *verdict = 0u;
        *reason = RS_CAP;
        return true;
    }
    return false;
}

// The first decided point in [lo, hi], hi being decided: its state index
// (the trajectory's event count), verdict and reason.
__device__ __noinline__ void trace_first(cptr<MonProg> mp, TraceRec R, uint32_t lo, uint32_t hi, double t_max,
                                         uint32_t max_events, uint32_t *events, uint32_t *verdict,
                                         uint32_t *reason)
{
    uint32_t vd = 0, rs = 0;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2u;
        if (trace_decided(mp, R, mid, t_max, max_events, &vd, &rs)) hi = mid;
        else lo = mid + 1u;
    }
    trace_decided(mp, R, lo, t_max, max_events, &vd, &rs);
    *events = lo >> 1;
    *verdict = vd;
    *reason = rs;
}

// ---------------------------------------------------------------------------
// The random numbers of event k of a trajectory: one Philox4x32-10 block
// keyed by the seed (wave-uniform: its key schedule runs on the scalar unit),
// counter (k, trajectory, model, 0); nl = -ln(u1) with u1 in
// (0,1], and u2 in [0,1).  They depend on nothing but (trajectory, k), so the
// persistent loop draws those of a lane's next event while the current event
// is still being computed (the two dependency chains overlap).
// ---------------------------------------------------------------------------
struct Draw {
    double nl, u2;
};

__device__ __forceinline__ Draw event_uniforms(const JobView &V, unsigned long long abs_idx, uint32_t k)
{
    // philox10(k, idx, model, 0; seed) with the first round written out: its
    // product of the model id is the job's (r1_hi, r1_lo), and the fourth
    // counter word is 0
    uint32_t k0 = (uint32_t)V.seed, k1 = (uint32_t)(V.seed >> 32);
    const uint64_t m0 = (uint64_t)k * 0xD2511F53ull;
    const uint32_t c0 = xor3(V.r1_hi, k0, (uint32_t)abs_idx);
    const uint32_t c2 = (uint32_t)(m0 >> 32) ^ k1;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    const U4 r = philox9(c0, V.r1_lo, c2, (uint32_t)m0, k0, k1);
    Draw d;
    d.nl = -ctr_log(unif_oc(r.a, r.b));
    d.u2 = unif_co(r.c, r.d);
    return d;
}

// ---------------------------------------------------------------------------
// One SSA event for this lane.  Returns the next time (inf when absorbing)
// and, unless absorbing, the state change of the selected channel.
// ---------------------------------------------------------------------------
// live: this lane steps its trajectory with the result (other lanes compute
// along and discard it).
template <int NB, class C>
__device__ __forceinline__ double draw_tail(const JobView &V, const C &X, const Draw &d, double t,
                                            Change *change, bool live, const double (&P)[NB], double acc);

template <int NB, class C>
__device__ __forceinline__ double ssa_draw(const JobView &V, const C &X, const Draw &d, double t,
                                           Change *change, bool live)
{
    const int M = __builtin_amdgcn_readfirstlane(V.M);
    const int nb = __builtin_amdgcn_readfirstlane(V.nb), bs = __builtin_amdgcn_readfirstlane(V.bs);
    cptr<int32_t> reac = uniform_ptr(V.reac);
    cptr<ChanDev> chan = uniform_ptr(V.chan);
    cptr<double> rate = uniform_ptr(V.rate);
    double P[NB];
    double acc = 0.0;
    if (NB <= 4) {
        // at most four channels, one per block
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j < M) acc = acc + propensity(reac[2 * j], reac[2 * j + 1], rate[j], X);
            P[j] = acc;
        }
    } else {
        // Blocks of whole kSubBlock-channel steps, each step unrolled so that
        // its table and count reads are issued together.  The tables are
        // padded with zero-rate channels to a multiple of kSubBlock: those add
        // exactly 0 to the running sum and are never selected.
        const int Mp = __builtin_amdgcn_readfirstlane(V.Mp);
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            P[q] = acc;
            if (q < nb) {
                const int j0 = q * bs;
                const int j1 = (j0 + bs < Mp) ? j0 + bs : Mp;
                for (int jj = j0; jj < j1; jj += kSubBlock) {
                    // Three phases per step: the channel entries (scalar
                    // loads), then the counts they name (LDS), then the
                    // arithmetic.  Kept apart, each phase waits once: scalar
                    // loads can return out of order, so mixed with LDS reads
                    // on the same wait counter they would force a wait per
                    // read.  One base per step and unsigned offsets let the
                    // compiler merge the step's entries into wide scalar loads.
                    const size_t jb = (size_t)(unsigned)__builtin_amdgcn_readfirstlane(jj);
                    cptr<ChanDev> ep = chan + jb;
                    cptr<double> cp = rate + jb;
                    ChanDev e[kSubBlock];
                    double cr[kSubBlock];
#pragma unroll
                    for (int r = 0; r < kSubBlock; ++r) {
                        e[r] = load_chan(ep + r);
                        cr[r] = cp[r];
                    }
                    int32_t xa[kSubBlock], xb[kSubBlock];
#pragma unroll
                    for (int r = 0; r < kSubBlock; ++r) {
                        xa[r] = X.at(e[r].a_off);
                        xb[r] = X.at(e[r].b_code & ~1);
                    }
#pragma unroll
                    for (int r = 0; r < kSubBlock; ++r)
                        acc = acc + chan_propensity(e[r], cr[r], xa[r], xb[r]);
                }
                P[q] = acc;
            }
        }
    }
    return draw_tail<NB>(V, X, d, t, change, live, P, acc);
}

// The draw after the first pass over the channels: P[q] holds the running
// sum at the end of block q (the total for q >= nb), acc the total a0.
// Selects the block whose running sum first exceeds u2 a0, re-runs the same
// running sum inside it to find the channel, and returns t + tau.
template <int NB, class C>
__device__ __forceinline__ double draw_tail(const JobView &V, const C &X, const Draw &d, double t,
                                            Change *change, bool live, const double (&P)[NB], double acc)
{
    const int M = __builtin_amdgcn_readfirstlane(V.M);
    const int nb = __builtin_amdgcn_readfirstlane(V.nb), bs = __builtin_amdgcn_readfirstlane(V.bs);
    cptr<int32_t> reac = uniform_ptr(V.reac);
    cptr<double> rate = uniform_ptr(V.rate);
    const double a0 = acc;
    if (!(a0 > 0.0)) return __builtin_inf();
    const double target = d.u2 * a0;
    // first block whose running sum exceeds the target (with at most four
    // channels, each channel is a block)
    const int nblk = NB <= 4 ? M : nb;
    int qsel = 0;
    double base = 0.0;
    bool found = false;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if (q < nblk) {
            const bool hit = !found && (P[q] > target);
            qsel = hit ? q : qsel;
            base = hit ? (q == 0 ? 0.0 : P[q - 1]) : base;
            found = found || hit;
        }
    }
    int jsel = qsel;
    if (NB > 4) {
        // Re-run the same running sum inside the selected block (identical
        // operations).  The block differs between lanes, so its table entries
        // are per-lane loads: each step reads its 16 entries first, so that
        // the loads overlap instead of waiting one by one.
        const int Mp = __builtin_amdgcn_readfirstlane(V.Mp);
        const int j0 = qsel * bs;
        const int j1 = (j0 + bs < Mp) ? j0 + bs : Mp;
        double s = base;
        jsel = j1 - 1;
        bool got = !live;
        cptr<ChanDev> chan = V.chan;
        for (int jj = j0; jj < j1; jj += kSubBlock) {
            ChanDev e[kSubBlock];
            double cr[kSubBlock];
#pragma unroll
            for (int r = 0; r < kSubBlock; ++r) {
                e[r] = load_chan(chan + (jj + r));
                cr[r] = rate[jj + r];
            }
            int32_t xa[kSubBlock], xb[kSubBlock];
#pragma unroll
            for (int r = 0; r < kSubBlock; ++r) {
                xa[r] = X.at(e[r].a_off);
                xb[r] = X.at(e[r].b_code & ~1);
            }
#pragma unroll
            for (int r = 0; r < kSubBlock; ++r) {
                s = s + chan_propensity(e[r], cr[r], xa[r], xb[r]);
                const bool hit = !got && s > target;
                jsel = hit ? jj + r : jsel;
                got = got || hit;
            }
            if (__ballot(!got) == 0) break;
        }
    }
    if (NB <= 4) {
        // at most four channels: pick the change among wave-uniform entries
        cptr<uint32_t> tab = uniform_ptr(V.chg);
        Change ch{tab[0], tab[1], tab[2], tab[3]};
#pragma unroll
        for (int q = 1; q < NB; ++q) {
            if (q < M && jsel == q) {
                ch.e0 = tab[4 * q];
                ch.e1 = tab[4 * q + 1];
                ch.e2 = tab[4 * q + 2];
                ch.e3 = tab[4 * q + 3];
            }
        }
        *change = ch;
    } else {
        cptr<uint32_t> chg = V.chg;
        *change = Change{chg[4 * jsel], chg[4 * jsel + 1], chg[4 * jsel + 2], chg[4 * jsel + 3]};
    }
    const double tau = d.nl / a0;
    return t + tau;
}

// ---------------------------------------------------------------------------
// Several lanes per trajectory (generic kernels, networks of more than four
// channels).
//
// A lane group is L consecutive lanes of one 16-lane row (L = 2, 4, 8 or 16)
// running one trajectory.  Every lane of the group holds the same time,
// event index, random numbers and monitor state, and its own copy of the
// counts, so the state change and the monitor run alike on each lane; only
// the pass over the channels is shared out.  The channels are taken in
// rounds of 8 L: in round q, rank r (the lane's index within its group) owns
// the 8 channels from 8 (q L + r) on.  First every lane computes the
// propensities of its 8 channels, all lanes at once.  Then the ranks add
// theirs to the running sum one after the other: rank r starts from the sum
// that rank r - 1 ended with (moved one lane up the row), and rank 0 of the
// next round from the sum that the round's last rank ended with.  These are
// exactly the additions of the sequential prefix in channel order, so the
// total a0 and every partial sum are the one-lane results bit for bit.
// Each lane keeps the sum at the end of its segment of each round.  The
// selected segment is the first whose end exceeds u2 a0 (one ballot per
// round); the group fetches the sum it starts from (the end of the segment
// before it) and re-runs it, every lane alike, to find the channel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dpp_f64_shr1(double v)
{
    // lane i of a 16-lane row receives lane i - 1
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xFFFFFFFFll), 0x111, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Rank 0 of each group of L lanes receives rank L - 1 of the same group: a
// rotation of the 16-lane row by 17 - L (lane i receives lane i - (17 - L)
// modulo 16, which is i + L - 1 within the group).
template <int L>
__device__ __forceinline__ double dpp_f64_last_to_first(double v)
{
    constexpr int ctrl = 0x120 + (17 - L) % 16;
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xFFFFFFFFll), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), ctrl, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ int shfl_i32(int v, int src_lane)
{
    return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}

__device__ __forceinline__ double shfl_f64(double v, int src_lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = shfl_i32((int)(unsigned)(b & 0xFFFFFFFFll), src_lane);
    const int hi = shfl_i32((int)(b >> 32), src_lane);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// The propensities of the 8 channels from j0 on (0 for a segment past the
// tables; such lanes read channels 0..7 and discard them).
template <class C>
__device__ __forceinline__ void segment_propensities(cptr<ChanDev> chan, cptr<double> rate, const C &X, int j0,
                                                     int Mp, double (&a)[kSubBlock])
{
    const bool in = j0 < Mp;
    const int jb = in ? j0 : 0;
    ChanDev e[kSubBlock];
    double cr[kSubBlock];
#pragma unroll
    for (int r = 0; r < kSubBlock; ++r) {
        e[r] = load_chan(chan + (jb + r));
        cr[r] = rate[jb + r];
    }
    int32_t xa[kSubBlock], xb[kSubBlock];
#pragma unroll
    for (int r = 0; r < kSubBlock; ++r) {
        xa[r] = X.at(e[r].a_off);
        xb[r] = X.at(e[r].b_code & ~1);
    }
#pragma unroll
    for (int r = 0; r < kSubBlock; ++r) a[r] = in ? chan_propensity(e[r], cr[r], xa[r], xb[r]) : 0.0;
}

template <int L, class C>
__device__ __forceinline__ double ssa_draw_group(const JobView &V, const C &X, const Draw &d, double t,
                                                 Change *change)
{
    const int Mp = __builtin_amdgcn_readfirstlane(V.Mp);
    const int lane = lane_id();
    const int rank = lane & (L - 1);
    const int gbase = lane - rank;
    const int rounds = (Mp + kSubBlock * L - 1) / (kSubBlock * L);   // at most kMaxGroupRounds (host)
    cptr<ChanDev> chan = V.chan;
    cptr<double> rate = V.rate;
    double seg_hi[kMaxGroupRounds];   // the running sum at the end of this lane's segment of each round
    double cur = 0.0;                 // the running sum this lane last ended a segment with
#pragma unroll
    for (int q = 0; q < kMaxGroupRounds; ++q) {
        seg_hi[q] = 0.0;
        if (q < rounds) {
            double a[kSubBlock];
            segment_propensities(chan, rate, X, (q * L + rank) * kSubBlock, Mp, a);
            // rank 0 continues from the sum the previous round's last rank ended with
            double in = q == 0 ? 0.0 : dpp_f64_last_to_first<L>(cur);
#pragma unroll
            for (int rr = 0; rr < L; ++rr) {
                if (rr > 0) in = dpp_f64_shr1(cur);   // rank rr: the sum rank rr - 1 ended with
                double s = in;
#pragma unroll
                for (int r = 0; r < kSubBlock; ++r) s = s + a[r];
                cur = rank == rr ? s : cur;
            }
            seg_hi[q] = cur;
        }
    }
    // the total: the end of the last rank's segment of the last round
    const double a0 = shfl_f64(cur, gbase + L - 1);
    const double target = d.u2 * a0;
    // first segment (round, rank) whose end exceeds the target
    const uint64_t gbits = (1ull << L) - 1ull;
    int qsel = 0, rsel = L - 1;
    bool found = false;
#pragma unroll
    for (int q = 0; q < kMaxGroupRounds; ++q) {
        if (q < rounds) {
            const uint64_t g = (__ballot(seg_hi[q] > target) >> gbase) & gbits;
            const bool hit = !found && g != 0ull;
            qsel = hit ? q : qsel;
            rsel = hit ? ffs64(g) : rsel;
            found = found || hit;
        }
    }
    // The selected segment starts where the previous one ended: rank rsel - 1
    // of round qsel, or the last rank of round qsel - 1 (0 before the first).
    // Every lane of the group fetches that sum and re-runs the selected
    // segment with identical operations.
    const int qprev = rsel > 0 ? qsel : qsel - 1;
    double prov = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxGroupRounds; ++q) prov = q == qprev ? seg_hi[q] : prov;
    double s = shfl_f64(prov, gbase + (rsel > 0 ? rsel - 1 : L - 1));
    s = qprev < 0 ? 0.0 : s;
    const int j0 = (qsel * L + rsel) * kSubBlock;
    double a[kSubBlock];
    segment_propensities(chan, rate, X, j0, Mp, a);
    int jsel = j0 + kSubBlock - 1;
    bool got = false;
#pragma unroll
    for (int r = 0; r < kSubBlock; ++r) {
        s = s + a[r];
        const bool hit = !got && s > target;
        jsel = hit ? j0 + r : jsel;
        got = got || hit;
    }
    jsel = jsel < Mp ? jsel : Mp - 1;   // only where nothing fires (a0 = 0, the change is unused)
    cptr<uint32_t> chg = V.chg;
    *change = Change{chg[4 * jsel], chg[4 * jsel + 1], chg[4 * jsel + 2], chg[4 * jsel + 3]};
    const double tau = d.nl / a0;
    return a0 > 0.0 ? t + tau : __builtin_inf();
}

// ---------------------------------------------------------------------------
// A direct-method variant for wide networks with tree-ordered sums (selected
// per job with SMC_TREE_SUMS; the statistical contract).
//
// Lane r of a group of L owns one contiguous block of the channels, at most
// kMaxGroupRounds steps of kSubBlock.  It adds its block's propensities in
// channel order and keeps the running sum at the end of each step.  The group
// forms the sums before and through each lane's block with a Hillis-Steele
// scan (log2 L DPP steps inside the 16-lane row); a0 is the scan's last value.
// The first lane whose scan value exceeds u2 a0 holds the channel: it looks up
// the step, and then the channel, against the local target u2 a0 - (sum before
// its block), and the re-run of that step reproduces its kept sums exactly.
//
// Channel j is still drawn with probability a_j / a0 and tau from Exp(a0), but
// a0 and the boundaries are associated differently from the sequential prefix
// of Sec. 2.1 and differ from it in the last bits.  The results therefore
// agree with the sequential kernels in distribution, and trajectory by
// trajectory except where a draw falls within a few ulps of a boundary; event
// times differ in the last bits.  Where re-association leaves a target just
// outside the selected block's own sums, the choice falls on the block's first
// or last channel of positive propensity, so a channel that cannot fire is
// never drawn.
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ double dpp_f64_shr(double v)
{
    // lane i of a 16-lane row receives lane i - K (0 where that leaves the row)
    constexpr int ctrl = 0x110 + K;
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xFFFFFFFFll), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), ctrl, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <int L, class C>
__device__ __forceinline__ double ssa_draw_tree(const JobView &V, const C &X, const Draw &d, double t,
                                                Change *change)
{
    const int Mp = __builtin_amdgcn_readfirstlane(V.Mp);
    const int lane = lane_id();
    const int rank = lane & (L - 1);
    const int gbase = lane - rank;
    const int nsub = (Mp + kSubBlock * L - 1) / (kSubBlock * L);   // at most kMaxGroupRounds (host)
    const int jb = rank * nsub * kSubBlock;
    cptr<ChanDev> chan = V.chan;
    cptr<double> rate = V.rate;
    double sub[kMaxGroupRounds];   // this lane's running block sum at the end of each step
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxGroupRounds; ++q) {
        if (q < nsub) {
            double a[kSubBlock];
            segment_propensities(chan, rate, X, jb + q * kSubBlock, Mp, a);
#pragma unroll
            for (int r = 0; r < kSubBlock; ++r) acc = acc + a[r];
        }
        sub[q] = acc;
    }
    // inclusive scan of the block sums over the group
    double inc = acc;
    if (L > 1) { const double v = dpp_f64_shr<1>(inc); inc = rank >= 1 ? inc + v : inc; }
    if (L > 2) { const double v = dpp_f64_shr<2>(inc); inc = rank >= 2 ? inc + v : inc; }
    if (L > 4) { const double v = dpp_f64_shr<4>(inc); inc = rank >= 4 ? inc + v : inc; }
    if (L > 8) { const double v = dpp_f64_shr<8>(inc); inc = rank >= 8 ? inc + v : inc; }
    double excl = dpp_f64_shr<1>(inc);
    excl = rank >= 1 ? excl : 0.0;
    const double a0 = shfl_f64(inc, gbase + L - 1);
    const double target = d.u2 * a0;
    // the block: the first lane of positive sum whose scan value exceeds the
    // target, else the last lane of positive sum
    const uint64_t gbits = (1ull << L) - 1ull;
    const uint64_t pos = (__ballot(acc > 0.0) >> gbase) & gbits;
    const uint64_t hit = (__ballot(acc > 0.0 && inc > target) >> gbase) & gbits;
    const int rsel = hit ? ffs64(hit) : (pos ? 63 - __builtin_clzll(pos) : L - 1);
    // every lane finds the step and channel in its own block; the group takes
    // lane rsel's.  Step: the first whose kept sum exceeds the local target,
    // else the last that adds a positive amount.
    const double tl = target - excl;
    int qs = 0;
    bool found = false;
    double prev = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxGroupRounds; ++q) {
        if (q < nsub && !found) {
            const bool grows = sub[q] > prev;
            qs = grows ? q : qs;
            found = grows && sub[q] > tl;
            prev = sub[q];
        }
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxGroupRounds; ++q) s = q + 1 == qs ? sub[q] : s;
    const int j0 = jb + qs * kSubBlock;
    double a[kSubBlock];
    segment_propensities(chan, rate, X, j0, Mp, a);
    int js = j0;
    bool got = false;
#pragma unroll
    for (int r = 0; r < kSubBlock; ++r) {
        s = s + a[r];
        if (!got) {
            js = a[r] > 0.0 ? j0 + r : js;
            got = a[r] > 0.0 && s > tl;
        }
    }
    int jsel = shfl_i32(js, gbase + rsel);
    jsel = jsel < Mp ? jsel : Mp - 1;   // only where nothing fires (a0 = 0, the change is unused)
    cptr<uint32_t> chg = V.chg;
    *change = Change{chg[4 * jsel], chg[4 * jsel + 1], chg[4 * jsel + 2], chg[4 * jsel + 3]};
    const double tau = d.nl / a0;
    return a0 > 0.0 ? t + tau : __builtin_inf();
}

// ---------------------------------------------------------------------------
// Access policies of the persistent loop.
//
// DynPolicy: the generic kernels.  Network and monitor tables are read from
// device memory through the job's pointers; counts live in LDS.
//
// StaticPolicy<Spec>: kernels specialised to one network structure and one
// formula (compiled at run time).  Spec supplies, as compile-time constants,
//   static constexpr int S, M;               species and channels
//   static constexpr NetTab<M> net;          reactants and packed changes
//   static constexpr MonProg mon;            compiled formula (no RPN predicates)
// Rate constants and initial counts still come from the job in device
// memory, so one specialised kernel serves every rate set of a sweep.  Counts
// live in registers; every table index is an immediate.  The arithmetic is
// the same sequence of operations as the generic path.
// ---------------------------------------------------------------------------
// G > 1: the kernel also runs jobs with G lanes per trajectory (kernels of
// their own, one per group size, so that each keeps its registers: the
// one-lane kernels as before, and a grouped kernel without spills).
template <int NB, int G = 1, bool kTree = false>
struct DynPolicy {
    using Counts = LdsCounts;
    using Sel = Change;
    static constexpr bool kGroups = G > 1 && NB > 4;
    __device__ static __forceinline__ Counts counts(int32_t *lds, int wid, int s_max, int lane)
    {
        Counts X;
        X.xs = lds + (size_t)wid * (size_t)(s_max + 1) * kWave;   // + the constant-1 row
        X.lane = lane;
        return X;
    }
    __device__ static __forceinline__ void init(Counts &X, const JobView &V)
    {
        X.init(uniform_ptr(V.x0), __builtin_amdgcn_readfirstlane(V.S));
    }
    __device__ static __forceinline__ double draw(const JobView &V, const Counts &X, const Draw &d,
                                                  double t, Sel *s, bool live)
    {
        if (kGroups && __builtin_amdgcn_readfirstlane(V.lanes) == G)
            return kTree ? ssa_draw_tree<(G > 1 ? G : 2)>(V, X, d, t, s)
                         : ssa_draw_group<(G > 1 ? G : 2)>(V, X, d, t, s);
        return ssa_draw<NB>(V, X, d, t, s, live);
    }
    __device__ static __forceinline__ void apply_if(Counts &X, const Sel &c, bool on)
    {
        if (on) X.apply(c.e0, c.e1, c.e2, c.e3);
    }
    __device__ static __forceinline__ uint32_t step(const JobView &V, MonState &ms, const Counts &X,
                                                    uint32_t k, double t)
    {
        return mon_step(uniform_ptr(V.mon), ms, X, k, t);
    }
    __device__ static __forceinline__ uint32_t advance(const JobView &V, MonState &ms, double tn,
                                                       bool absorbing)
    {
        return mon_advance(uniform_ptr(V.mon), ms, tn, absorbing);
    }
};

template <int M>
struct NetTab {
    int32_t reac[2 * M];
    uint32_t chg[4 * M];
};

template <int S>
struct RegCounts {
    int32_t x[S];
    __device__ __forceinline__ int32_t get(int s) const { return x[s]; }
};

template <class Spec>
struct StaticPolicy {
    static constexpr int S = Spec::S;
    static constexpr int M = Spec::M;
    static constexpr bool kGroups = false;
    using Counts = RegCounts<S>;
    using Sel = int;
    __device__ static __forceinline__ Counts counts(int32_t *, int, int, int) { return Counts{}; }
    __device__ static __forceinline__ void init(Counts &X, const JobView &V)
    {
#pragma unroll
        for (int s = 0; s < S; ++s) X.x[s] = V.x0[s];
    }
    __device__ static __forceinline__ double draw(const JobView &V, const Counts &X, const Draw &d,
                                                  double t, Sel *jsel, bool)
    {
        constexpr NetTab<M> T = Spec::net;
        cptr<double> rate = V.rate;
        double P[M];
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            acc = acc + propensity(T.reac[2 * j], T.reac[2 * j + 1], rate[j], X);
            P[j] = acc;
        }
        const double a0 = acc;
        const double target = d.u2 * a0;
        // u2 < 1 makes target < a0 = P[M-1], so some channel always qualifies
        int js = M - 1;
#pragma unroll
        for (int j = M - 2; j >= 0; --j) js = (P[j] > target) ? j : js;
        *jsel = js;
        // computed on every lane and discarded where a0 = 0 (absorbing): a
        // select keeps the event in one basic block
        const double tau = d.nl / a0;
        return a0 > 0.0 ? t + tau : __builtin_inf();
    }
    __device__ static __forceinline__ void apply_if(Counts &X, Sel js, bool on)
    {
        constexpr NetTab<M> T = Spec::net;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const bool hit = on && js == j;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t e = T.chg[4 * j + q];
                const uint32_t sp = e >> 16;
                if (sp != 0xFFFFu) X.x[sp] += hit ? (int32_t)(int16_t)(e & 0xFFFFu) : 0;
            }
        }
    }
    __device__ static __forceinline__ uint32_t step(const JobView &, MonState &ms, const Counts &X,
                                                    uint32_t k, double t)
    {
        constexpr MonProg mp = Spec::mon;
        return mon_step(&mp, ms, X, k, t);
    }
    __device__ static __forceinline__ uint32_t advance(const JobView &, MonState &ms, double tn,
                                                       bool absorbing)
    {
        constexpr MonProg mp = Spec::mon;
        return mon_advance(&mp, ms, tn, absorbing);
    }
};

// Kernels specialised to a wide network (more channels or species than
// StaticPolicy keeps in registers).  Counts live in LDS as in the generic
// kernels; the first pass over the channels, the bulk of an event, reads
// reactant indices as compile-time constants and every count once per event,
// so each channel costs only its propensity arithmetic.  The block selection,
// the re-run of the selected block and the state change are the generic
// kernels' (per-lane table reads; the block differs between lanes).  The
// operations and their order are the generic kernels', so results are
// identical.
template <int M>
struct ReacTab {
    int32_t reac[2 * M];
};

template <class Spec>
struct StaticWidePolicy {
    static constexpr int S = Spec::S;
    static constexpr int M = Spec::M;
    static constexpr int Mp = (M + kSubBlock - 1) / kSubBlock * kSubBlock;
    // the generic kernels' blocking (JobView::load)
    static constexpr int kNsub = Mp / kSubBlock;
    static constexpr int kNb = kNsub < kBlocks ? kNsub : kBlocks;
    static constexpr int kBs = (kNsub + kNb - 1) / kNb * kSubBlock;
    static constexpr bool kGroups = false;
    using Counts = LdsCounts;
    using Sel = Change;
    __device__ static __forceinline__ Counts counts(int32_t *lds, int wid, int, int lane)
    {
        Counts X;
        X.xs = lds + (size_t)wid * (size_t)(S + 1) * kWave;   // + the constant-1 row
        X.lane = lane;
        return X;
    }
    __device__ static __forceinline__ void init(Counts &X, const JobView &V) { X.init(uniform_ptr(V.x0), S); }
    __device__ static __forceinline__ double draw(const JobView &V, const Counts &X, const Draw &d,
                                                  double t, Sel *s, bool live)
    {
        constexpr ReacTab<M> T = Spec::wide;
        cptr<double> rate = uniform_ptr(V.rate);
        int32_t x[S];
#pragma unroll
        for (int q = 0; q < S; ++q) x[q] = X.get(q);
        double P[kBlocks];
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < kBlocks; ++q) {
            P[q] = acc;
            if (q < kNb) {
#pragma unroll
                for (int j = q * kBs; j < (q + 1) * kBs && j < Mp; ++j) {
                    const int ra = j < M ? T.reac[2 * j] : -1;
                    const int rb = j < M ? T.reac[2 * j + 1] : -1;
                    acc = acc + propensity_x(ra, rb, rate[j], ra < 0 ? 0 : x[ra], rb < 0 ? 0 : x[rb]);
                }
                P[q] = acc;
            }
        }
        return draw_tail<kBlocks>(V, X, d, t, s, live, P, acc);
    }
    __device__ static __forceinline__ void apply_if(Counts &X, const Sel &c, bool on)
    {
        if (on) X.apply(c.e0, c.e1, c.e2, c.e3);
    }
    __device__ static __forceinline__ uint32_t step(const JobView &, MonState &ms, const Counts &X, uint32_t k,
                                                    double t)
    {
        constexpr MonProg mp = Spec::mon;
        return mon_step(&mp, ms, X, k, t);
    }
    __device__ static __forceinline__ uint32_t advance(const JobView &, MonState &ms, double tn, bool absorbing)
    {
        constexpr MonProg mp = Spec::mon;
        return mon_advance(&mp, ms, tn, absorbing);
    }
};

// ---------------------------------------------------------------------------
// Stopping rule on the device.
// ---------------------------------------------------------------------------
__device__ unsigned long long sum_shards(unsigned long long (*arr)[kShards], int b)
{
    unsigned long long s = 0;
#pragma unroll 1
    for (int q = 0; q < kShards; ++q) s += ld_relaxed(&arr[b][q]);
    return s;
}

// A 64-bit value every lane holds identically, as a wave-uniform value.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) { return read_lane_u64(v, 0); }

// Ordering of the stopping-rule state.  Every access to it is an atomic
// operation at agent scope (read-modify-writes, and atomic loads and stores),
// so each location is coherent for the whole device; what needs care is the
// order in which a wave sees writes to *different* locations.  The batch of a
// finished trajectory is read from the published bounds, and an index of
// batch c+1 can only be claimed once the issue limit has passed bound[c].  So
// a wave that claims an index below a limit value must see every bound that
// the wave which raised the limit had seen or written.  That is the
// message-passing pattern of the HIP (C++) memory model:
//  - every raise of the limit (evaluate_batches, speculate) comes after a
//    release fence at agent scope;
//  - the limit load of an iterative claim is an acquire;
//  - a publishing wave also fences (release) before it stores the new bound,
//    and a wave that reads a bound in order to raise the limit (speculate),
//    or that completes a batch and evaluates it, fences (acquire) after the
//    read; so the chain bound -> limit -> claim holds through any number of
//    waves (read-read coherence covers the bound values read on the way).
// A release fence writes back this XCD's L2 and an acquire fence
// invalidates it; both run once per batch, per look-ahead step (one per 64
// completions at most) or per claim (one per 64 indices at least), never per
// event.  Fixed-size jobs never raise the limit and take none of them.
__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ unsigned long long ld_acquire(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_relaxed(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed_i32(int32_t *p, int32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of the TRUE verdicts of batches 0 .. b-1 (all complete, so their
// counter words no longer change), read by the whole wave in one round trip.
__device__ __forceinline__ unsigned long long yes_before(JobState *st, int b)
{
    const int lane = lane_id();
    unsigned long long v = 0;
    if (lane < b) v = ld_relaxed(&st->cnt[lane]) >> 32;
    return wave_sum_u64(v);
}

// Batch b is complete (its counter word is cw): apply Fig. 2.  Either the
// next bound is published (and, if that batch is complete already, it is
// evaluated in turn), or the job is finalised.  The whole wave runs this;
// exactly one wave evaluates each batch.
__device__ void evaluate_batches(const JobView &V, Control *ctl, int b, unsigned long long cw)
{
    JobState *st = V.st;
    const int lane = lane_id();
    for (;;) {
        const unsigned long long Y = yes_before(st, b) + (cw >> 32);
        const unsigned long long Bb = uniform_u64(ld_relaxed(&st->bound[b]));
        const double p_hat = (double)Y / (double)Bb;
        const unsigned long long Np = uniform_u64(next_sample(p_hat, V.eps, V.z, V.literal));
        // Indices up to the look-ahead limit may already be running as part
        // of the next batch; the look-ahead is a lower bound of Np (the
        // smallest Fig. 2 bound over the possible outcomes), so a smaller Np
        // would mean a miscounted batch: the job then stops with an error
        // instead.
        const unsigned long long lim_now = uniform_u64(ld_relaxed(&st->limit));
        if (Np > Bb && Np < lim_now) {
            if (lane == 0) {
                st->n_final = Bb;
                st->yes_final = Y;
                st->n_batches = b + 1;
                st->overflow = 2;
                st_relaxed_i32(&st->final_flag, 1);
                atomicSub(&ctl->open_jobs, 1);
            }
            return;
        }
        if (Np > Bb && b + 1 < kMaxBatches && Np <= V.capacity) {
            unsigned long long old = 0;
            const unsigned long long flag = kDoneFlag - (Np - Bb);
            fence_release();
            if (lane == 0) {
                // the bound is in place before any index of the new batch can
                // be claimed, and before the batch can be seen complete
                st_relaxed(&st->bound[b + 1], Np);
                st_relaxed_i32(&st->cur, b + 1);
                fence_release();
                atomicMax(&st->limit, Np);
                old = atomicAdd(&st->cnt[b + 1], flag);
            }
            const unsigned long long now = read_lane_u64(old, 0) + flag;
            if ((now & 0xFFFFFFFFull) == kDoneFlag) {
                fence_acquire();
                b = b + 1;
                cw = now;
                continue;
            }
            return;
        }
        if (lane == 0) {
            st->n_final = Bb;
            st->yes_final = Y;
            st->n_batches = b + 1;
            st->overflow = (Np > Bb) ? 1 : 0;
            st_relaxed_i32(&st->final_flag, 1);
            atomicSub(&ctl->open_jobs, 1);
        }
        return;
    }
}

// While batch c is pending (counter word cw, as last seen), raise the issue
// limit to the smallest next bound that any possible outcome of batch c
// would produce: the bound grows as the estimate moves towards 0.5, so the
// smallest is at one of the two extreme outcomes (all remaining FALSE, or all
// TRUE), computed with the very operations the evaluation will use.  Counts
// seen here can only lag, which widens the range of outcomes and lowers the
// bound.  The whole wave runs this.
__device__ void speculate(const JobView &V, int c, unsigned long long cw)
{
    JobState *st = V.st;
    const unsigned long long Bc = uniform_u64(ld_relaxed(&st->bound[c]));
    const unsigned long long Bp = c ? uniform_u64(ld_relaxed(&st->bound[c - 1])) : 0ull;
    if (Bc == 0) return;
    const unsigned long long size = Bc - Bp;
    const unsigned long long low = cw & 0xFFFFFFFFull;
    // the low word holds the completions, plus kDoneFlag - size once the
    // bound is published (it is: Bc is known)
    const unsigned long long done = low + size >= kDoneFlag ? low + size - kDoneFlag : low;
    const unsigned long long ylo = cw >> 32;
    if (done > size || ylo > done) return;
    const unsigned long long nlo = done - ylo;
    const unsigned long long Yprev = yes_before(st, c);
    const double plo = (double)(Yprev + ylo) / (double)Bc;
    const double phi = (double)(Yprev + size - nlo) / (double)Bc;
    unsigned long long g = next_sample(plo, V.eps, V.z, V.literal);
    const unsigned long long g2 = next_sample(phi, V.eps, V.z, V.literal);
    g = g2 < g ? g2 : g;
    if (V.literal && plo <= 0.5 && phi >= 0.5) {
        const unsigned long long g3 = next_sample(0.5, V.eps, V.z, V.literal);
        g = g3 < g ? g3 : g;
    }
    g = uniform_u64(g);
    if (g > Bc) {
        if (g > V.capacity) g = V.capacity;
        fence_acquire();      // what the publisher of bound[c] had seen ...
        fence_release();      // ... is seen by whoever claims below g
        if (lane_id() == 0) atomicMax(&st->limit, g);
    }
}

// ---------------------------------------------------------------------------
// Job selection and index claims.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool claimable(const Job *jobs, int j)
{
    JobState *st = jobs[j].st;
    return ld_relaxed(&st->next) < ld_relaxed(&st->limit) && ld_relaxed(&st->final_flag) == 0;
}

// Wave-cooperative scan for a job with issuable indices, starting at the
// wave's home job `start` (waves are spread evenly over the jobs, `wph` per
// job).  A job whose issuable range is small is left to the waves whose home
// is near it: a job at distance q (in scan order) is taken only if
// q * wph <= (room / 32 + wph) * (1 + idle), where room = limit - next and
// idle counts this wave's consecutive fruitless scans.  Without this, every
// idle wave of a launch converges on the one job whose limit has just risen
// (by a single index, say) and their claims serialise on its counter; the
// idle term lets distant waves in when the nearby ones stay busy.  No room
// exceeds room_max (the launch's largest capacity), so the scan ends at the
// first distance no job can qualify at.  any: take the first job with
// issuable indices at distance q0 or more, at any distance, and report its
// distance in *qf.
__device__ int pick_job(const Job *jobs, int n_jobs, int start, int wph, int idle, unsigned long long room_max,
                        bool any = false, int q0 = 0, int *qf = nullptr)
{
    const int lane = lane_id();
    const unsigned long long w = (unsigned long long)wph;
    const unsigned long long age = 1ull + (unsigned long long)(idle < 4096 ? idle : 4096);
    const unsigned long long reach = (room_max / 32ull + w) * age;
    for (int base = q0; base < n_jobs; base += kWave) {
        if (!any && (unsigned long long)base * w > reach) break;
        const int q = base + lane;
        int j = start + q;
        if (j >= n_jobs) j -= n_jobs;
        bool ok = false;
        if (q < n_jobs) {
            JobState *st = jobs[j].st;
            const unsigned long long nx = ld_relaxed(&st->next), lm = ld_relaxed(&st->limit);
            if (nx < lm && ld_relaxed(&st->final_flag) == 0)
                ok = any || (unsigned long long)q * w <= ((lm - nx) / 32ull + w) * age;
        }
        const uint64_t m = __ballot(ok);
        if (m) {
            const int l = ffs64(m);
            if (qf) *qf = base + l;
            return __builtin_amdgcn_readlane(j, l);
        }
    }
    return -1;
}

// Claim a chunk of consecutive relative indices below the job's issue limit;
// returns the count, *base = first.  The chunk shrinks as the remaining work
// shrinks (guided self-scheduling) so that the last trajectories spread over
// the waves, but never below what the wave runs at once (`slots`: one index
// per lane, or per lane group; nor below `need`) while that many remain: each
// claim is an atomic on one counter shared by every wave of the job.  Nor above
// four times that: a wave would sit on indices that idle waves could run.
//  - fixed-sample jobs: the limit never moves, so a fetch-add suffices (a
//    claim past the end simply gets nothing);
//  - iterative jobs: the limit rises while the job runs, so indices are
//    claimed by compare-and-swap below the current limit, with back-off.
__device__ int claim(JobState *st, bool iterative, int need, int slots, int n_waves, unsigned long long *base)
{
    unsigned long long cur = ld_relaxed(&st->next);
    unsigned long long lim = ld_relaxed(&st->limit);
    if (cur >= lim) return 0;
    unsigned long long want = (lim - cur) / (4ull * (unsigned long long)n_waves);
    if (want < (unsigned long long)need) want = (unsigned long long)need;
    // At least a wave's worth: claims of a few indices at a time (when lanes
    // finish one by one) turn the issue counter into a contended hot spot.
    if (want < (unsigned long long)slots) want = (unsigned long long)slots;
    if (want > 4ull * (unsigned long long)slots) want = 4ull * (unsigned long long)slots;
    if (!iterative) {
        const unsigned long long b = atomicAdd(&st->next, want);
        if (b >= lim) return 0;
        *base = b;
        return (int)((lim - b) < want ? (lim - b) : want);
    }
    lim = ld_acquire(&st->limit);   // see the ordering note at fence_release
    for (int tries = 0; tries < 16; ++tries) {
        if (cur >= lim) return 0;
        const unsigned long long w = (lim - cur) < want ? (lim - cur) : want;
        const unsigned long long prev = atomicCAS(&st->next, cur, cur + w);
        if (prev == cur) {
            *base = cur;
            return (int)w;
        }
        cur = prev;
        lim = ld_acquire(&st->limit);
        __builtin_amdgcn_s_sleep(4);
    }
    return 0;
}

struct KArgs {
    const Job *jobs;
    int n_jobs;
    int s_max;
    Control *ctl;
    const volatile int32_t *cancel;   // host-visible stop word
    int spin_limit;
    int waves_per_block;
    int static_first;                 // first launch: waves start on their static shares
    unsigned long long room_max;      // the largest capacity of the launch's jobs
};

// Add a wave's counts for batch b of its job to the sharded counters.
__device__ __forceinline__ void add_counts(JobState *st, int b, int shard, unsigned long long ny,
                                           unsigned long long nn, unsigned long long nt,
                                           unsigned long long ev)
{
    if (ny) atomicAdd(&st->yes[b][shard], ny);
    if (nn) atomicAdd(&st->no[b][shard], nn);
    if (nt) atomicAdd(&st->trunc[b][shard], nt);
    if (ev) atomicAdd(&st->events[b][shard], ev);
}

// ---------------------------------------------------------------------------
// The persistent kernel.
// ---------------------------------------------------------------------------
// kIter: the launch may hold iterative (Fig. 2) jobs.  Launches of fixed-size
// jobs only are compiled without the stopping-rule machinery, which would
// otherwise cost registers (occupancy) in the event loop.
// kTrace: the launch may hold trace programs (one lane per trajectory).
template <class Pol, bool kIter, bool kTrace = false>
__device__ __forceinline__ void persistent_body(KArgs A, int32_t *lds)
{
    const int lane = lane_id();
    // wave-uniform (the compiler cannot know that threadIdx.x / 64 is): keeps
    // the home job, the shard and everything loaded from them in scalar registers
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    typename Pol::Counts X = Pol::counts(lds, wid, A.s_max, lane);
    const int gwave = (int)blockIdx.x * A.waves_per_block + wid;
    const int shard = gwave & (kShards - 1);
    const int n_waves = (int)gridDim.x * A.waves_per_block;
    const int start = (int)(((long long)gwave * A.n_jobs) / n_waves);
    const int wph = n_waves > A.n_jobs ? n_waves / A.n_jobs : 1;   // waves per home job

    int cur = -1;
    JobView V;
    bool active = false, fin = false;
    unsigned long long ridx = 0;
    uint32_t k = 0, verdict = 0, reason = 0;
    double t = 0.0;
    MonState ms;
    mon_init(ms);
    Draw dr{0.0, 0.0};   // random numbers of the lane's next event (index k)
    uint32_t tr_lo = 0;  // trace programs: every point below this one is undecided
    uint32_t tr_every = 64;  // ... and the lane's interval between tests, in wave iterations
    int spins = 0;
    // scans that take any job: the jobs nearer than this (in this wave's scan
    // order) had no issuable indices left.  Such scans run only once no
    // iterative job is open, when no limit rises any more, so those jobs stay
    // exhausted.
    int any_from = 0;
    // wave-local pool of claimed, not yet started indices [pool_next, pool_end)
    unsigned long long pool_next = 0, pool_end = 0;
    // fixed-sample jobs: per-lane counts, added to the job once per wave
    uint32_t my_yes = 0, my_no = 0, my_trunc = 0;
    unsigned long long my_events = 0;
    if (A.static_first && start < A.n_jobs) {
        // First launch: start on the home job with this wave's own share of its
        // first indices, [c r, c r + c) below static_end for the wave's rank r
        // among the waves of that home, c = 64 / (lanes per trajectory) (set
        // up by init_jobs).  Thousands of
        // first claims on one counter would otherwise queue for tens of
        // microseconds.
        cur = start;
        V.load(A.jobs, cur);
        const unsigned long long per = (unsigned long long)(kWave / (Pol::kGroups ? __builtin_amdgcn_readfirstlane(V.lanes) : 1));
        const long long g0 = ((long long)start * n_waves + A.n_jobs - 1) / A.n_jobs;
        const unsigned long long lo = (unsigned long long)(gwave - g0) * per;
        const unsigned long long se = uniform_u64(ld_relaxed(&V.st->static_end));
        if (lo < se) {
            pool_next = lo;
            pool_end = lo + per < se ? lo + per : se;
        }
    }

    for (uint32_t it = 0;; ++it) {
        // Stop requests, checked once per 4096 iterations.  The host's stop
        // word lives in host memory, and reads of it cross the bus and queue
        // behind one another (thousands of waves reading it together stall for
        // hundreds of microseconds).  So at each check only the waves of one
        // counter shard (one in kShards), in turn, read it, and pass a request
        // on through a word in device memory that every wave reads.
        if ((it & 4095u) == 4095u) {
            int stop = 0;
            if (lane == 0) {
                stop = ld_relaxed(&A.ctl->stop);
                if (!stop && (((it >> 12) + (uint32_t)shard) & (kShards - 1)) == 0u) {
                    stop = *A.cancel;
                    if (stop) st_relaxed_i32(&A.ctl->stop, 1);
                }
            }
            if (uniform_i(stop)) break;
        }
        if (__ballot(active) == 0ull && pool_next == pool_end) {
            int j = pick_job(A.jobs, A.n_jobs, start, wph, spins, A.room_max);
            // A launch of fixed-size jobs only: a wave leaves once nothing is
            // near its home, so before leaving it takes any job with indices
            // left, however far (with many more jobs than waves, some would
            // otherwise lie out of every wave's reach).
            if (j < 0 && ld_relaxed(&A.ctl->open_jobs) <= 0)
                j = pick_job(A.jobs, A.n_jobs, start, wph, spins, A.room_max, true, any_from, &any_from);
            if (j != cur && cur >= 0 && !V.iterative) {
                // leaving a fixed-sample job: publish this wave's counts
                const unsigned long long ny = wave_sum_u64(my_yes), nn = wave_sum_u64(my_no);
                const unsigned long long nt = wave_sum_u64(my_trunc), ev = wave_sum_u64(my_events);
                if (lane == 0) add_counts(V.st, 0, shard, ny, nn, nt, ev);
                my_yes = my_no = my_trunc = my_events = 0;
            }
            if (j < 0) {
                cur = -1;
                if (ld_relaxed(&A.ctl->open_jobs) <= 0) break;
                // Idle waves back off longer after each fruitless scan of the
                // job table (its counters are read with coherent loads that
                // compete with the working waves' atomics).
                ++spins;
                const int naps = spins < 16 ? spins : 16;
                for (int z = 0; z < naps; ++z) __builtin_amdgcn_s_sleep(127);
                if (spins > A.spin_limit) break;
                continue;
            }
            spins = 0;
            if (j != cur) {
                cur = j;
                V.load(A.jobs, cur);
            }
        }
        // -------- refill idle lanes with new trajectory indices --------
        // With lane groups (L > 1) the L lanes of a group start, run and end
        // one trajectory together; the group is counted by its first lane.
        const int L = Pol::kGroups ? __builtin_amdgcn_readfirstlane(V.lanes) : 1;
        const int gbase = lane & ~(L - 1);
        const bool lead = lane == gbase;
        bool entered = false;   // this lane entered a state in this iteration
        const uint64_t need = __ballot(!active && lead);
        if (need) {
            const int n_need = __popcll(need);
            if (pool_next == pool_end) {
                unsigned long long base = 0;
                int got = 0;
                if (lane == 0) got = claim(V.st, V.iterative != 0, n_need, kWave / L, n_waves, &base);
                got = __builtin_amdgcn_readfirstlane(got);
                base = read_lane_u64(base, 0);
                pool_next = base;
                pool_end = base + (unsigned long long)got;
            }
            const unsigned long long avail = pool_end - pool_next;
            const int give = (unsigned long long)n_need < avail ? n_need : (int)avail;
            // rank of this lane's group among the idle groups
            const int r = L == 1 ? rank_in(need) : __popcll(need & ((1ull << gbase) - 1ull));
            if (!active && r < give) {
                ridx = pool_next + (unsigned long long)r;
                Pol::init(X, V);
                t = 0.0;
                k = 0;
                mon_init(ms);
                tr_lo = 0;
                tr_every = 64;
                active = true;
                entered = true;
            }
            pool_next += (unsigned long long)give;
        }
        if (__ballot(active) == 0ull) continue;

        // The event and the inspection of the state it enters run as straight-
        // line code on every lane, and each lane keeps only the results that
        // apply to it (selects, no divergent branches): masked-off lanes would
        // occupy the same issue slots anyway, and a single basic block lets the
        // compiler interleave the independent dependency chains below.
        //
        // Random numbers this lane needs next: those of event k + 1, or of
        // event 0 of a trajectory it has just started.  Nothing below feeds
        // them, so their computation overlaps the event.
        const Draw nxt = event_uniforms(V, V.first + ridx, entered ? 0u : k + 1u);

        // -------- trace programs: record, test at checkpoints --------
        if (kTrace && V.trace) {   // wave-uniform
            const bool ev_lane = active && !entered;
            typename Pol::Sel ch;
            const double tn = Pol::draw(V, X, dr, t, &ch, ev_lane);
            const TraceRec R = trace_rec(V.tr_base, V.tr_stride, V.tr_cap, V.tr_nskip, (unsigned long long)gwave,
                                         lane);
            bool tfin = false;
            uint32_t tk = k, tvd = 0, trs = 0;
            if (ev_lane) {
                R.t[(long)(k + 1u) << 6] = tn;   // the time state k is left
                // absorption, or the t_max rule, decides point 2k + 1
                if (__builtin_isinf(tn) || tn > V.t_max) {
                    trace_first(V.mon, R, tr_lo, 2u * k + 1u, V.t_max, V.max_events, &tk, &tvd, &trs);
                    tfin = true;
                }
            }
            const bool applied = ev_lane && !tfin;
            Pol::apply_if(X, ch, applied);
            t = applied ? tn : t;
            k = applied ? k + 1u : k;
            entered = entered || applied;
            if (entered) {
                R.t[(long)k << 6] = t;
                R.bits[(long)k << 6] = eval_preds(V.mon, X);
                if (k == 0u)   // a new trajectory: nothing is final yet
                    for (int q = 0; q < V.mon->tr_n; ++q) {
                        R.F(q) = 0;
                        R.RS(q) = 0;
                    }
                // checkpoints: the cap; 16 and 32 states (short trajectories);
                // and wave iterations at multiples of the lane's interval (64,
                // 128 or 256), so that the lanes due together share one
                // evaluation pass.  The interval follows the cost of a test:
                // the positions the last open test left to recompute (few
                // for short windows) against the events run past a decision
                // before it is seen.
                const bool sync = (it & (tr_every - 1u)) == tr_every - 1u;
                const bool cp = (V.max_events != 0u && k == V.max_events) || k == 15u || k == 31u || sync;
                if (cp) {
                    if (trace_decided(V.mon, R, 2u * k, V.t_max, V.max_events, &tvd, &trs)) {
                        trace_first(V.mon, R, tr_lo, 2u * k, V.t_max, V.max_events, &tk, &tvd, &trs);
                        tfin = true;
                    } else {
                        tr_lo = 2u * k + 1u;
                        const uint32_t open = trace_commit(V.mon, R, (int)k + 1);
                        tr_every = open < 128u ? 64u : (open < 256u ? 128u : 256u);
                    }
                }
            }
            dr.nl = entered ? nxt.nl : dr.nl;
            dr.u2 = entered ? nxt.u2 : dr.u2;
            fin = fin || tfin;
            verdict = tfin ? tvd : verdict;
            reason = tfin ? trs : reason;
            k = tfin ? tk : k;
        } else {
            // -------- one event per running lane --------
            const bool ev_lane = active && !entered;
            const bool capped = V.max_events != 0u && k == V.max_events;
            typename Pol::Sel ch;
            const double tn = Pol::draw(V, X, dr, t, &ch, ev_lane);
            const bool absorbing = __builtin_isinf(tn);
            MonState ms_adv = ms;
            const uint32_t va = Pol::advance(V, ms_adv, tn, absorbing);
            const bool stepping = ev_lane && !capped;
            const bool dec_time = stepping && va != 0u;
            const bool dec_tmax = stepping && va == 0u && tn > V.t_max;
            const bool applied = stepping && va == 0u && !(tn > V.t_max);
            ms_select(ms, ms_adv, stepping);
            Pol::apply_if(X, ch, applied);
            t = applied ? tn : t;
            k = applied ? k + 1u : k;
            entered = entered || applied;
            // capped, dec_time and dec_tmax exclude each other
            const bool dec_cap = ev_lane && capped;
            fin = fin || dec_cap || dec_time || dec_tmax;
            verdict = dec_time ? (va == 1u ? 1u : 0u) : (dec_cap || dec_tmax ? 0u : verdict);
            const uint32_t r_time = absorbing ? (uint32_t)RS_ABSORB : (uint32_t)RS_TIME;
            reason = dec_tmax ? (uint32_t)RS_TMAX : reason;
            reason = dec_time ? r_time : reason;
            reason = dec_cap ? (uint32_t)RS_CAP : reason;

            // -------- inspect the state just entered (new or after an event) --------
            MonState ms_st = ms;
            const uint32_t vs = Pol::step(V, ms_st, X, k, t);
            ms_select(ms, ms_st, entered);
            dr.nl = entered ? nxt.nl : dr.nl;   // field by field: a select of whole
            dr.u2 = entered ? nxt.u2 : dr.u2;   // structs would go through memory
            const bool dec_state = entered && vs != 0u;
            fin = fin || dec_state;
            verdict = dec_state ? (vs == 1u ? 1u : 0u) : verdict;
            reason = dec_state ? (uint32_t)RS_STATE : reason;
        }

        // -------- accounting of decided trajectories --------
        // (counted once per trajectory: by the first lane of its group)
        const bool fin_c = fin && lead;
        uint64_t fm = __ballot(fin_c);
        if (fm) {
            if (fin_c) {
                if (V.rec_events) V.rec_events[ridx] = k;
                if (V.rec_vr) V.rec_vr[ridx] = (uint8_t)(verdict | (reason << 1));
            }
            if (!kIter || !V.iterative) {
                if (fin_c) {
                    my_yes += verdict;
                    my_no += 1u - verdict;
                    my_trunc += (reason == RS_CAP) ? 1u : 0u;
                    my_events += k;
                }
                if (fin) {
                    fin = false;
                    active = false;
                }
                continue;
            }
            // batch of each finishing lane: the number of published bounds at
            // or below its index (the bounds are read once, one per lane)
            int b = 0;
            {
                const unsigned long long bq = lane < kMaxBatches ? ld_relaxed(&V.st->bound[lane]) : 0ull;
                if (fin_c) {
                    for (int q = 0; q < kMaxBatches - 1; ++q) {
                        const unsigned long long bb = read_lane_u64(bq, q);
                        if (bb == 0ull || ridx < bb) break;
                        ++b;
                    }
                }
            }
            while (fm) {
                const int Lf = ffs64(fm);
                const int b0 = __builtin_amdgcn_readlane(b, Lf);
                const bool sel = fin_c && (b == b0);
                const uint64_t sm = __ballot(sel);
                const uint32_t ny = (uint32_t)__popcll(__ballot(sel && verdict));
                const uint32_t nn = (uint32_t)__popcll(sm) - ny;
                const uint32_t nt = (uint32_t)__popcll(__ballot(sel && reason == RS_CAP));
                const unsigned long long ev = wave_sum_u64(sel ? (unsigned long long)k : 0ull);
                JobState *st = V.st;
                const unsigned long long delta = ((unsigned long long)ny << 32) | (unsigned long long)(ny + nn);
                unsigned long long old = 0;
                if (lane == Lf) {
                    add_counts(st, b0, shard, 0, 0, nt, ev);
                    old = atomicAdd(&st->cnt[b0], delta);
                }
                old = read_lane_u64(old, Lf);
                const unsigned long long now = old + delta;
                if ((now & 0xFFFFFFFFull) == kDoneFlag) {
                    fence_acquire();   // the bounds the batch's publisher had seen
                    evaluate_batches(V, A.ctl, b0, now);
                } else if (b0 == uniform_i(ld_relaxed(&st->cur))) {
                    // the look-ahead only moves with the counts: refresh it on
                    // a batch's first completions and every 64 after that
                    if ((old & 0xFFFFFFFFull) == 0ull || ((old >> 6) & 0x3FFFFFFull) != ((now >> 6) & 0x3FFFFFFull))
                        speculate(V, b0, now);
                }
                fm &= ~sm;
            }
            if (fin) {
                fin = false;
                active = false;
            }
        }
    }
    // publish the counts of a fixed-sample job this wave was still working on
    if (cur >= 0 && !V.iterative) {
        const unsigned long long ny = wave_sum_u64(my_yes), nn = wave_sum_u64(my_no);
        const unsigned long long nt = wave_sum_u64(my_trunc), ev = wave_sum_u64(my_events);
        if (lane == 0) add_counts(V.st, 0, shard, ny, nn, nt, ev);
    }
}

}  // namespace smc
