// smc_device.h -- data layout shared by the host runtime and the HIP kernels.
//
// Everything here lives in device memory.  One Job describes one model: its
// reaction network (Sec. 2.2), its compiled monitor program (Sec. 3.1-3.2),
// its stopping rule (Sec. 3.3, eqs. 3-4, Fig. 2) and its accounting state.
#pragma once
#ifndef __HIPCC_RTC__
#include <stdint.h>
#else
// the runtime compiler has no C library headers; it defines the fixed-width
// integer types in its own namespace
using __hip_internal::int16_t;
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint16_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
using __hip_internal::uint8_t;
#endif

namespace smc {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxBatches = 32;    // sample-size iterations per job
constexpr int kShards = 16;        // counter replicas (spread atomics over L2 channels)
constexpr int kMaxPreds = 16;      // state predicates per formula
constexpr int kMaxAtoms = 4;       // temporal monitors per formula
constexpr int kMaxProps = 12;      // state formulas (operands of the monitors)
constexpr int kMaxPropPreds = 5;   // predicates per state formula (truth table of 32 bits)
constexpr int kMaxNested = 2;      // monitors with a time register (nested, response, next-until, until-G)
constexpr int kMaxValOps = 96;     // arithmetic predicate programs
constexpr int kValStack = 4;       // arithmetic stack depth on the device
constexpr int kBlocks = 16;        // prefix-sum blocks for reaction selection
constexpr int kSubBlock = 8;       // channels per unrolled step of the blocked prefix
constexpr int kMaxGroupRounds = 8; // lane groups: rounds of 8 x lanes channels per event, at most
constexpr int kMaxTrace = 32;      // nodes of a trace program (formulas outside the compact monitors)
constexpr uint32_t kTraceMaxEvents = 1u << 20;   // event cap limit of a trace job
constexpr int kSpecMaxS = 16;      // specialised kernels: species counts in registers
constexpr int kSpecMaxM = 8;       // specialised kernels: channels
constexpr int kSpecWideMaxS = 128; // wide specialised kernels (counts in LDS): species
constexpr int kSpecWideMaxM = 512; //   and channels

enum CmpOp : int32_t { CMP_LT = 0, CMP_LE, CMP_GE, CMP_GT, CMP_EQ, CMP_NE };
enum ValOp : int32_t { VO_VAR = 0, VO_CONST, VO_ADD, VO_SUB, VO_MUL, VO_DIV, VO_NEG, VO_SQRT, VO_POWI };
enum PredKind : int32_t { PK_VAR = 0, PK_LINEAR = 1, PK_RPN = 2 };
enum AtomKind : int32_t { AK_PROP = 0, AK_UNTIL, AK_NEXT, AK_NESTED, AK_RESP, AK_NEXTU, AK_UNTILG };
enum Reason : int32_t { RS_STATE = 0, RS_TIME = 1, RS_ABSORB = 2, RS_CAP = 3, RS_TMAX = 4 };
enum TraceKind : int32_t { TN_TT = 0, TN_FF, TN_PRED, TN_NOT, TN_AND, TN_OR, TN_NEXT, TN_UNTIL };

// A state predicate over species counts x.
//  PK_VAR    : x[var] (op) c32                         (int32 compare)
//  PK_LINEAR : sum_q w[q] * x[vars[q]] + c  (op)  0    (integer, exact in int64)
//  PK_RPN    : two arithmetic stack programs evaluated in double in source
//              order, then compared
struct Pred {
    int32_t kind, op;
    int32_t var, c32;
    int32_t lo32, hi32, neg;   // PK_VAR as a range test: (lo32 <= x[var] <= hi32) != neg
    int32_t nterm;
    int32_t vars[4];
    int32_t pad0;
    int64_t w[4];
    int64_t c;
    int32_t lhs_off, lhs_len, rhs_off, rhs_len;
};

// A state formula: a boolean function of predicates off .. off+cnt-1, given
// by its truth table (bit i = value when the predicate bits read i).
struct Prop {
    int32_t off, cnt;
    uint32_t table;
    int32_t pad;
};

// A temporal monitor evaluated at position 0 of the path.
//  AK_PROP   : state formula p1 on the initial state.
//  AK_UNTIL  : p1 U[lo,hi] p2, negated when neg = 1 (G I p = not(tt U I not p)).
//  AK_NEXT   : X[lo,hi] p1.
//  AK_NESTED : p1 U[lo,hi] (p2 U[0,hi2] p3), registers (ok, latest start).
//  AK_RESP   : G[lo,hi](p1 | F[0,hi2] p2), negated when neg = 1; register: the
//              entry time of the oldest position whose obligation F[0,hi2] p2
//              is still open (-1: none).  Later open positions need not be
//              kept: a p2-state that meets the oldest one in time meets them.
//  AK_NEXTU  : X[lo,hi](p1 U[lo2,hi2] p2), the until negated when neg = 1
//              (X I G J p = X I not(tt U J not p)); register: the entry time
//              of state 1 (-1 before it), the origin of the until's window.
//  AK_UNTILG : p1 U[lo,hi] (p3 & G[0,hi2] p2); registers (ok, the entry time
//              of the earliest start whose G still runs, -1: none).  A break
//              of p2 ends every running start, and the earliest one's window
//              closes first, so later starts need not be kept.
struct Atom {
    int32_t kind;
    int32_t neg;
    int32_t p1, p2, p3;   // state-formula ids (-1 = none)
    int32_t slot;         // time register slot (nested until, response)
    double lo, hi, hi2, lo2;
};

// A node of a trace program: the formula itself as a tree (F I p written as
// tt U I p, G I p as not(tt U I not p), Sec. 3.1), children before parents,
// the root last.  pred: predicate id of TN_PRED, skip slot of TN_UNTIL; a, b:
// operands; [lo, hi]: the interval of TN_NEXT and TN_UNTIL.
struct TraceNode {
    int32_t kind, pred, a, b;
    double lo, hi;
};

// Compiled formula.  The top-level boolean combination of the monitors is a
// table: with t (f) the mask of monitors known true (false), bit t | f << n of
// topT (topF) says whether the formula is already true (false) in Kleene
// logic.  A formula outside the compact monitor classes is a trace program
// instead (trace = 1, n_atoms = 0): the kernel keeps the trajectory's states
// (entry times and predicate bits) and evaluates the formula on them.
struct MonProg {
    int32_t n_preds, n_atoms, n_props;
    int32_t all_var;   // every predicate is PK_VAR
    uint64_t topT[4], topF[4];
    Atom atoms[kMaxAtoms];
    Prop props[kMaxProps];
    Pred preds[kMaxPreds];
    int32_t vop[kMaxValOps];
    int32_t vvar[kMaxValOps];
    double vconst[kMaxValOps];
    double horizon;
    int32_t trace, tr_n, tr_nskip;   // tr_nskip: until nodes (TraceNode.pred is their skip slot)
    int32_t tr_pad;
    TraceNode tnodes[kMaxTrace];
};

// Reaction network tables (device memory, read-only in kernels).
//   reac[2j], reac[2j+1] = (ra, rb): ra < 0 zero order; rb < 0 first order;
//              ra == rb homodimer; otherwise two distinct reactants.
//   chg[4j+q] = four packed entries ((species & 0xFFFF) << 16) | (delta & 0xFFFF),
//              species 0xFFFF = unused.
// Channel j of a network for the generic kernels: h_j = (x_a (x_b - delta))
// gamma, c_j h_j being the propensity (Sec. 2.2).  a_off and the multiple of
// 256 in b_code are the byte offsets of the reactant rows in a wave's LDS
// slice; a missing reactant names row S, which holds the constant 1.  Bit 0
// of b_code marks x_a (x_a - 1) / 2, (delta, gamma) = (1, 1/2); otherwise
// (0, 1) for x_a x_b, x_a and 1.  Every factor is an integer or half-integer,
// so h_j is exact and c_j h_j rounds once.
struct ChanDev {
    int32_t a_off, b_code;
};

struct NetDev {
    int32_t S, M;
    int32_t Mp;   // M rounded up to kSubBlock: the tables hold Mp channels, the
                  // extra ones with rate 0, no reactants and no state change
    int32_t pad_;
    const int32_t *x0;
    const double *rate;
    const int32_t *reac;
    const uint32_t *chg;
    const ChanDev *chan;   // Mp entries
};

// The record area of one wave for a trace program of `cap` states, `n` nodes
// and `ns` until nodes, each part 256-byte aligned and interleaved over the
// wave's 64 lanes (element e of lane l at index 64 e + l), so that lanes
// reading the same position read adjacent words:
//   double   t[cap + 1]        entry times; t[m + 1] is also the time state m is left
//   uint32_t bits[cap]         predicate bits of each state (bit q: predicate q)
//   int32_t  need[kMaxTrace]   how many positions each node is evaluated at
//   int32_t  skip[ns][cap + 1] per until node: the next position that is not
//                              neutral (left operand true, right one false)
//   uint8_t  val[n][cap]       three-valued node values by position
struct TraceArea {
    static constexpr unsigned long long align(unsigned long long x) { return (x + 255ull) & ~255ull; }
    static constexpr unsigned long long bits_off(uint32_t cap) { return align(8ull * 64ull * (cap + 1ull)); }
    static constexpr unsigned long long need_off(uint32_t cap) { return bits_off(cap) + align(4ull * 64ull * cap); }
    // per node: the final-position counts, committed and being formed, and
    // (until nodes) the start of the final neutral run
    static constexpr unsigned long long fin_off(uint32_t cap) { return need_off(cap) + align(4ull * 64ull * kMaxTrace); }
    static constexpr unsigned long long skip_off(uint32_t cap)
    {
        return fin_off(cap) + align(4ull * 64ull * 3ull * kMaxTrace);
    }
    static constexpr unsigned long long val_off(uint32_t cap, int ns)
    {
        return skip_off(cap) + align(4ull * 64ull * (unsigned long long)ns * (cap + 1ull));
    }
    static constexpr unsigned long long bytes(uint32_t cap, int n, int ns)   // one wave
    {
        return val_off(cap, ns) + align(64ull * (unsigned long long)n * cap);
    }
};

// Per-job accounting (device memory).  Batch b covers relative trajectory
// indices [bound[b-1], bound[b]) with bound[-1] = 0; bound[b] = 0 means "not
// known yet".  Counters are replicated over kShards slots (spread atomics).
//
// Iterative jobs (Fig. 2) keep one counter word per batch, cnt[b] =
// (TRUE verdicts << 32) + low word, where completions add to the low word
// and the publication of bound[b] adds kDoneFlag - (bound[b] - bound[b-1]):
// the batch is complete exactly when the low word equals kDoneFlag, and the
// one atomic that makes it so (a completion or the publication) tells its
// wave to evaluate the batch.  Batch sizes stay below 2^30, so the low word
// never carries into the high one.
constexpr unsigned long long kDoneFlag = 1ull << 31;
constexpr unsigned long long kMaxBatchSize = 1ull << 30;

struct JobState {
    unsigned long long next;                 // relative indices issued
    unsigned long long limit;                // indices below this may be issued
    unsigned long long static_end;           // [0, static_end): first shares of the waves, see init_jobs
    unsigned long long bound[kMaxBatches];
    unsigned long long yes[kMaxBatches][kShards];    // fixed-sample jobs
    unsigned long long no[kMaxBatches][kShards];     // fixed-sample jobs
    unsigned long long events[kMaxBatches][kShards];
    unsigned long long trunc[kMaxBatches][kShards];
    unsigned long long cnt[kMaxBatches];             // iterative jobs, see above
    int32_t cur;                             // earliest batch not yet evaluated
    int32_t final_flag;                      // 1 = stopping rule satisfied
    int32_t n_batches;
    int32_t overflow;                        // ran out of batch slots
    unsigned long long n_final, yes_final;
};

struct Job {
    NetDev net;
    const MonProg *mon;
    unsigned long long seed;
    unsigned long long first;     // absolute index of relative index 0
    unsigned long long capacity;  // relative indices that may ever be issued
    unsigned long long n_first;   // end of the first batch
    uint32_t model_id;
    uint32_t max_events;          // 0 = none
    double t_max;
    int32_t iterative;            // 1 = Fig. 2 rule, 0 = fixed sample
    int32_t literal;              // paper's rounding step without the stop at 0.5
    int32_t lanes;                // lanes per trajectory: 1, or 2/4/8/16 (generic kernel, > 4 channels)
    int32_t trace;                // 1 = the formula is a trace program
    double eps, z;
    JobState *st;
    uint32_t *rec_events;         // optional per-index outputs (relative index)
    uint8_t *rec_vr;
    // trace programs: one record area per wave of the launch (wave w at
    // tr_base + w * tr_stride) for states 0 .. tr_cap - 1 of up to tr_nodes
    // nodes and tr_nskip until nodes, see TraceArea
    unsigned char *tr_base;
    unsigned long long tr_stride;
    uint32_t tr_cap;
    uint32_t tr_nodes;
    uint32_t tr_nskip;
    uint32_t tr_pad;
};

// Compact per-job outcome copied back to the host.
struct JobResult {
    unsigned long long n, yes, events, trunc, issued;
    int32_t batches, final_flag, overflow, pad;
};

// Launch-wide control block.
struct Control {
    int32_t open_jobs;            // iterative jobs not final yet
    int32_t stop;                 // a wave has seen the host's stop word
};

}  // namespace smc
