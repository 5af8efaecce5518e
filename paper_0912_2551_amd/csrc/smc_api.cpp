// smc_api.cpp -- the C ABI declared in include/smc.h (host runtime).
//
// Validates inputs, keeps network tables and compiled formulas in device
// memory, sets up one Job per model, launches the persistent SSA kernel, waits
// on it under a watchdog, and turns the per-job counts into estimates with
// the Wilson interval (eq. 3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "smc.h"
#include "smc_device.h"
#include "smc_internal.h"

using namespace smc;

struct smc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int n_cu = 256;
    int waves_per_cu = 0;
    int spec_mode = SMC_SPECIALIZE_AUTO;
    int spec_waves_per_simd = 0;
    int lanes = 0;   // lanes per trajectory (0: automatic)
    // autotuned configurations per model structure (see smc_autotune)
    std::map<std::pair<uint64_t, uint64_t>, smc_tune_result> tuned;
    // autotuned configurations per batch signature (see smc_autotune_batch)
    std::map<uint64_t, smc_batch_tune_result> tuned_batch;
    // specialised kernels per (network structure, formula structure,
    // iterative, occupancy hint): spares regenerating the kernel source
    std::map<std::tuple<uint64_t, uint64_t, int, int>, hipFunction_t> spec_fns;
    bool tuning = false;
    std::map<double, double> zcache;   // z_{1-alpha/2} per confidence level
    int last_kernel = -1;
    bool spec_warned = false;
    double watchdog = 300.0;
    int32_t *cancel_host = nullptr;   // pinned, read by kernels
    int32_t *cancel_dev = nullptr;
    std::atomic<int> cancel_req{0};
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
    // grow-only workspace
    Job *d_jobs = nullptr;
    size_t cap_jobs = 0;
    JobState *d_states = nullptr;
    size_t cap_states = 0;
    JobResult *d_results = nullptr;
    size_t cap_results = 0;
    Control *d_ctl = nullptr;
    char *d_rec = nullptr;
    size_t cap_rec = 0;
    // record areas of trace programs, one per lane of a launch (grow-only)
    unsigned char *d_trace = nullptr;
    size_t cap_trace = 0;
    // pinned staging for the per-launch copies (asynchronous DMA instead of
    // the staged copies of pageable memory)
    Job *h_jobs = nullptr;
    size_t cap_h_jobs = 0;
    JobResult *h_results = nullptr;
    size_t cap_h_results = 0;
    Control *h_ctl = nullptr;
    // the device's fixed job array for smc_estimate_batch_noalloc (mapped
    // when the context is created)
    void *noalloc_base = nullptr;
};

struct smc_net {
    smc_ctx *ctx = nullptr;
    uint64_t sid = 0;             // structure id: equal ids, equal (S, M, reac, chg)
    int S = 0, M = 0;
    std::vector<int32_t> x0;
    std::vector<double> rate;
    std::vector<int32_t> reac;    // [2M]
    std::vector<uint32_t> chg;    // [4M]
    std::vector<std::string> names;
    int32_t *d_x0 = nullptr;
    double *d_rate = nullptr;
    int32_t *d_reac = nullptr;
    uint32_t *d_chg = nullptr;
    ChanDev *d_chan = nullptr;
};

struct smc_formula {
    smc_ctx *ctx = nullptr;
    uint64_t sid = 0;             // structure id: equal ids, equal compiled programs
    MonProg prog;
    MonProg *d_prog = nullptr;
    double horizon = 0.0;
};

// Channels held by the device tables (see upload_net).
static int padded_channels(int M) { return (M + kSubBlock - 1) / kSubBlock * kSubBlock; }

namespace {

thread_local std::string g_create_error;

int fail(smc_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    else g_create_error = msg;
    return code;
}

int hip_fail(smc_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, e == hipErrorOutOfMemory ? SMC_E_NOMEM : SMC_E_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, call)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

template <typename T>
int ensure(smc_ctx *ctx, T *&ptr, size_t &cap, size_t n)
{
    if (n <= cap) return SMC_OK;
    const size_t want = std::max(n, cap * 2);
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    cap = 0;
    HIP_TRY(ctx, hipMalloc((void **)&ptr, want * sizeof(T)));
    cap = want;
    return SMC_OK;
}

template <typename T>
int ensure_pinned(smc_ctx *ctx, T *&ptr, size_t &cap, size_t n)
{
    if (n <= cap) return SMC_OK;
    const size_t want = std::max(n, cap * 2);
    if (ptr) (void)hipHostFree(ptr);
    ptr = nullptr;
    cap = 0;
    HIP_TRY(ctx, hipHostMalloc((void **)&ptr, want * sizeof(T), hipHostMallocDefault));
    cap = want;
    return SMC_OK;
}

// Process-wide ids of distinct structures (byte strings): equal ids, equal
// structures.  The table only grows, by one entry per distinct structure.
uint64_t intern_structure(const std::string &bytes)
{
    static std::mutex mu;
    static auto *tab = new std::map<std::string, uint64_t>();
    std::lock_guard<std::mutex> lock(mu);
    auto it = tab->find(bytes);
    if (it != tab->end()) return it->second;
    const uint64_t id = tab->size() + 1;
    tab->emplace(bytes, id);
    return id;
}

// Eq. 4 before rounding, in the contract's operation order.
double wilson_value(double p, double eps, double z)
{
    const double pq = p * (1.0 - p);
    const double e2 = eps * eps;
    const double d = p - 0.5;
    const double rad = pq * pq + (4.0 * e2) * (d * d);
    const double num = (pq - 2.0 * e2) + std::sqrt(rad);
    return (z * z) * num / (2.0 * e2);
}

double resolve_z(smc_ctx *ctx, const smc_params &p, bool cache = true)
{
    if (p.z > 0.0) return p.z;
    auto it = ctx->zcache.find(p.confidence);
    if (it != ctx->zcache.end()) return it->second;
    const double z = smc_z_value(p.confidence);
    if (cache) ctx->zcache.emplace(p.confidence, z);
    return z;
}

// Lanes per trajectory of a job: the request (the job's own, else the
// context's; 0 = automatic, which is one lane for now), on the generic kernels
// for networks of more than four channels only, raised so that the group
// covers the padded channels in at most kMaxGroupRounds rounds of kSubBlock
// channels per lane.
int lanes_for(int want, int M)
{
    if (want <= 1 || M <= 4) return 1;
    const int Mp = padded_channels(M);
    if (Mp > kMaxGroupRounds * kSubBlock * 16) return 1;
    int L = want;
    while (L < 16 && Mp > kMaxGroupRounds * kSubBlock * L) L *= 2;
    return L;
}

int job_lanes(const smc_ctx *ctx, const smc_params *p, int M)
{
    return lanes_for(p->lanes ? (int)p->lanes : ctx->lanes, M);
}

struct Prepared {
    Job job;
    const smc_net *net = nullptr;
    const smc_formula *f = nullptr;
    int S = 0, M = 0;
    uint64_t capacity = 0;
    double z = 0.0;
    bool speculate = true;   // iterative job: may run as a speculative launch
    bool tree = false;       // SMC_TREE_SUMS: tree-ordered sums where the job runs in lane groups
    bool auto_lanes = false; // lanes per trajectory left to the library (job and context: 0)
};

int prepare(smc_ctx *ctx, const smc_net *net, const smc_formula *f, const smc_params *p,
            uint64_t first, Prepared &out, bool cache_z = true)
{
    if (!net || !f || !p) return fail(ctx, SMC_E_INVALID, "null network, formula or parameters");
    if (net->ctx != ctx || f->ctx != ctx) return fail(ctx, SMC_E_INVALID, "handle from another context");
    if (std::isnan(p->t_max) || p->t_max < 0.0) return fail(ctx, SMC_E_INVALID, "t_max must be >= 0");
    if (p->lanes != 0 && p->lanes != 1 && p->lanes != 2 && p->lanes != 4 && p->lanes != 8 && p->lanes != 16)
        return fail(ctx, SMC_E_INVALID, "lanes per trajectory must be 0, 1, 2, 4, 8 or 16");
    if (std::isinf(f->horizon) && std::isinf(p->t_max) && p->max_events == 0)
        return fail(ctx, SMC_E_INVALID, "an unbounded formula needs t_max or max_events");
    if (f->prog.trace && (p->max_events == 0 || p->max_events > kTraceMaxEvents))
        return fail(ctx, SMC_E_INVALID, "a formula outside the compact monitor classes (a trace program) needs "
                                        "max_events in 1..2^20: its states are recorded up to the cap");
    const bool iterative = p->fixed_n == 0;
    double z = 0.0;
    if (iterative || p->z > 0.0 || (p->confidence > 0.0 && p->confidence < 1.0)) {
        if (p->z <= 0.0 && !(p->confidence > 0.0 && p->confidence < 1.0))
            return fail(ctx, SMC_E_INVALID, "confidence must lie in (0, 1)");
        z = resolve_z(ctx, *p, cache_z);
    }
    uint64_t n_first, capacity;
    if (iterative) {
        if (!(p->half_width > 0.0 && p->half_width < 0.5))
            return fail(ctx, SMC_E_INVALID, "half_width must lie in (0, 0.5)");
        const double start = (p->flags & SMC_CONSERVATIVE_START) ? 0.5 : 1.0;
        n_first = (uint64_t)std::ceil(wilson_value(start, p->half_width, z));
        capacity = (uint64_t)std::ceil(wilson_value(0.5, p->half_width, z));
        if (n_first < 1) n_first = 1;
        if (capacity < n_first) capacity = n_first;
    } else {
        n_first = p->fixed_n;
        capacity = p->fixed_n;
    }
    if (first + capacity > (1ull << 32))
        return fail(ctx, SMC_E_INVALID, "trajectory indices must stay below 2^32");
    if (iterative && capacity >= kMaxBatchSize)
        return fail(ctx, SMC_E_INVALID, "iterative sample sizes must stay below 2^30 (half_width too small)");
    Job &J = out.job;
    std::memset(&J, 0, sizeof(J));
    J.net.S = net->S;
    J.net.M = net->M;
    J.net.Mp = padded_channels(net->M);
    J.net.x0 = net->d_x0;
    J.net.rate = net->d_rate;
    J.net.reac = net->d_reac;
    J.net.chg = net->d_chg;
    J.net.chan = net->d_chan;
    J.mon = f->d_prog;
    J.seed = p->seed;
    J.first = first;
    J.capacity = capacity;
    J.n_first = n_first;
    J.model_id = p->model_id;
    J.max_events = p->max_events;
    J.t_max = p->t_max;
    J.iterative = iterative ? 1 : 0;
    J.literal = (p->flags & SMC_PAPER_ROUNDING) ? 1 : 0;
    J.lanes = f->prog.trace ? 1 : job_lanes(ctx, p, net->M);
    J.trace = f->prog.trace ? 1 : 0;
    J.eps = p->half_width;
    J.z = z;
    out.net = net;
    out.f = f;
    out.S = net->S;
    out.M = net->M;
    out.capacity = capacity;
    out.z = z;
    out.speculate = (p->flags & SMC_NO_SPECULATION) == 0;
    out.tree = (p->flags & SMC_TREE_SUMS) != 0;
    out.auto_lanes = p->lanes == 0 && ctx->lanes == 0;
    return SMC_OK;
}

// Whether two models share their structure (network tables and compiled
// formula), compared directly.
bool same_structure(const smc_net *a, const smc_formula *fa, const smc_net *b, const smc_formula *fb)
{
    return a->sid == b->sid && fa->sid == fb->sid;
}

// The structure of a model: network tables and compiled formula (rates,
// initial state, seeds and stopping parameters do not enter).
std::pair<uint64_t, uint64_t> structure_key(const smc_net *net, const smc_formula *f)
{
    return {net->sid, f->sid};
}

// The specialised kernel for a launch, if every job shares one network
// structure and formula that the specialisation supports (else nullptr).
int pick_spec_kernel(smc_ctx *ctx, const Prepared *P, int n, bool iterative, bool may_compile, hipFunction_t *fn)
{
    *fn = nullptr;
    if (ctx->spec_mode == SMC_SPECIALIZE_OFF || n == 0) return SMC_OK;
    const smc_net *n0 = P[0].net;
    const smc_formula *f0 = P[0].f;
    bool ok = n0 && f0 && spec_supported(n0->S, n0->M, f0->prog);
    for (int k = 1; ok && k < n; ++k)
        ok = P[k].net && P[k].f && same_structure(n0, f0, P[k].net, P[k].f);
    // lane groups run on the generic kernels only
    for (int k = 0; ok && k < n; ++k) ok = P[k].job.lanes == 1;
    if (!ok) {
        if (ctx->spec_mode == SMC_SPECIALIZE_REQUIRED)
            return fail(ctx, SMC_E_UNSUPPORTED, "jobs do not share one structure the specialised kernels support");
        return SMC_OK;
    }
    const auto key = std::make_tuple(n0->sid, f0->sid, iterative ? 1 : 0, ctx->spec_waves_per_simd);
    const auto hit = ctx->spec_fns.find(key);
    if (hit != ctx->spec_fns.end()) {
        *fn = hit->second;
        return SMC_OK;
    }
    if (!may_compile) {
        // loading a new code object allocates device memory
        if (ctx->spec_mode == SMC_SPECIALIZE_REQUIRED)
            return fail(ctx, SMC_E_UNSUPPORTED, "no specialised kernel compiled yet for this structure "
                                                "(an allocation-free call does not compile one)");
        return SMC_OK;
    }
    const std::string src =
        spec_source(n0->S, n0->M, n0->reac.data(), n0->chg.data(), f0->prog, ctx->spec_waves_per_simd, iterative);
    std::string err;
    if (spec_kernel(ctx->device, src, fn, err) == 0) {
        ctx->spec_fns.emplace(key, *fn);
    } else {
        *fn = nullptr;
        if (ctx->spec_mode == SMC_SPECIALIZE_REQUIRED) return fail(ctx, SMC_E_HIP, err);
        if (!ctx->spec_warned) {
            std::fprintf(stderr, "libsmc: using the generic kernel: %s\n", err.c_str());
            ctx->spec_warned = true;
        }
    }
    return SMC_OK;
}

int pick_waves_per_cu(const smc_ctx *ctx)
{
    if (ctx->waves_per_cu > 0) return ctx->waves_per_cu;
    return 16;
}

// The buffers of one run: device job descriptors, job states, results and
// control block, and their host-side staging (2n job descriptors).
struct Workspace {
    Job *d_jobs;
    JobState *d_states;
    JobResult *d_results;
    Control *d_ctl;
    Job *h_jobs;
    JobResult *h_results;
    Control *h_ctl;
    // pinned host staging: the result copy is queued behind the kernels;
    // otherwise it is made once they are done
    bool pinned;
    // allocate nothing: no speculative launch (it needs per-index records)
    // and no run-time compilation of a specialised kernel
    bool no_alloc;
};

int run_jobs_in(smc_ctx *ctx, Prepared *P, int n, const Workspace &W, JobResult *res, double *seconds);

// Run prepared jobs to completion in the context's (grow-only) workspace.
int run_jobs(smc_ctx *ctx, std::vector<Prepared> &P, std::vector<JobResult> &res, double *seconds)
{
    const int n = (int)P.size();
    if (ensure(ctx, ctx->d_jobs, ctx->cap_jobs, (size_t)n)) return SMC_E_NOMEM;
    if (ensure(ctx, ctx->d_states, ctx->cap_states, (size_t)n)) return SMC_E_NOMEM;
    if (ensure(ctx, ctx->d_results, ctx->cap_results, (size_t)n)) return SMC_E_NOMEM;
    if (ensure_pinned(ctx, ctx->h_jobs, ctx->cap_h_jobs, 2 * (size_t)n)) return SMC_E_NOMEM;
    if (ensure_pinned(ctx, ctx->h_results, ctx->cap_h_results, (size_t)n)) return SMC_E_NOMEM;
    const Workspace W{ctx->d_jobs, ctx->d_states, ctx->d_results, ctx->d_ctl,
                      ctx->h_jobs, ctx->h_results, ctx->h_ctl, true, false};
    res.assign(n, JobResult{});
    return run_jobs_in(ctx, P.data(), n, W, res.data(), seconds);
}

// Signature of a batch for smc_autotune_batch: the structures of its jobs in
// order (FNV-1a over the structure ids and the job count).
uint64_t batch_signature(const Prepared *P, int n)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xFFull;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)n);
    for (int k = 0; k < n; ++k) {
        mix(P[k].net ? P[k].net->sid : 0ull);
        mix(P[k].f ? P[k].f->sid : 0ull);
    }
    return h;
}

int run_jobs_in(smc_ctx *ctx, Prepared *P, int n, const Workspace &W, JobResult *res, double *seconds)
{
    // Tuned choices override the context's launch settings for this launch
    // only; they are restored on return.
    struct Restore {
        smc_ctx *c;
        int wpc, occ, mode;
        ~Restore()
        {
            c->waves_per_cu = wpc;
            c->spec_waves_per_simd = occ;
            c->spec_mode = mode;
        }
    } restore{ctx, ctx->waves_per_cu, ctx->spec_waves_per_simd, ctx->spec_mode};
    // A configuration tuned for this batch (smc_autotune_batch): its launch
    // shape, and its lanes per trajectory for the jobs that leave that choice
    // to the library.
    if (!ctx->tuned_batch.empty() && !ctx->tuning) {
        const auto it = ctx->tuned_batch.find(batch_signature(P, n));
        if (it != ctx->tuned_batch.end()) {
            ctx->waves_per_cu = it->second.waves_per_cu;
            for (int k = 0; k < n; ++k)
                if (P[k].auto_lanes) P[k].job.lanes = lanes_for(it->second.lanes, P[k].M);
        }
    }
    int s_max = 1, m_max = 1, n_iter = 0, group = 1, n_trace = 0, tr_nodes = 0, tr_nskip = 0;
    uint32_t tr_cap = 0;
    Job *jobs = W.h_jobs;   // the previous call's copies have completed
    for (int k = 0; k < n; ++k) {
        jobs[k] = P[k].job;
        jobs[k].st = W.d_states + k;
        s_max = std::max(s_max, P[k].S);
        m_max = std::max(m_max, P[k].M);
        n_iter += jobs[k].iterative;
        group = std::max(group, (int)jobs[k].lanes);
        if (jobs[k].trace) {
            ++n_trace;
            tr_cap = std::max(tr_cap, jobs[k].max_events + 1u);
            tr_nodes = std::max(tr_nodes, (int)P[k].f->prog.tr_n);
            tr_nskip = std::max(tr_nskip, (int)P[k].f->prog.tr_nskip);
        }
    }
    const size_t lds_wave = (size_t)(s_max + 1) * kWave * sizeof(int32_t);   // + the constant-1 row
    int wpb = (int)std::min<size_t>(4, std::max<size_t>(1, 65536 / lds_wave));
    if (lds_wave > 65536) return fail(ctx, SMC_E_INVALID, "network too large for one wave's LDS");
    // Trace programs: one record area per wave of the launch, within a budget
    // of device memory, which bounds the launch's waves; every job of such a
    // launch runs one lane per trajectory (on the trace-capable kernel).
    unsigned long long tr_slots = 0;   // lanes with a record area
    if (n_trace > 0) {
        if (W.no_alloc)
            return fail(ctx, SMC_E_UNSUPPORTED, "trace programs need record areas, which an allocation-free call "
                                                "does not allocate");
        const unsigned long long stride = TraceArea::bytes(tr_cap, tr_nodes, tr_nskip);   // one wave
        const unsigned long long per_block = (unsigned long long)kWave * wpb;
        // no more lanes than the device holds, than the trajectories need, or
        // than the budget allows
        unsigned long long want = 0;
        for (int k = 0; k < n; ++k) want += P[k].capacity;
        want = (want + per_block - 1) / per_block * per_block;
        tr_slots = std::min<unsigned long long>((unsigned long long)ctx->n_cu * 32ull * kWave,
                                                kTraceBudget / stride * kWave);
        tr_slots -= tr_slots % per_block;
        tr_slots = std::min(tr_slots, want);
        if (tr_slots == 0)
            return fail(ctx, SMC_E_NOMEM, "the record areas of one block of trace lanes exceed the 8 GiB budget "
                                          "(lower max_events)");
        if (ensure(ctx, ctx->d_trace, ctx->cap_trace, (size_t)(tr_slots / kWave * stride))) return SMC_E_NOMEM;
        for (int k = 0; k < n; ++k) {
            jobs[k].tr_base = ctx->d_trace;
            jobs[k].tr_stride = stride;
            jobs[k].tr_cap = tr_cap;
            jobs[k].tr_nodes = (uint32_t)tr_nodes;
            jobs[k].tr_nskip = (uint32_t)tr_nskip;
            jobs[k].lanes = 1;
            P[k].job.lanes = 1;
        }
        group = 1;
    }
    // One group size per launch (one grouped kernel per size): jobs that run
    // several lanes per trajectory take the largest requested, which is at
    // least what each of them needs; the results do not depend on it.
    // The grouped jobs of one launch also share the order of their sums.
    int n_tree = 0, n_grouped = 0;
    for (int k = 0; k < n; ++k) {
        if (jobs[k].lanes > 1) jobs[k].lanes = group;
        P[k].job.lanes = jobs[k].lanes;
        n_grouped += jobs[k].lanes > 1;
        n_tree += jobs[k].lanes > 1 && P[k].tree;
    }
    if (n_tree != 0 && n_tree != n_grouped)
        return fail(ctx, SMC_E_INVALID, "jobs of one call that run in lane groups must agree on SMC_TREE_SUMS");
    const bool tree = n_tree > 0;
    // Speculative launch: when every job is iterative and their capacities
    // together fit in one pass over the device's lanes, every index up to each
    // job's capacity runs at once, as a fixed-size launch that records
    // per-index outcomes; replay_wilson then applies Fig. 2 to those outcomes
    // in index order.  The results are the batch protocol's, bit for bit.  A
    // lone Wilson run is latency-bound: its batches would follow one another,
    // each as long as its longest trajectory, on a device that is mostly idle.
    // jobs[n .. 2n) keep the iterative descriptions for the replay.
    bool speculative = false;
    if (n_iter == n && !ctx->tuning && !W.no_alloc && n_trace == 0) {
        unsigned long long cap_total = 0;
        bool allow = true;
        for (int k = 0; k < n; ++k) {
            cap_total += P[k].capacity * (unsigned long long)P[k].job.lanes;
            allow = allow && P[k].speculate;
        }
        const unsigned long long lanes = (unsigned long long)ctx->n_cu * pick_waves_per_cu(ctx) * kWave;
        speculative = allow && cap_total <= lanes;
        if (speculative) {
            if (ensure(ctx, ctx->d_rec, ctx->cap_rec, (size_t)cap_total * (sizeof(uint32_t) + 1))) return SMC_E_NOMEM;
            uint32_t *ev = reinterpret_cast<uint32_t *>(ctx->d_rec);
            uint8_t *vr = reinterpret_cast<uint8_t *>(ev + cap_total);
            unsigned long long off = 0;
            for (int k = 0; k < n; ++k) {
                jobs[k].rec_events = ev + off;
                jobs[k].rec_vr = vr + off;
                jobs[n + k] = jobs[k];
                jobs[k].iterative = 0;
                jobs[k].n_first = jobs[k].capacity;
                off += jobs[k].capacity;
            }
            n_iter = 0;
        }
    }
    hipStream_t s = ctx->stream;
    HIP_TRY(ctx, hipMemcpyAsync(W.d_jobs, jobs, n * sizeof(Job), hipMemcpyHostToDevice, s));
    *ctx->cancel_host = 0;
    ctx->cancel_req.store(0);

    // A configuration tuned for this structure (fixed-size pilots) applies to
    // launches of fixed-size jobs that all share it.
    if (!ctx->tuned.empty() && !ctx->tuning && n_iter == 0 && P[0].net && P[0].f) {
        auto it = ctx->tuned.find(structure_key(P[0].net, P[0].f));
        bool same = it != ctx->tuned.end();
        for (int k = 1; same && k < n; ++k)
            same = P[k].net && P[k].f && same_structure(P[0].net, P[0].f, P[k].net, P[k].f);
        if (same) {
            ctx->waves_per_cu = it->second.waves_per_cu;
            ctx->spec_waves_per_simd = it->second.waves_per_simd;
            ctx->spec_mode = it->second.specialization;
        }
    }
    const int wpc = pick_waves_per_cu(ctx);
    // No more waves than there are trajectories to run at once: idle waves
    // only poll the job table.
    unsigned long long lanes_needed = 0;
    for (int k = 0; k < n; ++k) lanes_needed += P[k].capacity * (unsigned long long)P[k].job.lanes;
    const unsigned long long waves_needed = (lanes_needed + kWave - 1) / kWave;
    const unsigned long long waves = std::min<unsigned long long>((unsigned long long)ctx->n_cu * wpc, waves_needed);
    int grid = (int)std::max<unsigned long long>(1, (waves + wpb - 1) / wpb);
    if (n_trace > 0) grid = (int)std::min<unsigned long long>((unsigned long long)grid, tr_slots / ((unsigned long long)kWave * wpb));
    const int variant = n_trace > 0 ? 10
                      : group > 1 ? (tree ? 5 : 1) + __builtin_ctz((unsigned)group) : (m_max <= 4 ? 0 : 1);
    hipFunction_t spec_fn = nullptr;
    if (const int rc = pick_spec_kernel(ctx, P, n, n_iter > 0, !W.no_alloc, &spec_fn)) return rc;
    // wide specialised kernels keep counts in LDS like the generic ones
    const size_t spec_lds = (spec_fn && spec_wide(P[0].S, P[0].M)) ? lds_wave * wpb : 0;
    // Static first shares (see init_jobs) only where they cannot hold work
    // back: every job of fixed size, so that idle waves leave at once, and a
    // grid that fits on the device at once.  A wave that is not yet resident
    // would keep its share until resident waves leave, and an iterative batch
    // would wait for it.
    bool static_first = false;
    if (n_iter == 0) {
        const int per_cu = spec_fn ? module_blocks_per_cu(spec_fn, wpb, spec_lds)
                                   : persistent_blocks_per_cu(variant, false, wpb, lds_wave * wpb);
        static_first = per_cu > 0 && (long long)per_cu * ctx->n_cu >= grid;
    }
    HIP_TRY(ctx, launch_init(s, W.d_jobs, n, static_first ? grid * wpb : 0, W.d_ctl, n_iter));
    ctx->last_kernel = spec_fn ? SMC_KERNEL_SPECIALIZED
                       : variant == 0 ? SMC_KERNEL_GENERIC_SMALL
                       : variant == 1 ? SMC_KERNEL_GENERIC
                       : variant == 10 ? SMC_KERNEL_GENERIC_TRACE
                       : tree ? SMC_KERNEL_GENERIC_TREE : SMC_KERNEL_GENERIC_GROUPED;
    for (int k = 0; k < n; ++k) res[k] = JobResult{};
    unsigned long long room_max = 1;
    for (int k = 0; k < n; ++k) room_max = std::max(room_max, (unsigned long long)jobs[k].capacity);
    double total_ms = 0.0;
    const auto t_start = std::chrono::steady_clock::now();
    unsigned long long last_progress = ~0ull;
    int stalls = 0;
    for (int launch = 0; launch < 1000; ++launch) {
        int open = 0;
        if (launch == 0) open = n_iter;
        else
            for (int k = 0; k < n; ++k) open += (jobs[k].iterative && !res[k].final_flag);
        // init_jobs set the first launch's control block; the previous launch
        // (and its copies) completed before this point
        if (launch > 0) {
            *W.h_ctl = Control{};
            W.h_ctl->open_jobs = open;
            HIP_TRY(ctx, hipMemcpyAsync(W.d_ctl, W.h_ctl, sizeof(Control), hipMemcpyHostToDevice, s));
        }
        HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
        if (spec_fn)
            HIP_TRY(ctx, launch_module(spec_fn, grid, wpb, spec_lds, s, W.d_jobs, n, s_max, W.d_ctl,
                                       ctx->cancel_dev, 1 << 18, static_first && launch == 0, room_max));
        else
            HIP_TRY(ctx, launch_persistent(variant, n_iter > 0, grid, wpb, lds_wave * wpb, s, W.d_jobs, n, s_max,
                                           W.d_ctl, ctx->cancel_dev, 1 << 18, static_first && launch == 0,
                                           room_max));
        if (speculative) {
            HIP_TRY(ctx, hipMemcpyAsync(W.d_jobs, jobs + n, n * sizeof(Job), hipMemcpyHostToDevice, s));
            HIP_TRY(ctx, launch_replay(s, W.d_jobs, n, W.d_results));
        } else {
            HIP_TRY(ctx, launch_finalize(s, W.d_jobs, n, W.d_results));
        }
        HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
        // the results travel back in the same stream, without a round trip
        // through the host between the kernels' end and the copy (a copy to
        // pageable memory would hold the host until it is done, so there it
        // follows the wait)
        if (W.pinned)
            HIP_TRY(ctx, hipMemcpyAsync(W.h_results, W.d_results, n * sizeof(JobResult), hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipEventRecord(ctx->ev2, s));
        // wait under the watchdog
        for (;;) {
            const hipError_t q = hipEventQuery(ctx->ev2);
            if (q == hipSuccess) break;
            if (q != hipErrorNotReady) return hip_fail(ctx, q, "kernel");
            const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
            if ((ctx->watchdog > 0.0 && el > ctx->watchdog) || ctx->cancel_req.load())
                __atomic_store_n(ctx->cancel_host, 1, __ATOMIC_SEQ_CST);
            std::this_thread::yield();
        }
        float ms = 0.0f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        total_ms += ms;
        if (!W.pinned) {
            HIP_TRY(ctx, hipMemcpyAsync(W.h_results, W.d_results, n * sizeof(JobResult), hipMemcpyDeviceToHost, s));
            HIP_TRY(ctx, hipStreamSynchronize(s));
        }
        std::memcpy(res, W.h_results, n * sizeof(JobResult));
        if (*ctx->cancel_host) {
            *seconds = total_ms * 1e-3;
            return ctx->cancel_req.load() ? fail(ctx, SMC_E_CANCELLED, "cancelled")
                                          : fail(ctx, SMC_E_TIMEOUT, "watchdog time exceeded");
        }
        bool all = true;
        unsigned long long progress = 0;
        for (int k = 0; k < n; ++k) {
            all = all && res[k].final_flag;
            progress += res[k].issued + (unsigned long long)res[k].final_flag;
        }
        if (all) break;
        // Waves leave when they find no work for a while; a job still open
        // then needs another launch.  Launches that issue no trajectory and
        // finish no job would repeat forever: report that.
        if (progress == last_progress) {
            if (++stalls > 2) return fail(ctx, SMC_E_HIP, "stopping rule made no progress");
        } else {
            stalls = 0;
        }
        last_progress = progress;
    }
    *seconds = total_ms * 1e-3;
    for (int k = 0; k < n; ++k)
        if (!res[k].final_flag) return fail(ctx, SMC_E_HIP, "job did not finish");
    return SMC_OK;
}

void fill_result(const JobResult &r, double z, bool iterative, smc_result *out)
{
    out->n = r.n;
    out->wasted = (iterative && r.issued > r.n) ? r.issued - r.n : 0;
    out->successes = r.yes;
    out->events = r.events;
    out->truncated = r.trunc;
    out->batches = (uint64_t)r.batches;
    out->p_hat = r.n ? (double)r.yes / (double)r.n : 0.0;
    out->z = z;
    if (z > 0.0) smc_wilson_interval(r.yes, r.n, z, &out->lo, &out->hi);
    else {
        out->lo = 0.0;
        out->hi = 1.0;
    }
    // overflow 1: Fig. 2 needed more batches (or trajectories) than allowed;
    // 2: a published bound fell below the look-ahead (an internal error)
    out->status = r.overflow == 1 ? SMC_E_INVALID : r.overflow ? SMC_E_HIP : SMC_OK;
}

}  // namespace

// Accessors used by the surrogate's translation unit.
namespace smc {
int set_ctx_error(smc_ctx *ctx, int code, const std::string &msg) { return fail(ctx, code, msg); }
hipStream_t ctx_stream(smc_ctx *ctx) { return ctx->stream; }
int ctx_device(smc_ctx *ctx) { return ctx->device; }
}  // namespace smc

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int smc_ctx_create(int hip_device, void *hip_stream, smc_ctx **out)
{
    if (!out) return fail(nullptr, SMC_E_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) return fail(nullptr, SMC_E_HIP, "no HIP device");
    if (hip_device < 0 || hip_device >= count) return fail(nullptr, SMC_E_INVALID, "no such device");
    if ((e = hipSetDevice(hip_device)) != hipSuccess) return fail(nullptr, SMC_E_HIP, hipGetErrorString(e));
    smc_ctx *c = new smc_ctx();
    c->device = hip_device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
    if (hip_stream) c->stream = (hipStream_t)hip_stream;
    else {
        if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess) {
            delete c;
            return fail(nullptr, SMC_E_HIP, hipGetErrorString(e));
        }
        c->own_stream = true;
    }
    if ((e = hipHostMalloc((void **)&c->cancel_host, sizeof(int32_t), hipHostMallocMapped)) != hipSuccess ||
        (e = hipHostGetDevicePointer((void **)&c->cancel_dev, c->cancel_host, 0)) != hipSuccess ||
        (e = hipMalloc((void **)&c->d_ctl, sizeof(Control))) != hipSuccess ||
        (e = hipHostMalloc((void **)&c->h_ctl, sizeof(Control), hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreate(&c->ev0)) != hipSuccess || (e = hipEventCreate(&c->ev1)) != hipSuccess ||
        (e = hipEventCreate(&c->ev2)) != hipSuccess) {
        smc_ctx_destroy(c);
        return fail(nullptr, SMC_E_HIP, hipGetErrorString(e));
    }
    *c->cancel_host = 0;
    if ((e = noalloc_scratch(hip_device, &c->noalloc_base)) != hipSuccess) {
        smc_ctx_destroy(c);
        return fail(nullptr, SMC_E_HIP, std::string("fixed job array: ") + hipGetErrorString(e));
    }
    *out = c;
    return SMC_OK;
}

void smc_ctx_destroy(smc_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->d_jobs) (void)hipFree(c->d_jobs);
    if (c->d_states) (void)hipFree(c->d_states);
    if (c->d_results) (void)hipFree(c->d_results);
    if (c->d_rec) (void)hipFree(c->d_rec);
    if (c->d_trace) (void)hipFree(c->d_trace);
    if (c->d_ctl) (void)hipFree(c->d_ctl);
    if (c->cancel_host) (void)hipHostFree(c->cancel_host);
    if (c->h_jobs) (void)hipHostFree(c->h_jobs);
    if (c->h_results) (void)hipHostFree(c->h_results);
    if (c->h_ctl) (void)hipHostFree(c->h_ctl);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->ev2) (void)hipEventDestroy(c->ev2);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *smc_last_error(const smc_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int smc_set_watchdog(smc_ctx *c, double seconds)
{
    if (!c) return SMC_E_INVALID;
    c->watchdog = seconds;
    return SMC_OK;
}

int smc_set_specialization(smc_ctx *c, int mode)
{
    if (!c) return SMC_E_INVALID;
    if (mode != SMC_SPECIALIZE_AUTO && mode != SMC_SPECIALIZE_OFF && mode != SMC_SPECIALIZE_REQUIRED)
        return fail(c, SMC_E_INVALID, "unknown specialization mode");
    c->spec_mode = mode;
    return SMC_OK;
}

int smc_last_kernel(const smc_ctx *c) { return c ? c->last_kernel : -1; }

int smc_autotune(smc_ctx *c, const smc_net *net, const smc_formula *f, const smc_params *p, uint64_t pilot_n,
                 smc_tune_result *out)
{
    if (!c || !net || !f || !p || !out) return fail(c, SMC_E_INVALID, "null argument");
    if (pilot_n == 0 || pilot_n > (1ull << 26)) return fail(c, SMC_E_INVALID, "pilot_n must lie in 1..2^26");
    const auto key = structure_key(net, f);
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) {
        *out = it->second;
        return SMC_OK;
    }
    const int save_wpc = c->waves_per_cu, save_occ = c->spec_waves_per_simd, save_mode = c->spec_mode;
    struct Tuning {
        smc_ctx *c;
        Tuning(smc_ctx *x) : c(x) { c->tuning = true; }
        ~Tuning() { c->tuning = false; }
    } tuning_scope(c);
    smc_params q = *p;
    q.fixed_n = pilot_n;
    q.seed = p->seed ^ 0x9E3779B97F4A7C15ull;   // pilot trajectories are not the estimate's
    if (q.confidence <= 0.0 || q.confidence >= 1.0) q.confidence = 0.95;
    struct Cand {
        int mode, occ;
    };
    std::vector<Cand> cands = {{SMC_SPECIALIZE_OFF, 0}};
    if (spec_supported(net->S, net->M, f->prog))
        for (int occ : {0, 5, 6, 7, 8}) cands.push_back({SMC_SPECIALIZE_REQUIRED, occ});
    const int wpcs[] = {4, 8, 16, 24, 28, 32};
    smc_tune_result best{};
    best.events_per_s = -1.0;
    int tried = 0;
    double default_rate = 0.0;
    int rc = SMC_OK;
    for (const Cand &cd : cands) {
        for (int w : wpcs) {
            c->spec_mode = cd.mode;
            c->spec_waves_per_simd = cd.occ;
            c->waves_per_cu = w;
            smc_result r;
            double rate = 0.0;
            // first run compiles (specialised kernels) and warms up; the second is timed
            for (int rep = 0; rep < 2 && rc == SMC_OK; ++rep) {
                rc = smc_estimate(c, net, f, &q, &r);
                if (rc == SMC_OK && r.device_seconds > 0.0) rate = (double)r.events / r.device_seconds;
            }
            if (rc != SMC_OK) break;
            ++tried;
            if (cd.mode == SMC_SPECIALIZE_REQUIRED && cd.occ == 0 && w == 16) default_rate = rate;
            if (cd.mode == SMC_SPECIALIZE_OFF && w == 16 && cands.size() == 1) default_rate = rate;
            if (rate > best.events_per_s) {
                best.events_per_s = rate;
                best.waves_per_cu = w;
                best.waves_per_simd = cd.occ;
                best.specialization = cd.mode == SMC_SPECIALIZE_OFF ? SMC_SPECIALIZE_OFF : SMC_SPECIALIZE_AUTO;
            }
        }
        if (rc != SMC_OK) break;
    }
    if (rc != SMC_OK) {
        c->waves_per_cu = save_wpc;
        c->spec_waves_per_simd = save_occ;
        c->spec_mode = save_mode;
        return rc;
    }
    best.candidates = tried;
    best.default_events_per_s = default_rate;
    c->waves_per_cu = save_wpc;
    c->spec_waves_per_simd = save_occ;
    c->spec_mode = save_mode;
    c->tuned[key] = best;
    *out = best;
    return SMC_OK;
}

int smc_autotune_batch(smc_ctx *c, const smc_job *jobs, size_t n_jobs, double pilot_widen,
                       smc_batch_tune_result *out)
{
    if (!c || !jobs || !out || n_jobs == 0) return fail(c, SMC_E_INVALID, "null argument or no jobs");
    if (n_jobs > (1u << 20)) return fail(c, SMC_E_INVALID, "too many jobs");
    if (!(pilot_widen >= 1.0 && pilot_widen <= 64.0)) return fail(c, SMC_E_INVALID, "pilot_widen must lie in [1, 64]");
    HIP_TRY(c, hipSetDevice(c->device));
    // the signature of the batch as it will be estimated
    std::vector<Prepared> P(n_jobs);
    for (size_t k = 0; k < n_jobs; ++k)
        if (const int rc = prepare(c, jobs[k].net, jobs[k].formula, &jobs[k].params, 0, P[k])) return rc;
    const uint64_t sig = batch_signature(P.data(), (int)n_jobs);
    const auto hit = c->tuned_batch.find(sig);
    if (hit != c->tuned_batch.end()) {
        *out = hit->second;
        return SMC_OK;
    }
    // The pilot: the same jobs with the interval half-width widened by
    // pilot_widen (about pilot_widen^2 times fewer trajectories, eq. 4), or
    // fixed sizes divided by pilot_widen^2 (at least 64), on seeds of their
    // own, so that the estimate's own trajectories are not consumed.
    std::vector<smc_job> pj(jobs, jobs + n_jobs);
    bool wide = false;
    for (size_t k = 0; k < n_jobs; ++k) {
        smc_params &q = pj[k].params;
        q.seed ^= 0xD1B54A32D192ED03ull;
        if (q.fixed_n == 0) {
            q.half_width = std::min(0.45, q.half_width * pilot_widen);
        } else {
            q.fixed_n = std::max<uint64_t>(64, (uint64_t)((double)q.fixed_n / (pilot_widen * pilot_widen)));
        }
        wide = wide || (P[k].auto_lanes && P[k].M > 4);
    }
    const int save_wpc = c->waves_per_cu, save_lanes = c->lanes;
    struct Tuning {
        smc_ctx *c;
        int wpc, lanes;
        ~Tuning()
        {
            c->tuning = false;
            c->waves_per_cu = wpc;
            c->lanes = lanes;
        }
    } tuning_scope{c, save_wpc, save_lanes};
    c->tuning = true;
    std::vector<smc_result> r(n_jobs);
    auto pilot = [&](int lanes, int wpc, double *secs) {
        c->lanes = lanes;
        c->waves_per_cu = wpc;
        const int rc = smc_estimate_batch(c, pj.data(), n_jobs, r.data());
        *secs = r[0].device_seconds;
        return rc;
    };
    double t = 0.0;
    if (const int rc = pilot(1, 16, &t)) return rc;   // warm-up: specialised kernels compile here
    smc_batch_tune_result best{};
    best.lanes = 1;
    best.waves_per_cu = 16;
    best.seconds = 1e300;
    int tried = 0;
    // coordinate search: lanes per trajectory at 16 waves per CU (upwards
    // until a pilot takes 15 % longer than the best so far), then the waves
    // per CU at the best lanes
    int last_group = 0;
    for (int L : {1, 2, 4, 8, 16}) {
        if (L > 1 && !wide) break;
        // the group size a launch would run with this request (the widest
        // automatic job raises it): a request that gives the same group as
        // the previous one runs the same launch
        int group = 1;
        for (size_t k = 0; k < n_jobs; ++k)
            if (P[k].auto_lanes && !P[k].job.trace) group = std::max(group, lanes_for(L, P[k].M));
        if (group == last_group) continue;
        last_group = group;
        if (const int rc = pilot(L, 16, &t)) return rc;
        ++tried;
        if (L == 1) best.default_seconds = t;
        if (t < best.seconds) {
            best.seconds = t;
            best.lanes = group;   // the group the request gave
        } else if (t > 1.15 * best.seconds) {
            break;
        }
    }
    for (int w : {8, 32}) {
        if (const int rc = pilot(best.lanes, w, &t)) return rc;
        ++tried;
        if (t < best.seconds) {
            best.seconds = t;
            best.waves_per_cu = w;
        }
    }
    best.candidates = tried;
    c->tuned_batch[sig] = best;
    *out = best;
    return SMC_OK;
}

int smc_set_lanes_per_trajectory(smc_ctx *c, int lanes)
{
    if (!c) return SMC_E_INVALID;
    if (lanes != 0 && lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16)
        return fail(c, SMC_E_INVALID, "lanes per trajectory must be 0, 1, 2, 4, 8 or 16");
    c->lanes = lanes;
    return SMC_OK;
}

int smc_set_kernel_occupancy(smc_ctx *c, int waves_per_simd)
{
    if (!c) return SMC_E_INVALID;
    if (waves_per_simd < 0 || waves_per_simd > 8)
        return fail(c, SMC_E_INVALID, "waves per SIMD must lie in 0..8");
    c->spec_waves_per_simd = waves_per_simd;
    return SMC_OK;
}

int smc_set_waves_per_cu(smc_ctx *c, int w)
{
    if (!c) return SMC_E_INVALID;
    if (w < 0 || w > 32) return fail(c, SMC_E_INVALID, "waves_per_cu must lie in 0..32");
    c->waves_per_cu = w;
    return SMC_OK;
}

void smc_cancel(smc_ctx *c)
{
    if (c) c->cancel_req.store(1);
}

int smc_device_cus(const smc_ctx *c) { return c ? c->n_cu : 0; }

// ---- networks ----------------------------------------------------------------
// Device tables hold Mp = M rounded up to kSubBlock channels; the extra ones
// have rate 0, no reactants and no state change, so they add exactly 0 to
// every running sum and are never selected.
static int upload_net(smc_net *n)
{
    smc_ctx *c = n->ctx;
    const int Mp = padded_channels(n->M);
    std::vector<double> rate(Mp, 0.0);
    std::vector<int32_t> reac(2 * Mp, -1);
    std::vector<uint32_t> chg(4 * Mp, 0xFFFF0000u);
    std::copy(n->rate.begin(), n->rate.end(), rate.begin());
    std::copy(n->reac.begin(), n->reac.end(), reac.begin());
    std::copy(n->chg.begin(), n->chg.end(), chg.begin());
    HIP_TRY(c, hipMalloc((void **)&n->d_x0, n->S * sizeof(int32_t)));
    HIP_TRY(c, hipMalloc((void **)&n->d_rate, Mp * sizeof(double)));
    HIP_TRY(c, hipMalloc((void **)&n->d_reac, 2 * Mp * sizeof(int32_t)));
    HIP_TRY(c, hipMalloc((void **)&n->d_chg, 4 * Mp * sizeof(uint32_t)));
    HIP_TRY(c, hipMemcpy(n->d_x0, n->x0.data(), n->S * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(n->d_rate, rate.data(), Mp * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(n->d_reac, reac.data(), 2 * Mp * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(n->d_chg, chg.data(), 4 * Mp * sizeof(uint32_t), hipMemcpyHostToDevice));
    // the generic kernels' form of each channel (padding: zero-order, rate 0)
    std::vector<ChanDev> chan(Mp);
    const int32_t row = kWave * (int32_t)sizeof(int32_t);
    for (int j = 0; j < Mp; ++j) {
        const int ra = j < n->M ? n->reac[2 * j] : -1, rb = j < n->M ? n->reac[2 * j + 1] : -1;
        ChanDev &e = chan[j];
        e.a_off = (ra < 0 ? n->S : ra) * row;
        e.b_code = (rb < 0 ? n->S : rb) * row + ((ra >= 0 && ra == rb) ? 1 : 0);
    }
    HIP_TRY(c, hipMalloc((void **)&n->d_chan, Mp * sizeof(ChanDev)));
    HIP_TRY(c, hipMemcpy(n->d_chan, chan.data(), Mp * sizeof(ChanDev), hipMemcpyHostToDevice));
    return SMC_OK;
}

int smc_net_create(smc_ctx *c, const smc_net_desc *d, smc_net **out)
{
    if (!c || !d || !out) return fail(c, SMC_E_INVALID, "null argument");
    *out = nullptr;
    const int S = d->n_species, M = d->n_reactions;
    if (S < 1 || M < 1 || S > 16384) return fail(c, SMC_E_INVALID, "need 1 <= S <= 16384 and M >= 1");
    if (!d->x0 || !d->rate || !d->reactants || !d->change_idx || !d->change_val)
        return fail(c, SMC_E_INVALID, "missing network array");
    auto *n = new smc_net();
    n->ctx = c;
    n->S = S;
    n->M = M;
    n->x0.assign(d->x0, d->x0 + S);
    n->rate.assign(d->rate, d->rate + M);
    for (int s = 0; s < S; ++s)
        if (n->x0[s] < 0) {
            delete n;
            return fail(c, SMC_E_INVALID, "negative initial count");
        }
    n->reac.resize(2 * M);
    n->chg.resize(4 * M);
    for (int j = 0; j < M; ++j) {
        if (!(n->rate[j] >= 0.0) || std::isinf(n->rate[j])) {
            delete n;
            return fail(c, SMC_E_INVALID, "rate constants must be finite and >= 0");
        }
        int ra = d->reactants[2 * j], rb = d->reactants[2 * j + 1];
        if (ra < -1 || ra >= S || rb < -1 || rb >= S) {
            delete n;
            return fail(c, SMC_E_INVALID, "reactant index out of range");
        }
        if (ra < 0 && rb >= 0) std::swap(ra, rb);
        n->reac[2 * j] = ra;
        n->reac[2 * j + 1] = rb;
        uint32_t packed[4];
        std::vector<std::pair<int, int>> net_change;
        for (int q = 0; q < 4; ++q) {
            const int s = d->change_idx[4 * j + q], v = d->change_val[4 * j + q];
            if (s < -1 || s >= S || v < -32768 || v > 32767) {
                delete n;
                return fail(c, SMC_E_INVALID, "state change out of range");
            }
            packed[q] = s < 0 ? 0xFFFF0000u : (((uint32_t)s << 16) | ((uint32_t)v & 0xFFFFu));
            if (s >= 0) net_change.push_back({s, v});
        }
        // a reaction may not remove more molecules of a species than it consumes
        for (auto &sv : net_change) {
            int total = 0;
            for (auto &o : net_change)
                if (o.first == sv.first) total += o.second;
            const int consumed = (ra == sv.first) + (rb == sv.first);
            if (total < -consumed) {
                delete n;
                return fail(c, SMC_E_INVALID, "reaction consumes more than its reactants");
            }
        }
        for (int q = 0; q < 4; ++q) n->chg[4 * j + q] = packed[q];
    }
    for (int s = 0; s < S; ++s)
        n->names.push_back(d->names && d->names[s] ? std::string(d->names[s]) : "X" + std::to_string(s));
    {
        std::string b = "N";
        b.append((const char *)&n->S, sizeof n->S);
        b.append((const char *)&n->M, sizeof n->M);
        b.append((const char *)n->reac.data(), n->reac.size() * sizeof(int32_t));
        b.append((const char *)n->chg.data(), n->chg.size() * sizeof(uint32_t));
        n->sid = intern_structure(b);
    }
    const int rc = upload_net(n);
    if (rc != SMC_OK) {
        smc_net_destroy(n);
        return rc;
    }
    *out = n;
    return SMC_OK;
}

int smc_net_set_rates(smc_net *n, const double *rate)
{
    if (!n || !rate) return SMC_E_INVALID;
    for (int j = 0; j < n->M; ++j)
        if (!(rate[j] >= 0.0) || std::isinf(rate[j]))
            return fail(n->ctx, SMC_E_INVALID, "rate constants must be finite and >= 0");
    n->rate.assign(rate, rate + n->M);
    HIP_TRY(n->ctx, hipMemcpy(n->d_rate, n->rate.data(), n->M * sizeof(double), hipMemcpyHostToDevice));
    return SMC_OK;
}

void smc_net_destroy(smc_net *n)
{
    if (!n) return;
    if (n->d_x0) (void)hipFree(n->d_x0);
    if (n->d_rate) (void)hipFree(n->d_rate);
    if (n->d_reac) (void)hipFree(n->d_reac);
    if (n->d_chg) (void)hipFree(n->d_chg);
    if (n->d_chan) (void)hipFree(n->d_chan);
    delete n;
}

// ---- formulas ----------------------------------------------------------------
int smc_formula_compile(smc_ctx *c, const smc_net *net, const char *text, smc_formula **out)
{
    if (!c || !net || !text || !out) return fail(c, SMC_E_INVALID, "null argument");
    *out = nullptr;
    auto *f = new smc_formula();
    f->ctx = c;
    try {
        compile_formula(text, net->names, f->prog);
    } catch (const ParseFailure &e) {
        delete f;
        return fail(c, SMC_E_PARSE, e.what());
    } catch (const Unsupported &e) {
        delete f;
        return fail(c, SMC_E_UNSUPPORTED, e.what());
    } catch (const std::exception &e) {
        delete f;
        return fail(c, SMC_E_INVALID, e.what());
    }
    f->horizon = f->prog.horizon;
    f->sid = intern_structure(std::string("F") + std::string((const char *)&f->prog, sizeof(MonProg)));
    hipError_t e = hipMalloc((void **)&f->d_prog, sizeof(MonProg));
    if (e == hipSuccess) e = hipMemcpy(f->d_prog, &f->prog, sizeof(MonProg), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        smc_formula_destroy(f);
        return hip_fail(c, e, "formula upload");
    }
    *out = f;
    return SMC_OK;
}

double smc_formula_horizon(const smc_formula *f) { return f ? f->horizon : NAN; }

int smc_formula_check(const char *text, const char *const *names, int n_names, double *horizon, char *msg,
                      size_t cap)
{
    auto put = [&](const char *m) {
        if (msg && cap > 0) {
            std::strncpy(msg, m, cap - 1);
            msg[cap - 1] = '\0';
        }
    };
    put("");
    if (!text || n_names < 0 || (n_names > 0 && !names)) {
        put("null argument");
        return SMC_E_INVALID;
    }
    std::vector<std::string> nm;
    for (int s = 0; s < n_names; ++s) {
        if (!names[s]) {
            put("null species name");
            return SMC_E_INVALID;
        }
        nm.emplace_back(names[s]);
    }
    MonProg prog;
    try {
        compile_formula(text, nm, prog);
    } catch (const ParseFailure &e) {
        put(e.what());
        return SMC_E_PARSE;
    } catch (const Unsupported &e) {
        put(e.what());
        return SMC_E_UNSUPPORTED;
    } catch (const std::exception &e) {
        put(e.what());
        return SMC_E_INVALID;
    }
    if (horizon) *horizon = prog.horizon;
    return SMC_OK;
}

void smc_formula_destroy(smc_formula *f)
{
    if (!f) return;
    if (f->d_prog) (void)hipFree(f->d_prog);
    delete f;
}

// ---- estimation --------------------------------------------------------------
int smc_estimate_batch(smc_ctx *c, const smc_job *jobs, size_t n_jobs, smc_result *out)
{
    if (!c || (!jobs && n_jobs) || (!out && n_jobs)) return fail(c, SMC_E_INVALID, "null argument");
    if (n_jobs == 0) return SMC_OK;
    if (n_jobs > (1u << 20)) return fail(c, SMC_E_INVALID, "too many jobs");
    HIP_TRY(c, hipSetDevice(c->device));
    std::vector<Prepared> P(n_jobs);
    int first_err = SMC_OK;
    for (size_t k = 0; k < n_jobs; ++k) {
        std::memset(&out[k], 0, sizeof(smc_result));
        const int rc = prepare(c, jobs[k].net, jobs[k].formula, &jobs[k].params, 0, P[k]);
        if (rc != SMC_OK) {
            out[k].status = rc;
            return rc;
        }
    }
    std::vector<JobResult> res;
    double secs = 0.0;
    const int rc = run_jobs(c, P, res, &secs);
    if (rc != SMC_OK) {
        for (size_t k = 0; k < n_jobs; ++k) out[k].status = rc;
        return rc;
    }
    for (size_t k = 0; k < n_jobs; ++k) {
        fill_result(res[k], P[k].z, P[k].job.iterative != 0, &out[k]);
        out[k].device_seconds = secs;
        if (out[k].status != SMC_OK && first_err == SMC_OK) {
            first_err = out[k].status;
            c->err = res[k].overflow == 1 ? "stopping rule ran out of batch slots"
                                          : "stopping rule: a batch bound fell below the issued look-ahead";
        }
    }
    return first_err;
}

int smc_estimate_batch_noalloc(smc_ctx *c, const smc_job *jobs, size_t n_jobs, smc_result *out)
{
    static_assert(SMC_NOALLOC_MAX_JOBS == kNoallocJobs, "the fixed array holds kNoallocJobs jobs");
    if (!c || (!jobs && n_jobs) || (!out && n_jobs)) return fail(c, SMC_E_INVALID, "null argument");
    if (n_jobs > (size_t)SMC_NOALLOC_MAX_JOBS)
        return fail(c, SMC_E_INVALID, "smc_estimate_batch_noalloc takes at most SMC_NOALLOC_MAX_JOBS (64) jobs");
    if (n_jobs == 0) return SMC_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    if (!c->noalloc_base) return fail(c, SMC_E_HIP, "the fixed job array of this device is not mapped");
    // [Control | Job x kNoallocJobs | JobState x kNoallocJobs | JobResult x kNoallocJobs]
    char *base = static_cast<char *>(c->noalloc_base);
    Workspace W;
    W.d_ctl = reinterpret_cast<Control *>(base + kNoallocCtlOff);
    W.d_jobs = reinterpret_cast<Job *>(base + kNoallocJobsOff);
    W.d_states = reinterpret_cast<JobState *>(base + kNoallocStatesOff);
    W.d_results = reinterpret_cast<JobResult *>(base + kNoallocResultsOff);
    Job h_jobs[2 * kNoallocJobs];
    JobResult h_results[kNoallocJobs];
    Control h_ctl;
    W.h_jobs = h_jobs;
    W.h_results = h_results;
    W.h_ctl = &h_ctl;
    W.pinned = false;
    W.no_alloc = true;
    Prepared P[kNoallocJobs];
    for (size_t k = 0; k < n_jobs; ++k) {
        std::memset(&out[k], 0, sizeof(smc_result));
        const int rc = prepare(c, jobs[k].net, jobs[k].formula, &jobs[k].params, 0, P[k], false);
        if (rc != SMC_OK) {
            out[k].status = rc;
            return rc;
        }
    }
    JobResult res[kNoallocJobs];
    double secs = 0.0;
    const int rc = run_jobs_in(c, P, (int)n_jobs, W, res, &secs);
    if (rc != SMC_OK) {
        for (size_t k = 0; k < n_jobs; ++k) out[k].status = rc;
        return rc;
    }
    int first_err = SMC_OK;
    for (size_t k = 0; k < n_jobs; ++k) {
        fill_result(res[k], P[k].z, P[k].job.iterative != 0, &out[k]);
        out[k].device_seconds = secs;
        if (out[k].status != SMC_OK && first_err == SMC_OK) {
            first_err = out[k].status;
            c->err = res[k].overflow == 1 ? "stopping rule ran out of batch slots"
                                          : "stopping rule: a batch bound fell below the issued look-ahead";
        }
    }
    return first_err;
}

int smc_estimate(smc_ctx *c, const smc_net *net, const smc_formula *f, const smc_params *p, smc_result *out)
{
    if (!out) return fail(c, SMC_E_INVALID, "out is NULL");
    smc_job j;
    j.net = net;
    j.formula = f;
    if (p) j.params = *p;
    else std::memset(&j.params, 0, sizeof(j.params));
    return p ? smc_estimate_batch(c, &j, 1, out) : fail(c, SMC_E_INVALID, "params is NULL");
}

int smc_trajectories(smc_ctx *c, const smc_net *net, const smc_formula *f, const smc_params *p,
                     uint64_t first, uint64_t count, uint32_t *events, uint8_t *verdict_reason)
{
    if (!c || !p) return fail(c, SMC_E_INVALID, "null argument");
    if (count == 0) return SMC_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    smc_params q = *p;
    q.fixed_n = count;
    std::vector<Prepared> P(1);
    int rc = prepare(c, net, f, &q, first, P[0]);
    if (rc != SMC_OK) return rc;
    std::vector<JobResult> res;
    double secs = 0.0;
    if (p->flags & SMC_DEVICE_PTRS) {
        // the caller's device arrays are the kernel's record arrays
        if ((uintptr_t)events % alignof(uint32_t)) return fail(c, SMC_E_INVALID, "events must be 4-byte aligned");
        P[0].job.rec_events = events;
        P[0].job.rec_vr = verdict_reason;
        rc = run_jobs(c, P, res, &secs);
        if (rc != SMC_OK) return rc;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return SMC_OK;
    }
    const size_t bytes = count * (sizeof(uint32_t) + sizeof(uint8_t)) + 16;
    if (ensure(c, c->d_rec, c->cap_rec, bytes)) return SMC_E_NOMEM;
    auto *d_ev = (uint32_t *)c->d_rec;
    auto *d_vr = (uint8_t *)(d_ev + count);
    P[0].job.rec_events = d_ev;
    P[0].job.rec_vr = d_vr;
    rc = run_jobs(c, P, res, &secs);
    if (rc != SMC_OK) return rc;
    if (events) HIP_TRY(c, hipMemcpyAsync(events, d_ev, count * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
    if (verdict_reason) HIP_TRY(c, hipMemcpyAsync(verdict_reason, d_vr, count, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SMC_OK;
}

int smc_sample_state(smc_ctx *c, const smc_net *net, const smc_params *p, double T, uint64_t first,
                     uint64_t count, int32_t *counts)
{
    if (!c || !net || !p || !counts) return fail(c, SMC_E_INVALID, "null argument");
    if (count == 0) return SMC_OK;
    if (!(T >= 0.0)) return fail(c, SMC_E_INVALID, "T must be >= 0");
    if (first + count > (1ull << 32)) return fail(c, SMC_E_INVALID, "trajectory indices must stay below 2^32");
    if ((size_t)(net->S + 1) * kWave * sizeof(int32_t) > 65536) return fail(c, SMC_E_INVALID, "network too large");
    HIP_TRY(c, hipSetDevice(c->device));
    Job J;
    std::memset(&J, 0, sizeof(J));
    J.net.S = net->S;
    J.net.M = net->M;
    J.net.Mp = padded_channels(net->M);
    J.net.x0 = net->d_x0;
    J.net.rate = net->d_rate;
    J.net.reac = net->d_reac;
    J.net.chg = net->d_chg;
    J.net.chan = net->d_chan;
    J.seed = p->seed;
    J.first = first;
    J.model_id = p->model_id;
    if (ensure(c, c->d_jobs, c->cap_jobs, 1)) return SMC_E_NOMEM;
    const bool on_device = (p->flags & SMC_DEVICE_PTRS) != 0;
    if (on_device && (uintptr_t)counts % alignof(int32_t)) return fail(c, SMC_E_INVALID, "counts must be 4-byte aligned");
    const size_t bytes = count * (size_t)net->S * sizeof(int32_t);
    if (!on_device && ensure(c, c->d_rec, c->cap_rec, bytes)) return SMC_E_NOMEM;
    int32_t *d_out = on_device ? counts : (int32_t *)c->d_rec;
    HIP_TRY(c, hipMemcpyAsync(c->d_jobs, &J, sizeof(J), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, launch_sample_state(net->M <= 4 ? 0 : 1, c->stream, c->d_jobs, T, count, d_out, net->S));
    if (!on_device) HIP_TRY(c, hipMemcpyAsync(counts, c->d_rec, bytes, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SMC_OK;
}

int smc_wilson_next_device(smc_ctx *c, const uint64_t *successes, const uint64_t *n, size_t count,
                           double eps, double z, uint32_t flags, uint64_t *out)
{
    if (!c || (count && (!successes || !n || !out))) return fail(c, SMC_E_INVALID, "null argument");
    if (!(eps > 0.0 && eps < 0.5) || !(z > 0.0)) return fail(c, SMC_E_INVALID, "need 0 < eps < 0.5, z > 0");
    if (count == 0) return SMC_OK;
    if (count > (1u << 30)) return fail(c, SMC_E_INVALID, "count too large");
    for (size_t k = 0; k < count; ++k)
        if (n[k] == 0 || successes[k] > n[k]) return fail(c, SMC_E_INVALID, "need 0 <= successes <= n, n > 0");
    HIP_TRY(c, hipSetDevice(c->device));
    const size_t bytes = 3 * count * sizeof(uint64_t);
    if (ensure(c, c->d_rec, c->cap_rec, bytes)) return SMC_E_NOMEM;
    auto *d_y = (unsigned long long *)c->d_rec;
    auto *d_n = d_y + count;
    auto *d_o = d_n + count;
    HIP_TRY(c, hipMemcpyAsync(d_y, successes, count * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(d_n, n, count * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, launch_wilson_table(c->stream, d_y, d_n, (int)count, eps, z,
                                   (flags & SMC_PAPER_ROUNDING) ? 1 : 0, d_o));
    HIP_TRY(c, hipMemcpyAsync(out, d_o, count * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return SMC_OK;
}

// ---- Wilson formulas ---------------------------------------------------------
double smc_z_value(double confidence)
{
    if (!(confidence > 0.0 && confidence < 1.0)) return NAN;
    // Newton's method on Phi(z) = (1 + c) / 2 in extended precision.
    const long double q = 0.5L + 0.5L * (long double)confidence;
    long double z = std::sqrt(-2.0L * std::log(1.0L - q));   // rough start
    const long double inv_sqrt2 = 0.70710678118654752440084436210484903928L;
    const long double inv_sqrt2pi = 0.39894228040143267793994605993438186848L;
    for (int it = 0; it < 100; ++it) {
        const long double cdf = 0.5L * std::erfc(-z * inv_sqrt2);
        const long double pdf = inv_sqrt2pi * std::exp(-0.5L * z * z);
        const long double dz = (cdf - q) / pdf;
        z -= dz;
        if (std::fabs(dz) <= 1e-19L * std::fabs(z)) break;
    }
    return (double)z;
}

double smc_wilson_sample_value(double p, double eps, double z) { return wilson_value(p, eps, z); }

uint64_t smc_wilson_sample(double p, double eps, double z)
{
    const double v = wilson_value(p, eps, z);
    return v > 0.0 ? (uint64_t)std::ceil(v) : 0;
}

void smc_wilson_interval(uint64_t k, uint64_t n, double z, double *lo, double *hi)
{
    if (n == 0) {
        if (lo) *lo = 0.0;
        if (hi) *hi = 1.0;
        return;
    }
    const double nd = (double)n;
    const double p = (double)k / nd;
    const double z2 = z * z;
    const double center = p + z2 / (2.0 * nd);
    const double half = z * std::sqrt(p * (1.0 - p) / nd + z2 / ((4.0 * nd) * nd));
    const double den = 1.0 + z2 / nd;
    const double l = (center - half) / den;
    const double h = (center + half) / den;
    if (lo) *lo = l < 0.0 ? 0.0 : l;
    if (hi) *hi = h > 1.0 ? 1.0 : h;
}

}  // extern "C"
