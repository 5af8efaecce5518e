// ssa_kernel.hip -- the generic (table-driven) kernels of the SSA path and
// their host-side launchers.  The device code itself is in ssa_core.h.
#include <mutex>

#include "smc_internal.h"
#include "ssa_core.h"

namespace smc {

#ifndef SMC_MIN_WAVES_PER_EU
#define SMC_MIN_WAVES_PER_EU 1
#endif

// Persistent SSA + monitor kernel reading its tables from device memory.
template <int NB, bool kIter, int G = 1, bool kTree = false>
__global__ __launch_bounds__(256, SMC_MIN_WAVES_PER_EU) void ssa_persistent(KArgs A)
{
    extern __shared__ int32_t lds[];
    persistent_body<DynPolicy<NB, G, kTree>, kIter>(A, lds);
}

// Launches that hold trace programs (one lane per trajectory, any network).
template <bool kIter>
__global__ __launch_bounds__(256, SMC_MIN_WAVES_PER_EU) void ssa_persistent_trace(KArgs A)
{
    extern __shared__ int32_t lds[];
    persistent_body<DynPolicy<kBlocks>, kIter, true>(A, lds);
}

// The persistent kernel of a launch variant: 0 = at most 4 reaction channels,
// 1 = any network, 2..5 = any network, with jobs of 2, 4, 8 or 16 lanes per
// trajectory, 6..9 = the same with tree-ordered sums (SMC_TREE_SUMS), 10 =
// any network, the launch holding trace programs.
template <bool kIter>
static const void *persistent_kernel(int variant)
{
    switch (variant) {
    case 0: return reinterpret_cast<const void *>(&ssa_persistent<4, kIter>);
    case 1: return reinterpret_cast<const void *>(&ssa_persistent<kBlocks, kIter>);
    case 2: return reinterpret_cast<const void *>(&ssa_persistent<kBlocks, kIter, 2>);
    case 3: return reinterpret_cast<const void *>(&ssa_persistent<kBlocks, kIter, 4>);
    case 4: return reinterpret_cast<const void *>(&ssa_persistent<kBlocks, kIter, 8>);
    case 5: return reinterpret_cast<const void *>(&ssa_persistent<kBlocks, kIter, 16>);
    case 6: return reinterpret_cast<const void *>(&ssa_persistent<kBlocks, kIter, 2, true>);
    case 7: return reinterpret_cast<const void *>(&ssa_persistent<kBlocks, kIter, 4, true>);
    case 8: return reinterpret_cast<const void *>(&ssa_persistent<kBlocks, kIter, 8, true>);
    case 9: return reinterpret_cast<const void *>(&ssa_persistent<kBlocks, kIter, 16, true>);
    default: return reinterpret_cast<const void *>(&ssa_persistent_trace<kIter>);
    }
}

// ---------------------------------------------------------------------------
// SSA probe: state at time T of trajectories first .. first+count-1.
// ---------------------------------------------------------------------------
template <int NB, class C>
__global__ __launch_bounds__(256) void ssa_sample_state(const Job *jobp, double T,
                                                        unsigned long long count, int32_t *out,
                                                        int s_max)
{
    extern __shared__ int32_t lds[];
    const int lane = lane_id();
    const int wid = (int)(threadIdx.x / kWave);
    C X;
    X.xs = lds + (size_t)wid * (size_t)(s_max + 1) * kWave;   // + the constant-1 row
    X.lane = lane;
    JobView V;
    V.load(jobp, 0);
    const unsigned long long c = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = c < count;
    const int S = V.S;
    X.init(V.x0, S);
    double t = 0.0;
    uint32_t k = 0;
    bool run = live;
    while (__ballot(run) != 0ull) {
        if (run) {
            Change ch;
            const double tn = ssa_draw<NB>(V, X, event_uniforms(V, V.first + c, k), t, &ch, true);
            if (tn > T) {
                run = false;
            } else {
                X.apply(ch.e0, ch.e1, ch.e2, ch.e3);
                t = tn;
                k = k + 1u;
            }
        }
    }
    if (live)
        for (int s = 0; s < S; ++s) out[c * (unsigned long long)S + s] = X.get(s);
}

// Reset per-job accounting: batch 0 ends at n_first (the rest of the state
// was cleared by the caller).  The first issue limit also covers what every
// outcome of batch 0 would require: whatever the first estimate, the next
// bound is at least the Fig. 2 bound at the estimate's extremes (p = 0 or 1),
// so indices below it are issued at once instead of after the first
// completions.
// The first launch hands every wave a share of its home job's first indices
// without atomics: the waves whose home is job j (ranks 0 .. W_j - 1, see
// persistent_body) take [64 r, 64 r + 64) below static_end, and the job's
// issue counter starts at static_end.  n_waves = 0: no static shares.
// One block per job: the block clears the job's state, then one thread sets
// it up; block 0 also sets the launch's control block.
static_assert(sizeof(JobState) % sizeof(unsigned long long) == 0, "JobState is cleared in 8-byte words");

__global__ void init_jobs(const Job *jobs, int n_jobs, int n_waves, Control *ctl, int open_jobs)
{
    const int j = (int)blockIdx.x;
    if (j >= n_jobs) return;
    const Job &J = jobs[j];
    JobState *st = J.st;
    unsigned long long *words = reinterpret_cast<unsigned long long *>(st);
    for (int i = (int)threadIdx.x; i < (int)(sizeof(JobState) / sizeof(unsigned long long)); i += (int)blockDim.x)
        words[i] = 0ull;
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (j == 0) {
        ctl->open_jobs = open_jobs;
        ctl->stop = 0;
    }
    st->bound[0] = J.n_first;
    st->cnt[0] = kDoneFlag - J.n_first;   // batch 0's bound is published
    unsigned long long lim = J.n_first;
    if (J.iterative) {
        unsigned long long g = next_sample(0.0, J.eps, J.z, J.literal);
        const unsigned long long g1 = next_sample(1.0, J.eps, J.z, J.literal);
        g = g1 < g ? g1 : g;
        if (g > J.capacity) g = J.capacity;
        if (g > lim) lim = g;
    }
    st->limit = lim;
    unsigned long long se = 0;
    if (n_waves > 0) {
        const long long g0 = ((long long)j * n_waves + n_jobs - 1) / n_jobs;
        const long long g1 = ((long long)(j + 1) * n_waves + n_jobs - 1) / n_jobs;
        // a wave runs kWave / lanes trajectories at once
        se = (unsigned long long)(g1 - g0) * (unsigned long long)(kWave / (J.lanes > 1 ? J.lanes : 1));
        if (se > lim) se = lim;
    }
    st->static_end = se;
    st->next = se;
}

// Sum the counter shards of every job into its final numbers (fixed-sample
// jobs are finalised here; iterative jobs were finalised by the kernel) and
// write the compact outcome.
__global__ void finalize_jobs(const Job *jobs, int n_jobs, JobResult *out)
{
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= n_jobs) return;
    JobState *st = jobs[j].st;
    JobResult r;
    if (jobs[j].iterative) {
        r.n = st->n_final;
        r.yes = st->yes_final;
        r.events = 0;
        r.trunc = 0;
        for (int b = 0; b < st->n_batches; ++b) {   // trajectories past n_final are excluded
            r.events += sum_shards(st->events, b);
            r.trunc += sum_shards(st->trunc, b);
        }
        r.batches = st->n_batches;
        r.final_flag = st->final_flag;
        r.overflow = st->overflow;
    } else {
        r.n = st->bound[0];
        r.yes = sum_shards(st->yes, 0);
        r.events = sum_shards(st->events, 0);
        r.trunc = sum_shards(st->trunc, 0);
        r.batches = 1;
        r.final_flag = (st->next >= st->bound[0]) ? 1 : 0;
        r.overflow = 0;
    }
    r.issued = st->next;
    r.pad = 0;
    out[j] = r;
}

// Fig. 2 applied to verdicts recorded for every index up to a job's capacity
// (a speculative launch ran them all at once): the same bounds, estimate and
// counts as the batch protocol of the persistent kernel, which would see
// exactly these verdicts of exactly these indices, with the same operations
// (next_sample) deciding each bound.  One wave per job.
__global__ __launch_bounds__(64) void replay_wilson(const Job *jobs, int n_jobs, JobResult *out)
{
    const int j = (int)blockIdx.x;
    if (j >= n_jobs) return;
    const Job &J = jobs[j];
    const int lane = (int)threadIdx.x;
    unsigned long long Y = 0, lo = 0, B = J.n_first;
    int b = 0, overflow = 0;
    for (;;) {
        unsigned long long y = 0;   // TRUE verdicts among [lo, B)
        for (unsigned long long i = lo + (unsigned long long)lane; i < B; i += kWave) y += J.rec_vr[i] & 1u;
        Y += wave_sum_u64(y);
        const double p_hat = (double)Y / (double)B;
        const unsigned long long Np = next_sample(p_hat, J.eps, J.z, J.literal);
        if (Np > B && b + 1 < kMaxBatches && Np <= J.capacity) {
            lo = B;
            B = Np;
            ++b;
            continue;
        }
        overflow = Np > B ? 1 : 0;
        break;
    }
    unsigned long long ev = 0, tr = 0;
    for (unsigned long long i = (unsigned long long)lane; i < B; i += kWave) {
        ev += J.rec_events[i];
        tr += ((J.rec_vr[i] >> 1) == (uint8_t)RS_CAP) ? 1u : 0u;
    }
    ev = wave_sum_u64(ev);
    tr = wave_sum_u64(tr);
    if (lane == 0) {
        JobResult r;
        r.n = B;
        r.yes = Y;
        r.events = ev;
        r.trunc = tr;
        r.issued = J.capacity;
        r.batches = b + 1;
        r.final_flag = 1;
        r.overflow = overflow;
        r.pad = 0;
        out[j] = r;
    }
}

// Device-side eq. 4 over a table of (successes, n): used to check that the
// device and host stopping rules agree.
__global__ void wilson_table(const unsigned long long *yes, const unsigned long long *n, int count,
                             double eps, double z, int literal, unsigned long long *out)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= count) return;
    out[i] = next_sample((double)yes[i] / (double)n[i], eps, z, literal);
}

}  // namespace smc

// ---------------------------------------------------------------------------
// Host-side launch wrappers (called from the runtime, C++ linkage).
// ---------------------------------------------------------------------------
namespace smc {

// variant: see persistent_kernel; iterative:
// the launch holds jobs with the Fig. 2 stopping rule
hipError_t launch_persistent(int variant, bool iterative, int grid, int waves_per_block, size_t lds_bytes,
                             hipStream_t stream, const Job *jobs, int n_jobs, int s_max,
                             Control *ctl, const volatile int32_t *cancel, int spin_limit, int static_first,
                             unsigned long long room_max)
{
    KArgs a;
    a.jobs = jobs;
    a.n_jobs = n_jobs;
    a.s_max = s_max;
    a.ctl = ctl;
    a.cancel = cancel;
    a.spin_limit = spin_limit;
    a.waves_per_block = waves_per_block;
    a.static_first = static_first;
    a.room_max = room_max;
    const dim3 block(kWave * waves_per_block);
    const void *fn = iterative ? persistent_kernel<true>(variant) : persistent_kernel<false>(variant);
    void *args[] = {&a};
    const hipError_t e = hipLaunchKernel(fn, dim3(grid), block, args, lds_bytes, stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// Blocks of a persistent kernel that fit on one CU at once (0 if unknown).
int persistent_blocks_per_cu(int variant, bool iterative, int waves_per_block, size_t lds_bytes)
{
    int nb = 0;
    const int threads = kWave * waves_per_block;
    const void *fn = iterative ? persistent_kernel<true>(variant) : persistent_kernel<false>(variant);
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, lds_bytes);
    return e == hipSuccess ? nb : 0;
}

int module_blocks_per_cu(hipFunction_t fn, int waves_per_block, size_t lds_bytes)
{
    int nb = 0;
    const hipError_t e =
        hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kWave * waves_per_block, lds_bytes);
    return e == hipSuccess ? nb : 0;
}

hipError_t launch_module(hipFunction_t fn, int grid, int waves_per_block, size_t lds_bytes, hipStream_t stream,
                         const Job *jobs, int n_jobs, int s_max, Control *ctl,
                         const volatile int32_t *cancel, int spin_limit, int static_first,
                         unsigned long long room_max)
{
    KArgs a;
    a.jobs = jobs;
    a.n_jobs = n_jobs;
    a.s_max = s_max;
    a.ctl = ctl;
    a.cancel = cancel;
    a.spin_limit = spin_limit;
    a.waves_per_block = waves_per_block;
    a.static_first = static_first;
    a.room_max = room_max;
    void *params[] = {&a};
    return hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, (unsigned)(kWave * waves_per_block), 1, 1,
                                 (unsigned)lds_bytes, stream, params, nullptr);
}

hipError_t launch_sample_state(int variant, hipStream_t stream, const Job *job, double T,
                               unsigned long long count, int32_t *out, int s_max)
{
    const int threads = kWave;
    const unsigned long long blocks = (count + threads - 1) / threads;
    const size_t lds = (size_t)(s_max + 1) * kWave * sizeof(int32_t);
    if (variant == 0)
        hipLaunchKernelGGL((ssa_sample_state<4, LdsCounts>), dim3((unsigned)blocks), dim3(threads), lds,
                           stream, job, T, count, out, s_max);
    else
        hipLaunchKernelGGL((ssa_sample_state<kBlocks, LdsCounts>), dim3((unsigned)blocks), dim3(threads),
                           lds, stream, job, T, count, out, s_max);
    return hipGetLastError();
}

hipError_t launch_init(hipStream_t stream, const Job *jobs, int n_jobs, int n_waves, Control *ctl, int open_jobs)
{
    hipLaunchKernelGGL(init_jobs, dim3(n_jobs), dim3(256), 0, stream, jobs, n_jobs, n_waves, ctl, open_jobs);
    return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t stream, const Job *jobs, int n_jobs, JobResult *out)
{
    hipLaunchKernelGGL(finalize_jobs, dim3((n_jobs + 63) / 64), dim3(64), 0, stream, jobs, n_jobs,
                       out);
    return hipGetLastError();
}

hipError_t launch_replay(hipStream_t stream, const Job *jobs, int n_jobs, JobResult *out)
{
    hipLaunchKernelGGL(replay_wilson, dim3(n_jobs), dim3(kWave), 0, stream, jobs, n_jobs, out);
    return hipGetLastError();
}

hipError_t launch_wilson_table(hipStream_t stream, const unsigned long long *yes,
                               const unsigned long long *n, int count, double eps, double z,
                               int literal, unsigned long long *out)
{
    hipLaunchKernelGGL(wilson_table, dim3((count + 255) / 256), dim3(256), 0, stream, yes, n, count,
                       eps, z, literal, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The fixed job array of allocation-free runs (smc_estimate_batch_noalloc):
// job descriptors, per-job counters and results, and the control block, for
// at most kNoallocJobs jobs.  Every GPU holds its own copy at its own address
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not device memory: kernels are given the device address that
// hipGetSymbolAddress returns for it, looked up once per device with that
// device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

hipError_t noalloc_scratch(int device, void **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

}  // namespace smc
