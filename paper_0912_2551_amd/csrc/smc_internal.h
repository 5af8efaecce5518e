// smc_internal.h -- declarations shared by the host runtime translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>
#include <vector>

#include "smc_device.h"

namespace smc {

struct ParseFailure : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct Unsupported : std::runtime_error {
    using std::runtime_error::runtime_error;
};

// Device memory for the record areas of trace programs in one launch.
constexpr unsigned long long kTraceBudget = 8ull << 30;

// formula.cpp
void compile_formula(const std::string &text, const std::vector<std::string> &names, MonProg &out);

// ssa_kernel.hip (room_max: the largest capacity of the launch's jobs)
hipError_t launch_persistent(int nb_variant, bool iterative, int grid, int waves_per_block, size_t lds_bytes,
                             hipStream_t stream, const Job *jobs, int n_jobs, int s_max,
                             Control *ctl, const volatile int32_t *cancel, int spin_limit, int static_first,
                             unsigned long long room_max);
hipError_t launch_sample_state(int nb_variant, hipStream_t stream, const Job *job, double T,
                               unsigned long long count, int32_t *out, int s_max);
// a specialised persistent kernel (spec.cpp) with the generic kernel's arguments
hipError_t launch_module(hipFunction_t fn, int grid, int waves_per_block, size_t lds_bytes, hipStream_t stream,
                         const Job *jobs, int n_jobs, int s_max, Control *ctl,
                         const volatile int32_t *cancel, int spin_limit, int static_first,
                         unsigned long long room_max);
int persistent_blocks_per_cu(int variant, bool iterative, int waves_per_block, size_t lds_bytes);
int module_blocks_per_cu(hipFunction_t fn, int waves_per_block, size_t lds_bytes);
// Clears and sets up the jobs' state and the control block of the first
// launch.  n_waves: waves of the first launch (their static first shares), 0
// for none; open_jobs: iterative jobs of the launch.
hipError_t launch_init(hipStream_t stream, const Job *jobs, int n_jobs, int n_waves, Control *ctl, int open_jobs);
hipError_t launch_finalize(hipStream_t stream, const Job *jobs, int n_jobs, JobResult *out);
// Fig. 2 over recorded per-index verdicts (speculative launches)
hipError_t launch_replay(hipStream_t stream, const Job *jobs, int n_jobs, JobResult *out);
// Allocation-free runs (smc_estimate_batch_noalloc): the device address of the
// library's fixed job array on `device`, which must be the current device.
// The address is looked up once per device and kept.  Layout: the control
// block, then kNoallocJobs job descriptors, job states and results at the
// offsets below.
constexpr int kNoallocJobs = 64;
constexpr size_t kNoallocAlign = 256;
constexpr size_t noalloc_round(size_t b) { return (b + kNoallocAlign - 1) / kNoallocAlign * kNoallocAlign; }
constexpr size_t kNoallocCtlOff = 0;
constexpr size_t kNoallocJobsOff = kNoallocCtlOff + noalloc_round(sizeof(Control));
constexpr size_t kNoallocStatesOff = kNoallocJobsOff + noalloc_round(kNoallocJobs * sizeof(Job));
constexpr size_t kNoallocResultsOff = kNoallocStatesOff + noalloc_round(kNoallocJobs * sizeof(JobState));
constexpr size_t kNoallocBytes = kNoallocResultsOff + noalloc_round(kNoallocJobs * sizeof(JobResult));
hipError_t noalloc_scratch(int device, void **ptr);
hipError_t launch_wilson_table(hipStream_t stream, const unsigned long long *yes,
                               const unsigned long long *n, int count, double eps, double z,
                               int literal, unsigned long long *out);

// spec.cpp
bool spec_supported(int S, int M, const MonProg &mp);
// the specialised kernel of (S, M) keeps its counts in LDS (StaticWidePolicy)
bool spec_wide(int S, int M);
// waves_per_simd > 0: register budget for that many waves per SIMD
std::string spec_source(int S, int M, const int32_t *reac, const uint32_t *chg, const MonProg &mp,
                        int waves_per_simd, bool iterative);
int spec_kernel(int device, const std::string &src, hipFunction_t *fn, std::string &err);

}  // namespace smc
