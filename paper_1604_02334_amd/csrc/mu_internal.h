// Launch functions of the gfx950 kernels (host side), over the structures of
// mu_structs.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mu_structs.h"

namespace mu {

hipError_t launch_eval(const LaunchArgs &a, int mode, int count_f64, int shape, hipStream_t s);
// The Jacobian-mode evaluation (rows of kJacCols doubles into tmpl.model_out)
// of a uniform launch with one vector.
hipError_t launch_jac(const LaunchArgs &a, int count_f64, int shape, hipStream_t s);
// Gauss-Newton blocks: per histogram h, HR[h] (kJacCols x kJacCols) = sum of
// J_n J_n^T over its rows; units[3u .. 3u + 2] = (histogram, first row, end
// row) in histogram order, ufirst[h] = first unit of h (n_histo + 1 entries),
// part: n_units x 1024 doubles of scratch.
hipError_t launch_gram(const double *J, const int64_t *units, int n_units, double *part, const int32_t *ufirst,
                       int n_histo, double *HR, hipStream_t s);
// The kernel of a run-time compiled theory (module function `fn`) over a
// uniform or batched launch, in mode `mode` (cost, gradient, model, Jacobian).
hipError_t launch_rtc(hipFunction_t fn, const LaunchArgs &a, int mode, int count_f64, hipStream_t s);
// Slots of the allocation-free entry point: kStaticSlots per device, in a
// __device__ array; static_scratch_init (with the device made current)
// looks up its address on `device` once; static_scratch returns it (null
// before init).
constexpr int kStaticSlots = 32768;  // 8 MiB of slots
constexpr int kMaxDevices = 64;
hipError_t static_scratch_init(int device);
double *static_scratch(int device);
// A gradient launch g and a cost launch c of the same dataset and theory as
// one launch, for the cases eval_grad_cost_fused accepts (chi^2, compiled
// shapes, 32-bit counts; others take two launches); hipErrorNotSupported
// otherwise.
bool eval_grad_cost_fused(int count_f64, int shape, int cost_kind);
hipError_t launch_eval_grad_cost(const LaunchArgs &g, const LaunchArgs &c, int count_f64, int shape, hipStream_t s);
// Workgroups (of kBlock / kWave units each) of the evaluation kernel resident
// per compute unit (0 if unknown).
int eval_blocks_per_cu(int mode, int cost_kind, int count_f64, int shape);
// One batched launch over jobs of compiled shapes (each segment runs its
// job's shape) or, with generic != 0, of any theory (interpreted).
hipError_t launch_eval_batch(const LaunchArgs &a, int mode, int count_f64, int generic, hipStream_t s);
int eval_batch_blocks_per_cu(int mode, int cost_kind, int count_f64, int generic);
// Merge the slots of jobs [0, n_jobs) of `a` (uniform or batched).
// narrow: one wave per job (launches of many jobs of few histograms each).
hipError_t launch_merge(const LaunchArgs &a, int mode, int n_jobs, int lds_bytes, bool narrow, hipStream_t s);
// One launch merging a gradient launch's n_grad jobs and a cost launch's n_cost jobs.
hipError_t launch_merge_grad_cost(const LaunchArgs &g, int n_grad, const LaunchArgs &c, int n_cost, int lds_bytes,
                                  hipStream_t s);

}  // namespace mu
