// Data structures shared by the host runtime, the gfx950 kernels built with
// the library and the kernels compiled at run time (hipRTC) for user-defined
// theories: constants, theory / histogram / job records and launch
// arguments.  Plain data only (the run-time compilation receives this file and
// include/mu.h as in-memory headers, with MU_RTC defined).
#pragma once

#ifndef MU_RTC
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/mu.h"
#else
#include "mu.h"
#endif

namespace mu {

constexpr int kMaxT = MU_MAX_TERMS;
constexpr int kMaxFT = MU_MAX_FACTORS_PER_TERM;
// Resolved scalars of one (vector, histogram) pair, in a fixed order:
// 0 N0, 1 Nbkg, 2..2+kMaxT-1 term amplitudes, then argument a of factor i of
// term k at kArg0 + (k * kMaxFT + i) * 2 + a.
constexpr int kArg0 = 2 + kMaxT;
constexpr int kRS = kArg0 + kMaxT * kMaxFT * 2;  // 30
// Lane steps between a count's load and its use; the counts buffer is padded
// by kPrefetch x kBlock values, more than this many lane steps (of 64 values).
constexpr int kPrefetch = 4;
// The same for batched launches, which stream their counts from HBM (more
// bytes in flight per wave); the padding below covers it.
constexpr int kPrefetchStream = 8;
// Entries of the per-workgroup table of 1 / max(d, 1) for integer counts
// d < kInvTab (chi^2 kernels; FP64, 24 KiB of LDS: six workgroups of the
// cost kernel still fit one compute unit's 160 KiB).
constexpr int kInvTab = 3072;
// Integer counts d < 2^29 are stored as 32-bit values 8 d: the byte offset of
// their entry in that table (no shift before the lookup); kernels take
// d = stored / 8, which is exact.
constexpr uint32_t kCountScale = 8;
constexpr double kCountUnscale = 0.125;
constexpr double kCountIntLimit = 536870912.0;  // 2^29
// Functions of p formed once per segment and shared through LDS (more use the
// per-scalar path).
constexpr int kFunStage = 32;
// Partial slot of one tile: cost (s, c) then kRS gradient components.
constexpr int kSlot = 2 + kRS;  // 32 doubles
constexpr int kBlock = 256;     // threads per evaluation workgroup
constexpr int kWave = 64;       // lanes per wave: the unit of work of an evaluation launch
constexpr int kRefNone = -1;

// Gradient merge plan of one (theory, dataset) pair, int32, built on the host.
// The merge forms, per histogram h and active resolved scalar r (one whose
// reference is a parameter or a function value), the entry gR = sum over h's
// slots of dcost/dR_r, and adds it to the parameter (or, times F[i][k], to
// every parameter k of function i) that the map assigns to r in h's row.
// Layout: [0] n_act, [1] n_par, [2] block stride, act[kRS] at kPlanAct (the
// active scalars r, ascending); then per chunk c of kMergeChunk histograms a
// block at kPlanHead + c * stride: n_pe, n_fe, koff[n_par + 1] (parameter k's
// entries occupy positions koff[k] .. koff[k + 1] - 1 of the sorted list),
// dest[nh * n_act] (for entry e = hh * n_act + i: its position in the sorted
// list, entries of one parameter in entry order; or -1 - j for the j-th entry,
// in entry order, that feeds a function) and fi[n_fe] (the function of each
// function entry).
constexpr int kMergeChunk = 32;  // histograms per merge chunk
// merges of at least kNarrowJobs jobs of at most kNarrowHisto histograms
// each take one wave per job
constexpr int kNarrowJobs = 256, kNarrowHisto = 4;
constexpr int kPlanAct = 4;
constexpr int kPlanHead = 64;
constexpr int kPlanBlockMax = (3 + MU_MAX_PAR + 2 * kMergeChunk * kRS + 63) / 64 * 64;

constexpr __host__ __device__ int arg_index(int k, int i, int a) { return kArg0 + (k * kMaxFT + i) * 2 + a; }

struct DevRef {
  int32_t kind;  // mu_ref_kind, or kRefNone for an unused resolved scalar
  int32_t slot;
  double lit;
};

struct DevTheory {
  double tau_mu;
  double neg_inv_tau;  // -1 / tau_mu
  int32_t n_terms, n_par, n_fun, n_rows, n_slots, pad0;
  int32_t nf[kMaxT];
  int32_t prim[kMaxT][kMaxFT];
  double coef[kMaxT];
  DevRef rref[kRS];    // reference behind each resolved scalar
  const int32_t *map;  // device [n_rows][n_slots]
  const double *F;     // device [n_fun][n_par]
  const double *f0;    // device [n_fun]
};

struct DevHisto {
  int64_t off;    // offset of the first fit-range bin in the counts array
  int64_t n;      // fit-range bins
  int64_t first;  // index of the first fit-range bin in the histogram
  double t0_bin;
  double dt;
  int32_t map_row;
  int32_t pad;
};

// One evaluation job: a parameter vector over one dataset and theory.
struct DevJob {
  const DevTheory *th;
  const DevHisto *histos;
  const void *counts;
  const double *p;       // parameter vector (device)
  double *cost_out;      // [1]
  double *histo_out;     // [n_histo] or null
  double *grad_out;      // [n_par] or null
  double *model_out;     // per-bin N (model evaluation) or null
  const int32_t *plan;   // gradient merge plan (gradient launches) or null
  // Batched launches: the job's first bin in its launch's concatenated fit
  // ranges, that launch's bins per wave, the index of the job's first
  // histogram among the launch's histograms, and the launch's first slot.
  int64_t goff;
  int64_t split_w;
  int32_t jbase;
  int32_t slot_base;
  int32_t n_histo;
  int32_t shape;         // compiled shape of the theory (kShapeGeneric: interpreted)
};

// kModeJac: per bin, sqrt(c_n) dN_n/dR_r for every resolved scalar r into a
// row of kJacCols doubles (c_n: the cost term's second derivative in N),
// for the Gauss-Newton Hessian.
enum Mode : int { kModeCost = 0, kModeGrad = 1, kModeModel = 2, kModeJac = 3 };
constexpr int kJacCols = 32;  // kRS columns and zero padding

// Theory shapes with a compiled specialisation (see mu_eval.hip).
enum Shape : int {
  kShapeGeneric = 0,
  kShapeExpCos = 1,    // A se(lambda) tf(phi, nu)
  kShapeGaussCos = 2,  // A sg(sigma) tf(phi, nu)
  kShapeStg = 3,       // A stg(sigma)
  kShapeExpStg = 4,    // A1 se(lambda) + A2 stg(sigma)
  kShapeExpCosStg = 5,  // A1 se(lambda) tf(phi, nu) + A2 stg(sigma)
  kShapeCount = 6
};

struct LaunchArgs {
  // The unit of work is one wave of kWave lanes; a workgroup holds
  // kBlock / kWave units. Every launch cuts its concatenated work into equal
  // ranges of split_w bins, one per unit; a range is evaluated as the
  // (vector or job, histogram) segments it crosses, and segment (unit u,
  // histogram j of the launch's enumeration) owns slot u + j of `partial`.
  // Uniform launch (jobs == null): n_vec vectors of `total` fit-range bins
  // each over one dataset; job v is `tmpl` with its parameter vector and
  // outputs advanced by v strides; histogram h of vector v is j = v n_histo + h.
  DevJob tmpl;
  int64_t p_stride, grad_stride, histo_stride;
  // Batched launch: the jobs `job_list[0 .. n_vec)` of `jobs`, concatenated
  // in that order (`total` bins); unit u starts in job list entry
  // unit_start[2u] at its histogram unit_start[2u + 1]; histogram h of a job
  // is j = jbase + h.
  const DevJob *jobs;
  const int32_t *job_list;
  const int32_t *unit_start;
  int32_t n_units;
  int32_t cost_kind;
  int32_t anchor_every;  // lane steps between exact re-evaluations, 1..256
  int32_t counts_in_table;  // 1: every count of every job is an integer below kInvTab
  const double *inv_src;    // [kInvTab] 1 / max(i, 1) (device), copied to LDS by chi^2 launches
  int32_t n_vec;
  int64_t split_w;
  int64_t total;
  double *partial;    // this launch's slots
};

}  // namespace mu
