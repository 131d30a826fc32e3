// Host-side handle definitions of the C ABI (opaque to callers).
#pragma once

#include <hip/hip_runtime.h>

#include <deque>
#include <string>
#include <vector>

#include "mu_internal.h"

struct mu_ctx;

namespace mu {

constexpr int kMinTile = 1024, kMaxTile = 65536;
constexpr int kMaxSplit = 1 << 26;  // largest explicit bins-per-unit value
// Longest range of a gradient pass's wave: each lane sums at most 2^14 terms
// plainly (cost passes fold their sums by TwoSum at every anchor instead).
constexpr int kMaxGradSplit = 1 << 20;
constexpr int kDefaultAnchor = 64;

// Grow-only device buffer owned by a context.  A fixed buffer (memory the
// buffer does not own) never grows: ensure() then refuses larger requests.
struct DevBuf {
  void *ptr = nullptr;
  size_t cap = 0;
  bool fixed = false;
  mu_status ensure(mu_ctx *ctx, size_t bytes, bool zero);
  void release();
};

// Grow-only pinned host buffer owned by a context.
struct HostBuf {
  void *ptr = nullptr;
  size_t cap = 0;
  mu_status ensure(mu_ctx *ctx, size_t bytes);
  void release();
};

void set_err(mu_ctx *ctx, const char *fmt, ...);
mu_status hip_fail(mu_ctx *ctx, hipError_t e, const char *what);
mu_status check_pair(mu_ctx *ctx, const mu_data *d, const mu_theory *th);
// n_vec vectors over one dataset in one launch (mode: cost, grad or model).
mu_status eval_uniform(mu_ctx *ctx, mu_data *d, const mu_theory *th, int cost_kind, const double *params,
                       int32_t n_vec, unsigned mem, double *cost, double *histo, double *grad, double *model,
                       int mode);
// The same with device pointers only, on stream s with partial slots `partial`.
mu_status eval_dev(mu_ctx *ctx, mu_data *d, const mu_theory *th, int cost_kind, const double *dp, int32_t n_vec,
                   double *dc, double *dh, double *dg, double *dm, int mode, hipStream_t s, DevBuf &partial);
// n_jobs (dataset, theory, vector) jobs: one launch for the jobs of compiled
// shapes, one for the others, then one merge launch.
mu_status run_batch(mu_ctx *ctx, int32_t n_jobs, const mu_data *const *data, const mu_theory *const *th,
                    int cost_kind, int32_t ld, const double *params, unsigned mem, double *cost, double *grad);

}  // namespace mu

struct mu_ctx {
  int device = 0;
  int n_cu = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  int children = 0;
  int tile_bins = 0;  // 0: chosen per launch (tuned table, else heuristic)
  int anchor_every = mu::kDefaultAnchor;
  // measured best (tile, anchor) per (shape, mode, cost, log2 of bin-evaluations)
  struct Tuned {
    int key, tile, anchor;
  };
  std::vector<Tuned> tuned;
  // Bins per wave of a batched launch (generic: the interpreted kernel's
  // launch, else the compiled shapes' launch) of `work` bins.
  int64_t pick_batch(int generic, int mode, int cost, int count_f64, int64_t work, int *anchor) const;
  // Bins per wave of a split launch (single dataset, n_vec vectors).
  int64_t pick_split(int shape, int mode, int cost, int count_f64, int64_t work, int *anchor) const;
  int specialize = 1;  // use the compiled shape kernels when a theory matches one
  hipEvent_t staging_free = nullptr;  // recorded after each upload from `staging`
  double *d_inv = nullptr;  // [kInvTab] 1 / max(i, 1): source of the kernels' LDS table
  // partial_aux: the gradient pass's slots in mu_chi2_eval_grad
  mu::DevBuf partial, partial_aux, dparams, dout, djobs;
  mu::DevBuf jac, gram;  // mu_hesse: Jacobian rows, Gram partial blocks
  double *scratch = nullptr;  // this device's allocation-free slots (static_scratch)
  // kernels of run-time compiled theories, one module per distinct source
  struct RtcModule {
    std::string src;
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
  };
  std::vector<RtcModule> rtc;
  mu::HostBuf staging, staging_out;
  std::vector<mu::DevBuf> extra;
  void release_all();
  // Launch timing (events on `stream` around kernel launches while enabled).
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;  // created on demand, destroyed with the context
  struct Timed {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Timed> timed;
  // Records the start event of a timed launch; returns the index to close, or -1.
  int time_begin(int kind, hipStream_t s);
  void time_end(int idx, hipStream_t s);

  // Wait until the last upload from `staging` has been consumed.
  void wait_staging() {
    if (staging_free) (void)hipEventSynchronize(staging_free);
  }
  void mark_staging() {
    if (staging_free) (void)hipEventRecord(staging_free, stream);
  }
};

struct mu_data {
  mu_ctx *ctx = nullptr;
  void *counts = nullptr;  // FP32 or FP64 fit-range counts, concatenated
  int f64 = 0;
  int n_histo = 0;
  int max_row = 0;
  int64_t total = 0;
  int64_t longest = 0;     // bins of the longest fit range
  double max_count = 0.0;  // largest fit-range count
  std::vector<mu::DevHisto> hh;
  mu::DevHisto *d_hh = nullptr;  // device copy of hh
  // Gradient merge plans, one per theory used with this dataset (by theory
  // id), built on first use and kept until destruction.
  struct Plan {
    uint64_t theory_id;
    int32_t *d;
    int lds;  // dynamic LDS bytes its merge needs
  };
  std::vector<Plan> plans;
  mu_status grad_plan(const mu_theory *th, const int32_t **out, int *lds = nullptr);
  void free_dev();
};

struct mu_theory {
  mu_ctx *ctx = nullptr;
  uint64_t id = 0;  // unique per process (never reused, unlike the address)
  mu::DevTheory h;
  int shape = 0;  // mu::Shape of the program
  std::vector<int32_t> map;
  std::vector<double> F, f0;
  int32_t *d_map = nullptr;
  double *d_F = nullptr, *d_f0 = nullptr;
  mu::DevTheory *d_th = nullptr;
  hipFunction_t rtc_fn = nullptr;  // run-time compiled theory: its kernel (else null)
  int rtc_refs = 0;                // and the number of its expression references
  void free_dev();
};
