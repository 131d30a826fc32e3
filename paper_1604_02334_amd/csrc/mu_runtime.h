// Host-side handle definitions of the C ABI (opaque to callers).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "mu_internal.h"

struct mu_ctx;

namespace mu {

constexpr int kDefaultTile = 4096;
constexpr int kDefaultAnchor = 64;

// Grow-only device buffer owned by a context.
struct DevBuf {
  void *ptr = nullptr;
  size_t cap = 0;
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
mu_status run_batch(mu_ctx *ctx, int32_t n_jobs, const mu_data *const *data, const mu_theory *const *th,
                    int cost_kind, int32_t ld, const double *params, unsigned mem, double *cost, double *grad,
                    int64_t n_blocks);

}  // namespace mu

struct mu_ctx {
  int device = 0;
  int n_cu = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  int children = 0;
  int tile_bins = mu::kDefaultTile;
  int anchor_every = mu::kDefaultAnchor;
  int specialize = 1;  // use the compiled shape kernels when a theory matches one
  hipEvent_t staging_free = nullptr;  // recorded after each upload from `staging`
  mu::DevBuf partial, dparams, dout, djobs;
  mu::HostBuf staging, staging_out;
  std::vector<mu::DevBuf> extra;
  void release_all();
  // Wait until the last upload from `staging` has been consumed.
  void wait_staging() {
    if (staging_free) hipEventSynchronize(staging_free);
  }
  void mark_staging() {
    if (staging_free) hipEventRecord(staging_free, stream);
  }
};

struct mu_data {
  mu_ctx *ctx = nullptr;
  void *counts = nullptr;  // FP32 or FP64 fit-range counts, concatenated
  int f64 = 0;
  int n_histo = 0;
  int max_row = 0;
  int64_t total = 0;
  std::vector<mu::DevHisto> hh;
  mu::DevHisto *d_histos = nullptr;
  mu::DevTile *d_tiles = nullptr;
  int32_t n_tiles = 0;
  int tiles_for = -1;  // tile size the tables were built for
  mu_status build_tiles(int tile_bins);
};

struct mu_theory {
  mu_ctx *ctx = nullptr;
  mu::DevTheory h;
  int shape = 0;  // mu::Shape of the program
  std::vector<int32_t> map;
  std::vector<double> F, f0;
  int32_t *d_map = nullptr;
  double *d_F = nullptr, *d_f0 = nullptr;
  mu::DevTheory *d_th = nullptr;
  void free_dev();
};
