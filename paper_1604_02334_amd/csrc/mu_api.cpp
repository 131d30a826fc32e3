// Host runtime of the C ABI declared in include/mu.h: contexts, device-resident
// histograms, validated theory programs and evaluation launches.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "mu_internal.h"
#include "mu_runtime.h"

using namespace mu;

// ------------------------------------------------------------------ helpers

namespace mu {

void set_err(mu_ctx *ctx, const char *fmt, ...) {
  if (!ctx) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  ctx->err = buf;
}

static void put_msg(char *msg, int32_t len, const std::string &s) {
  if (msg && len > 0) {
    std::snprintf(msg, (size_t)len, "%s", s.c_str());
  }
}

mu_status hip_fail(mu_ctx *ctx, hipError_t e, const char *what) {
  set_err(ctx, "%s failed: %s", what, hipGetErrorString(e));
  return MU_E_DEVICE;
}

mu_status DevBuf::ensure(mu_ctx *ctx, size_t bytes, bool zero) {
  if (bytes <= cap) return MU_OK;
  if (fixed) {
    set_err(ctx, "the launch needs %zu bytes of partial slots, more than the %zu bytes of the fixed slot array",
            bytes, cap);
    return MU_E_UNSUPPORTED;
  }
  if (ptr) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ptr);
    ptr = nullptr;
    cap = 0;
  }
  size_t want = std::max<size_t>(bytes, 4096);
  want = (want + 4095) & ~size_t(4095);
  hipError_t e = hipMalloc(&ptr, want);
  if (e != hipSuccess) {
    ptr = nullptr;
    set_err(ctx, "device allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
    return MU_E_NOMEM;
  }
  cap = want;
  if (zero) {
    e = hipMemsetAsync(ptr, 0, want, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemsetAsync");
  }
  return MU_OK;
}

void DevBuf::release() {
  if (ptr && !fixed) (void)hipFree(ptr);
  ptr = nullptr;
  cap = 0;
}

mu_status HostBuf::ensure(mu_ctx *ctx, size_t bytes) {
  if (bytes <= cap) return MU_OK;
  if (ptr) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipHostFree(ptr);
    ptr = nullptr;
    cap = 0;
  }
  size_t want = std::max<size_t>(bytes, 4096);
  want = (want + 4095) & ~size_t(4095);
  hipError_t e = hipHostMalloc(&ptr, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    ptr = nullptr;
    set_err(ctx, "pinned host allocation of %zu bytes failed: %s", want, hipGetErrorString(e));
    return MU_E_NOMEM;
  }
  cap = want;
  return MU_OK;
}

void HostBuf::release() {
  if (ptr) (void)hipHostFree(ptr);
  ptr = nullptr;
  cap = 0;
}

}  // namespace mu

// ----------------------------------------------------------------- version

extern "C" int mu_abi_version(void) { return MU_ABI_VERSION; }

extern "C" const char *mu_status_string(mu_status s) {
  switch (s) {
    case MU_OK: return "ok";
    case MU_E_ARG: return "invalid argument";
    case MU_E_NODEVICE: return "no usable GPU";
    case MU_E_NOMEM: return "out of memory";
    case MU_E_DEVICE: return "HIP error";
    case MU_E_UNSUPPORTED: return "unsupported";
    case MU_E_STATE: return "invalid state";
  }
  return "unknown status";
}

// ----------------------------------------------------------------- context

static bool forced_nodevice() {
  const char *v = std::getenv("MU_FORCE_NODEVICE");
  return v && v[0] && std::strcmp(v, "0") != 0;
}

extern "C" mu_status mu_ctx_create(int device, void *hip_stream, unsigned flags, mu_ctx **out) {
  if (!out) return MU_E_ARG;
  *out = nullptr;
  if (flags != 0) return MU_E_ARG;
  if (forced_nodevice()) return MU_E_NODEVICE;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return MU_E_NODEVICE;
  if (device < 0 || device >= n) return MU_E_ARG;
  if (hipSetDevice(device) != hipSuccess) return MU_E_NODEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return MU_E_DEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return MU_E_UNSUPPORTED;
  // the allocation-free entry point's slots on this device (looked up once
  // per device, with the device current); without them only that entry
  // point is unavailable
  const hipError_t scratch_e = static_scratch_init(device);
  mu_ctx *c = new mu_ctx();
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  c->scratch = scratch_e == hipSuccess ? static_scratch(device) : nullptr;
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->own_stream = false;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return MU_E_DEVICE;
    }
    c->own_stream = true;
  }
  if (hipEventCreateWithFlags(&c->staging_free, hipEventDisableTiming) != hipSuccess) {
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return MU_E_DEVICE;
  }
  // 1 / max(i, 1) for i < kInvTab, correctly rounded (IEEE division), copied
  // into LDS by every chi^2 evaluation workgroup
  {
    std::vector<double> inv(kInvTab);
    for (int i = 0; i < kInvTab; ++i) inv[i] = 1.0 / (double)(i > 0 ? i : 1);
    hipError_t e = hipMalloc(&c->d_inv, inv.size() * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(c->d_inv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      if (c->d_inv) (void)hipFree(c->d_inv);
      (void)hipEventDestroy(c->staging_free);
      if (c->own_stream) (void)hipStreamDestroy(c->stream);
      delete c;
      return MU_E_DEVICE;
    }
  }
  *out = c;
  return MU_OK;
}

extern "C" mu_status mu_ctx_destroy(mu_ctx *ctx) {
  if (!ctx) return MU_E_ARG;
  if (ctx->children != 0) {
    set_err(ctx, "context still owns %d live handles", ctx->children);
    return MU_E_STATE;
  }
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->release_all();
  if (ctx->d_inv) (void)hipFree(ctx->d_inv);
  if (ctx->staging_free) (void)hipEventDestroy(ctx->staging_free);
  for (hipEvent_t ev : ctx->ev_pool) (void)hipEventDestroy(ev);
  for (auto &m : ctx->rtc)
    if (m.mod) (void)hipModuleUnload(m.mod);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return MU_OK;
}

void mu_ctx::release_all() {
  partial.release();
  partial_aux.release();
  dparams.release();
  dout.release();
  djobs.release();
  jac.release();
  gram.release();
  staging.release();
  staging_out.release();
  for (auto &b : extra) b.release();
}

int mu_ctx::time_begin(int kind, hipStream_t s) {
  if (!timing) return -1;
  const size_t need = 2 * (timed.size() + 1);
  while (ev_pool.size() < need) {
    hipEvent_t ev;
    // timing-only events: no system-scope fence (cache write-back) at each record
    if (hipEventCreateWithFlags(&ev, hipEventDisableSystemFence) != hipSuccess) return -1;  // best effort
    ev_pool.push_back(ev);
  }
  Timed t{kind, ev_pool[need - 2], ev_pool[need - 1]};
  if (hipEventRecord(t.a, s) != hipSuccess) return -1;
  timed.push_back(t);
  return (int)timed.size() - 1;
}

void mu_ctx::time_end(int idx, hipStream_t s) {
  if (idx >= 0) (void)hipEventRecord(timed[idx].b, s);  // timing only
}

extern "C" mu_status mu_ctx_timing(mu_ctx *ctx, int32_t enable) {
  if (!ctx) return MU_E_ARG;
  if (enable) ctx->timed.clear();
  ctx->timing = enable != 0;
  return MU_OK;
}

extern "C" mu_status mu_ctx_timing_read(mu_ctx *ctx, int32_t kind, int32_t *n_launches, double *total_ms) {
  if (!ctx) return MU_E_ARG;
  if (kind < MU_TIME_EVAL_COST || kind > MU_TIME_EVAL_GRAD_COST || !n_launches || !total_ms) {
    set_err(ctx, "mu_ctx_timing_read: unknown kind %d or NULL output", kind);
    return MU_E_ARG;
  }
  (void)hipSetDevice(ctx->device);
  int32_t n = 0;
  double tot = 0.0;
  for (const auto &t : ctx->timed) {
    if (t.kind != kind) continue;
    hipError_t e = hipEventSynchronize(t.b);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, t.a, t.b);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
    tot += ms;
    ++n;
  }
  *n_launches = n;
  *total_ms = tot;
  return MU_OK;
}

extern "C" const char *mu_ctx_last_error(const mu_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" mu_status mu_ctx_synchronize(mu_ctx *ctx) {
  if (!ctx) return MU_E_ARG;
  (void)hipSetDevice(ctx->device);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? MU_OK : hip_fail(ctx, e, "hipStreamSynchronize");
}

extern "C" mu_status mu_ctx_set_tile(mu_ctx *ctx, int32_t tile_bins) {
  if (!ctx) return MU_E_ARG;
  if (tile_bins == 0) {
    ctx->tile_bins = 0;
    return MU_OK;
  }
  if (tile_bins < kWave || tile_bins > kMaxSplit) {
    set_err(ctx, "tile_bins must be 0 or in [%d, %d]", kWave, kMaxSplit);
    return MU_E_ARG;
  }
  ctx->tile_bins = tile_bins;
  return MU_OK;
}

extern "C" int32_t mu_ctx_get_tile(const mu_ctx *ctx) { return ctx ? ctx->tile_bins : -1; }

extern "C" mu_status mu_ctx_set_anchor(mu_ctx *ctx, int32_t every) {
  if (!ctx) return MU_E_ARG;
  if (every == 0) {
    ctx->anchor_every = kDefaultAnchor;
    return MU_OK;
  }
  if (every < 1 || every > 256) {
    set_err(ctx, "anchor interval must be in [1, 256] lane steps");
    return MU_E_ARG;
  }
  ctx->anchor_every = every;
  return MU_OK;
}

extern "C" int32_t mu_ctx_get_anchor(const mu_ctx *ctx) { return ctx ? ctx->anchor_every : -1; }

extern "C" mu_status mu_ctx_set_specialize(mu_ctx *ctx, int32_t on) {
  if (!ctx || (on != 0 && on != 1)) return MU_E_ARG;
  ctx->specialize = on;
  return MU_OK;
}

// -------------------------------------------------------------- histograms

static mu_status check_histos(const mu_histo *h, int32_t n, std::string &why, bool *all_int) {
  if (!h || n <= 0) {
    why = "need at least one histogram";
    return MU_E_ARG;
  }
  bool ints = true;
  for (int32_t j = 0; j < n; ++j) {
    const mu_histo &x = h[j];
    char b[256];
    if (!x.counts) {
      std::snprintf(b, sizeof b, "histogram %d: counts is NULL", j);
      why = b;
      return MU_E_ARG;
    }
    if (x.n_bins <= 0 || !(x.dt > 0.0) || !std::isfinite(x.dt) || !std::isfinite(x.t0_bin)) {
      std::snprintf(b, sizeof b, "histogram %d: need n_bins > 0, finite dt > 0 and finite t0_bin", j);
      why = b;
      return MU_E_ARG;
    }
    if (x.first < 0 || x.last < x.first || x.last >= x.n_bins) {
      std::snprintf(b, sizeof b, "histogram %d: fit range [%lld, %lld] outside [0, %lld)", j, (long long)x.first,
                    (long long)x.last, (long long)x.n_bins);
      why = b;
      return MU_E_ARG;
    }
    if (x.map_row < 0) {
      std::snprintf(b, sizeof b, "histogram %d: negative map row", j);
      why = b;
      return MU_E_ARG;
    }
    if (x.last - x.first + 1 > (int64_t)1 << 40) {
      std::snprintf(b, sizeof b, "histogram %d: fit range too long", j);
      why = b;
      return MU_E_UNSUPPORTED;
    }
    for (int64_t n2 = x.first; n2 <= x.last; ++n2) {
      const double d = x.counts[n2];
      if (!std::isfinite(d) || d < 0.0) {
        std::snprintf(b, sizeof b, "histogram %d: count %lld is negative or non-finite", j, (long long)n2);
        why = b;
        return MU_E_ARG;
      }
      if (ints && (d != std::floor(d) || d >= kCountIntLimit)) ints = false;
    }
  }
  if (all_int) *all_int = ints;
  return MU_OK;
}

extern "C" mu_status mu_histo_check(const mu_histo *h, int32_t n_histo, char *msg, int32_t msg_len) {
  std::string why;
  mu_status s = check_histos(h, n_histo, why, nullptr);
  put_msg(msg, msg_len, s == MU_OK ? std::string("ok") : why);
  return s;
}

// The gradient merge plan of (th, this dataset); layout next to kPlanHead.
mu_status mu_data::grad_plan(const mu_theory *th, const int32_t **out, int *lds) {
  for (const Plan &p : plans)
    if (p.theory_id == th->id) {
      *out = p.d;
      if (lds) *lds = p.lds;
      return MU_OK;
    }
  const DevTheory &T = th->h;
  std::vector<int> act;
  for (int r = 0; r < kRS; ++r)
    if (T.rref[r].kind == MU_REF_PAR || T.rref[r].kind == MU_REF_FUN) act.push_back(r);
  const int na = (int)act.size(), n_par = T.n_par;
  const int n_chunks = (n_histo + kMergeChunk - 1) / kMergeChunk;
  std::vector<std::vector<int32_t>> blocks(n_chunks);
  size_t stride = 0;
  for (int c = 0; c < n_chunks; ++c) {
    const int h0 = c * kMergeChunk, nh = std::min(kMergeChunk, n_histo - h0);
    // target of each entry e = q * na + i: parameter m, or function m
    std::vector<int32_t> koff(n_par + 1, 0), dest(nh * na), fi;
    std::vector<int> par(nh * na, -1);
    for (int q = 0; q < nh; ++q)
      for (int i = 0; i < na; ++i) {
        const DevRef &ref = T.rref[act[i]];
        const int m = th->map[(size_t)hh[h0 + q].map_row * T.n_slots + ref.slot];
        const int e = q * na + i;
        if (ref.kind == MU_REF_PAR) {
          par[e] = m;
          koff[m + 1]++;
        } else {
          dest[e] = -1 - (int32_t)fi.size();
          fi.push_back(m);
        }
      }
    for (int k = 0; k < n_par; ++k) koff[k + 1] += koff[k];
    std::vector<int32_t> fill(koff.begin(), koff.end() - 1);
    for (int e = 0; e < nh * na; ++e)
      if (par[e] >= 0) dest[e] = fill[par[e]]++;
    std::vector<int32_t> &b = blocks[c];
    b.push_back(koff[n_par]);
    b.push_back((int32_t)fi.size());
    b.insert(b.end(), koff.begin(), koff.end());
    b.insert(b.end(), dest.begin(), dest.end());
    b.insert(b.end(), fi.begin(), fi.end());
    stride = std::max(stride, b.size());
  }
  stride = (stride + 63) / 64 * 64;
  if (stride > (size_t)kPlanBlockMax) {  // cannot happen: nh * n_act + n_fe <= 2 kMergeChunk kRS
    set_err(ctx, "gradient merge plan block of %zu entries", stride);
    return MU_E_UNSUPPORTED;
  }
  std::vector<int32_t> buf(kPlanHead + (size_t)n_chunks * stride, 0);
  buf[0] = na;
  buf[1] = n_par;
  buf[2] = (int32_t)stride;
  for (int i = 0; i < na; ++i) buf[kPlanAct + i] = act[i];
  for (int c = 0; c < n_chunks; ++c) std::copy(blocks[c].begin(), blocks[c].end(), buf.begin() + kPlanHead + c * stride);
  // the merge's dynamic LDS: acc_s, acc_c [n_par], srt, fsrt [min(n_histo,
  // kMergeChunk) na] doubles, then the plan block [stride] ints
  const size_t merge_lds = 8 * (2 * (size_t)n_par + 2 * (size_t)std::min(n_histo, kMergeChunk) * na) + 4 * stride;
  Plan p{th->id, nullptr, (int)((merge_lds + 15) / 16 * 16)};
  hipError_t e = hipMalloc(&p.d, buf.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemcpy(p.d, buf.data(), buf.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (p.d) (void)hipFree(p.d);
    return hip_fail(ctx, e, "gradient merge plan");
  }
  plans.push_back(p);
  *out = p.d;
  if (lds) *lds = p.lds;
  return MU_OK;
}

void mu_data::free_dev() {
  for (Plan &p : plans)
    if (p.d) (void)hipFree(p.d);
  plans.clear();
  if (counts) (void)hipFree(counts);
  counts = nullptr;
  if (d_hh) (void)hipFree(d_hh);
  d_hh = nullptr;
}

// Key of the tuned table: theory shape (kShapeCount: a batched launch of
// compiled shapes), mode, cost, launch kind (batched or single-dataset) and
// the size of the launch to a power of two.
static int tune_key(int shape, int mode, int cost, int split, int64_t work) {
  int lg = 0;
  while (((int64_t)1 << (lg + 1)) <= work) ++lg;
  return (((shape * 4 + mode) * 2 + cost) * 2 + split) * 64 + lg;
}

// Smallest default range per wave: a wave's segment prologue and first
// anchor cost about as much as 64 lane steps of the loop, so mid-sized
// launches (the paper's Table 1 sizes: 1.4 M to 6.8 M bins) take ranges of
// work / 512 bins, up to 4096, rather than one range per wave slot; large
// launches are above the floor anyway, and small ones keep one bin per lane.
static int64_t default_split_floor(int64_t work) {
  return std::min<int64_t>(4096, std::max<int64_t>(kWave, work / 512));
}

int64_t mu_ctx::pick_split(int shape, int mode, int cost, int count_f64, int64_t work, int *anchor) const {
  *anchor = anchor_every;
  if (tile_bins > 0) return tile_bins;
  const int key = tune_key(shape, mode, cost, 1, work);
  for (const Tuned &t : tuned)
    if (t.key == key) {
      *anchor = t.anchor;
      return t.tile;
    }
  // one range per resident wave of the cost kernel (the same ranges for the
  // cost and the gradient pass, so their costs agree bit for bit), but not
  // below default_split_floor
  const int per_cu = eval_blocks_per_cu(kModeCost, cost, count_f64, shape);
  const int64_t cap = (int64_t)std::max(per_cu, 1) * (kBlock / kWave) * std::max(n_cu, 1);
  return std::max<int64_t>(default_split_floor(work), (work + cap - 1) / cap);
}

int64_t mu_ctx::pick_batch(int generic, int mode, int cost, int count_f64, int64_t work, int *anchor) const {
  *anchor = anchor_every;
  if (tile_bins > 0) return tile_bins;
  const int key = tune_key(generic ? kShapeGeneric : kShapeCount, mode, cost, 0, work);
  for (const Tuned &t : tuned)
    if (t.key == key) {
      *anchor = t.anchor;
      return t.tile;
    }
  // one range per resident wave of the launch's kernel, but not below
  // default_split_floor
  const int per_cu = eval_batch_blocks_per_cu(mode, cost, count_f64, generic);
  const int64_t cap = (int64_t)std::max(per_cu, 1) * (kBlock / kWave) * std::max(n_cu, 1);
  return std::max<int64_t>(default_split_floor(work), (work + cap - 1) / cap);
}

extern "C" mu_status mu_data_create(mu_ctx *ctx, const mu_histo *h, int32_t n_histo, mu_data **out) {
  if (!ctx || !out) return MU_E_ARG;
  *out = nullptr;
  std::string why;
  bool ints = false;
  mu_status st = check_histos(h, n_histo, why, &ints);
  if (st != MU_OK) {
    set_err(ctx, "%s", why.c_str());
    return st;
  }
  (void)hipSetDevice(ctx->device);
  mu_data *d = new mu_data();
  d->ctx = ctx;
  d->n_histo = n_histo;
  d->f64 = ints ? 0 : 1;
  int64_t total = 0;
  d->hh.resize(n_histo);
  for (int j = 0; j < n_histo; ++j) {
    DevHisto &x = d->hh[j];
    x.off = total;
    x.n = h[j].last - h[j].first + 1;
    x.first = h[j].first;
    x.t0_bin = h[j].t0_bin;
    x.dt = h[j].dt;
    x.map_row = h[j].map_row;
    x.pad = 0;
    d->max_row = std::max(d->max_row, (int)h[j].map_row);
    d->longest = std::max(d->longest, x.n);
    total += x.n;
  }
  d->total = total;
  const size_t esz = d->f64 ? sizeof(double) : sizeof(uint32_t);
  // kPrefetch x kBlock values (16 lane steps of 64 values) of zero padding:
  // kernels read each lane's counts up to kPrefetchStream (<= 16) lane steps
  // ahead, and reads past the last bin land here
  static_assert(kPrefetchStream * kWave <= kPrefetch * kBlock, "padding covers the deepest count prefetch");
  const size_t padded = ((size_t)total + (size_t)kPrefetch * kBlock) * esz;
  hipError_t e = hipMalloc(&d->counts, padded);
  if (e != hipSuccess) {
    delete d;
    set_err(ctx, "device allocation for %lld bins failed", (long long)total);
    return MU_E_NOMEM;
  }
  // pack on the host, upload once
  {
    std::vector<char> buf(padded, 0);
    for (int j = 0; j < n_histo; ++j) {
      const DevHisto &x = d->hh[j];
      for (int64_t i = 0; i < x.n; ++i) {
        const double v = h[j].counts[x.first + i];
        d->max_count = std::max(d->max_count, v);
        if (d->f64)
          reinterpret_cast<double *>(buf.data())[x.off + i] = v;
        else
          reinterpret_cast<uint32_t *>(buf.data())[x.off + i] = (uint32_t)v * kCountScale;
      }
    }
    e = hipMemcpy(d->counts, buf.data(), buf.size(), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMalloc(&d->d_hh, d->hh.size() * sizeof(DevHisto));
  if (e == hipSuccess) e = hipMemcpy(d->d_hh, d->hh.data(), d->hh.size() * sizeof(DevHisto), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    d->free_dev();
    delete d;
    return hip_fail(ctx, e, "hipMemcpy(counts)");
  }
  ctx->children++;
  *out = d;
  return MU_OK;
}

extern "C" mu_status mu_data_destroy(mu_data *d) {
  if (!d) return MU_E_ARG;
  (void)hipSetDevice(d->ctx->device);
  (void)hipStreamSynchronize(d->ctx->stream);
  d->free_dev();
  d->ctx->children--;
  delete d;
  return MU_OK;
}

extern "C" int64_t mu_data_bins(const mu_data *d) { return d ? d->total : -1; }
extern "C" int32_t mu_data_histos(const mu_data *d) { return d ? d->n_histo : -1; }
extern "C" int32_t mu_data_is_f64(const mu_data *d) { return d ? d->f64 : -1; }

// ------------------------------------------------------------------ theory

static int prim_nargs(int p) {
  switch (p) {
    case MU_SE: return 1;
    case MU_GE: return 2;
    case MU_SG: return 1;
    case MU_STG: return 1;
    case MU_TF: return 2;
  }
  return -1;
}

static mu_status check_ref(const mu_theory_desc *d, const mu_ref &r, const char *what, std::string &why) {
  char b[256];
  if (r.kind == MU_REF_LIT) {
    if (!std::isfinite(r.literal)) {
      std::snprintf(b, sizeof b, "%s: literal is not finite", what);
      why = b;
      return MU_E_ARG;
    }
    return MU_OK;
  }
  if (r.kind != MU_REF_PAR && r.kind != MU_REF_FUN) {
    std::snprintf(b, sizeof b, "%s: unknown reference kind %d", what, r.kind);
    why = b;
    return MU_E_ARG;
  }
  if (r.slot < 0 || r.slot >= d->n_slots) {
    std::snprintf(b, sizeof b, "%s: slot %d outside [0, %d)", what, r.slot, d->n_slots);
    why = b;
    return MU_E_ARG;
  }
  const int lim = r.kind == MU_REF_PAR ? d->n_par : d->n_fun;
  for (int row = 0; row < d->n_rows; ++row) {
    const int v = d->map[row * d->n_slots + r.slot];
    if (v < 0 || v >= lim) {
      std::snprintf(b, sizeof b, "%s: map[%d][%d] = %d outside [0, %d) for a %s reference", what, row, r.slot, v, lim,
                    r.kind == MU_REF_PAR ? "parameter" : "function");
      why = b;
      return MU_E_ARG;
    }
  }
  return MU_OK;
}

static mu_status check_theory(const mu_theory_desc *d, std::string &why) {
  if (!d) {
    why = "null theory";
    return MU_E_ARG;
  }
  if (d->n_par < 1 || d->n_par > MU_MAX_PAR) {
    why = "n_par outside [1, MU_MAX_PAR]";
    return MU_E_ARG;
  }
  if (!(d->tau_mu > 0.0) || !std::isfinite(d->tau_mu)) {
    why = "tau_mu must be finite and > 0";
    return MU_E_ARG;
  }
  if (d->n_rows < 1 || d->n_slots < 1 || !d->map) {
    why = "the map needs at least one row and one slot";
    return MU_E_ARG;
  }
  if (d->n_fun < 0 || (d->n_fun > 0 && (!d->F || !d->f0))) {
    why = "n_fun > 0 needs F and f0";
    return MU_E_ARG;
  }
  if (d->n_fun > 0) {
    for (int64_t i = 0; i < (int64_t)d->n_fun * d->n_par; ++i)
      if (!std::isfinite(d->F[i])) {
        why = "F holds a non-finite value";
        return MU_E_ARG;
      }
    for (int i = 0; i < d->n_fun; ++i)
      if (!std::isfinite(d->f0[i])) {
        why = "f0 holds a non-finite value";
        return MU_E_ARG;
      }
  }
  if (d->n_terms < 0 || (d->n_terms > 0 && !d->terms)) {
    why = "bad term array";
    return MU_E_ARG;
  }
  if (d->n_terms > MU_MAX_TERMS) {
    why = "more than MU_MAX_TERMS terms";
    return MU_E_UNSUPPORTED;
  }
  if (d->n_factors < 0 || (d->n_factors > 0 && !d->factors)) {
    why = "bad factor array";
    return MU_E_ARG;
  }
  mu_status s;
  if ((s = check_ref(d, d->n0, "N0", why)) != MU_OK) return s;
  if ((s = check_ref(d, d->nbkg, "Nbkg", why)) != MU_OK) return s;
  std::vector<int> used(d->n_factors, 0);
  for (int k = 0; k < d->n_terms; ++k) {
    const mu_term &t = d->terms[k];
    char what[64];
    std::snprintf(what, sizeof what, "term %d amplitude", k);
    if (!std::isfinite(t.coef)) {
      why = "term coefficient is not finite";
      return MU_E_ARG;
    }
    if ((s = check_ref(d, t.amp, what, why)) != MU_OK) return s;
    if (t.n_factors < 0 || t.first_factor < 0 || t.first_factor + t.n_factors > d->n_factors) {
      why = "term factor range leaves the factor array";
      return MU_E_ARG;
    }
    if (t.n_factors > MU_MAX_FACTORS_PER_TERM) {
      why = "more than MU_MAX_FACTORS_PER_TERM factors in a term";
      return MU_E_UNSUPPORTED;
    }
    for (int i = 0; i < t.n_factors; ++i) {
      const int fi = t.first_factor + i;
      if (used[fi]++) {
        why = "factor ranges of two terms overlap";
        return MU_E_ARG;
      }
      const mu_factor &f = d->factors[fi];
      const int na = prim_nargs(f.prim);
      if (na < 0) {
        char b[64];
        std::snprintf(b, sizeof b, "factor %d: unknown primitive %d", fi, f.prim);
        why = b;
        return MU_E_ARG;
      }
      for (int a = 0; a < na; ++a) {
        std::snprintf(what, sizeof what, "factor %d argument %d", fi, a);
        if ((s = check_ref(d, f.arg[a], what, why)) != MU_OK) return s;
      }
      if (f.prim == MU_GE && f.arg[1].kind == MU_REF_LIT && !(f.arg[1].literal > 0.0)) {
        why = "a literal beta of ge must be > 0";
        return MU_E_ARG;
      }
    }
  }
  return MU_OK;
}

// The compiled specialisation that matches a theory program, if any.
static int detect_shape(const DevTheory &h) {
  if (h.n_terms == 1 && h.nf[0] == 2 && h.prim[0][0] == MU_SE && h.prim[0][1] == MU_TF) return kShapeExpCos;
  if (h.n_terms == 1 && h.nf[0] == 2 && h.prim[0][0] == MU_SG && h.prim[0][1] == MU_TF) return kShapeGaussCos;
  if (h.n_terms == 1 && h.nf[0] == 1 && h.prim[0][0] == MU_STG) return kShapeStg;
  if (h.n_terms == 2 && h.nf[0] == 1 && h.prim[0][0] == MU_SE && h.nf[1] == 1 && h.prim[1][0] == MU_STG)
    return kShapeExpStg;
  if (h.n_terms == 2 && h.nf[0] == 2 && h.prim[0][0] == MU_SE && h.prim[0][1] == MU_TF && h.nf[1] == 1 &&
      h.prim[1][0] == MU_STG)
    return kShapeExpCosStg;
  return kShapeGeneric;
}

extern "C" mu_status mu_theory_check(const mu_theory_desc *d, char *msg, int32_t msg_len) {
  std::string why;
  mu_status s = check_theory(d, why);
  put_msg(msg, msg_len, s == MU_OK ? std::string("ok") : why);
  return s;
}

extern "C" mu_status mu_theory_create(mu_ctx *ctx, const mu_theory_desc *d, mu_theory **out) {
  if (!ctx || !out) return MU_E_ARG;
  *out = nullptr;
  std::string why;
  mu_status s = check_theory(d, why);
  if (s != MU_OK) {
    set_err(ctx, "%s", why.c_str());
    return s;
  }
  (void)hipSetDevice(ctx->device);
  static std::atomic<uint64_t> next_id{1};
  mu_theory *th = new mu_theory();
  th->ctx = ctx;
  th->id = next_id++;
  DevTheory &h = th->h;
  std::memset(&h, 0, sizeof h);
  h.tau_mu = d->tau_mu;
  h.neg_inv_tau = -1.0 / d->tau_mu;
  h.n_terms = d->n_terms;
  h.n_par = d->n_par;
  h.n_fun = d->n_fun;
  h.n_rows = d->n_rows;
  h.n_slots = d->n_slots;
  for (int r = 0; r < kRS; ++r) h.rref[r].kind = kRefNone;
  auto put = [&](int r, const mu_ref &x) {
    h.rref[r].kind = x.kind;
    h.rref[r].slot = x.slot;
    h.rref[r].lit = x.literal;
  };
  put(0, d->n0);
  put(1, d->nbkg);
  for (int k = 0; k < d->n_terms; ++k) {
    const mu_term &t = d->terms[k];
    h.coef[k] = t.coef;
    h.nf[k] = t.n_factors;
    put(2 + k, t.amp);
    for (int i = 0; i < t.n_factors; ++i) {
      const mu_factor &f = d->factors[t.first_factor + i];
      h.prim[k][i] = f.prim;
      const int na = prim_nargs(f.prim);
      for (int a = 0; a < na; ++a) put(arg_index(k, i, a), f.arg[a]);
      // an unused second argument resolves to the literal 0
      if (na < 2) {
        h.rref[arg_index(k, i, 1)].kind = MU_REF_LIT;
        h.rref[arg_index(k, i, 1)].lit = 0.0;
      }
    }
  }
  th->shape = detect_shape(h);
  th->map.assign(d->map, d->map + (size_t)d->n_rows * d->n_slots);
  if (d->n_fun > 0) {
    th->F.assign(d->F, d->F + (size_t)d->n_fun * d->n_par);
    th->f0.assign(d->f0, d->f0 + d->n_fun);
  }
  hipError_t e = hipSuccess;
  auto up = [&](void **dst, const void *src, size_t n) {
    if (e != hipSuccess || n == 0) return;
    e = hipMalloc(dst, n);
    if (e == hipSuccess) e = hipMemcpy(*dst, src, n, hipMemcpyHostToDevice);
  };
  up((void **)&th->d_map, th->map.data(), th->map.size() * sizeof(int32_t));
  up((void **)&th->d_F, th->F.data(), th->F.size() * sizeof(double));
  up((void **)&th->d_f0, th->f0.data(), th->f0.size() * sizeof(double));
  h.map = th->d_map;
  h.F = th->d_F;
  h.f0 = th->d_f0;
  up((void **)&th->d_th, &h, sizeof h);
  if (e != hipSuccess) {
    th->free_dev();
    delete th;
    return hip_fail(ctx, e, "theory upload");
  }
  ctx->children++;
  *out = th;
  return MU_OK;
}

void mu_theory::free_dev() {
  if (d_map) (void)hipFree(d_map);
  if (d_F) (void)hipFree(d_F);
  if (d_f0) (void)hipFree(d_f0);
  if (d_th) (void)hipFree(d_th);
  d_map = nullptr;
  d_F = d_f0 = nullptr;
  d_th = nullptr;
}

extern "C" mu_status mu_theory_destroy(mu_theory *th) {
  if (!th) return MU_E_ARG;
  (void)hipSetDevice(th->ctx->device);
  (void)hipStreamSynchronize(th->ctx->stream);
  th->free_dev();
  th->ctx->children--;
  delete th;
  return MU_OK;
}

extern "C" int32_t mu_theory_npar(const mu_theory *th) { return th ? th->h.n_par : -1; }

// -------------------------------------------------------------- evaluation

namespace mu {

// Common argument checks for one (data, theory) pair.
mu_status check_pair(mu_ctx *ctx, const mu_data *d, const mu_theory *th) {
  if (!d || !th) {
    set_err(ctx, "null data or theory handle");
    return MU_E_ARG;
  }
  if (d->ctx != ctx || th->ctx != ctx) {
    set_err(ctx, "data and theory must belong to this context");
    return MU_E_ARG;
  }
  if (d->max_row >= th->h.n_rows) {
    set_err(ctx, "a histogram names map row %d but the theory has %d rows", d->max_row, th->h.n_rows);
    return MU_E_ARG;
  }
  return MU_OK;
}

}  // namespace mu

namespace mu {

// Evaluate n_vec vectors over one dataset in one launch.  mode: cost, grad, model.
static mu_status check_eval_args(mu_ctx *ctx, int cost_kind, unsigned mem, int32_t n_vec, const void *params) {
  if (mem != MU_MEM_HOST && mem != MU_MEM_DEVICE) {
    set_err(ctx, "mem must be MU_MEM_HOST or MU_MEM_DEVICE");
    return MU_E_ARG;
  }
  if (cost_kind != MU_COST_CHI2 && cost_kind != MU_COST_POISSON) {
    set_err(ctx, "unknown cost kind %d", cost_kind);
    return MU_E_ARG;
  }
  if (n_vec < 1 || !params) {
    set_err(ctx, "need n_vec >= 1 and a parameter array");
    return MU_E_ARG;
  }
  return MU_OK;
}

// A launched evaluation whose merge is still to be enqueued.
struct Pending {
  LaunchArgs a;
  int mode = 0, n_vec = 0, shape = 0, f64 = 0;
  int merge_lds = 0;  // dynamic LDS bytes of the merge (gradient mode)
  hipFunction_t rtc = nullptr;  // run-time compiled theory's kernel
};

// The evaluation launch of a prepared uniform launch: the theory's compiled
// shape or interpreted kernel, or its run-time compiled kernel.
static hipError_t launch_pending(const Pending &p, int mode, hipStream_t s) {
  if (p.rtc) return launch_rtc(p.rtc, p.a, mode, p.f64, s);
  return launch_eval(p.a, mode, p.f64, p.shape, s);
}

// Prepares (and, unless launch is false, enqueues) one evaluation launch;
// w_force > 0 replaces the chosen bins per wave.
static mu_status eval_launch(mu_ctx *ctx, mu_data *d, const mu_theory *th, int cost_kind, const double *dp,
                             int32_t n_vec, double *dc, double *dh, double *dg, double *dm, int mode, hipStream_t s,
                             DevBuf &partial, Pending &pend, bool launch = true, int64_t w_force = 0,
                             bool no_alloc = false) {
  mu_status st;
  const int shape = ctx->specialize ? th->shape : kShapeGeneric;
  int anchor = ctx->anchor_every;
  const int64_t work = (int64_t)n_vec * d->total;
  int64_t W = ctx->pick_split(shape, mode, cost_kind, d->f64, work, &anchor);
  if (w_force > 0) W = w_force;
  if (mode == kModeGrad) W = std::min<int64_t>(W, kMaxGradSplit);
  const int n_par = th->h.n_par;
  const int64_t n_units = (work + W - 1) / W;
  if (n_units + (int64_t)n_vec * d->n_histo > INT32_MAX) {
    set_err(ctx, "launch needs more than 2^31 work units");
    return MU_E_UNSUPPORTED;
  }
  if (mode != kModeModel) {
    // slot u + v * n_histo + h for every segment (see the split launch)
    const size_t n_slots = (size_t)n_units + (size_t)n_vec * d->n_histo;
    if ((st = partial.ensure(ctx, n_slots * kSlot * sizeof(double), false)) != MU_OK) return st;
  }
  const int32_t *plan = nullptr;
  int merge_lds = 0;
  if (mode == kModeGrad && (st = d->grad_plan(th, &plan, &merge_lds)) != MU_OK) return st;
  LaunchArgs a;
  std::memset(&a, 0, sizeof a);
  a.tmpl.th = th->d_th;
  a.tmpl.plan = plan;
  a.tmpl.histos = d->d_hh;
  a.tmpl.counts = d->counts;
  a.tmpl.p = dp;
  a.tmpl.cost_out = dc;
  a.tmpl.histo_out = dh;
  a.tmpl.grad_out = dg;
  a.tmpl.model_out = dm;
  a.tmpl.n_histo = d->n_histo;
  a.tmpl.shape = shape;
  a.p_stride = n_par;
  a.grad_stride = n_par;
  a.histo_stride = d->n_histo;
  a.jobs = nullptr;
  a.job_list = nullptr;
  a.unit_start = nullptr;
  a.n_units = (int32_t)n_units;
  a.cost_kind = cost_kind;
  a.anchor_every = anchor;
  a.counts_in_table = !d->f64 && d->max_count < kInvTab;
  a.inv_src = ctx->d_inv;
  a.n_vec = n_vec;
  a.split_w = W;
  a.total = d->total;
  a.partial = static_cast<double *>(partial.ptr);
  pend.a = a;
  pend.mode = mode;
  pend.n_vec = n_vec;
  pend.shape = shape;
  pend.f64 = d->f64;
  pend.rtc = th->rtc_fn;
  pend.merge_lds = merge_lds;
  if (!launch) return MU_OK;
  if (no_alloc) {  // no timing events (they are created on demand)
    hipError_t e = launch_pending(pend, mode, s);
    return e == hipSuccess ? MU_OK : hip_fail(ctx, e, "evaluation launch");
  }
  int ti = ctx->time_begin(mode == kModeGrad    ? MU_TIME_EVAL_GRAD
                           : mode == kModeModel ? MU_TIME_EVAL_MODEL
                                                : MU_TIME_EVAL_COST,
                           s);
  hipError_t e = launch_pending(pend, mode, s);
  ctx->time_end(ti, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "evaluation launch");
  return MU_OK;
}

static mu_status eval_merge(mu_ctx *ctx, const Pending &pend, hipStream_t s) {
  if (pend.mode == kModeModel) return MU_OK;
  const int ti = ctx->time_begin(MU_TIME_MERGE, s);
  const bool narrow = pend.n_vec >= kNarrowJobs && pend.a.tmpl.n_histo <= kNarrowHisto;
  hipError_t e = launch_merge(pend.a, pend.mode, pend.n_vec, pend.merge_lds, narrow, s);
  ctx->time_end(ti, s);
  return e == hipSuccess ? MU_OK : hip_fail(ctx, e, "merge launch");
}

mu_status eval_dev(mu_ctx *ctx, mu_data *d, const mu_theory *th, int cost_kind, const double *dp, int32_t n_vec,
                   double *dc, double *dh, double *dg, double *dm, int mode, hipStream_t s, DevBuf &partial) {
  Pending pend;
  mu_status st = eval_launch(ctx, d, th, cost_kind, dp, n_vec, dc, dh, dg, dm, mode, s, partial, pend);
  return st == MU_OK ? eval_merge(ctx, pend, s) : st;
}

mu_status eval_uniform(mu_ctx *ctx, mu_data *d, const mu_theory *th, int cost_kind, const double *params,
                       int32_t n_vec, unsigned mem, double *cost, double *histo, double *grad, double *model,
                       int mode) {
  mu_status st = check_eval_args(ctx, cost_kind, mem, n_vec, params);
  if (st != MU_OK) return st;
  (void)hipSetDevice(ctx->device);
  const int n_par = th->h.n_par;
  const size_t n_p = (size_t)n_vec * n_par;
  const size_t n_h = histo ? (size_t)n_vec * d->n_histo : 0;
  const size_t n_g = grad ? (size_t)n_vec * n_par : 0;
  const size_t n_c = mode == kModeModel ? 0 : (size_t)n_vec;
  const size_t n_m = mode == kModeModel ? (size_t)d->total : 0;
  const double *dp = params;
  double *dc = cost, *dh = histo, *dg = grad, *dm = model;
  hipError_t e;
  if (mem == MU_MEM_HOST) {
    if ((st = ctx->dparams.ensure(ctx, n_p * sizeof(double), false)) != MU_OK) return st;
    if ((st = ctx->dout.ensure(ctx, (n_c + n_h + n_g + n_m) * sizeof(double), false)) != MU_OK) return st;
    if ((st = ctx->staging.ensure(ctx, n_p * sizeof(double))) != MU_OK) return st;
    if ((st = ctx->staging_out.ensure(ctx, (n_c + n_h + n_g + n_m) * sizeof(double))) != MU_OK) return st;
    ctx->wait_staging();
    std::memcpy(ctx->staging.ptr, params, n_p * sizeof(double));
    e = hipMemcpyAsync(ctx->dparams.ptr, ctx->staging.ptr, n_p * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(params)");
    ctx->mark_staging();
    dp = static_cast<double *>(ctx->dparams.ptr);
    double *o = static_cast<double *>(ctx->dout.ptr);
    dc = n_c ? o : nullptr;
    dh = n_h ? o + n_c : nullptr;
    dg = n_g ? o + n_c + n_h : nullptr;
    dm = n_m ? o + n_c + n_h + n_g : nullptr;
  }
  if ((st = eval_dev(ctx, d, th, cost_kind, dp, n_vec, dc, dh, dg, dm, mode, ctx->stream, ctx->partial)) != MU_OK)
    return st;
  if (mem == MU_MEM_HOST) {
    const size_t n_out = n_c + n_h + n_g + n_m;
    e = hipMemcpyAsync(ctx->staging_out.ptr, ctx->dout.ptr, n_out * sizeof(double), hipMemcpyDeviceToHost,
                       ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(results)");
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    const double *o = static_cast<const double *>(ctx->staging_out.ptr);
    if (n_c) std::memcpy(cost, o, n_c * sizeof(double));
    if (n_h) std::memcpy(histo, o + n_c, n_h * sizeof(double));
    if (n_g) std::memcpy(grad, o + n_c + n_h, n_g * sizeof(double));
    if (n_m) std::memcpy(model, o + n_c + n_h + n_g, n_m * sizeof(double));
  }
  return MU_OK;
}

// Gradient pass and cost pass over one dataset with one merge launch.
mu_status eval_grad_and_costs(mu_ctx *ctx, mu_data *d, const mu_theory *th, int cost_kind, const double *pg,
                              int32_t n_grad, const double *pc, int32_t n_cost, unsigned mem, double *cost_g,
                              double *grad, double *cost_c) {
  mu_status st = check_eval_args(ctx, cost_kind, mem, n_grad, pg);
  if (st == MU_OK) st = check_eval_args(ctx, cost_kind, mem, n_cost, pc);
  if (st != MU_OK) return st;
  (void)hipSetDevice(ctx->device);
  const int n_par = th->h.n_par;
  const size_t n_pg = (size_t)n_grad * n_par, n_pc = (size_t)n_cost * n_par;
  const size_t n_out = (size_t)n_grad + (size_t)n_grad * n_par + (size_t)n_cost;
  const double *dpg = pg, *dpc = pc;
  double *dcg = cost_g, *dg = grad, *dcc = cost_c;
  hipError_t e;
  if (mem == MU_MEM_HOST) {
    if ((st = ctx->dparams.ensure(ctx, (n_pg + n_pc) * sizeof(double), false)) != MU_OK) return st;
    if ((st = ctx->dout.ensure(ctx, n_out * sizeof(double), false)) != MU_OK) return st;
    if ((st = ctx->staging.ensure(ctx, (n_pg + n_pc) * sizeof(double))) != MU_OK) return st;
    if ((st = ctx->staging_out.ensure(ctx, n_out * sizeof(double))) != MU_OK) return st;
    ctx->wait_staging();
    std::memcpy(ctx->staging.ptr, pg, n_pg * sizeof(double));
    std::memcpy(static_cast<double *>(ctx->staging.ptr) + n_pg, pc, n_pc * sizeof(double));
    e = hipMemcpyAsync(ctx->dparams.ptr, ctx->staging.ptr, (n_pg + n_pc) * sizeof(double), hipMemcpyHostToDevice,
                       ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(params)");
    ctx->mark_staging();
    dpg = static_cast<double *>(ctx->dparams.ptr);
    dpc = dpg + n_pg;
    dcg = static_cast<double *>(ctx->dout.ptr);
    dg = dcg + n_grad;
    dcc = dg + n_pg;
  }
  // both passes on the context's stream (their own slot buffers) as one
  // launch where a compiled kernel exists (else two), then one merge launch
  // for both: the gradient job's merge latency hides behind the cost jobs'
  // merges
  Pending pg_, pc_;
  if ((st = eval_launch(ctx, d, th, cost_kind, dpc, n_cost, dcc, nullptr, nullptr, nullptr, kModeCost, ctx->stream,
                        ctx->partial, pc_, false)) != MU_OK)
    return st;
  // In one launch the gradient waves run beside the cost waves, so longer
  // gradient ranges cost no time there and leave fewer slots to merge: at
  // least half a cost range, but at least 64 gradient waves (C2: 8192 bins
  // per wave in place of the 1024-2048 a gradient launch of its own prefers).
  const int shape = ctx->specialize ? th->shape : kShapeGeneric;
  const bool fused = !th->rtc_fn && eval_grad_cost_fused(d->f64, shape, cost_kind);
  int64_t wg = 0;
  if (fused && ctx->tile_bins == 0) {
    int anchor_g = 0;
    const int64_t work_g = (int64_t)n_grad * d->total;
    const int64_t wg_own = ctx->pick_split(shape, kModeGrad, cost_kind, d->f64, work_g, &anchor_g);
    wg = std::max<int64_t>(wg_own, std::min<int64_t>(pc_.a.split_w / 2, (work_g + 63) / 64));
  }
  if ((st = eval_launch(ctx, d, th, cost_kind, dpg, n_grad, dcg, nullptr, dg, nullptr, kModeGrad, ctx->stream,
                        ctx->partial_aux, pg_, false, wg)) != MU_OK)
    return st;
  if (fused) {
    const int ti = ctx->time_begin(MU_TIME_EVAL_GRAD_COST, ctx->stream);
    e = launch_eval_grad_cost(pg_.a, pc_.a, pg_.f64, pg_.shape, ctx->stream);
    ctx->time_end(ti, ctx->stream);
  } else {
    int ti = ctx->time_begin(MU_TIME_EVAL_GRAD, ctx->stream);
    e = launch_pending(pg_, kModeGrad, ctx->stream);
    ctx->time_end(ti, ctx->stream);
    if (e == hipSuccess) {
      ti = ctx->time_begin(MU_TIME_EVAL_COST, ctx->stream);
      e = launch_pending(pc_, kModeCost, ctx->stream);
      ctx->time_end(ti, ctx->stream);
    }
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "evaluation launch");
  const int ti = ctx->time_begin(MU_TIME_MERGE, ctx->stream);
  e = launch_merge_grad_cost(pg_.a, n_grad, pc_.a, n_cost, pg_.merge_lds, ctx->stream);
  ctx->time_end(ti, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "merge launch");
  if (mem == MU_MEM_HOST) {
    e = hipMemcpyAsync(ctx->staging_out.ptr, ctx->dout.ptr, n_out * sizeof(double), hipMemcpyDeviceToHost,
                       ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(results)");
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    const double *o = static_cast<const double *>(ctx->staging_out.ptr);
    std::memcpy(cost_g, o, n_grad * sizeof(double));
    std::memcpy(grad, o + n_grad, n_pg * sizeof(double));
    std::memcpy(cost_c, o + n_grad + n_pg, n_cost * sizeof(double));
  }
  return MU_OK;
}

}  // namespace mu

extern "C" mu_status mu_chi2_eval(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                                  const double *params, int32_t n_vec, unsigned mem, double *cost,
                                  double *cost_per_histo) {
  if (!ctx) return MU_E_ARG;
  mu_status st = check_pair(ctx, data, th);
  if (st != MU_OK) return st;
  if (!cost) {
    set_err(ctx, "cost output is NULL");
    return MU_E_ARG;
  }
  return eval_uniform(ctx, const_cast<mu_data *>(data), th, cost_kind, params, n_vec, mem, cost, cost_per_histo,
                      nullptr, nullptr, kModeCost);
}

extern "C" mu_status mu_chi2_eval_static(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                                         const double *params, int32_t n_vec, double *cost, double *cost_per_histo) {
  if (!ctx) return MU_E_ARG;
  mu_status st = check_pair(ctx, data, th);
  if (st != MU_OK) return st;
  if (!cost) {
    set_err(ctx, "cost output is NULL");
    return MU_E_ARG;
  }
  if ((st = check_eval_args(ctx, cost_kind, MU_MEM_DEVICE, n_vec, params)) != MU_OK) return st;
  if (!ctx->scratch) {
    set_err(ctx, "the allocation-free slots of device %d were not found (hipGetSymbolAddress failed)", ctx->device);
    return MU_E_DEVICE;
  }
  (void)hipSetDevice(ctx->device);
  // the same launch as mu_chi2_eval with device memory, its slots in the
  // device's static array (a fixed buffer: a launch needing more slots is
  // refused before anything is enqueued)
  DevBuf slots;
  slots.ptr = ctx->scratch;
  slots.cap = (size_t)kStaticSlots * kSlot * sizeof(double);
  slots.fixed = true;
  Pending pend;
  st = eval_launch(ctx, const_cast<mu_data *>(data), th, cost_kind, params, n_vec, cost, cost_per_histo, nullptr,
                   nullptr, kModeCost, ctx->stream, slots, pend, true, 0, true);
  if (st != MU_OK) return st;
  const bool narrow = pend.n_vec >= kNarrowJobs && pend.a.tmpl.n_histo <= kNarrowHisto;
  hipError_t e = launch_merge(pend.a, pend.mode, pend.n_vec, pend.merge_lds, narrow, ctx->stream);
  return e == hipSuccess ? MU_OK : hip_fail(ctx, e, "merge launch");
}

extern "C" mu_status mu_chi2_grad(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                                  const double *params, int32_t n_vec, unsigned mem, double *cost, double *grad) {
  if (!ctx) return MU_E_ARG;
  mu_status st = check_pair(ctx, data, th);
  if (st != MU_OK) return st;
  if (!cost || !grad) {
    set_err(ctx, "cost and grad outputs must not be NULL");
    return MU_E_ARG;
  }
  return eval_uniform(ctx, const_cast<mu_data *>(data), th, cost_kind, params, n_vec, mem, cost, nullptr, grad,
                      nullptr, kModeGrad);
}

extern "C" mu_status mu_chi2_eval_grad(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                                       const double *params_grad, int32_t n_grad, const double *params_cost,
                                       int32_t n_cost, unsigned mem, double *cost_grad, double *grad,
                                       double *cost) {
  if (!ctx) return MU_E_ARG;
  mu_status st = check_pair(ctx, data, th);
  if (st != MU_OK) return st;
  if (!cost_grad || !grad || !cost) {
    set_err(ctx, "cost_grad, grad and cost outputs must not be NULL");
    return MU_E_ARG;
  }
  return eval_grad_and_costs(ctx, const_cast<mu_data *>(data), th, cost_kind, params_grad, n_grad, params_cost,
                             n_cost, mem, cost_grad, grad, cost);
}

extern "C" mu_status mu_model_eval(mu_ctx *ctx, const mu_data *data, const mu_theory *th, const double *params,
                                   unsigned mem, double *out) {
  if (!ctx) return MU_E_ARG;
  mu_status st = check_pair(ctx, data, th);
  if (st != MU_OK) return st;
  if (!out) {
    set_err(ctx, "output is NULL");
    return MU_E_ARG;
  }
  return eval_uniform(ctx, const_cast<mu_data *>(data), th, MU_COST_CHI2, params, 1, mem, nullptr, nullptr, nullptr,
                      out, kModeModel);
}

extern "C" mu_status mu_chi2_batch(mu_ctx *ctx, int32_t n_jobs, const mu_data *const *data,
                                   const mu_theory *const *th, mu_cost cost_kind, int32_t ld, const double *params,
                                   unsigned mem, double *cost, double *grad) {
  if (!ctx) return MU_E_ARG;
  if (n_jobs < 1 || !data || !th || !params || !cost || ld < 1) {
    set_err(ctx, "need n_jobs >= 1, ld >= 1 and non-NULL data, theory, params and cost");
    return MU_E_ARG;
  }
  if (mem != MU_MEM_HOST && mem != MU_MEM_DEVICE) {
    set_err(ctx, "mem must be MU_MEM_HOST or MU_MEM_DEVICE");
    return MU_E_ARG;
  }
  if (cost_kind != MU_COST_CHI2 && cost_kind != MU_COST_POISSON) {
    set_err(ctx, "unknown cost kind %d", cost_kind);
    return MU_E_ARG;
  }
  mu_status st;
  int f64 = -1;
  for (int j = 0; j < n_jobs; ++j) {
    if ((st = check_pair(ctx, data[j], th[j])) != MU_OK) return st;
    if (th[j]->h.n_par > ld) {
      set_err(ctx, "job %d: theory has %d parameters but ld is %d", j, th[j]->h.n_par, ld);
      return MU_E_ARG;
    }
    if (f64 < 0) f64 = data[j]->f64;
    if (data[j]->f64 != f64) {
      set_err(ctx, "one batch cannot mix FP32-packed and FP64 datasets");
      return MU_E_UNSUPPORTED;
    }
  }
  (void)hipSetDevice(ctx->device);
  return run_batch(ctx, n_jobs, data, th, cost_kind, ld, params, mem, cost, grad);
}

namespace mu {

mu_status run_batch(mu_ctx *ctx, int32_t n_jobs, const mu_data *const *data, const mu_theory *const *th,
                    int cost_kind, int32_t ld, const double *params, unsigned mem, double *cost, double *grad) {
  mu_status st;
  hipError_t e;
  const int mode = grad ? kModeGrad : kModeCost;
  const int f64 = data[0]->f64;
  // launch 0: jobs of compiled shapes (each segment runs its job's shape);
  // launch 1: the interpreted theory programs (or FP64 counts); then one
  // launch per run-time compiled theory kernel
  std::vector<int32_t> list;
  list.reserve(n_jobs);
  struct Group {
    int32_t first = 0, n = 0;  // in `list`
    int64_t total = 0, W = 0, n_units = 0;
    int32_t n_histo = 0, slot_base = 0, anchor = 0, in_table = 1;
    hipFunction_t rtc = nullptr;
  };
  std::vector<Group> grp(2);
  for (int j = 0; j < n_jobs; ++j)
    if (th[j]->rtc_fn) {
      bool seen = false;
      for (size_t g = 2; g < grp.size(); ++g) seen = seen || grp[g].rtc == th[j]->rtc_fn;
      if (!seen) {
        grp.emplace_back();
        grp.back().rtc = th[j]->rtc_fn;
      }
    }
  const int n_groups = (int)grp.size();
  for (int g = 0; g < n_groups; ++g) {
    Group &G = grp[g];
    G.first = (int32_t)list.size();
    for (int j = 0; j < n_jobs; ++j) {
      int jg;
      if (th[j]->rtc_fn) {
        jg = -1;
        for (int q = 2; q < n_groups; ++q)
          if (grp[q].rtc == th[j]->rtc_fn) jg = q;
      } else {
        jg = (ctx->specialize && !f64 && th[j]->shape != kShapeGeneric) ? 0 : 1;
      }
      if (jg != g) continue;
      list.push_back(j);
      G.total += data[j]->total;
      G.n_histo += data[j]->n_histo;
      if (data[j]->f64 || data[j]->max_count >= kInvTab) G.in_table = 0;
    }
    G.n = (int32_t)list.size() - G.first;
  }
  int64_t slots = 0, units_all = 0;
  for (int g = 0; g < n_groups; ++g) {
    Group &G = grp[g];
    if (G.n == 0) continue;
    int anchor = ctx->anchor_every;
    G.W = ctx->pick_batch(g != 0, mode, cost_kind, f64, G.total, &anchor);
    if (mode == kModeGrad) G.W = std::min<int64_t>(G.W, kMaxGradSplit);
    G.anchor = anchor;
    G.n_units = (G.total + G.W - 1) / G.W;
    G.slot_base = (int32_t)std::min<int64_t>(slots, INT32_MAX);
    slots += G.n_units + G.n_histo;
    units_all += G.n_units;
  }
  if (slots > INT32_MAX) {
    set_err(ctx, "launch needs more than 2^31 work units");
    return MU_E_UNSUPPORTED;
  }
  const size_t n_p = (size_t)n_jobs * ld;
  const size_t n_c = (size_t)n_jobs;
  const size_t n_g = grad ? (size_t)n_jobs * ld : 0;
  const size_t jobs_bytes = (size_t)n_jobs * sizeof(DevJob);
  const size_t list_bytes = (size_t)n_jobs * sizeof(int32_t);
  const size_t start_bytes = (size_t)units_all * 2 * sizeof(int32_t);
  const size_t meta = ((jobs_bytes + list_bytes + start_bytes + 255) & ~size_t(255));
  const size_t up_bytes = meta + (mem == MU_MEM_HOST ? n_p * sizeof(double) : 0);
  if ((st = ctx->djobs.ensure(ctx, up_bytes, false)) != MU_OK) return st;
  if ((st = ctx->staging.ensure(ctx, up_bytes)) != MU_OK) return st;
  if ((st = ctx->partial.ensure(ctx, (size_t)slots * kSlot * sizeof(double), false)) != MU_OK) return st;
  if (mem == MU_MEM_HOST) {
    if ((st = ctx->dout.ensure(ctx, (n_c + n_g) * sizeof(double), false)) != MU_OK) return st;
    if ((st = ctx->staging_out.ensure(ctx, (n_c + n_g) * sizeof(double))) != MU_OK) return st;
  }
  // gradient merge plans first (they may upload)
  std::vector<const int32_t *> plans(n_jobs, nullptr);
  int merge_lds = 0;
  if (grad)
    for (int j = 0; j < n_jobs; ++j) {
      int lds = 0;
      if ((st = const_cast<mu_data *>(data[j])->grad_plan(th[j], &plans[j], &lds)) != MU_OK) return st;
      merge_lds = std::max(merge_lds, lds);
    }
  ctx->wait_staging();
  char *up = static_cast<char *>(ctx->staging.ptr);
  char *dup = static_cast<char *>(ctx->djobs.ptr);
  DevJob *jobs = reinterpret_cast<DevJob *>(up);
  int32_t *hl = reinterpret_cast<int32_t *>(up + jobs_bytes);
  int32_t *hs = reinterpret_cast<int32_t *>(up + jobs_bytes + list_bytes);
  const double *dp = params;
  if (mem == MU_MEM_HOST) {
    std::memcpy(up + meta, params, n_p * sizeof(double));
    dp = reinterpret_cast<const double *>(dup + meta);
  }
  double *dc = cost, *dg = grad;
  if (mem == MU_MEM_HOST) {
    dc = static_cast<double *>(ctx->dout.ptr);
    dg = grad ? dc + n_c : nullptr;
  }
  std::memcpy(hl, list.data(), list_bytes);
  int64_t start_at = 0;  // first unit_start entry of the group
  std::vector<int64_t> start_of(n_groups, 0);
  for (int g = 0; g < n_groups; ++g) {
    const Group &G = grp[g];
    start_of[g] = start_at;
    if (G.n == 0) continue;
    int64_t goff = 0;
    int32_t jbase = 0;
    for (int li = G.first; li < G.first + G.n; ++li) {
      const int j = list[li];
      DevJob &J = jobs[j];
      std::memset(&J, 0, sizeof J);
      J.th = th[j]->d_th;
      J.histos = data[j]->d_hh;
      J.counts = data[j]->counts;
      J.p = dp + (size_t)j * ld;
      J.cost_out = dc + j;
      J.grad_out = dg ? dg + (size_t)j * ld : nullptr;
      J.plan = plans[j];
      J.goff = goff;
      J.split_w = G.W;
      J.jbase = jbase;
      J.slot_base = G.slot_base;
      J.n_histo = data[j]->n_histo;
      J.shape = g == 0 ? th[j]->shape : kShapeGeneric;  // (run-time compiled groups do not read it)
      goff += data[j]->total;
      jbase += data[j]->n_histo;
    }
    // where each unit's range starts: (job-list entry within the group, histogram)
    int li = 0, h = 0;
    int64_t hend = data[list[G.first]]->hh[0].n;
    int64_t jstart = 0;
    for (int64_t u = 0; u < G.n_units; ++u) {
      const int64_t pos = u * G.W;
      while (pos >= hend) {
        const mu_data *dj = data[list[G.first + li]];
        if (++h == dj->n_histo) {
          h = 0;
          jstart += dj->total;
          ++li;
        }
        const mu_data *dn = data[list[G.first + li]];
        hend = jstart + dn->hh[h].off + dn->hh[h].n;
      }
      hs[2 * (start_at + u)] = li;
      hs[2 * (start_at + u) + 1] = h;
    }
    start_at += G.n_units;
  }
  e = hipMemcpyAsync(dup, up, up_bytes, hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(jobs)");
  ctx->mark_staging();
  double *part = static_cast<double *>(ctx->partial.ptr);
  for (int g = 0; g < n_groups; ++g) {
    const Group &G = grp[g];
    if (G.n == 0) continue;
    LaunchArgs a;
    std::memset(&a, 0, sizeof a);
    a.jobs = reinterpret_cast<const DevJob *>(dup);
    a.job_list = reinterpret_cast<const int32_t *>(dup + jobs_bytes) + G.first;
    a.unit_start = reinterpret_cast<const int32_t *>(dup + jobs_bytes + list_bytes) + 2 * start_of[g];
    a.n_units = (int32_t)G.n_units;
    a.n_vec = G.n;
    a.split_w = G.W;
    a.total = G.total;
    a.cost_kind = cost_kind;
    a.anchor_every = G.anchor;
    a.inv_src = ctx->d_inv;
    a.counts_in_table = G.in_table;
    a.partial = part + (size_t)G.slot_base * kSlot;
    const int ti = ctx->time_begin(grad ? MU_TIME_EVAL_GRAD : MU_TIME_EVAL_COST, ctx->stream);
    e = G.rtc ? launch_rtc(G.rtc, a, mode, f64, ctx->stream) : launch_eval_batch(a, mode, f64, g == 1, ctx->stream);
    ctx->time_end(ti, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "batched evaluation launch");
  }
  {
    LaunchArgs m;
    std::memset(&m, 0, sizeof m);
    m.jobs = reinterpret_cast<const DevJob *>(dup);
    m.partial = part;
    const int ti = ctx->time_begin(MU_TIME_MERGE, ctx->stream);
    int max_histo = 0;
    for (int j = 0; j < n_jobs; ++j) max_histo = std::max(max_histo, data[j]->n_histo);
    const bool narrow = n_jobs >= kNarrowJobs && max_histo <= kNarrowHisto;
    e = launch_merge(m, mode, n_jobs, merge_lds, narrow, ctx->stream);
    ctx->time_end(ti, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "merge launch");
  }
  if (mem == MU_MEM_HOST) {
    e = hipMemcpyAsync(ctx->staging_out.ptr, ctx->dout.ptr, (n_c + n_g) * sizeof(double), hipMemcpyDeviceToHost,
                       ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(results)");
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    const double *o = static_cast<const double *>(ctx->staging_out.ptr);
    std::memcpy(cost, o, n_c * sizeof(double));
    // entries past a job's n_par are left untouched
    if (grad)
      for (int j = 0; j < n_jobs; ++j)
        std::memcpy(grad + (size_t)j * ld, o + n_c + (size_t)j * ld, th[j]->h.n_par * sizeof(double));
  }
  return MU_OK;
}

}  // namespace mu

// ------------------------------------------------------------------ tuning

// The tuned (tile, anchor) of single-dataset launches of this theory's shape,
// mode, cost and size.
static void remember_key(mu_ctx *ctx, int key, int tile, int anchor) {
  for (auto &t : ctx->tuned)
    if (t.key == key) {
      t.tile = tile;
      t.anchor = anchor;
      return;
    }
  ctx->tuned.push_back({key, tile, anchor});
}

// The tuned (tile, anchor) of single-dataset launches of this theory's shape,
// mode, cost and size.
static void remember_tuned(mu_ctx *ctx, const mu_theory *th, int mode, int cost_kind, int64_t work, int tile,
                           int anchor) {
  const int shape = ctx->specialize ? th->shape : kShapeGeneric;
  remember_key(ctx, tune_key(shape, mode, cost_kind, 1, work), tile, anchor);
}

extern "C" mu_status mu_autotune_set(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                                     int32_t n_vec, int32_t grad, int32_t tile_bins, int32_t anchor_every) {
  if (!ctx) return MU_E_ARG;
  mu_status st = check_pair(ctx, data, th);
  if (st != MU_OK) return st;
  if (n_vec < 1 || (cost_kind != MU_COST_CHI2 && cost_kind != MU_COST_POISSON) || tile_bins < kWave ||
      tile_bins > kMaxSplit || anchor_every < 1 || anchor_every > 256) {
    set_err(ctx, "autotune_set needs n_vec >= 1, a cost kind, tile_bins in [%d, %d] and anchor_every in [1, 256]",
            kWave, kMaxSplit);
    return MU_E_ARG;
  }
  remember_tuned(ctx, th, grad ? kModeGrad : kModeCost, cost_kind, (int64_t)n_vec * data->total, tile_bins,
                 anchor_every);
  return MU_OK;
}

// A tuning candidate that reproduced the reference costs, with its time per
// launch (ms) from the first pass.
struct TuneCand {
  int64_t tile;
  int anchor;
  float ms;
};

// Final pass of both autotuners: the first pass times each candidate once,
// in a fixed order while the clocks ramp, so candidates within a few percent
// are not told apart. The fastest few are timed again in three interleaved
// rounds of more launches each, and the one with the lowest time in any
// round wins.
template <typename TimeOne>
static mu_status tune_final(std::vector<TuneCand> &passed, TimeOne &&time_one, int64_t &bt, int &ba, float &best) {
  constexpr int kFinalists = 4, kRounds = 3, kReps = 10;
  std::stable_sort(passed.begin(), passed.end(), [](const TuneCand &x, const TuneCand &y) { return x.ms < y.ms; });
  if (passed.size() > (size_t)kFinalists) passed.resize(kFinalists);
  for (TuneCand &c : passed) c.ms = 1e30f;
  for (int r = 0; r < kRounds; ++r)
    for (TuneCand &c : passed) {
      float ms = 0.f;
      const mu_status s = time_one(c.tile, c.anchor, kReps, ms);
      if (s != MU_OK) return s;
      c.ms = std::min(c.ms, ms);
    }
  for (const TuneCand &c : passed)
    if (c.ms < best) {
      best = c.ms;
      bt = c.tile;
      ba = c.anchor;
    }
  return MU_OK;
}

extern "C" mu_status mu_autotune(mu_ctx *ctx, const mu_data *data, const mu_theory *th, mu_cost cost_kind,
                                 const double *params, int32_t n_vec, unsigned mem, int32_t grad,
                                 int32_t *best_tile, int32_t *best_anchor, double *best_us) {
  if (!ctx) return MU_E_ARG;
  mu_status st = check_pair(ctx, data, th);
  if (st != MU_OK) return st;
  if (!params || n_vec < 1 || (mem != MU_MEM_HOST && mem != MU_MEM_DEVICE) ||
      (cost_kind != MU_COST_CHI2 && cost_kind != MU_COST_POISSON)) {
    set_err(ctx, "autotune needs parameters, n_vec >= 1, a memory kind and a cost kind");
    return MU_E_ARG;
  }
  (void)hipSetDevice(ctx->device);
  mu_data *d = const_cast<mu_data *>(data);
  const int n_par = th->h.n_par;
  const int mode = grad ? kModeGrad : kModeCost;
  double *buf = nullptr;
  const size_t n_p = (size_t)n_vec * n_par;
  const size_t n_out = (size_t)n_vec * (1 + (grad ? n_par : 0));
  hipError_t e = hipMalloc(&buf, (n_p + n_out) * sizeof(double));
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(autotune)");
  e = hipMemcpyAsync(buf, params, n_p * sizeof(double),
                     mem == MU_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, ctx->stream);
  if (e != hipSuccess) {
    (void)hipFree(buf);
    return hip_fail(ctx, e, "hipMemcpyAsync(autotune)");
  }
  double *dc = buf + n_p, *dg = grad ? dc + n_vec : nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipFree(buf);
    return hip_fail(ctx, e, "hipEventCreate(autotune)");
  }
  const int saved_tile = ctx->tile_bins, saved_anchor = ctx->anchor_every;
  std::vector<double> ref(n_vec), cur(n_vec);
  bool have_ref = false;
  int64_t bt = 0;
  int ba = 0;
  float best = 1e30f;
  // candidates (bins per wave of the split launch): whole multiples of the
  // resident wave count (every wave of a round equally loaded), and powers of
  // two
  std::vector<int64_t> cand;
  const int64_t work_all = (int64_t)n_vec * d->total;
  {
    const int shape = ctx->specialize ? th->shape : kShapeGeneric;
    const int per_cu = eval_blocks_per_cu(mode, cost_kind, d->f64, shape);
    const int64_t cap = (int64_t)std::max(per_cu, 1) * (kBlock / kWave) * std::max(ctx->n_cu, 1);
    for (int m : {1, 2, 3, 4, 6, 8}) {
      const int64_t w = std::max<int64_t>(kWave, (work_all + m * cap - 1) / (m * cap));
      if (std::find(cand.begin(), cand.end(), w) == cand.end()) cand.push_back(w);
    }
    for (int64_t w = kMinTile; w <= kMaxTile && w < work_all; w *= 2)
      if (std::find(cand.begin(), cand.end(), w) == cand.end()) cand.push_back(w);
  }
  // one candidate: two warm-up launches, then `reps` timed ones (ms per launch)
  auto time_one = [&](int64_t tile, int anchor, int reps, float &ms) -> mu_status {
    ctx->tile_bins = (int)tile;
    ctx->anchor_every = anchor;
    mu_status s = MU_OK;
    for (int w = 0; w < 2 && s == MU_OK; ++w)
      s = eval_uniform(ctx, d, th, cost_kind, buf, n_vec, MU_MEM_DEVICE, dc, nullptr, dg, nullptr, mode);
    if (s != MU_OK) return s;
    hipError_t he = hipEventRecord(e0, ctx->stream);
    for (int r = 0; r < reps && s == MU_OK && he == hipSuccess; ++r)
      s = eval_uniform(ctx, d, th, cost_kind, buf, n_vec, MU_MEM_DEVICE, dc, nullptr, dg, nullptr, mode);
    if (s != MU_OK) return s;
    ms = 0.f;
    if (he == hipSuccess) he = hipEventRecord(e1, ctx->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) return hip_fail(ctx, he, "autotune timing events");
    ms /= (float)reps;
    return MU_OK;
  };
  std::vector<TuneCand> passed;
  for (size_t ci = 0; ci < cand.size() && st == MU_OK; ++ci) {
    const int64_t tile = cand[ci];
    for (int anchor : {32, 64, 128, 256}) {
      float ms = 0.f;
      if ((st = time_one(tile, anchor, 5, ms)) != MU_OK) break;
      // every candidate must reproduce the first one's costs to rounding
      const hipError_t ce = hipMemcpy(cur.data(), dc, n_vec * sizeof(double), hipMemcpyDeviceToHost);
      if (ce != hipSuccess) {
        st = hip_fail(ctx, ce, "hipMemcpy(autotune costs)");
        break;
      }
      bool ok = true;
      if (!have_ref) {
        ref = cur;
        have_ref = true;
      } else {
        for (int v = 0; v < n_vec; ++v)
          if (!(std::fabs(cur[v] - ref[v]) <= 1e-12 * std::fabs(ref[v])) && !(std::isnan(cur[v]) && std::isnan(ref[v])))
            ok = false;
      }
      if (ok) passed.push_back({tile, anchor, ms});
    }
  }
  if (st == MU_OK) st = tune_final(passed, time_one, bt, ba, best);
  ctx->tile_bins = saved_tile;
  ctx->anchor_every = saved_anchor;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(ctx->stream);  // before freeing what the launches use
  (void)hipFree(buf);
  if (st != MU_OK) return st;
  if (bt == 0) {
    set_err(ctx, "no tuning candidate ran");
    return MU_E_DEVICE;
  }
  // remember the choice for launches of this shape, mode, cost and size
  remember_tuned(ctx, th, mode, cost_kind, work_all, (int)bt, ba);
  if (best_tile) *best_tile = (int32_t)bt;
  if (best_anchor) *best_anchor = ba;
  if (best_us) *best_us = best * 1e3;
  return MU_OK;
}

// Batched launches: the (bins per wave, anchor) pair that runs a batch of
// jobs fastest, remembered for batched launches of the same kind, mode, cost
// and size (to a power of two).
extern "C" mu_status mu_autotune_batch(mu_ctx *ctx, int32_t n_jobs, const mu_data *const *data,
                                       const mu_theory *const *th, mu_cost cost_kind, int32_t ld,
                                       const double *params, unsigned mem, int32_t grad, int32_t *best_tile,
                                       int32_t *best_anchor, double *best_us) {
  if (!ctx) return MU_E_ARG;
  if (n_jobs < 1 || !data || !th || !params || ld < 1 || (mem != MU_MEM_HOST && mem != MU_MEM_DEVICE) ||
      (cost_kind != MU_COST_CHI2 && cost_kind != MU_COST_POISSON)) {
    set_err(ctx, "autotune_batch needs n_jobs >= 1, data, theories, parameters, ld >= 1, a memory kind and a cost kind");
    return MU_E_ARG;
  }
  mu_status st = MU_OK;
  for (int j = 0; j < n_jobs; ++j) {
    if ((st = check_pair(ctx, data[j], th[j])) != MU_OK) return st;
    if (th[j]->h.n_par > ld || data[j]->f64 != data[0]->f64) {
      set_err(ctx, "job %d: more parameters than ld, or mixed count storage", j);
      return MU_E_ARG;
    }
  }
  (void)hipSetDevice(ctx->device);
  const int mode = grad ? kModeGrad : kModeCost;
  const int f64 = data[0]->f64;
  // the two launch groups of run_batch and their sizes
  int64_t total[2] = {0, 0};
  for (int j = 0; j < n_jobs; ++j) {
    const bool fixed = ctx->specialize && !f64 && th[j]->shape != kShapeGeneric;
    total[fixed ? 0 : 1] += data[j]->total;
  }
  const int lead = total[0] > 0 ? 0 : 1;
  const size_t n_p = (size_t)n_jobs * ld;
  double *buf = nullptr;
  hipError_t e = hipMalloc(&buf, (n_p + (size_t)n_jobs + (grad ? n_p : 0)) * sizeof(double));
  if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(autotune)");
  e = hipMemcpyAsync(buf, params, n_p * sizeof(double),
                     mem == MU_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, ctx->stream);
  if (e != hipSuccess) {
    (void)hipFree(buf);
    return hip_fail(ctx, e, "hipMemcpyAsync(autotune)");
  }
  double *dc = buf + n_p, *dg = grad ? dc + n_jobs : nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    (void)hipFree(buf);
    return hip_fail(ctx, e, "hipEventCreate(autotune)");
  }
  const int saved_tile = ctx->tile_bins, saved_anchor = ctx->anchor_every;
  std::vector<double> ref(n_jobs), cur(n_jobs);
  bool have_ref = false;
  int64_t bt = 0;
  int ba = 0;
  float best = 1e30f;
  std::vector<int64_t> cand;
  {
    const int per_cu = eval_batch_blocks_per_cu(mode, cost_kind, f64, lead);
    const int64_t cap = (int64_t)std::max(per_cu, 1) * (kBlock / kWave) * std::max(ctx->n_cu, 1);
    for (int m : {1, 2, 3, 4, 6, 8}) {
      const int64_t w = std::max<int64_t>(kWave, (total[lead] + m * cap - 1) / (m * cap));
      if (std::find(cand.begin(), cand.end(), w) == cand.end()) cand.push_back(w);
    }
    for (int64_t w = kMinTile; w <= kMaxTile && w < total[lead]; w *= 2)
      if (std::find(cand.begin(), cand.end(), w) == cand.end()) cand.push_back(w);
  }
  auto time_one = [&](int64_t tile, int anchor, int reps, float &ms) -> mu_status {
    ctx->tile_bins = (int)tile;
    ctx->anchor_every = anchor;
    mu_status s = MU_OK;
    for (int w = 0; w < 2 && s == MU_OK; ++w) s = run_batch(ctx, n_jobs, data, th, cost_kind, ld, buf, MU_MEM_DEVICE, dc, dg);
    if (s != MU_OK) return s;
    hipError_t he = hipEventRecord(e0, ctx->stream);
    for (int r = 0; r < reps && s == MU_OK && he == hipSuccess; ++r)
      s = run_batch(ctx, n_jobs, data, th, cost_kind, ld, buf, MU_MEM_DEVICE, dc, dg);
    if (s != MU_OK) return s;
    ms = 0.f;
    if (he == hipSuccess) he = hipEventRecord(e1, ctx->stream);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
    if (he != hipSuccess) return hip_fail(ctx, he, "autotune timing events");
    ms /= (float)reps;
    return MU_OK;
  };
  std::vector<TuneCand> passed;
  for (size_t ci = 0; ci < cand.size() && st == MU_OK; ++ci) {
    for (int anchor : {32, 64, 128, 256}) {
      const int64_t tile = std::min<int64_t>(cand[ci], kMaxSplit);
      float ms = 0.f;
      if ((st = time_one(tile, anchor, 5, ms)) != MU_OK) break;
      // every candidate must reproduce the first one's costs to rounding
      const hipError_t ce = hipMemcpy(cur.data(), dc, n_jobs * sizeof(double), hipMemcpyDeviceToHost);
      if (ce != hipSuccess) {
        st = hip_fail(ctx, ce, "hipMemcpy(autotune costs)");
        break;
      }
      bool ok = true;
      if (!have_ref) {
        ref = cur;
        have_ref = true;
      } else {
        for (int j = 0; j < n_jobs; ++j)
          if (!(std::fabs(cur[j] - ref[j]) <= 1e-12 * std::fabs(ref[j])) && !(std::isnan(cur[j]) && std::isnan(ref[j])))
            ok = false;
      }
      if (ok) passed.push_back({tile, anchor, ms});
    }
  }
  if (st == MU_OK) st = tune_final(passed, time_one, bt, ba, best);
  ctx->tile_bins = saved_tile;
  ctx->anchor_every = saved_anchor;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(ctx->stream);  // before freeing what the launches use
  (void)hipFree(buf);
  if (st != MU_OK) return st;
  if (bt == 0) {
    set_err(ctx, "no tuning candidate ran");
    return MU_E_DEVICE;
  }
  for (int g = 0; g < 2; ++g)
    if (total[g] > 0) remember_key(ctx, tune_key(g == 1 ? kShapeGeneric : kShapeCount, mode, cost_kind, 0, total[g]),
                                   (int)bt, ba);
  if (best_tile) *best_tile = (int32_t)bt;
  if (best_anchor) *best_anchor = ba;
  if (best_us) *best_us = best * 1e3;
  return MU_OK;
}

// ------------------------------------------------------- tuning cache file
//
//   mu-autotune 1
//   arch <device architecture name>
//   <shape> <mode> <cost> <kind> <log2 size> <bins per wave> <anchor>   (one line per choice)
//
// shape: 0 interpreted, 1..5 compiled shapes, 6 batched launch of compiled
// shapes; mode: 0 cost, 1 gradient; cost: 0 chi^2, 1 likelihood; kind:
// 0 batched, 1 single-dataset launch.

namespace {

struct CacheEntry {
  int shape, mode, cost, kind, lg, tile, anchor;
};

mu_status parse_cache(const char *path, std::string &arch, std::vector<CacheEntry> &out, std::string &why) {
  FILE *f = path ? std::fopen(path, "r") : nullptr;
  if (!f) {
    why = std::string("cannot open tuning cache ") + (path ? path : "(null)");
    return MU_E_ARG;
  }
  char line[512];
  int ln = 0;
  mu_status st = MU_OK;
  bool head = false, have_arch = false;
  while (std::fgets(line, sizeof line, f)) {
    ++ln;
    std::string l(line);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r' || l.back() == ' ')) l.pop_back();
    if (l.empty() || l[0] == '#') continue;
    if (!head) {
      if (l != "mu-autotune 1") {
        why = "tuning cache: line " + std::to_string(ln) + ": expected the header 'mu-autotune 1'";
        st = MU_E_ARG;
        break;
      }
      head = true;
      continue;
    }
    if (!have_arch) {
      char a[128];
      if (std::sscanf(l.c_str(), "arch %127s", a) != 1) {
        why = "tuning cache: line " + std::to_string(ln) + ": expected 'arch <name>'";
        st = MU_E_ARG;
        break;
      }
      arch = a;
      have_arch = true;
      continue;
    }
    CacheEntry c;
    char extra;
    if (std::sscanf(l.c_str(), "%d %d %d %d %d %d %d %c", &c.shape, &c.mode, &c.cost, &c.kind, &c.lg, &c.tile,
                    &c.anchor, &extra) != 7 ||
        c.shape < 0 || c.shape > kShapeCount || c.mode < 0 || c.mode > 1 || c.cost < 0 || c.cost > 1 || c.kind < 0 ||
        c.kind > 1 || c.lg < 0 || c.lg > 62 || c.tile < kWave || c.tile > kMaxSplit || c.anchor < 1 ||
        c.anchor > 256) {
      why = "tuning cache: line " + std::to_string(ln) + ": malformed or out-of-range entry";
      st = MU_E_ARG;
      break;
    }
    out.push_back(c);
  }
  std::fclose(f);
  if (st == MU_OK && (!head || !have_arch)) {
    why = "tuning cache: missing header or architecture line";
    st = MU_E_ARG;
  }
  return st;
}

}  // namespace

extern "C" mu_status mu_autotune_check_file(const char *path, char *msg, int32_t msg_len) {
  std::string arch, why;
  std::vector<CacheEntry> e;
  const mu_status st = parse_cache(path, arch, e, why);
  put_msg(msg, msg_len, st == MU_OK ? "ok: " + std::to_string(e.size()) + " entries for " + arch : why);
  return st;
}

extern "C" mu_status mu_autotune_save(mu_ctx *ctx, const char *path) {
  if (!ctx || !path) return MU_E_ARG;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipGetDeviceProperties");
  FILE *f = std::fopen(path, "w");
  if (!f) {
    set_err(ctx, "cannot write tuning cache %s", path);
    return MU_E_ARG;
  }
  std::fprintf(f, "mu-autotune 1\narch %s\n# shape mode cost kind log2_size bins_per_wave anchor\n", prop.gcnArchName);
  for (const auto &t : ctx->tuned) {
    int k = t.key;
    const int lg = k % 64;
    k /= 64;
    const int kind = k % 2;
    k /= 2;
    const int cost = k % 2;
    k /= 2;
    const int mode = k % 4;
    const int shape = k / 4;
    std::fprintf(f, "%d %d %d %d %d %d %d\n", shape, mode, cost, kind, lg, t.tile, t.anchor);
  }
  const bool ok = std::fclose(f) == 0;
  if (!ok) {
    set_err(ctx, "writing tuning cache %s failed", path);
    return MU_E_ARG;
  }
  return MU_OK;
}

extern "C" mu_status mu_autotune_load(mu_ctx *ctx, const char *path) {
  if (!ctx) return MU_E_ARG;
  std::string arch, why;
  std::vector<CacheEntry> ent;
  mu_status st = parse_cache(path, arch, ent, why);
  if (st != MU_OK) {
    set_err(ctx, "%s", why.c_str());
    return st;
  }
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipGetDeviceProperties");
  if (arch != prop.gcnArchName) {
    set_err(ctx, "tuning cache was written for %s, this device is %s", arch.c_str(), prop.gcnArchName);
    return MU_E_UNSUPPORTED;
  }
  for (const CacheEntry &c : ent)
    remember_key(ctx, (((c.shape * 4 + c.mode) * 2 + c.cost) * 2 + c.kind) * 64 + c.lg, c.tile, c.anchor);
  return MU_OK;
}
