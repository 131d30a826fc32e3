// Learned seeder: histogram generator, network training and inference on gfx950.
//
// Generator (one workgroup per sample): the sample's parameters theta =
// (N0, Nbkg, A, lambda, nu, phi) come from Philox4x32-10 uniforms (key = seed,
// counter = (sample index, 0xFFFFFFFF, 0 / 1)); each of the 1024 rebinned bins
// has the expected count sum_s N(t_s) over its 8 bins of 0.001 us (Eq. 1 with
// A(t) = A e^(-lambda t) cos(2 pi nu t + phi)) and one Poisson draw from
// counter (sample index, bin, iteration): inversion below a mean of 10,
// Hoermann's transformed rejection (PTRS, 1993) above.
//
// Network: 1024-512-256-128-8 perceptron with ReLU.  GEMMs use the
// 16x16x32 BF16 matrix-core instruction with FP32 accumulation; activations and
// gradients are rounded to BF16 where they feed a GEMM and kept in FP32
// elsewhere (bias, ReLU mask, bias gradient, Adam master weights).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mu_internal.h"
#include "mu_runtime.h"
#include "mu_seeder.h"

#pragma clang fp contract(off)

using namespace mu;

namespace {

constexpr int kDims[kSeedLayers + 1] = {1024, 512, 256, 128, 8};
constexpr double kTau = 2.1969811;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kFine = 8192, kCoarse = 1024, kRebin = 8;
constexpr double kDtFine = 0.001;

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ Philox

struct U4 {
  unsigned x, y, z, w;
};

__device__ __forceinline__ U4 philox(U4 c, unsigned k0, unsigned k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
    const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
    const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ double u01(unsigned x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

// ------------------------------------------------------------------ BF16

__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

// ------------------------------------------------------------- generator

__device__ void draw_theta(unsigned long long seed, unsigned long long idx, double th[6]) {
  const unsigned k0 = (unsigned)seed, k1 = (unsigned)(seed >> 32);
  const U4 a = philox(U4{(unsigned)idx, (unsigned)(idx >> 32), 0xFFFFFFFFu, 0u}, k0, k1);
  const U4 b = philox(U4{(unsigned)idx, (unsigned)(idx >> 32), 0xFFFFFFFFu, 1u}, k0, k1);
  const double u[6] = {u01(a.x), u01(a.y), u01(a.z), u01(a.w), u01(b.x), u01(b.y)};
  th[0] = exp(log(100.0) + u[0] * (log(1e5) - log(100.0)));
  th[1] = 1.0 + u[1] * (10.0 - 1.0);
  th[2] = 0.05 + u[2] * (0.3 - 0.05);
  th[3] = exp(log(0.05) + u[3] * (log(5.0) - log(0.05)));
  th[4] = exp(log(0.1) + u[4] * (log(50.0) - log(0.1)));
  th[5] = u[5] * kTwoPi;
}

// ln k! for the rejection test: the log-gamma function below k = 10, else
// Stirling's series for ln Gamma(k + 1) to the z^-5 term (its first omitted
// term is below 1 / (1680 z^7) = 6e-11 at z = 11), as the method itself
// prescribes; the full log-gamma costs several times as much and every lane
// of a wave runs it whenever one lane takes the slow test.
// out of line: the log-gamma's many constants would otherwise raise the
// generator's register count for a branch that rarely runs
__device__ __attribute__((noinline)) double x_lgamma(double x) { return lgamma(x); }
__device__ __forceinline__ double log_factorial(double k) {
  const double z = fmax(k, 10.0) + 1.0, iz = 1.0 / z, iz2 = iz * iz;
  double lf = (z - 0.5) * log(z) - z + 0.91893853320467274178 + iz * (1.0 / 12.0 - iz2 * (1.0 / 360.0 - iz2 * (1.0 / 1260.0)));
  // a wave-uniform test, so the log-gamma runs only in waves that need it
  if (__builtin_amdgcn_ballot_w64(k < 10.0) != 0) {
    asm volatile("");
    if (k < 10.0) lf = x_lgamma(k + 1.0);
  }
  return lf;
}

// One Poisson draw with mean mu from the counter stream (idx, bin, it).
__device__ double poisson(double mu, unsigned long long seed, unsigned long long idx, unsigned bin) {
  const unsigned k0 = (unsigned)seed, k1 = (unsigned)(seed >> 32);
  if (!(mu > 0.0)) return 0.0;
  if (mu < 10.0) {  // inversion of the cumulative distribution
    const U4 r = philox(U4{(unsigned)idx, (unsigned)(idx >> 32), bin, 0u}, k0, k1);
    const double u = u01(r.x);
    double p = exp(-mu), F = p;
    int k = 0;
    while (u > F && k < 200) {
      ++k;
      p *= mu / k;
      F += p;
    }
    return (double)k;
  }
  // transformed rejection with squeeze (Hoermann 1993)
  const double slam = sqrt(mu), loglam = log(mu);
  const double b = 0.931 + 2.53 * slam;
  const double a = -0.059 + 0.02483 * b;
  const double invalpha = 1.1239 + 1.1328 / (b - 3.4);
  const double vr = 0.9277 - 3.6224 / (b - 2.0);
  const double log_invalpha = log(invalpha);
  for (unsigned it = 0; it < 64; ++it) {
    const U4 r = philox(U4{(unsigned)idx, (unsigned)(idx >> 32), bin, it + 1u}, k0, k1);
    const double us_pair[2][2] = {{u01(r.x), u01(r.y)}, {u01(r.z), u01(r.w)}};
    for (int q = 0; q < 2; ++q) {
      const double U = us_pair[q][0] - 0.5, V = us_pair[q][1];
      const double us = 0.5 - fabs(U);
      const double k = floor((2.0 * a / us + b) * U + mu + 0.43);
      if (us >= 0.07 && V <= vr) return k;
      if (k < 0.0 || (us < 0.013 && V > us)) continue;
      if (log(V) + log_invalpha - log(a / (us * us) + b) <= -mu + k * loglam - log_factorial(k)) return k;
    }
  }
  return floor(mu + 0.5);  // not reached in practice (acceptance > 0.9 per try)
}

// Coarse mode: counts [n][1024] of rebinned bins (one Poisson draw of the
// summed mean of 8 fine bins); fine mode: counts [n][8192], one draw per fine
// bin (counter word 2 = 0x10000 + bin).  theta [n][6], targets [n][8] and mu
// (expected counts, [n][1024] or [n][8192]) are optional.
__global__ __launch_bounds__(256) void gen_kernel(unsigned long long seed, unsigned long long first, int n, int fine,
                                                  float *counts, double *theta, float *targets, double *mu_out) {
  const int s = blockIdx.x;
  if (s >= n) return;
  const unsigned long long idx = first + (unsigned long long)s;
  double th[6];
  draw_theta(seed, idx, th);
  const double w = kTwoPi * th[4];
  const int nb = fine ? kFine : kCoarse, sub = fine ? 1 : kRebin;
  // a rebinned bin's fine bins: the first from the bin's start state, the
  // others by one fine step of each factor (geometric decays, rotation); the
  // thread's first bin starts from a direct evaluation, each later one
  // (blockDim.x bins on) from one step of that stride
  const double r1 = exp(-kDtFine / kTau), r2 = exp(-th[3] * kDtFine);
  double sw, cw;
  sincos(w * kDtFine, &sw, &cw);
  const double t_first = (double)((int)threadIdx.x * sub) * kDtFine;
  const double t_stride = (double)((int)blockDim.x * sub) * kDtFine;
  double E1 = exp(-t_first / kTau), E2 = exp(-th[3] * t_first), SN, CS;
  sincos(w * t_first + th[5], &SN, &CS);
  const double R1 = exp(-t_stride / kTau), R2 = exp(-th[3] * t_stride);
  double SW, CW;
  sincos(w * t_stride, &SW, &CW);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    double e1 = E1, e2 = E2, sn = SN, cs = CS;
    {
      E1 *= R1;
      E2 *= R2;
      const double c2 = CS * CW - SN * SW;
      SN = SN * CW + CS * SW;
      CS = c2;
    }
    double mu = 0.0;
    for (int q = 0; q < sub; ++q) {
      mu += th[0] * e1 * (1.0 + th[2] * e2 * cs) + th[1];
      e1 *= r1;
      e2 *= r2;
      const double c2 = cs * cw - sn * sw;
      sn = sn * cw + cs * sw;
      cs = c2;
    }
    if (mu_out) mu_out[(size_t)s * nb + b] = mu;
    if (counts) counts[(size_t)s * nb + b] = (float)poisson(mu, seed, idx, (unsigned)(fine ? 0x10000 + b : b));
  }
  if (threadIdx.x == 0) {
    if (theta)
      for (int k = 0; k < 6; ++k) theta[(size_t)s * 6 + k] = th[k];
    if (targets) {
      float *T = targets + (size_t)s * 8;
      T[0] = (float)(th[2] / 0.3);
      T[1] = (float)((log(th[3]) - log(0.05)) / log(100.0));
      T[2] = (float)((log(th[4]) - log(0.1)) / log(500.0));
      T[3] = (float)cos(th[5]);
      T[4] = (float)sin(th[5]);
      T[5] = T[6] = T[7] = 0.0f;
    }
  }
}

// Rebin (by `rebin`) and form the network input, the asymmetry
//   x_b = (c_b - 8 Nbkg) / (8 N0 ebar_b) - 1, clipped to [-4, 4], as BF16,
// with N0 and Nbkg from the means m1, m2 of the first and last 256 fine bins
// (two equations m = N0 e + Nbkg, e the lifetime decay averaged over the
// window) and ebar_b the decay averaged over rebinned bin b.  m1 and m2 are
// also written for the default start.
// Inputs either from datasets (src: one count array per sample, 32-bit values
// holding 8 d) or from the generator's contiguous FP32 counts (contig).
__global__ __launch_bounds__(256) void prep_kernel(const uint32_t *const *src, const float *contig, int rebin, int n,
                                                   unsigned short *X, double *n0_out, double *m_first,
                                                   double *m_last) {
  const int s = blockIdx.x;
  if (s >= n) return;
  const uint32_t *pu = src ? src[s] : nullptr;
  const float *pf = src ? nullptr : contig + (size_t)s * kCoarse * rebin;
  constexpr int kWin = 32;  // rebinned bins per estimation window
  __shared__ double red[256];
  __shared__ double red2[256];
  double c[kCoarse / 256];
  double w1 = 0.0, w2 = 0.0;
  for (int q = 0; q < kCoarse / 256; ++q) {
    const int b = threadIdx.x + q * 256;
    double v = 0.0;
    for (int r = 0; r < rebin; ++r)
      v += pu ? (double)pu[b * rebin + r] * kCountUnscale : (double)pf[b * rebin + r];
    c[q] = v;
    if (b < kWin) w1 += v;
    if (b >= kCoarse - kWin) w2 += v;
  }
  red[threadIdx.x] = w1;
  red2[threadIdx.x] = w2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      red[threadIdx.x] += red[threadIdx.x + o];
      red2[threadIdx.x] += red2[threadIdx.x + o];
    }
    __syncthreads();
  }
  const double m1 = red[0] / (kWin * kRebin), m2 = red2[0] / (kWin * kRebin);
  const double r = exp(-kDtFine / kTau);
  const double e1 = (1.0 - pow(r, (double)(kWin * kRebin))) / ((kWin * kRebin) * (1.0 - r));
  const double e2 = e1 * pow(r, (double)(kFine - kWin * kRebin));
  double n0 = (m1 - m2) / (e1 - e2);
  double nb = m2 - n0 * e2;
  nb = nb > 0.1 ? nb : 0.1;
  n0 = n0 > 1.0 ? n0 : 1.0;
  const double kb = kRebin * kDtFine / kTau;
  const double avg = (1.0 - pow(r, (double)kRebin)) / (kRebin * (1.0 - r));
  for (int q = 0; q < kCoarse / 256; ++q) {
    const int b = threadIdx.x + q * 256;
    const double ebar = exp(-kb * (double)b) * avg;
    double x = (c[q] - kRebin * nb) / (kRebin * n0 * ebar) - 1.0;
    x = x < -4.0 ? -4.0 : (x > 4.0 ? 4.0 : x);
    X[(size_t)s * kCoarse + b] = f2bf((float)x);
  }
  if (threadIdx.x == 0) {
    if (n0_out) n0_out[s] = n0;
    if (m_first) m_first[s] = m1;
    if (m_last) m_last[s] = m2;
  }
}

// ------------------------------------------------------------------ GEMM

enum Epi { kEpiStore = 0, kEpiBiasRelu = 1, kEpiBias = 2, kEpiReluGrad = 3 };

struct GemmArgs {
  const unsigned short *A;  // A(i, k) = A[i * sAi + k * sAk]
  long long sAi, sAk;
  const unsigned short *B;  // B(k, j) = B[k * sBk + j * sBj]
  long long sBk, sBj;
  int M, N, K, epi;
  float *C;                 // FP32 result [M][N] (Z, Y, dW, or dZ)
  const float *bias;        // [N]
  unsigned short *Cbf;      // BF16 copy (next layer's input or G) [M][N]
  const float *Zprev;       // ReLU mask source [M][N]
};

// The epilogue of one output element v = C(row, col) (the full K sum).
__device__ __forceinline__ void gemm_store(const GemmArgs &g, int row, int col, float v) {
  const size_t o = (size_t)row * g.N + col;
  switch (g.epi) {
    case kEpiBiasRelu: {
      v += g.bias[col];
      g.C[o] = v;
      g.Cbf[o] = f2bf(v > 0.f ? v : 0.f);
      break;
    }
    case kEpiBias:
      g.C[o] = v + g.bias[col];
      break;
    case kEpiReluGrad: {
      const float dz = g.Zprev[o] > 0.f ? v : 0.f;
      g.C[o] = dz;
      g.Cbf[o] = f2bf(dz);
      break;
    }
    default:
      g.C[o] = v;
      break;
  }
}

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
constexpr int kTileK = 32;        // K per step: one 16x16x32 product per 16x16 tile
constexpr int kLdsK = kTileK + 8;  // padded LDS row (80 B)

// One 64 x 32 operand tile (64 rows of the M or N dimension, 32 of K) from
// global memory into registers: 8 elements per thread. KC: the operand is
// contiguous along K (element (r, k) at p[r * ld + k]), each thread reads 8
// consecutive k of one row; otherwise contiguous along the rows (element
// (r, k) at p[r + k * ld]), each thread reads 8 consecutive rows of one k.
// Elements outside [0, rows) x [k0, kend) read as zero.
template <bool KC>
__device__ __forceinline__ uint4 gemm_fetch(const unsigned short *p, long long ld, int rows, int r0, int k0, int kend) {
  const int t = threadIdx.x;
  const int r = KC ? r0 + (t >> 2) : r0 + (t & 7) * 8;
  const int k = KC ? k0 + (t & 3) * 8 : k0 + (t >> 3);
  if (KC) {
    if (r < rows && k + 8 <= kend && (ld & 7) == 0)
      return *reinterpret_cast<const uint4 *>(p + (size_t)r * ld + k);
  } else {
    if (k < kend && r + 8 <= rows && (ld & 7) == 0)
      return *reinterpret_cast<const uint4 *>(p + r + (size_t)k * ld);
  }
  // a ragged edge: element by element
  auto el = [&](int q) -> unsigned {
    if (KC) return (r < rows && k + q < kend) ? p[(size_t)r * ld + k + q] : 0u;
    return (k < kend && r + q < rows) ? p[r + q + (size_t)k * ld] : 0u;
  };
  return uint4{el(0) | (el(1) << 16), el(2) | (el(3) << 16), el(4) | (el(5) << 16), el(6) | (el(7) << 16)};
}

// The fetched elements into the LDS tile T[row][k] (K contiguous in LDS).
template <bool KC>
__device__ __forceinline__ void gemm_put(unsigned short (*T)[kLdsK], uint4 v) {
  const int t = threadIdx.x;
  if (KC) {
    *reinterpret_cast<uint4 *>(&T[t >> 2][(t & 3) * 8]) = v;
  } else {
    const int r = (t & 7) * 8, k = t >> 3;
    const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 8; ++q) T[r + q][k] = (unsigned short)(w[q >> 1] >> (16 * (q & 1)));
  }
}

// C = A B on 64 x 64 output tiles: four waves, each 32 x 32 = 2 x 2 products of
// 16 x 16 (v_mfma_f32_16x16x32_bf16, FP32 accumulation), K in steps of 32 with
// two LDS buffers (the next step's global reads are in flight during this
// step's products; one barrier per step). Workgroup z of the grid's third
// dimension takes K range [z kps, (z + 1) kps): with one range the epilogue
// runs here, otherwise the FP32 partial tile goes to part[z] and
// gemm_reduce_kernel sums the ranges in order. Lane l of a 16 x 16 product
// holds row l % 16 of A and column l % 16 of B with eight K elements each,
// the same eight for both, and receives C rows 4 (l / 16) + j, column l % 16.
template <bool AKC, bool BKC>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g, int kps, float *part) {
  __shared__ __align__(16) unsigned short As[2][64][kLdsK];
  __shared__ __align__(16) unsigned short Bs[2][64][kLdsK];
  const int bi = blockIdx.y * 64, bj = blockIdx.x * 64;
  const int kbeg = blockIdx.z * kps, kend = min(g.K, kbeg + kps);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lg = lane >> 4;
  const long long lda = AKC ? g.sAi : g.sAk, ldb = BKC ? g.sBj : g.sBk;
  float4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = float4v{0.f, 0.f, 0.f, 0.f};

  uint4 ra = gemm_fetch<AKC>(g.A, lda, g.M, bi, kbeg, kend);
  uint4 rb = gemm_fetch<BKC>(g.B, ldb, g.N, bj, kbeg, kend);
  gemm_put<AKC>(As[0], ra);
  gemm_put<BKC>(Bs[0], rb);
  __syncthreads();
  int cur = 0;
  for (int k0 = kbeg; k0 < kend; k0 += kTileK) {
    const bool more = k0 + kTileK < kend;
    if (more) {
      ra = gemm_fetch<AKC>(g.A, lda, g.M, bi, k0 + kTileK, kend);
      rb = gemm_fetch<BKC>(g.B, ldb, g.N, bj, k0 + kTileK, kend);
    }
    bf16x8 av[2], bv[2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
      av[ti] = *reinterpret_cast<const bf16x8 *>(&As[cur][wr + 16 * ti + li][8 * lg]);
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
      bv[tj] = *reinterpret_cast<const bf16x8 *>(&Bs[cur][wc + 16 * tj + li][8 * lg]);
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
        acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
    if (more) {
      gemm_put<AKC>(As[cur ^ 1], ra);
      gemm_put<BKC>(Bs[cur ^ 1], rb);
    }
    __syncthreads();
    cur ^= 1;
  }
  float *P = part ? part + (size_t)blockIdx.z * g.M * g.N : nullptr;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = bi + wr + 16 * ti + 4 * lg + j;
        const int col = bj + wc + 16 * tj + li;
        if (row >= g.M || col >= g.N) continue;
        if (P)
          P[(size_t)row * g.N + col] = acc[ti][tj][j];
        else
          gemm_store(g, row, col, acc[ti][tj][j]);
      }
}

// Sum of the K ranges' partial tiles in range order, then the epilogue.
__global__ __launch_bounds__(256) void gemm_reduce_kernel(GemmArgs g, const float *part, int n_split) {
  const long long mn = (long long)g.M * g.N;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= mn) return;
  float v = part[i];
  for (int z = 1; z < n_split; ++z) v += part[z * mn + i];
  gemm_store(g, (int)(i / g.N), (int)(i % g.N), v);
}

// ------------------------------------------------------- loss, bias, Adam

// dY = 2 w (Y - T) / B (FP32 and BF16) and per-block partial losses.
__global__ __launch_bounds__(256) void loss_kernel(const float *Y, const float *T, int B, float *dY,
                                                   unsigned short *dYbf, double *partial) {
  __shared__ double red[256];
  double loc = 0.0;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < B * 8) {
    const int o = e & 7;
    const float w = o < kSeedUsedOut ? 1.0f : 0.0f;
    const float d = Y[e] - T[e];
    const float gval = 2.0f * w * d / (float)B;
    dY[e] = gval;
    dYbf[e] = f2bf(gval);
    loc = (double)w * (double)d * (double)d;
  }
  red[threadIdx.x] = loc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void loss_final_kernel(const double *partial, int n, int B, float *loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += partial[i];
  *loss = (float)(s / B);
}

// db[n] = sum_b dZ[b][n] in a fixed order: 64-row slices, four row groups of
// 16 rows each combined in order, then the slices in order.
constexpr int kBiasRows = 64;

// The bias gradients of every layer in one pair of launches (after the
// backward pass, whose dZ of each layer stays in its own buffer): column
// block x of the layers' concatenated columns, row slice y, as above; then
// every column's slices in order.
struct BiasAll {
  const float *dZ[kSeedLayers];
  float *db[kSeedLayers];
  int N[kSeedLayers];
  int col0[kSeedLayers + 1];  // first concatenated column of each layer
};

__global__ __launch_bounds__(256) void bias_grad_all_kernel(BiasAll a, int B, float *part) {
  __shared__ float red[4][64];
  const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
  const int g = blockIdx.x * 64 + c;  // concatenated column
  int l = 0;
  while (l + 1 < kSeedLayers && g >= a.col0[l + 1]) ++l;
  const int n = g - a.col0[l], N = a.N[l];
  const int b0 = blockIdx.y * kBiasRows, b1 = min(B, b0 + kBiasRows);
  const bool on = g < a.col0[kSeedLayers];
  float s = 0.0f;
  if (on)
    for (int b = b0 + rg; b < b1; b += 4) s += a.dZ[l][(size_t)b * N + n];
  red[rg][c] = s;
  __syncthreads();
  if (rg == 0 && on) part[(size_t)blockIdx.y * a.col0[kSeedLayers] + g] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

__global__ __launch_bounds__(256) void bias_grad_all_final_kernel(BiasAll a, const float *part, int n_slices) {
  const int g = blockIdx.x * 256 + threadIdx.x;
  const int tot = a.col0[kSeedLayers];
  if (g >= tot) return;
  int l = 0;
  while (l + 1 < kSeedLayers && g >= a.col0[l + 1]) ++l;
  float s = part[g];
  for (int z = 1; z < n_slices; ++z) s += part[(size_t)z * tot + g];
  a.db[l][g - a.col0[l]] = s;
}

// One Adam step on FP32 master weights. The complements 1 - b1 and 1 - b2 come
// from the host, formed in double like the bias corrections c1 and c2: 1 - b2
// taken in FP32 from the rounded b2 is off by 1.3e-5 relative, which would
// scale the first steps by that much against the bias correction.
// Where each layer's weights sit in the parameters and in their BF16 copy.
struct WeightMap {
  long long off_w[kSeedLayers], off_wbf[kSeedLayers], size[kSeedLayers];
};

// It also writes the BF16 copy of each updated weight (the next forward
// pass's operand), so no conversion launches follow.
__global__ __launch_bounds__(256) void adam_kernel(float *w, const float *g, float *m, float *v, long long n,
                                                   float lr, float b1, float b2, float omb1, float omb2, float eps,
                                                   float c1, float c2, WeightMap wm, unsigned short *wbf) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
#pragma unroll
  for (int l = 0; l < kSeedLayers; ++l)
    if (i >= wm.off_w[l] && i < wm.off_w[l] + wm.size[l]) wbf[wm.off_wbf[l] + (i - wm.off_w[l])] = f2bf(wi);
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float *src, unsigned short *dst, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = f2bf(src[i]);
}

// Start parameters from the network output and the first / last window means.
__global__ __launch_bounds__(256) void decode_kernel(const float *Y, const double *m_first, const double *m_last,
                                                     int n, double *start, unsigned char *ok) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  // default start: N0 and Nbkg from two window means with the lifetime decay
  // averaged over each window (geometric sums), A, lambda, nu, phi fixed
  const double r = exp(-kDtFine / kTau);
  const double e1 = (1.0 - pow(r, 256.0)) / (256.0 * (1.0 - r));
  const double e2 = e1 * pow(r, (double)(kFine - 256));
  double n0 = (m_first[s] - m_last[s]) / (e1 - e2);
  double nb = m_last[s] - n0 * e2;
  nb = nb > 0.1 ? nb : 0.1;
  n0 = n0 > 1.0 ? n0 : 1.0;
  double *o = start + (size_t)s * 6;
  o[0] = n0;
  o[1] = nb;
  const float *y = Y + (size_t)s * 8;
  const double A = 0.3 * (double)y[0];
  const double lam = 0.05 * exp((double)y[1] * log(100.0));
  const double nu = 0.1 * exp((double)y[2] * log(500.0));
  const double phi = atan2((double)y[4], (double)y[3]);
  bool good = true;
  for (int k = 0; k < 5; ++k) good = good && isfinite(y[k]);
  good = good && A >= 0.01 && A <= 1.0 && lam >= 0.005 && lam <= 50.0 && nu >= 0.02 && nu <= 250.0;
  if (good) {
    o[2] = A;
    o[3] = lam;
    o[4] = nu;
    o[5] = phi;
  } else {
    o[2] = 0.175;
    o[3] = 0.5;
    o[4] = sqrt(5.0);
    o[5] = 0.0;
  }
  ok[s] = good ? 1 : 0;
}

// K ranges of a GEMM: enough workgroups to fill the chip (about two per
// CU), each range at least four K steps.
int gemm_splits(int M, int N, int K) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  const int by_fill = std::max(1, 512 / tiles);
  const int by_len = std::max(1, K / (4 * kTileK));
  return std::min(by_fill, by_len);
}

// C = A B with the epilogue g.epi; ws: FP32 workspace of ws_floats floats
// for the partial tiles of the K ranges (fewer ranges when it is short).
hipError_t gemm(const GemmArgs &g, float *ws, size_t ws_floats, hipStream_t s) {
  const size_t mn_sz = (size_t)g.M * g.N;
  const int n_split = (int)std::min<size_t>(gemm_splits(g.M, g.N, g.K), std::max<size_t>(1, ws_floats / mn_sz));
  const int kps = (g.K + n_split * kTileK - 1) / (n_split * kTileK) * kTileK;
  const int nz = (g.K + kps - 1) / kps;
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, nz), block(256);
  float *part = nz > 1 ? ws : nullptr;
  const bool akc = g.sAk == 1, bkc = g.sBk == 1;
  if (akc && bkc)
    hipLaunchKernelGGL((gemm_kernel<true, true>), grid, block, 0, s, g, kps, part);
  else if (akc)
    hipLaunchKernelGGL((gemm_kernel<true, false>), grid, block, 0, s, g, kps, part);
  else if (bkc)
    hipLaunchKernelGGL((gemm_kernel<false, true>), grid, block, 0, s, g, kps, part);
  else
    hipLaunchKernelGGL((gemm_kernel<false, false>), grid, block, 0, s, g, kps, part);
  if (nz > 1) {
    const long long mn = (long long)g.M * g.N;
    hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s, g, part, nz);
  }
  return hipGetLastError();
}

// Largest workspace any GEMM of a batch of B needs (floats).
size_t gemm_ws_floats(int B) {
  size_t w = 0;
  for (int l = 0; l < kSeedLayers; ++l) {
    const int K = kDims[l], N = kDims[l + 1];
    w = std::max(w, (size_t)gemm_splits(B, N, K) * B * N);  // forward
    w = std::max(w, (size_t)gemm_splits(N, K, B) * N * K);  // weight gradient
    w = std::max(w, (size_t)gemm_splits(B, K, N) * B * K);  // input gradient
  }
  return w;
}

}  // namespace

// ============================================================ host side

namespace mu {

size_t seeder_param_count() {
  size_t n = 0;
  for (int l = 0; l < kSeedLayers; ++l) n += (size_t)kDims[l] * kDims[l + 1] + kDims[l + 1];
  return n;
}

}  // namespace mu

struct mu_seeder {
  mu_ctx *ctx = nullptr;
  size_t n_params = 0, n_w = 0;
  size_t off_w[kSeedLayers], off_b[kSeedLayers], off_wbf[kSeedLayers];
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  unsigned short *wbf = nullptr;
  long long step = 0;
  int cap = 0;  // batch capacity of the activation buffers
  int fwd_B = 0, bwd_B = 0;  // batch of the last forward / backward pass (their buffers hold it)
  unsigned short *X[kSeedLayers] = {};   // BF16 input of each layer [cap][K_l]
  float *Z[kSeedLayers] = {};            // FP32 pre-activation / output [cap][N_l]
  float *dZ[kSeedLayers] = {};
  unsigned short *G[kSeedLayers] = {};   // BF16 dZ
  float *T = nullptr, *loss = nullptr, *counts = nullptr;
  double *partial = nullptr, *theta = nullptr, *scale = nullptr, *mf = nullptr, *ml = nullptr;
  double *start = nullptr;
  unsigned char *ok = nullptr;
  const float **srcs = nullptr;
  float *ws = nullptr;  // GEMM partial tiles of split K ranges
  size_t ws_floats = 0;
  float *bpart = nullptr;  // bias gradients' row-slice sums
  void free_acts();
  void free_all();
  mu_status ensure(int B);
};

void mu_seeder::free_acts() {
  for (int l = 0; l < kSeedLayers; ++l) {
    (void)hipFree(X[l]);
    (void)hipFree(Z[l]);
    (void)hipFree(dZ[l]);
    (void)hipFree(G[l]);
    X[l] = nullptr;
    Z[l] = dZ[l] = nullptr;
    G[l] = nullptr;
  }
  (void)hipFree(T);
  (void)hipFree(loss);
  (void)hipFree(counts);
  (void)hipFree(partial);
  (void)hipFree(theta);
  (void)hipFree(scale);
  (void)hipFree(mf);
  (void)hipFree(ml);
  (void)hipFree(start);
  (void)hipFree(ok);
  (void)hipFree(srcs);
  (void)hipFree(ws);
  (void)hipFree(bpart);
  ws = nullptr;
  bpart = nullptr;
  ws_floats = 0;
  T = loss = counts = nullptr;
  partial = theta = scale = mf = ml = start = nullptr;
  ok = nullptr;
  srcs = nullptr;
  cap = 0;
}

void mu_seeder::free_all() {
  free_acts();
  (void)hipFree(params);
  (void)hipFree(grads);
  (void)hipFree(m);
  (void)hipFree(v);
  (void)hipFree(wbf);
  params = grads = m = v = nullptr;
  wbf = nullptr;
}

mu_status mu_seeder::ensure(int B) {
  if (B <= cap) return MU_OK;
  (void)hipStreamSynchronize(ctx->stream);
  free_acts();
  hipError_t e = hipSuccess;
  auto al = [&](void **p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 256));
  };
  for (int l = 0; l < kSeedLayers; ++l) {
    al((void **)&X[l], (size_t)B * kDims[l] * 2);
    al((void **)&Z[l], (size_t)B * kDims[l + 1] * 4);
    al((void **)&dZ[l], (size_t)B * kDims[l + 1] * 4);
    al((void **)&G[l], (size_t)B * kDims[l + 1] * 2);
  }
  al((void **)&T, (size_t)B * 8 * 4);
  al((void **)&loss, 4);
  al((void **)&counts, (size_t)B * kCoarse * 4);
  al((void **)&partial, (size_t)((B * 8 + 255) / 256) * 8);
  al((void **)&theta, (size_t)B * 6 * 8);
  al((void **)&scale, (size_t)B * 8);
  al((void **)&mf, (size_t)B * 8);
  al((void **)&ml, (size_t)B * 8);
  al((void **)&start, (size_t)B * 6 * 8);
  al((void **)&ok, (size_t)B);
  al((void **)&srcs, (size_t)B * sizeof(void *));
  const size_t wsf = gemm_ws_floats(B);
  al((void **)&ws, wsf * 4);
  al((void **)&bpart, (size_t)((B + kBiasRows - 1) / kBiasRows) * (kDims[1] + kDims[2] + kDims[3] + kDims[4]) * 4);
  if (e != hipSuccess) {
    free_acts();
    set_err(ctx, "seeder activation buffers for a batch of %d: %s", B, hipGetErrorString(e));
    return MU_E_NOMEM;
  }
  cap = B;
  ws_floats = wsf;
  return MU_OK;
}

namespace {

hipError_t refresh_bf16(mu_seeder *S) {
  for (int l = 0; l < kSeedLayers; ++l) {
    const long long n = (long long)kDims[l] * kDims[l + 1];
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, S->ctx->stream,
                       S->params + S->off_w[l], S->wbf + S->off_wbf[l], n);
  }
  return hipGetLastError();
}

// Forward pass on S->X[0] for B samples; output in S->Z[last].
hipError_t forward(mu_seeder *S, int B) {
  hipError_t e = hipSuccess;
  S->fwd_B = B;
  S->bwd_B = 0;
  for (int l = 0; l < kSeedLayers && e == hipSuccess; ++l) {
    GemmArgs g;
    std::memset(&g, 0, sizeof g);
    const int K = kDims[l], N = kDims[l + 1];
    g.A = S->X[l];
    g.sAi = K;
    g.sAk = 1;
    g.B = S->wbf + S->off_wbf[l];  // B(k, j) = W[j][k]
    g.sBk = 1;
    g.sBj = K;
    g.M = B;
    g.N = N;
    g.K = K;
    g.C = S->Z[l];
    g.bias = S->params + S->off_b[l];
    if (l < kSeedLayers - 1) {
      g.epi = kEpiBiasRelu;
      g.Cbf = S->X[l + 1];
    } else {
      g.epi = kEpiBias;
    }
    e = gemm(g, S->ws, S->ws_floats, S->ctx->stream);
  }
  return e;
}

// Loss and gradients into S->grads for inputs S->X[0] and targets S->T.
hipError_t backward(mu_seeder *S, int B) {
  hipStream_t st = S->ctx->stream;
  S->bwd_B = B;
  const int L = kSeedLayers;
  const int nb = (B * 8 + 255) / 256;
  hipLaunchKernelGGL(loss_kernel, dim3(nb), dim3(256), 0, st, S->Z[L - 1], S->T, B, S->dZ[L - 1], S->G[L - 1],
                     S->partial);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(1), 0, st, S->partial, nb, B, S->loss);
  hipError_t e = hipGetLastError();
  for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
    const int K = kDims[l], N = kDims[l + 1];
    // dW[n][k] = sum_b G[b][n] X[b][k]
    GemmArgs g;
    std::memset(&g, 0, sizeof g);
    g.A = S->G[l];
    g.sAi = 1;
    g.sAk = N;
    g.B = S->X[l];
    g.sBk = K;
    g.sBj = 1;
    g.M = N;
    g.N = K;
    g.K = B;
    g.epi = kEpiStore;
    g.C = S->grads + S->off_w[l];
    if ((e = gemm(g, S->ws, S->ws_floats, st)) != hipSuccess) break;
    if (l > 0) {
      // dX[b][k] = sum_n G[b][n] W[n][k], masked by the previous layer's ReLU
      GemmArgs d;
      std::memset(&d, 0, sizeof d);
      d.A = S->G[l];
      d.sAi = N;
      d.sAk = 1;
      d.B = S->wbf + S->off_wbf[l];
      d.sBk = K;
      d.sBj = 1;
      d.M = B;
      d.N = K;
      d.K = N;
      d.epi = kEpiReluGrad;
      d.C = S->dZ[l - 1];
      d.Cbf = S->G[l - 1];
      d.Zprev = S->Z[l - 1];
      e = gemm(d, S->ws, S->ws_floats, st);
    }
    if (e == hipSuccess) e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  // bias gradients of all layers
  BiasAll ba;
  ba.col0[0] = 0;
  for (int l = 0; l < L; ++l) {
    ba.dZ[l] = S->dZ[l];
    ba.db[l] = S->grads + S->off_b[l];
    ba.N[l] = kDims[l + 1];
    ba.col0[l + 1] = ba.col0[l] + kDims[l + 1];
  }
  const int n_slices = (B + kBiasRows - 1) / kBiasRows, tot = ba.col0[L];
  hipLaunchKernelGGL(bias_grad_all_kernel, dim3((tot + 63) / 64, n_slices), dim3(256), 0, st, ba, B, S->bpart);
  hipLaunchKernelGGL(bias_grad_all_final_kernel, dim3((tot + 255) / 256), dim3(256), 0, st, ba, S->bpart, n_slices);
  return hipGetLastError();
}

hipError_t adam_step(mu_seeder *S, float lr) {
  S->step++;
  const double b1 = 0.9, b2 = 0.999;
  const float eps = 1e-8f;
  const float c1 = (float)(1.0 - std::pow(b1, (double)S->step));
  const float c2 = (float)(1.0 - std::pow(b2, (double)S->step));
  const long long n = (long long)S->n_params;
  WeightMap wm;
  for (int l = 0; l < kSeedLayers; ++l) {
    wm.off_w[l] = (long long)S->off_w[l];
    wm.off_wbf[l] = (long long)S->off_wbf[l];
    wm.size[l] = (long long)kDims[l] * kDims[l + 1];
  }
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, S->ctx->stream, S->params,
                     S->grads, S->m, S->v, n, lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), eps,
                     c1, c2, wm, S->wbf);
  return hipGetLastError();
}

mu_status copy_in(mu_ctx *ctx, void *dst, const void *src, size_t bytes, unsigned mem) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, mem == MU_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                                ctx->stream);
  if (e == hipSuccess && mem == MU_MEM_HOST) e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? MU_OK : hip_fail(ctx, e, "copy in");
}

mu_status copy_out(mu_ctx *ctx, void *dst, const void *src, size_t bytes, unsigned mem) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, mem == MU_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                                ctx->stream);
  if (e == hipSuccess && mem == MU_MEM_HOST) e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? MU_OK : hip_fail(ctx, e, "copy out");
}

bool mem_ok(unsigned mem) { return mem == MU_MEM_HOST || mem == MU_MEM_DEVICE; }

}  // namespace

// ------------------------------------------------------------------- ABI

extern "C" int64_t mu_seeder_param_count(void) { return (int64_t)seeder_param_count(); }

extern "C" mu_status mu_seeder_create(mu_ctx *ctx, const float *init_params, mu_seeder **out) {
  if (!ctx || !out || !init_params) return MU_E_ARG;
  *out = nullptr;
  const size_t n = seeder_param_count();
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(init_params[i])) {
      set_err(ctx, "initial seeder parameter %zu is not finite", i);
      return MU_E_ARG;
    }
  (void)hipSetDevice(ctx->device);
  mu_seeder *S = new mu_seeder();
  S->ctx = ctx;
  S->n_params = n;
  size_t o = 0, ob = 0;
  for (int l = 0; l < kSeedLayers; ++l) {
    S->off_w[l] = o;
    o += (size_t)kDims[l] * kDims[l + 1];
    S->off_b[l] = o;
    o += kDims[l + 1];
    S->off_wbf[l] = ob;
    ob += (size_t)kDims[l] * kDims[l + 1];
  }
  S->n_w = ob;
  hipError_t e = hipMalloc(&S->params, n * 4);
  if (e == hipSuccess) e = hipMalloc(&S->grads, n * 4);
  if (e == hipSuccess) e = hipMalloc(&S->m, n * 4);
  if (e == hipSuccess) e = hipMalloc(&S->v, n * 4);
  if (e == hipSuccess) e = hipMalloc(&S->wbf, ob * 2);
  if (e == hipSuccess) e = hipMemcpy(S->params, init_params, n * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(S->m, 0, n * 4);
  if (e == hipSuccess) e = hipMemset(S->v, 0, n * 4);
  if (e == hipSuccess) e = refresh_bf16(S);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    S->free_all();
    delete S;
    return hip_fail(ctx, e, "seeder allocation");
  }
  ctx->children++;
  *out = S;
  return MU_OK;
}

extern "C" mu_status mu_seeder_destroy(mu_seeder *S) {
  if (!S) return MU_E_ARG;
  (void)hipSetDevice(S->ctx->device);
  (void)hipStreamSynchronize(S->ctx->stream);
  S->free_all();
  S->ctx->children--;
  delete S;
  return MU_OK;
}

extern "C" mu_status mu_seeder_get_params(const mu_seeder *S, float *out) {
  if (!S || !out) return MU_E_ARG;
  hipError_t e = hipStreamSynchronize(S->ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(out, S->params, S->n_params * 4, hipMemcpyDeviceToHost);
  return e == hipSuccess ? MU_OK : MU_E_DEVICE;
}

extern "C" mu_status mu_seeder_get_grads(const mu_seeder *S, float *out) {
  if (!S || !out) return MU_E_ARG;
  hipError_t e = hipStreamSynchronize(S->ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(out, S->grads, S->n_params * 4, hipMemcpyDeviceToHost);
  return e == hipSuccess ? MU_OK : MU_E_DEVICE;
}

extern "C" int64_t mu_seeder_steps(const mu_seeder *S) { return S ? S->step : -1; }

extern "C" mu_status mu_gen_histos(mu_ctx *ctx, uint64_t seed, uint64_t first, int32_t n, int32_t fine,
                                   unsigned mem, float *counts, double *theta, double *mu) {
  if (!ctx || n < 1 || !mem_ok(mem) || (!counts && !theta && !mu)) {
    if (ctx) set_err(ctx, "mu_gen_histos needs n >= 1, a memory kind and at least one output");
    return MU_E_ARG;
  }
  (void)hipSetDevice(ctx->device);
  float *dc = counts;
  double *dt = theta, *dm = mu;
  void *tmp = nullptr;
  const size_t nb = fine ? kFine : kCoarse;
  const size_t bc = counts ? (size_t)n * nb * 4 : 0, bt = theta ? (size_t)n * 48 : 0, bm = mu ? (size_t)n * nb * 8 : 0;
  if (mem == MU_MEM_HOST) {
    hipError_t e = hipMalloc(&tmp, bc + bt + bm + 64);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc(gen)");
    char *p = static_cast<char *>(tmp);
    dm = mu ? reinterpret_cast<double *>(p) : nullptr;
    dt = theta ? reinterpret_cast<double *>(p + bm) : nullptr;
    dc = counts ? reinterpret_cast<float *>(p + bm + bt) : nullptr;
  }
  hipLaunchKernelGGL(gen_kernel, dim3(n), dim3(256), 0, ctx->stream, (unsigned long long)seed,
                     (unsigned long long)first, n, fine ? 1 : 0, dc, dt, (float *)nullptr, dm);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && mem == MU_MEM_HOST) {
    if (counts) e = hipMemcpyAsync(counts, dc, bc, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess && theta) e = hipMemcpyAsync(theta, dt, bt, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess && mu) e = hipMemcpyAsync(mu, dm, bm, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(tmp);
  }
  return e == hipSuccess ? MU_OK : hip_fail(ctx, e, "generator");
}

extern "C" mu_status mu_seeder_forward(mu_ctx *ctx, mu_seeder *S, const uint16_t *x_bf16, int32_t B, unsigned mem,
                                       float *y) {
  if (!ctx || !S || !x_bf16 || !y || B < 1 || !mem_ok(mem) || S->ctx != ctx) return MU_E_ARG;
  (void)hipSetDevice(ctx->device);
  mu_status st = S->ensure(B);
  if (st != MU_OK) return st;
  if ((st = copy_in(ctx, S->X[0], x_bf16, (size_t)B * kCoarse * 2, mem)) != MU_OK) return st;
  hipError_t e = forward(S, B);
  if (e != hipSuccess) return hip_fail(ctx, e, "seeder forward");
  return copy_out(ctx, y, S->Z[kSeedLayers - 1], (size_t)B * 8 * 4, mem);
}

extern "C" mu_status mu_seeder_layer(mu_ctx *ctx, const mu_seeder *S, int32_t layer, int32_t B, uint16_t *x_in,
                                     float *z, float *dz, uint16_t *g) {
  if (!ctx || !S || S->ctx != ctx || layer < 0 || layer >= kSeedLayers || B < 1) return MU_E_ARG;
  if (B > S->fwd_B || ((dz || g) && B > S->bwd_B)) {
    set_err(ctx, "mu_seeder_layer: the last forward (backward) pass held %d (%d) samples", S->fwd_B, S->bwd_B);
    return MU_E_STATE;
  }
  (void)hipSetDevice(ctx->device);
  const size_t K = kDims[layer], N = kDims[layer + 1];
  mu_status st = MU_OK;
  if (x_in) st = copy_out(ctx, x_in, S->X[layer], (size_t)B * K * 2, MU_MEM_HOST);
  if (st == MU_OK && z) st = copy_out(ctx, z, S->Z[layer], (size_t)B * N * 4, MU_MEM_HOST);
  if (st == MU_OK && dz) st = copy_out(ctx, dz, S->dZ[layer], (size_t)B * N * 4, MU_MEM_HOST);
  if (st == MU_OK && g) st = copy_out(ctx, g, S->G[layer], (size_t)B * N * 2, MU_MEM_HOST);
  return st;
}

extern "C" mu_status mu_seeder_train_step(mu_ctx *ctx, mu_seeder *S, const uint16_t *x_bf16, const float *targets,
                                          int32_t B, float lr, int32_t update, unsigned mem, float *loss) {
  if (!ctx || !S || !x_bf16 || !targets || B < 1 || !mem_ok(mem) || S->ctx != ctx || !(lr >= 0.0f)) return MU_E_ARG;
  (void)hipSetDevice(ctx->device);
  mu_status st = S->ensure(B);
  if (st != MU_OK) return st;
  if ((st = copy_in(ctx, S->X[0], x_bf16, (size_t)B * kCoarse * 2, mem)) != MU_OK) return st;
  if ((st = copy_in(ctx, S->T, targets, (size_t)B * 8 * 4, mem)) != MU_OK) return st;
  hipError_t e = forward(S, B);
  if (e == hipSuccess) e = backward(S, B);
  if (e == hipSuccess && update) e = adam_step(S, lr);
  if (e != hipSuccess) return hip_fail(ctx, e, "seeder training step");
  if (loss) return copy_out(ctx, loss, S->loss, 4, mem);
  return MU_OK;
}

extern "C" mu_status mu_seeder_train(mu_ctx *ctx, mu_seeder *S, const mu_seed_train_opts *o, float *loss_curve) {
  if (!ctx || !S || !o || S->ctx != ctx || o->batch < 1 || o->steps < 1 || !(o->lr > 0.0f)) {
    if (ctx) set_err(ctx, "mu_seeder_train needs a seeder, batch >= 1, steps >= 1 and lr > 0");
    return MU_E_ARG;
  }
  (void)hipSetDevice(ctx->device);
  const int B = o->batch;
  mu_status st = S->ensure(B);
  if (st != MU_OK) return st;
  for (int k = 0; k < o->steps; ++k) {
    const unsigned long long first = (unsigned long long)o->first_sample + (unsigned long long)k * B;
    hipLaunchKernelGGL(gen_kernel, dim3(B), dim3(256), 0, ctx->stream, (unsigned long long)o->seed, first, B, 0,
                       S->counts, S->theta, S->T, (double *)nullptr);
    hipLaunchKernelGGL(prep_kernel, dim3(B), dim3(256), 0, ctx->stream, (const uint32_t *const *)nullptr, S->counts, 1,
                       B, S->X[0], S->scale, (double *)nullptr, (double *)nullptr);
    // cosine decay from lr to lr * lr_final_frac
    const double frac = o->steps > 1 ? (double)k / (o->steps - 1) : 0.0;
    const double f = (double)o->lr_final_frac + (1.0 - o->lr_final_frac) * 0.5 * (1.0 + std::cos(M_PI * frac));
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = forward(S, B);
    if (e == hipSuccess) e = backward(S, B);
    if (e == hipSuccess) e = adam_step(S, (float)(o->lr * f));
    if (e == hipSuccess && loss_curve)
      e = hipMemcpyAsync(loss_curve + k, S->loss, 4, hipMemcpyDeviceToHost, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "seeder training");
  }
  hipError_t e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? MU_OK : hip_fail(ctx, e, "seeder training");
}

extern "C" mu_status mu_seed_infer(mu_ctx *ctx, const mu_seeder *Sc, int32_t n, const mu_data *const *data,
                                   double *start_out, uint8_t *ok_out) {
  mu_seeder *S = const_cast<mu_seeder *>(Sc);
  if (!ctx || !S || n < 1 || !data || !start_out || !ok_out || S->ctx != ctx) {
    if (ctx) set_err(ctx, "mu_seed_infer needs a seeder, n >= 1, data, start_out and ok_out");
    return MU_E_ARG;
  }
  std::vector<const uint32_t *> src(n);
  for (int i = 0; i < n; ++i) {
    const mu_data *d = data[i];
    if (!d || d->ctx != ctx || d->n_histo != 1 || d->f64 || d->total != kFine || d->hh[0].first != 0 ||
        std::fabs(d->hh[0].dt - kDtFine) > 1e-12 || d->hh[0].t0_bin != 0.0) {
      set_err(ctx, "dataset %d: the seeder reads one histogram of 8192 integer counts in 0.001 us bins from t = 0",
              i);
      return MU_E_ARG;
    }
    src[i] = static_cast<const uint32_t *>(d->counts);
  }
  (void)hipSetDevice(ctx->device);
  mu_status st = S->ensure(n);
  if (st != MU_OK) return st;
  hipError_t e = hipMemcpyAsync(S->srcs, src.data(), n * sizeof(void *), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(prep_kernel, dim3(n), dim3(256), 0, ctx->stream, (const uint32_t *const *)S->srcs,
                       (const float *)nullptr, kRebin, n,
                       S->X[0], S->scale, S->mf, S->ml);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = forward(S, n);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(decode_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, S->Z[kSeedLayers - 1], S->mf,
                       S->ml, n, S->start, S->ok);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(start_out, S->start, (size_t)n * 48, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(ok_out, S->ok, (size_t)n, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  return e == hipSuccess ? MU_OK : hip_fail(ctx, e, "seeder inference");
}

extern "C" mu_status mu_seeder_save(const mu_seeder *S, const char *path) {
  if (!S || !path) return MU_E_ARG;
  std::vector<float> p(S->n_params), m(S->n_params), v(S->n_params);
  (void)hipStreamSynchronize(S->ctx->stream);
  if (hipMemcpy(p.data(), S->params, S->n_params * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(m.data(), S->m, S->n_params * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(v.data(), S->v, S->n_params * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return MU_E_DEVICE;
  FILE *f = std::fopen(path, "wb");
  if (!f) return MU_E_ARG;
  const char magic[8] = {'M', 'U', 'S', 'E', 'E', 'D', '0', '1'};
  const long long n = (long long)S->n_params;
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&n, 8, 1, f) == 1 && std::fwrite(&S->step, 8, 1, f) == 1 &&
            std::fwrite(p.data(), 4, n, f) == (size_t)n && std::fwrite(m.data(), 4, n, f) == (size_t)n &&
            std::fwrite(v.data(), 4, n, f) == (size_t)n;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? MU_OK : MU_E_ARG;
}

extern "C" mu_status mu_seeder_load(mu_ctx *ctx, const char *path, mu_seeder **out) {
  if (!ctx || !path || !out) return MU_E_ARG;
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) {
    set_err(ctx, "cannot open %s", path);
    return MU_E_ARG;
  }
  char magic[8];
  long long n = 0, step = 0;
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "MUSEED01", 8) == 0 && std::fread(&n, 8, 1, f) == 1 &&
            std::fread(&step, 8, 1, f) == 1 && n == (long long)seeder_param_count();
  std::vector<float> p, m, v;
  if (ok) {
    p.resize(n);
    m.resize(n);
    v.resize(n);
    ok = std::fread(p.data(), 4, n, f) == (size_t)n && std::fread(m.data(), 4, n, f) == (size_t)n &&
         std::fread(v.data(), 4, n, f) == (size_t)n;
  }
  std::fclose(f);
  if (!ok) {
    set_err(ctx, "%s is not a seeder checkpoint of this architecture", path);
    return MU_E_ARG;
  }
  mu_status st = mu_seeder_create(ctx, p.data(), out);
  if (st != MU_OK) return st;
  (*out)->step = step;
  hipError_t e = hipMemcpy((*out)->m, m.data(), n * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy((*out)->v, v.data(), n * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    set_err(ctx, "hipMemcpy(seeder moments): %s", hipGetErrorString(e));
    (void)mu_seeder_destroy(*out);
    *out = nullptr;
    return MU_E_DEVICE;
  }
  return MU_OK;
}
