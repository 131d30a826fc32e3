// Gauss-Newton Hessian of the cost: H_R = sum_n J_n J_n^T per histogram,
// where row J_n holds sqrt(c_n) dN_n/dR_r for the kRS resolved scalars of the
// bin (written by the evaluation kernel's Jacobian mode; c_n = d^2 term /
// dN^2).  This is a dense FP64 contraction over the bins (K = bins, a 32 x 32
// output), done on the matrix cores with v_mfma_f64_16x16x4_f64.
//
// For one MFMA over rows k0 .. k0 + 3, lane l holds x = J[k0 + l/16][c + l%16]
// (c = 0 or 16): as the A operand that is A[i][k] = J[k0 + k][c + i], as the
// B operand B[k][j] = J[k0 + k][c' + j], so A x B accumulates the block
// sum_k J_k[c + i] J_k[c' + j].  Four accumulators give the four 16 x 16
// blocks of the 32 x 32 result.  Rows of a wave are one contiguous range of
// one histogram (a 1 KiB coalesced read per step); a second kernel sums each
// histogram's per-wave blocks in a fixed order with TwoSum, so the result is
// bitwise reproducible.

#include <hip/hip_runtime.h>

#include "mu_internal.h"

namespace mu {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

struct GPair {
  double s, c;
};

__device__ __forceinline__ GPair gpair_add(GPair x, double y) {
  const double s = x.s + y;
  const double bp = s - x.s;
  return GPair{s, x.c + ((x.s - (s - bp)) + (y - bp))};
}

// Units (waves): units[3u .. 3u + 2] = (histogram, first row, end row).
__global__ __launch_bounds__(256) void gram_kernel(const double *J, const int64_t *units, int n_units, double *part) {
  const int u = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + threadIdx.x / 64));
  const int l = threadIdx.x & 63;
  if (u >= n_units) return;
  const int64_t r0 = units[3 * u + 1], r1 = units[3 * u + 2];
  const int kk = l >> 4, c = l & 15;
  d4 a00 = {0.0, 0.0, 0.0, 0.0}, a01 = a00, a10 = a00, a11 = a00;
  int64_t r = r0;
  // two steps per iteration: four row loads in flight
  for (; r + 8 <= r1; r += 8) {
    const double *p0 = J + (r + kk) * kJacCols + c;
    const double *p1 = p0 + 4 * kJacCols;
    const double x0 = p0[0], x1 = p0[16], y0 = p1[0], y1 = p1[16];
    a00 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, x0, a00, 0, 0, 0);
    a01 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, x1, a01, 0, 0, 0);
    a10 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, x0, a10, 0, 0, 0);
    a11 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, x1, a11, 0, 0, 0);
    a00 = __builtin_amdgcn_mfma_f64_16x16x4f64(y0, y0, a00, 0, 0, 0);
    a01 = __builtin_amdgcn_mfma_f64_16x16x4f64(y0, y1, a01, 0, 0, 0);
    a10 = __builtin_amdgcn_mfma_f64_16x16x4f64(y1, y0, a10, 0, 0, 0);
    a11 = __builtin_amdgcn_mfma_f64_16x16x4f64(y1, y1, a11, 0, 0, 0);
  }
  for (; r < r1; r += 4) {  // the rest, rows past r1 read as zero
    const int64_t row = r + kk;
    double x0 = 0.0, x1 = 0.0;
    if (row < r1) {
      x0 = J[row * kJacCols + c];
      x1 = J[row * kJacCols + 16 + c];
    }
    a00 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, x0, a00, 0, 0, 0);
    a01 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, x1, a01, 0, 0, 0);
    a10 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, x0, a10, 0, 0, 0);
    a11 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, x1, a11, 0, 0, 0);
  }
  // part[u][q][v][lane]: block q (00, 01, 10, 11), accumulator element v
  double *o = part + (int64_t)u * 16 * 64 + l;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    o[(0 * 4 + v) * 64] = a00[v];
    o[(1 * 4 + v) * 64] = a01[v];
    o[(2 * 4 + v) * 64] = a10[v];
    o[(3 * 4 + v) * 64] = a11[v];
  }
}

// One workgroup per histogram h: its units are [ufirst[h], ufirst[h + 1]).
// Accumulator element v of lane l in block q is row l / 16 + 4 v, column
// l % 16 of that block (the 16 x 16 f64 MFMA's output layout, as measured
// against the oracle); block q = 2 a + b is rows 16 a .., columns 16 b ..
__global__ __launch_bounds__(256) void gram_merge_kernel(const double *part, const int32_t *ufirst, double *HR) {
  const int h = blockIdx.x;
  const int u0 = ufirst[h], u1 = ufirst[h + 1];
  for (int e = threadIdx.x; e < 16 * 64; e += 256) {
    GPair acc{0.0, 0.0};
    for (int u = u0; u < u1; ++u) acc = gpair_add(acc, part[(int64_t)u * 16 * 64 + e]);
    const int q = e / 256, v = (e / 64) % 4, l = e % 64;
    const int row = 16 * (q >> 1) + (l >> 4) + 4 * v, col = 16 * (q & 1) + (l & 15);
    HR[(int64_t)h * kJacCols * kJacCols + row * kJacCols + col] = acc.s + acc.c;
  }
}

}  // namespace

hipError_t launch_gram(const double *J, const int64_t *units, int n_units, double *part, const int32_t *ufirst,
                       int n_histo, double *HR, hipStream_t s) {
  if (n_units <= 0 || n_histo <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gram_kernel, dim3((n_units + 3) / 4), dim3(256), 0, s, J, units, n_units, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_merge_kernel, dim3(n_histo), dim3(256), 0, s, part, ufirst, HR);
  return hipGetLastError();
}

}  // namespace mu
