// Fused theory-evaluate-and-reduce kernels for gfx950.
//
// The unit of work is one wave (64 lanes; four waves per workgroup share its
// reciprocal table): a range of consecutive fit-range bins, evaluated as the
// (parameter vector, histogram) segments it crosses.  Lane l of a segment reads
// bins l, l + 64, l + 128, ... so that every step of the wave streams 64
// consecutive 32-bit counts (256 B) from memory.
//
// Per bin the lane evaluates the theory program (Listings 2-3), the histogram
// model (Eq. 1) and the cost term (Eq. 2 or Eq. 3); in gradient mode it also
// accumulates r dN/dR for every resolved scalar R (r = d term / dN).
//
// Evaluation by anchored recurrences.  The time grid is uniform, so along one
// lane (time step h = 64 dt) every primitive except the stretched
// exponential obeys an exact multiplicative recurrence:
//   e^(-t/tau), se:  v(t+h) = v(t) e^(-lambda h)                (geometric)
//   sg, stg:         g(t+h) = g(t) q(t),  q(t+h) = q(t) e^(-(sigma h)^2)
//                    with q(t) = e^(-sigma^2 h (t + h/2))       (second order)
//   tf:              (cos, sin)(theta + omega h) = rotation by omega h
//                    (cost and model passes, sin(omega h) >= 1/16: the real
//                    part alone by a three-term recurrence)
// Each lane evaluates the exact values at its first bin (the anchor) and
// re-anchors every `anchor_every` steps; the step constants are uniform and
// computed once per segment.  Rounding drift grows like k eps for the
// geometric and rotation sequences, k min(k, 1/sin(omega h)) eps / 2 for the
// three-term one and k^2 eps / 2 for the Gaussian one, so 256 steps between
// anchors keep every factor within ~4e-12 relative of its directly evaluated
// value.  ge (beta free) is evaluated directly.
//
// Reduction: per lane a plain FP64 sum over one anchor interval (at most 256
// bins), folded into a compensated (TwoSum) pair at every anchor, then
// compensated merges across the wave and across the segments of the job.  Each
// segment writes its own slot; a second, one-workgroup-per-job kernel merges
// the job's slots in a fixed order, so results are bitwise reproducible and
// no atomics or device-scope fences are used.

#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include <cmath>

#include "mu_internal.h"

// Every fused multiply-add below is written out: automatic contraction could
// round the cost pass and the gradient pass differently.
#pragma clang fp contract(off)

namespace mu {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kThird = 1.0 / 3.0;
constexpr double kInvPi = 0.318309886183790671537767526745;  // 1 / pi
constexpr double kTwoThird = 2.0 / 3.0;
constexpr int kSlots = kMaxT * kMaxFT;

struct Pair {
  double s, c;
};
struct D2 {
  double a, b;
};

// Theory shapes.  A fixed shape hard-wires the number of terms, the factors
// of each term and their primitives, so the compiler keeps only the states,
// step constants and accumulators that shape needs; the generic shape reads
// them from the theory program at run time.
// Structure of a theory program held in scalar registers by every wave.
struct TStruct {
  int nt;
  int nf[kMaxT];
  int prim[kMaxT][kMaxFT];
};

struct ShapeGeneric {
  static constexpr bool kFixed = false;
  static constexpr int kTerms = 0;
  static constexpr bool kScalable = false;
  __device__ static int nt(const TStruct &ts) { return ts.nt; }
  __device__ static int nf(const TStruct &ts, int k) { return ts.nf[k]; }
  __device__ static int prim(const TStruct &ts, int k, int f) { return ts.prim[k][f]; }
  __device__ static constexpr bool fold(const TStruct &, int) { return false; }
};

template <int NT, int NF0, int P00, int P01, int NF1, int P10, int P11>
struct ShapeFixed {
  static constexpr bool kFixed = true;
  static constexpr int kTerms = NT;
  // Cost and model passes may fold N0, the lifetime and each term's weight
  // into the state of the term's first factor when that factor follows a
  // linear recurrence (se, sg, tf) or is a lone stg (its constant part then
  // joins the lifetime state); no ge anywhere (ge needs t itself).
  static constexpr bool lead_ok(int p, int nf) {
    return p == MU_SE || p == MU_SG || p == MU_TF || (p == MU_STG && nf == 1);
  }
  static constexpr bool kScalable = lead_ok(P00, NF0) && (NT < 2 || lead_ok(P10, NF1)) && P00 != MU_GE &&
                                    P01 != MU_GE && P10 != MU_GE && P11 != MU_GE;
  __device__ static constexpr int nt(const TStruct &) { return NT; }
  __device__ static constexpr int nf(const TStruct &, int k) { return k == 0 ? NF0 : (k == 1 ? NF1 : 0); }
  __device__ static constexpr int prim(const TStruct &, int k, int f) {
    return k == 0 ? (f == 0 ? P00 : P01) : (f == 0 ? P10 : P11);
  }
  // A scaled term se(lambda) tf(phi, nu) is one complex state: the
  // exponential's step ratio joins the rotation's step and its value the
  // rotation's amplitude, so the term is the state's real part.
  __device__ static constexpr bool fold(const TStruct &, int k) {
    return (k == 0 ? NF0 : NF1) == 2 && (k == 0 ? P00 : P10) == MU_SE && (k == 0 ? P01 : P11) == MU_TF;
  }
};

using ShapeExpCos = ShapeFixed<1, 2, MU_SE, MU_TF, 0, 0, 0>;
using ShapeGaussCos = ShapeFixed<1, 2, MU_SG, MU_TF, 0, 0, 0>;
using ShapeStg = ShapeFixed<1, 1, MU_STG, 0, 0, 0, 0>;
using ShapeExpStg = ShapeFixed<2, 1, MU_SE, 0, 1, MU_STG, 0>;
using ShapeExpCosStg = ShapeFixed<2, 2, MU_SE, MU_TF, 1, MU_STG, 0>;

// Whether a compiled shape has a rotation factor.
template <typename Sh>
constexpr bool shape_has_tf() {
  if constexpr (!Sh::kFixed) {
    return false;
  } else {
    TStruct ts{};
    for (int kt = 0; kt < Sh::nt(ts); ++kt)
      for (int f = 0; f < Sh::nf(ts, kt); ++f)
        if (Sh::prim(ts, kt, f) == MU_TF) return true;
    return false;
  }
}

// Exponentials an anchor of a compiled shape needs: the lifetime, one per
// exponential factor, two per Gaussian factor (state and ratio).
template <typename Sh>
constexpr int anchor_exps() {
  if constexpr (!Sh::kFixed) {
    return 1;
  } else {
    TStruct ts{};
    int n = 1;
    for (int kt = 0; kt < Sh::nt(ts); ++kt)
      for (int f = 0; f < Sh::nf(ts, kt); ++f) {
        const int p = Sh::prim(ts, kt, f);
        n += p == MU_SE ? 1 : (p == MU_SG || p == MU_STG) ? 2 : 0;
      }
    return n;
  }
}


// Knuth's TwoSum applied to two compensated pairs.
__device__ __forceinline__ Pair pair_add(Pair x, Pair y) {
  double s = x.s + y.s;
  double bp = s - x.s;
  double e = (x.s - (s - bp)) + (y.s - bp);
  return Pair{s, x.c + y.c + e};
}

// Value of a compensated pair; an infinite sum keeps its sign (the correction
// term of TwoSum is NaN once the sum overflows to infinity).
__device__ __forceinline__ double pair_value(Pair x) { return isinf(x.s) ? x.s : x.s + x.c; }

__device__ __forceinline__ double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }

// Uniform copy of lane `src`'s value (scalar registers).
__device__ __forceinline__ double bcast(double v, int src) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Partner value through a DPP lane move (VALU, no LDS round trip): CTRL is a
// DPP control of the row (16 lanes): quad_perm [1,0,3,2] (0xB1), quad_perm
// [2,3,0,1] (0x4E), row_half_mirror (0x141), row_mirror (0x140).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Compensated sum over the wave, the same in every lane. Within a row of 16
// lanes: partner lanes 1 apart, then 2 (quad swaps), then the other half of
// the group of 8 (half mirror), then of the row (mirror); after each step all
// lanes of a group hold the same pair. pair_add is symmetric to the bit (the
// sum and the TwoSum error, which is exact, do not depend on the operand
// order; the corrections are added commutatively first), so partners need no
// ordering. The four row results are then combined in a fixed order.
__device__ __forceinline__ Pair wave_pair_sum(Pair p) {
  p = pair_add(p, Pair{dpp_d<0xB1>(p.s), dpp_d<0xB1>(p.c)});
  p = pair_add(p, Pair{dpp_d<0x4E>(p.s), dpp_d<0x4E>(p.c)});
  p = pair_add(p, Pair{dpp_d<0x141>(p.s), dpp_d<0x141>(p.c)});
  p = pair_add(p, Pair{dpp_d<0x140>(p.s), dpp_d<0x140>(p.c)});
  const Pair r0{bcast(p.s, 0), bcast(p.c, 0)}, r1{bcast(p.s, 16), bcast(p.c, 16)};
  const Pair r2{bcast(p.s, 32), bcast(p.c, 32)}, r3{bcast(p.s, 48), bcast(p.c, 48)};
  return pair_add(pair_add(r0, r1), pair_add(r2, r3));
}

// Plain sum over the wave, the same in every lane (addition is commutative,
// so partners agree without ordering).
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return (bcast(v, 0) + bcast(v, 16)) + (bcast(v, 32) + bcast(v, 48));
}


// Wave-uniform copies of values that are the same in every lane (scalar
// registers): for loads the compiler cannot prove uniform, e.g. after the
// workgroup has written memory that might alias them.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ double uni(double v) { return __longlong_as_double(uni((int64_t)__double_as_longlong(v))); }
__device__ __forceinline__ DevHisto uni(DevHisto x) {
  x.off = uni(x.off);
  x.n = uni(x.n);
  x.first = uni(x.first);
  x.t0_bin = uni(x.t0_bin);
  x.dt = uni(x.dt);
  x.map_row = uni(x.map_row);
  return x;
}

// Out-of-line transcendentals: they run at anchors and in the segment
// prologue, and one copy each keeps the kernels small.
__device__ __attribute__((noinline)) double x_exp(double x) { return exp(x); }
// cos and sin of pi x: the phase is reduced in half-cycles, exactly
__device__ __attribute__((noinline)) D2 x_sincospi(double x) {
  D2 r;
  sincospi(x, &r.b, &r.a);  // a = cos, b = sin
  return r;
}
// N exponentials in one call: the evaluations are independent and interleave.
template <int N>
struct DN {
  double v[N];
};
template <int N>
__device__ __attribute__((noinline)) DN<N> x_expn(DN<N> x) {
  DN<N> r;
#pragma unroll
  for (int i = 0; i < N; ++i) r.v[i] = exp(x.v[i]);
  return r;
}
// stretched exponential e^(-(l t)^b) and (l t)^b ln(l t)
__device__ __attribute__((noinline)) D2 x_ge(double lt, double beta) {
  const double xb = pow(lt, beta);
  D2 r;
  r.a = exp(-xb);
  r.b = (lt > 0.0) ? xb * log(lt) : 0.0;
  return r;
}
__device__ __attribute__((noinline)) double x_pow(double x, double y) { return pow(x, y); }

// ------------------------------------------------------------------ resolve

// Resolved scalar of reference r for parameter vector p and map row `row`;
// f_s: the function values, when already formed.
__device__ double resolve_ref(const DevTheory *th, DevRef r, const double *p, int row, const double *f_s) {
  if (r.kind == MU_REF_PAR) return p[th->map[row * th->n_slots + r.slot]];
  if (r.kind == MU_REF_FUN) {
    const int i = th->map[row * th->n_slots + r.slot];
    if (f_s) return f_s[i];
    const double *Fi = th->F + (int64_t)i * th->n_par;
    double s = 0.0;
    for (int k = 0; k < th->n_par; ++k) s = fma(Fi[k], p[k], s);
    return s + th->f0[i];
  }
  if (r.kind == MU_REF_LIT) return r.lit;
  return 0.0;
}

// ----------------------------------------------------- primitive recurrences

__host__ __device__ constexpr int prim_nargs(int kind) { return (kind == MU_GE || kind == MU_TF) ? 2 : 1; }

// Step constant w (0 or 1) of a primitive for the lane step h.
__device__ __forceinline__ double step_const(int kind, int w, double a0, double a1, double h) {
  switch (kind) {
    case MU_SE:
      return w == 0 ? x_exp(-a0 * h) : 0.0;
    case MU_SG:
    case MU_STG: {
      const double x = a0 * h;
      return w == 0 ? x_exp(-(x * x)) : 0.0;
    }
    case MU_TF: {
      const D2 cs = x_sincospi(2.0 * a1 * h);  // angle 2 pi nu h
      return w == 0 ? cs.a : cs.b;
    }
    default:
      return 0.0;
  }
}

// Exact state at time t (anchor).
__device__ __forceinline__ void anchor(int kind, double t, double a0, double a1, double h, double &s0, double &s1) {
  switch (kind) {
    case MU_SE:
      s0 = x_exp(-a0 * t);
      s1 = 0.0;
      break;
    case MU_SG:
    case MU_STG: {
      const double x = a0 * t;
      s0 = x_exp(-0.5 * (x * x));
      s1 = x_exp(-(a0 * a0) * h * (t + 0.5 * h));
      break;
    }
    case MU_TF: {
      // angle 2 pi nu t + phi, in half-cycles
      const D2 cs = x_sincospi(fma(2.0 * a1, t, a0 * kInvPi));
      s0 = cs.a;
      s1 = cs.b;
      break;
    }
    default:
      s0 = s1 = 0.0;
      break;
  }
}

// Advance the state by one lane step.
__device__ __forceinline__ void advance(int kind, double c0, double c1, double &s0, double &s1) {
  switch (kind) {
    case MU_SE:
      s0 *= c0;
      break;
    case MU_SG:
    case MU_STG:
      s0 *= s1;
      s1 *= c0;
      break;
    case MU_TF: {
      const double c = fma(s0, c0, -(s1 * c1));
      const double s = fma(s1, c0, s0 * c1);
      s0 = c;
      s1 = s;
      break;
    }
    default:
      break;
  }
}

// Primitive value at time t from its state.
__device__ __forceinline__ double value(int kind, double t, double a0, double a1, double s0) {
  switch (kind) {
    case MU_GE:
      return x_exp(-x_pow(a0 * t, a1));
    case MU_STG: {
      const double x = a0 * t;
      return fma(kTwoThird * fma(-x, x, 1.0), s0, kThird);
    }
    default:  // se, sg, tf: the state itself
      return s0;
  }
}

// Primitive value and derivatives in its arguments, from its state.
__device__ __forceinline__ double value_grad(int kind, double t, double a0, double a1, double s0, double s1,
                                             double &d0, double &d1) {
  switch (kind) {
    case MU_SE:
      d0 = -t * s0;
      d1 = 0.0;
      return s0;
    case MU_GE: {
      const double x = a0 * t;
      const D2 v = x_ge(x, a1);  // v.a = e^(-x^b), v.b = x^b ln x
      if (x > 0.0) {
        d0 = -a1 * x_pow(x, a1) / a0 * v.a;
        d1 = -v.b * v.a;
      } else {
        d0 = (a1 == 1.0) ? -t : 0.0;
        d1 = 0.0;
      }
      return v.a;
    }
    case MU_SG:
      d0 = -a0 * t * t * s0;
      d1 = 0.0;
      return s0;
    case MU_STG: {
      const double x = a0 * t;
      const double s2 = x * x;
      d0 = kTwoThird * a0 * t * t * (s2 - 3.0) * s0;
      d1 = 0.0;
      return fma(kTwoThird * fma(-x, x, 1.0), s0, kThird);
    }
    default:  // MU_TF: state (cos, sin)
      d0 = -s1;
      d1 = -kTwoPi * t * s1;
      return s0;
  }
}

// Per-bin cost term (Eq. 2 / Eq. 3) and its derivative in N.
// 1/v for normal v whose reciprocal is normal (v >= 1 for the counts,
// 2^-1000 < v < 2^1000 for the likelihood's expected counts): hardware
// reciprocal refined by one Newton step (< 1 ulp + rounding).
__device__ __forceinline__ double recip(double v) {
  double iv = __builtin_amdgcn_rcp(v);
  return fma(iv, fma(-v, iv, 1.0), iv);
}

// 1 / max(d, 1) of an integer count: from the workgroup's table (correctly
// rounded) below kInvTab, else by recip().
// raw = 8 d is the entry's byte offset; x is raw widened.
template <int TAB>
__device__ __forceinline__ double inv_count(uint32_t raw, double x, const double *tab) {
  const char *base = reinterpret_cast<const char *>(tab);
  // the host checked: every count is below kInvTab
  if constexpr (TAB == 1) return *reinterpret_cast<const double *>(base + raw);
  constexpr uint32_t kEnd = (uint32_t)kInvTab * kCountScale;
  double iv = *reinterpret_cast<const double *>(base + min(raw, kEnd - kCountScale));
  // a wave-uniform test, so the rare large counts cost a skipped scalar branch
  if (__builtin_amdgcn_ballot_w64(raw >= kEnd) != 0) {
    asm volatile("");  // keeps the branch: not speculated into every bin
    if (raw >= kEnd) iv = recip(x * kCountUnscale);
  }
  return iv;
}

// Natural logarithm of the likelihood's ratio q = d / N, inline (the
// library's logarithm, in double-double steps, took about 75 of the
// likelihood's 126 instructions per bin). q = m 2^e with m in [sqrt(1/2),
// sqrt(2)); ln m = 2 atanh(s) with s = (m - 1) / (m + 1), |s| <= 0.1716, as
// 2 s + 2 s u P(u), u = s^2, P(u) = sum_{k=0}^{9} u^k / (2k + 3) (the first
// term left out is below 1e-17 of the sum); then e ln 2 with ln 2 split in
// two, the high part of 24 significant bits so that e times it is exact.
// Within about 2 ulp. q = 0, +inf and NaN give -inf, +inf and NaN.
__device__ __forceinline__ double log_ratio(double q) {
  constexpr double kSqrtHalf = 0.70710678118654752440;
  constexpr double kLn2Hi = 0x1.62e42fp-1;          // ln 2 to 24 bits
  constexpr double kLn2Lo = 0x1.df473de6af279p-26;  // ln 2 - kLn2Hi
  int e;
  double m = frexp(q, &e);  // q = m 2^e, m in [1/2, 1)
  const bool low = m < kSqrtHalf;
  m = low ? m + m : m;
  e = low ? e - 1 : e;
  const double f = m - 1.0;  // exact
  const double sv = f * recip(2.0 + f);
  const double u = sv * sv;
  double P = 1.0 / 21.0;
  P = fma(P, u, 1.0 / 19.0);
  P = fma(P, u, 1.0 / 17.0);
  P = fma(P, u, 1.0 / 15.0);
  P = fma(P, u, 1.0 / 13.0);
  P = fma(P, u, 1.0 / 11.0);
  P = fma(P, u, 1.0 / 9.0);
  P = fma(P, u, 1.0 / 7.0);
  P = fma(P, u, 1.0 / 5.0);
  P = fma(P, u, 1.0 / 3.0);
  const double ts = sv + sv;
  const double ed = (double)e;
  const double r = fma(ed, kLn2Hi, fma(ed, kLn2Lo, fma(ts * u, P, ts)));
  return q == 0.0 ? -INFINITY : (q == INFINITY ? q : r);
}

// Per-bin cost term (Eq. 2 / Eq. 3) and its derivative in N. For chi^2 on
// integer counts the caller passes iv = 1 / max(d, 1); otherwise it is
// computed here.
template <int COST, bool WANT_DN, bool INT_DATA>
__device__ __forceinline__ double cost_term(double d, double N, double iv_int, double &dN) {
  if (COST == MU_COST_CHI2) {
    // variance d, or 1 for an empty bin
    const double iv = INT_DATA ? iv_int : recip(d > 0.0 ? d : 1.0);
    const double diff = d - N;
    if (WANT_DN) dN = -2.0 * diff * iv;
    return diff * diff * iv;
  } else {
    if (d > 0.0) {
      // q = d / N as d times the refined hardware reciprocal (within about
      // 2 ulp; the division's scaling and fix-up steps cost twice as many
      // instructions). A wave-uniform test sends waves with any N outside
      // [2^-1000, 2^1000], or not positive, to the division, which handles
      // every range.
      double q;
      if (__builtin_amdgcn_ballot_w64(!(N > 0x1p-1000 && N < 0x1p1000)) == 0)
        q = d * recip(N);
      else
        q = d / N;
      if (WANT_DN) dN = 2.0 * (1.0 - q);
      if (!(N > 0.0)) return (N <= 0.0) ? INFINITY : N;  // NaN stays NaN
      return 2.0 * ((N - d) + d * log_ratio(q));
    }
    if (WANT_DN) dN = 2.0;
    return 2.0 * N;
  }
}

// acc + the bin's cost term; chi^2 as acc + (d - N) ((d - N) / v) in one
// fused step. x is the stored count widened (8 d for integer storage), so
// d - N is one fused step too.
template <int COST, bool INT_DATA>
__device__ __forceinline__ double cost_add(double acc, double x, double N, double iv_int) {
  if (COST == MU_COST_CHI2) {
    const double diff = INT_DATA ? fma(x, kCountUnscale, -N) : x - N;
    const double iv = INT_DATA ? iv_int : recip(x > 0.0 ? x : 1.0);
    return fma(diff, diff * iv, acc);
  }
  double dN;
  return acc + cost_term<COST, false, INT_DATA>(INT_DATA ? x * kCountUnscale : x, N, iv_int, dN);
}

// ------------------------------------------------------------ merge kernel

// Compensated sum of slot component `c` over tiles k0, k0 + step, ... < k1:
// kU independent loads in flight, lanes of the kU-wide stripe combined in a
// fixed order.
__device__ Pair sum_slots(const double *P, int k0, int k1, int step, int c) {
  constexpr int kU = 8;
  Pair acc[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) acc[u] = Pair{0.0, 0.0};
  int k = k0;
  for (; k + (kU - 1) * step < k1; k += kU * step) {
    double v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = P[(int64_t)(k + u * step) * kSlot + c];
#pragma unroll
    for (int u = 0; u < kU; ++u) acc[u] = pair_add(acc[u], Pair{v[u], 0.0});
  }
  // the rest (fewer than kU): loads first, then the sums
  double v[kU - 1];
#pragma unroll
  for (int u = 0; u < kU - 1; ++u) v[u] = k + u * step < k1 ? P[(int64_t)(k + u * step) * kSlot + c] : 0.0;
#pragma unroll
  for (int u = 0; u < kU - 1; ++u) acc[u] = pair_add(acc[u], Pair{v[u], 0.0});
  Pair t = acc[0];
#pragma unroll
  for (int u = 1; u < kU; ++u) t = pair_add(t, acc[u]);
  return t;
}

// Same for the cost pairs (s, c) of tiles [k0, k1).
__device__ double sum_slot_pairs(const double *P, int k0, int k1) {
  Pair acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = Pair{0.0, 0.0};
  int k = k0;
  for (; k + 8 <= k1; k += 8) {
    Pair v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = Pair{P[(int64_t)(k + u) * kSlot], P[(int64_t)(k + u) * kSlot + 1]};
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = pair_add(acc[u], v[u]);
  }
  // the rest (fewer than 8), slot k + u into acc[u]: unrolled, so the
  // accumulators stay in registers
#pragma unroll
  for (int u = 0; u < 7; ++u)
    if (k + u < k1) acc[u] = pair_add(acc[u], Pair{P[(int64_t)(k + u) * kSlot], P[(int64_t)(k + u) * kSlot + 1]});
  Pair t = acc[0];
#pragma unroll
  for (int u = 1; u < 8; ++u) t = pair_add(t, acc[u]);
  return pair_value(t);
}

// Merge the slots of job J in a fixed order and write its outputs. Segment
// (unit u, histogram j of the launch's enumeration) owns slot u + j, so the
// slots of one histogram are a contiguous range, and the span of a job's
// histograms holds no undefined slot.
struct SlotMap {
  const double *P;
  const DevJob *J;
  int64_t W, vbase;  // bins per unit, first bin of the job in its launch
  int jbase;         // the job's first histogram in its launch's enumeration
  __device__ void range(int h, int &k0, int &k1) const {
    const int64_t s = vbase + J->histos[h].off;
    k0 = (int)(jbase + h + s / W);
    k1 = (int)(jbase + h + (s + J->histos[h].n - 1) / W) + 1;
  }
  __device__ void span(int &k0, int &k1) const {
    int t;
    range(0, k0, t);
    range(J->n_histo - 1, t, k1);
  }
};

template <int MODE, int NT>
__device__ void merge_job(const LaunchArgs &a, const DevJob &J, int job) {
  // Phase A issues every load that depends on nothing else (the slot span,
  // the plan's header and active scalars, the first chunk's histogram
  // records); phase B issues the cost slots, the first chunk's gradient slots
  // and its plan block together. Later histogram chunks add two rounds each.
  constexpr int HC = kMergeChunk;
  constexpr int kWaves = NT / 64;
  // threads of phase A's independent loads: spread over the waves when there
  // are several
  constexpr int kTSpan = NT >= 256 ? 64 : 1, kTAct = NT >= 256 ? 128 : 2, kTHdr = NT >= 256 ? 192 : 2 + kRS;
  constexpr bool G = MODE == kModeGrad;
  __shared__ Pair red[kWaves];
  __shared__ int span_s[2];
  __shared__ int rk0[HC], rk1[HC];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  SlotMap sm;
  sm.J = &J;
  if (a.jobs == nullptr) {
    sm.W = a.split_w;
    sm.P = a.partial;
    sm.vbase = (int64_t)job * a.total;
    sm.jbase = job * J.n_histo;
  } else {
    sm.W = J.split_w;
    sm.P = a.partial + (int64_t)J.slot_base * kSlot;
    sm.vbase = J.goff;
    sm.jbase = J.jbase;
  }
  const double *P = sm.P;
  const DevTheory *th = J.th;
  const int n_par = G ? th->n_par : 0;
  const bool need_chunks = G || J.histo_out != nullptr;

  // chain rule through the map / function array (gradient mode):
  //   g_k = sum_h sum_r gR[h][r] dR_r/dp_k, each gR[h][r] a sum over h's slots.
  // Per chunk of histograms the plan gives each entry e = (hh, i) its place:
  // in parameter k's contiguous run of srt (runs in koff, entries in entry
  // order within a run), or in the list of function entries fsrt (entry
  // order). Each parameter then sums its run and the function entries in that
  // fixed order, whatever the timing.
  // The gradient mode's arrays live in the launch's dynamic LDS, sized by the
  // host from the launch's plans (merge_lds_bytes): acc_s and acc_c [n_par],
  // then srt and fsrt [min(n_histo, HC) na], then pl [plan stride]. Small
  // jobs then leave room for many workgroups per CU.
  __shared__ int act[kRS], hdr[3];
  extern __shared__ __align__(16) double merge_dyn[];
  double *acc_s = merge_dyn, *acc_c = merge_dyn + n_par;
  double *srt = nullptr, *fsrt = nullptr;
  int *pl = nullptr;

  auto stage_ranges = [&](int h0) {
    const int nh = min(HC, J.n_histo - h0);
    for (int hh = tid; hh < nh; hh += NT) {
      int k0, k1;
      sm.range(h0 + hh, k0, k1);
      rk0[hh] = k0;
      rk1[hh] = k1;
    }
  };
  // per-histogram costs, the chunk's plan block and its gradient entries
  auto chunk_entries = [&](int h0) {
    const int nh = min(HC, J.n_histo - h0);
    if (J.histo_out)
      for (int hh = tid; hh < nh; hh += NT) J.histo_out[h0 + hh] = sum_slot_pairs(P, rk0[hh], rk1[hh]);
    if constexpr (G) {
      const int na = hdr[0], stride = hdr[2];
      const int32_t *blk = J.plan + kPlanHead + (int64_t)(h0 / HC) * stride;
      for (int q = tid; q < stride; q += NT) pl[q] = blk[q];
      const int32_t *dst = blk + 3 + n_par;
      // S adjacent lanes per entry (up to 8, while the entries fill the
      // workgroup) take its slots in turn; a fixed butterfly combines them
      const int ne = nh * na;
      int S = 1;
      while (S < 8 && ne * S * 2 <= NT) S <<= 1;
      for (int base = 0; base < ne * S; base += NT) {  // uniform: every lane reaches the shuffles
        const int t = base + tid, e = t / S, sl = t % S;
        const bool on = t < ne * S;
        Pair v{0.0, 0.0};
        int at = 0;
        if (on) {
          const int hh = e / na, i = e - hh * na;
          at = dst[e];
          v = sum_slots(P, rk0[hh] + sl, rk1[hh], S, 2 + act[i]);
        }
        for (int o = 1; o < S; o <<= 1) v = pair_add(v, Pair{__shfl_xor(v.s, o, 64), __shfl_xor(v.c, o, 64)});
        if (on && sl == 0) {
          if (at >= 0)
            srt[at] = pair_value(v);
          else
            fsrt[-1 - at] = pair_value(v);
        }
      }
    }
  };
  auto chunk_gather = [&](int h0) {
    if constexpr (G) {
      const int ne = min(HC, J.n_histo - h0) * hdr[0], n_fe = pl[1];
      const int *koff = pl + 2, *fi = pl + 3 + n_par + ne;
      for (int k = tid; k < n_par; k += NT) {
        Pair q{acc_s[k], acc_c[k]};
        for (int j = koff[k]; j < koff[k + 1]; ++j) q = pair_add(q, Pair{srt[j], 0.0});
        for (int f = 0; f < n_fe; ++f) q = pair_add(q, Pair{fsrt[f] * th->F[(int64_t)fi[f] * n_par + k], 0.0});
        acc_s[k] = q.s;
        acc_c[k] = q.c;
      }
    }
  };

  // ---- phase A
  if (tid == 0) {
    int k0, k1;
    sm.range(0, k0, k1);
    span_s[0] = k0;
  }
  if (tid == kTSpan) {
    int k0, k1;
    sm.range(J.n_histo - 1, k0, k1);
    span_s[1] = k1;
  }
  if constexpr (G) {
    if (tid >= kTAct && tid < kTAct + kRS) act[tid - kTAct] = J.plan[kPlanAct + tid - kTAct];
    if (tid >= kTHdr && tid < kTHdr + 3) hdr[tid - kTHdr] = J.plan[tid - kTHdr];
    for (int k = tid; k < n_par; k += NT) {
      acc_s[k] = 0.0;
      acc_c[k] = 0.0;
    }
  }
  if (need_chunks) stage_ranges(0);
  __syncthreads();
  if constexpr (G) {
    const int ne_max = min(J.n_histo, HC) * hdr[0];
    srt = acc_c + n_par;
    fsrt = srt + ne_max;
    pl = reinterpret_cast<int *>(fsrt + ne_max);
  }

  // ---- phase B: total cost (strided fixed assignment of slots to threads,
  // then a tree) and the first chunk
  Pair acc{0.0, 0.0};
  for (int k = span_s[0] + tid; k < span_s[1]; k += NT)
    acc = pair_add(acc, Pair{P[(int64_t)k * kSlot], P[(int64_t)k * kSlot + 1]});
  if (need_chunks) chunk_entries(0);
  acc = wave_pair_sum(acc);
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (tid == 0) {
    Pair t = red[0];
    for (int w = 1; w < kWaves; ++w) t = pair_add(t, red[w]);
    J.cost_out[0] = pair_value(t);
  }
  if (!need_chunks) return;
  chunk_gather(0);
  for (int h0 = HC; h0 < J.n_histo; h0 += HC) {
    __syncthreads();  // the previous chunk's entries are consumed
    stage_ranges(h0);
    __syncthreads();
    chunk_entries(h0);
    __syncthreads();
    chunk_gather(h0);
  }
  if constexpr (G) {
    __syncthreads();
    for (int k = tid; k < n_par; k += NT) J.grad_out[k] = pair_value(Pair{acc_s[k], acc_c[k]});
  }
}

// ------------------------------------------------------------------- kernel

// What one segment needs: bins [begin, begin + n) of one histogram's fit
// range (first bin `first` of the histogram, counts from `off` in the
// concatenated counts), evaluated for the parameter vector p; the wave's
// cost (and gradient) partials go to its slot.
struct SegIn {
  const double *inv_tab;  // chi^2 on integer counts: 1 / max(d, 1) for d < kInvTab (LDS)
  const DevTheory *th;
  const double *p;
  const void *counts;
  double *model_out;
  int64_t off, first, begin;
  double t0_bin, dt;
  int32_t map_row, n, anchor_every;
};

// One segment (see SegIn).
template <int COST, int MODE, typename CT, typename Sh, int TAB, int PF = kPrefetch>
__device__ __forceinline__ void eval_segment(const SegIn &S, double *slot) {
  const int tid = threadIdx.x;
  const DevTheory *th = S.th;
  const int row = S.map_row;
  TStruct ts;
  if constexpr (!Sh::kFixed) {
    ts.nt = __builtin_amdgcn_readfirstlane(th->n_terms);
#pragma unroll
    for (int k = 0; k < kMaxT; ++k) {
      ts.nf[k] = __builtin_amdgcn_readfirstlane(th->nf[k]);
#pragma unroll
      for (int f = 0; f < kMaxFT; ++f) ts.prim[k][f] = __builtin_amdgcn_readfirstlane(th->prim[k][f]);
    }
  }
  const int n_terms = Sh::nt(ts);
  const double neg_inv_tau = bcast(th->neg_inv_tau, 0);
  double coef[kMaxT];
#pragma unroll
  for (int k = 0; k < kMaxT; ++k) coef[k] = k < n_terms ? bcast(th->coef[k], 0) : 0.0;

  // Opaque to the optimiser: the lane masks of the lane-parallel prologue are
  // then formed in each segment rather than hoisted out of the segment loop,
  // where they stayed live across it in spilled scalar registers.
  int lane = tid & 63;
  asm volatile("" : "+v"(lane));
  // one LDS word per lane: the wave's function values in the prologue, then
  // the lane's compensation term
  static_assert(kFunStage <= kWave, "function stage within the wave's words");
  __shared__ double f_stage[kBlock / kWave][kWave];
  double *f_lane = &f_stage[tid / kWave][tid & (kWave - 1)];
  // resolved scalars of this (vector, histogram): lane r of every wave
  // resolves scalar r, then each is broadcast to scalar registers
  double R[kRS];
  {
    // the theory's functions f = F p + f0 (Sec. 4.2.1), once per segment: the
    // wave forms each dot product lane-parallel with a fixed-order sum and
    // shares them through its LDS row (a serial loop per scalar would wait on
    // n_par loads)
    double *f_s = f_stage[tid / kWave];  // this wave's copy
    const int n_fun = __builtin_amdgcn_readfirstlane(th->n_fun);
    const bool f_staged = n_fun > 0 && n_fun <= kFunStage;
    if (f_staged) {
      const int n_par = th->n_par;
      for (int i = 0; i < n_fun; ++i) {
        double acc = 0.0;
        for (int k = lane; k < n_par; k += kWave) acc = fma(th->F[(int64_t)i * n_par + k], S.p[k], acc);
        acc = wave_sum(acc);
        if (lane == 0) f_s[i] = acc + th->f0[i];
      }
      // the wave's own LDS writes precede its reads (in-order per wave);
      // this keeps the compiler from moving them across each other
      __builtin_amdgcn_wave_barrier();
    }
    const double mine = lane < kRS ? resolve_ref(th, th->rref[lane], S.p, row, f_staged ? f_s : nullptr) : 0.0;
#pragma unroll
    for (int r = 0; r < kRS; ++r) R[r] = bcast(mine, r);
  }
  const double n0 = R[0], nbkg = R[1];
  // term weights coef_k amp_k (uniform)
  double gw[kMaxT];
#pragma unroll
  for (int k = 0; k < kMaxT; ++k) gw[k] = k < n_terms ? coef[k] * R[2 + k] : 0.0;
  const double h = S.dt * (double)kWave;  // lane step

  // uniform step constants, one transcendental per lane of every wave, then
  // broadcast within the wave: lane 0: lifetime ratio; lane 1 + 2 s + w:
  // constant w of factor slot s
  // every lane first forms its argument, then the wave makes one exp call
  // and one sincospi call (masked), not one call per primitive kind
  double cst = 0.0;
  {
    double earg = 0.0, parg = 0.0;
    bool e_on = false, p_on = false;
    const int w = (lane - 1) & 1;
    if (lane == 0) {
      earg = neg_inv_tau * h;
      e_on = true;
    } else if (lane <= 2 * kSlots) {
      const int s = (lane - 1) >> 1;
      const int k = s / kMaxFT, f = s % kMaxFT;
      if (k < n_terms && f < Sh::nf(ts, k)) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int q = 0; q < kSlots; ++q) {
          // slots the shape does not use are left out at compile time (fixed
          // shapes), so the selection is a few compares rather than twelve
          if (!(q / kMaxFT < n_terms && q % kMaxFT < Sh::nf(ts, q / kMaxFT))) continue;
          if (q == s) {
            a0 = R[kArg0 + 2 * q];
            a1 = R[kArg0 + 2 * q + 1];
          }
        }
        const int kind = Sh::prim(ts, k, f);
        if (kind == MU_SE && w == 0) {
          earg = -a0 * h;
          e_on = true;
        } else if ((kind == MU_SG || kind == MU_STG) && w == 0) {
          const double x = a0 * h;
          earg = -(x * x);
          e_on = true;
        } else if (kind == MU_TF) {
          parg = 2.0 * a1 * h;  // angle 2 pi nu h
          p_on = true;
        }
      }
    }
    if (e_on) cst = x_exp(earg);
    if (p_on) {
      const D2 cs = x_sincospi(parg);
      cst = w == 0 ? cs.a : cs.b;
    }
  }
  const double rE = bcast(cst, 0);
  double c0[kSlots], c1[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    c0[s] = bcast(cst, 1 + 2 * s);
    c1[s] = bcast(cst, 2 + 2 * s);
  }

  // Scaled cost / model pass. N = N0 e^(-t/tau) (1 + sum_k w_k prod_f F_kf) +
  // Nbkg with w_k = coef_k amp_k is evaluated as
  //   N = E + Nbkg + sum_k L_k prod_{f>0} F_kf,
  // where L_k = N0 w_k e^(-t/tau) F_k0 is the scaled state of the term's
  // first factor (all its recurrences are linear: the lifetime ratio joins its
  // step constants), and E = N0 (1 + sum of w_k / 3 over lone-stg terms)
  // e^(-t/tau) carries the constant part of lone stg terms. stg factors keep
  // (2/3) g in their Gaussian state and u = sigma t as a state of their own.
  constexpr bool kDeriv = MODE == kModeGrad || MODE == kModeJac;  // per-factor values and derivatives
  constexpr bool kScaled = !kDeriv && Sh::kScalable;
  double ecoef = n0;  // E = ecoef e^(-t/tau)
  double su[kSlots];  // sigma h for stg slots
  if constexpr (kScaled) {
#pragma unroll
    for (int kt = 0; kt < kMaxT; ++kt) {
      if (kt < n_terms) {
        const int s = kt * kMaxFT;
        const int p = Sh::prim(ts, kt, 0);
        if (p == MU_SE) c0[s] *= rE;
        if (p == MU_TF) {
          c0[s] *= rE;
          c1[s] *= rE;
        }
        if (p == MU_STG) ecoef = fma(n0 * (coef[kt] * R[2 + kt]), kThird, ecoef);
        if (Sh::fold(ts, kt)) {
          c0[s + 1] *= c0[s];
          c1[s + 1] *= c0[s];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kSlots; ++s) su[s] = R[kArg0 + 2 * s] * h;
  }

  // Cost and model passes of compiled shapes with a rotation: when every
  // rotation turns by at least 1/16 rad-sine per lane step, its real part
  // alone follows x_{k+1} = a x_k - b x_{k-1} (a = 2 rho cos(theta),
  // b = rho^2; rho = 1 exactly for a rotation that is not scaled), which
  // needs neither the imaginary part nor a complex product. Its rounding grows
  // like k min(k, 1 / sin(theta)) eps/2 between anchors (below 3e-13 of the
  // term at 256 steps and this bound), against k eps for the rotation.
  constexpr bool kChebShape = kScaled && shape_has_tf<Sh>();
  double cheb_a[kSlots], cheb_b[kSlots], cheb_ib[kSlots];
  bool cheb_ok = false;
  if constexpr (kChebShape) {
    cheb_ok = true;
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      const int kt = s / kMaxFT, f = s % kMaxFT;
      cheb_a[s] = cheb_b[s] = cheb_ib[s] = 1.0;
      if (kt < n_terms && f < Sh::nf(ts, kt) && Sh::prim(ts, kt, f) == MU_TF) {
        const bool unit = f > 0 && !(f == 1 && Sh::fold(ts, kt));  // the step constants are cos and sin
        cheb_a[s] = 2.0 * c0[s];
        if (!unit) {
          cheb_b[s] = fma(c0[s], c0[s], c1[s] * c1[s]);
          cheb_ib[s] = 1.0 / cheb_b[s];
        }
        cheb_ok = cheb_ok && c1[s] * c1[s] >= cheb_b[s] * (1.0 / 256.0);
      }
    }
    cheb_ok = __builtin_amdgcn_readfirstlane((int)cheb_ok) != 0;
  }

  // per-lane states
  double E = 0.0;
  double s0[kSlots], s1[kSlots], u[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) s0[s] = s1[s] = u[s] = 0.0;

  // Cost pass: the lane's cost runs as a plain sum over one anchor interval
  // (at most 256 terms); at every anchor that sum is folded into the lane's
  // total by TwoSum, whose exact error accumulates in the lane's LDS word
  // (the stage of the function values, unused after the prologue), so the
  // lane's rounding error stays bounded however many bins the segment gives
  // it. The gradient pass sums plainly per lane (its ranges are capped at
  // kMaxGradSplit bins per wave, so at most 2^14 terms per lane).
  double lane_cost = 0.0, lane_sum = 0.0;
  volatile double *lane_err = f_lane;  // kept in LDS, not promoted to a register
  __builtin_amdgcn_wave_barrier();  // the prologue's reads of the stage come first
  *lane_err = 0.0;
  auto fold = [&]() {
    const double s = lane_sum + lane_cost;
    const double bp = s - lane_sum;
    *lane_err += (lane_sum - (s - bp)) + (lane_cost - bp);
    lane_sum = s;
    lane_cost = 0.0;
  };
  double g[kRS];
#pragma unroll
  for (int r = 0; r < kRS; ++r) g[r] = 0.0;

  const int64_t n_first = S.first + S.begin + lane;  // this lane's first bin
  const double t_first = ((double)n_first - S.t0_bin) * S.dt;
  // every lane has n_full bins; lanes below S.n % 64 have one more
  const int seg_n = __builtin_amdgcn_readfirstlane(S.n);  // wave-uniform: scalar loop control
  const int n_full = seg_n / kWave;
  const bool extra = lane < (seg_n % kWave);
  const int n_max = n_full + ((seg_n % kWave) != 0 ? 1 : 0);
  // FP32 storage holds integer counts only (the host checks), FP64 any value
  constexpr bool kIntData = sizeof(CT) == 4;
  // Counts are read PF lane steps ahead of their use, into a ring of
  // registers: dq[i] holds the count of the next step k with k % PF ==
  // i. Reads past a lane's last bin stay inside the counts buffer, which the
  // host pads by PF steps. Values stay in the storage type until use.
  const int64_t idx0 = S.off + S.begin + lane;
  typedef const __attribute__((address_space(1))) CT *GlobalCT;  // global loads, not flat
  const GlobalCT cp = (GlobalCT)(static_cast<const CT *>(S.counts) + idx0);
  CT dq[PF];
#pragma unroll
  for (int i = 0; i < PF; ++i) dq[i] = CT(0);
  if constexpr (MODE != kModeModel) {
#pragma unroll
    for (int i = 0; i < PF; ++i) dq[i] = cp[(int64_t)i * kWave];
  }
  // anchors at multiples of PF steps keep the ring aligned
  const int every = (S.anchor_every + PF - 1) / PF * PF;
  double t = t_first;

  // one bin: value, cost term (or model value), gradient, then advance
  // chi^2 on integer counts reads 1 / max(d, 1) from the workgroup's table
  constexpr bool kTable = COST == MU_COST_CHI2 && kIntData && MODE != kModeModel;
  auto inv_of = [&](CT raw, double x) -> double {
    if constexpr (kTable) return inv_count<TAB>((uint32_t)raw, x, S.inv_tab);
    return 0.0;
  };
  // x_cur: the stored count widened (8 d for integer storage); cheb_tag
  // selects the rotations' real-part recurrence (see above)
  auto bin_step = [&](auto cheb_tag, int k, double x_cur, double iv) {
    constexpr bool kCheb = decltype(cheb_tag)::value;
    const int64_t idx = idx0 + (int64_t)k * kWave;
      if constexpr (kScaled) {
        double acc = E + nbkg;
#pragma unroll
        for (int kt = 0; kt < kMaxT; ++kt) {
          if (kt < n_terms) {
            const int nf = Sh::nf(ts, kt);
            const int s = kt * kMaxFT;
            if (Sh::fold(ts, kt)) {
              acc += s0[s + 1];
            } else if (nf == 1) {
              if (Sh::prim(ts, kt, 0) == MU_STG) {
                acc = fma(fma(-u[s], u[s], 1.0), s0[s], acc);
              } else {
                acc += s0[s];
              }
            } else {
              double others = 1.0;
#pragma unroll
              for (int f = 1; f < kMaxFT; ++f) {
                if (f < nf) {
                  const int q = s + f;
                  const double v = Sh::prim(ts, kt, f) == MU_STG ? fma(fma(-u[q], u[q], 1.0), s0[q], kThird) : s0[q];
                  others = f == 1 ? v : others * v;
                }
              }
              acc = fma(s0[s], others, acc);
            }
          }
        }
        const double N = acc;
        if constexpr (MODE == kModeModel) {
          S.model_out[idx] = N;
        } else {
          lane_cost = cost_add<COST, kIntData>(lane_cost, x_cur, N, iv);
        }
      } else if constexpr (!kDeriv) {
        double A = 0.0;
#pragma unroll
        for (int kt = 0; kt < kMaxT; ++kt) {
          if (kt < n_terms) {
            double prod = 1.0;
#pragma unroll
            for (int f = 0; f < kMaxFT; ++f) {
              const int s = kt * kMaxFT + f;
              if (f < Sh::nf(ts, kt)) prod *= value(Sh::prim(ts, kt, f), t, R[kArg0 + 2 * s], R[kArg0 + 2 * s + 1], s0[s]);
            }
            A = fma(coef[kt] * R[2 + kt], prod, A);
          }
        }
        const double N = fma(n0 * E, 1.0 + A, nbkg);
        if constexpr (MODE == kModeModel) {
          S.model_out[idx] = N;
        } else {
          lane_cost = cost_add<COST, kIntData>(lane_cost, x_cur, N, iv);
        }
      } else {
        double val[kSlots], d0[kSlots], d1[kSlots];
        double tprod[kMaxT];
        double onepA = 1.0;  // 1 + A
#pragma unroll
        for (int kt = 0; kt < kMaxT; ++kt) {
          tprod[kt] = 1.0;
          if (kt < n_terms) {
#pragma unroll
            for (int f = 0; f < kMaxFT; ++f) {
              const int s = kt * kMaxFT + f;
              val[s] = 1.0;
              d0[s] = d1[s] = 0.0;
              if (f < Sh::nf(ts, kt)) {
                val[s] = value_grad(Sh::prim(ts, kt, f), t, R[kArg0 + 2 * s], R[kArg0 + 2 * s + 1], s0[s], s1[s], d0[s],
                                    d1[s]);
                tprod[kt] *= val[s];
              }
            }
            onepA = fma(gw[kt], tprod[kt], onepA);
          }
        }
        const double n0E = n0 * E;
        const double N = fma(n0E, onepA, nbkg);
        // hN = -(1/2) d term / dN; the sums below carry that factor and are
        // scaled by -2 once after the segment. Jacobian rows carry
        // sqrt(d^2 term / dN^2) instead: sqrt(2 / v) for chi^2, sqrt(2 d) / N
        // for the likelihood.
        double hN;
        if constexpr (MODE == kModeJac) {
          const double d_cur = kIntData ? x_cur * kCountUnscale : x_cur;
          if constexpr (COST == MU_COST_CHI2)
            hN = sqrt(2.0 * (kIntData ? iv : 1.0 / (d_cur > 0.0 ? d_cur : 1.0)));
          else
            hN = sqrt(2.0 * d_cur) / N;
        } else if constexpr (COST == MU_COST_CHI2 && kIntData) {
          const double diff = fma(x_cur, kCountUnscale, -N);
          const double w = diff * iv;
          lane_cost = fma(diff, w, lane_cost);
          hN = w;
        } else {
          double dN;
          const double d_cur = kIntData ? x_cur * kCountUnscale : x_cur;
          lane_cost += cost_term<COST, true, kIntData>(d_cur, N, iv, dN);
          hN = -0.5 * dN;
        }
        const double hE = hN * E;     // dN/dN0 = E (1 + A)
        const double hNE = hN * n0E;  // with N0 e^(-t/tau)
        // gradient: g_r += x y; Jacobian row: J_r = x y
        double jr[MODE == kModeJac ? kRS : 1];
        if constexpr (MODE == kModeJac) {
#pragma unroll
          for (int r = 0; r < kRS; ++r) jr[r] = 0.0;
        }
        auto put = [&](int r, double x, double y) {
          if constexpr (MODE == kModeJac)
            jr[r] = x * y;
          else
            g[r] = fma(x, y, g[r]);
        };
        put(0, hE, onepA);
        if constexpr (MODE == kModeJac)
          jr[1] = hN;
        else
          g[1] += hN;
#pragma unroll
        for (int kt = 0; kt < kMaxT; ++kt) {
          if (kt < n_terms) {
            put(2 + kt, hNE * coef[kt], tprod[kt]);
            const double ca = hNE * gw[kt];
#pragma unroll
            for (int f = 0; f < kMaxFT; ++f) {
              const int s = kt * kMaxFT + f;
              if (f < Sh::nf(ts, kt)) {
                double others = ca;
#pragma unroll
                for (int f2 = 0; f2 < kMaxFT; ++f2)
                  if (f2 != f && f2 < Sh::nf(ts, kt)) others *= val[kt * kMaxFT + f2];
                put(kArg0 + 2 * s, others, d0[s]);
                put(kArg0 + 2 * s + 1, others, d1[s]);
              }
            }
          }
        }
        if constexpr (MODE == kModeJac) {
          double *row = S.model_out + idx * kJacCols;
#pragma unroll
          for (int r = 0; r < kJacCols; ++r) row[r] = r < kRS ? jr[r < kRS ? r : 0] : 0.0;
        }
      }

      // advance every state by one lane step
      E *= rE;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        const int kt = s / kMaxFT, f = s % kMaxFT;
        if (kt < n_terms && f < Sh::nf(ts, kt) && !(kScaled && f == 0 && Sh::fold(ts, kt))) {
          if (kCheb && Sh::prim(ts, kt, f) == MU_TF) {
            const double nx = fma(cheb_a[s], s0[s], -(cheb_b[s] * s1[s]));
            s1[s] = s0[s];
            s0[s] = nx;
          } else {
            advance(Sh::prim(ts, kt, f), c0[s], c1[s], s0[s], s1[s]);
          }
          if (kScaled && Sh::prim(ts, kt, f) == MU_STG) u[s] += su[s];
        }
      }
    if constexpr (!kScaled) t += h;
  };

  auto run = [&](auto cheb_tag) {
  constexpr bool kCheb = decltype(cheb_tag)::value;
  for (int k0 = 0; k0 < n_max; k0 += every) {
    // exact re-evaluation (anchor) at the first step of the segment
    t = fma((double)k0, h, t_first);
    double life;
    if constexpr (Sh::kFixed) {
      // the shape's exponentials (lifetime, exponential and Gaussian states)
      // in one call; anchor() below then only places them
      constexpr int kNE = anchor_exps<Sh>();
      DN<kNE> ea;
      int q = 0;
      ea.v[q++] = neg_inv_tau * t;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        const int kt = s / kMaxFT, f = s % kMaxFT;
        if (kt < n_terms && f < Sh::nf(ts, kt)) {
          const int p = Sh::prim(ts, kt, f);
          const double a0 = R[kArg0 + 2 * s];
          if (p == MU_SE) ea.v[q++] = -a0 * t;
          if (p == MU_SG || p == MU_STG) {
            const double x = a0 * t;
            ea.v[q++] = -0.5 * (x * x);
            ea.v[q++] = -(a0 * a0) * h * (t + 0.5 * h);
          }
        }
      }
      ea = x_expn<kNE>(ea);
      q = 0;
      life = ea.v[q++];
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        const int kt = s / kMaxFT, f = s % kMaxFT;
        if (kt < n_terms && f < Sh::nf(ts, kt)) {
          const int p = Sh::prim(ts, kt, f);
          if (p == MU_SE) {
            s0[s] = ea.v[q++];
            s1[s] = 0.0;
          }
          if (p == MU_SG || p == MU_STG) {
            s0[s] = ea.v[q++];
            s1[s] = ea.v[q++];
          }
        }
      }
    } else {
      life = x_exp(neg_inv_tau * t);
    }
    E = kScaled ? ecoef * life : life;
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      const int kt = s / kMaxFT, f = s % kMaxFT;
      if (kt < n_terms && f < Sh::nf(ts, kt)) {
        const int p = Sh::prim(ts, kt, f);
        if (!Sh::kFixed || p == MU_TF || p == MU_GE)
          anchor(p, t, R[kArg0 + 2 * s], R[kArg0 + 2 * s + 1], h, s0[s], s1[s]);
        if constexpr (kScaled) {
          if (p == MU_STG) {
            u[s] = R[kArg0 + 2 * s] * t;
            s0[s] *= kTwoThird;
          }
          if (f == 0) {
            const double L = (n0 * (coef[kt] * R[2 + kt])) * life;
            s0[s] *= L;
            if (p == MU_TF) s1[s] *= L;
            if (p == MU_SG || p == MU_STG) s1[s] *= rE;  // q: the Gaussian step also carries the lifetime
          }
          if (f == 1 && Sh::fold(ts, kt)) {
            s0[s] *= s0[s - 1];
            s1[s] *= s0[s - 1];
          }
          // real-part recurrence: (x_k, x_{k-1}) = (Re z, Re(z / q))
          if (kCheb && p == MU_TF) s1[s] = fma(s0[s], c0[s], s1[s] * c1[s]) * cheb_ib[s];
        }
      }
    }
    const int k1 = min(n_full, k0 + every);
    int k = k0;
    // reads of steps k + PF .. k + 2 PF - 1 from one pointer
    GlobalCT nxt = cp + (int64_t)(k0 + PF) * kWave;
    for (; k + PF <= k1; k += PF, nxt += PF * kWave) {  // uniform trip count
#pragma unroll
      for (int i = 0; i < PF; ++i) {
        const double x = (double)dq[i];  // widened (and looked up) first: the load can reuse its register
        const double iv = inv_of(dq[i], x);
        if constexpr (MODE != kModeModel) {
          dq[i] = nxt[i * kWave];
          // keep the read here, a full PF steps before its use (the
          // scheduler would otherwise sink it towards the end of the loop)
          __builtin_amdgcn_sched_barrier(0);
        }
        bin_step(cheb_tag, k + i, x, iv);
      }
    }
    // only the last segment has a tail: under PF uniform steps, then
    // this lane's ragged extra step
    if (k < k0 + every) {
#pragma unroll
      for (int i = 0; i < PF; ++i)
        if (k + i < n_full || (extra && k + i == n_full))
          bin_step(cheb_tag, k + i, (double)dq[i], inv_of(dq[i], (double)dq[i]));
    }
    if constexpr (MODE == kModeCost) fold();
  }
  };
  if constexpr (kChebShape) {
    if (cheb_ok)
      run(std::true_type{});
    else
      run(std::false_type{});
  } else {
    run(std::false_type{});
  }
  if constexpr (MODE == kModeModel || MODE == kModeJac) return;

  // wave reduction of the cost (compensated) and the gradient (fixed tree);
  // lane 0 writes the segment's slot
  const Pair pc = wave_pair_sum(MODE == kModeCost ? Pair{lane_sum, *lane_err} : Pair{lane_cost, 0.0});
  if (lane == 0) {
    slot[0] = pc.s;
    slot[1] = pc.c;
  }
  if constexpr (MODE == kModeGrad) {
#pragma unroll
    for (int r = 0; r < kRS; ++r) {
      // scalars the shape cannot use are skipped at compile time for fixed shapes
      bool used = r < 2 + kMaxT ? (r < 2 || r - 2 < n_terms) : false;
      if (r >= kArg0) {
        const int q = (r - kArg0) >> 1, kt = q / kMaxFT, f = q % kMaxFT, ai = (r - kArg0) & 1;
        used = kt < n_terms && f < Sh::nf(ts, kt) && ai < prim_nargs(Sh::prim(ts, kt, f));
      }
      double sr = 0.0;
      // the lanes summed -(1/2) r dN/dR (exact scaling by a power of two)
      if (used && (th->rref[r].kind == MU_REF_PAR || th->rref[r].kind == MU_REF_FUN)) sr = -2.0 * wave_sum(g[r]);
      if (lane == 0) slot[2 + r] = sr;
    }
  }
}

// Index of the histogram whose fit range holds offset `off` of a vector's
// concatenated fit ranges (offsets are prefix sums, first 0).
__device__ __forceinline__ int histo_at(const DevHisto *hs, int n_histo, int64_t off) {
  int lo = 0, hi = n_histo - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (hs[mid].off <= off) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The unit of work is one wave (64 lanes; four per workgroup, which share the
// reciprocal table). Unit u is wave u % 4 of workgroup u / 4. Every launch
// cuts its work into equal ranges of split_w bins, one per unit, so every
// unit has the same work; a range is evaluated as the segments it crosses.
// Uniform launch: the n_vec x total (vector, bin) space of one dataset;
// histogram j = v * n_histo + h. Batched launch: the fit ranges of its jobs,
// concatenated in job-list order; histogram j = jbase + h of the job.
// Segment (unit u, histogram j) owns slot u + j: the sum grows by one or two
// from one segment to the next, so slots are unique and each histogram's
// slots are contiguous. When a range starts exactly at a histogram start,
// slot u + j - 1 belongs to no segment and is written as zero so that every
// slot inside a job's span is defined.
// Minimum waves per SIMD asked of the register allocator: the chi^2 cost
// kernels of the compiled shapes fit six (80 registers) without spilling;
// the others are left to the compiler's own choice.
template <int COST, int MODE, typename Sh, int TAB>
constexpr int eval_min_waves() {
  // without the table, the range test of large counts needs more registers
  // in the largest shape
  return (COST == MU_COST_CHI2 && MODE == kModeCost && Sh::kFixed) ? (TAB || Sh::kTerms < 2 ? 6 : 5) : 1;
}

// The workgroup's copy of the context's reciprocal table (chi^2 on integer
// counts), 16 B per load and store.
__device__ __forceinline__ void load_inv_table(double *inv_tab, const double *src) {
  static_assert(kInvTab % 2 == 0, "table copied in pairs");
  const double2 *s2 = reinterpret_cast<const double2 *>(src);
  double2 *d2 = reinterpret_cast<double2 *>(inv_tab);
  for (int i = threadIdx.x; i < kInvTab / 2; i += kBlock) d2[i] = s2[i];
  __syncthreads();
}

// Shape tag of launches whose segments each run their job's compiled shape
// (registers: those of the largest shape).
struct ShapeAny {
  static constexpr bool kFixed = true;
  static constexpr int kTerms = 2;
};

// One segment with the body of shape Sh, or with the job's own compiled
// shape under ShapeAny (a wave-uniform switch).
template <int COST, int MODE, typename CT, typename Sh, int TAB, int PF>
__device__ __forceinline__ void eval_segment_of(const SegIn &S, double *slot, int shape) {
  if constexpr (std::is_same<Sh, ShapeAny>::value) {
    switch (shape) {
      case kShapeExpCos: eval_segment<COST, MODE, CT, ShapeExpCos, TAB, PF>(S, slot); break;
      case kShapeGaussCos: eval_segment<COST, MODE, CT, ShapeGaussCos, TAB, PF>(S, slot); break;
      case kShapeStg: eval_segment<COST, MODE, CT, ShapeStg, TAB, PF>(S, slot); break;
      case kShapeExpStg: eval_segment<COST, MODE, CT, ShapeExpStg, TAB, PF>(S, slot); break;
      default: eval_segment<COST, MODE, CT, ShapeExpCosStg, TAB, PF>(S, slot); break;
    }
  } else {
    (void)shape;
    eval_segment<COST, MODE, CT, Sh, TAB, PF>(S, slot);
  }
}

// The work units (waves) of workgroup b of launch a.
// TAB = 1: every count of the launch is an integer below kInvTab (the table
// lookup needs neither clamp nor range test).
template <int COST, int MODE, typename CT, typename Sh, int TAB, int PF = kPrefetch>
__device__ __forceinline__ void eval_units(const LaunchArgs &a, int b, const double *inv_tab) {
  // each wave is one unit of work; no workgroup barrier after this point
  const int u = __builtin_amdgcn_readfirstlane(b * (kBlock / kWave) + (int)(threadIdx.x / kWave));  // wave-uniform
  const int lane = threadIdx.x & (kWave - 1);
  if (u >= a.n_units) return;
  const bool batch = a.jobs != nullptr;
  int64_t pos = (int64_t)u * a.split_w;
  const int64_t end = min(pos + a.split_w, batch ? a.total : (int64_t)a.n_vec * a.total);
  if (pos >= end) return;
  // v: the vector (uniform launch) or the job-list entry (batched launch)
  int v, h;
  DevJob J;
  int64_t vstart;  // first bin of vector / job v in the launch
  if (batch) {
    v = uni(a.unit_start[2 * u]);
    h = uni(a.unit_start[2 * u + 1]);
    J = a.jobs[uni(a.job_list[v])];
    vstart = uni(J.goff);
  } else {
    v = (int)(pos / a.total);
    vstart = (int64_t)v * a.total;
    J = a.tmpl;
    h = histo_at(J.histos, J.n_histo, pos - vstart);
  }
  int nh = uni(J.n_histo), jb = batch ? uni(J.jbase) : v * nh;
  if ((MODE == kModeCost || MODE == kModeGrad) && jb + h > 0 && pos == vstart + J.histos[h].off) {
    if (lane < kSlot) a.partial[((int64_t)u + jb + h - 1) * kSlot + lane] = 0.0;
  }
  for (;;) {
    SegIn S;
    const DevHisto H = uni(J.histos[h]);
    const int64_t h_start = vstart + H.off;
    const int64_t seg_end = min(end, h_start + H.n);
    S.th = J.th;
    S.p = batch ? J.p : J.p + (int64_t)v * a.p_stride;
    S.counts = J.counts;
    S.model_out = J.model_out;
    S.begin = pos - h_start;
    S.n = (int32_t)(seg_end - pos);
    S.off = H.off;
    S.first = H.first;
    S.t0_bin = H.t0_bin;
    S.dt = H.dt;
    S.map_row = H.map_row;
    S.anchor_every = a.anchor_every;
    S.inv_tab = inv_tab;
    eval_segment_of<COST, MODE, CT, Sh, TAB, PF>(S, a.partial + ((int64_t)u + jb + h) * kSlot, uni(J.shape));
    pos = seg_end;
    if (pos >= end) return;
    if (++h == nh) {
      h = 0;
      ++v;
      if (batch) {
        J = a.jobs[uni(a.job_list[v])];
        vstart = uni(J.goff);
        nh = uni(J.n_histo);
        jb = uni(J.jbase);
      } else {
        vstart += a.total;
        jb += nh;
      }
    }
  }
}

template <int COST, int MODE, typename CT>
constexpr bool eval_table() {
  return COST == MU_COST_CHI2 && sizeof(CT) == 4 && MODE != kModeModel;
}

template <int COST, int MODE, typename CT, typename Sh, int TAB, int PF = kPrefetch>
__global__ __launch_bounds__(kBlock, (eval_min_waves<COST, MODE, Sh, TAB>())) void eval_kernel(LaunchArgs a) {
  constexpr bool kTable = eval_table<COST, MODE, CT>();
  __shared__ __align__(16) double inv_tab[kTable ? kInvTab : 2];
  if constexpr (kTable) load_inv_table(inv_tab, a.inv_src);
  eval_units<COST, MODE, CT, Sh, TAB, PF>(a, blockIdx.x, inv_tab);
}

// A gradient pass and a cost pass over the same dataset and theory in one
// launch: workgroups [0, n_grad_blocks) take the gradient launch's units, the
// rest the cost launch's, so the gradient waves (few, latency-bound) run
// beside the cost waves instead of before them. Four waves per SIMD: the
// gradient body's registers.
template <int COST, typename CT, typename Sh, int TAB>
__global__ __launch_bounds__(kBlock, 4) void eval_grad_cost_kernel(LaunchArgs g, int n_grad_blocks, LaunchArgs c) {
  constexpr bool kTable = eval_table<COST, kModeCost, CT>();
  __shared__ __align__(16) double inv_tab[kTable ? kInvTab : 2];
  if constexpr (kTable) load_inv_table(inv_tab, c.inv_src);
  if ((int)blockIdx.x < n_grad_blocks)
    eval_units<COST, kModeGrad, CT, Sh, TAB>(g, blockIdx.x, inv_tab);
  else
    eval_units<COST, kModeCost, CT, Sh, TAB, kPrefetchStream>(c, blockIdx.x - n_grad_blocks, inv_tab);
}

// One workgroup per job: fixed-order merge of the job's slots.  It runs as
// its own launch after the evaluation kernel, whose completion makes every
// slot visible; no fences or atomics are needed inside the evaluation kernel.
template <int MODE, int NT = kBlock>
__device__ __forceinline__ void merge_block(const LaunchArgs &a, int job) {
  DevJob J;
  if (a.jobs == nullptr) {
    J = a.tmpl;
    J.p += job * a.p_stride;
    J.cost_out += job;
    if (J.histo_out) J.histo_out += job * a.histo_stride;
    if (J.grad_out) J.grad_out += job * a.grad_stride;
  } else {
    J = a.jobs[job];
  }
  merge_job<MODE, NT>(a, J, job);
}

// NT threads per job: one wave for launches of many small jobs (more jobs
// in flight per CU), else four.
template <int MODE, int NT>
__global__ __launch_bounds__(NT) void merge_kernel(LaunchArgs a) {
  merge_block<MODE, NT>(a, blockIdx.x);
}

// Merges of two launches in one: workgroups [0, n_first) merge the jobs of
// `first` (mode M0), the rest those of `second` (mode M1).
template <int M0, int M1>
__global__ __launch_bounds__(kBlock) void merge2_kernel(LaunchArgs first, int n_first, LaunchArgs second) {
  if ((int)blockIdx.x < n_first)
    merge_block<M0>(first, blockIdx.x);
  else
    merge_block<M1>(second, blockIdx.x - n_first);
}

template <int COST, int MODE, typename Sh>
hipError_t launch_shape(const LaunchArgs &a, int count_f64, hipStream_t s) {
  dim3 grid((a.n_units + kBlock / kWave - 1) / (kBlock / kWave)), block(kBlock);  // n_units counts units (waves)
  constexpr bool kTab = COST == MU_COST_CHI2 && MODE != kModeModel;
  if (count_f64)
    hipLaunchKernelGGL((eval_kernel<COST, MODE, double, ShapeGeneric, 0>), grid, block, 0, s, a);
  else if (kTab && a.counts_in_table)
    hipLaunchKernelGGL((eval_kernel<COST, MODE, uint32_t, Sh, kTab ? 1 : 0>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((eval_kernel<COST, MODE, uint32_t, Sh, 0>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <int COST, int MODE, typename Sh>
int occupancy_shape(int count_f64) {
  int nb = 0;
  hipError_t e;
  if (count_f64)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, reinterpret_cast<const void *>(&eval_kernel<COST, MODE, double, ShapeGeneric, 0>), kBlock, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, reinterpret_cast<const void *>(&eval_kernel<COST, MODE, uint32_t, Sh, 0>), kBlock, 0);
  return e == hipSuccess ? nb : 0;
}

template <int COST, int MODE>
int occupancy_typed(int count_f64, int shape) {
  switch (shape) {
    case kShapeExpCos: return occupancy_shape<COST, MODE, ShapeExpCos>(count_f64);
    case kShapeGaussCos: return occupancy_shape<COST, MODE, ShapeGaussCos>(count_f64);
    case kShapeStg: return occupancy_shape<COST, MODE, ShapeStg>(count_f64);
    case kShapeExpStg: return occupancy_shape<COST, MODE, ShapeExpStg>(count_f64);
    case kShapeExpCosStg: return occupancy_shape<COST, MODE, ShapeExpCosStg>(count_f64);
    default: return occupancy_shape<COST, MODE, ShapeGeneric>(count_f64);
  }
}

}  // namespace

int eval_blocks_per_cu(int mode, int cost_kind, int count_f64, int shape) {
  if (mode == kModeModel) return occupancy_typed<MU_COST_CHI2, kModeModel>(count_f64, shape);
  if (cost_kind == MU_COST_CHI2)
    return mode == kModeGrad ? occupancy_typed<MU_COST_CHI2, kModeGrad>(count_f64, shape)
                             : occupancy_typed<MU_COST_CHI2, kModeCost>(count_f64, shape);
  return mode == kModeGrad ? occupancy_typed<MU_COST_POISSON, kModeGrad>(count_f64, shape)
                           : occupancy_typed<MU_COST_POISSON, kModeCost>(count_f64, shape);
}

namespace {

template <int COST, typename Sh>
hipError_t launch_grad_cost_shape(const LaunchArgs &g, const LaunchArgs &c, hipStream_t s) {
  const int per = kBlock / kWave;
  const int nbg = (g.n_units + per - 1) / per, nbc = (c.n_units + per - 1) / per;
  dim3 grid(nbg + nbc), block(kBlock);
  constexpr int kTab = COST == MU_COST_CHI2 ? 1 : 0;
  if (kTab && c.counts_in_table && g.counts_in_table)
    hipLaunchKernelGGL((eval_grad_cost_kernel<COST, uint32_t, Sh, kTab>), grid, block, 0, s, g, nbg, c);
  else
    hipLaunchKernelGGL((eval_grad_cost_kernel<COST, uint32_t, Sh, 0>), grid, block, 0, s, g, nbg, c);
  return hipGetLastError();
}

template <int COST>
hipError_t launch_grad_cost_typed(const LaunchArgs &g, const LaunchArgs &c, int shape, hipStream_t s) {
  switch (shape) {
    case kShapeExpCos: return launch_grad_cost_shape<COST, ShapeExpCos>(g, c, s);
    case kShapeGaussCos: return launch_grad_cost_shape<COST, ShapeGaussCos>(g, c, s);
    case kShapeStg: return launch_grad_cost_shape<COST, ShapeStg>(g, c, s);
    case kShapeExpStg: return launch_grad_cost_shape<COST, ShapeExpStg>(g, c, s);
    case kShapeExpCosStg: return launch_grad_cost_shape<COST, ShapeExpCosStg>(g, c, s);
    default: return hipErrorNotSupported;
  }
}

}  // namespace

// chi^2 only: the likelihood's gradient body needs more registers than four
// waves per SIMD leave (it would spill)
bool eval_grad_cost_fused(int count_f64, int shape, int cost_kind) {
  return !count_f64 && shape > kShapeGeneric && shape < kShapeCount && cost_kind == MU_COST_CHI2;
}

hipError_t launch_eval_grad_cost(const LaunchArgs &g, const LaunchArgs &c, int count_f64, int shape, hipStream_t s) {
  if (!eval_grad_cost_fused(count_f64, shape, c.cost_kind) || g.cost_kind != c.cost_kind) return hipErrorNotSupported;
  if (g.n_units <= 0 || c.n_units <= 0) return hipErrorInvalidValue;
  if (g.anchor_every < 1 || g.anchor_every > 256 || c.anchor_every < 1 || c.anchor_every > 256)
    return hipErrorInvalidValue;
  return launch_grad_cost_typed<MU_COST_CHI2>(g, c, shape, s);
}

hipError_t launch_merge(const LaunchArgs &a, int mode, int n_jobs, int lds_bytes, bool narrow, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  dim3 grid(n_jobs), block(narrow ? kWave : kBlock);
  if (mode == kModeGrad) {
    if (narrow)
      hipLaunchKernelGGL((merge_kernel<kModeGrad, kWave>), grid, block, (size_t)lds_bytes, s, a);
    else
      hipLaunchKernelGGL((merge_kernel<kModeGrad, kBlock>), grid, block, (size_t)lds_bytes, s, a);
  } else {
    if (narrow)
      hipLaunchKernelGGL((merge_kernel<kModeCost, kWave>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((merge_kernel<kModeCost, kBlock>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_merge_grad_cost(const LaunchArgs &g, int n_grad, const LaunchArgs &c, int n_cost, int lds_bytes,
                                  hipStream_t s) {
  if (n_grad <= 0 || n_cost <= 0) return hipErrorInvalidValue;
  dim3 grid(n_grad + n_cost), block(kBlock);
  hipLaunchKernelGGL((merge2_kernel<kModeGrad, kModeCost>), grid, block, (size_t)lds_bytes, s, g, n_grad, c);
  return hipGetLastError();
}

namespace {

template <int COST, int MODE>
hipError_t launch_typed(const LaunchArgs &a, int count_f64, int shape, hipStream_t s) {
  switch (shape) {
    case kShapeExpCos: return launch_shape<COST, MODE, ShapeExpCos>(a, count_f64, s);
    case kShapeGaussCos: return launch_shape<COST, MODE, ShapeGaussCos>(a, count_f64, s);
    case kShapeStg: return launch_shape<COST, MODE, ShapeStg>(a, count_f64, s);
    case kShapeExpStg: return launch_shape<COST, MODE, ShapeExpStg>(a, count_f64, s);
    case kShapeExpCosStg: return launch_shape<COST, MODE, ShapeExpCosStg>(a, count_f64, s);
    default: return launch_shape<COST, MODE, ShapeGeneric>(a, count_f64, s);
  }
}

}  // namespace

namespace {

// Count prefetch depth of batched launches: the cost pass streams counts
// from HBM and keeps more reads in flight; the gradient pass (bound by its
// arithmetic) keeps the registers.
constexpr int batch_prefetch(int mode) { return mode == kModeCost ? kPrefetchStream : kPrefetch; }

template <int COST, int MODE>
hipError_t launch_batch_typed(const LaunchArgs &a, int count_f64, int generic, hipStream_t s) {
  dim3 grid((a.n_units + kBlock / kWave - 1) / (kBlock / kWave)), block(kBlock);
  constexpr bool kTab = COST == MU_COST_CHI2;
  if (count_f64)
    hipLaunchKernelGGL((eval_kernel<COST, MODE, double, ShapeGeneric, 0>), grid, block, 0, s, a);
  else if (generic)
    hipLaunchKernelGGL((eval_kernel<COST, MODE, uint32_t, ShapeGeneric, 0>), grid, block, 0, s, a);
  else if (kTab && a.counts_in_table)
    hipLaunchKernelGGL((eval_kernel<COST, MODE, uint32_t, ShapeAny, kTab ? 1 : 0, batch_prefetch(MODE)>), grid, block,
                       0, s, a);
  else
    hipLaunchKernelGGL((eval_kernel<COST, MODE, uint32_t, ShapeAny, 0, batch_prefetch(MODE)>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <int COST, int MODE>
int batch_occupancy(int count_f64, int generic) {
  int nb = 0;
  const void *k = (count_f64 || generic)
                      ? (count_f64 ? reinterpret_cast<const void *>(&eval_kernel<COST, MODE, double, ShapeGeneric, 0>)
                                   : reinterpret_cast<const void *>(&eval_kernel<COST, MODE, uint32_t, ShapeGeneric, 0>))
                      : reinterpret_cast<const void *>(&eval_kernel<COST, MODE, uint32_t, ShapeAny, 0, batch_prefetch(MODE)>);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kBlock, 0) == hipSuccess ? nb : 0;
}

}  // namespace

hipError_t launch_eval_batch(const LaunchArgs &a, int mode, int count_f64, int generic, hipStream_t s) {
  if (a.n_units <= 0) return hipSuccess;
  if (a.anchor_every < 1 || a.anchor_every > 256 || a.jobs == nullptr || a.split_w <= 0) return hipErrorInvalidValue;
  if (a.cost_kind == MU_COST_CHI2)
    return mode == kModeGrad ? launch_batch_typed<MU_COST_CHI2, kModeGrad>(a, count_f64, generic, s)
                             : launch_batch_typed<MU_COST_CHI2, kModeCost>(a, count_f64, generic, s);
  return mode == kModeGrad ? launch_batch_typed<MU_COST_POISSON, kModeGrad>(a, count_f64, generic, s)
                           : launch_batch_typed<MU_COST_POISSON, kModeCost>(a, count_f64, generic, s);
}

int eval_batch_blocks_per_cu(int mode, int cost_kind, int count_f64, int generic) {
  if (cost_kind == MU_COST_CHI2)
    return mode == kModeGrad ? batch_occupancy<MU_COST_CHI2, kModeGrad>(count_f64, generic)
                             : batch_occupancy<MU_COST_CHI2, kModeCost>(count_f64, generic);
  return mode == kModeGrad ? batch_occupancy<MU_COST_POISSON, kModeGrad>(count_f64, generic)
                           : batch_occupancy<MU_COST_POISSON, kModeCost>(count_f64, generic);
}

hipError_t launch_jac(const LaunchArgs &a, int count_f64, int shape, hipStream_t s) {
  if (a.n_units <= 0) return hipSuccess;
  if (a.anchor_every < 1 || a.anchor_every > 256 || a.jobs != nullptr || a.n_vec != 1 || !a.tmpl.model_out)
    return hipErrorInvalidValue;
  return a.cost_kind == MU_COST_CHI2 ? launch_typed<MU_COST_CHI2, kModeJac>(a, count_f64, shape, s)
                                     : launch_typed<MU_COST_POISSON, kModeJac>(a, count_f64, shape, s);
}

hipError_t launch_eval(const LaunchArgs &a, int mode, int count_f64, int shape, hipStream_t s) {
  if (a.n_units <= 0) return hipSuccess;
  if (a.anchor_every < 1 || a.anchor_every > 256) return hipErrorInvalidValue;
  if (mode == kModeModel) return launch_typed<MU_COST_CHI2, kModeModel>(a, count_f64, shape, s);
  if (a.cost_kind == MU_COST_CHI2)
    return mode == kModeGrad ? launch_typed<MU_COST_CHI2, kModeGrad>(a, count_f64, shape, s)
                             : launch_typed<MU_COST_CHI2, kModeCost>(a, count_f64, shape, s);
  return mode == kModeGrad ? launch_typed<MU_COST_POISSON, kModeGrad>(a, count_f64, shape, s)
                           : launch_typed<MU_COST_POISSON, kModeCost>(a, count_f64, shape, s);
}

// ------------------------------------------------------ allocation-free slots

// Partial slots of the allocation-free entry point (mu_chi2_eval_static): one
// array per device, part of the code object, held until the process ends.
// Host code never passes the array's name to a kernel: it uses the address
// hipGetSymbolAddress returns on each device.
static __device__ __align__(256) double scratch[(size_t)kStaticSlots * kSlot];

namespace {
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void *ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch[device] = static_cast<double *>(ptr);
  if (cur != device) hipSetDevice(cur);
  return e;
}

double *static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[device];
}

}  // namespace mu
