// Run-time compiled user theories (the paper's user functions, Sec. 4.2.1 and
// Listing 3: the theory is written as code and compiled when the fit starts).
//
// The asymmetry A(t) is an expression in a small language (mu.h states the
// grammar).  It is parsed here, its distinct parameter / function references
// become the theory's resolved scalars 2, 3, ... (N0 and Nbkg are 0 and 1, as
// for theory programs), and the expression is written as C++ over dual
// numbers (value and the derivatives in those references) into the kernel
// template mu_rtc_kernel.inc.  hipRTC compiles that source for gfx950 once
// per context and distinct source; the module's kernel then serves every
// launch mode (cost, gradient, model values, Jacobian rows) of the library's
// split and batched launches, and the merge kernels, gradient plans and
// fitter work unchanged.

#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mu_internal.h"
#include "mu_runtime.h"
// the build writes this file: kRtcStructs (mu_structs.h), kRtcMu (mu.h) and
// kRtcKernel (mu_rtc_kernel.inc) as string literals
#include "mu_rtc_sources.inc"

using namespace mu;

namespace {

enum Op { N_NUM, N_T, N_REF, N_NEG, N_ADD, N_SUB, N_MUL, N_DIV, N_POW, N_CALL };

struct Fn {
  const char *name;
  int nargs;
  const char *dual;  // the dual-number function in the kernel template
  bool takes_t;      // primitives: t is their implicit first argument
};
const Fn kFns[] = {{"exp", 1, "d_exp", false},   {"log", 1, "d_log", false},   {"sqrt", 1, "d_sqrt", false},
                   {"sin", 1, "d_sin", false},   {"cos", 1, "d_cos", false},   {"pow", 2, "d_pow", false},
                   {"j0", 1, "d_j0", false},     {"se", 1, "d_se", true},      {"ge", 2, "d_ge", true},
                   {"sg", 1, "d_sg", true},      {"stg", 1, "d_stg", true},    {"tf", 2, "d_tf", true},
                   {"sekt", 1, "d_sekt", true},  {"ab", 2, "d_ab", true},      {"b", 2, "d_b", true},
                   {"ifld", 5, "d_ifld", true},  {"ibsl", 5, "d_ibsl", true}};

struct Node {
  int op = N_NUM;
  double num = 0.0;
  int kind = 0, slot = 0;  // N_REF: MU_REF_PAR or MU_REF_FUN, map slot
  int fn = -1;             // N_CALL: index in kFns
  std::vector<int> kids;
};

// Limits that keep the recursive-descent parser's stack and the generated
// kernel bounded.
constexpr int kMaxNest = 200;
constexpr size_t kMaxExprLen = 1 << 16;
constexpr size_t kMaxNodes = 4096;  // bounds the tree's depth for the recursive emitter

struct Parser {
  const char *s;
  size_t i = 0;
  int nest = 0;  // unary() frames open (every recursion passes through unary)
  std::vector<Node> nodes;
  std::string err;

  void ws() {
    while (s[i] && std::isspace((unsigned char)s[i])) ++i;
  }
  bool fail(const std::string &m) {
    if (err.empty()) err = m + " at offset " + std::to_string(i);
    return false;
  }
  int add(Node n) {
    if (nodes.size() >= kMaxNodes) return fail("more than " + std::to_string(kMaxNodes) + " operations"), -1;
    nodes.push_back(std::move(n));
    return (int)nodes.size() - 1;
  }
  bool eat(char c) {
    ws();
    if (s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  int expr() {
    int a = term();
    for (;;) {
      if (a < 0) return -1;
      ws();
      const char c = s[i];
      if (c != '+' && c != '-') return a;
      ++i;
      const int b = term();
      if (b < 0) return -1;
      Node n;
      n.op = c == '+' ? N_ADD : N_SUB;
      n.kids = {a, b};
      a = add(n);
    }
  }
  int term() {
    int a = unary();
    for (;;) {
      if (a < 0) return -1;
      ws();
      const char c = s[i];
      if (c != '*' && c != '/') return a;
      ++i;
      const int b = unary();
      if (b < 0) return -1;
      Node n;
      n.op = c == '*' ? N_MUL : N_DIV;
      n.kids = {a, b};
      a = add(n);
    }
  }
  int unary() {
    if (nest >= kMaxNest) return fail("nesting deeper than " + std::to_string(kMaxNest)), -1;
    ++nest;
    const int r = unary_body();
    --nest;
    return r;
  }
  int unary_body() {
    if (eat('-')) {
      const int a = unary();
      if (a < 0) return -1;
      Node n;
      n.op = N_NEG;
      n.kids = {a};
      return add(n);
    }
    if (eat('+')) return unary();
    return power();
  }
  int power() {
    const int a = primary();
    if (a < 0) return -1;
    if (eat('^')) {
      const int b = unary();
      if (b < 0) return -1;
      Node n;
      n.op = N_POW;
      n.kids = {a, b};
      return add(n);
    }
    return a;
  }
  bool number(double &v) {
    ws();
    const char *p = s + i;
    if (!(std::isdigit((unsigned char)*p) || (*p == '.' && std::isdigit((unsigned char)p[1])))) return false;
    char *e = nullptr;
    v = std::strtod(p, &e);
    i += (size_t)(e - p);
    return true;
  }
  int primary() {
    ws();
    double v;
    if (number(v)) {
      Node n;
      n.op = N_NUM;
      n.num = v;
      return add(n);
    }
    if (eat('(')) {
      const int a = expr();
      if (a < 0) return -1;
      if (!eat(')')) return fail("expected ')'"), -1;
      return a;
    }
    if (!(std::isalpha((unsigned char)s[i]) || s[i] == '_')) return fail("expected a number, a name or '('"), -1;
    size_t j = i;
    while (std::isalnum((unsigned char)s[j]) || s[j] == '_') ++j;
    const std::string name(s + i, j - i);
    i = j;
    if (name == "t") {
      Node n;
      n.op = N_T;
      return add(n);
    }
    if (name == "pi") {
      Node n;
      n.op = N_NUM;
      n.num = 3.14159265358979323846;
      return add(n);
    }
    if ((name == "p" || name == "f") && eat('[')) {
      ws();
      size_t k = i;
      while (std::isdigit((unsigned char)s[k])) ++k;
      if (k == i) return fail("expected a slot number"), -1;
      const long slot = std::strtol(s + i, nullptr, 10);
      i = k;
      if (!eat(']')) return fail("expected ']'"), -1;
      Node n;
      n.op = N_REF;
      n.kind = name == "p" ? MU_REF_PAR : MU_REF_FUN;
      n.slot = slot > 1000000 ? 1000000 : (int)slot;
      return add(n);
    }
    int fn = -1;
    for (int q = 0; q < (int)(sizeof kFns / sizeof kFns[0]); ++q)
      if (name == kFns[q].name) fn = q;
    if (fn < 0) return fail("unknown name '" + name + "'"), -1;
    if (!eat('(')) return fail("expected '(' after " + name), -1;
    Node n;
    n.op = N_CALL;
    n.fn = fn;
    for (;;) {
      const int a = expr();
      if (a < 0) return -1;
      n.kids.push_back(a);
      if (eat(',')) continue;
      if (eat(')')) break;
      return fail("expected ',' or ')'"), -1;
    }
    if ((int)n.kids.size() != kFns[fn].nargs)
      return fail(name + " takes " + std::to_string(kFns[fn].nargs) + " argument(s)"), -1;
    return add(n);
  }
};

struct Parsed {
  std::vector<Node> nodes;
  int root = -1;
  std::vector<std::pair<int, int>> refs;  // distinct (kind, slot), first appearance
};

void collect(const Parsed &P, int k, std::vector<std::pair<int, int>> &refs) {
  const Node &n = P.nodes[k];
  if (n.op == N_REF) {
    const std::pair<int, int> r{n.kind, n.slot};
    bool seen = false;
    for (const auto &x : refs) seen = seen || x == r;
    if (!seen) refs.push_back(r);
  }
  for (int c : n.kids) collect(P, c, refs);
}

std::string emit(const Parsed &P, int k) {
  const Node &n = P.nodes[k];
  char b[64];
  switch (n.op) {
    case N_NUM:
      std::snprintf(b, sizeof b, "dc(%.17g)", n.num);
      return b;
    case N_T:
      return "dc(t)";
    case N_REF:
      for (size_t q = 0; q < P.refs.size(); ++q)
        if (P.refs[q] == std::make_pair(n.kind, n.slot)) return "R[" + std::to_string(q) + "]";
      return "dc(0.0)";
    case N_NEG:
      return "(-" + emit(P, n.kids[0]) + ")";
    case N_ADD:
      return "(" + emit(P, n.kids[0]) + " + " + emit(P, n.kids[1]) + ")";
    case N_SUB:
      return "(" + emit(P, n.kids[0]) + " - " + emit(P, n.kids[1]) + ")";
    case N_MUL:
      return "(" + emit(P, n.kids[0]) + " * " + emit(P, n.kids[1]) + ")";
    case N_DIV:
      return "(" + emit(P, n.kids[0]) + " / " + emit(P, n.kids[1]) + ")";
    case N_POW:
      return "d_pow(" + emit(P, n.kids[0]) + ", " + emit(P, n.kids[1]) + ")";
    default: {
      std::string s = std::string(kFns[n.fn].dual) + "(" + (kFns[n.fn].takes_t ? "t, " : "");
      for (size_t q = 0; q < n.kids.size(); ++q) s += (q ? ", " : "") + emit(P, n.kids[q]);
      return s + ")";
    }
  }
}

mu_status check_expr_ref(const mu_expr_theory_desc *d, int kind, int slot, const char *what, std::string &why) {
  char b[256];
  if (kind == MU_REF_LIT) {
    return MU_OK;
  }
  if (kind != MU_REF_PAR && kind != MU_REF_FUN) {
    std::snprintf(b, sizeof b, "%s: unknown reference kind %d", what, kind);
    why = b;
    return MU_E_ARG;
  }
  if (slot < 0 || slot >= d->n_slots) {
    std::snprintf(b, sizeof b, "%s: slot %d outside [0, %d)", what, slot, d->n_slots);
    why = b;
    return MU_E_ARG;
  }
  const int lim = kind == MU_REF_PAR ? d->n_par : d->n_fun;
  for (int row = 0; row < d->n_rows; ++row) {
    const int v = d->map[row * d->n_slots + slot];
    if (v < 0 || v >= lim) {
      std::snprintf(b, sizeof b, "%s: map[%d][%d] = %d outside [0, %d)", what, row, slot, v, lim);
      why = b;
      return MU_E_ARG;
    }
  }
  return MU_OK;
}

// Parse and validate; on success fills P and the generated kernel source.
mu_status parse_expr(const mu_expr_theory_desc *d, Parsed &P, std::string &src, std::string &why) {
  if (!d || !d->asymmetry) {
    why = "null descriptor or expression";
    return MU_E_ARG;
  }
  if (d->n_par < 1 || d->n_par > MU_MAX_PAR || !(d->tau_mu > 0.0) || !std::isfinite(d->tau_mu) || d->n_rows < 1 ||
      d->n_slots < 1 || !d->map || d->n_fun < 0 || (d->n_fun > 0 && (!d->F || !d->f0))) {
    why = "need 1 <= n_par <= MU_MAX_PAR, tau_mu > 0, a map of n_rows >= 1 x n_slots >= 1, and F, f0 when n_fun > 0";
    return MU_E_ARG;
  }
  mu_status st;
  if ((st = check_expr_ref(d, d->n0.kind, d->n0.slot, "n0", why)) != MU_OK) return st;
  if ((st = check_expr_ref(d, d->nbkg.kind, d->nbkg.slot, "nbkg", why)) != MU_OK) return st;
  if ((d->n0.kind == MU_REF_LIT && !std::isfinite(d->n0.literal)) ||
      (d->nbkg.kind == MU_REF_LIT && !std::isfinite(d->nbkg.literal))) {
    why = "a literal N0 or Nbkg is not finite";
    return MU_E_ARG;
  }
  if (std::strlen(d->asymmetry) > kMaxExprLen) {
    why = "expression longer than " + std::to_string(kMaxExprLen) + " characters";
    return MU_E_ARG;
  }
  Parser ps;
  ps.s = d->asymmetry;
  const int root = ps.expr();
  ps.ws();
  if (root < 0 || ps.s[ps.i] != '\0') {
    why = "expression: " + (ps.err.empty() ? std::string("unexpected text at offset ") + std::to_string(ps.i) : ps.err);
    return MU_E_ARG;
  }
  P.nodes = std::move(ps.nodes);
  P.root = root;
  collect(P, root, P.refs);
  if ((int)P.refs.size() > kRS - 2) {
    why = "expression: more than " + std::to_string(kRS - 2) + " distinct parameter / function references";
    return MU_E_UNSUPPORTED;
  }
  for (const auto &r : P.refs)
    if ((st = check_expr_ref(d, r.first, r.second, "expression reference", why)) != MU_OK) return st;
  src = kRtcKernel;
  const std::string k = std::to_string(P.refs.size()), e = emit(P, root);
  size_t at;
  while ((at = src.find("@K@")) != std::string::npos) src.replace(at, 3, k);
  while ((at = src.find("@EXPR@")) != std::string::npos) src.replace(at, 6, e);
  return MU_OK;
}

void put_text(char *msg, int32_t len, const std::string &s) {
  if (!msg || len <= 0) return;
  std::snprintf(msg, (size_t)len, "%s", s.c_str());
}

// hipRTC: compile `src` for gfx950 (the library's own flags) into a code object.
mu_status rtc_compile(const std::string &src, std::vector<char> &code, std::string &log) {
  static const char *kStdint =
      "typedef __hip_internal::int8_t int8_t; typedef __hip_internal::uint8_t uint8_t;\n"
      "typedef __hip_internal::int16_t int16_t; typedef __hip_internal::uint16_t uint16_t;\n"
      "typedef __hip_internal::int32_t int32_t; typedef __hip_internal::uint32_t uint32_t;\n"
      "typedef __hip_internal::int64_t int64_t; typedef __hip_internal::uint64_t uint64_t;\n";
  const char *hdrs[] = {kRtcStructs, kRtcMu, kStdint};
  const char *names[] = {"mu_structs.h", "mu.h", "stdint.h"};
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "mu_user_theory.hip", 3, hdrs, names) != HIPRTC_SUCCESS) {
    log = "hiprtcCreateProgram failed";
    return MU_E_DEVICE;
  }
  const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(prog, &ls);
  if (ls > 1) {
    log.resize(ls);
    hiprtcGetProgramLog(prog, &log[0]);
  }
  if (r != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    return MU_E_ARG;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  code.resize(cs);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  return MU_OK;
}

}  // namespace

extern "C" mu_status mu_theory_check_expr(const mu_expr_theory_desc *d, char *msg, int32_t msg_len) {
  Parsed P;
  std::string src, why;
  const mu_status st = parse_expr(d, P, src, why);
  put_text(msg, msg_len, st == MU_OK ? "ok: " + std::to_string(P.refs.size()) + " references" : why);
  return st;
}

extern "C" mu_status mu_theory_expr_source(const mu_expr_theory_desc *d, char *buf, int64_t buf_len, int64_t *needed) {
  Parsed P;
  std::string src, why;
  const mu_status st = parse_expr(d, P, src, why);
  if (st != MU_OK) return st;
  if (needed) *needed = (int64_t)src.size() + 1;
  if (buf && buf_len > 0) std::snprintf(buf, (size_t)buf_len, "%s", src.c_str());
  return MU_OK;
}

extern "C" mu_status mu_theory_compile_check(const mu_expr_theory_desc *d, char *msg, int32_t msg_len) {
  Parsed P;
  std::string src, why;
  mu_status st = parse_expr(d, P, src, why);
  if (st != MU_OK) {
    put_text(msg, msg_len, why);
    return st;
  }
  std::vector<char> code;
  std::string log;
  st = rtc_compile(src, code, log);
  put_text(msg, msg_len, st == MU_OK ? "ok: " + std::to_string(code.size()) + " bytes of gfx950 code" : log);
  return st;
}

extern "C" mu_status mu_theory_create_expr(mu_ctx *ctx, const mu_expr_theory_desc *d, mu_theory **out) {
  if (!ctx || !out) return MU_E_ARG;
  *out = nullptr;
  Parsed P;
  std::string src, why;
  mu_status st = parse_expr(d, P, src, why);
  if (st != MU_OK) {
    set_err(ctx, "%s", why.c_str());
    return st;
  }
  (void)hipSetDevice(ctx->device);
  // one module per distinct source on this context
  hipFunction_t fn = nullptr;
  for (const auto &m : ctx->rtc)
    if (m.src == src) fn = m.fn;
  if (!fn) {
    std::vector<char> code;
    std::string log;
    st = rtc_compile(src, code, log);
    if (st != MU_OK) {
      set_err(ctx, "run-time compilation failed: %s", log.c_str());
      return st;
    }
    mu_ctx::RtcModule m;
    m.src = src;
    hipError_t e = hipModuleLoadData(&m.mod, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&m.fn, m.mod, "mu_rtc_kernel");
    if (e != hipSuccess) {
      if (m.mod) (void)hipModuleUnload(m.mod);
      return hip_fail(ctx, e, "loading the compiled theory");
    }
    ctx->rtc.push_back(m);
    fn = m.fn;
  }
  // the theory record: N0, Nbkg and the expression's references as resolved
  // scalars 0, 1, 2, ...; no terms (the built-in kernels never run it)
  mu_theory_desc td;
  std::memset(&td, 0, sizeof td);
  td.tau_mu = d->tau_mu;
  td.n0 = d->n0;
  td.nbkg = d->nbkg;
  td.map = d->map;
  td.n_rows = d->n_rows;
  td.n_slots = d->n_slots;
  td.F = d->F;
  td.f0 = d->f0;
  td.n_fun = d->n_fun;
  td.n_par = d->n_par;
  mu_theory *th = nullptr;
  if ((st = mu_theory_create(ctx, &td, &th)) != MU_OK) return st;
  for (size_t q = 0; q < P.refs.size(); ++q) {
    th->h.rref[2 + q].kind = P.refs[q].first;
    th->h.rref[2 + q].slot = P.refs[q].second;
    th->h.rref[2 + q].lit = 0.0;
  }
  th->rtc_fn = fn;
  th->rtc_refs = (int)P.refs.size();
  th->shape = kShapeGeneric;
  hipError_t e = hipMemcpy(th->d_th, &th->h, sizeof th->h, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    mu_theory_destroy(th);
    return hip_fail(ctx, e, "theory upload");
  }
  *out = th;
  return MU_OK;
}

namespace mu {

hipError_t launch_rtc(hipFunction_t fn, const LaunchArgs &a, int mode, int count_f64, hipStream_t s) {
  if (a.n_units <= 0) return hipSuccess;
  LaunchArgs arg = a;
  int m = mode, f = count_f64;
  void *params[] = {&arg, &m, &f};
  return hipModuleLaunchKernel(fn, (unsigned)((a.n_units + 3) / 4), 1, 1, kBlock, 1, 1, 0, s, params, nullptr);
}

}  // namespace mu
