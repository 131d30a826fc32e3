/* A plain C99 caller of the library: header compiles as C, symbols link, the
 * device-free validators work.  Exit status 0 on success. */
#include <stdio.h>

#include "mu.h"

int main(void) {
  if (mu_abi_version() != MU_ABI_VERSION) return 1;
  double counts[4] = {3.0, 4.0, 0.0, 7.0};
  mu_histo h = {counts, 4, 0.01, 0.0, 0, 3, 0, 0};
  char msg[256];
  if (mu_histo_check(&h, 1, msg, sizeof msg) != MU_OK) return 2;
  h.last = 4;
  if (mu_histo_check(&h, 1, msg, sizeof msg) != MU_E_ARG) return 3;

  /* A(t) = A e^(-lambda t) cos(2 pi nu t + phi) with p = [N0, Nbkg, A, lambda, nu, phi] */
  mu_factor f[2];
  f[0].prim = MU_SE; f[0].reserved = 0;
  f[0].arg[0].kind = MU_REF_PAR; f[0].arg[0].slot = 3; f[0].arg[0].literal = 0.0;
  f[1].prim = MU_TF; f[1].reserved = 0;
  f[1].arg[0].kind = MU_REF_PAR; f[1].arg[0].slot = 5; f[1].arg[0].literal = 0.0;
  f[1].arg[1].kind = MU_REF_PAR; f[1].arg[1].slot = 4; f[1].arg[1].literal = 0.0;
  mu_term t;
  t.coef = 1.0;
  t.amp.kind = MU_REF_PAR; t.amp.slot = 2; t.amp.literal = 0.0;
  t.first_factor = 0; t.n_factors = 2;
  int32_t map[6] = {0, 1, 2, 3, 4, 5};
  mu_theory_desc d;
  d.tau_mu = 2.1969811;
  d.n0.kind = MU_REF_PAR; d.n0.slot = 0; d.n0.literal = 0.0;
  d.nbkg.kind = MU_REF_PAR; d.nbkg.slot = 1; d.nbkg.literal = 0.0;
  d.terms = &t; d.n_terms = 1; d.factors = f; d.n_factors = 2;
  d.map = map; d.n_rows = 1; d.n_slots = 6;
  d.F = NULL; d.f0 = NULL; d.n_fun = 0; d.n_par = 6;
  if (mu_theory_check(&d, msg, sizeof msg) != MU_OK) { fprintf(stderr, "%s\n", msg); return 4; }
  map[4] = 6; /* out of range parameter index */
  if (mu_theory_check(&d, msg, sizeof msg) != MU_E_ARG) return 5;

  mu_ctx *ctx = NULL;
  /* the caller sets MU_FORCE_NODEVICE=1 */
  if (mu_ctx_create(0, NULL, 0, &ctx) != MU_E_NODEVICE || ctx != NULL) return 6;
  printf("c consumer ok: %s\n", mu_status_string(MU_E_NODEVICE));
  return 0;
}
