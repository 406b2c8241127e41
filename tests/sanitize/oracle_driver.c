/* Host sanitizer driver for the CPU oracle (test infrastructure): every
 * public entry point of rbmc_oracle.c on small models, several
 * decompositions and overlaps.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer; any report aborts the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void* orc_model_create(int mx, int my, int T, double h, double log_kappa, double log_tau,
                       double rho, double log_sigma, const unsigned char* mask);
void orc_model_destroy(void* h);
int orc_model_csr_dims(void* h, int which, int64_t* dims);
int orc_model_csr(void* h, int which, int64_t* rp, int* ci, double* v);
void orc_grid_cores(int mx, int my, int T, int n_tslabs, int n_tiles_x, int n_tiles_y,
                    int* label);
int orc_subdomain_state(void* h, const int* label, int p, int n_l, unsigned char* state);
int orc_csr_logdet(int n, const int64_t* rp, const int* ci, const double* v, double* out);
int orc_model_sample(void* h, int n_k, const double* z, double* x);
int orc_model_rhs(void* h, int n_k, const double* z, double* b);
int orc_model_rbmc(void* h, const int* label, int n_parts, int n_l, int n_k, const double* x,
                   unsigned grad_mask, double* diag, double* diag_det, double* trace,
                   double* trace_det, double* err_est, int* fail_part);
int orc_model_cg(void* h, const unsigned char* sel, const double* b, double* x, double rtol,
                 int maxit);
int orc_model_entry(void* h, const int* label, int p, int n_l, int i, int n_k, const double* x,
                    double rtol, int maxit, double* out);
int orc_model_apply(void* h, int which, int n_rhs, const double* x, double* y);
int orc_model_nobs(void* h);

/* deterministic values in (-1, 1) */
static double val(uint64_t i) {
  uint64_t z = i * 0x9E3779B97F4A7C15ull;
  z ^= z >> 29;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 32;
  return (double)(z >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static int run(int mx, int my, int T, int P, int tx, int ty) {
  const int n = mx * my * T;
  unsigned char* mask = malloc((size_t)n);
  for (int i = 0; i < n; ++i) mask[i] = (val((uint64_t)i + 7) > 0.4);
  void* M = orc_model_create(mx, my, T, 1.0 / (mx - 1), 2.0, 0.0, 0.9, 0.0, mask);
  const int n_obs = orc_model_nobs(M);
  for (int which = 0; which < 6; ++which) {
    int64_t dims[3];
    if (orc_model_csr_dims(M, which, dims) != 0) continue;
    int64_t* rp = malloc(sizeof(int64_t) * (size_t)(dims[0] + 1));
    int* ci = malloc(sizeof(int) * (size_t)dims[2]);
    double* v = malloc(sizeof(double) * (size_t)dims[2]);
    orc_model_csr(M, which, rp, ci, v);
    if (which == 0) {
      double ld = 0.0;
      if (orc_csr_logdet((int)dims[0], rp, ci, v, &ld) != 0 || !isfinite(ld)) return 1;
    }
    free(rp);
    free(ci);
    free(v);
  }
  const int n_k = 5;
  double* z = malloc(sizeof(double) * (size_t)n_k * (n + n_obs));
  for (int64_t i = 0; i < (int64_t)n_k * (n + n_obs); ++i) z[i] = val((uint64_t)i);
  double* x = malloc(sizeof(double) * (size_t)n_k * n);
  double* b = malloc(sizeof(double) * (size_t)n_k * n);
  double* y = malloc(sizeof(double) * (size_t)n_k * (n + n_obs));
  if (orc_model_sample(M, n_k, z, x) != 0) return 2;
  orc_model_rhs(M, n_k, z, b);
  for (int which = 0; which < 6; ++which) orc_model_apply(M, which, 1, which == 5 ? z : x, y);
  int* label = malloc(sizeof(int) * (size_t)n);
  unsigned char* state = malloc((size_t)n);
  orc_grid_cores(mx, my, T, P, tx, ty, label);
  const int parts = P * tx * ty;
  double diag[4096], dd[4096], tr[4], trd[4], err = 0.0;
  if (n > 4096) return 3;
  for (int n_l = 0; n_l <= 2; ++n_l) {
    for (int p = 0; p < parts; ++p) orc_subdomain_state(M, label, p, n_l, state);
    int fail = -1;
    if (orc_model_rbmc(M, label, parts, n_l, n_k, x, 0xFu, diag, dd, tr, trd, &err, &fail) != 0)
      return 4;
    double out[2];
    if (orc_model_entry(M, label, parts - 1, n_l, n - 1, n_k, x, 1e-12, 100000, out) < 0) return 5;
  }
  unsigned char* sel = malloc((size_t)n);
  for (int i = 0; i < n; ++i) sel[i] = 1;
  double* cg = calloc((size_t)n, sizeof(double));
  if (orc_model_cg(M, sel, b, cg, 1e-12, 100000) < 0) return 6;
  free(sel);
  free(cg);
  free(label);
  free(state);
  free(z);
  free(x);
  free(b);
  free(y);
  free(mask);
  orc_model_destroy(M);
  return 0;
}

int main(void) {
  const int shapes[][6] = {{12, 10, 7, 3, 2, 2}, {9, 9, 5, 5, 1, 1}, {7, 7, 1, 1, 1, 1},
                           {16, 8, 6, 2, 3, 1}};
  for (int s = 0; s < 4; ++s) {
    const int* c = shapes[s];
    const int rc = run(c[0], c[1], c[2], c[3], c[4], c[5]);
    if (rc) {
      fprintf(stderr, "shape %d failed: %d\n", s, rc);
      return rc;
    }
  }
  printf("oracle driver ok\n");
  return 0;
}
