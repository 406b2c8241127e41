/*
 * Plain FP64 CPU oracle for the overlapping Rao-Blackwellized Monte Carlo
 * (RBMC) estimator of diag(Q^-1) and tr(Q^-1 dQ/dtheta_j).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the package smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * helper with the HIP library; the two sides meet only in the seeded input
 * generator, which holds none of the method's arithmetic.
 *
 * Deliberately slow and literal:
 *   - every matrix is assembled explicitly (CSR) from its defining formula,
 *     with generic sparse add / multiply / Kronecker product;
 *   - the overlap is grown by literal breadth-first search on the CSR graph
 *     (Alg. 4 of the paper, overlapping RBMC for the diagonal);
 *   - Q_AA^-1 entries come from a banded Cholesky factor of Q_AA and one
 *     forward/back solve per needed column (the plain definition of the
 *     inverse; no Takahashi recursion, no block structure);
 *   - the correction solves mu = Q_AA^-1 Q_AB x_B use the same factor.
 * Compile with -ffp-contract=off; every reduction runs in a fixed order so
 * results are reproducible bit for bit on any thread count.
 *
 * Paper: Zhumekenov, Krainski, Rue, "Parallel Selected Inversion for
 * Space-Time Gaussian Markov Random Fields" (arXiv 2309.05435).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* CSR sparse matrices                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nr, nc;
  int64_t* rp; /* nr + 1 */
  int* ci;
  double* v;
} csr_t;

static void csr_free(csr_t* a) {
  free(a->rp);
  free(a->ci);
  free(a->v);
  a->rp = NULL;
  a->ci = NULL;
  a->v = NULL;
}

typedef struct {
  int i, j;
  double v;
  int64_t seq; /* insertion order: duplicates are summed in this order */
} trip_t;

static int trip_cmp(const void* a, const void* b) {
  const trip_t* x = (const trip_t*)a;
  const trip_t* y = (const trip_t*)b;
  if (x->i != y->i) return x->i < y->i ? -1 : 1;
  if (x->j != y->j) return x->j < y->j ? -1 : 1;
  if (x->seq != y->seq) return x->seq < y->seq ? -1 : 1;
  return 0;
}

/* Build CSR from triplets; duplicate (i,j) are summed in the order given.
 * Structural entries are kept even when their value is zero, so the graph of
 * a matrix never depends on the numerical value of a parameter. */
static csr_t csr_from_trips(int nr, int nc, int64_t nt, trip_t* t) {
  csr_t a;
  a.nr = nr;
  a.nc = nc;
  for (int64_t k = 0; k < nt; ++k) t[k].seq = k;
  qsort(t, (size_t)nt, sizeof(trip_t), trip_cmp);
  int64_t nu = 0;
  for (int64_t k = 0; k < nt; ++k) {
    if (nu > 0 && t[nu - 1].i == t[k].i && t[nu - 1].j == t[k].j)
      t[nu - 1].v += t[k].v;
    else
      t[nu++] = t[k];
  }
  a.rp = (int64_t*)calloc((size_t)nr + 1, sizeof(int64_t));
  a.ci = (int*)malloc(sizeof(int) * (size_t)(nu > 0 ? nu : 1));
  a.v = (double*)malloc(sizeof(double) * (size_t)(nu > 0 ? nu : 1));
  for (int64_t k = 0; k < nu; ++k) {
    a.rp[t[k].i + 1]++;
    a.ci[k] = t[k].j;
    a.v[k] = t[k].v;
  }
  for (int r = 0; r < nr; ++r) a.rp[r + 1] += a.rp[r];
  return a;
}

static csr_t csr_identity_scaled(int n, double s) {
  trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)n);
  for (int i = 0; i < n; ++i) {
    t[i].i = i;
    t[i].j = i;
    t[i].v = s;
  }
  csr_t a = csr_from_trips(n, n, n, t);
  free(t);
  return a;
}

/* a*A + b*B */
static csr_t csr_axpby(double a, const csr_t* A, double b, const csr_t* B) {
  int64_t na = A->rp[A->nr], nb = B->rp[B->nr];
  trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)(na + nb + 1));
  int64_t k = 0;
  for (int r = 0; r < A->nr; ++r)
    for (int64_t q = A->rp[r]; q < A->rp[r + 1]; ++q) {
      t[k].i = r;
      t[k].j = A->ci[q];
      t[k].v = a * A->v[q];
      ++k;
    }
  for (int r = 0; r < B->nr; ++r)
    for (int64_t q = B->rp[r]; q < B->rp[r + 1]; ++q) {
      t[k].i = r;
      t[k].j = B->ci[q];
      t[k].v = b * B->v[q];
      ++k;
    }
  csr_t c = csr_from_trips(A->nr, A->nc, k, t);
  free(t);
  return c;
}

/* A * B (row by row, products summed in increasing order of the inner index) */
static csr_t csr_matmul(const csr_t* A, const csr_t* B) {
  int64_t cap = 1024, k = 0;
  trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)cap);
  for (int r = 0; r < A->nr; ++r)
    for (int64_t q = A->rp[r]; q < A->rp[r + 1]; ++q) {
      int mid = A->ci[q];
      for (int64_t u = B->rp[mid]; u < B->rp[mid + 1]; ++u) {
        if (k == cap) {
          cap *= 2;
          t = (trip_t*)realloc(t, sizeof(trip_t) * (size_t)cap);
        }
        t[k].i = r;
        t[k].j = B->ci[u];
        t[k].v = A->v[q] * B->v[u];
        ++k;
      }
    }
  csr_t c = csr_from_trips(A->nr, B->nc, k, t);
  free(t);
  return c;
}

/* Kronecker product A (x) B: entry ((ia*B.nr+ib),(ja*B.nc+jb)) = A_ia,ja B_ib,jb */
static csr_t csr_kron(const csr_t* A, const csr_t* B) {
  int64_t nt = A->rp[A->nr] * B->rp[B->nr];
  trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)(nt + 1));
  int64_t k = 0;
  for (int ia = 0; ia < A->nr; ++ia)
    for (int64_t qa = A->rp[ia]; qa < A->rp[ia + 1]; ++qa)
      for (int ib = 0; ib < B->nr; ++ib)
        for (int64_t qb = B->rp[ib]; qb < B->rp[ib + 1]; ++qb) {
          t[k].i = ia * B->nr + ib;
          t[k].j = A->ci[qa] * B->nc + B->ci[qb];
          t[k].v = A->v[qa] * B->v[qb];
          ++k;
        }
  csr_t c = csr_from_trips(A->nr * B->nr, A->nc * B->nc, k, t);
  free(t);
  return c;
}

static csr_t csr_copy_raw(int nr, int nc, const int64_t* rp, const int* ci, const double* v) {
  csr_t a;
  a.nr = nr;
  a.nc = nc;
  int64_t nz = rp[nr];
  a.rp = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nr + 1));
  a.ci = (int*)malloc(sizeof(int) * (size_t)(nz > 0 ? nz : 1));
  a.v = (double*)malloc(sizeof(double) * (size_t)(nz > 0 ? nz : 1));
  memcpy(a.rp, rp, sizeof(int64_t) * ((size_t)nr + 1));
  memcpy(a.ci, ci, sizeof(int) * (size_t)nz);
  memcpy(a.v, v, sizeof(double) * (size_t)nz);
  return a;
}

static double csr_get(const csr_t* A, int i, int j) {
  for (int64_t q = A->rp[i]; q < A->rp[i + 1]; ++q)
    if (A->ci[q] == j) return A->v[q];
  return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Space-time SPDE model                                                     */
/*                                                                           */
/* Spatial precision, alpha = 2, tau-linear reading, lumped mass C = h^2 I:  */
/*   Q_s = tau (kappa^4 C + 2 kappa^2 G + G C^-1 G)   (Sec. 2.1, eq:spde:2-4)*/
/* G = stiffness of the unit grid = graph Laplacian of the 4-neighbour grid. */
/* Temporal precision: stationary AR(1) with unit marginal variance,         */
/* Q_t = L^T L with L x = standardized innovations.                          */
/* Q_u = Q_t (x) Q_s  (separable Kronecker model, Sec. 2.2)                  */
/* Q   = Q_u + A^T Q_y A, A selects observed nodes, Q_y = sigma^-2 I          */
/*                                                   (Sec. 2.3, eq:lgm:2)    */
/* ------------------------------------------------------------------------ */

typedef struct {
  int mx, my, T;
  double h, kappa, tau, rho, sigma;
  int n_s, n, n_obs;
  csr_t G, Qs, dQs_logkappa, Qt, dQt_rho, Lt, Fs;
  csr_t Q, dQ[4]; /* d/dlogkappa, d/dlogtau, d/drho, d/dlogsigma */
  csr_t F;        /* n x (n + n_obs): b = F [z1; z2] */
  unsigned char* mask;
} orc_model;

static csr_t grid_laplacian(int mx, int my) {
  int n = mx * my;
  trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)(8 * n + 1));
  int64_t k = 0;
  for (int iy = 0; iy < my; ++iy)
    for (int ix = 0; ix < mx; ++ix) {
      int i = iy * mx + ix;
      const int dx[4] = {-1, 1, 0, 0}, dy[4] = {0, 0, -1, 1};
      for (int d = 0; d < 4; ++d) {
        int jx = ix + dx[d], jy = iy + dy[d];
        if (jx < 0 || jx >= mx || jy < 0 || jy >= my) continue;
        t[k].i = i;
        t[k].j = jy * mx + jx;
        t[k].v = -1.0;
        ++k;
        t[k].i = i;
        t[k].j = i;
        t[k].v = 1.0;
        ++k;
      }
    }
  csr_t g = csr_from_trips(n, n, k, t);
  free(t);
  return g;
}

/* innovation map of the stationary unit-variance AR(1):
 * (L x)_0 = x_0, (L x)_t = (x_t - rho x_{t-1}) / sqrt(1 - rho^2) */
static csr_t ar1_innovation(int T, double rho) {
  trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)(2 * T + 1));
  int64_t k = 0;
  double s = 1.0 / sqrt(1.0 - rho * rho);
  for (int i = 0; i < T; ++i) {
    t[k].i = i;
    t[k].j = i;
    t[k].v = (i == 0) ? 1.0 : s;
    ++k;
    if (i > 0) {
      t[k].i = i;
      t[k].j = i - 1;
      t[k].v = -rho * s;
      ++k;
    }
  }
  csr_t l = csr_from_trips(T, T, k, t);
  free(t);
  return l;
}

static csr_t csr_transpose(const csr_t* A) {
  int64_t nz = A->rp[A->nr];
  trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)(nz + 1));
  int64_t k = 0;
  for (int r = 0; r < A->nr; ++r)
    for (int64_t q = A->rp[r]; q < A->rp[r + 1]; ++q) {
      t[k].i = A->ci[q];
      t[k].j = r;
      t[k].v = A->v[q];
      ++k;
    }
  csr_t c = csr_from_trips(A->nc, A->nr, k, t);
  free(t);
  return c;
}

void* orc_model_create(int mx, int my, int T, double h, double log_kappa, double log_tau,
                       double rho, double log_sigma, const unsigned char* mask) {
  orc_model* M = (orc_model*)calloc(1, sizeof(orc_model));
  M->mx = mx;
  M->my = my;
  M->T = T;
  M->h = h;
  M->kappa = exp(log_kappa);
  M->tau = exp(log_tau);
  M->rho = rho;
  M->sigma = exp(log_sigma);
  M->n_s = mx * my;
  M->n = M->n_s * T;
  M->mask = (unsigned char*)malloc((size_t)M->n);
  memcpy(M->mask, mask, (size_t)M->n);
  M->n_obs = 0;
  for (int i = 0; i < M->n; ++i) M->n_obs += mask[i] ? 1 : 0;

  const double k2 = M->kappa * M->kappa, k4 = k2 * k2, tau = M->tau, h2 = h * h;
  const int ns = M->n_s, n = M->n;

  /* spatial */
  M->G = grid_laplacian(mx, my);
  csr_t C = csr_identity_scaled(ns, h2);
  csr_t Cinv = csr_identity_scaled(ns, 1.0 / h2);
  csr_t GCi = csr_matmul(&M->G, &Cinv);
  csr_t GCiG = csr_matmul(&GCi, &M->G);
  csr_t t1 = csr_axpby(k4, &C, 2.0 * k2, &M->G);
  M->Qs = csr_axpby(tau, &t1, tau, &GCiG);
  /* d/dlog kappa of tau(kappa^4 C + 2 kappa^2 G + G C^-1 G) = tau(4 kappa^4 C + 4 kappa^2 G) */
  M->dQs_logkappa = csr_axpby(4.0 * k4 * tau, &C, 4.0 * k2 * tau, &M->G);
  /* square root F_s = sqrt(tau) (kappa^2 C + G) C^{-1/2}: F_s F_s^T = Q_s */
  csr_t KC = csr_axpby(k2, &C, 1.0, &M->G);
  csr_t Cmh = csr_identity_scaled(ns, 1.0 / h);
  csr_t KCm = csr_matmul(&KC, &Cmh);
  csr_t zero = csr_identity_scaled(ns, 0.0);
  M->Fs = csr_axpby(sqrt(tau), &KCm, 0.0, &zero);

  /* temporal */
  M->Lt = ar1_innovation(T, rho);
  csr_t LtT = csr_transpose(&M->Lt);
  M->Qt = csr_matmul(&LtT, &M->Lt);
  {
    /* Q_t = R / (1 - rho^2), R = tridiag(-rho; 1, 1+rho^2, ..., 1+rho^2, 1; -rho)
     * dQ_t/drho = dR/drho / (1-rho^2) + 2 rho R / (1-rho^2)^2 */
    trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)(3 * T + 1));
    int64_t k = 0;
    const double a = 1.0 - rho * rho;
    for (int i = 0; i < T; ++i) {
      double R_ii = (i == 0 || i == T - 1) ? 1.0 : 1.0 + rho * rho;
      double dR_ii = (i == 0 || i == T - 1) ? 0.0 : 2.0 * rho;
      t[k].i = i;
      t[k].j = i;
      /* a single step has Q_t = [1], independent of rho */
      t[k].v = (T == 1) ? 0.0 : dR_ii / a + 2.0 * rho * R_ii / (a * a);
      ++k;
      if (i + 1 < T) {
        t[k].i = i;
        t[k].j = i + 1;
        t[k].v = -1.0 / a + 2.0 * rho * (-rho) / (a * a);
        ++k;
        t[k].i = i + 1;
        t[k].j = i;
        t[k].v = -1.0 / a + 2.0 * rho * (-rho) / (a * a);
        ++k;
      }
    }
    M->dQt_rho = csr_from_trips(T, T, k, t);
    free(t);
  }

  /* space-time */
  csr_t Qu = csr_kron(&M->Qt, &M->Qs);
  double* dvals = (double*)malloc(sizeof(double) * (size_t)n);
  for (int i = 0; i < n; ++i) dvals[i] = mask[i] ? 1.0 / (M->sigma * M->sigma) : 0.0;
  trip_t* td = (trip_t*)malloc(sizeof(trip_t) * (size_t)n);
  for (int i = 0; i < n; ++i) {
    td[i].i = i;
    td[i].j = i;
    td[i].v = dvals[i];
  }
  csr_t D = csr_from_trips(n, n, n, td);
  free(td);
  M->Q = csr_axpby(1.0, &Qu, 1.0, &D);
  M->dQ[0] = csr_kron(&M->Qt, &M->dQs_logkappa);
  M->dQ[1] = csr_axpby(1.0, &Qu, 0.0, &Qu);
  M->dQ[2] = csr_kron(&M->dQt_rho, &M->Qs);
  M->dQ[3] = csr_axpby(-2.0, &D, 0.0, &D);

  /* perturbation sampler map b = (F_t (x) F_s) z1 + A^T Q_y^{1/2} z2 with F_t = L^T */
  csr_t Ft = LtT;
  csr_t Fst = csr_kron(&Ft, &M->Fs);
  {
    int64_t nz = Fst.rp[n] + M->n_obs;
    trip_t* t = (trip_t*)malloc(sizeof(trip_t) * (size_t)(nz + 1));
    int64_t k = 0;
    for (int r = 0; r < n; ++r)
      for (int64_t q = Fst.rp[r]; q < Fst.rp[r + 1]; ++q) {
        t[k].i = r;
        t[k].j = Fst.ci[q];
        t[k].v = Fst.v[q];
        ++k;
      }
    int j = 0;
    for (int r = 0; r < n; ++r)
      if (mask[r]) {
        t[k].i = r;
        t[k].j = n + j;
        t[k].v = 1.0 / M->sigma;
        ++k;
        ++j;
      }
    M->F = csr_from_trips(n, n + M->n_obs, k, t);
    free(t);
  }
  csr_free(&Fst);
  csr_free(&Ft);
  csr_free(&Qu);
  csr_free(&D);
  free(dvals);
  csr_free(&C);
  csr_free(&Cinv);
  csr_free(&GCi);
  csr_free(&GCiG);
  csr_free(&t1);
  csr_free(&KC);
  csr_free(&Cmh);
  csr_free(&KCm);
  csr_free(&zero);
  return M;
}

void orc_model_destroy(void* h) {
  orc_model* M = (orc_model*)h;
  if (!M) return;
  csr_free(&M->G);
  csr_free(&M->Qs);
  csr_free(&M->dQs_logkappa);
  csr_free(&M->Qt);
  csr_free(&M->dQt_rho);
  csr_free(&M->Lt);
  csr_free(&M->Fs);
  csr_free(&M->Q);
  for (int j = 0; j < 4; ++j) csr_free(&M->dQ[j]);
  csr_free(&M->F);
  free(M->mask);
  free(M);
}

/* which: 0 = Q, 1..4 = dQ/d(log kappa, log tau, rho, log sigma), 5 = F,
 * 6 = Q_s, 7 = Q_t, 8 = G */
static const csr_t* model_mat(const orc_model* M, int which) {
  switch (which) {
    case 0: return &M->Q;
    case 1: return &M->dQ[0];
    case 2: return &M->dQ[1];
    case 3: return &M->dQ[2];
    case 4: return &M->dQ[3];
    case 5: return &M->F;
    case 6: return &M->Qs;
    case 7: return &M->Qt;
    case 8: return &M->G;
    default: return NULL;
  }
}

/* dims[0] = rows, dims[1] = cols, dims[2] = nnz */
int orc_model_csr_dims(void* h, int which, int64_t* dims) {
  const csr_t* A = model_mat((orc_model*)h, which);
  if (!A) return -1;
  dims[0] = A->nr;
  dims[1] = A->nc;
  dims[2] = A->rp[A->nr];
  return 0;
}

int orc_model_csr(void* h, int which, int64_t* rp, int* ci, double* v) {
  const csr_t* A = model_mat((orc_model*)h, which);
  if (!A) return -1;
  memcpy(rp, A->rp, sizeof(int64_t) * ((size_t)A->nr + 1));
  memcpy(ci, A->ci, sizeof(int) * (size_t)A->rp[A->nr]);
  memcpy(v, A->v, sizeof(double) * (size_t)A->rp[A->nr]);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Partition of the space-time grid into cores (time slabs x spatial boxes)  */
/* ------------------------------------------------------------------------ */

/* split [0, len) into parts pieces: the first (len mod parts) get one more */
static int piece_of(int idx, int len, int parts) {
  int base = len / parts, extra = len % parts;
  int big = extra * (base + 1);
  if (idx < big) return idx / (base + 1);
  return extra + (idx - big) / base;
}

void orc_grid_cores(int mx, int my, int T, int n_tslabs, int n_tiles_x, int n_tiles_y,
                    int* label) {
  int ns = mx * my;
  for (int t = 0; t < T; ++t)
    for (int iy = 0; iy < my; ++iy)
      for (int ix = 0; ix < mx; ++ix) {
        int p = (piece_of(t, T, n_tslabs) * n_tiles_y + piece_of(iy, my, n_tiles_y)) * n_tiles_x +
                piece_of(ix, mx, n_tiles_x);
        label[t * ns + iy * mx + ix] = p;
      }
}

/* ------------------------------------------------------------------------ */
/* Overlap growth by breadth-first search (Alg. 4, first phase):             */
/*   Omega* = Omega_p; S = N(Omega*) \ Omega*; repeat n_l times:             */
/*   Omega* = Omega* u S; S = N(Omega*) \ Omega*.                             */
/* state[i] = 1 core, 2 overlap (in Omega* but not core), 3 separator, 0 out */
/* ------------------------------------------------------------------------ */

static void grow_overlap(const csr_t* Q, const int* label, int p, int n_l, unsigned char* state) {
  int n = Q->nr;
  memset(state, 0, (size_t)n);
  for (int i = 0; i < n; ++i)
    if (label[i] == p) state[i] = 1;
  /* S = N(Omega*) \ Omega* */
  for (int l = 0; l <= n_l; ++l) {
    unsigned char* nb = (unsigned char*)calloc((size_t)n, 1);
    for (int i = 0; i < n; ++i)
      if (state[i] == 1 || state[i] == 2)
        for (int64_t q = Q->rp[i]; q < Q->rp[i + 1]; ++q) {
          int j = Q->ci[q];
          if (state[j] == 0) nb[j] = 1;
        }
    for (int i = 0; i < n; ++i)
      if (nb[i]) state[i] = (l < n_l) ? 2 : 3;
    free(nb);
  }
}

/* state per node for subdomain p; returns 0 */
int orc_subdomain_state(void* h, const int* label, int p, int n_l, unsigned char* state) {
  orc_model* M = (orc_model*)h;
  grow_overlap(&M->Q, label, p, n_l, state);
  return 0;
}

int orc_csr_subdomain_state(int n, const int64_t* rp, const int* ci, const double* v,
                            const int* label, int p, int n_l, unsigned char* state) {
  csr_t Q = csr_copy_raw(n, n, rp, ci, v);
  grow_overlap(&Q, label, p, n_l, state);
  csr_free(&Q);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Banded Cholesky (entries outside the band of the matrix are zero)          */
/* Lb[i*(bw+1) + (i-j)] = L_ij for max(0,i-bw) <= j <= i                      */
/* ------------------------------------------------------------------------ */

static int band_chol(int N, int bw, double* Lb) {
  const int w = bw + 1;
  for (int i = 0; i < N; ++i) {
    int j0 = i - bw > 0 ? i - bw : 0;
    for (int j = j0; j <= i; ++j) {
      double s = Lb[(int64_t)i * w + (i - j)];
      int k0 = j - bw > j0 ? j - bw : j0;
      for (int k = k0; k < j; ++k) s -= Lb[(int64_t)i * w + (i - k)] * Lb[(int64_t)j * w + (j - k)];
      if (j == i) {
        if (!(s > 0.0)) return -(i + 1);
        Lb[(int64_t)i * w] = sqrt(s);
      } else {
        Lb[(int64_t)i * w + (i - j)] = s / Lb[(int64_t)j * w];
      }
    }
  }
  return 0;
}

/* solve (L L^T) x = b in place */
static void band_solve(int N, int bw, const double* Lb, double* x) {
  const int w = bw + 1;
  for (int i = 0; i < N; ++i) {
    double s = x[i];
    int k0 = i - bw > 0 ? i - bw : 0;
    for (int k = k0; k < i; ++k) s -= Lb[(int64_t)i * w + (i - k)] * x[k];
    x[i] = s / Lb[(int64_t)i * w];
  }
  for (int i = N - 1; i >= 0; --i) {
    double s = x[i];
    int k1 = i + bw < N - 1 ? i + bw : N - 1;
    for (int k = i + 1; k <= k1; ++k) s -= Lb[(int64_t)k * w + (k - i)] * x[k];
    x[i] = s / Lb[(int64_t)i * w];
  }
}

/* Banded Cholesky of the principal submatrix Q[idx, idx] (idx ascending).
 * loc[g] = local index of global g, or -1. Returns factor (caller frees). */
static double* factor_principal(const csr_t* Q, int N, const int* idx, const int* loc, int* bw_out,
                                int* info) {
  int bw = 0;
  for (int a = 0; a < N; ++a) {
    int g = idx[a];
    for (int64_t q = Q->rp[g]; q < Q->rp[g + 1]; ++q) {
      int b = loc[Q->ci[q]];
      if (b >= 0 && a - b > bw) bw = a - b;
    }
  }
  const int w = bw + 1;
  double* Lb = (double*)calloc((size_t)N * (size_t)w, sizeof(double));
  for (int a = 0; a < N; ++a) {
    int g = idx[a];
    for (int64_t q = Q->rp[g]; q < Q->rp[g + 1]; ++q) {
      int b = loc[Q->ci[q]];
      if (b >= 0 && b <= a) Lb[(int64_t)a * w + (a - b)] += Q->v[q];
    }
  }
  *info = band_chol(N, bw, Lb);
  *bw_out = bw;
  return Lb;
}

/* log det of the full matrix via banded Cholesky; returns 0 or -(row+1) */
int orc_csr_logdet(int n, const int64_t* rp, const int* ci, const double* v, double* out) {
  csr_t Q = csr_copy_raw(n, n, rp, ci, v);
  int* idx = (int*)malloc(sizeof(int) * (size_t)n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  int bw, info;
  double* Lb = factor_principal(&Q, n, idx, idx, &bw, &info);
  double s = 0.0;
  if (info == 0)
    for (int i = 0; i < n; ++i) s += 2.0 * log(Lb[(int64_t)i * (bw + 1)]);
  *out = s;
  free(Lb);
  free(idx);
  csr_free(&Q);
  return info;
}

/* ------------------------------------------------------------------------ */
/* Exact sampling x ~ N(0, Q^-1) by perturbation (Sec. 2.4 / Sec. 3.3):      */
/*   b = F z,  F F^T = Q,  x = Q^-1 b  (banded Cholesky of the full Q)        */
/* z: n_k x ncols(F) row-major; x: n_k x n row-major                          */
/* ------------------------------------------------------------------------ */

int orc_model_sample(void* h, int n_k, const double* z, double* x) {
  orc_model* M = (orc_model*)h;
  const int n = M->n, nz = M->n + M->n_obs;
  int* idx = (int*)malloc(sizeof(int) * (size_t)n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  int bw, info;
  double* Lb = factor_principal(&M->Q, n, idx, idx, &bw, &info);
  if (info == 0) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < n_k; ++k) {
      double* xk = x + (int64_t)k * n;
      const double* zk = z + (int64_t)k * nz;
      for (int r = 0; r < n; ++r) {
        double s = 0.0;
        for (int64_t q = M->F.rp[r]; q < M->F.rp[r + 1]; ++q) s += M->F.v[q] * zk[M->F.ci[q]];
        xk[r] = s;
      }
      band_solve(n, bw, Lb, xk);
    }
  }
  free(Lb);
  free(idx);
  return info;
}

/* b = F z only (perturbation right-hand side) */
int orc_model_rhs(void* h, int n_k, const double* z, double* b) {
  orc_model* M = (orc_model*)h;
  const int n = M->n, nz = M->n + M->n_obs;
  for (int k = 0; k < n_k; ++k)
    for (int r = 0; r < n; ++r) {
      double s = 0.0;
      for (int64_t q = M->F.rp[r]; q < M->F.rp[r + 1]; ++q) s += M->F.v[q] * z[(int64_t)k * nz + M->F.ci[q]];
      b[(int64_t)k * n + r] = s;
    }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Overlapping RBMC for the diagonal and the traces                          */
/*   (Alg. 4 for diag; Alg. 3 off-diagonal rows + eq:hyperpar:4 for traces)  */
/*                                                                           */
/* For each core p with extension A = Omega_p* and separator B = S_p:        */
/*   diag_i  = (Q_AA^-1)_ii + (1/n_k) sum_k (mu^(k)_i)^2,  i in Omega_p      */
/*   mu^(k)  = Q_AA^-1 Q_AB x^(k)_B                                          */
/*   trace_j += sum_{i in Omega_p} sum_{c in A} [(Q_AA^-1)_ic                */
/*              + (1/n_k) sum_k mu^(k)_i mu^(k)_c] (dQ_j)_ic                 */
/* Samples x: n_k x n row-major (one global set shared by every p).          */
/* Outputs: diag (n), diag_det (n) = (Q_AA^-1)_ii part, trace (n_dq),        */
/* trace_det (n_dq), and plug-in MC error estimate (mean over i of           */
/* sqrt(2/pi) sqrt(2/n_k) m_i / diag_i, m_i = (1/n_k) sum_k mu_i^2).         */
/* ------------------------------------------------------------------------ */

static int rbmc_core(const csr_t* Q, int n_dq, const csr_t* const* dQ, const int* label, int n_parts,
                     int n_l, int n_k, const double* x, double* diag, double* diag_det,
                     double* trace, double* trace_det, double* err_est, int* fail_part) {
  const int n = Q->nr;
  for (int j = 0; j < n_dq; ++j) {
    trace[j] = 0.0;
    trace_det[j] = 0.0;
  }
  double err_sum = 0.0;
  int status = 0;
  unsigned char* state = (unsigned char*)malloc((size_t)n);
  int* loc = (int*)malloc(sizeof(int) * (size_t)n);
  for (int i = 0; i < n; ++i) loc[i] = -1;

  for (int p = 0; p < n_parts; ++p) {
    grow_overlap(Q, label, p, n_l, state);
    int N = 0, Nc = 0;
    for (int i = 0; i < n; ++i)
      if (state[i] == 1 || state[i] == 2) ++N;
    int* idx = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    int* core = (int*)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    N = 0;
    for (int i = 0; i < n; ++i)
      if (state[i] == 1 || state[i] == 2) {
        loc[i] = N;
        idx[N++] = i;
        if (state[i] == 1) core[Nc++] = i;
      }
    if (Nc == 0) {
      for (int a = 0; a < N; ++a) loc[idx[a]] = -1;
      free(idx);
      free(core);
      continue;
    }
    int bw, info;
    double* Lb = factor_principal(Q, N, idx, loc, &bw, &info);
    if (info != 0) {
      status = -2;
      if (fail_part) *fail_part = p;
      free(Lb);
      for (int a = 0; a < N; ++a) loc[idx[a]] = -1;
      free(idx);
      free(core);
      break;
    }
    /* deterministic part: one column of Q_AA^-1 per core row */
    double* cdiag = (double*)malloc(sizeof(double) * (size_t)Nc);
    double* ctr = (double*)calloc((size_t)Nc * (size_t)(n_dq > 0 ? n_dq : 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
    for (int c = 0; c < Nc; ++c) {
      double* col = (double*)calloc((size_t)N, sizeof(double));
      int i = core[c];
      col[loc[i]] = 1.0;
      band_solve(N, bw, Lb, col);
      cdiag[c] = col[loc[i]];
      for (int j = 0; j < n_dq; ++j) {
        double s = 0.0;
        const csr_t* D = dQ[j];
        for (int64_t q = D->rp[i]; q < D->rp[i + 1]; ++q) {
          int b = loc[D->ci[q]];
          if (b >= 0) s += col[b] * D->v[q];
        }
        ctr[(int64_t)c * n_dq + j] = s;
      }
      free(col);
    }
    /* Monte Carlo part: mu^(k) = Q_AA^-1 Q_AB x_B^(k) */
    double* mu = (double*)calloc((size_t)N * (size_t)(n_k > 0 ? n_k : 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < n_k; ++k) {
      double* m = mu + (int64_t)k * N;
      const double* xk = x + (int64_t)k * n;
      for (int a = 0; a < N; ++a) {
        int g = idx[a];
        double s = 0.0;
        for (int64_t q = Q->rp[g]; q < Q->rp[g + 1]; ++q) {
          int col = Q->ci[q];
          if (state[col] == 3) s += Q->v[q] * xk[col];
        }
        m[a] = s;
      }
      band_solve(N, bw, Lb, m);
    }
    /* accumulate in a fixed order */
    for (int c = 0; c < Nc; ++c) {
      int i = core[c];
      double msq = 0.0;
      for (int k = 0; k < n_k; ++k) {
        double v = mu[(int64_t)k * N + loc[i]];
        msq += v * v;
      }
      double mbar = n_k > 0 ? msq / n_k : 0.0;
      diag_det[i] = cdiag[c];
      diag[i] = cdiag[c] + mbar;
      if (n_k > 0 && diag[i] > 0.0)
        err_sum += sqrt(2.0 / ORC_PI) * sqrt(2.0 / n_k) * mbar / diag[i];
      for (int j = 0; j < n_dq; ++j) {
        trace_det[j] += ctr[(int64_t)c * n_dq + j];
        trace[j] += ctr[(int64_t)c * n_dq + j];
        if (n_k > 0) {
          const csr_t* D = dQ[j];
          double s = 0.0;
          for (int k = 0; k < n_k; ++k) {
            const double* m = mu + (int64_t)k * N;
            double dm = 0.0;
            for (int64_t q = D->rp[i]; q < D->rp[i + 1]; ++q) {
              int b = loc[D->ci[q]];
              if (b >= 0) dm += D->v[q] * m[b];
            }
            s += m[loc[i]] * dm;
          }
          trace[j] += s / n_k;
        }
      }
    }
    free(mu);
    free(cdiag);
    free(ctr);
    free(Lb);
    for (int a = 0; a < N; ++a) loc[idx[a]] = -1;
    free(idx);
    free(core);
  }
  if (err_est) *err_est = err_sum / (n > 0 ? n : 1);
  free(loc);
  free(state);
  return status;
}

/* Model entry: dQ for the bits of grad_mask (bit0 log kappa, bit1 log tau,
 * bit2 rho, bit3 log sigma), traces written in that order. */
int orc_model_rbmc(void* h, const int* label, int n_parts, int n_l, int n_k, const double* x,
                   unsigned grad_mask, double* diag, double* diag_det, double* trace,
                   double* trace_det, double* err_est, int* fail_part) {
  orc_model* M = (orc_model*)h;
  const csr_t* dq[4];
  int nd = 0;
  for (int j = 0; j < 4; ++j)
    if (grad_mask & (1u << j)) dq[nd++] = &M->dQ[j];
  return rbmc_core(&M->Q, nd, dq, label, n_parts, n_l, n_k, x, diag, diag_det, trace, trace_det,
                   err_est, fail_part);
}

/* Generic entry on any SPD CSR matrix (used for the paper's AR(1) example). */
int orc_csr_rbmc(int n, const int64_t* rp, const int* ci, const double* v, int n_dq,
                 const int64_t* const* drp, const int* const* dci, const double* const* dv,
                 const int* label, int n_parts, int n_l, int n_k, const double* x, double* diag,
                 double* diag_det, double* trace, double* trace_det, double* err_est,
                 int* fail_part) {
  csr_t Q = csr_copy_raw(n, n, rp, ci, v);
  csr_t* D = (csr_t*)malloc(sizeof(csr_t) * (size_t)(n_dq > 0 ? n_dq : 1));
  const csr_t** dq = (const csr_t**)malloc(sizeof(csr_t*) * (size_t)(n_dq > 0 ? n_dq : 1));
  for (int j = 0; j < n_dq; ++j) {
    D[j] = csr_copy_raw(n, n, drp[j], dci[j], dv[j]);
    dq[j] = &D[j];
  }
  int st = rbmc_core(&Q, n_dq, dq, label, n_parts, n_l, n_k, x, diag, diag_det, trace, trace_det,
                     err_est, fail_part);
  for (int j = 0; j < n_dq; ++j) csr_free(&D[j]);
  free(D);
  free(dq);
  csr_free(&Q);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Single entries at any size: plain conjugate gradients on Q restricted to  */
/* a node set (all nodes if sel == NULL), used to check sampled outputs of   */
/* large runs one by one.  Returns iterations used (or -1 if not converged). */
/* ------------------------------------------------------------------------ */

static int cg_restricted(const csr_t* Q, const unsigned char* sel, const double* b, double* x,
                         double rtol, int maxit) {
  const int n = Q->nr;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* p = (double*)malloc(sizeof(double) * (size_t)n);
  double* q = (double*)malloc(sizeof(double) * (size_t)n);
  double bb = 0.0;
  for (int i = 0; i < n; ++i) {
    x[i] = 0.0;
    r[i] = (sel == NULL || sel[i]) ? b[i] : 0.0;
    p[i] = r[i];
    bb += r[i] * r[i];
  }
  double rr = bb;
  int it = 0, ok = (bb == 0.0);
  while (!ok && it < maxit) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      if (sel == NULL || sel[i])
        for (int64_t k = Q->rp[i]; k < Q->rp[i + 1]; ++k) {
          int c = Q->ci[k];
          if (sel == NULL || sel[c]) s += Q->v[k] * p[c];
        }
      q[i] = s;
    }
    double pq = 0.0;
    for (int i = 0; i < n; ++i) pq += p[i] * q[i];
    double alpha = rr / pq, rr2 = 0.0;
    for (int i = 0; i < n; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
      rr2 += r[i] * r[i];
    }
    ++it;
    if (sqrt(rr2) <= rtol * sqrt(bb)) ok = 1;
    double beta = rr2 / rr;
    rr = rr2;
    for (int i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
  }
  free(r);
  free(p);
  free(q);
  return ok ? it : -1;
}

/* Solve Q[sel,sel] x = b[sel] (sel == NULL: the full Q). */
int orc_model_cg(void* h, const unsigned char* sel, const double* b, double* x, double rtol,
                 int maxit) {
  return cg_restricted(&((orc_model*)h)->Q, sel, b, x, rtol, maxit);
}

/* The estimator at a single node i of core p, at any size:
 *   y = Q_AA^-1 e_i (conjugate gradients on Q_AA),
 *   det = y_i = (Q_AA^-1)_ii,  mu^(k)_i = y^T Q_AB x_B^(k),
 *   out[0] = det, out[1] = det + (1/n_k) sum_k (mu^(k)_i)^2.
 * Returns CG iterations, or -1 if CG did not reach rtol. */
int orc_model_entry(void* h, const int* label, int p, int n_l, int i, int n_k, const double* x,
                    double rtol, int maxit, double* out) {
  orc_model* M = (orc_model*)h;
  const csr_t* Q = &M->Q;
  const int n = Q->nr;
  unsigned char* state = (unsigned char*)malloc((size_t)n);
  unsigned char* sel = (unsigned char*)malloc((size_t)n);
  grow_overlap(Q, label, p, n_l, state);
  for (int a = 0; a < n; ++a) sel[a] = (state[a] == 1 || state[a] == 2);
  double* e = (double*)calloc((size_t)n, sizeof(double));
  double* y = (double*)calloc((size_t)n, sizeof(double));
  e[i] = 1.0;
  int it = cg_restricted(Q, sel, e, y, rtol, maxit);
  double det = y[i], msq = 0.0;
  for (int k = 0; k < n_k; ++k) {
    const double* xk = x + (int64_t)k * n;
    double mu = 0.0;
    for (int a = 0; a < n; ++a) {
      if (!sel[a] || y[a] == 0.0) continue;
      double r = 0.0;
      for (int64_t q = Q->rp[a]; q < Q->rp[a + 1]; ++q)
        if (state[Q->ci[q]] == 3) r += Q->v[q] * xk[Q->ci[q]];
      mu += y[a] * r;
    }
    msq += mu * mu;
  }
  out[0] = det;
  out[1] = det + (n_k > 0 ? msq / n_k : 0.0);
  free(state);
  free(sel);
  free(e);
  free(y);
  return it;
}

/* y = Op x for Op in {Q, dQ_j, F}; x has ncols entries per rhs */
int orc_model_apply(void* h, int which, int n_rhs, const double* x, double* y) {
  const csr_t* A = model_mat((orc_model*)h, which);
  if (!A) return -1;
  for (int k = 0; k < n_rhs; ++k)
    for (int r = 0; r < A->nr; ++r) {
      double s = 0.0;
      for (int64_t q = A->rp[r]; q < A->rp[r + 1]; ++q) s += A->v[q] * x[(int64_t)k * A->nc + A->ci[q]];
      y[(int64_t)k * A->nr + r] = s;
    }
  return 0;
}

int orc_model_nobs(void* h) { return ((orc_model*)h)->n_obs; }
double orc_csr_get(void* h, int which, int i, int j) {
  const csr_t* A = model_mat((orc_model*)h, which);
  return A ? csr_get(A, i, j) : 0.0;
}
