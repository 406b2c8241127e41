// Posterior mean with fixed effects (Sec. 3.1, eq:mean:3-5) and the
// fixed-effects term of the latent variances (eq:var:1).  The solves with
// Q_uu run on the sampler's conjugate gradients; the kernels here build their
// right-hand sides, reduce the thin products with the covariates, solve the
// small Schur system and combine the solutions:
//   k_mean_rhs      [A_u^T Q_y y, Q_ubeta] as n x (n_beta + 1) columns
//   k_mean_gram     per-row-block partial dot products of two column sets
//   k_mean_gram_sum the partials summed over row blocks in a fixed order
//   k_mean_schur    S = Q_betabeta - Q_betau Q_uu^-1 Q_ubeta, its Cholesky
//                   factor, mu_beta and S^-1 (one workgroup)
//   k_mean_combine  mu_u = w - W mu_beta, diag(W S^-1 W^T)
// Every reduction has a fixed order for a given size, so a call repeats
// bitwise.
#include "rbmc_impl.h"

namespace rbmc {

namespace {
constexpr int kGramThreads = 256;
constexpr int kGramMaxBlocks = 2048;  // row blocks of a Gram launch
constexpr int kGT = 8;                // x and y columns of a block's pair tile

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
}  // namespace

// B[c ldb + i], c = 0..n_beta: column 0 = tau_y y_r and column j + 1 =
// tau_y a_j[r] at an observed node i of rank r (A_u^T Q_y y and A_u^T Q_y
// A_beta: Q_y = tau_y I), zero at the other nodes.
__global__ __launch_bounds__(256) void k_mean_rhs(int n, int n_obs, const int* __restrict__ rank,
                                                  double tau_y, const double* __restrict__ y,
                                                  const double* __restrict__ a, int nb,
                                                  double* __restrict__ b, size_t ldb) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int r = G(rank)[i];
  const bool obs = r >= 0;
  G(b)[i] = obs ? tau_y * G(y)[r] : 0.0;
  for (int j = 0; j < nb; ++j)
    G(b)[(size_t)(j + 1) * ldb + i] = obs ? tau_y * G(a)[(size_t)j * n_obs + r] : 0.0;
}

// part[rb np + p], p = j ny + c: the sum over the rows of row block rb
// (rows rb 256 + t + k nrb 256) of x_j[r] y_c[r]; column 0 of the y set is
// y0, columns c >= 1 are y1 + (c - 1) ldy.  Block (rb, tile) streams its rows
// once for a tile of kGT x columns by kGT y columns, each thread keeping the
// tile's products of its rows in registers; the block's sums then follow a
// fixed shuffle and LDS tree.
__global__ __launch_bounds__(kGramThreads) void k_mean_gram(
    int L, int nx, const double* __restrict__ x, size_t ldx, int ny,
    const double* __restrict__ y0, const double* __restrict__ y1, size_t ldy,
    double* __restrict__ part, int nrb) {
  __shared__ double red[kGramThreads / 64][kGT * kGT];
  const int tid = threadIdx.x, rb = blockIdx.x;
  const int ntx = (nx + kGT - 1) / kGT;
  const int j0 = (blockIdx.y % ntx) * kGT, c0 = (blockIdx.y / ntx) * kGT;
  const int nj = min(kGT, nx - j0), nc = min(kGT, ny - c0);
  const double* xp[kGT];
  const double* yp[kGT];
#pragma unroll
  for (int j = 0; j < kGT; ++j) xp[j] = x + (size_t)(j0 + (j < nj ? j : 0)) * ldx;
#pragma unroll
  for (int c = 0; c < kGT; ++c) {
    const int cc = c0 + (c < nc ? c : 0);
    yp[c] = cc == 0 ? y0 : y1 + (size_t)(cc - 1) * ldy;
  }
  double acc[kGT][kGT];
#pragma unroll
  for (int j = 0; j < kGT; ++j)
#pragma unroll
    for (int c = 0; c < kGT; ++c) acc[j][c] = 0.0;
  const size_t step = (size_t)nrb * kGramThreads;
  for (size_t r = (size_t)rb * kGramThreads + tid; r < (size_t)L; r += step) {
    double xv[kGT], yv[kGT];
#pragma unroll
    for (int j = 0; j < kGT; ++j) xv[j] = j < nj ? G(xp[j])[r] : 0.0;
#pragma unroll
    for (int c = 0; c < kGT; ++c) yv[c] = c < nc ? G(yp[c])[r] : 0.0;
#pragma unroll
    for (int j = 0; j < kGT; ++j)
#pragma unroll
      for (int c = 0; c < kGT; ++c) acc[j][c] = fma(xv[j], yv[c], acc[j][c]);
  }
  const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int j = 0; j < kGT; ++j)
#pragma unroll
    for (int c = 0; c < kGT; ++c)
      if (j < nj && c < nc) {
        const double v = wave_sum(acc[j][c]);
        if (lane == 0) red[wave][j * kGT + c] = v;
      }
  __syncthreads();
  if (tid < kGT * kGT) {
    const int j = tid / kGT, c = tid % kGT;
    if (j < nj && c < nc) {
      double v = red[0][tid];
#pragma unroll
      for (int w = 1; w < kGramThreads / 64; ++w) v += red[w][tid];
      G(part)[(size_t)rb * nx * ny + (size_t)(j0 + j) * ny + (c0 + c)] = v;
    }
  }
}

// out[p] = sum over the row blocks of part[b np + p], one block per pair
__global__ __launch_bounds__(kGramThreads) void k_mean_gram_sum(int np, int nblk,
                                                                const double* __restrict__ part,
                                                                double* __restrict__ out) {
  __shared__ double red[kGramThreads / 64];
  const int p = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int b = tid; b < nblk; b += kGramThreads) s += G(part)[(size_t)b * np + p];
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double v = red[0];
#pragma unroll
    for (int w = 1; w < kGramThreads / 64; ++w) v += red[w];
    G(out)[p] = v;
  }
}

// g = Q_betau [w, W] and h = A_beta^T [y, A_beta] (n_beta x (n_beta + 1),
// row j at j (n_beta + 1)), q = Q_beta's diagonal.  Writes out[0] = 0, or
// k + 1 if the k-th pivot of S was not positive; out[1 + j] = mu_beta[j];
// out[1 + n_beta + j n_beta + k] = (S^-1)_jk.  S's two triangles are
// averaged: Q_betau Q_uu^-1 Q_ubeta is symmetric, its computed value only to
// the solves' tolerance.
__global__ __launch_bounds__(256) void k_mean_schur(int nb, const double* __restrict__ g,
                                                    const double* __restrict__ h,
                                                    const double* __restrict__ q, double tau_y,
                                                    double* __restrict__ out) {
  __shared__ double S[kMaxFixedEffects][kMaxFixedEffects + 1];
  __shared__ double X[kMaxFixedEffects + 1][kMaxFixedEffects + 1];
  __shared__ double rhs[kMaxFixedEffects];
  __shared__ int bad;
  const int tid = threadIdx.x, ny = nb + 1;
  if (tid == 0) bad = 0;
  for (int e = tid; e < nb * nb; e += 256) {
    const int j = e / nb, k = e % nb;
    const double sjk = tau_y * G(h)[j * ny + k + 1] - G(g)[j * ny + k + 1];
    const double skj = tau_y * G(h)[k * ny + j + 1] - G(g)[k * ny + j + 1];
    S[j][k] = 0.5 * (sjk + skj) + (j == k ? G(q)[j] : 0.0);
  }
  for (int j = tid; j < nb; j += 256) rhs[j] = tau_y * G(h)[j * ny] - G(g)[j * ny];
  __syncthreads();
  // S = L L^T, L overwriting the lower triangle (right-looking)
  for (int k = 0; k < nb; ++k) {
    if (tid == 0) {
      double d = S[k][k];
      if (!(d > 0.0)) {
        if (!bad) bad = k + 1;
        d = 1.0;  // keeps the rest finite; the host reports the failure
      }
      S[k][k] = sqrt(d);
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < nb; i += 256) S[i][k] /= S[k][k];
    __syncthreads();
    const int w = nb - k - 1;
    for (int e = tid; e < w * w; e += 256) {
      const int i = k + 1 + e / w, j = k + 1 + e % w;
      if (j <= i) S[i][j] -= S[i][k] * S[j][k];
    }
    __syncthreads();
  }
  // thread c < n_beta: column c of S^-1 (L L^T x = e_c); thread n_beta:
  // mu_beta (L L^T x = rhs)
  if (tid <= nb) {
    double* x = X[tid];
    for (int i = 0; i < nb; ++i) {
      double v = tid == nb ? rhs[i] : (i == tid ? 1.0 : 0.0);
      for (int k = 0; k < i; ++k) v -= S[i][k] * x[k];
      x[i] = v / S[i][i];
    }
    for (int i = nb - 1; i >= 0; --i) {
      double v = x[i];
      for (int k = i + 1; k < nb; ++k) v -= S[k][i] * x[k];
      x[i] = v / S[i][i];
    }
  }
  __syncthreads();
  if (tid == 0) G(out)[0] = (double)bad;
  for (int j = tid; j < nb; j += 256) G(out)[1 + j] = X[nb][j];
  for (int e = tid; e < nb * nb; e += 256) {
    const int j = e / nb, k = e % nb;
    G(out)[1 + nb + e] = X[k][j];
  }
}

// mu_u[i] = w[i] - sum_j W_j[i] mu_beta[j] (w = column 0, W_j = column
// j + 1 of the solutions) and var_add[i] = sum_jk W_j[i] (S^-1)_jk W_k[i].
template <int NB>
__global__ __launch_bounds__(256) void k_mean_combine(int n, int nb, const double* __restrict__ w,
                                                      size_t ldw, const double* __restrict__ sol,
                                                      double* __restrict__ mu_u,
                                                      double* __restrict__ var_add) {
  __shared__ double mb[NB > 0 ? NB : 1];
  __shared__ double si[NB > 0 ? NB : 1][NB > 0 ? NB : 1];
  const int tid = threadIdx.x;
  for (int j = tid; j < NB; j += 256) mb[j] = j < nb ? G(sol)[1 + j] : 0.0;
  for (int e = tid; e < NB * NB; e += 256) {
    const int j = e / NB, k = e % NB;
    si[j][k] = (j < nb && k < nb) ? G(sol)[1 + nb + j * nb + k] : 0.0;
  }
  __syncthreads();
  const size_t i = (size_t)blockIdx.x * 256 + tid;
  if (i >= (size_t)n) return;
  double t[NB > 0 ? NB : 1];
  double mu = G(w)[i];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    t[j] = j < nb ? G(w)[(size_t)(j + 1) * ldw + i] : 0.0;
    mu -= t[j] * mb[j];
  }
  G(mu_u)[i] = mu;
  if (var_add) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      double r = 0.0;
#pragma unroll
      for (int k = 0; k < NB; ++k) r += si[j][k] * t[k];
      v += t[j] * r;
    }
    G(var_add)[i] = v;
  }
}

void launch_mean_rhs(int n, int n_obs, const int* rank, double tau_y, const double* y,
                     const double* a, int nb, double* b, size_t ldb, hipStream_t s) {
  if (n <= 0) return;
  k_mean_rhs<<<(n + 255) / 256, 256, 0, s>>>(n, n_obs, rank, tau_y, y, a, nb, b, ldb);
}

int mean_gram_blocks(int L) {
  const int nb = (L + kGramThreads - 1) / kGramThreads;
  return nb < 1 ? 1 : (nb < kGramMaxBlocks ? nb : kGramMaxBlocks);
}

void launch_mean_gram(int L, int nx, const double* x, size_t ldx, int ny, const double* y0,
                      const double* y1, size_t ldy, double* part, double* out, hipStream_t s) {
  const int np = nx * ny;
  if (np <= 0) return;
  const int nrb = mean_gram_blocks(L);
  const dim3 grid(nrb, ((nx + kGT - 1) / kGT) * ((ny + kGT - 1) / kGT));
  k_mean_gram<<<grid, kGramThreads, 0, s>>>(L, nx, x, ldx, ny, y0, y1, ldy, part, nrb);
  k_mean_gram_sum<<<np, kGramThreads, 0, s>>>(np, nrb, part, out);
}

void launch_mean_schur(int nb, const double* g, const double* h, const double* q, double tau_y,
                       double* out, hipStream_t s) {
  k_mean_schur<<<1, 256, 0, s>>>(nb, g, h, q, tau_y, out);
}

void launch_mean_combine(int n, int nb, const double* w, size_t ldw, const double* sol,
                         double* mu_u, double* var_add, hipStream_t s) {
  if (n <= 0) return;
  const int grid = (n + 255) / 256;
  if (nb == 0)
    k_mean_combine<0><<<grid, 256, 0, s>>>(n, nb, w, ldw, sol, mu_u, var_add);
  else if (nb <= 4)
    k_mean_combine<4><<<grid, 256, 0, s>>>(n, nb, w, ldw, sol, mu_u, var_add);
  else if (nb <= 8)
    k_mean_combine<8><<<grid, 256, 0, s>>>(n, nb, w, ldw, sol, mu_u, var_add);
  else if (nb <= 16)
    k_mean_combine<16><<<grid, 256, 0, s>>>(n, nb, w, ldw, sol, mu_u, var_add);
  else
    k_mean_combine<kMaxFixedEffects><<<grid, 256, 0, s>>>(n, nb, w, ldw, sol, mu_u, var_add);
}

}  // namespace rbmc
