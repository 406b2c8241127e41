// Kernels of the Kronecker form of a subdomain inverse.
//
// A subdomain A = [t0, t0 + T_A) x R is a product of a time range and a
// spatial region, and the prior precision Q_t (x) Q_s restricted to a product
// set is the product of the restrictions.  With S = Q_s|R, V = (Q_t|[t0,
// t0+T_A))^-1 (a small dense T_A x T_A matrix) and the observed nodes of A
// collected by a selection P (o = (t_o, a_o), ordered by time, each time
// group padded to a multiple of 16 with unused slots),
//   Q_AA = V^-1 (x) S + P D_o P^T,
//   Q_AA^-1 = V (x) S^-1 - Z~ Y Z~^T,   Z~ = (V (x) S^-1) P,
//   Y = C^-1,  C = D_o^-1 + P^T (V (x) S^-1) P        (Woodbury identity).
// Column o of Z~ restricted to time t is V[t, t_o] Z[:, o] with
// Z[:, o] = S^-1[:, a_o], so every entry the estimator reads from Q_AA^-1 is
//   (Q_AA^-1)_{(t,a),(t',c)} = V[t,t'] S^-1[a,c]
//        - sum_{g,h} V[t,g] V[t',h] H_gh[a,c],
//   H_gh = Z_g Y_gh Z_h^T   (Z_g: the columns of time group g).
// The estimator needs on core rows only the diagonal and the 13-point
// stencil sums of Q_s and of K = dQ_s/dlog kappa against these entries.
// Since S S^-1 = I on R, the Q_s stencil sums reduce to
//   sum_c Qs[a,c] S^-1[a,c] = 1,    sum_c Qs[a,c] H_gh[a,c] = (X_g)[a, o_h(a)],
// with X_g = Z_g Y_{g,:} and o_h(a) the observation of node a at time h
// (zero if a is not observed then); the K sums need the row dots of X_g with
// K_R Z.  The kernels below form these per (g, h) and combine them with
// the rows of V.
#include <algorithm>

#include "rbmc_impl.h"

namespace rbmc {

namespace {
template <class T>
__device__ inline int kfind(const T* __restrict__ tasks, int n_tasks, int b) {
  int lo = 0, hi = n_tasks - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (tasks[mid].tile_start <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}
}  // namespace

// ---------------------------------------------------------------------------
// Per-node quantities of S^-1 on its region: dR[a] = S^-1_aa and the stencil
// sums qR[a] = sum_q Qs[a, nbr_q] S^-1[a, nbr_q], kR[a] likewise with K.
// One thread per region node; grid = tiles of 256 nodes.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_kron_region(const KronRegionTask* __restrict__ tasks,
                                                     int n_tasks) {
  const KronRegionTask tk = tasks[kfind(tasks, n_tasks, blockIdx.x)];
  const RegionDev rg = *tk.rg;
  const DevModel& m = *tk.dm;
  const int a = (blockIdx.x - tk.tile_start) * 256 + threadIdx.x;
  if (a >= rg.np) return;
  double d = 0.0, sq = 0.0, sk = 0.0;
  if (a < rg.nb) {
    const int node = G(rg.nodes)[a];
    // S^-1 is symmetric: row a is read as column a (contiguous)
    const gptr<const double> col = G(tk.inv) + (size_t)a * rg.np;
    d = col[a];
#pragma unroll
    for (int q = 0; q < kNS; ++q) {
      const int c = G(rg.nbr)[a * kNS + q];
      if (c < 0) continue;
      const double v = col[c];
      sq += G(m.qs)[(size_t)q * m.ns + node] * v;
      if (q < kN5) sk += G(m.kk)[(size_t)q * m.ns + node] * v;
    }
  }
  G(tk.dR)[a] = d;
  G(tk.qR)[a] = sq;
  G(tk.kR)[a] = sk;
}

void launch_kron_region(const KronRegionTask* d_tasks, int n_tasks, int total_tiles,
                        hipStream_t s) {
  if (total_tiles > 0) k_kron_region<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

// ---------------------------------------------------------------------------
// Z[:, o] = S^-1[:, a_o] (zero for unused slots), np x nc, ld np.
// C[o, o'] = V[t_o, t_o'] Z[a_o, o'] + [o = o'] sigma^2 (unused slots:
// identity).  Tiles of 256 rows x 8 columns.
// ---------------------------------------------------------------------------
namespace {
constexpr int kKC = 8;  // columns per tile of the gather and assembly kernels
}
int kron_cols_tiles(int rows, int cols) { return ((rows + 255) / 256) * ((cols + kKC - 1) / kKC); }

__global__ __launch_bounds__(256) void k_kron_build(const KronBuildTask* __restrict__ tasks,
                                                    int n_tasks) {
  const KronBuildTask tk = tasks[kfind(tasks, n_tasks, blockIdx.x)];
  const int tile = blockIdx.x - tk.tile_start;
  const int rows = tk.mode == 0 ? tk.np : tk.nc;
  const int rt = (rows + 255) / 256;
  const int r = (tile % rt) * 256 + threadIdx.x;
  const int c0 = (tile / rt) * kKC;
  if (r >= rows) return;
  if (tk.mode == 0) {  // gather Z
#pragma unroll
    for (int j = 0; j < kKC; ++j) {
      const int o = c0 + j;
      if (o >= tk.nc) break;
      const int ao = G(tk.obs_a)[o];
      G(tk.out)[(size_t)o * tk.np + r] = ao >= 0 ? G(tk.inv)[(size_t)ao * tk.np + r] : 0.0;
    }
  } else {  // capacitance C, from Z
    const int ar = G(tk.obs_a)[r];
    const int tr = G(tk.obs_t)[r];
#pragma unroll
    for (int j = 0; j < kKC; ++j) {
      const int o = c0 + j;
      if (o >= tk.nc) break;
      const int ao = G(tk.obs_a)[o];
      double v;
      if (ar < 0 || ao < 0) {
        v = (r == o) ? 1.0 : 0.0;
      } else {
        const int to = G(tk.obs_t)[o];
        v = G(tk.V)[tr * tk.TA + to] * G(tk.Z)[(size_t)o * tk.np + ar];
        if (r == o) v += tk.noise;
      }
      G(tk.out)[(size_t)o * tk.nc + r] = v;
    }
  }
}

void launch_kron_build(const KronBuildTask* d_tasks, int n_tasks, int total_tiles,
                       hipStream_t s) {
  if (total_tiles > 0) k_kron_build<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

// ---------------------------------------------------------------------------
// Group reductions for time group g (X = X_g = Z_g Y_{g,:}, np x nc):
//   part[((g TA + h) 3 + 0) np + a] = sum_{o in h} X[a,o] Z[a,o]
//   part[((g TA + h) 3 + 1) np + a] = X[a, o_h(a)]   (Q_s stencil sum)
//   part[((g TA + h) 3 + 2) np + a] = sum_{o in h} X[a,o] KZ[a,o]
// Workgroup: 64 rows (one per lane) x 4 waves; wave w takes groups
// h = w, w + 4, ...; the 64 lanes read 64 consecutive rows of a column.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_kron_reduce(const KronReduceTask* __restrict__ tasks,
                                                     int n_tasks) {
  const KronReduceTask tk = tasks[kfind(tasks, n_tasks, blockIdx.x)];
  const int tile = blockIdx.x - tk.tile_start;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int a = tile * 64 + lane;
  if (a >= tk.np) return;
  const gptr<const double> X = G(tk.X), Z = G(tk.Z), KZ = G(tk.KZ);
  for (int h = wave; h < tk.TA; h += 4) {
    const int o0 = G(tk.goff)[h], o1 = o0 + G(tk.gpad)[h];
    double p = 0.0, sq = 0.0, sk = 0.0;
    for (int o = o0; o < o1; ++o) {
      const size_t at = (size_t)o * tk.np + a;
      const double x = X[at];
      p = fma(x, Z[at], p);
      sk = fma(x, KZ[at], sk);
      if (G(tk.obs_a)[o] == a) sq += x;
    }
    const size_t base = ((size_t)(tk.g * tk.TA + h) * 3) * tk.np + a;
    G(tk.part)[base] = p;
    G(tk.part)[base + tk.np] = sq;
    G(tk.part)[base + 2 * (size_t)tk.np] = sk;
  }
}

void launch_kron_reduce(const KronReduceTask* d_tasks, int n_tasks, int total_tiles,
                        hipStream_t s) {
  if (total_tiles > 0) k_kron_reduce<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

// ---------------------------------------------------------------------------
// Combination at a core step t (local) for the core rows of the region:
//   diag  = V[t,t] dR[a] - u^T P u,                  u = V[t, :]
//   Qs(t') = V[t,t'] qR[a] - u^T SQ w(t'),           w(t') = V[t', :]
//   K(t')  = V[t,t'] kR[a] - u^T SK w(t'),           t' = t, t+1, t-1
// (P, SQ, SK: the T_A x T_A group matrices of node a).  diag goes to
// diag_out; the three slots (t'=t, t+1, t-1) of the sums D*diag, Qs, K over
// the tile's core rows go to partial[(out_index + sl nchk + chunk) 3 + j],
// the layout the dense-block extraction uses.  One tile = 256 region rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_kron_det(const KronDetTask* __restrict__ tasks,
                                                  int n_tasks) {
  __shared__ double red[7][256];
  const KronDetTask tk = tasks[kfind(tasks, n_tasks, blockIdx.x)];
  const RegionDev rg = *tk.rg;
  const DevModel& m = *tk.dm;
  const int chunk = blockIdx.x - tk.tile_start;
  const int tid = threadIdx.x;
  const int a = chunk * 256 + tid;
  const int TA = tk.TA, t = tk.t;
  const gptr<const double> V = G(tk.V);
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};  // D diag, Qs x3, K x3
  if (a < rg.nb && G(rg.in_box)[a]) {
    const size_t np = rg.np;
    const gptr<const double> part = G(tk.part);
    double cp = 0.0, cq[3] = {0, 0, 0}, ck[3] = {0, 0, 0};
    for (int h = 0; h < TA; ++h) {
      double vp = 0.0, vq = 0.0, vk = 0.0;
      for (int g = 0; g < TA; ++g) {
        const double u = V[t * TA + g];
        const size_t base = ((size_t)(g * TA + h) * 3) * np + a;
        vp = fma(u, part[base], vp);
        vq = fma(u, part[base + np], vq);
        vk = fma(u, part[base + 2 * np], vk);
      }
      cp = fma(V[t * TA + h], vp, cp);
#pragma unroll
      for (int sl = 0; sl < 3; ++sl) {
        const int tp = t + (sl == 0 ? 0 : (sl == 1 ? 1 : -1));
        if (tp < 0 || tp >= TA) continue;
        const double w = V[tp * TA + h];
        cq[sl] = fma(w, vq, cq[sl]);
        ck[sl] = fma(w, vk, ck[sl]);
      }
    }
    const double diag = V[t * TA + t] * G(tk.dR)[a] - cp;
    const size_t i = (size_t)(tk.t0 + t) * m.ns + G(rg.nodes)[a];
    G(tk.diag_out)[i] = diag;
    acc[0] = G(m.dvec)[i] * diag;
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      const int tp = t + (sl == 0 ? 0 : (sl == 1 ? 1 : -1));
      if (tp < 0 || tp >= TA) continue;
      const double vtt = V[t * TA + tp];
      acc[1 + sl] = vtt * G(tk.qR)[a] - cq[sl];
      acc[4 + sl] = vtt * G(tk.kR)[a] - ck[sl];
    }
  }
#pragma unroll
  for (int j = 0; j < 7; ++j) red[j][tid] = acc[j];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st)
#pragma unroll
      for (int j = 0; j < 7; ++j) red[j][tid] += red[j][tid + st];
    __syncthreads();
  }
  if (tid < 9) {
    const int sl = tid / 3, j = tid % 3;
    const double v = j == 0 ? (sl == 0 ? red[0][0] : 0.0) : red[(j == 1 ? 1 : 4) + sl][0];
    G(tk.partial)[((size_t)tk.out_index + (size_t)sl * tk.nchk + chunk) * 3 + j] = v;
  }
}

void launch_kron_det(const KronDetTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s) {
  if (total_tiles > 0) k_kron_det<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

// ---------------------------------------------------------------------------
// Time mixing of stacked panels (np x n_k per local step, step t at
// t np n_k): out_t = beta In_t + alpha sum_t' V[t,t'] U_t'  (out may alias In;
// U must not alias out).  Thread per (row, sample); up to kMix output steps
// are held in registers, so for TA <= kMix every input entry is read once.
// ---------------------------------------------------------------------------
constexpr int kMix = 24;
constexpr int kMixV = 64;  // chains up to this many steps read V from LDS

__global__ __launch_bounds__(256) void k_kron_tmix(const KronMixTask* __restrict__ tasks,
                                                   int n_tasks) {
  __shared__ double vs[kMix * kMixV];  // rows t0 .. t0 + kMix of V, zero beyond TA
  const KronMixTask tk = tasks[kfind(tasks, n_tasks, blockIdx.x)];
  const size_t e = (size_t)(blockIdx.x - tk.tile_start) * 256 + threadIdx.x;
  const size_t panel = (size_t)tk.np * tk.n_k;
  const int TA = tk.TA;
  const gptr<const double> V = G(tk.V), U = G(tk.U);
  const bool lds = TA <= kMixV;
  for (int t0 = 0; t0 < TA; t0 += kMix) {
    if (lds) {
      __syncthreads();
      for (int q = threadIdx.x; q < kMix * TA; q += 256) {
        const int j = q / TA, tp = q % TA;
        vs[q] = t0 + j < TA ? V[(t0 + j) * TA + tp] : 0.0;
      }
      __syncthreads();
    }
    if (e >= panel) continue;
    double acc[kMix];
#pragma unroll
    for (int j = 0; j < kMix; ++j) acc[j] = 0.0;
    if (lds) {
      for (int tp = 0; tp < TA; ++tp) {
        const double u = U[(size_t)tp * panel + e];
#pragma unroll
        for (int j = 0; j < kMix; ++j) acc[j] = fma(vs[j * TA + tp], u, acc[j]);
      }
    } else {
      for (int tp = 0; tp < TA; ++tp) {
        const double u = U[(size_t)tp * panel + e];
#pragma unroll
        for (int j = 0; j < kMix; ++j)
          if (t0 + j < TA) acc[j] = fma(V[(t0 + j) * TA + tp], u, acc[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < kMix; ++j) {
      if (t0 + j >= TA) break;
      const size_t at = (size_t)(t0 + j) * panel + e;
      double v = tk.alpha * acc[j];
      if (tk.beta != 0.0) v += tk.beta * G(tk.In)[at];
      G(tk.out)[at] = v;
    }
  }
}

int kron_mix_tiles(int np, int n_k) { return (int)(((size_t)np * n_k + 255) / 256); }

void launch_kron_tmix(const KronMixTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s) {
  if (total_tiles > 0) k_kron_tmix<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

// ---------------------------------------------------------------------------
// v[o + nc k] = U[a_o + np (k + n_k t_o)] (zero for unused slots): the
// observed entries of stacked panels.  Tiles of 256 slots x 8 samples.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_kron_obs(const KronObsTask* __restrict__ tasks,
                                                  int n_tasks) {
  const KronObsTask tk = tasks[kfind(tasks, n_tasks, blockIdx.x)];
  const int tile = blockIdx.x - tk.tile_start;
  const int rt = (tk.nc + 255) / 256;
  const int o = (tile % rt) * 256 + threadIdx.x;
  const int k0 = (tile / rt) * kKC;
  if (o >= tk.nc) return;
  const int ao = G(tk.obs_a)[o], to = ao >= 0 ? G(tk.obs_t)[o] : 0;
#pragma unroll
  for (int j = 0; j < kKC; ++j) {
    const int k = k0 + j;
    if (k >= tk.n_k) break;
    G(tk.v)[(size_t)k * tk.nc + o] =
        ao >= 0 ? G(tk.U)[(size_t)ao + (size_t)tk.np * ((size_t)k + (size_t)tk.n_k * to)] : 0.0;
  }
}

void launch_kron_obs(const KronObsTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s) {
  if (total_tiles > 0) k_kron_obs<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

// ---------------------------------------------------------------------------
// Fill: p[i] = value for i < n (a kernel, so it can sit in captured graphs).
// ---------------------------------------------------------------------------
__global__ void k_fill(double* __restrict__ p, size_t n, double value) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = value;
}

void launch_fill(double* p, size_t n, double value, hipStream_t s) {
  if (n == 0) return;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 8192);
  k_fill<<<(unsigned)blocks, 256, 0, s>>>(p, n, value);
}

}  // namespace rbmc

namespace rbmc {

// ---------------------------------------------------------------------------
// Standard normals from a counter-based generator: Philox4x32-10 (Salmon,
// Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC11)
// with key = seed, counter = (pair index, 0, 0), and the Box-Muller transform
// of the two 53-bit uniforms the four output words give.  Element e of the
// stream is the first (e even) or second (e odd) normal of pair e / 2, so any
// element depends only on (seed, e): chunks of a stream are the stream.
// ---------------------------------------------------------------------------
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__global__ void k_normals(uint64_t seed, uint64_t offset, size_t count, double* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    const uint64_t e = offset + i, pr = e >> 1;
    uint32_t c[4] = {(uint32_t)pr, (uint32_t)(pr >> 32), 0u, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t a = ((uint64_t)c[0] << 32) | c[1], b = ((uint64_t)c[2] << 32) | c[3];
    const double u = (double)(a >> 11) * 0x1.0p-53 + 0x1.0p-54;  // (0, 1)
    const double v = (double)(b >> 11) * 0x1.0p-53;              // [0, 1)
    const double rad = sqrt(-2.0 * log(u));
    double sn, cs;
    sincospi(2.0 * v, &sn, &cs);
    out[i] = (e & 1) ? rad * sn : rad * cs;
  }
}

void launch_normals(uint64_t seed, uint64_t offset, size_t count, double* out, hipStream_t s) {
  if (count == 0) return;
  const size_t blocks = std::min<size_t>((count + 255) / 256, 16384);
  k_normals<<<(unsigned)blocks, 256, 0, s>>>(seed, offset, count, out);
}

// Plug-in error terms of an estimate: partial[b] = sum over the block's nodes
// of (diag - det) / diag (the Monte Carlo share of each estimate).
__global__ __launch_bounds__(256) void k_mc_share(const double* __restrict__ diag,
                                                  const double* __restrict__ det, size_t n,
                                                  double* __restrict__ partial) {
  __shared__ double red[256];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const double d = diag[i];
    if (d > 0.0) acc += (d - det[i]) / d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

int mc_share_blocks(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 1024); }

void launch_mc_share(const double* diag, const double* det, size_t n, double* partial,
                     hipStream_t s) {
  if (n > 0) k_mc_share<<<mc_share_blocks(n), 256, 0, s>>>(diag, det, n, partial);
}

}  // namespace rbmc
