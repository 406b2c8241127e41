// Kernels on chain panels: gather/scatter between global multi-vectors and
// padded region panels, the correction right-hand sides Q_AB x_B, and the
// reductions that turn dense Q_AA^-1 blocks and correction panels into the
// estimator's diagonal and trace contributions.  Every task carries its own
// model and region pointers, so one launch serves chains of many models.
#include <climits>

#include "rbmc_impl.h"

namespace rbmc {

namespace {
constexpr int PT_N = 64;   // nodes per panel tile
constexpr int PT_K = 64;   // samples per panel tile

template <class T>
__device__ inline int find_task_of(const T* __restrict__ tasks, int n_tasks, int b) {
  int lo = 0, hi = n_tasks - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (tasks[mid].tile_start <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}
}  // namespace

int panel_tiles(int np, int n_k) { return (np / PT_N) * ((n_k + PT_K - 1) / PT_K); }

__global__ __launch_bounds__(256) void k_panels(const PanelTask* __restrict__ tasks, int n_tasks) {
  const int b = blockIdx.x;
  const PanelTask tk = tasks[find_task_of(tasks, n_tasks, b)];
  const RegionDev rg = *tk.rg;
  const DevModel m = *tk.dm;
  const int n_k = tk.n_k;
  const int tile = b - tk.tile_start;
  const int tiles_k = (n_k + PT_K - 1) / PT_K;
  const int a = (tile / tiles_k) * PT_N + (threadIdx.x & 63);
  const int kbase = (tile % tiles_k) * PT_K;
  const bool real = a < rg.nb;
  const int node = real ? G(rg.nodes)[a] : 0;
  const size_t base = (size_t)tk.t * m.ns + node;

  if (tk.mode == 0) {
    for (int kk = threadIdx.x >> 6; kk < PT_K; kk += 4) {
      const int k = kbase + kk;
      if (k >= n_k) break;
      G(tk.P)[(size_t)k * rg.np + a] = real ? G(tk.X)[(size_t)k * m.n + base] : 0.0;
    }
  } else if (tk.mode == 1) {
    if (!real) return;
    for (int kk = threadIdx.x >> 6; kk < PT_K; kk += 4) {
      const int k = kbase + kk;
      if (k >= n_k) break;
      G(tk.Xout)[(size_t)k * m.n + base] = G(tk.P)[(size_t)k * rg.np + a];
    }
  } else if (tk.mode == 4) {
    if (!real) return;
    for (int kk = threadIdx.x >> 6; kk < PT_K; kk += 4) {
      const int k = kbase + kk;
      if (k >= n_k) break;
      G(tk.P)[(size_t)k * rg.np + a] += tk.w * G(tk.X)[(size_t)k * m.n + base];
    }
  } else {
    // mode 2: r_a = sum over neighbours j of (t, node) outside A = [t0, t0+T)
    // x R of Q_aj x_j; mode 3: over the neighbours whose node is outside R;
    // row a of the panel is region row ar (the row list, or a)
    const int ar = tk.rows ? G(tk.rows)[a] : (real ? a : -1);
    const int ld = tk.rows ? tk.ld : rg.np;
    const int nd = ar >= 0 ? G(rg.nodes)[ar] : 0;
    const int ix = nd % m.mx, iy = nd / m.mx;
    // coefficients of the 3 x 13 space-time neighbours, zero for those in A
    // or off the grid (static indices: the arrays stay in registers)
    double cf[3][kNS];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int tt = tk.t + d - 1;
      const bool t_ok = ar >= 0 && tt >= 0 && tt < m.T;
      const bool t_in = tt >= tk.t0 && tt < tk.t0 + tk.T;
      const double wt = d == 1 ? G(m.qd)[tk.t] : m.qo;
#pragma unroll
      for (int q = 0; q < kNS; ++q) {
        const int jx = ix + kSdx[q], jy = iy + kSdy[q];
        const bool ok = t_ok && jx >= 0 && jx < m.mx && jy >= 0 && jy < m.my &&
                        !((t_in || tk.mode == 3) && G(rg.nbr)[ar * kNS + q] >= 0);
        cf[d][q] = ok ? wt * G(m.qs)[(size_t)q * m.ns + nd] : 0.0;
      }
    }
    const size_t at = (size_t)tk.t * m.ns + nd;
    for (int kk = threadIdx.x >> 6; kk < PT_K; kk += 4) {
      const int k = kbase + kk;
      if (k >= n_k) break;
      const gptr<const double> xk = G(tk.X) + (size_t)k * m.n + at;
      double v = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < kNS; ++q)
          if (cf[d][q] != 0.0)
            v += cf[d][q] * xk[(long)(d - 1) * m.ns + kSdy[q] * m.mx + kSdx[q]];
      G(tk.P)[(size_t)k * ld + a] = v;
    }
  }
}

void launch_panels(const PanelTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s) {
  if (total_tiles <= 0) return;
  k_panels<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

// ---------------------------------------------------------------------------
// Deterministic-part extraction. One workgroup per 256 region rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_extract(const ExtractTask* __restrict__ tasks,
                                                 int n_tasks) {
  __shared__ double red[3][256];
  const int b = blockIdx.x;
  const ExtractTask tk = tasks[find_task_of(tasks, n_tasks, b)];
  const RegionDev rg = *tk.rg;
  const DevModel& m = *tk.dm;
  const int chunk = b - tk.tile_start;
  const int a = chunk * 256 + threadIdx.x;
  double sd = 0.0, sq = 0.0, sk = 0.0;
  if (a < rg.nb && G(rg.in_box)[a]) {
    const int node = G(rg.nodes)[a];
    auto el = [&](int r, int c) {  // Sigma block entry (r, c) in region-local indices
      return tk.trans ? G(tk.M)[(size_t)r * tk.ld + c] : G(tk.M)[(size_t)c * tk.ld + r];
    };
    for (int q = 0; q < kNS; ++q) {
      const int c = G(rg.nbr)[a * kNS + q];
      if (c < 0) continue;
      const double v = tk.sign * el(a, c);
      sq += G(m.qs)[(size_t)q * m.ns + node] * v;
      if (q < kN5) sk += G(m.kk)[(size_t)q * m.ns + node] * v;
      if (q == 0 && tk.kind == 0) {
        const size_t i = (size_t)tk.t * m.ns + node;
        G(tk.diag_out)[i] = v;
        sd = G(m.dvec)[i] * v;
      }
    }
  }
  red[0][threadIdx.x] = sd;
  red[1][threadIdx.x] = sq;
  red[2][threadIdx.x] = sk;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 3)
    G(tk.partial)[((size_t)tk.out_index + chunk) * 3 + threadIdx.x] = red[threadIdx.x][0];
}

void launch_extract(const ExtractTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s) {
  if (total_tiles <= 0) return;
  k_extract<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

// ---------------------------------------------------------------------------
// Off-diagonal time blocks on the stencil pattern only.  For a core step t
// and a neighbouring step t' = t +- 1 of the chain,
//   Sigma_{t,t'}[a, c] = scale * sum_k W[k, c] Sigma_tt[k, a],
// with W = Q_R S'^-1 (S' the Schur complement inverse on the far side of t,
// one stencil pass) and scale = -q_o; only the 13 stencil neighbours c of
// each core row a are formed.  They enter the traces exactly as k_extract's
// off-diagonal slots do (sum over c of Q_s / K coefficient x entry).
//
// Workgroup = 256 region rows, one per thread.  The neighbour columns of the
// 256 rows form one contiguous span [lo, hi] of W's columns (the region is
// ordered by grid rows; a stencil reaches two grid rows up and down).  The
// shared index k is walked in chunks of kOdK: the chunk of Sigma's 256
// columns and of W's span is staged in LDS (coalesced 64-byte column pieces),
// then each thread adds kOdK terms to its 13 dot products from LDS.  A tile
// whose span exceeds kOdSpan streams its columns from global memory instead,
// one wave per row.
// ---------------------------------------------------------------------------
namespace {
constexpr int kOdK = 8, kOdLd = kOdK + 1, kOdSpan = 528;
}

__global__ __launch_bounds__(256) void k_offdiag(const OffdiagTask* __restrict__ tasks,
                                                 int n_tasks) {
  __shared__ double sg_s[256 * kOdLd];
  __shared__ double w_s[kOdSpan * kOdLd];
  __shared__ double red[2][256];
  __shared__ int span_lo, span_hi;
  const int b = blockIdx.x;
  const OffdiagTask tk = tasks[find_task_of(tasks, n_tasks, b)];
  const RegionDev rg = *tk.rg;
  const DevModel& m = *tk.dm;
  const int chunk = b - tk.tile_start;
  const int tid = threadIdx.x;
  const int a0 = chunk * 256, a = a0 + tid;
  const bool row = a < rg.nb && G(rg.in_box)[a];
  int nbr[kNS];
  int lo = INT_MAX, hi = -1;
#pragma unroll
  for (int q = 0; q < kNS; ++q) {
    nbr[q] = row ? G(rg.nbr)[a * kNS + q] : -1;
    if (nbr[q] >= 0) {
      lo = min(lo, nbr[q]);
      hi = max(hi, nbr[q]);
    }
  }
  if (tid == 0) {
    span_lo = INT_MAX;
    span_hi = -1;
  }
  __syncthreads();
  if (row) {
    atomicMin(&span_lo, lo);
    atomicMax(&span_hi, hi);
  }
  __syncthreads();
  const int slo = span_lo, span = span_hi - span_lo + 1;
  double acc[kNS];
#pragma unroll
  for (int q = 0; q < kNS; ++q) acc[q] = 0.0;
  const int nrows = min(256, rg.nb - a0);  // Sigma columns of this tile
  if (span > 0 && span <= kOdSpan) {
    for (int k0 = 0; k0 < rg.nb; k0 += kOdK) {
      const int kc = min(kOdK, rg.nb - k0);
      // all loads of a thread in flight at once: column tid / 8 + 32 i, k = tid % 8
      constexpr int kSg = 256 * kOdK / 256, kW = (kOdSpan * kOdK + 255) / 256;
      const int kk = tid % kOdK, c0 = tid / kOdK;
      const bool kin = kk < kc;
      double ls[kSg], lw[kW];
#pragma unroll
      for (int i = 0; i < kSg; ++i) {
        const int col = c0 + 32 * i;
        ls[i] = (kin && col < nrows) ? G(tk.Sig)[(size_t)(a0 + col) * tk.ld + k0 + kk] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < kW; ++i) {
        const int col = c0 + 32 * i;
        lw[i] = (kin && col < span) ? G(tk.W)[(size_t)(slo + col) * tk.ld + k0 + kk] : 0.0;
      }
      __syncthreads();  // the previous chunk is no longer read
#pragma unroll
      for (int i = 0; i < kSg; ++i) sg_s[(c0 + 32 * i) * kOdLd + kk] = ls[i];
#pragma unroll
      for (int i = 0; i < kW; ++i)
        if (c0 + 32 * i < kOdSpan) w_s[(c0 + 32 * i) * kOdLd + kk] = lw[i];
      __syncthreads();
      if (row) {
#pragma unroll
        for (int kk = 0; kk < kOdK; ++kk) {
          const double sv = sg_s[tid * kOdLd + kk];
#pragma unroll
          for (int q = 0; q < kNS; ++q)
            if (nbr[q] >= 0) acc[q] = fma(w_s[(nbr[q] - slo) * kOdLd + kk], sv, acc[q]);
        }
      }
    }
  } else if (span > 0) {  // wide regions: one wave per row, columns from global memory
    const int lane = tid & 63, wave = tid >> 6;
    double accw[kNS];
    for (int r = wave; r < nrows; r += 4) {
      const int ar = a0 + r;
      if (!G(rg.in_box)[ar]) continue;
      int nb2[kNS];
#pragma unroll
      for (int q = 0; q < kNS; ++q) {
        nb2[q] = G(rg.nbr)[ar * kNS + q];
        accw[q] = 0.0;
      }
      const gptr<const double> sg = G(tk.Sig) + (size_t)ar * tk.ld;
      for (int k = lane; k < rg.nb; k += 64) {
        const double sv = sg[k];
#pragma unroll
        for (int q = 0; q < kNS; ++q)
          if (nb2[q] >= 0) accw[q] = fma(tk.W[(size_t)nb2[q] * tk.ld + k], sv, accw[q]);
      }
#pragma unroll
      for (int q = 0; q < kNS; ++q) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) accw[q] += __shfl_xor(accw[q], off, 64);
      }
      // row ar's sums go to its own thread (tid = r) through LDS
      if (lane == 0)
#pragma unroll
        for (int q = 0; q < kNS; ++q) w_s[r * kNS + q] = accw[q];
    }
    __syncthreads();
    if (row)
#pragma unroll
      for (int q = 0; q < kNS; ++q) acc[q] = w_s[tid * kNS + q];
  }
  double sq = 0.0, sk = 0.0;
  if (row) {
    const int node = G(rg.nodes)[a];
#pragma unroll
    for (int q = 0; q < kNS; ++q) {
      if (nbr[q] < 0) continue;
      const double v = tk.scale * acc[q];
      sq += G(m.qs)[(size_t)q * m.ns + node] * v;
      if (q < kN5) sk += G(m.kk)[(size_t)q * m.ns + node] * v;
    }
  }
  red[0][tid] = sq;
  red[1][tid] = sk;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
      red[0][tid] += red[0][tid + st];
      red[1][tid] += red[1][tid + st];
    }
    __syncthreads();
  }
  if (tid < 3)
    G(tk.partial)[((size_t)tk.out_index + chunk) * 3 + tid] = tid == 0 ? 0.0 : red[tid - 1][0];
}

void launch_offdiag(const OffdiagTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s) {
  if (total_tiles <= 0) return;
  k_offdiag<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

// ---------------------------------------------------------------------------
// Monte Carlo part.  Workgroup = 256 region rows, one per thread, looping over
// the samples.  The rows of mu_{t-1}, mu_t, mu_{t+1} that the workgroup's
// stencils reach form a window [w0, w1] of region rows; for groups of
// samples the three windows are staged in LDS (coalesced loads, each entry
// once) and the 3 x 13 neighbour reads come from LDS.  Windows that do not
// fit (very wide regions) are read from global memory directly.
// Outputs: diag on core rows and 8 partial sums per workgroup:
//   [0..2] mu_t . (Q_s mu_{t-1,t,t+1}), [3..5] mu_t . (K mu_{t-1,t,t+1}),
//   [6] sum D mu_t^2 (all divided by n_k), [7] sum of m_a / s2_a.
// ---------------------------------------------------------------------------
namespace {
constexpr int kMcLds = 4096;  // doubles of staged windows
constexpr int kMcS = 4;       // core steps per task at most
constexpr int kMcU = 16;      // window loads in flight per thread (kMcLds / 256)
}

// a / b for 0 <= a, 0 < b, both below 2^13 (window indices; inv = 1 / b in
// FP32): the FP32 quotient is within 2^-10 of a / b, so its truncation is
// off by at most one, and one step each way corrects it
__device__ __forceinline__ int mc_div(int a, int b, float inv) {
  int q = (int)((float)a * inv);
  if (q * b > a) --q;
  if ((q + 1) * b <= a) ++q;
  return q;
}

// MULTI: tasks of up to kMcS steps whose windows fit in LDS (the host checks);
// else one step per task, with a direct global-memory path for windows that
// do not fit.
template <bool MULTI>
__global__ __launch_bounds__(256) void k_mc(const McTask* __restrict__ tasks, int n_tasks) {
  __shared__ double red[8][256];
  __shared__ double win[kMcLds];
  __shared__ int span[2];
  const int b = blockIdx.x;
  const McTask tk = tasks[find_task_of(tasks, n_tasks, b)];
  const RegionDev rg = *tk.rg;
  const DevModel& m = *tk.dm;
  const int n_k = tk.n_k;
  const int chunk = b - tk.tile_start;
  const int a = chunk * 256 + threadIdx.x;
  const bool mine = a < rg.nb && G(rg.in_box)[a];
  constexpr int kS = MULTI ? kMcS : 1;    // register arrays per step
  const int S = MULTI ? tk.steps : 1;     // steps of this task
  const int nP = S + 2;                   // panels they read: steps tl - 1 .. tl + S
  // panel d (0 <= d < nP): local step tl - 1 + d of the stack, or mu[d]
#define RBMC_MC_PANEL(d)                                                                    \
  (tk.stack ? ((tk.tl - 1 + (d) >= 0 && tk.tl - 1 + (d) < tk.ta)                           \
                   ? tk.stack + (size_t)(tk.tl - 1 + (d)) * tk.np * n_k                      \
                   : (const double*)nullptr)                                                 \
            : ((d) == 0 ? tk.mu[0] : (d) == 1 ? tk.mu[1] : tk.mu[2]))
  double acc[kS][8];
#pragma unroll
  for (int s = 0; s < kS; ++s)
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[s][c] = 0.0;
  int nbr[kNS];
  double cq[kNS], ck[kN5], dv[kS];
  int lo = INT_MAX, hi = -1;
  int node = 0;
  if (mine) {
    node = G(rg.nodes)[a];
#pragma unroll
    for (int s = 0; s < kS; ++s)
      dv[s] = s < S ? G(m.dvec)[(size_t)(tk.t + s) * m.ns + node] : 0.0;
#pragma unroll
    for (int q = 0; q < kNS; ++q) {
      nbr[q] = G(rg.nbr)[a * kNS + q];
      cq[q] = G(m.qs)[(size_t)q * m.ns + node];
      if (q < kN5) ck[q] = G(m.kk)[(size_t)q * m.ns + node];
      if (nbr[q] >= 0) {
        lo = min(lo, nbr[q]);
        hi = max(hi, nbr[q]);
      }
    }
  }
  if (threadIdx.x == 0) {
    span[0] = INT_MAX;
    span[1] = -1;
  }
  __syncthreads();
  if (mine) {
    atomicMin(&span[0], lo);
    atomicMax(&span[1], hi);
  }
  __syncthreads();
  const int w0 = span[0], wn = span[1] >= span[0] ? span[1] - span[0] + 1 : 0;
  const int sk = wn > 0 ? min(4, kMcLds / (nP * wn)) : 0;
  // one sample: mu_s = MU(s) (the row's entry of step s's panel), Y(p, row)
  // reads row of panel p (zero for a panel outside the chain).  Each panel's
  // stencil sums serve every step that reads it: step s reads panels
  // s, s + 1, s + 2 as its t - 1, t, t + 1.
#define RBMC_MC_SAMPLE(MU, Y)                                    \
  {                                                              \
    double mu_[kS];                                              \
    _Pragma("unroll") for (int s = 0; s < kS; ++s) {             \
      mu_[s] = s < S ? (MU(s)) : 0.0;                            \
      acc[s][7] += mu_[s] * mu_[s];                              \
      acc[s][6] += dv[s] * mu_[s] * mu_[s];                      \
    }                                                            \
    _Pragma("unroll") for (int p = 0; p < kS + 2; ++p) {         \
      if (p >= nP) break;                                        \
      double vq = 0.0, vk = 0.0;                                 \
      _Pragma("unroll") for (int q = 0; q < kNS; ++q) {          \
        if (nbr[q] < 0) continue;                                \
        const double y = Y(p, nbr[q]);                           \
        vq += cq[q] * y;                                         \
        if (q < kN5) vk += ck[q] * y;                            \
      }                                                          \
      _Pragma("unroll") for (int d = 0; d < 3; ++d) {            \
        const int s = p - d;                                     \
        if (s >= 0 && s < kS) {                                  \
          acc[s][d] += mu_[s] * vq;                              \
          acc[s][3 + d] += mu_[s] * vk;                          \
        }                                                        \
      }                                                          \
    }                                                            \
  }
  const float inv_wn = wn > 0 ? 1.0f / (float)wn : 0.0f, inv_np = 1.0f / (float)nP;
  if (sk > 0) {
    for (int k0 = 0; k0 < n_k; k0 += sk) {
      const int kc = min(sk, n_k - k0);
      const int tot = kc * nP * wn;
      // kMcU loads in flight per thread, then their LDS stores
      for (int e0 = threadIdx.x; e0 < tot; e0 += kMcU * 256) {
        double v[kMcU];
#pragma unroll
        for (int u = 0; u < kMcU; ++u) {
          const int e = e0 + u * 256;
          const int jd = mc_div(e, wn, inv_wn), r = e - jd * wn;
          const int j = mc_div(jd, nP, inv_np), d = jd - j * nP;
          const double* pm = RBMC_MC_PANEL(d);
          v[u] = e < tot && pm ? G(pm)[(size_t)(k0 + j) * tk.np + w0 + r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kMcU; ++u)
          if (e0 + u * 256 < tot) win[e0 + u * 256] = v[u];
      }
      __syncthreads();
      if (mine)
        for (int j = 0; j < kc; ++j) {
          const int wj = j * nP * wn - w0;
#define RBMC_MC_LDS(d, row) win[wj + (d) * wn + (row)]
#define RBMC_MC_MU(s) win[wj + ((s) + 1) * wn + a]
          RBMC_MC_SAMPLE(RBMC_MC_MU, RBMC_MC_LDS)
#undef RBMC_MC_MU
#undef RBMC_MC_LDS
        }
      __syncthreads();
    }
  } else if (!MULTI && mine) {
    for (int k = 0; k < n_k; ++k) {
      const size_t off = (size_t)k * tk.np;
#define RBMC_MC_GLOBAL(d, row) \
  (RBMC_MC_PANEL(d) ? G(RBMC_MC_PANEL(d))[off + (row)] : 0.0)
#define RBMC_MC_GMU(s) RBMC_MC_GLOBAL((s) + 1, a)
      RBMC_MC_SAMPLE(RBMC_MC_GMU, RBMC_MC_GLOBAL)
#undef RBMC_MC_GMU
#undef RBMC_MC_GLOBAL
    }
  }
#undef RBMC_MC_SAMPLE
#undef RBMC_MC_PANEL
  // per step: diagonal, then the 8 partial sums of the workgroup; the ratio
  // m_a / s2_a (MC part over estimate) feeds the plug-in error estimate
  const int nch = mc_chunks(tk.np);
#pragma unroll
  for (int s = 0; s < kS; ++s) {
    if (s >= S) break;
#pragma unroll
    for (int c = 0; c < 8; ++c) red[c][threadIdx.x] = acc[s][c];
    __syncthreads();
    double ratio = 0.0;
    if (mine) {
      const size_t i = (size_t)(tk.t + s) * m.ns + node;
      const double mhat = red[7][threadIdx.x] * tk.scale;
      const double est = G(tk.diag_out)[i] + mhat;
      G(tk.diag_out)[i] = est;
      ratio = est > 0.0 ? mhat / est : 0.0;
    }
    __syncthreads();
    red[7][threadIdx.x] = ratio;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st)
        for (int c = 0; c < 8; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x < 8) {
      const double v = threadIdx.x == 7 ? red[7][0] : red[threadIdx.x][0] * tk.scale;
      const size_t at = ((size_t)tk.out_index + (size_t)s * nch + chunk) * 8 + threadIdx.x;
      G(tk.partial)[at] = tk.accum ? G(tk.partial)[at] + v : v;
    }
    __syncthreads();
  }
}

// Alg. 2: Var(x_S) from the zero-mean samples, one thread per separator node:
// diag[sep[i]] = (accum ? diag[sep[i]] : 0) + scale sum_k x_k[sep[i]]^2,
// column k of x at x + k ldx (no columns when nk = 0)
__global__ __launch_bounds__(256) void k_sep_var(const int* __restrict__ sep, int nsep,
                                                 const double* __restrict__ x, long ldx, int nk,
                                                 double scale, int accum,
                                                 double* __restrict__ diag) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nsep) return;
  const int node = G(sep)[i];
  double acc = 0.0;
  for (int k = 0; k < nk; ++k) {
    const double v = G(x)[(size_t)k * ldx + node];
    acc += v * v;
  }
  const gptr<double> d = G(diag);
  d[node] = (accum ? d[node] : 0.0) + scale * acc;
}

void launch_sep_var(const int* sep, int nsep, const double* x, long ldx, int nk, double scale,
                    int accum, double* diag, hipStream_t s) {
  if (nsep <= 0) return;
  k_sep_var<<<(nsep + 255) / 256, 256, 0, s>>>(sep, nsep, x, ldx, nk, scale, accum, diag);
}

int mc_max_steps() { return kMcS; }
int mc_lds_doubles() { return kMcLds; }

void launch_mc(const McTask* d_tasks, int n_tasks, int total_tiles, int multi, hipStream_t s) {
  if (total_tiles <= 0) return;
  if (multi)
    k_mc<true><<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
  else
    k_mc<false><<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

}  // namespace rbmc
