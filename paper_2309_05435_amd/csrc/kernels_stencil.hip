// Matrix-free space-time operators and the PCG vector kernels.
//
// Q = Q_t (x) Q_s + D is applied as the 13-point spatial stencil of Q_s on
// each time layer followed by a 3-point time combination:
//   u_t = Q_s x_t,   (Q x)_t = q_{t,t-1} u_{t-1} + q_{t,t} u_t + q_{t,t+1} u_{t+1} + D_t x_t.
// A workgroup owns a 32 x 16 spatial tile of one column (model, sample) and
// walks through time.  Each layer of the tile (with a halo of 2) passes once
// through LDS (two slots, alternating by step parity); a thread keeps the
// stencil results u of its two nodes for three consecutive layers in
// registers, so every x value is read from HBM once per application and each
// step needs a single barrier.  The spatial stencil coefficients of a thread's
// two nodes do not depend on time: they are read once, into registers, before
// the walk.
//
// All kernels work on column sets: a column is one sample of one model, with
// its own length and offset, so one launch serves many uneven models.
#include "rbmc_impl.h"

namespace rbmc {

namespace {

constexpr int TX = 32, TY = 16, HX = TX + 4, HY = TY + 4;
constexpr int NTHR = 256;

// Weights of the time combination for output step t.
__device__ inline void time_weights(const DevModel& m, int kind, int t, double& wm, double& w0,
                                    double& wp) {
  if (kind == 3) {
    wm = m.dqo;
    w0 = m.dqd[t];
    wp = m.dqo;
  } else if (kind == 5) {
    wm = 0.0;  // F_t = L^T: (t,t) -> L_tt, (t,t+1) -> L_{t+1,t}
    w0 = m.ld[t];
    wp = m.lo;
  } else if (kind == 4) {
    wm = 0.0;
    w0 = 0.0;
    wp = 0.0;
  } else {
    wm = m.qo;
    w0 = m.qd[t];
    wp = m.qo;
  }
  if (t == 0) wm = 0.0;
  if (t == m.T - 1) wp = 0.0;
}

// KIND: 0 Q, 1 dQ/dlog kappa, 2 dQ/dlog tau, 3 dQ/drho, 4 dQ/dlog sigma, 5 F.
// Grid (max tiles, columns); DOT: partial sums of x.y per (column, tile).
template <int KIND, bool DOT>
__global__ __launch_bounds__(NTHR, 4) void k_space_time_op(ColSet cs, const double* __restrict__ x,
                                                        double* __restrict__ y,
                                                        double* __restrict__ partial) {
  __shared__ double slot[2][HY * HX];
  __shared__ double red[NTHR];
  const int col = blockIdx.y;
  const DevModel& m = cs.dms[cs.model[col]];
  const int ntx = (m.mx + TX - 1) / TX;
  const int tile = blockIdx.x;
  const int tid = threadIdx.x;
  const bool live = tile < ntx * ((m.my + TY - 1) / TY);
  if (!live) {
    if (DOT && tid == 0) partial[(size_t)col * cs.max_tiles + tile] = 0.0;
    return;
  }
  const int bx = (tile % ntx) * TX, by = (tile / ntx) * TY;
  const double* xk = x + (KIND == 5 ? cs.in_off[col] : cs.off[col]);
  double* yk = y + cs.off[col];
  const int T = m.T;
  // a sample's node indices fit 32 bits (the planner refuses larger models)
  const uint32_t ns = (uint32_t)m.ns;
  const int lx = tid % TX, ly = tid / TX;  // ly in [0, 8): rows ly and ly + 8
  // the thread's two nodes: spatial index (0 outside the grid) and whether inside
  int sn[2];
  bool in[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int gx = bx + lx, gy = by + ly + 8 * h;
    in[h] = gx < m.mx && gy < m.my;
    sn[h] = in[h] ? gy * m.mx + gx : 0;
  }
  double acc = 0.0;
  if (KIND == 4) {  // diagonal only: -2 D
    for (int t = 0; t < T; ++t) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (!in[h]) continue;
        const size_t i = (size_t)t * ns + sn[h];
        const double xi = xk[i];
        const double v = obs_at(m, i) ? -2.0 * m.dobs * xi : 0.0;
        yk[i] = v;
        if (DOT) acc += v * xi;
      }
    }
  } else {
    // stencil coefficients of the thread's two nodes (13 for Q_s, 5 for K, F_s)
    constexpr int NC = (KIND == 0 || KIND == 2 || KIND == 3) ? kNS : kN5;
    const double* __restrict__ cf_src = (KIND == 1) ? m.kk : (KIND == 5) ? m.fs : m.qs;
    double cf[2][NC];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < NC; ++q) cf[h][q] = in[h] ? cf_src[(size_t)q * ns + sn[h]] : 0.0;

    // halo entries e = tid + NTHR j of the tile: spatial offset and whether
    // inside the grid (fixed over time).  A layer is fetched into registers two
    // steps ahead of its store to LDS (two register buffers, alternating by
    // step parity), so its loads are in flight during two steps' arithmetic.
    // The loads are unconditional: entries outside the grid or the time range
    // read element 0 and are stored as 0.
    constexpr int NL = (HX * HY + NTHR - 1) / NTHR;
    int hoff[NL];
    bool hin[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int e = tid + NTHR * j;
      const int gx = bx + e % HX - 2, gy = by + e / HX - 2;
      hin[j] = e < HX * HY && gx >= 0 && gx < m.mx && gy >= 0 && gy < m.my;
      hoff[j] = hin[j] ? gy * m.mx + gx : 0;
    }
    double preA[NL], preB[NL];
#define RBMC_ST_FETCH(TT, PRE)                                                        \
  _Pragma("unroll") for (int j = 0; j < NL; ++j) {                                  \
    const bool ok_ = hin[j] && (TT) < T;                                            \
    const double v_ = xk[ok_ ? (uint32_t)(TT) * ns + hoff[j] : 0u];                    \
    PRE[j] = ok_ ? v_ : 0.0;                                                        \
  }
#define RBMC_ST_PUT(BUF, PRE)                                                         \
  _Pragma("unroll") for (int j = 0; j < NL; ++j) {                                  \
    const int e_ = tid + NTHR * j;                                                  \
    if (e_ < HX * HY) slot[BUF][e_] = PRE[j];                                       \
  }
    // LDS index of each node's centre
    int ctr[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) ctr[h] = (ly + 8 * h + 2) * HX + lx + 2;
    auto stencil = [&](int buf, int h) {
      const double* sl = slot[buf] + ctr[h];
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < NC; ++q) v += cf[h][q] * sl[kSdy[q] * HX + kSdx[q]];
      return v;
    };
    double um[2] = {0.0, 0.0}, u0[2], up[2];
    // one output step t: layer t + 1 from the register buffer into slot
    // (t + 1) & 1, layer t + 3 fetched into the same buffer, u_{t+1} from LDS.
    // Slot (t + 1) & 1 was last read before the previous step's barrier (x_{t-1}
    // at the nodes) or after the barrier before it (u_{t-1}).
#define RBMC_ST_STEP(TT, PRE)                                                         \
  {                                                                                 \
    const int t_ = (TT);                                                            \
    double wm, w0, wp;                                                              \
    time_weights(m, KIND, t_, wm, w0, wp);                                          \
    double xt[2];                                                                   \
    uint32_t ob[2];                                                                 \
    _Pragma("unroll") for (int h = 0; h < 2; ++h) {                                 \
      xt[h] = slot[t_ & 1][ctr[h]];                                                 \
      ob[h] = (KIND == 0 || KIND == 5) ? m.obs_bits[((uint32_t)t_ * ns + sn[h]) >> 5] : 0u; \
    }                                                                               \
    RBMC_ST_PUT((t_ + 1) & 1, PRE)                                                  \
    RBMC_ST_FETCH(t_ + 3, PRE)                                                      \
    __syncthreads();                                                                \
    _Pragma("unroll") for (int h = 0; h < 2; ++h) {                                 \
      up[h] = stencil((t_ + 1) & 1, h);                                             \
      const uint32_t i = (uint32_t)t_ * ns + sn[h];                                 \
      const bool o = (ob[h] >> (i & 31)) & 1u;                                      \
      double v = wm * um[h] + w0 * u0[h] + wp * up[h];                              \
      if (KIND == 0 && o) v += m.dobs * xt[h];                                      \
      if (KIND == 5 && o) v += sqrt(m.dobs) * xk[(size_t)m.n + obs_rank_at(m, i)];  \
      if (in[h]) {                                                                  \
        yk[i] = v;                                                                  \
        if (DOT) acc += v * xt[h];                                                  \
      }                                                                             \
      um[h] = u0[h];                                                                \
      u0[h] = up[h];                                                                \
    }                                                                               \
  }
    // layer 0 into slot 0 and u_0; layers 1 and 2 in flight
    RBMC_ST_FETCH(0, preA)
    RBMC_ST_PUT(0, preA)
    RBMC_ST_FETCH(1, preA)
    RBMC_ST_FETCH(2, preB)
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) u0[h] = stencil(0, h);
    for (int t = 0; t < T; t += 2) {
      RBMC_ST_STEP(t, preA)
      if (t + 1 < T) RBMC_ST_STEP(t + 1, preB)
    }
#undef RBMC_ST_STEP
#undef RBMC_ST_PUT
#undef RBMC_ST_FETCH
  }
  if (DOT) {
    red[tid] = acc;
    __syncthreads();
    for (int st = NTHR / 2; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    if (tid == 0) partial[(size_t)col * cs.max_tiles + tile] = red[0];
  }
}

}  // namespace

int stencil_tiles(int mx, int my) { return ((mx + TX - 1) / TX) * ((my + TY - 1) / TY); }

// An empty kernel of this file: launching it makes the runtime load this
// file's device code (each source file's kernels form their own code object,
// loaded on the first launch of any of them).
__global__ void k_load_stencil_module() {}

void load_stencil_module(hipStream_t s) { k_load_stencil_module<<<1, 64, 0, s>>>(); }

void launch_apply_op(const ColSet& cs, int op, const double* x, double* y, hipStream_t s) {
  if (cs.ncols <= 0) return;
  dim3 grid(cs.max_tiles, cs.ncols);
  switch (op) {
    case RBMC_OP_Q: k_space_time_op<0, false><<<grid, NTHR, 0, s>>>(cs, x, y, nullptr); break;
    case RBMC_OP_DQ_LOGKAPPA: k_space_time_op<1, false><<<grid, NTHR, 0, s>>>(cs, x, y, nullptr); break;
    case RBMC_OP_DQ_LOGTAU: k_space_time_op<2, false><<<grid, NTHR, 0, s>>>(cs, x, y, nullptr); break;
    case RBMC_OP_DQ_RHO: k_space_time_op<3, false><<<grid, NTHR, 0, s>>>(cs, x, y, nullptr); break;
    case RBMC_OP_DQ_LOGSIGMA: k_space_time_op<4, false><<<grid, NTHR, 0, s>>>(cs, x, y, nullptr); break;
    case RBMC_OP_F: k_space_time_op<5, false><<<grid, NTHR, 0, s>>>(cs, x, y, nullptr); break;
    default: break;
  }
}

void launch_spmm_dot(const ColSet& cs, const double* p, double* q, double* partial,
                     hipStream_t s) {
  if (cs.ncols <= 0) return;
  dim3 grid(cs.max_tiles, cs.ncols);
  k_space_time_op<0, true><<<grid, NTHR, 0, s>>>(cs, p, q, partial);
}

// ---------------------------------------------------------------------------
// Deterministic per-column reductions: partial[k * nchunk + c] -> out[k]
// ---------------------------------------------------------------------------

__global__ void k_reduce_partials(const double* __restrict__ partial, int nchunk,
                                  double* __restrict__ out) {
  __shared__ double red[256];
  const int k = blockIdx.x, tid = threadIdx.x;
  double a = 0.0;
  for (int c = tid; c < nchunk; c += 256) a += partial[(size_t)k * nchunk + c];
  red[tid] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) out[k] = red[0];
}

void launch_reduce_partials(const double* partial, int nchunk, int n_rhs, double* out,
                            hipStream_t s) {
  if (n_rhs > 0) k_reduce_partials<<<n_rhs, 256, 0, s>>>(partial, nchunk, out);
}

constexpr int kDotBlock = 256, kDotPer = 8;
int dot_chunks(int n) { return (n + kDotBlock * kDotPer - 1) / (kDotBlock * kDotPer); }

// grid (dot_chunks(max_len), ncols); partial[col * nchunk + chunk]
__global__ void k_dot_partials(ColSet cs, const double* __restrict__ a,
                               const double* __restrict__ b, double* __restrict__ partial,
                               int nchunk) {
  __shared__ double red[kDotBlock];
  const int col = blockIdx.y, c = blockIdx.x, tid = threadIdx.x;
  const int n = cs.len[col];
  const double* ak = a + cs.off[col];
  const double* bk = b + cs.off[col];
  double acc = 0.0;
  const int base = c * kDotBlock * kDotPer;
#pragma unroll
  for (int j = 0; j < kDotPer; ++j) {
    int i = base + j * kDotBlock + tid;
    if (i < n) acc += ak[i] * bk[i];
  }
  red[tid] = acc;
  __syncthreads();
  for (int st = kDotBlock / 2; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) partial[(size_t)col * nchunk + c] = red[0];
}

void launch_dot_partials(const ColSet& cs, const double* a, const double* b, double* partial,
                         hipStream_t s) {
  if (cs.ncols <= 0) return;
  const int nch = dot_chunks(cs.max_len);
  k_dot_partials<<<dim3(nch, cs.ncols), kDotBlock, 0, s>>>(cs, a, b, partial, nch);
}

// x += alpha p ; r -= alpha q ; partial sums of r.r   (alpha = rz / pq, 0 if inactive)
__global__ void k_pcg_xr(ColSet cs, const double* __restrict__ p, const double* __restrict__ q,
                         double* __restrict__ x, double* __restrict__ r,
                         const double* __restrict__ rz, const double* __restrict__ pq,
                         const uint8_t* __restrict__ active, double* __restrict__ partial,
                         int nchunk) {
  __shared__ double red[kDotBlock];
  const int k = blockIdx.y, c = blockIdx.x, tid = threadIdx.x;
  const double alpha = active[k] ? rz[k] / pq[k] : 0.0;
  const size_t off = cs.off[k];
  const int n = cs.len[k];
  double acc = 0.0;
  const int base = c * kDotBlock * kDotPer;
#pragma unroll
  for (int j = 0; j < kDotPer; ++j) {
    int i = base + j * kDotBlock + tid;
    if (i < n) {
      double rv = r[off + i];
      if (alpha != 0.0) {
        x[off + i] += alpha * p[off + i];
        rv -= alpha * q[off + i];
        r[off + i] = rv;
      }
      acc += rv * rv;
    }
  }
  red[tid] = acc;
  __syncthreads();
  for (int st = kDotBlock / 2; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) partial[(size_t)k * nchunk + c] = red[0];
}

void launch_pcg_xr(const ColSet& cs, const double* p, const double* q, double* x, double* r,
                   const double* rz, const double* pq, const uint8_t* active,
                   double* rr_partial, hipStream_t s) {
  if (cs.ncols <= 0) return;
  const int nch = dot_chunks(cs.max_len);
  k_pcg_xr<<<dim3(nch, cs.ncols), kDotBlock, 0, s>>>(cs, p, q, x, r, rz, pq, active, rr_partial,
                                                     nch);
}

// p = z + beta p (first iteration: p = z); active columns only.
// beta = rz_new / rz_old, or (rz_new - rz_sub) / rz_old (flexible form, with
// rz_sub = r_new . z_old, for a preconditioner that varies between iterations)
__global__ void k_pcg_p(ColSet cs, const double* __restrict__ z, double* __restrict__ p,
                        const double* __restrict__ rz_new, const uint8_t* __restrict__ active,
                        const double* __restrict__ rz_old, const double* __restrict__ rz_sub,
                        int first) {
  const int k = blockIdx.y;
  if (!active[k]) return;
  const double beta =
      first ? 0.0 : (rz_sub ? rz_new[k] - rz_sub[k] : rz_new[k]) / rz_old[k];
  const size_t off = cs.off[k];
  const int n = cs.len[k];
  // the first direction does not read p: its previous contents may be any
  // bit pattern (0 times a stale NaN is NaN)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[off + i] = first ? z[off + i] : z[off + i] + beta * p[off + i];
}

__global__ void k_copy_scalars(const double* __restrict__ src, double* __restrict__ dst,
                               const uint8_t* __restrict__ active, int n_rhs) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_rhs && active[k]) dst[k] = src[k];
}

void launch_pcg_p(const ColSet& cs, const double* z, double* p, const double* rz_new,
                  double* rz_old, const uint8_t* active, int first, hipStream_t s,
                  const double* rz_sub) {
  if (cs.ncols <= 0) return;
  const int bx = std::min((cs.max_len + 255) / 256, 1024);
  k_pcg_p<<<dim3(bx, cs.ncols), 256, 0, s>>>(cs, z, p, rz_new, active, rz_old, rz_sub, first);
  k_copy_scalars<<<(cs.ncols + 255) / 256, 256, 0, s>>>(rz_new, rz_old, active, cs.ncols);
}

// convergence test per column: active <- active && ||r|| > rtol ||b||; count iterations
__global__ void k_pcg_check(const double* __restrict__ rr, const double* __restrict__ bb,
                            double rtol, uint8_t* __restrict__ active, int* __restrict__ it_count,
                            int* __restrict__ n_active, int n_rhs) {
  __shared__ int cnt[256];
  int tid = threadIdx.x, c = 0;
  for (int k = tid; k < n_rhs; k += 256) {
    if (active[k]) {
      it_count[k] += 1;
      // a NaN residual is not convergence: the column keeps iterating to the
      // iteration limit and the call reports it
      if (sqrt(rr[k]) <= rtol * sqrt(bb[k])) active[k] = 0;
    }
    c += active[k] ? 1 : 0;
  }
  cnt[tid] = c;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) cnt[tid] += cnt[tid + st];
    __syncthreads();
  }
  if (tid == 0) *n_active = cnt[0];
}

void launch_pcg_check(const double* rr, const double* bb, double rtol, uint8_t* active,
                      int* it_count, int* n_active, int n_rhs, hipStream_t s) {
  k_pcg_check<<<1, 256, 0, s>>>(rr, bb, rtol, active, it_count, n_active, n_rhs);
}

// ---------------------------------------------------------------------------
// Spectral preconditioner M = Q_t (x) Q_s + dbar I.  Q_s is a polynomial in
// the Neumann grid Laplacian G = G_x (+) G_y, which the 2-D DCT-II
// diagonalizes; in that basis M splits into one symmetric tridiagonal
// T x T system per spatial frequency f:
//   (lambda_f Q_t + dbar I) y_f = r_f,
// diagonal lambda_f q_d(t) + dbar, off-diagonal lambda_f q_o.  The forward
// elimination coefficients c'_t = a / den_t and 1 / den_t (den_0 = b_0,
// den_t = b_t - a c'_{t-1}) depend on f and t only: they are formed once per
// theta; the solve then streams each column forward and back.
// ---------------------------------------------------------------------------
__global__ void k_spec_coef(SpecCoefTask tk) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= tk.ns) return;
  const double lam = tk.lam[f];
  const double a = lam * tk.qo;
  double cp = 0.0;
  for (int t = 0; t < tk.T; ++t) {
    const double b = lam * tk.qd[t] + tk.dbar;
    const double den = (t == 0) ? b : b - a * cp;
    cp = a / den;
    tk.cp[(size_t)t * tk.ns + f] = cp;
    tk.id[(size_t)t * tk.ns + f] = 1.0 / den;
  }
  tk.off[f] = a;
}

void launch_spec_coef(const SpecCoefTask& t, hipStream_t s) {
  if (t.ns > 0) k_spec_coef<<<(t.ns + 255) / 256, 256, 0, s>>>(t);
}

// One thread per (column, frequency f): the tridiagonal solve of the T values
// y[t ns + f].  Column-major grid (columns in grid.x, frequency blocks in
// grid.y) when the frequency blocks fit grid.y: the workgroups resident at
// one time then share their frequencies, so the coefficients c'_t and
// 1 / den_t of those frequencies are read from HBM about once per XCD instead
// of once per column.
namespace {
constexpr int kSpecCh = 8;

struct SpecIdx {
  int col, f;
};
__device__ inline SpecIdx spec_idx(int colfast) {
  return colfast ? SpecIdx{(int)blockIdx.x, (int)(blockIdx.y * 256 + threadIdx.x)}
                 : SpecIdx{(int)blockIdx.y, (int)(blockIdx.x * 256 + threadIdx.x)};
}
}  // namespace

// T <= TR: the column lives in registers (one read and one write of y); the
// loads of each sweep's coefficients are issued together.
template <int TR>
__global__ __launch_bounds__(256) void k_spec_solve_reg(ColSet cs, double* __restrict__ y,
                                                        int colfast) {
  const SpecIdx ix = spec_idx(colfast);
  const DevModel& m = cs.dms[cs.model[ix.col]];
  const int f = ix.f;
  if (f >= m.ns || m.sp_cp == nullptr) return;
  const gptr<double> yk = G(y + cs.off[ix.col]);
  const gptr<const double> id = G((const double*)m.sp_id), cp = G((const double*)m.sp_cp);
  const double a = m.sp_off[f];
  const int T = m.T;
  // a sample's node indices fit 32 bits (the planner refuses larger models)
  const uint32_t ns = (uint32_t)m.ns;
  double v[TR];
#pragma unroll
  for (int t = 0; t < TR; ++t)
    if (t < T) v[t] = yk[t * ns + f];
  double prev = 0.0;
#pragma unroll
  for (int t = 0; t < TR; ++t)  // forward elimination
    if (t < T) {
      prev = (v[t] - a * prev) * id[t * ns + f];
      v[t] = prev;
    }
#pragma unroll
  for (int t = TR - 2; t >= 0; --t)  // back substitution
    if (t < T - 1) {
      prev = v[t] - cp[t * ns + f] * prev;
      v[t] = prev;
    }
#pragma unroll
  for (int t = 0; t < TR; ++t)
    if (t < T) yk[t * ns + f] = v[t];
}

// Any T: the walk in time goes in chunks of kSpecCh steps (the chunk's loads
// are issued together, then the recurrence runs in registers and the chunk is
// stored); the forward results pass through y.
__global__ __launch_bounds__(256) void k_spec_solve(ColSet cs, double* __restrict__ y,
                                                    int colfast) {
  const SpecIdx ix = spec_idx(colfast);
  const DevModel& m = cs.dms[cs.model[ix.col]];
  const int f = ix.f;
  if (f >= m.ns || m.sp_cp == nullptr) return;
  const gptr<double> yk = G(y + cs.off[ix.col]);
  const gptr<const double> id = G((const double*)m.sp_id), cp = G((const double*)m.sp_cp);
  const double a = m.sp_off[f];
  const int T = m.T;
  const uint32_t ns = (uint32_t)m.ns;
  double prev = 0.0, v[kSpecCh], c[kSpecCh];
  for (int t0 = 0; t0 < T; t0 += kSpecCh) {  // forward elimination
#pragma unroll
    for (int j = 0; j < kSpecCh; ++j)
      if (t0 + j < T) {
        v[j] = yk[(t0 + j) * ns + f];
        c[j] = id[(t0 + j) * ns + f];
      }
#pragma unroll
    for (int j = 0; j < kSpecCh; ++j)
      if (t0 + j < T) {
        prev = (v[j] - a * prev) * c[j];
        v[j] = prev;
      }
#pragma unroll
    for (int j = 0; j < kSpecCh; ++j)
      if (t0 + j < T) yk[(t0 + j) * ns + f] = v[j];
  }
  for (int t1 = T - 1; t1 > 0; t1 -= kSpecCh) {  // back substitution, steps t1 - 1 down
#pragma unroll
    for (int j = 0; j < kSpecCh; ++j) {
      const int t = t1 - 1 - j;
      if (t >= 0) {
        v[j] = yk[t * ns + f];
        c[j] = cp[t * ns + f];
      }
    }
#pragma unroll
    for (int j = 0; j < kSpecCh; ++j)
      if (t1 - 1 - j >= 0) {
        prev = v[j] - c[j] * prev;
        v[j] = prev;
      }
#pragma unroll
    for (int j = 0; j < kSpecCh; ++j)
      if (t1 - 1 - j >= 0) yk[(t1 - 1 - j) * ns + f] = v[j];
  }
}

void launch_spec_solve(const ColSet& cs, double* y, hipStream_t s) {
  if (cs.ncols <= 0) return;
  // the largest model's spatial size bounds the frequency index
  const int fb = (cs.max_ns + 255) / 256;
  const int colfast = fb <= 65535 ? 1 : 0;
  const dim3 grid = colfast ? dim3(cs.ncols, fb) : dim3(fb, cs.ncols);
  if (cs.max_T <= 16)
    k_spec_solve_reg<16><<<grid, 256, 0, s>>>(cs, y, colfast);
  else if (cs.max_T <= 32)
    k_spec_solve_reg<32><<<grid, 256, 0, s>>>(cs, y, colfast);
  else if (cs.max_T <= 48)
    k_spec_solve_reg<48><<<grid, 256, 0, s>>>(cs, y, colfast);
  else if (cs.max_T <= 64)
    k_spec_solve_reg<64><<<grid, 256, 0, s>>>(cs, y, colfast);
  else
    k_spec_solve<<<grid, 256, 0, s>>>(cs, y, colfast);
}

// Direct transform along one axis for models without the GEMM route:
// forward  y[.., k, ..] = sum_i C[k, i] x[.., i, ..];  inverse uses C^T.
// grid (element blocks of the longest column, columns)
__global__ __launch_bounds__(256) void k_dct_direct(ColSet cs, const double* __restrict__ x,
                                                    double* __restrict__ y, int axis,
                                                    int inverse) {
  const int col = blockIdx.y;
  const DevModel& m = cs.dms[cs.model[col]];
  if (m.spec_gemm || m.dct_x == nullptr) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= cs.len[col]) return;
  const int t = i / m.ns, rem = i - t * m.ns, iy = rem / m.mx, ix = rem - iy * m.mx;
  const double* xk = x + cs.off[col];
  const int len = axis == 0 ? m.mx : m.my;
  const int k = axis == 0 ? ix : iy;
  const int stride = axis == 0 ? 1 : m.mx;
  const double* C = axis == 0 ? m.dct_x : m.dct_y;
  const size_t base = (size_t)t * m.ns + (axis == 0 ? (size_t)iy * m.mx : (size_t)ix);
  double acc = 0.0;
  for (int j = 0; j < len; ++j) {
    const double c = inverse ? C[(size_t)k * len + j] : C[(size_t)j * len + k];
    acc = fma(c, xk[base + (size_t)j * stride], acc);
  }
  y[cs.off[col] + i] = acc;
}

void launch_dct_direct(const ColSet& cs, const double* x, double* y, int axis, int inverse,
                       hipStream_t s) {
  if (cs.ncols <= 0) return;
  k_dct_direct<<<dim3((cs.max_len + 255) / 256, cs.ncols), 256, 0, s>>>(cs, x, y, axis, inverse);
}

}  // namespace rbmc
