// 3-D convolutions of the learned correction to the block-Jacobi
// preconditioner: 3 x 3 x 3 kernels over the space-time grid (t, y, x) of a
// sample, no bias, zero outside the valid box of each volume.  Weights are
// stored in BF16 and widened to FP32; activations and accumulation are FP32.
//
// Layout: a batch of B volumes, each C channels x (T x MY x MX) voxels,
// channel-major (voxel index (t * MY + y) * MX + x, the node order of the
// model).  Weights W[co][ci][tap], tap = (dt + 1) * 9 + (dy + 1) * 3 + (dx + 1).
#include "rbmc_impl.h"

namespace rbmc {

namespace {
constexpr int CT = 4, CY = 8, CX = 32;              // output tile per workgroup
constexpr int HT = CT + 2, HY = CY + 2, HX = CX + 2;
constexpr int HV = HT * HY * HX;                    // staged input voxels per channel
constexpr int CCH = 4;                              // input channels staged per pass

__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
}  // namespace

int conv_tiles(const ConvGeom& g) {
  return ((g.T + CT - 1) / CT) * ((g.MY + CY - 1) / CY) * ((g.MX + CX - 1) / CX);
}

// out[b][co] (=|+=) scale * sum_ci sum_tap W[co][ci][tap] f(in[b][ci][v + tap]) (* [mask > 0])
// with f = max(0, .) when relu_in; voxels outside the valid box of volume b
// read as zero and are written as zero.  Grid (tiles, B); 256 threads, each
// owning one (y, x) column of the tile and its CT time steps.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv3d(ConvArgs a) {
  constexpr int NCH = CIN < CCH ? CIN : CCH;
  __shared__ float tile[NCH * HV];
  __shared__ __align__(16) float ws[NCH * 27 * COUT];
  const ConvGeom g = a.geom;
  const int b = blockIdx.y;
  const ConvBox box = a.boxes ? a.boxes[b] : ConvBox{0, g.T, 0, g.MY, 0, g.MX};
  const int ntx = (g.MX + CX - 1) / CX, nty = (g.MY + CY - 1) / CY;
  const int tile_id = blockIdx.x;
  const int tx = tile_id % ntx, ty = (tile_id / ntx) % nty, tt = tile_id / (ntx * nty);
  const int x0 = tx * CX, y0 = ty * CY, t0 = tt * CT;
  const int tid = threadIdx.x, lx = tid & (CX - 1), ly = tid >> 5;
  const size_t V = (size_t)g.T * g.MY * g.MX;
  const float* in = a.in + (size_t)b * CIN * V;

  float acc[COUT][CT];
#pragma unroll
  for (int co = 0; co < COUT; ++co)
#pragma unroll
    for (int k = 0; k < CT; ++k) acc[co][k] = 0.f;

  for (int c0 = 0; c0 < CIN; c0 += NCH) {
    __syncthreads();
    for (int e = tid; e < NCH * HV; e += 256) {
      const int cl = e / HV, r = e % HV;
      const int hx = r % HX, hy = (r / HX) % HY, ht = r / (HX * HY);
      const int t = t0 - 1 + ht, y = y0 - 1 + hy, x = x0 - 1 + hx;
      float v = 0.f;
      if (t >= box.t0 && t < box.t1 && y >= box.y0 && y < box.y1 && x >= box.x0 && x < box.x1) {
        v = in[(size_t)(c0 + cl) * V + ((size_t)t * g.MY + y) * g.MX + x];
        if (a.relu_in) v = fmaxf(v, 0.f);
      }
      tile[e] = v;
    }
    for (int e = tid; e < NCH * 27 * COUT; e += 256) {  // ws[cl][tap][co]
      const int co = e % COUT, tap = (e / COUT) % 27, cl = e / (COUT * 27);
      ws[e] = bf16_to_f32(a.w[((size_t)co * CIN + c0 + cl) * 27 + tap]);
    }
    __syncthreads();
#pragma unroll 1
    for (int cl = 0; cl < NCH; ++cl) {
#pragma unroll 1
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          float col[HT];
#pragma unroll
          for (int h = 0; h < HT; ++h) col[h] = tile[cl * HV + (h * HY + ly + dy) * HX + lx + dx];
#pragma unroll
          for (int dt = 0; dt < 3; ++dt) {
            const float* wp = &ws[(cl * 27 + dt * 9 + dy * 3 + dx) * COUT];
#pragma unroll
            for (int co = 0; co < COUT; ++co) {
              const float wv = wp[co];
#pragma unroll
              for (int k = 0; k < CT; ++k) acc[co][k] = fmaf(wv, col[k + dt], acc[co][k]);
            }
          }
        }
    }
  }
  const int y = y0 + ly, x = x0 + lx;
  if (y >= g.MY || x >= g.MX) return;
  float* out = a.out + (size_t)b * COUT * V;
  const float* mask = a.mask ? a.mask + (size_t)b * COUT * V : nullptr;
#pragma unroll
  for (int k = 0; k < CT; ++k) {
    const int t = t0 + k;
    if (t >= g.T) break;
    const bool valid = t >= box.t0 && t < box.t1 && y >= box.y0 && y < box.y1 && x >= box.x0 &&
                       x < box.x1;
    const size_t v = ((size_t)t * g.MY + y) * g.MX + x;
#pragma unroll
    for (int co = 0; co < COUT; ++co) {
      float r = valid ? a.scale * acc[co][k] : 0.f;
      if (mask && !(mask[(size_t)co * V + v] > 0.f)) r = 0.f;
      if (a.accumulate) out[(size_t)co * V + v] += r;
      else out[(size_t)co * V + v] = r;
    }
  }
}

void launch_conv3d(const ConvArgs& a, int cin, int cout, int batch, hipStream_t s) {
  const dim3 grid(conv_tiles(a.geom), batch);
  if (cin == 2 && cout == 16) k_conv3d<2, 16><<<grid, 256, 0, s>>>(a);
  else if (cin == 16 && cout == 16) k_conv3d<16, 16><<<grid, 256, 0, s>>>(a);
  else if (cin == 16 && cout == 1) k_conv3d<16, 1><<<grid, 256, 0, s>>>(a);
  else if (cin == 1 && cout == 16) k_conv3d<1, 16><<<grid, 256, 0, s>>>(a);
}

// Weight gradient partial sums: for each workgroup (tile, batch item),
//   part[wg][co][ci][tap] = sum over the tile's valid voxels v of
//                            gout[b][co][v] * f(ain[b][ci][v + tap]).
// Thread = (pair (co, ci), tap group); the tile's gout and ain (with halo)
// are staged in LDS per input-channel chunk.
namespace {
constexpr int WT = 2, WY = 8, WX = 32;  // voxel tile of the weight gradient
constexpr int WHT = WT + 2, WHY = WY + 2, WHX = WX + 2, WHV = WHT * WHY * WHX;
constexpr int WV = WT * WY * WX;
}  // namespace

int conv_wgrad_tiles(const ConvGeom& g) {
  return ((g.T + WT - 1) / WT) * ((g.MY + WY - 1) / WY) * ((g.MX + WX - 1) / WX);
}

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv3d_wgrad(ConvWArgs a) {
  constexpr int NCH = CIN < CCH ? CIN : CCH;
  constexpr int NPAIR = COUT * NCH;
  constexpr int NGRP = 256 / NPAIR;                  // thread groups per pair
  constexpr int TPG = (27 + NGRP - 1) / NGRP;        // taps per group
  __shared__ float ain[NCH * WHV];
  __shared__ float gout[COUT * WV];
  const ConvGeom g = a.geom;
  const int b = blockIdx.y;
  const ConvBox box = a.boxes ? a.boxes[b] : ConvBox{0, g.T, 0, g.MY, 0, g.MX};
  const int ntx = (g.MX + WX - 1) / WX, nty = (g.MY + WY - 1) / WY;
  const int tx = blockIdx.x % ntx, ty = (blockIdx.x / ntx) % nty, tt = blockIdx.x / (ntx * nty);
  const int x0 = tx * WX, y0 = ty * WY, t0 = tt * WT;
  const int tid = threadIdx.x;
  const size_t V = (size_t)g.T * g.MY * g.MX;
  const size_t wg = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
  float* part = a.partial + wg * (size_t)COUT * CIN * 27;
  // output gradient of the tile (zero outside the valid box / grid)
  for (int e = tid; e < COUT * WV; e += 256) {
    const int co = e / WV, r = e % WV;
    const int x = x0 + r % WX, y = y0 + (r / WX) % WY, t = t0 + r / (WX * WY);
    float v = 0.f;
    if (t < g.T && y < g.MY && x < g.MX && t >= box.t0 && t < box.t1 && y >= box.y0 &&
        y < box.y1 && x >= box.x0 && x < box.x1)
      v = a.gout[((size_t)b * COUT + co) * V + ((size_t)t * g.MY + y) * g.MX + x];
    gout[e] = v;
  }
  const int pair = tid % NPAIR, grp = tid / NPAIR;
  const int co = pair / NCH, cl = pair % NCH;
  for (int c0 = 0; c0 < CIN; c0 += NCH) {
    __syncthreads();
    for (int e = tid; e < NCH * WHV; e += 256) {
      const int c = e / WHV, r = e % WHV;
      const int hx = r % WHX, hy = (r / WHX) % WHY, ht = r / (WHX * WHY);
      const int t = t0 - 1 + ht, y = y0 - 1 + hy, x = x0 - 1 + hx;
      float v = 0.f;
      if (t >= box.t0 && t < box.t1 && y >= box.y0 && y < box.y1 && x >= box.x0 && x < box.x1) {
        v = a.ain[((size_t)b * CIN + c0 + c) * V + ((size_t)t * g.MY + y) * g.MX + x];
        if (a.relu_in) v = fmaxf(v, 0.f);
      }
      ain[e] = v;
    }
    __syncthreads();
    float s[TPG];
#pragma unroll
    for (int j = 0; j < TPG; ++j) s[j] = 0.f;
    if (grp < NGRP) {
      for (int r = 0; r < WV; ++r) {
        const float gv = gout[co * WV + r];
        const int lx = r % WX, ly = (r / WX) % WY, lt = r / (WX * WY);
#pragma unroll
        for (int j = 0; j < TPG; ++j) {
          const int tap = grp * TPG + j;
          if (tap < 27) {
            const int dt = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
            s[j] = fmaf(gv, ain[cl * WHV + ((lt + dt) * WHY + ly + dy) * WHX + lx + dx], s[j]);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < TPG; ++j) {
        const int tap = grp * TPG + j;
        if (tap < 27) part[((size_t)co * CIN + c0 + cl) * 27 + tap] = s[j];
      }
    }
  }
}

void launch_conv3d_wgrad(const ConvWArgs& a, int cin, int cout, int batch, hipStream_t s) {
  const dim3 grid(conv_wgrad_tiles(a.geom), batch);
  if (cin == 2 && cout == 16) k_conv3d_wgrad<2, 16><<<grid, 256, 0, s>>>(a);
  else if (cin == 16 && cout == 16) k_conv3d_wgrad<16, 16><<<grid, 256, 0, s>>>(a);
  else if (cin == 16 && cout == 1) k_conv3d_wgrad<16, 1><<<grid, 256, 0, s>>>(a);
}

// sum over nwg partial rows of length len: out[i] = sum_w part[w * len + i]
__global__ void k_sum_rows(const float* __restrict__ part, int nwg, int len,
                           float* __restrict__ out) {
  const int i = blockIdx.x;
  __shared__ float red[256];
  float s = 0.f;
  for (int w = threadIdx.x; w < nwg; w += 256) s += part[(size_t)w * len + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

void launch_sum_rows(const float* part, int nwg, int len, float* out, hipStream_t s) {
  if (len > 0) k_sum_rows<<<len, 256, 0, s>>>(part, nwg, len, out);
}

// Flip and transpose weights for the input-gradient convolution:
// wt[ci][co][tap] = w[co][ci][26 - tap].
__global__ void k_conv_wflip(const uint16_t* __restrict__ w, int cin, int cout,
                             uint16_t* __restrict__ wt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cin * cout * 27) return;
  const int tap = e % 27, co = (e / 27) % cout, ci = e / (27 * cout);
  wt[e] = w[((size_t)co * cin + ci) * 27 + (26 - tap)];
}

void launch_conv_wflip(const uint16_t* w, int cin, int cout, uint16_t* wt, hipStream_t s) {
  const int n = cin * cout * 27;
  k_conv_wflip<<<(n + 255) / 256, 256, 0, s>>>(w, cin, cout, wt);
}

// Adam step on FP32 master weights; writes the BF16 copy (round to nearest even).
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ pb, int n, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = gr[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  uint32_t u = __float_as_uint(pi);
  u += 0x7fffu + ((u >> 16) & 1u);
  pb[i] = (uint16_t)(u >> 16);
}

void launch_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, int n, float lr,
                 float b1, float b2, float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  k_adam<<<(n + 255) / 256, 256, 0, s>>>(p, g, m, v, pb, n, lr, b1, b2, eps, c1, c2);
}

// FP32 -> BF16 copy (round to nearest even)
__global__ void k_to_bf16(const float* __restrict__ p, uint16_t* __restrict__ pb, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t u = __float_as_uint(p[i]);
  u += 0x7fffu + ((u >> 16) & 1u);
  pb[i] = (uint16_t)(u >> 16);
}

void launch_to_bf16(const float* p, uint16_t* pb, int n, hipStream_t s) {
  if (n > 0) k_to_bf16<<<(n + 255) / 256, 256, 0, s>>>(p, pb, n);
}

// ---------------------------------------------------------------------------
// Data movement of the learned correction
// ---------------------------------------------------------------------------

// Two-channel input volumes of the network from FP64 columns:
// vol[c][0][v] = r[c * n + v] * s_c,  vol[c][1][v] = u[c * n + v] * s_c,
// s_c = 1 / sqrt(rr[c]) (0 if rr[c] <= 0; 1 when rr is null).
__global__ void k_cols2_to_vol(const double* __restrict__ r, const double* __restrict__ u, size_t n,
                               const double* __restrict__ rr, float* __restrict__ vol) {
  const int c = blockIdx.y;
  const double r2 = rr ? rr[c] : 1.0;
  const double sc = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
  float* o = vol + (size_t)c * 2 * n;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (size_t)gridDim.x * blockDim.x) {
    o[v] = (float)(r[(size_t)c * n + v] * sc);
    o[n + v] = (float)(u[(size_t)c * n + v] * sc);
  }
}

void launch_cols2_to_vol(const double* r, const double* u, size_t n, const double* rr, float* vol,
                         int ncols, hipStream_t s) {
  if (ncols > 0) k_cols2_to_vol<<<dim3(256, ncols), 256, 0, s>>>(r, u, n, rr, vol);
}

// y[c * n + v] (=|+=) vol[c][v] * sqrt(rr[c]) (rr null: 1); active (if given) gates columns
__global__ void k_vol_to_cols(const float* __restrict__ vol, size_t n, const double* __restrict__ rr,
                              const uint8_t* __restrict__ active, double* __restrict__ y,
                              int accumulate) {
  const int c = blockIdx.y;
  if (active && !active[c]) return;
  const double sc = rr ? (rr[c] > 0.0 ? sqrt(rr[c]) : 0.0) : 1.0;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (size_t)gridDim.x * blockDim.x) {
    const double val = (double)vol[(size_t)c * n + v] * sc;
    if (accumulate) y[(size_t)c * n + v] += val;
    else y[(size_t)c * n + v] = val;
  }
}

void launch_vol_to_cols(const float* vol, size_t n, const double* rr, const uint8_t* active,
                        double* y, int ncols, int accumulate, hipStream_t s) {
  if (ncols > 0) k_vol_to_cols<<<dim3(256, ncols), 256, 0, s>>>(vol, n, rr, active, y, accumulate);
}

// Training pairs from PCG state: for each column c with slot[c] >= 0,
//   R[slot] = r_c / |r_c|,  U[slot] = u_c / |r_c|,  E[slot] = (xs_c - x_c) / |r_c|
// (|r_c|^2 = rr[c] > 0).  Grid (blocks, ncols).
__global__ void k_pair_store(const double* __restrict__ r, const double* __restrict__ u,
                             const double* __restrict__ xs, const double* __restrict__ x, size_t n,
                             const double* __restrict__ rr, const int* __restrict__ slot,
                             float* __restrict__ R, float* __restrict__ U, float* __restrict__ E) {
  const int c = blockIdx.y;
  const int sl = slot[c];
  if (sl < 0 || !(rr[c] > 0.0)) return;
  const double sc = 1.0 / sqrt(rr[c]);
  const size_t o = (size_t)sl * n, ci = (size_t)c * n;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (size_t)gridDim.x * blockDim.x) {
    R[o + v] = (float)(r[ci + v] * sc);
    U[o + v] = (float)(u[ci + v] * sc);
    E[o + v] = (float)((xs[ci + v] - x[ci + v]) * sc);
  }
}

void launch_pair_store(const double* r, const double* u, const double* xs, const double* x,
                       size_t n, const double* rr, const int* slot, float* R, float* U, float* E,
                       int ncols, hipStream_t s) {
  if (ncols > 0) k_pair_store<<<dim3(256, ncols), 256, 0, s>>>(r, u, xs, x, n, rr, slot, R, U, E);
}

// Network input of a training batch: vin[b][0] = R[sl_b], vin[b][1] = su * U[sl_b]
__global__ void k_pack_train(const float* __restrict__ R, const float* __restrict__ U,
                             const int* __restrict__ slots, size_t n, float su,
                             float* __restrict__ vin) {
  const int b = blockIdx.y;
  const size_t o = (size_t)slots[b] * n;
  float* d = vin + (size_t)b * 2 * n;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (size_t)gridDim.x * blockDim.x) {
    d[v] = R[o + v];
    d[n + v] = su * U[o + v];
  }
}

void launch_pack_train(const float* R, const float* U, const int* slots, size_t n, float su,
                       float* vin, int batch, hipStream_t s) {
  if (batch > 0) k_pack_train<<<dim3(256, batch), 256, 0, s>>>(R, U, slots, n, su, vin);
}

// Energy residual of a batch (FP64 columns b * n): d_b = U[sl_b] + y_b / su - E[sl_b]
// (y null: the network's output taken as zero, i.e. block Jacobi alone)
__global__ void k_energy_d(const float* __restrict__ U, const float* __restrict__ E,
                           const float* __restrict__ y, const int* __restrict__ slots, size_t n,
                           float inv_su, double* __restrict__ d) {
  const int b = blockIdx.y;
  const size_t o = (size_t)slots[b] * n;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (size_t)gridDim.x * blockDim.x) {
    double val = (double)U[o + v] - (double)E[o + v];
    if (y) val += (double)y[(size_t)b * n + v] * (double)inv_su;
    d[(size_t)b * n + v] = val;
  }
}

void launch_energy_d(const float* U, const float* E, const float* y, const int* slots, size_t n,
                     float inv_su, double* d, int batch, hipStream_t s) {
  if (batch > 0) k_energy_d<<<dim3(256, batch), 256, 0, s>>>(U, E, y, slots, n, inv_su, d);
}

// Block partial sums of a_b . q_b (FP64; a either FP64 columns or, with af,
// FP32 rows at slot sl_b) into part[b * gridDim.x + blk]; with gy, also the
// output gradient gy_b = coef[b] * q_b (FP32).
__global__ void k_energy_dot(const double* __restrict__ a, const float* __restrict__ af,
                             const int* __restrict__ slots, const double* __restrict__ q,
                             const float* __restrict__ qf, size_t n,
                             const float* __restrict__ coef, float* __restrict__ gy,
                             double* __restrict__ part) {
  __shared__ double red[256];
  const int b = blockIdx.y;
  const size_t oa = af ? (size_t)slots[b] * n : (size_t)b * n;
  const size_t oq = qf ? (size_t)slots[b] * n : (size_t)b * n;
  double acc = 0.0;
  for (size_t v = (size_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (size_t)gridDim.x * blockDim.x) {
    const double av = af ? (double)af[oa + v] : a[oa + v];
    const double qv = qf ? (double)qf[oq + v] : q[oq + v];
    acc += av * qv;
    if (gy) gy[(size_t)b * n + v] = (float)(coef[b] * qv);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = red[0];
}

void launch_energy_dot(const double* a, const float* af, const int* slots, const double* q,
                       const float* qf, size_t n, const float* coef, float* gy, double* part,
                       int nblk, int batch, hipStream_t s) {
  if (batch > 0)
    k_energy_dot<<<dim3(nblk, batch), 256, 0, s>>>(a, af, slots, q, qf, n, coef, gy, part);
}

// Safeguarded correction, per column c (columns of length n):
//   g = (vr - vqu) / vqv if vqv > 0 (else 0);  z_c += g v_c
// (only active columns).
__global__ void k_gamma_axpy(const double* __restrict__ v, double* __restrict__ z, size_t n,
                             const double* __restrict__ vr, const double* __restrict__ vqu,
                             const double* __restrict__ vqv, const uint8_t* __restrict__ active) {
  const int c = blockIdx.y;
  if (active && !active[c]) return;
  const double den = vqv[c];
  if (!(den > 0.0)) return;
  const double g = (vr[c] - vqu[c]) / den;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    z[(size_t)c * n + i] += g * v[(size_t)c * n + i];
}

void launch_gamma_axpy(const double* v, double* z, size_t n, const double* vr, const double* vqu,
                       const double* vqv, const uint8_t* active, int ncols, hipStream_t s) {
  if (ncols > 0) k_gamma_axpy<<<dim3(256, ncols), 256, 0, s>>>(v, z, n, vr, vqu, vqv, active);
}

}  // namespace rbmc
