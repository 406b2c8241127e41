// Orthonormal DCT-II / DCT-III along one axis of many 2-D slices, by fast
// Fourier transforms: the diagonalizing transform of the Neumann grid
// Laplacian in the spectral preconditioner, O(N log N) per line and one read
// and one write of the data per axis (the transform is bound by HBM, not by
// arithmetic).
//
// Forward (Makhoul, IEEE TASSP 28(1), 1980): with v[n] = x[2n],
// v[N-1-n] = x[2n+1] and V = FFT_N(v),
//   X[k] = s_k Re(exp(-i pi k / 2N) V[k]),  s_0 = sqrt(1/N), s_k = sqrt(2/N).
// Inverse (X -> x = C^T X): with Y_k = X_k / s_k (Y_N = 0),
//   V[k] = exp(i pi k / 2N) (Y_k - i Y_{N-k}),  v = IFFT_N(V),
// and x read back through the same reordering.  v is real, so two lines
// share one complex transform (one as the real, one as the imaginary part);
// their spectra are separated by the Hermitian symmetry of each.
//
// Workgroup: 256 threads and 2048 complex values in LDS, i.e. P = 2048 / N
// line pairs, plus the N/2 twiddles; decimation in time on bit-reversed
// input, in place, in radix-4 steps (and one radix-2 step when log2 N is odd).
#include "rbmc_impl.h"

namespace rbmc {

namespace {
constexpr int kFftSlots = 2048;  // complex values per workgroup
constexpr int kFftThreads = 256;

__device__ __forceinline__ int fft_find(const FftTask* __restrict__ t, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (t[mid].tile_start <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// position of x[m] in v
__device__ __forceinline__ int fft_vpos(int m, int N) {
  return (m & 1) ? N - 1 - (m >> 1) : (m >> 1);
}

__device__ __forceinline__ int fft_rev(int i, int lg) {
  return (int)(__brev((unsigned)i) >> (32 - lg));
}

// LDS placement of the complex value at logical index x (x < 2048): bits 0-4
// are XORed with functions of bits 5-10, a bijection that spreads the strided
// butterfly accesses and the bit-reversed scatter over the 64 LDS banks (bank
// conflicts of every access pattern of the transform counted for lengths 16 to
// 2048 with a 64-bank, 4-byte model: about a quarter of those of the identity
// placement, none worse than 2-way).
__device__ __forceinline__ int fsw(int x) {
  return x ^ ((x >> 6) & 31) ^ ((x >> 5) & 15) ^ (((x >> 6) & 7) << 2);
}
// placement of twiddle pair t (t < 1024), read as one 16-byte access: the
// stage strides N / 2h become distinct banks
__device__ __forceinline__ int tsw(int t) { return t ^ ((t >> 4) & 15) ^ ((t >> 8) & 3); }
}  // namespace

// AXIS 0: lines are contiguous (element stride 1, consecutive lines mx
// apart); AXIS 1: element stride mx, consecutive lines adjacent.  Thread
// mappings keep global accesses coalesced in both cases.
template <int AXIS>
__global__ __launch_bounds__(kFftThreads, 4) void k_dct_fft(const FftTask* __restrict__ tasks,
                                                            int n_tasks, int total_tiles,
                                                            int per_xcd) {
  extern __shared__ double fft_lds[];  // zr, zi (kFftSlots each), then N/2 twiddle pairs
  __shared__ long lbase[2 * kFftSlots / 16];  // offsets of the workgroup's lines
  double* zr = fft_lds;  // value x at fsw(x)
  double* zi = fft_lds + kFftSlots;
  double2* twl = (double2*)(fft_lds + 2 * kFftSlots);  // pair t at tsw(t)
  // workgroups are dispatched round-robin over the 8 XCDs: consecutive tiles
  // (neighbouring lines, which share 128-byte segments along axis 1) go to
  // one XCD, so the second half of each segment is read from its L2
  const int tile = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (tile >= total_tiles) return;
  const FftTask tk = tasks[fft_find(tasks, n_tasks, tile)];
  // N = 2^lg, P = 2^(11 - lg) line pairs, L = 2P lines: index math by shifts
  const int N = tk.N, lg = tk.lg, lp = 11 - lg, ll = lp + 1, P = 1 << lp, L = 1 << ll;
  const long g0 = (long)(tile - tk.tile_start) * L;  // first line of the workgroup
  const long nlines = (long)tk.nslices * tk.nl;
  const gptr<const double> in = G(tk.in);
  const gptr<double> out = G(tk.out);
  const gptr<const double> tw = G(tk.tw), ph = G(tk.ph);
  const long est = tk.estride;
  for (int q = threadIdx.x; q < N / 2; q += kFftThreads) twl[tsw(q)] = double2{tw[2 * q], tw[2 * q + 1]};
  for (int i = threadIdx.x; i < L; i += kFftThreads) {
    const long g = g0 + i;
    lbase[i] = (g / tk.nl) * tk.sstride + (g % tk.nl) * tk.lstride;
  }
  __syncthreads();
  auto base = [&](int i) -> long { return lbase[i]; };
  // P N = kFftSlots for every N, so each loop below has a fixed trip count
  // per thread: unrolled, its global loads are all in flight at once
  constexpr int kLN = 2 * kFftSlots / kFftThreads;  // (line, element) pairs per thread
  constexpr int kPN = kFftSlots / kFftThreads;      // (pair, frequency) pairs per thread
  if (!tk.inverse) {
    double v[kLN];
#pragma unroll
    for (int r = 0; r < kLN; ++r) {
      const int q = threadIdx.x + r * kFftThreads;
      const int i = AXIS == 0 ? q >> lg : q & (L - 1);
      const int m = AXIS == 0 ? q & (N - 1) : q >> ll;
      v[r] = g0 + i < nlines ? in[base(i) + m * est] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < kLN; ++r) {
      const int q = threadIdx.x + r * kFftThreads;
      const int i = AXIS == 0 ? q >> lg : q & (L - 1);
      const int m = AXIS == 0 ? q & (N - 1) : q >> ll;
      const int at = fsw((i >> 1) * N + fft_rev(fft_vpos(m, N), lg));
      if (i & 1) zi[at] = v[r]; else zr[at] = v[r];
    }
  } else {
    const double sn0 = sqrt(1.0 / N), sn = sqrt(2.0 / N);
    constexpr int kH = kPN / 2;  // two halves: fewer registers live
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      double y[kH][4], c[kH], s[kH];
#pragma unroll
      for (int r0 = 0; r0 < kH; ++r0) {
        const int q = threadIdx.x + (hf * kH + r0) * kFftThreads;
        const int p = AXIS == 0 ? q >> lg : q & (P - 1);
        const int k = AXIS == 0 ? q & (N - 1) : q >> lp;
        const int kr = (N - k) & (N - 1);
        c[r0] = ph[2 * k];
        s[r0] = ph[2 * k + 1];
#pragma unroll
        for (int part = 0; part < 2; ++part) {
          const int i = 2 * p + part;
          const bool ok = g0 + i < nlines;
          const long b = ok ? base(i) : 0;
          y[r0][2 * part] = ok ? in[b + k * est] : 0.0;
          y[r0][2 * part + 1] = ok && k ? in[b + kr * est] : 0.0;
        }
      }
#pragma unroll
      for (int r0 = 0; r0 < kH; ++r0) {
        const int q = threadIdx.x + (hf * kH + r0) * kFftThreads;
        const int p = AXIS == 0 ? q >> lg : q & (P - 1);
        const int k = AXIS == 0 ? q & (N - 1) : q >> lp;
        const double inv_k = 1.0 / (k ? sn : sn0), inv_r = 1.0 / sn;
        // V = (c + i s)(Y_k - i Y_{N-k}) for both lines, Z = V_A + i V_B
        const double ya = y[r0][0] * inv_k, yra = y[r0][1] * inv_r;
        const double yb = y[r0][2] * inv_k, yrb = y[r0][3] * inv_r;
        const double va_r = c[r0] * ya + s[r0] * yra, va_i = s[r0] * ya - c[r0] * yra;
        const double vb_r = c[r0] * yb + s[r0] * yrb, vb_i = s[r0] * yb - c[r0] * yrb;
        const int at = fsw(p * N + fft_rev(k, lg));
        zr[at] = va_r - vb_i;
        zi[at] = va_i + vb_r;
      }
    }
  }
  __syncthreads();
  const double sgn = tk.inverse ? -1.0 : 1.0;  // twiddles exp(-+2 pi i j / N)
  // radix-4 steps: the radix-2 stages h and 2h at once on the four entries
  // i0 + {0, h, 2h, 3h} of a block of 4h (j = i0 mod h):
  //   b0,1 = a0 +- w1 a1, b2,3 = a2 +- w1 a3             (w1 = W_2h^j)
  //   c0,2 = b0 +- w2 b2, c1,3 = b1 +- w3 b3   (w2 = W_4h^j, w3 = -+i w2)
  int h = 1, lh = 0;
  for (; 4 * h <= N; h <<= 2, lh += 2) {
#pragma unroll
    for (int r = 0; r < kFftSlots / 4 / kFftThreads; ++r) {
      const int u = threadIdx.x + r * kFftThreads;
      const int p = u >> (lg - 2), b = u & ((N >> 2) - 1);
      const int j = b & (h - 1);
      const int i0 = (p << lg) + ((b >> lh) << (lh + 2)) + j;
      const int t1 = j * (N >> (lh + 1)), t2 = j * (N >> (lh + 2));
      const double2 w1 = twl[tsw(t1)], w2 = twl[tsw(t2)];
      const double w1r = w1.x, w1i = -sgn * w1.y;
      const double w2r = w2.x, w2i = -sgn * w2.y;
      const double w3r = sgn * w2i, w3i = -sgn * w2r;  // -+i w2
      const int x0 = fsw(i0), x1 = fsw(i0 + h), x2 = fsw(i0 + 2 * h), x3 = fsw(i0 + 3 * h);
      const double a0r = zr[x0], a0i = zi[x0];
      const double a1r = zr[x1], a1i = zi[x1];
      const double a2r = zr[x2], a2i = zi[x2];
      const double a3r = zr[x3], a3i = zi[x3];
      const double m1r = w1r * a1r - w1i * a1i, m1i = w1r * a1i + w1i * a1r;
      const double m3r = w1r * a3r - w1i * a3i, m3i = w1r * a3i + w1i * a3r;
      const double b0r = a0r + m1r, b0i = a0i + m1i, b1r = a0r - m1r, b1i = a0i - m1i;
      const double b2r = a2r + m3r, b2i = a2i + m3i, b3r = a2r - m3r, b3i = a2i - m3i;
      const double n2r = w2r * b2r - w2i * b2i, n2i = w2r * b2i + w2i * b2r;
      const double n3r = w3r * b3r - w3i * b3i, n3i = w3r * b3i + w3i * b3r;
      zr[x0] = b0r + n2r;
      zi[x0] = b0i + n2i;
      zr[x2] = b0r - n2r;
      zi[x2] = b0i - n2i;
      zr[x1] = b1r + n3r;
      zi[x1] = b1i + n3i;
      zr[x3] = b1r - n3r;
      zi[x3] = b1i - n3i;
    }
    __syncthreads();
  }
  if (h < N) {  // log2 N odd: one radix-2 stage (h = N / 2)
#pragma unroll
    for (int r = 0; r < kFftSlots / 2 / kFftThreads; ++r) {
      const int u = threadIdx.x + r * kFftThreads;
      const int p = u >> (lg - 1), j = u & ((N >> 1) - 1);
      const int i0 = fsw(p * N + j), i1 = fsw(p * N + j + h);
      const double2 w = twl[tsw(j)];
      const double wr = w.x, wi = -sgn * w.y;
      const double ar = zr[i1], ai = zi[i1];
      const double tr = wr * ar - wi * ai, ti = wr * ai + wi * ar;
      const double br = zr[i0], bi = zi[i0];
      zr[i1] = br - tr;
      zi[i1] = bi - ti;
      zr[i0] = br + tr;
      zi[i0] = bi + ti;
    }
    __syncthreads();
  }
  if (!tk.inverse) {
    const double sn0 = sqrt(1.0 / N), sn = sqrt(2.0 / N);
#pragma unroll
    for (int r = 0; r < kLN; ++r) {
      const int q = threadIdx.x + r * kFftThreads;
      const int i = AXIS == 0 ? q >> lg : q & (L - 1);
      const int k = AXIS == 0 ? q & (N - 1) : q >> ll;
      const int p = i >> 1, kr = (N - k) & (N - 1);
      const double c = ph[2 * k], s = ph[2 * k + 1];
      const int xk = fsw(p * N + k), xr = fsw(p * N + kr);
      const double ar = zr[xk], ai = zi[xk];
      const double br = zr[xr], bi = zi[xr];
      // V_A = (Z_k + conj Z_{N-k}) / 2,  V_B = (Z_k - conj Z_{N-k}) / 2i
      const double vr = (i & 1) ? 0.5 * (ai + bi) : 0.5 * (ar + br);
      const double vi = (i & 1) ? -0.5 * (ar - br) : 0.5 * (ai - bi);
      // Re(exp(-i pi k / 2N) V)
      if (g0 + i < nlines) out[base(i) + k * est] = (k ? sn : sn0) * (c * vr + s * vi);
    }
  } else {
    const double scale = 1.0 / N;
#pragma unroll
    for (int r = 0; r < kLN; ++r) {
      const int q = threadIdx.x + r * kFftThreads;
      const int i = AXIS == 0 ? q >> lg : q & (L - 1);
      const int m = AXIS == 0 ? q & (N - 1) : q >> ll;
      const int at = fsw((i >> 1) * N + fft_vpos(m, N));
      if (g0 + i < nlines) out[base(i) + m * est] = scale * ((i & 1) ? zi[at] : zr[at]);
    }
  }
}

int fft_tiles(int N, long lines) {
  const int L = 2 * (kFftSlots / N);
  return (int)((lines + L - 1) / L);
}

bool fft_length_ok(int N) { return N >= 16 && N <= kFftSlots && (N & (N - 1)) == 0; }

void launch_dct_fft(const FftTask* d_tasks, int n_tasks, int total_tiles, int axis, int max_n,
                    hipStream_t s) {
  if (total_tiles <= 0) return;
  const size_t lds = (2 * (size_t)kFftSlots + max_n) * sizeof(double);
  const int per_xcd = (total_tiles + 7) / 8;
  if (axis == 0)
    k_dct_fft<0><<<per_xcd * 8, kFftThreads, lds, s>>>(d_tasks, n_tasks, total_tiles, per_xcd);
  else
    k_dct_fft<1><<<per_xcd * 8, kFftThreads, lds, s>>>(d_tasks, n_tasks, total_tiles, per_xcd);
}

}  // namespace rbmc
