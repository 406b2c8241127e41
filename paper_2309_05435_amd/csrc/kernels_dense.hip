// Dense FP64 kernels for the spatial blocks of the block-tridiagonal chains:
//   - grouped GEMM on the FP64 matrix cores (v_mfma_f64_16x16x4f64);
//   - in-place inversion of SPD blocks by the block Gauss-Jordan sweep,
//     whose rank-64 updates also run on the matrix cores;
//   - products of the restricted 13-point stencil Q_R with dense blocks.
// Dense blocks are column-major, padded to multiples of 64 with identity on
// the padded diagonal.
#include "rbmc_impl.h"

namespace rbmc {

typedef double v4d __attribute__((ext_vector_type(4)));

// FP64 16x16x4 matrix-core product. Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator register i of lane l holds C[l/16 + 4 i][l%16].
__device__ inline v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Grouped GEMM.  Workgroup tile 128 x 128 (four waves of 64 x 64), BK = 16.
// LDS holds A and B tiles with k contiguous per row/column (stride 18 to
// spread banks).  In MFMA step s lane group g = l/16 contributes k = 4g + s,
// so each lane reads its four k values of a row with one 32-byte access.
// ---------------------------------------------------------------------------
namespace {
constexpr int GBM = 128, GBN = 128, GBK = 16, GLDS = GBK + 2;
}

// Each thread moves 8 doubles of the A tile and 8 of the B tile per K step.
// Rows/columns that are contiguous in memory go to contiguous LDS (k-major
// per row); the other orientation is written with a stride.
struct TileRegs {
  double2 v[4];
};

__device__ inline void load_a(const GemmTask& tk, int m0, int k0, int tid, TileRegs& r) {
  if (!tk.transA) {  // column-major A: 8 consecutive rows of one column k
    const int kk = tid >> 4, mm = (tid & 15) * 8, gm = m0 + mm;
    const double* src = tk.A + (size_t)(k0 + kk) * tk.lda + gm;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = gm + 2 * j;
      if (c + 1 < tk.M) r.v[j] = *(const double2*)(src + 2 * j);
      else r.v[j] = double2{c < tk.M ? src[2 * j] : 0.0, 0.0};
    }
  } else {  // A^T stored column-major: 8 consecutive k of one row m
    const int mm = tid >> 1, kk = (tid & 1) * 8, gm = m0 + mm;
    const double* src = tk.A + (size_t)gm * tk.lda + k0 + kk;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      r.v[j] = (gm < tk.M) ? *(const double2*)(src + 2 * j) : double2{0.0, 0.0};
  }
}

__device__ inline void store_a(const GemmTask& tk, int tid, const TileRegs& r, double* As) {
  if (!tk.transA) {
    const int kk = tid >> 4, mm = (tid & 15) * 8;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      As[(mm + 2 * j) * GLDS + kk] = r.v[j].x;
      As[(mm + 2 * j + 1) * GLDS + kk] = r.v[j].y;
    }
  } else {
    const int mm = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
    for (int j = 0; j < 4; ++j) *(double2*)&As[mm * GLDS + kk + 2 * j] = r.v[j];
  }
}

__device__ inline void load_b(const GemmTask& tk, int n0, int k0, int tid, TileRegs& r) {
  if (!tk.transB) {  // column-major B: 8 consecutive k of one column n
    const int nn = tid >> 1, kk = (tid & 1) * 8, gn = n0 + nn;
    const double* src = tk.B + (size_t)gn * tk.ldb + k0 + kk;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      r.v[j] = (gn < tk.N) ? *(const double2*)(src + 2 * j) : double2{0.0, 0.0};
  } else {  // B^T stored column-major: 8 consecutive n of one row k
    const int kk = tid >> 4, nn = (tid & 15) * 8, gn = n0 + nn;
    const double* src = tk.B + (size_t)(k0 + kk) * tk.ldb + gn;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = gn + 2 * j;
      if (c + 1 < tk.N) r.v[j] = *(const double2*)(src + 2 * j);
      else r.v[j] = double2{c < tk.N ? src[2 * j] : 0.0, 0.0};
    }
  }
}

__device__ inline void store_b(const GemmTask& tk, int tid, const TileRegs& r, double* Bs) {
  if (!tk.transB) {
    const int nn = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
    for (int j = 0; j < 4; ++j) *(double2*)&Bs[nn * GLDS + kk + 2 * j] = r.v[j];
  } else {
    const int kk = tid >> 4, nn = (tid & 15) * 8;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      Bs[(nn + 2 * j) * GLDS + kk] = r.v[j].x;
      Bs[(nn + 2 * j + 1) * GLDS + kk] = r.v[j].y;
    }
  }
}

int gemm_task_tiles(int M, int N, int lower) {
  const int tm = (M + GBM - 1) / GBM, tn = (N + GBN - 1) / GBN;
  return lower ? tm * (tm + 1) / 2 : tm * tn;
}

// Workgroups are dispatched round-robin over the 8 XCDs; the logical tile of
// a workgroup is chosen so that each XCD walks a contiguous range of tiles
// (neighbouring tiles share A row panels in its L2).  The K loop prefetches
// the next A/B tiles into registers while the matrix cores consume the
// current LDS tiles.
__global__ __launch_bounds__(256, 2) void k_gemm_f64(const GemmTask* __restrict__ tasks,
                                                     int n_tasks, int total_tiles, int per_xcd) {
  __shared__ double As[GBM * GLDS];
  __shared__ double Bs[GBN * GLDS];
  const int b = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (b >= total_tiles) return;
  int lo = 0, hi = n_tasks - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (tasks[mid].tile_start <= b) lo = mid; else hi = mid - 1;
  }
  const GemmTask tk = tasks[lo];
  const int tile = b - tk.tile_start;
  int tm, tn;
  if (tk.lower) {  // enumerate (tm, tn), tm >= tn
    tm = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((tm + 1) * (tm + 2) / 2 <= tile) ++tm;
    while (tm * (tm + 1) / 2 > tile) --tm;
    tn = tile - tm * (tm + 1) / 2;
  } else {
    tm = tile / tk.tiles_n;
    tn = tile % tk.tiles_n;
  }
  const int m0 = tm * GBM, n0 = tn * GBN;
  if (tk.skip1 > tk.skip0) {
    const bool rows_hit = m0 < tk.skip1 && m0 + GBM > tk.skip0;
    const bool cols_hit = n0 < tk.skip1 && n0 + GBN > tk.skip0;
    if (rows_hit || cols_hit) return;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int l16 = lane & 15, g = lane >> 4;

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  TileRegs ra, rb;
  load_a(tk, m0, 0, tid, ra);
  load_b(tk, n0, 0, tid, rb);
  store_a(tk, tid, ra, As);
  store_b(tk, tid, rb, Bs);
  __syncthreads();
  for (int k0 = 0; k0 < tk.K; k0 += GBK) {
    const bool more = k0 + GBK < tk.K;
    if (more) {
      load_a(tk, m0, k0 + GBK, tid, ra);
      load_b(tk, n0, k0 + GBK, tid, rb);
    }
    double a[4][4], bb[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double* pa = &As[(wm + i * 16 + l16) * GLDS + 4 * g];
      double2 x0 = *(const double2*)pa, x1 = *(const double2*)(pa + 2);
      a[i][0] = x0.x; a[i][1] = x0.y; a[i][2] = x1.x; a[i][3] = x1.y;
      const double* pb = &Bs[(wn + i * 16 + l16) * GLDS + 4 * g];
      double2 y0 = *(const double2*)pb, y1 = *(const double2*)(pb + 2);
      bb[i][0] = y0.x; bb[i][1] = y0.y; bb[i][2] = y1.x; bb[i][3] = y1.y;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma64(a[i][s], bb[j][s], acc[i][j]);
    __syncthreads();
    if (more) {
      store_a(tk, tid, ra, As);
      store_b(tk, tid, rb, Bs);
      __syncthreads();
    }
  }
  // ---- epilogue: C = alpha acc + beta Cin
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + wn + j * 16 + l16;
      if (gn >= tk.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + g + 4 * r;
        if (gm >= tk.M) continue;
        double v = tk.alpha * acc[i][j][r];
        if (tk.beta != 0.0) v += tk.beta * tk.Cin[(size_t)gn * tk.ldcin + gm];
        tk.C[(size_t)gn * tk.ldc + gm] = v;
      }
    }
}

// ---------------------------------------------------------------------------
// Mixed-precision grouped GEMM: FP64 operands and result, products on the
// FP32 matrix cores (v_mfma_f32_16x16x4f32).  Operands are rounded to FP32
// when staged into LDS; each K chunk of 16 is accumulated in FP32 and then
// added to FP64 accumulators, so the error is that of rounding the operands
// (about 2^-24 relative per element) rather than of a long FP32 sum.
// Same 128 x 128 tiles and task semantics as k_gemm_f64; eight waves of
// 64 x 32 keep the FP64 accumulators within the register budget.
// FP32 16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator
// register i of lane l holds C[4 (l/16) + i][l%16].
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));

namespace {
constexpr int XLD = GBK + 4;  // LDS row stride (floats) of the k-contiguous tiles

struct XRegs {
  double2 v[2];
};

__device__ inline void xload_a(const GemmTask& tk, int m0, int k0, int tid, XRegs& r) {
  if (!tk.transA) {  // 4 consecutive rows of column k
    const int kk = tid >> 5, gm = m0 + (tid & 31) * 4;
    const double* src = tk.A + (size_t)(k0 + kk) * tk.lda + gm;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = gm + 2 * j;
      if (c + 1 < tk.M) r.v[j] = *(const double2*)(src + 2 * j);
      else r.v[j] = double2{c < tk.M ? src[2 * j] : 0.0, 0.0};
    }
  } else {  // 4 consecutive k of row m
    const int gm = m0 + (tid >> 2), kk = (tid & 3) * 4;
    const double* src = tk.A + (size_t)gm * tk.lda + k0 + kk;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      r.v[j] = (gm < tk.M) ? *(const double2*)(src + 2 * j) : double2{0.0, 0.0};
  }
}

__device__ inline void xstore_a(const GemmTask& tk, int tid, const XRegs& r, float* As) {
  if (!tk.transA) {
    const int kk = tid >> 5, mm = (tid & 31) * 4;
    As[(mm + 0) * XLD + kk] = (float)r.v[0].x;
    As[(mm + 1) * XLD + kk] = (float)r.v[0].y;
    As[(mm + 2) * XLD + kk] = (float)r.v[1].x;
    As[(mm + 3) * XLD + kk] = (float)r.v[1].y;
  } else {
    const int mm = tid >> 2, kk = (tid & 3) * 4;
    *(float4*)&As[mm * XLD + kk] =
        float4{(float)r.v[0].x, (float)r.v[0].y, (float)r.v[1].x, (float)r.v[1].y};
  }
}

__device__ inline void xload_b(const GemmTask& tk, int n0, int k0, int tid, XRegs& r) {
  if (!tk.transB) {  // 4 consecutive k of column n
    const int gn = n0 + (tid >> 2), kk = (tid & 3) * 4;
    const double* src = tk.B + (size_t)gn * tk.ldb + k0 + kk;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      r.v[j] = (gn < tk.N) ? *(const double2*)(src + 2 * j) : double2{0.0, 0.0};
  } else {  // 4 consecutive n of row k
    const int kk = tid >> 5, gn = n0 + (tid & 31) * 4;
    const double* src = tk.B + (size_t)(k0 + kk) * tk.ldb + gn;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = gn + 2 * j;
      if (c + 1 < tk.N) r.v[j] = *(const double2*)(src + 2 * j);
      else r.v[j] = double2{c < tk.N ? src[2 * j] : 0.0, 0.0};
    }
  }
}

__device__ inline void xstore_b(const GemmTask& tk, int tid, const XRegs& r, float* Bs) {
  if (!tk.transB) {
    const int nn = tid >> 2, kk = (tid & 3) * 4;
    *(float4*)&Bs[nn * XLD + kk] =
        float4{(float)r.v[0].x, (float)r.v[0].y, (float)r.v[1].x, (float)r.v[1].y};
  } else {
    const int kk = tid >> 5, nn = (tid & 31) * 4;
    Bs[(nn + 0) * XLD + kk] = (float)r.v[0].x;
    Bs[(nn + 1) * XLD + kk] = (float)r.v[0].y;
    Bs[(nn + 2) * XLD + kk] = (float)r.v[1].x;
    Bs[(nn + 3) * XLD + kk] = (float)r.v[1].y;
  }
}
}  // namespace

__global__ __launch_bounds__(512, 1) void k_gemm_mx(const GemmTask* __restrict__ tasks,
                                                    int n_tasks, int total_tiles, int per_xcd) {
  __shared__ float As[GBM * XLD];
  __shared__ float Bs[GBN * XLD];
  const int b = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (b >= total_tiles) return;
  int lo = 0, hi = n_tasks - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (tasks[mid].tile_start <= b) lo = mid; else hi = mid - 1;
  }
  const GemmTask tk = tasks[lo];
  const int tile = b - tk.tile_start;
  int tm, tn;
  if (tk.lower) {
    tm = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
    while ((tm + 1) * (tm + 2) / 2 <= tile) ++tm;
    while (tm * (tm + 1) / 2 > tile) --tm;
    tn = tile - tm * (tm + 1) / 2;
  } else {
    tm = tile / tk.tiles_n;
    tn = tile % tk.tiles_n;
  }
  const int m0 = tm * GBM, n0 = tn * GBN;
  if (tk.skip1 > tk.skip0) {
    const bool rows_hit = m0 < tk.skip1 && m0 + GBM > tk.skip0;
    const bool cols_hit = n0 < tk.skip1 && n0 + GBN > tk.skip0;
    if (rows_hit || cols_hit) return;
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 2) * 64, wn = (wave & 3) * 32;
  const int l16 = lane & 15, g = lane >> 4;

  double acc[4][2][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0.0;

  XRegs ra, rb;
  xload_a(tk, m0, 0, tid, ra);
  xload_b(tk, n0, 0, tid, rb);
  xstore_a(tk, tid, ra, As);
  xstore_b(tk, tid, rb, Bs);
  __syncthreads();
  for (int k0 = 0; k0 < tk.K; k0 += GBK) {
    const bool more = k0 + GBK < tk.K;
    if (more) {
      xload_a(tk, m0, k0 + GBK, tid, ra);
      xload_b(tk, n0, k0 + GBK, tid, rb);
    }
    float4 a[4], bb[2];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = *(const float4*)&As[(wm + i * 16 + l16) * XLD + 4 * g];
#pragma unroll
    for (int j = 0; j < 2; ++j) bb[j] = *(const float4*)&Bs[(wn + j * 16 + l16) * XLD + 4 * g];
    v4f c32[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) c32[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        c32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].x, bb[j].x, c32[i][j], 0, 0, 0);
        c32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].y, bb[j].y, c32[i][j], 0, 0, 0);
        c32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].z, bb[j].z, c32[i][j], 0, 0, 0);
        c32[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].w, bb[j].w, c32[i][j], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)c32[i][j][r];
    __syncthreads();
    if (more) {
      xstore_a(tk, tid, ra, As);
      xstore_b(tk, tid, rb, Bs);
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gn = n0 + wn + j * 16 + l16;
      if (gn >= tk.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + 4 * g + r;
        if (gm >= tk.M) continue;
        double v = tk.alpha * acc[i][j][r];
        if (tk.beta != 0.0) v += tk.beta * tk.Cin[(size_t)gn * tk.ldcin + gm];
        tk.C[(size_t)gn * tk.ldc + gm] = v;
      }
    }
}

void launch_gemm(const GemmTask* d_tasks, int n_tasks, int total_tiles, hipStream_t s,
                 int mixed) {
  if (total_tiles <= 0) return;
  const int per_xcd = (total_tiles + 7) / 8;
  if (mixed)
    k_gemm_mx<<<per_xcd * 8, 512, 0, s>>>(d_tasks, n_tasks, total_tiles, per_xcd);
  else
    k_gemm_f64<<<per_xcd * 8, 256, 0, s>>>(d_tasks, n_tasks, total_tiles, per_xcd);
}

// ---------------------------------------------------------------------------
// SPD inversion by the block Gauss-Jordan sweep (block size 64).
// Sweeping pivot block k of a symmetric M:
//   M_kk <- -M_kk^-1, M_ik <- M_ik M_kk^-1, M_kj <- M_kk^-1 M_kj,
//   M_ij <- M_ij - M_ik M_kk^-1 M_kj   (i, j != k);
// after all pivots M holds -A^-1.  Pivot blocks are Schur complements of an
// SPD matrix, hence SPD.  Only the lower block triangle is kept current.
// ---------------------------------------------------------------------------
namespace {
constexpr int JB = 64;
constexpr int JLD = JB + 1;

// In-LDS sweep of a 64x64 SPD block P (ld JLD): P <- P^-1.  Returns false on
// a non-positive pivot.
// Thread tid owns column c = tid % 64 and rows r = tid / 64 + 4 j (j < 16); the
// 16 owned entries live in registers for the whole sweep, so a pivot step is
// one broadcast of row/column p through LDS and 16 independent updates.
__device__ bool lds_spd_inverse(double* P, double* rowp, double* colp, int tid) {
  const int c = tid & 63, r0 = tid >> 6;
  double v[16];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = P[(r0 + 4 * j) * JLD + c];
  bool ok = true;
  for (int p = 0; p < JB; ++p) {
    // publish row p and column p of the current matrix
    if ((p & 3) == r0) rowp[c] = v[p >> 2];
    if (c == p) {
#pragma unroll
      for (int j = 0; j < 16; ++j) colp[r0 + 4 * j] = v[j];
    }
    __syncthreads();
    const double piv = rowp[p];
    if (!(piv > 0.0)) ok = false;
    const double ip = 1.0 / piv;
    const double rc = rowp[c] * ip;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int r = r0 + 4 * j;
      const double cr = colp[r];
      double nv = v[j] - cr * rc;
      if (c == p) nv = cr * ip;
      if (r == p) nv = (c == p) ? -ip : rc;
      v[j] = nv;
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 16; ++j) P[(r0 + 4 * j) * JLD + c] = -v[j];
  __syncthreads();
  return ok;
}
}  // namespace

// Pivot kernel: one workgroup per task inverts the 64 x 64 pivot block k
// (symmetrized from the lower triangle) into Pi.
__global__ __launch_bounds__(256) void k_gj_pivot(const InvTask* __restrict__ tasks, int kblk) {
  __shared__ double P[JB * JLD];
  __shared__ double rowp[JB], colp[JB];
  const InvTask tk = tasks[blockIdx.x];
  if (kblk >= tk.np / JB) return;
  const int tid = threadIdx.x, kb = kblk * JB, np = tk.np;
  for (int e = tid; e < JB * JB; e += 256) {
    const int r = e % JB, c = e / JB;
    const int rr = r > c ? r : c, cc = r > c ? c : r;
    P[r * JLD + c] = tk.M[(size_t)(kb + cc) * np + kb + rr];
  }
  const bool ok = lds_spd_inverse(P, rowp, colp, tid);
  if (!ok && tid == 0) atomicCAS(tk.info, 0, kblk + 1);
  for (int e = tid; e < JB * JB; e += 256) tk.Pi[e] = P[(e % JB) * JLD + e / JB];
}

// Panel kernel: grid (np/64 row blocks, tasks).  B_i = M_ik (lower-stored: i > k
// from M, i < k from M_ki^T, i = k the pivot block), U_i = B_i Pi (U_k = Pi),
// on the matrix cores; B_i and U_i go to the task's panels.
__global__ __launch_bounds__(256) void k_gj_panel(const InvTask* __restrict__ tasks, int kblk) {
  __shared__ double Bt[JB * JLD];
  __shared__ double Ps[JB * JLD];
  const InvTask tk = tasks[blockIdx.y];
  const int nblk = tk.np / JB;
  const int i = blockIdx.x;
  if (kblk >= nblk || i >= nblk) return;
  const int tid = threadIdx.x;
  const int kb = kblk * JB, ib = i * JB, np = tk.np;
  for (int e = tid; e < JB * JB; e += 256) {
    const int r = e % JB, c = e / JB;
    double v;
    if (i > kblk) v = tk.M[(size_t)(kb + c) * np + ib + r];
    else if (i < kblk) v = tk.M[(size_t)(ib + r) * np + kb + c];
    else {
      const int rr = r > c ? r : c, cc = r > c ? c : r;
      v = tk.M[(size_t)(kb + cc) * np + kb + rr];
    }
    Bt[r * JLD + c] = v;
    Ps[c * JLD + r] = tk.Pi[(size_t)c * JB + r];  // Ps[col][row] : k contiguous per column
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6, l16 = lane & 15, g = lane >> 4;
  if (i == kblk) {
    for (int e = tid; e < JB * JB; e += 256) {
      const int r = e % JB, c = e / JB;
      tk.U[(size_t)c * np + ib + r] = tk.Pi[(size_t)c * JB + r];
      tk.Bp[(size_t)c * np + ib + r] = Bt[r * JLD + c];
    }
    return;
  }
  // wave w: rows 16w..16w+15 of U_i = B_i Pi
  v4d acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < JB; k0 += 4) {
    const double a = Bt[(w * 16 + l16) * JLD + k0 + g];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = mfma64(a, Ps[(c * 16 + l16) * JLD + k0 + g], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = w * 16 + g + 4 * r, col = c * 16 + l16;
      tk.U[(size_t)col * np + ib + row] = acc[c][r];
    }
  for (int e = tid; e < JB * JB; e += 256) {
    const int r = e % JB, c = e / JB;
    tk.Bp[(size_t)c * np + ib + r] = Bt[r * JLD + c];
  }
}

// Rank-64 update of the lower block triangle: grid (lower tiles, tasks).
//   tile (i, j), i >= j:
//     i, j != k : M_ij -= U_i B_j^T
//     i > k = j : M_ik  = U_i
//     i = k > j : M_kj  = U_j^T
//     i = j = k : M_kk  = -U_k
__global__ __launch_bounds__(256) void k_gj_update(const InvTask* __restrict__ tasks, int kblk) {
  __shared__ double Us[JB * JLD];
  __shared__ double Bs[JB * JLD];
  const InvTask tk = tasks[blockIdx.y];
  const int nblk = tk.np / JB;
  if (kblk >= nblk) return;
  const int t = blockIdx.x;
  if (t >= nblk * (nblk + 1) / 2) return;
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  const int j = t - i * (i + 1) / 2;
  const int np = tk.np, ib = i * JB, jb = j * JB;
  const int tid = threadIdx.x;
  double* Mt = tk.M;
  if (i == kblk || j == kblk) {
    for (int e = tid; e < JB * JB; e += 256) {
      const int r = e % JB, c = e / JB;
      double v;
      if (i == kblk && j == kblk) v = -tk.U[(size_t)c * np + kblk * JB + r];
      else if (j == kblk) v = tk.U[(size_t)c * np + ib + r];
      else v = tk.U[(size_t)r * np + jb + c];
      Mt[(size_t)(jb + c) * np + ib + r] = v;
    }
    return;
  }
  for (int e = tid; e < JB * JB; e += 256) {
    const int r = e % JB, q = e / JB;
    Us[r * JLD + q] = tk.U[(size_t)q * np + ib + r];
    Bs[r * JLD + q] = tk.Bp[(size_t)q * np + jb + r];
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6, l16 = lane & 15, g = lane >> 4;
  v4d acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < JB; k0 += 4) {
    const double a = Us[(w * 16 + l16) * JLD + k0 + g];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = mfma64(a, Bs[(c * 16 + l16) * JLD + k0 + g], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = ib + w * 16 + g + 4 * r, col = jb + c * 16 + l16;
      Mt[(size_t)col * np + row] -= acc[c][r];
    }
}

// M (holding -A^-1 in its lower triangle) -> A^-1, full symmetric
__global__ void k_gj_finish(const InvTask* __restrict__ tasks) {
  const InvTask tk = tasks[blockIdx.y];
  const int np = tk.np;
  const size_t tot = (size_t)np * np;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % np), c = (int)(e / np);
    if (r >= c) {
      const double v = -tk.M[(size_t)c * np + r];
      tk.M[(size_t)c * np + r] = v;
      if (r != c) tk.M[(size_t)r * np + c] = v;
    }
  }
}

void launch_gj_step(const InvTask* d_tasks, int n_tasks, int max_np, int kblk, hipStream_t s) {
  const int maxblk = max_np / JB;
  if (n_tasks <= 0 || kblk >= maxblk) return;
  k_gj_pivot<<<n_tasks, 256, 0, s>>>(d_tasks, kblk);
  k_gj_panel<<<dim3(maxblk, n_tasks), 256, 0, s>>>(d_tasks, kblk);
  k_gj_update<<<dim3(maxblk * (maxblk + 1) / 2, n_tasks), 256, 0, s>>>(d_tasks, kblk);
}

void launch_gj_finish(const InvTask* d_tasks, int n_tasks, hipStream_t s) {
  if (n_tasks <= 0) return;
  k_gj_finish<<<dim3(1024, n_tasks), 256, 0, s>>>(d_tasks);
}

// ---------------------------------------------------------------------------
// Outer (block 256) level of the sweep.  Tiles are 64 x 64.
// ---------------------------------------------------------------------------
int gj2_tiles(int np, int w) { return (np / 64) * (w / 64); }

template <class T>
__device__ inline int find_task(const T* __restrict__ tasks, int n_tasks, int b) {
  int lo = 0, hi = n_tasks - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (tasks[mid].tile_start <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// B[r, c] = M[r, kb + c] (from the lower triangle), P = B[kb:kb+w, :]
__global__ __launch_bounds__(256) void k_gj2_gather(const Gj2Task* __restrict__ tasks,
                                                    int n_tasks) {
  __shared__ double T[64 * 65];
  const Gj2Task tk = tasks[find_task(tasks, n_tasks, blockIdx.x)];
  const int tile = blockIdx.x - tk.tile_start;
  const int tw = tk.w / 64;
  const int r0 = (tile / tw) * 64, c0 = (tile % tw) * 64;
  const int np = tk.np, tid = threadIdx.x;
  const int col0 = tk.kb + c0;  // global column of the tile
  const bool lower = r0 >= col0 + 64 || r0 == col0;  // whole tile (or diagonal tile) below
  if (r0 >= col0 + 64) {
    for (int e = tid; e < 4096; e += 256) {
      const int r = e % 64, c = e / 64;
      T[c * 65 + r] = tk.M[(size_t)(col0 + c) * np + r0 + r];
    }
  } else if (r0 + 64 <= col0) {  // strictly above: read the transposed lower tile
    for (int e = tid; e < 4096; e += 256) {
      const int c = e % 64, r = e / 64;
      T[c * 65 + r] = tk.M[(size_t)(r0 + r) * np + col0 + c];
    }
  } else {  // diagonal tile
    for (int e = tid; e < 4096; e += 256) {
      const int r = e % 64, c = e / 64;
      const int gr = r0 + r, gc = col0 + c;
      T[c * 65 + r] = gr >= gc ? tk.M[(size_t)gc * np + gr] : tk.M[(size_t)gr * np + gc];
    }
  }
  (void)lower;
  __syncthreads();
  for (int e = tid; e < 4096; e += 256) {
    const int r = e % 64, c = e / 64;
    const double v = T[c * 65 + r];
    tk.B[(size_t)(c0 + c) * np + r0 + r] = v;
    const int pr = r0 + r - tk.kb;
    if (pr >= 0 && pr < tk.w) tk.P[(size_t)(c0 + c) * tk.w + pr] = v;
  }
}

// Swept block row/column: M[r, kb+c] = U[r, c] (r >= kb + w),
// M[kb+r, j] = U[j, r] (j < kb), M[kb+r, kb+c] = -P^-1[r, c].
// Tiles: (np/64) x (w/64) over (row block of U, column c).
__global__ __launch_bounds__(256) void k_gj2_fix(const Gj2Task* __restrict__ tasks, int n_tasks) {
  __shared__ double T[64 * 65];
  const Gj2Task tk = tasks[find_task(tasks, n_tasks, blockIdx.x)];
  const int tile = blockIdx.x - tk.tile_start;
  const int tw = tk.w / 64;
  const int r0 = (tile / tw) * 64, c0 = (tile % tw) * 64;
  const int np = tk.np, tid = threadIdx.x, kb = tk.kb;
  if (r0 >= kb + tk.w) {  // below the pivot: column block
    for (int e = tid; e < 4096; e += 256) {
      const int r = e % 64, c = e / 64;
      tk.M[(size_t)(kb + c0 + c) * np + r0 + r] = tk.U[(size_t)(c0 + c) * np + r0 + r];
    }
  } else if (r0 < kb) {  // left of the pivot: row block (lower part), transposed
    for (int e = tid; e < 4096; e += 256) {
      const int r = e % 64, c = e / 64;
      T[c * 65 + r] = tk.U[(size_t)(c0 + c) * np + r0 + r];  // U[j = r0+r, c0+c]
    }
    __syncthreads();
    for (int e = tid; e < 4096; e += 256) {
      const int c = e % 64, r = e / 64;  // M[kb + c0 + c, r0 + r] = U[r0 + r, c0 + c]
      tk.M[(size_t)(r0 + r) * np + kb + c0 + c] = T[c * 65 + r];
    }
  } else {  // pivot block
    for (int e = tid; e < 4096; e += 256) {
      const int r = e % 64, c = e / 64;
      tk.M[(size_t)(kb + c0 + c) * np + r0 + r] = -tk.P[(size_t)(c0 + c) * tk.w + (r0 - kb) + r];
    }
  }
}

void launch_gj2_gather(const Gj2Task* d_tasks, int n_tasks, int total_tiles, hipStream_t s) {
  if (total_tiles > 0) k_gj2_gather<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

void launch_gj2_fix(const Gj2Task* d_tasks, int n_tasks, int total_tiles, hipStream_t s) {
  if (total_tiles > 0) k_gj2_fix<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
}

// ---------------------------------------------------------------------------
// Restricted-stencil products: out = alpha Q_R op(M) + gamma Q_R + diag(dv)
//                                    (+ I on the padded diagonal) + beta In
// on 64 x 64 output tiles; rows are region nodes (padded to np).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rstencil(const StencilTask* __restrict__ tasks,
                                                  int n_tasks) {
  __shared__ double tileT[64 * 65];
  int lo = 0, hi = n_tasks - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (tasks[mid].tile_start <= b) lo = mid; else hi = mid - 1;
  }
  const StencilTask tk = tasks[lo];
  const RegionDev rg = *tk.rg;
  const double* __restrict__ qs = tk.qs;
  const int ns = tk.ns;
  const int tile = b - tk.tile_start;
  const int tiles_c = (tk.ncols + 63) / 64;
  const int a0 = (tile / tiles_c) * 64, c0 = (tile % tiles_c) * 64;
  const int tid = threadIdx.x;
  const bool square = (tk.dv != nullptr) || tk.pad_identity || tk.gamma != 0.0;

  // the sparse terms (gamma Q_R, diag(dv), padded identity) are added by
  // k_sparse_add after this pass
  auto extra = [&](int a, int c, double v) {
    if (tk.beta != 0.0) v += tk.beta * tk.In[(size_t)c * tk.ldin + a];
    return v;
  };
  (void)square;

  if (!tk.trans) {
    // thread -> row a (fast), 16 columns
    const int a = a0 + (tid & 63);
    int nbr[kNS];
    double cf[kNS];
    const bool real = a < rg.nb;
    if (real) {
      const int node = rg.nodes[a];
#pragma unroll
      for (int q = 0; q < kNS; ++q) {
        nbr[q] = rg.nbr[a * kNS + q];
        cf[q] = qs[(size_t)q * ns + node];
      }
    }
    for (int cc = (tid >> 6); cc < 64; cc += 4) {
      const int c = c0 + cc;
      if (c >= tk.ncols) break;
      double v = 0.0;
      if (real && tk.alpha != 0.0) {
        const double* mc = tk.M + (size_t)c * tk.ldm;
#pragma unroll
        for (int q = 0; q < kNS; ++q)
          if (nbr[q] >= 0) v += cf[q] * mc[nbr[q]];
        v *= tk.alpha;
      }
      tk.out[(size_t)c * tk.ldout + a] = extra(a, c, v);
    }
  } else {
    // thread -> column c (fast), 16 rows; transpose through LDS for the store
    const int cl = tid & 63, c = c0 + cl;
    for (int ar = (tid >> 6); ar < 64; ar += 4) {
      const int a = a0 + ar;
      double v = 0.0;
      if (a < rg.nb && c < tk.ncols && tk.alpha != 0.0) {
        const int node = rg.nodes[a];
#pragma unroll
        for (int q = 0; q < kNS; ++q) {
          const int nb = rg.nbr[a * kNS + q];
          if (nb >= 0) v += qs[(size_t)q * ns + node] * tk.M[(size_t)nb * tk.ldm + c];
        }
        v *= tk.alpha;
      }
      tileT[ar * 65 + cl] = v;
    }
    __syncthreads();
    const int al = tid & 63, a = a0 + al;
    for (int cc = (tid >> 6); cc < 64; cc += 4) {
      const int c2 = c0 + cc;
      if (c2 >= tk.ncols) break;
      tk.out[(size_t)c2 * tk.ldout + a] = extra(a, c2, tileT[al * 65 + cc]);
    }
  }
}

// out += gamma Q_R + diag(dv) + I on the padded diagonal: one thread per row,
// touching only the stencil positions.  Grid (row blocks of 256, tasks).
__global__ __launch_bounds__(256) void k_sparse_add(const StencilTask* __restrict__ tasks) {
  const StencilTask tk = tasks[blockIdx.y];
  if (tk.gamma == 0.0 && tk.dv == nullptr && !tk.pad_identity) return;
  const RegionDev rg = *tk.rg;
  const double* __restrict__ qs = tk.qs;
  const int ns = tk.ns;
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= rg.np) return;
  if (a < rg.nb) {
    const int node = rg.nodes[a];
    if (tk.gamma != 0.0)
      for (int q = 0; q < kNS; ++q) {
        const int c = rg.nbr[a * kNS + q];
        if (c >= 0) tk.out[(size_t)c * tk.ldout + a] += tk.gamma * qs[(size_t)q * ns + node];
      }
    if (tk.dv) tk.out[(size_t)a * tk.ldout + a] += tk.dv[node];
  } else if (tk.pad_identity) {
    tk.out[(size_t)a * tk.ldout + a] += 1.0;
  }
}

void launch_rstencil(const StencilTask* d_tasks, int n_tasks, int total_tiles, int max_np,
                     hipStream_t s) {
  if (total_tiles <= 0) return;
  k_rstencil<<<total_tiles, 256, 0, s>>>(d_tasks, n_tasks);
  if (max_np > 0) k_sparse_add<<<dim3((max_np + 255) / 256, n_tasks), 256, 0, s>>>(d_tasks);
}

// Lower triangle -> upper triangle (full symmetric), 64 x 64 tiles through LDS.
// Grid (lower tiles of the largest block, tasks).
__global__ __launch_bounds__(256) void k_mirror(const InvTask* __restrict__ tasks) {
  __shared__ double T[64 * 65];
  const InvTask tk = tasks[blockIdx.y];
  const int np = tk.np, nt = np / 64;
  const int t = blockIdx.x;
  if (t >= nt * (nt + 1) / 2) return;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  while (I * (I + 1) / 2 > t) --I;
  const int J = t - I * (I + 1) / 2;
  const int tid = threadIdx.x;
  for (int e = tid; e < 4096; e += 256) {  // lower tile (rows I, cols J)
    const int r = e % 64, c = e / 64;
    T[c * 65 + r] = tk.M[(size_t)(J * 64 + c) * np + I * 64 + r];
  }
  __syncthreads();
  for (int e = tid; e < 4096; e += 256) {  // upper tile (rows J, cols I): M[J+c, I+r] = T[c][r]
    const int c = e % 64, r = e / 64;
    if (I == J && c <= r) continue;  // diagonal tile: only its strict upper part
    tk.M[(size_t)(I * 64 + r) * np + J * 64 + c] = T[c * 65 + r];
  }
}

void launch_mirror(const InvTask* d_tasks, int n_tasks, int max_np, hipStream_t s) {
  const int nt = max_np / 64;
  if (n_tasks > 0 && nt > 0) k_mirror<<<dim3(nt * (nt + 1) / 2, n_tasks), 256, 0, s>>>(d_tasks);
}

}  // namespace rbmc
